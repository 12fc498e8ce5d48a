// sl_api.hip -- host runtime behind the C ABI of spinlat.h: device buffers,
// the rebuild pipeline (cells, lists, colour classes, permutation), the
// step schedule and the observables. All per-step work runs in the kernels
// of sl_dyn.hip; this file only orders launches on the system's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/spinlat.h"
#include "sl_device.h"
#include "sl_kernels.h"
#include "sl_mlp_host.h"

using namespace sl;

namespace {

thread_local std::string g_create_err = "";

constexpr int kThermoCap = 1 << 16;
constexpr int kJpBatch = 16;

struct Atoms {
  double *rx[2] = {nullptr, nullptr}, *ry[2] = {nullptr, nullptr}, *rz[2] = {nullptr, nullptr};
  double *vx = nullptr, *vy = nullptr, *vz = nullptr;
  double *bx = nullptr, *by = nullptr, *bz = nullptr;
  double *mass = nullptr;
  void *sx = nullptr, *sy = nullptr, *sz = nullptr;
  int *id = nullptr, *colour = nullptr, *cell = nullptr;
  int *nspin = nullptr, *nall = nullptr, *nbr = nullptr;
  unsigned long long *wmask = nullptr;  // same-colour spin-segment slots
};

struct ProfRec {
  int kind;
  hipEvent_t a, b;
  double work;
};

struct SlotMeta {
  int64_t boundary = -1;
  double dt = 0.0;
  bool rebuilt_after = false;
};

}  // namespace

struct sl_system {
  sl_params prm{};
  sl_potential pot{};
  PotConst pc{};
  bool have_pot = false;
  int n = 0, ld = 0, prec = SL_FP64;
  double L[3] = {0, 0, 0}, invL[3] = {0, 0, 0};
  double skin = 0.3;
  int max_nbr = 80, max_spin = 32;
  int Kbase = 0;                        // palette of the last full colouring
  int spin_lanes = 2, force_lanes = 1;  // lanes per atom (tuning only)
  int small_class = 512;                // fused small-class threshold (-1: off)
  hipStream_t st = nullptr;
  bool own_stream = false;

  Atoms a[2];
  int cur = 0;  // live Atoms copy
  int pos = 0;  // position buffer holding the current boundary

  // scratch
  int ncell = 0, nc[3] = {1, 1, 1};
  int *ccount = nullptr, *cstart = nullptr, *cfill = nullptr, *catoms = nullptr;
  int cell_cap = 0;
  int *bcount = nullptr, *bstart = nullptr, *bfill = nullptr;
  int bin_cap = 0;
  int *skey = nullptr, *perm = nullptr, *inv = nullptr, *uinv = nullptr, *ctmp = nullptr;
  double *kx = nullptr, *ky = nullptr, *kz = nullptr;
  double *stage = nullptr;  // 3n doubles
  int *err = nullptr, *seen = nullptr, *jpcnt = nullptr, *maxc = nullptr;
  int *jplist[2] = {nullptr, nullptr};  // ready lists of the colouring rounds
  unsigned long long *jpmask[2] = {nullptr, nullptr};  // conflict / earlier-key slot masks
  unsigned long long *dslot = nullptr;
  double *pred = nullptr;  // [force blocks][3] predictor terms of one launch
  unsigned int *done = nullptr;
  double *partial = nullptr, *red_out = nullptr;
  double *thermo = nullptr;
  double *ring = nullptr;      // pinned host [4 boundaries][8]
  double *ring_dev = nullptr;  // device alias of ring
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  SlotMeta meta[4];

  // state
  bool have_state = false, have_list = false, user_list = false, have_colour = false;
  bool have_D = false;
  int K = 0;
  std::vector<int> class_off;
  int64_t step = 0, rebuilds = 0;
  int jp_rounds = 0, seen_spin = 0, seen_all = 0;
  int sticky = 0;
  std::vector<int64_t> thermo_steps;
  int thermo_read = 0;

  // learned potential (FP32 form): unordered pairs of the list with their
  // mirror slots, and one (J, J', phi, phi') table per position buffer
  sl_mlp *mlp = nullptr;
  int mlp_mode = SL_MLP_SPLINE;  // how the learned potential is evaluated
  int2 *mpairs = nullptr;
  int *mirror = nullptr, *mcnt = nullptr, *mstart = nullptr;
  int npair = 0, mpair_cap = 0;
  float4 *tab[2] = {nullptr, nullptr};
  bool tab_ok[2] = {false, false};
  // exchange-coefficient cache per position buffer (analytic potential)
  int jcache = -1;  // set from the precision at creation (on for FP32)
  // spin ordering: colour classes, or the paper's sectors / serial order
  int ordering = SL_ORDER_COLOUR;
  double row_q = 0.0;  // list row order: 0 cell loop, > 0 displacement grid (A)
  // split force (tuning): the pair pass runs on st2 while the spins update
  int overlap = -1;
  hipStream_t st2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double *fp = nullptr;  // [4][ld] pair force and pair energy
  int sgrid[3] = {1, 1, 1};
  unsigned long long *skeys[2] = {nullptr, nullptr};
  int *svals[2] = {nullptr, nullptr};
  int *scount = nullptr, *soff = nullptr;
  int s_nbins_cap = 0;
  void *cub_tmp = nullptr;
  size_t cub_bytes = 0;
  void *jc[2] = {nullptr, nullptr};
  double *eam = nullptr;  // embedded-atom F'(rho), F(rho) per atom [2][ld]
  bool jc_ok[2] = {false, false};

  bool prof = false;
  int prof_every = 1;     // time the launches of every prof_every-th step
  bool prof_now = false;  // the current step is timed
  std::vector<ProfRec> prof_recs;
  std::vector<hipEvent_t> ev_pool;
  int64_t prof_launch[5] = {0, 0, 0, 0, 0};
  double prof_ms[5] = {0, 0, 0, 0, 0};
  double prof_work[5] = {0, 0, 0, 0, 0};

  std::string last_err;
};

namespace {

int fail(sl_system *S, int code, const std::string &msg) {
  if (S) S->last_err = msg;
  else g_create_err = msg;
  return code;
}

#define HIPCHK(S, x)                                                                      \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      return fail((S), SL_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_));       \
  } while (0)

#define CHK(x)            \
  do {                    \
    int rc_ = (x);        \
    if (rc_) return rc_;  \
  } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  // Not cleared: a clear on the null stream would not be ordered with the
  // library's non-blocking stream. Every buffer is written before it is read
  // (list slots past a row's end are masked, and gathered indices are
  // range-checked before use).
  return hipMalloc((void **)p, count * sizeof(T));
}

void dfree(void *p) {
  if (p) (void)hipFree(p);
}

double list_radius(const sl_system *S) {
  double rc = S->pot.ex_rc;
  if (!S->prm.frozen && S->pot.morse_on && S->pot.morse_rc > rc) rc = S->pot.morse_rc;
  if (!S->prm.frozen && S->pot.eam_on) rc = std::max(rc, std::max(S->pot.eam_d, S->pot.eam_c));
  return rc + (S->prm.frozen ? 0.0 : S->skin);
}

double spin_radius(const sl_system *S) {
  return S->pot.ex_rc + (S->prm.frozen ? 0.0 : S->skin);
}

// Spins closer than this at colouring time may not share a colour; a
// same-colour pair farther apart is watched by the rebuild rule instead.
// With a user list (no rebuilds) every spin-segment entry conflicts.
double colour_radius(const sl_system *S) {
  return S->pot.ex_rc + (S->prm.frozen ? 0.0 : S->skin / 3.0);
}

int check_box(sl_system *S) {
  const double rl = list_radius(S);
  for (int d = 0; d < 3; ++d)
    if (S->L[d] < 2.0 * rl)
      return fail(S, SL_E_BOX, "box side " + std::to_string(S->L[d]) +
                                   " A is below twice the list radius " + std::to_string(rl));
  return SL_OK;
}

void make_potconst(sl_system *S) {
  const sl_potential &p = S->pot;
  PotConst &c = S->pc;
  std::memset(&c, 0, sizeof(c));
  c.morse_on = (p.morse_on && !S->prm.frozen) ? 1 : 0;
  c.mD = p.morse_D;
  c.mA = p.morse_alpha;
  c.mR0 = p.morse_r0;
  c.mRc = p.morse_rc;
  c.mRc2 = p.morse_rc * p.morse_rc;
  if (p.morse_shift) {
    const double e = std::exp(-p.morse_alpha * (p.morse_rc - p.morse_r0));
    c.mMc = p.morse_D * (e * e - 2.0 * e);
    c.mdMc = -2.0 * p.morse_alpha * p.morse_D * (e * e - e);
  }
  c.ex_on = (p.ex_alpha != 0.0 && p.ex_rc > 0.0) ? 1 : 0;
  c.eA4 = 4.0 * p.ex_alpha;
  c.eG = p.ex_gamma;
  c.eInvD2 = 1.0 / (p.ex_delta * p.ex_delta);
  c.eRc2 = p.ex_rc * p.ex_rc;
  c.eA8InvD2 = 8.0 * p.ex_alpha / (p.ex_delta * p.ex_delta);
  if (p.ex_shift && p.ex_rc > 0.0) {
    const double u = p.ex_rc * p.ex_rc / (p.ex_delta * p.ex_delta), e = std::exp(-u);
    const double dJc = c.eA8InvD2 * p.ex_rc * e * (1.0 - (1.0 + 2.0 * p.ex_gamma) * u + p.ex_gamma * u * u);
    c.eJc = 4.0 * p.ex_alpha * u * (1.0 - p.ex_gamma * u) * e;
    c.eJq = dJc / (2.0 * p.ex_rc);
    c.eJr = dJc / p.ex_rc;
  }
  for (int d = 0; d < 3; ++d) {
    c.zB[d] = p.zeeman_g * kMuB * p.B[d];
    c.zw[d] = c.zB[d] / kHbar;
    c.an[d] = p.aniso_n[d];
  }
  c.aK = p.aniso_K;
  c.aK2h = 2.0 * p.aniso_K / kHbar;
  c.aniso_on = p.aniso_K != 0.0 ? 1 : 0;
  c.aniso_split = (c.aniso_on && p.aniso_split && !(p.lambda > 0.0)) ? 1 : 0;
  c.langevin = p.lambda > 0.0 ? 1 : 0;
  c.lam = p.lambda;
  c.lamfac = 1.0 / (1.0 + p.lambda * p.lambda);
  c.lat_on = (p.lat_gamma > 0.0 && !S->prm.frozen) ? 1 : 0;
  c.lat_g = p.lat_gamma;
  c.lat_kT = kKb * p.lat_temperature;
  const bool neel = p.neel_alpha != 0.0 && p.neel_rc > 0.0;
  const bool dmi = p.dmi_alpha != 0.0 && p.dmi_rc > 0.0;
  c.soc_on = (neel || dmi) ? 1 : 0;
  if (neel) {
    c.nA4 = 4.0 * p.neel_alpha;
    c.nG = p.neel_gamma;
    c.nInvD2 = 1.0 / (p.neel_delta * p.neel_delta);
    c.nRc2 = p.neel_rc * p.neel_rc;
    c.nA8InvD2 = 8.0 * p.neel_alpha / (p.neel_delta * p.neel_delta);
  }
  c.eam_on = (p.eam_on && !S->prm.frozen) ? 1 : 0;
  c.fA = p.eam_A;
  c.fd = p.eam_d;
  c.fbeta = p.eam_beta;
  c.fc = p.eam_c;
  c.fc0 = p.eam_c0;
  c.fc1 = p.eam_c1;
  c.fc2 = p.eam_c2;
  c.fd2 = p.eam_d * p.eam_d;
  c.fcc2 = p.eam_c * p.eam_c;
  if (dmi) {
    c.dA4 = 4.0 * p.dmi_alpha;
    c.dG = p.dmi_gamma;
    c.dInvD2 = 1.0 / (p.dmi_delta * p.dmi_delta);
    c.dRc2 = p.dmi_rc * p.dmi_rc;
    c.dA8InvD2 = 8.0 * p.dmi_alpha / (p.dmi_delta * p.dmi_delta);
    for (int d = 0; d < 3; ++d) c.dn[d] = p.dmi_n[d];
  }
}

template <typename real>
SysView<real> view(sl_system *S, int posbuf) {
  Atoms &A = S->a[S->cur];
  SysView<real> v;
  v.n = S->n;
  v.ld = S->ld;
  v.kcap = S->max_nbr;
  for (int d = 0; d < 3; ++d) {
    v.L[d] = S->L[d];
    v.invL[d] = S->invL[d];
  }
  v.rx = A.rx[posbuf];
  v.ry = A.ry[posbuf];
  v.rz = A.rz[posbuf];
  v.sx = (real *)A.sx;
  v.sy = (real *)A.sy;
  v.sz = (real *)A.sz;
  v.nbr = A.nbr;
  v.nspin = A.nspin;
  v.nall = A.nall;
  v.id = A.id;
  v.tab = nullptr;
  v.spl = SplineView{};
  const bool jc_use = (!S->mlp || S->mlp_mode == SL_MLP_SPLINE) && S->jcache > 0 && !S->pc.soc_on;
  v.jc = (jc_use && S->jc_ok[posbuf]) ? (const real *)S->jc[posbuf] : nullptr;
  v.eam = S->pc.eam_on ? S->eam : nullptr;
  if (S->mlp && S->mlp_mode == SL_MLP_SPLINE) {
    v.spl = S->mlp->spline_view();
    v.spl.jshift = S->pot.ex_shift ? 1 : 0;
  } else if (S->mlp) {
    v.tab = S->tab[posbuf];
  }
  return v;
}

// --- profiling -------------------------------------------------------------
hipEvent_t get_event(sl_system *S) {
  if (!S->ev_pool.empty()) {
    hipEvent_t e = S->ev_pool.back();
    S->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

struct ProfScope {
  sl_system *S;
  int kind;
  double work;
  hipEvent_t a = nullptr;
  hipStream_t st;
  ProfScope(sl_system *S_, int kind_, double work_, hipStream_t st_ = nullptr)
      : S(S_), kind(kind_), work(work_), st(st_ ? st_ : S_->st) {
    if (S->prof_now) {
      a = get_event(S);
      (void)hipEventRecord(a, st);
    }
  }
  ~ProfScope() {
    if (a) {
      hipEvent_t b = get_event(S);
      (void)hipEventRecord(b, st);
      S->prof_recs.push_back({kind, a, b, work});
    }
  }
};

void prof_collect(sl_system *S) {
  if (S->prof_recs.empty()) return;
  (void)hipStreamSynchronize(S->st);
  for (auto &r : S->prof_recs) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    S->prof_launch[r.kind] += 1;
    S->prof_ms[r.kind] += ms;
    S->prof_work[r.kind] += r.work;
    S->ev_pool.push_back(r.a);
    S->ev_pool.push_back(r.b);
  }
  S->prof_recs.clear();
}

// --- device error word ------------------------------------------------------
int read_err(sl_system *S) {
  int e = 0;
  HIPCHK(S, hipMemcpyAsync(&e, S->err, sizeof(int), hipMemcpyDeviceToHost, S->st));
  HIPCHK(S, hipStreamSynchronize(S->st));
  S->sticky |= e;
  return SL_OK;
}

int sticky_code(sl_system *S) {
  if (S->sticky & kErrNonFinite) return fail(S, SL_E_NONFINITE, "non-finite force, velocity or position");
  if (S->sticky & kErrNbrOverflow)
    return fail(S, SL_E_NBR_OVERFLOW, "neighbour row overflow: seen " + std::to_string(S->seen_all) +
                                          " (spin " + std::to_string(S->seen_spin) + "), capacity " +
                                          std::to_string(S->max_nbr) + " (spin " +
                                          std::to_string(S->max_spin) + ")");
  if (S->sticky & kErrColour) return fail(S, SL_E_COLOR, "two interacting spins share a colour");
  return SL_OK;
}

// --- allocation -------------------------------------------------------------
int alloc_atoms(sl_system *S, Atoms &A) {
  const int n = S->n;
  const size_t rs = S->prec == SL_FP64 ? sizeof(double) : sizeof(float);
  for (int b = 0; b < 2; ++b) {
    HIPCHK(S, dalloc(&A.rx[b], n));
    HIPCHK(S, dalloc(&A.ry[b], n));
    HIPCHK(S, dalloc(&A.rz[b], n));
  }
  HIPCHK(S, dalloc(&A.vx, n));
  HIPCHK(S, dalloc(&A.vy, n));
  HIPCHK(S, dalloc(&A.vz, n));
  HIPCHK(S, dalloc(&A.bx, n));
  HIPCHK(S, dalloc(&A.by, n));
  HIPCHK(S, dalloc(&A.bz, n));
  HIPCHK(S, dalloc(&A.mass, n));
  HIPCHK(S, hipMalloc(&A.sx, rs * (n > 0 ? n : 1)));
  HIPCHK(S, hipMalloc(&A.sy, rs * (n > 0 ? n : 1)));
  HIPCHK(S, hipMalloc(&A.sz, rs * (n > 0 ? n : 1)));
  HIPCHK(S, dalloc(&A.id, n));
  HIPCHK(S, dalloc(&A.colour, n));
  HIPCHK(S, dalloc(&A.wmask, n));
  HIPCHK(S, dalloc(&A.cell, n));
  HIPCHK(S, dalloc(&A.nspin, n));
  HIPCHK(S, dalloc(&A.nall, n));
  HIPCHK(S, dalloc(&A.nbr, (size_t)S->ld * S->max_nbr));
  HIPCHK(S, hipMemsetAsync(A.nspin, 0, sizeof(int) * n, S->st));
  HIPCHK(S, hipMemsetAsync(A.nall, 0, sizeof(int) * n, S->st));
  return SL_OK;
}

void free_atoms(Atoms &A) {
  for (int b = 0; b < 2; ++b) {
    dfree(A.rx[b]); dfree(A.ry[b]); dfree(A.rz[b]);
  }
  dfree(A.vx); dfree(A.vy); dfree(A.vz);
  dfree(A.bx); dfree(A.by); dfree(A.bz);
  dfree(A.mass); dfree(A.sx); dfree(A.sy); dfree(A.sz);
  dfree(A.id); dfree(A.colour); dfree(A.cell); dfree(A.wmask);
  dfree(A.nspin); dfree(A.nall); dfree(A.nbr);
  A = Atoms();
}

int ensure_cells(sl_system *S, int ncell) {
  if (ncell + 1 <= S->cell_cap) return SL_OK;
  dfree(S->ccount); dfree(S->cstart); dfree(S->cfill);
  S->cell_cap = ncell + 1;
  HIPCHK(S, dalloc(&S->ccount, S->cell_cap));
  HIPCHK(S, dalloc(&S->cstart, S->cell_cap + 1));
  HIPCHK(S, dalloc(&S->cfill, S->cell_cap));
  return SL_OK;
}

int ensure_bins(sl_system *S, int nbin) {
  if (nbin + 1 <= S->bin_cap) return SL_OK;
  dfree(S->bcount); dfree(S->bstart); dfree(S->bfill);
  S->bin_cap = nbin + 1;
  HIPCHK(S, dalloc(&S->bcount, S->bin_cap));
  HIPCHK(S, dalloc(&S->bstart, S->bin_cap + 1));
  HIPCHK(S, dalloc(&S->bfill, S->bin_cap));
  return SL_OK;
}

void cell_grid(sl_system *S, CellGrid &G) {
  const double rl = list_radius(S);
  for (int d = 0; d < 3; ++d) {
    int k = rl > 0 ? (int)std::floor(S->L[d] / rl) : 1;
    if (k < 3) k = 1;
    if (k > 1024) k = 1024;
    G.nc[d] = k;
    G.L[d] = S->L[d];
  }
  // at most ~2 cells per atom: larger cells are still valid, only slower
  const long cap = std::max<long>(2L * S->n, 27L);
  while ((long)G.nc[0] * G.nc[1] * G.nc[2] > cap) {
    int d = 0;
    for (int e = 1; e < 3; ++e)
      if (G.nc[e] > G.nc[d]) d = e;
    if (G.nc[d] <= 3) break;
    G.nc[d] = std::max(3, (G.nc[d] * 4) / 5);
  }
  for (int d = 0; d < 3; ++d) S->nc[d] = G.nc[d];
  S->ncell = G.nc[0] * G.nc[1] * G.nc[2];
}

// Cell index of every atom at the current positions and the sorted cell
// member lists (cstart/catoms).
int bin_cells(sl_system *S, CellGrid &G) {
  Atoms &A = S->a[S->cur];
  cell_grid(S, G);
  CHK(ensure_cells(S, S->ncell));
  launch_zero_i(S->ncell, S->ccount, S->st);
  launch_cell_assign(S->n, A.rx[S->pos], A.ry[S->pos], A.rz[S->pos], G, A.cell, S->ccount, S->st);
  launch_scan(S->ccount, S->cstart, S->ncell, S->st);
  launch_zero_i(S->ncell, S->cfill, S->st);
  launch_bucket_scatter(S->n, A.cell, S->cstart, S->cfill, S->catoms, S->st);
  launch_bucket_sort(S->ncell, S->cstart, S->catoms, S->st);
  return SL_OK;
}

ColourArgs colour_args(sl_system *S) {
  Atoms &A = S->a[S->cur];
  ColourArgs C;
  C.n = S->n;
  C.ld = S->ld;
  C.nbr = A.nbr;
  C.nspin = A.nspin;
  C.id = A.id;
  C.kx = S->kx;
  C.ky = S->ky;
  C.kz = S->kz;
  C.colour = A.colour;
  C.kbase = S->Kbase;
  C.rx = A.rx[S->pos];
  C.ry = A.ry[S->pos];
  C.rz = A.rz[S->pos];
  for (int d = 0; d < 3; ++d) {
    C.L[d] = S->L[d];
    C.invL[d] = S->invL[d];
  }
  const double rc = colour_radius(S);
  C.cr2 = S->user_list ? 1e300 : rc * rc;
  return C;
}

// Colouring rounds until every atom has a colour. Round r reads ready list
// r % 2 with count r % 3 and writes list (r + 1) % 2 with count (r + 1) % 3.
int jp_rounds(sl_system *S, const ColourArgs &C) {
  HIPCHK(S, hipMemsetAsync(S->jpcnt, 0, 3 * sizeof(int), S->st));
  launch_colour_indeg(C, S->ctmp, S->jpmask[0], S->jpmask[1], S->jplist[0], &S->jpcnt[0], S->st);
  int r = 0;
  for (;;) {
    for (int b = 0; b < kJpBatch; ++b, ++r)
      launch_colour_round(C, S->ctmp, S->jpmask[0], S->jpmask[1], S->jplist[r & 1],
                          &S->jpcnt[r % 3], S->jplist[(r + 1) & 1], &S->jpcnt[(r + 1) % 3],
                          &S->jpcnt[(r + 2) % 3], S->st);
    int rem = 0;
    HIPCHK(S, hipMemcpyAsync(&rem, &S->jpcnt[r % 3], sizeof(int), hipMemcpyDeviceToHost, S->st));
    HIPCHK(S, hipStreamSynchronize(S->st));
    if (rem == 0) break;
    if (r > S->n + 2 * kJpBatch) return fail(S, SL_E_COLOR, "colouring rounds made no progress");
  }
  S->jp_rounds = r;
  return SL_OK;
}

// Unordered pairs of the current list for the learned-potential table.
int mlp_pairs(sl_system *S) {
  Atoms &A = S->a[S->cur];
  const int n = S->n;
  launch_mlp_pair_count(n, S->ld, A.nbr, A.nall, S->mcnt, S->st);
  launch_scan(S->mcnt, S->mstart, n, S->st);
  int tot = 0;
  HIPCHK(S, hipMemcpyAsync(&tot, S->mstart + n, sizeof(int), hipMemcpyDeviceToHost, S->st));
  HIPCHK(S, hipStreamSynchronize(S->st));
  if (tot > S->mpair_cap) {
    dfree(S->mpairs);
    dfree(S->mirror);
    S->mpair_cap = tot + tot / 4 + 64;
    HIPCHK(S, dalloc(&S->mpairs, S->mpair_cap));
    HIPCHK(S, dalloc(&S->mirror, S->mpair_cap));
  }
  launch_mlp_pair_fill(n, S->ld, A.nbr, A.nall, S->mstart, S->mpairs, S->mirror, S->err, S->st);
  S->npair = tot;
  S->tab_ok[0] = S->tab_ok[1] = false;
  return SL_OK;
}

// Table of the learned potential at the positions of buffer b.
int ensure_table(sl_system *S, int b) {
  if (!S->mlp || S->mlp_mode != SL_MLP_PAIRWISE || S->tab_ok[b]) return SL_OK;
  Atoms &A = S->a[S->cur];
  MlpTableArgs T;
  T.npair = S->npair;
  T.ld = S->ld;
  T.pairs = S->mpairs;
  T.mirror = S->mirror;
  T.nbr = A.nbr;
  T.rx = A.rx[b];
  T.ry = A.ry[b];
  T.rz = A.rz[b];
  for (int d = 0; d < 3; ++d) {
    T.L[d] = S->L[d];
    T.invL[d] = S->invL[d];
  }
  T.tab = S->tab[b];
  {
    ProfScope ps(S, 3, (double)S->npair);
    MlpCfgDev cfg = S->mlp->cfg();
    cfg.jshift = S->pot.ex_shift ? 1 : 0;
    launch_mlp_table(T, S->mlp->w, cfg, S->mlp->yc, S->st);
  }
  S->tab_ok[b] = true;
  return SL_OK;
}

// Exchange coefficients of buffer b's positions for the spin phases (once
// per drift; the analytic potential only).
template <typename real>
int ensure_jcache(sl_system *S, int b) {
  if ((S->mlp && S->mlp_mode != SL_MLP_SPLINE) || S->jcache <= 0 || S->pc.soc_on || S->jc_ok[b])
    return SL_OK;
  if (!S->jc[b]) {
    real *p = nullptr;
    HIPCHK(S, dalloc(&p, (size_t)S->ld * S->max_nbr));
    S->jc[b] = p;
  }
  SysView<real> v = view<real>(S, b);
  {
    ProfScope ps(S, 3, (double)S->n);
    launch_jcache<real>(v, S->pc, (real *)S->jc[b], S->pot.ex_rc * S->pot.ex_rc, S->st);
  }
  S->jc_ok[b] = true;
  return SL_OK;
}

// Colour classes (repairing the previous colouring when there is one) and
// permutation of all per-atom arrays into (colour, cell) order.
int colour_and_permute(sl_system *S, bool repair) {
  ProfScope ps(S, 2, 0.0);
  const int n = S->n;
  CellGrid G;
  {
    Atoms &A = S->a[S->cur];
    cell_grid(S, G);
    CHK(ensure_cells(S, S->ncell));
    launch_zero_i(S->ncell, S->ccount, S->st);
    launch_cell_assign(n, A.rx[S->pos], A.ry[S->pos], A.rz[S->pos], G, A.cell, S->ccount, S->st);
    launch_keys(n, A.rx[S->pos], A.ry[S->pos], A.rz[S->pos], S->L, S->kx, S->ky, S->kz, S->st);
  }
  ColourArgs C = colour_args(S);
  // the palette of a full colouring (or of a colouring the caller set) is
  // the base one; a repair drops atoms outside it so they can move back
  bool set_base = !(repair && S->have_colour);
  if (!S->have_colour) {
    launch_colour_fill(n, C.colour, -1, S->st);
  } else if (repair) {
    launch_colour_mark(C, S->ctmp, S->st);
    HIPCHK(S, hipMemcpyAsync(C.colour, S->ctmp, sizeof(int) * n, hipMemcpyDeviceToDevice, S->st));
  }
  CHK(jp_rounds(S, C));
  int mc = -1;
  for (int attempt = 0; attempt < 2; ++attempt) {
    HIPCHK(S, hipMemsetAsync(S->maxc, 0xff, sizeof(int), S->st));
    launch_colour_stats(C, S->maxc, S->err, S->st);
    HIPCHK(S, hipMemcpyAsync(&mc, S->maxc, sizeof(int), hipMemcpyDeviceToHost, S->st));
    CHK(read_err(S));
    CHK(sticky_code(S));
    if (mc + 1 <= 32 || attempt == 1) break;
    launch_colour_fill(n, C.colour, -1, S->st);  // too many colours: start over
    CHK(jp_rounds(S, C));
    set_base = true;
  }
  S->K = n > 0 ? mc + 1 : 0;
  if (set_base) S->Kbase = S->K;
  S->have_colour = true;

  // permutation: counting sort by colour * ncell + cell, buckets in old order
  const int nbin = S->K * S->ncell;
  CHK(ensure_bins(S, nbin));
  Atoms &A = S->a[S->cur];
  Atoms &B = S->a[1 - S->cur];
  launch_zero_i(nbin, S->bcount, S->st);
  launch_sort_key(n, A.colour, A.cell, S->ncell, S->skey, S->bcount, S->st);
  launch_scan(S->bcount, S->bstart, nbin, S->st);
  launch_zero_i(nbin, S->bfill, S->st);
  launch_bucket_scatter(n, S->skey, S->bstart, S->bfill, S->perm, S->st);
  launch_bucket_sort(nbin, S->bstart, S->perm, S->st);
  launch_inverse(n, S->perm, S->inv, S->st);
  PermuteArgs P;
  std::memset(&P, 0, sizeof(P));
  P.n = n;
  P.perm = S->perm;
  int k = 0;
  for (int b = 0; b < 2; ++b) {
    P.src_d[k] = A.rx[b]; P.dst_d[k++] = B.rx[b];
    P.src_d[k] = A.ry[b]; P.dst_d[k++] = B.ry[b];
    P.src_d[k] = A.rz[b]; P.dst_d[k++] = B.rz[b];
  }
  P.src_d[k] = A.vx; P.dst_d[k++] = B.vx;
  P.src_d[k] = A.vy; P.dst_d[k++] = B.vy;
  P.src_d[k] = A.vz; P.dst_d[k++] = B.vz;
  P.src_d[k] = A.bx; P.dst_d[k++] = B.bx;
  P.src_d[k] = A.by; P.dst_d[k++] = B.by;
  P.src_d[k] = A.bz; P.dst_d[k++] = B.bz;
  P.src_d[k] = A.mass; P.dst_d[k++] = B.mass;
  if (S->prec == SL_FP64) {
    P.src_d[k] = (const double *)A.sx; P.dst_d[k++] = (double *)B.sx;
    P.src_d[k] = (const double *)A.sy; P.dst_d[k++] = (double *)B.sy;
    P.src_d[k] = (const double *)A.sz; P.dst_d[k++] = (double *)B.sz;
  } else {
    P.src_f[0] = (const float *)A.sx; P.dst_f[0] = (float *)B.sx;
    P.src_f[1] = (const float *)A.sy; P.dst_f[1] = (float *)B.sy;
    P.src_f[2] = (const float *)A.sz; P.dst_f[2] = (float *)B.sz;
    P.nf = 3;
  }
  P.nd = k;
  P.src_i[0] = A.id; P.dst_i[0] = B.id;
  P.src_i[1] = A.colour; P.dst_i[1] = B.colour;
  P.src_i[2] = A.cell; P.dst_i[2] = B.cell;
  P.ni = 3;
  launch_permute_atoms(P, S->st);
  launch_permute_nbr(n, S->ld, S->perm, S->inv, A.nbr, A.nspin, A.nall, B.nbr, B.nspin, B.nall, S->st);
  S->cur = 1 - S->cur;
  S->jc_ok[0] = S->jc_ok[1] = false;
  // class offsets = bucket starts of the first cell of every colour
  std::vector<int> bs(nbin + 1);
  HIPCHK(S, hipMemcpyAsync(bs.data(), S->bstart, sizeof(int) * (nbin + 1), hipMemcpyDeviceToHost, S->st));
  HIPCHK(S, hipStreamSynchronize(S->st));
  S->class_off.assign(S->K + 1, 0);
  for (int c = 0; c <= S->K; ++c) S->class_off[c] = bs[(size_t)c * S->ncell];
  {
    Atoms &N = S->a[S->cur];
    launch_watch_mask(n, S->ld, N.nbr, N.nspin, N.colour, N.wmask, S->st);
  }
  if (S->mlp) CHK(mlp_pairs(S));
  return SL_OK;
}

// Full rebuild at the current boundary: cells, lists, colour repair, order.
int rebuild(sl_system *S) {
  if (S->user_list) return colour_and_permute(S, false);
  CHK(check_box(S));
  {
    ProfScope ps(S, 2, (double)S->n);
    CellGrid G;
    CHK(bin_cells(S, G));
    Atoms &A = S->a[S->cur];
    NbrBuildArgs B;
    B.n = S->n;
    B.ld = S->ld;
    B.max_nbr = S->max_nbr;
    B.max_spin = S->max_spin;
    const double rs = spin_radius(S), rl = std::max(list_radius(S), rs);
    B.rs2 = rs * rs;
    B.rl2 = rl * rl;
    B.G = G;
    B.rx = A.rx[S->pos];
    B.ry = A.ry[S->pos];
    B.rz = A.rz[S->pos];
    B.cell = A.cell;
    B.cstart = S->cstart;
    B.catoms = S->catoms;
    B.nbr = A.nbr;
    B.nspin = A.nspin;
    B.nall = A.nall;
    B.bx = A.bx;
    B.by = A.by;
    B.bz = A.bz;
    B.err = S->err;
    B.seen = S->seen;
    B.row_q = S->row_q;
    HIPCHK(S, hipMemsetAsync(S->seen, 0, 2 * sizeof(int), S->st));
    launch_nbr_build(B, S->st);
    int seen[2] = {0, 0};
    HIPCHK(S, hipMemcpyAsync(seen, S->seen, sizeof(seen), hipMemcpyDeviceToHost, S->st));
    CHK(read_err(S));
    S->seen_spin = seen[0];
    S->seen_all = seen[1];
    CHK(sticky_code(S));
  }
  S->have_list = true;
  S->rebuilds++;
  return colour_and_permute(S, true);
}

int ensure_ready(sl_system *S) {
  if (!S->have_state) return fail(S, SL_E_STATE, "no state set");
  if (!S->have_pot) return fail(S, SL_E_STATE, "no potential set");
  if (!S->have_list) {
    CHK(rebuild(S));
  } else if (!S->have_colour) {
    CHK(colour_and_permute(S, false));
  }
  return SL_OK;
}

// --- launches ---------------------------------------------------------------
double noise_amp(const sl_system *S, double h);

// One launch of class c: nrep successive updates at buffer posbuf, or with
// dual set the two updates across the drift (the first at posbuf, the
// second at the other buffer).
template <typename real>
void spin_launch(sl_system *S, int posbuf, int c, int nrep, const int64_t *steps, const int *subs,
                 double h, bool dual = false) {
  SpinPhaseArgs A;
  std::memset(&A, 0, sizeof(A));
  A.begin = S->class_off[c];
  A.end = S->class_off[c + 1];
  A.nrep = nrep;
  A.h = h;
  A.amp = noise_amp(S, h);
  for (int r = 0; r < nrep; ++r) {
    A.step[r] = steps[r];
    A.sub[r] = subs[r];
  }
  A.seed = S->prm.seed;
  A.replica = S->prm.replica;
  A.rs2 = S->pot.ex_rc * S->pot.ex_rc;
  ProfScope ps(S, 0, (double)(A.end - A.begin) * nrep);  // atom updates
  if (dual) {
    const SysView<real> v2 = view<real>(S, 1 - posbuf);
    launch_spin_phase<real>(view<real>(S, posbuf), S->pc, A, S->spin_lanes, S->st, &v2);
  } else {
    launch_spin_phase<real>(view<real>(S, posbuf), S->pc, A, S->spin_lanes, S->st);
  }
}

// A run of dt/4 updates (class, step, sub) applied in order. Consecutive
// updates of one class are merged into one launch (up to kMaxRep); runs of
// consecutive small classes go to one single-workgroup launch.
struct Upd {
  int c;
  int64_t step;
  int sub;
};

constexpr int kTailTotalMax = 4096;  // atoms of one fused run

struct Item {
  int c, nrep;
  int64_t steps[kMaxRep];
  int subs[kMaxRep];
};

double noise_amp(const sl_system *S, double h) {
  if (!S->pc.langevin) return 0.0;
  const double lam = S->pot.lambda;
  const double DS = lam * (1.0 + lam * lam) * kKb * S->pot.temperature / kHbar;
  return std::sqrt(2.0 * DS / std::fabs(h));
}

// Sectored / serial ordering (Sec. 5.1, Eq. spin_ST_sectoring): classes and
// subdomains of the atoms at the positions of buffer posbuf, sorted by
// (class, subdomain, id).
int sect_classes(const sl_system *S) { return S->ordering == SL_ORDER_SECTORS ? 8 : 1; }
int sect_nproc(const sl_system *S) {
  return S->ordering == SL_ORDER_SECTORS ? S->sgrid[0] * S->sgrid[1] * S->sgrid[2] : 1;
}

int sect_prepare(sl_system *S, int posbuf) {
  const int n = S->n, np = sect_nproc(S), nb = sect_classes(S) * np;
  if (!S->skeys[0]) {
    for (int b = 0; b < 2; ++b) {
      HIPCHK(S, dalloc(&S->skeys[b], (size_t)n));
      HIPCHK(S, dalloc(&S->svals[b], (size_t)n));
    }
  }
  if (nb + 1 > S->s_nbins_cap) {
    dfree(S->scount);
    dfree(S->soff);
    S->scount = S->soff = nullptr;
    S->s_nbins_cap = 0;
    HIPCHK(S, dalloc(&S->scount, (size_t)nb + 1));
    HIPCHK(S, dalloc(&S->soff, (size_t)nb + 1));
    S->s_nbins_cap = nb + 1;
  }
  Atoms &A = S->a[S->cur];
  SectKeyArgs K;
  std::memset(&K, 0, sizeof(K));
  K.n = n;
  K.rx = A.rx[posbuf];
  K.ry = A.ry[posbuf];
  K.rz = A.rz[posbuf];
  for (int d = 0; d < 3; ++d) {
    K.L[d] = S->L[d];
    K.g[d] = S->sgrid[d];
  }
  K.nproc = np;
  K.serial = S->ordering == SL_ORDER_SERIAL ? 1 : 0;
  K.id = A.id;
  K.keys = S->skeys[0];
  K.vals = S->svals[0];
  K.count = S->scount;
  launch_zero_i(nb + 1, S->scount, S->st);
  launch_sect_keys(K, S->st);
  if (sect_sort(K, nb, S->skeys[1], S->svals[1], S->soff, &S->cub_tmp, &S->cub_bytes, S->st))
    return fail(S, SL_E_HIP, "sector sort failed");
  return SL_OK;
}

// One spin half-step in the sectored / serial order: classes forward with
// sub-update sub_fwd, then backward with sub_fwd + 1.
template <typename real>
void sect_half(sl_system *S, int posbuf, int64_t step, int sub_fwd, double h) {
  (void)ensure_jcache<real>(S, posbuf);
  const int nc = sect_classes(S);
  SectPhaseArgs A;
  std::memset(&A, 0, sizeof(A));
  A.nproc = sect_nproc(S);
  A.off = S->soff;
  A.order = S->svals[1];
  A.h = h;
  A.amp = noise_amp(S, h);
  A.rs2 = S->pot.ex_rc * S->pot.ex_rc;
  A.step = step;
  A.seed = S->prm.seed;
  A.replica = S->prm.replica;
  const SysView<real> v = view<real>(S, posbuf);
  for (int q = 0; q < 2 * nc; ++q) {
    A.backward = q >= nc ? 1 : 0;
    A.cls = q < nc ? q : 2 * nc - 1 - q;
    A.sub = sub_fwd + A.backward;
    ProfScope ps(S, 0, (double)S->n / nc);
    launch_sect_phase<real>(v, S->pc, A, S->st);
  }
}

template <typename real>
void run_updates(sl_system *S, int posbuf, const std::vector<Upd> &u, double h) {
  (void)ensure_table(S, posbuf);
  (void)ensure_jcache<real>(S, posbuf);
  std::vector<Item> items;
  for (size_t i = 0; i < u.size();) {
    Item it;
    it.c = u[i].c;
    it.nrep = 0;
    while (i < u.size() && u[i].c == it.c && it.nrep < kMaxRep) {
      it.steps[it.nrep] = u[i].step;
      it.subs[it.nrep] = u[i].sub;
      ++it.nrep;
      ++i;
    }
    items.push_back(it);
  }
  auto size_of = [&](int c) { return S->class_off[c + 1] - S->class_off[c]; };
  size_t q = 0;
  while (q < items.size()) {
    size_t r = q;
    long tot = 0, upd = 0;
    while (r < items.size() && (int)(r - q) < kMaxTail) {
      const int sz = size_of(items[r].c);
      if (sz > S->small_class || tot + sz > kTailTotalMax) break;
      tot += sz;
      upd += (long)sz * items[r].nrep;
      ++r;
    }
    if (r - q >= 2) {
      TailArgs T;
      std::memset(&T, 0, sizeof(T));
      T.nitems = (int)(r - q);
      for (size_t k = q; k < r; ++k) {
        TailItem &ti = T.item[k - q];
        ti.begin = S->class_off[items[k].c];
        ti.end = S->class_off[items[k].c + 1];
        ti.nrep = items[k].nrep;
        for (int e = 0; e < items[k].nrep; ++e) {
          ti.step[e] = items[k].steps[e];
          ti.sub[e] = items[k].subs[e];
        }
      }
      T.h = h;
      T.amp = noise_amp(S, h);
      T.seed = S->prm.seed;
      T.replica = S->prm.replica;
      T.rs2 = S->pot.ex_rc * S->pot.ex_rc;
      ProfScope ps(S, 0, (double)upd);
      launch_spin_tail<real>(view<real>(S, posbuf), S->pc, T, S->spin_lanes, S->st);
      q = r;
    } else {
      spin_launch<real>(S, posbuf, items[q].c, items[q].nrep, items[q].steps, items[q].subs, h);
      ++q;
    }
  }
}

// Forward (classes 1..K) then backward (K..1) sweep of one spin half-step.
void half_step_updates(const sl_system *S, int64_t step, int sub_fwd, std::vector<Upd> &u) {
  for (int c = 0; c < S->K; ++c) u.push_back({c, step, sub_fwd});
  for (int c = S->K - 1; c >= 0; --c) u.push_back({c, step, sub_fwd + 1});
}

// With split set, the pair pass of this boundary (pair_launch) has filled
// S->fp and the launch is the spin pass.
template <typename real>
int force_launch(sl_system *S, int posbuf, int mode, double dt, int64_t boundary,
                 bool split = false) {
  Atoms &A = S->a[S->cur];
  ForceArgs F;
  std::memset(&F, 0, sizeof(F));
  F.mode = mode;
  F.dt = dt;
  F.ftm2v = 1.0 / kMvv2e;
  F.mass = A.mass;
  F.vx = A.vx;
  F.vy = A.vy;
  F.vz = A.vz;
  F.nx = A.rx[1 - posbuf];
  F.ny = A.ry[1 - posbuf];
  F.nz = A.rz[1 - posbuf];
  F.bx = A.bx;
  F.by = A.by;
  F.bz = A.bz;
  F.partial = S->partial;
  F.dslot = S->dslot;
  F.done = S->done;
  F.pred = S->pred;
  F.err = S->err;
  F.wmask = A.wmask;
  F.frozen = S->prm.frozen;
  F.seed = S->prm.seed;
  F.replica = S->prm.replica;
  F.step = boundary;
  F.fp = split ? S->fp : nullptr;
  CHK(ensure_table(S, posbuf));
  if (mode & kModeNext) S->tab_ok[1 - posbuf] = S->jc_ok[1 - posbuf] = false;
  const int slot = (int)(boundary & 3);
  F.host_out = S->ring_dev + 8 * slot;
  if (mode & (kModeFinal | kModeNext)) {
    S->ring[8 * slot + 3] = 0.0;
    S->meta[slot].boundary = boundary;
    S->meta[slot].dt = dt;
    S->meta[slot].rebuilt_after = false;
  }
  {
    ProfScope ps(S, 1, (double)S->n);
    const SysView<real> v = view<real>(S, posbuf);
    if (split) {
      launch_force_spin<real>(v, S->pc, F, S->force_lanes, S->st);
    } else {
      launch_eam_density<real>(v, S->pc, S->st);
      launch_force<real>(v, S->pc, F, S->force_lanes, S->st);
    }
  }
  if (mode & (kModeFinal | kModeNext))
    launch_pred_reduce(S->pred, force_blocks(S->n, S->force_lanes), S->err, F.host_out, S->st);
  if (mode & (kModeFinal | kModeNext)) HIPCHK(S, hipEventRecord(S->ev[slot], S->st));
  return SL_OK;
}

// Split force: whether this system takes it, the second stream, its two
// events and the pair buffer (made on first use), and the pair pass of a
// boundary on the second stream (the embedded-atom density pass first).
bool split_ok(const sl_system *S) {
  return S->overlap > 0 && !S->mlp && (S->force_lanes == 1 || S->force_lanes == 2);
}

int ensure_split(sl_system *S) {
  if (!S->st2) HIPCHK(S, hipStreamCreateWithFlags(&S->st2, hipStreamNonBlocking));
  if (!S->ev_fork) HIPCHK(S, hipEventCreateWithFlags(&S->ev_fork, hipEventDisableTiming));
  if (!S->ev_join) HIPCHK(S, hipEventCreateWithFlags(&S->ev_join, hipEventDisableTiming));
  if (!S->fp) HIPCHK(S, dalloc(&S->fp, (size_t)4 * S->ld));
  return SL_OK;
}

template <typename real>
void pair_launch(sl_system *S, int posbuf, bool energy) {
  ForceArgs F;
  std::memset(&F, 0, sizeof(F));
  F.fp = S->fp;
  F.err = S->err;
  ProfScope ps(S, 4, (double)S->n, S->st2);
  const SysView<real> v = view<real>(S, posbuf);
  launch_eam_density<real>(v, S->pc, S->st2);
  launch_pair<real>(v, S->pc, F, S->force_lanes, energy, S->st2);
}

int record_thermo(sl_system *S, int64_t boundary) {
  const int nb = force_blocks(S->n, S->force_lanes);
  const int k = (int)S->thermo_steps.size();
  if (k >= kThermoCap) return SL_OK;
  launch_reduce8(S->partial, nb, S->thermo + (size_t)k * 8, S->st);
  S->thermo_steps.push_back(boundary);
  return SL_OK;
}

template <typename real>
int energy_now(sl_system *S, double out[8]) {
  CHK(force_launch<real>(S, S->pos, kModeEnergy, 0.0, -1));
  const int nb = force_blocks(S->n, S->force_lanes);
  launch_reduce8(S->partial, nb, S->red_out, S->st);
  HIPCHK(S, hipMemcpyAsync(out, S->red_out, 8 * sizeof(double), hipMemcpyDeviceToHost, S->st));
  CHK(read_err(S));
  return sticky_code(S);
}

// Wait until the force kernel of `boundary` finished and decide from its
// predictor whether the list must be rebuilt before the step after next:
//   D = max|r - r_build| + 2a max|v|        >= skin/2 - 0.01, or
//   W = min watched |r_i - r_j| - 4a max|v| <  ex_rc + 0.01,
// the watched pairs being same-colour spin-segment entries, and a the larger
// of |dt| of the step after `boundary` and |dt_next| of the step to be
// decided (they differ when a call changes dt). When the list was rebuilt at
// that boundary after the predictor was taken, the build positions are that
// boundary's (D term 0) and no same-colour pair is closer than the colour
// radius.
int wait_predictor(sl_system *S, int64_t boundary, double dt_next, bool *due) {
  *due = false;
  const int slot = (int)(boundary & 3);
  if (boundary < 0 || S->meta[slot].boundary != boundary) return SL_OK;
  HIPCHK(S, hipEventSynchronize(S->ev[slot]));
  const double *o = S->ring + 8 * slot;
  if (o[3] != 1.0) return fail(S, SL_E_HIP, "rebuild predictor not written");
  S->sticky |= (int)o[2];
  CHK(sticky_code(S));
  const bool rb = S->meta[slot].rebuilt_after;
  const double adt = std::max(std::fabs(S->meta[slot].dt), std::fabs(dt_next));
  const double D = (rb ? 0.0 : o[0]) + 2.0 * adt * o[1];
  const double W = (rb ? colour_radius(S) : std::sqrt(o[4])) - 4.0 * adt * o[1];
  *due = D >= S->skin / 2.0 - 0.01 ||
         (S->ordering == SL_ORDER_COLOUR && W < S->pot.ex_rc + 0.01);
  return SL_OK;
}

template <typename real>
int step_frozen(sl_system *S, int64_t n, double dt) {
  const double h = dt / 4.0;
  const int te = S->prm.thermo_every;
  int64_t k = 0;
  S->prof_now = S->prof;  // every launch of a frozen run is timed
  while (k < n) {
    // steps up to the next thermo sample go in one merged update list
    int64_t chunk = n - k;
    if (te > 0) {
      const int64_t to_sample = te - (S->step % te);
      chunk = std::min(chunk, to_sample);
    }
    chunk = std::min<int64_t>(chunk, 64);
    if (S->ordering != SL_ORDER_COLOUR) {
      CHK(sect_prepare(S, S->pos));
      for (int64_t q = 0; q < chunk; ++q) {
        sect_half<real>(S, S->pos, S->step + q, 0, h);
        sect_half<real>(S, S->pos, S->step + q, 2, h);
      }
    } else {
      std::vector<Upd> u;
      for (int64_t q = 0; q < chunk; ++q) {
        half_step_updates(S, S->step + q, 0, u);
        half_step_updates(S, S->step + q, 2, u);
      }
      run_updates<real>(S, S->pos, u, h);
    }
    S->step += chunk;
    k += chunk;
    if (te > 0 && S->step % te == 0) {
      CHK(force_launch<real>(S, S->pos, kModeEnergy, 0.0, -1));
      CHK(record_thermo(S, S->step));
    }
  }
  S->prof_now = false;
  return SL_OK;
}

template <typename real>
int step_coupled(sl_system *S, int64_t n, double dt, bool built) {
  const double h = dt / 4.0;
  const int te = S->prm.thermo_every;
  const int64_t k0 = S->step;
  // decision for the first step uses the predictor of the boundary before it
  if (!S->user_list && S->have_D) {
    bool due;
    CHK(wait_predictor(S, k0 - 1, dt, &due));
    if (due) {
      CHK(rebuild(S));
      built = true;
    }
  }
  CHK(force_launch<real>(S, S->pos, kModeNext, dt, k0));
  // a boundary that (re)built the list counts as rebuilt for the predictor
  if (built) S->meta[k0 & 3].rebuilt_after = true;
  S->have_D = true;
  for (int64_t k = k0; k < k0 + n; ++k) {
    // timed steps: the first of the call and every prof_every-th after it
    S->prof_now = S->prof && ((k - k0) % S->prof_every == 0);
    if (k > k0 && !S->user_list) {
      bool due;
      CHK(wait_predictor(S, k - 1, dt, &due));
      if (due) {
        CHK(rebuild(S));
        S->meta[k & 3].rebuilt_after = true;
      }
    }
    const int64_t b = k + 1;
    int mode = kModeFinal;
    if (k + 1 < k0 + n) mode |= kModeNext;
    const bool sample = te > 0 && b % te == 0;
    if (sample) mode |= kModeEnergy;
    // split force: the pair pass of boundary b needs only the positions of
    // b (already drifted into the other buffer), so it runs on the second
    // stream while the spins of this step update
    const bool split = split_ok(S);
    if (split) {
      CHK(ensure_split(S));
      HIPCHK(S, hipEventRecord(S->ev_fork, S->st));
      HIPCHK(S, hipStreamWaitEvent(S->st2, S->ev_fork, 0));
      pair_launch<real>(S, 1 - S->pos, sample);
      HIPCHK(S, hipEventRecord(S->ev_join, S->st2));
    }
    if (S->ordering != SL_ORDER_COLOUR) {
      // classes from the positions at the start of the step
      CHK(sect_prepare(S, S->pos));
      sect_half<real>(S, S->pos, k, 0, h);
      sect_half<real>(S, 1 - S->pos, k, 2, h);
    } else {
      std::vector<Upd> u, w;
      half_step_updates(S, k, 0, u);
      half_step_updates(S, k, 2, w);
      // the first class closes one half-step and opens the next: its two
      // updates around the drift go in one dual launch when it is large
      // enough for its own launch anyway
      const int c0 = u.back().c;
      const bool dual = S->K >= 2 && w.front().c == c0 &&
                        S->class_off[c0 + 1] - S->class_off[c0] > S->small_class;
      if (dual) {
        u.pop_back();
        w.erase(w.begin());
        run_updates<real>(S, S->pos, u, h);
        (void)ensure_table(S, 1 - S->pos);
        (void)ensure_jcache<real>(S, 1 - S->pos);
        const int64_t st2[2] = {k, k};
        const int sb2[2] = {1, 2};
        spin_launch<real>(S, S->pos, c0, 2, st2, sb2, h, true);
        run_updates<real>(S, 1 - S->pos, w, h);
      } else {
        run_updates<real>(S, S->pos, u, h);
        run_updates<real>(S, 1 - S->pos, w, h);
      }
    }
    if (split) HIPCHK(S, hipStreamWaitEvent(S->st, S->ev_join, 0));
    CHK(force_launch<real>(S, 1 - S->pos, mode, dt, b, split));
    if (sample) CHK(record_thermo(S, b));
    S->pos = 1 - S->pos;
    S->step = b;
  }
  S->prof_now = false;
  return SL_OK;
}

int load_aos(sl_system *S, const double *src, int where, std::vector<double> &host) {
  const size_t bytes = sizeof(double) * 3 * (size_t)S->n;
  host.resize(3 * (size_t)S->n);
  if (where == SL_DEVICE) {
    HIPCHK(S, hipMemcpyAsync(host.data(), src, bytes, hipMemcpyDeviceToHost, S->st));
    HIPCHK(S, hipStreamSynchronize(S->st));
  } else {
    std::memcpy(host.data(), src, bytes);
  }
  return SL_OK;
}

}  // namespace

// ============================================================================
extern "C" {

int sl_create(const sl_params *p, sl_system **out) {
  if (!out) return fail(nullptr, SL_E_ARG, "out is NULL");
  *out = nullptr;
  if (!p) return fail(nullptr, SL_E_ARG, "params is NULL");
  if (p->n_atoms < 1 || p->n_atoms > (1 << 28)) return fail(nullptr, SL_E_ARG, "n_atoms out of range");
  if (p->precision != SL_FP64 && p->precision != SL_FP32) return fail(nullptr, SL_E_ARG, "bad precision");
  for (int d = 0; d < 3; ++d)
    if (!(p->box[d] > 0.0) || !std::isfinite(p->box[d])) return fail(nullptr, SL_E_BOX, "box sides must be positive");
  if (p->skin < 0.0) return fail(nullptr, SL_E_ARG, "negative skin");
  if (p->max_nbr < 0 || p->max_spin_nbr < 0 || p->max_spin_nbr > 63)
    return fail(nullptr, SL_E_ARG, "bad neighbour capacities");
  sl_system *S = new sl_system();
  S->prm = *p;
  S->n = (int)p->n_atoms;
  S->ld = (S->n + 63) / 64 * 64;
  S->prec = p->precision;
  for (int d = 0; d < 3; ++d) {
    S->L[d] = p->box[d];
    S->invL[d] = 1.0 / p->box[d];
  }
  S->skin = p->frozen ? 0.0 : p->skin;
  S->max_nbr = p->max_nbr > 0 ? p->max_nbr : 80;
  S->jcache = S->prec == SL_FP32 ? 1 : -1;
  S->max_spin = p->max_spin_nbr > 0 ? p->max_spin_nbr : 32;
  if (S->max_spin > S->max_nbr) S->max_spin = S->max_nbr;
  int rc = SL_OK;
  auto bail = [&](int code) {
    g_create_err = S->last_err;
    sl_destroy(S);
    return code;
  };
  if (p->stream) {
    S->st = (hipStream_t)p->stream;
  } else {
    if (hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking) != hipSuccess) {
      S->st = nullptr;
      S->last_err = "hipStreamCreate failed";
      return bail(SL_E_HIP);
    }
    S->own_stream = true;
  }
  if ((rc = alloc_atoms(S, S->a[0])) || (rc = alloc_atoms(S, S->a[1]))) return bail(rc == SL_E_HIP ? SL_E_NOMEM : rc);
  const int n = S->n;
  const int nb = force_blocks(n, 8);
#define A_(x) if (hipSuccess != (x)) { S->last_err = #x; return bail(SL_E_NOMEM); }
  A_(dalloc(&S->catoms, n));
  A_(dalloc(&S->skey, n));
  A_(dalloc(&S->perm, n));
  A_(dalloc(&S->inv, n));
  A_(dalloc(&S->uinv, n));
  A_(dalloc(&S->ctmp, n));
  A_(dalloc(&S->kx, n));
  A_(dalloc(&S->ky, n));
  A_(dalloc(&S->kz, n));
  A_(dalloc(&S->stage, 3 * (size_t)n));
  A_(dalloc(&S->err, 1));
  A_(dalloc(&S->seen, 2));
  A_(dalloc(&S->jpcnt, 3));
  A_(dalloc(&S->jplist[0], (size_t)n));
  A_(dalloc(&S->jplist[1], (size_t)n));
  A_(dalloc(&S->jpmask[0], (size_t)n));
  A_(dalloc(&S->jpmask[1], (size_t)n));
  A_(dalloc(&S->maxc, 1));
  A_(dalloc(&S->dslot, 3));
  A_(dalloc(&S->done, 1));
  A_(dalloc(&S->partial, (size_t)nb * 8));
  A_(dalloc(&S->pred, (size_t)nb * 3));
  A_(dalloc(&S->red_out, 8));
  A_(dalloc(&S->thermo, (size_t)kThermoCap * 8));
  A_(hipHostMalloc((void **)&S->ring, 32 * sizeof(double), hipHostMallocCoherent | hipHostMallocMapped));
  for (int k = 0; k < 4; ++k) A_(hipEventCreateWithFlags(&S->ev[k], hipEventDisableTiming));
  A_(hipHostGetDevicePointer((void **)&S->ring_dev, S->ring, 0));
#undef A_
  std::memset(S->ring, 0, 32 * sizeof(double));
  (void)hipMemsetAsync(S->err, 0, sizeof(int), S->st);
  {
    // running max slots start at 0, the running min at "no watched pair"
    const double inf = kInf;
    unsigned long long init[3] = {0ull, 0ull, 0ull};
    std::memcpy(&init[2], &inf, sizeof(inf));
    (void)hipMemcpy(S->dslot, init, sizeof(init), hipMemcpyHostToDevice);
  }
  (void)hipMemsetAsync(S->done, 0, sizeof(unsigned int), S->st);
  launch_iota(n, S->a[0].id, S->st);
  if (hipStreamSynchronize(S->st) != hipSuccess) {
    S->last_err = "initial synchronisation failed";
    return bail(SL_E_HIP);
  }
  *out = S;
  return SL_OK;
}

int sl_destroy(sl_system *S) {
  if (!S) return SL_OK;
  if (S->st) (void)hipStreamSynchronize(S->st);
  if (S->st2) (void)hipStreamSynchronize(S->st2);
  for (auto &r : S->prof_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : S->ev_pool) (void)hipEventDestroy(e);
  for (int k = 0; k < 4; ++k)
    if (S->ev[k]) (void)hipEventDestroy(S->ev[k]);
  free_atoms(S->a[0]);
  free_atoms(S->a[1]);
  for (void *p : {(void *)S->ccount, (void *)S->cstart, (void *)S->cfill, (void *)S->catoms,
                  (void *)S->bcount, (void *)S->bstart, (void *)S->bfill, (void *)S->skey,
                  (void *)S->perm, (void *)S->inv, (void *)S->uinv, (void *)S->ctmp,
                  (void *)S->kx, (void *)S->ky, (void *)S->kz, (void *)S->stage, (void *)S->err,
                  (void *)S->seen, (void *)S->jpcnt, (void *)S->maxc, (void *)S->dslot,
                  (void *)S->jplist[0], (void *)S->jplist[1], (void *)S->jpmask[0],
                  (void *)S->jpmask[1],
                  (void *)S->done, (void *)S->partial, (void *)S->pred, (void *)S->red_out, (void *)S->thermo,
                  (void *)S->mpairs, (void *)S->mirror, (void *)S->mcnt, (void *)S->mstart,
                  (void *)S->tab[0], (void *)S->tab[1], S->jc[0], S->jc[1], (void *)S->eam,
                  (void *)S->skeys[0], (void *)S->skeys[1], (void *)S->svals[0],
                  (void *)S->svals[1], (void *)S->scount, (void *)S->soff, S->cub_tmp,
                  (void *)S->fp})
    dfree(p);
  if (S->ev_fork) (void)hipEventDestroy(S->ev_fork);
  if (S->ev_join) (void)hipEventDestroy(S->ev_join);
  if (S->st2) (void)hipStreamDestroy(S->st2);
  if (S->ring) (void)hipHostFree(S->ring);
  if (S->own_stream && S->st) (void)hipStreamDestroy(S->st);
  delete S;
  return SL_OK;
}

int sl_set_potential(sl_system *S, const sl_potential *pot) {
  if (!S || !pot) return fail(S, SL_E_ARG, "NULL argument");
  const double vals[] = {pot->morse_D, pot->morse_alpha, pot->morse_r0, pot->morse_rc,
                         pot->ex_alpha, pot->ex_gamma, pot->ex_delta, pot->ex_rc, pot->zeeman_g,
                         pot->B[0], pot->B[1], pot->B[2], pot->aniso_K, pot->aniso_n[0],
                         pot->aniso_n[1], pot->aniso_n[2], pot->lambda, pot->temperature,
                         pot->lat_gamma, pot->lat_temperature, pot->neel_alpha,
                         pot->neel_gamma, pot->neel_delta, pot->neel_rc, pot->dmi_alpha,
                         pot->dmi_gamma, pot->dmi_delta, pot->dmi_rc, pot->dmi_n[0],
                         pot->dmi_n[1], pot->dmi_n[2]};
  for (double v : vals)
    if (!std::isfinite(v)) return fail(S, SL_E_ARG, "non-finite potential parameter");
  if (pot->ex_delta <= 0.0 || pot->ex_rc < 0.0 || pot->morse_rc < 0.0 || pot->lambda < 0.0 ||
      pot->temperature < 0.0 || pot->lat_gamma < 0.0 || pot->lat_temperature < 0.0)
    return fail(S, SL_E_ARG, "invalid potential parameter");
  const bool neel = pot->neel_alpha != 0.0 && pot->neel_rc > 0.0;
  const bool dmi = pot->dmi_alpha != 0.0 && pot->dmi_rc > 0.0;
  if ((neel && (pot->neel_delta <= 0.0 || pot->neel_rc > pot->ex_rc)) ||
      (dmi && (pot->dmi_delta <= 0.0 || pot->dmi_rc > pot->ex_rc)))
    return fail(S, SL_E_ARG, "Neel/DMI terms need delta > 0 and a cutoff within ex_rc");
  if (dmi) {
    const double nn = pot->dmi_n[0] * pot->dmi_n[0] + pot->dmi_n[1] * pot->dmi_n[1] +
                      pot->dmi_n[2] * pot->dmi_n[2];
    if (std::fabs(nn - 1.0) > 1e-12) return fail(S, SL_E_ARG, "dmi_n must be a unit vector");
  }
  if ((neel || dmi) && S->mlp)
    return fail(S, SL_E_ARG, "Neel/DMI terms need the analytic exchange (a learned pair potential is set)");
  if (pot->eam_on) {
    const double ev[] = {pot->eam_A, pot->eam_d, pot->eam_beta, pot->eam_c, pot->eam_c0,
                         pot->eam_c1, pot->eam_c2};
    for (double v : ev)
      if (!std::isfinite(v)) return fail(S, SL_E_ARG, "non-finite embedded-atom parameter");
    if (pot->eam_A < 0.0 || pot->eam_d <= 0.0 || pot->eam_c <= 0.0)
      return fail(S, SL_E_ARG, "embedded-atom terms need A >= 0, d > 0 and c > 0");
    if (S->mlp) return fail(S, SL_E_ARG, "embedded-atom terms cannot be combined with a learned pair potential");
  }
  if (pot->eam_on && !S->eam) HIPCHK(S, dalloc(&S->eam, 2 * (size_t)S->ld));
  S->pot = *pot;
  S->have_pot = true;
  make_potconst(S);
  CHK(check_box(S));
  if (!S->user_list) S->have_list = false;
  S->have_D = false;
  return SL_OK;
}

int sl_set_state(sl_system *S, const double *r, const double *v, const double *s,
                 const double *mass, int where) {
  if (!S) return fail(S, SL_E_ARG, "NULL system");
  if (where != SL_HOST && where != SL_DEVICE) return fail(S, SL_E_ARG, "bad 'where'");
  if (!S->have_state && (!r || !v || !s || !mass))
    return fail(S, SL_E_ARG, "the first sl_set_state needs r, v, s and mass");
  CHK(sl_synchronize(S));
  const int n = S->n;
  std::vector<double> hr, hv, hs, hm;
  if (r) CHK(load_aos(S, r, where, hr));
  if (v) CHK(load_aos(S, v, where, hv));
  if (s) CHK(load_aos(S, s, where, hs));
  if (mass) {
    hm.resize(n);
    if (where == SL_DEVICE) {
      HIPCHK(S, hipMemcpy(hm.data(), mass, sizeof(double) * n, hipMemcpyDeviceToHost));
    } else {
      std::memcpy(hm.data(), mass, sizeof(double) * n);
    }
  }
  for (auto *vec : {&hr, &hv, &hs, &hm})
    for (double x : *vec)
      if (!std::isfinite(x)) return fail(S, SL_E_NONFINITE, "non-finite value in the state");
  for (double x : hm)
    if (!(x > 0.0)) return fail(S, SL_E_ARG, "masses must be positive");
  for (int i = 0; s && i < n; ++i) {
    const double q = std::sqrt(hs[3 * i] * hs[3 * i] + hs[3 * i + 1] * hs[3 * i + 1] + hs[3 * i + 2] * hs[3 * i + 2]);
    if (std::fabs(q - 1.0) > 1e-12) return fail(S, SL_E_ARG, "spin " + std::to_string(i) + " is not a unit vector");
  }
  Atoms &A = S->a[S->cur];
  auto up = [&](const std::vector<double> &h, double *x, double *y, double *z) -> int {
    HIPCHK(S, hipMemcpyAsync(S->stage, h.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, S->st));
    launch_load_vec(n, A.id, S->stage, x, y, z, S->st);
    HIPCHK(S, hipStreamSynchronize(S->st));
    return SL_OK;
  };
  if (r) CHK(up(hr, A.rx[S->pos], A.ry[S->pos], A.rz[S->pos]));
  if (v) CHK(up(hv, A.vx, A.vy, A.vz));
  if (s) {
    if (S->prec == SL_FP64) {
      CHK(up(hs, (double *)A.sx, (double *)A.sy, (double *)A.sz));
    } else {
      HIPCHK(S, hipMemcpyAsync(S->stage, hs.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, S->st));
      launch_load_vec_f(n, A.id, S->stage, (float *)A.sx, (float *)A.sy, (float *)A.sz, S->st);
      HIPCHK(S, hipStreamSynchronize(S->st));
    }
  }
  if (mass) {
    HIPCHK(S, hipMemcpyAsync(S->stage, hm.data(), sizeof(double) * n, hipMemcpyHostToDevice, S->st));
    launch_load_scalar(n, A.id, S->stage, A.mass, S->st);
    HIPCHK(S, hipStreamSynchronize(S->st));
  }
  S->have_state = true;
  if (!S->user_list) S->have_list = false;
  S->have_colour = false;
  S->have_D = false;
  S->tab_ok[0] = S->tab_ok[1] = false;
  S->jc_ok[0] = S->jc_ok[1] = false;
  S->sticky = 0;
  HIPCHK(S, hipMemsetAsync(S->err, 0, sizeof(int), S->st));
  return SL_OK;
}

int sl_get_state(sl_system *S, double *r, double *v, double *s, int where) {
  if (!S) return fail(S, SL_E_ARG, "NULL system");
  if (!S->have_state) return fail(S, SL_E_STATE, "no state set");
  CHK(sl_synchronize(S));
  const int n = S->n;
  Atoms &A = S->a[S->cur];
  auto down = [&](double *dst, const double *x, const double *y, const double *z, bool f32) -> int {
    if (!dst) return SL_OK;
    if (f32) launch_store_vec_f(n, A.id, (const float *)x, (const float *)y, (const float *)z, S->stage, S->st);
    else launch_store_vec(n, A.id, x, y, z, S->stage, S->st);
    HIPCHK(S, hipMemcpyAsync(dst, S->stage, sizeof(double) * 3 * n,
                             where == SL_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, S->st));
    HIPCHK(S, hipStreamSynchronize(S->st));
    return SL_OK;
  };
  CHK(down(r, A.rx[S->pos], A.ry[S->pos], A.rz[S->pos], false));
  CHK(down(v, A.vx, A.vy, A.vz, false));
  CHK(down(s, (const double *)A.sx, (const double *)A.sy, (const double *)A.sz, S->prec == SL_FP32));
  return SL_OK;
}

int sl_set_neighbor(sl_system *S, double skin, int max_nbr) {
  if (!S) return fail(S, SL_E_ARG, "NULL system");
  if (skin < 0.0 || max_nbr < 0) return fail(S, SL_E_ARG, "bad skin or capacity");
  if (!S->prm.frozen) S->skin = skin;
  if (max_nbr > 0 && max_nbr != S->max_nbr) {
    CHK(sl_synchronize(S));
    dfree(S->a[0].nbr);
    dfree(S->a[1].nbr);
    S->a[0].nbr = S->a[1].nbr = nullptr;
    S->max_nbr = max_nbr;
    if (S->max_spin > max_nbr) S->max_spin = max_nbr;
    HIPCHK(S, dalloc(&S->a[0].nbr, (size_t)S->ld * S->max_nbr));
    HIPCHK(S, dalloc(&S->a[1].nbr, (size_t)S->ld * S->max_nbr));
    for (int b = 0; b < 2; ++b) {
      if (S->tab[b]) {
        dfree(S->tab[b]);
        S->tab[b] = nullptr;
        HIPCHK(S, dalloc(&S->tab[b], (size_t)S->ld * S->max_nbr));
      }
      dfree(S->jc[b]);  // reallocated at the next use with the new capacity
      S->jc[b] = nullptr;
      S->jc_ok[b] = false;
    }
  }
  S->user_list = false;
  S->have_list = false;
  S->have_D = false;
  if (S->have_pot) CHK(check_box(S));
  return SL_OK;
}

int sl_set_neighbor_list(sl_system *S, const int *offsets, const int *idx, int where) {
  if (!S || !offsets) return fail(S, SL_E_ARG, "NULL argument");
  if (!S->have_state || !S->have_pot) return fail(S, SL_E_STATE, "set state and potential first");
  CHK(sl_synchronize(S));
  const int n = S->n;
  std::vector<int> off(n + 1);
  if (where == SL_DEVICE) HIPCHK(S, hipMemcpy(off.data(), offsets, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
  else std::memcpy(off.data(), offsets, sizeof(int) * (n + 1));
  if (off[0] != 0) return fail(S, SL_E_ARG, "offsets[0] must be 0");
  for (int i = 0; i < n; ++i)
    if (off[i + 1] < off[i]) return fail(S, SL_E_ARG, "offsets must be non-decreasing");
  const int tot = off[n];
  std::vector<int> ix(tot);
  if (tot > 0) {
    if (!idx) return fail(S, SL_E_ARG, "idx is NULL");
    if (where == SL_DEVICE) HIPCHK(S, hipMemcpy(ix.data(), idx, sizeof(int) * tot, hipMemcpyDeviceToHost));
    else std::memcpy(ix.data(), idx, sizeof(int) * tot);
  }
  for (int i = 0; i < n; ++i)
    for (int p = off[i]; p < off[i + 1]; ++p)
      if (ix[p] < 0 || ix[p] >= n || ix[p] == i) return fail(S, SL_E_ARG, "neighbour index out of range");
  int *doff = nullptr, *didx = nullptr;
  HIPCHK(S, dalloc(&doff, n + 1));
  HIPCHK(S, dalloc(&didx, tot));
  HIPCHK(S, hipMemcpy(doff, off.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice));
  if (tot > 0) HIPCHK(S, hipMemcpy(didx, ix.data(), sizeof(int) * tot, hipMemcpyHostToDevice));
  Atoms &A = S->a[S->cur];
  launch_user_inverse(n, A.id, S->uinv, S->st);
  CsrArgs C;
  C.n = n;
  C.ld = S->ld;
  C.max_nbr = S->max_nbr;
  C.off = doff;
  C.idx = didx;
  C.id = A.id;
  C.uinv = S->uinv;
  C.rx = A.rx[S->pos];
  C.ry = A.ry[S->pos];
  C.rz = A.rz[S->pos];
  for (int d = 0; d < 3; ++d) {
    C.L[d] = S->L[d];
    C.invL[d] = S->invL[d];
  }
  const double rs = spin_radius(S);
  C.rs2 = rs * rs;
  C.nbr = A.nbr;
  C.nspin = A.nspin;
  C.nall = A.nall;
  C.bx = A.bx;
  C.by = A.by;
  C.bz = A.bz;
  C.err = S->err;
  launch_csr_to_ell(C, S->st);
  CHK(read_err(S));
  dfree(doff);
  dfree(didx);
  CHK(sticky_code(S));
  S->user_list = true;
  S->have_list = true;
  S->have_D = false;
  return SL_OK;
}

int64_t sl_get_neighbor_list(sl_system *S, int *nspin, int *nall, int *idx, int64_t cap) {
  if (!S) return fail(S, SL_E_ARG, "NULL system");
  if (!S->have_list) return fail(S, SL_E_STATE, "no neighbour list");
  CHK(sl_synchronize(S));
  const int n = S->n;
  Atoms &A = S->a[S->cur];
  std::vector<int> ns(n), na(n), id(n), nb((size_t)S->ld * S->max_nbr);
  HIPCHK(S, hipMemcpy(ns.data(), A.nspin, sizeof(int) * n, hipMemcpyDeviceToHost));
  HIPCHK(S, hipMemcpy(na.data(), A.nall, sizeof(int) * n, hipMemcpyDeviceToHost));
  HIPCHK(S, hipMemcpy(id.data(), A.id, sizeof(int) * n, hipMemcpyDeviceToHost));
  HIPCHK(S, hipMemcpy(nb.data(), A.nbr, sizeof(int) * nb.size(), hipMemcpyDeviceToHost));
  std::vector<int> uinv(n);
  for (int i = 0; i < n; ++i) uinv[id[i]] = i;
  int64_t tot = 0;
  for (int u = 0; u < n; ++u) {
    const int i = uinv[u];
    if (nspin) nspin[u] = ns[i];
    if (nall) nall[u] = na[i];
    tot += na[i];
  }
  if (idx && cap >= tot) {
    int64_t p = 0;
    for (int u = 0; u < n; ++u) {
      const int i = uinv[u];
      for (int k = 0; k < na[i]; ++k) idx[p++] = id[nb[(size_t)k * S->ld + i]];
    }
  }
  return tot;
}

int sl_set_coloring(sl_system *S, const int *colour, int where) {
  if (!S || !colour) return fail(S, SL_E_ARG, "NULL argument");
  CHK(ensure_ready(S));
  CHK(sl_synchronize(S));
  const int n = S->n;
  std::vector<int> cu(n), id(n), ci(n);
  if (where == SL_DEVICE) HIPCHK(S, hipMemcpy(cu.data(), colour, sizeof(int) * n, hipMemcpyDeviceToHost));
  else std::memcpy(cu.data(), colour, sizeof(int) * n);
  for (int x : cu)
    if (x < 0 || x > 63) return fail(S, SL_E_ARG, "colours must lie in 0..63");
  Atoms &A = S->a[S->cur];
  HIPCHK(S, hipMemcpy(id.data(), A.id, sizeof(int) * n, hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i) ci[i] = cu[id[i]];
  HIPCHK(S, hipMemcpy(A.colour, ci.data(), sizeof(int) * n, hipMemcpyHostToDevice));
  ColourArgs C = colour_args(S);
  HIPCHK(S, hipMemsetAsync(S->maxc, 0xff, sizeof(int), S->st));
  launch_colour_stats(C, S->maxc, S->err, S->st);
  CHK(read_err(S));
  if (S->sticky & kErrColour) {
    S->sticky &= ~kErrColour;
    HIPCHK(S, hipMemsetAsync(S->err, 0, sizeof(int), S->st));
    HIPCHK(S, hipStreamSynchronize(S->st));
    S->have_colour = false;
    return fail(S, SL_E_COLOR, "colouring puts two interacting spins in one class");
  }
  S->have_colour = true;
  return colour_and_permute(S, false);
}

int sl_get_coloring(sl_system *S, int *colour, int *K) {
  if (!S) return fail(S, SL_E_ARG, "NULL system");
  CHK(sl_synchronize(S));
  if (K) *K = S->have_colour ? S->K : 0;
  if (!colour) return SL_OK;
  const int n = S->n;
  if (!S->have_colour) {
    for (int i = 0; i < n; ++i) colour[i] = -1;
    return SL_OK;
  }
  Atoms &A = S->a[S->cur];
  std::vector<int> id(n), ci(n);
  HIPCHK(S, hipMemcpy(id.data(), A.id, sizeof(int) * n, hipMemcpyDeviceToHost));
  HIPCHK(S, hipMemcpy(ci.data(), A.colour, sizeof(int) * n, hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i) colour[id[i]] = ci[i];
  return SL_OK;
}

int sl_set_step(sl_system *S, int64_t step) {
  if (!S) return fail(S, SL_E_ARG, "NULL system");
  CHK(sl_synchronize(S));
  S->step = step;
  for (auto &m : S->meta) m = SlotMeta();
  S->have_D = false;
  return SL_OK;
}

int sl_step(sl_system *S, int64_t n, double dt) {
  if (!S) return fail(S, SL_E_ARG, "NULL system");
  if (n < 0 || !std::isfinite(dt)) return fail(S, SL_E_ARG, "bad step count or dt");
  const int64_t rb0 = S->rebuilds;
  CHK(ensure_ready(S));
  CHK(sticky_code(S));
  if (n == 0) return SL_OK;
  if (S->prm.frozen)
    return S->prec == SL_FP64 ? step_frozen<double>(S, n, dt) : step_frozen<float>(S, n, dt);
  const bool built = S->rebuilds != rb0;  // the list was built at this boundary
  return S->prec == SL_FP64 ? step_coupled<double>(S, n, dt, built)
                            : step_coupled<float>(S, n, dt, built);
}

int sl_get_energy(sl_system *S, sl_energy *out) {
  if (!S || !out) return fail(S, SL_E_ARG, "NULL argument");
  CHK(sl_synchronize(S));
  CHK(ensure_ready(S));
  double e[8];
  CHK(S->prec == SL_FP64 ? energy_now<double>(S, e) : energy_now<float>(S, e));
  out->kin = e[0];
  out->pair = e[1];
  out->exchange = e[2];
  out->zeeman = e[3];
  out->aniso = e[4];
  out->total = e[0] + e[1] + e[2] + e[3] + e[4];
  return SL_OK;
}

int sl_get_magnetization(sl_system *S, double M[3]) {
  if (!S || !M) return fail(S, SL_E_ARG, "NULL argument");
  CHK(sl_synchronize(S));
  CHK(ensure_ready(S));
  double e[8];
  CHK(S->prec == SL_FP64 ? energy_now<double>(S, e) : energy_now<float>(S, e));
  M[0] = e[5];
  M[1] = e[6];
  M[2] = e[7];
  return SL_OK;
}

int sl_get_thermo(sl_system *S, int max, int64_t *steps, sl_energy *e, double *M, int *count) {
  if (!S) return fail(S, SL_E_ARG, "NULL system");
  CHK(sl_synchronize(S));
  const int avail = (int)S->thermo_steps.size() - S->thermo_read;
  const int k = std::max(0, std::min(max, avail));
  if (k > 0) {
    std::vector<double> buf((size_t)k * 8);
    HIPCHK(S, hipMemcpy(buf.data(), S->thermo + (size_t)S->thermo_read * 8, sizeof(double) * 8 * k,
                        hipMemcpyDeviceToHost));
    for (int q = 0; q < k; ++q) {
      const double *b = &buf[(size_t)q * 8];
      if (steps) steps[q] = S->thermo_steps[S->thermo_read + q];
      if (e) {
        e[q].kin = b[0]; e[q].pair = b[1]; e[q].exchange = b[2]; e[q].zeeman = b[3]; e[q].aniso = b[4];
        e[q].total = b[0] + b[1] + b[2] + b[3] + b[4];
      }
      if (M) { M[3 * q] = b[5]; M[3 * q + 1] = b[6]; M[3 * q + 2] = b[7]; }
    }
    S->thermo_read += k;
  }
  if (S->thermo_read == (int)S->thermo_steps.size()) {
    S->thermo_steps.clear();
    S->thermo_read = 0;
  }
  if (count) *count = k;
  return SL_OK;
}

int sl_get_stats(sl_system *S, sl_stats *out) {
  if (!S || !out) return fail(S, SL_E_ARG, "NULL argument");
  out->step = S->step;
  out->rebuilds = S->rebuilds;
  out->n_colours = S->have_colour ? S->K : 0;
  out->jp_rounds = S->jp_rounds;
  out->max_spin_nbr_seen = S->seen_spin;
  out->max_nbr_seen = S->seen_all;
  return SL_OK;
}

int sl_synchronize(sl_system *S) {
  if (!S) return fail(S, SL_E_ARG, "NULL system");
  HIPCHK(S, hipStreamSynchronize(S->st));
  CHK(read_err(S));
  return sticky_code(S);
}

int sl_set_mlp(sl_system *S, sl_mlp *m) {
  if (!S) return fail(S, SL_E_ARG, "NULL system");
  CHK(sl_synchronize(S));
  if (m) {
    if (S->prec != SL_FP32) return fail(S, SL_E_ARG, "the learned potential runs in the FP32 form");
    if (!m->have_weights) return fail(S, SL_E_STATE, "the MLP has no weights");
    if (S->pc.soc_on) return fail(S, SL_E_ARG, "the Neel/DMI terms need the analytic exchange");
    if (S->pc.eam_on) return fail(S, SL_E_ARG, "embedded-atom terms cannot be combined with a learned pair potential");
    (void)hipStreamSynchronize(m->st);
    for (int b = 0; b < 2; ++b)
      if (!S->tab[b]) HIPCHK(S, dalloc(&S->tab[b], (size_t)S->ld * S->max_nbr));
    if (!S->mcnt) {
      HIPCHK(S, dalloc(&S->mcnt, S->n));
      HIPCHK(S, dalloc(&S->mstart, S->n + 1));
    }
  }
  S->mlp = m;
  S->tab_ok[0] = S->tab_ok[1] = false;
  S->jc_ok[0] = S->jc_ok[1] = false;
  if (m && S->have_list && S->have_colour) CHK(mlp_pairs(S));
  return SL_OK;
}

int sl_set_mlp_mode(sl_system *S, int mode) {
  if (!S || !(mode == SL_MLP_PAIRWISE || mode == SL_MLP_SPLINE))
    return fail(S, SL_E_ARG, "mode must be SL_MLP_PAIRWISE or SL_MLP_SPLINE");
  CHK(sl_synchronize(S));
  S->mlp_mode = mode;
  S->tab_ok[0] = S->tab_ok[1] = false;
  S->jc_ok[0] = S->jc_ok[1] = false;
  return SL_OK;
}

int sl_set_tuning(sl_system *S, const sl_tuning *t) {
  if (!S || !t) return fail(S, SL_E_ARG, "NULL argument");
  auto ok = [](int x) { return x == 0 || x == 1 || x == 2 || x == 4 || x == 8; };
  if (!ok(t->spin_lanes) || !ok(t->force_lanes)) return fail(S, SL_E_ARG, "lanes must be 1, 2, 4 or 8");
  if (t->small_class < -1) return fail(S, SL_E_ARG, "small_class must be >= -1");
  if (t->jcache < -1 || t->jcache > 1) return fail(S, SL_E_ARG, "jcache must be -1, 0 or 1");
  if (t->overlap < -1 || t->overlap > 1) return fail(S, SL_E_ARG, "overlap must be -1, 0 or 1");
  CHK(sl_synchronize(S));
  S->spin_lanes = t->spin_lanes ? t->spin_lanes : 2;
  S->force_lanes = t->force_lanes ? t->force_lanes : 1;
  S->small_class = t->small_class == 0 ? 512 : t->small_class;
  S->jcache = t->jcache == 0 ? (S->prec == SL_FP32 ? 1 : -1) : t->jcache;
  S->overlap = t->overlap == 0 ? -1 : t->overlap;
  return SL_OK;
}

int sl_get_tuning(sl_system *S, sl_tuning *t) {
  if (!S || !t) return fail(S, SL_E_ARG, "NULL argument");
  t->spin_lanes = S->spin_lanes;
  t->force_lanes = S->force_lanes;
  t->small_class = S->small_class;
  t->jcache = S->jcache;
  t->overlap = S->overlap;
  return SL_OK;
}

int sl_set_profiling(sl_system *S, int on) {
  if (!S) return fail(S, SL_E_ARG, "NULL system");
  if (S->prof && !on) prof_collect(S);  // totals stay readable after stopping
  if (on < 0) return fail(S, SL_E_ARG, "profiling period must be >= 0");
  if (on && !S->prof)
    for (int k = 0; k < 5; ++k) {        // a new measurement starts from zero
      S->prof_launch[k] = 0;
      S->prof_ms[k] = 0.0;
      S->prof_work[k] = 0.0;
    }
  S->prof = on != 0;
  S->prof_every = on > 1 ? on : 1;
  S->prof_now = false;  // set per step inside sl_step
  return SL_OK;
}

int sl_get_profile(sl_system *S, int kind, int64_t *launches, double *ms, double *work_items) {
  if (!S || kind < 0 || kind > 4) return fail(S, SL_E_ARG, "bad argument");
  prof_collect(S);
  if (launches) *launches = S->prof_launch[kind];
  if (ms) *ms = S->prof_ms[kind];
  if (work_items) *work_items = S->prof_work[kind];
  return SL_OK;
}

const char *sl_last_error(const sl_system *S) {
  if (!S) return g_create_err.c_str();
  return S->last_err.c_str();
}

}  // extern "C"

// ============================================================================
// Fields and learned-potential training.
int mfail_str(sl_mlp *m, int code, const std::string &msg);

namespace {

template <typename real>
int fields_now(sl_system *S, double *F, double *hw, int where) {
  const int n = S->n;
  double *dF = nullptr, *dW = nullptr;
  HIPCHK(S, dalloc(&dF, 3 * (size_t)n));
  HIPCHK(S, dalloc(&dW, 3 * (size_t)n));
  CHK(ensure_table(S, S->pos));
  FieldArgs A;
  std::memset(&A, 0, sizeof(A));
  A.F = dF;
  A.hw = dW;
  launch_eam_density<real>(view<real>(S, S->pos), S->pc, S->st);
  launch_fields<real>(view<real>(S, S->pos), S->pc, A, S->st);
  Atoms &At = S->a[S->cur];
  for (int q = 0; q < 2; ++q) {
    double *src = q ? dW : dF, *dst = q ? hw : F;
    if (!dst) continue;
    launch_store_vec(n, At.id, src, src + n, src + 2 * (size_t)n, S->stage, S->st);
    HIPCHK(S, hipMemcpyAsync(dst, S->stage, sizeof(double) * 3 * n,
                             where == SL_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, S->st));
    HIPCHK(S, hipStreamSynchronize(S->st));
  }
  dfree(dF);
  dfree(dW);
  return sticky_code(S);
}

// Lattice temperature from the kinetic energy (Eq. lattice_temperature) and
// spin temperature (Eq. spin_temperature): T_S = sum |s x h|^2 / (2 k_B sum
// s.h) with h = hbar omega, both sums fixed-order device reductions.
template <typename real>
int temps_now(sl_system *S, double *TL, double *TS) {
  const int n = S->n;
  if (TL) {
    double e[8];
    CHK(energy_now<real>(S, e));
    *TL = n > 0 ? 2.0 * e[0] / (3.0 * n * kKb) : 0.0;
  }
  if (TS) {
    double *ts = nullptr;
    HIPCHK(S, dalloc(&ts, 2 * (size_t)n + 2));
    CHK(ensure_table(S, S->pos));
    FieldArgs A;
    std::memset(&A, 0, sizeof(A));
    A.ts = ts;
    launch_eam_density<real>(view<real>(S, S->pos), S->pc, S->st);
    launch_fields<real>(view<real>(S, S->pos), S->pc, A, S->st);
    launch_sum_d(ts, n, ts + 2 * (size_t)n, S->st);
    launch_sum_d(ts + n, n, ts + 2 * (size_t)n + 1, S->st);
    double h[2] = {0.0, 0.0};
    hipError_t e1 = hipMemcpyAsync(h, ts + 2 * (size_t)n, 2 * sizeof(double), hipMemcpyDeviceToHost, S->st);
    hipError_t e2 = e1 == hipSuccess ? hipStreamSynchronize(S->st) : e1;
    dfree(ts);
    HIPCHK(S, e2);
    *TS = h[1] != 0.0 ? h[0] / (2.0 * kKb * h[1]) : 0.0;
  }
  return sticky_code(S);
}

int mlp_trainer(sl_mlp *m, const sl_dataset *d) {
  sl_system *S = m->trainer;
  if (S && (S->n != d->n_atoms || S->L[0] != d->box[0] || S->L[1] != d->box[1] || S->L[2] != d->box[2])) {
    sl_destroy(S);
    m->trainer = S = nullptr;
  }
  if (!S) {
    sl_params p;
    std::memset(&p, 0, sizeof(p));
    p.n_atoms = d->n_atoms;
    for (int k = 0; k < 3; ++k) p.box[k] = d->box[k];
    p.precision = SL_FP32;
    p.skin = 0.0;
    p.stream = m->st;
    int rc = sl_create(&p, &S);
    if (rc) return mfail_str(m, rc, std::string("trainer: ") + sl_last_error(nullptr));
    sl_potential pot;
    std::memset(&pot, 0, sizeof(pot));
    pot.morse_on = 1;
    pot.morse_rc = m->rc;
    pot.morse_shift = 1;
    pot.ex_alpha = 1.0;
    pot.ex_delta = 1.0;
    pot.ex_rc = m->ex_rc;
    pot.zeeman_g = 2.0;
    pot.aniso_n[2] = 1.0;
    rc = sl_set_potential(S, &pot);
    if (rc) {
      std::string e = S->last_err;
      sl_destroy(S);
      return mfail_str(m, rc, "trainer: " + e);
    }
    // training differentiates the network at every pair: per-pair table
    S->mlp_mode = SL_MLP_PAIRWISE;
    m->trainer = S;
  }
  return SL_OK;
}

}  // namespace

int mfail_str(sl_mlp *m, int code, const std::string &msg) {
  if (m) m->last_err = msg;
  return code;
}

extern "C" {

int sl_set_ordering(sl_system *S, int ordering, const int grid[3]) {
  if (!S) return fail(S, SL_E_ARG, "NULL system");
  if (ordering != SL_ORDER_COLOUR && ordering != SL_ORDER_SECTORS && ordering != SL_ORDER_SERIAL)
    return fail(S, SL_E_ARG, "unknown ordering");
  int g[3] = {1, 1, 1};
  if (ordering == SL_ORDER_SECTORS) {
    if (!grid) return fail(S, SL_E_ARG, "the sectored ordering needs a subdomain grid");
    long np = 1;
    for (int d = 0; d < 3; ++d) {
      if (grid[d] < 1) return fail(S, SL_E_ARG, "subdomain grid entries must be >= 1");
      g[d] = grid[d];
      np *= grid[d];
    }
    if (np > (1 << 20)) return fail(S, SL_E_ARG, "too many subdomains");
    // a sector must be at least the spin radius wide, so that atoms in the
    // same sector of different subdomains never interact
    const double rs = spin_radius(S);
    for (int d = 0; d < 3; ++d)
      if (S->L[d] / (2.0 * g[d]) < rs)
        return fail(S, SL_E_ARG, "sector width " + std::to_string(S->L[d] / (2.0 * g[d])) +
                                     " A is below the spin radius " + std::to_string(rs));
  }
  CHK(sl_synchronize(S));
  S->ordering = ordering;
  for (int d = 0; d < 3; ++d) S->sgrid[d] = g[d];
  return SL_OK;
}

int sl_set_row_order(sl_system *S, double quantum) {
  if (!S) return fail(S, SL_E_ARG, "NULL system");
  if (!(quantum >= 0.0) || !std::isfinite(quantum)) return fail(S, SL_E_ARG, "row-order grid step must be finite and >= 0");
  CHK(sl_synchronize(S));
  S->row_q = quantum;
  if (!S->user_list) {
    S->have_list = false;
    S->have_D = false;
  }
  return SL_OK;
}

int sl_get_temperatures(sl_system *S, double *T_lattice, double *T_spin) {
  if (!S) return fail(S, SL_E_ARG, "NULL system");
  CHK(sl_synchronize(S));
  CHK(ensure_ready(S));
  return S->prec == SL_FP64 ? temps_now<double>(S, T_lattice, T_spin)
                            : temps_now<float>(S, T_lattice, T_spin);
}

int sl_get_fields(sl_system *S, double *F, double *hw, int where) {
  if (!S) return fail(S, SL_E_ARG, "NULL system");
  CHK(sl_synchronize(S));
  CHK(ensure_ready(S));
  return S->prec == SL_FP64 ? fields_now<double>(S, F, hw, where) : fields_now<float>(S, F, hw, where);
}

int sl_mlp_loss_grad(sl_mlp *m, const sl_dataset *d, int snap, const double w[3], double *loss,
                     float *grad) {
  if (!m || !d || !w || !loss) return mfail_str(m, SL_E_ARG, "NULL argument");
  if (!m->have_weights) return mfail_str(m, SL_E_STATE, "no weights set");
  if (snap < 0 || snap >= d->n_snapshots || d->n_atoms < 2) return mfail_str(m, SL_E_ARG, "bad snapshot");
  CHK(mlp_trainer(m, d));
  sl_system *S = m->trainer;
  const int n = S->n;
  const size_t off = (size_t)snap * n * 3;
  std::vector<double> zeros(3 * (size_t)n, 0.0), ones(n, 1.0);
  int rc = sl_set_state(S, d->r + off, zeros.data(), d->s + off, ones.data(), SL_HOST);
  if (rc) return mfail_str(m, rc, std::string("snapshot state: ") + S->last_err);
  rc = sl_set_mlp(S, m);
  if (rc) return mfail_str(m, rc, S->last_err);
  rc = ensure_ready(S);
  if (rc) return mfail_str(m, rc, S->last_err);
  rc = ensure_table(S, S->pos);
  if (rc) return mfail_str(m, rc, S->last_err);
  // references in internal order
  Atoms &A = S->a[S->cur];
  double *ref = nullptr, *out = nullptr;
  float *gbuf = nullptr, *rp = nullptr, *part = nullptr;
  float4 *yb = nullptr, *s4 = nullptr;
  float2 *sh = nullptr;
  const int P = S->npair;
  const int nw = mlp_backward_waves(P);
  auto cleanup = [&]() {
    for (void *q : {(void *)ref, (void *)out, (void *)gbuf, (void *)rp, (void *)part, (void *)yb, (void *)s4, (void *)sh})
      dfree(q);
  };
#define TCHK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { cleanup(); return mfail_str(m, SL_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); } } while (0)
  TCHK(dalloc(&ref, 6 * (size_t)n));
  TCHK(dalloc(&out, 8 * (size_t)n + 8));
  TCHK(dalloc(&gbuf, 6 * (size_t)n));
  TCHK(dalloc(&rp, (size_t)P + 1));
  TCHK(dalloc(&yb, (size_t)P + 1));
  TCHK(dalloc(&sh, (size_t)P + 1));
  TCHK(dalloc(&s4, 4));
  TCHK(dalloc(&part, (size_t)nw * SL_MLP_NPARAM));
  for (int q = 0; q < 2; ++q) {
    const double *src = (q ? d->hw : d->F) + off;
    TCHK(hipMemcpyAsync(S->stage, src, sizeof(double) * 3 * n, hipMemcpyHostToDevice, S->st));
    double *dst = ref + (size_t)q * 3 * n;
    launch_load_vec(n, A.id, S->stage, dst, dst + n, dst + 2 * (size_t)n, S->st);
  }
  FieldArgs Fa;
  std::memset(&Fa, 0, sizeof(Fa));
  double *e_at = out, *lossp = out + n, *sums = out + 8 * (size_t)n;
  Fa.e = e_at;
  Fa.Fref = ref;
  Fa.hwref = ref + 3 * (size_t)n;
  Fa.wF = w[1];
  Fa.wW = w[2];
  Fa.gF = gbuf;
  Fa.gW = gbuf + 3 * (size_t)n;
  Fa.lossp = lossp;
  launch_fields<float>(view<float>(S, S->pos), S->pc, Fa, S->st);
  launch_sum_d(e_at, n, sums, S->st);
  launch_sum_d(lossp, n, sums + 1, S->st);
  double hs[2];
  TCHK(hipMemcpyAsync(hs, sums, sizeof(hs), hipMemcpyDeviceToHost, S->st));
  TCHK(hipStreamSynchronize(S->st));
  const double eres = (hs[0] - d->E[snap]) / n;
  *loss = w[0] * eres * eres + hs[1];
  if (grad) {
    PairAdjArgs Pa;
    std::memset(&Pa, 0, sizeof(Pa));
    Pa.npair = P;
    Pa.ld = S->ld;
    Pa.n = n;
    Pa.pairs = S->mpairs;
    Pa.nbr = A.nbr;
    Pa.rx = A.rx[S->pos];
    Pa.ry = A.ry[S->pos];
    Pa.rz = A.rz[S->pos];
    for (int k = 0; k < 3; ++k) {
      Pa.L[k] = S->L[k];
      Pa.invL[k] = S->invL[k];
    }
    Pa.sx = (const float *)A.sx;
    Pa.sy = (const float *)A.sy;
    Pa.sz = (const float *)A.sz;
    Pa.gF = Fa.gF;
    Pa.gW = Fa.gW;
    Pa.dE = (float)(2.0 * w[0] * eres / n);
    Pa.sJ = (float)m->sJ;
    Pa.sP = (float)m->sP;
    Pa.ex_rc = (float)m->ex_rc;
    Pa.rc = (float)m->rc;
    Pa.rp = rp;
    Pa.ybar = yb;
    Pa.shift = sh;
    launch_pair_adjoint(Pa, S->st);
    launch_mlp_backward(rp, yb, P, m->w, m->wt, m->cfg(), part, S->st);
    launch_mlp_grad_reduce(part, nw, m->grad, 0, S->st);
    // the shifted-force constants y1(rc), y1'(rc): one more point
    launch_sum_f2(sh, P, s4, S->st);
    float rcf = (float)m->rc;
    TCHK(hipMemcpyAsync(rp + P, &rcf, sizeof(float), hipMemcpyHostToDevice, S->st));
    launch_mlp_backward(rp + P, s4, 1, m->w, m->wt, m->cfg(), part, S->st);
    launch_mlp_grad_reduce(part, 1, m->grad, 1, S->st);
    TCHK(hipMemcpyAsync(grad, m->grad, sizeof(float) * SL_MLP_NPARAM, hipMemcpyDeviceToHost, S->st));
    TCHK(hipStreamSynchronize(S->st));
  }
#undef TCHK
  cleanup();
  return SL_OK;
}

int sl_mlp_train(sl_mlp *m, const sl_dataset *d, const sl_train_opts *o, sl_train_log *log) {
  if (!m || !d || !o) return mfail_str(m, SL_E_ARG, "NULL argument");
  if (o->epochs < 0) return mfail_str(m, SL_E_ARG, "negative epochs");
  const float lr = (float)(o->lr > 0 ? o->lr : 1e-3), b1 = (float)(o->beta1 > 0 ? o->beta1 : 0.9);
  const float b2 = (float)(o->beta2 > 0 ? o->beta2 : 0.999), eps = (float)(o->eps > 0 ? o->eps : 1e-8);
  const double w[3] = {o->w_E, o->w_F, o->w_W};
  std::vector<int> order(d->n_snapshots);
  for (int k = 0; k < d->n_snapshots; ++k) order[k] = k;
  uint64_t x = o->seed * 6364136223846793005ull + 1442695040888963407ull;
  std::vector<float> g(SL_MLP_NPARAM);
  double first = 0.0, last = 0.0;
  int64_t updates = 0;
  for (int ep = 0; ep < o->epochs; ++ep) {
    for (int k = d->n_snapshots - 1; k > 0; --k) {  // Fisher-Yates with an LCG
      x = x * 6364136223846793005ull + 1442695040888963407ull;
      const int q = (int)((x >> 33) % (uint64_t)(k + 1));
      std::swap(order[k], order[q]);
    }
    double sum = 0.0;
    for (int k = 0; k < d->n_snapshots; ++k) {
      double L = 0.0;
      CHK(sl_mlp_loss_grad(m, d, order[k], w, &L, g.data()));
      sum += L;
      m->adam_t += 1;
      launch_adam(m->master, m->adam_m, m->adam_v, m->grad, SL_MLP_NPARAM, lr, b1, b2, eps,
                  (int)m->adam_t, m->trainer->st);
      (void)hipStreamSynchronize(m->trainer->st);
      CHK(mlp_refresh(m));
      ++updates;
    }
    const double mean = d->n_snapshots ? sum / d->n_snapshots : 0.0;
    if (ep == 0) first = mean;
    last = mean;
  }
  if (log) {
    log->loss_first = first;
    log->loss_last = last;
    log->updates = updates;
  }
  return SL_OK;
}

}  // extern "C"


// ============================================================================
// Autotuner: times launch shapes on scratch copies and keeps the fastest.
namespace {

// State of S in user order, masses included.
int user_state(sl_system *S, std::vector<double> &r, std::vector<double> &v,
               std::vector<double> &sp, std::vector<double> &m) {
  const int n = S->n;
  r.resize(3 * (size_t)n);
  v.resize(3 * (size_t)n);
  sp.resize(3 * (size_t)n);
  m.resize(n);
  CHK(sl_get_state(S, r.data(), v.data(), sp.data(), SL_HOST));
  std::vector<double> mi(n);
  std::vector<int> id(n);
  Atoms &A = S->a[S->cur];
  HIPCHK(S, hipMemcpy(mi.data(), A.mass, sizeof(double) * n, hipMemcpyDeviceToHost));
  HIPCHK(S, hipMemcpy(id.data(), A.id, sizeof(int) * n, hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i) m[id[i]] = mi[i];
  if (S->prec == SL_FP32)  // FP32 spins are unit to FP32 rounding only
    for (int i = 0; i < n; ++i) {
      double *q = &sp[3 * (size_t)i];
      const double inv = 1.0 / std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
      q[0] *= inv; q[1] *= inv; q[2] *= inv;
    }
  return SL_OK;
}

// Scratch copy of S (parameters, interactions, learned potential, user
// list, state and step counter) on its own stream.
int clone_system(sl_system *S, sl_system **out) {
  *out = nullptr;
  CHK(sl_synchronize(S));
  sl_params p = S->prm;
  p.stream = nullptr;
  p.skin = S->skin;
  p.max_nbr = S->max_nbr;
  p.max_spin_nbr = S->max_spin;
  sl_system *C = nullptr;
  int rc = sl_create(&p, &C);
  if (rc) return fail(S, rc, std::string("autotune copy: ") + sl_last_error(nullptr));
  auto bail = [&](int code) {
    const std::string e = C->last_err;
    sl_destroy(C);
    return fail(S, code, "autotune copy: " + e);
  };
  if ((rc = sl_set_potential(C, &S->pot))) return bail(rc);
  std::vector<double> r, v, sp, m;
  CHK(user_state(S, r, v, sp, m));
  if ((rc = sl_set_state(C, r.data(), v.data(), sp.data(), m.data(), SL_HOST))) return bail(rc);
  if (S->user_list) {
    const int n = S->n;
    std::vector<int> ns(n), na(n);
    const int64_t tot = sl_get_neighbor_list(S, ns.data(), na.data(), nullptr, 0);
    if (tot < 0) return bail((int)tot);
    std::vector<int> idx(std::max<int64_t>(tot, 1)), off(n + 1, 0);
    const int64_t t2 = sl_get_neighbor_list(S, ns.data(), na.data(), idx.data(), tot);
    if (t2 < 0) return bail((int)t2);
    for (int i = 0; i < n; ++i) off[i + 1] = off[i] + na[i];
    if ((rc = sl_set_neighbor_list(C, off.data(), idx.data(), SL_HOST))) return bail(rc);
  }
  if (S->mlp && (rc = sl_set_mlp(C, S->mlp))) return bail(rc);
  if (S->mlp && (rc = sl_set_mlp_mode(C, S->mlp_mode))) return bail(rc);
  if ((rc = sl_set_ordering(C, S->ordering, S->sgrid))) return bail(rc);
  if ((rc = sl_set_row_order(C, S->row_q))) return bail(rc);
  if ((rc = sl_set_step(C, S->step))) return bail(rc);
  *out = C;
  return SL_OK;
}

// Optional cache of tuned shapes: one JSON object per line in the file named
// by SL_TUNE_CACHE, keyed by the device and the workload's shape.
std::string tune_key(const std::string &what) {
  hipDeviceProp_t prop;
  int dev = 0;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    arch = prop.gcnArchName;
  return arch + " " + what;
}

bool cache_lookup(const std::string &key, int vals[4]) {
  const char *path = std::getenv("SL_TUNE_CACHE");
  if (!path) return false;
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  const std::string want = "{\"key\": \"" + key + "\"";
  while (std::fgets(line, sizeof(line), f)) {
    if (std::strncmp(line, want.c_str(), want.size()) != 0) continue;
    const char *q = std::strstr(line, "\"vals\": [");
    if (q && std::sscanf(q, "\"vals\": [%d, %d, %d, %d]", &vals[0], &vals[1], &vals[2], &vals[3]) == 4)
      found = true;
  }
  std::fclose(f);
  return found;
}

void cache_store(const std::string &key, const int vals[4]) {
  const char *path = std::getenv("SL_TUNE_CACHE");
  if (!path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "{\"key\": \"%s\", \"vals\": [%d, %d, %d, %d]}\n", key.c_str(), vals[0], vals[1],
               vals[2], vals[3]);
  std::fclose(f);
}

}  // namespace

extern "C" {

int sl_autotune(sl_system *S, int steps, double dt, sl_tuning *chosen) {
  if (!S || steps < 1 || !std::isfinite(dt) || dt == 0.0) return fail(S, SL_E_ARG, "bad autotune arguments");
  CHK(ensure_ready(S));
  const std::string key = tune_key(
      "system n=" + std::to_string(S->n) + " prec=" + std::to_string(S->prec) +
      " frozen=" + std::to_string(S->prm.frozen) + " langevin=" + std::to_string(S->pc.langevin) +
      " aniso=" + std::to_string(S->pc.aniso_on) + " mlp=" + std::to_string(S->mlp ? 1 : 0) +
      " K=" + std::to_string(S->K));
  int v[4];
  if (!cache_lookup(key, v)) {
    sl_system *C = nullptr;
    CHK(clone_system(S, &C));
    // Every candidate (spin lanes, force lanes, J cache) runs a window of
    // `steps` steps on the clone, timed with events on its stream: the whole
    // step counts, so the cache's own kernel and its effect on the other
    // kernels (it shares the caches with them) are part of the comparison.
    // A window with a list rebuild in it is run again; four rounds over
    // all candidates, the best window of each counts.
    const int trial[8][3] = {{2, 1, -1}, {1, 1, 1}, {2, 1, 1}, {1, 1, -1},
                             {4, 1, 1}, {4, 1, -1}, {2, 2, -1}, {1, 2, 1}};
    double best[8];
    for (double &b : best) b = 1e300;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = SL_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = SL_E_HIP;
    // sustained load first: the device's clocks and caches then are those of
    // a long run, not of a device that has just been idle
    if (rc == SL_OK) rc = sl_step(C, 6 * steps, dt);
    // the order of the candidates rotates from round to round, so no shape
    // always follows the same other one
    for (int pass = 0; pass < 4 && rc == SL_OK; ++pass)
      for (int q = 0; q < 8 && rc == SL_OK; ++q) {
        const int t = (q + 3 * pass) % 8;
        sl_tuning tt{trial[t][0], trial[t][1], S->small_class, trial[t][2], S->overlap};
        if ((rc = sl_set_tuning(C, &tt))) break;
        if ((rc = sl_step(C, 3, dt))) break;
        for (int attempt = 0; attempt < 3 && rc == SL_OK; ++attempt) {
          const int64_t rb0 = C->rebuilds;
          if (hipEventRecord(e0, C->st) != hipSuccess) { rc = SL_E_HIP; break; }
          if ((rc = sl_step(C, steps, dt))) break;
          if (hipEventRecord(e1, C->st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rc = SL_E_HIP;
            break;
          }
          float ms = 0.f;
          if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = SL_E_HIP; break; }
          if (C->rebuilds != rb0) continue;  // a rebuild in the window: run it again
          best[t] = std::min(best[t], (double)ms / steps);
          break;
        }
      }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    const std::string err = rc ? C->last_err : std::string();
    sl_destroy(C);
    if (rc) return fail(S, rc, "autotune trial: " + err);
    int bt = 0;
    for (int t = 1; t < 8; ++t)
      if (best[t] < best[bt]) bt = t;
    v[0] = trial[bt][0];
    v[1] = S->prm.frozen ? 1 : trial[bt][1];
    v[2] = S->small_class;
    v[3] = trial[bt][2];
    cache_store(key, v);
  }
  sl_tuning t{v[0], v[1], v[2], v[3], S->overlap};
  CHK(sl_set_tuning(S, &t));
  if (chosen) *chosen = t;
  return SL_OK;
}

}  // extern "C"

// ============================================================================
// Batched replicas.
namespace {
struct BatchRep {
  double cur_dm = 0, cur_vm = 0, cur_dt = 0, prev_dm = 0, prev_vm = 0, prev_dt = 0;
  double cur_wm = kInf, prev_wm = kInf;
  int cur_rebuilt = 0, prev_rebuilt = 0, have_prev = 0;
  bool valid = false;
};
}  // namespace

struct sl_batch {
  int R = 0, prec = SL_FP64;
  std::vector<sl_system *> sys;
  std::vector<BatchRep> rep;
  hipStream_t st = nullptr;
  void *d_desc = nullptr;
  std::vector<char> h_desc;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_lanes = -1;
  int lanes = 2;
  int mode = SL_BATCH_PHASED;
  double row_q = 0.0;  // list row order of every replica
  std::vector<sl_params> params;     // creation parameters, for autotune clones
  std::vector<sl_potential> pots;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  int64_t launches = 0, rebuilds = 0;
  std::string last_err;
};

namespace {

thread_local std::string g_batch_err;

int bfail(sl_batch *B, int code, const std::string &msg) {
  if (B) B->last_err = msg;
  else g_batch_err = msg;
  return code;
}

#define BCHK(B, x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) return bfail((B), SL_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define BSYS(B, r, x)                                                         \
  do {                                                                       \
    int rc_ = (x);                                                           \
    if (rc_) return bfail((B), rc_, "replica " + std::to_string(r) + ": " + (B)->sys[r]->last_err); \
  } while (0)

// Whether any replica has the spin-orbit pair terms (their kernel variants
// then serve every replica; zero coefficients leave the others unchanged).
bool batch_soc(const sl_batch *B) {
  for (const sl_system *S : B->sys)
    if (S->pc.soc_on) return true;
  return false;
}

// Force variant of the batch kernels: 4 with spin-orbit terms, 8 with
// embedded-atom terms (in any replica).
int batch_variant(const sl_batch *B) {
  int v = batch_soc(B) ? 4 : 0;
  for (const sl_system *S : B->sys)
    if (S->pc.eam_on) v |= 8;
  return v;
}

// Descriptor of replica r for the batched kernels (current buffers, class
// offsets, step, predictor state of the last two boundaries).
template <typename real>
int fill_desc(sl_batch *B, int r, double dt, int64_t target, RepDesc<real> &d) {
  sl_system *S = B->sys[r];
  std::memset(&d, 0, sizeof(d));
  d.V[0] = view<real>(S, 0);
  d.V[1] = view<real>(S, 1);
  d.P = S->pc;
  Atoms &A = S->a[S->cur];
  d.F.ftm2v = 1.0 / kMvv2e;
  d.F.mass = A.mass;
  d.F.vx = A.vx; d.F.vy = A.vy; d.F.vz = A.vz;
  d.F.bx = A.bx; d.F.by = A.by; d.F.bz = A.bz;
  d.F.err = S->err;
  d.F.wmask = A.wmask;
  d.F.dslot = S->dslot;
  d.F.done = S->done;
  d.F.pred = S->pred;
  d.F.seed = S->prm.seed;
  d.F.replica = S->prm.replica;
  if (S->K > kMaxClass) return bfail(B, SL_E_COLOR, "replica " + std::to_string(r) + " has too many colours");
  d.K = S->K;
  for (int c = 0; c <= S->K; ++c) d.off[c] = S->class_off[c];
  d.pos = S->pos;
  d.step = S->step;
  d.target = target;
  d.dt = dt;
  d.h = dt / 4.0;
  d.amp = noise_amp(S, dt / 4.0);
  d.rs2 = S->pot.ex_rc * S->pot.ex_rc;
  d.thr = S->skin / 2.0 - 0.01;
  d.wr = colour_radius(S);
  d.ex_rc = S->pot.ex_rc;
  d.seed = S->prm.seed;
  d.replica = S->prm.replica;
  d.user_list = S->user_list ? 1 : 0;
  const BatchRep &q = B->rep[r];
  d.cur_dm = q.cur_dm; d.cur_vm = q.cur_vm; d.cur_dt = q.cur_dt; d.cur_rebuilt = q.cur_rebuilt;
  d.prev_dm = q.prev_dm; d.prev_vm = q.prev_vm; d.prev_dt = q.prev_dt;
  d.cur_wm = q.cur_wm; d.prev_wm = q.prev_wm;
  d.prev_rebuilt = q.prev_rebuilt; d.have_prev = q.have_prev;
  d.ring = S->ring_dev;
  return SL_OK;
}

template <typename real>
int batch_launch(sl_batch *B) {
  if (!B->exec || B->graph_lanes != B->lanes) {
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
    BCHK(B, hipStreamBeginCapture(B->st, hipStreamCaptureModeThreadLocal));
    launch_batch_run<real>((RepDesc<real> *)B->d_desc, B->R, B->lanes, batch_variant(B), B->st);
    BCHK(B, hipStreamEndCapture(B->st, &B->graph));
    BCHK(B, hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    B->graph_lanes = B->lanes;
  }
  BCHK(B, hipGraphLaunch(B->exec, B->st));
  B->launches++;
  return SL_OK;
}

template <typename real>
int batch_step(sl_batch *B, int64_t n, double dt) {
  const int R = B->R;
  std::vector<int64_t> k0(R);
  // call start of every replica: rebuild decision, first kick and drift
  for (int r = 0; r < R; ++r) {
    sl_system *S = B->sys[r];
    const int64_t rb0 = S->rebuilds;
    BSYS(B, r, ensure_ready(S));
    bool built = S->rebuilds != rb0;
    BatchRep &q = B->rep[r];
    if (!S->user_list && S->have_D && q.valid && q.have_prev) {
      const double adt = std::max(std::fabs(q.prev_dt), std::fabs(dt));
      const double D = (q.prev_rebuilt ? 0.0 : q.prev_dm) + 2.0 * adt * q.prev_vm;
      const double W = (q.prev_rebuilt ? colour_radius(S) : std::sqrt(q.prev_wm)) - 4.0 * adt * q.prev_vm;
      if (D >= S->skin / 2.0 - 0.01 || W < S->pot.ex_rc + 0.01) {
        BSYS(B, r, rebuild(S));
        B->rebuilds++;
        built = true;
      }
    }
    k0[r] = S->step;
    BSYS(B, r, force_launch<real>(S, S->pos, kModeNext, dt, S->step));
    bool due_unused;
    BSYS(B, r, wait_predictor(S, S->step, dt, &due_unused));
    const double *o = S->ring + 8 * (int)(S->step & 3);
    q.prev_dm = q.cur_dm; q.prev_vm = q.cur_vm; q.prev_dt = q.cur_dt; q.prev_wm = q.cur_wm;
    q.prev_rebuilt = q.cur_rebuilt; q.have_prev = q.valid ? 1 : 0;
    q.cur_dm = o[0]; q.cur_vm = o[1]; q.cur_wm = o[4]; q.cur_dt = dt;
    q.cur_rebuilt = built ? 1 : 0;
    q.valid = true;
    S->have_D = true;
  }
  const size_t dsz = sizeof(RepDesc<real>);
  for (;;) {
    bool any = false;
    for (int r = 0; r < R; ++r) {
      sl_system *S = B->sys[r];
      RepDesc<real> d;
      CHK(fill_desc<real>(B, r, dt, k0[r] + n, d));
      std::memcpy(B->h_desc.data() + r * dsz, &d, dsz);
      if (d.step < d.target) any = true;
    }
    if (!any) break;
    BCHK(B, hipMemcpyAsync(B->d_desc, B->h_desc.data(), dsz * R, hipMemcpyHostToDevice, B->st));
    CHK(batch_launch<real>(B));
    BCHK(B, hipMemcpyAsync(B->h_desc.data(), B->d_desc, dsz * R, hipMemcpyDeviceToHost, B->st));
    BCHK(B, hipStreamSynchronize(B->st));
    for (int r = 0; r < R; ++r) {
      sl_system *S = B->sys[r];
      RepDesc<real> d;
      std::memcpy(&d, B->h_desc.data() + r * dsz, dsz);
      S->pos = d.pos;
      S->step = d.step;
      BatchRep &q = B->rep[r];
      q.cur_dm = d.cur_dm; q.cur_vm = d.cur_vm; q.cur_dt = d.cur_dt; q.cur_rebuilt = d.cur_rebuilt;
      q.prev_dm = d.prev_dm; q.prev_vm = d.prev_vm; q.prev_dt = d.prev_dt;
      q.cur_wm = d.cur_wm; q.prev_wm = d.prev_wm;
      q.prev_rebuilt = d.prev_rebuilt; q.have_prev = d.have_prev;
      if (d.stopped) {
        BSYS(B, r, rebuild(S));
        q.cur_rebuilt = 1;
        B->rebuilds++;
      }
    }
  }
  for (int r = 0; r < R; ++r) BSYS(B, r, sl_synchronize(B->sys[r]));
  return SL_OK;
}


// Phase-batched mode: every spin phase and force pass is one launch over
// all replicas; the host pipelines one step ahead exactly as step_coupled
// does for one system (decision before step k from the predictor of
// boundary k-1), with one event per boundary for the whole batch.
template <typename real>
int batch_step_phased(sl_batch *B, int64_t n, double dt) {
  const int R = B->R;
  const size_t dsz = sizeof(RepDesc<real>);
  std::vector<int64_t> k0(R);
  std::vector<int> pos0(R);
  // call start: same decision as the persistent mode (predictor state of
  // the previous call's last two boundaries)
  for (int r = 0; r < R; ++r) {
    sl_system *S = B->sys[r];
    const int64_t rb0 = S->rebuilds;
    BSYS(B, r, ensure_ready(S));
    bool built = S->rebuilds != rb0;
    BatchRep &q = B->rep[r];
    if (!S->user_list && S->have_D && q.valid && q.have_prev) {
      const double adt = std::max(std::fabs(q.prev_dt), std::fabs(dt));
      const double D = (q.prev_rebuilt ? 0.0 : q.prev_dm) + 2.0 * adt * q.prev_vm;
      const double W = (q.prev_rebuilt ? colour_radius(S) : std::sqrt(q.prev_wm)) - 4.0 * adt * q.prev_vm;
      if (D >= S->skin / 2.0 - 0.01 || W < S->pot.ex_rc + 0.01) {
        BSYS(B, r, rebuild(S));
        B->rebuilds++;
        built = true;
      }
    }
    k0[r] = S->step;
    pos0[r] = S->pos;
    const int slot = (int)(S->step & 3);
    S->ring[8 * slot + 3] = 0.0;
    S->meta[slot].boundary = S->step;
    S->meta[slot].dt = dt;
    S->meta[slot].rebuilt_after = built;
    RepDesc<real> d;
    CHK(fill_desc<real>(B, r, dt, k0[r] + n, d));
    std::memcpy(B->h_desc.data() + r * dsz, &d, dsz);
  }
  BCHK(B, hipMemcpyAsync(B->d_desc, B->h_desc.data(), dsz * R, hipMemcpyHostToDevice, B->st));
  BCHK(B, hipStreamSynchronize(B->st));
  auto extents = [&](int &Kmax, int &max_class, int &max_n) {
    Kmax = 0; max_class = 0; max_n = 0;
    for (auto *S : B->sys) {
      Kmax = std::max(Kmax, S->K);
      max_n = std::max(max_n, S->n);
      for (int c = 0; c < S->K; ++c)
        max_class = std::max(max_class, S->class_off[c + 1] - S->class_off[c]);
    }
  };
  int Kmax, max_class, max_n;
  extents(Kmax, max_class, max_n);
  const RepDesc<real> *D = (const RepDesc<real> *)B->d_desc;
  BatchPhase bp{};
  bp.kk = 0;
  bp.after = 0;
  launch_batch_force<real>(D, R, max_n, kModeNext, bp, B->lanes, batch_variant(B), B->st);
  BCHK(B, hipEventRecord(B->ev[0], B->st));
  for (int64_t kk = 0; kk < n; ++kk) {
    if (kk > 0) {
      // rebuild decision for step kk from the predictor of boundary kk - 1
      BCHK(B, hipEventSynchronize(B->ev[(kk - 1) & 3]));
      bool changed = false;
      for (int r = 0; r < R; ++r) {
        sl_system *S = B->sys[r];
        if (S->user_list) continue;
        const int64_t b = k0[r] + kk - 1;
        const int slot = (int)(b & 3);
        const double *o = S->ring + 8 * slot;
        if (o[3] != 1.0) return bfail(B, SL_E_HIP, "replica " + std::to_string(r) + ": predictor not written");
        S->sticky |= (int)o[2];
        BSYS(B, r, sticky_code(S));
        const bool rb = S->meta[slot].rebuilt_after;
        const double adt = std::fabs(dt);
        const double Dv = (rb ? 0.0 : o[0]) + 2.0 * adt * o[1];
        const double Wv = (rb ? colour_radius(S) : std::sqrt(o[4])) - 4.0 * adt * o[1];
        if (Dv >= S->skin / 2.0 - 0.01 || Wv < S->pot.ex_rc + 0.01) {
          BSYS(B, r, rebuild(S));
          B->rebuilds++;
          S->meta[(b + 1) & 3].rebuilt_after = true;
          RepDesc<real> d;
          CHK(fill_desc<real>(B, r, dt, k0[r] + n, d));
          d.pos = pos0[r];  // kernels index buffers from the call start
          d.step = k0[r];
          std::memcpy(B->h_desc.data() + r * dsz, &d, dsz);
          BCHK(B, hipMemcpyAsync((char *)B->d_desc + r * dsz, B->h_desc.data() + r * dsz, dsz,
                                 hipMemcpyHostToDevice, B->st));
          changed = true;
        }
      }
      if (changed) {
        BCHK(B, hipStreamSynchronize(B->st));
        extents(Kmax, max_class, max_n);
      }
    }
    bp.kk = (int)kk;
    for (int half = 0; half < 2; ++half) {
      bp.half = half;
      bp.Kmax = Kmax;
      for (int p = 0; p < 2 * Kmax - 1; ++p) {
        bp.p = p;
        launch_batch_spin<real>(D, R, max_class, bp, B->lanes, batch_soc(B), B->st);
      }
    }
    const int mode = kk + 1 < n ? (kModeFinal | kModeNext) : kModeFinal;
    for (int r = 0; r < R; ++r) {
      sl_system *S = B->sys[r];
      const int64_t b = k0[r] + kk + 1;
      const int slot = (int)(b & 3);
      S->ring[8 * slot + 3] = 0.0;
      S->meta[slot].boundary = b;
      S->meta[slot].dt = dt;
      S->meta[slot].rebuilt_after = false;
      S->pos = 1 - S->pos;
      S->step = b;
    }
    bp.after = 1;
    launch_batch_force<real>(D, R, max_n, mode, bp, B->lanes, batch_variant(B), B->st);
    bp.after = 0;
    BCHK(B, hipEventRecord(B->ev[(kk + 1) & 3], B->st));
    B->launches += 2 * (2 * Kmax - 1) + 1;
  }
  BCHK(B, hipStreamSynchronize(B->st));
  // predictor state of the last two boundaries, for the next call's start
  for (int r = 0; r < R; ++r) {
    sl_system *S = B->sys[r];
    BatchRep &q = B->rep[r];
    const int64_t bl = k0[r] + n, bp2 = bl - 1;
    const double *oc = S->ring + 8 * (int)(bl & 3);
    const double *op = S->ring + 8 * (int)(bp2 & 3);
    S->sticky |= (int)oc[2];
    BSYS(B, r, sticky_code(S));
    q.prev_dm = op[0]; q.prev_vm = op[1]; q.prev_wm = op[4]; q.prev_dt = dt;
    q.prev_rebuilt = S->meta[bp2 & 3].rebuilt_after ? 1 : 0;
    q.cur_dm = oc[0]; q.cur_vm = oc[1]; q.cur_wm = oc[4]; q.cur_dt = dt;
    q.cur_rebuilt = S->meta[bl & 3].rebuilt_after ? 1 : 0;
    q.have_prev = 1;
    q.valid = true;
    S->have_D = true;
  }
  return SL_OK;
}
}  // namespace

extern "C" {

int sl_batch_create(int R, const sl_params *params, const sl_potential *pots, sl_batch **out) {
  if (!out || R < 1 || !params || !pots) return bfail(nullptr, SL_E_ARG, "bad arguments");
  *out = nullptr;
  for (int r = 0; r < R; ++r) {
    if (params[r].precision != params[0].precision)
      return bfail(nullptr, SL_E_ARG, "all replicas must share one precision");
    if (params[r].frozen) return bfail(nullptr, SL_E_ARG, "batched replicas are coupled systems");
  }
  sl_batch *B = new sl_batch();
  B->R = R;
  B->prec = params[0].precision;
  auto bail = [&](int code) {
    g_batch_err = B->last_err;
    sl_batch_destroy(B);
    return code;
  };
  if (hipStreamCreateWithFlags(&B->st, hipStreamNonBlocking) != hipSuccess) {
    B->st = nullptr;
    B->last_err = "hipStreamCreate failed";
    return bail(SL_E_HIP);
  }
  for (int k = 0; k < 4; ++k)
    if (hipEventCreateWithFlags(&B->ev[k], hipEventDisableTiming) != hipSuccess) {
      B->ev[k] = nullptr;
      B->last_err = "hipEventCreate failed";
      return bail(SL_E_HIP);
    }
  B->sys.assign(R, nullptr);
  B->rep.assign(R, BatchRep());
  B->params.assign(params, params + R);
  B->pots.assign(pots, pots + R);
  for (int r = 0; r < R; ++r) {
    sl_params p = params[r];
    p.stream = B->st;
    int rc = sl_create(&p, &B->sys[r]);
    if (rc) {
      B->last_err = "replica " + std::to_string(r) + ": " + sl_last_error(nullptr);
      return bail(rc);
    }
    rc = sl_set_potential(B->sys[r], &pots[r]);
    if (rc) {
      B->last_err = "replica " + std::to_string(r) + ": " + B->sys[r]->last_err;
      return bail(rc);
    }
  }
  const size_t dsz = B->prec == SL_FP64 ? sizeof(RepDesc<double>) : sizeof(RepDesc<float>);
  B->h_desc.assign(dsz * R, 0);
  if (hipMalloc(&B->d_desc, dsz * R) != hipSuccess) {
    B->last_err = "descriptor allocation failed";
    return bail(SL_E_NOMEM);
  }
  *out = B;
  return SL_OK;
}

int sl_batch_destroy(sl_batch *B) {
  if (!B) return SL_OK;
  if (B->st) (void)hipStreamSynchronize(B->st);
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  for (auto *S : B->sys)
    if (S) sl_destroy(S);
  if (B->d_desc) (void)hipFree(B->d_desc);
  for (auto &e : B->ev)
    if (e) (void)hipEventDestroy(e);
  if (B->st) (void)hipStreamDestroy(B->st);
  delete B;
  return SL_OK;
}

int sl_batch_set_state(sl_batch *B, int r, const double *x, const double *v, const double *s,
                       const double *mass, int where) {
  if (!B || r < 0 || r >= B->R) return bfail(B, SL_E_ARG, "bad replica");
  BSYS(B, r, sl_set_state(B->sys[r], x, v, s, mass, where));
  B->rep[r] = BatchRep();
  return SL_OK;
}

int sl_batch_get_state(sl_batch *B, int r, double *x, double *v, double *s, int where) {
  if (!B || r < 0 || r >= B->R) return bfail(B, SL_E_ARG, "bad replica");
  BSYS(B, r, sl_get_state(B->sys[r], x, v, s, where));
  return SL_OK;
}

int sl_batch_get_energy(sl_batch *B, int r, sl_energy *e) {
  if (!B || r < 0 || r >= B->R) return bfail(B, SL_E_ARG, "bad replica");
  BSYS(B, r, sl_get_energy(B->sys[r], e));
  return SL_OK;
}

int sl_batch_get_temperatures(sl_batch *B, int r, double *T_lattice, double *T_spin) {
  if (!B || r < 0 || r >= B->R) return bfail(B, SL_E_ARG, "bad replica");
  BSYS(B, r, sl_get_temperatures(B->sys[r], T_lattice, T_spin));
  return SL_OK;
}

int sl_batch_step(sl_batch *B, int64_t n, double dt) {
  if (!B) return bfail(B, SL_E_ARG, "NULL batch");
  if (n < 0 || !std::isfinite(dt)) return bfail(B, SL_E_ARG, "bad step count or dt");
  if (n == 0) return SL_OK;
  if (B->mode == SL_BATCH_PHASED)
    return B->prec == SL_FP64 ? batch_step_phased<double>(B, n, dt)
                              : batch_step_phased<float>(B, n, dt);
  return B->prec == SL_FP64 ? batch_step<double>(B, n, dt) : batch_step<float>(B, n, dt);
}


int sl_batch_autotune(sl_batch *B, int steps, double dt, int *mode, int *lanes) {
  if (!B || steps < 1 || !std::isfinite(dt) || dt == 0.0) return bfail(B, SL_E_ARG, "bad autotune arguments");
  std::string what = "batch R=" + std::to_string(B->R) + " prec=" + std::to_string(B->prec);
  int64_t natoms = 0;
  for (auto *S : B->sys) natoms += S->n;
  what += " atoms=" + std::to_string(natoms);
  const std::string key = tune_key(what);
  int v[4] = {0, 0, 0, 0};
  if (!cache_lookup(key, v)) {
    sl_batch *C = nullptr;
    int rc = sl_batch_create(B->R, B->params.data(), B->pots.data(), &C);
    if (rc) return bfail(B, rc, std::string("autotune copy: ") + sl_batch_last_error(nullptr));
    rc = sl_batch_set_row_order(C, B->row_q);
    for (int r = 0; r < B->R && rc == SL_OK; ++r) {
      sl_system *S = B->sys[r];
      std::vector<double> x, vv, sp, m;
      if ((rc = user_state(S, x, vv, sp, m))) break;
      if ((rc = sl_batch_set_state(C, r, x.data(), vv.data(), sp.data(), m.data(), SL_HOST))) break;
      if ((rc = sl_set_step(C->sys[r], S->step))) break;
    }
    // (mode, lanes) trials timed on the whole batch
    const int trial[5][2] = {{SL_BATCH_PHASED, 1}, {SL_BATCH_PHASED, 2}, {SL_BATCH_PHASED, 4},
                             {SL_BATCH_PERSISTENT, 1}, {SL_BATCH_PERSISTENT, 2}};
    double best = 1e300;
    v[0] = B->mode;
    v[1] = B->lanes;
    v[2] = 0;
    v[3] = 0;
    for (int t = 0; t < 5 && rc == SL_OK; ++t) {
      C->mode = trial[t][0];
      C->lanes = trial[t][1];
      if ((rc = sl_batch_step(C, 2, dt))) break;
      if (hipStreamSynchronize(C->st) != hipSuccess) { rc = SL_E_HIP; break; }
      const auto t0 = std::chrono::steady_clock::now();
      if ((rc = sl_batch_step(C, steps, dt))) break;
      if (hipStreamSynchronize(C->st) != hipSuccess) { rc = SL_E_HIP; break; }
      const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (el < best) {
        best = el;
        v[0] = trial[t][0];
        v[1] = trial[t][1];
      }
    }
    const std::string err = rc ? C->last_err : std::string();
    sl_batch_destroy(C);
    if (rc) return bfail(B, rc, "autotune trial: " + err);
    cache_store(key, v);
  }
  B->mode = v[0];
  B->lanes = v[1];
  if (mode) *mode = v[0];
  if (lanes) *lanes = v[1];
  return SL_OK;
}

int sl_batch_set_mode(sl_batch *B, int mode) {
  if (!B || !(mode == SL_BATCH_PERSISTENT || mode == SL_BATCH_PHASED))
    return bfail(B, SL_E_ARG, "mode must be SL_BATCH_PERSISTENT or SL_BATCH_PHASED");
  B->mode = mode;
  return SL_OK;
}

int sl_batch_get_mode(sl_batch *B, int *mode) {
  if (!B || !mode) return bfail(B, SL_E_ARG, "NULL argument");
  *mode = B->mode;
  return SL_OK;
}

int sl_batch_set_lanes(sl_batch *B, int lanes) {
  if (!B || !(lanes == 1 || lanes == 2 || lanes == 4)) return bfail(B, SL_E_ARG, "lanes must be 1, 2 or 4");
  B->lanes = lanes;
  return SL_OK;
}

int sl_batch_set_row_order(sl_batch *B, double quantum) {
  if (!B) return bfail(B, SL_E_ARG, "NULL batch");
  if (!(quantum >= 0.0) || !std::isfinite(quantum))
    return bfail(B, SL_E_ARG, "row-order grid step must be finite and >= 0");
  for (int r = 0; r < B->R; ++r) {
    const int rc = sl_set_row_order(B->sys[r], quantum);
    if (rc) return bfail(B, rc, B->sys[r]->last_err);
  }
  B->row_q = quantum;
  return SL_OK;
}

int sl_batch_get_stats(sl_batch *B, int64_t *launches, int64_t *rebuilds, int *lanes) {
  if (!B) return bfail(B, SL_E_ARG, "NULL batch");
  if (launches) *launches = B->launches;
  if (rebuilds) *rebuilds = B->rebuilds;
  if (lanes) *lanes = B->lanes;
  return SL_OK;
}

const char *sl_batch_last_error(const sl_batch *B) { return B ? B->last_err.c_str() : g_batch_err.c_str(); }

}  // extern "C"
