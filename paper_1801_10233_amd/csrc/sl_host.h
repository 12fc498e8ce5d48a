// sl_host.h -- host-side state shared by the translation units of the
// library's runtime (sl_system.hip: handles, step schedule, observables;
// sl_rebuild.hip: cell lists, neighbour lists, colour classes and the
// permutation; sl_train.hip: the learned potential's loss and training;
// sl_tune.hip: the autotuner; sl_batch_api.hip: batched replicas). Internal:
// the interface is spinlat.h.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/spinlat.h"
#include "sl_device.h"
#include "sl_kernels.h"
#include "sl_mlp_host.h"

namespace sl {


// message of the last failed sl_create (no handle to hold it)
extern thread_local std::string g_create_err;

constexpr int kThermoCap = 1 << 16;
constexpr int kJpBatch = 16;
constexpr int kPinWords = 128;  // rebuild read-back: report at 0, class offsets at 16
constexpr int kSmallClassDefault = 128;

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
  int launches;  // launches between the two events
};

struct SlotMeta {
  int64_t boundary = -1;
  double dt = 0.0;
  bool rebuilt_after = false;
};


}  // namespace sl

using namespace sl;

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
  // Runs of consecutive classes of at most this many atoms share one
  // single-workgroup launch (-1: never). Meant for the few-atom classes a
  // colour repair adds; at 500 atoms per class (2000-atom lattice) separate
  // launches are 2x faster, so the default stays well below that.
  int small_class = kSmallClassDefault;
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
  int2 *ftile = nullptr;   // [force blocks] atom range of each force block (slabs per XCD)
  int ftile_n = 0;         // blocks of the tiled force launch (0: untiled)
  int ftile_lanes = -1;    // force lanes the tiles were made for (-1: stale)
  std::vector<int2> ftile_host;
  int2 *jtile = nullptr;   // the same slab tiles with 256 atoms per block (exchange cache)
  int jtile_n = 0;
  std::vector<int2> jtile_host;
  unsigned int *done = nullptr;
  double *partial = nullptr, *red_out = nullptr;
  double *thermo = nullptr;
  double *ring = nullptr;      // pinned host [4 boundaries][8]
  double *ring_dev = nullptr;  // device alias of ring
  int *pin = nullptr;          // pinned host words read back by a rebuild [kPinWords]
  int *pin_dev = nullptr;      // device alias of pin
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
  // Class 0 has already taken the first spin update of step `step` (merged
  // into the launch that closed the previous step); its spins at the step
  // boundary are held at [n + i] of the spin arrays for the force launch.
  bool held = false;
  int prof_group = -1;    // kind of the open run of launches (ProfGroup), or -1
  int prof_group_n = 0;
  double prof_group_work = 0.0;
  std::vector<ProfRec> prof_recs;
  std::vector<hipEvent_t> ev_pool;
  int64_t prof_launch[5] = {0, 0, 0, 0, 0};
  double prof_ms[5] = {0, 0, 0, 0, 0};
  double prof_work[5] = {0, 0, 0, 0, 0};

  std::string last_err;
};

namespace sl {

inline int fail(sl_system *S, int code, const std::string &msg) {
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
inline hipError_t dalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  // Not cleared: a clear on the null stream would not be ordered with the
  // library's non-blocking stream. Every buffer is written before it is read
  // (list slots past a row's end are masked, and gathered indices are
  // range-checked before use).
  return hipMalloc((void **)p, count * sizeof(T));
}

inline void dfree(void *p) {
  if (p) (void)hipFree(p);
}

template <typename real>
inline SysView<real> view(sl_system *S, int posbuf) {
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
  v.held = 0;
  if (S->mlp && S->mlp_mode == SL_MLP_SPLINE) {
    v.spl = S->mlp->spline_view();
    v.spl.jshift = S->pot.ex_shift ? 1 : 0;
  } else if (S->mlp) {
    v.tab = S->tab[posbuf];
  }
  return v;
}

// --- profiling -------------------------------------------------------------
inline hipEvent_t get_event(sl_system *S) {
  if (!S->ev_pool.empty()) {
    hipEvent_t e = S->ev_pool.back();
    S->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// One launch between two events on its stream; inside a ProfGroup of the same
// kind the launch is counted in the group and records no events of its own.
struct ProfScope {
  sl_system *S;
  int kind;
  double work;
  hipEvent_t a = nullptr;
  hipStream_t st;
  ProfScope(sl_system *S_, int kind_, double work_, hipStream_t st_ = nullptr)
      : S(S_), kind(kind_), work(work_), st(st_ ? st_ : S_->st) {
    if (!S->prof_now) return;
    if (S->prof_group == kind && st == S->st) {
      S->prof_group_n += 1;
      S->prof_group_work += work;
      return;
    }
    a = get_event(S);
    (void)hipEventRecord(a, st);
  }
  ~ProfScope() {
    if (a) {
      hipEvent_t b = get_event(S);
      (void)hipEventRecord(b, st);
      S->prof_recs.push_back({kind, a, b, work, 1});
    }
  }
};

// A run of consecutive launches of one kind on the library stream, with
// nothing else launched between them: two events around the whole run, so
// that the average launch time is not inflated by an event pair per launch.
struct ProfGroup {
  sl_system *S;
  hipEvent_t a = nullptr;
  ProfGroup(sl_system *S_, int kind) : S(S_) {
    if (!S->prof_now || S->prof_group >= 0) return;
    a = get_event(S);
    (void)hipEventRecord(a, S->st);
    S->prof_group = kind;
    S->prof_group_n = 0;
    S->prof_group_work = 0.0;
  }
  ~ProfGroup() {
    if (!a) return;
    hipEvent_t b = get_event(S);
    (void)hipEventRecord(b, S->st);
    if (S->prof_group_n > 0) {
      S->prof_recs.push_back({S->prof_group, a, b, S->prof_group_work, S->prof_group_n});
    } else {
      S->ev_pool.push_back(a);
      S->ev_pool.push_back(b);
    }
    S->prof_group = -1;
  }
};

// --- sl_system.hip ----------------------------------------------------------
double list_radius(const sl_system *S);
double spin_radius(const sl_system *S);
double colour_radius(const sl_system *S);
int check_box(sl_system *S);
void make_potconst(sl_system *S);
void prof_collect(sl_system *S);
int read_err(sl_system *S);
int sticky_code(sl_system *S);
int alloc_atoms(sl_system *S, Atoms &A);
void free_atoms(Atoms &A);
int ensure_table(sl_system *S, int b);
double noise_amp(const sl_system *S, double h);
int record_thermo(sl_system *S, int64_t boundary);
int wait_predictor(sl_system *S, int64_t boundary, double dt_next, bool *due);
int load_aos(sl_system *S, const double *src, int where, std::vector<double> &host);
// (instantiated for double and float)
int force_tiles(sl_system *S);
int force_nb(const sl_system *S);
int force_block_cap(int n);
template <typename real>
int force_launch(sl_system *S, int posbuf, int mode, double dt, int64_t boundary,
                 bool split = false);
template <typename real>
int energy_now(sl_system *S, double out[8]);
template <typename real>
int fields_now(sl_system *S, double *F, double *hw, int where);
template <typename real>
int temps_now(sl_system *S, double *TL, double *TS);

// --- sl_rebuild.hip ---------------------------------------------------------
int ensure_cells(sl_system *S, int ncell);
int ensure_bins(sl_system *S, int nbin);
void cell_grid(sl_system *S, CellGrid &G);
int bin_cells(sl_system *S, CellGrid &G);
ColourArgs colour_args(sl_system *S);
int jp_rounds(sl_system *S, const ColourArgs &C);
int mlp_pairs(sl_system *S);
int colour_and_permute(sl_system *S, bool repair);
int rebuild(sl_system *S);
int ensure_ready(sl_system *S);

// --- sl_tune.hip ------------------------------------------------------------
int user_state(sl_system *S, std::vector<double> &r, std::vector<double> &v,
               std::vector<double> &sp, std::vector<double> &m);
int clone_system(sl_system *S, sl_system **out);
std::string tune_key(const std::string &what);
bool cache_lookup(const std::string &key, int vals[4]);
void cache_store(const std::string &key, const int vals[4]);

// --- sl_train.hip -----------------------------------------------------------
int mlp_trainer(sl_mlp *m, const sl_dataset *d);
int mfail_str(sl_mlp *m, int code, const std::string &msg);

}  // namespace sl
