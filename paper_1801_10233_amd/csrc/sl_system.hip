// sl_system.hip -- the system handle behind the C ABI of spinlat.h: device
// buffers, the step schedule and the observables. All per-step work runs in
// the kernels of sl_dyn.hip and sl_force.hip; this file orders launches on
// the system's stream. The rebuild pipeline is in sl_rebuild.hip.
#include "sl_host.h"

namespace sl {

thread_local std::string g_create_err = "";






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




void prof_collect(sl_system *S) {
  if (S->prof_recs.empty()) return;
  (void)hipStreamSynchronize(S->st);
  for (auto &r : S->prof_recs) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    S->prof_launch[r.kind] += r.launches;
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
  // spins: [0, n) the state, [n, 2n) the step-boundary state of class 0
  // while the next step's first update of it is already applied
  HIPCHK(S, hipMalloc(&A.sx, rs * (n > 0 ? 2 * n : 1)));
  HIPCHK(S, hipMalloc(&A.sy, rs * (n > 0 ? 2 * n : 1)));
  HIPCHK(S, hipMalloc(&A.sz, rs * (n > 0 ? 2 * n : 1)));
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
    CHK(force_tiles(S));
    launch_jcache<real>(v, S->pc, (real *)S->jc[b], S->pot.ex_rc * S->pot.ex_rc,
                        S->jtile_n > 0 ? S->jtile : nullptr, S->jtile_n, S->st);
  }
  S->jc_ok[b] = true;
  return SL_OK;
}


// --- launches ---------------------------------------------------------------
double noise_amp(const sl_system *S, double h);

// One launch of class c: nrep successive updates at buffer posbuf, or with
// dual set the two updates across the drift (the first at posbuf, the
// second at the other buffer).
template <typename real>
void spin_launch(sl_system *S, int posbuf, int c, int nrep, const int64_t *steps, const int *subs,
                 double h, bool dual = false, bool keep = false) {
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
  A.keep = keep && nrep == 2 ? 1 : 0;
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

// keep_last: the last item is the two updates of class 0 around a step
// boundary; its launch holds the state between them for the force launch.
template <typename real>
void run_updates(sl_system *S, int posbuf, const std::vector<Upd> &u, double h,
                 bool keep_last = false) {
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
  ProfGroup pg(S, 0);  // the loop launches spin phases only
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
      spin_launch<real>(S, posbuf, items[q].c, items[q].nrep, items[q].steps, items[q].subs, h,
                        false, keep_last && q + 1 == items.size());
      ++q;
    }
  }
}

// Forward (classes 1..K) then backward (K..1) sweep of one spin half-step.
void half_step_updates(const sl_system *S, int64_t step, int sub_fwd, std::vector<Upd> &u) {
  for (int c = 0; c < S->K; ++c) u.push_back({c, step, sub_fwd});
  for (int c = S->K - 1; c >= 0; --c) u.push_back({c, step, sub_fwd + 1});
}

// Capacity of the per-block buffers of a force launch: untiled launches of up
// to 8 lanes per atom, or a tile table (at most 8 partial tiles per class).
int force_block_cap(int n) { return force_blocks(n, 8) + 8 * (kMaxClass + 8); }

// Blocks of the current force launch (the rows of its partial sums).
int force_nb(const sl_system *S) {
  return S->ftile_n > 0 && S->ftile_lanes == S->force_lanes ? S->ftile_n
                                                             : force_blocks(S->n, S->force_lanes);
}

// Tile tables of the force launch (per atoms per block) and of the
// exchange-cache launch (256). Blocks are dispatched to the eight XCDs
// round-robin (block b to XCD b % 8), and each XCD has its own L2. XCD x is
// given the x-th eighth, in the atom order (z slowest), of every colour class: one slab of
// the box, whose neighbour data its L2 then serves for all classes, instead
// of half of the box for one class. Inside an XCD the tiles of the classes
// are interleaved by their place in the slab, so the blocks in flight on an
// XCD cover a thin layer of it. Classes of fewer than 8 tiles (the few atoms
// a repair adds, scattered over the box) go first, spread over the XCDs.
// Launches of fewer than 64 tiles stay untiled.
static int slab_tiles(sl_system *S, int per, int2 *dev, std::vector<int2> &host, int &nout) {
  nout = 0;
  if (S->K <= 0 || S->n <= 0 || !dev || (int)S->class_off.size() < S->K + 1) return SL_OK;
  struct Tile {
    double key;
    int a, b;
  };
  std::vector<Tile> xl[8];
  int total = 0, spread = 0;
  for (int c = S->K - 1; c >= 0; --c) {
    const int b0 = S->class_off[c], b1 = S->class_off[c + 1];
    const int T = (b1 - b0 + per - 1) / per;
    total += T;
    for (int t = 0; t < T; ++t) {
      const int a = b0 + t * per, b = std::min(b1, a + per);
      if (T < 8) {
        xl[spread % 8].push_back({-1.0, a, b});
        ++spread;
      } else {
        const int x = (int)(((long)t * 8) / T);
        const int lo = (int)(((long)T * x + 7) / 8), hi = (int)(((long)T * (x + 1) + 7) / 8);
        xl[x].push_back({(t - lo + 0.5) / (double)std::max(1, hi - lo), a, b});
      }
    }
  }
  if (total < 64) return SL_OK;
  size_t m = 0;
  for (auto &v : xl) {
    std::stable_sort(v.begin(), v.end(), [](const Tile &p, const Tile &q) { return p.key < q.key; });
    m = std::max(m, v.size());
  }
  const int nb = (int)(8 * m);
  if (nb > force_block_cap(S->n)) return SL_OK;
  host.assign((size_t)nb, make_int2(0, 0));
  for (int x = 0; x < 8; ++x)
    for (size_t k = 0; k < xl[x].size(); ++k) host[8 * k + x] = make_int2(xl[x][k].a, xl[x][k].b);
  HIPCHK(S, hipMemcpyAsync(dev, host.data(), sizeof(int2) * nb, hipMemcpyHostToDevice, S->st));
  nout = nb;
  return SL_OK;
}

int force_tiles(sl_system *S) {
  if (S->ftile_lanes == S->force_lanes) return SL_OK;
  S->ftile_lanes = S->force_lanes;
  CHK(slab_tiles(S, kBlock / S->force_lanes, S->ftile, S->ftile_host, S->ftile_n));
  return slab_tiles(S, kBlock, S->jtile, S->jtile_host, S->jtile_n);
}

// With split set, the pair pass of this boundary (pair_launch) has filled
// S->fp and the launch is the spin pass.
template <typename real>
int force_launch(sl_system *S, int posbuf, int mode, double dt, int64_t boundary,
                 bool split) {
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
  CHK(force_tiles(S));
  F.tiles = S->ftile_n > 0 ? S->ftile : nullptr;
  F.ntiles = S->ftile_n;
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
    SysView<real> v = view<real>(S, posbuf);
    v.held = S->held ? S->class_off[1] : 0;
    if (split) {
      launch_force_spin<real>(v, S->pc, F, S->force_lanes, S->st);
    } else {
      launch_eam_density<real>(v, S->pc, S->st);
      launch_force<real>(v, S->pc, F, S->force_lanes, S->st);
    }
  }
  if (mode & (kModeFinal | kModeNext))
    launch_pred_reduce(S->pred, force_nb(S), S->err, F.host_out, S->st);
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
  const int nb = force_nb(S);
  const int k = (int)S->thermo_steps.size();
  if (k >= kThermoCap) return SL_OK;
  launch_reduce8(S->partial, nb, S->thermo + (size_t)k * 8, S->st);
  S->thermo_steps.push_back(boundary);
  return SL_OK;
}

template <typename real>
int energy_now(sl_system *S, double out[8]) {
  CHK(force_launch<real>(S, S->pos, kModeEnergy, 0.0, -1));
  const int nb = force_nb(S);
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

// Undo a held first update of class 0: its spins go back to the step
// boundary's (before a rebuild at that boundary, or when a call ends early).
int release_held(sl_system *S) {
  if (!S->held) return SL_OK;
  S->held = false;
  Atoms &A = S->a[S->cur];
  const size_t rs = S->prec == SL_FP64 ? sizeof(double) : sizeof(float);
  const size_t m = (size_t)S->class_off[1];
  for (void *p : {A.sx, A.sy, A.sz})
    HIPCHK(S, hipMemcpyAsync(p, (char *)p + rs * S->n, rs * m, hipMemcpyDeviceToDevice, S->st));
  return SL_OK;
}

struct HeldGuard {  // a call never returns with a held update
  sl_system *S;
  ~HeldGuard() { (void)release_held(S); }
};

template <typename real>
int step_coupled(sl_system *S, int64_t n, double dt, bool built) {
  const double h = dt / 4.0;
  const int te = S->prm.thermo_every;
  CHK(release_held(S));
  HeldGuard guard{S};
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
    // timed steps: with prof_every 1 all, else the second of the call (the
    // first of a call has one spin launch more) and every prof_every-th after it
    S->prof_now = S->prof && (S->prof_every == 1 || (k - k0) % S->prof_every == (n > 1 ? 1 : 0));
    if (k > k0 && !S->user_list) {
      bool due;
      CHK(wait_predictor(S, k - 1, dt, &due));
      if (due) {
        CHK(release_held(S));
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
      if (S->held) {  // class 0's first update of this step is done
        u.erase(u.begin());
        S->held = false;
      }
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
        // the symmetric sweep over classes (Eq. spin_ST_sectoring) ends this step and
        // starts the next with class 0, at the drifted positions, with nothing
        // in between but the force launch, which reads the held state between
        // the two updates: one launch (undone by release_held if the list is
        // rebuilt at that boundary)
        const bool hold = c0 == 0 && w.back().c == 0 && k + 1 < k0 + n;
        if (hold) w.push_back({0, k + 1, 0});
        run_updates<real>(S, 1 - S->pos, w, h, hold);
        S->held = hold;
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


template int force_launch<double>(sl_system *, int, int, double, int64_t, bool);
template int force_launch<float>(sl_system *, int, int, double, int64_t, bool);
template int energy_now<double>(sl_system *, double[8]);
template int energy_now<float>(sl_system *, double[8]);
template int fields_now<double>(sl_system *, double *, double *, int);
template int fields_now<float>(sl_system *, double *, double *, int);
template int temps_now<double>(sl_system *, double *, double *);
template int temps_now<float>(sl_system *, double *, double *);

}  // namespace sl

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
  const int nb = force_block_cap(n);
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
  A_(dalloc(&S->jpcnt, 6));
  A_(dalloc(&S->jplist[0], (size_t)n));
  A_(dalloc(&S->jplist[1], (size_t)n));
  A_(dalloc(&S->jpmask[0], (size_t)n));
  A_(dalloc(&S->jpmask[1], (size_t)n));
  A_(dalloc(&S->maxc, 1));
  A_(dalloc(&S->dslot, 3));
  A_(dalloc(&S->done, 1));
  A_(dalloc(&S->partial, (size_t)nb * 8));
  A_(dalloc(&S->pred, (size_t)nb * 3));
  A_(dalloc(&S->ftile, (size_t)nb));
  A_(dalloc(&S->jtile, (size_t)nb));
  A_(dalloc(&S->red_out, 8));
  A_(dalloc(&S->thermo, (size_t)kThermoCap * 8));
  A_(hipHostMalloc((void **)&S->ring, 32 * sizeof(double), hipHostMallocCoherent | hipHostMallocMapped));
  for (int k = 0; k < 4; ++k) A_(hipEventCreateWithFlags(&S->ev[k], hipEventDisableTiming));
  A_(hipHostGetDevicePointer((void **)&S->ring_dev, S->ring, 0));
  A_(hipHostMalloc((void **)&S->pin, kPinWords * sizeof(int), hipHostMallocCoherent | hipHostMallocMapped));
  A_(hipHostGetDevicePointer((void **)&S->pin_dev, S->pin, 0));
#undef A_
  std::memset(S->ring, 0, 32 * sizeof(double));
  (void)hipMemsetAsync(S->err, 0, sizeof(int), S->st);
  (void)hipMemsetAsync(S->seen, 0, 2 * sizeof(int), S->st);
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
                  (void *)S->done, (void *)S->partial, (void *)S->pred, (void *)S->ftile, (void *)S->jtile, (void *)S->red_out, (void *)S->thermo,
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
  if (S->pin) (void)hipHostFree(S->pin);
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
  // the pair-coefficient caches hold values of the old potential (a user
  // list keeps its list and colouring, so no rebuild would drop them)
  S->tab_ok[0] = S->tab_ok[1] = false;
  S->jc_ok[0] = S->jc_ok[1] = false;
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
  // a colouring of the old list may not be one of the new list: the next
  // step colours and orders the atoms again (sl_set_coloring after this
  // call sets the caller's), which also drops the caches of the old list
  S->have_colour = false;
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
  S->small_class = t->small_class == 0 ? kSmallClassDefault : t->small_class;
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

}  // extern "C"
