// sl_batch_api.hip -- batched replicas behind the sl_batch_* entry points:
// one system per replica, advanced by the persistent kernel (replayed from a
// hipGraph) or by the phase-batched kernels of sl_batch.hip, and their
// autotuner.
#include "sl_host.h"

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

