// sl_train.hip -- loss, gradient and Adam training of the learned pair
// potential on snapshots (BF16-MFMA forward, tangent and reverse kernels of
// sl_mlp.hip), through a private system that holds the snapshot geometry.
#include "sl_host.h"

namespace sl {

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


int mfail_str(sl_mlp *m, int code, const std::string &msg) {
  if (m) m->last_err = msg;
  return code;
}

}  // namespace sl

extern "C" {

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
