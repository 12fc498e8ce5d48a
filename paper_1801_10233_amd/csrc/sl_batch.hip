// sl_batch.hip -- batched replicas on gfx950: the persistent kernel (one
// workgroup runs all steps of one replica) and the phase-batched kernels
// (one launch per colour phase or force pass over every replica).
#include "sl_step.h"

namespace sl {

// ---------------------------------------------------------------------------
// Batched replicas in one persistent launch: workgroup b owns replica b and
// runs its steps one after another -- the colour classes of both spin
// half-steps separated by workgroup barriers, then force, kicks and drift --
// with the same per-step rebuild rule as the single-system path: before a
// step (other than the first of a launch) the predictor of the boundary
// before the previous one decides; if a rebuild is due the replica stops
// and the host rebuilds it before the next launch. Replicas are
// independent, so no two workgroups ever wait on each other.
template <typename real, int LANES, int MLP>
__global__ __launch_bounds__(kBatchBlock) void k_batch_run(RepDesc<real> *D) {
  __shared__ double redm[kBatchBlock / 64][3];
  __shared__ double bcast[3];
  RepDesc<real> &d = D[blockIdx.x];
  const int t = threadIdx.x, l = t & (LANES - 1), per = kBatchBlock / LANES;
  int pos = d.pos;
  int64_t step = d.step;
  const int64_t target = d.target;
  double cdm = d.cur_dm, cvm = d.cur_vm, cdt = d.cur_dt, cwm = d.cur_wm;
  double pdm = d.prev_dm, pvm = d.prev_vm, pdt = d.prev_dt, pwm = d.prev_wm;
  int crb = d.cur_rebuilt, prb = d.prev_rebuilt, havep = d.have_prev;
  int stopped = 0;
  bool first = true;
  const int K = d.K;
  while (step < target) {
    if (!first && !d.user_list && havep) {
      const double Dp = (prb ? 0.0 : pdm) + 2.0 * fabs(pdt) * pvm;
      const double Wp = (prb ? d.wr : sqrt(pwm)) - 4.0 * fabs(pdt) * pvm;
      if (Dp >= d.thr || Wp < d.ex_rc + 0.01) { stopped = 1; break; }
    }
    first = false;
    for (int half = 0; half < 2; ++half) {
      const SysView<real> &V = d.V[half == 0 ? pos : 1 - pos];
      const int subf = 2 * half;
      for (int q = 0; q < 2 * K - 1; ++q) {
        const int c = q < K ? q : 2 * K - 2 - q;
        int64_t st[kMaxRep] = {step, step, step, step};
        int sb[kMaxRep] = {subf, subf + 1, 0, 0};
        int nrep = 1;
        if (q == K - 1) nrep = 2;
        else if (q > K - 1) sb[0] = subf + 1;
        const int b0 = d.off[c], b1 = d.off[c + 1];
        for (int base = b0; base < b1; base += per) {
          const int i = base + t / LANES;
          spin_update<real, true, true, LANES, (MLP & 7)>(V, d.P, i, i < b1, l, nrep, st, sb, d.h, d.amp,
                                                     d.seed, d.replica, d.rs2);
        }
        __syncthreads();
      }
    }
    // force at the boundary after this step (positions 1 - pos); the drift
    // of the next step goes to buffer pos
    if ((MLP & 8) && d.P.eam_on) {
      // embedded-atom densities first (read by every atom's force)
      const SysView<real> &Wd = d.V[1 - pos];
      for (int base = 0; base < Wd.n; base += kBatchBlock)
        if (base + t < Wd.n) eam_density_atom<real>(Wd, d.P, base + t);
      __syncthreads();
    }
    ForceArgs F = d.F;
    F.dt = d.dt;
    F.step = step + 1;
    F.nx = d.V[pos].rx == nullptr ? nullptr : const_cast<double *>(d.V[pos].rx);
    F.ny = const_cast<double *>(d.V[pos].ry);
    F.nz = const_cast<double *>(d.V[pos].rz);
    const SysView<real> &W = d.V[1 - pos];
    const bool next = step + 1 < target;
    double bdm = 0.0, bvm = 0.0, bwm = kInf;
    for (int base = 0; base < W.n; base += per) {
      const int i = base + t / LANES;
      double e[8], dm = 0.0, vm = 0.0, wm = kInf;
      if (next) force_atom<real, kModeFinal | kModeNext, LANES, MLP>(W, d.P, F, i, i < W.n, l, e, dm, vm, wm);
      else force_atom<real, kModeFinal, LANES, MLP>(W, d.P, F, i, i < W.n, l, e, dm, vm, wm);
      bdm = fmax(bdm, dm);
      bvm = fmax(bvm, vm);
      bwm = fmin(bwm, wm);
    }
    bdm = wave_max(bdm);
    bvm = wave_max(bvm);
    bwm = wave_min(bwm);
    if ((t & 63) == 0) { redm[t >> 6][0] = bdm; redm[t >> 6][1] = bvm; redm[t >> 6][2] = bwm; }
    __syncthreads();
    if (t == 0) {
      double a = 0.0, b = 0.0, c = kInf;
      for (int w = 0; w < kBatchBlock / 64; ++w) {
        a = fmax(a, redm[w][0]);
        b = fmax(b, redm[w][1]);
        c = fmin(c, redm[w][2]);
      }
      bcast[0] = a;
      bcast[1] = b;
      bcast[2] = c;
    }
    __syncthreads();
    pdm = cdm; pvm = cvm; pdt = cdt; pwm = cwm; prb = crb; havep = 1;
    cdm = bcast[0]; cvm = bcast[1]; cwm = bcast[2]; cdt = d.dt; crb = 0;
    pos = 1 - pos;
    ++step;
    __syncthreads();
  }
  if (t == 0) {
    d.pos = pos;
    d.step = step;
    d.cur_dm = cdm; d.cur_vm = cvm; d.cur_dt = cdt; d.cur_wm = cwm; d.cur_rebuilt = crb;
    d.prev_dm = pdm; d.prev_vm = pvm; d.prev_dt = pdt; d.prev_wm = pwm; d.prev_rebuilt = prb;
    d.have_prev = havep;
    d.stopped = stopped;
  }
}

template <typename real, int MLP>
static void batch_run_lanes(RepDesc<real> *D, int R, int lanes, hipStream_t st) {
  switch (lanes) {
    case 1: hipLaunchKernelGGL((k_batch_run<real, 1, MLP>), dim3(R), dim3(kBatchBlock), 0, st, D); break;
    case 2: hipLaunchKernelGGL((k_batch_run<real, 2, MLP>), dim3(R), dim3(kBatchBlock), 0, st, D); break;
    default: hipLaunchKernelGGL((k_batch_run<real, 4, MLP>), dim3(R), dim3(kBatchBlock), 0, st, D); break;
  }
}

template <typename real>
void launch_batch_run(RepDesc<real> *D, int R, int lanes, int variant, hipStream_t st) {
  if (R <= 0) return;
  switch (variant) {
    case 4: batch_run_lanes<real, 4>(D, R, lanes, st); break;
    case 8: batch_run_lanes<real, 8>(D, R, lanes, st); break;
    case 12: batch_run_lanes<real, 12>(D, R, lanes, st); break;
    default: batch_run_lanes<real, 0>(D, R, lanes, st); break;
  }
}
template void launch_batch_run<double>(RepDesc<double> *, int, int, int, hipStream_t);
template void launch_batch_run<float>(RepDesc<float> *, int, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Phase-batched replicas: one launch covers every replica's share of one
// colour phase (blockIdx.y = replica, blockIdx.x = tile of its class), so
// the whole device works on each phase instead of one workgroup per replica.
// All replicas advance in lockstep inside a call; replica r is at step
// d.step + kk with its current positions in buffer d.pos ^ (kk & 1).
template <typename real, int LANES, int MLP>
__global__ __launch_bounds__(kBlock) void k_batch_spin(const RepDesc<real> *D, BatchPhase bp) {
  const RepDesc<real> &d = D[blockIdx.y];
  const int K = d.K;
  const int subf = 2 * bp.half;
  int c, nrep = 1, s0 = subf, s1 = subf + 1;
  if (bp.p < bp.Kmax) {
    if (bp.p >= K) return;
    c = bp.p;
    if (c == K - 1) nrep = 2;
  } else {
    c = K - 2 - (bp.p - bp.Kmax);
    if (c < 0) return;
    s0 = subf + 1;
  }
  const int b0 = d.off[c], b1 = d.off[c + 1];
  const int base = b0 + (int)blockIdx.x * (kBlock / LANES);
  if (base >= b1) return;
  const int i = base + (int)threadIdx.x / LANES, l = threadIdx.x & (LANES - 1);
  const int pos = d.pos ^ (bp.kk & 1);
  const int64_t step = d.step + bp.kk;
  const int64_t st[kMaxRep] = {step, step, step, step};
  const int sb[kMaxRep] = {s0, s1, 0, 0};
  spin_update<real, true, true, LANES, MLP>(d.V[bp.half == 0 ? pos : 1 - pos], d.P, i, i < b1,
                                             l, nrep, st, sb, d.h, d.amp, d.seed, d.replica,
                                             d.rs2);
}

// Force, kicks and drift of every replica at one boundary; each block stores
// its replica's rebuild predictor terms, which k_batch_pred_reduce joins into
// the replica's pinned slot (as k_pred_reduce does for one system).
template <typename real, int MODE, int LANES, int MLP>
__global__ __launch_bounds__(kBlock) void k_batch_force(const RepDesc<real> *D, BatchPhase bp) {
  __shared__ double redm[kBlock / 64][3];
  const RepDesc<real> &d = D[blockIdx.y];
  const int n = d.V[0].n;
  const int per = kBlock / LANES;
  const int nb = (n + per - 1) / per;
  if ((int)blockIdx.x >= nb) return;
  // buffer holding this boundary's positions; the drift goes to the other
  const int cur = bp.after ? 1 - (d.pos ^ (bp.kk & 1)) : d.pos;
  const int64_t boundary = d.step + bp.kk + bp.after;
  ForceArgs F = d.F;
  F.dt = d.dt;
  F.step = boundary;
  F.nx = const_cast<double *>(d.V[1 - cur].rx);
  F.ny = const_cast<double *>(d.V[1 - cur].ry);
  F.nz = const_cast<double *>(d.V[1 - cur].rz);
  F.host_out = d.ring + 8 * (int)(boundary & 3);
  const int i = (int)blockIdx.x * per + (int)threadIdx.x / LANES, l = threadIdx.x & (LANES - 1);
  double e[8], dm = 0.0, vm = 0.0, wm = kInf;
  force_atom<real, MODE, LANES, MLP>(d.V[cur], d.P, F, i, i < n, l, e, dm, vm, wm);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double a = wave_max(dm), b = wave_max(vm), c = wave_min(wm);
  if (lane == 0) { redm[wv][0] = a; redm[wv][1] = b; redm[wv][2] = c; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = 0.0, y = 0.0, z = kInf;
    for (int w = 0; w < kBlock / 64; ++w) {
      x = fmax(x, redm[w][0]);
      y = fmax(y, redm[w][1]);
      z = fmin(z, redm[w][2]);
    }
    // per-block terms as plain stores, joined per replica by k_batch_pred_reduce
    F.pred[(size_t)blockIdx.x * 3 + 0] = x;
    F.pred[(size_t)blockIdx.x * 3 + 1] = y;
    F.pred[(size_t)blockIdx.x * 3 + 2] = z;
  }
}

// One block per replica: joins the per-block predictor terms of the force
// pass with the same BatchPhase into the replica's pinned slot (error word,
// then the written marker last).
template <typename real>
__global__ __launch_bounds__(kBlock) void k_batch_pred_reduce(const RepDesc<real> *D, BatchPhase bp,
                                                              int per) {
  __shared__ double s[3][kBlock / 64];
  const RepDesc<real> &d = D[blockIdx.x];
  const int nb = (d.V[0].n + per - 1) / per;
  const int64_t boundary = d.step + bp.kk + bp.after;
  double *host_out = d.ring + 8 * (int)(boundary & 3);
  double a = 0.0, b = 0.0, c = kInf;
  for (int k = threadIdx.x; k < nb; k += kBlock) {
    a = fmax(a, d.F.pred[(size_t)k * 3 + 0]);
    b = fmax(b, d.F.pred[(size_t)k * 3 + 1]);
    c = fmin(c, d.F.pred[(size_t)k * 3 + 2]);
  }
  a = wave_max(a);
  b = wave_max(b);
  c = wave_min(c);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { s[0][wv] = a; s[1][wv] = b; s[2][wv] = c; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) {
      a = fmax(a, s[0][w]);
      b = fmax(b, s[1][w]);
      c = fmin(c, s[2][w]);
    }
    const int e = atomicOr(d.F.err, 0);
    host_out[0] = a;
    host_out[1] = b;
    host_out[2] = (double)e;
    host_out[4] = c;
    __threadfence_system();
    host_out[3] = 1.0;  // written marker
  }
}

template <typename real, int MLP>
static void batch_spin_lanes(const RepDesc<real> *D, const dim3 &grid, const BatchPhase &bp,
                             int lanes, hipStream_t st) {
  switch (lanes) {
    case 1: hipLaunchKernelGGL((k_batch_spin<real, 1, MLP>), grid, dim3(kBlock), 0, st, D, bp); break;
    case 4: hipLaunchKernelGGL((k_batch_spin<real, 4, MLP>), grid, dim3(kBlock), 0, st, D, bp); break;
    default: hipLaunchKernelGGL((k_batch_spin<real, 2, MLP>), grid, dim3(kBlock), 0, st, D, bp); break;
  }
}

template <typename real>
void launch_batch_spin(const RepDesc<real> *D, int R, int max_class, const BatchPhase &bp,
                       int lanes, bool soc, hipStream_t st) {
  if (R <= 0 || max_class <= 0) return;
  const int per = kBlock / lanes;
  const dim3 grid((max_class + per - 1) / per, R);
  if (soc) batch_spin_lanes<real, 4>(D, grid, bp, lanes, st);
  else batch_spin_lanes<real, 0>(D, grid, bp, lanes, st);
}

template <typename real, int MODE, int MLP>
static void batch_force_mode(const RepDesc<real> *D, const dim3 &grid, const BatchPhase &bp,
                             int lanes, hipStream_t st) {
  switch (lanes) {
    case 2: hipLaunchKernelGGL((k_batch_force<real, MODE, 2, MLP>), grid, dim3(kBlock), 0, st, D, bp); break;
    case 4: hipLaunchKernelGGL((k_batch_force<real, MODE, 4, MLP>), grid, dim3(kBlock), 0, st, D, bp); break;
    default: hipLaunchKernelGGL((k_batch_force<real, MODE, 1, MLP>), grid, dim3(kBlock), 0, st, D, bp); break;
  }
}

template <typename real, int MLP>
static void batch_force_any(const RepDesc<real> *D, const dim3 &grid, int mode,
                            const BatchPhase &bp, int lanes, hipStream_t st) {
  if (mode == kModeNext) batch_force_mode<real, kModeNext, MLP>(D, grid, bp, lanes, st);
  else if (mode == kModeFinal) batch_force_mode<real, kModeFinal, MLP>(D, grid, bp, lanes, st);
  else batch_force_mode<real, kModeFinal | kModeNext, MLP>(D, grid, bp, lanes, st);
}

// Embedded-atom densities of every replica at the boundary a force pass with
// the same BatchPhase will use.
template <typename real>
__global__ __launch_bounds__(kBlock) void k_batch_density(const RepDesc<real> *D, BatchPhase bp) {
  const RepDesc<real> &d = D[blockIdx.y];
  const int cur = bp.after ? 1 - (d.pos ^ (bp.kk & 1)) : d.pos;
  const int i = (int)blockIdx.x * kBlock + (int)threadIdx.x;
  if (i < d.V[cur].n && d.P.eam_on) eam_density_atom<real>(d.V[cur], d.P, i);
}

template <typename real>
void launch_batch_force(const RepDesc<real> *D, int R, int max_n, int mode, const BatchPhase &bp,
                        int lanes, int variant, hipStream_t st) {
  if (R <= 0 || max_n <= 0) return;
  if (variant & 8)
    hipLaunchKernelGGL((k_batch_density<real>), dim3((max_n + kBlock - 1) / kBlock, R), dim3(kBlock),
                       0, st, D, bp);
  const int per = kBlock / lanes;
  const dim3 grid((max_n + per - 1) / per, R);
  switch (variant) {
    case 4: batch_force_any<real, 4>(D, grid, mode, bp, lanes, st); break;
    case 8: batch_force_any<real, 8>(D, grid, mode, bp, lanes, st); break;
    case 12: batch_force_any<real, 12>(D, grid, mode, bp, lanes, st); break;
    default: batch_force_any<real, 0>(D, grid, mode, bp, lanes, st); break;
  }
  // atoms per block of the instance batch_force_mode ran (it takes 1 lane
  // for any count other than 2 and 4)
  const int per_k = kBlock / ((lanes == 2 || lanes == 4) ? lanes : 1);
  hipLaunchKernelGGL((k_batch_pred_reduce<real>), dim3(R), dim3(kBlock), 0, st, D, bp, per_k);
}
template void launch_batch_spin<double>(const RepDesc<double> *, int, int, const BatchPhase &, int, bool, hipStream_t);
template void launch_batch_spin<float>(const RepDesc<float> *, int, int, const BatchPhase &, int, bool, hipStream_t);
template void launch_batch_force<double>(const RepDesc<double> *, int, int, int, const BatchPhase &, int, int, hipStream_t);
template void launch_batch_force<float>(const RepDesc<float> *, int, int, int, const BatchPhase &, int, int, hipStream_t);

}  // namespace sl
