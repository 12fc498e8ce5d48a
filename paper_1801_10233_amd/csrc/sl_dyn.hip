// sl_dyn.hip -- spin kernels of the spin-lattice step on gfx950:
//   * k_spin_phase: one colour class of a spin sweep (Sec. 3 / Sec. 5.1);
//   * k_spin_tail:  a run of small classes in one workgroup;
//   * k_jcache:     the optional exchange-coefficient cache;
//   * k_reduce8:    fixed-order second pass of the block partial sums.
#include "sl_step.h"

#ifndef SL_JC_CHUNK
#define SL_JC_CHUNK 5  // list slots per round of the exchange-cache kernel
                       // (3, 4 and 5 measured alike, 6, 7, 8 and 14 slower)
#endif

namespace sl {

template <typename real, bool LANGEVIN, bool ANISO, int LANES, int MLP, bool DUAL>
__global__ __launch_bounds__(kBlock) void k_spin_phase(SysView<real> S, PotConst P,
                                                       SpinPhaseArgs A, SysView<real> S2) {
  // LANES consecutive lanes share one atom: each gathers every LANES-th
  // neighbour, the partial sums are combined with cross-lane shuffles and
  // the first lane rotates and stores the spin.
  const int t = xcd_tile(blockIdx.x, gridDim.x) * kSpinBlock + threadIdx.x;
  const int l = t & (LANES - 1);
  const int i = A.begin + t / LANES;
  spin_update<real, LANGEVIN, ANISO, LANES, MLP, DUAL>(S, P, i, i < A.end, l, A.nrep, A.step,
                                                       A.sub, A.h, A.amp, A.seed, A.replica,
                                                       A.rs2, &S2, !DUAL && A.keep != 0);
}

// A run of small classes (a few atoms each, e.g. the extra colours a repair
// adds) in one workgroup: the items are applied in order with a workgroup
// barrier between them, which keeps the class order of the sweep while
// paying one launch for the whole run.
template <typename real, bool LANGEVIN, bool ANISO, int LANES, int MLP>
__global__ __launch_bounds__(kTailBlock) void k_spin_tail(SysView<real> S, PotConst P,
                                                          TailArgs T) {
  const int l = threadIdx.x & (LANES - 1);
  const int per = kTailBlock / LANES;
  for (int q = 0; q < T.nitems; ++q) {
    const TailItem &it = T.item[q];
    for (int base = it.begin; base < it.end; base += per) {
      const int i = base + (int)threadIdx.x / LANES;
      spin_update<real, LANGEVIN, ANISO, LANES, MLP>(S, P, i, i < it.end, l, it.nrep, it.step,
                                                     it.sub, T.h, T.amp, T.seed, T.replica, T.rs2);
    }
    __syncthreads();
  }
}



// Exchange coefficients at one set of positions (the optional pair
// coefficient cache): J(r_ij) for every spin-segment entry, with the same
// expression as the spin phase's own evaluation. Positions change only at
// the drift, so one evaluation serves the two spin half-steps that use
// these positions (Sec. 3: coefficients must be re-evaluated after the
// positions move, and only then).
template <typename real, bool SPL>
__global__ __launch_bounds__(kBlock) void k_jcache(SysView<real> S, PotConst P, real *out,
                                                   double rs2, const int2 *tiles) {
  // with a tile table, block b takes the atom range of entry b (one spatial
  // slab of every class per XCD, as in the force launch)
  int i, end;
  if (tiles) {
    const int2 rg = tiles[blockIdx.x];
    i = rg.x + (int)threadIdx.x;
    end = rg.y;
  } else {
    i = blockIdx.x * blockDim.x + threadIdx.x;
    end = S.n;
  }
  if (i >= end) return;
  const int ns = S.nspin[i];
  const double rix = S.rx[i], riy = S.ry[i], riz = S.rz[i];
  // slots in chunks of SL_JC_CHUNK with all loads of a chunk issued before
  // use (the row's own slots only: ns <= kcap)
  constexpr int CH = SL_JC_CHUNK;
  for (int k0 = 0; k0 < ns; k0 += CH) {
    int jj[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int k = k0 + c;
      const int j = k < ns ? S.nbr[(size_t)k * S.ld + i] : i;
      jj[c] = (unsigned)j < (unsigned)S.n ? j : i;
    }
    double xj[CH], yj[CH], zj[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      xj[c] = S.rx[jj[c]];
      yj[c] = S.ry[jj[c]];
      zj[c] = S.rz[jj[c]];
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int k = k0 + c;
      if (k >= ns) break;
      const double dx = min_image(rix - xj[c], S.L[0], S.invL[0]);
      const double dy = min_image(riy - yj[c], S.L[1], S.invL[1]);
      const double dz = min_image(riz - zj[c], S.L[2], S.invL[2]);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (SPL) {  // learned potential (spline form): J with its own cut
        out[(size_t)k * S.ld + i] = (real)spline_phys(S.spl, (float)sqrt(r2)).x;
      } else {
        out[(size_t)k * S.ld + i] = r2 < rs2 ? exch_J<real>(P, r2) : (real)0;
      }
    }
  }
}

template <typename real>
void launch_jcache(const SysView<real> &S, const PotConst &P, real *out, double rs2,
                   const int2 *tiles, int ntiles, hipStream_t st) {
  if (S.n <= 0) return;
  const dim3 grid(tiles ? ntiles : (S.n + kBlock - 1) / kBlock);
  if (S.spl.t) hipLaunchKernelGGL((k_jcache<real, true>), grid, dim3(kBlock), 0, st, S, P, out, rs2, tiles);
  else hipLaunchKernelGGL((k_jcache<real, false>), grid, dim3(kBlock), 0, st, S, P, out, rs2, tiles);
}
template void launch_jcache<double>(const SysView<double> &, const PotConst &, double *, double,
                                    const int2 *, int, hipStream_t);
template void launch_jcache<float>(const SysView<float> &, const PotConst &, float *, double,
                                   const int2 *, int, hipStream_t);

// Fixed-order sum of nb partial rows of 8 doubles (deterministic result).
__global__ __launch_bounds__(256) void k_reduce8(const double *partial, int nb, double *out) {
  __shared__ double buf[256][8];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += 256)
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] += partial[(size_t)b * 8 + c];
#pragma unroll
  for (int c = 0; c < 8; ++c) buf[threadIdx.x][c] = acc[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int c = 0; c < 8; ++c) buf[threadIdx.x][c] += buf[threadIdx.x + w][c];
    __syncthreads();
  }
  if (threadIdx.x < 8) out[threadIdx.x] = buf[0][threadIdx.x];
}


// ---------------------------------------------------------------------------
// Host launchers. The learned-potential variants (table lookups instead of
// the analytic J and V) exist in the FP32 form only; variant 4 is the
// analytic potential with the spin-orbit pair terms.
template <typename real, int LANES, int MLP, bool DUAL>
static void spin_phase_lanes3(const SysView<real> &S, const PotConst &P, const SpinPhaseArgs &A,
                              const SysView<real> &S2, hipStream_t st) {
  const long threads = (long)(A.end - A.begin) * LANES;
  const int nb = (int)((threads + kSpinBlock - 1) / kSpinBlock);
  const bool lg = P.langevin != 0, an = P.aniso_on != 0;
  if (lg && an) hipLaunchKernelGGL((k_spin_phase<real, true, true, LANES, MLP, DUAL>), dim3(nb), dim3(kSpinBlock), 0, st, S, P, A, S2);
  else if (lg) hipLaunchKernelGGL((k_spin_phase<real, true, false, LANES, MLP, DUAL>), dim3(nb), dim3(kSpinBlock), 0, st, S, P, A, S2);
  else if (an) hipLaunchKernelGGL((k_spin_phase<real, false, true, LANES, MLP, DUAL>), dim3(nb), dim3(kSpinBlock), 0, st, S, P, A, S2);
  else hipLaunchKernelGGL((k_spin_phase<real, false, false, LANES, MLP, DUAL>), dim3(nb), dim3(kSpinBlock), 0, st, S, P, A, S2);
}

template <typename real, int LANES, int MLP>
static void spin_phase_lanes2(const SysView<real> &S, const PotConst &P, const SpinPhaseArgs &A,
                              const SysView<real> *S2, hipStream_t st) {
  if (S2) spin_phase_lanes3<real, LANES, MLP, true>(S, P, A, *S2, st);
  else spin_phase_lanes3<real, LANES, MLP, false>(S, P, A, S, st);
}

template <typename real, int LANES>
static void spin_phase_lanes(const SysView<real> &S, const PotConst &P, const SpinPhaseArgs &A,
                             const SysView<real> *S2, hipStream_t st) {
  if (P.soc_on) spin_phase_lanes2<real, LANES, 4>(S, P, A, S2, st);
  else if (S.jc) spin_phase_lanes2<real, LANES, 3>(S, P, A, S2, st);
  else if (sizeof(real) == 4 && S.spl.t) spin_phase_lanes2<real, LANES, (sizeof(real) == 4 ? 2 : 0)>(S, P, A, S2, st);
  else if (sizeof(real) == 4 && S.tab) spin_phase_lanes2<real, LANES, (sizeof(real) == 4 ? 1 : 0)>(S, P, A, S2, st);
  else spin_phase_lanes2<real, LANES, 0>(S, P, A, S2, st);
}

template <typename real>
void launch_spin_phase(const SysView<real> &S, const PotConst &P, const SpinPhaseArgs &A,
                       int lanes, hipStream_t st, const SysView<real> *S2) {
  if (A.end - A.begin <= 0) return;
  switch (lanes) {
    case 1: spin_phase_lanes<real, 1>(S, P, A, S2, st); break;
    case 2: spin_phase_lanes<real, 2>(S, P, A, S2, st); break;
    case 8: spin_phase_lanes<real, 8>(S, P, A, S2, st); break;
    default: spin_phase_lanes<real, 4>(S, P, A, S2, st); break;
  }
}

template <typename real, int LANES, int MLP>
static void spin_tail_lanes2(const SysView<real> &S, const PotConst &P, const TailArgs &T,
                             hipStream_t st) {
  const bool lg = P.langevin != 0, an = P.aniso_on != 0;
  if (lg && an) hipLaunchKernelGGL((k_spin_tail<real, true, true, LANES, MLP>), dim3(1), dim3(kTailBlock), 0, st, S, P, T);
  else if (lg) hipLaunchKernelGGL((k_spin_tail<real, true, false, LANES, MLP>), dim3(1), dim3(kTailBlock), 0, st, S, P, T);
  else if (an) hipLaunchKernelGGL((k_spin_tail<real, false, true, LANES, MLP>), dim3(1), dim3(kTailBlock), 0, st, S, P, T);
  else hipLaunchKernelGGL((k_spin_tail<real, false, false, LANES, MLP>), dim3(1), dim3(kTailBlock), 0, st, S, P, T);
}

template <typename real, int LANES>
static void spin_tail_lanes(const SysView<real> &S, const PotConst &P, const TailArgs &T,
                            hipStream_t st) {
  if (P.soc_on) spin_tail_lanes2<real, LANES, 4>(S, P, T, st);
  else if (S.jc) spin_tail_lanes2<real, LANES, 3>(S, P, T, st);
  else if (sizeof(real) == 4 && S.spl.t) spin_tail_lanes2<real, LANES, (sizeof(real) == 4 ? 2 : 0)>(S, P, T, st);
  else if (sizeof(real) == 4 && S.tab) spin_tail_lanes2<real, LANES, (sizeof(real) == 4 ? 1 : 0)>(S, P, T, st);
  else spin_tail_lanes2<real, LANES, 0>(S, P, T, st);
}

template <typename real>
void launch_spin_tail(const SysView<real> &S, const PotConst &P, const TailArgs &T, int lanes,
                      hipStream_t st) {
  if (T.nitems <= 0) return;
  switch (lanes) {
    case 1: spin_tail_lanes<real, 1>(S, P, T, st); break;
    case 2: spin_tail_lanes<real, 2>(S, P, T, st); break;
    case 8: spin_tail_lanes<real, 8>(S, P, T, st); break;
    default: spin_tail_lanes<real, 4>(S, P, T, st); break;
  }
}


void launch_reduce8(const double *partial, int nb, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce8, dim3(1), dim3(256), 0, st, partial, nb, out);
}


template void launch_spin_phase<double>(const SysView<double> &, const PotConst &,
                                        const SpinPhaseArgs &, int, hipStream_t,
                                        const SysView<double> *);
template void launch_spin_phase<float>(const SysView<float> &, const PotConst &,
                                       const SpinPhaseArgs &, int, hipStream_t,
                                       const SysView<float> *);
template void launch_spin_tail<double>(const SysView<double> &, const PotConst &,
                                       const TailArgs &, int, hipStream_t);
template void launch_spin_tail<float>(const SysView<float> &, const PotConst &, const TailArgs &,
                                      int, hipStream_t);

}  // namespace sl
