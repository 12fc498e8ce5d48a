// sl_force.hip -- force kernels of the spin-lattice step on gfx950:
//   * k_eam_density: first pass of the embedded-atom terms;
//   * k_force:       pair + magneto-mechanical force (Eq. p_advance), fused
//                    with the velocity-Verlet half kicks and the drift into
//                    the other position buffer, energies on sampled steps
//                    and the per-block terms of the rebuild predictor;
//   * k_pred_reduce: one block joining those terms and handing them to the
//                    host.
#include "sl_step.h"

namespace sl {

template <typename real>
__global__ __launch_bounds__(kBlock) void k_eam_density(SysView<real> S, PotConst P) {
  const int i = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i < S.n) eam_density_atom<real>(S, P, i);
}

template <typename real>
void launch_eam_density(const SysView<real> &S, const PotConst &P, hipStream_t st) {
  if (S.n > 0 && P.eam_on && S.eam)
    hipLaunchKernelGGL((k_eam_density<real>), dim3((S.n + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       st, S, P);
}
template void launch_eam_density<double>(const SysView<double> &, const PotConst &, hipStream_t);
template void launch_eam_density<float>(const SysView<float> &, const PotConst &, hipStream_t);


template <typename real, int MODE, int LANES, int MLP>
__global__ __launch_bounds__(kBlock, kForceWaves) void k_force(SysView<real> S, PotConst P, ForceArgs A) {
  __shared__ double red[kBlock / 64][8];
  __shared__ double redm[kBlock / 64][3];
  // With a tile table (A.tiles) block b takes the atom range the host gave
  // it: XCD b % 8 holds the same spatial slab of every colour class, so its
  // L2 serves the neighbour gathers of all classes of that slab. Without
  // one, tiles are taken from the end of the atom order first: the last
  // colour classes may hold a few atoms scattered over the whole box
  // (repairs), whose gathers miss the caches; starting them first hides
  // their latency behind the bulk instead of leaving them as the tail.
  int tile, i, l;
  bool valid;
  if (A.tiles) {
    const int2 rg = A.tiles[blockIdx.x];
    tile = blockIdx.x;
    i = rg.x + (int)threadIdx.x / LANES;
    l = threadIdx.x & (LANES - 1);
    valid = i < rg.y;
  } else {
    tile = gridDim.x - 1 - xcd_tile(blockIdx.x, gridDim.x);
    const int t = tile * kBlock + threadIdx.x;
    l = t & (LANES - 1);
    i = t / LANES;
    valid = i < S.n;
  }
  double e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double dm = 0.0, vm = 0.0, wm = kInf;
  force_atom<real, MODE, LANES, MLP>(S, P, A, i, valid, l, e, dm, vm, wm);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (MODE & kModeEnergy) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double x = wave_sum(e[c]);
      if (lane == 0) red[wv][c] = x;
    }
  }
  if (MODE & (kModeFinal | kModeNext)) {
    const double a = wave_max(dm), b = wave_max(vm), c = wave_min(wm);
    if (lane == 0) { redm[wv][0] = a; redm[wv][1] = b; redm[wv][2] = c; }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (MODE & kModeEnergy) {
      for (int c = 0; c < 8; ++c) {
        double x = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) x += red[w][c];
        A.partial[(size_t)tile * 8 + c] = x;
      }
    }
    // Predictor terms go out as plain per-block stores; k_pred_reduce joins
    // them. (Device-scope atomics on three shared words, plus a completion
    // counter, cost ~50 us per launch at 1688 blocks: they serialise across
    // the XCDs.)
    if (MODE & (kModeFinal | kModeNext)) {
      double a = 0.0, b = 0.0, c = kInf;
      for (int w = 0; w < kBlock / 64; ++w) {
        a = fmax(a, redm[w][0]);
        b = fmax(b, redm[w][1]);
        c = fmin(c, redm[w][2]);
      }
      A.pred[(size_t)tile * 3 + 0] = a;
      A.pred[(size_t)tile * 3 + 1] = b;
      A.pred[(size_t)tile * 3 + 2] = c;
    }
  }
}

// Joins the per-block predictor terms of one force launch (max, max, min:
// exact in any order) and writes them, with the sticky error word, to the
// pinned host slot; the written marker goes last.
__global__ __launch_bounds__(kBlock) void k_pred_reduce(const double *pred, int nb, int *err,
                                                        double *host_out) {
  __shared__ double s[3][kBlock / 64];
  double a = 0.0, b = 0.0, c = kInf;
  for (int k = threadIdx.x; k < nb; k += kBlock) {
    a = fmax(a, pred[(size_t)k * 3 + 0]);
    b = fmax(b, pred[(size_t)k * 3 + 1]);
    c = fmin(c, pred[(size_t)k * 3 + 2]);
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
    const int e = atomicOr(err, 0);
    host_out[0] = a;
    host_out[1] = b;
    host_out[2] = (double)e;
    host_out[4] = c;
    __threadfence_system();
    host_out[3] = 1.0;  // written marker
  }
}

void launch_pred_reduce(const double *pred, int nb, int *err, double *host_out, hipStream_t st) {
  hipLaunchKernelGGL(k_pred_reduce, dim3(1), dim3(kBlock), 0, st, pred, nb, err, host_out);
}


template <typename real, int LANES, int MLP>
static void force_lanes2(const SysView<real> &S, const PotConst &P, const ForceArgs &A,
                         hipStream_t st) {
  const long threads = (long)S.n * LANES;
  const int nb = A.tiles ? A.ntiles : (int)((threads + kBlock - 1) / kBlock);
  switch (A.mode) {
#define SL_FORCE_CASE(m) \
  case m: hipLaunchKernelGGL((k_force<real, m, LANES, MLP>), dim3(nb), dim3(kBlock), 0, st, S, P, A); break;
    SL_FORCE_CASE(1) SL_FORCE_CASE(2) SL_FORCE_CASE(3) SL_FORCE_CASE(4)
    SL_FORCE_CASE(5) SL_FORCE_CASE(6) SL_FORCE_CASE(7)
#undef SL_FORCE_CASE
    default: break;
  }
}

template <typename real, int LANES>
static void force_lanes(const SysView<real> &S, const PotConst &P, const ForceArgs &A,
                        hipStream_t st) {
  if (P.soc_on && P.eam_on) force_lanes2<real, LANES, 12>(S, P, A, st);
  else if (P.eam_on) force_lanes2<real, LANES, 8>(S, P, A, st);
  else if (P.soc_on) force_lanes2<real, LANES, 4>(S, P, A, st);
  else if (sizeof(real) == 4 && S.spl.t) force_lanes2<real, LANES, (sizeof(real) == 4 ? 2 : 0)>(S, P, A, st);
  else if (sizeof(real) == 4 && S.tab) force_lanes2<real, LANES, (sizeof(real) == 4 ? 1 : 0)>(S, P, A, st);
  else force_lanes2<real, LANES, 0>(S, P, A, st);
}

// Pair pass of the split force: the spin-independent terms of every atom
// into A.fp (MODE is 0 or kModeEnergy: with it the pair energy is stored
// too). No reductions, kicks or predictor: the spin pass does those.
template <typename real, int MODE, int LANES, int MLP>
__global__ __launch_bounds__(kBlock, kForceWaves) void k_pair(SysView<real> S, PotConst P, ForceArgs A) {
  const int tile = gridDim.x - 1 - xcd_tile(blockIdx.x, gridDim.x);
  const int t = tile * kBlock + threadIdx.x;
  const int l = t & (LANES - 1);
  const int i = t / LANES;
  double e[8];
  double dm = 0.0, vm = 0.0, wm = kInf;
  force_atom<real, MODE, LANES, MLP | 16>(S, P, A, i, i < S.n, l, e, dm, vm, wm);
}

template <typename real, int LANES, int MLP>
static void pair_lanes2(const SysView<real> &S, const PotConst &P, const ForceArgs &A,
                        bool energy, hipStream_t st) {
  const int nb = (int)(((long)S.n * LANES + kBlock - 1) / kBlock);
  if (energy)
    hipLaunchKernelGGL((k_pair<real, kModeEnergy, LANES, MLP>), dim3(nb), dim3(kBlock), 0, st, S, P, A);
  else
    hipLaunchKernelGGL((k_pair<real, 0, LANES, MLP>), dim3(nb), dim3(kBlock), 0, st, S, P, A);
}

template <typename real>
void launch_pair(const SysView<real> &S, const PotConst &P, const ForceArgs &A, int lanes,
                 bool energy, hipStream_t st) {
  if (S.n <= 0) return;
  if (lanes == 2) {
    if (P.eam_on) pair_lanes2<real, 2, 8>(S, P, A, energy, st);
    else pair_lanes2<real, 2, 0>(S, P, A, energy, st);
  } else {
    if (P.eam_on) pair_lanes2<real, 1, 8>(S, P, A, energy, st);
    else pair_lanes2<real, 1, 0>(S, P, A, energy, st);
  }
}
template void launch_pair<double>(const SysView<double> &, const PotConst &, const ForceArgs &, int,
                                  bool, hipStream_t);
template void launch_pair<float>(const SysView<float> &, const PotConst &, const ForceArgs &, int,
                                 bool, hipStream_t);

// Spin pass of the split force (the pair pass must have filled A.fp).
template <typename real>
void launch_force_spin(const SysView<real> &S, const PotConst &P, const ForceArgs &A, int lanes,
                       hipStream_t st) {
  if (S.n <= 0) return;
  if (lanes == 2) {
    if (P.soc_on) force_lanes2<real, 2, 4 | 32>(S, P, A, st);
    else force_lanes2<real, 2, 32>(S, P, A, st);
  } else {
    if (P.soc_on) force_lanes2<real, 1, 4 | 32>(S, P, A, st);
    else force_lanes2<real, 1, 32>(S, P, A, st);
  }
}
template void launch_force_spin<double>(const SysView<double> &, const PotConst &,
                                        const ForceArgs &, int, hipStream_t);
template void launch_force_spin<float>(const SysView<float> &, const PotConst &, const ForceArgs &,
                                       int, hipStream_t);

// Blocks needed by a force launch (rows of the partial-sum buffer).
int force_blocks(int n, int lanes) { return (int)(((long)n * lanes + kBlock - 1) / kBlock); }

template <typename real>
void launch_force(const SysView<real> &S, const PotConst &P, const ForceArgs &A, int lanes,
                  hipStream_t st) {
  if (S.n <= 0) return;
  switch (lanes) {
    case 1: force_lanes<real, 1>(S, P, A, st); break;
    case 2: force_lanes<real, 2>(S, P, A, st); break;
    case 8: force_lanes<real, 8>(S, P, A, st); break;
    default: force_lanes<real, 4>(S, P, A, st); break;
  }
}


template void launch_force<double>(const SysView<double> &, const PotConst &, const ForceArgs &,
                                   int, hipStream_t);
template void launch_force<float>(const SysView<float> &, const PotConst &, const ForceArgs &, int,
                                  hipStream_t);

}  // namespace sl
