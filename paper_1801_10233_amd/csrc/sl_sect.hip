// sl_sect.hip -- the paper's own spin ordering on gfx950 (Sec. 5.1, Eq.
// spin_ST_sectoring): the box is split into gx x gy x gz processor
// subdomains, each bisected once per dimension into 8 sectors; class k is
// sector k of every subdomain. Within a class the subdomains are
// independent (a sector is at least the spin radius wide, so two atoms in
// sector k of different subdomains never interact) and run in parallel, one
// thread each; inside one subdomain's sector the atoms are updated one after
// another in id order (reversed on backward sweeps), as one processor of the
// paper would. The serial ordering of Eq. spin_ST_decomposition is the same
// machinery with one class and one subdomain.
#include <hipcub/hipcub.hpp>

#include "sl_step.h"

namespace sl {

// Sector and subdomain of every atom from its wrapped position at the start
// of the step; key = (bin << 32) | id with bin = class * nproc + subdomain.
__global__ __launch_bounds__(kBlock) void k_sect_keys(SectKeyArgs A) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  int bin = 0;
  if (A.serial == 0) {
    const double r[3] = {A.rx[i], A.ry[i], A.rz[i]};
    int p[3], b[3];
    for (int a = 0; a < 3; ++a) {
      const double x = r[a] - A.L[a] * floor(r[a] / A.L[a]);
      const double f = x / A.L[a] * A.g[a];
      int q = (int)floor(f);
      if (q >= A.g[a]) q = A.g[a] - 1;
      if (!(q >= 0)) q = 0;  // never outside the grid, whatever the input
      p[a] = q;
      b[a] = (f - q) >= 0.5;
    }
    const int sec = b[0] + 2 * b[1] + 4 * b[2];
    const int prc = p[0] + A.g[0] * (p[1] + A.g[1] * p[2]);
    bin = sec * A.nproc + prc;
  }
  A.keys[i] = ((unsigned long long)(unsigned)bin << 32) | (unsigned)A.id[i];
  A.vals[i] = i;
  atomicAdd(&A.count[bin], 1);
}

// Offsets of the bins and the atoms sorted by (bin, id). Temporary storage
// is grown on demand through *tmp / *tmp_bytes (owned by the caller).
int sect_sort(const SectKeyArgs &A, int nbins, unsigned long long *keys_out, int *vals_out,
              int *off, void **tmp, size_t *tmp_bytes, hipStream_t st) {
  if (A.n <= 0) return 0;
  int bits = 32 + 1;
  while ((1ll << (bits - 32)) < (long long)nbins) ++bits;
  size_t need_sort = 0, need_scan = 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, need_sort, A.keys, keys_out, A.vals, vals_out,
                                         A.n, 0, bits, st) != hipSuccess)
    return -1;
  if (hipcub::DeviceScan::ExclusiveSum(nullptr, need_scan, A.count, off, nbins + 1, st) !=
      hipSuccess)
    return -1;
  const size_t need = need_sort > need_scan ? need_sort : need_scan;
  if (need > *tmp_bytes) {
    if (*tmp) (void)hipFree(*tmp);
    *tmp = nullptr;
    *tmp_bytes = 0;
    if (hipMalloc(tmp, need) != hipSuccess) return -1;
    *tmp_bytes = need;
  }
  size_t b1 = *tmp_bytes, b2 = *tmp_bytes;
  if (hipcub::DeviceRadixSort::SortPairs(*tmp, b1, A.keys, keys_out, A.vals, vals_out, A.n, 0,
                                         bits, st) != hipSuccess)
    return -1;
  if (hipcub::DeviceScan::ExclusiveSum(*tmp, b2, A.count, off, nbins + 1, st) != hipSuccess)
    return -1;
  return 0;
}

void launch_sect_keys(const SectKeyArgs &A, hipStream_t st) {
  if (A.n > 0) hipLaunchKernelGGL(k_sect_keys, dim3((A.n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, A);
}

// One class of a sectored sweep: thread q walks subdomain q's atoms of the
// class in order, one full spin update each.
template <typename real, bool LANGEVIN, bool ANISO, int MLP>
__global__ __launch_bounds__(64) void k_sect_phase(SysView<real> S, PotConst P, SectPhaseArgs A) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= A.nproc) return;
  const int b = A.cls * A.nproc + q;
  const int beg = A.off[b], cnt = A.off[b + 1] - beg;
  const int64_t step[kMaxRep] = {A.step, A.step, A.step, A.step};
  const int sub[kMaxRep] = {A.sub, A.sub, A.sub, A.sub};
  for (int t = 0; t < cnt; ++t) {
    const int i = A.order[A.backward ? beg + cnt - 1 - t : beg + t];
    spin_update<real, LANGEVIN, ANISO, 1, MLP>(S, P, i, true, 0, 1, step, sub, A.h, A.amp, A.seed,
                                               A.replica, A.rs2);
  }
}

template <typename real, int MLP>
static void sect_phase_variant(const SysView<real> &S, const PotConst &P, const SectPhaseArgs &A,
                               hipStream_t st) {
  const dim3 grid((A.nproc + 63) / 64), blk(64);
  const bool lg = P.langevin != 0, an = P.aniso_on != 0;
  if (lg && an) hipLaunchKernelGGL((k_sect_phase<real, true, true, MLP>), grid, blk, 0, st, S, P, A);
  else if (lg) hipLaunchKernelGGL((k_sect_phase<real, true, false, MLP>), grid, blk, 0, st, S, P, A);
  else if (an) hipLaunchKernelGGL((k_sect_phase<real, false, true, MLP>), grid, blk, 0, st, S, P, A);
  else hipLaunchKernelGGL((k_sect_phase<real, false, false, MLP>), grid, blk, 0, st, S, P, A);
}

template <typename real>
void launch_sect_phase(const SysView<real> &S, const PotConst &P, const SectPhaseArgs &A,
                       hipStream_t st) {
  if (A.nproc <= 0) return;
  if (P.soc_on) sect_phase_variant<real, 4>(S, P, A, st);
  else if (S.jc) sect_phase_variant<real, 3>(S, P, A, st);
  else if (sizeof(real) == 4 && S.spl.t) sect_phase_variant<real, (sizeof(real) == 4 ? 2 : 0)>(S, P, A, st);
  else if (sizeof(real) == 4 && S.tab) sect_phase_variant<real, (sizeof(real) == 4 ? 1 : 0)>(S, P, A, st);
  else sect_phase_variant<real, 0>(S, P, A, st);
}
template void launch_sect_phase<double>(const SysView<double> &, const PotConst &,
                                        const SectPhaseArgs &, hipStream_t);
template void launch_sect_phase<float>(const SysView<float> &, const PotConst &,
                                       const SectPhaseArgs &, hipStream_t);

}  // namespace sl
