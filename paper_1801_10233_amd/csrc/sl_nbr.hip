// sl_nbr.hip -- rebuild-step kernels on gfx950: cell binning, neighbour
// lists, colour classes of non-interacting spins and the permutation of
// the per-atom arrays into (colour, row, x) order.
//
// Colour classes play the role of the paper's sectors (Sec. 5.1): a set of
// spins none of which interact, so all of them can be rotated at once while
// the product of single-spin propagators keeps the order of
// Eq. spin_ST_sectoring. The colouring is first-fit greedy in ascending
// lexicographic key (z, y, x, id); on the GPU it is computed by
// Jones-Plassmann rounds with that key as priority: an atom is coloured once
// every earlier-key neighbour is, with the smallest colour none of its
// coloured neighbours holds, which gives exactly the greedy result.
#include "sl_device.h"
#include "sl_kernels.h"

namespace sl {

static inline int nblocks(int n) { return (n + kBlock - 1) / kBlock; }

__device__ __forceinline__ double wrap(double x, double L) { return x - L * floor(x / L); }

__device__ __forceinline__ int cell_coord(double x, double L, int nc) {
  int k = (int)(wrap(x, L) / L * nc);
  return k < 0 ? 0 : (k >= nc ? nc - 1 : k);
}

__global__ void k_cell_assign(int n, const double *rx, const double *ry, const double *rz,
                              CellGrid G, int *cell, int *count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int cx = cell_coord(rx[i], G.L[0], G.nc[0]);
  const int cy = cell_coord(ry[i], G.L[1], G.nc[1]);
  const int cz = cell_coord(rz[i], G.L[2], G.nc[2]);
  const int c = (cz * G.nc[1] + cy) * G.nc[0] + cx;
  cell[i] = c;
  atomicAdd(&count[c], 1);
}

__global__ __launch_bounds__(1024) void k_scan(const int *in, int *out, int n) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int beg = min(t * chunk, n), end = min(beg + chunk, n);
  int s = 0;
  for (int k = beg; k < end; ++k) s += in[k];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = t > 0 ? part[t - 1] : 0;
  for (int k = beg; k < end; ++k) {
    out[k] = run;
    run += in[k];
  }
  if (t == 1023) out[n] = part[1023];
}

__global__ void k_bucket_scatter(int n, const int *key, const int *start, int *fill, int *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = key[i];
  out[start[b] + atomicAdd(&fill[b], 1)] = i;
}

__global__ void k_bucket_sort_x(int nbucket, const int *start, int *items, const double *x) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbucket) return;
  const int a = start[b], e = start[b + 1];
  for (int p = a + 1; p < e; ++p) {
    const int v = items[p];
    const double xv = x[v];
    int q = p - 1;
    while (q >= a) {
      const int u = items[q];
      const double xu = x[u];
      if (xu < xv || (xu == xv && u < v)) break;
      items[q + 1] = u;
      --q;
    }
    items[q + 1] = v;
  }
}

__global__ void k_cell_positions(int n, const int *catoms, const double *rx, const double *ry,
                                 const double *rz, double *cx, double *cy, double *cz) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int j = catoms[p];
  cx[p] = rx[j];
  cy[p] = ry[j];
  cz[p] = rz[j];
}

__global__ void k_bucket_sort(int nbucket, const int *start, int *items) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbucket) return;
  const int a = start[b], e = start[b + 1];
  for (int p = a + 1; p < e; ++p) {
    const int x = items[p];
    int q = p - 1;
    while (q >= a && items[q] > x) {
      items[q + 1] = items[q];
      --q;
    }
    items[q + 1] = x;
  }
}

// Full neighbour rows from the 27 surrounding cells (fewer when a side has
// under three cells: then that side is one cell and the minimum image
// covers it). The spin segment (r^2 < rs2) comes first, then the rest of
// the row (rs2 <= r^2 < rl2); inside each segment entries follow the cell
// loop order, atoms ascending inside a cell, so rows are deterministic.
// kNbrLanes lanes share one atom, each scanning a contiguous run of the
// cells: a counting sweep, a segmented prefix sum over the lanes, then a
// writing sweep that puts every entry at its place in that order. With 16
// lanes the serial chain per thread is ~16x shorter, which small systems
// (too few atoms to fill the device) need; large systems take one lane per
// atom. Atoms are taken in cell order (thread group p builds the row of
// catoms[p]) and candidates' positions come from the cell-ordered copy
// (cx, cy, cz), so the lanes of a wavefront work on a few cells and read
// the same candidate runs, whatever the order of the atom arrays.
constexpr int kNbrManyAtoms = 1 << 16;  // from here on one lane per atom

template <int kNbrLanes>
__global__ __launch_bounds__(kBlock) void k_nbr_build(NbrBuildArgs A) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int p0 = (int)(t / kNbrLanes), l = (int)(t % kNbrLanes);
  const bool valid = p0 < A.n;
  const int i = valid ? A.catoms[p0] : 0;
  const int ox = A.G.nc[0] >= 3 ? 1 : 0, oy = A.G.nc[1] >= 3 ? 1 : 0, oz = A.G.nc[2] >= 3 ? 1 : 0;
  const int wx = 2 * ox + 1, wy = 2 * oy + 1, M = wx * wy * (2 * oz + 1);
  const int m0 = M * l / kNbrLanes, m1 = M * (l + 1) / kNbrLanes;
  const double Lx = A.G.L[0], Ly = A.G.L[1], Lz = A.G.L[2];
  const double iLx = 1.0 / Lx, iLy = 1.0 / Ly, iLz = 1.0 / Lz;
  double rix = 0, riy = 0, riz = 0;
  int cx = 0, cy = 0, cz = 0;
  if (valid) {
    rix = A.cx[p0]; riy = A.cy[p0]; riz = A.cz[p0];
    const int c = A.cell[i];
    cx = c % A.G.nc[0]; cy = (c / A.G.nc[0]) % A.G.nc[1]; cz = c / (A.G.nc[0] * A.G.nc[1]);
  }
  int cnt[2] = {0, 0};   // spin, rest
  int off[2] = {0, 0};
  for (int sweep = 0; sweep < 2; ++sweep) {
    if (valid)
      for (int m = m0; m < m1; ++m) {
        const int dx = m % wx - ox, dy = (m / wx) % wy - oy, dz = m / (wx * wy) - oz;
        const int qx = (cx + dx + A.G.nc[0]) % A.G.nc[0];
        const int qy = (cy + dy + A.G.nc[1]) % A.G.nc[1];
        const int qz = (cz + dz + A.G.nc[2]) % A.G.nc[2];
        const int q = (qz * A.G.nc[1] + qy) * A.G.nc[0] + qx;
        for (int p = A.cstart[q]; p < A.cstart[q + 1]; ++p) {
          if (p == p0) continue;
          const double ddx = min_image(rix - A.cx[p], Lx, iLx);
          const double ddy = min_image(riy - A.cy[p], Ly, iLy);
          const double ddz = min_image(riz - A.cz[p], Lz, iLz);
          const double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
          if (r2 >= A.rl2 && r2 >= A.rs2) continue;
          const int seg = r2 < A.rs2 ? 0 : 1;
          if (sweep == 0) {
            ++cnt[seg];
          } else {
            const int k = off[seg]++;
            if (k < A.max_nbr) A.nbr[(size_t)k * A.ld + i] = A.catoms[p];
          }
        }
      }
    if (sweep == 0) {
      // inclusive scans of both counts over the lanes of this atom
      int ps = cnt[0], pr = cnt[1];
#pragma unroll
      for (int o = 1; o < kNbrLanes; o <<= 1) {
        const int a = __shfl_up(ps, o, kNbrLanes), b = __shfl_up(pr, o, kNbrLanes);
        if (l >= o) { ps += a; pr += b; }
      }
      const int ts = __shfl(ps, kNbrLanes - 1, kNbrLanes), tr = __shfl(pr, kNbrLanes - 1, kNbrLanes);
      off[0] = ps - cnt[0];
      off[1] = ts + pr - cnt[1];
      cnt[0] = ts;
      cnt[1] = tr;
    }
  }
  if (!valid || l != 0) return;
  const int ns = cnt[0], nt = cnt[0] + cnt[1];
  if (nt > A.max_nbr || ns > A.max_spin) atomicOr(A.err, kErrNbrOverflow);
  atomicMax(&A.seen[0], ns);
  atomicMax(&A.seen[1], nt);
  A.nspin[i] = min(ns, A.max_spin);
  A.nall[i] = min(nt, A.max_nbr);
  A.bx[i] = rix;
  A.by[i] = riy;
  A.bz[i] = riz;
}

// Row order by displacement: each segment of a freshly built row is sorted
// by the key (z, y, x of r_j - r_i rounded to the grid 1/invq, 10 bits each,
// then j). With the atoms sorted spatially, slot k of neighbouring rows then
// holds neighbours at the same lattice offset, which lie next to each other
// in memory: the gathers of one slot across a wavefront touch few cache
// lines. One thread per atom; the keys of a segment sit in LDS, one column
// per thread (slot-major, so a wavefront's reads hit distinct banks), and
// every entry goes straight to its rank (keys are unique: they end in j).
// Segments longer than kOrderMax keep the cell-loop order.
constexpr int kOrderBlock = 64, kOrderMax = 64;
__global__ __launch_bounds__(kOrderBlock) void k_row_order(NbrBuildArgs A, double invq) {
  __shared__ unsigned long long key[kOrderMax * kOrderBlock];
  const int t = threadIdx.x;
  const int i = blockIdx.x * kOrderBlock + t;
  if (i >= A.n) return;
  const double Lx = A.G.L[0], Ly = A.G.L[1], Lz = A.G.L[2];
  const double iLx = 1.0 / Lx, iLy = 1.0 / Ly, iLz = 1.0 / Lz;
  const double rix = A.rx[i], riy = A.ry[i], riz = A.rz[i];
  const int ns = A.nspin[i], na = A.nall[i];
  auto q10 = [&](double d) -> unsigned long long {
    const double q = fmin(fmax(rint(d * invq), -511.0), 511.0);
    return (unsigned long long)((int)q + 512);
  };
  for (int seg = 0; seg < 2; ++seg) {
    const int beg = seg == 0 ? 0 : ns, end = seg == 0 ? ns : na;
    const int m = end - beg;
    if (m < 2 || m > kOrderMax) continue;
    for (int f = 0; f < m; ++f) {
      const int j = A.nbr[(size_t)(beg + f) * A.ld + i];
      const double dx = min_image(A.rx[j] - rix, Lx, iLx);
      const double dy = min_image(A.ry[j] - riy, Ly, iLy);
      const double dz = min_image(A.rz[j] - riz, Lz, iLz);
      const unsigned long long q = (q10(dz) << 20) | (q10(dy) << 10) | q10(dx);
      key[f * kOrderBlock + t] = (q << 32) | (unsigned)j;
    }
    for (int e = 0; e < m; ++e) {
      const unsigned long long ke = key[e * kOrderBlock + t];
      int rank = 0;
      for (int f = 0; f < m; ++f) rank += key[f * kOrderBlock + t] < ke ? 1 : 0;
      A.nbr[(size_t)(beg + rank) * A.ld + i] = (int)(unsigned)(ke & 0xffffffffull);
    }
  }
}

__global__ void k_keys(int n, const double *rx, const double *ry, const double *rz, double Lx,
                       double Ly, double Lz, double *kx, double *ky, double *kz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  kx[i] = wrap(rx[i], Lx);
  ky[i] = wrap(ry[i], Ly);
  kz[i] = wrap(rz[i], Lz);
}

// key(j) < key(i) in the order (z, y, x, user id).
__device__ __forceinline__ bool key_less(const ColourArgs &A, int j, int i) {
  const double zj = A.kz[j], zi = A.kz[i];
  if (zj != zi) return zj < zi;
  const double yj = A.ky[j], yi = A.ky[i];
  if (yj != yi) return yj < yi;
  const double xj = A.kx[j], xi = A.kx[i];
  if (xj != xi) return xj < xi;
  return A.id[j] < A.id[i];
}

// Whether list entry j of atom i is an edge of the colouring graph.
__device__ __forceinline__ bool conflict(const ColourArgs &A, int i, int j) {
  const double dx = min_image(A.rx[i] - A.rx[j], A.L[0], A.invL[0]);
  const double dy = min_image(A.ry[i] - A.ry[j], A.L[1], A.invL[1]);
  const double dz = min_image(A.rz[i] - A.rz[j], A.L[2], A.invL[2]);
  return dx * dx + dy * dy + dz * dz < A.cr2;
}

__global__ void k_colour_fill(int n, int *colour, int value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) colour[i] = value;
}

__global__ void k_colour_mark(ColourArgs A, int *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const int c = A.colour[i];
  bool drop = c >= A.kbase;
  for (int k = 0; k < A.nspin[i]; ++k) {
    const int j = A.nbr[(size_t)k * A.ld + i];
    if (A.colour[j] == c && key_less(A, j, i) && conflict(A, i, j)) drop = true;
  }
  out[i] = drop ? -1 : c;
}

// One Jones-Plassmann round. A neighbour coloured during this same round is
// either seen with its final colour or seen uncoloured (then this atom waits
// a round); both give the sequential greedy result, only the round count
// can differ.
// Colour atom i if every conflicting neighbour of earlier key has its
// colour (first free colour among all coloured conflicting neighbours);
// returns false when it has to wait for a later round.
__device__ __forceinline__ bool colour_try(const ColourArgs &A, int i) {
  volatile int *col = A.colour;
  unsigned long long used = 0ull;
  for (int k = 0; k < A.nspin[i]; ++k) {
    const int j = A.nbr[(size_t)k * A.ld + i];
    if (!conflict(A, i, j)) continue;
    const int cj = col[j];
    if (cj >= 0) {
      used |= 1ull << (cj & 63);
    } else if (key_less(A, j, i)) {
      return false;
    }
  }
  col[i] = __ffsll((long long)~used) - 1;
  return true;
}

// Key-priority first-fit colouring driven by readiness: every uncoloured
// atom counts its uncoloured conflicting neighbours of earlier key; atoms at
// zero are ready. Ready atoms never conflict with each other (of two
// conflicting uncoloured atoms the later one still waits for the earlier),
// so a round colours all of them at once; each then releases its later-key
// uncoloured neighbours, and an atom whose count reaches zero joins the next
// ready list. Every atom is coloured once all its earlier-key neighbours
// are, from the colours around it then -- the sequential greedy's choice --
// and each round touches only the atoms that became ready.
__global__ void k_colour_indeg(ColourArgs A, int *indeg, unsigned long long *cmask,
                               unsigned long long *emask, int *list, int *count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n || A.colour[i] >= 0) return;
  // spin-segment slots that are edges of the colouring graph, and those of
  // them whose atom comes earlier in key order (the segment has < 64 slots)
  unsigned long long cm = 0ull, em = 0ull;
  int c = 0;
  const int ns = A.nspin[i] < 64 ? A.nspin[i] : 64;
  for (int k = 0; k < ns; ++k) {
    const int j = A.nbr[(size_t)k * A.ld + i];
    if (!conflict(A, i, j)) continue;
    cm |= 1ull << k;
    if (key_less(A, j, i)) {
      em |= 1ull << k;
      if (A.colour[j] < 0) ++c;
    }
  }
  cmask[i] = cm;
  emask[i] = em;
  indeg[i] = c;
  if (c == 0) list[atomicAdd(count, 1)] = i;
}

// One round: colour the ready atoms, release their later neighbours. The
// counter of the round after next is cleared here (nothing else touches it
// in this round). The slot loads of a chunk go out together, then the
// colour loads: each ready atom costs a few memory round trips.
constexpr int kColourChunk = 16;
// Load of a word another thread of the workgroup may have written in an
// earlier round of the same launch: an agent-scope atomic load, which reads
// the L2 (the device-wide rounds get the same guarantee from their launch
// boundaries).
__device__ __forceinline__ int load_l2(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One ready atom of a round: first-fit colour against its coloured
// conflicting neighbours, then the later-key uncoloured neighbours lose one
// wait each, and the one whose count reaches zero joins the next list.
template <bool L2>
__device__ __forceinline__ void colour_one(const ColourArgs &A, int i, int *indeg,
                                           const unsigned long long *cmask,
                                           const unsigned long long *emask, int *out,
                                           int *out_count) {
  const unsigned long long cm = cmask[i], em = emask[i];
  const int ns = A.nspin[i] < 64 ? A.nspin[i] : 64;
  unsigned long long used = 0ull;
  for (int k0 = 0; k0 < ns; k0 += kColourChunk) {
    int jj[kColourChunk];
#pragma unroll
    for (int q = 0; q < kColourChunk; ++q) {
      const int k = k0 + q;
      jj[q] = (k < ns && ((cm >> k) & 1ull)) ? A.nbr[(size_t)k * A.ld + i] : -1;
    }
#pragma unroll
    for (int q = 0; q < kColourChunk; ++q) {
      const int cj = jj[q] >= 0 ? (L2 ? load_l2(&A.colour[jj[q]]) : A.colour[jj[q]]) : -1;
      if (cj >= 0) used |= 1ull << (cj & 63);
    }
  }
  A.colour[i] = __ffsll((long long)~used) - 1;
  const unsigned long long later = cm & ~em;
  for (int k0 = 0; k0 < ns; k0 += kColourChunk) {
    int jj[kColourChunk];
#pragma unroll
    for (int q = 0; q < kColourChunk; ++q) {
      const int k = k0 + q;
      jj[q] = (k < ns && ((later >> k) & 1ull)) ? A.nbr[(size_t)k * A.ld + i] : -1;
    }
#pragma unroll
    for (int q = 0; q < kColourChunk; ++q) {
      const int j = jj[q];
      if (j >= 0 && (L2 ? load_l2(&A.colour[j]) : A.colour[j]) < 0 && atomicSub(&indeg[j], 1) == 1)
        out[atomicAdd(out_count, 1)] = j;
    }
  }
}

__global__ void k_colour_round(ColourArgs A, int *indeg, const unsigned long long *cmask,
                               const unsigned long long *emask, const int *in,
                               const int *in_count, int *out, int *out_count, int *clear_next) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *clear_next = 0;
  const int m = *in_count;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x)
    colour_one<false>(A, in[t], indeg, cmask, emask, out, out_count);
}

// Rounds r0, r0 + 1, ... in one workgroup, with a workgroup barrier between
// rounds, for as long as the ready list is non-empty and at most nmax long
// and at most max_rounds rounds: most rounds of a colouring, and all of a
// repair, hold a few dozen atoms, which one workgroup serves in a few
// microseconds while a launch per round costs its dispatch. Lists and
// counters follow the rotation of k_colour_round (round r reads list r % 2
// with count r % 3); done[0] gets the number of rounds run.
constexpr int kFinishBlock = 1024;
__global__ __launch_bounds__(kFinishBlock) void k_colour_finish(
    ColourArgs A, int *indeg, const unsigned long long *cmask, const unsigned long long *emask,
    int *list0, int *list1, int *count, int r0, int max_rounds, int nmax, int *done) {
  __shared__ int m_s;
  int r = r0;
  for (; r < r0 + max_rounds; ++r) {
    if (threadIdx.x == 0) {
      m_s = load_l2(&count[r % 3]);
      atomicExch(&count[(r + 2) % 3], 0);
    }
    __syncthreads();
    const int m = m_s;
    if (m == 0 || m > nmax) break;
    const int *in = (r & 1) ? list1 : list0;
    int *out = (r & 1) ? list0 : list1;
    for (int t = threadIdx.x; t < m; t += kFinishBlock)
      colour_one<true>(A, load_l2(&in[t]), indeg, cmask, emask, out, &count[(r + 1) % 3]);
    __syncthreads();
  }
  if (threadIdx.x == 0) done[0] = r - r0;
}

__global__ void k_colour_stats(ColourArgs A, int *maxc, int *err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const int c = A.colour[i];
  atomicMax(maxc, c);
  for (int k = 0; k < A.nspin[i]; ++k) {
    const int j = A.nbr[(size_t)k * A.ld + i];
    if (A.colour[j] == c && conflict(A, i, j)) atomicOr(err, kErrColour);
  }
  if (c < 0) atomicOr(err, kErrColour);
}

__global__ void k_watch_mask(int n, int ld, const int *nbr, const int *nspin, const int *colour,
                             unsigned long long *wmask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = colour[i];
  const int ns = nspin[i] < 64 ? nspin[i] : 64;
  unsigned long long m = 0ull;
  for (int k = 0; k < ns; ++k)
    if (colour[nbr[(size_t)k * ld + i]] == c) m |= 1ull << k;
  wmask[i] = m;
}

// ky, kz are wrapped positions in [0, L): the row is the nearest multiple
// of the spacing, the last half spacing wrapping to row 0.
__global__ void k_row_key(int n, const int *colour, const double *ky, const double *kz,
                          RowGrid R, int *key, int *count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int y = (int)floor(ky[i] * R.inv_y + 0.5), z = (int)floor(kz[i] * R.inv_z + 0.5);
  y = y >= R.ny ? y - R.ny : (y < 0 ? 0 : y);
  z = z >= R.nz ? z - R.nz : (z < 0 ? 0 : z);
  const int k = (colour[i] * R.nz + z) * R.ny + y;
  key[i] = k;
  atomicAdd(&count[k], 1);
}

__global__ void k_inverse(int n, const int *perm, int *inv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) inv[perm[i]] = i;
}

__global__ void k_permute_atoms(PermuteArgs A) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const int o = A.perm[i];
  for (int k = 0; k < A.nd; ++k) A.dst_d[k][i] = A.src_d[k][o];
  for (int k = 0; k < A.nf; ++k) A.dst_f[k][i] = A.src_f[k][o];
  for (int k = 0; k < A.ni; ++k) A.dst_i[k][i] = A.src_i[k][o];
}

__global__ void k_permute_nbr(int n, int ld, const int *perm, const int *inv, const int *nbr_old,
                              const int *nspin_old, const int *nall_old, int *nbr_new,
                              int *nspin_new, int *nall_new) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int o = perm[i];
  const int na = nall_old[o];
  for (int k = 0; k < na; ++k) nbr_new[(size_t)k * ld + i] = inv[nbr_old[(size_t)k * ld + o]];
  nspin_new[i] = nspin_old[o];
  nall_new[i] = na;
}

__global__ void k_csr_to_ell(CsrArgs A) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const int u = A.id[i];
  const int a = A.off[u], b = A.off[u + 1];
  const double rix = A.rx[i], riy = A.ry[i], riz = A.rz[i];
  int ns = 0, nt = 0;
  for (int pass = 0; pass < 2; ++pass)
    for (int p = a; p < b; ++p) {
      const int j = A.uinv[A.idx[p]];
      const double dx = min_image(rix - A.rx[j], A.L[0], A.invL[0]);
      const double dy = min_image(riy - A.ry[j], A.L[1], A.invL[1]);
      const double dz = min_image(riz - A.rz[j], A.L[2], A.invL[2]);
      const bool sp = dx * dx + dy * dy + dz * dz < A.rs2;
      if (sp != (pass == 0)) continue;
      if (nt < A.max_nbr) A.nbr[(size_t)nt * A.ld + i] = j;
      ++nt;
      if (pass == 0) ++ns;
    }
  if (nt > A.max_nbr) atomicOr(A.err, kErrNbrOverflow);
  A.nspin[i] = min(ns, A.max_nbr);
  A.nall[i] = min(nt, A.max_nbr);
  A.bx[i] = rix;
  A.by[i] = riy;
  A.bz[i] = riz;
}

__global__ void k_user_inverse(int n, const int *id, int *uinv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) uinv[id[i]] = i;
}

__global__ void k_load_vec(int n, const int *id, const double *aos, double *x, double *y,
                           double *z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t u = (size_t)id[i] * 3;
  x[i] = aos[u];
  y[i] = aos[u + 1];
  z[i] = aos[u + 2];
}

__global__ void k_load_vec_f(int n, const int *id, const double *aos, float *x, float *y,
                             float *z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t u = (size_t)id[i] * 3;
  x[i] = (float)aos[u];
  y[i] = (float)aos[u + 1];
  z[i] = (float)aos[u + 2];
}

__global__ void k_store_vec(int n, const int *id, const double *x, const double *y,
                            const double *z, double *aos) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t u = (size_t)id[i] * 3;
  aos[u] = x[i];
  aos[u + 1] = y[i];
  aos[u + 2] = z[i];
}

__global__ void k_store_vec_f(int n, const int *id, const float *x, const float *y,
                              const float *z, double *aos) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t u = (size_t)id[i] * 3;
  aos[u] = x[i];
  aos[u + 1] = y[i];
  aos[u + 2] = z[i];
}

__global__ void k_load_scalar(int n, const int *id, const double *src, double *dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[id[i]];
}

__global__ void k_copy_d(int n, const double *src, double *dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_iota(int n, int *id) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) id[i] = i;
}

__global__ void k_zero_i(int n, int *p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
void launch_cell_assign(int n, const double *rx, const double *ry, const double *rz,
                        const CellGrid &G, int *cell, int *count, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_cell_assign, dim3(nblocks(n)), dim3(kBlock), 0, st, n, rx, ry, rz, G, cell, count);
}
void launch_scan(const int *in, int *out, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, in, out, n);
}
void launch_bucket_scatter(int n, const int *key, const int *start, int *fill, int *out,
                           hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_bucket_scatter, dim3(nblocks(n)), dim3(kBlock), 0, st, n, key, start, fill, out);
}
void launch_bucket_sort_x(int nbucket, const int *start, int *items, const double *x,
                          hipStream_t st) {
  if (nbucket > 0) hipLaunchKernelGGL(k_bucket_sort_x, dim3(nblocks(nbucket)), dim3(kBlock), 0, st, nbucket, start, items, x);
}
void launch_cell_positions(int n, const int *catoms, const double *rx, const double *ry,
                           const double *rz, double *cx, double *cy, double *cz, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_cell_positions, dim3(nblocks(n)), dim3(kBlock), 0, st, n, catoms, rx, ry, rz, cx, cy, cz);
}
void launch_bucket_sort(int nbucket, const int *start, int *items, hipStream_t st) {
  if (nbucket > 0) hipLaunchKernelGGL(k_bucket_sort, dim3(nblocks(nbucket)), dim3(kBlock), 0, st, nbucket, start, items);
}
void launch_nbr_build(const NbrBuildArgs &A, hipStream_t st) {
  if (A.n <= 0) return;
  if (A.n >= kNbrManyAtoms) {
    hipLaunchKernelGGL(k_nbr_build<1>, dim3((unsigned)((A.n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, A);
  } else {
    const long threads = (long)A.n * 16;
    hipLaunchKernelGGL(k_nbr_build<16>, dim3((unsigned)((threads + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, A);
  }
  if (A.row_q > 0.0)
    hipLaunchKernelGGL(k_row_order, dim3((unsigned)((A.n + kOrderBlock - 1) / kOrderBlock)),
                       dim3(kOrderBlock), 0, st, A, 1.0 / A.row_q);
}
void launch_keys(int n, const double *rx, const double *ry, const double *rz, const double L[3],
                 double *kx, double *ky, double *kz, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_keys, dim3(nblocks(n)), dim3(kBlock), 0, st, n, rx, ry, rz, L[0], L[1], L[2], kx, ky, kz);
}
void launch_colour_fill(int n, int *colour, int value, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_colour_fill, dim3(nblocks(n)), dim3(kBlock), 0, st, n, colour, value);
}
void launch_colour_mark(const ColourArgs &A, int *colour_out, hipStream_t st) {
  if (A.n > 0) hipLaunchKernelGGL(k_colour_mark, dim3(nblocks(A.n)), dim3(kBlock), 0, st, A, colour_out);
}
void launch_colour_indeg(const ColourArgs &A, int *indeg, unsigned long long *cmask,
                         unsigned long long *emask, int *list, int *count, hipStream_t st) {
  if (A.n > 0)
    hipLaunchKernelGGL(k_colour_indeg, dim3(nblocks(A.n)), dim3(kBlock), 0, st, A, indeg, cmask,
                       emask, list, count);
}
void launch_colour_round(const ColourArgs &A, int *indeg, const unsigned long long *cmask,
                         const unsigned long long *emask, const int *in, const int *in_count,
                         int *out, int *out_count, int *clear_next, hipStream_t st) {
  hipLaunchKernelGGL(k_colour_round, dim3(64), dim3(kBlock), 0, st, A, indeg, cmask, emask, in,
                     in_count, out, out_count, clear_next);
}
// Words the host reads after a rebuild's launches, written into pinned
// host memory (one synchronisation for all): the colouring counters and
// rounds, the largest colour and the colouring's own error word, the
// sticky error word and the largest rows of the list build.
__global__ void k_rebuild_report(const int *jp, const int *err, const int *seen, int *out) {
  if (threadIdx.x == 0) {
    for (int k = 0; k < 6; ++k) out[k] = jp[k];
    out[6] = *err;
    out[7] = seen[0];
    out[8] = seen[1];
    __threadfence_system();
  }
}

// Class offsets out[c] = bstart[c * nrow], c = 0..K, into pinned memory.
__global__ void k_class_offsets(const int *bstart, int nrow, int K, int *out) {
  const int c = threadIdx.x;
  if (c <= K) out[c] = bstart[(size_t)c * nrow];
  __threadfence_system();
}

void launch_rebuild_report(const int *jp, const int *err, const int *seen, int *out,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_rebuild_report, dim3(1), dim3(64), 0, st, jp, err, seen, out);
}
void launch_class_offsets(const int *bstart, int nrow, int K, int *out, hipStream_t st) {
  hipLaunchKernelGGL(k_class_offsets, dim3(1), dim3(64), 0, st, bstart, nrow, K, out);
}
void launch_colour_finish(const ColourArgs &A, int *indeg, const unsigned long long *cmask,
                          const unsigned long long *emask, int *list0, int *list1, int *count,
                          int r0, int max_rounds, int nmax, int *done, hipStream_t st) {
  hipLaunchKernelGGL(k_colour_finish, dim3(1), dim3(kFinishBlock), 0, st, A, indeg, cmask, emask,
                     list0, list1, count, r0, max_rounds, nmax, done);
}
void launch_colour_stats(const ColourArgs &A, int *maxc, int *err, hipStream_t st) {
  if (A.n > 0) hipLaunchKernelGGL(k_colour_stats, dim3(nblocks(A.n)), dim3(kBlock), 0, st, A, maxc, err);
}
void launch_watch_mask(int n, int ld, const int *nbr, const int *nspin, const int *colour,
                       unsigned long long *wmask, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_watch_mask, dim3(nblocks(n)), dim3(kBlock), 0, st, n, ld, nbr, nspin, colour, wmask);
}
void launch_row_key(int n, const int *colour, const double *ky, const double *kz,
                    const RowGrid &R, int *key, int *count, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_row_key, dim3(nblocks(n)), dim3(kBlock), 0, st, n, colour, ky, kz, R, key, count);
}
void launch_inverse(int n, const int *perm, int *inv, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_inverse, dim3(nblocks(n)), dim3(kBlock), 0, st, n, perm, inv);
}
void launch_permute_atoms(const PermuteArgs &A, hipStream_t st) {
  if (A.n > 0) hipLaunchKernelGGL(k_permute_atoms, dim3(nblocks(A.n)), dim3(kBlock), 0, st, A);
}
void launch_permute_nbr(int n, int ld, const int *perm, const int *inv, const int *nbr_old,
                        const int *nspin_old, const int *nall_old, int *nbr_new, int *nspin_new,
                        int *nall_new, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_permute_nbr, dim3(nblocks(n)), dim3(kBlock), 0, st, n, ld, perm, inv, nbr_old, nspin_old, nall_old, nbr_new, nspin_new, nall_new);
}
void launch_csr_to_ell(const CsrArgs &A, hipStream_t st) {
  if (A.n > 0) hipLaunchKernelGGL(k_csr_to_ell, dim3(nblocks(A.n)), dim3(kBlock), 0, st, A);
}
void launch_user_inverse(int n, const int *id, int *uinv, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_user_inverse, dim3(nblocks(n)), dim3(kBlock), 0, st, n, id, uinv);
}
void launch_load_vec(int n, const int *id, const double *aos, double *x, double *y, double *z,
                     hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_load_vec, dim3(nblocks(n)), dim3(kBlock), 0, st, n, id, aos, x, y, z);
}
void launch_load_vec_f(int n, const int *id, const double *aos, float *x, float *y, float *z,
                       hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_load_vec_f, dim3(nblocks(n)), dim3(kBlock), 0, st, n, id, aos, x, y, z);
}
void launch_store_vec(int n, const int *id, const double *x, const double *y, const double *z,
                      double *aos, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_store_vec, dim3(nblocks(n)), dim3(kBlock), 0, st, n, id, x, y, z, aos);
}
void launch_store_vec_f(int n, const int *id, const float *x, const float *y, const float *z,
                        double *aos, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_store_vec_f, dim3(nblocks(n)), dim3(kBlock), 0, st, n, id, x, y, z, aos);
}
void launch_load_scalar(int n, const int *id, const double *src, double *dst, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_load_scalar, dim3(nblocks(n)), dim3(kBlock), 0, st, n, id, src, dst);
}
void launch_copy_d(int n, const double *src, double *dst, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_copy_d, dim3(nblocks(n)), dim3(kBlock), 0, st, n, src, dst);
}
void launch_iota(int n, int *id, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_iota, dim3(nblocks(n)), dim3(kBlock), 0, st, n, id);
}
void launch_zero_i(int n, int *p, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_zero_i, dim3(nblocks(n)), dim3(kBlock), 0, st, n, p);
}

}  // namespace sl
