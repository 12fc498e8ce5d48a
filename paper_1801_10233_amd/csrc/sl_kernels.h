// sl_kernels.h -- host-side launchers of the gfx950 kernels (internal).
#pragma once

#include "sl_device.h"

namespace sl {

// --- per-step kernels (sl_dyn.hip) ---
// `lanes` (1, 2, 4 or 8) consecutive lanes cooperate on one atom.
// With S2 (the same system at its other position buffer) the launch is the
// dual update: A.nrep == 2, the first update's field at S, the second's at S2.
template <typename real>
void launch_spin_phase(const SysView<real> &S, const PotConst &P, const SpinPhaseArgs &A,
                       int lanes, hipStream_t st, const SysView<real> *S2 = nullptr);
template <typename real>
void launch_spin_tail(const SysView<real> &S, const PotConst &P, const TailArgs &T, int lanes,
                      hipStream_t st);
template <typename real>
void launch_force(const SysView<real> &S, const PotConst &P, const ForceArgs &A, int lanes,
                  hipStream_t st);
// Split force of the analytic forms (1 or 2 lanes per atom): the pair pass
// stores the spin-independent force (and, with energy, the pair energy) of
// every atom in A.fp; the spin pass adds the spin-dependent terms of the
// spin segment to it and does what the fused launch does after the gather.
template <typename real>
void launch_pair(const SysView<real> &S, const PotConst &P, const ForceArgs &A, int lanes,
                 bool energy, hipStream_t st);
template <typename real>
void launch_force_spin(const SysView<real> &S, const PotConst &P, const ForceArgs &A, int lanes,
                       hipStream_t st);
int force_blocks(int n, int lanes);
// Joins the per-block rebuild predictor terms (pred[nb][3]) of a force launch
// into the pinned host slot host_out, with the error word and the marker.
void launch_pred_reduce(const double *pred, int nb, int *err, double *host_out, hipStream_t st);
template <typename real>
void launch_batch_run(RepDesc<real> *D, int R, int lanes, int variant, hipStream_t st);
// Embedded-atom first pass (F'(rho), F(rho) of every atom) at the positions
// of a view, before the force launch that reads them.
template <typename real>
void launch_eam_density(const SysView<real> &S, const PotConst &P, hipStream_t st);
// Exchange-coefficient cache: J(r_ij) per spin-segment entry (ELL layout);
// tiles (or null): atom range of each 256-thread block.
template <typename real>
void launch_jcache(const SysView<real> &S, const PotConst &P, real *out, double rs2,
                   const int2 *tiles, int ntiles, hipStream_t st);
// Phase-batched mode: one colour phase of every replica (max_class = the
// largest class of any replica) and one force pass of every replica (max_n =
// the largest replica; mode kModeNext at the call start, kModeFinal with or
// without kModeNext after a step). soc selects the spin variant with the
// spin-orbit pair terms (needed when any replica has them); variant is the
// force variant (4: spin-orbit terms, 8: embedded-atom terms, 12: both), the
// embedded-atom densities being computed first.
template <typename real>
void launch_batch_spin(const RepDesc<real> *D, int R, int max_class, const BatchPhase &bp,
                       int lanes, bool soc, hipStream_t st);
template <typename real>
void launch_batch_force(const RepDesc<real> *D, int R, int max_n, int mode, const BatchPhase &bp,
                        int lanes, int variant, hipStream_t st);
void launch_reduce8(const double *partial, int nb, double *out, hipStream_t st);

// --- sectored ordering (sl_sect.hip) ---
void launch_sect_keys(const SectKeyArgs &A, hipStream_t st);
int sect_sort(const SectKeyArgs &A, int nbins, unsigned long long *keys_out, int *vals_out,
              int *off, void **tmp, size_t *tmp_bytes, hipStream_t st);
template <typename real>
void launch_sect_phase(const SysView<real> &S, const PotConst &P, const SectPhaseArgs &A,
                       hipStream_t st);

// --- rebuild kernels (sl_nbr.hip) ---
struct CellGrid {
  int nc[3];
  double L[3];
};

// Cell of every atom from its wrapped position; histogram of cell sizes.
void launch_cell_assign(int n, const double *rx, const double *ry, const double *rz,
                        const CellGrid &G, int *cell, int *count, hipStream_t st);
// Exclusive scan of n ints into out[0..n] (out[n] = total), one block.
void launch_scan(const int *in, int *out, int n, hipStream_t st);
// Counting-sort scatter by key, then each bucket sorted ascending so the
// result does not depend on the order the atomics were served in.
void launch_bucket_scatter(int n, const int *key, const int *start, int *fill, int *out,
                           hipStream_t st);
void launch_bucket_sort(int nbucket, const int *start, int *items, hipStream_t st);
// Each bucket's items ascending by (x[item], item).
void launch_bucket_sort_x(int nbucket, const int *start, int *items, const double *x,
                          hipStream_t st);

struct NbrBuildArgs {
  int n, ld, max_nbr, max_spin;
  double rs2, rl2;
  CellGrid G;
  const double *rx, *ry, *rz;
  const double *cx, *cy, *cz;  // positions in cell order (cx[p] = rx[catoms[p]])
  const int *cell, *cstart, *catoms;
  int *nbr, *nspin, *nall;
  double *bx, *by, *bz;   // reference positions written at build time
  int *err;
  int *seen;              // [2]: largest spin segment and row
  double row_q;           // > 0: sort each row segment by the displacement
                          // rounded to this grid step (A); 0: cell-loop order
};
void launch_nbr_build(const NbrBuildArgs &A, hipStream_t st);
// Positions in cell order, for the neighbour build.
void launch_cell_positions(int n, const int *catoms, const double *rx, const double *ry,
                           const double *rz, double *cx, double *cy, double *cz, hipStream_t st);

// Lexicographic colouring keys (z, y, x wrapped) of the current positions.
void launch_keys(int n, const double *rx, const double *ry, const double *rz, const double L[3],
                 double *kx, double *ky, double *kz, hipStream_t st);

struct ColourArgs {
  int n, ld;
  const int *nbr, *nspin, *id;
  const double *kx, *ky, *kz;
  int *colour;
  int kbase;  // colours >= kbase are dropped by a repair
  // spin-segment entries conflict (may not share a colour) when closer than
  // sqrt(cr2) at these positions
  const double *rx, *ry, *rz;
  double L[3], invL[3];
  double cr2;
};
void launch_colour_fill(int n, int *colour, int value, hipStream_t st);
// Uncolour every atom that shares its colour with an earlier-key neighbour,
// and every atom whose colour lies outside the base palette.
void launch_colour_mark(const ColourArgs &A, int *colour_out, hipStream_t st);
// Key-priority first-fit colouring by readiness: counts of uncoloured
// earlier-key conflicting neighbours and the first ready list, then one
// round (colour the ready list; newly ready atoms go to *out; *clear_next is
// zeroed for the round after).
// The conflict and earlier-key slot masks (cmask, emask) are computed once
// by the first pass and read by every round.
void launch_colour_indeg(const ColourArgs &A, int *indeg, unsigned long long *cmask,
                         unsigned long long *emask, int *list, int *count, hipStream_t st);
void launch_colour_round(const ColourArgs &A, int *indeg, const unsigned long long *cmask,
                         const unsigned long long *emask, const int *in, const int *in_count,
                         int *out, int *out_count, int *clear_next, hipStream_t st);
// Rebuild read-back into pinned host memory: out[0..5] = jp[0..5] (ready
// counts, rounds, largest colour, colouring error word), out[6] = *err,
// out[7..8] = seen[0..1]; and the class offsets out[c] = bstart[c * nrow]
// for c = 0..K (K < 64).
void launch_rebuild_report(const int *jp, const int *err, const int *seen, int *out,
                           hipStream_t st);
void launch_class_offsets(const int *bstart, int nrow, int K, int *out, hipStream_t st);
// Rounds from r0 in one workgroup while the ready list is non-empty and at
// most nmax long (at most max_rounds); done[0] = rounds run.
void launch_colour_finish(const ColourArgs &A, int *indeg, const unsigned long long *cmask,
                          const unsigned long long *emask, int *list0, int *list1, int *count,
                          int r0, int max_rounds, int nmax, int *done, hipStream_t st);
void launch_colour_stats(const ColourArgs &A, int *maxc, int *err, hipStream_t st);

// Per atom, the spin-segment slots (< 64) whose entry has the atom's colour.
void launch_watch_mask(int n, int ld, const int *nbr, const int *nspin, const int *colour,
                       unsigned long long *wmask, hipStream_t st);

// Permutation key of the atom order: colour class, then the rows of a fine
// (y, z) grid, z slowest (one bucket per class and row); inside a row the
// atoms go by x (launch_bucket_sort_x). Row y of the grid collects the
// positions within half a spacing of y * Ly / ny, so that lattice planes at
// multiples of the spacing keep their row through thermal motion.
struct RowGrid {
  int ny, nz;
  double inv_y, inv_z;  // ny / Ly, nz / Lz
};
void launch_row_key(int n, const int *colour, const double *ky, const double *kz,
                    const RowGrid &R, int *key, int *count, hipStream_t st);
void launch_inverse(int n, const int *perm, int *inv, hipStream_t st);

struct PermuteArgs {
  int n;
  const int *perm;              // new -> old
  const double *src_d[16];
  double *dst_d[16];
  int nd;
  const float *src_f[3];
  float *dst_f[3];
  int nf;
  const int *src_i[4];
  int *dst_i[4];
  int ni;
};
void launch_permute_atoms(const PermuteArgs &A, hipStream_t st);
void launch_permute_nbr(int n, int ld, const int *perm, const int *inv, const int *nbr_old,
                        const int *nspin_old, const int *nall_old, int *nbr_new, int *nspin_new,
                        int *nall_new, hipStream_t st);

// User CSR (user ids) -> internal ELL, spin-radius entries first.
struct CsrArgs {
  int n, ld, max_nbr;
  const int *off, *idx;      // user CSR
  const int *id, *uinv;      // internal -> user, user -> internal
  const double *rx, *ry, *rz;
  double L[3], invL[3];
  double rs2;
  int *nbr, *nspin, *nall;
  double *bx, *by, *bz;
  int *err;
};
void launch_csr_to_ell(const CsrArgs &A, hipStream_t st);
void launch_user_inverse(int n, const int *id, int *uinv, hipStream_t st);

// State transfer between user AoS double[N][3] and internal SoA.
void launch_load_vec(int n, const int *id, const double *aos, double *x, double *y, double *z,
                     hipStream_t st);
void launch_load_vec_f(int n, const int *id, const double *aos, float *x, float *y, float *z,
                       hipStream_t st);
void launch_store_vec(int n, const int *id, const double *x, const double *y, const double *z,
                      double *aos, hipStream_t st);
void launch_store_vec_f(int n, const int *id, const float *x, const float *y, const float *z,
                        double *aos, hipStream_t st);
void launch_load_scalar(int n, const int *id, const double *src, double *dst, hipStream_t st);
void launch_copy_d(int n, const double *src, double *dst, hipStream_t st);
void launch_iota(int n, int *id, hipStream_t st);
void launch_zero_i(int n, int *p, hipStream_t st);

}  // namespace sl
