// sl_rebuild.hip -- the rebuild pipeline of a system: cell binning, the
// device neighbour-list build with the rows' order, colour classes (a full
// colouring or the repair of the last one) and the permutation of every
// per-atom array into (colour, row, x) order.
#include "sl_host.h"

namespace sl {

int ensure_cells(sl_system *S, int ncell) {
  if (ncell + 1 <= S->cell_cap) return SL_OK;
  dfree(S->ccount); dfree(S->cstart); dfree(S->cfill);
  S->cell_cap = ncell + 1;
  HIPCHK(S, dalloc(&S->ccount, S->cell_cap));
  HIPCHK(S, dalloc(&S->cstart, S->cell_cap + 1));
  HIPCHK(S, dalloc(&S->cfill, S->cell_cap));
  return SL_OK;
}

int ensure_bins(sl_system *S, int nbin) {
  if (nbin + 1 <= S->bin_cap) return SL_OK;
  dfree(S->bcount); dfree(S->bstart); dfree(S->bfill);
  S->bin_cap = nbin + 1;
  HIPCHK(S, dalloc(&S->bcount, S->bin_cap));
  HIPCHK(S, dalloc(&S->bstart, S->bin_cap + 1));
  HIPCHK(S, dalloc(&S->bfill, S->bin_cap));
  return SL_OK;
}

void cell_grid(sl_system *S, CellGrid &G) {
  const double rl = list_radius(S);
  for (int d = 0; d < 3; ++d) {
    int k = rl > 0 ? (int)std::floor(S->L[d] / rl) : 1;
    if (k < 3) k = 1;
    if (k > 1024) k = 1024;
    G.nc[d] = k;
    G.L[d] = S->L[d];
  }
  // at most ~2 cells per atom: larger cells are still valid, only slower
  const long cap = std::max<long>(2L * S->n, 27L);
  while ((long)G.nc[0] * G.nc[1] * G.nc[2] > cap) {
    int d = 0;
    for (int e = 1; e < 3; ++e)
      if (G.nc[e] > G.nc[d]) d = e;
    if (G.nc[d] <= 3) break;
    G.nc[d] = std::max(3, (G.nc[d] * 4) / 5);
  }
  for (int d = 0; d < 3; ++d) S->nc[d] = G.nc[d];
  S->ncell = G.nc[0] * G.nc[1] * G.nc[2];
}

// Cell index of every atom at the current positions and the sorted cell
// member lists (cstart/catoms).
int bin_cells(sl_system *S, CellGrid &G) {
  Atoms &A = S->a[S->cur];
  cell_grid(S, G);
  CHK(ensure_cells(S, S->ncell));
  launch_zero_i(S->ncell, S->ccount, S->st);
  launch_cell_assign(S->n, A.rx[S->pos], A.ry[S->pos], A.rz[S->pos], G, A.cell, S->ccount, S->st);
  launch_scan(S->ccount, S->cstart, S->ncell, S->st);
  launch_zero_i(S->ncell, S->cfill, S->st);
  launch_bucket_scatter(S->n, A.cell, S->cstart, S->cfill, S->catoms, S->st);
  launch_bucket_sort(S->ncell, S->cstart, S->catoms, S->st);
  return SL_OK;
}

ColourArgs colour_args(sl_system *S) {
  Atoms &A = S->a[S->cur];
  ColourArgs C;
  C.n = S->n;
  C.ld = S->ld;
  C.nbr = A.nbr;
  C.nspin = A.nspin;
  C.id = A.id;
  C.kx = S->kx;
  C.ky = S->ky;
  C.kz = S->kz;
  C.colour = A.colour;
  C.kbase = S->Kbase;
  C.rx = A.rx[S->pos];
  C.ry = A.ry[S->pos];
  C.rz = A.rz[S->pos];
  for (int d = 0; d < 3; ++d) {
    C.L[d] = S->L[d];
    C.invL[d] = S->invL[d];
  }
  const double rc = colour_radius(S);
  C.cr2 = S->user_list ? 1e300 : rc * rc;
  return C;
}

// Colouring rounds until every atom has a colour, then its statistics.
// Round r reads ready list r % 2 with count r % 3 and writes list (r + 1) % 2
// with count (r + 1) % 3. Rounds with at most kFinishMax ready atoms run in
// one workgroup (k_colour_finish, up to kFinishRounds per launch); longer
// lists take batches of kJpBatch device-wide rounds. After each workgroup
// launch the statistics (largest colour, conflicts, own error word) are
// computed as if the colouring were complete and read back with the
// counters, the sticky error word and the list build's largest rows in one
// host synchronisation; a repair usually needs just that one. *mc gets the
// largest colour.
constexpr int kFinishMax = 4096, kFinishRounds = 4096;
int jp_rounds(sl_system *S, const ColourArgs &C, int *mc) {
  HIPCHK(S, hipMemsetAsync(S->jpcnt, 0, 4 * sizeof(int), S->st));
  launch_colour_indeg(C, S->ctmp, S->jpmask[0], S->jpmask[1], S->jplist[0], &S->jpcnt[0], S->st);
  int r = 0;
  for (;;) {
    launch_colour_finish(C, S->ctmp, S->jpmask[0], S->jpmask[1], S->jplist[0], S->jplist[1],
                         S->jpcnt, r, kFinishRounds, kFinishMax, &S->jpcnt[3], S->st);
    HIPCHK(S, hipMemsetAsync(&S->jpcnt[4], 0xff, sizeof(int), S->st));
    HIPCHK(S, hipMemsetAsync(&S->jpcnt[5], 0, sizeof(int), S->st));
    launch_colour_stats(C, &S->jpcnt[4], &S->jpcnt[5], S->st);
    launch_rebuild_report(S->jpcnt, S->err, S->seen, S->pin_dev, S->st);
    HIPCHK(S, hipStreamSynchronize(S->st));
    const int *h = S->pin;
    r += h[3];
    const int rem = h[r % 3];
    if (rem == 0) {
      *mc = h[4];
      S->sticky |= h[5] | h[6];
      S->seen_spin = h[7];
      S->seen_all = h[8];
      break;
    }
    if (r > S->n + 2 * kJpBatch) return fail(S, SL_E_COLOR, "colouring rounds made no progress");
    if (rem > kFinishMax)
      for (int b = 0; b < kJpBatch; ++b, ++r)
        launch_colour_round(C, S->ctmp, S->jpmask[0], S->jpmask[1], S->jplist[r & 1],
                            &S->jpcnt[r % 3], S->jplist[(r + 1) & 1], &S->jpcnt[(r + 1) % 3],
                            &S->jpcnt[(r + 2) % 3], S->st);
  }
  S->jp_rounds = r;
  return SL_OK;
}

// Unordered pairs of the current list for the learned-potential table.
int mlp_pairs(sl_system *S) {
  Atoms &A = S->a[S->cur];
  const int n = S->n;
  launch_mlp_pair_count(n, S->ld, A.nbr, A.nall, S->mcnt, S->st);
  launch_scan(S->mcnt, S->mstart, n, S->st);
  int tot = 0;
  HIPCHK(S, hipMemcpyAsync(&tot, S->mstart + n, sizeof(int), hipMemcpyDeviceToHost, S->st));
  HIPCHK(S, hipStreamSynchronize(S->st));
  if (tot > S->mpair_cap) {
    dfree(S->mpairs);
    dfree(S->mirror);
    S->mpair_cap = tot + tot / 4 + 64;
    HIPCHK(S, dalloc(&S->mpairs, S->mpair_cap));
    HIPCHK(S, dalloc(&S->mirror, S->mpair_cap));
  }
  launch_mlp_pair_fill(n, S->ld, A.nbr, A.nall, S->mstart, S->mpairs, S->mirror, S->err, S->st);
  S->npair = tot;
  S->tab_ok[0] = S->tab_ok[1] = false;
  return SL_OK;
}

// Rows of the atom order: spaced by the list rows' order grid when there is
// one (a lattice spacing), else by the mean interatomic distance; at most
// about one row per atom.
RowGrid row_grid(const sl_system *S) {
  const double V = S->L[0] * S->L[1] * S->L[2];
  const double h = S->row_q > 0.0 ? S->row_q : std::cbrt(V / std::max(1, S->n));
  int ny = std::max(1, std::min(4096, (int)std::lround(S->L[1] / h)));
  int nz = std::max(1, std::min(4096, (int)std::lround(S->L[2] / h)));
  while ((long)ny * nz > std::max(1, S->n) && (ny > 1 || nz > 1)) {
    ny = std::max(1, (ny * 4) / 5);
    nz = std::max(1, (nz * 4) / 5);
  }
  RowGrid R;
  R.ny = ny;
  R.nz = nz;
  R.inv_y = ny / S->L[1];
  R.inv_z = nz / S->L[2];
  return R;
}

// Colour classes (repairing the previous colouring when there is one) and
// permutation of all per-atom arrays into (colour, row, x) order.
int colour_and_permute(sl_system *S, bool repair) {
  ProfScope ps(S, 2, 0.0);
  const int n = S->n;
  CellGrid G;
  {
    Atoms &A = S->a[S->cur];
    cell_grid(S, G);
    CHK(ensure_cells(S, S->ncell));
    launch_zero_i(S->ncell, S->ccount, S->st);
    launch_cell_assign(n, A.rx[S->pos], A.ry[S->pos], A.rz[S->pos], G, A.cell, S->ccount, S->st);
    launch_keys(n, A.rx[S->pos], A.ry[S->pos], A.rz[S->pos], S->L, S->kx, S->ky, S->kz, S->st);
  }
  ColourArgs C = colour_args(S);
  // the palette of a full colouring (or of a colouring the caller set) is
  // the base one; a repair drops atoms outside it so they can move back
  bool set_base = !(repair && S->have_colour);
  if (!S->have_colour) {
    launch_colour_fill(n, C.colour, -1, S->st);
  } else if (repair) {
    launch_colour_mark(C, S->ctmp, S->st);
    HIPCHK(S, hipMemcpyAsync(C.colour, S->ctmp, sizeof(int) * n, hipMemcpyDeviceToDevice, S->st));
  }
  int mc = -1;
  CHK(jp_rounds(S, C, &mc));
  CHK(sticky_code(S));
  if (mc + 1 > 32) {
    launch_colour_fill(n, C.colour, -1, S->st);  // too many colours: start over
    CHK(jp_rounds(S, C, &mc));
    CHK(sticky_code(S));
    set_base = true;
  }
  S->K = n > 0 ? mc + 1 : 0;
  if (set_base) S->Kbase = S->K;
  S->have_colour = true;

  // permutation: counting sort by (colour, row of the fine grid), each row
  // by x. With the rows one lattice spacing apart, consecutive atoms of a
  // class run along a lattice row, and so do their neighbours at one list
  // slot (rows ordered by displacement): a wavefront's gather of one slot
  // reads a few runs of consecutive atoms instead of one or two atoms from
  // each of many cells.
  const RowGrid R = row_grid(S);
  const int nrow = R.ny * R.nz;
  const int nbin = S->K * nrow;
  CHK(ensure_bins(S, nbin));
  Atoms &A = S->a[S->cur];
  Atoms &B = S->a[1 - S->cur];
  launch_zero_i(nbin, S->bcount, S->st);
  launch_row_key(n, A.colour, S->ky, S->kz, R, S->skey, S->bcount, S->st);
  launch_scan(S->bcount, S->bstart, nbin, S->st);
  launch_zero_i(nbin, S->bfill, S->st);
  launch_bucket_scatter(n, S->skey, S->bstart, S->bfill, S->perm, S->st);
  launch_bucket_sort_x(nbin, S->bstart, S->perm, S->kx, S->st);
  launch_inverse(n, S->perm, S->inv, S->st);
  PermuteArgs P;
  std::memset(&P, 0, sizeof(P));
  P.n = n;
  P.perm = S->perm;
  int k = 0;
  for (int b = 0; b < 2; ++b) {
    P.src_d[k] = A.rx[b]; P.dst_d[k++] = B.rx[b];
    P.src_d[k] = A.ry[b]; P.dst_d[k++] = B.ry[b];
    P.src_d[k] = A.rz[b]; P.dst_d[k++] = B.rz[b];
  }
  P.src_d[k] = A.vx; P.dst_d[k++] = B.vx;
  P.src_d[k] = A.vy; P.dst_d[k++] = B.vy;
  P.src_d[k] = A.vz; P.dst_d[k++] = B.vz;
  P.src_d[k] = A.bx; P.dst_d[k++] = B.bx;
  P.src_d[k] = A.by; P.dst_d[k++] = B.by;
  P.src_d[k] = A.bz; P.dst_d[k++] = B.bz;
  P.src_d[k] = A.mass; P.dst_d[k++] = B.mass;
  if (S->prec == SL_FP64) {
    P.src_d[k] = (const double *)A.sx; P.dst_d[k++] = (double *)B.sx;
    P.src_d[k] = (const double *)A.sy; P.dst_d[k++] = (double *)B.sy;
    P.src_d[k] = (const double *)A.sz; P.dst_d[k++] = (double *)B.sz;
  } else {
    P.src_f[0] = (const float *)A.sx; P.dst_f[0] = (float *)B.sx;
    P.src_f[1] = (const float *)A.sy; P.dst_f[1] = (float *)B.sy;
    P.src_f[2] = (const float *)A.sz; P.dst_f[2] = (float *)B.sz;
    P.nf = 3;
  }
  P.nd = k;
  P.src_i[0] = A.id; P.dst_i[0] = B.id;
  P.src_i[1] = A.colour; P.dst_i[1] = B.colour;
  P.src_i[2] = A.cell; P.dst_i[2] = B.cell;
  P.ni = 3;
  launch_permute_atoms(P, S->st);
  launch_permute_nbr(n, S->ld, S->perm, S->inv, A.nbr, A.nspin, A.nall, B.nbr, B.nspin, B.nall, S->st);
  S->cur = 1 - S->cur;
  S->jc_ok[0] = S->jc_ok[1] = false;
  // class offsets = bucket starts of the first cell of every colour
  if (S->K + 1 > kPinWords - 16) return fail(S, SL_E_COLOR, "too many colour classes");
  launch_class_offsets(S->bstart, nrow, S->K, S->pin_dev + 16, S->st);
  HIPCHK(S, hipStreamSynchronize(S->st));
  S->class_off.assign(S->K + 1, 0);
  for (int c = 0; c <= S->K; ++c) S->class_off[c] = S->pin[16 + c];
  S->ftile_lanes = -1;  // the force launch's tiles follow the classes
  {
    Atoms &N = S->a[S->cur];
    launch_watch_mask(n, S->ld, N.nbr, N.nspin, N.colour, N.wmask, S->st);
  }
  if (S->mlp) CHK(mlp_pairs(S));
  return SL_OK;
}

// Full rebuild at the current boundary: cells, lists, colour repair, order.
int rebuild(sl_system *S) {
  if (S->user_list) return colour_and_permute(S, false);
  CHK(check_box(S));
  {
    ProfScope ps(S, 2, (double)S->n);
    CellGrid G;
    CHK(bin_cells(S, G));
    Atoms &A = S->a[S->cur];
    NbrBuildArgs B;
    B.n = S->n;
    B.ld = S->ld;
    B.max_nbr = S->max_nbr;
    B.max_spin = S->max_spin;
    const double rs = spin_radius(S), rl = std::max(list_radius(S), rs);
    B.rs2 = rs * rs;
    B.rl2 = rl * rl;
    B.G = G;
    B.rx = A.rx[S->pos];
    B.ry = A.ry[S->pos];
    B.rz = A.rz[S->pos];
    B.cell = A.cell;
    B.cstart = S->cstart;
    B.catoms = S->catoms;
    // cell-ordered positions in the staging buffer (free during a rebuild)
    B.cx = S->stage;
    B.cy = S->stage + S->n;
    B.cz = S->stage + 2 * (size_t)S->n;
    launch_cell_positions(S->n, S->catoms, B.rx, B.ry, B.rz, S->stage, S->stage + S->n,
                          S->stage + 2 * (size_t)S->n, S->st);
    B.nbr = A.nbr;
    B.nspin = A.nspin;
    B.nall = A.nall;
    B.bx = A.bx;
    B.by = A.by;
    B.bz = A.bz;
    B.err = S->err;
    B.seen = S->seen;
    B.row_q = S->row_q;
    HIPCHK(S, hipMemsetAsync(S->seen, 0, 2 * sizeof(int), S->st));
    launch_nbr_build(B, S->st);
    // the build's error word and largest rows are read back with the
    // colouring's report (one host synchronisation for both); an
    // overflowing row only truncates what the colouring sees meanwhile
  }
  S->have_list = true;
  S->rebuilds++;
  return colour_and_permute(S, true);
}

int ensure_ready(sl_system *S) {
  if (!S->have_state) return fail(S, SL_E_STATE, "no state set");
  if (!S->have_pot) return fail(S, SL_E_STATE, "no potential set");
  if (!S->have_list) {
    CHK(rebuild(S));
  } else if (!S->have_colour) {
    CHK(colour_and_permute(S, false));
  }
  return SL_OK;
}

}  // namespace sl
