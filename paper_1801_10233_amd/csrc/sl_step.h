// sl_step.h -- device parts of one spin-lattice step, shared by the
// single-system kernels (sl_dyn.hip, sl_force.hip) and the batched kernels
// (sl_batch.hip): the spin update of one atom, the force gather of one atom
// with the kicks and the drift, and the embedded-atom density of one atom.
// One thread (or LANES lanes) per atom; per-atom data in structure-of-arrays
// form so the own-atom loads and stores of a wavefront are coalesced, and
// neighbour data gathered through L2 (atoms are sorted by cell inside a
// colour class).
#pragma once

#include <type_traits>

#include "sl_device.h"
#include "sl_kernels.h"

#ifndef SL_SPIN_FIRST
#define SL_SPIN_FIRST 7  // slots of the first round with one lane per atom
#endif
#ifndef SL_SPIN_LATER
#define SL_SPIN_LATER 8  // slots of each later round with one lane per atom
#endif

#ifndef SL_FORCE_CHUNK0
#define SL_FORCE_CHUNK0 2  // force-gather slots per round in the spin segment
#endif
#ifndef SL_FORCE_CHUNK1
#define SL_FORCE_CHUNK1 SL_FORCE_CHUNK  // the same in the rest of the row (positions only)
#endif

namespace sl {

// Cayley rotation of Sec. 3 about w with step h, in place (an exact
// rotation by 2 atan(h|w|/2); |s| is kept in exact arithmetic).
template <typename real>
__device__ __forceinline__ void cayley_rot(real &sx, real &sy, real &sz, real wx, real wy, real wz,
                                           real h) {
  const real cx = wy * sz - wz * sy, cy = wz * sx - wx * sz, cz = wx * sy - wy * sx;
  const real ws = wx * sx + wy * sy + wz * sz;
  const real w2 = wx * wx + wy * wy + wz * wz;
  const real q = h * h * (real)0.25;
  const real inv = (real)1 / ((real)1 + q * w2);
  const real nx = (sx + h * cx + q * ((real)2 * wx * ws - w2 * sx)) * inv;
  const real ny = (sy + h * cy + q * ((real)2 * wy * ws - w2 * sy)) * inv;
  const real nz = (sz + h * cz + q * ((real)2 * wz * ws - w2 * sz)) * inv;
  sx = nx; sy = ny; sz = nz;
}

// ---------------------------------------------------------------------------
// Spin colour phase. For every atom i of one class (no two of them
// interact): omega_i = (1/hbar)[sum_j J(r_ij) s_j + g mu_B B + 2K(s_i.n)n]
// over the spin segment of its list, then s_i is rotated in closed form by
// the Cayley map with step h (Sec. 3). With the spin bath, the rotation
// vector is W = (omega + eta + lambda s x omega)/(1 + lambda^2) with eta
// drawn from the Philox stream of (atom id, step, replica, sub-update)
// (Sec. 4.1, Eq. sLLG). nrep > 1 applies consecutive updates of the same
// class in one launch (nothing else changes in between); the exchange sum
// does not depend on s_i, so it is gathered once.
// One spin update (or nrep successive ones) of atom i, shared by the
// per-class launch and the fused small-class launch. All LANES lanes of an
// atom must call it (cross-lane shuffles); `valid` masks the tail.
// Neighbour slots one lane gathers per round of the spin phase (value: the
// first round, later: each later one). With one lane per atom a first round
// of 7 and a second of 8 cover the 14 entries of a bcc spin segment at the
// exchange cutoff and the 15 or 16 that thermal motion puts into some rows
// (measured at 432 000 atoms: 7 + 7, 7 + 9, 6 + 8, 6 + 10, 5 + 9 and 8 + 8
// were slower); with two lanes the same per lane (the batched replicas' step
// 4 % faster than with rounds of 8).
template <int LANES, int MLP = 0>
struct SpinChunk {
  static constexpr int value = LANES >= 8 ? 2 : (LANES >= 4 ? 4 : (LANES == 2 ? 7 : SL_SPIN_FIRST));
  static constexpr int later = LANES == 1 ? SL_SPIN_LATER : (LANES == 2 ? 8 : value);
};
// The spin-orbit variant holds a field vector per slot besides the
// coefficient, and its dual form a second one: 4 slots per round keep it
// well below the 256-register limit (at 8 its dual forms reached 256
// registers plus accumulation-register spills and gave wrong results on
// MI355X, in instances that changed with unrelated code edits).
template <int LANES>
struct SpinChunk<LANES, 4> {
  static constexpr int value = LANES >= 8 ? 2 : 4;
  static constexpr int later = value;
};

// DUAL: two successive updates of one class at two sets of positions (the
// last update of a spin half-step and the first of the next, with the drift
// in between): the neighbour spins are the same for both (no other class
// moves in between), so they are gathered once and the exchange field is
// summed at the positions of S for the first update and of S2 (same atoms,
// same list, the other position buffer) for the second; nrep must be 2.
template <typename real, bool LANGEVIN, bool ANISO, int LANES, int MLP, bool DUAL = false>
__device__ __forceinline__ void spin_update(const SysView<real> &S, const PotConst &P, int i,
                                            bool valid, int l, int nrep, const int64_t *step,
                                            const int *sub, double hd, double ampd,
                                            uint64_t seed, uint32_t replica, double rs2,
                                            const SysView<real> *S2 = nullptr,
                                            bool keep0 = false) {
  // Latency is what bounds this update, so every load that does not depend
  // on another is issued at once: the row length, the own position, spin
  // and id, and the list entries of the first round (taken unconditionally
  // up to the list capacity; a slot past the row end is masked afterwards,
  // and any index outside [0, n) is replaced by i before it is used). The
  // gathers of positions and spins follow in one batch, and the Philox
  // noise of the first update is computed while they are in flight.
  constexpr int CH0 = SpinChunk<LANES, MLP>::value, CH1 = SpinChunk<LANES, MLP>::later;
  real ax = 0, ay = 0, az = 0;
  real bx = 0, by = 0, bz = 0;  // DUAL: field at the positions of S2
  real sx = 0, sy = 0, sz = 0;
  real g0[3] = {0, 0, 0};
  uint32_t aid = 0;
  if (valid) {
    const int ld = S.ld;
    const int ns = S.nspin[i];
    const double rix = S.rx[i], riy = S.ry[i], riz = S.rz[i];
    double rix2 = 0, riy2 = 0, riz2 = 0;
    if (DUAL) { rix2 = S2->rx[i]; riy2 = S2->ry[i]; riz2 = S2->rz[i]; }
    sx = S.sx[i]; sy = S.sy[i]; sz = S.sz[i];
    if (LANGEVIN) aid = (uint32_t)S.id[i];
    // one round of CH slots from base (a generic lambda, so that the first
    // round and the later ones can differ in size)
    auto gather_round = [&](auto chunk, int base, bool first) {
      // the first round loads its slots before the row length is known;
      // later ones (the row length has arrived) load only the row's own
      constexpr int CH = decltype(chunk)::value;
      const int kend = first ? S.kcap : ns;
      int jj[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int k = base + LANES * c;
        const int j = k < kend ? S.nbr[(size_t)k * ld + i] : i;
        jj[c] = (unsigned)j < (unsigned)S.n ? j : i;
      }
      real qx[CH], qy[CH], qz[CH], J[CH];
      real hx[CH], hy[CH], hz[CH];  // MLP == 4: Neel and DMI field of the pair
      double px[CH], py[CH], pz[CH];
      float jt[CH];
      real jr[CH];
      // DUAL: the same at the second positions
      real J2[CH], hx2[CH], hy2[CH], hz2[CH];
      double px2[CH], py2[CH], pz2[CH];
      float jt2[CH];
      real jr2[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int k = base + LANES * c;
        if (MLP == 1) {
          jt[c] = k < kend ? S.tab[(size_t)k * ld + i].x : 0.f;
          if (DUAL) jt2[c] = k < kend ? S2->tab[(size_t)k * ld + i].x : 0.f;
        } else if (MLP == 3) {
          jr[c] = k < kend ? S.jc[(size_t)k * ld + i] : (real)0;
          if (DUAL) jr2[c] = k < kend ? S2->jc[(size_t)k * ld + i] : (real)0;
        } else {
          px[c] = S.rx[jj[c]]; py[c] = S.ry[jj[c]]; pz[c] = S.rz[jj[c]];
          if (DUAL) { px2[c] = S2->rx[jj[c]]; py2[c] = S2->ry[jj[c]]; pz2[c] = S2->rz[jj[c]]; }
        }
        qx[c] = S.sx[jj[c]]; qy[c] = S.sy[jj[c]]; qz[c] = S.sz[jj[c]];
      }
      if (LANGEVIN && first && l == 0)
        gauss3(seed, aid, step[0], replica, sub[0], g0);
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const bool in = base + LANES * c < ns;
        if (MLP == 1) {
          J[c] = in ? (real)jt[c] : (real)0;
        } else if (MLP == 3) {
          J[c] = in ? jr[c] : (real)0;
        } else if (MLP == 2) {
          const double dx = min_image(rix - px[c], S.L[0], S.invL[0]);
          const double dy = min_image(riy - py[c], S.L[1], S.invL[1]);
          const double dz = min_image(riz - pz[c], S.L[2], S.invL[2]);
          const float r = (float)sqrt(dx * dx + dy * dy + dz * dz);
          J[c] = in ? (real)spline_phys(S.spl, r).x : (real)0;
        } else {
          const double dx = min_image(rix - px[c], S.L[0], S.invL[0]);
          const double dy = min_image(riy - py[c], S.L[1], S.invL[1]);
          const double dz = min_image(riz - pz[c], S.L[2], S.invL[2]);
          const double r2 = dx * dx + dy * dy + dz * dz;
          const real Jc = exch_J<real>(P, r2);
          J[c] = (in && r2 < rs2) ? Jc : (real)0;
          if (MLP == 4) {
            hx[c] = hy[c] = hz[c] = (real)0;
            if (in) soc_field<real>(P, dx, dy, dz, r2, qx[c], qy[c], qz[c], hx[c], hy[c], hz[c]);
          }
        }
      }
      if (DUAL) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const bool in = base + LANES * c < ns;
          if (MLP == 1) {
            J2[c] = in ? (real)jt2[c] : (real)0;
          } else if (MLP == 3) {
            J2[c] = in ? jr2[c] : (real)0;
          } else if (MLP == 2) {
            const double dx = min_image(rix2 - px2[c], S.L[0], S.invL[0]);
            const double dy = min_image(riy2 - py2[c], S.L[1], S.invL[1]);
            const double dz = min_image(riz2 - pz2[c], S.L[2], S.invL[2]);
            const float r = (float)sqrt(dx * dx + dy * dy + dz * dz);
            J2[c] = in ? (real)spline_phys(S.spl, r).x : (real)0;
          } else {
            const double dx = min_image(rix2 - px2[c], S.L[0], S.invL[0]);
            const double dy = min_image(riy2 - py2[c], S.L[1], S.invL[1]);
            const double dz = min_image(riz2 - pz2[c], S.L[2], S.invL[2]);
            const double r2 = dx * dx + dy * dy + dz * dz;
            const real Jc = exch_J<real>(P, r2);
            J2[c] = (in && r2 < rs2) ? Jc : (real)0;
            if (MLP == 4) {
              hx2[c] = hy2[c] = hz2[c] = (real)0;
              if (in) soc_field<real>(P, dx, dy, dz, r2, qx[c], qy[c], qz[c], hx2[c], hy2[c], hz2[c]);
            }
          }
        }
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        ax += J[c] * qx[c];
        ay += J[c] * qy[c];
        az += J[c] * qz[c];
        if (MLP == 4) {
          ax += hx[c];
          ay += hy[c];
          az += hz[c];
        }
        if (DUAL) {
          bx += J2[c] * qx[c];
          by += J2[c] * qy[c];
          bz += J2[c] * qz[c];
          if (MLP == 4) {
            bx += hx2[c];
            by += hy2[c];
            bz += hz2[c];
          }
        }
      }
    };
    gather_round(std::integral_constant<int, CH0>{}, l, true);
    for (int base = l + LANES * CH0; base < ns; base += LANES * CH1)
      gather_round(std::integral_constant<int, CH1>{}, base, false);
  }
#pragma unroll
  for (int o = LANES / 2; o > 0; o >>= 1) {
    ax += __shfl_xor(ax, o, 64);
    ay += __shfl_xor(ay, o, 64);
    az += __shfl_xor(az, o, 64);
    if (DUAL) {
      bx += __shfl_xor(bx, o, 64);
      by += __shfl_xor(by, o, 64);
      bz += __shfl_xor(bz, o, 64);
    }
  }
  if (!valid || l != 0) return;
  const real h = (real)hd;
  const real ih = (real)(1.0 / kHbar);
  for (int rep = 0; rep < nrep; ++rep) {
    if (keep0 && rep == 1) {  // the state between the two updates, for the force
      S.sx[S.n + i] = sx;
      S.sy[S.n + i] = sy;
      S.sz[S.n + i] = sz;
    }
    const bool second = DUAL && rep == 1;
    real ex = (second ? bx : ax) + (real)P.zB[0], ey = (second ? by : ay) + (real)P.zB[1],
         ez = (second ? bz : az) + (real)P.zB[2];
    if (ANISO && P.aniso_split) {  // set only without the spin bath
      // symmetric split A(h/2) X(h) A(h/2): A rotates about n at the rate
      // (2K/hbar)(s.n), which A itself keeps fixed; X about the field
      // without the anisotropy (it does not depend on s_i)
      const real n0 = (real)P.an[0], n1 = (real)P.an[1], n2 = (real)P.an[2];
      const real k2 = (real)2 * (real)P.aK * ih;
      const real hh = (real)0.5 * h;
      real c = k2 * (sx * n0 + sy * n1 + sz * n2);
      cayley_rot<real>(sx, sy, sz, c * n0, c * n1, c * n2, hh);
      cayley_rot<real>(sx, sy, sz, ex * ih, ey * ih, ez * ih, h);
      c = k2 * (sx * n0 + sy * n1 + sz * n2);
      cayley_rot<real>(sx, sy, sz, c * n0, c * n1, c * n2, hh);
      if (sizeof(real) == 4) {
        const real rn = (real)rsqrtf((float)(sx * sx + sy * sy + sz * sz));
        sx *= rn; sy *= rn; sz *= rn;
      }
      continue;
    }
    if (ANISO) {
      const real sn2 = (real)2 * (real)P.aK * (sx * (real)P.an[0] + sy * (real)P.an[1] + sz * (real)P.an[2]);
      ex += sn2 * (real)P.an[0];
      ey += sn2 * (real)P.an[1];
      ez += sn2 * (real)P.an[2];
    }
    real wx = ex * ih, wy = ey * ih, wz = ez * ih;
    if (LANGEVIN) {
      real g[3] = {g0[0], g0[1], g0[2]};
      if (rep > 0) gauss3(seed, aid, step[rep], replica, sub[rep], g);
      const real lam = (real)P.lam, amp = (real)ampd, f = (real)P.lamfac;
      const real cx = sy * wz - sz * wy, cy = sz * wx - sx * wz, cz = sx * wy - sy * wx;
      wx = (wx + amp * g[0] + lam * cx) * f;
      wy = (wy + amp * g[1] + lam * cy) * f;
      wz = (wz + amp * g[2] + lam * cz) * f;
    }
    // Cayley rotation of Sec. 3 (Omelyan): exact rotation about W by
    // 2 atan(h|W|/2); preserves |s| in exact arithmetic.
    const real cx = wy * sz - wz * sy, cy = wz * sx - wx * sz, cz = wx * sy - wy * sx;
    const real ws = wx * sx + wy * sy + wz * sz;
    const real w2 = wx * wx + wy * wy + wz * wz;
    const real q = h * h * (real)0.25;
    const real inv = (real)1 / ((real)1 + q * w2);
    real nx = (sx + h * cx + q * ((real)2 * wx * ws - w2 * sx)) * inv;
    real ny = (sy + h * cy + q * ((real)2 * wy * ws - w2 * sy)) * inv;
    real nz = (sz + h * cz + q * ((real)2 * wz * ws - w2 * sz)) * inv;
    if (sizeof(real) == 4) {
      // FP32 form: renormalise after every rotation.
      const real rn = (real)rsqrtf((float)(nx * nx + ny * ny + nz * nz));
      nx *= rn; ny *= rn; nz *= rn;
    }
    sx = nx; sy = ny; sz = nz;
  }
  S.sx[i] = sx;
  S.sy[i] = sy;
  S.sz[i] = sz;
}


// ---------------------------------------------------------------------------
// Force, kicks and drift at one step boundary. With e_ij = (r_i - r_j)/r:
//   F_i = sum_j [-V'(r) + J'(r) s_i.s_j] e_ij        (Eq. p_advance)
// over the full list (both i and j own the pair, no atomics), then
//   FINAL: v += (dt/2) F/m              (last half kick of the step)
//   NEXT:  v += (dt/2) F/m; r' = r + dt v  (first half kick and drift of the
//          next step, written to the other position buffer)
//   ENERGY: per-atom energies (pairs halved) and M, block partial sums.
// Every launch with a kick also reduces max |r - r_build| and max |v| at
// this boundary for the rebuild decision, block by block; a one-block join
// after the launch hands them, with the sticky error word, to pinned host
// memory.
// Per-atom part of the force launch (shared with the batched persistent
// kernel): force on atom i over its list row, split over LANES lanes, then on
// the first lane the kicks, the drift into the other position buffer, the
// energy terms e[8] = (kin, pair, exchange, Zeeman, aniso, Mx, My, Mz) and
// the rebuild predictor terms |r - r_build| and |v|.
// Variant MLP of the force gather: MLP & 7 selects the pair terms (0 analytic,
// 1 learned per-pair table, 2 learned spline, 4 analytic with the spin-orbit
// pair terms); MLP & 8 adds the embedded-atom terms, whose F'(rho) of every
// atom a first pass (k_eam_density) has stored.
// Split force (analytic forms only): MLP & 16 is the pair pass, which sums
// the spin-independent terms (Morse, embedded atom) over the whole row and
// stores them in A.fp, and does nothing else; it depends on the positions
// alone, so it can run while the spins are still being updated. MLP & 32 is
// the spin pass: the spin-dependent terms over the spin segment only, plus
// the stored pair part, then the kicks, drift, energies and predictor as in
// the fused form.
template <typename real, int MODE, int LANES, int MLP>
__device__ __forceinline__ void force_atom(const SysView<real> &S, const PotConst &P,
                                           const ForceArgs &A, int i, bool valid, int l,
                                           double e[8], double &dm, double &vm, double &wm) {
  constexpr int kV = MLP & 7;
  constexpr bool kEam = (MLP & 8) != 0;
  constexpr bool kPairPass = (MLP & 16) != 0, kSpinPass = (MLP & 32) != 0;
  static_assert(!(kPairPass || kSpinPass) || kV == 0 || kV == 4,
                "the split force covers the analytic forms only");
  static_assert(!(kPairPass && kSpinPass), "one pass at a time");
  real fx = 0, fy = 0, fz = 0;
  real ep = 0, ee = 0;
  double rix = 0, riy = 0, riz = 0;
  real six = 0, siy = 0, siz = 0;
  if (valid) {
    rix = S.rx[i]; riy = S.ry[i]; riz = S.rz[i];
    const int is = i < S.held ? S.n + i : i;
    six = S.sx[is]; siy = S.sy[is]; siz = S.sz[is];
    const int ns = S.nspin[i], na = S.nall[i];
    const int ld = S.ld;
    // the variant may serve replicas without the embedded-atom terms
    const bool eam = kEam && !kSpinPass && P.eam_on;
    const real fpi = eam ? (real)S.eam[i] : (real)0;
    if (eam && (MODE & kModeEnergy) && l == 0) ep += (real)S.eam[ld + i];
    // spin-segment slots holding a pair of one colour class are watched
    const unsigned long long wmk =
        (!kPairPass && (MODE & (kModeFinal | kModeNext)) && A.wmask) ? A.wmask[i] : 0ull;
    // Two segments of the row, each gathered in chunks (all loads of a
    // chunk in flight together): the spin segment [0, ns) needs positions
    // and spins, the rest [ns, na) lies beyond the exchange cutoff (its
    // build-time distance exceeds ex_rc + skin, and no atom has moved more
    // than skin/2) and needs positions only.
    // (the two segments are unrolled: each copy knows whether it needs the
    // neighbour spins, and schedules all of a chunk's loads together)
    // the two segments as one generic lambda called twice, so that each
    // knows at compile time whether it needs the neighbour spins and takes
    // its own chunk size
    auto segment = [&](auto segc, auto chunkc) {
      constexpr int seg = decltype(segc)::value;
      constexpr int CHF = decltype(chunkc)::value;
      const int beg = seg == 0 ? 0 : ns, end = seg == 0 ? ns : na;
      for (int base = beg + l; base < end; base += LANES * CHF) {
        int jj[CHF];
#pragma unroll
        for (int c = 0; c < CHF; ++c) {
          const int k = base + LANES * c;
          jj[c] = k < end ? S.nbr[(size_t)k * ld + i] : i;
        }
        double px[CHF], py[CHF], pz[CHF];
        real sij[CHF];
        real qx[CHF], qy[CHF], qz[CHF];  // spin segment
        real fpj[CHF];                                   // kEam
        float4 tt[CHF];
#pragma unroll
        for (int c = 0; c < CHF; ++c) {
          px[c] = S.rx[jj[c]]; py[c] = S.ry[jj[c]]; pz[c] = S.rz[jj[c]];
          if (kEam) fpj[c] = eam ? (real)S.eam[jj[c]] : (real)0;
          if (seg == 0 && !kPairPass) {
            const int js = jj[c] < S.held ? S.n + jj[c] : jj[c];
            qx[c] = S.sx[js]; qy[c] = S.sy[js]; qz[c] = S.sz[js];
          }
        }
#pragma unroll
        for (int c = 0; c < CHF; ++c)
          sij[c] = (seg == 0 && !kPairPass) ? six * qx[c] + siy * qy[c] + siz * qz[c] : (real)0;
        if (kV == 1) {
#pragma unroll
          for (int c = 0; c < CHF; ++c) {
            const int k = base + LANES * c;
            tt[c] = k < end ? S.tab[(size_t)k * ld + i] : make_float4(0.f, 0.f, 0.f, 0.f);
          }
        }
#pragma unroll
        for (int c = 0; c < CHF; ++c) {
          const bool use = base + LANES * c < end;
          const double dxd = min_image(rix - px[c], S.L[0], S.invL[0]);
          const double dyd = min_image(riy - py[c], S.L[1], S.invL[1]);
          const double dzd = min_image(riz - pz[c], S.L[2], S.invL[2]);
          const double r2d = use ? dxd * dxd + dyd * dyd + dzd * dzd : 1.0;
          if (!kPairPass && seg == 0 && use && ((wmk >> (base + LANES * c)) & 1ull)) wm = fmin(wm, r2d);
          const real dx = (real)dxd, dy = (real)dyd, dz = (real)dzd;
          const double rinvd = rsqrt_nr(r2d);
          const real r = (real)(r2d * rinvd), rinv = (real)rinvd;
          real cc = 0;
          if (kV == 2) tt[c] = use ? spline_phys(S.spl, (float)r) : make_float4(0.f, 0.f, 0.f, 0.f);
          if (kV == 1 || kV == 2) {
            // learned phi'(r), J'(r) (and phi, J for energies) from the table
            cc = -(real)tt[c].w + (real)tt[c].y * sij[c];
            if (MODE & kModeEnergy) {
              ep += (real)0.5 * (real)tt[c].z;
              ee -= (real)0.5 * (real)tt[c].x * sij[c];
            }
          } else {
            if (!kSpinPass && P.morse_on && r2d < P.mRc2) {
              const real ex = exp_pair(-(real)P.mA * (r - (real)P.mR0));
              const real dM = -(real)2 * (real)P.mA * (real)P.mD * (ex * ex - ex);
              cc -= dM - (real)P.mdMc;
              if (MODE & kModeEnergy)
                ep += use ? (real)0.5 * ((real)P.mD * (ex * ex - (real)2 * ex) - (real)P.mMc -
                                         (r - (real)P.mRc) * (real)P.mdMc)
                          : (real)0;
            }
            if (!kPairPass && seg == 0 && P.ex_on && r2d < P.eRc2) {
              const real u = (real)(r2d * P.eInvD2);
              const real eu = exp_pair(-u);
              const real dJ = (real)P.eA8InvD2 * r * eu *
                                  ((real)1 - ((real)1 + (real)2 * (real)P.eG) * u + (real)P.eG * u * u) -
                              r * (real)P.eJr;
              cc += dJ * sij[c];
              if (MODE & kModeEnergy) {
                const real Jv = (real)P.eA4 * u * ((real)1 - (real)P.eG * u) * eu -
                                ((real)P.eJc + (real)(r2d - P.eRc2) * (real)P.eJq);
                ee -= use ? (real)0.5 * Jv * sij[c] : (real)0;
              }
            }
          }
          if (kEam && eam) {
            // -[phi'(r) + (F'(rho_i) + F'(rho_j)) f'(r)]
            if (r2d < P.fd2) {
              const real x = r - (real)P.fd;
              cc -= (fpi + fpj[c]) * ((real)2 * x + (real)3 * (real)P.fbeta * x * x / (real)P.fd);
            }
            if (r2d < P.fcc2) {
              const real x = r - (real)P.fc;
              const real q = (real)P.fc0 + (real)P.fc1 * r + (real)P.fc2 * r * r;
              cc -= (real)2 * x * q + x * x * ((real)P.fc1 + (real)2 * (real)P.fc2 * r);
              if (MODE & kModeEnergy) ep += use ? (real)0.5 * x * x * q : (real)0;
            }
          }
          const real cr = use ? cc * rinv : (real)0;
          fx += cr * dx;
          fy += cr * dy;
          fz += cr * dz;
          if (kV == 4 && !kPairPass && seg == 0 && use) {
            const real es = soc_force<real>(P, dxd, dyd, dzd, r2d, six, siy, siz, qx[c], qy[c],
                                            qz[c], fx, fy, fz);
            if (MODE & kModeEnergy) ee += (real)0.5 * es;
          }
        }
      }
    };
    segment(std::integral_constant<int, 0>{}, std::integral_constant<int, SL_FORCE_CHUNK0>{});
    if (!kSpinPass)
      segment(std::integral_constant<int, 1>{}, std::integral_constant<int, SL_FORCE_CHUNK1>{});
  }
#pragma unroll
  for (int o = LANES / 2; o > 0; o >>= 1) {
    fx += __shfl_xor(fx, o, 64);
    fy += __shfl_xor(fy, o, 64);
    fz += __shfl_xor(fz, o, 64);
    if (MODE & kModeEnergy) {
      ep += __shfl_xor(ep, o, 64);
      ee += __shfl_xor(ee, o, 64);
    }
  }
  if (kPairPass) {
    if (valid && l == 0) {
      const int ld = S.ld;
      A.fp[i] = (double)fx;
      A.fp[ld + i] = (double)fy;
      A.fp[2 * ld + i] = (double)fz;
      if (MODE & kModeEnergy) A.fp[3 * ld + i] = (double)ep;
    }
    return;
  }
  if (kSpinPass && valid && l == 0) {
    const int ld = S.ld;
    fx += (real)A.fp[i];
    fy += (real)A.fp[ld + i];
    fz += (real)A.fp[2 * ld + i];
    if (MODE & kModeEnergy) ep += (real)A.fp[3 * ld + i];
  }
  if (valid && l == 0) {
    if (!isfinite((double)fx) || !isfinite((double)fy) || !isfinite((double)fz))
      atomicOr(A.err, kErrNonFinite);
    if (MODE & (kModeFinal | kModeNext)) {
      const double m = A.mass[i];
      double vx = A.vx[i], vy = A.vy[i], vz = A.vz[i];
      const double kx = 0.5 * A.dt * (double)fx / m * A.ftm2v;
      const double ky = 0.5 * A.dt * (double)fy / m * A.ftm2v;
      const double kz = 0.5 * A.dt * (double)fz / m * A.ftm2v;
      if (MODE & kModeFinal) { vx += kx; vy += ky; vz += kz; }
      if (MODE & kModeEnergy) e[0] = 0.5 * m * (vx * vx + vy * vy + vz * vz) * kMvv2e;
      // rebuild predictor at this boundary
      {
        const double bx = rix - A.bx[i], by = riy - A.by[i], bz = riz - A.bz[i];
        dm = sqrt(bx * bx + by * by + bz * bz);
        vm = sqrt(vx * vx + vy * vy + vz * vz);
      }
      if (MODE & kModeNext) {
        vx += kx; vy += ky; vz += kz;
        double nx, ny, nz;
        if (P.lat_on) {
          // lattice bath (Eq. p_advance_T): exact Ornstein-Uhlenbeck step of
          // the friction and noise between two half drifts
          const double hd = 0.5 * A.dt;
          const double c = exp(-P.lat_g * fabs(A.dt) / m);
          const double sg = sqrt((1.0 - c * c) * P.lat_kT / m * A.ftm2v);
          double g[3];
          gauss3(A.seed ^ kLatticeKeyTag, (uint32_t)S.id[i], A.step, A.replica, 0, g);
          nx = rix + hd * vx; ny = riy + hd * vy; nz = riz + hd * vz;
          vx = c * vx + sg * g[0];
          vy = c * vy + sg * g[1];
          vz = c * vz + sg * g[2];
          nx += hd * vx; ny += hd * vy; nz += hd * vz;
        } else {
          nx = rix + A.dt * vx; ny = riy + A.dt * vy; nz = riz + A.dt * vz;
        }
        A.nx[i] = nx; A.ny[i] = ny; A.nz[i] = nz;
        if (!isfinite(nx) || !isfinite(ny) || !isfinite(nz)) atomicOr(A.err, kErrNonFinite);
      }
      A.vx[i] = vx; A.vy[i] = vy; A.vz[i] = vz;
    } else if (MODE & kModeEnergy) {
      const double m = A.mass[i];
      const double vx = A.vx[i], vy = A.vy[i], vz = A.vz[i];
      e[0] = 0.5 * m * (vx * vx + vy * vy + vz * vz) * kMvv2e;
    }
    if (MODE & kModeEnergy) {
      e[1] = (double)ep;
      e[2] = (double)ee;
      e[3] = -(P.zB[0] * (double)six + P.zB[1] * (double)siy + P.zB[2] * (double)siz);
      const double sn = P.an[0] * (double)six + P.an[1] * (double)siy + P.an[2] * (double)siz;
      e[4] = -P.aK * sn * sn;
      e[5] = (double)six; e[6] = (double)siy; e[7] = (double)siz;
    }
  }
}

// First pass of the embedded-atom terms: rho_i = sum_j f(r_ij) over the whole
// list row, then F'(rho_i) and F(rho_i) for the force pass (one thread per
// atom; one force-gather chunk of neighbours' positions in flight together).
template <typename real>
__device__ __forceinline__ void eam_density_atom(const SysView<real> &S, const PotConst &P, int i) {
  const int na = S.nall[i], ld = S.ld;
  const double rix = S.rx[i], riy = S.ry[i], riz = S.rz[i];
  real rho = 0;
  for (int base = 0; base < na; base += kForceChunk) {
    int jj[kForceChunk];
#pragma unroll
    for (int c = 0; c < kForceChunk; ++c) {
      const int k = base + c;
      jj[c] = k < na ? S.nbr[(size_t)k * ld + i] : i;
    }
    double px[kForceChunk], py[kForceChunk], pz[kForceChunk];
#pragma unroll
    for (int c = 0; c < kForceChunk; ++c) {
      px[c] = S.rx[jj[c]]; py[c] = S.ry[jj[c]]; pz[c] = S.rz[jj[c]];
    }
#pragma unroll
    for (int c = 0; c < kForceChunk; ++c) {
      const double dx = min_image(rix - px[c], S.L[0], S.invL[0]);
      const double dy = min_image(riy - py[c], S.L[1], S.invL[1]);
      const double dz = min_image(riz - pz[c], S.L[2], S.invL[2]);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (base + c < na && r2 < P.fd2) {
        const real x = (real)sqrt(r2) - (real)P.fd;
        rho += x * x + (real)P.fbeta * x * x * x / (real)P.fd;
      }
    }
  }
  const double sq = rho > (real)0 ? sqrt((double)rho) : 0.0;
  S.eam[i] = sq > 0.0 ? -0.5 * P.fA / sq : 0.0;
  S.eam[ld + i] = -P.fA * sq;
}


}  // namespace sl
