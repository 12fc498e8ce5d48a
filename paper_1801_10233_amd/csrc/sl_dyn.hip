// sl_dyn.hip -- per-step kernels of the spin-lattice step on gfx950:
//   * k_spin_phase: one colour class of a spin sweep (Sec. 3 / Sec. 5.1);
//   * k_force:      pair + magneto-mechanical force (Eq. p_advance), fused
//                   with the velocity-Verlet half kicks and the drift into
//                   the other position buffer, energies on sampled steps
//                   and the rebuild predictor;
//   * k_reduce8:    fixed-order second pass of the block partial sums.
// One thread per atom; per-atom data in structure-of-arrays form so the
// own-atom loads and stores of a wavefront are fully coalesced, neighbour
// data gathered through L2 (atoms are sorted by cell inside a class).
#include "sl_device.h"
#include "sl_kernels.h"

namespace sl {

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
// Neighbour slots one lane gathers per round of the spin phase: with one or
// two lanes per atom the first round covers 16 list slots (the whole spin
// segment of bcc at the exchange cutoff, 14 entries) in one go.
template <int LANES>
struct SpinChunk {
  static constexpr int value = LANES >= 8 ? 2 : (LANES >= 4 ? 4 : 8);
};

template <typename real, bool LANGEVIN, bool ANISO, int LANES, int MLP>
__device__ __forceinline__ void spin_update(const SysView<real> &S, const PotConst &P, int i,
                                            bool valid, int l, int nrep, const int64_t *step,
                                            const int *sub, double hd, double ampd,
                                            uint64_t seed, uint32_t replica, double rs2) {
  // Latency is what bounds this update, so every load that does not depend
  // on another is issued at once: the row length, the own position, spin
  // and id, and the list entries of the first round (taken unconditionally
  // up to the list capacity; a slot past the row end is masked afterwards,
  // and any index outside [0, n) is replaced by i before it is used). The
  // gathers of positions and spins follow in one batch, and the Philox
  // noise of the first update is computed while they are in flight.
  constexpr int CH = SpinChunk<LANES>::value;
  real ax = 0, ay = 0, az = 0;
  real sx = 0, sy = 0, sz = 0;
  real g0[3] = {0, 0, 0};
  uint32_t aid = 0;
  if (valid) {
    const int ld = S.ld;
    const int ns = S.nspin[i];
    const double rix = S.rx[i], riy = S.ry[i], riz = S.rz[i];
    sx = S.sx[i]; sy = S.sy[i]; sz = S.sz[i];
    if (LANGEVIN) aid = (uint32_t)S.id[i];
    for (int base = l, round = 0; round == 0 || base < ns; base += LANES * CH, ++round) {
      int jj[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int k = base + LANES * c;
        const int j = k < S.kcap ? S.nbr[(size_t)k * ld + i] : i;
        jj[c] = (unsigned)j < (unsigned)S.n ? j : i;
      }
      real qx[CH], qy[CH], qz[CH], J[CH];
      real hx[CH], hy[CH], hz[CH];  // MLP == 4: Neel and DMI field of the pair
      double px[CH], py[CH], pz[CH];
      float jt[CH];
      real jr[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        if (MLP == 1) {
          const int k = base + LANES * c;
          jt[c] = k < S.kcap ? S.tab[(size_t)k * ld + i].x : 0.f;
        } else if (MLP == 3) {
          const int k = base + LANES * c;
          jr[c] = k < S.kcap ? S.jc[(size_t)k * ld + i] : (real)0;
        } else {
          px[c] = S.rx[jj[c]]; py[c] = S.ry[jj[c]]; pz[c] = S.rz[jj[c]];
        }
        qx[c] = S.sx[jj[c]]; qy[c] = S.sy[jj[c]]; qz[c] = S.sz[jj[c]];
      }
      if (LANGEVIN && round == 0 && l == 0)
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
          const real u = (real)(r2 * P.eInvD2);
          const real Jc = (real)P.eA4 * u * ((real)1 - (real)P.eG * u) * exp(-u);
          J[c] = (in && r2 < rs2) ? Jc : (real)0;
          if (MLP == 4) {
            hx[c] = hy[c] = hz[c] = (real)0;
            if (in) soc_field<real>(P, dx, dy, dz, r2, qx[c], qy[c], qz[c], hx[c], hy[c], hz[c]);
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
      }
    }
  }
#pragma unroll
  for (int o = LANES / 2; o > 0; o >>= 1) {
    ax += __shfl_xor(ax, o, 64);
    ay += __shfl_xor(ay, o, 64);
    az += __shfl_xor(az, o, 64);
  }
  if (!valid || l != 0) return;
  const real h = (real)hd;
  const real ih = (real)(1.0 / kHbar);
  for (int rep = 0; rep < nrep; ++rep) {
    real ex = ax + (real)P.zB[0], ey = ay + (real)P.zB[1], ez = az + (real)P.zB[2];
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

template <typename real, bool LANGEVIN, bool ANISO, int LANES, int MLP>
__global__ __launch_bounds__(kBlock) void k_spin_phase(SysView<real> S, PotConst P,
                                                       SpinPhaseArgs A) {
  // LANES consecutive lanes share one atom: each gathers every LANES-th
  // neighbour, the partial sums are combined with cross-lane shuffles and
  // the first lane rotates and stores the spin.
  const int t = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const int l = t & (LANES - 1);
  const int i = A.begin + t / LANES;
  spin_update<real, LANGEVIN, ANISO, LANES, MLP>(S, P, i, i < A.end, l, A.nrep, A.step, A.sub,
                                                 A.h, A.amp, A.seed, A.replica, A.rs2);
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

// ---------------------------------------------------------------------------
// Force, kicks and drift at one step boundary. With e_ij = (r_i - r_j)/r:
//   F_i = sum_j [-V'(r) + J'(r) s_i.s_j] e_ij        (Eq. p_advance)
// over the full list (both i and j own the pair, no atomics), then
//   FINAL: v += (dt/2) F/m              (last half kick of the step)
//   NEXT:  v += (dt/2) F/m; r' = r + dt v  (first half kick and drift of the
//          next step, written to the other position buffer)
//   ENERGY: per-atom energies (pairs halved) and M, block partial sums.
// Every launch with a kick also reduces max |r - r_build| and max |v| at
// this boundary for the rebuild decision; the last block to finish hands
// them, with the sticky error word, to pinned host memory.
// Per-atom part of the force launch (shared with the batched persistent
// kernel): force on atom i over its list row, split over LANES lanes, then on
// the first lane the kicks, the drift into the other position buffer, the
// energy terms e[8] = (kin, pair, exchange, Zeeman, aniso, Mx, My, Mz) and
// the rebuild predictor terms |r - r_build| and |v|.
template <typename real, int MODE, int LANES, int MLP>
__device__ __forceinline__ void force_atom(const SysView<real> &S, const PotConst &P,
                                           const ForceArgs &A, int i, bool valid, int l,
                                           double e[8], double &dm, double &vm, double &wm) {
  real fx = 0, fy = 0, fz = 0;
  real ep = 0, ee = 0;
  double rix = 0, riy = 0, riz = 0;
  real six = 0, siy = 0, siz = 0;
  if (valid) {
    rix = S.rx[i]; riy = S.ry[i]; riz = S.rz[i];
    six = S.sx[i]; siy = S.sy[i]; siz = S.sz[i];
    const int ns = S.nspin[i], na = S.nall[i];
    const int ld = S.ld;
    // spin-segment slots holding a pair of one colour class are watched
    const unsigned long long wmk =
        ((MODE & (kModeFinal | kModeNext)) && A.wmask) ? A.wmask[i] : 0ull;
    // Two segments of the row, each gathered in chunks (all loads of a
    // chunk in flight together): the spin segment [0, ns) needs positions
    // and spins, the rest [ns, na) lies beyond the exchange cutoff (its
    // build-time distance exceeds ex_rc + skin, and no atom has moved more
    // than skin/2) and needs positions only.
    for (int seg = 0; seg < 2; ++seg) {
      const int beg = seg == 0 ? 0 : ns, end = seg == 0 ? ns : na;
      for (int base = beg + l; base < end; base += LANES * kForceChunk) {
        int jj[kForceChunk];
#pragma unroll
        for (int c = 0; c < kForceChunk; ++c) {
          const int k = base + LANES * c;
          jj[c] = k < end ? S.nbr[(size_t)k * ld + i] : i;
        }
        double px[kForceChunk], py[kForceChunk], pz[kForceChunk];
        real sij[kForceChunk];
        real qx[kForceChunk], qy[kForceChunk], qz[kForceChunk];  // MLP == 4
        float4 tt[kForceChunk];
#pragma unroll
        for (int c = 0; c < kForceChunk; ++c) {
          px[c] = S.rx[jj[c]]; py[c] = S.ry[jj[c]]; pz[c] = S.rz[jj[c]];
        }
        if (seg == 0 && MLP == 4) {
#pragma unroll
          for (int c = 0; c < kForceChunk; ++c) {
            qx[c] = S.sx[jj[c]]; qy[c] = S.sy[jj[c]]; qz[c] = S.sz[jj[c]];
            sij[c] = six * qx[c] + siy * qy[c] + siz * qz[c];
          }
        } else if (seg == 0) {
#pragma unroll
          for (int c = 0; c < kForceChunk; ++c)
            sij[c] = six * S.sx[jj[c]] + siy * S.sy[jj[c]] + siz * S.sz[jj[c]];
        } else {
#pragma unroll
          for (int c = 0; c < kForceChunk; ++c) sij[c] = 0;
        }
        if (MLP == 1) {
#pragma unroll
          for (int c = 0; c < kForceChunk; ++c) {
            const int k = base + LANES * c;
            tt[c] = k < end ? S.tab[(size_t)k * ld + i] : make_float4(0.f, 0.f, 0.f, 0.f);
          }
        }
#pragma unroll
        for (int c = 0; c < kForceChunk; ++c) {
          const bool use = base + LANES * c < end;
          const double dxd = min_image(rix - px[c], S.L[0], S.invL[0]);
          const double dyd = min_image(riy - py[c], S.L[1], S.invL[1]);
          const double dzd = min_image(riz - pz[c], S.L[2], S.invL[2]);
          const double r2d = use ? dxd * dxd + dyd * dyd + dzd * dzd : 1.0;
          if (seg == 0 && use && ((wmk >> (base + LANES * c)) & 1ull)) wm = fmin(wm, r2d);
          const real dx = (real)dxd, dy = (real)dyd, dz = (real)dzd;
          const double rinvd = rsqrt_nr(r2d);
          const real r = (real)(r2d * rinvd), rinv = (real)rinvd;
          real cc = 0;
          if (MLP == 2) tt[c] = use ? spline_phys(S.spl, (float)r) : make_float4(0.f, 0.f, 0.f, 0.f);
          if (MLP == 1 || MLP == 2) {
            // learned phi'(r), J'(r) (and phi, J for energies) from the table
            cc = -(real)tt[c].w + (real)tt[c].y * sij[c];
            if (MODE & kModeEnergy) {
              ep += (real)0.5 * (real)tt[c].z;
              ee -= (real)0.5 * (real)tt[c].x * sij[c];
            }
          } else {
            if (P.morse_on && r2d < P.mRc2) {
              const real ex = exp(-(real)P.mA * (r - (real)P.mR0));
              const real dM = -(real)2 * (real)P.mA * (real)P.mD * (ex * ex - ex);
              cc -= dM - (real)P.mdMc;
              if (MODE & kModeEnergy)
                ep += use ? (real)0.5 * ((real)P.mD * (ex * ex - (real)2 * ex) - (real)P.mMc -
                                         (r - (real)P.mRc) * (real)P.mdMc)
                          : (real)0;
            }
            if (seg == 0 && P.ex_on && r2d < P.eRc2) {
              const real u = (real)(r2d * P.eInvD2);
              const real eu = exp(-u);
              const real dJ = (real)P.eA8InvD2 * r * eu *
                              ((real)1 - ((real)1 + (real)2 * (real)P.eG) * u + (real)P.eG * u * u);
              cc += dJ * sij[c];
              if (MODE & kModeEnergy)
                ee -= use ? (real)0.5 * (real)P.eA4 * u * ((real)1 - (real)P.eG * u) * eu * sij[c]
                          : (real)0;
            }
          }
          const real cr = use ? cc * rinv : (real)0;
          fx += cr * dx;
          fy += cr * dy;
          fz += cr * dz;
          if (MLP == 4 && seg == 0 && use) {
            const real es = soc_force<real>(P, dxd, dyd, dzd, r2d, six, siy, siz, qx[c], qy[c],
                                            qz[c], fx, fy, fz);
            if (MODE & kModeEnergy) ee += (real)0.5 * es;
          }
        }
      }
    }
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

template <typename real, int MODE, int LANES, int MLP>
__global__ __launch_bounds__(kBlock, kForceWaves) void k_force(SysView<real> S, PotConst P, ForceArgs A) {
  __shared__ double red[kBlock / 64][8];
  __shared__ double redm[kBlock / 64][3];
  __shared__ int last;
  // Tiles are taken from the end of the atom order first: the last colour
  // classes may hold a few atoms scattered over the whole box (repairs),
  // whose gathers miss the caches; starting them first hides their latency
  // behind the bulk instead of leaving them as the tail of the launch.
  const int tile = gridDim.x - 1 - xcd_tile(blockIdx.x, gridDim.x);
  const int t = tile * kBlock + threadIdx.x;
  const int l = t & (LANES - 1);
  const int i = t / LANES;
  double e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double dm = 0.0, vm = 0.0, wm = kInf;
  force_atom<real, MODE, LANES, MLP>(S, P, A, i, i < S.n, l, e, dm, vm, wm);
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
    last = 0;
    if (MODE & (kModeFinal | kModeNext)) {
      double a = 0.0, b = 0.0, c = kInf;
      for (int w = 0; w < kBlock / 64; ++w) {
        a = fmax(a, redm[w][0]);
        b = fmax(b, redm[w][1]);
        c = fmin(c, redm[w][2]);
      }
      // non-negative doubles order like their bit patterns
      atomicMax(&A.dslot[0], (unsigned long long)__double_as_longlong(a));
      atomicMax(&A.dslot[1], (unsigned long long)__double_as_longlong(b));
      atomicMin(&A.dslot[2], (unsigned long long)__double_as_longlong(c));
      __threadfence();
      const unsigned prev = atomicAdd(A.done, 1u);
      last = (prev == gridDim.x - 1);
    }
  }
  __syncthreads();
  if ((MODE & (kModeFinal | kModeNext)) && last && threadIdx.x == 0) {
    __threadfence();
    const unsigned long long a = atomicExch(&A.dslot[0], 0ull);
    const unsigned long long b = atomicExch(&A.dslot[1], 0ull);
    const unsigned long long c = atomicExch(&A.dslot[2], (unsigned long long)__double_as_longlong(kInf));
    atomicExch(A.done, 0u);
    const int err = atomicOr(A.err, 0);
    A.host_out[0] = __longlong_as_double((long long)a);
    A.host_out[1] = __longlong_as_double((long long)b);
    A.host_out[2] = (double)err;
    A.host_out[4] = __longlong_as_double((long long)c);
    A.host_out[3] = 1.0;  // written marker
  }
}

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
          spin_update<real, true, true, LANES, MLP>(V, d.P, i, i < b1, l, nrep, st, sb, d.h, d.amp,
                                                     d.seed, d.replica, d.rs2);
        }
        __syncthreads();
      }
    }
    // force at the boundary after this step (positions 1 - pos); the drift
    // of the next step goes to buffer pos
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
void launch_batch_run(RepDesc<real> *D, int R, int lanes, bool soc, hipStream_t st) {
  if (R <= 0) return;
  if (soc) batch_run_lanes<real, 4>(D, R, lanes, st);
  else batch_run_lanes<real, 0>(D, R, lanes, st);
}
template void launch_batch_run<double>(RepDesc<double> *, int, int, bool, hipStream_t);
template void launch_batch_run<float>(RepDesc<float> *, int, int, bool, hipStream_t);

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

// Force, kicks and drift of every replica at one boundary, with each
// replica's rebuild predictor reduced by its own last block into its own
// pinned slot (as k_force does for one system).
template <typename real, int MODE, int LANES, int MLP>
__global__ __launch_bounds__(kBlock) void k_batch_force(const RepDesc<real> *D, BatchPhase bp) {
  __shared__ double redm[kBlock / 64][3];
  __shared__ int last;
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
    atomicMax(&F.dslot[0], (unsigned long long)__double_as_longlong(x));
    atomicMax(&F.dslot[1], (unsigned long long)__double_as_longlong(y));
    atomicMin(&F.dslot[2], (unsigned long long)__double_as_longlong(z));
    __threadfence();
    last = (atomicAdd(F.done, 1u) == (unsigned)nb - 1);
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __threadfence();
    const unsigned long long x = atomicExch(&F.dslot[0], 0ull);
    const unsigned long long y = atomicExch(&F.dslot[1], 0ull);
    const unsigned long long z = atomicExch(&F.dslot[2], (unsigned long long)__double_as_longlong(kInf));
    atomicExch(F.done, 0u);
    const int err = atomicOr(F.err, 0);
    F.host_out[0] = __longlong_as_double((long long)x);
    F.host_out[1] = __longlong_as_double((long long)y);
    F.host_out[2] = (double)err;
    F.host_out[4] = __longlong_as_double((long long)z);
    F.host_out[3] = 1.0;  // written marker
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

template <typename real>
void launch_batch_force(const RepDesc<real> *D, int R, int max_n, int mode, const BatchPhase &bp,
                        int lanes, bool soc, hipStream_t st) {
  if (R <= 0 || max_n <= 0) return;
  const int per = kBlock / lanes;
  const dim3 grid((max_n + per - 1) / per, R);
  if (soc) batch_force_any<real, 4>(D, grid, mode, bp, lanes, st);
  else batch_force_any<real, 0>(D, grid, mode, bp, lanes, st);
}
template void launch_batch_spin<double>(const RepDesc<double> *, int, int, const BatchPhase &, int, bool, hipStream_t);
template void launch_batch_spin<float>(const RepDesc<float> *, int, int, const BatchPhase &, int, bool, hipStream_t);
template void launch_batch_force<double>(const RepDesc<double> *, int, int, int, const BatchPhase &, int, bool, hipStream_t);
template void launch_batch_force<float>(const RepDesc<float> *, int, int, int, const BatchPhase &, int, bool, hipStream_t);

// Exchange coefficients at one set of positions (the optional pair
// coefficient cache): J(r_ij) for every spin-segment entry, with the same
// expression as the spin phase's own evaluation. Positions change only at
// the drift, so one evaluation serves the two spin half-steps that use
// these positions (Sec. 3: coefficients must be re-evaluated after the
// positions move, and only then).
template <typename real, bool SPL>
__global__ __launch_bounds__(kBlock) void k_jcache(SysView<real> S, PotConst P, real *out,
                                                   double rs2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  const int ns = S.nspin[i];
  const double rix = S.rx[i], riy = S.ry[i], riz = S.rz[i];
  // slots in chunks of 8 with all loads of a chunk issued before use; the
  // slot rows below kcap exist for every atom, so their loads need no guard
  constexpr int CH = 8;
  for (int k0 = 0; k0 < ns; k0 += CH) {
    int jj[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int k = k0 + c;
      const int j = k < S.kcap ? S.nbr[(size_t)k * S.ld + i] : i;
      jj[c] = (k < ns && (unsigned)j < (unsigned)S.n) ? j : i;
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
        const real u = (real)(r2 * P.eInvD2);
        const real Jc = (real)P.eA4 * u * ((real)1 - (real)P.eG * u) * exp(-u);
        out[(size_t)k * S.ld + i] = r2 < rs2 ? Jc : (real)0;
      }
    }
  }
}

template <typename real>
void launch_jcache(const SysView<real> &S, const PotConst &P, real *out, double rs2,
                   hipStream_t st) {
  if (S.n <= 0) return;
  const dim3 grid((S.n + kBlock - 1) / kBlock);
  if (S.spl.t) hipLaunchKernelGGL((k_jcache<real, true>), grid, dim3(kBlock), 0, st, S, P, out, rs2);
  else hipLaunchKernelGGL((k_jcache<real, false>), grid, dim3(kBlock), 0, st, S, P, out, rs2);
}
template void launch_jcache<double>(const SysView<double> &, const PotConst &, double *, double, hipStream_t);
template void launch_jcache<float>(const SysView<float> &, const PotConst &, float *, double, hipStream_t);

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
template <typename real, int LANES, int MLP>
static void spin_phase_lanes2(const SysView<real> &S, const PotConst &P, const SpinPhaseArgs &A,
                              hipStream_t st) {
  const long threads = (long)(A.end - A.begin) * LANES;
  const int nb = (int)((threads + kBlock - 1) / kBlock);
  const bool lg = P.langevin != 0, an = P.aniso_on != 0;
  if (lg && an) hipLaunchKernelGGL((k_spin_phase<real, true, true, LANES, MLP>), dim3(nb), dim3(kBlock), 0, st, S, P, A);
  else if (lg) hipLaunchKernelGGL((k_spin_phase<real, true, false, LANES, MLP>), dim3(nb), dim3(kBlock), 0, st, S, P, A);
  else if (an) hipLaunchKernelGGL((k_spin_phase<real, false, true, LANES, MLP>), dim3(nb), dim3(kBlock), 0, st, S, P, A);
  else hipLaunchKernelGGL((k_spin_phase<real, false, false, LANES, MLP>), dim3(nb), dim3(kBlock), 0, st, S, P, A);
}

template <typename real, int LANES>
static void spin_phase_lanes(const SysView<real> &S, const PotConst &P, const SpinPhaseArgs &A,
                             hipStream_t st) {
  if (P.soc_on) spin_phase_lanes2<real, LANES, 4>(S, P, A, st);
  else if (S.jc) spin_phase_lanes2<real, LANES, 3>(S, P, A, st);
  else if (sizeof(real) == 4 && S.spl.t) spin_phase_lanes2<real, LANES, (sizeof(real) == 4 ? 2 : 0)>(S, P, A, st);
  else if (sizeof(real) == 4 && S.tab) spin_phase_lanes2<real, LANES, (sizeof(real) == 4 ? 1 : 0)>(S, P, A, st);
  else spin_phase_lanes2<real, LANES, 0>(S, P, A, st);
}

template <typename real>
void launch_spin_phase(const SysView<real> &S, const PotConst &P, const SpinPhaseArgs &A,
                       int lanes, hipStream_t st) {
  if (A.end - A.begin <= 0) return;
  switch (lanes) {
    case 1: spin_phase_lanes<real, 1>(S, P, A, st); break;
    case 2: spin_phase_lanes<real, 2>(S, P, A, st); break;
    case 8: spin_phase_lanes<real, 8>(S, P, A, st); break;
    default: spin_phase_lanes<real, 4>(S, P, A, st); break;
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

template <typename real, int LANES, int MLP>
static void force_lanes2(const SysView<real> &S, const PotConst &P, const ForceArgs &A,
                         hipStream_t st) {
  const long threads = (long)S.n * LANES;
  const int nb = (int)((threads + kBlock - 1) / kBlock);
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
  if (P.soc_on) force_lanes2<real, LANES, 4>(S, P, A, st);
  else if (sizeof(real) == 4 && S.spl.t) force_lanes2<real, LANES, (sizeof(real) == 4 ? 2 : 0)>(S, P, A, st);
  else if (sizeof(real) == 4 && S.tab) force_lanes2<real, LANES, (sizeof(real) == 4 ? 1 : 0)>(S, P, A, st);
  else force_lanes2<real, LANES, 0>(S, P, A, st);
}

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

void launch_reduce8(const double *partial, int nb, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce8, dim3(1), dim3(256), 0, st, partial, nb, out);
}

template void launch_spin_phase<double>(const SysView<double> &, const PotConst &,
                                        const SpinPhaseArgs &, int, hipStream_t);
template void launch_spin_phase<float>(const SysView<float> &, const PotConst &,
                                       const SpinPhaseArgs &, int, hipStream_t);
template void launch_spin_tail<double>(const SysView<double> &, const PotConst &,
                                       const TailArgs &, int, hipStream_t);
template void launch_spin_tail<float>(const SysView<float> &, const PotConst &, const TailArgs &,
                                      int, hipStream_t);
template void launch_force<double>(const SysView<double> &, const PotConst &, const ForceArgs &,
                                   int, hipStream_t);
template void launch_force<float>(const SysView<float> &, const PotConst &, const ForceArgs &, int,
                                  hipStream_t);

}  // namespace sl
