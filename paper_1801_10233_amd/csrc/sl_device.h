// sl_device.h -- device-side helpers and kernel argument blocks of the
// gfx950 spin-lattice library. Layout in HBM: one array per component
// (structure of arrays) in the library's internal atom order, which groups
// atoms by colour class and, inside a class, by cell; neighbour lists are
// ELL blocks, entry k of atom i at nbr[k * ld + i] so that a wavefront
// reading entry k of 64 consecutive atoms makes one coalesced access.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sl {

// Physical constants (CODATA 2018).
constexpr double kHbar = 6.582119569e-4;       // eV ps
constexpr double kKb = 8.617333262e-5;         // eV/K
constexpr double kMuB = 5.7883818060e-5;       // eV/T
constexpr double kMvv2e = 1.0364269652680506e-4;  // eV per amu A^2/ps^2

constexpr double kInf = 1e300;     // "no watched pair" distance squared
constexpr int kMaxRep = 4;        // consecutive updates one spin launch can do
// Workgroup of the spin phase: one wavefront. A class of 108 000 atoms at one
// lane per atom is 1688 wavefronts; in 256-thread groups the 422 groups
// leave 166 CUs with two and 90 with one, in single-wave groups every CU gets
// six or seven (2.6 % faster per step at 432 000 atoms).
constexpr int kSpinBlock = 64;
constexpr int kSpinChunk = 4;     // neighbours per lane gathered together (spin phase)
// Neighbours per lane gathered together in the force gather. With
// displacement-ordered rows 4 beats 8 (117 against 128 us per launch at
// 432 000 atoms: fewer registers, more waves in flight) and 16 (195 us).
#ifndef SL_FORCE_CHUNK
#define SL_FORCE_CHUNK 4
#endif
constexpr int kForceChunk = SL_FORCE_CHUNK;
#ifndef SL_FORCE_WAVES
#define SL_FORCE_WAVES 1
#endif
constexpr int kForceWaves = SL_FORCE_WAVES;  // minimum waves per SIMD asked of the force kernel
constexpr int kBlock = 256;       // threads per block of the per-atom kernels
constexpr int kBatchBlock = 512;  // threads of the workgroup that runs one replica

// Sticky device error bits.
enum : int { kErrNbrOverflow = 1, kErrNonFinite = 2, kErrColour = 4 };

// Interaction constants, precomputed on the host.
struct PotConst {
  int morse_on;
  double mD, mA, mR0, mRc2;
  double mMc, mdMc, mRc;  // shifted-force offsets M(rc), M'(rc); 0 if plain
  int ex_on;
  double eA4, eG, eInvD2, eRc2, eA8InvD2;  // 4 alpha, gamma, 1/delta^2, rc^2, 8 alpha/delta^2
  // shifted exchange J(r) - eJc - (r^2 - rc^2) eJq, derivative J'(r) - r eJr,
  // eJc = J(rc), eJq = J'(rc)/(2 rc), eJr = J'(rc)/rc; all three 0 when off
  double eJc, eJq, eJr;
  double zw[3];       // g mu_B B / hbar, rad/ps
  double zB[3];       // g mu_B B, eV (energy)
  double aK;          // K, eV
  double aK2h;        // 2K/hbar
  double an[3];
  int aniso_on;
  int aniso_split;    // symmetric anisotropy split of the update (no bath)
  int langevin;
  double lam, lamfac;  // lambda, 1/(1+lambda^2)
  int lat_on;          // lattice bath
  double lat_g;        // gamma_L, amu/ps
  double lat_kT;       // k_B T_L, eV
  // spin-orbit pair terms (Neel g1 and DMI magnitude, Bethe-Slater form:
  // 4 alpha, gamma, 1/delta^2, rc^2, 8 alpha/delta^2) and the DMI axis
  int soc_on;
  double nA4, nG, nInvD2, nRc2, nA8InvD2;
  double dA4, dG, dInvD2, dRc2, dA8InvD2;
  double dn[3];
  // embedded-atom terms (Finnis-Sinclair form): F(rho) = -A sqrt(rho),
  // f(r) = (r-d)^2 + beta (r-d)^3/d for r < d, phi(r) = (r-c)^2 (c0 + c1 r +
  // c2 r^2) for r < c
  int eam_on;
  double fA, fd, fbeta, fc, fc0, fc1, fc2, fd2, fcc2;  // fd2 = d^2, fcc2 = c^2
};

// One FMA a*b + c as a three-operand VOP3 instruction. Written as a plain
// fma, the Horner steps below come out as a copy of the loop-invariant
// coefficient into the destination plus the two-operand form, two
// instructions per step.
__device__ __forceinline__ double fma3(double a, double b, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}

// e^x in FP64 by Cody and Waite's range reduction, x = k ln2 + t with
// |t| <= ln2/2 (ln2 split into a high part with 11 trailing zero bits, so
// k ln2_hi is exact, and a low part), the Taylor series of e^t to degree 13
// (truncation error below 5e-18 relative), and the scaling by 2^k. Without
// the library's range checks it is about 20 instructions; the clamp to
// [-746, 710] keeps the result 0 or inf where e^x underflows or overflows
// (a NaN argument comes out finite: the pair terms carry it on through r).
// Within 1 ulp of the C library's exp over [-700, 10] (2e7 random arguments).
__device__ __forceinline__ double exp_cw(double x) {
  x = fmin(fmax(x, -746.0), 710.0);
  const double k = rint(x * 1.4426950408889634074);
  double t = fma(-k, 6.93147180369123816490e-01, x);
  t = fma(-k, 1.90821492927058770002e-10, t);
  double p = fma3(1.0 / 6227020800.0, t, 1.0 / 479001600.0);
  p = fma3(p, t, 1.0 / 39916800.0);
  p = fma3(p, t, 1.0 / 3628800.0);
  p = fma3(p, t, 1.0 / 362880.0);
  p = fma3(p, t, 1.0 / 40320.0);
  p = fma3(p, t, 1.0 / 5040.0);
  p = fma3(p, t, 1.0 / 720.0);
  p = fma3(p, t, 1.0 / 120.0);
  p = fma3(p, t, 1.0 / 24.0);
  p = fma3(p, t, 1.0 / 6.0);
  p = fma(p, t, 0.5);
  p = fma(p, t, 1.0);
  p = fma(p, t, 1.0);
  return ldexp(p, (int)k);
}
// e^x of the pair terms: exp_cw in FP64, the library's expf in FP32.
__device__ __forceinline__ double exp_pair(double x) { return exp_cw(x); }
__device__ __forceinline__ float exp_pair(float x) { return expf(x); }

// Exchange J(r) at r^2 < rc^2 (Eq. BSfunction), less the shift in r^2 (its
// constants are 0 unless the shifted form is on, so the plain form's value is
// unchanged bit for bit). `real` sets the precision of the exp.
template <typename real>
__device__ __forceinline__ real exch_J(const PotConst &P, double r2) {
  const real u = (real)(r2 * P.eInvD2);
  const real J = (real)P.eA4 * u * ((real)1 - (real)P.eG * u) * exp_pair(-u);
  return J - ((real)P.eJc + (real)(r2 - P.eRc2) * (real)P.eJq);
}

// Key tag of the lattice-noise Philox stream (key = seed ^ tag).
constexpr uint64_t kLatticeKeyTag = 0x6C61747469636521ull;

// Per-system geometry and arrays (device pointers).
// Learned pair potential as a cubic Hermite spline of the network's raw
// outputs (y0, y0', y1, y1') tabulated at r0 + k dr, k = 0..last. The
// interpolant's derivative is exact, so forces are the gradient of the
// energy that is reported (the dynamics conserve it).
struct SplineView {
  const float4 *t;   // null: no spline
  float r0, dr, idr;
  int last;
  float sJ, sP;      // output scales
  float y1c, d1c;    // raw y1(rc), y1'(rc) (shifted-force constants)
  float exrc, rc;    // cuts of J (Heaviside) and phi
  int jshift;        // J in shifted-force form at exrc (the potential's ex_shift)
  float y0c, d0c;    // raw y0(exrc), y0'(exrc) of the spline
};

// (J, J', phi, phi') at r from the spline (cut and shifted-force rules as
// for the network itself).
__device__ __forceinline__ float4 spline_phys(const SplineView &s, float r) {
  float u = (r - s.r0) * s.idr;
  u = fminf(fmaxf(u, 0.0f), (float)s.last);
  const int k = min((int)u, s.last - 1);
  const float x = u - (float)k, x2 = x * x, x3 = x2 * x;
  const float4 a = s.t[k], b = s.t[k + 1];
  const float h00 = 2.0f * x3 - 3.0f * x2 + 1.0f, h10 = x3 - 2.0f * x2 + x;
  const float h01 = 3.0f * x2 - 2.0f * x3, h11 = x3 - x2;
  const float g00 = 6.0f * (x2 - x), g10 = 3.0f * x2 - 4.0f * x + 1.0f, g11 = 3.0f * x2 - 2.0f * x;
  const float y0 = h00 * a.x + h01 * b.x + s.dr * (h10 * a.y + h11 * b.y);
  const float d0 = g00 * (a.x - b.x) * s.idr + g10 * a.y + g11 * b.y;
  const float y1 = h00 * a.z + h01 * b.z + s.dr * (h10 * a.w + h11 * b.w);
  const float d1 = g00 * (a.z - b.z) * s.idr + g10 * a.w + g11 * b.w;
  float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
  if (r < s.exrc) {
    o.x = s.jshift ? s.sJ * (y0 - s.y0c - (r * r - s.exrc * s.exrc) * s.d0c / (2.0f * s.exrc))
                   : s.sJ * y0;
    o.y = s.jshift ? s.sJ * (d0 - r * s.d0c / s.exrc) : s.sJ * d0;
  }
  if (r < s.rc) {
    o.z = s.sP * (y1 - s.y1c - (r - s.rc) * s.d1c);
    o.w = s.sP * (d1 - s.d1c);
  }
  return o;
}

template <typename real>
struct SysView {
  int n;          // atoms
  int ld;         // leading dimension of the ELL lists (>= n, padded)
  int kcap;       // slots per ELL row (list capacity)
  double L[3], invL[3];
  const double *rx, *ry, *rz;  // positions used by this launch
  real *sx, *sy, *sz;          // spins
  const int *nbr;              // ELL neighbour indices
  const int *nspin, *nall;     // segment lengths
  const int *id;               // user id of each internal atom
  const float4 *tab;           // learned-potential table (J, J', phi, phi') per
                               // list entry at these positions, or null
  SplineView spl;              // learned potential as a spline (spl.t null: unused)
  const real *jc;              // exchange coefficients J(r_ij) per spin-segment
                               // entry at these positions, or null
  double *eam;                 // embedded-atom terms of these positions:
                               // F'(rho_i) at [i], F(rho_i) at [ld + i]
  int held;                    // force launches: atoms [0, held) take their spin
                               // at [n + i], the state at this step boundary, held
                               // there by a spin launch that went on to the next
                               // step's first update of their class (0: none)
};

struct SpinPhaseArgs {
  int begin, end;             // atoms [begin, end) = one colour class
  int nrep;                   // consecutive updates of this class (1..4)
  double h;                   // dt/4 (signed)
  double amp;                 // sqrt(2 D_S / |h|), noise amplitude
  int64_t step[kMaxRep];      // step counter of each update
  int sub[kMaxRep];           // sub-update index 0..3 of each update
  uint64_t seed;
  uint32_t replica;
  double rs2;                 // exchange cutoff squared
  int keep;                   // nrep 2: store the spin after the first update at
                              // [n + i] (the step-boundary state the force reads)
};

// Sectored (or serial) ordering: keys of the per-step sort and one class of a
// sectored sweep.
struct SectKeyArgs {
  int n;
  const double *rx, *ry, *rz;
  double L[3];
  int g[3], nproc;
  int serial;                 // 1: one class, one subdomain (id order)
  const int *id;
  unsigned long long *keys;   // out: (bin << 32) | id
  int *vals;                  // out: internal index
  int *count;                 // [nbins + 1], zeroed before the launch
};

struct SectPhaseArgs {
  int cls, nproc, backward;
  const int *off;             // [nbins + 1] bin offsets into order
  const int *order;           // internal indices sorted by (bin, id)
  double h, amp, rs2;
  int64_t step;
  int sub;
  uint64_t seed;
  uint32_t replica;
};

// Fused run of small colour classes (one workgroup).
constexpr int kMaxTail = 16;
constexpr int kTailBlock = 512;   // 2 waves per SIMD: room for 256 VGPRs, no spills
struct TailItem {
  int begin, end, nrep;
  int64_t step[kMaxRep];
  int sub[kMaxRep];
};
struct TailArgs {
  int nitems;
  TailItem item[kMaxTail];
  double h, amp;
  uint64_t seed;
  uint32_t replica;
  double rs2;
};

struct ForceArgs {
  int mode;                   // bit 1: final kick, 2: next kick + drift, 4: energy
  double dt;
  double ftm2v;               // 1/kMvv2e
  const double *mass;
  double *vx, *vy, *vz;
  double *nx, *ny, *nz;       // next positions (drift target)
  const double *bx, *by, *bz; // positions at the last build
  double *partial;            // [nblocks][8] energy and M partial sums
  unsigned long long *dslot;  // [3] device max of |r - r_build| and |v|, min of
                              // the watched squared distance (bits)
  unsigned int *done;         // block completion counter
  double *host_out;           // pinned host: {dmax, vmax, err, marker, wmin^2}
  const unsigned long long *wmask;  // per atom: bit k set when spin-segment
                                    // slot k holds a same-colour (watched) pair
  int *err;                   // sticky error word (device)
  int frozen;
  uint64_t seed;              // Philox seed and replica of the lattice noise
  uint32_t replica;
  int64_t step;               // step whose drift this launch computes
  double *pred;               // [blocks][3] per-block rebuild predictor terms:
                              // max |r - r_build|, max |v|, min watched r^2
  double *fp;                 // [4][ld] split force: pair force x, y, z and the
                              // pair energy of each atom, written by the pair
                              // pass and added by the spin pass
  const int2 *tiles;          // [ntiles] atom range [x, y) of each block, or
  int ntiles;                 // null: blocks cover the atom order in tiles
};

enum : int { kModeFinal = 1, kModeNext = 2, kModeEnergy = 4 };

// One replica of a batch, as seen by the persistent kernel.
constexpr int kMaxClass = 32;
template <typename real>
struct RepDesc {
  SysView<real> V[2];          // views with position buffer 0 / 1
  PotConst P;
  ForceArgs F;                 // mass, velocities, reference positions, error word
  int K;
  int off[kMaxClass + 1];      // class offsets
  int pos;                     // buffer holding the positions of the current boundary
  int64_t step, target;
  double dt, h, amp, rs2, thr;
  uint64_t seed;
  uint32_t replica;
  int user_list;
  // rebuild predictor terms (max |r - r_build|, max |v|, dt of the step)
  // of the current boundary and of the one before, and whether a rebuild
  // happened at the current boundary after its terms were taken
  double cur_dm, cur_vm, cur_dt, prev_dm, prev_vm, prev_dt;
  double cur_wm, prev_wm;      // closest watched same-colour distance squared
  double wr;                   // colour radius (watched distance after a rebuild)
  double ex_rc;                // exchange cutoff
  int cur_rebuilt, prev_rebuilt, have_prev;
  int stopped;                 // out: the step at `step` needs a rebuild first
  double *ring;                // pinned host predictor slots [4][8] (phase mode)
};

// One launch of the phase-batched mode: every replica's share of colour
// phase p of a spin half-step, or of a force pass. Replica r (K_r classes)
// visits class p for p < K_r - 1, its last class twice in a row at
// p = K_r - 1 and class K_r - 2 - (p - Kmax) for p >= Kmax; any other phase
// leaves it idle, so each replica keeps its own forward/backward order.
struct BatchPhase {
  int p, Kmax;
  int half;   // spin: 0 first half-step (boundary positions), 1 second
  int kk;     // steps since the call started: replica step = step + kk
  int after;  // force: 1 at the boundary after step kk, 0 at the call start
};

// -------------------------------------------------------------------------
// Block index -> work tile. Consecutive blocks are dispatched round robin
// over the 8 XCDs, each with its own L2; remap so that every XCD receives a
// contiguous range of tiles (spatially adjacent atoms share neighbours, so
// their gathers hit the same L2).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int nx = 8;
  int x = b % nx, k = b / nx;
  int q = nb / nx, r = nb % nx;
  return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ double min_image(double d, double L, double invL) {
  return d - L * rint(d * invL);
}

// 1/sqrt(x), x > 0, to about one ulp in FP64: the hardware estimate
// (relative error near 2^-23) refined by two Newton steps
// y <- y + (y/2)(1 - x y^2), each of which squares the relative error.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  return y;
}

// -------------------------------------------------------------------------
// Spin-orbit pair terms (appendix A) of one pair, d = r_i - r_j, r2 = |d|^2:
//   Neel: E = -g1(r) [(e.s_i)(e.s_j) - s_i.s_j/3]
//   DMI:  E = D_ij.(s_i x s_j), D_ij = dm(r) (n x e_ij), e_ij = -d/r
// with g1 and dm of the Bethe-Slater form. soc_field adds the pair's share
// of hbar omega_i (-dE/ds_i, a function of s_j only); soc_force adds
// -dE/dr_i and returns E.
template <typename real>
__device__ __forceinline__ void soc_field(const PotConst &P, double dxd, double dyd, double dzd,
                                          double r2d, real sx, real sy, real sz, real &hx,
                                          real &hy, real &hz) {
  const real dx = (real)dxd, dy = (real)dyd, dz = (real)dzd;
  if (r2d < P.nRc2) {
    const real u = (real)(r2d * P.nInvD2);
    const real g1 = (real)P.nA4 * u * ((real)1 - (real)P.nG * u) * exp(-u);
    const real t = g1 * (dx * sx + dy * sy + dz * sz) / (real)r2d;
    const real th = g1 / (real)3;
    hx += t * dx - th * sx;
    hy += t * dy - th * sy;
    hz += t * dz - th * sz;
  }
  if (r2d < P.dRc2) {
    const real u = (real)(r2d * P.dInvD2);
    const real dm = (real)P.dA4 * u * ((real)1 - (real)P.dG * u) * exp(-u);
    const real f = -dm * (real)(1.0 / sqrt(r2d));
    const real n0 = (real)P.dn[0], n1 = (real)P.dn[1], n2 = (real)P.dn[2];
    const real Dx = f * (n1 * dz - n2 * dy), Dy = f * (n2 * dx - n0 * dz), Dz = f * (n0 * dy - n1 * dx);
    hx += Dy * sz - Dz * sy;
    hy += Dz * sx - Dx * sz;
    hz += Dx * sy - Dy * sx;
  }
}

template <typename real>
__device__ __forceinline__ real soc_force(const PotConst &P, double dxd, double dyd, double dzd,
                                          double r2d, real six, real siy, real siz, real sjx,
                                          real sjy, real sjz, real &fx, real &fy, real &fz) {
  const real dx = (real)dxd, dy = (real)dyd, dz = (real)dzd, r2 = (real)r2d;
  const real rinv = (real)(1.0 / sqrt(r2d)), r = r2 * rinv;
  real en = 0;
  if (r2d < P.nRc2) {
    const real u = (real)(r2d * P.nInvD2), eu = exp(-u);
    const real g1 = (real)P.nA4 * u * ((real)1 - (real)P.nG * u) * eu;
    const real dg1 = (real)P.nA8InvD2 * r * eu *
                     ((real)1 - ((real)1 + (real)2 * (real)P.nG) * u + (real)P.nG * u * u);
    const real a = six * dx + siy * dy + siz * dz, b = sjx * dx + sjy * dy + sjz * dz;
    const real c = six * sjx + siy * sjy + siz * sjz;
    const real ang = a * b / r2 - c / (real)3;
    const real kr = dg1 * rinv * ang - (real)2 * g1 * a * b / (r2 * r2);
    const real kb = g1 / r2;
    fx += kr * dx + kb * (six * b + sjx * a);
    fy += kr * dy + kb * (siy * b + sjy * a);
    fz += kr * dz + kb * (siz * b + sjz * a);
    en -= g1 * ang;
  }
  if (r2d < P.dRc2) {
    const real u = (real)(r2d * P.dInvD2), eu = exp(-u);
    const real dm = (real)P.dA4 * u * ((real)1 - (real)P.dG * u) * eu;
    const real ddm = (real)P.dA8InvD2 * r * eu *
                     ((real)1 - ((real)1 + (real)2 * (real)P.dG) * u + (real)P.dG * u * u);
    const real n0 = (real)P.dn[0], n1 = (real)P.dn[1], n2 = (real)P.dn[2];
    const real Xx = siy * sjz - siz * sjy, Xy = siz * sjx - six * sjz, Xz = six * sjy - siy * sjx;
    const real Yx = Xy * n2 - Xz * n1, Yy = Xz * n0 - Xx * n2, Yz = Xx * n1 - Xy * n0;
    const real dY = dx * Yx + dy * Yy + dz * Yz;
    const real kr = (ddm * rinv - dm / r2) * dY * rinv, ky = dm * rinv;
    fx += kr * dx + ky * Yx;
    fy += kr * dy + ky * Yy;
    fz += kr * dz + ky * Yz;
    en -= dm * rinv * dY;
  }
  return en;
}

// -------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): a 10-round bijection
// of a 128-bit counter under a 64-bit key.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    uint32_t lo0 = M0 * c[0], hi0 = __umulhi(M0, c[0]);
    uint32_t lo1 = M1 * c[2], hi1 = __umulhi(M1, c[2]);
    uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += W0; k1 += W1;
  }
}

// Three standard normals for one spin update: counter (atom id, step lo,
// step hi, replica<<2|sub), key (seed lo, seed hi); u = (x + 1/2) 2^-32 and
// Box-Muller on (u0, u1) and (u2, u3).
__device__ __forceinline__ void gauss3(uint64_t seed, uint32_t id, int64_t step,
                                       uint32_t replica, int sub, double g[3]) {
  uint32_t c[4] = {id, (uint32_t)((uint64_t)step & 0xffffffffu),
                   (uint32_t)((uint64_t)step >> 32), (replica << 2) | (uint32_t)(sub & 3)};
  philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  const double s = 1.0 / 4294967296.0;
  const double twopi = 6.283185307179586;
  double u0 = ((double)c[0] + 0.5) * s, u1 = ((double)c[1] + 0.5) * s;
  double u2 = ((double)c[2] + 0.5) * s, u3 = ((double)c[3] + 0.5) * s;
  double ra = sqrt(-2.0 * log(u0)), rb = sqrt(-2.0 * log(u2));
  double sn, cs;
  sincos(twopi * u1, &sn, &cs);
  g[0] = ra * cs;
  g[1] = ra * sn;
  g[2] = rb * cos(twopi * u3);
}

__device__ __forceinline__ void gauss3(uint64_t seed, uint32_t id, int64_t step,
                                       uint32_t replica, int sub, float g[3]) {
  uint32_t c[4] = {id, (uint32_t)((uint64_t)step & 0xffffffffu),
                   (uint32_t)((uint64_t)step >> 32), (replica << 2) | (uint32_t)(sub & 3)};
  philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  const float s = 2.3283064365386963e-10f;
  const float twopi = 6.2831853071795865f;
  float u0 = ((float)(c[0] >> 8) + 0.5f) * (s * 256.0f);
  float u1 = ((float)(c[1] >> 8) + 0.5f) * (s * 256.0f);
  float u2 = ((float)(c[2] >> 8) + 0.5f) * (s * 256.0f);
  float u3 = ((float)(c[3] >> 8) + 0.5f) * (s * 256.0f);
  float ra = sqrtf(-2.0f * logf(u0)), rb = sqrtf(-2.0f * logf(u2));
  float sn, cs;
  sincosf(twopi * u1, &sn, &cs);
  g[0] = ra * cs;
  g[1] = ra * sn;
  g[2] = rb * cosf(twopi * u3);
}

// -------------------------------------------------------------------------
// Wavefront (64 lanes) and block reductions.
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

__device__ __forceinline__ double wave_min(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o, 64));
  return x;
}

}  // namespace sl
