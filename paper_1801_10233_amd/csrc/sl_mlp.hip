// sl_mlp.hip -- per-pair learned potential on gfx950 BF16 matrix cores.
//
// Network (5378 parameters): r -> 16 Gaussian RBF -> silu(64) -> silu(64)
// -> 2 raw outputs y = (y0, y1); physical outputs
//   J(r)   = sJ y0(r)                          for r < ex_rc (Heaviside)
//   phi(r) = sP [y1(r) - y1(rc) - (r - rc) y1'(rc)]   for r < rc (shifted force)
// plus their r-derivatives, carried through the network as a forward-mode
// tangent stream that shares every weight tile with the value stream.
//
// One wavefront evaluates 32 pairs per tile with v_mfma_f32_32x32x16_bf16
// (FP32 accumulation): layer 1 is W1[64x16] . B[16 x 32 pairs] (two 32-row
// tiles), layer 2 is W2[64x64] . A1[64 x 32 pairs] (two row tiles x four
// K blocks), each for the value and the tangent. Results come out of the
// MFMA with the lane index on the pair and the register index on the hidden
// unit; the layer-2 weights are stored with their columns permuted so that
// those registers are directly the layer-2 B operand (no LDS transpose).
// Layer 3 (2 outputs) is a VALU dot product plus one cross-half shuffle.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/spinlat.h"
#include "sl_device.h"
#include "sl_kernels.h"
#include "sl_mlp.h"

namespace sl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Row of the 32x32 MFMA result held by lane half h in register v.
__device__ __forceinline__ int c_row(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

// Layer-1 hidden unit that sits in B slot (kb, h, e) of layer 2.
__host__ __device__ inline int l2_unit(int kb, int h, int e) {
  return 32 * (kb >> 1) + 16 * (kb & 1) + 8 * (e >> 2) + 4 * h + (e & 3);
}

// Logistic sigmoid with the hardware reciprocal (about 1 ulp): the IEEE
// division took ten instructions per unit, the largest share of the VALU
// work of the per-pair network (the result feeds BF16 operands).
__device__ __forceinline__ float sigm(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

// silu(z) = z s and its derivative s + z s (1 - s) = s + a - a s, s = sigm(z).
__device__ __forceinline__ void silu_d(float z, float &a, float &da) {
  const float s = sigm(z);
  a = z * s;
  da = fmaf(-a, s, s + a);
}

// Swizzle FP32 master parameters (layout W1[64x16], c1, W2[64x64], c2,
// W3[2x64], c3) into the MFMA operand layout.
__global__ void k_mlp_swizzle(const float *p, MlpDevWeights *w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const float *W1 = p, *c1 = W1 + 64 * 16, *W2 = c1 + 64, *c2 = W2 + 64 * 64;
  const float *W3 = c2 + 64, *c3 = W3 + 2 * 64;
  if (t < 2 * 64 * 8) {  // W1s[tile][lane][e] = W1[32 tile + lane%32][8 (lane/32) + e]
    const int tile = t / 512, l = (t / 8) % 64, e = t % 8;
    w->W1s[tile][l][e] = (__bf16)W1[(32 * tile + (l & 31)) * 16 + 8 * (l >> 5) + e];
  }
  if (t < 2 * 4 * 64 * 8) {  // W2s[tile][kb][lane][e] = W2[32 tile + lane%32][unit(kb, h, e)]
    const int tile = t / 2048, kb = (t / 512) % 4, l = (t / 8) % 64, e = t % 8;
    w->W2s[tile][kb][l][e] = (__bf16)W2[(32 * tile + (l & 31)) * 64 + l2_unit(kb, l >> 5, e)];
  }
  if (t < 64) {
    w->c1[t] = c1[t];
    w->c2[t] = c2[t];
    w->W3[0][t] = W3[t];
    w->W3[1][t] = W3[64 + t];
  }
  if (t < 2) w->c3[t] = c3[t];
}

// Raw outputs (y0, y0', y1, y1') of the pair held by this lane's column.
// All 64 lanes must call it; lanes j and j+32 evaluate the same pair.
__device__ __forceinline__ float4 mlp_tile(const MlpDevWeights &w, const MlpCfgDev &c, float r) {
  const int l = threadIdx.x & 63, h = l >> 5;
  // An opaque zero added to the bias and layer-3 indices: it keeps those LDS
  // reads inside the caller's tile loop. Hoisted out of it they held 128
  // registers per lane and left one wave per SIMD.
  int lo = 0;
  asm volatile("" : "+s"(lo));
  // lane half h holds rows 8q + 4h + (0..3) of each 32-row tile (c_row):
  // float4 q of tile t sits at float4 index 8t + 2q + h
  const float4 *c1p = (const float4 *)w.c1 + h + lo, *c2p = (const float4 *)w.c2 + h + lo;
  const float4 *w30 = (const float4 *)w.W3[0] + h + lo, *w31 = (const float4 *)w.W3[1] + h + lo;
  bf16x8 bv, bd;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float x = (r - (float)(8 * h + e) * c.mu_step) * c.inv_sigma;
    const float b = __expf(-x * x);
    bv[e] = (__bf16)b;
    bd[e] = (__bf16)(b * (-2.0f * x * c.inv_sigma));
  }
  f32x16 z1[2], d1[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const bf16x8 a = *(const bf16x8 *)&w.W1s[t][l][0];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 b = c1p[8 * t + 2 * q];
      z1[t][4 * q] = b.x; z1[t][4 * q + 1] = b.y; z1[t][4 * q + 2] = b.z; z1[t][4 * q + 3] = b.w;
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) d1[t][v] = 0.0f;
    z1[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv, z1[t], 0, 0, 0);
    d1[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bd, d1[t], 0, 0, 0);
  }
  // silu and its tangent; registers become the layer-2 B operands
  bf16x8 av[4], ad[4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float a, da;
      silu_d(z1[t][v], a, da);
      const int kb = 2 * t + (v >> 3), e = v & 7;
      av[kb][e] = (__bf16)a;
      ad[kb][e] = (__bf16)(da * d1[t][v]);
    }
  f32x16 z2[2], d2[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 b = c2p[8 * t + 2 * q];
      z2[t][4 * q] = b.x; z2[t][4 * q + 1] = b.y; z2[t][4 * q + 2] = b.z; z2[t][4 * q + 3] = b.w;
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) d2[t][v] = 0.0f;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const bf16x8 a = *(const bf16x8 *)&w.W2s[t][kb][l][0];
      z2[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, av[kb], z2[t], 0, 0, 0);
      d2[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, ad[kb], d2[t], 0, 0, 0);
    }
  }
  float y0 = 0.f, y1 = 0.f, dy0 = 0.f, dy1 = 0.f;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 u0 = w30[8 * t + 2 * q], u1 = w31[8 * t + 2 * q];
      const float a0[4] = {u0.x, u0.y, u0.z, u0.w}, a1[4] = {u1.x, u1.y, u1.z, u1.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float a2, da2;
        silu_d(z2[t][4 * q + e], a2, da2);
        da2 *= d2[t][4 * q + e];
        y0 += a0[e] * a2;
        y1 += a1[e] * a2;
        dy0 += a0[e] * da2;
        dy1 += a1[e] * da2;
      }
    }
  y0 += __shfl_xor(y0, 32, 64);
  y1 += __shfl_xor(y1, 32, 64);
  dy0 += __shfl_xor(dy0, 32, 64);
  dy1 += __shfl_xor(dy1, 32, 64);
  return make_float4(y0 + w.c3[0], dy0, y1 + w.c3[1], dy1);
}

// Physical outputs from the raw ones (cut and shifted-force rules); yc holds
// y1(rc), y1'(rc), y0(ex_rc), y0'(ex_rc).
__device__ __forceinline__ float4 mlp_physical(const MlpCfgDev &c, const float *yc, float r,
                                               float4 y) {
  float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
  if (r < c.ex_rc) {
    // shifted J: y0(r) - y0(ex_rc) - (r^2 - ex_rc^2) y0'(ex_rc) / (2 ex_rc)
    o.x = c.jshift ? c.sJ * (y.x - yc[2] - (r * r - c.ex_rc * c.ex_rc) * yc[3] / (2.0f * c.ex_rc))
                   : c.sJ * y.x;
    o.y = c.jshift ? c.sJ * (y.y - r * yc[3] / c.ex_rc) : c.sJ * y.y;
  }
  if (r < c.rc) {
    o.z = c.sP * (y.z - yc[0] - (r - c.rc) * yc[1]);
    o.w = c.sP * (y.w - yc[1]);
  }
  return o;
}

__device__ __forceinline__ void stage_weights(MlpDevWeights &dst, const MlpDevWeights *src) {
  const int n = sizeof(MlpDevWeights) / 16;
  const int4 *s = (const int4 *)src;
  int4 *d = (int4 *)&dst;
  for (int k = threadIdx.x; k < n; k += blockDim.x) d[k] = s[k];
  __syncthreads();
}

// Outputs at given distances: raw (y0, y0', y1, y1') when raw != 0, else
// (J, J', phi, phi').
__global__ __launch_bounds__(256) void k_mlp_eval(const float *r, int P, const MlpDevWeights *wg,
                                                  MlpCfgDev c, const float *yc, int raw,
                                                  float4 *out) {
  __shared__ MlpDevWeights w;
  stage_weights(w, wg);
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nwave = (gridDim.x * blockDim.x) >> 6;
  const int l = threadIdx.x & 63;
  const int ntile = (P + 31) / 32;
  for (int tile = wave; tile < ntile; tile += nwave) {
    const int p = tile * 32 + (l & 31);
    const float rv = p < P ? r[p] : c.rc;
    const float4 y = mlp_tile(w, c, rv);
    if (l < 32 && p < P) out[p] = raw ? y : mlp_physical(c, yc, rv, y);
  }
}

// Per-pair table for the dynamics: for every list entry (i, k) with j > i,
// the outputs at r_ij are written to the entry and to its mirror (j, k').
__global__ __launch_bounds__(256, 2) void k_mlp_table(MlpTableArgs A, const MlpDevWeights *wg,
                                                   MlpCfgDev c, const float *yc) {
  __shared__ MlpDevWeights w;
  stage_weights(w, wg);
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nwave = (gridDim.x * blockDim.x) >> 6;
  const int l = threadIdx.x & 63;
  const int ntile = (A.npair + 31) / 32;
  for (int tile = wave; tile < ntile; tile += nwave) {
    const int p = tile * 32 + (l & 31);
    float rv = c.rc;
    int i = 0, k = 0, j = 0;
    if (p < A.npair) {
      const int2 e = A.pairs[p];
      i = e.x;
      k = e.y;
      j = A.nbr[(size_t)k * A.ld + i];
      const double dx = min_image(A.rx[i] - A.rx[j], A.L[0], A.invL[0]);
      const double dy = min_image(A.ry[i] - A.ry[j], A.L[1], A.invL[1]);
      const double dz = min_image(A.rz[i] - A.rz[j], A.L[2], A.invL[2]);
      rv = (float)sqrt(dx * dx + dy * dy + dz * dz);
    }
    const float4 y = mlp_tile(w, c, rv);
    if (l < 32 && p < A.npair) {
      const float4 o = mlp_physical(c, yc, rv, y);
      A.tab[(size_t)k * A.ld + i] = o;
      A.tab[(size_t)A.mirror[p] * A.ld + j] = o;
    }
  }
}

void launch_mlp_swizzle(const float *p, MlpDevWeights *w, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_swizzle, dim3(16), dim3(256), 0, st, p, w);
}

static int mlp_grid(int P) {
  const int tiles = (P + 31) / 32;
  const int blocks = (tiles + 3) / 4;
  return blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096;
}

void launch_mlp_eval(const float *r, int P, const MlpDevWeights *w, const MlpCfgDev &c,
                     const float *yc, int raw, float4 *out, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_eval, dim3(mlp_grid(P)), dim3(256), 0, st, r, P, w, c, yc, raw, out);
}

// One wavefront per grid distance, lane h = hidden unit h of both layers;
// FP64 arithmetic on the FP32 master parameters (layout W1[64x16], c1,
// W2[64x64], c2, W3[2x64], c3), value and r-tangent together. Unlike the
// BF16 operand path this is smooth in r at the scale of the spline grid.
__global__ __launch_bounds__(64) void k_mlp_grid(const float *p, double r0, double dr, int P,
                                                 double sigma, double mu, float4 *out) {
  __shared__ double a1[64], t1[64];
  const int q = blockIdx.x, h = threadIdx.x;
  if (q >= P) return;
  const float *W1 = p, *c1 = W1 + 64 * 16, *W2 = c1 + 64, *c2 = W2 + 64 * 64;
  const float *W3 = c2 + 64, *c3 = W3 + 2 * 64;
  const double r = r0 + q * dr;
  double z = c1[h], dz = 0.0;
  for (int k = 0; k < 16; ++k) {
    const double x = (r - k * mu) / sigma, b = exp(-x * x);
    z += (double)W1[h * 16 + k] * b;
    dz += (double)W1[h * 16 + k] * (-2.0 * x / sigma) * b;
  }
  double s = 1.0 / (1.0 + exp(-z));
  a1[h] = z * s;
  t1[h] = s * (1.0 + z * (1.0 - s)) * dz;
  __syncthreads();
  double z2 = c2[h], dz2 = 0.0;
  for (int k = 0; k < 64; ++k) {
    z2 += (double)W2[h * 64 + k] * a1[k];
    dz2 += (double)W2[h * 64 + k] * t1[k];
  }
  s = 1.0 / (1.0 + exp(-z2));
  const double a2 = z2 * s, t2 = s * (1.0 + z2 * (1.0 - s)) * dz2;
  double y0 = W3[h] * a2, d0 = W3[h] * t2, y1 = W3[64 + h] * a2, d1 = W3[64 + h] * t2;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    y0 += __shfl_xor(y0, o, 64);
    d0 += __shfl_xor(d0, o, 64);
    y1 += __shfl_xor(y1, o, 64);
    d1 += __shfl_xor(d1, o, 64);
  }
  if (h == 0) out[q] = make_float4((float)(y0 + c3[0]), (float)d0, (float)(y1 + c3[1]), (float)d1);
}

void launch_mlp_grid(const float *params, double r0, double dr, int P, double sigma,
                     double mu_step, float4 *out, hipStream_t st) {
  if (P > 0) hipLaunchKernelGGL(k_mlp_grid, dim3(P), dim3(64), 0, st, params, r0, dr, P, sigma, mu_step, out);
}

void launch_mlp_table(const MlpTableArgs &A, const MlpDevWeights *w, const MlpCfgDev &c,
                      const float *yc, hipStream_t st) {
  if (A.npair <= 0) return;
  hipLaunchKernelGGL(k_mlp_table, dim3(mlp_grid(A.npair)), dim3(256), 0, st, A, w, c, yc);
}

}  // namespace sl

namespace sl {

// Unordered pairs of the list: entries (i, k) with j = nbr[k][i] > i, and
// for each the slot k' where i appears in the row of j.
__global__ void k_mlp_pair_count(int n, int ld, const int *nbr, const int *nall, int *cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = 0;
  for (int k = 0; k < nall[i]; ++k) c += nbr[(size_t)k * ld + i] > i;
  cnt[i] = c;
}

__global__ void k_mlp_pair_fill(int n, int ld, const int *nbr, const int *nall, const int *start,
                                int2 *pairs, int *mirror, int *err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int p = start[i];
  for (int k = 0; k < nall[i]; ++k) {
    const int j = nbr[(size_t)k * ld + i];
    if (j <= i) continue;
    int kk = -1;
    for (int q = 0; q < nall[j]; ++q)
      if (nbr[(size_t)q * ld + j] == i) { kk = q; break; }
    if (kk < 0) {  // asymmetric list: cannot mirror
      atomicOr(err, kErrNbrOverflow);
      kk = k;
    }
    pairs[p] = make_int2(i, k);
    mirror[p] = kk;
    ++p;
  }
}

void launch_mlp_pair_count(int n, int ld, const int *nbr, const int *nall, int *cnt,
                           hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_mlp_pair_count, dim3((n + 255) / 256), dim3(256), 0, st, n, ld, nbr, nall, cnt);
}

void launch_mlp_pair_fill(int n, int ld, const int *nbr, const int *nall, const int *start,
                          int2 *pairs, int *mirror, int *err, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_mlp_pair_fill, dim3((n + 255) / 256), dim3(256), 0, st, n, ld, nbr, nall, start, pairs, mirror, err);
}

}  // namespace sl

namespace sl {

__global__ void k_mlp_swizzle_t(const float *p, MlpDevWeightsT *w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const float *W2 = p + 64 * 16 + 64;
  if (t < 2 * 4 * 64 * 8) {  // W2Ts[tile][kb][lane][e] = W2[unit(kb, h, e)][32 tile + lane%32]
    const int tile = t / 2048, kb = (t / 512) % 4, l = (t / 8) % 64, e = t % 8;
    w->W2Ts[tile][kb][l][e] = (__bf16)W2[l2_unit(kb, l >> 5, e) * 64 + 32 * tile + (l & 31)];
  }
}

void launch_mlp_swizzle_t(const float *p, MlpDevWeightsT *w, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_swizzle_t, dim3(16), dim3(256), 0, st, p, w);
}

__device__ __forceinline__ float dsilu(float z, float s) { return s * (1.0f + z * (1.0f - s)); }
__device__ __forceinline__ float d2silu(float z, float s) {
  return s * (1.0f - s) * (2.0f + z * (1.0f - 2.0f * s));
}

// Per-wave LDS staging of the reverse pass, [unit][pair] in BF16 so that
// both MFMA operands of the weight-gradient products (reduction over the 32
// pairs of a tile) are 16-byte row reads.
struct BwdStage {
  __bf16 z2b[64][32], z2d[64][32];   // dL/dz2, dL/dz2' (rows: layer-2 units)
  __bf16 a1[64][32], a1d[64][32];    // a1, a1' (rows: layer-1 units)
  __bf16 z1b[64][32], z1d[64][32];   // dL/dz1, dL/dz1'
  __bf16 a2[64][32], a2d[64][32];    // a2, a2'
  __bf16 b[32][32], bd[32][32];      // RBF features and tangents (rows 16..31 zero)
  __bf16 yb[32][32], ybd[32][32];    // output adjoints (rows 0, 1; rest zero)
};

__device__ __forceinline__ bf16x8 lds8(const __bf16 *row, int k0) {
  return *(const bf16x8 *)(row + k0);
}

// Reverse pass. Each wave owns a strided set of 32-pair tiles, recomputes
// the forward with the tape kept in registers, pushes the adjoints back
// through layer 3, layer 2 (MFMA with W2^T) and the silu value/tangent
// rules, and accumulates
//   dW2 = sum_p [zbar2 a1^T + zbar2' a1'^T]      (4 tiles 32x32)
//   dW1 | dc1 = sum_p [zbar1 (b | 1)^T + zbar1' b'^T]   (2 tiles, cols 0..15 | 16)
//   dW3^T | dc2 = sum_p [a2 (ybar | 0 | 1)... ]  (2 tiles, cols 0..1 | 2)
// in MFMA accumulators; dc3 by a wave sum. The wave's partial gradient is
// written in the parameter layout at the end.
__global__ __launch_bounds__(64) void k_mlp_backward(const float *r, const float4 *ybar, int P,
                                                     const MlpDevWeights *w,
                                                     const MlpDevWeightsT *wt, MlpCfgDev c,
                                                     float *partial) {
  __shared__ BwdStage sg;
  const int l = threadIdx.x, h = l >> 5, j = l & 31;
  const int wave = blockIdx.x, nwave = gridDim.x;
  f32x16 gW2[2][2], gW1[2], gW3[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      gW2[a][0][v] = 0.f; gW2[a][1][v] = 0.f; gW1[a][v] = 0.f; gW3[a][v] = 0.f;
    }
  }
  float gc3_0 = 0.f, gc3_1 = 0.f;
  // constant rows of the staging area: zero padding and the ones row
  for (int k = l; k < 32 * 32; k += 64) {
    const int row = k / 32, col = k % 32;
    if (row >= 16) { sg.b[row][col] = (__bf16)(row == 16 ? 1.0f : 0.0f); sg.bd[row][col] = (__bf16)0.f; }
    if (row >= 2) { sg.yb[row][col] = (__bf16)0.f; sg.ybd[row][col] = (__bf16)0.f; }
  }
  const int ntile = (P + 31) / 32;
  for (int tile = wave; tile < ntile; tile += nwave) {
    const int p = tile * 32 + j;
    const bool valid = p < P;
    const float rv = valid ? r[p] : c.rc;
    const float4 yb = valid ? ybar[p] : make_float4(0.f, 0.f, 0.f, 0.f);
    // ---- forward with tape
    bf16x8 bv, bd;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float x = (rv - (float)(8 * h + e) * c.mu_step) * c.inv_sigma;
      const float b = __expf(-x * x);
      bv[e] = (__bf16)b;
      bd[e] = (__bf16)(b * (-2.0f * x * c.inv_sigma));
      sg.b[8 * h + e][j] = bv[e];
      sg.bd[8 * h + e][j] = bd[e];
    }
    f32x16 z1[2], d1[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const bf16x8 a = *(const bf16x8 *)&w->W1s[t][l][0];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        z1[t][v] = w->c1[32 * t + c_row(v, h)];
        d1[t][v] = 0.0f;
      }
      z1[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv, z1[t], 0, 0, 0);
      d1[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bd, d1[t], 0, 0, 0);
    }
    bf16x8 av[4], ad[4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float z = z1[t][v], s = sigm(z);
        const int kb = 2 * t + (v >> 3), e = v & 7;
        av[kb][e] = (__bf16)(z * s);
        ad[kb][e] = (__bf16)(dsilu(z, s) * d1[t][v]);
        const int u = 32 * t + c_row(v, h);
        sg.a1[u][j] = av[kb][e];
        sg.a1d[u][j] = ad[kb][e];
      }
    f32x16 z2[2], d2[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        z2[t][v] = w->c2[32 * t + c_row(v, h)];
        d2[t][v] = 0.0f;
      }
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const bf16x8 a = *(const bf16x8 *)&w->W2s[t][kb][l][0];
        z2[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, av[kb], z2[t], 0, 0, 0);
        d2[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, ad[kb], d2[t], 0, 0, 0);
      }
    }
    // ---- output adjoints through layer 3 and the layer-2 silu
    if (h == 0) {
      sg.yb[0][j] = (__bf16)yb.x;  // dL/dy0
      sg.yb[1][j] = (__bf16)yb.z;  // dL/dy1
      sg.ybd[0][j] = (__bf16)yb.y; // dL/dy0'
      sg.ybd[1][j] = (__bf16)yb.w; // dL/dy1'
    }
    {
      float s0 = yb.x, s1 = yb.z;
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) {
        s0 += __shfl_xor(s0, o, 64);
        s1 += __shfl_xor(s1, o, 64);
      }
      if (l == 0) { gc3_0 += s0; gc3_1 += s1; }
    }
    bf16x8 zb[4], zd[4];  // dL/dz2, dL/dz2' as B operands (layer-2 unit order)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int u = 32 * t + c_row(v, h);
        const float z = z2[t][v], s = sigm(z);
        const float a2 = z * s, da2 = dsilu(z, s) * d2[t][v];
        const float ab = w->W3[0][u] * yb.x + w->W3[1][u] * yb.z;     // dL/da2
        const float adb = w->W3[0][u] * yb.y + w->W3[1][u] * yb.w;    // dL/da2'
        const float zbar = d2silu(z, s) * d2[t][v] * adb + dsilu(z, s) * ab;
        const float zdbar = dsilu(z, s) * adb;
        const int kb = 2 * t + (v >> 3), e = v & 7;
        zb[kb][e] = (__bf16)zbar;
        zd[kb][e] = (__bf16)zdbar;
        sg.z2b[u][j] = zb[kb][e];
        sg.z2d[u][j] = zd[kb][e];
        sg.a2[u][j] = (__bf16)a2;
        sg.a2d[u][j] = (__bf16)da2;
      }
    // ---- back through layer 2: dL/da1 = W2^T dL/dz2 (and tangent)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      f32x16 g1, g1d;
#pragma unroll
      for (int v = 0; v < 16; ++v) { g1[v] = 0.f; g1d[v] = 0.f; }
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const bf16x8 a = *(const bf16x8 *)&wt->W2Ts[t][kb][l][0];
        g1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, zb[kb], g1, 0, 0, 0);
        g1d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, zd[kb], g1d, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int u = 32 * t + c_row(v, h);
        const float z = z1[t][v], s = sigm(z);
        sg.z1b[u][j] = (__bf16)(d2silu(z, s) * d1[t][v] * g1d[v] + dsilu(z, s) * g1[v]);
        sg.z1d[u][j] = (__bf16)(dsilu(z, s) * g1d[v]);
      }
    }
    __syncthreads();
    // ---- weight gradients: reductions over the 32 pairs of the tile
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int k0 = 16 * ks + 8 * h;
#pragma unroll
      for (int to = 0; to < 2; ++to) {
        const bf16x8 Az = lds8(sg.z2b[32 * to + j], k0), Azd = lds8(sg.z2d[32 * to + j], k0);
        const bf16x8 Az1 = lds8(sg.z1b[32 * to + j], k0), Az1d = lds8(sg.z1d[32 * to + j], k0);
        const bf16x8 Aa2 = lds8(sg.a2[32 * to + j], k0), Aa2d = lds8(sg.a2d[32 * to + j], k0);
#pragma unroll
        for (int ti = 0; ti < 2; ++ti) {
          const bf16x8 Ba = lds8(sg.a1[32 * ti + j], k0), Bad = lds8(sg.a1d[32 * ti + j], k0);
          gW2[to][ti] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Az, Ba, gW2[to][ti], 0, 0, 0);
          gW2[to][ti] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Azd, Bad, gW2[to][ti], 0, 0, 0);
        }
        const bf16x8 Bb = lds8(sg.b[j], k0), Bbd = lds8(sg.bd[j], k0);
        gW1[to] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Az1, Bb, gW1[to], 0, 0, 0);
        gW1[to] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Az1d, Bbd, gW1[to], 0, 0, 0);
        // dW3^T[u][o] = sum_p a2[u] ybar_o + a2'[u] ybar'_o; column 2 gives dc2
        const bf16x8 By = lds8(sg.yb[j], k0), Byd = lds8(sg.ybd[j], k0);
        gW3[to] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Aa2, By, gW3[to], 0, 0, 0);
        gW3[to] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Aa2d, Byd, gW3[to], 0, 0, 0);
      }
    }
    // dc2 = sum_p dL/dz2 lands in column 3 of the same accumulators (a B
    // operand whose column 3 is all ones).
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int k0 = 16 * ks + 8 * h;
#pragma unroll
      for (int to = 0; to < 2; ++to) {
        const bf16x8 Az = lds8(sg.z2b[32 * to + j], k0);
        bf16x8 ones;
#pragma unroll
        for (int e = 0; e < 8; ++e) ones[e] = (__bf16)(j == 3 ? 1.0f : 0.0f);
        gW3[to] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Az, ones, gW3[to], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // ---- write the partial gradient of this wave in the parameter layout
  float *g = partial + (size_t)wave * 5378;
  float *gW1p = g, *gc1p = g + 1024, *gW2p = g + 1088, *gc2p = g + 5184, *gW3p = g + 5248,
        *gc3p = g + 5376;
#pragma unroll
  for (int to = 0; to < 2; ++to)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = 32 * to + c_row(v, h);
#pragma unroll
      for (int ti = 0; ti < 2; ++ti) gW2p[row * 64 + 32 * ti + j] = gW2[to][ti][v];
      if (j < 16) gW1p[row * 16 + j] = gW1[to][v];
      if (j == 16) gc1p[row] = gW1[to][v];
      if (j < 2) gW3p[j * 64 + row] = gW3[to][v];
      if (j == 3) gc2p[row] = gW3[to][v];
    }
  if (l == 0) { gc3p[0] = gc3_0; gc3p[1] = gc3_1; }
}

int mlp_backward_waves(int P) {
  const int tiles = (P + 31) / 32;
  return tiles < 2048 ? (tiles > 0 ? tiles : 1) : 2048;
}

void launch_mlp_backward(const float *r, const float4 *ybar, int P, const MlpDevWeights *w,
                         const MlpDevWeightsT *wt, const MlpCfgDev &c, float *partial,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_backward, dim3(mlp_backward_waves(P)), dim3(64), 0, st, r, ybar, P, w,
                     wt, c, partial);
}

// grad[q] (+)= sum over waves of partial[w][q], in wave order.
__global__ void k_mlp_grad_reduce(const float *partial, int nwave, float *grad, int acc) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 5378) return;
  float s = 0.f;
  for (int w = 0; w < nwave; ++w) s += partial[(size_t)w * 5378 + q];
  grad[q] = acc ? grad[q] + s : s;
}

void launch_mlp_grad_reduce(const float *partial, int nwave, float *grad, int accumulate,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_grad_reduce, dim3((5378 + 255) / 256), dim3(256), 0, st, partial, nwave,
                     grad, accumulate);
}

// Adam on the FP32 master parameters (bias-corrected, step t >= 1).
__global__ void k_adam(float *p, float *m, float *v, const float *g, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.f - b1) * gq;
  const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

void launch_adam(float *p, float *m, float *v, const float *g, int n, float lr, float b1, float b2,
                 float eps, int t, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, p, m, v, g, n, lr, b1, b2, eps,
                     c1, c2);
}

}  // namespace sl

namespace sl {

// Per-atom force, exchange part of hbar omega and energy (pair + exchange,
// pairs halved) of the current state, from the analytic J and V or from the
// learned-potential table; with references, also the loss residual terms:
//   gF_i = 2 wF (F_i - Fref_i)/(3N),  gW_i = 2 wW (hw_i - hwref_i)/(3N),
//   lossp_i = [wF |F_i - Fref_i|^2 + wW |hw_i - hwref_i|^2]/(3N).
template <typename real, int MLP>
__global__ void k_fields(SysView<real> S, PotConst P, FieldArgs A) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  const double rix = S.rx[i], riy = S.ry[i], riz = S.rz[i];
  const double six = S.sx[i], siy = S.sy[i], siz = S.sz[i];
  double f[3] = {0, 0, 0}, hw[3] = {0, 0, 0}, e = 0.0;
  const int ld = S.ld;
  for (int k = 0; k < S.nall[i]; ++k) {
    const int j = S.nbr[(size_t)k * ld + i];
    const double dx = min_image(rix - S.rx[j], S.L[0], S.invL[0]);
    const double dy = min_image(riy - S.ry[j], S.L[1], S.invL[1]);
    const double dz = min_image(riz - S.rz[j], S.L[2], S.invL[2]);
    const double r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2);
    const double sjx = S.sx[j], sjy = S.sy[j], sjz = S.sz[j];
    const double sij = six * sjx + siy * sjy + siz * sjz;
    double J = 0, dJ = 0, V = 0, dV = 0;
    if (MLP) {
      const float4 t = MLP == 2 ? spline_phys(S.spl, (float)r) : S.tab[(size_t)k * ld + i];
      J = t.x; dJ = t.y; V = t.z; dV = t.w;
    } else {
      if (P.ex_on && r2 < P.eRc2) {
        const double u = r2 * P.eInvD2, eu = exp(-u);
        J = P.eA4 * u * (1.0 - P.eG * u) * eu;
        dJ = P.eA8InvD2 * r * eu * (1.0 - (1.0 + 2.0 * P.eG) * u + P.eG * u * u);
        J -= P.eJc + (r2 - P.eRc2) * P.eJq;
        dJ -= r * P.eJr;
      }
      if (P.morse_on && r2 < P.mRc2) {
        const double ex = exp(-P.mA * (r - P.mR0));
        V = P.mD * (ex * ex - 2.0 * ex) - P.mMc - (r - P.mRc) * P.mdMc;
        dV = -2.0 * P.mA * P.mD * (ex * ex - ex) - P.mdMc;
      }
    }
    const double c = (-dV + dJ * sij) / r;
    f[0] += c * dx; f[1] += c * dy; f[2] += c * dz;
    hw[0] += J * sjx; hw[1] += J * sjy; hw[2] += J * sjz;
    e += 0.5 * (V - J * sij);
    if (!MLP && P.eam_on) {
      // embedded-atom terms (densities from the first pass)
      if (r2 < P.fd2) {
        const double x = r - P.fd;
        const double df = 2.0 * x + 3.0 * P.fbeta * x * x / P.fd;
        const double cf = -(S.eam[i] + S.eam[j]) * df / r;
        f[0] += cf * dx; f[1] += cf * dy; f[2] += cf * dz;
      }
      if (r2 < P.fcc2) {
        const double x = r - P.fc, q = P.fc0 + P.fc1 * r + P.fc2 * r * r;
        const double dphi = 2.0 * x * q + x * x * (P.fc1 + 2.0 * P.fc2 * r);
        f[0] -= dphi * dx / r; f[1] -= dphi * dy / r; f[2] -= dphi * dz / r;
        e += 0.5 * x * x * q;
      }
    }
    if (!MLP && P.soc_on) {
      // Neel and DMI pair terms (appendix A)
      soc_field<double>(P, dx, dy, dz, r2, sjx, sjy, sjz, hw[0], hw[1], hw[2]);
      e += 0.5 * soc_force<double>(P, dx, dy, dz, r2, six, siy, siz, sjx, sjy, sjz, f[0], f[1], f[2]);
    }
  }
  const size_t n = S.n;
  if (!MLP && P.eam_on) e += S.eam[(size_t)S.ld + i];
  if (A.ts) {
    // conservative field hbar omega_i: exchange, Zeeman and anisotropy
    const double sn = P.an[0] * six + P.an[1] * siy + P.an[2] * siz;
    const double wx = hw[0] + P.zB[0] + 2.0 * P.aK * sn * P.an[0];
    const double wy = hw[1] + P.zB[1] + 2.0 * P.aK * sn * P.an[1];
    const double wz = hw[2] + P.zB[2] + 2.0 * P.aK * sn * P.an[2];
    const double cx = siy * wz - siz * wy, cy = siz * wx - six * wz, cz = six * wy - siy * wx;
    A.ts[i] = cx * cx + cy * cy + cz * cz;
    A.ts[n + i] = six * wx + siy * wy + siz * wz;
  }
  if (A.F) { A.F[i] = f[0]; A.F[n + i] = f[1]; A.F[2 * n + i] = f[2]; }
  if (A.hw) { A.hw[i] = hw[0]; A.hw[n + i] = hw[1]; A.hw[2 * n + i] = hw[2]; }
  if (A.e) A.e[i] = e;
  if (A.Fref) {
    double lf = 0.0, lw = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double R = f[a] - A.Fref[a * n + i], Q = hw[a] - A.hwref[a * n + i];
      lf += R * R;
      lw += Q * Q;
      A.gF[a * n + i] = (float)(2.0 * A.wF * R / (3.0 * n));
      A.gW[a * n + i] = (float)(2.0 * A.wW * Q / (3.0 * n));
    }
    A.lossp[i] = (A.wF * lf + A.wW * lw) / (3.0 * n);
  }
}

// Per unordered pair: adjoints of J, J', phi, phi' from the residuals, as
// raw output adjoints of the network, and the pair's share of the adjoints
// of the shifted-force constants y1(rc), y1'(rc).
__global__ void k_pair_adjoint(PairAdjArgs A) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= A.npair) return;
  const int2 e2 = A.pairs[p];
  const int i = e2.x, j = A.nbr[(size_t)e2.y * A.ld + i];
  const double dx = min_image(A.rx[i] - A.rx[j], A.L[0], A.invL[0]);
  const double dy = min_image(A.ry[i] - A.ry[j], A.L[1], A.invL[1]);
  const double dz = min_image(A.rz[i] - A.rz[j], A.L[2], A.invL[2]);
  const float r = (float)sqrt(dx * dx + dy * dy + dz * dz);
  const float ex = (float)dx / r, ey = (float)dy / r, ez = (float)dz / r;
  const size_t n = A.n;
  const float si[3] = {A.sx[i], A.sy[i], A.sz[i]}, sj[3] = {A.sx[j], A.sy[j], A.sz[j]};
  const float sij = si[0] * sj[0] + si[1] * sj[1] + si[2] * sj[2];
  float aJ = -A.dE * sij, dc = 0.f;
  const float ev[3] = {ex, ey, ez};
  for (int a = 0; a < 3; ++a) {
    aJ += A.gW[a * n + i] * sj[a] + A.gW[a * n + j] * si[a];
    dc += (A.gF[a * n + i] - A.gF[a * n + j]) * ev[a];
  }
  const float aP = A.dE, adP = -dc, adJ = dc * sij;
  float4 yb = make_float4(0.f, 0.f, 0.f, 0.f);
  float2 sh = make_float2(0.f, 0.f);
  if (r < A.ex_rc) { yb.x = aJ * A.sJ; yb.y = adJ * A.sJ; }
  if (r < A.rc) {
    yb.z = aP * A.sP;
    yb.w = adP * A.sP;
    sh.x = -aP * A.sP;
    sh.y = -(aP * A.sP * (r - A.rc) + adP * A.sP);
  }
  A.rp[p] = r;
  A.ybar[p] = yb;
  A.shift[p] = sh;
}

// Fixed-order sums (one block): out[0] = sum of x (double), or of a float2.
__global__ __launch_bounds__(256) void k_sum_d(const double *x, int n, double *out) {
  __shared__ double b[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += x[k];
  b[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) b[threadIdx.x] += b[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = b[0];
}

__global__ __launch_bounds__(256) void k_sum_f2(const float2 *x, int n, float4 *out) {
  __shared__ double b0[256], b1[256];
  double s0 = 0.0, s1 = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) { s0 += x[k].x; s1 += x[k].y; }
  b0[threadIdx.x] = s0;
  b1[threadIdx.x] = s1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) { b0[threadIdx.x] += b0[threadIdx.x + w]; b1[threadIdx.x] += b1[threadIdx.x + w]; }
    __syncthreads();
  }
  // raw adjoints of the single point r = rc: (0, 0, dL/dy1(rc), dL/dy1'(rc))
  if (threadIdx.x == 0) *out = make_float4(0.f, 0.f, (float)b0[0], (float)b1[0]);
}

template <typename real>
void launch_fields(const SysView<real> &S, const PotConst &P, const FieldArgs &A, hipStream_t st) {
  const int nb = (S.n + 255) / 256;
  if (sizeof(real) == 4 && S.spl.t) hipLaunchKernelGGL((k_fields<real, (sizeof(real) == 4 ? 2 : 0)>), dim3(nb), dim3(256), 0, st, S, P, A);
  else if (sizeof(real) == 4 && S.tab) hipLaunchKernelGGL((k_fields<real, (sizeof(real) == 4 ? 1 : 0)>), dim3(nb), dim3(256), 0, st, S, P, A);
  else hipLaunchKernelGGL((k_fields<real, 0>), dim3(nb), dim3(256), 0, st, S, P, A);
}
template void launch_fields<double>(const SysView<double> &, const PotConst &, const FieldArgs &, hipStream_t);
template void launch_fields<float>(const SysView<float> &, const PotConst &, const FieldArgs &, hipStream_t);

void launch_pair_adjoint(const PairAdjArgs &A, hipStream_t st) {
  if (A.npair > 0) hipLaunchKernelGGL(k_pair_adjoint, dim3((A.npair + 255) / 256), dim3(256), 0, st, A);
}
void launch_sum_d(const double *x, int n, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_d, dim3(1), dim3(256), 0, st, x, n, out);
}
void launch_sum_f2(const float2 *x, int n, float4 *out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_f2, dim3(1), dim3(256), 0, st, x, n, out);
}

}  // namespace sl
