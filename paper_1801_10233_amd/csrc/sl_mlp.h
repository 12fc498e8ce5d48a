// sl_mlp.h -- device structures of the per-pair MLP (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sl_device.h"

namespace sl {

// Weights in the MFMA operand layout (see sl_mlp.hip), staged to LDS.
struct __attribute__((aligned(16))) MlpDevWeights {
  __bf16 W1s[2][64][8];       // layer-1 A tiles: [row tile][lane][k]
  __bf16 W2s[2][4][64][8];    // layer-2 A tiles: [row tile][k block][lane][k]
  float c1[64], c2[64];
  float W3[2][64];
  float c3[2];
  float pad[2];
};

// Transposed layer-2 tiles for the reverse pass (A operand of W2^T).
struct __attribute__((aligned(16))) MlpDevWeightsT {
  __bf16 W2Ts[2][4][64][8];
};

struct MlpCfgDev {
  float inv_sigma, mu_step, sJ, sP, ex_rc, rc;
  int jshift;  // J in shifted-force form at ex_rc (a system's ex_shift)
};

struct MlpTableArgs {
  int npair, ld;
  const int2 *pairs;      // (i, k) list entries with j > i
  const int *mirror;      // slot k' of i in the row of j
  const int *nbr;
  const double *rx, *ry, *rz;
  double L[3], invL[3];
  float4 *tab;            // (J, J', phi, phi') per list entry
};

struct FieldArgs {
  double *F, *hw, *e;             // outputs, SoA [3][n] / [n], may be null
  const double *Fref, *hwref;     // references (internal order) or null
  double wF, wW;
  float *gF, *gW;                 // residual adjoints [3][n]
  double *lossp;                  // per-atom loss terms
  double *ts;                     // spin-temperature terms [2][n]:
                                  // |s x h_i|^2, s.h_i (h_i = hbar omega_i)
};
template <typename real>
void launch_fields(const SysView<real> &S, const PotConst &P, const FieldArgs &A, hipStream_t st);

struct PairAdjArgs {
  int npair, ld, n;
  const int2 *pairs;
  const int *nbr;
  const double *rx, *ry, *rz;
  double L[3], invL[3];
  const float *sx, *sy, *sz;
  const float *gF, *gW;
  float dE, sJ, sP, ex_rc, rc;
  float *rp;
  float4 *ybar;
  float2 *shift;
};
void launch_pair_adjoint(const PairAdjArgs &A, hipStream_t st);
void launch_sum_d(const double *x, int n, double *out, hipStream_t st);
void launch_sum_f2(const float2 *x, int n, float4 *out, hipStream_t st);

void launch_mlp_pair_count(int n, int ld, const int *nbr, const int *nall, int *cnt,
                           hipStream_t st);
void launch_mlp_pair_fill(int n, int ld, const int *nbr, const int *nall, const int *start,
                          int2 *pairs, int *mirror, int *err, hipStream_t st);
void launch_mlp_swizzle(const float *p, MlpDevWeights *w, hipStream_t st);
void launch_mlp_swizzle_t(const float *p, MlpDevWeightsT *w, hipStream_t st);
// Reverse pass over P pairs: r[P] and raw output adjoints
// (dL/dy0, dL/dy0', dL/dy1, dL/dy1') per pair; per-wave partial gradients
// (SL_MLP_NPARAM floats each) into partial[nwave][...]; returns nwave.
int mlp_backward_waves(int P);
void launch_mlp_backward(const float *r, const float4 *ybar, int P, const MlpDevWeights *w,
                         const MlpDevWeightsT *wt, const MlpCfgDev &c, float *partial,
                         hipStream_t st);
void launch_mlp_grad_reduce(const float *partial, int nwave, float *grad, int accumulate,
                            hipStream_t st);
void launch_adam(float *p, float *m, float *v, const float *g, int n, float lr, float b1,
                 float b2, float eps, int t, hipStream_t st);
void launch_mlp_eval(const float *r, int P, const MlpDevWeights *w, const MlpCfgDev &c,
                     const float *yc, int raw, float4 *out, hipStream_t st);
void launch_mlp_table(const MlpTableArgs &A, const MlpDevWeights *w, const MlpCfgDev &c,
                      const float *yc, hipStream_t st);
// Raw outputs (y0, y0', y1, y1') of the FP32 master network evaluated in
// FP64 at r0 + q dr, q = 0..P-1 (the spline table of the dynamics).
void launch_mlp_grid(const float *params, double r0, double dr, int P, double sigma,
                     double mu_step, float4 *out, hipStream_t st);

}  // namespace sl
