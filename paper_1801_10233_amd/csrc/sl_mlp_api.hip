// sl_mlp_api.hip -- C ABI of the per-pair learned potential (sl_mlp_*).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/spinlat.h"
#include "sl_mlp_host.h"

using namespace sl;

namespace {

thread_local std::string g_mlp_err;

int mfail(sl_mlp *m, int code, const std::string &msg) {
  if (m) m->last_err = msg;
  else g_mlp_err = msg;
  return code;
}

#define MCHK(m, x)                                                                   \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) return mfail((m), SL_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

extern "C" {

int sl_mlp_create(const sl_mlp_spec *spec, sl_mlp **out) {
  if (!out) return mfail(nullptr, SL_E_ARG, "out is NULL");
  *out = nullptr;
  sl_mlp *m = new sl_mlp();
  if (hipGetDevice(&m->device) != hipSuccess) m->device = 0;
  if (spec) {
    if (spec->sigma > 0) m->sigma = spec->sigma;
    if (spec->mu_step > 0) m->mu_step = spec->mu_step;
    if (spec->sJ != 0) m->sJ = spec->sJ;
    if (spec->sP != 0) m->sP = spec->sP;
    if (spec->ex_rc > 0) m->ex_rc = spec->ex_rc;
    if (spec->rc > 0) m->rc = spec->rc;
    m->st = (hipStream_t)spec->stream;
  }
  auto bail = [&](int code) {
    g_mlp_err = m->last_err;
    sl_mlp_destroy(m);
    return code;
  };
  if (!m->st) {
    if (hipStreamCreateWithFlags(&m->st, hipStreamNonBlocking) != hipSuccess) {
      m->st = nullptr;
      m->last_err = "hipStreamCreate failed";
      return bail(SL_E_HIP);
    }
    m->own_stream = true;
  }
  if (hipMalloc((void **)&m->master, sizeof(float) * SL_MLP_NPARAM) != hipSuccess ||
      hipMalloc((void **)&m->wt, sizeof(MlpDevWeightsT)) != hipSuccess ||
      hipMalloc((void **)&m->grad, sizeof(float) * SL_MLP_NPARAM) != hipSuccess ||
      hipMalloc((void **)&m->adam_m, sizeof(float) * SL_MLP_NPARAM) != hipSuccess ||
      hipMalloc((void **)&m->adam_v, sizeof(float) * SL_MLP_NPARAM) != hipSuccess ||
      hipMalloc((void **)&m->w, sizeof(MlpDevWeights)) != hipSuccess ||
      hipMalloc((void **)&m->yc, sizeof(float) * 4) != hipSuccess ||
      hipMalloc((void **)&m->scratch4, sizeof(float4) * 64) != hipSuccess ||
      hipMalloc((void **)&m->spl, sizeof(float4) * sl_mlp::kSplinePoints) != hipSuccess) {
    m->last_err = "device allocation failed";
    return bail(SL_E_NOMEM);
  }
  *out = m;
  return SL_OK;
}

int sl_mlp_destroy(sl_mlp *m) {
  if (!m) return SL_OK;
  if (m->st) (void)hipStreamSynchronize(m->st);
  if (m->trainer) sl_destroy(m->trainer);
  for (void *p : {(void *)m->master, (void *)m->w, (void *)m->yc, (void *)m->scratch4,
                  (void *)m->wt, (void *)m->grad, (void *)m->adam_m, (void *)m->adam_v,
                  (void *)m->spl})
    if (p) (void)hipFree(p);
  if (m->own_stream && m->st) (void)hipStreamDestroy(m->st);
  delete m;
  return SL_OK;
}

}  // extern "C"

// Refresh the BF16 operand copy and the shifted-force constants after the
// FP32 master parameters changed (stream ordered).
int mlp_refresh(sl_mlp *m) {
  launch_mlp_swizzle(m->master, m->w, m->st);
  launch_mlp_swizzle_t(m->master, m->wt, m->st);
  // raw outputs at r = rc and r = ex_rc -> yc = (y1(rc), y1'(rc), y0(ex_rc),
  // y0'(ex_rc)): the shifted-force constants of phi and of a shifted J
  const float rr[2] = {(float)m->rc, (float)m->ex_rc};
  float *d_r = (float *)(m->scratch4 + 32);
  MCHK(m, hipMemcpyAsync(d_r, rr, sizeof(rr), hipMemcpyHostToDevice, m->st));
  launch_mlp_eval(d_r, 2, m->w, m->cfg(), m->yc, 1, m->scratch4, m->st);
  MCHK(m, hipMemcpyAsync(m->yc, (float *)m->scratch4 + 2, 2 * sizeof(float), hipMemcpyDeviceToDevice, m->st));
  MCHK(m, hipMemcpyAsync(m->yc + 2, (float *)(m->scratch4 + 1), 2 * sizeof(float),
                         hipMemcpyDeviceToDevice, m->st));
  // spline table: the master network in FP64 on the grid; its last point is
  // rc, which gives the shifted-force constants of the spline form
  const double dr = (m->rc - sl_mlp::kSplineR0) / (sl_mlp::kSplinePoints - 1);
  launch_mlp_grid(m->master, sl_mlp::kSplineR0, dr, sl_mlp::kSplinePoints, m->sigma, m->mu_step,
                  m->spl, m->st);
  float4 last;
  MCHK(m, hipMemcpyAsync(&last, m->spl + sl_mlp::kSplinePoints - 1, sizeof(float4),
                         hipMemcpyDeviceToHost, m->st));
  // the spline's y0 and y0' at ex_rc (its cubic Hermite interpolant there),
  // the constants of a shifted J in the spline form
  double u = (m->ex_rc - sl_mlp::kSplineR0) / dr;
  u = std::min(std::max(u, 0.0), (double)(sl_mlp::kSplinePoints - 1));
  const int k = std::min((int)u, sl_mlp::kSplinePoints - 2);
  float4 ab[2];
  MCHK(m, hipMemcpyAsync(ab, m->spl + k, 2 * sizeof(float4), hipMemcpyDeviceToHost, m->st));
  MCHK(m, hipStreamSynchronize(m->st));
  m->spl_yc[0] = last.z;
  m->spl_yc[1] = last.w;
  {
    const float x = (float)(u - k), x2 = x * x, x3 = x2 * x, fdr = (float)dr, idr = (float)(1.0 / dr);
    const float h00 = 2.0f * x3 - 3.0f * x2 + 1.0f, h10 = x3 - 2.0f * x2 + x;
    const float h01 = 3.0f * x2 - 2.0f * x3, h11 = x3 - x2;
    const float g00 = 6.0f * (x2 - x), g10 = 3.0f * x2 - 4.0f * x + 1.0f, g11 = 3.0f * x2 - 2.0f * x;
    m->spl_j0[0] = h00 * ab[0].x + h01 * ab[1].x + fdr * (h10 * ab[0].y + h11 * ab[1].y);
    m->spl_j0[1] = g00 * (ab[0].x - ab[1].x) * idr + g10 * ab[0].y + g11 * ab[1].y;
  }
  m->have_weights = true;
  return SL_OK;
}

extern "C" {

int sl_mlp_set_weights(sl_mlp *m, const float *params, int n, int where) {
  if (!m || !params) return mfail(m, SL_E_ARG, "NULL argument");
  if (n != SL_MLP_NPARAM) return mfail(m, SL_E_ARG, "expected SL_MLP_NPARAM parameters");
  if (where == SL_HOST) {
    for (int k = 0; k < n; ++k)
      if (!std::isfinite(params[k])) return mfail(m, SL_E_NONFINITE, "non-finite weight");
  }
  MCHK(m, hipMemcpyAsync(m->master, params, sizeof(float) * n,
                         where == SL_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, m->st));
  MCHK(m, hipMemsetAsync(m->adam_m, 0, sizeof(float) * n, m->st));
  MCHK(m, hipMemsetAsync(m->adam_v, 0, sizeof(float) * n, m->st));
  m->adam_t = 0;
  return mlp_refresh(m);
}

int sl_mlp_get_weights(sl_mlp *m, float *params, int n, int where) {
  if (!m || !params) return mfail(m, SL_E_ARG, "NULL argument");
  if (n != SL_MLP_NPARAM) return mfail(m, SL_E_ARG, "expected SL_MLP_NPARAM parameters");
  MCHK(m, hipMemcpyAsync(params, m->master, sizeof(float) * n,
                         where == SL_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, m->st));
  MCHK(m, hipStreamSynchronize(m->st));
  return SL_OK;
}

int sl_mlp_eval(sl_mlp *m, const double *r, int64_t P, double *out, int where) {
  if (!m || (P > 0 && (!r || !out))) return mfail(m, SL_E_ARG, "NULL argument");
  if (!m->have_weights) return mfail(m, SL_E_STATE, "no weights set");
  if (P <= 0) return SL_OK;
  if (P > (1 << 28)) return mfail(m, SL_E_ARG, "too many distances");
  std::vector<double> hr(P);
  if (where == SL_DEVICE) MCHK(m, hipMemcpy(hr.data(), r, sizeof(double) * P, hipMemcpyDeviceToHost));
  else std::memcpy(hr.data(), r, sizeof(double) * P);
  std::vector<float> fr(P);
  for (int64_t k = 0; k < P; ++k) fr[k] = (float)hr[k];
  float *d_r = nullptr;
  float4 *d_o = nullptr;
  MCHK(m, hipMalloc((void **)&d_r, sizeof(float) * P));
  MCHK(m, hipMalloc((void **)&d_o, sizeof(float4) * P));
  MCHK(m, hipMemcpyAsync(d_r, fr.data(), sizeof(float) * P, hipMemcpyHostToDevice, m->st));
  launch_mlp_eval(d_r, (int)P, m->w, m->cfg(), m->yc, 0, d_o, m->st);
  std::vector<float4> ho(P);
  MCHK(m, hipMemcpyAsync(ho.data(), d_o, sizeof(float4) * P, hipMemcpyDeviceToHost, m->st));
  MCHK(m, hipStreamSynchronize(m->st));
  (void)hipFree(d_r);
  (void)hipFree(d_o);
  std::vector<double> hout(4 * P);
  for (int64_t k = 0; k < P; ++k) {
    hout[4 * k] = ho[k].x;
    hout[4 * k + 1] = ho[k].y;
    hout[4 * k + 2] = ho[k].z;
    hout[4 * k + 3] = ho[k].w;
  }
  if (where == SL_DEVICE) MCHK(m, hipMemcpy(out, hout.data(), sizeof(double) * 4 * P, hipMemcpyHostToDevice));
  else std::memcpy(out, hout.data(), sizeof(double) * 4 * P);
  return SL_OK;
}

const char *sl_mlp_last_error(const sl_mlp *m) { return m ? m->last_err.c_str() : g_mlp_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// sl_mlp_eval without device allocation. Its staging (FP32 distances, the
// network's FP32 outputs, FP64 outputs or host input) lives in one file-scope
// device array per GPU, `scratch`, of SL_MLP_EVAL_STATIC_MAX distances:
//   [0, 4 MAX)         float  r32[MAX]
//   [4 MAX, 20 MAX)    float4 o4[MAX]
//   [20 MAX, 52 MAX)   double o64[4 MAX] (also the staging of host input)
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is resolved once per device with hipGetSymbolAddress and
// only that address is ever passed to kernels and copies.
namespace {

constexpr size_t kStaticMax = SL_MLP_EVAL_STATIC_MAX;
constexpr size_t kStaticBytes = kStaticMax * (4 + 16 + 32);
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {

std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's `scratch` (resolved on the first call on
// the device, with that device current).
int scratch_address(sl_mlp *m, int dev, unsigned char **out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return mfail(m, SL_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (unsigned char *)p;
  }
  *out = g_scratch_ptr[dev];
  return SL_OK;
}

__global__ void k_f64_to_f32(const double *src, float *dst, int P) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < P) dst[q] = (float)src[q];
}

__global__ void k_f32x4_to_f64(const float4 *src, double *dst, int P) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < P) {
    const float4 o = src[q];
    dst[4 * (size_t)q] = o.x;
    dst[4 * (size_t)q + 1] = o.y;
    dst[4 * (size_t)q + 2] = o.z;
    dst[4 * (size_t)q + 3] = o.w;
  }
}

}  // namespace

extern "C" {

int sl_mlp_eval_static(sl_mlp *m, const double *r, int64_t P, double *out, int where) {
  if (!m || (P > 0 && (!r || !out))) return mfail(m, SL_E_ARG, "NULL argument");
  if (where != SL_HOST && where != SL_DEVICE) return mfail(m, SL_E_ARG, "bad `where`");
  if (!m->have_weights) return mfail(m, SL_E_STATE, "no weights set");
  if (P < 0 || P > (int64_t)kStaticMax)
    return mfail(m, SL_E_ARG, "P = " + std::to_string(P) + " outside [0, SL_MLP_EVAL_STATIC_MAX = " +
                                  std::to_string(kStaticMax) + "]");
  if (P == 0) return SL_OK;
  int dev = -1;
  MCHK(m, hipGetDevice(&dev));
  if (dev != m->device)
    return mfail(m, SL_E_ARG, "device " + std::to_string(dev) + " is current, the handle's is " +
                                  std::to_string(m->device));
  if (dev < 0 || dev >= kMaxDevices) return mfail(m, SL_E_ARG, "device index out of range");
  unsigned char *base = nullptr;
  const int rc = scratch_address(m, dev, &base);
  if (rc) return rc;
  float *r32 = (float *)base;
  float4 *o4 = (float4 *)(base + 4 * kStaticMax);
  double *o64 = (double *)(base + 20 * kStaticMax);
  const int n = (int)P;
  const dim3 grid((n + 255) / 256), block(256);
  const double *src = r;
  if (where == SL_HOST) {
    MCHK(m, hipMemcpyAsync(o64, r, sizeof(double) * P, hipMemcpyHostToDevice, m->st));
    src = o64;
  }
  hipLaunchKernelGGL(k_f64_to_f32, grid, block, 0, m->st, src, r32, n);
  launch_mlp_eval(r32, n, m->w, m->cfg(), m->yc, 0, o4, m->st);
  if (where == SL_DEVICE) {
    hipLaunchKernelGGL(k_f32x4_to_f64, grid, block, 0, m->st, o4, out, n);
    MCHK(m, hipGetLastError());
    return SL_OK;  // asynchronous on the handle's stream
  }
  hipLaunchKernelGGL(k_f32x4_to_f64, grid, block, 0, m->st, o4, o64, n);
  MCHK(m, hipMemcpyAsync(out, o64, sizeof(double) * 4 * P, hipMemcpyDeviceToHost, m->st));
  MCHK(m, hipStreamSynchronize(m->st));
  return SL_OK;
}

}  // extern "C"
