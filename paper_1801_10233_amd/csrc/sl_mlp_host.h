// sl_mlp_host.h -- host-side state of an sl_mlp handle (internal).
#pragma once

#include <string>

#include "sl_mlp.h"

struct sl_mlp {
  double sigma = 0.4, mu_step = 5.0 / 15.0, sJ = 0.01, sP = 1.0, ex_rc = 3.5, rc = 5.0;
  hipStream_t st = nullptr;
  bool own_stream = false;
  int device = 0;                       // device current at creation
  float *master = nullptr;              // FP32 master parameters (device)
  sl::MlpDevWeights *w = nullptr;       // BF16 operand copy (device)
  float *yc = nullptr;                  // raw y1(rc), y1'(rc) (device)
  float4 *scratch4 = nullptr;           // small staging
  sl::MlpDevWeightsT *wt = nullptr;     // transposed layer-2 tiles (reverse pass)
  float *grad = nullptr, *adam_m = nullptr, *adam_v = nullptr;
  int64_t adam_t = 0;
  struct sl_system *trainer = nullptr;  // geometry of the training snapshots
  bool have_weights = false;
  // raw outputs tabulated for the spline form of the dynamics
  static constexpr int kSplinePoints = 4096;
  static constexpr double kSplineR0 = 0.5;  // A; closer pairs take the end value
  float4 *spl = nullptr;
  float spl_yc[2] = {0.f, 0.f};             // spline's y1(rc), y1'(rc)
  float spl_j0[2] = {0.f, 0.f};             // spline's y0(ex_rc), y0'(ex_rc)
  std::string last_err;
  sl::SplineView spline_view() const {
    sl::SplineView v;
    v.t = spl;
    v.r0 = (float)kSplineR0;
    v.dr = (float)((rc - kSplineR0) / (kSplinePoints - 1));
    v.idr = (float)((kSplinePoints - 1) / (rc - kSplineR0));
    v.last = kSplinePoints - 1;
    v.sJ = (float)sJ;
    v.sP = (float)sP;
    v.y1c = spl_yc[0];
    v.d1c = spl_yc[1];
    v.exrc = (float)ex_rc;
    v.rc = (float)rc;
    v.jshift = 0;  // set by the system that uses it
    v.y0c = spl_j0[0];
    v.d0c = spl_j0[1];
    return v;
  }
  sl::MlpCfgDev cfg() const {
    sl::MlpCfgDev c;
    c.inv_sigma = (float)(1.0 / sigma);
    c.mu_step = (float)mu_step;
    c.sJ = (float)sJ;
    c.sP = (float)sP;
    c.ex_rc = (float)ex_rc;
    c.rc = (float)rc;
    c.jshift = 0;  // set by the system that uses it
    return c;
  }
};

// Refresh the BF16 copy and the shifted-force constants after the master
// parameters changed.
int mlp_refresh(sl_mlp *m);
