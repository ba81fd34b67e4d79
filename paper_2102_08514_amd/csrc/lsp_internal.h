// Types and launcher declarations shared by the host translation units of the
// library (lsp_api.hip and the per-spline spec_<name>.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "../../include/lsp.h"
#include "lsp_kernels.hip"
#include "lsp_binned.hip"

struct lsp_plan_s {
  int spec;
};

struct lsp_vol_s {
  int spec;
  int dtype;
  lsp::Vol vol;
  int64_t total;
};

namespace lsp_host {

// per spline type SP; defined in lsp_launch.hip, instantiated in spec_<name>.hip
template <class SP>
lsp_status eval_spec(const lsp_vol_s* v, const float* x, int64_t n, const void* ws, void* f, void* grad,
                     hipStream_t st);
template <class SP>
lsp_status mse_spec(const lsp_vol_s* v, const float* x, const float* y, int64_t n, const void* ws, float* f,
                    float* dldf, float* dldx, double* loss, hipStream_t st);
template <class SP>
lsp_status adj_spec(const lsp_vol_s* v, const float* x, const float* g, int64_t n, const void* ws,
                    float* const* grad_c, float* grad_x, hipStream_t st, bool g_saved);
template <class SP>
lsp_status sched_size_spec(const lsp_vol_s* v, int64_t n, size_t* bytes);
template <class SP>
lsp_status sched_fwd_size_spec(const lsp_vol_s* v, int64_t n, size_t* bytes);
template <class SP>
lsp_status sched_spec(const lsp_vol_s* v, const float* x, int64_t n, void* ws, hipStream_t st);
template <class SP>
lsp_status rays_spec(const lsp_vol_s* v, const lsp::RayParams& rp, int64_t ray0, int64_t nrays, float* out,
                     float* samples, hipStream_t st);

template <class SP>
lsp_status render_spec(const lsp_vol_s* v, const lsp::RayParams& rp, const lsp::RenderParams& rd, const float* tf,
                       int64_t ray0, int64_t nrays, float* out, hipStream_t st);

}  // namespace lsp_host
