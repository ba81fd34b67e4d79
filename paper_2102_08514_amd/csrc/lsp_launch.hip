// Host-side launchers of the HIP kernels, one set per spline type.  Each
// spline's launchers are compiled in a translation unit of their own
// (spec_<name>.hip, through LSP_INSTANTIATE); lsp_api.hip only dispatches.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "lsp_internal.h"

namespace lsp_host {

using namespace lsp;

// ---------------------------------------------------------------------------
// binned schedule: geometry and workspace layout (bytes, 256-aligned):
//   hist[tiles][nkeys] tot[nkeys+1] start[nkeys+1] partial[1024] recs[items]
//   fpart[items] gpart[items][S]   (per-coset partials, coset-split splines)
//   priv[units][region]            (the adjoint's per-unit LDS regions)
constexpr size_t kLdsMax = 160 * 1024;    // LDS of one gfx950 workgroup
constexpr size_t kLdsEval = 64 * 1024;    // keep several evaluation workgroups per CU
constexpr int kAbsMaxParts = 1024;         // blocks of the max |g| reduction
constexpr unsigned long long kMinUnits = 1024;        // fewer units than this: smaller bricks
constexpr unsigned long long kMinEvalGroups = 2048;   // fewer units than this: several workgroups per unit
constexpr unsigned kScanSingle = 1u << 13;  // key totals scanned by one workgroup up to this count
constexpr unsigned kOutlierGroups = 128;      // workgroups of the outlier kernels (grid-stride loops)
// key histogram budget: 3-D bricks stay at 16^3 cells for the big volumes
// (fewer, fuller bricks amortise the staged halo); 4-D needs the full LDS to
// keep 8^4 bricks with sub-region keys
template <class SP>
constexpr size_t hist_budget() { return SP::S == 3 ? 64 * 1024 : kLdsMax; }

struct Bin {
  BinGeom g;
  bool split;
  int at_size;
  size_t region;        // floats per coset of a unit's staged region
  size_t off_hist, off_tot, off_start, off_partial, off_recs, off_fpart, off_gpart, off_priv, bytes;
  size_t lds_eval;      // 0: evaluate from global memory
  size_t lds_adj;       // fixed-point gradient region (+ coefficient region when staged)
  size_t lds_adj_g;     // fixed-point gradient region alone
  bool adj_stage_c;
  size_t off_gmax;      // max |g| partials and result (the adjoint's fixed-point scale)
  size_t off_gsave;     // dL/df of the last scheduled MSE forward (schedule order, or by query if split)
};

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
inline unsigned grid_of(long long n, int block = 256) { return static_cast<unsigned>((n + block - 1) / block); }
inline unsigned fill_grid(long long n) { return static_cast<unsigned>(std::min<long long>((n + 255) / 256, 4096)); }

template <class SP>
Bin make_bin(const lsp_vol_s* v, int64_t n) {
  Bin bn{};
  bn.split = SplitPolicy<SP>::value;
  bn.at_size = v->dtype == LSP_F64 ? 8 : 4;
  BinGeom& g = bn.g;
  g.n = n;
  g.items = bn.split ? n * SP::M : n;
  g.upb = bn.split ? SP::M : 1;
  g.kpb = bn.split ? SP::K : 1;
  // the smallest brick (from 8 cells a side) whose key histogram fits the
  // LDS budget; 4-cell bricks when 8-cell ones would leave fewer than
  // kMinUnits units, too few workgroups to balance 256 CUs
  auto units_at = [&](int bshift) {
    unsigned long long nbr = 1;
    for (int d = 0; d < SP::S; ++d)
      nbr *= static_cast<unsigned long long>((v->vol.dims[d] + (1 << bshift) - 1) >> bshift);
    return nbr;
  };
  g.bshift = units_at(3) * g.upb < kMinUnits && (units_at(2) * g.upb * g.kpb + 1) * 4 <= hist_budget<SP>() ? 2 : 3;
  for (;; ++g.bshift) {
    unsigned long long nbr = 1;
    for (int d = 0; d < SP::S; ++d) {
      g.nb[d] = (v->vol.dims[d] + (1 << g.bshift) - 1) >> g.bshift;
      nbr *= static_cast<unsigned long long>(g.nb[d]);
    }
    if ((nbr * g.upb * g.kpb + 1) * 4 <= hist_budget<SP>()) {
      g.nbricks = static_cast<unsigned>(nbr);
      g.nunits = static_cast<unsigned>(nbr * g.upb);
      g.okey = static_cast<unsigned>(nbr * g.upb * g.kpb);
      g.nkeys = g.okey + 1;
      break;
    }
  }
  // evaluation workgroups per unit: enough for kMinEvalGroups workgroups in
  // all, as long as each still gets 2048 items or more on average
  {
    const unsigned long long want = (kMinEvalGroups + g.nunits - 1) / g.nunits;
    const unsigned long long fill = static_cast<unsigned long long>(g.items) / (2048ull * g.nunits);
    g.wpu = static_cast<unsigned>(std::max<unsigned long long>(1, std::min<unsigned long long>({8, want, fill})));
  }
  g.tiles = static_cast<int>(std::max<long long>(1, std::min<long long>(256, (g.items + 4095) / 4096)));
  g.tile_items = (g.items + g.tiles - 1) / g.tiles;
  const int nc = bn.split ? 1 : SP::M;
  bn.region = static_cast<size_t>(Staged<SP>::volume(1 << g.bshift));
  const size_t eval_lds = nc * bn.region * bn.at_size;
  // 3-D: several small staged regions per CU; 4-D: one region of up to the
  // whole LDS, evaluated by a 512-thread workgroup
  bn.lds_eval = eval_lds <= (SP::S == 3 ? kLdsEval : kLdsMax) ? eval_lds : 0;
  const size_t grad_lds = nc * bn.region * 8;   // 64-bit fixed-point accumulators
  const size_t coef_lds = nc * bn.region * 4;
  bn.adj_stage_c = SP::S == 3 && grad_lds + coef_lds <= kLdsMax;
  bn.lds_adj_g = grad_lds;
  bn.lds_adj = grad_lds + (bn.adj_stage_c ? coef_lds : 0);
  size_t o = 0;
  bn.off_hist = o; o = align256(o + 4ull * g.tiles * g.nkeys);
  bn.off_tot = o; o = align256(o + 4ull * (g.nkeys + 1));
  bn.off_start = o; o = align256(o + 4ull * (g.nkeys + 1));
  bn.off_partial = o; o = align256(o + 4ull * 1024);
  bn.off_recs = o; o = align256(o + sizeof(Rec<SP::S>) * static_cast<size_t>(g.items));
  bn.off_fpart = o; o = align256(o + (bn.split ? static_cast<size_t>(bn.at_size) * g.items : 0));
  bn.off_gpart = o; o = align256(o + (bn.split ? static_cast<size_t>(bn.at_size) * g.items * SP::S : 0));
  bn.off_priv = o; o = align256(o + (grad_lds <= kLdsMax ? 4ull * g.nunits * nc * bn.region : 0));
  bn.off_gmax = o; o = align256(o + 4ull * (kAbsMaxParts + 1));
  bn.off_gsave = o; o = align256(o + 4ull * static_cast<size_t>(bn.split ? g.n : g.items));
  bn.bytes = o;
  return bn;
}

// Record placement through LDS windows of 16384 items (k_bin_place_win),
// when a window holds two or more records per key on average, with chunks of
// 2^cshift records passing through LDS; 0: the direct placement.  LDS: two
// words per key and one record per chunk position.
template <class SP>
size_t place_window_lds(const BinGeom& g, int cshift) {
  return 8ull * g.nkeys + (sizeof(Rec<SP::S>) << cshift);
}

template <class SP>
int place_window_shift(const BinGeom& g) {
  constexpr long long kWindow = 16384;
  // 4-D items keep 64 coordinates per thread in registers and spill: direct placement
  if (SP::S != 3 || g.nkeys >= (1u << 17)) return 0;
  if (std::min<long long>(kWindow, g.tile_items) < 2ll * g.nkeys) return 0;
  int c = 0;
  for (int k = 10; k <= 14; ++k)
    if (place_window_lds<SP>(g, k) <= kLdsMax) c = k;
  return c;
}

// The windowed placement with the window's queries in LDS (k_bin_place_winq)
// for (query, coset) items of splines with M >= 4 cosets, when the window
// holds two or more records per key on average.
template <class SP>
size_t place_winq_lds(const BinGeom& g) {
  constexpr size_t W = 16384, WQ = W / SP::M + 2;
  return 4ull * (WQ * SP::S + W + 2ull * g.nkeys);
}

template <class SP>
bool place_winq(const BinGeom& g) {
  if constexpr (!SplitPolicy<SP>::value || SP::M < 4) {
    return false;
  } else {
    if (g.nkeys >= (1u << 17)) return false;
    if (std::min<long long>(16384, g.tile_items) < 2ll * g.nkeys) return false;
    return place_winq_lds<SP>(g) <= kLdsMax;
  }
}

template <class SP>
lsp_status run_schedule(const lsp_vol_s* v, const float* x, int64_t n, void* ws, hipStream_t st) {
  const Bin bn = make_bin<SP>(v, n);
  const BinGeom& g = bn.g;
  char* base = static_cast<char*>(ws);
  unsigned* hist = reinterpret_cast<unsigned*>(base + bn.off_hist);
  unsigned* tot = reinterpret_cast<unsigned*>(base + bn.off_tot);
  unsigned* start = reinterpret_cast<unsigned*>(base + bn.off_start);
  unsigned* partial = reinterpret_cast<unsigned*>(base + bn.off_partial);
  Rec<SP::S>* recs = reinterpret_cast<Rec<SP::S>*>(base + bn.off_recs);
  const size_t lds = 4ull * g.nkeys;
  constexpr bool SPLIT = SplitPolicy<SP>::value;
  hipLaunchKernelGGL((k_bin_hist<SP, SPLIT>), dim3(g.tiles), dim3(1024), lds, st, v->vol, g, x, hist);
  hipLaunchKernelGGL(k_bin_colscan<>, dim3(grid_of(g.nkeys + 1)), dim3(256), 0, st, hist, g.tiles, g.nkeys, tot);
  const unsigned nscan = g.nkeys + 1;
  const unsigned nblocks = (nscan + kScanBlock - 1) / kScanBlock;
  if (nscan <= kScanSingle) {
    hipLaunchKernelGGL(k_scan_single<>, dim3(1), dim3(1024), 0, st, tot, start, nscan);
  } else {
    hipLaunchKernelGGL(k_scan_blocks<>, dim3(nblocks), dim3(256), 0, st, tot, start, partial, nscan);
    hipLaunchKernelGGL(k_scan_top<>, dim3(1), dim3(256), 0, st, partial, nblocks);
    hipLaunchKernelGGL(k_scan_add<>, dim3(nblocks), dim3(256), 0, st, start, partial, nscan);
  }
  const int cshift = place_window_shift<SP>(g);
  if constexpr (SP::S == 3) {
    if (cshift)
      hipLaunchKernelGGL((k_bin_place_win<SP, SPLIT>), dim3(g.tiles), dim3(1024), place_window_lds<SP>(g, cshift),
                         st, v->vol, g, x, hist, start, recs, cshift);
  }
  const bool winq = !cshift && place_winq<SP>(g);
  if constexpr (SPLIT && SP::M >= 4) {
    if (winq)
      hipLaunchKernelGGL((k_bin_place_winq<SP>), dim3(g.tiles), dim3(1024), place_winq_lds<SP>(g), st, v->vol, g, x,
                         hist, start, recs);
  }
  if (!cshift && !winq)
    hipLaunchKernelGGL((k_bin_place<SP, SPLIT>), dim3(g.tiles), dim3(1024), lds, st, v->vol, g, x, hist, start,
                       recs);
  return hipGetLastError() == hipSuccess ? LSP_OK : LSP_ERR_HIP;
}

inline unsigned unit_grid(unsigned nunits) { return 8u * ((nunits + 7u) / 8u); }

template <class SP, class CT, class AT, bool MSE>
lsp_status launch_binned_eval(const lsp_vol_s* v, int64_t n, const void* ws, AT* f, AT* grad, const float* y,
                              float* dldf, double* loss, hipStream_t st) {
  const Bin bn = make_bin<SP>(v, n);
  const BinGeom& g = bn.g;
  const char* base = static_cast<const char*>(ws);
  const unsigned* start = reinterpret_cast<const unsigned*>(base + bn.off_start);
  const Rec<SP::S>* recs = reinterpret_cast<const Rec<SP::S>*>(base + bn.off_recs);
  constexpr bool SPLIT = SplitPolicy<SP>::value;
  const float inv_n = 1.0f / static_cast<float>(n);
  float* gsave = MSE ? reinterpret_cast<float*>(const_cast<char*>(base) + bn.off_gsave) : nullptr;
  const dim3 grid(unit_grid(g.nunits * g.wpu));
  // the unit's coefficients are staged in LDS when the region fits
  constexpr int NT = SP::S == 3 ? 256 : 512;
#define LSP_EVAL_BINNED(GRAD_, STAGE_, MSE_)                                                                   \
  do {                                                                                                           \
    if constexpr (SP::S == 4)                                                                                    \
      hipLaunchKernelGGL((k_eval_binned_w4<SP, CT, AT, GRAD_, SPLIT, STAGE_, MSE_, NT>), grid, dim3(NT),          \
                         bn.lds_eval, st, v->vol, g, recs, start, fo, go, y, inv_n, dldf, loss, gsave);          \
    else                                                                                                         \
      hipLaunchKernelGGL((k_eval_binned<SP, CT, AT, GRAD_, SPLIT, STAGE_, MSE_, NT>), grid, dim3(NT),             \
                         bn.lds_eval, st, v->vol, g, recs, start, fo, go, y, inv_n, dldf, loss, gsave);          \
    hipLaunchKernelGGL((k_eval_outliers<SP, CT, AT, GRAD_, SPLIT, MSE_>), dim3(kOutlierGroups), dim3(256), 0,    \
                       st, v->vol, g, recs, start, fo, go, y, inv_n, dldf, loss, gsave);                          \
  } while (0)
  if constexpr (SPLIT) {
    AT* fo = reinterpret_cast<AT*>(const_cast<char*>(base) + bn.off_fpart);
    AT* go = reinterpret_cast<AT*>(const_cast<char*>(base) + bn.off_gpart);
    if (bn.lds_eval) {
      if (grad) LSP_EVAL_BINNED(true, true, false); else LSP_EVAL_BINNED(false, true, false);
    } else {
      if (grad) LSP_EVAL_BINNED(true, false, false); else LSP_EVAL_BINNED(false, false, false);
    }
    const dim3 cg(std::min(grid_of(n), 1024u));
    if (grad)
      hipLaunchKernelGGL((k_combine<SP, AT, true, MSE>), cg, dim3(256), 0, st, fo, go, static_cast<long long>(n), f,
                         grad, y, inv_n, dldf, loss, gsave);
    else
      hipLaunchKernelGGL((k_combine<SP, AT, false, MSE>), cg, dim3(256), 0, st, fo, go, static_cast<long long>(n), f,
                         grad, y, inv_n, dldf, loss, gsave);
  } else {
    AT* fo = f;
    AT* go = grad;
    if (bn.lds_eval) {
      if (grad) LSP_EVAL_BINNED(true, true, MSE); else LSP_EVAL_BINNED(false, true, MSE);
    } else {
      if (grad) LSP_EVAL_BINNED(true, false, MSE); else LSP_EVAL_BINNED(false, false, MSE);
    }
  }
#undef LSP_EVAL_BINNED
  return hipGetLastError() == hipSuccess ? LSP_OK : LSP_ERR_HIP;
}

template <class SP, class CT, class AT>
lsp_status launch_eval(const lsp_vol_s* v, const float* x, int64_t n, const void* ws, void* f, void* grad,
                       hipStream_t st) {
  AT* fo = static_cast<AT*>(f);
  AT* go = static_cast<AT*>(grad);
  if (ws) return launch_binned_eval<SP, CT, AT, false>(v, n, ws, fo, go, nullptr, nullptr, nullptr, st);
  if (grad)
    hipLaunchKernelGGL((k_eval<SP, CT, AT, true, false>), dim3(grid_of(n)), dim3(256), 0, st, v->vol, x,
                       static_cast<long long>(n), nullptr, fo, go);
  else
    hipLaunchKernelGGL((k_eval<SP, CT, AT, false, false>), dim3(grid_of(n)), dim3(256), 0, st, v->vol, x,
                       static_cast<long long>(n), nullptr, fo, go);
  return hipGetLastError() == hipSuccess ? LSP_OK : LSP_ERR_HIP;
}

template <class SP>
lsp_status eval_spec(const lsp_vol_s* v, const float* x, int64_t n, const void* ws, void* f, void* grad,
                     hipStream_t st) {
  switch (v->dtype) {
    case LSP_F32: return launch_eval<SP, float, float>(v, x, n, ws, f, grad, st);
    case LSP_BF16: return launch_eval<SP, bf16_t, float>(v, x, n, ws, f, grad, st);
    case LSP_F16: return launch_eval<SP, f16_t, float>(v, x, n, ws, f, grad, st);
    case LSP_F64: return launch_eval<SP, double, double>(v, x, n, ws, f, grad, st);
  }
  return LSP_ERR_DTYPE;
}

template <class SP, class CT>
lsp_status launch_mse(const lsp_vol_s* v, const float* x, const float* y, int64_t n, const void* ws, float* f,
                      float* dldf, float* dldx, double* loss, hipStream_t st) {
  const float inv_n = 1.0f / static_cast<float>(n);
  if (ws) return launch_binned_eval<SP, CT, float, true>(v, n, ws, f, dldx, y, dldf, loss, st);
  if (dldx)
    hipLaunchKernelGGL((k_eval_mse<SP, CT, true>), dim3(grid_of(n)), dim3(256), 0, st, v->vol, x, y,
                       static_cast<long long>(n), inv_n, f, dldf, dldx, loss);
  else
    hipLaunchKernelGGL((k_eval_mse<SP, CT, false>), dim3(grid_of(n)), dim3(256), 0, st, v->vol, x, y,
                       static_cast<long long>(n), inv_n, f, dldf, dldx, loss);
  return hipGetLastError() == hipSuccess ? LSP_OK : LSP_ERR_HIP;
}

template <class SP>
lsp_status mse_spec(const lsp_vol_s* v, const float* x, const float* y, int64_t n, const void* ws, float* f,
                    float* dldf, float* dldx, double* loss, hipStream_t st) {
  switch (v->dtype) {
    case LSP_F32: return launch_mse<SP, float>(v, x, y, n, ws, f, dldf, dldx, loss, st);
    case LSP_BF16: return launch_mse<SP, bf16_t>(v, x, y, n, ws, f, dldf, dldx, loss, st);
    case LSP_F16: return launch_mse<SP, f16_t>(v, x, y, n, ws, f, dldf, dldx, loss, st);
  }
  return LSP_ERR_DTYPE;
}

template <class SP, class CT>
lsp_status launch_adj(const lsp_vol_s* v, const float* x, const float* g, int64_t n, const void* ws,
                      float* const* grad_c, float* grad_x, hipStream_t st, bool g_saved) {
  GradVol gv{};
  for (int k = 0; k < SP::M; ++k) gv.base[k] = grad_c[k];
  if (!ws) {
    if (grad_x)
      hipLaunchKernelGGL((k_adjoint<SP, CT, true, false>), dim3(grid_of(n)), dim3(256), 0, st, v->vol, gv, x, g,
                         static_cast<long long>(n), nullptr, grad_x);
    else
      hipLaunchKernelGGL((k_adjoint<SP, CT, false, false>), dim3(grid_of(n)), dim3(256), 0, st, v->vol, gv, x, g,
                         static_cast<long long>(n), nullptr, grad_x);
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_ERR_HIP;
  }
  const Bin bn = make_bin<SP>(v, n);
  const BinGeom& gm = bn.g;
  // g_saved: the upstream gradient is the dL/df that the last scheduled MSE
  // forward left in the workspace (schedule order unless coset-split)
  if (g_saved) g = reinterpret_cast<const float*>(static_cast<const char*>(ws) + bn.off_gsave);
  // the gather pass: one block per 256-site run along axis 0 of each row of
  // the other axes, per coset
  const unsigned segs = grid_of(v->vol.dims[0]);
  unsigned long long rows = 1;
  for (int d = 1; d < SP::S; ++d) rows *= static_cast<unsigned long long>(v->vol.dims[d]);
  if (bn.lds_adj_g > kLdsMax || rows * segs > 0x7fffffffull) {
    // a unit's region does not fit in LDS (large 4-D bricks): scatter-add
    // with global atomics in the given order
    if (g_saved) return LSP_ERR_UNSUPPORTED;
    if (grad_x)
      hipLaunchKernelGGL((k_adjoint<SP, CT, true, false>), dim3(grid_of(n)), dim3(256), 0, st, v->vol, gv, x, g,
                         static_cast<long long>(n), nullptr, grad_x);
    else
      hipLaunchKernelGGL((k_adjoint<SP, CT, false, false>), dim3(grid_of(n)), dim3(256), 0, st, v->vol, gv, x, g,
                         static_cast<long long>(n), nullptr, grad_x);
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_ERR_HIP;
  }
  const char* base = static_cast<const char*>(ws);
  const unsigned* start = reinterpret_cast<const unsigned*>(base + bn.off_start);
  const Rec<SP::S>* recs = reinterpret_cast<const Rec<SP::S>*>(base + bn.off_recs);
  float* priv = reinterpret_cast<float*>(const_cast<char*>(base) + bn.off_priv);
  constexpr bool SPLIT = SplitPolicy<SP>::value;
  float* gx_out = grad_x;
  if constexpr (SPLIT) gx_out = reinterpret_cast<float*>(const_cast<char*>(base) + bn.off_gpart);
  const dim3 grid(unit_grid(gm.nunits));
  const size_t lds_g = bn.lds_adj_g;
  const int gsorted = (g_saved && !SPLIT) ? 1 : 0;
  // max |g|: the power-of-two scale of the fixed-point regions
  unsigned* gparts = reinterpret_cast<unsigned*>(const_cast<char*>(base) + bn.off_gmax);
  unsigned* gmax = gparts + kAbsMaxParts;
  const unsigned parts = std::min(grid_of(n), static_cast<unsigned>(kAbsMaxParts));
  hipLaunchKernelGGL(k_absmax_partial<>, dim3(parts), dim3(256), 0, st, g, static_cast<long long>(n), gparts);
  hipLaunchKernelGGL(k_absmax_final<>, dim3(1), dim3(1024), 0, st, gparts, static_cast<int>(parts), gmax);
  // items outside the brick grid: float atomics into grad_c, before the gather pass
  if (grad_x)
    hipLaunchKernelGGL((k_adjoint_outliers<SP, CT, true, SPLIT>), dim3(kOutlierGroups), dim3(256), 0, st, v->vol, gv,
                       gm, recs, start, g, gx_out, gsorted);
  else
    hipLaunchKernelGGL((k_adjoint_outliers<SP, CT, false, SPLIT>), dim3(kOutlierGroups), dim3(256), 0, st, v->vol,
                       gv, gm, recs, start, g, gx_out, gsorted);
  if (grad_x) {
    if (bn.adj_stage_c)
      hipLaunchKernelGGL((k_adjoint_binned<SP, CT, true, SPLIT, true>), grid, dim3(512), bn.lds_adj, st, v->vol, gv,
                         gm, recs, start, g, gx_out, priv, gmax, gsorted);
    else
      hipLaunchKernelGGL((k_adjoint_binned<SP, CT, true, SPLIT, false>), grid, dim3(512), lds_g, st, v->vol, gv, gm,
                         recs, start, g, gx_out, priv, gmax, gsorted);
  } else {
    hipLaunchKernelGGL((k_adjoint_binned<SP, CT, false, SPLIT, false>), grid, dim3(512), lds_g, st, v->vol, gv, gm,
                       recs, start, g, gx_out, priv, gmax, gsorted);
  }
  const unsigned rpb = v->vol.dims[0] >= 256 ? 1u : 256u / static_cast<unsigned>(v->vol.dims[0]);
  const unsigned blocks = static_cast<unsigned>((rows + rpb - 1) / rpb) * segs;
  GatherDiv gd{};
  gd.d0 = make_udiv(static_cast<unsigned>(v->vol.dims[0]));
  for (int d = 1; d < SP::S; ++d) gd.dim[d] = make_udiv(static_cast<unsigned>(v->vol.dims[d]));
  hipLaunchKernelGGL((k_adjoint_gather<SP, SPLIT>), dim3(blocks, SP::M), dim3(256), 0, st, v->vol, gv, gm, start, priv,
                     segs, rpb, static_cast<unsigned>(rows), gd);
  if (SPLIT && grad_x)
    hipLaunchKernelGGL((k_combine_gx<SP>), dim3(fill_grid(n * SP::S)), dim3(256), 0, st, gx_out,
                       static_cast<long long>(n), grad_x);
  return hipGetLastError() == hipSuccess ? LSP_OK : LSP_ERR_HIP;
}

template <class SP>
lsp_status adj_spec(const lsp_vol_s* v, const float* x, const float* g, int64_t n, const void* ws,
                    float* const* grad_c, float* grad_x, hipStream_t st, bool g_saved) {
  switch (v->dtype) {
    case LSP_F32: return launch_adj<SP, float>(v, x, g, n, ws, grad_c, grad_x, st, g_saved);
    case LSP_BF16: return launch_adj<SP, bf16_t>(v, x, g, n, ws, grad_c, grad_x, st, g_saved);
    case LSP_F16: return launch_adj<SP, f16_t>(v, x, g, n, ws, grad_c, grad_x, st, g_saved);
  }
  return LSP_ERR_DTYPE;
}

template <class SP>
lsp_status sched_size_spec(const lsp_vol_s* v, int64_t n, size_t* bytes) {
  *bytes = make_bin<SP>(v, n).bytes;
  return LSP_OK;
}

// bytes of the workspace the schedule and the forward use: the layout up to
// the adjoint's per-unit regions (key histograms, scans, records, partials)
template <class SP>
lsp_status sched_fwd_size_spec(const lsp_vol_s* v, int64_t n, size_t* bytes) {
  *bytes = make_bin<SP>(v, n).off_priv;
  return LSP_OK;
}

template <class SP>
lsp_status sched_spec(const lsp_vol_s* v, const float* x, int64_t n, void* ws, hipStream_t st) {
  return run_schedule<SP>(v, x, n, ws, st);
}

template <class SP, class CT>
lsp_status launch_rays(const lsp_vol_s* v, const RayParams& rp, int64_t ray0, int64_t nrays, float* out,
                       float* samples, hipStream_t st) {
  const int block = 256;
  const long long grid = (nrays + block - 1) / block;
  hipLaunchKernelGGL((k_rays<SP, CT>), dim3(static_cast<unsigned>(grid)), dim3(block), 0, st, v->vol, rp,
                     static_cast<long long>(ray0), static_cast<long long>(nrays), out, samples);
  return hipGetLastError() == hipSuccess ? LSP_OK : LSP_ERR_HIP;
}

template <class SP>
lsp_status rays_spec(const lsp_vol_s* v, const RayParams& rp, int64_t ray0, int64_t nrays, float* out,
                     float* samples, hipStream_t st) {
  if constexpr (SP::S != 3) {
    return LSP_ERR_UNSUPPORTED;
  } else {
    switch (v->dtype) {
      case LSP_F32: return launch_rays<SP, float>(v, rp, ray0, nrays, out, samples, st);
      case LSP_BF16: return launch_rays<SP, bf16_t>(v, rp, ray0, nrays, out, samples, st);
      case LSP_F16: return launch_rays<SP, f16_t>(v, rp, ray0, nrays, out, samples, st);
    }
    return LSP_ERR_DTYPE;
  }
}

template <class SP, class CT>
lsp_status launch_render(const lsp_vol_s* v, const RayParams& rp, const RenderParams& rd, const float* tf,
                         int64_t ray0, int64_t nrays, float* out, hipStream_t st) {
  const int block = 256;
  const long long grid = (nrays + block - 1) / block;
  hipLaunchKernelGGL((k_render<SP, CT>), dim3(static_cast<unsigned>(grid)), dim3(block), 0, st, v->vol, rp, rd,
                     reinterpret_cast<const float4*>(tf), static_cast<long long>(ray0),
                     static_cast<long long>(nrays), reinterpret_cast<float4*>(out));
  return hipGetLastError() == hipSuccess ? LSP_OK : LSP_ERR_HIP;
}

template <class SP>
lsp_status render_spec(const lsp_vol_s* v, const RayParams& rp, const RenderParams& rd, const float* tf,
                       int64_t ray0, int64_t nrays, float* out, hipStream_t st) {
  if constexpr (SP::S != 3) {
    return LSP_ERR_UNSUPPORTED;
  } else {
    switch (v->dtype) {
      case LSP_F32: return launch_render<SP, float>(v, rp, rd, tf, ray0, nrays, out, st);
      case LSP_BF16: return launch_render<SP, bf16_t>(v, rp, rd, tf, ray0, nrays, out, st);
      case LSP_F16: return launch_render<SP, f16_t>(v, rp, rd, tf, ray0, nrays, out, st);
    }
    return LSP_ERR_DTYPE;
  }
}

}  // namespace lsp_host

// explicit instantiation of every launcher of spline type SP
#define LSP_INSTANTIATE(SP)                                                                                      \
  namespace lsp_host {                                                                                          \
  template lsp_status eval_spec<SP>(const lsp_vol_s*, const float*, int64_t, const void*, void*, void*,          \
                                    hipStream_t);                                                               \
  template lsp_status mse_spec<SP>(const lsp_vol_s*, const float*, const float*, int64_t, const void*, float*,   \
                                   float*, float*, double*, hipStream_t);                                       \
  template lsp_status adj_spec<SP>(const lsp_vol_s*, const float*, const float*, int64_t, const void*,           \
                                   float* const*, float*, hipStream_t, bool);                                   \
  template lsp_status sched_size_spec<SP>(const lsp_vol_s*, int64_t, size_t*);                                  \
  template lsp_status sched_fwd_size_spec<SP>(const lsp_vol_s*, int64_t, size_t*);                              \
  template lsp_status sched_spec<SP>(const lsp_vol_s*, const float*, int64_t, void*, hipStream_t);               \
  template lsp_status rays_spec<SP>(const lsp_vol_s*, const RayParams&, int64_t, int64_t, float*, float*,        \
                                    hipStream_t);                                                               \
  template lsp_status render_spec<SP>(const lsp_vol_s*, const RayParams&, const RenderParams&, const float*,     \
                                      int64_t, int64_t, float*, hipStream_t);                                   \
  }
