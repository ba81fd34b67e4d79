// Host side of the C ABI declared in include/lsp.h: plan matching, argument
// validation and kernel dispatch.  All launches are asynchronous on the
// caller's stream; nothing here allocates device memory.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lsp.h"
#include "lsp_kernels.hip"
#include "lsp_binned.hip"

namespace {

using namespace lsp;

enum SpecId { kBccLinear = 0, kCcZp, kBccQuartic, kFcc6, kD4s8, kD48, kNumSpecs };

struct SpecDesc {
  const char* name;
  int s, ndir, D, M, det, deg, K, Q, fold_even, nmon, omin, omax;
  std::vector<std::vector<int>> dirs;
  std::vector<std::vector<int>> shifts;
  std::vector<int> nsite, nnz;
  int lookups;
};

template <class SP>
SpecDesc describe(const char* name) {
  SpecDesc d{};
  d.name = name;
  d.s = SP::S; d.ndir = SP::NDIR; d.D = SP::D; d.M = SP::M; d.det = SP::DETL; d.deg = SP::DEG;
  d.K = SP::K; d.Q = SP::Q; d.fold_even = SP::FOLD_D ? 1 : 0; d.nmon = SP::NMON;
  d.omin = SP::OMIN; d.omax = SP::OMAX;
  for (int j = 0; j < SP::NDIR; ++j) d.dirs.emplace_back(SP::XI[j], SP::XI[j] + SP::S);
  for (int k = 0; k < SP::M; ++k) d.shifts.emplace_back(SP::SHIFT[k], SP::SHIFT[k] + SP::S);
  for (int k = 0; k < SP::K; ++k) { d.nsite.push_back(SP::NSITE[k]); d.nnz.push_back(SP::NNZ[k]); }
  return d;
}

const std::vector<SpecDesc>& specs() {
  static const std::vector<SpecDesc> all = {
      describe<SplineBccLinear>("bcc_linear"), describe<SplineCcZp>("cc_zp"),
      describe<SplineBccQuartic>("bcc_quartic"), describe<SplineFcc6>("fcc_6dir"),
      describe<SplineD4s8>("d4s_8dir"), describe<SplineD48>("d4_8dir")};
  return all;
}

}  // namespace

struct lsp_plan_s {
  int spec;
};

struct lsp_vol_s {
  int spec;
  int dtype;
  Vol vol;
  int64_t total;
};

namespace {

// exact small-integer linear algebra on the host
long long det_int(const std::vector<std::vector<long long>>& A) {
  const int n = static_cast<int>(A.size());
  if (n == 1) return A[0][0];
  long long det = 0;
  for (int c = 0; c < n; ++c) {
    std::vector<std::vector<long long>> m;
    for (int r = 1; r < n; ++r) {
      std::vector<long long> row;
      for (int cc = 0; cc < n; ++cc)
        if (cc != c) row.push_back(A[r][cc]);
      m.push_back(row);
    }
    det += ((c & 1) ? -1 : 1) * A[0][c] * det_int(m);
  }
  return det;
}

// adjugate: adj(A) A = det(A) I
std::vector<std::vector<long long>> adj_int(const std::vector<std::vector<long long>>& A) {
  const int n = static_cast<int>(A.size());
  std::vector<std::vector<long long>> adj(n, std::vector<long long>(n, 1));
  if (n == 1) return adj;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      std::vector<std::vector<long long>> m;
      for (int r = 0; r < n; ++r) {
        if (r == i) continue;
        std::vector<long long> row;
        for (int c = 0; c < n; ++c)
          if (c != j) row.push_back(A[r][c]);
        m.push_back(row);
      }
      adj[j][i] = (((i + j) & 1) ? -1 : 1) * det_int(m);
    }
  return adj;
}

long long gcdll(long long a, long long b) {
  a = a < 0 ? -a : a;
  b = b < 0 ? -b : b;
  while (b) { long long t = a % b; a = b; b = t; }
  return a;
}

bool on_lattice(const std::vector<std::vector<long long>>& adj, long long det, const std::vector<long long>& v) {
  const int n = static_cast<int>(v.size());
  for (int i = 0; i < n; ++i) {
    long long acc = 0;
    for (int j = 0; j < n; ++j) acc += adj[i][j] * v[j];
    if (acc % det != 0) return false;
  }
  return true;
}

std::vector<int> canon_dir(std::vector<int> v) {
  std::vector<int> neg(v.size());
  for (size_t i = 0; i < v.size(); ++i) neg[i] = -v[i];
  return std::max(v, neg);
}

// ---------------------------------------------------------------------------
// binned schedule: geometry and workspace layout (bytes, 256-aligned):
//   hist[tiles][nkeys] tot[nkeys+1] start[nkeys+1] partial[1024] recs[items]
//   fpart[items] gpart[items][S]   (per-coset partials, coset-split splines)
//   priv[units][region]            (the adjoint's per-unit LDS regions)
constexpr size_t kLdsMax = 160 * 1024;    // LDS of one gfx950 workgroup
constexpr size_t kLdsEval = 64 * 1024;    // keep several evaluation workgroups per CU
constexpr int kAbsMaxParts = 1024;         // blocks of the max |g| reduction
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
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
unsigned grid_of(long long n, int block = 256) { return static_cast<unsigned>((n + block - 1) / block); }
unsigned fill_grid(long long n) { return static_cast<unsigned>(std::min<long long>((n + 255) / 256, 4096)); }

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
  for (g.bshift = 3;; ++g.bshift) {
    unsigned long long nbr = 1;
    for (int d = 0; d < SP::S; ++d) {
      g.nb[d] = (v->vol.dims[d] + (1 << g.bshift) - 1) >> g.bshift;
      nbr *= static_cast<unsigned long long>(g.nb[d]);
    }
    if (nbr * g.upb * g.kpb * 4 <= hist_budget<SP>()) {
      g.nbricks = static_cast<unsigned>(nbr);
      g.nunits = static_cast<unsigned>(nbr * g.upb);
      g.nkeys = static_cast<unsigned>(nbr * g.upb * g.kpb);
      break;
    }
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
  bn.bytes = o;
  return bn;
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
  hipLaunchKernelGGL(k_bin_colscan, dim3(grid_of(g.nkeys + 1)), dim3(256), 0, st, hist, g.tiles, g.nkeys, tot);
  const unsigned nscan = g.nkeys + 1;
  const unsigned nblocks = (nscan + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_scan_blocks, dim3(nblocks), dim3(256), 0, st, tot, start, partial, nscan);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, st, partial, nblocks);
  hipLaunchKernelGGL(k_scan_add, dim3(nblocks), dim3(256), 0, st, start, partial, nscan);
  hipLaunchKernelGGL((k_bin_place<SP, SPLIT>), dim3(g.tiles), dim3(1024), lds, st, v->vol, g, x, hist, start,
                     recs);
  return hipGetLastError() == hipSuccess ? LSP_OK : LSP_ERR_HIP;
}

unsigned unit_grid(unsigned nunits) { return 8u * ((nunits + 7u) / 8u); }

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
  const dim3 grid(unit_grid(g.nunits));
  // the unit's coefficients are staged in LDS when the region fits
  constexpr int NT = SP::S == 3 ? 256 : 512;
#define LSP_EVAL_BINNED(GRAD_, STAGE_, MSE_)                                                                 \
  hipLaunchKernelGGL((k_eval_binned<SP, CT, AT, GRAD_, SPLIT, STAGE_, MSE_, NT>), grid, dim3(NT), bn.lds_eval, \
                     st, v->vol, g, recs, start, fo, go, y, inv_n, dldf, loss)
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
                         grad, y, inv_n, dldf, loss);
    else
      hipLaunchKernelGGL((k_combine<SP, AT, false, MSE>), cg, dim3(256), 0, st, fo, go, static_cast<long long>(n), f,
                         grad, y, inv_n, dldf, loss);
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
                      float* const* grad_c, float* grad_x, hipStream_t st) {
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
  if (bn.lds_adj_g > kLdsMax) {
    // a unit's region does not fit in LDS (large 4-D bricks): scatter-add
    // with global atomics in the given order
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
  // max |g|: the power-of-two scale of the fixed-point regions
  unsigned* gparts = reinterpret_cast<unsigned*>(const_cast<char*>(base) + bn.off_gmax);
  unsigned* gmax = gparts + kAbsMaxParts;
  const unsigned parts = std::min(grid_of(n), static_cast<unsigned>(kAbsMaxParts));
  hipLaunchKernelGGL(k_absmax_partial, dim3(parts), dim3(256), 0, st, g, static_cast<long long>(n), gparts);
  hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(1024), 0, st, gparts, static_cast<int>(parts), gmax);
  if (grad_x) {
    if (bn.adj_stage_c)
      hipLaunchKernelGGL((k_adjoint_binned<SP, CT, true, SPLIT, true>), grid, dim3(512), bn.lds_adj, st, v->vol, gv,
                         gm, recs, start, g, gx_out, priv, gmax);
    else
      hipLaunchKernelGGL((k_adjoint_binned<SP, CT, true, SPLIT, false>), grid, dim3(512), lds_g, st, v->vol, gv, gm,
                         recs, start, g, gx_out, priv, gmax);
  } else {
    hipLaunchKernelGGL((k_adjoint_binned<SP, CT, false, SPLIT, false>), grid, dim3(512), lds_g, st, v->vol, gv, gm,
                       recs, start, g, gx_out, priv, gmax);
  }
  long long sites = 1;
  for (int d = 0; d < SP::S; ++d) sites *= v->vol.dims[d];
  hipLaunchKernelGGL((k_adjoint_gather<SP, SPLIT>), dim3(grid_of(sites * SP::M)), dim3(256), 0, st, v->vol, gv, gm,
                     start, priv, sites);
  if (SPLIT && grad_x)
    hipLaunchKernelGGL((k_combine_gx<SP>), dim3(grid_of(n * SP::S)), dim3(256), 0, st, gx_out,
                       static_cast<long long>(n), grad_x);
  return hipGetLastError() == hipSuccess ? LSP_OK : LSP_ERR_HIP;
}

template <class SP>
lsp_status adj_spec(const lsp_vol_s* v, const float* x, const float* g, int64_t n, const void* ws,
                    float* const* grad_c, float* grad_x, hipStream_t st) {
  switch (v->dtype) {
    case LSP_F32: return launch_adj<SP, float>(v, x, g, n, ws, grad_c, grad_x, st);
    case LSP_BF16: return launch_adj<SP, bf16_t>(v, x, g, n, ws, grad_c, grad_x, st);
    case LSP_F16: return launch_adj<SP, f16_t>(v, x, g, n, ws, grad_c, grad_x, st);
  }
  return LSP_ERR_DTYPE;
}

template <class SP>
lsp_status sched_size_spec(const lsp_vol_s* v, int64_t n, size_t* bytes) {
  *bytes = make_bin<SP>(v, n).bytes;
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

#define LSP_DISPATCH(spec, FN, ...)                        \
  switch (spec) {                                          \
    case kBccLinear: return FN<SplineBccLinear>(__VA_ARGS__); \
    case kCcZp: return FN<SplineCcZp>(__VA_ARGS__);           \
    case kBccQuartic: return FN<SplineBccQuartic>(__VA_ARGS__); \
    case kFcc6: return FN<SplineFcc6>(__VA_ARGS__);           \
    case kD4s8: return FN<SplineD4s8>(__VA_ARGS__);           \
    case kD48: return FN<SplineD48>(__VA_ARGS__);             \
  }                                                        \
  return LSP_ERR_UNSUPPORTED;

}  // namespace

extern "C" {

const char* lsp_status_string(lsp_status s) {
  switch (s) {
    case LSP_OK: return "ok";
    case LSP_ERR_NULL: return "a required pointer is NULL";
    case LSP_ERR_INVALID: return "invalid argument";
    case LSP_ERR_UNSUPPORTED: return "no generated tables for this lattice / direction matrix";
    case LSP_ERR_DTYPE: return "unsupported or mismatched coefficient dtype";
    case LSP_ERR_DIMS: return "coefficient dims out of range";
    case LSP_ERR_HIP: return "HIP runtime error";
    case LSP_ERR_NOT_ON_LATTICE: return "a direction of Xi is not a lattice vector";
  }
  return "unknown status";
}

lsp_status lsp_plan_create(int32_t s, const int32_t* L, int32_t n, const int32_t* Xi, uint32_t flags,
                           lsp_plan* out) {
  (void)flags;
  if (!L || !Xi || !out) return LSP_ERR_NULL;
  *out = nullptr;
  if (s < 1 || s > 4 || n < s || n > 16) return LSP_ERR_INVALID;
  std::vector<std::vector<long long>> A(s, std::vector<long long>(s));
  for (int r = 0; r < s; ++r)
    for (int c = 0; c < s; ++c) A[r][c] = L[r * s + c];
  const long long det = det_int(A);
  if (det == 0) return LSP_ERR_INVALID;
  const auto adj = adj_int(A);  // L^{-1} = adj / det
  // D: smallest positive integer with D L^{-1} integral
  long long g = det;
  for (auto& row : adj)
    for (long long v : row) g = gcdll(g, v);
  const long long D = (det < 0 ? -det : det) / g;
  std::vector<std::vector<int>> dirs;
  for (int j = 0; j < n; ++j) {
    std::vector<long long> v(s);
    std::vector<int> vi(s);
    for (int a = 0; a < s; ++a) { v[a] = Xi[a * n + j]; vi[a] = Xi[a * n + j]; }
    if (!on_lattice(adj, det, v)) return LSP_ERR_NOT_ON_LATTICE;
    dirs.push_back(canon_dir(vi));
  }
  // rank of Xi must be s
  {
    bool spans = false;
    std::vector<int> idx(s);
    // try all s-subsets of columns for a nonzero determinant
    std::vector<int> sel(n, 0);
    std::fill(sel.begin(), sel.begin() + s, 1);
    std::sort(sel.begin(), sel.end(), std::greater<int>());
    do {
      std::vector<std::vector<long long>> B(s, std::vector<long long>(s));
      int c = 0;
      for (int j = 0; j < n; ++j)
        if (sel[j]) {
          for (int a = 0; a < s; ++a) B[a][c] = Xi[a * n + j];
          ++c;
        }
      if (det_int(B) != 0) { spans = true; break; }
    } while (std::prev_permutation(sel.begin(), sel.end()));
    if (!spans) return LSP_ERR_INVALID;
  }
  std::sort(dirs.begin(), dirs.end());
  // coset shifts of L Z^s in [0, D)^s
  std::vector<std::vector<int>> shifts;
  {
    std::vector<long long> v(s, 0);
    long long total = 1;
    for (int a = 0; a < s; ++a) total *= D;
    for (long long code = 0; code < total; ++code) {
      long long c = code;
      std::vector<int> vi(s);
      for (int a = 0; a < s; ++a) { v[a] = c % D; vi[a] = static_cast<int>(v[a]); c /= D; }
      if (on_lattice(adj, det, v)) shifts.push_back(vi);
    }
  }
  for (int id = 0; id < kNumSpecs; ++id) {
    const SpecDesc& sd = specs()[id];
    if (sd.s != s || sd.ndir != n || sd.D != D || sd.M != static_cast<int>(shifts.size())) continue;
    std::vector<std::vector<int>> sdirs;
    for (auto& dv : sd.dirs) sdirs.push_back(canon_dir(dv));
    std::sort(sdirs.begin(), sdirs.end());
    if (sdirs != dirs) continue;
    if (sd.shifts != shifts) continue;
    lsp_plan p = new (std::nothrow) lsp_plan_s;
    if (!p) return LSP_ERR_INVALID;
    p->spec = id;
    *out = p;
    return LSP_OK;
  }
  return LSP_ERR_UNSUPPORTED;
}

lsp_status lsp_plan_info(lsp_plan plan, lsp_info* out) {
  if (!plan || !out) return LSP_ERR_NULL;
  std::memset(out, 0, sizeof(*out));
  const SpecDesc& sd = specs()[plan->spec];
  out->s = sd.s; out->n_dirs = sd.ndir; out->det_l = sd.det; out->D = sd.D; out->n_cosets = sd.M;
  for (int k = 0; k < sd.M; ++k)
    for (int a = 0; a < sd.s; ++a) out->shifts[k][a] = sd.shifts[k][a];
  out->degree = sd.deg; out->n_subregions = sd.K; out->n_planes = sd.Q; out->fold_even = sd.fold_even;
  for (int k = 0; k < sd.K && k < 16; ++k) { out->stencil[k] = sd.nsite[k]; out->nnz[k] = sd.nnz[k]; }
  // every query gathers the same total over its cosets when K = 1; report the
  // sub-region-averaged total otherwise
  long long tot = 0;
  for (int v : sd.nsite) tot += v;
  out->lookups = static_cast<int32_t>((tot * sd.M + sd.K / 2) / sd.K);
  out->n_monomials = sd.nmon;
  out->offset_min = sd.omin; out->offset_max = sd.omax;
  std::strncpy(out->name, sd.name, sizeof(out->name) - 1);
  return LSP_OK;
}

lsp_status lsp_plan_destroy(lsp_plan plan) {
  if (!plan) return LSP_ERR_NULL;
  delete plan;
  return LSP_OK;
}

lsp_status lsp_vol_bind(lsp_plan plan, int32_t dtype, const void* const* coset_ptrs, const int64_t* dims,
                        lsp_vol* out) {
  if (!plan || !coset_ptrs || !dims || !out) return LSP_ERR_NULL;
  *out = nullptr;
  if (dtype < LSP_F32 || dtype > LSP_F64) return LSP_ERR_DTYPE;
  const SpecDesc& sd = specs()[plan->spec];
  lsp_vol v = new (std::nothrow) lsp_vol_s;
  if (!v) return LSP_ERR_INVALID;
  std::memset(&v->vol, 0, sizeof(v->vol));
  int64_t total = 1;
  for (int a = 0; a < sd.s; ++a) {
    if (dims[a] < 1 || dims[a] > (1 << 20)) { delete v; return LSP_ERR_DIMS; }
    v->vol.stride[a] = static_cast<int>(total);
    v->vol.dims[a] = static_cast<int>(dims[a]);
    total *= dims[a];
    if (total >= (int64_t(1) << 31)) { delete v; return LSP_ERR_DIMS; }
  }
  for (int k = 0; k < sd.M; ++k) {
    if (!coset_ptrs[k]) { delete v; return LSP_ERR_NULL; }
    v->vol.base[k] = coset_ptrs[k];
  }
  v->spec = plan->spec;
  v->dtype = dtype;
  v->total = total;
  *out = v;
  return LSP_OK;
}

lsp_status lsp_vol_release(lsp_vol vol) {
  if (!vol) return LSP_ERR_NULL;
  delete vol;
  return LSP_OK;
}

static lsp_status check_pv(lsp_plan plan, lsp_vol vol) {
  if (!plan || !vol) return LSP_ERR_NULL;
  if (plan->spec != vol->spec) return LSP_ERR_INVALID;
  return LSP_OK;
}

lsp_status lsp_eval(lsp_plan plan, lsp_vol vol, const float* x, int64_t n, void* f, void* grad_x, void* stream) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (n < 0) return LSP_ERR_INVALID;
  if (n == 0) return LSP_OK;
  if (!x || !f) return LSP_ERR_NULL;
  if (n > (int64_t(1) << 40)) return LSP_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  LSP_DISPATCH(plan->spec, eval_spec, vol, x, n, nullptr, f, grad_x, s)
}

lsp_status lsp_eval_mse(lsp_plan plan, lsp_vol vol, const float* x, const float* y, int64_t n, float* f,
                        float* dloss_df, float* dloss_dx, double* loss, void* stream) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (n < 0) return LSP_ERR_INVALID;
  if (n == 0) return LSP_OK;
  if (!x || !y || !f || !dloss_df || !loss) return LSP_ERR_NULL;
  if (vol->dtype == LSP_F64) return LSP_ERR_DTYPE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  LSP_DISPATCH(plan->spec, mse_spec, vol, x, y, n, nullptr, f, dloss_df, dloss_dx, loss, s)
}

lsp_status lsp_eval_adjoint(lsp_plan plan, lsp_vol vol, const float* x, const float* g, int64_t n,
                            float* const* grad_c, float* grad_x, void* stream) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (n < 0) return LSP_ERR_INVALID;
  if (n == 0) return LSP_OK;
  if (!x || !g || !grad_c) return LSP_ERR_NULL;
  const SpecDesc& sd = specs()[plan->spec];
  for (int k = 0; k < sd.M; ++k)
    if (!grad_c[k]) return LSP_ERR_NULL;
  if (vol->dtype == LSP_F64) return LSP_ERR_DTYPE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  LSP_DISPATCH(plan->spec, adj_spec, vol, x, g, n, nullptr, grad_c, grad_x, s)
}

lsp_status lsp_eval_rays(lsp_plan plan, lsp_vol vol, const float* c, const float* A, int32_t W, int32_t H,
                         int32_t steps, int64_t ray0, int64_t nrays, float* out, float* samples, void* stream) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (!c || !A) return LSP_ERR_NULL;
  if (W <= 0 || H <= 0 || (W & 7) || (H & 7) || steps <= 0 || ray0 < 0 || nrays < 0 ||
      ray0 + nrays > static_cast<int64_t>(W) * H)
    return LSP_ERR_INVALID;
  if (nrays == 0) return LSP_OK;
  if (!out) return LSP_ERR_NULL;
  if (vol->dtype == LSP_F64) return LSP_ERR_DTYPE;
  RayParams rp{};
  for (int a = 0; a < 3; ++a) rp.c[a] = c[a];
  for (int a = 0; a < 9; ++a) rp.A[a] = A[a];
  rp.W = W; rp.H = H; rp.steps = steps;
  hipStream_t s = static_cast<hipStream_t>(stream);
  LSP_DISPATCH(plan->spec, rays_spec, vol, rp, ray0, nrays, out, samples, s)
}

static lsp_status check_ws(lsp_plan plan, lsp_vol vol, int64_t n, const void* ws, size_t ws_bytes) {
  if (!ws) return LSP_ERR_NULL;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return LSP_ERR_INVALID;
  size_t need = 0;
  lsp_status st = lsp_schedule_size(plan, vol, n, &need);
  if (st != LSP_OK) return st;
  return ws_bytes >= need ? LSP_OK : LSP_ERR_INVALID;
}

lsp_status lsp_schedule_size(lsp_plan plan, lsp_vol vol, int64_t n, size_t* bytes) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (!bytes) return LSP_ERR_NULL;
  if (n < 0 || n * specs()[plan->spec].M >= (int64_t(1) << 32)) return LSP_ERR_INVALID;
  LSP_DISPATCH(plan->spec, sched_size_spec, vol, n, bytes)
}

lsp_status lsp_schedule(lsp_plan plan, lsp_vol vol, const float* x, int64_t n, void* workspace, size_t ws_bytes,
                        void* stream) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (n < 0) return LSP_ERR_INVALID;
  if ((st = check_ws(plan, vol, n, workspace, ws_bytes)) != LSP_OK) return st;
  if (n == 0) return LSP_OK;
  if (!x) return LSP_ERR_NULL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  LSP_DISPATCH(plan->spec, sched_spec, vol, x, n, workspace, s)
}

lsp_status lsp_eval_scheduled(lsp_plan plan, lsp_vol vol, const float* x, int64_t n, const void* workspace,
                              size_t ws_bytes, void* f, void* grad_x, void* stream) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (n < 0) return LSP_ERR_INVALID;
  if ((st = check_ws(plan, vol, n, workspace, ws_bytes)) != LSP_OK) return st;
  if (n == 0) return LSP_OK;
  if (!x || !f) return LSP_ERR_NULL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  LSP_DISPATCH(plan->spec, eval_spec, vol, x, n, workspace, f, grad_x, s)
}

lsp_status lsp_eval_mse_scheduled(lsp_plan plan, lsp_vol vol, const float* x, const float* y, int64_t n,
                                  const void* workspace, size_t ws_bytes, float* f, float* dloss_df, float* dloss_dx,
                                  double* loss, void* stream) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (n < 0) return LSP_ERR_INVALID;
  if ((st = check_ws(plan, vol, n, workspace, ws_bytes)) != LSP_OK) return st;
  if (n == 0) return LSP_OK;
  if (!x || !y || !f || !dloss_df || !loss) return LSP_ERR_NULL;
  if (vol->dtype == LSP_F64) return LSP_ERR_DTYPE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  LSP_DISPATCH(plan->spec, mse_spec, vol, x, y, n, workspace, f, dloss_df, dloss_dx, loss, s)
}

lsp_status lsp_eval_adjoint_scheduled(lsp_plan plan, lsp_vol vol, const float* x, const float* g, int64_t n,
                                      const void* workspace, size_t ws_bytes, float* const* grad_c, float* grad_x,
                                      void* stream) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (n < 0) return LSP_ERR_INVALID;
  if ((st = check_ws(plan, vol, n, workspace, ws_bytes)) != LSP_OK) return st;
  if (n == 0) return LSP_OK;
  if (!x || !g || !grad_c) return LSP_ERR_NULL;
  const SpecDesc& sd = specs()[plan->spec];
  for (int k = 0; k < sd.M; ++k)
    if (!grad_c[k]) return LSP_ERR_NULL;
  if (vol->dtype == LSP_F64) return LSP_ERR_DTYPE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  LSP_DISPATCH(plan->spec, adj_spec, vol, x, g, n, workspace, grad_c, grad_x, s)
}

}  // extern "C"
