// Host side of the C ABI declared in include/lsp.h: plan matching, argument
// validation and kernel dispatch.  All launches are asynchronous on the
// caller's stream; nothing here allocates device memory.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "lsp_internal.h"

namespace {

using namespace lsp;

enum SpecId {
  kBccLinear = 0, kCcZp, kBccQuartic, kFcc6, kD4s8, kD48,
  kCcTp2, kCcTp3, kCcTp4, kCcLinearRd, kBccQuinticRd,
  kBccVoronoi1, kFccVoronoi1, kCcBccVoronoi1, kCcFccVoronoi1, kFccVoronoi2, kCcFccVoronoi2, kNumSpecs
};

struct SpecDesc {
  const char* name;
  int s, ndir, D, M, det, deg, K, Q, fold_even, nmon, omin, omax;
  std::vector<std::vector<int>> dirs;
  std::vector<std::vector<int>> shifts;
  std::vector<int> nsite, nnz, fma_b, fma_w;
  int lookups;
  int grad_terms;
  int kind;                                // 0 box spline, 1 Voronoi spline
  int vor_n;                               // Voronoi: V_n
  std::vector<std::vector<long long>> vor_lv;  // Voronoi: the cell's lattice (s x s, row-major rows)
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
  for (int k = 0; k < SP::K; ++k) {
    d.nsite.push_back(SP::NSITE[k]);
    d.nnz.push_back(SP::NNZ[k]);
    d.fma_b.push_back(SP::FMA_B[k]);
    d.fma_w.push_back(SP::FMA_W[k]);
  }
  d.kind = SP::KIND;
  d.vor_n = 0;
  if constexpr (SP::KIND == 1) {
    d.vor_n = SP::VOR_N;
    for (int r = 0; r < SP::S; ++r) d.vor_lv.emplace_back(SP::VOR_LV[r], SP::VOR_LV[r] + SP::S);
  }
  d.grad_terms = 0;
  for (int m = 0; m < SP::NMON; ++m)
    for (int r = 0; r < SP::S; ++r) d.grad_terms += SP::MDER[m][r] >= 0 ? 1 : 0;
  return d;
}

const std::vector<SpecDesc>& specs() {
  static const std::vector<SpecDesc> all = {
      describe<SplineBccLinear>("bcc_linear"), describe<SplineCcZp>("cc_zp"),
      describe<SplineBccQuartic>("bcc_quartic"), describe<SplineFcc6>("fcc_6dir"),
      describe<SplineD4s8>("d4s_8dir"), describe<SplineD48>("d4_8dir"),
      describe<SplineCcTp2>("cc_tp2"), describe<SplineCcTp3>("cc_tp3"), describe<SplineCcTp4>("cc_tp4"),
      describe<SplineCcLinearRd>("cc_linear_rd"), describe<SplineBccQuinticRd>("bcc_quintic_rd"),
      describe<SplineBccVoronoi1>("bcc_voronoi1"), describe<SplineFccVoronoi1>("fcc_voronoi1"),
      describe<SplineCcBccVoronoi1>("cc_bcc_voronoi1"), describe<SplineCcFccVoronoi1>("cc_fcc_voronoi1"),
      describe<SplineFccVoronoi2>("fcc_voronoi2"), describe<SplineCcFccVoronoi2>("cc_fcc_voronoi2")};
  return all;
}

}  // namespace

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

// |det L|, the adjugate, D (smallest positive integer with D L^{-1} integral)
// and the coset shifts of L Z^s in [0, D)^s, ordered by sum_a l_a D^a.
struct LatticeShape {
  long long det;
  long long D;
  std::vector<std::vector<long long>> adj;
  std::vector<std::vector<int>> shifts;
};

bool lattice_shape(int s, const int32_t* L, LatticeShape& out) {
  std::vector<std::vector<long long>> A(s, std::vector<long long>(s));
  for (int r = 0; r < s; ++r)
    for (int c = 0; c < s; ++c) A[r][c] = L[r * s + c];
  const long long det = det_int(A);
  if (det == 0) return false;
  out.adj = adj_int(A);  // L^{-1} = adj / det
  out.det = det < 0 ? -det : det;
  long long g = det;
  for (auto& row : out.adj)
    for (long long v : row) g = gcdll(g, v);
  out.D = out.det / g;
  out.shifts.clear();
  std::vector<long long> v(s, 0);
  long long total = 1;
  for (int a = 0; a < s; ++a) total *= out.D;
  for (long long code = 0; code < total; ++code) {
    long long c = code;
    std::vector<int> vi(s);
    for (int a = 0; a < s; ++a) { v[a] = c % out.D; vi[a] = static_cast<int>(v[a]); c /= out.D; }
    if (on_lattice(out.adj, det, v)) out.shifts.push_back(vi);
  }
  return true;
}

lsp_status make_plan(int id, lsp_plan* out) {
  lsp_plan p = new (std::nothrow) lsp_plan_s;
  if (!p) return LSP_ERR_INVALID;
  p->spec = id;
  *out = p;
  return LSP_OK;
}

// Launch limits of the given-order kernels: one work item per lane in a 1-D
// grid whose global size must stay below 2^32.
constexpr int64_t kMaxQueries = int64_t(1) << 31;

// What a schedule workspace was filled for.  The workspace layout (key
// histograms, record offsets, partial buffers) depends on the plan, the
// volume dims, the dtype class and n, and the records hold the queries x;
// the scheduled calls refuse a workspace that lsp_schedule filled for
// anything else.  Keyed by workspace address; bounded.
struct SchedKey {
  int spec;
  int dims[kMaxDim];
  int wide;            // FP64 volume (8-byte partials) or not
  const float* x;
  int64_t n;
  bool operator==(const SchedKey& o) const {
    for (int d = 0; d < kMaxDim; ++d)
      if (dims[d] != o.dims[d]) return false;
    return spec == o.spec && wide == o.wide && x == o.x && n == o.n;
  }
};

std::mutex g_sched_mu;
std::unordered_map<const void*, SchedKey>& sched_registry() {
  static std::unordered_map<const void*, SchedKey> reg;
  return reg;
}
constexpr size_t kMaxSchedRecords = 1 << 16;

SchedKey sched_key(lsp_plan plan, lsp_vol vol, const float* x, int64_t n) {
  SchedKey k{};
  k.spec = plan->spec;
  for (int d = 0; d < kMaxDim; ++d) k.dims[d] = vol->vol.dims[d];
  k.wide = vol->dtype == LSP_F64 ? 1 : 0;
  k.x = x;
  k.n = n;
  return k;
}

void sched_record(const void* ws, const SchedKey& k) {
  std::lock_guard<std::mutex> lk(g_sched_mu);
  auto& reg = sched_registry();
  if (reg.size() >= kMaxSchedRecords && reg.find(ws) == reg.end()) reg.clear();
  reg[ws] = k;
}

void sched_forget(const void* ws) {
  std::lock_guard<std::mutex> lk(g_sched_mu);
  sched_registry().erase(ws);
}

bool sched_matches(const void* ws, const SchedKey& k) {
  std::lock_guard<std::mutex> lk(g_sched_mu);
  auto& reg = sched_registry();
  auto it = reg.find(ws);
  return it != reg.end() && it->second == k;
}

#define LSP_DISPATCH(spec, FN, ...)                                   \
  switch (spec) {                                                     \
    case kBccLinear: return lsp_host::FN<SplineBccLinear>(__VA_ARGS__); \
    case kCcZp: return lsp_host::FN<SplineCcZp>(__VA_ARGS__);           \
    case kBccQuartic: return lsp_host::FN<SplineBccQuartic>(__VA_ARGS__); \
    case kFcc6: return lsp_host::FN<SplineFcc6>(__VA_ARGS__);           \
    case kD4s8: return lsp_host::FN<SplineD4s8>(__VA_ARGS__);           \
    case kD48: return lsp_host::FN<SplineD48>(__VA_ARGS__);             \
    case kCcTp2: return lsp_host::FN<SplineCcTp2>(__VA_ARGS__);         \
    case kCcTp3: return lsp_host::FN<SplineCcTp3>(__VA_ARGS__);         \
    case kCcTp4: return lsp_host::FN<SplineCcTp4>(__VA_ARGS__);         \
    case kCcLinearRd: return lsp_host::FN<SplineCcLinearRd>(__VA_ARGS__); \
    case kBccQuinticRd: return lsp_host::FN<SplineBccQuinticRd>(__VA_ARGS__); \
    case kBccVoronoi1: return lsp_host::FN<SplineBccVoronoi1>(__VA_ARGS__); \
    case kFccVoronoi1: return lsp_host::FN<SplineFccVoronoi1>(__VA_ARGS__); \
    case kCcBccVoronoi1: return lsp_host::FN<SplineCcBccVoronoi1>(__VA_ARGS__); \
    case kCcFccVoronoi1: return lsp_host::FN<SplineCcFccVoronoi1>(__VA_ARGS__); \
    case kFccVoronoi2: return lsp_host::FN<SplineFccVoronoi2>(__VA_ARGS__); \
    case kCcFccVoronoi2: return lsp_host::FN<SplineCcFccVoronoi2>(__VA_ARGS__); \
  }                                                                   \
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
    case LSP_ERR_TOO_LARGE: return "the input needs more than the static scratch (LSP_STATIC_SCRATCH_BYTES)";
  }
  return "unknown status";
}

lsp_status lsp_plan_create(int32_t s, const int32_t* L, int32_t n, const int32_t* Xi, uint32_t flags,
                           lsp_plan* out) {
  (void)flags;
  if (!L || !Xi || !out) return LSP_ERR_NULL;
  *out = nullptr;
  if (s < 1 || s > 4 || n < s || n > 16) return LSP_ERR_INVALID;
  LatticeShape lat;
  if (!lattice_shape(s, L, lat)) return LSP_ERR_INVALID;
  std::vector<std::vector<int>> dirs;
  for (int j = 0; j < n; ++j) {
    std::vector<long long> v(s);
    std::vector<int> vi(s);
    for (int a = 0; a < s; ++a) { v[a] = Xi[a * n + j]; vi[a] = Xi[a * n + j]; }
    if (!on_lattice(lat.adj, lat.det, v)) return LSP_ERR_NOT_ON_LATTICE;
    dirs.push_back(canon_dir(vi));
  }
  // rank of Xi must be s
  {
    bool spans = false;
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
  for (int id = 0; id < kNumSpecs; ++id) {
    const SpecDesc& sd = specs()[id];
    if (sd.kind != 0 || sd.s != s || sd.ndir != n || sd.D != lat.D ||
        sd.M != static_cast<int>(lat.shifts.size()))
      continue;
    std::vector<std::vector<int>> sdirs;
    for (auto& dv : sd.dirs) sdirs.push_back(canon_dir(dv));
    std::sort(sdirs.begin(), sdirs.end());
    if (sdirs != dirs) continue;
    if (sd.shifts != lat.shifts) continue;
    return make_plan(id, out);
  }
  return LSP_ERR_UNSUPPORTED;
}

lsp_status lsp_plan_create_voronoi(int32_t s, const int32_t* L, const int32_t* Lv, int32_t n, uint32_t flags,
                                   lsp_plan* out) {
  (void)flags;
  if (!L || !Lv || !out) return LSP_ERR_NULL;
  *out = nullptr;
  if (s < 1 || s > 4 || n < 1) return LSP_ERR_INVALID;
  LatticeShape lat, vlat;
  if (!lattice_shape(s, L, lat) || !lattice_shape(s, Lv, vlat)) return LSP_ERR_INVALID;
  // L_v must be a sublattice of L (partition of unity on L)
  for (int c = 0; c < s; ++c) {
    std::vector<long long> v(s);
    for (int a = 0; a < s; ++a) v[a] = Lv[a * s + c];
    if (!on_lattice(lat.adj, lat.det, v)) return LSP_ERR_NOT_ON_LATTICE;
  }
  for (int id = 0; id < kNumSpecs; ++id) {
    const SpecDesc& sd = specs()[id];
    if (sd.kind != 1 || sd.s != s || sd.vor_n != n || sd.D != lat.D || sd.shifts != lat.shifts) continue;
    // same Voronoi lattice: equal |det| and every basis vector of either inside the other
    std::vector<int32_t> slv(s * s);
    for (int r = 0; r < s; ++r)
      for (int c = 0; c < s; ++c) slv[r * s + c] = static_cast<int32_t>(sd.vor_lv[r][c]);
    LatticeShape spec_v;
    if (!lattice_shape(s, slv.data(), spec_v) || spec_v.det != vlat.det) continue;
    bool same = true;
    for (int c = 0; c < s && same; ++c) {
      std::vector<long long> v(s);
      for (int a = 0; a < s; ++a) v[a] = Lv[a * s + c];
      same = on_lattice(spec_v.adj, spec_v.det, v);
    }
    if (!same) continue;
    return make_plan(id, out);
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
  for (int k = 0; k < sd.K && k < 16; ++k) {
    out->stencil[k] = sd.nsite[k];
    out->nnz[k] = sd.nnz[k];
    out->fma_b[k] = sd.fma_b[k];
    out->fma_w[k] = sd.fma_w[k];
  }
  out->grad_terms = sd.grad_terms;
  // every query gathers the same total over its cosets when K = 1; report the
  // sub-region-averaged total otherwise
  long long tot = 0;
  for (int v : sd.nsite) tot += v;
  out->lookups = static_cast<int32_t>((tot * sd.M + sd.K / 2) / sd.K);
  out->n_monomials = sd.nmon;
  out->offset_min = sd.omin; out->offset_max = sd.omax;
  std::strncpy(out->name, sd.name, sizeof(out->name) - 1);
  out->kind = sd.kind;
  out->voronoi_n = sd.vor_n;
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
  const int64_t esize = dtype == LSP_F64 ? 8 : (dtype == LSP_F32 ? 4 : 2);
  v->vol.bytes32 = total * esize < (int64_t(1) << 32) ? 1 : 0;
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
  if (n > kMaxQueries) return LSP_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  LSP_DISPATCH(plan->spec, eval_spec, vol, x, n, nullptr, f, grad_x, s)
}

lsp_status lsp_eval_mse(lsp_plan plan, lsp_vol vol, const float* x, const float* y, int64_t n, float* f,
                        float* dloss_df, float* dloss_dx, double* loss, void* stream) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (n < 0) return LSP_ERR_INVALID;
  if (n == 0) return LSP_OK;
  if (!x || !y || !loss) return LSP_ERR_NULL;
  if (vol->dtype == LSP_F64) return LSP_ERR_DTYPE;
  if (n > kMaxQueries) return LSP_ERR_INVALID;
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
  if (n > kMaxQueries) return LSP_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  LSP_DISPATCH(plan->spec, adj_spec, vol, x, g, n, nullptr, grad_c, grad_x, s, false)
}

lsp_status lsp_eval_rays(lsp_plan plan, lsp_vol vol, const float* c, const float* A, int32_t W, int32_t H,
                         int32_t steps, int64_t ray0, int64_t nrays, float* out, float* samples, void* stream) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (!c || !A) return LSP_ERR_NULL;
  if (W <= 0 || H <= 0 || (W & 7) || (H & 7) || steps <= 0 || ray0 < 0 || nrays < 0 ||
      ray0 + nrays > static_cast<int64_t>(W) * H || nrays > kMaxQueries)
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

lsp_status lsp_render(lsp_plan plan, lsp_vol vol, const float* c, const float* A, int32_t W, int32_t H,
                      int32_t steps, int64_t ray0, int64_t nrays, const float* tf,
                      const lsp_render_params* params, float* rgba, void* stream) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (!c || !A || !params) return LSP_ERR_NULL;
  if (W <= 0 || H <= 0 || (W & 7) || (H & 7) || steps <= 0 || ray0 < 0 || nrays < 0 ||
      ray0 + nrays > static_cast<int64_t>(W) * H || nrays > kMaxQueries)
    return LSP_ERR_INVALID;
  const lsp_render_params& p = *params;
  if (p.tf_len < 2 || !(p.f1 > p.f0) || !(p.grad_eps >= 0.f)) return LSP_ERR_INVALID;
  if (nrays == 0) return LSP_OK;
  if (!tf || !rgba) return LSP_ERR_NULL;
  if (reinterpret_cast<uintptr_t>(tf) & 15 || reinterpret_cast<uintptr_t>(rgba) & 15) return LSP_ERR_INVALID;
  if (vol->dtype == LSP_F64) return LSP_ERR_DTYPE;
  RayParams rp{};
  for (int a = 0; a < 3; ++a) rp.c[a] = c[a];
  for (int a = 0; a < 9; ++a) rp.A[a] = A[a];
  rp.W = W; rp.H = H; rp.steps = steps;
  RenderParams rd{};
  rd.f0 = p.f0; rd.f1 = p.f1; rd.ambient = p.ambient; rd.diffuse = p.diffuse; rd.grad_eps = p.grad_eps;
  rd.alpha_stop = p.alpha_stop; rd.tf_len = p.tf_len;
  hipStream_t s = static_cast<hipStream_t>(stream);
  LSP_DISPATCH(plan->spec, render_spec, vol, rp, rd, tf, ray0, nrays, rgba, s)
}

static lsp_status check_ws(lsp_plan plan, lsp_vol vol, int64_t n, const void* ws, size_t ws_bytes) {
  if (!ws) return LSP_ERR_NULL;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return LSP_ERR_INVALID;
  size_t need = 0;
  lsp_status st = lsp_schedule_size(plan, vol, n, &need);
  if (st != LSP_OK) return st;
  return ws_bytes >= need ? LSP_OK : LSP_ERR_INVALID;
}

// a *_scheduled call: the workspace must hold a schedule of these queries for
// this plan and a volume of the same dims and dtype class
static lsp_status check_sched(lsp_plan plan, lsp_vol vol, const float* x, int64_t n, const void* ws,
                              size_t ws_bytes) {
  lsp_status st = check_ws(plan, vol, n, ws, ws_bytes);
  if (st != LSP_OK) return st;
  return sched_matches(ws, sched_key(plan, vol, x, n)) ? LSP_OK : LSP_ERR_INVALID;
}

lsp_status lsp_schedule_size(lsp_plan plan, lsp_vol vol, int64_t n, size_t* bytes) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (!bytes) return LSP_ERR_NULL;
  if (n < 0 || n * specs()[plan->spec].M >= (int64_t(1) << 32)) return LSP_ERR_INVALID;
  LSP_DISPATCH(plan->spec, sched_size_spec, vol, n, bytes)
}

static lsp_status dispatch_schedule(lsp_plan plan, lsp_vol vol, const float* x, int64_t n, void* workspace,
                                    hipStream_t s) {
  LSP_DISPATCH(plan->spec, sched_spec, vol, x, n, workspace, s)
}

lsp_status lsp_schedule(lsp_plan plan, lsp_vol vol, const float* x, int64_t n, void* workspace, size_t ws_bytes,
                        void* stream) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (n < 0) return LSP_ERR_INVALID;
  if ((st = check_ws(plan, vol, n, workspace, ws_bytes)) != LSP_OK) return st;
  if (n > 0 && !x) return LSP_ERR_NULL;
  sched_forget(workspace);
  if (n > 0 && (st = dispatch_schedule(plan, vol, x, n, workspace, static_cast<hipStream_t>(stream))) != LSP_OK)
    return st;
  sched_record(workspace, sched_key(plan, vol, x, n));
  return LSP_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free schedule + evaluation: the workspace is `scratch`, a static
// device array.  Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, once per device, and is kept
// per device (every GPU holds its own copy of the array).
static __device__ __align__(256) unsigned char scratch[LSP_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on the first
// call on that device, with that device current)
lsp_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LSP_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LSP_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LSP_OK;
}
}  // namespace

static lsp_status static_need(lsp_plan plan, lsp_vol vol, int64_t n, size_t* bytes) {
  LSP_DISPATCH(plan->spec, sched_fwd_size_spec, vol, n, bytes)
}

lsp_status lsp_eval_scheduled_static(lsp_plan plan, lsp_vol vol, const float* x, int64_t n, void* f, void* grad_x,
                                     void* stream) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (n < 0) return LSP_ERR_INVALID;
  if (n == 0) return LSP_OK;
  if (!x || !f) return LSP_ERR_NULL;
  if (n * specs()[plan->spec].M >= (int64_t(1) << 32)) return LSP_ERR_INVALID;
  size_t need = 0;
  if ((st = static_need(plan, vol, n, &need)) != LSP_OK) return st;
  if (need > LSP_STATIC_SCRATCH_BYTES) return LSP_ERR_TOO_LARGE;
  void* ws = nullptr;
  if ((st = scratch_address(&ws)) != LSP_OK) return st;
  // the schedule writes every word of the workspace it later reads (key
  // histograms, scans, records, partials), so nothing needs clearing first
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = dispatch_schedule(plan, vol, x, n, ws, s)) != LSP_OK) return st;
  LSP_DISPATCH(plan->spec, eval_spec, vol, x, n, ws, f, grad_x, s)
}

lsp_status lsp_eval_scheduled(lsp_plan plan, lsp_vol vol, const float* x, int64_t n, const void* workspace,
                              size_t ws_bytes, void* f, void* grad_x, void* stream) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (n < 0) return LSP_ERR_INVALID;
  if ((st = check_sched(plan, vol, x, n, workspace, ws_bytes)) != LSP_OK) return st;
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
  if ((st = check_sched(plan, vol, x, n, workspace, ws_bytes)) != LSP_OK) return st;
  if (n == 0) return LSP_OK;
  if (!x || !y || !loss) return LSP_ERR_NULL;
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
  if ((st = check_sched(plan, vol, x, n, workspace, ws_bytes)) != LSP_OK) return st;
  if (n == 0) return LSP_OK;
  if (!x || !g || !grad_c) return LSP_ERR_NULL;
  const SpecDesc& sd = specs()[plan->spec];
  for (int k = 0; k < sd.M; ++k)
    if (!grad_c[k]) return LSP_ERR_NULL;
  if (vol->dtype == LSP_F64) return LSP_ERR_DTYPE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  LSP_DISPATCH(plan->spec, adj_spec, vol, x, g, n, workspace, grad_c, grad_x, s, false)
}

lsp_status lsp_mse_backward_scheduled(lsp_plan plan, lsp_vol vol, const float* x, int64_t n, const void* workspace,
                                      size_t ws_bytes, float* const* grad_c, void* stream) {
  lsp_status st = check_pv(plan, vol);
  if (st != LSP_OK) return st;
  if (n < 0) return LSP_ERR_INVALID;
  if ((st = check_sched(plan, vol, x, n, workspace, ws_bytes)) != LSP_OK) return st;
  if (n == 0) return LSP_OK;
  if (!x || !grad_c) return LSP_ERR_NULL;
  const SpecDesc& sd = specs()[plan->spec];
  for (int k = 0; k < sd.M; ++k)
    if (!grad_c[k]) return LSP_ERR_NULL;
  if (vol->dtype == LSP_F64) return LSP_ERR_DTYPE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  LSP_DISPATCH(plan->spec, adj_spec, vol, x, nullptr, n, workspace, grad_c, nullptr, s, true)
}

}  // extern "C"
