// HIP kernels (gfx950) for the fast evaluation of the lattice convolution sum
//     f(x) = sum_n c_n phi(x - n),   phi = |det L| M_Xi(. + c0)
// (Horacsek & Alim, Eq. conv_sum; the fast scheme of Sec. 4, Algorithm 1).
//
// One query per lane.  Per coset k (Sec. 4.1, Eq. coset_form):
//   1. shift into the coset cell: i = floor((x - l_k)/D), u = x - l_k - D i - D/2
//      (the map rho of Sec. 4.1 onto the region of evaluation [0, D)^s);
//   2. fold u by a signed permutation T of the spline's symmetry group into the
//      fundamental chamber (a sorting network on |u|; Sec. 4.3 symmetry
//      analysis, used here instead of the sigma table of Sec. 4.2);
//   3. select the sub-region from the few splitting planes left inside the
//      chamber (predicated compares, Sec. 4.2);
//   4. gather the sub-region's fixed stencil, renamed through T
//      (pi(n) = T^{-1}(n - 1/2) + 1/2, the rigid renaming of Sec. 4.3);
//   5. evaluate the sub-region's polynomial (generated straight-line code).
// The coset contributions are summed (Algorithm 1, outer loop).
//
// The gathers read the coefficient arrays directly through the cache
// hierarchy; the per-lane work is VALU FMAs.  No MFMA: the weights differ per
// query, there is no shared dense operand.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lsp {

// ----------------------------------------------------------------------------
// generated tables (one struct per spline)
#include "generated/bcc_linear.inc"
#include "generated/cc_zp.inc"
#include "generated/bcc_quartic.inc"
#include "generated/fcc_6dir.inc"
#include "generated/d4s_8dir.inc"
#include "generated/d4_8dir.inc"
#include "generated/cc_tp2.inc"
#include "generated/cc_tp3.inc"
#include "generated/cc_tp4.inc"
#include "generated/cc_linear_rd.inc"
#include "generated/bcc_quintic_rd.inc"
#include "generated/bcc_voronoi1.inc"
#include "generated/fcc_voronoi1.inc"
#include "generated/cc_bcc_voronoi1.inc"
#include "generated/cc_fcc_voronoi1.inc"
#include "generated/fcc_voronoi2.inc"
#include "generated/cc_fcc_voronoi2.inc"

constexpr int kMaxCosets = 8;
constexpr int kMaxDim = 4;

// Coefficient volume: one array per coset, same dims, x fastest.
struct Vol {
  const void* base[kMaxCosets];
  int dims[kMaxDim];
  int stride[kMaxDim];  // elements
  int bytes32;          // every coset array spans fewer than 2^32 bytes
};

struct GradVol {
  float* base[kMaxCosets];
};

// Select coset k's pointer / shift with a compare chain: k may differ per lane
// (coset-split work items), and a lane-indexed kernel-argument array would be
// copied to scratch memory.
template <int M, class P>
__device__ __forceinline__ P pick(const P* arr, int k) {
  P p = arr[0];
#pragma unroll
  for (int j = 1; j < M; ++j) p = (k == j) ? arr[j] : p;
  return p;
}

template <class SP>
__device__ __forceinline__ int coset_shift(int k, int d) {
  int v = SP::SHIFT[0][d];
#pragma unroll
  for (int j = 1; j < SP::M; ++j) v = (k == j) ? SP::SHIFT[j][d] : v;
  return v;
}

// ----------------------------------------------------------------------------
// coefficient storage types
struct bf16_t { uint16_t v; };
struct f16_t { _Float16 v; };

template <class CT, class AT> __device__ __forceinline__ AT load_coef(const CT* p);
template <> __device__ __forceinline__ float load_coef<float, float>(const float* p) { return *p; }
template <> __device__ __forceinline__ float load_coef<bf16_t, float>(const bf16_t* p) {
  return __uint_as_float(static_cast<uint32_t>(p->v) << 16);
}
template <> __device__ __forceinline__ float load_coef<f16_t, float>(const f16_t* p) {
  return static_cast<float>(p->v);
}
template <> __device__ __forceinline__ double load_coef<double, double>(const double* p) { return *p; }

// ----------------------------------------------------------------------------
// per-coset geometry of one query: cell index, folded point, folded strides
template <class SP, class AT>
struct Folded {
  int i[SP::S];       // cell index (coset array index of the cell origin)
  AT up[SP::S];       // folded offset from the cell centre, in the chamber
  int ax[SP::S];      // folded axis r comes from original axis ax[r]
  int sg[SP::S];      // and carries sign sg[r]: up[r] = sg[r] * u[ax[r]]
  int pi[SP::S];      // cell index along original axis ax[r]
  int neg;            // bit d: u[d] < 0 (original axis d)
  bool interior;      // the whole stencil lies inside the stored arrays
};

template <class AT> __device__ __forceinline__ AT afloor(AT v);
template <> __device__ __forceinline__ float afloor<float>(float v) { return floorf(v); }
template <> __device__ __forceinline__ double afloor<double>(double v) { return floor(v); }

// compare-exchange of the sorting network (positions are compile-time)
template <int P, int Q, class AT>
__device__ __forceinline__ void cswap(AT* v, int* ax, int* sg, int* pi) {
  const bool sw = v[P] < v[Q];
  const AT tv = sw ? v[Q] : v[P], uv = sw ? v[P] : v[Q];
  v[P] = tv; v[Q] = uv;
  const int ta = sw ? ax[Q] : ax[P], ua = sw ? ax[P] : ax[Q];
  ax[P] = ta; ax[Q] = ua;
  const int ts = sw ? sg[Q] : sg[P], us = sw ? sg[P] : sg[Q];
  sg[P] = ts; sg[Q] = us;
  const int tp = sw ? pi[Q] : pi[P], up = sw ? pi[P] : pi[Q];
  pi[P] = tp; pi[Q] = up;
}

// extent and element stride of original axis a (a varies per lane): selects
// between computed values, never an indexed array (which would live in
// scratch memory)
template <int S>
__device__ __forceinline__ int axis_stride(const int* dims, int a) {
  const int n0 = dims[0];
  const int n01 = n0 * dims[1];
  int s = (a == 1) ? n0 : 1;
  s = (a == 2) ? n01 : s;
  if constexpr (S == 4) s = (a == 3) ? n01 * dims[2] : s;
  return s;
}

template <int S>
__device__ __forceinline__ int axis_dim(const int* dims, int a) {
  const int n0 = dims[0], n1 = dims[1], n2 = dims[2];
  int n = (a == 1) ? n1 : n0;
  n = (a == 2) ? n2 : n;
  if constexpr (S == 4) n = (a == 3) ? dims[3] : n;
  return n;
}

template <class SP, class AT>
__device__ __forceinline__ void fold_query(const AT* x, int k, const Vol& vol, Folded<SP, AT>& F) {
  constexpr int S = SP::S;
  AT a[S];
  bool interior = true;
  int neg = 0;
#pragma unroll
  for (int d = 0; d < S; ++d) {
    AT xp = x[d] - AT(coset_shift<SP>(k, d));
    AT fl = afloor<AT>(xp * AT(1.0 / SP::D));
    // keep the index arithmetic in range for huge or non-finite queries
    fl = fl > AT(1 << 24) ? AT(1 << 24) : (fl < AT(-(1 << 24)) ? AT(-(1 << 24)) : fl);
    int id = (fl == fl) ? static_cast<int>(fl) : 0;   // NaN queries: any in-range cell
    AT u = (xp - AT(SP::D) * fl) - AT(0.5 * SP::D);
    F.i[d] = id;
    F.pi[d] = id;
    interior = interior && (id + SP::OMIN >= 0) && (id + SP::OMAX < vol.dims[d]);
    a[d] = u;
    F.ax[d] = d;
    F.sg[d] = (u >= AT(0)) ? 1 : -1;
    neg |= (u < AT(0)) ? (1 << d) : 0;
  }
  F.neg = neg;
  F.interior = interior;
  AT v[S];
#pragma unroll
  for (int d = 0; d < S; ++d) v[d] = a[d] < AT(0) ? -a[d] : a[d];
  // sorting network, descending on |u|, carrying axis and sign
  if constexpr (S == 3) {
    cswap<0, 1>(v, F.ax, F.sg, F.pi); cswap<1, 2>(v, F.ax, F.sg, F.pi); cswap<0, 1>(v, F.ax, F.sg, F.pi);
  } else {
    cswap<0, 1>(v, F.ax, F.sg, F.pi); cswap<2, 3>(v, F.ax, F.sg, F.pi); cswap<0, 2>(v, F.ax, F.sg, F.pi);
    cswap<1, 3>(v, F.ax, F.sg, F.pi); cswap<1, 2>(v, F.ax, F.sg, F.pi);
  }
  if constexpr (SP::FOLD_D) {
    // even sign changes only: an odd number of negative components leaves the
    // smallest folded coordinate negative
    int neg = 0;
#pragma unroll
    for (int d = 0; d < S; ++d) neg += (F.sg[d] < 0);
    if (neg & 1) { v[S - 1] = -v[S - 1]; F.sg[S - 1] = -F.sg[S - 1]; }
  }
#pragma unroll
  for (int d = 0; d < S; ++d) F.up[d] = v[d];
}

// The second coset of D Z^s u (D Z^s + (1,...,1)) with D = 2 (BCC; the B
// fold): per axis, u_1 = u_0 - 1 when u_0 >= 0 (same cell) and u_0 + 1 when
// u_0 < 0 (the cell below), so |u_1| = 1 - |u_0| and the sign flips.  The
// descending order of |u_1| is that of |u_0| reversed: coset 1's fold is read
// off coset 0's instead of recomputed.  Exact for |x| >= 1 (|u_0| is then a
// multiple of a power of two no finer than 2^-23).
template <class SP>
constexpr bool complement_coset() {
  if (SP::M != 2 || SP::D != 2 || SP::FOLD_D) return false;
  for (int d = 0; d < SP::S; ++d)
    if (SP::SHIFT[1][d] != 1) return false;
  return true;
}

template <class SP, class AT>
__device__ __forceinline__ void fold_complement(const Folded<SP, AT>& F0, const Vol& vol, Folded<SP, AT>& F1) {
  constexpr int S = SP::S;
  bool interior = true;
#pragma unroll
  for (int d = 0; d < S; ++d) {
    const int id = F0.i[d] - ((F0.neg >> d) & 1);
    F1.i[d] = id;
    interior = interior && (id + SP::OMIN >= 0) && (id + SP::OMAX < vol.dims[d]);
  }
  F1.interior = interior;
  F1.neg = ~F0.neg & ((1 << S) - 1);
#pragma unroll
  for (int r = 0; r < S; ++r) {
    F1.up[r] = AT(1) - F0.up[S - 1 - r];
    F1.ax[r] = F0.ax[S - 1 - r];
    F1.sg[r] = -F0.sg[S - 1 - r];
    // cell index along axis ax[r]: one lower where u_0 < 0 there (sg_0 < 0)
    F1.pi[r] = F0.pi[S - 1 - r] - (F0.sg[S - 1 - r] < 0 ? 1 : 0);
  }
}

// Gather through the fold: folded site J maps to original offset
// o[ax[r]] = J[r] if sg[r] > 0 else 1 - J[r].
template <class SP, class CT, class AT, bool CHECK>
struct Gather {
  const CT* origin;   // array element of folded site J = 0
  const CT* safe;     // any valid element (used for masked loads)
  int st[SP::S];      // folded signed strides
  int jlo[SP::S], jhi[SP::S];  // CHECK: valid J range per folded axis

  __device__ __forceinline__ void init(const Vol& vol, int k, const Folded<SP, AT>& F) {
    const CT* base = static_cast<const CT*>(pick<SP::M>(vol.base, k));
    safe = base;
    long long off = 0;
#pragma unroll
    for (int d = 0; d < SP::S; ++d) off += static_cast<long long>(F.i[d]) * vol.stride[d];
#pragma unroll
    for (int r = 0; r < SP::S; ++r) {
      const int a = F.ax[r];
      const int s = axis_stride<SP::S>(vol.dims, a);
      st[r] = F.sg[r] > 0 ? s : -s;
      if (F.sg[r] < 0) off += s;
      if constexpr (CHECK) {
        const int ia = F.pi[r], n = axis_dim<SP::S>(vol.dims, a);
        // sg > 0: 0 <= ia + J < n ; sg < 0: 0 <= ia + 1 - J < n
        jlo[r] = F.sg[r] > 0 ? -ia : ia + 2 - n;
        jhi[r] = F.sg[r] > 0 ? n - 1 - ia : ia + 1;
      }
    }
    origin = base + off;
  }

  template <int J0, int J1, int J2, int J3 = 0>
  __device__ __forceinline__ AT c() const {
    constexpr int J[4] = {J0, J1, J2, J3};
    int off = 0;
#pragma unroll
    for (int r = 0; r < SP::S; ++r) off += J[r] * st[r];
    if constexpr (CHECK) {
      bool ok = true;
#pragma unroll
      for (int r = 0; r < SP::S; ++r) ok = ok && (J[r] >= jlo[r]) && (J[r] <= jhi[r]);
      const CT* p = ok ? origin + off : safe;
      AT v = load_coef<CT, AT>(p);
      return ok ? v : AT(0);
    } else {
      return load_coef<CT, AT>(origin + off);
    }
  }
};

// Interior gather with 32-bit byte offsets from the coset's base: per folded
// axis the multiples J st_r (bytes) are tabulated once per query, so a site's
// address is one three-input add, taken by the load as a 32-bit offset to a
// base that is uniform over the wave.  Needs every coset array below 4 GiB
// and the whole stencil inside the array (interior queries).
template <class SP, class CT, class AT>
struct GatherInterior {
  static constexpr int JLO = SP::OMIN < 1 - SP::OMAX ? SP::OMIN : 1 - SP::OMAX;
  static constexpr int JHI = SP::OMAX > 1 - SP::OMIN ? SP::OMAX : 1 - SP::OMIN;
  static constexpr int NJ = JHI - JLO + 1;
  const char* base;
  unsigned p[SP::S][NJ];   // p[r][J - JLO] = J st_r bytes; axis 0 also carries the origin

  __device__ __forceinline__ void init(const Vol& vol, int k, const Folded<SP, AT>& F) {
    base = static_cast<const char*>(pick<SP::M>(vol.base, k));
    int off = 0;
#pragma unroll
    for (int d = 0; d < SP::S; ++d) off += F.i[d] * vol.stride[d];
    int st[SP::S];
#pragma unroll
    for (int r = 0; r < SP::S; ++r) {
      const int sa = axis_stride<SP::S>(vol.dims, F.ax[r]);
      st[r] = F.sg[r] > 0 ? sa : -sa;
      if (F.sg[r] < 0) off += sa;
    }
#pragma unroll
    for (int r = 0; r < SP::S; ++r) {
      const unsigned step = static_cast<unsigned>(st[r]) * static_cast<unsigned>(sizeof(CT));
      p[r][-JLO] = r == 0 ? static_cast<unsigned>(off) * static_cast<unsigned>(sizeof(CT)) : 0u;
#pragma unroll
      for (int j = -JLO + 1; j < NJ; ++j) p[r][j] = p[r][j - 1] + step;
#pragma unroll
      for (int j = -JLO - 1; j >= 0; --j) p[r][j] = p[r][j + 1] - step;
    }
  }
  template <int J0, int J1, int J2, int J3 = 0>
  __device__ __forceinline__ AT c() const {
    unsigned a = p[0][J0 - JLO] + p[1][J1 - JLO] + p[2][J2 - JLO];
    if constexpr (SP::S == 4) a += p[3][J3 - JLO];
    return load_coef<CT, AT>(reinterpret_cast<const CT*>(base + a));
  }
};

// Scatter-add of g * w_j into the gradient volume (adjoint, FP32 atomics).
template <class SP, bool CHECK>
struct Scatter {
  float* origin;
  int st[SP::S];
  int jlo[SP::S], jhi[SP::S];
  float g;

  __device__ __forceinline__ void init(const Vol& vol, float* base, const Folded<SP, float>& F, float gq) {
    long long off = 0;
#pragma unroll
    for (int d = 0; d < SP::S; ++d) off += static_cast<long long>(F.i[d]) * vol.stride[d];
#pragma unroll
    for (int r = 0; r < SP::S; ++r) {
      const int a = F.ax[r];
      const int s = axis_stride<SP::S>(vol.dims, a);
      st[r] = F.sg[r] > 0 ? s : -s;
      if (F.sg[r] < 0) off += s;
      if constexpr (CHECK) {
        const int ia = F.pi[r], n = axis_dim<SP::S>(vol.dims, a);
        jlo[r] = F.sg[r] > 0 ? -ia : ia + 2 - n;
        jhi[r] = F.sg[r] > 0 ? n - 1 - ia : ia + 1;
      }
    }
    origin = base + off;
    g = gq;
  }

  template <int J0, int J1, int J2, int J3 = 0>
  __device__ __forceinline__ void put(float w) {
    constexpr int J[4] = {J0, J1, J2, J3};
    int off = 0;
#pragma unroll
    for (int r = 0; r < SP::S; ++r) off += J[r] * st[r];
    if constexpr (CHECK) {
      bool ok = true;
#pragma unroll
      for (int r = 0; r < SP::S; ++r) ok = ok && (J[r] >= jlo[r]) && (J[r] <= jhi[r]);
      if (ok) atomicAdd(origin + off, g * w);
    } else {
      atomicAdd(origin + off, g * w);
    }
  }
};

// monomials of the folded point about the sub-region's origin (a chamber
// vertex chosen by the generator for the sparsest polynomials)
template <class SP, class AT>
__device__ __forceinline__ void monomials(const AT* up, int ob, AT* mono) {
  AT z[SP::S];
#pragma unroll
  for (int d = 0; d < SP::S; ++d) z[d] = up[d] - SP::template origin<AT>(ob, d);
  mono[0] = AT(1);
#pragma unroll
  for (int m = 1; m < SP::NMON; ++m) mono[m] = mono[SP::MPARENT[m]] * z[SP::MVAR[m]];
}

// psi and, optionally, its gradient in the folded frame from b and the monomials
template <class SP, class AT, bool GRAD>
__device__ __forceinline__ AT poly_eval(const AT* b, const AT* mono, AT* dpsi) {
  AT psi = AT(0);
#pragma unroll
  for (int m = 0; m < SP::NMON; ++m) psi = fma(b[m], mono[m], psi);
  if constexpr (GRAD) {
#pragma unroll
    for (int r = 0; r < SP::S; ++r) {
      AT acc = AT(0);
#pragma unroll
      for (int m = 0; m < SP::NMON; ++m) {
        if (SP::MDER[m][r] >= 0) acc = fma(b[m] * AT(SP::MONO[m][r]), mono[SP::MDER[m][r]], acc);
      }
      dpsi[r] = acc;
    }
  }
  return psi;
}

// folded-frame gradient back to the original frame: up[r] = sg[r] u[ax[r]],
// so d/du[ax[r]] = sg[r] d/dup[r]
template <class SP, class AT>
__device__ __forceinline__ void unfold_grad(const Folded<SP, AT>& F, const AT* dpsi, AT* gx) {
  AT w[SP::S];
#pragma unroll
  for (int r = 0; r < SP::S; ++r) w[r] = F.sg[r] > 0 ? dpsi[r] : -dpsi[r];
#pragma unroll
  for (int d = 0; d < SP::S; ++d) {
    AT v = w[SP::S - 1];
#pragma unroll
    for (int r = SP::S - 2; r >= 0; --r) v = (F.ax[r] == d) ? w[r] : v;
    gx[d] += v;
  }
}

// one coset's contribution (value, and gradient in the original frame) from
// its folded geometry
template <class SP, class CT, class AT, bool GRAD>
__device__ __forceinline__ void coset_contrib_folded(const Vol& vol, int k, const Folded<SP, AT>& F, AT& f, AT* gx) {
  const int ob = SP::template orbit<AT>(F.up);
  AT b[SP::NMON];
  if (F.interior && vol.bytes32) {
    GatherInterior<SP, CT, AT> g;
    g.init(vol, k, F);
    SP::template b_any<AT>(ob, g, b);
  } else if (F.interior) {
    Gather<SP, CT, AT, false> g;
    g.init(vol, k, F);
    SP::template b_any<AT>(ob, g, b);
  } else {
    Gather<SP, CT, AT, true> g;
    g.init(vol, k, F);
    SP::template b_any<AT>(ob, g, b);
  }
  AT mono[SP::NMON];
  monomials<SP, AT>(F.up, ob, mono);
  AT dpsi[SP::S];
  f += poly_eval<SP, AT, GRAD>(b, mono, dpsi);
  if constexpr (GRAD) unfold_grad<SP, AT>(F, dpsi, gx);
}

template <class SP, class CT, class AT, bool GRAD>
__device__ __forceinline__ void coset_contrib(const Vol& vol, int k, const AT* xq, AT& f, AT* gx) {
  Folded<SP, AT> F;
  fold_query<SP, AT>(xq, k, vol, F);
  coset_contrib_folded<SP, CT, AT, GRAD>(vol, k, F, f, gx);
}

// every coset of one query (Algorithm 1, outer loop)
template <class SP, class CT, class AT, bool GRAD>
__device__ __forceinline__ void all_cosets(const Vol& vol, const AT* xq, AT& f, AT* gx) {
  if constexpr (complement_coset<SP>()) {
    Folded<SP, AT> F0, F1;
    fold_query<SP, AT>(xq, 0, vol, F0);
    coset_contrib_folded<SP, CT, AT, GRAD>(vol, 0, F0, f, gx);
    fold_complement<SP, AT>(F0, vol, F1);
    coset_contrib_folded<SP, CT, AT, GRAD>(vol, 1, F1, f, gx);
  } else {
#pragma unroll
    for (int k = 0; k < SP::M; ++k) coset_contrib<SP, CT, AT, GRAD>(vol, k, xq, f, gx);
  }
}

// adjoint of one coset: scatter g * w_j into the gradient volume, and (GRADX)
// accumulate the folded-frame gradient of psi mapped back to x
template <class SP, class CT, bool GRADX>
__device__ __forceinline__ void coset_adjoint(const Vol& vol, const GradVol& gvol, int k, const float* xq,
                                              float gq, float* gx) {
  Folded<SP, float> F;
  fold_query<SP, float>(xq, k, vol, F);
  const int ob = SP::template orbit<float>(F.up);
  float mono[SP::NMON];
  monomials<SP, float>(F.up, ob, mono);
  float* gbase = pick<SP::M>(gvol.base, k);
  if (F.interior) {
    Scatter<SP, false> sc;
    sc.init(vol, gbase, F, gq);
    SP::template w_any<float>(ob, sc, mono);
  } else {
    Scatter<SP, true> sc;
    sc.init(vol, gbase, F, gq);
    SP::template w_any<float>(ob, sc, mono);
  }
  if constexpr (GRADX) {
    float b[SP::NMON];
    if (F.interior) {
      Gather<SP, CT, float, false> g;
      g.init(vol, k, F);
      SP::template b_any<float>(ob, g, b);
    } else {
      Gather<SP, CT, float, true> g;
      g.init(vol, k, F);
      SP::template b_any<float>(ob, g, b);
    }
    float dpsi[SP::S];
    (void)poly_eval<SP, float, true>(b, mono, dpsi);
    unfold_grad<SP, float>(F, dpsi, gx);
  }
}

// ----------------------------------------------------------------------------
// Work items.  Without a schedule item t is query t.  With a schedule
// (counting sort, below) perm[t] names the item: a query (all cosets in one
// lane), or, when the spline has several sub-regions (SPLIT), one
// (query, coset) pair q * M + k, so that a wave holds one sub-region.
template <class SP, bool SPLIT>
__device__ __forceinline__ void item_of(long long t, const unsigned* perm, long long& q, int& k) {
  const long long it = perm ? static_cast<long long>(perm[t]) : t;
  if constexpr (SPLIT) {
    q = it / SP::M;
    k = static_cast<int>(it - q * SP::M);
  } else {
    q = it;
    k = 0;
  }
}

// forward: f (and grad) at N queries, x as N x S float32 (row-major).
// SPLIT: f and grad must be zero on entry; lanes add their coset's share.
template <class SP, class CT, class AT, bool GRAD, bool SPLIT>
__global__ void __launch_bounds__(256) k_eval(Vol vol, const float* __restrict__ x, long long n_items,
                                              const unsigned* __restrict__ perm, AT* __restrict__ f,
                                              AT* __restrict__ grad) {
  const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_items) return;
  long long q;
  int k;
  item_of<SP, SPLIT>(t, perm, q, k);
  AT xq[SP::S];
#pragma unroll
  for (int d = 0; d < SP::S; ++d) xq[d] = static_cast<AT>(x[q * SP::S + d]);
  AT acc = AT(0);
  AT gx[SP::S];
#pragma unroll
  for (int d = 0; d < SP::S; ++d) gx[d] = AT(0);
  if constexpr (SPLIT) {
    coset_contrib<SP, CT, AT, GRAD>(vol, k, xq, acc, gx);
    atomicAdd(f + q, acc);
    if constexpr (GRAD) {
#pragma unroll
      for (int d = 0; d < SP::S; ++d) atomicAdd(grad + q * SP::S + d, gx[d]);
    }
  } else {
    all_cosets<SP, CT, AT, GRAD>(vol, xq, acc, gx);
    f[q] = acc;
    if constexpr (GRAD) {
#pragma unroll
      for (int d = 0; d < SP::S; ++d) grad[q * SP::S + d] = gx[d];
    }
  }
}

// mean-squared-error head on a complete f: dL/df = 2 (f - y) / N, L += sum (f - y)^2 / N
__device__ __forceinline__ void mse_reduce(float r2, double inv_n, double* loss) {
  // every thread of the block calls this: wave sums, then one atomic per block
  __shared__ float wave_sum[16];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) r2 += __shfl_xor(r2, o, 64);
  if ((threadIdx.x & 63) == 0) wave_sum[threadIdx.x >> 6] = r2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (unsigned w = 0; w < (blockDim.x + 63) / 64; ++w) tot += static_cast<double>(wave_sum[w]);
    atomicAdd(loss, tot * inv_n);
  }
}

// forward fused with the MSE head (whole queries per lane); GRAD also writes
// dL/dx = dL/df * grad f
template <class SP, class CT, bool GRAD>
__global__ void __launch_bounds__(256) k_eval_mse(Vol vol, const float* __restrict__ x, const float* __restrict__ y,
                                                  long long n, float inv_n, float* __restrict__ f,
                                                  float* __restrict__ dldf, float* __restrict__ dldx,
                                                  double* __restrict__ loss) {
  const long long q = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  float r2 = 0.f;
  if (q < n) {
    float xq[SP::S];
#pragma unroll
    for (int d = 0; d < SP::S; ++d) xq[d] = x[q * SP::S + d];
    float acc = 0.f;
    float gx[SP::S];
#pragma unroll
    for (int d = 0; d < SP::S; ++d) gx[d] = 0.f;
    all_cosets<SP, CT, float, GRAD>(vol, xq, acc, gx);
    const float r = acc - y[q];
    const float dl = 2.f * r * inv_n;
    if (f) f[q] = acc;      // optional
    if (dldf) dldf[q] = dl;
    if constexpr (GRAD) {
#pragma unroll
      for (int d = 0; d < SP::S; ++d) dldx[q * SP::S + d] = dl * gx[d];
    }
    r2 = r * r;
  }
  mse_reduce(r2, static_cast<double>(inv_n), loss);
}

// adjoint: grad_c[site] += g_q * w_site(x_q) (scatter-add), grad_x = g_q * grad f.
// SPLIT: grad_x must be zero on entry.
template <class SP, class CT, bool GRADX, bool SPLIT>
__global__ void __launch_bounds__(256) k_adjoint(Vol vol, GradVol gvol, const float* __restrict__ x,
                                                 const float* __restrict__ gout, long long n_items,
                                                 const unsigned* __restrict__ perm, float* __restrict__ grad_x) {
  const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_items) return;
  long long q;
  int k;
  item_of<SP, SPLIT>(t, perm, q, k);
  float xq[SP::S];
#pragma unroll
  for (int d = 0; d < SP::S; ++d) xq[d] = x[q * SP::S + d];
  const float gq = gout[q];
  float gx[SP::S];
#pragma unroll
  for (int d = 0; d < SP::S; ++d) gx[d] = 0.f;
  if constexpr (SPLIT) {
    coset_adjoint<SP, CT, GRADX>(vol, gvol, k, xq, gq, gx);
    if constexpr (GRADX) {
#pragma unroll
      for (int d = 0; d < SP::S; ++d) atomicAdd(grad_x + q * SP::S + d, gq * gx[d]);
    }
  } else {
#pragma unroll
    for (int kk = 0; kk < SP::M; ++kk) coset_adjoint<SP, CT, GRADX>(vol, gvol, kk, xq, gq, gx);
    if constexpr (GRADX) {
#pragma unroll
      for (int d = 0; d < SP::S; ++d) grad_x[q * SP::S + d] = gq * gx[d];
    }
  }
}

// ----------------------------------------------------------------------------
// small utility kernels
template <class T>
__global__ void __launch_bounds__(256) k_fill_zero(T* __restrict__ p, long long n) {
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    p[i] = T(0);
}

// exclusive scan, three launches: per-1024 block scans, a scan of the block
// totals (at most 1024 blocks), and the block offsets added back
constexpr int kScanBlock = 1024;

__device__ __forceinline__ unsigned block_exclusive_scan(unsigned v, unsigned* lds, unsigned& total) {
  // 256 threads
  const int tid = threadIdx.x;
  lds[tid] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    unsigned add = tid >= off ? lds[tid - off] : 0u;
    __syncthreads();
    lds[tid] += add;
    __syncthreads();
  }
  total = lds[255];
  const unsigned incl = lds[tid];
  __syncthreads();
  return incl - v;
}

template <int = 0>
__global__ void __launch_bounds__(256) k_scan_blocks(const unsigned* __restrict__ in, unsigned* __restrict__ out,
                                                     unsigned* __restrict__ partial, unsigned n) {
  __shared__ unsigned lds[256];
  const unsigned base = blockIdx.x * kScanBlock + threadIdx.x * 4;
  unsigned v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = (base + j < n) ? in[base + j] : 0u;
  const unsigned sum = v[0] + v[1] + v[2] + v[3];
  unsigned total;
  unsigned run = block_exclusive_scan(sum, lds, total);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

template <int = 0>
__global__ void __launch_bounds__(256) k_scan_top(unsigned* __restrict__ partial, unsigned nblocks) {
  __shared__ unsigned lds[256];
  const unsigned base = threadIdx.x * 4;
  unsigned v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = (base + j < nblocks) ? partial[base + j] : 0u;
  unsigned total;
  unsigned run = block_exclusive_scan(v[0] + v[1] + v[2] + v[3], lds, total);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (base + j < nblocks) partial[base + j] = run;
    run += v[j];
  }
}

template <int = 0>
__global__ void __launch_bounds__(256) k_scan_add(unsigned* __restrict__ out, const unsigned* __restrict__ partial,
                                                  unsigned n) {
  const unsigned add = partial[blockIdx.x];
  const unsigned base = blockIdx.x * kScanBlock + threadIdx.x * 4;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (base + j < n) out[base + j] += add;
}

// Ray-marched samples (orthographic): sample (ray r, step j) is at
//   p = c + A t,  t = ((2u+1)/W - 1, (2v+1)/H - 1, (2j+1)/S - 1)
// with pixel (u, v) from the ray index in 8x8 tiles (one wave per tile).
// Per ray: sum of f and of grad f over the steps (4 floats); optionally every
// sample's f and grad f (4 floats each).
struct RayParams {
  float c[3];
  float A[9];   // row-major 3x3
  int W, H, steps;
};

__device__ __forceinline__ void ray_pixel(long long r, int W, int& u, int& v) {
  const long long tile = r >> 6;
  const int within = static_cast<int>(r & 63);
  const int tiles_x = W >> 3;
  u = static_cast<int>(tile % tiles_x) * 8 + (within & 7);
  v = static_cast<int>(tile / tiles_x) * 8 + (within >> 3);
}

template <class SP, class CT>
__global__ void __launch_bounds__(256) k_rays(Vol vol, RayParams rp, long long ray0, long long nrays,
                                              float* __restrict__ out, float* __restrict__ samples) {
  static_assert(SP::S == 3, "rays are 3-D");
  const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nrays) return;
  const long long r = ray0 + t;
  int pu, pv;
  ray_pixel(r, rp.W, pu, pv);
  // exact in float32: (2u+1)/W - 1 for power-of-two W
  const float tu = __fsub_rn(__fmul_rn(static_cast<float>(2 * pu + 1), 1.0f / rp.W), 1.0f);
  const float tv = __fsub_rn(__fmul_rn(static_cast<float>(2 * pv + 1), 1.0f / rp.H), 1.0f);
  float base[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    base[a] = __fadd_rn(__fadd_rn(rp.c[a], __fmul_rn(rp.A[3 * a + 0], tu)), __fmul_rn(rp.A[3 * a + 1], tv));
  float sf = 0.f, sg0 = 0.f, sg1 = 0.f, sg2 = 0.f;
  const float invs = 1.0f / rp.steps;
  for (int j = 0; j < rp.steps; ++j) {
    const float tj = __fsub_rn(__fmul_rn(static_cast<float>(2 * j + 1), invs), 1.0f);
    float xq[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xq[a] = __fadd_rn(base[a], __fmul_rn(rp.A[3 * a + 2], tj));
    float f = 0.f;
    float gx[3] = {0.f, 0.f, 0.f};
    all_cosets<SP, CT, float, true>(vol, xq, f, gx);
    sf += f; sg0 += gx[0]; sg1 += gx[1]; sg2 += gx[2];
    if (samples) {
      float* o = samples + (t * rp.steps + j) * 4;
      o[0] = f; o[1] = gx[0]; o[2] = gx[1]; o[3] = gx[2];
    }
  }
  out[t * 4 + 0] = sf; out[t * 4 + 1] = sg0; out[t * 4 + 2] = sg1; out[t * 4 + 3] = sg2;
}

// Volume rendering around the ray sampler: every sample's f picks an RGBA
// value from a transfer function (tf_len entries spanning [f0, f1], linear
// between entries, clamped at the ends); its colour is shaded with the
// gradient as a normal under a light along the viewing direction d,
//   shade = ambient + diffuse |grad f . d| / |grad f|   (ambient + diffuse
//   where |grad f| <= grad_eps), and the samples are composited front to
// back (sample 0 is nearest the viewer):
//   C += (1 - A) alpha shade rgb,  A += (1 - A) alpha,
// stopping once A >= alpha_stop.
struct RenderParams {
  float f0, f1;
  float ambient, diffuse;
  float grad_eps;
  float alpha_stop;
  int tf_len;
};

template <class SP, class CT>
__global__ void __launch_bounds__(256) k_render(Vol vol, RayParams rp, RenderParams rd,
                                                const float4* __restrict__ tf, long long ray0, long long nrays,
                                                float4* __restrict__ out) {
  static_assert(SP::S == 3, "rays are 3-D");
  const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nrays) return;
  const long long r = ray0 + t;
  int pu, pv;
  ray_pixel(r, rp.W, pu, pv);
  const float tu = __fsub_rn(__fmul_rn(static_cast<float>(2 * pu + 1), 1.0f / rp.W), 1.0f);
  const float tv = __fsub_rn(__fmul_rn(static_cast<float>(2 * pv + 1), 1.0f / rp.H), 1.0f);
  float base[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    base[a] = __fadd_rn(__fadd_rn(rp.c[a], __fmul_rn(rp.A[3 * a + 0], tu)), __fmul_rn(rp.A[3 * a + 1], tv));
  float dv[3] = {rp.A[2], rp.A[5], rp.A[8]};
  const float dn = 1.0f / sqrtf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
#pragma unroll
  for (int a = 0; a < 3; ++a) dv[a] *= dn;
  const float tscale = static_cast<float>(rd.tf_len - 1) / (rd.f1 - rd.f0);
  const float tmax = static_cast<float>(rd.tf_len - 1);
  float c0 = 0.f, c1 = 0.f, c2 = 0.f, acc = 0.f;
  const float invs = 1.0f / rp.steps;
  for (int j = 0; j < rp.steps && acc < rd.alpha_stop; ++j) {
    const float tj = __fsub_rn(__fmul_rn(static_cast<float>(2 * j + 1), invs), 1.0f);
    float xq[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xq[a] = __fadd_rn(base[a], __fmul_rn(rp.A[3 * a + 2], tj));
    float f = 0.f;
    float gx[3] = {0.f, 0.f, 0.f};
    all_cosets<SP, CT, float, true>(vol, xq, f, gx);
    float sidx = (f - rd.f0) * tscale;
    sidx = fminf(fmaxf(sidx, 0.f), tmax);       // also maps NaN to 0
    const int i = min(static_cast<int>(sidx), rd.tf_len - 2);
    const float w = sidx - static_cast<float>(i);
    const float4 lo = tf[i], hi = tf[i + 1];
    const float gn = sqrtf(gx[0] * gx[0] + gx[1] * gx[1] + gx[2] * gx[2]);
    const float cosv = fabsf(gx[0] * dv[0] + gx[1] * dv[1] + gx[2] * dv[2]);
    const float shade = rd.ambient + rd.diffuse * (gn > rd.grad_eps ? cosv / gn : 1.0f);
    const float alpha = lo.w + w * (hi.w - lo.w);
    const float wgt = (1.0f - acc) * alpha;
    c0 += wgt * shade * (lo.x + w * (hi.x - lo.x));
    c1 += wgt * shade * (lo.y + w * (hi.y - lo.y));
    c2 += wgt * shade * (lo.z + w * (hi.z - lo.z));
    acc += wgt;
  }
  out[t] = make_float4(c0, c1, c2, acc);
}

}  // namespace lsp
