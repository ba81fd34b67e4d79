// Binned evaluation of random queries (gfx950).
//
// The fast scheme of Sec. 4 evaluates each query from a fixed stencil of
// coefficients around its cell.  For queries in random order the stencils of
// neighbouring lanes are unrelated and every gather misses the caches.  The
// paper points out that combining the reads of one coset exploits data
// locality (Sec. 4, memory layout); here the queries are binned by brick of
// cells first, and one workgroup evaluates one brick:
//
//   1. k_bin_hist   per tile of items, an LDS histogram of item keys;
//   2. k_bin_colscan + exclusive scan: the start of every key's run and of
//      every (tile, key) sub-run in the key-sorted order;
//   3. k_bin_place  per tile, LDS cursors place each item's record
//      (query coordinates + item id) at its sorted position; a tile's items of
//      one key land contiguously.  For 3-D splines with few keys
//      k_bin_place_win first sorts windows of the tile by key in LDS, so that
//      each key's records of a window leave as one contiguous run;
//   4. k_eval_binned: one workgroup per unit (a brick, or a (brick, coset)
//      pair for coset-split items) stages the unit's coefficients (plus the
//      stencil halo, zero outside the volume) into LDS with coalesced loads,
//      then evaluates its queries from LDS;
//   5. k_adjoint_binned + k_adjoint_gather: the adjoint accumulates the
//      scatter-add g * w into an LDS copy of the unit's region, in 64-bit
//      fixed point scaled by a power of two from max |g| (k_absmax_*), and
//      stores it as floats with plain coalesced writes to the unit's private
//      slot; a gather pass then sums, for every site, the (at most 2^s) unit
//      regions covering it.  No global atomics, no float atomics, and the
//      result does not depend on the order of the additions.
//
// key = unit * kpb + sub-region, unit = brick (linear, x fastest) * upb + coset:
// for splines whose several sub-regions (after the fold) carry costly
// polynomials a work item is one (query, coset) pair and the items of a unit
// are grouped by sub-region, so a wave runs one polynomial set instead of
// predicating all of them (Sec. 4.3).  Per-coset results go to partial
// buffers and are summed by a combine kernel.
#pragma once

namespace lsp {

struct BinGeom {
  int bshift;           // brick edge B = 1 << bshift cells per axis
  int nb[kMaxDim];      // bricks per axis
  unsigned nbricks;
  int upb;              // units per brick: M for coset-split items, else 1
  unsigned nunits;      // nbricks * upb
  int kpb;              // keys per unit: K for coset-split items, else 1
  unsigned okey;        // nunits * kpb: the outlier key (queries outside the brick grid)
  unsigned nkeys;       // okey + 1
  int tiles;            // histogram tiles
  long long tile_items;
  long long n;          // queries
  long long items;      // work items (n, or n * M when split)
  unsigned wpu;         // evaluation workgroups per unit (several when units are few)
};

// Work items are (query, coset) pairs, grouped by sub-region, when the spline
// has several sub-regions with costly polynomials; cheap ones are evaluated
// per query with the sub-region branch left to diverge.
template <class SP>
struct SplitPolicy {
  static constexpr int avg_nnz() {
    int t = 0;
    for (int k = 0; k < SP::K; ++k) t += SP::NNZ[k];
    return t / SP::K;
  }
  // costly pieces, or many sub-regions (a wave of whole queries would run
  // most of them): one (query, coset) item per lane, keyed by sub-region
  static constexpr bool value = SP::K > 1 && (avg_nnz() >= 200 || SP::K >= 8);
};

template <int S> struct Rec;
template <> struct Rec<3> { float4 a; };             // x0 x1 x2 | item
template <> struct Rec<4> { float4 a; uint4 b; };    // x0..x3 | item

template <class SP> struct Staged {
  // Per coset the staged cells are [b B - MARGIN + OMIN, b B + B - 1 + OMAX]
  // per axis.  A whole-query item is binned by its coset-0 cell, and another
  // coset's cell index can be one less (MARGIN = 1); a (query, coset) item is
  // binned by its own coset's cell, and a one-coset lattice has no other
  // coset (MARGIN = 0).
  static constexpr int MARGIN = (SplitPolicy<SP>::value || SP::M == 1) ? 0 : 1;
  __host__ __device__ static constexpr int width(int B) { return B + MARGIN + SP::OMAX - SP::OMIN; }
  __host__ __device__ static constexpr int volume(int B) {
    int v = 1;
    for (int d = 0; d < SP::S; ++d) v *= width(B);
    return v;
  }
};

template <class SP, bool SPLIT>
__device__ __forceinline__ void split_item(long long t, long long& q, int& k) {
  if constexpr (SPLIT) {
    q = t / SP::M;
    k = static_cast<int>(t - q * SP::M);
  } else {
    q = t;
    k = 0;
  }
}

// cell index of coset k for query x (as fold_query computes it)
template <class SP>
__device__ __forceinline__ int cell_of(const float* xq, int k, int d) {
  float fl = floorf((xq[d] - static_cast<float>(coset_shift<SP>(k, d))) * (1.0f / SP::D));
  fl = fl > 1e7f ? 1e7f : (fl < -1e7f ? -1e7f : fl);
  return (fl == fl) ? static_cast<int>(fl) : 0;
}

// An item's key: its unit and sub-region, or the outlier key when its cell
// lies outside the brick grid.  Inside it, the item's stencil (every coset's,
// for a whole query) lies in the unit's staged region, so the unit kernels
// need no global-memory path.
template <class SP, bool SPLIT>
__device__ __forceinline__ unsigned item_key(const Vol& vol, const BinGeom& g, const float* xq, int k) {
  unsigned brick = 0, mul = 1;
  bool inside = true;
#pragma unroll
  for (int d = 0; d < SP::S; ++d) {
    const int b = cell_of<SP>(xq, k, d) >> g.bshift;
    inside = inside && b >= 0 && b < g.nb[d];
    brick += static_cast<unsigned>(b) * mul;
    mul *= static_cast<unsigned>(g.nb[d]);
  }
  if (!inside) return g.okey;
  const unsigned unit = brick * static_cast<unsigned>(g.upb) + (SPLIT ? static_cast<unsigned>(k) : 0u);
  unsigned key = unit * static_cast<unsigned>(g.kpb);
  if constexpr (SPLIT) {
    Folded<SP, float> F;
    fold_query<SP, float>(xq, k, vol, F);
    key += static_cast<unsigned>(SP::template orbit<float>(F.up));
  }
  return key;
}

template <class SP>
__device__ __forceinline__ void load_x(const float* __restrict__ x, long long q, float* xq) {
#pragma unroll
  for (int d = 0; d < SP::S; ++d) xq[d] = x[q * SP::S + d];
}

// items per thread whose query loads are in flight together
constexpr int kBinBatch = 4;

// 1. per-tile histogram of keys (dynamic LDS: nkeys counters)
template <class SP, bool SPLIT>
__global__ void __launch_bounds__(1024) k_bin_hist(Vol vol, BinGeom g, const float* __restrict__ x,
                                                   unsigned* __restrict__ hist) {
  extern __shared__ unsigned cnt[];
  for (unsigned i = threadIdx.x; i < g.nkeys; i += blockDim.x) cnt[i] = 0u;
  __syncthreads();
  const long long t0 = static_cast<long long>(blockIdx.x) * g.tile_items;
  const long long t1 = t0 + g.tile_items < g.items ? t0 + g.tile_items : g.items;
  constexpr int U = kBinBatch;
  for (long long tb = t0 + threadIdx.x; tb < t1; tb += U * blockDim.x) {
    float xq[U][SP::S];
    int kk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long t = tb + static_cast<long long>(u) * blockDim.x;
      long long q;
      split_item<SP, SPLIT>(t < t1 ? t : t0, q, kk[u]);
      load_x<SP>(x, q, xq[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (tb + static_cast<long long>(u) * blockDim.x < t1) atomicAdd(cnt + item_key<SP, SPLIT>(vol, g, xq[u], kk[u]), 1u);
  }
  __syncthreads();
  unsigned* out = hist + static_cast<size_t>(blockIdx.x) * g.nkeys;
  for (unsigned i = threadIdx.x; i < g.nkeys; i += blockDim.x) out[i] = cnt[i];
}

// 2. per key: exclusive running sum over tiles (in place) and the key total
template <int = 0>
__global__ void __launch_bounds__(256) k_bin_colscan(unsigned* __restrict__ hist, int tiles, unsigned nkeys,
                                                     unsigned* __restrict__ tot) {
  const unsigned key = blockIdx.x * blockDim.x + threadIdx.x;
  if (key > nkeys) return;
  if (key == nkeys) {
    tot[key] = 0u;
    return;
  }
  unsigned run = 0u;
  int t = 0;
  for (; t + 16 <= tiles; t += 16) {
    unsigned h[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) h[j] = hist[static_cast<size_t>(t + j) * nkeys + key];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      hist[static_cast<size_t>(t + j) * nkeys + key] = run;
      run += h[j];
    }
  }
  for (; t < tiles; ++t) {
    unsigned* p = hist + static_cast<size_t>(t) * nkeys + key;
    const unsigned h = *p;
    *p = run;
    run += h;
  }
  tot[key] = run;
}

// 3. place each item's record at its sorted position
template <class SP, bool SPLIT>
__global__ void __launch_bounds__(1024) k_bin_place(Vol vol, BinGeom g, const float* __restrict__ x,
                                                    const unsigned* __restrict__ hist,
                                                    const unsigned* __restrict__ start, Rec<SP::S>* __restrict__ recs) {
  extern __shared__ unsigned cur[];
  const unsigned* h = hist + static_cast<size_t>(blockIdx.x) * g.nkeys;
  for (unsigned i = threadIdx.x; i < g.nkeys; i += blockDim.x) cur[i] = h[i] + start[i];
  __syncthreads();
  const long long t0 = static_cast<long long>(blockIdx.x) * g.tile_items;
  const long long t1 = t0 + g.tile_items < g.items ? t0 + g.tile_items : g.items;
  constexpr int U = kBinBatch;
  for (long long tb = t0 + threadIdx.x; tb < t1; tb += U * blockDim.x) {
    float xq[U][SP::S];
    int kk[U];
    unsigned pos[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long t = tb + static_cast<long long>(u) * blockDim.x;
      long long q;
      split_item<SP, SPLIT>(t < t1 ? t : t0, q, kk[u]);
      load_x<SP>(x, q, xq[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (tb + static_cast<long long>(u) * blockDim.x < t1)
        pos[u] = atomicAdd(cur + item_key<SP, SPLIT>(vol, g, xq[u], kk[u]), 1u);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long t = tb + static_cast<long long>(u) * blockDim.x;
      if (t >= t1) continue;
      Rec<SP::S> r;
      if constexpr (SP::S == 3) {
        r.a = make_float4(xq[u][0], xq[u][1], xq[u][2], __uint_as_float(static_cast<unsigned>(t)));
      } else {
        r.a = make_float4(xq[u][0], xq[u][1], xq[u][2], xq[u][3]);
        r.b = make_uint4(static_cast<unsigned>(t), 0u, 0u, 0u);
      }
      recs[pos[u]] = r;
    }
  }
}

template <class SP>
__device__ __forceinline__ Rec<SP::S> make_rec(const float* xq, long long t) {
  Rec<SP::S> r;
  if constexpr (SP::S == 3) {
    r.a = make_float4(xq[0], xq[1], xq[2], __uint_as_float(static_cast<unsigned>(t)));
  } else {
    r.a = make_float4(xq[0], xq[1], xq[2], xq[3]);
    r.b = make_uint4(static_cast<unsigned>(t), 0u, 0u, 0u);
  }
  return r;
}

// Exclusive scan out[i] = in[0] + ... + in[i - 1], i < n, by a 1024-thread
// workgroup (in == out allowed); tmp: 16 words of LDS.  Each thread takes a
// contiguous run of ceil(n / 1024) entries.
__device__ __forceinline__ void block_scan_1024(const unsigned* in, unsigned* out, unsigned n, unsigned* tmp) {
  const unsigned tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const unsigned per = (n + 1023u) >> 10;
  const unsigned b = min(tid * per, n), e = min(b + per, n);
  unsigned s = 0u;
  for (unsigned i = b; i < e; ++i) s += in[i];
  unsigned v = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned u = __shfl_up(v, off, 64);
    if (lane >= static_cast<unsigned>(off)) v += u;
  }
  if (lane == 63u) tmp[wave] = v;
  __syncthreads();
  if (tid < 64u) {
    unsigned w = tid < 16u ? tmp[tid] : 0u;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      const unsigned u = __shfl_up(w, off, 64);
      if (lane >= static_cast<unsigned>(off)) w += u;
    }
    if (tid < 16u) tmp[tid] = w;
  }
  __syncthreads();
  unsigned run = v - s + (wave ? tmp[wave - 1] : 0u);
  for (unsigned i = b; i < e; ++i) {
    const unsigned c = in[i];
    out[i] = run;
    run += c;
  }
}

// the whole exclusive scan of the key totals in one workgroup (small key counts)
template <int = 0>
__global__ void __launch_bounds__(1024) k_scan_single(const unsigned* __restrict__ in, unsigned* __restrict__ out,
                                                      unsigned n) {
  __shared__ unsigned tmp[16];
  block_scan_1024(in, out, n, tmp);
}

// 3'. place records through an LDS counting sort of windows of W = 16384
// items, so that a window's records of one key are written by neighbouring
// lanes as one contiguous run.  Scattered single records cost about one
// memory-fabric write request each; runs of several records share them.
// Each thread keeps its 16 items' coordinates in registers (x is read once,
// coalesced); after the window's key counts are scanned the records pass
// through LDS in chunks of C = 2^cshift sorted positions.  LDS: the chunk's
// records (item word = key << 15 | index in window), the tile's cursor per
// key, and the window's key counts (then starts).  Keys < 2^17.
template <class SP, bool SPLIT>
__global__ void __launch_bounds__(1024) k_bin_place_win(Vol vol, BinGeom g, const float* __restrict__ x,
                                                        const unsigned* __restrict__ hist,
                                                        const unsigned* __restrict__ start,
                                                        Rec<SP::S>* __restrict__ recs, int cshift) {
  extern __shared__ unsigned lds_place[];
  constexpr int R = 16;                 // items per thread and window
  constexpr unsigned W = 1024u * R;
  constexpr int U = kBinBatch;
  const unsigned nk = g.nkeys, C = 1u << cshift, tid = threadIdx.x;
  Rec<SP::S>* crec = reinterpret_cast<Rec<SP::S>*>(lds_place);   // C; its first 16 words also serve the scan
  unsigned* gcur = reinterpret_cast<unsigned*>(crec + C);         // nk: next record slot of each key
  unsigned* wst = gcur + nk;                                       // nk: window counts, then starts
  const unsigned* h = hist + static_cast<size_t>(blockIdx.x) * nk;
  for (unsigned i = tid; i < nk; i += blockDim.x) {
    gcur[i] = h[i] + start[i];
    wst[i] = 0u;
  }
  __syncthreads();
  const long long t0 = static_cast<long long>(blockIdx.x) * g.tile_items;
  const long long t1 = t0 + g.tile_items < g.items ? t0 + g.tile_items : g.items;
  for (long long w0 = t0; w0 < t1; w0 += W) {
    const unsigned nw = static_cast<unsigned>(t1 - w0 < static_cast<long long>(W) ? t1 - w0 : W);
    float xr[R][SP::S];
    unsigned pk[R];                     // key << 15 | rank of the item among the window's items of its key
#pragma unroll
    for (int r0 = 0; r0 < R; r0 += U) {
      if (static_cast<unsigned>(r0) * 1024u >= nw) break;
      int kk[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const unsigned j = static_cast<unsigned>(r0 + u) * 1024u + tid;
        long long q;
        split_item<SP, SPLIT>(w0 + (j < nw ? j : 0u), q, kk[u]);
        load_x<SP>(x, q, xr[r0 + u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const unsigned j = static_cast<unsigned>(r0 + u) * 1024u + tid;
        pk[r0 + u] = 0u;
        if (j < nw) {
          const unsigned key = item_key<SP, SPLIT>(vol, g, xr[r0 + u], kk[u]);
          pk[r0 + u] = (key << 15) | atomicAdd(wst + key, 1u);
        }
      }
    }
    __syncthreads();
    block_scan_1024(wst, wst, nk, reinterpret_cast<unsigned*>(crec));
    __syncthreads();
    for (unsigned c0 = 0; c0 < nw; c0 += C) {
      // the records of sorted positions [c0, c0 + C) into LDS
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (static_cast<unsigned>(r) * 1024u >= nw) break;
        const unsigned j = static_cast<unsigned>(r) * 1024u + tid;
        if (j < nw) {
          const unsigned key = pk[r] >> 15;
          const unsigned sp = wst[key] + (pk[r] & 0x7fffu) - c0;
          if (sp < C) crec[sp] = make_rec<SP>(xr[r], (key << 15) | j);
        }
      }
      __syncthreads();
      // lane i writes the i-th record of the chunk
      const unsigned m = nw - c0 < C ? nw - c0 : C;
      for (unsigned i = tid; i < m; i += blockDim.x) {
        Rec<SP::S> rc = crec[i];
        unsigned p;
        if constexpr (SP::S == 3) p = __float_as_uint(rc.a.w); else p = rc.b.x;
        const unsigned key = p >> 15;
        const unsigned pos = gcur[key] + (c0 + i - wst[key]);
        const unsigned item = static_cast<unsigned>(w0) + (p & 0x7fffu);
        if constexpr (SP::S == 3) rc.a.w = __uint_as_float(item); else rc.b.x = item;
        recs[pos] = rc;
      }
      __syncthreads();
    }
    // advance the cursors by the window's counts, clear the counts
    for (unsigned key = tid; key < nk; key += blockDim.x)
      gcur[key] += (key + 1u < nk ? wst[key + 1u] : nw) - wst[key];
    __syncthreads();
    for (unsigned key = tid; key < nk; key += blockDim.x) wst[key] = 0u;
    __syncthreads();
  }
}

// 3''. the windowed placement for (query, coset) items of splines with many
// cosets (M >= 4): a window of 16384 items covers at most 16384 / M + 1
// queries, whose coordinates are kept in LDS (one copy per query instead of
// one per item in registers), and the window's items in key order are kept
// as packed words key << 15 | index in window, so each key's records of a
// window leave as one contiguous run.  LDS: the window's queries, the sorted
// words, the tile's cursor per key and the window's key counts (then
// starts).  Keys < 2^17.
template <class SP>
__global__ void __launch_bounds__(1024) k_bin_place_winq(Vol vol, BinGeom g, const float* __restrict__ x,
                                                         const unsigned* __restrict__ hist,
                                                         const unsigned* __restrict__ start,
                                                         Rec<SP::S>* __restrict__ recs) {
  extern __shared__ unsigned lds_place[];
  constexpr int S = SP::S, M = SP::M, R = 16;
  constexpr unsigned W = 1024u * R;
  constexpr unsigned WQ = W / M + 2;    // queries a window can touch
  const unsigned nk = g.nkeys, tid = threadIdx.x;
  float* xw = reinterpret_cast<float*>(lds_place);                 // WQ * S
  unsigned* sorted = lds_place + WQ * S;                            // W; its first 16 words also serve the scan
  unsigned* gcur = sorted + W;                                      // nk
  unsigned* wst = gcur + nk;                                        // nk
  const unsigned* h = hist + static_cast<size_t>(blockIdx.x) * nk;
  for (unsigned i = tid; i < nk; i += blockDim.x) {
    gcur[i] = h[i] + start[i];
    wst[i] = 0u;
  }
  __syncthreads();
  const long long t0 = static_cast<long long>(blockIdx.x) * g.tile_items;
  const long long t1 = t0 + g.tile_items < g.items ? t0 + g.tile_items : g.items;
  for (long long w0 = t0; w0 < t1; w0 += W) {
    const unsigned nw = static_cast<unsigned>(t1 - w0 < static_cast<long long>(W) ? t1 - w0 : W);
    const long long q0 = w0 / M;
    const unsigned nq = static_cast<unsigned>((w0 + nw - 1) / M - q0 + 1);
    // the window's queries into LDS, coalesced
    for (unsigned e = tid; e < nq * S; e += blockDim.x) xw[e] = x[q0 * S + e];
    __syncthreads();
    unsigned pk[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const unsigned j = static_cast<unsigned>(r) * 1024u + tid;
      pk[r] = 0u;
      if (j < nw) {
        long long q;
        int k;
        split_item<SP, true>(w0 + j, q, k);
        const unsigned key = item_key<SP, true>(vol, g, xw + (q - q0) * S, k);
        pk[r] = (key << 15) | atomicAdd(wst + key, 1u);
      }
    }
    __syncthreads();
    block_scan_1024(wst, wst, nk, sorted);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const unsigned j = static_cast<unsigned>(r) * 1024u + tid;
      if (j < nw) {
        const unsigned key = pk[r] >> 15;
        sorted[wst[key] + (pk[r] & 0x7fffu)] = (key << 15) | j;
      }
    }
    __syncthreads();
    // lane i writes the i-th record of the window
    for (unsigned i = tid; i < nw; i += blockDim.x) {
      const unsigned p = sorted[i];
      const unsigned key = p >> 15;
      const long long t = w0 + (p & 0x7fffu);
      const float* xq = xw + (t / M - q0) * S;
      recs[gcur[key] + (i - wst[key])] = make_rec<SP>(xq, t);
    }
    __syncthreads();
    for (unsigned key = tid; key < nk; key += blockDim.x)
      gcur[key] += (key + 1u < nk ? wst[key + 1u] : nw) - wst[key];
    __syncthreads();
    for (unsigned key = tid; key < nk; key += blockDim.x) wst[key] = 0u;
    __syncthreads();
  }
}

template <class SP>
__device__ __forceinline__ unsigned rec_item(const Rec<SP::S>& r, float* xq) {
  if constexpr (SP::S == 3) {
    xq[0] = r.a.x; xq[1] = r.a.y; xq[2] = r.a.z;
    return __float_as_uint(r.a.w);
  } else {
    xq[0] = r.a.x; xq[1] = r.a.y; xq[2] = r.a.z; xq[3] = r.a.w;
    return r.b.x;
  }
}

// query index of a record's item
template <class SP, bool SPLIT>
__device__ __forceinline__ long long rec_query(const Rec<SP::S>& r) {
  float xs[SP::S];
  long long q;
  int k;
  split_item<SP, SPLIT>(rec_item<SP>(r, xs), q, k);
  return q;
}

// unit handled by this workgroup: each XCD (blocks are dealt round-robin to
// the 8 XCDs) takes a contiguous run of units, so neighbouring bricks share
// their halo in one L2
__device__ __forceinline__ long long unit_of_block(unsigned nunits) {
  const unsigned per = (nunits + 7u) / 8u;
  const unsigned xcd = blockIdx.x & 7u, slot = blockIdx.x >> 3;
  if (slot >= per) return -1;
  const unsigned u = xcd * per + slot;
  return u < nunits ? static_cast<long long>(u) : -1;
}

// staged coefficient region of one brick
template <class SP, class AT>
struct StageInfo {
  int org[SP::S];     // global cell index of the region origin per axis
  int W;              // region width
  int vol;            // W^S
  int ls[SP::S];      // LDS strides
};

template <class SP, class AT>
__device__ __forceinline__ void stage_info(const BinGeom& g, long long brick, StageInfo<SP, AT>& si) {
  const int B = 1 << g.bshift;
  si.W = Staged<SP>::width(B);
  long long rem = brick;
  int st = 1;
#pragma unroll
  for (int d = 0; d < SP::S; ++d) {
    const int b = static_cast<int>(rem % g.nb[d]);
    rem /= g.nb[d];
    si.org[d] = b * B - Staged<SP>::MARGIN + SP::OMIN;
    si.ls[d] = st;
    st *= si.W;
  }
  si.vol = st;
}

constexpr int kStageBatch = 8;

// stage cosets [k0, k0 + ncos) of the region into lds[(k - k0) * vol + r],
// zero outside the stored arrays.  A thread walks the region with a stride of
// blockDim.x elements, carrying its per-axis position digit by digit instead
// of dividing by W for every element; out-of-range elements load a valid
// element and are replaced by zero.
template <class SP, class CT, class AT>
__device__ __forceinline__ void stage_load(const Vol& vol, const StageInfo<SP, AT>& si, int k0, int ncos, AT* lds) {
  const int W = si.W, NT = static_cast<int>(blockDim.x);
  int step[SP::S], start[SP::S];
  {
    int a = NT, b = static_cast<int>(threadIdx.x);
#pragma unroll
    for (int d = 0; d < SP::S; ++d) {
      step[d] = d + 1 < SP::S ? a % W : a;
      start[d] = d + 1 < SP::S ? b % W : b;
      a /= W;
      b /= W;
    }
  }
  // kStageBatch loads in flight per thread before their LDS writes
  constexpr int U = kStageBatch;
  for (int kl = 0; kl < ncos; ++kl) {
    const CT* base = static_cast<const CT*>(pick<SP::M>(vol.base, k0 + kl));
    AT* dst = lds + kl * si.vol;
    int pos[SP::S];
#pragma unroll
    for (int d = 0; d < SP::S; ++d) pos[d] = start[d];
    for (int e0 = static_cast<int>(threadIdx.x); e0 < si.vol; e0 += U * NT) {
      AT v[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        bool in = e0 + u * NT < si.vol;
        int off = 0;
#pragma unroll
        for (int d = 0; d < SP::S; ++d) {
          const int c = si.org[d] + pos[d];
          in = in && static_cast<unsigned>(c) < static_cast<unsigned>(vol.dims[d]);
          off += c * vol.stride[d];
        }
        v[u] = load_coef<CT, AT>(base + (in ? off : 0));
        ok[u] = in;
        int carry = 0;
#pragma unroll
        for (int d = 0; d < SP::S; ++d) {
          pos[d] += step[d] + carry;
          if (d + 1 < SP::S) {
            carry = pos[d] >= W;
            pos[d] -= carry ? W : 0;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * NT;
        if (e < si.vol) dst[e] = ok[u] ? v[u] : AT(0);
      }
    }
  }
}

// LDS stride W^a of original axis a (a varies per lane: computed values only)
template <class SP, class AT>
__device__ __forceinline__ int lds_stride(const StageInfo<SP, AT>& si, int a) {
  const int W = si.W, W2 = W * W;
  int v = (a == 1) ? W : 1;
  v = (a == 2) ? W2 : v;
  if constexpr (SP::S == 4) v = (a == 3) ? W2 * W : v;
  return v;
}

// item's stencil inside the staged region?
template <class SP, class AT>
__device__ __forceinline__ bool stageable(const StageInfo<SP, AT>& si, const Folded<SP, AT>& F) {
  bool ok = true;
#pragma unroll
  for (int d = 0; d < SP::S; ++d) {
    const int li = F.i[d] - si.org[d];
    ok = ok && (li + SP::OMIN >= 0) && (li + SP::OMAX < si.W);
  }
  return ok;
}

// gather / scatter through the fold inside an LDS region
// Byte offsets of the folded stencil inside an LDS region.  A site J (folded
// frame) sits at  origin + sum_r J_r st_r  elements, with st_r the signed
// stride of folded axis r.  Per axis the multiples J st_r are tabulated once
// per query (one add per entry), so a site's address is one three-input add
// of table entries instead of a multiply-add chain per site.
template <class SP, int ESIZE>
struct FoldedOffsets {
  static constexpr int JLO = SP::OMIN < 1 - SP::OMAX ? SP::OMIN : 1 - SP::OMAX;
  static constexpr int JHI = SP::OMAX > 1 - SP::OMIN ? SP::OMAX : 1 - SP::OMIN;
  static constexpr int NJ = JHI - JLO + 1;
  unsigned p[SP::S][NJ];   // p[r][J - JLO] = J st_r (bytes); axis 0 also carries the origin

  template <class AT>
  __device__ __forceinline__ void init(const StageInfo<SP, AT>& si, const Folded<SP, AT>& F) {
    int off = 0;
#pragma unroll
    for (int d = 0; d < SP::S; ++d) off += (F.i[d] - si.org[d]) * si.ls[d];
    int st[SP::S];
#pragma unroll
    for (int r = 0; r < SP::S; ++r) {
      const int s = lds_stride<SP, AT>(si, F.ax[r]);
      st[r] = F.sg[r] > 0 ? s * ESIZE : -s * ESIZE;
      if (F.sg[r] < 0) off += s;
    }
#pragma unroll
    for (int r = 0; r < SP::S; ++r) {
      const unsigned z = r == 0 ? static_cast<unsigned>(off * ESIZE) : 0u;
      p[r][-JLO] = z;
#pragma unroll
      for (int j = -JLO + 1; j < NJ; ++j) p[r][j] = p[r][j - 1] + static_cast<unsigned>(st[r]);
#pragma unroll
      for (int j = -JLO - 1; j >= 0; --j) p[r][j] = p[r][j + 1] - static_cast<unsigned>(st[r]);
    }
  }
  template <int J0, int J1, int J2, int J3>
  __device__ __forceinline__ unsigned at() const {
    unsigned a = p[0][J0 - JLO] + p[1][J1 - JLO] + p[2][J2 - JLO];
    if constexpr (SP::S == 4) a += p[3][J3 - JLO];
    return a;
  }
};

template <class SP, class AT>
struct GatherLds {
  const char* region;
  FoldedOffsets<SP, sizeof(AT)> o;
  __device__ __forceinline__ void init(const AT* region_, const StageInfo<SP, AT>& si, const Folded<SP, AT>& F) {
    region = reinterpret_cast<const char*>(region_);
    o.init(si, F);
  }
  template <int J0, int J1, int J2, int J3 = 0>
  __device__ __forceinline__ AT c() const {
    return *reinterpret_cast<const AT*>(region + o.template at<J0, J1, J2, J3>());
  }
};

// Fixed-point value of a float with |v| < 2^51, rounded to the nearest
// integer: v = hi 2^24 + lo with hi = trunc(v 2^-24); the split is exact, so
// the only rounding is that of lo.
__device__ __forceinline__ long long to_fixed(float v) {
  const float hi = truncf(v * 0x1p-24f);
  const float lo = fmaf(hi, -0x1p24f, v);
  return static_cast<long long>(static_cast<int>(hi)) * (1ll << 24) + static_cast<long long>(__float2int_rn(lo));
}

// Scatter-add into an LDS region of 64-bit fixed-point accumulators: gs is
// g_q times the unit's power-of-two scale.  Integer LDS atomics are an order
// of magnitude faster than float ones on this hardware, and integer sums do
// not depend on the order of the additions.
template <class SP>
struct ScatterLds {
  char* region;
  FoldedOffsets<SP, 8> o;
  float gs;
  __device__ __forceinline__ void init(unsigned long long* region_, const StageInfo<SP, float>& si,
                                       const Folded<SP, float>& F, float gscaled) {
    region = reinterpret_cast<char*>(region_);
    o.init(si, F);
    gs = gscaled;
  }
  template <int J0, int J1, int J2, int J3 = 0>
  __device__ __forceinline__ void put(float w) {
    atomicAdd(reinterpret_cast<unsigned long long*>(region + o.template at<J0, J1, J2, J3>()),
              static_cast<unsigned long long>(to_fixed(gs * w)));
  }
};

// f(integral_constant<int, I>) for I = 0 .. N-1, unrolled at compile time
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Whole-query lanes of a spline with several polynomial pieces run every
// piece that some lane of the wave needs (the pieces branch on the
// sub-region).  All pieces' stencil offsets lie in the box [JLO, JHI]^S of
// FoldedOffsets, so a slot per box position lets the branches share their
// memory work:
//   BoxGatherLds loads the box sites before the branch; the compiler drops
//   the loads of positions that no piece reads, which leaves the union of the
//   pieces' stencils, loaded once instead of once per piece;
//   BoxScatterLds only collects each piece's weights in the branch and
//   converts and adds every position once after it; positions that no piece
//   writes keep the constant zero and their adds fold away.
// The values and the fixed-point terms are those of GatherLds / ScatterLds.
template <class SP, int ESIZE>
struct Box {
  using FO = FoldedOffsets<SP, ESIZE>;
  static constexpr int NJ = FO::NJ, JLO = FO::JLO;
  static constexpr int N = SP::S == 3 ? NJ * NJ * NJ : NJ * NJ * NJ * NJ;
  template <int J0, int J1, int J2, int J3>
  static constexpr int slot() {
    return (J0 - JLO) + NJ * ((J1 - JLO) + NJ * ((J2 - JLO) + (SP::S == 4 ? NJ * (J3 - JLO) : 0)));
  }
  // component d of box position i
  static constexpr int jc(int i, int d) {
    for (int e = 0; e < d; ++e) i /= NJ;
    return i % NJ + JLO;
  }
  template <int I>
  __device__ __forceinline__ static unsigned at(const FO& o) {
    return o.template at<jc(I, 0), jc(I, 1), jc(I, 2), jc(I, 3)>();
  }
};

// multi-piece splines evaluated whole-query per lane
template <class SP>
constexpr bool box_pieces() { return SP::K > 1 && !SplitPolicy<SP>::value; }

template <class SP, class AT>
struct BoxGatherLds {
  using B = Box<SP, sizeof(AT)>;
  AT v[B::N];
  __device__ __forceinline__ void init(const AT* region, const StageInfo<SP, AT>& si, const Folded<SP, AT>& F) {
    typename B::FO o;
    o.init(si, F);
    const char* r = reinterpret_cast<const char*>(region);
    static_for<B::N>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      v[I] = *reinterpret_cast<const AT*>(r + B::template at<I>(o));
    });
  }
  template <int J0, int J1, int J2, int J3 = 0>
  __device__ __forceinline__ AT c() const {
    return v[B::template slot<J0, J1, J2, J3>()];
  }
};

template <class SP>
struct BoxScatterLds {
  using B = Box<SP, 8>;
  char* region;
  typename B::FO o;
  float gs;
  float w[B::N];
  __device__ __forceinline__ void init(unsigned long long* region_, const StageInfo<SP, float>& si,
                                       const Folded<SP, float>& F, float gscaled) {
    region = reinterpret_cast<char*>(region_);
    o.init(si, F);
    gs = gscaled;
#pragma unroll
    for (int i = 0; i < B::N; ++i) w[i] = 0.f;
  }
  template <int J0, int J1, int J2, int J3 = 0>
  __device__ __forceinline__ void put(float wv) {
    w[B::template slot<J0, J1, J2, J3>()] += wv;
  }
  __device__ __forceinline__ void flush() {
    static_for<B::N>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      if (w[I] != 0.f)
        atomicAdd(reinterpret_cast<unsigned long long*>(region + B::template at<I>(o)),
                  static_cast<unsigned long long>(to_fixed(gs * w[I])));
    });
  }
};

// Power-of-two scale 2^shift of a unit's fixed-point region, shift = E - eg
// with gmax < 2^eg.  |g w| <= gmax (the weights lie in [0, 1]) and a site
// receives at most one term per item, so every scaled term is below 2^E and
// a site's sum below items 2^E <= 2^61.  E = min(50, 61 - bit length of
// items): terms are resolved to 2^-E of 2^eg (< 2 gmax).  The scaling is
// applied with ldexp, so tiny or huge gradients cannot overflow a factor.
__device__ __forceinline__ int unit_shift(unsigned items, float gmax) {
  const int bits = 32 - __clz(static_cast<int>(items | 1u));
  const int E = min(50, 61 - bits);
  int eg = 0;
  (void)frexpf(gmax > 0.f && gmax <= 3.402823466e38f ? gmax : 1.f, &eg);
  return E - eg;
}

// one coset's psi (and folded gradient mapped back to x) from LDS or global.
// region: the LDS copy of coset k's part of the unit's region (or null).
template <class SP, class CT, class AT, bool GRAD, bool STAGE>
__device__ __forceinline__ void coset_binned_folded(const Vol& vol, const StageInfo<SP, AT>& si, const AT* region,
                                                    int k, const Folded<SP, AT>& F, AT& f, AT* gx) {
  const int ob = SP::template orbit<AT>(F.up);
  AT b[SP::NMON];
  if constexpr (STAGE) {
    // every item of a unit is stageable (queries outside the brick grid are
    // scheduled apart, under the outlier key); a violation shows as NaN
    if (stageable<SP, AT>(si, F)) {
      if constexpr (box_pieces<SP>()) {
        BoxGatherLds<SP, AT> g;
        g.init(region, si, F);
        SP::template b_any<AT>(ob, g, b);
      } else {
        GatherLds<SP, AT> g;
        g.init(region, si, F);
        SP::template b_any<AT>(ob, g, b);
      }
    } else {
#pragma unroll
      for (int m = 0; m < SP::NMON; ++m) b[m] = AT(__builtin_nanf(""));
    }
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

template <class SP, class CT, class AT, bool GRAD, bool STAGE>
__device__ __forceinline__ void coset_binned(const Vol& vol, const StageInfo<SP, AT>& si, const AT* region, int k,
                                             const AT* xq, AT& f, AT* gx) {
  Folded<SP, AT> F;
  fold_query<SP, AT>(xq, k, vol, F);
  coset_binned_folded<SP, CT, AT, GRAD, STAGE>(vol, si, region, k, F, f, gx);
}

struct UnitRange {
  long long unit, brick;
  int kunit;            // the unit's coset (coset-split units)
  unsigned lo, hi;      // its items in the sorted records
};

template <bool SPLIT>
__device__ __forceinline__ bool unit_range(const BinGeom& g, const unsigned* start, UnitRange& u,
                                           unsigned wpu = 1, unsigned* part = nullptr) {
  // with wpu > 1 consecutive virtual blocks share a unit, each taking every
  // wpu-th run of blockDim.x items
  const long long vb = unit_of_block(g.nunits * wpu);
  if (vb < 0) return false;
  u.unit = vb / wpu;
  if (part) *part = static_cast<unsigned>(vb - u.unit * wpu);
  u.brick = u.unit / g.upb;
  u.kunit = SPLIT ? static_cast<int>(u.unit - u.brick * g.upb) : 0;
  const unsigned k0 = static_cast<unsigned>(u.unit) * g.kpb;
  u.lo = start[k0];
  u.hi = start[k0 + g.kpb];
  return u.lo != u.hi;
}

// One work item of the binned forward: record coordinates xf and item id,
// target yq (MSE) and schedule position t.
//   not SPLIT: f[q] (and grad[q]) directly.  SPLIT: fpart[k * n + q] (and
//   gpart) for the combine kernel.  MSE (not SPLIT): also dL/df, and grad
//   receives dL/dx = dL/df * grad f.
template <class SP, class CT, class AT, bool GRAD, bool SPLIT, bool STAGE, bool MSE>
__device__ __forceinline__ void eval_item(const Vol& vol, const BinGeom& g, const StageInfo<SP, AT>& si,
                                          const AT* lds, const float* xf, unsigned item, float yq, unsigned t,
                                          AT* __restrict__ f, AT* __restrict__ grad, float inv_n,
                                          float* __restrict__ dldf, float* __restrict__ gsave, float& r2) {
  long long q;
  int k;
  split_item<SP, SPLIT>(item, q, k);
  AT xq[SP::S];
#pragma unroll
  for (int d = 0; d < SP::S; ++d) xq[d] = static_cast<AT>(xf[d]);
  AT acc = AT(0);
  AT gx[SP::S];
#pragma unroll
  for (int d = 0; d < SP::S; ++d) gx[d] = AT(0);
  if constexpr (SPLIT) {
    coset_binned<SP, CT, AT, GRAD, STAGE>(vol, si, lds, k, xq, acc, gx);
    const long long slot = static_cast<long long>(k) * g.n + q;
    f[slot] = acc;
    if constexpr (GRAD) {
#pragma unroll
      for (int d = 0; d < SP::S; ++d) grad[slot * SP::S + d] = gx[d];
    }
  } else {
    if constexpr (complement_coset<SP>()) {
      Folded<SP, AT> F0, F1;
      fold_query<SP, AT>(xq, 0, vol, F0);
      coset_binned_folded<SP, CT, AT, GRAD, STAGE>(vol, si, lds, 0, F0, acc, gx);
      fold_complement<SP, AT>(F0, vol, F1);
      coset_binned_folded<SP, CT, AT, GRAD, STAGE>(vol, si, STAGE ? lds + si.vol : lds, 1, F1, acc, gx);
    } else {
#pragma unroll
      for (int kk = 0; kk < SP::M; ++kk)
        coset_binned<SP, CT, AT, GRAD, STAGE>(vol, si, STAGE ? lds + kk * si.vol : lds, kk, xq, acc, gx);
    }
    if (f) f[q] = acc;    // optional for the MSE head
    AT scale = AT(1);
    if constexpr (MSE) {
      const float r = static_cast<float>(acc) - yq;
      const float dl = 2.f * r * inv_n;
      if (dldf) dldf[q] = dl;
      if (gsave) gsave[t] = dl;   // in schedule order, for the fused backward
      r2 += r * r;
      scale = static_cast<AT>(dl);
    }
    if constexpr (GRAD) {
#pragma unroll
      for (int d = 0; d < SP::S; ++d) grad[q * SP::S + d] = scale * gx[d];
    }
  }
}

// 4a. forward, one workgroup per unit (see eval_item for the outputs)
template <class SP, class CT, class AT, bool GRAD, bool SPLIT, bool STAGE, bool MSE>
__device__ __forceinline__ void eval_binned_body(const Vol& vol, const BinGeom& g,
                                                 const Rec<SP::S>* __restrict__ recs,
                                                 const unsigned* __restrict__ start, AT* __restrict__ f,
                                                 AT* __restrict__ grad, const float* __restrict__ y, float inv_n,
                                                 float* __restrict__ dldf, double* __restrict__ loss,
                                                 float* __restrict__ gsave) {
  extern __shared__ unsigned char smem[];
  AT* lds = reinterpret_cast<AT*>(smem);
  UnitRange u;
  unsigned part = 0;
  if (!unit_range<SPLIT>(g, start, u, g.wpu, &part)) return;
  StageInfo<SP, AT> si;
  stage_info<SP, AT>(g, u.brick, si);
  if constexpr (STAGE) {
    stage_load<SP, CT, AT>(vol, si, SPLIT ? u.kunit : 0, SPLIT ? 1 : SP::M, lds);
    __syncthreads();
  }
  float r2 = 0.f;
  const unsigned step = g.wpu * blockDim.x;
  const unsigned first = u.lo + part * blockDim.x + threadIdx.x;
  // the next record is loaded while this one is evaluated
  Rec<SP::S> cur = recs[min(first, u.hi - 1)];
  float ycur = 0.f;
  if constexpr (MSE && !SPLIT) ycur = y[rec_query<SP, SPLIT>(cur)];
  for (unsigned t = first; t < u.hi; t += step) {
    const Rec<SP::S> nxt = recs[min(t + step, u.hi - 1)];
    float ynxt = 0.f;
    if constexpr (MSE && !SPLIT) ynxt = y[rec_query<SP, SPLIT>(nxt)];
    float xf[SP::S];
    const unsigned item = rec_item<SP>(cur, xf);
    const float yq = ycur;
    cur = nxt;
    ycur = ynxt;
    eval_item<SP, CT, AT, GRAD, SPLIT, STAGE, MSE>(vol, g, si, lds, xf, item, yq, t, f, grad, inv_n, dldf, gsave, r2);
  }
  if constexpr (MSE && !SPLIT) mse_reduce(r2, static_cast<double>(inv_n), loss);
}

template <class SP, class CT, class AT, bool GRAD, bool SPLIT, bool STAGE, bool MSE, int NT>
__global__ void __launch_bounds__(NT) k_eval_binned(Vol vol, BinGeom g, const Rec<SP::S>* __restrict__ recs,
                                                     const unsigned* __restrict__ start, AT* __restrict__ f,
                                                     AT* __restrict__ grad, const float* __restrict__ y, float inv_n,
                                                     float* __restrict__ dldf, double* __restrict__ loss,
                                                     float* __restrict__ gsave) {
  eval_binned_body<SP, CT, AT, GRAD, SPLIT, STAGE, MSE>(vol, g, recs, start, f, grad, y, inv_n, dldf, loss, gsave);
}

// The same for 4-D units (512 threads) held to 128 VGPRs, i.e. 4 waves per
// SIMD and two workgroups per CU, where the unconstrained code needs a few
// registers more.
template <class SP, class CT, class AT, bool GRAD, bool SPLIT, bool STAGE, bool MSE, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
k_eval_binned_w4(Vol vol, BinGeom g, const Rec<SP::S>* __restrict__ recs, const unsigned* __restrict__ start,
                 AT* __restrict__ f, AT* __restrict__ grad, const float* __restrict__ y, float inv_n,
                 float* __restrict__ dldf, double* __restrict__ loss, float* __restrict__ gsave) {
  eval_binned_body<SP, CT, AT, GRAD, SPLIT, STAGE, MSE>(vol, g, recs, start, f, grad, y, inv_n, dldf, loss, gsave);
}

// 4a'. forward of the items under the outlier key (queries outside the brick
// grid), from global memory with zero padding; a grid-stride loop over the
// key's records, usually none
template <class SP, class CT, class AT, bool GRAD, bool SPLIT, bool MSE>
__global__ void __launch_bounds__(256) k_eval_outliers(Vol vol, BinGeom g, const Rec<SP::S>* __restrict__ recs,
                                                       const unsigned* __restrict__ start, AT* __restrict__ f,
                                                       AT* __restrict__ grad, const float* __restrict__ y, float inv_n,
                                                       float* __restrict__ dldf, double* __restrict__ loss,
                                                       float* __restrict__ gsave) {
  const unsigned lo = start[g.okey], hi = start[g.okey + 1];
  StageInfo<SP, AT> si{};
  float r2 = 0.f;
  for (unsigned t = lo + blockIdx.x * blockDim.x + threadIdx.x; t < hi; t += gridDim.x * blockDim.x) {
    float xf[SP::S];
    const unsigned item = rec_item<SP>(recs[t], xf);
    float yq = 0.f;
    if constexpr (MSE && !SPLIT) yq = y[item];
    eval_item<SP, CT, AT, GRAD, SPLIT, false, MSE>(vol, g, si, nullptr, xf, item, yq, t, f, grad, inv_n, dldf,
                                                   gsave, r2);
  }
  if constexpr (MSE && !SPLIT) mse_reduce(r2, static_cast<double>(inv_n), loss);
}

// 4b. combine per-coset partials: f = sum_k fpart[k], grad likewise; with the
// MSE head also dL/df, the loss, and grad = dL/df * grad f
template <class SP, class AT, bool GRAD, bool MSE>
__global__ void __launch_bounds__(256) k_combine(const AT* __restrict__ fpart, const AT* __restrict__ gpart,
                                                 long long n, AT* __restrict__ f, AT* __restrict__ grad,
                                                 const float* __restrict__ y, float inv_n, float* __restrict__ dldf,
                                                 double* __restrict__ loss, float* __restrict__ gsave) {
  float r2 = 0.f;
  for (long long q = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; q < n;
       q += static_cast<long long>(gridDim.x) * blockDim.x) {
    AT acc = AT(0);
#pragma unroll
    for (int k = 0; k < SP::M; ++k) acc += fpart[k * n + q];
    if (f) f[q] = acc;      // optional for the MSE head
    AT scale = AT(1);
    if constexpr (MSE) {
      const float r = static_cast<float>(acc) - y[q];
      const float dl = 2.f * r * inv_n;
      if (dldf) dldf[q] = dl;
      if (gsave) gsave[q] = dl;     // by query, for the fused backward
      r2 += r * r;
      scale = static_cast<AT>(dl);
    }
    if constexpr (GRAD) {
#pragma unroll
      for (int d = 0; d < SP::S; ++d) {
        AT sum = AT(0);
#pragma unroll
        for (int k = 0; k < SP::M; ++k) sum += gpart[(k * n + q) * SP::S + d];
        grad[q * SP::S + d] = scale * sum;
      }
    }
  }
  if constexpr (MSE) mse_reduce(r2, static_cast<double>(inv_n), loss);
}

// One work item of the binned adjoint: grad_c += g w(x) and, with GRADX,
// grad_x = g grad f (SPLIT: the (query, coset) partial).  LDS_G: the
// scatter-add goes into the unit's fixed-point LDS region; returns false if
// the item's stencil leaves that region (never, for items of a unit).  Else
// (items under the outlier key) it goes to global memory with float atomics.
template <class SP, class CT, bool GRADX, bool SPLIT, bool LDS_G, bool STAGE_C>
__device__ __forceinline__ bool adjoint_item(const Vol& vol, const GradVol& gvol, const BinGeom& g,
                                             const StageInfo<SP, float>& si, unsigned long long* lds_g,
                                             const float* lds_c, int shift, const float* xq, unsigned item, float gq,
                                             float* __restrict__ grad_x) {
  constexpr int NC = SPLIT ? 1 : SP::M;
  long long q;
  int k;
  split_item<SP, SPLIT>(item, q, k);
  // a query that is not finite adds nothing (fixed point cannot carry NaN);
  // its grad_x is NaN
  bool finite = true;
#pragma unroll
  for (int d = 0; d < SP::S; ++d) finite = finite && isfinite(xq[d]);
  if (!finite) {
    if constexpr (GRADX) {
      const long long slot = SPLIT ? static_cast<long long>(k) * g.n + q : q;
#pragma unroll
      for (int d = 0; d < SP::S; ++d) grad_x[slot * SP::S + d] = __int_as_float(0x7fc00000);
    }
    return true;
  }
  bool ok = true;
  float gx[SP::S];
#pragma unroll
  for (int d = 0; d < SP::S; ++d) gx[d] = 0.f;
#pragma unroll
  for (int kk = 0; kk < NC; ++kk) {
    const int kc = SPLIT ? k : kk;
    Folded<SP, float> F;
    fold_query<SP, float>(xq, kc, vol, F);
    const int ob = SP::template orbit<float>(F.up);
    float mono[SP::NMON];
    monomials<SP, float>(F.up, ob, mono);
    bool staged = false;
    if constexpr (LDS_G) {
      staged = stageable<SP, float>(si, F);
      if (staged) {
        if constexpr (box_pieces<SP>()) {
          BoxScatterLds<SP> sc;
          sc.init(lds_g + kk * si.vol, si, F, ldexpf(gq, shift));
          SP::template w_any<float>(ob, sc, mono);
          sc.flush();
        } else {
          ScatterLds<SP> sc;
          sc.init(lds_g + kk * si.vol, si, F, ldexpf(gq, shift));
          SP::template w_any<float>(ob, sc, mono);
        }
      } else {
        ok = false;
      }
    } else if (F.interior) {
      Scatter<SP, false> sc;
      sc.init(vol, pick<SP::M>(gvol.base, kc), F, gq);
      SP::template w_any<float>(ob, sc, mono);
    } else {
      Scatter<SP, true> sc;
      sc.init(vol, pick<SP::M>(gvol.base, kc), F, gq);
      SP::template w_any<float>(ob, sc, mono);
    }
    if constexpr (GRADX) {
      float b[SP::NMON];
      if constexpr (STAGE_C) {
        if (staged) {
          if constexpr (box_pieces<SP>()) {
            BoxGatherLds<SP, float> gg;
            gg.init(lds_c + kk * si.vol, si, F);
            SP::template b_any<float>(ob, gg, b);
          } else {
            GatherLds<SP, float> gg;
            gg.init(lds_c + kk * si.vol, si, F);
            SP::template b_any<float>(ob, gg, b);
          }
        } else {
#pragma unroll
          for (int m = 0; m < SP::NMON; ++m) b[m] = __builtin_nanf("");
        }
      } else if (F.interior) {
        Gather<SP, CT, float, false> gg;
        gg.init(vol, kc, F);
        SP::template b_any<float>(ob, gg, b);
      } else {
        Gather<SP, CT, float, true> gg;
        gg.init(vol, kc, F);
        SP::template b_any<float>(ob, gg, b);
      }
      float dpsi[SP::S];
      (void)poly_eval<SP, float, true>(b, mono, dpsi);
      unfold_grad<SP, float>(F, dpsi, gx);
    }
  }
  if constexpr (GRADX) {
    const long long slot = SPLIT ? static_cast<long long>(k) * g.n + q : q;
#pragma unroll
    for (int d = 0; d < SP::S; ++d) grad_x[slot * SP::S + d] = gq * gx[d];
  }
  return ok;
}

// 5a. adjoint, one workgroup per unit: scatter-add g * w into an LDS copy of
// the unit's region, then store the region to the unit's private slot
// priv[unit][ncos][vol] with plain writes (k_adjoint_gather sums the slots).
// Queries outside the brick grid are not in any unit (k_adjoint_outliers).
//   GRADX, not SPLIT: grad_x[q] = g_q * grad f; SPLIT: gpart[k * n + q].
template <class SP, class CT, bool GRADX, bool SPLIT, bool STAGE_C>
__global__ void __launch_bounds__(512) k_adjoint_binned(Vol vol, GradVol gvol, BinGeom g,
                                                        const Rec<SP::S>* __restrict__ recs,
                                                        const unsigned* __restrict__ start,
                                                        const float* __restrict__ gout, float* __restrict__ grad_x,
                                                        float* __restrict__ priv, const unsigned* __restrict__ gmax_bits,
                                                        int g_sorted) {
  extern __shared__ unsigned char smem[];
  UnitRange u;
  if (!unit_range<SPLIT>(g, start, u)) return;
  StageInfo<SP, float> si;
  stage_info<SP, float>(g, u.brick, si);
  constexpr int NC = SPLIT ? 1 : SP::M;
  unsigned long long* lds_g = reinterpret_cast<unsigned long long*>(smem);   // fixed-point gradient region
  float* lds_c = reinterpret_cast<float*>(lds_g + NC * si.vol);               // coefficient region (STAGE_C)
  const float gmax = __uint_as_float(*gmax_bits);
  const int shift = unit_shift(u.hi - u.lo, gmax);
  for (int e = threadIdx.x; e < NC * si.vol; e += blockDim.x) lds_g[e] = 0ull;
  if constexpr (STAGE_C) stage_load<SP, CT, float>(vol, si, SPLIT ? u.kunit : 0, NC, lds_c);
  __syncthreads();
  // software pipeline: records are loaded two queries ahead, the (randomly
  // placed) upstream gradient one query ahead, so a whole query's work hides
  // each load
  // g_sorted: gout holds g in schedule order (item t), else by query
  const unsigned last = u.hi - 1;
  Rec<SP::S> cur = recs[min(u.lo + threadIdx.x, last)];
  Rec<SP::S> nxt = recs[min(u.lo + threadIdx.x + blockDim.x, last)];
  float gcur = g_sorted ? gout[min(u.lo + threadIdx.x, last)] : gout[rec_query<SP, SPLIT>(cur)];
  int bad = 0;
  for (unsigned t = u.lo + threadIdx.x; t < u.hi; t += blockDim.x) {
    const Rec<SP::S> nn = recs[min(t + 2 * blockDim.x, last)];
    const float gnxt = g_sorted ? gout[min(t + blockDim.x, last)] : gout[rec_query<SP, SPLIT>(nxt)];
    float xq[SP::S];
    const unsigned item = rec_item<SP>(cur, xq);
    const float gq = gcur;
    cur = nxt;
    nxt = nn;
    gcur = gnxt;
    if (!adjoint_item<SP, CT, GRADX, SPLIT, true, STAGE_C>(vol, gvol, g, si, lds_g, lds_c, shift, xq, item, gq,
                                                           grad_x))
      bad = 1;
  }
  // back to float; a non-finite upstream gradient makes the region NaN (and
  // so would an item outside the region, which the schedule never places in
  // a unit)
  const bool finite = gmax <= 3.402823466e38f && !__syncthreads_or(bad);
  float* out = priv + static_cast<size_t>(u.unit) * NC * si.vol;
  for (int e = threadIdx.x; e < NC * si.vol; e += blockDim.x)
    out[e] = finite ? ldexpf(static_cast<float>(static_cast<long long>(lds_g[e])), -shift) : __int_as_float(0x7fc00000);
}

// 5a'. adjoint of the items under the outlier key (queries outside the brick
// grid): float atomics into grad_c, before the gather pass adds the units'
// regions; a grid-stride loop over the key's records, usually none
template <class SP, class CT, bool GRADX, bool SPLIT>
__global__ void __launch_bounds__(256) k_adjoint_outliers(Vol vol, GradVol gvol, BinGeom g,
                                                          const Rec<SP::S>* __restrict__ recs,
                                                          const unsigned* __restrict__ start,
                                                          const float* __restrict__ gout, float* __restrict__ grad_x,
                                                          int g_sorted) {
  const unsigned lo = start[g.okey], hi = start[g.okey + 1];
  StageInfo<SP, float> si{};
  for (unsigned t = lo + blockIdx.x * blockDim.x + threadIdx.x; t < hi; t += gridDim.x * blockDim.x) {
    float xq[SP::S];
    const unsigned item = rec_item<SP>(recs[t], xq);
    long long q;
    int k;
    split_item<SP, SPLIT>(item, q, k);
    const float gq = g_sorted ? gout[t] : gout[q];
    (void)adjoint_item<SP, CT, GRADX, SPLIT, false, false>(vol, gvol, g, si, nullptr, nullptr, 0, xq, item, gq,
                                                           grad_x);
  }
}

// max |g| over the upstream gradient, as the bits of a non-negative float
// (their unsigned order is the float order; NaN compares above +inf):
// partial maxima per block, then one block reduces them.
__device__ __forceinline__ unsigned block_max_u32(unsigned v, unsigned* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, static_cast<unsigned>(__shfl_xor(static_cast<int>(v), off)));
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < static_cast<int>(blockDim.x / 64); ++w) v = max(v, red[w]);
  }
  return v;
}

template <int = 0>
__global__ void __launch_bounds__(256) k_absmax_partial(const float* __restrict__ gout, long long n,
                                                        unsigned* __restrict__ partial) {
  __shared__ unsigned red[4];
  unsigned m = 0u;
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    m = max(m, __float_as_uint(fabsf(gout[i])));
  m = block_max_u32(m, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

template <int = 0>
__global__ void __launch_bounds__(1024) k_absmax_final(const unsigned* __restrict__ partial, int parts,
                                                       unsigned* __restrict__ out) {
  __shared__ unsigned red[16];
  unsigned m = 0u;
  for (int i = threadIdx.x; i < parts; i += blockDim.x) m = max(m, partial[i]);
  m = block_max_u32(m, red);
  if (threadIdx.x == 0) *out = m;
}

// n / d for any 32-bit n by a multiply-high (Granlund and Montgomery's
// round-up method): l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1,
// t = mulhi(m, n), n / d = (t + ((n - t) >> 1)) >> (l - 1); l = 0 means d = 1.
struct UDiv {
  unsigned m;
  int l;
};

__host__ inline UDiv make_udiv(unsigned d) {
  if (d <= 1u) return UDiv{0u, 0};
  int l = 0;
  while ((1ull << l) < d) ++l;
  return UDiv{static_cast<unsigned>(((1ull << 32) * ((1ull << l) - d)) / d + 1ull), l};
}

__device__ __forceinline__ unsigned udiv(unsigned n, UDiv v) {
  if (v.l == 0) return n;
  const unsigned t = __umulhi(v.m, n);
  return (t + ((n - t) >> 1)) >> (v.l - 1);
}

// divisors of the gather pass's index decomposition: the row length d0 (short
// rows) and the extents of axes 1 .. S-1
struct GatherDiv {
  UDiv d0;
  UDiv dim[kMaxDim];
};

// 5b. grad_c[k][site] += sum of the private regions of the units covering the
// site.  blockIdx.y is the coset; a block covers a run of 256 sites along
// axis 0 of one row of the other axes, or, for short rows (n_0 < 256), rpb
// whole rows.  Every index is 32-bit.
template <class SP, bool SPLIT>
__global__ void __launch_bounds__(256) k_adjoint_gather(Vol vol, GradVol gvol, BinGeom g,
                                                        const unsigned* __restrict__ start,
                                                        const float* __restrict__ priv, unsigned segs,
                                                        unsigned rpb, unsigned rows, GatherDiv gd) {
  constexpr int S = SP::S;
  constexpr int NC = SPLIT ? 1 : SP::M;
  constexpr int MG = Staged<SP>::MARGIN;
  const int k = static_cast<int>(blockIdx.y);
  const unsigned d0 = static_cast<unsigned>(vol.dims[0]);
  const unsigned blk = blockIdx.x / segs;
  const unsigned seg = blockIdx.x - blk * segs;
  const unsigned roff = rpb == 1 ? 0u : udiv(threadIdx.x, gd.d0);
  int c[S];
  c[0] = static_cast<int>(rpb == 1 ? seg * 256u + threadIdx.x : threadIdx.x - roff * d0);
  const unsigned row = blk * rpb + roff;
  if (roff >= rpb || c[0] >= static_cast<int>(d0) || row >= rows) return;
  {
    unsigned r = row;
#pragma unroll
    for (int d = 1; d < S; ++d) {
      const unsigned qd = udiv(r, gd.dim[d]);
      c[d] = static_cast<int>(r - qd * static_cast<unsigned>(vol.dims[d]));
      r = qd;
    }
  }
  const int bs = g.bshift;
  const int W = Staged<SP>::width(1 << bs);
  const int vol_r = Staged<SP>::volume(1 << bs);
  // bricks b whose region [b B - MARGIN + OMIN, b B + B - 1 + OMAX] holds c
  // (arithmetic shifts floor negative values)
  int blo[S], bcnt[S];
#pragma unroll
  for (int d = 0; d < S; ++d) {
    int lo = (c[d] - SP::OMAX) >> bs;
    int hi = (c[d] + MG - SP::OMIN) >> bs;
    lo = lo < 0 ? 0 : lo;
    hi = hi >= g.nb[d] ? g.nb[d] - 1 : hi;
    blo[d] = lo;
    bcnt[d] = hi - lo + 1;
  }
  float sum = 0.f;
  const int n3 = S == 4 ? bcnt[S - 1] : 1;
  for (int i3 = 0; i3 < n3; ++i3)
    for (int i2 = 0; i2 < bcnt[2]; ++i2)
      for (int i1 = 0; i1 < bcnt[1]; ++i1)
        for (int i0 = 0; i0 < bcnt[0]; ++i0) {
          const int idx[4] = {i0, i1, i2, i3};
          unsigned brick = 0, mul = 1;
          int local = 0, ls = 1;
#pragma unroll
          for (int d = 0; d < S; ++d) {
            const int b = blo[d] + idx[d];
            brick += static_cast<unsigned>(b) * mul;
            mul *= static_cast<unsigned>(g.nb[d]);
            local += (c[d] - (b << bs) + MG - SP::OMIN) * ls;
            ls *= W;
          }
          const unsigned unit = brick * g.upb + (SPLIT ? static_cast<unsigned>(k) : 0u);
          const unsigned k0 = unit * g.kpb;
          // an empty unit never wrote its slot: load it anyway (its loads
          // then overlap the emptiness test) and drop the value
          const bool used = start[k0] != start[k0 + g.kpb];
          const float v = priv[(static_cast<size_t>(unit) * NC + (SPLIT ? 0 : k)) * vol_r + local];
          sum += used ? v : 0.f;
        }
  long long off = 0;
#pragma unroll
  for (int d = 0; d < S; ++d) off += static_cast<long long>(c[d]) * vol.stride[d];
  float* gc = pick<SP::M>(gvol.base, k);
  gc[off] += sum;
}

// sum the per-coset grad_x partials of a split adjoint
template <class SP>
__global__ void __launch_bounds__(256) k_combine_gx(const float* __restrict__ gpart, long long n,
                                                    float* __restrict__ grad_x) {
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n * SP::S;
       i += static_cast<long long>(gridDim.x) * blockDim.x) {
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < SP::M; ++k) s += gpart[k * n * SP::S + i];
    grad_x[i] = s;
  }
}

}  // namespace lsp
