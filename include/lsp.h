/*
 * lsp.h -- C ABI of the lattice box-spline evaluation library (gfx950).
 *
 * The library evaluates the lattice convolution sum
 *
 *     f(x) = sum_{n in L Z^s} c_n phi(x - n),    phi(w) = |det L| M_Xi(w + c0),
 *
 * (Horacsek & Alim, "Automatic Generation of Interpolants for Lattice
 * Samplings: Part I", Eq. conv_sum with h = 1) for a box spline M_Xi (Sec. 3,
 * box-spline definition) centred at the origin (c0 = half the sum of the
 * directions) and scaled to a partition of unity on the lattice (the
 * requirement on phi stated in Sec. 4.1), at many query points, with the
 * paper's fast scheme (Sec. 4, Algorithm 1).  It also gives the spatial
 * gradient, the adjoint (transpose) of c -> f, a mean-squared-error head, a
 * ray-marching sample generator and a volume renderer (Sec. 5.1), and a
 * cache-friendly evaluation order for large random query batches
 * (lsp_schedule and the *_scheduled entry points).
 *
 * Conventions
 *  - Status: every function returns lsp_status (0 = LSP_OK, < 0 error); no
 *    exception or abort crosses the ABI.  lsp_status_string() describes a code.
 *  - Lattice storage (Sec. 4.1, Cartesian coset decomposition GL = D I): the
 *    lattice is the union of M cosets D Z^s + l_k, D the smallest positive
 *    integer with D Z^s inside L Z^s, shifts l_k in [0, D)^s ordered by
 *    sum_a l_a D^a (l_0 = 0).  Coset k is an s-D array; element i (x index
 *    fastest) holds c at the lattice site D i + l_k.  Sites outside the
 *    stored arrays have c = 0 (zero extension).
 *  - Queries: N x s float32, row-major, world coordinates (h = 1).  NaN or
 *    infinite queries yield NaN outputs and never read out of bounds.
 *  - Memory: all data pointers are device pointers owned by the caller and
 *    must stay valid until the work queued on the stream completes.  Plans
 *    own their host tables only.  No entry point allocates device memory or
 *    synchronises; all work is queued on `stream` (a hipStream_t, NULL for
 *    the default stream).
 *  - Supported splines: the library ships generated tables for a fixed set
 *    of (lattice, direction matrix) pairs (lsp_plan_create matches L by its
 *    coset structure and Xi up to column order and column signs), and of
 *    Voronoi splines (lsp_plan_create_voronoi): phi = |det L| V_n, with V_n
 *    the (n+1)-fold self-convolution of the normalised indicator of the
 *    Voronoi cell of a lattice L_v contained in L (Sec. 3, Voronoi splines).
 *    Every entry point below works the same for both kinds of plan.
 */
#ifndef LSP_H
#define LSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lsp_status;
#define LSP_OK 0
#define LSP_ERR_NULL (-1)          /* a required pointer is NULL */
#define LSP_ERR_INVALID (-2)       /* malformed argument (sizes, rank, lattice) */
#define LSP_ERR_UNSUPPORTED (-3)   /* no generated tables for this (L, Xi) */
#define LSP_ERR_DTYPE (-4)         /* unknown or mismatched dtype */
#define LSP_ERR_DIMS (-5)          /* coefficient dims out of range */
#define LSP_ERR_HIP (-6)           /* a HIP runtime call failed */
#define LSP_ERR_NOT_ON_LATTICE (-7)/* a direction of Xi is not a lattice vector */
#define LSP_ERR_TOO_LARGE (-8)     /* the input needs more than the library's static scratch */

/* coefficient storage types */
#define LSP_F32 0
#define LSP_BF16 1   /* bfloat16 (upper half of an IEEE float32) */
#define LSP_F16 2    /* IEEE half */
#define LSP_F64 3    /* float64: evaluation then runs in FP64 (accuracy check) */

typedef struct lsp_plan_s* lsp_plan;
typedef struct lsp_vol_s* lsp_vol;

typedef struct {
  int32_t s;                /* dimension */
  int32_t n_dirs;           /* directions in Xi */
  int32_t det_l;            /* |det L| */
  int32_t D;                /* coset sub-lattice spacing */
  int32_t n_cosets;         /* M */
  int32_t shifts[8][4];     /* coset shifts l_k */
  int32_t degree;           /* polynomial degree of the pieces (n - s) */
  int32_t n_subregions;     /* K: non-equivalent sub-regions after the fold */
  int32_t n_planes;         /* Q: splitting planes inside the fold chamber */
  int32_t fold_even;        /* 1 if the fold group is the even-sign subgroup */
  int32_t stencil[16];      /* sites gathered per coset, per sub-region */
  int32_t lookups;          /* sites with nonzero weight per query (Table 1) */
  int32_t n_monomials;      /* monomials per polynomial piece */
  int32_t nnz[16];          /* nonzero polynomial coefficients per sub-region */
  int32_t offset_min;       /* per-axis site offset range around the cell */
  int32_t offset_max;
  char name[32];            /* spline name */
  /* operation counts of the generated polynomial code, per coset and query:
   * fma_b[k] multiply-adds of b = A c (the piece's monomial coefficients from
   * the gathered stencil) and fma_w[k] of the stencil weights w = A^T mono
   * (adjoint), both after common-subexpression factoring, for sub-region k;
   * grad_terms: multiply-adds of the gradient from b and the monomials */
  int32_t fma_b[16];
  int32_t fma_w[16];
  int32_t grad_terms;
  int32_t kind;             /* 0: box spline; 1: Voronoi spline (n_dirs counts the cell's zonotope generators) */
  int32_t voronoi_n;        /* Voronoi splines: n of V_n */
} lsp_info;

/* Create a plan for lattice L (s x s, row-major; columns generate the lattice)
 * and direction matrix Xi (s x n, row-major; columns are the directions),
 * s in {3, 4}.  Errors: LSP_ERR_NULL, LSP_ERR_INVALID (singular L, n < s),
 * LSP_ERR_NOT_ON_LATTICE (a direction outside L Z^s, so phi would not be a
 * partition of unity), LSP_ERR_UNSUPPORTED.  flags: reserved, pass 0. */
lsp_status lsp_plan_create(int32_t s, const int32_t* L, int32_t n, const int32_t* Xi, uint32_t flags,
                           lsp_plan* out);
/* Create a plan for the Voronoi spline V_n of the lattice Lv (s x s,
 * row-major, columns generate it) used on the lattice L (s x s): phi(w) =
 * |det L| V_n(w), V_0 = 1/|det Lv| on the Voronoi cell of Lv (the points at
 * least as close to the origin as to any other site of Lv) and V_n =
 * V_0 * V_{n-1} (Sec. 3, Voronoi splines).  phi is a partition of unity on L
 * because Lv is a sublattice of L.  Shipped: BCC and FCC V_1 on their own
 * lattices and on Z^3, FCC V_2 on FCC and on Z^3 (Table 1's Voronoi rows).  Lv is
 * matched as a lattice (any basis).  Errors: LSP_ERR_NULL, LSP_ERR_INVALID
 * (singular L or Lv, n < 1), LSP_ERR_NOT_ON_LATTICE (Lv not inside L),
 * LSP_ERR_UNSUPPORTED (no tables).  flags: reserved, pass 0. */
lsp_status lsp_plan_create_voronoi(int32_t s, const int32_t* L, const int32_t* Lv, int32_t n, uint32_t flags,
                                   lsp_plan* out);
lsp_status lsp_plan_info(lsp_plan plan, lsp_info* out);
lsp_status lsp_plan_destroy(lsp_plan plan);

/* Bind M device arrays (one per coset, in shift order) of dtype `dtype` and
 * dims[0..s-1] (x first; same for every coset; each dim in [1, 2^20], total
 * elements below 2^31).  The view is non-owning. */
lsp_status lsp_vol_bind(lsp_plan plan, int32_t dtype, const void* const* coset_ptrs, const int64_t* dims,
                        lsp_vol* out);
lsp_status lsp_vol_release(lsp_vol vol);

/* Forward (Algorithm 1): f[q] for N queries x (device, N x s float32).  f and
 * grad_x are float32, or float64 when the volume is LSP_F64.  grad_x (N x s,
 * row-major) may be NULL; otherwise it receives the spatial gradient of f. */
lsp_status lsp_eval(lsp_plan plan, lsp_vol vol, const float* x, int64_t n, void* f, void* grad_x,
                    void* stream);

/* Forward with a mean-squared-error head against targets y (N float32):
 * writes f (unless f is NULL: a training step needs only the loss and the
 * gradients), dL/df = 2 (f - y) / N (unless dloss_df is NULL), and adds
 * L = sum (f - y)^2 / N to *loss
 * (float64; the caller zeroes it).  If dloss_dx is not NULL it also receives
 * dL/dx = dL/df * grad f (N x s) -- the loss gradient for the queries, known
 * already in the forward pass.  Float32/bf16/f16 volumes. */
lsp_status lsp_eval_mse(lsp_plan plan, lsp_vol vol, const float* x, const float* y, int64_t n, float* f,
                        float* dloss_df, float* dloss_dx, double* loss, void* stream);

/* Adjoint: for upstream gradients g (N float32) adds sum_q g_q phi(x_q - site)
 * into grad_c (M float32 device arrays shaped like the volume; the caller
 * zeroes them; FP32 atomics, so the summation order is not deterministic)
 * and, if grad_x is not NULL, writes grad_x[q] = g_q * grad f(x_q) (N x s).
 * Float32/bf16/f16 volumes. */
lsp_status lsp_eval_adjoint(lsp_plan plan, lsp_vol vol, const float* x, const float* g, int64_t n,
                            float* const* grad_c, float* grad_x, void* stream);

/* Ray-marched samples (3-D only): ray r in [ray0, ray0 + nrays) covers pixel
 * (u, v) in 8x8 tiles (tile = r / 64 in row-major tile order, within-tile
 * index r % 64 = (v % 8) * 8 + u % 8) of a W x H image; its samples are
 *   p_j = c + A ((2u+1)/W - 1, (2v+1)/H - 1, (2j+1)/steps - 1),  j < steps,
 * every product and sum rounded to float32 (no fused multiply-add).  Writes
 * per ray (sum_j f, sum_j grad f) as 4 floats to out (nrays x 4); if samples
 * is not NULL also every sample's (f, grad f) (nrays x steps x 4).
 * W and H multiples of 8; c[3], A[9] row-major host arrays. */
lsp_status lsp_eval_rays(lsp_plan plan, lsp_vol vol, const float* c, const float* A, int32_t W, int32_t H,
                         int32_t steps, int64_t ray0, int64_t nrays, float* out, float* samples, void* stream);

/* Volume rendering (3-D only; the application the paper measures in Sec. 5.1:
 * volumetric, not iso-surface, with a mostly transparent transfer function so
 * that rays cross the whole volume).  Rays and samples as in lsp_eval_rays.
 * Each sample's f selects an RGBA value from the transfer function tf
 * (device, tf_len float4 entries, 16-byte aligned; entry 0 at f0, entry
 * tf_len - 1 at f1, linear in between, clamped outside); its colour is shaded
 * with grad f as the normal under a light along the ray direction d:
 *   shade = ambient + diffuse |grad f . d| / |grad f|
 * (ambient + diffuse where |grad f| <= grad_eps), and the samples are
 * composited front to back from sample 0:
 *   C += (1 - A) alpha shade rgb,   A += (1 - A) alpha,
 * stopping once A >= alpha_stop (a value above 1 marches every step).
 * Writes (C, A) per ray to rgba (device, nrays x 4 float32, 16-byte aligned).
 * Errors: LSP_ERR_INVALID for bad geometry, tf_len < 2, f1 <= f0 or
 * grad_eps < 0; LSP_ERR_DTYPE for LSP_F64 volumes. */
typedef struct lsp_render_params {
  float f0, f1;             /* transfer-function domain */
  float ambient, diffuse;   /* shading weights */
  float grad_eps;           /* below this gradient norm the sample is unshaded */
  float alpha_stop;         /* early ray termination threshold */
  int32_t tf_len;           /* transfer-function entries (>= 2) */
} lsp_render_params;

lsp_status lsp_render(lsp_plan plan, lsp_vol vol, const float* c, const float* A, int32_t W, int32_t H,
                      int32_t steps, int64_t ray0, int64_t nrays, const float* tf,
                      const lsp_render_params* params, float* rgba, void* stream);

/* Query schedule (evaluation order).  Random queries gather from random
 * places of the volume; ordering the work items so that neighbouring lanes
 * read neighbouring coefficients makes the stencil gathers hit the caches
 * (the paper notes that combining the reads of a coset exploits data
 * locality, Sec. 4).  lsp_schedule computes that order with a counting sort
 * on the GPU (per-tile LDS histograms, a scan, and a placement pass that
 * writes each query's record to its sorted position): key = brick of cells
 * (8^s cells, coarser when there would be more than 16384 keys) and, for
 * splines whose several sub-regions carry costly polynomials, the
 * sub-region -- an item is then one (query, coset) pair, so a wave evaluates
 * one polynomial set instead of predicating all of them (Sec. 4.3).  The
 * scheduled calls run one workgroup per unit (a brick, or a (brick, coset)
 * pair for coset-split items), which in 3-D stages the unit's coefficients
 * plus the stencil halo in LDS.  The scheduled adjoint accumulates its
 * scatter-add in an LDS copy of the unit's region, stores it to a private
 * slot of the workspace, and a gather pass sums the slots covering every site
 * (no global atomics, fixed order per site; only queries outside the volume
 * scatter with atomics).
 *
 * lsp_schedule_size: device workspace bytes for n queries (depends on the
 * plan, the volume dims and n).  lsp_schedule: fills that caller-owned,
 * 256-byte aligned workspace from the queries x (no allocation).  The
 * *_scheduled calls then evaluate the same x (same n) in that order; results
 * land at each query's own index, exactly as the unscheduled calls.
 * Errors: LSP_ERR_NULL, LSP_ERR_INVALID (workspace too small or misaligned,
 * n * cosets >= 2^32).  The scheduled adjoint sums each unit's terms in
 * 64-bit fixed point (scale: a power of two from max |g|, terms resolved to
 * 2^-49 max|g| or finer for units of fewer than 2048 items), so its result does
 * not depend on the order of the additions; a non-finite g makes the
 * affected grad_c entries NaN, while a query that is not finite adds nothing
 * to grad_c and gets a NaN grad_x (the given-order adjoint turns that
 * query's sites NaN).
 * Items whose stencil leaves their unit's
 * region (queries outside the stored volume), and volumes whose units do
 * not fit in LDS, fall back to float atomics. */
lsp_status lsp_schedule_size(lsp_plan plan, lsp_vol vol, int64_t n, size_t* bytes);
lsp_status lsp_schedule(lsp_plan plan, lsp_vol vol, const float* x, int64_t n, void* workspace, size_t ws_bytes,
                        void* stream);
lsp_status lsp_eval_scheduled(lsp_plan plan, lsp_vol vol, const float* x, int64_t n, const void* workspace,
                              size_t ws_bytes, void* f, void* grad_x, void* stream);
lsp_status lsp_eval_mse_scheduled(lsp_plan plan, lsp_vol vol, const float* x, const float* y, int64_t n,
                                  const void* workspace, size_t ws_bytes, float* f, float* dloss_df, float* dloss_dx,
                                  double* loss, void* stream);
lsp_status lsp_eval_adjoint_scheduled(lsp_plan plan, lsp_vol vol, const float* x, const float* g, int64_t n,
                                      const void* workspace, size_t ws_bytes, float* const* grad_c, float* grad_x,
                                      void* stream);

/* The backward of a scheduled MSE step without handing dL/df back and forth:
 * adds sum_q (dL/df)_q phi(x_q - site) into grad_c (as lsp_eval_adjoint_
 * scheduled with g = dL/df), reading the dL/df that the preceding
 * lsp_eval_mse_scheduled call on the same queries and workspace left in the
 * workspace (in schedule order, so the reads are coalesced).  With this call
 * that forward may pass dloss_df = NULL.  LSP_ERR_UNSUPPORTED when the
 * volume's units do not fit in LDS (use lsp_eval_adjoint_scheduled then). */
lsp_status lsp_mse_backward_scheduled(lsp_plan plan, lsp_vol vol, const float* x, int64_t n, const void* workspace,
                                      size_t ws_bytes, float* const* grad_c, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the binned
 * forward of lsp_schedule + lsp_eval_scheduled in one call, with the schedule
 * workspace taken from a static device array of LSP_STATIC_SCRATCH_BYTES
 * (64 MiB) that each GPU the library runs on holds until the process ends.
 * Arguments and outputs are those of lsp_eval_scheduled without the workspace;
 * f and grad_x are written in query order.  LSP_ERR_TOO_LARGE when the
 * part of the schedule workspace the forward uses (key histograms, records
 * and per-coset partials: roughly 16-24 bytes per 3-D query plus the key
 * histograms) exceeds the scratch; nothing is launched then.  Every call on one GPU shares that
 * GPU's scratch and leaves it holding the last call's schedule: calls that
 * overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  Allocates nothing. */
#define LSP_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
lsp_status lsp_eval_scheduled_static(lsp_plan plan, lsp_vol vol, const float* x, int64_t n, void* f, void* grad_x,
                                     void* stream);

const char* lsp_status_string(lsp_status status);

#ifdef __cplusplus
}
#endif

#endif /* LSP_H */
