/*
 * gsp2.h - graph-partitioned SP2 (G-SP2) density matrices on AMD Instinct
 * MI355X (gfx950).  C ABI of libgsp2.so.
 *
 * Method: Ghale et al., "Task-based Parallel Computation of the Density
 * Matrix in Quantum-based Molecular Dynamics using Graph Partitioning",
 * arXiv:1801.10016.  A previous density matrix P_prev is thresholded into an
 * undirected graph G_tau (Methods, "Graph Theory"); a given partition of its
 * vertices defines, for every part, a core (the part's vertices) and a halo
 * (vertices outside the part adjacent to a core vertex); each part's dense
 * core+halo sub-block of H is purified by SP2 (Methods, eqs. (1)-(3)) with a
 * branch sequence common to all parts, chosen from the summed core trace;
 * each part's core columns are reassembled into the sparse P (Fig. 1
 * description in the Introduction).
 *
 * Conventions for every call:
 *  - Every function returns gsp2_status; nothing throws or aborts across
 *    the ABI.  On failure gsp2_last_error() gives a thread-local message.
 *  - "device" pointers are HIP device memory on the current device; "host"
 *    pointers are ordinary host memory.  The caller owns every buffer it
 *    passes; the library owns the plan and its device workspace.
 *  - Indices are 0-based.  CSR arrays: row_ptr has n+1 int64 entries,
 *    col has nnz int32 entries, val has nnz entries of type `dtype`.
 *    Column indices of a row need not be sorted; duplicates are not allowed.
 *  - Work is enqueued on the plan's HIP stream (set at creation, changed
 *    with gsp2_plan_set_stream) in stream order.
 */
#ifndef GSP2_H
#define GSP2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GSP2_OK = 0,
    GSP2_E_INVALID = 1,        /* bad argument, size mismatch, empty part, non-finite H */
    GSP2_E_HIP = 2,            /* a HIP runtime call failed */
    GSP2_E_OOM = 3,            /* device or host allocation failed */
    GSP2_E_NOT_CONVERGED = 4,  /* the stop rule did not fire within max_iter products (or was
                                  switched off), or the iteration left the finite range */
    GSP2_E_WRONG_TRACE = 5,    /* the returned P's trace misses n_occ by more than trace_tol */
    GSP2_E_UNSUPPORTED = 6     /* option not available in this library */
} gsp2_status;

typedef enum { GSP2_F32 = 0, GSP2_F64 = 1 } gsp2_dtype;

typedef enum {
    GSP2_ALPHA_TRACE = 0,      /* branch from the summed core trace each product */
    GSP2_ALPHA_REPLAY = 1      /* branch sequence supplied by the caller */
} gsp2_alpha_mode;

/* Operand precision of the SP2 products.  Accumulation, the master copy of
 * every iterate and the eq. (2) update are FP32 in all modes but
 * GSP2_PREC_FP64, where they are FP64; traces are FP64 in every mode. */
typedef enum {
    GSP2_PREC_FP32 = 0,        /* FP32 operands (v_mfma_f32_32x32x2_f32) */
    GSP2_PREC_FP16 = 1,        /* FP16 operands (v_mfma_f32_32x32x16_f16) */
    GSP2_PREC_BF16 = 2,        /* BF16 operands (v_mfma_f32_32x32x16_bf16) */
    GSP2_PREC_FP16X3 = 3,      /* split FP16 operands: X = A + 2^-11 B with A = fp16(X) and
                                  B = fp16(2^11 (X - A)); X^2 as 2^-11 (A B + B A) + A A, three
                                  FP16 products accumulated in FP32, about as accurate as FP32
                                  products (the dropped B B term is 2^-22 relative) */
    GSP2_PREC_FP64 = 4         /* FP64 operands, accumulation, iterate and update
                                  (v_mfma_f64_16x16x4_f64): the double-precision dgemm
                                  arithmetic of the paper's runs (Results); P is written in FP64 */
} gsp2_precision;
/* Forms of the product kernel; gsp2_plan_tune times them on a plan's own
 * sub-problems and keeps the fastest per precision.  All forms of one
 * precision give the same arithmetic.  T128 and T128_SKIP give the same bits
 * for FP32, FP16 and BF16 operands; with split FP16 operands a block above
 * the diagonal of a diagonal tile sums its two cross terms in the other
 * order than the block below it, so there the two forms agree to FP32
 * rounding (T128_SKIP mirrors the block above, T128 forms both). */
typedef enum {
    GSP2_KERNEL_AUTO = 0,      /* the form gsp2_plan_tune kept for the precision, else the default:
                                  T128_SKIP for FP32 and FP64 products, T256 for 16-bit ones */
    GSP2_KERNEL_T128 = 1,      /* 128 x 128 product tiles, two workgroups per CU, every 32 x 32
                                  block of the padded tile formed */
    GSP2_KERNEL_T128_SKIP = 2, /* 128 x 128 tiles; 32 x 32 blocks lying wholly in the zero padding,
                                  and the blocks below the diagonal of a diagonal tile (transposes
                                  of blocks above it), form no products, and the blocks a tile
                                  forms are dealt evenly to its four waves. */
    GSP2_KERNEL_T256 = 3       /* 256 x 256 tiles, one workgroup per CU; 16-bit operands only */
} gsp2_kernel;

/* The 16-bit modes need every part's padded size (s_k rounded up to 128) to
 * be at most 46,336, so that a part's operand matrix is under 4 GiB; larger
 * plans get GSP2_E_UNSUPPORTED from gsp2_density for those modes. */

/* Sparse matrix in CSR form.  All four arrays are device pointers. */
typedef struct {
    int32_t n;                 /* rows = columns */
    int64_t nnz;
    const int64_t *row_ptr;    /* device, n+1 */
    const int32_t *col;        /* device, nnz */
    const void *val;           /* device, nnz, gsp2_dtype `dtype` */
    int32_t dtype;             /* GSP2_F32 or GSP2_F64 */
} gsp2_csr;

typedef struct gsp2_plan_s *gsp2_plan;   /* opaque, library-owned */

/* Plan options.  Zero-initialised means defaults. */
typedef struct {
    int32_t tile;              /* macro-tile edge of the FP32 product: 0 = automatic, or 128 */
    int32_t n_systems;         /* independent systems batched in the plan: 0 or 1 = one */
    const int32_t *part_system;/* host, n_parts ids in [0, n_systems), every system used by at
                                  least one part: the system of every part.  Ignored (may be
                                  NULL) when n_systems <= 1. */
    int32_t tile16;            /* macro-tile edge of the 16-bit products: 0 = automatic (the
                                  form gsp2_plan_tune kept for the precision, else 256 x 256
                                  tiles), 128 or 256 (fixed: GSP2_KERNEL_T128 or T256, which
                                  gsp2_plan_tune does not override; a run's `kernel` does) */
    int32_t reserved[3];
} gsp2_plan_options;

/* Summary of a plan, filled by gsp2_plan_query. */
typedef struct {
    int32_t n;                 /* vertices (rows of H and P) */
    int32_t n_parts;
    int32_t max_s;             /* largest sub-problem s_k = c_k + h_k */
    int32_t min_s;
    int64_t nnz_graph;         /* off-diagonal entries of P_prev with |value| > tau */
    int64_t nnz_P;             /* stored entries of P: sum_k c_k s_k */
    int64_t sum_s;             /* sum_k s_k */
    double sum_s3;             /* eq. (4): C = sum_k s_k^3 */
    int32_t tile;              /* macro-tile edge in use */
    int32_t n_tiles;           /* product tiles per SP2 iteration (upper triangles) */
    int64_t workspace_bytes;   /* device memory held by the plan */
    double plan_ms;            /* host wall time of gsp2_plan_create */
    int32_t n_systems;         /* independent systems in the plan (1 unless batched) */
    int32_t pad_;
} gsp2_plan_info;

/* Options of one density-matrix computation.  Fill with
 * gsp2_run_options_default() and change what is needed. */
typedef struct {
    int32_t max_iter;          /* most matrix products per P (1..GSP2_MAX_ITER), default 60 */
    int32_t alpha_mode;        /* gsp2_alpha_mode, default GSP2_ALPHA_TRACE */
    const int8_t *alpha_seq;   /* host, replay mode only: n_alpha entries, each +1 or -1 */
    int32_t n_alpha;           /* replay mode: number of products to apply (<= GSP2_MAX_ITER) */
    int32_t stop_rule;         /* trace mode: 1 = stop when idempotency stops improving
                                  (default); 0 = always form max_iter products (the run then
                                  ends with GSP2_E_NOT_CONVERGED: nothing shows convergence) */
    double trace_tol;          /* allowed |Tr P - n_occ| of the returned P, checked at the end of
                                  every run (trace mode: after the stop and any refinement;
                                  replay mode: after the replayed branches), default 0.5 */
    int32_t timing;            /* 1 = record HIP events around every phase and product
                                  (read with gsp2_run_timing); default 0 */
    int32_t precision;         /* gsp2_precision of the products, default GSP2_PREC_FP32 */
    int32_t refine;            /* refinement products (FP32, split FP16 with refine_precision, FP64
                                  in GSP2_PREC_FP64 runs) appended
                                  after the stop, alternating X^2 and 2X - X^2, 0..8, default 0;
                                  max_iter + refine <= GSP2_MAX_ITER */
    int32_t persistent;        /* must be 0 (one launch per product, all in one HIP graph).
                                  1 would put all products before the stop in one persistent
                                  launch with a grid barrier per product; that path is switched
                                  off in this library and returns GSP2_E_UNSUPPORTED. */
    /* Batched plans only (n_systems > 1); NULL otherwise. */
    const double *n_occ_system;      /* host, n_systems: occupation of every system (required;
                                        replaces the n_occ argument of gsp2_density) */
    const int8_t *alpha_seq_system;  /* host, replay mode: n_systems rows of GSP2_MAX_ITER
                                        branches, row-major; NULL = alpha_seq for every system */
    const int32_t *n_alpha_system;   /* host, n_systems lengths of those rows (<= GSP2_MAX_ITER) */
    int32_t symmetrize;        /* 0 (default): P[idx_k, j] = X_k[:, j] as assembled from each
                                  part's core columns, which need not be symmetric; 1: every
                                  stored entry whose mirror is stored too becomes the mean of the
                                  two, and an entry whose mirror lies outside P's pattern is kept */
    int32_t kernel;            /* gsp2_kernel of the products, default GSP2_KERNEL_AUTO; anything
                                  else overrides the plan's tile16 and the tuned form.  The FP32
                                  refinement products use the FP32 form (tuned or default). */
    int32_t refine_precision;  /* operands of the refinement products: GSP2_PREC_FP32 (default) or,
                                  after 16-bit products (FP16 or BF16), GSP2_PREC_FP16X3: split FP16
                                  products on 256 x 256 tiles, about as accurate as FP32 ones at a
                                  third of their time; the iterate is split into its two FP16
                                  parts once, when the main phase ends */
    int32_t pad2_;
} gsp2_run_options;

#define GSP2_MAX_ITER 100

/* Outcome of one density-matrix computation (filled when info != NULL). */
typedef struct {
    int32_t status;            /* gsp2_status of the run */
    int32_t n_products;        /* products formed, including a discarded last one */
    int32_t n_alpha;           /* branches applied to reach the returned P */
    int32_t result_iterate;    /* index t of the returned iterate X_t */
    int32_t n_refine;          /* refinement products among n_products */
    int32_t precision;         /* gsp2_precision of the run */
    double eps_min, eps_max;   /* Gershgorin bounds of H */
    double trace;              /* summed core trace of the returned P */
    double idempotency;        /* e_t = Tr[X_t] - Tr[X_t^2] of the returned iterate (NaN if not formed) */
    int8_t alpha[GSP2_MAX_ITER];           /* applied branches, +1 = 2X - X^2, -1 = X^2 */
    double traces[GSP2_MAX_ITER + 1];      /* Tr[X_t], t = 0 .. n_alpha */
    double errors[GSP2_MAX_ITER];          /* e_t for each product t */
} gsp2_run_info;

/* Device times of the last timed run (gsp2_run_options.timing = 1). */
typedef struct {
    int32_t n_products;                    /* entries of product_ms */
    float setup_ms;                        /* Gershgorin bounds, X0 gather, first trace */
    float sp2_ms;                          /* all products with their control steps */
    float scatter_ms;                      /* core columns into P */
    float total_ms;                        /* first to last kernel of the run */
    float persistent_ms;                   /* the persistent product launch (persistent runs) */
    float product_ms[GSP2_MAX_ITER];       /* the product kernel of product t alone (per-product
                                              launches only: refinement products of persistent runs) */
} gsp2_timing;

/* Outcome of one backward pass (filled when info != NULL). */
typedef struct {
    int32_t status;            /* gsp2_status of the pass */
    int32_t n_alpha;           /* products differentiated */
    int32_t checkpoint_every;  /* products per checkpoint segment */
    int32_t row_min, row_max;  /* rows of H attaining eps_min and eps_max */
    double eps_min, eps_max;
    double d_eps_min, d_eps_max;   /* dL/d eps_min, dL/d eps_max */
    int64_t workspace_bytes;   /* temporary device memory the pass used */
} gsp2_backward_info;

/* Human-readable name of a status code (static string). */
const char *gsp2_status_string(gsp2_status s);

/* Message describing the last failure on the calling thread ("" if none). */
const char *gsp2_last_error(void);

/* Fill *opt with the defaults listed in gsp2_run_options. */
gsp2_status gsp2_run_options_default(gsp2_run_options *opt);

/*
 * Build a plan: threshold P_prev into G_tau on the GPU (an edge u-v, u != v,
 * when |P_prev[u,v]| > tau or |P_prev[v,u]| > tau, compared in double
 * precision; Methods, "Graph Theory"), derive every part's core and
 * one-hop halo (core vertices ascending, then halo vertices ascending),
 * allocate the device workspace and upload the index lists.
 *
 *  P_prev  device CSR, n x n (a previous density matrix, or any matrix whose
 *          pattern and magnitudes define the graph).
 *  tau     threshold, >= 0.
 *  part    host, n int32 part ids in [0, n_parts); every part non-empty.
 *  n_parts >= 1.
 *  opt     nullable.
 *  stream  hipStream_t to use (NULL = default stream).
 *  out     receives the plan; NULL on failure.
 * Blocks the calling thread until the graph has been built.
 * Batched plans (opt->n_systems > 1) hold several independent systems, the
 * paper's sub-problem batch taken across systems as well as parts: P_prev, H
 * and P are the block-diagonal unions of the systems (a system's vertices
 * need not be contiguous), opt->part_system names the system of every part,
 * and every product launch carries the tiles of all systems still iterating.
 * Each system keeps its own Gershgorin bounds, occupation, core trace, branch
 * sequence, stop and status, so its P is what a plan of that system alone
 * computes (bit for bit when its parts keep their relative order).
 * Errors: GSP2_E_INVALID (sizes, ids, empty part or system, a graph edge
 * between two systems), GSP2_E_OOM, GSP2_E_HIP.
 */
gsp2_status gsp2_plan_create(const gsp2_csr *P_prev, double tau, const int32_t *part,
                             int32_t n_parts, const gsp2_plan_options *opt, void *stream,
                             gsp2_plan *out);

/* Plan summary; sub_sizes and core_sizes (host, n_parts int32 each) are
 * nullable and receive s_k and c_k.  Errors: GSP2_E_INVALID. */
gsp2_status gsp2_plan_query(gsp2_plan plan, gsp2_plan_info *info, int32_t *core_sizes,
                            int32_t *sub_sizes);

/* CSC pattern of P: column j (in part k) holds the rows of part k's core and
 * halo, in ascending order.  col_ptr: host, n+1 int64; row_idx: host,
 * nnz_P int32.  Errors: GSP2_E_INVALID. */
gsp2_status gsp2_plan_pattern(gsp2_plan plan, int64_t *col_ptr, int32_t *row_idx);

/* Global vertex ids of part k's sub-problem in local order (core ascending,
 * then halo ascending).  idx: host, s_k int32.  Errors: GSP2_E_INVALID. */
gsp2_status gsp2_plan_part_index(gsp2_plan plan, int32_t k, int32_t *idx);

/* Use another HIP stream for later calls on this plan. */
gsp2_status gsp2_plan_set_stream(gsp2_plan plan, void *stream);

/*
 * One density matrix P from H:
 *   eps_min, eps_max from the Gershgorin discs of the whole H (Methods, SP2);
 *   X0_k = (eps_max I - H[idx_k, idx_k]) / (eps_max - eps_min)    (eq. (1));
 *   then, for t = 0, 1, ...: Y_k = X_k X_k on every part (eq. (2)),
 *   e_t = Tr[X_t] - Tr[Y_t]; stop (trace mode, stop_rule = 1) at the first
 *   t >= 2 with |e_t| >= |e_{t-2}| and |e_{t-2}| < max(1, n u), u the unit
 *   roundoff of the product operands (2^-24, 2^-11, 2^-8, 2^-22, 2^-53 for FP32,
 *   FP16, BF16, split FP16, FP64), returning X_t; otherwise
 *   X_k <- 2 X_k - Y_k when Tr[X_t] <= n_occ, else X_k <- Y_k (replay mode:
 *   the supplied branches, then the trace check).  Tr is the sum over parts
 *   of the diagonal of each part's core rows.  P[idx_k, j] = X_k[:, j]
 *   for each core column j of part k; other entries are not stored.
 *   In a batched plan every quantity above (bounds, n, n_occ, traces,
 *   branches, stop) is per system; n is then the system's vertex count and
 *   H must not couple two systems (such entries would only widen the
 *   Gershgorin discs of their rows).
 * Arithmetic: products on the matrix cores with FP32 accumulation and FP32,
 * FP16 or BF16 operands (run->precision); the master iterate and the update
 * stay FP32; Gershgorin bounds, X0 and all traces are FP64.  GSP2_PREC_FP64
 * runs every step in FP64 (operands, accumulation, iterate, update, P).
 * With refine > 0, that many FP32 products (FP64 in FP64 runs) follow the
 * stop (or the last replayed branch), alternating X^2 and 2X - X^2 (each pair
 * a purification sweep that drives every eigenvalue to the nearer of 0 and
 * 1), and the last one is returned.
 * Status: the run fails with GSP2_E_WRONG_TRACE when the returned P's trace
 * misses n_occ by more than run->trace_tol (in trace mode too: a wrong final
 * trace marks a failed SP2 run), and with GSP2_E_NOT_CONVERGED when the stop
 * rule did not fire within max_iter products or was switched off
 * (stop_rule = 0); P_val is written in both cases.
 *
 *  H       device CSR, n x n, symmetric; its pattern may change between calls.
 *  n_occ   number of occupied states N_el / 2, 0 <= n_occ <= n (ignored by
 *          batched plans, which take run->n_occ_system).
 *  run     nullable (defaults).
 *  P_val   device, nnz_P values in the order of gsp2_plan_pattern, doubles
 *          when run->precision is GSP2_PREC_FP64 and floats otherwise;
 *          caller-owned.
 *  info    nullable; otherwise n_systems structs, one per system of the plan.
 *          When given, the call waits for the results and returns the first
 *          failing system's status (GSP2_OK if none); otherwise it returns
 *          after enqueueing.
 * All kernels of the run form one HIP graph, built on the first call and
 * replayed while H's arrays, P_val and the options other than the
 * occupations and replayed branches stay the same (those two are uploaded
 * to the device before each launch).
 * Errors: GSP2_E_INVALID (arguments, non-finite H, eps_max <= eps_min),
 * GSP2_E_NOT_CONVERGED, GSP2_E_WRONG_TRACE, GSP2_E_HIP.  On error the
 * contents of P_val are unspecified.
 */
gsp2_status gsp2_density(gsp2_plan plan, const gsp2_csr *H, double n_occ,
                         const gsp2_run_options *run, void *P_val, gsp2_run_info *info);

/*
 * gsp2_density without allocation, for callers that cannot allocate device
 * memory (code under HIP stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, arithmetic, kernels and results as
 * gsp2_density; the per-run buffers (run state, per-system parameters, trace
 * partials, Gershgorin discs and the iterates: 2 x sum_k s_pad_k^2 values of
 * 4 bytes, 8 in FP64 runs, plus 16-bit operand copies in 16-bit runs) live in
 * a static device array of 64 MiB that every GPU the library runs on holds
 * until the process ends, instead of the plan's workspace.  The kernels are
 * launched directly on the plan's stream (no HIP graph); the plan's own index
 * lists and descriptors (built by gsp2_plan_create) are read as they are.
 * The call makes no hipMalloc, hipFree or other allocation.  Nothing in the
 * array needs clearing: every run writes each part of it before reading it.
 * Every call on one GPU shares the array, which keeps the last call's
 * contents: calls that overlap on one GPU (several streams, several plans,
 * several threads) race, and must be ordered by the caller.
 * gsp2_run_status and gsp2_run_timing keep describing the last gsp2_density
 * run of the plan; pass info to see this call's outcome.
 * Errors: as gsp2_density; GSP2_E_UNSUPPORTED when the run needs more than
 * the static array holds (the message gives both sizes); GSP2_E_INVALID for
 * run->timing = 1 (events would need allocation).
 */
gsp2_status gsp2_density_noalloc(gsp2_plan plan, const gsp2_csr *H, double n_occ,
                                 const gsp2_run_options *run, void *P_val, gsp2_run_info *info);

/* Wait for the last gsp2_density on this plan and report its device times,
 * measured with HIP events on the plan's stream.  Errors: GSP2_E_INVALID
 * when the last run was not timed. */
gsp2_status gsp2_run_timing(gsp2_plan plan, gsp2_timing *out);

/*
 * Reverse mode of gsp2_density for a fixed branch sequence (the sequence of a
 * forward run, from gsp2_run_info.alpha, replayed), with FP32 products:
 *   the seed of part k is dL/dP on its core columns, symmetrised (every
 *   iterate is symmetric; only symmetric perturbations of H are considered);
 *   for each product in reverse, with X_t recomputed from checkpoints taken
 *   every ceil(sqrt(n_alpha)) products: G <- GX + XG after X' = X^2, or
 *   G <- 2G - (GX + XG) after X' = 2X - X^2 (eq. (2));
 *   dL/dH_sub = -G_0 / (eps_max - eps_min) for every part (eq. (1)), summed
 *   over parts into H's stored entries, plus dL/d eps_max = (tr G_0 -
 *   <G_0, X_0>)/D and dL/d eps_min = <G_0, X_0>/D through the Gershgorin
 *   rows that attain the bounds (lowest row on ties).
 * The result is the gradient under symmetric perturbations of H, split evenly
 * between H_uv and H_vu.  FP64 atomics accumulate it, so the summation order
 * (and the last bits) may vary between runs.
 *
 *  H          device CSR, the H of the forward run.
 *  alpha_seq  host, n_alpha branches (+1 / -1), 0 <= n_alpha <= GSP2_MAX_ITER.
 *  dLdP_val   device, nnz_P floats in the order of gsp2_plan_pattern.
 *  dLdH_val   device, H.nnz doubles (out), caller-owned.
 *  info       nullable.
 * Allocates (ceil(n/k) + k + 1) arena-sized FP32 buffers for the pass
 * (k = ceil(sqrt(n_alpha))) and frees them before returning; waits for the result.
 * Errors: GSP2_E_INVALID (arguments, non-finite H), GSP2_E_OOM, GSP2_E_HIP,
 * GSP2_E_UNSUPPORTED (batched plans).
 */
gsp2_status gsp2_backward(gsp2_plan plan, const gsp2_csr *H, const int8_t *alpha_seq, int32_t n_alpha,
                          const float *dLdP_val, double *dLdH_val, gsp2_backward_info *info);

/* Wait for the last gsp2_density on this plan and report it (info: n_systems structs). */
gsp2_status gsp2_run_status(gsp2_plan plan, gsp2_run_info *info);

/* Release the plan and its device memory (waits for its stream).  NULL is a no-op. */
void gsp2_plan_destroy(gsp2_plan plan);

/* Graph G_tau of a plan (the threshold of P_prev), as the directed adjacency
 * the GPU built: row v lists the columns u != v with |P_prev[v,u]| > tau, in
 * stored order.  adj_ptr: host, n+1 int64; adj_col: host, nnz_graph int32,
 * nullable (pass NULL first to size it from adj_ptr[n]).  Errors: GSP2_E_INVALID. */
gsp2_status gsp2_plan_graph(gsp2_plan plan, int64_t *adj_ptr, int32_t *adj_col);

/* Matrix-core rate probe.  Runs back-to-back MFMAs of the product kernels'
 * shape and operand format (`precision`: FP32, FP16 or BF16 operands; split
 * FP16 runs FP16 MFMAs) on every CU, two waves per SIMD, for about 30 ms on
 * `stream` (nullable: the null stream), and returns the rate reached in
 * TFLOP/s: the measured counterpart of the published peak, at the clock the
 * GPU runs at.  Allocates and frees a small device buffer; waits for the
 * stream. */
gsp2_status gsp2_probe_mfma(int32_t precision, void *stream, double *tflops);

/* Result of gsp2_plan_tune. */
#define GSP2_TUNE_MAX 4
typedef struct {
    int32_t precision;         /* the gsp2_precision tuned */
    int32_t chosen;            /* the gsp2_kernel kept */
    int32_t n_candidates;      /* entries of candidate and ms */
    int32_t n_products;        /* products timed per candidate */
    int32_t candidate[GSP2_TUNE_MAX];   /* gsp2_kernel of each candidate, in the order timed */
    double ms[GSP2_TUNE_MAX];           /* mean product time of each candidate */
} gsp2_tune_info;

/* Autotuner of the product kernel (the paper's products are dense
 * matrix-matrix sub-problems, Methods, eq. (4); their tiling is this
 * library's choice).  Times n_products products of the plan's own
 * sub-problems, built from H, with each candidate form: FP32 and FP64
 * products GSP2_KERNEL_T128 and T128_SKIP; 16-bit products T128, T128_SKIP
 * and T256.
 * Keeps the form with the lowest mean product time for `precision`, except
 * that another form replaces the default (GSP2_KERNEL_AUTO's) only when it is
 * more than 1% faster, so that near ties keep the default; gsp2_density then uses it for that precision unless the run names a form
 * or (16-bit products) the plan was created with a fixed tile16.  The
 * products replay alternating branches (X^2, 2X - X^2, ...), so every
 * product carries the same work as in a run; the trace check of those runs
 * is not applied.  Runs on the plan's stream and waits for it.
 *
 *  H           device CSR as for gsp2_density.
 *  n_occ       as for gsp2_density (batched plans: ignored).
 *  precision   GSP2_PREC_FP32, GSP2_PREC_FP16, GSP2_PREC_BF16 or GSP2_PREC_FP16X3.
 *  n_products  2..GSP2_MAX_ITER products per candidate (after one untimed run).
 *  info        nullable; filled with the timings and the choice.
 * Returns GSP2_E_INVALID for FP64 (one form only) or a bad n_products; the
 * plan's previous choice is kept on any error.  The library allocates and
 * frees a P-sized scratch output of its own. */
gsp2_status gsp2_plan_tune(gsp2_plan plan, const gsp2_csr *H, double n_occ, int32_t precision,
                           int32_t n_products, gsp2_tune_info *info);

/* Options of gsp2_partition_anneal.  Zero-initialised means defaults. */
typedef struct {
    int32_t sweeps;            /* passes over all vertices; 0 = 40 */
    int32_t pad_;
    double t0;                 /* starting temperature in units of 3 (C / n_parts)^(2/3), the
                                  change of C when a part of mean cost grows by one vertex;
                                  0 = 2; negative = no uphill moves */
    double cooling;            /* temperature factor per sweep, in (0, 1]; 0 = 0.85 */
    uint64_t seed;             /* seed of the move generator */
    int32_t reserved[4];
} gsp2_anneal_options;

/*
 * Host-only (no GPU needed): refine a partition to lower the cost of eq. (4),
 * C = sum_k (c_k + h_k)^3, by simulated annealing, the alternative to METIS
 * that the paper's graph-theory section evaluates.  Single-vertex moves of
 * boundary vertices to a neighbouring part, the exact change of C from the
 * neighbour counts, Metropolis acceptance with a geometric temperature
 * schedule; no part is emptied (n_parts stays fixed).  The best partition
 * seen is written back.  Deterministic for a given seed.
 *  adj_ptr, adj_col  host CSR of the graph (the union of both orientations
 *                    is used; self loops are ignored), as gsp2_plan_graph gives.
 *  part              host, n int32 ids in [0, n_parts), every part non-empty;
 *                    in: the starting partition, out: the refined one.
 *  opt               nullable (defaults).
 *  cost_before, cost_after  nullable: C of the partition given and returned.
 * Errors: GSP2_E_INVALID.
 */
gsp2_status gsp2_partition_anneal(int32_t n, const int64_t *adj_ptr, const int32_t *adj_col, int32_t n_parts,
                                  int32_t *part, const gsp2_anneal_options *opt, int64_t *cost_before,
                                  int64_t *cost_after);

/*
 * Host-only (no GPU needed): the graph of the locality construction that the
 * paper's graph-theory section names as an alternative to thresholding an
 * earlier P: beyond a localization radius, elements of P are taken as zero.
 * Orbitals u != v are adjacent when their atoms lie closer than `radius`
 * (minimum image in a cubic periodic box of edge `box`; open boundaries
 * when box <= 0); orbitals of one atom are always adjacent.  The result
 * seeds a plan where no earlier P exists (pass it as P_prev with unit values
 * and any tau in [0, 1)), or feeds gsp2_partition_anneal.
 *  orbital_atom  host, n_orb int32 atom ids in [0, n_atoms).
 *  xyz           host, 3 n_atoms doubles (x, y, z of every atom).
 *  radius        > 0 (same length unit as xyz and box).
 *  adj_ptr       host, n_orb + 1 int64 (out).
 *  adj_col       host, adj_ptr[n_orb] int32 (out), nullable: pass NULL first
 *                to size it.  Every row lists its columns ascending; the
 *                graph is symmetric and has no self loops.
 * Errors: GSP2_E_INVALID.
 */
gsp2_status gsp2_locality_graph(int32_t n_orb, const int32_t *orbital_atom, int32_t n_atoms, const double *xyz,
                                double radius, double box, int64_t *adj_ptr, int32_t *adj_col);

/*
 * Host-only planning step (no GPU needed): core and one-hop halo of every
 * part of an undirected graph given by a directed adjacency (the union of
 * both orientations is used; self loops are ignored).
 *  adj_ptr, adj_col  host CSR of the adjacency, n+1 / adj_ptr[n] entries.
 *  part              host, n int32 ids in [0, n_parts).
 *  sub_ptr           host, n_parts+1 int64 (out): offsets into sub_idx.
 *  sub_idx           host, sub_ptr[n_parts] int32 (out), nullable: pass NULL
 *                    first to size it, then call again.
 *  core_count        host, n_parts int32 (out), nullable.
 * Errors: GSP2_E_INVALID.
 */
gsp2_status gsp2_core_halo_host(int32_t n, const int64_t *adj_ptr, const int32_t *adj_col,
                                const int32_t *part, int32_t n_parts, int64_t *sub_ptr,
                                int32_t *sub_idx, int32_t *core_count);

/* Outcome of gsp2_sparse_sp2_host. */
typedef struct {
    int32_t status;            /* GSP2_OK, GSP2_E_NOT_CONVERGED or GSP2_E_WRONG_TRACE */
    int32_t n_products;        /* products formed, including a discarded last one */
    int32_t n_alpha;           /* branches applied */
    int32_t pad_;
    double eps_min, eps_max;   /* Gershgorin bounds of H */
    double trace;              /* Tr P */
    double idempotency;        /* e_t = Tr[X_t] - Tr[X_t^2] of the returned iterate */
    int64_t nnz;               /* stored entries of P */
    int8_t alpha[GSP2_MAX_ITER];
} gsp2_sparse_sp2_info;

/* Host-only (no GPU needed): the very first density matrix, by SP2 of the
 * whole H in numerically thresholded sparse algebra, the standard scheme
 * that provides P before any graph or partition exists (Fig. 1 description
 * in the Introduction; the threshold is the same kind of parameter as the
 * graph's tau, Methods, "Graph Theory").  The steps are those of a dense
 * run: Gershgorin bounds, eq. (1), then per product the stop rule (stop at
 * the first product t >= 2 whose idempotency measure |e_t| has stopped
 * falling below |e_{t-2}| < 1; the product just formed is discarded), the
 * trace rule for the branch and eq. (2); every iterate keeps only its
 * entries with |x| > eps (eps = 0 keeps every nonzero).  Sparse products on
 * the host threads; the result does not depend on their number.
 *
 *  n, H_row_ptr, H_col, H_val  host CSR of H (symmetric, FP64), both triangles stored.
 *  n_occ       occupied states, 0 <= n_occ <= n.
 *  eps         threshold, >= 0.
 *  max_iter    product budget, 1..GSP2_MAX_ITER.
 *  P_row_ptr   host, n+1: filled with P's row pointer.
 *  P_col, P_val host, P_row_ptr[n] entries each, or both NULL: only
 *              P_row_ptr and info are filled (size query; a second call with
 *              the arrays recomputes the same P).
 *  info        nullable.
 * Returns GSP2_E_INVALID for bad arguments or a flat spectrum bound; else the
 * run's status (P is filled in every case). */
gsp2_status gsp2_sparse_sp2_host(int32_t n, const int64_t *H_row_ptr, const int32_t *H_col, const double *H_val,
                                 double n_occ, double eps, int32_t max_iter, int64_t *P_row_ptr, int32_t *P_col,
                                 double *P_val, gsp2_sparse_sp2_info *info);

#ifdef __cplusplus
}
#endif

#endif /* GSP2_H */
