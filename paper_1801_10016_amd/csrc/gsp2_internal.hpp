// Layouts shared by the host planner, the ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "gsp2.h"

namespace gsp2 {

// Macro tile of the SP2 product (rows x columns of Y computed by one
// workgroup) and the K depth staged through LDS per pipeline step.
constexpr int kTile = 128;
constexpr int kKChunk = 32;
constexpr int kTileWide = 256;      // product tile of 16-bit operands
// 16-bit products address a part's operand matrix as one buffer of under
// 4 GiB: s_pad^2 * 2 bytes < 2^32
constexpr int kMaxWidePad = 46336;
// rows per gather chunk (one workgroup each); also the row block of the
// fixup after 16-bit products.  Divides 128, so chunks never straddle s_pad.
constexpr int kRowsPerChunk = 16;

// XCDs of an MI355X: workgroup b of a launch runs on XCD b mod kXcds.
constexpr int kXcds = 8;

// Row kernels (threshold, Gershgorin, scatter) give one wave to a row in
// 256-thread workgroups: rows per workgroup.
constexpr int kRowsPerBlock = 4;

// One part of the partition, as the device sees it.
struct PartDesc {
    int64_t x_off;      // float offset of the part's s_pad x s_pad block in each X buffer
    int32_t idx_off;    // offset of its vertex list (local order) in the index arena
    int32_t s;          // sub-problem size c + h
    int32_t c;          // core size
    int32_t s_pad;      // s rounded up to a multiple of kTile (padding is zero)
    int32_t perm_off;   // offset of its sorted-position -> local-index map
    int32_t sys;        // system of the part (0 unless the plan is batched)
};
static_assert(sizeof(PartDesc) == 32, "PartDesc layout");

// One upper-triangle macro tile (ti <= tj) of one part's product; part < 0
// marks an empty tile that pads the launch.
struct TileDesc {
    int32_t part, ti, tj, diag_slot;   // diag_slot >= 0 only when ti == tj
};

// A run of consecutive local rows of one part, built by one gather workgroup.
struct RowChunk {
    int32_t part, r0, r1, pad_;
};

// Run-time state of one system's density-matrix computation, in device
// memory (one per system of the plan).  Written only by the control kernels,
// one workgroup per system.
struct RunState {
    double n_occ;
    double trace_tol;
    double eps_min, eps_max;
    double trX;                 // Tr[X_t] of the current iterate
    double idem;                // e_t of the returned iterate
    double stop_floor;
    int32_t n_steps;            // product budget (trace mode) or replay length
    int32_t mode;               // gsp2_alpha_mode
    int32_t stop_rule;
    int32_t t;                  // products formed and kept so far (= index of X_t)
    int32_t cur;                // buffer holding X_t
    int32_t alpha;              // branch for the next product
    int32_t done;
    int32_t status;             // gsp2_status
    int32_t result_buf;
    int32_t result_t;
    int32_t n_products;
    int32_t phase;              // 0: main products, 1: FP32 refinement products
    int32_t refine;             // refinement products requested
    int32_t refine_left;
    int32_t n_refine;           // refinement products formed
    int32_t main_status;        // status of the main phase, reported at the end
    int32_t n_main;             // products formed in the main phase
    int32_t precision;
    int32_t row_min, row_max;   // rows attaining eps_min and eps_max (lowest index on ties)
    int8_t alpha_seq[GSP2_MAX_ITER];
    int8_t alpha_hist[GSP2_MAX_ITER];
    double traces[GSP2_MAX_ITER + 1];
    double errors[GSP2_MAX_ITER];
};

// Control words of the persistent product kernel (cleared before each launch).
struct PersistCtl {
    unsigned arrive;                    // grid-barrier arrivals, monotonic within a launch
    unsigned fail;                      // set when a bounded wait expires
    unsigned pad_[2];
    unsigned head[GSP2_MAX_ITER][kXcds];  // per product, per XCD tile-queue head
};

// Per-call parameters baked into the run's kernels (the same for every system).
struct RunParams {
    double trace_tol;
    int32_t n_steps;            // main-phase product launches: the largest budget of any system
    int32_t mode;
    int32_t stop_rule;
    int32_t precision;          // gsp2_precision of the main phase
    int32_t refine;             // FP32 products after the main phase
    int32_t persistent;         // 1: main-phase products in one persistent launch
    int32_t kernel;             // gsp2_kernel of the main-phase products (resolved, never AUTO)
    int32_t kernel32;           // gsp2_kernel of the refinement products (T128 or T128_SKIP)
    int32_t symmetrize;         // scatter the mean of mirrored stored pairs
    int32_t refine_prec;        // gsp2_precision of the refinement products (FP32, FP16X3 or FP64)
};
static_assert(sizeof(RunParams) == 48, "RunParams layout (no implicit padding: graph keys compare bytes)");

// Per-call parameters of one system, uploaded to the device before each run.
struct SysParams {
    double n_occ;
    double stop_floor;          // max(1, n u): |e_{t-2}| must be below it for the stop rule
    int32_t n_steps;            // main-phase product budget of this system
    int32_t pad_;
    int8_t alpha_seq[GSP2_MAX_ITER];
    int8_t pad2_[4];
};
static_assert(sizeof(SysParams) % 8 == 0, "SysParams layout");

// Device buffers of a plan, passed to the launchers.
struct DevicePlan {
    int32_t n;
    int32_t n_parts;
    int32_t n_tiles;
    int32_t n_diag;
    int32_t n_chunks;
    int32_t max_s_pad;
    int32_t gersh_blocks;       // row blocks of the Gershgorin kernel
    int32_t n_sys;              // systems (1 unless batched)
    float *buf[2];
    double *buf64[2];           // FP64 iterates (FP64 products), allocated on the first FP64 run
    void *shadow[2];            // 16-bit operand copies of the two X buffers (mixed precision)
    void *shadow_lo[2];         // scaled FP16 low parts of the two X buffers (split FP16 products)
    const PartDesc *parts;
    const TileDesc *tiles;
    const TileDesc *tiles_s;    // the same tiles, each XCD's short ones last (the skip form's order)
    const TileDesc *tiles_w;    // 256 x 256 tiles of the 16-bit products (same layout rules)
    int32_t n_tiles_w;
    int32_t pad_w_;
    const RowChunk *chunks;
    const int32_t *idx;         // index arena (local order)
    const int32_t *perm;        // per part: sorted position -> local index
    const int32_t *invperm;     // per part: local index -> sorted position
    const int64_t *col_ptr;     // CSC column pointers of P, n+1
    const int32_t *col_part;    // part of every column
    const int32_t *col_local;   // local index of every column in its part
    int32_t list_len;           // entries per XCD list (n_tiles / kXcds)
    int32_t persist_grid;       // workgroups of the persistent launch
    long long persist_timeout;  // wall-clock ticks a persistent wait may last
    PersistCtl *persist;
    double *diag_partials;      // 2 x n_diag x 2 (double-buffered by product parity)
    double *x0_partials;        // n_chunks
    double *row_bounds;         // n x 3: Gershgorin lower and upper end, non-finite flag of every row
    const int32_t *sys_rows;    // vertices of every system, ascending, grouped by system
    const int32_t *sys_row_ptr; // n_sys + 1 offsets into sys_rows
    const int32_t *sys_chunk_ptr;   // n_sys + 1: gather chunks are grouped by system
    const int32_t *sys_diag_ptr;    // n_sys + 1: diagonal-tile slots are grouped by system
    SysParams *sys_params;      // n_sys
    RunState *state;            // n_sys
};

// Optional event records of a timed run.  step[2t] / step[2t+1] bracket the
// product kernel of product t.
struct RunEvents {
    hipEvent_t begin, setup_end, sp2_end, end, persist_begin, persist_end;
    hipEvent_t step[2 * GSP2_MAX_ITER];
};

// Sink for the kernels and event records of one run: launched directly on a
// stream (graph == nullptr), or appended as a linear chain of nodes to a HIP
// graph built explicitly (event-record nodes keep their timestamps there).
struct Recorder {
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphNode_t last = nullptr;
    hipError_t err = hipSuccess;

    void add_kernel(const void *func, dim3 grid, dim3 block, void **args) {
        if (err != hipSuccess) return;
        if (!graph) {
            err = hipLaunchKernel(func, grid, block, args, 0, stream);
            return;
        }
        hipKernelNodeParams p{};
        p.func = const_cast<void *>(func);
        p.gridDim = grid;
        p.blockDim = block;
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        hipGraphNode_t node = nullptr;
        err = hipGraphAddKernelNode(&node, graph, last ? &last : nullptr, last ? 1 : 0, &p);
        if (err == hipSuccess) last = node;
    }
    void add_event(hipEvent_t e) {
        if (err != hipSuccess || !e) return;
        if (!graph) {
            err = hipEventRecord(e, stream);
            return;
        }
        hipGraphNode_t node = nullptr;
        err = hipGraphAddEventRecordNode(&node, graph, last ? &last : nullptr, last ? 1 : 0, e);
        if (err == hipSuccess) last = node;
    }
};

// Work buffers of one backward pass (all arena-sized FP32 except where noted).
struct BackwardBuffers {
    int seg;                    // products per checkpoint segment
    float *ckpt[GSP2_MAX_ITER + 1];   // X_{seg * k}
    float *slot[GSP2_MAX_ITER];       // iterates recomputed inside one segment
    float *g[2];                // cotangent ping-pong
    double *eps_partials;       // n_chunks x 2
    double *d_eps;              // 2: dL/d eps_min, dL/d eps_max
};

// Launchers (kernels.hip).  The threshold launchers enqueue on `stream`.
hipError_t launch_threshold_count(const gsp2_csr &P, double tau, int32_t *counts, hipStream_t s);
hipError_t launch_threshold_fill(const gsp2_csr &P, double tau, const int64_t *out_ptr,
                                 int32_t *out_col, hipStream_t s);
hipError_t launch_density(const DevicePlan &dp, const gsp2_csr &H, const RunParams &rp,
                          void *P_val, Recorder &rec, const RunEvents *ev);
// Reverse pass for a known branch sequence: dL/dH on H's stored entries.
hipError_t launch_backward(const DevicePlan &dp, const gsp2_csr &H, const RunParams &rp, const int8_t *alphas,
                           int n, const float *dLdP, double *dLdH, const BackwardBuffers &bb, hipStream_t s);
// Matrix-core rate probe: n_blocks workgroups of kProbeThreads threads of
// back-to-back MFMAs; *flops receives the matrix-core flops the launch performs.
constexpr int kProbeThreads = 256;
hipError_t probe_mfma(int precision, int n_iter, int n_blocks, float *out, hipStream_t s, int64_t *flops);
// Workgroups of the persistent product kernel that the device keeps resident.
hipError_t persistent_grid(int precision, int *grid);

// Static device scratch of gsp2_density_noalloc (kernels.hip): its size, and
// its address on the current device (looked up once per device).
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
hipError_t static_scratch(void **ptr);

// Simulated-annealing refinement of a partition for eq. (4) (partition.cpp).
struct AnnealResult {
    int64_t cost_before, cost_after;
    int64_t moves;
};
AnnealResult anneal_partition(int32_t n, const int64_t *adj_ptr, const int32_t *adj_col, int32_t n_parts,
                              int32_t *part, int32_t sweeps, double t0, double cooling, uint64_t seed);

// SP2 of the whole matrix in thresholded sparse algebra, on the host
// (sparse_sp2.cpp).
struct SparseSP2Result {
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> val;
    std::vector<int8_t> alphas;
    int32_t status = 0, n_products = 0;
    double eps_min = 0.0, eps_max = 0.0, trace = 0.0, idempotency = 0.0;
};
SparseSP2Result sparse_sp2(int32_t n, const int64_t *rp, const int32_t *ci, const double *hv, double n_occ,
                           double eps, int32_t max_iter, double trace_tol, int n_threads);

// Graph of the locality construction: orbitals adjacent when their atoms are
// closer than `radius` (partition.cpp).
void locality_graph(int32_t n_orb, const int32_t *orbital_atom, int32_t n_atoms, const double *xyz, double radius,
                    double box, std::vector<int64_t> &adj_ptr, std::vector<int32_t> &adj_col);

}  // namespace gsp2
