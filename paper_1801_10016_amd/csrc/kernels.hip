// HIP kernels of the G-SP2 hot path for CDNA4 (gfx950), wave64.
//
//  threshold   G_tau from a previous P                (Methods, "Graph Theory")
//  gershgorin  spectral bounds of each system's H      (Methods, SP2: Gershgorin discs)
//  gather_x0   dense core+halo blocks of eq. (1)       (Fig. 1 description: sub-matrices of H)
//  sp2_step    X^2 on the matrix cores + eq. (2) update + core-trace partials
//  control     FP64 trace reductions, branch and stop decisions (eq. (2) branch rule, idempotency)
//  scatter     core columns into the sparse P          (Fig. 1 description: reassembly)
#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>
#include <tuple>
#include <utility>

#include "gsp2_internal.hpp"

namespace gsp2 {

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
static_assert(kBlock / kWave == kRowsPerBlock, "row kernels: one wave per row");

template <typename T>
__device__ __forceinline__ double as_double(T v) { return static_cast<double>(v); }

// Deterministic wave sum (fixed butterfly).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Deterministic block sum of two doubles; result valid in thread 0.
__device__ __forceinline__ void block_sum2(double &a, double &b) {
    __shared__ double red[2][kBlock / kWave];
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) { red[0][w] = a; red[1][w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = 0.0; b = 0.0;
        for (int i = 0; i < kBlock / kWave; ++i) { a += red[0][i]; b += red[1][i]; }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// a1: threshold.  One wave per row; entries kept in their stored order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_threshold_count(const int64_t *__restrict__ row_ptr,
                                                            const int32_t *__restrict__ col,
                                                            const T *__restrict__ val, int32_t n,
                                                            double tau, int32_t *__restrict__ counts) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t row = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (row >= n) return;
    const int64_t b = row_ptr[row], e = row_ptr[row + 1];
    int cnt = 0;
    for (int64_t i = b + lane; i < e; i += kWave)
        cnt += (col[i] != row && fabs(as_double(val[i])) > tau) ? 1 : 0;
    cnt = wave_sum_int(cnt);
    if (lane == 0) counts[row] = cnt;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_threshold_fill(const int64_t *__restrict__ row_ptr,
                                                           const int32_t *__restrict__ col,
                                                           const T *__restrict__ val, int32_t n,
                                                           double tau, const int64_t *__restrict__ out_ptr,
                                                           int32_t *__restrict__ out_col) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t row = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (row >= n) return;
    const int64_t b = row_ptr[row], e = row_ptr[row + 1];
    int64_t o = out_ptr[row];
    const int64_t o_end = out_ptr[row + 1];
    for (int64_t base = b; base < e; base += kWave) {
        const int64_t i = base + lane;
        const bool keep = i < e && col[i] != row && fabs(as_double(val[i])) > tau;
        const uint64_t m = __ballot(keep);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (keep && o + before < o_end) out_col[o + before] = col[i];
        o += __popcll(m);
    }
}

// ---------------------------------------------------------------------------
// a4: Gershgorin bounds.  One wave per row, FP64: the lower and upper end of
// the row's disc and a non-finite flag.  A system's bounds are the extremes
// over its rows, taken with the lowest row winning ties, so the rows that
// attain them (and the bounds' derivatives) are well defined.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void keep_lo(double &lo, double &row, double l2, double r2) {
    if (l2 < lo || (l2 == lo && r2 < row)) { lo = l2; row = r2; }
}
__device__ __forceinline__ void keep_hi(double &hi, double &row, double h2, double r2) {
    if (h2 > hi || (h2 == hi && r2 < row)) { hi = h2; row = r2; }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gershgorin(const int64_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ col,
                                                       const T *__restrict__ val, int32_t n,
                                                       double *__restrict__ row_bounds) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t row = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (row >= n) return;                       // whole waves leave together
    const int64_t b = row_ptr[row], e = row_ptr[row + 1];
    double rad = 0.0, d = 0.0, nf = 0.0;
    for (int64_t i = b + lane; i < e; i += kWave) {
        const double v = as_double(val[i]);
        if (!isfinite(v)) nf = 1.0;
        if (col[i] == row) d += v; else rad += fabs(v);
    }
    rad = wave_sum(rad);
    d = wave_sum(d);
    nf = wave_sum(nf);
    if (lane == 0) {
        double *out = row_bounds + 3 * row;
        out[0] = d - rad;
        out[1] = d + rad;
        out[2] = nf;
    }
}

// Reduce the discs of every system's rows and initialise its run state.
// One workgroup per system.
__global__ __launch_bounds__(kBlock) void k_run_init(const double *__restrict__ row_bounds,
                                                     const int32_t *__restrict__ sys_rows,
                                                     const int32_t *__restrict__ sys_row_ptr, RunParams rp,
                                                     const SysParams *__restrict__ sys_params,
                                                     RunState *__restrict__ st_all) {
    __shared__ double s_lo[kBlock], s_hi[kBlock], s_bad[kBlock], s_rlo[kBlock], s_rhi[kBlock];
    const int sys = blockIdx.x;
    double lo = INFINITY, hi = -INFINITY, bad = 0.0, rlo = 1e300, rhi = 1e300;
    for (int i = sys_row_ptr[sys] + threadIdx.x; i < sys_row_ptr[sys + 1]; i += kBlock) {
        const int32_t r = sys_rows[i];
        const double *rb = row_bounds + 3 * (int64_t)r;
        keep_lo(lo, rlo, rb[0], (double)r);
        keep_hi(hi, rhi, rb[1], (double)r);
        bad = fmax(bad, rb[2]);
    }
    s_lo[threadIdx.x] = lo; s_hi[threadIdx.x] = hi; s_bad[threadIdx.x] = bad;
    s_rlo[threadIdx.x] = rlo; s_rhi[threadIdx.x] = rhi;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int i = 1; i < kBlock; ++i) {
        keep_lo(lo, rlo, s_lo[i], s_rlo[i]);
        keep_hi(hi, rhi, s_hi[i], s_rhi[i]);
        bad = fmax(bad, s_bad[i]);
    }
    RunState *st = st_all + sys;
    const SysParams &sp = sys_params[sys];
    st->row_min = rlo < 1e300 ? (int)rlo : -1;
    st->row_max = rhi < 1e300 ? (int)rhi : -1;
    st->n_occ = sp.n_occ;
    st->trace_tol = rp.trace_tol;
    st->stop_floor = sp.stop_floor;
    st->eps_min = lo;
    st->eps_max = hi;
    st->trX = 0.0;
    st->idem = NAN;
    st->n_steps = sp.n_steps;
    st->mode = rp.mode;
    st->stop_rule = rp.stop_rule;
    st->t = 0;
    st->cur = 0;
    st->alpha = 0;
    st->result_buf = 0;
    st->result_t = 0;
    st->n_products = 0;
    st->phase = 0;
    st->refine = rp.refine;
    st->refine_left = 0;
    st->n_refine = 0;
    st->main_status = GSP2_OK;
    st->n_main = 0;
    st->precision = rp.precision;
    for (int i = 0; i < GSP2_MAX_ITER; ++i) {
        st->alpha_seq[i] = sp.alpha_seq[i];
        st->alpha_hist[i] = 0;
        st->errors[i] = NAN;
        st->traces[i] = NAN;
    }
    st->traces[GSP2_MAX_ITER] = NAN;
    const bool ok = bad == 0.0 && isfinite(lo) && isfinite(hi) && hi > lo;
    st->status = ok ? GSP2_OK : GSP2_E_INVALID;
    st->done = ok ? 0 : 1;
}

// ---------------------------------------------------------------------------
// a5: gather + X0 (eq. (1)).  One workgroup per chunk of rows of one part,
// each wave building one row at a time in its own LDS segment, so that the
// four waves work on four rows without workgroup barriers; every row of the
// padded block (s_pad wide) is written exactly once, as whole coalesced
// rows.
// ---------------------------------------------------------------------------
constexpr int kGatherLdsIdx = 8192;    // vertex list held in LDS up to this size
constexpr int kGatherChunkBytes = 8192;  // row segment built in LDS per wave and pass (2,048 FP32 or 1,024 FP64)

// Orders a wave's LDS accesses: writes by any lane before the call are seen
// by reads of any lane after it.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int find_sorted(const int32_t *a, int n, int32_t key) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (lo < n && a[lo] == key) ? lo : -1;
}

// Four floats rounded to the 16-bit operand format (round to nearest even).
__device__ __forceinline__ uint2 pack4_fp16(float4 v) {
    union { _Float16 h[4]; uint2 u; } x;
    x.h[0] = (_Float16)v.x; x.h[1] = (_Float16)v.y; x.h[2] = (_Float16)v.z; x.h[3] = (_Float16)v.w;
    return x.u;
}
__device__ __forceinline__ uint2 pack4_bf16(float4 v) {
    union { __bf16 h[4]; uint2 u; } x;
    x.h[0] = (__bf16)v.x; x.h[1] = (__bf16)v.y; x.h[2] = (__bf16)v.z; x.h[3] = (__bf16)v.w;
    return x.u;
}
__device__ __forceinline__ uint2 pack4(float4 v, int precision) {
    return precision == GSP2_PREC_BF16 ? pack4_bf16(v) : pack4_fp16(v);
}
// Low parts of split FP16 operands: L = fp16(2^11 (x - fp16(x))), so that
// x = fp16(x) + 2^-11 L to about 2^-22 relative (the scaling keeps L normal).
__device__ __forceinline__ uint2 pack4_fp16_lo(float4 v) {
    union { _Float16 h[4]; uint2 u; } x;
    x.h[0] = (_Float16)((v.x - (float)(_Float16)v.x) * 0x1p11f);
    x.h[1] = (_Float16)((v.y - (float)(_Float16)v.y) * 0x1p11f);
    x.h[2] = (_Float16)((v.z - (float)(_Float16)v.z) * 0x1p11f);
    x.h[3] = (_Float16)((v.w - (float)(_Float16)v.w) * 0x1p11f);
    return x.u;
}

template <typename T, typename XT>
__global__ __launch_bounds__(kBlock) void k_gather_x0(const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col,
                                                      const T *__restrict__ val,
                                                      const PartDesc *__restrict__ parts,
                                                      const RowChunk *__restrict__ chunks,
                                                      const int32_t *__restrict__ idx_arena,
                                                      XT *__restrict__ X, uint16_t *__restrict__ Xs,
                                                      uint16_t *__restrict__ Xlo,
                                                      const RunState *__restrict__ st_all,
                                                      double *__restrict__ x0_partials) {
    constexpr int kChunk = kGatherChunkBytes / static_cast<int>(sizeof(XT));   // a multiple of 128
    __shared__ int32_t idx_s[kGatherLdsIdx];
    __shared__ uint4 row_u4[kBlock / kWave][kGatherChunkBytes / 16];
    __shared__ double tr_s[kBlock / kWave];
    const RowChunk ch = chunks[blockIdx.x];
    const PartDesc pd = parts[ch.part];
    const RunState *st = st_all + pd.sys;
    if (st->done) return;
    const int32_t *idx_g = idx_arena + pd.idx_off;
    const bool in_lds = pd.s <= kGatherLdsIdx;
    if (in_lds) {
        for (int i = threadIdx.x; i < pd.s; i += kBlock) idx_s[i] = idx_g[i];
        __syncthreads();
    }
    const int32_t *idx = in_lds ? idx_s : idx_g;
    const double emin = st->eps_min, emax = st->eps_max;
    const double inv = 1.0 / (emax - emin);
    const int ld = pd.s_pad;
    XT *Xp = X + pd.x_off;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint4 *row_u = row_u4[wave];
    XT *row_s = reinterpret_cast<XT *>(row_u);
    const int prec = st->precision;
    double tr = 0.0;
    for (int r = ch.r0 + wave; r < ch.r1; r += kBlock / kWave) {
        const bool real = r < pd.s;
        const int64_t g = real ? idx[r] : -1;
        const int64_t hb = real ? row_ptr[g] : 0, he = real ? row_ptr[g + 1] : 0;
        for (int c0 = 0; c0 < ld; c0 += kChunk) {
            const int cw = min(kChunk, ld - c0);         // a multiple of 128
            const int n16 = cw * static_cast<int>(sizeof(XT)) / 16;
            for (int i = lane; i < n16; i += kWave) row_u[i] = make_uint4(0u, 0u, 0u, 0u);
            wave_lds_sync();
            if (real && lane == 0 && r >= c0 && r < c0 + cw)
                row_s[r - c0] = static_cast<XT>(emax * inv);          // H_gg = 0 if not stored
            wave_lds_sync();
            for (int64_t e = hb + lane; e < he; e += kWave) {
                const int32_t cg = col[e];
                int q = find_sorted(idx, pd.c, cg);
                if (q < 0) {
                    q = find_sorted(idx + pd.c, pd.s - pd.c, cg);
                    if (q >= 0) q += pd.c;
                }
                if (q >= c0 && q < c0 + cw) {
                    const double h = as_double(val[e]);
                    const double x = (cg == g) ? (emax - h) * inv : -h * inv;
                    row_s[q - c0] = static_cast<XT>(x);
                }
            }
            wave_lds_sync();
            if (real && r < pd.c && lane == 0 && r >= c0 && r < c0 + cw)
                tr += static_cast<double>(row_s[r - c0]);
            uint4 *dst = reinterpret_cast<uint4 *>(Xp + (int64_t)r * ld + c0);
            if constexpr (sizeof(XT) == 4) {
                uint2 *dsh = Xs ? reinterpret_cast<uint2 *>(Xs + pd.x_off + (int64_t)r * ld + c0) : nullptr;
                uint2 *dlo = Xlo ? reinterpret_cast<uint2 *>(Xlo + pd.x_off + (int64_t)r * ld + c0) : nullptr;
                // plain 16-bit copies hold X without its diagonal: the products
                // take the diagonal terms exactly in FP32 (sp2_tile_wide)
                const int dq = (r >= c0 && r < c0 + cw && prec != GSP2_PREC_FP16X3) ? r - c0 : -1;
                for (int i = lane; i < n16; i += kWave) {
                    const uint4 u = row_u[i];
                    dst[i] = u;
                    const float4 v = __builtin_bit_cast(float4, u);
                    if (dsh) {
                        float4 w = v;
                        if ((dq >> 2) == i) {
                            if ((dq & 3) == 0) w.x = 0.0f;
                            else if ((dq & 3) == 1) w.y = 0.0f;
                            else if ((dq & 3) == 2) w.z = 0.0f;
                            else w.w = 0.0f;
                        }
                        dsh[i] = pack4(w, prec);
                    }
                    if (dlo) dlo[i] = pack4_fp16_lo(v);
                }
            } else {
                for (int i = lane; i < n16; i += kWave) dst[i] = row_u[i];
            }
            wave_lds_sync();                             // reads done before the next zeroing
        }
    }
    // one partial per workgroup, the waves' sums added in a fixed order
    if (lane == 0) tr_s[wave] = tr;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) t += tr_s[w];
        x0_partials[blockIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
// a7: control state of a run.  The branch and stop decisions are a pure
// function of this state and the two trace sums of a product, so every
// workgroup of the persistent kernel takes them identically; between
// per-product launches the state lives in RunState.
// ---------------------------------------------------------------------------
struct Ctl {
    double n_occ, trace_tol, stop_floor, trX, idem, e1, e2;   // e1 = e_{t-1}, e2 = e_{t-2}
    int n_steps, mode, stop_rule, t, cur, alpha, done, status, result_buf, result_t, n_products;
    int phase, refine, refine_left, n_refine, main_status, n_main;
};

__device__ Ctl ctl_load(const RunState *st) {
    Ctl c;
    c.n_occ = st->n_occ; c.trace_tol = st->trace_tol; c.stop_floor = st->stop_floor;
    c.trX = st->trX; c.idem = st->idem;
    c.n_steps = st->n_steps; c.mode = st->mode; c.stop_rule = st->stop_rule; c.t = st->t; c.cur = st->cur;
    c.alpha = st->alpha; c.done = st->done; c.status = st->status; c.result_buf = st->result_buf;
    c.result_t = st->result_t; c.n_products = st->n_products; c.phase = st->phase; c.refine = st->refine;
    c.refine_left = st->refine_left; c.n_refine = st->n_refine; c.main_status = st->main_status;
    c.n_main = st->n_main;
    c.e1 = c.t >= 1 ? st->errors[c.t - 1] : NAN;
    c.e2 = c.t >= 2 ? st->errors[c.t - 2] : NAN;
    return c;
}

__device__ void ctl_store(RunState *st, const Ctl &c) {
    st->trX = c.trX; st->idem = c.idem; st->t = c.t; st->cur = c.cur; st->alpha = c.alpha; st->done = c.done;
    st->status = c.status; st->result_buf = c.result_buf; st->result_t = c.result_t;
    st->n_products = c.n_products; st->phase = c.phase; st->refine_left = c.refine_left;
    st->n_refine = c.n_refine; st->main_status = c.main_status; st->n_main = c.n_main;
}

// Status of a finished run: a trace-mode run whose result misses the
// occupation by more than trace_tol has failed (a wrong final trace marks a
// failed SP2 run, Methods, SP2 section); replay runs check it at the end of
// the replayed branches.
__device__ __forceinline__ int occupation_status(const Ctl &c, int status, double trace) {
    if (status == GSP2_OK && c.mode == GSP2_ALPHA_TRACE && !(fabs(trace - c.n_occ) <= c.trace_tol))
        return GSP2_E_WRONG_TRACE;
    return status;
}

// End of the main phase: hand over to the refinement products, or stop.
// Refinement alternates X^2 and 2X - X^2 whatever the trace: one pair maps
// an eigenvalue l to 2 l^2 - l^4, whose stable fixed points are 0 and 1
// (split at (sqrt(5) - 1) / 2), so every pair drives each eigenvalue to the
// nearer of the two, quadratically.  The trace rule would keep picking the
// branch that moves the trace towards n_occ; once the occupation is settled
// that doubles the distance of eigenvalues near 0 (or near 1) at each product.
// `trace` is Tr of the iterate the main phase ends on.
__device__ void finish_main(Ctl &c, int result_buf, int result_t, int status, bool refinable, double trace) {
    c.n_main = c.n_products;
    if (refinable && c.refine > 0) {
        c.phase = 1;
        c.main_status = status;
        c.cur = result_buf;
        c.t = result_t;
        c.refine_left = c.refine;
        c.alpha = -1;
        return;
    }
    c.done = 1;
    c.result_buf = result_buf;
    c.result_t = result_t;
    c.status = occupation_status(c, status, trace);
}

// One product's decision from Tr[X_t^2] (ty) and Tr[X_{t+1}] (tx): the
// stop rule, the branch of the next product, the end of a phase.  History
// arrays are written only when `writer`.
__device__ void decide(Ctl &c, double ty, double tx, RunState *st, bool writer) {
    const int t = c.t;
    const double e = c.trX - ty;                // e_t = Tr[X_t] - Tr[X_t^2]
    if (writer) st->errors[t] = e;
    c.n_products += 1;
    if (!isfinite(ty) || !isfinite(tx)) {       // left the finite range: keep X_t
        if (c.phase == 0) c.n_main = c.n_products;
        c.done = 1;
        c.result_buf = c.cur;
        c.result_t = t;
        c.status = GSP2_E_NOT_CONVERGED;
        return;
    }
    // the bound applies to |e|: in finite precision e turns negative once X_t is idempotent to rounding
    if (c.phase == 0 && c.mode == GSP2_ALPHA_TRACE && c.stop_rule && t >= 2 && fabs(e) >= fabs(c.e2) &&
        fabs(c.e2) < c.stop_floor) {
        c.idem = e;                             // X_t is the result; X_t^2 is discarded
        finish_main(c, c.cur, t, GSP2_OK, true, c.trX);
        return;
    }
    if (writer) {
        st->alpha_hist[t] = (int8_t)c.alpha;
        st->traces[t + 1] = tx;
    }
    c.cur ^= 1;
    c.trX = tx;
    c.t = t + 1;
    c.e2 = c.e1;
    c.e1 = e;
    if (c.phase == 1) {
        c.n_refine += 1;
        c.idem = e;
        if (--c.refine_left == 0) {
            c.done = 1;
            c.result_buf = c.cur;
            c.result_t = t + 1;
            c.status = occupation_status(c, c.main_status, tx);
            return;
        }
        c.alpha = -c.alpha;
        return;
    }
    if (c.n_products >= c.n_steps) {
        // trace mode: the stop rule did not fire within the budget (or was
        // switched off), so the run has not shown convergence
        const int status = c.mode == GSP2_ALPHA_REPLAY
                               ? (fabs(tx - c.n_occ) <= c.trace_tol ? GSP2_OK : GSP2_E_WRONG_TRACE)
                               : GSP2_E_NOT_CONVERGED;
        finish_main(c, c.cur, t + 1, status, true, tx);
        return;
    }
    c.alpha = (c.mode == GSP2_ALPHA_REPLAY) ? (int)st->alpha_seq[t + 1] : (tx <= c.n_occ ? 1 : -1);
}

// Reduce the X0 core-trace partials of every system (one workgroup each,
// over the system's run of gather chunks); pick the first branch.
__global__ __launch_bounds__(kBlock) void k_run_start(const double *__restrict__ x0_partials,
                                                      const int32_t *__restrict__ sys_chunk_ptr,
                                                      RunState *__restrict__ st_all) {
    RunState *st = st_all + blockIdx.x;
    if (st->done) return;
    const int c0 = sys_chunk_ptr[blockIdx.x], c1 = sys_chunk_ptr[blockIdx.x + 1];
    double a = 0.0, b = 0.0;
    for (int i = c0 + threadIdx.x; i < c1; i += kBlock) a += x0_partials[i];
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        Ctl c = ctl_load(st);
        c.trX = a;
        st->traces[0] = a;
        if (c.n_steps <= 0) {
            const int status = (c.mode == GSP2_ALPHA_REPLAY && fabs(a - c.n_occ) > c.trace_tol)
                                   ? GSP2_E_WRONG_TRACE : GSP2_OK;
            finish_main(c, 0, 0, status, true, a);
        } else {
            c.alpha = (c.mode == GSP2_ALPHA_REPLAY) ? (int)st->alpha_seq[0] : (a <= c.n_occ ? 1 : -1);
        }
        ctl_store(st, c);
    }
}

typedef float v16f __attribute__((ext_vector_type(16)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Operand formats of the product.  Every format moves 128-byte row segments
// per K chunk (32 FP32 or 64 FP16/BF16 values), staged in LDS rows of 144 bytes.
template <typename Op> struct OpFmt;
template <> struct OpFmt<float> { static constexpr int kK = 32; };
template <> struct OpFmt<_Float16> { static constexpr int kK = 64; };
template <> struct OpFmt<__bf16> { static constexpr int kK = 64; };
constexpr int kLdsRow = 9;                  // uint4 per LDS row: 8 data + 1 pad

__device__ __forceinline__ v16f mfma_chunk_q(const uint4 &a, const uint4 &b, v16f c, float) {
    // four 32x32x2 FP32 steps; lane half h holds k = 16h + 4q + e for e = 0..3
    const float4 fa = *reinterpret_cast<const float4 *>(&a);
    const float4 fb = *reinterpret_cast<const float4 *>(&b);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(fa.x, fb.x, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(fa.y, fb.y, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(fa.z, fb.z, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(fa.w, fb.w, c, 0, 0, 0);
    return c;
}
__device__ __forceinline__ v16f mfma_chunk_q(const uint4 &a, const uint4 &b, v16f c, _Float16) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(*reinterpret_cast<const v8h *>(&a),
                                                  *reinterpret_cast<const v8h *>(&b), c, 0, 0, 0);
}
__device__ __forceinline__ v16f mfma_chunk_q(const uint4 &a, const uint4 &b, v16f c, __bf16) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const v8bf *>(&a),
                                                   *reinterpret_cast<const v8bf *>(&b), c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// a6: one SP2 product on the matrix cores.
//
// Each workgroup computes one 128x128 tile Y[I,J] = sum_k X[I,k] X[J,k] of
// one part (X is symmetric, so both operands are row panels with k
// contiguous), for ti <= tj only; the eq. (2) update X' = Y or 2X - Y, in
// FP32 against the FP32 master X, is fused into the epilogue and written to
// the other buffer at (I,J) and, mirrored, at (J,I), so every iterate stays
// symmetric: exactly, except with split FP16 operands, whose two cross terms
// a diagonal tile sums in opposite orders for Y[i][j] and Y[j][i] where it
// forms both (the two agree to FP32 rounding, and X_old read at the mirrored
// position is the other rounding).  With 16-bit operands the epilogue also
// writes the rounded copy of X' that the next product reads.  Diagonal tiles
// emit FP64 partial sums of Y and X' over the part's core diagonal.
//
// 256 threads = 4 waves in a 2x2 grid, each wave a 64x64 sub-tile as 2x2
// blocks of 32x32 MFMA output (the skip form deals the blocks of diagonal and
// edge tiles to the waves instead).  Operands are staged through LDS in K chunks,
// two LDS buffers and two register sets deep.  Within a
// chunk, lane half h of an MFMA operand takes the k values of its half of
// every 16-byte group, for A and B alike, so each lane reads whole 16-byte
// LDS words.
// ---------------------------------------------------------------------------
// The 32 x 32 blocks a 128 x 128 tile forms in the skip form, dealt to its
// four waves (wave-uniform; see sp2_tile): blocks wholly in the zero padding
// and, in a diagonal tile, blocks below the diagonal are not formed.  Off the
// diagonal the formed blocks go round robin in row-major order; in a diagonal
// tile the blocks on the diagonal stay with the waves that hold them in the
// 2 x 2 grid (0 and 3) and every other block goes to the least loaded wave
// (the lowest on ties).  A wave gets at most 3 (a diagonal tile forms 10, a
// tile that is not full at most 12).  deal_slot gives slot j of wave wv: the
// block row and column (br, bc), or -1 if the wave has fewer blocks.  Each
// slot is found by its own pass, so that nothing is indexed at run time.
__device__ __forceinline__ void deal_slot(int I0, int J0, int s, bool diag, int wv, int j, int &br, int &bc) {
    br = -1;
    bc = -1;
    int mine = 0;
    auto take = [&](int r, int c) __attribute__((always_inline)) {
        if (mine == j) { br = r; bc = c; }
        ++mine;
    };
    if (!diag) {
        int u = 0;
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c)
                if (I0 + 32 * r < s && J0 + 32 * c < s) {
                    if ((u & 3) == wv) take(r, c);
                    ++u;
                }
    } else {
        int l0 = 0, l1 = 0, l2 = 0, l3 = 0;         // blocks dealt to each wave
        for (int b = 0; b < 4; ++b)
            if (I0 + 32 * b < s) {
                if (b < 2) { ++l0; if (wv == 0) take(b, b); }
                else { ++l3; if (wv == 3) take(b, b); }
            }
        for (int r = 0; r < 4; ++r)
            for (int c = r + 1; c < 4; ++c)
                if (I0 + 32 * c < s) {
                    int w = 0, lw = l0;
                    if (l1 < lw) { w = 1; lw = l1; }
                    if (l2 < lw) { w = 2; lw = l2; }
                    if (l3 < lw) { w = 3; lw = l3; }
                    if (w == 0) ++l0; else if (w == 1) ++l1; else if (w == 2) ++l2; else ++l3;
                    if (w == wv) take(r, c);
                }
    }
}

constexpr int kLdsWords = 2 * 2 * kTile * kLdsRow;  // [buffer][A/B][row * 9 + word]

// kAdj (FP32 only): the adjoint step instead of the product.  buf0 holds the
// cotangent G of X_{t+1} (operand and "old" value of the update), buf1 gets
// the cotangent of X_t, lo0 holds X_t, and the tile accumulates
// sum_k G[I,k] X[J,k] + X[I,k] G[J,k] (the split form's two cross-term
// segments with G and X_t for the two parts); no trace partials.
template <typename Op, bool kSplit = false, bool kSkip = false, bool kAdj = false>
__device__ __forceinline__ void sp2_tile(const TileDesc td, const PartDesc pd, int cur, float alpha,
                                         float *__restrict__ buf0, float *__restrict__ buf1,
                                         Op *__restrict__ sh0, Op *__restrict__ sh1,
                                         double *__restrict__ diag_partials, uint4 *__restrict__ lds_base,
                                         Op *__restrict__ lo0 = nullptr, Op *__restrict__ lo1 = nullptr) {
    constexpr bool kF32 = sizeof(Op) == 4;
    constexpr int kK = OpFmt<Op>::kK;
    constexpr bool kTwo = kSplit || kAdj;       // operands from two matrices (H, L)
    static_assert(!kAdj || (kF32 && !kSplit), "the adjoint step has FP32 operands");
    auto lds = [&](int b, int ab) { return lds_base + (b * 2 + ab) * kTile * kLdsRow; };
    const float *__restrict__ X = (cur ? buf1 : buf0) + pd.x_off;
    float *__restrict__ Xn = (cur ? buf0 : buf1) + pd.x_off;
    const Op *__restrict__ Xop = kF32 ? reinterpret_cast<const Op *>(X) : (cur ? sh1 : sh0) + pd.x_off;
    Op *__restrict__ Xnop = kF32 ? nullptr : (cur ? sh0 : sh1) + pd.x_off;
    // split operands: the scaled low parts of X and of the next iterate
    const Op *__restrict__ Xlo = kTwo ? (cur ? lo1 : lo0) + pd.x_off : nullptr;
    Op *__restrict__ Xnlo = kSplit ? (cur ? lo0 : lo1) + pd.x_off : nullptr;
    const int ld = pd.s_pad;
    const int I0 = td.ti * kTile, J0 = td.tj * kTile;
    const bool diag = td.ti == td.tj;

    const int tid = threadIdx.x;
    // global -> LDS: 8 threads per 128-byte row segment, 32 rows per pass
    const int lr = tid >> 3, lw = tid & 7;
    const char *AgH = reinterpret_cast<const char *>(Xop + (int64_t)(I0 + lr) * ld) + lw * 16;
    const char *BgH = reinterpret_cast<const char *>(Xop + (int64_t)(J0 + lr) * ld) + lw * 16;
    const char *AgL = kTwo ? reinterpret_cast<const char *>(Xlo + (int64_t)(I0 + lr) * ld) + lw * 16 : nullptr;
    const char *BgL = kTwo ? reinterpret_cast<const char *>(Xlo + (int64_t)(J0 + lr) * ld) + lw * 16 : nullptr;
    const int64_t pass_bytes = (int64_t)32 * ld * sizeof(Op);

    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int l32 = lane & 31, kh = lane >> 5;

    v16f acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;

    // K chunks.  Plain: the nk chunks of X[I,:] X[J,:].  Split (X = H + 2^-11 L):
    // nk chunks of H[I,:] L[J,:], nk of L[I,:] H[J,:], the accumulator scaled by
    // 2^-11 (exact), then nk of H[I,:] H[J,:].  Both panels are staged for
    // every chunk, except in a diagonal tile of the one-operand skip form,
    // where the B panel is the A panel.
    //
    // Operands arrive two chunks ahead in two register sets: chunk c + 1 is
    // stored into LDS after the MFMAs of chunk c, from the set loaded before
    // the MFMAs of chunk c - 1.  The loop takes chunks in pairs with the sets
    // fixed, and an odd count ends with one more chunk from buffer 0; past the
    // end the last chunk is loaded again, so every load is unconditional, and
    // the last steps store it again into a buffer no wave reads again.
    // Columns from s on are zero padding, so the K loop stops at the first
    // chunk count covering s (exact: the skipped terms are zeros).
    const int nk = (pd.s + kK - 1) / kK;
    const int nc = kSplit ? 3 * nk : kAdj ? 2 * nk : nk;
    uint4 pa00, pa01, pa02, pa03, pb00, pb01, pb02, pb03;   // register set 0
    uint4 pa10, pa11, pa12, pa13, pb10, pb11, pb12, pb13;   // register set 1
    const char *Ap_ = AgH, *Bp_ = BgH;
    int64_t kb_ = 0;
#define GSP2_SRC(c)                                                                                \
    do {                                                                                           \
        const int c_ = (c);                                                                        \
        Ap_ = AgH; Bp_ = BgH; kb_ = (int64_t)c_ * 128;                                             \
        if constexpr (kTwo) {                                                                      \
            const int seg_ = c_ / nk;                                                              \
            Ap_ = seg_ == 1 ? AgL : AgH;                                                           \
            Bp_ = seg_ == 0 ? BgL : BgH;                                                           \
            kb_ = (int64_t)(c_ - seg_ * nk) * 128;                                                 \
        }                                                                                          \
    } while (0)
    // SHR: a diagonal tile of the skip form with one operand (not the split or
    // adjoint forms), whose B panel is its A panel: the B rows are neither loaded nor stored,
    // and B fragments are read from the A region
#define GSP2_LD(S, c, SHR)                                                                         \
    do {                                                                                           \
        GSP2_SRC(c);                                                                               \
        pa##S##0 = *reinterpret_cast<const uint4 *>(Ap_ + kb_);                                    \
        pa##S##1 = *reinterpret_cast<const uint4 *>(Ap_ + pass_bytes + kb_);                       \
        pa##S##2 = *reinterpret_cast<const uint4 *>(Ap_ + 2 * pass_bytes + kb_);                   \
        pa##S##3 = *reinterpret_cast<const uint4 *>(Ap_ + 3 * pass_bytes + kb_);                   \
        if constexpr (!(SHR)) {                                                                    \
            pb##S##0 = *reinterpret_cast<const uint4 *>(Bp_ + kb_);                                \
            pb##S##1 = *reinterpret_cast<const uint4 *>(Bp_ + pass_bytes + kb_);                   \
            pb##S##2 = *reinterpret_cast<const uint4 *>(Bp_ + 2 * pass_bytes + kb_);               \
            pb##S##3 = *reinterpret_cast<const uint4 *>(Bp_ + 3 * pass_bytes + kb_);               \
        }                                                                                          \
    } while (0)
#define GSP2_ST(b, S, SHR)                                                                         \
    do {                                                                                           \
        uint4 *As_ = lds(b, 0) + lr * kLdsRow + lw;                                                \
        As_[0] = pa##S##0; As_[32 * kLdsRow] = pa##S##1;                                           \
        As_[64 * kLdsRow] = pa##S##2; As_[96 * kLdsRow] = pa##S##3;                                \
        if constexpr (!(SHR)) {                                                                    \
            uint4 *Bs_ = lds(b, 1) + lr * kLdsRow + lw;                                            \
            Bs_[0] = pb##S##0; Bs_[32 * kLdsRow] = pb##S##1;                                       \
            Bs_[64 * kLdsRow] = pb##S##2; Bs_[96 * kLdsRow] = pb##S##3;                            \
        }                                                                                          \
    } while (0)
    // kSkip: work the matrix cores can leave out, exactly (wave-uniform):
    //  * a 32-row (or 32-column) block that starts at or beyond s lies in the
    //    zero padding, so its products are zero (the epilogue still writes
    //    those zeros: padding must stay zero);
    //  * in a diagonal tile a 32 x 32 block below the diagonal is the
    //    transpose of the block above it (the same products in the same
    //    order), so it is not formed and the block above writes both.
    // A full off-diagonal tile keeps the 2 x 2 wave grid.  Any other tile
    // deals the blocks it must form to the four waves, so the waves carry
    // equal work and the tile takes as long as its largest share (at most 3
    // of the 4 blocks a wave of the grid forms: a diagonal tile has 10, an
    // edge tile at most 12): off the diagonal, round robin in row-major
    // order; in a diagonal tile the 32 x 32 blocks on the diagonal stay with
    // the waves that hold them in the grid (0 and 3, so the FP64 trace
    // partials are summed in the grid's order and both forms give the same
    // bits), and each other block goes to the least loaded wave (the lowest
    // on ties).  The choice is made once per tile: each wave runs a
    // straight-line K loop for its block count, so no branch sits among the
    // MFMAs.
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const bool grid_tile = !kSkip || (!diag && I0 + 96 < pd.s && J0 + 96 < pd.s);
    int g_r[3] = {-1, -1, -1}, g_c[3] = {-1, -1, -1};
    int n_mine = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (!grid_tile) deal_slot(I0, J0, pd.s, diag, wv, j, g_r[j], g_c[j]);
        if (g_r[j] >= 0) n_mine = j + 1;
    }
    // kind 0: the wave's 2 x 2 blocks of the grid; 2: none; 3 + M: the wave's
    // M dealt blocks (slot j in acc[j / 2][j % 2])
    auto compute_kind = [&](int buf, auto kind, auto shr) __attribute__((always_inline)) {
        constexpr int K = decltype(kind)::value;
        if constexpr (K == 2) return;
        const uint4 *Asb = lds(buf, 0);
        const uint4 *Bsb = lds(buf, decltype(shr)::value ? 0 : 1);
        // interleave the LDS fragment reads with the MFMAs (3.5% faster FP32
        // products than the default schedule, measured)
        __builtin_amdgcn_iglp_opt(1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            // FP32: word kh*4+q of the row (k = 16 kh + 4 q + e); 16-bit: word 2q+kh (k = 16 q + 8 kh + e)
            const int w = kF32 ? kh * 4 + q : 2 * q + kh;
            if constexpr (K == 0) {
                uint4 fa[2], fb[2];
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    fa[m] = Asb[(wr * 64 + m * 32 + l32) * kLdsRow + w];
                    fb[m] = Bsb[(wc * 64 + m * 32 + l32) * kLdsRow + w];
                }
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int nn = 0; nn < 2; ++nn) acc[m][nn] = mfma_chunk_q(fa[m], fb[nn], acc[m][nn], Op{});
            } else if constexpr (K >= 4) {
                constexpr int M = K - 3;
                uint4 fa[M], fb[M];
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    fa[j] = Asb[(g_r[j] * 32 + l32) * kLdsRow + w];
                    fb[j] = Bsb[(g_c[j] * 32 + l32) * kLdsRow + w];
                }
#pragma unroll
                for (int j = 0; j < M; ++j)
                    acc[j >> 1][j & 1] = mfma_chunk_q(fa[j], fb[j], acc[j >> 1][j & 1], Op{});
            }
        }
    };
    auto kloop = [&](auto kind, auto shr) __attribute__((always_inline)) {
        constexpr bool kShr = decltype(shr)::value;
        GSP2_LD(0, 0, kShr);
        GSP2_ST(0, 0, kShr);
        GSP2_LD(1, min(1, nc - 1), kShr);
        __syncthreads();
        int kc = 0;
        for (; kc + 1 < nc; kc += 2) {
            if constexpr (kSplit) {
                if (kc == 2 * nk) {             // cross terms done: scale them by 2^-11
#pragma unroll
                    for (int m = 0; m < 2; ++m)
#pragma unroll
                        for (int nn = 0; nn < 2; ++nn) acc[m][nn] *= 0x1p-11f;
                }
            }
            GSP2_LD(0, min(kc + 2, nc - 1), kShr);
            compute_kind(0, kind, shr);
            GSP2_ST(1, 1, kShr);
            __syncthreads();
            GSP2_LD(1, min(kc + 3, nc - 1), kShr);
            compute_kind(1, kind, shr);
            GSP2_ST(0, 0, kShr);
            __syncthreads();
        }
        if (kc < nc) {                          // an odd count's last chunk, stored in buffer 0
            if constexpr (kSplit) {
                if (kc == 2 * nk) {             // (nk = 1: the H H chunk is this one)
#pragma unroll
                    for (int m = 0; m < 2; ++m)
#pragma unroll
                        for (int nn = 0; nn < 2; ++nn) acc[m][nn] *= 0x1p-11f;
                }
            }
            compute_kind(0, kind, shr);
            __syncthreads();                    // as after a pair: LDS is free again when the loop ends
        }
    };
    auto kloops = [&](auto shr) __attribute__((always_inline)) {
        if constexpr (!kSkip) {
            kloop(std::integral_constant<int, 0>{}, shr);
        } else {
            // (a diagonal tile is never a grid tile here)
            if constexpr (!decltype(shr)::value) {
                if (grid_tile) {
                    kloop(std::integral_constant<int, 0>{}, shr);
                    return;
                }
            }
            if (n_mine == 0) kloop(std::integral_constant<int, 2>{}, shr);
            else if (n_mine == 1) kloop(std::integral_constant<int, 4>{}, shr);
            else if (n_mine == 2) kloop(std::integral_constant<int, 5>{}, shr);
            else kloop(std::integral_constant<int, 6>{}, shr);
        }
    };
    // Only the skip form shares the panel: it runs its diagonal tiles after
    // the full ones.  In the plain form's list, tiles of one length keep the
    // workgroups in step; shorter diagonal tiles among them spread the
    // resident tiles over more panels, and the HBM reads grew by half
    // (measured), more than the loads saved.
    if constexpr (kTwo || !kSkip) kloops(std::false_type{});
    else if (diag) kloops(std::true_type{});
    else kloops(std::false_type{});
#undef GSP2_SRC
#undef GSP2_LD
#undef GSP2_ST

    // Epilogue.  Accumulator element i of lane (l32, kh) in a 32x32 block is
    // row 8*(i/4) + 4*kh + (i%4), column l32.  Plain 16-bit operands carry X
    // without its diagonal D (X = D + O): the matrix cores formed O O, and
    // the epilogue adds D O + O D + D^2 in FP32, (d_r + d_c) X_rc off the
    // diagonal and d_r^2 on it, so the diagonal is never rounded.
    constexpr bool kExactDiag = !kF32 && !kSplit;
    double tY = 0.0, tX = 0.0;
    // X_old (for X' = 2X - Y and, with plain 16-bit operands, the diagonal
    // terms) is read at the mirrored position, X[r][c] = X[c][r] (X is
    // symmetric), as one float4 per lane and row group, for all of the wave's
    // blocks before any store: a wave's loads complete in order behind its
    // earlier stores, so reads between stores would wait for them.
    // (Split operands, whose epilogue holds more registers, read them one
    // block at a time, just before that block's stores.)
    const bool need_xo = kExactDiag || alpha > 0.0f;
    constexpr bool kAllAhead = !kSplit;
    float4 xo4[kAllAhead ? 4 : 1][4];           // [block slot][row group]
    auto load_xo = [&](int slot, int ro, int co) __attribute__((always_inline)) {
        const int cg = J0 + co + l32;
        const int sl = kAllAhead ? slot : 0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int rg0 = I0 + ro + g * 8 + kh * 4;
            xo4[sl][g] = need_xo ? *reinterpret_cast<const float4 *>(X + (int64_t)cg * ld + rg0)
                                 : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
    };
    // one 32 x 32 block of the tile (its first row and column within the
    // tile: ro, co) from its accumulator, written at its place and, with
    // write_mirror, transposed at the mirrored place
    auto emit_block = [&](const v16f &a, int slot, int ro, int co, bool write_mirror) __attribute__((always_inline)) {
        if constexpr (!kAllAhead) load_xo(slot, ro, co);
        const int sl = kAllAhead ? slot : 0;
        const int cg = J0 + co + l32;
        const float dc = kExactDiag ? X[(int64_t)cg * (ld + 1)] : 0.0f;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int rg0 = I0 + ro + g * 8 + kh * 4;
            const float xov[4] = {xo4[sl][g].x, xo4[sl][g].y, xo4[sl][g].z, xo4[sl][g].w};
            float xn[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int rg = rg0 + e;
                const float yacc = a[4 * g + e];
                const float xo = xov[e];
                float y = yacc;
                if constexpr (kExactDiag) {
                    const float dr = X[(int64_t)rg * (ld + 1)];
                    // explicit FMAs: every inlined copy of this epilogue rounds alike
                    y = rg == cg ? __builtin_fmaf(dr, dr, yacc) : __builtin_fmaf(dr + dc, xo, yacc);
                }
                const float v = alpha > 0.0f ? (2.0f * xo - y) : y;
                xn[e] = v;
                Xn[(int64_t)rg * ld + cg] = v;
                if constexpr (!kF32) {
                    const Op h = (kExactDiag && rg == cg) ? static_cast<Op>(0.0f) : static_cast<Op>(v);
                    Xnop[(int64_t)rg * ld + cg] = h;
                    if constexpr (kSplit)
                        Xnlo[(int64_t)rg * ld + cg] = static_cast<Op>((v - static_cast<float>(h)) * 0x1p11f);
                }
                if (!kAdj && diag && rg == cg && rg < pd.c) {
                    tY += static_cast<double>(y);
                    tX += static_cast<double>(v);
                }
            }
            if (write_mirror) {
                const float4 v4 = make_float4(xn[0], xn[1], xn[2], xn[3]);
                *reinterpret_cast<float4 *>(Xn + (int64_t)cg * ld + rg0) = v4;
                if constexpr (!kF32) {
                    union { Op h[4]; uint2 u; } pk, pl;
#pragma unroll
                    for (int e = 0; e < 4; ++e) pk.h[e] = static_cast<Op>(xn[e]);
                    *reinterpret_cast<uint2 *>(Xnop + (int64_t)cg * ld + rg0) = pk.u;
                    if constexpr (kSplit) {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            pl.h[e] = static_cast<Op>((xn[e] - static_cast<float>(pk.h[e])) * 0x1p11f);
                        *reinterpret_cast<uint2 *>(Xnlo + (int64_t)cg * ld + rg0) = pl.u;
                    }
                }
            }
        }
    };
    // a block wholly in the zero padding: its products and X_old are zero,
    // so X' is +0 there (as the grid forms it), written without reading
    auto emit_zero = [&](int ro, int co, bool write_mirror) __attribute__((always_inline)) {
        const int cg = J0 + co + l32;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int rg0 = I0 + ro + g * 8 + kh * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                Xn[(int64_t)(rg0 + e) * ld + cg] = 0.0f;
                if constexpr (!kF32) {
                    Xnop[(int64_t)(rg0 + e) * ld + cg] = static_cast<Op>(0.0f);
                    if constexpr (kSplit) Xnlo[(int64_t)(rg0 + e) * ld + cg] = static_cast<Op>(0.0f);
                }
            }
            if (write_mirror) {
                *reinterpret_cast<float4 *>(Xn + (int64_t)cg * ld + rg0) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if constexpr (!kF32) {
                    *reinterpret_cast<uint2 *>(Xnop + (int64_t)cg * ld + rg0) = make_uint2(0u, 0u);
                    if constexpr (kSplit) *reinterpret_cast<uint2 *>(Xnlo + (int64_t)cg * ld + rg0) = make_uint2(0u, 0u);
                }
            }
        }
    };
    if (grid_tile) {
        if constexpr (kAllAhead) {
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int nn = 0; nn < 2; ++nn) load_xo(2 * m + nn, wr * 64 + m * 32, wc * 64 + nn * 32);
        }
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int nn = 0; nn < 2; ++nn)
                emit_block(acc[m][nn], 2 * m + nn, wr * 64 + m * 32, wc * 64 + nn * 32, !diag);
    } else {
        if constexpr (kAllAhead) {
#pragma unroll
            for (int j = 0; j < 3; ++j)
                if (j < n_mine) load_xo(j, 32 * g_r[j], 32 * g_c[j]);
        }
#pragma unroll
        for (int j = 0; j < 3; ++j)
            if (j < n_mine) emit_block(acc[j >> 1][j & 1], j, 32 * g_r[j], 32 * g_c[j], !diag || g_r[j] < g_c[j]);
        // the padding blocks of the tile (both triangles of a diagonal tile),
        // dealt round robin
        int k = 0;
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
                if (I0 + 32 * r < pd.s && J0 + 32 * c < pd.s) continue;
                if ((k & 3) == wv) emit_zero(32 * r, 32 * c, !diag);
                ++k;
            }
    }
    if (!kAdj && diag) {
        block_sum2(tY, tX);
        if (tid == 0) {
            diag_partials[2 * td.diag_slot + 0] = tY;
            diag_partials[2 * td.diag_slot + 1] = tX;
        }
    }
}

template <typename Op, bool kSplit = false, bool kSkip = false>
__global__ __launch_bounds__(kBlock, 2) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_sp2_step(const TileDesc *__restrict__ tiles,
                                                        const PartDesc *__restrict__ parts,
                                                        float *__restrict__ buf0, float *__restrict__ buf1,
                                                        Op *__restrict__ sh0, Op *__restrict__ sh1,
                                                        const RunState *__restrict__ st_all,
                                                        double *__restrict__ diag_partials, int phase,
                                                        Op *__restrict__ lo0, Op *__restrict__ lo1) {
    __shared__ uint4 lds[kLdsWords];
    const TileDesc td = tiles[blockIdx.x];
    if (td.part < 0) return;                    // padding of a short XCD list
    const PartDesc pd = parts[td.part];
    const RunState *st = st_all + pd.sys;       // each system runs, stops and branches on its own
    if (st->done || st->phase != phase) return;
    sp2_tile<Op, kSplit, kSkip>(td, pd, st->cur, static_cast<float>(st->alpha), buf0, buf1, sh0, sh1,
                                diag_partials, lds, lo0, lo1);
}

// ---------------------------------------------------------------------------
// a6 in FP64 (the paper's dgemm arithmetic): one SP2 product with FP64
// operands, accumulation, master iterate and update, on
// v_mfma_f64_16x16x4_f64.
//
// The tile scheme is the FP32 kernel's: 128 x 128 tiles of the upper
// triangle, 4 waves in a 2 x 2 grid of 64 x 64 sub-tiles, operands staged
// through two LDS buffers in K chunks of 128 bytes per row (16 doubles), the
// update fused into the epilogue and written at (I,J) and mirrored at (J,I).
// A wave's sub-tile is 4 x 4 blocks of 16 x 16 MFMA output (four doubles per
// lane each).  MFMA step q of a chunk gives lane group g = lane / 16 the
// column 4 g + q of its row, for A and B alike, so each lane reads its four
// columns of a chunk as 32 contiguous bytes of LDS.  FP64 MFMAs are slow
// enough that one chunk's matrix work covers the next chunk's loads, so one
// register set suffices.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

template <bool kSkip = false>
__device__ __forceinline__ void sp2_tile64(const TileDesc td, const PartDesc pd, int cur, double alpha,
                                           double *__restrict__ buf0, double *__restrict__ buf1,
                                           double *__restrict__ diag_partials, uint4 *__restrict__ lds_base) {
    auto lds = [&](int b, int ab) { return lds_base + (b * 2 + ab) * kTile * kLdsRow; };
    const double *__restrict__ X = (cur ? buf1 : buf0) + pd.x_off;
    double *__restrict__ Xn = (cur ? buf0 : buf1) + pd.x_off;
    const int ld = pd.s_pad;
    const int I0 = td.ti * kTile, J0 = td.tj * kTile;
    const bool diag = td.ti == td.tj;
    const int tid = threadIdx.x;
    // global -> LDS: 8 threads per 128-byte row segment, 32 rows per pass
    const int lr = tid >> 3, lw = tid & 7;
    const char *Ag = reinterpret_cast<const char *>(X + (int64_t)(I0 + lr) * ld) + lw * 16;
    const char *Bg = reinterpret_cast<const char *>(X + (int64_t)(J0 + lr) * ld) + lw * 16;
    const int64_t pass_bytes = (int64_t)32 * ld * sizeof(double);
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int l16 = lane & 15, g = lane >> 4;

    v4d acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};

    // The skip form deals the tile's 32 x 32 blocks to the waves as sp2_tile
    // does (deal_slot); a 32 x 32 block is 2 x 2 MFMA blocks of 16 x 16, and
    // sub-block (a, b) of slot j accumulates in acc[2 (j / 2) + a][2 (j % 2) + b].
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const bool grid_tile = !kSkip || (!diag && I0 + 96 < pd.s && J0 + 96 < pd.s);
    int g_r[3] = {-1, -1, -1}, g_c[3] = {-1, -1, -1};
    int n_mine = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (!grid_tile) deal_slot(I0, J0, pd.s, diag, wv, j, g_r[j], g_c[j]);
        if (g_r[j] >= 0) n_mine = j + 1;
    }

    // columns from s on are zero padding: the K loop stops at the first
    // chunk that covers s (the skipped terms are exact zeros)
    constexpr int kK64 = 16;
    const int nk = (pd.s + kK64 - 1) / kK64;
    uint4 pa0, pa1, pa2, pa3, pb0, pb1, pb2, pb3;
#define GSP2_LD64(c)                                                                               \
    do {                                                                                           \
        const int64_t kb_ = (int64_t)(c) * 128;                                                    \
        pa0 = *reinterpret_cast<const uint4 *>(Ag + kb_);                                          \
        pa1 = *reinterpret_cast<const uint4 *>(Ag + pass_bytes + kb_);                             \
        pa2 = *reinterpret_cast<const uint4 *>(Ag + 2 * pass_bytes + kb_);                         \
        pa3 = *reinterpret_cast<const uint4 *>(Ag + 3 * pass_bytes + kb_);                         \
        pb0 = *reinterpret_cast<const uint4 *>(Bg + kb_);                                          \
        pb1 = *reinterpret_cast<const uint4 *>(Bg + pass_bytes + kb_);                             \
        pb2 = *reinterpret_cast<const uint4 *>(Bg + 2 * pass_bytes + kb_);                         \
        pb3 = *reinterpret_cast<const uint4 *>(Bg + 3 * pass_bytes + kb_);                         \
    } while (0)
#define GSP2_ST64(b)                                                                               \
    do {                                                                                           \
        uint4 *As_ = lds(b, 0) + lr * kLdsRow + lw;                                                \
        uint4 *Bs_ = lds(b, 1) + lr * kLdsRow + lw;                                                \
        As_[0] = pa0; As_[32 * kLdsRow] = pa1; As_[64 * kLdsRow] = pa2; As_[96 * kLdsRow] = pa3;   \
        Bs_[0] = pb0; Bs_[32 * kLdsRow] = pb1; Bs_[64 * kLdsRow] = pb2; Bs_[96 * kLdsRow] = pb3;   \
    } while (0)
    // kind 0: the wave's 4 x 4 MFMA blocks of the grid; 2: none; 3 + M: its M dealt blocks
    auto compute = [&](int b, auto kind) __attribute__((always_inline)) {
        constexpr int K = decltype(kind)::value;
        if constexpr (K == 2) return;
        const uint4 *Asb = lds(b, 0);
        const uint4 *Bsb = lds(b, 1);
        if constexpr (K == 0) {
            // MFMA steps in two halves (steps 2h, 2h + 1: the h-th 16 bytes of
            // a lane's row piece)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                double fa[4][2], fb[4][2];          // [block][step in half]
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const double2 va = __builtin_bit_cast(double2, Asb[(wr * 64 + m * 16 + l16) * kLdsRow + 2 * g + h]);
                    const double2 vb = __builtin_bit_cast(double2, Bsb[(wc * 64 + m * 16 + l16) * kLdsRow + 2 * g + h]);
                    fa[m][0] = va.x; fa[m][1] = va.y;
                    fb[m][0] = vb.x; fb[m][1] = vb.y;
                }
#pragma unroll
                for (int qq = 0; qq < 2; ++qq)
#pragma unroll
                    for (int m = 0; m < 4; ++m)
#pragma unroll
                        for (int nn = 0; nn < 4; ++nn)
                            acc[m][nn] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[m][qq], fb[nn][qq], acc[m][nn], 0, 0, 0);
            }
        } else if constexpr (K >= 4) {
            constexpr int M = K - 3;
            // MFMA steps in two halves (steps 2h, 2h + 1: the h-th 16 bytes of a
            // lane's row piece), each element in the same k order as the grid
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int j = 0; j < M; ++j) {       // one slot's fragments at a time
                    double fa[2][2], fb[2][2];      // [sub-block row / column][step in half]
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        const double2 va = __builtin_bit_cast(
                            double2, Asb[(g_r[j] * 32 + a * 16 + l16) * kLdsRow + 2 * g + h]);
                        const double2 vb = __builtin_bit_cast(
                            double2, Bsb[(g_c[j] * 32 + a * 16 + l16) * kLdsRow + 2 * g + h]);
                        fa[a][0] = va.x; fa[a][1] = va.y;
                        fb[a][0] = vb.x; fb[a][1] = vb.y;
                    }
#pragma unroll
                    for (int qq = 0; qq < 2; ++qq)
#pragma unroll
                        for (int a = 0; a < 2; ++a)
#pragma unroll
                            for (int bb = 0; bb < 2; ++bb) {
                                v4d &c = acc[2 * (j >> 1) + a][2 * (j & 1) + bb];
                                c = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a][qq], fb[bb][qq], c, 0, 0, 0);
                            }
                }
        }
    };
    auto kloop = [&](auto kind) __attribute__((always_inline)) {
        GSP2_LD64(0);
        GSP2_ST64(0);
        __syncthreads();
        for (int kc = 0; kc < nk; ++kc) {
            const int b = kc & 1;
            if (kc + 1 < nk) GSP2_LD64(kc + 1);
            compute(b, kind);
            if (kc + 1 < nk) GSP2_ST64(b ^ 1);
            __syncthreads();
        }
    };
    if constexpr (!kSkip) {
        kloop(std::integral_constant<int, 0>{});
    } else {
        if (grid_tile) kloop(std::integral_constant<int, 0>{});
        else if (n_mine == 0) kloop(std::integral_constant<int, 2>{});
        else if (n_mine == 1) kloop(std::integral_constant<int, 4>{});
        else if (n_mine == 2) kloop(std::integral_constant<int, 5>{});
        else kloop(std::integral_constant<int, 6>{});
    }
#undef GSP2_LD64
#undef GSP2_ST64

    // Epilogue.  Element v of a 16 x 16 block's accumulator in lane (l16, g)
    // is row 4 v + g, column l16 (the FP64 MFMA interleaves its output rows
    // over the lane groups, unlike the 16 x 16 FP32 and 16-bit forms).  X_old
    // and the direct writes are 16 consecutive columns of one row per lane
    // group; each mirrored row receives 4 consecutive doubles per MFMA row
    // group.
    double tY = 0.0, tX = 0.0;
    const bool upd = alpha > 0.0;
    // one 16 x 16 block (first row and column within the tile: ro, co)
    auto emit16 = [&](const v4d &a, int ro, int co, bool write_mirror) __attribute__((always_inline)) {
        const int cg = J0 + co + l16;
        const int rb = I0 + ro + g;
        double xo[4] = {0.0, 0.0, 0.0, 0.0};
        if (upd) {
#pragma unroll
            for (int v = 0; v < 4; ++v) xo[v] = X[(int64_t)(rb + 4 * v) * ld + cg];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rg = rb + 4 * v;
            const double y = a[v];
            const double val = upd ? (2.0 * xo[v] - y) : y;
            Xn[(int64_t)rg * ld + cg] = val;
            if (write_mirror) Xn[(int64_t)cg * ld + rg] = val;
            if (diag && rg == cg && cg < pd.c) {
                tY += y;
                tX += val;
            }
        }
    };
    if (grid_tile) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int nn = 0; nn < 4; ++nn) emit16(acc[m][nn], wr * 64 + m * 16, wc * 64 + nn * 16, !diag);
    } else {
#pragma unroll
        for (int j = 0; j < 3; ++j)
            if (j < n_mine) {
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int bb = 0; bb < 2; ++bb)
                        emit16(acc[2 * (j >> 1) + a][2 * (j & 1) + bb], g_r[j] * 32 + a * 16, g_c[j] * 32 + bb * 16,
                               !diag || g_r[j] < g_c[j]);
            }
        // 32 x 32 blocks wholly in the padding: X' is +0 there, written without reading
        int k = 0;
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
                if (I0 + 32 * r < pd.s && J0 + 32 * c < pd.s) continue;
                if ((k & 3) == wv) {
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int bb = 0; bb < 2; ++bb) {
                            const int cg = J0 + 32 * c + bb * 16 + l16;
                            const int rb = I0 + 32 * r + a * 16 + g;
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                Xn[(int64_t)(rb + 4 * v) * ld + cg] = 0.0;
                                if (!diag) Xn[(int64_t)cg * ld + rb + 4 * v] = 0.0;
                            }
                        }
                }
                ++k;
            }
    }
    if (diag) {
        block_sum2(tY, tX);
        if (tid == 0) {
            diag_partials[2 * td.diag_slot + 0] = tY;
            diag_partials[2 * td.diag_slot + 1] = tX;
        }
    }
}

template <bool kSkip>
__global__ __launch_bounds__(kBlock, 2) void k_sp2_step64(const TileDesc *__restrict__ tiles,
                                                       const PartDesc *__restrict__ parts,
                                                       double *__restrict__ buf0, double *__restrict__ buf1,
                                                       const RunState *__restrict__ st_all,
                                                       double *__restrict__ diag_partials, int phase) {
    __shared__ uint4 lds[kLdsWords];
    const TileDesc td = tiles[blockIdx.x];
    if (td.part < 0) return;
    const PartDesc pd = parts[td.part];
    const RunState *st = st_all + pd.sys;
    if (st->done || st->phase != phase) return;
    sp2_tile64<kSkip>(td, pd, st->cur, static_cast<double>(st->alpha), buf0, buf1, diag_partials, lds);
}

// ---------------------------------------------------------------------------
// a6 with 16-bit operands: 256 x 256 product tiles.
//
// At 16 bits the matrix cores run sixteen times faster than at FP32, so the
// product is limited by how fast operands reach them.  A 256 x 256 tile
// halves the operand bytes per flop against a 128-wide one, both from L2
// and through LDS.  256 threads = 4 waves in a 2 x 2 grid, one wave per
// SIMD, each wave a 128 x 128 sub-tile as 4 x 4 blocks of 32 x 32 MFMA
// output (256 accumulator registers): 8 LDS fragment reads feed 16 MFMAs.
// Two LDS buffers of 2 x 256 rows x 144 B (147,456 bytes) hold one
// workgroup per CU; operands arrive by buffer loads two chunks ahead, in
// two register sets, and are stored into LDS between the MFMAs of the
// chunk before.  Tiles step by 256 over the part; where s_pad is an odd
// multiple of 128, the last tile row and column are half empty: those rows
// are neither loaded nor computed.  A diagonal tile's trace partials go to
// the two 128-tile slots it covers, so the control kernels are those of the
// 128-tile product.
// ---------------------------------------------------------------------------
constexpr int kTileW = 256;
constexpr int kBlockW = 256;
constexpr int kBufferWord3 = 0x00020000;   // raw buffer descriptor word 3 on gfx9-family parts
constexpr int kLdsWordsW = 2 * 2 * kTileW * kLdsRow;  // [buffer][A/B][row * 9 + word]: 147,456 bytes

template <typename Op, bool kSplit>
__device__ __forceinline__ void sp2_tile_wide(const TileDesc td, const PartDesc pd, int cur, float alpha,
                                              float *__restrict__ buf0, float *__restrict__ buf1,
                                              Op *__restrict__ sh0, Op *__restrict__ sh1, Op *__restrict__ lo0,
                                              Op *__restrict__ lo1, double *__restrict__ diag_partials,
                                              uint4 *__restrict__ lds_base) {
    static_assert(sizeof(Op) == 2, "wide tiles are for 16-bit operands");
    constexpr int kK = OpFmt<Op>::kK;
    __shared__ double red[2][kBlockW / kWave];
    auto lds = [&](int b, int ab) { return lds_base + (b * 2 + ab) * kTileW * kLdsRow; };
    const float *__restrict__ X = (cur ? buf1 : buf0) + pd.x_off;
    float *__restrict__ Xn = (cur ? buf0 : buf1) + pd.x_off;
    const Op *__restrict__ Xop = (cur ? sh1 : sh0) + pd.x_off;
    Op *__restrict__ Xnop = (cur ? sh0 : sh1) + pd.x_off;
    const Op *__restrict__ Xlo = kSplit ? (cur ? lo1 : lo0) + pd.x_off : nullptr;
    Op *__restrict__ Xnlo = kSplit ? (cur ? lo0 : lo1) + pd.x_off : nullptr;
    const int ld = pd.s_pad;
    const int I0 = td.ti * kTileW, J0 = td.tj * kTileW;
    const bool diag = td.ti == td.tj;
    const bool fullA = I0 + kTileW <= ld, fullB = J0 + kTileW <= ld;   // else 128 rows remain

    const int tid = threadIdx.x;
    // global -> LDS: 8 threads per 128-byte row segment, 32 rows per pass,
    // passes 4 to 7 only where the panel has all 256 rows.  Buffer loads:
    // the part's operand matrix is one buffer, each lane keeps a 32-bit
    // offset and the pass and chunk offsets are uniform (scalar registers).
    const int lr = tid >> 3, lw = tid & 7;
    const uint32_t mat_bytes = static_cast<uint32_t>(ld) * static_cast<uint32_t>(ld) * sizeof(Op);
    const __amdgpu_buffer_rsrc_t rH = __builtin_amdgcn_make_buffer_rsrc(const_cast<Op *>(Xop), 0, mat_bytes,
                                                                          kBufferWord3);
    const __amdgpu_buffer_rsrc_t rL =
        kSplit ? __builtin_amdgcn_make_buffer_rsrc(const_cast<Op *>(Xlo), 0, mat_bytes, kBufferWord3) : rH;
    // the host keeps s_pad <= kMaxWidePad, so every offset fits 32 bits
    const uint32_t offA = (static_cast<uint32_t>(I0 + lr) * ld + lw * 8) * sizeof(Op);
    const uint32_t offB = (static_cast<uint32_t>(J0 + lr) * ld + lw * 8) * sizeof(Op);
    const uint32_t pass_bytes = 32u * ld * sizeof(Op);
    uint32_t passA[8], passB[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        passA[p] = (fullA ? p : (p & 3)) * pass_bytes;
        passB[p] = (fullB ? p : (p & 3)) * pass_bytes;
    }

    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;        // rows wr*128.., columns wc*128..
    const int l32 = lane & 31, kh = lane >> 5;
    const bool active = (wr == 0 || fullA) && (wc == 0 || fullB);

    v16f acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;

    // chunks as in sp2_tile: plain nk of X X; split nk of H L, nk of L H,
    // the scale by 2^-11, nk of H H.  Both panels are staged for every
    // chunk, except in a diagonal tile with plain operands, where the B panel
    // is the A panel.
    const int nk = ld / kK;
    uint4 pa[2][8], pb[2][8];
#define GSP2W_SRC(c, ra, rb, kb)                                                                   \
    do {                                                                                           \
        if constexpr (kSplit) {                                                                    \
            const int seg_ = (c) / nk;                                                             \
            ra = seg_ == 1 ? rL : rH;                                                              \
            rb = seg_ == 0 ? rL : rH;                                                              \
            kb = static_cast<uint32_t>((c) - seg_ * nk) * 128u;                                    \
        } else {                                                                                   \
            ra = rH; rb = rH; kb = static_cast<uint32_t>(c) * 128u;                                \
        }                                                                                          \
    } while (0)
    // every pass is loaded and stored, so no register keeps a value from an
    // earlier chunk; a half-empty panel repeats its first 128 rows in passes
    // 4 to 7 (in bounds; those LDS rows are not read).  Two register sets:
    // chunk c + 2 is loaded while chunk c + 1 waits to be stored.
    // SHR: a diagonal tile with plain operands, whose B panel is its A panel:
    // the B rows are neither loaded nor stored, and B fragments are read from
    // the A region (half the panel requests to L2 and the LDS stores)
#define GSP2W_LOAD(S, ra, rb, kb, SHR)                                                             \
    do {                                                                                           \
        _Pragma("unroll") for (int p_ = 0; p_ < 8; ++p_) {                                         \
            pa[S][p_] = __builtin_bit_cast(                                                        \
                uint4, __builtin_amdgcn_raw_buffer_load_b128(ra, offA, passA[p_] + (kb), 0));      \
            if constexpr (!(SHR))                                                                  \
                pb[S][p_] = __builtin_bit_cast(                                                    \
                    uint4, __builtin_amdgcn_raw_buffer_load_b128(rb, offB, passB[p_] + (kb), 0));  \
        }                                                                                          \
    } while (0)
#define GSP2W_STORE(b, S, SHR)                                                                     \
    do {                                                                                           \
        uint4 *As_ = lds(b, 0) + lr * kLdsRow + lw;                                                \
        uint4 *Bs_ = lds(b, 1) + lr * kLdsRow + lw;                                                \
        _Pragma("unroll") for (int p_ = 0; p_ < 8; ++p_) {                                         \
            As_[p_ * 32 * kLdsRow] = pa[S][p_];                                                    \
            if constexpr (!(SHR)) Bs_[p_ * 32 * kLdsRow] = pb[S][p_];                              \
        }                                                                                          \
    } while (0)

    // the MFMAs of one chunk from LDS buffer buf, with the stores of the
    // next chunk (register set sa, sb, loaded a chunk earlier) into the
    // other buffer folded into its steps 0 to 2.  Every wave runs the MFMAs
    // (a branch around them would make the accumulators flow through
    // VGPRs); an inactive wave's results are discarded.  The fragments of
    // step q + 1 are read while the MFMAs of step q run, interleaved with
    // them; a scheduling barrier per step keeps the compiler from moving
    // memory operations across steps.  The workgroup barrier sits before step 3:
    // by then every wave has stored its part of the next chunk and read the
    // last fragments of this one, so step 3's MFMAs cover the reads of the
    // next chunk's step-0 fragments.
    uint4 fa[2][4], fb[2][4];
    auto frags = [&](int b, int q, uint4 *fa_, uint4 *fb_, auto shr) __attribute__((always_inline)) {
        const uint4 *Asb = lds(b, 0);
        const uint4 *Bsb = lds(b, decltype(shr)::value ? 0 : 1);
        const int w = 2 * q + kh;               // k = 16 q + 8 kh + e
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            fa_[m] = Asb[(wr * 128 + m * 32 + l32) * kLdsRow + w];
            fb_[m] = Bsb[(wc * 128 + m * 32 + l32) * kLdsRow + w];
        }
    };
    auto compute = [&](int buf, uint4 (&sa)[8], uint4 (&sb)[8], __amdgpu_buffer_rsrc_t ra,
                       __amdgpu_buffer_rsrc_t rb, uint32_t kb, auto shr) __attribute__((always_inline)) {
        constexpr bool kShr = decltype(shr)::value;
        uint4 *As_ = lds(buf ^ 1, 0) + lr * kLdsRow + lw;
        uint4 *Bs_ = lds(buf ^ 1, 1) + lr * kLdsRow + lw;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q + 1 < 4) {
                frags(buf, q + 1, fa[(q + 1) & 1], fb[(q + 1) & 1], shr);
            } else {
                __syncthreads();
                frags(buf ^ 1, 0, fa[0], fb[0], shr);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int nn = 0; nn < 4; ++nn)
                    acc[m][nn] = mfma_chunk_q(fa[q & 1][m], fb[q & 1][nn], acc[m][nn], Op{});
            // passes 0-2 in step 0, 3-5 in step 1, 6-7 in step 2; each
            // register is loaded again (chunk c + 3) as soon as it is stored
            const int p0 = 3 * q, np = q < 2 ? 3 : (q == 2 ? 2 : 0);
#pragma unroll
            for (int p = 0; p < np; ++p) {
                As_[(p0 + p) * 32 * kLdsRow] = sa[p0 + p];
                if constexpr (!kShr) Bs_[(p0 + p) * 32 * kLdsRow] = sb[p0 + p];
                sa[p0 + p] = __builtin_bit_cast(
                    uint4, __builtin_amdgcn_raw_buffer_load_b128(ra, offA, passA[p0 + p] + kb, 0));
                if constexpr (!kShr)
                    sb[p0 + p] = __builtin_bit_cast(
                        uint4, __builtin_amdgcn_raw_buffer_load_b128(rb, offB, passB[p0 + p] + kb, 0));
            }
            // the compiler's MFMA / LDS interleave for one wave per SIMD (3% faster
            // than placing one LDS access after each of the first MFMAs, measured)
            __builtin_amdgcn_iglp_opt(1);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    // one pass over chunks [c0, c1): chunk c computes from LDS buffer
    // (c - c0) & 1 while chunk c + 1 waits in registers to be stored into
    // the other buffer and chunk c + 2 is being loaded.  Chunk counts are
    // even (s_pad is a multiple of 128, a chunk 64 columns), so the loop
    // takes chunks in pairs and every MFMA block is unconditional.  The last
    // pair stores its final chunk a second time into the buffer it already
    // occupies, which no wave reads during that step, and its last step
    // reads fragments that are not used.  The barriers at entry and exit
    // keep LDS reuse (a second pass, the epilogue) clear of these reads.
    auto run = [&](int c0, int c1, auto shr) __attribute__((always_inline)) {
        constexpr bool kShr = decltype(shr)::value;
        __amdgpu_buffer_rsrc_t ra, rb;
        uint32_t kb;
        __syncthreads();
        GSP2W_SRC(c0, ra, rb, kb);
        GSP2W_LOAD(0, ra, rb, kb, kShr);
        GSP2W_STORE(0, 0, kShr);
        GSP2W_SRC(c0 + 1, ra, rb, kb);
        GSP2W_LOAD(1, ra, rb, kb, kShr);
        GSP2W_SRC(min(c0 + 2, c1 - 1), ra, rb, kb);
        GSP2W_LOAD(0, ra, rb, kb, kShr);
        __syncthreads();
        frags(0, 0, fa[0], fb[0], shr);
        for (int kc = c0; kc < c1; kc += 2) {
            // past the end the last chunk is loaded again, so that every
            // load is unconditional and the waits before the stores count
            // exactly the loads issued after them
            GSP2W_SRC(min(kc + 3, c1 - 1), ra, rb, kb);
            compute(0, pa[1], pb[1], ra, rb, kb, shr);
            GSP2W_SRC(min(kc + 4, c1 - 1), ra, rb, kb);
            compute(1, pa[0], pb[0], ra, rb, kb, shr);
        }
        __syncthreads();
    };
    const std::false_type own_b;
    if constexpr (kSplit) {
        run(0, 2 * nk, own_b);                  // cross terms H L and L H
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int nn = 0; nn < 4; ++nn) acc[m][nn] *= 0x1p-11f;
        run(2 * nk, 3 * nk, own_b);             // H H
    } else {
        if (diag) run(0, nk, std::true_type{});
        else run(0, nk, own_b);
    }
#undef GSP2W_SRC
#undef GSP2W_LOAD
#undef GSP2W_STORE

    // Epilogue: as in sp2_tile, over this wave's 4 x 4 blocks, one 32-row
    // band m at a time.  X_old is only needed for X' = 2X - Y; each lane's
    // four rows of one column are read at the mirrored position (X is
    // symmetric), all sixteen reads before any of the band's stores, so the
    // wave waits on memory once per band rather than once per element group.
    // The mirrored writes leave the registers as float4 columns; the direct
    // writes go through this wave's own 16 KB of LDS (free after the last
    // chunk's barrier), so that they too are 16-byte row pieces: 2 rows x
    // 512 contiguous bytes per store instruction.
    //
    // The FP32 master is not written in full during the 16-bit products:
    // plain operands write it on the diagonal tiles and at the mirrored
    // (lower) positions only, which is all the next product reads; split
    // operands do not write it at all and read X_old as hi + 2^-11 lo.  The
    // fixup after the last product completes it (k_wide_fixup).
    constexpr int kBandRow = 132;               // floats per LDS band row: 128 + 4 pad
    float *band = reinterpret_cast<float *>(lds_base) + wave * 32 * kBandRow;
    // Plain operands carry X without its diagonal D (X = D + O): the matrix
    // cores formed O O, and the epilogue adds D O + O D + D^2 in FP32,
    // (d_r + d_c) X_rc off the diagonal and d_r^2 on it, so the diagonal (two
    // thirds of X's norm here) is never rounded to 16 bits.  The tile's
    // diagonal entries of X are staged in LDS behind the four bands.
    float *d_row = reinterpret_cast<float *>(lds_base) + 4 * 32 * kBandRow;
    float *d_col = d_row + kTileW;
    if constexpr (!kSplit) {
        d_row[tid] = I0 + tid < ld ? X[(int64_t)(I0 + tid) * (ld + 1)] : 0.0f;
        d_col[tid] = J0 + tid < ld ? X[(int64_t)(J0 + tid) * (ld + 1)] : 0.0f;
        __syncthreads();
    }
    double tY = 0.0, tX = 0.0;
    if (active) {
        const bool upd = alpha > 0.0f;
        float4 xo[4][4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if (upd || !kSplit) {
#pragma unroll
                for (int nn = 0; nn < 4; ++nn) {
                    const int cg = J0 + wc * 128 + nn * 32 + l32;
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const int rg0 = I0 + wr * 128 + m * 32 + g * 8 + kh * 4;
                        if constexpr (kSplit) {
                            union { uint2 u; Op h[4]; } hi, lo;
                            hi.u = *reinterpret_cast<const uint2 *>(Xop + (int64_t)cg * ld + rg0);
                            lo.u = *reinterpret_cast<const uint2 *>(Xlo + (int64_t)cg * ld + rg0);
                            xo[nn][g] = make_float4(
                                static_cast<float>(hi.h[0]) + static_cast<float>(lo.h[0]) * 0x1p-11f,
                                static_cast<float>(hi.h[1]) + static_cast<float>(lo.h[1]) * 0x1p-11f,
                                static_cast<float>(hi.h[2]) + static_cast<float>(lo.h[2]) * 0x1p-11f,
                                static_cast<float>(hi.h[3]) + static_cast<float>(lo.h[3]) * 0x1p-11f);
                        } else {
                            xo[nn][g] = *reinterpret_cast<const float4 *>(X + (int64_t)cg * ld + rg0);
                        }
                    }
                }
            }
#pragma unroll
            for (int nn = 0; nn < 4; ++nn) {
                const int cg = J0 + wc * 128 + nn * 32 + l32;
                uint2 pkg[4];                           // 16-bit X' of this lane's rows, per g (plain)
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int rg0 = I0 + wr * 128 + m * 32 + g * 8 + kh * 4;
                    const float4 x4 = xo[nn][g];
                    const float xov[4] = {x4.x, x4.y, x4.z, x4.w};
                    float xn[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        float y = acc[m][nn][4 * g + e];
                        if constexpr (!kSplit) {
                            const int rl = wr * 128 + m * 32 + g * 8 + kh * 4 + e, cl = wc * 128 + nn * 32 + l32;
                            const float dr = d_row[rl];
                            y = (diag && rl == cl) ? __builtin_fmaf(dr, dr, y)
                                                   : __builtin_fmaf(dr + d_col[cl], xov[e], y);
                        }
                        const float v = upd ? (2.0f * xov[e] - y) : y;
                        xn[e] = v;
                        band[(g * 8 + kh * 4 + e) * kBandRow + nn * 32 + l32] = v;
                        if (diag && rg0 + e == cg && cg < pd.c) {
                            tY += static_cast<double>(y);
                            tX += static_cast<double>(v);
                        }
                    }
                    if (!diag) {
                        if constexpr (!kSplit) {
                            const float4 v4 = make_float4(xn[0], xn[1], xn[2], xn[3]);
                            *reinterpret_cast<float4 *>(Xn + (int64_t)cg * ld + rg0) = v4;
                        }
                        union { Op h[4]; uint2 u; } pk, pl;
#pragma unroll
                        for (int e = 0; e < 4; ++e) pk.h[e] = static_cast<Op>(xn[e]);
                        if constexpr (kSplit) {
                            *reinterpret_cast<uint2 *>(Xnop + (int64_t)cg * ld + rg0) = pk.u;
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                pl.h[e] = static_cast<Op>((xn[e] - static_cast<float>(pk.h[e])) * 0x1p11f);
                            *reinterpret_cast<uint2 *>(Xnlo + (int64_t)cg * ld + rg0) = pl.u;
                        } else {
                            pkg[g] = pk.u;
                        }
                    }
                }
                // plain operands: the 16-bit mirrored writes as 16-byte pieces.
                // For g = 2p, 2p + 1 the lane halves swap one quadruple each, so
                // lane half 0 holds rows 16p .. 16p + 7 of column cg and half 1
                // rows 16p + 8 .. 16p + 15 (split operands keep 8-byte pieces:
                // the exchange costs them more than it saves)
                if (!kSplit && !diag) {
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        const int rgp = I0 + wr * 128 + m * 32 + 16 * p + 8 * kh;
                        const uint2 sh = kh ? pkg[2 * p] : pkg[2 * p + 1];
                        const uint2 rh = make_uint2(__shfl_xor(sh.x, 32, kWave), __shfl_xor(sh.y, 32, kWave));
                        const uint4 oh = kh ? make_uint4(rh.x, rh.y, pkg[2 * p + 1].x, pkg[2 * p + 1].y)
                                            : make_uint4(pkg[2 * p].x, pkg[2 * p].y, rh.x, rh.y);
                        *reinterpret_cast<uint4 *>(Xnop + (int64_t)cg * ld + rgp) = oh;
                    }
                }
            }
            // the band's rows back from LDS (the wave's own, written above).
            // Plain operands: lane (r4, c8) takes row 4 i + r4, columns 8 c8 ..
            // 8 c8 + 7, one 16-byte piece of the 16-bit copy.  Split operands:
            // lane (r2, c4) takes row 2 i + r2, columns 4 c4 .. 4 c4 + 3, one
            // 8-byte piece of each of hi and lo (the 16-byte form was slower
            // there).
            if constexpr (kSplit) {
                const int c4 = lane & 31, r2 = lane >> 5;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int r = 2 * i + r2;
                    const float4 v4 = *reinterpret_cast<const float4 *>(band + r * kBandRow + c4 * 4);
                    const int64_t o = (int64_t)(I0 + wr * 128 + m * 32 + r) * ld + J0 + wc * 128 + c4 * 4;
                    const float xv[4] = {v4.x, v4.y, v4.z, v4.w};
                    union { Op h[4]; uint2 u; } pk, pl;
#pragma unroll
                    for (int e = 0; e < 4; ++e) pk.h[e] = static_cast<Op>(xv[e]);
                    *reinterpret_cast<uint2 *>(Xnop + o) = pk.u;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        pl.h[e] = static_cast<Op>((xv[e] - static_cast<float>(pk.h[e])) * 0x1p11f);
                    *reinterpret_cast<uint2 *>(Xnlo + o) = pl.u;
                }
            } else {
                const int c8 = lane & 15, r4 = lane >> 4;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int r = 4 * i + r4;
                    const float4 va = *reinterpret_cast<const float4 *>(band + r * kBandRow + c8 * 8);
                    const float4 vb = *reinterpret_cast<const float4 *>(band + r * kBandRow + c8 * 8 + 4);
                    const int64_t o = (int64_t)(I0 + wr * 128 + m * 32 + r) * ld + J0 + wc * 128 + c8 * 8;
                    if (diag) {
                        *reinterpret_cast<float4 *>(Xn + o) = va;
                        *reinterpret_cast<float4 *>(Xn + o + 4) = vb;
                    }
                    const float xv[8] = {va.x, va.y, va.z, va.w, vb.x, vb.y, vb.z, vb.w};
                    union { Op h[8]; uint4 u; } pk;
                    // the operand copy's diagonal stays zero
                    const int dloc = diag ? (wr * 128 + m * 32 + r) - (wc * 128 + c8 * 8) : -1;
#pragma unroll
                    for (int e = 0; e < 8; ++e) pk.h[e] = e == dloc ? static_cast<Op>(0.0f) : static_cast<Op>(xv[e]);
                    *reinterpret_cast<uint4 *>(Xnop + o) = pk.u;
                }
            }
        }
    }
    if (diag) {
        // only the waves with wr == wc hold diagonal elements; one FP64
        // partial per 128-row half, summed in a fixed order
        tY = wave_sum(tY);
        tX = wave_sum(tX);
        if (lane == 0) { red[0][wave] = tY; red[1][wave] = tX; }
        __syncthreads();
        if (tid == 0) {
            for (int h = 0; h < (fullA ? 2 : 1); ++h) {
                const double y = red[0][h * 2 + 0] + red[0][h * 2 + 1];
                const double x = red[1][h * 2 + 0] + red[1][h * 2 + 1];
                diag_partials[2 * (td.diag_slot + h) + 0] = y;
                diag_partials[2 * (td.diag_slot + h) + 1] = x;
            }
        }
    }
}

template <typename Op, bool kSplit>
__global__ __launch_bounds__(kBlockW, 1) void k_sp2_wide(const TileDesc *__restrict__ tiles,
                                                         const PartDesc *__restrict__ parts,
                                                         float *__restrict__ buf0, float *__restrict__ buf1,
                                                         Op *__restrict__ sh0, Op *__restrict__ sh1,
                                                         const RunState *__restrict__ st_all,
                                                         double *__restrict__ diag_partials,
                                                         Op *__restrict__ lo0, Op *__restrict__ lo1, int phase) {
    __shared__ uint4 lds_w[kLdsWordsW];
    const TileDesc td = tiles[blockIdx.x];
    if (td.part < 0) return;
    const PartDesc pd = parts[td.part];
    const RunState *st = st_all + pd.sys;
    if (st->done || st->phase != phase) return;
    sp2_tile_wide<Op, kSplit>(td, pd, st->cur, static_cast<float>(st->alpha), buf0, buf1, sh0, sh1, lo0, lo1,
                              diag_partials, lds_w);
}

// After the last 16-bit product of the main phase: complete the FP32 master
// of each system's result buffer (the one refinement starts from, or the
// scatter reads).  One workgroup per chunk of 16 rows of one part.  Plain
// 16-bit products left the upper triangle outside the diagonal tiles stale:
// row r takes X[r][c] = X[c][r] for c > r, each thread one column c, reading
// the 16 rows' values of row c as 64 contiguous bytes.  Split products left
// FP32 X unwritten: X = hi + 2^-11 lo, in the operand copies' rounding.
template <typename Op, bool kSplit>
__global__ __launch_bounds__(kBlock) void k_wide_fixup(const PartDesc *__restrict__ parts,
                                                       const RowChunk *__restrict__ chunks,
                                                       float *__restrict__ buf0, float *__restrict__ buf1,
                                                       const Op *__restrict__ hi0, const Op *__restrict__ hi1,
                                                       const Op *__restrict__ lo0, const Op *__restrict__ lo1,
                                                       const RunState *__restrict__ st_all, int after_refine) {
    const RowChunk ch = chunks[blockIdx.x];
    const PartDesc pd = parts[ch.part];
    const RunState *st = st_all + pd.sys;
    if (st->status == GSP2_E_INVALID || st->status == GSP2_E_HIP) return;
    // after split refinement products: only the systems that formed them
    if (after_refine && st->n_refine == 0) return;
    const int b = st->phase == 1 ? st->cur : st->result_buf;
    float *X = (b ? buf1 : buf0) + pd.x_off;
    const int ld = pd.s_pad;
    if constexpr (kSplit) {
        const Op *H = (b ? hi1 : hi0) + pd.x_off;
        const Op *L = (b ? lo1 : lo0) + pd.x_off;
        for (int r = ch.r0; r < ch.r1; ++r) {
            const uint2 *h4 = reinterpret_cast<const uint2 *>(H + (int64_t)r * ld);
            const uint2 *l4 = reinterpret_cast<const uint2 *>(L + (int64_t)r * ld);
            float4 *x4 = reinterpret_cast<float4 *>(X + (int64_t)r * ld);
            for (int i = threadIdx.x; i < ld / 4; i += kBlock) {
                union { uint2 u; Op h[4]; } a, c;
                a.u = h4[i];
                c.u = l4[i];
                x4[i] = make_float4(static_cast<float>(a.h[0]) + static_cast<float>(c.h[0]) * 0x1p-11f,
                                    static_cast<float>(a.h[1]) + static_cast<float>(c.h[1]) * 0x1p-11f,
                                    static_cast<float>(a.h[2]) + static_cast<float>(c.h[2]) * 0x1p-11f,
                                    static_cast<float>(a.h[3]) + static_cast<float>(c.h[3]) * 0x1p-11f);
            }
        }
    } else {
        constexpr int kRows = kRowsPerChunk;    // r0 is a multiple of it
        for (int c = ch.r0 + 1 + threadIdx.x; c < ld; c += kBlock) {
            const float4 *src = reinterpret_cast<const float4 *>(X + (int64_t)c * ld + ch.r0);
            float v[kRows];
#pragma unroll
            for (int q = 0; q < kRows / 4; ++q) {
                const float4 t = src[q];
                v[4 * q] = t.x; v[4 * q + 1] = t.y; v[4 * q + 2] = t.z; v[4 * q + 3] = t.w;
            }
#pragma unroll
            for (int i = 0; i < kRows; ++i)
                if (ch.r0 + i < ch.r1 && c > ch.r0 + i) X[(int64_t)(ch.r0 + i) * ld + c] = v[i];
        }
    }
}

// Before split-FP16 refinement products that follow 16-bit main products:
// split each refining system's iterate (its FP32 master, complete after the
// main phase's fixup) into the two FP16 operand parts the split product
// reads, X = hi + 2^-11 lo with hi = fp16(X), lo = fp16(2^11 (X - hi)).  One
// workgroup per chunk of rows of one part, four entries per thread.
__global__ __launch_bounds__(kBlock) void k_split_operands(const PartDesc *__restrict__ parts,
                                                           const RowChunk *__restrict__ chunks,
                                                           const float *__restrict__ buf0,
                                                           const float *__restrict__ buf1,
                                                           _Float16 *__restrict__ hi0, _Float16 *__restrict__ hi1,
                                                           _Float16 *__restrict__ lo0, _Float16 *__restrict__ lo1,
                                                           const RunState *__restrict__ st_all) {
    const RowChunk ch = chunks[blockIdx.x];
    const PartDesc pd = parts[ch.part];
    const RunState *st = st_all + pd.sys;
    if (st->done || st->phase != 1) return;     // no refinement for this system
    const int b = st->cur;
    const float *X = (b ? buf1 : buf0) + pd.x_off;
    _Float16 *H = (b ? hi1 : hi0) + pd.x_off;
    _Float16 *L = (b ? lo1 : lo0) + pd.x_off;
    const int ld = pd.s_pad;
    for (int r = ch.r0; r < ch.r1; ++r) {
        const float4 *x4 = reinterpret_cast<const float4 *>(X + (int64_t)r * ld);
        uint2 *h4 = reinterpret_cast<uint2 *>(H + (int64_t)r * ld);
        uint2 *l4 = reinterpret_cast<uint2 *>(L + (int64_t)r * ld);
        for (int i = threadIdx.x; i < ld / 4; i += kBlock) {
            const float4 v = x4[i];
            const float x[4] = {v.x, v.y, v.z, v.w};
            union { _Float16 h[4]; uint2 u; } a, c;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                a.h[e] = static_cast<_Float16>(x[e]);
                c.h[e] = static_cast<_Float16>((x[e] - static_cast<float>(a.h[e])) * 0x1p11f);
            }
            h4[i] = a.u;
            l4[i] = c.u;
        }
    }
}

// a7 between per-product launches: reduce the product's trace partials in a
// fixed order and take the decision.  One workgroup per system, over the
// system's run of diagonal-tile slots.
__global__ __launch_bounds__(kBlock) void k_sp2_decide(const double *__restrict__ diag_partials,
                                                       const int32_t *__restrict__ sys_diag_ptr,
                                                       RunState *__restrict__ st_all, int phase) {
    RunState *st = st_all + blockIdx.x;
    if (st->done || st->phase != phase) return;
    const int d0 = sys_diag_ptr[blockIdx.x], d1 = sys_diag_ptr[blockIdx.x + 1];
    double ty = 0.0, tx = 0.0;
    for (int i = d0 + threadIdx.x; i < d1; i += kBlock) {
        ty += diag_partials[2 * i];
        tx += diag_partials[2 * i + 1];
    }
    block_sum2(ty, tx);
    if (threadIdx.x != 0) return;
    Ctl c = ctl_load(st);
    decide(c, ty, tx, st, true);
    ctl_store(st, c);
}

// ---------------------------------------------------------------------------
// a9: every product of the main phase in one persistent launch.
//
// The grid holds as many workgroups as the GPU keeps resident (CUs x
// occupancy).  For each product, workgroup b takes tiles from the queue of
// its XCD (b mod 8; the plan's tile list is eight interleaved per-XCD lists)
// through an atomic head, then steals from the other XCDs' queues.  A grid
// barrier closes the product; then every workgroup reduces the same trace
// partials in the same order and takes the same decision, so no second
// barrier is needed.  Trace partials are double-buffered by product parity:
// a workgroup can be at most one product ahead of the slowest.  Only
// workgroup 0 writes the run state.  Every wait is bounded by the device
// wall clock; on expiry a fail flag is raised, every workgroup leaves, and
// the run reports an error instead of hanging.
// ---------------------------------------------------------------------------
__device__ bool grid_barrier(PersistCtl *pc, unsigned target, long long t_end, int *ok_s) {
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        __threadfence();
        atomicAdd(&pc->arrive, 1u);
        while (__hip_atomic_load(&pc->arrive, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(&pc->fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                (long long)wall_clock64() > t_end) {
                __hip_atomic_store(&pc->fail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
        *ok_s = ok;
    }
    __syncthreads();
    return *ok_s != 0;
}

__global__ __launch_bounds__(kBlock) void k_persist_reset(PersistCtl *pc) {
    unsigned *w = reinterpret_cast<unsigned *>(pc);
    for (int i = threadIdx.x; i < (int)(sizeof(PersistCtl) / sizeof(unsigned)); i += kBlock) w[i] = 0u;
}

template <typename Op>
__global__ __launch_bounds__(kBlock, 2) void k_sp2_persistent(const TileDesc *__restrict__ tiles, int list_len,
                                                              const PartDesc *__restrict__ parts,
                                                              float *__restrict__ buf0, float *__restrict__ buf1,
                                                              Op *__restrict__ sh0, Op *__restrict__ sh1,
                                                              RunState *__restrict__ st,
                                                              double *__restrict__ partials, int n_diag,
                                                              PersistCtl *__restrict__ pc, long long timeout_ticks) {
    __shared__ uint4 lds[kLdsWords];
    __shared__ Ctl c_s;
    __shared__ int q_s, ok_s;
    if (threadIdx.x == 0) c_s = ctl_load(st);
    __syncthreads();
    if (c_s.done || c_s.phase != 0) return;     // same state for every workgroup
    const long long t_end = (long long)wall_clock64() + timeout_ticks;
    const unsigned G = gridDim.x;
    const int my_x = blockIdx.x % kXcds;
    const bool writer = blockIdx.x == 0;
    unsigned n_barriers = 0;
    while (true) {
        const int kq = c_s.n_products;          // product ordinal in this phase
        double *part_t = partials + (size_t)(kq & 1) * n_diag * 2;
        const int cur = c_s.cur;
        const float alpha = static_cast<float>(c_s.alpha);
        for (int probe = 0; probe < kXcds; ++probe) {
            const int x = (my_x + probe) % kXcds;
            while (true) {
                if (threadIdx.x == 0) q_s = (int)atomicAdd(&pc->head[kq][x], 1u);
                __syncthreads();
                const int q = q_s;
                __syncthreads();
                if (q >= list_len) break;
                const TileDesc td = tiles[(size_t)q * kXcds + x];
                if (td.part >= 0) sp2_tile<Op>(td, parts[td.part], cur, alpha, buf0, buf1, sh0, sh1, part_t, lds);
            }
        }
        ++n_barriers;
        if (!grid_barrier(pc, n_barriers * G, t_end, &ok_s)) return;
        double ty = 0.0, tx = 0.0;
        for (int i = threadIdx.x; i < n_diag; i += kBlock) {
            ty += part_t[2 * i];
            tx += part_t[2 * i + 1];
        }
        block_sum2(ty, tx);
        if (threadIdx.x == 0) {
            Ctl c = c_s;
            decide(c, ty, tx, st, writer);
            c_s = c;
        }
        __syncthreads();
        if (c_s.done || c_s.phase != 0) break;
    }
    if (writer && threadIdx.x == 0) ctl_store(st, c_s);
}

// After the persistent launch: a raised fail flag ends the run with an error.
__global__ __launch_bounds__(kBlock) void k_persist_check(const PersistCtl *__restrict__ pc,
                                                          RunState *__restrict__ st) {
    if (threadIdx.x == 0 && pc->fail != 0u) {
        st->done = 1;
        st->status = GSP2_E_HIP;
        st->main_status = GSP2_E_HIP;
    }
}

// ---------------------------------------------------------------------------
// a8: scatter.  One wave per column of P; the column's rows are the part's
// vertices in ascending global order, read from the (symmetric) row of the
// final iterate through the sorted-position map.  With `symmetrize`, a
// stored entry (i, j) whose mirror (j, i) is stored too becomes the mean of
// the two (both computed from the final iterates, so the pair gets the same
// value); an entry whose mirror the pattern does not hold is kept.
// ---------------------------------------------------------------------------
template <typename XT>
__global__ __launch_bounds__(kBlock) void k_scatter(const PartDesc *__restrict__ parts,
                                                    const int32_t *__restrict__ perm_arena,
                                                    const int32_t *__restrict__ idx_arena,
                                                    const int64_t *__restrict__ col_ptr,
                                                    const int32_t *__restrict__ col_part,
                                                    const int32_t *__restrict__ col_local, int32_t n,
                                                    const XT *__restrict__ buf0, const XT *__restrict__ buf1,
                                                    const RunState *__restrict__ st_all, XT *__restrict__ P_val,
                                                    int symmetrize) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t j = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (j >= n) return;
    const PartDesc pd = parts[col_part[j]];
    const RunState *st = st_all + pd.sys;
    if (st->status == GSP2_E_INVALID || st->status == GSP2_E_HIP) return;
    const XT *Xr = (st->result_buf ? buf1 : buf0) + pd.x_off + (int64_t)col_local[j] * pd.s_pad;
    const int32_t *perm = perm_arena + pd.perm_off;
    XT *out = P_val + col_ptr[j];
    if (!symmetrize) {
        for (int t = lane; t < pd.s; t += kWave) out[t] = Xr[perm[t]];
        return;
    }
    const int32_t *idx = idx_arena + pd.idx_off;
    for (int t = lane; t < pd.s; t += kWave) {
        const int loc = perm[t];
        const XT v = Xr[loc];
        const int32_t i = idx[loc];             // global row of this entry
        // the mirror (j, i) sits in column i, held by the part where i is core
        const PartDesc pq = parts[col_part[i]];
        const int32_t *iq = idx_arena + pq.idx_off;
        int r = find_sorted(iq, pq.c, (int32_t)j);
        if (r < 0) {
            r = find_sorted(iq + pq.c, pq.s - pq.c, (int32_t)j);
            if (r >= 0) r += pq.c;
        }
        if (r < 0) {
            out[t] = v;
        } else {
            const RunState *sq = st_all + pq.sys;
            const XT *Xq = (sq->result_buf ? buf1 : buf0) + pq.x_off;
            // P[j, i] = X_q[r][local i] = X_q[local i][r] (every iterate is symmetric)
            const XT w = Xq[(int64_t)col_local[i] * pq.s_pad + r];
            out[t] = static_cast<XT>(0.5) * (v + w);
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint of the recursion (reverse mode, FP32 products, FP64 reductions).
//
// For a fixed branch sequence, the cotangent G of X_{t+1} (kept symmetric:
// the seed is symmetrised and the step preserves symmetry) maps to the
// cotangent of X_t as GX + XG (alpha = -1) or 2G - (GX + XG) (alpha = +1).
// With G and X symmetric, tile (I,J) of GX + XG is
//     sum_k G[I,k] X[J,k] + X[I,k] G[J,k],
// two row-panel products accumulated into one tile: the forward kernel's
// data flow with the K loop run over two panel pairs (sp2_tile's kAdj).
// ---------------------------------------------------------------------------

// One forward product with the buffers and branch given explicitly (the
// backward pass replays a known sequence).
__global__ __launch_bounds__(kBlock, 2) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_sp2_fixed(const TileDesc *__restrict__ tiles,
                                                         const PartDesc *__restrict__ parts,
                                                         float *__restrict__ X_in, float *__restrict__ X_out,
                                                         float alpha, double *__restrict__ diag_partials) {
    __shared__ uint4 lds[kLdsWords];
    const TileDesc td = tiles[blockIdx.x];
    if (td.part < 0) return;
    // the skip form (same bits as the full grid), over its own tile order
    sp2_tile<float, false, true>(td, parts[td.part], 0, alpha, X_in, X_out, nullptr, nullptr, diag_partials, lds);
}

__global__ __launch_bounds__(kBlock, 2) void k_adj_step(const TileDesc *__restrict__ tiles,
                                                        const PartDesc *__restrict__ parts,
                                                        const float *__restrict__ G_in, float *__restrict__ G_out,
                                                        const float *__restrict__ X, float alpha) {
    __shared__ uint4 lds[kLdsWords];
    const TileDesc td = tiles[blockIdx.x];
    if (td.part < 0) return;
    // G_in is only read (operand and old value); the skip form, over its own tile order
    sp2_tile<float, false, true, true>(td, parts[td.part], 0, alpha, const_cast<float *>(G_in), G_out, nullptr,
                                       nullptr, nullptr, lds, const_cast<float *>(X), nullptr);
}

// Seed: part k's cotangent is dL/dP on its core columns (rows in local
// order), zero elsewhere, symmetrised.  One workgroup per row chunk.
__global__ __launch_bounds__(kBlock) void k_adj_seed(const PartDesc *__restrict__ parts,
                                                     const RowChunk *__restrict__ chunks,
                                                     const int32_t *__restrict__ idx_arena,
                                                     const int32_t *__restrict__ invperm_arena,
                                                     const int64_t *__restrict__ col_ptr,
                                                     const float *__restrict__ dLdP, float *__restrict__ G) {
    const RowChunk ch = chunks[blockIdx.x];
    const PartDesc pd = parts[ch.part];
    const int32_t *idx = idx_arena + pd.idx_off;
    const int32_t *inv = invperm_arena + pd.perm_off;
    const int ld = pd.s_pad;
    float *Gp = G + pd.x_off;
    for (int r = ch.r0; r < ch.r1; ++r) {
        for (int b = threadIdx.x; b < ld; b += kBlock) {
            float g1 = 0.0f, g2 = 0.0f;
            if (r < pd.s && b < pd.c) g1 = dLdP[col_ptr[idx[b]] + inv[r]];     // column b, row r
            if (b < pd.s && r < pd.c) g2 = dLdP[col_ptr[idx[r]] + inv[b]];     // column r, row b
            Gp[(int64_t)r * ld + b] = 0.5f * (g1 + g2);
        }
    }
}

// dL/dH_sub = -G0 / (eps_max - eps_min), accumulated over parts into H's
// stored entries (FP64 atomics: a value's summation order may vary).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_dh(const int64_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col,
                                                   const PartDesc *__restrict__ parts,
                                                   const RowChunk *__restrict__ chunks,
                                                   const int32_t *__restrict__ idx_arena,
                                                   const float *__restrict__ G0, const RunState *__restrict__ st,
                                                   double *__restrict__ dLdH) {
    __shared__ int32_t idx_s[kGatherLdsIdx];
    if (st->done) return;
    const RowChunk ch = chunks[blockIdx.x];
    const PartDesc pd = parts[ch.part];
    const int32_t *idx_g = idx_arena + pd.idx_off;
    const bool in_lds = pd.s <= kGatherLdsIdx;
    if (in_lds) {
        for (int i = threadIdx.x; i < pd.s; i += kBlock) idx_s[i] = idx_g[i];
        __syncthreads();
    }
    const int32_t *idx = in_lds ? idx_s : idx_g;
    const double inv = 1.0 / (st->eps_max - st->eps_min);
    const float *Gp = G0 + pd.x_off;
    const int ld = pd.s_pad;
    for (int r = ch.r0; r < min(ch.r1, pd.s); ++r) {
        const int64_t g = idx[r];
        for (int64_t e = row_ptr[g] + threadIdx.x; e < row_ptr[g + 1]; e += kBlock) {
            const int32_t cg = col[e];
            int q = find_sorted(idx, pd.c, cg);
            if (q < 0) {
                q = find_sorted(idx + pd.c, pd.s - pd.c, cg);
                if (q >= 0) q += pd.c;
            }
            if (q >= 0) atomicAdd(dLdH + e, -static_cast<double>(Gp[(int64_t)r * ld + q]) * inv);
        }
    }
}

// Per row chunk: sum of G0 .* X0 and of G0's diagonal (for the bound terms).
__global__ __launch_bounds__(kBlock) void k_adj_eps_partials(const PartDesc *__restrict__ parts,
                                                             const RowChunk *__restrict__ chunks,
                                                             const float *__restrict__ G0,
                                                             const float *__restrict__ X0,
                                                             double *__restrict__ out) {
    const RowChunk ch = chunks[blockIdx.x];
    const PartDesc pd = parts[ch.part];
    const int ld = pd.s_pad;
    double gx = 0.0, tr = 0.0;
    for (int r = ch.r0; r < min(ch.r1, pd.s); ++r) {
        const float *gr = G0 + pd.x_off + (int64_t)r * ld;
        const float *xr = X0 + pd.x_off + (int64_t)r * ld;
        for (int b = threadIdx.x; b < pd.s; b += kBlock) gx += (double)gr[b] * (double)xr[b];
        if (threadIdx.x == 0) tr += (double)gr[r];
    }
    block_sum2(gx, tr);
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = gx;
        out[2 * blockIdx.x + 1] = tr;
    }
}

__device__ __forceinline__ double sgn(double v) { return (v > 0.0) - (v < 0.0); }

// The Gershgorin bounds' share: dL/d eps_max = (tr G0 - <G0, X0>) / D falls
// on row i of eps_max = H_ii + sum |H_ij|, dL/d eps_min = <G0, X0> / D on row
// j of eps_min = H_jj - sum |H_jl|; off-diagonal shares are split evenly
// between H_uv and H_vu.  One workgroup.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_eps_apply(const double *__restrict__ partials, int n_chunks,
                                                          const RunState *__restrict__ st,
                                                          const int64_t *__restrict__ row_ptr,
                                                          const int32_t *__restrict__ col,
                                                          const T *__restrict__ val, double *__restrict__ dLdH,
                                                          double *__restrict__ d_eps) {
    if (st->done) return;
    double gx = 0.0, tr = 0.0;
    for (int i = threadIdx.x; i < n_chunks; i += kBlock) {
        gx += partials[2 * i];
        tr += partials[2 * i + 1];
    }
    block_sum2(gx, tr);
    if (threadIdx.x != 0) return;
    const double D = st->eps_max - st->eps_min;
    const double g_max = (tr - gx) / D, g_min = gx / D;
    d_eps[0] = g_min;
    d_eps[1] = g_max;
    const int rows[2] = {st->row_max, st->row_min};
    const double gs[2] = {g_max, -g_min};
    for (int q = 0; q < 2; ++q) {
        const int row = rows[q];
        if (row < 0) continue;
        const double g = q == 0 ? g_max : g_min;
        for (int64_t e = row_ptr[row]; e < row_ptr[row + 1]; ++e) {
            const int32_t c = col[e];
            if (c == row) {
                dLdH[e] += g;
                continue;
            }
            const double w = gs[q] * sgn(as_double(val[e]));
            dLdH[e] += 0.5 * w;
            for (int64_t f = row_ptr[c]; f < row_ptr[c + 1]; ++f)
                if (col[f] == row) { dLdH[f] += 0.5 * w; break; }
        }
    }
}

// Hand a kernel and its arguments (converted to the kernel's parameter types)
// to the recorder; the recorder copies them at launch or node creation.
template <typename... KArgs, std::size_t... I, typename... Args>
void record_impl(Recorder &rec, void (*f)(KArgs...), dim3 grid, dim3 block, std::index_sequence<I...>,
                 Args &&...args) {
    std::tuple<KArgs...> vals(std::forward<Args>(args)...);
    void *ptrs[sizeof...(KArgs) > 0 ? sizeof...(KArgs) : 1] = {static_cast<void *>(&std::get<I>(vals))...};
    rec.add_kernel(reinterpret_cast<const void *>(f), grid, block, ptrs);
}
template <typename... KArgs, typename... Args>
void record(Recorder &rec, void (*f)(KArgs...), dim3 grid, dim3 block, Args &&...args) {
    record_impl(rec, f, grid, block, std::index_sequence_for<KArgs...>{}, std::forward<Args>(args)...);
}

template <typename T>
hipError_t density_typed(const DevicePlan &dp, const gsp2_csr &H, const RunParams &rp, void *P_val,
                         Recorder &rec, const RunEvents *ev) {
    const T *hv = static_cast<const T *>(H.val);
    const dim3 blk(kBlock);
    if (ev) rec.add_event(ev->begin);
    const dim3 sys(dp.n_sys);
    record(rec, k_gershgorin<T>, dim3(dp.gersh_blocks), blk, H.row_ptr, H.col, hv, dp.n, dp.row_bounds);
    record(rec, k_run_init, sys, blk, dp.row_bounds, dp.sys_rows, dp.sys_row_ptr, rp, dp.sys_params, dp.state);
    const bool f64 = rp.precision == GSP2_PREC_FP64;
    const bool mixed = rp.precision == GSP2_PREC_FP16 || rp.precision == GSP2_PREC_BF16 ||
                       rp.precision == GSP2_PREC_FP16X3;
    const bool split = rp.precision == GSP2_PREC_FP16X3;
    uint16_t *sh0 = mixed ? static_cast<uint16_t *>(dp.shadow[0]) : nullptr;
    uint16_t *lo0 = split ? static_cast<uint16_t *>(dp.shadow_lo[0]) : nullptr;
    if (f64)
        record(rec, k_gather_x0<T, double>, dim3(dp.n_chunks), blk, H.row_ptr, H.col, hv, dp.parts, dp.chunks,
               dp.idx, dp.buf64[0], (uint16_t *)nullptr, (uint16_t *)nullptr, dp.state, dp.x0_partials);
    else
        record(rec, k_gather_x0<T, float>, dim3(dp.n_chunks), blk, H.row_ptr, H.col, hv, dp.parts, dp.chunks,
               dp.idx, dp.buf[0], sh0, lo0, dp.state, dp.x0_partials);
    record(rec, k_run_start, sys, blk, dp.x0_partials, dp.sys_chunk_ptr, dp.state);
    if (ev) rec.add_event(ev->setup_end);
    const dim3 grid(dp.n_tiles);
    float *b0 = dp.buf[0], *b1 = dp.buf[1];
    if (rp.persistent && rp.n_steps > 0) {
        // the persistent kernel keeps one system's control state and has no
        // split-operand or FP64 form: anything else is refused here too
        if (dp.n_sys != 1 || (rp.precision != GSP2_PREC_FP32 && rp.precision != GSP2_PREC_FP16 &&
                              rp.precision != GSP2_PREC_BF16))
            return hipErrorInvalidValue;
        const dim3 pg(dp.persist_grid);
        record(rec, k_persist_reset, dim3(1), blk, dp.persist);
        if (ev) rec.add_event(ev->persist_begin);
        if (rp.precision == GSP2_PREC_FP16)
            record(rec, k_sp2_persistent<_Float16>, pg, blk, dp.tiles, dp.list_len, dp.parts, b0, b1,
                   static_cast<_Float16 *>(dp.shadow[0]), static_cast<_Float16 *>(dp.shadow[1]), dp.state,
                   dp.diag_partials, dp.n_diag, dp.persist, dp.persist_timeout);
        else if (rp.precision == GSP2_PREC_BF16)
            record(rec, k_sp2_persistent<__bf16>, pg, blk, dp.tiles, dp.list_len, dp.parts, b0, b1,
                   static_cast<__bf16 *>(dp.shadow[0]), static_cast<__bf16 *>(dp.shadow[1]), dp.state,
                   dp.diag_partials, dp.n_diag, dp.persist, dp.persist_timeout);
        else
            record(rec, k_sp2_persistent<float>, pg, blk, dp.tiles, dp.list_len, dp.parts, b0, b1, (float *)nullptr,
                   (float *)nullptr, dp.state, dp.diag_partials, dp.n_diag, dp.persist, dp.persist_timeout);
        if (ev) rec.add_event(ev->persist_end);
        record(rec, k_persist_check, dim3(1), blk, dp.persist, dp.state);
    }
    _Float16 *h16[2] = {static_cast<_Float16 *>(dp.shadow[0]), static_cast<_Float16 *>(dp.shadow[1])};
    _Float16 *l16[2] = {static_cast<_Float16 *>(dp.shadow_lo[0]), static_cast<_Float16 *>(dp.shadow_lo[1])};
    __bf16 *b16[2] = {static_cast<__bf16 *>(dp.shadow[0]), static_cast<__bf16 *>(dp.shadow[1])};
    const dim3 grid_w(dp.n_tiles_w), blk_w(kBlockW);
    // the product kernel of form `form` with operands of `prec` (phase 0 or 1)
    auto product = [&](int form, int prec, int phase) {
        const bool skip = form == GSP2_KERNEL_T128_SKIP;
        const TileDesc *tl = skip ? dp.tiles_s : dp.tiles;     // the skip form's order: short tiles last
        if (prec == GSP2_PREC_FP64) {
            record(rec, skip ? k_sp2_step64<true> : k_sp2_step64<false>, grid, blk, tl, dp.parts, dp.buf64[0],
                   dp.buf64[1], dp.state, dp.diag_partials, phase);
        } else if (prec == GSP2_PREC_FP32) {
            auto k = skip ? k_sp2_step<float, false, true> : k_sp2_step<float, false, false>;
            record(rec, k, grid, blk, tl, dp.parts, b0, b1, (float *)nullptr, (float *)nullptr, dp.state,
                   dp.diag_partials, phase, (float *)nullptr, (float *)nullptr);
        } else if (form == GSP2_KERNEL_T256) {
            if (prec == GSP2_PREC_FP16)
                record(rec, k_sp2_wide<_Float16, false>, grid_w, blk_w, dp.tiles_w, dp.parts, b0, b1, h16[0],
                       h16[1], dp.state, dp.diag_partials, (_Float16 *)nullptr, (_Float16 *)nullptr, phase);
            else if (prec == GSP2_PREC_FP16X3)
                record(rec, k_sp2_wide<_Float16, true>, grid_w, blk_w, dp.tiles_w, dp.parts, b0, b1, h16[0],
                       h16[1], dp.state, dp.diag_partials, l16[0], l16[1], phase);
            else
                record(rec, k_sp2_wide<__bf16, false>, grid_w, blk_w, dp.tiles_w, dp.parts, b0, b1, b16[0],
                       b16[1], dp.state, dp.diag_partials, (__bf16 *)nullptr, (__bf16 *)nullptr, phase);
        } else if (prec == GSP2_PREC_FP16) {
            auto k = skip ? k_sp2_step<_Float16, false, true> : k_sp2_step<_Float16, false, false>;
            record(rec, k, grid, blk, tl, dp.parts, b0, b1, h16[0], h16[1], dp.state, dp.diag_partials,
                   phase, (_Float16 *)nullptr, (_Float16 *)nullptr);
        } else if (prec == GSP2_PREC_FP16X3) {
            auto k = skip ? k_sp2_step<_Float16, true, true> : k_sp2_step<_Float16, true, false>;
            record(rec, k, grid, blk, tl, dp.parts, b0, b1, h16[0], h16[1], dp.state, dp.diag_partials,
                   phase, l16[0], l16[1]);
        } else {
            auto k = skip ? k_sp2_step<__bf16, false, true> : k_sp2_step<__bf16, false, false>;
            record(rec, k, grid, blk, tl, dp.parts, b0, b1, b16[0], b16[1], dp.state, dp.diag_partials,
                   phase, (__bf16 *)nullptr, (__bf16 *)nullptr);
        }
    };
    for (int it = 0; it < (rp.persistent ? 0 : rp.n_steps); ++it) {
        if (ev) rec.add_event(ev->step[2 * it]);
        product(rp.kernel, rp.precision, 0);
        if (ev) rec.add_event(ev->step[2 * it + 1]);
        record(rec, k_sp2_decide, sys, blk, dp.diag_partials, dp.sys_diag_ptr, dp.state, 0);
    }
    // 16-bit products on 256 x 256 tiles leave the FP32 master incomplete
    if (!rp.persistent && rp.n_steps > 0 && mixed && rp.kernel == GSP2_KERNEL_T256) {
        if (rp.precision == GSP2_PREC_FP16)
            record(rec, k_wide_fixup<_Float16, false>, dim3(dp.n_chunks), blk, dp.parts, dp.chunks, b0, b1,
                   (const _Float16 *)nullptr, (const _Float16 *)nullptr, (const _Float16 *)nullptr,
                   (const _Float16 *)nullptr, dp.state, 0);
        else if (rp.precision == GSP2_PREC_BF16)
            record(rec, k_wide_fixup<__bf16, false>, dim3(dp.n_chunks), blk, dp.parts, dp.chunks, b0, b1,
                   (const __bf16 *)nullptr, (const __bf16 *)nullptr, (const __bf16 *)nullptr,
                   (const __bf16 *)nullptr, dp.state, 0);
        else if (rp.precision == GSP2_PREC_FP16X3)
            record(rec, k_wide_fixup<_Float16, true>, dim3(dp.n_chunks), blk, dp.parts, dp.chunks, b0, b1,
                   (const _Float16 *)h16[0], (const _Float16 *)h16[1], (const _Float16 *)l16[0],
                   (const _Float16 *)l16[1], dp.state, 0);
    }
    // refinement products: FP32 (FP64 in FP64 runs), or split FP16 on the
    // iterate split once into its FP16 parts
    const bool split_refine = rp.refine > 0 && rp.refine_prec == GSP2_PREC_FP16X3;
    if (split_refine)
        record(rec, k_split_operands, dim3(dp.n_chunks), blk, dp.parts, dp.chunks, (const float *)b0,
               (const float *)b1, h16[0], h16[1], l16[0], l16[1], dp.state);
    for (int r = 0; r < rp.refine; ++r) {
        const int slot = rp.n_steps + r;
        if (ev) rec.add_event(ev->step[2 * slot]);
        if (split_refine)
            product(GSP2_KERNEL_T256, GSP2_PREC_FP16X3, 1);
        else
            product(rp.kernel32, f64 ? GSP2_PREC_FP64 : GSP2_PREC_FP32, 1);
        if (ev) rec.add_event(ev->step[2 * slot + 1]);
        record(rec, k_sp2_decide, sys, blk, dp.diag_partials, dp.sys_diag_ptr, dp.state, 1);
    }
    if (split_refine)
        record(rec, k_wide_fixup<_Float16, true>, dim3(dp.n_chunks), blk, dp.parts, dp.chunks, b0, b1,
               (const _Float16 *)h16[0], (const _Float16 *)h16[1], (const _Float16 *)l16[0],
               (const _Float16 *)l16[1], dp.state, 1);
    if (ev) rec.add_event(ev->sp2_end);
    const int wpb = kBlock / kWave;
    if (f64)
        record(rec, k_scatter<double>, dim3((dp.n + wpb - 1) / wpb), blk, dp.parts, dp.perm, dp.idx, dp.col_ptr,
               dp.col_part, dp.col_local, dp.n, (const double *)dp.buf64[0], (const double *)dp.buf64[1], dp.state,
               static_cast<double *>(P_val), rp.symmetrize);
    else
        record(rec, k_scatter<float>, dim3((dp.n + wpb - 1) / wpb), blk, dp.parts, dp.perm, dp.idx, dp.col_ptr,
               dp.col_part, dp.col_local, dp.n, (const float *)dp.buf[0], (const float *)dp.buf[1], dp.state,
               static_cast<float *>(P_val), rp.symmetrize);
    if (ev) rec.add_event(ev->end);
    return rec.err;
}

template <typename T>
hipError_t backward_typed(const DevicePlan &dp, const gsp2_csr &H, const RunParams &rp, const int8_t *alphas,
                          int n, const float *dLdP, double *dLdH, const BackwardBuffers &bb, hipStream_t s) {
    Recorder rec;
    rec.stream = s;
    const T *hv = static_cast<const T *>(H.val);
    const dim3 blk(kBlock), grid(dp.n_tiles), chunks(dp.n_chunks);
    record(rec, k_gershgorin<T>, dim3(dp.gersh_blocks), blk, H.row_ptr, H.col, hv, dp.n, dp.row_bounds);
    record(rec, k_run_init, dim3(dp.n_sys), blk, dp.row_bounds, dp.sys_rows, dp.sys_row_ptr, rp, dp.sys_params,
           dp.state);
    record(rec, k_gather_x0<T, float>, chunks, blk, H.row_ptr, H.col, hv, dp.parts, dp.chunks, dp.idx, bb.ckpt[0],
           (uint16_t *)nullptr, (uint16_t *)nullptr, dp.state, dp.x0_partials);
    const int k = bb.seg;
    const int nseg = n > 0 ? (n + k - 1) / k : 1;
    // forward replay, keeping X_{seg k}
    float *cur = bb.ckpt[0];
    for (int t = 0; t + 1 <= (nseg - 1) * k; ++t) {
        float *out = ((t + 1) % k == 0) ? bb.ckpt[(t + 1) / k] : (cur == dp.buf[0] ? dp.buf[1] : dp.buf[0]);
        record(rec, k_sp2_fixed, grid, blk, dp.tiles_s, dp.parts, cur, out, (float)alphas[t], dp.diag_partials);
        cur = out;
    }
    // seed and reverse sweep, segment by segment from the last
    float *g_cur = bb.g[0], *g_oth = bb.g[1];
    record(rec, k_adj_seed, chunks, blk, dp.parts, dp.chunks, dp.idx, dp.invperm, dp.col_ptr, dLdP, g_cur);
    for (int seg = nseg - 1; seg >= 0 && n > 0; --seg) {
        const int t0 = seg * k, t1 = (t0 + k < n) ? t0 + k : n;
        for (int i = 1; i < t1 - t0; ++i) {
            float *in = (i == 1) ? bb.ckpt[seg] : bb.slot[i - 2];
            record(rec, k_sp2_fixed, grid, blk, dp.tiles_s, dp.parts, in, bb.slot[i - 1], (float)alphas[t0 + i - 1],
                   dp.diag_partials);
        }
        for (int t = t1 - 1; t >= t0; --t) {
            const float *X = (t == t0) ? bb.ckpt[seg] : bb.slot[t - t0 - 1];
            record(rec, k_adj_step, grid, blk, dp.tiles_s, dp.parts, (const float *)g_cur, g_oth, X, (float)alphas[t]);
            float *tmp = g_cur; g_cur = g_oth; g_oth = tmp;
        }
    }
    if (rec.err != hipSuccess) return rec.err;
    hipError_t e = hipMemsetAsync(dLdH, 0, sizeof(double) * (size_t)H.nnz, s);
    if (e != hipSuccess) return e;
    record(rec, k_adj_dh<T>, chunks, blk, H.row_ptr, H.col, dp.parts, dp.chunks, dp.idx, (const float *)g_cur,
           (const RunState *)dp.state, dLdH);
    record(rec, k_adj_eps_partials, chunks, blk, dp.parts, dp.chunks, (const float *)g_cur,
           (const float *)bb.ckpt[0], bb.eps_partials);
    record(rec, k_adj_eps_apply<T>, dim3(1), blk, (const double *)bb.eps_partials, dp.n_chunks,
           (const RunState *)dp.state, H.row_ptr, H.col, hv, dLdH, bb.d_eps);
    return rec.err;
}

}  // namespace

hipError_t launch_backward(const DevicePlan &dp, const gsp2_csr &H, const RunParams &rp, const int8_t *alphas,
                           int n, const float *dLdP, double *dLdH, const BackwardBuffers &bb, hipStream_t s) {
    if (H.dtype == GSP2_F64) return backward_typed<double>(dp, H, rp, alphas, n, dLdP, dLdH, bb, s);
    return backward_typed<float>(dp, H, rp, alphas, n, dLdP, dLdH, bb, s);
}

hipError_t persistent_grid(int precision, int *grid) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (precision == GSP2_PREC_FP16)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sp2_persistent<_Float16>, kBlock, 0);
    else if (precision == GSP2_PREC_BF16)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sp2_persistent<__bf16>, kBlock, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sp2_persistent<float>, kBlock, 0);
    if (e != hipSuccess) return e;
    *grid = cus * per_cu;
    return hipSuccess;
}

hipError_t launch_threshold_count(const gsp2_csr &P, double tau, int32_t *counts, hipStream_t s) {
    const int wpb = kBlock / kWave;
    const dim3 grid((P.n + wpb - 1) / wpb);
    if (P.dtype == GSP2_F64)
        hipLaunchKernelGGL(k_threshold_count<double>, grid, dim3(kBlock), 0, s, P.row_ptr, P.col,
                           static_cast<const double *>(P.val), P.n, tau, counts);
    else
        hipLaunchKernelGGL(k_threshold_count<float>, grid, dim3(kBlock), 0, s, P.row_ptr, P.col,
                           static_cast<const float *>(P.val), P.n, tau, counts);
    return hipGetLastError();
}

hipError_t launch_threshold_fill(const gsp2_csr &P, double tau, const int64_t *out_ptr, int32_t *out_col,
                                 hipStream_t s) {
    const int wpb = kBlock / kWave;
    const dim3 grid((P.n + wpb - 1) / wpb);
    if (P.dtype == GSP2_F64)
        hipLaunchKernelGGL(k_threshold_fill<double>, grid, dim3(kBlock), 0, s, P.row_ptr, P.col,
                           static_cast<const double *>(P.val), P.n, tau, out_ptr, out_col);
    else
        hipLaunchKernelGGL(k_threshold_fill<float>, grid, dim3(kBlock), 0, s, P.row_ptr, P.col,
                           static_cast<const float *>(P.val), P.n, tau, out_ptr, out_col);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Matrix-core rate probe: back-to-back MFMAs of the product kernels' shape
// (32 x 32 output blocks) on eight independent accumulators per wave, so
// the matrix pipe never waits on a result; two waves per SIMD on every CU.
// What the products reach is stated against this measured rate as well as
// against the published peak.  The sums go to `out` so no MFMA is removed.
// ---------------------------------------------------------------------------
constexpr int kProbeAcc = 8;

static_assert(kProbeThreads == kBlock, "probe workgroups are kBlock threads");

template <typename Op>
__global__ __launch_bounds__(kBlock) void k_mfma_probe(int n_iter, float *__restrict__ out) {
    v16f acc[kProbeAcc];
#pragma unroll
    for (int j = 0; j < kProbeAcc; ++j)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[j][i] = 0.0f;
    const float x = 1e-3f * static_cast<float>(threadIdx.x & 7);
    uint4 a, b;
    {
        union { Op h[16 / sizeof(Op)]; uint4 u; } ua, ub;
#pragma unroll
        for (int e = 0; e < static_cast<int>(16 / sizeof(Op)); ++e) {
            ua.h[e] = static_cast<Op>(x + 1e-4f * e);
            ub.h[e] = static_cast<Op>(x - 1e-4f * e);
        }
        a = ua.u;
        b = ub.u;
    }
    for (int it = 0; it < n_iter; ++it) {
#pragma unroll
        for (int j = 0; j < kProbeAcc; ++j) acc[j] = mfma_chunk_q(a, b, acc[j], Op{});
    }
    float t = 0.0f;
#pragma unroll
    for (int j = 0; j < kProbeAcc; ++j)
#pragma unroll
        for (int i = 0; i < 16; ++i) t += acc[j][i];
    out[blockIdx.x * kBlock + threadIdx.x] = t;
}

hipError_t probe_mfma(int precision, int n_iter, int n_blocks, float *out, hipStream_t s, int64_t *flops) {
    // flops of one mfma_chunk_q call: four 32x32x2 FP32 MFMAs (k = 8 in all),
    // or one 32x32x16 16-bit MFMA
    const int64_t per_call = 2LL * 32 * 32 * (precision == GSP2_PREC_FP32 ? 8 : 16);
    *flops = per_call * kProbeAcc * (int64_t)n_iter * n_blocks * (kBlock / kWave);
    if (precision == GSP2_PREC_FP32)
        hipLaunchKernelGGL(k_mfma_probe<float>, dim3(n_blocks), dim3(kBlock), 0, s, n_iter, out);
    else if (precision == GSP2_PREC_BF16)
        hipLaunchKernelGGL(k_mfma_probe<__bf16>, dim3(n_blocks), dim3(kBlock), 0, s, n_iter, out);
    else
        hipLaunchKernelGGL(k_mfma_probe<_Float16>, dim3(n_blocks), dim3(kBlock), 0, s, n_iter, out);
    return hipGetLastError();
}

hipError_t launch_density(const DevicePlan &dp, const gsp2_csr &H, const RunParams &rp, void *P_val,
                          Recorder &rec, const RunEvents *ev) {
    if (H.dtype == GSP2_F64) return density_typed<double>(dp, H, rp, P_val, rec, ev);
    return density_typed<float>(dp, H, rp, P_val, rec, ev);
}

// ---------------------------------------------------------------------------
// Static device scratch of gsp2_density_noalloc: the per-run buffers of a
// density matrix (run state, per-system parameters, trace partials,
// Gershgorin discs and the iterates) live in this file-scope array instead
// of memory the library allocates, for callers that cannot allocate.  Every
// GPU the library runs on holds its own copy until the process ends.  In
// host code the array's name is only a stand-in: its device address on the
// current device comes from hipGetSymbolAddress, looked up once per device
// and kept.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(void **ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace gsp2
