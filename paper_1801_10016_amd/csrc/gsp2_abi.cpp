// C ABI of libgsp2.so: plan construction (graph threshold on the GPU, host
// core/halo planning, device workspace) and density-matrix runs captured
// once into a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "gsp2.h"
#include "gsp2_internal.hpp"

using namespace gsp2;

namespace {

thread_local std::string g_last_error;

struct Failure {
    gsp2_status status;
    std::string msg;
};

[[noreturn]] void fail(gsp2_status s, const std::string &m) { throw Failure{s, m}; }

void check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) fail(GSP2_E_OOM, std::string(what) + ": out of device memory");
    fail(GSP2_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename F>
gsp2_status guarded(F &&f) {
    try {
        g_last_error.clear();
        f();
        return GSP2_OK;
    } catch (const Failure &x) {
        g_last_error = x.msg;
        return x.status;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return GSP2_E_OOM;
    } catch (const std::exception &x) {
        g_last_error = x.what();
        return GSP2_E_INVALID;
    } catch (...) {
        g_last_error = "unknown failure";
        return GSP2_E_INVALID;
    }
}

template <typename T>
T *dev_alloc(size_t count, const char *what, int64_t &total) {
    if (count == 0) count = 1;
    void *p = nullptr;
    check_hip(hipMalloc(&p, count * sizeof(T)), what);
    total += (int64_t)(count * sizeof(T));
    return static_cast<T *>(p);
}

template <typename T>
void upload(T *dst, const std::vector<T> &src, hipStream_t s, const char *what) {
    if (src.empty()) return;
    check_hip(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s), what);
}

// Checks of a host graph (directed CSR) and a partition of its vertices;
// returns the core count of every part.
std::vector<int32_t> check_graph_and_parts(int32_t n, const int64_t *adj_ptr, const int32_t *adj_col,
                                           const int32_t *part, int32_t n_parts) {
    if (n < 1) fail(GSP2_E_INVALID, "n must be >= 1");
    if (n_parts < 1) fail(GSP2_E_INVALID, "n_parts must be >= 1");
    if (!adj_ptr || !part) fail(GSP2_E_INVALID, "null pointer");
    const int64_t nnz = adj_ptr[n];
    if (adj_ptr[0] != 0 || nnz < 0) fail(GSP2_E_INVALID, "bad adjacency row pointer");
    if (nnz > 0 && !adj_col) fail(GSP2_E_INVALID, "null adjacency columns");
    for (int32_t v = 0; v < n; ++v)
        if (adj_ptr[v + 1] < adj_ptr[v]) fail(GSP2_E_INVALID, "adjacency row pointer not monotone");
    for (int64_t e = 0; e < nnz; ++e)
        if (adj_col[e] < 0 || adj_col[e] >= n) fail(GSP2_E_INVALID, "adjacency column out of range");
    std::vector<int32_t> core_count(n_parts, 0);
    for (int32_t v = 0; v < n; ++v) {
        if (part[v] < 0 || part[v] >= n_parts)
            fail(GSP2_E_INVALID, "part id out of range at vertex " + std::to_string(v));
        core_count[part[v]]++;
    }
    for (int32_t k = 0; k < n_parts; ++k)
        if (core_count[k] == 0) fail(GSP2_E_INVALID, "part " + std::to_string(k) + " is empty");
    return core_count;
}

// Core and one-hop halo of every part (host).  adj: directed CSR; the union
// of both orientations is the undirected graph; self loops ignored.
void plan_core_halo(int32_t n, const int64_t *adj_ptr, const int32_t *adj_col, const int32_t *part,
                    int32_t n_parts, std::vector<int64_t> &sub_ptr, std::vector<int32_t> &sub_idx,
                    std::vector<int32_t> &core_count) {
    core_count = check_graph_and_parts(n, adj_ptr, adj_col, part, n_parts);
    const int64_t nnz = adj_ptr[n];
    // cores, ascending
    std::vector<int64_t> core_ptr(n_parts + 1, 0);
    for (int32_t k = 0; k < n_parts; ++k) core_ptr[k + 1] = core_ptr[k] + core_count[k];
    std::vector<int32_t> core_list(n);
    {
        std::vector<int64_t> fill(core_ptr.begin(), core_ptr.end() - 1);
        for (int32_t v = 0; v < n; ++v) core_list[fill[part[v]]++] = v;
    }
    // transpose, for in-neighbours
    std::vector<int64_t> tr_ptr(n + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) tr_ptr[adj_col[e] + 1]++;
    for (int32_t v = 0; v < n; ++v) tr_ptr[v + 1] += tr_ptr[v];
    std::vector<int32_t> tr_col(nnz);
    {
        std::vector<int64_t> fill(tr_ptr.begin(), tr_ptr.end() - 1);
        for (int32_t u = 0; u < n; ++u)
            for (int64_t e = adj_ptr[u]; e < adj_ptr[u + 1]; ++e) tr_col[fill[adj_col[e]]++] = u;
    }
    std::vector<int32_t> stamp(n, -1);
    std::vector<int32_t> halo;
    sub_ptr.assign(n_parts + 1, 0);
    sub_idx.clear();
    sub_idx.reserve(n);
    for (int32_t k = 0; k < n_parts; ++k) {
        const int32_t *core = core_list.data() + core_ptr[k];
        const int32_t c = core_count[k];
        for (int32_t i = 0; i < c; ++i) stamp[core[i]] = k;
        halo.clear();
        for (int32_t i = 0; i < c; ++i) {
            const int32_t u = core[i];
            for (int64_t e = adj_ptr[u]; e < adj_ptr[u + 1]; ++e) {
                const int32_t w = adj_col[e];
                if (stamp[w] != k) { stamp[w] = k; halo.push_back(w); }
            }
            for (int64_t e = tr_ptr[u]; e < tr_ptr[u + 1]; ++e) {
                const int32_t w = tr_col[e];
                if (stamp[w] != k) { stamp[w] = k; halo.push_back(w); }
            }
        }
        std::sort(halo.begin(), halo.end());
        sub_idx.insert(sub_idx.end(), core, core + c);
        sub_idx.insert(sub_idx.end(), halo.begin(), halo.end());
        sub_ptr[k + 1] = (int64_t)sub_idx.size();
    }
}

struct GraphKey {
    const void *h_ptr = nullptr, *h_col = nullptr, *h_val = nullptr;
    int64_t h_nnz = -1;
    int32_t h_dtype = -1;
    void *p_val = nullptr;
    RunParams rp{};
    bool timing = false;
    bool operator==(const GraphKey &o) const {
        return h_ptr == o.h_ptr && h_col == o.h_col && h_val == o.h_val && h_nnz == o.h_nnz &&
               h_dtype == o.h_dtype && p_val == o.p_val && timing == o.timing &&
               std::memcmp(&rp, &o.rp, sizeof(rp)) == 0;
    }
};

}  // namespace

struct gsp2_plan_s {
    int32_t n = 0, n_parts = 0, tile = kTile;
    int32_t tile16_fixed = 0;             // plan option: 0 = tuned or default
    int32_t kernel_tuned[5] = {0, 0, 0, 0, 0};   // gsp2_plan_tune's gsp2_kernel per precision, 0 = none
    int32_t n_sys = 1;
    std::vector<int32_t> part_system;     // system of every part
    std::vector<int32_t> sys_size;        // vertices of every system
    SysParams *h_sys = nullptr;           // pinned staging of the per-system parameters
    hipEvent_t sys_uploaded = nullptr;    // recorded after each upload from h_sys
    bool sys_upload_pending = false;
    hipStream_t stream = nullptr;
    int64_t nnz_graph = 0;
    double plan_ms = 0.0;
    std::vector<int32_t> part;
    std::vector<int64_t> adj_ptr;         // G_tau as built (directed, host)
    std::vector<int32_t> adj_col;
    std::vector<int64_t> sub_ptr;
    std::vector<int32_t> sub_idx, core_count;
    std::vector<PartDesc> desc;
    std::vector<TileDesc> tiles, tiles_s, tiles_w;
    std::vector<RowChunk> chunks;
    std::vector<int32_t> perm;
    std::vector<int64_t> col_ptr;
    std::vector<int32_t> col_part, col_local;
    int32_t n_diag = 0;
    int64_t arena_floats = 0;
    int64_t workspace_bytes = 0;
    DevicePlan dp{};
    std::vector<void *> dev_ptrs;
    RunState *h_state = nullptr;      // pinned copy for run_info
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    GraphKey key;
    bool have_graph = false;
    RunParams last_rp{};
    bool ran = false;
    bool last_timed = false;
    RunEvents ev{};
    bool have_events = false;

    void make_events() {
        if (have_events) return;
        check_hip(hipEventCreate(&ev.begin), "event");
        check_hip(hipEventCreate(&ev.setup_end), "event");
        check_hip(hipEventCreate(&ev.sp2_end), "event");
        check_hip(hipEventCreate(&ev.end), "event");
        check_hip(hipEventCreate(&ev.persist_begin), "event");
        check_hip(hipEventCreate(&ev.persist_end), "event");
        for (auto &x : ev.step) check_hip(hipEventCreate(&x), "event");
        have_events = true;
    }

    ~gsp2_plan_s() {
        if (stream) (void)hipStreamSynchronize(stream); else (void)hipDeviceSynchronize();
        if (have_events) {
            (void)hipEventDestroy(ev.begin); (void)hipEventDestroy(ev.setup_end);
            (void)hipEventDestroy(ev.sp2_end); (void)hipEventDestroy(ev.end);
            (void)hipEventDestroy(ev.persist_begin); (void)hipEventDestroy(ev.persist_end);
            for (auto &x : ev.step) (void)hipEventDestroy(x);
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (void *p : dev_ptrs) (void)hipFree(p);
        if (h_state) (void)hipHostFree(h_state);
        if (h_sys) (void)hipHostFree(h_sys);
        if (sys_uploaded) (void)hipEventDestroy(sys_uploaded);
    }
    // Copy h_sys to the device in stream order.  The staging buffer is
    // rewritten only after the previous copy from it has completed.
    void wait_sys_staging() {
        if (sys_upload_pending) check_hip(hipEventSynchronize(sys_uploaded), "parameter upload");
        sys_upload_pending = false;
    }
    void upload_sys() {
        check_hip(hipMemcpyAsync(dp.sys_params, h_sys, sizeof(SysParams) * (size_t)n_sys, hipMemcpyHostToDevice,
                                 stream), "upload system parameters");
        check_hip(hipEventRecord(sys_uploaded, stream), "parameter upload");
        sys_upload_pending = true;
    }
    template <typename T>
    T *alloc(size_t count, const char *what) {
        T *p = dev_alloc<T>(count, what, workspace_bytes);
        dev_ptrs.push_back(p);
        return p;
    }
};

extern "C" {

const char *gsp2_status_string(gsp2_status s) {
    switch (s) {
        case GSP2_OK: return "GSP2_OK";
        case GSP2_E_INVALID: return "GSP2_E_INVALID";
        case GSP2_E_HIP: return "GSP2_E_HIP";
        case GSP2_E_OOM: return "GSP2_E_OOM";
        case GSP2_E_NOT_CONVERGED: return "GSP2_E_NOT_CONVERGED";
        case GSP2_E_WRONG_TRACE: return "GSP2_E_WRONG_TRACE";
        case GSP2_E_UNSUPPORTED: return "GSP2_E_UNSUPPORTED";
    }
    return "GSP2_UNKNOWN";
}

const char *gsp2_last_error(void) { return g_last_error.c_str(); }

gsp2_status gsp2_run_options_default(gsp2_run_options *opt) {
    return guarded([&] {
        if (!opt) fail(GSP2_E_INVALID, "null options");
        opt->max_iter = 60;
        opt->alpha_mode = GSP2_ALPHA_TRACE;
        opt->alpha_seq = nullptr;
        opt->n_alpha = 0;
        opt->stop_rule = 1;
        opt->trace_tol = 0.5;
        opt->timing = 0;
        opt->precision = GSP2_PREC_FP32;
        opt->refine = 0;
        opt->persistent = 0;
        opt->n_occ_system = nullptr;
        opt->alpha_seq_system = nullptr;
        opt->n_alpha_system = nullptr;
        opt->symmetrize = 0;
        opt->kernel = GSP2_KERNEL_AUTO;
        opt->refine_precision = GSP2_PREC_FP32;
        opt->pad2_ = 0;
    });
}

gsp2_status gsp2_core_halo_host(int32_t n, const int64_t *adj_ptr, const int32_t *adj_col, const int32_t *part,
                                int32_t n_parts, int64_t *sub_ptr, int32_t *sub_idx, int32_t *core_count) {
    return guarded([&] {
        if (!sub_ptr) fail(GSP2_E_INVALID, "null sub_ptr");
        std::vector<int64_t> sp;
        std::vector<int32_t> si, cc;
        plan_core_halo(n, adj_ptr, adj_col, part, n_parts, sp, si, cc);
        std::copy(sp.begin(), sp.end(), sub_ptr);
        if (sub_idx) std::copy(si.begin(), si.end(), sub_idx);
        if (core_count) std::copy(cc.begin(), cc.end(), core_count);
    });
}

gsp2_status gsp2_plan_create(const gsp2_csr *P_prev, double tau, const int32_t *part, int32_t n_parts,
                             const gsp2_plan_options *opt, void *stream, gsp2_plan *out) {
    if (out) *out = nullptr;
    gsp2_plan_s *plan = nullptr;
    const gsp2_status st = guarded([&] {
        const auto t0 = std::chrono::steady_clock::now();
        if (!out) fail(GSP2_E_INVALID, "null output handle");
        if (!P_prev) fail(GSP2_E_INVALID, "null P_prev");
        if (!part) fail(GSP2_E_INVALID, "null part");
        if (P_prev->n < 1) fail(GSP2_E_INVALID, "P_prev.n must be >= 1");
        if (P_prev->nnz < 0) fail(GSP2_E_INVALID, "P_prev.nnz must be >= 0");
        if (!P_prev->row_ptr || (P_prev->nnz > 0 && (!P_prev->col || !P_prev->val)))
            fail(GSP2_E_INVALID, "null P_prev array");
        if (P_prev->dtype != GSP2_F32 && P_prev->dtype != GSP2_F64) fail(GSP2_E_INVALID, "bad P_prev.dtype");
        if (!(tau >= 0.0) || !std::isfinite(tau)) fail(GSP2_E_INVALID, "tau must be finite and >= 0");
        if (n_parts < 1 || n_parts > P_prev->n) fail(GSP2_E_INVALID, "need 1 <= n_parts <= n");
        if (opt && opt->tile != 0 && opt->tile != kTile) fail(GSP2_E_UNSUPPORTED, "tile must be 0 or 128");
        if (opt && opt->tile16 != 0 && opt->tile16 != kTile && opt->tile16 != kTileWide)
            fail(GSP2_E_INVALID, "tile16 must be 0, 128 or 256");
        const int32_t n_sys = (opt && opt->n_systems > 1) ? opt->n_systems : 1;
        if (opt && opt->n_systems < 0) fail(GSP2_E_INVALID, "n_systems must be >= 0");
        if (n_sys > n_parts) fail(GSP2_E_INVALID, "more systems than parts");
        if (n_sys > 1 && !opt->part_system) fail(GSP2_E_INVALID, "null part_system for a batched plan");
        plan = new gsp2_plan_s();
        plan->n = P_prev->n;
        plan->n_parts = n_parts;
        plan->n_sys = n_sys;
        plan->tile16_fixed = opt ? opt->tile16 : 0;
        plan->stream = static_cast<hipStream_t>(stream);
        hipStream_t s = plan->stream;
        const int32_t n = plan->n;
        plan->part.assign(part, part + n);
        plan->part_system.assign(n_parts, 0);
        if (n_sys > 1) {
            std::vector<int32_t> used(n_sys, 0);
            for (int32_t k = 0; k < n_parts; ++k) {
                const int32_t y = opt->part_system[k];
                if (y < 0 || y >= n_sys) fail(GSP2_E_INVALID, "part_system out of range at part " + std::to_string(k));
                plan->part_system[k] = y;
                used[y] = 1;
            }
            for (int32_t y = 0; y < n_sys; ++y)
                if (!used[y]) fail(GSP2_E_INVALID, "system " + std::to_string(y) + " has no part");
        }

        // a1: threshold on the GPU, then bring the directed adjacency home
        int64_t tmp_bytes = 0;
        int32_t *d_counts = dev_alloc<int32_t>(n, "threshold counts", tmp_bytes);
        std::vector<int32_t> counts(n);
        std::vector<int64_t> adj_ptr(n + 1, 0);
        std::vector<int32_t> adj_col;
        int64_t *d_adj_ptr = nullptr;
        int32_t *d_adj_col = nullptr;
        try {
            if (P_prev->nnz > 0) {
                check_hip(launch_threshold_count(*P_prev, tau, d_counts, s), "threshold count");
                check_hip(hipMemcpyAsync(counts.data(), d_counts, n * sizeof(int32_t), hipMemcpyDeviceToHost, s),
                          "copy counts");
                check_hip(hipStreamSynchronize(s), "threshold count");
            } else {
                std::fill(counts.begin(), counts.end(), 0);
            }
            for (int32_t v = 0; v < n; ++v) adj_ptr[v + 1] = adj_ptr[v] + counts[v];
            const int64_t nnz_adj = adj_ptr[n];
            adj_col.resize(nnz_adj);
            if (nnz_adj > 0) {
                d_adj_ptr = dev_alloc<int64_t>(n + 1, "adjacency", tmp_bytes);
                d_adj_col = dev_alloc<int32_t>(nnz_adj, "adjacency", tmp_bytes);
                check_hip(hipMemcpyAsync(d_adj_ptr, adj_ptr.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s),
                          "upload adjacency pointer");
                check_hip(launch_threshold_fill(*P_prev, tau, d_adj_ptr, d_adj_col, s), "threshold fill");
                check_hip(hipMemcpyAsync(adj_col.data(), d_adj_col, nnz_adj * sizeof(int32_t), hipMemcpyDeviceToHost, s),
                          "copy adjacency");
                check_hip(hipStreamSynchronize(s), "threshold fill");
            }
        } catch (...) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(d_counts); (void)hipFree(d_adj_ptr); (void)hipFree(d_adj_col);
            throw;
        }
        (void)hipFree(d_counts); (void)hipFree(d_adj_ptr); (void)hipFree(d_adj_col);

        // a3: cores and halos (host)
        plan_core_halo(n, adj_ptr.data(), adj_col.data(), part, n_parts, plan->sub_ptr, plan->sub_idx,
                       plan->core_count);
        if (n_sys > 1) {
            // systems are independent: no edge of the graph may join two of them
            for (int32_t v = 0; v < n; ++v) {
                const int32_t yv = plan->part_system[part[v]];
                for (int64_t e = adj_ptr[v]; e < adj_ptr[v + 1]; ++e) {
                    const int32_t w = adj_col[e];
                    if (plan->part_system[part[w]] != yv)
                        fail(GSP2_E_INVALID, "graph edge " + std::to_string(v) + "-" + std::to_string(w) +
                                                 " joins systems " + std::to_string(yv) + " and " +
                                                 std::to_string(plan->part_system[part[w]]));
                }
            }
        }
        plan->nnz_graph = (int64_t)adj_col.size();
        plan->adj_ptr.swap(adj_ptr);
        plan->adj_col.swap(adj_col);

        // descriptors, LPT tile list, gather chunks, P pattern
        const int T = kTile;
        plan->desc.resize(n_parts);
        int64_t xoff = 0;
        int32_t max_s_pad = 0;
        for (int32_t k = 0; k < n_parts; ++k) {
            PartDesc d{};
            d.s = (int32_t)(plan->sub_ptr[k + 1] - plan->sub_ptr[k]);
            d.c = plan->core_count[k];
            d.s_pad = ((d.s + T - 1) / T) * T;
            d.idx_off = (int32_t)plan->sub_ptr[k];
            d.perm_off = (int32_t)plan->sub_ptr[k];
            d.x_off = xoff;
            d.sys = plan->part_system[k];
            xoff += (int64_t)d.s_pad * d.s_pad;
            max_s_pad = std::max(max_s_pad, d.s_pad);
            plan->desc[k] = d;
        }
        plan->arena_floats = xoff;
        // Tile order.  A workgroup b of a launch runs on XCD b mod kXcds, so
        // work is dealt to XCDs by LPT and each XCD's list walks its parts in
        // kTileBlock x kTileBlock blocks of tiles: the workgroups resident on
        // one XCD then share a few row and column panels in that XCD's L2.
        // The unit dealt is a whole part, or, for a part holding more than
        // half an XCD's share of the work (one dense block, a few large parts),
        // each of its blocks, so that no XCD idles while one carries a large
        // part.  Grid index b takes entry b / kXcds of XCD (b mod kXcds)'s
        // list; short lists are padded with empty tiles.
        constexpr int kXcds = 8;
        constexpr int kTileBlock = 8;                  // 128-tiles per block edge
        constexpr int kBlockRows = kTileBlock * T;     // rows per block edge (4 256-tiles as well)
        std::vector<int32_t> order(n_parts);
        std::iota(order.begin(), order.end(), 0);
        auto work = [&](int32_t k) {
            const double nt = plan->desc[k].s_pad / T;
            return nt * (nt + 1) / 2 * plan->desc[k].s_pad;
        };
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return work(a) > work(b); });
        std::vector<int32_t> rank(n_parts);
        double total_work = 0.0;
        for (int32_t i = 0; i < n_parts; ++i) {
            rank[order[i]] = i;
            total_work += work(order[i]);
        }
        struct Unit { int32_t k, bi, bj; double w; };   // bi < 0: the whole part
        std::vector<Unit> units;
        for (int32_t k : order) {
            if (work(k) <= 0.5 * total_work / kXcds) {
                units.push_back(Unit{k, -1, -1, work(k)});
                continue;
            }
            const int nt = plan->desc[k].s_pad / T;
            for (int bi = 0; bi < nt; bi += kTileBlock)
                for (int bj = bi; bj < nt; bj += kTileBlock) {
                    double tiles = 0.0;
                    for (int ti = bi; ti < std::min(bi + kTileBlock, nt); ++ti)
                        tiles += std::min(bj + kTileBlock, nt) - std::max(ti, bj);
                    units.push_back(Unit{k, bi / kTileBlock, bj / kTileBlock, tiles * plan->desc[k].s_pad});
                }
        }
        std::stable_sort(units.begin(), units.end(), [](const Unit &a, const Unit &b) { return a.w > b.w; });
        std::vector<double> load(kXcds, 0.0);
        std::vector<std::vector<Unit>> xcd_units(kXcds);
        for (const Unit &u : units) {
            const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            load[x] += u.w;
            xcd_units[x].push_back(u);
        }
        // within an XCD: parts in LPT order, a split part's blocks row by row
        for (auto &l : xcd_units)
            std::stable_sort(l.begin(), l.end(), [&](const Unit &a, const Unit &b) {
                if (rank[a.k] != rank[b.k]) return rank[a.k] < rank[b.k];
                return a.bi != b.bi ? a.bi < b.bi : a.bj < b.bj;
            });
        // Trace partials of the diagonal tiles: slots grouped by system, then
        // by part and tile row, so a system's traces are reduced in an order
        // that does not depend on the other systems of the batch.
        std::vector<std::vector<int32_t>> sys_parts(n_sys);
        for (int32_t k = 0; k < n_parts; ++k) sys_parts[plan->part_system[k]].push_back(k);
        std::vector<int32_t> diag_base(n_parts, 0);
        std::vector<int32_t> sys_diag_ptr(n_sys + 1, 0), sys_chunk_ptr(n_sys + 1, 0);
        int32_t slot = 0;
        for (int32_t y = 0; y < n_sys; ++y) {
            for (int32_t k : sys_parts[y]) {
                diag_base[k] = slot;
                slot += plan->desc[k].s_pad / T;
            }
            sys_diag_ptr[y + 1] = slot;
        }
        // the tiles of one unit at tile edge `edge` (blocks of kBlockRows / edge
        // tiles): all of them (which = 0), only the full off-diagonal ones
        // (1), or only the diagonal tiles and those reaching past s - 32, the
        // tiles the skip form forms in part (2).
        auto unit_tiles = [&](const Unit &u, int edge, int diag_step, int which, std::vector<TileDesc> &out) {
            const int32_t k = u.k;
            const int s_k = plan->desc[k].s;
            const int nt = (plan->desc[k].s_pad + edge - 1) / edge;
            const int tb = kBlockRows / edge;
            const int b_lo = u.bi < 0 ? 0 : u.bi, b_hi = u.bi < 0 ? (nt + tb - 1) / tb : u.bi + 1;
            for (int BI = b_lo; BI < b_hi; ++BI) {
                const int c_lo = u.bi < 0 ? BI : u.bj, c_hi = u.bi < 0 ? (nt + tb - 1) / tb : u.bj + 1;
                for (int BJ = c_lo; BJ < c_hi; ++BJ)
                    for (int ti = BI * tb; ti < std::min((BI + 1) * tb, nt); ++ti)
                        for (int tj = std::max(ti, BJ * tb); tj < std::min((BJ + 1) * tb, nt); ++tj) {
                            const bool full = ti != tj && (tj + 1) * edge - 32 < s_k;
                            if ((which == 1 && !full) || (which == 2 && full)) continue;
                            out.push_back(TileDesc{k, ti, tj, ti == tj ? diag_base[k] + diag_step * ti : -1});
                        }
            }
        };
        // The skip form's list holds the same tiles per XCD, but an XCD's full
        // tiles first and its short ones (formed in part, so ending early)
        // after all of them: amid full tiles a short one puts the workgroups
        // that share the XCD's L2 out of step with the panel chunks they read
        // together, and the offset lasts while the tiles that follow are equal.
        std::vector<std::vector<TileDesc>> lists(kXcds), lists_s(kXcds);
        for (int x = 0; x < kXcds; ++x) {
            for (const Unit &u : xcd_units[x]) unit_tiles(u, T, 1, 0, lists[x]);
            for (const Unit &u : xcd_units[x]) unit_tiles(u, T, 1, 1, lists_s[x]);
            for (const Unit &u : xcd_units[x]) unit_tiles(u, T, 1, 2, lists_s[x]);
        }
        size_t longest = 0;
        for (auto &l : lists) longest = std::max(longest, l.size());
        for (size_t q = 0; q < longest; ++q)
            for (int x = 0; x < kXcds; ++x) {
                plan->tiles.push_back(q < lists[x].size() ? lists[x][q] : TileDesc{-1, 0, 0, -1});
                plan->tiles_s.push_back(q < lists_s[x].size() ? lists_s[x][q] : TileDesc{-1, 0, 0, -1});
            }
        // The same units for the 256 x 256 tiles of the 16-bit products, in
        // blocks of 4 x 4 (the same panels as 8 x 8 blocks of 128-tiles).  A
        // diagonal 256-tile covers 128-tile diagonal slots 2t and 2t + 1.
        std::vector<std::vector<TileDesc>> lists_w(kXcds);
        for (int x = 0; x < kXcds; ++x)
            for (const Unit &u : xcd_units[x]) unit_tiles(u, kTileWide, 2, 0, lists_w[x]);
        longest = 0;
        for (auto &l : lists_w) longest = std::max(longest, l.size());
        for (size_t q = 0; q < longest; ++q)
            for (int x = 0; x < kXcds; ++x)
                plan->tiles_w.push_back(q < lists_w[x].size() ? lists_w[x][q] : TileDesc{-1, 0, 0, -1});
        plan->n_diag = slot;
        for (int32_t y = 0; y < n_sys; ++y) {
            for (int32_t k : sys_parts[y])
                for (int r0 = 0; r0 < plan->desc[k].s_pad; r0 += kRowsPerChunk)
                    plan->chunks.push_back(RowChunk{k, r0, std::min(r0 + kRowsPerChunk, plan->desc[k].s_pad), 0});
            sys_chunk_ptr[y + 1] = (int32_t)plan->chunks.size();
        }
        // vertices of every system, ascending, for the per-system Gershgorin bounds
        std::vector<int32_t> sys_row_ptr(n_sys + 1, 0), sys_rows(n);
        plan->sys_size.assign(n_sys, 0);
        for (int32_t v = 0; v < n; ++v) plan->sys_size[plan->part_system[part[v]]]++;
        for (int32_t y = 0; y < n_sys; ++y) sys_row_ptr[y + 1] = sys_row_ptr[y] + plan->sys_size[y];
        {
            std::vector<int32_t> fill(sys_row_ptr.begin(), sys_row_ptr.end() - 1);
            for (int32_t v = 0; v < n; ++v) sys_rows[fill[plan->part_system[part[v]]]++] = v;
        }
        plan->perm.resize(plan->sub_idx.size());
        for (int32_t k = 0; k < n_parts; ++k) {
            const int64_t b = plan->sub_ptr[k];
            const int32_t s = plan->desc[k].s, c = plan->desc[k].c;
            const int32_t *ix = plan->sub_idx.data() + b;
            // merge the two ascending runs (core, halo) by global id
            int32_t i = 0, j = c, t = 0;
            while (i < c || j < s) {
                if (j >= s || (i < c && ix[i] < ix[j])) plan->perm[b + t++] = i++;
                else plan->perm[b + t++] = j++;
            }
        }
        plan->col_ptr.assign(n + 1, 0);
        plan->col_part.resize(n);
        plan->col_local.resize(n);
        {
            std::vector<int32_t> seen(n_parts, 0);
            for (int32_t j = 0; j < n; ++j) {
                const int32_t k = part[j];
                plan->col_part[j] = k;
                plan->col_local[j] = seen[k]++;    // cores are ascending, so this is j's local index
                plan->col_ptr[j + 1] = plan->col_ptr[j] + plan->desc[k].s;
            }
        }

        // device workspace
        DevicePlan &dp = plan->dp;
        dp.n = n;
        dp.n_parts = n_parts;
        dp.n_tiles = (int32_t)plan->tiles.size();
        dp.n_diag = plan->n_diag;
        dp.n_chunks = (int32_t)plan->chunks.size();
        dp.max_s_pad = max_s_pad;
        dp.gersh_blocks = (n + kRowsPerBlock - 1) / kRowsPerBlock;
        dp.n_sys = n_sys;
        dp.buf[0] = plan->alloc<float>(plan->arena_floats, "X buffer 0");
        dp.buf[1] = plan->alloc<float>(plan->arena_floats, "X buffer 1");
        auto *d_parts = plan->alloc<PartDesc>(n_parts, "part descriptors");
        auto *d_tiles = plan->alloc<TileDesc>(plan->tiles.size(), "tiles");
        auto *d_tiles_s = plan->alloc<TileDesc>(plan->tiles_s.size(), "tiles, short ones last");
        auto *d_tiles_w = plan->alloc<TileDesc>(plan->tiles_w.size(), "wide tiles");
        auto *d_chunks = plan->alloc<RowChunk>(plan->chunks.size(), "row chunks");
        auto *d_idx = plan->alloc<int32_t>(plan->sub_idx.size(), "index arena");
        auto *d_perm = plan->alloc<int32_t>(plan->perm.size(), "perm arena");
        auto *d_invperm = plan->alloc<int32_t>(plan->perm.size(), "inverse perm arena");
        {
            std::vector<int32_t> inv(plan->perm.size());
            for (int32_t k = 0; k < n_parts; ++k) {
                const int64_t b = plan->sub_ptr[k];
                for (int32_t t = 0; t < plan->desc[k].s; ++t) inv[b + plan->perm[b + t]] = t;
            }
            upload(d_invperm, inv, s, "upload inverse perm");
            check_hip(hipStreamSynchronize(s), "upload inverse perm");
        }
        auto *d_colptr = plan->alloc<int64_t>(n + 1, "col_ptr");
        auto *d_colpart = plan->alloc<int32_t>(n, "col_part");
        auto *d_collocal = plan->alloc<int32_t>(n, "col_local");
        dp.diag_partials = plan->alloc<double>(4 * (size_t)std::max(1, plan->n_diag), "diag partials");
        dp.list_len = dp.n_tiles / kXcds;
        dp.persist = plan->alloc<PersistCtl>(1, "persistent control");
        {
            int rate_khz = 0, dev = 0;
            check_hip(hipGetDevice(&dev), "device");
            check_hip(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev), "wall clock rate");
            dp.persist_timeout = (long long)std::max(rate_khz, 1000) * 1000LL * 20;   // 20 s
        }
        dp.x0_partials = plan->alloc<double>(plan->chunks.size(), "x0 partials");
        dp.row_bounds = plan->alloc<double>(3 * (size_t)n, "gershgorin discs");
        auto *d_sys_rows = plan->alloc<int32_t>(n, "system rows");
        auto *d_sys_row_ptr = plan->alloc<int32_t>(n_sys + 1, "system row pointer");
        auto *d_sys_chunk_ptr = plan->alloc<int32_t>(n_sys + 1, "system chunk pointer");
        auto *d_sys_diag_ptr = plan->alloc<int32_t>(n_sys + 1, "system slot pointer");
        dp.sys_params = plan->alloc<SysParams>(n_sys, "system parameters");
        dp.state = plan->alloc<RunState>(n_sys, "run state");
        upload(d_sys_rows, sys_rows, s, "upload system rows");
        upload(d_sys_row_ptr, sys_row_ptr, s, "upload system rows");
        upload(d_sys_chunk_ptr, sys_chunk_ptr, s, "upload system chunks");
        upload(d_sys_diag_ptr, sys_diag_ptr, s, "upload system slots");
        dp.sys_rows = d_sys_rows;
        dp.sys_row_ptr = d_sys_row_ptr;
        dp.sys_chunk_ptr = d_sys_chunk_ptr;
        dp.sys_diag_ptr = d_sys_diag_ptr;
        upload(d_parts, plan->desc, s, "upload parts");
        upload(d_tiles, plan->tiles, s, "upload tiles");
        upload(d_tiles_s, plan->tiles_s, s, "upload tiles, short ones last");
        upload(d_tiles_w, plan->tiles_w, s, "upload wide tiles");
        upload(d_chunks, plan->chunks, s, "upload chunks");
        upload(d_idx, plan->sub_idx, s, "upload index");
        upload(d_perm, plan->perm, s, "upload perm");
        upload(d_colptr, plan->col_ptr, s, "upload col_ptr");
        upload(d_colpart, plan->col_part, s, "upload col_part");
        upload(d_collocal, plan->col_local, s, "upload col_local");
        check_hip(hipMemsetAsync(dp.state, 0, sizeof(RunState) * (size_t)n_sys, s), "clear state");
        dp.parts = d_parts;
        dp.tiles = d_tiles;
        dp.tiles_s = d_tiles_s;
        dp.tiles_w = d_tiles_w;
        dp.n_tiles_w = (int32_t)plan->tiles_w.size();
        dp.chunks = d_chunks;
        dp.idx = d_idx;
        dp.perm = d_perm;
        dp.invperm = d_invperm;
        dp.col_ptr = d_colptr;
        dp.col_part = d_colpart;
        dp.col_local = d_collocal;
        check_hip(hipHostMalloc((void **)&plan->h_state, sizeof(RunState) * (size_t)n_sys, hipHostMallocDefault),
                  "pinned state");
        check_hip(hipHostMalloc((void **)&plan->h_sys, sizeof(SysParams) * (size_t)n_sys, hipHostMallocDefault),
                  "pinned parameters");
        check_hip(hipEventCreateWithFlags(&plan->sys_uploaded, hipEventDisableTiming), "event");
        check_hip(hipStreamSynchronize(s), "plan upload");
        plan->plan_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        *out = plan;
    });
    if (st != GSP2_OK) delete plan;
    return st;
}

gsp2_status gsp2_plan_query(gsp2_plan plan, gsp2_plan_info *info, int32_t *core_sizes, int32_t *sub_sizes) {
    return guarded([&] {
        if (!plan) fail(GSP2_E_INVALID, "null plan");
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->n = plan->n;
            info->n_parts = plan->n_parts;
            int32_t mx = 0, mn = INT32_MAX;
            double s3 = 0.0;
            int64_t nnzp = 0;
            for (const auto &d : plan->desc) {
                mx = std::max(mx, d.s);
                mn = std::min(mn, d.s);
                s3 += (double)d.s * d.s * d.s;
                nnzp += (int64_t)d.c * d.s;
            }
            info->max_s = mx;
            info->min_s = mn;
            info->nnz_graph = plan->nnz_graph;
            info->nnz_P = nnzp;
            info->sum_s = (int64_t)plan->sub_idx.size();
            info->sum_s3 = s3;
            info->tile = plan->tile;
            info->n_tiles = (int32_t)plan->tiles.size();
            info->workspace_bytes = plan->workspace_bytes;
            info->plan_ms = plan->plan_ms;
            info->n_systems = plan->n_sys;
        }
        for (int32_t k = 0; k < plan->n_parts; ++k) {
            if (core_sizes) core_sizes[k] = plan->desc[k].c;
            if (sub_sizes) sub_sizes[k] = plan->desc[k].s;
        }
    });
}

gsp2_status gsp2_plan_pattern(gsp2_plan plan, int64_t *col_ptr, int32_t *row_idx) {
    return guarded([&] {
        if (!plan) fail(GSP2_E_INVALID, "null plan");
        if (col_ptr) std::copy(plan->col_ptr.begin(), plan->col_ptr.end(), col_ptr);
        if (row_idx) {
            for (int32_t j = 0; j < plan->n; ++j) {
                const PartDesc &d = plan->desc[plan->col_part[j]];
                const int32_t *ix = plan->sub_idx.data() + d.idx_off;
                const int32_t *pm = plan->perm.data() + d.perm_off;
                int32_t *dst = row_idx + plan->col_ptr[j];
                for (int32_t t = 0; t < d.s; ++t) dst[t] = ix[pm[t]];
            }
        }
    });
}

gsp2_status gsp2_plan_part_index(gsp2_plan plan, int32_t k, int32_t *idx) {
    return guarded([&] {
        if (!plan) fail(GSP2_E_INVALID, "null plan");
        if (k < 0 || k >= plan->n_parts) fail(GSP2_E_INVALID, "part out of range");
        if (!idx) fail(GSP2_E_INVALID, "null idx");
        std::copy(plan->sub_idx.begin() + plan->sub_ptr[k], plan->sub_idx.begin() + plan->sub_ptr[k + 1], idx);
    });
}

gsp2_status gsp2_probe_mfma(int32_t precision, void *stream, double *tflops) {
    float *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const gsp2_status st = guarded([&] {
        if (!tflops) fail(GSP2_E_INVALID, "null tflops");
        if (precision < GSP2_PREC_FP32 || precision > GSP2_PREC_FP16X3) fail(GSP2_E_INVALID, "bad precision");
        int dev = 0, cus = 0;
        check_hip(hipGetDevice(&dev), "device");
        check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
        const int blocks = 2 * std::max(cus, 1);                // two 4-wave workgroups per CU
        hipStream_t s = static_cast<hipStream_t>(stream);
        check_hip(hipMalloc(&out, sizeof(float) * (size_t)blocks * kProbeThreads), "probe output");
        check_hip(hipEventCreate(&e0), "event");
        check_hip(hipEventCreate(&e1), "event");
        // about 30 ms at the published peak: 16-bit MFMAs run 16 times as
        // many flops per cycle as FP32 ones and twice as many per call
        const int n_iter = precision == GSP2_PREC_FP32 ? 12000 : 96000;
        int64_t flops = 0;
        check_hip(probe_mfma(precision, n_iter / 16, blocks, out, s, &flops), "probe warm-up");
        check_hip(hipEventRecord(e0, s), "event");
        check_hip(probe_mfma(precision, n_iter, blocks, out, s, &flops), "probe");
        check_hip(hipEventRecord(e1, s), "event");
        check_hip(hipEventSynchronize(e1), "probe");
        float ms = 0.0f;
        check_hip(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        *tflops = ms > 0.0f ? (double)flops / (ms * 1e-3) / 1e12 : 0.0;
    });
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);             // waits for the probe launches
    return st;
}

gsp2_status gsp2_plan_tune(gsp2_plan plan, const gsp2_csr *H, double n_occ, int32_t precision,
                           int32_t n_products, gsp2_tune_info *info) {
    float *scratch = nullptr;
    const gsp2_status st = guarded([&] {
        if (!plan || !H) fail(GSP2_E_INVALID, "null argument");
        const bool wide16 = precision == GSP2_PREC_FP16 || precision == GSP2_PREC_BF16 ||
                            precision == GSP2_PREC_FP16X3;
        if (precision != GSP2_PREC_FP32 && precision != GSP2_PREC_FP64 && !wide16)
            fail(GSP2_E_INVALID, "gsp2_plan_tune takes a product precision");
        if (n_products < 2 || n_products > GSP2_MAX_ITER) fail(GSP2_E_INVALID, "n_products out of range");
        int64_t nnz_p = 0;
        for (const auto &d : plan->desc) nnz_p += (int64_t)d.c * d.s;
        const size_t p_elem = precision == GSP2_PREC_FP64 ? sizeof(double) : sizeof(float);   // P's type
        check_hip(hipMalloc(&scratch, p_elem * (size_t)std::max<int64_t>(nnz_p, 1)), "tuner scratch output");
        std::vector<int8_t> seq(n_products);
        for (int i = 0; i < n_products; ++i) seq[i] = (i % 2) ? 1 : -1;
        std::vector<double> occ(plan->n_sys, n_occ);
        gsp2_run_options o;
        gsp2_run_options_default(&o);
        o.max_iter = n_products;
        o.alpha_mode = GSP2_ALPHA_REPLAY;
        o.alpha_seq = seq.data();
        o.n_alpha = n_products;
        o.timing = 1;
        o.precision = precision;
        if (plan->n_sys > 1) o.n_occ_system = occ.data();
        const int32_t cand[3] = {GSP2_KERNEL_T128, GSP2_KERNEL_T128_SKIP, GSP2_KERNEL_T256};
        const int n_cand = wide16 ? 3 : 2;
        double ms[3] = {0.0, 0.0, 0.0};
        int best = 0;
        for (int c = 0; c < n_cand; ++c) {
            o.kernel = cand[c];
            gsp2_status r = GSP2_OK;
            for (int rep = 0; rep < 2 && r == GSP2_OK; ++rep)    // the first run builds the graph
                r = gsp2_density(plan, H, n_occ, &o, scratch, nullptr);
            gsp2_timing t;
            if (r == GSP2_OK) r = gsp2_run_timing(plan, &t);
            if (r != GSP2_OK) fail(r, std::string("tuning run: ") + g_last_error);
            double sum = 0.0;
            for (int i = 0; i < t.n_products; ++i) sum += t.product_ms[i];
            ms[c] = t.n_products > 0 ? sum / t.n_products : 0.0;
            if (ms[c] < ms[best]) best = c;
        }
        // another form replaces the default only when it is more than 1% faster
        // (beyond the run-to-run spread), so near ties keep the default
        const int dflt = wide16 ? 2 : 1;
        if (ms[best] > 0.99 * ms[dflt]) best = dflt;
        plan->kernel_tuned[precision] = cand[best];
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->precision = precision;
            info->chosen = cand[best];
            info->n_candidates = n_cand;
            info->n_products = n_products;
            for (int c = 0; c < n_cand; ++c) {
                info->candidate[c] = cand[c];
                info->ms[c] = ms[c];
            }
        }
    });
    if (scratch) (void)hipFree(scratch);     // waits for the tuning runs
    return st;
}

gsp2_status gsp2_plan_graph(gsp2_plan plan, int64_t *adj_ptr, int32_t *adj_col) {
    return guarded([&] {
        if (!plan) fail(GSP2_E_INVALID, "null plan");
        if (!adj_ptr) fail(GSP2_E_INVALID, "null adj_ptr");
        std::copy(plan->adj_ptr.begin(), plan->adj_ptr.end(), adj_ptr);
        if (adj_col) std::copy(plan->adj_col.begin(), plan->adj_col.end(), adj_col);
    });
}

gsp2_status gsp2_partition_anneal(int32_t n, const int64_t *adj_ptr, const int32_t *adj_col, int32_t n_parts,
                                  int32_t *part, const gsp2_anneal_options *opt, int64_t *cost_before,
                                  int64_t *cost_after) {
    return guarded([&] {
        check_graph_and_parts(n, adj_ptr, adj_col, part, n_parts);
        const int32_t sweeps = (opt && opt->sweeps > 0) ? opt->sweeps : 40;
        const double t0 = (opt && opt->t0 != 0.0) ? opt->t0 : 2.0;
        const double cooling = (opt && opt->cooling != 0.0) ? opt->cooling : 0.85;
        if (opt && opt->sweeps < 0) fail(GSP2_E_INVALID, "sweeps must be >= 0");
        if (!(cooling > 0.0 && cooling <= 1.0)) fail(GSP2_E_INVALID, "cooling must be in (0, 1]");
        if (!std::isfinite(t0)) fail(GSP2_E_INVALID, "t0 must be finite");
        const AnnealResult r = anneal_partition(n, adj_ptr, adj_col, n_parts, part, sweeps, std::max(t0, 0.0),
                                                cooling, opt ? opt->seed : 0);
        if (cost_before) *cost_before = r.cost_before;
        if (cost_after) *cost_after = r.cost_after;
    });
}

gsp2_status gsp2_locality_graph(int32_t n_orb, const int32_t *orbital_atom, int32_t n_atoms, const double *xyz,
                                double radius, double box, int64_t *adj_ptr, int32_t *adj_col) {
    return guarded([&] {
        if (n_orb < 1 || n_atoms < 1) fail(GSP2_E_INVALID, "need n_orb >= 1 and n_atoms >= 1");
        if (!orbital_atom || !xyz || !adj_ptr) fail(GSP2_E_INVALID, "null pointer");
        if (!(radius > 0.0) || !std::isfinite(radius)) fail(GSP2_E_INVALID, "radius must be finite and > 0");
        if (!std::isfinite(box)) fail(GSP2_E_INVALID, "box must be finite");
        for (int32_t u = 0; u < n_orb; ++u)
            if (orbital_atom[u] < 0 || orbital_atom[u] >= n_atoms)
                fail(GSP2_E_INVALID, "atom id out of range at orbital " + std::to_string(u));
        for (int64_t i = 0; i < 3 * (int64_t)n_atoms; ++i)
            if (!std::isfinite(xyz[i])) fail(GSP2_E_INVALID, "non-finite coordinate");
        std::vector<int64_t> ptr;
        std::vector<int32_t> col;
        locality_graph(n_orb, orbital_atom, n_atoms, xyz, radius, box, ptr, col);
        std::copy(ptr.begin(), ptr.end(), adj_ptr);
        if (adj_col) std::copy(col.begin(), col.end(), adj_col);
    });
}

gsp2_status gsp2_sparse_sp2_host(int32_t n, const int64_t *H_row_ptr, const int32_t *H_col, const double *H_val,
                                 double n_occ, double eps, int32_t max_iter, int64_t *P_row_ptr, int32_t *P_col,
                                 double *P_val, gsp2_sparse_sp2_info *info) {
    gsp2_status run_status = GSP2_OK;
    const gsp2_status st = guarded([&] {
        if (n < 1) fail(GSP2_E_INVALID, "need n >= 1");
        if (!H_row_ptr || !P_row_ptr) fail(GSP2_E_INVALID, "null pointer");
        if ((P_col == nullptr) != (P_val == nullptr)) fail(GSP2_E_INVALID, "P_col and P_val go together");
        if (H_row_ptr[0] != 0) fail(GSP2_E_INVALID, "H_row_ptr[0] must be 0");
        for (int32_t i = 0; i < n; ++i)
            if (H_row_ptr[i + 1] < H_row_ptr[i]) fail(GSP2_E_INVALID, "H_row_ptr must not decrease");
        const int64_t nnz = H_row_ptr[n];
        if (nnz > 0 && (!H_col || !H_val)) fail(GSP2_E_INVALID, "null H arrays");
        for (int64_t e = 0; e < nnz; ++e) {
            if (H_col[e] < 0 || H_col[e] >= n) fail(GSP2_E_INVALID, "column index out of range");
            if (!std::isfinite(H_val[e])) fail(GSP2_E_INVALID, "non-finite H");
        }
        if (!(n_occ >= 0.0) || !(n_occ <= (double)n)) fail(GSP2_E_INVALID, "need 0 <= n_occ <= n");
        if (!(eps >= 0.0) || !std::isfinite(eps)) fail(GSP2_E_INVALID, "eps must be finite and >= 0");
        if (max_iter < 1 || max_iter > GSP2_MAX_ITER) fail(GSP2_E_INVALID, "max_iter out of range");
        const int n_threads = (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
        SparseSP2Result r = sparse_sp2(n, H_row_ptr, H_col, H_val, n_occ, eps, max_iter, 0.5, n_threads);
        if (!(r.eps_max > r.eps_min)) fail(GSP2_E_INVALID, "flat spectrum bounds (eps_max <= eps_min)");
        std::copy(r.ptr.begin(), r.ptr.end(), P_row_ptr);
        if (P_col) {
            std::copy(r.col.begin(), r.col.end(), P_col);
            std::copy(r.val.begin(), r.val.end(), P_val);
        }
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->status = r.status;
            info->n_products = r.n_products;
            info->n_alpha = (int32_t)r.alphas.size();
            info->eps_min = r.eps_min;
            info->eps_max = r.eps_max;
            info->trace = r.trace;
            info->idempotency = r.idempotency;
            info->nnz = r.ptr.back();
            std::copy(r.alphas.begin(), r.alphas.end(), info->alpha);
        }
        run_status = (gsp2_status)r.status;
        if (run_status != GSP2_OK)
            g_last_error = run_status == GSP2_E_WRONG_TRACE ? "trace of the result misses n_occ by more than 0.5"
                                                            : "no convergence within max_iter products";
    });
    return st != GSP2_OK ? st : run_status;
}

gsp2_status gsp2_plan_set_stream(gsp2_plan plan, void *stream) {
    return guarded([&] {
        if (!plan) fail(GSP2_E_INVALID, "null plan");
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (s != plan->stream) {
            check_hip(plan->stream ? hipStreamSynchronize(plan->stream) : hipDeviceSynchronize(), "set stream");
            plan->stream = s;
        }
    });
}

static void fill_info(const RunState &r, gsp2_run_info *info) {
    std::memset(info, 0, sizeof(*info));
    info->status = r.status;
    info->n_products = r.n_products;
    info->n_alpha = r.t;
    info->result_iterate = r.result_t;
    info->n_refine = r.n_refine;
    info->precision = r.precision;
    info->eps_min = r.eps_min;
    info->eps_max = r.eps_max;
    info->trace = (r.result_t >= 0 && r.result_t <= GSP2_MAX_ITER) ? r.traces[r.result_t] : NAN;
    info->idempotency = r.idem;
    for (int i = 0; i < GSP2_MAX_ITER; ++i) {
        info->alpha[i] = r.alpha_hist[i];
        info->errors[i] = r.errors[i];
        info->traces[i] = r.traces[i];
    }
    info->traces[GSP2_MAX_ITER] = r.traces[GSP2_MAX_ITER];
}

// Wait for the run whose state is at `dev_state` (the plan's own, or the
// static scratch's) and report it.
static gsp2_status collect(gsp2_plan_s *plan, const RunState *dev_state, gsp2_run_info *info) {
    gsp2_status run_status = GSP2_OK;
    const gsp2_status st = guarded([&] {
        check_hip(hipMemcpyAsync(plan->h_state, dev_state, sizeof(RunState) * (size_t)plan->n_sys,
                                 hipMemcpyDeviceToHost, plan->stream), "copy run state");
        check_hip(hipStreamSynchronize(plan->stream), "run");
        int32_t bad = -1;
        for (int32_t y = 0; y < plan->n_sys; ++y) {
            if (info) fill_info(plan->h_state[y], info + y);
            if (bad < 0 && plan->h_state[y].status != GSP2_OK) bad = y;
        }
        if (bad >= 0) {
            run_status = (gsp2_status)plan->h_state[bad].status;
            const RunState &r = plan->h_state[bad];
            char buf[256];
            if (run_status == GSP2_E_INVALID)
                std::snprintf(buf, sizeof buf, "H rejected: Gershgorin bounds [%g, %g] not finite or empty",
                              r.eps_min, r.eps_max);
            else if (run_status == GSP2_E_HIP)
                std::snprintf(buf, sizeof buf, "persistent product kernel: a grid-barrier wait expired");
            else if (run_status == GSP2_E_NOT_CONVERGED)
                std::snprintf(buf, sizeof buf, "no convergence after %d products", r.n_products);
            else
                std::snprintf(buf, sizeof buf, "trace %.6f differs from n_occ %.6f by more than %g",
                              r.traces[r.result_t], r.n_occ, r.trace_tol);
            g_last_error = buf;
            if (plan->n_sys > 1) g_last_error = "system " + std::to_string(bad) + ": " + g_last_error;
        }
    });
    if (st != GSP2_OK) return st;
    return run_status;
}

// Checks of one density-matrix call shared by gsp2_density and
// gsp2_density_noalloc: the run parameters, and the per-system parameters
// staged in the plan's pinned buffer for the upload before the launch.
static RunParams prepare_run(gsp2_plan_s *plan, const gsp2_csr *H, double n_occ, const gsp2_run_options &o,
                             void *P_val) {
    if (!plan) fail(GSP2_E_INVALID, "null plan");
    if (!H) fail(GSP2_E_INVALID, "null H");
    if (H->n != plan->n) fail(GSP2_E_INVALID, "H.n differs from the plan");
    if (H->nnz < 0 || !H->row_ptr || (H->nnz > 0 && (!H->col || !H->val)))
        fail(GSP2_E_INVALID, "bad H arrays");
    if (H->dtype != GSP2_F32 && H->dtype != GSP2_F64) fail(GSP2_E_INVALID, "bad H.dtype");
    if (!P_val) fail(GSP2_E_INVALID, "null P_val");
    const int32_t n_sys = plan->n_sys;
    if (n_sys > 1 && !o.n_occ_system) fail(GSP2_E_INVALID, "a batched plan needs n_occ_system");
    RunParams rp{};
    rp.trace_tol = o.trace_tol;
    rp.mode = o.alpha_mode;
    rp.stop_rule = o.stop_rule ? 1 : 0;
    if (o.precision != GSP2_PREC_FP32 && o.precision != GSP2_PREC_FP16 && o.precision != GSP2_PREC_BF16 &&
        o.precision != GSP2_PREC_FP16X3 && o.precision != GSP2_PREC_FP64)
        fail(GSP2_E_INVALID, "bad precision");
    const bool wide16 = o.precision == GSP2_PREC_FP16 || o.precision == GSP2_PREC_BF16 ||
                        o.precision == GSP2_PREC_FP16X3;
    if (wide16 && plan->dp.max_s_pad > kMaxWidePad)
        fail(GSP2_E_UNSUPPORTED, "16-bit products need every padded sub-problem size <= " +
                                     std::to_string(kMaxWidePad));
    if (o.refine < 0 || o.refine > 8) fail(GSP2_E_INVALID, "refine must be in 0..8");
    if (o.symmetrize != 0 && o.symmetrize != 1) fail(GSP2_E_INVALID, "symmetrize must be 0 or 1");
    rp.precision = o.precision;
    rp.refine = o.refine;
    rp.persistent = o.persistent ? 1 : 0;
    rp.symmetrize = o.symmetrize;
    // the product kernel's form: named by the run, else the plan's fixed
    // 16-bit tile edge, else the tuned form, else the default
    if (o.kernel < GSP2_KERNEL_AUTO || o.kernel > GSP2_KERNEL_T256) fail(GSP2_E_INVALID, "bad kernel");
    if (o.kernel == GSP2_KERNEL_T256 && !wide16) fail(GSP2_E_INVALID, "256 x 256 tiles take 16-bit products only");
    if (o.kernel != GSP2_KERNEL_AUTO)
        rp.kernel = o.kernel;
    else if (wide16 && plan->tile16_fixed)
        rp.kernel = plan->tile16_fixed == kTile ? GSP2_KERNEL_T128 : GSP2_KERNEL_T256;
    else if (plan->kernel_tuned[o.precision])
        rp.kernel = plan->kernel_tuned[o.precision];
    else
        rp.kernel = wide16 ? GSP2_KERNEL_T256 : GSP2_KERNEL_T128_SKIP;
    rp.refine_prec = o.precision == GSP2_PREC_FP64 ? GSP2_PREC_FP64 : GSP2_PREC_FP32;
    if (o.refine_precision == GSP2_PREC_FP16X3) {
        if (o.precision != GSP2_PREC_FP16 && o.precision != GSP2_PREC_BF16)
            fail(GSP2_E_INVALID, "split FP16 refinement products follow FP16 or BF16 products only");
        rp.refine_prec = GSP2_PREC_FP16X3;
    } else if (o.refine_precision != GSP2_PREC_FP32) {
        fail(GSP2_E_INVALID, "refine_precision must be GSP2_PREC_FP32 or GSP2_PREC_FP16X3");
    }
    if (o.precision == GSP2_PREC_FP32 || o.precision == GSP2_PREC_FP64)
        rp.kernel32 = rp.kernel;                // the refinement products take the main products' form
    else
        rp.kernel32 = plan->kernel_tuned[GSP2_PREC_FP32] ? plan->kernel_tuned[GSP2_PREC_FP32] : GSP2_KERNEL_T128_SKIP;
    if (rp.persistent && (n_sys > 1 || (rp.precision != GSP2_PREC_FP32 && rp.precision != GSP2_PREC_FP16 &&
                                         rp.precision != GSP2_PREC_BF16)))
        fail(GSP2_E_UNSUPPORTED, "the persistent product launch takes one system and FP32, FP16 or BF16 products");
    if (rp.persistent)
        fail(GSP2_E_UNSUPPORTED,
             "the persistent product launch is switched off: its first GPU run did not return and the "
             "cause has not been established");
    if (rp.persistent) {
        int grid = 0;
        check_hip(persistent_grid(rp.precision, &grid), "occupancy");
        if (grid < 1) fail(GSP2_E_UNSUPPORTED, "persistent product kernel cannot be resident");
        plan->dp.persist_grid = std::min(grid, plan->dp.n_tiles);
    }
    // per-system parameters, staged for the upload that precedes the launch
    plan->wait_sys_staging();
    std::memset(plan->h_sys, 0, sizeof(SysParams) * (size_t)n_sys);
    // the stop rule's floor max(1, n u), u the unit roundoff of the product operands
    const double u = o.precision == GSP2_PREC_FP16     ? std::ldexp(1.0, -11)
                     : o.precision == GSP2_PREC_BF16   ? std::ldexp(1.0, -8)
                     : o.precision == GSP2_PREC_FP16X3 ? std::ldexp(1.0, -22)
                     : o.precision == GSP2_PREC_FP64   ? std::ldexp(1.0, -53)
                                                       : std::ldexp(1.0, -24);
    if (!(o.trace_tol >= 0.0)) fail(GSP2_E_INVALID, "trace_tol must be >= 0");
    if (o.alpha_mode == GSP2_ALPHA_REPLAY) {
    } else if (o.alpha_mode == GSP2_ALPHA_TRACE) {
        if (o.max_iter < 1 || o.max_iter > GSP2_MAX_ITER) fail(GSP2_E_INVALID, "max_iter out of range");
    } else {
        fail(GSP2_E_INVALID, "bad alpha_mode");
    }
    const bool own_seq = n_sys > 1 && o.alpha_mode == GSP2_ALPHA_REPLAY && o.alpha_seq_system;
    if (own_seq && !o.n_alpha_system) fail(GSP2_E_INVALID, "null n_alpha_system");
    rp.n_steps = 0;
    for (int32_t y = 0; y < n_sys; ++y) {
        SysParams &sp = plan->h_sys[y];
        const std::string who = n_sys > 1 ? " (system " + std::to_string(y) + ")" : "";
        const double occ = n_sys > 1 ? o.n_occ_system[y] : n_occ;
        if (!(occ >= 0.0) || !(occ <= (double)plan->sys_size[y])) fail(GSP2_E_INVALID, "need 0 <= n_occ <= n" + who);
        sp.n_occ = occ;
        sp.stop_floor = std::max(1.0, plan->sys_size[y] * u);
        if (o.alpha_mode == GSP2_ALPHA_TRACE) {
            sp.n_steps = o.max_iter;
        } else {
            const int32_t na = own_seq ? o.n_alpha_system[y] : o.n_alpha;
            const int8_t *seq = own_seq ? o.alpha_seq_system + (size_t)y * GSP2_MAX_ITER : o.alpha_seq;
            if (na < 0 || na > GSP2_MAX_ITER) fail(GSP2_E_INVALID, "n_alpha out of range" + who);
            if (na > 0 && !seq) fail(GSP2_E_INVALID, "null alpha_seq");
            for (int i = 0; i < na; ++i) {
                if (seq[i] != 1 && seq[i] != -1) fail(GSP2_E_INVALID, "alpha must be +1 or -1" + who);
                sp.alpha_seq[i] = seq[i];
            }
            sp.n_steps = na;
        }
        rp.n_steps = std::max(rp.n_steps, sp.n_steps);
    }
    if (rp.n_steps + rp.refine > GSP2_MAX_ITER) fail(GSP2_E_INVALID, "max_iter + refine exceeds GSP2_MAX_ITER");
    return rp;
}

gsp2_status gsp2_density(gsp2_plan plan, const gsp2_csr *H, double n_occ, const gsp2_run_options *run,
                         void *P_val, gsp2_run_info *info) {
    gsp2_status st = guarded([&] {
        gsp2_run_options def;
        gsp2_run_options_default(&def);
        const gsp2_run_options &o = run ? *run : def;
        const RunParams rp = prepare_run(plan, H, n_occ, o, P_val);
        const bool wide16 = rp.precision == GSP2_PREC_FP16 || rp.precision == GSP2_PREC_BF16 ||
                            rp.precision == GSP2_PREC_FP16X3;
        if (rp.precision == GSP2_PREC_FP64 && !plan->dp.buf64[0]) {
            // FP64 iterates, allocated on the first FP64 run
            plan->dp.buf64[0] = plan->alloc<double>(plan->arena_floats, "FP64 X buffer 0");
            plan->dp.buf64[1] = plan->alloc<double>(plan->arena_floats, "FP64 X buffer 1");
        }
        if (wide16 && !plan->dp.shadow[0]) {
            // 16-bit operand copies of both X buffers, allocated on the first mixed-precision run
            plan->dp.shadow[0] = plan->alloc<uint16_t>(plan->arena_floats, "16-bit X copy 0");
            plan->dp.shadow[1] = plan->alloc<uint16_t>(plan->arena_floats, "16-bit X copy 1");
        }
        const bool split_any = rp.precision == GSP2_PREC_FP16X3 || (rp.refine > 0 && rp.refine_prec == GSP2_PREC_FP16X3);
        if (split_any && !plan->dp.shadow_lo[0]) {
            plan->dp.shadow_lo[0] = plan->alloc<uint16_t>(plan->arena_floats, "FP16 low parts 0");
            plan->dp.shadow_lo[1] = plan->alloc<uint16_t>(plan->arena_floats, "FP16 low parts 1");
        }
        GraphKey k;
        k.h_ptr = H->row_ptr; k.h_col = H->col; k.h_val = H->val; k.h_nnz = H->nnz; k.h_dtype = H->dtype;
        k.p_val = P_val; k.rp = rp; k.timing = o.timing != 0;
        const RunEvents *evp = nullptr;
        if (o.timing) { plan->make_events(); evp = &plan->ev; }
        plan->upload_sys();
        const bool eager = std::getenv("GSP2_EAGER") != nullptr;
        if (eager) {
            Recorder rec;
            rec.stream = plan->stream;
            check_hip(launch_density(plan->dp, *H, rp, P_val, rec, evp), "launch density");
        } else {
            if (!plan->have_graph || !(plan->key == k)) {
                if (plan->exec) { check_hip(hipGraphExecDestroy(plan->exec), "graph destroy"); plan->exec = nullptr; }
                if (plan->graph) { check_hip(hipGraphDestroy(plan->graph), "graph destroy"); plan->graph = nullptr; }
                plan->have_graph = false;
                check_hip(hipGraphCreate(&plan->graph, 0), "graph create");
                Recorder rec;
                rec.graph = plan->graph;
                check_hip(launch_density(plan->dp, *H, rp, P_val, rec, evp), "build graph");
                check_hip(hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0), "graph instantiate");
                plan->key = k;
                plan->have_graph = true;
            }
            check_hip(hipGraphLaunch(plan->exec, plan->stream), "graph launch");
        }
        plan->last_rp = rp;
        plan->ran = true;
        plan->last_timed = o.timing != 0;
    });
    if (st != GSP2_OK || !info) return st;
    return collect(plan, plan->dp.state, info);
}

gsp2_status gsp2_density_noalloc(gsp2_plan plan, const gsp2_csr *H, double n_occ, const gsp2_run_options *run,
                                 void *P_val, gsp2_run_info *info) {
    const RunState *dev_state = nullptr;
    gsp2_status st = guarded([&] {
        gsp2_run_options def;
        gsp2_run_options_default(&def);
        const gsp2_run_options &o = run ? *run : def;
        if (o.timing) fail(GSP2_E_INVALID, "timing is not available without allocation (it needs events)");
        const RunParams rp = prepare_run(plan, H, n_occ, o, P_val);
        const bool wide16 = rp.precision == GSP2_PREC_FP16 || rp.precision == GSP2_PREC_BF16 ||
                            rp.precision == GSP2_PREC_FP16X3;
        // every per-run buffer of the plan, laid out in the static scratch
        size_t off = 0;
        auto take = [&](size_t bytes) {
            const size_t at = off;
            off += (bytes + 255) & ~size_t(255);
            return at;
        };
        const int32_t n_sys = plan->n_sys;
        const size_t arena = (size_t)plan->arena_floats;
        const size_t o_state = take(sizeof(RunState) * (size_t)n_sys);
        const size_t o_sys = take(sizeof(SysParams) * (size_t)n_sys);
        const size_t o_diag = take(sizeof(double) * 4 * (size_t)std::max(1, plan->n_diag));
        const size_t o_x0 = take(sizeof(double) * (size_t)std::max(1, plan->dp.n_chunks));
        const size_t o_rows = take(sizeof(double) * 3 * (size_t)plan->n);
        const size_t elem = rp.precision == GSP2_PREC_FP64 ? sizeof(double) : sizeof(float);
        const size_t o_x[2] = {take(elem * arena), take(elem * arena)};
        size_t o_sh[2] = {0, 0}, o_lo[2] = {0, 0};
        if (wide16) { o_sh[0] = take(2 * arena); o_sh[1] = take(2 * arena); }
        const bool split_any = rp.precision == GSP2_PREC_FP16X3 || (rp.refine > 0 && rp.refine_prec == GSP2_PREC_FP16X3);
        if (split_any) { o_lo[0] = take(2 * arena); o_lo[1] = take(2 * arena); }
        if (off > kStaticScratchBytes)
            fail(GSP2_E_UNSUPPORTED, "this run needs " + std::to_string(off) + " bytes of device scratch; the "
                                     "static scratch of gsp2_density_noalloc holds " +
                                     std::to_string(kStaticScratchBytes));
        void *base = nullptr;
        check_hip(static_scratch(&base), "static scratch address");
        char *b = static_cast<char *>(base);
        DevicePlan dp = plan->dp;
        dp.state = reinterpret_cast<RunState *>(b + o_state);
        dp.sys_params = reinterpret_cast<SysParams *>(b + o_sys);
        dp.diag_partials = reinterpret_cast<double *>(b + o_diag);
        dp.x0_partials = reinterpret_cast<double *>(b + o_x0);
        dp.row_bounds = reinterpret_cast<double *>(b + o_rows);
        dp.buf[0] = dp.buf[1] = nullptr;
        dp.buf64[0] = dp.buf64[1] = nullptr;
        dp.shadow[0] = dp.shadow[1] = dp.shadow_lo[0] = dp.shadow_lo[1] = nullptr;
        dp.persist = nullptr;
        for (int i = 0; i < 2; ++i) {
            if (rp.precision == GSP2_PREC_FP64) dp.buf64[i] = reinterpret_cast<double *>(b + o_x[i]);
            else dp.buf[i] = reinterpret_cast<float *>(b + o_x[i]);
            if (wide16) dp.shadow[i] = b + o_sh[i];
            if (split_any) dp.shadow_lo[i] = b + o_lo[i];
        }
        // per-system parameters into the scratch, in stream order; the next
        // call rewrites the pinned staging buffer only after this copy ends
        check_hip(hipMemcpyAsync(dp.sys_params, plan->h_sys, sizeof(SysParams) * (size_t)n_sys,
                                 hipMemcpyHostToDevice, plan->stream), "upload system parameters");
        check_hip(hipEventRecord(plan->sys_uploaded, plan->stream), "parameter upload");
        plan->sys_upload_pending = true;
        Recorder rec;
        rec.stream = plan->stream;
        check_hip(launch_density(dp, *H, rp, P_val, rec, nullptr), "launch density");
        dev_state = dp.state;
    });
    if (st != GSP2_OK || !info) return st;
    return collect(plan, dev_state, info);
}

gsp2_status gsp2_run_status(gsp2_plan plan, gsp2_run_info *info) {
    if (!plan) { g_last_error = "null plan"; return GSP2_E_INVALID; }
    if (!plan->ran) { g_last_error = "no run on this plan"; return GSP2_E_INVALID; }
    return collect(plan, plan->dp.state, info);
}

gsp2_status gsp2_run_timing(gsp2_plan plan, gsp2_timing *out) {
    return guarded([&] {
        if (!plan || !out) fail(GSP2_E_INVALID, "null argument");
        if (!plan->ran || !plan->last_timed) fail(GSP2_E_INVALID, "the last run on this plan was not timed");
        check_hip(hipMemcpyAsync(plan->h_state, plan->dp.state, sizeof(RunState) * (size_t)plan->n_sys,
                                 hipMemcpyDeviceToHost, plan->stream), "copy run state");
        check_hip(hipStreamSynchronize(plan->stream), "timed run");
        std::memset(out, 0, sizeof(*out));
        const RunEvents &e = plan->ev;
        check_hip(hipEventElapsedTime(&out->setup_ms, e.begin, e.setup_end), "elapsed");
        check_hip(hipEventElapsedTime(&out->sp2_ms, e.setup_end, e.sp2_end), "elapsed");
        check_hip(hipEventElapsedTime(&out->scatter_ms, e.sp2_end, e.end), "elapsed");
        check_hip(hipEventElapsedTime(&out->total_ms, e.begin, e.end), "elapsed");
        // main-phase products occupy the first launch slots, refinement products
        // the slots after the main-phase budget
        // launches that carried work: the most any system formed
        int max_main = 0, max_ref = 0;
        for (int32_t y = 0; y < plan->n_sys; ++y) {
            max_main = std::max(max_main, plan->h_state[y].n_main);
            max_ref = std::max(max_ref, plan->h_state[y].n_refine);
        }
        if (plan->last_rp.persistent && plan->last_rp.n_steps > 0)
            check_hip(hipEventElapsedTime(&out->persistent_ms, e.persist_begin, e.persist_end), "elapsed");
        const int n_main = plan->last_rp.persistent ? 0 : std::min(max_main, plan->last_rp.n_steps);
        const int n_ref = std::min(max_ref, plan->last_rp.refine);
        out->n_products = n_main + n_ref;
        for (int t = 0; t < n_main; ++t)
            check_hip(hipEventElapsedTime(&out->product_ms[t], e.step[2 * t], e.step[2 * t + 1]), "elapsed");
        for (int q = 0; q < n_ref; ++q) {
            const int slot = plan->last_rp.n_steps + q;
            check_hip(hipEventElapsedTime(&out->product_ms[n_main + q], e.step[2 * slot], e.step[2 * slot + 1]),
                      "elapsed");
        }
    });
}

gsp2_status gsp2_backward(gsp2_plan plan, const gsp2_csr *H, const int8_t *alpha_seq, int32_t n_alpha,
                          const float *dLdP_val, double *dLdH_val, gsp2_backward_info *info) {
    std::vector<void *> temps;
    auto release = [&] {
        for (void *p : temps) (void)hipFree(p);
        temps.clear();
    };
    gsp2_status st = guarded([&] {
        if (!plan) fail(GSP2_E_INVALID, "null plan");
        if (plan->n_sys > 1) fail(GSP2_E_UNSUPPORTED, "backward pass of a batched plan");
        if (!H || H->n != plan->n) fail(GSP2_E_INVALID, "H missing or of another size");
        if (H->nnz < 0 || !H->row_ptr || (H->nnz > 0 && (!H->col || !H->val)))
            fail(GSP2_E_INVALID, "bad H arrays");
        if (H->dtype != GSP2_F32 && H->dtype != GSP2_F64) fail(GSP2_E_INVALID, "bad H.dtype");
        if (n_alpha < 0 || n_alpha > GSP2_MAX_ITER) fail(GSP2_E_INVALID, "n_alpha out of range");
        if (n_alpha > 0 && !alpha_seq) fail(GSP2_E_INVALID, "null alpha_seq");
        if (!dLdP_val || !dLdH_val) fail(GSP2_E_INVALID, "null gradient array");
        for (int i = 0; i < n_alpha; ++i)
            if (alpha_seq[i] != 1 && alpha_seq[i] != -1) fail(GSP2_E_INVALID, "alpha must be +1 or -1");
        const int n = n_alpha;
        int k = 1;
        while (k * k < n) ++k;
        const int nseg = n > 0 ? (n + k - 1) / k : 1;
        int64_t bytes = 0;
        BackwardBuffers bb{};
        bb.seg = k;
        auto arena = [&](const char *what) {
            float *p = dev_alloc<float>(plan->arena_floats, what, bytes);
            temps.push_back(p);
            return p;
        };
        for (int i = 0; i < nseg; ++i) bb.ckpt[i] = arena("backward checkpoint");
        for (int i = 0; i + 1 < k && i + 1 < n; ++i) bb.slot[i] = arena("backward segment iterate");
        bb.g[0] = arena("backward cotangent");
        bb.g[1] = arena("backward cotangent");
        bb.eps_partials = dev_alloc<double>(2 * (size_t)plan->dp.n_chunks, "backward partials", bytes);
        temps.push_back(bb.eps_partials);
        bb.d_eps = dev_alloc<double>(2, "backward bound cotangents", bytes);
        temps.push_back(bb.d_eps);
        RunParams rp{};
        rp.trace_tol = 1e300;
        rp.n_steps = n;
        rp.mode = GSP2_ALPHA_REPLAY;
        rp.precision = GSP2_PREC_FP32;
        plan->wait_sys_staging();
        SysParams &sp = plan->h_sys[0];
        std::memset(&sp, 0, sizeof sp);
        sp.stop_floor = 1.0;
        sp.n_steps = n;
        for (int i = 0; i < n; ++i) sp.alpha_seq[i] = alpha_seq[i];
        plan->upload_sys();
        check_hip(launch_backward(plan->dp, *H, rp, alpha_seq, n, dLdP_val, dLdH_val, bb, plan->stream),
                  "launch backward");
        double d_eps[2] = {0.0, 0.0};
        check_hip(hipMemcpyAsync(plan->h_state, plan->dp.state, sizeof(RunState), hipMemcpyDeviceToHost,
                                 plan->stream), "copy run state");
        check_hip(hipMemcpyAsync(d_eps, bb.d_eps, sizeof d_eps, hipMemcpyDeviceToHost, plan->stream), "copy d_eps");
        check_hip(hipStreamSynchronize(plan->stream), "backward");
        const RunState &r = *plan->h_state;
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->status = r.status == GSP2_E_INVALID ? GSP2_E_INVALID : GSP2_OK;
            info->n_alpha = n;
            info->checkpoint_every = k;
            info->row_min = r.row_min;
            info->row_max = r.row_max;
            info->eps_min = r.eps_min;
            info->eps_max = r.eps_max;
            info->d_eps_min = d_eps[0];
            info->d_eps_max = d_eps[1];
            info->workspace_bytes = bytes;
        }
        if (r.status == GSP2_E_INVALID) fail(GSP2_E_INVALID, "H rejected: Gershgorin bounds not finite or empty");
    });
    if (plan && plan->stream) (void)hipStreamSynchronize(plan->stream);
    release();
    return st;
}

void gsp2_plan_destroy(gsp2_plan plan) { delete plan; }

}  // extern "C"
