// C ABI of the library (declared in include/tc.h).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "mlp.h"
#include "pipeline.h"
#include "tc.h"

struct tc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipEvent_t events[tcx::NSTAGE + 1] = {};
    float stage_ms[tcx::NSTAGE] = {};
    int have_times = 0;
    std::string last_error;
    tcx::Ctrl* h_ctrl = nullptr;          // pinned host copy of the control block
    uint8_t* d_learned = nullptr;         // device [256] kernel per bucket from the selector network
    int learned_ready = 0;
    uint16_t* d_chunk = nullptr;          // device [256] tile-size overrides (0 = default)
    uint8_t* d_group = nullptr;           // device [256] lanes-per-edge overrides (0 = default)
    uint8_t* d_given = nullptr;           // device [256] caller-chosen kernels (tc_profile_choices)
    uint16_t* d_given_chunk = nullptr;    // device [256] caller-chosen tile sizes (tc_profile_choices)
    int grid_override[tcx::NKERNEL] = {0, 0, 0};
    // selector network: float32 master, Adam moments, gradient, bf16 compute copy,
    // and the per-sample training buffers (allocated on first use)
    float* d_master = nullptr;
    float* d_adam_m = nullptr;
    float* d_adam_v = nullptr;
    float* d_grad = nullptr;
    float* d_loss = nullptr;
    tcx::MlpCompute* d_cw = nullptr;
    // tile network: float32 master and compute copy, its per-bucket scales
    float* d_tile_master = nullptr;
    tcx::MlpCompute* d_cw_tile = nullptr;
    uint8_t* d_learned_tile = nullptr;
    int tile_ready = 0;
    float* d_acts = nullptr;
    int adam_step = 0;
    // batched counting: a stream for capture when the context's stream is the
    // null stream, and the captured graph of the last batch shape
    hipStream_t own_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    struct {   // sizes and workspace of the captured batch (the edge list is read through the workspace)
        int64_t E, N;
        int32_t G, select;
        const void* ws;
    } graph_key = {};
    uint64_t* h_counts_pinned = nullptr;
    size_t h_counts_cap = 0;
    void* d_scratch = nullptr;   // this device's copy of `scratch` (tc_count_triangles_noalloc)
};

// Fixed scratch of tc_count_triangles_noalloc: the pipeline workspace of graphs
// up to TC_NOALLOC_SCRATCH_BYTES, one copy per GPU for the life of the process.
// Host code never uses this name as an address: the device address comes from
// hipGetSymbolAddress, once per device, in tc_create.
static __device__ __align__(256) unsigned char scratch[TC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

tc_status hip_fail(tc_ctx* ctx, hipError_t e, const char* what) {
    if (ctx) {
        char buf[256];
        snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
        ctx->last_error = buf;
    }
    return TC_ERR_HIP;
}

tc_status arg_fail(tc_ctx* ctx, tc_status st, const char* what) {
    if (ctx) ctx->last_error = what;
    return st;
}

bool options_ok(const tc_options* o) {
    if (!o) return true;
    if (o->select < TC_SELECT_HEURISTIC || o->select > TC_FORCE_BITMAP) return false;
    for (int i = 0; i < 6; ++i)
        if (o->reserved[i]) return false;
    return true;
}

// 2E endpoints are indexed with 32-bit positions, with room for one sort tile
constexpr int64_t kMaxEdges = ((int64_t)1 << 31) - ((int64_t)1 << 20);

// Common checks and the run of the pipeline; returns with the control block
// copied to ctx->h_ctrl on success.
// With d_result set, nothing waits for the device: T and the range status go
// to d_result[0..1] on the stream.
tc_status run(tc_ctx* ctx, const int32_t* d_edges, int64_t E, int32_t n, void* ws, size_t ws_bytes,
              const tc_options* opts, tcx::RunArgs& ra, uint64_t* d_result = nullptr) {
    if (!ctx) return TC_ERR_INVALID_ARG;
    ctx->last_error.clear();
    if (E < 0 || n < 0) return arg_fail(ctx, TC_ERR_INVALID_ARG, "negative size");
    if (E > kMaxEdges) return arg_fail(ctx, TC_ERR_UNSUPPORTED, "num_edges must be below 2^31 - 2^20");
    if (!options_ok(opts)) return arg_fail(ctx, TC_ERR_INVALID_ARG, "bad options");
    if (E > 0 && !d_edges) return arg_fail(ctx, TC_ERR_INVALID_ARG, "null edge list");
    if (((uintptr_t)d_edges & 7u) != 0) return arg_fail(ctx, TC_ERR_INVALID_ARG, "edge list must be 8-byte aligned");
    if (E > 0 && n == 0) return arg_fail(ctx, TC_ERR_VERTEX_RANGE, "edges given for an empty vertex set");
    const tcx::Layout L = tcx::make_layout(E, n);
    const bool sym = ra.formulation == tcx::FORM_FULL || ra.formulation == tcx::FORM_MATRIX;
    if (E > 0) {
        if (!ws) return arg_fail(ctx, TC_ERR_INVALID_ARG, "null workspace");
        if (ws_bytes < L.total + (sym ? tcx::sym_extra_bytes(E, n) : 0))
            return arg_fail(ctx, TC_ERR_WORKSPACE, "workspace too small");
    }
    DeviceGuard guard(ctx->device);
    const int sel = opts ? opts->select : TC_SELECT_HEURISTIC;
    if (sel == TC_SELECT_LEARNED && !ctx->learned_ready)
        return arg_fail(ctx, TC_ERR_INVALID_ARG, "no selector network loaded or trained");
    const bool timing = opts && (opts->flags & TC_F_STAGE_TIMING);
    if (d_result && timing) return arg_fail(ctx, TC_ERR_INVALID_ARG, "stage timing needs a synchronising call");
    ra.stream = ctx->stream;
    ra.ws = ws;
    ra.edges = d_edges;
    ra.E = E;
    ra.n = n;
    ra.select = sel;
    ra.mlp = ctx->learned_ready ? ctx->d_cw : nullptr;
    ra.learned = ctx->d_learned;
    ra.mlp_tile = ctx->tile_ready ? ctx->d_cw_tile : nullptr;
    ra.learned_tile = ctx->d_learned_tile;
    if (!ra.chunk_override) ra.chunk_override = ctx->d_chunk;
    ra.group_override = ctx->d_group;
    ra.grid_override = ctx->grid_override;
    ra.events = timing ? ctx->events : nullptr;
    if (E == 0 && d_result) {
        tcx::fill_u64(d_result, 0ull, 2, ctx->stream);
        if (ra.per_vertex && n > 0) tcx::fill_u64(ra.per_vertex, 0ull, (size_t)n, ctx->stream);
        ctx->have_times = 0;
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? TC_OK : hip_fail(ctx, e, "queue zero result");
    }
    if (E == 0) {
        memset(ctx->h_ctrl, 0, sizeof(tcx::Ctrl));
        if (ra.per_vertex && n > 0) {
            hipError_t e = hipMemsetAsync(ra.per_vertex, 0, sizeof(uint64_t) * (size_t)n, ctx->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) return hip_fail(ctx, e, "zero per-vertex output");
        }
        ctx->have_times = 0;
        return TC_OK;
    }
    tcx::RunResult rr;
    hipError_t e = tcx::run_pipeline(ra, &rr);
    if (e != hipSuccess) return hip_fail(ctx, e, "launch");
    if (d_result) {
        tcx::publish_result(rr.ctrl_dev, d_result, (uint64_t)TC_ERR_VERTEX_RANGE, (uint64_t)TC_ERR_HIP, ctx->stream);
        ctx->have_times = 0;
        e = hipGetLastError();
        return e == hipSuccess ? TC_OK : hip_fail(ctx, e, "queue result");
    }
    e = hipMemcpyAsync(ctx->h_ctrl, rr.ctrl_dev, sizeof(tcx::Ctrl), hipMemcpyDeviceToHost, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "read control block");
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "synchronise");
    ctx->have_times = 0;
    if (timing) {
        for (int s = 0; s < tcx::NSTAGE; ++s) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ctx->events[s], ctx->events[s + 1]) != hipSuccess) ms = -1.f;
            ctx->stage_ms[s] = ms;
        }
        ctx->have_times = 1;
    }
    if (ctx->h_ctrl->err & 1u) return arg_fail(ctx, TC_ERR_VERTEX_RANGE, "vertex id outside [0, num_vertices)");
    if (ctx->h_ctrl->err) return arg_fail(ctx, TC_ERR_HIP, "internal bound violated");
    return TC_OK;
}

}  // namespace

extern "C" {

tc_status tc_create(tc_ctx** out, int device, void* hip_stream) {
    if (!out) return TC_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return TC_ERR_INVALID_ARG;
    tc_ctx* ctx = new tc_ctx;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    DeviceGuard guard(device);
    hipError_t e = hipHostMalloc((void**)&ctx->h_ctrl, sizeof(tcx::Ctrl), hipHostMallocDefault);
    for (int i = 0; e == hipSuccess && i <= tcx::NSTAGE; ++i) e = hipEventCreate(&ctx->events[i]);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_learned, tcx::NBUCKET);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_chunk, sizeof(uint16_t) * tcx::NBUCKET);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_group, tcx::NBUCKET);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_given, tcx::NBUCKET);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_given_chunk, sizeof(uint16_t) * tcx::NBUCKET);
    if (e == hipSuccess) e = hipMemset(ctx->d_chunk, 0, sizeof(uint16_t) * tcx::NBUCKET);
    if (e == hipSuccess) e = hipMemset(ctx->d_group, 0, tcx::NBUCKET);
    const size_t np = sizeof(float) * tcx::MLP_NPARAM;
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_master, np);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_adam_m, np);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_adam_v, np);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_grad, np);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_loss, sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_cw, sizeof(tcx::MlpCompute));
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_tile_master, np);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_cw_tile, sizeof(tcx::MlpCompute));
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_learned_tile, tcx::NBUCKET);
    if (e == hipSuccess && device < kMaxScratchDevices) {   // the fixed scratch's address on this device
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e == hipSuccess) g_scratch_ptr[device] = p;
        }
        ctx->d_scratch = g_scratch_ptr[device];
    }
    if (e != hipSuccess) {
        tc_destroy(ctx);
        return TC_ERR_HIP;
    }
    *out = ctx;
    return TC_OK;
}

tc_status tc_destroy(tc_ctx* ctx) {
    if (!ctx) return TC_ERR_INVALID_ARG;
    {
        DeviceGuard guard(ctx->device);
        for (int i = 0; i <= tcx::NSTAGE; ++i)
            if (ctx->events[i]) (void)hipEventDestroy(ctx->events[i]);
        if (ctx->h_ctrl) (void)hipHostFree(ctx->h_ctrl);
        if (ctx->d_learned) (void)hipFree(ctx->d_learned);
        if (ctx->d_chunk) (void)hipFree(ctx->d_chunk);
        if (ctx->d_group) (void)hipFree(ctx->d_group);
        if (ctx->d_given) (void)hipFree(ctx->d_given);
        if (ctx->d_given_chunk) (void)hipFree(ctx->d_given_chunk);
        float* bufs[] = {ctx->d_master, ctx->d_adam_m, ctx->d_adam_v, ctx->d_grad, ctx->d_loss, ctx->d_acts};
        for (float* p : bufs)
            if (p) (void)hipFree(p);
        if (ctx->d_cw) (void)hipFree(ctx->d_cw);
        if (ctx->d_tile_master) (void)hipFree(ctx->d_tile_master);
        if (ctx->d_cw_tile) (void)hipFree(ctx->d_cw_tile);
        if (ctx->d_learned_tile) (void)hipFree(ctx->d_learned_tile);
        if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
        if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
        if (ctx->h_counts_pinned) (void)hipHostFree(ctx->h_counts_pinned);
    }
    delete ctx;
    return TC_OK;
}

tc_status tc_workspace_size(int64_t num_edges, int32_t num_vertices, const tc_options* opts, size_t* bytes) {
    if (!bytes || num_edges < 0 || num_vertices < 0 || !options_ok(opts)) return TC_ERR_INVALID_ARG;
    if (num_edges > kMaxEdges) return TC_ERR_UNSUPPORTED;
    *bytes = tcx::make_layout(num_edges, num_vertices).total;
    return TC_OK;
}

tc_status tc_count_triangles(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                             void* d_workspace, size_t workspace_bytes, const tc_options* opts, uint64_t* h_count,
                             uint64_t* d_per_vertex) {
    if (!h_count) return arg_fail(ctx, TC_ERR_INVALID_ARG, "null count output");
    tcx::RunArgs ra = {};
    ra.per_vertex = d_per_vertex;
    tc_status st = run(ctx, d_edges, num_edges, num_vertices, d_workspace, workspace_bytes, opts, ra);
    if (st == TC_OK) *h_count = ctx->h_ctrl->total;
    return st;
}

tc_status tc_count_triangles_async(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                                   void* d_workspace, size_t workspace_bytes, const tc_options* opts,
                                   uint64_t* d_result, uint64_t* d_per_vertex) {
    if (!d_result) return arg_fail(ctx, TC_ERR_INVALID_ARG, "null result output");
    if (((uintptr_t)d_result & 7u) != 0) return arg_fail(ctx, TC_ERR_INVALID_ARG, "result must be 8-byte aligned");
    tcx::RunArgs ra = {};
    ra.per_vertex = d_per_vertex;
    return run(ctx, d_edges, num_edges, num_vertices, d_workspace, workspace_bytes, opts, ra, d_result);
}

tc_status tc_count_triangles_noalloc(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                                    const tc_options* opts, uint64_t* d_result, uint64_t* d_per_vertex) {
    if (!ctx) return TC_ERR_INVALID_ARG;
    if (num_edges < 0 || num_vertices < 0) return arg_fail(ctx, TC_ERR_INVALID_ARG, "negative size");
    if (num_edges > kMaxEdges) return arg_fail(ctx, TC_ERR_UNSUPPORTED, "num_edges must be below 2^31 - 2^20");
    if (tcx::make_layout(num_edges, num_vertices).total > (size_t)TC_NOALLOC_SCRATCH_BYTES)
        return arg_fail(ctx, TC_ERR_WORKSPACE, "graph needs more workspace than the fixed scratch holds "
                                               "(tc_workspace_size > TC_NOALLOC_SCRATCH_BYTES)");
    if (!ctx->d_scratch) return arg_fail(ctx, TC_ERR_UNSUPPORTED, "no fixed scratch on this device");
    return tc_count_triangles_async(ctx, d_edges, num_edges, num_vertices, ctx->d_scratch,
                                    (size_t)TC_NOALLOC_SCRATCH_BYTES, opts, d_result, d_per_vertex);
}

tc_status tc_formulation_workspace_size(int64_t num_edges, int32_t num_vertices, const tc_options* opts,
                                        int formulation, size_t* bytes) {
    if (!bytes || num_edges < 0 || num_vertices < 0 || !options_ok(opts)) return TC_ERR_INVALID_ARG;
    if (formulation < TC_FORM_FILTERED || formulation > TC_FORM_MATRIX_UPPER) return TC_ERR_INVALID_ARG;
    if (num_edges > kMaxEdges) return TC_ERR_UNSUPPORTED;
    const bool sym = formulation == TC_FORM_FULL || formulation == TC_FORM_MATRIX;
    *bytes = tcx::make_layout(num_edges, num_vertices).total +
             (sym ? tcx::sym_extra_bytes(num_edges, num_vertices) : 0);
    return TC_OK;
}

tc_status tc_count_triangles_formulation(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges,
                                         int32_t num_vertices, void* d_workspace, size_t workspace_bytes,
                                         const tc_options* opts, int formulation, uint64_t* h_count,
                                         uint64_t* h_sum) {
    if (!h_count) return arg_fail(ctx, TC_ERR_INVALID_ARG, "null count output");
    if (formulation < TC_FORM_FILTERED || formulation > TC_FORM_MATRIX_UPPER)
        return arg_fail(ctx, TC_ERR_INVALID_ARG, "unknown formulation");
    tcx::RunArgs ra = {};
    ra.formulation = formulation;
    tc_status st = run(ctx, d_edges, num_edges, num_vertices, d_workspace, workspace_bytes, opts, ra);
    if (st != TC_OK) return st;
    const uint64_t sum = ctx->h_ctrl->total;
    const uint64_t k = (uint64_t)tcx::form_multiple(formulation);
    if (sum % k) return arg_fail(ctx, TC_ERR_HIP, "internal bound violated");
    *h_count = sum / k;
    if (h_sum) *h_sum = sum;
    return TC_OK;
}

tc_status tc_clustering(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                        void* d_workspace, size_t workspace_bytes, const tc_options* opts, double* d_coeff,
                        uint64_t* d_per_vertex, uint64_t* h_count, uint64_t* h_wedges, double* h_transitivity) {
    if (!h_count || !h_wedges || !h_transitivity || (num_vertices > 0 && !d_coeff))
        return arg_fail(ctx, TC_ERR_INVALID_ARG, "null output");
    tcx::RunArgs ra = {};
    ra.clustering = d_coeff;
    ra.per_vertex = d_per_vertex;
    tc_status st = run(ctx, d_edges, num_edges, num_vertices, d_workspace, workspace_bytes, opts, ra);
    if (st != TC_OK) return st;
    if (num_edges == 0 && num_vertices > 0) {   // no edges: every degree is zero
        DeviceGuard guard(ctx->device);
        hipError_t e = hipMemsetAsync(d_coeff, 0, sizeof(double) * (size_t)num_vertices, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "zero coefficients");
    }
    const uint64_t T = ctx->h_ctrl->total, W = ctx->h_ctrl->wedges;
    *h_count = T;
    *h_wedges = W;
    *h_transitivity = W ? 3.0 * (double)T / (double)W : 0.0;
    return TC_OK;
}

tc_status tc_edge_counts(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                         void* d_workspace, size_t workspace_bytes, const tc_options* opts, int32_t* d_out_edges,
                         uint32_t* d_out_counts, int64_t* h_num_out, uint64_t* h_count) {
    if (!h_num_out || !h_count || (num_edges > 0 && (!d_out_edges || !d_out_counts)))
        return arg_fail(ctx, TC_ERR_INVALID_ARG, "null output");
    tcx::RunArgs ra = {};
    ra.per_edge_counts = d_out_counts;
    ra.per_edge_pairs = d_out_edges;
    tc_status st = run(ctx, d_edges, num_edges, num_vertices, d_workspace, workspace_bytes, opts, ra);
    if (st == TC_OK) {
        *h_num_out = ctx->h_ctrl->m;
        *h_count = ctx->h_ctrl->total;
    }
    return st;
}

tc_status tc_list_workspace_size(int64_t num_edges, int32_t num_vertices, const tc_options* opts, size_t* bytes) {
    if (!bytes || num_edges < 0 || num_vertices < 0 || !options_ok(opts)) return TC_ERR_INVALID_ARG;
    *bytes = tcx::make_layout(num_edges, num_vertices).total + tcx::list_extra_bytes(num_edges);
    return TC_OK;
}

tc_status tc_list_triangles(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                            void* d_workspace, size_t workspace_bytes, const tc_options* opts, int32_t* d_out,
                            int64_t capacity, uint64_t* h_count) {
    if (!h_count || capacity < 0 || (capacity > 0 && !d_out))
        return arg_fail(ctx, TC_ERR_INVALID_ARG, "null output or negative capacity");
    if (num_edges < 0 || num_vertices < 0) return arg_fail(ctx, TC_ERR_INVALID_ARG, "negative size");
    const size_t base = tcx::make_layout(num_edges, num_vertices).total;
    if (num_edges > 0 && workspace_bytes < base + tcx::list_extra_bytes(num_edges))
        return arg_fail(ctx, TC_ERR_WORKSPACE, "workspace below tc_list_workspace_size");
    char* ws = (char*)d_workspace;
    uint64_t* offs = (uint64_t*)(ws + base);
    uint32_t* cnt = (uint32_t*)(ws + base + tcx::align_up(8 * ((size_t)num_edges + 1), 256));
    // pass 1: the count and the per-edge counts
    tcx::RunArgs ra = {};
    ra.per_edge_counts = num_edges > 0 ? cnt : nullptr;
    tc_status st = run(ctx, d_edges, num_edges, num_vertices, d_workspace, workspace_bytes, opts, ra);
    if (st != TC_OK) return st;
    const uint64_t T = ctx->h_ctrl->total;
    *h_count = T;
    if (T == 0) return TC_OK;
    if (T > (uint64_t)capacity) return arg_fail(ctx, TC_ERR_WORKSPACE, "output capacity below the triangle count");
    // slot offsets per in-edge, then pass 2 writes the triangles
    DeviceGuard guard(ctx->device);
    const tcx::Layout L = tcx::make_layout(num_edges, num_vertices);
    const tcx::Ctrl* dctrl = (const tcx::Ctrl*)(ws + L.ctrl);
    const size_t m = ctx->h_ctrl->m;
    tcx::widen_u32_u64(cnt, offs, dctrl, (size_t)num_edges, ctx->stream);
    tcx::scan_exclusive_sum_u64(offs, offs, m, ws + L.scan_tmp, ctx->stream);
    tcx::fill_u32(cnt, 0u, m, ctx->stream);
    tcx::RunArgs r2 = ra;
    r2.per_edge_counts = nullptr;
    r2.events = nullptr;
    r2.list_off = offs;
    r2.list_cur = cnt;
    r2.list_out = d_out;
    r2.list_cap = (uint64_t)capacity;
    hipError_t e = tcx::run_list_pass(r2);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&ctx->h_ctrl->err, &dctrl->err, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "list triangles");
    if (ctx->h_ctrl->err) return arg_fail(ctx, TC_ERR_HIP, "internal: listing pass disagrees with the count");
    return TC_OK;
}

tc_status tc_edge_support(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                          void* d_workspace, size_t workspace_bytes, const tc_options* opts, int32_t* d_out_edges,
                          uint32_t* d_out_support, int64_t* h_num_out, uint64_t* h_count) {
    if (!h_num_out || !h_count || (num_edges > 0 && (!d_out_edges || !d_out_support)))
        return arg_fail(ctx, TC_ERR_INVALID_ARG, "null output");
    tcx::RunArgs ra = {};
    ra.support = d_out_support;
    ra.per_edge_pairs = d_out_edges;
    tc_status st = run(ctx, d_edges, num_edges, num_vertices, d_workspace, workspace_bytes, opts, ra);
    if (st == TC_OK) {
        *h_num_out = ctx->h_ctrl->m;
        *h_count = ctx->h_ctrl->total;
    }
    return st;
}

tc_status tc_build_csr(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                       void* d_workspace, size_t workspace_bytes, const tc_options* opts, int32_t* d_rank,
                       int64_t* d_offsets, int32_t* d_col, int64_t* h_num_out) {
    if (!h_num_out || !d_offsets || (num_vertices > 0 && !d_rank) || (num_edges > 0 && !d_col))
        return arg_fail(ctx, TC_ERR_INVALID_ARG, "null output");
    tcx::RunArgs ra = {};
    ra.csr_rank = d_rank;
    ra.csr_off = d_offsets;
    ra.csr_col = d_col;
    if (num_edges == 0) {
        // every vertex is isolated: identity ranks and empty rows
        if (!ctx) return TC_ERR_INVALID_ARG;
        if (num_vertices < 0) return arg_fail(ctx, TC_ERR_INVALID_ARG, "negative size");
        DeviceGuard guard(ctx->device);
        hipError_t e = hipMemsetAsync(d_offsets, 0, sizeof(int64_t) * ((size_t)num_vertices + 1), ctx->stream);
        if (e == hipSuccess && num_vertices > 0) {
            int32_t* h = new int32_t[num_vertices];
            for (int32_t i = 0; i < num_vertices; ++i) h[i] = i;
            e = hipMemcpyAsync(d_rank, h, sizeof(int32_t) * (size_t)num_vertices, hipMemcpyHostToDevice, ctx->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
            delete[] h;
        } else if (e == hipSuccess) {
            e = hipStreamSynchronize(ctx->stream);
        }
        if (e != hipSuccess) return hip_fail(ctx, e, "empty CSR");
        *h_num_out = 0;
        return TC_OK;
    }
    tc_status st = run(ctx, d_edges, num_edges, num_vertices, d_workspace, workspace_bytes, opts, ra);
    if (st == TC_OK) *h_num_out = ctx->h_ctrl->m;
    return st;
}

size_t tc_radix_sort_workspace_size(int64_t count) {
    return count > 0 ? tcx::radix_temp_bytes((size_t)count) : 0;
}

tc_status tc_radix_sort_u64(tc_ctx* ctx, uint64_t* d_keys, uint64_t* d_keys_alt, int64_t count, int32_t bit_lo,
                            int32_t bit_hi, void* d_workspace, size_t workspace_bytes) {
    if (!ctx) return TC_ERR_INVALID_ARG;
    ctx->last_error.clear();
    if (count < 0 || bit_lo < 0 || bit_hi > 64 || bit_lo > bit_hi) return arg_fail(ctx, TC_ERR_INVALID_ARG, "bad range");
    if (count > kMaxEdges) return arg_fail(ctx, TC_ERR_UNSUPPORTED, "count must be < 2^31");
    if (count == 0 || bit_lo == bit_hi) return TC_OK;
    if (!d_keys || !d_keys_alt || !d_workspace) return arg_fail(ctx, TC_ERR_INVALID_ARG, "null pointer");
    if (workspace_bytes < tcx::radix_temp_bytes((size_t)count))
        return arg_fail(ctx, TC_ERR_WORKSPACE, "workspace too small");
    DeviceGuard guard(ctx->device);
    uint32_t* d_err = tcx::radix_err_word(d_workspace, (size_t)count);
    tcx::fill_u32(d_err, 0u, 1, ctx->stream);
    const int alt = tcx::radix_sort_u64(d_keys, d_keys_alt, nullptr, nullptr, nullptr, (size_t)count, bit_lo, bit_hi,
                                        d_workspace, ctx->stream, false, false, d_err);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && alt)
        e = hipMemcpyAsync(d_keys, d_keys_alt, sizeof(uint64_t) * (size_t)count, hipMemcpyDeviceToDevice, ctx->stream);
    uint32_t h_err = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h_err, d_err, sizeof(h_err), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "radix sort");
    if (h_err) {   // a look-back wait ran out (an internal bound; never in a correct run)
        ctx->last_error = "radix sort: a look-back wait ran out";
        return TC_ERR_HIP;
    }
    return TC_OK;
}

tc_status tc_radix_partition_u64(tc_ctx* ctx, const uint64_t* d_in, uint64_t* d_out, int64_t count, int32_t shift,
                                 int32_t bits, void* d_workspace, size_t workspace_bytes) {
    if (!ctx) return TC_ERR_INVALID_ARG;
    ctx->last_error.clear();
    if (count < 0 || shift < 0 || bits < 1 || bits > 8 || shift + bits > 64)
        return arg_fail(ctx, TC_ERR_INVALID_ARG, "bad count, shift or bits");
    if (count > kMaxEdges) return arg_fail(ctx, TC_ERR_UNSUPPORTED, "count must be < 2^31");
    if (count == 0) return TC_OK;
    if (!d_in || !d_out || !d_workspace) return arg_fail(ctx, TC_ERR_INVALID_ARG, "null pointer");
    if ((const void*)d_in == (const void*)d_out) return arg_fail(ctx, TC_ERR_INVALID_ARG, "d_in and d_out must differ");
    if (workspace_bytes < tcx::radix_temp_bytes((size_t)count))
        return arg_fail(ctx, TC_ERR_WORKSPACE, "workspace too small");
    DeviceGuard guard(ctx->device);
    tcx::radix_pass_u64(d_in, d_out, (size_t)count, shift, bits, tcx::RadixXf{tcx::RX_NONE, nullptr, 0, 0, 0},
                        d_workspace, ctx->stream, nullptr, false);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "radix partition");
    return TC_OK;
}

tc_status tc_sort_runs_u64(tc_ctx* ctx, uint64_t* d_keys, uint64_t* d_tmp, int64_t count, int32_t shift) {
    if (!ctx) return TC_ERR_INVALID_ARG;
    ctx->last_error.clear();
    if (count < 0 || shift < 1 || shift > 32) return arg_fail(ctx, TC_ERR_INVALID_ARG, "bad count or shift");
    if (count > kMaxEdges) return arg_fail(ctx, TC_ERR_UNSUPPORTED, "count must be < 2^31");
    if (count == 0) return TC_OK;
    if (!d_keys || !d_tmp) return arg_fail(ctx, TC_ERR_INVALID_ARG, "null pointer");
    if ((uintptr_t)d_keys % 16 != 0) return arg_fail(ctx, TC_ERR_INVALID_ARG, "keys must be 16-byte aligned");
    DeviceGuard guard(ctx->device);
    tcx::sort_runs_u64(d_keys, d_tmp, (size_t)count, shift, false, 0ull, nullptr, 0u, ctx->stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "run sort");
    return TC_OK;
}

tc_status tc_last_stats(const tc_ctx* ctx, tc_stats* out) {
    if (!ctx || !out) return TC_ERR_INVALID_ARG;
    const tcx::Ctrl& c = *ctx->h_ctrl;
    memset(out, 0, sizeof(*out));
    out->num_edges_kept = c.m;
    out->num_pairs_valid = c.m_valid;
    out->num_tiles = c.ntiles;
    for (int k = 0; k <= tcx::NKERNEL; ++k) out->tile_begin[k] = c.tile_begin[k];
    for (int b = 0; b < tcx::NBUCKET; ++b) {
        out->bucket_vertices[b] = c.bucket_nv[b];
        out->bucket_in_edges[b] = c.bucket_in[b];
        out->bucket_out_edges[b] = c.bucket_out[b];
        out->bucket_work[b] = c.bucket_work[b];
        out->bucket_kernel[b] = c.choice[b];
        out->bucket_chunk[b] = c.chunk[b];
        out->bucket_group[b] = c.group[b];
    }
    return TC_OK;
}

tc_status tc_batch_workspace_size(int64_t total_edges, int64_t total_vertices, int32_t num_graphs,
                                  const tc_options* opts, size_t* bytes) {
    if (!bytes || total_edges < 0 || total_vertices < 0 || num_graphs < 0 || !options_ok(opts))
        return TC_ERR_INVALID_ARG;
    if (total_edges > kMaxEdges || total_vertices >= ((int64_t)1 << 31)) return TC_ERR_UNSUPPORTED;
    *bytes = tcx::make_batch_layout(total_edges, total_vertices, num_graphs).total;
    return TC_OK;
}

tc_status tc_count_triangles_batch(tc_ctx* ctx, const int32_t* d_edges, const int64_t* h_edge_offsets,
                                   const int32_t* h_num_vertices, int32_t num_graphs, void* d_workspace,
                                   size_t workspace_bytes, const tc_options* opts, uint64_t* h_counts) {
    if (!ctx) return TC_ERR_INVALID_ARG;
    ctx->last_error.clear();
    if (num_graphs < 0 || (num_graphs > 0 && (!h_edge_offsets || !h_num_vertices || !h_counts)))
        return arg_fail(ctx, TC_ERR_INVALID_ARG, "null argument");
    if (!options_ok(opts)) return arg_fail(ctx, TC_ERR_INVALID_ARG, "bad options");
    if (num_graphs == 0) return TC_OK;
    if (h_edge_offsets[0] != 0) return arg_fail(ctx, TC_ERR_INVALID_ARG, "edge_offsets[0] must be 0");
    if (h_edge_offsets[num_graphs] == 0) {   // no pairs at all: every count is zero
        for (int32_t g = 0; g < num_graphs; ++g) {
            if (h_num_vertices[g] < 0) return arg_fail(ctx, TC_ERR_INVALID_ARG, "vertex counts must be >= 0");
            h_counts[g] = 0;
        }
        return TC_OK;
    }
    int64_t N = 0;
    std::vector<int64_t> voff((size_t)num_graphs + 1);
    for (int32_t g = 0; g < num_graphs; ++g) {
        if (h_edge_offsets[g + 1] < h_edge_offsets[g] || h_num_vertices[g] < 0)
            return arg_fail(ctx, TC_ERR_INVALID_ARG, "edge offsets must not decrease; vertex counts >= 0");
        voff[g] = N;
        N += h_num_vertices[g];
    }
    voff[num_graphs] = N;
    const int64_t E = h_edge_offsets[num_graphs];
    if (E > kMaxEdges || N >= ((int64_t)1 << 31)) return arg_fail(ctx, TC_ERR_UNSUPPORTED, "batch too large");
    if (E > 0 && !d_edges) return arg_fail(ctx, TC_ERR_INVALID_ARG, "null edge list");
    if (((uintptr_t)d_edges & 7u) != 0) return arg_fail(ctx, TC_ERR_INVALID_ARG, "edge list must be 8-byte aligned");
    const tcx::BatchLayout B = tcx::make_batch_layout(E, N, num_graphs);
    if (!d_workspace || workspace_bytes < B.total) return arg_fail(ctx, TC_ERR_WORKSPACE, "workspace too small");
    const int sel = opts ? opts->select : TC_SELECT_HEURISTIC;
    if (sel == TC_SELECT_LEARNED && !ctx->learned_ready)
        return arg_fail(ctx, TC_ERR_INVALID_ARG, "no selector network loaded or trained");
    const bool capture = !(opts && (opts->flags & TC_F_NO_GRAPH));
    DeviceGuard guard(ctx->device);
    hipError_t e = hipSuccess;
    hipStream_t s = ctx->stream;
    if (!s) {   // the null stream cannot be captured: use the context's own stream
        if (!ctx->own_stream) e = hipStreamCreate(&ctx->own_stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "create stream");
        s = ctx->own_stream;
    }
    if ((size_t)num_graphs > ctx->h_counts_cap) {
        if (ctx->h_counts_pinned) (void)hipHostFree(ctx->h_counts_pinned);
        ctx->h_counts_pinned = nullptr;
        ctx->h_counts_cap = 0;
        e = hipHostMalloc((void**)&ctx->h_counts_pinned, sizeof(uint64_t) * (size_t)num_graphs, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(ctx, e, "pinned counts");
        ctx->h_counts_cap = (size_t)num_graphs;
    }
    char* ws = (char*)d_workspace;
    // graph descriptions and the edge list's address go to the device outside any
    // captured graph (the copies read pageable host memory before they return)
    e = hipMemcpyAsync(ws + B.eptr, &d_edges, sizeof(void*), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + B.eoff, h_edge_offsets, sizeof(int64_t) * ((size_t)num_graphs + 1),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + B.voff, voff.data(), sizeof(int64_t) * voff.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + B.nv, h_num_vertices, sizeof(int32_t) * (size_t)num_graphs, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy graph offsets");

    tcx::RunArgs ra = {};
    ra.stream = s;
    ra.ws = d_workspace;
    ra.select = sel;
    ra.mlp = ctx->learned_ready ? ctx->d_cw : nullptr;
    ra.learned = ctx->d_learned;
    ra.mlp_tile = ctx->tile_ready ? ctx->d_cw_tile : nullptr;
    ra.learned_tile = ctx->d_learned_tile;
    ra.chunk_override = ctx->d_chunk;
    ra.group_override = ctx->d_group;
    ra.grid_override = ctx->grid_override;
    tcx::BatchArgs ba = {d_edges, E, N, num_graphs};
    const bool same = ctx->graph_exec && ctx->graph_key.E == E && ctx->graph_key.N == N &&
                      ctx->graph_key.G == num_graphs && ctx->graph_key.select == sel &&
                      ctx->graph_key.ws == d_workspace;
    if (capture && !same) {
        if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
        if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
        ctx->graph_exec = nullptr;
        ctx->graph = nullptr;
        e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(ctx, e, "begin capture");
        hipError_t le = tcx::run_batch(ba, ra);
        e = hipStreamEndCapture(s, &ctx->graph);
        if (le != hipSuccess) e = le;
        if (e == hipSuccess) e = hipGraphInstantiate(&ctx->graph_exec, ctx->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return hip_fail(ctx, e, "capture batch");
        ctx->graph_key = {E, N, num_graphs, sel, d_workspace};
    }
    if (capture) e = hipGraphLaunch(ctx->graph_exec, s);
    else e = tcx::run_batch(ba, ra);
    if (e != hipSuccess) return hip_fail(ctx, e, "launch batch");
    e = hipMemcpyAsync(ctx->h_ctrl, ws + B.pipe.ctrl, sizeof(tcx::Ctrl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->h_counts_pinned, ws + B.counts, sizeof(uint64_t) * (size_t)num_graphs,
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(ctx, e, "read batch counts");
    ctx->have_times = 0;
    if (ctx->h_ctrl->err & 1u) return arg_fail(ctx, TC_ERR_VERTEX_RANGE, "vertex id outside its graph's range");
    if (ctx->h_ctrl->err) return arg_fail(ctx, TC_ERR_HIP, "internal bound violated");
    memcpy(h_counts, ctx->h_counts_pinned, sizeof(uint64_t) * (size_t)num_graphs);
    return TC_OK;
}

tc_status tc_set_tile_shapes(tc_ctx* ctx, const uint16_t* h_chunk, const uint8_t* h_group) {
    if (!ctx) return TC_ERR_INVALID_ARG;
    DeviceGuard guard(ctx->device);
    std::vector<uint16_t> c(tcx::NBUCKET, 0);
    std::vector<uint8_t> g(tcx::NBUCKET, 0);
    if (h_chunk) memcpy(c.data(), h_chunk, sizeof(uint16_t) * tcx::NBUCKET);
    if (h_group) memcpy(g.data(), h_group, tcx::NBUCKET);
    hipError_t e = hipMemcpy(ctx->d_chunk, c.data(), sizeof(uint16_t) * tcx::NBUCKET, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_group, g.data(), tcx::NBUCKET, hipMemcpyHostToDevice);
    return e == hipSuccess ? TC_OK : hip_fail(ctx, e, "set tile shapes");
}

tc_status tc_bucket_features(const tc_ctx* ctx, float* h_features) {
    if (!ctx || !h_features) return TC_ERR_INVALID_ARG;
    memcpy(h_features, ctx->h_ctrl->features, sizeof(ctx->h_ctrl->features));
    return TC_OK;
}

// Lay out the tiles under selection mode `select`, then time each busy bucket's
// tiles alone with the kernel the mode chose for it (median of `repeats`).
// ms_row(kernel) gives the output row for a kernel.
static tc_status profile_pass(tc_ctx* ctx, const int32_t* d_edges, int64_t E, int32_t n, void* ws, size_t ws_bytes,
                              int select, int32_t repeats, float* h_ms, bool row_per_kernel, float* h_features) {
    tc_options o = {};
    o.select = select;
    tcx::RunArgs ra = {};
    ra.stop_before_isect = 1;
    tc_status st = run(ctx, d_edges, E, n, ws, ws_bytes, &o, ra);
    if (st != TC_OK) return st;
    if (h_features) memcpy(h_features, ctx->h_ctrl->features, sizeof(ctx->h_ctrl->features));
    DeviceGuard guard(ctx->device);
    const tcx::Layout L = tcx::make_layout(E, n);
    std::vector<uint32_t> tstart((size_t)n + 1);
    hipError_t e = hipMemcpy(tstart.data(), (char*)ws + L.tstart, sizeof(uint32_t) * tstart.size(),
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "read tile starts");
    const tcx::Ctrl c = *ctx->h_ctrl;
    for (int b = 0; b < tcx::NBUCKET - 1; ++b) {
        if (c.bucket_nv[b] == 0 || c.bend[b] <= c.bstart[b]) continue;
        const uint32_t t0 = tstart[c.bstart[b]], t1 = tstart[c.bend[b]];
        if (t1 <= t0) continue;
        const int k = c.choice[b];
        std::vector<float> ms;
        for (int r = 0; r < repeats; ++r) {
            (void)hipEventRecord(ctx->events[0], ctx->stream);
            e = tcx::launch_isect_range(ra, k, t0, t1);
            (void)hipEventRecord(ctx->events[1], ctx->stream);
            if (e == hipSuccess) e = hipEventSynchronize(ctx->events[1]);
            float t = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, ctx->events[0], ctx->events[1]);
            if (e != hipSuccess) return hip_fail(ctx, e, "profile launch");
            ms.push_back(t);
        }
        std::sort(ms.begin(), ms.end());
        h_ms[(row_per_kernel ? k * tcx::NBUCKET : 0) + b] = ms[ms.size() / 2];
    }
    return TC_OK;
}

tc_status tc_profile_buckets(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                             void* d_workspace, size_t workspace_bytes, int32_t repeats, float* h_ms,
                             float* h_features) {
    if (!ctx || !h_ms || repeats < 1 || repeats > 64) return arg_fail(ctx, TC_ERR_INVALID_ARG, "bad arguments");
    for (int i = 0; i < tcx::NKERNEL * tcx::NBUCKET; ++i) h_ms[i] = -1.f;
    if (num_edges == 0) return TC_OK;
    for (int k = 0; k < tcx::NKERNEL; ++k) {   // merge, bsearch, bitmap follow in order
        tc_status st = profile_pass(ctx, d_edges, num_edges, num_vertices, d_workspace, workspace_bytes,
                                    TC_FORCE_MERGE + k, repeats, h_ms, true, k == 0 ? h_features : nullptr);
        if (st != TC_OK) return st;
    }
    return TC_OK;
}

tc_status tc_profile_selected(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                              void* d_workspace, size_t workspace_bytes, const tc_options* opts, int32_t repeats,
                              float* h_ms) {
    if (!ctx || !h_ms || repeats < 1 || repeats > 64 || !options_ok(opts))
        return arg_fail(ctx, TC_ERR_INVALID_ARG, "bad arguments");
    for (int i = 0; i < tcx::NBUCKET; ++i) h_ms[i] = -1.f;
    if (num_edges == 0) return TC_OK;
    return profile_pass(ctx, d_edges, num_edges, num_vertices, d_workspace, workspace_bytes,
                        opts ? opts->select : TC_SELECT_HEURISTIC, repeats, h_ms, false, nullptr);
}

tc_status tc_profile_choices(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                             void* d_workspace, size_t workspace_bytes, const uint8_t* h_choice,
                             const uint16_t* h_chunk, int32_t repeats, float* h_ms, uint64_t* h_count) {
    if (!ctx || !h_choice || !h_ms || repeats < 1 || repeats > 64)
        return arg_fail(ctx, TC_ERR_INVALID_ARG, "bad arguments");
    for (int i = 0; i < 1 + tcx::NKERNEL; ++i) h_ms[i] = 0.f;
    if (h_count) *h_count = 0;
    if (num_edges == 0) return TC_OK;
    DeviceGuard guard(ctx->device);
    std::vector<uint16_t> chunk(tcx::NBUCKET, 0);
    if (h_chunk) memcpy(chunk.data(), h_chunk, sizeof(uint16_t) * tcx::NBUCKET);
    hipError_t e = hipMemcpy(ctx->d_given, h_choice, tcx::NBUCKET, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(ctx->d_given_chunk, chunk.data(), sizeof(uint16_t) * tcx::NBUCKET, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy choices");
    tc_options o = {};
    tcx::RunArgs ra = {};
    ra.stop_before_isect = 1;
    ra.given = ctx->d_given;
    ra.chunk_override = ctx->d_given_chunk;
    tc_status st = run(ctx, d_edges, num_edges, num_vertices, d_workspace, workspace_bytes, &o, ra);
    if (st != TC_OK) return st;
    std::vector<float> ms[1 + tcx::NKERNEL];
    for (int r = 0; r < repeats; ++r) {
        e = tcx::launch_isect_stage(ra, ctx->events);
        if (e == hipSuccess) e = hipEventSynchronize(ctx->events[tcx::NKERNEL]);
        float tot = 0.f;
        for (int k = 0; k < tcx::NKERNEL && e == hipSuccess; ++k) {
            float t = 0.f;
            e = hipEventElapsedTime(&t, ctx->events[k], ctx->events[k + 1]);
            ms[1 + k].push_back(t);
            tot += t;
        }
        if (e != hipSuccess) return hip_fail(ctx, e, "profile intersection stage");
        ms[0].push_back(tot);
    }
    for (int i = 0; i < 1 + tcx::NKERNEL; ++i) {
        std::sort(ms[i].begin(), ms[i].end());
        h_ms[i] = ms[i][ms[i].size() / 2];
    }
    e = hipMemcpyAsync(ctx->h_ctrl, (char*)d_workspace + tcx::make_layout(num_edges, num_vertices).ctrl,
                       sizeof(tcx::Ctrl), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "read control block");
    if (ctx->h_ctrl->err) return arg_fail(ctx, TC_ERR_HIP, "internal bound violated");
    if (h_count) *h_count = ctx->h_ctrl->total;
    return TC_OK;
}

static tc_status ensure_acts(tc_ctx* ctx) {
    if (ctx->d_acts) return TC_OK;
    const size_t per = 4 * tcx::MLP_H + tcx::MLP_OUT + 1;
    hipError_t e = hipMalloc((void**)&ctx->d_acts, sizeof(float) * per * tcx::MLP_MAX_BATCH);
    return e == hipSuccess ? TC_OK : hip_fail(ctx, e, "selector buffers");
}

static tcx::MlpActs acts_of(tc_ctx* ctx, int B) {
    tcx::MlpActs a;
    float* p = ctx->d_acts;
    a.h1 = p; p += (size_t)B * tcx::MLP_H;
    a.h2 = p; p += (size_t)B * tcx::MLP_H;
    a.dh1 = p; p += (size_t)B * tcx::MLP_H;
    a.dh2 = p; p += (size_t)B * tcx::MLP_H;
    a.dz = p; p += (size_t)B * tcx::MLP_OUT;
    a.loss = p;
    return a;
}

tc_status tc_selector_set_params(tc_ctx* ctx, const float* h_params) {
    if (!ctx || !h_params) return TC_ERR_INVALID_ARG;
    DeviceGuard guard(ctx->device);
    const size_t np = sizeof(float) * tcx::MLP_NPARAM;
    hipError_t e = hipMemcpyAsync(ctx->d_master, h_params, np, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->d_adam_m, 0, np, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->d_adam_v, 0, np, ctx->stream);
    if (e == hipSuccess) {
        tcx::mlp_cast(ctx->d_master, ctx->d_cw, ctx->stream);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "set selector parameters");
    ctx->adam_step = 0;
    ctx->learned_ready = 1;
    return TC_OK;
}

tc_status tc_selector_set_tile_params(tc_ctx* ctx, const float* h_params) {
    if (!ctx) return TC_ERR_INVALID_ARG;
    if (!h_params) {
        ctx->tile_ready = 0;
        return TC_OK;
    }
    DeviceGuard guard(ctx->device);
    hipError_t e = hipMemcpyAsync(ctx->d_tile_master, h_params, sizeof(float) * tcx::MLP_NPARAM,
                                  hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) {
        tcx::mlp_cast(ctx->d_tile_master, ctx->d_cw_tile, ctx->stream);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "set tile network parameters");
    ctx->tile_ready = 1;
    return TC_OK;
}

tc_status tc_selector_get_tile_params(tc_ctx* ctx, float* h_params) {
    if (!ctx || !h_params) return TC_ERR_INVALID_ARG;
    if (!ctx->tile_ready) return arg_fail(ctx, TC_ERR_INVALID_ARG, "no tile network parameters set");
    DeviceGuard guard(ctx->device);
    hipError_t e = hipMemcpyAsync(h_params, ctx->d_tile_master, sizeof(float) * tcx::MLP_NPARAM,
                                  hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    return e == hipSuccess ? TC_OK : hip_fail(ctx, e, "get tile network parameters");
}

tc_status tc_selector_get_params(tc_ctx* ctx, float* h_params) {
    if (!ctx || !h_params) return TC_ERR_INVALID_ARG;
    if (!ctx->learned_ready) return arg_fail(ctx, TC_ERR_INVALID_ARG, "no selector parameters set");
    DeviceGuard guard(ctx->device);
    hipError_t e = hipMemcpyAsync(h_params, ctx->d_master, sizeof(float) * tcx::MLP_NPARAM, hipMemcpyDeviceToHost,
                                  ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    return e == hipSuccess ? TC_OK : hip_fail(ctx, e, "get selector parameters");
}

// ---- selector parameter files
namespace {
// The numbers of the array after "key": in text (the first such key).
bool json_floats(const std::string& text, const char* key, std::vector<float>& out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = text.find(k);
    if (p == std::string::npos) return false;
    p = text.find_first_not_of(" \t\r\n", p + k.size());
    if (p == std::string::npos || text[p] != ':') return false;
    p = text.find_first_not_of(" \t\r\n", p + 1);
    if (p == std::string::npos || text[p] != '[') return false;
    out.clear();
    const char* base = text.c_str();
    ++p;
    for (;;) {
        p = text.find_first_not_of(" \t\r\n", p);
        if (p == std::string::npos) return false;
        if (text[p] == ']') return true;
        char* end = nullptr;
        const float v = strtof(base + p, &end);
        if (end == base + p) return false;
        out.push_back(v);
        p = text.find_first_not_of(" \t\r\n", (size_t)(end - base));
        if (p == std::string::npos) return false;
        if (text[p] == ',') ++p;
        else if (text[p] != ']') return false;
    }
}

bool write_floats(FILE* f, const char* key, const std::vector<float>& v) {
    if (fprintf(f, "\"%s\": [", key) < 0) return false;
    for (size_t i = 0; i < v.size(); ++i)
        if (fprintf(f, i ? ", %.9g" : "%.9g", (double)v[i]) < 0) return false;
    return fprintf(f, "]") >= 0;
}
}  // namespace

tc_status tc_selector_load(tc_ctx* ctx, const char* path) {
    if (!ctx) return TC_ERR_INVALID_ARG;
    ctx->last_error.clear();
    if (!path) return arg_fail(ctx, TC_ERR_INVALID_ARG, "null path");
    FILE* f = fopen(path, "rb");
    if (!f) return arg_fail(ctx, TC_ERR_INVALID_ARG, "cannot open the selector parameter file");
    std::string text;
    char buf[65536];
    size_t got;
    while ((got = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    const bool read_ok = !ferror(f);
    fclose(f);
    if (!read_ok) return arg_fail(ctx, TC_ERR_INVALID_ARG, "cannot read the selector parameter file");
    if (text.find("\"tc-selector-v1\"") == std::string::npos)
        return arg_fail(ctx, TC_ERR_INVALID_ARG, "not a tc-selector-v1 parameter file");
    std::vector<float> p, t;
    if (!json_floats(text, "params", p) || p.size() != (size_t)tcx::MLP_NPARAM)
        return arg_fail(ctx, TC_ERR_INVALID_ARG, "params: not TC_SELECTOR_NUM_PARAMS numbers");
    const bool has_tile = text.find("\"tile_params\"") != std::string::npos;
    if (has_tile && (!json_floats(text, "tile_params", t) || t.size() != (size_t)tcx::MLP_NPARAM))
        return arg_fail(ctx, TC_ERR_INVALID_ARG, "tile_params: not TC_SELECTOR_NUM_PARAMS numbers");
    const tc_status st = tc_selector_set_params(ctx, p.data());
    if (st != TC_OK) return st;
    return tc_selector_set_tile_params(ctx, has_tile ? t.data() : nullptr);
}

tc_status tc_selector_save(tc_ctx* ctx, const char* path) {
    if (!ctx) return TC_ERR_INVALID_ARG;
    ctx->last_error.clear();
    if (!path) return arg_fail(ctx, TC_ERR_INVALID_ARG, "null path");
    std::vector<float> p(tcx::MLP_NPARAM), t;
    tc_status st = tc_selector_get_params(ctx, p.data());
    if (st != TC_OK) return st;
    if (ctx->tile_ready) {
        t.resize(tcx::MLP_NPARAM);
        st = tc_selector_get_tile_params(ctx, t.data());
        if (st != TC_OK) return st;
    }
    FILE* f = fopen(path, "wb");
    if (!f) return arg_fail(ctx, TC_ERR_INVALID_ARG, "cannot open the file for writing");
    bool ok = fprintf(f, "{\"format\": \"tc-selector-v1\", \"num_params\": %d, ", (int)tcx::MLP_NPARAM) >= 0;
    ok = ok && write_floats(f, "params", p) && fprintf(f, ", \"meta\": {}") >= 0;
    if (ok && !t.empty()) ok = fprintf(f, ", ") >= 0 && write_floats(f, "tile_params", t);
    ok = ok && fprintf(f, "}\n") >= 0;
    ok = (fclose(f) == 0) && ok;
    if (!ok) return arg_fail(ctx, TC_ERR_INVALID_ARG, "cannot write the selector parameter file");
    return TC_OK;
}

tc_status tc_selector_forward(tc_ctx* ctx, const float* d_x, int32_t batch, float* d_logits) {
    if (!ctx || batch < 0 || (batch > 0 && (!d_x || !d_logits))) return TC_ERR_INVALID_ARG;
    if (!ctx->learned_ready) return arg_fail(ctx, TC_ERR_INVALID_ARG, "no selector parameters set");
    DeviceGuard guard(ctx->device);
    tcx::mlp_forward(ctx->d_cw, d_x, batch, d_logits, ctx->stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    return e == hipSuccess ? TC_OK : hip_fail(ctx, e, "selector forward");
}

static tc_status selector_grad(tc_ctx* ctx, const float* d_x, const int32_t* d_labels, const float* d_weights,
                               int32_t batch, float* h_loss) {
    if (!ctx || batch < 1 || batch > tcx::MLP_MAX_BATCH || !d_x || !d_labels) return TC_ERR_INVALID_ARG;
    if (!ctx->learned_ready) return arg_fail(ctx, TC_ERR_INVALID_ARG, "no selector parameters set");
    tc_status st = ensure_acts(ctx);
    if (st != TC_OK) return st;
    tcx::mlp_gradient(ctx->d_cw, d_x, d_labels, d_weights, batch, acts_of(ctx, batch), ctx->d_grad, ctx->d_loss,
                      ctx->stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && h_loss)
        e = hipMemcpyAsync(h_loss, ctx->d_loss, sizeof(float), hipMemcpyDeviceToHost, ctx->stream);
    return e == hipSuccess ? TC_OK : hip_fail(ctx, e, "selector gradient");
}

tc_status tc_selector_gradient(tc_ctx* ctx, const float* d_x, const int32_t* d_labels, const float* d_weights,
                               int32_t batch, float* d_grad, float* h_loss) {
    if (!ctx) return TC_ERR_INVALID_ARG;
    DeviceGuard guard(ctx->device);
    tc_status st = selector_grad(ctx, d_x, d_labels, d_weights, batch, h_loss);
    if (st != TC_OK) return st;
    hipError_t e = hipSuccess;
    if (d_grad)
        e = hipMemcpyAsync(d_grad, ctx->d_grad, sizeof(float) * tcx::MLP_NPARAM, hipMemcpyDeviceToDevice,
                           ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    return e == hipSuccess ? TC_OK : hip_fail(ctx, e, "selector gradient");
}

tc_status tc_selector_train_step(tc_ctx* ctx, const float* d_x, const int32_t* d_labels, const float* d_weights,
                                 int32_t batch, float lr, float* h_loss) {
    if (!ctx || !(lr > 0.f)) return TC_ERR_INVALID_ARG;
    DeviceGuard guard(ctx->device);
    tc_status st = selector_grad(ctx, d_x, d_labels, d_weights, batch, h_loss);
    if (st != TC_OK) return st;
    ctx->adam_step += 1;
    tcx::mlp_adam(ctx->d_master, ctx->d_grad, ctx->d_adam_m, ctx->d_adam_v, lr, ctx->adam_step, ctx->stream);
    tcx::mlp_cast(ctx->d_master, ctx->d_cw, ctx->stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    return e == hipSuccess ? TC_OK : hip_fail(ctx, e, "selector train step");
}

int32_t tc_stage_times(const tc_ctx* ctx, float* ms, int32_t cap) {
    if (!ctx || !ms || !ctx->have_times) return 0;
    int32_t k = cap < tcx::NSTAGE ? cap : tcx::NSTAGE;
    for (int32_t i = 0; i < k; ++i) ms[i] = ctx->stage_ms[i];
    return k;
}

const char* tc_stage_name(int32_t stage) { return tcx::stage_name(stage); }

const char* tc_status_string(tc_status s) {
    switch (s) {
        case TC_OK: return "ok";
        case TC_ERR_INVALID_ARG: return "invalid argument";
        case TC_ERR_VERTEX_RANGE: return "vertex id out of range";
        case TC_ERR_WORKSPACE: return "workspace too small";
        case TC_ERR_HIP: return "HIP runtime error";
        case TC_ERR_UNSUPPORTED: return "unsupported size";
    }
    return "unknown status";
}

const char* tc_last_error(const tc_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

}  // extern "C"
