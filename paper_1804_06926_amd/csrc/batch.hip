// Batched counting: many graphs as one disjoint union.
//
// Triangles never span two components, so the union's count splits exactly
// by graph. Each graph's vertices get a contiguous id range; the ordinary
// pipeline runs once on the union and the intersection kernels also
// accumulate, per middle vertex, the triangles in which it is the middle
// vertex of the (degree, id) order (every triangle has exactly one). The
// count of graph g is the sum of those values over g's id range, taken in a
// fixed order by one block per graph.
#include "common.h"
#include "internal.h"
#include "pipeline.h"

namespace tcx {

constexpr int BT_NT = 256;
constexpr int BT_EDGES_PER_BLOCK = 4096;

// Local pair -> union pair; ids outside [0, n_g) become (-1, -1), which the
// pipeline reports as out of range and drops. The caller's edge list is read
// through a pointer held in the workspace (written before each launch), so a
// captured graph serves any edge buffer of the same sizes.
__global__ __launch_bounds__(BT_NT) void k_union_edges(const int2* const* __restrict__ edges_at, uint64_t E,
                                                       const int64_t* __restrict__ eoff, int32_t G,
                                                       const int32_t* __restrict__ nv,
                                                       const int64_t* __restrict__ voff, int2* __restrict__ out) {
    __shared__ int32_t s_g0;
    const uint64_t c0 = (uint64_t)blockIdx.x * BT_EDGES_PER_BLOCK;
    if (c0 >= E) return;
    if (threadIdx.x == 0) {   // graph of the chunk's first edge: largest g with eoff[g] <= c0
        int32_t lo = 0, hi = G - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if ((uint64_t)eoff[mid] <= c0) lo = mid;
            else hi = mid - 1;
        }
        s_g0 = lo;
    }
    __syncthreads();
    const int2* __restrict__ edges = *edges_at;
    int32_t g = s_g0;
    const uint64_t c1 = c0 + BT_EDGES_PER_BLOCK < E ? c0 + BT_EDGES_PER_BLOCK : E;
    for (uint64_t i = c0 + threadIdx.x; i < c1; i += BT_NT) {
        while (g + 1 < G && (uint64_t)eoff[g + 1] <= i) ++g;
        const int2 e = edges[i];
        const int32_t n = nv[g];
        const int64_t base = voff[g];
        const bool ok = e.x >= 0 && e.x < n && e.y >= 0 && e.y < n;
        out[i] = ok ? make_int2((int)(base + e.x), (int)(base + e.y)) : make_int2(-1, -1);
    }
}

// counts[g] = sum of middle counts over g's vertex range.
__global__ __launch_bounds__(BT_NT) void k_graph_sums(const uint64_t* __restrict__ middle,
                                                      const int64_t* __restrict__ voff, int32_t G,
                                                      uint64_t* __restrict__ counts) {
    __shared__ uint64_t red[BT_NT / WAVE];
    for (int32_t g = blockIdx.x; g < G; g += gridDim.x) {
        uint64_t acc = 0;
        for (int64_t v = voff[g] + threadIdx.x; v < voff[g + 1]; v += BT_NT) acc += middle[v];
        acc = wave_sum_u64(acc);
        if (lane_id() == 0) red[wave_id()] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t s = 0;
            for (int k = 0; k < BT_NT / WAVE; ++k) s += red[k];
            counts[g] = s;
        }
        __syncthreads();
    }
}

BatchLayout make_batch_layout(int64_t E, int64_t N, int32_t G) {
    BatchLayout B;
    B.pipe = make_layout(E, (int32_t)N);
    size_t o = B.pipe.total;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + (bytes ? bytes : 1), 256); return r; };
    B.union_edges = take(8 * (size_t)E);
    B.eptr = take(sizeof(void*));
    B.eoff = take(8 * ((size_t)G + 1));
    B.voff = take(8 * ((size_t)G + 1));
    B.nv = take(4 * (size_t)G);
    B.middle = take(8 * (size_t)N);
    B.counts = take(8 * (size_t)G);
    B.total = o;
    return B;
}

hipError_t run_batch(const BatchArgs& b, RunArgs& r) {
    char* ws = (char*)r.ws;
    const BatchLayout B = make_batch_layout(b.E, b.N, b.G);
    int2* uedges = (int2*)(ws + B.union_edges);
    const unsigned nblk = (unsigned)((b.E + BT_EDGES_PER_BLOCK - 1) / BT_EDGES_PER_BLOCK);
    if (b.E > 0)
        hipLaunchKernelGGL(k_union_edges, dim3(nblk), dim3(BT_NT), 0, r.stream, (const int2* const*)(ws + B.eptr),
                           (uint64_t)b.E,
                           (const int64_t*)(ws + B.eoff), b.G, (const int32_t*)(ws + B.nv),
                           (const int64_t*)(ws + B.voff), uedges);
    r.edges = (const int32_t*)uedges;
    r.E = b.E;
    r.n = (int32_t)b.N;
    r.per_middle = (uint64_t*)(ws + B.middle);
    RunResult rr;
    hipError_t e = run_pipeline(r, &rr);
    if (e != hipSuccess) return e;
    unsigned g = (unsigned)(b.G < 4096 ? b.G : 4096);
    hipLaunchKernelGGL(k_graph_sums, dim3(g > 0 ? g : 1), dim3(BT_NT), 0, r.stream, (const uint64_t*)(ws + B.middle),
                       (const int64_t*)(ws + B.voff), b.G, (uint64_t*)(ws + B.counts));
    return hipGetLastError();
}

}  // namespace tcx
