// The counting pipeline on one stream: edge-list generation and filtering,
// CSR construction, degree-pair bucketing, kernel selection and intersection.
//
// Stages (Algorithm 2; Section 4.2 for the filter, the induced subgraph and
// dynamic grouping):
//   degree    validate ids, canonicalise, count incidences (self-loops dropped)
//   rank      sort vertices by (degree, id): rank = position
//   orient    keep each pair once as (rank lo, rank hi), compacted
//   sort      radix sort of the oriented pairs -> rows contiguous, ascending
//   csr       drop repeated pairs, emit col/src and row offsets
//   bucket    per middle vertex v: (in-edges with a non-empty tail, |N+(v)|)
//   select    choose the intersection strategy and tile shape per bucket
//   group     order vertices by (strategy, bucket); lay out in-edge segments
//             and tiles; scatter in-edges into their segments
//   isect     the three intersection kernels, each over its tile range
//   finish    map per-vertex / per-edge outputs back to original ids
#include <string.h>

#include "common.h"
#include "internal.h"
#include "isect.h"
#include "pipeline.h"

namespace tcx {

constexpr int NT = 256;

static unsigned grid_for(size_t n, unsigned cap = 16384) {
    size_t g = (n + NT - 1) / NT;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// ------------------------------------------------------------------ degree
__global__ __launch_bounds__(NT) void k_degree(const int2* __restrict__ edges, uint64_t E, int32_t n,
                                               uint32_t* __restrict__ deg, Ctrl* ctrl) {
    bool bad = false;
    for (uint64_t i = (uint64_t)blockIdx.x * NT + threadIdx.x; i < E; i += (uint64_t)gridDim.x * NT) {
        const int2 e = edges[i];
        if (e.x < 0 || e.x >= n || e.y < 0 || e.y >= n) { bad = true; continue; }
        if (e.x == e.y) continue;
        atomicAdd(&deg[e.x], 1u);
        atomicAdd(&deg[e.y], 1u);
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(&ctrl->err, 1u);
}

__global__ __launch_bounds__(NT) void k_vertex_keys(const uint32_t* __restrict__ deg, int32_t n,
                                                    uint64_t* __restrict__ keys) {
    for (int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x; v < n; v += (int64_t)gridDim.x * NT)
        keys[v] = ((uint64_t)deg[v] << 32) | (uint32_t)v;
}

__global__ __launch_bounds__(NT) void k_rank(const uint64_t* __restrict__ sorted, int32_t n,
                                             uint32_t* __restrict__ rank, uint32_t* __restrict__ inv) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const uint32_t v = (uint32_t)sorted[i];
        rank[v] = (uint32_t)i;
        inv[i] = v;
    }
}

// ------------------------------------------------------------------ orient (filter by degree order)
// Pairs become (lo rank << nb) | hi rank; loops and invalid ids are dropped.
// Compaction: one atomic per wave reserves room for the wave's valid pairs.
__global__ __launch_bounds__(NT) void k_orient(const int2* __restrict__ edges, uint64_t E, int32_t n,
                                               const uint32_t* __restrict__ rank, int nb,
                                               uint64_t* __restrict__ keys, Ctrl* ctrl) {
    const uint64_t stride = (uint64_t)gridDim.x * NT;
    const uint64_t first = (uint64_t)blockIdx.x * NT + (threadIdx.x & ~(uint64_t)(WAVE - 1));
    for (uint64_t wbase = first; wbase < E; wbase += stride) {
        const uint64_t i = wbase + lane_id();
        bool valid = false;
        uint64_t key = 0;
        if (i < E) {
            const int2 e = edges[i];
            if (e.x >= 0 && e.x < n && e.y >= 0 && e.y < n && e.x != e.y) {
                const uint32_t a = rank[e.x], b = rank[e.y];
                const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
                key = ((uint64_t)lo << nb) | hi;
                valid = true;
            }
        }
        const uint64_t mask = __ballot(valid);
        uint32_t base = 0;
        if (lane_id() == 0 && mask) base = atomicAdd(&ctrl->m_valid, (uint32_t)__popcll(mask));
        base = __shfl(base, 0, WAVE);
        if (valid) keys[base + __popcll(mask & lanes_below())] = key;
    }
}

// ------------------------------------------------------------------ unique + CSR
constexpr int UQ_MAX_BLOCKS = 1024;

__global__ __launch_bounds__(NT) void k_unique_count(const uint64_t* __restrict__ keys, const Ctrl* ctrl,
                                                     uint32_t chunk, uint32_t* __restrict__ partial, uint32_t nblk) {
    const uint32_t mv = ctrl->m_valid;
    const uint64_t b0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t b1 = b0 + chunk < mv ? b0 + chunk : mv;
    uint32_t c = 0;
    for (uint64_t i = b0 + threadIdx.x; i < b1; i += NT) c += (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
    c = wave_sum(c);
    __shared__ uint32_t red[NT / WAVE];
    if (lane_id() == 0) red[wave_id()] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int k = 0; k < NT / WAVE; ++k) s += red[k];
        partial[blockIdx.x] = s;
        if (blockIdx.x == 0) partial[nblk] = 0;
    }
}

__global__ __launch_bounds__(NT) void k_unique_write(const uint64_t* __restrict__ keys, Ctrl* ctrl, uint32_t chunk,
                                                     const uint32_t* __restrict__ partial, uint32_t nblk, int nb,
                                                     uint32_t* __restrict__ col, uint32_t* __restrict__ src,
                                                     uint32_t* __restrict__ rowend) {
    __shared__ uint32_t scratch[NT / WAVE];
    const uint32_t mv = ctrl->m_valid;
    const uint64_t b0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t b1 = b0 + chunk < mv ? b0 + chunk : mv;
    const uint64_t lowmask = (nb >= 64) ? ~0ull : ((1ull << nb) - 1ull);
    uint32_t carry = partial[blockIdx.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->m = partial[nblk];
    for (uint64_t base = b0; base < b1; base += NT) {
        const uint64_t i = base + threadIdx.x;
        const bool valid = i < b1;
        uint64_t key = 0;
        uint32_t keep = 0;
        if (valid) {
            key = keys[i];
            keep = (i == 0 || key != keys[i - 1]) ? 1u : 0u;
        }
        uint32_t total;
        const uint32_t excl = block_exclusive_scan<NT>(keep, scratch, &total);
        if (valid) {
            const uint32_t s = (uint32_t)(key >> nb);
            const uint32_t pos = carry + excl;
            if (keep) {
                col[pos] = (uint32_t)(key & lowmask);
                src[pos] = s;
            }
            if (i + 1 == mv || (uint32_t)(keys[i + 1] >> nb) != s) rowend[s] = pos + keep;
        }
        carry += total;
    }
}

// ------------------------------------------------------------------ buckets
__global__ __launch_bounds__(NT) void k_indeg(const uint32_t* __restrict__ col, const uint32_t* __restrict__ src,
                                              const uint32_t* __restrict__ off, const Ctrl* ctrl,
                                              uint32_t* __restrict__ indeg) {
    const uint32_t m = ctrl->m;
    for (uint64_t e = (uint64_t)blockIdx.x * NT + threadIdx.x; e < m; e += (uint64_t)gridDim.x * NT) {
        const uint32_t s = src[e];
        if (e + 1 < off[s + 1]) atomicAdd(&indeg[col[e]], 1u);
    }
}

__device__ __forceinline__ uint32_t bucket_of(uint32_t din, uint32_t dout) {
    if (din == 0 || dout == 0) return BUCKET_NONE;
    const uint32_t li = min(14, floor_log2(din));
    const uint32_t lo = min(15, floor_log2(dout));
    return 16u * li + lo;
}

__global__ __launch_bounds__(NT) void k_vbucket(const uint32_t* __restrict__ off, const uint32_t* __restrict__ indeg,
                                                int32_t n, uint8_t* __restrict__ vbucket, Ctrl* ctrl) {
    __shared__ uint32_t s_nv[NBUCKET];
    __shared__ unsigned long long s_in[NBUCKET], s_out[NBUCKET], s_work[NBUCKET];
    for (int b = threadIdx.x; b < NBUCKET; b += NT) { s_nv[b] = 0; s_in[b] = 0; s_out[b] = 0; s_work[b] = 0; }
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x; v < n; v += (int64_t)gridDim.x * NT) {
        const uint32_t din = indeg[v], dout = off[v + 1] - off[v];
        const uint32_t b = bucket_of(din, dout);
        vbucket[v] = (uint8_t)b;
        if (b != BUCKET_NONE) {
            atomicAdd(&s_nv[b], 1u);
            atomicAdd(&s_in[b], (unsigned long long)din);
            atomicAdd(&s_out[b], (unsigned long long)dout);
            atomicAdd(&s_work[b], (unsigned long long)din * dout);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < NBUCKET; b += NT) {
        if (s_nv[b]) {
            atomicAdd(&ctrl->bucket_nv[b], s_nv[b]);
            atomicAdd((unsigned long long*)&ctrl->bucket_in[b], s_in[b]);
            atomicAdd((unsigned long long*)&ctrl->bucket_out[b], s_out[b]);
            atomicAdd((unsigned long long*)&ctrl->bucket_work[b], s_work[b]);
        }
    }
}

// ------------------------------------------------------------------ selection
// One thread per bucket. The heuristic follows the paper's dynamic grouping:
// a fixed degree threshold decides between the cooperative (staged) and the
// per-pair strategies; here the staged LDS bitmap takes middle vertices with
// many in-edges, binary search takes few in-edges against long lists, and
// merge-path takes the rest.
__device__ int heuristic_choice(int b) {
    const int li = b >> 4, lo = b & 15;   // floor log2 of in-degree and out-degree
    if (li >= 3) return KER_BITMAP;
    if (lo >= 5) return KER_BSEARCH;
    return KER_MERGE;
}

__global__ __launch_bounds__(NBUCKET) void k_select(Ctrl* ctrl, int mode, const uint8_t* __restrict__ learned,
                                                    const uint16_t* __restrict__ chunk_override,
                                                    const uint8_t* __restrict__ group_override) {
    __shared__ uint32_t s_key[NBUCKET];
    const int b = threadIdx.x;
    int ch;
    if (mode == SEL_FORCE_MERGE) ch = KER_MERGE;
    else if (mode == SEL_FORCE_BSEARCH) ch = KER_BSEARCH;
    else if (mode == SEL_FORCE_BITMAP) ch = KER_BITMAP;
    else if (mode == SEL_LEARNED && learned) ch = learned[b] < NKERNEL ? learned[b] : heuristic_choice(b);
    else ch = heuristic_choice(b);
    const int lo = b & 15;
    // tile shape: in-edges per tile and lanes per in-edge
    uint32_t chunk = (ch == KER_BITMAP) ? 256u : 128u;
    uint32_t group = lo >= 9 ? 64u : (lo >= 3 ? (1u << (lo - 3)) : 1u);
    if (chunk_override && chunk_override[b]) chunk = chunk_override[b];
    if (group_override && group_override[b]) group = group_override[b];
    if (ch == KER_BITMAP && chunk > (uint32_t)CHUNK_MAX) chunk = CHUNK_MAX;
    if (chunk < 16u) chunk = 16u;
    if (group > 64u || (group & (group - 1u))) group = 64u;
    if (group < 1u) group = 1u;
    ctrl->choice[b] = (uint8_t)ch;
    ctrl->chunk[b] = (uint16_t)chunk;
    ctrl->group[b] = (uint8_t)group;
    // slot order: (kernel, heavier tiles first); the empty bucket last
    const int li = b >> 4;
    const uint32_t key = (b == BUCKET_NONE) ? 0xFFFFFFFFu : ((uint32_t)ch << 16) | (uint32_t)(255 - (16 * lo + li));
    s_key[b] = key;
    __syncthreads();
    uint32_t r = 0;
    for (int q = 0; q < NBUCKET; ++q) r += (s_key[q] < key || (s_key[q] == key && q < b)) ? 1u : 0u;
    ctrl->slot[b] = (uint8_t)r;
}

__global__ __launch_bounds__(NT) void k_vkeys_slot(const uint8_t* __restrict__ vbucket, int32_t n, const Ctrl* ctrl,
                                                   uint64_t* __restrict__ keys) {
    for (int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x; v < n; v += (int64_t)gridDim.x * NT)
        keys[v] = ((uint64_t)ctrl->slot[vbucket[v]] << 32) | (uint32_t)v;
}

__global__ __launch_bounds__(NT) void k_vpos(const uint64_t* __restrict__ sorted, int32_t n,
                                             const uint8_t* __restrict__ vbucket, const uint32_t* __restrict__ indeg,
                                             const Ctrl* ctrl, uint32_t* __restrict__ vlist,
                                             uint32_t* __restrict__ pos_of, uint32_t* __restrict__ seg,
                                             uint32_t* __restrict__ ntile) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const uint32_t v = (uint32_t)sorted[i];
        const uint32_t b = vbucket[v];
        vlist[i] = v;
        pos_of[v] = (uint32_t)i;
        const uint32_t din = b == BUCKET_NONE ? 0u : indeg[v];
        const uint32_t K = ctrl->chunk[b];
        seg[i] = din;
        ntile[i] = din ? (din + K - 1) / K : 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) { seg[n] = 0; ntile[n] = 0; }
}

__global__ __launch_bounds__(NT) void k_emit_tiles(const uint32_t* __restrict__ vlist,
                                                   const uint8_t* __restrict__ vbucket,
                                                   const uint32_t* __restrict__ tstart, int32_t n, Ctrl* ctrl,
                                                   uint64_t* __restrict__ tiles, uint64_t tile_cap) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const uint32_t b = vbucket[vlist[i]];
        const int kk = b == BUCKET_NONE ? NKERNEL : ctrl->choice[b];
        int kprev = -1;
        if (i > 0) {
            const uint32_t bp = vbucket[vlist[i - 1]];
            kprev = bp == BUCKET_NONE ? NKERNEL : ctrl->choice[bp];
        }
        const uint32_t t0 = tstart[i], t1 = tstart[i + 1];
        for (uint32_t t = t0; t < t1 && t < tile_cap; ++t) tiles[t] = (uint64_t)(uint32_t)i | ((uint64_t)(t - t0) << 32);
        for (int k = kprev + 1; k <= kk; ++k) ctrl->tile_begin[k] = t0;
        if (i == n - 1) {
            for (int k = kk + 1; k <= NKERNEL; ++k) ctrl->tile_begin[k] = tstart[n];
            ctrl->ntiles = tstart[n];
        }
    }
}

__global__ __launch_bounds__(NT) void k_csc(const uint32_t* __restrict__ col, const uint32_t* __restrict__ src,
                                            const uint32_t* __restrict__ off, const Ctrl* ctrl,
                                            const uint8_t* __restrict__ vbucket, const uint32_t* __restrict__ pos_of,
                                            const uint32_t* __restrict__ seg_start, uint32_t* __restrict__ cursor,
                                            uint64_t* __restrict__ csc, uint64_t cap) {
    const uint32_t m = ctrl->m;
    for (uint64_t e = (uint64_t)blockIdx.x * NT + threadIdx.x; e < m; e += (uint64_t)gridDim.x * NT) {
        const uint32_t end = off[src[e] + 1];
        if (e + 1 >= end) continue;
        const uint32_t v = col[e];
        if (vbucket[v] == BUCKET_NONE) continue;
        const uint32_t slot = seg_start[pos_of[v]] + atomicAdd(&cursor[v], 1u);
        if (slot < cap) csc[slot] = (uint64_t)e | ((uint64_t)end << 32);
    }
}

// ------------------------------------------------------------------ outputs
__global__ __launch_bounds__(NT) void k_map_pv(const uint64_t* __restrict__ pv, const uint32_t* __restrict__ inv,
                                               int32_t n, uint64_t* __restrict__ out) {
    for (int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x; r < n; r += (int64_t)gridDim.x * NT) out[inv[r]] = pv[r];
}

__global__ __launch_bounds__(NT) void k_map_edges(const uint32_t* __restrict__ col, const uint32_t* __restrict__ src,
                                                  const uint32_t* __restrict__ inv, const Ctrl* ctrl,
                                                  int2* __restrict__ out) {
    const uint32_t m = ctrl->m;
    for (uint64_t e = (uint64_t)blockIdx.x * NT + threadIdx.x; e < m; e += (uint64_t)gridDim.x * NT)
        out[e] = make_int2((int)inv[src[e]], (int)inv[col[e]]);
}

__global__ __launch_bounds__(NT) void k_export_csr(const uint32_t* __restrict__ rank, const uint32_t* __restrict__ off,
                                                   const uint32_t* __restrict__ col, const Ctrl* ctrl, int32_t n,
                                                   int32_t* __restrict__ o_rank, int64_t* __restrict__ o_off,
                                                   int32_t* __restrict__ o_col) {
    const uint32_t m = ctrl->m;
    const uint64_t stride = (uint64_t)gridDim.x * NT;
    for (uint64_t i = (uint64_t)blockIdx.x * NT + threadIdx.x; i < (uint64_t)n + 1; i += stride) {
        if (i < (uint64_t)n) o_rank[i] = (int32_t)rank[i];
        o_off[i] = (int64_t)off[i];
    }
    for (uint64_t e = (uint64_t)blockIdx.x * NT + threadIdx.x; e < m; e += stride) o_col[e] = (int32_t)col[e];
}

// ------------------------------------------------------------------ workspace layout
Layout make_layout(int64_t E, int32_t n) {
    Layout L;
    const size_t A = 256;
    const size_t nn = (size_t)n, ee = (size_t)E;
    const size_t kcap = ee > nn ? ee : nn;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + (bytes ? bytes : 1), A); return r; };
    L.ctrl = take(sizeof(Ctrl));
    L.deg = take(4 * nn);
    L.rank = take(4 * nn);
    L.inv = take(4 * nn);
    L.vbucket = take(nn);
    L.pos_of = take(4 * nn);
    L.vlist = take(4 * nn);
    L.cursor = take(4 * nn);
    L.seg = take(4 * (nn + 1));
    L.tstart = take(4 * (nn + 1));
    L.off = take(4 * (nn + 1));
    L.rowend = take(4 * nn);
    L.pv = take(8 * nn);
    L.keysA = take(8 * kcap);
    L.keysB = take(8 * kcap);
    L.col = take(4 * ee);
    L.src = take(4 * ee);
    L.tile_cap = ee / 16 + nn + 1;
    L.tiles = take(8 * L.tile_cap);
    L.partial = take(4 * (UQ_MAX_BLOCKS + 1));
    L.scan_tmp = take(scan_temp_bytes());
    L.radix_tmp = take(radix_temp_bytes(kcap));
    L.total = o;
    return L;
}

// ------------------------------------------------------------------ the pipeline
int stage_count() { return NSTAGE; }
const char* stage_name(int s) {
    static const char* names[NSTAGE] = {"degree", "rank", "orient", "sort", "csr", "bucket",
                                        "group", "isect_merge", "isect_bsearch", "isect_bitmap", "finish"};
    return (s >= 0 && s < NSTAGE) ? names[s] : "";
}

hipError_t run_pipeline(const RunArgs& r, RunResult* out) {
    hipStream_t s = r.stream;
    char* ws = (char*)r.ws;
    const Layout L = make_layout(r.E, r.n);
    const int64_t E = r.E;
    const int32_t n = r.n;
    Ctrl* ctrl = (Ctrl*)(ws + L.ctrl);
    uint32_t* deg = (uint32_t*)(ws + L.deg);
    uint32_t* rank = (uint32_t*)(ws + L.rank);
    uint32_t* inv = (uint32_t*)(ws + L.inv);
    uint8_t* vbucket = (uint8_t*)(ws + L.vbucket);
    uint32_t* pos_of = (uint32_t*)(ws + L.pos_of);
    uint32_t* vlist = (uint32_t*)(ws + L.vlist);
    uint32_t* cursor = (uint32_t*)(ws + L.cursor);
    uint32_t* seg = (uint32_t*)(ws + L.seg);
    uint32_t* tstart = (uint32_t*)(ws + L.tstart);
    uint32_t* off = (uint32_t*)(ws + L.off);
    uint32_t* rowend = (uint32_t*)(ws + L.rowend);
    uint64_t* pv = (uint64_t*)(ws + L.pv);
    uint64_t* keysA = (uint64_t*)(ws + L.keysA);
    uint64_t* keysB = (uint64_t*)(ws + L.keysB);
    uint32_t* col = (uint32_t*)(ws + L.col);
    uint32_t* src = (uint32_t*)(ws + L.src);
    uint64_t* tiles = (uint64_t*)(ws + L.tiles);
    uint32_t* partial = (uint32_t*)(ws + L.partial);
    void* scan_tmp = ws + L.scan_tmp;
    void* radix_tmp = ws + L.radix_tmp;
    const int2* edges = (const int2*)r.edges;
    const size_t kcap = (size_t)(E > n ? E : n);

    auto mark = [&](int stage) {
        if (r.events) hipEventRecord(r.events[stage], s);
    };
    mark(0);
    // ---- degree
    fill_u32((uint32_t*)ctrl, 0u, sizeof(Ctrl) / 4, s);
    fill_u32(deg, 0u, (size_t)n, s);
    hipLaunchKernelGGL(k_degree, dim3(grid_for((size_t)E)), dim3(NT), 0, s, edges, (uint64_t)E, n, deg, ctrl);
    mark(1);
    // ---- rank: sort (degree, id); degrees of a multigraph are < 2E + 1
    hipLaunchKernelGGL(k_vertex_keys, dim3(grid_for((size_t)n)), dim3(NT), 0, s, deg, n, keysA);
    {
        const int dbits = bits_for((uint64_t)2 * (uint64_t)E + 1);
        const int alt = radix_sort_u64(keysA, keysB, nullptr, nullptr, nullptr, (size_t)n, 32, 32 + dbits,
                                       radix_tmp, s);
        hipLaunchKernelGGL(k_rank, dim3(grid_for((size_t)n)), dim3(NT), 0, s, alt ? keysB : keysA, n, rank, inv);
    }
    mark(2);
    // ---- orient
    const int nb = bits_for((uint64_t)n);
    hipLaunchKernelGGL(k_orient, dim3(grid_for((size_t)E)), dim3(NT), 0, s, edges, (uint64_t)E, n, rank, nb, keysA,
                       ctrl);
    mark(3);
    // ---- sort oriented pairs
    const int alt = radix_sort_u64(keysA, keysB, nullptr, nullptr, &ctrl->m_valid, (size_t)E, 0, 2 * nb, radix_tmp, s);
    uint64_t* sorted = alt ? keysB : keysA;
    mark(4);
    // ---- unique + CSR
    {
        uint32_t nblk = (uint32_t)((E + 8191) / 8192);
        if (nblk > (uint32_t)UQ_MAX_BLOCKS) nblk = UQ_MAX_BLOCKS;
        if (nblk < 1) nblk = 1;
        uint32_t chunk = (uint32_t)(((uint64_t)E + nblk - 1) / nblk);
        chunk = (chunk + NT - 1) / NT * NT;
        nblk = (uint32_t)(((uint64_t)E + chunk - 1) / chunk);
        if (nblk < 1) nblk = 1;
        hipLaunchKernelGGL(k_unique_count, dim3(nblk), dim3(NT), 0, s, sorted, ctrl, chunk, partial, nblk);
        scan_exclusive_sum_u32(partial, partial, (size_t)nblk + 1, scan_tmp, s);
        fill_u32(rowend, 0u, (size_t)n, s);
        hipLaunchKernelGGL(k_unique_write, dim3(nblk), dim3(NT), 0, s, sorted, ctrl, chunk, partial, nblk, nb, col,
                           src, rowend);
        fill_u32(off, 0u, 1, s);
        scan_inclusive_max_u32(rowend, off + 1, (size_t)n, scan_tmp, s);
    }
    mark(5);
    if (r.csr_rank) {   // CSR export only: stop after the induced subgraph
        hipLaunchKernelGGL(k_export_csr, dim3(grid_for(kcap)), dim3(NT), 0, s, rank, off, col, ctrl, n, r.csr_rank,
                           r.csr_off, r.csr_col);
        out->ctrl_dev = ctrl;
        return hipGetLastError();
    }
    // ---- buckets (deg is reused for in-degrees)
    fill_u32(deg, 0u, (size_t)n, s);
    hipLaunchKernelGGL(k_indeg, dim3(grid_for((size_t)E)), dim3(NT), 0, s, col, src, off, ctrl, deg);
    hipLaunchKernelGGL(k_vbucket, dim3(grid_for((size_t)n, 2048)), dim3(NT), 0, s, off, deg, n, vbucket, ctrl);
    hipLaunchKernelGGL(k_select, dim3(1), dim3(NBUCKET), 0, s, ctrl, r.select, r.learned, r.chunk_override,
                       r.group_override);
    mark(6);
    // ---- group: order vertices by (kernel, bucket), segments, tiles, in-edge scatter
    hipLaunchKernelGGL(k_vkeys_slot, dim3(grid_for((size_t)n)), dim3(NT), 0, s, vbucket, n, ctrl, keysA);
    {
        const int a2 = radix_sort_u64(keysA, keysB, nullptr, nullptr, nullptr, (size_t)n, 32, 40, radix_tmp, s);
        hipLaunchKernelGGL(k_vpos, dim3(grid_for((size_t)n)), dim3(NT), 0, s, a2 ? keysB : keysA, n, vbucket, deg,
                           ctrl, vlist, pos_of, seg, tstart);
    }
    scan_exclusive_sum_u32(seg, seg, (size_t)n + 1, scan_tmp, s);
    scan_exclusive_sum_u32(tstart, tstart, (size_t)n + 1, scan_tmp, s);
    hipLaunchKernelGGL(k_emit_tiles, dim3(grid_for((size_t)n)), dim3(NT), 0, s, vlist, vbucket, tstart, n, ctrl,
                       tiles, (uint64_t)L.tile_cap);
    fill_u32(cursor, 0u, (size_t)n, s);
    uint64_t* csc = keysA;   // the vertex keys are no longer needed
    hipLaunchKernelGGL(k_csc, dim3(grid_for((size_t)E)), dim3(NT), 0, s, col, src, off, ctrl, vbucket, pos_of, seg,
                       cursor, csc, (uint64_t)kcap);
    if (r.per_edge_counts) fill_u32(r.per_edge_counts, 0u, (size_t)E, s);
    if (r.per_vertex) fill_u64(pv, 0ull, (size_t)n, s);
    mark(7);
    // ---- intersections
    IsectArgs ia;
    ia.ctrl = ctrl;
    ia.off = off;
    ia.col = col;
    ia.src = src;
    ia.csc = csc;
    ia.seg_start = seg;
    ia.vlist = vlist;
    ia.vbucket = vbucket;
    ia.tiles = tiles;
    ia.per_edge = r.per_edge_counts;
    ia.per_vertex = r.per_vertex ? pv : nullptr;
    const int order[NKERNEL] = {KER_MERGE, KER_BSEARCH, KER_BITMAP};
    for (int q = 0; q < NKERNEL; ++q) {
        const int k = order[q];
        launch_isect(k, ia, r.grid_override ? r.grid_override[k] : 0, s);
        mark(8 + q);
    }
    // ---- finish
    if (r.per_vertex)
        hipLaunchKernelGGL(k_map_pv, dim3(grid_for((size_t)n)), dim3(NT), 0, s, pv, inv, n, r.per_vertex);
    if (r.per_edge_pairs)
        hipLaunchKernelGGL(k_map_edges, dim3(grid_for((size_t)E)), dim3(NT), 0, s, col, src, inv, ctrl,
                           (int2*)r.per_edge_pairs);
    mark(NSTAGE);
    out->ctrl_dev = ctrl;
    return hipGetLastError();
}

}  // namespace tcx
