// Per-edge intersection kernels (Section 3.2, Algorithm 2 "Compute_Intersection";
// Section 4.2, dynamic grouping and the large/small neighbour-list kernels).
//
// The graph is the degree-ordered CSR over ranks: row u holds N+(u), the
// neighbours ranked above u, ascending. For a kept edge e = (u -> v) at
// position p of row u, a common neighbour w of N+(u) and N+(v) must rank above
// v, so only the tail of row u after p can match:
//     c_e = | row_u[p+1 ..] intersected with N+(v) |  =  | N+(u) intersected with N+(v) |.
// Work is grouped by the middle vertex v: a tile is v together with a chunk
// of its in-edges (entries e | row_end(u) << 32). Three interchangeable
// strategies compute the same c_e for every in-edge of a tile:
//   merge   : merge-path split of (tail, N+(v)) across a group of lanes
//   bsearch : binary search of each element of the shorter list in the other
//   bitmap  : N+(v) staged once per tile as an LDS bitmap; tails streamed
//             through it (long tails by a whole wave, short ones by one lane)
// Each hit adds 1 to the exact 64-bit triangle count; optional outputs are
// the per-edge counts c_e and per-vertex counts t[u], t[v], t[w].
#include "common.h"
#include "internal.h"
#include "isect.h"

namespace tcx {

constexpr int IS_NT = 256;
constexpr int BM_WORDS = 4096;            // 131072-bit window (16 KiB)
constexpr uint32_t BM_BITS = BM_WORDS * 32u;
constexpr int STAGE_MAX = 4096;           // N+(v) staged in LDS by merge/bsearch when it fits
constexpr uint32_t LONG_TAIL = 32;        // bitmap kernel: tails this long go to a whole wave

struct TileView {
    uint32_t v, e0, e1, b0, b1;
};

__device__ __forceinline__ bool next_tile(const IsectArgs& a, int ker, uint32_t* s_tile, TileView* tv) {
    if (threadIdx.x == 0) *s_tile = a.ctrl->tile_begin[ker] + atomicAdd(&a.ctrl->tile_next[ker], 1u);
    __syncthreads();
    const uint32_t t = *s_tile;
    __syncthreads();
    if (t >= a.ctrl->tile_begin[ker + 1]) return false;
    const uint64_t d = a.tiles[t];
    const uint32_t i = (uint32_t)d, j = (uint32_t)(d >> 32);
    const uint32_t v = a.vlist[i];
    const uint32_t K = a.ctrl->chunk[a.vbucket[v]];
    const uint32_t s0 = a.seg_start[i], s1 = a.seg_start[i + 1];
    tv->v = v;
    tv->e0 = s0 + j * K;
    tv->e1 = tv->e0 + K < s1 ? tv->e0 + K : s1;
    tv->b0 = a.off[v];
    tv->b1 = a.off[v + 1];
    return true;
}

__device__ __forceinline__ void edge_done(const IsectArgs& a, uint32_t e, uint32_t v, uint32_t c) {
    if (a.per_edge) a.per_edge[e] = c;
    if (a.per_vertex && c) {
        atomicAdd((unsigned long long*)&a.per_vertex[a.src[e]], (unsigned long long)c);
        atomicAdd((unsigned long long*)&a.per_vertex[v], (unsigned long long)c);
    }
}

__device__ __forceinline__ void hit_vertex(const IsectArgs& a, uint32_t w) {
    if (a.per_vertex) atomicAdd((unsigned long long*)&a.per_vertex[w], 1ull);
}

__device__ __forceinline__ void block_flush_total(const IsectArgs& a, uint64_t acc) {
    __shared__ uint64_t red[IS_NT / WAVE];
    acc = wave_sum_u64(acc);
    if (lane_id() == 0) red[wave_id()] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        for (int i = 0; i < IS_NT / WAVE; ++i) s += red[i];
        if (s) atomicAdd((unsigned long long*)&a.ctrl->total, (unsigned long long)s);
    }
}

// ------------------------------------------------------------------ LDS bitmap
__global__ __launch_bounds__(IS_NT) void k_isect_bitmap(IsectArgs a) {
    __shared__ uint32_t bm[BM_WORDS];
    __shared__ uint32_t s_start[CHUNK_MAX];
    __shared__ uint32_t s_end[CHUNK_MAX];
    __shared__ uint16_t s_long[CHUNK_MAX];
    __shared__ uint16_t s_short[CHUNK_MAX];
    __shared__ uint32_t s_nlong, s_nshort, s_long_next, s_tile;
    for (int i = threadIdx.x; i < BM_WORDS; i += IS_NT) bm[i] = 0;
    const int l = lane_id();
    uint64_t acc = 0;
    TileView tv;
    while (next_tile(a, KER_BITMAP, &s_tile, &tv)) {
        const uint32_t ne = tv.e1 - tv.e0;
        const uint32_t nb = tv.b1 - tv.b0;
        if (threadIdx.x == 0) { s_nlong = 0; s_nshort = 0; s_long_next = 0; }
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < ne; k += IS_NT) {
            const uint64_t ent = a.csc[tv.e0 + k];
            const uint32_t s = (uint32_t)ent + 1u, e = (uint32_t)(ent >> 32);
            s_start[k] = s;
            s_end[k] = e;
            if (e - s >= LONG_TAIL) s_long[atomicAdd(&s_nlong, 1u)] = (uint16_t)k;
            else s_short[atomicAdd(&s_nshort, 1u)] = (uint16_t)k;
        }
        const uint32_t lo = a.col[tv.b0], hi = a.col[tv.b1 - 1];
        const uint32_t base = lo & ~31u;
        const uint32_t nwin = (hi - base) / BM_BITS + 1;
        __syncthreads();
        const uint32_t nlong = s_nlong, nshort = s_nshort;
        for (uint32_t win = 0; win < nwin; ++win) {
            const uint32_t wlo = base + win * BM_BITS;
            for (uint32_t j = threadIdx.x; j < nb; j += IS_NT) {
                const uint32_t x = a.col[tv.b0 + j];
                if (x >= wlo && x - wlo < BM_BITS) atomicOr(&bm[(x - wlo) >> 5], 1u << ((x - wlo) & 31u));
            }
            __syncthreads();
            // long tails: one wave per in-edge, lanes stride the tail
            if (nwin == 1) {
                while (true) {
                    uint32_t q = 0;
                    if (l == 0) q = atomicAdd(&s_long_next, 1u);
                    q = __shfl(q, 0, WAVE);
                    if (q >= nlong) break;
                    const uint32_t k = s_long[q];
                    const uint32_t s = s_start[k], e = s_end[k];
                    uint32_t c = 0;
                    for (uint32_t p = s + l; p < e; p += WAVE) {
                        const uint32_t x = a.col[p] - wlo;
                        if (x < BM_BITS && ((bm[x >> 5] >> (x & 31u)) & 1u)) {
                            ++c;
                            hit_vertex(a, x + wlo);
                        }
                    }
                    c = wave_sum(c);
                    acc += (l == 0) ? c : 0u;
                    if (l == 0) edge_done(a, s - 1u, tv.v, c);
                }
                // short tails: one lane per in-edge
                for (uint32_t q = threadIdx.x; q < nshort; q += IS_NT) {
                    const uint32_t k = s_short[q];
                    const uint32_t s = s_start[k], e = s_end[k];
                    uint32_t c = 0;
                    for (uint32_t p = s; p < e; ++p) {
                        const uint32_t x = a.col[p] - wlo;
                        if (x < BM_BITS && ((bm[x >> 5] >> (x & 31u)) & 1u)) {
                            ++c;
                            hit_vertex(a, x + wlo);
                        }
                    }
                    acc += c;
                    edge_done(a, s - 1u, tv.v, c);
                }
            } else {
                // several windows (N+(v) spans more than 2^17 ranks): one lane per
                // in-edge; the per-edge output accumulates across windows
                for (uint32_t k = threadIdx.x; k < ne; k += IS_NT) {
                    const uint32_t s = s_start[k], e = s_end[k];
                    uint32_t c = 0;
                    for (uint32_t p = s; p < e; ++p) {
                        const uint32_t x = a.col[p] - wlo;
                        if (x < BM_BITS && ((bm[x >> 5] >> (x & 31u)) & 1u)) {
                            ++c;
                            hit_vertex(a, x + wlo);
                        }
                    }
                    acc += c;
                    // accumulate the per-edge count across windows in place
                    if (a.per_edge) a.per_edge[s - 1u] = (win ? a.per_edge[s - 1u] : 0u) + c;
                    if (a.per_vertex && c) {
                        atomicAdd((unsigned long long*)&a.per_vertex[a.src[s - 1u]], (unsigned long long)c);
                        atomicAdd((unsigned long long*)&a.per_vertex[tv.v], (unsigned long long)c);
                    }
                }
            }
            __syncthreads();
            for (uint32_t j = threadIdx.x; j < nb; j += IS_NT) {
                const uint32_t x = a.col[tv.b0 + j];
                if (x >= wlo && x - wlo < BM_BITS) bm[(x - wlo) >> 5] = 0u;
            }
            __syncthreads();
        }
    }
    block_flush_total(a, acc);
}

// ------------------------------------------------------------------ shared helpers for edge-centric kernels
// N+(v) is staged in LDS when it fits; otherwise it is read from global memory.
struct ListRef {
    const uint32_t* p;
};

// Number of elements of A taken in the first d outputs of the merge of A and
// B, A first on ties (merge-path split, Green et al. / Odeh et al.).
__device__ __forceinline__ uint32_t merge_split(const uint32_t* A, uint32_t na, const uint32_t* B, uint32_t nb,
                                                uint32_t d) {
    uint32_t lo = d > nb ? d - nb : 0u;
    uint32_t hi = d < na ? d : na;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (A[mid] <= B[d - 1u - mid]) lo = mid + 1u;
        else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------ merge path
__global__ __launch_bounds__(IS_NT) void k_isect_merge(IsectArgs a) {
    __shared__ uint32_t sb[STAGE_MAX];
    __shared__ uint32_t s_tile;
    uint64_t acc = 0;
    TileView tv;
    while (next_tile(a, KER_MERGE, &s_tile, &tv)) {
        const uint32_t nb = tv.b1 - tv.b0;
        const bool staged = nb <= (uint32_t)STAGE_MAX;
        if (staged)
            for (uint32_t j = threadIdx.x; j < nb; j += IS_NT) sb[j] = a.col[tv.b0 + j];
        __syncthreads();
        const uint32_t* B = staged ? sb : a.col + tv.b0;
        const uint32_t g = a.ctrl->group[a.vbucket[tv.v]];          // lanes per in-edge (power of 2)
        const uint32_t gi = threadIdx.x / g, gl = threadIdx.x % g;  // group index, lane in group
        const uint32_t ngroups = IS_NT / g;
        const uint32_t ne = tv.e1 - tv.e0;
        const uint32_t rounds = (ne + ngroups - 1) / ngroups;
        for (uint32_t r = 0; r < rounds; ++r) {
            const uint32_t k = r * ngroups + gi;
            uint32_t c = 0, e = 0;
            if (k < ne) {
                const uint64_t ent = a.csc[tv.e0 + k];
                e = (uint32_t)ent;
                const uint32_t s = e + 1u, end = (uint32_t)(ent >> 32);
                const uint32_t* A = a.col + s;
                const uint32_t na = end - s;
                const uint32_t tot = na + nb;
                const uint32_t d0 = (uint32_t)(((uint64_t)tot * gl) / g);
                const uint32_t d1 = (uint32_t)(((uint64_t)tot * (gl + 1u)) / g);
                uint32_t i = merge_split(A, na, B, nb, d0);
                uint32_t jb = d0 - i;
                for (uint32_t step = d0; step < d1; ++step) {
                    if (i < na && (jb >= nb || A[i] <= B[jb])) {
                        if (jb < nb && A[i] == B[jb]) {
                            ++c;
                            hit_vertex(a, A[i]);
                        }
                        ++i;
                    } else {
                        ++jb;
                    }
                }
            }
            // reduce within the group of g lanes (g divides the wave)
            for (uint32_t o = g >> 1; o > 0; o >>= 1) c += __shfl_xor(c, (int)o, WAVE);
            if (k < ne && gl == 0) {
                acc += c;
                edge_done(a, e, tv.v, c);
            }
        }
        __syncthreads();
    }
    block_flush_total(a, acc);
}

// ------------------------------------------------------------------ binary search
__device__ __forceinline__ bool contains(const uint32_t* L, uint32_t n, uint32_t x) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (L[mid] < x) lo = mid + 1u;
        else hi = mid;
    }
    return lo < n && L[lo] == x;
}

__global__ __launch_bounds__(IS_NT) void k_isect_bsearch(IsectArgs a) {
    __shared__ uint32_t sb[STAGE_MAX];
    __shared__ uint32_t s_tile;
    uint64_t acc = 0;
    TileView tv;
    while (next_tile(a, KER_BSEARCH, &s_tile, &tv)) {
        const uint32_t nb = tv.b1 - tv.b0;
        const bool staged = nb <= (uint32_t)STAGE_MAX;
        if (staged)
            for (uint32_t j = threadIdx.x; j < nb; j += IS_NT) sb[j] = a.col[tv.b0 + j];
        __syncthreads();
        const uint32_t* B = staged ? sb : a.col + tv.b0;
        const uint32_t g = a.ctrl->group[a.vbucket[tv.v]];
        const uint32_t gi = threadIdx.x / g, gl = threadIdx.x % g;
        const uint32_t ngroups = IS_NT / g;
        const uint32_t ne = tv.e1 - tv.e0;
        const uint32_t rounds = (ne + ngroups - 1) / ngroups;
        for (uint32_t r = 0; r < rounds; ++r) {
            const uint32_t k = r * ngroups + gi;
            uint32_t c = 0, e = 0;
            if (k < ne) {
                const uint64_t ent = a.csc[tv.e0 + k];
                e = (uint32_t)ent;
                const uint32_t s = e + 1u, end = (uint32_t)(ent >> 32);
                const uint32_t* A = a.col + s;
                const uint32_t na = end - s;
                if (na <= nb) {
                    for (uint32_t q = gl; q < na; q += g) {
                        const uint32_t x = A[q];
                        if (contains(B, nb, x)) {
                            ++c;
                            hit_vertex(a, x);
                        }
                    }
                } else {
                    for (uint32_t q = gl; q < nb; q += g) {
                        const uint32_t x = B[q];
                        if (contains(A, na, x)) {
                            ++c;
                            hit_vertex(a, x);
                        }
                    }
                }
            }
            for (uint32_t o = g >> 1; o > 0; o >>= 1) c += __shfl_xor(c, (int)o, WAVE);
            if (k < ne && gl == 0) {
                acc += c;
                edge_done(a, e, tv.v, c);
            }
        }
        __syncthreads();
    }
    block_flush_total(a, acc);
}

// ------------------------------------------------------------------ launchers
static int g_num_cu = 0;

static int num_cu() {
    if (!g_num_cu) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) g_num_cu = p.multiProcessorCount;
        if (g_num_cu <= 0) g_num_cu = 256;
    }
    return g_num_cu;
}

int isect_blocks_per_cu(int ker) {
    switch (ker) {
        case KER_BITMAP: return 6;
        default: return 8;
    }
}

void launch_isect(int ker, const IsectArgs& a, int grid, hipStream_t s) {
    if (grid <= 0) grid = num_cu() * isect_blocks_per_cu(ker);
    switch (ker) {
        case KER_MERGE: hipLaunchKernelGGL(k_isect_merge, dim3(grid), dim3(IS_NT), 0, s, a); break;
        case KER_BSEARCH: hipLaunchKernelGGL(k_isect_bsearch, dim3(grid), dim3(IS_NT), 0, s, a); break;
        default: hipLaunchKernelGGL(k_isect_bitmap, dim3(grid), dim3(IS_NT), 0, s, a); break;
    }
}

}  // namespace tcx
