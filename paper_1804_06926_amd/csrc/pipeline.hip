// The counting pipeline on one stream: edge-list generation and filtering,
// CSR construction, degree-pair bucketing, kernel selection and intersection.
//
// Stages (Algorithm 2; Section 4.2 for the filter, the induced subgraph and
// dynamic grouping):
//   degree    validate ids, count input pairs per vertex (self-loops dropped)
//   rank      sort vertices by (degree, id): rank = position
//   orient    each pair as (rank lo, rank hi); loops / bad ids -> sentinel
//   sort      radix sort of the oriented pairs -> rows contiguous, ascending
//   csr       drop repeats and sentinels, emit col/src, row offsets
//   csc       in-edges (u -> v) with a non-empty tail of row u, grouped by v
//             (stable radix sort on v), in-offsets from the group boundaries
//             (the other formulations instead group all in-edges and build the
//             symmetric adjacency beside the filtered CSR)
//   bucket    per middle vertex v: (in-edges with work, |N+(v)|) -> bucket
//   select    choose the intersection strategy and tile shape per bucket
//   group     order vertices by (strategy, bucket); emit tiles
//   isect     the three intersection kernels, each over its tile range
//   finish    map per-vertex / per-edge outputs back to original ids
// No stage relies on atomics to one address: compaction and grouping go
// through sorts and scans, so every intermediate array is deterministic. The
// kernels that write the keys of a sort also take the per-tile digit counts of
// its first pass (one read of the keys less per sort).
#include <math.h>
#include <string.h>

#include "common.h"
#include "internal.h"
#include "isect.h"
#include "mlp.h"
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
// Input degree = loop-free valid pairs per vertex. Device-wide atomics would
// serialise on hub vertices, so the 2E endpoints are first partitioned by
// their high bits (one radix pass for ids of up to 24 bits, two up to 27), and
// each bucket of 2^bw vertices is then counted in an LDS histogram of up to
// 2^15 counters (128 KB); a wider bucket is counted in parts, each block
// reading the whole bucket and counting the ids of its own part. Endpoints
// of loops and invalid pairs are written as `sentinel`; with sentinel = n - 1
// each block also records how many it wrote, and they are taken off vertex
// n - 1 at the end. Wider ids fall back to a full sort of the endpoints
// (sentinel n, which sorts last) and run boundaries.
constexpr int DEG_MAX_BW = 14;        // buckets of 2^14 vertices beyond 24-bit ids (two passes)
constexpr int DEG_MAX_CW = 15;        // LDS histogram of at most 2^15 counters (128 KB)
constexpr int DEG_MAX_BUCKET_BITS = 13;   // up to 8192 buckets (ids below 2^27)
constexpr unsigned DEG_EP_BLOCKS = 1024;

__global__ __launch_bounds__(NT) void k_endpoints(const int2* __restrict__ edges, uint64_t E, int32_t n,
                                                  uint32_t sentinel, uint32_t* __restrict__ keys, Ctrl* ctrl,
                                                  uint32_t* __restrict__ nsent, uint32_t* __restrict__ counts,
                                                  uint32_t ntiles, uint32_t tile_keys, RadixDigit dg,
                                                  uint32_t* __restrict__ pcounts, uint32_t pf, RadixDigit pdg,
                                                  uint32_t* __restrict__ p2tot) {
    // tile t = endpoints [t * tile_keys, (t + 1) * tile_keys) = pairs [t * EPT, (t + 1) * EPT),
    // in rounds of NT * PER pairs; with counts set, the first digit of the endpoint sort is
    // counted per tile. With pcounts set, the digit pdg of the first id is counted too, per
    // tile of pf endpoint tiles: the first pass of the orientation's pair partition, whose
    // tiles hold pf * EPT pairs. With p2tot set, the same digit of the second id is counted
    // over all pairs (added into p2tot[256]): the digit totals of that partition's second
    // pass, which then takes its offsets by look-back.
    constexpr uint32_t PER = 4;
    const uint32_t EPT = tile_keys / 2;
    const uint32_t pntiles = (ntiles + pf - 1) / pf;
    __shared__ uint32_t red[NT / WAVE];
    __shared__ TileCounts tc, tp, tq;
    tc.clear();
    if (pcounts) tp.clear();
    if (p2tot) tq.clear();
    __syncthreads();
    bool bad = false;
    uint32_t sent = 0;
    for (uint32_t pt = blockIdx.x; pt < pntiles; pt += gridDim.x) {
     for (uint32_t tile = pt * pf; tile < (pt + 1) * pf && tile < ntiles; ++tile) {
      for (uint32_t r = 0; r < EPT; r += PER * NT) {
        int2 ed[PER];
#pragma unroll
        for (uint32_t k = 0; k < PER; ++k) {
            const uint64_t i = (uint64_t)tile * EPT + r + k * NT + threadIdx.x;
            ed[k] = i < E ? edges[i] : make_int2(0, 0);
        }
#pragma unroll
        for (uint32_t k = 0; k < PER; ++k) {
            const uint64_t i = (uint64_t)tile * EPT + r + k * NT + threadIdx.x;
            if (i >= E) continue;
            const int2 e = ed[k];
            const bool in_range = e.x >= 0 && e.x < n && e.y >= 0 && e.y < n;
            bad |= !in_range;
            const bool ok = in_range && e.x != e.y;
            const uint32_t a = ok ? (uint32_t)e.x : sentinel, b = ok ? (uint32_t)e.y : sentinel;
            ((uint2*)keys)[i] = make_uint2(a, b);
            sent += ok ? 0u : 2u;
            if (counts) {
                tc.add((a >> dg.shift) & dg.mask);
                tc.add((b >> dg.shift) & dg.mask);
            }
            if (pcounts) tp.add(((uint32_t)e.x >> pdg.shift) & pdg.mask);
            if (p2tot) tq.add(((uint32_t)e.y >> pdg.shift) & pdg.mask);
        }
      }
        if (counts) tc.flush(counts, ntiles, tile);
     }
        if (pcounts) tp.flush(pcounts, pntiles, pt);
    }
    if (p2tot) {
        __syncthreads();
        const uint32_t t = tq.w[0][threadIdx.x] + tq.w[1][threadIdx.x] + tq.w[2][threadIdx.x] + tq.w[3][threadIdx.x];
        if (t) atomicAdd(&p2tot[threadIdx.x], t);
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(&ctrl->err, 1u);
    sent = wave_sum(sent);
    if (lane_id() == 0) red[wave_id()] = sent;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < NT / WAVE; ++k) t += red[k];
        nsent[blockIdx.x] = t;
    }
}

// bstart[b] = first position of bucket b (ids >> bw == b) in the endpoints,
// which the partition left ordered by bucket; bstart[nb] = len.
__global__ __launch_bounds__(NT) void k_bucket_starts(const uint32_t* __restrict__ ep, uint32_t len, int bw,
                                                      uint32_t nb, uint32_t* __restrict__ bstart) {
    for (uint32_t b = blockIdx.x * NT + threadIdx.x; b <= nb; b += gridDim.x * NT) {
        uint32_t lo = 0, hi = len;
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if ((ep[mid] >> bw) < b) lo = mid + 1;
            else hi = mid;
        }
        bstart[b] = b == nb ? len : lo;
    }
}

// Block (bucket b, part pt, split sp) counts, in LDS, the ids of part pt (ids
// whose bits [cw, bw) equal pt, cw = min(bw, CW)) among its share of bucket b.
// One split: plain stores of every count of the part; several: atomic adds
// into the zeroed degree array. The 2^15-counter histogram leaves room for one
// block per CU, so that size runs 1024 threads.
template <int CW, int NTB>
__global__ __launch_bounds__(NTB) void k_bucket_count(const uint32_t* __restrict__ ep,
                                                      const uint32_t* __restrict__ bstart, int bw, uint32_t parts,
                                                      uint32_t splits, int32_t n, uint32_t* __restrict__ deg) {
    __shared__ uint32_t h[1u << CW];
    const int cw = bw < CW ? bw : CW;
    const uint32_t nh = 1u << cw, hmask = nh - 1u, bmask = (1u << bw) - 1u;
    const uint32_t b = blockIdx.x / (parts * splits), rem = blockIdx.x % (parts * splits);
    const uint32_t pt = rem / splits, sp = rem % splits;
    for (uint32_t j = threadIdx.x; j < nh; j += NTB) h[j] = 0;
    __syncthreads();
    const uint32_t s0 = bstart[b], s1 = bstart[b + 1];
    const uint32_t len = s1 - s0;
    const uint32_t a0 = s0 + (uint32_t)(((uint64_t)len * sp) / splits);
    const uint32_t a1 = s0 + (uint32_t)(((uint64_t)len * (sp + 1)) / splits);
    constexpr int U = 8;
    for (uint32_t i0 = a0; i0 < a1; i0 += NTB * U) {
        uint32_t x[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {   // loads in flight together
            const uint32_t i = i0 + k * NTB + threadIdx.x;
            x[k] = i < a1 ? ep[i] : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const uint32_t loc = x[k] & bmask;
            if (x[k] != 0xFFFFFFFFu && (loc >> cw) == pt) atomicAdd(&h[loc & hmask], 1u);
        }
    }
    __syncthreads();
    const uint64_t v0 = ((uint64_t)b << bw) + ((uint64_t)pt << cw);
    for (uint32_t j = threadIdx.x; j < nh; j += NTB) {
        const uint64_t v = v0 + j;
        if (v >= (uint64_t)n) break;
        if (splits == 1) deg[v] = h[j];
        else if (h[j]) atomicAdd(&deg[v], h[j]);
    }
}

static void launch_bucket_count(const uint32_t* ep, const uint32_t* bst, int bw, uint32_t nb, uint32_t splits,
                                int32_t n, uint32_t* deg, hipStream_t s) {
    const int cw = bw < DEG_MAX_CW ? bw : DEG_MAX_CW;
    const uint32_t parts = 1u << (bw - cw);
    const dim3 grid(nb * parts * splits);
    if (cw <= 12)
        hipLaunchKernelGGL((k_bucket_count<12, NT>), grid, dim3(NT), 0, s, ep, bst, bw, parts, splits, n, deg);
    else if (cw == 13)
        hipLaunchKernelGGL((k_bucket_count<13, NT>), grid, dim3(NT), 0, s, ep, bst, bw, parts, splits, n, deg);
    else if (cw == 14)   // ids past 24 bits: 2^14 counters (64 KB), 1024 threads (8 blocks ran 2 waves per SIMD)
        hipLaunchKernelGGL((k_bucket_count<14, 1024>), grid, dim3(1024), 0, s, ep, bst, bw, parts, splits, n, deg);
    else
        hipLaunchKernelGGL((k_bucket_count<DEG_MAX_CW, 1024>), grid, dim3(1024), 0, s, ep, bst, bw, parts, splits, n,
                           deg);
}

// deg[n - 1] -= the sentinel endpoints written by k_endpoints.
__global__ __launch_bounds__(NT) void k_drop_sentinels(const uint32_t* __restrict__ nsent, uint32_t nblocks,
                                                       int32_t n, uint32_t* __restrict__ deg) {
    __shared__ uint32_t red[NT / WAVE];
    uint32_t t = 0;
    for (uint32_t i = threadIdx.x; i < nblocks; i += NT) t += nsent[i];
    t = wave_sum(t);
    if (lane_id() == 0) red[wave_id()] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int k = 0; k < NT / WAVE; ++k) s += red[k];
        deg[n - 1] -= s;
    }
}

// dend[v] = one past the last occurrence of v among the sorted endpoints.
__global__ __launch_bounds__(NT) void k_endpoint_bounds(const uint32_t* __restrict__ keys, uint64_t len, int32_t n,
                                                        uint32_t* __restrict__ dend) {
    for (uint64_t i = (uint64_t)blockIdx.x * NT + threadIdx.x; i < len; i += (uint64_t)gridDim.x * NT) {
        const uint32_t v = keys[i];
        if (v < (uint32_t)n && (i + 1 == len || keys[i + 1] != v)) dend[v] = (uint32_t)(i + 1);
    }
}

// Key (degree, id); OFFSETS: deg holds degree offsets [n + 1], else counts [n].
template <bool OFFSETS>
__global__ __launch_bounds__(NT) void k_vertex_keys(const uint32_t* __restrict__ deg, int32_t n,
                                                    uint64_t* __restrict__ keys) {
    for (int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x; v < n; v += (int64_t)gridDim.x * NT) {
        const uint32_t d = OFFSETS ? deg[v + 1] - deg[v] : deg[v];
        keys[v] = ((uint64_t)d << 32) | (uint32_t)v;
    }
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
// Pair -> (lo rank << nb) | hi rank. Loops and invalid ids become the all-ones
// sentinel on 2*nb bits, which exceeds every valid key (lo rank <= n - 2).
// Eight pairs per thread per step, all loads issued before any is used: the
// rank lookups are random gathers, so the kernel lives on memory-level
// parallelism.
constexpr int OR_U = 8;
// sort tiles (radix_tile_keys) are whole multiples of one round, OR_U * NT keys
// U pairs per thread per step: 16 where the tile is a multiple of 16 * NT
// (4096- and 8192-key tiles; 0.21 -> 0.20 ms at R-MAT 20, no change at larger
// sizes, where the gathers' line traffic bounds the kernel), else OR_U.
template <int U>
__global__ __launch_bounds__(NT) void k_orient(const int2* __restrict__ edges, uint64_t E, int32_t n,
                                               const uint32_t* __restrict__ rank, int nb, uint64_t sentinel,
                                               uint64_t* __restrict__ keys, uint32_t* __restrict__ counts,
                                               uint32_t ntiles, uint32_t tile_keys, RadixDigit dg) {
    // block step = one tile of the pair sort; its first digit is counted as the keys are made
    __shared__ TileCounts tc;
    tc.clear();
    __syncthreads();
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
      for (uint32_t r = 0; r < tile_keys; r += U * NT) {
        const uint64_t i0 = (uint64_t)tile * tile_keys + r + threadIdx.x;
        int2 ed[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const uint64_t i = i0 + (uint64_t)k * NT;
            ed[k] = i < E ? edges[i] : make_int2(-1, -1);
        }
        uint32_t ra[U], rb[U];
        bool ok[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            ok[k] = ed[k].x >= 0 && ed[k].x < n && ed[k].y >= 0 && ed[k].y < n && ed[k].x != ed[k].y;
            ra[k] = rank[ok[k] ? ed[k].x : 0];
            rb[k] = rank[ok[k] ? ed[k].y : 0];
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const uint64_t i = i0 + (uint64_t)k * NT;
            if (i < E) {
                const uint32_t lo = ra[k] < rb[k] ? ra[k] : rb[k], hi = ra[k] < rb[k] ? rb[k] : ra[k];
                const uint64_t key = ok[k] ? (((uint64_t)lo << nb) | hi) : sentinel;
                keys[i] = key;
                if (counts) tc.add((uint32_t)(key >> dg.shift) & dg.mask);
            }
        }
      }
        if (counts) tc.flush(counts, ntiles, tile);
    }
}

// Orientation past 2^21 vertices. There the rank table (4 bytes per vertex)
// outgrows an XCD's 4 MB L2, and two random rank gathers per pair cost two cache
// lines from beyond it. Instead the pairs pass through two stable radix passes
// (radix_pass_u64): one on the high bits of the first id, one on the high bits of
// the second that also replaces the first id by its rank as the pair moves. The
// first pass of the pair sort then reads (second id << 32 | rank of the first
// id), grouped by the second id's high bits, looks up the second rank and forms
// the oriented key as it loads each pair (RX_ORIENT, in its histogram and its
// scatter alike). The blocks of each pass look up ranks in a few
// 2^(vbits - 8)-id ranges at a time, which stay in L2.
constexpr int ORIENT_PART_MIN_BITS = 21;
constexpr int ORIENT_PART_BITS = 8;   // digit of each partition pass

// ------------------------------------------------------------------ unique + CSR
// The sorted pair keys in runs of equal keys: the first of each run is kept,
// sentinel keys (loops, invalid ids; they sort last) are dropped. Each block
// owns a chunk of whole 2048-key tiles, whose kept keys the row sort has
// counted; in a tile, thread t takes the UQ_ITEMS consecutive keys from
// t * UQ_ITEMS (four 16-byte loads, in flight together), so a block scans once
// per tile rather than once per 256 keys; the kept keys are compacted in LDS
// and written out in contiguous runs.
constexpr int UQ_MAX_BLOCKS = 1024;
constexpr int UQ_ITEMS = 8;
constexpr uint32_t UQ_TILE = NT * UQ_ITEMS;

struct Chunking {
    uint32_t nblk, chunk;
};

static Chunking chunking(uint64_t len) {
    uint32_t nblk = (uint32_t)((len + 8191) / 8192);
    if (nblk > (uint32_t)UQ_MAX_BLOCKS) nblk = UQ_MAX_BLOCKS;
    if (nblk < 1) nblk = 1;
    uint64_t chunk = (len + nblk - 1) / nblk;
    chunk = (chunk + UQ_TILE - 1) / UQ_TILE * UQ_TILE;
    if (chunk == 0) chunk = UQ_TILE;
    nblk = (uint32_t)((len + chunk - 1) / chunk);
    if (nblk < 1) nblk = 1;
    return {nblk, (uint32_t)chunk};
}

struct alignas(16) U64x2 {
    uint64_t a, b;
};

// Keys i0 .. i0 + UQ_ITEMS - 1 (i0 a multiple of UQ_ITEMS); `fill` past E.
__device__ __forceinline__ void uq_load(const uint64_t* __restrict__ keys, uint64_t i0, uint64_t E, uint64_t fill,
                                        uint64_t (&k)[UQ_ITEMS]) {
    if (i0 + UQ_ITEMS <= E) {
        const U64x2* p = (const U64x2*)(keys + i0);   // 64-byte aligned
#pragma unroll
        for (int q = 0; q < UQ_ITEMS / 2; ++q) {
            const U64x2 v = p[q];
            k[2 * q] = v.a;
            k[2 * q + 1] = v.b;
        }
    } else {
#pragma unroll
        for (int j = 0; j < UQ_ITEMS; ++j) k[j] = i0 + j < E ? keys[i0 + j] : fill;
    }
}

// Bit j: key i0 + j is the first of its run and not the sentinel.
__device__ __forceinline__ uint32_t uq_keep(const uint64_t* __restrict__ keys, uint64_t i0, uint64_t sentinel,
                                            const uint64_t (&k)[UQ_ITEMS]) {
    uint64_t prev = i0 > 0 ? keys[i0 - 1] : ~k[0];
    uint32_t keep = 0;
#pragma unroll
    for (int j = 0; j < UQ_ITEMS; ++j) {
        keep |= (k[j] != sentinel && k[j] != prev) ? 1u << j : 0u;
        prev = k[j];
    }
    return keep;
}

// Keeps the first of every run of equal keys; rowend[s] = number of kept keys
// up to and including the last key of row s.
__global__ __launch_bounds__(NT) void k_unique_write(const uint64_t* __restrict__ keys, uint64_t E, uint64_t sentinel,
                                                     Ctrl* ctrl, uint32_t chunk, const uint32_t* __restrict__ partial,
                                                     uint32_t nblk, int nb, uint32_t* __restrict__ col,
                                                     uint32_t* __restrict__ src, uint32_t* __restrict__ rowend) {
    __shared__ uint32_t scratch[NT / WAVE];
    __shared__ uint32_t s_col[UQ_TILE], s_src[UQ_TILE];   // the tile's kept keys, compacted
    const uint64_t b0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t b1 = b0 + chunk < E ? b0 + chunk : E;
    const uint64_t lowmask = (1ull << nb) - 1ull;
    uint32_t carry = partial[blockIdx.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->m = partial[nblk];
    for (uint64_t t0 = b0; t0 < b1; t0 += UQ_TILE) {   // the same trip count in every thread
        const uint64_t i0 = t0 + (uint64_t)threadIdx.x * UQ_ITEMS;
        uint64_t k[UQ_ITEMS];
        uint32_t keep = 0;
        uint64_t next = sentinel;   // the key after this thread's last one
        if (i0 < b1) {
            uq_load(keys, i0, E, sentinel, k);
            keep = uq_keep(keys, i0, sentinel, k);
            if (i0 + UQ_ITEMS < E) next = keys[i0 + UQ_ITEMS];
        }
        uint32_t total;
        const uint32_t ex = block_exclusive_scan<NT>((uint32_t)__popc(keep), scratch, &total);
        uint32_t pos = carry + ex, lp = ex;
        if (i0 < b1) {
#pragma unroll
            for (int j = 0; j < UQ_ITEMS; ++j) {
                if (k[j] == sentinel) break;   // the sentinels (and the fill past E) come last
                const uint32_t s = (uint32_t)(k[j] >> nb);
                const uint32_t kp = (keep >> j) & 1u;
                if (kp) {
                    s_col[lp] = (uint32_t)(k[j] & lowmask);
                    s_src[lp] = s;
                }
                pos += kp;
                lp += kp;
                // the sentinel's row differs from every valid row
                const uint64_t nx = j + 1 < UQ_ITEMS ? k[j + 1] : next;
                if ((uint32_t)(nx >> nb) != s) rowend[s] = pos;
            }
        }
        // the kept keys leave in contiguous runs (a thread's own ones are up to
        // eight scattered 4-byte stores per lane otherwise)
        __syncthreads();
        for (uint32_t q = threadIdx.x; q < total; q += NT) {
            col[carry + q] = s_col[q];
            src[carry + q] = s_src[q];
        }
        __syncthreads();
        carry += total;
    }
}

// ------------------------------------------------------------------ CSC (in-edges grouped by v)
// Key of an in-edge e = (u -> v) with a non-empty tail: v in the bits above
// sh, then e, and (packed form, lbits > 0) the tail length in the low lbits
// bits; others get v = n - 1 and sort last: the top-ranked vertex has no
// out-neighbours, so none of its in-edges has work, and ids then need
// bits_for(n) bits, not bits_for(n + 1) (one pass less when n is a power of
// two). In-edges of other vertices without out-neighbours keep their group:
// such a vertex gets no bucket and no tile, so they are never read (testing
// d+(v) here would cost a random gather per edge). A length that does not fit
// the packed field is stored as all ones, and the row end of u is gathered for
// that entry later. Packing saves that gather for the others.
__global__ __launch_bounds__(NT) void k_csc_keys(const uint32_t* __restrict__ col, const uint32_t* __restrict__ src,
                                                 const uint32_t* __restrict__ off, Ctrl* ctrl, int32_t n,
                                                 uint64_t* __restrict__ keys, int sh, int lbits,
                                                 uint32_t* __restrict__ counts, uint32_t ntiles, uint32_t tile_keys,
                                                 RadixDigit dg) {
    __shared__ TileCounts tc;
    tc.clear();
    __syncthreads();
    const uint32_t m = ctrl->m;
    const uint64_t esc = (1ull << lbits) - 1ull;   // escape: length gathered at expansion
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
      for (uint32_t r = 0; r < tile_keys; r += OR_U * NT) {
        const uint64_t e0 = (uint64_t)tile * tile_keys + r + threadIdx.x;
        uint32_t v[OR_U], u[OR_U];
#pragma unroll
        for (int k = 0; k < OR_U; ++k) {   // loads of all OR_U edges in flight together
            const uint64_t e = e0 + (uint64_t)k * NT;
            v[k] = e < m ? col[e] : 0u;
            u[k] = e < m ? src[e] : 0u;
        }
        uint32_t end[OR_U];
#pragma unroll
        for (int k = 0; k < OR_U; ++k) end[k] = off[u[k] + 1];   // rows ascend with e: near-sequential
#pragma unroll
        for (int k = 0; k < OR_U; ++k) {
            const uint64_t e = e0 + (uint64_t)k * NT;
            if (e >= m) continue;
            const bool work = e + 1 < end[k];   // a non-empty tail
            uint64_t low = e;
            if (lbits > 0) {
                const uint64_t len = work ? end[k] - (e + 1) : 0u;
                low = (low << lbits) | (len < esc ? len : esc);
            }
            const uint64_t key = ((uint64_t)(work ? v[k] : (uint32_t)(n - 1)) << sh) | low;
            keys[e] = key;
            if (counts) tc.add((uint32_t)(key >> dg.shift) & dg.mask);
        }
      }
        if (counts) tc.flush(counts, ntiles, tile);
    }
}

// One pass over the sorted in-edge keys: inend[v] = one past the last in-edge
// of v and m_active from the group boundaries, and each key with work written
// to out (the other buffer: neighbours' keys are still being read) as the tail
// range of its edge e, start (e + 1) | end << 32, so a kernel reads it in one
// load. Packed keys carry the length; otherwise the row end of u is gathered.
// Thread t takes keys 2t and 2t + 1 (16-byte loads and stores, coalesced
// across the wave) and reads the key after them.
__device__ __forceinline__ uint64_t csc_range(uint64_t key, uint64_t emask, uint64_t lmask, int lbits,
                                              const uint32_t* __restrict__ src, const uint32_t* __restrict__ off) {
    uint32_t e, end;
    if (lbits > 0) {
        e = (uint32_t)((key >> lbits) & emask);
        const uint64_t len = key & lmask;
        end = len != lmask ? e + 1u + (uint32_t)len : off[src[e] + 1];
    } else {
        e = (uint32_t)key;
        end = off[src[e] + 1];
    }
    return (uint64_t)(e + 1u) | ((uint64_t)end << 32);
}

__global__ __launch_bounds__(NT) void k_csc_finish(const uint64_t* __restrict__ keys, uint64_t* __restrict__ out,
                                                   Ctrl* ctrl, int32_t n, uint32_t* __restrict__ inend, int sh,
                                                   const uint32_t* __restrict__ src,
                                                   const uint32_t* __restrict__ off, int ebits, int lbits) {
    const uint32_t m = ctrl->m;
    const uint32_t last = (uint32_t)(n - 1);   // the group of in-edges without work
    const uint64_t emask = (1ull << ebits) - 1ull, lmask = (1ull << lbits) - 1ull;
    const uint64_t none = (uint64_t)last << sh;
    for (uint64_t i0 = ((uint64_t)blockIdx.x * NT + threadIdx.x) * 2; i0 < m; i0 += (uint64_t)gridDim.x * NT * 2) {
        uint64_t k0, k1;
        if (i0 + 2 <= m) {
            const U64x2 v = *(const U64x2*)(keys + i0);   // 16-byte aligned
            k0 = v.a;
            k1 = v.b;
        } else {
            k0 = keys[i0];
            k1 = none;
        }
        const uint64_t k2 = i0 + 2 < m ? keys[i0 + 2] : none;
        const uint32_t v0 = (uint32_t)(k0 >> sh), v1 = (uint32_t)(k1 >> sh), v2 = (uint32_t)(k2 >> sh);
        if (v0 < last && v1 != v0) {
            inend[v0] = (uint32_t)(i0 + 1);
            if (v1 == last) ctrl->m_active = (uint32_t)(i0 + 1);
        }
        if (i0 + 1 < m && v1 < last && v2 != v1) {
            inend[v1] = (uint32_t)(i0 + 2);
            if (v2 == last) ctrl->m_active = (uint32_t)(i0 + 2);
        }
        const uint64_t r0 = v0 < last ? csc_range(k0, emask, lmask, lbits, src, off) : 0ull;
        const uint64_t r1 = v1 < last ? csc_range(k1, emask, lmask, lbits, src, off) : 0ull;
        if (i0 + 2 <= m) {
            U64x2 w;
            w.a = r0;
            w.b = r1;
            *(U64x2*)(out + i0) = w;
        } else {
            out[i0] = r0;
        }
    }
}

// ------------------------------------------------------------------ the other formulations
// All in-edges, grouped by v and, inside a group, in CSR order (so by u): key
// v << sh | e, sorted on the v bits only (the sort is stable).
__global__ __launch_bounds__(NT) void k_sym_keys(const uint32_t* __restrict__ col, const Ctrl* ctrl,
                                                 uint64_t* __restrict__ keys, int sh) {
    const uint32_t m = ctrl->m;
    for (uint64_t e = (uint64_t)blockIdx.x * NT + threadIdx.x; e < m; e += (uint64_t)gridDim.x * NT)
        keys[e] = ((uint64_t)col[e] << sh) | e;
}

// inend[v] = one past the last in-edge of v in the sorted order.
__global__ __launch_bounds__(NT) void k_sym_bounds(const uint64_t* __restrict__ keys, const Ctrl* ctrl,
                                                   uint32_t* __restrict__ inend, int sh) {
    const uint32_t m = ctrl->m;
    for (uint64_t i = (uint64_t)blockIdx.x * NT + threadIdx.x; i < m; i += (uint64_t)gridDim.x * NT) {
        const uint64_t v = keys[i] >> sh;
        if (i + 1 == m || (keys[i + 1] >> sh) != v) inend[v] = (uint32_t)(i + 1);
    }
}

// Row offsets of the symmetric adjacency: row v holds N-(v) (in-neighbours,
// all ranked below v) and then N+(v), so fo[v] = inoff[v] + off[v].
__global__ __launch_bounds__(NT) void k_sym_rows(const uint32_t* __restrict__ inoff, const uint32_t* __restrict__ off,
                                                 int32_t n, uint32_t* __restrict__ fo) {
    for (int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x; v <= n; v += (int64_t)gridDim.x * NT)
        fo[v] = inoff[v] + off[v];
}

// Per sorted in-edge i = (u -> v), edge e: (full rows) the two copies of the
// edge in the symmetric adjacency, u at position i - inoff[v] of row v's lower
// part (fo[v] + i - inoff[v] = off[v] + i) and v at position e - off[u] of row
// u's upper part (fo[u] + indeg(u) + e - off[u] = inoff[u + 1] + e); then the
// key becomes the range that the edge streams, start | end << 32.
__global__ __launch_bounds__(NT) void k_sym_build(uint64_t* __restrict__ keys, const Ctrl* ctrl,
                                                  const uint32_t* __restrict__ src, const uint32_t* __restrict__ col,
                                                  const uint32_t* __restrict__ off, const uint32_t* __restrict__ inoff,
                                                  uint32_t* __restrict__ fcol, int sh, int form) {
    const uint32_t m = ctrl->m;
    const uint64_t emask = (1ull << sh) - 1ull;
    for (uint64_t i = (uint64_t)blockIdx.x * NT + threadIdx.x; i < m; i += (uint64_t)gridDim.x * NT) {
        const uint64_t key = keys[i];
        const uint32_t v = (uint32_t)(key >> sh), e = (uint32_t)(key & emask);
        const uint32_t u = src[e];
        const uint32_t ua = off[u], ub = off[u + 1];
        uint32_t st = ua, en = ub;   // MATRIX_UPPER: N+(u) in the oriented columns
        if (form != FORM_MATRIX_UPPER) {
            const uint32_t i0 = inoff[u], i1 = inoff[u + 1];
            fcol[off[v] + (uint32_t)i] = u;
            fcol[i1 + e] = v;
            st = form == FORM_FULL ? i0 + ua : i1 + ua;   // whole row of u, or its upper part
            en = i1 + ub;
        }
        keys[i] = (uint64_t)st | ((uint64_t)en << 32);
    }
}

// ------------------------------------------------------------------ buckets
__device__ __forceinline__ uint32_t bucket_of(uint32_t din, uint32_t dout) {
    if (din == 0 || dout == 0) return BUCKET_NONE;
    const uint32_t li = min(14, floor_log2(din));
    const uint32_t lo = min(15, floor_log2(dout));
    return 16u * li + lo;
}

__global__ __launch_bounds__(NT) void k_vbucket(const uint32_t* __restrict__ off, const uint32_t* __restrict__ col,
                                                const uint32_t* __restrict__ inoff, int32_t n,
                                                uint8_t* __restrict__ vbucket, Ctrl* ctrl) {
    __shared__ uint32_t s_nv[NBUCKET];
    __shared__ unsigned long long s_in[NBUCKET], s_out[NBUCKET], s_work[NBUCKET], s_win[NBUCKET];
    for (int b = threadIdx.x; b < NBUCKET; b += NT) {
        s_nv[b] = 0;
        s_in[b] = 0;
        s_out[b] = 0;
        s_work[b] = 0;
        s_win[b] = 0;
    }
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x; v < n; v += (int64_t)gridDim.x * NT) {
        const uint32_t din = inoff[v + 1] - inoff[v], dout = off[v + 1] - off[v];
        const uint32_t b = bucket_of(din, dout);
        vbucket[v] = (uint8_t)b;
        if (b != BUCKET_NONE) {
            atomicAdd(&s_nv[b], 1u);
            atomicAdd(&s_in[b], (unsigned long long)din);
            atomicAdd(&s_out[b], (unsigned long long)dout);
            atomicAdd(&s_work[b], (unsigned long long)din * dout);
            // windows the bitmap strategy walks for this middle list (first one
            // aligned down to a word)
            const uint32_t lo = col[off[v]], hi = col[off[v + 1] - 1];
            atomicAdd(&s_win[b], (unsigned long long)(((hi - (lo & ~31u)) >> BM_WINDOW_LOG2) + 1u));
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < NBUCKET; b += NT) {
        if (s_nv[b]) {
            atomicAdd(&ctrl->bucket_nv[b], s_nv[b]);
            atomicAdd((unsigned long long*)&ctrl->bucket_in[b], s_in[b]);
            atomicAdd((unsigned long long*)&ctrl->bucket_out[b], s_out[b]);
            atomicAdd((unsigned long long*)&ctrl->bucket_work[b], s_work[b]);
            atomicAdd((unsigned long long*)&ctrl->bucket_win[b], s_win[b]);
        }
    }
}

// ------------------------------------------------------------------ selection
// One thread per bucket. The heuristic follows the paper's dynamic grouping:
// fixed degree thresholds decide between the cooperative (staged) and the
// per-pair strategies. Here the staged LDS bitmap takes middle vertices with
// at least 64 in-edges, or at least 16 in-edges and 64 out-neighbours (the
// bitmap's set-up is then amortised), binary search takes lists of at least
// 16 out-neighbours, and merge-path the rest. The thresholds were chosen from
// per-bucket timings of all three kernels on R-MAT and Chung-Lu graphs of
// 2^17 to 2^22 vertices and on a batch of 4096 small Chung-Lu graphs.
__device__ int heuristic_choice(int b) {
    const int li = b >> 4, lo = b & 15;   // floor log2 of in-degree and out-degree
    if (li >= 6 || (li >= 4 && lo >= 6)) return KER_BITMAP;
    if (lo >= 4) return KER_BSEARCH;
    return KER_MERGE;
}

constexpr uint32_t EDGE_CHUNK_MAX = 2048;   // in-edges per tile of the edge-centric kernels
constexpr unsigned long long EDGE_TILES = 512;

__global__ __launch_bounds__(NBUCKET) void k_select(Ctrl* ctrl, int mode, const uint8_t* __restrict__ learned,
                                                    const uint8_t* __restrict__ learned_tile,
                                                    const uint16_t* __restrict__ chunk_override,
                                                    const uint8_t* __restrict__ group_override, int whole_rows) {
    __shared__ uint32_t s_key[NBUCKET];
    const int b = threadIdx.x;
    int ch;
    if (mode == SEL_FORCE_MERGE) ch = KER_MERGE;
    else if (mode == SEL_FORCE_BSEARCH) ch = KER_BSEARCH;
    else if (mode == SEL_FORCE_BITMAP) ch = KER_BITMAP;
    else if (mode == SEL_LEARNED && learned) ch = learned[b] < NKERNEL ? learned[b] : heuristic_choice(b);
    else ch = heuristic_choice(b);
    const int lo = b & 15, li = b >> 4;
    // tile shape: in-edges per tile and lanes per in-edge.
    // Bitmap tiles of vertices with at least 256 in-edges, and of whole-row tails
    // (cut per bitmap window), take the largest chunk: a tile's set-up (entry
    // table, bitmap of the middle list, dependent loads of its descriptors) is
    // then spread over the most in-edges (measured at R-MAT 20: bitmap kernel
    // 1.24 -> 1.08 ms against 256 in-edges everywhere).
    // The edge-centric kernels' tiles of vertices with short lists (fewer than
    // 64 out-neighbours) grow with the bucket's in-edges, to about EDGE_TILES
    // tiles per bucket, between 256 and 2048 in-edges: their per-tile set-up is
    // a chain of dependent loads that the short lists do not hide (measured: a
    // random geometric graph of 2^23 vertices, merge 6.9 -> 4.4 ms and binary
    // search 5.6 -> 4.2 ms; R-MAT 20, whose edge-kernel buckets are small,
    // keeps 256; longer lists gained nothing and lost at R-MAT 24). The shape
    // depends on the bucket alone, so a bucket timed alone (selector training)
    // runs as it does among the others.
    uint32_t chunk = (ch == KER_BITMAP && (whole_rows || li >= 8)) ? (uint32_t)CHUNK_MAX : 256u;
    if (ch != KER_BITMAP && lo <= 5) {
        const unsigned long long per = ctrl->bucket_in[b] / EDGE_TILES;
        chunk = per < 256ull ? 256u : (per > (unsigned long long)EDGE_CHUNK_MAX ? EDGE_CHUNK_MAX : (uint32_t)per);
    }
    uint32_t group = lo >= 9 ? 64u : (lo >= 3 ? (1u << (lo - 3)) : 1u);
    // the tile network scales the rule's tile size by 1/2, 1 or 2
    if (learned_tile && learned_tile[b] == 0) chunk = chunk / 2u;
    else if (learned_tile && learned_tile[b] == 2) chunk = chunk * 2u;
    if (chunk_override && chunk_override[b]) chunk = chunk_override[b];
    if (group_override && group_override[b]) group = group_override[b];
    const uint32_t cmax = ch == KER_BITMAP ? (uint32_t)CHUNK_MAX : EDGE_CHUNK_MAX;
    if (chunk > cmax) chunk = cmax;
    if (chunk < 16u) chunk = 16u;
    if (group > 64u || (group & (group - 1u))) group = 64u;
    if (group < 1u) group = 1u;
    ctrl->choice[b] = (uint8_t)ch;
    ctrl->chunk[b] = (uint16_t)chunk;
    ctrl->group[b] = (uint8_t)group;
    // slot order: (kernel, heavier tiles first); the empty bucket last
    const uint32_t key = (b == BUCKET_NONE) ? 0xFFFFFFFFu : ((uint32_t)ch << 16) | (uint32_t)(255 - (16 * lo + li));
    s_key[b] = key;
    __syncthreads();
    uint32_t r = 0;
    for (int q = 0; q < NBUCKET; ++q) r += (s_key[q] < key || (s_key[q] == key && q < b)) ? 1u : 0u;
    ctrl->slot[b] = (uint8_t)r;
}

// Vertices per multi-vertex tile for bucket b (1 = chunks of single vertices).
__device__ __forceinline__ uint32_t tile_group(const Ctrl* ctrl, uint32_t b) {
    const uint32_t li = b >> 4;
    if (li >= 14) return 1u;
    const uint32_t maxin = 2u << li;   // in-degrees of the bucket are below this
    const uint32_t K = ctrl->chunk[b];
    if (2u * maxin > K) return 1u;
    const uint32_t g = K / maxin;
    // the edge-centric kernels stage the tile's lists in LDS when they fit:
    // no more vertices than STAGE_MAX list elements at the bucket's longest
    const uint32_t lo = b & 15u;
    const uint32_t stage_cap = lo >= 12 ? 1u : (uint32_t)STAGE_MAX / (2u << lo);
    const uint32_t cap = ctrl->choice[b] == KER_BITMAP ? (uint32_t)SEG_MAX_BITMAP
                                                       : (stage_cap < (uint32_t)SEG_MAX ? stage_cap : (uint32_t)SEG_MAX);
    return g > cap ? cap : (g > 1u ? g : 1u);
}

__global__ __launch_bounds__(NT) void k_vkeys_slot(const uint8_t* __restrict__ vbucket, int32_t n, const Ctrl* ctrl,
                                                   uint64_t* __restrict__ keys) {
    for (int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x; v < n; v += (int64_t)gridDim.x * NT)
        keys[v] = ((uint64_t)ctrl->slot[vbucket[v]] << 32) | (uint32_t)v;
}

__global__ __launch_bounds__(NT) void k_vpos(const uint64_t* __restrict__ sorted, int32_t n,
                                             const uint8_t* __restrict__ vbucket, Ctrl* ctrl,
                                             uint32_t* __restrict__ vlist) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const uint32_t v = (uint32_t)sorted[i];
        const uint32_t slot = (uint32_t)(sorted[i] >> 32);
        vlist[i] = v;
        const uint32_t b = vbucket[v];
        if (i == 0 || (uint32_t)(sorted[i - 1] >> 32) != slot) ctrl->bstart[b] = (uint32_t)i;
        if (i == n - 1 || (uint32_t)(sorted[i + 1] >> 32) != slot) ctrl->bend[b] = (uint32_t)(i + 1);
    }
}

__global__ __launch_bounds__(NT) void k_ntiles(const uint32_t* __restrict__ vlist, const uint8_t* __restrict__ vbucket,
                                               const uint32_t* __restrict__ inoff, int32_t n, const Ctrl* ctrl,
                                               uint32_t* __restrict__ ntile) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const uint32_t v = vlist[i];
        const uint32_t b = vbucket[v];
        uint32_t t = 0;
        if (b != BUCKET_NONE) {
            const uint32_t g = tile_group(ctrl, b);
            if (g > 1) {
                t = ((uint32_t)i - ctrl->bstart[b]) % g == 0 ? 1u : 0u;
            } else {
                const uint32_t din = inoff[v + 1] - inoff[v];
                const uint32_t K = ctrl->chunk[b];
                t = (din + K - 1) / K;
            }
        }
        ntile[i] = t;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ntile[n] = 0;
}

__global__ __launch_bounds__(NT) void k_emit_tiles(const uint32_t* __restrict__ vlist,
                                                   const uint8_t* __restrict__ vbucket,
                                                   const uint32_t* __restrict__ inoff,
                                                   const uint32_t* __restrict__ tstart, int32_t n, Ctrl* ctrl,
                                                   uint4* __restrict__ tiles, uint64_t tile_cap) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const uint32_t b = vbucket[vlist[i]];
        const int kk = b == BUCKET_NONE ? NKERNEL : ctrl->choice[b];
        int kprev = -1;
        if (i > 0) {
            const uint32_t bp = vbucket[vlist[i - 1]];
            kprev = bp == BUCKET_NONE ? NKERNEL : ctrl->choice[bp];
        }
        const uint32_t t0 = tstart[i], t1 = tstart[i + 1];
        if (t1 > t0 && b != BUCKET_NONE) {
            const uint32_t g = tile_group(ctrl, b);
            if (g > 1) {
                const uint32_t cnt = min(g, ctrl->bend[b] - (uint32_t)i);
                if (t0 < tile_cap) tiles[t0] = make_uint4((uint32_t)i, cnt, 0u, TILE_MULTI);
            } else {
                const uint32_t v = vlist[i];
                const uint32_t K = ctrl->chunk[b];
                const uint32_t e_beg = inoff[v], e_end = inoff[v + 1];
                for (uint32_t t = t0; t < t1 && t < tile_cap; ++t) {
                    const uint32_t e0 = e_beg + (t - t0) * K;
                    tiles[t] = make_uint4(v, e0, (e0 + K < e_end ? e0 + K : e_end) - e0, 0u);
                }
            }
        }
        for (int k = kprev + 1; k <= kk; ++k) ctrl->tile_begin[k] = t0;
        if (i == n - 1) {
            for (int k = kk + 1; k <= NKERNEL; ++k) ctrl->tile_begin[k] = tstart[n];
            ctrl->ntiles = tstart[n];
        }
    }
}

// ------------------------------------------------------------------ outputs
__global__ __launch_bounds__(NT) void k_map_pv(const uint64_t* __restrict__ pv, const uint32_t* __restrict__ inv,
                                               int32_t n, uint64_t* __restrict__ out) {
    for (int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x; r < n; r += (int64_t)gridDim.x * NT) out[inv[r]] = pv[r];
}

// ------------------------------------------------------------------ clustering epilogue
// Local clustering coefficient C(v) = t[v] / C(d(v), 2) (zero when d(v) < 2)
// and the number of wedges (paths of length two) sum_v C(d(v), 2), which with
// T gives the transitivity 3T / wedges. d(v) is the simple-graph degree: the
// out-degree of v's CSR row plus its in-degree over the kept edges.
constexpr unsigned CL_MAX_BLOCKS = 4096;   // block partials live in the intersection partials

__global__ __launch_bounds__(NT) void k_indeg(const uint32_t* __restrict__ col, const Ctrl* ctrl,
                                              uint32_t* __restrict__ indeg) {
    const uint32_t m = ctrl->m;
    for (uint64_t e = (uint64_t)blockIdx.x * NT + threadIdx.x; e < m; e += (uint64_t)gridDim.x * NT)
        atomicAdd(&indeg[col[e]], 1u);
}

__global__ __launch_bounds__(NT) void k_clustering(const uint64_t* __restrict__ t, const uint32_t* __restrict__ inv,
                                                   const uint32_t* __restrict__ off,
                                                   const uint32_t* __restrict__ indeg, int32_t n,
                                                   double* __restrict__ coeff, uint64_t* __restrict__ partials) {
    __shared__ uint64_t red[NT / WAVE];
    uint64_t acc = 0;
    for (int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x; r < n; r += (int64_t)gridDim.x * NT) {
        const uint64_t d = (uint64_t)(off[r + 1] - off[r]) + indeg[r];
        const uint64_t w = d < 2 ? 0ull : d * (d - 1) / 2;
        acc += w;
        coeff[inv[r]] = w ? (double)t[r] / (double)w : 0.0;
    }
    acc = wave_sum_u64(acc);
    if (lane_id() == 0) red[wave_id()] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        for (int i = 0; i < NT / WAVE; ++i) s += red[i];
        partials[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(NT) void k_sum_wedges(const uint64_t* __restrict__ partials, unsigned count, Ctrl* ctrl) {
    __shared__ uint64_t red[NT / WAVE];
    uint64_t acc = 0;
    for (unsigned i = threadIdx.x; i < count; i += NT) acc += partials[i];
    acc = wave_sum_u64(acc);
    if (lane_id() == 0) red[wave_id()] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        for (int i = 0; i < NT / WAVE; ++i) s += red[i];
        ctrl->wedges = s;
    }
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

__global__ void k_set_tile_range(Ctrl* ctrl, int ker, uint32_t t0, uint32_t t1) {
    if (threadIdx.x == 0) {
        ctrl->tile_begin[ker] = t0;
        ctrl->tile_begin[ker + 1] = t1;
        ctrl->tile_next[ker] = 0;
    }
}

// The intersection kernels' shared tile counters, zeroed before a relaunch.
static void reset_tile_counters(Ctrl* ctrl, hipStream_t s) {
    fill_u32(ctrl->tile_next, 0u, NKERNEL + 1, s);
}

// result[0] = T, result[1] = range_status when an id was out of range, else 0.
__global__ void k_publish(const Ctrl* ctrl, uint64_t* result, uint64_t range_status, uint64_t internal_status) {
    if (threadIdx.x == 0) {
        result[0] = ctrl->total;
        result[1] = (ctrl->err & 1u) ? range_status : (ctrl->err ? internal_status : 0ull);
    }
}

void publish_result(const Ctrl* ctrl, uint64_t* result, uint64_t range_status, uint64_t internal_status,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, ctrl, result, range_status, internal_status);
}

// Packed in-edge keys: v, e, and the tail length in the bits left over (at
// most what the bound d+(u) <= sqrt(2E) needs; lengths that do not fit are
// escaped). Without room for at least 6 length bits, e alone is kept.
struct CscPacking {
    int sh, ebits, lbits;
};

static CscPacking csc_packing(int64_t E, int32_t n) {
    const uint64_t twoE = 2ull * (uint64_t)E;
    uint64_t r = (uint64_t)sqrt((double)twoE);   // floor(sqrt(2E)), the bound on d+(u)
    while (r * r > twoE) --r;
    while ((r + 1) * (r + 1) <= twoE) ++r;
    const int eb = bits_for((uint64_t)E), vb = bits_for((uint64_t)n);
    int lb = bits_for(r + 2);   // lengths below r + 1, plus the escape value
    if (lb > 64 - vb - eb) lb = 64 - vb - eb;
    if (lb >= 6) return {eb + lb, eb, lb};
    return {32, 32, 0};
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
    L.deg = take(4 * (nn + 1));
    L.rank = take(4 * nn);
    L.inv = take(4 * nn);
    L.vbucket = take(nn);
    L.vlist = take(4 * nn);
    L.tstart = take(4 * (nn + 1));
    L.off = take(4 * (nn + 1));
    L.inoff = take(4 * (nn + 1));
    L.rowend = take(4 * nn);
    L.pv = take(8 * nn);
    L.vkeysA = take(8 * nn);
    L.vkeysB = take(8 * nn);
    L.keysA = take(8 * kcap);
    L.keysB = take(8 * kcap);
    L.col = take(4 * ee);
    L.src = take(4 * ee);
    L.tile_cap = ee / 16 + nn + 1;
    L.tiles = take(16 * L.tile_cap);
    L.partial = take(4 * (UQ_MAX_BLOCKS + 1));
    L.bstart = take(4 * ((1u << DEG_MAX_BUCKET_BITS) + 4));
    L.isect_partials = take(isect_partials_bytes());
    L.scan_tmp = take(scan_temp_bytes());
    L.lb_aux = take(4 * 256);
    L.radix_tmp = take(radix_temp_bytes(2 * ee > nn ? 2 * ee : nn));
    L.total = o;
    return L;
}

// ------------------------------------------------------------------ the pipeline
int stage_count() { return NSTAGE; }
const char* stage_name(int s) {
    static const char* names[NSTAGE] = {"degree", "rank", "orient", "sort", "csr", "csc", "bucket",
                                        "group", "isect_merge", "isect_bsearch", "isect_bitmap", "finish"};
    return (s >= 0 && s < NSTAGE) ? names[s] : "";
}

// The symmetric adjacency of the other formulations, after the pipeline's own workspace.
static uint32_t* sym_off(const RunArgs& r, const Layout& L) { return (uint32_t*)((char*)r.ws + L.total); }
static uint32_t* sym_col(const RunArgs& r, const Layout& L) {
    return (uint32_t*)((char*)r.ws + L.total + align_up(4 * ((size_t)r.n + 1), 256));
}

static IsectArgs isect_args(const RunArgs& r, const Layout& L, uint64_t* csc) {
    char* ws = (char*)r.ws;
    const bool sym = r.formulation == FORM_FULL || r.formulation == FORM_MATRIX;
    IsectArgs ia;
    ia.ctrl = (Ctrl*)(ws + L.ctrl);
    ia.off = sym ? sym_off(r, L) : (const uint32_t*)(ws + L.off);
    ia.col = sym ? sym_col(r, L) : (const uint32_t*)(ws + L.col);
    ia.src = (const uint32_t*)(ws + L.src);
    ia.csc = csc;
    ia.inoff = (const uint32_t*)(ws + L.inoff);
    ia.vlist = (const uint32_t*)(ws + L.vlist);
    ia.vbucket = (const uint8_t*)(ws + L.vbucket);
    ia.tiles = (const uint4*)(ws + L.tiles);
    ia.per_edge = r.per_edge_counts;
    ia.per_vertex = (r.per_vertex || r.clustering) ? (uint64_t*)(ws + L.pv) : nullptr;
    ia.per_middle = r.per_middle ? (uint64_t*)(ws + L.pv) : nullptr;
    ia.support = r.support;
    ia.list_off = r.list_off;
    ia.list_cur = r.list_cur;
    ia.list_out = r.list_out;
    ia.list_cap = r.list_cap;
    ia.inv = (const uint32_t*)(ws + L.inv);
    ia.col_narrow = (sym ? 2 * r.E : r.E) < ((int64_t)1 << 30) ? 1u : 0u;   // m <= E
    ia.clip = r.formulation != FORM_FILTERED ? 1u : 0u;
    return ia;
}

// Where the CSC array ended up (it depends on the parity of the sort passes;
// the filtered form's tail ranges are written to the buffer its sort left free).
static uint64_t* csc_of(const RunArgs& r, const Layout& L) {
    char* ws = (char*)r.ws;
    const int nb = bits_for((uint64_t)r.n) > 0 ? bits_for((uint64_t)r.n) : 1;
    const int p1 = (nb + 7) / 8;                       // radix passes of the pair sort (on the row)
    const int p2 = (bits_for((uint64_t)r.n) + 7) / 8;   // passes of the CSC sort
    uint64_t* sorted = (p1 & 1) ? (uint64_t*)(ws + L.keysB) : (uint64_t*)(ws + L.keysA);
    uint64_t* other = (p1 & 1) ? (uint64_t*)(ws + L.keysA) : (uint64_t*)(ws + L.keysB);
    const bool keys_in_sorted = (p2 & 1) != 0;
    return keys_in_sorted == (r.formulation == FORM_FILTERED) ? other : sorted;
}

hipError_t launch_isect_stage(const RunArgs& r, hipEvent_t* ev) {
    const Layout L = make_layout(r.E, r.n);
    const IsectArgs ia = isect_args(r, L, csc_of(r, L));
    uint64_t* partials = (uint64_t*)((char*)r.ws + L.isect_partials);
    const int order[NKERNEL] = {KER_MERGE, KER_BSEARCH, KER_BITMAP};
    reset_tile_counters(ia.ctrl, r.stream);
    if (ev) (void)hipEventRecord(ev[0], r.stream);
    for (int q = 0; q < NKERNEL; ++q) {
        const int k = order[q];
        launch_isect(k, ia, r.grid_override ? r.grid_override[k] : 0, partials, r.stream);
        if (ev) (void)hipEventRecord(ev[1 + q], r.stream);
    }
    launch_reduce_total(partials, ia.ctrl, r.stream);
    return hipGetLastError();
}

hipError_t run_list_pass(const RunArgs& r) {
    const Layout L = make_layout(r.E, r.n);
    const IsectArgs ia = isect_args(r, L, csc_of(r, L));
    uint64_t* partials = (uint64_t*)((char*)r.ws + L.isect_partials);
    reset_tile_counters(ia.ctrl, r.stream);
    for (int k = 0; k < NKERNEL; ++k) launch_isect(k, ia, r.grid_override ? r.grid_override[k] : 0, partials, r.stream);
    return hipGetLastError();
}

__global__ __launch_bounds__(NT) void k_widen(const uint32_t* __restrict__ in, uint64_t* __restrict__ out,
                                              const Ctrl* ctrl) {
    const uint32_t m = ctrl->m;
    for (uint64_t i = (uint64_t)blockIdx.x * NT + threadIdx.x; i < m; i += (uint64_t)gridDim.x * NT) out[i] = in[i];
}

void widen_u32_u64(const uint32_t* in, uint64_t* out, const Ctrl* ctrl, size_t cap, hipStream_t s) {
    hipLaunchKernelGGL(k_widen, dim3(grid_for(cap)), dim3(NT), 0, s, in, out, ctrl);
}

size_t sym_extra_bytes(int64_t E, int32_t n) {
    return align_up(4 * ((size_t)n + 1), 256) + align_up(8 * ((size_t)E > 0 ? (size_t)E : 1), 256);
}

size_t list_extra_bytes(int64_t E) {
    return align_up(8 * ((size_t)E + 1), 256) + align_up(4 * ((size_t)E > 0 ? (size_t)E : 1), 256);
}

hipError_t launch_isect_range(const RunArgs& r, int ker, uint32_t t0, uint32_t t1) {
    const Layout L = make_layout(r.E, r.n);
    IsectArgs ia = isect_args(r, L, csc_of(r, L));
    hipLaunchKernelGGL(k_set_tile_range, dim3(1), dim3(64), 0, r.stream, ia.ctrl, ker, t0, t1);   // zeroes the counter
    launch_isect(ker, ia, r.grid_override ? r.grid_override[ker] : 0, (uint64_t*)((char*)r.ws + L.isect_partials),
                 r.stream);
    return hipGetLastError();
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
    uint32_t* vlist = (uint32_t*)(ws + L.vlist);
    uint32_t* tstart = (uint32_t*)(ws + L.tstart);
    uint32_t* off = (uint32_t*)(ws + L.off);
    uint32_t* inoff = (uint32_t*)(ws + L.inoff);
    uint32_t* rowend = (uint32_t*)(ws + L.rowend);
    uint64_t* pv = (uint64_t*)(ws + L.pv);
    uint64_t* vkeysA = (uint64_t*)(ws + L.vkeysA);
    uint64_t* vkeysB = (uint64_t*)(ws + L.vkeysB);
    uint64_t* keysA = (uint64_t*)(ws + L.keysA);
    uint64_t* keysB = (uint64_t*)(ws + L.keysB);
    uint32_t* col = (uint32_t*)(ws + L.col);
    uint32_t* src = (uint32_t*)(ws + L.src);
    uint4* tiles = (uint4*)(ws + L.tiles);
    uint32_t* partial = (uint32_t*)(ws + L.partial);
    void* scan_tmp = ws + L.scan_tmp;
    void* radix_tmp = ws + L.radix_tmp;
    const int2* edges = (const int2*)r.edges;
    const size_t kcap = (size_t)(E > n ? E : n);

    auto mark = [&](int stage) {
        if (r.events) (void)hipEventRecord(r.events[stage], s);
    };
    mark(0);
    // ---- degree: input pairs per vertex, from the sorted endpoints
    fill_u32((uint32_t*)ctrl, 0u, sizeof(Ctrl) / 4, s);
    // bucket width: one partition pass of at most 8 bits up to 24-bit ids (buckets
    // of 2^16 vertices counted in two parts at 24 bits), two (buckets of 2^14) up to 27 bits
    const int vbits = bits_for((uint64_t)n);               // vertex ids fit in vbits bits
    const bool orient_part = vbits >= ORIENT_PART_MIN_BITS;
    uint32_t* p1_counts = nullptr;   // the orientation's first partition pass, counted by k_endpoints
    uint32_t p1_f = 1;
    // and the digit totals of its second pass, which with 8192-key tiles (2^26 pairs or more)
    // then looks back instead of running a histogram pass
    uint32_t* p2_tot =
        orient_part && radix_tile_keys((size_t)E, 8) == 8192u ? (uint32_t*)(ws + L.lb_aux) : nullptr;
    const int bw = vbits <= 20 ? (vbits < 12 ? vbits : 12) : (vbits <= 24 ? vbits - 8 : DEG_MAX_BW);
    const bool bucketed = vbits - bw <= DEG_MAX_BUCKET_BITS;
    {
        uint32_t* ep = (uint32_t*)keysA;       // 2E uint32 fit in E uint64
        uint32_t* ep_alt = (uint32_t*)keysB;
        // the endpoint sort's first digit is counted by k_endpoints as it writes the keys
        const uint32_t ep_tile = radix_tile_keys((size_t)(2 * E), 4);
        const uint32_t ep_tiles = (uint32_t)(((uint64_t)(2 * E) + ep_tile - 1) / ep_tile);
        const bool ep_sort = !bucketed || vbits > bw;
        const RadixDigit ep_dg = bucketed ? radix_first_digit(bw, vbits) : radix_first_digit(0, bits_for((uint64_t)n + 1));
        // past 2^21 vertices the orientation's first partition pass (pairs by the high bits
        // of the first id) takes its digit counts from here too, kept in the column array
        // until then; its tiles hold one or two endpoint tiles' pairs
        const uint32_t pt_pairs = radix_tile_keys((size_t)E, 8);
        const uint64_t pt_tiles = ((uint64_t)E + pt_pairs - 1) / pt_pairs;
        if (orient_part && pt_pairs % (ep_tile / 2) == 0 && pt_pairs / (ep_tile / 2) <= 2 &&
            256u * (pt_tiles + 1) <= (uint64_t)E) {   // the count table fits the column array
            p1_counts = col;
            p1_f = pt_pairs / (ep_tile / 2);
        }
        const uint32_t p1_tiles = (ep_tiles + p1_f - 1) / p1_f;
        const unsigned eg = p1_tiles < DEG_EP_BLOCKS ? p1_tiles : DEG_EP_BLOCKS;
        if (p2_tot) fill_u32(p2_tot, 0u, 256, s);
        hipLaunchKernelGGL(k_endpoints, dim3(eg), dim3(NT), 0, s, edges, (uint64_t)E, n,
                           bucketed ? (uint32_t)(n - 1) : (uint32_t)n, ep, ctrl, partial,
                           ep_sort ? radix_first_counts(radix_tmp) : nullptr, ep_tiles, ep_tile, ep_dg, p1_counts,
                           p1_f, RadixDigit{vbits - ORIENT_PART_BITS, (1u << ORIENT_PART_BITS) - 1u}, p2_tot);
        if (bucketed) {
            // partition by bits [bw, vbits), then count per bucket
            const uint32_t nb = 1u << (vbits - bw);
            int a0 = 0;
            if (vbits > bw)
                a0 = radix_sort_u32(ep, ep_alt, nullptr, nullptr, nullptr, (size_t)(2 * E), bw, vbits, radix_tmp, s,
                                    true, true, &ctrl->err);   // a grouping: the order inside a bucket is free
            uint32_t* bst = (uint32_t*)(ws + L.bstart);
            hipLaunchKernelGGL(k_bucket_starts, dim3(grid_for((size_t)nb + 1)), dim3(NT), 0, s, a0 ? ep_alt : ep,
                               (uint32_t)(2 * E), bw, nb, bst);
            uint32_t splits = 1;
            while (nb * splits < 256u && (uint64_t)splits * 65536u < (uint64_t)(2 * E) && splits < 64u) splits *= 2;
            if (splits > 1) fill_u32(deg, 0u, (size_t)n, s);
            launch_bucket_count(a0 ? ep_alt : ep, bst, bw, nb, splits, n, deg, s);
            hipLaunchKernelGGL(k_drop_sentinels, dim3(1), dim3(NT), 0, s, partial, eg, n, deg);
        } else {
            const int a0 = radix_sort_u32(ep, ep_alt, nullptr, nullptr, nullptr, (size_t)(2 * E), 0,
                                          bits_for((uint64_t)n + 1), radix_tmp, s, true, true,
                                          &ctrl->err);   // whole keys
            fill_u32(rowend, 0u, (size_t)n, s);
            hipLaunchKernelGGL(k_endpoint_bounds, dim3(grid_for((size_t)(2 * E))), dim3(NT), 0, s, a0 ? ep_alt : ep,
                               (uint64_t)(2 * E), n, rowend);
            fill_u32(deg, 0u, 1, s);
            scan_inclusive_max_u32(rowend, deg + 1, (size_t)n, scan_tmp, s);   // deg[] holds degree offsets
        }
    }
    mark(1);
    // ---- rank: sort (degree, id); degrees are below 2E + 1
    if (bucketed)
        hipLaunchKernelGGL(k_vertex_keys<false>, dim3(grid_for((size_t)n)), dim3(NT), 0, s, deg, n, vkeysA);
    else
        hipLaunchKernelGGL(k_vertex_keys<true>, dim3(grid_for((size_t)n)), dim3(NT), 0, s, deg, n, vkeysA);
    {
        const int dbits = bits_for((uint64_t)2 * (uint64_t)E + 1);
        const int alt = radix_sort_u64(vkeysA, vkeysB, nullptr, nullptr, nullptr, (size_t)n, 32, 32 + dbits,
                                       radix_tmp, s, false, false, &ctrl->err);
        hipLaunchKernelGGL(k_rank, dim3(grid_for((size_t)n)), dim3(NT), 0, s, alt ? vkeysB : vkeysA, n, rank, inv);
    }
    mark(2);
    // ---- orient
    const int nb = bits_for((uint64_t)n) > 0 ? bits_for((uint64_t)n) : 1;
    const uint64_t sentinel = (2 * nb >= 64) ? ~0ull : ((1ull << (2 * nb)) - 1ull);
    const uint32_t e_tile = radix_tile_keys((size_t)E, 8);
    const uint32_t e_tiles = (uint32_t)(((uint64_t)E + e_tile - 1) / e_tile);
    const bool part = orient_part;
    if (part) {
        // pairs by their first id's high bits, then by their second's (first id -> rank);
        // both passes only group the pairs for locality of the rank lookups
        const int ob = ORIENT_PART_BITS;
        radix_pass_u64((const uint64_t*)edges, keysB, (size_t)E, vbits - ob, ob, RadixXf{RX_NONE, nullptr, n, 0, 0},
                       radix_tmp, s, p1_counts, false);
        radix_pass_u64(keysB, keysA, (size_t)E, 32 + vbits - ob, ob, RadixXf{RX_RANK_LOW, rank, n, 0, 0}, radix_tmp,
                       s, nullptr, false, MoreTot{nullptr, 0, 0, 0, 0}, p2_tot, &ctrl->err);
    } else if (e_tile % (16 * NT) == 0)
        hipLaunchKernelGGL(k_orient<16>, dim3(e_tiles < 16384u ? e_tiles : 16384u), dim3(NT), 0, s, edges,
                           (uint64_t)E, n, rank, nb, sentinel, keysA, radix_first_counts(radix_tmp), e_tiles, e_tile,
                           radix_first_digit(nb, 2 * nb));
    else
        hipLaunchKernelGGL(k_orient<OR_U>, dim3(e_tiles < 16384u ? e_tiles : 16384u), dim3(NT), 0, s, edges,
                           (uint64_t)E, n, rank, nb, sentinel, keysA, radix_first_counts(radix_tmp), e_tiles, e_tile,
                           radix_first_digit(nb, 2 * nb));
    mark(3);
    // ---- sort oriented pairs: a radix sort on the lower rank (the row; its first
    // digit counted by k_orient or, past 2^21 vertices, taken by a first pass that
    // orients each pair as it loads it), then every row sorted on chip by the
    // higher rank. The row sort fixes the order inside a row, so the first pass
    // only partitions; the later ones are stable.
    int alt;
    if (part) {
        // the orienting pass's histogram also counts the digits of the passes after
        // it, so that those look back with no histogram pass of their own
        const int w0 = radix_digit_width(nb);
        const MoreTot rest = radix_sort_totals(radix_tmp, (size_t)E, 8, nb + w0, 2 * nb);
        radix_pass_u64(keysA, keysB, (size_t)E, nb, w0, RadixXf{RX_ORIENT, rank, n, nb, sentinel}, radix_tmp, s,
                       nullptr, false, rest);
        alt = 1 - radix_sort_u64(keysB, keysA, nullptr, nullptr, nullptr, (size_t)E, nb + w0, 2 * nb, radix_tmp, s,
                                 false, false, &ctrl->err, rest.n > 0);
    } else {
        alt = radix_sort_u64(keysA, keysB, nullptr, nullptr, nullptr, (size_t)E, nb, 2 * nb, radix_tmp, s, true,
                             true, &ctrl->err);
    }
    uint64_t* sorted = alt ? keysB : keysA;
    uint64_t* other = alt ? keysA : keysB;
    // the row sort also counts the kept (first of equal) keys per chunk of the unique pass
    const Chunking uc = chunking((uint64_t)E);
    fill_u32(partial, 0u, (size_t)uc.nblk + 1, s);
    sort_runs_u64(sorted, other, (size_t)E, nb, true, sentinel, partial, uc.chunk, s);
    mark(4);
    // ---- unique + CSR
    {
        const Chunking c = uc;
        scan_exclusive_sum_u32(partial, partial, (size_t)c.nblk + 1, scan_tmp, s);
        fill_u32(rowend, 0u, (size_t)n, s);
        hipLaunchKernelGGL(k_unique_write, dim3(c.nblk), dim3(NT), 0, s, sorted, (uint64_t)E, sentinel, ctrl, c.chunk,
                           partial, c.nblk, nb, col, src, rowend);
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
    const int nbv = bits_for((uint64_t)n);
    uint64_t* csc;
    const uint32_t* moff = off;   // offsets of the middle lists
    if (r.formulation == FORM_FILTERED) {
        // ---- CSC: in-edges with work grouped by v (the sorted pair keys are free now);
        // in-edge groups: ids 0 .. n - 1 (n - 1 = no work). Each in-edge carries its
        // own edge index and tail, so the order inside a group is free: the
        // sort's first pass only partitions.
        const CscPacking pk = csc_packing(E, n);
        hipLaunchKernelGGL(k_csc_keys, dim3(e_tiles < 16384u ? e_tiles : 16384u), dim3(NT), 0, s, col, src, off,
                           ctrl, n, other, pk.sh, pk.lbits, radix_first_counts(radix_tmp), e_tiles, e_tile,
                           radix_first_digit(pk.sh, pk.sh + nbv));
        const int alt2 = radix_sort_u64(other, sorted, nullptr, nullptr, &ctrl->m, (size_t)E, pk.sh, pk.sh + nbv,
                                        radix_tmp, s, true, true, &ctrl->err);
        // bounds and tail ranges in one pass, into the buffer the sort left free
        const uint64_t* ckeys = alt2 ? sorted : other;
        csc = alt2 ? other : sorted;
        fill_u32(rowend, 0u, (size_t)n, s);
        hipLaunchKernelGGL(k_csc_finish, dim3(grid_for(((size_t)E + 1) / 2)), dim3(NT), 0, s, ckeys,
                           csc, ctrl, n, rowend, pk.sh, src, off, pk.ebits, pk.lbits);
        fill_u32(inoff, 0u, 1, s);
        scan_inclusive_max_u32(rowend, inoff + 1, (size_t)n, scan_tmp, s);
    } else {
        // ---- all in-edges grouped by v; the symmetric adjacency; the streamed ranges
        const int sh = bits_for((uint64_t)E) > 0 ? bits_for((uint64_t)E) : 1;
        hipLaunchKernelGGL(k_sym_keys, dim3(grid_for((size_t)E)), dim3(NT), 0, s, col, ctrl, other, sh);
        const int alt2 =
            radix_sort_u64(other, sorted, nullptr, nullptr, &ctrl->m, (size_t)E, sh, sh + nbv, radix_tmp, s, false,
                           false, &ctrl->err);
        csc = alt2 ? sorted : other;
        fill_u32(rowend, 0u, (size_t)n, s);
        hipLaunchKernelGGL(k_sym_bounds, dim3(grid_for((size_t)E)), dim3(NT), 0, s, csc, ctrl, rowend, sh);
        fill_u32(inoff, 0u, 1, s);
        scan_inclusive_max_u32(rowend, inoff + 1, (size_t)n, scan_tmp, s);
        uint32_t* fo = sym_off(r, L);
        if (r.formulation != FORM_MATRIX_UPPER) {
            hipLaunchKernelGGL(k_sym_rows, dim3(grid_for((size_t)n + 1)), dim3(NT), 0, s, inoff, off, n, fo);
            moff = fo;
        }
        hipLaunchKernelGGL(k_sym_build, dim3(grid_for((size_t)E)), dim3(NT), 0, s, csc, ctrl, src, col, off, inoff,
                           sym_col(r, L), sh, r.formulation);
    }
    mark(6);
    // ---- buckets + selection
    const uint32_t* mcol = (r.formulation == FORM_FULL || r.formulation == FORM_MATRIX) ? sym_col(r, L) : col;
    hipLaunchKernelGGL(k_vbucket, dim3(grid_for((size_t)n, 2048)), dim3(NT), 0, s, moff, mcol, inoff, n, vbucket,
                       ctrl);
    const bool learned = !r.given && r.select == SEL_LEARNED && r.mlp && r.learned;
    const bool learned_tile = learned && r.mlp_tile && r.learned_tile;
    if (learned) mlp_select((const MlpCompute*)r.mlp, ctrl, r.learned, s);
    else bucket_features_launch(ctrl, s);
    if (learned_tile) mlp_select((const MlpCompute*)r.mlp_tile, ctrl, r.learned_tile, s);
    hipLaunchKernelGGL(k_select, dim3(1), dim3(NBUCKET), 0, s, ctrl, r.given ? (int)SEL_LEARNED : r.select,
                       r.given ? r.given : (learned ? r.learned : nullptr), learned_tile ? r.learned_tile : nullptr,
                       r.chunk_override, r.group_override, r.formulation != FORM_FILTERED ? 1 : 0);
    mark(7);
    // ---- group: order vertices by (kernel, bucket); tiles
    hipLaunchKernelGGL(k_vkeys_slot, dim3(grid_for((size_t)n)), dim3(NT), 0, s, vbucket, n, ctrl, vkeysA);
    {
        const int a3 = radix_sort_u64(vkeysA, vkeysB, nullptr, nullptr, nullptr, (size_t)n, 32, 40, radix_tmp, s,
                                      false, false, &ctrl->err);
        hipLaunchKernelGGL(k_vpos, dim3(grid_for((size_t)n)), dim3(NT), 0, s, a3 ? vkeysB : vkeysA, n, vbucket, ctrl,
                           vlist);
    }
    hipLaunchKernelGGL(k_ntiles, dim3(grid_for((size_t)n)), dim3(NT), 0, s, vlist, vbucket, inoff, n, ctrl, tstart);
    scan_exclusive_sum_u32(tstart, tstart, (size_t)n + 1, scan_tmp, s);
    hipLaunchKernelGGL(k_emit_tiles, dim3(grid_for((size_t)n)), dim3(NT), 0, s, vlist, vbucket, inoff, tstart, n,
                       ctrl, tiles, (uint64_t)L.tile_cap);
    if (r.per_edge_counts) fill_u32(r.per_edge_counts, 0u, (size_t)E, s);
    if (r.support) fill_u32(r.support, 0u, (size_t)E, s);
    if (r.per_vertex || r.per_middle || r.clustering) fill_u64(pv, 0ull, (size_t)n, s);
    mark(8);
    if (r.stop_before_isect) {
        out->ctrl_dev = ctrl;
        return hipGetLastError();
    }
    // ---- intersections
    const IsectArgs ia = isect_args(r, L, csc);
    uint64_t* partials = (uint64_t*)(ws + L.isect_partials);
    const int order[NKERNEL] = {KER_MERGE, KER_BSEARCH, KER_BITMAP};
    for (int q = 0; q < NKERNEL; ++q) {
        const int k = order[q];
        launch_isect(k, ia, r.grid_override ? r.grid_override[k] : 0, partials, s);
        mark(9 + q);
    }
    launch_reduce_total(partials, ctrl, s);
    // ---- finish
    if (r.per_vertex)
        hipLaunchKernelGGL(k_map_pv, dim3(grid_for((size_t)n)), dim3(NT), 0, s, pv, inv, n, r.per_vertex);
    else if (r.per_middle)
        hipLaunchKernelGGL(k_map_pv, dim3(grid_for((size_t)n)), dim3(NT), 0, s, pv, inv, n, r.per_middle);
    if (r.clustering) {   // the degree offsets are dead by now: reuse them for the simple in-degree
        fill_u32(deg, 0u, (size_t)n, s);
        hipLaunchKernelGGL(k_indeg, dim3(grid_for((size_t)E)), dim3(NT), 0, s, col, ctrl, deg);
        const unsigned g = grid_for((size_t)n, CL_MAX_BLOCKS);
        hipLaunchKernelGGL(k_clustering, dim3(g), dim3(NT), 0, s, pv, inv, off, deg, n, r.clustering, partials);
        hipLaunchKernelGGL(k_sum_wedges, dim3(1), dim3(NT), 0, s, partials, g, ctrl);
    }
    if (r.per_edge_pairs)
        hipLaunchKernelGGL(k_map_edges, dim3(grid_for((size_t)E)), dim3(NT), 0, s, col, src, inv, ctrl,
                           (int2*)r.per_edge_pairs);
    mark(NSTAGE);
    out->ctrl_dev = ctrl;
    return hipGetLastError();
}

}  // namespace tcx
