// Device primitives: fills, three-phase scans and an LSD radix sort of 64-bit keys.
//
// The radix sort is the CSR builder of the method's "induced subgraph" step
// (Section 4.2, optimisations for edge list generation): edges are sorted
// by (source, destination) so every row of the filtered graph is contiguous
// and ascending. Keys are sorted in ceil(bits / 8) passes of equal digit
// widths; a pass is a per-tile digit histogram, an exclusive scan of the
// digit-major histogram, and a stable scatter that ranks equal digits inside
// each wave with ballots.
#include "common.h"
#include "internal.h"

namespace tcx {

// ------------------------------------------------------------------ fills
template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* p, T v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = v;
}

static unsigned grid_for(size_t n, unsigned cap = 8192) {
    size_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
}
void fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_fill<uint64_t>, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
}

// ------------------------------------------------------------------ scans
// Three phases over a fixed number of blocks: per-block reduction, a scan of
// the block partials in one block, then each block scans its chunk with its
// partial as the carry-in. Works in place (out == in).
constexpr int SCAN_NT = 256;
constexpr int SCAN_MAX_BLOCKS = 1024;
constexpr int SCAN_ITEMS = 8;   // elements per thread per step

struct OpSum {
    template <typename T> __device__ static T apply(T a, T b) { return a + b; }
    template <typename T> __device__ static T ident() { return T(0); }
};
struct OpMax {
    template <typename T> __device__ static T apply(T a, T b) { return a > b ? a : b; }
    template <typename T> __device__ static T ident() { return T(0); }
};

template <typename Op, typename T>
__device__ T block_reduce(T v, T* scratch) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v = Op::apply(v, (T)__shfl_xor(v, o, WAVE));
    if (lane_id() == 0) scratch[wave_id()] = v;
    __syncthreads();
    T r = Op::template ident<T>();
    for (int i = 0; i < SCAN_NT / WAVE; ++i) r = Op::apply(r, scratch[i]);
    __syncthreads();
    return r;
}

template <typename Op, typename T>
__device__ T block_scan_inclusive(T v, T* scratch, T* total) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const T t = (T)__shfl_up(v, o, WAVE);
        if (l >= o) v = Op::apply(v, t);
    }
    if (l == WAVE - 1) scratch[wave_id()] = v;
    __syncthreads();
    T base = Op::template ident<T>(), all = Op::template ident<T>();
    for (int i = 0; i < SCAN_NT / WAVE; ++i) {
        if (i < wave_id()) base = Op::apply(base, scratch[i]);
        all = Op::apply(all, scratch[i]);
    }
    __syncthreads();
    *total = all;
    return Op::apply(base, v);
}

template <typename Op, typename T>
__global__ __launch_bounds__(SCAN_NT) void k_scan_reduce(const T* in, size_t len, size_t chunk, T* partial) {
    __shared__ T scratch[SCAN_NT / WAVE];
    const size_t b0 = (size_t)blockIdx.x * chunk;
    const size_t b1 = b0 + chunk < len ? b0 + chunk : len;
    T acc = Op::template ident<T>();
    for (size_t base = b0; base < b1; base += (size_t)SCAN_NT * SCAN_ITEMS) {
        T v[SCAN_ITEMS];
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {   // loads in flight together
            const size_t i = base + (size_t)k * SCAN_NT + threadIdx.x;
            v[k] = i < b1 ? in[i] : Op::template ident<T>();
        }
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) acc = Op::apply(acc, v[k]);
    }
    acc = block_reduce<Op>(acc, scratch);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// Exclusive scan of up to SCAN_MAX_BLOCKS partials in one block; partial[nb] = total.
template <typename Op, typename T>
__global__ __launch_bounds__(SCAN_NT) void k_scan_partials(T* partial, int nb) {
    __shared__ T scratch[SCAN_NT / WAVE];
    constexpr int PER = SCAN_MAX_BLOCKS / SCAN_NT;
    T v[PER];
    T local = Op::template ident<T>();
    for (int k = 0; k < PER; ++k) {
        const int i = threadIdx.x * PER + k;
        v[k] = i < nb ? partial[i] : Op::template ident<T>();
        local = Op::apply(local, v[k]);
    }
    T total;
    T inc = block_scan_inclusive<Op>(local, scratch, &total);
    // exclusive base for this thread = inclusive of previous thread
    T prev = (T)__shfl_up(inc, 1, WAVE);
    __shared__ T wave_last[SCAN_NT / WAVE];
    if (lane_id() == WAVE - 1) wave_last[wave_id()] = inc;
    __syncthreads();
    if (lane_id() == 0) prev = wave_id() == 0 ? Op::template ident<T>() : wave_last[wave_id() - 1];
    T run = prev;
    for (int k = 0; k < PER; ++k) {
        const int i = threadIdx.x * PER + k;
        if (i < nb) partial[i] = run;
        run = Op::apply(run, v[k]);
    }
    if (threadIdx.x == 0) partial[nb] = total;
}

template <typename Op, typename T, bool INCLUSIVE>
__global__ __launch_bounds__(SCAN_NT) void k_scan_down(const T* in, T* out, size_t len, size_t chunk,
                                                       const T* partial) {
    __shared__ T scratch[SCAN_NT / WAVE];
    const size_t b0 = (size_t)blockIdx.x * chunk;
    const size_t b1 = b0 + chunk < len ? b0 + chunk : len;
    T carry = partial[blockIdx.x];
    // SCAN_ITEMS consecutive elements per thread: loaded together, scanned in
    // registers, then one block scan of the thread totals per SCAN_NT * SCAN_ITEMS
    for (size_t base = b0; base < b1; base += (size_t)SCAN_NT * SCAN_ITEMS) {
        const size_t i0 = base + (size_t)threadIdx.x * SCAN_ITEMS;
        T v[SCAN_ITEMS];
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) v[k] = i0 + k < b1 ? in[i0 + k] : Op::template ident<T>();
        T run = Op::template ident<T>();
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) run = Op::apply(run, v[k]);
        T total;
        const T inc = block_scan_inclusive<Op>(run, scratch, &total);
        // exclusive prefix of this thread's run within the block step
        T acc;
        {
            const T prev_inc = (T)__shfl_up(inc, 1, WAVE);
            __shared__ T wave_last[SCAN_NT / WAVE];
            if (lane_id() == WAVE - 1) wave_last[wave_id()] = inc;
            __syncthreads();
            T before = Op::template ident<T>();
            if (lane_id() != 0) before = prev_inc;
            else if (wave_id() != 0) before = wave_last[wave_id() - 1];
            __syncthreads();
            acc = Op::apply(carry, before);
        }
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            if (i0 + k < b1) {
                const T nxt = Op::apply(acc, v[k]);
                out[i0 + k] = INCLUSIVE ? nxt : acc;
                acc = nxt;
            }
        }
        carry = Op::apply(carry, total);
    }
}

size_t scan_temp_bytes() { return sizeof(uint64_t) * (SCAN_MAX_BLOCKS + 1); }

template <typename Op, typename T, bool INCLUSIVE>
static void scan_impl(const T* in, T* out, size_t len, void* temp, hipStream_t s) {
    if (len == 0) return;
    int nb = (int)((len + 8191) / 8192);
    if (nb > SCAN_MAX_BLOCKS) nb = SCAN_MAX_BLOCKS;
    if (nb < 1) nb = 1;
    size_t chunk = (len + nb - 1) / nb;
    chunk = (chunk + SCAN_NT - 1) / SCAN_NT * SCAN_NT;
    nb = (int)((len + chunk - 1) / chunk);
    T* partial = (T*)temp;
    hipLaunchKernelGGL((k_scan_reduce<Op, T>), dim3(nb), dim3(SCAN_NT), 0, s, in, len, chunk, partial);
    hipLaunchKernelGGL((k_scan_partials<Op, T>), dim3(1), dim3(SCAN_NT), 0, s, partial, nb);
    hipLaunchKernelGGL((k_scan_down<Op, T, INCLUSIVE>), dim3(nb), dim3(SCAN_NT), 0, s, in, out, len, chunk,
                       (const T*)partial);
}

void scan_exclusive_sum_u32(const uint32_t* in, uint32_t* out, size_t len, void* temp, hipStream_t s) {
    scan_impl<OpSum, uint32_t, false>(in, out, len, temp, s);
}
void scan_inclusive_max_u32(const uint32_t* in, uint32_t* out, size_t len, void* temp, hipStream_t s) {
    scan_impl<OpMax, uint32_t, true>(in, out, len, temp, s);
}
void scan_exclusive_sum_u64(const uint64_t* in, uint64_t* out, size_t len, void* temp, hipStream_t s) {
    scan_impl<OpSum, uint64_t, false>(in, out, len, temp, s);
}

// ------------------------------------------------------------------ radix sort
// A tile is RS_NT threads x ITEMS keys: 16 keys per lane (4096-key tiles, longer
// runs of equal digits for the scatter, half the count table) for sorts of at
// least 2^22 keys, 8 (2048-key tiles, twice the blocks) below, and 32 for sorts
// of at least 2^26 keys (8192-key tiles: the scatter's runs of a uniform digit
// grow from 16 to 32 keys; its blocks run 512 threads of 16 keys, so they keep
// four waves per SIMD). For the 32-bit endpoint partition of R-MAT 24 (2^29 keys)
// the 8192-key tiles took the degree stage from 4.00 to 3.79 ms; with 256
// threads of 32 keys they had lost (two waves per SIMD).
constexpr int RS_NT = 256;
constexpr int RS_WAVES = RS_NT / WAVE;
constexpr int RS_ITEMS_SMALL = 8, RS_ITEMS_LARGE = 16, RS_ITEMS_HUGE = 32;
constexpr size_t RS_LARGE_CAP = (size_t)1 << 22, RS_HUGE_CAP = (size_t)1 << 26;

uint32_t radix_tile_keys(size_t cap, int key_bytes) {
    const int items = cap >= RS_HUGE_CAP ? RS_ITEMS_HUGE
                      : cap >= RS_LARGE_CAP                ? RS_ITEMS_LARGE
                                                           : RS_ITEMS_SMALL;
    return (uint32_t)(RS_NT * items);
}

__device__ __forceinline__ uint32_t rs_count(const uint32_t* d_count, uint32_t cap) {
    const uint32_t c = d_count ? *d_count : cap;
    return c < cap ? c : cap;
}

// Keys move unchanged.
struct XfIdentity {
    template <typename KeyT>
    __device__ __forceinline__ KeyT operator()(KeyT k) const { return k; }
};
// 64-bit keys whose low 32 bits are a vertex id: the id is replaced by its rank
// (ids outside [0, n): 0xFFFFFFFF) as the key moves; the high half, which holds
// the digit of the pass, is unchanged.
struct XfRankLow {
    const uint32_t* rank;
    int32_t n;   // >= 1: an id out of range reads rank[0] and discards it (no branch around the gather)
    __device__ __forceinline__ uint64_t operator()(uint64_t k) const {
        const int32_t a = (int32_t)(uint32_t)k;
        const bool ok = a >= 0 && a < n;
        const uint32_t r = rank[ok ? a : 0];
        return (k & 0xFFFFFFFF00000000ull) | (ok ? r : 0xFFFFFFFFu);
    }
};

// (b << 32 | rank of a) -> the oriented pair key (min rank << nb | max rank),
// or the sentinel (an invalid id, or a loop: equal ranks). The rank of b is
// looked up here; the pass before left the keys grouped by b's high bits.
struct XfOrient {
    const uint32_t* rank;
    int32_t n;
    int nb;
    uint64_t sentinel;
    __device__ __forceinline__ uint64_t operator()(uint64_t k) const {
        const int32_t b = (int32_t)(uint32_t)(k >> 32);
        const uint32_t ra = (uint32_t)k;
        const bool okb = b >= 0 && b < n;
        const uint32_t rb = rank[okb ? b : 0];
        const bool good = okb && ra != 0xFFFFFFFFu && ra != rb;
        const uint32_t lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
        return good ? (((uint64_t)lo << nb) | hi) : sentinel;
    }
};

// Global digit counts for the passes of a sort that look back (no histogram
// pass of their own; MoreTot): a kernel that reads every key anyway (the
// sort's first pass, or an earlier pass's histogram) adds them. The counts go
// to LDS counters cnt[(q * 256 + d) * copies + c], lane l adding to copy
// c = l % copies: the later digits of rank keys are skewed (the hubs' ranks),
// and the copies, in different banks, split the lanes of a wave that share a
// digit over several addresses.
__device__ __forceinline__ void more_add(uint32_t* cnt, int copies, const MoreTot& more, uint64_t key) {
    const uint32_t c = (uint32_t)lane_id() & (uint32_t)(copies - 1);
    for (int q = 0; q < more.n; ++q) {
        const int sh = more.shift + q * more.bits;
        const int wb = more.hi - sh < more.bits ? more.hi - sh : more.bits;
        const uint32_t d = (uint32_t)(key >> sh) & ((1u << wb) - 1u);
        atomicAdd(&cnt[(q * 256 + d) * copies + c], 1u);
    }
}
__device__ __forceinline__ void more_flush(const uint32_t* cnt, int copies, const MoreTot& more) {
    for (int i = threadIdx.x; i < more.n * 256; i += blockDim.x) {
        uint32_t t = 0;
        for (int c = 0; c < copies; ++c) t += cnt[i * copies + c];
        if (t) atomicAdd(&more.tot[i], t);
    }
}

// Per-tile digit counts, written digit-major: hist[d * ntiles + tile]; digits of
// the keys as xf transforms them.
// TOT: also the global counts of a later sort's digits (MoreTot), in four
// copies of LDS counters.
template <typename KeyT, int RS_ITEMS, typename XF = XfIdentity, bool TOT = false>
__global__ __launch_bounds__(RS_NT) void k_radix_hist(const KeyT* __restrict__ keys, const uint32_t* d_count,
                                                      uint32_t cap, int shift, uint32_t dmask,
                                                      uint32_t* __restrict__ hist,
                                                      uint32_t ntiles, XF xf = XF(),
                                                      MoreTot more = MoreTot{nullptr, 0, 0, 0, 0}) {
    constexpr int RS_TILE = RS_NT * RS_ITEMS, RS_WAVE_SPAN = WAVE * RS_ITEMS;   // keys per tile / per wave
    constexpr int COPIES = 4;
    __shared__ uint32_t wcnt[RS_WAVES][256];
    __shared__ uint32_t mcnt[TOT ? LB_MAX_MORE * 256 * COPIES : 1];
    for (int i = threadIdx.x; i < RS_WAVES * 256; i += RS_NT) (&wcnt[0][0])[i] = 0;
    if (TOT)
        for (int i = threadIdx.x; i < more.n * 256 * COPIES; i += RS_NT) mcnt[i] = 0;
    __syncthreads();
    const uint32_t n = rs_count(d_count, cap);
    const int w = wave_id(), l = lane_id();
    const uint32_t base = blockIdx.x * RS_TILE + w * RS_WAVE_SPAN;
    uint32_t dg[RS_ITEMS];
    KeyT kk[RS_ITEMS];
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const uint32_t i = base + it * WAVE + l;
        kk[it] = i < n ? keys[i] : KeyT(0);
    }
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {   // every lane transforms (no branch around the gathers)
        const uint32_t i = base + it * WAVE + l;
        const KeyT t = xf(kk[it]);
        const uint32_t dd = (uint32_t)(t >> shift) & dmask;
        dg[it] = i < n ? dd : 0u;
        if (TOT && i < n) more_add(mcnt, COPIES, more, (uint64_t)t);
    }
    // counts only (no ranks): one LDS add per key into the wave's histogram, none
    // waited on. A wave whose valid keys all share one digit (sorted stretches:
    // 64-bit keys here hold degree ranks, whose top digit the hubs' in-edges
    // dominate, and a 32-bit histogram runs for the second partition pass of
    // wide vertex ids, whose keys the first pass grouped by their top bits)
    // adds its count once from lane 0 instead of 64 adds on one counter. The
    // test is uniform (valid lanes are a prefix of the wave), so it costs a few
    // scalar operations per key, not a leader search.
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const uint64_t act = __ballot(base + it * WAVE + l < n);
        const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)dg[it]);
        const uint64_t same = __ballot(dg[it] == d0) & act;
        if (same == act) {
            if (l == 0 && act) atomicAdd(&wcnt[w][d0], (uint32_t)__popcll(act));
        } else if ((act >> l) & 1u) {
            atomicAdd(&wcnt[w][dg[it]], 1u);
        }
    }
    __syncthreads();
    const int d = threadIdx.x;
    uint32_t t = 0;
#pragma unroll
    for (int k = 0; k < RS_WAVES; ++k) t += wcnt[k][d];
    hist[(size_t)d * ntiles + blockIdx.x] = t;
    if (TOT) more_flush(mcnt, COPIES, more);
}

// Block (d, s): exclusive scan, in place, of segment s (RS_ROW_SEG tile counts)
// of digit d's row hist[d * ntiles .. +ntiles). With one segment per row the
// row total goes to digit_tot[d]; otherwise the segment total goes to
// seg_tot[d * nseg + s] and k_radix_rowfix adds the carries.
constexpr int RS_ROW_ITEMS = 8;
constexpr uint32_t RS_ROW_SEG = 4 * RS_NT * RS_ROW_ITEMS;   // 8192 tile counts per segment
__global__ __launch_bounds__(RS_NT) void k_radix_rowscan(uint32_t* __restrict__ hist, uint32_t ntiles,
                                                         uint32_t* __restrict__ digit_tot,
                                                         uint32_t* __restrict__ seg_tot) {
    __shared__ uint32_t scratch[RS_WAVES];
    uint32_t* row = hist + (size_t)blockIdx.x * ntiles;
    const uint32_t s0 = blockIdx.y * RS_ROW_SEG;
    const uint32_t s1 = s0 + RS_ROW_SEG < ntiles ? s0 + RS_ROW_SEG : ntiles;
    uint32_t carry = 0;
    for (uint32_t base = s0; base < s1; base += RS_NT * RS_ROW_ITEMS) {
        const uint32_t i0 = base + threadIdx.x * RS_ROW_ITEMS;
        uint32_t v[RS_ROW_ITEMS], sum = 0;
#pragma unroll
        for (int k = 0; k < RS_ROW_ITEMS; ++k) {
            v[k] = i0 + k < s1 ? row[i0 + k] : 0u;
            sum += v[k];
        }
        uint32_t total;
        uint32_t run = carry + block_exclusive_scan<RS_NT>(sum, scratch, &total);
#pragma unroll
        for (int k = 0; k < RS_ROW_ITEMS; ++k) {
            if (i0 + k < s1) row[i0 + k] = run;
            run += v[k];
        }
        carry += total;
    }
    if (threadIdx.x == 0) {
        if (gridDim.y == 1) digit_tot[blockIdx.x] = carry;
        else seg_tot[blockIdx.x * gridDim.y + blockIdx.y] = carry;
    }
}

// Block (d, s): adds the totals of segments 0..s-1 to segment s; the last
// segment's block also writes the row total.
__global__ __launch_bounds__(RS_NT) void k_radix_rowfix(uint32_t* __restrict__ hist, uint32_t ntiles,
                                                        const uint32_t* __restrict__ seg_tot,
                                                        uint32_t* __restrict__ digit_tot) {
    const uint32_t d = blockIdx.x, sg = blockIdx.y, nseg = gridDim.y;
    uint32_t carry = 0;
    for (uint32_t q = 0; q < sg; ++q) carry += seg_tot[d * nseg + q];
    if (sg == nseg - 1 && threadIdx.x == 0) digit_tot[d] = carry + seg_tot[d * nseg + sg];
    if (sg == 0 || carry == 0) return;
    uint32_t* row = hist + (size_t)d * ntiles;
    const uint32_t s0 = sg * RS_ROW_SEG;
    const uint32_t s1 = s0 + RS_ROW_SEG < ntiles ? s0 + RS_ROW_SEG : ntiles;
    for (uint32_t i = s0 + threadIdx.x; i < s1; i += RS_NT) row[i] += carry;
}

// NT_ threads of RS_ITEMS keys each: 8192-key tiles run 512 threads of 16 keys
// (half the registers per lane of 256 x 32, twice the waves per CU); threads
// 0..255 own the digits in the per-digit scans. Each key passes through xf as it
// is loaded (the transform must leave the digit of the pass unchanged).
// RANK says how a key gets its rank among the wave's keys of its digit:
//   RANK_MATCH   stable: the lanes of equal digit found by 8 ballots (VALU);
//   RANK_MASK    stable: each lane sets its bit in a 64-bit LDS mask of its
//                digit, reads the mask back and the lowest lane clears it; the
//                LDS applies one wave's instructions in order, so the read sees
//                exactly this instruction's lanes of that digit (few VALU
//                operations, one LDS round trip per key);
//   RANK_ATOMIC  the order inside a digit is whatever the LDS adds give, and
//                the pass only partitions: for a pass whose later users never
//                look at that order (the first pass of an LSD sort whose
//                equal-key order is free, a grouping). One add per key, all of
//                a thread's adds in flight together.
// The masks use the key tile's LDS, free until the ranks are known.
enum { RANK_MATCH = 0, RANK_MASK = 1, RANK_ATOMIC = 2 };

template <typename KeyT, bool HAS_VAL, int RS_ITEMS, int NT_ = RS_NT, typename XF = XfIdentity, int RANK = RANK_MATCH,
          bool TOT = false>
__global__ __launch_bounds__(NT_) void k_radix_scatter(const KeyT* __restrict__ kin,
                                                         const uint32_t* __restrict__ vin,
                                                         KeyT* __restrict__ kout, uint32_t* __restrict__ vout,
                                                         const uint32_t* d_count, uint32_t cap, int shift,
                                                         uint32_t dmask,
                                                         const uint32_t* __restrict__ hist_scan, uint32_t ntiles,
                                                         const uint32_t* __restrict__ digit_tot, XF xf,
                                                         MoreTot more = MoreTot{nullptr, 0, 0, 0, 0}) {
    constexpr int NW = NT_ / WAVE;
    constexpr int RS_TILE = NT_ * RS_ITEMS, RS_WAVE_SPAN = WAVE * RS_ITEMS;
    static_assert(NT_ >= 256, "a thread per digit");
    __shared__ uint32_t wcnt[NW][256];
    __shared__ uint32_t gofs[256];
    __shared__ uint32_t scratch[NW];
    __shared__ __align__(16) KeyT skey[RS_TILE];
    __shared__ uint32_t sval[HAS_VAL ? RS_TILE : 1];
    constexpr bool MASK_IN_TILE = sizeof(KeyT) * RS_TILE >= sizeof(uint64_t) * 256 * NW;
    __shared__ uint64_t mask_own[RANK == RANK_MASK && !MASK_IN_TILE ? NW : 1][RANK == RANK_MASK ? 256 : 1];
    uint64_t (*wmask)[256] = MASK_IN_TILE ? reinterpret_cast<uint64_t (*)[256]>(skey)
                                          : reinterpret_cast<uint64_t (*)[256]>(mask_own);
    for (int i = threadIdx.x; i < NW * 256; i += NT_) {
        (&wcnt[0][0])[i] = 0;
        if (RANK == RANK_MASK) (&wmask[0][0])[i] = 0ull;
    }
    __syncthreads();
    const uint32_t n = rs_count(d_count, cap);
    const int w = wave_id(), l = lane_id();
    const uint32_t tile0 = blockIdx.x * RS_TILE;
    const uint32_t base = tile0 + w * RS_WAVE_SPAN;
    KeyT k[RS_ITEMS];
    uint32_t v[RS_ITEMS];
    uint32_t loc[RS_ITEMS];   // digit | (rank within (wave, digit)) << 8
    // all loads first, so that they are in flight together (the ranking below
    // has wave barriers that no load may cross)
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const uint32_t i = base + it * WAVE + l;
        k[it] = i < n ? kin[i] : KeyT(0);
        if (HAS_VAL) v[it] = i < n ? vin[i] : 0u;
    }
    // every lane transforms, lanes past the end their zero key, so that no branch
    // separates the gathers of a transform: all of them are in flight together
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const uint64_t t = xf(k[it]);
        k[it] = base + it * WAVE + l < n ? t : k[it];
    }
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const uint32_t i = base + it * WAVE + l;
        const bool valid = i < n;
        const uint32_t d = (uint32_t)(k[it] >> shift) & dmask;
        if (RANK != RANK_ATOMIC) {
            uint64_t peers;
            if (RANK == RANK_MATCH) {
                peers = match_digit8(d, __ballot(valid));
            } else {
                if (valid) atomicOr((unsigned long long*)&wmask[w][d], 1ull << l);
                __builtin_amdgcn_wave_barrier();
                peers = valid ? wmask[w][d] : 0ull;
                __builtin_amdgcn_wave_barrier();
            }
            const uint32_t r = (uint32_t)__popcll(peers & lanes_below());
            const uint32_t prev = wcnt[w][d];
            __builtin_amdgcn_wave_barrier();
            if (valid && r == 0) {
                wcnt[w][d] = prev + (uint32_t)__popcll(peers);
                if (RANK == RANK_MASK) wmask[w][d] = 0ull;
            }
            __builtin_amdgcn_wave_barrier();
            loc[it] = d | ((prev + r) << 8);
        } else {
            // one LDS atomic per key, none waited on before the next key's: the
            // ranks of one digit are the counter's successive values in whatever
            // order the LDS applies the adds (equal digits in one wave serialise
            // there, at worst 64 adds on one address per instruction)
            // (lanes past the end add 0 to digit 0's counter: no branch, so no
            // wait between the atomics)
            const uint32_t r = atomicAdd(&wcnt[w][valid ? d : 0u], valid ? 1u : 0u);
            loc[it] = d | (r << 8);
        }
    }
    __syncthreads();
    {
        // wcnt[q][d] becomes the tile position of wave q's first key of digit d,
        // gofs[d] the output position of the tile's first key of digit d minus
        // its tile position: one LDS lookup per key in each phase below
        const bool own = threadIdx.x < 256;   // threads past the digits add zeros to the scans
        const int d = own ? (int)threadIdx.x : 0;
        uint32_t run = 0;
        if (own) {
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                const uint32_t c = wcnt[q][d];
                wcnt[q][d] = run;
                run += c;
            }
        }
        const uint32_t excl = block_exclusive_scan<NT_>(run, scratch);
        // digit base = keys with a smaller digit; plus this tile's offset in its digit row
        const uint32_t dbase = block_exclusive_scan<NT_>(own ? digit_tot[d] : 0u, scratch);
        if (own) {
#pragma unroll
            for (int q = 0; q < NW; ++q) wcnt[q][d] += excl;
            gofs[d] = dbase + hist_scan[(size_t)d * ntiles + blockIdx.x] - excl;
        }
    }
    __syncthreads();
    {
        uint32_t pb[RS_ITEMS];   // all lookups in flight before the first write
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it) pb[it] = wcnt[w][loc[it] & 255u];
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it) {
            if (base + it * WAVE + l < n) {
                const uint32_t p = pb[it] + (loc[it] >> 8);
                skey[p] = k[it];
                if (HAS_VAL) sval[p] = v[it];
            }
        }
    }
    __syncthreads();
    // TOT: the later digits are counted in wcnt, free once the keys sit in LDS,
    // in as many copies as fit
    static_assert(!TOT || NW * 256 >= LB_MAX_MORE * 256 * 2, "two copies of the counts fit the wave counters");
    const int copies = !TOT ? 1 : more.n <= 1 ? 8 : more.n == 2 ? 4 : 2;
    if (TOT) {
        for (int i = threadIdx.x; i < NW * 256; i += NT_) (&wcnt[0][0])[i] = 0;
        __syncthreads();
    }
    const uint32_t tile_n = n > tile0 ? (n - tile0 < (uint32_t)RS_TILE ? n - tile0 : (uint32_t)RS_TILE) : 0u;
    {
        // thread t writes tile positions t, t + NT_, ...: consecutive threads,
        // consecutive positions, so each digit's run goes out coalesced
        KeyT key[RS_ITEMS];
        uint32_t go[RS_ITEMS];
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it) key[it] = skey[it * NT_ + threadIdx.x];   // in the tile's LDS
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it) go[it] = gofs[(uint32_t)(key[it] >> shift) & dmask];
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it) {
            const uint32_t j = it * NT_ + threadIdx.x;
            const uint32_t pos = go[it] + j;
            if (j < tile_n && pos < n) {   // pos < n: always, when the histogram scan is consistent
                kout[pos] = key[it];
                if (HAS_VAL) vout[pos] = sval[j];
            }
        }
        if (TOT) {
#pragma unroll
            for (int it = 0; it < RS_ITEMS; ++it)
                if (it * NT_ + threadIdx.x < tile_n) more_add(&wcnt[0][0], copies, more, (uint64_t)key[it]);
        }
    }
    if (TOT) {
        __syncthreads();
        more_flush(&wcnt[0][0], copies, more);
    }
}

// A later pass of a large sort in one kernel: the per-tile digit offsets come
// from the tiles before it (decoupled look-back) instead of a count table
// built by a histogram pass. Tiles are taken in order from a counter, so a
// tile only ever waits for tiles that a running block holds. Each tile
// publishes, per digit, its count (flag 1) as soon as it has ranked its keys,
// then walks back over the tiles before it, adding counts until it meets a
// running total (flag 2), and publishes its own running total. status holds one
// 64-bit word per (tile, digit), zeroed before the pass: flag in bits 63..62,
// value in bits 31..0. digit_tot: the pass's global digit counts. The waits
// are bounded: a wait that runs past LB_SPIN polls sets bit 1 of *err and the
// keys go out clamped in place (wrong order, no access out of bounds).
constexpr uint32_t LB_SPIN = 1u << 16;
template <typename KeyT, int RS_ITEMS, int NT_, int RANK, typename XF = XfIdentity>
__global__ __launch_bounds__(NT_) void k_radix_scatter_lb(const KeyT* __restrict__ kin, KeyT* __restrict__ kout,
                                                            const uint32_t* d_count, uint32_t cap, int shift,
                                                            uint32_t dmask, const uint32_t* __restrict__ digit_tot,
                                                            uint64_t* status, uint32_t* tile_ctr, uint32_t* err,
                                                            XF xf = XF()) {
    constexpr int NW = NT_ / WAVE;
    constexpr int RS_TILE = NT_ * RS_ITEMS, RS_WAVE_SPAN = WAVE * RS_ITEMS;
    static_assert(NT_ >= 256, "a thread per digit");
    __shared__ uint32_t wcnt[NW][256];
    __shared__ uint32_t gofs[256];
    __shared__ uint32_t scratch[NW];
    __shared__ uint32_t s_tile;
    __shared__ __align__(16) KeyT skey[RS_TILE];
    constexpr bool MASK_IN_TILE = sizeof(KeyT) * RS_TILE >= sizeof(uint64_t) * 256 * NW;
    __shared__ uint64_t mask_own[RANK == RANK_MASK && !MASK_IN_TILE ? NW : 1][RANK == RANK_MASK ? 256 : 1];
    uint64_t (*wmask)[256] = MASK_IN_TILE ? reinterpret_cast<uint64_t (*)[256]>(skey)
                                          : reinterpret_cast<uint64_t (*)[256]>(mask_own);
    const uint32_t n = rs_count(d_count, cap);
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_ctr, 1u);
    for (int i = threadIdx.x; i < NW * 256; i += NT_) {
        (&wcnt[0][0])[i] = 0;
        if (RANK == RANK_MASK) (&wmask[0][0])[i] = 0ull;
    }
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t tile0 = tile * RS_TILE;
    if (tile0 >= n) return;   // empty: every tile after it is empty too, and none waits on it
    const int w = wave_id(), l = lane_id();
    const bool own = threadIdx.x < 256;
    const int dd = own ? (int)threadIdx.x : 0;
    const uint32_t base = tile0 + w * RS_WAVE_SPAN;
    KeyT k[RS_ITEMS];
    uint32_t loc[RS_ITEMS];
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const uint32_t i = base + it * WAVE + l;
        k[it] = i < n ? kin[i] : KeyT(0);
    }
    // keys with a smaller digit (the same for every tile), while the keys load
    const uint32_t dbase = block_exclusive_scan<NT_>(own ? digit_tot[dd] : 0u, scratch);
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {   // no branch around a transform's gathers
        const KeyT t = xf(k[it]);
        k[it] = base + it * WAVE + l < n ? t : k[it];
    }
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const uint32_t i = base + it * WAVE + l;
        const bool valid = i < n;
        const uint32_t d = (uint32_t)(k[it] >> shift) & dmask;
        if (RANK == RANK_ATOMIC) {   // a partition: ranks from LDS adds
            loc[it] = d | (atomicAdd(&wcnt[w][valid ? d : 0u], valid ? 1u : 0u) << 8);
            continue;
        }
        uint64_t peers;
        if (RANK == RANK_MATCH) {
            peers = match_digit8(d, __ballot(valid));
        } else {
            if (valid) atomicOr((unsigned long long*)&wmask[w][d], 1ull << l);
            __builtin_amdgcn_wave_barrier();
            peers = valid ? wmask[w][d] : 0ull;
            __builtin_amdgcn_wave_barrier();
        }
        const uint32_t r = (uint32_t)__popcll(peers & lanes_below());
        const uint32_t prev = wcnt[w][d];
        __builtin_amdgcn_wave_barrier();
        if (valid && r == 0) {
            wcnt[w][d] = prev + (uint32_t)__popcll(peers);
            if (RANK == RANK_MASK) wmask[w][d] = 0ull;
        }
        __builtin_amdgcn_wave_barrier();
        loc[it] = d | ((prev + r) << 8);
    }
    __syncthreads();
    uint32_t run = 0, excl;   // thread d: the tile's keys of digit d, and of the digits below d
    uint64_t* st = status + (size_t)tile * 256 + dd;
    {
        if (own) {
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                const uint32_t c = wcnt[q][dd];
                wcnt[q][dd] = run;
                run += c;
            }
            // this tile's count, for the tiles after it, as early as it is known
            __hip_atomic_store(st, (tile == 0 ? (2ull << 62) : (1ull << 62)) | run, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        excl = block_exclusive_scan<NT_>(run, scratch);
        if (own) {
#pragma unroll
            for (int q = 0; q < NW; ++q) wcnt[q][dd] += excl;
        }
    }
    __syncthreads();
    {   // the keys into LDS in digit order: needs only the positions inside the tile
        uint32_t pb[RS_ITEMS];
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it) pb[it] = wcnt[w][loc[it] & 255u];
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it)
            if (base + it * WAVE + l < n) skey[pb[it] + (loc[it] >> 8)] = k[it];
    }
    // then the look-back, by which time the tiles before have had the LDS pass
    // too to publish their totals
    if (own) {
        uint32_t before = 0;   // keys of digit dd in the tiles before this one
        if (tile > 0) {
            uint32_t j = tile - 1, spins = 0;
            for (;;) {
                const uint64_t v = __hip_atomic_load(status + (size_t)j * 256 + dd, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t f = (uint32_t)(v >> 62);
                if (f == 0) {
                    if (++spins > LB_SPIN) {
                        atomicOr(err, 2u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                before += (uint32_t)v;
                if (f == 2 || j == 0) break;
                --j;
            }
            __hip_atomic_store(st, (2ull << 62) | (before + run), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        gofs[dd] = dbase + before - excl;
    }
    __syncthreads();
    const uint32_t tile_n = n - tile0 < (uint32_t)RS_TILE ? n - tile0 : (uint32_t)RS_TILE;
    {
        KeyT key[RS_ITEMS];
        uint32_t go[RS_ITEMS];
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it) key[it] = skey[it * NT_ + threadIdx.x];
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it) go[it] = gofs[(uint32_t)(key[it] >> shift) & dmask];
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it) {
            const uint32_t j = it * NT_ + threadIdx.x;
            const uint32_t pos = go[it] + j;
            if (j < tile_n) kout[pos < n ? pos : n - 1] = key[it];
        }
    }
}

// Temporary layout: histogram table [256][ntiles + 1] | digit totals [256] (in the
// scan-temporary area) | segment totals [256][segments]. Sized for the
// smaller tiles, whose table is the larger.
static size_t rs_ntiles(size_t cap, uint32_t tile) { return (cap + tile - 1) / tile; }
static size_t rs_nseg(size_t ntiles) { return (ntiles + RS_ROW_SEG - 1) / RS_ROW_SEG; }

// Look-back region (end of the temporary): per pass p of a sort, its digit
// totals [LB_PASSES][256] and its tile counter [LB_PASSES]; an error word.
constexpr int LB_PASSES = LB_MAX_MORE + 1;
constexpr size_t LB_WORDS = LB_PASSES * 256 + LB_PASSES + 1;
static size_t rs_lb_offset(size_t cap) {
    const size_t ntiles = rs_ntiles(cap, RS_NT * RS_ITEMS_SMALL);
    return align_up(sizeof(uint32_t) * 256 * (ntiles + 1), 256) + align_up(scan_temp_bytes(), 256) +
           align_up(sizeof(uint32_t) * 256 * (rs_nseg(ntiles) + 1), 256);
}

size_t radix_temp_bytes(size_t cap) { return rs_lb_offset(cap) + align_up(sizeof(uint32_t) * LB_WORDS, 256); }

uint32_t* radix_err_word(void* temp, size_t cap) {
    return (uint32_t*)((char*)temp + rs_lb_offset(cap)) + LB_PASSES * 256 + LB_PASSES;
}


// Digit width of a sort over `bits` bits: the passes an 8-bit digit needs,
// with the bits spread evenly over them (a narrow last digit would crowd all
// keys into a few counters of the histogram).
static int digit_width(int bits) {
    const int passes = (bits + 7) / 8;
    return (bits + passes - 1) / passes;
}

MoreTot radix_sort_totals(void* temp, size_t cap, int key_bytes, int bit_lo, int bit_hi) {
    const int bits = bit_hi - bit_lo;
    if (bits <= 0 || radix_tile_keys(cap, key_bytes) != (uint32_t)(RS_NT * RS_ITEMS_HUGE)) return {nullptr, 0, 0, 0, 0};
    const int width = digit_width(bits);
    const int np = (bits + width - 1) / width;
    if (np > LB_MAX_MORE) return {nullptr, 0, 0, 0, 0};
    return {(uint32_t*)((char*)temp + rs_lb_offset(cap)), np, bit_lo, width, bit_hi};
}

RadixDigit radix_first_digit(int bit_lo, int bit_hi) {
    const int bits = bit_hi - bit_lo;
    const int w = bits > 0 ? digit_width(bits) : 0;
    return {bit_lo, w > 0 ? (uint32_t)((1u << w) - 1u) : 0u};
}

uint32_t* radix_first_counts(void* temp) { return (uint32_t*)temp; }

// The ranking of a pass: lane masks for 32-bit keys (twice the keys per byte
// moved, so the 8-ballot match costs twice as much per byte there); for
// 64-bit keys the match when stable, the LDS adds when not.
template <typename KeyT>
constexpr int rank_for(bool stable) {
    return sizeof(KeyT) == 4 ? RANK_MASK : (stable ? RANK_MATCH : RANK_ATOMIC);
}

template <typename KeyT, int RS_ITEMS, int RANK>
static void scatter_launch(const KeyT* kin, const uint32_t* vin, KeyT* kout, uint32_t* vout, const uint32_t* d_count,
                           size_t cap, int shift, uint32_t dmask, const uint32_t* hist, uint32_t ntiles,
                           const uint32_t* digit_tot, hipStream_t s) {
    if (RS_ITEMS == RS_ITEMS_HUGE) {   // 8192-key tiles: 512 threads of 16 keys
        if (vin)
            hipLaunchKernelGGL((k_radix_scatter<KeyT, true, RS_ITEMS / 2, 2 * RS_NT, XfIdentity, RANK>), dim3(ntiles),
                               dim3(2 * RS_NT), 0, s, kin, vin, kout, vout, d_count, (uint32_t)cap, shift, dmask,
                               hist, ntiles, digit_tot, XfIdentity());
        else
            hipLaunchKernelGGL((k_radix_scatter<KeyT, false, RS_ITEMS / 2, 2 * RS_NT, XfIdentity, RANK>),
                               dim3(ntiles), dim3(2 * RS_NT), 0, s, kin, nullptr, kout, nullptr, d_count,
                               (uint32_t)cap, shift, dmask, hist, ntiles, digit_tot, XfIdentity());
    } else if (vin) {
        hipLaunchKernelGGL((k_radix_scatter<KeyT, true, RS_ITEMS, RS_NT, XfIdentity, RANK>), dim3(ntiles), dim3(RS_NT),
                           0, s, kin, vin, kout, vout, d_count, (uint32_t)cap, shift, dmask, hist, ntiles, digit_tot,
                           XfIdentity());
    } else {
        hipLaunchKernelGGL((k_radix_scatter<KeyT, false, RS_ITEMS, RS_NT, XfIdentity, RANK>), dim3(ntiles),
                           dim3(RS_NT), 0, s, kin, nullptr, kout, nullptr, d_count, (uint32_t)cap, shift, dmask, hist,
                           ntiles, digit_tot, XfIdentity());
    }
}

template <typename KeyT, int RS_ITEMS>
static int radix_sort(KeyT* keys, KeyT* keys_alt, uint32_t* vals, uint32_t* vals_alt, const uint32_t* d_count,
                      size_t cap, int bit_lo, int bit_hi, void* temp, hipStream_t s, bool first_counted,
                      bool first_unstable, uint32_t* err, bool totals_given) {
    const int width = digit_width(bit_hi - bit_lo);
    const int npasses = (bit_hi - bit_lo + width - 1) / width;
    // 8192-key tiles, 64-bit keys only, several passes: the passes after the first
    // look back (no histogram pass); the first pass counts their digits. With the
    // totals given (counted by an earlier kernel), every pass looks back. (The one
    // 32-bit sort this large with several passes, the endpoint sort of ids wider
    // than 27 bits, keeps its histogram passes.)
    constexpr bool LB_TILES = RS_ITEMS == RS_ITEMS_HUGE && sizeof(KeyT) == 8;
    const bool all_lb = totals_given && LB_TILES && !vals && npasses <= LB_MAX_MORE;
    const bool lookback = all_lb || (LB_TILES && !vals && npasses >= 2 && npasses - 1 <= LB_MAX_MORE);
    uint32_t* lb = (uint32_t*)((char*)temp + rs_lb_offset(cap));   // totals | tile counters | error word
    if (lookback) {
        if (all_lb) fill_u32(lb + LB_PASSES * 256, 0u, LB_PASSES, s);   // the counters; the totals are given
        else fill_u32(lb, 0u, LB_PASSES * 256 + LB_PASSES, s);
        if (!err) err = lb + LB_PASSES * 256 + LB_PASSES;
    }
    const uint32_t ntiles = (uint32_t)rs_ntiles(cap, RS_NT * RS_ITEMS);
    uint32_t* hist = (uint32_t*)temp;
    void* scan_tmp = (char*)temp + align_up(sizeof(uint32_t) * 256 * (ntiles + 1), 256);
    uint32_t* digit_tot = (uint32_t*)scan_tmp;   // 256 digit totals
    uint32_t* seg_tot = (uint32_t*)((char*)scan_tmp + align_up(scan_temp_bytes(), 256));
    const uint32_t nseg = (uint32_t)rs_nseg(ntiles);
    KeyT* kin = keys;
    KeyT* kout = keys_alt;
    uint32_t* vin = vals;
    uint32_t* vout = vals_alt;
    int passes = 0;
    for (int shift = bit_lo; shift < bit_hi; shift += width, ++passes) {
        const int dbits = bit_hi - shift < width ? bit_hi - shift : width;   // the last digit may be narrower
        const uint32_t dmask = (1u << dbits) - 1u;
        if constexpr (LB_TILES) {
            if (lookback && (passes > 0 || all_lb)) {
                uint64_t* status = (uint64_t*)temp;   // the count table's room: ntiles * 256 words fit
                fill_u64(status, 0ull, (size_t)ntiles * 256, s);
                constexpr int IT = RS_ITEMS / 2, NTS = 2 * RS_NT;
                hipLaunchKernelGGL((k_radix_scatter_lb<KeyT, IT, NTS, rank_for<KeyT>(true)>), dim3(ntiles), dim3(NTS),
                                   0, s, kin, kout, d_count, (uint32_t)cap, shift, dmask, lb + passes * 256,
                                   status, lb + LB_PASSES * 256 + passes, err);
                KeyT* tk = kin; kin = kout; kout = tk;
                continue;
            }
        }
        if (!(first_counted && passes == 0))
            hipLaunchKernelGGL((k_radix_hist<KeyT, RS_ITEMS>), dim3(ntiles), dim3(RS_NT), 0, s, kin, d_count,
                               (uint32_t)cap, shift, dmask, hist, ntiles);
        hipLaunchKernelGGL(k_radix_rowscan, dim3(256, nseg), dim3(RS_NT), 0, s, hist, ntiles, digit_tot, seg_tot);
        if (nseg > 1)
            hipLaunchKernelGGL(k_radix_rowfix, dim3(256, nseg), dim3(RS_NT), 0, s, hist, ntiles, seg_tot, digit_tot);
        bool done = false;
        if constexpr (LB_TILES) {
            if (lookback) {   // the first pass: 8192-key tiles, keys only
                constexpr int IT = RS_ITEMS / 2, NTS = 2 * RS_NT;
                const MoreTot more{lb + 256, npasses - 1, shift + width, width, bit_hi};
                if (first_unstable)
                    hipLaunchKernelGGL((k_radix_scatter<KeyT, false, IT, NTS, XfIdentity, rank_for<KeyT>(false), true>),
                                       dim3(ntiles), dim3(NTS), 0, s, kin, nullptr, kout, nullptr, d_count,
                                       (uint32_t)cap, shift, dmask, hist, ntiles, digit_tot, XfIdentity(), more);
                else
                    hipLaunchKernelGGL((k_radix_scatter<KeyT, false, IT, NTS, XfIdentity, rank_for<KeyT>(true), true>),
                                       dim3(ntiles), dim3(NTS), 0, s, kin, nullptr, kout, nullptr, d_count,
                                       (uint32_t)cap, shift, dmask, hist, ntiles, digit_tot, XfIdentity(), more);
                done = true;
            }
        }
        if (done)
            ;
        else if (first_unstable && passes == 0)
            scatter_launch<KeyT, RS_ITEMS, rank_for<KeyT>(false)>(kin, vals ? vin : nullptr, kout, vout, d_count, cap,
                                                                  shift, dmask, hist, ntiles, digit_tot, s);
        else
            scatter_launch<KeyT, RS_ITEMS, rank_for<KeyT>(true)>(kin, vals ? vin : nullptr, kout, vout, d_count, cap,
                                                                 shift, dmask, hist, ntiles, digit_tot, s);
        KeyT* tk = kin; kin = kout; kout = tk;
        uint32_t* tv = vin; vin = vout; vout = tv;
    }
    return passes & 1;   // 1: result is in keys_alt / vals_alt
}

template <typename KeyT>
static int radix_sort_any(KeyT* keys, KeyT* keys_alt, uint32_t* vals, uint32_t* vals_alt, const uint32_t* d_count,
                          size_t cap, int bit_lo, int bit_hi, void* temp, hipStream_t s, bool first_counted,
                          bool first_unstable, uint32_t* err, bool totals_given) {
    if (cap == 0 || bit_hi <= bit_lo) return 0;
    const uint32_t tile = radix_tile_keys(cap, (int)sizeof(KeyT));
    if (tile == RS_NT * RS_ITEMS_HUGE)
        return radix_sort<KeyT, RS_ITEMS_HUGE>(keys, keys_alt, vals, vals_alt, d_count, cap, bit_lo, bit_hi, temp, s,
                                               first_counted, first_unstable, err, totals_given);
    if (tile == RS_NT * RS_ITEMS_LARGE)
        return radix_sort<KeyT, RS_ITEMS_LARGE>(keys, keys_alt, vals, vals_alt, d_count, cap, bit_lo, bit_hi, temp, s,
                                                first_counted, first_unstable, err, totals_given);
    return radix_sort<KeyT, RS_ITEMS_SMALL>(keys, keys_alt, vals, vals_alt, d_count, cap, bit_lo, bit_hi, temp, s,
                                            first_counted, first_unstable, err, totals_given);
}

template <int RS_ITEMS, typename XF>
static void radix_pass_xf(const uint64_t* kin, uint64_t* kout, size_t cap, int shift, int bits, XF xf,
                          bool hist_xf, uint32_t* counted, bool stable, const MoreTot& more,
                          const uint32_t* lb_tot, uint32_t* err, void* temp, hipStream_t s) {
    const uint32_t ntiles = (uint32_t)rs_ntiles(cap, RS_NT * RS_ITEMS);
    if constexpr (RS_ITEMS == RS_ITEMS_HUGE) {
        if (lb_tot) {   // the digit totals are given: one look-back kernel, no histogram
            uint32_t* lb = (uint32_t*)((char*)temp + rs_lb_offset(cap));
            uint32_t* ctr = lb + LB_PASSES * 256 + (LB_PASSES - 1);   // the last pass slot's counter
            if (!err) err = lb + LB_PASSES * 256 + LB_PASSES;
            uint64_t* status = (uint64_t*)temp;
            fill_u64(status, 0ull, (size_t)ntiles * 256, s);
            fill_u32(ctr, 0u, 1, s);
            constexpr int IT = RS_ITEMS / 2, NTS = 2 * RS_NT;
            const uint32_t dmask = (1u << bits) - 1u;
            if (stable)
                hipLaunchKernelGGL((k_radix_scatter_lb<uint64_t, IT, NTS, rank_for<uint64_t>(true), XF>), dim3(ntiles),
                                   dim3(NTS), 0, s, kin, kout, nullptr, (uint32_t)cap, shift, dmask, lb_tot, status,
                                   ctr, err, xf);
            else
                hipLaunchKernelGGL((k_radix_scatter_lb<uint64_t, IT, NTS, RANK_ATOMIC, XF>), dim3(ntiles), dim3(NTS), 0,
                                   s, kin, kout, nullptr, (uint32_t)cap, shift, dmask, lb_tot, status, ctr, err, xf);
            return;
        }
    }
    uint32_t* hist = counted ? counted : (uint32_t*)temp;
    void* scan_tmp = (char*)temp + align_up(sizeof(uint32_t) * 256 * (ntiles + 1), 256);
    uint32_t* digit_tot = (uint32_t*)scan_tmp;
    uint32_t* seg_tot = (uint32_t*)((char*)scan_tmp + align_up(scan_temp_bytes(), 256));
    const uint32_t nseg = (uint32_t)rs_nseg(ntiles);
    const uint32_t dmask = (1u << bits) - 1u;
    if (counted)   // the kernel that wrote or read the keys before has counted the digits
        ;
    else if (more.n > 0) {   // also the global counts for a later sort
        fill_u32(more.tot, 0u, (size_t)more.n * 256, s);
        hipLaunchKernelGGL((k_radix_hist<uint64_t, RS_ITEMS, XF, true>), dim3(ntiles), dim3(RS_NT), 0, s, kin, nullptr,
                           (uint32_t)cap, shift, dmask, hist, ntiles, xf, more);
    } else if (hist_xf)   // the digit depends on the transformed key
        hipLaunchKernelGGL((k_radix_hist<uint64_t, RS_ITEMS, XF>), dim3(ntiles), dim3(RS_NT), 0, s, kin, nullptr,
                           (uint32_t)cap, shift, dmask, hist, ntiles, xf);
    else
        hipLaunchKernelGGL((k_radix_hist<uint64_t, RS_ITEMS>), dim3(ntiles), dim3(RS_NT), 0, s, kin, nullptr,
                           (uint32_t)cap, shift, dmask, hist, ntiles, XfIdentity());
    hipLaunchKernelGGL(k_radix_rowscan, dim3(256, nseg), dim3(RS_NT), 0, s, hist, ntiles, digit_tot, seg_tot);
    if (nseg > 1)
        hipLaunchKernelGGL(k_radix_rowfix, dim3(256, nseg), dim3(RS_NT), 0, s, hist, ntiles, seg_tot, digit_tot);
    constexpr bool HUGE_TILES = RS_ITEMS == RS_ITEMS_HUGE;   // 8192-key tiles: 512 threads of 16 keys
    constexpr int IT = HUGE_TILES ? RS_ITEMS / 2 : RS_ITEMS;
    constexpr int NTS = HUGE_TILES ? 2 * RS_NT : RS_NT;
    if (stable)
        hipLaunchKernelGGL((k_radix_scatter<uint64_t, false, IT, NTS, XF, rank_for<uint64_t>(true)>), dim3(ntiles),
                           dim3(NTS), 0, s, kin, nullptr, kout, nullptr, nullptr, (uint32_t)cap, shift, dmask, hist,
                           ntiles, digit_tot, xf);
    else
        hipLaunchKernelGGL((k_radix_scatter<uint64_t, false, IT, NTS, XF, rank_for<uint64_t>(false)>), dim3(ntiles),
                           dim3(NTS), 0, s, kin, nullptr, kout, nullptr, nullptr, (uint32_t)cap, shift, dmask, hist,
                           ntiles, digit_tot, xf);
}

template <int RS_ITEMS>
static void radix_pass_kind(const uint64_t* kin, uint64_t* kout, size_t cap, int shift, int bits, const RadixXf& x,
                            uint32_t* counted, bool stable, const MoreTot& more, const uint32_t* lb_tot,
                            uint32_t* err, void* temp, hipStream_t s) {
    if (x.kind == RX_RANK_LOW)   // the digit lies in the untouched high half
        radix_pass_xf<RS_ITEMS>(kin, kout, cap, shift, bits, XfRankLow{x.rank, x.n}, false, counted, stable, more,
                                lb_tot, err, temp, s);
    else if (x.kind == RX_ORIENT)
        radix_pass_xf<RS_ITEMS>(kin, kout, cap, shift, bits, XfOrient{x.rank, x.n, x.nb, x.sentinel}, true, counted,
                                stable, more, lb_tot, err, temp, s);
    else
        radix_pass_xf<RS_ITEMS>(kin, kout, cap, shift, bits, XfIdentity(), false, counted, stable, more, lb_tot, err,
                                temp, s);
}

void radix_pass_u64(const uint64_t* kin, uint64_t* kout, size_t cap, int shift, int bits, const RadixXf& xf,
                    void* temp, hipStream_t s, uint32_t* counted, bool stable, const MoreTot& more,
                    const uint32_t* lb_tot, uint32_t* err) {
    if (cap == 0 || bits <= 0) return;
    const uint32_t tile = radix_tile_keys(cap, 8);
    if (tile == RS_NT * RS_ITEMS_HUGE)
        radix_pass_kind<RS_ITEMS_HUGE>(kin, kout, cap, shift, bits, xf, counted, stable, more, lb_tot, err, temp, s);
    else if (tile == RS_NT * RS_ITEMS_LARGE)
        radix_pass_kind<RS_ITEMS_LARGE>(kin, kout, cap, shift, bits, xf, counted, stable, more, lb_tot, err, temp, s);
    else
        radix_pass_kind<RS_ITEMS_SMALL>(kin, kout, cap, shift, bits, xf, counted, stable, more, lb_tot, err, temp, s);
}

int radix_digit_width(int bits) { return digit_width(bits); }

int radix_sort_u64(uint64_t* keys, uint64_t* keys_alt, uint32_t* vals, uint32_t* vals_alt, const uint32_t* d_count,
                   size_t cap, int bit_lo, int bit_hi, void* temp, hipStream_t s, bool first_counted,
                   bool first_unstable, uint32_t* err, bool totals_given) {
    return radix_sort_any<uint64_t>(keys, keys_alt, vals, vals_alt, d_count, cap, bit_lo, bit_hi, temp, s,
                                    first_counted, first_unstable, err, totals_given);
}

int radix_sort_u32(uint32_t* keys, uint32_t* keys_alt, uint32_t* vals, uint32_t* vals_alt, const uint32_t* d_count,
                   size_t cap, int bit_lo, int bit_hi, void* temp, hipStream_t s, bool first_counted,
                   bool first_unstable, uint32_t* err) {
    return radix_sort_any<uint32_t>(keys, keys_alt, vals, vals_alt, d_count, cap, bit_lo, bit_hi, temp, s,
                                    first_counted, first_unstable, err, false);
}

}  // namespace tcx
