// Sorting runs in place: keys already grouped by their high bits (key >> shift,
// ascending) are ordered by the whole key inside each run of equal high bits.
//
// The pair sort of the CSR build uses it. A stable radix sort on the lower rank
// of each oriented pair (its row) groups the pairs by row; this pass then orders
// every row by the higher rank, which the forward algorithm's sorted out-lists
// need (Section 3.2). Rows are short (the out-degree in (degree, id) order is at
// most sqrt(2m) on simple input), so one pass over the keys with each row sorted
// on chip replaces the radix passes over the higher rank's bits.
//
// A block takes a tile of SR_TILE positions and sorts the runs that start in it
// (a run may extend past the tile; the block reads and writes it whole). Other
// blocks read only the high bits of those positions, which a permutation inside
// a run leaves unchanged, so the in-place writes race with nothing. The block
// reads its tile once and keeps the low bits in LDS, with the overflow of its
// last run. By length:
//   - up to SR_SHORT: the runs starting in one 64-position window, up to the
//     first longer one, are sorted together by a bitonic network across the wave
//     (64 or 128 slots, each holding its run's index in the window above its low
//     bits, which keeps the runs apart);
//   - up to SR_MED: one wave, a bitonic network over the low bits held in
//     registers (the next power of two, up to 32 per lane);
//   - up to SR_BLOCK: the whole block, the same network over four waves, whose
//     cross-wave steps exchange through LDS;
//   - longer (only input with many repeated pairs has such rows): the whole
//     block, LSD radix passes over the low bits in `tmp` (the run's own range
//     of it) with the counters in LDS.
#include "common.h"
#include "internal.h"

namespace tcx {
namespace {

constexpr int SR_NT = 256;
constexpr int SR_NW = SR_NT / WAVE;
constexpr uint32_t SR_TILE = 4096;                 // positions per block
constexpr uint32_t SR_PER = SR_TILE / SR_NT;       // consecutive positions per thread in the scan for starts
constexpr uint32_t SR_WIN = 64;                    // positions per window of short runs
constexpr uint32_t SR_NWIN = SR_TILE / SR_WIN;
constexpr uint32_t SR_SHORT = 64;
constexpr uint32_t SR_MED = 2048;                  // one wave, at most 32 values per lane
constexpr uint32_t SR_BLOCK = 4096;                // the block, 16 values per lane
constexpr uint32_t SR_MAXMED = SR_TILE / (SR_SHORT + 1) + 1;   // medium runs that can start in one tile
constexpr uint32_t SR_MAXLONG = SR_TILE / (SR_MED + 1) + 1;   // runs past SR_MED that can start in one tile

struct SortRunsArgs {
    uint64_t* keys;
    uint64_t* tmp;       // as many keys as `keys`: a long run uses its own range of it
    uint32_t len;
    int shift;           // 1..32
    uint32_t skip;       // 1: a run whose first key is skip_key is left alone (it holds only that key)
    uint64_t skip_key;
    int passes, dw;      // radix passes over the low shift bits, and the digit width of each
    uint32_t* kept;      // non-null: per chunk of positions, += the keys that differ from their predecessor
    uint32_t chunk;      //   (the first of each run of equal keys; runs left alone are not counted)
};

struct alignas(16) Key2 {
    uint64_t a, b;
};

// Lanes of `active` whose digit (nbits wide) equals this lane's.
__device__ __forceinline__ uint64_t match_bits(uint32_t d, uint64_t active, int nbits) {
    uint64_t peers = active;
    for (int b = 0; b < nbits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

// ---- lane exchanges without LDS: DPP moves inside 16-lane rows, the gfx950
// permlane swaps across rows.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, false);
}

// {a, b} = this lane's value and lane l ^ M's, in either order (what a
// compare-exchange needs): M = 16 and 32 by the permlane swaps, which leave the
// two in their two outputs; M < 16 by DPP (quad permutations for 1 and 2, a
// half-row mirror then a quad reversal for 4, a row rotation by 8 for 8).
template <int M>
__device__ __forceinline__ void lane_pair(uint32_t x, uint32_t& a, uint32_t& b) {
    if constexpr (M == 16 || M == 32) {
        const auto p = M == 16 ? __builtin_amdgcn_permlane16_swap(x, x, false, false)
                               : __builtin_amdgcn_permlane32_swap(x, x, false, false);
        a = p[0];
        b = p[1];
    } else {
        static_assert(M == 1 || M == 2 || M == 4 || M == 8, "lane partner");
        a = x;
        if constexpr (M == 1) b = dpp_mov<0xB1>(x);
        else if constexpr (M == 2) b = dpp_mov<0x4E>(x);
        else if constexpr (M == 4) b = dpp_mov<0x1B>(dpp_mov<0x141>(x));
        else b = dpp_mov<0x128>(x);
    }
}

// The value of lane l ^ M, M = 2^t - 1 (the mirror partners of the flip steps):
// quad reversals and row mirrors by DPP; 16 and 32 added by a permlane swap and
// a select of the output that holds the partner.
template <int M>
__device__ __forceinline__ uint32_t lane_mirror(uint32_t x) {
    if constexpr (M == 1) return dpp_mov<0xB1>(x);
    else if constexpr (M == 3) return dpp_mov<0x1B>(x);
    else if constexpr (M == 7) return dpp_mov<0x141>(x);
    else if constexpr (M == 15) return dpp_mov<0x140>(x);
    else if constexpr (M == 31) {
        const auto p = __builtin_amdgcn_permlane16_swap(dpp_mov<0x140>(x), dpp_mov<0x140>(x), false, false);
        return (lane_id() & 16) ? p[0] : p[1];
    } else {
        static_assert(M == 63, "mirror partner");
        const uint32_t y = lane_mirror<31>(x);
        const auto p = __builtin_amdgcn_permlane32_swap(y, y, false, false);
        return (lane_id() & 32) ? p[0] : p[1];
    }
}

// The same on 64-bit values, one half at a time (both halves come from the same lane).
template <int M>
__device__ __forceinline__ void lane_pair(uint64_t x, uint64_t& a, uint64_t& b) {
    uint32_t al, bl, ah, bh;
    lane_pair<M>((uint32_t)x, al, bl);
    lane_pair<M>((uint32_t)(x >> 32), ah, bh);
    a = ((uint64_t)ah << 32) | al;
    b = ((uint64_t)bh << 32) | bl;
}

template <int M>
__device__ __forceinline__ uint64_t lane_mirror(uint64_t x) {
    return ((uint64_t)lane_mirror<M>((uint32_t)(x >> 32)) << 32) | lane_mirror<M>((uint32_t)x);
}

template <typename T>
__device__ __forceinline__ void ce(T& a, T& b) {   // ascending compare-exchange
    const T lo = a < b ? a : b, hi = a < b ? b : a;
    a = lo;
    b = hi;
}

// ---- bitonic sorting networks in registers, all compare-exchanges ascending
// (each phase k starts with a flip step that pairs e with e ^ (k - 1), then
// halves with e ^ j, j = k/4 .. 1). A wave holds 64P values, P per lane,
// element e = lane * P + r in x[r]: pairs inside a lane are two registers,
// pairs across lanes one DPP or permlane exchange.
template <typename T, int P, int J>
__device__ __forceinline__ void half_clean(T (&x)[P]) {
    if constexpr (J >= 1) {
        if constexpr (J < P) {
#pragma unroll
            for (int r = 0; r < P; ++r)
                if ((r & J) == 0) ce(x[r], x[r | J]);
        } else {
            constexpr int M = J / P;
            const bool lower = (lane_id() & M) == 0;
#pragma unroll
            for (int r = 0; r < P; ++r) {
                T a, b;
                lane_pair<M>(x[r], a, b);
                x[r] = (a < b) == lower ? a : b;
            }
        }
        half_clean<T, P, J / 2>(x);
    }
}

template <typename T, int P, int K>
__device__ __forceinline__ void flip(T (&x)[P]) {
    if constexpr (K <= P) {
#pragma unroll
        for (int r = 0; r < P; ++r)
            if ((r & (K / 2)) == 0) ce(x[r], x[r ^ (K - 1)]);
    } else {   // partner: lane l ^ (K/P - 1), register P - 1 - r
        const bool lower = (lane_id() & (K / (2 * P))) == 0;
        T y[P];
#pragma unroll
        for (int r = 0; r < P; ++r) y[r] = lane_mirror<K / P - 1>(x[P - 1 - r]);
#pragma unroll
        for (int r = 0; r < P; ++r) x[r] = (x[r] < y[r]) == lower ? x[r] : y[r];
    }
}

// Phases K .. KMAX (KMAX <= 64P): after phase 64P the wave's values ascend.
template <typename T, int P, int K, int KMAX>
__device__ __forceinline__ void sort_phases(T (&x)[P]) {
    if constexpr (K <= KMAX) {
        flip<T, P, K>(x);
        half_clean<T, P, K / 4>(x);
        sort_phases<T, P, K * 2, KMAX>(x);
    }
}

template <typename T, int P>
__device__ __forceinline__ void sort_wave(T (&x)[P]) {
    sort_phases<T, P, 2, 64 * P>(x);
}

// LDS position of tile-relative position p: one word of skew per 64 keeps the
// strided reads of the register sorts (lane l, element r at l * P + r) free of
// bank conflicts.
__host__ __device__ constexpr uint32_t sk(uint32_t p) { return p + (p >> 6); }

// The short runs of one window, slots [0, S) = tile positions [sp0, sp0 + S),
// S <= 127, P slots per lane (1 or 2): each slot's low bits with the index of
// its run inside the span above them (T = uint32_t when shift <= 25: at most
// 127 runs, 7 bits), sorted by the network; each position keeps its own high
// bits.
template <typename T, int P>
__device__ __forceinline__ uint32_t sort_window(uint64_t* keys, const uint32_t* v, const uint16_t* flag,
                                                uint32_t sp0, uint32_t S, int sh) {
    const uint32_t l = (uint32_t)lane_id();
    const int cs = sizeof(T) == 4 ? sh : 32;
    const uint64_t lmask = (1ull << sh) - 1ull;
    const uint64_t below = lanes_below();
    uint64_t o[P];
    T x[P];
    uint32_t before = 0;   // run starts in this lane's earlier slots
    bool st[P];
#pragma unroll
    for (int r = 0; r < P; ++r) {
        const uint32_t s = l * P + r, p = sp0 + s;
        o[r] = s < S ? keys[p] : 0ull;   // the high bits: loads in flight under the network
        st[r] = s < S && ((flag[p >> 4] >> (p & 15)) & 1u);
    }
    uint32_t prior = 0;    // run starts in the slots of the lanes below
#pragma unroll
    for (int r = 0; r < P; ++r) prior += (uint32_t)__popcll(__ballot(st[r]) & below);
#pragma unroll
    for (int r = 0; r < P; ++r) {
        const uint32_t s = l * P + r;
        before += st[r] ? 1u : 0u;
        const T ri = (T)(prior + before - 1u);   // slot 0 starts a run
        x[r] = s < S ? (T)((ri << cs) | (T)v[sk(sp0 + s)]) : ~T(0);
    }
    sort_wave<T, P>(x);
    // the slots whose value differs from the slot before (the run index is part
    // of it), counted across the wave
    T prev = __shfl_up(x[P - 1], 1, WAVE);
    uint32_t kept = 0;
#pragma unroll
    for (int r = 0; r < P; ++r) {
        const uint32_t s = l * P + r;
        if (s < S) keys[sp0 + s] = (o[r] & ~lmask) | ((uint64_t)x[r] & lmask);
        kept += (uint32_t)__popcll(__ballot(s < S && (s == 0 || x[r] != prev)));
        prev = x[r];
    }
    return kept;
}

// One wave: the run's low bits v[sk(st) ..] (L of them, L <= 64 * P) sorted in
// registers and put back in place.
template <int P>
__device__ __forceinline__ void wave_sort_run(uint32_t* v, uint32_t st, uint32_t L) {
    const uint32_t e0 = (uint32_t)lane_id() * P;
    uint32_t x[P];
#pragma unroll
    for (int r = 0; r < P; ++r) x[r] = e0 + r < L ? v[sk(st + e0 + r)] : 0xFFFFFFFFu;   // padding sorts last
    sort_wave<uint32_t, P>(x);
#pragma unroll
    for (int r = 0; r < P; ++r)
        if (e0 + r < L) v[sk(st + e0 + r)] = x[r];
}

// The whole block: N = 256 * P values (v[sk(0) ..], L of them, padded), four
// waves of 64P each sorted in registers; the steps that pair different waves
// exchange through v.
template <int P>
__device__ void block_bitonic(uint32_t* v, uint32_t L) {
    constexpr uint32_t N = 256u * P, WSPAN = 64u * P;
    const uint32_t e0 = (uint32_t)wave_id() * WSPAN + (uint32_t)lane_id() * P;
    uint32_t x[P];
#pragma unroll
    for (int r = 0; r < P; ++r) x[r] = e0 + r < L ? v[sk(e0 + r)] : 0xFFFFFFFFu;
    sort_wave<uint32_t, P>(x);
    for (uint32_t k = 2 * WSPAN; k <= N; k <<= 1) {
        for (uint32_t j = k - 1; j >= WSPAN; j = (j == k - 1) ? k / 4 : j / 2) {   // the flip, then halving
            __syncthreads();
#pragma unroll
            for (int r = 0; r < P; ++r) v[sk(e0 + r)] = x[r];
            __syncthreads();
            const bool lower = (e0 & (j == k - 1 ? k / 2 : j)) == 0;
#pragma unroll
            for (int r = 0; r < P; ++r) {
                const uint32_t y = v[sk((e0 + r) ^ j)];
                x[r] = (x[r] < y) == lower ? x[r] : y;
            }
        }
        half_clean<uint32_t, P, 32 * P>(x);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < P; ++r)
        if (e0 + r < L) v[sk(e0 + r)] = x[r];
    __syncthreads();
}

// The whole block: the same passes with the values in global memory (tA holds
// 2L uint32, the run's own range of tmp) and per-wave counters in LDS; each
// wave owns a contiguous quarter of the run, which keeps the passes stable.
__device__ void block_sort_run(uint64_t* run, uint32_t* tA, uint32_t L, const SortRunsArgs& a,
                               uint32_t (*cntw)[256], uint32_t* scan) {
    const int w = wave_id(), l = lane_id();
    const int sh = a.shift;
    const uint64_t hi = (run[0] >> sh) << sh;
    const uint64_t lmask = (1ull << sh) - 1ull;
    const uint32_t dmask = (1u << a.dw) - 1u;
    uint32_t* tB = tA + L;
    for (uint32_t i = threadIdx.x; i < L; i += SR_NT) tA[i] = (uint32_t)(run[i] & lmask);
    __threadfence();
    __syncthreads();
    const uint32_t Q = (L + SR_NW - 1) / SR_NW;
    const uint32_t q0 = (uint32_t)w * Q < L ? (uint32_t)w * Q : L;
    const uint32_t q1 = q0 + Q < L ? q0 + Q : L;
    uint32_t* cnt = cntw[w];
    for (int p = 0; p < a.passes; ++p) {
        const int ps = p * a.dw;
        const bool last = p + 1 == a.passes;
        for (int d = l; d < 256; d += WAVE) cnt[d] = 0u;
        __builtin_amdgcn_wave_barrier();
        for (uint32_t i = q0 + l; i < q1; i += WAVE) atomicAdd(&cnt[(tA[i] >> ps) & dmask], 1u);
        __syncthreads();
        {   // thread d: digit d's start for each wave's part
            const uint32_t d = threadIdx.x;
            uint32_t c[SR_NW], tot = 0;
#pragma unroll
            for (int q = 0; q < SR_NW; ++q) {
                c[q] = cntw[q][d];
                tot += c[q];
            }
            uint32_t o = block_exclusive_scan<SR_NT>(tot, scan);
#pragma unroll
            for (int q = 0; q < SR_NW; ++q) {
                cntw[q][d] = o;
                o += c[q];
            }
        }
        __syncthreads();
        for (uint32_t i0 = q0; i0 < q1; i0 += WAVE) {
            const uint32_t i = i0 + l;
            const bool valid = i < q1;
            const uint32_t v = valid ? tA[i] : 0u;
            const uint32_t d = (v >> ps) & dmask;
            const uint64_t peers = match_bits(d, __ballot(valid), a.dw);
            const uint32_t r = (uint32_t)__popcll(peers & lanes_below());
            const uint32_t b = cnt[d];
            __builtin_amdgcn_wave_barrier();
            if (valid && r == 0) cnt[d] = b + (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
            if (valid) {
                if (last) run[b + r] = hi | v;
                else tB[b + r] = v;
            }
        }
        __threadfence();
        __syncthreads();
        uint32_t* t = tA;
        tA = tB;
        tB = t;
    }
}

constexpr uint32_t SR_SPAN = SR_TILE + SR_MED;   // the tile and the overflow of its last run
constexpr uint32_t SR_NFLAG = SR_TILE / 16 + 8;  // run-start bits, 16 positions each (none past the tile)
// s_v holds tile-relative positions 0 .. SR_SPAN - 1 (the tile, then the overflow of
// its last row) and, for the long rows, block network elements 0 .. SR_BLOCK - 1, each at
// its skewed index sk(p)
constexpr uint32_t SR_VMAX = SR_SPAN > SR_BLOCK ? SR_SPAN : SR_BLOCK;
constexpr uint32_t SR_LDS = sk(SR_VMAX - 1) + 1;
static_assert(sk(SR_SPAN - 1) < SR_LDS && sk(SR_BLOCK - 1) < SR_LDS, "skewed LDS index past the array");

__global__ __launch_bounds__(SR_NT, 4) void k_sort_runs(SortRunsArgs a) {
    __shared__ uint32_t s_v[SR_LDS];                   // low bits of the keys, tile-relative position p at sk(p)
    __shared__ uint16_t s_bnd[SR_TILE];                 // run starts in the tile, ascending
    __shared__ uint16_t s_flag[SR_NFLAG];
    __shared__ uint32_t s_wf[SR_NWIN + 1];              // first run index per window
    __shared__ uint16_t s_med[SR_MAXMED];
    __shared__ uint32_t s_long[SR_MAXLONG];
    __shared__ uint32_t s_scan[SR_NW];
    __shared__ uint32_t s_nbnd, s_lastend, s_skippos, s_nmed, s_nlong, s_medctr;
    __shared__ uint32_t s_cnt[SR_NW][256];
    __shared__ uint32_t s_kept[8];                      // kept keys per chunk c0 .. c0 + 7

    const uint32_t t0 = (gridDim.x - 1 - blockIdx.x) * SR_TILE;   // the last tiles, whose runs are longest, first
    const uint32_t c0 = a.kept ? t0 / a.chunk : 0u;
    // kept keys at tile-relative position rel (cnt of them, all in rel's chunk)
    auto add_kept = [&](uint32_t rel, uint32_t cnt) {
        const uint32_t c = (t0 + rel) / a.chunk - c0;
        if (c < 8) atomicAdd(&s_kept[c], cnt);
        else atomicAdd(&a.kept[c0 + c], cnt);
    };
    // a wave's kept keys over positions [rel0, rel0 + len), tot of them (uniform): one add
    // when they share a chunk, else one per position (kept_at says which)
    auto wave_kept = [&](uint32_t rel0, uint32_t len, uint32_t tot, auto kept_at) {
        if ((t0 + rel0) / a.chunk == (t0 + rel0 + len - 1) / a.chunk) {
            if (lane_id() == 0 && tot) add_kept(rel0, tot);
        } else {
            kept_at();
        }
    };
    const uint32_t len = a.len;
    const int sh = a.shift;
    const uint64_t lmask = (1ull << sh) - 1ull;
    const int w = wave_id(), l = lane_id();
    uint64_t* const keys = a.keys + t0;   // tile-relative
    if (threadIdx.x == 0) {
        s_skippos = 0xFFFFFFFFu;
        s_nmed = 0;
        s_nlong = 0;
        s_medctr = 0;
    }
    if (threadIdx.x < SR_NFLAG - SR_TILE / 16) s_flag[SR_TILE / 16 + threadIdx.x] = 0;
    if (threadIdx.x < 8) s_kept[threadIdx.x] = 0;
    __syncthreads();
    // ---- run starts: a position whose high bits differ from its predecessor's
    {
        const uint32_t p0 = t0 + threadIdx.x * SR_PER;
        uint64_t k[SR_PER];
        if (p0 + SR_PER <= len) {
            const Key2* p = (const Key2*)(a.keys + p0);   // 128-byte aligned
#pragma unroll
            for (uint32_t q = 0; q < SR_PER / 2; ++q) {
                const Key2 v = p[q];
                k[2 * q] = v.a;
                k[2 * q + 1] = v.b;
            }
        } else {
#pragma unroll
            for (uint32_t j = 0; j < SR_PER; ++j) k[j] = p0 + j < len ? a.keys[p0 + j] : 0ull;
        }
        uint64_t ph = p0 > 0 && p0 <= len ? a.keys[p0 - 1] >> sh : 0ull;
        uint32_t flags = 0;
#pragma unroll
        for (uint32_t j = 0; j < SR_PER; ++j) {
            const uint32_t p = p0 + j;
            s_v[sk(threadIdx.x * SR_PER + j)] = (uint32_t)(k[j] & lmask);
            if (p < len) {
                const uint64_t h = k[j] >> sh;
                if (p == 0 || h != ph) {
                    flags |= 1u << j;
                    if (a.skip && k[j] == a.skip_key) s_skippos = p - t0;   // at most one run starts with it
                }
                ph = h;
            }
        }
        s_flag[threadIdx.x] = (uint16_t)flags;
        uint32_t total;
        uint32_t o = block_exclusive_scan<SR_NT>((uint32_t)__popc(flags), s_scan, &total);
        if ((threadIdx.x & 3) == 0) s_wf[threadIdx.x >> 2] = o;
        if (threadIdx.x == 0) {
            s_wf[SR_NWIN] = total;
            s_nbnd = total;
        }
#pragma unroll
        for (uint32_t j = 0; j < SR_PER; ++j)
            if ((flags >> j) & 1u) s_bnd[o++] = (uint16_t)(threadIdx.x * SR_PER + j);
    }
    __syncthreads();
    const uint32_t nbnd = s_nbnd;
    if (nbnd == 0) return;   // the whole tile lies in a run that starts earlier
    // ---- where the tile's last run ends: a 64-way search past the tile
    if (w == 0) {
        const uint64_t hl = keys[s_bnd[nbnd - 1]] >> sh;
        uint32_t lo = t0 + SR_TILE < len ? t0 + SR_TILE : len;   // [last start, lo) lies in the run
        uint32_t hi = len;                                      // [hi, len) does not
        while (lo < hi) {
            const uint32_t step = (hi - lo + WAVE - 1) / WAVE;
            const uint32_t q = lo + (uint32_t)l * step;
            const bool in = q < hi && (a.keys[q] >> sh) == hl;
            const uint32_t c = (uint32_t)__popcll(__ballot(in));   // the probes in the run are a prefix
            if (c == 0) {
                hi = lo;
            } else {
                const uint32_t nlo = lo + (c - 1) * step + 1;
                const uint32_t qc = lo + c * step;
                if (c < (uint32_t)WAVE && qc < hi) hi = qc;
                lo = nlo;
            }
            lo = __builtin_amdgcn_readfirstlane(lo);
            hi = __builtin_amdgcn_readfirstlane(hi);
        }
        if (l == 0) s_lastend = lo - t0;
    }
    __syncthreads();
    const uint32_t lastend = s_lastend, skippos = s_skippos;
    auto run_end = [&](uint32_t i) -> uint32_t { return i + 1 < nbnd ? (uint32_t)s_bnd[i + 1] : lastend; };
    {   // the last run's positions past the tile, when it is sorted in LDS
        const uint32_t st = s_bnd[nbnd - 1];
        if (lastend > SR_TILE && lastend - st <= SR_MED && st != skippos)
            for (uint32_t p = SR_TILE + threadIdx.x; p < lastend; p += SR_NT) s_v[sk(p)] = (uint32_t)(keys[p] & lmask);
    }
    // ---- medium and long runs
    for (uint32_t i = threadIdx.x; i < nbnd; i += SR_NT) {
        const uint32_t st = s_bnd[i];
        const uint32_t L = run_end(i) - st;
        if (st == skippos || L <= SR_SHORT) continue;
        if (L <= SR_MED) s_med[atomicAdd(&s_nmed, 1u)] = (uint16_t)i;
        else s_long[atomicAdd(&s_nlong, 1u)] = i;
    }
    __syncthreads();
    // ---- short runs, window by window
    for (uint32_t win = w; win < SR_NWIN; win += SR_NW) {
        const uint32_t r0 = s_wf[win], r1 = s_wf[win + 1];
        if (r0 == r1) continue;
        const uint32_t r = r0 + l;
        const bool has = r < r1;
        uint32_t L = 0;
        bool bad = false;
        if (has) {
            const uint32_t st = s_bnd[r];
            L = run_end(r) - st;
            bad = L > SR_SHORT || st == skippos;
        }
        const uint64_t mb = __ballot(bad);
        const uint32_t cut = mb ? (uint32_t)__ffsll((unsigned long long)mb) - 1u : r1 - r0;
        if (cut == 0) continue;
        const uint32_t sp0 = s_bnd[r0];
        if (__ballot(has && (uint32_t)l < cut && L >= 2) == 0) {   // single keys only: nothing to sort
            if (a.kept)
                wave_kept(sp0, cut, cut, [&] {
                    if ((uint32_t)l < cut) add_kept(sp0 + l, 1u);
                });
            continue;
        }
        const uint32_t S = run_end(r0 + cut - 1) - sp0;   // at most 127
        uint32_t kept;
        if (sh <= 25) {
            if (S <= 64) kept = sort_window<uint32_t, 1>(keys, s_v, s_flag, sp0, S, sh);
            else kept = sort_window<uint32_t, 2>(keys, s_v, s_flag, sp0, S, sh);
        } else {
            if (S <= 64) kept = sort_window<uint64_t, 1>(keys, s_v, s_flag, sp0, S, sh);
            else kept = sort_window<uint64_t, 2>(keys, s_v, s_flag, sp0, S, sh);
        }
        if (a.kept)
            wave_kept(sp0, S, kept, [&] {   // a chunk boundary inside the span: position by position
                for (uint32_t q = l; q < S; q += WAVE) {
                    const uint64_t k = keys[sp0 + q];
                    if (q == 0 || k != keys[sp0 + q - 1]) add_kept(sp0 + q, 1u);
                }
            });
    }
    // ---- medium runs, one wave each: a register sort of the next power of two
    {
        const uint32_t nmed = s_nmed;
        for (;;) {
            uint32_t idx = 0;
            if (l == 0) idx = atomicAdd(&s_medctr, 1u);
            idx = __builtin_amdgcn_readfirstlane(idx);
            if (idx >= nmed) break;
            const uint32_t i = s_med[idx];
            const uint32_t st = s_bnd[i], L = run_end(i) - st;
            const uint64_t hi = (keys[st] >> sh) << sh;
            if (L <= 128) wave_sort_run<2>(s_v, st, L);
            else if (L <= 256) wave_sort_run<4>(s_v, st, L);
            else if (L <= 512) wave_sort_run<8>(s_v, st, L);
            else if (L <= 1024) wave_sort_run<16>(s_v, st, L);
            else wave_sort_run<32>(s_v, st, L);
            __builtin_amdgcn_wave_barrier();
            uint32_t kept = 0;
            for (uint32_t p0 = 0; p0 < L; p0 += WAVE) {
                const uint32_t p = p0 + l;
                const uint32_t v = p < L ? s_v[sk(st + p)] : 0u;
                if (p < L) keys[st + p] = hi | v;
                if (a.kept) kept += (uint32_t)__popcll(__ballot(p < L && (p == 0 || v != s_v[sk(st + p - 1)])));
            }
            if (a.kept)
                wave_kept(st, L, kept, [&] {
                    for (uint32_t p = l; p < L; p += WAVE)
                        if (p == 0 || s_v[sk(st + p)] != s_v[sk(st + p - 1)]) add_kept(st + p, 1u);
                });
        }
    }
    // ---- long runs, the whole block: a network over LDS up to SR_BLOCK, else radix passes in tmp
    __syncthreads();
    const uint32_t nlong = s_nlong;
    for (uint32_t q = 0; q < nlong; ++q) {
        const uint32_t i = s_long[q];
        const uint32_t st = s_bnd[i], L = run_end(i) - st;
        uint64_t* run = keys + st;
        if (L <= SR_BLOCK) {
            const uint64_t hi = (run[0] >> sh) << sh;
            for (uint32_t p = threadIdx.x; p < L; p += SR_NT) s_v[sk(p)] = (uint32_t)(run[p] & lmask);
            __syncthreads();
            if (L <= SR_BLOCK / 2) block_bitonic<SR_BLOCK / 2 / SR_NT>(s_v, L);
            else block_bitonic<SR_BLOCK / SR_NT>(s_v, L);
            for (uint32_t p = threadIdx.x; p < L; p += SR_NT) {
                const uint32_t v = s_v[sk(p)];
                run[p] = hi | v;
                if (a.kept && (p == 0 || v != s_v[sk(p - 1)])) add_kept(st + p, 1u);
            }
            __syncthreads();
        } else {
            block_sort_run(run, (uint32_t*)(a.tmp + t0 + st), L, a, s_cnt, s_scan);
            if (a.kept)
                for (uint32_t p = threadIdx.x; p < L; p += SR_NT)
                    if (p == 0 || run[p] != run[p - 1]) add_kept(st + p, 1u);
        }
    }
    if (a.kept) {
        __syncthreads();
        if (threadIdx.x < 8 && s_kept[threadIdx.x]) atomicAdd(&a.kept[c0 + threadIdx.x], s_kept[threadIdx.x]);
    }
}

}  // namespace

void sort_runs_u64(uint64_t* keys, uint64_t* tmp, size_t len, int shift, bool skip, uint64_t skip_key,
                   uint32_t* kept, uint32_t chunk, hipStream_t s) {
    if (len == 0) return;
    SortRunsArgs a;
    a.keys = keys;
    a.tmp = tmp;
    a.len = (uint32_t)len;
    a.shift = shift;
    a.skip = skip ? 1u : 0u;
    a.skip_key = skip_key;
    a.passes = (shift + 7) / 8;
    a.dw = (shift + a.passes - 1) / a.passes;
    a.kept = kept;
    a.chunk = chunk > 0 ? chunk : 1u;
    const uint32_t grid = (uint32_t)((len + SR_TILE - 1) / SR_TILE);
    hipLaunchKernelGGL(k_sort_runs, dim3(grid), dim3(SR_NT), 0, s, a);
}

}  // namespace tcx
