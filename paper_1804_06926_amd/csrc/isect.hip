// Per-edge intersection kernels (Section 3.2, Algorithm 2 "Compute_Intersection";
// Section 4.2, dynamic grouping and the large/small neighbour-list kernels).
//
// The graph is the degree-ordered CSR over ranks: row u holds N+(u), the
// neighbours ranked above u, ascending. For a kept edge e = (u -> v) at
// position p of row u, a common neighbour w of N+(u) and N+(v) must rank above
// v, so only the tail of row u after p can match:
//     c_e = | row_u[p+1 ..] intersected with N+(v) |  =  | N+(u) intersected with N+(v) |.
// Work is grouped by the middle vertex v. A tile is either one vertex v with a
// chunk of its in-edges, or several vertices of one bucket with all their
// in-edges. Three interchangeable strategies compute the same c_e for every
// in-edge of a tile:
//   merge   : merge-path split of (tail, N+(v)) across a group of lanes
//   bsearch : binary search of each element of the shorter list in the other
//   bitmap  : N+(v) staged once per vertex as an LDS bitmap; all tails of the
//             tile streamed through it as one flat, coalesced item range
// Each hit adds 1 to the exact 64-bit triangle count; optional outputs are
// the per-edge counts c_e, the per-vertex counts t[u], t[v], t[w] and the
// edge support (triangles per edge: a hit w adds 1 to edges uv, uw and vw;
// uw is the tail element's own CSR position, vw the position of w in N+(v)).
// Block b starts with tile b; after that the blocks take tiles in order from a
// shared counter (one atomic per tile), so a block that drew light tiles takes
// more: tiles are ordered heaviest bucket first, which makes this a
// longest-first schedule. Blocks without a first tile exit at once (small
// graphs). The counter is zeroed before each launch (launch_isect callers).
// Each block writes its partial count and one reduction adds them in a fixed
// order; T does not depend on which block counted which tile (integer sums).
// A second pass of the same kernels writes the triangles themselves (listing).
// The same kernels serve the paper's other formulations (whole neighbour
// lists; the matrix formulation of Section 3.3): an entry's range is then a
// whole row that may reach below and above the middle list, and the bitmap
// kernel cuts it to each window it tests (clipped mode, counts only).
#include "common.h"
#include "internal.h"
#include "isect.h"

namespace tcx {

constexpr int IS_NT = 256;
constexpr int BM_WORDS = 4096;            // 131072-bit window (16 KiB)
constexpr uint32_t BM_BITS = BM_WORDS * 32u;
static_assert(BM_BITS == (1u << BM_WINDOW_LOG2), "the selector's window feature counts these windows");
constexpr int UNROLL = 8;                 // bitmap kernel: tail loads in flight per lane
constexpr uint32_t WT_MAX = 1024;         // bitmap kernel: 64-item windows per chunk of the item range
constexpr uint32_t LONG_TAIL = 64;        // bitmap kernel: tails of at least one window are walked directly
constexpr int NV_MAX = 2048;              // bitmap kernel, per-vertex mode: N+(v) kept for t[w] gathering
constexpr int PARTIALS_PER_KERNEL = 4096; // max blocks per intersection launch

template <int N>
struct SegsT {
    uint32_t v[N];
    uint32_t e0[N];
    uint32_t pref[N + 1];
    uint32_t scratch[IS_NT / WAVE];
};
using Segs = SegsT<SEG_MAX>;

// The next tile for this block after its first (static) one: t0 + the shared
// counter of kernel ker, which is zero when the launch starts. Called by the
// whole block (barriers); the value is the same in every thread.
__device__ __forceinline__ uint32_t grab_tile(Ctrl* ctrl, int ker, uint32_t t0, uint32_t* s_tile) {
    __syncthreads();   // every thread has read the previous value
    if (threadIdx.x == 0) *s_tile = t0 + atomicAdd(&ctrl->tile_next[ker], 1u);
    __syncthreads();
    return *s_tile;
}

// Decode tile t into segments (v, first in-edge, count); returns the count.
// Called by the whole block; contains barriers.
template <int N>
__device__ uint32_t load_tile(const IsectArgs& a, uint32_t t, SegsT<N>& S) {
    const uint4 d = a.tiles[t];
    uint32_t nseg, cnt = 0;
    if (d.w & TILE_MULTI) {
        nseg = d.y;
        if (nseg > (uint32_t)N) nseg = N;   // the tile layout never makes more
        if (threadIdx.x < nseg) {
            const uint32_t v = a.vlist[d.x + threadIdx.x];
            S.v[threadIdx.x] = v;
            S.e0[threadIdx.x] = a.inoff[v];
            cnt = a.inoff[v + 1] - a.inoff[v];
        }
    } else {   // one vertex: no scan needed
        if (threadIdx.x == 0) {
            S.v[0] = d.x;
            S.e0[0] = d.y;
            S.pref[0] = 0;
            S.pref[1] = d.z;
        }
        __syncthreads();
        return 1;
    }
    uint32_t total;
    const uint32_t excl = block_exclusive_scan<IS_NT>(cnt, S.scratch, &total);
    if (threadIdx.x < nseg) S.pref[threadIdx.x] = excl;
    if (threadIdx.x == 0) S.pref[nseg] = total;
    __syncthreads();
    return nseg;
}

__device__ __forceinline__ void edge_done(const IsectArgs& a, uint32_t e, uint32_t v, uint32_t c,
                                          bool middle = true) {
    if (a.per_edge) a.per_edge[e] = c;
    if (a.support && c) atomicAdd(&a.support[e], c);
    if (middle && a.per_middle && c) atomicAdd((unsigned long long*)&a.per_middle[v], (unsigned long long)c);
    if (a.per_vertex && c) {
        atomicAdd((unsigned long long*)&a.per_vertex[a.src[e]], (unsigned long long)c);
        atomicAdd((unsigned long long*)&a.per_vertex[v], (unsigned long long)c);
    }
}

__device__ __forceinline__ void hit_vertex(const IsectArgs& a, uint32_t w) {
    if (a.per_vertex) atomicAdd((unsigned long long*)&a.per_vertex[w], 1ull);
}

// Triangle (u, v, w) of in-edge e = (u -> v) at list slot pos, original ids.
__device__ __forceinline__ void list_write(const IsectArgs& a, uint64_t pos, uint32_t e, uint32_t w) {
    if (pos >= a.list_cap) {   // only if the two passes disagree
        atomicOr(&a.ctrl->err, 8u);
        return;
    }
    int32_t* o = a.list_out + 3 * pos;
    o[0] = (int32_t)a.inv[a.src[e]];
    o[1] = (int32_t)a.inv[a.col[e]];
    o[2] = (int32_t)a.inv[w];
}

// A hit w = col[ea] = col[eb] for in-edge ein: ea is the edge (u, w) of the
// tail, eb the edge (v, w).
__device__ __forceinline__ void hit(const IsectArgs& a, uint32_t w, uint32_t ea, uint32_t eb, uint32_t ein) {
    hit_vertex(a, w);
    if (a.support) {
        atomicAdd(&a.support[ea], 1u);
        atomicAdd(&a.support[eb], 1u);
    }
    if (a.list_out) list_write(a, a.list_off[ein] + atomicAdd(&a.list_cur[ein], 1u), ein, w);
}

// Position of x in the ascending list L[0..n), or n when absent.
__device__ __forceinline__ uint32_t find_pos(const uint32_t* L, uint32_t n, uint32_t x) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (L[mid] < x) lo = mid + 1u;
        else hi = mid;
    }
    return (lo < n && L[lo] == x) ? lo : n;
}

__device__ __forceinline__ void block_partial(uint64_t acc, uint64_t* partials) {
    __shared__ uint64_t red[IS_NT / WAVE];
    acc = wave_sum_u64(acc);
    if (lane_id() == 0) red[wave_id()] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        for (int i = 0; i < IS_NT / WAVE; ++i) s += red[i];
        partials[blockIdx.x] = s;
    }
}

// ------------------------------------------------------------------ LDS bitmap
// Element i of col. NARROW: the array is below 4 GiB, so a 32-bit byte offset
// from the (scalar) base addresses it and no 64-bit address math is needed.
template <bool NARROW>
__device__ __forceinline__ uint32_t col_at(const uint32_t* col, uint32_t i) {
    if (NARROW) return *(const uint32_t*)((const char*)col + (uint32_t)(i << 2));
    return col[i];
}

// Outputs of a bitmap launch: T only; also per in-edge counts (per-edge or
// per-middle-vertex outputs); or also gathered per-vertex counts or edge
// support (the hits per element of N+(v), for t[w] and the support of edge
// vw, are gathered in LDS); or the triangle list (the per-entry count is the
// cursor of the entry's slots). Each mode sizes its LDS to what it uses.
// BM_CLIP counts only, for tails that are whole rows: each tail and the middle
// list are cut to the window being tested, and windows holding no element of
// the middle list are skipped.
enum { BM_COUNT = 0, BM_ENTRY = 1, BM_GATHER = 2, BM_LIST = 3, BM_CLIP = 4, BM_NMODE = 5 };

constexpr int EH = CHUNK_MAX / IS_NT;   // entries of a vertex per thread

// First position p in [p, e) of the ascending col whose value is at least x (e if none).
template <bool NARROW>
__device__ __forceinline__ uint32_t first_at_least(const uint32_t* col, uint32_t p, uint32_t e, uint64_t x) {
    while (p < e) {
        const uint32_t mid = p + ((e - p) >> 1);
        if ((uint64_t)col_at<NARROW>(col, mid) < x) p = mid + 1u;
        else e = mid;
    }
    return p;
}

// The same search by a whole wave, the same result in every lane: 64 probes
// per step narrow the range 64-fold, so a list of d elements costs about
// log64(d) dependent loads instead of log2(d).
template <bool NARROW>
__device__ __forceinline__ uint32_t wave_first_at_least(const uint32_t* col, uint32_t p, uint32_t e, uint64_t x) {
    const uint32_t ln = (uint32_t)lane_id();
    while (e - p > (uint32_t)WAVE) {
        const uint32_t step = (e - p + WAVE - 1) / WAVE;
        const uint32_t q = p + (ln + 1u) * step - 1u;   // last element of the lane's step
        const bool below = q < e && (uint64_t)col_at<NARROW>(col, q) < x;
        const uint32_t c = (uint32_t)__popcll(__ballot(below));   // steps wholly below x
        const uint32_t np = p + c * step;
        e = np + step < e ? np + step : e;
        p = np;
    }
    const uint32_t q = p + ln;
    const bool below = q < e && (uint64_t)col_at<NARROW>(col, q) < x;
    return p + (uint32_t)__popcll(__ballot(below));
}

// Entry table of one vertex's in-edges in a tile, in LDS: entry k streams
// items [s_pref[k], s_pref[k + 1]) of a flat item range, item q at
// col[s_base[k] + q] (s_base = start - s_pref, modular). Tails of at least
// LONG_TAIL items come first, then the shorter non-empty ones; empty tails are
// left out, so s_pref is strictly increasing. Thread t holds entries EH * t ..
// EH * t + EH - 1 (start st_h, length len_h; length 0 past the vertex's
// entries) and later owns the table slots with the same indexes, so each
// phase needs one block scan. Returns the entries kept; nl = long entries,
// L = total items. Whole block; contains barriers.
template <bool CNT>
__device__ __forceinline__ uint32_t entry_table(const uint32_t (&st_h)[EH], const uint32_t (&len_h)[EH],
                                                uint32_t* s_pref, uint32_t* s_base, uint32_t* s_cnt,
                                                uint32_t* scratch, uint32_t& nl, uint32_t& L) {
    uint32_t f = 0;   // long entries in the high half, non-empty short ones in the low half
#pragma unroll
    for (int h = 0; h < EH; ++h) f += len_h[h] >= LONG_TAIL ? 0x10000u : (len_h[h] ? 1u : 0u);
    uint32_t total;
    const uint32_t ex = block_exclusive_scan<IS_NT>(f, scratch, &total);
    const uint32_t cl = total >> 16, cs = total & 0xFFFFu;
    uint32_t pl = ex >> 16, ps = cl + (ex & 0xFFFFu);
#pragma unroll
    for (int h = 0; h < EH; ++h) {   // lengths and starts in table order
        if (!len_h[h]) continue;
        const uint32_t pos = len_h[h] >= LONG_TAIL ? pl++ : ps++;
        s_pref[pos] = len_h[h];
        s_base[pos] = st_h[h];
        if (CNT) s_cnt[pos] = 0;
    }
    __syncthreads();
    const uint32_t nt = cl + cs;
    uint32_t len[EH], st[EH], sum = 0;
#pragma unroll
    for (int h = 0; h < EH; ++h) {   // this thread's slots, rewritten in place below
        const uint32_t k = EH * threadIdx.x + (uint32_t)h;
        len[h] = k < nt ? s_pref[k] : 0u;
        st[h] = k < nt ? s_base[k] : 0u;
        sum += len[h];
    }
    uint32_t items;
    uint32_t run = block_exclusive_scan<IS_NT>(sum, scratch, &items);
#pragma unroll
    for (int h = 0; h < EH; ++h) {
        const uint32_t k = EH * threadIdx.x + (uint32_t)h;
        if (k < nt) {
            s_pref[k] = run;
            s_base[k] = st[h] - run;
        }
        run += len[h];
    }
    if (threadIdx.x == 0) s_pref[nt] = items;
    nl = cl;
    L = items;
    return nt;
}

// Six blocks of four waves fit a CU by LDS in every mode but the gathering one
// (44 KB); the register budget is held to the same occupancy (80 VGPRs).
template <int MODE, bool NARROW>
__global__ __launch_bounds__(IS_NT, MODE == BM_GATHER ? 1 : 6) void k_isect_bitmap(IsectArgs a, uint64_t* partials) {
    constexpr bool GATHER = MODE == BM_GATHER;
    constexpr bool CLIP = MODE == BM_CLIP;
    constexpr bool need_cnt = MODE != BM_COUNT && !CLIP;
    __shared__ uint32_t s_nv[GATHER ? NV_MAX : 1];
    __shared__ uint32_t s_wc[GATHER ? NV_MAX : 1];
    __shared__ uint32_t bm[BM_WORDS + 1];        // + one always-zero word for out-of-window positions
    __shared__ uint16_t s_wst[WT_MAX];           // entry holding the first item of each window of a chunk
    __shared__ uint32_t s_pref[CHUNK_MAX + 1];
    __shared__ uint32_t s_cnt[need_cnt ? CHUNK_MAX : 1];
    __shared__ uint32_t s_base[CHUNK_MAX + 1];   // entry nt is read (unused) by lanes past the end
    __shared__ uint8_t s_flag[IS_NT / WAVE][UNROLL][WAVE];    // entry-start marks, one slot per item offset
    __shared__ SegsT<SEG_MAX_BITMAP> S;
    for (int i = threadIdx.x; i <= BM_WORDS; i += IS_NT) bm[i] = 0;
    for (int i = threadIdx.x; i < (IS_NT / WAVE) * UNROLL * WAVE; i += IS_NT) (&s_flag[0][0][0])[i] = 0;
    uint64_t acc = 0;
    __shared__ uint32_t s_tile;
    const uint32_t t_begin = a.ctrl->tile_begin[KER_BITMAP], t_end = a.ctrl->tile_begin[KER_BITMAP + 1];
    for (uint32_t t = t_begin + blockIdx.x; t < t_end; t = grab_tile(a.ctrl, KER_BITMAP, t_begin + gridDim.x, &s_tile)) {
        const uint32_t nseg = load_tile(a, t, S);
        for (uint32_t sg = 0; sg < nseg; ++sg) {
            const uint32_t v = S.v[sg];
            const uint32_t e0 = S.e0[sg];
            const uint32_t ne = S.pref[sg + 1] - S.pref[sg];
            const uint32_t b0 = a.off[v], b1 = a.off[v + 1];
            const uint32_t nb = b1 - b0;
            // the vertex's entries (ne <= CHUNK_MAX = EH * IS_NT: EH consecutive ones per thread)
            uint32_t st_h[EH], len_h[EH];
#pragma unroll
            for (int h = 0; h < EH; ++h) {
                const uint32_t k = EH * threadIdx.x + (uint32_t)h;
                st_h[h] = len_h[h] = 0;
                if (k < ne) {
                    const uint64_t ent = a.csc[e0 + k];   // tail start | tail end << 32
                    st_h[h] = (uint32_t)ent;
                    len_h[h] = (uint32_t)(ent >> 32) - st_h[h];
                }
            }
            // the table: once per vertex, or per window when the tails are clipped
            uint32_t nt = 0, nl = 0, L = 0;
            if (!CLIP) nt = entry_table<need_cnt>(st_h, len_h, s_pref, s_base, s_cnt, S.scratch, nl, L);
            const uint32_t lo = a.col[b0], hi = a.col[b1 - 1];
            const uint32_t base = lo & ~31u;
            const uint32_t nwin = (hi - base) / BM_BITS + 1;
            if (GATHER && nb <= (uint32_t)NV_MAX) {
                for (uint32_t j = threadIdx.x; j < nb; j += IS_NT) {
                    s_nv[j] = a.col[b0 + j];
                    s_wc[j] = 0u;
                }
            }
            __syncthreads();
            // clipped tails: each entry keeps a cursor (st_h, with len_h left) and the
            // value under it, so a window that holds none of its elements costs no load
            uint64_t cv_h[EH];
            if (CLIP) {
#pragma unroll
                for (int h = 0; h < EH; ++h)
                    cv_h[h] = len_h[h] ? (uint64_t)col_at<NARROW>(a.col, st_h[h]) : ~0ull;
            }
            uint32_t mnext = 0;   // clipped: first element of the middle list not yet in a window
            for (uint32_t win = 0; win < nwin; ++win) {
                const uint32_t wlo = base + win * BM_BITS;
                uint32_t j0 = 0, j1 = nb;   // elements of the middle list set in this window
                if (CLIP) {
                    const uint64_t whi = (uint64_t)wlo + BM_BITS;
                    j0 = mnext;
                    j1 = wave_first_at_least<NARROW>(a.col, b0 + j0, b1, whi) - b0;
                    mnext = j1;
                    if (j1 == j0) continue;   // same for the whole block: nothing to match here
                    // each tail cut to [wlo, whi); what lies above stays for the next windows
                    uint32_t cs_h[EH], cl_h[EH];
#pragma unroll
                    for (int h = 0; h < EH; ++h) {
                        uint32_t p = st_h[h];
                        const uint32_t e = p + len_h[h];
                        uint32_t e2 = p;
                        if (cv_h[h] < whi) {
                            // elements below wlo belong to windows without middle elements
                            if (cv_h[h] < wlo) p = first_at_least<NARROW>(a.col, p, e, wlo);
                            e2 = first_at_least<NARROW>(a.col, p, e, whi);
                            cv_h[h] = e2 < e ? (uint64_t)col_at<NARROW>(a.col, e2) : ~0ull;
                        }
                        cs_h[h] = p;
                        cl_h[h] = e2 - p;
                        st_h[h] = e2;
                        len_h[h] = e - e2;
                    }
                    nt = entry_table<false>(cs_h, cl_h, s_pref, s_base, s_cnt, S.scratch, nl, L);
                }
                for (uint32_t j = j0 + threadIdx.x; j < j1; j += IS_NT) {
                    const uint32_t x = a.col[b0 + j] - wlo;
                    if (x < BM_BITS) atomicOr(&bm[x >> 5], 1u << (x & 31u));
                }
                __syncthreads();
                // All tails of the tile form one flat item range [0, L); item q of
                // entry k lives at col[base[k] + q]. The range is cut into 64-item
                // windows, taken in chunks of WT_MAX windows: per chunk a table gives
                // the entry holding each window's first item, and wave w walks a
                // contiguous, 64-aligned quarter of the chunk in rounds of UNROLL
                // windows (one item per lane per window). A round runs in phases,
                // each over all UNROLL windows: read the windows' first entries from
                // the table; mark the entry starts inside each window (lane ln looks
                // at entry first + 1 + ln and marks its start offset in a per-wave
                // slot array); read the slots back as a ballot mask, so that a lane's
                // entry is first + (starts at or before its offset); issue the tail
                // loads, unconditional (lanes past the end read a valid address);
                // test the bitmap. Rounds that lie inside the long tails (placed
                // first) skip the marks: there an entry spans at least one window,
                // so one compare with the next entry's start gives a lane's entry.
                const uint32_t wv = (uint32_t)wave_id(), ln = (uint32_t)lane_id();
                const uint32_t Llong = s_pref[nl];   // items of the long tails: [0, Llong)
                for (uint32_t c0 = 0; c0 < L; c0 += WT_MAX * WAVE) {
                    const uint32_t c1 = L - c0 < WT_MAX * WAVE ? L : c0 + WT_MAX * WAVE;
                    const uint32_t nwc = (c1 - c0 + WAVE - 1) / WAVE;   // windows in this chunk
                    // window table: entry k covers items [pref[k], pref[k+1])
                    for (uint32_t k = threadIdx.x; k < nt; k += IS_NT) {
                        const uint32_t p0 = s_pref[k] > c0 ? s_pref[k] : c0;
                        const uint32_t p1 = s_pref[k + 1] < c1 ? s_pref[k + 1] : c1;
                        for (uint32_t w = (p0 - c0 + WAVE - 1) / WAVE; p0 < p1 && w * WAVE + c0 < p1; ++w)
                            s_wst[w] = (uint16_t)k;
                    }
                    __syncthreads();
                    const uint32_t span = (c1 - c0 + WAVE - 1) / WAVE;   // windows, split over the waves
                    const uint32_t q0 = c0 + WAVE * ((span * wv) / (IS_NT / WAVE));
                    const uint32_t qe = c0 + WAVE * ((span * (wv + 1)) / (IS_NT / WAVE));
                    const uint32_t q1 = qe < c1 ? qe : c1;
                    const uint32_t lim = Llong < q1 ? Llong : q1;   // rounds below lim see long tails only
                    for (uint32_t W = q0; W < q1; W += WAVE * UNROLL) {
                        uint32_t xs[UNROLL], ks[UNROLL], kj[UNROLL];
#pragma unroll
                        for (int j = 0; j < UNROLL; ++j) {   // same address in all lanes: broadcast
                            const uint32_t wi = (W - c0) / WAVE + (uint32_t)j;
                            kj[j] = s_wst[wi < nwc ? wi : nwc - 1u];
                        }
                        if (W + WAVE * UNROLL <= lim) {
                            // long tails only: an entry spans at least one window, so at most
                            // one entry starts inside a window; a lane's entry is the window's
                            // first entry, plus one at or after the next start
#pragma unroll
                            for (int j = 0; j < UNROLL; ++j) {
                                const uint32_t nx = s_pref[kj[j] + 1u];
                                ks[j] = kj[j] + (W + j * WAVE + ln >= nx ? 1u : 0u);
                            }
                            uint32_t ad[UNROLL];
#pragma unroll
                            for (int j = 0; j < UNROLL; ++j) ad[j] = s_base[ks[j]] + W + j * WAVE + ln;
#pragma unroll
                            for (int j = 0; j < UNROLL; ++j) xs[j] = col_at<NARROW>(a.col, ad[j]) - wlo;
                        } else {
                            // mark the starts (pref is strictly increasing, so the marked offsets
                            // are distinct and at least 1). Entries past the last one read
                            // pref[nt] = L: a start at or after item L moves only lanes whose
                            // items lie beyond q1 (unused).
                            uint32_t o[UNROLL];
    #pragma unroll
                            for (int j = 0; j < UNROLL; ++j) {
                                const uint32_t kk = kj[j] + 1u + ln;
                                o[j] = s_pref[kk < nt ? kk : nt] - (W + j * WAVE);
                            }
    #pragma unroll
                            for (int j = 0; j < UNROLL; ++j)
                                if (o[j] < 64u) s_flag[wv][j][o[j]] = 1;
                            // the lanes of the wave exchange marks through LDS: keep the
                            // mark / read / clear phases in program order
                            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                            uint32_t f[UNROLL];
    #pragma unroll
                            for (int j = 0; j < UNROLL; ++j) f[j] = s_flag[wv][j][ln];
    #pragma unroll
                            for (int j = 0; j < UNROLL; ++j) s_flag[wv][j][ln] = 0;   // each lane clears its own slot
                            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    #pragma unroll
                            for (int j = 0; j < UNROLL; ++j) {
                                const uint64_t M = __ballot(f[j] != 0u);
                                const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                                    (uint32_t)(M >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)M, 0u));
                                ks[j] = kj[j] + below + (f[j] != 0u ? 1u : 0u);
                            }
                            uint32_t ad[UNROLL];
    #pragma unroll
                            for (int j = 0; j < UNROLL; ++j) {
                                const uint32_t q = W + j * WAVE + ln;
                                const uint32_t sb = s_base[ks[j]];
                                ad[j] = q < q1 ? sb + q : b0;
                            }
    #pragma unroll
                            for (int j = 0; j < UNROLL; ++j) xs[j] = col_at<NARROW>(a.col, ad[j]);
    #pragma unroll
                            for (int j = 0; j < UNROLL; ++j)
                                xs[j] = (W + j * WAVE + ln < q1) ? xs[j] - wlo : 0xFFFFFFFFu;
                        }
                        // membership: bit positions past the window map to the spare
                        // always-zero word bm[BM_WORDS]
                        uint32_t wd[UNROLL];
#pragma unroll
                        for (int j = 0; j < UNROLL; ++j) wd[j] = bm[(xs[j] < BM_BITS ? xs[j] : BM_BITS) >> 5];
                        uint32_t hits = 0;
#pragma unroll
                        for (int j = 0; j < UNROLL; ++j) hits += __builtin_amdgcn_ubfe(wd[j], xs[j], 1u);
                        acc += hits;
                        if (!need_cnt) continue;
#pragma unroll
                        for (int j = 0; j < UNROLL; ++j) {
                            const uint32_t x = xs[j];
                            if ((wd[j] >> (x & 31u)) & 1u) {
                                const uint32_t slot = atomicAdd(&s_cnt[ks[j]], 1u);
                                if (MODE == BM_LIST) {
                                    const uint32_t e = s_base[ks[j]] + s_pref[ks[j]] - 1u;
                                    list_write(a, a.list_off[e] + slot, e, x + wlo);
                                }
                                if (GATHER) {
                                    const uint32_t w = x + wlo;
                                    if (a.support)   // edge (u, w): the tail element's own position
                                        atomicAdd(&a.support[s_base[ks[j]] + W + (uint32_t)j * WAVE + ln], 1u);
                                    if (nb <= (uint32_t)NV_MAX) {   // w's slot in N+(v), flushed per vertex
                                        uint32_t lo3 = 0, hi3 = nb - 1;
                                        while (lo3 < hi3) {
                                            const uint32_t mid = (lo3 + hi3) >> 1;
                                            if (s_nv[mid] < w) lo3 = mid + 1;
                                            else hi3 = mid;
                                        }
                                        atomicAdd(&s_wc[lo3], 1u);
                                    } else {
                                        hit_vertex(a, w);
                                        if (a.support) atomicAdd(&a.support[b0 + find_pos(a.col + b0, nb, w)], 1u);
                                    }
                                }
                            }
                        }
                    }
                    __syncthreads();   // the table is rebuilt for the next chunk
                }
                __syncthreads();
                for (uint32_t j = j0 + threadIdx.x; j < j1; j += IS_NT) {
                    const uint32_t x = a.col[b0 + j] - wlo;
                    if (x < BM_BITS) bm[x >> 5] = 0u;
                }
                __syncthreads();
            }
            if (GATHER && nb <= (uint32_t)NV_MAX) {
                for (uint32_t j = threadIdx.x; j < nb; j += IS_NT) {
                    const uint32_t c = s_wc[j];
                    if (!c) continue;
                    if (a.per_vertex) atomicAdd((unsigned long long*)&a.per_vertex[s_nv[j]], (unsigned long long)c);
                    if (a.support) atomicAdd(&a.support[b0 + j], c);
                }
            }
            if (need_cnt) {
                uint32_t seg_hits = 0;
                for (uint32_t k = threadIdx.x; k < nt; k += IS_NT) {
                    edge_done(a, s_base[k] + s_pref[k] - 1u, v, s_cnt[k], false);
                    seg_hits += s_cnt[k];
                }
                if (a.per_middle) {   // one update per vertex and tile
                    uint32_t total;
                    (void)block_exclusive_scan<IS_NT>(seg_hits, S.scratch, &total);
                    if (threadIdx.x == 0 && total)
                        atomicAdd((unsigned long long*)&a.per_middle[v], (unsigned long long)total);
                }
            }
            __syncthreads();
        }
    }
    block_partial(acc, partials);
}

// ------------------------------------------------------------------ shared helpers for edge-centric kernels
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

// Segment holding flattened in-edge q (largest sg with pref[sg] <= q).
__device__ __forceinline__ uint32_t find_seg(const Segs& S, uint32_t nseg, uint32_t q) {
    uint32_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (S.pref[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Elements X[q] (q = gl, gl + g, ...) of one list searched in the ascending
// list Y (ny > 0) by a group of g lanes: four elements per lane at a time, as
// four interleaved branch-free lower bounds (halving the range each step),
// so that every step issues four independent loads. Returns the matches; a
// match at X[q] = Y[p] is edge ex0 + q and edge ey0 + p.
__device__ __forceinline__ uint32_t search_list(const IsectArgs& a, const uint32_t* X, uint32_t nx,
                                                const uint32_t* Y, uint32_t ny, uint32_t g, uint32_t gl,
                                                uint32_t ex0, uint32_t ey0, uint32_t ein) {
    uint32_t c = 0;
    if (ny == 0) return 0;
    for (uint32_t q0 = gl; q0 < nx; q0 += 4u * g) {
        uint32_t xv[4], bs[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t q = q0 + (uint32_t)u * g;
            xv[u] = X[q < nx ? q : nx - 1u];
            bs[u] = 0;
        }
        for (uint32_t len = ny; len > 1;) {
            const uint32_t half = len >> 1;
            uint32_t yv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) yv[u] = Y[bs[u] + half];
#pragma unroll
            for (int u = 0; u < 4; ++u) bs[u] = yv[u] < xv[u] ? bs[u] + half : bs[u];
            len -= half;
        }
        // bs = last position below x (or 0): the lower bound is bs or bs + 1
        uint32_t y0[4], y1[4], lb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) y0[u] = Y[bs[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            lb[u] = bs[u] + (y0[u] < xv[u] ? 1u : 0u);
            y1[u] = Y[lb[u] < ny ? lb[u] : ny - 1u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t q = q0 + (uint32_t)u * g;
            if (q < nx && lb[u] < ny && y1[u] == xv[u]) {
                ++c;
                hit(a, xv[u], ex0 + q, ey0 + lb[u], ein);
            }
        }
    }
    return c;
}

// One in-edge by a group of g lanes: merge path (MERGE) or binary search.
// ea0, eb0: CSR positions of A[0] (the tail) and B[0] (N+(v)); the in-edge
// itself sits just before its tail, at ea0 - 1.
template <bool MERGE>
__device__ __forceinline__ uint32_t isect_edge(const IsectArgs& a, const uint32_t* A, uint32_t na, const uint32_t* B,
                                               uint32_t nb, uint32_t g, uint32_t gl, uint32_t ea0, uint32_t eb0) {
    uint32_t c = 0;
    if (MERGE) {
        // The lane's diagonal range [d0, d1) of the merge path consumes the A
        // elements [i0, i1); each A element is consumed by exactly one lane and
        // counts when it equals the B head at that point, which (B ascending)
        // is the first B element not below it. So the lane walks its A
        // elements, four loaded at a time, with a monotone cursor into B that
        // starts at the diagonal's B position d0 - i0.
        const uint32_t tot = na + nb;
        const uint32_t d0 = (uint32_t)(((uint64_t)tot * gl) / g);
        const uint32_t d1 = (uint32_t)(((uint64_t)tot * (gl + 1u)) / g);
        const uint32_t i0 = merge_split(A, na, B, nb, d0);
        const uint32_t i1 = merge_split(A, na, B, nb, d1);
        uint32_t j = d0 - i0;
        for (uint32_t i = i0; i < i1; i += 4u) {
            uint32_t av[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) av[u] = A[i + u < i1 ? i + u : i1 - 1u];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (i + u >= i1) break;
                while (j < nb && B[j] < av[u]) ++j;
                if (j < nb && B[j] == av[u]) {
                    ++c;
                    hit(a, av[u], ea0 + i + u, eb0 + j, ea0 - 1u);
                }
            }
        }
    } else if (na <= nb) {
        c = search_list(a, A, na, B, nb, g, gl, ea0, eb0, ea0 - 1u);   // tail elements searched in N+(v)
    } else {
        c = search_list(a, B, nb, A, na, g, gl, eb0, ea0, ea0 - 1u);   // N+(v) searched in the tail
    }
    return c;
}

template <bool MERGE>
__global__ __launch_bounds__(IS_NT, MERGE ? 7 : 6) void k_isect_edges(IsectArgs a, uint64_t* partials) {
    __shared__ uint32_t sb[STAGE_MAX];
    __shared__ uint32_t s_boff[SEG_MAX + 1];
    __shared__ Segs S;
    constexpr int KER = MERGE ? KER_MERGE : KER_BSEARCH;
    uint64_t acc = 0;
    __shared__ uint32_t s_tile;
    const uint32_t t_begin = a.ctrl->tile_begin[KER], t_end = a.ctrl->tile_begin[KER + 1];
    for (uint32_t t = t_begin + blockIdx.x; t < t_end; t = grab_tile(a.ctrl, KER, t_begin + gridDim.x, &s_tile)) {
        const uint32_t nseg = load_tile(a, t, S);
        const uint32_t v0 = S.v[0];
        // stage the N+(v) lists of all the tile's vertices back to back when they fit
        uint32_t dl = 0;
        if (threadIdx.x < nseg) dl = a.off[S.v[threadIdx.x] + 1] - a.off[S.v[threadIdx.x]];
        uint32_t TB;
        const uint32_t bex = block_exclusive_scan<IS_NT>(dl, S.scratch, &TB);
        if (threadIdx.x < nseg) s_boff[threadIdx.x] = bex;
        if (threadIdx.x == 0) s_boff[nseg] = TB;
        __syncthreads();
        const bool staged = TB <= (uint32_t)STAGE_MAX;
        if (staged) {
            for (uint32_t j = threadIdx.x; j < TB; j += IS_NT) {
                uint32_t lo2 = 0, hi2 = nseg - 1;   // segment holding list position j
                while (lo2 < hi2) {
                    const uint32_t mid = (lo2 + hi2 + 1) >> 1;
                    if (s_boff[mid] <= j) lo2 = mid;
                    else hi2 = mid - 1;
                }
                sb[j] = a.col[a.off[S.v[lo2]] + (j - s_boff[lo2])];
            }
        }
        __syncthreads();
        const uint32_t g = a.ctrl->group[a.vbucket[v0]];            // lanes per in-edge (power of 2)
        const uint32_t gi = threadIdx.x / g, gl = threadIdx.x % g;  // group index, lane in group
        const uint32_t ngroups = IS_NT / g;
        const uint32_t ne = S.pref[nseg];
        const uint32_t rounds = (ne + ngroups - 1) / ngroups;
        // each round's in-edge entry (tail start | end << 32) is loaded one round ahead,
        // so that its latency overlaps the intersection before it
        uint32_t sg_next = 0;
        uint64_t ent_next = 0;
        if (gi < ne) {
            sg_next = nseg == 1 ? 0u : find_seg(S, nseg, gi);
            ent_next = a.csc[S.e0[sg_next] + (gi - S.pref[sg_next])];
        }
        for (uint32_t r = 0; r < rounds; ++r) {
            const uint32_t q = r * ngroups + gi;
            const uint32_t sg = sg_next;
            const uint64_t ent = ent_next;
            const uint32_t qn = q + ngroups;
            if (qn < ne) {
                sg_next = nseg == 1 ? 0u : find_seg(S, nseg, qn);
                ent_next = a.csc[S.e0[sg_next] + (qn - S.pref[sg_next])];
            }
            uint32_t c = 0, e = 0, v = 0;
            if (q < ne) {
                v = S.v[sg];
                const uint32_t s = (uint32_t)ent, end = (uint32_t)(ent >> 32);
                e = s - 1u;
                const uint32_t nb = s_boff[sg + 1] - s_boff[sg];
                const uint32_t bo = a.off[v];
                // two call sites, so that each knows whether N+(v) is in LDS or in global memory
                if (staged) c = isect_edge<MERGE>(a, a.col + s, end - s, sb + s_boff[sg], nb, g, gl, s, bo);
                else c = isect_edge<MERGE>(a, a.col + s, end - s, a.col + bo, nb, g, gl, s, bo);
            }
            // reduce within the group of g lanes (g divides the wave)
            for (uint32_t o = g >> 1; o > 0; o >>= 1) c += __shfl_xor(c, (int)o, WAVE);
            if (q < ne && gl == 0) {
                acc += c;
                edge_done(a, e, v, c);
            }
        }
        __syncthreads();
    }
    block_partial(acc, partials);
}

// Sum of the per-block partial counts of all three kernels, in a fixed order.
__global__ __launch_bounds__(IS_NT) void k_reduce_total(const uint64_t* __restrict__ partials, uint32_t count,
                                                        Ctrl* ctrl) {
    uint64_t acc = 0;
    for (uint32_t i = threadIdx.x; i < count; i += IS_NT) acc += partials[i];
    block_partial(acc, &ctrl->total);
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

// Persistent grids: as many blocks as the CUs hold at once (LDS and registers
// decide), so that no block starts late and stretches the tail.
static int resident_blocks(const void* fn) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, IS_NT, 0) != hipSuccess || b <= 0) b = 1;
    return b;
}

static int bitmap_mode(const IsectArgs& a) {
    if (a.clip) return BM_CLIP;   // whole-row tails: counts only
    if (a.list_out) return BM_LIST;
    if (a.per_vertex || a.support) return BM_GATHER;
    if (a.per_edge || a.per_middle) return BM_ENTRY;
    return BM_COUNT;
}

static const void* bitmap_fn(int mode, bool narrow) {
    switch (mode) {
        case BM_LIST: return narrow ? (const void*)k_isect_bitmap<BM_LIST, true>
                                    : (const void*)k_isect_bitmap<BM_LIST, false>;
        case BM_GATHER: return narrow ? (const void*)k_isect_bitmap<BM_GATHER, true>
                                      : (const void*)k_isect_bitmap<BM_GATHER, false>;
        case BM_ENTRY: return narrow ? (const void*)k_isect_bitmap<BM_ENTRY, true>
                                     : (const void*)k_isect_bitmap<BM_ENTRY, false>;
        case BM_CLIP: return narrow ? (const void*)k_isect_bitmap<BM_CLIP, true>
                                    : (const void*)k_isect_bitmap<BM_CLIP, false>;
        default: return narrow ? (const void*)k_isect_bitmap<BM_COUNT, true>
                               : (const void*)k_isect_bitmap<BM_COUNT, false>;
    }
}

int isect_blocks_per_cu(int ker, int mode) {
    static int cache[NKERNEL][BM_NMODE] = {};
    int& c = cache[ker][mode];
    if (!c) {
        const void* fn = ker == KER_MERGE     ? (const void*)k_isect_edges<true>
                         : ker == KER_BSEARCH ? (const void*)k_isect_edges<false>
                                              : bitmap_fn(mode, true);
        c = resident_blocks(fn);
    }
    return c;
}

size_t isect_partials_bytes() { return sizeof(uint64_t) * NKERNEL * PARTIALS_PER_KERNEL; }

void launch_isect(int ker, const IsectArgs& a, int grid, uint64_t* partials, hipStream_t s) {
    const int mode = ker == KER_BITMAP ? bitmap_mode(a) : 0;
    if (grid <= 0) grid = num_cu() * isect_blocks_per_cu(ker, mode);
    if (grid > PARTIALS_PER_KERNEL) grid = PARTIALS_PER_KERNEL;
    uint64_t* p = partials + (size_t)ker * PARTIALS_PER_KERNEL;
    fill_u64(p, 0ull, PARTIALS_PER_KERNEL, s);
    switch (ker) {
        case KER_MERGE: hipLaunchKernelGGL(k_isect_edges<true>, dim3(grid), dim3(IS_NT), 0, s, a, p); break;
        case KER_BSEARCH: hipLaunchKernelGGL(k_isect_edges<false>, dim3(grid), dim3(IS_NT), 0, s, a, p); break;
        default: {
            const bool nw = a.col_narrow != 0;
            if (mode == BM_LIST) {
                if (nw) hipLaunchKernelGGL((k_isect_bitmap<BM_LIST, true>), dim3(grid), dim3(IS_NT), 0, s, a, p);
                else hipLaunchKernelGGL((k_isect_bitmap<BM_LIST, false>), dim3(grid), dim3(IS_NT), 0, s, a, p);
            } else if (mode == BM_GATHER) {
                if (nw) hipLaunchKernelGGL((k_isect_bitmap<BM_GATHER, true>), dim3(grid), dim3(IS_NT), 0, s, a, p);
                else hipLaunchKernelGGL((k_isect_bitmap<BM_GATHER, false>), dim3(grid), dim3(IS_NT), 0, s, a, p);
            } else if (mode == BM_CLIP) {
                if (nw) hipLaunchKernelGGL((k_isect_bitmap<BM_CLIP, true>), dim3(grid), dim3(IS_NT), 0, s, a, p);
                else hipLaunchKernelGGL((k_isect_bitmap<BM_CLIP, false>), dim3(grid), dim3(IS_NT), 0, s, a, p);
            } else if (mode == BM_ENTRY) {
                if (nw) hipLaunchKernelGGL((k_isect_bitmap<BM_ENTRY, true>), dim3(grid), dim3(IS_NT), 0, s, a, p);
                else hipLaunchKernelGGL((k_isect_bitmap<BM_ENTRY, false>), dim3(grid), dim3(IS_NT), 0, s, a, p);
            } else {
                if (nw) hipLaunchKernelGGL((k_isect_bitmap<BM_COUNT, true>), dim3(grid), dim3(IS_NT), 0, s, a, p);
                else hipLaunchKernelGGL((k_isect_bitmap<BM_COUNT, false>), dim3(grid), dim3(IS_NT), 0, s, a, p);
            }
            break;
        }
    }
}

void launch_reduce_total(uint64_t* partials, Ctrl* ctrl, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_total, dim3(1), dim3(IS_NT), 0, s, partials, (uint32_t)(NKERNEL * PARTIALS_PER_KERNEL),
                       ctrl);
}

}  // namespace tcx
