// Internal host-side launchers shared between the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tcx {

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }


// Global digit counts for the passes of a later sort, taken by a kernel that
// reads every key anyway, so that those passes look back with no histogram
// pass of their own: digit q (bits [shift + q * bits, min(that + bits, hi)),
// q < n <= LB_MAX_MORE), count of value d in tot[q * 256 + d].
constexpr int LB_MAX_MORE = 3;
struct MoreTot {
    uint32_t* tot;
    int n, shift, bits, hi;
};

// ---- prims.hip
void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
void fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s);
size_t scan_temp_bytes();
void scan_exclusive_sum_u32(const uint32_t* in, uint32_t* out, size_t len, void* temp, hipStream_t s);
void scan_inclusive_max_u32(const uint32_t* in, uint32_t* out, size_t len, void* temp, hipStream_t s);
void scan_exclusive_sum_u64(const uint64_t* in, uint64_t* out, size_t len, void* temp, hipStream_t s);
size_t radix_temp_bytes(size_t cap);
// Stable LSD sort of keys on bits [bit_lo, bit_hi) in ceil(bits / 8) passes of
// (nearly) equal digit widths, optional uint32 payload. The count is read from
// d_count on the device (nullptr: cap). With first_counted, the kernel that
// wrote the keys has already filled the first pass's per-tile digit counts
// (radix_first_counts, see TileCounts). With first_unstable, the first pass
// only partitions (ranks by LDS atomics): the keys come out sorted on
// [bit_lo, bit_hi), but keys equal on those bits in no particular order, so
// use it where that order is free (the whole key sorted, or a grouping).
// 64-bit sorts of 2^26 keys or more without payload take their passes after the first
// in one kernel each (decoupled look-back, no histogram pass); a wait there
// that runs out sets bit 1 of *err (nullptr: radix_err_word(temp, cap)). With
// totals_given, an earlier kernel has counted radix_sort_totals(...) and every
// pass looks back. Returns 1 when the sorted data ended up in the *_alt buffers.
int radix_sort_u64(uint64_t* keys, uint64_t* keys_alt, uint32_t* vals, uint32_t* vals_alt, const uint32_t* d_count,
                   size_t cap, int bit_lo, int bit_hi, void* temp, hipStream_t s, bool first_counted = false,
                   bool first_unstable = false, uint32_t* err = nullptr, bool totals_given = false);
int radix_sort_u32(uint32_t* keys, uint32_t* keys_alt, uint32_t* vals, uint32_t* vals_alt, const uint32_t* d_count,
                   size_t cap, int bit_lo, int bit_hi, void* temp, hipStream_t s, bool first_counted = false,
                   bool first_unstable = false, uint32_t* err = nullptr);
// The word in a sort's temporary (cap keys) where its look-back passes report
// a wait that ran out (bit 1).
uint32_t* radix_err_word(void* temp, size_t cap);
// The counts a sort of cap keys of key_bytes bytes on [bit_lo, bit_hi), in
// temporary temp, takes with totals_given; n == 0 when that sort cannot look
// back on all its passes (then nothing needs counting).
MoreTot radix_sort_totals(void* temp, size_t cap, int key_bytes, int bit_lo, int bit_hi);


// Keys per tile of a sort of cap keys of key_bytes bytes (2048, 4096 or 8192;
// a multiple of 2048).
uint32_t radix_tile_keys(size_t cap, int key_bytes);
// What a radix pass does to each key as it loads it (the orientation's passes):
//   RX_NONE      nothing;
//   RX_RANK_LOW  the low 32 bits, a vertex id a, become rank[a] (0xFFFFFFFF for a
//                outside [0, n)); the pass's digit must lie in the high half;
//   RX_ORIENT    (b << 32 | rank of a) becomes the oriented pair key
//                (min rank << nb | max rank), or `sentinel` for a pair with an
//                invalid id or a loop (equal ranks); digits come from the result.
enum { RX_NONE = 0, RX_RANK_LOW = 1, RX_ORIENT = 2 };
struct RadixXf {
    int kind;
    const uint32_t* rank;
    int32_t n;   // >= 1 for RX_RANK_LOW and RX_ORIENT (lanes past the end read rank[0])
    int nb;
    uint64_t sentinel;
};
// One radix pass of 64-bit keys on bits [shift, shift + bits), bits <= 8, from
// kin to kout (the two must differ), each key transformed as `xf` says.
// counted: the per-tile digit counts, already taken by an earlier kernel
// (counts[d * ntiles + tile], tiles of radix_tile_keys(cap, 8) keys; the pass
// turns them into offsets in place); nullptr: the pass counts them itself.
// stable: keys of equal digit keep their input order; otherwise their order
// is arbitrary (a partition).
// more (n > 0): the pass's histogram kernel also takes these global counts
// (zeroing them first); ignored when the counts come from `counted`.
// lb_tot: the global counts of this pass's digit (256), taken by an earlier
// kernel; with 8192-key tiles (2^26 keys or more) the pass then runs as one
// look-back kernel with no histogram (a wait that runs out sets bit 1 of *err;
// nullptr: radix_err_word(temp, cap)); otherwise it is ignored.
void radix_pass_u64(const uint64_t* kin, uint64_t* kout, size_t cap, int shift, int bits, const RadixXf& xf,
                    void* temp, hipStream_t s, uint32_t* counted, bool stable,
                    const MoreTot& more = MoreTot{nullptr, 0, 0, 0, 0}, const uint32_t* lb_tot = nullptr,
                    uint32_t* err = nullptr);
// Digit width of each pass of a sort over `bits` bits (equal widths, at most 8).
int radix_digit_width(int bits);
struct RadixDigit {
    int shift;
    uint32_t mask;
};
// The first digit of a sort over [bit_lo, bit_hi).
RadixDigit radix_first_digit(int bit_lo, int bit_hi);
// The first pass's count table inside temp: counts[d * ntiles + tile], 256
// rows, ntiles = ceil(cap / radix_tile_keys(cap, key bytes)).
uint32_t* radix_first_counts(void* temp);

// ---- runsort.hip
// Keys grouped by key >> shift (ascending; 1 <= shift <= 32) are sorted by the
// whole key inside each run of equal high bits, in place; keys 16-byte aligned,
// tmp as many keys as keys (scratch for runs longer than 4096). With skip, a
// run whose first key is skip_key (it must hold only that key) is left alone.
// With kept non-null, kept[p / chunk] += the keys at positions p that differ
// from the key before them, over the runs sorted (kept must start at zero).
void sort_runs_u64(uint64_t* keys, uint64_t* tmp, size_t len, int shift, bool skip, uint64_t skip_key,
                   uint32_t* kept, uint32_t chunk, hipStream_t s);

// ---- control block shared by all stages (device memory, zeroed per call)
constexpr int NBUCKET = 256;          // degree-pair buckets; 255 = no work
constexpr int BUCKET_NONE = 255;
constexpr int NKERNEL = 3;            // 0 merge-path, 1 binary search, 2 LDS bitmap
constexpr int BM_WINDOW_LOG2 = 17;    // ids covered by one LDS bitmap window
enum { KER_MERGE = 0, KER_BSEARCH = 1, KER_BITMAP = 2 };

struct Ctrl {
    uint64_t total;                   // triangle count
    uint32_t err;                     // bit 0: vertex id out of range
    uint32_t m_valid;                 // oriented, loop-free pairs before de-duplication
    uint32_t m;                       // unique oriented edges
    uint32_t ntiles;                  // tiles emitted
    uint32_t tile_begin[NKERNEL + 1]; // tile range per intersection kernel
    uint32_t m_active;                // in-edges with work (non-empty tail, d+(v) > 0)
    uint32_t pad0;
    uint32_t tile_next[NKERNEL + 1];  // per intersection kernel: tiles handed out after the first per block
                                      // (zeroed before every launch)
    uint64_t wedges;                  // sum over v of C(d(v), 2), simple degree (clustering runs only)
    uint32_t bstart[NBUCKET];         // first / one-past-last position of each bucket
    uint32_t bend[NBUCKET];           //   in the (kernel, bucket)-ordered vertex list
    uint32_t bucket_nv[NBUCKET];      // vertices per bucket
    uint64_t bucket_in[NBUCKET];      // sum of in-degrees (non-empty tails) per bucket
    uint64_t bucket_out[NBUCKET];     // sum of out-degrees per bucket
    uint64_t bucket_work[NBUCKET];    // sum of d-(v) * d+(v) per bucket
    uint64_t bucket_win[NBUCKET];     // sum of the bitmap windows spanned by the middle lists per bucket
    uint8_t choice[NBUCKET];          // kernel per bucket
    uint8_t slot[NBUCKET];            // bucket -> position in (kernel, bucket) order
    uint16_t chunk[NBUCKET];          // in-edges per tile, per bucket
    uint8_t group[NBUCKET];           // lanes per in-edge for the edge-centric kernels
    uint8_t pad1[NBUCKET];
    float features[NBUCKET][6];       // selector-network input per bucket
};

// Tiles, 16 bytes each, decoded without further dependent loads where
// possible: {v, first in-edge, in-edge count, 0} for a chunk of one vertex's
// in-edges; {i, g, 0, TILE_MULTI} for the g vertices starting at position i of
// the ordered vertex list (whole in-edge lists).
constexpr uint32_t TILE_MULTI = 0x80000000u;
constexpr int SEG_MAX = 256;          // vertices per multi-vertex tile
constexpr int SEG_MAX_BITMAP = 32;    // vertices per multi-vertex tile of the bitmap kernel

}  // namespace tcx
