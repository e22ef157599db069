/*
 * tc.h - exact triangle counting on one MI355X (gfx950), C ABI.
 *
 * The library implements the intersection-based formulation of exact
 * triangle counting (Wang, Wang, Yang, Owens, "A Comparative Study on Exact
 * Triangle Counting Algorithms on the GPU", HPGP 2016; Section 3.2 and
 * Algorithm 2, with the edge-list optimisations of Section 4.2):
 *   1. canonicalise the input pairs, drop self-loops and repeats;
 *   2. keep every undirected edge once, directed from the lower to the higher
 *      vertex in (degree, id) order (the degree filter of Section 4.2);
 *   3. build the filtered CSR (the "induced subgraph" of Section 4.2) with a
 *      device radix sort;
 *   4. intersect the two out-neighbour lists of every kept edge; the sizes
 *      sum to the triangle count (Algorithm 2).
 *
 * Conventions for every entry point
 *   - Pointers prefixed d_ are device pointers on the context's device;
 *     h_ pointers are host pointers. The caller owns every buffer.
 *   - Inputs are never modified. The library allocates no device memory per
 *     call: scratch space is the caller's workspace, sized by
 *     tc_workspace_size().
 *   - Edge lists are int32 pairs, row-major [num_edges][2], in any order and
 *     direction. Self-loops and repeated pairs are accepted and ignored.
 *   - Every call returns a status. Host-detectable errors (null pointers,
 *     negative sizes, small workspace) return before any launch. A vertex id
 *     outside [0, num_vertices) is detected on the device and reported as
 *     TC_ERR_VERTEX_RANGE after the stream is synchronised; outputs are
 *     then left unspecified (host outputs are not written).
 *   - Calls on one context are serialised on its stream; a context is not
 *     thread-safe.
 *   - Limits: num_vertices < 2^31, num_edges < 2^31 - 2^20 (TC_ERR_UNSUPPORTED
 *     beyond).
 */
#ifndef TC_MI355X_TC_H
#define TC_MI355X_TC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tc_status {
    TC_OK = 0,
    TC_ERR_INVALID_ARG = 1,   /* null pointer, negative size, bad option */
    TC_ERR_VERTEX_RANGE = 2,  /* an edge names a vertex outside [0, num_vertices) */
    TC_ERR_WORKSPACE = 3,     /* workspace smaller than tc_workspace_size() */
    TC_ERR_HIP = 4,           /* a HIP runtime call failed; see tc_last_error() */
    TC_ERR_UNSUPPORTED = 5    /* size beyond the documented limits */
} tc_status;

/* Which intersection strategy handles each degree-pair bucket. Every choice
 * gives the same exact counts; only the time differs. */
typedef enum tc_select {
    TC_SELECT_HEURISTIC = 0,  /* fixed thresholds on the bucket's degrees */
    TC_SELECT_LEARNED = 1,    /* the context's trained selector network */
    TC_FORCE_MERGE = 2,       /* merge-path for every bucket */
    TC_FORCE_BSEARCH = 3,     /* binary search for every bucket */
    TC_FORCE_BITMAP = 4       /* LDS bitmap for every bucket */
} tc_select;

/* Option flags. */
#define TC_F_STAGE_TIMING 0x1u  /* record per-stage times (tc_stage_times) */
#define TC_F_NO_GRAPH 0x2u      /* batched counting: launch directly instead of replaying a captured graph */

typedef struct tc_options {
    int32_t select;           /* a tc_select value */
    uint32_t flags;           /* TC_F_* bits */
    int32_t reserved[6];      /* must be zero */
} tc_options;

typedef struct tc_ctx tc_ctx;

/* Create a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = the device's null stream). */
tc_status tc_create(tc_ctx** ctx, int device, void* hip_stream);
tc_status tc_destroy(tc_ctx* ctx);

/* Bytes of device workspace that a call with these sizes needs. The value
 * depends only on the arguments, so one workspace serves every call with
 * equal or smaller sizes. */
tc_status tc_workspace_size(int64_t num_edges, int32_t num_vertices, const tc_options* opts, size_t* bytes);

/*
 * Exact triangle count T of the undirected simple graph denoted by the edge
 * list (Algorithm 2: the sum of the per-edge intersection sizes).
 *   h_count       out: T (host).
 *   d_per_vertex  out, optional (NULL): uint64[num_vertices], t[v] = number
 *                 of triangles containing v (original ids).
 */
tc_status tc_count_triangles(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                             void* d_workspace, size_t workspace_bytes, const tc_options* opts,
                             uint64_t* h_count, uint64_t* d_per_vertex);

/*
 * tc_count_triangles without any host synchronisation: the work is queued on
 * the context's stream and the call returns. On completion
 *   d_result[0] = T, d_result[1] = 0, or TC_ERR_VERTEX_RANGE when an id lies
 *   outside [0, num_vertices), or TC_ERR_HIP when an internal bound check
 *   failed (in both cases d_result[0] and d_per_vertex are meaningless).
 * d_result: uint64[2], device memory, 8-byte aligned. Host-detectable errors
 * return before anything is queued. The workspace and outputs must stay
 * untouched until the stream reaches the end of the call; calls queued on one
 * stream may share a workspace. TC_F_STAGE_TIMING is rejected here.
 */
tc_status tc_count_triangles_async(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                                   void* d_workspace, size_t workspace_bytes, const tc_options* opts,
                                   uint64_t* d_result, uint64_t* d_per_vertex);

/*
 * Triangle-based graph measures named in Section 1 and, as a small extension
 * of the method, at the end of Section 5: the local clustering coefficient
 * (Watts and Strogatz) and the transitivity ratio.
 *   d_coeff         out: double[num_vertices] (original ids),
 *                   C(v) = t[v] / C(d(v), 2), with d(v) the degree in the
 *                   simple graph; 0 when d(v) < 2.
 *   d_per_vertex    out, optional (NULL): uint64 t[v] as in tc_count_triangles.
 *   h_count         out: T.
 *   h_wedges        out: number of wedges (paths of two edges), sum of C(d(v), 2).
 *   h_transitivity  out: 3 T / wedges (0 without wedges).
 * Both ratios are one correctly rounded double division of exact integers
 * (the integers converted to double first).
 */
tc_status tc_clustering(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                        void* d_workspace, size_t workspace_bytes, const tc_options* opts, double* d_coeff,
                        uint64_t* d_per_vertex, uint64_t* h_count, uint64_t* h_wedges, double* h_transitivity);

/*
 * Per-edge intersection sizes (the per-edge list that Algorithm 2 sums). For
 * each kept edge (u -> v), u before v in (degree, id) order, writes
 *   d_out_edges[i] = {u, v} (original ids) and
 *   d_out_counts[i] = |N+(u) intersected with N+(v)|, the triangles whose two
 *   lowest vertices are u and v.
 * Edges come in CSR order (by rank of u, then rank of v). Capacity of both
 * outputs: num_edges entries. h_num_out receives the number m of kept edges;
 * h_count receives T (= sum of the counts).
 */
tc_status tc_edge_counts(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                         void* d_workspace, size_t workspace_bytes, const tc_options* opts,
                         int32_t* d_out_edges, uint32_t* d_out_counts, int64_t* h_num_out, uint64_t* h_count);

/*
 * Triangle listing (Section 1: the counting algorithms also enumerate the
 * triangles they count). Writes the T triangles to d_out as int32 triples of
 * original ids (u, v, w), u before v before w in (degree, id) order: the
 * triangles of each kept edge (u, v) are contiguous, edges in CSR order,
 * the order inside an edge unspecified. capacity = triples d_out holds.
 * h_count receives T in every case; when T > capacity the call returns
 * TC_ERR_WORKSPACE and writes nothing to d_out (allocate T triples and call
 * again). The workspace must hold tc_list_workspace_size() bytes.
 */
tc_status tc_list_workspace_size(int64_t num_edges, int32_t num_vertices, const tc_options* opts, size_t* bytes);
tc_status tc_list_triangles(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                            void* d_workspace, size_t workspace_bytes, const tc_options* opts, int32_t* d_out,
                            int64_t capacity, uint64_t* h_count);

/*
 * Edge support: for each kept edge, the number of triangles that contain it
 * (Section 1: the triangles the counting algorithms enumerate are the input
 * of k-truss decomposition). Same output layout as tc_edge_counts:
 * d_out_edges[i] = {u, v} (original ids, u before v in (degree, id) order) and
 * d_out_support[i] (uint32), CSR order, capacity num_edges entries each;
 * h_num_out = m, h_count = T (the supports sum to 3T).
 */
tc_status tc_edge_support(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                          void* d_workspace, size_t workspace_bytes, const tc_options* opts,
                          int32_t* d_out_edges, uint32_t* d_out_support, int64_t* h_num_out, uint64_t* h_count);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * count as tc_count_triangles_async, with the workspace taken from a fixed
 * scratch array that the library holds on each GPU for the life of the
 * process (TC_NOALLOC_SCRATCH_BYTES per GPU; its device address is looked up
 * once per device by tc_create). The call allocates nothing; inputs and
 * outputs are the caller's, as for tc_count_triangles_async (d_result uint64[2]
 * device, d_per_vertex optional). A graph whose tc_workspace_size exceeds
 * TC_NOALLOC_SCRATCH_BYTES is rejected with TC_ERR_WORKSPACE before anything
 * is queued. Every call on one GPU uses the same scratch: calls queued on one
 * stream run one after another, but calls that overlap on one GPU (other
 * streams, other contexts of that device) race and give undefined results.
 */
#define TC_NOALLOC_SCRATCH_BYTES (64u << 20)
tc_status tc_count_triangles_noalloc(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                                    const tc_options* opts, uint64_t* d_result, uint64_t* d_per_vertex);

/*
 * The paper's other formulations of the same count, for comparison with the
 * filtered one above. All run the same canonicalisation, degree order and
 * filtered CSR, then stream, for every kept edge (u -> v), one list of u
 * against one list of v through the same three intersection kernels (counts
 * only, no per-edge or per-vertex outputs):
 *   TC_FORM_FILTERED     N+(u) against N+(v): T (Section 4.2,
 *                        "tc-intersection-filtered"; same as
 *                        tc_count_triangles).
 *   TC_FORM_FULL         N(u) against N(v), the whole neighbour lists over
 *                        the half-filtered edge list (Section 4.2 without the
 *                        induced subgraph, "tc-intersection-full" of the
 *                        speedup figure of Section 5): each triangle is found
 *                        at its three edges, so the sum is 3T.
 *   TC_FORM_MATRIX       Algorithm 3 with the rows in (degree, id) order:
 *                        C = A o (L U) and T = (1/2) sum C, where row v of C
 *                        collects, over the rows u of L(v, :) (the in-
 *                        neighbours of v), the U row of u (N+(u)) masked by
 *                        the A row of v (N(v)); B = L U is never formed.
 *                        The sum is sum C = 2T.
 *   TC_FORM_MATRIX_UPPER the same with the mask cut to the upper triangle
 *                        (Section 3.3, first optimisation of the matrix
 *                        implementation): N+(u) against N+(v), sum T.
 * h_count receives T; h_sum (optional, may be NULL) the sum of the hits
 * before the division (3T, 2T or T). A sum that the multiple does not divide
 * is reported as TC_ERR_HIP (internal bound violated). The workspace must
 * hold tc_formulation_workspace_size() bytes (the full and matrix forms add
 * the symmetric adjacency: 4 (n + 1) + 8 num_edges bytes, rounded up).
 * Selection modes as for tc_count_triangles.
 */
typedef enum tc_formulation {
    TC_FORM_FILTERED = 0,
    TC_FORM_FULL = 1,
    TC_FORM_MATRIX = 2,
    TC_FORM_MATRIX_UPPER = 3
} tc_formulation;

tc_status tc_formulation_workspace_size(int64_t num_edges, int32_t num_vertices, const tc_options* opts,
                                        int formulation, size_t* bytes);
tc_status tc_count_triangles_formulation(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges,
                                         int32_t num_vertices, void* d_workspace, size_t workspace_bytes,
                                         const tc_options* opts, int formulation, uint64_t* h_count,
                                         uint64_t* h_sum);

/*
 * Batched counting of many graphs in one pass (not in the paper; its small-
 * graph overhead remark in Section 5 motivates it). Graph g's pairs are
 * d_edges[h_edge_offsets[g] .. h_edge_offsets[g+1]) with graph-local ids in
 * [0, h_num_vertices[g]). The graphs are counted as one disjoint union:
 * every triangle lies inside one graph, and each is attributed to its graph
 * through its middle vertex, so h_counts[g] (host, uint64) is exact.
 * By default the whole device work of a call is captured once as a HIP graph
 * and replayed on later calls with the same sizes, edge pointer, workspace
 * and selection mode (TC_F_NO_GRAPH launches directly). If the context's
 * stream is the null stream, the work runs on a stream owned by the context.
 * Workspace: tc_batch_workspace_size(total pairs, total vertices, graphs).
 * An id outside its own graph's range yields TC_ERR_VERTEX_RANGE.
 */
tc_status tc_batch_workspace_size(int64_t total_edges, int64_t total_vertices, int32_t num_graphs,
                                  const tc_options* opts, size_t* bytes);
tc_status tc_count_triangles_batch(tc_ctx* ctx, const int32_t* d_edges, const int64_t* h_edge_offsets,
                                   const int32_t* h_num_vertices, int32_t num_graphs, void* d_workspace,
                                   size_t workspace_bytes, const tc_options* opts, uint64_t* h_counts);

/*
 * Tile shapes per degree-pair bucket (the autotuner's output): h_chunk[256]
 * in-edges per tile (16..2048, at most 512 for buckets the bitmap strategy
 * serves; values outside are clamped; 0 = default), h_group[256] lanes per
 * in-edge for merge path and binary search (power of two 1..64; 0 = default).
 * NULL resets to the defaults. Shapes change speed only, never counts.
 */
tc_status tc_set_tile_shapes(tc_ctx* ctx, const uint16_t* h_chunk, const uint8_t* h_group);

/*
 * The filtered CSR of Section 4.2 ("induced subgraph"): vertices relabelled
 * by rank in (degree, id) order, each undirected edge kept once from the
 * lower to the higher rank, rows ascending.
 *   d_rank     out: int32[num_vertices], rank of each original vertex.
 *   d_offsets  out: int64[num_vertices + 1] row offsets over ranks.
 *   d_col      out: int32[num_edges] capacity, column ranks.
 *   h_num_out  out: number m of kept edges.
 */
tc_status tc_build_csr(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                       void* d_workspace, size_t workspace_bytes, const tc_options* opts, int32_t* d_rank,
                       int64_t* d_offsets, int32_t* d_col, int64_t* h_num_out);

/*
 * The library's device radix sort (the CSR builder of step 3), exposed for
 * reuse: stable ascending sort of `count` uint64 keys on bits [bit_lo,
 * bit_hi), 8 bits per pass. d_keys holds the input and receives the result;
 * d_keys_alt is caller scratch of the same size. Workspace: at least
 * tc_radix_sort_workspace_size(count) bytes. From 2^26 keys, sorts of two to
 * four passes take the passes after the first in one kernel each, whose tiles
 * wait (boundedly) for the tiles before them; TC_ERR_HIP if such a wait ever
 * runs out (an internal bound, not a property of the keys).
 */
size_t tc_radix_sort_workspace_size(int64_t count);
tc_status tc_radix_sort_u64(tc_ctx* ctx, uint64_t* d_keys, uint64_t* d_keys_alt, int64_t count, int32_t bit_lo,
                            int32_t bit_hi, void* d_workspace, size_t workspace_bytes);

/*
 * One radix pass of the CSR builder (step 3) that only partitions: the count
 * uint64 keys of d_in are written to d_out grouped by their digit
 * (key >> shift) & (2^bits - 1), digits ascending, keys of one digit in no
 * particular order (ranks come from atomics, so the order can change from
 * call to call). It is the form the builder uses where the order inside a
 * digit is free: the first pass of a sort whose equal keys are identical or
 * re-sorted later, and the grouping passes.
 *   d_in, d_out  count uint64 each, device, distinct buffers.
 *   shift, bits  0 <= shift, 1 <= bits <= 8, shift + bits <= 64.
 *   d_workspace  at least tc_radix_sort_workspace_size(count) bytes.
 * Errors: TC_ERR_INVALID_ARG (null or equal pointers, bad shift or bits),
 * TC_ERR_UNSUPPORTED (count >= 2^31), TC_ERR_WORKSPACE; the call synchronises
 * its stream.
 */
tc_status tc_radix_partition_u64(tc_ctx* ctx, const uint64_t* d_in, uint64_t* d_out, int64_t count, int32_t shift,
                                 int32_t bits, void* d_workspace, size_t workspace_bytes);

/*
 * The second half of the CSR builder's pair sort (step 3), exposed for reuse:
 * the keys, already grouped by their high bits (key >> shift, runs of equal
 * high bits in ascending order), are sorted by the whole key inside every run,
 * in place, so a pair list sorted by row leaves with each row sorted by column
 * (the sorted out-lists of Section 3.2). Runs of up to 64 keys are sorted
 * together by a network across a wave, up to 2048 by one wave's registers, up
 * to 4096 by a whole block, longer ones by a whole block's radix passes in
 * d_tmp. Any key order is safe (runs are the maximal stretches of equal high
 * bits); only grouped input yields a sorted array.
 *   d_keys  count uint64 keys, 16-byte aligned, device; sorted in place.
 *   d_tmp   caller scratch of count uint64, device (runs longer than 4096).
 *   shift   1..32.
 * Errors: TC_ERR_INVALID_ARG (null or misaligned pointer, bad shift or count),
 * TC_ERR_UNSUPPORTED (count >= 2^31); the call synchronises its stream.
 */
tc_status tc_sort_runs_u64(tc_ctx* ctx, uint64_t* d_keys, uint64_t* d_tmp, int64_t count, int32_t shift);

/*
 * Work statistics of the last successful counting call on the context.
 * Buckets are the degree-pair classes of the dynamic grouping (Section 4.2):
 * for a middle vertex v with d_in in-edges whose tail is non-empty and
 * d_out = |N+(v)|, bucket = 16 * min(14, floor(log2 d_in)) + min(15,
 * floor(log2 d_out)); bucket 255 holds the vertices with no work.
 */
typedef struct tc_stats {
    uint64_t num_edges_kept;          /* m: unique undirected edges */
    uint64_t num_pairs_valid;         /* loop-free in-range input pairs */
    uint32_t num_tiles;               /* intersection tiles */
    uint32_t tile_begin[4];           /* tile range per strategy: merge, bsearch, bitmap */
    uint32_t bucket_vertices[256];
    uint64_t bucket_in_edges[256];
    uint64_t bucket_out_edges[256];
    uint64_t bucket_work[256];        /* sum over v of d_in(v) * d_out(v) */
    uint8_t bucket_kernel[256];       /* 0 merge, 1 bsearch, 2 bitmap */
    uint16_t bucket_chunk[256];       /* in-edges per tile */
    uint8_t bucket_group[256];        /* lanes per in-edge (merge, bsearch) */
} tc_stats;

tc_status tc_last_stats(const tc_ctx* ctx, tc_stats* out);

/*
 * Kernel selection per bucket by a learned network. The paper divides the
 * edge list into small- and large-list groups with a hand-chosen threshold
 * and proposes a third, one-large-one-small kernel (Section 4.2 and the
 * intersection summary of Section 5); here a small network picks among the
 * three strategies per degree-pair bucket, and the fixed thresholds remain
 * the fallback. Counts never depend on the choice.
 *
 * Network: 6 features -> 32 -> 32 -> 3 logits (ReLU), bfloat16 weights
 * rounded from a float32 master copy, float32 biases and accumulation.
 * Parameter vector (float32, TC_SELECTOR_NUM_PARAMS entries, in order):
 * W1 [32][6], b1 [32], W2 [32][32], b2 [32], W3 [3][32], b3 [3]; logit 0 is
 * merge path, 1 binary search, 2 LDS bitmap.
 * Features of bucket b (float32): floor(log2 d_in)/14, floor(log2 d_out)/15,
 * log2(1+windows)/32, log2(1+in-edges)/32, log2(1+out-edges)/32,
 * log2(1+sum d_in*d_out)/48, where windows = sum over the bucket's vertices v
 * of the 2^17-id LDS-bitmap windows spanned by the middle list of v (from its
 * first element rounded down to a multiple of 32 to its last).
 */
#define TC_SELECTOR_NUM_PARAMS 1379
#define TC_SELECTOR_NUM_FEATURES 6

/* Features of the 256 buckets of the last counting call: h_features [256][6]. */
tc_status tc_bucket_features(const tc_ctx* ctx, float* h_features);

/*
 * Timing data for training the selector: for each strategy k (0 merge,
 * 1 binary search, 2 bitmap) and bucket b, the median over `repeats` (1..64)
 * launches of strategy k on bucket b's tiles alone, in milliseconds, into
 * h_ms[k * 256 + b] (-1 where the bucket is empty). h_features (optional)
 * receives the bucket features [256][6]. Uses the same workspace as
 * tc_count_triangles.
 */
tc_status tc_profile_buckets(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                             void* d_workspace, size_t workspace_bytes, int32_t repeats, float* h_ms,
                             float* h_features);

/* Like tc_profile_buckets, but each bucket is timed only with the strategy
 * that opts->select chooses for it (the current tile shapes apply):
 * h_ms[256], -1 where the bucket is empty. Used by the tile-shape autotuner. */
tc_status tc_profile_selected(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                              void* d_workspace, size_t workspace_bytes, const tc_options* opts, int32_t repeats,
                              float* h_ms);

/*
 * Timing data for training the selector inside the combined launch: the
 * pipeline runs up to the tile layout with the caller's choice per bucket,
 * then the whole intersection stage (the three kernels over their tile
 * ranges, as a counting call launches them, and the reduction of T) runs
 * `repeats` (1..64) times. h_choice [256] (host): strategy per degree-pair
 * bucket (0 merge path, 1 binary search, 2 LDS bitmap; any other value: the
 * fixed thresholds' choice); h_chunk [256] (host) or NULL: in-edges per tile
 * per bucket (0: the default rule; clamped as for tc_set_tile_shapes).
 * h_ms [4] receives the medians, in milliseconds, of the stage (the sum of the
 * three kernels) and of each kernel; h_count (optional) receives T from the
 * last repeat. A bucket's cost is read from the change in the stage time when
 * only its entry changes. Uses the same workspace as tc_count_triangles.
 */
tc_status tc_profile_choices(tc_ctx* ctx, const int32_t* d_edges, int64_t num_edges, int32_t num_vertices,
                             void* d_workspace, size_t workspace_bytes, const uint8_t* h_choice,
                             const uint16_t* h_chunk, int32_t repeats, float* h_ms, uint64_t* h_count);

/* Load float32 master parameters (host); resets the Adam state and enables
 * TC_SELECT_LEARNED on this context. */
tc_status tc_selector_set_params(tc_ctx* ctx, const float* h_params);
tc_status tc_selector_get_params(tc_ctx* ctx, float* h_params);

/*
 * The tile network: the same shape, parameter layout and kernels as the
 * strategy network above, trained separately. In TC_SELECT_LEARNED mode its
 * argmax per bucket scales the fixed rule's in-edges per tile by 1/2 (logit 0),
 * 1 (logit 1) or 2 (logit 2) before the usual clamping (tiles of 16 to 512
 * in-edges for the bitmap strategy, 2048 for the others); tile sizes set with
 * tc_set_tile_shapes still take precedence. h_params NULL removes the network
 * (the rule's tile sizes apply). Tile sizes change the speed, never the count.
 */
tc_status tc_selector_set_tile_params(tc_ctx* ctx, const float* h_params);
tc_status tc_selector_get_tile_params(tc_ctx* ctx, float* h_params);

/*
 * Selector parameter files: JSON {"format": "tc-selector-v1", "num_params":
 * TC_SELECTOR_NUM_PARAMS, "params": [...], "meta": {...}, "tile_params":
 * [...]} (tile_params optional), the format the training driver writes.
 * tc_selector_load installs both networks (as tc_selector_set_params and
 * tc_selector_set_tile_params; no tile_params removes the tile network);
 * tc_selector_save writes the context's current parameters (floats printed
 * with 9 significant digits, which float32 values survive exactly).
 * Errors: TC_ERR_INVALID_ARG for a null argument, a file that cannot be opened,
 * read or written, or one that is not in this format (tc_last_error says which).
 */
tc_status tc_selector_load(tc_ctx* ctx, const char* path);
tc_status tc_selector_save(tc_ctx* ctx, const char* path);

/* Logits d_logits [batch][3] of features d_x [batch][6] (device arrays). */
tc_status tc_selector_forward(tc_ctx* ctx, const float* d_x, int32_t batch, float* d_logits);

/*
 * Gradient of the weighted softmax cross-entropy
 *   (1/batch) * sum_s w_s * (logsumexp(z_s) - z_s[y_s])
 * with respect to the float32 master parameters (passed through the bfloat16
 * rounding unchanged). d_labels int32 [batch] in 0..2; d_weights float32
 * [batch] or NULL (all ones); d_grad float32 [TC_SELECTOR_NUM_PARAMS] or
 * NULL; h_loss receives the loss (optional). batch in 1..65536.
 */
tc_status tc_selector_gradient(tc_ctx* ctx, const float* d_x, const int32_t* d_labels, const float* d_weights,
                               int32_t batch, float* d_grad, float* h_loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on that
 * gradient, then the bfloat16 compute copy is refreshed. */
tc_status tc_selector_train_step(tc_ctx* ctx, const float* d_x, const int32_t* d_labels, const float* d_weights,
                                 int32_t batch, float lr, float* h_loss);

/*
 * Per-stage device times (milliseconds) of the last call made with
 * TC_F_STAGE_TIMING, and their names. Returns the number of stages written
 * (at most `cap`).
 */
int32_t tc_stage_times(const tc_ctx* ctx, float* ms, int32_t cap);
const char* tc_stage_name(int32_t stage);

const char* tc_status_string(tc_status status);
/* Text of the last error recorded on the context (empty if none). */
const char* tc_last_error(const tc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* TC_MI355X_TC_H */
