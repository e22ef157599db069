// Host-side interface of the counting pipeline.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "internal.h"

namespace tcx {

enum { SEL_HEURISTIC = 0, SEL_LEARNED = 1, SEL_FORCE_MERGE = 2, SEL_FORCE_BSEARCH = 3, SEL_FORCE_BITMAP = 4 };

// What each in-edge (u -> v) of the degree-ordered graph streams against which
// list of its middle vertex v, and the multiple of T that the sum of the hits is:
//   FILTERED     : tail of N+(u) after v  against N+(v)  -> T
//   FULL         : N(u)                   against N(v)   -> 3T
//   MATRIX       : U row of u = N+(u)     against A row of v = N(v)   -> 2T
//   MATRIX_UPPER : N+(u)                  against N+(v)  -> T
enum { FORM_FILTERED = 0, FORM_FULL = 1, FORM_MATRIX = 2, FORM_MATRIX_UPPER = 3, FORM_COUNT = 4 };
inline int form_multiple(int f) { return f == FORM_FULL ? 3 : (f == FORM_MATRIX ? 2 : 1); }

constexpr int NSTAGE = 12;

struct Layout {
    size_t ctrl, deg, rank, inv, vbucket, vlist, tstart, off, inoff, rowend, pv;
    size_t vkeysA, vkeysB, keysA, keysB, col, src, tiles, partial, bstart, isect_partials, scan_tmp, lb_aux, radix_tmp;
    size_t tile_cap;
    size_t total;
};

Layout make_layout(int64_t E, int32_t n);

struct RunArgs {
    hipStream_t stream;
    void* ws;
    const int32_t* edges;
    int64_t E;
    int32_t n;
    int select;
    const void* mlp;                 // device MlpCompute (selector network), or null
    uint8_t* learned;                // device [256] kernel per bucket written by the network
    const void* mlp_tile;            // device MlpCompute (tile network), or null
    uint8_t* learned_tile;           // device [256] tile scale per bucket written by the tile network
    const uint8_t* given;            // device [256] kernel per bucket chosen by the caller (values
                                     // >= NKERNEL: the heuristic's), or null; overrides select
    int stop_before_isect;           // leave after the tiles are laid out (bucket profiling)
    const uint16_t* chunk_override;  // device [256] or null
    const uint8_t* group_override;   // device [256] or null
    const int* grid_override;        // host [3] or null
    uint64_t* per_vertex;            // device [n] or null (original ids)
    uint64_t* per_middle;            // device [n] or null (original ids): triangles with v in the middle
                                     // (exclusive with per_vertex: both use the same scratch)
    double* clustering;              // device [n] or null (original ids): t[v] / C(d(v), 2); sets ctrl->wedges
    uint32_t* per_edge_counts;       // device [E] or null (CSR order)
    uint32_t* support;               // device [E] or null (CSR order): triangles containing each kept edge
    int32_t* per_edge_pairs;         // device [E][2] or null
    int32_t* csr_rank;               // device [n] or null (CSR export)
    int64_t* csr_off;                // device [n+1]
    int32_t* csr_col;                // device [E]
    hipEvent_t* events;              // NSTAGE + 1 events, or null
    const uint64_t* list_off;        // triangle listing pass: device [m] slot offsets per in-edge, or null
    uint32_t* list_cur;              //   device [m] zeroed cursors
    int32_t* list_out;               //   device [list_cap][3] output
    uint64_t list_cap;
    int formulation;                 // FORM_*; other than FORM_FILTERED: T only (no per-edge or
                                     // per-vertex outputs), workspace make_layout + sym_extra_bytes
};

struct RunResult {
    Ctrl* ctrl_dev;
};

hipError_t run_pipeline(const RunArgs& r, RunResult* out);
// Copies T and the status of a finished run to result[0..1] (device): range_status
// for an id out of range, internal_status for a violated internal bound, else 0.
void publish_result(const Ctrl* ctrl, uint64_t* result, uint64_t range_status, uint64_t internal_status,
                    hipStream_t s);

// ---- batched counting (batch.hip)
struct BatchLayout {
    Layout pipe;   // the union graph's pipeline workspace comes first
    size_t union_edges, eptr, eoff, voff, nv, middle, counts;
    size_t total;
};
BatchLayout make_batch_layout(int64_t E, int64_t N, int32_t G);

struct BatchArgs {
    const int32_t* edges;   // device [E][2], graph-local ids, graphs in order (its address is
                            // copied to the workspace's eptr slot before the launch)
    int64_t E;              // total pairs
    int64_t N;              // total vertices
    int32_t G;              // graphs
};
// Enqueue the whole batched count (graph offsets already in the workspace).
// r carries the stream, workspace and selection; its graph fields are set here.
hipError_t run_batch(const BatchArgs& b, RunArgs& r);
// After a full run on the same workspace: the three intersection kernels again,
// writing the triangle list (r.list_*).
hipError_t run_list_pass(const RunArgs& r);
// out[i] = in[i] for i < m (device count), widening.
void widen_u32_u64(const uint32_t* in, uint64_t* out, const Ctrl* ctrl, size_t cap, hipStream_t s);
// Extra workspace of tc_list_triangles after make_layout(E, n).total: slot offsets, counts / cursors.
size_t list_extra_bytes(int64_t E);
// Extra workspace of the other formulations after make_layout(E, n).total: the
// symmetric adjacency (row offsets and 2m columns).
size_t sym_extra_bytes(int64_t E, int32_t n);
// After a run with stop_before_isect: one intersection kernel over tiles [t0, t1).
hipError_t launch_isect_range(const RunArgs& r, int ker, uint32_t t0, uint32_t t1);
// After a run with stop_before_isect: the whole intersection stage as the pipeline
// launches it (the three kernels over their tile ranges, then the reduction of T
// into the control block); ev (null, or 4 events) is recorded before the first
// kernel and after each.
hipError_t launch_isect_stage(const RunArgs& r, hipEvent_t* ev);
int stage_count();
const char* stage_name(int s);

}  // namespace tcx
