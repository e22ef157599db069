// Arguments of the intersection kernels (device pointers into the workspace).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace tcx {

constexpr int CHUNK_MAX = 512;   // in-edges per tile (LDS-resident entry table)
constexpr int STAGE_MAX = 4096;  // list elements of a tile that merge/bsearch stage in LDS (else read in place)

struct IsectArgs {
    Ctrl* ctrl;                 // control block: tile ranges, tile shapes, the total
    const uint32_t* off;       // [n+1] CSR row offsets (ranks)
    const uint32_t* col;        // [m]   CSR columns, rows ascending
    const uint32_t* src;        // [m]   row of each edge
    const uint64_t* csc;        // [m_active] tail start | tail end << 32, grouped by middle vertex
    const uint32_t* inoff;      // [n+1] start of each vertex's in-edges in csc
    const uint32_t* vlist;      // [n]   vertices in (kernel, bucket) order
    const uint8_t* vbucket;     // [n]   bucket of each vertex
    const uint4* tiles;         // [ntiles] tile descriptors (see TILE_MULTI)
    uint32_t* per_edge;         // [m] or null: c_e in CSR edge order
    uint64_t* per_vertex;       // [n] or null: t[] in rank space
    uint64_t* per_middle;       // [n] or null: triangles whose middle vertex is v (rank space)
    uint32_t* support;          // [m] or null: triangles containing each kept edge (CSR edge order)
    uint32_t col_narrow;        // 1 when col spans less than 4 GiB (32-bit byte offsets suffice)
    // triangle listing (second pass): triangle i of in-edge e goes to
    // list_out[3 * (list_off[e] + i)], as original ids (u, v, w)
    const uint64_t* list_off;   // [m] or null
    uint32_t* list_cur;         // [m] zeroed: per-edge cursors of the edge-centric kernels
    int32_t* list_out;          // [list_cap][3]
    uint64_t list_cap;          // triples list_out holds; a slot beyond sets error bit 3
    const uint32_t* inv;        // [n] rank -> original id
    // 1: the tails are whole rows that may reach below and above the middle
    // list (the full-list and matrix formulations); the bitmap kernel then clips
    // each tail to the window it is testing. Count only.
    uint32_t clip;
};

// Blocks of one intersection kernel resident per CU (from the occupancy API);
// mode: the bitmap kernel's output mode (0 for the edge kernels).
int isect_blocks_per_cu(int ker, int mode);
size_t isect_partials_bytes();
// One intersection kernel over its tile range; per-block partial counts go to
// partials (isect_partials_bytes() of workspace shared by the three kernels).
void launch_isect(int ker, const IsectArgs& a, int grid, uint64_t* partials, hipStream_t s);
// ctrl->total = sum of all partial counts.
void launch_reduce_total(uint64_t* partials, Ctrl* ctrl, hipStream_t s);

}  // namespace tcx
