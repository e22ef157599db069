// Arguments of the intersection kernels (device pointers into the workspace).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace tcx {

constexpr int CHUNK_MAX = 512;   // in-edges per bitmap tile (LDS-resident tail table)

struct IsectArgs {
    Ctrl* ctrl;
    const uint32_t* off;        // [n+1] CSR row offsets (ranks)
    const uint32_t* col;        // [m]   CSR columns, rows ascending
    const uint32_t* src;        // [m]   row of each edge
    const uint64_t* csc;        // [in-edges] e | row_end(u) << 32, grouped by (kernel, bucket, v)
    const uint32_t* seg_start;  // [n+1] start of each vertex's in-edge segment (bucket order)
    const uint32_t* vlist;      // [n]   vertices in bucket order
    const uint8_t* vbucket;     // [n]   bucket of each vertex
    const uint64_t* tiles;      // [ntiles] vertex position | chunk << 32
    uint32_t* per_edge;         // [m] or null: c_e in CSR edge order
    uint64_t* per_vertex;       // [n] or null: t[] in rank space
};

int isect_blocks_per_cu(int ker);
void launch_isect(int ker, const IsectArgs& a, int grid, hipStream_t s);

}  // namespace tcx
