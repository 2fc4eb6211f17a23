// Fused Runge-Kutta stage: one pass over the columns of every refinement
// level computes q_out = a q^n + b q_s + c M^-1 Z^T (m_L R_L(Z q_s)).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "devmesh.h"

namespace sem {

struct HostMesh;

// Host-built tables of the fused path (device pointers).
//
// Columns are coloured so that no two columns of one colour contribute to a
// common unique node or hanging point; each colour is one launch.  For every
// (column, position) `first` says whether this column is the lowest-coloured
// contributor of its node: the first contributor writes the node, later ones
// add to it (plain read-modify-write, ordered by the launches).
struct FusedTables {
    const int32_t* col_order;   // columns sorted by colour; inside a colour by
                                // decreasing work (hanging positions), then Morton
    const int32_t* color_ptr;   // n_color + 1 offsets into col_order (host copy below)
    int n_color;
    const uint8_t* first;       // per (column, position)
    double* cH;                 // hanging-point contributions [F][n_hh][nzn]
    int layers_per_chunk;       // layers handled together by one workgroup step
    int thread_order;           // FP64 thread order: 0 = nodes of the planes between
                                // elements first, 1 = vertical index fastest,
                                // 2 = split element
    // Position map and interpolation rows the kernel reads (the mesh's own,
    // extended when the plan has side columns).  Side columns (the columns
    // of the small colour classes of an uneven mesh) run in the launches of
    // the other colours, spread to even them out; every position of theirs
    // maps to a pseudo hanging
    // point past the mesh's n_hh, whose row is the unit row of its node (or a
    // copy of its hanging row), so that the kernel stores the position's
    // contribution in cH unchanged; the tail launch assembles them.
    const int32_t* gmap;
    const int32_t *hang_ptr, *hang_src;
    const double* hang_w;
    const int32_t* hreal;       // per (pseudo) hanging point: index into the
                                // surface and reference rows ([0, n_h + n_hh))
    int64_t fsh;                // field stride of cH: (hanging + pseudo points) * ldz
};

// Tail launch: the unique nodes that receive side-slot or hanging-point
// contributions, each summing them in a fixed order and finishing the node.
struct TailTables {
    const int32_t* h;           // n: unique horizontal node
    const uint8_t* first;       // n: no column launch writes the node first
    // per node a flat list of contribution rows (hanging or pseudo hanging
    // points of cH) in groups: the node's side slots (weight 1), then per
    // hanging point of its Z^T row that point (when a column launch writes
    // it) and its side slots (weight w of the row); estart marks a group's
    // first entry and carries its weight; row -1 adds nothing
    const int32_t *eptr, *erow;
    const double* ew;
    const uint8_t* estart;
    const double* cH;           // hanging and pseudo hanging points
    int n;
    int64_t fsh;                // field stride of cH
};

// Block layout: the work unit is a 2 x 2 block of columns of one level (a
// sibling family, or four level-0 columns), split vertically into segments of
// `Ls` layers.  Blocks are coloured so that blocks of one colour share no
// node; a segment's planes are its own except the plane it shares with the
// segment above or below, whose first writer is the even segment (launches
// run colour by colour, even segments before odd ones).  Columns in no block
// run through the column kernel in their colour's turn.
struct BlockTables {
    const int32_t* order;       // blocks sorted by colour
    const int32_t* pos_g;       // n_blk * (2N+1)^2: unique node or -(hh+1) per block position
    const uint8_t* pos_first;   // n_blk * (2N+1)^2: first contributor of its node
    const int32_t* blk_col;     // n_blk: a member column (all four share the geometry)
    double* cH;                 // hanging-point contributions (the column layout's buffer)
    int64_t fsh;                // its field stride
    int n_seg, Ls;              // vertical segments, layers per segment
};

// Owns the device memory of the tables.
struct FusedPlan {
    FusedTables t{};                      // column layout (every column)
    std::vector<int32_t> color_ptr_host;
    TailTables tail{};                    // column layout with side columns
    bool has_tail = false;
    int layout = 0;                       // SEM_LAYOUT_COLUMNS, _COLUMNS_KZ, _COLUMNS_SPLIT or _BLOCKS
    BlockTables bt{};                     // block layout
    FusedTables ts{};                     // block layout: the columns in no block
    std::vector<int32_t> blk_ptr_host, single_ptr_host;   // per colour
    int n_unit_color = 0;
    std::vector<void*> allocs;
    int64_t bytes = 0;
};
// layout SEM_LAYOUT_COLUMNS / _COLUMNS_KZ / _COLUMNS_SPLIT: param = layers per
// chunk (0 = default);
// SEM_LAYOUT_BLOCKS: param = vertical segments (0 = default)
int fused_plan_build(const HostMesh& H, int layout, int param, FusedPlan& plan);
void fused_plan_free(FusedPlan& plan);
bool fused_lpc_supported(int N, int layers_per_chunk);
// whether the split-element thread order applies (two or more layers per
// chunk, every pair of threads of a plane node in one wave)
bool fused_split_supported(int N, int layers_per_chunk);
bool fused_blocks_supported(const HostMesh& H);

// Whether sem_stage evaluates the optional dissipation inside the column
// kernel (FP64, box elements, column layout) instead of a pre-pass.
bool fused_dissipation_inline(const DevMesh& m, const FusedPlan& plan, int precision);

// Launches the column kernel and the shared-node kernel on `stream`.
int fused_stage_launch(const DevMesh& m, const FusedPlan& plan, double a, double b, double c,
                       const double* qn, const double* qs, double* qout, int precision,
                       hipStream_t stream);

}  // namespace sem
