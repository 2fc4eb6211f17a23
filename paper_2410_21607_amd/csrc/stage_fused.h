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
    const int32_t* col_order;   // columns sorted by colour (Morton order inside)
    const int32_t* color_ptr;   // n_color + 1 offsets into col_order (host copy below)
    int n_color;
    const uint8_t* first;       // per (column, position)
    double* cH;                 // hanging-point contributions [F][n_hh][nzn]
    int layers_per_chunk;       // layers handled together by one workgroup step
};

// Owns the device memory of the tables.
struct FusedPlan {
    FusedTables t{};
    std::vector<int32_t> color_ptr_host;
    std::vector<void*> allocs;
    int64_t bytes = 0;
};
int fused_plan_build(const HostMesh& H, int layers_per_chunk, FusedPlan& plan);
void fused_plan_free(FusedPlan& plan);
bool fused_lpc_supported(int N, int layers_per_chunk);

// Launches the column kernel and the shared-node kernel on `stream`.
int fused_stage_launch(const DevMesh& m, const FusedPlan& plan, double a, double b, double c,
                       const double* qn, const double* qs, double* qout, int precision,
                       hipStream_t stream);

}  // namespace sem
