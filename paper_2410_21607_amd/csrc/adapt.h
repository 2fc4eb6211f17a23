// Host-side adaptation of the column layout and the solution-transfer rows
// between two meshes (C++17, no HIP).
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "mesh_build.h"

namespace sem {

// One adaptation pass (Section 4.1: whole columns are split into 2 x 2
// children or four siblings are merged):
//   1. split every column flagged +1 whose level is below lvl_max;
//   2. restore 2:1 face+corner balance by splitting every leaf that touches a
//      leaf two or more levels finer (the coarsest balanced refinement);
//   3. merge each family of four sibling leaves flagged -1 whose parent box
//      touches no leaf more than one level finer than the parent, all merges
//      decided on the layout of step 2.
// The result is sorted along the Morton curve of the finest level present.
int adapt_layout(int nx0, int ny0, bool periodic_x, bool periodic_y, int n_col,
                 const int32_t* lev, const int32_t* ix, const int32_t* iy,
                 const int8_t* flags, int lvl_max,
                 std::vector<std::array<int32_t, 3>>& out, std::string& err);

// Rows of the horizontal transfer matrix T (n_h(to) x n_h(from)) such that
// q_to[f][h][kz] = sum_r w[r] q_from[f][src[r]][kz] (the vertical structure
// is shared, so the transfer acts on horizontal nodes only):
//  * a node of a column that exists in both layouts, or of a child of a split
//    column, takes the old field at its position (the old element polynomial,
//    through the hanging rows of the old mesh where needed);
//  * a node that belongs only to merged parents takes the lumped-mass
//    weighted average of their discrete L2 projections of the four children.
struct TransferRows {
    std::vector<int32_t> ptr, src;
    std::vector<double> w;
};
int build_transfer(const HostMesh& from, const HostMesh& to, TransferRows& T, std::string& err);

}  // namespace sem
