// Host-side construction of the column mesh tables (C++17, no HIP).
//
// The mesh is a horizontal quadtree of columns over n_z vertical layers
// (refinement is horizontal and by whole columns, Section 4.1 of the paper).
// Because refinement never touches the vertical, every table factorises into
// a horizontal part (unique horizontal nodes, hanging points, their
// interpolation rows) and a vertical part (nzn = n_z*N + 1 vertical nodes).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace sem {

struct Basis1D {
    int N = 0;
    std::vector<double> x;   // LGL nodes, N+1
    std::vector<double> w;   // LGL weights, N+1
    std::vector<double> D;   // D[i*(N+1)+j] = l_j'(x_i)
};

// LGL nodes by Newton iteration on P_N' from Chebyshev-Lobatto guesses,
// weights 2/(N(N+1)P_N^2), derivative matrix from barycentric weights.
Basis1D make_basis(int N);

// Lagrange weights l_m(s) of the LGL nodes at one point s.
void lagrange_weights(const Basis1D& b, double s, double* out);

struct HostMesh {
    // description
    int N = 0, np1 = 0, n_z = 0, nzn = 0, nx0 = 0, ny0 = 0, max_level = 0;
    int ldz = 0;   // padded row stride (128-byte multiple) of [field][h][kz] arrays
    bool periodic_x = true, periodic_y = true;
    double Lx = 0, Ly = 0;
    double f = 0, g = 0, R_d = 0, c_p = 0, p00 = 0;
    Basis1D basis;
    std::vector<double> z_edges, dz, zn;   // n_z+1, n_z, nzn
    int n_col = 0;
    std::vector<int32_t> col_level, col_ix, col_iy;
    std::vector<double> col_dx, col_dy, col_x0, col_y0;
    std::vector<double> col_sx, col_sy, sz;   // 2/dx, 2/dy per column, 2/dz per layer

    // horizontal numbering
    int64_t n_h = 0, n_hh = 0;
    std::vector<int32_t> gmap;       // n_col*(N+1)^2: h >= 0, or -(hh+1)
    std::vector<double> h_xy, hh_xy; // 2*n_h, 2*n_hh
    // hanging rows (resolved to non-hanging horizontal nodes)
    std::vector<int32_t> hang_ptr, hang_src;
    std::vector<double> hang_w;
    // transposed rows: for each listed h, (hh, w) pairs
    std::vector<int32_t> hT_list, hT_ptr, hT_hh;
    std::vector<double> hT_w;
    // assembly CSR: slots c*(N+1)^2 + pos contributing to each h / hh
    std::vector<int32_t> asm_ptr, asm_slot, asmH_ptr, asmH_slot;
    // inverse lumped mass factors: M_G(h, kz) = M_H[h] * M_V[kz]
    std::vector<double> minv_h, minv_v;
    // sibling families (4 ids) per column, -1 when not a complete family
    std::vector<int32_t> sib;
    // horizontal neighbours: columns sharing at least one unique horizontal
    // node (across faces or corners), CSR over columns, ascending ids
    std::vector<int32_t> nbr_ptr, nbr_col;
    // column blocks: every 2 x 2 square of leaf columns of one level whose
    // lower-left member has even indices (a sibling family, or four level-0
    // columns) forms a block; blk_cols holds its four columns, member
    // q = qx + 2 qy at (2 bx + qx, 2 by + qy).  col_block[c] is the block of
    // column c, or -1 for a column in no block.  Unique horizontal nodes are
    // numbered block by block (positions in row order), so that the rows a
    // block touches first are consecutive in memory.
    std::vector<int32_t> blk_cols, col_block;
};

struct MeshInput {
    int N, nx0, ny0, n_z, n_col;
    const int32_t *lev, *ix, *iy;
    double Lx, Ly;
    const double* z_edges;
    bool periodic_x, periodic_y;
    double f, g, R_d, c_p, p00;
};

// Returns 0 on success, or a negative SEM_ERR_* code with a message in err.
int build_host_mesh(const MeshInput& in, HostMesh& out, std::string& err);

}  // namespace sem
