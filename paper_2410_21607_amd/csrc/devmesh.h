// Device-side view of a column mesh: plain pointers into the handle's tables,
// passed to kernels by value.
#pragma once

#include <cstdint>

namespace sem {

struct DevMesh {
    int N, n_z, nzn, n_col;
    int ldz;                  // row stride of [field][h][kz] arrays: nzn rounded up to 16
    int n_h, n_hh, n_hT;
    double f, g, gamma;
    const int32_t* gmap;      // n_col*(N+1)^2: h >= 0, or -(hh+1)
    const double *col_dx, *col_dy, *dz;
    const double *col_sx, *col_sy, *sz;   // 2/dx, 2/dy per column, 2/dz per layer
    const int32_t *hang_ptr, *hang_src;
    const double* hang_w;
    const int32_t *hT_list, *hT_ptr, *hT_hh;
    const double* hT_w;
    const int32_t *asm_ptr, *asm_slot, *asmH_ptr, *asmH_slot;
    const double *minv_h, *minv_v;
    const int32_t *sib, *col_level;
    const int32_t *nbr_ptr, *nbr_col;   // horizontal neighbour columns (CSR)
    const double *D, *w;      // LGL derivative matrix and weights
    const double *rho0, *theta0, *dth0, *p0;   // reference state per kz
    const double *inv_rho0, *inv_theta0;       // their reciprocals per kz
    double binom[11];   // binom[n] = C(gamma, n): Taylor coefficients of (1+x)^gamma
    // optional dissipation (sem_mesh_set_dissipation): Smagorinsky constant
    // (0 = off), absorbing-layer rate per kz (null = off), and the assembled
    // dissipation tendency per unique node that the fused stage adds (null = none)
    double cs;
    const double* sponge;
    const double* rx;
    // terrain-following coordinates (sem_mesh_set_terrain; zs null = flat
    // boxes): surface height per unique horizontal node then per hanging
    // point (the coarse face's interpolant), n_h + n_hh rows; the unit surface
    // normal [3][n_h]; the inverse horizontal lumped mass with the terrain
    // factor; the reference state [5][n_h + n_hh][ldz] (rho0, 1/rho0,
    // 1/theta0, p0, dtheta0/dz; hanging rows interpolated); the factor
    // (H - zf)/(H - z0) per vertical node and 1/(H - z0)
    const double* zs;
    const double* nrm;
    const double* minv_ht;
    const double* ref_n;
    const double* tfac;
    double inv_depth;
    double z_top, depth;      // H and H - z0 (physical heights z = H - t_f (H - z0 - zs))
    double sp_gamma, sp_depth;   // absorbing layer (terrain: evaluated per node)
};

}  // namespace sem
