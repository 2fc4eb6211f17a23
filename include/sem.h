/*
 * sem.h -- C ABI of the MI355X spectral-element right-hand-side library.
 *
 * The library evaluates, on one AMD Instinct MI355X (gfx950), the per-stage
 * right-hand side of the dry compressible Euler equations written for the
 * perturbation variables (rho', u, v, w, theta') about a hydrostatic
 * reference state (Tissaoui, Guimond, Giraldo & Marras, arXiv 2410.21607,
 * Section 2, eqs. mass_split / mom_split / ent_split), discretised by
 * continuous-Galerkin spectral elements on hexahedral columns with
 * tensor-product Legendre-Gauss-Lobatto (LGL) points and inexact (lumped)
 * integration (Section 3), assembled by direct stiffness summation with the
 * hanging-node rule of Section 3.1, advanced by explicit third-order
 * Runge-Kutta stages (Section 5), and adapted with the threshold criterion of
 * Section 4.1.  The mesh is a horizontal quadtree of columns (refinement is
 * horizontal only and acts on whole columns, Section 4.1) over n_z vertical
 * layers; horizontal neighbours differ by at most one level (2:1 balance).
 *
 * Conventions shared by every call
 * --------------------------------
 * Fields      : F = 5, in the order rho' [kg m-3], u, v, w [m s-1], theta' [K].
 * Unique nodes: a non-hanging global node is a pair (h, kz) of a unique
 *               horizontal node h in [0, n_h) and a vertical node
 *               kz in [0, nzn), nzn = n_z*N + 1 (kz = layer*N + k).
 *               n_dof = n_h * nzn.
 * State layout: double q[F][n_h][ldz] (field-major, kz fastest), device memory,
 *               with the row stride ldz = nzn rounded up to a multiple of 16
 *               (128 bytes), so that each vertical row starts on a cache line.
 *               Entries kz >= nzn are padding: compute calls never read them;
 *               only sem_stage_update (element-wise) writes them.  Unique
 *               horizontal nodes are numbered block by block (2 x 2 column
 *               blocks, then the other columns, in column order).
 * Hanging     : a hanging point hh in [0, n_hh) is a horizontal position on a
 *               fine column's face that is not a node of the coarser neighbour
 *               (Section 3.1); hanging values are double hv[F][n_hh][ldz].
 * Elements    : e = c*n_z + layer for column c (in the order given at create)
 *               and layer in [0, n_z); local node l = i + (N+1)(j + (N+1)k)
 *               with i along x, j along y, k along z (Section 3, basis).
 *               Element arrays are double rE[F][n_elem][(N+1)^3].
 * Domain      : x in [-Lx/2, Lx/2], y in [-Ly/2, Ly/2], z in [z_0, z_nz].
 *               Column (level l, ix, iy) covers cell (ix, iy) of the
 *               (nx0 2^l) x (ny0 2^l) grid.  Bottom and top are rigid lids:
 *               the w tendency is zero there.  Non-periodic lateral sides
 *               carry no boundary condition (operator tests only).
 * Ownership   : every array argument is caller-owned; pointers named d_* are
 *               device pointers, h_* host pointers.  The library never frees or
 *               keeps them.  A mesh handle owns its device tables and its
 *               workspace, sized at creation, so compute calls never allocate.
 * Streams     : `stream` is a hipStream_t (NULL = the default stream).  Compute
 *               calls are asynchronous on it; device faults surface at the
 *               caller's next synchronisation.
 * Errors      : calls return SEM_OK (0) or a negative code; sem_last_error()
 *               returns a thread-local message for the last failure.
 *               Argument, shape and mesh validation happens on the host before
 *               any launch.
 */
#ifndef SEM_H
#define SEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SEM_OK        0
#define SEM_ERR_ARG  -1   /* bad argument (null pointer, size, range)      */
#define SEM_ERR_N    -2   /* unsupported polynomial order                   */
#define SEM_ERR_MESH -3   /* invalid layout: overlap, gap, 2:1 violation    */
#define SEM_ERR_HIP  -4   /* HIP runtime error (allocation, launch, copy)   */
#define SEM_ERR_STATE -5  /* call made before a required set-up call        */
#define SEM_ERR_HOST -6   /* host-side failure: memory or threads exhausted */

#define SEM_MAX_N 8       /* polynomial orders 1..8 are supported           */
#define SEM_MAX_LEVEL 12
#define SEM_NFIELDS 5

#define SEM_FP64 0        /* all arithmetic in double                        */
#define SEM_FP32 1        /* element arithmetic in float on perturbations;   */
                          /* p' is evaluated in double and rounded once;     */
                          /* assembly, mass and stage update stay double     */

#define SEM_SCATTER 0     /* sem_nc_project: unique nodes -> hanging points  */
#define SEM_GATHER  1     /* sem_nc_project: hanging points -> unique nodes  */

#define SEM_LAYOUT_COLUMNS    0 /* sem_stage work layouts (sem_stage_set_layout) */
#define SEM_LAYOUT_BLOCKS     1
#define SEM_LAYOUT_COLUMNS_KZ 2
#define SEM_LAYOUT_COLUMNS_SPLIT 3

#define SEM_ASSEMBLE 0    /* sem_dss phases */
#define SEM_FINALIZE 1

#define SEM_NFEAT 16      /* forecaster features per element                */
#define SEM_MLP_IN 16     /* forecaster network: 16 -> 64 -> 64 -> 3         */
#define SEM_MLP_HIDDEN 64
#define SEM_MLP_OUT 3
#define SEM_MLP_NPARAM 5443 /* 64*16 + 64 + 64*64 + 64 + 3*64 + 3          */
#define SEM_MLP_WORK 260  /* mlp_backward workspace floats per sample        */
#define SEM_MLP_NOALLOC_MAX 2048 /* largest batch of mlp_backward_noalloc     */

#define SEM_CRIT_SPEED 0  /* amr_flag criteria: |u| at every node           */
#define SEM_CRIT_VORTZ 1  /* vertical vorticity dv/dx - du/dy (element-local)*/

typedef struct sem_mesh sem_mesh;

/* Mesh description (all host memory, read only during sem_mesh_create). */
typedef struct {
    int32_t N;                 /* polynomial order, 1..SEM_MAX_N               */
    int32_t nx0, ny0;          /* level-0 column grid                          */
    int32_t n_z;               /* number of vertical layers                    */
    int32_t n_col;             /* number of leaf columns                       */
    const int32_t *h_col_level, *h_col_ix, *h_col_iy; /* n_col each          */
    double Lx, Ly;             /* horizontal domain size [m]                   */
    const double *h_z_edges;   /* n_z + 1 strictly increasing heights [m]      */
    int32_t periodic_x, periodic_y;
    double f, g, R_d, c_p, p00; /* Coriolis [s-1], gravity, gas constants, p00 */
} sem_mesh_desc;

typedef struct {
    int32_t N, n_z, nzn, ldz, max_level;
    int64_t n_col, n_elem, n_h, n_hh, n_dof, n_hang, n_local;
    int64_t workspace_bytes;   /* device memory held by the handle            */
} sem_mesh_info;

/* Build the column mesh (Sections 3, 3.1, 4.1): validate the layout (no
 * overlap, full cover, 2:1 face+corner balance), number the unique and
 * hanging nodes, build the interpolation rows of hanging points (composed
 * until every source is a non-hanging node), the lumped mass
 * M_G = Z^T m_L and the assembly tables, and upload them.  *out receives a
 * handle to destroy with sem_mesh_destroy.  The host build runs on
 * SEM_HOST_THREADS threads when that variable is set, else on
 * OMP_NUM_THREADS, else on the hardware count (at most 32; one thread for
 * small meshes); the tables do not depend on the count.
 * Errors: SEM_ERR_ARG, SEM_ERR_N, SEM_ERR_MESH, SEM_ERR_HIP. */
int sem_mesh_create(const sem_mesh_desc *desc, sem_mesh **out);
int sem_mesh_destroy(sem_mesh *mesh);

/* Host-only planning (no GPU needed): run the same layout validation and
 * numbering as sem_mesh_create and report sizes in *info; when the arrays are
 * non-NULL also fill h_hxy[2*n_h], h_hhxy[2*n_hh], h_z[nzn] (as in
 * sem_mesh_coords) and h_mass[n_dof], the assembled lumped mass M_G at each
 * unique node, packed as [h][kz] (no padding).  Call once with NULL arrays to learn the sizes. */
int sem_mesh_plan(const sem_mesh_desc *desc, sem_mesh_info *info, double *h_hxy,
                  double *h_hhxy, double *h_z, double *h_mass);
int sem_mesh_get_info(const sem_mesh *mesh, sem_mesh_info *out);

/* Node coordinates (host outputs, any may be NULL): h_hxy[2*n_h] (x, y of each
 * unique horizontal node), h_hhxy[2*n_hh] (x, y of each hanging point),
 * h_z[nzn] (height of each vertical node).  Used to match numberings by
 * position and to evaluate the reference state. */
int sem_mesh_coords(const sem_mesh *mesh, double *h_hxy, double *h_hhxy, double *h_z);

/* Hydrostatic reference state (Section 2, eqs. rho_split..hydro_bal) per
 * vertical node, host arrays of length nzn: rho0, theta0 and d theta0/dz.
 * The reference pressure is p0 = p00 (R_d rho0 theta0 / p00)^(c_p/c_v), the
 * equation of state applied to the reference, so that p' = 0 at rest.
 * Must be called before any compute call. */
int sem_mesh_set_reference(sem_mesh *mesh, const double *h_rho0,
                           const double *h_theta0, const double *h_dtheta0dz);

/* Optional dissipation of the paper's model setup (Section 5), added to the
 * right-hand side of sem_rhs and sem_stage when enabled (all zero = off):
 *   horizontal Smagorinsky-Lilly: the momentum equations gain the horizontal
 *     divergence of 2 nu_t S, S = (grad u + grad u^T)/2 from element-local
 *     derivatives, nu_t = (Cs Delta)^2 sqrt(2 S:S), Delta = (dx + dy)/(2N) the
 *     element's mean horizontal node spacing:
 *       R_u += d/dx(2 nu S_xx) + d/dy(2 nu S_xy)   (v: S_yx, S_yy; w: S_zx, S_zy)
 *   Rayleigh absorbing layer under the domain top: every perturbation field
 *     gains -R(z) q', R(z) = min(1, max(0, sponge_gamma sin^2(pi/2 (1 - (z_top
 *     - z)/sponge_depth)))) for z >= z_top - sponge_depth, zero below.
 * Both are evaluated in FP64 element by element (strong form, like the other
 * terms) and assembled with the same direct stiffness summation.  With
 * terrain set (sem_mesh_set_terrain) the derivatives are the physical ones
 * (chain rule of the mapping) and z is each node's physical height.  In
 * sem_stage at SEM_FP64 on meshes without terrain in the column layout the
 * terms are computed inside the column passes (the element stress in LDS);
 * otherwise (terrain, SEM_FP32, the block layout) they run as a pre-pass
 * whose assembled tendency the column pass adds.  Enabling allocates the
 * pre-pass buffers once (5 element-local and 2 state arrays); compute calls
 * never allocate.  Synchronises the device.
 * Compute calls read the settings when they are enqueued: a HIP graph
 * captured before this call keeps replaying the previous ones. */
int sem_mesh_set_dissipation(sem_mesh *mesh, double Cs, double sponge_gamma,
                             double sponge_depth);

/* Terrain-following coordinates: the basis of Section 3 on mapped hexahedra
 * (the mappings xi(x), eta(x), zeta(x) of that section are affine for the
 * paper's box elements; here the vertical one follows the terrain).
 *   h_zs[n_h]: surface height above the flat bottom z0 = z_edges[0] at every
 *     unique horizontal node (sem_mesh_coords order), 0 <= zs < H - z0 with
 *     H = z_edges[n_z].  A node at flat height zf moves to
 *     z = zf + zs (H - zf) / (H - z0); columns keep their horizontal boxes.
 *   h_rho0, h_theta0, h_dtheta0dz[n_dof], packed [h][kz]: the reference state
 *     at every node's physical height (p0 is the equation of state of rho0,
 *     theta0, as in sem_mesh_set_reference).
 * Hanging points (Section 3.1) take the coarse face's interpolant of zs and
 * of the reference state, so the mapped mesh stays watertight across 2:1
 * faces.  sem_stage then takes every derivative by the chain rule with the
 * discrete metric of the mapping (dzs/dx, dzs/dy from the element's nodal
 * zs), uses the mapped lumped masses (w_i w_j w_k det J, assembled with the
 * modified DSS), keeps the rigid lid at the top, and at the terrain surface
 * removes the component of the momentum tendency along the unit normal
 * n ~ (-dzs/dx, -dzs/dy, 1), whose horizontal gradient is averaged over the
 * columns sharing the node with the lumped masses.  Flat terrain (all
 * zs = 0) reproduces the box-element stage.
 * sem_rhs (element contributions with the mapped masses) and sem_dss
 * (FINALIZE: the terrain inverse mass, the surface rule and the top lid) do
 * the same per call, and amr_flag takes the vorticity criterion through the
 * same chain rule.  SEM_FP32 (sem_stage, sem_rhs) keeps the metric factors
 * in FP64 and rounds them to float with the rest of the element arithmetic.
 * amr_features and the dissipation (sem_mesh_set_dissipation) take their
 * derivatives through the same chain rule.
 * h_zs = NULL removes the terrain.  As for the dissipation, a HIP graph
 * captured before this call keeps the previous geometry: capture after it.
 * Arrays are copied; synchronises the
 * device.  Errors: SEM_ERR_ARG (null mesh, zs out of range, non-positive
 * reference), SEM_ERR_MESH (non-positive assembled mass), SEM_ERR_HIP. */
int sem_mesh_set_terrain(sem_mesh *mesh, const double *h_zs, const double *h_rho0,
                         const double *h_theta0, const double *h_dtheta0dz);

/* Physical height of every unique node (host output h_z[n_dof], packed
 * [h][kz]) under the terrain-following mapping of sem_mesh_set_terrain:
 * z = zf + zs (H - zf) / (H - z0) for a node at flat height zf over a unique
 * horizontal node with surface height zs.  h_zs[n_h] gives the surface to
 * map with (it need not be set on the handle: the reference state at the
 * physical heights is needed before sem_mesh_set_terrain); h_zs = NULL uses
 * the handle's terrain, or flat heights when none is set.  Host only.
 * Errors: SEM_ERR_ARG (null mesh or h_z, zs outside [0, H - z0)). */
int sem_mesh_heights(const sem_mesh *mesh, const double *h_zs, double *h_z);

/* Set-up epoch of a mesh handle: a counter that every call changing what a
 * captured HIP graph of compute calls would read (sem_stage_tune,
 * sem_stage_set_layout, sem_stage_autotune, sem_mesh_set_reference,
 * sem_mesh_set_terrain, sem_mesh_set_dissipation) increments.  A graph captured at epoch e may be
 * replayed only while the epoch is still e; afterwards it can read freed
 * tables or stale settings, so capture it again. */
int sem_mesh_get_epoch(const sem_mesh *mesh, int64_t *epoch);

/* Modified-DSS interpolation across nonconforming faces (Section 3.1).
 * SEM_SCATTER: d_dst = hv[F][n_hh][ldz] is overwritten with Z_h d_src, the
 *              values at hanging points interpolated from d_src = q[F][n_h][ldz].
 * SEM_GATHER : d_dst = acc[F][n_h][ldz] += Z_h^T d_src, d_src = c[F][n_hh][ldz]
 *              holding contributions summed at hanging points.
 * A mesh without hanging points makes both a no-op. */
int sem_nc_project(const sem_mesh *mesh, int dir, const double *d_src,
                   double *d_dst, void *stream);

/* Element right-hand side (Section 2 perturbation equations, strong form,
 * collocated at the LGL nodes of every element, Section 3), multiplied by the
 * lumped LGL mass w_i w_j w_k |J_e|:
 *   d_rE[F][n_elem][(N+1)^3] = m_l * R_l.
 * Inputs: d_q = q[F][n_h][ldz], d_hv = hanging values from SEM_SCATTER (may
 * be NULL when n_hh = 0).  precision = SEM_FP64 or SEM_FP32. */
int sem_rhs(const sem_mesh *mesh, const double *d_q, const double *d_hv,
            double *d_rE, int precision, void *stream);

/* Direct stiffness summation (Section 3.1).
 * SEM_ASSEMBLE: d_acc[F][n_h][ldz] = sum of d_rE over the local copies of each
 *               unique node; d_c[F][n_hh][ldz] = the same at hanging points
 *               (pass d_c to sem_nc_project(SEM_GATHER) to add Z_h^T c).
 * SEM_FINALIZE: d_r[F][n_h][ldz] = d_acc / M_G, then r_w = 0 on the lids.
 * Unused pointers for a phase may be NULL. */
int sem_dss(const sem_mesh *mesh, int phase, const double *d_rE, double *d_acc,
            double *d_c, double *d_r, void *stream);

/* Runge-Kutta stage combination (Section 5), element-wise over 5*n_h*ldz values:
 *   d_qout = a*d_qn + b*d_qs + c*d_r        (any pointers may alias). */
int sem_stage_update(const sem_mesh *mesh, double a, double b, double c,
                     const double *d_qn, const double *d_qs, const double *d_r,
                     double *d_qout, void *stream);

/* Fused stage: d_qout = a*d_qn + b*d_qs + c*R(d_qs), with R the full
 * right-hand side (scatter, element RHS, assembly, gather, finalize, lid rule)
 * evaluated without storing element-local data.  Work units (columns, or
 * 2 x 2 column blocks: sem_stage_set_layout) are coloured so that units of
 * one colour share no node; the launches of one colour cover the units of
 * every refinement level of that colour (a workgroup marches up one column
 * or one block in chunks of stacked elements).  The first colour touching a
 * node writes a*q^n + b*q_s + c*M^-1*(its contribution); later colours add
 * their contributions (plain read-modify-write; the launches order them, so
 * results are deterministic and bit-identical from run to run).  Hanging
 * points collect their contributions in the handle's buffer, which one more
 * launch adds to the coarse face nodes (Z^T).  d_qout must not alias d_qs or
 * d_qn.  Calls on one handle must not overlap.  Allocates nothing; the kernel
 * nodes (colours + 1 on meshes with hanging points) can be captured in a HIP
 * graph. */
int sem_stage(const sem_mesh *mesh, double a, double b, double c,
              const double *d_qn, const double *d_qs, double *d_qout,
              int precision, void *stream);

/* Work decomposition of sem_stage (chosen by the autotuner, or by hand):
 * layers_per_chunk = stacked elements handled by one workgroup, one thread per
 * unique node of the chunk ((N+1)^2 (layers_per_chunk N + 1) threads).
 * 0 = default (the deepest chunk of at most 512 threads).  Supported: 1, 2, 4
 * and 8 at N <= 4, 1, 2 and 4 at N = 5, 1 and 2 at N = 6, 7, and 1 at N = 8
 * (workgroups within 1024 threads and a CU's 160 KB of LDS).  Rebuilds
 * the handle's fused tables and synchronises the device.  sem_stage_get_tune
 * reports the current value. */
int sem_stage_tune(sem_mesh *mesh, int layers_per_chunk);
int sem_stage_get_tune(const sem_mesh *mesh, int *layers_per_chunk);

/* Work layout of sem_stage (the LDS tile layout and workgroup packing):
 *   SEM_LAYOUT_COLUMNS: a workgroup per column, chunks of `param` layers
 *     (as sem_stage_tune; 0 = default); in FP64 the threads of the nodes on
 *     the planes between stacked elements come first (they take two z
 *     derivatives), in float the vertical index runs fastest;
 *   SEM_LAYOUT_COLUMNS_KZ: the same with the vertical index fastest in FP64
 *     too (fewer rows per wave in the global loads and stores, the second z
 *     derivative spread over every wave).  In this natural order a
 *     position's nodes below the chunk's top plane take consecutive threads
 *     and the top plane's nodes come last, so that at N = 4 with four layers
 *     per chunk a wave's loads and stores cover whole 128-byte lines;
 *   SEM_LAYOUT_COLUMNS_SPLIT: in FP64 a thread per (element, local node) of
 *     each position, so that each thread takes one element's z derivatives
 *     and a node between two elements has two threads (the lower hands its
 *     part to the upper by a wave shuffle); needs param >= 2 and every such
 *     pair in one wave (otherwise SEM_ERR_ARG); float runs the natural order.
 *   The three column orders give bit-identical results without the optional
 *   dissipation (with it, the split order sums the absorbing-layer and stress
 *   parts of a plane node in another order, within 1e-14);
 *   SEM_LAYOUT_BLOCKS: a workgroup per 2 x 2 block of columns of one level
 *     (a sibling family, or four level-0 columns), a (2N+1)^2 tile per layer,
 *     the column in `param` vertical segments (0 = enough segments for about
 *     1024 workgroups per launch); columns in no block run as in the column
 *     layout.  Orders 3 to 5 on meshes with blocks (box elements: with
 *     terrain set, sem_stage runs the column layout).
 * The faces inside a block are summed in the workgroup; blocks are coloured
 * like columns, so the results are deterministic in either layout (they
 * differ between layouts by the order of the sums, within 1e-14).  Meshes
 * start in the column layout.  Rebuilds the handle's tables and
 * synchronises the device.  sem_stage_get_layout reports the layout and its
 * parameter (layers per chunk, or the number of segments). */
int sem_stage_set_layout(sem_mesh *mesh, int layout, int param);
int sem_stage_get_layout(const sem_mesh *mesh, int *layout, int *param);

/* Autotuner: times every supported work layout on this mesh (the column
 * layout at each supported layers_per_chunk, in FP64 in each thread order,
 * the block layout at 1, 2, 4, ... vertical segments; reps fused stages
 * each, HIP events on `stream`, d_qout used as scratch), keeps the fastest
 * with sem_stage_set_layout, and reports
 * it (*best_lpc = the column layout's layers per chunk, see
 * sem_stage_get_layout for the layout; *best_ms = mean stage time in ms;
 * either may be NULL).  Synchronises the stream. */
int sem_stage_autotune(sem_mesh *mesh, const double *d_qn, const double *d_qs,
                       double *d_qout, int precision, int reps, int *best_lpc,
                       float *best_ms, void *stream);

/* Refinement flags (Section 4.1).  Criterion C at every node of every element
 * from element-local values: SEM_CRIT_SPEED |u| or SEM_CRIT_VORTZ dv/dx-du/dy.
 * h_thr[0..lvl_max-1] = threshold(1..lvl_max), non-decreasing (host memory).
 * d_adapt_elem[n_elem] (int8): +1 if some node has C > threshold(lvl+1) and
 * lvl < lvl_max; -1 if every node has C <= threshold(lvl) and lvl > 0; else 0.
 * d_adapt_col[n_col] (int8): +1 if any element of the column is +1; -1 if all
 * elements of the column and of its three siblings are -1; else 0. */
int amr_flag(const sem_mesh *mesh, const double *d_q, int criterion,
             const double *h_thr, int lvl_max, int8_t *d_adapt_elem,
             int8_t *d_adapt_col, void *stream);

/* One adaptation pass of the column layout (Section 4.1: a column is refined
 * by splitting it into a 2 x 2 block of columns, four sibling columns are
 * coarsened by merging them into their parent).  Host only, no GPU needed.
 * Inputs: desc (only nx0, ny0, periodic_x/y and the column list are read; the
 * list must tile the domain without overlap), h_adapt_col[n_col] in
 * {-1, 0, +1} (for example amr_flag's d_adapt_col copied to the host) and
 * lvl_max.  The pass:
 *   1. splits every column flagged +1 whose level is below lvl_max;
 *   2. restores 2:1 face+corner balance by splitting every column that
 *      touches a column two or more levels finer, until none does (the
 *      coarsest balanced layout containing step 1);
 *   3. merges every family of four sibling columns all flagged -1 whose
 *      parent would touch no column more than one level finer; every merge is
 *      decided on the layout of step 2, so the result is order-independent.
 * Output: *n_out = number of columns; when cap >= *n_out the columns are
 * written to h_level/h_ix/h_iy[cap] in Morton order of the finest level
 * present, else SEM_ERR_ARG is returned (call with cap = 0 and NULL arrays to
 * learn the size).  Errors: SEM_ERR_ARG, SEM_ERR_MESH (invalid input layout). */
int sem_adapt_columns(const sem_mesh_desc *desc, const int8_t *h_adapt_col, int lvl_max,
                      int32_t cap, int32_t *h_level, int32_t *h_ix, int32_t *h_iy,
                      int32_t *n_out);

/* Solution transfer onto an adapted mesh.  The paper delegates it to its
 * mesh library; the rule implemented here (both meshes must share order N,
 * base grid, domain and vertical layers, and every column of `to` must be a
 * column of `from`, a child of one, or the parent of four):
 *   * a node of a column present in both meshes, or of a child of a split
 *     column, takes the old field at its position: the old element
 *     polynomial, exact for the interpolation of a split;
 *   * a node belonging only to merged parents takes the lumped-mass weighted
 *     average of the parents' discrete L2 projections of their four children
 *     (the projection conserves each parent's sum of m q).
 * The transfer is horizontal (the vertical is untouched), a sparse matrix T
 * of n_h(to) rows over the n_h(from) horizontal nodes:
 *   q_to[f][h][kz] = sum_r w[r] q_from[f][src[r]][kz],  kz < nzn,
 * and zero in the row padding.
 * sem_transfer_create builds T from two mesh handles and uploads it (the
 * handle does not keep the meshes); sem_transfer_apply launches it on
 * `stream` (d_q_from = q[F][n_h(from)][ldz], d_q_to = q[F][n_h(to)][ldz],
 * not aliased; allocates nothing).  sem_transfer_plan is the host-only
 * variant: it builds both meshes from their descriptions and returns T in CSR
 * form, *nnz entries, h_ptr[n_h(to)+1], h_src[nnz], h_w[nnz] (any array
 * may be NULL to learn nnz first). */
typedef struct sem_transfer sem_transfer;
int sem_transfer_create(const sem_mesh *from, const sem_mesh *to, sem_transfer **out);
int sem_transfer_apply(const sem_transfer *t, const double *d_q_from, double *d_q_to,
                       void *stream);
int sem_transfer_destroy(sem_transfer *t);
int sem_transfer_plan(const sem_mesh_desc *from, const sem_mesh_desc *to, int64_t *nnz,
                      int32_t *h_ptr, int32_t *h_src, double *h_w);

/* ---------------------------------------------------------------------------
 * Refinement forecaster.  The paper's criterion (Section 4.1) thresholds a
 * field at the element's nodes at the moment of adaptation; its conclusions
 * call for better criteria.  The forecaster predicts the decision several
 * adaptation intervals ahead with a small network on per-element features,
 * so that the mesh can be rebuilt less often; its flags are combined with
 * the criterion's, which overrides every refinement the forecaster misses.
 * ------------------------------------------------------------------------- */

/* Per-element features, d_feat[n_elem][SEM_NFEAT] (float), each raw value
 * multiplied by h_scale[i] (host, SEM_NFEAT floats).  Raw features, from
 * element-local values and derivatives (LGL derivative matrix, as in the
 * criterion; with terrain set, the physical derivatives by the chain rule of
 * the mapping and p' from the per-node reference), zeta = dv/dx - du/dy,
 * u_h = (u, v):
 *   0 level, 1 max|zeta|, 2 mean zeta over the element's nodes, 3 max|u_h|,
 *   4 max|w|, 5 max theta', 6 min theta', 7 max|grad p'|, 8 max|grad theta'|,
 *   9 max|div u|, 10 max rho' - min rho', 11 largest feature-1 value and
 *   12 largest feature-3 value over the elements of the same layer in the
 *   horizontal neighbour columns (columns sharing a unique node), 13 feature 3
 *   minus its value for d_q_prev, 14 feature 1 minus its value for d_q_prev,
 *   15 the criterion's element flag d_plain_elem[e] (from amr_flag).
 * d_dem[n_elem] (int8) = the level the criterion asks for: the largest l in
 * 1..lvl_max with C_max > threshold(l) (0 if none), C as in amr_flag.
 * d_q, d_q_prev: states on this mesh (q[F][n_h][ldz]).  Uses the handle's
 * feature scratch, so calls on one handle must not overlap.  Errors:
 * SEM_ERR_STATE (neither a reference nor terrain set), SEM_ERR_ARG. */
int amr_features(const sem_mesh *mesh, const double *d_q, const double *d_q_prev,
                 const int8_t *d_plain_elem, int criterion, const double *h_thr, int lvl_max,
                 const float *h_scale, float *d_feat, int8_t *d_dem, void *stream);

/* Forecast flags combined with the criterion's.  d_logits[n_elem][3] from
 * mlp_forward; class = argmax (first maximum on ties) in {0 coarsen, 1 keep,
 * 2 refine}, clamped so that level 0 never coarsens and lvl_max never
 * refines.  Element flag: +1 if the forecast or d_plain_elem is +1, -1 if
 * both are -1, else 0 -> d_adapt_elem[n_elem]; column flags d_adapt_col[n_col]
 * by the column rule of amr_flag. */
int amr_forecast_flags(const sem_mesh *mesh, const float *d_logits, const int8_t *d_plain_elem,
                       int lvl_max, int8_t *d_adapt_elem, int8_t *d_adapt_col, void *stream);

/* Maximum horizontal wind (the paper's intensity measure, Section 5):
 * *d_vmax (device) = max sqrt(u^2 + v^2) over the unique nodes whose
 * horizontal position (as reported by sem_mesh_coords) lies in
 * [x0, x1] x [y0, y1], every height; 0 if none.  Uses the handle's scratch,
 * so calls on one handle must not overlap. */
int sem_max_wind(const sem_mesh *mesh, const double *d_q, double x0, double x1, double y0,
                 double y1, double *d_vmax, void *stream);

/* Training labels (host only): for every element (column c, layer) of the
 * layout `at`, the class clip(D - level, -1, 1) + 1 in {0, 1, 2}, where D is
 * the criterion's level (d_dem of amr_features) of the element of the same
 * layer in the layout `later` that contains the column, or the largest over
 * the later columns inside it.  h_dem_later[n_elem(later)], h_class[n_elem(at)]. */
int sem_forecast_labels(const sem_mesh_desc *at, const sem_mesh_desc *later,
                        const int8_t *h_dem_later, int8_t *h_class);

/* Network 16 -> 64 -> 64 -> 3, tanh hidden activations, FP32.  d_params is
 * one array of SEM_MLP_NPARAM floats: W1[64][16], b1[64], W2[64][64], b2[64],
 * W3[3][64], b3[3] (z = W x + b per layer).
 * mlp_forward : d_logits[n][3] for inputs d_x[n][16].
 * mlp_backward: the gradient of the mean softmax cross-entropy over a batch of
 *   n samples, d_grad[SEM_MLP_NPARAM], and the loss itself, *d_loss (device).
 *   d_x[n_rows][16] and d_class[n_rows] (class in {0,1,2}) hold the data;
 *   sample b is row d_idx[b], or row b when d_idx is NULL (then n <= n_rows).
 *   Indices outside [0, n_rows) and classes outside {0,1,2} are clamped into
 *   range (memory safety; the binding checks them).  d_work: n*SEM_MLP_WORK
 *   floats of caller-owned scratch.  Sums over the batch run in a fixed order
 *   (deterministic).
 * mlp_adam_step: Adam with bias correction, step t >= 1:
 *   m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 *   p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
int mlp_forward(const float *d_params, const float *d_x, int64_t n, float *d_logits, void *stream);
int mlp_backward(const float *d_params, const float *d_x, int64_t n_rows, const int8_t *d_class,
                 const int32_t *d_idx, int64_t n, float *d_work, float *d_grad, float *d_loss,
                 void *stream);
int mlp_adam_step(float *d_params, const float *d_grad, float *d_m, float *d_v, int t, float lr,
                  float beta1, float beta2, float eps, void *stream);

/* mlp_backward without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, training loops that must not
 * call hipMalloc).  Same arguments, kernels and results as mlp_backward
 * minus d_work: the per-sample workspace is a file-scope device array of
 * SEM_MLP_NOALLOC_MAX * SEM_MLP_WORK floats (about 2.1 MB per GPU, held until
 * the process ends), whose device address is looked up once per GPU on its
 * first call.  The call itself allocates nothing.  Errors: SEM_ERR_ARG also
 * for n > SEM_MLP_NOALLOC_MAX.  Every call on one GPU uses that GPU's single
 * array, so calls that overlap on one GPU (other streams, other threads)
 * race: order them on one stream.  No state carries over between calls
 * (each call writes every workspace entry it reads). */
int mlp_backward_noalloc(const float *d_params, const float *d_x, int64_t n_rows,
                         const int8_t *d_class, const int32_t *d_idx, int64_t n,
                         float *d_grad, float *d_loss, void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *sem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SEM_H */
