// Fused Runge-Kutta stage for gfx950.
//
// q_out = a q^n + b q_s + c M^-1 Z^T (m_L R_L(Z q_s)) in one pass over the
// columns of every refinement level, without ever storing the element-local
// right-hand side.
//
// Column kernel.  A workgroup owns one column and marches up through it in
// chunks of `layers_per_chunk` stacked elements; one thread per unique node of
// the chunk, or (split-element order) per element and local node, so that a
// node between two stacked elements has two (the thread orders are described
// at the mapping below; the accesses of one horizontal position are
// contiguous in the [field][h][kz] state layout):
//   * load the node of q_s (hanging positions interpolate the coarse face
//     nodes: the scatter of Section 3.1) and evaluate the pointwise fields of
//     Section 2 (rho u, rho v, rho w, u, v, w, p', theta') into LDS;
//   * sum-factorised derivatives along x, y, z read the chunk tile from LDS
//     (Section 3: tensor-product LGL basis, affine boxes); a node on the plane
//     between two stacked elements shares its x and y derivatives and takes
//     the z derivative of each element;
//   * the strong-form right-hand side times the lumped LGL mass, summed over
//     the elements of the chunk, is the column's contribution to the node; the
//     plane between two chunks is completed through an LDS carry;
//   * the node is then updated in place: the first contributor (lowest colour)
//     writes a q^n + b q_s + c M^-1 contribution, later colours add
//     c M^-1 contribution; hanging positions collect their contribution in a
//     buffer instead (Z^T below).
// Columns are coloured so that no two columns of one colour share a node: each
// colour is one launch, so the read-modify-writes never race and the order of
// the sums is fixed (deterministic results).  Within a launch the columns
// start in order of decreasing work.
// Hanging-point kernel (meshes with hanging nodes): every coarse face node
// adds c M^-1 sum_hh w_hh c_hh, the transpose of the scatter (Section 3.1).
#include "stage_fused.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <string>
#include <type_traits>

#include "mesh_build.h"
#include "sem.h"

namespace sem {

namespace {

constexpr int NF = SEM_NFIELDS;
// LDS tiles: rho u, rho v, rho w and u singly; (v, w) and (p', theta') as pairs

template <int NP, int LPC, bool SE = false>
constexpr int wg_threads() {
    return ((NP * NP * (SE ? LPC * NP : LPC * (NP - 1) + 1) + 63) / 64) * 64;
}

// Split-element thread order: a thread per (element, local node) of each
// position, so that a node on the plane between two stacked elements has two
// threads, each taking one element's z derivatives.  The lower one hands its
// part to the upper one (the next lane) by a shuffle, so every such pair must
// sit in one wave.
template <int NP, int LPC>
constexpr bool se_pairs_in_wave() {
    for (int p = 0; p < NP * NP; ++p)
        for (int el = 1; el < LPC; ++el)
            if ((p * LPC * NP + el * NP) % 64 == 0) return false;
    return true;
}
// Thread orders of the column kernel: 0 = the nodes of the planes between
// stacked elements first, 1 = natural (vertical index fastest), 2 = split
// element.  The order an instance actually runs: float always takes the
// natural one, and so does the split order where it does not apply (one
// layer per chunk, or a pair across two waves).
template <int NP, int LPC, typename T, int ORD>
constexpr int eff_order() {
    if (sizeof(T) == 4) return 1;
    if (ORD == 2 && !(LPC > 1 && se_pairs_in_wave<NP, LPC>())) return 1;
    return ORD;
}
// threads of a column-kernel workgroup
template <int NP, int LPC, int ORD>
constexpr int col_threads() {
    return wg_threads<NP, LPC, ORD == 2>();
}

// (1+x)^gamma - 1 for the ideal-gas pressure ratio.  For |x| <= 1/64 the
// Taylor polynomial sum_{n=1..10} C(gamma, n) x^n is used (the first neglected
// term is below 2^-66 |gamma x|, far under one ulp); otherwise
// expm1(gamma log1p(x)).  That general branch is kept out of line: inlined,
// the compiler hoists its polynomial constants out of the chunk loop, where
// they hold about 30 registers for the whole kernel.
__device__ __noinline__ double pow1p_minus1_far(double x, double gamma) {
    return expm1(gamma * log1p(x));
}
__device__ __forceinline__ double pow1p_minus1(const DevMesh& m, double x) {
    if (fabs(x) <= 1.0 / 64.0) {
        double s = m.binom[10];
#pragma unroll
        for (int n = 9; n >= 1; --n) s = s * x + m.binom[n];
        return s * x;
    }
    return pow1p_minus1_far(x, m.gamma);
}

// At least four waves per SIMD: two workgroups share a CU, so that one can
// compute while the other waits on memory.  The instance with the sub-grid
// stress (DISS) needs about 155 VGPRs in the planes-first and natural orders:
// held to 128 it spilled some 40 of them and ran 15% slower than with the
// bound relaxed to two waves (it then runs at three).  In the split-element
// order it needs about 150; held to 128 it spills about 20 and runs 13%
// faster than at three waves, so that order keeps the bound of four.
// Within a workgroup the global
// loads of a chunk are issued one phase early: while the derivatives of chunk
// ch run, the update base of its nodes, the next chunk's q_s (direct nodes)
// and the next chunk's slice of the per-level tables are already in flight.
// TER: terrain-following coordinates.  The columns keep their
// horizontal boxes; with g_s = 1/(1 - zs/(H - z0)) per position and
// t_f = (H - zf)/(H - z0) per level, the chain rule of the mapping gives, with
// d/dzf the box derivative 2/dz d/dzeta,
//   d/dx = d/dx|box + a_x d/dzf,  d/dy = d/dy|box + a_y d/dzf,  d/dz = g_s d/dzf,
//   a_x = -t_f g_s dzs/dx,  a_y = -t_f g_s dzs/dy,
// so advection becomes the box horizontal part plus (u a_x + v a_y + w g_s) d/dzf.
// The lumped mass gains the factor 1/g_s = 1 - zs/(H - z0) per position; it
// still factorises into a horizontal part (assembled on the host with that
// factor, hanging positions through their rows) and the vertical one.
// Hanging positions take the coarse face's interpolant of zs and of the
// reference state (host tables), so the mesh stays watertight.
template <int NP, int LPC, typename T, bool TER, bool DISS, int ORD>
__global__ void __launch_bounds__((col_threads<NP, LPC, ORD>()), (DISS && ORD != 2) ? 2 : 4)
k_stage_columns(DevMesh m, FusedTables ft, int col0, int ncol, double a, double b, double c,
                const double* __restrict__ qn, const double* __restrict__ qs,
                double* __restrict__ qo) {
    constexpr int NP2 = NP * NP, N = NP - 1;
    constexpr int NK = LPC * N + 1;               // vertical nodes of a full chunk
    // LDS tile stride per position: one pad double at N = 4 (18 instead of
    // 17 at four layers per chunk: stages 1-1.5 % faster in the natural and
    // split-element orders and in float).  Not at N = 7: with two layers in
    // the split-element order a pad of one or two measured 7 % slower, with
    // the same count of LDS bank conflicts and more wave cycles waiting on
    // memory (its 16-wave workgroup runs one per CU either way)
    constexpr int TS = NK + (NP == 5 ? 1 : 0);
    constexpr bool SE = ORD == 2;
    // loads issued one phase early (next chunk's q_s, the update base after
    // the tile barrier): box elements always, terrain in the split order
    constexpr bool PRE = !TER || SE;
    constexpr int WGT = wg_threads<NP, LPC, SE>();
    __shared__ T tile[4][NP2 * TS];               // rho u, rho v, rho w, u: [field][p][kzl], kzl fastest
    __shared__ double carry[2][NF][NP2];
    __shared__ T sD[NP2];
    // per position and tap, the x and y coefficients side by side: one 2-wide
    // LDS read serves both derivatives of a call
    using T2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
    __shared__ T2 sDxy[NP2 * NP];
    // (v, w) and (p', theta'), always differentiated together: one 2-wide
    // element per node, so one LDS read per tap serves both fields
    __shared__ T2 tpr[2][NP2 * TS];
    __shared__ double sW[NP];
    // the chunk's slice of the per-level tables, double-buffered: rho0,
    // 1/rho0, 1/theta0, p0, dtheta0/dz, 1/M_v at its NK levels, then dz and
    // 2/dz of its LPC layers
    constexpr int SL = 6 * NK + 2 * LPC;
    __shared__ double slice[2][SL];
    // DISS: the sub-grid stress 2 nu (S_xx, S_xy, S_yy, S_xz, S_yz) of every
    // element of the chunk at its nodes, [component][position][element][k]
    constexpr int TAU = DISS ? NP2 * LPC * NP : 1;
    __shared__ double stau[DISS ? 5 : 1][TAU];
    const int tid = threadIdx.x;
    for (int t = tid; t < NP2; t += WGT) sD[t] = T(m.D[t]);
    for (int t = tid; t < NP2 * NP; t += WGT) {
        const int pp = t / NP, mm = t - pp * NP;
        sDxy[t].x = T(m.D[(pp % NP) * NP + mm]);
        sDxy[t].y = T(m.D[(pp / NP) * NP + mm]);
    }
    for (int t = tid; t < NP; t += WGT) sW[t] = m.w[t];
    // this thread's slice entry: source table, offset, step per chunk, limit
    const double* sl_src = nullptr;
    int sl_off = 0, sl_step = 0, sl_lim = 0;
    if (tid < 6 * NK) {
        const int tab = tid / NK;
        if constexpr (TER)   // reference per node instead; t_f in slot 0
            sl_src = tab == 0 ? m.tfac : tab == 5 ? m.minv_v : nullptr;
        else
            sl_src = tab == 0 ? m.rho0 : tab == 1 ? m.inv_rho0 : tab == 2 ? m.inv_theta0
                   : tab == 3 ? m.p0 : tab == 4 ? m.dth0 : m.minv_v;
        sl_off = tid - tab * NK;
        sl_step = LPC * (NP - 1);
        sl_lim = m.nzn;
    } else if (tid < SL) {
        const int e = tid - 6 * NK;
        sl_src = e < LPC ? m.dz : m.sz;
        sl_off = e < LPC ? e : e - LPC;
        sl_step = LPC;
        sl_lim = m.n_z;
    }
    auto slice_value = [&](int ch2) {
        const int k = sl_off + ch2 * sl_step;
        if constexpr (TER) return (sl_src && k < sl_lim) ? sl_src[k] : 0.0;
        else return k < sl_lim ? sl_src[k] : 0.0;
    };
    if (tid < SL) slice[0][tid] = slice_value(0);

    // Workgroups start in block order (and go to the 8 XCDs round-robin);
    // the plan lists each colour's columns by decreasing work, so that the
    // costliest start first and the last, partly filled round of resident
    // workgroups holds the cheapest.  Columns of one colour share no node and
    // no cache line, so their order does not matter to the L2s.
    const int item = blockIdx.x;
    const int col = ft.col_order[col0 + min(item, ncol - 1)];

    // Thread -> node of the chunk, by the thread order ORD.
    //  1 (and always in float): natural, kzl fastest within a position, so
    //    that the global loads and stores of a wave cover few rows and lines;
    //    every wave then carries the same LDS load.  A position's first
    //    LPC*N nodes take consecutive threads and the chunk's top plane (the
    //    next chunk's bottom) follows in the last threads: at N = 4 with four
    //    layers a wave then holds four whole 16-node row segments, each one
    //    aligned 128-byte line per field, instead of 17-node segments that
    //    straddle two lines and start anywhere in a wave.
    //  0 (FP64): nodes on the planes between two stacked elements (LPC-1 per
    //    position, two z derivatives each) come first, so that they fill
    //    waves of their own instead of making every wave run a second pass of
    //    FP64 z derivatives with most lanes masked, and so that these longest
    //    waves are the oldest, which issue first; nodes inside an element or
    //    on the chunk's bottom/top follow (RG per position).
    //  2 (SE, FP64): a thread per (element, local node) of each position,
    //    elements in order; the lower thread of a plane between two elements
    //    (dupe) only computes its element's part and hands it to the next lane.
    // Which order is faster depends on the order N, the chunk depth and the
    // terms (the autotuner times all three).
    constexpr int RG = LPC * (N - 1) + 2;
    int kzl, p;
    int el_t = 0, kk_t = 0;                       // SE: the thread's element and local node
    if constexpr (SE) {
        constexpr int NE = LPC * NP;
        p = tid < NP2 * NE ? tid / NE : NP2;
        const int r = tid < NP2 * NE ? tid - p * NE : 0;
        el_t = r / NP;
        kk_t = r - el_t * NP;
        kzl = el_t * N + kk_t;
    } else if constexpr (ORD == 1) {
        constexpr int NB = NK - 1;                // nodes below the chunk's top plane
        if (tid < NP2 * NB) {
            p = tid / NB;
            kzl = tid - p * NB;
        } else if (tid < NP2 * NK) {
            p = tid - NP2 * NB;
            kzl = NB;
        } else {
            p = NP2;
            kzl = 0;
        }
    } else {
        constexpr int NI = (LPC > 1) ? NP2 * (LPC - 1) : 0;
        if (tid < NI) {
            p = tid / (LPC - 1 > 0 ? LPC - 1 : 1);
            kzl = (tid - p * (LPC - 1) + 1) * N;
        } else if (tid < NI + NP2 * RG) {
            const int t2 = tid - NI;
            p = t2 / RG;
            const int r = t2 - p * RG;
            if (r == 0) kzl = 0;
            else if (r == RG - 1) kzl = NK - 1;
            else if constexpr (N > 1) kzl = ((r - 1) / (N - 1)) * N + (r - 1) % (N - 1) + 1;
            else kzl = 0;
        } else {
            p = NP2;
            kzl = 0;
        }
    }
    __shared__ double s_zs[TER ? NP2 : 1];
    __shared__ double s_ter[TER ? 4 : 1][TER ? NP2 : 1];   // g_s, g_s dzs/dx, g_s dzs/dy, 1/g_s
    if constexpr (TER) {
        for (int t = tid; t < NP2; t += WGT) {
            const int gz = ft.gmap[col * NP2 + t];
            s_zs[t] = m.zs[gz >= 0 ? gz : ft.hreal[-gz - 1]];
        }
    }
    const bool lane_ok = (p < NP2) && (item < ncol);
    const int pc = lane_ok ? p : 0;               // position used for table lookups
    const int i = pc % NP, j = pc / NP;
    const int nzn = m.nzn;
    const int64_t fs = int64_t(m.n_h) * m.ldz;
    const int64_t fsh = ft.fsh;
    const int64_t fsr = int64_t(m.n_h + m.n_hh) * m.ldz;   // terrain reference rows

    int g = 0, r_beg = 0, r_end = 0;
    bool first = false;
    const double dxc = m.col_dx[col], dyc = m.col_dy[col];
    const T sx = T(m.col_sx[col]), sy = T(m.col_sy[col]);
    if (lane_ok) {
        g = ft.gmap[col * NP2 + pc];
        first = ft.first[col * NP2 + pc] != 0;
        if (g < 0) {
            r_beg = ft.hang_ptr[-g - 1];
            r_end = ft.hang_ptr[-g];
        }
    }
    // q_s of the next chunk (direct nodes).  Split-element order: the first
    // chunk's is requested here already, so that it arrives while the
    // per-position tables are set up (in the other orders that measured
    // slower, so their first chunk loads in the chunk loop)
    double pf[NF] = {0, 0, 0, 0, 0};
    if constexpr (SE) {
        const bool act0 = lane_ok && el_t < min(LPC, m.n_z);
        if (act0 && g >= 0) {
            const int64_t o = int64_t(g) * m.ldz + kzl;
#pragma unroll
            for (int f = 0; f < NF; ++f) pf[f] = qs[f * fs + o];
        }
    }
    // per-position constants in LDS rather than in every thread's registers:
    // the horizontal inverse mass and the horizontal mass weight
    __shared__ double s_mh[NP2], s_mij[NP2];
    // row offset g * ldz of every direct position (read where needed rather
    // than kept in registers across the chunk loop)
    __shared__ int64_t s_row[NP2];
    // terrain: row offset of every position's reference rows (hanging points
    // after the unique nodes)
    __shared__ int64_t s_rrow[TER ? NP2 : 1];
    for (int t = tid; t < NP2; t += WGT) {
        const int gt = ft.gmap[col * NP2 + t];
        s_mh[t] = gt >= 0 ? (TER ? m.minv_ht[gt] : m.minv_h[gt]) : 0.0;
        s_row[t] = gt >= 0 ? int64_t(gt) * m.ldz : 0;
        if constexpr (TER) s_rrow[t] = int64_t(gt >= 0 ? gt : ft.hreal[-gt - 1]) * m.ldz;
    }
    __syncthreads();
    for (int t = tid; t < NP2; t += WGT) s_mij[t] = sW[t % NP] * sW[t / NP] * 0.125 * dxc * dyc;
    const T2* Dxy = &sDxy[pc * NP];
    const int lx0 = (j * NP) * TS + kzl, ly0 = i * TS + kzl;
    // terrain: g_s and g_s times the box derivatives of zs per position (LDS)
    if constexpr (TER) {
        for (int t = tid; t < NP2; t += WGT) {
            const int ti = t % NP, tj = t / NP;
            double zx = 0.0, zy = 0.0;
            for (int mm = 0; mm < NP; ++mm) {
                zx += double(sD[ti * NP + mm]) * s_zs[tj * NP + mm];
                zy += double(sD[tj * NP + mm]) * s_zs[mm * NP + ti];
            }
            const double gs = 1.0 / (1.0 - s_zs[t] * m.inv_depth);
            s_ter[0][t] = gs;
            s_ter[1][t] = gs * zx * m.col_sx[col];
            s_ter[2][t] = gs * zy * m.col_sy[col];
            s_ter[3][t] = 1.0 - s_zs[t] * m.inv_depth;
        }
        __syncthreads();
    }

    const int n_chunk = (m.n_z + LPC - 1) / LPC;
    for (int ch = 0; ch < n_chunk; ++ch) {
        const int L0 = ch * LPC;
        const int L1 = min(L0 + LPC, m.n_z);
        const int nk = (L1 - L0) * N + 1;
        bool active = lane_ok && (kzl < nk);
        // SE: the lower thread of a plane between two elements of the chunk
        // only computes (dupe); the node's other work is its upper thread's
        bool dupe = false;
        if constexpr (SE) {
            active = lane_ok && el_t < L1 - L0;
            dupe = kk_t == N && el_t + 1 < L1 - L0;
        }
        const int kz = L0 * N + kzl;
        const int lidx = pc * TS + kzl;
        double qv[NF] = {0, 0, 0, 0, 0};
        T rho = T(1);
        if (active) {
            if (g >= 0) {
                if (PRE && (SE || ch > 0)) {
#pragma unroll
                    for (int f = 0; f < NF; ++f) qv[f] = pf[f];
                } else {
                    const int64_t o = s_row[pc] + kz;
#pragma unroll
                    for (int f = 0; f < NF; ++f) qv[f] = qs[f * fs + o];
                }
            } else {
                for (int r = r_beg; r < r_end; ++r) {
                    const double w = ft.hang_w[r];
                    const int64_t o = int64_t(ft.hang_src[r]) * m.ldz + kz;
#pragma unroll
                    for (int f = 0; f < NF; ++f) qv[f] += w * qs[f * fs + o];
                }
            }
            double r0d, irho0, ith0, p0v;
            if constexpr (TER) {
                // per node; hanging rows hold the coarse face's interpolant
                const int64_t o = s_rrow[pc] + kz;
                r0d = m.ref_n[o];
                irho0 = m.ref_n[fsr + o];
                ith0 = m.ref_n[2 * fsr + o];
                p0v = m.ref_n[3 * fsr + o];
            } else {
                const double* sp = slice[ch & 1];
                r0d = sp[kzl];
                irho0 = sp[NK + kzl];
                ith0 = sp[2 * NK + kzl];
                p0v = sp[3 * NK + kzl];
            }
            rho = T(r0d) + T(qv[0]);
            const T u = T(qv[1]), v = T(qv[2]), w = T(qv[3]);
            if (!dupe) {
            tile[0][lidx] = rho * u;
            tile[1][lidx] = rho * v;
            tile[2][lidx] = rho * w;
            tile[3][lidx] = u;
            {
                T2 vw;
                vw.x = v;
                vw.y = w;
                tpr[0][lidx] = vw;
            }
            {
                // p' = p0 ((rho theta)/(rho0 theta0))^gamma - p0 with x = a + b + a b,
                // a = rho'/rho0, b = theta'/theta0 (no cancellation against p0).
                // Evaluated in FP64 from the FP64 state in both precisions and
                // rounded once: the hydrostatic balance in the w tendency
                // cancels most of dp'/dz, so a float evaluation's few-ulp error
                // would dominate the float variant's error there.
                const double ra = qv[0] * irho0, tb = qv[4] * ith0;
                T2 pt;
                pt.x = T(p0v * pow1p_minus1(m, ra + tb + ra * tb));
                pt.y = T(qv[4]);
                tpr[1][lidx] = pt;
            }
            }
        }
        __syncthreads();
        // update base of the nodes finished in this chunk (q^n for the first
        // contributor, not read when a = 0; the partial q_out for later colours)
        double base[NF] = {0, 0, 0, 0, 0};
        if (PRE && active && !dupe && g >= 0 && !(kzl == nk - 1 && L1 < m.n_z) && (!first || a != 0.0)) {
            const double* bp = first ? qn : qo;
            const int64_t o = s_row[pc] + kz;
#pragma unroll
            for (int f = 0; f < NF; ++f) base[f] = bp[f * fs + o];
        }
        const double* sb = slice[ch & 1];
        double sl_next = 0.0;
        if (tid < SL && ch + 1 < n_chunk) sl_next = slice_value(ch + 1);
        // prefetch the next chunk's q_s (PRE: box elements, and terrain in
        // the split-element order; the other terrain instances need those
        // registers for their metric terms)
        if (PRE && ch + 1 < n_chunk && lane_ok && g >= 0) {
            const int L0n = L0 + LPC;
            const int neln = min(L0n + LPC, m.n_z) - L0n;
            if (SE ? el_t < neln : kzl < neln * N + 1) {
                const int64_t o = s_row[pc] + L0n * N + kzl;
#pragma unroll
                for (int f = 0; f < NF; ++f) pf[f] = qs[f * fs + o];
            }
        }
        double acc[NF] = {0, 0, 0, 0, 0};
        // derivatives and the node's contribution (acc) from the elements of the chunk
        if (active) {
            // d/dx of tiles tx, tx2 and d/dy of tiles ty, ty2 at this node.  The
            // empty asm pins the results before the next fields' LDS reads may
            // be issued (memory clobber), which bounds the live registers; it
            // also makes the LGL coefficients be read from LDS again after it,
            // so each call serves two fields with one read of each coefficient
            // (that halves the coefficient reads, about a quarter of the LDS
            // traffic of the derivative phase).
            auto dxy = [&](int tx, int ty, int tx2, int ty2, T& ox, T& oy, T& ox2, T& oy2) {
                T ax = 0, ay = 0, ax2 = 0, ay2 = 0;
#pragma unroll
                for (int mm = 0; mm < NP; ++mm) {
                    const T2 cxy = Dxy[mm];
                    const T cx = cxy.x, cy = cxy.y;
                    ax += cx * tile[tx][lx0 + mm * TS];
                    ay += cy * tile[ty][ly0 + mm * NP * TS];
                    ax2 += cx * tile[tx2][lx0 + mm * TS];
                    ay2 += cy * tile[ty2][ly0 + mm * NP * TS];
                }
                asm volatile("" : "+v"(ax), "+v"(ay), "+v"(ax2), "+v"(ay2) : : "memory");
                ox = ax * sx;
                oy = ay * sy;
                ox2 = ax2 * sx;
                oy2 = ay2 * sy;
            };
            // the same for the two fields of a pair
            auto dxyp = [&](int pr, T& ox, T& oy, T& ox2, T& oy2) {
                T ax = 0, ay = 0, ax2 = 0, ay2 = 0;
#pragma unroll
                for (int mm = 0; mm < NP; ++mm) {
                    const T2 cxy = Dxy[mm];
                    const T cx = cxy.x, cy = cxy.y;
                    const T2 a = tpr[pr][lx0 + mm * TS], b = tpr[pr][ly0 + mm * NP * TS];
                    ax += cx * a.x;
                    ay += cy * b.x;
                    ax2 += cx * a.y;
                    ay2 += cy * b.y;
                }
                asm volatile("" : "+v"(ax), "+v"(ay), "+v"(ax2), "+v"(ay2) : : "memory");
                ox = ax * sx;
                oy = ay * sy;
                ox2 = ax2 * sx;
                oy2 = ay2 * sy;
            };
            const T u = T(qv[1]), v = T(qv[2]), w = T(qv[3]);
            const T inv_rho = T(1) / rho;
            const T f = T(m.f), gr = T(m.g);
            // the parts of R without z derivatives
            T Rh[NF], ax, ay, bx, by;
            double gxy[6] = {0, 0, 0, 0, 0, 0};   // DISS: du/dx, du/dy, dv/dx, dv/dy, dw/dx, dw/dy
            dxy(0, 1, 3, 3, ax, ay, bx, by);
            Rh[0] = -(ax + ay);
            Rh[1] = -(u * bx + v * by) + f * v;
            if constexpr (DISS) { gxy[0] = bx; gxy[1] = by; }
            dxyp(0, ax, ay, bx, by);
            Rh[2] = -(u * ax + v * ay) - f * u;
            Rh[3] = -(u * bx + v * by) - T(qv[0]) * inv_rho * gr;
            if constexpr (DISS) { gxy[2] = ax; gxy[3] = ay; gxy[4] = bx; gxy[5] = by; }
            dxyp(1, bx, by, ax, ay);
            Rh[1] -= bx * inv_rho;
            Rh[2] -= by * inv_rho;
            if constexpr (TER) {
                Rh[4] = -(u * ax + v * ay) - w * T(m.ref_n[4 * fsr + s_rrow[pc] + kz]);
            }
            else Rh[4] = -(u * ax + v * ay) - w * T(sb[4 * NK + kzl]);
            // terrain: a_x, a_y and the advecting vertical speed per node
            T a_x = 0, a_y = 0, wt = w, gs = 1;
            if constexpr (TER) {
                const double tf = sb[kzl];
                gs = T(s_ter[0][pc]);
                a_x = T(-tf * s_ter[1][pc]);
                a_y = T(-tf * s_ter[2][pc]);
                wt = u * a_x + v * a_y + w * gs;
            }
            // elements of this chunk holding the node: (element, local k)
            const bool inner_plane = (kzl % N == 0) && kzl > 0 && kzl < nk - 1;
            const int e_first = SE ? el_t : (kzl == nk - 1) ? (kzl - 1) / N : (inner_plane ? kzl / N - 1 : kzl / N);
            const int n_el = (!SE && inner_plane) ? 2 : 1;
            for (int s2 = 0; s2 < n_el; ++s2) {
                const int el = e_first + s2;
                const int kk = kzl - el * N;
                const double dzl = sb[6 * NK + el];
                const T sz = T(sb[6 * NK + LPC + el]);
                const T* Dz = &sD[kk * NP];
                const int lz0 = pc * TS + el * N;
                // two fields per call, as for d/dx and d/dy
                auto ddz = [&](int tz, int tz2, T& oz, T& oz2) {
                    T az = 0, az2 = 0;
#pragma unroll
                    for (int mm = 0; mm < NP; ++mm) {
                        const T cz = Dz[mm];
                        az += cz * tile[tz][lz0 + mm];
                        az2 += cz * tile[tz2][lz0 + mm];
                    }
                    asm volatile("" : "+v"(az), "+v"(az2) : : "memory");
                    oz = az * sz;
                    oz2 = az2 * sz;
                };
                auto ddzp = [&](int pr, T& oz, T& oz2) {
                    T az = 0, az2 = 0;
#pragma unroll
                    for (int mm = 0; mm < NP; ++mm) {
                        const T cz = Dz[mm];
                        const T2 a = tpr[pr][lz0 + mm];
                        az += cz * a.x;
                        az2 += cz * a.y;
                    }
                    asm volatile("" : "+v"(az), "+v"(az2) : : "memory");
                    oz = az * sz;
                    oz2 = az2 * sz;
                };
                T R[NF], z0, z1;
                if constexpr (TER) {
                    ddzp(1, z0, z1);
                    const T pz = z0 * inv_rho;
                    R[4] = Rh[4] - wt * z1;
                    ddzp(0, z0, z1);
                    R[2] = Rh[2] - wt * z0 - a_y * pz;
                    R[3] = Rh[3] - wt * z1 - gs * pz;
                    T z2, z3;
                    ddz(0, 1, z0, z1);
                    ddz(2, 3, z2, z3);
                    R[0] = Rh[0] - (a_x * z0 + a_y * z1 + gs * z2);
                    R[1] = Rh[1] - wt * z3 - a_x * pz;
                } else {
                    ddz(2, 3, z0, z1);
                    R[0] = Rh[0] - z0;
                    R[1] = Rh[1] - w * z1;
                    double guz = 0.0;
                    if constexpr (DISS) guz = z1;
                    ddzp(0, z0, z1);
                    R[2] = Rh[2] - w * z0;
                    if constexpr (DISS) {
                        // the element's strain (Section 5, sub-grid model):
                        // S = (grad u + grad u^T)/2, nu = (Cs Delta)^2 sqrt(2 S:S),
                        // Delta = (dx + dy)/(2N); the stress 2 nu S goes to LDS
                        const double sxx = gxy[0], syy = gxy[3], szz = z1;
                        const double sxy = 0.5 * (gxy[1] + gxy[2]);
                        const double sxz = 0.5 * (guz + gxy[4]);
                        const double syz = 0.5 * (double(z0) + gxy[5]);
                        const double ss = sxx * sxx + syy * syy + szz * szz +
                                          2.0 * (sxy * sxy + sxz * sxz + syz * syz);
                        const double cd = m.cs * (dxc + dyc) / (2.0 * N);
                        const double two_nu = 2.0 * cd * cd * sqrt(2.0 * ss);
                        const int ti = pc * (LPC * NP) + el * NP + kk;
                        stau[0][ti] = two_nu * sxx;
                        stau[1][ti] = two_nu * sxy;
                        stau[2][ti] = two_nu * syy;
                        stau[3][ti] = two_nu * sxz;
                        stau[4][ti] = two_nu * syz;
                    }
                    T z2, z3;
                    ddzp(1, z2, z3);
                    R[3] = Rh[3] - w * z1 - z2 * inv_rho;
                    R[4] = Rh[4] - w * z3;
                }
                const double mass = s_mij[pc] * sW[kk] * dzl;
                {
                    // each element's part rounded on its own (no fused
                    // multiply-add into the sum), as the split order forms it
#pragma clang fp contract(off)
#pragma unroll
                    for (int fl = 0; fl < NF; ++fl) acc[fl] += mass * double(R[fl]);
                }
                if constexpr (DISS) {
                    // absorbing layer: -R(z) q' for every field
                    if (m.sponge) {
                        const double rz = m.sponge[kz] * mass;
#pragma unroll
                        for (int fl = 0; fl < NF; ++fl) acc[fl] -= rz * qv[fl];
                    }
                }
            }
        }
        // DISS: horizontal divergence of each element's stress at the node,
        // once every node has written its elements' entries of the stress tile
        if constexpr (DISS) {
            __syncthreads();
            if (active && m.cs > 0.0) {
                const bool inner_plane = (kzl % N == 0) && kzl > 0 && kzl < nk - 1;
                const int e_first = SE ? el_t : (kzl == nk - 1) ? (kzl - 1) / N : (inner_plane ? kzl / N - 1 : kzl / N);
                const int n_el = (!SE && inner_plane) ? 2 : 1;
                for (int s2 = 0; s2 < n_el; ++s2) {
                    const int el = e_first + s2;
                    const int kk = kzl - el * N;
                    const double mass = s_mij[pc] * sW[kk] * sb[6 * NK + el];
                    const int tx0 = (j * NP) * (LPC * NP) + el * NP + kk;
                    const int ty0 = i * (LPC * NP) + el * NP + kk;
                    double dx[3] = {0, 0, 0}, dy[3] = {0, 0, 0};
#pragma unroll
                    for (int mm = 0; mm < NP; ++mm) {
                        const T2 cxy = Dxy[mm];
                        const int ox = tx0 + mm * (LPC * NP), oy = ty0 + mm * NP * (LPC * NP);
                        dx[0] += double(cxy.x) * stau[0][ox];   // d/dx S_xx
                        dx[1] += double(cxy.x) * stau[1][ox];   // d/dx S_xy
                        dx[2] += double(cxy.x) * stau[3][ox];   // d/dx S_xz
                        dy[0] += double(cxy.y) * stau[1][oy];   // d/dy S_xy
                        dy[1] += double(cxy.y) * stau[2][oy];   // d/dy S_yy
                        dy[2] += double(cxy.y) * stau[4][oy];   // d/dy S_yz
                    }
                    const double sxd = double(sx), syd = double(sy);
                    acc[1] += mass * (dx[0] * sxd + dy[0] * syd);
                    acc[2] += mass * (dx[1] * sxd + dy[1] * syd);
                    acc[3] += mass * (dx[2] * sxd + dy[2] * syd);
                }
            }
        }
        // SE: the lower element's part of a plane node, from the previous
        // lane (summed in the order of the other thread orders)
        if constexpr (SE) {
#pragma unroll
            for (int fl = 0; fl < NF; ++fl) {
                const double lo = __shfl_up(acc[fl], 1);
                if (active && kk_t == 0 && el_t > 0) acc[fl] = lo + acc[fl];
            }
        }
        // the carry of the chunk's top plane, or the node's update
        if (active && !dupe) {
            if (kzl == nk - 1 && L1 < m.n_z) {
                // top plane of the chunk: finished by the next chunk
#pragma unroll
                for (int fl = 0; fl < NF; ++fl) carry[ch & 1][fl][pc] = acc[fl];
            } else {
                if (kzl == 0 && ch > 0) {
#pragma unroll
                    for (int fl = 0; fl < NF; ++fl) acc[fl] += carry[(ch - 1) & 1][fl][pc];
                }
                if constexpr (TER) {
                    // mapped lumped mass: the box mass times 1 - zs/(H - z0)
                    const double mf = s_ter[3][pc];
#pragma unroll
                    for (int fl = 0; fl < NF; ++fl) acc[fl] *= mf;
                }
                if (g >= 0) {
                    bool lid = (kz == 0) || (kz == nzn - 1);
                    if constexpr (TER) {
                        // terrain surface: drop the momentum tendency along the
                        // unit normal (the top stays a rigid lid)
                        if (kz == 0) {
                            const double n0 = m.nrm[g], n1 = m.nrm[m.n_h + g], n2 = m.nrm[2 * m.n_h + g];
                            const double dn = acc[1] * n0 + acc[2] * n1 + acc[3] * n2;
                            acc[1] -= dn * n0;
                            acc[2] -= dn * n1;
                            acc[3] -= dn * n2;
                        }
                        lid = (kz == nzn - 1);
                    }
                    const double mi = c * s_mh[pc] * sb[5 * NK + kzl];
                    const int64_t o = s_row[pc] + kz;
                    if (!PRE && (!first || a != 0.0)) {
                        // the terrain instances outside the split-element
                        // order load their base here (registers)
                        const double* bp = first ? qn : qo;
#pragma unroll
                        for (int f = 0; f < NF; ++f) base[f] = bp[f * fs + o];
                    }
                    if (first) {
                        // the dissipation pre-pass (if any) is already assembled:
                        // the first contributor adds it once
                        double rx[NF] = {0, 0, 0, 0, 0};
                        if (m.rx) {
#pragma unroll
                            for (int fl = 0; fl < NF; ++fl) rx[fl] = c * m.rx[fl * fs + o];
                        }
#pragma unroll
                        for (int fl = 0; fl < NF; ++fl) {
                            const double tend = (fl == 3 && lid) ? 0.0 : mi * acc[fl];
                            qo[fl * fs + o] = a * base[fl] + b * qv[fl] + tend + rx[fl];
                        }
                    } else {
#pragma unroll
                        for (int fl = 0; fl < NF; ++fl)
                            if (!(fl == 3 && lid)) qo[fl * fs + o] = base[fl] + mi * acc[fl];
                    }
                } else {
                    const int64_t o = int64_t(-g - 1) * m.ldz + kz;
                    if (first) {
#pragma unroll
                        for (int fl = 0; fl < NF; ++fl) ft.cH[fl * fsh + o] = acc[fl];
                    } else {
#pragma unroll
                        for (int fl = 0; fl < NF; ++fl) ft.cH[fl * fsh + o] += acc[fl];
                    }
                }
            }
        }
        if (tid < SL && ch + 1 < n_chunk) slice[(ch + 1) & 1][tid] = sl_next;
        __syncthreads();
    }
}

// Z^T: coarse face nodes receive the hanging-point contributions
__global__ void k_stage_hanging(DevMesh m, FusedTables ft, double c, double* __restrict__ qo) {
    const int nzn = m.nzn;
    const int64_t n = int64_t(m.n_hT) * nzn;
    const int64_t fs = int64_t(m.n_h) * m.ldz;
    const int64_t fsh = ft.fsh;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int li = int(t / nzn), kz = int(t - int64_t(li) * nzn);
        const int h = m.hT_list[li];
        double s[NF] = {0, 0, 0, 0, 0};
        for (int r = m.hT_ptr[li]; r < m.hT_ptr[li + 1]; ++r) {
            const double w = m.hT_w[r];
            const int64_t o = int64_t(m.hT_hh[r]) * m.ldz + kz;
#pragma unroll
            for (int f = 0; f < NF; ++f) s[f] += w * ft.cH[f * fsh + o];
        }
        bool lid = (kz == 0) || (kz == nzn - 1);
        double mi = c * m.minv_h[h] * m.minv_v[kz];
        if (m.zs) {
            // terrain: mapped masses; at the surface drop the momentum
            // tendency along the normal (linear, so per contribution)
            mi = c * m.minv_ht[h] * m.minv_v[kz];
            if (kz == 0) {
                const double n0 = m.nrm[h], n1 = m.nrm[m.n_h + h], n2 = m.nrm[2 * m.n_h + h];
                const double dn = s[1] * n0 + s[2] * n1 + s[3] * n2;
                s[1] -= dn * n0;
                s[2] -= dn * n1;
                s[3] -= dn * n2;
            }
            lid = (kz == nzn - 1);
        }
        const int64_t o = int64_t(h) * m.ldz + kz;
#pragma unroll
        for (int f = 0; f < NF; ++f)
            if (!(f == 3 && lid)) qo[f * fs + o] += mi * s[f];
    }
}

// Block kernel.  A workgroup owns one vertical segment of a 2 x 2 block of
// columns of one level and marches up through it one layer (one element per
// column) at a time; one thread per node of the block's (2N+1) x (2N+1)
// positions and the layer's N+1 planes.  The block's own faces (the plane
// x = x_mid of its two columns in x, y = y_mid likewise) are summed inside
// the workgroup: a node there belongs to two (four at the centre) of the
// block's elements, which differ only in the derivative across that face, so
// the thread sums the x (y) derivative parts of its elements, weights the
// other horizontal direction and the pointwise terms by the element count,
// and takes one z derivative per element of the layer.  Only the block's
// outer faces are shared with other blocks (read-modify-write across
// colours), and only the segment's end planes with the neighbouring segments.
template <int NP>
constexpr int blk_threads() {
    return (((2 * NP - 1) * (2 * NP - 1) * NP + 63) / 64) * 64;
}

template <int NP, typename T>
__global__ void __launch_bounds__(blk_threads<NP>(), 4)
k_stage_blocks(DevMesh m, BlockTables bt, int b0, int nblk, int seg_par, int n_iseg, double a,
               double b, double c, const double* __restrict__ qn, const double* __restrict__ qs,
               double* __restrict__ qo) {
    constexpr int N = NP - 1, NK = NP, PX = 2 * N + 1, PP = PX * PX;
    constexpr int NA = 4 * N * N;                 // positions inside the block's faces
    constexpr int WGT = blk_threads<NP>();
    using T2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
    __shared__ T tile[4][PP * NK];                // rho u, rho v, rho w, u: [field][p][kzl]
    __shared__ T2 tpr[2][PP * NK];                // (v, w), (p', theta')
    __shared__ double carry[2][NF][PP];
    __shared__ T sD[NP * NP];
    __shared__ T2 sDxy[NP * NP * NP];
    __shared__ double sW[NP];
    constexpr int SL = 6 * NK + 2;                // rho0, 1/rho0, 1/theta0, p0, dth0, 1/M_v; dz, 2/dz
    __shared__ double slice[2][SL];
    __shared__ double s_mh[PP], s_mij[PP];
    __shared__ int64_t s_row[PP];
    const int tid = threadIdx.x;
    for (int t = tid; t < NP * NP; t += WGT) sD[t] = T(m.D[t]);
    for (int t = tid; t < NP * NP * NP; t += WGT) {
        const int pp = t / NP, mm = t - pp * NP;
        sDxy[t].x = T(m.D[(pp % NP) * NP + mm]);
        sDxy[t].y = T(m.D[(pp / NP) * NP + mm]);
    }
    for (int t = tid; t < NP; t += WGT) sW[t] = m.w[t];

    // work item: (block, segment of this launch's parity), blocks of one
    // XCD contiguous in the colour's (Morton-ordered) list
    const int G = gridDim.x;
    const int xcd = blockIdx.x & 7, rr = blockIdx.x >> 3;
    const int item = xcd * (G >> 3) + min(xcd, G & 7) + rr;
    const int bi = min(item / n_iseg, nblk - 1);
    const int seg = 2 * (item - (item / n_iseg) * n_iseg) + seg_par;
    const int blk = bt.order[b0 + bi];
    const int Lb = seg * bt.Ls, Le = min(Lb + bt.Ls, m.n_z);
    const int nl = Le - Lb;                       // layers (chunks) of the segment

    // slice entry of this thread: source table, offset in the layer
    const double* sl_src = nullptr;
    int sl_off = 0, sl_lim = 0, sl_step = 0;
    if (tid < 6 * NK) {
        const int tab = tid / NK;
        sl_src = tab == 0 ? m.rho0 : tab == 1 ? m.inv_rho0 : tab == 2 ? m.inv_theta0
               : tab == 3 ? m.p0 : tab == 4 ? m.dth0 : m.minv_v;
        sl_off = tid - tab * NK;
        sl_step = N;
        sl_lim = m.nzn;
    } else if (tid < SL) {
        sl_src = tid == 6 * NK ? m.dz : m.sz;
        sl_step = 1;
        sl_lim = m.n_z;
    }
    auto slice_value = [&](int L) {
        const int k = sl_off + L * sl_step;
        return (sl_src && k < sl_lim) ? sl_src[k] : 0.0;
    };
    if (tid < SL) slice[0][tid] = slice_value(Lb);

    // thread -> (position, plane): positions inside the block's own faces
    // first (one element in x and y), then the face positions (two or four
    // elements), so that the longer work sits in the last waves
    const int rank = tid / NK, kzl = tid - rank * NK;
    int I = 0, J = 0, nx = 1, ny = 1;
    if (rank < NA) {
        I = rank % (2 * N);
        J = rank / (2 * N);
        I += (I >= N);
        J += (J >= N);
    } else if (rank < NA + 2 * N) {
        const int r = rank - NA;
        I = N;
        J = r + (r >= N);
        nx = 2;
    } else if (rank < NA + 4 * N) {
        const int r = rank - NA - 2 * N;
        J = N;
        I = r + (r >= N);
        ny = 2;
    } else {
        I = J = N;
        nx = ny = 2;
    }
    const bool lane_ok = rank < PP && item < nblk * n_iseg;
    const int p = lane_ok ? I + PX * J : 0;
    const int64_t fs = int64_t(m.n_h) * m.ldz;
    const int64_t fsh = bt.fsh;
    const int col = bt.blk_col[blk];
    const double dxc = m.col_dx[col], dyc = m.col_dy[col];
    const T sx = T(m.col_sx[col]), sy = T(m.col_sy[col]);
    int g = 0, r_beg = 0, r_end = 0;
    bool first_h = false;
    if (lane_ok) {
        g = bt.pos_g[int64_t(blk) * PP + p];
        first_h = bt.pos_first[int64_t(blk) * PP + p] != 0;
        if (g < 0) {
            r_beg = m.hang_ptr[-g - 1];
            r_end = m.hang_ptr[-g];
        }
    }
    for (int t = tid; t < PP; t += WGT) {
        const int gt = bt.pos_g[int64_t(blk) * PP + t];
        const int ti = t % PX, tj = t / PX;
        const int il = ti <= N ? ti : ti - N, jl = tj <= N ? tj : tj - N;
        s_mh[t] = gt >= 0 ? m.minv_h[gt] : 0.0;
        s_row[t] = gt >= 0 ? int64_t(gt) * m.ldz : 0;
        s_mij[t] = m.w[il] * m.w[jl] * 0.125 * dxc * dyc;
    }
    __syncthreads();
    // element-local indices along x and y (the left / lower element at a face)
    const int il0 = I <= N ? I : I - N, jl0 = J <= N ? J : J - N;
    const int qx0 = I < N ? 0 : (I > N ? 1 : 0), qy0 = J < N ? 0 : (J > N ? 1 : 0);
    const T nn = T(nx * ny);
    const int nt = nx > ny ? nx : ny;

    double pf[NF] = {0, 0, 0, 0, 0};              // q_s of the next layer (direct nodes)
    for (int ch = 0; ch < nl; ++ch) {
        const int L = Lb + ch;
        const int kz = L * N + kzl;
        const int lidx = p * NK + kzl;
        double qv[NF] = {0, 0, 0, 0, 0};
        T rho = T(1);
        const double* sp = slice[ch & 1];
        if (lane_ok) {
            if (g >= 0) {
                if (ch > 0) {
#pragma unroll
                    for (int f = 0; f < NF; ++f) qv[f] = pf[f];
                } else {
                    const int64_t o = s_row[p] + kz;
#pragma unroll
                    for (int f = 0; f < NF; ++f) qv[f] = qs[f * fs + o];
                }
            } else {
                for (int r = r_beg; r < r_end; ++r) {
                    const double w = m.hang_w[r];
                    const int64_t o = int64_t(m.hang_src[r]) * m.ldz + kz;
#pragma unroll
                    for (int f = 0; f < NF; ++f) qv[f] += w * qs[f * fs + o];
                }
            }
            const double r0d = sp[kzl], irho0 = sp[NK + kzl], ith0 = sp[2 * NK + kzl],
                         p0v = sp[3 * NK + kzl];
            rho = T(r0d) + T(qv[0]);
            const T u = T(qv[1]), v = T(qv[2]), w = T(qv[3]);
            tile[0][lidx] = rho * u;
            tile[1][lidx] = rho * v;
            tile[2][lidx] = rho * w;
            tile[3][lidx] = u;
            {
                T2 vw;
                vw.x = v;
                vw.y = w;
                tpr[0][lidx] = vw;
            }
            {
                // p' from the FP64 state without cancellation against p0
                const double ra = qv[0] * irho0, tb = qv[4] * ith0;
                T2 pt;
                pt.x = T(p0v * pow1p_minus1(m, ra + tb + ra * tb));
                pt.y = T(qv[4]);
                tpr[1][lidx] = pt;
            }
        }
        __syncthreads();
        // the node is finished in this layer unless it is the top plane of a
        // layer that is not the segment's last; the segment's end planes are
        // shared with the neighbouring segments, whose even member writes first
        const bool top_carry = (kzl == N) && (ch < nl - 1);
        const bool seg_end = (kzl == 0 && ch == 0 && seg > 0) || (kzl == N && ch == nl - 1 && Le < m.n_z);
        const bool first = first_h && !((seg & 1) && seg_end);
        double base[NF] = {0, 0, 0, 0, 0};
        if (lane_ok && g >= 0 && !top_carry && (!first || a != 0.0)) {
            const double* bp = first ? qn : qo;
            const int64_t o = s_row[p] + kz;
#pragma unroll
            for (int f = 0; f < NF; ++f) base[f] = bp[f * fs + o];
        }
        double sl_next = 0.0;
        if (tid < SL && ch + 1 < nl) sl_next = slice_value(L + 1);
        if (lane_ok && g >= 0 && ch + 1 < nl) {
            const int64_t o = s_row[p] + kz + N;
#pragma unroll
            for (int f = 0; f < NF; ++f) pf[f] = qs[f * fs + o];
        }
        if (lane_ok) {
            const T u = T(qv[1]), v = T(qv[2]), w = T(qv[3]);
            const T inv_rho = T(1) / rho;
            // derivative parts of the horizontal directions, summed over the
            // elements of the block holding the node: iteration t takes x
            // element min(t, nx-1) with weight ny (0 once t >= nx) and y
            // element min(t, ny-1) with weight nx (0 once t >= ny)
            T Rh[NF] = {0, 0, 0, 0, 0};
            for (int t = 0; t < nt; ++t) {
                const int ex = t < nx ? t : nx - 1, ey = t < ny ? t : ny - 1;
                const int qx = nx == 2 ? ex : qx0, qy = ny == 2 ? ey : qy0;
                const int il = nx == 2 ? (ex == 0 ? N : 0) : il0;
                const int jl = ny == 2 ? (ey == 0 ? N : 0) : jl0;
                const T wsx = t < nx ? sx * T(ny) : T(0), wsy = t < ny ? sy * T(nx) : T(0);
                const T2* Dxy = &sDxy[(il + NP * jl) * NP];
                const int lx0 = (qx * N + PX * J) * NK + kzl, ly0 = (I + PX * qy * N) * NK + kzl;
                auto dxy = [&](int tx, int ty, int tx2, int ty2, T& ox, T& oy, T& ox2, T& oy2) {
                    T ax = 0, ay = 0, ax2 = 0, ay2 = 0;
#pragma unroll
                    for (int mm = 0; mm < NP; ++mm) {
                        const T2 cxy = Dxy[mm];
                        ax += cxy.x * tile[tx][lx0 + mm * NK];
                        ay += cxy.y * tile[ty][ly0 + mm * PX * NK];
                        ax2 += cxy.x * tile[tx2][lx0 + mm * NK];
                        ay2 += cxy.y * tile[ty2][ly0 + mm * PX * NK];
                    }
                    asm volatile("" : "+v"(ax), "+v"(ay), "+v"(ax2), "+v"(ay2) : : "memory");
                    ox = ax * wsx;
                    oy = ay * wsy;
                    ox2 = ax2 * wsx;
                    oy2 = ay2 * wsy;
                };
                auto dxyp = [&](int pr, T& ox, T& oy, T& ox2, T& oy2) {
                    T ax = 0, ay = 0, ax2 = 0, ay2 = 0;
#pragma unroll
                    for (int mm = 0; mm < NP; ++mm) {
                        const T2 cxy = Dxy[mm];
                        const T2 va = tpr[pr][lx0 + mm * NK], vb = tpr[pr][ly0 + mm * PX * NK];
                        ax += cxy.x * va.x;
                        ay += cxy.y * vb.x;
                        ax2 += cxy.x * va.y;
                        ay2 += cxy.y * vb.y;
                    }
                    asm volatile("" : "+v"(ax), "+v"(ay), "+v"(ax2), "+v"(ay2) : : "memory");
                    ox = ax * wsx;
                    oy = ay * wsy;
                    ox2 = ax2 * wsx;
                    oy2 = ay2 * wsy;
                };
                T ax, ay, bx, by;
                dxy(0, 1, 3, 3, ax, ay, bx, by);
                Rh[0] -= ax + ay;
                Rh[1] -= u * bx + v * by;
                dxyp(0, ax, ay, bx, by);
                Rh[2] -= u * ax + v * ay;
                Rh[3] -= u * bx + v * by;
                dxyp(1, bx, by, ax, ay);
                Rh[1] -= bx * inv_rho;
                Rh[2] -= by * inv_rho;
                Rh[4] -= u * ax + v * ay;
            }
            // pointwise terms, once per element holding the node
            const T f = T(m.f), gr = T(m.g);
            Rh[1] += nn * (f * v);
            Rh[2] -= nn * (f * u);
            Rh[3] -= nn * (T(qv[0]) * inv_rho * gr);
            Rh[4] -= nn * (w * T(sp[4 * NK + kzl]));
            // z derivatives of the layer's element
            const T sz = T(sp[6 * NK + 1]) * nn;
            const T* Dz = &sD[kzl * NP];
            const int lz0 = p * NK;
            auto ddz = [&](int tz, int tz2, T& oz, T& oz2) {
                T az = 0, az2 = 0;
#pragma unroll
                for (int mm = 0; mm < NP; ++mm) {
                    const T cz = Dz[mm];
                    az += cz * tile[tz][lz0 + mm];
                    az2 += cz * tile[tz2][lz0 + mm];
                }
                asm volatile("" : "+v"(az), "+v"(az2) : : "memory");
                oz = az * sz;
                oz2 = az2 * sz;
            };
            auto ddzp = [&](int pr, T& oz, T& oz2) {
                T az = 0, az2 = 0;
#pragma unroll
                for (int mm = 0; mm < NP; ++mm) {
                    const T cz = Dz[mm];
                    const T2 va = tpr[pr][lz0 + mm];
                    az += cz * va.x;
                    az2 += cz * va.y;
                }
                asm volatile("" : "+v"(az), "+v"(az2) : : "memory");
                oz = az * sz;
                oz2 = az2 * sz;
            };
            T R[NF], z0, z1, z2, z3;
            ddz(2, 3, z0, z1);
            R[0] = Rh[0] - z0;
            R[1] = Rh[1] - w * z1;
            ddzp(0, z0, z1);
            R[2] = Rh[2] - w * z0;
            ddzp(1, z2, z3);
            R[3] = Rh[3] - w * z1 - z2 * inv_rho;
            R[4] = Rh[4] - w * z3;
            const double mass = s_mij[p] * sW[kzl] * sp[6 * NK];
            double acc[NF];
#pragma unroll
            for (int fl = 0; fl < NF; ++fl) acc[fl] = mass * double(R[fl]);
            if (top_carry) {
#pragma unroll
                for (int fl = 0; fl < NF; ++fl) carry[ch & 1][fl][p] = acc[fl];
            } else {
                if (kzl == 0 && ch > 0) {
#pragma unroll
                    for (int fl = 0; fl < NF; ++fl) acc[fl] += carry[(ch - 1) & 1][fl][p];
                }
                if (g >= 0) {
                    const bool lid = (kz == 0) || (kz == m.nzn - 1);
                    const double mi = c * s_mh[p] * sp[5 * NK + kzl];
                    const int64_t o = s_row[p] + kz;
                    if (first) {
                        double rx[NF] = {0, 0, 0, 0, 0};
                        if (m.rx) {
#pragma unroll
                            for (int fl = 0; fl < NF; ++fl) rx[fl] = c * m.rx[fl * fs + o];
                        }
#pragma unroll
                        for (int fl = 0; fl < NF; ++fl) {
                            const double tend = (fl == 3 && lid) ? 0.0 : mi * acc[fl];
                            qo[fl * fs + o] = a * base[fl] + b * qv[fl] + tend + rx[fl];
                        }
                    } else {
#pragma unroll
                        for (int fl = 0; fl < NF; ++fl)
                            if (!(fl == 3 && lid)) qo[fl * fs + o] = base[fl] + mi * acc[fl];
                    }
                } else {
                    const int64_t o = int64_t(-g - 1) * m.ldz + kz;
                    if (first) {
#pragma unroll
                        for (int fl = 0; fl < NF; ++fl) bt.cH[fl * fsh + o] = acc[fl];
                    } else {
#pragma unroll
                        for (int fl = 0; fl < NF; ++fl) bt.cH[fl * fsh + o] += acc[fl];
                    }
                }
            }
        }
        if (tid < SL && ch + 1 < nl) slice[(ch + 1) & 1][tid] = sl_next;
        __syncthreads();
    }
}

// Tail of a column-layout stage with side columns: every unique node that
// receives side-slot contributions or hanging-point contributions (Z^T) sums
// them in a fixed order and is finished here: written whole when no column
// launch wrote it first, else added to.
__global__ void k_stage_tail(DevMesh m, TailTables tl, double a, double b, double c,
                             const double* __restrict__ qn, const double* __restrict__ qs,
                             double* __restrict__ qo) {
    const int nzn = m.nzn;
    const int64_t n = int64_t(tl.n) * nzn;
    const int64_t fs = int64_t(m.n_h) * m.ldz;
    const int64_t fsh = tl.fsh;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int li = int(t / nzn), kz = int(t - int64_t(li) * nzn);
        const int h = tl.h[li];
        const bool fst = tl.first[li] != 0;
        const int64_t ob = int64_t(h) * m.ldz + kz;
        // the node's own values first: they depend only on the node, so
        // their round trips overlap the contribution sums below
        double bn[NF], bs[NF], br[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if (fst) {
                bn[f] = a != 0.0 ? qn[f * fs + ob] : 0.0;
                bs[f] = qs[f * fs + ob];
                br[f] = m.rx ? m.rx[f * fs + ob] : 0.0;
            } else {
                bn[f] = qo[f * fs + ob];
                bs[f] = 0.0;
                br[f] = 0.0;
            }
        }
        // the node's groups of contribution rows (side slots; per hanging
        // point of its Z^T row, that point and its side slots), each summed
        // and then added times its weight
        double s[NF] = {0, 0, 0, 0, 0}, v[NF] = {0, 0, 0, 0, 0};
        double wc = 0.0;
        for (int e = tl.eptr[li]; e < tl.eptr[li + 1]; ++e) {
            if (tl.estart[e]) {
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    s[f] += wc * v[f];
                    v[f] = 0.0;
                }
                wc = tl.ew[e];
            }
            const int row = tl.erow[e];
            if (row >= 0) {
                const int64_t o = int64_t(row) * m.ldz + kz;
#pragma unroll
                for (int f = 0; f < NF; ++f) v[f] += tl.cH[f * fsh + o];
            }
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) s[f] += wc * v[f];
        bool lid = (kz == 0) || (kz == nzn - 1);
        double mi = c * m.minv_h[h] * m.minv_v[kz];
        if (m.zs) {
            mi = c * m.minv_ht[h] * m.minv_v[kz];
            if (kz == 0) {
                const double n0 = m.nrm[h], n1 = m.nrm[m.n_h + h], n2 = m.nrm[2 * m.n_h + h];
                const double dn = s[1] * n0 + s[2] * n1 + s[3] * n2;
                s[1] -= dn * n0;
                s[2] -= dn * n1;
                s[3] -= dn * n2;
            }
            lid = (kz == nzn - 1);
        }
        const int64_t o = ob;
        if (fst) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const double tend = (f == 3 && lid) ? 0.0 : mi * s[f];
                const double rx = m.rx ? c * br[f] : 0.0;
                qo[f * fs + o] = (a != 0.0 ? a * bn[f] : 0.0) + b * bs[f] + tend + rx;
            }
        } else {
#pragma unroll
            for (int f = 0; f < NF; ++f)
                if (!(f == 3 && lid)) qo[f * fs + o] = bn[f] + mi * s[f];
        }
    }
}

// (order, layers per chunk) instances: at most 1024 threads and 117 KB of LDS
// per workgroup (the largest: N = 7, two layers, with the sub-grid stress; a CU
// has 160 KB)
#define SEM_FUSED_INSTANCES(X) \
    X(1, 1) X(1, 2) X(1, 4) X(1, 8) \
    X(2, 1) X(2, 2) X(2, 4) X(2, 8) \
    X(3, 1) X(3, 2) X(3, 4) X(3, 8) \
    X(4, 1) X(4, 2) X(4, 4) X(4, 8) \
    X(5, 1) X(5, 2) X(5, 4)         \
    X(6, 1) X(6, 2)                 \
    X(7, 1) X(7, 2)                 \
    X(8, 1)

template <typename T, bool TER, bool DISS, int ORD>
int launch_k(const DevMesh& m, const FusedTables& t, int col0, int ncol, double a, double b,
             double c, const double* qn, const double* qs, double* qo, hipStream_t s) {
    switch (m.N * 32 + t.layers_per_chunk) {
#define CASE(NN, LP)                                                                        \
    case NN * 32 + LP:                                                                      \
        hipLaunchKernelGGL((k_stage_columns<NN + 1, LP, T, TER, DISS,                       \
                                            eff_order<NN + 1, LP, T, ORD>()>),              \
                           dim3(ncol), dim3(col_threads<NN + 1, LP, eff_order<NN + 1, LP, T, ORD>()>()), \
                           0, s, m, t, col0, ncol, a, b, c, qn, qs, qo);                    \
        break;
        SEM_FUSED_INSTANCES(CASE)
#undef CASE
        default: return SEM_ERR_ARG;
    }
    return (hipGetLastError() == hipSuccess) ? SEM_OK : SEM_ERR_HIP;
}

// the float instances always take the natural thread order
template <typename T, bool TER, bool DISS = false>
int launch_t(const DevMesh& m, const FusedTables& t, int col0, int ncol, double a, double b,
             double c, const double* qn, const double* qs, double* qo, hipStream_t s) {
    if constexpr (sizeof(T) == 4)
        return launch_k<T, TER, DISS, 1>(m, t, col0, ncol, a, b, c, qn, qs, qo, s);
    else if (t.thread_order == 2)
        return launch_k<T, TER, DISS, 2>(m, t, col0, ncol, a, b, c, qn, qs, qo, s);
    else if (t.thread_order == 1)
        return launch_k<T, TER, DISS, 1>(m, t, col0, ncol, a, b, c, qn, qs, qo, s);
    else
        return launch_k<T, TER, DISS, 0>(m, t, col0, ncol, a, b, c, qn, qs, qo, s);
}

}  // namespace

bool fused_lpc_supported(int N, int lpc) {
    switch (N * 32 + lpc) {
#define CASE(NN, LP) case NN * 32 + LP: return true;
        SEM_FUSED_INSTANCES(CASE)
#undef CASE
        default: return false;
    }
}

bool fused_split_supported(int N, int lpc) {
    if (!fused_lpc_supported(N, lpc) || lpc < 2) return false;
    const int np = N + 1;
    for (int p = 0; p < np * np; ++p)
        for (int el = 1; el < lpc; ++el)
            if ((p * lpc * np + el * np) % 64 == 0) return false;
    return true;
}

bool fused_blocks_supported(const HostMesh& H) {
    return H.N >= 3 && H.N <= 5 && !H.blk_cols.empty();
}

namespace {

// greedy colouring in the given order of units that conflict when they
// contribute to a common unique node or hanging point; returns the colours
std::vector<int32_t> colour_units(const HostMesh& H, const std::vector<int32_t>& unit_of_col,
                                  int n_unit, const std::vector<int32_t>& unit_order, int& n_color) {
    const int np2 = H.np1 * H.np1;
    std::vector<std::vector<int32_t>> adj(static_cast<size_t>(n_unit));
    auto link = [&](const std::vector<int32_t>& ptr, const std::vector<int32_t>& slot, int64_t n) {
        for (int64_t x = 0; x < n; ++x)
            for (int32_t q = ptr[x]; q < ptr[x + 1]; ++q)
                for (int32_t r = ptr[x]; r < ptr[x + 1]; ++r) {
                    const int32_t u1 = unit_of_col[slot[q] / np2], u2 = unit_of_col[slot[r] / np2];
                    if (u1 != u2) adj[u1].push_back(u2);
                }
    };
    link(H.asm_ptr, H.asm_slot, H.n_h);
    link(H.asmH_ptr, H.asmH_slot, H.n_hh);
    std::vector<int32_t> color(size_t(n_unit), -1);
    n_color = 0;
    for (int32_t u : unit_order) {
        std::vector<char> used(size_t(n_color) + 1, 0);
        for (int32_t o : adj[u])
            if (color[o] >= 0) used[color[o]] = 1;
        int k = 0;
        while (used[k]) ++k;
        color[u] = k;
        n_color = std::max(n_color, k + 1);
    }
    return color;
}

}  // namespace

int fused_plan_build(const HostMesh& H, int layout, int param, FusedPlan& P) {
    const int np2 = H.np1 * H.np1;
    const bool columns = layout == SEM_LAYOUT_COLUMNS || layout == SEM_LAYOUT_COLUMNS_KZ ||
                         layout == SEM_LAYOUT_COLUMNS_SPLIT;
    int lpc = columns ? param : 0;
    if (lpc < 1) {
        // default: the deepest supported chunk of at most 512 threads
        lpc = 1;
        while (fused_lpc_supported(H.N, lpc * 2) && np2 * (2 * lpc * H.N + 1) <= 512) lpc *= 2;
    }
    if (!fused_lpc_supported(H.N, lpc)) return SEM_ERR_ARG;
    if (layout == SEM_LAYOUT_COLUMNS_SPLIT && !fused_split_supported(H.N, lpc)) return SEM_ERR_ARG;
    if (layout == SEM_LAYOUT_BLOCKS && !fused_blocks_supported(H)) return SEM_ERR_ARG;
    if (!columns && layout != SEM_LAYOUT_BLOCKS) return SEM_ERR_ARG;
    auto up = [&](const void* src, size_t bytes, void** dst) -> int {
        *dst = nullptr;
        if (bytes == 0) return SEM_OK;
        if (hipMalloc(dst, bytes) != hipSuccess) return SEM_ERR_HIP;
        P.allocs.push_back(*dst);
        P.bytes += int64_t(bytes);
        if (src && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return SEM_ERR_HIP;
        return SEM_OK;
    };
    // first contributor of every node: the lowest colour among its units
    auto mark_first = [&](const std::vector<int32_t>& unit_of_col, const std::vector<int32_t>& color,
                          auto&& set_first) {
        auto mark = [&](const std::vector<int32_t>& ptr, const std::vector<int32_t>& slot, int64_t n) {
            for (int64_t x = 0; x < n; ++x) {
                int32_t best = -1;
                for (int32_t q = ptr[x]; q < ptr[x + 1]; ++q)
                    if (best < 0 || color[unit_of_col[slot[q] / np2]] < color[unit_of_col[best / np2]])
                        best = slot[q];
                if (best >= 0) set_first(best);
            }
        };
        mark(H.asm_ptr, H.asm_slot, H.n_h);
        mark(H.asmH_ptr, H.asmH_slot, H.n_hh);
    };
    void* d;
    int rc;
    // ---- column layout over every column (also the terrain path)
    {
        std::vector<int32_t> unit_of_col(static_cast<size_t>(H.n_col)), corder(static_cast<size_t>(H.n_col));
        for (int c = 0; c < H.n_col; ++c) unit_of_col[c] = corder[c] = c;
        int n_color = 0;
        // greedy colouring in column order (the caller's order; Morton keeps it local)
        std::vector<int32_t> color = colour_units(H, unit_of_col, H.n_col, corder, n_color);
        // side columns: the colour classes beyond the fourth that hold fewer
        // than a quarter of the largest class's columns.  Their launches
        // would be short and latency-bound; instead they run in the launches
        // of the other colours (they only read q_s and write their own
        // slots) and the tail launch assembles their contributions.
        std::vector<int32_t> csize(size_t(n_color), 0);
        for (int cidx = 0; cidx < H.n_col; ++cidx) ++csize[color[cidx]];
        const int32_t cmax = *std::max_element(csize.begin(), csize.end());
        std::vector<char> small(size_t(n_color), 0);
        for (int k = 4; k < n_color; ++k) small[k] = 4 * csize[k] < cmax;
        std::vector<int32_t> side_of_col(static_cast<size_t>(H.n_col), -1), side_cols;
        for (int cidx = 0; cidx < H.n_col; ++cidx)
            if (small[color[cidx]]) {
                side_of_col[cidx] = int32_t(side_cols.size());
                side_cols.push_back(cidx);
            }
        // each colour's columns (the first colour's with the side columns)
        // by decreasing work: the hanging positions of a column interpolate
        // their values and store to the hanging buffer.  Stable, so equal
        // columns keep the caller's (Morton) order.
        std::vector<int32_t> n_hang(static_cast<size_t>(H.n_col), 0);
        for (int cidx = 0; cidx < H.n_col; ++cidx)
            for (int pos = 0; pos < np2; ++pos) n_hang[cidx] += H.gmap[size_t(cidx) * np2 + pos] < 0;
        // the side columns go to the launches with the fewest columns (one at
        // a time, in their order), so that the launches come out even
        std::vector<std::vector<int32_t>> side_of_k(static_cast<size_t>(n_color));
        {
            std::vector<int64_t> load(static_cast<size_t>(n_color), INT64_MAX);
            for (int k = 0; k < n_color; ++k)
                if (!small[k]) load[k] = csize[k];
            for (int32_t sc : side_cols) {
                const int k = int(std::min_element(load.begin(), load.end()) - load.begin());
                side_of_k[k].push_back(sc);
                ++load[k];
            }
        }
        std::vector<int32_t> order, cptr(1, 0);
        for (int k = 0; k < n_color; ++k) {
            if (small[k]) continue;
            const size_t k0 = order.size();
            for (int cidx = 0; cidx < H.n_col; ++cidx)
                if (color[cidx] == k) order.push_back(cidx);
            order.insert(order.end(), side_of_k[k].begin(), side_of_k[k].end());
            std::stable_sort(order.begin() + k0, order.end(),
                             [&](int32_t x, int32_t y) { return n_hang[x] > n_hang[y]; });
            cptr.push_back(int32_t(order.size()));
        }
        n_color = int(cptr.size()) - 1;
        // positions of side columns become pseudo hanging points n_hh + k (N+1)^2 + pos
        const int64_t n_pseudo = int64_t(side_cols.size()) * np2;
        auto pseudo = [&](int32_t slot) {
            return int32_t(H.n_hh + int64_t(side_of_col[slot / np2]) * np2 + slot % np2);
        };
        std::vector<int32_t> gmap_x(H.gmap), hptr_x(H.hang_ptr), hsrc_x(H.hang_src);
        std::vector<double> hw_x(H.hang_w);
        std::vector<int32_t> hreal(static_cast<size_t>(H.n_hh + n_pseudo));
        for (int64_t hh = 0; hh < H.n_hh; ++hh) hreal[hh] = int32_t(H.n_h + hh);
        if (hptr_x.empty()) hptr_x.push_back(0);
        for (int32_t sc : side_cols)
            for (int pos = 0; pos < np2; ++pos) {
                const int32_t slot = sc * np2 + pos, g = H.gmap[slot];
                if (g >= 0) {
                    hsrc_x.push_back(g);
                    hw_x.push_back(1.0);
                    hreal[pseudo(slot)] = g;
                } else {
                    for (int32_t r = H.hang_ptr[-g - 1]; r < H.hang_ptr[-g]; ++r) {
                        hsrc_x.push_back(H.hang_src[r]);
                        hw_x.push_back(H.hang_w[r]);
                    }
                    hreal[pseudo(slot)] = int32_t(H.n_h - g - 1);
                }
                hptr_x.push_back(int32_t(hsrc_x.size()));
                gmap_x[slot] = -(pseudo(slot) + 1);
            }
        // first writers among the columns that write nodes themselves; every
        // pseudo point has exactly one writer
        std::vector<int32_t> wcolor(color);
        for (int32_t sc : side_cols) wcolor[sc] = INT32_MAX;
        std::vector<uint8_t> first(H.gmap.size(), 0);
        mark_first(unit_of_col, wcolor, [&](int32_t slot) {
            if (side_of_col[slot / np2] < 0) first[slot] = 1;
        });
        for (int32_t sc : side_cols)
            for (int pos = 0; pos < np2; ++pos) first[size_t(sc) * np2 + pos] = 1;
        auto upv = [&](const auto& v, auto** dst) -> int {
            void* pd = nullptr;
            const size_t bytes = v.size() * sizeof(v[0]);
            // an empty table still gets a (never read) 8-byte allocation
            int r2 = up(bytes ? static_cast<const void*>(v.data()) : nullptr,
                        std::max<size_t>(bytes, 8), &pd);
            *dst = static_cast<std::remove_pointer_t<decltype(dst)>>(pd);
            return r2;
        };
        if ((rc = upv(gmap_x, &P.t.gmap)) != SEM_OK) return rc;
        if ((rc = upv(hptr_x, &P.t.hang_ptr)) != SEM_OK) return rc;
        if ((rc = upv(hsrc_x, &P.t.hang_src)) != SEM_OK) return rc;
        if ((rc = upv(hw_x, &P.t.hang_w)) != SEM_OK) return rc;
        if ((rc = upv(hreal, &P.t.hreal)) != SEM_OK) return rc;
        P.t.fsh = (H.n_hh + n_pseudo) * H.ldz;
        if (!side_cols.empty()) {
            // tail tables: unique nodes with side slots or Z^T rows
            auto is_side = [&](int32_t slot) { return side_of_col[slot / np2] >= 0; };
            std::vector<int32_t> hT_row(static_cast<size_t>(H.n_h), -1);
            for (size_t li = 0; li < H.hT_list.size(); ++li) hT_row[H.hT_list[li]] = int32_t(li);
            std::vector<int32_t> th, tsptr(1, 0), tsslot, thptr(1, 0), thh;
            std::vector<double> thw;
            std::vector<uint8_t> tfirst;
            for (int64_t h = 0; h < H.n_h; ++h) {
                bool any_side = false, any_direct = false;
                for (int32_t q = H.asm_ptr[h]; q < H.asm_ptr[h + 1]; ++q) {
                    if (is_side(H.asm_slot[q])) any_side = true;
                    else any_direct = true;
                }
                if (!any_side && hT_row[h] < 0) continue;
                th.push_back(int32_t(h));
                tfirst.push_back(any_direct ? 0 : 1);
                for (int32_t q = H.asm_ptr[h]; q < H.asm_ptr[h + 1]; ++q)
                    if (is_side(H.asm_slot[q])) tsslot.push_back(pseudo(H.asm_slot[q]));
                tsptr.push_back(int32_t(tsslot.size()));
                if (hT_row[h] >= 0) {
                    const int32_t li = hT_row[h];
                    for (int32_t r = H.hT_ptr[li]; r < H.hT_ptr[li + 1]; ++r) {
                        thh.push_back(H.hT_hh[r]);
                        thw.push_back(H.hT_w[r]);
                    }
                }
                thptr.push_back(int32_t(thh.size()));
            }
            std::vector<int32_t> hsptr(1, 0), hsslot;
            std::vector<uint8_t> hvalid(static_cast<size_t>(std::max<int64_t>(H.n_hh, 1)), 0);
            for (int64_t hh = 0; hh < H.n_hh; ++hh) {
                for (int32_t q = H.asmH_ptr[hh]; q < H.asmH_ptr[hh + 1]; ++q) {
                    if (is_side(H.asmH_slot[q])) hsslot.push_back(pseudo(H.asmH_slot[q]));
                    else hvalid[hh] = 1;
                }
                hsptr.push_back(int32_t(hsslot.size()));
            }
            if (hsptr.size() == 1) hsptr.push_back(0);
            // one flat list per tail node: its side slots (a group of weight
            // 1), then per hanging point of its Z^T row a group of weight w:
            // the point's own contribution (if a column writes it) and its
            // side slots.  A group sums its rows first and enters the node's
            // sum times its weight, in the order of Z^T; a group with no row
            // gets one entry of row -1 (adds nothing).
            std::vector<int32_t> eptr(1, 0), erow;
            std::vector<double> ew;
            std::vector<uint8_t> estart;
            auto entry = [&](int32_t row, bool start, double w) {
                erow.push_back(row);
                estart.push_back(start ? 1 : 0);
                ew.push_back(w);
            };
            for (size_t li = 0; li < th.size(); ++li) {
                for (int32_t q = tsptr[li]; q < tsptr[li + 1]; ++q) entry(tsslot[q], q == tsptr[li], 1.0);
                for (int32_t r = thptr[li]; r < thptr[li + 1]; ++r) {
                    const int32_t hh = thh[r];
                    bool any = false;
                    if (hvalid[hh]) { entry(hh, true, thw[r]); any = true; }
                    for (int32_t q = hsptr[hh]; q < hsptr[hh + 1]; ++q) { entry(hsslot[q], !any, thw[r]); any = true; }
                    if (!any) entry(-1, true, thw[r]);
                }
                eptr.push_back(int32_t(erow.size()));
            }
            TailTables& T = P.tail;
            if ((rc = upv(th, &T.h)) != SEM_OK) return rc;
            if ((rc = upv(tfirst, &T.first)) != SEM_OK) return rc;
            if ((rc = upv(eptr, &T.eptr)) != SEM_OK) return rc;
            if ((rc = upv(erow, &T.erow)) != SEM_OK) return rc;
            if ((rc = upv(ew, &T.ew)) != SEM_OK) return rc;
            if ((rc = upv(estart, &T.estart)) != SEM_OK) return rc;
            T.n = int(th.size());
            T.fsh = P.t.fsh;
            P.has_tail = true;
        }
        if ((rc = up(order.data(), order.size() * 4, &d)) != SEM_OK) return rc;
        P.t.col_order = static_cast<const int32_t*>(d);
        if ((rc = up(cptr.data(), cptr.size() * 4, &d)) != SEM_OK) return rc;
        P.t.color_ptr = static_cast<const int32_t*>(d);
        if ((rc = up(first.data(), first.size(), &d)) != SEM_OK) return rc;
        P.t.first = static_cast<const uint8_t*>(d);
        if ((rc = up(nullptr, size_t(NF) * P.t.fsh * 8, &d)) != SEM_OK) return rc;
        P.t.cH = static_cast<double*>(d);
        P.tail.cH = P.t.cH;
        P.t.n_color = n_color;
        P.t.layers_per_chunk = lpc;
        P.t.thread_order = layout == SEM_LAYOUT_COLUMNS_KZ ? 1 : layout == SEM_LAYOUT_COLUMNS_SPLIT ? 2 : 0;
        P.color_ptr_host = cptr;
    }
    P.layout = columns ? layout : SEM_LAYOUT_COLUMNS;
    if (columns) return SEM_OK;

    // ---- block layout: units are the 2 x 2 blocks and the columns in no block
    const int N = H.N, PX = 2 * N + 1, PP = PX * PX;
    const int nb = int(H.blk_cols.size() / 4);
    std::vector<int32_t> unit_of_col(static_cast<size_t>(H.n_col)), singles, unit_first_col;
    for (int c = 0; c < H.n_col; ++c) {
        if (H.col_block[c] >= 0) unit_of_col[c] = H.col_block[c];
        else {
            unit_of_col[c] = nb + int32_t(singles.size());
            singles.push_back(c);
        }
    }
    const int n_unit = nb + int(singles.size());
    unit_first_col.assign(size_t(n_unit), H.n_col);
    for (int c = 0; c < H.n_col; ++c)
        unit_first_col[unit_of_col[c]] = std::min(unit_first_col[unit_of_col[c]], c);
    std::vector<int32_t> uorder(static_cast<size_t>(n_unit));
    for (int u = 0; u < n_unit; ++u) uorder[u] = u;
    std::stable_sort(uorder.begin(), uorder.end(),
                     [&](int32_t x, int32_t y) { return unit_first_col[x] < unit_first_col[y]; });
    int n_color = 0;
    std::vector<int32_t> color = colour_units(H, unit_of_col, n_unit, uorder, n_color);
    // block position of every slot of a block's columns
    auto block_pos = [&](int32_t slot) {
        const int c = slot / np2, pos = slot - c * np2;
        const int i = pos % H.np1, j = pos / H.np1;
        const int32_t* bc = &H.blk_cols[size_t(H.col_block[c]) * 4];
        int q = 0;
        while (bc[q] != c) ++q;
        return (i + (q & 1) * N) + PX * (j + (q >> 1) * N);
    };
    std::vector<uint8_t> pos_first(size_t(nb) * PP, 0), first_s(H.gmap.size(), 0);
    mark_first(unit_of_col, color, [&](int32_t slot) {
        const int c = slot / np2;
        if (H.col_block[c] >= 0) pos_first[size_t(H.col_block[c]) * PP + block_pos(slot)] = 1;
        else first_s[slot] = 1;
    });
    std::vector<int32_t> pos_g(static_cast<size_t>(nb) * PP, 0), blk_col(static_cast<size_t>(nb));
    for (int b = 0; b < nb; ++b) {
        blk_col[b] = H.blk_cols[size_t(b) * 4];
        for (int q = 0; q < 4; ++q) {
            const int c = H.blk_cols[size_t(b) * 4 + q];
            for (int pos = 0; pos < np2; ++pos) {
                const int32_t slot = c * np2 + pos;
                pos_g[size_t(b) * PP + block_pos(slot)] = H.gmap[slot];
            }
        }
    }
    std::vector<int32_t> border, sorder, bptr(size_t(n_color) + 1, 0), sptr(size_t(n_color) + 1, 0);
    for (int k = 0; k < n_color; ++k) {
        for (int32_t u : uorder) {
            if (color[u] != k) continue;
            if (u < nb) border.push_back(u);
            else sorder.push_back(singles[u - nb]);
        }
        bptr[k + 1] = int32_t(border.size());
        sptr[k + 1] = int32_t(sorder.size());
    }
    // vertical segments: by default enough for about 1024 workgroups per
    // launch of the largest colour (two resident per CU on 256 CUs, both
    // parities), at least one layer each
    int S = param;
    if (S < 1) {
        int nbmax = 1;
        for (int k = 0; k < n_color; ++k) nbmax = std::max(nbmax, bptr[k + 1] - bptr[k]);
        S = 1;
        while (S < H.n_z && nbmax * S < 1024) S *= 2;
    }
    S = std::min(S, H.n_z);
    const int Ls = (H.n_z + S - 1) / S;
    if ((rc = up(border.data(), border.size() * 4, &d)) != SEM_OK) return rc;
    P.bt.order = static_cast<const int32_t*>(d);
    if ((rc = up(pos_g.data(), pos_g.size() * 4, &d)) != SEM_OK) return rc;
    P.bt.pos_g = static_cast<const int32_t*>(d);
    if ((rc = up(pos_first.data(), pos_first.size(), &d)) != SEM_OK) return rc;
    P.bt.pos_first = static_cast<const uint8_t*>(d);
    if ((rc = up(blk_col.data(), blk_col.size() * 4, &d)) != SEM_OK) return rc;
    P.bt.blk_col = static_cast<const int32_t*>(d);
    P.bt.cH = P.t.cH;
    P.bt.Ls = Ls;
    P.bt.n_seg = (H.n_z + Ls - 1) / Ls;
    P.bt.fsh = P.t.fsh;
    P.ts = P.t;
    // the columns in no block read the mesh's own position map and rows (the
    // column layout's pseudo hanging points belong to its side columns only)
    if ((rc = up(H.gmap.data(), H.gmap.size() * 4, &d)) != SEM_OK) return rc;
    P.ts.gmap = static_cast<const int32_t*>(d);
    if (H.n_hh > 0) {
        if ((rc = up(H.hang_ptr.data(), H.hang_ptr.size() * 4, &d)) != SEM_OK) return rc;
        P.ts.hang_ptr = static_cast<const int32_t*>(d);
        if ((rc = up(H.hang_src.data(), H.hang_src.size() * 4, &d)) != SEM_OK) return rc;
        P.ts.hang_src = static_cast<const int32_t*>(d);
        if ((rc = up(H.hang_w.data(), H.hang_w.size() * 8, &d)) != SEM_OK) return rc;
        P.ts.hang_w = static_cast<const double*>(d);
    }
    P.ts.col_order = nullptr;
    if (!sorder.empty()) {
        if ((rc = up(sorder.data(), sorder.size() * 4, &d)) != SEM_OK) return rc;
        P.ts.col_order = static_cast<const int32_t*>(d);
    }
    if ((rc = up(first_s.data(), first_s.size(), &d)) != SEM_OK) return rc;
    P.ts.first = static_cast<const uint8_t*>(d);
    P.ts.color_ptr = nullptr;
    P.ts.n_color = n_color;
    P.ts.thread_order = 0;
    P.blk_ptr_host = bptr;
    P.single_ptr_host = sptr;
    P.n_unit_color = n_color;
    P.layout = SEM_LAYOUT_BLOCKS;
    return SEM_OK;
}

void fused_plan_free(FusedPlan& P) {
    for (void* p : P.allocs) (void)hipFree(p);
    P.allocs.clear();
    P.bytes = 0;
}

template <typename T>
int launch_blocks(const DevMesh& m, const BlockTables& bt, int b0, int nblk, int par, int n_iseg,
                  double a, double b, double c, const double* qn, const double* qs, double* qo,
                  hipStream_t s) {
    const unsigned grid = unsigned(nblk) * unsigned(n_iseg);
    switch (m.N) {
#define CASE(NN)                                                                              \
    case NN:                                                                                  \
        hipLaunchKernelGGL((k_stage_blocks<NN + 1, T>), dim3(grid), dim3(blk_threads<NN + 1>()), 0, \
                           s, m, bt, b0, nblk, par, n_iseg, a, b, c, qn, qs, qo);           \
        break;
        CASE(3) CASE(4) CASE(5)
#undef CASE
        default: return SEM_ERR_ARG;
    }
    return (hipGetLastError() == hipSuccess) ? SEM_OK : SEM_ERR_HIP;
}

bool fused_dissipation_inline(const DevMesh& m, const FusedPlan& P, int prec) {
    return (m.cs > 0.0 || m.sponge) && !m.zs && prec == SEM_FP64 && P.layout != SEM_LAYOUT_BLOCKS;
}

int fused_stage_launch(const DevMesh& m_in, const FusedPlan& P, double a, double b, double c,
                       const double* qn, const double* qs, double* qo, int prec, hipStream_t s) {
    const bool f32 = prec == SEM_FP32;
    // the optional dissipation inside the column kernel (FP64, box
    // elements): no pre-pass tendency is added
    const bool diss = fused_dissipation_inline(m_in, P, prec);
    DevMesh m = m_in;
    if (diss) m.rx = nullptr;
    if (P.layout == SEM_LAYOUT_BLOCKS && !m.zs) {
        // colour by colour: the colour's blocks, even segments then odd
        // ones, then its columns in no block
        const BlockTables& bt = P.bt;
        for (int k = 0; k < P.n_unit_color; ++k) {
            const int b0 = P.blk_ptr_host[k], nb = P.blk_ptr_host[k + 1] - b0;
            for (int par = 0; par < 2 && nb > 0; ++par) {
                const int n_iseg = par == 0 ? (bt.n_seg + 1) / 2 : bt.n_seg / 2;
                if (n_iseg == 0) continue;
                const int rc = f32 ? launch_blocks<float>(m, bt, b0, nb, par, n_iseg, a, b, c, qn, qs, qo, s)
                                   : launch_blocks<double>(m, bt, b0, nb, par, n_iseg, a, b, c, qn, qs, qo, s);
                if (rc != SEM_OK) return rc;
            }
            const int s0 = P.single_ptr_host[k], ns = P.single_ptr_host[k + 1] - s0;
            if (ns > 0) {
                const int rc = f32 ? launch_t<float, false>(m, P.ts, s0, ns, a, b, c, qn, qs, qo, s)
                                   : launch_t<double, false>(m, P.ts, s0, ns, a, b, c, qn, qs, qo, s);
                if (rc != SEM_OK) return rc;
            }
        }
    } else {
        const FusedTables& t = P.t;
        for (int k = 0; k < t.n_color; ++k) {
            const int col0 = P.color_ptr_host[k];
            const int ncol = P.color_ptr_host[k + 1] - col0;
            if (ncol == 0) continue;
            int rc;
            if (m.zs) {
                rc = f32 ? launch_t<float, true>(m, t, col0, ncol, a, b, c, qn, qs, qo, s)
                         : launch_t<double, true>(m, t, col0, ncol, a, b, c, qn, qs, qo, s);
            } else if (diss) {
                rc = launch_t<double, false, true>(m, t, col0, ncol, a, b, c, qn, qs, qo, s);
            } else {
                rc = f32 ? launch_t<float, false>(m, t, col0, ncol, a, b, c, qn, qs, qo, s)
                         : launch_t<double, false>(m, t, col0, ncol, a, b, c, qn, qs, qo, s);
            }
            if (rc != SEM_OK) return rc;
        }
    }
    const bool tail = P.has_tail && !(P.layout == SEM_LAYOUT_BLOCKS && !m.zs);
    const int64_t n2 = int64_t(tail ? P.tail.n : m.n_hT) * m.nzn;
    if (n2 > 0) {
        const int64_t g = std::min<int64_t>((n2 + 255) / 256, 65536);
        if (tail)
            hipLaunchKernelGGL(k_stage_tail, dim3(unsigned(g)), dim3(256), 0, s, m, P.tail, a, b, c, qn, qs, qo);
        else
            hipLaunchKernelGGL(k_stage_hanging, dim3(unsigned(g)), dim3(256), 0, s, m, P.t, c, qo);
        if (hipGetLastError() != hipSuccess) return SEM_ERR_HIP;
    }
    return SEM_OK;
}

}  // namespace sem
