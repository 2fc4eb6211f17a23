// Fused Runge-Kutta stage for gfx950.
//
// q_out = a q^n + b q_s + c M^-1 Z^T (m_L R_L(Z q_s)) in one pass over the
// columns of every refinement level, without ever storing the element-local
// right-hand side.
//
// Column kernel.  A workgroup owns one column and marches up through it in
// chunks of `layers_per_chunk` stacked elements; one thread per unique node of
// the chunk (vertical index fastest, so that the accesses of one horizontal
// position are contiguous in the [field][h][kz] state layout):
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
// the sums is fixed (deterministic results).
// Hanging-point kernel (meshes with hanging nodes): every coarse face node
// adds c M^-1 sum_hh w_hh c_hh, the transpose of the scatter (Section 3.1).
#include "stage_fused.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <type_traits>

#include "mesh_build.h"
#include "sem.h"

namespace sem {

namespace {

constexpr int NF = SEM_NFIELDS;
// LDS tiles: rho u, rho v, rho w and u singly; (v, w) and (p', theta') as pairs

template <int NP, int LPC>
constexpr int wg_threads() {
    return ((NP * NP * (LPC * (NP - 1) + 1) + 63) / 64) * 64;
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
// compute while the other waits on memory.  Within a workgroup the global
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
template <int NP, int LPC, typename T, bool TER>
__global__ void __launch_bounds__(((NP * NP * (LPC * (NP - 1) + 1) + 63) / 64) * 64, 4)
k_stage_columns(DevMesh m, FusedTables ft, int col0, int ncol, double a, double b, double c,
                const double* __restrict__ qn, const double* __restrict__ qs,
                double* __restrict__ qo) {
    constexpr int NP2 = NP * NP, N = NP - 1;
    constexpr int NK = LPC * N + 1;               // vertical nodes of a full chunk
    constexpr int WGT = wg_threads<NP, LPC>();
    __shared__ T tile[4][NP2 * NK];               // rho u, rho v, rho w, u: [field][p][kzl], kzl fastest
    __shared__ double carry[2][NF][NP2];
    __shared__ T sD[NP2];
    // per position and tap, the x and y coefficients side by side: one 2-wide
    // LDS read serves both derivatives of a call
    using T2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
    __shared__ T2 sDxy[NP2 * NP];
    // (v, w) and (p', theta'), always differentiated together: one 2-wide
    // element per node, so one LDS read per tap serves both fields
    __shared__ T2 tpr[2][NP2 * NK];
    __shared__ double sW[NP];
    // the chunk's slice of the per-level tables, double-buffered: rho0,
    // 1/rho0, 1/theta0, p0, dtheta0/dz, 1/M_v at its NK levels, then dz and
    // 2/dz of its LPC layers
    constexpr int SL = 6 * NK + 2 * LPC;
    __shared__ double slice[2][SL];
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

    // Workgroups go to the 8 XCDs round-robin by id; give each XCD a
    // contiguous (Morton-ordered) range of this colour's columns.
    const int G = gridDim.x;
    const int xcd = blockIdx.x & 7, rr = blockIdx.x >> 3;
    const int item = xcd * (G >> 3) + min(xcd, G & 7) + rr;
    const int col = ft.col_order[col0 + min(item, ncol - 1)];

    // Thread -> node of the chunk.  FP64: nodes on the planes between two
    // stacked elements (LPC-1 per position, two z derivatives each) come
    // first, so that they fill waves of their own instead of making every
    // wave run a second pass of FP64 z derivatives with most lanes masked,
    // and so that these longest waves are the oldest, which issue first;
    // nodes inside an element or on the chunk's bottom/top follow (RG per
    // position).  Float: the natural order (kzl fastest within a position); the
    // masked second pass is cheap at the float rate, and every wave then
    // carries the same LDS load, so no wave waits long at the barriers.
    constexpr int RG = LPC * (N - 1) + 2;
    int kzl, p;
    if constexpr (sizeof(T) == 4) {
        p = tid < NP2 * NK ? tid / NK : NP2;
        kzl = tid < NP2 * NK ? tid - p * NK : 0;
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
            const int gz = m.gmap[col * NP2 + t];
            s_zs[t] = m.zs[gz >= 0 ? gz : m.n_h - gz - 1];
        }
    }
    const bool lane_ok = (p < NP2) && (item < ncol);
    const int pc = lane_ok ? p : 0;               // position used for table lookups
    const int i = pc % NP, j = pc / NP;
    const int nzn = m.nzn;
    const int64_t fs = int64_t(m.n_h) * m.ldz;
    const int64_t fsh = int64_t(m.n_hh) * m.ldz;
    const int64_t fsr = int64_t(m.n_h + m.n_hh) * m.ldz;   // terrain reference rows

    int g = 0, r_beg = 0, r_end = 0;
    bool first = false;
    const double dxc = m.col_dx[col], dyc = m.col_dy[col];
    const T sx = T(m.col_sx[col]), sy = T(m.col_sy[col]);
    if (lane_ok) {
        g = m.gmap[col * NP2 + pc];
        first = ft.first[col * NP2 + pc] != 0;
        if (g < 0) {
            r_beg = m.hang_ptr[-g - 1];
            r_end = m.hang_ptr[-g];
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
        const int gt = m.gmap[col * NP2 + t];
        s_mh[t] = gt >= 0 ? (TER ? m.minv_ht[gt] : m.minv_h[gt]) : 0.0;
        s_row[t] = gt >= 0 ? int64_t(gt) * m.ldz : 0;
        if constexpr (TER) s_rrow[t] = int64_t(gt >= 0 ? gt : m.n_h - gt - 1) * m.ldz;
    }
    __syncthreads();
    for (int t = tid; t < NP2; t += WGT) s_mij[t] = sW[t % NP] * sW[t / NP] * 0.125 * dxc * dyc;
    const T2* Dxy = &sDxy[pc * NP];
    const int lx0 = (j * NP) * NK + kzl, ly0 = i * NK + kzl;
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
    double pf[NF] = {0, 0, 0, 0, 0};              // q_s of the next chunk (direct nodes)
    for (int ch = 0; ch < n_chunk; ++ch) {
        const int L0 = ch * LPC;
        const int L1 = min(L0 + LPC, m.n_z);
        const int nk = (L1 - L0) * N + 1;
        const bool active = lane_ok && (kzl < nk);
        const int kz = L0 * N + kzl;
        const int lidx = pc * NK + kzl;
        double qv[NF] = {0, 0, 0, 0, 0};
        T rho = T(1);
        if (active) {
            if (g >= 0) {
                if (!TER && ch > 0) {
#pragma unroll
                    for (int f = 0; f < NF; ++f) qv[f] = pf[f];
                } else {
                    const int64_t o = s_row[pc] + kz;
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
        __syncthreads();
        // update base of the nodes finished in this chunk (q^n for the first
        // contributor, not read when a = 0; the partial q_out for later colours)
        double base[NF] = {0, 0, 0, 0, 0};
        if (!TER && active && g >= 0 && !(kzl == nk - 1 && L1 < m.n_z) && (!first || a != 0.0)) {
            const double* bp = first ? qn : qo;
            const int64_t o = s_row[pc] + kz;
#pragma unroll
            for (int f = 0; f < NF; ++f) base[f] = bp[f * fs + o];
        }
        const double* sb = slice[ch & 1];
        double sl_next = 0.0;
        if (tid < SL && ch + 1 < n_chunk) sl_next = slice_value(ch + 1);
        // prefetch the next chunk's q_s (box elements: the terrain instance
        // needs those registers for its metric terms)
        if (!TER && ch + 1 < n_chunk && lane_ok && g >= 0) {
            const int L0n = L0 + LPC;
            const int nkn = (min(L0n + LPC, m.n_z) - L0n) * N + 1;
            if (kzl < nkn) {
                const int64_t o = s_row[pc] + L0n * N + kzl;
#pragma unroll
                for (int f = 0; f < NF; ++f) pf[f] = qs[f * fs + o];
            }
        }
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
                    ax += cx * tile[tx][lx0 + mm * NK];
                    ay += cy * tile[ty][ly0 + mm * NP * NK];
                    ax2 += cx * tile[tx2][lx0 + mm * NK];
                    ay2 += cy * tile[ty2][ly0 + mm * NP * NK];
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
                    const T2 a = tpr[pr][lx0 + mm * NK], b = tpr[pr][ly0 + mm * NP * NK];
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
            dxy(0, 1, 3, 3, ax, ay, bx, by);
            Rh[0] = -(ax + ay);
            Rh[1] = -(u * bx + v * by) + f * v;
            dxyp(0, ax, ay, bx, by);
            Rh[2] = -(u * ax + v * ay) - f * u;
            Rh[3] = -(u * bx + v * by) - T(qv[0]) * inv_rho * gr;
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
            double acc[NF] = {0, 0, 0, 0, 0};
            // elements of this chunk holding the node: (element, local k)
            const bool inner_plane = (kzl % N == 0) && kzl > 0 && kzl < nk - 1;
            const int e_first = (kzl == nk - 1) ? (kzl - 1) / N : (inner_plane ? kzl / N - 1 : kzl / N);
            const int n_el = inner_plane ? 2 : 1;
            for (int s2 = 0; s2 < n_el; ++s2) {
                const int el = e_first + s2;
                const int kk = kzl - el * N;
                const double dzl = sb[6 * NK + el];
                const T sz = T(sb[6 * NK + LPC + el]);
                const T* Dz = &sD[kk * NP];
                const int lz0 = pc * NK + el * N;
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
                    ddzp(0, z0, z1);
                    R[2] = Rh[2] - w * z0;
                    T z2, z3;
                    ddzp(1, z2, z3);
                    R[3] = Rh[3] - w * z1 - z2 * inv_rho;
                    R[4] = Rh[4] - w * z3;
                }
                const double mass = s_mij[pc] * sW[kk] * dzl;
#pragma unroll
                for (int fl = 0; fl < NF; ++fl) acc[fl] += mass * double(R[fl]);
            }
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
                    if (TER && (!first || a != 0.0)) {
                        // the terrain instance loads its base here (registers)
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
    const int64_t fsh = int64_t(m.n_hh) * m.ldz;
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

// (order, layers per chunk) instances with <= 1024 threads and <= 64 KB LDS
#define SEM_FUSED_INSTANCES(X) \
    X(1, 1) X(1, 2) X(1, 4) X(1, 8) \
    X(2, 1) X(2, 2) X(2, 4) X(2, 8) \
    X(3, 1) X(3, 2) X(3, 4) X(3, 8) \
    X(4, 1) X(4, 2) X(4, 4) X(4, 8) \
    X(5, 1) X(5, 2) X(5, 4)         \
    X(6, 1) X(6, 2)                 \
    X(7, 1) X(7, 2)                 \
    X(8, 1)

template <typename T, bool TER>
int launch_t(const DevMesh& m, const FusedTables& t, int col0, int ncol, double a, double b,
             double c, const double* qn, const double* qs, double* qo, hipStream_t s) {
    switch (m.N * 32 + t.layers_per_chunk) {
#define CASE(NN, LP)                                                                    \
    case NN * 32 + LP:                                                                  \
        hipLaunchKernelGGL((k_stage_columns<NN + 1, LP, T, TER>), dim3(ncol),           \
                           dim3(wg_threads<NN + 1, LP>()), 0, s, m, t, col0, ncol, a, b, \
                           c, qn, qs, qo);                                              \
        break;
        SEM_FUSED_INSTANCES(CASE)
#undef CASE
        default: return SEM_ERR_ARG;
    }
    return (hipGetLastError() == hipSuccess) ? SEM_OK : SEM_ERR_HIP;
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

int fused_plan_build(const HostMesh& H, int lpc, FusedPlan& P) {
    const int np2 = H.np1 * H.np1;
    if (lpc < 1) {
        // default: the deepest supported chunk of at most 512 threads
        lpc = 1;
        while (fused_lpc_supported(H.N, lpc * 2) && np2 * (2 * lpc * H.N + 1) <= 512) lpc *= 2;
    }
    if (!fused_lpc_supported(H.N, lpc)) return SEM_ERR_ARG;
    // conflict lists: the columns contributing to each unique node / hanging point
    std::vector<std::vector<int32_t>> adj(size_t(H.n_col));
    auto link = [&](const std::vector<int32_t>& ptr, const std::vector<int32_t>& slot, int64_t n) {
        for (int64_t x = 0; x < n; ++x)
            for (int32_t q = ptr[x]; q < ptr[x + 1]; ++q)
                for (int32_t r = ptr[x]; r < ptr[x + 1]; ++r) {
                    const int32_t c1 = slot[q] / np2, c2 = slot[r] / np2;
                    if (c1 != c2) adj[c1].push_back(c2);
                }
    };
    link(H.asm_ptr, H.asm_slot, H.n_h);
    link(H.asmH_ptr, H.asmH_slot, H.n_hh);
    // greedy colouring in column order (the caller's order; Morton keeps it local)
    std::vector<int32_t> color(size_t(H.n_col), -1);
    int n_color = 0;
    for (int cidx = 0; cidx < H.n_col; ++cidx) {
        std::vector<char> used(size_t(n_color) + 1, 0);
        for (int32_t o : adj[cidx])
            if (color[o] >= 0) used[color[o]] = 1;
        int k = 0;
        while (used[k]) ++k;
        color[cidx] = k;
        n_color = std::max(n_color, k + 1);
    }
    std::vector<int32_t> order, cptr(size_t(n_color) + 1, 0);
    for (int k = 0; k < n_color; ++k) {
        for (int cidx = 0; cidx < H.n_col; ++cidx)
            if (color[cidx] == k) order.push_back(cidx);
        cptr[k + 1] = int32_t(order.size());
    }
    // first contributor of every node: the lowest colour among its columns
    std::vector<uint8_t> first(H.gmap.size(), 0);
    auto mark = [&](const std::vector<int32_t>& ptr, const std::vector<int32_t>& slot, int64_t n) {
        for (int64_t x = 0; x < n; ++x) {
            int32_t best = -1;
            for (int32_t q = ptr[x]; q < ptr[x + 1]; ++q)
                if (best < 0 || color[slot[q] / np2] < color[best / np2]) best = slot[q];
            if (best >= 0) first[best] = 1;
        }
    };
    mark(H.asm_ptr, H.asm_slot, H.n_h);
    mark(H.asmH_ptr, H.asmH_slot, H.n_hh);
    auto up = [&](const void* src, size_t bytes, void** dst) -> int {
        *dst = nullptr;
        if (bytes == 0) return SEM_OK;
        if (hipMalloc(dst, bytes) != hipSuccess) return SEM_ERR_HIP;
        P.allocs.push_back(*dst);
        P.bytes += int64_t(bytes);
        if (src && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return SEM_ERR_HIP;
        return SEM_OK;
    };
    void* d;
    int rc;
    if ((rc = up(order.data(), order.size() * 4, &d)) != SEM_OK) return rc;
    P.t.col_order = static_cast<const int32_t*>(d);
    if ((rc = up(cptr.data(), cptr.size() * 4, &d)) != SEM_OK) return rc;
    P.t.color_ptr = static_cast<const int32_t*>(d);
    if ((rc = up(first.data(), first.size(), &d)) != SEM_OK) return rc;
    P.t.first = static_cast<const uint8_t*>(d);
    if ((rc = up(nullptr, size_t(NF) * H.n_hh * H.ldz * 8, &d)) != SEM_OK) return rc;
    P.t.cH = static_cast<double*>(d);
    P.t.n_color = n_color;
    P.t.layers_per_chunk = lpc;
    P.color_ptr_host = cptr;
    return SEM_OK;
}

void fused_plan_free(FusedPlan& P) {
    for (void* p : P.allocs) (void)hipFree(p);
    P.allocs.clear();
    P.bytes = 0;
}

int fused_stage_launch(const DevMesh& m, const FusedPlan& P, double a, double b, double c,
                       const double* qn, const double* qs, double* qo, int prec, hipStream_t s) {
    const FusedTables& t = P.t;
    for (int k = 0; k < t.n_color; ++k) {
        const int col0 = P.color_ptr_host[k];
        const int ncol = P.color_ptr_host[k + 1] - col0;
        if (ncol == 0) continue;
        int rc;
        if (m.zs) {
            rc = (prec == SEM_FP32) ? launch_t<float, true>(m, t, col0, ncol, a, b, c, qn, qs, qo, s)
                                    : launch_t<double, true>(m, t, col0, ncol, a, b, c, qn, qs, qo, s);
        } else {
            rc = (prec == SEM_FP32) ? launch_t<float, false>(m, t, col0, ncol, a, b, c, qn, qs, qo, s)
                                    : launch_t<double, false>(m, t, col0, ncol, a, b, c, qn, qs, qo, s);
        }
        if (rc != SEM_OK) return rc;
    }
    const int64_t n2 = int64_t(m.n_hT) * m.nzn;
    if (n2 > 0) {
        const int64_t g = std::min<int64_t>((n2 + 255) / 256, 65536);
        hipLaunchKernelGGL(k_stage_hanging, dim3(unsigned(g)), dim3(256), 0, s, m, t, c, qo);
        if (hipGetLastError() != hipSuccess) return SEM_ERR_HIP;
    }
    return SEM_OK;
}

}  // namespace sem
