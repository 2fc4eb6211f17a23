// HIP kernels and C ABI of the spectral-element right-hand-side library
// (gfx950).  See include/sem.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <array>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "adapt.h"
#include "handle.h"
#include "nodeval.h"

namespace sem {
std::string& last_error() {
    thread_local std::string msg;
    return msg;
}
}  // namespace sem

namespace {

using sem::fail;
constexpr int NF = SEM_NFIELDS;

}  // namespace

using sem::DevMesh;

// ====================================================================== kernels
namespace sem {

__global__ void k_nc_scatter(DevMesh m, const double* __restrict__ src, double* __restrict__ dst) {
    const int64_t n = int64_t(m.n_hh) * m.nzn;
    const int64_t fs = int64_t(m.n_h) * m.ldz, fsh = int64_t(m.n_hh) * m.ldz;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int hh = int(t / m.nzn), kz = int(t % m.nzn);
        double s[NF] = {0, 0, 0, 0, 0};
        for (int r = m.hang_ptr[hh]; r < m.hang_ptr[hh + 1]; ++r) {
            const double w = m.hang_w[r];
            const int64_t base = int64_t(m.hang_src[r]) * m.ldz + kz;
#pragma unroll
            for (int f = 0; f < NF; ++f) s[f] += w * src[f * fs + base];
        }
        const int64_t o = int64_t(hh) * m.ldz + kz;
#pragma unroll
        for (int f = 0; f < NF; ++f) dst[f * fsh + o] = s[f];
    }
}

__global__ void k_nc_gather(DevMesh m, const double* __restrict__ src, double* __restrict__ dst) {
    const int64_t n = int64_t(m.n_hT) * m.nzn;
    const int64_t fs = int64_t(m.n_h) * m.ldz;
    const int64_t fsh = int64_t(m.n_hh) * m.ldz;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int li = int(t / m.nzn), kz = int(t % m.nzn);
        const int h = m.hT_list[li];
        double s[NF] = {0, 0, 0, 0, 0};
        for (int r = m.hT_ptr[li]; r < m.hT_ptr[li + 1]; ++r) {
            const double w = m.hT_w[r];
            const int64_t base = int64_t(m.hT_hh[r]) * m.ldz + kz;
#pragma unroll
            for (int f = 0; f < NF; ++f) s[f] += w * src[f * fsh + base];
        }
        const int64_t o = int64_t(h) * m.ldz + kz;
#pragma unroll
        for (int f = 0; f < NF; ++f) dst[f * fs + o] += s[f];
    }
}

// Element right-hand side, one workgroup per element, one thread per node.
template <int NP, typename T>
__global__ void __launch_bounds__(((NP * NP * NP + 63) / 64) * 64)
k_rhs(DevMesh m, const double* __restrict__ q, const double* __restrict__ hv,
      double* __restrict__ rE) {
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP;
    constexpr int N = NP - 1;
    __shared__ T tile[8][NP3];
    __shared__ T sD[NP2];
    __shared__ double s_zs[NP2];          // terrain: surface height per position
    const int e = blockIdx.x;
    const int c = e / m.n_z, layer = e - c * m.n_z;
    const int t = threadIdx.x;
    if (t < NP2) sD[t] = T(m.D[t]);
    const int i = t % NP, j = (t / NP) % NP, k = t / NP2;
    const int kz = layer * N + k;
    const int64_t fs = int64_t(m.n_h) * m.ldz, fsh = int64_t(m.n_hh) * m.ldz;
    const int64_t fsr = int64_t(m.n_h + m.n_hh) * m.ldz;   // terrain reference rows
    const bool ter = m.zs != nullptr;
    if (ter && t < NP2) {
        const int gz = m.gmap[c * NP2 + t];
        s_zs[t] = m.zs[gz >= 0 ? gz : m.n_h - gz - 1];
    }
    T rp = 0, u = 0, v = 0, w = 0, tp = 0, rho = 1, rho_p = 0;
    double dth0 = 0.0;
    if (t < NP3) {
        const int g = m.gmap[c * NP2 + i + NP * j];
        double x[NF];
        if (g >= 0) {
#pragma unroll
            for (int f = 0; f < NF; ++f) x[f] = q[f * fs + int64_t(g) * m.ldz + kz];
        } else {
#pragma unroll
            for (int f = 0; f < NF; ++f) x[f] = hv[f * fsh + int64_t(-g - 1) * m.ldz + kz];
        }
        // reference state: per vertical node, or per node with terrain (the
        // hanging rows hold the coarse face's interpolant)
        double r0, ir0, ith0, p0;
        if (ter) {
            const int64_t o = int64_t(g >= 0 ? g : m.n_h - g - 1) * m.ldz + kz;
            r0 = m.ref_n[o];
            ir0 = m.ref_n[fsr + o];
            ith0 = m.ref_n[2 * fsr + o];
            p0 = m.ref_n[3 * fsr + o];
            dth0 = m.ref_n[4 * fsr + o];
        } else {
            r0 = m.rho0[kz];
            ir0 = 1.0 / r0;
            ith0 = 1.0 / m.theta0[kz];
            p0 = m.p0[kz];
            dth0 = m.dth0[kz];
        }
        rp = T(x[0]); u = T(x[1]); v = T(x[2]); w = T(x[3]); tp = T(x[4]);
        rho_p = rp;
        rho = T(r0) + rp;
        // p' = p0 expm1(gamma (log1p(rho'/rho0) + log1p(theta'/theta0))):
        // the ideal-gas pressure minus the reference pressure, free of
        // cancellation; in FP64 for both precisions, rounded once (the
        // hydrostatic balance in the w tendency cancels most of dp'/dz)
        const T pp = T(p0 * expm1(m.gamma * (log1p(x[0] * ir0) + log1p(x[4] * ith0))));
        tile[0][t] = rho * u;
        tile[1][t] = rho * v;
        tile[2][t] = rho * w;
        tile[3][t] = u;
        tile[4][t] = v;
        tile[5][t] = w;
        tile[6][t] = pp;
        tile[7][t] = tp;
    }
    __syncthreads();
    if (t >= NP3) return;
    const T sx = T(2.0 / m.col_dx[c]), sy = T(2.0 / m.col_dy[c]), sz = T(2.0 / m.dz[layer]);
    T d[8][3];
#pragma unroll
    for (int a = 0; a < 8; ++a) d[a][0] = d[a][1] = d[a][2] = 0;
#pragma unroll
    for (int mm = 0; mm < NP; ++mm) {
        const T dxm = sD[i * NP + mm], dym = sD[j * NP + mm], dzm = sD[k * NP + mm];
        const int ox = mm + NP * (j + NP * k), oy = i + NP * (mm + NP * k), oz = i + NP * (j + NP * mm);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            d[a][0] += dxm * tile[a][ox];
            d[a][1] += dym * tile[a][oy];
            d[a][2] += dzm * tile[a][oz];
        }
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) { d[a][0] *= sx; d[a][1] *= sy; d[a][2] *= sz; }
    // terrain-following mapping: d/dx = box d/dx + a_x d/dzf, d/dy likewise,
    // d/dz = g_s d/dzf (g_s = 1/(1 - zs/(H - z0)), a_x = -g_s (H - zf)/(H - z0) dzs/dx)
    double mfac = 1.0;
    if (ter) {
        double zx = 0.0, zy = 0.0;
        for (int mm = 0; mm < NP; ++mm) {
            zx += m.D[i * NP + mm] * s_zs[mm + NP * j];
            zy += m.D[j * NP + mm] * s_zs[i + NP * mm];
        }
        mfac = 1.0 - s_zs[i + NP * j] * m.inv_depth;
        const double gs = 1.0 / mfac, tg = m.tfac[kz] * gs;
        const T ax = T(-tg * zx * m.col_sx[c]), ay = T(-tg * zy * m.col_sy[c]);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            d[a][0] += ax * d[a][2];
            d[a][1] += ay * d[a][2];
            d[a][2] *= T(gs);
        }
    }
    const T f = T(m.f), g = T(m.g);
    const T inv_rho = T(1) / rho;
    T R[NF];
    R[0] = -(d[0][0] + d[1][1] + d[2][2]);
    R[1] = -(u * d[3][0] + v * d[3][1] + w * d[3][2]) - d[6][0] * inv_rho + f * v;
    R[2] = -(u * d[4][0] + v * d[4][1] + w * d[4][2]) - d[6][1] * inv_rho - f * u;
    R[3] = -(u * d[5][0] + v * d[5][1] + w * d[5][2]) - d[6][2] * inv_rho - rho_p * inv_rho * g;
    R[4] = -(u * d[7][0] + v * d[7][1] + w * d[7][2]) - w * T(dth0);
    const double mass = m.w[i] * m.w[j] * m.w[k] * 0.125 * m.col_dx[c] * m.col_dy[c] * m.dz[layer] * mfac;
    const int64_t es = int64_t(m.n_col) * m.n_z * NP3;
#pragma unroll
    for (int fld = 0; fld < NF; ++fld) rE[fld * es + int64_t(e) * NP3 + t] = mass * double(R[fld]);
}

// Sub-grid and absorbing-layer tendencies of one element, times the lumped
// mass (the paper's model setup, Section 5): horizontal Smagorinsky-Lilly,
//   R_u += d/dx(2 nu S_xx) + d/dy(2 nu S_xy), and likewise for v (S_yx, S_yy)
//   and w (S_zx, S_zy), nu = (C_s Delta)^2 sqrt(2 S:S), Delta = (dx+dy)/(2N),
// with S from the element-local velocity derivatives; and the Rayleigh layer,
// R_f -= R(kz) q'_f for every field.  accumulate = true adds to rE (the
// unfused element right-hand side), false overwrites it; col selects the
// column-row layout of rE (see sum_local).
// stacked elements of one column per workgroup (about 500 threads)
template <int NP>
constexpr int dissip_layers() { return NP * NP * NP <= 125 ? 4 : (NP * NP * NP <= 343 ? 2 : 1); }

template <int NP>
__global__ void __launch_bounds__(((dissip_layers<NP>() * NP * NP * NP + 63) / 64) * 64)
k_dissip(DevMesh m, const double* __restrict__ q, const double* __restrict__ hv,
         double* __restrict__ rE, bool accumulate, bool col) {
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP;
    constexpr int N = NP - 1;
    constexpr int L = dissip_layers<NP>(), NPL = L * NP3;
    __shared__ double sv[3][NPL];       // u, v, w of the L elements
    __shared__ double st[5][NPL];       // 2 nu (S_xx, S_xy, S_yy, S_xz, S_yz)
    __shared__ double sD[NP2];
    __shared__ double s_zs[NP2];        // terrain: surface height per position
    const int nzb = (m.n_z + L - 1) / L;
    const int c = blockIdx.x / nzb, layer0 = (blockIdx.x - c * nzb) * L;
    const int t = threadIdx.x;
    if (t < NP2) sD[t] = m.D[t];
    // node of this thread, k fastest, then the element of the stack (vertical
    // runs of the state and of the column-row output are contiguous); tl is
    // its index in the LDS tiles, el * NP3 + the element-local index
    const int k = t % NP, el = (t / NP) % L, i = (t / (NP * L)) % NP, j = t / (NP * L * NP);
    const int layer = layer0 + el;
    const bool active = t < NPL && layer < m.n_z;
    const int e = c * m.n_z + layer;
    const int eo = el * NP3;
    const int tl = eo + i + NP * (j + NP * k);
    const int kz = layer * N + k;
    const int64_t fs = int64_t(m.n_h) * m.ldz, fsh = int64_t(m.n_hh) * m.ldz;
    const bool ter = m.zs != nullptr;
    if (ter && t < NP2) {
        const int gz = m.gmap[c * NP2 + t];
        s_zs[t] = m.zs[gz >= 0 ? gz : m.n_h - gz - 1];
    }
    double x[NF] = {0, 0, 0, 0, 0};
    if (active) {
        const int g = m.gmap[c * NP2 + i + NP * j];
        if (g >= 0) {
#pragma unroll
            for (int f = 0; f < NF; ++f) x[f] = q[f * fs + int64_t(g) * m.ldz + kz];
        } else {
#pragma unroll
            for (int f = 0; f < NF; ++f) x[f] = hv[f * fsh + int64_t(-g - 1) * m.ldz + kz];
        }
        sv[0][tl] = x[1];
        sv[1][tl] = x[2];
        sv[2][tl] = x[3];
    }
    __syncthreads();
    const double sx = 2.0 / m.col_dx[c], sy = 2.0 / m.col_dy[c], sz = active ? 2.0 / m.dz[layer] : 0.0;
    // terrain-following mapping: d/dx = box d/dx + a_x d/dzf, d/dy likewise,
    // d/dz = g_s d/dzf (g_s = 1/(1 - zs/(H - z0)), a_x = -g_s (H - zf)/(H - z0) dzs/dx);
    // the lumped mass gains 1/g_s
    double ax = 0.0, ay = 0.0, gs = 1.0, mfac = 1.0;
    if (ter && active) {
        double zx = 0.0, zy = 0.0;
        for (int mm = 0; mm < NP; ++mm) {
            zx += sD[i * NP + mm] * s_zs[mm + NP * j];
            zy += sD[j * NP + mm] * s_zs[i + NP * mm];
        }
        mfac = 1.0 - s_zs[i + NP * j] * m.inv_depth;
        gs = 1.0 / mfac;
        const double tg = m.tfac[kz] * gs;
        ax = -tg * zx * sx;
        ay = -tg * zy * sy;
    }
    double R[NF] = {0, 0, 0, 0, 0};
    const bool sgs = m.cs > 0.0;
    if (sgs && active) {
        double g3[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};   // g3[a][b] = d(u_a)/d(x_b)
        for (int mm = 0; mm < NP; ++mm) {
            const double dxm = sD[i * NP + mm], dym = sD[j * NP + mm], dzm = sD[k * NP + mm];
            const int ox = eo + mm + NP * (j + NP * k), oy = eo + i + NP * (mm + NP * k),
                      oz = eo + i + NP * (j + NP * mm);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                g3[a][0] += dxm * sv[a][ox];
                g3[a][1] += dym * sv[a][oy];
                g3[a][2] += dzm * sv[a][oz];
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) { g3[a][0] *= sx; g3[a][1] *= sy; g3[a][2] *= sz; }
        if (ter) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                g3[a][0] += ax * g3[a][2];
                g3[a][1] += ay * g3[a][2];
                g3[a][2] *= gs;
            }
        }
        const double sxx = g3[0][0], syy = g3[1][1], szz = g3[2][2];
        const double sxy = 0.5 * (g3[0][1] + g3[1][0]);
        const double sxz = 0.5 * (g3[0][2] + g3[2][0]);
        const double syz = 0.5 * (g3[1][2] + g3[2][1]);
        const double ss = sxx * sxx + syy * syy + szz * szz + 2.0 * (sxy * sxy + sxz * sxz + syz * syz);
        const double delta = (m.col_dx[c] + m.col_dy[c]) / (2.0 * N);
        const double cd = m.cs * delta;
        const double two_nu = 2.0 * cd * cd * sqrt(2.0 * ss);
        st[0][tl] = two_nu * sxx;
        st[1][tl] = two_nu * sxy;
        st[2][tl] = two_nu * syy;
        st[3][tl] = two_nu * sxz;
        st[4][tl] = two_nu * syz;
    }
    __syncthreads();
    if (!active) return;
    if (sgs) {
        double dx_[5] = {0, 0, 0, 0, 0}, dy_[5] = {0, 0, 0, 0, 0}, dz_[5] = {0, 0, 0, 0, 0};
        for (int mm = 0; mm < NP; ++mm) {
            const double dxm = sD[i * NP + mm], dym = sD[j * NP + mm], dzm = sD[k * NP + mm];
            const int ox = eo + mm + NP * (j + NP * k), oy = eo + i + NP * (mm + NP * k),
                      oz = eo + i + NP * (j + NP * mm);
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                dx_[a] += dxm * st[a][ox];
                dy_[a] += dym * st[a][oy];
                if (ter) dz_[a] += dzm * st[a][oz];
            }
        }
        // physical d/dx and d/dy of the stresses (box part plus the mapping's)
        double tx[5], ty[5];
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            tx[a] = dx_[a] * sx + ax * (dz_[a] * sz);
            ty[a] = dy_[a] * sy + ay * (dz_[a] * sz);
        }
        R[1] = tx[0] + ty[1];
        R[2] = tx[1] + ty[2];
        R[3] = tx[3] + ty[4];
    }
    if (m.sponge) {
        double rz = m.sponge[kz];
        if (ter) {
            // the layer at the node's physical height z = H - t_f (H - z0 - zs)
            const double zp = m.z_top - m.tfac[kz] * (m.depth - s_zs[i + NP * j]);
            rz = 0.0;
            if (zp >= m.z_top - m.sp_depth) {
                const double sn = sin(0.5 * M_PI * (1.0 - (m.z_top - zp) / m.sp_depth));
                rz = fmin(1.0, fmax(0.0, m.sp_gamma * sn * sn));
            }
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) R[f] -= rz * x[f];
    }
    const double mass = m.w[i] * m.w[j] * m.w[k] * 0.125 * m.col_dx[c] * m.col_dy[c] * m.dz[layer] * mfac;
    const int64_t es = int64_t(m.n_col) * m.n_z * NP3;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const int64_t o = f * es + (col ? (int64_t(c) * NP2 + i + NP * j) * (int64_t(m.n_z) * NP) + layer * NP + k
                                        : int64_t(e) * NP3 + (tl - eo));
        rE[o] = (accumulate ? rE[o] : 0.0) + mass * R[f];
    }
}

// sum of element contributions at the local copies of (slot-list, kz)
// rE layouts: element-local [F][elem][k][j][i] (col = false, the sem_rhs /
// sem_dss layout), or column rows [F][col][pos][layer][k] (col = true, the
// dissipation pre-pass's own buffer), where consecutive kz are contiguous.
__device__ __forceinline__ void sum_local(const DevMesh& m, const double* __restrict__ rE,
                                          const int* __restrict__ slots, int s0, int s1, int kz,
                                          double* out, bool col) {
    const int np1 = m.N + 1, np2 = np1 * np1, np3 = np2 * np1;
    const int64_t es = int64_t(m.n_col) * m.n_z * np3;
    int lay[2], kk[2], nv = 0;
    if (kz % m.N == 0 && kz > 0 && kz < m.nzn - 1) {
        lay[0] = kz / m.N - 1; kk[0] = m.N;
        lay[1] = kz / m.N;     kk[1] = 0;
        nv = 2;
    } else {
        lay[0] = (kz == m.nzn - 1) ? m.n_z - 1 : kz / m.N;
        kk[0] = kz - lay[0] * m.N;
        nv = 1;
    }
    for (int f = 0; f < NF; ++f) out[f] = 0.0;
    for (int s = s0; s < s1; ++s) {
        const int slot = slots[s];
        const int c = slot / np2, pos = slot - c * np2;
        for (int a = 0; a < nv; ++a) {
            const int64_t idx = col ? (int64_t(c) * np2 + pos) * (int64_t(m.n_z) * np1) + lay[a] * np1 + kk[a]
                                    : int64_t(c * m.n_z + lay[a]) * np3 + pos + np2 * kk[a];
#pragma unroll
            for (int f = 0; f < NF; ++f) out[f] += rE[f * es + idx];
        }
    }
}

__global__ void k_assemble(DevMesh m, const double* __restrict__ rE, double* __restrict__ acc, bool col) {
    const int64_t n = int64_t(m.n_h) * m.nzn;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int h = int(t / m.nzn), kz = int(t % m.nzn);
        double s[NF];
        sum_local(m, rE, m.asm_slot, m.asm_ptr[h], m.asm_ptr[h + 1], kz, s, col);
        const int64_t o = int64_t(h) * m.ldz + kz, fs = int64_t(m.n_h) * m.ldz;
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f * fs + o] = s[f];
    }
}

__global__ void k_assemble_hang(DevMesh m, const double* __restrict__ rE, double* __restrict__ cH, bool col) {
    const int64_t n = int64_t(m.n_hh) * m.nzn;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int hh = int(t / m.nzn), kz = int(t % m.nzn);
        double s[NF];
        sum_local(m, rE, m.asmH_slot, m.asmH_ptr[hh], m.asmH_ptr[hh + 1], kz, s, col);
        const int64_t o = int64_t(hh) * m.ldz + kz, fsh = int64_t(m.n_hh) * m.ldz;
#pragma unroll
        for (int f = 0; f < NF; ++f) cH[f * fsh + o] = s[f];
    }
}

// r = M_G^-1 acc at unique node (h, kz), then the boundary rules: rigid lids;
// with terrain the surface keeps only the tangential part of the momentum
// tendency
__device__ __forceinline__ void finalize_node(const DevMesh& m, int h, int kz, double* v) {
    const bool ter = m.zs != nullptr;
    const double minv = (ter ? m.minv_ht[h] : m.minv_h[h]) * m.minv_v[kz];
    const bool lid = ter ? (kz == m.nzn - 1) : (kz == 0 || kz == m.nzn - 1);
#pragma unroll
    for (int f = 0; f < NF; ++f) v[f] *= minv;
    if (ter && kz == 0) {
        const double n0 = m.nrm[h], n1 = m.nrm[m.n_h + h], n2 = m.nrm[2 * m.n_h + h];
        const double dn = v[1] * n0 + v[2] * n1 + v[3] * n2;
        v[1] -= dn * n0;
        v[2] -= dn * n1;
        v[3] -= dn * n2;
    }
    if (lid) v[3] = 0.0;
}

__global__ void k_finalize(DevMesh m, const double* __restrict__ acc, double* __restrict__ r) {
    const int64_t n = int64_t(m.n_h) * m.nzn;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int h = int(t / m.nzn), kz = int(t % m.nzn);
        const int64_t o = int64_t(h) * m.ldz + kz, fs = int64_t(m.n_h) * m.ldz;
        double v[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) v[f] = acc[f * fs + o];
        finalize_node(m, h, kz, v);
#pragma unroll
        for (int f = 0; f < NF; ++f) r[f * fs + o] = v[f];
    }
}

// assemble and finalize in one pass, for meshes without hanging points (no
// Z^T contribution has to arrive between the two)
__global__ void k_assemble_finalize(DevMesh m, const double* __restrict__ rE, double* __restrict__ r, bool col) {
    const int64_t n = int64_t(m.n_h) * m.nzn;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int h = int(t / m.nzn), kz = int(t % m.nzn);
        double v[NF];
        sum_local(m, rE, m.asm_slot, m.asm_ptr[h], m.asm_ptr[h + 1], kz, v, col);
        finalize_node(m, h, kz, v);
        const int64_t o = int64_t(h) * m.ldz + kz, fs = int64_t(m.n_h) * m.ldz;
#pragma unroll
        for (int f = 0; f < NF; ++f) r[f * fs + o] = v[f];
    }
}

__global__ void k_update(int64_t n, double a, double b, double c, const double* qn,
                         const double* qs, const double* r, double* qout) {
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n;
         t += int64_t(gridDim.x) * blockDim.x)
        qout[t] = a * qn[t] + b * qs[t] + c * r[t];
}

struct Thr { double v[SEM_MAX_LEVEL]; };

template <int NP>
__global__ void __launch_bounds__(((NP * NP * NP + 63) / 64) * 64)
k_amr_elem(DevMesh m, const double* __restrict__ q, int criterion, Thr thr, int lvl_max,
           int8_t* __restrict__ adapt) {
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, N = NP - 1;
    __shared__ double su[NP3], sv[NP3];
    __shared__ double red[1024 / 64];
    __shared__ double s_zs[NP2];          // terrain: surface height per position
    const int e = blockIdx.x;
    const int c = e / m.n_z, layer = e - c * m.n_z;
    const int t = threadIdx.x;
    const int i = t % NP, j = (t / NP) % NP, k = t / NP2;
    const int kz = layer * N + k;
    if (m.zs && t < NP2) {
        const int gz = m.gmap[c * NP2 + t];
        s_zs[t] = m.zs[gz >= 0 ? gz : m.n_h - gz - 1];
    }
    double u = 0, v = 0, w = 0;
    if (t < NP3) {
        const int g = m.gmap[c * NP2 + i + NP * j];
        u = node_value(m, q, g, 1, kz);
        v = node_value(m, q, g, 2, kz);
        w = node_value(m, q, g, 3, kz);
        su[t] = u;
        sv[t] = v;
    }
    __syncthreads();
    double C = -INFINITY;
    if (t < NP3) {
        if (criterion == SEM_CRIT_SPEED) {
            C = sqrt(u * u + v * v + w * w);
        } else {
            double vx = 0, uy = 0;
            for (int mm = 0; mm < NP; ++mm) {
                vx += m.D[i * NP + mm] * sv[mm + NP * (j + NP * k)];
                uy += m.D[j * NP + mm] * su[i + NP * (mm + NP * k)];
            }
            C = vx * (2.0 / m.col_dx[c]) - uy * (2.0 / m.col_dy[c]);
            if (m.zs) {
                // terrain-following mapping: d/dx = box d/dx + a_x d/dzf, d/dy likewise
                double vz = 0, uz = 0, zx = 0, zy = 0;
                for (int mm = 0; mm < NP; ++mm) {
                    vz += m.D[k * NP + mm] * sv[i + NP * (j + NP * mm)];
                    uz += m.D[k * NP + mm] * su[i + NP * (j + NP * mm)];
                    zx += m.D[i * NP + mm] * s_zs[mm + NP * j];
                    zy += m.D[j * NP + mm] * s_zs[i + NP * mm];
                }
                const double sz = 2.0 / m.dz[layer];
                const double tg = m.tfac[kz] / (1.0 - s_zs[i + NP * j] * m.inv_depth);
                const double ax = -tg * zx * (2.0 / m.col_dx[c]), ay = -tg * zy * (2.0 / m.col_dy[c]);
                C += ax * vz * sz - ay * uz * sz;
            }
        }
    }
    // workgroup maximum
    for (int off = 32; off > 0; off >>= 1) C = fmax(C, __shfl_xor(C, off));
    if ((t & 63) == 0) red[t >> 6] = C;
    __syncthreads();
    if (t == 0) {
        double cm = red[0];
        for (int a = 1; a < int(blockDim.x >> 6); ++a) cm = fmax(cm, red[a]);
        const int lv = m.col_level[c];
        int8_t flag = 0;
        if (lv < lvl_max && cm > thr.v[lv]) flag = 1;
        else if (lv > 0 && cm <= thr.v[lv - 1]) flag = -1;
        adapt[e] = flag;
    }
}

__global__ void k_amr_col(DevMesh m, const int8_t* __restrict__ ae, int8_t* __restrict__ ac) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m.n_col) return;
    ac[c] = column_rule(m, ae, c);
}

// Solution transfer between two meshes with the same vertical structure:
// every row (new horizontal node) is a short weighted sum of old horizontal
// nodes, applied to the whole vertical row of each field.  One wavefront per
// row and field; kz fastest, so reads and writes are whole 128-byte lines.
// The padding entries kz in [nzn, ldz) are written as zero.
__global__ void __launch_bounds__(64)
k_transfer(const int32_t* __restrict__ ptr, const int32_t* __restrict__ src,
           const double* __restrict__ w, int64_t n_rows, int64_t n_h_from, int nzn, int ldz,
           const double* __restrict__ qa, double* __restrict__ qb) {
    for (int64_t t = blockIdx.x; t < n_rows * SEM_NFIELDS; t += gridDim.x) {
        const int64_t h = t % n_rows;
        const int f = int(t / n_rows);
        const int r0 = ptr[h], r1 = ptr[h + 1];
        const double* qf = qa + f * n_h_from * ldz;
        double* out = qb + (f * n_rows + h) * ldz;
        for (int kz = threadIdx.x; kz < ldz; kz += 64) {
            double acc = 0.0;
            if (kz < nzn)
                for (int r = r0; r < r1; ++r) acc += w[r] * qf[int64_t(src[r]) * ldz + kz];
            out[kz] = acc;
        }
    }
}

}  // namespace sem

// ====================================================================== helpers
namespace {

int grid_for(int64_t n, int block = 256) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return int(g);
}

template <typename T>
int launch_rhs_t(const sem_mesh* M, const double* q, const double* hv, double* rE, hipStream_t s) {
    const DevMesh& d = M->d;
    const int nb = d.n_col * d.n_z;
    switch (d.N) {
#define CASE(NN)                                                                             \
    case NN:                                                                                 \
        hipLaunchKernelGGL((sem::k_rhs<NN + 1, T>), dim3(nb), dim3((((NN + 1) * (NN + 1) * (NN + 1) + 63) / 64) * 64), 0, s, d, q, hv, rE); \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: return fail(SEM_ERR_N, "unsupported N");
    }
    HIPCHK(hipGetLastError());
    return SEM_OK;
}

int check_mesh(const sem_mesh* M) {
    if (!M) return fail(SEM_ERR_ARG, "null mesh");
    if (!M->have_ref && !M->d.zs)
        return fail(SEM_ERR_STATE, "sem_mesh_set_reference has not been called");
    return SEM_OK;
}


}  // namespace

// m * (sub-grid + absorbing-layer tendency) of every element into rE
// (added to what is there when accumulate is true), in the element layout or
// in column rows (col)
int launch_dissip(const sem_mesh* M, const double* q, const double* hv, double* rE, bool accumulate,
                  bool col, hipStream_t s) {
    const DevMesh& d = M->d;
    switch (d.N) {
#define CASE(NN)                                                                                  \
    case NN: {                                                                                    \
        constexpr int L = sem::dissip_layers<NN + 1>();                                           \
        const int nb = d.n_col * ((d.n_z + L - 1) / L);                                           \
        hipLaunchKernelGGL((sem::k_dissip<NN + 1>), dim3(nb),                                     \
                           dim3(((L * (NN + 1) * (NN + 1) * (NN + 1) + 63) / 64) * 64), 0, s, d, q, \
                           hv, rE, accumulate, col);                                              \
        break;                                                                                    \
    }
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: return fail(SEM_ERR_N, "unsupported N");
    }
    HIPCHK(hipGetLastError());
    return SEM_OK;
}

bool dissipation_on(const sem_mesh* M) { return M->d.cs > 0.0 || M->d.sponge != nullptr; }

static int sem_launch_rhs(const sem_mesh* M, const double* q, const double* hv, double* rE, int prec,
                   hipStream_t s) {
    int rc;
    if (prec == SEM_FP64) rc = launch_rhs_t<double>(M, q, hv, rE, s);
    else if (prec == SEM_FP32) rc = launch_rhs_t<float>(M, q, hv, rE, s);
    else return fail(SEM_ERR_ARG, "precision must be SEM_FP64 or SEM_FP32");
    if (rc == SEM_OK && dissipation_on(M)) rc = launch_dissip(M, q, hv, rE, true, false, s);
    return rc;
}

// dissipation tendency of q per unique node (M^-1 Z^T m R_dissip, lid rule)
// into the handle's buffer, read by the fused stage
int dissip_prepass(const sem_mesh* M, const double* q, hipStream_t s) {
    const DevMesh& d = M->d;
    const double* hv = nullptr;
    if (d.n_hh > 0) {
        hipLaunchKernelGGL(sem::k_nc_scatter, dim3(grid_for(int64_t(d.n_hh) * d.nzn)), dim3(256), 0, s, d, q,
                           M->diss_c);
        hv = M->diss_c;
    }
    // the pre-pass's own element buffer in column rows: the assembly then
    // reads consecutive kz from consecutive addresses
    int rc = launch_dissip(M, q, hv, M->diss_rE, false, true, s);
    if (rc != SEM_OK) return rc;
    if (d.n_hh == 0) {
        hipLaunchKernelGGL(sem::k_assemble_finalize, dim3(grid_for(int64_t(d.n_h) * d.nzn)), dim3(256), 0, s, d,
                           M->diss_rE, M->diss_r, true);
        HIPCHK(hipGetLastError());
        return SEM_OK;
    }
    hipLaunchKernelGGL(sem::k_assemble, dim3(grid_for(int64_t(d.n_h) * d.nzn)), dim3(256), 0, s, d, M->diss_rE,
                       M->diss_acc, true);
    hipLaunchKernelGGL(sem::k_assemble_hang, dim3(grid_for(int64_t(d.n_hh) * d.nzn)), dim3(256), 0, s, d,
                       M->diss_rE, M->diss_c, true);
    hipLaunchKernelGGL(sem::k_nc_gather, dim3(grid_for(int64_t(d.n_hT) * d.nzn)), dim3(256), 0, s, d,
                       M->diss_c, M->diss_acc);
    hipLaunchKernelGGL(sem::k_finalize, dim3(grid_for(int64_t(d.n_h) * d.nzn)), dim3(256), 0, s, d, M->diss_acc,
                       M->diss_r);
    HIPCHK(hipGetLastError());
    return SEM_OK;
}

// ====================================================================== C ABI
extern "C" {

const char* sem_last_error(void) { return sem::last_error().c_str(); }

static int sem_mesh_create_impl(const sem_mesh_desc* desc, sem_mesh** out) {
    if (!desc || !out) return fail(SEM_ERR_ARG, "null argument");
    *out = nullptr;
    sem::MeshInput in{desc->N, desc->nx0, desc->ny0, desc->n_z, desc->n_col,
                      desc->h_col_level, desc->h_col_ix, desc->h_col_iy, desc->Lx, desc->Ly,
                      desc->h_z_edges, desc->periodic_x != 0, desc->periodic_y != 0,
                      desc->f, desc->g, desc->R_d, desc->c_p, desc->p00};
    std::unique_ptr<sem_mesh> M(new sem_mesh());
    std::string err;
    int rc = sem::build_host_mesh(in, M->host, err);
    if (rc != SEM_OK) return fail(rc, err);
    const sem::HostMesh& H = M->host;
    DevMesh& d = M->d;
    d.N = H.N; d.n_z = H.n_z; d.nzn = H.nzn; d.ldz = H.ldz; d.n_col = H.n_col;
    d.n_h = int(H.n_h); d.n_hh = int(H.n_hh); d.n_hT = int(H.hT_list.size());
    d.f = H.f; d.g = H.g;
    d.gamma = H.c_p / (H.c_p - H.R_d);
    {
        // C(gamma, n) by the product rule in extended precision
        long double cgam = (long double)H.c_p / ((long double)H.c_p - (long double)H.R_d);
        long double cn = 1.0L;
        d.binom[0] = 1.0;
        for (int n = 1; n <= 10; ++n) {
            cn *= (cgam - (long double)(n - 1)) / (long double)n;
            d.binom[n] = (double)cn;
        }
    }
#define UP(vec, field) if ((rc = M->upload(vec, &d.field)) != SEM_OK) return rc;
    UP(H.gmap, gmap) UP(H.col_dx, col_dx) UP(H.col_dy, col_dy) UP(H.dz, dz)
    UP(H.col_sx, col_sx) UP(H.col_sy, col_sy) UP(H.sz, sz)
    UP(H.hang_ptr, hang_ptr) UP(H.hang_src, hang_src) UP(H.hang_w, hang_w)
    UP(H.hT_list, hT_list) UP(H.hT_ptr, hT_ptr) UP(H.hT_hh, hT_hh) UP(H.hT_w, hT_w)
    UP(H.asm_ptr, asm_ptr) UP(H.asm_slot, asm_slot) UP(H.asmH_ptr, asmH_ptr)
    UP(H.asmH_slot, asmH_slot) UP(H.minv_h, minv_h) UP(H.minv_v, minv_v)
    UP(H.sib, sib) UP(H.col_level, col_level) UP(H.basis.D, D) UP(H.basis.w, w)
    UP(H.nbr_ptr, nbr_ptr) UP(H.nbr_col, nbr_col)
#undef UP
    if ((rc = M->upload(H.h_xy, &M->d_hxy)) != SEM_OK) return rc;
    HIPCHK(hipMalloc(&M->wind_part, sizeof(double) * 256));
    HIPCHK(hipMalloc(&M->feat_aux, sizeof(double) * 2 * size_t(std::max<int64_t>(1, int64_t(H.n_col) * H.n_z))));
    M->ws_bytes += int64_t(sizeof(double)) * 2 * int64_t(H.n_col) * H.n_z;
    if ((rc = sem::fused_plan_build(H, SEM_LAYOUT_COLUMNS, 0, M->fused)) != SEM_OK)
        return fail(rc, "could not build the fused-stage tables");
    *out = M.release();
    return SEM_OK;
}

int sem_mesh_create(const sem_mesh_desc* desc, sem_mesh** out) {
    return sem::guarded("sem_mesh_create", [&] { return sem_mesh_create_impl(desc, out); });
}

static int sem_mesh_plan_impl(const sem_mesh_desc* desc, sem_mesh_info* o, double* hxy, double* hhxy, double* z,
                  double* mass) {
    if (!desc || !o) return fail(SEM_ERR_ARG, "null argument");
    sem::MeshInput in{desc->N, desc->nx0, desc->ny0, desc->n_z, desc->n_col,
                      desc->h_col_level, desc->h_col_ix, desc->h_col_iy, desc->Lx, desc->Ly,
                      desc->h_z_edges, desc->periodic_x != 0, desc->periodic_y != 0,
                      desc->f, desc->g, desc->R_d, desc->c_p, desc->p00};
    sem::HostMesh H;
    std::string err;
    int rc = sem::build_host_mesh(in, H, err);
    if (rc != SEM_OK) return fail(rc, err);
    o->N = H.N; o->n_z = H.n_z; o->nzn = H.nzn; o->ldz = H.ldz; o->max_level = H.max_level;
    o->n_col = H.n_col; o->n_elem = int64_t(H.n_col) * H.n_z;
    o->n_h = H.n_h; o->n_hh = H.n_hh;
    o->n_dof = H.n_h * H.nzn; o->n_hang = H.n_hh * H.nzn;
    o->n_local = o->n_elem * H.np1 * H.np1 * H.np1;
    o->workspace_bytes = 0;
    if (hxy) std::memcpy(hxy, H.h_xy.data(), H.h_xy.size() * sizeof(double));
    if (hhxy) std::memcpy(hhxy, H.hh_xy.data(), H.hh_xy.size() * sizeof(double));
    if (z) std::memcpy(z, H.zn.data(), H.zn.size() * sizeof(double));
    if (mass)
        for (int64_t h = 0; h < H.n_h; ++h)
            for (int kz = 0; kz < H.nzn; ++kz)
                mass[h * H.nzn + kz] = 1.0 / (H.minv_h[h] * H.minv_v[kz]);
    return SEM_OK;
}

int sem_mesh_plan(const sem_mesh_desc* desc, sem_mesh_info* o, double* hxy, double* hhxy, double* z,
                  double* mass) {
    return sem::guarded("sem_mesh_plan", [&] { return sem_mesh_plan_impl(desc, o, hxy, hhxy, z, mass); });
}

int sem_mesh_destroy(sem_mesh* mesh) {
    if (!mesh) return fail(SEM_ERR_ARG, "null mesh");
    delete mesh;
    return SEM_OK;
}

int sem_mesh_get_info(const sem_mesh* M, sem_mesh_info* o) {
    if (!M || !o) return fail(SEM_ERR_ARG, "null argument");
    const sem::HostMesh& H = M->host;
    o->N = H.N; o->n_z = H.n_z; o->nzn = H.nzn; o->ldz = H.ldz; o->max_level = H.max_level;
    o->n_col = H.n_col; o->n_elem = int64_t(H.n_col) * H.n_z;
    o->n_h = H.n_h; o->n_hh = H.n_hh;
    o->n_dof = H.n_h * H.nzn; o->n_hang = H.n_hh * H.nzn;
    o->n_local = o->n_elem * H.np1 * H.np1 * H.np1;
    o->workspace_bytes = M->ws_bytes + M->fused.bytes;
    return SEM_OK;
}

static int sem_mesh_coords_impl(const sem_mesh* M, double* hxy, double* hhxy, double* z) {
    if (!M) return fail(SEM_ERR_ARG, "null mesh");
    const sem::HostMesh& H = M->host;
    if (hxy) std::memcpy(hxy, H.h_xy.data(), H.h_xy.size() * sizeof(double));
    if (hhxy) std::memcpy(hhxy, H.hh_xy.data(), H.hh_xy.size() * sizeof(double));
    if (z) std::memcpy(z, H.zn.data(), H.zn.size() * sizeof(double));
    return SEM_OK;
}

int sem_mesh_coords(const sem_mesh* M, double* hxy, double* hhxy, double* z) {
    return sem::guarded("sem_mesh_coords", [&] { return sem_mesh_coords_impl(M, hxy, hhxy, z); });
}

static int sem_mesh_set_reference_impl(sem_mesh* M, const double* rho0, const double* theta0,
                           const double* dth0) {
    if (!M || !rho0 || !theta0 || !dth0) return fail(SEM_ERR_ARG, "null argument");
    const sem::HostMesh& H = M->host;
    std::vector<double> r(rho0, rho0 + H.nzn), t(theta0, theta0 + H.nzn), dt(dth0, dth0 + H.nzn),
        p0(H.nzn), ir(H.nzn), it(H.nzn);
    const double gam = H.c_p / (H.c_p - H.R_d);
    for (int k = 0; k < H.nzn; ++k) {
        if (!(r[k] > 0) || !(t[k] > 0)) return fail(SEM_ERR_ARG, "reference state must be positive");
        p0[k] = H.p00 * std::pow(H.R_d * r[k] * t[k] / H.p00, gam);
        ir[k] = 1.0 / r[k];
        it[k] = 1.0 / t[k];
    }
    const std::vector<double>* src[6] = {&r, &t, &dt, &p0, &ir, &it};
    const double** dst[6] = {&M->d.rho0, &M->d.theta0, &M->d.dth0, &M->d.p0, &M->d.inv_rho0,
                             &M->d.inv_theta0};
    for (int q = 0; q < 6; ++q) {
        if (M->have_ref) {
            HIPCHK(hipMemcpy((void*)*dst[q], src[q]->data(), H.nzn * 8, hipMemcpyHostToDevice));
        } else {
            int rc = M->upload(*src[q], dst[q]);
            if (rc != SEM_OK) return rc;
        }
    }
    M->have_ref = true;
    ++M->epoch;
    return SEM_OK;
}

int sem_mesh_set_reference(sem_mesh* M, const double* rho0, const double* theta0,
                           const double* dth0) {
    return sem::guarded("sem_mesh_set_reference", [&] { return sem_mesh_set_reference_impl(M, rho0, theta0, dth0); });
}

static int sem_mesh_set_terrain_impl(sem_mesh* M, const double* zs, const double* rho0, const double* theta0,
                         const double* dth0) {
    if (!M) return fail(SEM_ERR_ARG, "null mesh");
    const sem::HostMesh& H = M->host;
    DevMesh& d = M->d;
    HIPCHK(hipDeviceSynchronize());
    if (!zs) {
        d.zs = d.nrm = d.minv_ht = d.ref_n = d.tfac = nullptr;
        M->zs_host.clear();
        ++M->epoch;
        return SEM_OK;
    }
    if (!rho0 || !theta0 || !dth0) return fail(SEM_ERR_ARG, "null reference array");
    const double z0 = H.z_edges.front(), top = H.z_edges.back(), depth = top - z0;
    for (int64_t h = 0; h < H.n_h; ++h)
        if (!(zs[h] >= 0.0) || !(zs[h] < depth))
            return fail(SEM_ERR_ARG, "terrain heights must lie in [0, H - z0)");
    const int np1 = H.np1, np2 = np1 * np1, nzn = H.nzn, ldz = H.ldz;
    const int64_t nh = H.n_h, nhh = H.n_hh;
    for (int64_t h = 0; h < nh; ++h)
        for (int k = 0; k < nzn; ++k)
            if (!(rho0[h * nzn + k] > 0.0) || !(theta0[h * nzn + k] > 0.0))
                return fail(SEM_ERR_ARG, "reference state must be positive");
    // one buffer: zs[n_h + n_hh], nrm[3][n_h], minv_ht[n_h],
    // ref_n[5][n_h + n_hh][ldz] (hanging points after the unique nodes), tfac[nzn]
    const int64_t fs = (nh + nhh) * ldz;
    const int64_t total = nh + nhh + 3 * nh + nh + 5 * fs + nzn;
    std::vector<double> buf(size_t(total), 0.0);
    double* b_zs = buf.data();
    double* b_zh = b_zs + nh;
    double* b_n = b_zh + nhh;
    double* b_mi = b_n + 3 * nh;
    double* b_ref = b_mi + nh;
    double* b_tf = b_ref + 5 * fs;
    const double gam = H.c_p / (H.c_p - H.R_d);
    auto fill_ref = [&](double* dst, int64_t stride, int64_t o, double r, double t, double dt) {
        dst[o] = r;
        dst[stride + o] = 1.0 / r;
        dst[2 * stride + o] = 1.0 / t;
        dst[3 * stride + o] = H.p00 * std::pow(H.R_d * r * t / H.p00, gam);
        dst[4 * stride + o] = dt;
    };
    for (int64_t h = 0; h < nh; ++h) {
        b_zs[h] = zs[h];
        for (int k = 0; k < nzn; ++k) {
            const int64_t src = h * nzn + k;
            fill_ref(b_ref, fs, h * ldz + k, rho0[src], theta0[src], dth0[src]);
        }
    }
    // hanging points: the coarse face's interpolant of zs and of the reference
    for (int64_t hh = 0; hh < nhh; ++hh) {
        double z = 0.0;
        for (int32_t r = H.hang_ptr[hh]; r < H.hang_ptr[hh + 1]; ++r) z += H.hang_w[r] * zs[H.hang_src[r]];
        b_zh[hh] = z;
        for (int k = 0; k < nzn; ++k) {
            double ri = 0.0, ti = 0.0, di = 0.0;
            for (int32_t r = H.hang_ptr[hh]; r < H.hang_ptr[hh + 1]; ++r) {
                const int64_t src = int64_t(H.hang_src[r]) * nzn + k;
                ri += H.hang_w[r] * rho0[src];
                ti += H.hang_w[r] * theta0[src];
                di += H.hang_w[r] * dth0[src];
            }
            if (!(ri > 0.0) || !(ti > 0.0)) return fail(SEM_ERR_ARG, "reference state must be positive");
            fill_ref(b_ref, fs, (nh + hh) * ldz + k, ri, ti, di);
        }
    }
    // per column position: the element-local gradient of zs (LGL derivative
    // of its nodal values times 2/dx, 2/dy) and the horizontal lumped mass
    // with the terrain factor (1 - zs/(H - z0)); both are summed onto the
    // unique horizontal nodes, hanging positions through their rows (Z^T)
    std::vector<double> gx(size_t(nh), 0.0), gy(size_t(nh), 0.0), wt(size_t(nh), 0.0), mh(size_t(nh), 0.0);
    const std::vector<double>& Dm = H.basis.D;
    const std::vector<double>& w = H.basis.w;
    std::vector<double> zp(static_cast<size_t>(np2));
    for (int c = 0; c < H.n_col; ++c) {
        const int32_t* gm = &H.gmap[size_t(c) * np2];
        for (int p = 0; p < np2; ++p) zp[p] = gm[p] >= 0 ? zs[gm[p]] : b_zh[-gm[p] - 1];
        for (int j = 0; j < np1; ++j)
            for (int i = 0; i < np1; ++i) {
                double sx = 0.0, sy = 0.0;
                for (int m = 0; m < np1; ++m) {
                    sx += Dm[i * np1 + m] * zp[j * np1 + m];
                    sy += Dm[j * np1 + m] * zp[m * np1 + i];
                }
                sx *= H.col_sx[c];
                sy *= H.col_sy[c];
                const double wij = w[i] * w[j] * 0.25 * H.col_dx[c] * H.col_dy[c];
                const double mt = wij * (1.0 - zp[j * np1 + i] / depth);
                const int32_t g = gm[j * np1 + i];
                auto add = [&](int64_t h, double f) {
                    gx[h] += f * mt * sx;
                    gy[h] += f * mt * sy;
                    wt[h] += f * mt;
                    mh[h] += f * mt;
                };
                if (g >= 0) add(g, 1.0);
                else
                    for (int32_t r = H.hang_ptr[-g - 1]; r < H.hang_ptr[-g]; ++r) add(H.hang_src[r], H.hang_w[r]);
            }
    }
    for (int64_t h = 0; h < nh; ++h) {
        if (!(mh[h] > 0.0)) return fail(SEM_ERR_MESH, "non-positive assembled mass");
        const double nx = -gx[h] / wt[h], ny = -gy[h] / wt[h];
        const double inv = 1.0 / std::sqrt(1.0 + nx * nx + ny * ny);
        b_n[h] = nx * inv;
        b_n[nh + h] = ny * inv;
        b_n[2 * nh + h] = inv;
        b_mi[h] = 1.0 / mh[h];
    }
    for (int k = 0; k < nzn; ++k) b_tf[k] = (top - H.zn[k]) / depth;
    if (M->terrain_bytes != int64_t(sizeof(double)) * total) {
        if (M->terrain_buf) {
            (void)hipFree(M->terrain_buf);
            M->ws_bytes -= M->terrain_bytes;
            M->terrain_buf = nullptr;
            M->terrain_bytes = 0;
        }
        HIPCHK(hipMalloc(&M->terrain_buf, sizeof(double) * total));
        M->terrain_bytes = int64_t(sizeof(double)) * total;
        M->ws_bytes += M->terrain_bytes;
    }
    HIPCHK(hipMemcpy(M->terrain_buf, buf.data(), sizeof(double) * total, hipMemcpyHostToDevice));
    double* base = M->terrain_buf;
    d.zs = base;
    d.nrm = base + nh + nhh;
    d.minv_ht = d.nrm + 3 * nh;
    d.ref_n = d.minv_ht + nh;
    d.tfac = d.ref_n + 5 * fs;
    d.inv_depth = 1.0 / depth;
    d.z_top = top;
    d.depth = depth;
    M->zs_host.assign(zs, zs + nh);
    ++M->epoch;
    return SEM_OK;
}

int sem_mesh_set_terrain(sem_mesh* M, const double* zs, const double* rho0, const double* theta0,
                         const double* dth0) {
    return sem::guarded("sem_mesh_set_terrain", [&] { return sem_mesh_set_terrain_impl(M, zs, rho0, theta0, dth0); });
}

static int sem_mesh_heights_impl(const sem_mesh* M, const double* zs, double* z) {
    if (!M || !z) return fail(SEM_ERR_ARG, "null argument");
    const sem::HostMesh& H = M->host;
    const double z0 = H.z_edges.front(), top = H.z_edges.back(), depth = top - z0;
    const double* s = zs ? zs : (M->zs_host.empty() ? nullptr : M->zs_host.data());
    if (zs)
        for (int64_t h = 0; h < H.n_h; ++h)
            if (!(zs[h] >= 0.0) || !(zs[h] < depth))
                return fail(SEM_ERR_ARG, "terrain heights must lie in [0, H - z0)");
    for (int64_t h = 0; h < H.n_h; ++h)
        for (int k = 0; k < H.nzn; ++k) {
            const double zf = H.zn[k];
            z[h * H.nzn + k] = s ? zf + s[h] * (top - zf) / depth : zf;
        }
    return SEM_OK;
}

int sem_mesh_heights(const sem_mesh* M, const double* zs, double* z) {
    return sem::guarded("sem_mesh_heights", [&] { return sem_mesh_heights_impl(M, zs, z); });
}

static int sem_nc_project_impl(const sem_mesh* M, int dir, const double* src, double* dst, void* stream) {
    if (!M) return fail(SEM_ERR_ARG, "null mesh");
    if (dir != SEM_SCATTER && dir != SEM_GATHER) return fail(SEM_ERR_ARG, "bad direction");
    const DevMesh& d = M->d;
    if (d.n_hh == 0) return SEM_OK;
    if (!src || !dst) return fail(SEM_ERR_ARG, "null array");
    hipStream_t s = (hipStream_t)stream;
    if (dir == SEM_SCATTER)
        hipLaunchKernelGGL(sem::k_nc_scatter, dim3(grid_for(int64_t(d.n_hh) * d.nzn)), dim3(256), 0, s, d, src, dst);
    else
        hipLaunchKernelGGL(sem::k_nc_gather, dim3(grid_for(int64_t(d.n_hT) * d.nzn)), dim3(256), 0, s, d, src, dst);
    HIPCHK(hipGetLastError());
    return SEM_OK;
}

int sem_nc_project(const sem_mesh* M, int dir, const double* src, double* dst, void* stream) {
    return sem::guarded("sem_nc_project", [&] { return sem_nc_project_impl(M, dir, src, dst, stream); });
}

static int sem_rhs_impl(const sem_mesh* M, const double* q, const double* hv, double* rE, int prec, void* stream) {
    int rc = check_mesh(M);
    if (rc != SEM_OK) return rc;
    if (!q || !rE || (M->d.n_hh > 0 && !hv)) return fail(SEM_ERR_ARG, "null array");
    return sem_launch_rhs(M, q, hv, rE, prec, (hipStream_t)stream);
}

int sem_rhs(const sem_mesh* M, const double* q, const double* hv, double* rE, int prec, void* stream) {
    return sem::guarded("sem_rhs", [&] { return sem_rhs_impl(M, q, hv, rE, prec, stream); });
}

static int sem_dss_impl(const sem_mesh* M, int phase, const double* rE, double* acc, double* c, double* r,
            void* stream) {
    if (!M) return fail(SEM_ERR_ARG, "null mesh");
    const DevMesh& d = M->d;
    hipStream_t s = (hipStream_t)stream;
    if (phase == SEM_ASSEMBLE) {
        if (!rE || !acc || (d.n_hh > 0 && !c)) return fail(SEM_ERR_ARG, "null array");
        hipLaunchKernelGGL(sem::k_assemble, dim3(grid_for(int64_t(d.n_h) * d.nzn)), dim3(256), 0, s, d, rE, acc,
                           false);
        if (d.n_hh > 0)
            hipLaunchKernelGGL(sem::k_assemble_hang, dim3(grid_for(int64_t(d.n_hh) * d.nzn)), dim3(256), 0, s, d, rE, c,
                               false);
    } else if (phase == SEM_FINALIZE) {
        if (!acc || !r) return fail(SEM_ERR_ARG, "null array");
        hipLaunchKernelGGL(sem::k_finalize, dim3(grid_for(int64_t(d.n_h) * d.nzn)), dim3(256), 0, s, d, acc, r);
    } else {
        return fail(SEM_ERR_ARG, "bad phase");
    }
    HIPCHK(hipGetLastError());
    return SEM_OK;
}

int sem_dss(const sem_mesh* M, int phase, const double* rE, double* acc, double* c, double* r,
            void* stream) {
    return sem::guarded("sem_dss", [&] { return sem_dss_impl(M, phase, rE, acc, c, r, stream); });
}

static int sem_stage_update_impl(const sem_mesh* M, double a, double b, double c, const double* qn,
                     const double* qs, const double* r, double* qout, void* stream) {
    if (!M) return fail(SEM_ERR_ARG, "null mesh");
    if (!qn || !qs || !r || !qout) return fail(SEM_ERR_ARG, "null array");
    const int64_t n = int64_t(NF) * M->d.n_h * M->d.ldz;
    hipLaunchKernelGGL(sem::k_update, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, n, a, b, c,
                       qn, qs, r, qout);
    HIPCHK(hipGetLastError());
    return SEM_OK;
}

int sem_stage_update(const sem_mesh* M, double a, double b, double c, const double* qn,
                     const double* qs, const double* r, double* qout, void* stream) {
    return sem::guarded("sem_stage_update", [&] { return sem_stage_update_impl(M, a, b, c, qn, qs, r, qout, stream); });
}

static int sem_stage_impl(const sem_mesh* M, double a, double b, double c, const double* qn, const double* qs,
              double* qout, int prec, void* stream) {
    int rc = check_mesh(M);
    if (rc != SEM_OK) return rc;
    if (!qn || !qs || !qout) return fail(SEM_ERR_ARG, "null array");
    if (qout == qs || qout == qn) return fail(SEM_ERR_ARG, "qout must not alias qs or qn");
    if (prec != SEM_FP64 && prec != SEM_FP32) return fail(SEM_ERR_ARG, "bad precision");
    if (dissipation_on(M) && !sem::fused_dissipation_inline(M->d, M->fused, prec) &&
        (rc = dissip_prepass(M, qs, (hipStream_t)stream)) != SEM_OK)
        return rc;
    rc = sem::fused_stage_launch(M->d, M->fused, a, b, c, qn, qs, qout, prec, (hipStream_t)stream);
    if (rc != SEM_OK) return fail(rc, "fused stage launch failed");
    return SEM_OK;
}

int sem_stage(const sem_mesh* M, double a, double b, double c, const double* qn, const double* qs,
              double* qout, int prec, void* stream) {
    return sem::guarded("sem_stage", [&] { return sem_stage_impl(M, a, b, c, qn, qs, qout, prec, stream); });
}

static int sem_mesh_set_dissipation_impl(sem_mesh* M, double cs, double sponge_gamma, double sponge_depth) {
    if (!M) return fail(SEM_ERR_ARG, "null mesh");
    if (!(cs >= 0.0) || !(sponge_gamma >= 0.0) || (sponge_gamma > 0.0 && !(sponge_depth > 0.0)))
        return fail(SEM_ERR_ARG, "need Cs >= 0, sponge_gamma >= 0 and sponge_depth > 0");
    const sem::HostMesh& H = M->host;
    DevMesh& d = M->d;
    HIPCHK(hipDeviceSynchronize());
    if (cs == 0.0 && sponge_gamma == 0.0) {
        d.cs = 0.0;
        d.sponge = nullptr;
        d.rx = nullptr;
        ++M->epoch;
        return SEM_OK;
    }
    const int64_t nloc = int64_t(H.n_col) * H.n_z * H.np1 * H.np1 * H.np1;
    const int64_t nst = int64_t(NF) * H.n_h * H.ldz, nhs = int64_t(NF) * H.n_hh * H.ldz;
    if (!M->diss_rE) {
        HIPCHK(hipMalloc(&M->diss_rE, sizeof(double) * NF * nloc));
        HIPCHK(hipMalloc(&M->diss_acc, sizeof(double) * nst));
        HIPCHK(hipMalloc(&M->diss_r, sizeof(double) * nst));
        HIPCHK(hipMalloc(&M->diss_c, sizeof(double) * std::max<int64_t>(nhs, 1)));
        HIPCHK(hipMalloc(&M->diss_sponge, sizeof(double) * H.nzn));
        // the row padding of the tendency stays zero (finalize writes kz < nzn only)
        HIPCHK(hipMemset(M->diss_r, 0, sizeof(double) * nst));
        M->ws_bytes += int64_t(sizeof(double)) * (NF * nloc + 2 * nst + std::max<int64_t>(nhs, 1) + H.nzn);
    }
    // absorbing layer per vertical node: min(1, max(0, gamma sin^2(pi/2 (1 - (z_top - z)/depth))))
    // inside z >= z_top - depth, zero below
    std::vector<double> sp(H.nzn, 0.0);
    const double ztop = H.z_edges.back();
    for (int kz = 0; kz < H.nzn; ++kz) {
        const double z = H.zn[kz];
        if (sponge_gamma > 0.0 && z >= ztop - sponge_depth) {
            const double sn = std::sin(0.5 * M_PI * (1.0 - (ztop - z) / sponge_depth));
            sp[kz] = std::min(1.0, std::max(0.0, sponge_gamma * sn * sn));
        }
    }
    HIPCHK(hipMemcpy(M->diss_sponge, sp.data(), sizeof(double) * H.nzn, hipMemcpyHostToDevice));
    d.cs = cs;
    d.sponge = sponge_gamma > 0.0 ? M->diss_sponge : nullptr;
    d.sp_gamma = sponge_gamma;
    d.sp_depth = sponge_depth;
    d.rx = M->diss_r;
    ++M->epoch;
    return SEM_OK;
}

int sem_mesh_set_dissipation(sem_mesh* M, double cs, double sponge_gamma, double sponge_depth) {
    return sem::guarded("sem_mesh_set_dissipation", [&] { return sem_mesh_set_dissipation_impl(M, cs, sponge_gamma, sponge_depth); });
}

static int sem_stage_set_layout_impl(sem_mesh* M, int layout, int param) {
    if (!M) return fail(SEM_ERR_ARG, "null mesh");
    const bool columns = layout == SEM_LAYOUT_COLUMNS || layout == SEM_LAYOUT_COLUMNS_KZ ||
                         layout == SEM_LAYOUT_COLUMNS_SPLIT;
    if (!columns && layout != SEM_LAYOUT_BLOCKS)
        return fail(SEM_ERR_ARG, "unknown layout");
    if (param < 0) return fail(SEM_ERR_ARG, "negative layout parameter");
    if (columns && param > 0 && !sem::fused_lpc_supported(M->host.N, param))
        return fail(SEM_ERR_ARG, "unsupported layers_per_chunk for this order");
    if (layout == SEM_LAYOUT_COLUMNS_SPLIT && param > 0 && !sem::fused_split_supported(M->host.N, param))
        return fail(SEM_ERR_ARG, "the split-element order needs two or more layers per chunk");
    if (layout == SEM_LAYOUT_BLOCKS && !sem::fused_blocks_supported(M->host))
        return fail(SEM_ERR_ARG, "no block layout for this mesh (order 3 to 5 with 2 x 2 column blocks)");
    sem::FusedPlan P;
    int rc = sem::fused_plan_build(M->host, layout, param, P);
    if (rc != SEM_OK) { sem::fused_plan_free(P); return fail(rc, "could not build the fused-stage tables"); }
    HIPCHK(hipDeviceSynchronize());
    sem::fused_plan_free(M->fused);
    M->fused = P;
    ++M->epoch;
    return SEM_OK;
}

int sem_stage_set_layout(sem_mesh* M, int layout, int param) {
    return sem::guarded("sem_stage_set_layout", [&] { return sem_stage_set_layout_impl(M, layout, param); });
}

int sem_stage_get_layout(const sem_mesh* M, int* layout, int* param) {
    if (!M || !layout || !param) return fail(SEM_ERR_ARG, "null argument");
    *layout = M->fused.layout;
    *param = M->fused.layout == SEM_LAYOUT_BLOCKS ? M->fused.bt.n_seg : M->fused.t.layers_per_chunk;
    return SEM_OK;
}

static int sem_stage_tune_impl(sem_mesh* M, int layers_per_chunk) {
    if (!M) return fail(SEM_ERR_ARG, "null mesh");
    if (layers_per_chunk < 0 ||
        (layers_per_chunk > 0 && !sem::fused_lpc_supported(M->host.N, layers_per_chunk)))
        return fail(SEM_ERR_ARG, "unsupported layers_per_chunk for this order");
    return sem_stage_set_layout(M, SEM_LAYOUT_COLUMNS, layers_per_chunk);
}

int sem_stage_tune(sem_mesh* M, int layers_per_chunk) {
    return sem::guarded("sem_stage_tune", [&] { return sem_stage_tune_impl(M, layers_per_chunk); });
}

static int sem_stage_autotune_impl(sem_mesh* M, const double* qn, const double* qs, double* qout, int prec,
                       int reps, int* best_lpc, float* best_ms, void* stream) {
    int rc = check_mesh(M);
    if (rc != SEM_OK) return rc;
    if (!qn || !qs || !qout) return fail(SEM_ERR_ARG, "null array");
    if (qout == qs || qout == qn) return fail(SEM_ERR_ARG, "qout must not alias qs or qn");
    if (prec != SEM_FP64 && prec != SEM_FP32) return fail(SEM_ERR_ARG, "bad precision");
    if (reps < 1) reps = 5;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // candidates: single columns in chunks of 1, 2, 4, 8 layers, in FP64 in
    // each thread order (float runs the natural order in any); column
    // blocks in 1, 2, 4, ... vertical segments (distinct segment lengths)
    std::vector<std::pair<int, int>> cand;
    for (int lpc = 1; lpc <= 16; lpc *= 2)
        if (sem::fused_lpc_supported(M->host.N, lpc) && lpc <= 2 * M->host.n_z) {
            cand.push_back({SEM_LAYOUT_COLUMNS, lpc});
            if (prec == SEM_FP64) {
                cand.push_back({SEM_LAYOUT_COLUMNS_KZ, lpc});
                if (sem::fused_split_supported(M->host.N, lpc))
                    cand.push_back({SEM_LAYOUT_COLUMNS_SPLIT, lpc});
            }
        }
    if (sem::fused_blocks_supported(M->host) && !M->d.zs) {
        int last_ls = -1;
        for (int S = 1; S <= M->host.n_z; S *= 2) {
            const int ls = (M->host.n_z + S - 1) / S;
            if (ls == last_ls) continue;
            last_ls = ls;
            cand.push_back({SEM_LAYOUT_BLOCKS, S});
        }
    }
    int best = -1;
    float best_t = 0.0f;
    for (size_t ci = 0; ci < cand.size(); ++ci) {
        sem::FusedPlan P;
        if (sem::fused_plan_build(M->host, cand[ci].first, cand[ci].second, P) != SEM_OK) {
            sem::fused_plan_free(P);
            continue;
        }
        // warm-up, then timed repetitions (the stage coefficients do not
        // change the work; qout is scratch here)
        rc = sem::fused_stage_launch(M->d, P, 0.5, 0.5, 1e-3, qn, qs, qout, prec, s);
        if (rc == SEM_OK) {
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < reps && rc == SEM_OK; ++r)
                rc = sem::fused_stage_launch(M->d, P, 0.5, 0.5, 1e-3, qn, qs, qout, prec, s);
            (void)hipEventRecord(e1, s);
        }
        float ms = 0.0f;
        if (rc == SEM_OK && hipEventSynchronize(e1) == hipSuccess &&
            hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
            ms /= float(reps);
            if (best < 0 || ms < best_t) { best = int(ci); best_t = ms; }
        }
        (void)hipStreamSynchronize(s);
        sem::fused_plan_free(P);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best < 0) return fail(SEM_ERR_HIP, "autotuning found no working configuration");
    if ((rc = sem_stage_set_layout(M, cand[best].first, cand[best].second)) != SEM_OK) return rc;
    if (best_lpc) *best_lpc = M->fused.t.layers_per_chunk;
    if (best_ms) *best_ms = best_t;
    return SEM_OK;
}

int sem_stage_autotune(sem_mesh* M, const double* qn, const double* qs, double* qout, int prec,
                       int reps, int* best_lpc, float* best_ms, void* stream) {
    return sem::guarded("sem_stage_autotune", [&] { return sem_stage_autotune_impl(M, qn, qs, qout, prec, reps, best_lpc, best_ms, stream); });
}

int sem_stage_get_tune(const sem_mesh* M, int* layers_per_chunk) {
    if (!M || !layers_per_chunk) return fail(SEM_ERR_ARG, "null argument");
    *layers_per_chunk = M->fused.t.layers_per_chunk;
    return SEM_OK;
}

int sem_mesh_get_epoch(const sem_mesh* M, int64_t* epoch) {
    if (!M || !epoch) return fail(SEM_ERR_ARG, "null argument");
    *epoch = M->epoch;
    return SEM_OK;
}

static int amr_flag_impl(const sem_mesh* M, const double* q, int criterion, const double* thr, int lvl_max,
             int8_t* ae, int8_t* ac, void* stream) {
    if (!M) return fail(SEM_ERR_ARG, "null mesh");
    if (!q || !ae || !ac) return fail(SEM_ERR_ARG, "null array");
    if (criterion != SEM_CRIT_SPEED && criterion != SEM_CRIT_VORTZ) return fail(SEM_ERR_ARG, "bad criterion");
    if (lvl_max < 0 || lvl_max > SEM_MAX_LEVEL) return fail(SEM_ERR_ARG, "lvl_max out of range");
    if (lvl_max > 0 && !thr) return fail(SEM_ERR_ARG, "null thresholds");
    sem::Thr T{};
    for (int l = 0; l < lvl_max; ++l) {
        T.v[l] = thr[l];
        if (l > 0 && thr[l] < thr[l - 1]) return fail(SEM_ERR_ARG, "thresholds must be non-decreasing");
    }
    const DevMesh& d = M->d;
    hipStream_t s = (hipStream_t)stream;
    const int nb = d.n_col * d.n_z;
    switch (d.N) {
#define CASE(NN)                                                                        \
    case NN:                                                                            \
        hipLaunchKernelGGL((sem::k_amr_elem<NN + 1>), dim3(nb), dim3((((NN + 1) * (NN + 1) * (NN + 1) + 63) / 64) * 64), 0, s, d, q, criterion, T, lvl_max, ae); \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: return fail(SEM_ERR_N, "unsupported N");
    }
    hipLaunchKernelGGL(sem::k_amr_col, dim3((d.n_col + 255) / 256), dim3(256), 0, s, d, ae, ac);
    HIPCHK(hipGetLastError());
    return SEM_OK;
}

int amr_flag(const sem_mesh* M, const double* q, int criterion, const double* thr, int lvl_max,
             int8_t* ae, int8_t* ac, void* stream) {
    return sem::guarded("amr_flag", [&] { return amr_flag_impl(M, q, criterion, thr, lvl_max, ae, ac, stream); });
}

// ------------------------------------------------------------ adaptation
static sem::MeshInput input_of(const sem_mesh_desc* d) {
    return sem::MeshInput{d->N, d->nx0, d->ny0, d->n_z, d->n_col, d->h_col_level, d->h_col_ix,
                          d->h_col_iy, d->Lx, d->Ly, d->h_z_edges, d->periodic_x != 0,
                          d->periodic_y != 0, d->f, d->g, d->R_d, d->c_p, d->p00};
}

static int sem_adapt_columns_impl(const sem_mesh_desc* desc, const int8_t* flags, int lvl_max, int32_t cap,
                      int32_t* lev, int32_t* ix, int32_t* iy, int32_t* n_out) {
    if (!desc || !flags || !n_out) return fail(SEM_ERR_ARG, "null argument");
    if (cap < 0 || (cap > 0 && (!lev || !ix || !iy))) return fail(SEM_ERR_ARG, "bad output arrays");
    std::vector<std::array<int32_t, 3>> out;
    std::string err;
    int rc = sem::adapt_layout(desc->nx0, desc->ny0, desc->periodic_x != 0, desc->periodic_y != 0,
                               desc->n_col, desc->h_col_level, desc->h_col_ix, desc->h_col_iy, flags,
                               lvl_max, out, err);
    if (rc != SEM_OK) return fail(rc, err);
    *n_out = int32_t(out.size());
    if (int64_t(out.size()) > cap)
        return fail(SEM_ERR_ARG, "output capacity " + std::to_string(cap) + " < " +
                                     std::to_string(out.size()) + " columns");
    for (size_t i = 0; i < out.size(); ++i) {
        lev[i] = out[i][0];
        ix[i] = out[i][1];
        iy[i] = out[i][2];
    }
    return SEM_OK;
}

int sem_adapt_columns(const sem_mesh_desc* desc, const int8_t* flags, int lvl_max, int32_t cap,
                      int32_t* lev, int32_t* ix, int32_t* iy, int32_t* n_out) {
    return sem::guarded("sem_adapt_columns", [&] { return sem_adapt_columns_impl(desc, flags, lvl_max, cap, lev, ix, iy, n_out); });
}

static int sem_transfer_plan_impl(const sem_mesh_desc* from, const sem_mesh_desc* to, int64_t* nnz,
                      int32_t* ptr, int32_t* src, double* w) {
    if (!from || !to || !nnz) return fail(SEM_ERR_ARG, "null argument");
    sem::HostMesh A, B;
    std::string err;
    int rc = sem::build_host_mesh(input_of(from), A, err);
    if (rc == SEM_OK) rc = sem::build_host_mesh(input_of(to), B, err);
    if (rc != SEM_OK) return fail(rc, err);
    sem::TransferRows T;
    if ((rc = sem::build_transfer(A, B, T, err)) != SEM_OK) return fail(rc, err);
    *nnz = int64_t(T.src.size());
    if (ptr) std::memcpy(ptr, T.ptr.data(), T.ptr.size() * sizeof(int32_t));
    if (src) std::memcpy(src, T.src.data(), T.src.size() * sizeof(int32_t));
    if (w) std::memcpy(w, T.w.data(), T.w.size() * sizeof(double));
    return SEM_OK;
}

int sem_transfer_plan(const sem_mesh_desc* from, const sem_mesh_desc* to, int64_t* nnz,
                      int32_t* ptr, int32_t* src, double* w) {
    return sem::guarded("sem_transfer_plan", [&] { return sem_transfer_plan_impl(from, to, nnz, ptr, src, w); });
}

static int sem_transfer_create_impl(const sem_mesh* from, const sem_mesh* to, sem_transfer** out) {
    if (!from || !to || !out) return fail(SEM_ERR_ARG, "null argument");
    *out = nullptr;
    sem::TransferRows T;
    std::string err;
    int rc = sem::build_transfer(from->host, to->host, T, err);
    if (rc != SEM_OK) return fail(rc, err);
    std::unique_ptr<sem_transfer> X(new sem_transfer());
    X->n_from = from->host.n_h;
    X->n_to = to->host.n_h;
    X->nzn = to->host.nzn;
    X->ldz = to->host.ldz;
    X->nnz = int64_t(T.src.size());
    for (int32_t s : T.src)
        if (s < 0 || s >= X->n_from) return fail(SEM_ERR_MESH, "transfer row source out of range");
    HIPCHK(hipMalloc(&X->ptr, T.ptr.size() * sizeof(int32_t)));
    HIPCHK(hipMemcpy(X->ptr, T.ptr.data(), T.ptr.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if (X->nnz > 0) {
        HIPCHK(hipMalloc(&X->src, T.src.size() * sizeof(int32_t)));
        HIPCHK(hipMalloc(&X->w, T.w.size() * sizeof(double)));
        HIPCHK(hipMemcpy(X->src, T.src.data(), T.src.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(X->w, T.w.data(), T.w.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    *out = X.release();
    return SEM_OK;
}

int sem_transfer_create(const sem_mesh* from, const sem_mesh* to, sem_transfer** out) {
    return sem::guarded("sem_transfer_create", [&] { return sem_transfer_create_impl(from, to, out); });
}

static int sem_transfer_apply_impl(const sem_transfer* X, const double* q_from, double* q_to, void* stream) {
    if (!X) return fail(SEM_ERR_ARG, "null transfer");
    if (!q_from || !q_to) return fail(SEM_ERR_ARG, "null array");
    if (q_from == q_to) return fail(SEM_ERR_ARG, "q_to must not alias q_from");
    if (X->n_to == 0) return SEM_OK;
    hipStream_t s = (hipStream_t)stream;
    const int64_t work = X->n_to * SEM_NFIELDS;
    const int grid = int(std::min<int64_t>(work, 1 << 20));
    hipLaunchKernelGGL(sem::k_transfer, dim3(grid), dim3(64), 0, s, X->ptr, X->src, X->w, X->n_to,
                       X->n_from, X->nzn, X->ldz, q_from, q_to);
    HIPCHK(hipGetLastError());
    return SEM_OK;
}

int sem_transfer_apply(const sem_transfer* X, const double* q_from, double* q_to, void* stream) {
    return sem::guarded("sem_transfer_apply", [&] { return sem_transfer_apply_impl(X, q_from, q_to, stream); });
}

int sem_transfer_destroy(sem_transfer* X) {
    delete X;
    return SEM_OK;
}

}  // extern "C"
