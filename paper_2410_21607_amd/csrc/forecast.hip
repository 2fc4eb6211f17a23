// Refinement forecaster, mesh side (gfx950): per-element features, the
// combination of forecast and criterion flags, and training labels.
//
// The paper's refinement criterion (Section 4.1) is a threshold on a field
// at the element's nodes; its closing section asks for better criteria.  The
// forecaster predicts, for every element, the refinement decision a few
// adaptation intervals ahead from 16 features of the element and its
// neighbours; its flags are combined with the plain criterion so that the
// criterion overrides every refinement the forecaster misses.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "handle.h"
#include "nodeval.h"

namespace sem {

namespace {

struct Scale16 { float v[SEM_NFEAT]; };
struct ThrF { double v[SEM_MAX_LEVEL]; };

// accumulators of the element pass: 13 maxima and one sum
enum { A_ZABS, A_UH, A_W, A_TMAX, A_TMIN, A_GP, A_GT, A_DIV, A_RMAX, A_RMIN, A_UHP, A_ZABSP,
       A_CRIT, A_NMAX, A_ZSUM = A_NMAX, A_N };

__device__ __forceinline__ double wave_max(double x) {
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off));
    return x;
}
__device__ __forceinline__ double wave_sum(double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

}  // namespace

// One workgroup per element, one thread per local node.  Raw features:
//  0 level, 1 max|zeta|, 2 mean zeta, 3 max|u_h|, 4 max|w|, 5 max theta',
//  6 min theta', 7 max|grad p'|, 8 max|grad theta'|, 9 max|div u|,
//  10 rho' range, 11-12 (neighbour pass), 13 change of max|u_h| and
//  14 change of max|zeta| since q_prev, 15 the criterion's own flag;
// zeta = dv/dx - du/dy and every derivative element-local (tensor-product
// LGL derivative, as in the criterion; over terrain-following coordinates the
// physical derivative by the chain rule of the mapping: d/dx = box d/dx +
// a_x d/dzf, d/dy likewise, d/dz = g_s d/dzf, and p' from the per-node
// reference).  dem = number of thresholds the criterion's element maximum
// exceeds (the level the criterion asks for).
template <int NP>
__global__ void __launch_bounds__(((NP * NP * NP + 63) / 64) * 64)
k_features(DevMesh m, const double* __restrict__ q, const double* __restrict__ qp,
           const int8_t* __restrict__ plain, int criterion, ThrF thr, int lvl_max, Scale16 sc,
           float* __restrict__ feat, double* __restrict__ aux, int8_t* __restrict__ dem) {
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, N = NP - 1;
    constexpr int NW = (NP3 + 63) / 64;
    __shared__ double su[NP3], sv[NP3], sw[NP3], st[NP3], spp[NP3], sup[NP3], svp[NP3];
    __shared__ double red[NW][A_N];
    __shared__ double s_zs[NP2];          // terrain: surface height per position
    const int e = blockIdx.x;
    const int c = e / m.n_z, layer = e - c * m.n_z;
    const int t = threadIdx.x;
    const bool act = t < NP3;
    const int i = t % NP, j = (t / NP) % NP, k = t / NP2;
    const int kz = layer * N + k;
    const bool ter = m.zs != nullptr;
    if (ter && t < NP2) {
        const int gz = m.gmap[c * NP2 + t];
        s_zs[t] = m.zs[gz >= 0 ? gz : m.n_h - gz - 1];
    }
    double rp = 0, u = 0, v = 0, w = 0, tp = 0, up = 0, vp = 0;
    if (act) {
        const int g = m.gmap[c * NP2 + i + NP * j];
        rp = node_value(m, q, g, 0, kz);
        u = node_value(m, q, g, 1, kz);
        v = node_value(m, q, g, 2, kz);
        w = node_value(m, q, g, 3, kz);
        tp = node_value(m, q, g, 4, kz);
        up = node_value(m, qp, g, 1, kz);
        vp = node_value(m, qp, g, 2, kz);
        su[t] = u; sv[t] = v; sw[t] = w; st[t] = tp; sup[t] = up; svp[t] = vp;
        // p' = p0 ((1 + rho'/rho0)(1 + theta'/theta0))^gamma - p0 without cancellation
        if (ter) {
            // per-node reference (hanging rows: the coarse face's interpolant)
            const int64_t fsr = int64_t(m.n_h + m.n_hh) * m.ldz;
            const int64_t o = int64_t(g >= 0 ? g : m.n_h - g - 1) * m.ldz + kz;
            spp[t] = m.ref_n[3 * fsr + o] *
                     expm1(m.gamma * (log1p(rp * m.ref_n[fsr + o]) + log1p(tp * m.ref_n[2 * fsr + o])));
        } else {
            spp[t] = m.p0[kz] * expm1(m.gamma * (log1p(rp / m.rho0[kz]) + log1p(tp / m.theta0[kz])));
        }
    }
    __syncthreads();
    double a[A_N];
#pragma unroll
    for (int r = 0; r < A_N; ++r) a[r] = -INFINITY;
    a[A_ZSUM] = 0.0;
    if (act) {
        const double sx = 2.0 / m.col_dx[c], sy = 2.0 / m.col_dy[c], szz = 2.0 / m.dz[layer];
        double vx = 0, uy = 0, ux = 0, vy = 0, wz = 0, px = 0, py = 0, pz = 0, tx = 0, ty = 0,
               tz = 0, vpx = 0, upy = 0;
        for (int mm = 0; mm < NP; ++mm) {
            const double dxm = m.D[i * NP + mm], dym = m.D[j * NP + mm], dzm = m.D[k * NP + mm];
            const int ox = mm + NP * (j + NP * k), oy = i + NP * (mm + NP * k), oz = i + NP * (j + NP * mm);
            vx += dxm * sv[ox]; ux += dxm * su[ox]; px += dxm * spp[ox]; tx += dxm * st[ox];
            vpx += dxm * svp[ox];
            uy += dym * su[oy]; vy += dym * sv[oy]; py += dym * spp[oy]; ty += dym * st[oy];
            upy += dym * sup[oy];
            wz += dzm * sw[oz]; pz += dzm * spp[oz]; tz += dzm * st[oz];
        }
        vx *= sx; ux *= sx; px *= sx; tx *= sx; vpx *= sx;
        uy *= sy; vy *= sy; py *= sy; ty *= sy; upy *= sy;
        wz *= szz; pz *= szz; tz *= szz;
        if (ter) {
            // terrain-following mapping: g_s = 1/(1 - zs/(H - z0)),
            // a_x = -g_s (H - zf)/(H - z0) dzs/dx, a_y likewise
            double uz = 0, vz = 0, upz = 0, vpz = 0, zx = 0, zy = 0;
            for (int mm = 0; mm < NP; ++mm) {
                const double dzm = m.D[k * NP + mm];
                const int oz = i + NP * (j + NP * mm);
                uz += dzm * su[oz]; vz += dzm * sv[oz]; upz += dzm * sup[oz]; vpz += dzm * svp[oz];
                zx += m.D[i * NP + mm] * s_zs[mm + NP * j];
                zy += m.D[j * NP + mm] * s_zs[i + NP * mm];
            }
            uz *= szz; vz *= szz; upz *= szz; vpz *= szz;
            const double gs = 1.0 / (1.0 - s_zs[i + NP * j] * m.inv_depth);
            const double tg = m.tfac[kz] * gs;
            const double ax = -tg * zx * sx, ay = -tg * zy * sy;
            vx += ax * vz; ux += ax * uz; px += ax * pz; tx += ax * tz; vpx += ax * vpz;
            uy += ay * uz; vy += ay * vz; py += ay * pz; ty += ay * tz; upy += ay * upz;
            wz *= gs; pz *= gs; tz *= gs;
        }
        const double zeta = vx - uy, zetap = vpx - upy;
        a[A_ZABS] = fabs(zeta);
        a[A_ZSUM] = zeta;
        a[A_UH] = sqrt(u * u + v * v);
        a[A_W] = fabs(w);
        a[A_TMAX] = tp;
        a[A_TMIN] = -tp;
        a[A_GP] = sqrt(px * px + py * py + pz * pz);
        a[A_GT] = sqrt(tx * tx + ty * ty + tz * tz);
        a[A_DIV] = fabs(ux + vy + wz);
        a[A_RMAX] = rp;
        a[A_RMIN] = -rp;
        a[A_UHP] = sqrt(up * up + vp * vp);
        a[A_ZABSP] = fabs(zetap);
        a[A_CRIT] = (criterion == SEM_CRIT_SPEED) ? sqrt(u * u + v * v + w * w) : zeta;
    }
#pragma unroll
    for (int r = 0; r < A_NMAX; ++r) a[r] = wave_max(a[r]);
    a[A_ZSUM] = wave_sum(a[A_ZSUM]);
    if ((t & 63) == 0)
#pragma unroll
        for (int r = 0; r < A_N; ++r) red[t >> 6][r] = a[r];
    __syncthreads();
    if (t == 0) {
        double b[A_N];
        for (int r = 0; r < A_N; ++r) b[r] = red[0][r];
        for (int q2 = 1; q2 < NW; ++q2) {
            for (int r = 0; r < A_NMAX; ++r) b[r] = fmax(b[r], red[q2][r]);
            b[A_ZSUM] += red[q2][A_ZSUM];
        }
        const int lv = m.col_level[c];
        double f[SEM_NFEAT];
        f[0] = lv;
        f[1] = b[A_ZABS];
        f[2] = b[A_ZSUM] / NP3;
        f[3] = b[A_UH];
        f[4] = b[A_W];
        f[5] = b[A_TMAX];
        f[6] = -b[A_TMIN];
        f[7] = b[A_GP];
        f[8] = b[A_GT];
        f[9] = b[A_DIV];
        f[10] = b[A_RMAX] + b[A_RMIN];
        f[11] = 0.0;
        f[12] = 0.0;
        f[13] = b[A_UH] - b[A_UHP];
        f[14] = b[A_ZABS] - b[A_ZABSP];
        f[15] = plain[e];
        for (int r = 0; r < SEM_NFEAT; ++r) feat[int64_t(e) * SEM_NFEAT + r] = float(f[r] * double(sc.v[r]));
        aux[2 * int64_t(e)] = b[A_ZABS];
        aux[2 * int64_t(e) + 1] = b[A_UH];
        int d = 0;
        for (int l = 1; l <= lvl_max; ++l)
            if (b[A_CRIT] > thr.v[l - 1]) d = l;
        dem[e] = int8_t(d);
    }
}

// features 11 and 12: the largest max|zeta| and max|u_h| over the elements of
// the same layer in the horizontal neighbour columns
__global__ void k_features_nbr(DevMesh m, const double* __restrict__ aux, Scale16 sc,
                               float* __restrict__ feat) {
    const int64_t n = int64_t(m.n_col) * m.n_z;
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int c = int(e / m.n_z), layer = int(e % m.n_z);
        double zm = 0.0, um = 0.0;
        for (int r = m.nbr_ptr[c]; r < m.nbr_ptr[c + 1]; ++r) {
            const int64_t e2 = int64_t(m.nbr_col[r]) * m.n_z + layer;
            zm = fmax(zm, aux[2 * e2]);
            um = fmax(um, aux[2 * e2 + 1]);
        }
        feat[e * SEM_NFEAT + 11] = float(zm * double(sc.v[11]));
        feat[e * SEM_NFEAT + 12] = float(um * double(sc.v[12]));
    }
}

// forecast class (argmax of the logits, first maximum on ties: 0 coarsen,
// 1 keep, 2 refine), clamped to the level range, combined with the
// criterion's flag: refine if either refines, coarsen only if both coarsen
__global__ void k_forecast_elem(DevMesh m, const float* __restrict__ logits,
                                const int8_t* __restrict__ plain, int lvl_max,
                                int8_t* __restrict__ out) {
    const int64_t n = int64_t(m.n_col) * m.n_z;
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x) {
        const float* z = logits + 3 * e;
        int cls = 0;
        if (z[1] > z[cls]) cls = 1;
        if (z[2] > z[cls]) cls = 2;
        int f = cls - 1;
        const int lv = m.col_level[int(e / m.n_z)];
        if (f == 1 && lv >= lvl_max) f = 0;
        if (f == -1 && lv == 0) f = 0;
        const int p = plain[e];
        out[e] = int8_t((p == 1 || f == 1) ? 1 : ((p == -1 && f == -1) ? -1 : 0));
    }
}

__global__ void k_forecast_col(DevMesh m, const int8_t* __restrict__ ae, int8_t* __restrict__ ac) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < m.n_col) ac[c] = column_rule(m, ae, c);
}

// maximum horizontal wind sqrt(u^2 + v^2) over the unique nodes whose
// horizontal position lies in [x0, x1] x [y0, y1]: per-block maxima, then one
// block over the partial results (a maximum does not depend on order)
constexpr int WIND_BLOCKS = 256;

__global__ void __launch_bounds__(256)
k_max_wind(DevMesh m, const double* __restrict__ q, const double* __restrict__ hxy, double x0,
           double x1, double y0, double y1, double* __restrict__ part) {
    __shared__ double red[4];
    const int64_t n = int64_t(m.n_h) * m.nzn;
    const int64_t fs = int64_t(m.n_h) * m.ldz;
    double best = 0.0;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t h = t / m.nzn;
        const int kz = int(t - h * m.nzn);
        const double x = hxy[2 * h], y = hxy[2 * h + 1];
        if (x < x0 || x > x1 || y < y0 || y > y1) continue;
        const double u = q[fs + h * m.ldz + kz], v = q[2 * fs + h * m.ldz + kz];
        best = fmax(best, sqrt(u * u + v * v));
    }
    for (int off = 32; off > 0; off >>= 1) best = fmax(best, __shfl_xor(best, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ void __launch_bounds__(256)
k_max_wind_final(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double red[4];
    double best = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) best = fmax(best, part[t]);
    for (int off = 32; off > 0; off >>= 1) best = fmax(best, __shfl_xor(best, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) *out = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

}  // namespace sem

namespace {
using sem::fail;

inline uint64_t ckey(int l, int64_t x, int64_t y) {
    return (uint64_t(l) << 58) | (uint64_t(x) << 29) | uint64_t(y);
}
}  // namespace

extern "C" {

static int amr_features_impl(const sem_mesh* M, const double* q, const double* q_prev, const int8_t* plain,
                 int criterion, const double* thr, int lvl_max, const float* scale, float* feat,
                 int8_t* dem, void* stream) {
    if (!M) return fail(SEM_ERR_ARG, "null mesh");
    if (!M->have_ref && !M->d.zs)
        return fail(SEM_ERR_STATE, "neither sem_mesh_set_reference nor sem_mesh_set_terrain has been called");
    if (!q || !q_prev || !plain || !feat || !dem || !scale) return fail(SEM_ERR_ARG, "null array");
    if (criterion != SEM_CRIT_SPEED && criterion != SEM_CRIT_VORTZ) return fail(SEM_ERR_ARG, "bad criterion");
    if (lvl_max < 0 || lvl_max > SEM_MAX_LEVEL) return fail(SEM_ERR_ARG, "lvl_max out of range");
    if (lvl_max > 0 && !thr) return fail(SEM_ERR_ARG, "null thresholds");
    sem::ThrF T{};
    for (int l = 0; l < lvl_max; ++l) {
        T.v[l] = thr[l];
        if (l > 0 && thr[l] < thr[l - 1]) return fail(SEM_ERR_ARG, "thresholds must be non-decreasing");
    }
    sem::Scale16 S{};
    for (int r = 0; r < SEM_NFEAT; ++r) S.v[r] = scale[r];
    const sem::DevMesh& d = M->d;
    hipStream_t s = (hipStream_t)stream;
    const int nb = d.n_col * d.n_z;
    switch (d.N) {
#define CASE(NN)                                                                              \
    case NN:                                                                                  \
        hipLaunchKernelGGL((sem::k_features<NN + 1>), dim3(nb),                               \
                           dim3((((NN + 1) * (NN + 1) * (NN + 1) + 63) / 64) * 64), 0, s, d, q, \
                           q_prev, plain, criterion, T, lvl_max, S, feat, M->feat_aux, dem);  \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: return fail(SEM_ERR_N, "unsupported N");
    }
    HIPCHK(hipGetLastError());
    const int grid = std::max(1, std::min((nb + 255) / 256, 65536));
    hipLaunchKernelGGL(sem::k_features_nbr, dim3(grid), dim3(256), 0, s, d, M->feat_aux, S, feat);
    HIPCHK(hipGetLastError());
    return SEM_OK;
}

int amr_features(const sem_mesh* M, const double* q, const double* q_prev, const int8_t* plain,
                 int criterion, const double* thr, int lvl_max, const float* scale, float* feat,
                 int8_t* dem, void* stream) {
    return sem::guarded("amr_features", [&] { return amr_features_impl(M, q, q_prev, plain, criterion, thr, lvl_max, scale, feat, dem, stream); });
}

static int amr_forecast_flags_impl(const sem_mesh* M, const float* logits, const int8_t* plain, int lvl_max,
                       int8_t* ae, int8_t* ac, void* stream) {
    if (!M) return fail(SEM_ERR_ARG, "null mesh");
    if (!logits || !plain || !ae || !ac) return fail(SEM_ERR_ARG, "null array");
    if (ae == plain) return fail(SEM_ERR_ARG, "d_adapt_elem must not alias d_plain_elem");
    if (lvl_max < 0 || lvl_max > SEM_MAX_LEVEL) return fail(SEM_ERR_ARG, "lvl_max out of range");
    const sem::DevMesh& d = M->d;
    hipStream_t s = (hipStream_t)stream;
    const int nb = d.n_col * d.n_z;
    const int grid = std::max(1, std::min((nb + 255) / 256, 65536));
    hipLaunchKernelGGL(sem::k_forecast_elem, dim3(grid), dim3(256), 0, s, d, logits, plain, lvl_max, ae);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(sem::k_forecast_col, dim3((d.n_col + 255) / 256), dim3(256), 0, s, d, ae, ac);
    HIPCHK(hipGetLastError());
    return SEM_OK;
}

int amr_forecast_flags(const sem_mesh* M, const float* logits, const int8_t* plain, int lvl_max,
                       int8_t* ae, int8_t* ac, void* stream) {
    return sem::guarded("amr_forecast_flags", [&] { return amr_forecast_flags_impl(M, logits, plain, lvl_max, ae, ac, stream); });
}

static int sem_max_wind_impl(const sem_mesh* M, const double* q, double x0, double x1, double y0, double y1,
                 double* vmax, void* stream) {
    if (!M) return fail(SEM_ERR_ARG, "null mesh");
    if (!q || !vmax) return fail(SEM_ERR_ARG, "null array");
    if (!(x0 <= x1 && y0 <= y1)) return fail(SEM_ERR_ARG, "empty box");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(sem::k_max_wind, dim3(sem::WIND_BLOCKS), dim3(256), 0, s, M->d, q, M->d_hxy,
                       x0, x1, y0, y1, M->wind_part);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(sem::k_max_wind_final, dim3(1), dim3(256), 0, s, M->wind_part,
                       sem::WIND_BLOCKS, vmax);
    HIPCHK(hipGetLastError());
    return SEM_OK;
}

int sem_max_wind(const sem_mesh* M, const double* q, double x0, double x1, double y0, double y1,
                 double* vmax, void* stream) {
    return sem::guarded("sem_max_wind", [&] { return sem_max_wind_impl(M, q, x0, x1, y0, y1, vmax, stream); });
}

static int sem_forecast_labels_impl(const sem_mesh_desc* at, const sem_mesh_desc* later, const int8_t* dem_later,
                        int8_t* cls) {
    if (!at || !later || !dem_later || !cls) return fail(SEM_ERR_ARG, "null argument");
    if (at->n_z != later->n_z || at->nx0 != later->nx0 || at->ny0 != later->ny0 || at->n_z < 1)
        return fail(SEM_ERR_ARG, "the two layouts differ in base grid or layers");
    const int nz = at->n_z;
    // later columns, and the largest dem per layer over the descendants of
    // every coarser cell
    std::unordered_map<uint64_t, int> col;
    std::unordered_map<uint64_t, std::vector<int8_t>> below;
    col.reserve(size_t(later->n_col) * 2);
    for (int c = 0; c < later->n_col; ++c) {
        const int l = later->h_col_level[c];
        const int64_t x = later->h_col_ix[c], y = later->h_col_iy[c];
        if (l < 0 || l > SEM_MAX_LEVEL) return fail(SEM_ERR_MESH, "bad level in the later layout");
        col[ckey(l, x, y)] = c;
        for (int a = l - 1; a >= 0; --a) {
            auto& v = below[ckey(a, x >> (l - a), y >> (l - a))];
            if (v.empty()) v.assign(nz, int8_t(-1));
            for (int z = 0; z < nz; ++z) v[z] = std::max(v[z], dem_later[int64_t(c) * nz + z]);
        }
    }
    for (int c = 0; c < at->n_col; ++c) {
        const int l = at->h_col_level[c];
        const int64_t x = at->h_col_ix[c], y = at->h_col_iy[c];
        int found = -1;
        for (int a = l; a >= 0 && found < 0; --a) {
            auto it = col.find(ckey(a, x >> (l - a), y >> (l - a)));
            if (it != col.end()) found = it->second;
        }
        const std::vector<int8_t>* desc = nullptr;
        if (found < 0) {
            auto it = below.find(ckey(l, x, y));
            if (it == below.end()) return fail(SEM_ERR_MESH, "a column of the first layout is not covered by the later one");
            desc = &it->second;
        }
        for (int z = 0; z < nz; ++z) {
            const int d = found >= 0 ? dem_later[int64_t(found) * nz + z] : (*desc)[z];
            cls[int64_t(c) * nz + z] = int8_t(std::max(-1, std::min(1, d - l)) + 1);
        }
    }
    return SEM_OK;
}

int sem_forecast_labels(const sem_mesh_desc* at, const sem_mesh_desc* later, const int8_t* dem_later,
                        int8_t* cls) {
    return sem::guarded("sem_forecast_labels", [&] { return sem_forecast_labels_impl(at, later, dem_later, cls); });
}

}  // extern "C"
