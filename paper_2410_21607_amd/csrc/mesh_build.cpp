// Host-side construction of the column mesh tables.
//
// Positions are identified by exact integer keys instead of floating-point
// coordinates.  Along one axis, a node of a level-l column sits either on the
// dyadic lattice (the column's two edges and, for even N, its midpoint) or at
// an interior LGL position, which is irrational and therefore never shared
// with a column of another level.  Lattice positions are counted in units of
// half the finest column width; interior positions are keyed by
// (level, cell, i).  Two nodes coincide exactly when their keys match.
//
// A boundary node of a fine column hangs when a coarser column containing the
// point does not have it among its own nodes (Section 3.1).  Its value is the
// coarse column's face polynomial there, and the rows are composed until every
// source is a non-hanging node (chains appear with three or more levels, or
// with odd N where coarse edge midpoints are not nodes).
#include "mesh_build.h"
#include "host_par.h"

#include <array>

#include <algorithm>
#include <cmath>
#include <map>
#include <unordered_map>
#include <utility>

#include "sem.h"

namespace sem {

// ------------------------------------------------------------------ basis
static void legendre(int N, double x, double& P, double& dP) {
    // P_N(x) and P_N'(x) by the three-term recurrence
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (N == 0) { P = 1.0; dP = 0.0; return; }
    for (int n = 2; n <= N; ++n) {
        double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
        double d2 = d0 + (2.0 * n - 1.0) * p1;   // P_n' = P_{n-2}' + (2n-1) P_{n-1}
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    P = p1; dP = d1;
}

Basis1D make_basis(int N) {
    Basis1D b;
    b.N = N;
    const int n = N + 1;
    b.x.assign(n, 0.0);
    b.w.assign(n, 0.0);
    b.D.assign(n * n, 0.0);
    b.x[0] = -1.0;
    b.x[N] = 1.0;
    for (int j = 1; j < N; ++j) {
        double x = -std::cos(M_PI * j / N);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(N, x, P, dP);
            // Legendre ODE: (1-x^2) P'' = 2x P' - N(N+1) P
            double d2P = (2.0 * x * dP - N * (N + 1.0) * P) / (1.0 - x * x);
            double dx = dP / d2P;
            x -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        b.x[j] = x;
    }
    for (int j = 0; j < n; ++j) {   // exact symmetry
        double s = 0.5 * (b.x[j] - b.x[N - j]);
        b.x[j] = s;
    }
    if (N % 2 == 0) b.x[N / 2] = 0.0;
    for (int j = 0; j < n; ++j) {
        double P, dP;
        legendre(N, b.x[j], P, dP);
        b.w[j] = 2.0 / (N * (N + 1.0) * P * P);
    }
    // barycentric weights lambda_j = 1 / prod_{k != j}(x_j - x_k)
    std::vector<double> lam(n, 1.0);
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k)
            if (k != j) lam[j] /= (b.x[j] - b.x[k]);
    for (int i = 0; i < n; ++i) {
        double row = 0.0;
        for (int j = 0; j < n; ++j) {
            if (i == j) continue;
            double d = (lam[j] / lam[i]) / (b.x[i] - b.x[j]);
            b.D[i * n + j] = d;
            row += d;
        }
        b.D[i * n + i] = -row;   // rows of D annihilate constants
    }
    return b;
}

void lagrange_weights(const Basis1D& b, double s, double* out) {
    const int n = b.N + 1;
    for (int m = 0; m < n; ++m) {
        if (std::fabs(s - b.x[m]) < 1e-13) {   // exactly on a node
            for (int k = 0; k < n; ++k) out[k] = (k == m) ? 1.0 : 0.0;
            return;
        }
    }
    for (int m = 0; m < n; ++m) {
        double v = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != m) v *= (s - b.x[k]) / (b.x[m] - b.x[k]);
        out[m] = v;
    }
}

// ------------------------------------------------------------------ keys
namespace {

constexpr int64_t GLL_TAG = int64_t(1) << 62;

struct Key2 {
    int64_t kx, ky;
    bool operator==(const Key2& o) const { return kx == o.kx && ky == o.ky; }
};
struct Key2Hash {
    size_t operator()(const Key2& k) const {
        uint64_t h = uint64_t(k.kx) * 0x9E3779B97F4A7C15ull;
        h ^= uint64_t(k.ky) + 0x632BE59BD9B4E019ull + (h << 6) + (h >> 2);
        return size_t(h);
    }
};

struct Axis {
    int n0;          // level-0 cells
    int L;           // finest level
    bool periodic;
    int64_t total() const { return int64_t(n0) << (L + 1); }
    int64_t width(int l) const { return int64_t(1) << (L - l + 1); }
    // key of node i of cell `cell` at level l
    int64_t key(int N, int l, int64_t cell, int i) const {
        int64_t W = width(l), X;
        if (i == 0) X = cell * W;
        else if (i == N) X = (cell + 1) * W;
        else if (N % 2 == 0 && 2 * i == N) X = cell * W + W / 2;
        else return GLL_TAG | (int64_t(l) << 52) | (cell << 8) | int64_t(i);
        if (periodic) X %= total();
        return X;
    }
    static bool is_lattice(int64_t k) { return (k & GLL_TAG) == 0; }
    // cells (unwrapped index) at level lc that contain the position of key k
    int candidates(int64_t k, int lc, int64_t* out) const {
        if (is_lattice(k)) {
            int64_t W = width(lc);
            if (k % W == 0) { out[0] = k / W - 1; out[1] = k / W; return 2; }
            out[0] = k / W;
            return 1;
        }
        int l = int((k >> 52) & 0x3FF);
        int64_t cell = (k >> 8) & ((int64_t(1) << 44) - 1);
        out[0] = cell >> (l - lc);
        return 1;
    }
    // reference coordinate of key k inside the (unwrapped) cell cu at level lc
    double ref_coord(const Basis1D& b, int64_t k, int lc, int64_t cu) const {
        if (is_lattice(k)) {
            int64_t W = width(lc);
            double t = double(k - cu * W) / double(W);
            return 2.0 * t - 1.0;
        }
        int l = int((k >> 52) & 0x3FF);
        int64_t cell = (k >> 8) & ((int64_t(1) << 44) - 1);
        int i = int(k & 0xFF);
        int64_t off = cell - (cu << (l - lc));
        double t = (double(off) + 0.5 * (1.0 + b.x[i])) / double(int64_t(1) << (l - lc));
        return 2.0 * t - 1.0;
    }
    bool wrap(int64_t cu, int lc, int64_t& c) const {
        int64_t nl = int64_t(n0) << lc;
        if (periodic) { c = ((cu % nl) + nl) % nl; return true; }
        if (cu < 0 || cu >= nl) return false;
        c = cu;
        return true;
    }
};

using Row = std::vector<std::pair<int32_t, double>>;

// Open-addressing table from a pair of non-negative 64-bit keys to int32
// (linear probing, load factor at most 1/2, no erase, one entry per probe):
// the numbering of ~10^6 positions needs no node allocation per entry.  The
// table starts at twice the expected size and doubles when half full.
class PairTable {
  public:
    explicit PairTable(size_t n_expected) {
        size_t cap = 16;
        while (cap < 2 * n_expected + 2) cap <<= 1;
        e_.assign(cap, Entry{-1, 0, 0});
        mask_ = cap - 1;
    }
    // value of (a, b), or -1 when absent
    int32_t find(int64_t a, int64_t b) const {
        for (size_t i = slot(a, b);; i = (i + 1) & mask_) {
            const Entry& e = e_[i];
            if (e.a < 0) return -1;
            if (e.a == a && e.b == b) return e.v;
        }
    }
    // value of (a, b); inserts v (and sets inserted) when absent
    int32_t find_or_insert(int64_t a, int64_t b, int32_t v, bool& inserted) {
        if (2 * (size_ + 1) > mask_ + 1) grow();
        for (size_t i = slot(a, b);; i = (i + 1) & mask_) {
            Entry& e = e_[i];
            if (e.a < 0) {
                e = Entry{a, b, v};
                ++size_;
                inserted = true;
                return v;
            }
            if (e.a == a && e.b == b) {
                inserted = false;
                return e.v;
            }
        }
    }
    size_t size() const { return size_; }
    template <typename F>
    void for_each(F f) const {
        for (const Entry& e : e_)
            if (e.a >= 0) f(e.a, e.b, e.v);
    }

  private:
    struct Entry {
        int64_t a, b;
        int32_t v;
    };
    void grow() {
        std::vector<Entry> old(2 * (mask_ + 1), Entry{-1, 0, 0});
        old.swap(e_);
        mask_ = e_.size() - 1;
        for (const Entry& e : old) {
            if (e.a < 0) continue;
            size_t i = slot(e.a, e.b);
            while (e_[i].a >= 0) i = (i + 1) & mask_;
            e_[i] = e;
        }
    }
    size_t slot(int64_t a, int64_t b) const {
        uint64_t h = uint64_t(a) * 0x9E3779B97F4A7C15ull;
        h ^= uint64_t(b) + 0x632BE59BD9B4E019ull + (h << 6) + (h >> 2);
        h ^= h >> 29;
        return size_t(h) & mask_;
    }
    std::vector<Entry> e_;
    size_t mask_ = 0, size_ = 0;
};

// bucket of a position key (a mix independent of the tables' slot hash)
inline int key_bucket(int64_t a, int64_t b, int P) {
    uint64_t h = uint64_t(a) ^ ((uint64_t(b) << 32) | (uint64_t(b) >> 32));
    h += 0x9E3779B97F4A7C15ull;
    h = (h ^ (h >> 30)) * 0xBF58476D1CE4E5B9ull;
    h = (h ^ (h >> 27)) * 0x94D049BB133111EBull;
    h ^= h >> 31;
    return int((h >> 32) % uint64_t(P));
}

}  // namespace

// ------------------------------------------------------------------ build
int build_host_mesh(const MeshInput& in, HostMesh& m, std::string& err) {
    if (in.N < 1 || in.N > SEM_MAX_N) { err = "N must be in [1, 8]"; return SEM_ERR_N; }
    if (in.nx0 < 1 || in.ny0 < 1 || in.n_z < 1 || in.n_col < 1) {
        err = "nx0, ny0, n_z and n_col must be positive"; return SEM_ERR_ARG;
    }
    if (!(in.Lx > 0) || !(in.Ly > 0)) { err = "Lx and Ly must be positive"; return SEM_ERR_ARG; }
    if (!in.lev || !in.ix || !in.iy || !in.z_edges) { err = "null description array"; return SEM_ERR_ARG; }
    for (int k = 0; k < in.n_z; ++k)
        if (!(in.z_edges[k + 1] > in.z_edges[k])) { err = "z_edges must increase"; return SEM_ERR_ARG; }
    const int N = in.N, np1 = N + 1, np2 = np1 * np1;
    m.N = N; m.np1 = np1; m.n_z = in.n_z; m.nzn = in.n_z * N + 1;
    // rows padded to whole 128-byte lines: a chunk of a row then starts on a
    // line boundary (packed rows, which save the line that holds little more
    // than the top node, measured 12 % slower in the column kernel)
    m.ldz = (m.nzn + 15) / 16 * 16;
    m.nx0 = in.nx0; m.ny0 = in.ny0; m.periodic_x = in.periodic_x; m.periodic_y = in.periodic_y;
    m.Lx = in.Lx; m.Ly = in.Ly;
    m.f = in.f; m.g = in.g; m.R_d = in.R_d; m.c_p = in.c_p; m.p00 = in.p00;
    if (!(in.c_p > in.R_d) || !(in.R_d > 0) || !(in.p00 > 0)) {
        err = "need c_p > R_d > 0 and p00 > 0"; return SEM_ERR_ARG;
    }
    m.basis = make_basis(N);
    const Basis1D& B = m.basis;
    m.n_col = in.n_col;
    m.col_level.assign(in.lev, in.lev + in.n_col);
    m.col_ix.assign(in.ix, in.ix + in.n_col);
    m.col_iy.assign(in.iy, in.iy + in.n_col);
    int L = 0;
    for (int c = 0; c < in.n_col; ++c) {
        int l = in.lev[c];
        if (l < 0 || l > SEM_MAX_LEVEL) { err = "column level out of range"; return SEM_ERR_MESH; }
        if (in.ix[c] < 0 || in.ix[c] >= (int64_t(in.nx0) << l) ||
            in.iy[c] < 0 || in.iy[c] >= (int64_t(in.ny0) << l)) {
            err = "column index out of range for its level"; return SEM_ERR_MESH;
        }
        L = std::max(L, l);
    }
    m.max_level = L;
    // ---- cover / overlap / 2:1 balance on the finest grid
    const int64_t nxf = int64_t(in.nx0) << L, nyf = int64_t(in.ny0) << L;
    if (nxf * nyf > (int64_t(1) << 27)) { err = "finest grid too large"; return SEM_ERR_MESH; }
    std::vector<int32_t> owner(size_t(nxf * nyf), -1);
    for (int c = 0; c < in.n_col; ++c) {
        int64_t s = int64_t(1) << (L - in.lev[c]);
        for (int64_t a = 0; a < s; ++a)
            for (int64_t b = 0; b < s; ++b) {
                int64_t fx = in.ix[c] * s + a, fy = in.iy[c] * s + b;
                int32_t& o = owner[size_t(fx * nyf + fy)];
                if (o >= 0) { err = "columns overlap"; return SEM_ERR_MESH; }
                o = c;
            }
    }
    for (auto o : owner)
        if (o < 0) { err = "columns do not cover the domain"; return SEM_ERR_MESH; }
    // the finest cells around each column (edges and corners): 2:1 balance,
    // and whether a coarser column touches the column at all (only then can
    // one of its boundary nodes hang)
    std::vector<char> has_coarser(size_t(in.n_col), 0);
    std::vector<char> unbalanced(size_t(in.n_col), 0);
    parallel_ranges(size_t(in.n_col), host_threads(owner.size()), [&](size_t c0, size_t c1, int) {
        for (size_t c = c0; c < c1; ++c) {
            const int l = in.lev[c];
            const int64_t s = int64_t(1) << (L - l);
            // the ring of finest cells just outside the column, side by side
            for (int64_t r = 0; r < 4 * (s + 1); ++r) {
                const int64_t side = r / (s + 1), k = r % (s + 1);
                int64_t a, b;
                if (side == 0) { a = k - 1; b = -1; }          // south, from the corner (-1, -1)
                else if (side == 1) { a = s; b = k - 1; }     // east
                else if (side == 2) { a = s - k; b = s; }      // north
                else { a = -1; b = s - k; }                    // west
                int64_t fx = in.ix[c] * s + a, fy = in.iy[c] * s + b;
                if (in.periodic_x) fx = ((fx % nxf) + nxf) % nxf;
                else if (fx < 0 || fx >= nxf) continue;
                if (in.periodic_y) fy = ((fy % nyf) + nyf) % nyf;
                else if (fy < 0 || fy >= nyf) continue;
                const int lo = in.lev[owner[size_t(fx * nyf + fy)]];
                if (std::abs(lo - l) > 1) unbalanced[c] = 1;
                if (lo < l) has_coarser[c] = 1;
            }
        }
    });
    for (char u : unbalanced)
        if (u) { err = "2:1 balance violated"; return SEM_ERR_MESH; }
    // ---- column geometry
    m.col_dx.resize(in.n_col); m.col_dy.resize(in.n_col);
    m.col_x0.resize(in.n_col); m.col_y0.resize(in.n_col);
    for (int c = 0; c < in.n_col; ++c) {
        double wx = in.Lx / double(int64_t(in.nx0) << in.lev[c]);
        double wy = in.Ly / double(int64_t(in.ny0) << in.lev[c]);
        m.col_dx[c] = wx; m.col_dy[c] = wy;
        m.col_x0[c] = -0.5 * in.Lx + in.ix[c] * wx;
        m.col_y0[c] = -0.5 * in.Ly + in.iy[c] * wy;
        m.col_sx.push_back(2.0 / wx);
        m.col_sy.push_back(2.0 / wy);
    }
    // ---- interior LGL positions must not meet the lattice or the
    //      interior positions of the adjacent level (checked on [0, 1])
    {
        std::vector<std::pair<double, int>> pts;
        for (int l = 0; l <= 1; ++l)
            for (int cell = 0; cell < (1 << l); ++cell)
                for (int i = 1; i < N; ++i) {
                    if (N % 2 == 0 && 2 * i == N) continue;
                    pts.push_back({(cell + 0.5 * (1.0 + B.x[i])) / (1 << l), l});
                }
        for (int q = 0; q <= 8; ++q) pts.push_back({q / 8.0, 2});
        std::sort(pts.begin(), pts.end());
        for (size_t a = 1; a < pts.size(); ++a)
            if (pts[a].second != pts[a - 1].second && pts[a].first - pts[a - 1].first < 1e-9) {
                err = "LGL positions of adjacent levels coincide"; return SEM_ERR_N;
            }
    }
    // ---- vertical
    m.z_edges.assign(in.z_edges, in.z_edges + in.n_z + 1);
    m.dz.resize(in.n_z);
    m.zn.assign(m.nzn, 0.0);
    std::vector<double> mv(m.nzn, 0.0);
    for (int e = 0; e < in.n_z; ++e) {
        m.dz[e] = in.z_edges[e + 1] - in.z_edges[e];
        m.sz.push_back(2.0 / m.dz[e]);
        for (int k = 0; k < np1; ++k) {
            int kz = e * N + k;
            if (k < N) m.zn[kz] = in.z_edges[e] + 0.5 * (1.0 + B.x[k]) * m.dz[e];
            mv[kz] += B.w[k] * 0.5 * m.dz[e];
        }
    }
    m.zn[m.nzn - 1] = in.z_edges[in.n_z];
    m.minv_v.resize(m.nzn);
    for (int kz = 0; kz < m.nzn; ++kz) m.minv_v[kz] = 1.0 / mv[kz];

    // ---- horizontal keys and hanging status
    Axis ax{in.nx0, L, in.periodic_x}, ay{in.ny0, L, in.periodic_y};
    // column of (level, ix, iy)
    PairTable cmap(size_t(in.n_col));
    auto lkey = [](int l, int64_t x) { return (int64_t(l) << 40) | x; };
    for (int c = 0; c < in.n_col; ++c) {
        bool ins;
        cmap.find_or_insert(lkey(in.lev[c], in.ix[c]), in.iy[c], c, ins);
    }
    auto kx_of = [&](int c, int i) { return ax.key(N, in.lev[c], in.ix[c], i); };
    auto ky_of = [&](int c, int j) { return ay.key(N, in.lev[c], in.iy[c], j); };

    // source column (or -1) and reference coords for every (c, pos)
    std::vector<int32_t> src_col(size_t(in.n_col) * np2, -1);
    std::vector<double> src_sx(size_t(in.n_col) * np2, 0.0), src_sy(size_t(in.n_col) * np2, 0.0);
    // columns are independent here (each writes its own slots)
    parallel_ranges(size_t(in.n_col), host_threads(size_t(in.n_col) * np2), [&](size_t c0, size_t c1, int) {
    for (int c = int(c0); c < int(c1); ++c) {
        int l = in.lev[c];
        // a coarser column holding one of c's boundary nodes owns a finest
        // cell next to c; by the 2:1 balance it is one level coarser
        if (l == 0 || !has_coarser[c]) continue;
        for (int j = 0; j < np1; ++j)
            for (int i = 0; i < np1; ++i) {
                if (i != 0 && i != N && j != 0 && j != N) continue;
                int64_t kx = kx_of(c, i), ky = ky_of(c, j);
                bool found = false;
                for (int lc = l - 1; lc < l && !found; ++lc) {
                    int64_t cxs[2], cys[2];
                    int nxc = ax.candidates(kx, lc, cxs), nyc = ay.candidates(ky, lc, cys);
                    for (int a = 0; a < nxc && !found; ++a)
                        for (int b2 = 0; b2 < nyc && !found; ++b2) {
                            int64_t cx, cy;
                            if (!ax.wrap(cxs[a], lc, cx) || !ay.wrap(cys[b2], lc, cy)) continue;
                            const int cc = cmap.find(lkey(lc, cx), cy);
                            if (cc < 0) continue;
                            // only the coarse column's lattice nodes (its edges and,
                            // for even N, its middle) can coincide with a finer
                            // column's position; its other keys carry its level
                            auto lattice_node = [&](int64_t k, auto key_of) {
                                if (!Axis::is_lattice(k)) return false;
                                if (key_of(cc, 0) == k || key_of(cc, N) == k) return true;
                                return N % 2 == 0 && key_of(cc, N / 2) == k;
                            };
                            const bool nx_ = lattice_node(kx, kx_of), ny_ = lattice_node(ky, ky_of);
                            if (nx_ && ny_) continue;   // a node of the coarse column
                            size_t s = size_t(c) * np2 + i + np1 * j;
                            src_col[s] = cc;
                            src_sx[s] = ax.ref_coord(B, kx, lc, cxs[a]);
                            src_sy[s] = ay.ref_coord(B, ky, lc, cys[b2]);
                            found = true;
                        }
                }
            }
    }
    });
    // ---- column blocks (2 x 2 squares of leaf columns of one level)
    m.col_block.assign(size_t(in.n_col), -1);
    for (int c = 0; c < in.n_col; ++c) {
        if (m.col_block[c] >= 0) continue;
        const int l = in.lev[c];
        const int64_t bx = in.ix[c] & ~int64_t(1), by = in.iy[c] & ~int64_t(1);
        if (bx + 1 >= (int64_t(in.nx0) << l) || by + 1 >= (int64_t(in.ny0) << l)) continue;
        int32_t ids[4];
        bool ok = true;
        for (int q = 0; q < 4 && ok; ++q) {
            const int32_t id = cmap.find(lkey(l, bx + (q & 1)), by + (q >> 1));
            if (id < 0 || m.col_block[id] >= 0) ok = false;
            else ids[q] = id;
        }
        if (!ok) continue;
        const int32_t b = int32_t(m.blk_cols.size() / 4);
        for (int q = 0; q < 4; ++q) {
            m.blk_cols.push_back(ids[q]);
            m.col_block[ids[q]] = b;
        }
    }
    // ---- number unique nodes (first touch) and hanging points
    // keys of lattice positions are >= 0; interior LGL keys carry GLL_TAG (also >= 0)
    // Positions strictly inside a column belong to that column alone (never
    // shared, never hanging): they take the next id directly.  The others
    // (4N per column) go through the table.
    if (int64_t(in.n_col) * np2 >= (int64_t(1) << 31)) {
        err = "mesh too large for 32-bit node indices"; return SEM_ERR_MESH;
    }
    std::vector<size_t> hh_first;   // (c, pos) slot that defined each hanging point
    // visiting order: units (a block, or a column in no block) by their
    // lowest column id; a block's positions in row order over its
    // (2N+1) x (2N+1) grid, every column slot at a position in turn
    std::vector<int64_t> visit_at(size_t(in.n_col) + 1, 0);   // first visit of each column's unit
    for (int c = 0; c < in.n_col; ++c) {
        const int32_t b = m.col_block[c];
        int64_t n = np2;
        if (b >= 0) {
            const int32_t* bc = &m.blk_cols[size_t(b) * 4];
            n = c == *std::min_element(bc, bc + 4) ? 4 * np2 : 0;
        }
        visit_at[size_t(c) + 1] = visit_at[size_t(c)] + n;
    }
    std::vector<std::array<int32_t, 3>> visit(size_t(visit_at.back()));   // (column, i, j)
    parallel_ranges(size_t(in.n_col), host_threads(visit.size()), [&](size_t c0, size_t c1, int) {
        for (size_t c = c0; c < c1; ++c) {
            size_t v = size_t(visit_at[c]);
            if (visit_at[c + 1] == visit_at[c]) continue;
            const int32_t b = m.col_block[c];
            if (b < 0) {
                for (int j = 0; j < np1; ++j)
                    for (int i = 0; i < np1; ++i) visit[v++] = {int32_t(c), i, j};
                continue;
            }
            const int32_t* bc = &m.blk_cols[size_t(b) * 4];
            for (int J = 0; J <= 2 * N; ++J)
                for (int I = 0; I <= 2 * N; ++I)
                    for (int q = 0; q < 4; ++q) {
                        const int qx = q & 1, qy = q >> 1;
                        const int i = I - qx * N, j = J - qy * N;
                        if (i < 0 || i > N || j < 0 || j > N) continue;
                        visit[v++] = {bc[q], i, j};
                    }
        }
    });
    // First-touch numbering in visiting order.  A visit is a position
    // strictly inside its column (class 0: never shared, never hanging, it
    // takes the next id), a conforming boundary position (1) or a hanging
    // one (2); the id of a keyed position is given at its first visit (its
    // leader).  Leaders are found in parallel: keys go to buckets by hash,
    // each bucket keeps visiting order and finds first occurrences with its
    // own table; one ordered pass then hands out the ids.
    const size_t nv = visit.size();
    const int T = host_threads(nv);
    std::vector<int8_t> cls(nv);
    std::vector<int64_t> kxs(nv, 0), kys(nv, 0);
    parallel_ranges(nv, T, [&](size_t b, size_t e, int) {
        for (size_t v = b; v < e; ++v) {
            const int c = visit[v][0], i = visit[v][1], j = visit[v][2];
            const size_t s = size_t(c) * np2 + i + np1 * j;
            if (src_col[s] >= 0) cls[v] = 2;
            else cls[v] = (i > 0 && i < N && j > 0 && j < N) ? 0 : 1;
            if (cls[v]) {
                kxs[v] = kx_of(c, i);
                kys[v] = ky_of(c, j);
            }
        }
    });
    const int P = T;
    std::vector<std::vector<std::vector<int32_t>>> part(static_cast<size_t>(T),
                                                        std::vector<std::vector<int32_t>>(static_cast<size_t>(P)));
    parallel_ranges(nv, T, [&](size_t b, size_t e, int t) {
        for (size_t v = b; v < e; ++v)
            if (cls[v]) part[size_t(t)][size_t(key_bucket(kxs[v], kys[v], P))].push_back(int32_t(v));
    });
    std::vector<int32_t> lead(nv, -1);
    std::vector<char> bucket_clash(size_t(P), 0);
    parallel_ranges(size_t(P), P, [&](size_t q0, size_t q1, int) {
        for (size_t q = q0; q < q1; ++q) {
            size_t cnt = 0;
            for (int t = 0; t < T; ++t) cnt += part[size_t(t)][q].size();
            PairTable conf(cnt / 2 + 16), hang(16);
            for (int t = 0; t < T; ++t)
                for (int32_t v : part[size_t(t)][q]) {
                    bool ins;
                    PairTable& tab = cls[size_t(v)] == 1 ? conf : hang;
                    lead[size_t(v)] = tab.find_or_insert(kxs[size_t(v)], kys[size_t(v)], v, ins);
                }
            hang.for_each([&](int64_t a2, int64_t b2, int32_t) {
                if (conf.find(a2, b2) >= 0) bucket_clash[q] = 1;
            });
        }
    });
    part.clear();
    // ids in visiting order: the new ids of a range of visits start after
    // those of the ranges before it (a prefix sum over the ranges)
    auto is_new = [&](size_t v) { return cls[v] == 0 || lead[v] == int32_t(v); };
    std::vector<int64_t> base_u(size_t(T) + 1, 0), base_h(size_t(T) + 1, 0);
    parallel_ranges(nv, T, [&](size_t b, size_t e, int t) {
        int64_t u = 0, h = 0;
        for (size_t v = b; v < e; ++v)
            if (is_new(v)) (cls[v] == 2 ? h : u) += 1;
        base_u[size_t(t) + 1] = u;
        base_h[size_t(t) + 1] = h;
    });
    for (int t = 0; t < T; ++t) {
        base_u[size_t(t) + 1] += base_u[size_t(t)];
        base_h[size_t(t) + 1] += base_h[size_t(t)];
    }
    const int32_t n_unique = int32_t(base_u[size_t(T)]), n_hh = int32_t(base_h[size_t(T)]);
    m.gmap.assign(size_t(in.n_col) * np2, 0);
    m.h_xy.assign(2 * size_t(n_unique), 0.0);
    m.hh_xy.assign(2 * size_t(n_hh), 0.0);
    hh_first.assign(size_t(n_hh), 0);
    std::vector<int32_t> idof(nv, -1);
    parallel_ranges(nv, T, [&](size_t b, size_t e, int t) {
        int32_t u = int32_t(base_u[size_t(t)]), h = int32_t(base_h[size_t(t)]);
        for (size_t v = b; v < e; ++v) {
            if (!is_new(v)) continue;
            const int c = visit[v][0], i = visit[v][1], j = visit[v][2];
            const size_t s = size_t(c) * np2 + i + np1 * j;
            const double x = m.col_x0[c] + 0.5 * (1.0 + B.x[i]) * m.col_dx[c];
            const double y = m.col_y0[c] + 0.5 * (1.0 + B.x[j]) * m.col_dy[c];
            if (cls[v] == 2) {
                idof[v] = h;
                m.hh_xy[2 * size_t(h)] = x;
                m.hh_xy[2 * size_t(h) + 1] = y;
                hh_first[size_t(h)] = s;
                m.gmap[s] = -(h + 1);
                ++h;
            } else {
                idof[v] = u;
                m.h_xy[2 * size_t(u)] = x;
                m.h_xy[2 * size_t(u) + 1] = y;
                m.gmap[s] = u;
                ++u;
            }
        }
    });
    parallel_ranges(nv, T, [&](size_t b, size_t e, int) {
        for (size_t v = b; v < e; ++v) {
            if (is_new(v)) continue;
            const int c = visit[v][0], i = visit[v][1], j = visit[v][2];
            const size_t s = size_t(c) * np2 + i + np1 * j;
            const int32_t id = idof[size_t(lead[v])];
            m.gmap[s] = cls[v] == 2 ? -(id + 1) : id;
        }
    });
    bool clash = false;
    for (char cb : bucket_clash) clash = clash || cb;
    if (clash) { err = "a hanging point is also a conforming node"; return SEM_ERR_MESH; }
    m.n_h = int64_t(n_unique);
    m.n_hh = int64_t(n_hh);
    if (m.n_h * int64_t(m.ldz) >= (int64_t(1) << 31) || m.n_hh * int64_t(m.ldz) >= (int64_t(1) << 31) ||
        int64_t(in.n_col) * in.n_z * np1 * np2 >= (int64_t(1) << 31)) {
        err = "mesh too large for 32-bit node indices"; return SEM_ERR_MESH;
    }
    // ---- rows of every (c, pos), composed until the sources are unique nodes
    // rows of hanging slots only (a conforming slot is the unit row of its node)
    std::vector<int32_t> row_of(size_t(in.n_col) * np2, -1);
    std::vector<Row> rows;
    std::vector<char> done(row_of.size(), 0);
    std::vector<double> wx(np1), wy(np1);
    // process coarse levels first so that sources are complete
    std::vector<int> order(in.n_col);
    for (int c = 0; c < in.n_col; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return in.lev[a] < in.lev[b]; });
    for (int c : order)
        for (int p = 0; p < np2; ++p) {
            size_t s = size_t(c) * np2 + p;
            if (src_col[s] < 0) { done[s] = 1; continue; }
            int cc = src_col[s];
            lagrange_weights(B, src_sx[s], wx.data());
            lagrange_weights(B, src_sy[s], wy.data());
            std::map<int32_t, double> acc;
            for (int b2 = 0; b2 < np1; ++b2)
                for (int a = 0; a < np1; ++a) {
                    double wt = wx[a] * wy[b2];
                    if (wt == 0.0) continue;
                    size_t ss = size_t(cc) * np2 + a + np1 * b2;
                    if (!done[ss]) { err = "hanging chain does not resolve"; return SEM_ERR_MESH; }
                    if (row_of[ss] < 0) acc[m.gmap[ss]] += wt;
                    else for (auto& e : rows[row_of[ss]]) acc[e.first] += wt * e.second;
                }
            row_of[s] = int32_t(rows.size());
            rows.emplace_back();
            for (auto& e : acc)
                if (e.second != 0.0) rows.back().push_back(e);
            done[s] = 1;
        }
    // hanging rows (one per hanging point)
    m.hang_ptr.assign(size_t(m.n_hh) + 1, 0);
    for (int64_t hh = 0; hh < m.n_hh; ++hh) {
        const Row& r = rows[row_of[hh_first[hh]]];
        for (auto& e : r) { m.hang_src.push_back(e.first); m.hang_w.push_back(e.second); }
        m.hang_ptr[hh + 1] = int32_t(m.hang_src.size());
    }
    // transposed rows (a counting sort by source, stable in hanging-point order)
    {
        std::vector<int32_t> tp(size_t(m.n_h) + 1, 0);
        for (int32_t q = 0; q < m.hang_ptr[size_t(m.n_hh)]; ++q) ++tp[size_t(m.hang_src[q]) + 1];
        for (int64_t h = 0; h < m.n_h; ++h) tp[h + 1] += tp[h];
        std::vector<int32_t> thh(size_t(tp.back()));
        std::vector<double> tw(size_t(tp.back()));
        std::vector<int32_t> fill(tp.begin(), tp.end() - 1);
        for (int64_t hh = 0; hh < m.n_hh; ++hh)
            for (int32_t q = m.hang_ptr[hh]; q < m.hang_ptr[hh + 1]; ++q) {
                const int32_t at = fill[size_t(m.hang_src[q])]++;
                thh[size_t(at)] = int32_t(hh);
                tw[size_t(at)] = m.hang_w[q];
            }
        m.hT_ptr.push_back(0);
        for (int64_t h = 0; h < m.n_h; ++h) {
            if (tp[h + 1] == tp[h]) continue;
            m.hT_list.push_back(int32_t(h));
            for (int32_t q = tp[h]; q < tp[h + 1]; ++q) {
                m.hT_hh.push_back(thh[size_t(q)]);
                m.hT_w.push_back(tw[size_t(q)]);
            }
            m.hT_ptr.push_back(int32_t(m.hT_hh.size()));
        }
    }
    // assembly CSR and horizontal lumped mass
    {
        // CSR by counting (slots in increasing order within every node)
        m.asm_ptr.assign(size_t(m.n_h) + 1, 0);
        m.asmH_ptr.assign(size_t(m.n_hh) + 1, 0);
        for (int32_t g : m.gmap) {
            if (g >= 0) ++m.asm_ptr[size_t(g) + 1];
            else ++m.asmH_ptr[size_t(-g - 1) + 1];
        }
        for (int64_t h = 0; h < m.n_h; ++h) m.asm_ptr[h + 1] += m.asm_ptr[h];
        for (int64_t h = 0; h < m.n_hh; ++h) m.asmH_ptr[h + 1] += m.asmH_ptr[h];
        m.asm_slot.assign(size_t(m.asm_ptr.back()), 0);
        m.asmH_slot.assign(size_t(m.asmH_ptr.back()), 0);
        std::vector<int32_t> fa(m.asm_ptr.begin(), m.asm_ptr.end() - 1);
        std::vector<int32_t> fh(m.asmH_ptr.begin(), m.asmH_ptr.end() - 1);
        std::vector<double> mh(size_t(m.n_h), 0.0);
        for (int c = 0; c < in.n_col; ++c)
            for (int j = 0; j < np1; ++j)
                for (int i = 0; i < np1; ++i) {
                    size_t s = size_t(c) * np2 + i + np1 * j;
                    int32_t g = m.gmap[s];
                    double mass = B.w[i] * B.w[j] * 0.25 * m.col_dx[c] * m.col_dy[c];
                    if (g >= 0) { m.asm_slot[size_t(fa[g]++)] = int32_t(s); mh[g] += mass; }
                    else {
                        m.asmH_slot[size_t(fh[-g - 1]++)] = int32_t(s);
                        for (auto& e : rows[row_of[s]]) mh[e.first] += mass * e.second;
                    }
                }
        m.minv_h.resize(size_t(m.n_h));
        for (int64_t h = 0; h < m.n_h; ++h) {
            if (!(mh[h] > 0)) { err = "non-positive assembled mass"; return SEM_ERR_MESH; }
            m.minv_h[h] = 1.0 / mh[h];
        }
    }
    // sibling families
    m.sib.assign(size_t(in.n_col) * 4, -1);
    parallel_ranges(size_t(in.n_col), host_threads(size_t(in.n_col) * np2), [&](size_t c0, size_t c1, int) {
    for (int c = int(c0); c < int(c1); ++c) {
        int l = in.lev[c];
        if (l == 0) continue;
        int64_t bx = in.ix[c] & ~int64_t(1), by = in.iy[c] & ~int64_t(1);
        int32_t ids[4];
        bool ok = true;
        for (int q = 0; q < 4 && ok; ++q) {
            const int32_t id = cmap.find(lkey(l, bx + (q & 1)), by + (q >> 1));
            if (id < 0) ok = false; else ids[q] = id;
        }
        if (ok) for (int q = 0; q < 4; ++q) m.sib[size_t(c) * 4 + q] = ids[q];
    }
    });
    // horizontal neighbours through shared unique horizontal nodes: the
    // assembly CSR lists the slots (hence columns) at every node; each range
    // of columns collects its lists, then the ranges are joined in order
    {
        const int TN = host_threads(size_t(in.n_col) * np2);
        std::vector<std::vector<int32_t>> lists(static_cast<size_t>(TN));
        std::vector<int32_t> count(size_t(in.n_col), 0);
        parallel_ranges(size_t(in.n_col), TN, [&](size_t c0, size_t c1, int t) {
            std::vector<int32_t> list;
            for (size_t c = c0; c < c1; ++c) {
                list.clear();
                for (int pos = 0; pos < np2; ++pos) {
                    const int32_t g = m.gmap[c * np2 + pos];
                    if (g < 0) continue;
                    for (int r = m.asm_ptr[size_t(g)]; r < m.asm_ptr[size_t(g) + 1]; ++r) {
                        const int32_t cc = m.asm_slot[size_t(r)] / np2;
                        if (cc != int32_t(c)) list.push_back(cc);
                    }
                }
                std::sort(list.begin(), list.end());
                list.erase(std::unique(list.begin(), list.end()), list.end());
                count[c] = int32_t(list.size());
                lists[size_t(t)].insert(lists[size_t(t)].end(), list.begin(), list.end());
            }
        });
        m.nbr_ptr.assign(size_t(in.n_col) + 1, 0);
        for (int c = 0; c < in.n_col; ++c) m.nbr_ptr[size_t(c) + 1] = m.nbr_ptr[size_t(c)] + count[size_t(c)];
        m.nbr_col.clear();
        m.nbr_col.reserve(size_t(m.nbr_ptr.back()));
        for (auto& l : lists) m.nbr_col.insert(m.nbr_col.end(), l.begin(), l.end());
    }
    return SEM_OK;
}

}  // namespace sem
