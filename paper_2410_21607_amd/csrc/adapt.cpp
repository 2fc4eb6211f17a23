// Column-layout adaptation and solution-transfer rows (host, C++17).
#include "adapt.h"

#include <algorithm>
#include <cmath>
#include <deque>
#include <unordered_map>
#include <unordered_set>
#include <utility>

#include "sem.h"

namespace sem {

namespace {

inline uint64_t ckey(int l, int64_t x, int64_t y) {
    return (uint64_t(l) << 58) | (uint64_t(x) << 29) | uint64_t(y);
}

struct Grid {
    int nx0, ny0;
    bool px, py;
    // wrap (or reject) a cell index at level l
    bool wrap(int l, int64_t& x, int64_t& y) const {
        const int64_t nx = int64_t(nx0) << l, ny = int64_t(ny0) << l;
        if (px) x = ((x % nx) + nx) % nx;
        else if (x < 0 || x >= nx) return false;
        if (py) y = ((y % ny) + ny) % ny;
        else if (y < 0 || y >= ny) return false;
        return true;
    }
};

// level of the leaf covering cell (l, x, y), or -1 when the cell is split
int covering_level(const std::unordered_set<uint64_t>& leaves, int l, int64_t x, int64_t y) {
    for (int a = l; a >= 0; --a)
        if (leaves.count(ckey(a, x >> (l - a), y >> (l - a)))) return a;
    return -1;
}

uint64_t morton(int64_t x, int64_t y) {
    uint64_t k = 0;
    for (int b = 0; b < 29; ++b) {
        k |= uint64_t((x >> b) & 1) << (2 * b);
        k |= uint64_t((y >> b) & 1) << (2 * b + 1);
    }
    return k;
}

}  // namespace

int adapt_layout(int nx0, int ny0, bool periodic_x, bool periodic_y, int n_col,
                 const int32_t* lev, const int32_t* ix, const int32_t* iy,
                 const int8_t* flags, int lvl_max,
                 std::vector<std::array<int32_t, 3>>& out, std::string& err) {
    if (nx0 < 1 || ny0 < 1 || n_col < 1 || !lev || !ix || !iy || !flags) {
        err = "adapt: bad layout arguments";
        return SEM_ERR_ARG;
    }
    if (lvl_max < 0 || lvl_max > SEM_MAX_LEVEL) {
        err = "adapt: lvl_max out of range";
        return SEM_ERR_ARG;
    }
    const Grid G{nx0, ny0, periodic_x, periodic_y};
    std::unordered_set<uint64_t> old;
    old.reserve(size_t(n_col) * 2);
    int depth_in = 0;
    for (int c = 0; c < n_col; ++c) {
        const int l = lev[c];
        if (l < 0 || l > SEM_MAX_LEVEL || ix[c] < 0 || iy[c] < 0 ||
            ix[c] >= (int64_t(nx0) << l) || iy[c] >= (int64_t(ny0) << l)) {
            err = "adapt: column " + std::to_string(c) + " out of range";
            return SEM_ERR_MESH;
        }
        if (!old.insert(ckey(l, ix[c], iy[c])).second) {
            err = "adapt: duplicate column";
            return SEM_ERR_MESH;
        }
        depth_in = std::max(depth_in, l);
    }
    // the input must tile the domain: no column inside another, full area
    {
        long double area = 0;
        for (int c = 0; c < n_col; ++c) {
            for (int a = lev[c] - 1; a >= 0; --a)
                if (old.count(ckey(a, ix[c] >> (lev[c] - a), iy[c] >> (lev[c] - a)))) {
                    err = "adapt: overlapping columns";
                    return SEM_ERR_MESH;
                }
            area += std::ldexp(1.0L, -2 * lev[c]);
        }
        if (std::fabs(double(area) - double(nx0) * ny0) > 1e-9) {
            err = "adapt: columns do not cover the domain";
            return SEM_ERR_MESH;
        }
    }
    // 1. split
    std::unordered_set<uint64_t> leaves;
    leaves.reserve(size_t(n_col) * 4);
    std::deque<std::array<int64_t, 3>> work;
    auto add = [&](int l, int64_t x, int64_t y) {
        leaves.insert(ckey(l, x, y));
        work.push_back({l, x, y});
    };
    for (int c = 0; c < n_col; ++c) {
        const int l = lev[c];
        if (flags[c] == 1 && l < lvl_max) {
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) add(l + 1, 2 * int64_t(ix[c]) + a, 2 * int64_t(iy[c]) + b);
        } else {
            add(l, ix[c], iy[c]);
        }
    }
    // 2. balance: a leaf at level l forces every neighbouring cell at level l
    // to be covered by a leaf of level >= l-1; splitting pushes new work
    while (!work.empty()) {
        const auto t = work.front();
        work.pop_front();
        const int l = int(t[0]);
        if (!leaves.count(ckey(l, t[1], t[2])) || l < 2) continue;
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy) {
                if (!dx && !dy) continue;
                int64_t x = t[1] + dx, y = t[2] + dy;
                if (!G.wrap(l, x, y)) continue;
                for (;;) {
                    const int a = covering_level(leaves, l, x, y);
                    if (a < 0 || a >= l - 1) break;
                    const int64_t px = x >> (l - a), py = y >> (l - a);
                    leaves.erase(ckey(a, px, py));
                    for (int u = 0; u < 2; ++u)
                        for (int v = 0; v < 2; ++v) add(a + 1, 2 * px + u, 2 * py + v);
                }
            }
    }
    // 3. merges, all decided on the balanced layout
    std::unordered_set<uint64_t> flagged;
    for (int c = 0; c < n_col; ++c)
        if (flags[c] == -1 && lev[c] > 0) flagged.insert(ckey(lev[c], ix[c], iy[c]));
    std::vector<std::array<int64_t, 3>> merges;
    std::unordered_set<uint64_t> seen;
    for (int c = 0; c < n_col; ++c) {
        if (flags[c] != -1 || lev[c] == 0) continue;
        const int l = lev[c];
        const int64_t px = ix[c] >> 1, py = iy[c] >> 1;
        if (!seen.insert(ckey(l - 1, px, py)).second) continue;
        bool ok = true;
        for (int u = 0; u < 2 && ok; ++u)
            for (int v = 0; v < 2 && ok; ++v) {
                const uint64_t k = ckey(l, 2 * px + u, 2 * py + v);
                ok = flagged.count(k) && leaves.count(k);
            }
        // the 12 level-l cells around the parent must not be split further
        for (int64_t x = 2 * px - 1; x <= 2 * px + 2 && ok; ++x)
            for (int64_t y = 2 * py - 1; y <= 2 * py + 2 && ok; ++y) {
                if (x >= 2 * px && x <= 2 * px + 1 && y >= 2 * py && y <= 2 * py + 1) continue;
                int64_t wx = x, wy = y;
                if (!G.wrap(l, wx, wy)) continue;
                ok = covering_level(leaves, l, wx, wy) >= 0;
            }
        if (ok) merges.push_back({l - 1, px, py});
    }
    for (const auto& m : merges) {
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v)
                leaves.erase(ckey(int(m[0]) + 1, 2 * m[1] + u, 2 * m[2] + v));
        leaves.insert(ckey(int(m[0]), m[1], m[2]));
    }
    // Morton order of the finest level present
    int depth = 0;
    std::vector<std::array<int32_t, 3>> cols;
    cols.reserve(leaves.size());
    for (uint64_t k : leaves) {
        const int l = int(k >> 58);
        cols.push_back({l, int32_t((k >> 29) & ((1u << 29) - 1)), int32_t(k & ((1u << 29) - 1))});
        depth = std::max(depth, l);
    }
    std::vector<std::pair<uint64_t, size_t>> order(cols.size());
    for (size_t i = 0; i < cols.size(); ++i) {
        const int s = depth - cols[i][0];
        order[i] = {morton(int64_t(cols[i][1]) << s, int64_t(cols[i][2]) << s), i};
    }
    std::sort(order.begin(), order.end());
    out.clear();
    out.reserve(cols.size());
    for (const auto& o : order) out.push_back(cols[o.second]);
    return SEM_OK;
}

// ------------------------------------------------------------------ transfer
namespace {

// solve A X = B in place (n x n, B n x m), Gauss-Jordan with partial pivoting
bool solve(int n, int m, std::vector<double>& A, std::vector<double>& B) {
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
        if (A[p * n + c] == 0.0) return false;
        if (p != c) {
            for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[p * n + k]);
            for (int k = 0; k < m; ++k) std::swap(B[c * m + k], B[p * m + k]);
        }
        const double inv = 1.0 / A[c * n + c];
        for (int k = 0; k < n; ++k) A[c * n + k] *= inv;
        for (int k = 0; k < m; ++k) B[c * m + k] *= inv;
        for (int r = 0; r < n; ++r) {
            if (r == c || A[r * n + c] == 0.0) continue;
            const double f = A[r * n + c];
            for (int k = 0; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            for (int k = 0; k < m; ++k) B[r * m + k] -= f * B[c * m + k];
        }
    }
    return true;
}

// 1-D projection from two children onto their parent:
// P_a = Mt^-1 I_a^T W with I_a[n][m] = l_m((x_n + 2a - 1)/2) (child node n
// seen from the parent) and Mt = sum_a I_a^T W I_a, the parent mass matrix
// integrated with the children's LGL rule.  P[a][i*np1+m].
void projection_1d(const Basis1D& b, std::vector<double> P[2]) {
    const int n = b.N + 1;
    std::vector<double> I[2];
    for (int a = 0; a < 2; ++a) {
        I[a].assign(n * n, 0.0);
        for (int r = 0; r < n; ++r)
            lagrange_weights(b, 0.5 * (b.x[r] + (2 * a - 1)), &I[a][r * n]);
    }
    std::vector<double> Mt(n * n, 0.0), rhs(n * 2 * n, 0.0);
    for (int a = 0; a < 2; ++a)
        for (int i = 0; i < n; ++i) {
            for (int k = 0; k < n; ++k) {
                double s = 0.0;
                for (int r = 0; r < n; ++r) s += I[a][r * n + i] * b.w[r] * I[a][r * n + k];
                Mt[i * n + k] += s;
            }
            for (int r = 0; r < n; ++r) rhs[i * 2 * n + a * n + r] = I[a][r * n + i] * b.w[r];
        }
    solve(n, 2 * n, Mt, rhs);
    for (int a = 0; a < 2; ++a) {
        P[a].assign(n * n, 0.0);
        for (int i = 0; i < n; ++i)
            for (int r = 0; r < n; ++r) P[a][i * n + r] = rhs[i * 2 * n + a * n + r];
    }
}

struct RowAcc {
    std::vector<std::pair<int32_t, double>> e;
    void add(int32_t s, double w) {
        if (w != 0.0) e.push_back({s, w});
    }
    void finish(double scale, TransferRows& T) {
        // stable insertion sort by source (rows hold a few dozen entries at
        // most; most rows of an unchanged column hold one)
        for (size_t k = 1; k < e.size(); ++k) {
            const std::pair<int32_t, double> v = e[k];
            size_t q = k;
            for (; q > 0 && e[q - 1].first > v.first; --q) e[q] = e[q - 1];
            e[q] = v;
        }
        size_t i = 0;
        while (i < e.size()) {
            double s = 0.0;
            size_t j = i;
            for (; j < e.size() && e[j].first == e[i].first; ++j) s += e[j].second;
            if (s != 0.0) {
                T.src.push_back(e[i].first);
                T.w.push_back(s * scale);
            }
            i = j;
        }
        T.ptr.push_back(int32_t(T.src.size()));
        e.clear();
    }
};

}  // namespace

int build_transfer(const HostMesh& A, const HostMesh& B, TransferRows& T, std::string& err) {
    if (A.N != B.N || A.nx0 != B.nx0 || A.ny0 != B.ny0 || A.n_z != B.n_z ||
        A.periodic_x != B.periodic_x || A.periodic_y != B.periodic_y || A.Lx != B.Lx ||
        A.Ly != B.Ly || A.z_edges != B.z_edges) {
        err = "transfer: the two meshes differ in order, base grid, domain or vertical layers";
        return SEM_ERR_ARG;
    }
    const int n = A.np1, n2 = n * n;
    std::unordered_map<uint64_t, int> idx;
    idx.reserve(size_t(A.n_col) * 2);
    for (int c = 0; c < A.n_col; ++c) idx[ckey(A.col_level[c], A.col_ix[c], A.col_iy[c])] = c;
    // relation of every new column to the old layout
    enum Kind : int8_t { SAME = 0, CHILD = 1, PARENT = 2 };
    std::vector<int8_t> kind(B.n_col);
    std::vector<std::array<int, 4>> src(B.n_col);
    for (int c = 0; c < B.n_col; ++c) {
        const int l = B.col_level[c];
        const int64_t x = B.col_ix[c], y = B.col_iy[c];
        auto it = idx.find(ckey(l, x, y));
        if (it != idx.end()) {
            kind[c] = SAME;
            src[c] = {it->second, -1, -1, -1};
            continue;
        }
        if (l > 0 && (it = idx.find(ckey(l - 1, x >> 1, y >> 1))) != idx.end()) {
            kind[c] = CHILD;
            src[c] = {it->second, -1, -1, -1};
            continue;
        }
        kind[c] = PARENT;
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                auto k = idx.find(ckey(l + 1, 2 * x + a, 2 * y + b));
                if (k == idx.end()) {
                    err = "transfer: column " + std::to_string(c) +
                          " of the new mesh has no counterpart one level apart";
                    return SEM_ERR_MESH;
                }
                src[c][a + 2 * b] = k->second;
            }
    }
    // (column, position) slots of every new unique horizontal node, in
    // increasing slot order: the assembly CSR of the new mesh
    const std::vector<int32_t>& hp = B.asm_ptr;
    const std::vector<int32_t>& hcp = B.asm_slot;
    std::vector<double> P[2];
    projection_1d(A.basis, P);
    std::vector<double> lx(n), ly(n);
    // value of old column co at local horizontal position pos, times wt
    auto old_local = [&](RowAcc& acc, int co, int pos, double wt) {
        const int32_t g = A.gmap[int64_t(co) * n2 + pos];
        if (g >= 0) {
            acc.add(g, wt);
            return;
        }
        const int hh = -g - 1;
        for (int r = A.hang_ptr[hh]; r < A.hang_ptr[hh + 1]; ++r) acc.add(A.hang_src[r], wt * A.hang_w[r]);
    };
    T.ptr.assign(1, 0);
    T.ptr.reserve(size_t(B.n_h) + 1);
    T.src.clear();
    T.w.clear();
    T.src.reserve(size_t(B.n_h) * 2);
    T.w.reserve(size_t(B.n_h) * 2);
    RowAcc acc;
    for (int64_t h = 0; h < B.n_h; ++h) {
        int pick = -1;   // a SAME slot first, else a CHILD slot
        for (int r = hp[h]; r < hp[h + 1]; ++r) {
            const int c = hcp[r] / n2;
            if (kind[c] == SAME) { pick = hcp[r]; break; }
            if (kind[c] == CHILD && pick < 0) pick = hcp[r];
        }
        if (pick >= 0) {
            const int c = pick / n2, pos = pick % n2;
            if (kind[c] == SAME) {
                old_local(acc, src[c][0], pos, 1.0);
            } else {
                const int i = pos % n, j = pos / n;
                const int a = B.col_ix[c] & 1, b = B.col_iy[c] & 1;
                lagrange_weights(A.basis, 0.5 * (A.basis.x[i] + (2 * a - 1)), lx.data());
                lagrange_weights(A.basis, 0.5 * (A.basis.x[j] + (2 * b - 1)), ly.data());
                for (int q = 0; q < n; ++q)
                    for (int m = 0; m < n; ++m)
                        if (lx[m] != 0.0 && ly[q] != 0.0) old_local(acc, src[c][0], m + n * q, lx[m] * ly[q]);
            }
            acc.finish(1.0, T);
            continue;
        }
        // merged parents only: mass-weighted average of their projections
        double wsum = 0.0;
        for (int r = hp[h]; r < hp[h + 1]; ++r) {
            const int c = hcp[r] / n2, pos = hcp[r] % n2;
            const int i = pos % n, j = pos / n;
            const double wm = A.basis.w[i] * A.basis.w[j] * B.col_dx[c] * B.col_dy[c];
            wsum += wm;
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a)
                    for (int q = 0; q < n; ++q)
                        for (int m = 0; m < n; ++m) {
                            const double wt = P[a][i * n + m] * P[b][j * n + q];
                            if (wt != 0.0) old_local(acc, src[c][a + 2 * b], m + n * q, wm * wt);
                        }
        }
        acc.finish(1.0 / wsum, T);
    }
    return SEM_OK;
}

}  // namespace sem
