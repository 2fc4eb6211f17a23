// Device helpers shared by the HIP translation units: the value of one field
// at an element-local horizontal slot (through the hanging rows when the slot
// is a hanging point) and the column rule of the refinement flags.
#pragma once

#include <hip/hip_runtime.h>

#include "devmesh.h"

namespace sem {

// value of field f at horizontal slot g (unique node or hanging point) and kz,
// interpolating hanging points through their rows
__device__ __forceinline__ double node_value(const DevMesh& m, const double* __restrict__ q,
                                             int g, int f, int kz) {
    const int64_t fs = int64_t(m.n_h) * m.ldz;
    if (g >= 0) return q[f * fs + int64_t(g) * m.ldz + kz];
    const int hh = -g - 1;
    double s = 0.0;
    for (int t = m.hang_ptr[hh]; t < m.hang_ptr[hh + 1]; ++t)
        s += m.hang_w[t] * q[f * fs + int64_t(m.hang_src[t]) * m.ldz + kz];
    return s;
}

// Column rule of the refinement flags (Section 4.1 refines and coarsens whole
// columns): +1 if any element of column c is +1; -1 if every element of the
// column and of its three siblings is -1; else 0.
__device__ __forceinline__ int8_t column_rule(const DevMesh& m, const int8_t* __restrict__ ae, int c) {
    auto col_state = [&](int cc, bool& any_ref, bool& all_crs) {
        any_ref = false;
        all_crs = true;
        for (int z = 0; z < m.n_z; ++z) {
            const int8_t a = ae[cc * m.n_z + z];
            any_ref = any_ref || (a == 1);
            all_crs = all_crs && (a == -1);
        }
    };
    bool r, cr;
    col_state(c, r, cr);
    if (r) return 1;
    if (cr && m.sib[4 * c] >= 0) {
        bool ok = true;
        for (int s = 0; s < 4; ++s) {
            bool r2, c2;
            col_state(m.sib[4 * c + s], r2, c2);
            ok = ok && c2 && !r2;
        }
        if (ok) return -1;
    }
    return 0;
}

}  // namespace sem
