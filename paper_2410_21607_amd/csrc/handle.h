// Internal definitions shared by the HIP translation units of the library:
// the mesh handle, the error channel behind sem_last_error, and HIPCHK.
#pragma once

#include <hip/hip_runtime.h>

#include <exception>
#include <string>
#include <vector>

#include "devmesh.h"
#include "mesh_build.h"
#include "sem.h"
#include "stage_fused.h"

namespace sem {

// thread-local message of the last failed call on this thread
std::string& last_error();

inline int fail(int code, const std::string& msg) {
    last_error() = msg;
    return code;
}

// Entry points with host-side work run through this: a C++ exception (host
// memory or threads exhausted) becomes SEM_ERR_HOST with its message instead
// of crossing the C boundary.
template <typename F>
int guarded(const char* name, F&& f) {
    try {
        return f();
    } catch (const std::exception& e) {
        return fail(SEM_ERR_HOST, std::string(name) + ": " + e.what());
    } catch (...) {
        return fail(SEM_ERR_HOST, std::string(name) + ": host-side failure");
    }
}

}  // namespace sem

#define HIPCHK(x)                                                                        \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess)                                                            \
            return sem::fail(SEM_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct sem_mesh {
    sem::HostMesh host;
    sem::DevMesh d{};
    std::vector<void*> allocs;
    bool have_ref = false;
    sem::FusedPlan fused;
    double* feat_aux = nullptr;   // 2 doubles per element (amr_features)
    // dissipation pre-pass of the fused stage (allocated when enabled)
    double *diss_rE = nullptr, *diss_acc = nullptr, *diss_c = nullptr, *diss_r = nullptr;
    double* diss_sponge = nullptr;
    double* wind_part = nullptr;  // 256 partial maxima (sem_max_wind)
    double* terrain_buf = nullptr; // zs, normals, per-node reference, tfac (sem_mesh_set_terrain)
    int64_t terrain_bytes = 0;
    const double* d_hxy = nullptr; // x, y of every unique horizontal node
    std::vector<double> zs_host;   // terrain heights per unique horizontal node (empty = flat)
    int64_t ws_bytes = 0;
    // bumped by every call that changes what a captured kernel node reads
    // (tables freed or moved, settings passed by value)
    int64_t epoch = 0;
    ~sem_mesh() {
        sem::fused_plan_free(fused);
        if (feat_aux) (void)hipFree(feat_aux);
        for (double* p : {diss_rE, diss_acc, diss_c, diss_r, diss_sponge})
            if (p) (void)hipFree(p);
        if (wind_part) (void)hipFree(wind_part);
        if (terrain_buf) (void)hipFree(terrain_buf);
        for (void* p : allocs) (void)hipFree(p);
    }
    template <typename T>
    int upload(const std::vector<T>& v, const T** dst) {
        if (v.empty()) { *dst = nullptr; return SEM_OK; }
        void* p = nullptr;
        HIPCHK(hipMalloc(&p, v.size() * sizeof(T)));
        allocs.push_back(p);
        HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        ws_bytes += int64_t(v.size() * sizeof(T));
        *dst = static_cast<const T*>(p);
        return SEM_OK;
    }
};

struct sem_transfer {
    int64_t n_from = 0, n_to = 0;   // horizontal nodes of the two meshes
    int nzn = 0, ldz = 0;
    int64_t nnz = 0;
    int32_t* ptr = nullptr;
    int32_t* src = nullptr;
    double* w = nullptr;
    ~sem_transfer() {
        if (ptr) (void)hipFree(ptr);
        if (src) (void)hipFree(src);
        if (w) (void)hipFree(w);
    }
};

