// Multilayer perceptron of the refinement forecaster (gfx950, FP32):
// 16 -> 64 -> 64 -> 3 with tanh, softmax cross-entropy, Adam.
//
// Parameters are one flat float array: W1[64][16], b1[64], W2[64][64], b2[64],
// W3[3][64], b3[3] (5443 floats, staged in LDS by every workgroup).
//
// Training step = three launches:
//   k_mlp_samples : one thread per sample: forward pass, softmax, the
//                   per-sample back-propagated errors of the three layers and
//                   the sample's loss, written to the workspace;
//   k_mlp_grad    : the batch sum of every parameter's gradient, 16
//                   interleaved batch segments per parameter combined in a
//                   fixed order (deterministic, accumulated in double);
//   k_adam        : element-wise Adam update.
#include <cmath>
#include <mutex>

#include "handle.h"

namespace sem {

namespace {

constexpr int NI = SEM_MLP_IN, NH = SEM_MLP_HIDDEN, NO = SEM_MLP_OUT;
constexpr int OW1 = 0, OB1 = OW1 + NH * NI, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NO * NH, NP = OB3 + NO;
static_assert(NP == SEM_MLP_NPARAM, "parameter count");
// workspace per sample: h1, h2, d1, d2 (64 each), d3 (3), loss (1)
constexpr int WH1 = 0, WH2 = WH1 + NH, WD1 = WH2 + NH, WD2 = WD1 + NH, WD3 = WD2 + NH,
              WL = WD3 + NO, WN = WL + 1;
static_assert(WN == SEM_MLP_WORK, "workspace per sample");

__device__ __forceinline__ void stage_params(const float* __restrict__ p, float* sp) {
    for (int r = threadIdx.x; r < NP; r += blockDim.x) sp[r] = p[r];
    __syncthreads();
}

// hidden layers and logits of one sample
__device__ __forceinline__ void forward_one(const float* sp, const float* __restrict__ xin,
                                            float* h1, float* h2, float* z3) {
    float x[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) x[i] = xin[i];
#pragma unroll
    for (int o = 0; o < NH; ++o) {
        float s = sp[OB1 + o];
#pragma unroll
        for (int i = 0; i < NI; ++i) s = fmaf(sp[OW1 + o * NI + i], x[i], s);
        h1[o] = tanhf(s);
    }
#pragma unroll
    for (int o = 0; o < NH; ++o) {
        float s = sp[OB2 + o];
#pragma unroll
        for (int h = 0; h < NH; ++h) s = fmaf(sp[OW2 + o * NH + h], h1[h], s);
        h2[o] = tanhf(s);
    }
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        float s = sp[OB3 + o];
#pragma unroll
        for (int h = 0; h < NH; ++h) s = fmaf(sp[OW3 + o * NH + h], h2[h], s);
        z3[o] = s;
    }
}

}  // namespace

__global__ void __launch_bounds__(256)
k_mlp_forward(const float* __restrict__ p, const float* __restrict__ x, int64_t n,
              float* __restrict__ logits) {
    __shared__ float sp[NP];
    stage_params(p, sp);
    for (int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; b < n;
         b += int64_t(gridDim.x) * blockDim.x) {
        float h1[NH], h2[NH], z3[NO];
        forward_one(sp, x + b * NI, h1, h2, z3);
#pragma unroll
        for (int o = 0; o < NO; ++o) logits[b * NO + o] = z3[o];
    }
}

__global__ void __launch_bounds__(256)
k_mlp_samples(const float* __restrict__ p, const float* __restrict__ x,
              const int8_t* __restrict__ cls, const int32_t* __restrict__ idx, int64_t n,
              int64_t n_rows, float* __restrict__ work) {
    __shared__ float sp[NP];
    stage_params(p, sp);
    const float inv_n = 1.0f / float(n);
    for (int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; b < n;
         b += int64_t(gridDim.x) * blockDim.x) {
        const int64_t s = idx ? min(max(int64_t(idx[b]), int64_t(0)), n_rows - 1) : b;
        float h1[NH], h2[NH], z3[NO];
        forward_one(sp, x + s * NI, h1, h2, z3);
        const int lab = min(max(int(cls[s]), 0), NO - 1);
        // softmax and cross-entropy
        float zm = fmaxf(z3[0], fmaxf(z3[1], z3[2]));
        float ex[NO], se = 0.0f;
#pragma unroll
        for (int o = 0; o < NO; ++o) { ex[o] = expf(z3[o] - zm); se += ex[o]; }
        float* wb = work + b * WN;
        float d3[NO];
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            d3[o] = (ex[o] / se - (o == lab ? 1.0f : 0.0f)) * inv_n;
            wb[WD3 + o] = d3[o];
        }
        wb[WL] = -(z3[lab] - zm - logf(se));
        // layer 2 error: (W3^T d3) * (1 - h2^2)
        float d2[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            float s2 = 0.0f;
#pragma unroll
            for (int o = 0; o < NO; ++o) s2 = fmaf(sp[OW3 + o * NH + h], d3[o], s2);
            d2[h] = s2 * (1.0f - h2[h] * h2[h]);
            wb[WH2 + h] = h2[h];
            wb[WD2 + h] = d2[h];
        }
        // layer 1 error: (W2^T d2) * (1 - h1^2)
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            float s1 = 0.0f;
#pragma unroll
            for (int o = 0; o < NH; ++o) s1 = fmaf(sp[OW2 + o * NH + h], d2[o], s1);
            wb[WH1 + h] = h1[h];
            wb[WD1 + h] = s1 * (1.0f - h1[h] * h1[h]);
        }
    }
}

// gradient of every parameter (and, in the last slot, the mean loss) as a
// batch sum: a workgroup owns 64 consecutive slots and splits the batch into
// 16 interleaved segments (b = seg, seg + 16, ...), each summed in sample
// order in double; the 16 partial sums are then added in segment order, so
// the result does not depend on scheduling.
constexpr int GRAD_SLOTS = 64, GRAD_SEGS = 16;

__global__ void __launch_bounds__(GRAD_SLOTS * GRAD_SEGS)
k_mlp_grad(const float* __restrict__ x, const int32_t* __restrict__ idx, int64_t n,
           int64_t n_rows, const float* __restrict__ work, float* __restrict__ grad,
           float* __restrict__ loss) {
    __shared__ double part[GRAD_SEGS][GRAD_SLOTS];
    const int q = threadIdx.x % GRAD_SLOTS, seg = threadIdx.x / GRAD_SLOTS;
    const int r = blockIdx.x * GRAD_SLOTS + q;
    double s = 0.0;
    if (r == NP) {                       // mean loss
        for (int64_t b = seg; b < n; b += GRAD_SEGS) s += work[b * WN + WL];
    } else if (r < OB1) {                // W1[o][i] = sum d1[o] x[i]
        const int o = r / NI, i = r % NI;
        for (int64_t b = seg; b < n; b += GRAD_SEGS) {
            const int64_t sm = idx ? min(max(int64_t(idx[b]), int64_t(0)), n_rows - 1) : b;
            s += double(work[b * WN + WD1 + o]) * double(x[sm * NI + i]);
        }
    } else if (r < OW2) {                // b1[o] = sum d1[o]
        const int o = r - OB1;
        for (int64_t b = seg; b < n; b += GRAD_SEGS) s += work[b * WN + WD1 + o];
    } else if (r < OB2) {                // W2[o][h] = sum d2[o] h1[h]
        const int o = (r - OW2) / NH, h = (r - OW2) % NH;
        for (int64_t b = seg; b < n; b += GRAD_SEGS)
            s += double(work[b * WN + WD2 + o]) * double(work[b * WN + WH1 + h]);
    } else if (r < OW3) {                // b2[o] = sum d2[o]
        const int o = r - OB2;
        for (int64_t b = seg; b < n; b += GRAD_SEGS) s += work[b * WN + WD2 + o];
    } else if (r < OB3) {                // W3[o][h] = sum d3[o] h2[h]
        const int o = (r - OW3) / NH, h = (r - OW3) % NH;
        for (int64_t b = seg; b < n; b += GRAD_SEGS)
            s += double(work[b * WN + WD3 + o]) * double(work[b * WN + WH2 + h]);
    } else if (r < NP) {                 // b3[o] = sum d3[o]
        const int o = r - OB3;
        for (int64_t b = seg; b < n; b += GRAD_SEGS) s += work[b * WN + WD3 + o];
    }
    part[seg][q] = s;
    __syncthreads();
    if (seg == 0 && r <= NP) {
        double t = 0.0;
        for (int k = 0; k < GRAD_SEGS; ++k) t += part[k][q];
        if (r == NP) *loss = float(t / double(n));
        else grad[r] = float(t);
    }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= NP) return;
    const float gr = g[r];
    const float mr = b1 * m[r] + (1.0f - b1) * gr;
    const float vr = b2 * v[r] + (1.0f - b2) * gr * gr;
    m[r] = mr;
    v[r] = vr;
    p[r] -= lr * (mr / c1) / (sqrtf(vr / c2) + eps);
}

// Workspace of mlp_backward_noalloc: one array per GPU, held until the
// process ends, shared by every call on that GPU (see sem.h).
static __device__ __align__(256) float scratch[size_t(SEM_MLP_NOALLOC_MAX) * SEM_MLP_WORK];

}  // namespace sem

namespace {
using sem::fail;

// device address of `scratch` on each GPU, looked up once per device with
// that device current (the host-side name is not a device address)
constexpr int kMaxDevices = 64;
float* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

int scratch_for_current_device(float** out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SEM_ERR_HIP, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(sem::scratch)));
        if (!p) return fail(SEM_ERR_HIP, "no device address for the workspace array");
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return SEM_OK;
}

int grid_of(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return int(g);
}
}  // namespace

extern "C" {

static int mlp_forward_impl(const float* p, const float* x, int64_t n, float* logits, void* stream) {
    if (!p || !logits || (n > 0 && !x)) return fail(SEM_ERR_ARG, "null array");
    if (n < 0) return fail(SEM_ERR_ARG, "negative sample count");
    if (n == 0) return SEM_OK;
    hipLaunchKernelGGL(sem::k_mlp_forward, dim3(grid_of(n)), dim3(256), 0, (hipStream_t)stream,
                       p, x, n, logits);
    HIPCHK(hipGetLastError());
    return SEM_OK;
}

int mlp_forward(const float* p, const float* x, int64_t n, float* logits, void* stream) {
    return sem::guarded("mlp_forward", [&] { return mlp_forward_impl(p, x, n, logits, stream); });
}

static int mlp_backward_impl(const float* p, const float* x, int64_t n_rows, const int8_t* cls,
                 const int32_t* idx, int64_t n, float* work, float* grad, float* loss, void* stream) {
    if (!p || !x || !cls || !work || !grad || !loss) return fail(SEM_ERR_ARG, "null array");
    if (n < 1) return fail(SEM_ERR_ARG, "empty batch");
    if (n_rows < 1 || (!idx && n > n_rows)) return fail(SEM_ERR_ARG, "batch larger than the data");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(sem::k_mlp_samples, dim3(grid_of(n)), dim3(256), 0, s, p, x, cls, idx, n,
                       n_rows, work);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(sem::k_mlp_grad, dim3((SEM_MLP_NPARAM + 1 + sem::GRAD_SLOTS - 1) / sem::GRAD_SLOTS),
                       dim3(sem::GRAD_SLOTS * sem::GRAD_SEGS), 0, s, x, idx, n, n_rows, work, grad, loss);
    HIPCHK(hipGetLastError());
    return SEM_OK;
}

int mlp_backward(const float* p, const float* x, int64_t n_rows, const int8_t* cls,
                 const int32_t* idx, int64_t n, float* work, float* grad, float* loss, void* stream) {
    return sem::guarded("mlp_backward", [&] { return mlp_backward_impl(p, x, n_rows, cls, idx, n, work, grad, loss, stream); });
}

static int mlp_backward_noalloc_impl(const float* p, const float* x, int64_t n_rows, const int8_t* cls,
                         const int32_t* idx, int64_t n, float* grad, float* loss, void* stream) {
    if (!p || !x || !cls || !grad || !loss) return fail(SEM_ERR_ARG, "null array");
    if (n < 1) return fail(SEM_ERR_ARG, "empty batch");
    if (n > SEM_MLP_NOALLOC_MAX)
        return fail(SEM_ERR_ARG, "batch larger than SEM_MLP_NOALLOC_MAX samples (use mlp_backward "
                                 "with a caller workspace)");
    if (n_rows < 1 || (!idx && n > n_rows)) return fail(SEM_ERR_ARG, "batch larger than the data");
    float* work = nullptr;
    int rc = scratch_for_current_device(&work);
    if (rc != SEM_OK) return rc;
    // the same two kernels as mlp_backward; k_mlp_samples writes every
    // workspace entry that k_mlp_grad reads (the first n samples), so nothing
    // left by an earlier call is read and no clearing is needed
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(sem::k_mlp_samples, dim3(grid_of(n)), dim3(256), 0, s, p, x, cls, idx, n,
                       n_rows, work);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(sem::k_mlp_grad, dim3((SEM_MLP_NPARAM + 1 + sem::GRAD_SLOTS - 1) / sem::GRAD_SLOTS),
                       dim3(sem::GRAD_SLOTS * sem::GRAD_SEGS), 0, s, x, idx, n, n_rows, work, grad, loss);
    HIPCHK(hipGetLastError());
    return SEM_OK;
}

int mlp_backward_noalloc(const float* p, const float* x, int64_t n_rows, const int8_t* cls,
                         const int32_t* idx, int64_t n, float* grad, float* loss, void* stream) {
    return sem::guarded("mlp_backward_noalloc", [&] { return mlp_backward_noalloc_impl(p, x, n_rows, cls, idx, n, grad, loss, stream); });
}

static int mlp_adam_step_impl(float* p, const float* g, float* m, float* v, int t, float lr, float beta1,
                  float beta2, float eps, void* stream) {
    if (!p || !g || !m || !v) return fail(SEM_ERR_ARG, "null array");
    if (t < 1) return fail(SEM_ERR_ARG, "Adam step count starts at 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f))
        return fail(SEM_ERR_ARG, "bad Adam hyper-parameters");
    const float c1 = float(1.0 - std::pow(double(beta1), t));
    const float c2 = float(1.0 - std::pow(double(beta2), t));
    hipLaunchKernelGGL(sem::k_adam, dim3((SEM_MLP_NPARAM + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, p, g, m, v, lr, beta1, beta2, eps, c1, c2);
    HIPCHK(hipGetLastError());
    return SEM_OK;
}

int mlp_adam_step(float* p, const float* g, float* m, float* v, int t, float lr, float beta1,
                  float beta2, float eps, void* stream) {
    return sem::guarded("mlp_adam_step", [&] { return mlp_adam_step_impl(p, g, m, v, t, lr, beta1, beta2, eps, stream); });
}

}  // extern "C"
