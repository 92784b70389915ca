// bc_mlp.hip -- the level-policy network: 5 features -> 32 -> 32 -> 3,
// ReLU hidden layers, FP32.  Training kernels (forward, backward, Adam) and
// batch prediction.  The same weights drive the per-level choice inside the
// step kernels (choose_variant in bc_common.h).
//
// Loss over n samples (x_i, y_i, mask_i), y_ij = log2 of the measured time of
// variant j at that level, mask_ij = 1 when it was measured:
//     L = sum_ij mask_ij (f(x_i)_j - y_ij)^2 / (2 * sum_ij mask_ij).
// Gradients are reduced over samples in sample order by one thread per
// parameter, so they do not depend on the launch shape.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bc.h"
#include "bc_dev.h"

namespace bcx {

constexpr int kIn = kMlpIn, kH = kMlpH, kOut = kMlpOut;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kOut * kH, kP = oB3 + kOut;
static_assert(kP == kMlpParams, "parameter layout");

// Per-sample forward and backward: one thread per sample.  Writes the hidden
// activations and the back-propagated errors that the parameter gradients
// need, plus the sample's squared error (pre-scaled).
__global__ __launch_bounds__(256) void mlp_rows(const float *__restrict__ w, const float *__restrict__ X,
                                                const float *__restrict__ Y, const uint8_t *__restrict__ mask,
                                                int64_t n, const float *__restrict__ inv_p, float *__restrict__ H1,
                                                float *__restrict__ H2, float *__restrict__ D1,
                                                float *__restrict__ D2, float *__restrict__ D3,
                                                float *__restrict__ sq) {
    __shared__ float sw[kP];
    for (int i = threadIdx.x; i < kP; i += blockDim.x) sw[i] = w[i];
    __syncthreads();
    const float inv_cnt = *inv_p;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        float x[kIn], h1[kH], h2[kH], y[kOut], d3[kOut], d2[kH];
        for (int i = 0; i < kIn; ++i) x[i] = X[r * kIn + i];
        for (int j = 0; j < kH; ++j) {
            float s = sw[oB1 + j];
            for (int i = 0; i < kIn; ++i) s += sw[oW1 + j * kIn + i] * x[i];
            h1[j] = fmaxf(s, 0.0f);
        }
        for (int j = 0; j < kH; ++j) {
            float s = sw[oB2 + j];
            for (int i = 0; i < kH; ++i) s += sw[oW2 + j * kH + i] * h1[i];
            h2[j] = fmaxf(s, 0.0f);
        }
        float e = 0.0f;
        for (int k = 0; k < kOut; ++k) {
            float s = sw[oB3 + k];
            for (int i = 0; i < kH; ++i) s += sw[oW3 + k * kH + i] * h2[i];
            y[k] = s;
            const float m = mask[r * kOut + k] ? 1.0f : 0.0f;
            const float diff = (s - Y[r * kOut + k]) * m;
            d3[k] = diff * inv_cnt;
            e += diff * diff;
        }
        for (int i = 0; i < kH; ++i) {
            float s = 0.0f;
            for (int k = 0; k < kOut; ++k) s += sw[oW3 + k * kH + i] * d3[k];
            d2[i] = h2[i] > 0.0f ? s : 0.0f;
        }
        for (int i = 0; i < kH; ++i) {
            float s = 0.0f;
            for (int j = 0; j < kH; ++j) s += sw[oW2 + j * kH + i] * d2[j];
            D1[r * kH + i] = h1[i] > 0.0f ? s : 0.0f;
            H1[r * kH + i] = h1[i];
            H2[r * kH + i] = h2[i];
            D2[r * kH + i] = d2[i];
        }
        for (int k = 0; k < kOut; ++k) D3[r * kOut + k] = d3[k];
        sq[r] = 0.5f * e * inv_cnt;
    }
}

// 1 / (number of measured targets), or 0 when there are none (the loss and
// gradient are then 0).  One workgroup; integer count, so the order of the
// additions does not matter.
__global__ __launch_bounds__(256) void mlp_mask_count(const uint8_t *__restrict__ mask, int64_t n,
                                                      float *__restrict__ inv) {
    __shared__ unsigned long long part[256];
    unsigned long long c = 0;
    for (int64_t i = threadIdx.x; i < n * kOut; i += blockDim.x) c += mask[i] ? 1u : 0u;
    part[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *inv = part[0] ? 1.0f / (float)part[0] : 0.0f;
}

// One thread per parameter: gradient = sum over samples, in sample order.
// Thread kP also sums the loss.
__global__ __launch_bounds__(256) void mlp_grad(const float *__restrict__ X, const float *__restrict__ H1,
                                                const float *__restrict__ H2, const float *__restrict__ D1,
                                                const float *__restrict__ D2, const float *__restrict__ D3,
                                                const float *__restrict__ sq, int64_t n, float *__restrict__ grad,
                                                float *__restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kP) return;
    float g = 0.0f;
    if (p == kP) {
        for (int64_t r = 0; r < n; ++r) g += sq[r];
        *loss = g;
        return;
    }
    if (p < oB1) {
        const int j = p / kIn, i = p % kIn;
        for (int64_t r = 0; r < n; ++r) g += D1[r * kH + j] * X[r * kIn + i];
    } else if (p < oW2) {
        const int j = p - oB1;
        for (int64_t r = 0; r < n; ++r) g += D1[r * kH + j];
    } else if (p < oB2) {
        const int q = p - oW2, j = q / kH, i = q % kH;
        for (int64_t r = 0; r < n; ++r) g += D2[r * kH + j] * H1[r * kH + i];
    } else if (p < oW3) {
        const int j = p - oB2;
        for (int64_t r = 0; r < n; ++r) g += D2[r * kH + j];
    } else if (p < oB3) {
        const int q = p - oW3, k = q / kH, i = q % kH;
        for (int64_t r = 0; r < n; ++r) g += D3[r * kOut + k] * H2[r * kH + i];
    } else {
        const int k = p - oB3;
        for (int64_t r = 0; r < n; ++r) g += D3[r * kOut + k];
    }
    grad[p] = g;
}

// Adam (Kingma & Ba), step t >= 1.
__global__ void mlp_adam(float *__restrict__ w, const float *__restrict__ grad, float *__restrict__ m1,
                         float *__restrict__ m2, int t, float lr, float b1, float b2, float eps) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kP) return;
    const float g = grad[p];
    const float a = b1 * m1[p] + (1.0f - b1) * g;
    const float b = b2 * m2[p] + (1.0f - b2) * g * g;
    m1[p] = a;
    m2[p] = b;
    const float ah = a / (1.0f - powf(b1, (float)t));
    const float bh = b / (1.0f - powf(b2, (float)t));
    w[p] -= lr * ah / (sqrtf(bh) + eps);
}

__global__ void mlp_predict(const float *__restrict__ w, const float *__restrict__ X, int64_t n,
                            float *__restrict__ Y) {
    __shared__ float sw[kP];
    for (int i = threadIdx.x; i < kP; i += blockDim.x) sw[i] = w[i];
    __syncthreads();
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        float x[kIn], h1[kH], h2[kH];
        for (int i = 0; i < kIn; ++i) x[i] = X[r * kIn + i];
        for (int j = 0; j < kH; ++j) {
            float s = sw[oB1 + j];
            for (int i = 0; i < kIn; ++i) s += sw[oW1 + j * kIn + i] * x[i];
            h1[j] = fmaxf(s, 0.0f);
        }
        for (int j = 0; j < kH; ++j) {
            float s = sw[oB2 + j];
            for (int i = 0; i < kH; ++i) s += sw[oW2 + j * kH + i] * h1[i];
            h2[j] = fmaxf(s, 0.0f);
        }
        for (int k = 0; k < kOut; ++k) {
            float s = sw[oB3 + k];
            for (int i = 0; i < kH; ++i) s += sw[oW3 + k * kH + i] * h2[i];
            Y[r * kOut + k] = s;
        }
    }
}

}  // namespace bcx

using namespace bcx;

namespace {

// Device buffers for one training / gradient call.
struct MlpBufs {
    float *w = nullptr, *X = nullptr, *Y = nullptr, *H1 = nullptr, *H2 = nullptr, *D1 = nullptr, *D2 = nullptr,
          *D3 = nullptr, *sq = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr, *loss = nullptr,
          *inv = nullptr;
    uint8_t *mask = nullptr;
    bool owned = true;  // false: views into the static scratch (nothing to free)
    ~MlpBufs() {
        if (!owned) return;
        void *ps[] = {w, X, Y, H1, H2, D1, D2, D3, sq, grad, m1, m2, loss, inv, mask};
        for (void *p : ps)
            if (p) (void)hipFree(p);
    }
};

}  // namespace

// Records the thread-local error text (bc_api.hip) and returns s.
bc_status bc_set_error(bc_status s, const char *msg);

#define MLP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess)                                                         \
            return bc_set_error(_e == hipErrorOutOfMemory ? BC_ERR_OUT_OF_MEMORY : BC_ERR_DEVICE, \
                                (std::string(#expr) + ": " + hipGetErrorString(_e)).c_str()); \
    } while (0)

static bc_status mlp_upload(MlpBufs &b, const float *weights, const float *X, const float *Y, const uint8_t *mask,
                            int64_t n, hipStream_t st) {
    const size_t N = (size_t)(n > 0 ? n : 1);
    MLP_TRY(hipMalloc((void **)&b.w, kP * sizeof(float)));
    MLP_TRY(hipMalloc((void **)&b.X, N * kIn * sizeof(float)));
    MLP_TRY(hipMalloc((void **)&b.Y, N * kOut * sizeof(float)));
    MLP_TRY(hipMalloc((void **)&b.mask, N * kOut));
    MLP_TRY(hipMalloc((void **)&b.H1, N * kH * sizeof(float)));
    MLP_TRY(hipMalloc((void **)&b.H2, N * kH * sizeof(float)));
    MLP_TRY(hipMalloc((void **)&b.D1, N * kH * sizeof(float)));
    MLP_TRY(hipMalloc((void **)&b.D2, N * kH * sizeof(float)));
    MLP_TRY(hipMalloc((void **)&b.D3, N * kOut * sizeof(float)));
    MLP_TRY(hipMalloc((void **)&b.sq, N * sizeof(float)));
    MLP_TRY(hipMalloc((void **)&b.grad, kP * sizeof(float)));
    MLP_TRY(hipMalloc((void **)&b.m1, kP * sizeof(float)));
    MLP_TRY(hipMalloc((void **)&b.m2, kP * sizeof(float)));
    MLP_TRY(hipMalloc((void **)&b.loss, sizeof(float)));
    MLP_TRY(hipMalloc((void **)&b.inv, sizeof(float)));
    MLP_TRY(hipMemcpyAsync(b.w, weights, kP * sizeof(float), hipMemcpyHostToDevice, st));
    if (n > 0) {
        MLP_TRY(hipMemcpyAsync(b.X, X, (size_t)n * kIn * sizeof(float), hipMemcpyHostToDevice, st));
        MLP_TRY(hipMemcpyAsync(b.Y, Y, (size_t)n * kOut * sizeof(float), hipMemcpyHostToDevice, st));
        MLP_TRY(hipMemcpyAsync(b.mask, mask, (size_t)n * kOut, hipMemcpyHostToDevice, st));
    }
    return BC_OK;
}

static bc_status mlp_check(const float *weights, const float *X, const float *Y, const uint8_t *mask, int64_t n) {
    if (!weights || n < 1 || !X || !Y || !mask) return bc_set_error(BC_ERR_INVALID_ARG, "NULL argument or n < 1");
    int64_t cnt = 0;
    for (int64_t i = 0; i < n * kOut; ++i) cnt += mask[i] ? 1 : 0;
    if (cnt == 0) return bc_set_error(BC_ERR_INVALID_ARG, "no measured targets (mask is all zero)");
    for (int64_t i = 0; i < n * kIn; ++i)
        if (!std::isfinite(X[i])) return bc_set_error(BC_ERR_INVALID_ARG, "non-finite feature");
    for (int64_t i = 0; i < n * kOut; ++i)
        if (mask[i] && !std::isfinite(Y[i])) return bc_set_error(BC_ERR_INVALID_ARG, "non-finite target");
    return BC_OK;
}

static void mlp_count(MlpBufs &b, int64_t n, hipStream_t st) {
    mlp_mask_count<<<1, 256, 0, st>>>(b.mask, n, b.inv);
}

static void mlp_step_grad(MlpBufs &b, int64_t n, hipStream_t st) {
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    mlp_rows<<<blocks, 256, 0, st>>>(b.w, b.X, b.Y, b.mask, n, b.inv, b.H1, b.H2, b.D1, b.D2, b.D3, b.sq);
    mlp_grad<<<(kP + 1 + 255) / 256, 256, 0, st>>>(b.X, b.H1, b.H2, b.D1, b.D2, b.D3, b.sq, n, b.grad, b.loss);
}

extern "C" bc_status bc_mlp_loss_grad(const float *weights, const float *X, const float *Y, const uint8_t *mask,
                                      int64_t n, float *loss, float *grad, void *stream) {
    bc_status s = mlp_check(weights, X, Y, mask, n);
    if (s != BC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    MlpBufs b;
    s = mlp_upload(b, weights, X, Y, mask, n, st);
    if (s != BC_OK) return s;
    mlp_count(b, n, st);
    mlp_step_grad(b, n, st);
    MLP_TRY(hipGetLastError());
    float l = 0.0f;
    std::vector<float> g(kP);
    MLP_TRY(hipMemcpyAsync(&l, b.loss, sizeof(float), hipMemcpyDeviceToHost, st));
    MLP_TRY(hipMemcpyAsync(g.data(), b.grad, kP * sizeof(float), hipMemcpyDeviceToHost, st));
    MLP_TRY(hipStreamSynchronize(st));
    if (loss) *loss = l;
    if (grad) std::memcpy(grad, g.data(), kP * sizeof(float));
    return BC_OK;
}

// ------------------------------------------------ allocation-free variant
// bc_mlp_loss_grad_noalloc keeps every intermediate of the loss and gradient
// (hidden activations, back-propagated errors, per-sample squared errors and
// the target count) in this fixed array: no device memory is allocated per
// call.  Each GPU holds its own copy for the life of the process.  Host code
// must not pass the array's name to a kernel (on the host it only stands for
// the symbol): the device address comes from hipGetSymbolAddress, taken once
// per device on the first call there.
constexpr int64_t kNoAllocMaxSamples = 16384;
constexpr size_t kNoAllocFloats = (size_t)kNoAllocMaxSamples * (4 * kH + kOut + 1) + 64;
static __device__ __align__(256) float scratch[kNoAllocFloats];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static bc_status scratch_address(float **out) {
    int dev = -1;
    MLP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return bc_set_error(BC_ERR_NOT_SUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        MLP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return bc_set_error(BC_ERR_DEVICE, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = (float *)p;
    }
    *out = g_scratch_ptr[dev];
    return BC_OK;
}

extern "C" bc_status bc_mlp_loss_grad_noalloc(const float *weights, const float *X, const float *Y,
                                              const uint8_t *mask, int64_t n, float *loss, float *grad,
                                              void *stream) {
    if (!weights || !X || !Y || !mask || !loss || !grad) return bc_set_error(BC_ERR_INVALID_ARG, "NULL argument");
    if (n < 1 || n > kNoAllocMaxSamples)
        return bc_set_error(BC_ERR_INVALID_ARG, ("n must be in [1, " + std::to_string(kNoAllocMaxSamples) +
                                                 "] for the allocation-free call").c_str());
    float *sc = nullptr;
    bc_status s = scratch_address(&sc);
    if (s != BC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    MlpBufs b;
    b.owned = false;
    b.w = const_cast<float *>(weights);
    b.X = const_cast<float *>(X);
    b.Y = const_cast<float *>(Y);
    b.mask = const_cast<uint8_t *>(mask);
    b.grad = grad;
    b.loss = loss;
    // scratch layout: H1, H2, D1, D2 [n][kH] each, D3 [n][kOut], sq [n], inv [1]
    const size_t N = (size_t)n;
    b.H1 = sc;
    b.H2 = b.H1 + N * kH;
    b.D1 = b.H2 + N * kH;
    b.D2 = b.D1 + N * kH;
    b.D3 = b.D2 + N * kH;
    b.sq = b.D3 + N * kOut;
    b.inv = b.sq + N;
    mlp_count(b, n, st);
    mlp_step_grad(b, n, st);
    MLP_TRY(hipGetLastError());
    return BC_OK;
}

extern "C" bc_status bc_mlp_train(float *weights, const float *X, const float *Y, const uint8_t *mask, int64_t n,
                                  int32_t steps, float lr, float *final_loss, void *stream) {
    bc_status s = mlp_check(weights, X, Y, mask, n);
    if (s != BC_OK) return s;
    if (steps < 0 || !(lr > 0.0f) || !std::isfinite(lr)) return bc_set_error(BC_ERR_INVALID_ARG, "bad steps or lr");
    for (int i = 0; i < kP; ++i)
        if (!std::isfinite(weights[i])) return bc_set_error(BC_ERR_INVALID_ARG, "non-finite initial weight");
    hipStream_t st = (hipStream_t)stream;
    MlpBufs b;
    s = mlp_upload(b, weights, X, Y, mask, n, st);
    if (s != BC_OK) return s;
    MLP_TRY(hipMemsetAsync(b.m1, 0, kP * sizeof(float), st));
    MLP_TRY(hipMemsetAsync(b.m2, 0, kP * sizeof(float), st));
    mlp_count(b, n, st);
    for (int t = 1; t <= steps; ++t) {
        mlp_step_grad(b, n, st);
        mlp_adam<<<(kP + 255) / 256, 256, 0, st>>>(b.w, b.grad, b.m1, b.m2, t, lr, 0.9f, 0.999f, 1e-8f);
    }
    mlp_step_grad(b, n, st);  // loss of the final weights
    MLP_TRY(hipGetLastError());
    std::vector<float> w(kP);
    float l = 0.0f;
    MLP_TRY(hipMemcpyAsync(w.data(), b.w, kP * sizeof(float), hipMemcpyDeviceToHost, st));
    MLP_TRY(hipMemcpyAsync(&l, b.loss, sizeof(float), hipMemcpyDeviceToHost, st));
    MLP_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < kP; ++i)
        if (!std::isfinite(w[i])) return bc_set_error(BC_ERR_DEVICE, "training diverged (non-finite weights)");
    std::memcpy(weights, w.data(), kP * sizeof(float));
    if (final_loss) *final_loss = l;
    return BC_OK;
}

extern "C" bc_status bc_mlp_predict(const float *weights, const float *X, int64_t n, float *Y, void *stream) {
    if (!weights || !X || !Y || n < 0) return bc_set_error(BC_ERR_INVALID_ARG, "NULL argument or n < 0");
    if (n == 0) return BC_OK;
    hipStream_t st = (hipStream_t)stream;
    float *dw = nullptr, *dx = nullptr, *dy = nullptr;
    auto cleanup = [&]() {
        if (dw) (void)hipFree(dw);
        if (dx) (void)hipFree(dx);
        if (dy) (void)hipFree(dy);
    };
    hipError_t e = hipMalloc((void **)&dw, kP * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&dx, (size_t)n * kIn * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&dy, (size_t)n * kOut * sizeof(float));
    if (e == hipSuccess) e = hipMemcpyAsync(dw, weights, kP * sizeof(float), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dx, X, (size_t)n * kIn * sizeof(float), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        mlp_predict<<<(int)std::min<int64_t>((n + 255) / 256, 4096), 256, 0, st>>>(dw, dx, n, dy);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(Y, dy, (size_t)n * kOut * sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    cleanup();
    if (e != hipSuccess) return bc_set_error(BC_ERR_DEVICE, hipGetErrorString(e));
    return BC_OK;
}
