// Pivot network kernels: batched training (forward + backward + Adam, FP32
// gradients, optional BF16 forward), single-sample inference used by the
// Filter-Borůvka pivot sampler, and the loaded model store.
//
// Loss: mean over the batch of (z - t)^2 / 2, z the pre-sigmoid output and
// t the target logit.  In BF16 mode weights, inputs and hidden activations
// are rounded to bfloat16 before every product (accumulation stays FP32);
// the backward pass uses those rounded values.
#include <string.h>

#include <mutex>

#include "host.h"
#include "mlp.h"
#include "prim.h"

namespace msf {

// One sample per thread; gradients summed per workgroup in LDS, then added
// to `grad` (kMlpParams floats, zeroed by the caller).  z_out / loss optional.
template <bool BF16>
__global__ __launch_bounds__(256) void k_mlp_train(const float* __restrict__ params,
                                                   const float* __restrict__ x,
                                                   const float* __restrict__ target, int64_t B,
                                                   float* __restrict__ grad,
                                                   float* __restrict__ z_out,
                                                   float* __restrict__ loss) {
    __shared__ float P[kMlpParams];
    __shared__ float Gs[kMlpParams];
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) {
        P[i] = BF16 ? bf16r(params[i]) : params[i];
        Gs[i] = 0.f;
    }
    __syncthreads();
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    float lsum = 0.f;
    if (b < B) {
        float xi[kMlpIn], h1[kMlpH], h2[kMlpH];
        for (int i = 0; i < kMlpIn; ++i) xi[i] = BF16 ? bf16r(x[b * kMlpIn + i]) : x[b * kMlpIn + i];
        for (int j = 0; j < kMlpH; ++j) {
            float acc = P[kMlpOffB1 + j];
            for (int i = 0; i < kMlpIn; ++i) acc += P[kMlpOffW1 + j * kMlpIn + i] * xi[i];
            acc = acc > 0.f ? acc : 0.f;
            h1[j] = BF16 ? bf16r(acc) : acc;
        }
        for (int j = 0; j < kMlpH; ++j) {
            float acc = P[kMlpOffB2 + j];
            for (int k = 0; k < kMlpH; ++k) acc += P[kMlpOffW2 + j * kMlpH + k] * h1[k];
            acc = acc > 0.f ? acc : 0.f;
            h2[j] = BF16 ? bf16r(acc) : acc;
        }
        float z = P[kMlpOffB3];
        for (int j = 0; j < kMlpH; ++j) z += P[kMlpOffW3 + j] * h2[j];
        if (z_out) z_out[b] = z;
        if (grad) {
            const float t = target[b];
            lsum = 0.5f * (z - t) * (z - t);
            const float dz = (z - t) / (float)B;
            atomicAdd(&Gs[kMlpOffB3], dz);
            float dh2[kMlpH];
            for (int j = 0; j < kMlpH; ++j) {
                atomicAdd(&Gs[kMlpOffW3 + j], dz * h2[j]);
                dh2[j] = h2[j] > 0.f ? dz * P[kMlpOffW3 + j] : 0.f;
            }
            for (int j = 0; j < kMlpH; ++j) {
                if (dh2[j] == 0.f) continue;
                atomicAdd(&Gs[kMlpOffB2 + j], dh2[j]);
                for (int k = 0; k < kMlpH; ++k)
                    atomicAdd(&Gs[kMlpOffW2 + j * kMlpH + k], dh2[j] * h1[k]);
            }
            for (int k = 0; k < kMlpH; ++k) {
                if (h1[k] <= 0.f) continue;
                float d = 0.f;
                for (int j = 0; j < kMlpH; ++j) d += P[kMlpOffW2 + j * kMlpH + k] * dh2[j];
                if (d == 0.f) continue;
                atomicAdd(&Gs[kMlpOffB1 + k], d);
                for (int i = 0; i < kMlpIn; ++i) atomicAdd(&Gs[kMlpOffW1 + k * kMlpIn + i], d * xi[i]);
            }
        }
    }
    if (grad) {
        __syncthreads();
        for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x)
            if (Gs[i] != 0.f) atomicAdd(&grad[i], Gs[i]);
        float l = lsum;
        for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
        if (lane_id() == 0 && loss) atomicAdd(loss, l / (float)B);
    }
}

// Adam (Kingma & Ba 2015) on FP32 master parameters.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// -------------------------------------------------------------- model store

namespace {
std::mutex g_model_mu;
float* g_model_dev = nullptr;      // bf16-rounded FP32 parameters on the device
bool g_model_loaded = false;
constexpr uint32_t kBlobMagic = 0x5046534d;   // "MSFP"
constexpr uint32_t kBlobVersion = 1;
}  // namespace

const float* mlp_device_params() {
    std::lock_guard<std::mutex> l(g_model_mu);
    return g_model_loaded ? g_model_dev : nullptr;
}

}  // namespace msf

using namespace msf;

extern "C" {

int msf_pivot_model_load(const void* blob, size_t bytes) {
    // blob: uint32 magic, version, inputs, hidden; then kMlpParams float32
    if (!blob || bytes != 16 + sizeof(float) * (size_t)kMlpParams) return MSF_EINVAL;
    uint32_t hdr[4];
    memcpy(hdr, blob, 16);
    if (hdr[0] != kBlobMagic || hdr[1] != kBlobVersion || hdr[2] != (uint32_t)kMlpIn ||
        hdr[3] != (uint32_t)kMlpH)
        return MSF_EINVAL;
    float host[kMlpParams];
    memcpy(host, (const char*)blob + 16, sizeof host);
    for (int i = 0; i < kMlpParams; ++i) {
        if (!(host[i] == host[i]) || host[i] > 1e30f || host[i] < -1e30f) return MSF_EINVAL;
        host[i] = bf16r(host[i]);   // inference runs on bfloat16 weights
    }
    std::lock_guard<std::mutex> l(g_model_mu);
    if (!g_model_dev) HIP_TRY(hipMalloc((void**)&g_model_dev, sizeof host));
    HIP_TRY(hipMemcpy(g_model_dev, host, sizeof host, hipMemcpyHostToDevice));
    g_model_loaded = true;
    return MSF_OK;
}

int msf_pivot_model_clear(void) {
    std::lock_guard<std::mutex> l(g_model_mu);
    g_model_loaded = false;
    return MSF_OK;
}

int msf_pivot_model_loaded(void) { return mlp_device_params() ? 1 : 0; }

int msf_mlp_param_count(void) { return kMlpParams; }

int msf_mlp_forward(const float* params, const float* x, int64_t B, float* z_out, int bf16,
                    void* stream) {
    if (B < 0 || (B > 0 && (!params || !x || !z_out))) return MSF_EINVAL;
    if (B == 0) return MSF_OK;
    const unsigned grid = (unsigned)((B + 255) / 256);
    hipStream_t s = (hipStream_t)stream;
    if (bf16)
        hipLaunchKernelGGL(k_mlp_train<true>, dim3(grid), dim3(256), 0, s, params, x, nullptr, B,
                           nullptr, z_out, nullptr);
    else
        hipLaunchKernelGGL(k_mlp_train<false>, dim3(grid), dim3(256), 0, s, params, x, nullptr, B,
                           nullptr, z_out, nullptr);
    HIP_TRY(hipGetLastError());
    return MSF_OK;
}

int msf_mlp_grad(const float* params, const float* x, const float* target, int64_t B, int bf16,
                 float* grad_out, float* loss_out, void* stream) {
    if (B <= 0 || !params || !x || !target || !grad_out || !loss_out) return MSF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemsetAsync(grad_out, 0, sizeof(float) * kMlpParams, s));
    HIP_TRY(hipMemsetAsync(loss_out, 0, sizeof(float), s));
    const unsigned grid = (unsigned)((B + 255) / 256);
    if (bf16)
        hipLaunchKernelGGL(k_mlp_train<true>, dim3(grid), dim3(256), 0, s, params, x, target, B,
                           grad_out, nullptr, loss_out);
    else
        hipLaunchKernelGGL(k_mlp_train<false>, dim3(grid), dim3(256), 0, s, params, x, target, B,
                           grad_out, nullptr, loss_out);
    HIP_TRY(hipGetLastError());
    return MSF_OK;
}

int msf_mlp_adam(float* params, const float* grad, float* m, float* v, float lr, float beta1,
                 float beta2, float eps, int step, void* stream) {
    if (!params || !grad || !m || !v || step < 1 || !(lr > 0.f)) return MSF_EINVAL;
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       params, grad, m, v, kMlpParams, lr, beta1, beta2, eps, c1, c2);
    HIP_TRY(hipGetLastError());
    return MSF_OK;
}

}  // extern "C"
