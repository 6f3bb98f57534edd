// Pivot network: a 16 -> 64 -> 64 -> 1 perceptron (ReLU hidden layers,
// logistic output) that maps statistics of a Filter-Borůvka pivot sample to
// the sample quantile used as pivot.  Not part of the paper, which takes the
// sample median; any pivot gives the same MSF, the network only changes time.
#pragma once
#include "common.h"

namespace msf {

constexpr int kMlpIn = 16;
constexpr int kMlpH = 64;
// FP32 parameter vector layout: W1[H][IN], b1[H], W2[H][H], b2[H], w3[H], b3.
constexpr int kMlpOffW1 = 0;
constexpr int kMlpOffB1 = kMlpOffW1 + kMlpH * kMlpIn;
constexpr int kMlpOffW2 = kMlpOffB1 + kMlpH;
constexpr int kMlpOffB2 = kMlpOffW2 + kMlpH * kMlpH;
constexpr int kMlpOffW3 = kMlpOffB2 + kMlpH;
constexpr int kMlpOffB3 = kMlpOffW3 + kMlpH;
constexpr int kMlpParams = kMlpOffB3 + 1;
constexpr float kQMin = 1.0f / 1024.0f;   // quantile clamp of the network output

// Round to the nearest bfloat16 (ties to even) and return it as a float.
__host__ __device__ __forceinline__ float bf16r(float f) {
    uint32_t b;
    __builtin_memcpy(&b, &f, 4);
    if ((b & 0x7f800000u) == 0x7f800000u) return f;    // inf / nan unchanged
    b += 0x7fffu + ((b >> 16) & 1u);
    b &= 0xffff0000u;
    float r;
    __builtin_memcpy(&r, &b, 4);
    return r;
}

// Network output on one feature vector, computed by one workgroup: threads
// 0..63 each own a hidden unit.  w: bf16-rounded parameters; x, h: LDS
// scratch of kMlpIn and 2 * kMlpH floats.  Every thread must call it.
__device__ __forceinline__ float mlp_infer_block(const float* __restrict__ w, float* x, float* h) {
    const int j = threadIdx.x;
    if (j < kMlpH) {
        float acc = w[kMlpOffB1 + j];
        for (int i = 0; i < kMlpIn; ++i) acc += w[kMlpOffW1 + j * kMlpIn + i] * bf16r(x[i]);
        h[j] = bf16r(acc > 0.f ? acc : 0.f);
    }
    __syncthreads();
    if (j < kMlpH) {
        float acc = w[kMlpOffB2 + j];
        for (int k = 0; k < kMlpH; ++k) acc += w[kMlpOffW2 + j * kMlpH + k] * h[k];
        h[kMlpH + j] = bf16r(acc > 0.f ? acc : 0.f);
    }
    __syncthreads();
    float z = w[kMlpOffB3];
    for (int k = 0; k < kMlpH; ++k) z += w[kMlpOffW3 + k] * h[kMlpH + k];
    return z;
}

// Device copy of the loaded network for inference (null when none is loaded).
const float* mlp_device_params();

}  // namespace msf
