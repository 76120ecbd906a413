// mlp_device.h -- device building blocks of the surrogate network shared by
// the training / inference kernels and the Front2VOF surrogate path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ebit_mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kNIn = 20, kKIn = 32, kNH = 128;
constexpr int kOW1 = 0, kOB1 = kOW1 + kNIn * kNH, kOW2 = kOB1 + kNH, kOB2 = kOW2 + kNH * kNH, kOW3 = kOB2 + kNH,
              kOB3 = kOW3 + kNH, kNParam = kOB3 + 1;
constexpr int kRow1 = 40, kRow2 = 136;   // padded LDS rows: conflict-free 16-byte fragment reads

// FP32 -> bfloat16, round to nearest, ties to even
__device__ __forceinline__ __bf16 to_bf16(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __builtin_bit_cast(__bf16, (uint16_t)(u >> 16));
}

// make LDS writes of the wave visible to its other lanes
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// weights staged in LDS in the layout of the B operands of the forward pass
struct alignas(16) MlpWeights {
    __bf16 w1[kNH * kRow1];    // [j][k] = W1[k][j], k < 20; zero for 20 <= k < 32
    __bf16 w2[kNH * kRow2];    // [j][k] = W2[k][j]
    float b1[kNH], b2[kNH], w3[kNH];
    float b3;
};

// the bfloat16 weights of the forward pass and W2 once more as [k][j] (the B
// operand of dz2 W2^T in the backward pass): built in device memory from the
// FP32 parameters, then copied whole into LDS by every workgroup
struct alignas(16) MlpImage {
    MlpWeights W;
    __bf16 w2r[kNH * kRow2];
};

// the image entries of parameter p (value v); W1 columns 20..31 are zero and
// are written by pack_w1_slot, the other pad entries are never read
__device__ __forceinline__ void image_store(MlpImage *img, int p, float v)
{
    if (p < kOB1) {
        const int k = p / kNH, j = p % kNH;
        img->W.w1[j * kRow1 + k] = to_bf16(v);
    } else if (p < kOW2) {
        img->W.b1[p - kOB1] = v;
    } else if (p < kOB2) {
        const int q = p - kOW2, k = q / kNH, j = q % kNH;
        const __bf16 b = to_bf16(v);
        img->W.w2[j * kRow2 + k] = b;
        img->w2r[k * kRow2 + j] = b;
    } else if (p < kOW3) {
        img->W.b2[p - kOB2] = v;
    } else if (p < kOB3) {
        img->W.w3[p - kOW3] = v;
    } else {
        img->W.b3 = v;
    }
}

// slot t < kNH * kRow1 of the W1 image: W1[k][j] for k < 20, zero otherwise
__device__ __forceinline__ void pack_w1_slot(MlpImage *img, const float *__restrict__ theta, int t)
{
    const int j = t / kRow1, k = t % kRow1;
    img->W.w1[t] = k < kNIn ? to_bf16(theta[kOW1 + k * kNH + j]) : to_bf16(0.f);
}

// copy `bytes` (a multiple of 16) from device memory into LDS, whole block.
// Each lane issues the loads of up to kCopyBatch rounds before their LDS
// stores, so the copy waits for memory once per batch instead of once per
// 16-byte round (a block's copy of the weights image is 6 to 20 rounds).
constexpr int kCopyBatch = 8;
__device__ __forceinline__ void copy_to_lds(void *dst, const void *__restrict__ src, int bytes)
{
    const uint4 *s = (const uint4 *)src;
    uint4 *d = (uint4 *)dst;
    const int n = bytes / 16, nt = (int)blockDim.x;
    // indices past the end are clamped to the last entry: those lanes copy
    // it once more (the same value), and the loop body has no branch that
    // would pull each load down to its store
    for (int i0 = (int)threadIdx.x; i0 < n; i0 += kCopyBatch * nt) {
        uint4 v[kCopyBatch];
#pragma unroll
        for (int r = 0; r < kCopyBatch; ++r) v[r] = s[min(i0 + r * nt, n - 1)];
#pragma unroll
        for (int r = 0; r < kCopyBatch; ++r) d[min(i0 + r * nt, n - 1)] = v[r];
    }
}

__device__ inline void load_weights(MlpWeights &W, const float *__restrict__ theta)
{
    for (int i = threadIdx.x; i < kNH * kKIn; i += blockDim.x) {
        int k = i / kNH, j = i % kNH;
        W.w1[j * kRow1 + k] = k < kNIn ? to_bf16(theta[kOW1 + k * kNH + j]) : to_bf16(0.f);
    }
    for (int i = threadIdx.x; i < kNH * kNH; i += blockDim.x) {
        int k = i / kNH, j = i % kNH;
        W.w2[j * kRow2 + k] = to_bf16(theta[kOW2 + k * kNH + j]);
    }
    for (int i = threadIdx.x; i < kNH; i += blockDim.x) {
        W.b1[i] = theta[kOB1 + i];
        W.b2[i] = theta[kOB2 + i];
        W.w3[i] = theta[kOW3 + i];
    }
    if (threadIdx.x == 0) W.b3 = theta[kOB3];
}

// A fragment of 16 input rows (bfloat16, 32 per row) starting at row0
__device__ __forceinline__ bf16x8 load_x(const uint16_t *__restrict__ x, long m, long row0)
{
    const int l = threadIdx.x & 63;
    const long row = row0 + (l & 15);
    u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
    if (row < m) v = *(const u16x8 *)(x + row * kKIn + 8 * (l >> 4));
    return __builtin_bit_cast(bf16x8, v);
}

// Forward pass of 16 rows by one wave.  `ax` is the A fragment of the input
// rows; h1s is the wave's LDS tile of the first hidden layer (16 x kRow2).
// out[r] receives y for row 4 (l/16) + r in every lane; z1o / z2o (optional)
// the first / second layer products without bias (accumulator layout).
__device__ inline void forward_tile(const MlpWeights &W, __bf16 *h1s, bf16x8 ax, float out[4], f32x4 *z1o,
                                    f32x4 *z2o)
{
    const int l = threadIdx.x & 63;
    const int lr = l & 15, lg = l >> 4;
    f32x4 acc[8];
#pragma unroll
    for (int jt = 0; jt < 8; ++jt) {
        bf16x8 b = *(const bf16x8 *)&W.w1[(16 * jt + lr) * kRow1 + 8 * lg];
        acc[jt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, b, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    }
#pragma unroll
    for (int jt = 0; jt < 8; ++jt) {
        const int j = 16 * jt + lr;
        const float b1 = W.b1[j];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float z = acc[jt][r] + b1;
            h1s[(4 * lg + r) * kRow2 + j] = to_bf16(z > 0.f ? z : 0.f);
        }
        if (z1o) z1o[jt] = acc[jt];
    }
    wave_sync();
#pragma unroll
    for (int jt = 0; jt < 8; ++jt) acc[jt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        bf16x8 a = *(const bf16x8 *)&h1s[lr * kRow2 + 32 * ks + 8 * lg];
#pragma unroll
        for (int jt = 0; jt < 8; ++jt) {
            bf16x8 b = *(const bf16x8 *)&W.w2[(16 * jt + lr) * kRow2 + 32 * ks + 8 * lg];
            acc[jt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[jt], 0, 0, 0);
        }
    }
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int jt = 0; jt < 8; ++jt) {
        const int j = 16 * jt + lr;
        const float b2 = W.b2[j], w3 = W.w3[j];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float z = acc[jt][r] + b2;
            part[r] += (z > 0.f ? z : 0.f) * w3;
        }
        if (z2o) z2o[jt] = acc[jt];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float v = part[r];
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        out[r] = 1.f / (1.f + expf(-(v + W.b3)));
    }
    wave_sync();   // h1s may be rewritten by the next tile
}

}  // namespace ebit_mlp
