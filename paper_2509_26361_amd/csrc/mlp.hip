// mlp.hip -- the learned Front2VOF surrogate on gfx950 matrix cores.
//
// A multilayer perceptron 20 -> 128 -> 128 -> 1 (ReLU, ReLU, sigmoid) maps a
// cell's 12 edge-marker fractions and 8 corner colours to its volume
// fraction.  Products run on v_mfma_f32_16x16x32_bf16 (bfloat16 operands,
// FP32 accumulation); biases, activations, the last layer and the loss stay in
// FP32.  Operand layout of that instruction (16 x 32 A, 32 x 16 B, 16 x 16 D):
// lane l supplies row l%16 of A and column l%16 of B, with k = 8 (l/16) .. +7;
// it receives rows 4 (l/16) .. +3 of column l%16 of D.
//
// Parameters (FP32 master vector): W1 (20 x 128, in x out), b1, W2 (128 x
// 128), b2, w3 (128), b3 -- 19329 numbers.  Inputs are bfloat16 rows of 32
// (features 0..19, zeros after).  Rounding to bfloat16 is to nearest, ties
// to even, at: inputs, W1, W2, the first hidden layer before the second
// product, and in the backward pass dz2 and dz1 before their products.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "../../include/ebit.h"
#include "mlp_device.h"

using namespace ebit_mlp;

namespace {

// --------------------------------------------------------------------------
// inference
// --------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ theta, const uint16_t *__restrict__ x,
                                                     long m, float *__restrict__ y)
{
    __shared__ MlpWeights W;
    __shared__ __bf16 h1s[4][16 * kRow2];
    load_weights(W, theta);
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const long ntiles = (m + 15) / 16;
    for (long tile = (long)blockIdx.x * 4 + wave; tile < ntiles; tile += (long)gridDim.x * 4) {
        float out[4];
        forward_tile(W, h1s[wave], load_x(x, m, tile * 16), out, nullptr, nullptr);
        const int l = threadIdx.x & 63;
        if ((l & 15) == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                long row = tile * 16 + 4 * (l >> 4) + r;
                if (row < m) y[row] = out[r];
            }
        }
    }
}

// --------------------------------------------------------------------------
// training: per-workgroup partial gradients, fixed-order reduction, Adam
// --------------------------------------------------------------------------

constexpr int kPartial = kNParam + 1;     // gradient + loss sum

struct GradShared {
    MlpImage img;                          // weights; img.w2r: W2 as [k][j] for dz2 W2^T
    __bf16 xt[4][16 * kRow1];              // input tiles
    __bf16 h1[4][16 * kRow2];              // first hidden layer (bf16)
    __bf16 dz2[4][16 * kRow2];
    __bf16 dz1[4][16 * kRow2];
    float red[4][3][kNH];                  // per-wave column sums: dw3, db1, db2
    float reds[4][2];                      // db3, loss
};

// sum over the 4 lanes groups that share a column (lanes l, l^16, l^32, l^48)
__device__ __forceinline__ float col_sum(float v)
{
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// the parameters' image (see MlpImage), built by one launch
__global__ __launch_bounds__(256) void k_mlp_pack(const float *__restrict__ theta, MlpImage *__restrict__ img)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < kNH * kRow1) pack_w1_slot(img, theta, t);
    else if (t < kNH * kRow1 + kNParam - kOB1) image_store(img, kOB1 + (t - kNH * kRow1), theta[kOB1 + (t - kNH * kRow1)]);
}
constexpr int kPackThreads = kNH * kRow1 + kNParam - kOB1;

// A fragment of batch rows row0 .. row0 + 15: batch row r is data row
// idx[r] (idx NULL: row r); rows past the batch or with an index outside
// [0, nrows) read as zero
__device__ __forceinline__ bf16x8 load_batch_x(const uint16_t *__restrict__ x, const int64_t *__restrict__ idx,
                                               long nrows, long m, long row0)
{
    const int l = threadIdx.x & 63;
    const long row = row0 + (l & 15);
    u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
    if (row < m) {
        const long src = idx ? idx[row] : row;
        if (src >= 0 && src < nrows) v = *(const u16x8 *)(x + src * kKIn + 8 * (l >> 4));
    }
    return __builtin_bit_cast(bf16x8, v);
}

__global__ __launch_bounds__(256) void k_mlp_grad(const MlpImage *__restrict__ img, const uint16_t *__restrict__ x,
                                                  const float *__restrict__ c, const int64_t *__restrict__ idx,
                                                  long nrows, long m, float *__restrict__ partial)
{
    __shared__ GradShared S;
    copy_to_lds(&S.img, img, (int)sizeof(MlpImage));
    __syncthreads();
    const MlpWeights &W = S.img.W;
    const int wave = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int lr = l & 15, lg = l >> 4;
    const float inv_m = 2.0f / (float)m;

    f32x4 gW2[16];      // this wave owns dW2 tiles (kt = 2 wave + kt2, jt): kt2 in {0,1}, jt 0..7
    f32x4 gW1[4];       // dW1 tiles (kin tile 0..1, jt = 2 wave + jt2)
#pragma unroll
    for (int t = 0; t < 16; ++t) gW2[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 4; ++t) gW1[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float pw3[8], pb1[8], pb2[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) pw3[t] = pb1[t] = pb2[t] = 0.f;
    float pb3 = 0.f, ploss = 0.f;

    const long ngroups = (m + 63) / 64;
    for (long g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const long row0 = g * 64 + 16 * wave;
        // forward, keeping z1 and z2 (accumulator layout) and h1 in LDS
        f32x4 z1[8], z2[8];
        float yv[4];
        const bf16x8 ax = load_batch_x(x, idx, nrows, m, row0);
        *(bf16x8 *)&S.xt[wave][lr * kRow1 + 8 * lg] = ax;
        forward_tile(W, S.h1[wave], ax, yv, z1, z2);
        // dz3 for rows 4 lg + r (valid in lanes lr == 0, broadcast to the group)
        float dz3[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            long row = row0 + 4 * lg + r;
            float v = 0.f;
            long src = -1;
            if (lr == 0 && row < m) src = idx ? idx[row] : row;
            if (src >= 0 && src < nrows) {
                float cy = c[src];
                float d = yv[r] - cy;
                ploss += d * d;
                v = inv_m * d * yv[r] * (1.f - yv[r]);
                pb3 += v;
            }
            dz3[r] = __shfl(v, lg << 4);
        }
        // dw3, dz2 = dz3 w3 [z2 > 0], db2
#pragma unroll
        for (int jt = 0; jt < 8; ++jt) {
            const int j = 16 * jt + lr;
            const float w3 = W.w3[j], b2 = W.b2[j];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float zz = z2[jt][r] + b2;
                float h2 = zz > 0.f ? zz : 0.f;
                pw3[jt] += h2 * dz3[r];
                float d2 = zz > 0.f ? dz3[r] * w3 : 0.f;
                pb2[jt] += d2;
                S.dz2[wave][(4 * lg + r) * kRow2 + j] = to_bf16(d2);
            }
        }
        wave_sync();
        // dh1 = dz2 W2^T, dz1 = dh1 [z1 > 0], db1
        f32x4 dh[8];
#pragma unroll
        for (int kt = 0; kt < 8; ++kt) dh[kt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            bf16x8 a = *(const bf16x8 *)&S.dz2[wave][lr * kRow2 + 32 * ks + 8 * lg];
#pragma unroll
            for (int kt = 0; kt < 8; ++kt) {
                bf16x8 b = *(const bf16x8 *)&S.img.w2r[(16 * kt + lr) * kRow2 + 32 * ks + 8 * lg];
                dh[kt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, dh[kt], 0, 0, 0);
            }
        }
#pragma unroll
        for (int kt = 0; kt < 8; ++kt) {
            const int k = 16 * kt + lr;
            const float b1 = W.b1[k];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float d1 = (z1[kt][r] + b1) > 0.f ? dh[kt][r] : 0.f;
                pb1[kt] += d1;
                S.dz1[wave][(4 * lg + r) * kRow2 + k] = to_bf16(d1);
            }
        }
        __syncthreads();
        // dW2 += h1^T dz2 over the group's 64 rows (two k-steps of 32 rows)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
            for (int kt2 = 0; kt2 < 2; ++kt2) {
                const int kk = 16 * (2 * wave + kt2) + lr;       // hidden index (row of dW2)
                bf16x8 a;
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    int row = 32 * ks + 8 * lg + v;
                    a[v] = S.h1[row >> 4][(row & 15) * kRow2 + kk];
                }
#pragma unroll
                for (int jt = 0; jt < 8; ++jt) {
                    bf16x8 b;
#pragma unroll
                    for (int v = 0; v < 8; ++v) {
                        int row = 32 * ks + 8 * lg + v;
                        b[v] = S.dz2[row >> 4][(row & 15) * kRow2 + 16 * jt + lr];
                    }
                    gW2[kt2 * 8 + jt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, gW2[kt2 * 8 + jt], 0, 0, 0);
                }
            }
            // dW1 += X^T dz1
#pragma unroll
            for (int it = 0; it < 2; ++it) {
                const int kin = 16 * it + lr;
                bf16x8 a;
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    int row = 32 * ks + 8 * lg + v;
                    a[v] = S.xt[row >> 4][(row & 15) * kRow1 + kin];
                }
#pragma unroll
                for (int jt2 = 0; jt2 < 2; ++jt2) {
                    const int jt = 2 * wave + jt2;
                    bf16x8 b;
#pragma unroll
                    for (int v = 0; v < 8; ++v) {
                        int row = 32 * ks + 8 * lg + v;
                        b[v] = S.dz1[row >> 4][(row & 15) * kRow2 + 16 * jt + lr];
                    }
                    gW1[it * 2 + jt2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, gW1[it * 2 + jt2], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }

    // write this block's partial gradient in parameter order
    float *P = partial + (size_t)blockIdx.x * kPartial;
#pragma unroll
    for (int kt2 = 0; kt2 < 2; ++kt2)
#pragma unroll
        for (int jt = 0; jt < 8; ++jt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int k = 16 * (2 * wave + kt2) + 4 * lg + r, j = 16 * jt + lr;
                P[kOW2 + k * kNH + j] = gW2[kt2 * 8 + jt][r];
            }
#pragma unroll
    for (int it = 0; it < 2; ++it)
#pragma unroll
        for (int jt2 = 0; jt2 < 2; ++jt2)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int kin = 16 * it + 4 * lg + r, j = 16 * (2 * wave + jt2) + lr;
                if (kin < kNIn) P[kOW1 + kin * kNH + j] = gW1[it * 2 + jt2][r];
            }
    // column sums: over the 4 row groups of the wave, then over the 4 waves
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        float a3 = col_sum(pw3[t]), a1 = col_sum(pb1[t]), a2 = col_sum(pb2[t]);
        if (lg == 0) {
            S.red[wave][0][16 * t + lr] = a3;
            S.red[wave][1][16 * t + lr] = a1;
            S.red[wave][2][16 * t + lr] = a2;
        }
    }
    {
        float s3 = pb3, sl = ploss;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            s3 += __shfl_xor(s3, off);
            sl += __shfl_xor(sl, off);
        }
        if (l == 0) {
            S.reds[wave][0] = s3;
            S.reds[wave][1] = sl;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kNH; j += blockDim.x) {
        float a3 = 0.f, a1 = 0.f, a2 = 0.f;
        for (int w = 0; w < 4; ++w) {
            a3 += S.red[w][0][j];
            a1 += S.red[w][1][j];
            a2 += S.red[w][2][j];
        }
        P[kOW3 + j] = a3;
        P[kOB1 + j] = a1;
        P[kOB2 + j] = a2;
    }
    if (threadIdx.x == 0) {
        P[kOB3] = S.reds[0][0] + S.reds[1][0] + S.reds[2][0] + S.reds[3][0];
        P[kNParam] = S.reds[0][1] + S.reds[1][1] + S.reds[2][1] + S.reds[3][1];
    }
}

// Sum of the block partials of entry p (kNParam: the loss sum), the same
// fixed order at every call: wave w of the block adds blocks
// [w q, (w + 1) q) in order (q = ceil(nblocks / 4)), then the four wave sums
// are added in wave order.  Valid in the lanes of wave 0.
__device__ __forceinline__ float reduce_partials(const float *__restrict__ partial, int nblocks, int p,
                                                 float (*red)[64])
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = (nblocks + 3) / 4, b0 = wave * q, b1 = min(nblocks, b0 + q);
    float s = 0.f;
    if (p < kPartial) {
        int b = b0;
        for (; b + 8 <= b1; b += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = partial[(size_t)(b + u) * kPartial + p];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; b < b1; ++b) s += partial[(size_t)b * kPartial + p];
    }
    red[wave][lane] = s;
    __syncthreads();
    return ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// gradient (and the loss, mean over the m rows) from the partials: 64
// entries per workgroup
__global__ __launch_bounds__(256) void k_mlp_reduce(const float *__restrict__ partial, int nblocks, long m,
                                                    float *__restrict__ grad, float *__restrict__ loss)
{
    __shared__ float red[4][64];
    const int p = blockIdx.x * 64 + (threadIdx.x & 63);
    const float s = reduce_partials(partial, nblocks, p, red);
    if (threadIdx.x >= 64) return;
    if (p < kNParam) grad[p] = s;
    else if (p == kNParam && loss) *loss = s / (float)m;
}

struct AdamStep {
    float lr, bc1, bc2;   // learning rate, bias corrections 1 - beta^t
};

// Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on parameter p
__device__ __forceinline__ float adam_update(float *__restrict__ theta, float *__restrict__ m1,
                                             float *__restrict__ m2, int p, float g, AdamStep a)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float u = b1 * m1[p] + (1.f - b1) * g;
    float v = b2 * m2[p] + (1.f - b2) * g * g;
    m1[p] = u;
    m2[p] = v;
    float mh = u / a.bc1, vh = v / a.bc2;
    float t = theta[p] - a.lr * mh / (sqrtf(vh) + eps);
    theta[p] = t;
    return t;
}

__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ theta, float *__restrict__ m1,
                                                  float *__restrict__ m2, const float *__restrict__ grad, AdamStep a)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNParam) return;
    adam_update(theta, m1, m2, p, grad[p], a);
}

// one training step after k_mlp_grad: gradient from the partials, Adam, and
// the new parameters into the image the next step's gradient reads
__global__ __launch_bounds__(256) void k_mlp_reduce_adam(const float *__restrict__ partial, int nblocks, long m,
                                                         float *__restrict__ loss, float *__restrict__ theta,
                                                         float *__restrict__ m1, float *__restrict__ m2,
                                                         MlpImage *__restrict__ img, AdamStep a)
{
    __shared__ float red[4][64];
    const int p = blockIdx.x * 64 + (threadIdx.x & 63);
    const float s = reduce_partials(partial, nblocks, p, red);
    if (threadIdx.x >= 64) return;
    if (p < kNParam) image_store(img, p, adam_update(theta, m1, m2, p, s, a));
    else if (p == kNParam && loss) *loss = s / (float)m;
}

constexpr int kGradBlocks = 256;
constexpr size_t kPartialBytes = (size_t)kGradBlocks * kPartial * sizeof(float);   // a multiple of 16

inline MlpImage *image_of(void *work) { return (MlpImage *)((char *)work + kPartialBytes); }

inline int grad_blocks(long m)
{
    const long groups = (m + 63) / 64;
    return groups < kGradBlocks ? (int)groups : kGradBlocks;
}

inline AdamStep adam_step(int64_t t, float lr)
{
    return AdamStep{lr, (float)(1.0 - pow(0.9, (double)t)), (float)(1.0 - pow(0.999, (double)t))};
}

// work space: partial sums, then the parameters' image (16-byte aligned)
inline int scratch_ok(const void *work, size_t bytes)
{
    if (!work || ((uintptr_t)work & 15)) return EBIT_EINVAL;
    return bytes < kPartialBytes + sizeof(MlpImage) ? EBIT_ESCRATCH : EBIT_OK;
}

// gradient of the mean squared error over m rows: the parameters' image,
// per-workgroup partial sums (grad_blocks(m) of them, kPartial floats
// apart, from `partial`), their fixed-order sum
int launch_gradient(const float *theta, const void *x_bf16, const float *c, int64_t m, float *grad, float *loss,
                    float *partial, MlpImage *img, hipStream_t st)
{
    const int blocks = grad_blocks(m);
    hipLaunchKernelGGL(k_mlp_pack, dim3((kPackThreads + 255) / 256), dim3(256), 0, st, theta, img);
    hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(256), 0, st, img, (const uint16_t *)x_bf16, c,
                       (const int64_t *)nullptr, (long)m, (long)m, partial);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kPartial + 63) / 64), dim3(256), 0, st, (const float *)partial, blocks,
                       (long)m, grad, loss);
    return hipGetLastError() == hipSuccess ? EBIT_OK : EBIT_EHIP;
}

// --------------------------------------------------------------------------
// the gradient's work space in a static device array, for callers that
// cannot allocate (ebit_mlp_gradient_static): the partial sums of
// grad_blocks(EBIT_MLP_STATIC_MAX_ROWS) workgroups, then the image.  Every
// GPU holds its own copy at its own address; host code uses only the address
// hipGetSymbolAddress returns for the current device, never the array's name.
// --------------------------------------------------------------------------

constexpr int kStaticBlocks = (EBIT_MLP_STATIC_MAX_ROWS + 63) / 64;
static_assert(kStaticBlocks <= kGradBlocks, "static work space larger than the allocating path's");
constexpr size_t kStaticPartialBytes = ((size_t)kStaticBlocks * kPartial * sizeof(float) + 255) / 256 * 256;
constexpr size_t kStaticBytes = kStaticPartialBytes + sizeof(MlpImage);

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
char *g_static_addr[kMaxDevices];

}  // namespace

static __device__ __align__(256) char scratch[kStaticBytes];

namespace {

// address of the current device's copy of the static array (looked up once
// per device, with that device current)
int static_scratch(char **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return EBIT_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return EBIT_EHIP;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return EBIT_EHIP;
        g_static_addr[dev] = (char *)p;
    }
    *out = g_static_addr[dev];
    return EBIT_OK;
}

}  // namespace

extern "C" {

int ebit_mlp_param_count(void) { return kNParam; }

size_t ebit_mlp_scratch_bytes(void) { return kPartialBytes + sizeof(MlpImage); }

int ebit_mlp_forward(const float *theta, const void *x_bf16, int64_t m, float *y, void *stream)
{
    if (!theta || !x_bf16 || !y || m < 0) return EBIT_EINVAL;
    if (m == 0) return EBIT_OK;
    long tiles = (m + 15) / 16;
    int blocks = (int)((tiles + 3) / 4);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(256), 0, (hipStream_t)stream, theta,
                       (const uint16_t *)x_bf16, (long)m, y);
    return hipGetLastError() == hipSuccess ? EBIT_OK : EBIT_EHIP;
}

int ebit_mlp_gradient(const float *theta, const void *x_bf16, const float *c, int64_t m, float *grad, float *loss,
                      void *work, size_t work_bytes, void *stream)
{
    if (!theta || !x_bf16 || !c || !grad || m <= 0) return EBIT_EINVAL;
    if (int e = scratch_ok(work, work_bytes)) return e;
    return launch_gradient(theta, x_bf16, c, m, grad, loss, (float *)work, image_of(work), (hipStream_t)stream);
}

int ebit_mlp_gradient_static(const float *theta, const void *x_bf16, const float *c, int64_t m, float *grad,
                             float *loss, void *stream)
{
    if (!theta || !x_bf16 || !c || !grad || m <= 0) return EBIT_EINVAL;
    if (m > EBIT_MLP_STATIC_MAX_ROWS) return EBIT_ETOOBIG;
    char *base = nullptr;
    if (int e = static_scratch(&base)) return e;
    return launch_gradient(theta, x_bf16, c, m, grad, loss, (float *)base,
                           (MlpImage *)(base + kStaticPartialBytes), (hipStream_t)stream);
}

int ebit_mlp_adam(float *theta, float *m1, float *m2, const float *grad, int64_t step, float lr, void *stream)
{
    if (!theta || !m1 || !m2 || !grad || step < 1) return EBIT_EINVAL;
    hipLaunchKernelGGL(k_mlp_adam, dim3((kNParam + 255) / 256), dim3(256), 0, (hipStream_t)stream, theta, m1, m2, grad,
                       adam_step(step, lr));
    return hipGetLastError() == hipSuccess ? EBIT_OK : EBIT_EHIP;
}

int ebit_mlp_train(float *theta, float *m1, float *m2, const void *x_bf16, const float *c, int64_t nrows,
                   const int64_t *idx, int64_t batch, int64_t steps, const float *lr, int64_t step0, float *losses,
                   void *work, size_t work_bytes, void *stream)
{
    if (!theta || !m1 || !m2 || !x_bf16 || !c || nrows <= 0 || batch <= 0 || steps < 0 || step0 < 0) return EBIT_EINVAL;
    if (steps > 0 && !lr) return EBIT_EINVAL;
    if (!idx && batch > nrows) return EBIT_EINVAL;
    if (int e = scratch_ok(work, work_bytes)) return e;
    if (steps == 0) return EBIT_OK;
    const int blocks = grad_blocks(batch);
    hipStream_t st = (hipStream_t)stream;
    MlpImage *img = image_of(work);
    hipLaunchKernelGGL(k_mlp_pack, dim3((kPackThreads + 255) / 256), dim3(256), 0, st, theta, img);
    for (int64_t s = 0; s < steps; ++s) {
        hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(256), 0, st, img, (const uint16_t *)x_bf16, c,
                           idx ? idx + s * batch : (const int64_t *)nullptr, (long)nrows, (long)batch,
                           (float *)work);
        hipLaunchKernelGGL(k_mlp_reduce_adam, dim3((kPartial + 63) / 64), dim3(256), 0, st, (const float *)work,
                           blocks, (long)batch, losses ? losses + s : (float *)nullptr, theta, m1, m2, img,
                           adam_step(step0 + s + 1, lr[s]));
        if ((s & 255) == 255 && hipGetLastError() != hipSuccess) return EBIT_EHIP;
    }
    return hipGetLastError() == hipSuccess ? EBIT_OK : EBIT_EHIP;
}

}  // extern "C"
