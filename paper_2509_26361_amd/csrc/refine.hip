// refine.hip -- the AMR-compatible refinement band (paper sec. 2.3: every
// cell of the 3x3x3 block around an interfacial cell is refined to the finest
// level, and a Courant number of at most one keeps the interface inside that
// region for the next step).
//
// One streaming pass over the periodic n^3 grid.  A workgroup owns a tile of
// 32 x 4 x 4 cells (x fastest: whole 32-byte runs of the flags and mask rows)
// and stages the flags of its 35 x 7 x 7 nodes (the tile, one node below and
// two above on each axis) in LDS; from them the interfacial bits of the
// 34 x 6 x 6 cells around the tile, then each tile cell's 3x3x3 OR.  Bricks
// of 4^3 cells and the counts come out of the same tile.  The pass reads
// about 1.7 bytes and writes 1 byte per cell: HBM bound.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ebit.h"

namespace {

constexpr int TX = 32, TY = 4, TZ = 4;                 // cells per tile
constexpr int NX = TX + 3, NY = TY + 3, NZ = TZ + 3;   // staged nodes: -1 .. T+1
constexpr int IX = TX + 2, IY = TY + 2, IZ = TZ + 2;   // interfacial bits: cells -1 .. T
constexpr int kThreads = 256;

__device__ __forceinline__ int wrapr(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__global__ __launch_bounds__(kThreads) void k_refine(int n, const uint8_t *__restrict__ fl,
                                                    const uint8_t *__restrict__ mask_prev,
                                                    uint8_t *__restrict__ mask, uint8_t *__restrict__ bricks,
                                                    unsigned long long *__restrict__ counts)
{
    __shared__ uint8_t nodes[NZ][NY][NX];
    __shared__ uint8_t inter[IZ][IY][IX];
    __shared__ uint8_t tmask[TZ][TY][TX];
    __shared__ unsigned red[4][kThreads / 64];
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
    const int t = threadIdx.x;
    for (int k = t; k < NX * NY * NZ; k += kThreads) {
        const int ix = k % NX, iy = (k / NX) % NY, iz = k / (NX * NY);
        const long q = (long)wrapr(x0 - 1 + ix, n) + (long)n * ((long)wrapr(y0 - 1 + iy, n) +
                                                               (long)n * (long)wrapr(z0 - 1 + iz, n));
        nodes[iz][iy][ix] = fl[q];
    }
    __syncthreads();
    // cell c (local -1 .. T, stored at c + 1) is interfacial when one of its
    // 12 edges carries a marker: x-edges at nodes c + (0, a, b), y-edges at
    // c + (a, 0, b), z-edges at c + (a, b, 0), a, b in {0, 1}
    for (int k = t; k < IX * IY * IZ; k += kThreads) {
        const int cx = k % IX, cy = (k / IX) % IY, cz = k / (IX * IY);
        uint8_t any = 0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                any |= nodes[cz + b][cy + a][cx] & 0x10;
                any |= nodes[cz + b][cy][cx + a] & 0x20;
                any |= nodes[cz][cy + b][cx + a] & 0x40;
            }
        inter[cz][cy][cx] = any ? 1 : 0;
    }
    __syncthreads();
    unsigned c_int = 0, c_mask = 0, c_esc = 0;
    for (int k = t; k < TX * TY * TZ; k += kThreads) {
        const int cx = k % TX, cy = (k / TX) % TY, cz = k / (TX * TY);
        const int x = x0 + cx;
        uint8_t m = 0;
#pragma unroll
        for (int dz = 0; dz < 3; ++dz)
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) m |= inter[cz + dz][cy + dy][cx + dx];
        tmask[cz][cy][cx] = x < n ? m : 0;
        if (x < n) {
            const long q = (long)x + (long)n * ((long)(y0 + cy) + (long)n * (long)(z0 + cz));
            mask[q] = m;
            const uint8_t it = inter[cz + 1][cy + 1][cx + 1];
            c_int += it;
            c_mask += m;
            if (mask_prev && it && !mask_prev[q]) ++c_esc;
        }
    }
    __syncthreads();
    // bricks: the tile holds TX / 4 of them along x, one along y and z
    unsigned c_brick = 0;
    if (t < TX / 4 && x0 + 4 * t < n) {
        uint8_t any = 0;
        for (int cz = 0; cz < TZ; ++cz)
            for (int cy = 0; cy < TY; ++cy)
                for (int cx = 4 * t; cx < 4 * t + 4; ++cx) any |= tmask[cz][cy][cx];
        const int nb = n / 4;
        bricks[(long)(x0 / 4 + t) + (long)nb * ((long)blockIdx.y + (long)nb * (long)blockIdx.z)] = any;
        c_brick = any;
    }
    // counts: wave sums, then one atomic add per workgroup and count (integers: order-free)
    unsigned v[4] = {c_int, c_mask, c_brick, c_esc};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        unsigned s = v[j];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if ((t & 63) == 0) red[j][t >> 6] = s;
    }
    __syncthreads();
    if (t < 4) {
        unsigned s = 0;
        for (int w = 0; w < kThreads / 64; ++w) s += red[t][w];
        if (s) atomicAdd(&counts[t], (unsigned long long)s);
    }
}

__global__ void k_refine_zero(unsigned long long *counts)
{
    if (threadIdx.x < 4) counts[threadIdx.x] = 0;
}

}  // namespace

extern "C" {

int ebit_refine_band(int32_t n, const uint8_t *flags, const uint8_t *mask_prev, uint8_t *mask, uint8_t *bricks,
                     int64_t *counts, void *stream)
{
    if (n < 8 || n > 1024 || (n & 3) || !flags || !mask || !bricks || !counts) return EBIT_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_refine_zero, dim3(1), dim3(64), 0, st, (unsigned long long *)counts);
    const dim3 grid((unsigned)((n + TX - 1) / TX), (unsigned)(n / TY), (unsigned)(n / TZ));
    hipLaunchKernelGGL(k_refine, grid, dim3(kThreads), 0, st, n, flags, mask_prev, mask, bricks,
                       (unsigned long long *)counts);
    return hipGetLastError() == hipSuccess ? EBIT_OK : EBIT_EHIP;
}

}  // extern "C"
