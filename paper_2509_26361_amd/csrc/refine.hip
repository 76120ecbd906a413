// refine.hip -- the AMR-compatible refinement band (paper sec. 2.3: every
// cell of the 3x3x3 block around an interfacial cell is refined to the finest
// level, and a Courant number of at most one keeps the interface inside that
// region for the next step).
//
// One streaming pass over the periodic n^3 grid.  A workgroup owns a tile of
// 32 x 4 x 4 cells and stages the flags of the nodes around it in LDS; from
// there everything runs on 32-bit words that hold four consecutive cells (one
// byte each, 0 or 1): the interfacial bytes of the 36 cell rows around the
// tile, the OR along x by byte shifts across word boundaries, then along y and
// z by ORing whole words of neighbouring rows.  A 4^3 brick is one word wide,
// so the brick flags are ORs of words, and the counts are popcounts of words.
// The mask is written as whole words.  About 1.7 bytes read and 1 written per
// cell: HBM bound.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ebit.h"

namespace {

constexpr int TX = 32, TY = 4, TZ = 4;            // cells per tile
constexpr int WX = TX / 4;                        // words per output row
constexpr int IW = WX + 2;                        // words per cell row: cells x0-4 .. x0+TX+3
constexpr int NW = IW + 1;                        // words per node row: nodes x0-4 .. x0+TX+7
constexpr int RY = TY + 2, RZ = TZ + 2;           // cell rows: y0-1 .. y0+TY, z0-1 .. z0+TZ
constexpr int NY = TY + 3, NZ = TZ + 3;           // node rows: one more on y and z
constexpr int kThreads = TZ * TY * WX;            // one thread per output word
constexpr int kStage = (NY * NZ * NW + kThreads - 1) / kThreads;   // staged node words per thread
constexpr uint32_t kOnes = 0x01010101u;
// counts: kSets sets of four, each on a 256-byte line of its own; workgroup b
// adds its nonzero counts to set b % kSets (few adds per address), a last
// pass adds the sets in order
constexpr int kSets = 64, kSetStride = 32;

__device__ __forceinline__ int wrapr(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// the four nodes starting one node later: word w shifted down a byte, the
// next word's lowest byte on top (little endian: byte 0 is the lowest node)
__device__ __forceinline__ uint32_t next1(uint32_t w, uint32_t w1) { return (w >> 8) | (w1 << 24); }

// 1 in each byte of w that is not zero, else 0
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t w)
{
    w |= w >> 4;
    w |= w >> 2;
    w |= w >> 1;
    return w & kOnes;
}

__global__ __launch_bounds__(kThreads) void k_refine(int n, const uint8_t *__restrict__ fl,
                                                    const uint8_t *__restrict__ mask_prev,
                                                    uint8_t *__restrict__ mask, uint8_t *__restrict__ bricks,
                                                    unsigned long long *__restrict__ sets)
{
    __shared__ uint32_t nodes[NZ][NY][NW];    // node flags, node x0 - 4 + b at byte b of the row
    __shared__ uint32_t inter[RZ][RY][IW];    // interfacial bytes, cell x0 - 4 + b at byte b
    __shared__ uint32_t dx[RZ][RY][WX];       // OR along x, cells x0 .. x0 + TX - 1
    __shared__ uint32_t red[4][kThreads / 64];
    __shared__ uint32_t bword[WX];
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
    const int t = threadIdx.x;
    // stage the node rows as whole words (x0 and n are multiples of 4, so a
    // word never straddles the periodic wrap); every load issued before the
    // first LDS store, the threads past the end load word 0 again and store
    // nothing
    {
        const uint32_t *fw = (const uint32_t *)fl;
        long qa[kStage];
#pragma unroll
        for (int r = 0; r < kStage; ++r) {
            const int k0 = t + r * kThreads;
            const int k = k0 < NY * NZ * NW ? k0 : 0;
            const int w = k % NW, iy = (k / NW) % NY, iz = k / (NW * NY);
            qa[r] = ((long)wrapr(x0 - 4 + 4 * w, n) +
                     (long)n * ((long)wrapr(y0 - 1 + iy, n) + (long)n * (long)wrapr(z0 - 1 + iz, n))) >> 2;
        }
        uint32_t v[kStage];
#pragma unroll
        for (int r = 0; r < kStage; ++r) v[r] = fw[qa[r]];
#pragma unroll
        for (int r = 0; r < kStage; ++r) {
            const int k = t + r * kThreads;
            if (k < NY * NZ * NW) (&nodes[0][0][0])[k] = v[r];
        }
    }
    if (t < WX) bword[t] = 0;
    __syncthreads();
    // interfacial bytes: cell c has a marker on one of its 12 edges -- x-edges
    // (bit 4) at nodes c + (0, a, b), y-edges (bit 5) at c + (a, 0, b), z-edges
    // (bit 6) at c + (a, b, 0), a, b in {0, 1}
    for (int k = t; k < RZ * RY * IW; k += kThreads) {
        const int w = k % IW, ry = (k / IW) % RY, rz = k / (IW * RY);
        const uint32_t a00 = nodes[rz][ry][w], a10 = nodes[rz][ry + 1][w];
        const uint32_t a01 = nodes[rz + 1][ry][w], a11 = nodes[rz + 1][ry + 1][w];
        const uint32_t b00 = next1(a00, nodes[rz][ry][w + 1]);
        const uint32_t b10 = next1(a10, nodes[rz][ry + 1][w + 1]);
        const uint32_t b01 = next1(a01, nodes[rz + 1][ry][w + 1]);
        const uint32_t ex = (a00 | a10 | a01 | a11) & 0x10101010u;
        const uint32_t ey = (a00 | a01 | b00 | b01) & 0x20202020u;
        const uint32_t ez = (a00 | a10 | b00 | b10) & 0x40404040u;
        inter[rz][ry][w] = ((ex >> 4) | (ey >> 5) | (ez >> 6)) & kOnes;
    }
    __syncthreads();
    // OR along x: output word j (cells x0 + 4j ..) is cell word j + 1
    for (int k = t; k < RZ * RY * WX; k += kThreads) {
        const int j = k % WX, ry = (k / WX) % RY, rz = k / (WX * RY);
        const uint32_t c = inter[rz][ry][j + 1], l = inter[rz][ry][j], r = inter[rz][ry][j + 2];
        dx[rz][ry][j] = c | (c << 8) | (l >> 24) | (c >> 8) | (r << 24);
    }
    __syncthreads();
    // OR along y and z: this thread's output word, its counts and its brick
    const int j = t % WX, cy = (t / WX) % TY, cz = t / (WX * TY);
    uint32_t m = 0;
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) m |= dx[cz + dz][cy + dy][j];
    const uint32_t it = inter[cz + 1][cy + 1][j + 1];
    const int x = x0 + 4 * j;
    uint32_t c_int = 0, c_mask = 0, c_esc = 0;
    if (x < n) {
        const long q = (long)x + (long)n * ((long)(y0 + cy) + (long)n * (long)(z0 + cz));
        *(uint32_t *)(mask + q) = m;
        c_int = __popc(it);
        c_mask = __popc(m);
        if (mask_prev) c_esc = __popc(it & ~nonzero_bytes(*(const uint32_t *)(mask_prev + q)) & kOnes);
        if (m) atomicOr(&bword[j], 1u);     // a brick is word j of the tile's 16 rows
    }
    __syncthreads();
    uint32_t c_brick = 0;
    if (t < WX && x0 + 4 * t < n) {
        const int nb = n / 4;
        bricks[(long)(x0 / 4 + t) + (long)nb * ((long)blockIdx.y + (long)nb * (long)blockIdx.z)] = (uint8_t)bword[t];
        c_brick = bword[t];
    }
    // counts: wave sums, then the workgroup's nonzero counts into its set
    const uint32_t cv[4] = {c_int, c_mask, c_brick, c_esc};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t s = cv[k];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if ((t & 63) == 0) red[k][t >> 6] = s;
    }
    __syncthreads();
    if (t < 4) {
        uint32_t s = 0;
        for (int w = 0; w < kThreads / 64; ++w) s += red[t][w];
        const long b = (long)blockIdx.x + (long)gridDim.x * ((long)blockIdx.y + (long)gridDim.y * (long)blockIdx.z);
        if (s) atomicAdd(&sets[(b % kSets) * kSetStride + t], (unsigned long long)s);
    }
}

__global__ void k_refine_zero(unsigned long long *sets)
{
    for (int k = threadIdx.x; k < kSets * 4; k += blockDim.x) sets[(k >> 2) * kSetStride + (k & 3)] = 0ull;
}

// the four totals: the sets added in order (integers)
__global__ void k_refine_sum(const unsigned long long *__restrict__ sets, unsigned long long *__restrict__ counts)
{
    if (threadIdx.x < 4) {
        unsigned long long s = 0;
        for (int k = 0; k < kSets; ++k) s += sets[k * kSetStride + threadIdx.x];
        counts[threadIdx.x] = s;
    }
}

}  // namespace

extern "C" {

size_t ebit_refine_work_bytes(int32_t n)
{
    if (n < 8 || n > 1024 || (n & 3)) return 0;
    return (size_t)kSets * kSetStride * sizeof(unsigned long long);
}

int ebit_refine_band(int32_t n, const uint8_t *flags, const uint8_t *mask_prev, uint8_t *mask, uint8_t *bricks,
                     int64_t *counts, void *work, size_t work_bytes, void *stream)
{
    if (n < 8 || n > 1024 || (n & 3) || !flags || !mask || !bricks || !counts || !work || ((uintptr_t)work & 7))
        return EBIT_EINVAL;
    if (((uintptr_t)flags & 3) || ((uintptr_t)mask & 3) || ((uintptr_t)mask_prev & 3)) return EBIT_EINVAL;
    if (work_bytes < ebit_refine_work_bytes(n)) return EBIT_ESCRATCH;
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)((n + TX - 1) / TX), (unsigned)(n / TY), (unsigned)(n / TZ));
    unsigned long long *sets = (unsigned long long *)work;
    hipLaunchKernelGGL(k_refine_zero, dim3(1), dim3(256), 0, st, sets);
    hipLaunchKernelGGL(k_refine, grid, dim3(kThreads), 0, st, n, flags, mask_prev, mask, bricks, sets);
    hipLaunchKernelGGL(k_refine_sum, dim3(1), dim3(64), 0, st, (const unsigned long long *)sets,
                       (unsigned long long *)counts);
    return hipGetLastError() == hipSuccess ? EBIT_OK : EBIT_EHIP;
}

}  // extern "C"
