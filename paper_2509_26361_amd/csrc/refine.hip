// refine.hip -- the AMR-compatible refinement band (paper sec. 2.3: every
// cell of the 3x3x3 block around an interfacial cell is refined to the finest
// level, and a Courant number of at most one keeps the interface inside that
// region for the next step).
//
// One pass over the periodic n^3 grid in tiles of 32 x 8 x 8 cells, taken in
// turn by persistent workgroups (see k_refine).  A tile's node flags are
// staged in LDS as 32-bit words; from there everything runs on words that
// hold four consecutive cells (one byte each, 0 or 1): the interfacial bytes
// of the 100 cell rows around the tile, the OR along x by byte shifts across
// word boundaries, then along y and z by ORing whole words of neighbouring
// rows.  A 4^3 brick is one word wide, so the brick flags are ORs of words,
// and the counts are popcounts of words.  The mask is written as whole words.
// About 1 byte is read (the halo rows come from L2) and 1 written per cell;
// the four LDS passes and their barriers per tile, not HBM, set the time.
// The last tile along y and z may reach past n (n is a multiple of 4): its
// cells beyond n are not written.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ebit.h"

namespace {

#ifndef EBIT_REFINE_TZ
#define EBIT_REFINE_TZ 8
#endif
#ifndef EBIT_REFINE_AHEAD
#define EBIT_REFINE_AHEAD 2
#endif
#ifndef EBIT_REFINE_GRID
#define EBIT_REFINE_GRID 1024
#endif
constexpr int TX = 32, TY = 8, TZ = EBIT_REFINE_TZ;   // cells per tile
constexpr int BY = TY / 4, BZ = TZ / 4;           // bricks per tile along y and z
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
// pass adds the sets in order.  (Summing them in the workgroup that finishes
// last needs a device-scope release per workgroup, which writes back the L2
// holding the freshly written mask: 28 us more than the extra launch.)
constexpr int kSets = 64, kSetStride = 32;
constexpr int kGrid = EBIT_REFINE_GRID;    // persistent workgroups (four of 512 threads per CU on 256 CUs)
constexpr int kAhead = EBIT_REFINE_AHEAD;  // tiles whose node words are in flight while one is computed

// periodic index for -n <= i < 2n (the y and z rows of a tile: n >= 8)
__device__ __forceinline__ int wrapr(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
// periodic index for -n <= i (the x words of a tile reach x0 + 39, more than
// one period past x0 when n < 36)
__device__ __forceinline__ int wrapm(int i, int n) { return i < 0 ? i + n : i % n; }

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

// Persistent workgroups, XCD-aware: workgroup ids are dealt to the eight XCDs
// round robin, so the workgroups b = x mod 8 (one XCD) take the x-th eighth
// of the tiles (x fastest, then y, then z: a slab along z), workgroup j of
// them the tiles j, j + Gx, ... of it.  The workgroups of an XCD running
// together work on neighbouring tiles of their slab and find their halo rows
// in that XCD's L2.  The node words of the next tile are loaded while the
// current one is computed; counts are summed over the workgroup's tiles and
// added to its set once.  The thread's coordinates in the staging and in the
// three LDS passes are the same for every tile and are computed once.
__global__ __launch_bounds__(kThreads) void k_refine(int n, const uint8_t *__restrict__ fl,
                                                    const uint8_t *__restrict__ mask_prev,
                                                    uint8_t *__restrict__ mask, uint8_t *__restrict__ bricks,
                                                    unsigned long long *__restrict__ sets)
{
    __shared__ uint32_t nodes[NZ][NY][NW];    // node flags, node x0 - 4 + b at byte b of the row
    __shared__ uint32_t inter[RZ][RY][IW];    // interfacial bytes, cell x0 - 4 + b at byte b
    __shared__ uint32_t dx[RZ][RY][WX];       // OR along x, cells x0 .. x0 + TX - 1
    __shared__ uint32_t red[4][kThreads / 64];
    __shared__ uint32_t bword[BZ][BY][WX];
    const int t = threadIdx.x;
    const int ntx = (n + TX - 1) / TX, nty = (n + TY - 1) / TY, ntz = (n + TZ - 1) / TZ;
    const int ntiles = ntx * nty * ntz;
    const uint32_t *fw = (const uint32_t *)fl;
    // the thread's staged node words of the next kAhead tiles (the threads
    // past the end load word 0 again and store nothing), all loads issued
    // before their first use
    uint32_t v[kAhead][kStage];
    int sw[kStage], sy[kStage], sz[kStage];   // staged word r: word, row along y, row along z
#pragma unroll
    for (int r = 0; r < kStage; ++r) {
        const int k0 = t + r * kThreads;
        const int k = k0 < NY * NZ * NW ? k0 : 0;
        sw[r] = k % NW;
        sy[r] = (k / NW) % NY;
        sz[r] = k / (NW * NY);
    }
    // the x words of a tile reach x0 + 39, more than one period past x0 when n < 36
    const bool wrap_twice = n < 4 * NW;
    auto load_tile = [&](int tile, uint32_t *vs) {
        const int x0 = (tile % ntx) * TX, y0 = ((tile / ntx) % nty) * TY, z0 = (tile / (ntx * nty)) * TZ;
        long qa[kStage];
#pragma unroll
        for (int r = 0; r < kStage; ++r) {
            const int xw = x0 - 4 + 4 * sw[r];
            const int x = wrap_twice ? wrapm(xw, n) : wrapr(xw, n);
            qa[r] = ((long)x + (long)n * ((long)wrapr(y0 - 1 + sy[r], n) + (long)n * (long)wrapr(z0 - 1 + sz[r], n))) >> 2;
        }
#pragma unroll
        for (int r = 0; r < kStage; ++r) vs[r] = fw[qa[r]];
    };
    // LDS offsets of the thread's items in the two passes (-1: none)
    constexpr int kIR = (RZ * RY * IW + kThreads - 1) / kThreads, kDR = (RZ * RY * WX + kThreads - 1) / kThreads;
    int io[kIR], inode[kIR], doff[kDR], dsrc[kDR];
#pragma unroll
    for (int i = 0; i < kIR; ++i) {
        const int k = t + i * kThreads;
        const int w = k % IW, ry = (k / IW) % RY, rz = k / (IW * RY);
        io[i] = k < RZ * RY * IW ? k : -1;
        inode[i] = (rz * NY + ry) * NW + w;
    }
#pragma unroll
    for (int i = 0; i < kDR; ++i) {
        const int k = t + i * kThreads;
        const int j = k % WX, ry = (k / WX) % RY, rz = k / (WX * RY);
        doff[i] = k < RZ * RY * WX ? k : -1;
        dsrc[i] = (rz * RY + ry) * IW + j;
    }
    uint32_t c_int = 0, c_mask = 0, c_brick = 0, c_esc = 0;
    const int G = (int)gridDim.x, b = (int)blockIdx.x;
    const int nx = G < 8 ? G : 8, x = b % nx, j0 = b / nx;
    const int Gx = (G - x + nx - 1) / nx;                 // workgroups b' < G with b' = x mod nx
    const int per = (ntiles + nx - 1) / nx;
    const int t0 = x * per, t1 = min(t0 + per, ntiles);  // this XCD's tiles
#pragma unroll
    for (int sl = 0; sl < kAhead; ++sl)
        if (t0 + j0 + sl * Gx < t1) load_tile(t0 + j0 + sl * Gx, v[sl]);
    for (int base = t0 + j0; base < t1; base += kAhead * Gx)
#pragma unroll
    for (int sl = 0; sl < kAhead; ++sl) {
        const int tile = base + sl * Gx;
        if (tile >= t1) break;
        const int x0 = (tile % ntx) * TX, y0 = ((tile / ntx) % nty) * TY, z0 = (tile / (ntx * nty)) * TZ;
#pragma unroll
        for (int r = 0; r < kStage; ++r) {
            const int k = t + r * kThreads;
            if (k < NY * NZ * NW) (&nodes[0][0][0])[k] = v[sl][r];
        }
        if (t < BZ * BY * WX) (&bword[0][0][0])[t] = 0;
        __syncthreads();
        if (tile + kAhead * Gx < t1) load_tile(tile + kAhead * Gx, v[sl]);
        // interfacial bytes: cell c has a marker on one of its 12 edges -- x-edges
        // (bit 4) at nodes c + (0, a, b), y-edges (bit 5) at c + (a, 0, b), z-edges
        // (bit 6) at c + (a, b, 0), a, b in {0, 1}
        {
            const uint32_t *nd = &nodes[0][0][0];
#pragma unroll
            for (int i = 0; i < kIR; ++i) {
                if (io[i] < 0) continue;
                const int o = inode[i];
                const uint32_t a00 = nd[o], a10 = nd[o + NW];
                const uint32_t a01 = nd[o + NY * NW], a11 = nd[o + NY * NW + NW];
                const uint32_t b00 = next1(a00, nd[o + 1]);
                const uint32_t b10 = next1(a10, nd[o + NW + 1]);
                const uint32_t b01 = next1(a01, nd[o + NY * NW + 1]);
                const uint32_t ex = (a00 | a10 | a01 | a11) & 0x10101010u;
                const uint32_t ey = (a00 | a01 | b00 | b01) & 0x20202020u;
                const uint32_t ez = (a00 | a10 | b00 | b10) & 0x40404040u;
                (&inter[0][0][0])[io[i]] = ((ex >> 4) | (ey >> 5) | (ez >> 6)) & kOnes;
            }
        }
        __syncthreads();
        // OR along x: output word j (cells x0 + 4j ..) is cell word j + 1
        {
            const uint32_t *in = &inter[0][0][0];
#pragma unroll
            for (int i = 0; i < kDR; ++i) {
                if (doff[i] < 0) continue;
                const int o = dsrc[i];
                const uint32_t c = in[o + 1], l = in[o], r = in[o + 2];
                (&dx[0][0][0])[doff[i]] = c | (c << 8) | (l >> 24) | (c >> 8) | (r << 24);
            }
        }
        __syncthreads();
        // OR along y and z: this thread's output word, its counts and its brick
        {
            const int j = t % WX, cy = (t / WX) % TY, cz = t / (WX * TY);
            uint32_t m = 0;
#pragma unroll
            for (int dz = 0; dz < 3; ++dz)
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) m |= dx[cz + dz][cy + dy][j];
            const uint32_t it = inter[cz + 1][cy + 1][j + 1];
            const int x = x0 + 4 * j, y = y0 + cy, z = z0 + cz;
            if (x < n && y < n && z < n) {
                const long q = (long)x + (long)n * ((long)y + (long)n * (long)z);
                *(uint32_t *)(mask + q) = m;
                c_int += __popc(it);
                c_mask += __popc(m);
                if (mask_prev) c_esc += __popc(it & ~nonzero_bytes(*(const uint32_t *)(mask_prev + q)) & kOnes);
                if (m) atomicOr(&bword[cz >> 2][cy >> 2][j], 1u);   // a brick is word j of 4 x 4 of the tile's rows
            }
        }
        __syncthreads();
        if (t < BZ * BY * WX) {
            // read and then cleared by the same thread at the next tile's start
            const int bj = t % WX, by = (t / WX) % BY, bz = t / (WX * BY);
            const int nb = n / 4, gx = x0 / 4 + bj, gy = y0 / 4 + by, gz = z0 / 4 + bz;
            if (gx < nb && gy < nb && gz < nb) {
                bricks[(long)gx + (long)nb * ((long)gy + (long)nb * (long)gz)] = (uint8_t)bword[bz][by][bj];
                c_brick += bword[bz][by][bj];
            }
        }
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
        unsigned long long s = 0;
        for (int w = 0; w < kThreads / 64; ++w) s += red[t][w];
        if (s) atomicAdd(&sets[(blockIdx.x % kSets) * kSetStride + t], s);
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
    const int ntiles = ((n + TX - 1) / TX) * ((n + TY - 1) / TY) * ((n + TZ - 1) / TZ);
    const dim3 grid((unsigned)(ntiles < kGrid ? ntiles : kGrid));
    unsigned long long *sets = (unsigned long long *)work;
    hipLaunchKernelGGL(k_refine_zero, dim3(1), dim3(256), 0, st, sets);
    hipLaunchKernelGGL(k_refine, grid, dim3(kThreads), 0, st, n, flags, mask_prev, mask, bricks, sets);
    hipLaunchKernelGGL(k_refine_sum, dim3(1), dim3(64), 0, st, (const unsigned long long *)sets,
                       (unsigned long long *)counts);
    return hipGetLastError() == hipSuccess ? EBIT_OK : EBIT_EHIP;
}

}  // extern "C"
