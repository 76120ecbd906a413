// curvature.hip -- interface curvature by height functions and the
// continuum-surface-force (CSF) term, from the volume fraction C that
// Front2VOF produces (paper sec. 2.5: C is coupled to the flow solver through
// a well-balanced CSF term with generalised height-function curvature).
//
// Curvature: a streaming pass over the whole periodic n^3 grid (x fastest,
// one thread per cell, few registers) writes the zeros of the cells away from
// the interface and compacts the cells with 0 < C < 1 into a list by wave
// ballot; two dense passes over that list, one lane per cell, gather the
// 3x3x7 stencils through the caches (the heights need many registers, which
// would starve the streaming pass of occupancy).  The CSF pass streams the
// grid again.  All arithmetic is FP64 (C in FP32 is widened on load) in the
// order stated in include/ebit.h, so results are reproducible bit for bit.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/ebit.h"

namespace {

constexpr int kCurvBlock = 256;
// The list is kLists sub-lists, each with its own append counter on a cache
// line of its own: workgroup b of the streaming pass appends to sub-list
// b % kLists, one atomic add per workgroup, so the appends of the whole grid
// spread over kLists addresses instead of queueing on one.
constexpr int kLists = 256;
constexpr int kDenseBlocks = 1024;   // grid of the dense passes (grid-stride over the listed cells)
constexpr int kCtrStride = 32;       // 128 bytes between counters

inline long list_cap(long N)
{
    const long blocks = (N + kCurvBlock - 1) / kCurvBlock;
    return ((blocks + kLists - 1) / kLists) * kCurvBlock;   // the cells of every workgroup that appends to it
}

enum : uint8_t { KS_NONE = 0, KS_HF = 1, KS_HF_OTHER = 2, KS_MEAN = 3, KS_MISSING = 4 };

__device__ __forceinline__ int wrapc(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T>
struct Grid {
    const T *__restrict__ C;
    int n;
    __device__ __forceinline__ double at(int x, int y, int z) const
    {
        return (double)C[(long)wrapc(x, n) + (long)n * ((long)wrapc(y, n) + (long)n * (long)wrapc(z, n))];
    }
    __device__ __forceinline__ double at3(const int p[3]) const { return at(p[0], p[1], p[2]); }
};

// The 3x3x3 block of C around p, nb[dz + 1][dy + 1][dx + 1]: every cell the
// three Youngs gradients read, loaded in one round (27 loads issued together)
template <typename T>
__device__ __forceinline__ void block3(const Grid<T> &g, const int p[3], double nb[3][3][3])
{
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) nb[dz + 1][dy + 1][dx + 1] = g.at(p[0] + dx, p[1] + dy, p[2] + dz);
}

// Youngs' gradient component along d from the block: weights (1,2,1) x
// (1,2,1) over the 3x3 cells across d (a on the lower other axis, outer; b
// inner)
__device__ __forceinline__ double youngs(const double nb[3][3][3], int d)
{
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    double acc = 0.0;
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
            const double w = (double)((2 - abs(a)) * (2 - abs(b)));
            int up[3] = {0, 0, 0}, dn[3] = {0, 0, 0};
            up[t1] += a; up[t2] += b; up[d] += 1;
            dn[t1] += a; dn[t2] += b; dn[d] -= 1;
            acc += w * (nb[up[2] + 1][up[1] + 1][up[0] + 1] - nb[dn[2] + 1][dn[1] + 1][dn[0] + 1]);
        }
    return acc;
}

// Heights of the 9 columns of 7 cells along d; false when a column's ends
// are not one full and one empty cell, or orientations differ.  The 63 loads
// are issued before any test.
template <typename T>
__device__ __forceinline__ bool heights(const Grid<T> &g, const int p[3], int d, double z[3][3], int &orient)
{
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    double col[3][3][7];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                int q[3] = {p[0], p[1], p[2]};
                q[t1] += a - 1;
                q[t2] += b - 1;
                q[d] += k - 3;
                col[a][b][k] = g.at3(q);
            }
    orient = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            int o;
            if (col[a][b][0] == 1.0 && col[a][b][6] == 0.0) o = 1;
            else if (col[a][b][0] == 0.0 && col[a][b][6] == 1.0) o = -1;
            else return false;
            if (orient && o != orient) return false;
            orient = o;
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < 7; ++k) s += col[a][b][k];
            z[a][b] = o == 1 ? s - 3.5 : 3.5 - s;
        }
    return true;
}

__device__ __forceinline__ double kappa_of(const double z[3][3], int o, double h)
{
    const double za = (z[2][1] - z[0][1]) / 2.0;
    const double zb = (z[1][2] - z[1][0]) / 2.0;
    const double zaa = z[2][1] - 2.0 * z[1][1] + z[0][1];
    const double zbb = z[1][2] - 2.0 * z[1][1] + z[1][0];
    const double zab = (z[2][2] - z[2][0] - z[0][2] + z[0][0]) / 4.0;
    const double num = zaa * (1.0 + zb * zb) + zbb * (1.0 + za * za) - 2.0 * zab * za * zb;
    const double t = 1.0 + za * za + zb * zb;
    const double den = t * sqrt(t);
    return ((double)(-o) * num) / (den * h);
}

// pass 1 (streaming, few registers): every cell's status 0 and curvature 0,
// except the cells with 0 < C < 1, which are appended to a list (one atomic
// add per wave, positions by ballot prefix) for the dense passes
template <typename T>
__global__ __launch_bounds__(kCurvBlock) void k_curv_scan(const T *__restrict__ C, long N, T *__restrict__ kap,
                                                         uint8_t *__restrict__ status, uint32_t *__restrict__ list,
                                                         unsigned *__restrict__ count, long cap)
{
    __shared__ unsigned wcnt[kCurvBlock / 64];
    __shared__ unsigned base;
    const long q = (long)blockIdx.x * kCurvBlock + threadIdx.x;
    const bool in = q < N;
    const double c = in ? (double)C[q] : 0.0;
    const bool mixed = in && c > 0.0 && c < 1.0;
    if (in) {
        kap[q] = (T)0;
        status[q] = mixed ? KS_MISSING : KS_NONE;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long bal = __ballot(mixed);
    if (lane == 0) wcnt[wave] = (unsigned)__popcll(bal);
    __syncthreads();
    unsigned before = 0, tot = 0;
    for (int w = 0; w < kCurvBlock / 64; ++w) {
        before += w < wave ? wcnt[w] : 0u;
        tot += wcnt[w];
    }
    if (tot == 0) return;                      // uniform over the workgroup
    const int sub = (int)(blockIdx.x % kLists);
    if (threadIdx.x == 0) base = atomicAdd(&count[sub * kCtrStride], tot);
    __syncthreads();
    if (mixed) list[(long)sub * cap + base + before + (unsigned)__popcll(bal & ((1ull << lane) - 1ull))] = (uint32_t)q;
}

// The sub-lists taken as one range: pre[k] = cells in sub-lists before k
// (one workgroup of kLists threads scans the kLists counters in LDS), and
// cell i of the range lies in the last sub-list k with pre[k] <= i.
struct ListRange {
    uint32_t *pre;   // kLists + 1 entries in LDS
    __device__ __forceinline__ void build(const unsigned *__restrict__ count, uint32_t *wtot)
    {
        const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
        const uint32_t c = count[t * kCtrStride];
        uint32_t v = c;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t u = __shfl_up(v, off);
            if (lane >= off) v += u;
        }
        if (lane == 63) wtot[wave] = v;
        __syncthreads();
        uint32_t run = v - c;
        for (int w = 0; w < wave; ++w) run += wtot[w];
        pre[t] = run;
        if (t == kLists - 1) pre[kLists] = run + c;
        __syncthreads();
    }
    __device__ __forceinline__ uint32_t total() const { return pre[kLists]; }
    __device__ __forceinline__ long cell(const uint32_t *__restrict__ list, long cap, uint32_t i) const
    {
        int lo = 0, hi = kLists;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pre[mid] <= i) lo = mid;
            else hi = mid;
        }
        return (long)list[(long)lo * cap + (i - pre[lo])];
    }
};
static_assert(kCurvBlock == kLists, "one thread per sub-list counter in ListRange::build");

// Item i of the dense passes for this thread: the listed cells go in chunks
// of 64 (one wave), chunk c to wave c / G of workgroup c % G, so that a few
// tens of thousands of cells spread over every CU rather than filling the
// first workgroups (each lane gathers a 3x3x7 stencil: the texture units of
// the CUs that hold the cells are the limit).  A bijection of [0, 4 G 64).
__device__ __forceinline__ uint32_t dense_first()
{
    return (((uint32_t)threadIdx.x >> 6) * gridDim.x + blockIdx.x) * 64u + ((uint32_t)threadIdx.x & 63u);
}

// pass 2 (dense over the list, one lane per interfacial cell): height-function
// curvature (status 1 or 2); status 4 stays where no direction has 9 valid
// columns
template <typename T>
__global__ __launch_bounds__(kCurvBlock) void k_curv_hf(const T *__restrict__ C, int n, T *__restrict__ kap,
                                                       uint8_t *__restrict__ status, const uint32_t *__restrict__ list,
                                                       const unsigned *__restrict__ count, long cap)
{
    __shared__ uint32_t pre[kLists + 1], wtot[kCurvBlock / 64];
    ListRange lr{pre};
    lr.build(count, wtot);
    const Grid<T> g{C, n};
    const double h = 1.0 / (double)n;
    for (uint32_t i = dense_first(); i < lr.total(); i += gridDim.x * kCurvBlock) {
        const long q = lr.cell(list, cap, i);
        const int p[3] = {(int)(q % n), (int)((q / n) % n), (int)(q / ((long)n * n))};
        double gd[3];
        {
            double nb[3][3][3];
            block3(g, p, nb);
#pragma unroll
            for (int d = 0; d < 3; ++d) gd[d] = fabs(youngs(nb, d));
        }
        // candidate order: decreasing |g_d|, ties by lower axis
        int ord[3] = {0, 1, 2};
        for (int a = 1; a < 3; ++a)
            for (int b = a; b > 0 && gd[ord[b]] > gd[ord[b - 1]]; --b) {
                const int t = ord[b]; ord[b] = ord[b - 1]; ord[b - 1] = t;
            }
        for (int r = 0; r < 3; ++r) {
            double z[3][3];
            int o;
            if (!heights(g, p, ord[r], z, o)) continue;
            kap[q] = (T)kappa_of(z, o, h);
            status[q] = r == 0 ? KS_HF : KS_HF_OTHER;
            break;
        }
    }
}

// pass 3 (over the list): a cell without heights takes the mean curvature of
// its neighbours that have one (status 1 or 2, never changed by this pass),
// in [k][j][i] order
template <typename T>
__global__ __launch_bounds__(kCurvBlock) void k_curv_fill(int n, T *__restrict__ kap, uint8_t *__restrict__ status,
                                                         const uint32_t *__restrict__ list,
                                                         const unsigned *__restrict__ count, long cap)
{
    __shared__ uint32_t pre[kLists + 1], wtot[kCurvBlock / 64];
    ListRange lr{pre};
    lr.build(count, wtot);
    for (uint32_t i = dense_first(); i < lr.total(); i += gridDim.x * kCurvBlock) {
        const long q = lr.cell(list, cap, i);
        if (status[q] != KS_MISSING) continue;
        const int x = (int)(q % n), y = (int)((q / n) % n), z = (int)(q / ((long)n * n));
        // the 26 statuses in one round, then the curvatures of the valid
        // neighbours in another, summed in [dz][dy][dx] order
        long r[27];
        uint8_t t[27];
#pragma unroll
        for (int k = 0; k < 27; ++k) {
            const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
            r[k] = (long)wrapc(x + dx, n) + (long)n * ((long)wrapc(y + dy, n) + (long)n * (long)wrapc(z + dz, n));
        }
#pragma unroll
        for (int k = 0; k < 27; ++k) t[k] = k == 13 ? (uint8_t)KS_NONE : status[r[k]];
        double kv[27];
#pragma unroll
        for (int k = 0; k < 27; ++k) kv[k] = (t[k] == KS_HF || t[k] == KS_HF_OTHER) ? (double)kap[r[k]] : 0.0;
        double s = 0.0;
        int cnt = 0;
#pragma unroll
        for (int k = 0; k < 27; ++k)
            if (t[k] == KS_HF || t[k] == KS_HF_OTHER) {
                s += kv[k];
                ++cnt;
            }
        if (cnt) {
            kap[q] = (T)(s / (double)cnt);
            status[q] = KS_MEAN;
        }
    }
}

__global__ void k_curv_zero(unsigned *count)
{
    for (int k = threadIdx.x; k < kLists; k += blockDim.x) count[k * kCtrStride] = 0u;
}

// CSF force on the lower face of every cell along each axis
template <typename T>
__global__ __launch_bounds__(kCurvBlock) void k_csf(const T *__restrict__ C, const T *__restrict__ kap,
                                                   const uint8_t *__restrict__ status, int n, double sigma,
                                                   T *__restrict__ F0, T *__restrict__ F1, T *__restrict__ F2)
{
    const long N = (long)n * n * n;
    const long q = (long)blockIdx.x * kCurvBlock + threadIdx.x;
    if (q >= N) return;
    const int p[3] = {(int)(q % n), (int)((q / n) % n), (int)(q / ((long)n * n))};
    const long str[3] = {1, (long)n, (long)n * n};
    const double c = (double)C[q];
    const double k = (double)kap[q];
    const uint8_t sv = status[q];
    const bool v = sv >= KS_HF && sv <= KS_MEAN;
    const double h = 1.0 / (double)n;
    T *const F[3] = {F0, F1, F2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const long r = p[d] == 0 ? q + (long)(n - 1) * str[d] : q - str[d];
        const double cm = (double)C[r];
        double f = 0.0;
        if (cm != c) {
            const uint8_t sm = status[r];
            const bool vm = sm >= KS_HF && sm <= KS_MEAN;
            const double km = (double)kap[r];
            const double kf = (v && vm) ? (k + km) / 2.0 : (v ? k : (vm ? km : 0.0));
            f = ((sigma * kf) * (c - cm)) / h;
        }
        F[d][q] = (T)f;
    }
}

inline bool grid_ok(int n, int precision) { return n >= 8 && n <= 1024 && (precision == EBIT_FP64 || precision == EBIT_FP32); }

}  // namespace

extern "C" {

size_t ebit_curvature_work_bytes(int32_t n)
{
    if (n < 8 || n > 1024) return 0;
    const long N = (long)n * n * n;
    return (size_t)kLists * kCtrStride * sizeof(unsigned) + (size_t)kLists * list_cap(N) * sizeof(uint32_t);
}

int ebit_curvature(int32_t n, int32_t precision, const void *C, void *kappa, uint8_t *status, void *work,
                   size_t work_bytes, void *stream)
{
    if (!grid_ok(n, precision) || !C || !kappa || !status || !work || ((uintptr_t)work & 3)) return EBIT_EINVAL;
    if (work_bytes < ebit_curvature_work_bytes(n)) return EBIT_ESCRATCH;
    const long N = (long)n * n * n;
    const dim3 grid((unsigned)((N + kCurvBlock - 1) / kCurvBlock));
    const dim3 dense(kDenseBlocks);
    const long cap = list_cap(N);
    unsigned *count = (unsigned *)work;
    uint32_t *list = (uint32_t *)((char *)work + (size_t)kLists * kCtrStride * sizeof(unsigned));
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_curv_zero, dim3(1), dim3(256), 0, st, count);
    if (precision == EBIT_FP64) {
        hipLaunchKernelGGL(k_curv_scan<double>, grid, dim3(kCurvBlock), 0, st, (const double *)C, N, (double *)kappa,
                           status, list, count, cap);
        hipLaunchKernelGGL(k_curv_hf<double>, dense, dim3(kCurvBlock), 0, st, (const double *)C, n, (double *)kappa,
                           status, (const uint32_t *)list, (const unsigned *)count, cap);
        hipLaunchKernelGGL(k_curv_fill<double>, dense, dim3(kCurvBlock), 0, st, n, (double *)kappa, status,
                           (const uint32_t *)list, (const unsigned *)count, cap);
    } else {
        hipLaunchKernelGGL(k_curv_scan<float>, grid, dim3(kCurvBlock), 0, st, (const float *)C, N, (float *)kappa,
                           status, list, count, cap);
        hipLaunchKernelGGL(k_curv_hf<float>, dense, dim3(kCurvBlock), 0, st, (const float *)C, n, (float *)kappa,
                           status, (const uint32_t *)list, (const unsigned *)count, cap);
        hipLaunchKernelGGL(k_curv_fill<float>, dense, dim3(kCurvBlock), 0, st, n, (float *)kappa, status,
                           (const uint32_t *)list, (const unsigned *)count, cap);
    }
    return hipGetLastError() == hipSuccess ? EBIT_OK : EBIT_EHIP;
}

int ebit_csf(int32_t n, int32_t precision, const void *C, const void *kappa, const uint8_t *status, double sigma,
             void *const *F, void *stream)
{
    if (!grid_ok(n, precision) || !C || !kappa || !status || !F || !F[0] || !F[1] || !F[2]) return EBIT_EINVAL;
    const long N = (long)n * n * n;
    const dim3 grid((unsigned)((N + kCurvBlock - 1) / kCurvBlock));
    hipStream_t st = (hipStream_t)stream;
    if (precision == EBIT_FP64)
        hipLaunchKernelGGL(k_csf<double>, grid, dim3(kCurvBlock), 0, st, (const double *)C, (const double *)kappa,
                           status, n, sigma, (double *)F[0], (double *)F[1], (double *)F[2]);
    else
        hipLaunchKernelGGL(k_csf<float>, grid, dim3(kCurvBlock), 0, st, (const float *)C, (const float *)kappa,
                           status, n, sigma, (float *)F[0], (float *)F[1], (float *)F[2]);
    return hipGetLastError() == hipSuccess ? EBIT_OK : EBIT_EHIP;
}

}  // extern "C"
