// ebit.hip -- MI355X (gfx950) implementation of the EBIT hot path behind the
// C ABI of include/ebit.h: marker initialisation, the direction-split
// advection sweep and Front2VOF (Pan et al., arXiv 2509.26361, secs. 2.1-2.5,
// 3.1), plus a deterministic compensated volume reduction.
//
// Band.  Work is restricted to 4x4x4-node bricks near the interface.  Sweep t
// processes the bricks next to (26-neighbourhood) a brick that held a marker
// after sweep t-1, and the bricks that sweep t-1 found not quiet (it may have
// changed them): markers move at most one cell per sweep and every output
// depends only on markers within three cells, so outside the band the state
// is constant and the result equals a full-grid sweep; the second set keeps
// both state buffers equal outside the band.
//
// Lists.  Each sweep builds the band list of the next one: a brick holding a
// marker claims its 27 neighbours (an atomic exchange of a per-brick stamp
// decides the one claimant) and appends the new ones, wave-aggregated, to one
// of kSub sub-lists with a counter each (sub-list = wave id mod kSub), so no
// single address takes more than a few dozen appends per sweep (atomics on
// one address serialise).  A sub-list holds twice its fair share; a brick
// that finds it full goes to the list's overflow sub-list.  The same scheme
// builds the list of bricks that the next Front2VOF must revisit.
//
// Waves.  Both kernels run one 64-lane wave per workgroup over a fixed grid
// of nw waves; a fixed map deals the list items to the waves (balanced to one
// brick), runs of 16 consecutive items -- bricks appended together, hence
// neighbours -- to the waves of one XCD.
// A sweep wave stages each brick and a halo in LDS (one lane per node), writes
// the new colours, aligned markers and uniform face colours, and queues the
// work that needs the neighbourhood (new unaligned markers, colours of faces
// whose corners differ) in LDS; the queue is then run densely, one task per
// lane, by one code path for both planes (the plane axis is a run-time value).
// Front2VOF waves classify each brick's cells (full, empty, interfacial) and
// queue the interfacial ones, whose volumes are then computed one per lane.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/ebit.h"
#include "ebit_device.h"
#include "mlp_device.h"

using namespace ebit;

// occupancy targets (waves per SIMD) of the sweep and Front2VOF kernels
#ifndef EBIT_SWEEP_WAVES
#define EBIT_SWEEP_WAVES 3
#endif
#ifndef EBIT_F2V_WAVES
#define EBIT_F2V_WAVES 3
#endif

namespace {

constexpr int kRedBlocks = 1024;
#ifndef EBIT_SUBLISTS
#define EBIT_SUBLISTS 64
#endif
constexpr int kSub = EBIT_SUBLISTS;   // sub-lists per brick list (a power of two, at most 64)
constexpr int kNum = kSub + 1;    // lengths per list: the sub-lists, then the overflow
#ifndef EBIT_NUM_PAD
#define EBIT_NUM_PAD 16
#endif
constexpr int kPad = EBIT_NUM_PAD; // lengths are kPad words apart: atomics on one cache line serialise
#ifndef EBIT_MAX_WAVES
#define EBIT_MAX_WAVES 3072
#endif
constexpr int kMaxWaves = EBIT_MAX_WAVES;   // waves of the sweep / Front2VOF grids
#ifndef EBIT_TASK_CAP
#define EBIT_TASK_CAP 512
#endif
#ifndef EBIT_SLOT_CAP
#define EBIT_SLOT_CAP 256
#endif
constexpr int kTaskCap = EBIT_TASK_CAP;   // sweep: queued tasks per wave
constexpr int kSlotCap = EBIT_SLOT_CAP;   // sweep: queued face nodes per wave
constexpr int kCellCap = 192;     // Front2VOF: queued interfacial cells per wave
constexpr int kClaimCap = 16;     // sweep: queued bricks whose neighbours join the next lists
#ifndef EBIT_ORDER_MIN_N
#define EBIT_ORDER_MIN_N 512
#endif
#ifndef EBIT_SURR_WAVES
#define EBIT_SURR_WAVES 8
#endif
constexpr int kSurrWaves = EBIT_SURR_WAVES;   // waves per block of the surrogate pass (sharing the weights)
#ifndef EBIT_SURR_BLOCKS
#define EBIT_SURR_BLOCKS 256   // one block (weights and tiles in 124 KB of LDS) per CU, each looping over segments
#endif
// sweep: bricks staged together -- two on brick-ordered lists (large
// grids, many bricks per wave), one on claim-ordered lists (a few bricks per
// wave, where a second brick in the batch only lengthens the first's round)
#ifndef EBIT_BATCH
#define EBIT_BATCH 2
#endif
#ifndef EBIT_BATCH_SMALL
#define EBIT_BATCH_SMALL 1
#endif

// totals reduced from the per-wave counters
enum {
    ST_FALLBACK = 0, ST_MULTI, ST_CFL, ST_MERGED, ST_ACTIVE, ST_INTER_SUM /* sum of gen * delta */, ST_INTER, ST_AMB,
    ST_MARK0, ST_MARK1, ST_MARK2, ST_CMAX /* bits of the largest |Courant number| (float) */, ST_ANNIH, ST_SURR,
    ST_AFACE /* faces with four markers in the current state */, ST_COUNT = 16
};
// per-wave counters: cumulative over sweeps / Front2VOF calls, except the
// last-Front2VOF ones (CS_AMB, CS_SURR); CS_CMAX holds the bits of a non-negative float
// (ordered like the float) and is reduced by maximum
enum { CS_FALLBACK = 0, CS_MULTI, CS_CFL, CS_MERGED, CS_ACTIVE, CS_INTER_GEN, CS_INTER, CS_AMB, CS_CMAX, CS_ANNIH,
       CS_SURR, CS_COUNT };

struct Geo {
    int n;
    int nb1;        // bricks per axis
    long nn;        // n*n
    int nb;         // bricks
    int nw;         // waves of the sweep / Front2VOF grids
    long segcap;    // interfacial-cell segment length per wave
    int scap;       // entries per sub-list of a brick list
};

int waves_for(int n)
{
    const long nb = (long)(n / 4) * (n / 4) * (n / 4);
    const long w = nb < 64 ? 64 : (nb > kMaxWaves ? kMaxWaves : nb);
    return (int)(w & ~7L);      // a whole number of waves per XCD
}

// entries per sub-list of a brick list: twice the fair share of nb
int scap_for(int n)
{
    const int nb = (n / 4) * (n / 4) * (n / 4);
    return (2 * nb + kSub - 1) / kSub + 64;
}

// items per wave are at most ceil(nb / nw) + 2 under item_of()
long segcap_for(int n)
{
    const long nb = (long)(n / 4) * (n / 4) * (n / 4);
    const long nw = waves_for(n);
    return ((nb + nw - 1) / nw + 2) * 64;
}

constexpr int kOrderBlocks = 1024;   // workgroups of the band-ordering pass

// device work space carved out of the caller's scratch buffer
struct Work {
    uint32_t *cm;        // cm[b] == t <=> brick b is in the band list of sweep t (the last one it joined)
    uint32_t *fmark;     // fmark[b] == g <=> brick b is in the revisit list of Front2VOF generation g
    uint32_t *bcnt;      // interfacial cells of brick b at its last Front2VOF visit
    uint32_t *bchg;      // last sweep that changed brick b (see k_sweep)
    uint32_t *blist[4];  // band list of sweep t: blist[t % 4], kSub sub-lists of scap entries, overflow of nb
    uint32_t *bnum;      // [4][kNum] sub-list lengths, kPad words apart
    uint32_t *flist[3];  // revisit list of generation g: flist[g % 3]
    uint32_t *fnum;      // [3][kNum], kPad words apart
    uint32_t *ctask;     // per wave segcap interfacial cells of the last Front2VOF
    uint32_t *ccnt;      // [nw] their counts
    unsigned long long *cs;     // [CS_COUNT][nw] per-wave counters
    uint32_t *dcnt;      // [nw] surrogate-dataset rows per wave
    long long *doff;     // [nw] their offsets in the output
    unsigned long long *stat;   // ST_* totals
    double *part;        // 2 * kRedBlocks reduction partials
    double *epart;       // 6 * kRedBlocks partials of the error sums (ebit_errors), then the 6 totals
    ebit_mlp::MlpImage *simg;   // the surrogate's weights in the layout its kernel stages in LDS
    uint32_t *ocnt;      // [kOrderBlocks] band-ordering counts / offsets
    // rmask[buf][b]: the rows of brick b (16 rows of four nodes, y + 4 z) that
    // may hold a marker in state buffer buf, 16 bits per edge family x, y, z;
    // exact where a sweep over a brick-ordered list wrote the brick last, all
    // ones after ebit_init and where a sweep over a claim-ordered list did
    unsigned long long *rmask[2];
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t work_layout(int n, Work *w, char *base)
{
    const size_t nb = (size_t)(n / 4) * (n / 4) * (n / 4);
    const size_t nw = (size_t)waves_for(n);
    const size_t seg = (size_t)segcap_for(n);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return base ? base + o : nullptr; };
    char *p;
    p = take(nb * 4); if (w) w->cm = (uint32_t *)p;
    p = take(nb * 4); if (w) w->fmark = (uint32_t *)p;
    p = take(nb * 4); if (w) w->bcnt = (uint32_t *)p;
    p = take(nb * 4); if (w) w->bchg = (uint32_t *)p;
    const size_t lsz = ((size_t)kSub * scap_for(n) + nb) * 4;
    for (int k = 0; k < 4; ++k) { p = take(lsz); if (w) w->blist[k] = (uint32_t *)p; }
    p = take(4 * kNum * kPad * 4); if (w) w->bnum = (uint32_t *)p;
    for (int k = 0; k < 3; ++k) { p = take(lsz); if (w) w->flist[k] = (uint32_t *)p; }
    p = take(3 * kNum * kPad * 4); if (w) w->fnum = (uint32_t *)p;
    p = take(nw * seg * 4); if (w) w->ctask = (uint32_t *)p;
    p = take(nw * 4); if (w) w->ccnt = (uint32_t *)p;
    p = take(CS_COUNT * nw * 8); if (w) w->cs = (unsigned long long *)p;
    p = take(nw * 4); if (w) w->dcnt = (uint32_t *)p;
    p = take(nw * 8); if (w) w->doff = (long long *)p;
    p = take(ST_COUNT * sizeof(unsigned long long)); if (w) w->stat = (unsigned long long *)p;
    p = take(2 * kRedBlocks * sizeof(double)); if (w) w->part = (double *)p;
    p = take(6 * (kRedBlocks + 1) * sizeof(double)); if (w) w->epart = (double *)p;
    p = take(sizeof(ebit_mlp::MlpImage)); if (w) w->simg = (ebit_mlp::MlpImage *)p;
    p = take(kOrderBlocks * 4); if (w) w->ocnt = (uint32_t *)p;
    for (int k = 0; k < 2; ++k) { p = take(nb * 8); if (w) w->rmask[k] = (unsigned long long *)p; }
    return off;
}

// Bricks in lists are packed coordinates bx | by << 10 | bz << 20 (at most
// 256 bricks per axis); per-brick arrays are indexed by bx + nb1 (by + nb1 bz).
__device__ __forceinline__ uint32_t bpack(int bx, int by, int bz)
{
    return (uint32_t)bx | ((uint32_t)by << 10) | ((uint32_t)bz << 20);
}
__device__ __forceinline__ int bx_of(uint32_t p) { return (int)(p & 1023u); }
__device__ __forceinline__ int by_of(uint32_t p) { return (int)((p >> 10) & 1023u); }
__device__ __forceinline__ int bz_of(uint32_t p) { return (int)(p >> 20); }
__device__ __forceinline__ int blin(uint32_t p, int nb1) { return bx_of(p) + nb1 * (by_of(p) + nb1 * bz_of(p)); }
__device__ __forceinline__ uint32_t bpack_lin(int b, int nb1) { return bpack(b % nb1, (b / nb1) % nb1, b / (nb1 * nb1)); }
__device__ __forceinline__ uint32_t brick_shift(uint32_t p, int nb1, int dx, int dy, int dz)
{
    return bpack(wrp(bx_of(p) + dx, nb1), wrp(by_of(p) + dy, nb1), wrp(bz_of(p) + dz, nb1));
}

// the rows (four consecutive lanes each) of a ballot that hold a set bit, as
// 16 bits: bit r for lanes 4 r .. 4 r + 3
__device__ __forceinline__ uint32_t rows16(unsigned long long b)
{
    b |= b >> 1;
    b |= b >> 2;
    b &= 0x1111111111111111ull;        // bit 4 r: row r
    b = (b | (b >> 3)) & 0x0303030303030303ull;
    b = (b | (b >> 6)) & 0x000F000F000F000Full;
    b = (b | (b >> 12)) & 0x000000FF000000FFull;
    b = (b | (b >> 24)) & 0xFFFFull;
    return (uint32_t)b;
}

// sum of a per-lane value over the wave (result valid in every lane)
__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// inclusive prefix sum over the lanes of the wave
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t u = __shfl_up(v, off);
        if (lane >= off) v += u;
    }
    return v;
}

// Claims of list membership, batched per wave.  Two lists at once: the
// bricks of the 3x3x3 neighbourhoods of `na` source bricks and the `ns`
// bricks of srcS themselves join list A (membership markA[b] == vA), and the
// bricks at offsets (0 or -1 on each axis) of `nbr` source bricks join list B.  An atomic exchange of the mark decides
// the one claimant of each brick, which appends it, wave-aggregated, to
// sub-list `sub` of its list.  Up to four claims per lane are in flight.
struct ClaimList {
    uint32_t *mark;
    uint32_t v;
    uint32_t *list;
    uint32_t *num;
};

// brick b at position q of sub-list `sub`, or in the overflow sub-list when
// the sub-list is full
__device__ __forceinline__ void list_put(const ClaimList &L, uint32_t q, uint32_t b, int sub, uint32_t scap,
                                         uint32_t ocap)
{
    if (q < scap) {
        L.list[(size_t)sub * scap + q] = b;
        return;
    }
    const uint32_t o = atomicAdd(&L.num[kSub * kPad], 1u);
    if (o < ocap) L.list[(size_t)kSub * scap + o] = b;
}

// Claims: for each brick of srcA its 27-neighbourhood, restricted by its
// mask (NULL: none; bit d: the neighbour at offset (d % 3, d / 3 % 3, d / 9)
// - 1 is claimed), into list A; the bricks of srcS themselves into A; for
// each brick of srcB the bricks at offsets -(d & 1, d >> 1 & 1, d >> 2) for
// the bits d of its mask (NULL: all 8) into list B.
__device__ __forceinline__ void claim_two(const uint32_t *srcA, const uint32_t *maskA, int na, const uint32_t *srcS,
                                          int ns, const uint32_t *srcB, const uint8_t *maskB, int nbr, int nb1,
                                          ClaimList A, ClaimList B, int sub, uint32_t scap, uint32_t ocap)
{
    const int lane = threadIdx.x & 63;
    const int ta = na * 27 + ns, total = ta + nbr * 8;
    for (int base = 0; base < total; base += 256) {
        uint32_t nbk[4];
        bool take[4], inA[4], use[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = base + 64 * u + lane;
            take[u] = false;
            inA[u] = c < ta;
            use[u] = c < total;
            nbk[u] = 0;
            if (c < na * 27) {
                const uint32_t b = srcA[c / 27];
                const int d = c % 27;
                if (maskA && !((maskA[c / 27] >> d) & 1u)) use[u] = false;
                nbk[u] = brick_shift(b, nb1, d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1);
            } else if (c < ta) {
                nbk[u] = srcS[c - na * 27];
            } else if (c < total) {
                const uint32_t b = srcB[(c - ta) >> 3];
                const int d = (c - ta) & 7;
                if (maskB && !((maskB[(c - ta) >> 3] >> d) & 1)) use[u] = false;
                nbk[u] = brick_shift(b, nb1, -(d & 1), -((d >> 1) & 1), -(d >> 2));
            }
        }
        // the four exchanges are issued before any result is compared, so
        // that they are in flight together
        uint32_t old[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const ClaimList &L = inA[u] ? A : B;
            old[u] = L.v;
            if (use[u]) old[u] = atomicExch(&L.mark[blin(nbk[u], nb1)], L.v);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) take[u] = use[u] && old[u] != (inA[u] ? A.v : B.v);
        unsigned long long balA[4], balB[4];
        int cA = 0, cB = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            balA[u] = __ballot(take[u] && inA[u]);
            balB[u] = __ballot(take[u] && !inA[u]);
            cA += __popcll(balA[u]);
            cB += __popcll(balB[u]);
        }
        // lane 0 adds to A's counter and lane 1 to B's in one instruction
        // (one round trip; an add of zero leaves its counter as it is)
        uint32_t p = 0;
        if (lane < 2) p = atomicAdd(lane == 0 ? &A.num[sub * kPad] : &B.num[sub * kPad], (uint32_t)(lane == 0 ? cA : cB));
        uint32_t pA = __shfl(p, 0), pB = __shfl(p, 1);
        const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t qa = pA + (uint32_t)__popcll(balA[u] & lt), qb = pB + (uint32_t)__popcll(balB[u] & lt);
            if (take[u] && inA[u]) list_put(A, qa, nbk[u], sub, scap, ocap);
            if (take[u] && !inA[u]) list_put(B, qb, nbk[u], sub, scap, ocap);
            pA += (uint32_t)__popcll(balA[u]);
            pB += (uint32_t)__popcll(balB[u]);
        }
    }
}

// The i-th item of wave w (of nw, a multiple of 8).  Items go in chunks of
// kXcdChunk consecutive list entries -- bricks appended together, hence
// neighbours -- and chunk c to the waves of XCD c mod 8 (workgroup ids are
// dealt to the eight XCDs round robin), which take the XCD's items round
// robin: neighbouring bricks are processed near each other in time under one
// L2, which then serves the halos they share.  Increasing in i.
constexpr uint32_t kXcdChunk = 16;
__device__ __forceinline__ uint32_t item_of(uint32_t w, uint32_t i, uint32_t nw)
{
    const uint32_t x = w & 7u, nj = nw >> 3;
    const uint32_t idx = (w >> 3) + i * nj;
    return ((idx / kXcdChunk) * 8u + x) * kXcdChunk + idx % kXcdChunk;
}

// The items of wave w when the list is in brick order: XCD x takes the x-th
// eighth of the list, its waves equal consecutive runs of it, so that an XCD
// works on one region and a wave on neighbouring bricks, whose task stencils
// share cache lines.  Past the wave's run: ~0u.
struct Runs {
    uint32_t first, len;   // the wave's run: items first .. first + len - 1
    __device__ __forceinline__ void init(uint32_t w, uint32_t nw, uint32_t total)
    {
        const uint32_t x = w & 7u, j = w >> 3, nj = nw >> 3;
        const uint32_t cx = __builtin_amdgcn_readfirstlane((total + 7u) / 8u);
        const uint32_t cw = __builtin_amdgcn_readfirstlane((cx + nj - 1u) / nj);
        const uint32_t r0 = min(j * cw, cx), r1 = min(r0 + cw, cx);
        first = x * cx + r0;
        len = r1 - r0;
    }
    __device__ __forceinline__ uint32_t item(uint32_t i) const { return i < len ? first + i : ~0u; }
};

// Items of a grid: the entries of a list, its kSub sub-lists and then its
// overflow sub-list.  The inclusive prefix sums of the sub-list lengths are
// kept in LDS (pre[0..kSub)).
struct Items {
    uint32_t s0;            // items in the sub-lists
    uint32_t total;         // all items
    const uint32_t *l0;
    const uint32_t *pre;
    uint32_t scap;
    __device__ __forceinline__ void init(uint32_t *lds, const uint32_t *num0, const uint32_t *list0, uint32_t scap_,
                                         uint32_t ocap)
    {
        const int lane = threadIdx.x & 63;
        const uint32_t inc0 = wave_incl_scan(lane < kSub ? min(num0[lane * kPad], scap_) : 0u);
        if (lane < kSub) lds[lane] = inc0;
        s0 = __shfl(inc0, kSub - 1);
        total = s0 + min(num0[kSub * kPad], ocap);
        l0 = list0;
        pre = lds;
        scap = scap_;
        __syncthreads();
    }
    // brick of item k < total, a different k per lane
    __device__ __forceinline__ int brick_lane(uint32_t k) const
    {
        if (k >= s0) return (int)l0[(size_t)kSub * scap + (k - s0)];   // overflow sub-list
        // j = the sub-lists that end at or before k (binary search)
        int j = 0;
#pragma unroll
        for (int st = kSub / 2; st >= 1; st >>= 1)
            if (pre[j + st - 1] <= k) j += st;
        const uint32_t excl = j > 0 ? pre[j - 1] : 0u;
        return (int)l0[(size_t)j * scap + (k - excl)];
    }
};

// ---------------------------------------------------------------------------
// a0: initialisation (sec. 3.1)
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_init(Geo g, const double *__restrict__ phi, const double *__restrict__ pf0,
                                              const double *__restrict__ pf1, const double *__restrict__ pf2,
                                              const double *__restrict__ se0, const double *__restrict__ se1,
                                              const double *__restrict__ se2, uint8_t *__restrict__ fl, T *__restrict__ s0,
                                              T *__restrict__ s1, T *__restrict__ s2)
{
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long N = g.nn * g.n;
    if (q >= N) return;
    int n = g.n;
    int x = (int)(q % n), y = (int)((q / n) % n), z = (int)(q / g.nn);
    auto at = [&](int dx, int dy, int dz) -> long {
        return (long)wrp(x + dx, n) + (long)n * wrp(y + dy, n) + g.nn * wrp(z + dz, n);
    };
    const double *pf[3] = {pf0, pf1, pf2};
    const double *se[3] = {se0, se1, se2};
    T *s[3] = {s0, s1, s2};
    double p0 = phi[q];
    int c0 = p0 > 0.0;
    // colours at p + {e_x, e_y, e_z, e_x+e_y, e_y+e_z, e_x+e_z}
    int cx = phi[at(1, 0, 0)] > 0.0, cy = phi[at(0, 1, 0)] > 0.0, cz = phi[at(0, 0, 1)] > 0.0;
    int cxy = phi[at(1, 1, 0)] > 0.0, cyz = phi[at(0, 1, 1)] > 0.0, cxz = phi[at(1, 0, 1)] > 0.0;
    int ce[3] = {cx, cy, cz};
    uint8_t out = (uint8_t)c0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        T v = T(0);
        if (ce[e] != c0) {
            long qb = e == 0 ? at(1, 0, 0) : (e == 1 ? at(0, 1, 0) : at(0, 0, 1));
            double sv = se[e] ? se[e][q] : p0 / (p0 - phi[qb]);
            v = clamp_frac<T>((T)sv);
            out |= (uint8_t)(1u << (4 + e));
        }
        s[e][q] = v;
    }
    // a face with normal a has edges along b, c at p and along b at p+e_c, along c at p+e_b
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int b = (a + 1) % 3, c = (a + 2) % 3;
        int cb = ce[b], cc = ce[c];
        int cbc = (b == 0 && c == 1) || (b == 1 && c == 0) ? cxy : ((b == 1 && c == 2) || (b == 2 && c == 1) ? cyz : cxz);
        bool any = (c0 != cb) || (c0 != cc) || (cb != cbc) || (cc != cbc);
        int col = any ? (pf[a][q] > 0.0) : c0;
        out |= (uint8_t)(col << (1 + a));
    }
    fl[q] = out;
}

// Band list of the first sweep (t = 2; stamps start at 0) of a freshly
// initialised (or caller-filled) state: the bricks next to a brick holding a
// marker.
__global__ __launch_bounds__(64) void k_init_band(Geo g, const uint8_t *__restrict__ fl, Work w)
{
    const int lane = threadIdx.x;
    for (int b = blockIdx.x; b < g.nb; b += gridDim.x) {
        int bx = b % g.nb1, by = (b / g.nb1) % g.nb1, bz = b / (g.nb1 * g.nb1);
        int x = bx * 4 + (lane & 3), y = by * 4 + ((lane >> 2) & 3), z = bz * 4 + (lane >> 4);
        long q = x + (long)g.n * y + g.nn * z;
        const bool hasm = __ballot((fl[q] & 0x70) != 0) != 0;
        if (hasm) {
            const ClaimList A{w.cm, 2u, w.blist[2], w.bnum + 2 * kNum * kPad};
            const uint32_t bp = bpack(bx, by, bz);
            claim_two(&bp, nullptr, 1, nullptr, 0, nullptr, nullptr, 0, g.nb1, A, A, blockIdx.x % kSub,
                      (uint32_t)g.scap, (uint32_t)g.nb);
        }
    }
}

// A brick list rewritten in brick order (bx fastest, then by, bz): the
// bricks whose stamp equals `val` (the band list of sweep t: cm == t; the
// revisit list of Front2VOF generation g: fmark == g), all in the overflow
// sub-list, the kSub sub-lists emptied.  Consecutive items are then
// neighbouring bricks, which the item schedule hands to one XCD in runs of
// kXcdChunk, so the 128-byte lines a run's brick rows share (four bricks per
// line of a fraction array) and its halos are fetched into that XCD's L2
// once.  Three passes: counts per block of `per` bricks, their exclusive
// scan, the writes.
struct OrderArgs {
    const uint32_t *stamp;
    uint32_t val;
    uint32_t *out;        // the list's overflow sub-list
    uint32_t *num;        // the list's kNum lengths, kPad words apart
    uint32_t *cnt;        // [kOrderBlocks]
    uint32_t nb, per;
    int nb1;
};

__global__ __launch_bounds__(256) void k_order_count(OrderArgs o)
{
    __shared__ uint32_t ws[4];
    const uint32_t b0 = blockIdx.x * o.per, b1 = min(b0 + o.per, o.nb);
    int c = 0;
    for (uint32_t b = b0 + threadIdx.x; b < b1; b += 256) c += o.stamp[b] == o.val ? 1 : 0;
    c = wave_sum(c);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = (uint32_t)c;
    __syncthreads();
    if (threadIdx.x == 0) o.cnt[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ __launch_bounds__(1024) void k_order_scan(OrderArgs o, int nblk)
{
    __shared__ uint32_t sc[1024];
    const int i = threadIdx.x;
    const uint32_t v = i < nblk ? o.cnt[i] : 0u;
    sc[i] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t add = i >= off ? sc[i - off] : 0u;
        __syncthreads();
        sc[i] += add;
        __syncthreads();
    }
    if (i < nblk) o.cnt[i] = sc[i] - v;
    if (i < kSub) o.num[i * kPad] = 0;
    if (i == 1023) o.num[kSub * kPad] = sc[1023];
}

__global__ __launch_bounds__(256) void k_order_write(OrderArgs o)
{
    __shared__ uint32_t ws[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t b0 = blockIdx.x * o.per, b1 = min(b0 + o.per, o.nb);
    uint32_t pos = o.cnt[blockIdx.x];
    for (uint32_t c0 = b0; c0 < b1; c0 += 256) {
        const uint32_t b = c0 + threadIdx.x;
        const bool m = b < b1 && o.stamp[b] == o.val;
        const unsigned long long bal = __ballot(m);
        if (lane == 0) ws[wave] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t before = 0;
        for (int k = 0; k < wave; ++k) before += ws[k];
        if (m) o.out[pos + before + __popcll(bal & ((1ull << lane) - 1ull))] = bpack_lin((int)b, o.nb1);
        pos += ws[0] + ws[1] + ws[2] + ws[3];
        __syncthreads();
    }
}

// zero the stamps, list lengths and counters
__global__ void k_zero_work(Work w, Geo g)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < g.nb) {
        w.cm[i] = 0;
        w.fmark[i] = 0;
        w.bcnt[i] = 0;
        w.bchg[i] = 0;
        w.rmask[0][i] = ~0ull;
        w.rmask[1][i] = ~0ull;
    }
    if (i < 4 * kNum) w.bnum[i * kPad] = 0;
    if (i < 3 * kNum) w.fnum[i * kPad] = 0;
    if (i < g.nw) {
        w.ccnt[i] = 0;
        for (int k = 0; k < CS_COUNT; ++k) w.cs[k * g.nw + i] = 0;
    }
    if (i < ST_COUNT) w.stat[i] = 0;
}

// every row of every brick may hold a marker, in both buffers (Work::rmask)
__global__ __launch_bounds__(256) void k_rmask_ones(Work w, Geo g)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < g.nb; i += (long)gridDim.x * blockDim.x) {
        w.rmask[0][i] = ~0ull;
        w.rmask[1][i] = ~0ull;
    }
}

// ---------------------------------------------------------------------------
// a1-a4: one sweep along axis D (secs. 2.1-2.4)
// ---------------------------------------------------------------------------

template <typename T>
struct SweepArgs {
    Geo g;
    const uint8_t *fl;
    const T *s[3];
    uint8_t *flo;
    T *so[3];
    unsigned long long *rmo;   // row masks of the buffer written (Work::rmask)
    const T *U;
    T c;              // (dt n) g
    Work w;
    uint32_t t;       // sweep sequence number (>= 2)
    uint32_t fgen;    // generation of the next Front2VOF
    int full;         // process every brick
    int run;          // the list is in brick order: waves take runs of it (Runs)
    int nd;           // axis of the next sweep when known (ebit_advance), else -1
};

// Brick tile: flags and advected coordinate of the D-edge markers of the
// brick's nodes and their neighbours at offsets -1..+1 along D and +1 across,
// indexed iD + kAD (i1 + kAA i2), (iD, i1, i2) = offsets (+1, 0, 0) along (D, A1, A2).
constexpr int kAD = 6, kAA = 5, kATile = kAD * kAA * kAA;

// The queued tasks of a sweep wave, one per lane: a node whose face in the
// plane (D, A1) (type bit 0 clear) or (D, A2) has differing corners -- that
// face's colour, and with type bit 1 the circle-fit placement of the node's
// new marker on the edge across (whose end colours differ, so the face's
// corners do too); bit 2 is the node's new colour.  Face colours are gathered
// per node in the slot table and the node's flags byte is written once.  RUN
// (large grids, ordered lists): the tasks' first load round reads only the
// entries of existing markers -- fewer cache lines where the traffic bounds
// the sweep, at the price of registers that the small grids' latency-bound
// sweep is better without.
template <typename T, int D, int RUN>
__device__ __forceinline__ void run_tasks(const SweepArgs<T> &a, const uint32_t *tq, const uint8_t *tt,
                                          const uint16_t *ts, int ntask, const uint32_t *sq, uint32_t *sb,
                                          int nslot, int &fbt, int &multit)
{
    constexpr int A1 = (D + 1) % 3, A2 = (D + 2) % 3;
    const int lane = threadIdx.x;
    const int n = a.g.n;
    const long nn = a.g.nn;
    const long str[3] = {1, (long)n, nn};
    for (int base = 0; base < ntask; base += 64) {
        const int i = base + lane;
        if (i < ntask) {
            const uint32_t pk = tq[i];
            const int ty = tt[i];
            const bool second = ty & 1;             // plane (D, A2)
            const int unal = (ty >> 1) & 1, c00 = (ty >> 2) & 1;
            const int P[3] = {(int)(pk & 1023u), (int)((pk >> 10) & 1023u), (int)(pk >> 20)};
            const uint32_t q = (uint32_t)P[0] + __umul24((uint32_t)P[1], (uint32_t)n) + __umul24((uint32_t)P[2], (uint32_t)nn);
            PlaneTask<T, D, RUN> p;
            p.fl = a.fl;
            p.sD = a.s[D];
            p.sA = second ? a.s[A2] : a.s[A1];
            p.U = a.U;
            p.c = a.c;
            p.n = n;
            p.ci = P[D];
            p.cj = second ? P[A2] : P[A1];
            p.strD = (uint32_t)str[D];
            p.strA = (uint32_t)(second ? str[A2] : str[A1]);
            p.base = second ? __umul24((uint32_t)P[A1], (uint32_t)str[A1]) : __umul24((uint32_t)P[A2], (uint32_t)str[A2]);
            p.hb = 4 + D;
            p.vb = second ? 4 + A2 : 4 + A1;
            p.fb = second ? 1 + A1 : 1 + A2;
            p.fetch_flags();
            T sv = T(0);
            const int par = p.run(unal, c00, sv, fbt, multit);
            if (unal) (second ? a.so[A2] : a.so[A1])[q] = sv;
            if (par) atomicOr(&sb[ts[i]], 1u << p.fb);
        }
    }
    __syncthreads();
    for (int s = lane; s < nslot; s += 64) a.flo[sq[s]] = (uint8_t)sb[s];
    __syncthreads();
}

// One sweep: wave w takes the items w, w + nw, ... of the sweep's band list.  Per brick, one
// lane per node: new node colours (one flip per aligned marker crossing a
// node, Fig. 4), the aligned markers (land on the edge they reach, pairs
// annihilate, Fig. 5a), which edges carry a marker afterwards (one marker iff
// the end colours differ, sec. 2.2), the colour of faces with uniform
// corners; the rest is queued.  The bricks next to a brick holding markers
// join the next sweep's list; bricks whose cells change join the next
// Front2VOF's list.
template <typename T, int D, int RUN>
__device__ __forceinline__ void sweep_wave(const SweepArgs<T> &a, const int wv, const int nw)
{
    constexpr int A1 = (D + 1) % 3, A2 = (D + 2) % 3;
    constexpr int kBatch = RUN ? EBIT_BATCH : EBIT_BATCH_SMALL;
    __shared__ uint8_t tfl[kBatch][kATile];
    __shared__ double txd[kBatch][kATile];
    __shared__ uint32_t tq[kTaskCap];
    __shared__ uint8_t tt[kTaskCap];
    __shared__ uint16_t ts[kTaskCap];
    __shared__ uint32_t sq[kSlotCap], sb[kSlotCap];
    __shared__ uint32_t mbr[kClaimCap], cbr[kClaimCap], sbr[kClaimCap];
    __shared__ uint32_t mmk[kClaimCap];
    __shared__ uint8_t cmk[kClaimCap];
    __shared__ uint32_t ipre[kSub];
    const int lane = threadIdx.x;
    const int n = a.g.n, nb1 = a.g.nb1, nb = a.g.nb;
    const uint32_t t = a.t;
    uint32_t *cm_next = a.w.cm;
    const int sub = wv % kSub;
    uint32_t *lnext = a.w.blist[(t + 1) % 4], *nnext = a.w.bnum + ((t + 1) % 4) * kNum * kPad;
    uint32_t *lrev = a.w.flist[a.fgen % 3], *nrev = a.w.fnum + (a.fgen % 3) * kNum * kPad;
    if (wv == 0)   // sweep t+2's list starts empty
        for (int i = lane; i < kNum; i += 64) a.w.bnum[(((t + 2) % 4) * kNum + i) * kPad] = 0;
    const long str[3] = {1, (long)n, a.g.nn};
    const int lu[3] = {lane & 3, (lane >> 2) & 3, lane >> 4};
    const int tself = (lu[D] + 1) + kAD * (lu[A1] + kAA * lu[A2]);
    int ext[3], lo[3];
    ext[D] = kAD; ext[A1] = kAA; ext[A2] = kAA;
    lo[D] = -1; lo[A1] = 0; lo[A2] = 0;

    // tile coordinates of the lane's staging entries kk = lane + 64 r (lane constants),
    // packed: offset along x | y << 4 | z << 8 | LDS index << 12
    constexpr int kR = (kATile + 63) / 64;
    uint32_t tpk[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int kk = lane + 64 * r;
        const int kc = kk < kATile ? kk : kATile - 1;
        const int kt[3] = {kc % ext[0], (kc / ext[0]) % ext[1], kc / (ext[0] * ext[1])};
        const int ti = kt[D] + kAD * (kt[A1] + kAA * kt[A2]);
        tpk[r] = (uint32_t)(kt[0] | (kt[1] << 4) | (kt[2] << 8) | (ti << 12));
    }
    const uint32_t un = (uint32_t)n, unn = (uint32_t)a.g.nn;
    auto tnode = [&](const int org[3], uint32_t pk, int &gpd) -> uint32_t {
        int gp[3];
#pragma unroll
        for (int e = 0; e < 3; ++e) gp[e] = wrp(org[e] + lo[e] + (int)((pk >> (4 * e)) & 15u), n);
        gpd = gp[D];
        return (uint32_t)gp[0] + __umul24((uint32_t)gp[1], un) + __umul24((uint32_t)gp[2], unn);
    };
    Items it;
    if (a.full) {
        it.total = (uint32_t)nb;
    } else {
        it.init(ipre, a.w.bnum + (t % 4) * kNum * kPad, a.w.blist[t % 4], (uint32_t)a.g.scap, (uint32_t)nb);
    }
    int ntask = 0, nslot = 0, nact = 0, nm = 0, nc = 0, ns = 0;
    int fbc = 0, cflc = 0, mergedc = 0, fbt = 0, multit = 0;
    float cmax = 0.f;   // largest |displacement| of a marker this wave owns, in cells
    auto claims = [&]() {
        __syncthreads();
        claim_two(mbr, mmk, nm, sbr, ns, cbr, cmk, nc, nb1, ClaimList{cm_next, t + 1, lnext, nnext},
                  ClaimList{a.w.fmark, a.fgen, lrev, nrev}, sub, (uint32_t)a.g.scap, (uint32_t)nb);
        __syncthreads();
        nm = 0;
        nc = 0;
        ns = 0;
    };
    // this wave's items item_of(wv, i), resolved one per lane (a static
    // schedule: a shared counter handing out items cost more than the
    // imbalance it removes)
    // RUN (the list is in brick order): the wave's run of the list; else item_of
    Runs ru;
    if (RUN) ru.init((uint32_t)wv, (uint32_t)nw, it.total);
    auto item = [&](uint32_t i) { return RUN ? ru.item(i) : item_of((uint32_t)wv, i, (uint32_t)nw); };
    for (uint32_t i0 = 0; item(i0) < it.total; i0 += 64) {
        int bl = -1;
        {
            const uint32_t k = item(i0 + (uint32_t)lane);
            const bool have = k < it.total;
            // packed brick coordinates (-1: none)
            int bb = a.full ? (have ? (int)bpack_lin((int)k, nb1) : -1) : it.brick_lane(have ? k : 0);
            if (!have || bb < 0 || bx_of((uint32_t)bb) >= nb1 || by_of((uint32_t)bb) >= nb1 || bz_of((uint32_t)bb) >= nb1)
                bb = -1;
            bl = bb;
        }
        unsigned long long pend = __ballot(bl >= 0);
        while (pend) {
            // a batch of up to kBatch bricks, staged together: all flag loads,
            // then all marker loads (D-edge markers of the tiles, and the
            // unaligned markers stored at the lane's own nodes, for the Courant
            // check), then the Euler step (eq. Eq_marker_dis) into the tiles
            int bb[kBatch];
            int nbat = 0;
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
                bb[j] = -1;
                if (pend) {
                    const int src = __ffsll((long long)pend) - 1;
                    pend &= pend - 1;
                    bb[j] = __builtin_amdgcn_readfirstlane(__shfl(bl, src));
                    ++nbat;
                }
            }
            if (nm + kBatch > kClaimCap || nc + kBatch > kClaimCap || ns + kBatch > kClaimCap) claims();
            int cfl = 0;
            uint8_t fr[kBatch][kR], fown[kBatch];
            uint32_t lastchg[kBatch];
            bool quiet[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
                fown[j] = 0;
                lastchg[j] = 0;
#pragma unroll
                for (int r = 0; r < kR; ++r) fr[j][r] = 0;
                if (j >= nbat) continue;
                const int b = bb[j];
                const int org[3] = {bx_of((uint32_t)b) * 4, by_of((uint32_t)b) * 4, bz_of((uint32_t)b) * 4};
                fown[j] = a.fl[(uint32_t)(org[0] + lu[0]) + __umul24((uint32_t)(org[1] + lu[1]), un) +
                               __umul24((uint32_t)(org[2] + lu[2]), unn)];
#pragma unroll
                for (int r = 0; r < kR; ++r) {
                    int gpd;
                    fr[j][r] = a.fl[tnode(org, tpk[r], gpd)];
                }
                lastchg[j] = a.w.bchg[blin((uint32_t)b, nb1)];
            }
            // A brick whose tile (halo included) holds no marker, and whose
            // faces containing D already carry their nodes' colour, is left
            // unchanged by the sweep (a consistent state has uniform colours
            // there; only faces normal to D may keep another colour); if it
            // was also unchanged by the previous sweep, both buffers already
            // hold it and it needs no work at all.
            bool skip[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
                bool anym = false;
#pragma unroll
                for (int r = 0; r < kR; ++r) {
                    const uint32_t f = fr[j][r];
                    anym |= (f & 0x70) != 0 || (((f >> (1 + A1)) ^ f) & 1) != 0 || (((f >> (1 + A2)) ^ f) & 1) != 0;
                }
                quiet[j] = j < nbat && __ballot(anym) == 0;
                skip[j] = quiet[j] && !a.full && lastchg[j] + 2 <= t;
            }
            T sD[kBatch][kR], U0[kBatch][kR], UD[kBatch][kR];
            T sAo[kBatch][2], UAo[kBatch][2], Uown[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
#pragma unroll
                for (int r = 0; r < kR; ++r) sD[j][r] = U0[j][r] = UD[j][r] = T(0);
                sAo[j][0] = sAo[j][1] = UAo[j][0] = UAo[j][1] = Uown[j] = T(0);
                if (j >= nbat) continue;
                const int b = bb[j];
                const int org[3] = {bx_of((uint32_t)b) * 4, by_of((uint32_t)b) * 4, bz_of((uint32_t)b) * 4};
#pragma unroll
                for (int r = 0; r < kR; ++r) {
                    if ((fr[j][r] >> (4 + D)) & 1) {
                        int gpd;
                        const uint32_t q = tnode(org, tpk[r], gpd);
                        sD[j][r] = a.s[D][q];
                        U0[j][r] = a.U[q];
                        UD[j][r] = a.U[gpd + 1 == n ? q - (uint32_t)(n - 1) * (uint32_t)str[D] : q + (uint32_t)str[D]];
                    }
                }
                const long qs = (long)(org[0] + lu[0]) + str[1] * (org[1] + lu[1]) + str[2] * (org[2] + lu[2]);
                if (fown[j] & ((1u << (4 + A1)) | (1u << (4 + A2)))) Uown[j] = a.U[qs];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int A = e == 0 ? A1 : A2;
                    if ((fown[j] >> (4 + A)) & 1) {
                        const long q1 = org[A] + lu[A] + 1 == n ? qs - (long)(n - 1) * str[A] : qs + str[A];
                        sAo[j][e] = a.s[A][qs];
                        UAo[j][e] = a.U[q1];
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
                if (j >= nbat) continue;
#pragma unroll
                for (int r = 0; r < kR; ++r) {
                    const int kk = lane + 64 * r;
                    if (kk >= kATile) continue;
                    const int kt[3] = {(int)(tpk[r] & 15u), (int)((tpk[r] >> 4) & 15u), (int)((tpk[r] >> 8) & 15u)};
                    const int ti = (int)(tpk[r] >> 12);
                    double xd = 0.0;
                    if ((fr[j][r] >> (4 + D)) & 1) {
                        T u = U0[j][r] + sD[j][r] * (UD[j][r] - U0[j][r]);
                        T del = a.c * u;
                        xd = (double)sD[j][r] + (double)del;
                        const bool own = kt[D] >= 1 && kt[D] < 5 && kt[A1] < 4 && kt[A2] < 4;
                        if (own && fabs((double)del) > 1.0) ++cfl;
                        if (own) cmax = fmaxf(cmax, fabsf((float)del));
                    }
                    tfl[j][ti] = fr[j][r];
                    txd[j][ti] = xd;
                }
                // Courant check of the unaligned markers stored at this node
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int A = e == 0 ? A1 : A2;
                    if ((fown[j] >> (4 + A)) & 1) {
                        T del = a.c * (Uown[j] + sAo[j][e] * (UAo[j][e] - Uown[j]));
                        if (fabs((double)del) > 1.0) ++cfl;
                        cmax = fmaxf(cmax, fabsf((float)del));
                    }
                }
            }
            __syncthreads();
            // new colours of the tile nodes whose D-predecessor is in the tile
            for (int kk = lane; kk < nbat * kATile; kk += 64) {
                const int j = kk / kATile, k0 = kk - j * kATile;
                if (k0 % kAD == 0) continue;
                uint8_t f = tfl[j][k0], fm = tfl[j][k0 - 1];
                int c = f & 1;
                if (((fm >> (4 + D)) & 1) && txd[j][k0 - 1] >= 1.0) c ^= 1;
                if (((f >> (4 + D)) & 1) && txd[j][k0] < 0.0) c ^= 1;
                tfl[j][k0] = (uint8_t)((f & 0x7f) | (c << 7));
            }
            __syncthreads();
            for (int j = 0; j < nbat; ++j) {
            int b = bb[0];
            bool skipj = skip[0];
            uint32_t lastj = lastchg[0];
#pragma unroll
            for (int u = 1; u < kBatch; ++u)
                if (j == u) { b = bb[u]; skipj = skip[u]; lastj = lastchg[u]; }
            if (skipj) continue;
            if (ntask + 2 * 64 > kTaskCap || nslot + 64 > kSlotCap) {
                run_tasks<T, D, RUN>(a, tq, tt, ts, ntask, sq, sb, nslot, fbt, multit);
                ntask = 0;
                nslot = 0;
            }
            ++nact;
            const int org[3] = {bx_of((uint32_t)b) * 4, by_of((uint32_t)b) * 4, bz_of((uint32_t)b) * 4};
            const long qs = (long)(org[0] + lu[0]) + str[1] * (org[1] + lu[1]) + str[2] * (org[2] + lu[2]);
            // RUN: the rows of the brick that may hold markers in the buffer
            // this sweep writes (loaded here, used by the stores below)
            const unsigned long long om = RUN ? a.rmo[blin((uint32_t)b, nb1)] : 0ull;
            const uint8_t *tf = tfl[j];
            const double *tx = txd[j];
            auto ncol = [&](int di, int d1, int d2) { return (tf[tself + di + kAD * (d1 + kAA * d2)] >> 7) & 1; };
            const uint8_t fself = tf[tself];
            const int c00 = ncol(0, 0, 0), c10 = ncol(1, 0, 0);
            uint8_t out = (uint8_t)c00;
            T sdn = T(0);
            int fb = 0, merged = 0;
            {
                uint8_t fm = tf[tself - 1], fp = tf[tself + 1];
                bool hm = (fm >> (4 + D)) & 1, h0 = (fself >> (4 + D)) & 1, hp = (fp >> (4 + D)) & 1;
                double xm = tx[tself - 1], x0 = tx[tself], xp = tx[tself + 1];
                bool lm = hm && xm >= 1.0, l0 = h0 && x0 >= 0.0 && x0 < 1.0, lp = hp && xp < 0.0;
                int kl = (int)lm + (int)l0 + (int)lp;
                if (c00 != c10) {
                    double v;
                    if (kl == 1) v = lm ? xm - 1.0 : (l0 ? x0 : xp + 1.0);
                    else if (kl == 3) {
                        double v0 = xm - 1.0, v1 = x0, v2 = xp + 1.0;
                        double lo2 = v0 < v1 ? v0 : v1, hi = v0 < v1 ? v1 : v0;
                        v = v2 < lo2 ? lo2 : (v2 > hi ? hi : v2);
                        merged += 1;
                    } else {
                        v = 0.5;
                        fb += 1;
                    }
                    sdn = clamp_frac<T>((T)v);
                    out |= (uint8_t)(1u << (4 + D));
                } else if (kl >= 2) {
                    merged += 1 + (1 << 16);   // an annihilated pair: counted in the upper half too
                }
            }
            out |= (uint8_t)(fself & (1u << (1 + D)));   // faces normal to D keep their colour
            bool task[4];
            {
                const int c01 = ncol(0, 1, 0), c11 = ncol(1, 1, 0);   // plane (D, A1)
                task[0] = c00 != c01;
                task[2] = !(c00 == c10 && c00 == c01 && c00 == c11);
                if (task[0]) out |= (uint8_t)(1u << (4 + A1));
                if (!task[2]) out |= (uint8_t)(c00 << (1 + A2));
            }
            {
                const int c01 = ncol(0, 0, 1), c11 = ncol(1, 0, 1);   // plane (D, A2)
                task[1] = c00 != c01;
                task[3] = !(c00 == c10 && c00 == c01 && c00 == c11);
                if (task[1]) out |= (uint8_t)(1u << (4 + A2));
                if (!task[3]) out |= (uint8_t)(c00 << (1 + A1));
            }
            const bool fnode = task[2] || task[3];
            const unsigned long long mbal = __ballot((out & 0x70) != 0);           // nodes with markers
            const unsigned long long cbal = __ballot(((out ^ fself) & 0x71) != 0); // colour / marker changed
            const bool hasm = mbal != 0, chg = cbal != 0;
            // unchanged by this sweep: no marker and no face task in the brick,
            // flags as before (its fractions are 0 then, before and after);
            // bchg records the last sweep that changed the brick
            const bool same = !hasm && __ballot(fnode) == 0 && __ballot(((out ^ fself) & 0x7f) != 0) == 0;
            if (!same && lane == 0) a.w.bchg[blin((uint32_t)b, nb1)] = t;
            // unchanged now and by the previous sweep: both buffers hold it already
            if (!(same && !a.full && lastj + 2 <= t)) {
                if (RUN) {
                    // a row of fractions (four lanes, 32 or 16 bytes) is written
                    // only if one of its edges holds a marker now or may hold one
                    // in the buffer written (elsewhere that buffer already holds
                    // the zeros); whole rows, so that no store covers part of a
                    // row.  This saves HBM writes on large bands; on small grids,
                    // bound by the waves' chains of rounds, the plain stores
                    // below are faster.
                    const unsigned long long nm =
                        ((unsigned long long)rows16(__ballot(((out >> (4 + D)) & 1) != 0)) << (16 * D)) |
                        ((unsigned long long)rows16(__ballot(task[0])) << (16 * A1)) |
                        ((unsigned long long)rows16(__ballot(task[1])) << (16 * A2));
                    const unsigned long long wm = (nm | om) >> (lane >> 2);
                    if ((wm >> (16 * D)) & 1) a.so[D][qs] = sdn;
                    if (!task[0] && ((wm >> (16 * A1)) & 1)) a.so[A1][qs] = T(0);
                    if (!task[1] && ((wm >> (16 * A2)) & 1)) a.so[A2][qs] = T(0);
                    if (lane == 0) a.rmo[blin((uint32_t)b, nb1)] = nm;
                } else {
                    // (the row masks are left stale: rmask_before_sweep)
                    a.so[D][qs] = sdn;
                    if (!task[0]) a.so[A1][qs] = T(0);
                    if (!task[1]) a.so[A2][qs] = T(0);
                }
                if (!fnode) a.flo[qs] = out;
            }
            // queue: unaligned markers of both planes, then the face nodes and their faces
            {
                // a task's node as packed coordinates x | y << 10 | z << 20
                const uint32_t tpos = (uint32_t)(org[0] + lu[0]) | ((uint32_t)(org[1] + lu[1]) << 10) |
                                      ((uint32_t)(org[2] + lu[2]) << 20);
                const unsigned long long lt = (1ull << lane) - 1ull;
                unsigned long long bal = __ballot(fnode);
                const int slot = nslot + __popcll(bal & lt);
                if (fnode) { sq[slot] = (uint32_t)qs; sb[slot] = out; }
                nslot += __popcll(bal);
                bal = __ballot(task[2]);
                if (task[2]) {
                    const int i = ntask + __popcll(bal & lt);
                    tq[i] = tpos;
                    tt[i] = (uint8_t)(0 | ((int)task[0] << 1) | (c00 << 2));
                    ts[i] = (uint16_t)slot;
                }
                ntask += __popcll(bal);
                bal = __ballot(task[3]);
                if (task[3]) {
                    const int i = ntask + __popcll(bal & lt);
                    tq[i] = tpos;
                    tt[i] = (uint8_t)(1 | ((int)task[1] << 1) | (c00 << 2));
                    ts[i] = (uint16_t)slot;
                }
                ntask += __popcll(bal);
            }
            // lists: the next sweep takes the bricks next to a brick holding
            // markers now; Front2VOF revisits the cells of bricks that hold
            // markers or whose colours / markers changed (a cell also reads the
            // edges stored at its upper neighbours)
            // a brick this sweep changed joins the next sweep's list itself
            // (through its markers' neighbourhood when it holds markers), so
            // that the next sweep copies it into the other buffer
            const bool self = !hasm && !same;
            // the neighbours the next sweep can change from this brick's
            // markers: along its axis D' nodes -1..+1 from a marker along D'
            // (landing edges, crossed nodes) and -2..+1 from one across it
            // (face colours read the segments of three faces); across D'
            // rows -1..0 from a marker along D' (the edges across whose end
            // colours change, faces with it on their upper edge) and the
            // marker's own row otherwise; unknown next axis: all 26
            // lanes whose node has local coordinate 0, <= 1, 3 along axis e
            // (lane = x + 4 y + 16 z)
            constexpr unsigned long long k0[3] = {0x1111111111111111ull, 0x000F000F000F000Full, 0xFFFFull};
            constexpr unsigned long long k1[3] = {0x3333333333333333ull, 0x00FF00FF00FF00FFull, 0xFFFFFFFFull};
            constexpr unsigned long long k3[3] = {0x8888888888888888ull, 0xF000F000F000F000ull, 0xFFFF000000000000ull};
            uint32_t m27 = 0x7ffffffu;
            if (hasm && a.nd >= 0) {
                const int Dn = a.nd, An = (Dn + 1) % 3, Bn = (Dn + 2) % 3;
                // markers on edges along D' / across it
                const unsigned long long mD = __ballot(((out >> (4 + Dn)) & 1) != 0);
                const unsigned long long mX = __ballot((out & 0x70 & ~(0x10 << Dn)) != 0);
                // allowed offsets per axis: bit 0 -1, bit 1 0, bit 2 +1.  Along
                // D' a marker along D' reaches -1..+1, one across it -2..+1 (the
                // face colours); across D' only markers along D' reach a row
                // below (-1)
                int al[3];
                al[Dn] = 2 | (((mD & k0[Dn]) | (mX & k1[Dn])) != 0 ? 1 : 0) | (((mD | mX) & k3[Dn]) != 0 ? 4 : 0);
                al[An] = 2 | ((mD & k0[An]) != 0 ? 1 : 0);
                al[Bn] = 2 | ((mD & k0[Bn]) != 0 ? 1 : 0);
                m27 = 0;
                for (int d = 0; d < 27; ++d)
                    if (((al[0] >> (d % 3)) & (al[1] >> (d / 3 % 3)) & (al[2] >> (d / 9))) & 1) m27 |= 1u << d;
            }
            // Front2VOF: a cell of a lower neighbour reads this brick's nodes
            // of coordinate 0 along the axes it is lower along; the neighbour
            // at -1 along axis e needs a revisit only if such a node holds a
            // marker or changed
            uint32_t fm8 = 0xffu;
            if (hasm || chg) {
                const unsigned long long rel = mbal | cbal;
                const int lx = (rel & k0[0]) != 0, ly = (rel & k0[1]) != 0, lz = (rel & k0[2]) != 0;
                fm8 = 0;
                for (int d = 0; d < 8; ++d)
                    if ((!(d & 1) || lx) && (!(d & 2) || ly) && (!(d & 4) || lz)) fm8 |= 1u << d;
            }
            if (lane == 0) {
                if (hasm) { mbr[nm] = (uint32_t)b; mmk[nm] = m27; }
                if (self) sbr[ns] = (uint32_t)b;
                if (hasm || chg) { cbr[nc] = (uint32_t)b; cmk[nc] = (uint8_t)fm8; }
            }
            nm += hasm ? 1 : 0;
            ns += self ? 1 : 0;
            nc += (hasm || chg) ? 1 : 0;
            fbc += fb;
            mergedc += merged;
            }
            cflc += cfl;
            __syncthreads();   // the tiles are reused by the next batch
        }
    }
    run_tasks<T, D, RUN>(a, tq, tt, ts, ntask, sq, sb, nslot, fbt, multit);
    claims();
    // this wave's counters (the wave owns its slot)
    fbc = wave_sum(fbc + fbt);
    cflc = wave_sum(cflc);
    // per lane: merges in the lower 16 bits, annihilations in the upper ones
    // (at most one of each per brick, under 2^15 bricks per wave)
    const int annc = wave_sum(mergedc >> 16);
    mergedc = wave_sum(mergedc & 0xFFFF);
    multit = wave_sum(multit);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cmax = fmaxf(cmax, __shfl_xor(cmax, off));
    // (adds whose result is not waited for)
    if (lane == 0) {
        const int nwv = a.g.nw;
        if (fbc) atomicAdd(&a.w.cs[CS_FALLBACK * nwv + wv], (unsigned long long)fbc);
        if (multit) atomicAdd(&a.w.cs[CS_MULTI * nwv + wv], (unsigned long long)multit);
        if (cflc) atomicAdd(&a.w.cs[CS_CFL * nwv + wv], (unsigned long long)cflc);
        if (mergedc) atomicAdd(&a.w.cs[CS_MERGED * nwv + wv], (unsigned long long)mergedc);
        if (annc) atomicAdd(&a.w.cs[CS_ANNIH * nwv + wv], (unsigned long long)annc);
        if (nact) atomicAdd(&a.w.cs[CS_ACTIVE * nwv + wv], (unsigned long long)nact * 64ull);
        if (cmax > 0.f) atomicMax(&a.w.cs[CS_CMAX * nwv + wv], (unsigned long long)__float_as_uint(cmax));
    }
}

template <typename T, int D, int RUN>
__global__ __launch_bounds__(64, EBIT_SWEEP_WAVES) void k_sweep(SweepArgs<T> a)
{
    sweep_wave<T, D, RUN>(a, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// a5: Front2VOF (sec. 2.5)
// ---------------------------------------------------------------------------
// Cell-local numbering: corner k = ox + 2 oy + 4 oz; edge 4e + oA + 2 oB runs
// along axis e with offsets oA, oB along the other two axes A < B.

struct FaceTab {
    int8_t corner[6][4];   // counter-clockwise about the outward normal
    int8_t edge[6][4];     // edge m joins corner m and corner m+1
    int8_t axis[6];
    int8_t upper[6];
};

__host__ __device__ constexpr int edge_of(int c0, int c1)
{
    // the axis where the corners differ and the offsets of the other two
    int d = c0 ^ c1;
    int e = d == 1 ? 0 : (d == 2 ? 1 : 2);
    int o[3] = {c0 & 1, (c0 >> 1) & 1, (c0 >> 2) & 1};
    int A = e == 0 ? 1 : 0, B = e == 2 ? 1 : 2;
    return 4 * e + o[A] + 2 * o[B];
}

__host__ __device__ constexpr FaceTab make_tab()
{
    FaceTab t{};
    int f = 0;
    for (int a = 0; a < 3; ++a)
        for (int sg = 0; sg < 2; ++sg) {
            int b = (a + 1) % 3, c = (a + 2) % 3;
            // (b, c, a) right-handed: upper face (0,0),(1,0),(1,1),(0,1) in (b,c); lower reversed
            int cb[4] = {0, 1, 1, 0}, cc[4] = {0, 0, 1, 1};
            for (int m = 0; m < 4; ++m) {
                int mm = sg ? m : (4 - m) % 4;
                int o[3] = {0, 0, 0};
                o[a] = sg;
                o[b] = cb[mm];
                o[c] = cc[mm];
                t.corner[f][m] = (int8_t)(o[0] + 2 * o[1] + 4 * o[2]);
            }
            for (int m = 0; m < 4; ++m) t.edge[f][m] = (int8_t)edge_of(t.corner[f][m], t.corner[f][(m + 1) % 4]);
            t.axis[f] = (int8_t)a;
            t.upper[f] = (int8_t)sg;
            ++f;
        }
    return t;
}

constexpr FaceTab kTab = make_tab();

template <typename T>
struct Pt { T x, y, z; };

// position of the marker on cell edge `id` with fraction s (cell frame)
template <typename T>
__device__ __forceinline__ Pt<T> edge_point(int id, T s)
{
    int e = id >> 2;
    T oA = T(id & 1), oB = T((id >> 1) & 1);
    if (e == 0) return {s, oA, oB};
    if (e == 1) return {oA, s, oB};
    return {oA, oB, s};
}

// Reference-phase volume fraction of one cell (sec. 2.5) from its 8 corner
// flag bytes f[k] (corner k = ox + 2 oy + 4 oz), the 12-bit marker mask `has`
// and the 12 marker fractions.  Face segments are oriented from the marker
// where a counter-clockwise walk (about the outward normal) leaves the
// reference phase to the one where it re-enters; four-marker faces cut off
// the corners whose colour differs from the face-centre colour.  Loops are
// the connected sets of segments (separated segments for internal
// ambiguity, sec. 2.4); each loop is fanned from its marker centroid and the
// volume follows from Gauss's theorem: (1/3) sum of the phase-1 areas of the
// three far faces + (1/6) sum over triangles (X_c, X_k+1, X_k) of the triple
// product.  Returns C; *amb = 1 for a 4-marker face or more than one loop.
template <typename T>
__device__ __forceinline__ T cell_volume(const uint8_t f[8], int has, const T sv[12], int &amb_out)
{
    int colb = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) colb |= (f[k] & 1) << k;
    T C;
    int amb = 0, inter = 0;
    if (has == 0) {
        C = (T)(colb & 1);
    } else {
        inter = 1;
        // face segments: oriented from the marker where a counter-clockwise
        // walk leaves the reference phase to the one where it re-enters
        uint64_t lab = 0;            // loop label per marker, 4 bits each
#pragma unroll
        for (int id = 0; id < 12; ++id) lab |= (uint64_t)id << (4 * id);
        Pt<T> S = {T(0), T(0), T(0)};
        T A1[3] = {T(0), T(0), T(0)};
        int four = 0;
        // segments kept for the multi-loop path: start/end edge ids, one byte
        // (start | end << 4) per segment in two words (registers, not scratch)
        int segs = 0;
        uint64_t sg[2] = {0, 0};
#pragma unroll
        for (int fc = 0; fc < 6; ++fc) {
            int cl[4], mk[4], ex[4], ed[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                cl[m] = (colb >> kTab.corner[fc][m]) & 1;
                ed[m] = kTab.edge[fc][m];
                mk[m] = (has >> ed[m]) & 1;
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) ex[m] = cl[m] & (cl[(m + 1) & 3] ^ 1);
            int cnt = mk[0] + mk[1] + mk[2] + mk[3];
            int ns = 0, st[2] = {0, 0}, en[2] = {0, 0};
            if (cnt == 2) {
                int xs = 0, xe = 0;
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    if (mk[m]) { if (ex[m]) xs = m; else xe = m; }
                st[0] = xs; en[0] = xe; ns = 1;
            } else if (cnt == 4) {
                four = 1;
                const int a_ = kTab.axis[fc];
                const int kf = kTab.upper[fc] ? (a_ == 0 ? 1 : (a_ == 1 ? 2 : 4)) : 0;
                const int ff = (f[kf] >> (1 + a_)) & 1;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    if (cl[m] == ff) continue;
                    int mb = (m + 3) & 3;
                    st[ns] = ex[mb] ? mb : m;
                    en[ns] = ex[mb] ? m : mb;
                    ++ns;
                }
            }
            T acc = T(0);
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (k >= ns) continue;
                int is = ed[0], ie = ed[0];
                T ss = sv[ed[0]], se = sv[ed[0]];
#pragma unroll
                for (int m = 1; m < 4; ++m) {
                    if (st[k] == m) { is = ed[m]; ss = sv[ed[m]]; }
                    if (en[k] == m) { ie = ed[m]; se = sv[ed[m]]; }
                }
                Pt<T> Ps = edge_point<T>(is, ss), Pe = edge_point<T>(ie, se);
                // X_end x X_start (fan orientation of sec. 2.5)
                S.x += Pe.y * Ps.z - Pe.z * Ps.y;
                S.y += Pe.z * Ps.x - Pe.x * Ps.z;
                S.z += Pe.x * Ps.y - Pe.y * Ps.x;
                if (kTab.upper[fc]) {
                    const int a_ = kTab.axis[fc];
                    const int bb = (a_ + 1) % 3, cc = (a_ + 2) % 3;
                    T us = bb == 0 ? Ps.x : (bb == 1 ? Ps.y : Ps.z);
                    T vs = cc == 0 ? Ps.x : (cc == 1 ? Ps.y : Ps.z);
                    T ue = bb == 0 ? Pe.x : (bb == 1 ? Pe.y : Pe.z);
                    T ve = cc == 0 ? Pe.x : (cc == 1 ? Pe.y : Pe.z);
                    acc += us * ve - ue * vs;
                }
                // merge loop labels
                uint64_t la = (lab >> (4 * is)) & 15, lb = (lab >> (4 * ie)) & 15;
                if (la != lb) {
                    uint64_t keep = la < lb ? la : lb, drop = la < lb ? lb : la;
#pragma unroll
                    for (int id = 0; id < 12; ++id)
                        if (((lab >> (4 * id)) & 15) == drop) lab = (lab & ~(15ull << (4 * id))) | (keep << (4 * id));
                }
                {
                    const uint64_t v = (uint64_t)(is | (ie << 4)) << (8 * (segs & 7));
                    if (segs < 8) sg[0] |= v;
                    else sg[1] |= v;
                }
                ++segs;
            }
            if (kTab.upper[fc]) {
                // phase-1 area of the far face (Green): right side u = 1 is
                // edge 1, top side v = 1 is edge 2 of the counter-clockwise walk
                T Lr = mk[1] ? (cl[1] ? sv[ed[1]] : T(1) - sv[ed[1]]) : (T)cl[1];
                T Lt = mk[2] ? (cl[3] ? sv[ed[2]] : T(1) - sv[ed[2]]) : (T)cl[3];
                A1[kTab.axis[fc]] = T(0.5) * ((Lr + Lt) + acc);
            }
        }
        // loops: count the roots (markers labelled with their own id)
        int nloops = 0;
#pragma unroll
        for (int id = 0; id < 12; ++id)
            if (((has >> id) & 1) && ((lab >> (4 * id)) & 15) == (uint64_t)id) ++nloops;
        T fan = T(0);
        if (nloops == 1) {
            T gx = T(0), gy = T(0), gz = T(0);
            int nm = 0;
#pragma unroll
            for (int id = 0; id < 12; ++id) {
                if (!((has >> id) & 1)) continue;
                Pt<T> P = edge_point<T>(id, sv[id]);
                gx += P.x; gy += P.y; gz += P.z;
                ++nm;
            }
            gx = gx / (T)nm; gy = gy / (T)nm; gz = gz / (T)nm;
            fan = gx * S.x + gy * S.y + gz * S.z;
        } else {
            // separated loops (sec. 2.4): one centroid per loop
#pragma unroll
            for (int r = 0; r < 12; ++r) {
                if (!((has >> r) & 1) || ((lab >> (4 * r)) & 15) != (uint64_t)r) continue;
                T gx = T(0), gy = T(0), gz = T(0);
                int nm = 0;
#pragma unroll
                for (int id = 0; id < 12; ++id) {
                    if (!((has >> id) & 1) || ((lab >> (4 * id)) & 15) != (uint64_t)r) continue;
                    Pt<T> P = edge_point<T>(id, sv[id]);
                    gx += P.x; gy += P.y; gz += P.z;
                    ++nm;
                }
                gx = gx / (T)nm; gy = gy / (T)nm; gz = gz / (T)nm;
                Pt<T> Sr = {T(0), T(0), T(0)};
                for (int k = 0; k < segs; ++k) {
                    const uint64_t w = k < 8 ? sg[0] : sg[1];
                    const int is = (int)((w >> (8 * (k & 7))) & 15), ie = (int)((w >> (8 * (k & 7) + 4)) & 15);
                    if (((lab >> (4 * is)) & 15) != (uint64_t)r) continue;
                    T ss = T(0), se = T(0);
#pragma unroll
                    for (int id = 0; id < 12; ++id) {
                        if (id == is) ss = sv[id];
                        if (id == ie) se = sv[id];
                    }
                    Pt<T> Ps = edge_point<T>(is, ss), Pe = edge_point<T>(ie, se);
                    Sr.x += Pe.y * Ps.z - Pe.z * Ps.y;
                    Sr.y += Pe.z * Ps.x - Pe.x * Ps.z;
                    Sr.z += Pe.x * Ps.y - Pe.y * Ps.x;
                }
                fan += gx * Sr.x + gy * Sr.y + gz * Sr.z;
            }
        }
        C = ((A1[0] + A1[1]) + A1[2]) / T(3) + fan / T(6);
        amb = four || nloops > 1;
    }
    amb_out = amb;
    (void)inter;
    return C;
}


template <typename T>
struct F2VArgs {
    Geo g;
    const uint8_t *fl;
    const T *s[3];
    T *C;
    Work w;
    uint32_t gen;     // this Front2VOF's generation
    int full;
    int run;          // the list is in brick order: waves take runs of it (Runs)
};

// node indices of the 8 corners of cell (x, y, z) (corner k = ox + 2 oy + 4 oz)
__device__ __forceinline__ void corner_index(int n, long nn, int x, int y, int z, uint32_t qc[8])
{
    const uint32_t un = (uint32_t)n, unn = (uint32_t)nn;
    const uint32_t x0 = (uint32_t)x, x1 = x + 1 == n ? 0u : (uint32_t)x + 1u;
    const uint32_t y0 = __umul24((uint32_t)y, un), y1 = __umul24(y + 1 == n ? 0u : (uint32_t)y + 1u, un);
    const uint32_t z0 = __umul24((uint32_t)z, unn), z1 = __umul24(z + 1 == n ? 0u : (uint32_t)z + 1u, unn);
    qc[0] = x0 + y0 + z0;
    qc[1] = x1 + y0 + z0;
    qc[2] = x0 + y1 + z0;
    qc[3] = x1 + y1 + z0;
    qc[4] = x0 + y0 + z1;
    qc[5] = x1 + y0 + z1;
    qc[6] = x0 + y1 + z1;
    qc[7] = x1 + y1 + z1;
}

// cell coordinates packed in 30 bits (n <= 1024) and back
__device__ __forceinline__ uint32_t pack_xyz(int x, int y, int z)
{
    return (uint32_t)x | ((uint32_t)y << 10) | ((uint32_t)z << 20);
}
__device__ __forceinline__ void unpack_xyz(uint32_t p, int &x, int &y, int &z)
{
    x = (int)(p & 1023u);
    y = (int)((p >> 10) & 1023u);
    z = (int)(p >> 20);
}

// 12-bit marker mask of a cell; edge id 4e + oA + 2 oB starts at the corner
// with offsets oA, oB along the two other axes A < B
__device__ __forceinline__ int marker_mask(const uint8_t f[8])
{
    int has = 0;
#pragma unroll
    for (int id = 0; id < 12; ++id) {
        int e = id >> 2, oA = id & 1, oB = (id >> 1) & 1;
        int cx = e == 0 ? 0 : oA, cy = e == 1 ? 0 : (e == 0 ? oA : oB), cz = e == 2 ? 0 : oB;
        has |= ((f[cx + 2 * cy + 4 * cz] >> (4 + e)) & 1) << id;
    }
    return has;
}

// corner of the cell at which marker edge `id` starts
__device__ __forceinline__ int edge_corner(int id)
{
    const int e = id >> 2, oA = id & 1, oB = (id >> 1) & 1;
    const int cx = e == 0 ? 0 : oA, cy = e == 1 ? 0 : (e == 0 ? oA : oB), cz = e == 2 ? 0 : oB;
    return cx + 2 * cy + 4 * cz;
}

// Volume fractions of queued interfacial cells (one per lane, first `cnt`
// entries of the queue; flags from the queue, fractions from memory).
// Returns the number of ambiguous cells among them.
template <typename T>
__device__ __forceinline__ int f2v_cells(const F2VArgs<T> &a, const uint32_t *cq, const uint64_t *cf, int cnt)
{
    const int lane = threadIdx.x & 63;
    int amb = 0;
    if (lane < cnt) {
        int x, y, z;
        unpack_xyz(cq[lane], x, y, z);
        const uint64_t pk = cf[lane];
        uint8_t f[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) f[k] = (uint8_t)(pk >> (8 * k));
        uint32_t qc[8];
        corner_index(a.g.n, a.g.nn, x, y, z, qc);
        const uint32_t q = qc[0];
        const int has = marker_mask(f);
        T sv[12];
#pragma unroll
        for (int id = 0; id < 12; ++id) sv[id] = ((has >> id) & 1) ? a.s[id >> 2][qc[edge_corner(id)]] : T(0);
        a.C[q] = cell_volume<T>(f, has, sv, amb);
    }
    return wave_sum(amb);
}

// Front2VOF, wave w over items w, w + nw, ... of the revisit list (or every
// brick): a cell without a marker is full or empty (its corner colour); the
// others are queued, their volume fractions computed 64 at a time, and listed
// in the wave's interfacial-cell segment (the cells of this Front2VOF, for
// the surrogate and its training rows).  With `classify` set only the
// segment is written for the interfacial cells.
template <typename T>
__device__ __forceinline__ void f2v_wave(const F2VArgs<T> &a, const int classify, const int wv, const int nw)
{
    __shared__ uint32_t cq[kCellCap];
    __shared__ uint64_t cf[kCellCap];
    __shared__ uint32_t ipre[kSub];
    const int lane = threadIdx.x;
    const int n = a.g.n, nb1 = a.g.nb1, nb = a.g.nb;
    const long nn = a.g.nn;
    const uint32_t gen = a.gen;
    // generation gen + 2 starts empty (gen - 1's Front2VOF has ended; the
    // sweeps writing gen + 1's list may run beside this one)
    if (wv == 0)
        for (int i = lane; i < kNum; i += 64) a.w.fnum[(((gen + 2) % 3) * kNum + i) * kPad] = 0;
    Items it;
    if (a.full) {
        it.total = (uint32_t)nb;
    } else {
        it.init(ipre, a.w.fnum + (gen % 3) * kNum * kPad, a.w.flist[gen % 3], (uint32_t)a.g.scap, (uint32_t)nb);
    }
    uint32_t *seg = a.w.ctask + (size_t)wv * a.g.segcap;
    long np = 0;
    int nq = 0, ambc = 0;
    long long delta = 0;
    // this wave's items, item_of(wv, i) or its run of an ordered list (static:
    // the wave's interfacial-cell segment holds the at most ceil(nb / nw) + 2
    // bricks either gives), resolved one per lane
    Runs ru;
    if (a.run) ru.init((uint32_t)wv, (uint32_t)nw, it.total);
    auto item = [&](uint32_t i) { return a.run ? ru.item(i) : item_of((uint32_t)wv, i, (uint32_t)nw); };
    for (uint32_t i0 = 0; item(i0) < it.total; i0 += 64) {
        int bl = -1;
        {
            const uint32_t k = item(i0 + (uint32_t)lane);
            const bool have = k < it.total;
            int bb = a.full ? (have ? (int)bpack_lin((int)k, nb1) : -1) : it.brick_lane(have ? k : 0);
            if (!have || bb < 0 || bx_of((uint32_t)bb) >= nb1 || by_of((uint32_t)bb) >= nb1 || bz_of((uint32_t)bb) >= nb1)
                bb = -1;
            bl = bb;
        }
        unsigned long long pend = __ballot(bl >= 0);
        while (pend) {
            const int src = __ffsll((long long)pend) - 1;
            pend &= pend - 1;
            const int b = __shfl(bl, src);
            const int x = bx_of((uint32_t)b) * 4 + (lane & 3), y = by_of((uint32_t)b) * 4 + ((lane >> 2) & 3),
                      z = bz_of((uint32_t)b) * 4 + (lane >> 4);
            const int bi = blin((uint32_t)b, nb1);
            uint32_t qc[8];
            corner_index(n, nn, x, y, z, qc);
            const uint32_t q = qc[0];
            uint8_t f[8];
    #pragma unroll
            for (int kk = 0; kk < 8; ++kk) f[kk] = a.fl[qc[kk]];
            const int has = marker_mask(f);
            if (!has) a.C[q] = (T)(f[0] & 1);
            const unsigned long long bal = __ballot(has != 0);
            const int r = __popcll(bal & ((1ull << lane) - 1ull));
            if (has) {
                uint64_t pk = 0;
    #pragma unroll
                for (int kk = 0; kk < 8; ++kk) pk |= (uint64_t)f[kk] << (8 * kk);
                cq[nq + r] = pack_xyz(x, y, z);
                cf[nq + r] = pk;
                if (np + r < a.g.segcap) seg[np + r] = (uint32_t)q;
            }
            const int cnt = __popcll(bal);
            nq += cnt;
            np += cnt;
            delta += (long long)cnt - (long long)a.w.bcnt[bi];
            __syncthreads();
            if (lane == 0) a.w.bcnt[bi] = (uint32_t)cnt;
            if (classify) {
                nq = 0;
            } else if (nq >= 64) {
                ambc += f2v_cells<T>(a, cq, cf, 64);
                __syncthreads();
                const int rest = nq - 64;
                uint32_t mq = 0;
                uint64_t mf = 0;
                if (lane < rest) { mq = cq[64 + lane]; mf = cf[64 + lane]; }
                __syncthreads();
                if (lane < rest) { cq[lane] = mq; cf[lane] = mf; }
                __syncthreads();
                nq = rest;
            }
        }
    }
    if (!classify && nq > 0) ambc += f2v_cells<T>(a, cq, cf, nq);
    if (lane == 0) {
        const int nwv = a.g.nw;
        a.w.ccnt[wv] = (uint32_t)(np < a.g.segcap ? np : a.g.segcap);
        // the interfacial count changes by delta at this generation; the sum
        // over generations of the count follows from the sums of delta and
        // gen * delta (adds whose result is not waited for)
        if (delta) {
            atomicAdd(&a.w.cs[CS_INTER * nwv + wv], (unsigned long long)delta);
            atomicAdd(&a.w.cs[CS_INTER_GEN * nwv + wv], (unsigned long long)((long long)gen * delta));
        }
        if (!classify) {
            a.w.cs[CS_AMB * nwv + wv] = (unsigned long long)ambc;
            a.w.cs[CS_SURR * nwv + wv] = 0ull;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(64, EBIT_F2V_WAVES) void k_f2v(F2VArgs<T> a, int classify)
{
    f2v_wave<T>(a, classify, blockIdx.x, gridDim.x);
}

// A Front2VOF and the x sweep that follows it, in one grid: the sweep reads
// the state the Front2VOF reads and writes the other buffer, so the two are
// independent.  The sweep's workgroups come first and fill the chip; the
// Front2VOF's start as sweep waves retire and fill the sweep's tail (both
// parts have a multiple of 8 waves, so each keeps its XCD-aware mapping).
template <typename T, int RUN>
__global__ __launch_bounds__(64, EBIT_SWEEP_WAVES) void k_f2v_sweep_x(SweepArgs<T> s, F2VArgs<T> f, int classify)
{
    const int b = blockIdx.x, nw = s.g.nw;
    if (b < nw) sweep_wave<T, 0, RUN>(s, b, nw);
    else f2v_wave<T>(f, classify, b - nw, nw);
}


// Topology of a cell from flags alone (sec. 2.4): a face with four markers,
// or face segments that close into more than one loop, make the cell
// ambiguous (the surrogate's inputs do not determine its shape).
__device__ __forceinline__ int cell_ambiguous(const uint8_t f[8], int has)
{
    int colb = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) colb |= (f[k] & 1) << k;
    uint64_t lab = 0;
#pragma unroll
    for (int id = 0; id < 12; ++id) lab |= (uint64_t)id << (4 * id);
#pragma unroll
    for (int fc = 0; fc < 6; ++fc) {
        int mk[4], ed[4], cnt = 0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            ed[m] = kTab.edge[fc][m];
            mk[m] = (has >> ed[m]) & 1;
            cnt += mk[m];
        }
        if (cnt == 4) return 1;
        if (cnt == 2) {
            int ia = -1, ib = -1;
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (mk[m]) { if (ia < 0) ia = ed[m]; else ib = ed[m]; }
            uint64_t la = (lab >> (4 * ia)) & 15, lb = (lab >> (4 * ib)) & 15;
            if (la != lb) {
                uint64_t keep = la < lb ? la : lb, drop = la < lb ? lb : la;
#pragma unroll
                for (int id = 0; id < 12; ++id)
                    if (((lab >> (4 * id)) & 15) == drop) lab = (lab & ~(15ull << (4 * id))) | (keep << (4 * id));
            }
        }
    }
    int roots = 0;
#pragma unroll
    for (int id = 0; id < 12; ++id)
        if (((has >> id) & 1) && ((lab >> (4 * id)) & 15) == (uint64_t)id) ++roots;
    (void)colb;
    return roots > 1;
}

// load an interfacial cell: corner flags, marker mask, fractions
template <typename T>
__device__ __forceinline__ int load_cell(const F2VArgs<T> &a, long q, uint8_t f[8], T sv[12])
{
    const int n = a.g.n;
    uint32_t qc[8];
    const uint32_t uq = (uint32_t)q, un = (uint32_t)n, qn = uq / un;   // n^3 < 2^32: 32-bit division
    corner_index(n, a.g.nn, (int)(uq - qn * un), (int)(qn % un), (int)(qn / un), qc);
#pragma unroll
    for (int k = 0; k < 8; ++k) f[k] = a.fl[qc[k]];
    const int has = marker_mask(f);
#pragma unroll
    for (int id = 0; id < 12; ++id) {
        int e = id >> 2, oA = id & 1, oB = (id >> 1) & 1;
        int cx = e == 0 ? 0 : oA, cy = e == 1 ? 0 : (e == 0 ? oA : oB), cz = e == 2 ? 0 : oB;
        sv[id] = ((has >> id) & 1) ? a.s[e][qc[cx + 2 * cy + 4 * cz]] : T(0);
    }
    return has;
}

// surrogate input row of a cell: 12 fractions then 8 corner colours (bf16)
template <typename T>
__device__ __forceinline__ void put_features(__bf16 *row, const uint8_t f[8], const T sv[12])
{
#pragma unroll
    for (int id = 0; id < 12; ++id) row[id] = ebit_mlp::to_bf16((float)sv[id]);
#pragma unroll
    for (int k = 0; k < 8; ++k) row[12 + k] = ebit_mlp::to_bf16((float)(f[k] & 1));
#pragma unroll
    for (int k = 20; k < ebit_mlp::kKIn; ++k) row[k] = ebit_mlp::to_bf16(0.f);
}

// Front2VOF phase B with the learned surrogate: unambiguous interfacial cells
// take the network's volume fraction, computed on matrix cores 16 cells at a
// time; ambiguous ones fall back to the geometric construction.  The
// interfacial-cell segments of the classify pass are taken as one array (a
// prefix sum of their lengths in LDS), 64 cells per wave at a time, so short
// segments do not leave tiles empty; the block's waves share the weights in
// LDS (a block without cells does not copy them).
template <typename T>
__global__ __launch_bounds__(64 * kSurrWaves) void k_f2v_b_surr(F2VArgs<T> a)
{
    using namespace ebit_mlp;
    constexpr int kThreads = 64 * kSurrWaves;
    constexpr int kPer = (kMaxWaves + kThreads - 1) / kThreads;
    __shared__ MlpWeights W;
    __shared__ __bf16 xs[kSurrWaves][64 * kRow1];
    __shared__ __bf16 h1s[kSurrWaves][16 * kRow2];
    __shared__ uint32_t rows[kSurrWaves][64];
    __shared__ uint32_t pre[kMaxWaves + 1];
    __shared__ uint32_t wtot[kSurrWaves];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lg = lane >> 4;
    const int nc = a.g.nw;
    const uint32_t segcap = (uint32_t)a.g.segcap;
    // exclusive prefix of the segment lengths: pre[k] = cells before segment k
    {
        uint32_t v[kPer], sum = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int k = (int)threadIdx.x * kPer + j;
            v[j] = k < nc ? min(a.w.ccnt[k], segcap) : 0u;
            sum += v[j];
        }
        const uint32_t incl = wave_incl_scan(sum);
        if (lane == 63) wtot[wave] = incl;
        __syncthreads();
        uint32_t run = incl - sum;
        for (int w = 0; w < wave; ++w) run += wtot[w];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int k = (int)threadIdx.x * kPer + j;
            if (k < nc) pre[k] = run;
            run += v[j];
        }
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int w = 0; w < kSurrWaves; ++w) tot += wtot[w];
            pre[nc] = tot;
        }
        __syncthreads();
    }
    const uint32_t total = pre[nc];
    const uint32_t nchunks = (total + 63) / 64;
    const uint32_t gw = gridDim.x * kSurrWaves, gwv = blockIdx.x * kSurrWaves + wave;
    // the ambiguous- and network-cell slots: one per wave of this grid, the rest zero
    if (blockIdx.x == 0)
        for (int k = (int)gw + (int)threadIdx.x; k < nc; k += kThreads) {
            a.w.cs[CS_AMB * nc + k] = 0ull;
            a.w.cs[CS_SURR * nc + k] = 0ull;
        }
    if (blockIdx.x * kSurrWaves < nchunks) copy_to_lds(&W, &a.w.simg->W, (int)sizeof(MlpWeights));
    __syncthreads();
    int ambc = 0, nsurc = 0;
    for (uint32_t chunk = gwv; chunk < nchunks; chunk += gw) {
        const uint32_t i = chunk * 64 + (uint32_t)lane;
        const bool valid = i < total;
        long q = 0;
        uint8_t f[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        T sv[12];
        int has = 0, amb = 0;
        if (valid) {
            // segment of cell i: the last k with pre[k] <= i
            int lo = 0, hi = nc;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (pre[mid] <= i) lo = mid;
                else hi = mid;
            }
            q = (long)a.w.ctask[(size_t)lo * a.g.segcap + (i - pre[lo])];
            has = load_cell<T>(a, q, f, sv);
            amb = cell_ambiguous(f, has);
        }
        if (valid && amb) {
            int am = 0;
            a.C[q] = cell_volume<T>(f, has, sv, am);
            ambc += 1;
        }
        const bool sur = valid && !amb;
        const unsigned long long bal = __ballot(sur);
        const int nsur = __popcll(bal);
        nsurc += nsur;
        if (sur) {
            const int pos = __popcll(bal & ((1ull << lane) - 1ull));
            put_features<T>(&xs[wave][pos * kRow1], f, sv);
            rows[wave][pos] = (uint32_t)q;
        }
        wave_sync();
        for (int t0 = 0; t0 < nsur; t0 += 16) {
            const int rrow = t0 + lr;
            u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
            if (rrow < nsur) v = *(const u16x8 *)&xs[wave][rrow * kRow1 + 8 * lg];
            float out[4];
            forward_tile(W, h1s[wave], __builtin_bit_cast(bf16x8, v), out, nullptr, nullptr);
            if (lr == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rr = t0 + 4 * lg + r;
                    if (rr < nsur) a.C[rows[wave][rr]] = (T)out[r];
                }
            }
        }
        wave_sync();
    }
    const int sa = wave_sum(ambc);
    if (lane == 0 && (int)gwv < nc) {
        a.w.cs[CS_AMB * nc + gwv] = (unsigned long long)sa;
        a.w.cs[CS_SURR * nc + gwv] = (unsigned long long)nsurc;
    }
}

// the surrogate's weights image from its FP32 parameters
__global__ __launch_bounds__(256) void k_surr_pack(const float *__restrict__ theta, ebit_mlp::MlpImage *__restrict__ img)
{
    using namespace ebit_mlp;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < kNH * kRow1) pack_w1_slot(img, theta, t);
    else if (t < kNH * kRow1 + kNParam - kOB1) image_store(img, kOB1 + (t - kNH * kRow1), theta[kOB1 + (t - kNH * kRow1)]);
}
constexpr int kSurrPackThreads = ebit_mlp::kNH * ebit_mlp::kRow1 + ebit_mlp::kNParam - ebit_mlp::kOB1;

// Surrogate training rows: per segment, the unambiguous interfacial cells of
// the last Front2VOF (count pass, then write pass at host-computed offsets).
template <typename T>
__global__ __launch_bounds__(64) void k_dataset(F2VArgs<T> a, int write, uint16_t *__restrict__ xout,
                                                float *__restrict__ cout, long cap)
{
    const int lane = threadIdx.x;
    const int nc = a.g.nw;
    for (int ch = blockIdx.x; ch < nc; ch += gridDim.x) {
        const uint32_t count = min(a.w.ccnt[ch], (uint32_t)a.g.segcap);
        long pos = write ? a.w.doff[ch] : 0;
        for (uint32_t base = 0; base < count; base += 64) {
            const uint32_t i = base + lane;
            const bool valid = i < count;
            uint8_t f[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            T sv[12];
            int has = 0, amb = 1;
            if (valid) {
                has = load_cell<T>(a, (long)a.w.ctask[(size_t)ch * a.g.segcap + i], f, sv);
                amb = cell_ambiguous(f, has);
            }
            const bool take = valid && !amb;
            const unsigned long long bal = __ballot(take);
            if (write && take) {
                const long r = pos + __popcll(bal & ((1ull << lane) - 1ull));
                if (r < cap) {
                    __bf16 row[ebit_mlp::kKIn];
                    put_features<T>(row, f, sv);
#pragma unroll
                    for (int k = 0; k < ebit_mlp::kKIn; ++k) xout[r * ebit_mlp::kKIn + k] = __builtin_bit_cast(uint16_t, row[k]);
                    int am = 0;
                    cout[r] = (float)cell_volume<T>(f, has, sv, am);
                }
            }
            pos += __popcll(bal);
        }
        if (!write && lane == 0) a.w.dcnt[ch] = (uint32_t)pos;
    }
}

// totals of the per-wave counters (integer sums: order-free)
__global__ __launch_bounds__(256) void k_stats_reduce(Work w, Geo g)
{
    __shared__ unsigned long long red[CS_COUNT][4];
    unsigned long long acc[CS_COUNT];
    for (int k = 0; k < CS_COUNT; ++k) acc[k] = 0;
    for (int ch = threadIdx.x; ch < g.nw; ch += blockDim.x)
        for (int k = 0; k < CS_COUNT; ++k) {
            const unsigned long long v = w.cs[k * g.nw + ch];
            acc[k] = k == CS_CMAX ? max(acc[k], v) : acc[k] + v;
        }
    for (int k = 0; k < CS_COUNT; ++k) {
        unsigned long long v = acc[k];
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long u = __shfl_xor(v, off);
            v = k == CS_CMAX ? max(v, u) : v + u;
        }
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < CS_COUNT) {
        const int k = threadIdx.x;
        unsigned long long v = k == CS_CMAX ? max(max(red[k][0], red[k][1]), max(red[k][2], red[k][3]))
                                            : red[k][0] + red[k][1] + red[k][2] + red[k][3];
        const int map[CS_COUNT] = {ST_FALLBACK, ST_MULTI, ST_CFL, ST_MERGED, ST_ACTIVE, ST_INTER_SUM, ST_INTER, ST_AMB,
                                   ST_CMAX, ST_ANNIH, ST_SURR};
        w.stat[map[k]] = v;
    }
}

// ---------------------------------------------------------------------------
// a6: deterministic compensated volume sum and marker counts
// ---------------------------------------------------------------------------

__device__ __forceinline__ void neumaier_add(double &s, double &c, double v)
{
    double t = s + v;
    if (fabs(s) >= fabs(v)) c += (s - t) + v;
    else c += (v - t) + s;
    s = t;
}

template <typename T>
__global__ __launch_bounds__(256) void k_vol_partial(const T *__restrict__ C, const uint8_t *__restrict__ fl, int n,
                                                     double *__restrict__ part, unsigned long long *__restrict__ stat)
{
    __shared__ double ss[256], sc[256];
    double s = 0.0, c = 0.0;
    int m0 = 0, m1 = 0, m2 = 0, af = 0;
    const uint32_t un = (uint32_t)n, unn = un * un;
    const long N = (long)unn * n;
    long stride = (long)gridDim.x * blockDim.x;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < N; q += stride) {
        neumaier_add(s, c, (double)C[q]);
        uint8_t f = fl[q];
        m0 += (f >> 4) & 1;
        m1 += (f >> 5) & 1;
        m2 += (f >> 6) & 1;
        // faces whose lowest corner is this node with a marker on each of their
        // four edges (sec. 2.4's face ambiguity), one family per normal axis
        if (f & 0x70) {
            const uint32_t uq = (uint32_t)q, x = uq % un, y = (uq / un) % un, z = uq / unn;
            const uint8_t fx = fl[uq + (x + 1 == un ? 0u - (un - 1) : 1u)];
            const uint8_t fy = fl[uq + (y + 1 == un ? 0u - (un - 1) * un : un)];
            const uint8_t fz = fl[uq + (z + 1 == un ? 0u - (un - 1) * unn : unn)];
            af += (f >> 5) & (fz >> 5) & (f >> 6) & (fy >> 6) & 1;   // normal x: y-edges, z-edges
            af += (f >> 4) & (fz >> 4) & (f >> 6) & (fx >> 6) & 1;   // normal y: x-edges, z-edges
            af += (f >> 4) & (fy >> 4) & (f >> 5) & (fx >> 5) & 1;   // normal z: x-edges, y-edges
        }
    }
    ss[threadIdx.x] = s;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            double s1 = ss[threadIdx.x], c1 = sc[threadIdx.x];
            neumaier_add(s1, c1, ss[threadIdx.x + h]);
            ss[threadIdx.x] = s1;
            sc[threadIdx.x] = c1 + sc[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ss[0];
        part[2 * blockIdx.x + 1] = sc[0];
    }
    // marker counts (integer, order-free)
    for (int off = 32; off > 0; off >>= 1) {
        m0 += __shfl_down(m0, off);
        m1 += __shfl_down(m1, off);
        m2 += __shfl_down(m2, off);
        af += __shfl_down(af, off);
    }
    if ((threadIdx.x & 63) == 0) {
        if (m0) atomicAdd(&stat[ST_MARK0], (unsigned long long)m0);
        if (m1) atomicAdd(&stat[ST_MARK1], (unsigned long long)m1);
        if (m2) atomicAdd(&stat[ST_MARK2], (unsigned long long)m2);
        if (af) atomicAdd(&stat[ST_AFACE], (unsigned long long)af);
    }
}

__global__ void k_vol_final(double *part, int nblocks)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0, c = 0.0;
        for (int k = 0; k < nblocks; ++k) {
            neumaier_add(s, c, part[2 * k]);
            c += part[2 * k + 1];
        }
        part[2 * nblocks] = s;
        part[2 * nblocks + 1] = c;
    }
}

// error sums against a reference C0 (secs. 3.1-3.2, eqs. Eq_error_surface and
// Eq_error_shape): compensated sums of C, of C0 and of |C - C0|, each with the
// same fixed reduction order as k_vol_partial
template <typename T>
__global__ __launch_bounds__(256) void k_err_partial(const T *__restrict__ C, const T *__restrict__ C0, long N,
                                                     double *__restrict__ part)
{
    __shared__ double ss[3][256], sc[3][256];
    double s[3] = {0.0, 0.0, 0.0}, c[3] = {0.0, 0.0, 0.0};
    long stride = (long)gridDim.x * blockDim.x;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < N; q += stride) {
        const double a = (double)C[q], b = (double)C0[q];
        neumaier_add(s[0], c[0], a);
        neumaier_add(s[1], c[1], b);
        neumaier_add(s[2], c[2], fabs(a - b));
    }
    for (int k = 0; k < 3; ++k) {
        ss[k][threadIdx.x] = s[k];
        sc[k][threadIdx.x] = c[k];
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            for (int k = 0; k < 3; ++k) {
                double s1 = ss[k][threadIdx.x], c1 = sc[k][threadIdx.x];
                neumaier_add(s1, c1, ss[k][threadIdx.x + h]);
                ss[k][threadIdx.x] = s1;
                sc[k][threadIdx.x] = c1 + sc[k][threadIdx.x + h];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        part[6 * blockIdx.x + 2 * threadIdx.x] = ss[threadIdx.x][0];
        part[6 * blockIdx.x + 2 * threadIdx.x + 1] = sc[threadIdx.x][0];
    }
}

__global__ void k_err_final(double *part, int nblocks)
{
    if (blockIdx.x == 0 && threadIdx.x < 3) {
        const int k = threadIdx.x;
        double s = 0.0, c = 0.0;
        for (int b = 0; b < nblocks; ++b) {
            neumaier_add(s, c, part[6 * b + 2 * k]);
            c += part[6 * b + 2 * k + 1];
        }
        part[6 * nblocks + 2 * k] = s;
        part[6 * nblocks + 2 * k + 1] = c;
    }
}

__global__ void k_zero_marks(unsigned long long *stat)
{
    if (threadIdx.x < 3) stat[ST_MARK0 + threadIdx.x] = 0;
    if (threadIdx.x == 3) stat[ST_AFACE] = 0;
}

}  // namespace
// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct ebit_ctx {
    int n;
    int precision;
    void *s[2][3];
    uint8_t *flags[2];
    int cur;
    Work w;
    Geo g;
    uint32_t t;            // next sweep's sequence number (the first sweep is 2)
    uint32_t fgen;         // next Front2VOF generation
    uint32_t last_t_f2v;   // sweep counter at the last Front2VOF
    int full;              // process every brick
    const void *lastC;     // C array of the previous Front2VOF
    int surr;              // the surrogate is set (weights image in w.simg); 0: geometric Front2VOF only
    int fuse;              // ebit_advance launches a Front2VOF with the next x sweep
    int order;             // each sweep's band list is put in brick order first
    int next_dir;          // axis of the sweep after the one being launched, -1 if not known
    int rm_dirty;          // a sweep over a claim-ordered list left Work::rmask stale
    int timing;            // bracket every timing-th launch of each kind with events (0: off)
    unsigned tseen[3];     // launches of each kind since timing was switched on
    int tsel;              // the current launch is bracketed
    hipEvent_t *ev;        // 2 * kTimed events
    uint8_t *ev_kind;      // 0 sweep, 1 Front2VOF, 2 Front2VOF with the x sweep
    int ev_n;              // launches recorded since the last ebit_timing
    double mass_sum;       // ebit_errors: sum of |V - V0| / V0 since the last reset
    int64_t mass_n;        // and the number of calls in it
};

namespace {

hipStream_t S(void *p) { return (hipStream_t)p; }

int check_launch()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        fprintf(stderr, "ebit: HIP error %s\n", hipGetErrorString(e));
        return EBIT_EHIP;
    }
    return EBIT_OK;
}

int clampi(int v, int hi) { return v < hi ? (v > 0 ? v : 1) : hi; }

constexpr int kTimed = 8192;   // launches timed between two ebit_timing calls

// every c->timing-th launch of each kind is bracketed (events perturb the
// stream, so a sample of the launches keeps the timed run representative)
void time_begin(ebit_ctx *c, hipStream_t st, int kind)
{
    c->tsel = 0;
    if (!c->timing || !c->ev || c->ev_n >= kTimed) return;
    if (c->tseen[kind]++ % (unsigned)c->timing != 0) return;
    c->tsel = 1;
    (void)hipEventRecord(c->ev[2 * c->ev_n], st);
}

void time_end(ebit_ctx *c, hipStream_t st, int kind)
{
    if (!c->tsel) return;
    (void)hipEventRecord(c->ev[2 * c->ev_n + 1], st);
    c->ev_kind[c->ev_n++] = (uint8_t)kind;
    c->tsel = 0;
}

template <typename T>
SweepArgs<T> sweep_args(const ebit_ctx *c, const void *U, T cf)
{
    SweepArgs<T> a;
    a.g = c->g;
    a.fl = c->flags[c->cur];
    a.flo = c->flags[c->cur ^ 1];
    a.rmo = c->w.rmask[c->cur ^ 1];
    for (int e = 0; e < 3; ++e) {
        a.s[e] = (const T *)c->s[c->cur][e];
        a.so[e] = (T *)c->s[c->cur ^ 1][e];
    }
    a.U = (const T *)U;
    a.c = cf;
    a.w = c->w;
    a.t = c->t;
    a.fgen = c->fgen;
    a.full = c->full;
    a.run = c->order && !c->full;
    a.nd = c->next_dir;
    return a;
}

// a brick list in brick order (see OrderArgs)
void order_list(const ebit_ctx *c, const uint32_t *stamp, uint32_t val, uint32_t *list, uint32_t *num, hipStream_t st)
{
    OrderArgs o;
    o.stamp = stamp;
    o.val = val;
    o.out = list + (size_t)kSub * c->g.scap;
    o.num = num;
    o.cnt = c->w.ocnt;
    o.nb = (uint32_t)c->g.nb;
    o.per = (o.nb + kOrderBlocks - 1) / kOrderBlocks;
    o.nb1 = c->g.nb1;
    const int nblk = (int)((o.nb + o.per - 1) / o.per);
    hipLaunchKernelGGL(k_order_count, dim3(nblk), dim3(256), 0, st, o);
    hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(1024), 0, st, o, nblk);
    hipLaunchKernelGGL(k_order_write, dim3(nblk), dim3(256), 0, st, o);
}

// the band list of the next sweep (c->t)
void order_band(const ebit_ctx *c, hipStream_t st)
{
    if (!c->order || c->full) return;
    const uint32_t t = c->t;
    order_list(c, c->w.cm, t, c->w.blist[t % 4], c->w.bnum + (t % 4) * kNum * kPad, st);
}

// the revisit list of Front2VOF generation gen (not for a full Front2VOF)
void order_revisit(const ebit_ctx *c, uint32_t gen, int full, hipStream_t st)
{
    if (!c->order || full) return;
    order_list(c, c->w.fmark, gen, c->w.flist[gen % 3], c->w.fnum + (gen % 3) * kNum * kPad, st);
}

// Row masks (Work::rmask) before a sweep: kept by sweeps over brick-ordered
// lists, which read them; a sweep over a claim-ordered list neither reads nor
// updates them, so the next brick-ordered one first sets them all to ones.
void rmask_before_sweep(ebit_ctx *c, int run, hipStream_t st)
{
    if (!run) {
        c->rm_dirty = 1;
    } else if (c->rm_dirty) {
        hipLaunchKernelGGL(k_rmask_ones, dim3(clampi((c->g.nb + 255) / 256, 4096)), dim3(256), 0, st, c->w, c->g);
        c->rm_dirty = 0;
    }
}

template <typename T, int D>
void launch_sweep(ebit_ctx *c, const void *U, T cf, hipStream_t st)
{
    order_band(c, st);
    const SweepArgs<T> a = sweep_args<T>(c, U, cf);
    rmask_before_sweep(c, a.run, st);
    time_begin(c, st, 0);
    if (a.run) hipLaunchKernelGGL((k_sweep<T, D, 1>), dim3(c->g.nw), dim3(64), 0, st, a);
    else hipLaunchKernelGGL((k_sweep<T, D, 0>), dim3(c->g.nw), dim3(64), 0, st, a);
    time_end(c, st, 0);
}

template <typename T>
F2VArgs<T> f2v_args(const ebit_ctx *c, void *C, int full)
{
    F2VArgs<T> a;
    a.g = c->g;
    a.fl = c->flags[c->cur];
    for (int e = 0; e < 3; ++e) a.s[e] = (const T *)c->s[c->cur][e];
    a.C = (T *)C;
    a.w = c->w;
    a.gen = c->fgen;
    a.full = full;
    a.run = c->order && !full;
    return a;
}

template <typename T>
int sweep_impl(ebit_ctx *c, int dir, const void *U, double g, double dt, hipStream_t st)
{
    double cd = (dt * (double)c->n) * g;
    T cf = (T)cd;
    if (dir == 0) launch_sweep<T, 0>(c, U, cf, st);
    else if (dir == 1) launch_sweep<T, 1>(c, U, cf, st);
    else launch_sweep<T, 2>(c, U, cf, st);
    c->t++;
    c->cur ^= 1;
    return check_launch();
}

template <typename T>
int f2v_impl(ebit_ctx *c, void *C, hipStream_t st)
{
    int full = c->full || C != c->lastC;
    if (!full && c->last_t_f2v == c->t) return EBIT_OK;   // nothing moved since the last call
    const F2VArgs<T> a = f2v_args<T>(c, C, full);
    order_revisit(c, c->fgen, full, st);
    time_begin(c, st, 1);
    hipLaunchKernelGGL((k_f2v<T>), dim3(c->g.nw), dim3(64), 0, st, a, c->surr ? 1 : 0);
    if (c->surr)
        hipLaunchKernelGGL((k_f2v_b_surr<T>), dim3(clampi((c->g.nw + kSurrWaves - 1) / kSurrWaves, EBIT_SURR_BLOCKS)),
                           dim3(64 * kSurrWaves), 0, st, a);
    time_end(c, st, 1);
    c->fgen++;
    c->last_t_f2v = c->t;
    c->lastC = C;
    return check_launch();
}

// Front2VOF into C (after at least one sweep) and then the x sweep of the
// next step, as one launch of k_f2v_sweep_x.  With the surrogate set, the
// launch holds its classify pass and the network's pass follows: it reads
// the state the x sweep left untouched (the sweep writes the other buffer),
// and the y sweep, which overwrites that state, comes after it on the stream.
template <typename T>
int f2v_sweep_x_impl(ebit_ctx *c, void *C, const void *Ux, double g, double dt, hipStream_t st)
{
    const F2VArgs<T> f = f2v_args<T>(c, C, c->full || C != c->lastC);
    c->fgen++;
    c->last_t_f2v = c->t;
    c->lastC = C;
    const SweepArgs<T> a = sweep_args<T>(c, Ux, (T)((dt * (double)c->n) * g));
    order_revisit(c, f.gen, f.full, st);
    order_band(c, st);
    rmask_before_sweep(c, a.run, st);
    time_begin(c, st, 2);
    const int classify = c->surr ? 1 : 0;
    if (a.run) hipLaunchKernelGGL((k_f2v_sweep_x<T, 1>), dim3(2 * c->g.nw), dim3(64), 0, st, a, f, classify);
    else hipLaunchKernelGGL((k_f2v_sweep_x<T, 0>), dim3(2 * c->g.nw), dim3(64), 0, st, a, f, classify);
    if (c->surr)
        hipLaunchKernelGGL((k_f2v_b_surr<T>), dim3(clampi((c->g.nw + kSurrWaves - 1) / kSurrWaves, EBIT_SURR_BLOCKS)),
                           dim3(64 * kSurrWaves), 0, st, f);
    time_end(c, st, 2);
    c->t++;
    c->cur ^= 1;
    return check_launch();
}

// work space cleared, band list of the first sweep built from the state
int init_lists(ebit_ctx *c, hipStream_t st)
{
    const int nz = c->g.nb > c->g.nw ? c->g.nb : (c->g.nw > 4 * kNum ? c->g.nw : 4 * kNum);
    hipLaunchKernelGGL(k_zero_work, dim3((nz + 255) / 256), dim3(256), 0, st, c->w, c->g);
    hipLaunchKernelGGL(k_init_band, dim3(clampi(c->g.nb, kMaxWaves)), dim3(64), 0, st, c->g, c->flags[0], c->w);
    return check_launch();
}

template <typename T>
int dataset_impl(ebit_ctx *c, void *x_bf16, float *cout, int64_t cap, int64_t *count, hipStream_t st)
{
    if (c->fgen < 2) return EBIT_EINVAL;                  // no Front2VOF yet
    F2VArgs<T> a;
    a.g = c->g;
    a.fl = c->flags[c->cur];
    for (int e = 0; e < 3; ++e) a.s[e] = (const T *)c->s[c->cur][e];
    a.C = nullptr;
    a.w = c->w;
    a.gen = c->fgen - 1;
    a.full = 0;
    int grid = c->g.nw;
    hipLaunchKernelGGL((k_dataset<T>), dim3(grid), dim3(64), 0, st, a, 0, (uint16_t *)nullptr, (float *)nullptr, 0L);
    if (check_launch() != EBIT_OK) return EBIT_EHIP;
    const int nc = c->g.nw;
    uint32_t *hc = (uint32_t *)malloc((size_t)nc * 4);
    long long *ho = (long long *)malloc((size_t)nc * 8);
    if (!hc || !ho) { free(hc); free(ho); return EBIT_EINVAL; }
    int rc = EBIT_OK;
    if (hipMemcpyAsync(hc, c->w.dcnt, (size_t)nc * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) rc = EBIT_EHIP;
    long long tot = 0;
    for (int k = 0; k < nc && rc == EBIT_OK; ++k) { ho[k] = tot; tot += hc[k]; }
    if (rc == EBIT_OK && (hipMemcpyAsync(c->w.doff, ho, (size_t)nc * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
                          hipStreamSynchronize(st) != hipSuccess)) rc = EBIT_EHIP;
    free(hc);
    free(ho);
    if (rc != EBIT_OK) return rc;
    *count = tot;
    if (x_bf16 && cout && cap > 0) {
        hipLaunchKernelGGL((k_dataset<T>), dim3(grid), dim3(64), 0, st, a, 1, (uint16_t *)x_bf16, cout, (long)cap);
        rc = check_launch();
    }
    return rc;
}

}  // namespace

extern "C" {

size_t ebit_scratch_bytes(int32_t n)
{
    if (n < 8 || n % 4) return 0;
    return work_layout(n, nullptr, nullptr);
}

const char *ebit_strerror(int code)
{
    switch (code) {
    case EBIT_OK: return "ok";
    case EBIT_EINVAL: return "invalid argument";
    case EBIT_ECFL: return "Courant number above one";
    case EBIT_ESTATE: return "inconsistent state";
    case EBIT_EHIP: return "HIP runtime error";
    case EBIT_ENOSURR: return "surrogate weights missing";
    case EBIT_ESCRATCH: return "scratch buffer too small";
    case EBIT_ETOOBIG: return "input larger than the fixed work space allows";
    default: return "unknown error";
    }
}

int ebit_init(ebit_ctx **out, const ebit_desc *d, const double *phi_nodes, const double *const *phi_faces,
              const double *const *s_exact, void *stream)
{
    if (!out || !d) return EBIT_EINVAL;
    if (d->n < 8 || d->n % 4 || d->n > 1024) return EBIT_EINVAL;
    if (d->precision != EBIT_FP64 && d->precision != EBIT_FP32) return EBIT_EINVAL;
    for (int b = 0; b < 2; ++b) {
        if (!d->flags[b]) return EBIT_EINVAL;
        for (int e = 0; e < 3; ++e)
            if (!d->s[b][e]) return EBIT_EINVAL;
    }
    if (!d->scratch) return EBIT_EINVAL;
    if (d->scratch_bytes < ebit_scratch_bytes(d->n)) return EBIT_ESCRATCH;
    if (phi_nodes && (!phi_faces || !phi_faces[0] || !phi_faces[1] || !phi_faces[2])) return EBIT_EINVAL;
    if (s_exact && (!s_exact[0] || !s_exact[1] || !s_exact[2])) return EBIT_EINVAL;

    ebit_ctx *c = (ebit_ctx *)calloc(1, sizeof(ebit_ctx));
    if (!c) return EBIT_EINVAL;
    c->n = d->n;
    c->precision = d->precision;
    for (int b = 0; b < 2; ++b) {
        c->flags[b] = d->flags[b];
        for (int e = 0; e < 3; ++e) c->s[b][e] = d->s[b][e];
    }
    c->cur = 0;
    work_layout(d->n, &c->w, (char *)d->scratch);
    c->g.n = d->n;
    c->g.nb1 = d->n / 4;
    c->g.nn = (long)d->n * d->n;
    int nbricks = c->g.nb1 * c->g.nb1 * c->g.nb1;
    c->g.nb = nbricks;
    c->g.nw = waves_for(d->n);
    c->g.segcap = segcap_for(d->n);
    c->g.scap = scap_for(d->n);
    c->t = 2;
    c->fgen = 1;
    c->last_t_f2v = 0;
    c->full = 0;
    c->lastC = nullptr;
    c->surr = 0;
    c->fuse = 1;
    c->order = d->n >= EBIT_ORDER_MIN_N;
    c->next_dir = -1;
    c->rm_dirty = 0;
    hipStream_t st = S(stream);
    long N = (long)d->n * d->n * d->n;
    if (phi_nodes) {
        const double *se0 = s_exact ? s_exact[0] : nullptr, *se1 = s_exact ? s_exact[1] : nullptr,
                     *se2 = s_exact ? s_exact[2] : nullptr;
        if (c->precision == EBIT_FP64)
            hipLaunchKernelGGL(k_init<double>, dim3((N + 255) / 256), dim3(256), 0, st, c->g, phi_nodes, phi_faces[0],
                               phi_faces[1], phi_faces[2], se0, se1, se2, c->flags[0], (double *)c->s[0][0],
                               (double *)c->s[0][1], (double *)c->s[0][2]);
        else
            hipLaunchKernelGGL(k_init<float>, dim3((N + 255) / 256), dim3(256), 0, st, c->g, phi_nodes, phi_faces[0],
                               phi_faces[1], phi_faces[2], se0, se1, se2, c->flags[0], (float *)c->s[0][0],
                               (float *)c->s[0][1], (float *)c->s[0][2]);
    }
    // both buffers must agree outside the band: copy the initial state to buffer 1
    size_t es = c->precision == EBIT_FP64 ? sizeof(double) : sizeof(float);
    bool ok = hipMemcpyAsync(c->flags[1], c->flags[0], (size_t)N, hipMemcpyDeviceToDevice, st) == hipSuccess;
    for (int e = 0; e < 3 && ok; ++e)
        ok = hipMemcpyAsync(c->s[1][e], c->s[0][e], (size_t)N * es, hipMemcpyDeviceToDevice, st) == hipSuccess;
    if (!ok) {
        free(c);
        return EBIT_EHIP;
    }
    int rc = init_lists(c, st);
    if (rc != EBIT_OK) {
        free(c);
        return rc;
    }
    *out = c;
    return EBIT_OK;
}

int ebit_advect_sweep(ebit_ctx *c, int dir, const void *U_dir, double g, double dt, void *stream)
{
    if (!c || !U_dir || dir < 0 || dir > 2) return EBIT_EINVAL;
    if (!(dt >= 0.0) || !isfinite(g)) return EBIT_EINVAL;
    if (c->precision == EBIT_FP64) return sweep_impl<double>(c, dir, U_dir, g, dt, S(stream));
    return sweep_impl<float>(c, dir, U_dir, g, dt, S(stream));
}

int ebit_front2vof(ebit_ctx *c, void *C, void *stream)
{
    if (!c || !C) return EBIT_EINVAL;
    if (c->precision == EBIT_FP64) return f2v_impl<double>(c, C, S(stream));
    return f2v_impl<float>(c, C, S(stream));
}

int ebit_stats(ebit_ctx *c, const void *C, ebit_stats_t *out, void *stream)
{
    if (!c || !C || !out) return EBIT_EINVAL;
    hipStream_t st = S(stream);
    hipLaunchKernelGGL(k_zero_marks, dim3(1), dim3(64), 0, st, c->w.stat);
    hipLaunchKernelGGL(k_stats_reduce, dim3(1), dim3(256), 0, st, c->w, c->g);
    if (c->precision == EBIT_FP64)
        hipLaunchKernelGGL(k_vol_partial<double>, dim3(kRedBlocks - 1), dim3(256), 0, st, (const double *)C,
                           c->flags[c->cur], c->n, c->w.part, c->w.stat);
    else
        hipLaunchKernelGGL(k_vol_partial<float>, dim3(kRedBlocks - 1), dim3(256), 0, st, (const float *)C,
                           c->flags[c->cur], c->n, c->w.part, c->w.stat);
    hipLaunchKernelGGL(k_vol_final, dim3(1), dim3(64), 0, st, c->w.part, kRedBlocks - 1);
    int rc = check_launch();
    if (rc != EBIT_OK) return rc;
    // kRedBlocks-1 partial sums; the final pass stores its result after them
    double vol[2];
    unsigned long long stat[ST_COUNT];
    if (hipMemcpyAsync(vol, c->w.part + 2 * (kRedBlocks - 1), sizeof(vol), hipMemcpyDeviceToHost, st) != hipSuccess)
        return EBIT_EHIP;
    if (hipMemcpyAsync(stat, c->w.stat, sizeof(stat), hipMemcpyDeviceToHost, st) != hipSuccess) return EBIT_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return EBIT_EHIP;
    out->volume = vol[0];
    out->volume_comp = vol[1];
    out->n_interfacial = c->fgen > 1 ? (int64_t)stat[ST_INTER] : 0;
    out->n_ambiguous = c->fgen > 1 ? (int64_t)stat[ST_AMB] : 0;
    out->n_markers[0] = (int64_t)stat[ST_MARK0];
    out->n_markers[1] = (int64_t)stat[ST_MARK1];
    out->n_markers[2] = (int64_t)stat[ST_MARK2];
    out->n_fallback = (int64_t)stat[ST_FALLBACK];
    out->n_multi = (int64_t)stat[ST_MULTI];
    out->n_cfl = (int64_t)stat[ST_CFL];
    out->n_merged = (int64_t)stat[ST_MERGED];
    out->n_active_cells = (int64_t)stat[ST_ACTIVE];
    out->n_annihilated = (int64_t)stat[ST_ANNIH];
    out->n_ambig_faces = (int64_t)stat[ST_AFACE];
    out->n_surrogate = c->fgen > 1 ? (int64_t)stat[ST_SURR] : 0;
    out->step_sweeps = (int64_t)(c->t - 2);
    // count after generation j: S1(j) = sum of delta up to j; summed over the
    // generations 1..K so far: (K + 1) S1 - sum of j delta_j
    const int64_t K = (int64_t)c->fgen - 1;
    out->n_interfacial_sum = (K + 1) * (int64_t)stat[ST_INTER] - (int64_t)stat[ST_INTER_SUM];
    const uint32_t cbits = (uint32_t)stat[ST_CMAX];
    float cm;
    memcpy(&cm, &cbits, sizeof(cm));
    out->max_courant = (double)cm;
    return out->n_cfl ? EBIT_ECFL : EBIT_OK;
}

int ebit_errors(ebit_ctx *c, const void *C, const void *C0, int reset, ebit_errors_t *out, void *stream)
{
    if (!c || !C || !C0 || !out) return EBIT_EINVAL;
    hipStream_t st = S(stream);
    const long N = (long)c->n * c->n * c->n;
    if (c->precision == EBIT_FP64)
        hipLaunchKernelGGL(k_err_partial<double>, dim3(kRedBlocks), dim3(256), 0, st, (const double *)C,
                           (const double *)C0, N, c->w.epart);
    else
        hipLaunchKernelGGL(k_err_partial<float>, dim3(kRedBlocks), dim3(256), 0, st, (const float *)C,
                           (const float *)C0, N, c->w.epart);
    hipLaunchKernelGGL(k_err_final, dim3(1), dim3(64), 0, st, c->w.epart, kRedBlocks);
    int rc = check_launch();
    if (rc != EBIT_OK) return rc;
    double tot[6];
    if (hipMemcpyAsync(tot, c->w.epart + 6 * kRedBlocks, sizeof(tot), hipMemcpyDeviceToHost, st) != hipSuccess)
        return EBIT_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return EBIT_EHIP;
    out->volume = tot[0] + tot[1];
    out->volume_ref = tot[2] + tot[3];
    out->l1_diff = tot[4] + tot[5];
    out->e_shape = out->volume_ref > 0.0 ? out->l1_diff / out->volume_ref : 0.0;
    if (reset) {
        c->mass_sum = 0.0;
        c->mass_n = 0;
    }
    if (out->volume_ref > 0.0) {
        c->mass_sum += fabs(out->volume - out->volume_ref) / out->volume_ref;
        c->mass_n += 1;
    }
    out->samples = c->mass_n;
    out->e_mass = c->mass_n ? c->mass_sum / (double)c->mass_n : 0.0;
    return EBIT_OK;
}

int ebit_current(const ebit_ctx *c) { return c ? c->cur : -1; }

int ebit_set_surrogate(ebit_ctx *c, const float *theta)
{
    if (!c) return EBIT_EINVAL;
    if (!theta) {
        c->surr = 0;
        return EBIT_OK;
    }
    // theta may have been written on any stream; the image is complete before the call returns
    if (hipDeviceSynchronize() != hipSuccess) return EBIT_EHIP;
    hipLaunchKernelGGL(k_surr_pack, dim3((kSurrPackThreads + 255) / 256), dim3(256), 0, (hipStream_t)0, theta, c->w.simg);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize((hipStream_t)0) != hipSuccess) return EBIT_EHIP;
    c->surr = 1;
    return EBIT_OK;
}

int ebit_surrogate_dataset(ebit_ctx *c, void *x_bf16, float *cout, int64_t cap, int64_t *count, void *stream)
{
    if (!c || !count || cap < 0) return EBIT_EINVAL;
    if (c->precision == EBIT_FP64) return dataset_impl<double>(c, x_bf16, cout, cap, count, S(stream));
    return dataset_impl<float>(c, x_bf16, cout, cap, count, S(stream));
}

int ebit_set_option(ebit_ctx *c, int option, int value)
{
    if (!c) return EBIT_EINVAL;
    if (option == EBIT_OPT_FULL_GRID) {
        c->full = value != 0;
        return EBIT_OK;
    }
    if (option == EBIT_OPT_TIMING) {
        if (value && !c->ev) {
            hipEvent_t *ev = (hipEvent_t *)calloc(2 * kTimed, sizeof(hipEvent_t));
            uint8_t *kind = (uint8_t *)calloc(kTimed, 1);
            if (!ev || !kind) { free(ev); free(kind); return EBIT_EINVAL; }
            for (int k = 0; k < 2 * kTimed; ++k) {
                if (hipEventCreate(&ev[k]) != hipSuccess) {
                    for (int j = 0; j < k; ++j) (void)hipEventDestroy(ev[j]);
                    free(ev);
                    free(kind);
                    return EBIT_EHIP;
                }
            }
            c->ev = ev;
            c->ev_kind = kind;
            c->ev_n = 0;
        }
        c->timing = value > 0 ? value : 0;
        c->tseen[0] = c->tseen[1] = c->tseen[2] = 0;
        return EBIT_OK;
    }
    if (option == EBIT_OPT_FUSE) {
        c->fuse = value != 0;
        return EBIT_OK;
    }
    if (option == EBIT_OPT_ORDER) {
        c->order = value != 0;
        return EBIT_OK;
    }
    if (option == EBIT_OPT_SUBLIST_CAP) {
        if (value < 0) return EBIT_EINVAL;
        if (c->t != 2 || c->fgen != 1) return EBIT_ESTATE;   // the lists are rebuilt: only before any work
        const int full = scap_for(c->n);
        if (hipDeviceSynchronize() != hipSuccess) return EBIT_EHIP;
        c->g.scap = value > 0 && value < full ? value : full;
        const int rc = init_lists(c, nullptr);
        if (rc != EBIT_OK) return rc;
        return hipDeviceSynchronize() == hipSuccess ? EBIT_OK : EBIT_EHIP;
    }
    return EBIT_EINVAL;
}

int ebit_timing(ebit_ctx *c, ebit_timing_t *out)
{
    if (!c || !out) return EBIT_EINVAL;
    memset(out, 0, sizeof(*out));
    if (!c->ev || c->ev_n == 0) return EBIT_OK;
    if (hipEventSynchronize(c->ev[2 * c->ev_n - 1]) != hipSuccess) return EBIT_EHIP;
    for (int k = 0; k < c->ev_n; ++k) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]) != hipSuccess) return EBIT_EHIP;
        if (c->ev_kind[k] == 0) { out->sweeps++; out->sweep_ms += ms; }
        else if (c->ev_kind[k] == 1) { out->f2v++; out->f2v_ms += ms; }
        else { out->fused++; out->fused_ms += ms; }
    }
    c->ev_n = 0;
    return EBIT_OK;
}

int ebit_advance(ebit_ctx *c, int32_t nsteps, const void *const *U, const double *g, double dt, void *C,
                 void *stream)
{
    if (!c || nsteps < 0 || !U || !U[0] || !U[1] || !U[2] || (nsteps > 0 && !g)) return EBIT_EINVAL;
    // a Front2VOF due before the next x sweep goes into that sweep's launch
    // (with the surrogate: its classify pass; the network's pass follows)
    const int fuse = C && c->fuse;
    int pending = 0;
    for (int k = 0; k < nsteps; ++k) {
        for (int d = 0; d < 3; ++d) {
            int rc;
            // the sweep after this one (known within the call): its band takes
            // only the neighbours it can change
            c->next_dir = d < 2 ? d + 1 : (k + 1 < nsteps ? 0 : -1);
            if (d == 0 && pending) {
                if (!(dt >= 0.0) || !isfinite(g[k])) rc = EBIT_EINVAL;
                else rc = c->precision == EBIT_FP64 ? f2v_sweep_x_impl<double>(c, C, U[0], g[k], dt, S(stream))
                                                    : f2v_sweep_x_impl<float>(c, C, U[0], g[k], dt, S(stream));
                pending = 0;
            } else {
                rc = ebit_advect_sweep(c, d, U[d], g[k], dt, stream);
            }
            c->next_dir = -1;
            if (rc != EBIT_OK) return rc;
        }
        if (C) {
            if (fuse && k + 1 < nsteps) {
                pending = 1;
            } else {
                int rc = ebit_front2vof(c, C, stream);
                if (rc != EBIT_OK) return rc;
            }
        }
    }
    return EBIT_OK;
}

void ebit_destroy(ebit_ctx *c)
{
    if (!c) return;
    if (c->ev) {
        for (int k = 0; k < 2 * kTimed; ++k) (void)hipEventDestroy(c->ev[k]);
        free(c->ev);
        free(c->ev_kind);
    }
    free(c);
}

}  // extern "C"
