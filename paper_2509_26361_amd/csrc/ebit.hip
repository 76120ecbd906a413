// ebit.hip -- MI355X (gfx950) implementation of the EBIT hot path behind the
// C ABI of include/ebit.h: marker initialisation, the direction-split
// advection sweep and Front2VOF (Pan et al., arXiv 2509.26361, secs. 2.1-2.5,
// 3.1), plus a deterministic compensated volume reduction.
//
// Work is restricted to a band of 4x4x4-node bricks around the interface: a
// brick is processed when it or one of its 26 neighbours held a marker before
// the current or the previous sweep (markers move at most one cell per sweep
// and every output depends only on markers within three cells).  Outside the
// band the state is constant, so the result equals a full-grid sweep.  One
// wavefront handles one brick (64 nodes, one lane per node).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/ebit.h"
#include "ebit_device.h"

using namespace ebit;

namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kBlock = 64 * kWavesPerBlock;
constexpr int kRedBlocks = 1024;

enum {
    ST_FALLBACK = 0, ST_MULTI, ST_CFL, ST_MERGED, ST_INTERFACIAL, ST_AMBIG, ST_ACTIVE,
    ST_MARK0, ST_MARK1, ST_MARK2, ST_SWEEPS, ST_INTER_SUM, ST_COUNT = 16
};

// device work space carved out of the caller's scratch buffer
struct Work {
    uint8_t *bmark;      // brick holds a marker (after the last sweep that processed it)
    uint8_t *coreprev;   // brick was in the dilated marker set before the previous sweep
    uint8_t *touched;    // brick written since the last Front2VOF
    int32_t *list;       // active bricks
    uint32_t *cnt;       // [2] list lengths, used alternately
    unsigned long long *stat;   // ST_*
    double *part;        // 2 * kRedBlocks reduction partials
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t work_layout(int n, Work *w, char *base)
{
    size_t nb = (size_t)(n / 4) * (n / 4) * (n / 4);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return base ? base + o : nullptr; };
    char *p;
    p = take(nb); if (w) w->bmark = (uint8_t *)p;
    p = take(nb); if (w) w->coreprev = (uint8_t *)p;
    p = take(nb); if (w) w->touched = (uint8_t *)p;
    p = take(nb * 4); if (w) w->list = (int32_t *)p;
    p = take(2 * sizeof(uint32_t)); if (w) w->cnt = (uint32_t *)p;
    p = take(ST_COUNT * sizeof(unsigned long long)); if (w) w->stat = (unsigned long long *)p;
    p = take(2 * kRedBlocks * sizeof(double)); if (w) w->part = (double *)p;
    return off;
}

struct Geo {
    int n;
    int nb1;        // bricks per axis
    long nn;        // n*n
};

__device__ __forceinline__ void brick_node(const Geo &g, int b, int lane, int &x, int &y, int &z)
{
    int bx = b % g.nb1, by = (b / g.nb1) % g.nb1, bz = b / (g.nb1 * g.nb1);
    x = bx * 4 + (lane & 3);
    y = by * 4 + ((lane >> 2) & 3);
    z = bz * 4 + (lane >> 4);
}

__device__ __forceinline__ void wave_add(unsigned long long *dst, int v)
{
    // sum a per-lane count over the wave, one atomic per wave
    unsigned long long bal;
    int tot = 0;
#pragma unroll
    for (int bit = 0; bit < 4; ++bit) {
        bal = __ballot((v >> bit) & 1);
        tot += __popcll(bal) << bit;
    }
    if ((threadIdx.x & 63) == 0 && tot) atomicAdd(dst, (unsigned long long)tot);
}

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

// brick marks of a freshly initialised (or caller-filled) state; every brick
// is marked touched so the first Front2VOF covers the whole grid
__global__ __launch_bounds__(kBlock) void k_mark_all(Geo g, const uint8_t *__restrict__ fl, Work w, int nbricks)
{
    int b = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (b >= nbricks) return;
    int x, y, z;
    brick_node(g, b, lane, x, y, z);
    long q = x + (long)g.n * y + g.nn * z;
    unsigned long long bal = __ballot((fl[q] & 0x70) != 0);
    if (lane == 0) {
        w.bmark[b] = bal != 0;
        w.coreprev[b] = 0;
        w.touched[b] = 1;
    }
    if (b == 0 && lane == 0) {
        w.cnt[0] = 0;
        w.cnt[1] = 0;
#pragma unroll
        for (int t = 0; t < ST_COUNT; ++t) w.stat[t] = 0;
    }
}

// ---------------------------------------------------------------------------
// a1: band compaction
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool dilated(const Geo &g, const uint8_t *__restrict__ m, int b)
{
    int nb = g.nb1;
    int bx = b % nb, by = (b / nb) % nb, bz = b / (nb * nb);
    bool any = false;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
                any |= m[wrp(bx + dx, nb) + nb * (wrp(by + dy, nb) + nb * wrp(bz + dz, nb))] != 0;
    return any;
}

// Sweep work list: bricks in the dilated marker set now or before the
// previous sweep (full = every brick).  Appends to list, counter cnt[slot].
__global__ __launch_bounds__(256) void k_band_sweep(Geo g, Work w, int nbricks, int slot, int full)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    bool act = false;
    if (b < nbricks) {
        bool core = dilated(g, w.bmark, b);
        act = full || core || w.coreprev[b];
        w.coreprev[b] = core;
        if (act) w.touched[b] = 1;
    }
    // wave-aggregated append
    unsigned long long bal = __ballot(act);
    int lane = threadIdx.x & 63;
    uint32_t basei = 0;
    if (lane == 0 && bal) basei = atomicAdd(&w.cnt[slot], (uint32_t)__popcll(bal));
    basei = __shfl(basei, 0);
    if (act) {
        unsigned long long below = bal & ((1ull << lane) - 1ull);
        uint32_t at = basei + (uint32_t)__popcll(below);
        if (at < (uint32_t)nbricks) w.list[at] = b;
    }
}

// Front2VOF work list: bricks touched since the last Front2VOF, dilated
// (a cell reads edges of its +x/+y/+z neighbours).  Clears touched after a
// grid-wide pass: done by the Front2VOF kernel itself.
__global__ __launch_bounds__(256) void k_band_f2v(Geo g, Work w, int nbricks, int slot, int full)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    bool act = false;
    if (b < nbricks) act = full || dilated(g, w.touched, b);
    unsigned long long bal = __ballot(act);
    int lane = threadIdx.x & 63;
    uint32_t basei = 0;
    if (lane == 0 && bal) basei = atomicAdd(&w.cnt[slot], (uint32_t)__popcll(bal));
    basei = __shfl(basei, 0);
    if (act) {
        unsigned long long below = bal & ((1ull << lane) - 1ull);
        uint32_t at = basei + (uint32_t)__popcll(below);
        if (at < (uint32_t)nbricks) w.list[at] = b;
    }
    if (b == 0) {
        w.stat[ST_INTERFACIAL] = 0;
        w.stat[ST_AMBIG] = 0;
    }
}

__global__ void k_clear_touched(Work w, int nbricks)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nbricks) w.touched[b] = 0;
}

// ---------------------------------------------------------------------------
// a2-a4: one sweep along axis D (secs. 2.1-2.4)
// ---------------------------------------------------------------------------

template <typename T>
struct SweepArgs {
    Geo g;
    const uint8_t *fl;
    const T *s[3];
    uint8_t *flo;
    T *so[3];
    const T *U;
    T c;
    Work w;
    int slot;
};

template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs<T> a)
{
    constexpr int A1 = (D + 1) % 3, A2 = (D + 2) % 3;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int nwaves = gridDim.x * kWavesPerBlock;
    const int nbr = a.g.nb1 * a.g.nb1 * a.g.nb1;
    const int count = min((int)a.w.cnt[a.slot], nbr);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.w.cnt[a.slot ^ 1] = 0;              // for the next compaction
        atomicAdd(&a.w.stat[ST_ACTIVE], (unsigned long long)count * 64ull);
        atomicAdd(&a.w.stat[ST_SWEEPS], 1ull);
    }
    const int n = a.g.n;
    const long str[3] = {1, (long)n, a.g.nn};
    for (int t = wave; t < count; t += nwaves) {
        const int b = a.w.list[t];
        if ((unsigned)b >= (unsigned)nbr) continue;
        int P[3];
        brick_node(a.g, b, lane, P[0], P[1], P[2]);
        const long q = P[0] + str[1] * P[1] + str[2] * P[2];

        Plane<T, D, A1> p1;   // faces with normal A2
        p1.fl = a.fl; p1.sD = a.s[D]; p1.sA = a.s[A1]; p1.U = a.U; p1.c = a.c; p1.n = n;
        p1.ci = P[D]; p1.cj = P[A1]; p1.base = (long)P[A2] * str[A2]; p1.strD = str[D]; p1.strA = str[A1];
        Plane<T, D, A2> p2;   // faces with normal A1
        p2.fl = a.fl; p2.sD = a.s[D]; p2.sA = a.s[A2]; p2.U = a.U; p2.c = a.c; p2.n = n;
        p2.ci = P[D]; p2.cj = P[A2]; p2.base = (long)P[A1] * str[A1]; p2.strD = str[D]; p2.strA = str[A2];

        const uint8_t f0 = a.fl[q];
        int fb = 0, multi = 0, cfl = 0, merged = 0;

        // Courant check of the markers stored at this node
        {
            auto chk = [&](int e, const T *se) {
                if ((f0 >> (4 + e)) & 1) {
                    long q1 = q + (P[e] + 1 == n ? -(long)(n - 1) * str[e] : str[e]);
                    T s = se[q];
                    T U0 = a.U[q], U1 = a.U[q1];
                    T u = U0 + s * (U1 - U0);
                    T del = a.c * u;
                    if (fabs((double)del) > 1.0) cfl += 1;
                }
            };
            chk(0, a.s[0]);
            chk(1, a.s[1]);
            chk(2, a.s[2]);
        }

        // aligned markers and node colours (Fig. 4; annihilation, Fig. 5a)
        const int c00 = p1.newcol(0, 0);
        const int c10 = p1.newcol(1, 0);
        uint8_t out = (uint8_t)c00;
        T sd_new = T(0);
        {
            bool hm = p1.hhas(-1, 0), h0 = p1.hhas(0, 0), hp = p1.hhas(1, 0);
            double xm = hm ? p1.xd(-1, 0) : 0.0, x0 = h0 ? p1.xd(0, 0) : 0.0, xp = hp ? p1.xd(1, 0) : 0.0;
            bool lm = hm && xm >= 1.0, l0 = h0 && x0 >= 0.0 && x0 < 1.0, lp = hp && xp < 0.0;
            int k = (int)lm + (int)l0 + (int)lp;
            if (c00 != c10) {
                double v;
                if (k == 1) v = lm ? xm - 1.0 : (l0 ? x0 : xp + 1.0);
                else if (k == 3) {
                    double v0 = xm - 1.0, v1 = x0, v2 = xp + 1.0;
                    double lo = v0 < v1 ? v0 : v1, hi = v0 < v1 ? v1 : v0;
                    v = v2 < lo ? lo : (v2 > hi ? hi : v2);
                    merged += 1;
                } else {
                    v = 0.5;
                    fb += 1;
                }
                sd_new = clamp_frac<T>((T)v);
                out |= (uint8_t)(1u << (4 + D));
            } else if (k >= 2) {
                merged += 1;
            }
        }
        out |= (uint8_t)(f0 & (1u << (1 + D)));   // faces normal to D keep their colour

        // plane (D, A1): unaligned A1-edge and faces with normal A2
        T sa1_new = T(0);
        {
            const int c01 = p1.newcol(0, 1);
            if (c00 != c01) {
                sa1_new = p1.unaligned(fb, multi);
                out |= (uint8_t)(1u << (4 + A1));
            }
            const int c11 = p1.newcol(1, 1);
            int fc = (c00 == c10 && c00 == c01 && c00 == c11) ? c00 : p1.face_colour(c00);
            out |= (uint8_t)(fc << (1 + A2));
        }
        // plane (D, A2): unaligned A2-edge and faces with normal A1
        T sa2_new = T(0);
        {
            const int c01 = p2.newcol(0, 1);
            if (c00 != c01) {
                sa2_new = p2.unaligned(fb, multi);
                out |= (uint8_t)(1u << (4 + A2));
            }
            const int c11 = p2.newcol(1, 1);
            int fc = (c00 == c10 && c00 == c01 && c00 == c11) ? c00 : p2.face_colour(c00);
            out |= (uint8_t)(fc << (1 + A1));
        }
        a.flo[q] = out;
        a.so[D][q] = sd_new;
        a.so[A1][q] = sa1_new;
        a.so[A2][q] = sa2_new;

        unsigned long long bal = __ballot((out & 0x70) != 0);
        if (lane == 0) a.w.bmark[b] = bal != 0;
        if (__ballot(fb | multi | cfl | merged)) {
            wave_add(&a.w.stat[ST_FALLBACK], fb);
            wave_add(&a.w.stat[ST_MULTI], multi);
            wave_add(&a.w.stat[ST_CFL], cfl);
            wave_add(&a.w.stat[ST_MERGED], merged);
        }
    }
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

template <typename T>
struct F2VArgs {
    Geo g;
    const uint8_t *fl;
    const T *s[3];
    T *C;
    Work w;
    int slot;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_f2v(F2VArgs<T> a)
{
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int nwaves = gridDim.x * kWavesPerBlock;
    const int nbr = a.g.nb1 * a.g.nb1 * a.g.nb1;
    const int count = min((int)a.w.cnt[a.slot], nbr);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.w.cnt[a.slot ^ 1] = 0;
    const int n = a.g.n;
    for (int t = wave; t < count; t += nwaves) {
        const int b = a.w.list[t];
        if ((unsigned)b >= (unsigned)nbr) continue;
        int x, y, z;
        brick_node(a.g, b, lane, x, y, z);
        const int x1 = x + 1 == n ? 0 : x + 1, y1 = y + 1 == n ? 0 : y + 1, z1 = z + 1 == n ? 0 : z + 1;
        const long nn = a.g.nn;
        long qc[8];
        qc[0] = x + (long)n * y + nn * z;
        qc[1] = x1 + (long)n * y + nn * z;
        qc[2] = x + (long)n * y1 + nn * z;
        qc[3] = x1 + (long)n * y1 + nn * z;
        qc[4] = x + (long)n * y + nn * z1;
        qc[5] = x1 + (long)n * y + nn * z1;
        qc[6] = x + (long)n * y1 + nn * z1;
        qc[7] = x1 + (long)n * y1 + nn * z1;
        uint8_t f[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) f[k] = a.fl[qc[k]];
        int colb = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) colb |= (f[k] & 1) << k;
        // edges: id 4e + oA + 2 oB starts at corner with offset oA, oB
        int has = 0;
        T sv[12];
#pragma unroll
        for (int id = 0; id < 12; ++id) {
            int e = id >> 2, oA = id & 1, oB = (id >> 1) & 1;
            int ox = e == 0 ? 0 : oA, oy = e == 1 ? 0 : (e == 0 ? oA : oB), oz = e == 2 ? 0 : oB;
            int k = ox + 2 * oy + 4 * oz;
            int hb = (f[k] >> (4 + e)) & 1;
            has |= hb << id;
            sv[id] = hb ? a.s[e][qc[k]] : T(0);
        }
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
            // segments kept for the multi-loop path: start/end edge ids
            int segs = 0;
            uint8_t sst[12], sen[12];
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
                    sst[segs] = (uint8_t)is;
                    sen[segs] = (uint8_t)ie;
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
                        int is = sst[k], ie = sen[k];
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
        a.C[qc[0]] = C;
        if (__ballot(inter)) {
            wave_add(&a.w.stat[ST_INTERFACIAL], inter);
            wave_add(&a.w.stat[ST_INTER_SUM], inter);
            wave_add(&a.w.stat[ST_AMBIG], amb);
        }
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
__global__ __launch_bounds__(256) void k_vol_partial(const T *__restrict__ C, const uint8_t *__restrict__ fl, long N,
                                                     double *__restrict__ part, unsigned long long *__restrict__ stat)
{
    __shared__ double ss[256], sc[256];
    double s = 0.0, c = 0.0;
    int m0 = 0, m1 = 0, m2 = 0;
    long stride = (long)gridDim.x * blockDim.x;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < N; q += stride) {
        neumaier_add(s, c, (double)C[q]);
        uint8_t f = fl[q];
        m0 += (f >> 4) & 1;
        m1 += (f >> 5) & 1;
        m2 += (f >> 6) & 1;
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
    }
    if ((threadIdx.x & 63) == 0) {
        if (m0) atomicAdd(&stat[ST_MARK0], (unsigned long long)m0);
        if (m1) atomicAdd(&stat[ST_MARK1], (unsigned long long)m1);
        if (m2) atomicAdd(&stat[ST_MARK2], (unsigned long long)m2);
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

__global__ void k_zero_marks(unsigned long long *stat)
{
    if (threadIdx.x < 3) stat[ST_MARK0 + threadIdx.x] = 0;
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
    int nbricks;
    int seq;            // compaction sequence number: list counter slot = seq & 1
    int full;           // process every brick
    const void *lastC;  // C array of the previous Front2VOF
    int grid_waves;     // persistent grid size (waves)
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

int persistent_blocks(const ebit_ctx *c)
{
    int need = (c->nbricks + kWavesPerBlock - 1) / kWavesPerBlock;
    int cap = c->grid_waves / kWavesPerBlock;
    return need < cap ? (need > 0 ? need : 1) : cap;
}

template <typename T, int D>
void launch_sweep(ebit_ctx *c, const void *U, T cf, hipStream_t st)
{
    SweepArgs<T> a;
    a.g = c->g;
    a.fl = c->flags[c->cur];
    a.flo = c->flags[c->cur ^ 1];
    for (int e = 0; e < 3; ++e) {
        a.s[e] = (const T *)c->s[c->cur][e];
        a.so[e] = (T *)c->s[c->cur ^ 1][e];
    }
    a.U = (const T *)U;
    a.c = cf;
    a.w = c->w;
    a.slot = c->seq & 1;
    hipLaunchKernelGGL((k_sweep<T, D>), dim3(persistent_blocks(c)), dim3(kBlock), 0, st, a);
}

template <typename T>
int sweep_impl(ebit_ctx *c, int dir, const void *U, double g, double dt, hipStream_t st)
{
    // compaction of this sweep's bricks
    int slot = c->seq & 1;
    hipLaunchKernelGGL(k_band_sweep, dim3((c->nbricks + 255) / 256), dim3(256), 0, st, c->g, c->w, c->nbricks, slot,
                       c->full);
    double cd = (dt * (double)c->n) * g;
    T cf = (T)cd;
    if (dir == 0) launch_sweep<T, 0>(c, U, cf, st);
    else if (dir == 1) launch_sweep<T, 1>(c, U, cf, st);
    else launch_sweep<T, 2>(c, U, cf, st);
    c->seq++;
    c->cur ^= 1;
    return check_launch();
}

template <typename T>
int f2v_impl(ebit_ctx *c, void *C, hipStream_t st)
{
    int full = c->full || C != c->lastC;
    int slot = c->seq & 1;
    hipLaunchKernelGGL(k_band_f2v, dim3((c->nbricks + 255) / 256), dim3(256), 0, st, c->g, c->w, c->nbricks, slot, full);
    F2VArgs<T> a;
    a.g = c->g;
    a.fl = c->flags[c->cur];
    for (int e = 0; e < 3; ++e) a.s[e] = (const T *)c->s[c->cur][e];
    a.C = (T *)C;
    a.w = c->w;
    a.slot = slot;
    hipLaunchKernelGGL((k_f2v<T>), dim3(persistent_blocks(c)), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_clear_touched, dim3((c->nbricks + 255) / 256), dim3(256), 0, st, c->w, c->nbricks);
    c->seq++;
    c->lastC = C;
    return check_launch();
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
    default: return "unknown error";
    }
}

int ebit_init(ebit_ctx **out, const ebit_desc *d, const double *phi_nodes, const double *const *phi_faces,
              const double *const *s_exact, void *stream)
{
    if (!out || !d) return EBIT_EINVAL;
    if (d->n < 8 || d->n % 4 || d->n > 2048) return EBIT_EINVAL;
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
    c->nbricks = c->g.nb1 * c->g.nb1 * c->g.nb1;
    c->seq = 0;
    c->full = 0;
    c->lastC = nullptr;
    c->grid_waves = 256 * 16;   // 16 waves per CU across 256 CUs
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
    hipLaunchKernelGGL(k_mark_all, dim3((c->nbricks + kWavesPerBlock - 1) / kWavesPerBlock), dim3(kBlock), 0, st,
                       c->g, c->flags[0], c->w, c->nbricks);
    int rc = check_launch();
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
    long N = (long)c->n * c->n * c->n;
    hipLaunchKernelGGL(k_zero_marks, dim3(1), dim3(64), 0, st, c->w.stat);
    if (c->precision == EBIT_FP64)
        hipLaunchKernelGGL(k_vol_partial<double>, dim3(kRedBlocks - 1), dim3(256), 0, st, (const double *)C,
                           c->flags[c->cur], N, c->w.part, c->w.stat);
    else
        hipLaunchKernelGGL(k_vol_partial<float>, dim3(kRedBlocks - 1), dim3(256), 0, st, (const float *)C,
                           c->flags[c->cur], N, c->w.part, c->w.stat);
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
    out->n_interfacial = (int64_t)stat[ST_INTERFACIAL];
    out->n_ambiguous = (int64_t)stat[ST_AMBIG];
    out->n_markers[0] = (int64_t)stat[ST_MARK0];
    out->n_markers[1] = (int64_t)stat[ST_MARK1];
    out->n_markers[2] = (int64_t)stat[ST_MARK2];
    out->n_fallback = (int64_t)stat[ST_FALLBACK];
    out->n_multi = (int64_t)stat[ST_MULTI];
    out->n_cfl = (int64_t)stat[ST_CFL];
    out->n_merged = (int64_t)stat[ST_MERGED];
    out->n_active_cells = (int64_t)stat[ST_ACTIVE];
    out->step_sweeps = (int64_t)stat[ST_SWEEPS];
    out->n_interfacial_sum = (int64_t)stat[ST_INTER_SUM];
    return out->n_cfl ? EBIT_ECFL : EBIT_OK;
}

int ebit_current(const ebit_ctx *c) { return c ? c->cur : -1; }

int ebit_set_option(ebit_ctx *c, int option, int value)
{
    if (!c) return EBIT_EINVAL;
    if (option == EBIT_OPT_FULL_GRID) {
        c->full = value != 0;
        return EBIT_OK;
    }
    return EBIT_EINVAL;
}

void ebit_destroy(ebit_ctx *c) { free(c); }

}  // extern "C"
