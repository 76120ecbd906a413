// ebit_device.h -- device-side building blocks of the EBIT hot path for gfx950.
//
// Geometry of the state (paper sec. 2.3, Fig. 6b): edge fractions s_x,s_y,s_z,
// vertex colour, face-centre colours, all indexed by the lowest node of the
// edge/face/cell, i + n*(j + n*k), periodic.  Flag bits: 0 node colour,
// 1+a face colour (normal a), 4+e marker on the edge along e.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ebit {

template <typename T> struct Lim;
template <> struct Lim<double> { static constexpr double smax = 0.9999999999999998; };   // 1 - 2^-52
template <> struct Lim<float> { static constexpr float smax = 0.99999994f; };             // 1 - 2^-24

__device__ __forceinline__ int wrp(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T>
__device__ __forceinline__ T clamp_frac(T v)
{
    if (!(v >= T(0))) v = T(0);
    if (v > Lim<T>::smax) v = Lim<T>::smax;
    return v;
}

// Crossing height of the segment P2-P3 (P2x < X0 <= P3x) with the line X = X0.
template <typename T>
__device__ __forceinline__ T line_cross(T X0, T P2x, T P2y, T P3x, T P3y)
{
    T t = X0 - P2x;
    T dy = P3y - P2y;
    T dx = P3x - P2x;
    T w = t * dy;
    return P2y + w / dx;
}

// Circle through T, P2, P3 (paper sec. 2.1, Fig. 2): root on the line X = 0
// lying on the arc P2..P3 that avoids T, i.e. on the far side of the chord
// from T.  u is the centre relative to P2, x0 = -P2x the line relative to P2;
// the roots are P2y + u_y -+ sqrt(u_y^2 - w), w = x0 (x0 - 2 u_x), the one
// nearer P2 taken in conjugate form.  Returns false for a straight line
// (collinear points or radius >= 1e6 cells).
template <typename T>
__device__ __forceinline__ bool circle_root(T Tx, T Ty, T P2x, T P2y, T P3x, T P3y, T &root, T &r2)
{
    T bx = P3x - P2x, by = P3y - P2y;
    T cx = Tx - P2x, cy = Ty - P2y;
    T D = T(2) * (bx * cy - by * cx);
    if (D == T(0)) return false;
    T B2 = bx * bx + by * by;
    T C2 = cx * cx + cy * cy;
    T ux = (cy * B2 - by * C2) / D;
    T uy = (bx * C2 - cx * B2) / D;
    r2 = ux * ux + uy * uy;
    if (!(r2 < T(1e12))) return false;
    T x0 = -P2x;
    T w = x0 * (x0 - T(2) * ux);
    T q = uy * uy - w;
    T t;
    if (!(q > T(0))) {
        t = uy;
    } else {
        T sq = sqrt(q);
        if (D > T(0)) t = uy > T(0) ? w / (uy + sq) : uy - sq;
        else t = uy < T(0) ? w / (uy - sq) : uy + sq;
    }
    root = P2y + t;
    return true;
}

// New unaligned marker height from the advected segment P2-P3 and its
// polyline neighbours P1 (of P2) and P4 (of P3): a marker already on the line
// stays; else the mean of the 1-2-3 and 2-3-4 circle roots, or the larger
// circle's root when r_max / r_min > 10 (paper sec. 2.1); the straight
// crossing `key` when a circle degenerates or the fit leaves the edge.
template <typename T>
__device__ __forceinline__ T fit_height(T P1x, T P1y, T P2x, T P2y, T P3x, T P3y, T P4x, T P4y, T key)
{
    if (P3x == T(0)) return clamp_frac<T>(P3y);
    T yA = T(0), rA2 = T(0), yB = T(0), rB2 = T(0), y;
    bool okA = circle_root<T>(P1x, P1y, P2x, P2y, P3x, P3y, yA, rA2);
    bool okB = circle_root<T>(P4x, P4y, P2x, P2y, P3x, P3y, yB, rB2);
    if (okA && okB) {
        if (rA2 > T(100) * rB2) y = yA;
        else if (rB2 > T(100) * rA2) y = yB;
        else y = T(0.5) * (yA + yB);
    } else {
        y = key;
    }
    if (!(y >= T(0) && y < T(1))) y = key;
    return clamp_frac<T>(y);
}

// One 2D problem of a sweep (paper sec. 2.3) seen from one task node: the
// plane spanned by the sweep axis D ("X") and an axis A ("Y", chosen at run
// time) through the node.  Offsets (i, j) are relative to the node.
// Horizontal edges H(i,j) run along D (aligned markers), vertical edges V(i,j)
// along A (unaligned); face Q(i,j) spans [i,i+1] x [j,j+1] and has normal B.
// Everything is read from the old state in global memory, in three rounds of
// independent loads: the flags of offsets i in [-3, 2], j in [-1, 2]; then the
// markers of the three candidate faces; then, for a new unaligned marker, the
// two polyline neighbours of the chosen segment.
// SPARSE: the first round reads only the entries of existing markers (fewer
// cache lines fetched; more registers)
template <typename T, int D, int SPARSE>
struct PlaneTask {
    const uint8_t *__restrict__ fl;
    const T *__restrict__ sD;     // fractions of the H markers
    const T *__restrict__ sA;     // fractions of the V markers
    const T *__restrict__ U;      // D-velocity at nodes
    T c;                          // (dt n) g
    int n;
    int ci, cj;                   // the node's coordinates along D and A
    uint32_t strD, strA, base;    // index strides of D and A; offset of the B coordinate (n <= 1024)
    int hb, vb, fb;               // flag bits: H marker, V marker, colour of Q(i,j)
    uint32_t xo[6], yo[4];        // index offsets of i = -3..2 along D and of j = -1..2 along A (+ base)
    // bits of the flags of offsets i = -3..2, j = -1..2 at bit (i + 3) + 6 (j + 1):
    uint32_t mH, mV, mF, mC;      // H marker, V marker, colour of Q(i,j), node colour

    __device__ __forceinline__ uint32_t node(int i, int j) const
    {
        return __umul24((uint32_t)wrp(ci + i, n), strD) + __umul24((uint32_t)wrp(cj + j, n), strA) + base;
    }
    static __device__ __forceinline__ int bit(int i, int j) { return (i + 3) + 6 * (j + 1); }
    __device__ __forceinline__ void fetch_flags()
    {
#pragma unroll
        for (int i = 0; i < 6; ++i) xo[i] = __umul24((uint32_t)wrp(ci + i - 3, n), strD);
#pragma unroll
        for (int j = 0; j < 4; ++j) yo[j] = __umul24((uint32_t)wrp(cj + j - 1, n), strA) + base;
        uint32_t b[24];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 6; ++i) b[i + 6 * j] = fl[xo[i] + yo[j]];
        mH = mV = mF = mC = 0;
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            mH |= ((b[k] >> hb) & 1u) << k;
            mV |= ((b[k] >> vb) & 1u) << k;
            mF |= ((b[k] >> fb) & 1u) << k;
            mC |= (b[k] & 1u) << k;
        }
    }
    __device__ __forceinline__ int hhas(int i, int j) const { return (mH >> bit(i, j)) & 1; }
    __device__ __forceinline__ int vhas(int i, int j) const { return (mV >> bit(i, j)) & 1; }
    // segments of Q(fi,fj) in the old state (sec. 2.2, 2.4), packed: bits 0-1 /
    // 2-3 the sides of the first segment (lower first), 4-5 / 6-7 the second,
    // 8-9 the number of segments.  A four-marker face cuts off the corners
    // whose colour differs from its centre colour.
    __device__ __forceinline__ int pairs(int fi, int fj) const
    {
        const int k00 = bit(fi, fj);
        const int h0 = (mH >> k00) & 1, v1 = (mV >> (k00 + 1)) & 1;
        const int h2 = (mH >> (k00 + 6)) & 1, v3 = (mV >> k00) & 1;
        const int m = h0 + v1 + h2 + v3;
        if (m == 2) {
            const int lo = h0 ? 0 : (v1 ? 1 : 2);
            const int hi = v3 ? 3 : (h2 ? 2 : 1);
            return lo | (hi << 2) | (1 << 8);
        }
        if (m == 4) {
            const int c00 = (mC >> k00) & 1, ff = (mF >> k00) & 1;
            return ff == c00 ? (0 | (1 << 2) | (2 << 4) | (3 << 6) | (2 << 8))
                             : (0 | (3 << 2) | (1 << 4) | (2 << 6) | (2 << 8));
        }
        return 0;
    }
    static __device__ __forceinline__ int nseg(int pk) { return pk >> 8; }
    static __device__ __forceinline__ int side_a(int pk, int t) { return (pk >> (4 * t)) & 3; }
    static __device__ __forceinline__ int side_b(int pk, int t) { return (pk >> (4 * t + 2)) & 3; }

    // far end, in the neighbouring face, of the segment through `side`'s
    // marker: the face (ni, nj) and its side
    __device__ __forceinline__ void neighbour(int fi, int fj, int side, int &ni, int &nj, int &other) const
    {
        ni = side == 1 ? fi + 1 : (side == 3 ? fi - 1 : fi);
        nj = side == 0 ? fj - 1 : (side == 2 ? fj + 1 : fj);
        const int ns = (side + 2) & 3;
        const int pk = pairs(ni, nj);
        other = ns;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (t >= nseg(pk)) break;
            if (side_a(pk, t) == ns) other = side_b(pk, t);
            else if (side_b(pk, t) == ns) other = side_a(pk, t);
        }
    }
    // where the marker of a side of Q(fi,fj) is stored: fraction array, its
    // node, the node across the edge (for the velocity), and the point's
    // integer offsets
    __device__ __forceinline__ void locate(int fi, int fj, int side, bool &hz, uint32_t &q, uint32_t &q1, int &xi,
                                           int &yj) const
    {
        hz = side == 0 || side == 2;
        xi = side == 1 ? fi + 1 : fi;
        yj = side == 2 ? fj + 1 : fj;
        q = node(xi, yj);
        q1 = hz ? node(xi + 1, yj) : node(xi, yj + 1);
    }
    // advanced positions of two markers given by locate(), loads first
    __device__ __forceinline__ void two_points(int fa, int fja, int sa, int fb, int fjb, int sb, double &Xa, double &Ya,
                                              double &Xb, double &Yb) const
    {
        bool ha, hb;
        uint32_t qa, qa1, qb, qb1;
        int xa, ya, xb, yb;
        locate(fa, fja, sa, ha, qa, qa1, xa, ya);
        locate(fb, fjb, sb, hb, qb, qb1, xb, yb);
        const T s_a = ha ? sD[qa] : sA[qa], s_b = hb ? sD[qb] : sA[qb];
        const T ua0 = U[qa], ua1 = U[qa1], ub0 = U[qb], ub1 = U[qb1];
        const T dela = c * (ua0 + s_a * (ua1 - ua0)), delb = c * (ub0 + s_b * (ub1 - ub0));
        if (ha) { Xa = (double)xa + ((double)s_a + (double)dela); Ya = (double)ya; }
        else { Xa = (double)xa + (double)dela; Ya = (double)ya + (double)s_a; }
        if (hb) { Xb = (double)xb + ((double)s_b + (double)delb); Yb = (double)yb; }
        else { Xb = (double)xb + (double)delb; Yb = (double)yb + (double)s_b; }
    }

    // Geometry (advected positions, crossings, circle fits) runs in FP64 in
    // both precisions; the FP32 form rounds only the velocity interpolation
    // and the stored result to FP32.
    // The task of one node in this plane (sec. 2.1, 2.3).  Always: the colour
    // at the centre of Q(0,0) relative to the advected polyline -- start from
    // the node's new colour c00, flip for aligned markers landing in [0, 1/2)
    // on the bottom line and for advected segments of faces -1..1 crossing
    // X = 1/2 below Y = 1/2 (returned).  With `unal` (the new end colours of
    // V(0,0) differ): the new marker on V(0,0) -- crossings of X = 0 by the
    // advected old segments of faces -2..0 of the row, the median one (by
    // height) refined by the circle fit (*sval).  Faces -2..1 of the row share
    // one round of loads, issued before any arithmetic.
    __device__ __forceinline__ int run(int unal, int c00, T &sval, int &fallback, int &multi) const
    {
        // velocities at nodes (k - 2, r), k = 0..4, r = 0, 1; fractions of H(f - 2, r),
        // f = 0..3, and of V(k - 2, 0)
        uint32_t qn[5][2];
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int r = 0; r < 2; ++r) qn[k][r] = xo[k + 1] + yo[r + 1];
        // every entry (a missing marker reads a valid entry, masked below), or
        // with SPARSE only those of existing markers (the others stay 0)
        T Un[5][2], sh_[4][2], sv_[5];
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const bool need = (k < 4 && hhas(k - 2, r)) || (k > 0 && hhas(k - 3, r)) || vhas(k - 2, 0);
                Un[k][r] = !SPARSE || need ? U[qn[k][r]] : T(0);
            }
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int r = 0; r < 2; ++r) sh_[f][r] = !SPARSE || hhas(f - 2, r) ? sD[qn[f][r]] : T(0);
#pragma unroll
        for (int k = 0; k < 5; ++k) sv_[k] = !SPARSE || vhas(k - 2, 0) ? sA[qn[k][0]] : T(0);
        // advected markers (X, Y relative to the node)
        double Hx[4][2], Vx[5], Vy[5];
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const T sx = sh_[f][r], u0 = Un[f][r];
                const T del = c * (u0 + sx * (Un[f + 1][r] - u0));
                Hx[f][r] = hhas(f - 2, r) ? (double)(f - 2) + ((double)sx + (double)del) : 0.0;
            }
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const T sy = sv_[k], u0 = Un[k][0];
            const T del = c * (u0 + sy * (Un[k][1] - u0));
            const bool v = vhas(k - 2, 0);
            Vx[k] = v ? (double)(k - 2) + (double)del : 0.0;
            Vy[k] = v ? 0.0 + (double)sy : 0.0;
        }
        // side of face f - 2 (see point())
        auto pt = [&](int f, int side, double &X, double &Y) {
            X = side == 0 ? Hx[f][0] : (side == 2 ? Hx[f][1] : (side == 3 ? Vx[f] : Vx[f + 1]));
            Y = side == 0 ? 0.0 : (side == 2 ? 1.0 : (side == 3 ? Vy[f] : Vy[f + 1]));
        };
        int pk[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) pk[f] = pairs(f - 2, 0);
        // crossing of segment t of face f with the line X = x0 (from the endpoint left of
        // the line to the one right of it); false if the segment does not cross it
        auto cross = [&](int f, int t, double x0, double &key) -> bool {
            if (t >= nseg(pk[f])) return false;
            double Ax, Ay, Bx, By;
            pt(f, side_a(pk[f], t), Ax, Ay);
            pt(f, side_b(pk[f], t), Bx, By);
            const bool sa = x0 <= Ax, sb = x0 <= Bx;
            if (sa == sb) return false;
            const double Lx = sa ? Bx : Ax, Ly = sa ? By : Ay, Rx = sa ? Ax : Bx, Ry = sa ? Ay : By;
            key = line_cross<double>(x0, Lx, Ly, Rx, Ry);
            return true;
        };
        // face-centre colour (faces -1..1)
        int par = c00;
#pragma unroll
        for (int f = 1; f < 4; ++f) {
            if (!hhas(f - 2, 0)) continue;
            const double X = Hx[f][0];
            if (0.0 <= X && X < 0.5) par ^= 1;
        }
#pragma unroll
        for (int f = 1; f < 4; ++f)
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                double y;
                if (cross(f, t, 0.5, y) && y < 0.5) par ^= 1;
            }
        if (!unal) return par;
        // new marker on V(0,0) (faces -2..0)
        double key[6];
        bool ok[6];
        int m = 0;
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                key[2 * f + t] = 0.0;
                ok[2 * f + t] = cross(f, t, 0.0, key[2 * f + t]);
                m += ok[2 * f + t] ? 1 : 0;
            }
        if ((m & 1) == 0) {          // no odd crossing set: keep the edge valid
            fallback += 1;
            sval = T(0.5);
            return par;
        }
        int pick = 0;
        if (m == 1) {
#pragma unroll
            for (int c0 = 5; c0 >= 0; --c0)
                if (ok[c0]) pick = c0;
        } else {
            multi += 1;
            // the median crossing by height (ties: enumeration order)
#pragma unroll
            for (int c0 = 0; c0 < 6; ++c0) {
                if (!ok[c0]) continue;
                int rank = 0;
#pragma unroll
                for (int c1 = 0; c1 < 6; ++c1)
                    if (ok[c1] && (key[c1] < key[c0] || (key[c1] == key[c0] && c1 < c0))) ++rank;
                if (rank == (m >> 1)) pick = c0;
            }
        }
        // the chosen segment, selected with compile-time indices (no scratch)
        const int fo = (pick >> 1) - 2;
        int sa_ = 0, sb_ = 0;
        double Ax = 0.0, Ay = 0.0, Bx = 0.0, By = 0.0;
        double kp = 0.0;
#pragma unroll
        for (int c0 = 0; c0 < 6; ++c0) {
            if (c0 != pick) continue;
            sa_ = side_a(pk[c0 >> 1], c0 & 1);
            sb_ = side_b(pk[c0 >> 1], c0 & 1);
            pt(c0 >> 1, sa_, Ax, Ay);
            pt(c0 >> 1, sb_, Bx, By);
            kp = key[c0];
        }
        int s2, s3;
        double P2x, P2y, P3x, P3y;
        if (0.0 <= Ax) { s2 = sb_; s3 = sa_; P2x = Bx; P2y = By; P3x = Ax; P3y = Ay; }
        else { s2 = sa_; s3 = sb_; P2x = Ax; P2y = Ay; P3x = Bx; P3y = By; }
        double P1x, P1y, P4x, P4y;
        int n1i, n1j, n1s, n4i, n4j, n4s;
        neighbour(fo, 0, s2, n1i, n1j, n1s);
        neighbour(fo, 0, s3, n4i, n4j, n4s);
        two_points(n1i, n1j, n1s, n4i, n4j, n4s, P1x, P1y, P4x, P4y);
        sval = clamp_frac<T>((T)fit_height<double>(P1x, P1y, P2x, P2y, P3x, P3y, P4x, P4y, kp));
        return par;
    }
};

}  // namespace ebit
