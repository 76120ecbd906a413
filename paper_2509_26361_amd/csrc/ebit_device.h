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

// One 2D problem of a sweep (paper sec. 2.3): the plane spanned by the sweep
// axis D ("X") and axis A ("Y") through a node.  Offsets (i, j) are relative
// to that node.  Horizontal edges H(i,j) run along D (aligned markers),
// vertical edges V(i,j) along A (unaligned); face Q(i,j) spans [i,i+1] x
// [j,j+1] and has normal B.  The accessor `Acc` supplies, per node offset:
//   f(i,j)    old flags (bit 7: the node's new colour after this sweep)
//   xd(i,j)   s + delta of the D-edge marker (decision precision, double)
//   dva(i,j)  delta of the A-edge marker (double)
//   sa(i,j)   fraction of the A-edge marker
template <typename T, int D, int A, class Acc>
struct PlaneAlg {
    static constexpr int B = 3 - D - A;
    Acc acc;

    __device__ __forceinline__ uint8_t f(int i, int j) const { return acc.f(i, j); }
    __device__ __forceinline__ int ncol(int i, int j) const { return (acc.f(i, j) >> 7) & 1; }
    __device__ __forceinline__ bool hhas(int i, int j) const { return (acc.f(i, j) >> (4 + D)) & 1; }
    __device__ __forceinline__ bool vhas(int i, int j) const { return (acc.f(i, j) >> (4 + A)) & 1; }

    // advected marker of a side, relative to the reference node
    // sides: 0 bottom H(fi,fj), 1 right V(fi+1,fj), 2 top H(fi,fj+1), 3 left V(fi,fj)
    __device__ __forceinline__ void point(int fi, int fj, int side, double &X, double &Y) const
    {
        switch (side) {
        case 0: X = (double)fi + acc.xd(fi, fj); Y = (double)fj; break;
        case 2: X = (double)fi + acc.xd(fi, fj + 1); Y = (double)(fj + 1); break;
        case 3: X = (double)fi + acc.dva(fi, fj); Y = (double)fj + (double)acc.sa(fi, fj); break;
        default: X = (double)(fi + 1) + acc.dva(fi + 1, fj); Y = (double)fj + (double)acc.sa(fi + 1, fj); break;
        }
    }

    // segments of face Q(fi,fj) from the old state (paper sec. 2.2, 2.4),
    // packed: bits 0-1 / 2-3 the sides of the first segment (lower first), bits
    // 4-5 / 6-7 the second; bits 8-9 the number of segments.  The segment
    // through side 0 comes first.
    __device__ __forceinline__ int pairs(int fi, int fj) const
    {
        uint8_t f00 = f(fi, fj), f10 = f(fi + 1, fj), f01 = f(fi, fj + 1);
        int h0 = (f00 >> (4 + D)) & 1, v1 = (f10 >> (4 + A)) & 1;
        int h2 = (f01 >> (4 + D)) & 1, v3 = (f00 >> (4 + A)) & 1;
        int m = h0 + v1 + h2 + v3;
        if (m == 2) {
            // the two sides present, lower first
            int lo = h0 ? 0 : (v1 ? 1 : 2);
            int hi = v3 ? 3 : (h2 ? 2 : 1);
            return lo | (hi << 2) | (1 << 8);
        }
        if (m == 4) {
            int c00 = f00 & 1;
            int ff = (f00 >> (1 + B)) & 1;
            // corners (1,0),(0,1) cut off: (0,1),(2,3); else corners (0,0),(1,1): (0,3),(1,2)
            return ff == c00 ? (0 | (1 << 2) | (2 << 4) | (3 << 6) | (2 << 8))
                             : (0 | (3 << 2) | (1 << 4) | (2 << 6) | (2 << 8));
        }
        return 0;
    }
    static __device__ __forceinline__ int nseg(int pk) { return pk >> 8; }
    static __device__ __forceinline__ int side_a(int pk, int t) { return (pk >> (4 * t)) & 3; }
    static __device__ __forceinline__ int side_b(int pk, int t) { return (pk >> (4 * t + 2)) & 3; }

    // far end, in the neighbouring face, of the segment through `side`'s marker
    __device__ __forceinline__ void neighbour(int fi, int fj, int side, double &X, double &Y) const
    {
        int ni = fi, nj = fj, ns;
        switch (side) {
        case 0: nj = fj - 1; ns = 2; break;
        case 2: nj = fj + 1; ns = 0; break;
        case 1: ni = fi + 1; ns = 3; break;
        default: ni = fi - 1; ns = 1; break;
        }
        int pk = pairs(ni, nj);
        int other = ns;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (t >= nseg(pk)) break;
            if (side_a(pk, t) == ns) other = side_b(pk, t);
            else if (side_b(pk, t) == ns) other = side_a(pk, t);
        }
        point(ni, nj, other, X, Y);
    }

    // New marker on V(0,0) (called where the new end colours differ): crossings
    // of X = 0 by advected old segments of faces -2..0 of the row; the median
    // one (by height) is refined by the circle fit.
    __device__ T unaligned(int &fallback, int &multi) const
    {
        T key[6];
        bool ok[6];
        int m = 0;
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            int pk = pairs(o - 2, 0);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                ok[2 * o + t] = false;
                key[2 * o + t] = T(0);
                if (t < nseg(pk)) {
                    double Ax, Ay, Bx, By;
                    point(o - 2, 0, side_a(pk, t), Ax, Ay);
                    point(o - 2, 0, side_b(pk, t), Bx, By);
                    bool sa = 0.0 <= Ax, sb = 0.0 <= Bx;
                    if (sa != sb) {
                        ok[2 * o + t] = true;
                        key[2 * o + t] = sa ? line_cross<T>(T(0), (T)Bx, (T)By, (T)Ax, (T)Ay)
                                            : line_cross<T>(T(0), (T)Ax, (T)Ay, (T)Bx, (T)By);
                        ++m;
                    }
                }
            }
        }
        if ((m & 1) == 0) {          // no odd crossing set: keep the edge valid
            fallback += 1;
            return T(0.5);
        }
        if (m > 1) multi += 1;
        int pick = 0;
#pragma unroll
        for (int c0 = 0; c0 < 6; ++c0) {
            if (!ok[c0]) continue;
            int rank = 0;
#pragma unroll
            for (int c1 = 0; c1 < 6; ++c1)
                if (ok[c1] && (key[c1] < key[c0] || (key[c1] == key[c0] && c1 < c0))) ++rank;
            if (rank == (m >> 1)) pick = c0;
        }
        int o = (pick >> 1) - 2, t = pick & 1;
        int pk = pairs(o, 0);
        int sa_ = side_a(pk, t), sb_ = side_b(pk, t);
        double Ax, Ay, Bx, By;
        point(o, 0, sa_, Ax, Ay);
        point(o, 0, sb_, Bx, By);
        int s2, s3;
        double P2x, P2y, P3x, P3y;
        if (0.0 <= Ax) { s2 = sb_; s3 = sa_; P2x = Bx; P2y = By; P3x = Ax; P3y = Ay; }
        else { s2 = sa_; s3 = sb_; P2x = Ax; P2y = Ay; P3x = Bx; P3y = By; }
        double P1x, P1y, P4x, P4y;
        neighbour(o, 0, s2, P1x, P1y);
        neighbour(o, 0, s3, P4x, P4y);
        return fit_height<T>((T)P1x, (T)P1y, (T)P2x, (T)P2y, (T)P3x, (T)P3y, (T)P4x, (T)P4y, key[pick]);
    }

    // Colour at the centre of face Q(0,0) relative to the advected polyline:
    // start from the new colour of node (0,0), flip for aligned markers landing
    // in [0, 1/2) on the bottom line and for advected segments crossing
    // X = 1/2 below Y = 1/2.
    __device__ int face_colour(int c00) const
    {
        int par = c00;
#pragma unroll
        for (int o = -1; o <= 1; ++o) {
            if (!hhas(o, 0)) continue;
            double X = (double)o + acc.xd(o, 0);
            if (0.0 <= X && X < 0.5) par ^= 1;
        }
#pragma unroll
        for (int o = -1; o <= 1; ++o) {
            int pk = pairs(o, 0);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                if (t >= nseg(pk)) break;
                double Ax, Ay, Bx, By;
                point(o, 0, side_a(pk, t), Ax, Ay);
                point(o, 0, side_b(pk, t), Bx, By);
                bool sa = 0.5 <= Ax, sb = 0.5 <= Bx;
                if (sa == sb) continue;
                T y = sa ? line_cross<T>(T(0.5), (T)Bx, (T)By, (T)Ax, (T)Ay)
                         : line_cross<T>(T(0.5), (T)Ax, (T)Ay, (T)Bx, (T)By);
                if (y < T(0.5)) par ^= 1;
            }
        }
        return par;
    }
};

}  // namespace ebit
