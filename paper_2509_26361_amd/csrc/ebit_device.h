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
// axis D ("X") and axis A ("Y") through the thread's node.  Offsets (i, j) are
// relative to that node.  Horizontal edges H(i,j) run along D (aligned
// markers), vertical edges V(i,j) along A (unaligned); face Q(i,j) spans
// [i,i+1] x [j,j+1] and has normal B.
template <typename T, int D, int A>
struct Plane {
    static constexpr int B = 3 - D - A;
    const uint8_t *__restrict__ fl;
    const T *__restrict__ sD;
    const T *__restrict__ sA;
    const T *__restrict__ U;
    T c;             // (dt n) g: cell-unit displacement per unit velocity
    int n;
    int ci, cj;      // coordinates of the thread's node along D and A
    long base;       // index part of the fixed coordinate along B
    long strD, strA;

    __device__ __forceinline__ long node(int i, int j) const
    {
        return (long)wrp(ci + i, n) * strD + (long)wrp(cj + j, n) * strA + base;
    }
    __device__ __forceinline__ uint8_t f(int i, int j) const { return fl[node(i, j)]; }
    __device__ __forceinline__ int col(int i, int j) const { return f(i, j) & 1; }
    __device__ __forceinline__ bool hhas(int i, int j) const { return (f(i, j) >> (4 + D)) & 1; }
    __device__ __forceinline__ bool vhas(int i, int j) const { return (f(i, j) >> (4 + A)) & 1; }

    // Euler step (eq. Eq_marker_dis) of the aligned marker on H(i,j): its new
    // coordinate s + delta relative to node i (decisions in double).
    __device__ __forceinline__ double xd(int i, int j) const
    {
        long q = node(i, j);
        T s = sD[q];
        T U0 = U[q];
        T U1 = U[node(i + 1, j)];
        T u = U0 + s * (U1 - U0);
        T delta = c * u;
        return (double)s + (double)delta;
    }
    // displacement of the unaligned marker on V(i,j) (it keeps its Y)
    __device__ __forceinline__ double dva(int i, int j) const
    {
        long q = node(i, j);
        T s = sA[q];
        T U0 = U[q];
        T U1 = U[node(i, j + 1)];
        T u = U0 + s * (U1 - U0);
        return (double)(c * u);
    }

    // new colour of node (i,j): flips once per aligned marker crossing it
    __device__ __forceinline__ int newcol(int i, int j) const
    {
        int cc = col(i, j);
        if (hhas(i - 1, j) && xd(i - 1, j) >= 1.0) cc ^= 1;
        if (hhas(i, j) && xd(i, j) < 0.0) cc ^= 1;
        return cc;
    }

    // sides of a face: 0 bottom H(fi,fj), 1 right V(fi+1,fj), 2 top H(fi,fj+1), 3 left V(fi,fj)
    __device__ __forceinline__ bool side_has(int fi, int fj, int side) const
    {
        switch (side) {
        case 0: return hhas(fi, fj);
        case 1: return vhas(fi + 1, fj);
        case 2: return hhas(fi, fj + 1);
        default: return vhas(fi, fj);
        }
    }

    // advected marker of a side, relative to the thread's node
    __device__ __forceinline__ void point(int fi, int fj, int side, double &X, double &Y) const
    {
        switch (side) {
        case 0: X = (double)fi + xd(fi, fj); Y = (double)fj; break;
        case 2: X = (double)fi + xd(fi, fj + 1); Y = (double)(fj + 1); break;
        case 3: X = (double)fi + dva(fi, fj); Y = (double)fj + (double)sA[node(fi, fj)]; break;
        default: X = (double)(fi + 1) + dva(fi + 1, fj); Y = (double)fj + (double)sA[node(fi + 1, fj)]; break;
        }
    }

    // segments of face Q(fi,fj) from the old state (paper sec. 2.2, 2.4);
    // encoded as sides (a0,b0),(a1,b1) with a < b; the one through side 0 first
    __device__ __forceinline__ int pairs(int fi, int fj, int pr[2][2]) const
    {
        uint8_t f00 = f(fi, fj), f10 = f(fi + 1, fj), f01 = f(fi, fj + 1);
        int h0 = (f00 >> (4 + D)) & 1, v1 = (f10 >> (4 + A)) & 1;
        int h2 = (f01 >> (4 + D)) & 1, v3 = (f00 >> (4 + A)) & 1;
        int m = h0 + v1 + h2 + v3;
        if (m == 2) {
            int has[4] = {h0, v1, h2, v3};
            int k = 0;
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (has[t]) { pr[0][k] = t; ++k; }
            return 1;
        }
        if (m == 4) {
            int c00 = f00 & 1;
            int ff = (f00 >> (1 + B)) & 1;
            if (ff == c00) { pr[0][0] = 0; pr[0][1] = 1; pr[1][0] = 2; pr[1][1] = 3; }
            else { pr[0][0] = 0; pr[0][1] = 3; pr[1][0] = 1; pr[1][1] = 2; }
            return 2;
        }
        return 0;
    }

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
        int pr[2][2];
        int k = pairs(ni, nj, pr);
        int other = ns;
        for (int t = 0; t < k; ++t) {
            if (pr[t][0] == ns) other = pr[t][1];
            else if (pr[t][1] == ns) other = pr[t][0];
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
            int pr[2][2];
            int k = pairs(o - 2, 0, pr);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                ok[2 * o + t] = false;
                key[2 * o + t] = T(0);
                if (t < k) {
                    double Ax, Ay, Bx, By;
                    point(o - 2, 0, pr[t][0], Ax, Ay);
                    point(o - 2, 0, pr[t][1], Bx, By);
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
            fallback = 1;
            return T(0.5);
        }
        if (m > 1) multi = 1;
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
        int pr[2][2];
        pairs(o, 0, pr);
        double Ax, Ay, Bx, By;
        point(o, 0, pr[t][0], Ax, Ay);
        point(o, 0, pr[t][1], Bx, By);
        int s2, s3;
        double P2x, P2y, P3x, P3y;
        if (0.0 <= Ax) { s2 = pr[t][1]; s3 = pr[t][0]; P2x = Bx; P2y = By; P3x = Ax; P3y = Ay; }
        else { s2 = pr[t][0]; s3 = pr[t][1]; P2x = Ax; P2y = Ay; P3x = Bx; P3y = By; }
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
            double X = (double)o + xd(o, 0);
            if (0.0 <= X && X < 0.5) par ^= 1;
        }
#pragma unroll
        for (int o = -1; o <= 1; ++o) {
            int pr[2][2];
            int k = pairs(o, 0, pr);
            for (int t = 0; t < k; ++t) {
                double Ax, Ay, Bx, By;
                point(o, 0, pr[t][0], Ax, Ay);
                point(o, 0, pr[t][1], Bx, By);
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
