/*
 * ebit_oracle.c -- plain, slow CPU FP64 oracle of the 3D EBIT hot path:
 * marker initialisation, one direction-split advection sweep, Front2VOF, and
 * the compensated volume sum.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The product path (the HIP
 * library) never calls it and the two share no code; they agree only on the
 * state layout below and on the readings of the paper listed in the design
 * notes.
 *
 * Paper: J. Pan, T. Long, R. Scardovelli, S. Popinet, S. Zaleski, "A
 * three-dimensional edge-based interface tracking (EBIT) method for
 * multiphase-flow simulations", arXiv 2509.26361.
 *   sec. 2.1  markers on grid lines; explicit Euler step (eq. Eq_marker_dis);
 *             aligned / unaligned markers of a 1D sweep (Fig. 1); circle fit
 *             for unaligned markers: mean of the 1-2-3 and 2-3-4 circles, the
 *             larger circle when r_max / r_min > 10 (Fig. 2)
 *   sec. 2.2  colour vertex at corners and centres; corner colour flips when
 *             a marker crosses the node (Fig. 4); at most one marker per edge,
 *             a marker exists iff the edge end colours differ; two markers on
 *             one edge annihilate (Fig. 5a)
 *   sec. 2.3  a sweep along d = 2D problems on the two face families that
 *             contain d (Fig. 5); data of Fig. 6b: edge fractions s_x,s_y,s_z,
 *             vertex colour, face-centre colours
 *   sec. 2.4  face ambiguity (4 markers on a face) resolved by the face-centre
 *             colour; internal ambiguity -> separated interface segments
 *   sec. 2.5  Front2VOF: closed loops of face segments, loop centroid (eq. for
 *             X_c), fan of N_m triangles, enclosed volume by Gauss's theorem
 *   sec. 3.1  markers initialised by linear interpolation of phi = R^2 - r^2
 *
 * Everything below that the paper leaves open is marked READING; each reading
 * is stated where it is used.
 *
 * State layout (shared with the HIP library as an interface, not as code):
 * periodic n^3 grid, node (i,j,k) -> i + n*(j + n*k).  Per node:
 *   flags bit 0      colour of node (i,j,k)            (1 = reference phase)
 *   flags bit 1+a    colour at the centre of the face with normal axis a whose
 *                    lowest corner is node (i,j,k)
 *   flags bit 4+e    a marker lies on the edge along axis e from node (i,j,k)
 *   s_e[idx]         its fraction in [0, S_MAX] from node (i,j,k); 0 if none
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define S_MAX 0.9999999999999998   /* 1 - 2^-52: largest fraction kept on an edge */

/* ------------------------------------------------------------------------ */
/* grid helpers                                                              */
/* ------------------------------------------------------------------------ */

static int wrapi(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

static long nidx(int n, int x, int y, int z)
{
    return (long)wrapi(x, n) + (long)n * ((long)wrapi(y, n) + (long)n * (long)wrapi(z, n));
}

static long nidx3(int n, const int p[3]) { return nidx(n, p[0], p[1], p[2]); }

static int bitof(uint8_t f, int b) { return (f >> b) & 1; }

static double clamp_frac(double v)
{
    if (!(v >= 0.0)) v = 0.0;
    if (v > S_MAX) v = S_MAX;
    return v;
}

/* ------------------------------------------------------------------------ */
/* a0: initialisation (sec. 3.1)                                             */
/* ------------------------------------------------------------------------ */

/*
 * colour = [phi > 0]; where the colours of an edge's ends differ, the marker
 * sits at the linear zero of phi, s = phi_a / (phi_a - phi_b) (sec. 3.1), or,
 * if s_exact is given, at s_exact (test mode: the exact crossing).
 * READING (face colours, not given in the paper): the face-centre colour is
 * [phi(face centre) > 0] when the face carries markers, and the colour of its
 * corners when it carries none.
 */
int orc_init(int n, const double *phi, const double *pf0, const double *pf1, const double *pf2,
             const double *se0, const double *se1, const double *se2,
             uint8_t *flags, double *s0, double *s1, double *s2)
{
    const double *pf[3] = {pf0, pf1, pf2};
    const double *se[3] = {se0, se1, se2};
    double *s[3] = {s0, s1, s2};
    long N = (long)n * n * n;
    if (n < 8) return -1;
    for (long q = 0; q < N; q++) flags[q] = phi[q] > 0.0 ? 1 : 0;
    for (int z = 0; z < n; z++)
        for (int y = 0; y < n; y++)
            for (int x = 0; x < n; x++) {
                int p[3] = {x, y, z};
                long q = nidx3(n, p);
                for (int e = 0; e < 3; e++) {
                    int r[3] = {x, y, z};
                    r[e] += 1;
                    long qb = nidx3(n, r);
                    int ca = bitof(flags[q], 0), cb = bitof(flags[qb], 0);
                    if (ca != cb) {
                        double v;
                        if (se[e]) v = se[e][q];
                        else v = phi[q] / (phi[q] - phi[qb]);
                        s[e][q] = clamp_frac(v);
                        flags[q] |= (uint8_t)(1u << (4 + e));
                    } else {
                        s[e][q] = 0.0;
                    }
                }
            }
    for (int z = 0; z < n; z++)
        for (int y = 0; y < n; y++)
            for (int x = 0; x < n; x++) {
                long q = nidx(n, x, y, z);
                for (int a = 0; a < 3; a++) {
                    int b = (a + 1) % 3, c = (a + 2) % 3;
                    /* the face's four edges: along b at p and p+e_c, along c at p and p+e_b */
                    int pc[3] = {x, y, z}; pc[c] += 1;
                    int pb[3] = {x, y, z}; pb[b] += 1;
                    int any = bitof(flags[q], 4 + b) | bitof(flags[nidx3(n, pc)], 4 + b)
                            | bitof(flags[q], 4 + c) | bitof(flags[nidx3(n, pb)], 4 + c);
                    int col = any ? (pf[a][q] > 0.0) : bitof(flags[q], 0);
                    if (col) flags[q] |= (uint8_t)(1u << (1 + a));
                }
            }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* a2-a4: one sweep along axis d (sec. 2.1-2.4)                              */
/* ------------------------------------------------------------------------ */

/* A 2D problem: the plane spanned by the sweep axis d ("X") and axis a ("Y")
 * at fixed coordinate kb along the third axis b.  Its faces are the faces with
 * normal b; its horizontal edges H(i,j) run along d (aligned markers), its
 * vertical edges V(i,j) along a (unaligned markers). */
typedef struct {
    int n, d, a, b, kb;
    const uint8_t *fl;    /* old flags */
    const double *sa;     /* old fractions along a */
    const double *xd;     /* advected local coordinate s + delta of d-edge markers */
    const double *dva;    /* displacement delta of a-edge markers */
} plane;

static long pnode(const plane *P, int i, int j)
{
    int p[3];
    p[P->d] = i; p[P->a] = j; p[P->b] = P->kb;
    return nidx3(P->n, p);
}

static int pcol(const plane *P, int i, int j) { return bitof(P->fl[pnode(P, i, j)], 0); }
static int hhas(const plane *P, int i, int j) { return bitof(P->fl[pnode(P, i, j)], 4 + P->d); }
static int vhas(const plane *P, int i, int j) { return bitof(P->fl[pnode(P, i, j)], 4 + P->a); }

/* Sides of face Q(fi,fj): 0 bottom H(fi,fj), 1 right V(fi+1,fj),
 * 2 top H(fi,fj+1), 3 left V(fi,fj). */
static int side_has(const plane *P, int fi, int fj, int side)
{
    switch (side) {
    case 0: return hhas(P, fi, fj);
    case 1: return vhas(P, fi + 1, fj);
    case 2: return hhas(P, fi, fj + 1);
    default: return vhas(P, fi, fj);
    }
}

/* Advected position of the marker on a side, in cell units relative to node
 * (ri,rj) of the plane.  Aligned markers move along X by their own delta;
 * unaligned markers keep Y and move along X by their delta (sec. 2.1). */
static void side_point(const plane *P, int fi, int fj, int side, int ri, int rj, double *X, double *Y)
{
    long q;
    switch (side) {
    case 0:
        q = pnode(P, fi, fj);
        *X = (double)(fi - ri) + P->xd[q];
        *Y = (double)(fj - rj);
        break;
    case 2:
        q = pnode(P, fi, fj + 1);
        *X = (double)(fi - ri) + P->xd[q];
        *Y = (double)(fj + 1 - rj);
        break;
    case 3:
        q = pnode(P, fi, fj);
        *X = (double)(fi - ri) + P->dva[q];
        *Y = (double)(fj - rj) + P->sa[q];
        break;
    default:
        q = pnode(P, fi + 1, fj);
        *X = (double)(fi + 1 - ri) + P->dva[q];
        *Y = (double)(fj - rj) + P->sa[q];
        break;
    }
}

/* Interface segments inside face Q(fi,fj) from the old state (sec. 2.2, 2.4).
 * Two markers: one segment.  Four markers (alternating corners): the corners
 * whose colour differs from the face-centre colour are cut off, each by the
 * segment joining the markers of its two sides.  Segments are listed with the
 * one through side 0 first; within a segment the lower side comes first. */
static int face_pairs(const plane *P, int fi, int fj, int pr[2][2])
{
    int has[4], m = 0;
    for (int t = 0; t < 4; t++) { has[t] = side_has(P, fi, fj, t); m += has[t]; }
    if (m == 2) {
        int k = 0;
        for (int t = 0; t < 4; t++) if (has[t]) pr[0][k++] = t;
        return 1;
    }
    if (m == 4) {
        int c00 = pcol(P, fi, fj);
        int ff = bitof(P->fl[pnode(P, fi, fj)], 1 + P->b);
        if (ff == c00) {            /* corners (1,0) and (0,1) cut off */
            pr[0][0] = 0; pr[0][1] = 1; pr[1][0] = 2; pr[1][1] = 3;
        } else {                    /* corners (0,0) and (1,1) cut off */
            pr[0][0] = 0; pr[0][1] = 3; pr[1][0] = 1; pr[1][1] = 2;
        }
        return 2;
    }
    return 0;
}

/* The marker on `side` of Q(fi,fj) also belongs to the neighbouring face across
 * that side; return the far end of its segment there (the polyline neighbour). */
static void polyline_neighbour(const plane *P, int fi, int fj, int side, int *gi, int *gj, int *gs)
{
    int ni = fi, nj = fj, ns;
    switch (side) {
    case 0: nj = fj - 1; ns = 2; break;
    case 2: nj = fj + 1; ns = 0; break;
    case 1: ni = fi + 1; ns = 3; break;
    default: ni = fi - 1; ns = 1; break;
    }
    int pr[2][2];
    int k = face_pairs(P, ni, nj, pr);
    int other = ns;
    for (int t = 0; t < k; t++) {
        if (pr[t][0] == ns) other = pr[t][1];
        else if (pr[t][1] == ns) other = pr[t][0];
    }
    *gi = ni; *gj = nj; *gs = other;
}

/* Crossing of the straight segment P2-P3 (P2x < X0 <= P3x) with the line X = X0. */
static double line_cross(double X0, double P2x, double P2y, double P3x, double P3y)
{
    double t = X0 - P2x;
    double dy = P3y - P2y;
    double dx = P3x - P2x;
    double w = t * dy;
    return P2y + w / dx;
}

/* Circle through T, P2, P3 (sec. 2.1, Fig. 2) and its intersection with the
 * line X = 0 that lies on the arc from P2 to P3 not containing T.  P2 is left
 * of the line and P3 right of it, so the chord crosses the line between the
 * two roots; the wanted root is on the other side of the chord from T: the
 * lower root when T is left of P2->P3 (D > 0), the upper one otherwise.
 * With u the centre relative to P2 and x0 = -P2x the line relative to P2, the
 * roots are P2y + t with t = u_y -+ sqrt(u_y^2 - w), w = x0 (x0 - 2 u_x); the
 * root nearer P2 is taken in the conjugate form w / (u_y +- sqrt(.)) so large
 * nearly straight circles keep their accuracy.
 * Returns 0 (a straight line, infinite radius) when the points are collinear
 * or the radius exceeds 1e6 cells (READING: threshold). */
static int circle_root(double Tx, double Ty, double P2x, double P2y, double P3x, double P3y,
                       double *root, double *r2out)
{
    double bx = P3x - P2x, by = P3y - P2y;
    double cx = Tx - P2x, cy = Ty - P2y;
    double D = 2.0 * (bx * cy - by * cx);
    if (D == 0.0) return 0;
    double B2 = bx * bx + by * by;
    double C2 = cx * cx + cy * cy;
    double ux = (cy * B2 - by * C2) / D;
    double uy = (bx * C2 - cx * B2) / D;
    double r2 = ux * ux + uy * uy;
    if (!(r2 < 1e12)) return 0;
    double x0 = -P2x;
    double w = x0 * (x0 - 2.0 * ux);
    double q = uy * uy - w;
    double t;
    if (!(q > 0.0)) {
        t = uy;                                   /* tangent */
    } else {
        double sq = sqrt(q);
        if (D > 0.0) t = uy > 0.0 ? w / (uy + sq) : uy - sq;    /* lower root */
        else t = uy < 0.0 ? w / (uy - sq) : uy + sq;            /* upper root */
    }
    *root = P2y + t;
    *r2out = r2;
    return 1;
}

/* Height (relative to node row j) at which the interface crosses X = 0 near
 * the advected segment P2-P3, from its polyline neighbours P1 (of P2) and P4
 * (of P3): mean of the roots of circles 1-2-3 and 2-3-4, or the root of the
 * larger circle when r_max / r_min > 10 (sec. 2.1, Fig. 2); `key` is the
 * straight-line crossing of P2-P3.  P2 is strictly left of the line, so for
 * P3 strictly right each circle arc P2..P3 crosses the line exactly once. */
static double fit_height(double P1x, double P1y, double P2x, double P2y, double P3x, double P3y,
                         double P4x, double P4y, double key)
{
    double yA = 0.0, rA2 = 0.0, yB = 0.0, rB2 = 0.0, y;
    /* READING: an advected marker that lies exactly on the grid line is where
     * the interface crosses it (a marker that did not move stays put); a
     * circle through it may touch the line twice near it. */
    if (P3x == 0.0) return clamp_frac(P3y);
    int okA = circle_root(P1x, P1y, P2x, P2y, P3x, P3y, &yA, &rA2);
    int okB = circle_root(P4x, P4y, P2x, P2y, P3x, P3y, &yB, &rB2);
    if (okA && okB) {
        if (rA2 > 100.0 * rB2) y = yA;          /* r_A / r_B > 10: larger circle */
        else if (rB2 > 100.0 * rA2) y = yB;
        else y = 0.5 * (yA + yB);               /* mean of the two circle fits */
    } else {
        y = key;                                /* a straight line is the larger "circle" */
    }
    if (!(y >= 0.0 && y < 1.0)) y = key;        /* READING: fit left the edge */
    return clamp_frac(y);
}

/* Test hook: fit_height() for points p = {P1x,P1y,P2x,P2y,P3x,P3y,P4x,P4y}
 * (P2x < 0 <= P3x); also returns the straight crossing in *key_out. */
double orc_fit_height(const double *p, double *key_out)
{
    double key = line_cross(0.0, p[2], p[3], p[4], p[5]);
    if (key_out) *key_out = key;
    return fit_height(p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7], key);
}

typedef struct {
    double key;          /* straight-line crossing */
    int fi, fj, s2, s3;  /* face and sides of P2 (left of the line) and P3 */
    double P2x, P2y, P3x, P3y;
} cand_t;

/* New marker on V(i,j) (the line X = i, rows j..j+1) of one plane.  Returns 1
 * and the fraction if the new end colours differ (sec. 2.2: one marker iff the
 * colours differ); counts fallbacks / multiple crossings. */
static int new_unaligned(const plane *P, const uint8_t *cn, int i, int j, double *s_out, long long *cnt)
{
    int e0 = bitof(cn[pnode(P, i, j)], 0), e1 = bitof(cn[pnode(P, i, j + 1)], 0);
    if (e0 == e1) return 0;
    /* advected old segments of row j crossing X = i: faces i-2..i (|delta| <= 1) */
    cand_t c[6];
    int m = 0;
    for (int o = -2; o <= 0; o++) {
        int fi = i + o, pr[2][2];
        int k = face_pairs(P, fi, j, pr);
        for (int t = 0; t < k; t++) {
            double Ax, Ay, Bx, By;
            side_point(P, fi, j, pr[t][0], i, j, &Ax, &Ay);
            side_point(P, fi, j, pr[t][1], i, j, &Bx, &By);
            int sA = 0.0 <= Ax, sB = 0.0 <= Bx;
            if (sA == sB) continue;
            cand_t cc;
            cc.fi = fi; cc.fj = j;
            if (!sA) { cc.s2 = pr[t][0]; cc.s3 = pr[t][1]; cc.P2x = Ax; cc.P2y = Ay; cc.P3x = Bx; cc.P3y = By; }
            else     { cc.s2 = pr[t][1]; cc.s3 = pr[t][0]; cc.P2x = Bx; cc.P2y = By; cc.P3x = Ax; cc.P3y = Ay; }
            cc.key = line_cross(0.0, cc.P2x, cc.P2y, cc.P3x, cc.P3y);
            /* stable insertion by crossing height (enumeration order breaks ties) */
            int pos = m;
            while (pos > 0 && c[pos - 1].key > cc.key) { c[pos] = c[pos - 1]; pos--; }
            c[pos] = cc;
            m++;
        }
    }
    if ((m & 1) == 0) {
        /* READING: cannot happen for a consistent state (crossing parity equals
         * the colour difference); keep the edge valid with a central marker */
        cnt[0]++;
        *s_out = 0.5;
        return 1;
    }
    if (m > 1) cnt[1]++;
    const cand_t *C = &c[m / 2];   /* READING: median crossing when several */
    int g1i, g1j, g1s, g4i, g4j, g4s;
    double P1x, P1y, P4x, P4y;
    polyline_neighbour(P, C->fi, C->fj, C->s2, &g1i, &g1j, &g1s);
    side_point(P, g1i, g1j, g1s, i, j, &P1x, &P1y);
    polyline_neighbour(P, C->fi, C->fj, C->s3, &g4i, &g4j, &g4s);
    side_point(P, g4i, g4j, g4s, i, j, &P4x, &P4y);
    *s_out = fit_height(P1x, P1y, C->P2x, C->P2y, C->P3x, C->P3y, P4x, P4y, C->key);
    return 1;
}

/* READING (face-centre colour update; the paper defers the rule to its 2D
 * predecessor): a face of the plane with no new marker takes its corner
 * colour; otherwise its colour is the phase at the face centre relative to the
 * advected polyline, found by walking from node (i,j) along the bottom line to
 * X = i + 1/2 and then up to the centre, flipping once per crossing. */
static int new_face_colour(const plane *P, const uint8_t *cn, int i, int j)
{
    int c00 = bitof(cn[pnode(P, i, j)], 0), c10 = bitof(cn[pnode(P, i + 1, j)], 0);
    int c01 = bitof(cn[pnode(P, i, j + 1)], 0), c11 = bitof(cn[pnode(P, i + 1, j + 1)], 0);
    if (c00 == c10 && c00 == c01 && c00 == c11) return c00;
    int par = c00;
    for (int o = -1; o <= 1; o++) {
        if (!hhas(P, i + o, j)) continue;
        double X = (double)o + P->xd[pnode(P, i + o, j)];
        if (0.0 <= X && X < 0.5) par ^= 1;
    }
    for (int o = -1; o <= 1; o++) {
        int fi = i + o, pr[2][2];
        int k = face_pairs(P, fi, j, pr);
        for (int t = 0; t < k; t++) {
            double Ax, Ay, Bx, By;
            side_point(P, fi, j, pr[t][0], i, j, &Ax, &Ay);
            side_point(P, fi, j, pr[t][1], i, j, &Bx, &By);
            int sA = 0.5 <= Ax, sB = 0.5 <= Bx;
            if (sA == sB) continue;
            double y = sA ? line_cross(0.5, Bx, By, Ax, Ay) : line_cross(0.5, Ax, Ay, Bx, By);
            if (y < 0.5) par ^= 1;
        }
    }
    return par;
}

/*
 * One sweep along axis d with time factor g and step dt (sec. 2.1-2.4).
 * U is the d-component of the node velocity (spatial factor).  Reads the old
 * state (flags_in, s*_in) and writes the new one (flags_out, s*_out).
 * counters[0] fallbacks (no odd crossing set), [1] edges with >1 crossing,
 * [2] markers with |delta| > 1 (CFL contract broken), [3] aligned edges on
 * which more than one marker landed, [4] those of them where the markers
 * annihilated (an even number landed: the end colours agree, no marker).
 * READINGS: node velocity, linear along the marker's own edge (the paper's
 * bilinear interpolation restricted to an edge); delta = (dt n) g u (cell
 * units); time level t^n for all three sweeps; half-open node rule: a point X
 * is at or above node i iff i <= X.
 */
int orc_sweep(int n, int d, double g, double dt, const double *U,
              const uint8_t *fl, const double *sx, const double *sy, const double *sz,
              uint8_t *flo, double *sxo, double *syo, double *szo, long long *counters)
{
    if (n < 8 || d < 0 || d > 2) return -1;
    const double *s[3] = {sx, sy, sz};
    double *so[3] = {sxo, syo, szo};
    long N = (long)n * n * n;
    double c = (dt * (double)n) * g;
    double *xd = (double *)malloc(sizeof(double) * N);
    double *dv[3] = {NULL, NULL, NULL};
    uint8_t *cn = (uint8_t *)malloc(N);
    long long cnt[5] = {0, 0, 0, 0, 0};

    /* Euler step of every marker (eq. Eq_marker_dis) */
    for (int e = 0; e < 3; e++) if (e != d) dv[e] = (double *)malloc(sizeof(double) * N);
    long long ncfl = 0;
#pragma omp parallel for reduction(+ : ncfl)
    for (int z = 0; z < n; z++)
        for (int y = 0; y < n; y++)
            for (int x = 0; x < n; x++) {
                int p[3] = {x, y, z};
                long q = nidx3(n, p);
                for (int e = 0; e < 3; e++) {
                    double val = 0.0;
                    if (bitof(fl[q], 4 + e)) {
                        int r[3] = {x, y, z};
                        r[e] += 1;
                        double U0 = U[q], U1 = U[nidx3(n, r)];
                        double u = U0 + s[e][q] * (U1 - U0);
                        double delta = c * u;
                        if (fabs(delta) > 1.0) ncfl++;
                        val = e == d ? s[e][q] + delta : delta;
                    }
                    if (e == d) xd[q] = val; else dv[e][q] = val;
                }
            }

    cnt[2] = ncfl;
    /* aligned markers and node colours, one d-line at a time (sec. 2.1, Fig. 4) */
#pragma omp parallel for
    for (int z = 0; z < n; z++)
        for (int y = 0; y < n; y++)
            for (int x = 0; x < n; x++) {
                int p[3] = {x, y, z};
                int pm[3] = {x, y, z}; pm[d] -= 1;
                long q = nidx3(n, p), qm = nidx3(n, pm);
                int col = bitof(fl[q], 0);
                if (bitof(fl[qm], 4 + d) && xd[qm] >= 1.0) col ^= 1;   /* crossed upward */
                if (bitof(fl[q], 4 + d) && xd[q] < 0.0) col ^= 1;      /* crossed downward */
                cn[q] = (uint8_t)col;
            }
    long long nfb = 0, nmerge = 0, nannih = 0;
#pragma omp parallel for reduction(+ : nfb, nmerge, nannih)
    for (int z = 0; z < n; z++)
        for (int y = 0; y < n; y++)
            for (int x = 0; x < n; x++) {
                int p[3] = {x, y, z};
                int pm[3] = {x, y, z}; pm[d] -= 1;
                int pp[3] = {x, y, z}; pp[d] += 1;
                long q = nidx3(n, p), qm = nidx3(n, pm), qp = nidx3(n, pp);
                uint8_t out = cn[q];
                so[d][q] = 0.0;
                if (cn[q] != cn[qp]) {
                    double v[3];
                    int k = 0;
                    if (bitof(fl[qm], 4 + d) && xd[qm] >= 1.0) v[k++] = xd[qm] - 1.0;
                    if (bitof(fl[q], 4 + d) && xd[q] >= 0.0 && xd[q] < 1.0) v[k++] = xd[q];
                    if (bitof(fl[qp], 4 + d) && xd[qp] < 0.0) v[k++] = xd[qp] + 1.0;
                    double val;
                    if (k == 1) val = v[0];
                    else if (k == 3) {
                        /* READING: three markers on one edge -> the middle one survives */
                        double lo = v[0] < v[1] ? v[0] : v[1], hi = v[0] < v[1] ? v[1] : v[0];
                        val = v[2] < lo ? lo : (v[2] > hi ? hi : v[2]);
                        nmerge++;
                    } else { val = 0.5; nfb++; }
                    so[d][q] = clamp_frac(val);
                    out |= (uint8_t)(1u << (4 + d));
                } else {
                    int k = 0;
                    if (bitof(fl[qm], 4 + d) && xd[qm] >= 1.0) k++;
                    if (bitof(fl[q], 4 + d) && xd[q] >= 0.0 && xd[q] < 1.0) k++;
                    if (bitof(fl[qp], 4 + d) && xd[qp] < 0.0) k++;
                    if (k >= 2) { nmerge++; nannih++; }   /* annihilated pair (sec. 2.2) */
                }
                /* READING: face colours of the faces normal to d are not updated */
                out |= (uint8_t)(fl[q] & (1u << (1 + d)));
                flo[q] = out;
            }

    cnt[0] += nfb;
    cnt[3] += nmerge;
    cnt[4] += nannih;
    /* unaligned markers and face colours of the two planes containing d (sec. 2.3) */
    for (int fam = 0; fam < 2; fam++) {
        int a = (d + 1 + fam) % 3;
        int b = 3 - d - a;
        long long c0 = 0, c1 = 0;
#pragma omp parallel for reduction(+ : c0, c1)
        for (int kb = 0; kb < n; kb++) {
            long long lc[2] = {0, 0};
            plane P;
            P.n = n; P.d = d; P.a = a; P.b = b; P.kb = kb;
            P.fl = fl; P.sa = s[a]; P.xd = xd; P.dva = dv[a];
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++) {
                    long q = pnode(&P, i, j);
                    double val;
                    if (new_unaligned(&P, cn, i, j, &val, lc)) {
                        so[a][q] = val;
                        flo[q] |= (uint8_t)(1u << (4 + a));
                    } else {
                        so[a][q] = 0.0;
                    }
                    if (new_face_colour(&P, cn, i, j)) flo[q] |= (uint8_t)(1u << (1 + b));
                }
            c0 += lc[0];
            c1 += lc[1];
        }
        cnt[0] += c0;
        cnt[1] += c1;
    }
    if (counters) for (int t = 0; t < 5; t++) counters[t] += cnt[t];
    free(xd); free(cn);
    for (int e = 0; e < 3; e++) free(dv[e]);
    return cnt[2] ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* a5: Front2VOF (sec. 2.5)                                                  */
/* ------------------------------------------------------------------------ */

/* Cell-local edge numbering: edge 4e + oA + 2 oB runs along axis e with
 * offsets oA, oB along the other two axes A < B. */
static int edge_id(int e, const int off[3])
{
    int A = e == 0 ? 1 : 0, B = e == 2 ? 1 : 2;
    return 4 * e + off[A] + 2 * off[B];
}

/*
 * Reference-phase volume fraction of every cell (sec. 2.5).  Per cell:
 *  1. on each of the six faces, segments between its markers (two markers: one
 *     segment; four: the corners whose colour differs from the face-centre
 *     colour are cut off); each segment is oriented so that the reference
 *     phase lies on its left when the face is seen from outside the cell, i.e.
 *     from the marker where a counter-clockwise walk round the face leaves the
 *     phase to the marker where it re-enters it;
 *  2. the segments close into loops (each marker starts one segment and ends
 *     one); loops never cross the cell interior, which is the "separated
 *     segments" choice for internal ambiguity (sec. 2.4);
 *  3. loop centroid X_c = mean of its markers; fan triangles (X_c, X_k+1, X_k);
 *  4. Gauss: C = (1/3) sum_faces int x.n dS over the phase-1 part of the cell
 *     boundary: the three far faces contribute their phase-1 areas A1 (2D
 *     Green), the near faces nothing, each triangle det(X_c, X_k+1, X_k) / 2.
 * amb (may be NULL) receives 1 for cells with a 4-marker face or >1 loop.
 */
static int cell_f2v(int n, const uint8_t *fl, const double *const s[3], int x, int y, int z,
                    double *C_out, uint8_t *amb_out, double *loop_pts, int *loop_len)
{
    int col[2][2][2];
    for (int oz = 0; oz < 2; oz++)
        for (int oy = 0; oy < 2; oy++)
            for (int ox = 0; ox < 2; ox++)
                col[ox][oy][oz] = bitof(fl[nidx(n, x + ox, y + oy, z + oz)], 0);
    int has[12];
    double P[12][3];
    int nm = 0;
    for (int e = 0; e < 3; e++) {
        int A = e == 0 ? 1 : 0, B = e == 2 ? 1 : 2;
        for (int oB = 0; oB < 2; oB++)
            for (int oA = 0; oA < 2; oA++) {
                int off[3] = {0, 0, 0};
                off[A] = oA; off[B] = oB;
                int id = edge_id(e, off);
                long q = nidx(n, x + off[0], y + off[1], z + off[2]);
                has[id] = bitof(fl[q], 4 + e);
                nm += has[id];
                P[id][0] = (double)off[0];
                P[id][1] = (double)off[1];
                P[id][2] = (double)off[2];
                P[id][e] = has[id] ? s[e][q] : 0.0;
            }
    }
    if (nm == 0) {
        *C_out = (double)col[0][0][0];
        *amb_out = 0;
        return 0;
    }
    int succ[12];
    int four = 0;
    for (int t = 0; t < 12; t++) succ[t] = -1;
    double A1[3] = {0.0, 0.0, 0.0};
    /* segments of the six faces */
    for (int a = 0; a < 3; a++)
        for (int sg = 0; sg < 2; sg++) {
            int b = (a + 1) % 3, c = (a + 2) % 3;
            /* corners counter-clockwise about the outward normal;
             * (b, c, a) is right-handed, so the upper face runs
             * (0,0),(1,0),(1,1),(0,1) in (b,c) and the lower face
             * the reverse */
            static const int up[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
            static const int lo[4][2] = {{0, 0}, {0, 1}, {1, 1}, {1, 0}};
            int cb[4], cc[4], cl[4], eid[4], mk[4], ex[4];
            for (int m = 0; m < 4; m++) {
                cb[m] = sg ? up[m][0] : lo[m][0];
                cc[m] = sg ? up[m][1] : lo[m][1];
                int p3[3];
                p3[a] = sg; p3[b] = cb[m]; p3[c] = cc[m];
                cl[m] = col[p3[0]][p3[1]][p3[2]];
            }
            int cnt = 0;
            for (int m = 0; m < 4; m++) {
                int m1 = (m + 1) % 4;
                int off[3], e;
                off[a] = sg;
                if (cb[m] != cb[m1]) { e = b; off[b] = 0; off[c] = cc[m]; }
                else { e = c; off[c] = 0; off[b] = cb[m]; }
                eid[m] = edge_id(e, off);
                mk[m] = has[eid[m]];
                ex[m] = cl[m] == 1 && cl[m1] == 0;   /* walk leaves the phase */
                cnt += mk[m];
            }
            if (cnt == 2) {
                int xe = -1, en = -1;
                for (int m = 0; m < 4; m++)
                    if (mk[m]) { if (ex[m]) xe = eid[m]; else en = eid[m]; }
                succ[xe] = en;
            } else if (cnt == 4) {
                four = 1;
                int p3[3];
                p3[0] = x; p3[1] = y; p3[2] = z;
                p3[a] += sg;
                int ff = bitof(fl[nidx3(n, p3)], 1 + a);
                for (int m = 0; m < 4; m++) {
                    if (cl[m] == ff) continue;        /* corner kept by the centre */
                    int mb = (m + 3) % 4;              /* edge entering corner m */
                    int xe = ex[mb] ? eid[mb] : eid[m];
                    int en = ex[mb] ? eid[m] : eid[mb];
                    succ[xe] = en;
                }
            }
            if (sg == 1) {
                /* phase-1 area of the far face by Green's theorem in
                 * (u,v) = (b,c): right side u = 1 and top side v = 1
                 * contribute their phase-1 lengths, each segment
                 * (u_s v_e - u_e v_s) */
                double acc;
                {
                    /* right side: from corner (1,0) (m=1) to (1,1) (m=2): edge m = 1 */
                    double Lr;
                    if (mk[1]) Lr = cl[1] ? P[eid[1]][c] : 1.0 - P[eid[1]][c];
                    else Lr = (double)cl[1];
                    /* top side: corners (1,1) (m=2) and (0,1) (m=3): edge m = 2 */
                    double Lt;
                    if (mk[2]) Lt = cl[3] ? P[eid[2]][b] : 1.0 - P[eid[2]][b];
                    else Lt = (double)cl[3];
                    acc = Lr + Lt;
                }
                for (int m = 0; m < 4; m++) {
                    if (!mk[m] || !ex[m]) continue;
                    int xe = eid[m], en = succ[xe];
                    if (en < 0) continue;
                    double us = P[xe][b], vs = P[xe][c], ue = P[en][b], ve = P[en][c];
                    acc += us * ve - ue * vs;
                }
                A1[a] = 0.5 * acc;
            }
        }
    /* loops, centroid, fan (sec. 2.5) */
    int vis[12] = {0};
    int nloops = 0, npts = 0;
    double fan = 0.0;
    for (int e0 = 0; e0 < 12; e0++) {
        if (!has[e0] || vis[e0]) continue;
        int L[12], m = 0, cur = e0;
        do {
            L[m++] = cur;
            vis[cur] = 1;
            cur = succ[cur];
        } while (cur >= 0 && cur != e0 && m < 12);
        if (loop_len) {
            for (int t = 0; t < m; t++)
                for (int u = 0; u < 3; u++) loop_pts[3 * (npts + t) + u] = P[L[t]][u];
            loop_len[nloops] = m;
            npts += m;
        }
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int t = 0; t < m; t++) { gx += P[L[t]][0]; gy += P[L[t]][1]; gz += P[L[t]][2]; }
        gx = gx / (double)m; gy = gy / (double)m; gz = gz / (double)m;
        for (int t = 0; t < m; t++) {
            const double *pa = P[L[(t + 1) % m]], *pb = P[L[t]];
            double crx = pa[1] * pb[2] - pa[2] * pb[1];
            double cry = pa[2] * pb[0] - pa[0] * pb[2];
            double crz = pa[0] * pb[1] - pa[1] * pb[0];
            fan += gx * crx + gy * cry + gz * crz;
        }
        nloops++;
    }
    *C_out = ((A1[0] + A1[1]) + A1[2]) / 3.0 + fan / 6.0;
    *amb_out = (uint8_t)(four || nloops > 1);
    return nloops;
}

void orc_f2v(int n, const uint8_t *fl, const double *sx, const double *sy, const double *sz,
             double *C, uint8_t *amb)
{
    const double *s[3] = {sx, sy, sz};
#pragma omp parallel for
    for (int z = 0; z < n; z++)
        for (int y = 0; y < n; y++)
            for (int x = 0; x < n; x++) {
                long q0 = nidx(n, x, y, z);
                uint8_t a = 0;
                cell_f2v(n, fl, s, x, y, z, &C[q0], &a, NULL, NULL);
                if (amb) amb[q0] = a;
            }
}

/* Test hook: the loops of cell (x,y,z) in traversal order.  loop_pts receives
 * up to 12 points (xyz, cell frame), loop_len up to 6 lengths; returns the
 * number of loops and the cell's volume fraction in *C. */
int orc_cell_loops(int n, const uint8_t *fl, const double *sx, const double *sy, const double *sz,
                   int x, int y, int z, double *loop_pts, int *loop_len, double *C)
{
    const double *s[3] = {sx, sy, sz};
    uint8_t a = 0;
    return cell_f2v(n, fl, s, x, y, z, C, &a, loop_pts, loop_len);
}

/* ------------------------------------------------------------------------ */
/* a6: compensated volume sum                                                */
/* ------------------------------------------------------------------------ */

/* Neumaier-compensated sum of C over all cells, in index order; returns the
 * sum and stores the compensation term in *comp (the volume is sum + comp). */
double orc_volume(long ncell, const double *C, double *comp)
{
    double sum = 0.0, cmp = 0.0;
    for (long q = 0; q < ncell; q++) {
        double v = C[q];
        double t = sum + v;
        if (fabs(sum) >= fabs(v)) cmp += (sum - t) + v;
        else cmp += (v - t) + sum;
        sum = t;
    }
    if (comp) *comp = cmp;
    return sum;
}

/* Cells with at least one marker on their 12 edges. */
long orc_count_interfacial(int n, const uint8_t *fl)
{
    long cntc = 0;
    for (int z = 0; z < n; z++)
        for (int y = 0; y < n; y++)
            for (int x = 0; x < n; x++) {
                int any = 0;
                for (int e = 0; e < 3 && !any; e++) {
                    int A = e == 0 ? 1 : 0, B = e == 2 ? 1 : 2;
                    for (int oB = 0; oB < 2 && !any; oB++)
                        for (int oA = 0; oA < 2 && !any; oA++) {
                            int off[3] = {0, 0, 0};
                            off[A] = oA; off[B] = oB;
                            any = bitof(fl[nidx(n, x + off[0], y + off[1], z + off[2])], 4 + e);
                        }
                }
                cntc += any;
            }
    return cntc;
}
