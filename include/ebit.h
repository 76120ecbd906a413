/*
 * ebit.h -- C ABI of the MI355X library for the hot path of the 3D
 * Edge-Based Interface Tracking method (Pan, Long, Scardovelli, Popinet,
 * Zaleski, arXiv 2509.26361): direction-split interface advection and the
 * Front2VOF volume fraction on a uniform periodic grid.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid: n^3 cells of size h = 1/n, periodic, n a multiple of 4, 8 <= n <= 1024
 * (node indices fit 32 bits).
 * Node (i,j,k) has linear index i + n*(j + n*k) (x fastest); every array
 * below has n^3 entries in that order.
 *
 * State (sec. 2.3, Fig. 6b: one edge field, one vertex field, one face
 * field), per node:
 *   flags bit 0     colour of node (i,j,k): 1 = reference phase (sec. 2.2)
 *   flags bit 1+a   colour at the centre of the face with normal axis a whose
 *                   lowest corner is node (i,j,k) (sec. 2.3, 2.4)
 *   flags bit 4+e   a marker lies on the edge along axis e that starts at node
 *                   (i,j,k); at most one per edge, present iff the two end
 *                   colours differ (sec. 2.2)
 *   s_e             the marker's fraction along that edge, in [0, 1 - 2^-52]
 *                   (0 where there is none); double, or float in EBIT_FP32
 * Memory: all array pointers are DEVICE pointers owned by the caller; the
 * library never allocates or frees state memory.  Work space comes from the
 * caller's `scratch` buffer (ebit_scratch_bytes).  The context is a small
 * host object.
 * Streams: `stream` is a hipStream_t (NULL = the null stream); every call is
 * asynchronous on it unless stated otherwise.
 * Errors: entry points return EBIT_OK (0) or a negative code; argument errors
 * are detected on the host before anything is enqueued.  Conditions found on
 * the device (Courant number above one) are reported by ebit_stats.
 * Threads: one context per host thread at a time.
 */
#ifndef EBIT_H
#define EBIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    EBIT_OK = 0,
    EBIT_EINVAL = -1,   /* bad argument (null pointer, n, direction, size) */
    EBIT_ECFL = -2,     /* |Courant number| > 1 somewhere (sec. 2.3: CFL <= 1) */
    EBIT_ESTATE = -3,   /* inconsistent state */
    EBIT_EHIP = -4,     /* a HIP runtime call failed */
    EBIT_ENOSURR = -5,  /* surrogate weights missing */
    EBIT_ESCRATCH = -6, /* scratch buffer too small */
    EBIT_ETOOBIG = -7   /* input larger than a fixed work space allows */
};

enum { EBIT_FP64 = 0, EBIT_FP32 = 1 };

typedef struct ebit_ctx ebit_ctx;

/* Description of the caller's buffers.  The state is double-buffered: each
 * sweep reads buffer ebit_current() and writes the other one. */
typedef struct {
    int32_t n;              /* cells per axis */
    int32_t precision;      /* EBIT_FP64: s_e, U, C are double; EBIT_FP32: float */
    void *s[2][3];          /* s[buffer][axis]: marker fractions, n^3 each */
    uint8_t *flags[2];      /* flags[buffer]: n^3 bytes each */
    void *scratch;          /* device work space, >= ebit_scratch_bytes(n) bytes */
    size_t scratch_bytes;
} ebit_desc;

/* Bytes of device scratch the library needs for an n^3 grid.  The scratch
 * holds the context's work lists and per-brick records of what the state
 * buffers hold (e.g. which rows of a 4^3 brick may carry a fraction other
 * than zero); they are built by ebit_init and kept by the library's own
 * calls, so the state buffers and the scratch must not be written by anyone
 * else between calls (start again with ebit_init after doing so). */
size_t ebit_scratch_bytes(int32_t n);

/*
 * Create a context over the caller's buffers and initialise state buffer 0
 * from a sampled interface (sec. 3.1): node colour = [phi > 0]; where an
 * edge's end colours differ its marker sits at the linear zero of phi,
 * s = phi_a / (phi_a - phi_b), or at s_exact[e] if s_exact is not NULL (the
 * exact crossing, a test mode).  Face-centre colour = [phi_faces[a] > 0] on
 * faces that carry markers, the corner colour on faces that carry none.
 *   phi_nodes    device, n^3 doubles, or NULL: buffer 0 already holds a state
 *                (e.g. a checkpoint) and only the work lists are built
 *   phi_faces    3 device pointers (n^3 doubles each), required with phi_nodes
 *   s_exact      NULL or 3 device pointers (n^3 doubles each)
 * Returns EBIT_EINVAL / EBIT_ESCRATCH on bad arguments; *out is set only on
 * success.  Enqueued on `stream`.
 */
int ebit_init(ebit_ctx **out, const ebit_desc *desc, const double *phi_nodes,
              const double *const *phi_faces, const double *const *s_exact, void *stream);

/*
 * One one-dimensional advection sweep along axis `dir` (0 = x, 1 = y, 2 = z),
 * secs. 2.1-2.4: every marker moves by an explicit Euler step (eq.
 * Eq_marker_dis) with displacement (dt/h) * g * u in cell units, u the
 * node velocity U_dir interpolated linearly along the marker's own edge;
 * node colours flip where markers cross nodes (Fig. 4); markers on edges
 * along `dir` land on the edge they reach, pairs annihilating (Fig. 5a);
 * markers on the other edges are replaced by the crossings of the advected
 * interface with the grid lines, placed by the circle fit of sec. 2.1 on the
 * two face families that contain `dir`; the face-centre colours of those two
 * families are recomputed.  Reads buffer ebit_current(), writes the other one
 * and makes it current.
 *   U_dir   device, n^3 doubles (floats in EBIT_FP32): the `dir` component of
 *           the velocity's spatial factor at the nodes
 *   g, dt   time factor and time step; |(dt n) g U| must stay <= 1
 *           (otherwise the result is undefined and ebit_stats reports
 *           EBIT_ECFL).
 */
int ebit_advect_sweep(ebit_ctx *ctx, int dir, const void *U_dir, double g, double dt, void *stream);

/*
 * Front2VOF (sec. 2.5): reference-phase volume fraction of every cell from
 * the current state: face segments (paired by the face-centre colour on
 * faces with four markers), closed loops, loop centroid, fan of triangles,
 * enclosed volume by Gauss's theorem.
 *   C       device, n^3 doubles (floats in EBIT_FP32).  Only cells whose
 *           state may have changed since the previous call with the same C
 *           are rewritten; a different C pointer is filled completely.
 */
int ebit_front2vof(ebit_ctx *ctx, void *C, void *stream);

typedef struct {
    double volume;          /* sum of C over all cells (compensated, FP64) */
    double volume_comp;     /* its compensation term: volume + volume_comp */
    int64_t n_interfacial;  /* cells with a marker on any of their 12 edges, at the last ebit_front2vof */
    int64_t n_ambiguous;    /* cells recomputed by the last ebit_front2vof (all cells for a new C) with a
                               4-marker face or more than one loop */
    int64_t n_markers[3];   /* markers per edge family in the current state */
    int64_t n_fallback;     /* sweeps so far: edges placed by the no-crossing fallback */
    int64_t n_multi;        /* sweeps so far: new unaligned markers with > 1 crossing */
    int64_t n_cfl;          /* sweeps so far: markers moved by more than one cell */
    int64_t n_merged;       /* sweeps so far: aligned edges reached by > 1 marker */
    int64_t n_active_cells; /* sweeps so far: cells processed (work-list sizes) */
    int64_t step_sweeps;    /* sweeps so far */
    int64_t n_interfacial_sum; /* sum of n_interfacial over every ebit_front2vof so far */
    double max_courant;     /* sweeps so far: largest |(dt n) g u| of a marker, in cells (FP32 precision;
                               sec. 2.3 requires <= 1) */
    int64_t n_annihilated;  /* sweeps so far: aligned edges reached by an even number (>= 2) of markers,
                               which annihilate (sec. 2.2, Fig. 5a); included in n_merged */
    int64_t n_ambig_faces;  /* faces of the current state with a marker on each of their four edges
                               (sec. 2.4: resolved by the face-centre colour) */
    int64_t n_surrogate;    /* cells the learned surrogate computed in the last ebit_front2vof (0 when it
                               was not set) */
} ebit_stats_t;

/*
 * Statistics of the current state and of C (the array last passed to
 * ebit_front2vof).  Synchronises `stream`.  Returns EBIT_ECFL if any sweep
 * so far broke the Courant limit, else EBIT_OK.
 */
int ebit_stats(ebit_ctx *ctx, const void *C, ebit_stats_t *out, void *stream);

/* The paper's error measures (sec. 3.1.2, eqs. Eq_error_surface and
 * Eq_error_shape) of a volume-fraction field C against a reference C0 (the
 * initial field, or one from another run), both device arrays of n^3 cells in
 * the context's precision:
 *   volume, volume_ref   compensated sums of C and of C0 (cell units)
 *   l1_diff              sum over cells of |C - C0|
 *   e_shape              l1_diff / volume_ref (Eq_error_shape; meaningful
 *                        when the interface should be back where C0 has it)
 *   e_mass               mean of |volume - volume_ref| / volume_ref over the
 *                        calls since the last one with `reset` set, this one
 *                        included (Eq_error_surface when called once after
 *                        every step's ebit_front2vof with the initial C0)
 * One fixed-order reduction over both arrays (deterministic); synchronises
 * `stream`. */
typedef struct {
    double volume, volume_ref, l1_diff, e_shape, e_mass;
    int64_t samples;        /* calls in the e_mass mean */
} ebit_errors_t;
int ebit_errors(ebit_ctx *ctx, const void *C, const void *C0, int reset, ebit_errors_t *out, void *stream);

/* Index (0 or 1) of the state buffer holding the current state. */
int ebit_current(const ebit_ctx *ctx);

/*
 * `nsteps` steps of the hot path, launched from the library: per step k the
 * sweeps along x, y and z (ebit_advect_sweep with time factor g[k] and step
 * dt, the time level of the step for all three, sec. 2.3), then Front2VOF
 * into C (ebit_front2vof) unless C is NULL.  With EBIT_OPT_FUSE on (the
 * default), the Front2VOF of step k < nsteps - 1 runs in one launch with the
 * x sweep of step k + 1 -- with a surrogate set, its classify pass, the
 * network's pass following that launch (same results; C is complete when
 * the enqueued work ends).  Within the call each sweep knows the axis of the
 * next one and passes on a narrower band of bricks (again the same results).
 *   U       3 device pointers: U_x, U_y, U_z (n^3 each, the precision's type)
 *   g       host array of nsteps time factors
 * Returns the first error of the calls it makes (the steps before it are
 * enqueued).
 */
int ebit_advance(ebit_ctx *ctx, int32_t nsteps, const void *const *U, const double *g, double dt, void *C,
                 void *stream);

/* Option switches. */
enum {
    EBIT_OPT_FULL_GRID = 1,   /* 1: process every cell, not only the band */
    EBIT_OPT_TIMING = 2,      /* k > 0: bracket every k-th launch of each kind (sweep, Front2VOF,
                                 Front2VOF with an x sweep) with HIP events on its stream; 0: off */
    EBIT_OPT_FUSE = 3,        /* 1 (default): ebit_advance fuses a Front2VOF with the next x sweep;
                                 0: separate launches */
    EBIT_OPT_SUBLIST_CAP = 4, /* k > 0: at most k entries per sub-list of the brick lists, the rest in
                                 their overflow sub-list (for tests of that path); 0: the default.
                                 Only before the first sweep or Front2VOF (else EBIT_ESTATE); rebuilds
                                 the lists and synchronises the device. */
    EBIT_OPT_ORDER = 5        /* 1: before each sweep and each Front2VOF that is not over the whole
                                 grid, its brick list is rewritten in brick order (three small extra
                                 launches each; fewer HBM fetches on large bands); 0: claim order.
                                 Results are identical.  Default 1 for n >= 512, else 0. */
};
int ebit_set_option(ebit_ctx *ctx, int option, int value);

/* Launch times recorded while EBIT_OPT_TIMING is on (at most 8192 timed
 * launches between two calls; later ones are not timed).  Each bracketed
 * duration includes the launch's dispatch and completion on the stream. */
typedef struct {
    int64_t sweeps;         /* timed ebit_advect_sweep launches */
    double sweep_ms;        /* their summed duration */
    int64_t f2v;            /* timed Front2VOF launches (the surrogate's included) */
    double f2v_ms;
    int64_t fused;          /* timed launches of a Front2VOF with the next x sweep (ebit_advance) */
    double fused_ms;
} ebit_timing_t;

/* Read and reset the accumulated launch times.  Synchronises with the last
 * timed launch. */
int ebit_timing(ebit_ctx *ctx, ebit_timing_t *out);

/* ------------------------------------------------------------------------ *
 * Learned Front2VOF surrogate (not part of the paper): a multilayer
 * perceptron 20 -> 128 -> 128 -> 1 (ReLU, ReLU, sigmoid) from a cell's 12
 * edge-marker fractions (0 where an edge has no marker; edge id 4e + oA + 2 oB
 * along axis e with offsets oA, oB on the two other axes A < B) and its 8
 * corner colours (corner k = ox + 2 oy + 4 oz) to its volume fraction.
 * Parameters: float32 vector of ebit_mlp_param_count() numbers, in order
 * W1 (20 x 128, row-major in x out), b1 (128), W2 (128 x 128), b2 (128),
 * w3 (128), b3 (1).  Products run on bfloat16 matrix cores with float32
 * accumulation; rounding to bfloat16 (nearest, ties to even) happens at the
 * inputs, W1, W2 and the first hidden layer (forward) and at dz2, dz1
 * (backward).  Input rows x: bfloat16, 32 per row (features 0..19, then 0).
 * ------------------------------------------------------------------------ */

/* Number of parameters (19329). */
int ebit_mlp_param_count(void);

/* Device scratch bytes ebit_mlp_gradient and ebit_mlp_train need (partial
 * sums per workgroup and the parameters rounded to bfloat16 in the layout the
 * kernels stage; about 20 MB).  The scratch pointer must be 16-byte aligned. */
size_t ebit_mlp_scratch_bytes(void);

/* y[i] = network(x row i) for m rows (device pointers).  Async on stream. */
int ebit_mlp_forward(const float *theta, const void *x_bf16, int64_t m, float *y, void *stream);

/* Gradient of the mean squared error (1/m) sum (y_i - c_i)^2 with respect to
 * theta into grad (float32, param_count), the loss into *loss (device, may be
 * NULL).  Partial sums per workgroup are added in a fixed order
 * (deterministic).  scratch: device, >= ebit_mlp_scratch_bytes(). */
int ebit_mlp_gradient(const float *theta, const void *x_bf16, const float *c, int64_t m, float *grad, float *loss,
                      void *scratch, size_t scratch_bytes, void *stream);

/* Rows per call of ebit_mlp_gradient_static. */
#define EBIT_MLP_STATIC_MAX_ROWS 8192

/* ebit_mlp_gradient for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same result, bit for bit, as ebit_mlp_gradient on
 * the same rows, with the work space in a static device array of the library
 * (about 10 MB per GPU, held until the process ends) instead of a caller
 * buffer.  theta, x_bf16, c, grad, loss as for ebit_mlp_gradient.
 *   m       1 .. EBIT_MLP_STATIC_MAX_ROWS rows; larger m returns EBIT_ETOOBIG
 *           (nothing is enqueued)
 * Allocates nothing: no hipMalloc / hipFree, no library call that allocates.
 * The first call on a device looks up that device's copy of the array.  Every
 * call on one GPU shares that GPU's array, so calls that overlap on one GPU
 * (other streams, other host threads) race: order them on one stream.
 * Nothing in the array needs clearing: each call writes every entry it reads.
 * EBIT_EINVAL for null pointers or m <= 0; EBIT_EHIP if the device or the
 * array's address cannot be obtained. */
int ebit_mlp_gradient_static(const float *theta, const void *x_bf16, const float *c, int64_t m, float *grad,
                             float *loss, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step >= 1)
 * on theta with first / second moments m1, m2 (float32, param_count each). */
int ebit_mlp_adam(float *theta, float *m1, float *m2, const float *grad, int64_t step, float lr, void *stream);

/* `steps` training steps on the device without returning to the caller: step
 * s takes the mini-batch of rows idx[s batch .. (s + 1) batch - 1] of x / c
 * (nrows rows each; idx NULL: rows 0 .. batch - 1 every step), the gradient
 * of ebit_mlp_gradient on it, then the Adam step of ebit_mlp_adam with
 * learning rate lr[s] and step count step0 + s + 1.  Same results, bit for
 * bit, as those calls on the gathered rows.  idx: device int64, steps x batch
 * entries in [0, nrows) (an entry outside that range is not read: its row
 * counts as all-zero inputs with no loss, a wrong result, not a fault; the
 * caller checks).  lr: host, `steps` floats.  losses: device, `steps` floats
 * (the mean squared error of each step's batch before its update) or NULL.
 * theta / m1 / m2 are updated in place; scratch as for ebit_mlp_gradient.
 * Async on stream.  EBIT_EINVAL for null pointers, nrows <= 0, batch <= 0,
 * steps < 0, step0 < 0, batch > nrows without idx, or unaligned scratch. */
int ebit_mlp_train(float *theta, float *m1, float *m2, const void *x_bf16, const float *c, int64_t nrows,
                   const int64_t *idx, int64_t batch, int64_t steps, const float *lr, int64_t step0, float *losses,
                   void *scratch, size_t scratch_bytes, void *stream);

/* Use the surrogate inside ebit_front2vof (theta: device parameters, read
 * during this call: the weights are copied, rounded to bfloat16, into the
 * context's work area, so later changes to theta need another call; the call
 * synchronizes the device.  NULL switches back to the geometric construction
 * only).
 * Cells with a 4-marker face or more than one loop always use the geometric
 * Front2VOF of sec. 2.5; the others take the network's output. */
int ebit_set_surrogate(ebit_ctx *ctx, const float *theta);

/* Training rows for the surrogate from the current state: for every
 * unambiguous interfacial cell recomputed by the last ebit_front2vof (all of
 * them when that call used a new C), its input row (bfloat16, 32 per row) and
 * its geometric volume fraction (float32).  *count receives the number of
 * rows; at most cap rows are written (x_bf16 / c may be NULL to only count).
 * Rows are ordered by chunk (deterministic).  Synchronises stream. */
int ebit_surrogate_dataset(ebit_ctx *ctx, void *x_bf16, float *c, int64_t cap, int64_t *count, void *stream);

/* ------------------------------------------------------------------------ *
 * Coupling of C to a flow solver (sec. 2.5: the volume fraction from
 * Front2VOF feeds a well-balanced continuum-surface-force term whose
 * curvature comes from height functions).  Context-free: any n^3 periodic
 * C field (doubles, or floats with EBIT_FP32; h = 1/n), device pointers,
 * async on `stream`.  All arithmetic is FP64, in the order stated.
 * ------------------------------------------------------------------------ */

/* Curvature kappa (1/length) and a status per cell:
 *   0  C is 0 or 1 (kappa 0)
 *   1  height functions along the direction of the largest component of
 *      Youngs' gradient (weights (1,2,1) x (1,2,1) over the 3x3 cells
 *      across each axis of C(+1) - C(-1)); 2  along another one, tried in
 *      decreasing order of that component (ties: lower axis)
 *   3  no direction had heights: the mean of the neighbours (26, added in
 *      z, y, x order) with status 1 or 2;  4  none had (kappa 0)
 * Heights: for direction d the 9 columns at offsets -1..1 on the two other
 * axes, 7 cells each (-3..3 along d); a column is valid when its end cells
 * hold exactly 1 and 0, all 9 with the same orientation o (+1: phase 1 at
 * -3).  z = sum - 7/2 (o = +1) or 7/2 - sum, summing from -3 up; with
 * za, zb (central), zaa, zbb (second) and zab (cross, /4) differences of z,
 * kappa = -o (zaa (1 + zb^2) + zbb (1 + za^2) - 2 zab za zb) / (t sqrt(t) h),
 * t = 1 + za^2 + zb^2: positive where phase 1 is convex (2/R on a sphere).
 *   kappa   n^3 (the precision's type), status n^3 bytes: outputs
 *   work    device, >= ebit_curvature_work_bytes(n), 4-byte aligned: the list
 *           of cells with 0 < C < 1 that the dense passes take
 * EBIT_EINVAL for bad arguments, EBIT_ESCRATCH for a short work space. */
size_t ebit_curvature_work_bytes(int32_t n);   /* device work space of ebit_curvature (0 for a bad n) */
int ebit_curvature(int32_t n, int32_t precision, const void *C, void *kappa, uint8_t *status, void *work,
                   size_t work_bytes, void *stream);

/* CSF force density on the lower face of every cell along each axis:
 * F_d(p) = sigma kappa_f (C(p) - C(p - e_d)) / h, with kappa_f the mean of
 * the curvatures of the two cells that have status 1..3 (the one that has,
 * 0 if neither).  F: 3 device pointers, n^3 each (outputs). */
int ebit_csf(int32_t n, int32_t precision, const void *C, const void *kappa, const uint8_t *status, double sigma,
             void *const *F, void *stream);

/* The AMR-compatible refinement band (sec. 2.3: every cell of the 3x3x3
 * block around an interfacial cell is refined to the finest level; with a
 * Courant number of at most one the next step's interface stays inside it).
 * From a state's flags (n^3, the layout above; e.g. buffer ebit_current()):
 *   mask       n^3 bytes out: 1 where a cell lies in the 3x3x3 block of a cell
 *              with a marker on any of its 12 edges, else 0
 *   bricks     (n/4)^3 bytes out, brick (bx, by, bz) at bx + (n/4)(by + (n/4) bz):
 *              1 where one of its 4^3 cells is in the mask (block-structured
 *              refinement)
 *   mask_prev  NULL, or an earlier mask (n^3 bytes) to check against
 *   counts     4 device int64 out: interfacial cells, cells in the mask, bricks,
 *              interfacial cells outside mask_prev (0 without it)
 *   work       device, >= ebit_refine_work_bytes(n) (16 KB), 8-byte aligned: partial counts
 * flags, mask and mask_prev must be 4-byte aligned (whole words are read and written).
 * n a multiple of 4.  Async on `stream`.  EBIT_EINVAL / EBIT_ESCRATCH on bad
 * arguments. */
size_t ebit_refine_work_bytes(int32_t n);
int ebit_refine_band(int32_t n, const uint8_t *flags, const uint8_t *mask_prev, uint8_t *mask, uint8_t *bricks,
                     int64_t *counts, void *work, size_t work_bytes, void *stream);

/* Free the context (not the caller's buffers). */
void ebit_destroy(ebit_ctx *ctx);

/* Static message for an error code. */
const char *ebit_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* EBIT_H */
