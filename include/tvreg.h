/*
 * tvreg.h -- C ABI of the MI355X (gfx950) library for TV-regularised CT
 * reconstruction: the per-iteration evaluation of
 *
 *     phi(x) = 1/2 |A x - b|_2^2 + alpha T_tau(x),   x in Q = {x >= 0},
 *
 * (Sec. II-A, eq. 1, with the TV of eq. 2 Huber-smoothed by tau) and its
 * gradient, driven by the gradient projection method (Sec. III-A, eq. 6),
 * GPBB (Alg. 1) and UPN (Alg. 3, with BT of Alg. 2 and the mu estimate of
 * eq. 9), all stopped on the gradient map (Sec. III-D, eq. 10).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Volume x: nz x ny x nx, x fastest (index i + nx (j + ny k)); voxel
 *    (i, j, k) is the unit box [i - nx/2, i + 1 - nx/2] x [j - ny/2, ...] x
 *    [k - nz/2, ...], cells half-open.
 *  - Projection data: n_views x det_rows x det_cols, column fastest.
 *  - A (the paper's system matrix, left unspecified there): one ray through
 *    each detector pixel centre, a_ij = exact length of ray i in voxel j.
 *    View theta: e_s = (cos, sin, 0), e_u = (-sin, cos, 0), e_v = z; pixel
 *    centre u = (col - (cols-1)/2) pitch_u, w = (row - (rows-1)/2) pitch_v.
 *    Parallel beam: the line through u e_u + w e_v with direction e_s.
 *    Cone beam: the segment from R e_s to -(SDD - R) e_s + u e_u + w e_v.
 *    3D parallel beam (Sec. IV-A: view directions over the unit sphere):
 *    view v has the unit direction d = view_dirs[v] / |view_dirs[v]| and the
 *    detector axes e_u = e_z x d / |e_z x d| (e_x when d runs along z),
 *    e_v = d x e_u (for d = (cos, sin, 0) the parallel beam's axes); pixel
 *    (row, col) is the line through u e_u + w e_v along d.  Its A^T is
 *    evaluated by a voxel-driven gather over the same crossings.
 *  - Precision: TVREG_F32_RED64 stores vectors as float (32-bit) and forms
 *    every inner product, objective value, step length, line-search test and
 *    stop test in double; ray geometry is double in both modes.  TVREG_F64
 *    is double throughout.  "T" below is float or double accordingly.
 *  - Pointers named *_dev are device pointers (HIP); all device buffers are
 *    owned by the caller.  Every call is asynchronous on `stream` (a
 *    hipStream_t, NULL = default stream) unless stated otherwise.
 *  - Errors: a negative status means nothing was written; tvreg_last_error()
 *    returns a thread-local message.  A positive status means the outputs are
 *    valid but flagged.
 */
#ifndef TVREG_H
#define TVREG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TVREG_OK = 0,
    TVREG_EINVAL = -1,   /* bad argument (dimension, pointer, parameter) */
    TVREG_ENOMEM = -2,   /* workspace too small or allocation failed */
    TVREG_EDEVICE = -3,  /* HIP runtime error */
    TVREG_ENOTCONV = 1,  /* max_iter reached before the stop test held */
    TVREG_ESTALL = 2     /* a line-search cap was hit; last accepted x returned */
} tvreg_status;

typedef enum { TVREG_PARALLEL = 0, TVREG_CONE = 1, TVREG_PARALLEL_3D = 2 } tvreg_beam;
typedef enum { TVREG_F32_RED64 = 0, TVREG_F64 = 1 } tvreg_precision;
/* TVREG_NESTEROV: Nesterov's method for given mu and L (Sec. III-B, the rate
   of eq. 8): UPN's recursion with L_k = L_bar (no line search) and
   mu_k = mu_bar (no eq. 9 estimate); convergent when L_bar is at least the
   gradient's Lipschitz constant and mu_bar at most the strong-convexity
   parameter. */
typedef enum { TVREG_GP = 0, TVREG_GPBB = 1, TVREG_UPN = 2, TVREG_NESTEROV = 3 } tvreg_method;

/* Scan geometry (all lengths in voxel units, volume centred at the origin). */
typedef struct {
    int32_t nx, ny, nz;          /* volume size, each >= 1 */
    int32_t n_views;             /* >= 1 */
    const double *angles_rad;    /* host array of n_views view angles (copied);
                                    unused (may be NULL) for TVREG_PARALLEL_3D */
    tvreg_beam beam;
    int32_t det_cols, det_rows;  /* >= 1 */
    double pitch_u, pitch_v;     /* > 0 */
    double src_to_centre;        /* cone: R, must exceed the volume's half diagonal */
    double src_to_det;           /* cone: SDD, SDD - R must exceed the half diagonal */
    const double *view_dirs;     /* TVREG_PARALLEL_3D: host array of n_views directions
                                    (x, y, z), finite and nonzero, normalised and
                                    copied; ignored by the other beams */
} tvreg_geometry_desc;

typedef struct tvreg_geometry tvreg_geometry; /* opaque, library-owned */

/*
 * Builds the device-side ray tables of a geometry (a few doubles per view,
 * detector column and row; the only device memory the library allocates;
 * tvreg_solve and the unrolled UPN calls hold a page-locked host copy of
 * their few scalar sums for the duration of the call).
 * Returns TVREG_EINVAL for non-positive sizes or pitches, NULL pointers, or a
 * cone whose source or detector is inside the volume's bounding sphere.
 * Synchronous.
 */
tvreg_status tvreg_create_geometry(const tvreg_geometry_desc *desc, tvreg_precision precision,
                                   tvreg_geometry **out);
void tvreg_destroy_geometry(tvreg_geometry *geom);

/*
 * y = A x  (the forward mapping of Sec. IV-A).  x_dev: N values of T,
 * y_dev: m values of T (overwritten).  Ray sums accumulate in double.
 */
tvreg_status tvreg_project(const tvreg_geometry *geom, const void *x_dev, void *y_dev,
                           void *stream);
/*
 * The same y = A x as the solvers project: the companion copy of x for the
 * geometry's ray tile (see the tile shapes below) is written to ws_dev
 * (tvreg_project_workspace_bytes: N values of T) and the walk reads it, at
 * the solvers' rate.  Equal to tvreg_project's y bit for bit.  ENOMEM for a
 * short workspace.
 */
size_t tvreg_project_workspace_bytes(const tvreg_geometry *geom);
tvreg_status tvreg_project_ws(const tvreg_geometry *geom, const void *x_dev, void *y_dev,
                              void *ws_dev, size_t ws_bytes, void *stream);

/*
 * x = A^T r  (the data part of grad phi, Sec. III-A eq. 6 needs grad f).
 * r_dev: m values of T; x_dev: N values of T (overwritten).  Computed as a
 * gather: every voxel sums, view by view, the rays crossing it with the same
 * lengths the projector uses, in a fixed order (run-to-run bitwise
 * reproducible, no atomics).
 */
tvreg_status tvreg_backproject(const tvreg_geometry *geom, const void *r_dev, void *x_dev,
                               void *stream);

/*
 * Stored transpose (optional).  By default the backprojector evaluates every
 * ray/voxel length from the geometry on the fly.  A geometry can instead
 * hold A^T in caller-owned device memory, voxel-major, built once by the
 * same enumeration and crossing formula (each length rounded once to T), and
 * stream it: tvreg_backproject, tvreg_objective_grad, tvreg_solve,
 * tvreg_solve_batched (per problem) and the unrolled solver then use it.
 * The forward projector always walks the rays on the fly (cheaper than
 * streaming a ray-major copy).
 *
 * tvreg_matrix_plan counts the entries (GPU pass; needs scratch of
 * tvreg_matrix_scratch_bytes) and returns the bytes tvreg_matrix_attach will
 * need and, if nnz != NULL, the number of non-zeros.  tvreg_matrix_attach
 * builds the matrix into matrix_dev (which must stay allocated and unchanged
 * until tvreg_matrix_detach or tvreg_destroy_geometry) and switches the
 * geometry's backprojector to it; it synchronises `stream`.  Neither may run
 * while another call uses the geometry.  Size: about (sizeof(T) + 4) bytes
 * per stored entry plus slice padding (1.3e9 non-zeros, 12 GiB in FP32, for
 * a 256^3 cone-beam scan of 60 views at 384 x 256; 1.4 GiB when the scan's
 * symmetry is used, see below).
 */
/*
 * Symmetric storage.  A circular cone scan whose views are evenly spaced
 * over the full circle maps onto itself under turns of the volume about z:
 * with V divisible by 4 and a square volume of even side, turning by a
 * quarter carries ray (view v, row, col) onto ray (v + V/4, row, col) and
 * voxel (i, j, k) onto (nx - 1 - j, i, k), so both have the same length (V
 * even, ny even: the half turn, v + V/2 and (nx - 1 - i, ny - 1 - j)); with
 * nz even the mirror z -> -z carries row r onto rows - 1 - r and k onto
 * nz - 1 - k.  The stored transpose of such a geometry keeps only the voxels
 * of one cell of that group (a quadrant of the plane times the lower half in
 * z: one eighth of the entries for the 256^3 scan of 60 views) and its
 * product applies every entry to all images of its voxel.  The lengths of
 * the images are those of the stored voxel's rays: equal to the ones the
 * projector computes for the image rays up to the rounding of the view
 * angles' cosines (about 1e-16 relative before the rounding to T).  Used only
 * for the cone beam with an even detector in both directions (no ray runs
 * inside a voxel face), view directions matching the turn to 1e-12, and
 * views, rows and columns that pack into 31 bits.  On by default.
 * Without a stored transpose the on-the-fly backprojector uses the same
 * group (no packing limit): one thread finds the rays and lengths of its
 * cell voxels once per view and applies them to every image, so it does a
 * fraction of the ray arithmetic; the identity image's sums are the plain
 * gather's, bit for bit.
 * tvreg_set_symmetry(geom, 0) keeps every voxel (the plain layout and the
 * plain gather), 1 uses the symmetry again; it must precede
 * tvreg_matrix_plan / attach (EINVAL while a transpose is attached).  tvreg_matrix_symmetry returns the number
 * of voxels one stored entry serves (1, 2, 4 or 8) for the attached
 * transpose or, before attaching, for the one tvreg_matrix_attach would
 * build.
 */
tvreg_status tvreg_set_symmetry(tvreg_geometry *geom, int32_t use);
int32_t tvreg_matrix_symmetry(const tvreg_geometry *geom);

size_t tvreg_matrix_scratch_bytes(const tvreg_geometry *geom);
tvreg_status tvreg_matrix_plan(const tvreg_geometry *geom, void *scratch_dev, size_t scratch_bytes,
                               size_t *matrix_bytes, int64_t *nnz, void *stream);
tvreg_status tvreg_matrix_attach(tvreg_geometry *geom, void *matrix_dev, size_t matrix_bytes,
                                 void *stream);
tvreg_status tvreg_matrix_detach(tvreg_geometry *geom);

/*
 * Tile shapes of the on-the-fly operators (a performance choice only: every
 * shape gives bitwise identical projections and backprojections; the block
 * partial sums of the projector's fused residual norm, and so the last bits
 * of the solver's FP64 sums, follow the shape).
 *   project_tile_cols  detector columns of the ray tile one wavefront walks;
 *                      the tile is project_tile_cols x (64 / project_tile_cols)
 *                      pixels: 1, 2 (column tiles), 8, 16, 32 or 64 (row
 *                      tiles); default 2 for a detector with a multiple of
 *                      32 rows, else 64.  Inside
 *                      the solvers the projector reads a companion copy of
 *                      the volume made before each projection (z fastest for
 *                      column tiles, y fastest for row tiles);
 *                      tvreg_project reads the volume itself;
 *   project_waves      ray tiles per projector block, stacked along the
 *                      detector rows: 1, 2, 4 (default) or 8;
 *   backproject_depth  voxels per thread along z in the on-the-fly
 *                      backprojector: 4, 8 (default) or 16.
 * tvreg_autotune times every shape on the geometry (zero-filled synthetic
 * operands in `ws_dev`, `reps` launches per shape after one warm-up, HIP
 * events on `stream`), keeps the fastest of each operator in the geometry
 * and reports all timings; it synchronises `stream` and must not run while
 * another call uses the geometry.  The backprojector is timed on the fly
 * even when a stored transpose is attached.  tvreg_solve_batched runs every
 * problem with its own geometry's shapes, except a backprojector depth of 16,
 * which it runs at 8 (every depth gives bitwise the same result).
 */
typedef struct {
    int32_t project_tile_cols;
    int32_t project_waves;
    int32_t backproject_depth;
    int32_t reserved;            /* 0 */
    double project_ms[6][4];     /* tvreg_autotune: ms per projection, [tile cols 1, 2, 8, 16,
                                    32, 64][waves 1, 2, 4, 8] */
    double backproject_ms[3];    /* tvreg_autotune: ms per backprojection for depth 4, 8, 16 */
} tvreg_tuning;
size_t tvreg_autotune_workspace_bytes(const tvreg_geometry *geom);
tvreg_status tvreg_autotune(tvreg_geometry *geom, void *ws_dev, size_t ws_bytes, int32_t reps,
                            tvreg_tuning *out, void *stream);
/* the geometry's current shapes (timings zero) */
tvreg_status tvreg_get_tuning(const tvreg_geometry *geom, tvreg_tuning *out);
/* sets both shapes; EINVAL for a value outside the lists above */
tvreg_status tvreg_set_tuning(tvreg_geometry *geom, const tvreg_tuning *tuning);

/* Bytes of device workspace tvreg_tv_grad and tvreg_objective_grad need. */
size_t tvreg_tv_workspace_bytes(int32_t nx, int32_t ny, int32_t nz);

/*
 * grad_dev = grad T_tau(x) and, when tv_value_dev != NULL, *tv_value_dev =
 * T_tau(x) as one double in device memory (eq. 2 smoothed:
 * T_tau(x) = sum_j Phi_tau(D_j x), Phi_tau(z) = |z| - tau/2 for |z| >= tau,
 * |z|^2/(2 tau) otherwise; D_j forward differences, zero across the upper
 * volume faces).  workspace_dev may be NULL when tv_value_dev is NULL.
 */
tvreg_status tvreg_tv_grad(int32_t nx, int32_t ny, int32_t nz, tvreg_precision precision,
                           double tau, const void *x_dev, void *grad_dev, double *tv_value_dev,
                           void *workspace_dev, size_t workspace_bytes, void *stream);

/*
 * tvreg_tv_grad without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc).  Same kernels, arguments and results as tvreg_tv_grad (bit for
 * bit); the per-block partial sums of the TV value live in a static device
 * array of the library instead (about 3.75 MiB, one per device, held until
 * the process ends).  That array bounds the volume: the TV grid of
 * ceil(nx/64) x ceil(ny/4) x ceil(nz/16) blocks may have at most 32768
 * blocks (512^3 voxels fit); larger volumes return TVREG_EINVAL.  Calls on
 * one device share the array: calls that overlap in time on one GPU (other
 * streams, other threads) race and must be serialised by the caller.  The
 * call allocates nothing: no hipMalloc, no hipFree, no allocating library
 * routine.  The first call on a device looks the array's address up
 * (hipGetSymbolAddress), a synchronous runtime query.
 */
tvreg_status tvreg_tv_grad_noalloc(int32_t nx, int32_t ny, int32_t nz, tvreg_precision precision,
                                   double tau, const void *x_dev, void *grad_dev,
                                   double *tv_value_dev, void *stream);

/*
 * out_dev = H(y) v, the Hessian of T_tau at y applied to v (the derivative of
 * the gradient above along v): sum_j D_j^T dq_j with dq_j = D_j v / tau where
 * |D_j y| < tau and (e - u (u.e)) / |D_j y|, u = D_j y / |D_j y|, e = D_j v,
 * where |D_j y| >= tau.  With grad_dot_dev != NULL also *grad_dot_dev =
 * <v, grad T_tau(y)> (double, device; needs the workspace of
 * tvreg_tv_workspace_bytes).  out must not alias y or v.  Used by the
 * reverse pass of the unrolled solver; exposed for testing and reuse.
 */
tvreg_status tvreg_tv_hessvec(int32_t nx, int32_t ny, int32_t nz, tvreg_precision precision,
                              double tau, const void *y_dev, const void *v_dev, void *out_dev,
                              double *grad_dot_dev, void *workspace_dev, size_t workspace_bytes,
                              void *stream);

/* Bytes of device workspace tvreg_objective_grad needs for this geometry. */
size_t tvreg_objective_workspace_bytes(const tvreg_geometry *geom);

/*
 * One gradient evaluation: grad_dev = A^T (A x - b) + alpha grad T_tau(x)
 * and *phi_dev = 1/2 |A x - b|^2 + alpha T_tau(x) (double, device).
 * b_dev: m values of T.
 */
tvreg_status tvreg_objective_grad(const tvreg_geometry *geom, const void *b_dev, double alpha,
                                  double tau, const void *x_dev, void *grad_dev,
                                  double *phi_dev, void *workspace_dev, size_t workspace_bytes,
                                  void *stream);

typedef struct {
    tvreg_method method;
    double alpha, tau;
    double eps;              /* stop tolerance */
    int32_t stop_mode;       /* 0: |G|/|G_0| <= eps;  1: |G|/N <= eps (as printed) */
    int32_t max_iter;        /* outer iterations (BT or GPBB steps) */
    double L_bar;            /* initial Lipschitz estimate (Alg. 2/3 input), > 0;
                                NESTEROV: the given L */
    double mu_bar;           /* UPN initial mu; <= 0 selects L_0 / 4;
                                NESTEROV: the given mu, in [0, L_bar] */
    double rho_L;            /* BT growth factor, > 1 */
    int32_t gpbb_K;          /* GPBB nonmonotone memory, 0..16 */
    double gpbb_sigma;       /* GPBB sufficient-decrease weight */
    double gpbb_beta0;       /* GPBB initial step fraction in (0, 1) */
    int32_t max_trials;      /* cap on BT growths / GPBB squarings per iteration */
    double *hist_phi;        /* optional host arrays of hist_len entries: phi of */
    double *hist_gm;         /* each accepted point, |G|/|G_0| of each iteration, */
    double *hist_L;          /* and the step's L (1/theta for GPBB) */
    int32_t hist_len;
    int32_t use_box;         /* 0: Q = {x >= 0} (Sec. IV-A); 1: Q = [lower, upper]^N */
    double lower, upper;     /* use_box: lower < upper, either may be infinite */
} tvreg_solve_params;

typedef struct {
    int32_t iters;           /* outer iterations performed */
    int32_t grad_evals;      /* evaluations of grad f (A^T and TV gradient) */
    int32_t func_evals;      /* evaluations of f at trial points (A and TV value) */
    double phi;              /* phi at the returned x */
    double gm_rel;           /* last |G| / |G_0| */
    double gm_abs_over_N;    /* last |G| / N (the printed stop quantity) */
    double L, mu;            /* final Lipschitz and strong-convexity estimates */
    int32_t stop_reason;     /* tvreg_status of the run */
} tvreg_solve_info;

/* Bytes of device workspace tvreg_solve needs for this geometry and method. */
size_t tvreg_solve_workspace_bytes(const tvreg_geometry *geom, tvreg_method method);

/*
 * Solves min_{x in Q} phi(x) with GP (eq. 6, step 1/L_k from BT warm-started
 * at L_{k-1}), GPBB (Alg. 1), UPN (Alg. 3) or Nesterov's method for given mu
 * and L; Q is the nonnegative orthant or, with use_box, [lower, upper]^N
 * (P_Q a clip).  x_inout_dev holds x_0 on entry (projected onto Q) and the
 * last accepted iterate on return.
 * b_dev: m values of T.  The line-search decisions and the mu estimate are
 * evaluated in the rearranged form Bregman_f(x, y) vs L/2 |x - y|^2 (the
 * same inequality as Alg. 2 / eq. 9 without subtracting two objective
 * values).  Synchronises `stream` once per line-search trial (the calling
 * thread polls an event, so it stays busy while the device works) and before
 * returning; `info` is written on the host.  Returns TVREG_OK,
 * TVREG_ENOTCONV or TVREG_ESTALL, or a negative error.
 */
tvreg_status tvreg_solve(const tvreg_geometry *geom, const void *b_dev,
                         const tvreg_solve_params *params, void *x_inout_dev,
                         void *workspace_dev, size_t workspace_bytes, tvreg_solve_info *info,
                         void *stream);

/* Bytes of device workspace tvreg_solve_batched needs for these n geometries. */
size_t tvreg_solve_batched_workspace_bytes(int32_t n, const tvreg_geometry *const *geoms);

/*
 * n independent GP (eq. 6) or UPN (Alg. 3) solves run together: problem i has
 * its own geometry geoms[i], data b_dev[i] (m_i values of T), parameters
 * params[i] (alpha, eps, L_bar, ... each its own) and start / result
 * x_inout_dev[i] (N_i values of T).  The problems take exactly the steps and
 * decisions tvreg_solve takes for each of them alone (same kernels, same
 * partial-sum order, same double arithmetic for the line search of Alg. 2,
 * the mu estimate of eq. 9 and the stop test), so every result is the one
 * tvreg_solve returns; only the launch structure differs: one line-search
 * trial of every running problem is one round of grouped launches plus a
 * device-side control step, captured once as a HIP graph and replayed; the
 * host reads one running-problem count every `poll_rounds` rounds (<= 0
 * selects 8).
 * All geometries share one precision and one device.  GPBB is not batched
 * (TVREG_EINVAL); the history arrays of params are ignored.  geoms, b_dev,
 * params, x_inout_dev and infos are host arrays of n entries; b_dev and
 * x_inout_dev entries are device pointers.  infos[i] is written on the host,
 * its stop_reason holds problem i's status.  Returns TVREG_OK when every
 * problem converged, else TVREG_ESTALL if one stalled, else TVREG_ENOTCONV,
 * or a negative error.  Synchronises `stream`.
 */
tvreg_status tvreg_solve_batched(int32_t n, const tvreg_geometry *const *geoms,
                                 const void *const *b_dev, const tvreg_solve_params *params,
                                 void *const *x_inout_dev, void *workspace_dev,
                                 size_t workspace_bytes, int32_t poll_rounds,
                                 tvreg_solve_info *infos, void *stream);

/*
 * Differentiated form of UPN (not a passage of the paper: it differentiates
 * the map Alg. 3 applies).  The forward pass runs K UPN steps from x = 0:
 * step j maps y^(j) to x^(j+1) = P_Q(y^(j) - grad f(y^(j)) / L_j) with L_j
 * from BT (Alg. 2 in Bregman form, started at L_bar, then at L_{j-1}) or,
 * when L_replay != NULL, taken from L_replay[j] with no test; mu_j follows
 * eq. 9 (skipped while x^(j) = y^(j)), theta and beta follow Alg. 3, and
 * xK_dev receives x^(K) (the K-th BT output).  Uses params->alpha, tau,
 * L_bar, mu_bar, rho_L and max_trials; params->method must be TVREG_UPN and
 * use_box 0 (Q is the nonnegative orthant), else TVREG_EINVAL.  The tape
 * (device workspace of tvreg_unrolled_workspace_bytes) keeps the step
 * scalars and (x, y) every ckpt_every steps; L_out (host, K entries, may be
 * NULL) receives the L_j.
 * Returns TVREG_ESTALL when a BT search hits max_trials (no gradient then).
 *
 * The reverse pass, given dl/dx^(K) (N values of T, device), writes
 * *dl_dlogalpha (host double) and dl_db_dev (m values of T): the gradient of
 * l(x^(K)) with the L_j held fixed (decisions, not functions of alpha or b),
 * the min of eq. 9 differentiated on the branch the forward pass took and
 * P_Q through its mask [x^(j+1) > 0].  It recomputes each segment of
 * ckpt_every steps from its checkpoint (bit-identical to the forward pass)
 * and reads alpha, tau, K and ckpt_every from the tape.  b_dev must be the
 * data of the forward pass.  Both calls synchronise `stream`.
 */
size_t tvreg_unrolled_workspace_bytes(const tvreg_geometry *geom, int32_t K, int32_t ckpt_every);
tvreg_status tvreg_upn_unrolled_fwd(const tvreg_geometry *geom, const void *b_dev,
                                    const tvreg_solve_params *params, int32_t K,
                                    int32_t ckpt_every, const double *L_replay, double *L_out,
                                    void *xK_dev, void *tape_dev, size_t tape_bytes,
                                    void *stream);
tvreg_status tvreg_upn_unrolled_bwd(const tvreg_geometry *geom, const void *b_dev,
                                    void *tape_dev, size_t tape_bytes, const void *xK_bar_dev,
                                    double *dl_dlogalpha, void *dl_db_dev, void *stream);

/*
 * Opt-in instrumentation of tvreg_solve: when enabled, every kernel launch of
 * a solve is bracketed by HIP events on the solve's stream and the elapsed
 * times are summed per kernel (process-wide, thread-safe).  Used by the
 * benchmark to report live per-kernel durations; off by default.
 */
typedef enum {
    TVREG_KERNEL_PROJECT = 0,      /* projector (fused residual and sums) */
    TVREG_KERNEL_BACKPROJECT = 1,  /* gather backprojector */
    TVREG_KERNEL_TV = 2,           /* TV gradient / value / Bregman stencil */
    TVREG_KERNEL_TRIAL = 3,        /* projected trial step with TV value */
    TVREG_KERNEL_EXTRAPOLATE = 4,  /* UPN extrapolation of x and of the residual */
    TVREG_KERNEL_TRANSPOSE = 5,    /* y-fastest copy of the volume read by the projector */
    TVREG_KERNEL_COUNT = 6
} tvreg_kernel_id;
void tvreg_profile_enable(int32_t on);
void tvreg_profile_reset(void);
/* launches counted and their summed duration in milliseconds */
tvreg_status tvreg_profile_get(int32_t kernel, int64_t *count, double *total_ms);

/* Thread-local description of the last error (empty string if none). */
const char *tvreg_last_error(void);

/* Library version string. */
const char *tvreg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TVREG_H */
