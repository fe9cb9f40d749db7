/*
 * FP64 CPU oracle for TV-regularised CT reconstruction -- TEST INFRASTRUCTURE.
 *
 * Plain, slow, deliberately unoptimised reference for the method of
 * "Accelerated gradient methods for total-variation-based CT image
 * reconstruction" (Jorgensen, Jensen, Hansen, Jensen, Sidky, Pan).  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it; the product path never does.  It shares no code with the HIP
 * library.
 *
 * Parity status of each entry point is listed in oracle/__init__.py.
 */
#ifndef TVREG_ORACLE_H
#define TVREG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;
    int32_t n_views;
    const double *angles;   /* n_views view angles, radians */
    int32_t cone;           /* 0: parallel beam about z, 1: circular cone beam,
                               2: parallel beam along given directions (dirs) */
    int32_t cols, rows;     /* detector pixels */
    double pitch_u, pitch_v;
    double src_to_centre;   /* cone only */
    double src_to_det;      /* cone only */
    const double *dirs;     /* beam 2: n_views view directions (x, y, z), any length */
} og_geom;

enum { OG_GP = 0, OG_GPBB = 1, OG_UPN = 2, OG_NESTEROV = 3 };
enum { OG_CONVERGED = 0, OG_NOTCONV = 1, OG_STALL = 2 };

typedef struct {
    int32_t method;
    double alpha, tau, eps;
    int32_t stop_mode;      /* 0: ||G||/||G_0|| <= eps, 1: ||G||/N <= eps (Sec. III-D) */
    int32_t max_iter;
    double L_bar;           /* initial Lipschitz estimate (Alg. 2 / Alg. 3 input) */
    double mu_bar;          /* <= 0: use L_0 / 4 */
    double rho_L;           /* BT growth factor (> 1) */
    int32_t gpbb_K;         /* nonmonotone memory (Alg. 1) */
    double gpbb_sigma;
    double gpbb_beta0;
    int32_t max_trials;     /* BT cap */
    int32_t max_squarings;  /* GPBB cap */
    int32_t force_mu;       /* test hook: 0 normal, 1 mu_k := L_k (mu_0 = L_0),
                               2 mu_0 := L_0 then mu_k := 0 */
    int32_t bt_form;        /* 0: tests as printed (Alg. 2, eq. 9);
                               1: same inequality via the Bregman distance of f */
    double lower, upper;    /* Q = [lower, upper]^N (0, +inf: the nonnegative orthant);
                               the unrolled form always uses the orthant */
} og_params;

typedef struct {
    int32_t iters, grad_evals, func_evals, status;
    double phi, gm, gm0, L, mu;
} og_info;

/* geometry / projector (Sec. II-A: A is the system matrix) */
void og_ray_endpoints(const og_geom *g, int32_t v, int32_t row, int32_t col,
                      double p0[3], double p1[3]);
int32_t og_siddon(const og_geom *g, const double p0[3], const double p1[3],
                  int32_t *idx, double *len, double *work);
double og_slab_length(const double p0[3], const double p1[3], const double lo[3],
                      const double hi[3]);
void og_project(const og_geom *g, const double *x, double *y);
void og_backproject(const og_geom *g, const double *r, double *x);
void og_project_bruteforce(const og_geom *g, const double *x, double *y);
void og_matrix_dense(const og_geom *g, double *A);
double og_ray_sum(const og_geom *g, int32_t v, int32_t row, int32_t col, const double *x);
int64_t og_nnz(const og_geom *g);

/* smoothed TV (eq. 2 with a Huber-smoothed norm) */
double og_tv(int32_t nx, int32_t ny, int32_t nz, double tau, const double *x, double *grad);
double og_huber_bregman(const double a[3], const double b[3], const double d[3], double tau);
double og_tv_bregman(int32_t nx, int32_t ny, int32_t nz, double tau, const double *x,
                     const double *y);

/* objective and gradient of eq. 1 with smoothed TV */
double og_phi(const og_geom *g, const double *b, double alpha, double tau, const double *x);
double og_phi_grad(const og_geom *g, const double *b, double alpha, double tau,
                   const double *x, double *grad);
double og_gradmap_norm(int64_t n, const double *x, const double *grad, double nu);
double og_gradmap_norm_box(int64_t n, const double *x, const double *grad, double nu, double lo,
                           double hi);

/* solvers: GP (eq. 6), GPBB (Alg. 1), UPN (Alg. 3), all with the stop test of Sec. III-D */
int32_t og_solve(const og_geom *g, const double *b, const og_params *p, double *x,
                 og_info *info, double *hist_phi, double *hist_gm, double *hist_L,
                 double *hist_mu, double *hist_theta, int32_t hist_len);

/* same solvers on an explicit dense m x (nx*ny*nz) matrix (tiny systems only) */
int32_t og_solve_dense(int32_t m, int32_t nx, int32_t ny, int32_t nz, const double *A,
                       const double *b, const og_params *p, double *x, og_info *info,
                       double *hist_phi, double *hist_gm, double *hist_L, double *hist_mu,
                       double *hist_theta, int32_t hist_len);

/* differentiated form: Hessian-vector product of the smoothed TV, and K
   unrolled UPN steps from x = 0 with the reverse-mode gradient of
   l(x^(K)) with respect to alpha and b (L decisions held fixed) */
void og_tv_hessvec(int32_t nx, int32_t ny, int32_t nz, double tau, const double *y,
                   const double *v, double *out);
int32_t og_unrolled(const og_geom *g, const double *b, const og_params *p, int32_t K,
                    int32_t replay, double *L, double *xK, const double *xK_bar,
                    double *alpha_bar, double *b_bar, double *mu_out, double *beta_out,
                    int32_t *mu_state, uint64_t *signature);

int32_t og_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
