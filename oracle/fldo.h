/*
 * fldo.h -- interface of the FP64 CPU oracle (test infrastructure only; see
 * fldo.c).  Independent of the HIP library: no shared header, type or
 * constant.
 */
#ifndef FLDO_H
#define FLDO_H

#define FLDO_MAX_LEVELS 16
#define FLDO_MAX_AA 16

enum {
    FLDO_LIMITER_CDA = 0,
    FLDO_LIMITER_LP = 1,
    FLDO_LIMITER_SUM = 2,
    FLDO_LIMITER_MAX = 3,
    FLDO_LIMITER_KERSHAW = 4,
    FLDO_LIMITER_LARSEN = 5
};

enum { FLDO_METHOD_ALG1 = 0, FLDO_METHOD_MG = 1 };

enum {
    FLDO_CONVERGED = 0,
    FLDO_INVALID = 1,
    FLDO_NOT_CONVERGED = 4,
    FLDO_DIVERGED = 5
};

typedef struct fldo_params {
    int nx, ny, nz;           /* unknowns per axis, z fastest */
    double h;                 /* voxel edge length */
    int limiter;              /* FLDO_LIMITER_* */
    double larsen_n;          /* exponent of the Larsen-n limiter */
    double eps;               /* guard/initialisation tolerance (paper: 1e-20) */
    double sigma_eps;         /* extinction floor; <= 0 selects 1e-3/L at set-up */
    double phi_b;             /* Dirichlet ghost fluence */
    int mirror_d;             /* 0: ghost D = eps*h, 1: ghost D = D of the voxel inside */
    const double *ghost_phi;  /* optional padded (nx+2)(ny+2)(nz+2) ghost fluence */
    double jbar;              /* RMS emission (set-up output) */
    double jnorm;             /* ||j||_2 (set-up output) */
    double aniso_g;           /* phase-function anisotropy g: reduced extinction in D and R */
} fldo_params;

typedef struct fldo_solve_opts {
    int method;               /* FLDO_METHOD_* */
    double omega;             /* SOR factor of Alg. 1 */
    double omega_s;           /* relaxation of the multigrid smoother */
    int nu1, nu2;             /* pre/post smoothing sweeps */
    int max_coarsest;         /* max unknowns on the coarsest level */
    int max_iters;            /* Alg. 1 iterations or outer multigrid iterations */
    double tol;               /* stop when ||r||/||j|| <= tol */
    int check_every;          /* Alg. 1: iterations between residual checks */
    double theta;             /* multigrid correction step (step_mode 0) */
    int step_mode;            /* 0: p = e, fixed theta; 1: nonlinear PCG direction and step,
                                 restarted after a residual increase; 2: the same without
                                 restarts */
    double deflate_tau;       /* cluster threshold (x grid extent); <= 0 disables deflation */
    double restart_growth;    /* step_mode 1: restart when rel_k > restart_growth * rel_{k-1};
                                 <= 0 never restarts */
    double corr_scale;        /* factor on the prolongated coarse-grid correction */
    int aa_m;                 /* > 0: Anderson acceleration with this window replaces the
                                 conjugate-gradient step (the restart rule of step_mode 1
                                 clears its history) */
    double aa_reg;            /* Anderson: Tikhonov weight relative to the mean diagonal of
                                 the Gram matrix */
    int nu_coarse;            /* > 0: pre- and post-sweeps on every level l >= coarse_from
                                 (l = 0 the finest) instead of nu1 / nu2 */
    int coarse_from;          /* first level of nu_coarse, >= 1 */
} fldo_solve_opts;

typedef struct fldo_result {
    int status;
    int iterations;
    double rel;
    double rel_sweep;
    int history_len;
} fldo_result;

double fldo_limiter(int kind, double R, double larsen_n);
void fldo_limiter_array(int kind, double larsen_n, const double *R, double *F, long m);
int fldo_setup(fldo_params *p, const double *sigma_t, const double *albedo, const double *Q,
               double *sig_hat, double *sig_a);
void fldo_init_state(const fldo_params *p, double *phi, double *D);
void fldo_knudsen(const fldo_params *p, const double *phi, const double *sig_hat, double *R);
void fldo_limiter_pass(const fldo_params *p, const double *phi, const double *sig_hat, double *D);
double fldo_residual(const fldo_params *p, const double *phi, const double *D,
                     const double *sig_a, const double *j_src, double *r);
double fldo_nonlinear_residual(const fldo_params *p, const double *phi, const double *sig_hat,
                               const double *sig_a, const double *j_src, double *D_out,
                               double *r);
double fldo_alg1_iteration(const fldo_params *p, double omega, double *phi, double *D,
                           const double *sig_hat, const double *sig_a, const double *j_src);
int fldo_mg_levels(int nx, int ny, int nz, int max_coarsest, int *dims_out, int max_levels);
int fldo_cholesky_factor(int n, double *M);
void fldo_cholesky_solve(int n, const double *Lf, const double *rhs, double *x);
int fldo_linear_vcycle(int nx, int ny, int nz, double h, double d_ghost, int mirror,
                       const fldo_solve_opts *o, const double *D0, const double *sa0,
                       const double *b0, double *e0);
void fldo_level_residual(int nx, int ny, int nz, double h, double d_ghost, int mirror,
                         const double *D, const double *sa, const double *b, const double *e,
                         double *r);
int fldo_coarse_apply(int nx, int ny, int nz, double h, double d_ghost, int mirror,
                      const double *D0, const double *sa0, const double *x1, double *out1);
int fldo_clusters(int nx, int ny, int nz, double h, const double *sig_hat, double tau, int *label);
int fldo_solve(const fldo_params *p, const fldo_solve_opts *o, const double *sig_hat,
               const double *sig_a, const double *j_src, double *phi, double *D, double *hist,
               int cap, fldo_result *res);

/* Single-scatter source of a directional light along +z (see fldo.c). */
void fldo_light_bake(int nx, int ny, int nz, double h, double light, const double *sigma_t,
                     const double *albedo, double *q);

/* Primary ray-march of an orthographic camera along +z (see fldo.c). */
void fldo_render(int nx, int ny, int nz, double h, double background, const double *sigma_t,
                 const double *albedo, const double *src, const double *phi, double *image);

#endif
