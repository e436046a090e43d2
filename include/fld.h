/*
 * fld.h -- C ABI of the MI355X flux-limited diffusion (FLD) solver.
 *
 * The library solves the steady-state flux-limited diffusion equation of
 * Koerner et al., "Flux-Limited Diffusion for Multiple Scattering in
 * Participating Media" (CGF 33(2), 2014):
 *     div(D_F grad phi) = sigma_a phi - j,   D_F = F(R)/sigma_t,
 *     R = |grad phi| / (sigma_t phi)                  (Sec. 4, equations
 *     fld_radiative_diffusion_equation, fld_diffusion_coeff, fld_R),
 * discretised on a uniform voxel grid with the 7-point scheme of Sec. 5
 * (equation discretized_fld_diffusion_eqn, face coefficients
 * D_ps = (D_p + D_s)/2), central-difference gradients and the guarded
 * Knudsen number of Sec. 5 (grad_approx, knudsen_numerical), the extinction
 * floor sigma_eps = 1e-3/L and the initial state phi = eps*jbar*h,
 * D = eps*h of Algorithm 1.  CDA is the special case F = 1/3.
 *
 * Grids: every field holds nx*ny*nz float64 values, z fastest:
 *     index(i,j,k) = (i*ny + j)*nz + k          (a C-contiguous [nx][ny][nz]).
 * All nx*ny*nz voxels are unknowns.  The Dirichlet boundary is a ghost layer
 * one voxel outside them with fluence phi_b; its diffusion coefficient is
 * eps*h (the value Algorithm 1 gives boundary voxels, which it never
 * updates) or, with FLD_BOUNDARY_D_MIRROR, that of the voxel inside.
 *
 * Methods:
 *   FLD_METHOD_RBSOR  Algorithm 1 of the paper: red-black SOR with a per-voxel
 *                     D update ((i+j+k) even = red, red pass then black pass).
 *   FLD_METHOD_MG     Picard multigrid: D frozen from phi, FP64 residual, one
 *                     multigrid V-cycle per outer iteration as the
 *                     preconditioner of a nonlinear conjugate-gradient step
 *                     (the paper names nonlinear multigrid as future work,
 *                     Sec. 7).  FLD_PRECISION_MIXED runs the V-cycle in FP32
 *                     with FP32 accumulation and keeps the outer residual,
 *                     the outer update and the coarsest solve in FP64.
 *
 * Convergence: rel = ||r||_2 / ||j||_2 with r the residual of the
 * discretised equation (LHS - RHS, equation R_calc), D recomputed from phi
 * for every voxel; this equals the paper's normalised RMS residual
 * R-bar/j-bar taken over all unknowns.
 *
 * Errors: no call throws; every call returns an fld_status.  The text of the
 * last failure of a context is available from fld_last_error().  A context is
 * not thread-safe; different contexts are independent.  Device memory is
 * owned by the context and freed by fld_destroy().
 */
#ifndef FLD_H
#define FLD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fld_status {
    FLD_OK = 0,
    FLD_ERR_INVALID_ARGUMENT = 1, /* bad pointer, size, option or input value      */
    FLD_ERR_OUT_OF_MEMORY = 2,    /* device or host allocation failed               */
    FLD_ERR_DEVICE = 3,           /* a HIP runtime call failed                      */
    FLD_ERR_NOT_CONVERGED = 4,    /* max_iters reached; phi and report are written  */
    FLD_ERR_DIVERGED = 5,         /* residual became NaN/Inf; phi is written        */
    FLD_ERR_STATE = 6             /* call order violated (e.g. solve before medium) */
} fld_status;

/* Flux limiters of Sec. 4, Table 2 (and CDA). */
typedef enum fld_limiter {
    FLD_LIMITER_CDA = 0,     /* F = 1/3                                   */
    FLD_LIMITER_LP = 1,      /* Levermore-Pomraning (coth R - 1/R)/R      */
    FLD_LIMITER_SUM = 2,     /* 1/(3 + R)                                 */
    FLD_LIMITER_MAX = 3,     /* 1/max(3, R)                               */
    FLD_LIMITER_KERSHAW = 4, /* 2/(3 + sqrt(9 + 4R^2))                    */
    FLD_LIMITER_LARSEN = 5   /* (3^n + R^n)^(-1/n), n = larsen_n          */
} fld_limiter;

typedef enum fld_method { FLD_METHOD_RBSOR = 0, FLD_METHOD_MG = 1 } fld_method;
typedef enum fld_precision { FLD_PRECISION_FP64 = 0, FLD_PRECISION_MIXED = 1 } fld_precision;
typedef enum fld_boundary_d { FLD_BOUNDARY_D_PAPER = 0, FLD_BOUNDARY_D_MIRROR = 1 } fld_boundary_d;

typedef struct fld_options {
    size_t struct_size;   /* sizeof(fld_options); set by fld_default_options            */
    int limiter;          /* fld_limiter (default LP)                                    */
    double larsen_n;      /* Larsen-n exponent (default 2)                               */
    double eps;           /* guard / initialisation tolerance (default 1e-20)           */
    double sigma_eps;     /* extinction floor; <= 0 selects 1e-3/L, L = h*max(n) (default) */
    double phi_b;         /* ghost-layer fluence (default 0)                             */
    int boundary_d;       /* fld_boundary_d (default PAPER)                              */
    int method;           /* fld_method (default MG)                                     */
    int precision;        /* fld_precision (default FP64)                                */
    double omega;         /* Algorithm 1 SOR factor, 0 < omega < 2 (default 1)          */
    double omega_s;       /* multigrid smoother relaxation, 0 < omega_s < 2 (default 1)  */
    int nu1, nu2;         /* pre/post red-black sweeps per level (default 2, 2)          */
    int max_coarsest;     /* max cells of the coarsest level, <= 4096 (default 512)      */
    int max_iters;        /* Algorithm 1 iterations / outer MG iterations (default 10000) */
    double tol;           /* stop when rel <= tol (default 1e-6)                          */
    int check_every;      /* Algorithm 1: iterations between residual checks (default 1)  */
    int device;           /* HIP device ordinal (default 0)                              */
    void *stream;         /* hipStream_t for all work; NULL = the context's own stream   */
    int timing;           /* 1: bracket the hot kernels with HIP events (fld_report.kernel_*) */
    double deflate_tau;   /* multigrid: cluster-deflation threshold in units of the grid
                             extent L; voxels joined by faces whose classical coefficient
                             ((1/3)/sig_p + (1/3)/sig_s)/2 exceeds tau*L form clusters whose
                             constant mode is removed before each V-cycle; <= 0 disables
                             (default 1)                                                  */
    int graph;            /* multigrid: replay each outer iteration from a captured HIP graph
                             (two graphs, one per buffer parity; default 1).  With timing,
                             the events become event-record nodes of the graphs           */
    int task_cells0;      /* multigrid launch shape: cells per work-list task on the finest
                             level (power of two in [512, 65536], default 4096)            */
    int coarse_blocks;    /* multigrid launch shape: coarser levels use the largest power-of-
                             two task size in [256, 4096] that still gives this many tasks
                             per launch (64..65536, default 2048).  Neither shape changes
                             any result bit                                                */
    int colour_split;     /* mixed multigrid: store the finest-level FP32 fields red half /
                             black half, so a red-black half-sweep streams only the cells it
                             needs (used when nz % 8 == 0 and the grid coarsens; default 1).
                             Results are bit-identical to the natural order (0)            */
    double restart_growth;/* multigrid: the conjugate-gradient direction restarts (beta = 0)
                             after an outer iteration that raised ||r|| by more than this
                             factor; <= 0 never restarts (default 2)                       */
    double corr_scale;    /* multigrid: factor on the coarse-grid correction of the finest
                             level (piecewise-constant prolongation under-corrects; default 1) */
    double anisotropy_g;  /* phase-function anisotropy g in [0,1): the diffusion coefficient
                             and the Knudsen number use the reduced extinction
                             sigma_t (1 - albedo g) (Sec. 7); absorption is unchanged.
                             Batches need one channel per volume when g != 0 (default 0) */
    int deep_cells;       /* multigrid launch shape: coarse levels from the first one with at
                             most this many cells down to the coarsest run in one workgroup
                             per problem (two launches instead of several per level); 0
                             launches every level separately.  No result bit changes
                             (default 4096)                                                */
    double nested_tol;    /* multigrid grid sequencing: > 0 makes a solve from the paper's
                             initial state first solve the medium coarsened 2:1 (sigma_t and
                             Q averaged over the 8 children, albedo so that absorption is
                             averaged too; default schedule, at most 10000 iterations) to
                             this relative residual, and start from its fluence, constant
                             over each 2x2x2 block.  Needs
                             every axis even and anisotropy_g = 0; set up by fld_set_medium
                             (fld_batch_set_volume) in a second, coarse context (batch), 1/8
                             of the memory.  In a batch, a problem whose coarse solve
                             diverged starts from the paper's state.  0 disables (default)  */
    int aa_m;             /* multigrid outer step: 0 the preconditioned nonlinear conjugate-
                             gradient step (default); 1..16 Anderson acceleration of the
                             preconditioned Picard map x -> x + e(x) with this window (the
                             last aa_m pairs of differences of iterates and corrections,
                             least squares by regularised normal equations); the
                             restart_growth rule clears its history.  The coarse solve of
                             grid sequencing keeps the default step                        */
    double aa_reg;        /* Anderson: Tikhonov weight relative to the mean diagonal of the
                             Gram matrix of correction differences (default 1e-10)          */
    int fuse_lr;          /* multigrid: 1 forms D and the residual of the finest level in
                             one pass over LDS tiles when every grid has nz % 4 == 0 and
                             no direction update is pending (Anderson steps, and the first
                             iteration of a call); 0 (default) uses the separate limiter
                             and residual passes, which are faster with the LP limiter on
                             MI355X.  D and r are the same either way; only the grouping
                             of the partial sums of the residual norm differs               */
    int fuse_rb;          /* multigrid: 1 runs the finest level's smoothing sweeps in pairs
                             of single-pass red-black sweeps over LDS tiles, out of place
                             into a second correction buffer (20 instead of 28 bytes per
                             cell and sweep) when every grid has nz % 4 == 0; an odd
                             sweep left over uses the two half-sweeps.  0 (default): the
                             half-sweeps only.  The result is the same either way         */
    int debug_nan_iter;   /* failure injection (multigrid): k >= 1 writes NaN into voxel 0 of
                             every problem's phi after the residual of outer iteration k
                             is read, so the next residual is not finite and the solve
                             ends with FLD_ERR_DIVERGED at iteration k+1; 0 (default) off  */
    int nu_coarse;        /* multigrid: pre- and post-smoothing sweeps on every level from
                             coarse_from on (level 0 is the finest; the coarsest is solved,
                             not smoothed); 0 (default) keeps nu1 / nu2 there.  In [0,64].
                             The small levels cost little per sweep (their launches are
                             latency-bound), and a better coarse correction saves outer
                             iterations                                                    */
    int coarse_from;      /* first level that nu_coarse applies to, >= 1 (default 2)      */
    int nested_inherit;   /* grid sequencing: 1 gives the coarse solve this solve's schedule
                             (nu1, nu2, omega_s, corr_scale, restart_growth, aa_m, aa_reg,
                             and nu_coarse from level coarse_from - 1, at least 1: the same
                             level sizes); 0 (default) the default schedule               */
} fld_options;

typedef struct fld_report {
    size_t struct_size;   /* caller sets sizeof(fld_report)                               */
    int status;           /* fld_status of the solve                                      */
    int iterations;       /* Algorithm 1 iterations or outer MG iterations performed      */
    double rel;           /* final ||r||/||j||                                            */
    double rel_sweep;     /* Algorithm 1: last in-sweep R-bar/j-bar (NaN for MG)          */
    double *history;      /* caller-owned buffer for rel at every check (may be NULL)     */
    int history_cap;      /* its capacity                                                 */
    int history_len;      /* number of checks made (may exceed history_cap)               */
    double time_ms;       /* wall time of the solve (device-synchronised)                 */
    double voxel_updates; /* point updates applied (sweeps x cells, all levels)           */
    double bytes;         /* algorithmic HBM bytes of the timed kernels below             */
    /* With options.timing: per kernel class (0 finest-level smoother, 1 finest FP64
     * residual, 2 limiter pass, 3 conjugate-direction pass or, with aa_m > 0, the
     * Anderson update pass) the summed HIP-event time, the number of launches and
     * the algorithmic bytes those launches move. */
    double kernel_ms[4];
    double kernel_launches[4];
    double kernel_bytes[4];
    int nested_iterations;/* outer iterations of the coarse solve of grid sequencing (0 when
                             it did not run); included in time_ms and voxel_updates      */
} fld_report;

typedef struct fld_context fld_context;
typedef struct fld_batch fld_batch;

/* Fill *o with the defaults above.  Returns FLD_ERR_INVALID_ARGUMENT for NULL. */
fld_status fld_default_options(fld_options *o);

/* Create a solver for an nx*ny*nz grid with voxel edge h.  Allocates every
 * device buffer (including the multigrid hierarchy for FLD_METHOD_MG) on
 * o->device.  *out is owned by the caller until fld_destroy.
 * Errors: INVALID_ARGUMENT (NULL pointers, n < 1, h <= 0 or not finite, an
 * option out of range, MG on a grid whose coarsest level exceeds
 * max_coarsest cells); OUT_OF_MEMORY; DEVICE. */
fld_status fld_create(const fld_options *o, int nx, int ny, int nz, double h, fld_context **out);

/* Set the medium from host arrays of N values each (copied; the caller keeps
 * ownership): extinction sigma_t >= 0, albedo in [0,1], emission Q >= 0 (the
 * paper's j_p with the single-scatter source folded in, power per unit
 * volume).  Performs Algorithm 1's set-up (sigma <- max(sigma, sigma_eps),
 * RMS emission).  On a non-finite or out-of-range value returns
 * INVALID_ARGUMENT and names the first offending index in fld_last_error. */
fld_status fld_set_medium(fld_context *c, const double *sigma_t, const double *albedo,
                          const double *Q);

/* Same from device pointers (e.g. torch tensors), ordered on hip_stream (NULL
 * = the context's stream).  The library copies the data before returning, so
 * the caller may free the buffers once the call returns. */
fld_status fld_set_medium_device(fld_context *c, const double *d_sigma_t, const double *d_albedo,
                                 const double *d_Q, void *hip_stream);

/* Solve to o->tol.  phi_init (host, N values, may be NULL) is the start; NULL
 * starts from the paper's initial state, or, when resume != 0, from the
 * state the previous solve on this context left (iterations continue exactly
 * as if never stopped).  phi_out (host, N values) receives the fluence, also
 * on NOT_CONVERGED and DIVERGED.  rep may be NULL.
 * Errors: STATE before a medium is set; NOT_CONVERGED; DIVERGED; DEVICE. */
fld_status fld_solve(fld_context *c, const double *phi_init, double *phi_out, fld_report *rep);

/* Same with device pointers (may alias nothing else; d_phi_init may be NULL). */
fld_status fld_solve_device(fld_context *c, const double *d_phi_init, double *d_phi_out,
                            int resume, fld_report *rep);

/* Host variant of resume: continue from the context's current state. */
fld_status fld_solve_resume(fld_context *c, double *phi_out, fld_report *rep);

/* Nonlinear residual of phi (host, N values; NULL = the context's current
 * fluence): D recomputed from phi for every voxel, r = j - A(D) phi in FP64.
 * r_out (host, N values) may be NULL; *rel_out = ||r||_2/||j||_2. */
fld_status fld_residual(fld_context *c, const double *phi, double *r_out, double *rel_out);

/* Device-pointer variant of fld_residual (d_phi may be NULL, d_r_out may be NULL). */
fld_status fld_residual_device(fld_context *c, const double *d_phi, double *d_r_out,
                               double *rel_out);

/* Largest grid (cells) fld_residual_device_noalloc accepts: 128^3. */
#define FLD_NOALLOC_MAX_CELLS 2097152LL

/* fld_residual_device without any device allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results bit-identical to
 * fld_residual_device: d_phi (device, N values; NULL = the context's current
 * fluence) is read in place, d_r_out (device, N values) may be NULL, *rel_out
 * receives ||r||_2/||j||_2 (the call waits for the context's stream).  The
 * temporaries live in a fixed scratch area of 2 * FLD_NOALLOC_MAX_CELLS
 * doubles that the library holds on each GPU it runs on until the process
 * ends; calls that overlap in time on one GPU share it and race.  Errors:
 * INVALID_ARGUMENT for a NULL context or rel_out and for grids of more than
 * FLD_NOALLOC_MAX_CELLS cells; STATE before a medium is set; DEVICE. */
fld_status fld_residual_device_noalloc(fld_context *c, const double *d_phi, double *d_r_out,
                                       double *rel_out);

/* Free everything.  NULL is a no-op. */
void fld_destroy(fld_context *c);

/* Text of a status code (static storage). */
const char *fld_status_string(fld_status s);

/* Text of the last failure on c ("" if none; static "invalid context" for NULL). */
const char *fld_last_error(const fld_context *c);

/* Architecture name of HIP device `device` (for example "gfx950", without
 * feature suffixes) into buf[0..len-1], NUL-terminated.  Used to key tuned
 * launch options.  FLD_ERR_INVALID_ARGUMENT for a NULL buf, len < 2 or a bad
 * ordinal; FLD_ERR_DEVICE if the runtime query fails. */
fld_status fld_device_arch(int device, char *buf, int len);

/* Light baking: the single-scatter source of an external directional light,
 * q_ri = L_l sigma_s T, T the transmittance from the voxel towards the light
 * (the "deep shadow map" of Sec. 3; the paper bakes it by ray-marching,
 * Sec. 6).  The light of radiance `light` travels +z and enters every column
 * at its z = 0 face; in voxel k of a column
 *     T = exp(-h (sum_{k' < k} sigma_t + sigma_t(k)/2))
 * (midpoint of the voxel, raw sigma_t) and sigma_s = albedo * sigma_t.
 * d_sigma_t, d_albedo (per voxel) and d_q are device arrays of nx*ny*nz
 * float64 values, z fastest, owned by the caller; d_q must not alias the
 * inputs.  The work is enqueued on hip_stream (NULL: the null stream) and the
 * call returns without waiting.  FLD_ERR_INVALID_ARGUMENT for a NULL
 * pointer, a size < 1, h <= 0, a negative light or non-finite values of
 * either; FLD_ERR_DEVICE if the launch fails.  No context is needed. */
fld_status fld_light_bake(const double *d_sigma_t, const double *d_albedo, double light, int nx,
                          int ny, int nz, double h, double *d_q, void *hip_stream);

/* Primary ray-march of the image from the fluence (Sec. 3): the radiance
 * reaching the camera is the back-light attenuated by the whole ray plus,
 * for every sample, Delta x T(sample -> camera) Q, with the source in terms
 * of the diffusion solution 4 pi Q = q_ri + sigma_s phi + j.  Orthographic
 * camera on the +z side: one ray per (i, j) column travelling +z; the
 * sample of voxel k is attenuated by T = exp(-h (sigma_t(k)/2 +
 * sum_{k' > k} sigma_t)); `background` enters at z = 0 and is attenuated by
 * exp(-h sum_k sigma_t).  d_src holds q_ri + j (the emission given to the
 * solver), d_phi the fluence, sigma_s = albedo * sigma_t; all nx*ny*nz
 * float64, z fastest.  d_image: nx*ny float64, index i*ny + j.  Device
 * pointers owned by the caller; enqueued on hip_stream, no wait.  Errors as
 * for fld_light_bake (background must be finite and >= 0). */
fld_status fld_render(const double *d_sigma_t, const double *d_albedo, const double *d_src,
                      const double *d_phi, double background, int nx, int ny, int nz, double h,
                      double *d_image, void *hip_stream);

/* Batched solve: nvol volumes of sizes dims3[3v..3v+2] and edges h[v], each
 * with nchan colour channels that share the extinction field and have their
 * own albedo and emission (the per-channel albedo pattern of Sec. 6).  All
 * nvol*nchan solves advance together: every phase of an outer iteration is a
 * single launch over a work list covering all unconverged (volume, channel)
 * pairs.  Method is always MG; o->precision applies. */
fld_status fld_batch_create(const fld_options *o, int nvol, const int *dims3, const double *h,
                            int nchan, fld_batch **out);

/* Medium of volume v: sigma_t (N_v values), albedo[c] and Q[c] for each
 * channel c (N_v values each).  Host pointers, copied. */
fld_status fld_batch_set_volume(fld_batch *b, int v, const double *sigma_t,
                                const double *const *albedo, const double *const *Q);

/* Solve all pairs to o->tol.  phi_out[v*nchan + c] (host, N_v values, may be
 * NULL to skip the copy) receives each fluence.  rep (may be NULL) reports
 * the worst pair; per-pair iteration counts go to iters_out (may be NULL,
 * nvol*nchan ints).  Returns NOT_CONVERGED if any pair did not converge. */
fld_status fld_batch_solve(fld_batch *b, double *const *phi_out, int *iters_out,
                           fld_report *rep);

void fld_batch_destroy(fld_batch *b);
const char *fld_batch_last_error(const fld_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* FLD_H */
