/*
 * fldo.c -- plain FP64 CPU oracle for the flux-limited diffusion (FLD) solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP implementation.  It is deliberately slow and simple: scalar loops in
 * the order the paper writes the operations, compiled with -ffp-contract=off
 * so every multiply and add rounds on its own.
 *
 * Paper: Koerner, Portsmouth, Sadlo, Ertl, Eberhardt, "Flux-Limited Diffusion
 * for Multiple Scattering in Participating Media", CGF 33(2), 2014.
 *
 * Layout: every field holds nx*ny*nz unknowns, z fastest,
 *   idx(i,j,k) = (i*ny + j)*nz + k.
 * All nx*ny*nz voxels are unknowns; the Dirichlet boundary lives in a virtual
 * ghost layer one voxel outside them (the paper fixes the outermost voxel layer
 * of its grid, Sec. 5 "Numerical Method", boundary paragraph).  Ghost fluence
 * is phi_b (or a caller-supplied padded array), ghost diffusion coefficient is
 * eps*h (the paper's initial D, never updated on the boundary) or, in mirror
 * mode, the coefficient of the voxel inside.
 *
 * What pins each part to something other than itself (tests/test_oracle_*.py):
 *   limiters (fldo_limiter*)       Table 2 closed forms with mpmath-derived
 *                                  constants; R -> 0 and R -> inf limits; F <= 1/R;
 *                                  the small-R branch of LP; CDA constant
 *   set-up, Knudsen number, limiter exact gradients of linear fields; the guard
 *   pass (fldo_setup, fldo_knudsen, branches worked by hand; |E| <= phi after a
 *   fldo_limiter_pass)             pass (the flux-limiting bound of Sec. 4)
 *   residual (fldo_residual,       an independent scipy assembly of the same
 *   fldo_nonlinear_residual)       system; symmetric M-matrix; exact discrete power
 *                                  balance; bit-exact homogeneity in Q; axis
 *                                  permutation symmetry
 *   Algorithm 1 (fldo_alg1_*,      CDA equals a sparse direct solve; FLD equals a
 *   solve_alg1)                    brute-force Picard fixed point on <= 8^3; the
 *                                  CDA point source follows the closed-form
 *                                  Green's function, with second-order refinement;
 *                                  the SOR rate equals Young's formula from the
 *                                  Jacobi spectral radius
 *   multigrid (fldo_mg_levels,     Galerkin identity A_1 = P^T A_0 P / 8 in numpy;
 *   levels, smoother, transfers,   a single-level V-cycle is exact; Cholesky vs
 *   Cholesky, solve_mg)            numpy; the multigrid solve reaches the sparse
 *                                  direct / brute-force fixed points and the one of
 *                                  Algorithm 1; power balance at convergence
 *   clusters, deflation, restarts  scipy connected components; deflation and
 *                                  direction restarts keep the fixed point
 *   reduced extinction (aniso_g)   the CDA Green's function with D = 1/(3 sigma_t')
 *   light baking, render           closed forms of a homogeneous column; vacuum;
 *                                  linearity; product form of the transmittance
 */
#include <math.h>

/* Loops over fewer cells than this run on one thread: every loop writes each
 * cell independently (no reductions), so the thread count changes no result,
 * only the overhead of starting threads for the small grids of the tests and
 * the coarse levels. */
#define FLDO_PARALLEL(cells) ((cells) >= 65536L)
#include <stdlib.h>
#include <string.h>

#include "fldo.h"

static inline long idx3(int ny, int nz, int i, int j, int k)
{
    return ((long)i * ny + j) * nz + k;
}

static inline int inside(int nx, int ny, int nz, int i, int j, int k)
{
    return i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
}

/* ------------------------------------------------------------------------ */
/* Flux limiters, Sec. 4 Table 2 (and CDA, F = 1/3, Sec. 4 below the FLD     */
/* diffusion-coefficient equation).  Pinned against mpmath closed forms.     */
/* ------------------------------------------------------------------------ */

/* Levermore-Pomraning F(R) = (coth R - 1/R)/R.  Below R = 2 the difference
 * coth R - 1/R cancels, so there F comes from Lambert's continued fraction
 *   coth R - 1/R = R / (3 + R^2/(5 + R^2/(7 + ...))),
 * i.e. F = 1/(3 + R^2/(5 + R^2/(7 + ...))), truncated at the partial
 * denominator 25 (tail error below 1e-17 relative for R < 2).  Above it,
 * coth R = 1 + 2/expm1(2R). */
static double limiter_lp(double R)
{
    if (R < 2.0) {
        double x = R * R;
        double t = 25.0;
        for (int m = 11; m >= 1; --m)
            t = (double)(2 * m + 1) + x / t;
        return 1.0 / t;
    }
    double coth = 1.0 + 2.0 / expm1(2.0 * R);
    return (coth - 1.0 / R) / R;
}

static double limiter_larsen(double R, double n)
{
    /* (3^n + R^n)^(-1/n), written so R^n cannot overflow for large R. */
    if (R <= 3.0)
        return pow(pow(3.0, n) + pow(R, n), -1.0 / n);
    return (1.0 / R) * pow(1.0 + pow(3.0 / R, n), -1.0 / n);
}

double fldo_limiter(int kind, double R, double larsen_n)
{
    switch (kind) {
    case FLDO_LIMITER_CDA:
        return 1.0 / 3.0;
    case FLDO_LIMITER_LP:
        return limiter_lp(R);
    case FLDO_LIMITER_SUM:
        return 1.0 / (3.0 + R);
    case FLDO_LIMITER_MAX:
        return 1.0 / fmax(3.0, R);
    case FLDO_LIMITER_KERSHAW:
        return 2.0 / (3.0 + sqrt(9.0 + 4.0 * R * R));
    case FLDO_LIMITER_LARSEN:
        return limiter_larsen(R, larsen_n);
    default:
        return NAN;
    }
}

void fldo_limiter_array(int kind, double larsen_n, const double *R, double *F, long m)
{
    for (long q = 0; q < m; ++q)
        F[q] = fldo_limiter(kind, R[q], larsen_n);
}

/* ------------------------------------------------------------------------ */
/* Ghost-aware field access                                                 */
/* ------------------------------------------------------------------------ */

/* Fluence at (i,j,k); outside the unknowns this is the Dirichlet ghost value. */
static double phi_at(const fldo_params *p, const double *phi, int i, int j, int k)
{
    if (inside(p->nx, p->ny, p->nz, i, j, k))
        return phi[idx3(p->ny, p->nz, i, j, k)];
    if (p->ghost_phi)
        return p->ghost_phi[idx3(p->ny + 2, p->nz + 2, i + 1, j + 1, k + 1)];
    return p->phi_b;
}

/* Diffusion coefficient of neighbour (i,j,k) of voxel c. */
static double d_at(int nx, int ny, int nz, double d_ghost, int mirror, const double *D,
                   long c, int i, int j, int k)
{
    if (inside(nx, ny, nz, i, j, k))
        return D[idx3(ny, nz, i, j, k)];
    return mirror ? D[c] : d_ghost;
}

/* The six face neighbours in the fixed order x-, x+, y-, y+, z-, z+.  The
 * paper's stencil s(p) (Sec. 5, discretised FLD equation) names the six face
 * neighbours of p. */
static const int NB[6][3] = {
    {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};

/* ------------------------------------------------------------------------ */
/* Algorithm 1 set-up: extinction floor, absorption, RMS emission            */
/* ------------------------------------------------------------------------ */

int fldo_setup(fldo_params *p, const double *sigma_t, const double *albedo, const double *Q,
               double *sig_hat, double *sig_a)
{
    long n = (long)p->nx * p->ny * p->nz;
    int nmax = p->nx;
    if (p->ny > nmax) nmax = p->ny;
    if (p->nz > nmax) nmax = p->nz;
    double L = p->h * nmax;                      /* grid extent */
    if (!(p->sigma_eps > 0.0))
        p->sigma_eps = 1.0e-3 / L;               /* Sec. 5: sigma_eps = 1e-3/L */

    double sum_j2 = 0.0;
    for (long c = 0; c < n; ++c) {
        /* Alg. 1 set-up: sigma <- max(sigma, sigma_eps); the clamped value is
         * the sigma of the whole method, absorption term included.  With a
         * phase-function anisotropy g the diffusion coefficient and the
         * Knudsen number use the reduced extinction sigma_t (1 - albedo g)
         * (Sec. 7); the absorption (1 - albedo) sigma_t is not reduced. */
        sig_hat[c] = fmax(sigma_t[c] * (1.0 - albedo[c] * p->aniso_g), p->sigma_eps);
        sig_a[c] = (1.0 - albedo[c]) * fmax(sigma_t[c], p->sigma_eps);
        sum_j2 += Q[c] * Q[c];
    }
    p->jnorm = sqrt(sum_j2);
    p->jbar = sqrt(sum_j2 / (double)n);          /* RMS emission */
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Knudsen number and diffusion-coefficient update, Sec. 5 equations        */
/* grad_approx, knudsen_numerical, D_update.                                 */
/* ------------------------------------------------------------------------ */

/* Central-difference gradient magnitude at (i,j,k). */
static double grad_norm_at(const fldo_params *p, const double *phi, int i, int j, int k)
{
    double dx = phi_at(p, phi, i + 1, j, k) - phi_at(p, phi, i - 1, j, k);
    double dy = phi_at(p, phi, i, j + 1, k) - phi_at(p, phi, i, j - 1, k);
    double dz = phi_at(p, phi, i, j, k + 1) - phi_at(p, phi, i, j, k - 1);
    return sqrt(dx * dx + dy * dy + dz * dz) / (2.0 * p->h);
}

/* Guarded Knudsen number R_p = max(|grad phi|, eps*jbar) / max(sigma*phi, eps*jbar). */
static double knudsen_at(const fldo_params *p, const double *phi, const double *sig_hat,
                         int i, int j, int k)
{
    long c = idx3(p->ny, p->nz, i, j, k);
    double floor_ = p->eps * p->jbar;
    double num = fmax(grad_norm_at(p, phi, i, j, k), floor_);
    double den = fmax(sig_hat[c] * phi[c], floor_);
    return num / den;
}

/* D_p = F(R_p) / max(sigma_p, sigma_eps); sig_hat is already clamped. */
static double d_update_at(const fldo_params *p, const double *phi, const double *sig_hat,
                          int i, int j, int k)
{
    long c = idx3(p->ny, p->nz, i, j, k);
    double R = knudsen_at(p, phi, sig_hat, i, j, k);
    return fldo_limiter(p->limiter, R, p->larsen_n) / sig_hat[c];
}

void fldo_knudsen(const fldo_params *p, const double *phi, const double *sig_hat, double *R)
{
#pragma omp parallel for schedule(static) if (FLDO_PARALLEL((long)p->nx * p->ny * p->nz))
    for (int i = 0; i < p->nx; ++i)
        for (int j = 0; j < p->ny; ++j)
            for (int k = 0; k < p->nz; ++k)
                R[idx3(p->ny, p->nz, i, j, k)] = knudsen_at(p, phi, sig_hat, i, j, k);
}

/* Limiter pass: every D_p from the same fluence field. */
void fldo_limiter_pass(const fldo_params *p, const double *phi, const double *sig_hat, double *D)
{
#pragma omp parallel for schedule(static) if (FLDO_PARALLEL((long)p->nx * p->ny * p->nz))
    for (int i = 0; i < p->nx; ++i)
        for (int j = 0; j < p->ny; ++j)
            for (int k = 0; k < p->nz; ++k)
                D[idx3(p->ny, p->nz, i, j, k)] = d_update_at(p, phi, sig_hat, i, j, k);
}

/* ------------------------------------------------------------------------ */
/* Discretised FLD equation, Sec. 5 (discretized_fld_diffusion_eqn,          */
/* phi_update, R_calc).  numerator = j h^2 + sum_s D_ps phi_s,              */
/* denominator = (1-alpha) sigma h^2 + sum_s D_ps, D_ps = (D_p + D_s)/2.    */
/* ------------------------------------------------------------------------ */

static void num_den_at(const fldo_params *p, const double *phi, const double *D,
                       const double *sig_a, const double *j_src, int i, int j, int k,
                       double *num, double *den)
{
    long c = idx3(p->ny, p->nz, i, j, k);
    double h2 = p->h * p->h;
    double d_ghost = p->eps * p->h;
    double n_ = j_src[c] * h2;
    double d_ = sig_a[c] * h2;
    for (int s = 0; s < 6; ++s) {
        int a = i + NB[s][0], b = j + NB[s][1], e = k + NB[s][2];
        double Ds = d_at(p->nx, p->ny, p->nz, d_ghost, p->mirror_d, D, c, a, b, e);
        double Dps = 0.5 * (D[c] + Ds);
        n_ = n_ + Dps * phi_at(p, phi, a, b, e);
        d_ = d_ + Dps;
    }
    *num = n_;
    *den = d_;
}

/* True residual R_p = LHS - RHS of the discretised equation, for a given D
 * field.  Returns ||r||_2 (plain sequential sum). r may be NULL. */
double fldo_residual(const fldo_params *p, const double *phi, const double *D,
                     const double *sig_a, const double *j_src, double *r)
{
    long n = (long)p->nx * p->ny * p->nz;
    double h2 = p->h * p->h;
    double *rr = r ? r : (double *)malloc(sizeof(double) * n);
#pragma omp parallel for schedule(static) if (FLDO_PARALLEL((long)p->nx * p->ny * p->nz))
    for (int i = 0; i < p->nx; ++i)
        for (int j = 0; j < p->ny; ++j)
            for (int k = 0; k < p->nz; ++k) {
                double num, den;
                long c = idx3(p->ny, p->nz, i, j, k);
                num_den_at(p, phi, D, sig_a, j_src, i, j, k, &num, &den);
                rr[c] = (num - phi[c] * den) / h2;
            }
    double s = 0.0;
    for (long c = 0; c < n; ++c)
        s += rr[c] * rr[c];
    if (!r) free(rr);
    return sqrt(s);
}

/* Nonlinear residual of a fluence field: D recomputed from phi for every
 * voxel, then the residual.  Returns ||r||_2. */
double fldo_nonlinear_residual(const fldo_params *p, const double *phi, const double *sig_hat,
                               const double *sig_a, const double *j_src, double *D_out, double *r)
{
    long n = (long)p->nx * p->ny * p->nz;
    double *D = D_out ? D_out : (double *)malloc(sizeof(double) * n);
    fldo_limiter_pass(p, phi, sig_hat, D);
    double nr = fldo_residual(p, phi, D, sig_a, j_src, r);
    if (!D_out) free(D);
    return nr;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1: one red pass then one black pass.  Colour of (i,j,k) is     */
/* (i+j+k) mod 2 on 0-based unknown indices; red = even.                     */
/* ------------------------------------------------------------------------ */

/* Update every voxel of one colour.  Each voxel: Knudsen number from the
 * current fluence, new D_p, face coefficients with the neighbours' stored D,
 * phi' = numerator/denominator, residual with the pre-update phi_p, then the
 * SOR blend.  Voxels of one colour only read the other colour, so the visiting
 * order inside a colour does not change the result.  Rsq receives R_p^2. */
static void alg1_pass(const fldo_params *p, double omega, int colour, double *phi, double *D,
                      const double *sig_hat, const double *sig_a, const double *j_src,
                      double *Rsq)
{
    double h2 = p->h * p->h;
#pragma omp parallel for schedule(static) if (FLDO_PARALLEL((long)p->nx * p->ny * p->nz))
    for (int i = 0; i < p->nx; ++i)
        for (int j = 0; j < p->ny; ++j)
            for (int k = 0; k < p->nz; ++k) {
                if (((i + j + k) & 1) != colour)
                    continue;
                long c = idx3(p->ny, p->nz, i, j, k);
                D[c] = d_update_at(p, phi, sig_hat, i, j, k);
                double num, den;
                num_den_at(p, phi, D, sig_a, j_src, i, j, k, &num, &den);
                double Rp = (num - phi[c] * den) / h2;
                double phi_prime = num / den;
                phi[c] = omega * phi_prime + (1.0 - omega) * phi[c];
                Rsq[c] = Rp * Rp;
            }
}

/* One iteration (red + black).  Returns the sum of R_p^2 over all unknowns of
 * both passes (the paper's in-sweep monitor squared times N). */
double fldo_alg1_iteration(const fldo_params *p, double omega, double *phi, double *D,
                           const double *sig_hat, const double *sig_a, const double *j_src)
{
    long n = (long)p->nx * p->ny * p->nz;
    double *Rsq = (double *)malloc(sizeof(double) * n);
    alg1_pass(p, omega, 0, phi, D, sig_hat, sig_a, j_src, Rsq);
    alg1_pass(p, omega, 1, phi, D, sig_hat, sig_a, j_src, Rsq);
    double s = 0.0;
    for (long c = 0; c < n; ++c)
        s += Rsq[c];
    free(Rsq);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Multigrid for the correction equation.  The paper names nonlinear        */
/* multigrid only as future work (Sec. 7); every detail below is this       */
/* project's own specification:                                             */
/*  - levels: 2:1 cell-centred coarsening on all axes together while every  */
/*    axis is even and half of it is still >= 4; the coarsest level may     */
/*    hold at most max_coarsest cells;                                      */
/*  - finest operator: the discretised equation with D frozen (zero ghost   */
/*    correction);                                                          */
/*  - coarse operators: Galerkin products A_{l+1} = P^T A_l P / 8 for the   */
/*    piecewise-constant prolongation P (each coarse value copied to its 8  */
/*    children) and the 8-child mean restriction R = P^T / 8.  These stay   */
/*    7-point: a coarse face coefficient is half the sum of the four fine   */
/*    face coefficients lying on that face, and the coarse absorption is    */
/*    the 8-child mean;                                                     */
/*  - red-black Gauss-Seidel smoothing: red then black before the coarse    */
/*    correction, black then red after it (a symmetric cycle);              */
/*  - dense Cholesky on the coarsest level.                                 */
/* ------------------------------------------------------------------------ */

int fldo_mg_levels(int nx, int ny, int nz, int max_coarsest, int *dims_out, int max_levels)
{
    int L = 0;
    int a = nx, b = ny, c = nz;
    for (;;) {
        if (L < max_levels) {
            dims_out[3 * L + 0] = a;
            dims_out[3 * L + 1] = b;
            dims_out[3 * L + 2] = c;
        }
        ++L;
        if ((a % 2) || (b % 2) || (c % 2) || a / 2 < 4 || b / 2 < 4 || c / 2 < 4)
            break;
        a /= 2;
        b /= 2;
        c /= 2;
    }
    if ((long)a * b * c > max_coarsest)
        return -L;
    return L;
}

/* One level of the hierarchy: A e = b with zero ghost values for e.  The
 * finest level keeps cell coefficients D (its faces follow the discretised
 * equation); coarse levels store face coefficients f[axis] on an
 * (nx+1)(ny+1)(nz+1) array, f[axis](i,j,k) being the face below cell
 * (i,j,k) along that axis. */
typedef struct {
    int nx, ny, nz;
    double h;
    const double *D;
    double *f[3];
    double *sa, *b, *e, *r;
} mg_level;

static long face_idx(const mg_level *L, int i, int j, int k)
{
    return ((long)i * (L->ny + 1) + j) * (L->nz + 1) + k;
}

/* Coefficient of the face below cell (i,j,k) along axis ax, i.e. between
 * that cell and its neighbour one index lower along ax; either cell may be
 * a ghost. */
static double face(const mg_level *L, double d_ghost, int mirror, int ax, int i, int j, int k)
{
    if (!L->D)
        return L->f[ax][face_idx(L, i, j, k)];
    int lo[3] = {i, j, k};
    lo[ax] -= 1;
    int hi_in = inside(L->nx, L->ny, L->nz, i, j, k);
    int lo_in = inside(L->nx, L->ny, L->nz, lo[0], lo[1], lo[2]);
    if (hi_in && lo_in)
        return 0.5 * (L->D[idx3(L->ny, L->nz, i, j, k)] + L->D[idx3(L->ny, L->nz, lo[0], lo[1], lo[2])]);
    double Din = hi_in ? L->D[idx3(L->ny, L->nz, i, j, k)]
                       : L->D[idx3(L->ny, L->nz, lo[0], lo[1], lo[2])];
    return 0.5 * (Din + (mirror ? Din : d_ghost));
}

/* num = b h^2 + sum_s F_s e_s, den = sa h^2 + sum_s F_s, neighbours in the
 * order x-, x+, y-, y+, z-, z+ (ghost e = 0). */
static void level_num_den(const mg_level *L, double d_ghost, int mirror, const double *b,
                          const double *e, int i, int j, int k, double *num, double *den)
{
    long c = idx3(L->ny, L->nz, i, j, k);
    double h2 = L->h * L->h;
    double n_ = (b ? b[c] : 0.0) * h2;
    double d_ = L->sa[c] * h2;
    for (int s = 0; s < 6; ++s) {
        int ax = NB[s][0] ? 0 : (NB[s][1] ? 1 : 2);
        int up = NB[s][0] + NB[s][1] + NB[s][2] > 0;
        int a = i + NB[s][0], bb = j + NB[s][1], q = k + NB[s][2];
        double F = up ? face(L, d_ghost, mirror, ax, a, bb, q) : face(L, d_ghost, mirror, ax, i, j, k);
        double es = inside(L->nx, L->ny, L->nz, a, bb, q) ? e[idx3(L->ny, L->nz, a, bb, q)] : 0.0;
        n_ = n_ + F * es;
        d_ = d_ + F;
    }
    *num = n_;
    *den = d_;
}

static void level_smooth_colour(mg_level *L, double d_ghost, int mirror, int colour,
                                double omega_s)
{
#pragma omp parallel for schedule(static) if (FLDO_PARALLEL((long)L->nx * L->ny * L->nz))
    for (int i = 0; i < L->nx; ++i)
        for (int j = 0; j < L->ny; ++j)
            for (int k = 0; k < L->nz; ++k) {
                if (((i + j + k) & 1) != colour)
                    continue;
                long c = idx3(L->ny, L->nz, i, j, k);
                double num, den;
                level_num_den(L, d_ghost, mirror, L->b, L->e, i, j, k, &num, &den);
                L->e[c] = omega_s * (num / den) + (1.0 - omega_s) * L->e[c];
            }
}

/* r = b - A e. */
static void level_residual(const mg_level *L, double d_ghost, int mirror, double *r)
{
    double h2 = L->h * L->h;
#pragma omp parallel for schedule(static) if (FLDO_PARALLEL((long)L->nx * L->ny * L->nz))
    for (int i = 0; i < L->nx; ++i)
        for (int j = 0; j < L->ny; ++j)
            for (int k = 0; k < L->nz; ++k) {
                long c = idx3(L->ny, L->nz, i, j, k);
                double num, den;
                level_num_den(L, d_ghost, mirror, L->b, L->e, i, j, k, &num, &den);
                r[c] = (num - L->e[c] * den) / h2;
            }
}

/* out = A x (same formula with b = 0, sign flipped). */
static void level_apply(const mg_level *L, double d_ghost, int mirror, const double *x, double *out)
{
    double h2 = L->h * L->h;
#pragma omp parallel for schedule(static) if (FLDO_PARALLEL((long)L->nx * L->ny * L->nz))
    for (int i = 0; i < L->nx; ++i)
        for (int j = 0; j < L->ny; ++j)
            for (int k = 0; k < L->nz; ++k) {
                long c = idx3(L->ny, L->nz, i, j, k);
                double num, den;
                level_num_den(L, d_ghost, mirror, NULL, x, i, j, k, &num, &den);
                out[c] = (x[c] * den - num) / h2;
            }
}

/* Mean over the 8 children, children visited with x slowest, z fastest. */
static void mean8(int nxc, int nyc, int nzc, int nyf, int nzf, const double *fine, double *coarse)
{
#pragma omp parallel for schedule(static) if (FLDO_PARALLEL((long)nxc * nyc * nzc))
    for (int I = 0; I < nxc; ++I)
        for (int J = 0; J < nyc; ++J)
            for (int K = 0; K < nzc; ++K) {
                double s = 0.0;
                for (int di = 0; di < 2; ++di)
                    for (int dj = 0; dj < 2; ++dj)
                        for (int dk = 0; dk < 2; ++dk)
                            s = s + fine[idx3(nyf, nzf, 2 * I + di, 2 * J + dj, 2 * K + dk)];
                coarse[idx3(nyc, nzc, I, J, K)] = 0.125 * s;
            }
}

/* Galerkin face coefficients of level C from level F: half the sum of the
 * four fine faces on each coarse face (the two in-face indices visited in
 * lexicographic order). */
static void galerkin_faces(const mg_level *F, mg_level *C, double d_ghost, int mirror)
{
    int nc[3] = {C->nx, C->ny, C->nz};
    for (int ax = 0; ax < 3; ++ax) {
        int ext[3] = {nc[0], nc[1], nc[2]};
        ext[ax] += 1;
        for (int I = 0; I < ext[0]; ++I)
            for (int J = 0; J < ext[1]; ++J)
                for (int K = 0; K < ext[2]; ++K) {
                    double s = 0.0;
                    for (int u = 0; u < 2; ++u)
                        for (int v = 0; v < 2; ++v) {
                            int d[3] = {0, 0, 0};
                            int q = 0;
                            for (int a = 0; a < 3; ++a)
                                if (a != ax)
                                    d[a] = (q++ == 0) ? u : v;
                            s = s + face(F, d_ghost, mirror, ax, 2 * I + d[0], 2 * J + d[1],
                                         2 * K + d[2]);
                        }
                    C->f[ax][face_idx(C, I, J, K)] = 0.5 * s;
                }
    }
}

/* e_fine += P e_coarse: every fine cell receives its parent's value. */
static void prolong_add(const mg_level *C, mg_level *F, double scale)
{
#pragma omp parallel for schedule(static) if (FLDO_PARALLEL((long)F->nx * F->ny * F->nz))
    for (int i = 0; i < F->nx; ++i)
        for (int j = 0; j < F->ny; ++j)
            for (int k = 0; k < F->nz; ++k) {
                long c = idx3(F->ny, F->nz, i, j, k);
                F->e[c] = F->e[c] + scale * C->e[idx3(C->ny, C->nz, i / 2, j / 2, k / 2)];
            }
}

/* Dense Cholesky M = L L^T (lower triangle of M overwritten by L). */
int fldo_cholesky_factor(int n, double *M)
{
    for (int c = 0; c < n; ++c) {
        double d = M[(long)c * n + c];
        for (int q = 0; q < c; ++q)
            d = d - M[(long)c * n + q] * M[(long)c * n + q];
        if (!(d > 0.0))
            return -1;
        double lcc = sqrt(d);
        M[(long)c * n + c] = lcc;
        for (int r = c + 1; r < n; ++r) {
            double s = M[(long)r * n + c];
            for (int q = 0; q < c; ++q)
                s = s - M[(long)r * n + q] * M[(long)c * n + q];
            M[(long)r * n + c] = s / lcc;
        }
    }
    return 0;
}

void fldo_cholesky_solve(int n, const double *Lf, const double *rhs, double *x)
{
    for (int r = 0; r < n; ++r) {               /* L y = rhs */
        double s = rhs[r];
        for (int q = 0; q < r; ++q)
            s = s - Lf[(long)r * n + q] * x[q];
        x[r] = s / Lf[(long)r * n + r];
    }
    for (int r = n - 1; r >= 0; --r) {          /* L^T x = y */
        double s = x[r];
        for (int q = r + 1; q < n; ++q)
            s = s - Lf[(long)q * n + r] * x[q];
        x[r] = s / Lf[(long)r * n + r];
    }
}

/* Dense M = h^2 A of one level (natural z-fastest order). */
static void assemble_level(const mg_level *L, double d_ghost, int mirror, double *M)
{
    int n = L->nx * L->ny * L->nz;
    double h2 = L->h * L->h;
    memset(M, 0, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < L->nx; ++i)
        for (int j = 0; j < L->ny; ++j)
            for (int k = 0; k < L->nz; ++k) {
                long c = idx3(L->ny, L->nz, i, j, k);
                double diag = L->sa[c] * h2;
                for (int s = 0; s < 6; ++s) {
                    int ax = NB[s][0] ? 0 : (NB[s][1] ? 1 : 2);
                    int up = NB[s][0] + NB[s][1] + NB[s][2] > 0;
                    int a = i + NB[s][0], b = j + NB[s][1], q = k + NB[s][2];
                    double F = up ? face(L, d_ghost, mirror, ax, a, b, q)
                                  : face(L, d_ghost, mirror, ax, i, j, k);
                    diag = diag + F;
                    if (inside(L->nx, L->ny, L->nz, a, b, q))
                        M[c * n + idx3(L->ny, L->nz, a, b, q)] = -F;
                }
                M[c * n + c] = diag;
            }
}

/* V(nu1, nu2) cycle on levels[l..nlev-1] (nu_coarse sweeps before and after
 * on the levels from coarse_from on, when set).  Every level starts from a
 * zero correction, except the first when e_start is given: its smoothing then
 * starts from e_start (the cluster deflation step). */
static void vcycle(mg_level *lv, int l, int nlev, const fldo_solve_opts *o, double d_ghost,
                   int mirror, const double *chol, const double *e_start)
{
    mg_level *L = &lv[l];
    long n = (long)L->nx * L->ny * L->nz;
    if (l == nlev - 1) {
        double h2 = L->h * L->h;
        double *rhs = (double *)malloc(sizeof(double) * n);
        for (long c = 0; c < n; ++c)
            rhs[c] = L->b[c] * h2;
        fldo_cholesky_solve((int)n, chol, rhs, L->e);
        free(rhs);
        return;
    }
    if (e_start)
        memcpy(L->e, e_start, sizeof(double) * n);
    else
        memset(L->e, 0, sizeof(double) * n);
    const int coarse = l >= 1 && o->nu_coarse > 0 && l >= o->coarse_from;
    const int pre = coarse ? o->nu_coarse : o->nu1, post = coarse ? o->nu_coarse : o->nu2;
    for (int s = 0; s < pre; ++s) {
        level_smooth_colour(L, d_ghost, mirror, 0, o->omega_s);
        level_smooth_colour(L, d_ghost, mirror, 1, o->omega_s);
    }
    level_residual(L, d_ghost, mirror, L->r);
    mean8(lv[l + 1].nx, lv[l + 1].ny, lv[l + 1].nz, L->ny, L->nz, L->r, lv[l + 1].b);
    vcycle(lv, l + 1, nlev, o, d_ghost, mirror, chol, NULL);
    prolong_add(&lv[l + 1], L, l == 0 ? o->corr_scale : 1.0);
    for (int s = 0; s < post; ++s) {
        level_smooth_colour(L, d_ghost, mirror, 1, o->omega_s);
        level_smooth_colour(L, d_ghost, mirror, 0, o->omega_s);
    }
}

typedef struct {
    int nlev;
    mg_level lv[FLDO_MAX_LEVELS];
    double *chol;
} mg_hier;

static int hier_alloc(mg_hier *H, const int *dims, int nlev, double h)
{
    memset(H, 0, sizeof(*H));
    H->nlev = nlev;
    for (int l = 0; l < nlev; ++l) {
        mg_level *L = &H->lv[l];
        L->nx = dims[3 * l];
        L->ny = dims[3 * l + 1];
        L->nz = dims[3 * l + 2];
        L->h = h * (double)(1L << l);
        long n = (long)L->nx * L->ny * L->nz;
        L->e = (double *)calloc(n, sizeof(double));
        L->sa = (double *)calloc(n, sizeof(double));
        L->b = (double *)calloc(n, sizeof(double));
        L->r = (double *)calloc(n, sizeof(double));
        if (!L->e || !L->sa || !L->b || !L->r)
            return -1;
        if (l > 0) {
            long nf = (long)(L->nx + 1) * (L->ny + 1) * (L->nz + 1);
            for (int a = 0; a < 3; ++a) {
                L->f[a] = (double *)calloc(nf, sizeof(double));
                if (!L->f[a])
                    return -1;
            }
        }
    }
    long nc = (long)H->lv[nlev - 1].nx * H->lv[nlev - 1].ny * H->lv[nlev - 1].nz;
    H->chol = (double *)malloc(sizeof(double) * nc * nc);
    return H->chol ? 0 : -1;
}

static void hier_free(mg_hier *H)
{
    for (int l = 0; l < H->nlev; ++l) {
        free(H->lv[l].e);
        free(H->lv[l].sa);
        free(H->lv[l].b);
        free(H->lv[l].r);
        for (int a = 0; a < 3; ++a)
            free(H->lv[l].f[a]);
    }
    free(H->chol);
}

/* Coarse operators from the finest level's D and sa (sa only when asked),
 * then the Cholesky factor of the coarsest operator. */
static int hier_coarsen(mg_hier *H, int coarsen_sa, double d_ghost, int mirror)
{
    for (int l = 0; l + 1 < H->nlev; ++l) {
        mg_level *F = &H->lv[l], *C = &H->lv[l + 1];
        galerkin_faces(F, C, d_ghost, mirror);
        if (coarsen_sa)
            mean8(C->nx, C->ny, C->nz, F->ny, F->nz, F->sa, C->sa);
    }
    mg_level *Lc = &H->lv[H->nlev - 1];
    assemble_level(Lc, d_ghost, mirror, H->chol);
    return fldo_cholesky_factor(Lc->nx * Lc->ny * Lc->nz, H->chol);
}

/* ------------------------------------------------------------------------ */
/* Cluster deflation (this project's addition to the multigrid              */
/* preconditioner).  A cluster is a connected set of voxels joined by       */
/* strong faces: faces whose classical-diffusion coefficient                */
/* ((1/3)/sig_p + (1/3)/sig_s)/2 exceeds tau*L (L the grid extent).  Vacuum  */
/* bubbles and the voxels around them form such clusters; the fluence is    */
/* nearly constant over each and box coarsening cannot represent it.        */
/* Clusters never touch each other, so the Galerkin matrix of their         */
/* indicator functions is diagonal: d_c = sum_{p in c} sa_p + sum of the    */
/* coefficients (/h^2) of faces leaving c.  One deflation step              */
/* e1 = sum_c (sum_{p in c} r_p / d_c) 1_c precedes the V-cycle, which then */
/* works on r - A e1.  It does so by starting the finest smoothing from e1  */
/* with right-hand side r: every step of the cycle is affine in the         */
/* correction and the right-hand side, so this equals e1 plus a cycle from  */
/* zero on r - A e1, without forming A e1.                                  */
/* ------------------------------------------------------------------------ */

static int uf_find(int *parent, int x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];
        x = parent[x];
    }
    return x;
}

static void uf_union(int *parent, int a, int b)
{
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b)
        return;
    if (a < b)
        parent[b] = a;
    else
        parent[a] = b;
}

/* label[c] = cluster id (0..K-1, numbered by first voxel in index order) for
 * voxels in clusters of two or more voxels, -1 otherwise.  Returns K. */
int fldo_clusters(int nx, int ny, int nz, double h, const double *sig_hat, double tau, int *label)
{
    long n = (long)nx * ny * nz;
    int nmax = nx > ny ? (nx > nz ? nx : nz) : (ny > nz ? ny : nz);
    double thresh = tau * h * nmax;
    int *parent = (int *)malloc(sizeof(int) * n);
    int *size = (int *)calloc(n, sizeof(int));
    for (long c = 0; c < n; ++c)
        parent[c] = (int)c;
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j)
            for (int k = 0; k < nz; ++k) {
                long c = idx3(ny, nz, i, j, k);
                double dc = (1.0 / 3.0) / sig_hat[c];
                long up[3] = {i + 1 < nx ? idx3(ny, nz, i + 1, j, k) : -1,
                              j + 1 < ny ? idx3(ny, nz, i, j + 1, k) : -1,
                              k + 1 < nz ? idx3(ny, nz, i, j, k + 1) : -1};
                for (int a = 0; a < 3; ++a) {
                    if (up[a] < 0)
                        continue;
                    double F = 0.5 * (dc + (1.0 / 3.0) / sig_hat[up[a]]);
                    if (F > thresh)
                        uf_union(parent, (int)c, (int)up[a]);
                }
            }
    for (long c = 0; c < n; ++c)
        size[uf_find(parent, (int)c)] += 1;
    int K = 0;
    int *id = (int *)malloc(sizeof(int) * n);
    for (long c = 0; c < n; ++c)
        id[c] = -1;
    for (long c = 0; c < n; ++c) {
        int root = uf_find(parent, (int)c);
        if (size[root] < 2) {
            label[c] = -1;
            continue;
        }
        if (id[root] < 0)
            id[root] = K++;
        label[c] = id[root];
    }
    free(parent);
    free(size);
    free(id);
    return K;
}

/* Diagonal of the cluster Galerkin matrix for the finest operator A(D). */
static void cluster_diag(const mg_level *L, double d_ghost, int mirror, const int *label, int K,
                         double *d)
{
    double h2 = L->h * L->h;
    for (int q = 0; q < K; ++q)
        d[q] = 0.0;
    for (int i = 0; i < L->nx; ++i)
        for (int j = 0; j < L->ny; ++j)
            for (int k = 0; k < L->nz; ++k) {
                long c = idx3(L->ny, L->nz, i, j, k);
                int lc = label[c];
                if (lc < 0)
                    continue;
                double v = L->sa[c];
                for (int s = 0; s < 6; ++s) {
                    int ax = NB[s][0] ? 0 : (NB[s][1] ? 1 : 2);
                    int up = NB[s][0] + NB[s][1] + NB[s][2] > 0;
                    int a = i + NB[s][0], b = j + NB[s][1], q = k + NB[s][2];
                    int same = inside(L->nx, L->ny, L->nz, a, b, q) &&
                               label[idx3(L->ny, L->nz, a, b, q)] == lc;
                    if (same)
                        continue;
                    double F = up ? face(L, d_ghost, mirror, ax, a, b, q)
                                  : face(L, d_ghost, mirror, ax, i, j, k);
                    v = v + F / h2;
                }
                d[lc] = d[lc] + v;
            }
}

/* e1 = sum_c (sum_{p in c} r_p / d_c) 1_c. */
static void cluster_correction(long n, const int *label, int K, const double *d, const double *r,
                               double *sum, double *e1)
{
    for (int q = 0; q < K; ++q)
        sum[q] = 0.0;
    for (long c = 0; c < n; ++c)
        if (label[c] >= 0)
            sum[label[c]] = sum[label[c]] + r[c];
    for (long c = 0; c < n; ++c)
        e1[c] = label[c] >= 0 ? sum[label[c]] / d[label[c]] : 0.0;
}

/* Linear V-cycle on a caller-given finest system (test hook): e0 receives
 * one V(nu1,nu2) cycle from zero for A(D0) e = b0. */
int fldo_linear_vcycle(int nx, int ny, int nz, double h, double d_ghost, int mirror,
                       const fldo_solve_opts *o, const double *D0, const double *sa0,
                       const double *b0, double *e0)
{
    int dims[3 * FLDO_MAX_LEVELS];
    int nlev = fldo_mg_levels(nx, ny, nz, o->max_coarsest, dims, FLDO_MAX_LEVELS);
    if (nlev <= 0 || nlev > FLDO_MAX_LEVELS)
        return -1;
    mg_hier H;
    if (hier_alloc(&H, dims, nlev, h)) {
        hier_free(&H);
        return -2;
    }
    long n = (long)nx * ny * nz;
    H.lv[0].D = D0;
    memcpy(H.lv[0].sa, sa0, sizeof(double) * n);
    memcpy(H.lv[0].b, b0, sizeof(double) * n);
    int rc = hier_coarsen(&H, 1, d_ghost, mirror);
    if (rc == 0) {
        vcycle(H.lv, 0, nlev, o, d_ghost, mirror, H.chol, NULL);
        memcpy(e0, H.lv[0].e, sizeof(double) * n);
    }
    hier_free(&H);
    return rc;
}

/* Level-1 operator of the hierarchy applied to x1 (test hook): out1 = A_1 x1
 * with A_1 built from the finest D and sa by the Galerkin rule. */
int fldo_coarse_apply(int nx, int ny, int nz, double h, double d_ghost, int mirror,
                      const double *D0, const double *sa0, const double *x1, double *out1)
{
    if ((nx % 2) || (ny % 2) || (nz % 2))
        return -1;
    int dims[6] = {nx, ny, nz, nx / 2, ny / 2, nz / 2};
    mg_hier H;
    if (hier_alloc(&H, dims, 2, h)) {
        hier_free(&H);
        return -2;
    }
    long n = (long)nx * ny * nz;
    H.lv[0].D = D0;
    memcpy(H.lv[0].sa, sa0, sizeof(double) * n);
    galerkin_faces(&H.lv[0], &H.lv[1], d_ghost, mirror);
    mean8(nx / 2, ny / 2, nz / 2, ny, nz, H.lv[0].sa, H.lv[1].sa);
    level_apply(&H.lv[1], d_ghost, mirror, x1, out1);
    hier_free(&H);
    return 0;
}

/* Finest-level residual r = b - A(D) e with zero ghosts (test hook). */
void fldo_level_residual(int nx, int ny, int nz, double h, double d_ghost, int mirror,
                         const double *D, const double *sa, const double *b, const double *e,
                         double *r)
{
    mg_level L;
    memset(&L, 0, sizeof(L));
    L.nx = nx; L.ny = ny; L.nz = nz; L.h = h;
    L.D = D; L.sa = (double *)sa; L.b = (double *)b; L.e = (double *)e;
    level_residual(&L, d_ghost, mirror, r);
}

/* ------------------------------------------------------------------------ */
/* Solvers                                                                  */
/* ------------------------------------------------------------------------ */

static void record(double *hist, int cap, int *len, double v)
{
    if (hist && *len < cap)
        hist[*len] = v;
    ++*len;
}

/* Algorithm 1 to tolerance.  phi and D are the state (in: start, out: end).
 * The stopping test uses the true nonlinear residual, checked every
 * check_every iterations and after the last one. */
static int solve_alg1(const fldo_params *p, const fldo_solve_opts *o, const double *sig_hat,
                      const double *sig_a, const double *j_src, double *phi, double *D,
                      double *hist, int cap, fldo_result *res)
{
    long n = (long)p->nx * p->ny * p->nz;
    double *Dt = (double *)malloc(sizeof(double) * n);
    int it = 0, len = 0, status = FLDO_NOT_CONVERGED;
    double rel = NAN, rel_sweep = NAN;
    int every = o->check_every > 0 ? o->check_every : 1;
    for (;;) {
        if (it % every == 0 || it == o->max_iters) {
            rel = fldo_nonlinear_residual(p, phi, sig_hat, sig_a, j_src, Dt, NULL) / p->jnorm;
            record(hist, cap, &len, rel);
            if (!isfinite(rel)) { status = FLDO_DIVERGED; break; }
            if (rel <= o->tol) { status = FLDO_CONVERGED; break; }
            if (it >= o->max_iters) { status = FLDO_NOT_CONVERGED; break; }
        }
        double s = fldo_alg1_iteration(p, o->omega, phi, D, sig_hat, sig_a, j_src);
        rel_sweep = sqrt(s / (double)n) / p->jbar;
        ++it;
    }
    free(Dt);
    res->status = status;
    res->iterations = it;
    res->rel = rel;
    res->rel_sweep = rel_sweep;
    res->history_len = len;
    return status;
}

/* Anderson coefficients: gamma solves (G + lambda I) gamma = h with
 * G_ij = dF_i . dF_j, h_i = dF_i . f over the *na history columns (column i
 * of dF at dF + i*n), lambda = reg * trace(G) / na, by Cholesky.  When the
 * factorisation fails the history is dropped (*na = 0). */
static void anderson_coefficients(long n, int na, const double *dF, const double *f, double reg,
                                  double *gam, int *na_out)
{
    double G[FLDO_MAX_AA * FLDO_MAX_AA], h[FLDO_MAX_AA];
    *na_out = na;
    if (na == 0)
        return;
    for (int i = 0; i < na; ++i) {
        double hi = 0.0;
        for (long c = 0; c < n; ++c)
            hi += dF[(long)i * n + c] * f[c];
        h[i] = hi;
        for (int j = 0; j <= i; ++j) {
            double g = 0.0;
            for (long c = 0; c < n; ++c)
                g += dF[(long)i * n + c] * dF[(long)j * n + c];
            G[i * na + j] = g;
            G[j * na + i] = g;
        }
    }
    double tr = 0.0;
    for (int i = 0; i < na; ++i)
        tr += G[i * na + i];
    const double lambda = reg * tr / (double)na;
    for (int i = 0; i < na; ++i)
        G[i * na + i] = G[i * na + i] + lambda;
    if (fldo_cholesky_factor(na, G) != 0) {
        *na_out = 0;
        return;
    }
    fldo_cholesky_solve(na, G, h, gam);
}

/* Picard-multigrid with nonlinear preconditioned conjugate gradients.
 * Outer iteration k:
 *   D^k = limiter pass on phi^k (every voxel), r^k = j - A(D^k) phi^k (FP64),
 *   stop when ||r^k||/||j|| <= tol;
 *   e^k = the preconditioner applied to r^k: cluster deflation e1, then one
 *   V-cycle for A(D^k) e = r^k whose finest smoothing starts from e1 (equal
 *   to e1 plus a cycle from zero on r^k - A(D^k) e1);
 *   gamma_k = r^k.e^k; beta_k = max(0, (gamma_k - e^k.r^{k-1}) / gamma_{k-1})
 *   (Polak-Ribiere, restarted when negative; beta_0 = 0);
 *   p^k = e^k + beta_k p^{k-1};
 *   theta_k = (r^k.p^k) / (p^k.A(D^k) p^k)  (energy-optimal step);
 *   phi^{k+1} = phi^k + theta_k p^k.
 * With a constant D (CDA) this is preconditioned CG on the linear system.
 * step_mode 0 replaces the direction and step by p = e, theta = option.
 *
 * aa_m > 0 replaces the conjugate-gradient step by Anderson acceleration of
 * the preconditioned Picard map x -> x + e(x) (window m; Walker and Ni's
 * formulation):
 *   f_k = e^k; the history holds the last pairs dX_i = x_{i+1} - x_i,
 *   dF_i = f_{i+1} - f_i, oldest first; after an iteration that raised the
 *   residual norm by more than restart_growth (> 0) it is cleared;
 *   G_ij = dF_i . dF_j, h_i = dF_i . f_k; gamma solves
 *   (G + lambda I) gamma = h by Cholesky, lambda = aa_reg trace(G)/n_hist
 *   (a failed factorisation clears the history);
 *   x_{k+1} = x_k + f_k - sum_i gamma_i (dX_i + dF_i), the sum oldest first. */
static int solve_mg(const fldo_params *p, const fldo_solve_opts *o, const double *sig_hat,
                    const double *sig_a, const double *j_src, double *phi, double *hist,
                    int cap, fldo_result *res)
{
    int dims[3 * FLDO_MAX_LEVELS];
    int nlev = fldo_mg_levels(p->nx, p->ny, p->nz, o->max_coarsest, dims, FLDO_MAX_LEVELS);
    if (nlev <= 0 || nlev > FLDO_MAX_LEVELS)
        return FLDO_INVALID;
    mg_hier H;
    if (hier_alloc(&H, dims, nlev, p->h)) {
        hier_free(&H);
        return FLDO_INVALID;
    }
    long n = (long)p->nx * p->ny * p->nz;
    double d_ghost = p->eps * p->h;
    double *D = (double *)malloc(sizeof(double) * n);
    double *dir = (double *)calloc(n, sizeof(double));
    double *q = (double *)malloc(sizeof(double) * n);
    double *r_prev = (double *)calloc(n, sizeof(double));
    double *r = (double *)malloc(sizeof(double) * n);
    double *e1 = (double *)calloc(n, sizeof(double));
    double *e = H.lv[0].e;
    int *label = (int *)malloc(sizeof(int) * n);
    int K = o->deflate_tau > 0.0
                ? fldo_clusters(p->nx, p->ny, p->nz, p->h, sig_hat, o->deflate_tau, label)
                : 0;
    double *dcl = (double *)malloc(sizeof(double) * (K > 0 ? K : 1));
    double *scl = (double *)malloc(sizeof(double) * (K > 0 ? K : 1));
    H.lv[0].D = D;
    memcpy(H.lv[0].sa, sig_a, sizeof(double) * n);
    int it = 0, len = 0, status = FLDO_NOT_CONVERGED, first = 1;
    double rel = NAN, rel_prev = NAN, gamma_prev = 0.0;
    /* Anderson history: aa_m pairs (dX, dF), oldest first, plus f_{k-1} and
     * the last step x_k - x_{k-1} */
    const int am = o->aa_m > 0 ? o->aa_m : 0;
    double *aX = am ? (double *)malloc(sizeof(double) * n * am) : NULL;
    double *aF = am ? (double *)malloc(sizeof(double) * n * am) : NULL;
    double *f_prev = am ? (double *)malloc(sizeof(double) * n) : NULL;
    double *dx_last = am ? (double *)malloc(sizeof(double) * n) : NULL;
    int na = 0;
    for (;;) {
        fldo_limiter_pass(p, phi, sig_hat, D);
        rel = fldo_residual(p, phi, D, sig_a, j_src, r) / p->jnorm;
        record(hist, cap, &len, rel);
        if (!isfinite(rel)) { status = FLDO_DIVERGED; break; }
        if (rel <= o->tol) { status = FLDO_CONVERGED; break; }
        if (it >= o->max_iters) { status = FLDO_NOT_CONVERGED; break; }
        if (hier_coarsen(&H, first, d_ghost, p->mirror_d)) { status = FLDO_DIVERGED; break; }
        first = 0;
        /* preconditioner: cluster deflation, then one V-cycle whose finest
         * smoothing starts from the deflation step */
        if (K > 0) {
            cluster_diag(&H.lv[0], d_ghost, p->mirror_d, label, K, dcl);
            cluster_correction(n, label, K, dcl, r, scl, e1);
        }
        memcpy(H.lv[0].b, r, sizeof(double) * n);
        vcycle(H.lv, 0, nlev, o, d_ghost, p->mirror_d, H.chol, K > 0 ? e1 : NULL);
        if (am) {
            if (it > 0 && o->restart_growth > 0.0 && rel > o->restart_growth * rel_prev) {
                na = 0;
            } else if (it > 0) {
                if (na == am) {
                    memmove(aX, aX + n, sizeof(double) * n * (am - 1));
                    memmove(aF, aF + n, sizeof(double) * n * (am - 1));
                    --na;
                }
                for (long c = 0; c < n; ++c) {
                    aX[(long)na * n + c] = dx_last[c];
                    aF[(long)na * n + c] = e[c] - f_prev[c];
                }
                ++na;
            }
            rel_prev = rel;
            memcpy(f_prev, e, sizeof(double) * n);
            double gam[FLDO_MAX_AA];
            anderson_coefficients(n, na, aF, e, o->aa_reg, gam, &na);
            for (long c = 0; c < n; ++c) {
                double step = e[c];
                for (int i = 0; i < na; ++i)
                    step = step - gam[i] * (aX[(long)i * n + c] + aF[(long)i * n + c]);
                double x_new = phi[c] + step;
                dx_last[c] = x_new - phi[c];
                phi[c] = x_new;
            }
            ++it;
            continue;
        }
        double theta;
        if (o->step_mode == 1 || o->step_mode == 2) {
            double gamma = 0.0, e_rprev = 0.0;
            for (long c = 0; c < n; ++c) {
                gamma += r[c] * e[c];
                e_rprev += e[c] * r_prev[c];
            }
            /* Polak-Ribiere+ coefficient; mode 1 restarts (beta = 0) after an
             * iteration that raised the residual norm by more than the factor
             * restart_growth */
            double beta = 0.0;
            const int restart = o->step_mode == 1 && o->restart_growth > 0.0 &&
                                rel > o->restart_growth * rel_prev;
            if (it > 0 && !restart) {
                beta = (gamma - e_rprev) / gamma_prev;
                if (!(beta > 0.0))
                    beta = 0.0;
            }
            for (long c = 0; c < n; ++c)
                dir[c] = e[c] + beta * dir[c];
            level_apply(&H.lv[0], d_ghost, p->mirror_d, dir, q);
            double rp = 0.0, pq = 0.0;
            for (long c = 0; c < n; ++c) {
                rp += r[c] * dir[c];
                pq += dir[c] * q[c];
            }
            theta = rp / pq;
            gamma_prev = gamma;
            rel_prev = rel;
            memcpy(r_prev, r, sizeof(double) * n);
        } else {
            memcpy(dir, e, sizeof(double) * n);
            theta = o->theta;
        }
        for (long c = 0; c < n; ++c)
            phi[c] = phi[c] + theta * dir[c];
        ++it;
    }
    free(aX);
    free(aF);
    free(f_prev);
    free(dx_last);
    free(D);
    free(dir);
    free(q);
    free(r_prev);
    free(r);
    free(e1);
    free(label);
    free(dcl);
    free(scl);
    hier_free(&H);
    res->status = status;
    res->iterations = it;
    res->rel = rel;
    res->rel_sweep = NAN;
    res->history_len = len;
    return status;
}

/* Paper initial state (Alg. 1 / Sec. 5): phi = eps*jbar*h, D = eps*h. */
void fldo_init_state(const fldo_params *p, double *phi, double *D)
{
    long n = (long)p->nx * p->ny * p->nz;
    for (long c = 0; c < n; ++c) {
        if (phi) phi[c] = p->eps * p->jbar * p->h;
        if (D) D[c] = p->eps * p->h;
    }
}

int fldo_solve(const fldo_params *p, const fldo_solve_opts *o, const double *sig_hat,
               const double *sig_a, const double *j_src, double *phi, double *D, double *hist,
               int cap, fldo_result *res)
{
    memset(res, 0, sizeof(*res));
    long n = (long)p->nx * p->ny * p->nz;
    if (p->jbar == 0.0) {
        /* No emission: the fluence is the boundary value, nothing to solve. */
        for (long c = 0; c < n; ++c)
            phi[c] = p->phi_b;
        res->status = FLDO_CONVERGED;
        res->rel = 0.0;
        return FLDO_CONVERGED;
    }
    if (o->method == FLDO_METHOD_ALG1)
        return solve_alg1(p, o, sig_hat, sig_a, j_src, phi, D, hist, cap, res);
    return solve_mg(p, o, sig_hat, sig_a, j_src, phi, hist, cap, res);
}

/* ------------------------------------------------------------------------ */
/* Light baking (Sec. 3: single-scatter source of an external directional    */
/* light, q_ri = L_l sigma_s T with T the transmittance towards the light,   */
/* the "deep shadow map"; Sec. 6 bakes it by ray-marching).  Reading: the     */
/* light travels +z and enters at the z = 0 face; in voxel k of a column     */
/* T = exp(-h (sum_{k' < k} sigma_t + sigma_t(k)/2)) (midpoint of the voxel,  */
/* raw sigma_t), sigma_s = albedo sigma_t.  Pinned against the closed form of */
/* a homogeneous column and the product form of T.                           */
/* ------------------------------------------------------------------------ */
void fldo_light_bake(int nx, int ny, int nz, double h, double light, const double *sigma_t,
                     const double *albedo, double *q)
{
#pragma omp parallel for schedule(static) if (FLDO_PARALLEL((long)nx * ny * nz))
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            double tau = 0.0;                    /* sum of sigma_t over k' < k */
            for (int k = 0; k < nz; ++k) {
                long c = idx3(ny, nz, i, j, k);
                double s = sigma_t[c];
                double T = exp(-h * (tau + 0.5 * s));
                q[c] = light * albedo[c] * s * T;
                tau = tau + s;
            }
        }
}

/* ------------------------------------------------------------------------ */
/* Primary ray-march (Sec. 3): the radiance reaching the camera is the        */
/* attenuated back-light plus the source of every sample attenuated by the    */
/* transmittance between the sample and the ray's end, Delta x times the sum; */
/* with the diffusion solution the source is 4 pi Q = q_ri + sigma_s phi + j  */
/* (Sec. 3, the source in terms of phi).  Reading: an orthographic camera on  */
/* the +z side, one ray per (i, j) column travelling +z from the z = 0 face;  */
/* the sample of voxel k sees T = exp(-h (sigma_t(k)/2 + sum_{k' > k}         */
/* sigma_t)) (midpoint, as the bake), the back-light `background` enters at    */
/* z = 0 and is attenuated by exp(-h sum_k sigma_t).  src = q_ri + j (the     */
/* solver's emission), sigma_s = albedo sigma_t.  image: nx*ny, index i*ny+j. */
/* Pinned against the closed form of a homogeneous column.                    */
/* ------------------------------------------------------------------------ */
void fldo_render(int nx, int ny, int nz, double h, double background, const double *sigma_t,
                 const double *albedo, const double *src, const double *phi, double *image)
{
    const double four_pi = 4.0 * 3.14159265358979323846;
#pragma omp parallel for schedule(static) if (FLDO_PARALLEL((long)nx * ny * nz))
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            double tau = 0.0;                    /* sum of sigma_t over k' > k */
            double radiance = 0.0;
            for (int k = nz - 1; k >= 0; --k) {
                long c = idx3(ny, nz, i, j, k);
                double s = sigma_t[c];
                double T = exp(-h * (0.5 * s + tau));
                double Q = (src[c] + albedo[c] * s * phi[c]) / four_pi;
                radiance = radiance + h * T * Q;
                tau = tau + s;
            }
            image[(long)i * ny + j] = radiance + background * exp(-h * tau);
        }
}
