// fld_internal.h -- device-side descriptors shared by the HIP kernels and the
// host engine of libfld.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/fld.h"

namespace fld {

constexpr int kBlock = 256;          // threads per block of the work-list kernels
constexpr int kTaskCells = 4096;     // cells per work-list task
constexpr int kAaTaskCells = 16384;  // cells per task of the Anderson dot products
constexpr int kMaxLevels = 16;

// One multigrid level of one problem.  Arrays are z fastest,
// index (i*ny + j)*nz + k.  The finest level keeps cell coefficients D (its
// face coefficients follow the discretised equation, (D_p + D_s)/2 with the
// ghost rule); coarse levels keep Galerkin face coefficients f: three
// (nx+1)(ny+1)(face_zstride(nz)) arrays back to back, f[a](i,j,k) = face
// below (i,j,k) along axis a; rows along z are padded to a multiple of four
// entries so that a quad of faces is one aligned 16-byte load.
__host__ __device__ inline long long face_zstride(int nz)
{
    return (long long)((nz + 4) & ~3);     // nz + 1 rounded up to a multiple of 4
}

struct Grid {
    int nx, ny, nz, prob;
    long long n;
    double h2;       // h_l^2
    double dghost;   // ghost coefficient of the finest level (eps*h)
    int fine;        // 1: cell D, 0: face arrays
    int mirror;      // finest level: ghost D = D of the voxel inside
    int finer;       // index of the next finer grid in the same table (-1: none)
    int coarser;     // index of the next coarser grid (-1: none)
    int split;       // e, b, sa, D stored colour by colour (see Fine::split)
    short nu_pre;    // smoothing sweeps of this level before the coarse correction
    short nu_post;   // and after it
    void *e, *b, *sa, *D, *f;
    void *e2;        // finest level: second correction buffer of the fused sweep
    double *band;    // coarsest level: banded Cholesky factor of h^2 A, n*(ny*nz+1)
};

// A contiguous run of cells [start, start+count) of grid `grid`.
struct Task {
    int grid;
    int count;
    long long start;
};

// Finest-level FP64 state of one problem (one colour channel of one volume).
struct Fine {
    int nx, ny, nz, prob;
    long long n;
    double h, h2, dghost, eps, phi_b, larsen_n;
    int mirror, limiter, write_sighat;
    int split;           // precision-T fields e0, b0, D0, sa0 stored colour by colour in
                         // blocks of 64 cells: cell c of colour q = (i+j+k)&1 at
                         // (c>>6)*64 + q*32 + ((c>>1)&31); nz % 8 == 0
    double *sig_hat, *sa64, *j;
    double *phi[2];      // fluence ping-pong: phi^k lives in phi[k & 1]
    double *D64;         // limiter output (multigrid) / Algorithm 1 state D
    double *Dtmp;        // Algorithm 1: D of the true-residual check
    void *b0[2];         // V-cycle right-hand side ping-pong (precision T)
    void *e0;            // finest correction (precision T)
    void *p[2];          // search-direction ping-pong (precision T)
    void *D0, *sa0;      // finest coefficients in precision T
    const int *label;    // cluster of each voxel (-1: none), per volume
    const int *cpos;     // storage positions (precision-T fields) of the voxels of every
                         // cluster, cluster by cluster, per volume
    const int *rcells;   // rim voxels (a face leaves their cluster), cluster by cluster
    const unsigned short *rmask;  // per rim voxel: faces leaving the cluster (bits 0-5),
                                  // of which ghost faces (bits 6-11)
    int cbase;           // first global cluster index of this problem
    int ncl;             // clusters of this problem
    // Anderson acceleration (precision T, natural order): f of the previous
    // iteration, and the history ring, slot s of dF / dG = dX + dF at s*n
    void *aa_fprev, *aa_dF, *aa_dG;
};

// A tile of the fused limiter-residual pass: planes [i0, i0+ni) of rows
// [j0, j0+16) and cells [k0, k0+32) along z (clipped to the grid) of problem
// `prob`.
struct LrTile {
    int prob;
    int i0, ni;
    int j0, k0;
};
constexpr int kLrTileRows = 16, kLrTileCells = 32, kLrTilePlanes = 32;

// A run of cluster voxels: entries [start, start+count) of the problem's
// cpos (cell tasks) or rcells (rim tasks) list, all in global cluster `cl`.
struct CTask {
    int prob;
    int cl;
    int start;
    int count;
};

// Device workspace of one residual evaluation on a grid of at most
// max_cells cells: D and the right-hand-side copy of r (max_cells doubles
// each) and the problem descriptor.
struct ResidualWork {
    double *D;
    double *b;
    Fine *fine;
    long long max_cells;
};

// Engine entry points for code outside fld_engine.cpp: the residual of a
// device fluence of context c computed in workspace ws (nothing allocated),
// and the HIP device a context runs on.
fld_status residual_with_workspace(fld_context *c, const double *d_phi, double *d_r_out,
                                   double *rel_out, const ResidualWork *ws);
int context_device(const fld_context *c);

// Per-problem device scalars.
enum Scalar {
    S_JN2 = 0, S_JBAR, S_JNORM, S_RES2, S_REL, S_GAMMA, S_GAMMA_PREV, S_SIGMA, S_RP, S_PAP,
    S_BETA, S_THETA, S_SWEEP2, S_AUX, S_REL_PREV, S_COUNT
};

enum Limiter { L_CDA = 0, L_LP = 1, L_SUM = 2, L_MAX = 3, L_KERSHAW = 4, L_LARSEN = 5 };

// ---- launchers (fld_kernels.hip) ----------------------------------------
// Every launcher enqueues on `s`; tasks/grids/fines are device pointers.
// `active` (device, per problem, may be null) masks converged problems.

// Algorithm 1 set-up for one problem: sig_hat = max(sigma_t, sigma_eps)
// (written when f.write_sighat), sa = (1 - albedo) sig_hat, j = Q, partial
// sums of Q^2 per task.
// Fine-level launchers take `mixed` as a precision/layout mode: 0 FP64,
// 1 FP32 natural order, 2 FP32 colour-split, 3 FP32 decided per problem.
// Level launchers take sp: 0 natural, 1 colour-split finest level, 2 per
// problem.
void launch_setup(hipStream_t s, const Fine &f, const Task *tasks, int ntasks,
                  const double *sigma_t, const double *albedo, const double *Q,
                  double sigma_eps, double aniso_g, double *partials, int mixed);
void launch_sum_partials(hipStream_t s, int nprob, const int *range, const double *partials,
                         double *scal, int slot, const int *active);
void launch_after_setup(hipStream_t s, int nprob, const Fine *fines, double *scal);
void launch_init_phi(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                     const double *scal, int zero_dirs, int mixed);
// lim_kind: the limiter of every grid in the list (an LP-only kernel instance
// is launched for L_LP), or -1 when they differ
void launch_limiter(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                    const int *active, const double *scal, int src, int dst, int use_dir,
                    int dir_idx, int to_tmp, int mixed, int lim_kind);
void launch_residual(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                     const int *active, int src, int use_tmp, int b0_idx, double *r_out,
                     double *partials, int mixed);
void launch_rel(hipStream_t s, int nprob, double *scal, const int *active);
void launch_npcg_dots(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                      const int *active, int b0_idx, double *pg, double *ps, int mixed);
void launch_npcg_beta(hipStream_t s, int nprob, double *scal, const int *active, int first,
                      double restart_growth);
void launch_npcg_dir(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                     const int *active, const double *scal, int b0_idx, int pin, int pout,
                     double *prp, double *ppap, int mixed);
void launch_npcg_theta(hipStream_t s, int nprob, double *scal, const int *active);
// Cluster deflation.  launch_defl_sum_sa (once per medium): per cell task
// the sum of sa over its cluster cells; launch_defl_sum_b: per cell task the
// sum of b0; launch_defl_rim: per rim task the face terms F/h^2 of the faces
// leaving the cluster; launch_defl_finish: per cluster the sums of its task
// partials, into csa (sa_only) or alpha = s / (csa + rim); launch_defl_init:
// the finest level's starting correction e0 = alpha[label].
void launch_defl_sum_sa(hipStream_t s, const Fine *fines, const CTask *ct, int nct, double *psa,
                        int mixed);
void launch_defl_sum_b(hipStream_t s, const Fine *fines, const CTask *ct, int nct,
                       const int *active, int b0_idx, double *ps, int mixed);
void launch_defl_rim(hipStream_t s, const Fine *fines, const CTask *rt, int nrt,
                     const int *active, double *pd, int mixed);
void launch_defl_finish(hipStream_t s, int ncl_total, const int *crange, const int *rrange,
                        const int *cprob, const double *ps, const double *pd, double *csa,
                        double *alpha, const int *active, int sa_only);
void launch_defl_init(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                      const int *active, const double *alpha, int mixed);
// Grid sequencing: the 2:1 coarsened medium (sigma_t, albedo, Q) from the
// finest set-up fields, and the coarse fluence copied onto its 2x2x2 blocks.
void launch_nested_coarsen(hipStream_t s, const double *sig_hat, const double *sa,
                           const double *j, int nx, int ny, int nz, double *st_c, double *al_c,
                           double *q_c);
void launch_nested_prolong(hipStream_t s, const double *phi_c, int nx, int ny, int nz,
                           double *phi);
void launch_alg1_pass(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                      const double *scal, int colour, double omega, double *partials);
// Anderson acceleration of the outer iteration (window m <= aa_max_window()):
// per-problem state aai (aa_state_ints() ints) and aad (aa_state_doubles()
// doubles); reset at the start of a solve; per iteration dots (partials of
// 2(m+1) values per task), sums, solve (one thread per problem) and update
// phi[dst] = phi[src] + f - sum gamma dG, dG = dX + dF.
void launch_aa_reset(hipStream_t s, int nprob, int *aai);
void launch_aa_dots(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                    const int *active, int *aai, double *aad, int m, double *partials, int mixed);
void launch_aa_sums(hipStream_t s, int nprob, const int *range, const double *partials,
                    int ntasks, int *aai, double *aad, int m, const int *active);
void launch_aa_solve(hipStream_t s, int nprob, double *scal, int *aai, double *aad, int m,
                     double reg, double growth, const int *active);
void launch_aa_update(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                      const int *active, int *aai, double *aad, int src, int dst, int mixed);
int aa_max_window();
int aa_state_ints();
int aa_state_doubles();
// Write a problem descriptor to device memory (a kernel, not a copy).
void launch_put_fine(hipStream_t s, const Fine &f, Fine *dst);

// Multigrid level kernels, precision T = float (mixed) or double.  `grids`
// is the device table of every level of every problem; a task names the grid
// it works on (for restriction and Galerkin coarsening: the coarse grid, for
// prolongation: the fine grid).
template <typename T>
void launch_zero(hipStream_t s, const Grid *grids, const Task *tasks, int ntasks,
                 const int *active);
template <typename T>
void launch_smooth(hipStream_t s, const Grid *grids, const Task *tasks, int ntasks,
                   const int *active, int colour, double omega, bool finest);
// One half-sweep of a coarse (not the finest) level of a single problem, the
// level passed by value (no task list, no activity mask): block b smooths
// cells [b * task_cells, (b + 1) * task_cells); task_cells a multiple of 8.
// The same result as launch_smooth over that level's tasks.
template <typename T>
void launch_smooth_one(hipStream_t s, const Grid &g, int task_cells, int colour, double omega);
template <typename T>
void launch_restrict(hipStream_t s, const Grid *grids, const Task *tasks, int ntasks,
                     const int *active, int sp);
template <typename T>
void launch_prolong(hipStream_t s, const Grid *grids, const Task *tasks, int ntasks,
                    const int *active, int sp, double scale);
template <typename T>
void launch_galerkin(hipStream_t s, const Grid *grids, const Task *tasks, int ntasks,
                     const int *active, int sp);
template <typename T>
void launch_mean8_sa(hipStream_t s, const Grid *grids, const Task *tasks, int ntasks);
// Coarsest level: one block per listed grid.  fail[prob] is set to 1 when a
// pivot is not positive.
// Deep part of the V-cycle, one workgroup per root (the first level of a
// problem at or below the deep size limit): down (zero, Grid::nu_pre
// pre-sweeps, restrict) or up (prolong, Grid::nu_post post-sweeps) over the
// levels above the coarsest.
template <typename T>
void launch_deep(hipStream_t s, const Grid *grids, const int *roots, int count, const int *active,
                 double omega, bool down);
template <typename T>
void launch_coarse_solve(hipStream_t s, const Grid *grids, const int *ids, int count,
                         const int *active, int *fail, int max_n, int max_bw);
// Factor of the coarsest operator of each listed grid whose band fits in LDS,
// into Grid::band (the solve kernels and the tail then substitute only); it
// reads only the coarse operators, so it may run on a second stream beside the
// down-sweep.  fail[prob] is set to 1 when a pivot is not positive.
// Failure injection: phi[src][0] = NaN for each of the nprob problems.
void launch_poison(hipStream_t s, const Fine *fines, int nprob, int src);
// One red-black sweep of the finest level (first colour `first`, then the
// other) in one pass over LrTile tiles (tile.prob: the level-0 grid index),
// out of place: dir 0 reads Grid::e and writes Grid::e2, dir 1 the reverse.
// The same result as the two half-sweeps of launch_smooth.  Needs nz % 4 == 0.
template <typename T>
void launch_smooth_rb(hipStream_t s, const Grid *grids, const LrTile *tiles, int ntiles,
                      const int *active, int first, int dir, double omega, int sp);
// Limiter and residual of the finest level in one pass over LrTile tiles
// (grids with nz % 4 == 0): D (precision T; also FP64 when write_d64), r in
// b0[b0_idx] (precision T) and one partial sum of r^2 per tile; the same D and
// r as launch_limiter (without the direction update) + launch_residual.
void launch_lim_res(hipStream_t s, const Fine *fines, const LrTile *tiles, int ntiles,
                    const int *active, const double *scal, int src, int b0_idx, int write_d64,
                    double *partials, int mixed);
template <typename T>
void launch_coarse_factor(hipStream_t s, const Grid *grids, const int *ids, int count,
                          const int *active, int *fail, int max_n);
// Coarse tail in one launch per problem (one workgroup each): the deep levels
// from a root (at most tail_root_cells() cells, then at most tail_max_low()
// levels of at most tail_low_cells() cells) down to the coarsest solve and
// back, bit-identical to launch_deep + launch_coarse_solve + launch_deep.  A
// root equal to the coarsest level runs the coarsest solve alone.  lds_bytes:
// the largest tail_lds_need() of the listed problems, at most
// tail_lds_limit().
template <typename T>
void launch_tail(hipStream_t s, const Grid *grids, const int *roots, int count, const int *active,
                 int *fail, double omega, int lds_bytes);
long long tail_lds_need(long long nc, long long bw, long long deep_cells, long long scratch_cells,
                        int tsz);
int tail_lds_limit();
int tail_root_cells();
int tail_low_cells();
int tail_max_low();

}  // namespace fld
