// fld_kernels.hip -- HIP kernels of the flux-limited diffusion solve (gfx950).
//
// Work-list kernels: every launch walks a device table of tasks (runs of
// cells of one grid of one problem), so one launch serves one volume or a
// whole batch of volumes and colour channels.  Blocks stride over the task
// list; a task of a converged problem is skipped.  Reductions are
// deterministic: each task writes one partial sum, and partials are summed
// per problem in task order.
//
// Arithmetic follows the discretised equations of the paper (Sec. 5) in a
// fixed order (neighbours x-, x+, y-, y+, z-, z+), compiled without
// floating-point contraction so FP64 results match a plain scalar reference
// up to the rounding of library functions.
#include <hip/hip_runtime.h>

#include "fld_internal.h"

namespace fld {

namespace {

constexpr int kWave = 64;
// Index of a cell -> (i, j, k).  Cells number fewer than 2^31 and every
// axis fewer than 2^16, so (c + 1/2) * (1/nz) in FP64 lies at least 2^-17
// away from an integer while its rounding error stays below 2^-21: the
// truncation is the exact quotient.  This avoids 64-bit integer division.
struct Dec {
    double inv_ny, inv_nz;
    int ny, nz;
    __device__ Dec(int ny_, int nz_) : inv_ny(1.0 / ny_), inv_nz(1.0 / nz_), ny(ny_), nz(nz_) {}
    __device__ inline void operator()(long long c, int &i, int &j, int &k) const
    {
        const unsigned cu = (unsigned)c;
        const unsigned row = (unsigned)(((double)cu + 0.5) * inv_nz);
        k = (int)(cu - row * (unsigned)nz);
        const unsigned ii = (unsigned)(((double)row + 0.5) * inv_ny);
        j = (int)(row - ii * (unsigned)ny);
        i = (int)ii;
    }
};

__device__ inline void decode(long long c, int ny, int nz, int &i, int &j, int &k)
{
    Dec(ny, nz)(c, i, j, k);
}

// Sum of v over the block; the result is valid in thread 0.
__device__ double block_sum(double v)
{
    __shared__ double ws[kBlock / kWave];
    for (int o = kWave / 2; o > 0; o >>= 1)
        v += __shfl_down(v, o, kWave);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0)
        ws[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kBlock / kWave; ++q)
            t += ws[q];
    __syncthreads();
    return t;
}

// ---------------------------------------------------------------------------
// Quad access: a thread handles 4 consecutive cells along z (k0 % 4 == 0,
// nz % 4 == 0), so each array is read with one 16-byte (FP32) or two
// 16-byte (FP64) loads per neighbour direction.
// ---------------------------------------------------------------------------

__device__ inline void ld4(const float *p, float v[4])
{
    const float4 t = *reinterpret_cast<const float4 *>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
__device__ inline void ld4(const double *p, double v[4])
{
    const double2 a = *reinterpret_cast<const double2 *>(p);
    const double2 b = *reinterpret_cast<const double2 *>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ inline void ld4(const int *p, int v[4])
{
    const int4 t = *reinterpret_cast<const int4 *>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
__device__ inline void st4(float *p, const float v[4])
{
    *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ inline void st4(double *p, const double v[4])
{
    *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2 *>(p + 2) = make_double2(v[2], v[3]);
}

// ---------------------------------------------------------------------------
// Colour-split storage (finest level of the mixed form, nz % 8 == 0).  The
// cells pair up along z, c and c+1 (c even) sharing the compact index
// m = c >> 1; one of the two is red ((i+j+k) even), the other black.  Blocks
// of 32 compact indices are stored as 32 red values then 32 black values
// (2 x 128 bytes in FP32), so cell c of colour q lives at
// (c >> 6) * 64 + q * 32 + ((c >> 1) & 31).  A red-black half-sweep then
// streams whole cache lines of only the colours it needs, while a kernel
// walking cells in natural order still touches one contiguous window.  A
// natural quad c0..c0+3 (c0 % 4 == 0) is two pairs: two 2-value runs.
// Arrays hold n rounded up to 64 values.
// ---------------------------------------------------------------------------

__device__ inline long long sidx(long long c, int q)
{
    return ((c >> 6) << 6) + (q << 5) + ((c >> 1) & 31);
}
// Whether a kernel instance sees split storage: SP = 0 natural, 1 split,
// 2 decided per problem at run time (batches mixing both).
template <int SP>
__device__ inline bool layout_split(int flag)
{
    return SP == 2 ? flag != 0 : SP == 1;
}
// The same for a multigrid level: only finest levels are ever split.
template <int SP>
__device__ inline bool grid_split(const Grid &g)
{
    return SP == 2 ? g.split != 0 : SP == 1 && g.fine;
}
// Storage place of compact index m (= c >> 1) of colour q.
__device__ inline long long cpos(long long m, int q)
{
    return ((m >> 5) << 6) + (q << 5) + (m & 31);
}
template <typename V> struct Pair;
template <> struct Pair<float> { using type = float2; };
template <> struct Pair<double> { using type = double2; };
// Quad of natural cells c0..c0+3 whose first cell has colour q0.
template <typename V>
__device__ inline void ld4s(const V *base, long long c0, int q0, V v[4])
{
    using P2 = typename Pair<V>::type;
    const P2 a = *reinterpret_cast<const P2 *>(base + sidx(c0, q0));
    const P2 b = *reinterpret_cast<const P2 *>(base + sidx(c0, q0 ^ 1));
    v[0] = a.x; v[1] = b.x; v[2] = a.y; v[3] = b.y;
}
template <typename V>
__device__ inline void st4s(V *base, long long c0, int q0, const V v[4])
{
    using P2 = typename Pair<V>::type;
    *reinterpret_cast<P2 *>(base + sidx(c0, q0)) = P2{v[0], v[2]};
    *reinterpret_cast<P2 *>(base + sidx(c0, q0 ^ 1)) = P2{v[1], v[3]};
}
// Quad / single loads of a split or natural array inside a gather() around
// the quad at c0 (colour q0): its x/y neighbour quads and the cell before it
// along z have the other colour, the cell after it the same.
template <typename V>
struct QuadSrc {
    const V *base;
    long long c0;
    int q0, split;
    __device__ void quad(long long x, V v[4]) const
    {
        if (split)
            ld4s(base, x, x == c0 ? q0 : q0 ^ 1, v);
        else
            ld4(base + x, v);
    }
    __device__ V one(long long x) const
    {
        return split ? base[sidx(x, x < c0 ? q0 ^ 1 : q0)] : base[x];
    }
};

// The 7-point neighbourhood of a quad: centre values, the four in-plane /
// out-of-plane neighbour quads, and the single cells before and after it
// along z.  `G` is the value used for ghost cells (callers fill ghost quads
// themselves when the ghost depends on the cell).
template <typename V>
struct Hood {
    V c[4], xm[4], xp[4], ym[4], yp[4];
    V zl, zr;
    __device__ V zm(int m) const { return m == 0 ? zl : c[m - 1]; }
    __device__ V zp(int m) const { return m == 3 ? zr : c[m + 1]; }
};

// Fill a Hood from quad/single loaders; ghost quads take `ghost`.
template <typename V, typename L4, typename L1>
__device__ inline void gather(Hood<V> &h, L4 ld4f, L1 ld1f, long long c0, int i, int j, int k0,
                              int nx, int ny, int nz, long long sx, long long sy, V ghost)
{
    ld4f(c0, h.c);
    if (i > 0) ld4f(c0 - sx, h.xm); else for (int m = 0; m < 4; ++m) h.xm[m] = ghost;
    if (i < nx - 1) ld4f(c0 + sx, h.xp); else for (int m = 0; m < 4; ++m) h.xp[m] = ghost;
    if (j > 0) ld4f(c0 - sy, h.ym); else for (int m = 0; m < 4; ++m) h.ym[m] = ghost;
    if (j < ny - 1) ld4f(c0 + sy, h.yp); else for (int m = 0; m < 4; ++m) h.yp[m] = ghost;
    h.zl = k0 > 0 ? ld1f(c0 - 1) : ghost;
    h.zr = k0 + 4 < nz ? ld1f(c0 + 4) : ghost;
}

// Face coefficients of the four cells of a quad from cell coefficients
// (finest level): F = (D_p + D_s)/2, ghost coefficient dghost or (mirror) D_p.
// Order of the six faces: x-, x+, y-, y+, z-, z+.
template <typename V>
__device__ inline void quad_faces(const Hood<V> &D, int i, int j, int k0, int nx, int ny, int nz,
                                  bool mirror, V dghost, int m, V F[6])
{
    const V Dc = D.c[m];
    const V gD = mirror ? Dc : dghost;
    F[0] = (V)0.5 * (Dc + (i > 0 ? D.xm[m] : gD));
    F[1] = (V)0.5 * (Dc + (i < nx - 1 ? D.xp[m] : gD));
    F[2] = (V)0.5 * (Dc + (j > 0 ? D.ym[m] : gD));
    F[3] = (V)0.5 * (Dc + (j < ny - 1 ? D.yp[m] : gD));
    F[4] = (V)0.5 * (Dc + (k0 + m > 0 ? D.zm(m) : gD));
    F[5] = (V)0.5 * (Dc + (k0 + m < nz - 1 ? D.zp(m) : gD));
}

// ---------------------------------------------------------------------------
// Flux limiters F(R), Sec. 4 Table 2.
// ---------------------------------------------------------------------------

// Levermore-Pomraning (coth R - 1/R)/R.  For R < 2 the subtraction cancels;
// there the value comes from the continued fraction of coth (Lambert):
// coth R - 1/R = R/(3 + R^2/(5 + R^2/(7 + ...))), so
// F = 1/(3 + R^2/(5 + ... + R^2/25)).  Its convergents P_m/Q_m follow the
// forward three-term recurrence X_m = (2m+3) X_{m-1} + R^2 X_{m-2} (all
// terms positive, hence stable), which leaves a single division.  Above
// R = 2, coth R = 1 + 2/expm1(2R).
__device__ inline double limiter_lp(double R)
{
    if (R < 2.0) {
        const double x = R * R;
        double p0 = 1.0, p1 = 3.0, q0 = 0.0, q1 = 1.0;
#pragma unroll
        for (int m = 1; m <= 11; ++m) {
            const double b = (double)(2 * m + 3);
            const double p2 = b * p1 + x * p0, q2 = b * q1 + x * q0;
            p0 = p1; p1 = p2; q0 = q1; q1 = q2;
        }
        return q1 / p1;
    }
    const double coth = 1.0 + 2.0 / expm1(2.0 * R);
    return (coth - 1.0 / R) / R;
}

__device__ inline double limiter(int kind, double R, double n)
{
    switch (kind) {
    case L_CDA:
        return 1.0 / 3.0;
    case L_LP:
        return limiter_lp(R);
    case L_SUM:
        return 1.0 / (3.0 + R);
    case L_MAX:
        return 1.0 / fmax(3.0, R);
    case L_KERSHAW:
        return 2.0 / (3.0 + sqrt(9.0 + 4.0 * R * R));
    default:  // Larsen-n, written so R^n cannot overflow
        if (R <= 3.0)
            return pow(pow(3.0, n) + pow(R, n), -1.0 / n);
        return (1.0 / R) * pow(1.0 + pow(3.0 / R, n), -1.0 / n);
    }
}

// ---------------------------------------------------------------------------
// Finest level (FP64 state)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock)
k_setup(Fine f, const Task *tasks, int ntasks, const double *sigma_t, const double *albedo,
        const double *Q, double sigma_eps, double aniso_g, double *partials, float *sa32,
        double *sa64s)
{
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        double acc = 0.0;
        const Dec dec(f.ny, f.nz);
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x) {
            const long long c = tk.start + q;
            // transport extinction (reduced by the anisotropy g, Sec. 7) for
            // D and the Knudsen number; absorption from the clamped sigma_t
            if (f.write_sighat)
                f.sig_hat[c] = fmax(sigma_t[c] * (1.0 - albedo[c] * aniso_g), sigma_eps);
            const double sa = (1.0 - albedo[c]) * fmax(sigma_t[c], sigma_eps);
            f.sa64[c] = sa;
            if (sa32 || sa64s) {
                long long o = c;
                if (f.split) {
                    int i, j, k;
                    dec(c, i, j, k);
                    o = sidx(c, (i + j + k) & 1);
                }
                if (sa32)
                    sa32[o] = (float)sa;
                else
                    sa64s[o] = sa;
            }
            const double jq = Q[c];
            f.j[c] = jq;
            acc += jq * jq;
        }
        acc = block_sum(acc);
        if (threadIdx.x == 0)
            partials[t] = acc;
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_init_phi(const Fine *fines, const Task *tasks, int ntasks, const double *scal, int zero_dirs)
{
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        const Fine &f = fines[tk.grid];
        const double v = f.eps * scal[f.prob * S_COUNT + S_JBAR] * f.h;
        const Dec dec(f.ny, f.nz);
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x) {
            const long long c = tk.start + q;
            f.phi[0][c] = v;
            if (f.Dtmp)
                f.D64[c] = f.eps * f.h;
            if (zero_dirs) {
                ((T *)f.p[0])[c] = (T)0;
                ((T *)f.p[1])[c] = (T)0;
                long long o = c;
                if (f.split) {
                    int i, j, k;
                    dec(c, i, j, k);
                    o = sidx(c, (i + j + k) & 1);
                }
                ((T *)f.b0[0])[o] = (T)0;
                ((T *)f.b0[1])[o] = (T)0;
            }
        }
    }
}

// F(R) of a limiter pass instance: LK < 0 any limiter, chosen per voxel grid
// at run time; LK = L_LP Levermore-Pomraning alone.  The LP instance leaves
// the other kinds' pow() out of the kernel, and with it about 40 VGPRs: four
// waves per SIMD instead of three, and a fifth less time per pass.
template <int LK>
__device__ inline double limiter_of(int kind, double R, double n)
{
    return LK == L_LP ? limiter_lp(R) : limiter(kind, R, n);
}

// Limiter pass: (optionally) phi <- phi + theta*p, then for every voxel the
// central-difference gradient, the guarded Knudsen number and
// D = F(R)/sig_hat (Sec. 5: grad_approx, knudsen_numerical, D_update).
// DIR < 0: the direction update decided by use_dir at run time; 0 / 1: fixed.
template <typename T, int SP, int LK, int DIR>
__device__ inline void limiter_tasks(const Fine *fines, const Task *tasks, int ntasks,
                                     const int *active, const double *scal, int src, int dst,
                                     int use_dir_arg, int dir_idx, int to_tmp)
{
    const bool use_dir = DIR < 0 ? use_dir_arg != 0 : DIR == 1;
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        const Fine &f = fines[tk.grid];
        const bool sp = layout_split<SP>(f.split);
        if (active && !active[f.prob])
            continue;
        const double *__restrict__ phi = f.phi[src];
        const T *__restrict__ dir = (const T *)f.p[dir_idx];
        const double *__restrict__ sig_hat = f.sig_hat;
        double *__restrict__ phi_out = f.phi[dst];
        // the smoother's copy of D: FP32 in the mixed form; in the FP64 form
        // a colour-split copy, or D64 itself when the level keeps natural order
        T *__restrict__ Dlo = (T *)f.D0;
        const bool put_lo = !to_tmp && (sizeof(T) == 4 || sp);
        const double theta = use_dir ? scal[f.prob * S_COUNT + S_THETA] : 0.0;
        const double floor_ = f.eps * scal[f.prob * S_COUNT + S_JBAR];
        const long long sx = (long long)f.ny * f.nz, sy = f.nz;
        double *__restrict__ Dout = to_tmp ? f.Dtmp : f.D64;
        const Dec dec(f.ny, f.nz);
        if ((f.nz & 3) == 0) {
            auto L4 = [&](long long x, double v[4]) {
                ld4(phi + x, v);
                if (use_dir) {
                    T pv[4];
                    ld4(dir + x, pv);
                    for (int m = 0; m < 4; ++m)
                        v[m] = v[m] + theta * (double)pv[m];
                }
            };
            auto L1 = [&](long long x) {
                double v = phi[x];
                if (use_dir)
                    v = v + theta * (double)dir[x];
                return v;
            };
            for (int q = threadIdx.x; q < (tk.count >> 2); q += blockDim.x) {
                const long long c0 = tk.start + 4 * (long long)q;
                int i, j, k0;
                dec(c0, i, j, k0);
                Hood<double> P;
                gather(P, L4, L1, c0, i, j, k0, f.nx, f.ny, f.nz, sx, sy, f.phi_b);
                double sh[4], Rq[4], Dq[4];
                T Dlq[4];
                ld4(sig_hat + c0, sh);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const double dx = P.xp[m] - P.xm[m], dy = P.yp[m] - P.ym[m];
                    const double dz = P.zp(m) - P.zm(m);
                    const double grad = sqrt(dx * dx + dy * dy + dz * dz) / (2.0 * f.h);
                    Rq[m] = fmax(grad, floor_) / fmax(sh[m] * P.c[m], floor_);
                }
                if (use_dir && dst != src)
                    st4(phi_out + c0, P.c);
                // one cell at a time: unrolling the four limiter evaluations
                // raises the register footprint and halves the occupancy
#pragma unroll 1
                for (int m = 0; m < 4; ++m) {
                    Dq[m] = limiter_of<LK>(f.limiter, Rq[m], f.larsen_n) / sh[m];
                    Dlq[m] = (T)Dq[m];
                }
                st4(Dout + c0, Dq);
                if (put_lo) {
                    if (sp)
                        st4s(Dlo, c0, (i + j) & 1, Dlq);
                    else
                        st4(Dlo + c0, Dlq);
                }
            }
            continue;
        }
#pragma unroll 2
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x) {
            const long long c = tk.start + q;
            int i, j, k;
            dec(c, i, j, k);
            auto val = [&](long long x) {
                double v = phi[x];
                if (use_dir)
                    v = v + theta * (double)dir[x];
                return v;
            };
            const double pc = val(c);
            const double xm = i > 0 ? val(c - sx) : f.phi_b;
            const double xp = i < f.nx - 1 ? val(c + sx) : f.phi_b;
            const double ym = j > 0 ? val(c - sy) : f.phi_b;
            const double yp = j < f.ny - 1 ? val(c + sy) : f.phi_b;
            const double zm = k > 0 ? val(c - 1) : f.phi_b;
            const double zp = k < f.nz - 1 ? val(c + 1) : f.phi_b;
            const double dx = xp - xm, dy = yp - ym, dz = zp - zm;
            const double grad = sqrt(dx * dx + dy * dy + dz * dz) / (2.0 * f.h);
            const double sh = sig_hat[c];
            const double R = fmax(grad, floor_) / fmax(sh * pc, floor_);
            const double D = limiter_of<LK>(f.limiter, R, f.larsen_n) / sh;
            Dout[c] = D;
            if (put_lo)
                Dlo[sp ? sidx(c, (i + j + k) & 1) : c] = (T)D;
            if (use_dir && dst != src)
                phi_out[c] = pc;
        }
    }
}

template <typename T, int SP>
__global__ void __launch_bounds__(kBlock)
k_limiter(const Fine *fines, const Task *tasks, int ntasks, const int *active, const double *scal,
          int src, int dst, int use_dir, int dir_idx, int to_tmp)
{
    limiter_tasks<T, SP, -1, -1>(fines, tasks, ntasks, active, scal, src, dst, use_dir, dir_idx,
                                 to_tmp);
}

// LP without the direction update (the first pass of a solve, and every pass
// under Anderson acceleration), and LP with it (conjugate-gradient steps)
template <typename T, int SP>
__global__ void __launch_bounds__(kBlock)
k_limiter_lp(const Fine *fines, const Task *tasks, int ntasks, const int *active,
             const double *scal, int src, int dst, int use_dir, int dir_idx, int to_tmp)
{
    limiter_tasks<T, SP, L_LP, 0>(fines, tasks, ntasks, active, scal, src, dst, 0, dir_idx,
                                  to_tmp);
}

template <typename T, int SP>
__global__ void __launch_bounds__(kBlock)
k_limiter_lp_dir(const Fine *fines, const Task *tasks, int ntasks, const int *active,
                 const double *scal, int src, int dst, int use_dir, int dir_idx, int to_tmp)
{
    limiter_tasks<T, SP, L_LP, 1>(fines, tasks, ntasks, active, scal, src, dst, 1, dir_idx,
                                  to_tmp);
}

// Residual of the discretised equation (LHS - RHS, Sec. 5 R_calc):
// r = (num - phi*den)/h^2, num = j h^2 + sum_s D_ps phi_s,
// den = sa h^2 + sum_s D_ps, D_ps = (D_p + D_s)/2.  Writes r in precision T
// as the V-cycle right-hand side and per-task partial sums of r^2.
template <typename T, int SP>
__global__ void __launch_bounds__(kBlock)
k_residual(const Fine *fines, const Task *tasks, int ntasks, const int *active, int src,
           int use_tmp, int b0_idx, double *r_out, double *partials)
{
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        const Fine &f = fines[tk.grid];
        const bool sp = layout_split<SP>(f.split);
        if (active && !active[f.prob]) {
            if (threadIdx.x == 0)
                partials[t] = 0.0;
            continue;
        }
        const double *__restrict__ phi = f.phi[src];
        const double *__restrict__ D = use_tmp ? f.Dtmp : f.D64;
        const double *__restrict__ jsrc = f.j;
        const double *__restrict__ sa = f.sa64;
        T *__restrict__ b0 = (T *)f.b0[b0_idx];
        const long long sx = (long long)f.ny * f.nz, sy = f.nz;
        double acc = 0.0;
        const Dec dec(f.ny, f.nz);
        if ((f.nz & 3) == 0) {
            auto P4 = [&](long long x, double v[4]) { ld4(phi + x, v); };
            auto P1 = [&](long long x) { return phi[x]; };
            auto D4 = [&](long long x, double v[4]) { ld4(D + x, v); };
            auto D1 = [&](long long x) { return D[x]; };
            for (int q = threadIdx.x; q < (tk.count >> 2); q += blockDim.x) {
                const long long c0 = tk.start + 4 * (long long)q;
                int i, j, k0;
                dec(c0, i, j, k0);
                Hood<double> P, Dh;
                gather(P, P4, P1, c0, i, j, k0, f.nx, f.ny, f.nz, sx, sy, f.phi_b);
                gather(Dh, D4, D1, c0, i, j, k0, f.nx, f.ny, f.nz, sx, sy, f.dghost);
                double jq[4], saq[4], rq[4];
                T bq[4];
                ld4(jsrc + c0, jq);
                ld4(sa + c0, saq);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    double F[6];
                    quad_faces(Dh, i, j, k0, f.nx, f.ny, f.nz, f.mirror != 0, f.dghost, m, F);
                    double num = jq[m] * f.h2;
                    double den = saq[m] * f.h2;
                    num = num + F[0] * P.xm[m]; den = den + F[0];
                    num = num + F[1] * P.xp[m]; den = den + F[1];
                    num = num + F[2] * P.ym[m]; den = den + F[2];
                    num = num + F[3] * P.yp[m]; den = den + F[3];
                    num = num + F[4] * P.zm(m); den = den + F[4];
                    num = num + F[5] * P.zp(m); den = den + F[5];
                    rq[m] = (num - P.c[m] * den) / f.h2;
                    bq[m] = (T)rq[m];
                    acc += rq[m] * rq[m];
                }
                if (sp)
                    st4s(b0, c0, (i + j) & 1, bq);
                else
                    st4(b0 + c0, bq);
                if (r_out)
                    st4(r_out + c0, rq);
            }
        } else
#pragma unroll 2
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x) {
            const long long c = tk.start + q;
            int i, j, k;
            dec(c, i, j, k);
            const double Dc = D[c];
            const double gD = f.mirror ? Dc : f.dghost;
            double num = jsrc[c] * f.h2;
            double den = sa[c] * f.h2;
            double F;
            F = 0.5 * (Dc + (i > 0 ? D[c - sx] : gD));
            num = num + F * (i > 0 ? phi[c - sx] : f.phi_b);
            den = den + F;
            F = 0.5 * (Dc + (i < f.nx - 1 ? D[c + sx] : gD));
            num = num + F * (i < f.nx - 1 ? phi[c + sx] : f.phi_b);
            den = den + F;
            F = 0.5 * (Dc + (j > 0 ? D[c - sy] : gD));
            num = num + F * (j > 0 ? phi[c - sy] : f.phi_b);
            den = den + F;
            F = 0.5 * (Dc + (j < f.ny - 1 ? D[c + sy] : gD));
            num = num + F * (j < f.ny - 1 ? phi[c + sy] : f.phi_b);
            den = den + F;
            F = 0.5 * (Dc + (k > 0 ? D[c - 1] : gD));
            num = num + F * (k > 0 ? phi[c - 1] : f.phi_b);
            den = den + F;
            F = 0.5 * (Dc + (k < f.nz - 1 ? D[c + 1] : gD));
            num = num + F * (k < f.nz - 1 ? phi[c + 1] : f.phi_b);
            den = den + F;
            const double r = (num - phi[c] * den) / f.h2;
            b0[sp ? sidx(c, (i + j + k) & 1) : c] = (T)r;
            if (r_out)
                r_out[c] = r;
            acc += r * r;
        }
        acc = block_sum(acc);
        if (threadIdx.x == 0)
            partials[t] = acc;
    }
}

// gamma = b0 . e and sigma = e . b0_prev (conjugate-gradient coefficients).
template <typename T, int SP>
__global__ void __launch_bounds__(kBlock)
k_npcg_dots(const Fine *fines, const Task *tasks, int ntasks, const int *active, int b0_idx,
            double *pg, double *ps)
{
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        const Fine &f = fines[tk.grid];
        const bool sp = layout_split<SP>(f.split);
        if (active && !active[f.prob])
            continue;
        const T *b = (const T *)f.b0[b0_idx];
        const T *bp = (const T *)f.b0[b0_idx ^ 1];
        const T *e = (const T *)f.e0;
        double g = 0.0, sg = 0.0;
        const Dec dec(f.ny, f.nz);
        if ((f.nz & 3) == 0) {
            for (int q = threadIdx.x; q < (tk.count >> 2); q += blockDim.x) {
                const long long c0 = tk.start + 4 * (long long)q;
                T eq[4], bq[4], bpq[4];
                if (sp) {
                    int i, j, k0;
                    dec(c0, i, j, k0);
                    const int q0 = (i + j) & 1;
                    ld4s(e, c0, q0, eq);
                    ld4s(b, c0, q0, bq);
                    ld4s(bp, c0, q0, bpq);
                } else {
                    ld4(e + c0, eq);
                    ld4(b + c0, bq);
                    ld4(bp + c0, bpq);
                }
                for (int m = 0; m < 4; ++m) {
                    const double ev = (double)eq[m];
                    g += (double)bq[m] * ev;
                    sg += ev * (double)bpq[m];
                }
            }
        } else
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x) {
            const long long c = tk.start + q;
            long long o = c;
            if (sp) {
                int i, j, k;
                dec(c, i, j, k);
                o = sidx(c, (i + j + k) & 1);
            }
            const double ev = (double)e[o];
            g += (double)b[o] * ev;
            sg += ev * (double)bp[o];
        }
        g = block_sum(g);
        sg = block_sum(sg);
        if (threadIdx.x == 0) {
            pg[t] = g;
            ps[t] = sg;
        }
    }
}

// Limiter and residual in one pass (Sec. 5: gradient, Knudsen number and
// D update, then the residual with those D).  A block marches along x through
// a tile of kLrTy rows by kLrTz cells along z, keeping four planes of phi
// (two-cell halo, ghosts phi_b) and three planes of D (one-cell halo) in LDS.
// Step x forms D(x+1) on the tile and its halo, then the residual of plane x
// from LDS; the global loads of the next step (phi(x+3), sig_hat(x+2)) and
// this step's j and sa are issued at its start, so their latency is spent
// under the arithmetic.  sig_hat of a plane waits in the LDS slot its D will
// take (each thread reads it and writes the D of the same cell).  Per cell the
// arithmetic and its order are those of k_limiter and k_residual, so D and r
// are identical to theirs; only the partial sums of r^2 (one per tile) are
// grouped differently.  A halo D is formed by every tile that needs it.
// Writes r and D in precision T (D also in FP64 when write_d64) for the
// tile's own cells.  Needs nz % 4 == 0.
constexpr int kLrTy = kLrTileRows, kLrTz = kLrTileCells;
constexpr int kLrThreads = kLrTy * kLrTz / 4;          // one quad per thread
constexpr int kLrPy = kLrTy + 4, kLrPz = kLrTz + 4;    // phi planes
constexpr int kLrDy = kLrTy + 2, kLrDz = kLrTz + 2;    // D planes
constexpr int kLrPf = (kLrPy * kLrPz + kLrThreads - 1) / kLrThreads;   // phi values per thread
constexpr int kLrSf = (kLrDy * kLrDz + kLrThreads - 1) / kLrThreads;   // sig_hat values

template <typename T, int SP>
__global__ void __launch_bounds__(kLrThreads)
k_lim_res(const Fine *fines, const LrTile *tiles, int ntiles, const int *active,
          const double *scal, int src, int b0_idx, int write_d64, double *partials)
{
    __shared__ double Pl[4][kLrPy * kLrPz];
    __shared__ double Dl[3][kLrDy * kLrDz];
    __shared__ double red[kLrThreads / kWave];
    const int tid = threadIdx.x;
    // Workgroups are dealt to the 8 XCDs in turn, so virtual block v runs on
    // XCD v % 8: tile (v % 8) * chunk + v / 8 gives each XCD a contiguous run
    // of tiles, whose halos then meet in that XCD's L2.
    const int chunk = (ntiles + 7) / 8;
    for (int v = blockIdx.x; v < 8 * chunk; v += gridDim.x) {
        const int t = (v & 7) * chunk + (v >> 3);
        if (t >= ntiles)
            continue;
        const LrTile tl = tiles[t];
        const Fine &f = fines[tl.prob];
        const bool sp = layout_split<SP>(f.split);
        if (active && !active[f.prob]) {
            if (tid == 0)
                partials[t] = 0.0;
            continue;
        }
        const int nx = f.nx, ny = f.ny, nz = f.nz;
        const long long sx = (long long)ny * nz, sy = nz;
        const double *__restrict__ phi = f.phi[src];
        const double *__restrict__ sig_hat = f.sig_hat;
        const double *__restrict__ sa = f.sa64;
        const double *__restrict__ jsrc = f.j;
        T *__restrict__ b0 = (T *)f.b0[b0_idx];
        T *__restrict__ Dlo = (T *)f.D0;       // as in k_limiter
        const bool put_lo = sizeof(T) == 4 || sp;
        double *__restrict__ D64 = f.D64;
        const double floor_ = f.eps * scal[f.prob * S_COUNT + S_JBAR];
        const double pb = f.phi_b;
        const int i0 = tl.i0, i1 = tl.i0 + tl.ni, j0 = tl.j0, k0 = tl.k0;
        // this thread's quad of the tile
        const int jj = tid / (kLrTz / 4), kq = 4 * (tid - jj * (kLrTz / 4));
        const int j = j0 + jj, kc = k0 + kq;
        const bool own = j < ny && kc < nz;
        double acc = 0.0;
        double pf[kLrPf], sf[kLrSf];

        // phi of plane pl (ghosts phi_b) into registers / their LDS slot
        auto fetch_phi = [&](int pl) {
            const bool in_x = pl >= 0 && pl < nx;
#pragma unroll
            for (int u = 0; u < kLrPf; ++u) {
                const int e = tid + u * kLrThreads;
                const int r = e / kLrPz, q = e - r * kLrPz;
                const int jy = j0 - 2 + r, kz = k0 - 2 + q;
                pf[u] = pb;
                if (e < kLrPy * kLrPz && in_x && jy >= 0 && jy < ny && kz >= 0 && kz < nz)
                    pf[u] = phi[(long long)pl * sx + (long long)jy * sy + kz];
            }
        };
        auto commit_phi = [&](int pl) {
            double *P = Pl[(pl + 4) & 3];
#pragma unroll
            for (int u = 0; u < kLrPf; ++u) {
                const int e = tid + u * kLrThreads;
                if (e < kLrPy * kLrPz)
                    P[e] = pf[u];
            }
        };
        // sig_hat of plane pl on the D region, into registers / the D slot
        auto fetch_sig = [&](int pl) {
            const bool in_x = pl >= 0 && pl < nx;
#pragma unroll
            for (int u = 0; u < kLrSf; ++u) {
                const int e = tid + u * kLrThreads;
                const int r = e / kLrDz, q = e - r * kLrDz;
                const int jy = j0 - 1 + r, kz = k0 - 1 + q;
                sf[u] = 1.0;
                if (e < kLrDy * kLrDz && in_x && jy >= 0 && jy < ny && kz >= 0 && kz < nz)
                    sf[u] = sig_hat[(long long)pl * sx + (long long)jy * sy + kz];
            }
        };
        auto commit_sig = [&](int pl) {
            double *Dd = Dl[(pl + 3) % 3];
#pragma unroll
            for (int u = 0; u < kLrSf; ++u) {
                const int e = tid + u * kLrThreads;
                if (e < kLrDy * kLrDz)
                    Dd[e] = sf[u];
            }
        };
        // prologue: phi(i0-2 .. i0) and sig_hat(i0-1)
        fetch_phi(i0 - 2);
        commit_phi(i0 - 2);
        fetch_phi(i0 - 1);
        commit_phi(i0 - 1);
        fetch_phi(i0);
        commit_phi(i0);
        fetch_sig(i0 - 1);
        commit_sig(i0 - 1);
        __syncthreads();
        for (int x = i0 - 2; x < i1; ++x) {
            // the next step's loads, and this step's j and sa
            const bool more = x + 1 < i1;
            if (more) {
                fetch_phi(x + 3);
                fetch_sig(x + 2);
            }
            const bool res = x >= i0 && own;
            const long long c0 = (long long)(res ? x : 0) * sx + (long long)j * sy + kc;
            double jq[4], saq[4];
            if (res) {
                ld4(jsrc + c0, jq);
                ld4(sa + c0, saq);
            }
            // D of plane x+1 on the tile and its halo (sig_hat waits in its slot)
            const int pd = x + 1;
            if (pd >= 0 && pd < nx && pd <= i1) {
                const double *Pm = Pl[(pd + 3) & 3], *Pc = Pl[(pd + 4) & 3];
                const double *Pp = Pl[(pd + 5) & 3];
                double *Dd = Dl[(pd + 3) % 3];
                for (int e = tid; e < kLrDy * kLrDz; e += kLrThreads) {
                    const int r = e / kLrDz, q = e - r * kLrDz;
                    const int jy = j0 - 1 + r, kz = k0 - 1 + q;
                    if (jy < 0 || jy >= ny || kz < 0 || kz >= nz)
                        continue;
                    const int pc = (r + 1) * kLrPz + (q + 1);
                    const double dx = Pp[pc] - Pm[pc], dy = Pc[pc + kLrPz] - Pc[pc - kLrPz];
                    const double dz = Pc[pc + 1] - Pc[pc - 1];
                    const double grad = sqrt(dx * dx + dy * dy + dz * dz) / (2.0 * f.h);
                    const double sh = Dd[e];
                    const double R = fmax(grad, floor_) / fmax(sh * Pc[pc], floor_);
                    Dd[e] = limiter(f.limiter, R, f.larsen_n) / sh;
                }
            }
            __syncthreads();
            // residual of plane x
            if (res) {
                const double *Pm = Pl[(x + 3) & 3], *Pc = Pl[(x + 4) & 3];
                const double *Pp = Pl[(x + 5) & 3];
                const double *Dm = Dl[(x + 2) % 3], *Dc_ = Dl[(x + 3) % 3];
                const double *Dp = Dl[(x + 4) % 3];
                double rq[4], dq[4];
                T bq[4], dlo[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int k = kc + m;
                    const int pc = (jj + 2) * kLrPz + (kq + m + 2);
                    const int dc = (jj + 1) * kLrDz + (kq + m + 1);
                    const double Dcv = Dc_[dc];
                    const double gD = f.mirror ? Dcv : f.dghost;
                    double F[6];
                    F[0] = 0.5 * (Dcv + (x > 0 ? Dm[dc] : gD));
                    F[1] = 0.5 * (Dcv + (x < nx - 1 ? Dp[dc] : gD));
                    F[2] = 0.5 * (Dcv + (j > 0 ? Dc_[dc - kLrDz] : gD));
                    F[3] = 0.5 * (Dcv + (j < ny - 1 ? Dc_[dc + kLrDz] : gD));
                    F[4] = 0.5 * (Dcv + (k > 0 ? Dc_[dc - 1] : gD));
                    F[5] = 0.5 * (Dcv + (k < nz - 1 ? Dc_[dc + 1] : gD));
                    double num = jq[m] * f.h2;
                    double den = saq[m] * f.h2;
                    num = num + F[0] * Pm[pc]; den = den + F[0];
                    num = num + F[1] * Pp[pc]; den = den + F[1];
                    num = num + F[2] * Pc[pc - kLrPz]; den = den + F[2];
                    num = num + F[3] * Pc[pc + kLrPz]; den = den + F[3];
                    num = num + F[4] * Pc[pc - 1]; den = den + F[4];
                    num = num + F[5] * Pc[pc + 1]; den = den + F[5];
                    rq[m] = (num - Pc[pc] * den) / f.h2;
                    bq[m] = (T)rq[m];
                    acc += rq[m] * rq[m];
                    dq[m] = Dcv;
                    dlo[m] = (T)Dcv;
                }
                const int q0 = (x + j) & 1;
                if (sp)
                    st4s(b0, c0, q0, bq);
                else
                    st4(b0 + c0, bq);
                if (put_lo) {
                    if (sp)
                        st4s(Dlo, c0, q0, dlo);
                    else
                        st4(Dlo + c0, dlo);
                }
                if (write_d64)
                    st4(D64 + c0, dq);
            }
            __syncthreads();
            // phi(x+3) into the slot of phi(x-1), sig_hat(x+2) into that of D(x-1)
            if (more) {
                commit_phi(x + 3);
                commit_sig(x + 2);
            }
            __syncthreads();
        }
        // the tile's partial sum of r^2: wave shuffles, then the waves in order
        for (int o = kWave / 2; o > 0; o >>= 1)
            acc += __shfl_down(acc, o, kWave);
        if ((tid & (kWave - 1)) == 0)
            red[tid / kWave] = acc;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < kLrThreads / kWave; ++w)
                s += red[w];
            partials[t] = s;
        }
        __syncthreads();
    }
}

// p_new = e + beta p_old (stored in precision T) and the partial sums of
// r . p_new and p_new . A(D) p_new with the FP64 finest operator
// (A x)_c = (x_c den - sum_s D_ps x_s)/h^2, zero ghosts.
template <typename T, int SP>
__global__ void __launch_bounds__(kBlock)
k_npcg_dir(const Fine *fines, const Task *tasks, int ntasks, const int *active, const double *scal,
           int b0_idx, int pin, int pout, double *prp, double *ppap)
{
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        const Fine &f = fines[tk.grid];
        const bool sp = layout_split<SP>(f.split);
        if (active && !active[f.prob])
            continue;
        const T *__restrict__ e = (const T *)f.e0;
        const T *__restrict__ po = (const T *)f.p[pin];
        T *__restrict__ pn = (T *)f.p[pout];
        const T *__restrict__ b = (const T *)f.b0[b0_idx];
        const double *__restrict__ D = f.D64;
        const double *__restrict__ sa = f.sa64;
        const double beta = scal[f.prob * S_COUNT + S_BETA];
        const long long sx = (long long)f.ny * f.nz, sy = f.nz;
        double arp = 0.0, apap = 0.0;
        const Dec dec(f.ny, f.nz);
        if ((f.nz & 3) == 0) {
            QuadSrc<T> Es{e, 0, 0, sp};
            auto P4 = [&](long long x, double v[4]) {
                T ev[4], pv[4];
                Es.quad(x, ev);
                ld4(po + x, pv);
                for (int m = 0; m < 4; ++m)
                    v[m] = (double)(T)((double)ev[m] + beta * (double)pv[m]);
            };
            auto P1 = [&](long long x) {
                return (double)(T)((double)Es.one(x) + beta * (double)po[x]);
            };
            auto D4 = [&](long long x, double v[4]) { ld4(D + x, v); };
            auto D1 = [&](long long x) { return D[x]; };
            for (int q = threadIdx.x; q < (tk.count >> 2); q += blockDim.x) {
                const long long c0 = tk.start + 4 * (long long)q;
                int i, j, k0;
                dec(c0, i, j, k0);
                Es.c0 = c0;
                Es.q0 = (i + j) & 1;
                Hood<double> P, Dh;
                gather(P, P4, P1, c0, i, j, k0, f.nx, f.ny, f.nz, sx, sy, 0.0);
                gather(Dh, D4, D1, c0, i, j, k0, f.nx, f.ny, f.nz, sx, sy, f.dghost);
                double saq[4];
                T bq[4], pq[4];
                ld4(sa + c0, saq);
                if (sp)
                    ld4s(b, c0, Es.q0, bq);
                else
                    ld4(b + c0, bq);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    double F[6];
                    quad_faces(Dh, i, j, k0, f.nx, f.ny, f.nz, f.mirror != 0, f.dghost, m, F);
                    double nb = 0.0;
                    double den = saq[m] * f.h2;
                    nb = nb + F[0] * P.xm[m]; den = den + F[0];
                    nb = nb + F[1] * P.xp[m]; den = den + F[1];
                    nb = nb + F[2] * P.ym[m]; den = den + F[2];
                    nb = nb + F[3] * P.yp[m]; den = den + F[3];
                    nb = nb + F[4] * P.zm(m); den = den + F[4];
                    nb = nb + F[5] * P.zp(m); den = den + F[5];
                    const double pc = P.c[m];
                    const double Ap = (pc * den - nb) / f.h2;
                    pq[m] = (T)pc;
                    arp += (double)bq[m] * pc;
                    apap += pc * Ap;
                }
                st4(pn + c0, pq);
            }
        } else
#pragma unroll 2
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x) {
            const long long c = tk.start + q;
            int i, j, k;
            dec(c, i, j, k);
            const int qc = (i + j + k) & 1;
            auto eat = [&](long long x) {
                return sp ? e[sidx(x, x == c ? qc : qc ^ 1)] : e[x];
            };
            auto pv = [&](long long x) { return (double)(T)((double)eat(x) + beta * (double)po[x]); };
            const double Dc = D[c];
            const double gD = f.mirror ? Dc : f.dghost;
            const double pc = pv(c);
            double nb = 0.0;
            double den = sa[c] * f.h2;
            double F;
            F = 0.5 * (Dc + (i > 0 ? D[c - sx] : gD));
            nb = nb + F * (i > 0 ? pv(c - sx) : 0.0);
            den = den + F;
            F = 0.5 * (Dc + (i < f.nx - 1 ? D[c + sx] : gD));
            nb = nb + F * (i < f.nx - 1 ? pv(c + sx) : 0.0);
            den = den + F;
            F = 0.5 * (Dc + (j > 0 ? D[c - sy] : gD));
            nb = nb + F * (j > 0 ? pv(c - sy) : 0.0);
            den = den + F;
            F = 0.5 * (Dc + (j < f.ny - 1 ? D[c + sy] : gD));
            nb = nb + F * (j < f.ny - 1 ? pv(c + sy) : 0.0);
            den = den + F;
            F = 0.5 * (Dc + (k > 0 ? D[c - 1] : gD));
            nb = nb + F * (k > 0 ? pv(c - 1) : 0.0);
            den = den + F;
            F = 0.5 * (Dc + (k < f.nz - 1 ? D[c + 1] : gD));
            nb = nb + F * (k < f.nz - 1 ? pv(c + 1) : 0.0);
            den = den + F;
            const double Ap = (pc * den - nb) / f.h2;
            pn[c] = (T)pc;
            arp += (double)b[sp ? sidx(c, qc) : c] * pc;
            apap += pc * Ap;
        }
        arp = block_sum(arp);
        apap = block_sum(apap);
        if (threadIdx.x == 0) {
            prp[t] = arp;
            ppap[t] = apap;
        }
    }
}

// Cluster deflation, reductions.  The cluster Galerkin diagonal is
// d_c = sum_{p in c} sa_p + sum_{faces leaving c} F/h^2 and the right-hand
// side sum s_c = sum_{p in c} b0_p.  The absorption sum depends on the medium
// only and is formed once (k_defl_sum_sa); per outer iteration one pass sums
// b0 over the cluster cells, read at their precomputed storage positions
// (k_defl_sum_b), and one pass over the rim cells (cells with a face leaving
// their cluster) sums the face terms from the current coefficients
// (k_defl_rim).  A task covers cells (or rim cells) of one cluster; each
// writes one partial.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_defl_sum_sa(const Fine *fines, const CTask *ct, int nct, double *psa)
{
    for (int t = blockIdx.x; t < nct; t += gridDim.x) {
        const CTask tk = ct[t];
        const Fine &f = fines[tk.prob];
        const T *sa = (const T *)f.sa0;
        double acc = 0.0;
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x)
            acc += (double)sa[f.cpos[tk.start + q]];
        acc = block_sum(acc);
        if (threadIdx.x == 0)
            psa[t] = acc;
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_defl_sum_b(const Fine *fines, const CTask *ct, int nct, const int *active, int b0_idx, double *ps)
{
    for (int t = blockIdx.x; t < nct; t += gridDim.x) {
        const CTask tk = ct[t];
        const Fine &f = fines[tk.prob];
        if (active && !active[f.prob]) {
            if (threadIdx.x == 0)
                ps[t] = 0.0;
            continue;
        }
        const T *__restrict__ b = (const T *)f.b0[b0_idx];
        const int *__restrict__ pos = f.cpos + tk.start;
        double acc = 0.0;
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x)
            acc += (double)b[pos[q]];
        acc = block_sum(acc);
        if (threadIdx.x == 0)
            ps[t] = acc;
    }
}

template <typename T, int SP>
__global__ void __launch_bounds__(kBlock)
k_defl_rim(const Fine *fines, const CTask *rt, int nrt, const int *active, double *pd)
{
    for (int t = blockIdx.x; t < nrt; t += gridDim.x) {
        const CTask tk = rt[t];
        const Fine &f = fines[tk.prob];
        const bool sp = layout_split<SP>(f.split);
        if (active && !active[f.prob]) {
            if (threadIdx.x == 0)
                pd[t] = 0.0;
            continue;
        }
        const T *D = (const T *)f.D0;
        const long long sx = (long long)f.ny * f.nz, sy = f.nz;
        const double gD0 = (double)(T)f.dghost;
        const Dec dec(f.ny, f.nz);
        double ad = 0.0;
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x) {
            const long long c = f.rcells[tk.start + q];
            const int mask = f.rmask[tk.start + q];
            int qc = 0;
            if (sp) {
                int i, j, k;
                dec(c, i, j, k);
                qc = (i + j + k) & 1;
            }
            auto at = [&](long long x, int qq) { return sp ? sidx(x, qq) : x; };
            // faces leaving the cluster: bit s set for neighbour s (x-, x+,
            // y-, y+, z-, z+); bit s+6 set when it is a ghost
            const double Dc = (double)D[at(c, qc)];
            const double gD = f.mirror ? Dc : gD0;
            const long long off[6] = {-sx, sx, -sy, sy, -1, 1};
            double v = 0.0;
#pragma unroll
            for (int d = 0; d < 6; ++d)
                if (mask & (1 << d)) {
                    const bool ghost = (mask >> (d + 6)) & 1;
                    const double F = 0.5 * (Dc + (ghost ? gD : (double)D[at(c + off[d], qc ^ 1)]));
                    v = v + F / f.h2;
                }
            ad += v;
        }
        ad = block_sum(ad);
        if (threadIdx.x == 0)
            pd[t] = ad;
    }
}

// Per cluster: the sum of the partials of its cell tasks (range crange) and
// of its rim tasks (range rrange), one block per cluster.  With sa_only the
// cell partials are the absorption sums and go to csa; otherwise
// alpha_c = s_c / (csa_c + rim_c).
__global__ void __launch_bounds__(kBlock)
k_defl_finish(const int *crange, const int *rrange, const int *cprob, const double *ps,
              const double *pd, double *csa, double *alpha, const int *active, int sa_only)
{
    const int c = blockIdx.x;
    if (active && !active[cprob[c]])
        return;
    double sum = 0.0, rim = 0.0;
    for (int q = crange[c] + threadIdx.x; q < crange[c + 1]; q += blockDim.x)
        sum += ps[q];
    sum = block_sum(sum);
    if (!sa_only) {
        for (int q = rrange[c] + threadIdx.x; q < rrange[c + 1]; q += blockDim.x)
            rim += pd[q];
        rim = block_sum(rim);
    }
    if (threadIdx.x == 0) {
        if (sa_only)
            csa[c] = sum;
        else
            alpha[c] = sum / (csa[c] + rim);
    }
}

// Cluster deflation step as the finest level's starting correction:
// e0 = alpha[label] (zero outside clusters).  The finest smoothing of the
// V-cycle starts from it with the undeflated right-hand side; every step of
// the cycle is affine in the correction and the right-hand side, so this is
// e1 plus a cycle from zero on b0 - A e1, without forming A e1.
template <typename T, int SP>
__global__ void __launch_bounds__(kBlock)
k_defl_init(const Fine *fines, const Task *tasks, int ntasks, const int *active,
            const double *alpha)
{
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        const Fine &f = fines[tk.grid];
        const bool sp = layout_split<SP>(f.split);
        if (active && !active[f.prob])
            continue;
        T *__restrict__ e = (T *)f.e0;
        const int *__restrict__ lab = f.label;
        const double *__restrict__ al = alpha + f.cbase;
        const Dec dec(f.ny, f.nz);
        if ((f.nz & 3) == 0) {
            for (int q = threadIdx.x; q < (tk.count >> 2); q += blockDim.x) {
                const long long c0 = tk.start + 4 * (long long)q;
                int l[4];
                ld4(lab + c0, l);
                T v[4];
                for (int m = 0; m < 4; ++m)
                    v[m] = l[m] >= 0 ? (T)al[l[m]] : (T)0;
                if (sp) {
                    int i, j, k0;
                    dec(c0, i, j, k0);
                    st4s(e, c0, (i + j) & 1, v);
                } else {
                    st4(e + c0, v);
                }
            }
            continue;
        }
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x) {
            const long long c = tk.start + q;
            long long o = c;
            if (sp) {
                int i, j, k;
                dec(c, i, j, k);
                o = sidx(c, (i + j + k) & 1);
            }
            const int l = lab[c];
            e[o] = l >= 0 ? (T)al[l] : (T)0;
        }
    }
}

// Grid sequencing: the medium of a 2:1 coarser grid from the finest
// level's set-up fields, and the coarse fluence back on the fine grid.
// Coarse cell C averages its 8 children: sigma_t = mean(sig_hat) (already at
// or above the floor, so the coarse set-up keeps it), Q = mean(j), and the
// albedo 1 - mean(sa)/mean(sig_hat) makes the coarse absorption the mean of
// the fine one.
__global__ void __launch_bounds__(kBlock)
k_nested_coarsen(const double *__restrict__ sig_hat, const double *__restrict__ sa,
                 const double *__restrict__ j, int nx, int ny, int nz, double *__restrict__ st_c,
                 double *__restrict__ al_c, double *__restrict__ q_c)
{
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    const long long nc = (long long)cx * cy * cz;
    for (long long C = blockIdx.x * (long long)blockDim.x + threadIdx.x; C < nc;
         C += (long long)gridDim.x * blockDim.x) {
        const int K = (int)(C % cz), J = (int)((C / cz) % cy), I = (int)(C / ((long long)cy * cz));
        double s = 0.0, a = 0.0, q = 0.0;
        for (int di = 0; di < 2; ++di)
            for (int dj = 0; dj < 2; ++dj)
                for (int dk = 0; dk < 2; ++dk) {
                    const long long c =
                        ((long long)(2 * I + di) * ny + (2 * J + dj)) * nz + (2 * K + dk);
                    s = s + sig_hat[c];
                    a = a + sa[c];
                    q = q + j[c];
                }
        st_c[C] = s / 8.0;
        al_c[C] = s > 0.0 ? fmin(fmax(1.0 - a / s, 0.0), 1.0) : 0.0;
        q_c[C] = q / 8.0;
    }
}

__global__ void __launch_bounds__(kBlock)
k_nested_prolong(const double *__restrict__ phi_c, int nx, int ny, int nz,
                 double *__restrict__ phi)
{
    const long long n = (long long)nx * ny * nz;
    const int cy = ny / 2, cz = nz / 2;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(c % nz), jj = (int)((c / nz) % ny), i = (int)(c / ((long long)ny * nz));
        phi[c] = phi_c[((long long)(i / 2) * cy + jj / 2) * cz + k / 2];
    }
}

// Algorithm 1, one colour: per voxel Knudsen number from the current
// fluence, D_p update, face coefficients with the neighbours' stored D,
// residual with the pre-update phi_p, SOR blend of numerator/denominator.
// Voxels of one colour only read the other colour, so the pass is in place.
__global__ void __launch_bounds__(kBlock)
k_alg1_pass(const Fine *fines, const Task *tasks, int ntasks, const double *scal, int colour,
            double omega, double *partials)
{
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        const Fine &f = fines[tk.grid];
        double *phi = f.phi[0];
        double *D = f.D64;
        const double floor_ = f.eps * scal[f.prob * S_COUNT + S_JBAR];
        const long long sx = (long long)f.ny * f.nz, sy = f.nz;
        double acc = 0.0;
        const Dec dec(f.ny, f.nz);
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x) {
            const long long c = tk.start + q;
            int i, j, k;
            dec(c, i, j, k);
            if (((i + j + k) & 1) != colour)
                continue;
            const double pc = phi[c];
            const double xm = i > 0 ? phi[c - sx] : f.phi_b;
            const double xp = i < f.nx - 1 ? phi[c + sx] : f.phi_b;
            const double ym = j > 0 ? phi[c - sy] : f.phi_b;
            const double yp = j < f.ny - 1 ? phi[c + sy] : f.phi_b;
            const double zm = k > 0 ? phi[c - 1] : f.phi_b;
            const double zp = k < f.nz - 1 ? phi[c + 1] : f.phi_b;
            const double dx = xp - xm, dy = yp - ym, dz = zp - zm;
            const double grad = sqrt(dx * dx + dy * dy + dz * dz) / (2.0 * f.h);
            const double sh = f.sig_hat[c];
            const double R = fmax(grad, floor_) / fmax(sh * pc, floor_);
            const double Dc = limiter(f.limiter, R, f.larsen_n) / sh;
            D[c] = Dc;
            const double gD = f.mirror ? Dc : f.dghost;
            double num = f.j[c] * f.h2;
            double den = f.sa64[c] * f.h2;
            double F;
            F = 0.5 * (Dc + (i > 0 ? D[c - sx] : gD));
            num = num + F * xm;
            den = den + F;
            F = 0.5 * (Dc + (i < f.nx - 1 ? D[c + sx] : gD));
            num = num + F * xp;
            den = den + F;
            F = 0.5 * (Dc + (j > 0 ? D[c - sy] : gD));
            num = num + F * ym;
            den = den + F;
            F = 0.5 * (Dc + (j < f.ny - 1 ? D[c + sy] : gD));
            num = num + F * yp;
            den = den + F;
            F = 0.5 * (Dc + (k > 0 ? D[c - 1] : gD));
            num = num + F * zm;
            den = den + F;
            F = 0.5 * (Dc + (k < f.nz - 1 ? D[c + 1] : gD));
            num = num + F * zp;
            den = den + F;
            const double Rp = (num - pc * den) / f.h2;
            phi[c] = omega * (num / den) + (1.0 - omega) * pc;
            acc += Rp * Rp;
        }
        acc = block_sum(acc);
        if (threadIdx.x == 0)
            partials[t] = acc;
    }
}

// Per-problem sum of task partials, range[p] .. range[p+1].
__global__ void __launch_bounds__(kBlock)
k_sum_partials(const int *range, const double *partials, double *scal, int slot, const int *active)
{
    const int p = blockIdx.x;
    if (active && !active[p])
        return;
    double acc = 0.0;
    for (int q = range[p] + threadIdx.x; q < range[p + 1]; q += blockDim.x)
        acc += partials[q];
    acc = block_sum(acc);
    if (threadIdx.x == 0)
        scal[p * S_COUNT + slot] = acc;
}

__global__ void k_after_setup(int nprob, const Fine *fines, double *scal)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob)
        return;
    double *s = scal + p * S_COUNT;
    s[S_JBAR] = sqrt(s[S_JN2] / (double)fines[p].n);
    s[S_JNORM] = sqrt(s[S_JN2]);
}

__global__ void k_rel(int nprob, double *scal, const int *active)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob || (active && !active[p]))
        return;
    double *s = scal + p * S_COUNT;
    s[S_REL] = sqrt(s[S_RES2]) / s[S_JNORM];
}

// Polak-Ribiere+ coefficient of the conjugate-gradient step, restarted
// (beta = 0) at the first iteration and after an iteration that raised the
// residual norm by more than the factor `growth` (<= 0: no restarts).
__global__ void k_npcg_beta(int nprob, double *scal, const int *active, int first, double growth)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob || (active && !active[p]))
        return;
    double *s = scal + p * S_COUNT;
    double beta = 0.0;
    const bool restart = growth > 0.0 && s[S_REL] > growth * s[S_REL_PREV];
    if (!first && !restart) {
        beta = (s[S_GAMMA] - s[S_SIGMA]) / s[S_GAMMA_PREV];
        if (!(beta > 0.0))
            beta = 0.0;
    }
    s[S_BETA] = beta;
    s[S_GAMMA_PREV] = s[S_GAMMA];
    s[S_REL_PREV] = s[S_REL];
}

__global__ void k_npcg_theta(int nprob, double *scal, const int *active)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob || (active && !active[p]))
        return;
    double *s = scal + p * S_COUNT;
    s[S_THETA] = s[S_RP] / s[S_PAP];
}

// ---------------------------------------------------------------------------
// Anderson acceleration of the outer iteration (window m): the preconditioned
// Picard map x -> g(x) = x + f(x), f = the V-cycle's correction e0 (deflation
// included).  The history lives in a ring of m+1 slots of precision-T vectors
// in natural order: dF_s = f_{i+1} - f_i, and dG_s = dX_s + dF_s with
// dX_s = x_{i+1} - x_i, so that the update
//   x_{k+1} = x_k + f_k - sum_s gamma_s (dX_s + dF_s)
// reads one history vector per slot.  Per problem a small state records the
// committed slots oldest first, the pending slot (whose dG slot holds the dX
// the last update wrote; the next dots pass adds dF to it), the Gram matrix
// G_st = dF_s . dF_t and the coefficients.  Per iteration:
//   k_aa_dots    dF_p = f - f_prev into the pending slot p, dG_p += dF_p,
//                f_prev = f, and per task (kAaTaskCells cells, so a thread
//                sums several quads before the reduction) the partials of
//                dF_p . dF_s and dF_s . f for every slot s (dF_p for s = p);
//   k_aa_sums    per problem those sums in task order;
//   k_aa_solve   commit p (dropping the oldest when m are held) or, after an
//                iteration that raised ||r|| by more than restart_growth,
//                clear the history; gamma from (G + lambda I) gamma = h by
//                Cholesky, lambda = reg trace(G)/count (a failed
//                factorisation clears the history); choose the next pending
//                slot;
//   k_aa_update  x_{k+1} = x_k + f - sum_s gamma_s dG_s, oldest slot first,
//                and dG of the pending slot = x_{k+1} - x_k.
// A thread handles four consecutive cells (16-byte loads) when nz % 4 == 0.
// ---------------------------------------------------------------------------
constexpr int kAaMax = 16;                // largest window
constexpr int kAaSlots = kAaMax + 1;
// history vectors whose loads a thread issues together, in the dot products
// and in the update (4 values each in registers): several loads in flight
// per wave instead of one
template <typename T>
constexpr int kAaGroup = sizeof(T) == 4 ? 8 : 4;

// per-problem state: ints [order(kAaSlots), count, pending, pending_valid]
// and doubles [G (kAaSlots^2), gamma, dots dF_p.dF_s, dots dF_s.f]
constexpr int kAaInts = kAaSlots + 3;
constexpr int kAaDbls = kAaSlots * kAaSlots + 3 * kAaSlots;

struct AaView {
    int *I;
    double *G, *gam, *dd, *hf;
    __device__ AaView(int *ints, double *dbls, int p)
        : I(ints + p * kAaInts), G(dbls + (long long)p * kAaDbls),
          gam(G + kAaSlots * kAaSlots), dd(gam + kAaSlots), hf(dd + kAaSlots) {}
    __device__ int &count() { return I[kAaSlots]; }
    __device__ int &pending() { return I[kAaSlots + 1]; }
    __device__ int &pvalid() { return I[kAaSlots + 2]; }
};

// f = e0 of a cell (colour-split or natural storage)
template <typename T>
__device__ inline double f_one(const Fine &f, bool sp, const Dec &dec, long long c)
{
    const T *e = (const T *)f.e0;
    if (!sp)
        return (double)e[c];
    int i, j, k;
    dec(c, i, j, k);
    return (double)e[sidx(c, (i + j + k) & 1)];
}

// f of the quad c0..c0+3 (c0 % 4 == 0)
template <typename T>
__device__ inline void f_quad(const Fine &f, bool sp, const Dec &dec, long long c0, T v[4])
{
    const T *e = (const T *)f.e0;
    if (!sp) {
        ld4(e + c0, v);
        return;
    }
    int i, j, k0;
    dec(c0, i, j, k0);
    ld4s(e, c0, (i + j) & 1, v);
}

template <typename T, int SP>
__global__ void __launch_bounds__(kBlock)
k_aa_dots(const Fine *fines, const Task *tasks, int ntasks, const int *active, int *aai,
          double *aad, int m, double *partials)
{
    const int W = m + 1;
    __shared__ double red[kBlock / kWave][2 * kAaSlots];
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        const Fine &f = fines[tk.grid];
        const bool sp = layout_split<SP>(f.split);
        if (active && !active[f.prob])
            continue;
        AaView A(aai, aad, f.prob);
        const int pnd = A.pending();
        const long long n = f.n;
        T *__restrict__ fprev = (T *)f.aa_fprev;
        T *__restrict__ dF = (T *)f.aa_dF;           // slot s at dF + s*n
        T *__restrict__ dGp = (T *)f.aa_dG + (long long)pnd * n;
        double g[kAaSlots], hs[kAaSlots];
#pragma unroll
        for (int s = 0; s < kAaSlots; ++s)
            g[s] = hs[s] = 0.0;
        const Dec dec(f.ny, f.nz);
        if ((f.nz & 3) == 0) {
            for (int q = threadIdx.x; q < (tk.count >> 2); q += blockDim.x) {
                const long long c0 = tk.start + 4 * (long long)q;
                T fv[4], fp[4], dn[4], gp[4];
                f_quad<T>(f, sp, dec, c0, fv);
                ld4(fprev + c0, fp);
                ld4(dGp + c0, gp);
                for (int a = 0; a < 4; ++a) {
                    dn[a] = (T)((double)fv[a] - (double)fp[a]);
                    gp[a] = (T)((double)gp[a] + (double)dn[a]);
                }
                st4(fprev + c0, fv);
                st4(dF + (long long)pnd * n + c0, dn);
                st4(dGp + c0, gp);
                // slots in groups whose loads are all issued before any is
                // consumed, so a wave keeps several history loads in flight
#pragma unroll
                for (int s0 = 0; s0 < kAaSlots; s0 += kAaGroup<T>) {
                    T v[kAaGroup<T>][4];
#pragma unroll
                    for (int u = 0; u < kAaGroup<T>; ++u) {
                        const int s = s0 + u;
                        if (s < kAaSlots && s < W && s != pnd)
                            ld4(dF + (long long)s * n + c0, v[u]);
                    }
#pragma unroll
                    for (int u = 0; u < kAaGroup<T>; ++u) {
                        const int s = s0 + u;
                        if (s < kAaSlots && s < W) {
                            if (s == pnd)
                                for (int a = 0; a < 4; ++a)
                                    v[u][a] = dn[a];
                            for (int a = 0; a < 4; ++a) {
                                g[s] += (double)dn[a] * (double)v[u][a];
                                hs[s] += (double)v[u][a] * (double)fv[a];
                            }
                        }
                    }
                }
            }
        } else {
            for (int q = threadIdx.x; q < tk.count; q += blockDim.x) {
                const long long c = tk.start + q;
                const double fv = f_one<T>(f, sp, dec, c);
                const T dnew = (T)(fv - (double)fprev[c]);
                fprev[c] = (T)fv;
                dF[(long long)pnd * n + c] = dnew;
                dGp[c] = (T)((double)dGp[c] + (double)dnew);
                const double dn = (double)dnew;
#pragma unroll
                for (int s = 0; s < kAaSlots; ++s) {
                    if (s < W) {
                        const double v = s == pnd ? dn : (double)dF[(long long)s * n + c];
                        g[s] += dn * v;
                        hs[s] += v * fv;
                    }
                }
            }
        }
        // all 2W sums in one pass: wave shuffles, then one LDS row per wave;
        // partials are stored value-major, partials[w * ntasks + t]
        const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
#pragma unroll
        for (int s = 0; s < kAaSlots; ++s) {
            if (s < W) {
                double a = g[s], b = hs[s];
                for (int o = kWave / 2; o > 0; o >>= 1) {
                    a += __shfl_down(a, o, kWave);
                    b += __shfl_down(b, o, kWave);
                }
                if (lane == 0) {
                    red[wv][s] = a;
                    red[wv][W + s] = b;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < 2 * W) {
            double acc = 0.0;
            for (int q = 0; q < kBlock / kWave; ++q)
                acc += red[q][threadIdx.x];
            partials[(long long)threadIdx.x * ntasks + t] = acc;
        }
        __syncthreads();
    }
}

// per problem: the sums of the 2(m+1) partials over its tasks, in a fixed
// order; one block per (value, problem)
__global__ void __launch_bounds__(kBlock)
k_aa_sums(const int *range, const double *partials, int ntasks, int *aai, double *aad, int m,
          const int *active)
{
    const int w = blockIdx.x, p = blockIdx.y;
    if (active && !active[p])
        return;
    const int W = m + 1;
    AaView A(aai, aad, p);
    const double *pw = partials + (long long)w * ntasks;
    double acc = 0.0;
    for (int q = range[p] + threadIdx.x; q < range[p + 1]; q += blockDim.x)
        acc += pw[q];
    acc = block_sum(acc);
    if (threadIdx.x == 0) {
        if (w < W)
            A.dd[w] = acc;
        else
            A.hf[w - W] = acc;
    }
}

// one 64-lane block per problem: the first lane commits the pending slot (or
// clears the history) and picks the next one; the Cholesky factorisation and
// the forward substitution run right-looking across the lanes, which keeps
// every entry's subtractions in the order of the column-by-column algorithm
// (q = 0, 1, ...); the backward substitution is the first lane's
__global__ void __launch_bounds__(kWave)
k_aa_solve(int nprob, double *scal, int *aai, double *aad, int m, double reg, double growth,
           const int *active)
{
    __shared__ double L[kAaMax * kAaMax];
    __shared__ double y[kAaMax];
    __shared__ double Gs[kAaSlots * kAaSlots], dds[kAaSlots], hfs[kAaSlots];
    __shared__ int order[kAaSlots];
    __shared__ int s_cnt;
    __shared__ double s_lambda;
    const int p = blockIdx.x;
    if (p >= nprob || (active && !active[p]))
        return;
    const int tid = threadIdx.x;
    AaView A(aai, aad, p);
    for (int q = tid; q < kAaSlots * kAaSlots; q += blockDim.x)
        Gs[q] = A.G[q];
    for (int q = tid; q < kAaSlots; q += blockDim.x) {
        dds[q] = A.dd[q];
        hfs[q] = A.hf[q];
        order[q] = A.I[q];
    }
    __syncthreads();
    double *sc = scal + p * S_COUNT;
    if (tid == 0) {
        int cnt = A.count();
        const int pnd = A.pending();
        if (A.pvalid()) {
            if (growth > 0.0 && sc[S_REL] > growth * sc[S_REL_PREV]) {
                cnt = 0;                                  // restart: clear the history
            } else {
                if (cnt == m) {                           // drop the oldest
                    for (int a = 0; a + 1 < cnt; ++a)
                        order[a] = order[a + 1];
                    --cnt;
                }
                order[cnt++] = pnd;
                for (int a = 0; a < cnt; ++a) {
                    const int s = order[a];
                    Gs[pnd * kAaSlots + s] = dds[s];
                    Gs[s * kAaSlots + pnd] = dds[s];
                    A.G[pnd * kAaSlots + s] = dds[s];
                    A.G[s * kAaSlots + pnd] = dds[s];
                }
            }
        }
        sc[S_REL_PREV] = sc[S_REL];
        for (int s = 0; s < kAaSlots; ++s)
            A.gam[s] = 0.0;
        double tr = 0.0;
        for (int a = 0; a < cnt; ++a)
            tr += Gs[order[a] * kAaSlots + order[a]];
        s_lambda = cnt > 0 ? reg * tr / (double)cnt : 0.0;
        s_cnt = cnt;
    }
    __syncthreads();
    int cnt = s_cnt;
    if (cnt > 0) {
        // (G + lambda I) gamma = h over the committed slots, oldest first
        const double lambda = s_lambda;
        for (int q = tid; q < cnt * cnt; q += blockDim.x) {
            const int a = q / cnt, b = q - a * cnt;
            const double g = Gs[order[a] * kAaSlots + order[b]];
            L[a * kAaMax + b] = a == b ? g + lambda : g;
        }
        __syncthreads();
        bool ok = true;
        for (int c = 0; c < cnt; ++c) {
            const double d = L[c * kAaMax + c];
            if (!(d > 0.0)) {              // the same value in every lane
                ok = false;
                break;
            }
            const double lcc = sqrt(d);
            __syncthreads();
            if (tid == 0)
                L[c * kAaMax + c] = lcc;
            for (int r = c + 1 + tid; r < cnt; r += blockDim.x)
                L[r * kAaMax + c] = L[r * kAaMax + c] / lcc;
            __syncthreads();
            // trailing update of the lower triangle: L[r][k] -= L[r][c] L[k][c]
            const int w = cnt - c - 1;
            for (int q = tid; q < w * w; q += blockDim.x) {
                const int r = c + 1 + q / w, k = c + 1 + q % w;
                if (k <= r)
                    L[r * kAaMax + k] = L[r * kAaMax + k] - L[r * kAaMax + c] * L[k * kAaMax + c];
            }
            __syncthreads();
        }
        if (ok) {
            for (int r = tid; r < cnt; r += blockDim.x)
                y[r] = hfs[order[r]];
            __syncthreads();
            for (int r = 0; r < cnt; ++r) {
                if (tid == 0)
                    y[r] = y[r] / L[r * kAaMax + r];
                __syncthreads();
                for (int q = r + 1 + tid; q < cnt; q += blockDim.x)
                    y[q] = y[q] - L[q * kAaMax + r] * y[r];
                __syncthreads();
            }
            if (tid == 0) {
                for (int r = cnt - 1; r >= 0; --r) {
                    double s = y[r];
                    int q = r + 1;
                    for (; q + 3 < cnt; q += 4) {
                        double w[4], v[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            w[u] = L[(q + u) * kAaMax + r];
                            v[u] = y[q + u];
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            s = s - w[u] * v[u];
                    }
                    for (; q < cnt; ++q)
                        s = s - L[q * kAaMax + r] * y[q];
                    y[r] = s / L[r * kAaMax + r];
                }
                for (int a = 0; a < cnt; ++a)
                    A.gam[order[a]] = y[a];
            }
        } else {
            cnt = 0;
        }
    }
    if (tid != 0)
        return;
    A.count() = cnt;
    for (int a = 0; a < cnt; ++a)
        A.I[a] = order[a];
    // the next pending slot: the lowest slot not in the history
    int nxt = 0;
    for (; nxt < m + 1; ++nxt) {
        bool used = false;
        for (int a = 0; a < cnt; ++a)
            used = used || order[a] == nxt;
        if (!used)
            break;
    }
    A.pending() = nxt;
    A.pvalid() = 1;
}

__global__ void k_aa_reset(int nprob, int *aai)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob)
        return;
    int *I = aai + p * kAaInts;
    I[kAaSlots] = 0;        // count
    I[kAaSlots + 1] = 0;    // pending slot
    I[kAaSlots + 2] = 0;    // nothing pending
}

template <typename T, int SP>
__global__ void __launch_bounds__(kBlock)
k_aa_update(const Fine *fines, const Task *tasks, int ntasks, const int *active, int *aai,
            double *aad, int src, int dst)
{
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        const Fine &f = fines[tk.grid];
        const bool sp = layout_split<SP>(f.split);
        if (active && !active[f.prob])
            continue;
        AaView A(aai, aad, f.prob);
        const int cnt = A.count(), pnd = A.pending();
        int ord[kAaMax];
        double gm[kAaMax];
        for (int a = 0; a < cnt; ++a) {
            ord[a] = A.I[a];
            gm[a] = A.gam[ord[a]];
        }
        const long long n = f.n;
        const double *__restrict__ x = f.phi[src];
        double *__restrict__ xo = f.phi[dst];
        const T *__restrict__ dG = (const T *)f.aa_dG;
        T *__restrict__ dGp = (T *)f.aa_dG + (long long)pnd * n;
        const Dec dec(f.ny, f.nz);
        if ((f.nz & 3) == 0) {
            for (int q = threadIdx.x; q < (tk.count >> 2); q += blockDim.x) {
                const long long c0 = tk.start + 4 * (long long)q;
                T fv[4], dx[4];
                double step[4], xv[4], xn[4];
                f_quad<T>(f, sp, dec, c0, fv);
                for (int a = 0; a < 4; ++a)
                    step[a] = (double)fv[a];
                // history slots oldest first, in groups whose loads are all
                // issued before any is consumed
#pragma unroll
                for (int a0 = 0; a0 < kAaMax; a0 += kAaGroup<T>) {
                    T v[kAaGroup<T>][4];
#pragma unroll
                    for (int u = 0; u < kAaGroup<T>; ++u)
                        if (a0 + u < kAaMax && a0 + u < cnt)
                            ld4(dG + (long long)ord[a0 + u] * n + c0, v[u]);
#pragma unroll
                    for (int u = 0; u < kAaGroup<T>; ++u)
                        if (a0 + u < kAaMax && a0 + u < cnt)
                            for (int b = 0; b < 4; ++b)
                                step[b] = step[b] - gm[a0 + u] * (double)v[u][b];
                }
                ld4(x + c0, xv);
                for (int b = 0; b < 4; ++b) {
                    xn[b] = xv[b] + step[b];
                    dx[b] = (T)(xn[b] - xv[b]);
                }
                st4(xo + c0, xn);
                st4(dGp + c0, dx);
            }
            continue;
        }
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x) {
            const long long c = tk.start + q;
            double step = f_one<T>(f, sp, dec, c);
            for (int a = 0; a < cnt; ++a)
                step = step - gm[a] * (double)dG[(long long)ord[a] * n + c];
            const double xv = x[c];
            const double xn = xv + step;
            xo[c] = xn;
            dGp[c] = (T)(xn - xv);
        }
    }
}

// ---------------------------------------------------------------------------
// Multigrid levels, precision T
// ---------------------------------------------------------------------------

__device__ inline long long fidx(const Grid &g, int i, int j, int k)
{
    return ((long long)i * (g.ny + 1) + j) * face_zstride(g.nz) + k;
}

// Face coefficient below cell (i,j,k) along axis ax (either side may be a
// ghost; i,j,k may equal n along ax).
// Storage index of cell (i, j, k) of a level (natural, or colour-split on a
// split finest level).
__device__ inline long long cell_at(const Grid &g, int i, int j, int k, bool sp)
{
    const long long c = ((long long)i * g.ny + j) * g.nz + k;
    return sp ? sidx(c, (i + j + k) & 1) : c;
}

template <typename T>
__device__ inline T face_below(const Grid &g, int ax, int i, int j, int k, bool sp = false)
{
    if (!g.fine) {
        const long long nf = (long long)(g.nx + 1) * (g.ny + 1) * face_zstride(g.nz);
        return ((const T *)g.f)[ax * nf + fidx(g, i, j, k)];
    }
    const T *D = (const T *)g.D;
    int li = i, lj = j, lk = k;
    if (ax == 0) li -= 1; else if (ax == 1) lj -= 1; else lk -= 1;
    const bool hi_in = i < g.nx && j < g.ny && k < g.nz;
    const bool lo_in = li >= 0 && lj >= 0 && lk >= 0;
    if (hi_in && lo_in)
        return (T)0.5 * (D[cell_at(g, i, j, k, sp)] + D[cell_at(g, li, lj, lk, sp)]);
    const T Din = hi_in ? D[cell_at(g, i, j, k, sp)] : D[cell_at(g, li, lj, lk, sp)];
    return (T)0.5 * (Din + (g.mirror ? Din : (T)g.dghost));
}

// num = b h^2 + sum_s F_s e_s, den = sa h^2 + sum_s F_s (ghost e = 0),
// neighbours in the order x-, x+, y-, y+, z-, z+.  Finest level: faces from
// the cell coefficients, (D_p + D_s)/2, ghost coefficient eps*h or D_p.
template <typename T>
__device__ inline void cell_num_den(const Grid &g, const T *e, long long c, int i,
                                    int j, int k, T &num, T &den)
{
    const T h2 = (T)g.h2;
    const T *__restrict__ D = (const T *)g.D;
    const long long sx = (long long)g.ny * g.nz, sy = g.nz;
    // storage index of the cell / of a neighbour (the other colour)
    const int qc = (i + j + k) & 1;
    const long long oc = g.split ? sidx(c, qc) : c;
    auto at = [&](long long x) { return g.split ? sidx(x, qc ^ 1) : x; };
    const T Dc = D[oc];
    const T gD = g.mirror ? Dc : (T)g.dghost;
    T n_ = ((const T *)g.b)[oc] * h2;
    T d_ = ((const T *)g.sa)[oc] * h2;
    T F;
    F = (T)0.5 * (Dc + (i > 0 ? D[at(c - sx)] : gD));
    n_ = n_ + F * (i > 0 ? e[at(c - sx)] : (T)0);
    d_ = d_ + F;
    F = (T)0.5 * (Dc + (i < g.nx - 1 ? D[at(c + sx)] : gD));
    n_ = n_ + F * (i < g.nx - 1 ? e[at(c + sx)] : (T)0);
    d_ = d_ + F;
    F = (T)0.5 * (Dc + (j > 0 ? D[at(c - sy)] : gD));
    n_ = n_ + F * (j > 0 ? e[at(c - sy)] : (T)0);
    d_ = d_ + F;
    F = (T)0.5 * (Dc + (j < g.ny - 1 ? D[at(c + sy)] : gD));
    n_ = n_ + F * (j < g.ny - 1 ? e[at(c + sy)] : (T)0);
    d_ = d_ + F;
    F = (T)0.5 * (Dc + (k > 0 ? D[at(c - 1)] : gD));
    n_ = n_ + F * (k > 0 ? e[at(c - 1)] : (T)0);
    d_ = d_ + F;
    F = (T)0.5 * (Dc + (k < g.nz - 1 ? D[at(c + 1)] : gD));
    n_ = n_ + F * (k < g.nz - 1 ? e[at(c + 1)] : (T)0);
    d_ = d_ + F;
    num = n_;
    den = d_;
}

// Coarse level: Galerkin face coefficients f[axis] on the padded grid.
template <typename T>
__device__ inline void face_num_den(const Grid &g, const T *e, long long c, int i,
                                    int j, int k, T &num, T &den)
{
    const T h2 = (T)g.h2;
    const long long sx = (long long)g.ny * g.nz, sy = g.nz;
    const long long fy = face_zstride(g.nz), fx = (long long)(g.ny + 1) * fy;
    const long long nf = (long long)(g.nx + 1) * fx;
    const long long fi = (long long)i * fx + (long long)j * fy + k;
    const T *__restrict__ Fx = (const T *)g.f;
    const T *__restrict__ Fy = Fx + nf;
    const T *__restrict__ Fz = Fy + nf;
    T n_ = ((const T *)g.b)[c] * h2;
    T d_ = ((const T *)g.sa)[c] * h2;
    T F;
    F = Fx[fi];
    n_ = n_ + F * (i > 0 ? e[c - sx] : (T)0);
    d_ = d_ + F;
    F = Fx[fi + fx];
    n_ = n_ + F * (i < g.nx - 1 ? e[c + sx] : (T)0);
    d_ = d_ + F;
    F = Fy[fi];
    n_ = n_ + F * (j > 0 ? e[c - sy] : (T)0);
    d_ = d_ + F;
    F = Fy[fi + fy];
    n_ = n_ + F * (j < g.ny - 1 ? e[c + sy] : (T)0);
    d_ = d_ + F;
    F = Fz[fi];
    n_ = n_ + F * (k > 0 ? e[c - 1] : (T)0);
    d_ = d_ + F;
    F = Fz[fi + 1];
    n_ = n_ + F * (k < g.nz - 1 ? e[c + 1] : (T)0);
    d_ = d_ + F;
    num = n_;
    den = d_;
}

template <typename T>
__device__ inline void level_num_den(const Grid &g, const T *e, long long c, int i, int j, int k,
                                     T &num, T &den)
{
    if (g.fine)
        cell_num_den<T>(g, e, c, i, j, k, num, den);
    else
        face_num_den<T>(g, e, c, i, j, k, num, den);
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_zero(const Grid *grids, const Task *tasks, int ntasks, const int *active)
{
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        const Grid &g = grids[tk.grid];
        if (active && !active[g.prob])
            continue;
        T *e = (T *)g.e;
        if (g.split) {
            // the task's cells: compact run [start/2, (start+count)/2), both colours
            const long long m0 = tk.start >> 1;
            for (int q = threadIdx.x; q < (tk.count >> 1); q += blockDim.x) {
                e[cpos(m0 + q, 0)] = (T)0;
                e[cpos(m0 + q, 1)] = (T)0;
            }
            continue;
        }
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x)
            e[tk.start + q] = (T)0;
    }
}

// One red-black Gauss-Seidel half-sweep (in place: a colour reads only the
// other colour): e_p <- w num/den + (1-w) e_p.  Smoothed levels have even
// dimensions; a task's cells pair up along z and each thread updates the
// cell of the requested colour in its pair.
// Red-black half-sweep of the level smoother.  The finest level (cell D,
// face coefficients formed on the fly; FINE) and the coarse levels (stored
// Galerkin faces) are separate kernels, each compiled with its own paths only.
template <typename T, bool FINE>
__device__ __forceinline__ void smooth_task(const Grid &g, const Task tk, int colour, T omega)
{
    {
        T *e = (T *)g.e;
        const Dec dec(g.ny, g.nz);
        const int npairs = tk.count >> 1;
        if (FINE && g.split) {
            // colour-split finest level: the task's cells of this colour are
            // the compact run [start/2, (start+count)/2); a thread updates 4
            // of them (8 cells of one z row, k0 % 8 == 0), one 16-byte run of
            // each array.  Their x/y neighbours sit at the same compact places
            // of the other colour, their z neighbours one place to the left or
            // right.
            const T *__restrict__ Dall = (const T *)g.D;
            const T *__restrict__ bb = (const T *)g.b;
            const T *__restrict__ sa = (const T *)g.sa;
            const int oc = colour ^ 1;
            const long long hx = ((long long)g.ny * g.nz) >> 1, hy = g.nz >> 1;
            const T h2 = (T)g.h2;
            const T dgh = (T)g.dghost;
            const bool blend = omega != (T)1;
            for (int q = threadIdx.x; q < (tk.count >> 3); q += blockDim.x) {
                const long long c0 = tk.start + 8 * (long long)q;
                const long long m0 = c0 >> 1;
                int i, j, k0;
                dec(c0, i, j, k0);
                // this colour's cells: k = k0 + o + 2a, a = 0..3
                const int o = (colour ^ i ^ j) & 1;
                T X[4], DX[4], Dc[4], bq[4], saq[4];
                T xm[4] = {}, xp[4] = {}, ym[4] = {}, yp[4] = {}, own[4] = {};
                T Dxm[4] = {}, Dxp[4] = {}, Dym[4] = {}, Dyp[4] = {};
                const long long so = cpos(m0, colour), sx_ = cpos(m0, oc);
                ld4(e + sx_, X);
                ld4(Dall + sx_, DX);
                ld4(Dall + so, Dc);
                ld4(bb + so, bq);
                ld4(sa + so, saq);
                if (blend)
                    ld4(e + so, own);
                if (i > 0) {
                    const long long x = cpos(m0 - hx, oc);
                    ld4(e + x, xm);
                    ld4(Dall + x, Dxm);
                }
                if (i < g.nx - 1) {
                    const long long x = cpos(m0 + hx, oc);
                    ld4(e + x, xp);
                    ld4(Dall + x, Dxp);
                }
                if (j > 0) {
                    const long long x = cpos(m0 - hy, oc);
                    ld4(e + x, ym);
                    ld4(Dall + x, Dym);
                }
                if (j < g.ny - 1) {
                    const long long x = cpos(m0 + hy, oc);
                    ld4(e + x, yp);
                    ld4(Dall + x, Dyp);
                }
                // the z neighbour outside the loaded run: left (o = 0) or right
                T ez = (T)0, Dz = (T)0;
                if (o == 0 && k0 > 0) {
                    const long long x = cpos(m0 - 1, oc);
                    ez = e[x];
                    Dz = Dall[x];
                }
                if (o == 1 && k0 + 8 < g.nz) {
                    const long long x = cpos(m0 + 4, oc);
                    ez = e[x];
                    Dz = Dall[x];
                }
                T out[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int k = k0 + o + 2 * a;
                    const T Dp = Dc[a];
                    const T gD = g.mirror ? Dp : dgh;
                    T ezm, Dzm, ezp, Dzp;
                    if (o) {
                        ezm = X[a]; Dzm = DX[a];
                        ezp = a < 3 ? X[a + 1] : ez; Dzp = a < 3 ? DX[a + 1] : Dz;
                    } else {
                        ezm = a > 0 ? X[a - 1] : ez; Dzm = a > 0 ? DX[a - 1] : Dz;
                        ezp = X[a]; Dzp = DX[a];
                    }
                    T n_ = bq[a] * h2;
                    T d_ = saq[a] * h2;
                    T F;
                    F = (T)0.5 * (Dp + (i > 0 ? Dxm[a] : gD));
                    n_ = n_ + F * (i > 0 ? xm[a] : (T)0); d_ = d_ + F;
                    F = (T)0.5 * (Dp + (i < g.nx - 1 ? Dxp[a] : gD));
                    n_ = n_ + F * (i < g.nx - 1 ? xp[a] : (T)0); d_ = d_ + F;
                    F = (T)0.5 * (Dp + (j > 0 ? Dym[a] : gD));
                    n_ = n_ + F * (j > 0 ? ym[a] : (T)0); d_ = d_ + F;
                    F = (T)0.5 * (Dp + (j < g.ny - 1 ? Dyp[a] : gD));
                    n_ = n_ + F * (j < g.ny - 1 ? yp[a] : (T)0); d_ = d_ + F;
                    F = (T)0.5 * (Dp + (k > 0 ? Dzm : gD));
                    n_ = n_ + F * (k > 0 ? ezm : (T)0); d_ = d_ + F;
                    F = (T)0.5 * (Dp + (k < g.nz - 1 ? Dzp : gD));
                    n_ = n_ + F * (k < g.nz - 1 ? ezp : (T)0); d_ = d_ + F;
                    out[a] = omega * (n_ / d_) + ((T)1 - omega) * own[a];
                }
                st4(e + so, out);
            }
        } else if (FINE && (g.nz & 3) == 0) {
            const T *__restrict__ D = (const T *)g.D;
            const T *__restrict__ bb = (const T *)g.b;
            const T *__restrict__ sa = (const T *)g.sa;
            const long long sx = (long long)g.ny * g.nz, sy = g.nz;
            const T h2 = (T)g.h2;
            auto E4 = [&](long long x, T v[4]) { ld4(e + x, v); };
            auto E1 = [&](long long x) { return e[x]; };
            auto D4 = [&](long long x, T v[4]) { ld4(D + x, v); };
            auto D1 = [&](long long x) { return D[x]; };
            for (int q = threadIdx.x; q < (tk.count >> 2); q += blockDim.x) {
                const long long c0 = tk.start + 4 * (long long)q;
                int i, j, k0;
                dec(c0, i, j, k0);
                Hood<T> Eh, Dh;
                gather(Eh, E4, E1, c0, i, j, k0, g.nx, g.ny, g.nz, sx, sy, (T)0);
                gather(Dh, D4, D1, c0, i, j, k0, g.nx, g.ny, g.nz, sx, sy, (T)g.dghost);
                T bq[4], saq[4], out[4];
                ld4(bb + c0, bq);
                ld4(sa + c0, saq);
                const int first = (i + j + colour) & 1;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    out[m] = Eh.c[m];
                    if ((m & 1) != first)
                        continue;
                    T F[6];
                    quad_faces(Dh, i, j, k0, g.nx, g.ny, g.nz, g.mirror != 0, (T)g.dghost, m, F);
                    T n_ = bq[m] * h2;
                    T d_ = saq[m] * h2;
                    n_ = n_ + F[0] * Eh.xm[m]; d_ = d_ + F[0];
                    n_ = n_ + F[1] * Eh.xp[m]; d_ = d_ + F[1];
                    n_ = n_ + F[2] * Eh.ym[m]; d_ = d_ + F[2];
                    n_ = n_ + F[3] * Eh.yp[m]; d_ = d_ + F[3];
                    n_ = n_ + F[4] * Eh.zm(m); d_ = d_ + F[4];
                    n_ = n_ + F[5] * Eh.zp(m); d_ = d_ + F[5];
                    out[m] = omega * (n_ / d_) + ((T)1 - omega) * Eh.c[m];
                }
                st4(e + c0, out);
            }
        } else if (FINE) {
            for (int q = threadIdx.x; q < npairs; q += blockDim.x) {
                const long long c0 = tk.start + 2 * (long long)q;
                int i, j, k;
                dec(c0, i, j, k);
                const int odd = (i + j + colour) & 1;
                const long long c = c0 + odd;
                T num, den;
                cell_num_den<T>(g, e, c, i, j, k + odd, num, den);
                e[c] = omega * (num / den) + ((T)1 - omega) * e[c];
            }
        } else if ((g.nz & 3) == 0 && (tk.count & 3) == 0) {
            // coarse level, four cells along z per thread (two of this
            // colour): 16-byte loads of e, b, sa and of the x and y face
            // quads, the z faces as a quad plus one; per cell the arithmetic
            // and its order are those of face_num_den
            const T *__restrict__ bb = (const T *)g.b;
            const T *__restrict__ sa = (const T *)g.sa;
            const long long sx = (long long)g.ny * g.nz, sy = g.nz;
            const long long fy = face_zstride(g.nz), fx = (long long)(g.ny + 1) * fy;
            const long long nf = (long long)(g.nx + 1) * fx;
            const T *__restrict__ Fx = (const T *)g.f;
            const T *__restrict__ Fy = Fx + nf;
            const T *__restrict__ Fz = Fy + nf;
            const T h2 = (T)g.h2;
            auto E4 = [&](long long x, T v[4]) { ld4(e + x, v); };
            auto E1 = [&](long long x) { return e[x]; };
            for (int q = threadIdx.x; q < (tk.count >> 2); q += blockDim.x) {
                const long long c0 = tk.start + 4 * (long long)q;
                int i, j, k0;
                dec(c0, i, j, k0);
                Hood<T> Eh;
                gather(Eh, E4, E1, c0, i, j, k0, g.nx, g.ny, g.nz, sx, sy, (T)0);
                const long long fi = (long long)i * fx + (long long)j * fy + k0;
                T fxm[4], fxp[4], fym[4], fyp[4], fz[4], bq[4], saq[4], out[4];
                ld4(Fx + fi, fxm);
                ld4(Fx + fi + fx, fxp);
                ld4(Fy + fi, fym);
                ld4(Fy + fi + fy, fyp);
                ld4(Fz + fi, fz);
                const T fz4 = Fz[fi + 4];
                ld4(bb + c0, bq);
                ld4(sa + c0, saq);
                const int first = (i + j + colour) & 1;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    out[m] = Eh.c[m];
                    if ((m & 1) != first)
                        continue;
                    T n_ = bq[m] * h2;
                    T d_ = saq[m] * h2;
                    T F;
                    F = fxm[m];
                    n_ = n_ + F * Eh.xm[m];
                    d_ = d_ + F;
                    F = fxp[m];
                    n_ = n_ + F * Eh.xp[m];
                    d_ = d_ + F;
                    F = fym[m];
                    n_ = n_ + F * Eh.ym[m];
                    d_ = d_ + F;
                    F = fyp[m];
                    n_ = n_ + F * Eh.yp[m];
                    d_ = d_ + F;
                    F = fz[m];
                    n_ = n_ + F * Eh.zm(m);
                    d_ = d_ + F;
                    F = m < 3 ? fz[m + 1] : fz4;
                    n_ = n_ + F * Eh.zp(m);
                    d_ = d_ + F;
                    out[m] = omega * (n_ / d_) + ((T)1 - omega) * Eh.c[m];
                }
                st4(e + c0, out);
            }
        } else {
            for (int q = threadIdx.x; q < npairs; q += blockDim.x) {
                const long long c0 = tk.start + 2 * (long long)q;
                int i, j, k;
                dec(c0, i, j, k);
                const int odd = (i + j + colour) & 1;
                const long long c = c0 + odd;
                T num, den;
                face_num_den<T>(g, e, c, i, j, k + odd, num, den);
                e[c] = omega * (num / den) + ((T)1 - omega) * e[c];
            }
        }
    }
}

template <typename T, bool FINE>
__device__ __forceinline__ void smooth_tasks(const Grid *grids, const Task *tasks, int ntasks,
                                             const int *active, int colour, T omega)
{
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        const Grid &g = grids[tk.grid];
        if (active && !active[g.prob])
            continue;
        smooth_task<T, FINE>(g, tk, colour, omega);
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_smooth_fine(const Grid *grids, const Task *tasks, int ntasks, const int *active, int colour,
              T omega)
{
    smooth_tasks<T, true>(grids, tasks, ntasks, active, colour, omega);
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_smooth(const Grid *grids, const Task *tasks, int ntasks, const int *active, int colour, T omega)
{
    smooth_tasks<T, false>(grids, tasks, ntasks, active, colour, omega);
}

// The same half-sweep of one coarse level of a single problem, the level
// passed by value and block b taking cells [b * task_cells, ...): no task,
// grid or activity record to fetch before the cells' own loads, which is most
// of a small level's launch time.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_smooth_one(Grid g, int task_cells, int colour, T omega)
{
    const long long start = (long long)blockIdx.x * task_cells;
    const Task tk{0, (int)(g.n - start < task_cells ? g.n - start : task_cells), start};
    smooth_task<T, false>(g, tk, colour, omega);
}

// One red-black sweep of the finest level in a single pass, out of place
// (e -> e2 or back, dir): a block marches along x through a tile of kLrTy
// rows by kLrTz cells along z, keeping four planes of e and of D (two-cell
// halo) and two planes of b and sa (one-cell halo) in LDS.  Step x updates
// the first colour of plane x+1 on the tile and its halo, then the second
// colour of plane x on the tile, and stores plane x; the next planes' loads
// are issued at the start of the step.  Reading the old field only (the new
// one goes to the other buffer) makes a tile's halo independent of its
// neighbours' progress, so the result is the red and black half-sweeps'
// exactly: the same arithmetic per cell in the same order.  Each colour's new
// value is formed by every tile whose halo holds it; 20 bytes per cell of the
// grid move (e, D, b, sa read, e written) instead of 28 for two half-sweeps.
constexpr int kRbPf = (kLrPy * kLrPz + kLrThreads - 1) / kLrThreads;   // e, D per thread
constexpr int kRbBf = (kLrDy * kLrDz + kLrThreads - 1) / kLrThreads;   // b, sa per thread

template <typename T, int SP>
__global__ void __launch_bounds__(kLrThreads)
k_smooth_rb(const Grid *grids, const LrTile *tiles, int ntiles, const int *active, int first,
            int dir, T omega)
{
    __shared__ T El[4][kLrPy * kLrPz];
    __shared__ T Dl[4][kLrPy * kLrPz];
    __shared__ T Bl[2][kLrDy * kLrDz];
    __shared__ T Sl[2][kLrDy * kLrDz];
    const int tid = threadIdx.x;
    const int chunk = (ntiles + 7) / 8;       // tiles per XCD, as in k_lim_res
    for (int v = blockIdx.x; v < 8 * chunk; v += gridDim.x) {
        const int t = (v & 7) * chunk + (v >> 3);
        if (t >= ntiles)
            continue;
        const LrTile tl = tiles[t];
        const Grid &g = grids[tl.prob];
        if (active && !active[g.prob])
            continue;
        const bool sp = grid_split<SP>(g);
        const int nx = g.nx, ny = g.ny, nz = g.nz;
        const long long sx = (long long)ny * nz, sy = nz;
        const T *__restrict__ ein = (const T *)(dir ? g.e2 : g.e);
        T *__restrict__ eout = (T *)(dir ? g.e : g.e2);
        const T *__restrict__ Dg = (const T *)g.D;
        const T *__restrict__ bg = (const T *)g.b;
        const T *__restrict__ sg = (const T *)g.sa;
        const T h2 = (T)g.h2;
        const T dgh = (T)g.dghost;
        const int i0 = tl.i0, i1 = tl.i0 + tl.ni, j0 = tl.j0, k0 = tl.k0;
        auto at = [&](long long c, int q) { return sp ? sidx(c, q) : c; };
        T pe[kRbPf], pdv[kRbPf], pbv[kRbBf], psv[kRbBf];

        // e and D of plane pl on the two-cell halo region (ghost e = 0)
        auto fetch_ed = [&](int pl) {
            const bool in_x = pl >= 0 && pl < nx;
#pragma unroll
            for (int u = 0; u < kRbPf; ++u) {
                const int e = tid + u * kLrThreads;
                const int r = e / kLrPz, q = e - r * kLrPz;
                const int jy = j0 - 2 + r, kz = k0 - 2 + q;
                pe[u] = (T)0;
                pdv[u] = (T)0;
                if (e < kLrPy * kLrPz && in_x && jy >= 0 && jy < ny && kz >= 0 && kz < nz) {
                    const long long c = (long long)pl * sx + (long long)jy * sy + kz;
                    const long long o = at(c, (pl + jy + kz) & 1);
                    pe[u] = ein[o];
                    pdv[u] = Dg[o];
                }
            }
        };
        auto commit_ed = [&](int pl) {
            T *E = El[(pl + 4) & 3], *D = Dl[(pl + 4) & 3];
#pragma unroll
            for (int u = 0; u < kRbPf; ++u) {
                const int e = tid + u * kLrThreads;
                if (e < kLrPy * kLrPz) {
                    E[e] = pe[u];
                    D[e] = pdv[u];
                }
            }
        };
        // b and sa of plane pl on the one-cell halo region
        auto fetch_bs = [&](int pl) {
            const bool in_x = pl >= 0 && pl < nx;
#pragma unroll
            for (int u = 0; u < kRbBf; ++u) {
                const int e = tid + u * kLrThreads;
                const int r = e / kLrDz, q = e - r * kLrDz;
                const int jy = j0 - 1 + r, kz = k0 - 1 + q;
                pbv[u] = (T)0;
                psv[u] = (T)0;
                if (e < kLrDy * kLrDz && in_x && jy >= 0 && jy < ny && kz >= 0 && kz < nz) {
                    const long long c = (long long)pl * sx + (long long)jy * sy + kz;
                    const long long o = at(c, (pl + jy + kz) & 1);
                    pbv[u] = bg[o];
                    psv[u] = sg[o];
                }
            }
        };
        auto commit_bs = [&](int pl) {
            T *B = Bl[(pl + 2) & 1], *S = Sl[(pl + 2) & 1];
#pragma unroll
            for (int u = 0; u < kRbBf; ++u) {
                const int e = tid + u * kLrThreads;
                if (e < kLrDy * kLrDz) {
                    B[e] = pbv[u];
                    S[e] = psv[u];
                }
            }
        };
        // new value of cell (pl, jy, kz) of the region: the point update of the
        // half-sweep kernels, in their order (faces x-, x+, y-, y+, z-, z+)
        auto update = [&](int pl, int r, int q, int jy, int kz) {
            const T *Em = El[(pl + 3) & 3], *Ec = El[(pl + 4) & 3], *Ep = El[(pl + 5) & 3];
            const T *Dm = Dl[(pl + 3) & 3], *Dc = Dl[(pl + 4) & 3], *Dp = Dl[(pl + 5) & 3];
            const int pc = (r + 1) * kLrPz + (q + 1);          // in the e/D planes
            const int bc = r * kLrDz + q;                      // in the b/sa planes
            const T Dv = Dc[pc];
            const T gD = g.mirror ? Dv : dgh;
            T n_ = Bl[(pl + 2) & 1][bc] * h2;
            T d_ = Sl[(pl + 2) & 1][bc] * h2;
            T F;
            F = (T)0.5 * (Dv + (pl > 0 ? Dm[pc] : gD));
            n_ = n_ + F * (pl > 0 ? Em[pc] : (T)0); d_ = d_ + F;
            F = (T)0.5 * (Dv + (pl < nx - 1 ? Dp[pc] : gD));
            n_ = n_ + F * (pl < nx - 1 ? Ep[pc] : (T)0); d_ = d_ + F;
            F = (T)0.5 * (Dv + (jy > 0 ? Dc[pc - kLrPz] : gD));
            n_ = n_ + F * (jy > 0 ? Ec[pc - kLrPz] : (T)0); d_ = d_ + F;
            F = (T)0.5 * (Dv + (jy < ny - 1 ? Dc[pc + kLrPz] : gD));
            n_ = n_ + F * (jy < ny - 1 ? Ec[pc + kLrPz] : (T)0); d_ = d_ + F;
            F = (T)0.5 * (Dv + (kz > 0 ? Dc[pc - 1] : gD));
            n_ = n_ + F * (kz > 0 ? Ec[pc - 1] : (T)0); d_ = d_ + F;
            F = (T)0.5 * (Dv + (kz < nz - 1 ? Dc[pc + 1] : gD));
            n_ = n_ + F * (kz < nz - 1 ? Ec[pc + 1] : (T)0); d_ = d_ + F;
            return omega * (n_ / d_) + ((T)1 - omega) * Ec[pc];
        };

        // prologue: e, D of planes i0-2 .. i0, b, sa of plane i0-1
        fetch_ed(i0 - 2);
        commit_ed(i0 - 2);
        fetch_ed(i0 - 1);
        commit_ed(i0 - 1);
        fetch_ed(i0);
        commit_ed(i0);
        fetch_bs(i0 - 1);
        commit_bs(i0 - 1);
        __syncthreads();
        const int c2 = first ^ 1;
        for (int x = i0 - 2; x < i1; ++x) {
            const bool more = x + 1 < i1;
            if (more) {
                fetch_ed(x + 3);
                fetch_bs(x + 2);
            }
            // first colour on plane x+1, tile and halo
            const int pu = x + 1;
            if (pu >= 0 && pu < nx && pu <= i1) {
                T *Eu = El[(pu + 4) & 3];
                for (int e = tid; e < kLrDy * kLrDz; e += kLrThreads) {
                    const int r = e / kLrDz, q = e - r * kLrDz;
                    const int jy = j0 - 1 + r, kz = k0 - 1 + q;
                    if (jy < 0 || jy >= ny || kz < 0 || kz >= nz || ((pu + jy + kz) & 1) != first)
                        continue;
                    const T nv = update(pu, r, q, jy, kz);
                    Eu[(r + 1) * kLrPz + (q + 1)] = nv;
                }
            }
            __syncthreads();
            // second colour on plane x, the tile, then plane x stored
            if (x >= i0) {
                T *Ex = El[(x + 4) & 3];
                const int jj = tid / (kLrTz / 4), kq = 4 * (tid - jj * (kLrTz / 4));
                const int jy = j0 + jj, kc = k0 + kq;
                if (jy < ny && kc < nz) {
                    T nv[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int kz = kc + m;
                        nv[m] = ((x + jy + kz) & 1) == c2 ? update(x, jj + 1, kq + m + 1, jy, kz)
                                                           : (T)0;
                    }
                    T out[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int pc = (jj + 2) * kLrPz + (kq + m + 2);
                        out[m] = ((x + jy + kc + m) & 1) == c2 ? nv[m] : Ex[pc];
                    }
                    const long long c0 = (long long)x * sx + (long long)jy * sy + kc;
                    if (sp)
                        st4s(eout, c0, (x + jy) & 1, out);
                    else
                        st4(eout + c0, out);
                }
            }
            __syncthreads();
            if (more) {
                commit_ed(x + 3);
                commit_bs(x + 2);
            }
            __syncthreads();
        }
    }
}

// Coarse right-hand side = 8-child mean of the fine residual b - A e.
// Tasks run over the cells of the coarse grid.
template <typename T, int SP>
__global__ void __launch_bounds__(kBlock)
k_restrict(const Grid *grids, const Task *tasks, int ntasks, const int *active)
{
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        const Grid &C = grids[tk.grid];
        if (active && !active[C.prob])
            continue;
        const Grid &F = grids[C.finer];
        const bool sp = grid_split<SP>(F);
        const T *e = (const T *)F.e;
        T *bc = (T *)C.b;
        const T h2 = (T)F.h2;
        const Dec dec(C.ny, C.nz);
        if (F.fine && (F.nz & 3) == 0) {
            // two coarse cells along z per thread: their children form one fine
            // quad in each of the four (di, dj) rows
            const T *__restrict__ D = (const T *)F.D;
            const T *__restrict__ bf = (const T *)F.b;
            const T *__restrict__ sa = (const T *)F.sa;
            const long long sx = (long long)F.ny * F.nz, sy = F.nz;
                QuadSrc<T> Es{e, 0, 0, sp}, Ds{D, 0, 0, sp};
            auto E4 = [&](long long x, T v[4]) { Es.quad(x, v); };
            auto E1 = [&](long long x) { return Es.one(x); };
            auto D4 = [&](long long x, T v[4]) { Ds.quad(x, v); };
            auto D1 = [&](long long x) { return Ds.one(x); };
            for (int q = threadIdx.x; q < (tk.count >> 1); q += blockDim.x) {
                const long long cc = tk.start + 2 * (long long)q;
                int I, J, K;
                dec(cc, I, J, K);
                T s0 = (T)0, s1 = (T)0;
#pragma unroll 1
                for (int dd = 0; dd < 4; ++dd) {
                        const int di = dd >> 1, dj = dd & 1;
                        const int i = 2 * I + di, j = 2 * J + dj, k0 = 2 * K;
                        const long long c0 = ((long long)i * F.ny + j) * F.nz + k0;
                        const int q0 = (i + j) & 1;
                        Es.c0 = Ds.c0 = c0;
                        Es.q0 = Ds.q0 = q0;
                        Hood<T> Eh, Dh;
                        gather(Eh, E4, E1, c0, i, j, k0, F.nx, F.ny, F.nz, sx, sy, (T)0);
                        gather(Dh, D4, D1, c0, i, j, k0, F.nx, F.ny, F.nz, sx, sy, (T)F.dghost);
                        T bq[4], saq[4], r[4];
                        if (sp) {
                            ld4s(bf, c0, q0, bq);
                            ld4s(sa, c0, q0, saq);
                        } else {
                            ld4(bf + c0, bq);
                            ld4(sa + c0, saq);
                        }
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            T Fc[6];
                            quad_faces(Dh, i, j, k0, F.nx, F.ny, F.nz, F.mirror != 0, (T)F.dghost, m, Fc);
                            T n_ = bq[m] * h2;
                            T d_ = saq[m] * h2;
                            n_ = n_ + Fc[0] * Eh.xm[m]; d_ = d_ + Fc[0];
                            n_ = n_ + Fc[1] * Eh.xp[m]; d_ = d_ + Fc[1];
                            n_ = n_ + Fc[2] * Eh.ym[m]; d_ = d_ + Fc[2];
                            n_ = n_ + Fc[3] * Eh.yp[m]; d_ = d_ + Fc[3];
                            n_ = n_ + Fc[4] * Eh.zm(m); d_ = d_ + Fc[4];
                            n_ = n_ + Fc[5] * Eh.zp(m); d_ = d_ + Fc[5];
                            r[m] = (n_ - Eh.c[m] * d_) / h2;
                        }
                        s0 = s0 + r[0];
                        s0 = s0 + r[1];
                        s1 = s1 + r[2];
                        s1 = s1 + r[3];
                    }
                bc[cc] = (T)0.125 * s0;
                bc[cc + 1] = (T)0.125 * s1;
            }
            continue;
        }
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x) {
            const long long cc = tk.start + q;
            int I, J, K;
            dec(cc, I, J, K);
            T s = (T)0;
            for (int di = 0; di < 2; ++di)
                for (int dj = 0; dj < 2; ++dj)
                    for (int dk = 0; dk < 2; ++dk) {
                        const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
                        const long long c = ((long long)i * F.ny + j) * F.nz + k;
                        T num, den;
                        level_num_den<T>(F, e, c, i, j, k, num, den);
                        s = s + (num - e[sp ? cell_at(F, i, j, k, true) : c] * den) / h2;
                    }
            bc[cc] = (T)0.125 * s;
        }
    }
}

// e_fine += scale * e_coarse(parent).  Tasks run over the cells of the fine
// grid; scale != 1 only for the correction of the finest level.
template <typename T, int SP>
__global__ void __launch_bounds__(kBlock)
k_prolong(const Grid *grids, const Task *tasks, int ntasks, const int *active, double scale)
{
    const T s = (T)scale;
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        const Grid &F = grids[tk.grid];
        if (active && !active[F.prob])
            continue;
        const Grid &C = grids[F.coarser];
        const bool sp = grid_split<SP>(F);
        T *ef = (T *)F.e;
        const T *ec = (const T *)C.e;
        const Dec dec(F.ny, F.nz);
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x) {
            const long long c = tk.start + q;
            int i, j, k;
            dec(c, i, j, k);
            const long long o = sp ? sidx(c, (i + j + k) & 1) : c;
            ef[o] = ef[o] + s * ec[((long long)(i >> 1) * C.ny + (j >> 1)) * C.nz + (k >> 1)];
        }
    }
}

// Galerkin coarse faces: half the sum of the four fine faces on each coarse
// face (in-face indices in lexicographic order).  Tasks run over the padded
// (nx+1)(ny+1)(face_zstride(nz)) face grid of the coarse level.
template <typename T, int SP>
__global__ void __launch_bounds__(kBlock)
k_galerkin(const Grid *grids, const Task *tasks, int ntasks, const int *active)
{
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        const Grid &C = grids[tk.grid];
        if (active && !active[C.prob])
            continue;
        const Grid &F = grids[C.finer];
        const bool sp = grid_split<SP>(F);
        T *fc = (T *)C.f;
        // tasks run over the padded face grid; padding entries get zeros
        const long long nf = (long long)(C.nx + 1) * (C.ny + 1) * face_zstride(C.nz);
        const Dec dec(C.ny + 1, (int)face_zstride(C.nz));
        auto one = [&](long long c, int I, int J, int K) {
                // x faces
                T v = (T)0;
                if (J < C.ny && K < C.nz) {
                    T s = (T)0;
                    s = s + face_below<T>(F, 0, 2 * I, 2 * J, 2 * K, sp);
                    s = s + face_below<T>(F, 0, 2 * I, 2 * J, 2 * K + 1, sp);
                    s = s + face_below<T>(F, 0, 2 * I, 2 * J + 1, 2 * K, sp);
                    s = s + face_below<T>(F, 0, 2 * I, 2 * J + 1, 2 * K + 1, sp);
                    v = (T)0.5 * s;
                }
                fc[c] = v;
                v = (T)0;
                if (I < C.nx && K < C.nz) {
                    T s = (T)0;
                    s = s + face_below<T>(F, 1, 2 * I, 2 * J, 2 * K, sp);
                    s = s + face_below<T>(F, 1, 2 * I, 2 * J, 2 * K + 1, sp);
                    s = s + face_below<T>(F, 1, 2 * I + 1, 2 * J, 2 * K, sp);
                    s = s + face_below<T>(F, 1, 2 * I + 1, 2 * J, 2 * K + 1, sp);
                    v = (T)0.5 * s;
                }
                fc[nf + c] = v;
                v = (T)0;
                if (I < C.nx && J < C.ny && K <= C.nz) {
                    T s = (T)0;
                    s = s + face_below<T>(F, 2, 2 * I, 2 * J, 2 * K, sp);
                    s = s + face_below<T>(F, 2, 2 * I, 2 * J + 1, 2 * K, sp);
                    s = s + face_below<T>(F, 2, 2 * I + 1, 2 * J, 2 * K, sp);
                    s = s + face_below<T>(F, 2, 2 * I + 1, 2 * J + 1, 2 * K, sp);
                    v = (T)0.5 * s;
                }
                fc[2 * nf + c] = v;
        };
        if (F.fine && (F.nz & 3) == 0 && (tk.start & 1) == 0 && (tk.count & 1) == 0) {
            // finest level below: two coarse cells along z per thread, whose
            // fine faces come from quads of D (z rows 2K..2K+3) and the cell
            // before them; per face the arithmetic and the order of the sums
            // are face_below's and the loop's above
            const T *__restrict__ D = (const T *)F.D;
            const T gdh = (T)F.dghost;
            const bool mir = F.mirror != 0;
            auto quad = [&](int i, int j, int k0, T v[4]) {
                const long long x = ((long long)i * F.ny + j) * F.nz + k0;
                if (sp)
                    ld4s(D, x, (i + j) & 1, v);
                else
                    ld4(D + x, v);
            };
            auto face = [&](T hi, T lo, bool lo_in) {
                return lo_in ? (T)0.5 * (hi + lo) : (T)0.5 * (hi + (mir ? hi : gdh));
            };
            for (int q = threadIdx.x; q < (tk.count >> 1); q += blockDim.x) {
                const long long c = tk.start + 2 * (long long)q;
                int I, J, K;
                dec(c, I, J, K);
                if (!(I < C.nx && J < C.ny && K + 1 < C.nz)) {
                    one(c, I, J, K);
                    one(c + 1, I, J, K + 1);
                    continue;
                }
                const int i = 2 * I, j = 2 * J, k0 = 2 * K;
                // rows (i+di, j+dj), z k0..k0+3, and the cell at k0-1
                T r00[4], r01[4], r10[4], r11[4], xm0[4], xm1[4], ym0[4], ym1[4];
                quad(i, j, k0, r00);
                quad(i, j + 1, k0, r01);
                quad(i + 1, j, k0, r10);
                quad(i + 1, j + 1, k0, r11);
                const bool xin = i > 0, yin = j > 0, zin = k0 > 0;
                if (xin) {
                    quad(i - 1, j, k0, xm0);
                    quad(i - 1, j + 1, k0, xm1);
                }
                if (yin) {
                    quad(i, j - 1, k0, ym0);
                    quad(i + 1, j - 1, k0, ym1);
                }
                T z00 = (T)0, z01 = (T)0, z10 = (T)0, z11 = (T)0;
                if (zin) {
                    z00 = D[cell_at(F, i, j, k0 - 1, sp)];
                    z01 = D[cell_at(F, i, j + 1, k0 - 1, sp)];
                    z10 = D[cell_at(F, i + 1, j, k0 - 1, sp)];
                    z11 = D[cell_at(F, i + 1, j + 1, k0 - 1, sp)];
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {       // coarse cells K and K+1
                    const int a = 2 * h;            // fine z offset within the quad
                    T s = (T)0;
                    // x faces below (i, j+dj, k0+a+dk): lower cell (i-1, ...)
                    s = s + face(r00[a], xin ? xm0[a] : (T)0, xin);
                    s = s + face(r00[a + 1], xin ? xm0[a + 1] : (T)0, xin);
                    s = s + face(r01[a], xin ? xm1[a] : (T)0, xin);
                    s = s + face(r01[a + 1], xin ? xm1[a + 1] : (T)0, xin);
                    fc[c + h] = (T)0.5 * s;
                    // y faces below (i+di, j, k0+a+dk): lower cell (i+di, j-1, ...)
                    s = (T)0;
                    s = s + face(r00[a], yin ? ym0[a] : (T)0, yin);
                    s = s + face(r00[a + 1], yin ? ym0[a + 1] : (T)0, yin);
                    s = s + face(r10[a], yin ? ym1[a] : (T)0, yin);
                    s = s + face(r10[a + 1], yin ? ym1[a + 1] : (T)0, yin);
                    fc[nf + c + h] = (T)0.5 * s;
                    // z faces below (i+di, j+dj, k0+a): lower cell at k0+a-1
                    const bool zl = h == 1 || zin;
                    s = (T)0;
                    s = s + face(r00[a], h ? r00[1] : z00, zl);
                    s = s + face(r01[a], h ? r01[1] : z01, zl);
                    s = s + face(r10[a], h ? r10[1] : z10, zl);
                    s = s + face(r11[a], h ? r11[1] : z11, zl);
                    fc[2 * nf + c + h] = (T)0.5 * s;
                }
            }
            continue;
        }
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x) {
            const long long c = tk.start + q;
            int I, J, K;
            dec(c, I, J, K);
            one(c, I, J, K);
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_mean8_sa(const Grid *grids, const Task *tasks, int ntasks)
{
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const Task tk = tasks[t];
        const Grid &C = grids[tk.grid];
        const Grid &F = grids[C.finer];
        const T *sf = (const T *)F.sa;
        T *sc = (T *)C.sa;
        const Dec dec(C.ny, C.nz);
        for (int q = threadIdx.x; q < tk.count; q += blockDim.x) {
            const long long cc = tk.start + q;
            int I, J, K;
            dec(cc, I, J, K);
            T s = (T)0;
            for (int di = 0; di < 2; ++di)
                for (int dj = 0; dj < 2; ++dj)
                    for (int dk = 0; dk < 2; ++dk)
                        s = s + sf[cell_at(F, 2 * I + di, 2 * J + dj, 2 * K + dk, F.split)];
            sc[cc] = (T)0.125 * s;
        }
    }
}

// ---------------------------------------------------------------------------
// Deep part of the V-cycle.  Coarse levels of a few thousand cells are all
// launch overhead, so one workgroup per problem runs every level from its
// root (the first level at or below the size limit) down to the level above
// the coarsest, and back up, with barriers between the phases.  The coarsest
// solve between the two halves stays a kernel of its own.  Per cell the
// arithmetic is exactly that of the level kernels (face coefficients, the
// smoother's pair walk, the 8-child restriction, the parent prolongation).
// ---------------------------------------------------------------------------
constexpr int kDeepBlock = 1024;

template <typename T>
__device__ void deep_zero(const Grid &g)
{
    T *e = (T *)g.e;
    for (long long c = threadIdx.x; c < g.n; c += blockDim.x)
        e[c] = (T)0;
}

template <typename T>
__device__ void deep_smooth(const Grid &g, int colour, T omega)
{
    T *e = (T *)g.e;
    const Dec dec(g.ny, g.nz);
    for (long long q = threadIdx.x; q < (g.n >> 1); q += blockDim.x) {
        const long long c0 = 2 * q;
        int i, j, k;
        dec(c0, i, j, k);
        const int odd = (i + j + colour) & 1;
        const long long c = c0 + odd;
        T num, den;
        face_num_den<T>(g, e, c, i, j, k + odd, num, den);
        e[c] = omega * (num / den) + ((T)1 - omega) * e[c];
    }
}

// C.b = 8-child mean of the residual of F
template <typename T>
__device__ void deep_restrict(const Grid &F, const Grid &C)
{
    const T *e = (const T *)F.e;
    T *bc = (T *)C.b;
    const T h2 = (T)F.h2;
    const Dec dec(C.ny, C.nz);
    for (long long cc = threadIdx.x; cc < C.n; cc += blockDim.x) {
        int I, J, K;
        dec(cc, I, J, K);
        T s = (T)0;
        for (int di = 0; di < 2; ++di)
            for (int dj = 0; dj < 2; ++dj)
                for (int dk = 0; dk < 2; ++dk) {
                    const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
                    const long long c = ((long long)i * F.ny + j) * F.nz + k;
                    T num, den;
                    face_num_den<T>(F, e, c, i, j, k, num, den);
                    s = s + (num - e[c] * den) / h2;
                }
        bc[cc] = (T)0.125 * s;
    }
}

// F.e += C.e(parent)
template <typename T>
__device__ void deep_prolong(const Grid &F, const Grid &C)
{
    T *ef = (T *)F.e;
    const T *ec = (const T *)C.e;
    const T one = (T)1.0;
    const Dec dec(F.ny, F.nz);
    for (long long c = threadIdx.x; c < F.n; c += blockDim.x) {
        int i, j, k;
        dec(c, i, j, k);
        ef[c] = ef[c] + one * ec[((long long)(i >> 1) * C.ny + (j >> 1)) * C.nz + (k >> 1)];
    }
}

// Down: from the root, zero e, the level's pre-sweeps (red then black),
// restrict, to the level above the coarsest.
template <typename T>
__global__ void __launch_bounds__(kDeepBlock)
k_deep_down(const Grid *grids, const int *roots, const int *active, T omega)
{
    int gid = roots[blockIdx.x];
    if (active && !active[grids[gid].prob])
        return;
    while (grids[gid].coarser >= 0) {
        const Grid &g = grids[gid];
        deep_zero<T>(g);
        __syncthreads();
        for (int s = 0; s < g.nu_pre; ++s) {
            deep_smooth<T>(g, 0, omega);
            __syncthreads();
            deep_smooth<T>(g, 1, omega);
            __syncthreads();
        }
        deep_restrict<T>(g, grids[g.coarser]);
        __syncthreads();
        gid = g.coarser;
    }
}

// Up: from the level above the coarsest back to the root, prolongate and
// the level's post-sweeps (black then red).
template <typename T>
__global__ void __launch_bounds__(kDeepBlock)
k_deep_up(const Grid *grids, const int *roots, const int *active, T omega)
{
    const int root = roots[blockIdx.x];
    if (active && !active[grids[root].prob])
        return;
    int gid = root;
    while (grids[gid].coarser >= 0)
        gid = grids[gid].coarser;          // the coarsest
    while (gid != root) {
        gid = grids[gid].finer;
        const Grid &g = grids[gid];
        deep_prolong<T>(g, grids[g.coarser]);
        __syncthreads();
        for (int s = 0; s < g.nu_post; ++s) {
            deep_smooth<T>(g, 1, omega);
            __syncthreads();
            deep_smooth<T>(g, 0, omega);
            __syncthreads();
        }
    }
}

// Coarsest level: e = M^{-1} (h^2 b) with M = h^2 A in natural order (half
// bandwidth bw = ny*nz), factored by banded Cholesky in FP64 and solved in the
// same launch.  Band entry (r, q), r - bw <= q <= r, sits at
// W[r*(bw+1) + q - r + bw].
//
// The factor is right-looking with the forward substitution folded in: at
// column c every thread forms the multipliers it needs itself,
// L(r,c) = W(r,c)/L(c,c), and subtracts L(r,c) L(q,c) from its trailing
// entries and L(r,c) y_c from the right-hand side, so each entry receives its
// subtractions in ascending column order, the order of the textbook
// recurrence.  Column c is scaled in place one step later, when nothing reads
// it any more, which leaves one barrier per column.  The backward
// substitution runs row by row in one lane, each row's subtractions in
// ascending order.  Every value is therefore rounded as in the textbook dense
// algorithm.  W, diag (the factor's diagonal) and y (right-hand side in,
// solution out) may live in LDS or global memory.  Returns false in every
// thread when a pivot is not positive.
__device__ bool chol_band(double *__restrict__ W, double *__restrict__ diag,
                          double *__restrict__ y, int n, int bw)
{
    const int Wd = bw + 1;
    const int tid = threadIdx.x, nt = blockDim.x;
    bool bad = false;
    for (int c = 0; c < n; ++c) {
        const double d = W[(long long)c * Wd + bw];
        bad = bad || !(d > 0.0);
        const double lcc = sqrt(d);
        if (c > 0) {
            // column c-1 and y_{c-1} take their final (scaled) values
            const double lp = diag[c - 1];
            const int mp = min(bw, n - c);
            for (int a = tid; a < mp; a += nt) {
                double &w = W[(long long)(c + a) * Wd + (c - 1) - (c + a) + bw];
                w = w / lp;
            }
            if (tid == nt - 1)
                y[c - 1] = y[c - 1] / lp;
        }
        if (tid == 0)
            diag[c] = lcc;
        const int m = min(bw, n - 1 - c);       // rows below c in the band
        const double yc = y[c] / lcc;
        for (int x = tid; x < m * m; x += nt) {
            const int a = x / m, bb = x - a * m;
            if (bb > a)
                continue;
            const int r = c + 1 + a, q = c + 1 + bb;
            const double lrc = W[(long long)r * Wd + c - r + bw] / lcc;
            const double lqc = W[(long long)q * Wd + c - q + bw] / lcc;
            double &t = W[(long long)r * Wd + q - r + bw];
            t = t - lrc * lqc;
        }
        for (int a = tid; a < m; a += nt) {
            const int r = c + 1 + a;
            const double lrc = W[(long long)r * Wd + c - r + bw] / lcc;
            y[r] = y[r] - lrc * yc;
        }
        __syncthreads();
    }
    if (tid == 0) {
        y[n - 1] = y[n - 1] / diag[n - 1];     // the forward substitution's last row
        // L^T x = y, row by row, subtractions in ascending order; the band and
        // y entries of four subtractions are loaded before the first of them
        for (int r = n - 1; r >= 0; --r) {
            const int m = min(bw, n - 1 - r);
            double s = y[r];
            int a = 1;
            for (; a + 3 <= m; a += 4) {
                double w[4], v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    w[u] = W[(long long)(r + a + u) * Wd + r - (r + a + u) + bw];
                    v[u] = y[r + a + u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    s = s - w[u] * v[u];
            }
            for (; a <= m; ++a)
                s = s - W[(long long)(r + a) * Wd + r - (r + a) + bw] * y[r + a];
            y[r] = s / diag[r];
        }
    }
    __syncthreads();
    return !bad;
}

// Factorisation alone, as chol_band does it (the same operations in the same
// order, the right-hand side left out); the factor's diagonal goes to diag.
__device__ bool chol_factor(double *__restrict__ W, double *__restrict__ diag, int n, int bw)
{
    const int Wd = bw + 1;
    const int tid = threadIdx.x, nt = blockDim.x;
    bool bad = false;
    for (int c = 0; c < n; ++c) {
        const double d = W[(long long)c * Wd + bw];
        bad = bad || !(d > 0.0);
        const double lcc = sqrt(d);
        if (c > 0) {
            const double lp = diag[c - 1];
            const int mp = min(bw, n - c);
            for (int a = tid; a < mp; a += nt) {
                double &w = W[(long long)(c + a) * Wd + (c - 1) - (c + a) + bw];
                w = w / lp;
            }
        }
        if (tid == 0)
            diag[c] = lcc;
        const int m = min(bw, n - 1 - c);
        for (int x = tid; x < m * m; x += nt) {
            const int a = x / m, bb = x - a * m;
            if (bb > a)
                continue;
            const int r = c + 1 + a, q = c + 1 + bb;
            const double lrc = W[(long long)r * Wd + c - r + bw] / lcc;
            const double lqc = W[(long long)q * Wd + c - q + bw] / lcc;
            double &tt = W[(long long)r * Wd + q - r + bw];
            tt = tt - lrc * lqc;
        }
        __syncthreads();
    }
    return !bad;
}

// Ordering of one wavefront's own LDS accesses across lanes (no workgroup
// barrier): what a lane wrote before is seen by every lane after.
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// L L^T x = y with the factor of chol_factor in W (in LDS; its diagonal in
// the diagonal slots), by the 64 lanes of one wavefront: the forward
// substitution right-looking across the lanes, the backward substitution in
// the first lane.  Each y entry receives its subtractions in the order of
// chol_band (ascending columns forward, ascending rows backward), so the
// result is the same.  The other wavefronts must not touch W or y until a
// barrier after the call.
__device__ void chol_solve_wave(const double *__restrict__ W, double *__restrict__ y, int n,
                                int bw)
{
    const int Wd = bw + 1;
    const int lane = threadIdx.x & (kWave - 1);
    for (int c = 0; c < n; ++c) {
        if (lane == 0)
            y[c] = y[c] / W[(long long)c * Wd + bw];
        wave_lds_sync();
        const double yc = y[c];
        const int m = min(bw, n - 1 - c);
        for (int a = lane; a < m; a += kWave) {
            const int r = c + 1 + a;
            y[r] = y[r] - W[(long long)r * Wd + c - r + bw] * yc;
        }
        wave_lds_sync();
    }
    if (lane == 0) {
        for (int r = n - 1; r >= 0; --r) {
            const int m = min(bw, n - 1 - r);
            double s = y[r];
            int a = 1;
            for (; a + 7 <= m; a += 8) {
                double w[8], v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    w[u] = W[(long long)(r + a + u) * Wd + r - (r + a + u) + bw];
                    v[u] = y[r + a + u];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    s = s - w[u] * v[u];
            }
            for (; a <= m; ++a)
                s = s - W[(long long)(r + a) * Wd + r - (r + a) + bw] * y[r + a];
            y[r] = s / W[(long long)r * Wd + bw];
        }
    }
    wave_lds_sync();
}

// Rows of M = h^2 A for the coarsest grid g into the band W (one row per
// thread; face loads independent of each other).
template <typename T>
__device__ void chol_assemble(const Grid &g, double *W)
{
    const int n = (int)g.n, bw = g.ny * g.nz, Wd = bw + 1;
    const double h2 = g.h2;
    const T *sa = (const T *)g.sa;
    const Dec dec(g.ny, g.nz);
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        int i, j, k;
        dec(r, i, j, k);
        double *row = W + (long long)r * Wd;       // row[q - r + bw]
        const double fx0 = (double)face_below<T>(g, 0, i, j, k);
        const double fx1 = (double)face_below<T>(g, 0, i + 1, j, k);
        const double fy0 = (double)face_below<T>(g, 1, i, j, k);
        const double fy1 = (double)face_below<T>(g, 1, i, j + 1, k);
        const double fz0 = (double)face_below<T>(g, 2, i, j, k);
        const double fz1 = (double)face_below<T>(g, 2, i, j, k + 1);
        for (int d = 0; d < bw; ++d)
            row[d] = 0.0;
        double v = (double)sa[r] * h2;
        v = v + fx0;
        v = v + fx1;
        v = v + fy0;
        v = v + fy1;
        v = v + fz0;
        v = v + fz1;
        row[bw] = v;
        if (k > 0)
            row[bw - 1] = -fz0;
        if (j > 0)
            row[bw - g.nz] = -fy0;
        if (i > 0)
            row[0] = -fx0;
    }
}

constexpr int kCholLds = 64 * 1024;

// LDS: y and the diagonal (2 max_n doubles), then the band if it fits.
__host__ __device__ inline bool chol_in_lds(long long n, long long bw, long long max_n)
{
    return n * (bw + 1) * 8 + 2 * max_n * 8 <= kCholLds;
}

// Factor of the coarsest operator, one block per coarsest grid whose band
// fits in LDS: M = h^2 A assembled into LDS, factored (chol_factor) and stored
// in g.band with the factor's diagonal in the diagonal slots.  It depends only
// on the coarse operators, so it runs beside the down-sweep of the finer
// levels; the solve kernels then only substitute.  fail[prob] is set to 1 when
// a pivot is not positive.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_coarse_factor(const Grid *grids, const int *ids, const int *active, int *fail, int max_n)
{
    extern __shared__ double lds[];
    const Grid &g = grids[ids[blockIdx.x]];
    if (active && !active[g.prob])
        return;
    (void)max_n;
    const int n = (int)g.n, bw = g.ny * g.nz, Wd = bw + 1;
    if (!chol_in_lds(n, bw, n))
        return;                                // factored by k_coarse_solve itself
    double *diag = lds + n;
    double *W = lds + 2 * n;
    chol_assemble<T>(g, W);
    __syncthreads();
    const bool ok = chol_factor(W, diag, n, bw);
    __syncthreads();
    for (int x = threadIdx.x; x < n * Wd; x += blockDim.x) {
        const int r = x / Wd;
        g.band[x] = x - r * Wd == bw ? diag[r] : W[x];
    }
    if (threadIdx.x == 0 && !ok)
        fail[g.prob] = 1;
}

// Coarsest solve, one block per listed grid: with the factor of
// k_coarse_factor (copied into LDS) the two substitutions by one wavefront;
// a band too large for LDS is assembled, factored and solved here in global
// memory (chol_band).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_coarse_solve(const Grid *grids, const int *ids, const int *active, int *fail, int max_n)
{
    extern __shared__ double lds[];
    const Grid &g = grids[ids[blockIdx.x]];
    if (active && !active[g.prob])
        return;
    (void)max_n;
    const int n = (int)g.n, bw = g.ny * g.nz, Wd = bw + 1;
    double *y = lds, *diag = lds + n;
    const T *b = (const T *)g.b;
    for (int r = threadIdx.x; r < n; r += blockDim.x)
        y[r] = (double)b[r] * g.h2;
    if (chol_in_lds(n, bw, n)) {
        double *W = lds + 2 * n;
        for (int x = threadIdx.x; x < n * Wd; x += blockDim.x)
            W[x] = g.band[x];
        __syncthreads();
        if (threadIdx.x < kWave)
            chol_solve_wave(W, y, n, bw);
        __syncthreads();
    } else {
        chol_assemble<T>(g, g.band);
        __syncthreads();
        const bool ok = chol_band(g.band, diag, y, n, bw);
        if (threadIdx.x == 0 && !ok)
            fail[g.prob] = 1;
    }
    T *e = (T *)g.e;
    for (int r = threadIdx.x; r < n; r += blockDim.x)
        e[r] = (T)y[r];
}

// ---------------------------------------------------------------------------
// Coarse tail in one launch: the deep levels of a problem (its root, the
// first level of at most kTailRootCells cells, and up to two levels below it
// of at most kTailLowCells cells each), pre-smoothing, restriction, the
// coarsest Cholesky solve and the way back up, one workgroup per problem.
// The corrections of the deep levels and the band live in LDS; each thread
// keeps the face coefficients, b h^2 and the diagonal of the cells it owns
// (cell c of a level belongs to thread c mod kTailBlock) in registers, so a
// phase between two barriers touches LDS only.  Per cell the arithmetic is
// exactly that of the work-list level kernels: the same neighbour order, the
// same diagonal sum, the 8-child restriction in the same child order and the
// parent prolongation, so results are bit-identical to the kernel-per-phase
// path, which serves the problems whose tail does not fit.
// ---------------------------------------------------------------------------
constexpr int kTailBlock = 1024;
constexpr int kTailRootCells = 4 * kTailBlock;
constexpr int kTailLowCells = kTailBlock;
constexpr int kTailMaxLow = 2;
constexpr int kTailLds = 64 * 1024;

template <typename T>
struct CellCoef {
    T F[6];     // faces x-, x+, y-, y+, z-, z+
    T bh2;      // b h^2
    T den;      // sa h^2 + sum of the faces
};

template <typename T>
__device__ inline void tail_coef(const Grid &g, long long c, int i, int j, int k, CellCoef<T> &q,
                                 bool with_b)
{
    const T h2 = (T)g.h2;
    const long long fy = face_zstride(g.nz), fx = (long long)(g.ny + 1) * fy;
    const long long nf = (long long)(g.nx + 1) * fx;
    const long long fi = (long long)i * fx + (long long)j * fy + k;
    const T *Fx = (const T *)g.f;
    const T *Fy = Fx + nf;
    const T *Fz = Fy + nf;
    q.F[0] = Fx[fi];
    q.F[1] = Fx[fi + fx];
    q.F[2] = Fy[fi];
    q.F[3] = Fy[fi + fy];
    q.F[4] = Fz[fi];
    q.F[5] = Fz[fi + 1];
    T d_ = ((const T *)g.sa)[c] * h2;
    for (int s = 0; s < 6; ++s)
        d_ = d_ + q.F[s];
    q.den = d_;
    q.bh2 = with_b ? ((const T *)g.b)[c] * h2 : (T)0;
}

template <typename T>
__device__ inline T tail_num(const CellCoef<T> &q, const T *e, long long c, int i, int j, int k,
                             int nx, int ny, int nz)
{
    const long long sx = (long long)ny * nz, sy = nz;
    T n_ = q.bh2;
    n_ = n_ + q.F[0] * (i > 0 ? e[c - sx] : (T)0);
    n_ = n_ + q.F[1] * (i < nx - 1 ? e[c + sx] : (T)0);
    n_ = n_ + q.F[2] * (j > 0 ? e[c - sy] : (T)0);
    n_ = n_ + q.F[3] * (j < ny - 1 ? e[c + sy] : (T)0);
    n_ = n_ + q.F[4] * (k > 0 ? e[c - 1] : (T)0);
    n_ = n_ + q.F[5] * (k < nz - 1 ? e[c + 1] : (T)0);
    return n_;
}

// Phases over the cells a thread owns on one level (CPT cells per thread).
template <typename T, int CPT>
__device__ void tail_load(const Grid &g, CellCoef<T> (&q)[CPT], bool with_b)
{
    const Dec dec(g.ny, g.nz);
#pragma unroll
    for (int s = 0; s < CPT; ++s) {
        const long long c = threadIdx.x + (long long)s * kTailBlock;
        if (c < g.n) {
            int i, j, k;
            dec(c, i, j, k);
            tail_coef<T>(g, c, i, j, k, q[s], with_b);
        }
    }
}

template <typename T, int CPT>
__device__ void tail_smooth(const Grid &g, const CellCoef<T> (&q)[CPT], T *e, int colour, T omega)
{
    const Dec dec(g.ny, g.nz);
#pragma unroll
    for (int s = 0; s < CPT; ++s) {
        const long long c = threadIdx.x + (long long)s * kTailBlock;
        if (c < g.n) {
            int i, j, k;
            dec(c, i, j, k);
            if (((i + j + k) & 1) != colour)
                continue;
            const T num = tail_num<T>(q[s], e, c, i, j, k, g.nx, g.ny, g.nz);
            e[c] = omega * (num / q[s].den) + ((T)1 - omega) * e[c];
        }
    }
}

template <typename T, int CPT>
__device__ void tail_residual(const Grid &g, const CellCoef<T> (&q)[CPT], const T *e, T *r)
{
    const Dec dec(g.ny, g.nz);
    const T h2 = (T)g.h2;
#pragma unroll
    for (int s = 0; s < CPT; ++s) {
        const long long c = threadIdx.x + (long long)s * kTailBlock;
        if (c < g.n) {
            int i, j, k;
            dec(c, i, j, k);
            const T num = tail_num<T>(q[s], e, c, i, j, k, g.nx, g.ny, g.nz);
            r[c] = (num - e[c] * q[s].den) / h2;
        }
    }
}

template <typename T>
__device__ void tail_zero(const Grid &g, T *e)
{
    for (long long c = threadIdx.x; c < g.n; c += kTailBlock)
        e[c] = (T)0;
}

// e of level F += e of its parent on level C (both in LDS)
template <typename T>
__device__ void tail_prolong(const Grid &F, const Grid &C, T *ef, const T *ec)
{
    const T one = (T)1.0;
    const Dec dec(F.ny, F.nz);
    for (long long c = threadIdx.x; c < F.n; c += kTailBlock) {
        int i, j, k;
        dec(c, i, j, k);
        ef[c] = ef[c] + one * ec[((long long)(i >> 1) * C.ny + (j >> 1)) * C.nz + (k >> 1)];
    }
}

// 8-child mean of the residual r of level F for coarse cell (I, J, K).
template <typename T>
__device__ inline T tail_restrict(const Grid &F, const T *r, int I, int J, int K)
{
    T s = (T)0;
    for (int di = 0; di < 2; ++di)
        for (int dj = 0; dj < 2; ++dj)
            for (int dk = 0; dk < 2; ++dk)
                s = s + r[((long long)(2 * I + di) * F.ny + (2 * J + dj)) * F.nz + (2 * K + dk)];
    return (T)0.125 * s;
}

// LDS bytes the tail of a problem needs: band, diagonal and right-hand side of
// the coarsest level (FP64), the deep levels' corrections and one residual /
// coarsest-correction array (precision T).
__host__ __device__ inline long long tail_lds_bytes(long long nc, long long bw, long long deep_cells,
                                                    long long scratch_cells, int tsz)
{
    return (nc * (bw + 1) + 2 * nc) * 8 + (deep_cells + scratch_cells) * tsz;
}

template <typename T>
__global__ void __launch_bounds__(kTailBlock)
k_coarse_tail(const Grid *grids, const int *roots, const int *active, int *fail, T omega)
{
    extern __shared__ double lds[];
    const int root = roots[blockIdx.x];
    if (active && !active[grids[root].prob])
        return;
    int lv[kTailMaxLow + 2];
    int nl = 0;
    for (int gi = root;; gi = grids[gi].coarser) {
        lv[nl++] = gi;
        if (grids[gi].coarser < 0 || nl == kTailMaxLow + 2)
            break;
    }
    const int nd = nl - 1;                     // smoothed (deep) levels
    const Grid &Cg = grids[lv[nd]];
    const int nc = (int)Cg.n, bw = Cg.ny * Cg.nz;
    double *W = lds;
    double *diag = W + (long long)nc * (bw + 1);
    double *y = diag + nc;
    T *e[kTailMaxLow + 1];
    T *p = (T *)(y + nc);
    for (int l = 0; l < nd; ++l) {
        e[l] = p;
        p += grids[lv[l]].n;
    }
    T *r = p;                                  // residual, then the coarsest correction
    CellCoef<T> q0[4], q1[1], q2[1];
    if (nd >= 1)
        tail_load<T, 4>(grids[lv[0]], q0, true);
    if (nd >= 2)
        tail_load<T, 1>(grids[lv[1]], q1, false);
    if (nd >= 3)
        tail_load<T, 1>(grids[lv[2]], q2, false);
    // the coarsest factor (k_coarse_factor) into LDS
    for (int x = threadIdx.x; x < nc * (bw + 1); x += kTailBlock)
        W[x] = Cg.band[x];
    if (nd == 0)
        for (int c = threadIdx.x; c < nc; c += kTailBlock)
            y[c] = (double)((const T *)Cg.b)[c] * Cg.h2;
    // down: zero, the level's pre-sweeps (red then black), restrict
    for (int l = 0; l < nd; ++l) {
        const Grid &g = grids[lv[l]];
        tail_zero<T>(g, e[l]);
        __syncthreads();
        for (int s = 0; s < g.nu_pre; ++s)
            for (int colour = 0; colour < 2; ++colour) {
                if (l == 0)
                    tail_smooth<T, 4>(g, q0, e[0], colour, omega);
                else if (l == 1)
                    tail_smooth<T, 1>(g, q1, e[1], colour, omega);
                else
                    tail_smooth<T, 1>(g, q2, e[2], colour, omega);
                __syncthreads();
            }
        if (l == 0)
            tail_residual<T, 4>(g, q0, e[0], r);
        else if (l == 1)
            tail_residual<T, 1>(g, q1, e[1], r);
        else
            tail_residual<T, 1>(g, q2, e[2], r);
        __syncthreads();
        const Grid &C = grids[lv[l + 1]];
        const Dec dec(C.ny, C.nz);
        for (long long cc = threadIdx.x; cc < C.n; cc += kTailBlock) {
            int I, J, K;
            dec(cc, I, J, K);
            const T bv = tail_restrict<T>(g, r, I, J, K);
            if (l + 1 == nd)
                y[cc] = (double)bv * C.h2;
            else if (l + 1 == 1)
                q1[0].bh2 = bv * (T)C.h2;      // cc == threadIdx.x: one cell per thread
            else
                q2[0].bh2 = bv * (T)C.h2;
        }
        __syncthreads();
    }
    // coarsest (the band, y and the level data written above are complete)
    __syncthreads();
    if (threadIdx.x < kWave)
        chol_solve_wave(W, y, nc, bw);
    __syncthreads();
    if (nd == 0) {
        T *ec = (T *)Cg.e;
        for (int c = threadIdx.x; c < nc; c += kTailBlock)
            ec[c] = (T)y[c];
        return;
    }
    for (int c = threadIdx.x; c < nc; c += kTailBlock)
        r[c] = (T)y[c];
    __syncthreads();
    // up: prolongate, the level's post-sweeps (black then red)
    for (int l = nd - 1; l >= 0; --l) {
        const Grid &g = grids[lv[l]];
        tail_prolong<T>(g, grids[lv[l + 1]], e[l], l + 1 == nd ? r : e[l + 1]);
        __syncthreads();
        for (int s = 0; s < g.nu_post; ++s)
            for (int colour = 1; colour >= 0; --colour) {
                if (l == 0)
                    tail_smooth<T, 4>(g, q0, e[0], colour, omega);
                else if (l == 1)
                    tail_smooth<T, 1>(g, q1, e[1], colour, omega);
                else
                    tail_smooth<T, 1>(g, q2, e[2], colour, omega);
                __syncthreads();
            }
    }
    T *eg = (T *)grids[lv[0]].e;
    for (long long c = threadIdx.x; c < grids[lv[0]].n; c += kTailBlock)
        eg[c] = e[0][c];
}

__global__ void k_put_fine(Fine f, Fine *dst)
{
    if (threadIdx.x == 0)
        *dst = f;
}

inline int grid_for(int ntasks)
{
    // Enough blocks to fill 256 CUs several times; blocks stride over tasks.
    const int cap = 256 * 16;
    return ntasks < cap ? (ntasks > 0 ? ntasks : 1) : cap;
}

// One block per task, for stencil passes over the finest level: blocks are
// dispatched in task order, so the tasks resident at any moment form one
// contiguous run of planes and a plane's x-neighbours are read while it is
// still in L2.  (With blocks striding over tasks, the blocks drift apart
// and at 512^3 most x-neighbour planes are fetched from memory again.)
inline int grid_per_task(int ntasks)
{
    return ntasks > 0 ? ntasks : 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

// Kernel instance for a precision/layout mode: 0 FP64 natural, 1 FP32
// natural, 2 FP32 colour-split, 3 FP32 decided per problem, 4 FP64
// colour-split, 5 FP64 decided per problem (instances share one signature).
#define FLD_PICK(K, mode)                                                      \
    ((mode) == 0 ? K<double, 0>                                                \
     : (mode) == 1 ? K<float, 0>                                               \
     : (mode) == 2 ? K<float, 1>                                               \
     : (mode) == 3 ? K<float, 2> : (mode) == 4 ? K<double, 1> : K<double, 2>)
// Level kernels: the precision is the template's, sp is 0/1/2 as above.
#define FLD_PICK_SP(K, T, sp)                                                  \
    ((sp) == 0 ? K<T, 0> : (sp) == 1 ? K<T, 1> : K<T, 2>)

void launch_setup(hipStream_t s, const Fine &f, const Task *tasks, int ntasks,
                  const double *sigma_t, const double *albedo, const double *Q,
                  double sigma_eps, double aniso_g, double *partials, int mixed)
{
    hipLaunchKernelGGL(k_setup, dim3(grid_for(ntasks)), dim3(kBlock), 0, s, f, tasks, ntasks,
                       sigma_t, albedo, Q, sigma_eps, aniso_g, partials,
                       mixed ? (float *)f.sa0 : (float *)nullptr,
                       !mixed && f.split ? (double *)f.sa0 : (double *)nullptr);
}

void launch_sum_partials(hipStream_t s, int nprob, const int *range, const double *partials,
                         double *scal, int slot, const int *active)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(nprob), dim3(kBlock), 0, s, range, partials, scal,
                       slot, active);
}

void launch_after_setup(hipStream_t s, int nprob, const Fine *fines, double *scal)
{
    hipLaunchKernelGGL(k_after_setup, dim3((nprob + 63) / 64), dim3(64), 0, s, nprob, fines, scal);
}

void launch_init_phi(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                     const double *scal, int zero_dirs, int mixed)
{
    if (mixed)
        hipLaunchKernelGGL(k_init_phi<float>, dim3(grid_for(ntasks)), dim3(kBlock), 0, s, fines,
                           tasks, ntasks, scal, zero_dirs);
    else
        hipLaunchKernelGGL(k_init_phi<double>, dim3(grid_for(ntasks)), dim3(kBlock), 0, s, fines,
                           tasks, ntasks, scal, zero_dirs);
}

void launch_limiter(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                    const int *active, const double *scal, int src, int dst, int use_dir,
                    int dir_idx, int to_tmp, int mixed, int lim_kind)
{
    hipLaunchKernelGGL(lim_kind != L_LP ? FLD_PICK(k_limiter, mixed)
                       : use_dir         ? FLD_PICK(k_limiter_lp_dir, mixed)
                                         : FLD_PICK(k_limiter_lp, mixed),
                       dim3(grid_for(ntasks)), dim3(kBlock), 0, s, fines, tasks, ntasks, active,
                       scal, src, dst, use_dir, dir_idx, to_tmp);
}

void launch_residual(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                     const int *active, int src, int use_tmp, int b0_idx, double *r_out,
                     double *partials, int mixed)
{
    hipLaunchKernelGGL(FLD_PICK(k_residual, mixed), dim3(grid_per_task(ntasks)), dim3(kBlock), 0, s, fines,
                           tasks, ntasks, active, src, use_tmp, b0_idx, r_out, partials);
}

void launch_lim_res(hipStream_t s, const Fine *fines, const LrTile *tiles, int ntiles,
                    const int *active, const double *scal, int src, int b0_idx, int write_d64,
                    double *partials, int mixed)
{
    if (ntiles > 0)
        hipLaunchKernelGGL(FLD_PICK(k_lim_res, mixed), dim3(std::min(8 * ((ntiles + 7) / 8), 4096)),
                           dim3(kLrThreads), 0,
                           s, fines, tiles, ntiles, active, scal, src, b0_idx, write_d64,
                           partials);
}

__global__ void k_poison(const Fine *fines, int nprob, int src)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprob)
        fines[p].phi[src][0] = __builtin_nan("");
}

void launch_poison(hipStream_t s, const Fine *fines, int nprob, int src)
{
    hipLaunchKernelGGL(k_poison, dim3((nprob + 63) / 64), dim3(64), 0, s, fines, nprob, src);
}

void launch_rel(hipStream_t s, int nprob, double *scal, const int *active)
{
    hipLaunchKernelGGL(k_rel, dim3((nprob + 63) / 64), dim3(64), 0, s, nprob, scal, active);
}

void launch_npcg_dots(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                      const int *active, int b0_idx, double *pg, double *ps, int mixed)
{
    hipLaunchKernelGGL(FLD_PICK(k_npcg_dots, mixed), dim3(grid_for(ntasks)), dim3(kBlock), 0, s, fines,
                           tasks, ntasks, active, b0_idx, pg, ps);
}

void launch_defl_sum_sa(hipStream_t s, const Fine *fines, const CTask *ct, int nct, double *psa,
                        int mixed)
{
    if (nct <= 0)
        return;
    if (mixed)
        hipLaunchKernelGGL(k_defl_sum_sa<float>, dim3(grid_for(nct)), dim3(kBlock), 0, s, fines, ct,
                           nct, psa);
    else
        hipLaunchKernelGGL(k_defl_sum_sa<double>, dim3(grid_for(nct)), dim3(kBlock), 0, s, fines,
                           ct, nct, psa);
}

void launch_defl_sum_b(hipStream_t s, const Fine *fines, const CTask *ct, int nct,
                       const int *active, int b0_idx, double *ps, int mixed)
{
    if (nct <= 0)
        return;
    if (mixed)
        hipLaunchKernelGGL(k_defl_sum_b<float>, dim3(grid_for(nct)), dim3(kBlock), 0, s, fines, ct,
                           nct, active, b0_idx, ps);
    else
        hipLaunchKernelGGL(k_defl_sum_b<double>, dim3(grid_for(nct)), dim3(kBlock), 0, s, fines,
                           ct, nct, active, b0_idx, ps);
}

void launch_defl_rim(hipStream_t s, const Fine *fines, const CTask *rt, int nrt,
                     const int *active, double *pd, int mixed)
{
    if (nrt <= 0)
        return;
    hipLaunchKernelGGL(FLD_PICK(k_defl_rim, mixed), dim3(grid_for(nrt)), dim3(kBlock), 0, s, fines,
                       rt, nrt, active, pd);
}

void launch_defl_finish(hipStream_t s, int ncl_total, const int *crange, const int *rrange,
                        const int *cprob, const double *ps, const double *pd, double *csa,
                        double *alpha, const int *active, int sa_only)
{
    if (ncl_total > 0)
        hipLaunchKernelGGL(k_defl_finish, dim3(ncl_total), dim3(kBlock), 0, s, crange, rrange,
                           cprob, ps, pd, csa, alpha, active, sa_only);
}

void launch_defl_init(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                      const int *active, const double *alpha, int mixed)
{
    hipLaunchKernelGGL(FLD_PICK(k_defl_init, mixed), dim3(grid_for(ntasks)), dim3(kBlock), 0, s, fines,
                           tasks, ntasks, active, alpha);
}

void launch_nested_coarsen(hipStream_t s, const double *sig_hat, const double *sa,
                           const double *j, int nx, int ny, int nz, double *st_c, double *al_c,
                           double *q_c)
{
    const long long nc = (long long)(nx / 2) * (ny / 2) * (nz / 2);
    const long long blocks = (nc + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_nested_coarsen, dim3((int)std::min<long long>(blocks, 65536)),
                       dim3(kBlock), 0, s, sig_hat, sa, j, nx, ny, nz, st_c, al_c, q_c);
}

void launch_nested_prolong(hipStream_t s, const double *phi_c, int nx, int ny, int nz,
                           double *phi)
{
    const long long n = (long long)nx * ny * nz;
    const long long blocks = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_nested_prolong, dim3((int)std::min<long long>(blocks, 65536)),
                       dim3(kBlock), 0, s, phi_c, nx, ny, nz, phi);
}

void launch_npcg_beta(hipStream_t s, int nprob, double *scal, const int *active, int first,
                      double restart_growth)
{
    hipLaunchKernelGGL(k_npcg_beta, dim3((nprob + 63) / 64), dim3(64), 0, s, nprob, scal, active,
                       first, restart_growth);
}

void launch_npcg_dir(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                     const int *active, const double *scal, int b0_idx, int pin, int pout,
                     double *prp, double *ppap, int mixed)
{
    hipLaunchKernelGGL(FLD_PICK(k_npcg_dir, mixed), dim3(grid_for(ntasks)), dim3(kBlock), 0, s, fines,
                           tasks, ntasks, active, scal, b0_idx, pin, pout, prp, ppap);
}

void launch_npcg_theta(hipStream_t s, int nprob, double *scal, const int *active)
{
    hipLaunchKernelGGL(k_npcg_theta, dim3((nprob + 63) / 64), dim3(64), 0, s, nprob, scal, active);
}

void launch_aa_reset(hipStream_t s, int nprob, int *aai)
{
    hipLaunchKernelGGL(k_aa_reset, dim3((nprob + 63) / 64), dim3(64), 0, s, nprob, aai);
}

void launch_aa_dots(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                    const int *active, int *aai, double *aad, int m, double *partials, int mixed)
{
    hipLaunchKernelGGL(FLD_PICK(k_aa_dots, mixed), dim3(grid_for(ntasks)), dim3(kBlock), 0, s,
                       fines, tasks, ntasks, active, aai, aad, m, partials);
}

void launch_aa_sums(hipStream_t s, int nprob, const int *range, const double *partials,
                    int ntasks, int *aai, double *aad, int m, const int *active)
{
    hipLaunchKernelGGL(k_aa_sums, dim3(2 * (m + 1), nprob), dim3(kBlock), 0, s, range, partials,
                       ntasks, aai, aad, m, active);
}

void launch_aa_solve(hipStream_t s, int nprob, double *scal, int *aai, double *aad, int m,
                     double reg, double growth, const int *active)
{
    hipLaunchKernelGGL(k_aa_solve, dim3(nprob), dim3(kWave), 0, s, nprob, scal, aai, aad, m, reg,
                       growth, active);
}

void launch_aa_update(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                      const int *active, int *aai, double *aad, int src, int dst, int mixed)
{
    hipLaunchKernelGGL(FLD_PICK(k_aa_update, mixed), dim3(grid_for(ntasks)), dim3(kBlock), 0, s,
                       fines, tasks, ntasks, active, aai, aad, src, dst);
}

int aa_max_window() { return kAaMax; }
int aa_state_ints() { return kAaInts; }
int aa_state_doubles() { return kAaDbls; }

void launch_alg1_pass(hipStream_t s, const Fine *fines, const Task *tasks, int ntasks,
                      const double *scal, int colour, double omega, double *partials)
{
    hipLaunchKernelGGL(k_alg1_pass, dim3(grid_for(ntasks)), dim3(kBlock), 0, s, fines, tasks,
                       ntasks, scal, colour, omega, partials);
}

void launch_put_fine(hipStream_t s, const Fine &f, Fine *dst)
{
    hipLaunchKernelGGL(k_put_fine, dim3(1), dim3(64), 0, s, f, dst);
}

template <typename T>
void launch_zero(hipStream_t s, const Grid *grids, const Task *tasks, int ntasks,
                 const int *active)
{
    hipLaunchKernelGGL(k_zero<T>, dim3(grid_for(ntasks)), dim3(kBlock), 0, s, grids, tasks, ntasks,
                       active);
}

template <typename T>
void launch_smooth(hipStream_t s, const Grid *grids, const Task *tasks, int ntasks,
                   const int *active, int colour, double omega, bool finest)
{
    hipLaunchKernelGGL(finest ? k_smooth_fine<T> : k_smooth<T>, dim3(grid_for(ntasks)),
                       dim3(kBlock), 0, s, grids, tasks, ntasks, active, colour, (T)omega);
}

template <typename T>
void launch_smooth_one(hipStream_t s, const Grid &g, int task_cells, int colour, double omega)
{
    const long long blocks = (g.n + task_cells - 1) / task_cells;
    if (blocks > 0)
        hipLaunchKernelGGL(k_smooth_one<T>, dim3((unsigned)blocks), dim3(kBlock), 0, s, g,
                           task_cells, colour, (T)omega);
}

template <typename T>
void launch_restrict(hipStream_t s, const Grid *grids, const Task *tasks, int ntasks,
                     const int *active, int sp)
{
    hipLaunchKernelGGL(FLD_PICK_SP(k_restrict, T, sp), dim3(grid_for(ntasks)), dim3(kBlock), 0, s,
                       grids, tasks, ntasks, active);
}

template <typename T>
void launch_prolong(hipStream_t s, const Grid *grids, const Task *tasks, int ntasks,
                    const int *active, int sp, double scale)
{
    hipLaunchKernelGGL(FLD_PICK_SP(k_prolong, T, sp), dim3(grid_for(ntasks)), dim3(kBlock), 0, s,
                       grids, tasks, ntasks, active, scale);
}

template <typename T>
void launch_galerkin(hipStream_t s, const Grid *grids, const Task *tasks, int ntasks,
                     const int *active, int sp)
{
    hipLaunchKernelGGL(FLD_PICK_SP(k_galerkin, T, sp), dim3(grid_for(ntasks)), dim3(kBlock), 0, s,
                       grids, tasks, ntasks, active);
}

template <typename T>
void launch_mean8_sa(hipStream_t s, const Grid *grids, const Task *tasks, int ntasks)
{
    hipLaunchKernelGGL(k_mean8_sa<T>, dim3(grid_for(ntasks)), dim3(kBlock), 0, s, grids, tasks,
                       ntasks);
}

template <typename T>
void launch_coarse_solve(hipStream_t s, const Grid *grids, const int *ids, int count,
                         const int *active, int *fail, int max_n, int max_bw)
{
    (void)max_bw;
    if (count > 0)
        hipLaunchKernelGGL(k_coarse_solve<T>, dim3(count), dim3(kBlock), kCholLds, s, grids, ids,
                           active, fail, max_n);
}

template <typename T>
void launch_smooth_rb(hipStream_t s, const Grid *grids, const LrTile *tiles, int ntiles,
                      const int *active, int first, int dir, double omega, int sp)
{
    if (ntiles > 0)
        hipLaunchKernelGGL(FLD_PICK_SP(k_smooth_rb, T, sp), dim3(std::min(8 * ((ntiles + 7) / 8), 4096)),
                           dim3(kLrThreads), 0, s, grids, tiles, ntiles, active, first, dir,
                           (T)omega);
}
template <typename T>
void launch_coarse_factor(hipStream_t s, const Grid *grids, const int *ids, int count,
                          const int *active, int *fail, int max_n)
{
    if (count > 0)
        hipLaunchKernelGGL(k_coarse_factor<T>, dim3(count), dim3(kBlock), kCholLds, s, grids, ids,
                           active, fail, max_n);
}
template <typename T>
void launch_tail(hipStream_t s, const Grid *grids, const int *roots, int count, const int *active,
                 int *fail, double omega, int lds_bytes)
{
    if (count > 0)
        hipLaunchKernelGGL(k_coarse_tail<T>, dim3(count), dim3(kTailBlock), lds_bytes, s, grids,
                           roots, active, fail, (T)omega);
}

long long tail_lds_need(long long nc, long long bw, long long deep_cells, long long scratch_cells,
                        int tsz)
{
    return tail_lds_bytes(nc, bw, deep_cells, scratch_cells, tsz);
}

int tail_lds_limit() { return kTailLds; }
int tail_root_cells() { return kTailRootCells; }
int tail_low_cells() { return kTailLowCells; }
int tail_max_low() { return kTailMaxLow; }

template <typename T>
void launch_deep(hipStream_t s, const Grid *grids, const int *roots, int count, const int *active,
                 double omega, bool down)
{
    if (count > 0)
        hipLaunchKernelGGL(down ? k_deep_down<T> : k_deep_up<T>, dim3(count), dim3(kDeepBlock), 0, s,
                           grids, roots, active, (T)omega);
}

#define FLD_INSTANTIATE(T)                                                                       \
    template void launch_zero<T>(hipStream_t, const Grid *, const Task *, int, const int *);     \
    template void launch_smooth<T>(hipStream_t, const Grid *, const Task *, int, const int *,    \
                                   int, double, bool);                                           \
    template void launch_smooth_one<T>(hipStream_t, const Grid &, int, int, double);             \
    template void launch_restrict<T>(hipStream_t, const Grid *, const Task *, int, const int *, int); \
    template void launch_prolong<T>(hipStream_t, const Grid *, const Task *, int, const int *, int,  \
                                    double);  \
    template void launch_galerkin<T>(hipStream_t, const Grid *, const Task *, int, const int *, int); \
    template void launch_mean8_sa<T>(hipStream_t, const Grid *, const Task *, int);              \
    template void launch_coarse_solve<T>(hipStream_t, const Grid *, const int *, int,            \
                                         const int *, int *, int, int);                          \
    template void launch_deep<T>(hipStream_t, const Grid *, const int *, int, const int *,       \
                                 double, bool);                                                  \
    template void launch_tail<T>(hipStream_t, const Grid *, const int *, int, const int *, int *,  \
                                 double, int);                                                   \
    template void launch_coarse_factor<T>(hipStream_t, const Grid *, const int *, int,           \
                                          const int *, int *, int);                              \
    template void launch_smooth_rb<T>(hipStream_t, const Grid *, const LrTile *, int,            \
                                      const int *, int, int, double, int);

FLD_INSTANTIATE(float)
FLD_INSTANTIATE(double)

}  // namespace fld
