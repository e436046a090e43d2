// fld_render.hip -- the steps around the solve on the GPU (gfx950): baking the
// single-scatter source of a directional light (Sec. 3 and Sec. 6) and the
// primary ray-march of the image from the fluence (Sec. 3).
//
// Layout as everywhere in libfld: nx*ny*nz float64 values, z fastest, so a
// column along z is contiguous.  One wavefront walks one column in chunks of
// 64 cells (one per lane); the optical depth in front of each cell is an
// exclusive prefix sum of sigma_t along the column, formed by a wave scan
// with a carry between chunks.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/fld.h"

namespace {

constexpr int kWave = 64;
constexpr int kBakeBlock = 256;      // four columns per block

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ inline double wave_inclusive_sum(double v, int lane)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const double u = __shfl_up(v, off, kWave);
        if (lane >= off)
            v = v + u;
    }
    return v;
}

// q = L * albedo * sigma_t * T, T = exp(-h (sum_{k'<k} sigma_t + sigma_t(k)/2)):
// the light travels +z and enters each column at its z = 0 face.
__global__ void __launch_bounds__(kBakeBlock)
k_light_bake(const double *__restrict__ sigma_t, const double *__restrict__ albedo, double light,
             long long ncol, int nz, double h, double *__restrict__ q)
{
    const int lane = threadIdx.x & (kWave - 1);
    const long long waves = (long long)gridDim.x * (kBakeBlock / kWave);
    for (long long col = (long long)blockIdx.x * (kBakeBlock / kWave) + threadIdx.x / kWave;
         col < ncol; col += waves) {
        const long long base = col * nz;
        double carry = 0.0;                 // optical depth of the chunks already done
        for (int z0 = 0; z0 < nz; z0 += kWave) {
            const int k = z0 + lane;
            const bool in = k < nz;
            const double s = in ? sigma_t[base + k] : 0.0;
            const double incl = wave_inclusive_sum(s, lane);
            const double prev = __shfl_up(incl, 1, kWave);
            const double before = carry + (lane > 0 ? prev : 0.0);
            if (in) {
                const double T = exp(-h * (before + 0.5 * s));
                q[base + k] = light * albedo[base + k] * s * T;
            }
            carry = carry + __shfl(incl, kWave - 1, kWave);
        }
    }
}

// Sum over the 64 lanes, the same value in every lane.
__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v = v + __shfl_xor(v, off, kWave);
    return v;
}

// Primary ray-march of an orthographic camera on the +z side: one ray per
// (i, j) column, travelling +z.  The sample of voxel k contributes
// h T Q with T = exp(-h (sigma_t(k)/2 + sum_{k' > k} sigma_t)) and
// 4 pi Q = src + albedo sigma_t phi; the back-light enters at z = 0.  The
// wave walks the column from the camera side down, lane l on voxel kt - l.
__global__ void __launch_bounds__(kBakeBlock)
k_render(const double *__restrict__ sigma_t, const double *__restrict__ albedo,
         const double *__restrict__ src, const double *__restrict__ phi, double background,
         long long ncol, int nz, double h, double *__restrict__ image)
{
    const double inv_four_pi = 1.0 / (4.0 * 3.14159265358979323846);
    const int lane = threadIdx.x & (kWave - 1);
    const long long waves = (long long)gridDim.x * (kBakeBlock / kWave);
    for (long long col = (long long)blockIdx.x * (kBakeBlock / kWave) + threadIdx.x / kWave;
         col < ncol; col += waves) {
        const long long base = col * nz;
        double carry = 0.0;                 // optical depth of the chunks nearer the camera
        double radiance = 0.0;
        for (int kt = nz - 1; kt >= 0; kt -= kWave) {
            const int k = kt - lane;
            const bool in = k >= 0;
            const double s = in ? sigma_t[base + k] : 0.0;
            const double incl = wave_inclusive_sum(s, lane);
            const double prev = __shfl_up(incl, 1, kWave);
            const double after = carry + (lane > 0 ? prev : 0.0);
            double contrib = 0.0;
            if (in) {
                const double T = exp(-h * (0.5 * s + after));
                const double Q = (src[base + k] + albedo[base + k] * s * phi[base + k]) * inv_four_pi;
                contrib = h * T * Q;
            }
            radiance = radiance + wave_sum(contrib);
            carry = carry + __shfl(incl, kWave - 1, kWave);
        }
        if (lane == 0)
            image[col] = radiance + background * exp(-h * carry);
    }
}

}  // namespace

extern "C" fld_status fld_render(const double *d_sigma_t, const double *d_albedo,
                                 const double *d_src, const double *d_phi, double background,
                                 int nx, int ny, int nz, double h, double *d_image,
                                 void *hip_stream)
{
    if (!d_sigma_t || !d_albedo || !d_src || !d_phi || !d_image || nx < 1 || ny < 1 || nz < 1)
        return FLD_ERR_INVALID_ARGUMENT;
    if (!(h > 0.0 && std::isfinite(h)) || !(background >= 0.0 && std::isfinite(background)))
        return FLD_ERR_INVALID_ARGUMENT;
    if ((long long)nx * ny * nz > (1LL << 40))
        return FLD_ERR_INVALID_ARGUMENT;
    const long long ncol = (long long)nx * ny;
    const long long blocks = (ncol + kBakeBlock / kWave - 1) / (kBakeBlock / kWave);
    const int grid = (int)(blocks < (1LL << 20) ? blocks : (1LL << 20));
    hipLaunchKernelGGL(k_render, dim3(grid), dim3(kBakeBlock), 0, (hipStream_t)hip_stream,
                       d_sigma_t, d_albedo, d_src, d_phi, background, ncol, nz, h, d_image);
    return hipGetLastError() == hipSuccess ? FLD_OK : FLD_ERR_DEVICE;
}

extern "C" fld_status fld_light_bake(const double *d_sigma_t, const double *d_albedo, double light,
                                     int nx, int ny, int nz, double h, double *d_q,
                                     void *hip_stream)
{
    if (!d_sigma_t || !d_albedo || !d_q || nx < 1 || ny < 1 || nz < 1)
        return FLD_ERR_INVALID_ARGUMENT;
    if (!(h > 0.0 && std::isfinite(h)) || !(light >= 0.0 && std::isfinite(light)))
        return FLD_ERR_INVALID_ARGUMENT;
    if ((long long)nx * ny * nz > (1LL << 40))
        return FLD_ERR_INVALID_ARGUMENT;
    const long long ncol = (long long)nx * ny;
    const long long blocks = (ncol + kBakeBlock / kWave - 1) / (kBakeBlock / kWave);
    const int grid = (int)(blocks < (1LL << 20) ? blocks : (1LL << 20));
    hipLaunchKernelGGL(k_light_bake, dim3(grid), dim3(kBakeBlock), 0, (hipStream_t)hip_stream,
                       d_sigma_t, d_albedo, light, ncol, nz, h, d_q);
    return hipGetLastError() == hipSuccess ? FLD_OK : FLD_ERR_DEVICE;
}
