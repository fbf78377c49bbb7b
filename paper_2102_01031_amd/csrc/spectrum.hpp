// spectrum.hpp -- radial binning of the power of a real field's Fourier
// transform, for the discrete power spectrum of sec. 3.1 (eq. discretePS).
//
// Input: the half spectrum F(kz, ky, kx) of the unnormalised forward DFT of
// an N^3 real array (x fastest), kx in [0, N/2], as produced by a real-to-
// complex transform.  Mode n = (nx, ny, nz) with n_i in (-N/2, N/2]; the modes
// kx in (0, N/2) stand for themselves and their mirror images (-nx, -ny, -nz),
// which have the same |F| and |n|, so they count twice.  Bin b holds the modes
// with b <= |n| < b + 1.  Per block: sums of |F|^2 and mode counts per bin in
// LDS; a second kernel adds the block partials in block order.
#pragma once
#include "common.hpp"

namespace lat {

constexpr int kSpecThreads = 256;
constexpr int kSpecMaxBins = 448;   // >= floor(sqrt(3) 512/2) + 1

__global__ void __launch_bounds__(kSpecThreads) spectrum_bin(const double2 *__restrict__ F, int N, int nbins,
                                                             double *__restrict__ part_sum,
                                                             double *__restrict__ part_cnt)
{
    __shared__ double s_sum[kSpecMaxBins], s_cnt[kSpecMaxBins];
    for (int b = threadIdx.x; b < nbins; b += kSpecThreads) s_sum[b] = s_cnt[b] = 0.0;
    __syncthreads();
    const int H = N / 2 + 1;
    const size_t total = (size_t)N * N * H;
    for (size_t i = (size_t)blockIdx.x * kSpecThreads + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kSpecThreads) {
        const int kx = (int)(i % H);
        const size_t r = i / H;
        const int ky = (int)(r % N), kz = (int)(r / N);
        const long nx = kx, ny = ky <= N / 2 ? ky : ky - N, nz = kz <= N / 2 ? kz : kz - N;
        const long m = nx * nx + ny * ny + nz * nz;
        long b = (long)sqrt((double)m);
        while ((b + 1) * (b + 1) <= m) ++b;
        while (b * b > m) --b;
        if (b >= nbins) continue;
        const double w = (kx == 0 || 2 * kx == N) ? 1.0 : 2.0;
        const double2 f = F[i];
        atomicAdd(&s_sum[b], w * (f.x * f.x + f.y * f.y));
        atomicAdd(&s_cnt[b], w);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += kSpecThreads) {
        part_sum[(size_t)blockIdx.x * nbins + b] = s_sum[b];
        part_cnt[(size_t)blockIdx.x * nbins + b] = s_cnt[b];
    }
}

__global__ void spectrum_reduce(const double *__restrict__ part_sum, const double *__restrict__ part_cnt, int nblocks,
                                int nbins, double *__restrict__ sum, double *__restrict__ cnt)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    double s = 0.0, c = 0.0;
    for (int k = 0; k < nblocks; ++k) {
        s += part_sum[(size_t)k * nbins + b];
        c += part_cnt[(size_t)k * nbins + b];
    }
    sum[b] = s;
    cnt[b] = c;
}

// Seed of an adjoint from O = Delta(b) of one field (eq. discretePS).  With
// Delta(b) = c_b sum_{shell b} |F(n)|^2 over the full spectrum,
// dO/df(x) = 2 c_b sum_{shell b} Re[F(n) e^{+2 pi i n.x/N}]: the unnormalised
// complex-to-real inverse transform of the half spectrum kept on shell b and
// scaled by 2 c_b (the shell holds n with -n, so the masked spectrum stays
// Hermitian).  In place on F; also writes sum_{shell b} |F|^2 (mirror modes
// counted) to *out_sum, reduced in a fixed order: per thread, per wave, per
// block, then the last block adds the block partials in block order.
__global__ void __launch_bounds__(kSpecThreads) spectrum_shell_seed(double2 *__restrict__ F, int N, long bin,
                                                                    double scale, double *__restrict__ partials,
                                                                    unsigned *ticket, double *out_sum)
{
    __shared__ double lds_red[kSpecThreads / 64];
    __shared__ int last_flag;
    const int H = N / 2 + 1;
    const size_t total = (size_t)N * N * H;
    const size_t i = (size_t)blockIdx.x * kSpecThreads + threadIdx.x;
    double acc = 0.0;
    if (i < total) {
        const int kx = (int)(i % H);
        const size_t r = i / H;
        const int ky = (int)(r % N), kz = (int)(r / N);
        const long nx = kx, ny = ky <= N / 2 ? ky : ky - N, nz = kz <= N / 2 ? kz : kz - N;
        const long m = nx * nx + ny * ny + nz * nz;
        long b = (long)sqrt((double)m);
        while ((b + 1) * (b + 1) <= m) ++b;
        while (b * b > m) --b;
        double2 f = F[i];
        if (b == bin) {
            const double w = (kx == 0 || 2 * kx == N) ? 1.0 : 2.0;
            acc = w * (f.x * f.x + f.y * f.y);
            f.x *= scale;
            f.y *= scale;
        } else {
            f.x = f.y = 0.0;
        }
        F[i] = f;
    }
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const double ws = wave_sum(acc);
    if (lane == 0) lds_red[w] = ws;
    __syncthreads();
    if (tid == 0) {
        double sb = 0.0;
        for (int k = 0; k < kSpecThreads / 64; ++k) sb += lds_red[k];
        store_agent(&partials[blockIdx.x], sb);
        last_flag = ticket_arrive(ticket, gridDim.x) ? 1 : 0;
    }
    __syncthreads();
    if (last_flag) {
        double part = 0.0;
        for (int k = tid; k < (int)gridDim.x; k += kSpecThreads) part += load_agent(&partials[k]);
        const double pw = wave_sum(part);
        if (lane == 0) lds_red[w] = pw;
        __syncthreads();
        if (tid == 0) {
            double sb = 0.0;
            for (int k = 0; k < kSpecThreads / 64; ++k) sb += lds_red[k];
            *out_sum = sb;
            __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Shell sums for the lattice occupation number (eq. OccuppationNum) of one
// real field: from the half spectra F of phi and P of pi, per bin the sums of
// |F|^2, of |cp P + hub F|^2 (the transform of phi' + (a'/a) phi with
// phi' = cp pi, cp = a^{alpha-3}, hub = a'/a) and the mode count, mirror modes
// counted as in spectrum_bin.  Per-block LDS sums, then one row per block.
__global__ void __launch_bounds__(kSpecThreads) occupation_bin(const double2 *__restrict__ F,
                                                               const double2 *__restrict__ P, int N, int nbins,
                                                               double cp, double hub, double *__restrict__ part,
                                                               size_t stride)
{
    __shared__ double s_f[kSpecMaxBins], s_x[kSpecMaxBins], s_c[kSpecMaxBins];
    for (int b = threadIdx.x; b < nbins; b += kSpecThreads) s_f[b] = s_x[b] = s_c[b] = 0.0;
    __syncthreads();
    const int H = N / 2 + 1;
    const size_t total = (size_t)N * N * H;
    for (size_t i = (size_t)blockIdx.x * kSpecThreads + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kSpecThreads) {
        const int kx = (int)(i % H);
        const size_t r = i / H;
        const int ky = (int)(r % N), kz = (int)(r / N);
        const long nx = kx, ny = ky <= N / 2 ? ky : ky - N, nz = kz <= N / 2 ? kz : kz - N;
        const long m = nx * nx + ny * ny + nz * nz;
        long b = (long)sqrt((double)m);
        while ((b + 1) * (b + 1) <= m) ++b;
        while (b * b > m) --b;
        if (b >= nbins) continue;
        const double w = (kx == 0 || 2 * kx == N) ? 1.0 : 2.0;
        const double2 f = F[i], p = P[i];
        const double xr = cp * p.x + hub * f.x, xi = cp * p.y + hub * f.y;
        atomicAdd(&s_f[b], w * (f.x * f.x + f.y * f.y));
        atomicAdd(&s_x[b], w * (xr * xr + xi * xi));
        atomicAdd(&s_c[b], w);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += kSpecThreads) {
        part[(size_t)blockIdx.x * nbins + b] = s_f[b];
        part[stride + (size_t)blockIdx.x * nbins + b] = s_x[b];
        part[2 * stride + (size_t)blockIdx.x * nbins + b] = s_c[b];
    }
}

// nq quantities of per-block rows (quantity q at part + q stride) added in
// block order: tot[q * tot_stride + b]
__global__ void spectrum_reduce_q(const double *__restrict__ part, size_t stride, int nblocks, int nbins, int nq,
                                  double *__restrict__ tot, int tot_stride)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (b >= nbins || q >= nq) return;
    double s = 0.0;
    for (int k = 0; k < nblocks; ++k) s += part[q * stride + (size_t)k * nbins + b];
    tot[(size_t)q * tot_stride + b] = s;
}

// Sums of squares of up to two real arrays of n values (f1 may be null): per
// block part[2 block + s]; fixed grid, so the result does not vary run to run.
template <typename T>
__global__ void __launch_bounds__(kSpecThreads) sumsq_blocks(const T *__restrict__ f0, const T *__restrict__ f1,
                                                             size_t n, double *__restrict__ part)
{
    __shared__ double lds[2][kSpecThreads / 64];
    double a0 = 0.0, a1 = 0.0;
    for (size_t i = (size_t)blockIdx.x * kSpecThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kSpecThreads) {
        const double u = (double)f0[i];
        a0 += u * u;
        if (f1) {
            const double v = (double)f1[i];
            a1 += v * v;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double w0 = wave_sum(a0), w1 = wave_sum(a1);
    if (lane == 0) {
        lds[0][w] = w0;
        lds[1][w] = w1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double s = 0.0;
        for (int k = 0; k < kSpecThreads / 64; ++k) s += lds[threadIdx.x][k];
        part[2 * blockIdx.x + threadIdx.x] = s;
    }
}

__global__ void sumsq_reduce(const double *__restrict__ part, int nblocks, double *__restrict__ tot)
{
    const int s = threadIdx.x;
    if (s >= 2) return;
    double acc = 0.0;
    for (int k = 0; k < nblocks; ++k) acc += part[2 * k + s];
    tot[s] = acc;
}

// widen a float32 field into the float64 transform input
__global__ void widen_f32(const float *__restrict__ in, double *__restrict__ out, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = (double)in[i];
}

}  // namespace lat
