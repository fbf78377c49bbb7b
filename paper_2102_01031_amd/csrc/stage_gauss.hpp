// stage_gauss.hpp -- Gauss-consistent initial gauge momenta (sec. 5.5.1, eqs.
// kAi1 and GaugeCurrentFluc on the lattice).  With the links at the identity
// the Gauss law is the plain lattice divergence div- E = rho; its
// longitudinal solution is E_i = grad+_i chi with Lap chi = rho - <rho>,
// Lap = sum_i grad-_i grad+_i, whose Fourier symbol is
// -L(k) = -(4/dx^2) sum_i sin^2(pi k_i / N).  The charge density goes through
// a float64 real-to-complex transform (hipFFT), this file's symbol kernel,
// the inverse transform, and the forward-difference kernel.
#pragma once
#include "common.hpp"
#include "stage_su2.hpp"

namespace lat {

// SU(2) charge of colour a: rho(n) = g Im(psi^dag T_a pi_psi); flags any link
// that is not exactly the identity (the solve assumes unit links).
__global__ void gauss_charge_su2(const double *const *dbl, const double *const *dpi, const double *const *lnk,
                                 double g, int a, size_t V, double *__restrict__ rho, int *__restrict__ off_identity)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < V; n += (size_t)gridDim.x * blockDim.x) {
        double j[3];
        isospin(dbl[0][n], dbl[1][n], dbl[2][n], dbl[3][n], dpi[0][n], dpi[1][n], dpi[2][n], dpi[3][n], j[0], j[1],
                j[2]);
        rho[n] = g * j[a];
        if (a == 0) {
            bool bad = false;
#pragma unroll
            for (int i = 0; i < 3; ++i)
                bad |= lnk[4 * i][n] != 1.0 || lnk[4 * i + 1][n] != 0.0 || lnk[4 * i + 2][n] != 0.0 ||
                       lnk[4 * i + 3][n] != 0.0;
            if (bad) *off_identity = 1;
        }
    }
}

// U(1) charge: rho(n) = e kappa_g (phi0 pi1 - phi1 pi0)
__global__ void gauss_charge_u1(const double *__restrict__ p0, const double *__restrict__ p1,
                                const double *__restrict__ q0, const double *__restrict__ q1, double ek, size_t V,
                                double *__restrict__ rho)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < V; n += (size_t)gridDim.x * blockDim.x)
        rho[n] = ek * (p0[n] * q1[n] - p1[n] * q0[n]);
}

// chi~ = -rho~ / L(k) on the half spectrum (kx in [0, N/2]), chi~(0) = 0
__global__ void gauss_symbol(double2 *__restrict__ F, int N, double dx)
{
    const int NH = N / 2 + 1;
    const size_t H = (size_t)N * N * NH;
    const double pi = 3.14159265358979323846;
    for (size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x; m < H; m += (size_t)gridDim.x * blockDim.x) {
        const int kx = (int)(m % NH);
        const int ky = (int)((m / NH) % N);
        const int kz = (int)(m / ((size_t)NH * N));
        const double sx = sin(pi * kx / N), sy = sin(pi * ky / N), sz = sin(pi * kz / N);
        const double L = 4.0 / (dx * dx) * (sx * sx + sy * sy + sz * sz);
        double2 v = F[m];
        if (m == 0) {
            v.x = 0.0;
            v.y = 0.0;
        } else {
            v.x = -v.x / L;
            v.y = -v.y / L;
        }
        F[m] = v;
    }
}

// E_i(n) = (chi(n + i) - chi(n)) / dx with chi = inv_vol * the unnormalised inverse transform
__global__ void gauss_field(const double *__restrict__ chi, int N, double scale, double *__restrict__ e0,
                            double *__restrict__ e1, double *__restrict__ e2)
{
    const size_t V = (size_t)N * N * N;
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < V; n += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(n % N), y = (int)((n / N) % N), z = (int)(n / ((size_t)N * N));
        const size_t nx = (size_t)(x + 1 == N ? 0 : x + 1) + (size_t)N * ((size_t)y + (size_t)N * z);
        const size_t ny = (size_t)x + (size_t)N * ((size_t)(y + 1 == N ? 0 : y + 1) + (size_t)N * z);
        const size_t nz = (size_t)x + (size_t)N * ((size_t)y + (size_t)N * (size_t)(z + 1 == N ? 0 : z + 1));
        const double c = chi[n];
        e0[n] = (chi[nx] - c) * scale;
        e1[n] = (chi[ny] - c) * scale;
        e2[n] = (chi[nz] - c) * scale;
    }
}

}  // namespace lat
