// stage_u1.hpp -- one pass of the U(1) (Abelian-Higgs) lattice system, a = 1.
//
// Complex scalar phi = (phi0 + i phi1)/sqrt(2) (eq. ChargedScalars); psi = phi0 + i phi1.
// Links V_i(n) = exp(-i e dx A_i(n)); plaquette angle (U(1) toolkit, sec. 3.2)
//   theta_ij(n) = e dx [A_j(n+i) - A_j(n) - A_i(n+j) + A_i(n)],
// so that V_i V_{j,+i} V*_{i,+j} V*_j = exp(-i theta_ij).
// Forces, minus the derivative of the lattice Hamiltonian (sec. 5.5.2 kernels):
//   F_phi0 + i F_phi1 = dx^-2 sum_i [V_i psi(n+i) - 2 psi(n) + V*_i(n-i) psi(n-i)]
//                       - lambda/2 (|phi|^2 - v^2) psi
//   F_A_i = kappa_g J_i - (e dx^3)^-1 sum_{j != i} [sin theta_ij(n) - sin theta_ij(n-j)]
//   J_i   = (e/dx) Im[conj(psi(n)) V_i(n) psi(n+i)]
// Leapfrog pass: kick pi, piA by ck, then drift phi, A by hd (phi and A are read
// with neighbours and written to the other buffer; pi and piA in place).
// Energy pass (read only): momenta half-kicked by ck on the fly; energies
//   E_K^phi = (pi0^2 + pi1^2)/2, E_G^phi = sum_i |V_i psi(n+i) - psi(n)|^2 / (2 dx^2),
//   E_V = lambda/4 (|phi|^2 - v^2)^2, E_K^A = sum_i piA_i^2 / (2 kappa_g),
//   E_G^A = sum_{i<j} 2 sin^2(theta_ij/2) / (kappa_g e^2 dx^4),
// and the Gauss residual of the stored pairing (eq. GaussU1-eom at a = 1)
//   G = sum_i (piA_i(n) - piA_i(n-i))/dx - e kappa_g (phi0 pi1 - phi1 pi0).
#pragma once
#include "common.hpp"

namespace lat {

struct U1Args {
    const double *phi_in[2];
    double *phi_out[2];
    double *pi[2];
    const double *A_in[3];
    double *A_out[3];
    double *piA[3];
    int N, tiles_x, tiles_y;
    double dx, e, lam, v, kappa_g;
    double ck;   // kick weight
    double hd;   // drift weight
    double *partials;
    unsigned *ticket;
    ScaleRecord *sc;
};

enum U1Mode : int { kU1Step = 0, kU1Kick = 1, kU1Energy = 2 };
constexpr int kU1Sums = 8, kU1Maxes = 3;

__device__ inline size_t u1_at(int N, int x, int y, int z)
{
    return (size_t)x + (size_t)N * ((size_t)y + (size_t)N * (size_t)z);
}

template <int TX, int TY, int MODE>
__global__ void __launch_bounds__(TX *TY) u1_stage(const U1Args g)
{
    constexpr int NT = TX * TY;
    constexpr int NQ = kU1Sums + kU1Maxes;
    __shared__ double lds_red[(NT / 64) * NQ];
    __shared__ int last_flag;

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int lid = xcd_logical_block(blockIdx.x, gridDim.x);
    const int bx = lid % g.tiles_x;
    const int rest = lid / g.tiles_x;
    const int by = rest % g.tiles_y;
    const int z = rest / g.tiles_y;
    const int N = g.N;
    const int x = bx * TX + tx, y = by * TY + ty;
    const bool valid = x < N && y < N;

    double acc[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) acc[k] = 0.0;

    if (valid) {
        const int xm = x == 0 ? N - 1 : x - 1, xp = x + 1 == N ? 0 : x + 1;
        const int ym = y == 0 ? N - 1 : y - 1, yp = y + 1 == N ? 0 : y + 1;
        const int zm = z == 0 ? N - 1 : z - 1, zp = z + 1 == N ? 0 : z + 1;
        const size_t n = u1_at(N, x, y, z);
        const size_t nxp = u1_at(N, xp, y, z), nxm = u1_at(N, xm, y, z);
        const size_t nyp = u1_at(N, x, yp, z), nym = u1_at(N, x, ym, z);
        const size_t nzp = u1_at(N, x, y, zp), nzm = u1_at(N, x, y, zm);
        const double *Ax = g.A_in[0], *Ay = g.A_in[1], *Az = g.A_in[2];
        const double edx = g.e * g.dx;

        // plaquette angles at n and at n - j
        const double txy = edx * ((Ay[nxp] - Ay[n]) - Ax[nyp] + Ax[n]);
        const double txz = edx * ((Az[nxp] - Az[n]) - Ax[nzp] + Ax[n]);
        const double tyz = edx * ((Az[nyp] - Az[n]) - Ay[nzp] + Ay[n]);
        const double txy_xm = edx * ((Ay[n] - Ay[nxm]) - Ax[u1_at(N, xm, yp, z)] + Ax[nxm]);
        const double txz_xm = edx * ((Az[n] - Az[nxm]) - Ax[u1_at(N, xm, y, zp)] + Ax[nxm]);
        const double txy_ym = edx * ((Ay[u1_at(N, xp, ym, z)] - Ay[nym]) - Ax[n] + Ax[nym]);
        const double tyz_ym = edx * ((Az[n] - Az[nym]) - Ay[u1_at(N, x, ym, zp)] + Ay[nym]);
        const double txz_zm = edx * ((Az[u1_at(N, xp, y, zm)] - Az[nzm]) - Ax[n] + Ax[nzm]);
        const double tyz_zm = edx * ((Az[u1_at(N, x, yp, zm)] - Az[nzm]) - Ay[n] + Ay[nzm]);
        const double sxy = sin(txy), sxz = sin(txz), syz = sin(tyz);
        const double mag[3] = {(sxy - sin(txy_ym)) + (sxz - sin(txz_zm)),
                               (-sxy + sin(txy_xm)) + (syz - sin(tyz_zm)),
                               (-sxz + sin(txz_xm)) + (-syz + sin(tyz_ym))};

        // covariant Laplacian and current
        const double pr = g.phi_in[0][n], pim = g.phi_in[1][n];
        const size_t np_[3] = {nxp, nyp, nzp}, nm_[3] = {nxm, nym, nzm};
        double d2r = 0.0, d2i = 0.0, grad2 = 0.0, J[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double s, c, sm, cm;
            sincos(edx * g.A_in[i][n], &s, &c);
            sincos(edx * g.A_in[i][nm_[i]], &sm, &cm);
            s = -s;   // V_i(n) = c + i s ; conj(V_i(n-i)) = cm + i sm
            const double qr = g.phi_in[0][np_[i]], qi = g.phi_in[1][np_[i]];
            const double rr = g.phi_in[0][nm_[i]], ri = g.phi_in[1][nm_[i]];
            const double ar = c * qr - s * qi, ai = c * qi + s * qr;
            const double br = cm * rr - sm * ri, bi = cm * ri + sm * rr;
            d2r += ar - 2.0 * pr + br;
            d2i += ai - 2.0 * pim + bi;
            J[i] = g.e / g.dx * (pr * ai - pim * ar);
            if (MODE == kU1Energy) {
                const double dr = ar - pr, di = ai - pim;
                grad2 += dr * dr + di * di;
            }
        }
        const double m2 = 0.5 * (pr * pr + pim * pim);
        const double vp = 0.5 * g.lam * (m2 - g.v * g.v);
        const double inv_dx2 = 1.0 / (g.dx * g.dx);
        const double F0 = d2r * inv_dx2 - vp * pr;
        const double F1 = d2i * inv_dx2 - vp * pim;
        const double inv_edx3 = 1.0 / (g.e * g.dx * g.dx * g.dx);
        double FA[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) FA[i] = g.kappa_g * J[i] - mag[i] * inv_edx3;

        const double p0 = g.pi[0][n], p1 = g.pi[1][n];
        double pa[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) pa[i] = g.piA[i][n];

        if (MODE == kU1Energy) {
            const double s0 = p0 + g.ck * F0, s1 = p1 + g.ck * F1;
            acc[0] = 0.5 * (s0 * s0 + s1 * s1);
            acc[1] = grad2 * inv_dx2 * 0.5;
            const double u = m2 - g.v * g.v;
            acc[2] = 0.25 * g.lam * u * u;
            double ka = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double sa = pa[i] + g.ck * FA[i];
                ka += sa * sa;
            }
            acc[3] = ka / (2.0 * g.kappa_g);
            const double hxy = sin(0.5 * txy), hxz = sin(0.5 * txz), hyz = sin(0.5 * tyz);
            const double mg = 2.0 * hxy * hxy + 2.0 * hxz * hxz + 2.0 * hyz * hyz;
            acc[4] = mg / (g.kappa_g * g.e * g.e * g.dx * g.dx * g.dx * g.dx);
            // Gauss residual of the stored pairing
            const double div = ((pa[0] - g.piA[0][nxm]) + (pa[1] - g.piA[1][nym]) + (pa[2] - g.piA[2][nzm])) / g.dx;
            const double charge = g.e * g.kappa_g * (pr * p1 - pim * p0);
            const double G = div - charge;
            acc[5] = fabs(G);
            acc[6] = fabs(div + charge);
            acc[7] = fabs(div) + fabs(charge);
            acc[8] = fabs(G);
            acc[9] = fabs(div);
            acc[10] = fabs(charge);
        } else {
            const double q0 = p0 + g.ck * F0, q1 = p1 + g.ck * F1;
            g.pi[0][n] = q0;
            g.pi[1][n] = q1;
            double qa[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                qa[i] = pa[i] + g.ck * FA[i];
                g.piA[i][n] = qa[i];
            }
            if (MODE == kU1Step) {
                g.phi_out[0][n] = pr + g.hd * q0;
                g.phi_out[1][n] = pim + g.hd * q1;
#pragma unroll
                for (int i = 0; i < 3; ++i) g.A_out[i][n] = g.A_in[i][n] + g.hd * qa[i];
            }
        }
    }

    if constexpr (MODE == kU1Energy) {
        // block reduction: sums for [0, kU1Sums), maxes for the rest
        const int lane = tid & 63, w = tid >> 6;
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const double r = k < kU1Sums ? wave_sum(acc[k]) : wave_max(acc[k]);
            if (lane == 0) lds_red[w * NQ + k] = r;
        }
        __syncthreads();
        if (tid == 0) {
            for (int k = 0; k < NQ; ++k) {
                double r = 0.0;
                for (int i = 0; i < NT / 64; ++i)
                    r = k < kU1Sums ? r + lds_red[i * NQ + k] : fmax(r, lds_red[i * NQ + k]);
                store_agent(&g.partials[(size_t)lid * NQ + k], r);
            }
            const unsigned prev =
                __hip_atomic_fetch_add(g.ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            last_flag = (prev == gridDim.x - 1) ? 1 : 0;
        }
        __syncthreads();
        if (last_flag) {
            const int nb = gridDim.x;
            double part[NQ];
#pragma unroll
            for (int k = 0; k < NQ; ++k) part[k] = 0.0;
            for (int i = tid; i < nb; i += NT) {
#pragma unroll
                for (int k = 0; k < NQ; ++k) {
                    const double v = load_agent(&g.partials[(size_t)i * NQ + k]);
                    part[k] = k < kU1Sums ? part[k] + v : fmax(part[k], v);
                }
            }
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const double r = k < kU1Sums ? wave_sum(part[k]) : wave_max(part[k]);
                if (lane == 0) lds_red[w * NQ + k] = r;
            }
            __syncthreads();
            if (tid == 0) {
                for (int k = 0; k < NQ; ++k) {
                    double r = 0.0;
                    for (int i = 0; i < NT / 64; ++i)
                        r = k < kU1Sums ? r + lds_red[i * NQ + k] : fmax(r, lds_red[i * NQ + k]);
                    if (k < kU1Sums) g.sc->sums[k] = r;
                    else g.sc->maxes[k - kU1Sums] = r;
                }
                __hip_atomic_store(g.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

}  // namespace lat
