// stage_slab.hpp -- several leapfrog steps per launch for small lattices:
// temporal blocking with the block's window of planes in LDS.
//
// One block owns ZS consecutive z planes and YB consecutive y rows of each
// (all N columns in x, so x needs no halo).  For S steps it holds a window of
// ZS + 2 S planes by YB + 2 S rows (S extra on either side in z and y), one
// thread per (x, row) column of the window; step s (s = 0 .. S-1) advances the
// sites whose plane and row both lie in [s + 1, extent - 2 - s] of the window
// -- one plane and one row fewer on either side per step, the ones whose
// neighbours are still up to date -- so after S steps the block's own sites
// hold the state S steps later, exactly as S single-step passes would leave
// them.  Each step is the leapfrog pass of stage_scalar.hpp (kick, then drift
// of the kicked momenta; sec. 4.5.2):
//   F = ka1 Lap phi - ka3 dV/dphi,  pi += c1 F (+ c2 F),  phi += dend pi
// with the same expression order.
//
// A thread keeps its whole column (phi and pi of every window plane) in
// registers: the z neighbours are its own values, and only the four in-plane
// neighbours go through LDS, where each step publishes the planes it advances
// (write, barrier, read, barrier).  All global loads of the window are issued
// before the first use, and the step coefficients are staged in LDS with
// them.  Planes are read from the input arrays (periodic in y and z) and the
// block's own sites written to the output arrays, so blocks never read each
// other's results within a launch.  A launch may run fewer steps than S (the
// tail of a call): the own sites stay inside the advanced range.  Only for
// coefficients known before the launch: no expansion or a fixed background
// (no volume reduction between steps).
#pragma once
#include "common.hpp"

namespace lat {

constexpr int kSlabMaxThreads = 1024;

template <typename T>
struct SlabArgs {
    const T *phi_in[2], *pi_in[2];
    T *phi_out[2], *pi_out[2];
    int N, yb, steps;        // rows per block (the last band may own fewer), steps of this launch (1 .. S)
    double inv_dx2, lam, q;
    const PassCoef *coef;    // coefficients of the launch's first step, then one per step
};

// LDS the kernel needs: the step coefficients, then phi of the ZS + 2 S - 2
// advanced planes of each field, YB + 2 S rows of N sites each
template <int S>
constexpr size_t kSlabCoefBytes = (5 * S * sizeof(double) + 255) / 256 * 256;
template <typename T, int NF, int S, int ZS>
constexpr size_t slab_lds(int N, int yb)
{
    return kSlabCoefBytes<S> + (size_t)NF * (ZS + 2 * S - 2) * (size_t)(yb + 2 * S) * N * sizeof(T);
}

template <typename T, int NF, int S, int ZS>
__global__ void __launch_bounds__(kSlabMaxThreads) lf_slab(const SlabArgs<T> g)
{
    constexpr int RZ = ZS + 2 * S;               // planes of the window
    constexpr int RL = RZ - 2;                   // planes published in LDS (k = 1 .. RZ - 2)
    extern __shared__ __attribute__((aligned(16))) unsigned char slab_lds_raw[];
    const int N = g.N, NN = N * N;
    const int RY = g.yb + 2 * S, PN = RY * N;    // rows of the window, sites of a window plane
    double *const Cl = (double *)slab_lds_raw;   // [step][c1, c2, dend, ka1, ka3]
    T *const L = (T *)(slab_lds_raw + kSlabCoefBytes<S>);   // [f][k - 1][row][x]
    const int z0 = blockIdx.x * ZS, y0 = blockIdx.y * g.yb;
    const int tid = threadIdx.x;
    const int x = tid % N, yy = tid / N;         // column of the window
    const bool on = yy < RY;
    // neighbours in the window plane: periodic in x, y +- 1 inside the window
    const int sxp = x + 1 == N ? tid - x : tid + 1, sxm = x == 0 ? tid + N - 1 : tid - 1;
    const int syp = tid + N, sym = tid - N;
    auto LP = [&](int f, int k) { return L + ((size_t)f * RL + (k - 1)) * PN; };

    int y = (y0 - S + yy) % N;
    if (y < 0) y += N;
    T ph[NF][RZ], pv[NF][RZ];
    if (on) {
#pragma unroll
        for (int k = 0; k < RZ; ++k) {
            int z = (z0 - S + k) % N;
            if (z < 0) z += N;
            const size_t o = (size_t)z * NN + (size_t)y * N + x;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                ph[f][k] = g.phi_in[f][o];
                pv[f][k] = (k >= 1 && k <= RZ - 2) ? g.pi_in[f][o] : T(0);
            }
        }
    }
    if (tid < 5 * S) {
        const int s = tid / 5, m = tid % 5;
        const PassCoef *C = g.coef + (s < g.steps ? s : 0);
        Cl[tid] = m == 0 ? C->c1 : m == 1 ? C->c2 : m == 2 ? C->dend : m == 3 ? C->ka1 : C->ka3;
    }

    const T idx2 = (T)g.inv_dx2, lam = (T)g.lam, qc = (T)g.q;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        if (s >= g.steps) break;
        if (s > 0) __syncthreads();              // the previous step's neighbour reads are done
        if (on) {
#pragma unroll
            for (int k = s + 1; k <= RZ - 2 - s; ++k)
#pragma unroll
                for (int f = 0; f < NF; ++f) LP(f, k)[tid] = ph[f][k];
        }
        __syncthreads();                         // (the first one also publishes the coefficients)
        const T c1 = (T)Cl[5 * s], c2 = (T)Cl[5 * s + 1], de = (T)Cl[5 * s + 2], ka1 = (T)Cl[5 * s + 3],
                ka3 = (T)Cl[5 * s + 4];
        if (yy >= s + 1 && yy <= RY - 2 - s) {
#pragma unroll
            for (int k = s + 1; k <= RZ - 2 - s; ++k) {
                T lap[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const T *P = LP(f, k);
                    const T c0 = ph[f][k];
                    lap[f] = ((P[sxp] - T(2) * c0 + P[sxm]) + (P[syp] - T(2) * c0 + P[sym]) +
                              (ph[f][k + 1] - T(2) * c0 + ph[f][k - 1])) * idx2;
                }
                T dV[NF];
                if constexpr (NF == 1) {
                    const T u = ph[0][k];
                    dV[0] = lam * u * u * u;
                } else {
                    const T u = ph[0][k], w = ph[1][k];
                    dV[0] = lam * u * u * u + qc * u * w * w;
                    dV[1] = qc * u * u * w;
                }
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const T F = ka1 * lap[f] - ka3 * dV[f];
                    const T pm = pv[f][k] + c1 * F;
                    pv[f][k] = pm + c2 * F;
                }
            }
            // drift after every kick of the step: the kicks above read the
            // pre-drift phi of the z neighbours from these registers
#pragma unroll
            for (int k = s + 1; k <= RZ - 2 - s; ++k)
#pragma unroll
                for (int f = 0; f < NF; ++f) ph[f][k] = ph[f][k] + de * pv[f][k];
        }
    }

    // the own sites: rows [S, S + yb) and planes [S, S + ZS) of the window,
    // fewer in the last band or slab when yb or ZS does not divide N
    if (yy >= S && yy < S + g.yb && y0 + yy - S < N) {
#pragma unroll
        for (int k = S; k < S + ZS; ++k) {
            const int z = z0 + k - S;
            if (z >= N) break;
            const size_t o = (size_t)z * NN + (size_t)y * N + x;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                g.phi_out[f][o] = ph[f][k];
                g.pi_out[f][o] = pv[f][k];
            }
        }
    }
}

}  // namespace lat
