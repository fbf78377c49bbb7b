// stage_adjoint.hpp -- reverse step and adjoint of the velocity-Verlet map for
// two real fields with V = lambda/4 phi^4 + q/2 phi^2 chi^2, at a = 1 or on a
// fixed background a(t).
//
// A run of VV2 steps is a leapfrog whose pass p does
//   pi <- pi + cA F(phi_p) + cB F(phi_p);  phi_{p+1} = phi_p + h d_p pi,
// with F = kL Lap phi - kV grad V (sec. 4.5.2 kernel; kL = a_p^{1+alpha},
// kV = a_p^{3+alpha} at the kick time t_p), d_p = a(t_p + h/2)^{alpha-3},
// cA = h/2 (0 at the first point) and cB = h/2.  The reverse pass p, fused,
// does per site (dphi = -h d_p, dlam = h d_p):
//   reverse drift   phi_p  = phi_{p+1} + dphi pi       (on load, all stencil points)
//   adjoint drift   lpi    = lpi + dlam lphi           (on load, all stencil points)
//   reverse kick    pi     = (pi - cB F(phi_p)) - cA F(phi_p)
//   adjoint kick    lphi  += (cB + cA) [kL Lap lpi - kV H_V(phi_p) lpi]   (dF is symmetric)
//   coupling        dO/dq += (cA + cB) sum_n lpi . dF/dq,  dF/dq = -kV (phi chi^2, phi^2 chi)
// with the Hessian H_V = [[3 lambda phi^2 + q chi^2, 2 q phi chi], [2 q phi chi, q phi^2]].
// All four arrays of both fields are read with a one-site halo and written to
// the other buffer of their ping-pong pair.  Layout and tiling follow the
// scalar stage kernel: TX x TY column tiles marching through z chunks, drifted
// values of the current plane in LDS, z neighbours in a register window.
#pragma once
#include "common.hpp"

namespace lat {

struct AdjArgs {
    const double *phi_in[2], *pi_in[2], *lphi_in[2], *lpi_in[2];
    double *phi_out[2], *pi_out[2], *lphi_out[2], *lpi_out[2];
    int N, zc, tiles_x, tiles_y;
    double inv_dx2, lam, q;
    double dphi, dlam;   // drifts on load: phi += dphi * pi, lpi += dlam * lphi
    double cA, cB;       // the two half kicks of the forward pass
    double kL, kV;       // kernel factors a^{1+alpha}, a^{3+alpha} at this kick point
    double *partials;
    unsigned *ticket;
    double *dq_acc;      // device accumulator of dO/dq
    // if not null: each block adds its partial of dO/dq to its own slot (one
    // per block, summed by adj_dq_finish after the sweep) instead of a ticketed
    // last block adding the pass's sum to dq_acc
    double *dq_slots;
};

template <int TX, int TY>
__global__ void __launch_bounds__(TX *TY) adjoint_stage(const AdjArgs g)
{
    constexpr int NT = TX * TY;
    constexpr int NH = 2 * TX + 2 * TY;
    constexpr int LX = TX + 2;
    constexpr int NA = 4;   // LDS arrays: phi_0, phi_1, lpi_0, lpi_1 (drifted)
    static_assert(NH <= NT, "halo cells exceed the block's threads");
    __shared__ double lds[2][NA][(TY + 2) * LX];
    __shared__ double lds_red[NT / 64];
    __shared__ int last_flag;

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int lid = xcd_logical_block(blockIdx.x, gridDim.x);
    const int bx = lid % g.tiles_x;
    const int rest = lid / g.tiles_x;
    const int by = rest % g.tiles_y;
    const int bz = rest / g.tiles_y;
    const int N = g.N;
    const int x0 = bx * TX, y0 = by * TY;
    const int z0 = bz * g.zc;
    const int z1 = min(z0 + g.zc, N);
    const size_t NN = (size_t)N * (size_t)N;
    const bool valid = (x0 + tx < N) && (y0 + ty < N);
    const int own = ((x0 + tx) % N) + N * ((y0 + ty) % N);
    const int oslot = (1 + ty) * LX + 1 + tx;
    const bool has_halo = tid < NH;
    int hslot = 0, hoff = 0;
    if (has_halo) {
        int hx, hy, sx, sy;
        if (tid < TX) {
            sx = 1 + tid; sy = 0; hx = x0 + tid; hy = y0 - 1;
        } else if (tid < 2 * TX) {
            sx = 1 + tid - TX; sy = TY + 1; hx = x0 + tid - TX; hy = y0 + TY;
        } else if (tid < 2 * TX + TY) {
            sx = 0; sy = 1 + tid - 2 * TX; hx = x0 - 1; hy = y0 + tid - 2 * TX;
        } else {
            sx = TX + 1; sy = 1 + tid - 2 * TX - TY; hx = x0 + TX; hy = y0 + tid - 2 * TX - TY;
        }
        hx = ((hx % N) + N) % N;
        hy = ((hy % N) + N) % N;
        hslot = sy * LX + sx;
        hoff = hx + N * hy;
    }
    const double dph = g.dphi, dla = g.dlam, cA = g.cA, cB = g.cB;
    const double lam = g.lam, qc = g.q, idx2 = g.inv_dx2, kL = g.kL, kV = g.kV;

    // array a of a raw 4-tuple: 0 phi, 1 pi, 2 lphi, 3 lpi ; stencil quantities:
    // S0 = phi + dph * pi (fields 0, 1), S1 = lpi + dla * lphi (fields 0, 1)
    auto ld4 = [&](size_t o, double (&r)[2][4]) {
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            r[f][0] = g.phi_in[f][o];
            r[f][1] = g.pi_in[f][o];
            r[f][2] = g.lphi_in[f][o];
            r[f][3] = g.lpi_in[f][o];
        }
    };
    auto sten = [&](const double (&r)[2][4], double (&s)[NA]) {
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            s[f] = r[f][0] + dph * r[f][1];
            s[2 + f] = r[f][3] + dla * r[f][2];
        }
    };

    double wm[NA], w0[NA], wp[NA];   // drifted stencil values at z-1, z, z+1 (own column)
    double r0[2][4], r1[2][4];       // raw own values at z and z+1
    double oA[2][4], oB[2][4];       // own raw plane z+2 / z+3 in flight
    double hA[2][4], hB[2][4];       // halo raw plane z+1 / z+2 in flight
    {
        const size_t om = (size_t)(z0 == 0 ? N - 1 : z0 - 1) * NN;
        const size_t o0 = (size_t)z0 * NN;
        const size_t o1 = (size_t)((z0 + 1) % N) * NN;
        const size_t o2 = (size_t)(min(z0 + 2, z1) % N) * NN;
        const size_t oh1 = (size_t)(min(z0 + 1, z1 - 1) % N) * NN;
        double t[2][4];
        ld4(om + own, t);
        sten(t, wm);
        ld4(o0 + own, r0);
        sten(r0, w0);
        ld4(o1 + own, r1);
        sten(r1, wp);
        ld4(o2 + own, oA);
#pragma unroll
        for (int a = 0; a < NA; ++a) lds[0][a][oslot] = w0[a];
        if (has_halo) {
            ld4(o0 + hoff, t);
            double s[NA];
            sten(t, s);
#pragma unroll
            for (int a = 0; a < NA; ++a) lds[0][a][hslot] = s[a];
            ld4(oh1 + hoff, hA);
        }
    }
    __syncthreads();

    double dq = 0.0;
    auto plane = [&](const int z, double (&oi)[2][4], double (&hi)[2][4], double (&oo)[2][4],
                     double (&ho)[2][4]) {
        const int cur = (z - z0) & 1, nxt = cur ^ 1;
        int zo = min(z + 3, z1);
        if (zo >= N) zo -= N;
        int zh = min(z + 2, z1 - 1);
        if (zh >= N) zh -= N;
        ld4((size_t)zo * NN + own, oo);
        if (has_halo) ld4((size_t)zh * NN + hoff, ho);
        if (z + 1 < z1) {
#pragma unroll
            for (int a = 0; a < NA; ++a) lds[nxt][a][oslot] = wp[a];
            if (has_halo) {
                double s[NA];
                sten(hi, s);
#pragma unroll
                for (int a = 0; a < NA; ++a) lds[nxt][a][hslot] = s[a];
            }
        }
        {
            double lap[NA];
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const double *L = lds[cur][a];
                const double c0 = w0[a];
                lap[a] = ((L[oslot + 1] - 2.0 * c0 + L[oslot - 1]) + (L[oslot + LX] - 2.0 * c0 + L[oslot - LX]) +
                          (wp[a] - 2.0 * c0 + wm[a])) * idx2;
            }
            const double u = w0[0], v = w0[1], l0 = w0[2], l1 = w0[3];
            const double F0 = kL * lap[0] - kV * (lam * u * u * u + qc * u * v * v);
            const double F1 = kL * lap[1] - kV * (qc * u * u * v);
            const double h00 = 3.0 * lam * u * u + qc * v * v, h01 = 2.0 * qc * u * v, h11 = qc * u * u;
            const double G0 = kL * lap[2] - kV * (h00 * l0 + h01 * l1);
            const double G1 = kL * lap[3] - kV * (h01 * l0 + h11 * l1);
            const size_t oz = (size_t)z * NN + own;
            if (valid) {
                dq += (cA + cB) * kV * (-(l0 * u * v * v) - (l1 * u * u * v));
                const double np0 = (r0[0][1] - cB * F0) - cA * F0;
                const double np1 = (r0[1][1] - cB * F1) - cA * F1;
                const double nl0 = (r0[0][2] + cB * G0) + cA * G0;
                const double nl1 = (r0[1][2] + cB * G1) + cA * G1;
                __builtin_nontemporal_store(u, &g.phi_out[0][oz]);
                __builtin_nontemporal_store(v, &g.phi_out[1][oz]);
                __builtin_nontemporal_store(np0, &g.pi_out[0][oz]);
                __builtin_nontemporal_store(np1, &g.pi_out[1][oz]);
                __builtin_nontemporal_store(nl0, &g.lphi_out[0][oz]);
                __builtin_nontemporal_store(nl1, &g.lphi_out[1][oz]);
                __builtin_nontemporal_store(l0, &g.lpi_out[0][oz]);
                __builtin_nontemporal_store(l1, &g.lpi_out[1][oz]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            wm[a] = w0[a];
            w0[a] = wp[a];
        }
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int k = 0; k < 4; ++k) r0[f][k] = r1[f][k];
        sten(oi, wp);
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int k = 0; k < 4; ++k) r1[f][k] = oi[f][k];
    };

    for (int z = z0; z < z1; z += 2) {
        plane(z, oA, hA, oB, hB);
        if (z + 1 < z1) plane(z + 1, oB, hB, oA, hA);
    }

    // deterministic reduction of the coupling sensitivity
    const int lane = tid & 63, w = tid >> 6;
    const double ws = wave_sum(dq);
    if (lane == 0) lds_red[w] = ws;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int i = 0; i < NT / 64; ++i) s += lds_red[i];
        if (g.dq_slots) {
            g.dq_slots[lid] += s;   // this block's slot: no other block writes it
            last_flag = 0;
        } else {
            store_agent(&g.partials[lid], s);
            last_flag = ticket_arrive(g.ticket, gridDim.x) ? 1 : 0;
        }
    }
    __syncthreads();
    if (last_flag) {
        double part = 0.0;
        for (int i = tid; i < (int)gridDim.x; i += NT) part += load_agent(&g.partials[i]);
        const double pw = wave_sum(part);
        if (lane == 0) lds_red[w] = pw;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int i = 0; i < NT / 64; ++i) s += lds_red[i];
            *g.dq_acc += s;
            __hip_atomic_store(g.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Seed of the adjoint from O = (E_K^f + E_G^f)/rho, the energy fraction of
// field f, at scale factor a (sec. 4.4 energies, eq. EK_EG_EV: E_K =
// <pi^2>/(2 a^6), E_G = <|grad phi|^2>/(2 a^2)):  with w_s = [s == f] and V = N^3,
//   dO/dpi_s  = (w_s - O) pi_s / (a^6 V rho)
//   dO/dphi_s = (w_s (-Lap phi_s)/a^2 - O (-Lap phi_s/a^2 + dV/dphi_s)) / (V rho)
// and the sum of phi^2 chi^2 / 2 for the explicit coupling derivative.
struct SeedArgs {
    const double *phi[2], *pi[2];
    double *lphi[2], *lpi[2];
    int N;
    int field;           // f of the energy fraction
    double inv_dx2, lam, q, O, inv_vrho;
    double ia2, ia6;     // 1/a^2, 1/a^6 at the final time
    double *partials;
    unsigned *ticket;
    double *out_sum;
};

__global__ void __launch_bounds__(256) adjoint_seed(const SeedArgs g)
{
    __shared__ double lds_red[4];
    __shared__ int last_flag;
    const int N = g.N;
    const size_t V = (size_t)N * N * N;
    const size_t n = (size_t)blockIdx.x * 256 + threadIdx.x;
    double acc = 0.0;
    if (n < V) {
        const int x = (int)(n % N), y = (int)((n / N) % N), z = (int)(n / ((size_t)N * N));
        const size_t xp = n - x + (x + 1 == N ? 0 : x + 1), xm = n - x + (x == 0 ? N - 1 : x - 1);
        const size_t yp = n + (size_t)((y + 1 == N ? 0 : y + 1) - y) * N, ym = n + (size_t)((y == 0 ? N - 1 : y - 1) - y) * N;
        const size_t NN = (size_t)N * N;
        const size_t zp = n + (size_t)((z + 1 == N ? 0 : z + 1) - z) * NN, zm = n + (size_t)((z == 0 ? N - 1 : z - 1) - z) * NN;
        const double u = g.phi[0][n], v = g.phi[1][n];
        const double dV[2] = {g.lam * u * u * u + g.q * u * v * v, g.q * u * u * v};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const double *P = g.phi[s];
            const double c = P[n];
            const double lap = ((P[xp] - 2.0 * c + P[xm]) + (P[yp] - 2.0 * c + P[ym]) + (P[zp] - 2.0 * c + P[zm])) * g.inv_dx2;
            const double wsel = s == g.field ? 1.0 : 0.0;
            g.lphi[s][n] = (wsel * (-lap) * g.ia2 - g.O * (-lap * g.ia2 + dV[s])) * g.inv_vrho;
            g.lpi[s][n] = (wsel - g.O) * g.pi[s][n] * g.ia6 * g.inv_vrho;
        }
        acc = 0.5 * u * u * v * v;
    }
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const double ws = wave_sum(acc);
    if (lane == 0) lds_red[w] = ws;
    __syncthreads();
    if (tid == 0) {
        store_agent(&g.partials[blockIdx.x], lds_red[0] + lds_red[1] + lds_red[2] + lds_red[3]);
        last_flag = ticket_arrive(g.ticket, gridDim.x) ? 1 : 0;
    }
    __syncthreads();
    if (last_flag) {
        double part = 0.0;
        for (int i = tid; i < (int)gridDim.x; i += 256) part += load_agent(&g.partials[i]);
        const double pw = wave_sum(part);
        if (lane == 0) lds_red[w] = pw;
        __syncthreads();
        if (tid == 0) {
            *g.out_sum = lds_red[0] + lds_red[1] + lds_red[2] + lds_red[3];
            __hip_atomic_store(g.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// The per-block slots of dO/dq after a reverse sweep, added in block order
// (per thread, wave, then the waves in order) into *dq_acc: one block of 256.
__global__ void __launch_bounds__(256) adj_dq_finish(const double *slots, int nb, double *dq_acc)
{
    __shared__ double lds_red[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double part = 0.0;
    for (int i = tid; i < nb; i += 256) part += slots[i];
    const double ws = wave_sum(part);
    if (lane == 0) lds_red[w] = ws;
    __syncthreads();
    if (tid == 0) *dq_acc += ((lds_red[0] + lds_red[1]) + lds_red[2]) + lds_red[3];
}

__global__ void zero_doubles(double *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

}  // namespace lat
