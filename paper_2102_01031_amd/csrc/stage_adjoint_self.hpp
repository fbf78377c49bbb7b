// stage_adjoint_self.hpp -- adjoint of the velocity-Verlet evolution with the
// self-consistent expansion (sec. 4.5.2 Hamiltonian system with the scale
// factor as a dynamical variable), two real fields with
// V = lambda/4 phi^4 + q/2 phi^2 chi^2.  One step from (phi_n, pi_n, a_n, b_n):
//   (1) pi'  = pi_n + h/2 K(a_n, phi_n)
//   (2) b'   = b_n + h/2 K_a(a_n, E(phi_n, pi_n, a_n))
//   (3) a1   = a_n + h b'
//   (4) phi1 = phi_n + h abar^{alpha-3} pi',  abar = (a_n + a1)/2
//   (5) pi1  = pi' + h/2 K(a1, phi1)
//   (6) b1   = b' + h/2 K_a(a1, E(phi1, pi1, a1))
// with K = a^{1+alpha} Lap phi - a^{3+alpha} grad V and K_a = C(a) Q,
// C = a^{2 alpha+1} kappa^2/3, Q = (alpha-2) E_K + alpha E_G + (alpha+1) E_V.
//
// The reverse sweep visits the time points n = T, ..., 0 once each.  At point n
// it undoes, in order, (1) and (2) of step n (if n < T), then (6), (5), (4) of
// step n - 1 (if n > 0), all of which act on the state (phi_n, pi_n) at a_n:
//   - both b kicks at n have the weight h/2 lb with the same lb (the pull-backs
//     of (1) and (2) leave lb alone), so their field parts add up;
//   - the field kick of (1) pulls back the momentum adjoint lpi before the b
//     kicks add to it, the kick of (5) pulls back lpi after both;
//   - pi' of step n - 1 is rebuilt as pi_n - h/2 K(a_n, phi_n).
// One pass per point does all of that site by site and leaves per-block
// partial sums of the eight scalar products the scalar adjoints need; the next
// pass (or self_rev_finish) adds them up in block order in every block, so the
// chain of scalar adjoints (la, lb, dO/dq) runs on the device, in a fixed order,
// without a launch of its own.  (3) is the scalar step between points.
//
// The states of a segment are re-run from its checkpoint by self_rerun with
// the scale factors the forward sweep recorded.
#pragma once
#include "common.hpp"

namespace lat {

constexpr int kSelfAdjThreads = 256;
constexpr int kRevQ = 8;   // energy sums (4), kick products (3), drift product (1)

struct SelfAdjSite {
    size_t xp, xm, yp, ym, zp, zm;
};

// (32-bit index arithmetic: N^3 < 2^32)
__device__ inline SelfAdjSite self_adj_nbrs(size_t n, int N)
{
    const unsigned u = (unsigned)n, Nu = (unsigned)N, yz = u / Nu;
    const int x = (int)(u - yz * Nu), z = (int)(yz / Nu), y = (int)(yz - (unsigned)z * Nu);
    const size_t NN = (size_t)N * N;
    SelfAdjSite s;
    s.xp = n - x + (x + 1 == N ? 0 : x + 1);
    s.xm = n - x + (x == 0 ? N - 1 : x - 1);
    s.yp = n + (size_t)((y + 1 == N ? 0 : y + 1) - y) * N;
    s.ym = n + (size_t)((y == 0 ? N - 1 : y - 1) - y) * N;
    s.zp = n + (size_t)((z + 1 == N ? 0 : z + 1) - z) * NN;
    s.zm = n + (size_t)((z == 0 ? N - 1 : z - 1) - z) * NN;
    return s;
}

__device__ inline double self_adj_lap(const double *f, size_t n, const SelfAdjSite &s, double idx2)
{
    const double c = f[n];
    return ((f[s.xp] - 2.0 * c + f[s.xm]) + (f[s.yp] - 2.0 * c + f[s.ym]) + (f[s.zp] - 2.0 * c + f[s.zm])) * idx2;
}

// ---------------------------------------------------------------------------
// re-run of a segment: from (phi_j, pi'_j) to the state (phi_{j+1}, pi_{j+1})
// and pi'_{j+1}, with the recorded scale factors:
//   phi_{j+1} = phi_j + dr pi'_j,  K = ka1 Lap phi_{j+1} - ka3 grad V(phi_{j+1}),
//   pi_{j+1} = pi'_j + cf K,  pi'_{j+1} = pi_{j+1} + h/2 K
// (cf = h/2, dr = h abar^{alpha-3}).  The first call of a segment takes the
// checkpoint (phi, pi) with dr = cf = 0: it copies the state and forms pi'.
struct SelfRerunArgs {
    const double *phi_in[2], *pp_in[2];
    double *phi_out[2], *pi_out[2], *pp_out[2];
    int N;
    double inv_dx2, lam, q;
    double dr, cf, ch;       // drift, first and second half kick weights
    double ka1, ka3;         // a^{1+alpha}, a^{3+alpha} at the new point
};

__global__ void __launch_bounds__(kSelfAdjThreads) self_rerun(const SelfRerunArgs g)
{
    const int N = g.N;
    const size_t V = (size_t)N * N * N;
    const size_t n = (size_t)blockIdx.x * kSelfAdjThreads + threadIdx.x;
    if (n >= V) return;
    const SelfAdjSite s = self_adj_nbrs(n, N);
    double ph[2], lap[2];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        const double *P = g.phi_in[f], *Q = g.pp_in[f];
        auto at = [&](size_t m) { return P[m] + g.dr * Q[m]; };
        const double c = at(n);
        ph[f] = c;
        lap[f] = ((at(s.xp) - 2.0 * c + at(s.xm)) + (at(s.yp) - 2.0 * c + at(s.ym)) +
                  (at(s.zp) - 2.0 * c + at(s.zm))) * g.inv_dx2;
    }
    const double u = ph[0], w = ph[1];
    const double dV[2] = {g.lam * u * u * u + g.q * u * w * w, g.q * u * u * w};
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        const double K = g.ka1 * lap[f] - g.ka3 * dV[f];
        const double p1 = g.pp_in[f][n] + g.cf * K;
        g.phi_out[f][n] = ph[f];
        g.pi_out[f][n] = p1;
        g.pp_out[f][n] = p1 + g.ch * K;
    }
}

// ---------------------------------------------------------------------------
// scalar adjoints carried from point to point
struct SelfScalars {
    double la;   // adjoint of a at the current point (what is known of it so far)
    double lb;   // adjoint of b
    double dq;   // dO/dq accumulated
    double pad;
};

// one time point of the reverse sweep, with the powers of the scale factor
// its pieces need (formed on the host from the recorded a_n)
struct SelfPoint {
    double a;          // a_n
    double ka1, ka3;   // a_n^{1+alpha}, a_n^{3+alpha}
    double pa, pa2;    // a_n^alpha, a_n^{2+alpha}
    double C;          // a_n^{2 alpha+1} kappa^2 / 3
    double dr;         // h abar^{alpha-3}, abar = (a_{n-1} + a_n)/2, the drift of step n-1  (kB)
    double pbar;       // abar^{alpha-4}                                                   (kB)
    int kA;            // step n leaves n (n < T): (1), (2)
    int kB;            // step n - 1 ends at n (n > 0): (6), (5), (4), (3)
};

struct SelfConst {
    double h, alpha, kappa2, V, inv_dx2, lam, q;
};

// dK_a/da and dK_a/dq at point P from the energy sums E (sum pi^2,
// sum |grad+ phi|^2 over dx^2, sum V, sum phi^2 chi^2 / 2), K_a = C Q
__device__ inline void self_ka(const SelfPoint &P, const double *E, const SelfConst &k, double &dKda, double &dKdq)
{
    const double al = k.alpha, a = P.a;
    const double ia2 = 1.0 / (a * a), ia6 = ia2 * ia2 * ia2;
    const double EK = E[0] / (2.0 * k.V) * ia6, EG = E[1] / (2.0 * k.V) * ia2, EV = E[2] / k.V;
    const double Q = (al - 2.0) * EK + al * EG + (al + 1.0) * EV;
    dKda = (2.0 * al + 1.0) * P.C * Q / a + P.C * ((al - 2.0) * (-6.0) * EK / a + al * (-2.0) * EG / a);
    dKdq = P.C * (al + 1.0) * E[3] / k.V;
}

// The scalar part of point P from its sums tot (kRevQ, in the order of the
// pass): both b kicks' da terms, the field kicks' da and dq terms, and for
// kB the drift's dabar term and (3), which leaves la as the part of the
// adjoint of a_{n-1} known so far.
__device__ inline void self_rev_finalise(const SelfPoint &P, const double *tot, const SelfConst &k, SelfScalars &s)
{
    const double al = k.alpha, h = k.h;
    const int nbk = P.kA + P.kB;
    double dKda, dKdq;
    self_ka(P, tot, k, dKda, dKdq);
    const double wl = 0.5 * h * s.lb;
    double la = s.la + (double)nbk * wl * dKda + 0.5 * h * ((1.0 + al) * P.pa * tot[4] - (3.0 + al) * P.pa2 * tot[5]);
    s.dq += (double)nbk * wl * dKdq + 0.5 * h * P.ka3 * tot[6];
    if (P.kB) {
        const double labar = h * (al - 3.0) * P.pbar * tot[7];
        la += 0.5 * labar;      // a_n's share of abar
        s.lb += h * la;         // (3): a_n = a_{n-1} + h b'
        la = 0.5 * labar + la;  // a_{n-1}: its share of abar, and through (3)
    }
    s.la = la;
}

struct SelfRevArgs {
    const double *phi[2], *pi[2];   // the state at the point
    double *lphi[2];                // field adjoint, updated in place (own site)
    const double *lpi_in[2];        // momentum adjoint in (read with neighbours) ...
    double *lpi_out[2];             // ... and out
    int N, sites;                   // sites per thread
    SelfConst k;
    SelfPoint P;                    // this point
    SelfPoint Pp;                   // the point before (n + 1), finalised in the prologue
    int has_prev;
    const double *part_in;          // its per-block sums, kRevQ per block
    int nb_in;
    double *part_out;               // this pass's, kRevQ per block
    const SelfScalars *sc_in;
    SelfScalars *sc_out;            // written by block 0
};

template <int NT, int NQ>
__device__ inline void self_sum_partials(const double *part, int nb, double *lds_red, double (&tot)[NQ])
{
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    for (int i = threadIdx.x; i < nb; i += NT) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] += part[(size_t)i * NQ + q];
    }
    block_sums<NT, NQ>(acc, lds_red, tot);
}

__global__ void __launch_bounds__(kSelfAdjThreads) self_rev(const SelfRevArgs g)
{
    constexpr int NT = kSelfAdjThreads;
    __shared__ double lds_red[(NT / 64) * kRevQ];
    __shared__ double lds_lb;
    const int tid = threadIdx.x;
    // scalars up to this point: finalise the previous point in every block
    {
        double tot[kRevQ];
        if (g.has_prev) self_sum_partials<NT, kRevQ>(g.part_in, g.nb_in, lds_red, tot);
        if (tid == 0) {
            SelfScalars s = *g.sc_in;
            if (g.has_prev) self_rev_finalise(g.Pp, tot, g.k, s);
            lds_lb = s.lb;
            if (blockIdx.x == 0) *g.sc_out = s;
        }
        __syncthreads();
    }
    const SelfConst &k = g.k;
    const SelfPoint &P = g.P;
    const double lb = lds_lb;
    const int nbk = P.kA + P.kB;
    // b kick pull-back coefficients at a_n (both kicks), field kick weights
    const double ia2 = 1.0 / (P.a * P.a), ia6 = ia2 * ia2 * ia2;
    const double wl = 0.5 * k.h * lb;
    const double d0 = wl * P.C * k.alpha * ia2 / k.V, d1 = wl * P.C * (k.alpha + 1.0) / k.V;
    const double nd2 = (double)nbk * wl * P.C * (k.alpha - 2.0) * ia6 / k.V;
    const double c0 = 0.5 * k.h * P.ka1, c1 = 0.5 * k.h * P.ka3;
    const double fA = (double)P.kA, fB = (double)P.kB;

    const int N = g.N;
    const size_t V = (size_t)N * N * N;
    double acc[kRevQ];
#pragma unroll
    for (int q = 0; q < kRevQ; ++q) acc[q] = 0.0;
    for (int it = 0; it < g.sites; ++it) {
        const size_t n = ((size_t)blockIdx.x * g.sites + it) * NT + tid;
        if (n >= V) break;
        const SelfAdjSite s = self_adj_nbrs(n, N);
        const double u = g.phi[0][n], w = g.phi[1][n];
        const double dV[2] = {k.lam * u * u * u + k.q * u * w * w, k.q * u * u * w};
        const double h00 = 3.0 * k.lam * u * u + k.q * w * w, h01 = 2.0 * k.q * u * w, h11 = k.q * u * u;
        double Lp[2], y[2], Ly[2], l1[2], pv[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            const double *Pf = g.phi[f];
            const double c = Pf[n], ex = Pf[s.xp] - c, ey = Pf[s.yp] - c, ez = Pf[s.zp] - c;
            Lp[f] = self_adj_lap(Pf, n, s, k.inv_dx2);
            pv[f] = g.pi[f][n];
            const double lpi = g.lpi_in[f][n];
            l1[f] = lpi + nd2 * pv[f];                      // after both b kicks
            y[f] = fA * lpi + fB * l1[f];                  // what the two field kicks pull back
            Ly[f] = (fA + fB) * self_adj_lap(g.lpi_in[f], n, s, k.inv_dx2) +
                    fB * nd2 * self_adj_lap(g.pi[f], n, s, k.inv_dx2);
            acc[0] += pv[f] * pv[f];
            acc[1] += (ex * ex + ey * ey + ez * ez) * k.inv_dx2;
        }
        acc[2] += 0.25 * k.lam * u * u * u * u + 0.5 * k.q * u * u * w * w;
        acc[3] += 0.5 * u * u * w * w;
        const double Hy[2] = {h00 * y[0] + h01 * y[1], h01 * y[0] + h11 * y[1]};
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            const double lf = g.lphi[f][n] + (double)nbk * (d0 * (-Lp[f]) + d1 * dV[f]) + c0 * Ly[f] - c1 * Hy[f];
            acc[4] += y[f] * Lp[f];
            acc[5] += y[f] * dV[f];
            double lp = l1[f];
            if (P.kB) {
                const double pp = pv[f] - 0.5 * k.h * (P.ka1 * Lp[f] - P.ka3 * dV[f]);   // pi' of step n - 1
                acc[7] += lf * pp;
                lp += P.dr * lf;
            }
            g.lphi[f][n] = lf;
            g.lpi_out[f][n] = lp;
        }
        acc[6] += -(y[0] * u * w * w) - (y[1] * u * u * w);
    }
    double tot[kRevQ];
    block_sums<NT, kRevQ>(acc, lds_red, tot);
    if (tid == 0) {
#pragma unroll
        for (int q = 0; q < kRevQ; ++q) g.part_out[(size_t)blockIdx.x * kRevQ + q] = tot[q];
    }
}

// the last point's sums (one block)
__global__ void __launch_bounds__(kSelfAdjThreads) self_rev_finish(const double *part, int nb, const SelfPoint P,
                                                                   const SelfConst k, const SelfScalars *sc_in,
                                                                   SelfScalars *sc_out)
{
    constexpr int NT = kSelfAdjThreads;
    __shared__ double lds_red[(NT / 64) * kRevQ];
    double tot[kRevQ];
    self_sum_partials<NT, kRevQ>(part, nb, lds_red, tot);
    if (threadIdx.x == 0) {
        SelfScalars s = *sc_in;
        self_rev_finalise(P, tot, k, s);
        *sc_out = s;
    }
}

}  // namespace lat
