// stage_adjoint_self.hpp -- pieces of the adjoint of one velocity-Verlet step
// with the self-consistent expansion (sec. 4.5.2 Hamiltonian system with the
// scale factor as a dynamical variable), two real fields with
// V = lambda/4 phi^4 + q/2 phi^2 chi^2.  One step from (phi_n, pi_n, a_n, b_n):
//   (1) pi'  = pi_n + h/2 K(a_n, phi_n)
//   (2) b'   = b_n + h/2 K_a(a_n, E(phi_n, pi_n, a_n))
//   (3) a1   = a_n + h b'
//   (4) phi1 = phi_n + h abar^{alpha-3} pi',  abar = (a_n + a1)/2
//   (5) pi1  = pi' + h/2 K(a1, phi1)
//   (6) b1   = b' + h/2 K_a(a1, E(phi1, pi1, a1))
// with K = a^{1+alpha} Lap phi - a^{3+alpha} grad V and K_a = C(a) Q,
// C = a^{2 alpha+1} kappa^2/3, Q = (alpha-2) E_K + alpha E_G + (alpha+1) E_V.
// The field-shaped parts run one site per thread with neighbours through the
// caches and write per-block partial sums (NQ per block, fixed order) of the
// scalar products that the scalar adjoints of a and b need; three one-thread
// kernels per step pull those scalars back on the device.
#pragma once
#include "common.hpp"

namespace lat {

constexpr int kSelfAdjThreads = 256;

struct SelfAdjSite {
    size_t xp, xm, yp, ym, zp, zm;
};

__device__ inline SelfAdjSite self_adj_nbrs(size_t n, int N)
{
    const int x = (int)(n % N), y = (int)((n / N) % N), z = (int)(n / ((size_t)N * N));
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

// Block partial sums of NQ per-thread values, written to part[q * gridDim.x + block].
template <int NQ>
__device__ inline void self_adj_partials(const double (&v)[NQ], double *part)
{
    __shared__ double lds[NQ][kSelfAdjThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) lds[q][w] = s;
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        double s = 0.0;
        for (int k = 0; k < kSelfAdjThreads / 64; ++k) s += lds[threadIdx.x][k];
        part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
    }
}

struct SelfAdjArgs {
    const double *phi[2], *pi[2];   // the state the piece is taken at
    double *lphi[2], *lpi[2];       // adjoint arrays (updated in place, own site only)
    int N;
    double inv_dx2, lam, q;
    double c0, c1, c2;              // piece coefficients (see each kernel)
    double *part;                   // per-block partials
    const double *dcoef;            // b kick: its three coefficients, on the device
};

// Energy sums of (phi, pi), both fields together: sum pi^2,
// sum |grad+ phi|^2 (forward differences over dx), sum V, sum phi^2 chi^2 / 2.
// No adjoint update.
__global__ void __launch_bounds__(kSelfAdjThreads) self_adj_energy(const SelfAdjArgs g)
{
    const int N = g.N;
    const size_t V = (size_t)N * N * N;
    const size_t n = (size_t)blockIdx.x * kSelfAdjThreads + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (n < V) {
        const SelfAdjSite s = self_adj_nbrs(n, N);
        const double u = g.phi[0][n], w = g.phi[1][n];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            const double *P = g.phi[f];
            const double c = P[n], dx = P[s.xp] - c, dy = P[s.yp] - c, dz = P[s.zp] - c;
            v[0] += g.pi[f][n] * g.pi[f][n];
            v[1] += (dx * dx + dy * dy + dz * dz) * g.inv_dx2;
        }
        v[2] = 0.25 * g.lam * u * u * u * u + 0.5 * g.q * u * u * w * w;
        v[3] = 0.5 * u * u * w * w;
    }
    self_adj_partials<4>(v, g.part);
}

// Pull-back of a b kick b += wb K_a(a, E(phi, pi, a)) into the fields:
//   lphi_s += d0 (-Lap phi_s) + d1 dV/dphi_s,   lpi_s += d2 pi_s
// with (d0, d1, d2) = dcoef = wb lb C (alpha/(a^2 V), (alpha+1)/V, (alpha-2)/(a^6 V)).
__global__ void __launch_bounds__(kSelfAdjThreads) self_adj_bkick(const SelfAdjArgs g)
{
    const int N = g.N;
    const size_t V = (size_t)N * N * N;
    const size_t n = (size_t)blockIdx.x * kSelfAdjThreads + threadIdx.x;
    if (n >= V) return;
    const double d0 = g.dcoef[0], d1 = g.dcoef[1], d2 = g.dcoef[2];
    const SelfAdjSite s = self_adj_nbrs(n, N);
    const double u = g.phi[0][n], w = g.phi[1][n];
    const double dV[2] = {g.lam * u * u * u + g.q * u * w * w, g.q * u * u * w};
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        const double lap = self_adj_lap(g.phi[f], n, s, g.inv_dx2);
        g.lphi[f][n] += d0 * (-lap) + d1 * dV[f];
        g.lpi[f][n] += d2 * g.pi[f][n];
    }
}

// Pull-back of a field kick pi += wk K(a, phi), c0 = wk a^{1+alpha}, c1 = wk a^{3+alpha}:
//   lphi_s += c0 Lap lpi_s - c1 (H_V(phi) lpi)_s
// and partials of  sum lpi . (Lap phi) ,  sum lpi . dV/dphi ,  sum lpi . dF/dq
// (dF/dq = -(phi chi^2, phi^2 chi)), from which the host forms dK/da and dK/dq.
__global__ void __launch_bounds__(kSelfAdjThreads) self_adj_kick(const SelfAdjArgs g)
{
    const int N = g.N;
    const size_t V = (size_t)N * N * N;
    const size_t n = (size_t)blockIdx.x * kSelfAdjThreads + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    if (n < V) {
        const SelfAdjSite s = self_adj_nbrs(n, N);
        const double u = g.phi[0][n], w = g.phi[1][n];
        const double l0 = g.lpi[0][n], l1 = g.lpi[1][n];
        const double h00 = 3.0 * g.lam * u * u + g.q * w * w, h01 = 2.0 * g.q * u * w, h11 = g.q * u * u;
        const double dV0 = g.lam * u * u * u + g.q * u * w * w, dV1 = g.q * u * u * w;
        const double ll0 = self_adj_lap(g.lpi[0], n, s, g.inv_dx2), ll1 = self_adj_lap(g.lpi[1], n, s, g.inv_dx2);
        const double lp0 = self_adj_lap(g.phi[0], n, s, g.inv_dx2), lp1 = self_adj_lap(g.phi[1], n, s, g.inv_dx2);
        g.lphi[0][n] += g.c0 * ll0 - g.c1 * (h00 * l0 + h01 * l1);
        g.lphi[1][n] += g.c0 * ll1 - g.c1 * (h01 * l0 + h11 * l1);
        v[0] = l0 * lp0 + l1 * lp1;
        v[1] = l0 * dV0 + l1 * dV1;
        v[2] = -(l0 * u * w * w) - (l1 * u * u * w);
    }
    self_adj_partials<3>(v, g.part);
}

// Pull-back of the drift phi1 = phi_n + dr pi', with pi' = pi_n + c0 K(a_n, phi_n)
// rebuilt on the fly (c1 = a_n^{1+alpha}, c2 = a_n^{3+alpha}): partial of
// sum lphi . pi', then lpi += dr lphi.
struct SelfDriftArgs {
    SelfAdjArgs g;
    double dr;
};

__global__ void __launch_bounds__(kSelfAdjThreads) self_adj_drift(const SelfDriftArgs d)
{
    const SelfAdjArgs &g = d.g;
    const int N = g.N;
    const size_t V = (size_t)N * N * N;
    const size_t n = (size_t)blockIdx.x * kSelfAdjThreads + threadIdx.x;
    double v[1] = {0.0};
    if (n < V) {
        const SelfAdjSite s = self_adj_nbrs(n, N);
        const double u = g.phi[0][n], w = g.phi[1][n];
        const double dV[2] = {g.lam * u * u * u + g.q * u * w * w, g.q * u * u * w};
        double acc = 0.0;
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            const double K = g.c1 * self_adj_lap(g.phi[f], n, s, g.inv_dx2) - g.c2 * dV[f];
            const double pp = g.pi[f][n] + g.c0 * K;
            const double lf = g.lphi[f][n];
            acc += lf * pp;
            g.lpi[f][n] += d.dr * lf;
        }
        v[0] = acc;
    }
    self_adj_partials<1>(v, g.part);
}

// Scalar adjoints of one reverse step, on the device.  tot holds, in order:
// energy sums (sum pi^2, sum |grad+ phi|^2, sum V, sum phi^2 chi^2/2) at n + 1
// [0..3] and at n [4..7]; the field kick sums at n + 1 (sum lpi.Lap phi,
// sum lpi.dV/dphi, sum lpi.dF/dq) [8..10]; the drift sum lphi.pi' [11]; the
// field kick sums at n [12..14].
struct SelfScalars {
    double la, lb, dq;      // adjoints of a and b, and dO/dq, accumulated
    double la1, la0;        // adjoints of a_{n+1} and a_n within the step
    double bk[3];           // coefficients of the next b kick pull-back
};

struct SelfStepConst {
    double a0, a1, abar, h, alpha, kappa2, V;
};

// K_a = C Q at scale factor a from the energy sums S: C, 1/a^2, 1/a^6, dK_a/da, dK_a/dq
__device__ inline void self_ka(double a, const double *S, const SelfStepConst &k, double &C, double &ia2,
                               double &ia6, double &dKda, double &dKdq)
{
    const double al = k.alpha;
    ia2 = 1.0 / (a * a);
    ia6 = ia2 * ia2 * ia2;
    const double EK = S[0] / (2.0 * k.V) * ia6, EG = S[1] / (2.0 * k.V) * ia2, EV = S[2] / k.V;
    C = pow(a, 2.0 * al + 1.0) / 3.0 * k.kappa2;
    const double Q = (al - 2.0) * EK + al * EG + (al + 1.0) * EV;
    dKda = (2.0 * al + 1.0) * C * Q / a + C * ((al - 2.0) * (-6.0) * EK / a + al * (-2.0) * EG / a);
    dKdq = C * (al + 1.0) * S[3] / k.V;
}

__device__ inline void self_bk(SelfScalars *s, double wl, double C, double ia2, double ia6, const SelfStepConst &k)
{
    s->bk[0] = wl * C * k.alpha * ia2 / k.V;
    s->bk[1] = wl * C * (k.alpha + 1.0) / k.V;
    s->bk[2] = wl * C * (k.alpha - 2.0) * ia6 / k.V;
}

// (6): the b kick at n + 1 (before its field pull-back)
__global__ void self_scal_pre(const double *tot, const SelfStepConst k, SelfScalars *s)
{
    if (threadIdx.x != 0) return;
    double C, ia2, ia6, dKda, dKdq;
    self_ka(k.a1, tot, k, C, ia2, ia6, dKda, dKdq);
    const double wl = 0.5 * k.h * s->lb;
    self_bk(s, wl, C, ia2, ia6, k);
    s->la1 = s->la + wl * dKda;
    s->dq += wl * dKdq;
}

// (5), (4), (3) and the scalar part of (2)
__global__ void self_scal_mid(const double *tot, const SelfStepConst k, SelfScalars *s)
{
    if (threadIdx.x != 0) return;
    const double al = k.alpha, h = k.h;
    double la1 = s->la1 + 0.5 * h * ((1.0 + al) * pow(k.a1, al) * tot[8] - (3.0 + al) * pow(k.a1, 2.0 + al) * tot[9]);
    s->dq += 0.5 * h * pow(k.a1, 3.0 + al) * tot[10];
    const double labar = h * (al - 3.0) * pow(k.abar, al - 4.0) * tot[11];
    la1 += 0.5 * labar;
    double la0 = 0.5 * labar + la1;   // (3) a1 = a_n + h b'
    s->lb += h * la1;
    double C, ia2, ia6, dKda, dKdq;
    self_ka(k.a0, tot + 4, k, C, ia2, ia6, dKda, dKdq);
    const double wl = 0.5 * h * s->lb;
    self_bk(s, wl, C, ia2, ia6, k);
    s->la0 = la0 + wl * dKda;
    s->dq += wl * dKdq;
}

// (1): the field kick at n
__global__ void self_scal_post(const double *tot, const SelfStepConst k, SelfScalars *s)
{
    if (threadIdx.x != 0) return;
    const double al = k.alpha, h = k.h;
    s->la = s->la0 + 0.5 * h * ((1.0 + al) * pow(k.a0, al) * tot[12] - (3.0 + al) * pow(k.a0, 2.0 + al) * tot[13]);
    s->dq += 0.5 * h * pow(k.a0, 3.0 + al) * tot[14];
}

// Sum each of the nq rows of nb partials: block q, each thread a fixed strided
// subset in order, then the fixed wave and block tree; out[q].
__global__ void __launch_bounds__(kSelfAdjThreads) self_adj_reduce(const double *__restrict__ part, int nb, int nq,
                                                                   double *__restrict__ out)
{
    __shared__ double lds[kSelfAdjThreads / 64];
    const int q = blockIdx.x;
    if (q >= nq) return;
    double s = 0.0;
    for (int k = threadIdx.x; k < nb; k += kSelfAdjThreads) s += part[(size_t)q * nb + k];
    const double w = wave_sum(s);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kSelfAdjThreads / 64; ++i) t += lds[i];
        out[q] = t;
    }
}

}  // namespace lat
