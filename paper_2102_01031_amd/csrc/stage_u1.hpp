// stage_u1.hpp -- one pass of the U(1) (Abelian-Higgs) lattice system (the
// forces below at a = 1; in an expanding background each term carries its
// power of a, see U1Args).
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
#include "trig.hpp"

namespace lat {

struct U1Args {
    const double *phi_in[2];
    double *phi_out[2];
    double *pi[2];
    const double *A_in[3];
    double *A_out[3];
    double *piA[3];
    int N, tiles_x, tiles_y, zc;
    double dx, e, lam, v, kappa_g;
    double ck;   // kick weight (time)
    double hd;   // drift weight of phi (time times a^{alpha-3})
    // expanding background (sec. 5.5.2 kernels): the covariant Laplacian and the
    // current scale with la1 = a^{1+alpha}, the potential force with
    // la3 = a^{3+alpha}, the magnetic force with lam1 = a^{alpha-1}; hdA is the
    // drift weight of A (time times a^{alpha-1}).  All 1 (hdA = hd) at a = 1.
    double la1, la3, lam1, hdA;
    // if not null: {ck, la1, la3, lam1, hd, hdA} from device memory (written by
    // the self-consistent scale-factor kernels), in place of the values above
    const double *dw;
    double *partials;
    unsigned *ticket;
    ScaleRecord *sc;
    int defer;   // summing passes: leave the block partials, take no ticket
};

// kU1KickSums (row kernel only): the kick-only pass that also leaves the volume
// sums [0, 5) of the kicked state, as an energy pass with zero kick weight after
// it would (Gauss terms not measured: sums [5, 8) and the maxes are zero)
// kU1Drift: the drift alone (u1_drift), for a step pass whose kick weight is zero
enum U1Mode : int { kU1Step = 0, kU1Kick = 1, kU1Energy = 2, kU1KickSums = 3, kU1Drift = 4 };
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
    const int N = g.N;
    const int x = bx * TX + tx, y = by * TY + ty;
    const bool valid = x < N && y < N;
    // the energy pass takes a column of zc planes per block (fewer blocks, so
    // fewer ticket releases); the other passes one plane
    const int zb = MODE == kU1Energy ? (rest / g.tiles_y) * g.zc : rest / g.tiles_y;
    const int ze = MODE == kU1Energy ? min(zb + g.zc, N) : zb + 1;

    double acc[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) acc[k] = 0.0;

#pragma unroll 1
    for (int z = zb; z < ze; ++z) {
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
        const double sxy = lat_sin(txy), sxz = lat_sin(txz), syz = lat_sin(tyz);
        const double mag[3] = {(sxy - lat_sin(txy_ym)) + (sxz - lat_sin(txz_zm)),
                               (-sxy + lat_sin(txy_xm)) + (syz - lat_sin(tyz_zm)),
                               (-sxz + lat_sin(txz_xm)) + (-syz + lat_sin(tyz_ym))};

        // covariant Laplacian and current
        const double pr = g.phi_in[0][n], pim = g.phi_in[1][n];
        const size_t np_[3] = {nxp, nyp, nzp}, nm_[3] = {nxm, nym, nzm};
        double d2r = 0.0, d2i = 0.0, grad2 = 0.0, J[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double s, c, sm, cm;
            lat_sincos(edx * g.A_in[i][n], &s, &c);
            lat_sincos(edx * g.A_in[i][nm_[i]], &sm, &cm);
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
        double ck = g.ck, la1 = g.la1, la3 = g.la3, lm1 = g.lam1, hdP = g.hd, hdA = g.hdA;
        if (g.dw) {
            ck = g.dw[0];
            la1 = g.dw[1];
            la3 = g.dw[2];
            lm1 = g.dw[3];
            hdP = g.dw[4];
            hdA = g.dw[5];
        }
        const double m2 = 0.5 * (pr * pr + pim * pim);
        const double vp = 0.5 * g.lam * (m2 - g.v * g.v);
        const double inv_dx2 = 1.0 / (g.dx * g.dx);
        const double F0 = la1 * (d2r * inv_dx2) - la3 * (vp * pr);
        const double F1 = la1 * (d2i * inv_dx2) - la3 * (vp * pim);
        const double inv_edx3 = 1.0 / (g.e * g.dx * g.dx * g.dx);
        double FA[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) FA[i] = la1 * (g.kappa_g * J[i]) - lm1 * (mag[i] * inv_edx3);

        const double p0 = g.pi[0][n], p1 = g.pi[1][n];
        double pa[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) pa[i] = g.piA[i][n];

        if (MODE == kU1Energy) {
            double t[NQ];
            const double s0 = p0 + ck * F0, s1 = p1 + ck * F1;
            t[0] = 0.5 * (s0 * s0 + s1 * s1);
            t[1] = grad2 * inv_dx2 * 0.5;
            const double u = m2 - g.v * g.v;
            t[2] = 0.25 * g.lam * u * u;
            double ka = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double sa = pa[i] + ck * FA[i];
                ka += sa * sa;
            }
            t[3] = ka / (2.0 * g.kappa_g);
            const double hxy = lat_sin(0.5 * txy), hxz = lat_sin(0.5 * txz), hyz = lat_sin(0.5 * tyz);
            const double mg = 2.0 * hxy * hxy + 2.0 * hxz * hxz + 2.0 * hyz * hyz;
            t[4] = mg / (g.kappa_g * g.e * g.e * g.dx * g.dx * g.dx * g.dx);
            // Gauss residual of the stored pairing
            const double div = ((pa[0] - g.piA[0][nxm]) + (pa[1] - g.piA[1][nym]) + (pa[2] - g.piA[2][nzm])) / g.dx;
            const double charge = g.e * g.kappa_g * (pr * p1 - pim * p0);
            const double G = div - charge;
            t[5] = fabs(G);
            t[6] = fabs(div + charge);
            t[7] = fabs(div) + fabs(charge);
            t[8] = fabs(G);
            t[9] = fabs(div);
            t[10] = fabs(charge);
#pragma unroll
            for (int k = 0; k < NQ; ++k) acc[k] = k < kU1Sums ? acc[k] + t[k] : fmax(acc[k], t[k]);
        } else {
            const double q0 = p0 + ck * F0, q1 = p1 + ck * F1;
            g.pi[0][n] = q0;
            g.pi[1][n] = q1;
            double qa[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                qa[i] = pa[i] + ck * FA[i];
                g.piA[i][n] = qa[i];
            }
            if (MODE == kU1Step) {
                g.phi_out[0][n] = pr + hdP * q0;
                g.phi_out[1][n] = pim + hdP * q1;
#pragma unroll
                for (int i = 0; i < 3; ++i) g.A_out[i][n] = g.A_in[i][n] + hdA * qa[i];
            }
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
            // defer: the block partials are combined by a kernel after this one
            last_flag = g.defer ? 0 : (ticket_arrive(g.ticket, gridDim.x) ? 1 : 0);
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

// Drift only, with the record's weights hd = dw[4], hdA = dw[5]: phi' = phi + hd pi,
// A_i' = A_i + hdA piA_i into the other position buffers, one site per thread.
// The self-consistent steps' drift pass has zero kick weight, where a step
// pass forms the same values (p + 0 F = p) and rewrites the momenta unchanged:
// this reads 10 and writes 5 arrays, with no forces.
__global__ void __launch_bounds__(256) u1_drift(const U1Args g, unsigned vol)
{
    const unsigned n = blockIdx.x * 256u + threadIdx.x;
    if (n >= vol) return;
    const double hd = g.dw[4], hdA = g.dw[5];
#pragma unroll
    for (int c = 0; c < 2; ++c) g.phi_out[c][n] = g.phi_in[c][n] + hd * g.pi[c][n];
#pragma unroll
    for (int i = 0; i < 3; ++i) g.A_out[i][n] = g.A_in[i][n] + hdA * g.piA[i][n];
}

// ---------------------------------------------------------------------------
// Self-consistent expansion of the U(1) model (sec. 5.5.2, the b' equation with
// the gauge energies): one-thread kernels between the lattice passes.  An
// energy pass with ck = 0 leaves the raw volume sums in ScaleRecord::sums[0..4]
// (pi part, gradient, potential, electric, magnetic; the a = 1 forms), from
// which the energies at a are
//   E_K = S0/(V a^6), E_G = S1/(V a^2), E_V = S2/V, E_K^A = S3/(V a^4), E_G^A = S4/(V a^4),
// and the kernel of b is
//   K_a = a^{2 alpha+1}/3 kappa^2 [(alpha-2) E_K + alpha E_G + (alpha-1)(E_K^A + E_G^A) + (alpha+1) E_V].
// The weights of the next pass go to ScaleRecord::w in U1Args::dw order.
// ---------------------------------------------------------------------------
struct U1SelfConst {
    double alpha, kappa2, inv_vol;
};

__device__ inline double u1_kernel_b(double a, const double *S, const U1SelfConst &k)
{
    const double a2 = a * a, a4 = a2 * a2, a6 = a4 * a2;
    const double EK = S[0] * k.inv_vol / a6, EG = S[1] * k.inv_vol / a2, EV = S[2] * k.inv_vol;
    const double EA = S[3] * k.inv_vol / a4 + S[4] * k.inv_vol / a4;
    const double al = k.alpha;
    return pow(a, 2.0 * al + 1.0) / 3.0 * k.kappa2 *
           ((al - 2.0) * EK + al * EG + (al - 1.0) * EA + (al + 1.0) * EV);
}

// kick weights at the record's a: {ck, a^{1+alpha}, a^{3+alpha}, a^{alpha-1}, 0, 0}
__global__ void u1_self_kick_w(ScaleRecord *S, double ck, double alpha)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double a = S->a;
        S->w[0] = ck;
        S->w[1] = pow(a, 1.0 + alpha);
        S->w[2] = pow(a, 3.0 + alpha);
        S->w[3] = pow(a, alpha - 1.0);
        S->w[4] = 0.0;
        S->w[5] = 0.0;
    }
}

// keep the sums of the state before a kick (sums[8..12])
__global__ void u1_self_stash(ScaleRecord *S)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        for (int k = 0; k < 5; ++k) S->sums[8 + k] = S->sums[k];
}

// b += w K_a(a, sums[0..4]) (the sync's half kick, or a velocity-Verlet half kick)
__global__ void u1_self_b_kick(ScaleRecord *S, double w, U1SelfConst k)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) S->b += w * u1_kernel_b(S->a, S->sums, k);
}

// Leapfrog (reading A3): b += cL K_a(before, sums[8..12]) + cR K_a(after, sums[0..4]);
// velocity-Verlet (reading R1, cL = 0): b += cR K_a(sums[0..4]).  Then a' = a + h b and
// the drift weights {0, 1, 1, 1, h abar^{alpha-3}, h abar^{alpha-1}}, abar = (a + a')/2.
// Every call leaves the momentum sums of the kicked state (sums[0], sums[3]) in
// sums[8] and sums[11]: the drift that follows moves only the positions, so they
// are the next step's momentum sums before its kick.  With carry != 0 the sums
// before this step's kick were not measured: their momentum parts are those the
// previous call left, and their position parts (sums[1], [2], [4]) are the
// after-kick ones, the kick having moved only the momenta.  An energy pass with
// zero kick weight sums p + 0 F = p, so the carried sums equal measured ones bit
// for bit.
__global__ void u1_self_drift_w(ScaleRecord *S, double h, double cL, double cR, U1SelfConst k, int carry)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (carry) {
            S->sums[9] = S->sums[1];
            S->sums[10] = S->sums[2];
            S->sums[12] = S->sums[4];
        }
        const double a = S->a;
        double b = S->b;
        if (cL != 0.0) b += cL * u1_kernel_b(a, S->sums + 8, k);
        b += cR * u1_kernel_b(a, S->sums, k);
        const double a1 = a + h * b;
        const double am = 0.5 * (a + a1);
        S->w[0] = 0.0;
        S->w[1] = 1.0;
        S->w[2] = 1.0;
        S->w[3] = 1.0;
        S->w[4] = h * pow(am, k.alpha - 3.0);
        S->w[5] = h * pow(am, k.alpha - 1.0);
        S->a = a1;
        S->b = b;
        S->sums[8] = S->sums[0];
        S->sums[11] = S->sums[3];
    }
}

// Leapfrog pass for N = 64 * XS (XS in {1, 2}) that shares the transcendental
// work between neighbouring sites.  A block owns TY whole x rows and marches z
// over [z0, z1); each thread owns one site of each plane (row y0 + w / XS,
// x = 64 (w % XS) + lane for wavefront w).  Per plane every site evaluates its
// own three plaquette sines sin theta_ij(n) and its three link phases
// (cos, sin)(e dx A_i(n)) once; the values at n - x and n - y are read from
// LDS, those at n - z are carried in registers from the previous plane, and
// the row y0 - 1 below the block is evaluated by the block's threads, one
// operation each.  Every angle is formed by the same expression, in the same
// order, as in u1_stage: the same arithmetic without the repeated sines.
template <int XS, int TY, int MODE>
__global__ void __launch_bounds__(64 * XS * TY) u1_rows(const U1Args g)
{
    constexpr int NT = 64 * XS * TY;
    constexpr int NX = 64 * XS;               // == N
    constexpr int R = TY + 2;                 // LDS rows stand for y0 - 1 .. y0 + TY
    constexpr int NH = 2 * NX;                // halo cells per plane: LDS rows 0 and TY + 1
    constexpr int HPT = (NH + NT - 1) / NT;
    constexpr int NOP = 3 * NX;               // halo-row transcendental operations per plane
    constexpr int OPT = (NOP + NT - 1) / NT;

    // psi and A of the current plane, double-buffered by plane parity so that
    // storing plane z + 1 cannot race with the last reads of plane z
    __shared__ double s_p0[2][R * NX], s_p1[2][R * NX];           // psi, rows 0 .. TY+1
    __shared__ double s_ax[2][R * NX], s_az[2][R * NX];           // A_x, A_z, rows 0 .. TY+1
    __shared__ double s_ay[2][(TY + 1) * NX], s_ayn[2][NX];       // A_y rows 0 .. TY; A_y(row 0, z+1)
    __shared__ double s_sxy[(TY + 1) * NX], s_syz[(TY + 1) * NX]; // rows 0 .. TY
    __shared__ double s_cy[(TY + 1) * NX], s_sy[(TY + 1) * NX];   // phase of A_y, rows 0 .. TY
    __shared__ double s_sxz[TY * NX];                             // own rows (index row - 1)
    __shared__ double s_cx[TY * NX], s_sx[TY * NX];               // phase of A_x, own rows
    __shared__ double s_cz[TY * NX], s_sz[TY * NX];               // phase of A_z, own rows
    constexpr bool EN = MODE == kU1Energy || MODE == kU1KickSums;   // ends with the reduction
    constexpr int NQ = kU1Sums + kU1Maxes;
    __shared__ double lds_red[EN ? (NT / 64) * NQ : 1];
    __shared__ int last_flag;

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int r = w / XS + 1;                 // LDS row of this thread's site
    const int x = (w % XS) * 64 + lane;
    const int xm = (x - 1) & (NX - 1), xp = (x + 1) & (NX - 1);
    const int ro = r * NX + x;                // this site in rows 0 .. TY+1 arrays
    const int wo = (r - 1) * NX + x;          // this site in own-row arrays
    const int N = NX;
    const int lid = xcd_logical_block(blockIdx.x, gridDim.x);
    const int chunks = (N + g.zc - 1) / g.zc;
    const int bz = lid % chunks;
    const int by = lid / chunks;
    const int y0 = by * TY;
    const int z0 = bz * g.zc;
    const int z1 = min(z0 + g.zc, N);
    const unsigned NN = (unsigned)N * (unsigned)N;   // N^3 < 2^32
    const unsigned so = (unsigned)((y0 + r - 1) * N + x);   // site offset within a plane
    const int yb = (y0 == 0 ? N - 1 : y0 - 1) * N;
    const int yt = ((y0 + TY) % N) * N;

    const double edx = g.e * g.dx;
    const double inv_dx2 = 1.0 / (g.dx * g.dx);
    const double inv_edx3 = 1.0 / (g.e * g.dx * g.dx * g.dx);
    double ck = g.ck, la1 = g.la1, la3 = g.la3, lm1 = g.lam1, hd = g.hd, hdA = g.hdA;
    if (g.dw) {
        ck = g.dw[0];
        la1 = g.dw[1];
        la3 = g.dw[2];
        lm1 = g.dw[3];
        hd = g.dw[4];
        hdA = g.dw[5];
    }

    // halo cells: c < NX is row 0 (y0 - 1), else row TY + 1 (y0 + TY)
    int hrow[HPT], hx[HPT];
    unsigned hoff[HPT];
    bool hval[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
        const int c = tid + j * NT;
        hval[j] = c < NH;
        const bool bot = c < NX;
        hx[j] = bot ? c : c - NX;
        hrow[j] = bot ? 0 : TY + 1;
        hoff[j] = hval[j] ? (unsigned)((bot ? yb : yt) + hx[j]) : 0u;
    }

    double wm[2], w0[2], wp[2];   // psi at z - 1, z, z + 1
    double a0[3], a1[3];          // A at z, z + 1
    double czm, szm, sxzm, syzm;  // link phase of A_z and sines theta_xz, theta_yz at n - z
    double hp0[HPT], hp1[HPT], hax[HPT], hay[HPT], haz[HPT], hayn[HPT];
    double acc[NQ];   // energy mode: the site terms of u1_stage, summed over the column
#pragma unroll
    for (int k = 0; k < NQ; ++k) acc[k] = 0.0;

    // ---- prologue: window, A, halo rows of plane z0, carried values of plane z0 - 1
    {
        const unsigned om = (unsigned)(z0 == 0 ? N - 1 : z0 - 1) * NN;
        const unsigned o0 = (unsigned)z0 * NN;
        const unsigned o1 = (unsigned)((z0 + 1) % N) * NN;
        double am[3];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            wm[c] = ld32(g.phi_in[c], om + so);
            w0[c] = ld32(g.phi_in[c], o0 + so);
            wp[c] = ld32(g.phi_in[c], o1 + so);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            am[i] = ld32(g.A_in[i], om + so);
            a0[i] = ld32(g.A_in[i], o0 + so);
            a1[i] = ld32(g.A_in[i], o1 + so);
        }
        s_az[1][ro] = am[2];
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            hp0[j] = hp1[j] = hax[j] = hay[j] = haz[j] = hayn[j] = 0.0;
            if (hval[j]) {
                hp0[j] = ld32(g.phi_in[0], o0 + hoff[j]);
                hp1[j] = ld32(g.phi_in[1], o0 + hoff[j]);
                hax[j] = ld32(g.A_in[0], o0 + hoff[j]);
                haz[j] = ld32(g.A_in[2], o0 + hoff[j]);
                if (hrow[j] == 0) {
                    hay[j] = ld32(g.A_in[1], o0 + hoff[j]);
                    hayn[j] = ld32(g.A_in[1], o1 + hoff[j]);
                } else {
                    s_az[1][(TY + 1) * NX + hx[j]] = ld32(g.A_in[2], om + hoff[j]);
                }
            }
        }
        __syncthreads();
        const double txz = edx * ((s_az[1][r * NX + xp] - am[2]) - a0[0] + am[0]);
        const double tyz = edx * ((s_az[1][(r + 1) * NX + x] - am[2]) - a0[1] + am[1]);
        sxzm = lat_sin(txz);
        syzm = lat_sin(tyz);
        lat_sincos(edx * am[2], &szm, &czm);
        __syncthreads();
    }

    for (int z = z0; z < z1; ++z) {
        const unsigned oz = (unsigned)z * NN;
        const int b = (z - z0) & 1;
        // (A) plane z into LDS
        s_p0[b][ro] = w0[0];
        s_p1[b][ro] = w0[1];
        s_ax[b][ro] = a0[0];
        s_ay[b][ro] = a0[1];
        s_az[b][ro] = a0[2];
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            if (hval[j]) {
                const int hs = hrow[j] * NX + hx[j];
                s_p0[b][hs] = hp0[j];
                s_p1[b][hs] = hp1[j];
                s_ax[b][hs] = hax[j];
                s_az[b][hs] = haz[j];
                if (hrow[j] == 0) {
                    s_ay[b][hx[j]] = hay[j];
                    s_ayn[b][hx[j]] = hayn[j];
                }
            }
        }
        __syncthreads();

        // (B0) loads for the next plane: psi, A of plane z + 2 and the halo rows
        // of plane z + 1 (indices clamped to valid planes after the chunk's end)
        int z2 = min(z + 2, z1);
        if (z2 >= N) z2 -= N;
        int zh = min(z + 1, z1 - 1);
        if (zh >= N) zh -= N;
        int zhn = zh + 1;
        if (zhn >= N) zhn -= N;
        const unsigned o2 = (unsigned)z2 * NN, oh = (unsigned)zh * NN, ohn = (unsigned)zhn * NN;
        double nps[2], na[3];
#pragma unroll
        for (int c = 0; c < 2; ++c) nps[c] = ld32(g.phi_in[c], o2 + so);
#pragma unroll
        for (int i = 0; i < 3; ++i) na[i] = ld32(g.A_in[i], o2 + so);
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            if (hval[j]) {
                hp0[j] = ld32(g.phi_in[0], oh + hoff[j]);
                hp1[j] = ld32(g.phi_in[1], oh + hoff[j]);
                hax[j] = ld32(g.A_in[0], oh + hoff[j]);
                haz[j] = ld32(g.A_in[2], oh + hoff[j]);
                if (hrow[j] == 0) {
                    hay[j] = ld32(g.A_in[1], oh + hoff[j]);
                    hayn[j] = ld32(g.A_in[1], ohn + hoff[j]);
                }
            }
        }

        // (B) own plaquette sines and link phases into LDS; then the halo
        // row's, one operation per thread
        double th[3];   // own plaquette angles (the energy mode's magnetic term)
        {
            const double txy = edx * ((s_ay[b][r * NX + xp] - a0[1]) - s_ax[b][(r + 1) * NX + x] + a0[0]);
            const double txz = edx * ((s_az[b][r * NX + xp] - a0[2]) - a1[0] + a0[0]);
            const double tyz = edx * ((s_az[b][(r + 1) * NX + x] - a0[2]) - a1[1] + a0[1]);
            th[0] = txy;
            th[1] = txz;
            th[2] = tyz;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double t = j == 0 ? txy : (j == 1 ? txz : tyz);
                double *dst = j == 0 ? &s_sxy[ro] : (j == 1 ? &s_sxz[wo] : &s_syz[ro]);
                *dst = lat_sin(t);
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double t = edx * (j == 0 ? a0[0] : (j == 1 ? a0[1] : a0[2]));
                double sv, cv;
                lat_sincos(t, &sv, &cv);
                const int sl = j == 1 ? ro : wo;
                double *ds = j == 0 ? s_sx : (j == 1 ? s_sy : s_sz);
                double *dc = j == 0 ? s_cx : (j == 1 ? s_cy : s_cz);
                ds[sl] = sv;
                dc[sl] = cv;
            }
        }
#pragma unroll
        for (int j = 0; j < OPT; ++j) {
            const int id = tid + j * NT;
            if (id < NOP) {
                const int op = id / NX, hxo = id % NX;
                const int hxp = (hxo + 1) & (NX - 1);
                if (op == 0) {
                    double sv, cv;
                    lat_sincos(edx * s_ay[b][hxo], &sv, &cv);
                    s_sy[hxo] = sv;
                    s_cy[hxo] = cv;
                } else if (op == 1) {
                    s_sxy[hxo] = lat_sin(edx * ((s_ay[b][hxp] - s_ay[b][hxo]) - s_ax[b][NX + hxo] + s_ax[b][hxo]));
                } else {
                    s_syz[hxo] = lat_sin(edx * ((s_az[b][NX + hxo] - s_az[b][hxo]) - s_ayn[b][hxo] + s_ay[b][hxo]));
                }
            }
        }
        __syncthreads();

        // (C) forces, kick, drift
        {
            const unsigned o = oz + so;
            double pq[2], pa[3];
#pragma unroll
            for (int c = 0; c < 2; ++c) pq[c] = ld32(g.pi[c], o);
#pragma unroll
            for (int i = 0; i < 3; ++i) pa[i] = ld32(g.piA[i], o);
            const double sxy = s_sxy[ro], sxz = s_sxz[wo], syz = s_syz[ro];
            const double mag[3] = {(sxy - s_sxy[ro - NX]) + (sxz - sxzm),
                                   (-sxy + s_sxy[r * NX + xm]) + (syz - syzm),
                                   (-sxz + s_sxz[(r - 1) * NX + xm]) + (-syz + s_syz[ro - NX])};
            const double pr = w0[0], pim = w0[1];
            double d2r = 0.0, d2i = 0.0, J[3], grad2 = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                double qr, qi, rr, ri, sm, cm;
                if (i == 0) {
                    qr = s_p0[b][r * NX + xp]; qi = s_p1[b][r * NX + xp];
                    rr = s_p0[b][r * NX + xm]; ri = s_p1[b][r * NX + xm];
                    sm = s_sx[(r - 1) * NX + xm]; cm = s_cx[(r - 1) * NX + xm];
                } else if (i == 1) {
                    qr = s_p0[b][ro + NX]; qi = s_p1[b][ro + NX];
                    rr = s_p0[b][ro - NX]; ri = s_p1[b][ro - NX];
                    sm = s_sy[ro - NX]; cm = s_cy[ro - NX];
                } else {
                    qr = wp[0]; qi = wp[1];
                    rr = wm[0]; ri = wm[1];
                    sm = szm; cm = czm;
                }
                const int ow = i == 1 ? ro : wo;
                const double *Ls = i == 0 ? s_sx : (i == 1 ? s_sy : s_sz);
                const double *Lc = i == 0 ? s_cx : (i == 1 ? s_cy : s_cz);
                const double s = -Ls[ow], c = Lc[ow];   // V_i(n) = c + i s
                const double ar = c * qr - s * qi, ai = c * qi + s * qr;
                const double br = cm * rr - sm * ri, bi = cm * ri + sm * rr;
                d2r += ar - 2.0 * pr + br;
                d2i += ai - 2.0 * pim + bi;
                J[i] = g.e / g.dx * (pr * ai - pim * ar);
                if constexpr (EN) {
                    const double dr = ar - pr, di = ai - pim;
                    grad2 += dr * dr + di * di;
                }
            }
            const double m2 = 0.5 * (pr * pr + pim * pim);
            const double vp = 0.5 * g.lam * (m2 - g.v * g.v);
            const double F0 = la1 * (d2r * inv_dx2) - la3 * (vp * pr);
            const double F1 = la1 * (d2i * inv_dx2) - la3 * (vp * pim);
            const double q0 = pq[0] + ck * F0, q1 = pq[1] + ck * F1;
            if constexpr (MODE == kU1Energy) {
                // the energies and Gauss terms of u1_stage's energy mode
                double t[NQ];
                t[0] = 0.5 * (q0 * q0 + q1 * q1);
                t[1] = grad2 * inv_dx2 * 0.5;
                const double u = m2 - g.v * g.v;
                t[2] = 0.25 * g.lam * u * u;
                double ka = 0.0;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const double FA = la1 * (g.kappa_g * J[i]) - lm1 * (mag[i] * inv_edx3);
                    const double sa = pa[i] + ck * FA;
                    ka += sa * sa;
                }
                t[3] = ka / (2.0 * g.kappa_g);
                const double hxy = lat_sin(0.5 * th[0]), hxz = lat_sin(0.5 * th[1]), hyz = lat_sin(0.5 * th[2]);
                const double mg = 2.0 * hxy * hxy + 2.0 * hxz * hxz + 2.0 * hyz * hyz;
                t[4] = mg / (g.kappa_g * g.e * g.e * g.dx * g.dx * g.dx * g.dx);
                const int yy = y0 + r - 1;
                const unsigned oxm = oz + (unsigned)(yy * N + xm);
                const unsigned oym = oz + (unsigned)((yy == 0 ? N - 1 : yy - 1) * N + x);
                const unsigned ozm = (unsigned)(z == 0 ? N - 1 : z - 1) * NN + so;
                const double div = ((pa[0] - ld32(g.piA[0], oxm)) + (pa[1] - ld32(g.piA[1], oym)) +
                                    (pa[2] - ld32(g.piA[2], ozm))) / g.dx;
                const double charge = g.e * g.kappa_g * (pr * pq[1] - pim * pq[0]);
                const double G = div - charge;
                t[5] = fabs(G);
                t[6] = fabs(div + charge);
                t[7] = fabs(div) + fabs(charge);
                t[8] = fabs(G);
                t[9] = fabs(div);
                t[10] = fabs(charge);
#pragma unroll
                for (int k = 0; k < NQ; ++k) acc[k] = k < kU1Sums ? acc[k] + t[k] : fmax(acc[k], t[k]);
            } else {
                st32(g.pi[0], o, q0);
                st32(g.pi[1], o, q1);
                if constexpr (MODE == kU1Step) {
                    st32(g.phi_out[0], o, pr + hd * q0);
                    st32(g.phi_out[1], o, pim + hd * q1);
                }
                double ka = 0.0;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const double FA = la1 * (g.kappa_g * J[i]) - lm1 * (mag[i] * inv_edx3);
                    const double qa = pa[i] + ck * FA;
                    st32(g.piA[i], o, qa);
                    if constexpr (MODE == kU1Step) st32(g.A_out[i], o, a0[i] + hdA * qa);
                    if constexpr (MODE == kU1KickSums) ka += qa * qa;
                }
                if constexpr (MODE == kU1KickSums) {
                    // the terms the energy mode forms after this kick: there the
                    // stored momenta are q, qa and p + 0 F = p
                    double t[NQ];
                    t[0] = 0.5 * (q0 * q0 + q1 * q1);
                    t[1] = grad2 * inv_dx2 * 0.5;
                    const double u = m2 - g.v * g.v;
                    t[2] = 0.25 * g.lam * u * u;
                    t[3] = ka / (2.0 * g.kappa_g);
                    const double hxy = lat_sin(0.5 * th[0]), hxz = lat_sin(0.5 * th[1]), hyz = lat_sin(0.5 * th[2]);
                    const double mg = 2.0 * hxy * hxy + 2.0 * hxz * hxz + 2.0 * hyz * hyz;
                    t[4] = mg / (g.kappa_g * g.e * g.e * g.dx * g.dx * g.dx * g.dx);
#pragma unroll
                    for (int k = 5; k < NQ; ++k) t[k] = 0.0;
#pragma unroll
                    for (int k = 0; k < NQ; ++k) acc[k] = k < kU1Sums ? acc[k] + t[k] : fmax(acc[k], t[k]);
                }
            }
            czm = s_cz[wo];
            szm = s_sz[wo];
            sxzm = sxz;
            syzm = syz;
        }
        // no barrier here: plane z + 1 goes to the other psi / A buffers, and the
        // sines and phases read above are rewritten only after the next barrier
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            wm[c] = w0[c];
            w0[c] = wp[c];
            wp[c] = nps[c];
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            a0[i] = a1[i];
            a1[i] = na[i];
        }
    }

    if constexpr (EN) {
        // the block tree and last-block reduction of u1_stage's energy mode
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const double rv = k < kU1Sums ? wave_sum(acc[k]) : wave_max(acc[k]);
            if (lane == 0) lds_red[w * NQ + k] = rv;
        }
        __syncthreads();
        if (tid == 0) {
            for (int k = 0; k < NQ; ++k) {
                double rv = 0.0;
                for (int i = 0; i < NT / 64; ++i)
                    rv = k < kU1Sums ? rv + lds_red[i * NQ + k] : fmax(rv, lds_red[i * NQ + k]);
                store_agent(&g.partials[(size_t)lid * NQ + k], rv);
            }
            // defer: the block partials are combined by a kernel after this one
            last_flag = g.defer ? 0 : (ticket_arrive(g.ticket, gridDim.x) ? 1 : 0);
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
                const double rv = k < kU1Sums ? wave_sum(part[k]) : wave_max(part[k]);
                if (lane == 0) lds_red[w * NQ + k] = rv;
            }
            __syncthreads();
            if (tid == 0) {
                for (int k = 0; k < NQ; ++k) {
                    double rv = 0.0;
                    for (int i = 0; i < NT / 64; ++i)
                        rv = k < kU1Sums ? rv + lds_red[i * NQ + k] : fmax(rv, lds_red[i * NQ + k]);
                    if (k < kU1Sums) g.sc->sums[k] = rv;
                    else g.sc->maxes[k - kU1Sums] = rv;
                }
                __hip_atomic_store(g.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

}  // namespace lat
