// stage_su2.hpp -- SU(2) doublet with SU(2) links: the leapfrog pass
// (kick of the doublet momenta and electric fields, drift of the doublet and
// the links), the sync half kick, and the energy / Gauss reduction pass.
//
// Lattice system (sec. 3.2 SU(N) toolkit; sec. 5, eqs. higgsSU2-eom, SU2eom,
// GaussSU2-eom, energy-contrib, program variables with f_* = omega_*):
//   doublet Phi = (psi0, psi1)/sqrt2, psi0 = phi0 + i phi1, psi1 = phi2 + i phi3;
//   link U_i(n) = exp(-i g dx B_i^a T_a), T_a = sigma_a/2, stored as the unit
//   quaternion (w, x, y, z) with U = w I - i (x, y, z).sigma;
//   electric field E_i^a(n), conjugate to U_i(n) under U -> exp(-i eps g dx T_a) U.
// Hamiltonian per site: sum_c pi_c^2/2 + sum_i |U_i psi(n+i) - psi|^2/(2 dx^2)
//   + lambda/4 (|Phi|^2 - v^2)^2 + |E|^2/2 + 2/(g^2 dx^4) sum_{i<j} (2 - Tr P_ij),
//   P_ij(n) = U_i(n) U_j(n+i) U_i(n+j)^dag U_j(n)^dag.
// Kicks are minus its derivative:
//   pi_c  += ck [ (D^2 psi)_c - lambda/2 (|Phi|^2 - v^2) phi_c ]
//   E_i^a += ck [ (g/dx) Im(psi^dag T_a U_i psi(n+i))
//                 - 2/(g dx^3) vec_a(U_i sum_{j != i} (S+_ij + S-_ij)) ]
//   S+_ij = U_j(n+i) U_i(n+j)^dag U_j(n)^dag,  S-_ij = U_j(n+i-j)^dag U_i(n-j)^dag U_j(n-j)
// and the drifts phi += hd pi, U <- exp(-i hd g dx E^a T_a) U.
// One thread per site of each plane of a z column; neighbours through the
// caches.  Momenta are read at their own site only and updated in place;
// doublet and links are written out of place (the stencil reads the old values).
#pragma once
#include "common.hpp"

namespace lat {

struct SU2Args {
    const double *phi_in[4];
    double *phi_out[4];
    double *pi[4];
    const double *U_in[12];   // link i, component k at 4 i + k
    double *U_out[12];
    double *E[9];             // link i, colour a at 3 i + a
    // kSU2StepAoS: the doublet and the links as one 32-byte record per site
    // (phi0..phi3; w, x, y, z), read from *_in4 and written to *_out4
    const double4 *phi_in4;
    double4 *phi_out4;
    const double4 *U_in4[3];
    double4 *U_out4[3];
    int N, tiles_x, tiles_y, zc;   // zc: z planes per block
    int band;                      // > 0: y tiles per XCD band (tiles_y = 8 band), see su2_stage
    int down;                      // march the z column downward (sites are independent)
    double dx, g, lam, v;
    double ck;   // kick weight
    double hd;   // drift weight of the doublet (time times a^{alpha-3})
    // expanding background (sec. 5.5.2 kernels): the covariant Laplacian and
    // the current scale with la1 = a^{1+alpha}, the potential force with
    // la3 = a^{3+alpha}, the staple force with lam1 = a^{alpha-1}; hdU is the
    // link drift weight (time times a^{alpha-1}).  All 1 (hdU = hd) at a = 1.
    double la1, la3, lam1, hdU;
    // if not null: {ck, la1, la3, lam1, hd, hdU} from device memory (written by
    // the self-consistent scale-factor update)
    const double *dw;
    double *partials;
    unsigned *ticket;
    ScaleRecord *sc;
    int defer;   // summing passes: leave the block partials, take no ticket
};

// kSU2Drift: the drift alone (su2_drift), for a step pass whose kick weight is zero.
// kSU2KickSums: the kick-only pass that also leaves the volume sums [0, 5) of
// the kicked state, as an energy pass with zero kick weight after it would (in
// that pass's launch shape; Gauss terms not measured: the rest stays zero).
enum SU2Mode : int { kSU2Step = 0, kSU2Kick = 1, kSU2Energy = 2, kSU2StepAoS = 3, kSU2Drift = 4, kSU2KickSums = 5 };

// one 32-byte record through a 32-bit byte offset (valid while 32 N^3 < 2^32)
__device__ __forceinline__ double4 ld4(const double4 *base, unsigned i)
{
    return *(const double4 *)((const char *)base + (size_t)(i * 32u));
}
__device__ __forceinline__ void st4(double4 *base, unsigned i, double4 v)
{
    *(double4 *)((char *)base + (size_t)(i * 32u)) = v;
}

// Streamed accesses of the pass (the momenta, read and written once, and the
// output records): non-temporal when NT, so they do not displace the input
// records that neighbouring sites read again from L2.
typedef double su2_nd4 __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ double ld_s(const double *base, unsigned i)
{
    const double *p = (const double *)((const char *)base + (size_t)(i * 8u));
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT>
__device__ __forceinline__ void st_s(double *base, unsigned i, double v)
{
    double *p = (double *)((char *)base + (size_t)(i * 8u));
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}
template <bool NT>
__device__ __forceinline__ void st4_s(double4 *base, unsigned i, double4 v)
{
    if constexpr (NT) {
        const su2_nd4 w = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(w, (su2_nd4 *)((char *)base + (size_t)(i * 32u)));
    } else {
        st4(base, i, v);
    }
}
constexpr int kSU2Sums = 8, kSU2Maxes = 3;

// unit quaternion q = (w, v) for the matrix w I - i v.sigma
struct Q4 {
    double w, x, y, z;
};

__device__ __forceinline__ Q4 qmul(const Q4 &a, const Q4 &b)
{
    // (a0 - i a.s)(b0 - i b.s) = (a0 b0 - a.b) - i (a0 b + b0 a + a x b).s
    Q4 c;
    c.w = a.w * b.w - (a.x * b.x + a.y * b.y + a.z * b.z);
    c.x = a.w * b.x + b.w * a.x + (a.y * b.z - a.z * b.y);
    c.y = a.w * b.y + b.w * a.y + (a.z * b.x - a.x * b.z);
    c.z = a.w * b.z + b.w * a.z + (a.x * b.y - a.y * b.x);
    return c;
}

__device__ __forceinline__ Q4 qdag(const Q4 &a) { return Q4{a.w, -a.x, -a.y, -a.z}; }

__device__ __forceinline__ Q4 qadd(const Q4 &a, const Q4 &b) { return Q4{a.w + b.w, a.x + b.x, a.y + b.y, a.z + b.z}; }

// (r0 + i s0, r1 + i s1) = U (a + i b, c + i d), U = w I - i v.sigma
__device__ __forceinline__ void qapply(const Q4 &u, double a, double b, double c, double d, double &r0, double &s0,
                                       double &r1, double &s1)
{
    r0 = u.w * a + u.z * b - u.y * c + u.x * d;
    s0 = u.w * b - u.z * a - u.y * d - u.x * c;
    r1 = u.x * b + u.y * a + u.w * c - u.z * d;
    s1 = -u.x * a + u.y * b + u.w * d + u.z * c;
}

// Im(psi^dag T_a chi), a = 1..3, psi = (a + i b, c + i d), chi = (p + i q, r + i s)
__device__ __forceinline__ void isospin(double a, double b, double c, double d, double p, double q, double r, double s,
                                        double &j1, double &j2, double &j3)
{
    j1 = 0.5 * ((a * s - b * r) + (c * q - d * p));
    j2 = 0.5 * ((c * p + d * q) - (a * r + b * s));
    j3 = 0.5 * ((a * q - b * p) - (c * s - d * r));
}

// One site's pass.  Site indices are 32-bit element offsets (the caller
// checks 8 N^3 < 2^32), so every array access is a uniform base plus one
// 32-bit offset.  c[] = (x, y, z), cp[] / cm[] their periodic successors and
// predecessors.
// the pass weights of SU2Args, from device memory if SU2Args::dw is set
struct SU2W {
    double ck, la1, la3, lm1, hd, hdU;
};

__device__ inline SU2W su2_weights(const SU2Args &g)
{
    if (g.dw) return SU2W{g.dw[0], g.dw[1], g.dw[2], g.dw[3], g.dw[4], g.dw[5]};
    return SU2W{g.ck, g.la1, g.la3, g.lam1, g.hd, g.hdU};
}

template <int MODE, int NQ, bool NT>
__device__ __forceinline__ void su2_site(const SU2Args &g, const SU2W &wt, const int (&c)[3], const int (&cp)[3],
                                         const int (&cm)[3], double (&acc)[NQ])
{
    const unsigned N = (unsigned)g.N;
    auto off = [&](int x, int y, int z) { return (unsigned)x + N * ((unsigned)y + N * (unsigned)z); };
    // site index with coordinate i replaced by v (and optionally j by u)
    auto at1 = [&](int i, int v) {
        int q[3] = {c[0], c[1], c[2]};
        q[i] = v;
        return off(q[0], q[1], q[2]);
    };
    auto at2 = [&](int i, int v, int j, int u) {
        int q[3] = {c[0], c[1], c[2]};
        q[i] = v;
        q[j] = u;
        return off(q[0], q[1], q[2]);
    };
    constexpr bool AOS = MODE == kSU2StepAoS;
    auto L = [&](int i, unsigned m) {
        if constexpr (AOS) {
            const double4 v = ld4(g.U_in4[i], m);
            return Q4{v.x, v.y, v.z, v.w};
        } else {
            return Q4{ld32(g.U_in[4 * i], m), ld32(g.U_in[4 * i + 1], m), ld32(g.U_in[4 * i + 2], m),
                      ld32(g.U_in[4 * i + 3], m)};
        }
    };
    // the doublet at site m as (phi0, phi1, phi2, phi3)
    auto D = [&](unsigned m) {
        if constexpr (AOS) {
            return ld4(g.phi_in4, m);
        } else {
            return double4{ld32(g.phi_in[0], m), ld32(g.phi_in[1], m), ld32(g.phi_in[2], m), ld32(g.phi_in[3], m)};
        }
    };
    const unsigned n = off(c[0], c[1], c[2]);
    const double4 own = D(n);
    const double a0 = own.x, b0 = own.y, c0 = own.z, d0 = own.w;
    const double inv_dx2 = 1.0 / (g.dx * g.dx);
    const double gdx = g.g / g.dx;
    const double mcoef = 2.0 / (g.g * g.dx * g.dx * g.dx);

    double l0 = 0.0, l1 = 0.0, l2 = 0.0, l3 = 0.0;   // sum_i U psi(n+i) - 2 psi + U^dag psi(n-i)
    double grad2 = 0.0;
    double FE[9];
    Q4 Ul[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) Ul[i] = L(i, n);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const unsigned np = at1(i, cp[i]), nm = at1(i, cm[i]);
        double r0, s0, r1, s1;
        const double4 dp = D(np), dm = D(nm);
        qapply(Ul[i], dp.x, dp.y, dp.z, dp.w, r0, s0, r1, s1);
        double t0, u0, t1, u1;
        qapply(qdag(L(i, nm)), dm.x, dm.y, dm.z, dm.w, t0, u0, t1, u1);
        l0 += r0 - 2.0 * a0 + t0;
        l1 += s0 - 2.0 * b0 + u0;
        l2 += r1 - 2.0 * c0 + t1;
        l3 += s1 - 2.0 * d0 + u1;
        if (MODE == kSU2Energy || MODE == kSU2KickSums) {
            const double e0 = r0 - a0, e1 = s0 - b0, e2 = r1 - c0, e3 = s1 - d0;
            grad2 += e0 * e0 + e1 * e1 + e2 * e2 + e3 * e3;
        }
        double j1, j2, j3;
        isospin(a0, b0, c0, d0, r0, s0, r1, s1, j1, j2, j3);
        // staple sum of link i
        Q4 S{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (j == i) continue;
            const Q4 Sp = qmul(qmul(L(j, np), qdag(L(i, at1(j, cp[j])))), qdag(Ul[j]));   // U_j(n+i) U_i(n+j)^dag U_j^dag
            const Q4 Sm = qmul(qmul(qdag(L(j, at2(i, cp[i], j, cm[j]))), qdag(L(i, at1(j, cm[j])))),
                               L(j, at1(j, cm[j])));   // U_j(n+i-j)^dag U_i(n-j)^dag U_j(n-j)
            S = qadd(S, qadd(Sp, Sm));
        }
        const Q4 W = qmul(Ul[i], S);
        FE[3 * i + 0] = wt.la1 * (gdx * j1) - wt.lm1 * (mcoef * W.x);
        FE[3 * i + 1] = wt.la1 * (gdx * j2) - wt.lm1 * (mcoef * W.y);
        FE[3 * i + 2] = wt.la1 * (gdx * j3) - wt.lm1 * (mcoef * W.z);
    }
    const double m2 = 0.5 * (a0 * a0 + b0 * b0 + c0 * c0 + d0 * d0);
    const double vp = 0.5 * g.lam * (m2 - g.v * g.v);
    const double F[4] = {wt.la1 * (l0 * inv_dx2) - wt.la3 * (vp * a0), wt.la1 * (l1 * inv_dx2) - wt.la3 * (vp * b0),
                         wt.la1 * (l2 * inv_dx2) - wt.la3 * (vp * c0), wt.la1 * (l3 * inv_dx2) - wt.la3 * (vp * d0)};
    double pv[4], ev[9];
#pragma unroll
    for (int k = 0; k < 4; ++k) pv[k] = ld_s<NT>((const double *)g.pi[k], n);
#pragma unroll
    for (int k = 0; k < 9; ++k) ev[k] = ld_s<NT>((const double *)g.E[k], n);

    if (MODE == kSU2Energy) {
        double kin = 0.0, ke = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double s = pv[k] + wt.ck * F[k];
            kin += s * s;
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const double s = ev[k] + wt.ck * FE[k];
            ke += s * s;
        }
        acc[0] += 0.5 * kin;
        acc[1] += grad2 * inv_dx2 * 0.5;
        const double u = m2 - g.v * g.v;
        acc[2] += 0.25 * g.lam * u * u;
        acc[3] += 0.5 * ke;
        // magnetic: 2 - Tr P = 2 |p|^2 / (1 + p0) per plaquette (unitary P)
        double mg = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i + 1; j < 3; ++j) {
                const Q4 Pij = qmul(qmul(Ul[i], L(j, at1(i, cp[i]))), qmul(qdag(L(i, at1(j, cp[j]))), qdag(Ul[j])));
                mg += 2.0 * (Pij.x * Pij.x + Pij.y * Pij.y + Pij.z * Pij.z) / (1.0 + Pij.w);
            }
        acc[4] += 2.0 * mg / (g.g * g.g * g.dx * g.dx * g.dx * g.dx);
        // Gauss residual of the stored pairing: covariant backward divergence
        // of E (E_i(n-i) carried to n by U_i(n-i)^dag (E.sigma) U_i(n-i), a
        // rotation of the vector by the inverse of U's) minus the charge
        double dv[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const unsigned nm = at1(i, cm[i]);
            const Q4 u = L(i, nm);
            const double ex = ld32((const double *)g.E[3 * i], nm), ey = ld32((const double *)g.E[3 * i + 1], nm),
                         ez = ld32((const double *)g.E[3 * i + 2], nm);
            // t = 2 v x e ; e' = e - w t + v x t  (rotation by the inverse)
            const double tx2 = 2.0 * (u.y * ez - u.z * ey), ty2 = 2.0 * (u.z * ex - u.x * ez),
                         tz2 = 2.0 * (u.x * ey - u.y * ex);
            const double rx = ex - u.w * tx2 + (u.y * tz2 - u.z * ty2);
            const double ry = ey - u.w * ty2 + (u.z * tx2 - u.x * tz2);
            const double rz = ez - u.w * tz2 + (u.x * ty2 - u.y * tx2);
            dv[0] += (ev[3 * i] - rx) / g.dx;
            dv[1] += (ev[3 * i + 1] - ry) / g.dx;
            dv[2] += (ev[3 * i + 2] - rz) / g.dx;
        }
        double q1, q2, q3;
        isospin(a0, b0, c0, d0, pv[0], pv[1], pv[2], pv[3], q1, q2, q3);
        const double ch[3] = {g.g * q1, g.g * q2, g.g * q3};
        double G2 = 0.0, D2 = 0.0, C2 = 0.0, S2 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            G2 += (dv[k] - ch[k]) * (dv[k] - ch[k]);
            D2 += dv[k] * dv[k];
            C2 += ch[k] * ch[k];
            S2 += (dv[k] + ch[k]) * (dv[k] + ch[k]);
        }
        const double Gn = sqrt(G2), Dn = sqrt(D2), Cn = sqrt(C2);
        acc[5] += Gn;
        acc[6] += sqrt(S2);
        acc[7] += Dn + Cn;
        acc[8] = fmax(acc[8], Gn);
        acc[9] = fmax(acc[9], Dn);
        acc[10] = fmax(acc[10], Cn);
    } else {
        double pn[4], en[9];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            pn[k] = pv[k] + wt.ck * F[k];
            st_s<NT>(g.pi[k], n, pn[k]);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            en[k] = ev[k] + wt.ck * FE[k];
            st_s<NT>(g.E[k], n, en[k]);
        }
        if constexpr (MODE == kSU2KickSums) {
            // the terms the energy mode forms after this kick, where the stored
            // momenta are pn, en and p + 0 F = p
            double kin = 0.0, ke = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) kin += pn[k] * pn[k];
#pragma unroll
            for (int k = 0; k < 9; ++k) ke += en[k] * en[k];
            acc[0] += 0.5 * kin;
            acc[1] += grad2 * inv_dx2 * 0.5;
            const double u = m2 - g.v * g.v;
            acc[2] += 0.25 * g.lam * u * u;
            acc[3] += 0.5 * ke;
            double mg = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = i + 1; j < 3; ++j) {
                    const Q4 Pij =
                        qmul(qmul(Ul[i], L(j, at1(i, cp[i]))), qmul(qdag(L(i, at1(j, cp[j]))), qdag(Ul[j])));
                    mg += 2.0 * (Pij.x * Pij.x + Pij.y * Pij.y + Pij.z * Pij.z) / (1.0 + Pij.w);
                }
            acc[4] += 2.0 * mg / (g.g * g.g * g.dx * g.dx * g.dx * g.dx);
        }
        if (MODE == kSU2Step || AOS) {
            const double4 po{a0 + wt.hd * pn[0], b0 + wt.hd * pn[1], c0 + wt.hd * pn[2], d0 + wt.hd * pn[3]};
            if constexpr (AOS) {
                st4_s<NT>(g.phi_out4, n, po);
            } else {
                st_s<NT>(g.phi_out[0], n, po.x);
                st_s<NT>(g.phi_out[1], n, po.y);
                st_s<NT>(g.phi_out[2], n, po.z);
                st_s<NT>(g.phi_out[3], n, po.w);
            }
            const double hgdx = wt.hdU * g.g * g.dx;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                // exp(-i hdU g dx E.T) = cos(th/2) - i sin(th/2) e.sigma, th = hdU g dx |E|
                const double ex = en[3 * i], ey = en[3 * i + 1], ez = en[3 * i + 2];
                const double len = sqrt(ex * ex + ey * ey + ez * ez);
                double sh, chh;
                sincos(0.5 * (hgdx * len), &sh, &chh);
                Q4 R{chh, 0.0, 0.0, 0.0};
                if (len > 0.0) {
                    R.x = sh * ex / len;
                    R.y = sh * ey / len;
                    R.z = sh * ez / len;
                }
                const Q4 Un = qmul(R, Ul[i]);
                if constexpr (AOS) {
                    st4_s<NT>(g.U_out4[i], n, double4{Un.w, Un.x, Un.y, Un.z});
                } else {
                    st_s<NT>(g.U_out[4 * i], n, Un.w);
                    st_s<NT>(g.U_out[4 * i + 1], n, Un.x);
                    st_s<NT>(g.U_out[4 * i + 2], n, Un.y);
                    st_s<NT>(g.U_out[4 * i + 3], n, Un.z);
                }
            }
        }
    }
}

// Drift only, with the record's weights hd = dw[4], hdU = dw[5], on the plain
// arrays, one site per thread: the doublet phi + hd pi and the links
// exp(-i hdU g dx E.T) U, the step pass's drift formed by the same expressions
// (the compiler may contract them differently: equal to rounding).  The
// self-consistent steps' drift pass has zero kick weight, where a step pass
// computes the forces for nothing (p + 0 F = p) and rewrites the momenta and
// electric fields unchanged: this reads 29 arrays and writes 16.
__global__ void __launch_bounds__(256) su2_drift(const SU2Args g, unsigned vol)
{
    const unsigned n = blockIdx.x * 256u + threadIdx.x;
    if (n >= vol) return;
    const double hd = g.dw[4], hdU = g.dw[5];
#pragma unroll
    for (int k = 0; k < 4; ++k) g.phi_out[k][n] = g.phi_in[k][n] + hd * g.pi[k][n];
    const double hgdx = hdU * g.g * g.dx;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double ex = g.E[3 * i][n], ey = g.E[3 * i + 1][n], ez = g.E[3 * i + 2][n];
        const double len = sqrt(ex * ex + ey * ey + ez * ez);
        double sh, chh;
        sincos(0.5 * (hgdx * len), &sh, &chh);
        Q4 R{chh, 0.0, 0.0, 0.0};
        if (len > 0.0) {
            R.x = sh * ex / len;
            R.y = sh * ey / len;
            R.z = sh * ez / len;
        }
        const Q4 U{g.U_in[4 * i][n], g.U_in[4 * i + 1][n], g.U_in[4 * i + 2][n], g.U_in[4 * i + 3][n]};
        const Q4 Un = qmul(R, U);
        g.U_out[4 * i][n] = Un.w;
        g.U_out[4 * i + 1][n] = Un.x;
        g.U_out[4 * i + 2][n] = Un.y;
        g.U_out[4 * i + 3][n] = Un.z;
    }
}

// Block = TX x TY sites of a z column [z0, z0 + zc).  Logical blocks are
// dealt to the XCDs in contiguous ranges.  Plane-wide order (band = 0): x
// tile fastest, then y tile, then z chunk, so an XCD's resident blocks march
// whole planes together.  Band order (band > 0): XCD k owns the y tiles
// [k band, (k + 1) band) over all z chunks, x tile fastest, then y tile, then
// z chunk (in reverse when marching down), so its resident blocks cover a
// compact region and the records of the planes z - 1, z, z + 1 that a site's
// stencil reads stay in that XCD's L2 between their uses.
// Two waves per SIMD in every mode: the kick-only and energy passes then
// spill 24 and 28 bytes per lane to scratch instead of holding 256 VGPRs and
// 6 AGPRs at one wave (energy pass 361 -> 298 us at 128^3, self-consistent
// leapfrog step 1316 -> 1133 us); the record step pass fits in 240 VGPRs.
template <int TX, int TY, int MODE, bool STREAM>
__global__ void __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(2))) su2_stage(const SU2Args g)
{
    constexpr int NT = TX * TY;
    constexpr int NQ = kSU2Sums + kSU2Maxes;
    __shared__ double lds_red[(NT / 64) * NQ];
    __shared__ int last_flag;

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int lid = xcd_logical_block(blockIdx.x, gridDim.x);
    const int N = g.N;
    int bx, by, bz;
    if (g.band > 0) {
        const int per = gridDim.x / 8;   // the host launches 8 tiles_x band z-chunk blocks
        const int xcd = lid / per, r = lid % per;
        bx = r % g.tiles_x;
        const int r2 = r / g.tiles_x;
        by = xcd * g.band + r2 % g.band;
        bz = r2 / g.band;
        if (g.down) bz = (N + g.zc - 1) / g.zc - 1 - bz;
    } else {
        bx = lid % g.tiles_x;
        const int rest = lid / g.tiles_x;
        by = rest % g.tiles_y;
        bz = rest / g.tiles_y;
    }
    const int x = bx * TX + tx, y = by * TY + ty;
    const int z0 = bz * g.zc, z1 = min(z0 + g.zc, N);

    double acc[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) acc[k] = 0.0;

    const SU2W wt = su2_weights(g);
    if (x < N && y < N) {
        int c[3] = {x, y, z0}, cp[3], cm[3];
        cp[0] = x + 1 == N ? 0 : x + 1;
        cm[0] = x == 0 ? N - 1 : x - 1;
        cp[1] = y + 1 == N ? 0 : y + 1;
        cm[1] = y == 0 ? N - 1 : y - 1;
        for (int s = 0; s < z1 - z0; ++s) {
            const int z = g.down ? z1 - 1 - s : z0 + s;
            c[2] = z;
            cp[2] = z + 1 == N ? 0 : z + 1;
            cm[2] = z == 0 ? N - 1 : z - 1;
            su2_site<MODE, NQ, STREAM>(g, wt, c, cp, cm, acc);
        }
    }

    if constexpr (MODE == kSU2Energy || MODE == kSU2KickSums) {
        // block reduction: sums for [0, kSU2Sums), maxes for the rest; the last
        // block (ticket) combines the block partials in block order
        const int lane = tid & 63, w = tid >> 6;
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const double r = k < kSU2Sums ? wave_sum(acc[k]) : wave_max(acc[k]);
            if (lane == 0) lds_red[w * NQ + k] = r;
        }
        __syncthreads();
        if (tid == 0) {
            for (int k = 0; k < NQ; ++k) {
                double r = 0.0;
                for (int i = 0; i < NT / 64; ++i)
                    r = k < kSU2Sums ? r + lds_red[i * NQ + k] : fmax(r, lds_red[i * NQ + k]);
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
                    part[k] = k < kSU2Sums ? part[k] + v : fmax(part[k], v);
                }
            }
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const double r = k < kSU2Sums ? wave_sum(part[k]) : wave_max(part[k]);
                if (lane == 0) lds_red[w * NQ + k] = r;
            }
            __syncthreads();
            if (tid == 0) {
                for (int k = 0; k < NQ; ++k) {
                    double r = 0.0;
                    for (int i = 0; i < NT / 64; ++i)
                        r = k < kSU2Sums ? r + lds_red[i * NQ + k] : fmax(r, lds_red[i * NQ + k]);
                    if (k < kSU2Sums) g.sc->sums[k] = r;
                    else g.sc->maxes[k - kSU2Sums] = r;
                }
                __hip_atomic_store(g.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

}  // namespace lat

namespace lat {

// SoA <-> per-site records of the doublet and the links (kSU2StepAoS):
// a[0..3] the doublet components, a[4 + 4 i + k] component k of link i;
// r[0] the doublet records, r[1 + i] those of link i.
struct SU2Soa {
    double *a[16];
};
struct SU2Aos {
    double4 *r[4];
};

__global__ void su2_to_aos(const SU2Soa s, const SU2Aos d, size_t V)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < V; n += (size_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            d.r[q][n] = double4{s.a[4 * q][n], s.a[4 * q + 1][n], s.a[4 * q + 2][n], s.a[4 * q + 3][n]};
    }
}

__global__ void su2_from_aos(const SU2Aos s, const SU2Soa d, size_t V)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < V; n += (size_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double4 v = s.r[q][n];
            d.a[4 * q][n] = v.x;
            d.a[4 * q + 1][n] = v.y;
            d.a[4 * q + 2][n] = v.z;
            d.a[4 * q + 3][n] = v.w;
        }
    }
}

}  // namespace lat
