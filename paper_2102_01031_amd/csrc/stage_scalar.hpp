// stage_scalar.hpp -- one fused stencil pass over real scalar fields.
//
// Per site (sec. 4.5.2 Hamiltonian form; sec. 3.1 lattice derivatives):
//   drift on load      phi += dload * pi                      (all points the stencil reads)
//   Laplacian          Lap phi = dx^-2 sum_i [phi(n+i) - 2 phi(n) + phi(n-i)]  (periodic)
//   kernel             F_s = a^{1+alpha} Lap phi_s - a^{3+alpha} dV/dphi_s
//                      V = lambda/4 phi^4 (+ q/2 phi^2 chi^2 for two fields, sec. 4.2)
//   kick               pi += c1 F   -> momenta at the kick point
//   reductions         sum pi_s^2, sum_i (grad+_i phi_s)^2, sum V_m (float64)
//   kick               pi += c2 F
//   drift at end       phi += dend * pi                       (leapfrog only)
//
// Tiling: a block owns a TX x TY column of sites and marches through a chunk of
// z planes.  The drifted phi of the current plane (plus a one-site halo in x
// and y) sits in LDS; phi at z-1, z, z+1 of the block's own column sits in
// registers.  Global loads run one plane ahead of their use (own column two
// planes, halo one plane) so HBM latency overlaps the compute of the current
// plane.  Arrays read with a halo are written to the other buffer of a
// ping-pong pair; momenta read only at the own site may be updated in place.
//
// Reductions are deterministic: per-thread float64 partials over the block's
// planes, a fixed wavefront/LDS tree per block, one partial per block, and the
// last block to finish (ticket counter) sums the partials in block order.  In
// the self-consistent mode that block also advances b and a and writes the
// drift and kick coefficients of the next pass.
#pragma once
#include "common.hpp"

namespace lat {

template <typename T>
struct ScalarArgs {
    const T *phi_in[2];
    const T *pi_in[2];
    T *phi_out[2];
    T *pi_out[2];
    int N, zc, tiles_x, tiles_y;
    int y_fastest;          // whole-row kernel block order: 0 z chunk fastest, 1 y tile fastest
    int down;               // whole-row kernel: march each z chunk downward
    int zpair;              // whole-row kernel: odd z chunks march the other way (see stage_rows.hpp)
    int cached_out;         // whole-row kernel: ordinary stores (else non-temporal)
    int split;              // whole-row kernel, phased cache policies: first phase = split/8 of the march
    double inv_dx2;
    double lam, q;
    const PassCoef *coef;   // this pass
    PassCoef *coef_next;    // next pass (self-consistent mode)
    double *partials;       // [blocks][3*NF]
    unsigned *ticket;
    ScaleRecord *sc;
    int last_mode;
    double alpha, kappa2, inv_vol;
    // Deferred finalisation of the self-consistent passes of a lattice_step call.
    // A deferring pass (defer = 1) stores its block sums to `partials` with
    // plain stores and takes no ticket: no block waits on a device-wide fence.
    // The next pass finalises them in its prologue (fin != null): every block
    // sums the fin_nb partials in block order, applies the scale-factor update
    // of fin_mode with the previous pass's coefficients fin_coef to the record
    // fin_in, and takes the resulting kick and drift factors as its own; block 0
    // writes the updated record to fin_out.  The kernel boundary between the
    // passes orders the stores and loads.
    int defer;
    int fin_nb, fin_mode;
    const double *fin;
    const PassCoef *fin_coef;
    const ScaleRecord *fin_in;
    ScaleRecord *fin_out;
};

// Scale-factor half kicks and drift of the self-consistent mode (sec. 4.5.2,
// kernel K_a; second Friedmann equation eq. NewFriedmannEQsII):
//   E_K = sum_s <pi_s^2>/(2 a^6), E_G = sum_s <(grad+ phi_s)^2>/(2 a^2), E_V = <V>
//   K_a = a^{2 alpha+1}/3 kappa^2 [(alpha-2) E_K + alpha E_G + (alpha+1) E_V]
//   b += cL K_a; b += cR K_a; a' = a + h b; next drift h ((a + a')/2)^{alpha-3}
// The outcome of a reducing pass's scale-factor update.
struct SelfOut {
    double a, b, t;            // after the update (b kicked, a drifted)
    double ka1, ka3, dload;    // the next pass's kick factors and drift-on-load coefficient
    double a0, bl;             // a at the kick point, b after the left half kick only
};

// b and a after the update, from the two powers of the current a that the
// kernel K_a needs (a6 = a^6, p21 = a^{2 alpha + 1}).
struct SelfPre {
    double b, bl, a1;
};

template <int NF>
__device__ inline SelfPre self_core_vv(const PassCoef &C, const double *fin, const ScaleRecord *S, double alpha,
                                       double kappa2, double inv_vol, double inv_dx2, double a6, double p21)
{
    double a = S->a, b = S->b;
    double sk = 0.0, sg = 0.0, sv = 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        sk += fin[f];
        sg += fin[NF + f];
        sv += fin[2 * NF + f];
    }
    const double EK = sk * inv_vol / (2.0 * a6);
    const double EG = sg * inv_dx2 * inv_vol / (2.0 * a * a);
    const double EV = sv * inv_vol;
    const double Ka = p21 / 3.0 * kappa2 * ((alpha - 2.0) * EK + alpha * EG + (alpha + 1.0) * EV);
    b += C.cL * Ka;
    const double bl = b;
    b += C.cR * Ka;
    return SelfPre{b, bl, a + C.h * b};
}

// Leapfrog with self-consistent expansion (staggered: a at integer times, b
// half a step behind).  The pass kicked the momenta at time n and reduced
// the kicked momenta squared (fin[f]), E_G and E_V of phi_n; the momenta
// before the kick are those the previous kick reduced (sums[kPiPrev + f]).
//   b += cL K_a(a_n, E_K(before), E_G, E_V) + cR K_a(a_n, E_K(after), E_G, E_V)
//   a' = a + h b; next drift h ((a + a')/2)^{alpha-3}
// A full kick has cL = cR = h/2 (E_K the mean of the two), the half kick from
// synchronised momenta cL = 0, cR = h/2, and the sync kick (which reduced the
// momenta before its kick) cL = 0, cR = h/2 with h = 0.
template <int NF>
__device__ inline SelfPre self_core_lf(const PassCoef &C, const double *fin, const ScaleRecord *S, double alpha,
                                       double kappa2, double inv_vol, double inv_dx2, double a6, double p21)
{
    double a = S->a, b = S->b;
    double sk0 = 0.0, sk1 = 0.0, sg = 0.0, sv = 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        sk0 += S->sums[kPiPrev + f];
        sk1 += fin[f];
        sg += fin[NF + f];
        sv += fin[2 * NF + f];
    }
    const double EG = sg * inv_dx2 * inv_vol / (2.0 * a * a);
    const double EV = sv * inv_vol;
    const double pre = p21 / 3.0 * kappa2;
    const double K0 = pre * ((alpha - 2.0) * (sk0 * inv_vol / (2.0 * a6)) + alpha * EG + (alpha + 1.0) * EV);
    const double K1 = pre * ((alpha - 2.0) * (sk1 * inv_vol / (2.0 * a6)) + alpha * EG + (alpha + 1.0) * EV);
    const double bl = b + C.cL * K0;
    b += C.cL * K0 + C.cR * K1;
    return SelfPre{b, bl, a + C.h * b};
}

template <int NF>
__device__ inline SelfPre self_core(int mode, const PassCoef &C, const double *fin, const ScaleRecord *S,
                                    double alpha, double kappa2, double inv_vol, double inv_dx2, double a6, double p21)
{
    return mode == kLastSelfLF ? self_core_lf<NF>(C, fin, S, alpha, kappa2, inv_vol, inv_dx2, a6, p21)
                               : self_core_vv<NF>(C, fin, S, alpha, kappa2, inv_vol, inv_dx2, a6, p21);
}

// The update by one thread: K_a needs pow(a, 6) and pow(a, 2 alpha + 1), the
// next pass pow(a1, 1 + alpha), pow(a1, 3 + alpha) and pow((a + a1)/2, alpha - 3).
template <int NF>
__device__ inline SelfOut self_compute_mode(int mode, const PassCoef &C, const double *fin, const ScaleRecord *S,
                                            double alpha, double kappa2, double inv_vol, double inv_dx2)
{
    const double a = S->a;
    const SelfPre p = self_core<NF>(mode, C, fin, S, alpha, kappa2, inv_vol, inv_dx2, pow(a, 6.0),
                                    pow(a, 2.0 * alpha + 1.0));
    return SelfOut{p.a1, p.b, C.t_next, pow(p.a1, 1.0 + alpha), pow(p.a1, 3.0 + alpha),
                   C.h * pow(0.5 * (a + p.a1), alpha - 3.0), a, p.bl};
}

// The same update by the 64 lanes of one wave (fin valid in every lane): the
// powers of each stage are evaluated side by side in lanes 0 .. 2, so the
// update waits for two pow latencies instead of five.  Bitwise equal to
// self_compute_mode.
template <int NF>
__device__ inline SelfOut self_compute_wave(int mode, const PassCoef &C, const double *fin, const ScaleRecord *S,
                                            double alpha, double kappa2, double inv_vol, double inv_dx2)
{
    const int lane = threadIdx.x & 63;
    const double a = S->a;
    const double e1 = pow(a, lane == 0 ? 6.0 : 2.0 * alpha + 1.0);
    const SelfPre p = self_core<NF>(mode, C, fin, S, alpha, kappa2, inv_vol, inv_dx2, __shfl(e1, 0, 64),
                                    __shfl(e1, 1, 64));
    const double base = lane == 2 ? 0.5 * (a + p.a1) : p.a1;
    const double ex = lane == 0 ? 1.0 + alpha : (lane == 1 ? 3.0 + alpha : alpha - 3.0);
    const double e2 = pow(base, ex);
    return SelfOut{p.a1, p.b, C.t_next, __shfl(e2, 0, 64), __shfl(e2, 1, 64), C.h * __shfl(e2, 2, 64), a, p.bl};
}

// the record after the update: a, b, t, the raw sums, and for the leapfrog the
// kicked momenta's sums for the next kick; (a, b) at the kick point into traj
// when the pass asks for it
template <int NF>
__device__ inline void self_store(int mode, const SelfOut &o, const double *fin, ScaleRecord *S, double *traj)
{
    if (traj) {
        traj[0] = o.a0;
        traj[1] = o.bl;
    }
#pragma unroll
    for (int k = 0; k < 3 * NF; ++k) S->sums[k] = fin[k];
    if (mode == kLastSelfLF) {
#pragma unroll
        for (int f = 0; f < NF; ++f) S->sums[kPiPrev + f] = fin[f];
    }
    S->a = o.a;
    S->b = o.b;
    S->t = o.t;
}

template <int NF>
__device__ inline void self_update(const PassCoef &C, const double *fin, ScaleRecord *S, PassCoef *Nx, double alpha,
                                   double kappa2, double inv_vol, double inv_dx2)
{
    const SelfOut o = self_compute_mode<NF>(kLastSelf, C, fin, S, alpha, kappa2, inv_vol, inv_dx2);
    Nx->ka1 = o.ka1;
    Nx->ka3 = o.ka3;
    Nx->dload = o.dload;
    self_store<NF>(kLastSelf, o, fin, S, C.traj);
}

template <int NF>
__device__ inline void self_update_lf(const PassCoef &C, const double *fin, ScaleRecord *S, PassCoef *Nx,
                                      double alpha, double kappa2, double inv_vol, double inv_dx2)
{
    const SelfOut o = self_compute_mode<NF>(kLastSelfLF, C, fin, S, alpha, kappa2, inv_vol, inv_dx2);
    Nx->ka1 = o.ka1;
    Nx->ka3 = o.ka3;
    Nx->dload = o.dload;
    self_store<NF>(kLastSelfLF, o, fin, S, C.traj);
}

// Prologue of a pass that finalises the previous pass's deferred sums: the
// block sums the partials in block order (as the last block of a ticketed pass
// does), the first wave applies the update, and the new kick and drift
// factors are returned to every thread in C.
template <int NT, int NF, typename T>
__device__ inline void finalise_prologue(const ScalarArgs<T> &g, double *lds_red, double *lds_coef, PassCoef &C)
{
    constexpr int NQ = 3 * NF;
    const int tid = threadIdx.x;
    double part[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) part[k] = 0.0;
    for (int i = tid; i < g.fin_nb; i += NT) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) part[k] += g.fin[(size_t)i * NQ + k];
    }
    double fin[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) fin[k] = 0.0;
    block_sums<NT, NQ>(part, lds_red, fin);
    if (tid < 64) {
        // the sums from thread 0 to its wave, which applies the update
#pragma unroll
        for (int k = 0; k < NQ; ++k) fin[k] = __shfl(fin[k], 0, 64);
        const SelfOut o = self_compute_wave<NF>(g.fin_mode, *g.fin_coef, fin, g.fin_in, g.alpha, g.kappa2,
                                                g.inv_vol, g.inv_dx2);
        if (tid == 0) {
            lds_coef[0] = o.ka1;
            lds_coef[1] = o.ka3;
            lds_coef[2] = o.dload;
            if (blockIdx.x == 0) self_store<NF>(g.fin_mode, o, fin, g.fin_out, g.fin_coef->traj);
        }
    }
    __syncthreads();
    C.ka1 = lds_coef[0];
    C.ka3 = lds_coef[1];
    C.dload = lds_coef[2];
}

// The deferred sums of the last pass of a call, finalised by one block of NT
// threads (NT as the stencil kernel's, so the sums are added in the same order).
template <int NT, int NF>
__global__ void __launch_bounds__(NT) self_finish(const double *partials, int nb, int mode, const PassCoef *C,
                                                  const ScaleRecord *Sin, ScaleRecord *Sout, PassCoef *Nx,
                                                  double alpha, double kappa2, double inv_vol, double inv_dx2)
{
    constexpr int NQ = 3 * NF;
    __shared__ double lds_red[(NT / 64) * NQ];
    const int tid = threadIdx.x;
    double part[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) part[k] = 0.0;
    for (int i = tid; i < nb; i += NT) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) part[k] += partials[(size_t)i * NQ + k];
    }
    double fin[NQ];
    block_sums<NT, NQ>(part, lds_red, fin);
    if (tid == 0) {
        const SelfOut o = self_compute_mode<NF>(mode, *C, fin, Sin, alpha, kappa2, inv_vol, inv_dx2);
        Nx->ka1 = o.ka1;
        Nx->ka3 = o.ka3;
        Nx->dload = o.dload;
        if (Sout != Sin) {
            // carry what the update does not rewrite (the leapfrog's momentum sums)
            for (int k = 0; k < kMaxQ; ++k) Sout->sums[k] = Sin->sums[k];
        }
        self_store<NF>(mode, o, fin, Sout, C->traj);
    }
}

// copy of a record (one thread)
__global__ void record_copy(const ScaleRecord *src, ScaleRecord *dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

template <typename T, int NF, int TX, int TY, bool DLOAD, bool DEND, bool RED, bool WPHI, bool WPI>
__global__ void __launch_bounds__(TX *TY) scalar_stage(const ScalarArgs<T> g)
{
    constexpr int NT = TX * TY;
    constexpr int NQ = 3 * NF;
    constexpr int NH = 2 * TX + 2 * TY;
    constexpr int LX = TX + 2;
    static_assert(NH <= NT, "halo cells exceed the block's threads");
    static_assert(NT % 64 == 0, "block must be whole wavefronts");

    __shared__ T lds[2][NF][(TY + 2) * LX];
    __shared__ double lds_red[(NT / 64) * NQ];
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

    // own column (threads past the lattice edge hold wrapped copies so that
    // the LDS row always contains the periodic neighbours of valid sites)
    const bool valid = (x0 + tx < N) && (y0 + ty < N);
    const int own = ((x0 + tx) % N) + N * ((y0 + ty) % N);
    const int oslot = (1 + ty) * LX + 1 + tx;

    // halo cell of this thread: bottom row, top row, left column, right column
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

    PassCoef C = *g.coef;
    if (g.fin) {
        __shared__ double lds_coef[4];
        finalise_prologue<NT, NF>(g, lds_red, lds_coef, C);
    }
    const T dl = (T)C.dload, c1 = (T)C.c1, c2 = (T)C.c2, de = (T)C.dend;
    const T ka1 = (T)C.ka1, ka3 = (T)C.ka3, idx2 = (T)g.inv_dx2;
    const T lam = (T)g.lam, qc = (T)g.q;
    const double lamd = g.lam, qd = g.q;

    T fm[NF], f0[NF], fp[NF], p0[NF], pp[NF];
    // two register sets for loads in flight, swapped between consecutive planes:
    // own column raw plane z+2 and halo raw plane z+1 (set "in"), filled one plane
    // earlier; the plane's loads go to set "out".
    T ownA_f[NF], ownA_p[NF], haloA_f[NF], haloA_p[NF];
    T ownB_f[NF], ownB_p[NF], haloB_f[NF], haloB_p[NF];

    {
        const size_t om = (size_t)(z0 == 0 ? N - 1 : z0 - 1) * NN;
        const size_t o0 = (size_t)z0 * NN;
        const size_t o1 = (size_t)((z0 + 1) % N) * NN;
        // clamped like the in-loop prefetch: a plane past the chunk is never used
        const size_t o2 = (size_t)(min(z0 + 2, z1) % N) * NN;
        const size_t oh1 = (size_t)(min(z0 + 1, z1 - 1) % N) * NN;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const T *P = g.phi_in[f];
            const T *Q = g.pi_in[f];
            const T a = P[om + own];
            fm[f] = DLOAD ? a + dl * Q[om + own] : a;
            const T b = P[o0 + own];
            p0[f] = Q[o0 + own];
            f0[f] = DLOAD ? b + dl * p0[f] : b;
            const T c = P[o1 + own];
            pp[f] = Q[o1 + own];
            fp[f] = DLOAD ? c + dl * pp[f] : c;
            ownA_f[f] = P[o2 + own];
            ownA_p[f] = Q[o2 + own];
            haloA_f[f] = haloA_p[f] = T(0);
            lds[0][f][oslot] = f0[f];
            if (has_halo) {
                T h = P[o0 + hoff];
                if (DLOAD) h += dl * Q[o0 + hoff];
                lds[0][f][hslot] = h;
                haloA_f[f] = P[oh1 + hoff];
                if (DLOAD) haloA_p[f] = Q[oh1 + hoff];
            }
        }
    }
    __syncthreads();

    double acc[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) acc[k] = 0.0;

    auto plane = [&](const int z, T (&oci_f)[NF], T (&oci_p)[NF], T (&hci_f)[NF], T (&hci_p)[NF],
                     T (&ono_f)[NF], T (&ono_p)[NF], T (&hno_f)[NF], T (&hno_p)[NF]) {
        const int cur = (z - z0) & 1, nxt = cur ^ 1;
        // (A) loads one plane ahead: own column z+3, halo z+2 (clamped to the chunk)
        int zo = min(z + 3, z1);
        if (zo >= N) zo -= N;
        int zh = min(z + 2, z1 - 1);
        if (zh >= N) zh -= N;
        const size_t o3 = (size_t)zo * NN, o2 = (size_t)zh * NN;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            ono_f[f] = g.phi_in[f][o3 + own];
            ono_p[f] = g.pi_in[f][o3 + own];
            if (has_halo) {
                hno_f[f] = g.phi_in[f][o2 + hoff];
                if (DLOAD) hno_p[f] = g.pi_in[f][o2 + hoff];
            }
        }
        // (B) LDS plane z+1 from registers
        if (z + 1 < z1) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                lds[nxt][f][oslot] = fp[f];
                if (has_halo) lds[nxt][f][hslot] = DLOAD ? hci_f[f] + dl * hci_p[f] : hci_f[f];
            }
        }
        // (C) the site (x, y, z)
        {
            const size_t oz = (size_t)z * NN + own;
            T xp[NF], yp[NF], lap[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const T *L = lds[cur][f];
                const T xm = L[oslot - 1];
                xp[f] = L[oslot + 1];
                const T ym = L[oslot - LX];
                yp[f] = L[oslot + LX];
                const T c0 = f0[f];
                lap[f] = ((xp[f] - T(2) * c0 + xm) + (yp[f] - T(2) * c0 + ym) + (fp[f] - T(2) * c0 + fm[f])) * idx2;
            }
            T dV[NF];
            if constexpr (NF == 1) {
                const T u = f0[0];
                dV[0] = lam * u * u * u;
            } else {
                const T u = f0[0], w = f0[1];
                dV[0] = lam * u * u * u + qc * u * w * w;
                dV[1] = qc * u * u * w;
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const T F = ka1 * lap[f] - ka3 * dV[f];
                const T pm = p0[f] + c1 * F;
                if (RED && valid) {
                    const double pmd = (double)pm;
                    acc[f] += pmd * pmd;
                    const double gx = (double)(xp[f] - f0[f]);
                    const double gy = (double)(yp[f] - f0[f]);
                    const double gz = (double)(fp[f] - f0[f]);
                    acc[NF + f] += gx * gx + gy * gy + gz * gz;
                }
                const T pn = pm + c2 * F;
                const T fo = DEND ? f0[f] + de * pn : f0[f];
                if (valid) {
                    if (WPHI) g.phi_out[f][oz] = fo;
                    if (WPI) g.pi_out[f][oz] = pn;
                }
            }
            if (RED && valid) {
                const double u = (double)f0[0];
                acc[2 * NF] += 0.25 * lamd * u * u * u * u;
                if constexpr (NF == 2) {
                    const double w = (double)f0[1];
                    acc[2 * NF + 1] += 0.5 * qd * u * u * w * w;
                }
            }
        }
        __syncthreads();
        // (E) rotate the computed window; the in-set raw plane z+2 becomes phi(z+2)
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            fm[f] = f0[f];
            f0[f] = fp[f];
            p0[f] = pp[f];
            fp[f] = DLOAD ? oci_f[f] + dl * oci_p[f] : oci_f[f];
            pp[f] = oci_p[f];
        }
    };

    for (int z = z0; z < z1; z += 2) {
        plane(z, ownA_f, ownA_p, haloA_f, haloA_p, ownB_f, ownB_p, haloB_f, haloB_p);
        if (z + 1 < z1) plane(z + 1, ownB_f, ownB_p, haloB_f, haloB_p, ownA_f, ownA_p, haloA_f, haloA_p);
    }

    if constexpr (RED) {
        double tot[NQ];
        block_sums<NT, NQ>(acc, lds_red, tot);
        if (g.defer) {
            if (tid == 0) {
#pragma unroll
                for (int k = 0; k < NQ; ++k) g.partials[(size_t)lid * NQ + k] = tot[k];
            }
            return;
        }
        if (tid == 0) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) store_agent(&g.partials[(size_t)lid * NQ + k], tot[k]);
            last_flag = ticket_arrive(g.ticket, gridDim.x) ? 1 : 0;
        }
        __syncthreads();
        if (last_flag) {
            const int nb = gridDim.x;
            double part[NQ];
#pragma unroll
            for (int k = 0; k < NQ; ++k) part[k] = 0.0;
            for (int i = tid; i < nb; i += NT) {
#pragma unroll
                for (int k = 0; k < NQ; ++k) part[k] += load_agent(&g.partials[(size_t)i * NQ + k]);
            }
            double fin[NQ];
            block_sums<NT, NQ>(part, lds_red, fin);
            if (tid == 0) {
#pragma unroll
                for (int k = 0; k < NQ; ++k) g.sc->sums[k] = fin[k];
                if (g.last_mode == kLastSelf)
                    self_update<NF>(C, fin, g.sc, g.coef_next, g.alpha, g.kappa2, g.inv_vol, g.inv_dx2);
                else if (g.last_mode == kLastSelfLF)
                    self_update_lf<NF>(C, fin, g.sc, g.coef_next, g.alpha, g.kappa2, g.inv_vol, g.inv_dx2);
                __hip_atomic_store(g.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// Kick coefficients of the first pass of a self-consistent call from the
// current scale factor (no drift precedes it).
__global__ void self_prologue(PassCoef *c0, const ScaleRecord *S, double alpha)
{
    if (threadIdx.x == 0) {
        const double a = S->a;
        c0->ka1 = pow(a, 1.0 + alpha);
        c0->ka3 = pow(a, 3.0 + alpha);
        c0->dload = 0.0;
    }
}

}  // namespace lat
