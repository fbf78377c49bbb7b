// stage_rows.hpp -- the stencil pass of stage_scalar.hpp for N = 64 * XS with
// XS in {1, 2, 4}: a block owns whole x rows, so there is no x halo.
//
// Block = TY wavefronts; wavefront w owns row y0 + w and its lanes hold the XS
// sites x = lane + 64 k (k < XS), so every global load or store of a row is one
// contiguous 512-byte segment per k.  The drifted phi of the current plane for
// rows y0-1 .. y0+TY sits in LDS (the two halo rows are loaded one cell per
// thread); z neighbours come from a register window as in the tiled kernel.
// Block order: y tiles of one XCD are contiguous and each XCD walks every z
// chunk of its y slab, so halo rows between tiles and z-chunk boundaries are
// shared inside one L2.
// PF is the prefetch depth in planes: the loads issued while plane z is
// computed are for own plane z + 2 + PF and halo plane z + 1 + PF, landing in
// one of PF + 1 register sets that rotate with the (PF + 1)-fold unrolled z
// loop, so no register copies force an early wait on loads in flight.
#pragma once
#include "common.hpp"
#include "stage_scalar.hpp"

namespace lat {

template <typename T, int NF, int XS, int TY, bool DLOAD, bool DEND, bool RED, bool WPHI, bool WPI, int PF = 1>
__global__ void __launch_bounds__(64 * TY) scalar_rows(const ScalarArgs<T> g)
{
    static_assert(PF == 1 || PF == 2, "prefetch depth 1 or 2");
    constexpr int NT = 64 * TY;
    constexpr int NX = 64 * XS;           // == N
    constexpr int NQ = 3 * NF;
    constexpr int NH = 2 * NX;            // halo cells per plane (rows y0-1 and y0+TY)
    constexpr int HPT = (NH + NT - 1) / NT;

    __shared__ T lds[2][NF][(TY + 2) * NX];
    __shared__ double lds_red[(NT / 64) * NQ];
    __shared__ int last_flag;

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int N = NX;
    // logical block: z chunk fastest, then y tile
    const int lid = xcd_logical_block(blockIdx.x, gridDim.x);
    const int chunks = (N + g.zc - 1) / g.zc;
    const int bz = lid % chunks;
    const int by = lid / chunks;
    const int y0 = by * TY;
    const int z0 = bz * g.zc;
    const int z1 = min(z0 + g.zc, N);
    const unsigned NN = (unsigned)N * (unsigned)N;   // N^3 < 2^32

    const int yrow = y0 + w;
    const bool valid = yrow < N;
    const int yo = (yrow % N) * N;
    const int orow = (1 + w) * NX;

    int hslot[HPT], hoff[HPT];
    bool hval[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
        const int c = tid + j * NT;
        hval[j] = c < NH;
        const int r = c < NX ? 0 : 1;
        const int x = c - r * NX;
        int hy = r == 0 ? y0 - 1 : y0 + TY;
        hy = ((hy % N) + N) % N;
        hslot[j] = (r == 0 ? 0 : (TY + 1) * NX) + x;
        hoff[j] = hval[j] ? x + N * hy : 0;
    }

    const PassCoef C = *g.coef;
    const T dl = (T)C.dload, c1 = (T)C.c1, c2 = (T)C.c2, de = (T)C.dend;
    const T ka1 = (T)C.ka1, ka3 = (T)C.ka3, idx2 = (T)g.inv_dx2;
    const T lam = (T)g.lam, qc = (T)g.q;
    const double lamd = g.lam, qd = g.q;

    T fm[XS][NF], f0[XS][NF], fp[XS][NF], p0[XS][NF], pp[XS][NF];
    T oAf[XS][NF], oAp[XS][NF], oBf[XS][NF], oBp[XS][NF], oCf[XS][NF], oCp[XS][NF];
    T hAf[HPT][NF], hAp[HPT][NF], hBf[HPT][NF], hBp[HPT][NF], hCf[HPT][NF], hCp[HPT][NF];

    {
        const unsigned om = (unsigned)(z0 == 0 ? N - 1 : z0 - 1) * NN;
        const unsigned o0 = (unsigned)z0 * NN;
        const unsigned o1 = (unsigned)((z0 + 1) % N) * NN;
        const unsigned o2 = (unsigned)(min(z0 + 2, z1) % N) * NN;
        const unsigned oh1 = (unsigned)(min(z0 + 1, z1 - 1) % N) * NN;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const T *P = g.phi_in[f];
            const T *Q = g.pi_in[f];
#pragma unroll
            for (int k = 0; k < XS; ++k) {
                const int o = yo + lane + 64 * k;
                const T a = ld32(P, om + o);
                fm[k][f] = DLOAD ? a + dl * ld32(Q, om + o) : a;
                const T b = ld32(P, o0 + o);
                p0[k][f] = ld32(Q, o0 + o);
                f0[k][f] = DLOAD ? b + dl * p0[k][f] : b;
                const T c = ld32(P, o1 + o);
                pp[k][f] = ld32(Q, o1 + o);
                fp[k][f] = DLOAD ? c + dl * pp[k][f] : c;
                oAf[k][f] = ld32(P, o2 + o);
                oAp[k][f] = ld32(Q, o2 + o);
                lds[0][f][orow + lane + 64 * k] = f0[k][f];
            }
#pragma unroll
            for (int j = 0; j < HPT; ++j) {
                hAf[j][f] = hAp[j][f] = T(0);
                if (hval[j]) {
                    T h = ld32(P, o0 + hoff[j]);
                    if (DLOAD) h += dl * ld32(Q, o0 + hoff[j]);
                    lds[0][f][hslot[j]] = h;
                    hAf[j][f] = ld32(P, oh1 + hoff[j]);
                    if (DLOAD) hAp[j][f] = ld32(Q, oh1 + hoff[j]);
                }
            }
            if constexpr (PF == 2) {
                const unsigned o3 = (unsigned)(min(z0 + 3, z1) % N) * NN;
                const unsigned oh2 = (unsigned)(min(z0 + 2, z1 - 1) % N) * NN;
#pragma unroll
                for (int k = 0; k < XS; ++k) {
                    const int o = yo + lane + 64 * k;
                    oBf[k][f] = ld32(P, o3 + o);
                    oBp[k][f] = ld32(Q, o3 + o);
                }
#pragma unroll
                for (int j = 0; j < HPT; ++j) {
                    hBf[j][f] = hBp[j][f] = T(0);
                    if (hval[j]) {
                        hBf[j][f] = ld32(P, oh2 + hoff[j]);
                        if (DLOAD) hBp[j][f] = ld32(Q, oh2 + hoff[j]);
                    }
                }
            }
        }
    }
    __syncthreads();

    double acc[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) acc[k] = 0.0;

    auto plane = [&](const int z, T (&oif)[XS][NF], T (&oip)[XS][NF], T (&hif)[HPT][NF], T (&hip)[HPT][NF],
                     T (&oof)[XS][NF], T (&oop)[XS][NF], T (&hof)[HPT][NF], T (&hop)[HPT][NF]) {
        const int cur = (z - z0) & 1, nxt = cur ^ 1;
        int zo = min(z + 2 + PF, z1);
        if (zo >= N) zo -= N;
        int zh = min(z + 1 + PF, z1 - 1);
        if (zh >= N) zh -= N;
        const unsigned o3 = (unsigned)zo * NN, o2 = (unsigned)zh * NN;
        // (A) loads one plane ahead
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int k = 0; k < XS; ++k) {
                const int o = yo + lane + 64 * k;
                oof[k][f] = ld32(g.phi_in[f], o3 + o);
                oop[k][f] = ld32(g.pi_in[f], o3 + o);
            }
#pragma unroll
            for (int j = 0; j < HPT; ++j) {
                if (hval[j]) {
                    hof[j][f] = ld32(g.phi_in[f], o2 + hoff[j]);
                    if (DLOAD) hop[j][f] = ld32(g.pi_in[f], o2 + hoff[j]);
                }
            }
        }
        // (B) LDS plane z+1
        if (z + 1 < z1) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
#pragma unroll
                for (int k = 0; k < XS; ++k) lds[nxt][f][orow + lane + 64 * k] = fp[k][f];
#pragma unroll
                for (int j = 0; j < HPT; ++j)
                    if (hval[j]) lds[nxt][f][hslot[j]] = DLOAD ? hif[j][f] + dl * hip[j][f] : hif[j][f];
            }
        }
        // (C) the XS sites of this lane at plane z
        const unsigned oz = (unsigned)z * NN + yo;
#pragma unroll
        for (int k = 0; k < XS; ++k) {
            const int x = lane + 64 * k;
            const int xl = x == 0 ? NX - 1 : x - 1;
            const int xr = x == NX - 1 ? 0 : x + 1;
            T xp[NF], yp[NF], lap[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const T *L = lds[cur][f];
                const T c0 = f0[k][f];
                const T xm = L[orow + xl];
                xp[f] = L[orow + xr];
                const T ym = L[orow - NX + x];
                yp[f] = L[orow + NX + x];
                lap[f] = ((xp[f] - T(2) * c0 + xm) + (yp[f] - T(2) * c0 + ym) +
                          (fp[k][f] - T(2) * c0 + fm[k][f])) * idx2;
            }
            T dV[NF];
            if constexpr (NF == 1) {
                const T u = f0[k][0];
                dV[0] = lam * u * u * u;
            } else {
                const T u = f0[k][0], v = f0[k][1];
                dV[0] = lam * u * u * u + qc * u * v * v;
                dV[1] = qc * u * u * v;
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const T F = ka1 * lap[f] - ka3 * dV[f];
                const T pm = p0[k][f] + c1 * F;
                if (RED && valid) {
                    const double pmd = (double)pm;
                    acc[f] += pmd * pmd;
                    const double gx = (double)(xp[f] - f0[k][f]);
                    const double gy = (double)(yp[f] - f0[k][f]);
                    const double gz = (double)(fp[k][f] - f0[k][f]);
                    acc[NF + f] += gx * gx + gy * gy + gz * gz;
                }
                const T pn = pm + c2 * F;
                const T fo = DEND ? f0[k][f] + de * pn : f0[k][f];
                if (valid) {
                    if (WPHI) st32_nt(g.phi_out[f], oz + x, fo);
                    if (WPI) st32_nt(g.pi_out[f], oz + x, pn);
                }
            }
            if (RED && valid) {
                const double u = (double)f0[k][0];
                acc[2 * NF] += 0.25 * lamd * u * u * u * u;
                if constexpr (NF == 2) {
                    const double v = (double)f0[k][1];
                    acc[2 * NF + 1] += 0.5 * qd * u * u * v * v;
                }
            }
        }
        __syncthreads();
        // (E) rotate the computed window
#pragma unroll
        for (int k = 0; k < XS; ++k) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                fm[k][f] = f0[k][f];
                f0[k][f] = fp[k][f];
                p0[k][f] = pp[k][f];
                fp[k][f] = DLOAD ? oif[k][f] + dl * oip[k][f] : oif[k][f];
                pp[k][f] = oip[k][f];
            }
        }
    };

    if constexpr (PF == 1) {
        for (int z = z0; z < z1; z += 2) {
            plane(z, oAf, oAp, hAf, hAp, oBf, oBp, hBf, hBp);
            if (z + 1 < z1) plane(z + 1, oBf, oBp, hBf, hBp, oAf, oAp, hAf, hAp);
        }
    } else {
        // set A holds own plane z + 2 and halo plane z + 1, B the next ones; C is loaded
        for (int z = z0; z < z1; z += 3) {
            plane(z, oAf, oAp, hAf, hAp, oCf, oCp, hCf, hCp);
            if (z + 1 < z1) plane(z + 1, oBf, oBp, hBf, hBp, oAf, oAp, hAf, hAp);
            if (z + 2 < z1) plane(z + 2, oCf, oCp, hCf, hCp, oBf, oBp, hBf, hBp);
        }
    }

    if constexpr (RED) {
        double tot[NQ];
        block_sums<NT, NQ>(acc, lds_red, tot);
        if (tid == 0) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) store_agent(&g.partials[(size_t)lid * NQ + k], tot[k]);
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
                for (int k = 0; k < NQ; ++k) part[k] += load_agent(&g.partials[(size_t)i * NQ + k]);
            }
            double fin[NQ];
            block_sums<NT, NQ>(part, lds_red, fin);
            if (tid == 0) {
#pragma unroll
                for (int k = 0; k < NQ; ++k) g.sc->sums[k] = fin[k];
                if (g.last_mode == kLastSelf)
                    self_update<NF>(C, fin, g.sc, g.coef_next, g.alpha, g.kappa2, g.inv_vol, g.inv_dx2);
                __hip_atomic_store(g.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

}  // namespace lat
