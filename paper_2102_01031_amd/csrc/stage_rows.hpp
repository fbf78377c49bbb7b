// stage_rows.hpp -- the stencil pass of stage_scalar.hpp for N = 64 * XS with
// XS in {1, 2, 4}: a block owns whole x rows, so there is no x halo.
//
// Block = TY wavefronts; wavefront w owns row y0 + w and its lanes hold XS
// sites each, VW consecutive ones per access: x = VW lane + v + 64 VW j
// (v < VW, j < XS / VW), so every global load or store of a row is one
// contiguous 64 VW sizeof(T)-byte segment per j (VW = 16 / sizeof(T) gives
// 16-byte accesses).  The drifted phi of the current plane for rows
// y0-1 .. y0+TY sits in LDS (the two halo rows are loaded one VW-site vector
// per thread); z neighbours come from a register window as in the tiled kernel.
// Block order: the blocks of one XCD form either a y slab through every z
// chunk or a slab of whole planes (y tile fastest), so halo rows between
// tiles are shared inside one L2 except at the slab's faces.
// PF is the prefetch depth in planes: the loads issued while the plane of
// march step s is computed are for own plane s + 2 + PF and halo plane
// s + 1 + PF of the march, landing in one of PF + 1 register sets that rotate
// with the (PF + 1)-fold unrolled z loop, so no register copies force an early
// wait on loads in flight.
// A block marches its z chunk up or down (ScalarArgs::down): passes that
// alternate direction start on the planes the previous pass wrote last.  With
// ordinary stores (ScalarArgs::cached_out) instead of non-temporal ones those
// planes are still held in the memory-side cache when the next pass reads them.
#pragma once
#include <type_traits>

#include "common.hpp"
#include "stage_scalar.hpp"

namespace lat {

// A lane's VW consecutive sites of a row as one vector (VW = 1: the scalar).
template <typename T, int V>
struct RowVec {
    typedef T type __attribute__((ext_vector_type(V)));
};
template <typename T>
struct RowVec<T, 1> {
    typedef T type;
};

template <typename T, typename VT>
__device__ __forceinline__ T vget(const VT &x, int v)
{
    if constexpr (sizeof(VT) == sizeof(T)) return x;
    else return x[v];
}

template <typename T, typename VT>
__device__ __forceinline__ void vset(VT &x, int v, T val)
{
    if constexpr (sizeof(VT) == sizeof(T)) x = val;
    else x[v] = val;
}

// vector load / non-temporal store at element index i (32-bit byte offset, as ld32)
template <typename VT, typename T>
__device__ __forceinline__ VT ldv(const T *base, unsigned i)
{
    return *(const VT *)((const char *)base + (size_t)(i * (unsigned)sizeof(T)));
}

template <typename VT, typename T>
__device__ __forceinline__ void stv_nt(T *base, unsigned i, VT v)
{
    __builtin_nontemporal_store(v, (VT *)((char *)base + (size_t)(i * (unsigned)sizeof(T))));
}

// VW: sites per lane and access (1, or 16 / sizeof(T) for 16-byte loads and
// stores); lane l holds x = VW l + v + 64 VW j (v < VW, j < XS / VW), so the x
// neighbours inside a lane's group come from registers and only the two at
// the group's ends from the LDS row.
// Store policy in phase PH of the march (0: its first split / 8, 1: the rest)
// under policy LP:
//   0  stores by ScalarArgs::cached_out in both phases
//   1  non-temporal stores in phase 0, ordinary stores in phase 1: the planes
//      a pass writes last stay in the caches for the next pass, which marches
//      the other way and starts on them, while the rest streams past
// (st: 0 by cached_out, 1 non-temporal, 2 ordinary).  Loads are always
// ordinary: non-temporal loads measured slower, since each halo row is read
// again by the neighbouring block and loses its L2 hit.
template <int LP, int PH>
struct RowPolicy {
    static constexpr int st = LP == 0 ? 0 : (PH == 0 ? 1 : 2);
};

template <typename T, int NF, int XS, int TY, bool DLOAD, bool DEND, bool RED, bool WPHI, bool WPI, int PF = 1,
          int VW = 1, int LP = 0>
__global__ void __launch_bounds__(64 * TY) scalar_rows(const ScalarArgs<T> g)
{
    static_assert(PF >= 1 && PF <= 4, "prefetch depth 1 .. 4");
    static_assert(XS % VW == 0 && VW * sizeof(T) <= 16, "vector width");
    using VT = typename RowVec<T, VW>::type;
    constexpr int NT = 64 * TY;
    constexpr int NX = 64 * XS;           // == N
    constexpr int XV = XS / VW;           // vectors per lane and row
    constexpr int NQ = 3 * NF;
    constexpr int NHV = 2 * NX / VW;      // halo vectors per plane (rows y0-1 and y0+TY)
    constexpr int HPT = (NHV + NT - 1) / NT;

    __shared__ __attribute__((aligned(16))) T lds[2][NF][(TY + 2) * NX];
    __shared__ double lds_red[(NT / 64) * NQ];
    __shared__ int last_flag;

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int N = NX;
    // logical block: z chunk fastest, then y tile (each XCD's range of logical
    // blocks is a y slab through all z), or y tile fastest (an XCD's range is
    // a z slab of whole planes, or part of one)
    const int lid = xcd_logical_block(blockIdx.x, gridDim.x);
    const int chunks = (N + g.zc - 1) / g.zc;
    constexpr int tiles = (NX + TY - 1) / TY;
    const int bz = g.y_fastest ? lid / tiles : lid % chunks;
    const int by = g.y_fastest ? lid % tiles : lid / chunks;
    const int y0 = by * TY;
    const int z0 = bz * g.zc;
    const int z1 = min(z0 + g.zc, N);
    const int len = z1 - z0;
    // march direction: up (z0, z0 + 1, ...) or down (z1 - 1, z1 - 2, ...);
    // pl(k) is the k-th plane of the march, k = -1 .. len, wrapped periodically
    // with zpair, neighbouring chunks march in opposite directions, so the
    // plane on either side of a chunk boundary is read by both chunks at the
    // same time (both at their start, or both at their end)
    const bool down = (g.down != 0) != (g.zpair != 0 && (bz & 1) != 0);
    auto pl = [&](const int k) {
        int z = down ? z1 - 1 - k : z0 + k;
        if (z < 0) z += N;
        if (z >= N) z -= N;
        return z;
    };
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
        hval[j] = c < NHV;
        const int r = c < NX / VW ? 0 : 1;
        const int x = (c - r * (NX / VW)) * VW;
        int hy = r == 0 ? y0 - 1 : y0 + TY;
        hy = ((hy % N) + N) % N;
        hslot[j] = (r == 0 ? 0 : (TY + 1) * NX) + x;
        hoff[j] = hval[j] ? x + N * hy : 0;
    }

    const VT vzero = (VT)T(0);
    T fm[XS][NF], f0[XS][NF], fp[XS][NF], p0[XS][NF], pp[XS][NF];
    // register set s (s < PF + 1) of own-row phi, pi and halo-row phi, pi loads
    VT of[PF + 1][XV][NF], op[PF + 1][XV][NF], hf[PF + 1][HPT][NF], hp[PF + 1][HPT][NF];

    // first planes of the march: planes -1, 0, 1 of the own rows and plane 0
    // of the halo rows as loaded (the drift on load is applied below, once the
    // coefficients are known), set 0 .. PF-1 of the prefetch window.  Issued
    // before the prologue so that their latency overlaps it.
    VT ra[XV][NF], rpa[XV][NF], rb[XV][NF], rpb[XV][NF], rc[XV][NF], rpc[XV][NF];
    VT rh[HPT][NF], rph[HPT][NF];
    {
        const unsigned om = (unsigned)pl(-1) * NN;
        const unsigned o0 = (unsigned)pl(0) * NN;
        const unsigned o1 = (unsigned)pl(1) * NN;
        const unsigned o2 = (unsigned)pl(min(2, len)) * NN;
        const unsigned oh1 = (unsigned)pl(min(1, len - 1)) * NN;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const T *P = g.phi_in[f];
            const T *Q = g.pi_in[f];
#pragma unroll
            for (int j = 0; j < XV; ++j) {
                const int o = yo + VW * lane + 64 * VW * j;
                ra[j][f] = ldv<VT>(P, om + o);
                rpa[j][f] = DLOAD ? ldv<VT>(Q, om + o) : vzero;
                rb[j][f] = ldv<VT>(P, o0 + o);
                rpb[j][f] = ldv<VT>(Q, o0 + o);
                rc[j][f] = ldv<VT>(P, o1 + o);
                rpc[j][f] = ldv<VT>(Q, o1 + o);
                of[0][j][f] = ldv<VT>(P, o2 + o);
                op[0][j][f] = ldv<VT>(Q, o2 + o);
            }
#pragma unroll
            for (int j = 0; j < HPT; ++j) {
                rh[j][f] = rph[j][f] = hf[0][j][f] = hp[0][j][f] = vzero;
                if (hval[j]) {
                    rh[j][f] = ldv<VT>(P, o0 + hoff[j]);
                    if (DLOAD) rph[j][f] = ldv<VT>(Q, o0 + hoff[j]);
                    hf[0][j][f] = ldv<VT>(P, oh1 + hoff[j]);
                    if (DLOAD) hp[0][j][f] = ldv<VT>(Q, oh1 + hoff[j]);
                }
            }
            // sets 1 .. PF-1: own plane 2 + s of the march, halo plane 1 + s
#pragma unroll
            for (int st = 1; st < PF; ++st) {
                const unsigned os = (unsigned)pl(min(2 + st, len)) * NN;
                const unsigned ohs = (unsigned)pl(min(1 + st, len - 1)) * NN;
#pragma unroll
                for (int j = 0; j < XV; ++j) {
                    const int o = yo + VW * lane + 64 * VW * j;
                    of[st][j][f] = ldv<VT>(P, os + o);
                    op[st][j][f] = ldv<VT>(Q, os + o);
                }
#pragma unroll
                for (int j = 0; j < HPT; ++j) {
                    hf[st][j][f] = hp[st][j][f] = vzero;
                    if (hval[j]) {
                        hf[st][j][f] = ldv<VT>(P, ohs + hoff[j]);
                        if (DLOAD) hp[st][j][f] = ldv<VT>(Q, ohs + hoff[j]);
                    }
                }
            }
        }
    }

    PassCoef C = *g.coef;
    if (g.fin) {
        __shared__ double lds_coef[4];
        finalise_prologue<NT, NF>(g, lds_red, lds_coef, C);
    }
    const T dl = (T)C.dload, c1 = (T)C.c1, c2 = (T)C.c2, de = (T)C.dend;
    const T ka1 = (T)C.ka1, ka3 = (T)C.ka3, idx2 = (T)g.inv_dx2;
    const T lam = (T)g.lam, qc = (T)g.q;
    const T qv4 = (T)(0.25 * g.lam), qv2 = (T)(0.5 * g.q);   // V = lam/4 u^4 + q/2 u^2 v^2

    // the drift on load of the first planes; plane 0 into the LDS row
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int j = 0; j < XV; ++j) {
            const int x0 = VW * lane + 64 * VW * j;
            VT a = ra[j][f];
            if (DLOAD) a += dl * rpa[j][f];
            VT b = rb[j][f];
            const VT pb = rpb[j][f];
            if (DLOAD) b += dl * pb;
            VT c = rc[j][f];
            const VT pc = rpc[j][f];
            if (DLOAD) c += dl * pc;
            *(VT *)&lds[0][f][orow + x0] = b;
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int k = j * VW + v;
                fm[k][f] = vget<T>(a, v);
                f0[k][f] = vget<T>(b, v);
                p0[k][f] = vget<T>(pb, v);
                fp[k][f] = vget<T>(c, v);
                pp[k][f] = vget<T>(pc, v);
            }
        }
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            if (hval[j]) {
                VT h = rh[j][f];
                if (DLOAD) h += dl * rph[j][f];
                *(VT *)&lds[0][f][hslot[j]] = h;
            }
        }
    }
    __syncthreads();

    double acc[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) acc[k] = 0.0;

    // step sm of the march: plane pl(sm); fm holds the plane behind it in the
    // march, fp the plane ahead
    auto plane = [&](auto phase, const int sm, VT (&oif)[XV][NF], VT (&oip)[XV][NF], VT (&hif)[HPT][NF],
                     VT (&hip)[HPT][NF], VT (&oof)[XV][NF], VT (&oop)[XV][NF], VT (&hof)[HPT][NF],
                     VT (&hop)[HPT][NF]) {
        using Pol = RowPolicy<LP, decltype(phase)::value>;
        const bool nt_out = Pol::st == 0 ? g.cached_out == 0 : Pol::st == 1;
        const int cur = sm & 1, nxt = cur ^ 1;
        const unsigned o3 = (unsigned)pl(min(sm + 2 + PF, len)) * NN;
        const unsigned o2 = (unsigned)pl(min(sm + 1 + PF, len - 1)) * NN;
        // (A) loads PF planes ahead
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int j = 0; j < XV; ++j) {
                const int o = yo + VW * lane + 64 * VW * j;
                oof[j][f] = ldv<VT>(g.phi_in[f], o3 + o);
                oop[j][f] = ldv<VT>(g.pi_in[f], o3 + o);
            }
#pragma unroll
            for (int j = 0; j < HPT; ++j) {
                if (hval[j]) {
                    hof[j][f] = ldv<VT>(g.phi_in[f], o2 + hoff[j]);
                    if (DLOAD) hop[j][f] = ldv<VT>(g.pi_in[f], o2 + hoff[j]);
                }
            }
        }
        // (B) LDS: the plane ahead
        if (sm + 1 < len) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
#pragma unroll
                for (int j = 0; j < XV; ++j) {
                    VT u;
#pragma unroll
                    for (int v = 0; v < VW; ++v) vset<T>(u, v, fp[j * VW + v][f]);
                    *(VT *)&lds[nxt][f][orow + VW * lane + 64 * VW * j] = u;
                }
#pragma unroll
                for (int j = 0; j < HPT; ++j)
                    if (hval[j]) *(VT *)&lds[nxt][f][hslot[j]] = DLOAD ? hif[j][f] + dl * hip[j][f] : hif[j][f];
            }
        }
        // (C) the XS sites of this lane at plane pl(sm)
        const unsigned oz = (unsigned)pl(sm) * NN + yo;
#pragma unroll
        for (int j = 0; j < XV; ++j) {
            const int x0 = VW * lane + 64 * VW * j;
            const int xl = x0 == 0 ? NX - 1 : x0 - 1;
            const int xr = x0 + VW == NX ? 0 : x0 + VW;
            VT ymv[NF], ypv[NF], fov[NF], pnv[NF];
            T xlv[NF], xrv[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const T *L = lds[cur][f];
                ymv[f] = *(const VT *)&L[orow - NX + x0];
                ypv[f] = *(const VT *)&L[orow + NX + x0];
                xlv[f] = L[orow + xl];
                xrv[f] = L[orow + xr];
            }
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int k = j * VW + v;
                const int km = v == 0 ? k : k - 1, kp = v == VW - 1 ? k : k + 1;
                T xp[NF], yp[NF], zpv[NF], lap[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const T c0 = f0[k][f];
                    const T xm = v == 0 ? xlv[f] : f0[km][f];
                    xp[f] = v == VW - 1 ? xrv[f] : f0[kp][f];
                    const T ym = vget<T>(ymv[f], v);
                    yp[f] = vget<T>(ypv[f], v);
                    // z + 1 and z - 1 in lattice orientation, so both march
                    // directions evaluate the same expression
                    zpv[f] = down ? fm[k][f] : fp[k][f];
                    const T zm = down ? fp[k][f] : fm[k][f];
                    lap[f] = ((xp[f] - T(2) * c0 + xm) + (yp[f] - T(2) * c0 + ym) +
                              (zpv[f] - T(2) * c0 + zm)) * idx2;
                }
                T dV[NF];
                if constexpr (NF == 1) {
                    const T u = f0[k][0];
                    dV[0] = lam * u * u * u;
                } else {
                    const T u = f0[k][0], v2 = f0[k][1];
                    dV[0] = lam * u * u * u + qc * u * v2 * v2;
                    dV[1] = qc * u * u * v2;
                }
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const T F = ka1 * lap[f] - ka3 * dV[f];
                    const T pm = p0[k][f] + c1 * F;
                    if (RED && valid) {
                        // site terms in the field precision, volume sums in float64
                        const T gx = xp[f] - f0[k][f], gy = yp[f] - f0[k][f], gz = zpv[f] - f0[k][f];
                        acc[f] += (double)(pm * pm);
                        acc[NF + f] += (double)(gx * gx + gy * gy + gz * gz);
                    }
                    const T pn = pm + c2 * F;
                    vset<T>(fov[f], v, DEND ? f0[k][f] + de * pn : f0[k][f]);
                    vset<T>(pnv[f], v, pn);
                }
                if (RED && valid) {
                    const T u2 = f0[k][0] * f0[k][0];
                    acc[2 * NF] += (double)(qv4 * u2 * u2);
                    if constexpr (NF == 2) acc[2 * NF + 1] += (double)(qv2 * u2 * (f0[k][1] * f0[k][1]));
                }
            }
            if (valid) {
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    if (!nt_out) {
                        if (WPHI) *(VT *)((char *)g.phi_out[f] + (size_t)((oz + x0) * (unsigned)sizeof(T))) = fov[f];
                        if (WPI) *(VT *)((char *)g.pi_out[f] + (size_t)((oz + x0) * (unsigned)sizeof(T))) = pnv[f];
                    } else {
                        if (WPHI) stv_nt<VT>(g.phi_out[f], oz + x0, fov[f]);
                        if (WPI) stv_nt<VT>(g.pi_out[f], oz + x0, pnv[f]);
                    }
                }
            }
        }
        __syncthreads();
        // (E) rotate the computed window
#pragma unroll
        for (int j = 0; j < XV; ++j) {
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int k = j * VW + v;
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    fm[k][f] = f0[k][f];
                    f0[k][f] = fp[k][f];
                    p0[k][f] = pp[k][f];
                    const T a = vget<T>(oif[j][f], v);
                    fp[k][f] = DLOAD ? a + dl * vget<T>(oip[j][f], v) : a;
                    pp[k][f] = vget<T>(oip[j][f], v);
                }
            }
        }
    };

    // at unrolled step u set u holds own plane s + 2 and halo plane s + 1 (read
    // by the rotation), and set (u + PF) mod (PF + 1) receives the loads PF
    // planes ahead
    // the two phases of the march (the second starts at a multiple of PF + 1,
    // so the register sets rotate across the boundary as within a phase)
    const int mid = LP == 1 ? ((len * g.split / 8) / (PF + 1)) * (PF + 1) : 0;
    for (int sm = 0; sm < mid; sm += PF + 1) {
#pragma unroll
        for (int u = 0; u <= PF; ++u) {
            if (sm + u < len) {
                const int d = (u + PF) % (PF + 1);
                plane(std::integral_constant<int, 0>{}, sm + u, of[u], op[u], hf[u], hp[u], of[d], op[d], hf[d],
                      hp[d]);
            }
        }
    }
    for (int sm = mid; sm < len; sm += PF + 1) {
#pragma unroll
        for (int u = 0; u <= PF; ++u) {
            if (sm + u < len) {
                const int d = (u + PF) % (PF + 1);
                plane(std::integral_constant<int, LP == 1 ? 1 : 0>{}, sm + u, of[u], op[u], hf[u], hp[u], of[d],
                      op[d], hf[d], hp[d]);
            }
        }
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

}  // namespace lat
