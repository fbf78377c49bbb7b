// stage_batch.hpp -- one leapfrog pass (kick, then drift at end) over a batch of
// independent single-field lattices of different sizes in a single launch.
//
// Physics per site as in stage_scalar.hpp (sec. 4.5.2 at one kick point,
// V = lambda/4 phi^4).  Each block looks up its realization and tile in a work
// table.  Per realization, chosen by the autotuner for its lattice size, a
// block either marches a z chunk of a TX x TY tile (TX x TY = 256 threads,
// TX in {8, 16, 32, 64}; drifted-phi planes in LDS, z window in registers) or,
// with TX = 0, updates 256 consecutive sites with one thread each and reads
// the six neighbours through the caches (no LDS, no barrier: for small
// lattices, where a z march is a long serial chain over few blocks).
// The kick and drift coefficients are shared: every realization sits at the
// same time on the same background.  phi is read with a halo and written to the
// other buffer of its pair (buffer parity is a launch argument, so a captured
// graph of K passes needs no table updates); pi is updated in place or, while
// tuning, written to a scratch buffer.
#pragma once
#include "common.hpp"

namespace lat {

template <typename T>
struct BatchReal {
    T *phi[2];          // [0] caller buffer, [1] shadow
    T *pi;              // caller buffer
    T *pi_scratch;      // tuning target (state untouched)
    int N, tx, ty, zc;
    int tiles_x, tiles_y, pad0, pad1;
};

template <typename T>
struct BatchArgs {
    const BatchReal<T> *reals;
    const int2 *block_work;  // per launched block: (realization, block within it); -1: none
    const PassCoef *coef;
    int parity;              // phi read from buffer parity, written to parity ^ 1
    int tuning;              // 1: write pi to pi_scratch
    double inv_dx2, lam;
};

constexpr int kBatchThreads = 256;
constexpr int kBatchLds = 400;   // >= max (TX+2)(TY+2) over the tile shapes

template <typename T>
__global__ void __launch_bounds__(kBatchThreads) batch_lf_stage(const BatchArgs<T> g)
{
    __shared__ T lds[2][kBatchLds];
    // the host lays the table out in dispatch order: block b runs on XCD b % 8,
    // each realization sits on one XCD (its halos in one L2), the XCDs carry
    // balanced site counts, and each XCD starts with its longest blocks
    const int2 wk = g.block_work[blockIdx.x];
    if (wk.x < 0) return;
    const BatchReal<T> R = g.reals[wk.x];
    const int lid = wk.y;
    if (R.tx == 0) {
        // one site per thread; the same arithmetic, in the same order, as the tiled path
        const unsigned N = (unsigned)R.N, NN = N * N, V = NN * N;
        const unsigned i = (unsigned)lid * kBatchThreads + threadIdx.x;
        if (i >= V) return;
        const unsigned z = i / NN, rem = i - z * NN, y = rem / N, x = rem - y * N;
        const unsigned ixm = x == 0 ? i + N - 1 : i - 1, ixp = x == N - 1 ? i + 1 - N : i + 1;
        const unsigned iym = y == 0 ? i + NN - N : i - N, iyp = y == N - 1 ? i + N - NN : i + N;
        const unsigned izm = z == 0 ? i + V - NN : i - NN, izp = z == N - 1 ? i + NN - V : i + NN;
        const T *P = (g.parity ? R.phi[1] : R.phi[0]);
        const PassCoef C = *g.coef;
        const T c1 = (T)C.c1, c2 = (T)C.c2, de = (T)C.dend, ka1 = (T)C.ka1, ka3 = (T)C.ka3;
        const T idx2 = (T)g.inv_dx2, lam = (T)g.lam;
        const T f0 = ld32(P, i);
        const T lap = ((ld32(P, ixp) - T(2) * f0 + ld32(P, ixm)) + (ld32(P, iyp) - T(2) * f0 + ld32(P, iym)) +
                       (ld32(P, izp) - T(2) * f0 + ld32(P, izm))) * idx2;
        const T F = ka1 * lap - ka3 * (lam * f0 * f0 * f0);
        const T pn = (ld32((const T *)R.pi, i) + c1 * F) + c2 * F;
        st32((g.parity ? R.phi[0] : R.phi[1]), i, f0 + de * pn);
        st32(g.tuning ? R.pi_scratch : R.pi, i, pn);
        return;
    }
    const int TX = R.tx, TY = R.ty, LX = TX + 2;
    const int N = R.N;
    const int bx = lid % R.tiles_x;
    const int rest = lid / R.tiles_x;
    const int by = rest % R.tiles_y;
    const int bz = rest / R.tiles_y;
    const int x0 = bx * TX, y0 = by * TY;
    const int z0 = bz * R.zc;
    const int z1 = min(z0 + R.zc, N);
    const size_t NN = (size_t)N * (size_t)N;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const bool valid = (x0 + tx < N) && (y0 + ty < N);
    const int own = ((x0 + tx) % N) + N * ((y0 + ty) % N);
    const int oslot = (1 + ty) * LX + 1 + tx;
    const int NH = 2 * TX + 2 * TY;
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
    // buffers chosen by selects, not by indexing R.phi with a runtime value:
    // that would make R a per-thread array (moved to LDS or scratch)
    const T *P = (g.parity ? R.phi[1] : R.phi[0]);
    T *Pout = (g.parity ? R.phi[0] : R.phi[1]);
    const T *Q = R.pi;
    T *Qout = g.tuning ? R.pi_scratch : R.pi;
    const PassCoef C = *g.coef;
    const T c1 = (T)C.c1, c2 = (T)C.c2, de = (T)C.dend, ka1 = (T)C.ka1, ka3 = (T)C.ka3;
    const T idx2 = (T)g.inv_dx2, lam = (T)g.lam;

    T fm, f0, fp, p0, pp;
    T oA, oAp, hA, oB, oBp, hB;
    {
        const size_t om = (size_t)(z0 == 0 ? N - 1 : z0 - 1) * NN;
        const size_t o0 = (size_t)z0 * NN;
        const size_t o1 = (size_t)((z0 + 1) % N) * NN;
        const size_t o2 = (size_t)(min(z0 + 2, z1) % N) * NN;
        const size_t oh1 = (size_t)(min(z0 + 1, z1 - 1) % N) * NN;
        fm = P[om + own];
        f0 = P[o0 + own];
        p0 = Q[o0 + own];
        fp = P[o1 + own];
        pp = Q[o1 + own];
        oA = P[o2 + own];
        oAp = Q[o2 + own];
        hA = T(0);
        lds[0][oslot] = f0;
        if (has_halo) {
            lds[0][hslot] = P[o0 + hoff];
            hA = P[oh1 + hoff];
        }
    }
    oB = oBp = hB = T(0);
    __syncthreads();

    auto plane = [&](const int z, T &oi, T &oip, T &hi, T &oo, T &oop, T &ho) {
        const int cur = (z - z0) & 1, nxt = cur ^ 1;
        int zo = min(z + 3, z1);
        if (zo >= N) zo -= N;
        int zh = min(z + 2, z1 - 1);
        if (zh >= N) zh -= N;
        oo = P[(size_t)zo * NN + own];
        oop = Q[(size_t)zo * NN + own];
        if (has_halo) ho = P[(size_t)zh * NN + hoff];
        if (z + 1 < z1) {
            lds[nxt][oslot] = fp;
            if (has_halo) lds[nxt][hslot] = hi;
        }
        const T *L = lds[cur];
        const T lap = ((L[oslot + 1] - T(2) * f0 + L[oslot - 1]) + (L[oslot + LX] - T(2) * f0 + L[oslot - LX]) +
                       (fp - T(2) * f0 + fm)) * idx2;
        const T F = ka1 * lap - ka3 * (lam * f0 * f0 * f0);
        const T pn = (p0 + c1 * F) + c2 * F;
        if (valid) {
            const size_t oz = (size_t)z * NN + own;
            Pout[oz] = f0 + de * pn;
            Qout[oz] = pn;
        }
        __syncthreads();
        fm = f0;
        f0 = fp;
        p0 = pp;
        fp = oi;
        pp = oip;
    };
    for (int z = z0; z < z1; z += 2) {
        plane(z, oA, oAp, hA, oB, oBp, hB);
        if (z + 1 < z1) plane(z + 1, oB, oBp, hB, oA, oAp, hA);
    }
}

// copy the shadow phi of every realization back to the caller's buffer
template <typename T>
__global__ void batch_settle(const BatchReal<T> *reals, int n_real, int which)
{
    const int r = blockIdx.y;
    if (r >= n_real) return;
    const BatchReal<T> R = reals[r];
    const size_t V = (size_t)R.N * R.N * R.N;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += (size_t)gridDim.x * blockDim.x)
        (which ? R.phi[0] : R.phi[1])[i] = (which ? R.phi[1] : R.phi[0])[i];
}

}  // namespace lat
