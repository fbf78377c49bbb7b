// common.hpp -- device-side records shared by the kernels and the runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lat {

// Coefficients of one stencil pass at a kick point p of the schedule.
//   drift on load   phi += dload * pi            (the drift that ends at p)
//   kernel          F = ka1 * Lap(phi) - ka3 * dV/dphi       ka1 = a^{1+alpha}, ka3 = a^{3+alpha}
//   kicks           pi += c1 * F  (momenta now at p: energies sampled here)  pi += c2 * F
//   drift at end    phi += dend * pi            (leapfrog, local drift)
// Self-consistent expansion: the last block of pass p fills ka1, ka3, dload of
// pass p+1 from the energies it reduced (see ScaleRecord).
struct PassCoef {
    double ka1, ka3;
    double dload;
    double c1, c2;
    double dend;
    double h;       // sub-step leaving this kick point (0 at the last point)
    double cL, cR;  // weights of the two half kicks of b at this point
    double t;       // time at this kick point
    double t_next;  // time at the next kick point
    double *traj;   // if set, the update at this point stores (a, b) here: a at the
                    // point and b after its left half kick (integer time for VV2)
};

// Scale factor record on the device (self-consistent expansion) and the raw
// volume sums of the last reducing pass.
constexpr int kMaxQ = 16;
struct ScaleRecord {
    double a, b, t;
    double pad;
    double sums[kMaxQ];
    double maxes[4];
    double w[8];    // U(1) pass weights written on the device (self-consistent expansion)
};

// kLastSelf: velocity-Verlet update of b and a (self_update); kLastSelfLF:
// leapfrog update (self_update_lf), which also keeps the raw sums of the
// kicked momenta squared in ScaleRecord::sums[kPiPrev + f] for the next kick.
enum LastMode : int { kLastStore = 0, kLastSelf = 1, kLastSelfLF = 2 };
constexpr int kPiPrev = 8;

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ inline void store_agent(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline double load_agent(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A block's arrival at a last-block reduction, called by the thread that stored
// the block's partials: the ticket increment releases them at agent scope, and
// only the block that takes the last ticket then acquires.  An agent-scope
// acquire invalidates the XCD's L2, so taking it in every block would throw out
// the neighbour planes that the other blocks on that XCD still read.  The
// acquire fence after the increment that read the final count synchronises with
// every block's release (the increments form one release sequence).
__device__ inline bool ticket_arrive(unsigned *ticket, unsigned nblocks)
{
    const unsigned prev = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (prev != nblocks - 1) return false;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// Logical block id from the hardware block id: consecutive hardware blocks are
// dealt round-robin to the 8 XCDs, so give each XCD a contiguous range of
// logical tiles (neighbouring tiles then share that XCD's L2).
// Element access through a 32-bit byte offset from a uniform base pointer
// (valid while N^3 * sizeof(T) < 2^32, i.e. N <= 256 in float64).  Forming the
// offset in 32 bits lets the compiler use the scalar-base + 32-bit-offset
// global load and store forms, so every array shares one offset register
// instead of holding a 64-bit address per access.
template <typename T>
__device__ __forceinline__ T ld32(const T *base, unsigned i)
{
    return *(const T *)((const char *)base + (size_t)(i * (unsigned)sizeof(T)));
}

template <typename T>
__device__ __forceinline__ void st32(T *base, unsigned i, T v)
{
    *(T *)((char *)base + (size_t)(i * (unsigned)sizeof(T))) = v;
}

template <typename T>
__device__ __forceinline__ void st32_nt(T *base, unsigned i, T v)
{
    __builtin_nontemporal_store(v, (T *)((char *)base + (size_t)(i * (unsigned)sizeof(T))));
}

__device__ inline int xcd_logical_block(int b, int nb)
{
    const int per = nb / 8, rem = nb % 8;
    const int x = b % 8, j = b / 8;
    return x * per + (x < rem ? x : rem) + j;
}

// Block-wide deterministic sum of NQ values per thread into out[] (valid in thread 0).
template <int NT, int NQ>
__device__ inline void block_sums(double (&acc)[NQ], double *lds_red, double (&out)[NQ])
{
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double v = wave_sum(acc[q]);
        if (lane == 0) lds_red[w * NQ + q] = v;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double s = 0.0;
            for (int i = 0; i < NW; ++i) s += lds_red[i * NQ + q];
            out[q] = s;
        }
    }
    __syncthreads();
}

}  // namespace lat
