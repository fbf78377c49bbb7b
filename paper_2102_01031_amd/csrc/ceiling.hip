// ceiling.hip -- streaming-bandwidth ceilings of the GPU for the access
// patterns of the lattice kernels, measured with plain streaming kernels (no
// stencil, no reductions across blocks): the rate the stage kernels are
// compared with besides the HBM peak.  Each line printed is JSON:
//   copy          one array in, one out, 16 bytes per lane (1 GiB each)
//   streams4_256  4 float64 arrays in, 4 out, 256^3 each (the two-field stage)
//   streams4_256_16B  the same with 16 bytes per lane and access
//   streams10_128 10 float64 arrays in, 10 out, 128^3 each (the U(1) pass;
//                 the 336 MB working set is largely cache-resident)
//   read4_256     4 float64 arrays of 256^3 read and summed (the energy pass)
// Rates are bytes moved / kernel time from HIP events, mean of 20 launches
// after one warm-up launch.
//
// With the argument "series" the probe also runs ping-pong series: two sets of
// four float64 arrays of 256^3 (float32: "f32" patterns), launch k reading
// one set and writing the other, as consecutive stage passes do, so the
// memory-side cache sees the traffic of a real sequence of passes.  Each
// pattern is named pp<E>_<load policy>_<store policy>_<order>:
//   load / store policy: the cache-policy bits of the buffer access (plain;
//     nt = non-temporal; sc1 = system scope),
//   order: fix = every launch walks memory upward; alt = odd launches walk
//     it downward, so a launch starts on the data the previous one wrote last,
//   E: elements per thread (1, or 4 as four loads per array in flight).
// "lds" patterns move the four input arrays through LDS with 16-byte
// global-to-LDS loads before the stores.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <vector>

#define CK(x)                                                                            \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) {                                                          \
            std::fprintf(stderr, "%s: %s (line %d)\n", #x, hipGetErrorString(e_), __LINE__); \
            return 1;                                                                    \
        }                                                                                \
    } while (0)

typedef double d2 __attribute__((ext_vector_type(2)));

__global__ void __launch_bounds__(256) copy16(const d2 *__restrict__ a, d2 *__restrict__ b, size_t n2)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n2) __builtin_nontemporal_store(a[i], &b[i]);
}

template <int K>
struct Ptrs {
    const double *in[K];
    double *out[K];
};

template <int K>
__global__ void __launch_bounds__(256) streams(const Ptrs<K> p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        double x[K];
#pragma unroll
        for (int a = 0; a < K; ++a) x[a] = p.in[a][i];
#pragma unroll
        for (int a = 0; a < K; ++a) __builtin_nontemporal_store(x[a] + 1.0, &p.out[a][i]);
    }
}

// the same with 16 bytes per lane and access (two float64 per load and store)
template <int K>
__global__ void __launch_bounds__(256) streams16(const Ptrs<K> p, size_t n2)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n2; i += (size_t)gridDim.x * 256) {
        d2 x[K];
#pragma unroll
        for (int a = 0; a < K; ++a) x[a] = ((const d2 *)p.in[a])[i];
#pragma unroll
        for (int a = 0; a < K; ++a) __builtin_nontemporal_store(x[a] + 1.0, &((d2 *)p.out[a])[i]);
    }
}
__global__ void __launch_bounds__(256) read4(const Ptrs<4> p, size_t n, double *partial)
{
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        s += (p.in[0][i] * p.in[0][i] + p.in[1][i] * p.in[1][i]) + (p.in[2][i] * p.in[2][i] + p.in[3][i] * p.in[3][i]);
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}


// ---------------------------------------------------------------------------
// ping-pong series with explicit cache policies (buffer loads and stores)
// ---------------------------------------------------------------------------
// cache-policy bits of gfx950 buffer instructions
constexpr int kPlain = 0, kNT = 2, kSC1 = 16;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

// E elements per thread, in E rounds of 256 consecutive elements per block;
// block b covers elements [b * 256 E, (b + 1) * 256 E), taken in reverse block
// order when down != 0.  n is a multiple of 256 E (checked on the host).
template <typename T, int E, int LDP, int STP>
__global__ void __launch_bounds__(256) pp4(const Ptrs<4> p, unsigned n, int down)
{
    const unsigned nb = gridDim.x;
    const unsigned b = down ? nb - 1 - blockIdx.x : blockIdx.x;
    const unsigned bytes = n * (unsigned)sizeof(T);
    T x[4][E];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const __amdgpu_buffer_rsrc_t r = rsrc(p.in[a], bytes);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const unsigned i = (b * E + e) * 256 + threadIdx.x;
            if constexpr (sizeof(T) == 8)
                x[a][e] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8, 0, LDP));
            else
                x[a][e] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, i * 4, 0, LDP));
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const __amdgpu_buffer_rsrc_t w = rsrc(p.out[a], bytes);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const unsigned i = (b * E + e) * 256 + threadIdx.x;
            const T y = x[a][e] + T(1);
            if constexpr (sizeof(T) == 8) {
                typedef unsigned u2 __attribute__((ext_vector_type(2)));
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, y), w, i * 8, 0, STP);
            } else {
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, y), w, i * 4, 0, STP);
            }
        }
    }
}

// the four input arrays through LDS: each thread moves 16 bytes of each array
// with one global-to-LDS load, waits, and stores them from LDS.  Block b covers
// bytes [b * 4096, (b + 1) * 4096) of every array (n * 8 is a multiple of 4096).
template <int STP>
__global__ void __launch_bounds__(256) lds4(const Ptrs<4> p, unsigned n, int down)
{
    __shared__ __attribute__((aligned(16))) double buf[4][256 * 2];
    const unsigned nb = gridDim.x;
    const unsigned b = down ? nb - 1 - blockIdx.x : blockIdx.x;
    const unsigned e2 = b * 512 + 2 * threadIdx.x;   // first of this thread's two elements
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < 4; ++a)
        __builtin_amdgcn_global_load_lds((const void *)(p.in[a] + e2),
                                         (__attribute__((address_space(3))) void *)&buf[a][wave * 128], 16, 0, 0);
    __builtin_amdgcn_s_waitcnt(0);   // vmcnt(0): the LDS writes of this wave's loads have landed
    __syncthreads();
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const __amdgpu_buffer_rsrc_t w = rsrc(p.out[a], n * 8u);
        d2 v = *(const d2 *)&buf[a][2 * threadIdx.x];
        v += 1.0;
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), w, e2 * 8, 0, STP);
    }
}

template <typename F>
static float mean_ms(F &&launch)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.f;
    launch();
    (void)hipDeviceSynchronize();
    (void)hipEventRecord(e0, 0);
    for (int r = 0; r < 20; ++r) launch();
    (void)hipEventRecord(e1, 0);
    (void)hipEventSynchronize(e1);
    float ms = -1.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms / 20.f;
}

static void line(const char *name, double bytes, float ms)
{
    std::printf("{\"pattern\": \"%s\", \"bytes\": %.0f, \"us\": %.2f, \"GBs\": %.0f}\n", name, bytes, ms * 1e3,
                bytes / (ms * 1e-3) / 1e9);
}

// mean time per launch of a series of 20 ping-pong launches after two warm-up
// launches: launch k reads set k % 2 and writes the other; with alt != 0 odd
// launches walk memory downward
template <typename L>
static float series_ms(L &&launch, int alt)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.f;
    launch(0, 0);
    launch(1, alt);
    (void)hipDeviceSynchronize();
    (void)hipEventRecord(e0, 0);
    for (int k = 0; k < 20; ++k) launch(k & 1, alt ? (k & 1) : 0);
    (void)hipEventRecord(e1, 0);
    (void)hipEventSynchronize(e1);
    float ms = -1.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms / 20.f;
}

static const char *pol_name(int p) { return p == kNT ? "nt" : p == kSC1 ? "sc1" : "plain"; }

template <typename T, int E, int LDP, int STP>
static void pp_line(Ptrs<4> (&sets)[2], unsigned n, int alt)
{
    const unsigned g = n / (256u * E);
    const float ms = series_ms(
        [&](int s, int down) { hipLaunchKernelGGL((pp4<T, E, LDP, STP>), dim3(g), dim3(256), 0, 0, sets[s], n, down); },
        alt);
    char name[96];
    std::snprintf(name, sizeof(name), "pp%d%s_%s_%s_%s", E, sizeof(T) == 4 ? "f32" : "", pol_name(LDP),
                  pol_name(STP), alt ? "alt" : "fix");
    line(name, 8.0 * sizeof(T) * n, ms);
}

template <int STP>
static void lds_line(Ptrs<4> (&sets)[2], unsigned n, int alt)
{
    const unsigned g = n / 512u;
    const float ms = series_ms(
        [&](int s, int down) { hipLaunchKernelGGL((lds4<STP>), dim3(g), dim3(256), 0, 0, sets[s], n, down); }, alt);
    char name[96];
    std::snprintf(name, sizeof(name), "lds_%s_%s", pol_name(STP), alt ? "alt" : "fix");
    line(name, 8.0 * 8 * n, ms);
}

int main(int argc, char **argv)
{
    const bool series = argc > 1 && std::strcmp(argv[1], "series") == 0;
    std::vector<void *> owned;
    auto alloc = [&](size_t bytes, void **p) -> hipError_t {
        hipError_t e = hipMalloc(p, bytes);
        if (e == hipSuccess) {
            owned.push_back(*p);
            e = hipMemset(*p, 0, bytes);
        }
        return e;
    };
    {   // copy, 1 GiB
        const size_t bytes = (size_t)1 << 30, n2 = bytes / 16;
        void *a, *b;
        CK(alloc(bytes, &a));
        CK(alloc(bytes, &b));
        const unsigned g = (unsigned)((n2 + 255) / 256);
        const float ms = mean_ms([&] { hipLaunchKernelGGL(copy16, dim3(g), dim3(256), 0, 0, (const d2 *)a, (d2 *)b, n2); });
        line("copy", 2.0 * bytes, ms);
    }
    {   // 4 in, 4 out at 256^3
        const size_t n = (size_t)256 * 256 * 256;
        Ptrs<4> p{};
        for (int a = 0; a < 4; ++a) {
            void *x, *y;
            CK(alloc(n * 8, &x));
            CK(alloc(n * 8, &y));
            p.in[a] = (const double *)x;
            p.out[a] = (double *)y;
        }
        const float ms = mean_ms([&] { hipLaunchKernelGGL(streams<4>, dim3(65536), dim3(256), 0, 0, p, n); });
        line("streams4_256", 8.0 * 8 * n, ms);
        const float m16 = mean_ms([&] { hipLaunchKernelGGL(streams16<4>, dim3(32768), dim3(256), 0, 0, p, n / 2); });
        line("streams4_256_16B", 8.0 * 8 * n, m16);
        void *part;
        CK(alloc(4096 * 8, &part));
        const float mr = mean_ms([&] { hipLaunchKernelGGL(read4, dim3(4096), dim3(256), 0, 0, p, n, (double *)part); });
        line("read4_256", 4.0 * 8 * n, mr);
    }
    {   // 10 in, 10 out at 128^3
        const size_t n = (size_t)128 * 128 * 128;
        Ptrs<10> p{};
        for (int a = 0; a < 10; ++a) {
            void *x, *y;
            CK(alloc(n * 8, &x));
            CK(alloc(n * 8, &y));
            p.in[a] = (const double *)x;
            p.out[a] = (double *)y;
        }
        const float ms = mean_ms([&] { hipLaunchKernelGGL(streams<10>, dim3(8192), dim3(256), 0, 0, p, n); });
        line("streams10_128", 20.0 * 8 * n, ms);
    }
    if (series) {   // ping-pong series at 256^3: two sets of 4 arrays
        const unsigned n = 256u * 256u * 256u;   // a multiple of 256 * 4 and of 512
        Ptrs<4> sets[2] = {};
        for (int a = 0; a < 4; ++a) {
            void *x, *y;
            CK(alloc((size_t)n * 8, &x));
            CK(alloc((size_t)n * 8, &y));
            sets[0].in[a] = sets[1].out[a] = (double *)x;
            sets[1].in[a] = sets[0].out[a] = (double *)y;
        }
        for (int alt = 0; alt < 2; ++alt) {
            pp_line<double, 1, kPlain, kNT>(sets, n, alt);
            pp_line<double, 1, kPlain, kPlain>(sets, n, alt);
            pp_line<double, 1, kNT, kPlain>(sets, n, alt);
            pp_line<double, 1, kNT, kNT>(sets, n, alt);
            pp_line<double, 1, kSC1, kPlain>(sets, n, alt);
            pp_line<double, 1, kPlain, kSC1>(sets, n, alt);
            pp_line<double, 4, kPlain, kNT>(sets, n, alt);
            pp_line<double, 4, kPlain, kPlain>(sets, n, alt);
            pp_line<double, 4, kNT, kPlain>(sets, n, alt);
            pp_line<double, 4, kNT, kNT>(sets, n, alt);
            lds_line<kPlain>(sets, n, alt);
            lds_line<kNT>(sets, n, alt);
        }
        // float32: the same arrays hold 256^3 float32 values in their first half
        Ptrs<4> s32[2] = {};
        for (int s = 0; s < 2; ++s) s32[s] = sets[s];
        for (int alt = 0; alt < 2; ++alt) {
            pp_line<float, 1, kPlain, kNT>(reinterpret_cast<Ptrs<4>(&)[2]>(s32), n, alt);
            pp_line<float, 1, kPlain, kPlain>(reinterpret_cast<Ptrs<4>(&)[2]>(s32), n, alt);
            pp_line<float, 4, kPlain, kPlain>(reinterpret_cast<Ptrs<4>(&)[2]>(s32), n, alt);
            pp_line<float, 4, kNT, kPlain>(reinterpret_cast<Ptrs<4>(&)[2]>(s32), n, alt);
            pp_line<float, 4, kPlain, kNT>(reinterpret_cast<Ptrs<4>(&)[2]>(s32), n, alt);
        }
    }
    CK(hipGetLastError());
    for (void *p : owned) CK(hipFree(p));
    return 0;
}
