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
#include <hip/hip_runtime.h>

#include <cstdio>
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

int main()
{
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
    CK(hipGetLastError());
    for (void *p : owned) CK(hipFree(p));
    return 0;
}
