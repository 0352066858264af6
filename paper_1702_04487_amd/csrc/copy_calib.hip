// copy_calib -- a plain device-to-device copy of known size.
//
// It serves two measurements of the lattice kernels: the copy bandwidth that
// HBM actually sustains on this part (the practical ceiling beside the
// nominal peak), and the calibration of the traffic counters (FETCH_SIZE,
// WRITE_SIZE): each launch reads exactly `bytes` and writes exactly `bytes`,
// so the ratio of those to what a counter reports for this kernel scales the
// counter's reading for any other kernel.
//
// Usage: copy_calib [MiB per buffer (default 1792 = 14 planes of 2048 x 16384
//        floats, the size of one distribution buffer of that lattice)]
//        [timed launches per copy shape (default 10)]
// Besides the plain copies it times 14-plane copies of the same buffer (below)
// when the buffer is whole 32-row blocks of 2048-column rows.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                                    \
    do {                                                                                         \
        hipError_t e_ = (x);                                                                     \
        if (e_ != hipSuccess) {                                                                  \
            std::fprintf(stderr, "copy_calib: %s failed: %s\n", #x, hipGetErrorString(e_));     \
            return 1;                                                                            \
        }                                                                                        \
    } while (0)

template <typename T>
__global__ __launch_bounds__(256) void k_copy(const T* __restrict__ a, T* __restrict__ b, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

// Copies of 14 float planes of kWx columns (the distribution buffer of the
// lattice kernels): one node per thread with the planes of a row block
// interleaved or apart, and 32-row tiles walked by 256-column workgroups as
// the fused lattice kernel walks them.  Every launch reads and writes the
// whole buffer once.
constexpr int kPlanes = 14, kWx = 2048, kTileRows = 32;

template <bool ROW_INTERLEAVED>
__global__ __launch_bounds__(256) void k_planes_flat(const float* __restrict__ a, float* __restrict__ b, size_t n)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;   // node
    if (i >= n) return;
    const size_t y = i / kWx, x = i - y * kWx;
    float v[kPlanes];
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) v[p] = a[ROW_INTERLEAVED ? (y * kPlanes + p) * kWx + x : p * n + i];
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) b[ROW_INTERLEAVED ? (y * kPlanes + p) * kWx + x : p * n + i] = v[p];
}

__global__ __launch_bounds__(256) void k_planes_tiles(const float* __restrict__ a, float* __restrict__ b, size_t n)
{
    constexpr int strips = kWx / 256;
    const int rb = blockIdx.x / strips, strip = blockIdx.x % strips;
    const size_t x = (size_t)strip * 256 + threadIdx.x;
    for (int r = 0; r < kTileRows; ++r) {
        const size_t i = ((size_t)rb * kTileRows + r) * kWx + x;
        float v[kPlanes];
#pragma unroll
        for (int p = 0; p < kPlanes; ++p) v[p] = a[p * n + i];
#pragma unroll
        for (int p = 0; p < kPlanes; ++p) b[p * n + i] = v[p];
    }
}

int main(int argc, char** argv)
{
    const long long mib = argc > 1 ? std::atoll(argv[1]) : 1792;
    const int launches = argc > 2 ? std::atoi(argv[2]) : 10;
    if (mib < 1 || mib > 65536 || launches < 1 || launches > 1000) {
        std::fprintf(stderr, "copy_calib: MiB must lie in [1, 65536] and launches in [1, 1000]\n");
        return 2;
    }
    const size_t bytes = (size_t)mib << 20;
    void *a = nullptr, *b = nullptr;
    CK(hipMalloc(&a, bytes));
    CK(hipMalloc(&b, bytes));
    CK(hipMemset(a, 0x3c, bytes));
    CK(hipMemset(b, 0, bytes));
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    std::printf("copy_calib: every launch reads %zu B and writes %zu B (%zu KiB each)\n", bytes, bytes,
                bytes >> 10);
    double best = 0.0;
    // element width x grid: the copy shapes tried; the best rate is the
    // practical read+write ceiling
    for (int vec = 0; vec < 2; ++vec) {
        for (int grid : {4096, 16384, 65536}) {
            auto launch = [&]() {
                if (vec)
                    hipLaunchKernelGGL(k_copy<float4>, dim3(grid), dim3(256), 0, 0, (const float4*)a, (float4*)b,
                                       bytes / sizeof(float4));
                else
                    hipLaunchKernelGGL(k_copy<float>, dim3(grid), dim3(256), 0, 0, (const float*)a, (float*)b,
                                       bytes / sizeof(float));
            };
            launch();   // warm-up
            CK(hipGetLastError());
            CK(hipEventRecord(e0, 0));
            for (int r = 0; r < launches; ++r) launch();
            CK(hipGetLastError());
            CK(hipEventRecord(e1, 0));
            CK(hipEventSynchronize(e1));
            float ms = 0.f;
            CK(hipEventElapsedTime(&ms, e0, e1));
            ms /= launches;
            const double gbs = 2.0 * bytes / (ms * 1e-3) / 1e9;
            best = gbs > best ? gbs : best;
            std::printf("copy_calib: %-6s grid %6d x 256: %.4f ms per launch, %.1f GB/s read+write\n",
                        vec ? "float4" : "float", grid, ms, gbs);
        }
    }
    std::printf("copy_calib: best %.1f GB/s read+write\n", best);
    // the 14-plane copies, when the buffer is whole rows of 32-row tiles
    const size_t n = bytes / (sizeof(float) * kPlanes);
    if (bytes % (sizeof(float) * kPlanes) == 0 && n % ((size_t)kWx * kTileRows) == 0) {
        const float* A = (const float*)a;
        float* B = (float*)b;
        for (int shape = 0; shape < 3; ++shape) {
            auto launch = [&]() {
                const unsigned flat = (unsigned)((n + 255) / 256), tiles = (unsigned)(n / ((size_t)kWx * kTileRows) * (kWx / 256));
                if (shape == 0) hipLaunchKernelGGL(k_planes_flat<false>, dim3(flat), dim3(256), 0, 0, A, B, n);
                if (shape == 1) hipLaunchKernelGGL(k_planes_flat<true>, dim3(flat), dim3(256), 0, 0, A, B, n);
                if (shape == 2) hipLaunchKernelGGL(k_planes_tiles, dim3(tiles), dim3(256), 0, 0, A, B, n);
            };
            launch();
            CK(hipGetLastError());
            CK(hipEventRecord(e0, 0));
            for (int r = 0; r < launches; ++r) launch();
            CK(hipGetLastError());
            CK(hipEventRecord(e1, 0));
            CK(hipEventSynchronize(e1));
            float ms = 0.f;
            CK(hipEventElapsedTime(&ms, e0, e1));
            ms /= launches;
            static const char* names[3] = {"14 planes apart, a node per thread",
                                           "14 planes row-interleaved, a node per thread",
                                           "14 planes apart, 32-row tiles of 256 columns"};
            std::printf("copy_calib: %s: %.4f ms per launch, %.1f GB/s read+write\n", names[shape], ms,
                        2.0 * bytes / (ms * 1e-3) / 1e9);
        }
    }
    CK(hipFree(a));
    CK(hipFree(b));
    return 0;
}
