// Machine ceilings of one gfx950 GPU, measured rather than taken from the
// data sheet: the matrix-core rate of each MFMA the product kernels use
// (register operands, no memory traffic, 1, 2 and 4 waves per SIMD) and
// the HBM rate of a plain device-to-device copy and of a read-only stream
// over a buffer much larger than the last-level cache.  A standalone program,
// not part of the library; it prints one JSON object per measurement.
//
//   paper_2407_21637_amd/calibrate [scale]
//
// scale (default 1) multiplies the MFMA loops' length: at 1 each timed
// launch lasts about a millisecond; longer ones show the sustained rate
// under the card's power limit.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                     \
    do {                                                                             \
        hipError_t e_ = (x);                                                         \
        if (e_ != hipSuccess) {                                                      \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));             \
            std::exit(1);                                                            \
        }                                                                            \
    } while (0)

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

enum Kind { kF64 = 0, kF32 = 1, kF16 = 2, kBF16 = 3 };

// flops of one MFMA of each kind (2 M N K)
constexpr double kFlops[4] = {2.0 * 16 * 16 * 4, 2.0 * 16 * 16 * 4, 2.0 * 16 * 16 * 32, 2.0 * 16 * 16 * 32};
const char* kName[4] = {"v_mfma_f64_16x16x4f64", "v_mfma_f32_16x16x4f32", "v_mfma_f32_16x16x32_f16",
                        "v_mfma_f32_16x16x32_bf16"};

// NA independent accumulators per wave, iters rounds of NA MFMAs; the
// results are summed into out[block * 256 + thread] so nothing is dead code
template <int K, int NA>
__global__ __launch_bounds__(256) void k_mfma(double* out, int iters, float seed) {
    const float s = seed + float(threadIdx.x);
    if constexpr (K == kF64) {
        d4 acc[NA];
        for (int i = 0; i < NA; ++i) acc[i] = d4{0, 0, 0, 0};
        const double a = s, b = 1.0 / (1.0 + s);
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int i = 0; i < NA; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
        double t = 0;
        for (int i = 0; i < NA; ++i) t += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
        out[blockIdx.x * 256 + threadIdx.x] = t;
    } else {
        f4 acc[NA];
        for (int i = 0; i < NA; ++i) acc[i] = f4{0, 0, 0, 0};
        if constexpr (K == kF32) {
            const float a = s, b = 1.0f / (1.0f + s);
            for (int it = 0; it < iters; ++it)
#pragma unroll
                for (int i = 0; i < NA; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i], 0, 0, 0);
        } else if constexpr (K == kF16) {
            h8 a, b;
            for (int q = 0; q < 8; ++q) {
                a[q] = _Float16(s * 1e-3f + q);
                b[q] = _Float16(1.0f / (1.0f + s + q));
            }
            for (int it = 0; it < iters; ++it)
#pragma unroll
                for (int i = 0; i < NA; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc[i], 0, 0, 0);
        } else {
            b8 a, b;
            for (int q = 0; q < 8; ++q) {
                a[q] = __bf16(s * 1e-3f + q);
                b[q] = __bf16(1.0f / (1.0f + s + q));
            }
            for (int it = 0; it < iters; ++it)
#pragma unroll
                for (int i = 0; i < NA; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i], 0, 0, 0);
        }
        float t = 0;
        for (int i = 0; i < NA; ++i) t += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
        out[blockIdx.x * 256 + threadIdx.x] = t;
    }
}

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ a, float4* __restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < n; i += size_t(gridDim.x) * 256) b[i] = a[i];
}

// Read-only stream: every lane issues U independent 16-byte loads per
// step (grid-strided), sums them, and writes one value per workgroup at
// the end, so the kernel's HBM traffic is the buffer read once.
template <int U>
__global__ __launch_bounds__(256) void k_read(const float4* __restrict__ a, size_t n, float* __restrict__ out) {
    float acc = 0.0f;
    const size_t stride = size_t(gridDim.x) * 256;
    size_t i = blockIdx.x * size_t(256) + threadIdx.x;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = a[i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) acc += v[u].x + v[u].y + v[u].z + v[u].w;
    }
    for (; i < n; i += stride) {
        const float4 v = a[i];
        acc += v.x + v.y + v.z + v.w;
    }
    __shared__ float red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int t = 0; t < 256; ++t) s += red[t];
        out[blockIdx.x] = s;
    }
}

int compute_units() {
    hipDeviceProp_t p;
    CHECK(hipGetDeviceProperties(&p, 0));
    return p.multiProcessorCount;
}

template <int K, int NA>
void run_mfma(int cus, int waves_per_simd, int iters) {
    const int blocks = cus * waves_per_simd;      // 4 waves per block: one per SIMD
    double* out;
    CHECK(hipMalloc(&out, sizeof(double) * 256 * size_t(blocks)));
    hipLaunchKernelGGL((k_mfma<K, NA>), dim3(blocks), dim3(256), 0, 0, out, 16, 1.0f);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    CHECK(hipEventRecord(e0, 0));
    hipLaunchKernelGGL((k_mfma<K, NA>), dim3(blocks), dim3(256), 0, 0, out, iters, 1.0f);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    const double flops = double(blocks) * 4 * double(iters) * NA * kFlops[K];
    std::printf("{\"probe\": \"mfma\", \"instr\": \"%s\", \"waves_per_simd\": %d, \"accumulators\": %d, "
                "\"ms\": %.4f, \"tflops\": %.2f}\n",
                kName[K], waves_per_simd, NA, ms, flops / (ms * 1e-3) / 1e12);
    std::fflush(stdout);
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    CHECK(hipFree(out));
}

template <int K>
void sweep(int cus, int iters) {
    run_mfma<K, 8>(cus, 1, iters);
    run_mfma<K, 8>(cus, 2, iters);
    run_mfma<K, 4>(cus, 4, iters);
}

void run_copy(int cus) {
    const size_t bytes = size_t(1) << 30;          // 1 GiB each way
    const size_t n = bytes / sizeof(float4);
    float4 *a, *b;
    CHECK(hipMalloc(&a, bytes));
    CHECK(hipMalloc(&b, bytes));
    CHECK(hipMemset(a, 0, bytes));
    const int blocks = cus * 16;
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, 0, a, b, n);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const int reps = 10;
    CHECK(hipEventRecord(e0, 0));
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, 0, a, b, n);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    const double moved = 2.0 * double(bytes) * reps;
    std::printf("{\"probe\": \"copy\", \"bytes_each_way\": %zu, \"ms_per_copy\": %.4f, \"gbs\": %.1f}\n", bytes,
                ms / reps, moved / (ms * 1e-3) / 1e9);
    std::fflush(stdout);
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    CHECK(hipFree(a));
    CHECK(hipFree(b));
}

template <int U>
void run_read_one(const float4* a, size_t n, int blocks, float* out, size_t bytes) {
    hipLaunchKernelGGL(k_read<U>, dim3(blocks), dim3(256), 0, 0, a, n, out);     // warm-up (TLB, clocks)
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const int reps = 5;
    CHECK(hipEventRecord(e0, 0));
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(k_read<U>, dim3(blocks), dim3(256), 0, 0, a, n, out);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    std::printf("{\"probe\": \"read\", \"bytes\": %zu, \"workgroups\": %d, \"loads_in_flight_per_lane\": %d, "
                "\"ms_per_read\": %.4f, \"gbs\": %.1f}\n",
                bytes, blocks, U, ms / reps, double(bytes) * reps / (ms * 1e-3) / 1e9);
    std::fflush(stdout);
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
}

// A buffer 16x the 256 MB last-level cache, read once per launch: the
// achievable HBM read rate (no reuse can hide in the cache).
void run_read(int cus) {
    const size_t bytes = size_t(4) << 30;
    const size_t n = bytes / sizeof(float4);
    float4* a;
    float* out;
    CHECK(hipMalloc(&a, bytes));
    CHECK(hipMalloc(&out, sizeof(float) * 64 * size_t(cus)));
    CHECK(hipMemset(a, 0, bytes));
    for (int mult : {4, 8, 16, 32}) {
        run_read_one<4>(a, n, cus * mult, out, bytes);
        run_read_one<8>(a, n, cus * mult, out, bytes);
    }
    CHECK(hipFree(a));
    CHECK(hipFree(out));
}

int main(int argc, char** argv) {
    const int scale = argc > 1 ? std::atoi(argv[1]) : 1;
    if (scale < 1 || scale > 1000) {
        std::fprintf(stderr, "scale must be in [1, 1000]\n");
        return 1;
    }
    const int cus = compute_units();
    std::printf("{\"probe\": \"device\", \"compute_units\": %d, \"scale\": %d}\n", cus, scale);
    run_copy(cus);
    run_read(cus);
    sweep<kF64>(cus, 4000 * scale);
    sweep<kF32>(cus, 8000 * scale);
    sweep<kF16>(cus, 8000 * scale);
    sweep<kBF16>(cus, 8000 * scale);
    return 0;
}
