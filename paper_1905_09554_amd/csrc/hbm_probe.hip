// HBM bandwidth calibration: what plain streaming kernels reach on this GPU.
// It is the denominator next to the 8 TB/s datasheet peak when the step's
// achieved bandwidth is compared.  Prints one line per kernel and launch shape.
//
//   paper_1905_09554_amd/hbm_probe
//
// Kernels: float4 copy (read + write), float copy, float4 read-only (sum),
// float4 write-only (fill), and a 19-array stream (19 reads + 19 writes of
// float per node, the step's memory pattern without the stencil).
#include <hip/hip_runtime.h>

#include <cstdio>

#define CK(x)                                                                   \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                     \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      return 1;                                                                 \
    }                                                                           \
  } while (0)

__global__ void copy4(const float4* __restrict__ a, float4* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}
__global__ void copy1(const float* __restrict__ a, float* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}
__global__ void read4(const float4* __restrict__ a, float* __restrict__ out, size_t n) {
  float s = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const float4 v = a[i];
    s += v.x + v.y + v.z + v.w;
  }
  if (s == 1234.5f) out[0] = s;  // keeps the loads alive; never true for zero input
}
__global__ void write4(float4* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    b[i] = make_float4(1.f, 2.f, 3.f, 4.f);
}
__global__ void stream19(const float* __restrict__ a, float* __restrict__ b, size_t n,
                         size_t ps) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    float v[19];
#pragma unroll
    for (int q = 0; q < 19; ++q) v[q] = a[q * ps + i];
#pragma unroll
    for (int q = 0; q < 19; ++q) b[q * ps + i] = v[q] * 1.0001f;
  }
}

int main() {
  const size_t bytes = (size_t)4 << 30;  // two 4 GiB buffers
  float *a, *b, *o;
  CK(hipMalloc(&a, bytes));
  CK(hipMalloc(&b, bytes));
  CK(hipMalloc(&o, 64));
  CK(hipMemset(a, 0, bytes));
  CK(hipMemset(b, 0, bytes));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  const size_t n4 = bytes / 16, n1 = bytes / 4;
  // 19 arrays of n floats with stride ps: 19 * ps * 4 B = 2.55 GB < 4 GiB.
  const size_t n19 = 33554432, ps19 = n19 + 1088;
  auto run = [&](const char* name, int grid, double traffic, auto launch) -> int {
    launch();
    CK(hipDeviceSynchronize());
    CK(hipEventRecord(e0));
    for (int r = 0; r < 10; ++r) launch();
    CK(hipEventRecord(e1));
    CK(hipEventSynchronize(e1));
    float ms;
    CK(hipEventElapsedTime(&ms, e0, e1));
    ms /= 10;
    std::printf("%-10s grid %6d  %8.3f ms  %8.1f GB/s\n", name, grid, ms, traffic / ms / 1e6);
    std::fflush(stdout);
    return 0;
  };
  for (int grid : {1024, 4096, 16384, 65536}) {
    if (run("copy4", grid, 2.0 * bytes, [&] { copy4<<<grid, 256>>>((float4*)a, (float4*)b, n4); }))
      return 1;
    if (run("copy1", grid, 2.0 * bytes, [&] { copy1<<<grid, 256>>>(a, b, n1); })) return 1;
    if (run("read4", grid, 1.0 * bytes, [&] { read4<<<grid, 256>>>((float4*)a, o, n4); })) return 1;
    if (run("write4", grid, 1.0 * bytes, [&] { write4<<<grid, 256>>>((float4*)b, n4); })) return 1;
    if (run("stream19", grid, 2.0 * 19 * n19 * 4, [&] { stream19<<<grid, 256>>>(a, b, n19, ps19); }))
      return 1;
  }
  CK(hipFree(a));
  CK(hipFree(b));
  CK(hipFree(o));
  return 0;
}
