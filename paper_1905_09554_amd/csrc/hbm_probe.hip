// HBM bandwidth calibration: what plain streaming kernels reach on this GPU.
// It is the denominator next to the 8 TB/s datasheet peak when the step's
// achieved bandwidth is compared.  Prints one line per kernel and launch shape.
//
//   paper_1905_09554_amd/hbm_probe
//
// Kernels: float4 copy (read + write; also with non-temporal stores, with
// non-temporal loads and stores, and with four loads in flight per thread),
// float copy, float4 read-only (sum), float4 write-only (fill), and a
// 19-array stream (19 reads + 19 writes of float per node, the step's memory
// pattern without the stencil; also with non-temporal stores).
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
// The non-temporal builtins take clang's own vector types.
typedef float v4f __attribute__((ext_vector_type(4)));

// float4 copy with non-temporal stores, and with non-temporal loads too.
__global__ void copy4_nt(const v4f* __restrict__ a, v4f* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    __builtin_nontemporal_store(a[i], &b[i]);
}
__global__ void copy4_ntld(const v4f* __restrict__ a, v4f* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    __builtin_nontemporal_store(__builtin_nontemporal_load(&a[i]), &b[i]);
}
// Four float4 loads in flight per thread before the (non-temporal) stores.
__global__ void copy4_u4(const v4f* __restrict__ a, v4f* __restrict__ b, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const v4f v0 = a[i], v1 = a[i + stride], v2 = a[i + 2 * stride], v3 = a[i + 3 * stride];
    __builtin_nontemporal_store(v0, &b[i]);
    __builtin_nontemporal_store(v1, &b[i + stride]);
    __builtin_nontemporal_store(v2, &b[i + 2 * stride]);
    __builtin_nontemporal_store(v3, &b[i + 3 * stride]);
  }
  for (; i < n; i += stride) __builtin_nontemporal_store(a[i], &b[i]);
}
// The 19-array stream with non-temporal stores (as the step writes).
__global__ void stream19_nt(const float* __restrict__ a, float* __restrict__ b, size_t n,
                            size_t ps) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    float v[19];
#pragma unroll
    for (int q = 0; q < 19; ++q) v[q] = a[q * ps + i];
#pragma unroll
    for (int q = 0; q < 19; ++q) __builtin_nontemporal_store(v[q] * 1.0001f, &b[q * ps + i]);
  }
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
    std::printf("%-11s grid %6d  %8.3f ms  %8.1f GB/s\n", name, grid, ms, traffic / ms / 1e6);
    std::fflush(stdout);
    return 0;
  };
  for (int grid : {1024, 2048, 4096, 16384, 65536}) {
    if (run("copy4", grid, 2.0 * bytes, [&] { copy4<<<grid, 256>>>((float4*)a, (float4*)b, n4); }))
      return 1;
    if (run("copy4_nt", grid, 2.0 * bytes,
            [&] { copy4_nt<<<grid, 256>>>((v4f*)a, (v4f*)b, n4); }))
      return 1;
    if (run("copy4_ntld", grid, 2.0 * bytes,
            [&] { copy4_ntld<<<grid, 256>>>((v4f*)a, (v4f*)b, n4); }))
      return 1;
    if (run("copy4_u4", grid, 2.0 * bytes,
            [&] { copy4_u4<<<grid, 256>>>((v4f*)a, (v4f*)b, n4); }))
      return 1;
    if (run("stream19nt", grid, 2.0 * 19 * n19 * 4,
            [&] { stream19_nt<<<grid, 256>>>(a, b, n19, ps19); }))
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
