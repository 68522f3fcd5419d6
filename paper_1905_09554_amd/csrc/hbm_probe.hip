// HBM bandwidth calibration: what plain streaming kernels reach on this GPU.
// It is the denominator next to the 8 TB/s datasheet peak when the step's
// achieved bandwidth is compared.  Prints one line per kernel and launch shape.
//
//   paper_1905_09554_amd/hbm_probe [gridstride|onepass|stream|lds|pull|shift|wide|order|pull64|lds19|all]
//
// Families (every kernel moves a known number of bytes, timed over 10 launches
// after a warm-up with HIP events):
//  gridstride  float4 copy with a grid-stride loop (plain, non-temporal stores,
//              non-temporal loads and stores, four loads in flight per
//              thread), float copy, float4 read-only and write-only, for
//              256-, 512- and 1024-thread work-groups;
//  onepass     one pass over the buffer, no loop: work-group b copies its own
//              contiguous block of T * K float4, each thread K of them (all K
//              loads issued before the first store); also read-only and
//              write-only in the same shape;
//  stream      the step's memory pattern without its stencil: 19 arrays of
//              floats read and 19 written per node, one node per thread (one
//              pass), or a work-group marching a contiguous range of nodes with
//              the next chunk's 19 loads in flight during the current chunk's
//              stores (as the step carries the next plane in registers);
//  lds         float4 copy staged through LDS with gfx950's direct
//              global-to-LDS loads (global_load_lds_dwordx4): K float4 per
//              lane land in LDS without passing through registers, then each
//              lane reads its values back and stores them;
//  pull        the step's own pattern without the stencil (see pull_march),
//              in the 19-array layout and in blocks of 64 to 4096 nodes;
//  shift       the pull pattern in blocks of 1024 nodes with some of its x, y,
//              z shifts switched off, and with the x shift taken across lanes
//              from aligned loads (checked to store what the plain form does);
//  wide        the pull pattern with 2 or 4 consecutive nodes per lane (8- and
//              16-byte accesses) against one node per lane;
//  order       the pull pattern with its blocks of 1024 nodes in node order
//              or in tile-major order (a group's march is one contiguous run);
//  pull64      the pull pattern on float64 populations, tiles as the float64
//              step uses them and wider;
//  lds19       the same pattern with 16-byte direct global-to-LDS loads
//              (pull_lds), and a 19-array stream with 16-byte accesses.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>

#define CK(x)                                                                   \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                     \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      return 1;                                                                 \
    }                                                                           \
  } while (0)

// The non-temporal builtins take clang's own vector types.
typedef float v4f __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------- grid-stride
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

// ---------------------------------------------------------------- one pass
// Work-group b owns float4 elements [b T K, (b + 1) T K); thread t handles
// b T K + k T + t for k < K.  n must be a multiple of T K (checked on the
// host).  NT: non-temporal stores.
template <int K, bool NT>
__global__ void copy_onepass(const v4f* __restrict__ a, v4f* __restrict__ b) {
  const size_t base = (size_t)blockIdx.x * blockDim.x * K + threadIdx.x;
  v4f v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = a[base + (size_t)k * blockDim.x];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (NT)
      __builtin_nontemporal_store(v[k], &b[base + (size_t)k * blockDim.x]);
    else
      b[base + (size_t)k * blockDim.x] = v[k];
  }
}
template <int K>
__global__ void read_onepass(const v4f* __restrict__ a, float* __restrict__ out) {
  const size_t base = (size_t)blockIdx.x * blockDim.x * K + threadIdx.x;
  v4f v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = a[base + (size_t)k * blockDim.x];
  float s = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) s += v[k].x + v[k].y + v[k].z + v[k].w;
  if (s == 1234.5f) out[0] = s;
}
template <int K>
__global__ void write_onepass(v4f* __restrict__ b) {
  const size_t base = (size_t)blockIdx.x * blockDim.x * K + threadIdx.x;
  const v4f one = {1.f, 2.f, 3.f, 4.f};
#pragma unroll
  for (int k = 0; k < K; ++k) __builtin_nontemporal_store(one, &b[base + (size_t)k * blockDim.x]);
}

// ------------------------------------------------------------ 19-array stream
// One node per thread, one pass: n must be a multiple of the work-group size.
__global__ void stream19_onepass(const float* __restrict__ a, float* __restrict__ b, size_t ps) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  float v[19];
#pragma unroll
  for (int q = 0; q < 19; ++q) v[q] = a[q * ps + i];
#pragma unroll
  for (int q = 0; q < 19; ++q) __builtin_nontemporal_store(v[q] * 1.0001f, &b[q * ps + i]);
}
// Work-group b marches `chunks` consecutive chunks of blockDim.x nodes; the
// loads of chunk c + 1 are issued before the stores of chunk c.
__global__ void stream19_march(const float* __restrict__ a, float* __restrict__ b, size_t ps,
                               int chunks) {
  const size_t first = (size_t)blockIdx.x * chunks * blockDim.x + threadIdx.x;
  float cur[19], nxt[19];
#pragma unroll
  for (int q = 0; q < 19; ++q) cur[q] = a[q * ps + first];
  for (int c = 0; c < chunks; ++c) {
    const size_t i = first + (size_t)c * blockDim.x;
    const size_t j = c + 1 < chunks ? i + blockDim.x : i;
#pragma unroll
    for (int q = 0; q < 19; ++q) nxt[q] = a[q * ps + j];
#pragma unroll
    for (int q = 0; q < 19; ++q) __builtin_nontemporal_store(cur[q] * 1.0001f, &b[q * ps + i]);
#pragma unroll
    for (int q = 0; q < 19; ++q) cur[q] = nxt[q];
  }
}

// ------------------------------------------------- direct global-to-LDS copy
// Each wave loads K float4 per lane straight into its own LDS slice (the LDS
// address of a global_load_lds is the wave-uniform base plus 16 B per lane),
// waits, reads them back and stores them.  Work-group b owns T K float4 as in
// copy_onepass.
template <int K>
__global__ void copy_lds(const v4f* __restrict__ a, v4f* __restrict__ b) {
  extern __shared__ __attribute__((aligned(16))) v4f stage[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const size_t base = (size_t)blockIdx.x * blockDim.x * K + threadIdx.x;
  v4f* mine = stage + (size_t)wave * 64 * K;
#pragma unroll
  for (int k = 0; k < K; ++k)
    __builtin_amdgcn_global_load_lds((const void*)&a[base + (size_t)k * blockDim.x],
                                     (__attribute__((address_space(3))) void*)(mine + k * 64), 16,
                                     0, 0);
  __builtin_amdgcn_s_waitcnt(0);  // vmcnt(0): every load of this wave has landed
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int k = 0; k < K; ++k)
    __builtin_nontemporal_store(mine[k * 64 + lane], &b[base + (size_t)k * blockDim.x]);
}

// ------------------------------------------------------------ pull pattern
// The step's HBM pattern without its stencil, collision or halo: a box of
// nx x ny x nz nodes (nx = 256 here), work-group of 1024 threads owning a
// tile of 4 whole rows and marching zc planes; per plane each thread pulls
// the 19 populations of its node from the neighbours x - c_a (periodic), keeps
// them in registers for one plane, and stores the previous plane's 19 values
// at its own node (non-temporal).  Two population layouts:
//   soa    population a of node i at a * ps + i (19 arrays);
//   blkB   blocks of B consecutive nodes, the block's 19 populations
//          contiguous: ((i / B) * 19 + a) * B + i mod B (B = 64 ... 4096).
__device__ constexpr int PCX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ constexpr int PCY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int PCZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

// B = 0: the 19-array layout; B > 0: blocks of B consecutive nodes.
template <int B>
__device__ inline size_t paddr(int a, unsigned i, size_t ps) {
  if (B > 0) return ((size_t)(i / B) * 19 + a) * B + (i % B);
  return (size_t)a * ps + i;
}

// MASK switches the three shifts on (bit 0: x, bit 1: y, bit 2: z); a shift
// that is off reads the centre node's row, plane or column instead, which
// shows what each shift costs (7: the step's pattern).
template <int BLK, int MASK = 7>
__global__ void __launch_bounds__(1024)
pull_march(const float* __restrict__ src, float* __restrict__ dst, int nx, int ny, int nz,
           int zc, size_t ps) {
  const int tiles_y = ny / 4;
  const int ty = blockIdx.x % tiles_y, chunk = blockIdx.x / tiles_y;
  const int x = threadIdx.x % nx, y = ty * 4 + threadIdx.x / nx;
  const int z0 = chunk * zc, z1 = z0 + zc;
  const unsigned plane = (unsigned)nx * ny;
  const int xo[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
  const int yo[3] = {(y == 0 ? ny - 1 : y - 1) * nx, y * nx, (y == ny - 1 ? 0 : y + 1) * nx};
  float cur[19], nxt[19];
  auto load = [&](int z, float(&v)[19]) {
    const unsigned zo[3] = {(unsigned)(z == 0 ? nz - 1 : z - 1) * plane, (unsigned)z * plane,
                            (unsigned)(z == nz - 1 ? 0 : z + 1) * plane};
#pragma unroll
    for (int a = 0; a < 19; ++a) {
      const int cx = (MASK & 1) ? PCX[a] : 0, cy = (MASK & 2) ? PCY[a] : 0;
      const int cz = (MASK & 4) ? PCZ[a] : 0;
      const unsigned i = zo[1 - cz] + yo[1 - cy] + xo[1 - cx];
      v[a] = src[paddr<BLK>(a, i, ps)];
    }
  };
  load(z0, cur);
  for (int z = z0; z < z1; ++z) {
    load(z + 1 < nz ? z + 1 : 0, nxt);
    const unsigned i = (unsigned)z * plane + yo[1] + x;
#pragma unroll
    for (int a = 0; a < 19; ++a) __builtin_nontemporal_store(cur[a] * 1.0001f, &dst[paddr<BLK>(a, i, ps)]);
#pragma unroll
    for (int a = 0; a < 19; ++a) cur[a] = nxt[a];
  }
}

// The pull pattern on float64 populations (blocks of 1024 nodes): tiles of
// BX columns by NT / BX rows, as the float64 step uses (64 x 4 tiles of 256
// threads by default), each thread pulling the 19 values of its node.
template <int NT, int BX>
__global__ void __launch_bounds__(NT)
pull_march64(const double* __restrict__ src, double* __restrict__ dst, int nx, int ny, int nz,
             int zc) {
  constexpr int BY = NT / BX;
  const int ntx = nx / BX, nty = ny / BY;
  const int tile = blockIdx.x % (ntx * nty), chunk = blockIdx.x / (ntx * nty);
  const int x = (tile % ntx) * BX + (int)threadIdx.x % BX;
  const int y = (tile / ntx) * BY + (int)threadIdx.x / BX;
  const int z0 = chunk * zc, z1 = z0 + zc;
  const unsigned plane = (unsigned)nx * ny;
  const int xo[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
  const int yo[3] = {(y == 0 ? ny - 1 : y - 1) * nx, y * nx, (y == ny - 1 ? 0 : y + 1) * nx};
  double cur[19], nxt[19];
  auto load = [&](int z, double(&v)[19]) {
    const unsigned zo[3] = {(unsigned)(z == 0 ? nz - 1 : z - 1) * plane, (unsigned)z * plane,
                            (unsigned)(z == nz - 1 ? 0 : z + 1) * plane};
#pragma unroll
    for (int a = 0; a < 19; ++a) {
      const unsigned i = zo[1 - PCZ[a]] + yo[1 - PCY[a]] + xo[1 - PCX[a]];
      v[a] = src[paddr<1024>(a, i, 0)];
    }
  };
  load(z0, cur);
  for (int z = z0; z < z1; ++z) {
    load(z + 1 < nz ? z + 1 : 0, nxt);
    const unsigned i = (unsigned)z * plane + yo[1] + x;
#pragma unroll
    for (int a = 0; a < 19; ++a)
      __builtin_nontemporal_store(cur[a] * 1.0001, &dst[paddr<1024>(a, i, 0)]);
#pragma unroll
    for (int a = 0; a < 19; ++a) cur[a] = nxt[a];
  }
}

// The pull pattern in blocks of 1024 nodes (one 256 x 4 tile-plane each)
// with the blocks in node order (TM = 0: block b = z * 64 + tile row) or in
// tile-major order (TM = 1: block (tile row) * nz + z), so that a work-group's
// march through the planes reads and writes one contiguous run of memory.
template <int TM>
__device__ inline size_t oaddr(int a, unsigned i, unsigned bpp, unsigned nz) {
  unsigned b = i / 1024;
  if (TM) b = (b % bpp) * nz + b / bpp;
  return ((size_t)b * 19 + a) * 1024 + (i % 1024);
}

template <int TM>
__global__ void __launch_bounds__(1024)
pull_order(const float* __restrict__ src, float* __restrict__ dst, int nx, int ny, int nz,
           int zc) {
  const int tiles_y = ny / 4;
  const int ty = blockIdx.x % tiles_y, chunk = blockIdx.x / tiles_y;
  const int x = threadIdx.x % nx, y = ty * 4 + threadIdx.x / nx;
  const int z0 = chunk * zc, z1 = z0 + zc;
  const unsigned plane = (unsigned)nx * ny, bpp = plane / 1024;
  const int xo[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
  const int yo[3] = {(y == 0 ? ny - 1 : y - 1) * nx, y * nx, (y == ny - 1 ? 0 : y + 1) * nx};
  float cur[19], nxt[19];
  auto load = [&](int z, float(&v)[19]) {
    const unsigned zo[3] = {(unsigned)(z == 0 ? nz - 1 : z - 1) * plane, (unsigned)z * plane,
                            (unsigned)(z == nz - 1 ? 0 : z + 1) * plane};
#pragma unroll
    for (int a = 0; a < 19; ++a) {
      const unsigned i = zo[1 - PCZ[a]] + yo[1 - PCY[a]] + xo[1 - PCX[a]];
      v[a] = src[oaddr<TM>(a, i, bpp, (unsigned)nz)];
    }
  };
  load(z0, cur);
  for (int z = z0; z < z1; ++z) {
    load(z + 1 < nz ? z + 1 : 0, nxt);
    const unsigned i = (unsigned)z * plane + yo[1] + x;
#pragma unroll
    for (int a = 0; a < 19; ++a)
      __builtin_nontemporal_store(cur[a] * 1.0001f, &dst[oaddr<TM>(a, i, bpp, (unsigned)nz)]);
#pragma unroll
    for (int a = 0; a < 19; ++a) cur[a] = nxt[a];
  }
}

// The pull pattern (all three shifts) with every load aligned to the
// node's own column: a population with c_x = +1 takes the value of the lane
// to its left by a DPP wave shift (wave_shr:1), c_x = -1 that of the lane to
// its right (wave_shl:1), and the one lane at the wave's edge loads its value
// itself.  Each wave covers 64 consecutive nodes of one row (nx = 256).
// The lane whose source lies outside the wave (lane 0 for wave_shr, lane 63
// for wave_shl) keeps `old`: with bound_ctrl off, DPP does not write it.
__device__ inline float lane_from_left(float v, float old) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                               __builtin_bit_cast(int, v),
                                                               0x138, 0xF, 0xF, false));
}
__device__ inline float lane_from_right(float v, float old) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                               __builtin_bit_cast(int, v),
                                                               0x130, 0xF, 0xF, false));
}

template <int BLK>
__global__ void __launch_bounds__(1024)
pull_dpp(const float* __restrict__ src, float* __restrict__ dst, int nx, int ny, int nz, int zc,
         size_t ps) {
  const int tiles_y = ny / 4;
  const int ty = blockIdx.x % tiles_y, chunk = blockIdx.x / tiles_y;
  const int x = threadIdx.x % nx, y = ty * 4 + threadIdx.x / nx;
  const int lane = threadIdx.x & 63;
  const int z0 = chunk * zc, z1 = z0 + zc;
  const unsigned plane = (unsigned)nx * ny;
  // The wave's first and last column and their outer neighbours (periodic).
  const int xf = x - lane, xl = xf + 63;
  const int left = xf == 0 ? nx - 1 : xf - 1, right = xl == nx - 1 ? 0 : xl + 1;
  const int yo[3] = {(y == 0 ? ny - 1 : y - 1) * nx, y * nx, (y == ny - 1 ? 0 : y + 1) * nx};
  float cur[19], nxt[19], edge[19];
  // Issues the plane's aligned loads and the wave-edge loads; the lane
  // shifts are applied by fix() once the values have arrived.
  auto load = [&](int z) {
    const unsigned zo[3] = {(unsigned)(z == 0 ? nz - 1 : z - 1) * plane, (unsigned)z * plane,
                            (unsigned)(z == nz - 1 ? 0 : z + 1) * plane};
#pragma unroll
    for (int a = 0; a < 19; ++a) {
      const unsigned row = zo[1 - PCZ[a]] + yo[1 - PCY[a]];
      nxt[a] = src[paddr<BLK>(a, row + x, ps)];
      if (PCX[a] != 0) {
        const unsigned e = __builtin_amdgcn_readfirstlane(row + (PCX[a] > 0 ? left : right));
        edge[a] = src[paddr<BLK>(a, e, ps)];
      }
    }
  };
  auto fix = [&]() {
#pragma unroll
    for (int a = 0; a < 19; ++a) {
      if (PCX[a] > 0) nxt[a] = lane_from_left(nxt[a], edge[a]);
      if (PCX[a] < 0) nxt[a] = lane_from_right(nxt[a], edge[a]);
    }
  };
  load(z0);
  fix();
  for (int z = z0; z < z1; ++z) {
#pragma unroll
    for (int a = 0; a < 19; ++a) cur[a] = nxt[a];
    load(z + 1 < nz ? z + 1 : 0);
    const unsigned i = (unsigned)z * plane + yo[1] + x;
#pragma unroll
    for (int a = 0; a < 19; ++a) __builtin_nontemporal_store(cur[a] * 1.0001f, &dst[paddr<BLK>(a, i, ps)]);
    fix();
  }
}

// The pull pattern with W consecutive nodes of a row per lane (blocks of
// 1024 nodes, nx = 256): 19 loads of W values (8 or 16 bytes; the x-shifted
// ones start one node off, at 4-byte alignment) and 19 aligned stores of W
// values per lane and plane.  Bandwidth only: a vector that would wrap
// around the row is clamped into it, so the values at the row's ends are not
// the periodic ones.
template <int W, int NT>
__global__ void __launch_bounds__(NT)
pull_wide(const float* __restrict__ src, float* __restrict__ dst, int nx, int ny, int nz,
          int zc) {
  typedef float vw __attribute__((ext_vector_type(W)));
  const int rows = NT * W / nx;
  const int tiles_y = ny / rows;
  const int ty = blockIdx.x % tiles_y, chunk = blockIdx.x / tiles_y;
  const int x = (threadIdx.x * W) % nx, y = ty * rows + (threadIdx.x * W) / nx;
  const int z0 = chunk * zc, z1 = z0 + zc;
  const unsigned plane = (unsigned)nx * ny;
  const int yo[3] = {(y == 0 ? ny - 1 : y - 1) * nx, y * nx, (y == ny - 1 ? 0 : y + 1) * nx};
  vw cur[19], nxt[19];
  auto load = [&](int z, vw(&v)[19]) {
    const unsigned zo[3] = {(unsigned)(z == 0 ? nz - 1 : z - 1) * plane, (unsigned)z * plane,
                            (unsigned)(z == nz - 1 ? 0 : z + 1) * plane};
#pragma unroll
    for (int a = 0; a < 19; ++a) {
      const int xs = min(max(x - PCX[a], 0), nx - W);
      const unsigned i = zo[1 - PCZ[a]] + yo[1 - PCY[a]] + xs;
      __builtin_memcpy(&v[a], src + paddr<1024>(a, i, 0), sizeof(vw));
    }
  };
  load(z0, cur);
  for (int z = z0; z < z1; ++z) {
    load(z + 1 < nz ? z + 1 : 0, nxt);
    const unsigned i = (unsigned)z * plane + yo[1] + x;
#pragma unroll
    for (int a = 0; a < 19; ++a)
      __builtin_nontemporal_store(cur[a] * 1.0001f,
                                  reinterpret_cast<vw*>(dst + paddr<1024>(a, i, 0)));
#pragma unroll
    for (int a = 0; a < 19; ++a) cur[a] = nxt[a];
  }
}

__global__ void fill_pattern(float* __restrict__ a, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    a[i] = (float)((unsigned)(i * 2654435761u) >> 8) * 1e-6f;
}

__global__ void count_diff(const float* __restrict__ p, const float* __restrict__ q, size_t n,
                           unsigned* __restrict__ bad) {
  unsigned k = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    k += __float_as_uint(p[i]) != __float_as_uint(q[i]);
  if (k) atomicAdd(bad, k);
}

// The pull pattern with the loads done by gfx950's direct global-to-LDS
// loads, 16 bytes per lane (blocks of 1024 nodes, nx = ny = 256, tiles of 4
// rows, so one tile-plane is one block).  Per plane, for each population a
// and each of the tile's 4 rows, one wave copies the 1 KiB source row
// (row y - c_ay of plane z - c_az, unshifted in x) into LDS; after a barrier
// each thread reads its 19 pulled values (the x shift applied in LDS, with
// the periodic wrap) into registers.  The next plane's copies are issued
// before the current plane's stores.  OUT = 0: each thread stores its 19
// values (4 bytes per lane); OUT = 1: the values pass through LDS and leave
// as 16-byte stores.
__device__ constexpr int kRowsA[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int kPlaneA[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

template <int OUT>
__global__ void __launch_bounds__(1024)
pull_lds(const float* __restrict__ src, float* __restrict__ dst, int nz, int zc) {
  constexpr int NX = 256, NY = 256, B = 1024;
  extern __shared__ __attribute__((aligned(16))) float lds[];
  float* in = lds;              // [19][4][256]
  float* out = lds + 19 * B;    // [19][1024] (OUT = 1)
  const int ty = blockIdx.x % (NY / 4), chunk = blockIdx.x / (NY / 4);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int x = threadIdx.x & (NX - 1), yl = threadIdx.x >> 8;
  const int z0 = chunk * zc, z1 = z0 + zc;
  auto issue = [&](int z) {
    for (int p = wave; p < 19 * 4; p += 16) {
      const int a = p >> 2, r = p & 3;
      const int sy = (ty * 4 - kRowsA[a] + r + NY) % NY;
      const int sz = (z - kPlaneA[a] + nz) % nz;
      const unsigned node = ((unsigned)sz * NY + sy) * NX;
      const size_t base = ((size_t)(node / B) * 19 + a) * B + node % B;
      __builtin_amdgcn_global_load_lds((const void*)(src + base + lane * 4),
                                       (__attribute__((address_space(3))) void*)(in + p * NX), 16,
                                       0, 0);
    }
  };
  float cur[19];
  auto take = [&]() {
#pragma unroll
    for (int a = 0; a < 19; ++a) cur[a] = in[(a * 4 + yl) * NX + ((x - PCX[a]) & (NX - 1))];
  };
  issue(z0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  take();
  __syncthreads();
  for (int z = z0; z < z1; ++z) {
    if (z + 1 < z1) issue(z + 1);
    const size_t blk = ((size_t)z * (NY / 4) + ty) * 19 * B;
    if (OUT == 0) {
#pragma unroll
      for (int a = 0; a < 19; ++a)
        __builtin_nontemporal_store(cur[a] * 1.0001f, &dst[blk + a * B + threadIdx.x]);
    } else {
#pragma unroll
      for (int a = 0; a < 19; ++a) out[a * B + threadIdx.x] = cur[a] * 1.0001f;
      __syncthreads();
      const v4f* o4 = reinterpret_cast<const v4f*>(out);
      v4f* d4 = reinterpret_cast<v4f*>(dst + blk);
      for (int f = threadIdx.x; f < 19 * B / 4; f += 1024) __builtin_nontemporal_store(o4[f], &d4[f]);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (z + 1 < z1) take();
    __syncthreads();
  }
}

// 19-array stream with 4 consecutive nodes per lane (16-byte loads and
// stores), one pass: the access width of the copy kernels in the step's
// 19-stream shape.
__global__ void stream19x4_onepass(const v4f* __restrict__ a, v4f* __restrict__ b, size_t ps4) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  v4f v[19];
#pragma unroll
  for (int q = 0; q < 19; ++q) v[q] = a[q * ps4 + i];
#pragma unroll
  for (int q = 0; q < 19; ++q) __builtin_nontemporal_store(v[q] * 1.0001f, &b[q * ps4 + i]);
}

int main(int argc, char** argv) {
  const char* fam = argc > 1 ? argv[1] : "all";
  auto want = [&](const char* f) { return !std::strcmp(fam, "all") || !std::strcmp(fam, f); };
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
  auto run = [&](const char* name, int threads, int grid, double traffic, auto launch) -> int {
    launch();
    CK(hipGetLastError());
    CK(hipDeviceSynchronize());
    CK(hipEventRecord(e0));
    for (int r = 0; r < 10; ++r) launch();
    CK(hipEventRecord(e1));
    CK(hipEventSynchronize(e1));
    float ms;
    CK(hipEventElapsedTime(&ms, e0, e1));
    ms /= 10;
    std::printf("%-16s threads %5d grid %8d  %8.3f ms  %8.1f GB/s\n", name, threads, grid, ms,
                traffic / ms / 1e6);
    std::fflush(stdout);
    return 0;
  };
  if (want("gridstride")) {
    for (int t : {256, 512, 1024}) {
      for (int grid : {1024, 2048, 4096, 16384, 65536}) {
        if (run("copy4", t, grid, 2.0 * bytes,
                [&] { copy4<<<grid, t>>>((float4*)a, (float4*)b, n4); }))
          return 1;
        if (run("copy4_nt", t, grid, 2.0 * bytes,
                [&] { copy4_nt<<<grid, t>>>((v4f*)a, (v4f*)b, n4); }))
          return 1;
        if (run("copy4_ntld", t, grid, 2.0 * bytes,
                [&] { copy4_ntld<<<grid, t>>>((v4f*)a, (v4f*)b, n4); }))
          return 1;
        if (run("copy4_u4", t, grid, 2.0 * bytes,
                [&] { copy4_u4<<<grid, t>>>((v4f*)a, (v4f*)b, n4); }))
          return 1;
        if (run("copy1", t, grid, 2.0 * bytes, [&] { copy1<<<grid, t>>>(a, b, n1); })) return 1;
        if (run("read4", t, grid, 1.0 * bytes,
                [&] { read4<<<grid, t>>>((float4*)a, o, n4); }))
          return 1;
        if (run("write4", t, grid, 1.0 * bytes, [&] { write4<<<grid, t>>>((float4*)b, n4); }))
          return 1;
      }
    }
  }
  if (want("onepass")) {
    // n4 = 2^28 is a multiple of every T K below.
    for (int t : {256, 512, 1024}) {
      auto one = [&](auto kc) -> int {
        constexpr int K = decltype(kc)::value;
        const int grid = (int)(n4 / ((size_t)t * K));
        char name[32];
        std::snprintf(name, sizeof(name), "copy_1p_k%d", K);
        if (run(name, t, grid, 2.0 * bytes,
                [&] { copy_onepass<K, false><<<grid, t>>>((v4f*)a, (v4f*)b); }))
          return 1;
        std::snprintf(name, sizeof(name), "copy_1p_nt_k%d", K);
        if (run(name, t, grid, 2.0 * bytes,
                [&] { copy_onepass<K, true><<<grid, t>>>((v4f*)a, (v4f*)b); }))
          return 1;
        std::snprintf(name, sizeof(name), "read_1p_k%d", K);
        if (run(name, t, grid, 1.0 * bytes, [&] { read_onepass<K><<<grid, t>>>((v4f*)a, o); }))
          return 1;
        std::snprintf(name, sizeof(name), "write_1p_k%d", K);
        if (run(name, t, grid, 1.0 * bytes, [&] { write_onepass<K><<<grid, t>>>((v4f*)b); }))
          return 1;
        return 0;
      };
      if (one(std::integral_constant<int, 1>{}) || one(std::integral_constant<int, 2>{}) ||
          one(std::integral_constant<int, 4>{}) || one(std::integral_constant<int, 8>{}))
        return 1;
    }
  }
  if (want("stream")) {
    // n19 = 2^25 nodes: a multiple of every work-group size and chunk count.
    for (int t : {256, 512, 1024}) {
      const int grid = (int)(n19 / t);
      if (run("stream19_1p", t, grid, 2.0 * 19 * n19 * 4,
              [&] { stream19_onepass<<<grid, t>>>(a, b, ps19); }))
        return 1;
      for (int chunks : {4, 16, 64, 256}) {
        const int g = (int)(n19 / ((size_t)t * chunks));
        char name[32];
        std::snprintf(name, sizeof(name), "stream19_m%d", chunks);
        if (run(name, t, g, 2.0 * 19 * n19 * 4,
                [&] { stream19_march<<<g, t>>>(a, b, ps19, chunks); }))
          return 1;
      }
    }
  }
  if (want("lds")) {
    for (int t : {256, 512, 1024}) {
      auto one = [&](auto kc) -> int {
        constexpr int K = decltype(kc)::value;
        const int grid = (int)(n4 / ((size_t)t * K));
        const size_t lds = (size_t)t * K * 16;
        if (lds > 64 * 1024) return 0;  // within the default dynamic LDS limit
        char name[32];
        std::snprintf(name, sizeof(name), "copy_lds_k%d", K);
        return run(name, t, grid, 2.0 * bytes,
                   [&] { copy_lds<K><<<grid, t, lds>>>((v4f*)a, (v4f*)b); });
      };
      if (one(std::integral_constant<int, 1>{}) || one(std::integral_constant<int, 2>{}) ||
          one(std::integral_constant<int, 4>{}) || one(std::integral_constant<int, 8>{}))
        return 1;
    }
  }
  if (want("pull")) {
    // 256 x 256 x 512 box: 33.5 M nodes, 19 x 4 B x n = 2.55 GB per lattice.
    const int nx = 256, ny = 256, nz = 512;
    const size_t n = (size_t)nx * ny * nz, ps = n + 1088;
    for (int zc : {128, 8}) {
      const int grid = (ny / 4) * (nz / zc);
      auto one = [&](auto bc) -> int {
        constexpr int B = decltype(bc)::value;
        char name[32];
        std::snprintf(name, sizeof(name), "pull_blk%d_z%d", B, zc);
        return run(name, 1024, grid, 2.0 * 19 * n * 4,
                   [&] { pull_march<B><<<grid, 1024>>>(a, b, nx, ny, nz, zc, ps); });
      };
      if (one(std::integral_constant<int, 0>{}) || one(std::integral_constant<int, 64>{}) ||
          one(std::integral_constant<int, 256>{}) || one(std::integral_constant<int, 1024>{}) ||
          one(std::integral_constant<int, 4096>{}))
        return 1;
    }
  }
  if (want("shift")) {
    // The pull pattern in blocks of 1024 nodes with shifts switched off, and
    // with the x shift taken across lanes; first, that the lane-shift form
    // stores exactly what the plain form stores.
    const int nx = 256, ny = 256, nz = 512;
    const size_t n = (size_t)nx * ny * nz, ps = n, L = 19 * n;
    float* c;
    CK(hipMalloc(&c, L * 4));
    fill_pattern<<<65536, 256>>>(a, L);
    const int g8 = (ny / 4) * (nz / 8);
    pull_march<1024, 7><<<g8, 1024>>>(a, c, nx, ny, nz, 8, ps);
    pull_dpp<1024><<<g8, 1024>>>(a, b, nx, ny, nz, 8, ps);
    CK(hipMemset(o, 0, 64));
    count_diff<<<65536, 256>>>(b, c, L, (unsigned*)o);
    CK(hipGetLastError());
    unsigned bad = 0;
    CK(hipMemcpy(&bad, o, 4, hipMemcpyDeviceToHost));
    std::printf("pull_dpp against pull_march: %u of %zu stored values differ\n", bad, L);
    std::fflush(stdout);
    CK(hipFree(c));
    for (int zc : {128, 8}) {
      const int grid = (ny / 4) * (nz / zc);
      const double traffic = 2.0 * 19 * n * 4;
      auto one = [&](auto mc) -> int {
        constexpr int M = decltype(mc)::value;
        char name[32];
        std::snprintf(name, sizeof(name), "pull_mask%d_z%d", M, zc);
        return run(name, 1024, grid, traffic,
                   [&] { pull_march<1024, M><<<grid, 1024>>>(a, b, nx, ny, nz, zc, ps); });
      };
      if (one(std::integral_constant<int, 7>{}) || one(std::integral_constant<int, 6>{}) ||
          one(std::integral_constant<int, 5>{}) || one(std::integral_constant<int, 3>{}) ||
          one(std::integral_constant<int, 1>{}) || one(std::integral_constant<int, 0>{}))
        return 1;
      char name[32];
      std::snprintf(name, sizeof(name), "pull_dpp_z%d", zc);
      if (run(name, 1024, grid, traffic,
              [&] { pull_dpp<1024><<<grid, 1024>>>(a, b, nx, ny, nz, zc, ps); }))
        return 1;
    }
  }
  if (want("wide")) {
    // The pull pattern with 2 or 4 nodes per lane against 1 (same box).
    const int nx = 256, ny = 256, nz = 512;
    const size_t n = (size_t)nx * ny * nz;
    const double traffic = 2.0 * 19 * n * 4;
    for (int zc : {128, 8}) {
      char name[40];
      {
        const int grid = (ny / 4) * (nz / zc);
        std::snprintf(name, sizeof(name), "pull_w1_t1024_z%d", zc);
        if (run(name, 1024, grid, traffic,
                [&] { pull_march<1024, 7><<<grid, 1024>>>(a, b, nx, ny, nz, zc, n); }))
          return 1;
      }
      auto one = [&](auto wc, auto tc) -> int {
        constexpr int W = decltype(wc)::value, T = decltype(tc)::value;
        const int rows = T * W / nx;
        const int grid = (ny / rows) * (nz / zc);
        std::snprintf(name, sizeof(name), "pull_w%d_t%d_z%d", W, T, zc);
        return run(name, T, grid, traffic,
                   [&] { pull_wide<W, T><<<grid, T>>>(a, b, nx, ny, nz, zc); });
      };
      if (one(std::integral_constant<int, 2>{}, std::integral_constant<int, 1024>{}) ||
          one(std::integral_constant<int, 2>{}, std::integral_constant<int, 512>{}) ||
          one(std::integral_constant<int, 2>{}, std::integral_constant<int, 256>{}) ||
          one(std::integral_constant<int, 4>{}, std::integral_constant<int, 512>{}) ||
          one(std::integral_constant<int, 4>{}, std::integral_constant<int, 256>{}))
        return 1;
    }
  }
  if (want("order")) {
    // Node-ordered against tile-major blocks (same box as the pull family).
    const int nx = 256, ny = 256, nz = 512;
    const size_t n = (size_t)nx * ny * nz;
    const double traffic = 2.0 * 19 * n * 4;
    for (int zc : {128, 32, 8}) {
      const int grid = (ny / 4) * (nz / zc);
      char name[32];
      std::snprintf(name, sizeof(name), "pull_node_z%d", zc);
      if (run(name, 1024, grid, traffic,
              [&] { pull_order<0><<<grid, 1024>>>(a, b, nx, ny, nz, zc); }))
        return 1;
      std::snprintf(name, sizeof(name), "pull_tile_z%d", zc);
      if (run(name, 1024, grid, traffic,
              [&] { pull_order<1><<<grid, 1024>>>(a, b, nx, ny, nz, zc); }))
        return 1;
    }
  }
  if (want("pull64")) {
    // float64 populations: 256 x 256 x 256 box, 19 x 8 B x n = 2.55 GB.
    const int nx = 256, ny = 256, nz = 256;
    const size_t n = (size_t)nx * ny * nz;
    const double traffic = 2.0 * 19 * n * 8;
    double* a8 = reinterpret_cast<double*>(a);
    double* b8 = reinterpret_cast<double*>(b);
    for (int zc : {64, 16, 4}) {
      char name[40];
      auto one = [&](auto tc, auto bc) -> int {
        constexpr int T = decltype(tc)::value, BX = decltype(bc)::value;
        const int grid = (nx / BX) * (ny / (T / BX)) * (nz / zc);
        std::snprintf(name, sizeof(name), "pull64_t%d_%dx%d_z%d", T, BX, T / BX, zc);
        return run(name, T, grid, traffic,
                   [&] { pull_march64<T, BX><<<grid, T>>>(a8, b8, nx, ny, nz, zc); });
      };
      using I256 = std::integral_constant<int, 256>;
      using I512 = std::integral_constant<int, 512>;
      using I1024 = std::integral_constant<int, 1024>;
      using I64 = std::integral_constant<int, 64>;
      using I128 = std::integral_constant<int, 128>;
      if (one(I256{}, I64{}) || one(I256{}, I256{}) || one(I512{}, I128{}) ||
          one(I512{}, I256{}) || one(I1024{}, I256{}))
        return 1;
    }
  }
  if (want("lds19")) {
    // More than 64 KiB of dynamic LDS per work-group must be allowed first.
    CK(hipFuncSetAttribute(reinterpret_cast<const void*>(&pull_lds<0>),
                           hipFuncAttributeMaxDynamicSharedMemorySize, 19 * 1024 * 4));
    CK(hipFuncSetAttribute(reinterpret_cast<const void*>(&pull_lds<1>),
                           hipFuncAttributeMaxDynamicSharedMemorySize, 2 * 19 * 1024 * 4));
    const int nz = 512;
    const size_t n = (size_t)256 * 256 * nz;
    for (int zc : {128, 8}) {
      const int grid = 64 * (nz / zc);
      char name[32];
      std::snprintf(name, sizeof(name), "pull_lds_out0_z%d", zc);
      if (run(name, 1024, grid, 2.0 * 19 * n * 4,
              [&] { pull_lds<0><<<grid, 1024, 19 * 1024 * 4>>>(a, b, nz, zc); }))
        return 1;
      std::snprintf(name, sizeof(name), "pull_lds_out1_z%d", zc);
      if (run(name, 1024, grid, 2.0 * 19 * n * 4,
              [&] { pull_lds<1><<<grid, 1024, 2 * 19 * 1024 * 4>>>(a, b, nz, zc); }))
        return 1;
    }
    // 2^23 lanes of 4 nodes: the same 2^25 nodes as the float stream.
    const size_t n4 = n19 / 4, ps4 = n4 + 272;
    for (int t : {256, 1024}) {
      const int grid = (int)(n4 / t);
      if (run("stream19x4_1p", t, grid, 2.0 * 19 * n19 * 4,
              [&] { stream19x4_onepass<<<grid, t>>>((const v4f*)a, (v4f*)b, ps4); }))
        return 1;
    }
  }
  CK(hipFree(a));
  CK(hipFree(b));
  CK(hipFree(o));
  return 0;
}
