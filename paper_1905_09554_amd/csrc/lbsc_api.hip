// C ABI of the D3Q19 pseudo-potential lattice Boltzmann library (include/lbsc.h).
//
// Validation, the context, the device-memory layout inside the caller's
// buffer, and the order of launches.  All arithmetic of the method runs in the
// kernels of lbsc_device.hip.
//
// A context holds one or more members (boxes).  lbsc_init_fields makes a
// context of one member; lbsc_init_batch makes several, stepped together by
// one launch per step (or one cooperative launch for all steps).
//
// Caller buffer layout:
//   [member 0: lattice 0 | lattice 1] [member 1: ...] ... [aux]
//   aux = member table | tile table | barrier words | diagnostic partials |
//         diagnostic results
// With one array per population (a layout block of 0), a single box reserves
// room for a padding of up to kMaxPad between the arrays so its layout can be
// retuned in place, and batch members use the default pad; with populations
// in blocks (the layout of both storage types) there is no padding.
#include "lbsc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbsc_internal.h"

namespace {

struct Member {
  lbsc_params p;
  lbsc::StepArgs a;
  void* lat[2];
  size_t lat_bytes;  // capacity of each lattice
};

// Caller workspace of the adjoint: checkpoints of the forward run, the
// lattices and psi fields of one recomputed segment, the adjoint state.
struct AdjWork {
  bool ready = false;
  int64_t nsteps = 0;
  int32_t segment = 0;
  int ncp = 0;
  size_t lat_bytes = 0, psi_bytes = 0;
  char* cp = nullptr;    // ncp lattices
  char* ring = nullptr;  // segment + 1 lattices
  char* psi = nullptr;   // psi of every step of the segment
  char* P[2] = {nullptr, nullptr};
  char* R[2] = {nullptr, nullptr};
  char* psi_fbar = nullptr;    // 3 n values: psi(x) dL/dF(x)
  char* fbar_dot_v = nullptr;  // n values: dL/dF(x) . sum_b w_b psi(x + c_b) c_b
  double* partial = nullptr;
  double* acc = nullptr;  // dL/dG, dL/dtau, dL/ds_bulk, dL/ds_ghost
  double rates[2] = {0.0, 0.0};  // dL/ds_bulk, dL/ds_ghost of the last backward pass
  bool have_rates = false;
};

}  // namespace

struct lbsc_ctx {
  std::vector<Member> m;
  bool batch;
  int device;                    // HIP device holding the caller's buffer
  lbsc_tuning tune;
  hipStream_t stream;
  char* buf;
  size_t bytes;
  int cur;                       // lattice holding the current state
  lbsc::BatchMember* dmembers;   // device member table
  int4* dtiles;                  // device tile table
  int ntiles;
  long long tile_cap;
  unsigned* dsync;               // grid-barrier words (count, generation, error, 2 tile counters)
  double* part;                  // diagnostic partial sums
  double* dout;                  // diagnostic results: 4 + max nz doubles
  void* psi;                     // psi field of the two-kernel step (single box), or null
  int64_t step;
  AdjWork adj;
  std::string err;
};

namespace {

thread_local std::string g_init_err;

constexpr size_t kAlign = 256;
// Largest padding between population arrays (elements); a single box's
// buffer is sized for it so the layout can be retuned in place.
constexpr long long kMaxPad = 65536;
constexpr long long kDefaultPad = 1088;
// Polls of a grid barrier before it reports a timeout (about a second).
constexpr unsigned kSpinLimit = 1u << 23;
// Narrowest tile that does not span a whole row (one wavefront of columns);
// bounds the size of the tile table.
constexpr int kMinBlockX = 64;

// Device scratch of lbsc_interface_diagnostics_static, for callers that
// cannot allocate: the diagnostic results (4 + nz doubles) and the per-block
// partial sums (8 doubles per block), 16 MiB in all.  Each GPU holds its own
// copy for the life of the process.  Host code never passes `scratch` itself
// to a kernel (on the host it only names the variable): it passes the
// device address that hipGetSymbolAddress returned for the current device,
// resolved once per device when the first context is created there.
constexpr size_t kScratchDoubles = size_t(1) << 21;
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Resolves the scratch address of device `dev` (the current device) once.
hipError_t resolve_scratch(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_scratch_dev[dev] = static_cast<double*>(ptr);
  return e;
}

double* scratch_of(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_dev[dev];
}

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
size_t elem_size(const lbsc_params& p) { return p.precision == LBSC_F64 ? 8 : 4; }
long long nodes(const lbsc_params& p) { return (long long)p.nx * p.ny * p.nz; }
// Block length of the population layout of the storage type (0: one array
// per population, padded by the tuning's pop_pad).
long long layout_block(const lbsc_params& p) {
  return p.precision == LBSC_F64 ? lbsc::Layout<double>::kBlock : lbsc::Layout<float>::kBlock;
}
// Nodes a lattice holds room for: n rounded up to the layout's blocks, or
// to 64 nodes plus the padding between population arrays.
long long lattice_nodes(const lbsc_params& p, long long pad) {
  const long long B = layout_block(p);
  return B > 0 ? (nodes(p) + B - 1) / B * B : (nodes(p) + 63) / 64 * 64 + pad;
}

int fail(std::string* where, int code, const std::string& msg) {
  if (where) *where = msg;
  return code;
}

// Checks a parameter set; returns LBSC_OK or LBSC_EINVAL with a message.
int check_params(const lbsc_params* p, std::string* msg) {
  if (!p) return fail(msg, LBSC_EINVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1)
    return fail(msg, LBSC_EINVAL, "box dimensions must be >= 1");
  if (nodes(*p) > 0x7fffffffLL) return fail(msg, LBSC_EINVAL, "more than 2^31 - 1 nodes");
  if (p->collision != LBSC_BGK && p->collision != LBSC_MRT)
    return fail(msg, LBSC_EINVAL, "collision must be LBSC_BGK or LBSC_MRT");
  if (p->forcing != LBSC_FORCING_GUO && p->forcing != LBSC_FORCING_SHIFT)
    return fail(msg, LBSC_EINVAL, "forcing must be LBSC_FORCING_GUO or LBSC_FORCING_SHIFT");
  if (p->forcing == LBSC_FORCING_SHIFT && p->collision != LBSC_BGK)
    return fail(msg, LBSC_EINVAL, "velocity-shift forcing is defined for BGK only");
  if (p->precision != LBSC_F64 && p->precision != LBSC_F32_SHIFTED)
    return fail(msg, LBSC_EINVAL, "precision must be LBSC_F64 or LBSC_F32_SHIFTED");
  if (!std::isfinite(p->G)) return fail(msg, LBSC_EINVAL, "G must be finite");
  if (!(std::isfinite(p->psi_rho0) && p->psi_rho0 > 0))
    return fail(msg, LBSC_EINVAL, "psi_rho0 must be finite and > 0");
  if (!(std::isfinite(p->tau) && p->tau > 0.5))
    return fail(msg, LBSC_EINVAL, "tau must be finite and > 0.5");
  if (p->collision == LBSC_MRT) {
    if (!(p->s_bulk > 0 && p->s_bulk < 2)) return fail(msg, LBSC_EINVAL, "s_bulk must be in (0, 2)");
    if (!(p->s_ghost > 0 && p->s_ghost < 2))
      return fail(msg, LBSC_EINVAL, "s_ghost must be in (0, 2)");
  }
  if (p->precision == LBSC_F32_SHIFTED && !std::isfinite(p->rho_ref))
    return fail(msg, LBSC_EINVAL, "rho_ref must be finite");
  return LBSC_OK;
}

// Checks a batch: every member valid, one kernel family for all.
int check_batch(int32_t n, const lbsc_params* p, std::string* msg) {
  if (n < 1) return fail(msg, LBSC_EINVAL, "batch size must be >= 1");
  if (!p) return fail(msg, LBSC_EINVAL, "params is NULL");
  for (int32_t i = 0; i < n; ++i) {
    std::string m;
    if (check_params(&p[i], &m) != LBSC_OK)
      return fail(msg, LBSC_EINVAL, "member " + std::to_string(i) + ": " + m);
    if (p[i].precision != p[0].precision || p[i].collision != p[0].collision ||
        p[i].forcing != p[0].forcing)
      return fail(msg, LBSC_EINVAL,
                  "member " + std::to_string(i) + ": precision, collision and forcing must match");
  }
  return LBSC_OK;
}

// Tile of the fused step: bx columns by by rows, at most cap = npt * threads
// nodes.  Each plane of the z-march also reloads the tile's halo ring, one
// node per thread; a ring larger than the work-group costs a second round of
// dependent loads.  Default bx: whole rows when the group holds at least
// min_rows of them and their two halo rows fit one round (2 nx <= threads);
// else the widest multiple of 64 columns whose ring, 2 (bx + 2) + 2 by, fits
// one round with by = cap / bx >= min_rows; else the same with two rows.
// float64 tiles, 1024-thread groups and rows wider than half the group
// want four rows (measured: 64 x 4 beats whole rows two deep at 256
// threads; on rows of 384-672 nodes 128 x 4 tiles of 512 threads reach
// 25.2-28.4 GLUPS, 192 x 2 tiles 22.1 on 672), other float32 tiles two.
// Four psi planes of (by + 2)(bx + 2) values must fit the 160 KB of LDS of a
// CU.
int default_block_x(int nx, long long cap, int threads, int min_rows) {
  for (int rows = min_rows; rows >= 2; rows /= 2) {
    if ((long long)rows * nx <= cap && 2LL * nx <= threads) return nx;
    for (long long bx = std::min<long long>(nx, cap / rows) / 64 * 64; bx >= 64; bx -= 64)
      if (2 * (bx + 2) + 2 * (cap / bx) <= threads) return (int)bx;
  }
  return std::min<int>(nx, 64);
}

void tile_shape(int nx, int ny, long long cap, int threads, int block_x, int block_y, size_t elem,
                int* bx_out, int* by_out) {
  const int min_rows = (elem == 8 || threads >= 1024 || 2LL * nx > cap) ? 4 : 2;
  int bx = block_x > 0 ? block_x : default_block_x(nx, cap, threads, min_rows);
  if (bx > nx) bx = nx;
  if (bx > cap) bx = (int)cap;
  const int rows = (int)std::max(1LL, cap / bx);
  int by = block_y > 0 ? block_y : rows;
  if (by > rows) by = rows;
  if (by < 1) by = 1;
  if (by > ny) by = ny;
  while (by > 1 && 4LL * (by + 2) * (bx + 2) * (long long)elem > 160 * 1024) --by;
  *bx_out = bx;
  *by_out = by;
}

lbsc::StepArgs make_args(const lbsc_params& p, const lbsc_tuning& t, long long pad) {
  lbsc::StepArgs a;
  a.nx = p.nx;
  a.ny = p.ny;
  a.nz = p.nz;
  a.plane = p.nx * p.ny;
  a.n = nodes(p);
  a.ps = lattice_nodes(p, pad);
  tile_shape(p.nx, p.ny, (long long)t.nodes_per_thread * t.threads, t.threads, t.block_x,
             t.block_y, elem_size(p), &a.bx, &a.by);
  a.ntiles_x = (p.nx + a.bx - 1) / a.bx;
  a.ntiles_y = (p.ny + a.by - 1) / a.by;
  a.zchunk = t.z_chunk > 0 ? (t.z_chunk > p.nz ? p.nz : t.z_chunk) : p.nz;
  a.xcd_remap = t.xcd_remap;
  a.G = p.G;
  a.psi_rho0 = p.psi_rho0;
  a.tau = p.tau;
  a.omega = 1.0 / p.tau;
  a.s_bulk = p.s_bulk;
  a.s_ghost = p.s_ghost;
  a.rho_ref = p.precision == LBSC_F64 ? 0.0 : p.rho_ref;
  a.psi_out = nullptr;
  return a;
}

long long pad_of(const lbsc_tuning& t) { return t.pop_pad >= 0 ? t.pop_pad : kDefaultPad; }

// xy tiles times planes over all members: the number of work-groups with
// one-plane chunks.
long long tile_columns(const lbsc_params* p, int32_t n, int threads) {
  long long columns = 0;
  for (int32_t i = 0; i < n; ++i) {
    int bx = 1, by = 1;
    tile_shape(p[i].nx, p[i].ny, threads, threads, 0, 0, elem_size(p[i]), &bx, &by);
    columns += (long long)((p[i].nx + bx - 1) / bx) * ((p[i].ny + by - 1) / by) * p[i].nz;
  }
  return columns;
}

// Default chunk length and tile order for work-groups of t->threads.
void chunk_and_order(const lbsc_params* p, int32_t n, lbsc_tuning* t) {
  // Chunk length.  A single box on 1024-thread groups: one wave of 256 groups,
  // one per CU (no tail), up to 256 planes.  Otherwise about 512 groups of 1
  // to 64 planes: long marches keep the two extra halo planes of each chunk a
  // small fraction on large boxes, short ones give small boxes enough groups.
  const long long columns = tile_columns(p, n, t->threads);
  const bool one_wave = t->threads == 1024 && n == 1;
  const long long groups = one_wave ? 256 : 512;
  // Batches: chunks of at most 8 planes (the 64-ligament sweep: 13.87 ms per
  // step against 14.24 with 64-plane chunks, about 50 000 short-lived groups
  // whose tail wave is a small fraction of the step; with the populations in
  // blocks the batch autotuner finds 32-plane chunks a few per cent faster).
  const long long zmax = one_wave ? 256 : (n > 1 ? 8 : 64);
  long long zc = (columns + groups - 1) / groups;
  if (zc < 1) zc = 1;
  if (zc > zmax) zc = zmax;
  t->z_chunk = (int)zc;
  // Single boxes take XCD-local tile ranges: in both precisions they beat
  // plain dispatch order with the populations stored in blocks (256 x 256 x
  // 1024 MRT, float64 over eight waves of groups: 4.20 against 4.43 ms;
  // float32 in one wave: 2.08 against 2.12).  Batches run in plain dispatch
  // order: consecutive entries of the tile table are neighbouring tiles of
  // one member, so plain order keeps the groups in flight on one contiguous
  // stretch of memory; XCD-local ranges cut the L2-missing halo reads (fetch
  // 1.41 -> 1.11 x the algorithmic reads, the rest served by the memory-side
  // cache) but spread the groups over eight stretches and run slower (14.47
  // against 14.27 ms).
  t->xcd_remap = n > 1 ? 0 : 1;
}

lbsc_tuning default_tuning(const lbsc_params* p, int32_t n) {
  lbsc_tuning t;
  t.block_x = 0;
  t.block_y = 0;
  t.xcd_remap = 1;
  t.pop_pad = -1;
  t.nodes_per_thread = 1;
  t.persistent = 0;
  t.two_kernel = 0;
  // float64 (about 200 VGPRs, 2 waves per SIMD): 256-thread groups, two per
  // CU, so one group's loads overlap the other's collision.  float32 (about
  // 110 VGPRs): 512-thread groups, two per CU; boxes with rows of at most 256
  // nodes and at least 256 tiles run 1024-thread groups of whole rows four or
  // more deep instead, one per CU.  Measured: 32.0 against 29.3 GLUPS on
  // 256 x 256 x 1024, 29.9 against 27.9 on 128 x 128 x 512, 27.2 against 25.6
  // on 64 x 64 x 256, 27.5 against 26.1 on the 64-ligament batch: the deeper
  // tile's smaller halo ring outweighs the lost overlap.  Wider rows split
  // into tiles of whole 1024-thread groups lose (23.9 against 28.4 on
  // 384 x 384 x 1024) and take 512 threads.
  // Boxes too small to give 256 groups of 512 threads even with one-plane
  // chunks take 256-thread groups instead (32 x 32 x 64: 8.5 against 9.4 us
  // per step).
  int nx = 1;
  for (int32_t i = 0; i < n; ++i) nx = std::max(nx, p[i].nx);
  if (p[0].precision == LBSC_F64) {
    t.threads = 256;
  } else if (4 * nx <= 1024 && tile_columns(p, n, 1024) >= 256) {
    t.threads = 1024;
  } else if (tile_columns(p, n, 512) >= 256) {
    t.threads = 512;
  } else {
    t.threads = 256;
  }
  chunk_and_order(p, n, &t);
  return t;
}

// Capacity of a lattice: room for every padding up to `pad` in either layout.
size_t lattice_bytes(const lbsc_params& p, long long pad) {
  const long long room = std::max(lattice_nodes(p, pad), (nodes(p) + 63) / 64 * 64 + pad);
  return align_up((size_t)lbsc::Q * (size_t)room * elem_size(p));
}

// Sizes of the aux area (tile capacity: the finest tiling allowed, one row of
// min(nx, kMinBlockX) columns per plane).
struct AuxSizes {
  size_t members, tiles, sync, part, out, psi, total;
  long long tile_cap;
};

// with_psi: room for the psi field of the two-kernel step form (single box).
AuxSizes aux_sizes(int32_t n, const lbsc_params* p, bool with_psi) {
  AuxSizes s;
  long long cap = 0;
  int max_blocks = 0, max_nz = 0;
  for (int32_t i = 0; i < n; ++i) {
    const int bmin = std::min(p[i].nx, kMinBlockX);
    cap += (long long)p[i].ny * p[i].nz * ((p[i].nx + bmin - 1) / bmin);
    lbsc::StepArgs a;
    a.plane = p[i].nx * p[i].ny;
    a.nz = p[i].nz;
    max_blocks = std::max(max_blocks, lbsc::diag_blocks(a));
    max_nz = std::max(max_nz, p[i].nz);
  }
  s.tile_cap = cap;
  s.members = align_up((size_t)n * sizeof(lbsc::BatchMember));
  s.tiles = align_up((size_t)cap * sizeof(int4));
  s.sync = kAlign;
  s.part = align_up((size_t)max_blocks * 8 * sizeof(double));
  s.out = align_up((size_t)(4 + max_nz) * sizeof(double));
  s.psi = with_psi ? align_up((size_t)nodes(p[0]) * elem_size(p[0])) : 0;
  s.total = s.members + s.tiles + s.sync + s.part + s.out + s.psi;
  return s;
}

size_t batch_bytes(int32_t n, const lbsc_params* p, long long pad, bool with_psi) {
  size_t total = 0;
  for (int32_t i = 0; i < n; ++i) total += 2 * lattice_bytes(p[i], pad);
  return total + aux_sizes(n, p, with_psi).total;
}

int hip_fail(lbsc_ctx* c, hipError_t e, const char* what) {
  c->err = std::string(what) + ": " + hipGetErrorString(e);
  return LBSC_EHIP;
}

#define HIP_OR_FAIL(ctx, expr)                              \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) return hip_fail(ctx, _e, #expr);  \
  } while (0)

// Recomputes every member's tile list and uploads the member and tile tables
// (synchronously).
int rebuild_tables(lbsc_ctx* c) {
  std::vector<lbsc::BatchMember> hm(c->m.size());
  std::vector<int4> ht;
  for (size_t i = 0; i < c->m.size(); ++i) {
    const lbsc::StepArgs& a = c->m[i].a;
    hm[i].a = a;
    hm[i].lat[0] = c->m[i].lat[0];
    hm[i].lat[1] = c->m[i].lat[1];
    const int nchunks = (a.nz + a.zchunk - 1) / a.zchunk;
    const int ntxy = a.ntiles_x * a.ntiles_y;
    for (int zc = 0; zc < nchunks; ++zc)
      for (int t = 0; t < ntxy; ++t) ht.push_back(make_int4((int)i, t, zc, 0));
  }
  if ((long long)ht.size() > c->tile_cap)
    return fail(&c->err, LBSC_EINVAL, "tile table exceeds its capacity");
  c->ntiles = (int)ht.size();
  HIP_OR_FAIL(c, hipMemcpyAsync(c->dmembers, hm.data(), hm.size() * sizeof(hm[0]),
                                hipMemcpyHostToDevice, c->stream));
  HIP_OR_FAIL(c, hipMemcpyAsync(c->dtiles, ht.data(), ht.size() * sizeof(ht[0]),
                                hipMemcpyHostToDevice, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return LBSC_OK;
}

// Shared by lbsc_init_fields and lbsc_init_batch.
int create(lbsc_ctx** out, int32_t n, const lbsc_params* p, const double* const* rho0,
           void* dev_buf, size_t dev_bytes, void* hip_stream, bool batch) {
  g_init_err.clear();
  if (!out) return fail(&g_init_err, LBSC_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_batch(n, p, &g_init_err);
  if (rc != LBSC_OK) return rc;
  if (!rho0) return fail(&g_init_err, LBSC_EINVAL, "rho0_host is NULL");
  if (!dev_buf) return fail(&g_init_err, LBSC_EINVAL, "dev_buf is NULL");
  if (((uintptr_t)dev_buf) % kAlign != 0)
    return fail(&g_init_err, LBSC_EINVAL, "dev_buf must be 256-byte aligned");
  const long long pad = batch ? kDefaultPad : kMaxPad;
  const size_t need = batch_bytes(n, p, pad, !batch);
  if (dev_bytes < need)
    return fail(&g_init_err, LBSC_EINVAL,
                "dev_bytes " + std::to_string(dev_bytes) + " < required " + std::to_string(need));
  for (int32_t m = 0; m < n; ++m) {
    if (!rho0[m])
      return fail(&g_init_err, LBSC_EINVAL, "rho0 of member " + std::to_string(m) + " is NULL");
    const long long nn = nodes(p[m]);
    for (long long i = 0; i < nn; ++i) {
      const double r = rho0[m][i];
      if (!(std::isfinite(r) && r > 0))
        return fail(&g_init_err, LBSC_EINVAL,
                    "rho0 must be finite and > 0 (member " + std::to_string(m) + ", index " +
                        std::to_string(i) + ")");
    }
  }
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, dev_buf) != hipSuccess || attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return fail(&g_init_err, LBSC_EINVAL, "dev_buf is not device memory");
  }
  // The device that holds the buffer; its copy of the static scratch is
  // resolved with it current.
  const int dev = attr.device;
  if (dev < 0 || dev >= kMaxDevices)
    return fail(&g_init_err, LBSC_EINVAL, "dev_buf is on an unsupported device index");
  {
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess && prev != dev) e = hipSetDevice(dev);
    if (e == hipSuccess) e = resolve_scratch(dev);
    if (prev >= 0 && prev != dev) {
      const hipError_t e2 = hipSetDevice(prev);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess)
      return fail(&g_init_err, LBSC_EHIP,
                  std::string("device scratch address: ") + hipGetErrorString(e));
  }

  lbsc_ctx* c = new (std::nothrow) lbsc_ctx();
  if (!c) return fail(&g_init_err, LBSC_ENOMEM, "context allocation failed");
  c->batch = batch;
  c->device = dev;
  c->tune = default_tuning(p, n);
  c->stream = (hipStream_t)hip_stream;
  c->buf = (char*)dev_buf;
  c->bytes = dev_bytes;
  c->cur = 0;
  c->step = 0;
  c->m.resize(n);
  size_t off = 0;
  for (int32_t i = 0; i < n; ++i) {
    Member& mm = c->m[i];
    mm.p = p[i];
    mm.a = make_args(p[i], c->tune, kDefaultPad);
    mm.lat_bytes = lattice_bytes(p[i], pad);
    mm.lat[0] = c->buf + off;
    mm.lat[1] = c->buf + off + mm.lat_bytes;
    off += 2 * mm.lat_bytes;
  }
  const AuxSizes ax = aux_sizes(n, p, !batch);
  c->tile_cap = ax.tile_cap;
  c->dmembers = (lbsc::BatchMember*)(c->buf + off);
  off += ax.members;
  c->dtiles = (int4*)(c->buf + off);
  off += ax.tiles;
  c->dsync = (unsigned*)(c->buf + off);
  off += ax.sync;
  c->part = (double*)(c->buf + off);
  off += ax.part;
  c->dout = (double*)(c->buf + off);
  off += ax.out;
  c->psi = ax.psi ? (void*)(c->buf + off) : nullptr;

  // Stage each rho0 in the member's second lattice (19 N values >= N
  // doubles), then build the state in the first.
  hipError_t e = hipSuccess;
  for (int32_t i = 0; i < n && e == hipSuccess; ++i) {
    Member& mm = c->m[i];
    e = hipMemcpyAsync(mm.lat[1], rho0[i], (size_t)nodes(mm.p) * sizeof(double),
                       hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
      e = lbsc::launch_init(mm.p.precision, mm.lat[0], (const double*)mm.lat[1], mm.a, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    g_init_err = std::string("initialisation failed: ") + hipGetErrorString(e);
    delete c;
    return LBSC_EHIP;
  }
  rc = rebuild_tables(c);
  if (rc != LBSC_OK) {
    g_init_err = c->err;
    delete c;
    return rc;
  }
  *out = c;
  return LBSC_OK;
}

Member* member(lbsc_ctx* c, int32_t i) {
  if (!c) return nullptr;
  if (i < 0 || i >= (int32_t)c->m.size()) {
    c->err = "member index out of range";
    return nullptr;
  }
  return &c->m[i];
}

int step_batch(lbsc_ctx* c, int64_t nsteps) {
  lbsc::BatchLaunch L;
  const Member& m0 = c->m[0];
  L.prec = m0.p.precision;
  L.coll = m0.p.collision;
  L.forc = m0.p.forcing;
  L.threads = c->tune.threads;
  L.npt = c->tune.nodes_per_thread;
  L.members = c->dmembers;
  L.tiles = c->dtiles;
  L.ntiles = c->ntiles;
  L.remap = c->tune.xcd_remap;
  L.lds = 0;
  for (const Member& mm : c->m)
    L.lds = std::max(L.lds, (size_t)4 * (mm.a.by + 2) * (mm.a.bx + 2) * elem_size(mm.p));
  L.sync = c->dsync;
  L.spin_limit = kSpinLimit;
  if (c->tune.persistent) {
    if (nsteps > 0x7fffffff) return fail(&c->err, LBSC_EINVAL, "too many steps for one launch");
    L.persistent = 1;
    L.parity = c->cur;
    L.nsteps = (int)nsteps;
    HIP_OR_FAIL(c, hipMemsetAsync(c->dsync, 0, 5 * sizeof(unsigned), c->stream));
    HIP_OR_FAIL(c, lbsc::launch_batch(L, c->stream));
    unsigned flags[3];
    HIP_OR_FAIL(c, hipMemcpyAsync(flags, c->dsync, sizeof(flags), hipMemcpyDeviceToHost,
                                  c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    if (flags[2]) return fail(&c->err, LBSC_EHIP, "grid barrier timed out in the persistent step");
    if (nsteps & 1) c->cur ^= 1;
    c->step += nsteps;
    return LBSC_OK;
  }
  L.persistent = 0;
  L.nsteps = 1;
  for (int64_t i = 0; i < nsteps; ++i) {
    L.parity = c->cur;
    hipError_t e = lbsc::launch_batch(L, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "batched step launch");
    c->cur ^= 1;
    c->step += 1;
  }
  return LBSC_OK;
}

int moments_of(lbsc_ctx* c, Member* mm, double* rho_dev, double* u_dev, double* p_dev) {
  if (!rho_dev) return fail(&c->err, LBSC_EINVAL, "rho_dev is required");
  // The idle lattice (19 n storage values >= n doubles) holds psi.
  hipError_t e = lbsc::launch_moments(mm->p.precision, mm->lat[c->cur], rho_dev, u_dev, p_dev,
                                      (double*)mm->lat[c->cur ^ 1], mm->a, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "moments launch");
  return LBSC_OK;
}

// Interface diagnostics of member mm with the reduction partials and the
// results in `part` and `dres` (the context's aux area, or the static
// scratch); rho and psi go to the idle lattice.
int diagnostics_into(lbsc_ctx* c, Member* mm, double rho_v, double rho_l, lbsc_diag* out,
                     double* r_of_z_host, double* part, double* dres) {
  if (!out) return fail(&c->err, LBSC_EINVAL, "out is NULL");
  if (!(std::isfinite(rho_v) && std::isfinite(rho_l) && rho_l > rho_v))
    return fail(&c->err, LBSC_EINVAL, "need finite rho_l > rho_v");
  const int nz = mm->p.nz;
  hipError_t e = lbsc::launch_diagnostics(mm->p.precision, mm->lat[c->cur],
                                          (double*)mm->lat[c->cur ^ 1], part, dres, rho_v,
                                          rho_l, mm->a, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "diagnostics launch");
  // No heap memory on this path (the static-scratch entry point allocates
  // nothing): the four sums go to the stack, the slice areas A(z) to the
  // caller's r_of_z buffer (turned into radii in place) or, without one,
  // through a stack buffer a chunk at a time.
  double head[4];
  HIP_OR_FAIL(c, hipMemcpyAsync(head, dres, sizeof(head), hipMemcpyDeviceToHost, c->stream));
  if (r_of_z_host)
    HIP_OR_FAIL(c, hipMemcpyAsync(r_of_z_host, dres + 4, (size_t)nz * sizeof(double),
                                  hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  out->mass = head[0];
  out->mom[0] = head[1];
  out->mom[1] = head[2];
  out->mom[2] = head[3];
  out->reserved = 0;
  const double pi = 3.14159265358979323846;
  double rmin = INFINITY;
  int zmin = 0;
  constexpr int kChunk = 256;
  double tmp[kChunk];
  for (int z0 = 0; z0 < nz; z0 += kChunk) {
    const int len = std::min(kChunk, nz - z0);
    double* a = r_of_z_host ? r_of_z_host + z0 : tmp;
    if (!r_of_z_host) {
      HIP_OR_FAIL(c, hipMemcpyAsync(tmp, dres + 4 + z0, (size_t)len * sizeof(double),
                                    hipMemcpyDeviceToHost, c->stream));
      HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    }
    for (int k = 0; k < len; ++k) {
      const double r = std::sqrt(a[k] / pi);
      a[k] = r;
      if (r < rmin) {
        rmin = r;
        zmin = z0 + k;
      }
    }
  }
  out->r_min = rmin;
  out->z_argmin = zmin;
  if (!std::isfinite(head[0])) return fail(&c->err, LBSC_ENONFINITE, "mass is not finite");
  return LBSC_OK;
}

int diagnostics_of(lbsc_ctx* c, Member* mm, double rho_v, double rho_l, lbsc_diag* out,
                   double* r_of_z_host) {
  return diagnostics_into(c, mm, rho_v, rho_l, out, r_of_z_host, c->part, c->dout);
}

int get_state_of(lbsc_ctx* c, Member* mm, void* host, size_t bytes) {
  const size_t es = elem_size(mm->p);
  const size_t need = (size_t)lbsc::Q * mm->a.n * es;
  if (!host || bytes != need)
    return fail(&c->err, LBSC_EINVAL, "host buffer must hold 19 * N values of the storage type");
  hipError_t e = lbsc::launch_gather(mm->p.precision, mm->lat[c->cur], mm->a.ps,
                                     mm->lat[c->cur ^ 1], mm->a.ps, mm->a, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "gather launch");
  HIP_OR_FAIL(c, hipMemcpy2DAsync(host, mm->a.n * es, mm->lat[c->cur ^ 1], mm->a.ps * es,
                                  mm->a.n * es, lbsc::Q, hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return LBSC_OK;
}

int set_state_of(lbsc_ctx* c, Member* mm, const void* host, size_t bytes) {
  const size_t es = elem_size(mm->p);
  const size_t need = (size_t)lbsc::Q * mm->a.n * es;
  if (!host || bytes != need)
    return fail(&c->err, LBSC_EINVAL, "host buffer must hold 19 * N values of the storage type");
  HIP_OR_FAIL(c, hipMemcpy2DAsync(mm->lat[c->cur ^ 1], mm->a.ps * es, host, mm->a.n * es,
                                  mm->a.n * es, lbsc::Q, hipMemcpyHostToDevice, c->stream));
  hipError_t e = lbsc::launch_scatter(mm->p.precision, mm->lat[c->cur ^ 1], mm->a.ps,
                                      mm->lat[c->cur], mm->a.ps, mm->a, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "scatter launch");
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return LBSC_OK;
}

// Workspace layout of the adjoint for a single box (lattices sized for the
// largest padding so any tuning of the box fits).
struct AdjLayout {
  size_t lat, psi, cp, ring, psis, P, R, psi_fbar, fbar_dot_v, partial, acc, total;
  int ncp;
};

AdjLayout adj_layout(const lbsc_params& p, int64_t nsteps, int32_t segment) {
  AdjLayout L;
  lbsc::StepArgs a;
  a.n = nodes(p);
  L.ncp = (int)((nsteps + segment - 1) / segment);
  L.lat = lattice_bytes(p, kMaxPad);
  L.psi = align_up((size_t)a.n * elem_size(p));
  L.cp = (size_t)L.ncp * L.lat;
  L.ring = (size_t)(segment + 1) * L.lat;
  L.psis = (size_t)segment * L.psi;
  L.P = 2 * L.lat;
  L.R = 2 * L.psi;
  L.psi_fbar = align_up(3 * (size_t)a.n * elem_size(p));
  L.fbar_dot_v = align_up((size_t)a.n * elem_size(p));
  L.partial = align_up(4 * sizeof(double) * (size_t)lbsc::adj_blocks(a));
  L.acc = kAlign;
  L.total = L.cp + L.ring + L.psis + L.P + L.R + L.psi_fbar + L.fbar_dot_v + L.partial + L.acc;
  return L;
}

int check_adjoint(const lbsc_params* p, int64_t nsteps, int32_t segment, std::string* msg) {
  int rc = check_params(p, msg);
  if (rc != LBSC_OK) return rc;
  if (p->forcing != LBSC_FORCING_GUO)
    return fail(msg, LBSC_EINVAL, "the adjoint covers Guo forcing (BGK and MRT)");
  if (nsteps < 1) return fail(msg, LBSC_EINVAL, "nsteps must be >= 1");
  if (segment < 1 || segment > nsteps) return fail(msg, LBSC_EINVAL, "need 1 <= segment <= nsteps");
  if ((nsteps + segment - 1) / segment > (1 << 20))
    return fail(msg, LBSC_EINVAL, "too many checkpoints");
  return LBSC_OK;
}

}  // namespace

extern "C" {

size_t lbsc_state_bytes(const lbsc_params* p) {
  if (check_params(p, nullptr) != LBSC_OK) return 0;
  return batch_bytes(1, p, kMaxPad, true);
}

size_t lbsc_batch_state_bytes(int32_t n, const lbsc_params* p) {
  if (check_batch(n, p, nullptr) != LBSC_OK) return 0;
  return batch_bytes(n, p, kDefaultPad, false);
}

int lbsc_init_fields(lbsc_ctx** out, const lbsc_params* p, const double* rho0_host,
                     void* dev_buf, size_t dev_bytes, void* hip_stream) {
  if (!rho0_host) {
    g_init_err = "rho0_host is NULL";
    if (out) *out = nullptr;
    return LBSC_EINVAL;
  }
  const double* rho[1] = {rho0_host};
  return create(out, 1, p, rho, dev_buf, dev_bytes, hip_stream, false);
}

int lbsc_init_batch(lbsc_ctx** out, int32_t n, const lbsc_params* p,
                    const double* const* rho0_host, void* dev_buf, size_t dev_bytes,
                    void* hip_stream) {
  return create(out, n, p, rho0_host, dev_buf, dev_bytes, hip_stream, true);
}

int32_t lbsc_batch_size(const lbsc_ctx* c) { return c ? (int32_t)c->m.size() : -1; }

int lbsc_step(lbsc_ctx* c, int64_t nsteps) {
  if (!c) return LBSC_EINVAL;
  if (nsteps < 0) return fail(&c->err, LBSC_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return LBSC_OK;
  if (c->batch || c->tune.persistent) return step_batch(c, nsteps);
  Member& m0 = c->m[0];
  for (int64_t i = 0; i < nsteps; ++i) {
    hipError_t e =
        c->tune.two_kernel
            ? lbsc::launch_step_two_kernel(m0.p.precision, m0.p.collision, m0.p.forcing,
                                           m0.lat[c->cur], c->psi, m0.lat[c->cur ^ 1], m0.a,
                                           c->stream)
            : lbsc::launch_step(m0.p.precision, m0.p.collision, m0.p.forcing, c->tune.threads,
                                c->tune.nodes_per_thread, m0.lat[c->cur], m0.lat[c->cur ^ 1],
                                m0.a, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "step launch");
    c->cur ^= 1;
    c->step += 1;
  }
  return LBSC_OK;
}

int64_t lbsc_step_count(const lbsc_ctx* c) { return c ? c->step : -1; }

int lbsc_compute_moments(lbsc_ctx* c, double* rho_dev, double* u_dev, double* p_dev) {
  Member* mm = member(c, 0);
  if (!mm) return LBSC_EINVAL;
  return moments_of(c, mm, rho_dev, u_dev, p_dev);
}

int lbsc_member_moments(lbsc_ctx* c, int32_t i, double* rho_dev, double* u_dev, double* p_dev) {
  Member* mm = member(c, i);
  if (!mm) return LBSC_EINVAL;
  return moments_of(c, mm, rho_dev, u_dev, p_dev);
}

int lbsc_interface_diagnostics(lbsc_ctx* c, double rho_v, double rho_l, lbsc_diag* out,
                               double* r_of_z_host) {
  Member* mm = member(c, 0);
  if (!mm) return LBSC_EINVAL;
  return diagnostics_of(c, mm, rho_v, rho_l, out, r_of_z_host);
}

int lbsc_member_diagnostics(lbsc_ctx* c, int32_t i, double rho_v, double rho_l, lbsc_diag* out,
                            double* r_of_z_host) {
  Member* mm = member(c, i);
  if (!mm) return LBSC_EINVAL;
  return diagnostics_of(c, mm, rho_v, rho_l, out, r_of_z_host);
}

int lbsc_interface_diagnostics_static(lbsc_ctx* c, double rho_v, double rho_l, lbsc_diag* out,
                                      double* r_of_z_host) {
  Member* mm = member(c, 0);
  if (!mm) return LBSC_EINVAL;
  int dev = -1;
  HIP_OR_FAIL(c, hipGetDevice(&dev));
  if (dev != c->device) return fail(&c->err, LBSC_EINVAL, "the context's device must be current");
  double* base = scratch_of(dev);
  if (!base) return fail(&c->err, LBSC_ESTATE, "device scratch address not resolved");
  // Results first, then the partials from a 256-byte boundary.
  const size_t res = ((size_t)(4 + mm->p.nz) + 31) / 32 * 32;
  const size_t need = res + 8 * (size_t)lbsc::diag_blocks(mm->a);
  if (need > kScratchDoubles)
    return fail(&c->err, LBSC_EINVAL,
                "box too large for the static scratch: needs " + std::to_string(need * 8) +
                    " bytes of " + std::to_string(kScratchDoubles * 8) +
                    " (nz * ceil(nx * ny / 4096) * 64 + (4 + nz) * 8 bytes, rounded)");
  return diagnostics_into(c, mm, rho_v, rho_l, out, r_of_z_host, base + res, base);
}

int lbsc_get_state(lbsc_ctx* c, void* host, size_t bytes, int64_t* step) {
  Member* mm = member(c, 0);
  if (!mm) return LBSC_EINVAL;
  const int rc = get_state_of(c, mm, host, bytes);
  if (rc == LBSC_OK && step) *step = c->step;
  return rc;
}

int lbsc_member_get_state(lbsc_ctx* c, int32_t i, void* host, size_t bytes) {
  Member* mm = member(c, i);
  if (!mm) return LBSC_EINVAL;
  return get_state_of(c, mm, host, bytes);
}

int lbsc_set_state(lbsc_ctx* c, const void* host, size_t bytes, int64_t step) {
  Member* mm = member(c, 0);
  if (!mm) return LBSC_EINVAL;
  if (c->m.size() != 1) return fail(&c->err, LBSC_ESTATE, "use lbsc_member_set_state on a batch");
  if (step < 0) return fail(&c->err, LBSC_EINVAL, "step must be >= 0");
  const int rc = set_state_of(c, mm, host, bytes);
  if (rc == LBSC_OK) c->step = step;
  return rc;
}

int lbsc_member_set_state(lbsc_ctx* c, int32_t i, const void* host, size_t bytes) {
  Member* mm = member(c, i);
  if (!mm) return LBSC_EINVAL;
  return set_state_of(c, mm, host, bytes);
}

int lbsc_set_tuning(lbsc_ctx* c, const lbsc_tuning* t) {
  if (!c) return LBSC_EINVAL;
  if (!t) return fail(&c->err, LBSC_EINVAL, "tuning is NULL");
  std::vector<lbsc_params> ps;
  int nx_max = 1;
  for (const Member& mm : c->m) {
    ps.push_back(mm.p);
    nx_max = std::max(nx_max, mm.p.nx);
  }
  lbsc_tuning n = default_tuning(ps.data(), (int32_t)ps.size());
  if (t->threads) {
    if (t->threads != 256 && t->threads != 512 && t->threads != 1024)
      return fail(&c->err, LBSC_EINVAL, "threads must be 256, 512 or 1024");
    n.threads = t->threads;
    // The default chunk and tile order are those of the requested group size.
    chunk_and_order(ps.data(), (int32_t)ps.size(), &n);
  }
  if (t->z_chunk < 0 || t->block_y < 0 || t->block_x < 0)
    return fail(&c->err, LBSC_EINVAL, "negative tuning value");
  if (t->nodes_per_thread < 0 || t->nodes_per_thread > 2)
    return fail(&c->err, LBSC_EINVAL, "nodes_per_thread must be 0, 1 or 2");
  if (t->nodes_per_thread) n.nodes_per_thread = t->nodes_per_thread;
  const long long cap = (long long)n.nodes_per_thread * n.threads;
  if (t->block_x > 0 && t->block_x < kMinBlockX && t->block_x < nx_max)
    return fail(&c->err, LBSC_EINVAL, "block_x must be 0, >= 64 or >= nx");
  if (t->block_x > cap)
    return fail(&c->err, LBSC_EINVAL, "block_x exceeds nodes_per_thread * threads");
  if (t->block_y && (long long)t->block_y * std::max(1, t->block_x) > cap)
    return fail(&c->err, LBSC_EINVAL, "block_x * block_y exceeds nodes_per_thread * threads");
  if (t->pop_pad > kMaxPad) return fail(&c->err, LBSC_EINVAL, "pop_pad exceeds 65536");
  if (c->batch && t->pop_pad >= 0 && t->pop_pad != kDefaultPad && layout_block(c->m[0].p) == 0)
    return fail(&c->err, LBSC_EINVAL, "a batch keeps the default population padding");
  if (t->persistent != 0 && t->persistent != 1)
    return fail(&c->err, LBSC_EINVAL, "persistent must be 0 or 1");
  if (t->two_kernel != 0 && t->two_kernel != 1)
    return fail(&c->err, LBSC_EINVAL, "two_kernel must be 0 or 1");
  if (t->two_kernel && (c->batch || t->persistent))
    return fail(&c->err, LBSC_EINVAL, "the two-kernel step form is for a single box, one launch per step");
  if (t->z_chunk) n.z_chunk = t->z_chunk;
  n.block_y = t->block_y;
  n.block_x = t->block_x;
  if (t->xcd_remap >= 0) n.xcd_remap = t->xcd_remap ? 1 : 0;  // < 0: keep the default
  n.pop_pad = c->batch ? -1 : t->pop_pad;
  n.persistent = t->persistent;
  n.two_kernel = t->two_kernel;
  for (Member& mm : c->m) {
    const lbsc::StepArgs na = make_args(mm.p, n, pad_of(n));
    if (na.ps != mm.a.ps) {
      // New population stride: export the state through the free lattice and
      // import it again in the new layout.
      hipError_t e = lbsc::launch_gather(mm.p.precision, mm.lat[c->cur], mm.a.ps,
                                         mm.lat[c->cur ^ 1], na.ps, mm.a, c->stream);
      if (e == hipSuccess)
        e = lbsc::launch_scatter(mm.p.precision, mm.lat[c->cur ^ 1], na.ps, mm.lat[c->cur], na.ps,
                                 na, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "re-layout launch");
    }
    mm.a = na;
  }
  c->tune = n;
  return rebuild_tables(c);
}

int lbsc_get_tuning(const lbsc_ctx* c, lbsc_tuning* t) {
  if (!c || !t) return LBSC_EINVAL;
  const lbsc::StepArgs& a = c->m[0].a;
  *t = c->tune;
  if (!c->batch) {
    // A single box reports the effective rows per tile and chunk length; a
    // batch reports what was requested (members differ), so that the result
    // can be passed back to lbsc_set_tuning.
    t->block_x = a.bx;
    t->block_y = a.by;
    t->z_chunk = a.zchunk;
  }
  t->pop_pad = (int32_t)(a.ps - (a.n + 63) / 64 * 64);
  return LBSC_OK;
}

int lbsc_default_tuning(const lbsc_params* p, int32_t n, lbsc_tuning* t) {
  if (!t || check_batch(n, p, nullptr) != LBSC_OK) return LBSC_EINVAL;
  *t = default_tuning(p, n);
  if (n == 1) {
    // As lbsc_get_tuning reports it for a single box: the effective tile and
    // chunk, and the population padding.
    const lbsc::StepArgs a = make_args(p[0], *t, kDefaultPad);
    t->block_x = a.bx;
    t->block_y = a.by;
    t->z_chunk = a.zchunk;
    t->pop_pad = (int32_t)(a.ps - (a.n + 63) / 64 * 64);
  }
  return LBSC_OK;
}

size_t lbsc_adjoint_workspace_bytes(const lbsc_params* p, int64_t nsteps, int32_t segment) {
  if (check_adjoint(p, nsteps, segment, nullptr) != LBSC_OK) return 0;
  return adj_layout(*p, nsteps, segment).total;
}

int lbsc_adjoint_forward(lbsc_ctx* c, int64_t nsteps, int32_t segment, void* workspace,
                         size_t bytes) {
  if (!c) return LBSC_EINVAL;
  c->adj.ready = false;
  if (c->m.size() != 1) return fail(&c->err, LBSC_ESTATE, "the adjoint works on a single box");
  Member& mm = c->m[0];
  int rc = check_adjoint(&mm.p, nsteps, segment, &c->err);
  if (rc != LBSC_OK) return rc;
  if (c->step != 0) return fail(&c->err, LBSC_ESTATE, "the adjoint forward starts from the initial state");
  if (!workspace || ((uintptr_t)workspace) % kAlign != 0)
    return fail(&c->err, LBSC_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  const AdjLayout L = adj_layout(mm.p, nsteps, segment);
  if (bytes < L.total)
    return fail(&c->err, LBSC_EINVAL, "workspace smaller than lbsc_adjoint_workspace_bytes");
  AdjWork& w = c->adj;
  char* base = (char*)workspace;
  w.nsteps = nsteps;
  w.segment = segment;
  w.ncp = L.ncp;
  w.lat_bytes = L.lat;
  w.psi_bytes = L.psi;
  w.cp = base;
  base += L.cp;
  w.ring = base;
  base += L.ring;
  w.psi = base;
  base += L.psis;
  w.P[0] = base;
  w.P[1] = base + L.lat;
  base += L.P;
  w.R[0] = base;
  w.R[1] = base + L.psi;
  base += L.R;
  w.psi_fbar = base;
  base += L.psi_fbar;
  w.fbar_dot_v = base;
  base += L.fbar_dot_v;
  w.partial = (double*)base;
  base += L.partial;
  w.acc = (double*)base;
  const size_t used = (size_t)lbsc::Q * mm.a.ps * elem_size(mm.p);
  for (int k = 0; k < w.ncp; ++k) {
    HIP_OR_FAIL(c, hipMemcpyAsync(w.cp + (size_t)k * w.lat_bytes, mm.lat[c->cur], used,
                                  hipMemcpyDeviceToDevice, c->stream));
    const int64_t len = std::min<int64_t>(segment, nsteps - (int64_t)k * segment);
    rc = lbsc_step(c, len);
    if (rc != LBSC_OK) return rc;
  }
  w.ready = true;
  return LBSC_OK;
}

int lbsc_rmin_gradient(lbsc_ctx* c, double rho_v, double rho_l, double* rhobar_dev,
                       double* r_min) {
  Member* mm = member(c, 0);
  if (!mm) return LBSC_EINVAL;
  if (!rhobar_dev) return fail(&c->err, LBSC_EINVAL, "rhobar_dev is NULL");
  lbsc_diag d;
  int rc = diagnostics_of(c, mm, rho_v, rho_l, &d, nullptr);
  if (rc != LBSC_OK) return rc;
  if (!(d.r_min > 0)) return fail(&c->err, LBSC_EINVAL, "r_min is zero: the ligament has broken");
  rc = moments_of(c, mm, rhobar_dev, nullptr, nullptr);
  if (rc != LBSC_OK) return rc;
  const double coef = 1.0 / (2.0 * 3.14159265358979323846 * d.r_min * (rho_l - rho_v));
  HIP_OR_FAIL(c, lbsc::launch_rmin_grad(rhobar_dev, mm->a, d.z_argmin, coef, rho_v, rho_l,
                                        c->stream));
  if (r_min) *r_min = d.r_min;
  return LBSC_OK;
}

int lbsc_adjoint_backward(lbsc_ctx* c, const double* rhobar_dev, double* rho0bar_dev,
                          double* dL_dG, double* dL_dtau) {
  if (!c) return LBSC_EINVAL;
  AdjWork& w = c->adj;
  if (!w.ready || c->m.size() != 1)
    return fail(&c->err, LBSC_ESTATE, "call lbsc_adjoint_forward first");
  if (c->step != w.nsteps)
    return fail(&c->err, LBSC_ESTATE, "the state has moved since lbsc_adjoint_forward");
  if (!rhobar_dev || !rho0bar_dev) return fail(&c->err, LBSC_EINVAL, "NULL gradient buffer");
  Member& mm = c->m[0];
  const int prec = mm.p.precision;
  lbsc::AdjArgs g;
  g.a = mm.a;
  g.psi_fbar = w.psi_fbar;
  g.fbar_dot_v = w.fbar_dot_v;
  g.partial = w.partial;
  w.have_rates = false;
  HIP_OR_FAIL(c, hipMemsetAsync(w.acc, 0, 4 * sizeof(double), c->stream));
  HIP_OR_FAIL(c, hipMemsetAsync(w.partial, 0, 4 * sizeof(double) * (size_t)lbsc::adj_blocks(mm.a),
                                c->stream));
  int pc = 0;  // adjoint state of the step after the one being processed
  g.p_out = w.P[pc];
  g.r_out = w.R[pc];
  HIP_OR_FAIL(c, lbsc::launch_adjoint_seed(prec, g, rhobar_dev, c->stream));
  const size_t used = (size_t)lbsc::Q * mm.a.ps * elem_size(mm.p);
  for (int seg = w.ncp - 1; seg >= 0; --seg) {
    const int64_t len = std::min<int64_t>(w.segment, w.nsteps - (int64_t)seg * w.segment);
    // Recompute the segment, keeping every lattice and psi field it uses.
    HIP_OR_FAIL(c, hipMemcpyAsync(w.ring, w.cp + (size_t)seg * w.lat_bytes, used,
                                  hipMemcpyDeviceToDevice, c->stream));
    for (int64_t t = 0; t < len; ++t) {
      lbsc::StepArgs a2 = mm.a;
      a2.psi_out = w.psi + (size_t)t * w.psi_bytes;
      HIP_OR_FAIL(c, lbsc::launch_step(prec, mm.p.collision, mm.p.forcing, c->tune.threads,
                                       c->tune.nodes_per_thread,
                                       w.ring + (size_t)t * w.lat_bytes,
                                       w.ring + (size_t)(t + 1) * w.lat_bytes, a2, c->stream));
    }
    for (int64_t t = len - 1; t >= 0; --t) {
      g.bprev = w.ring + (size_t)t * w.lat_bytes;
      g.psi = w.psi + (size_t)t * w.psi_bytes;
      g.p_next = w.P[pc];
      g.r_next = w.R[pc];
      g.p_out = w.P[pc ^ 1];
      g.r_out = w.R[pc ^ 1];
      HIP_OR_FAIL(c, lbsc::launch_adjoint_step(prec, mm.p.collision, g, c->stream));
      pc ^= 1;
    }
  }
  g.p_next = w.P[pc];
  g.r_next = w.R[pc];
  HIP_OR_FAIL(c, lbsc::launch_adjoint_final(prec, g, rho0bar_dev, c->stream));
  HIP_OR_FAIL(c, lbsc::launch_adjoint_reduce(g, w.acc, c->stream));
  double acc[4];
  HIP_OR_FAIL(c, hipMemcpyAsync(acc, w.acc, sizeof(acc), hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  if (dL_dG) *dL_dG = acc[0];
  if (dL_dtau) *dL_dtau = acc[1];
  w.rates[0] = acc[2];
  w.rates[1] = acc[3];
  w.have_rates = true;
  return LBSC_OK;
}

int lbsc_adjoint_rate_gradients(const lbsc_ctx* c, double* dL_ds_bulk, double* dL_ds_ghost) {
  if (!c) return LBSC_EINVAL;
  if (!c->adj.have_rates) return LBSC_ESTATE;
  if (dL_ds_bulk) *dL_ds_bulk = c->adj.rates[0];
  if (dL_ds_ghost) *dL_ds_ghost = c->adj.rates[1];
  return LBSC_OK;
}

void lbsc_lattice(int32_t* c, double* w) { lbsc::lattice_tables(c, w); }

void lbsc_destroy(lbsc_ctx* c) { delete c; }

const char* lbsc_last_error(const lbsc_ctx* c) {
  return c ? c->err.c_str() : g_init_err.c_str();
}

}  // extern "C"
