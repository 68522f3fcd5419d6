// C ABI of the D3Q19 pseudo-potential lattice Boltzmann library (include/lbsc.h).
//
// Validation, the context, the device-memory layout inside the caller's
// buffer, and the order of launches.  All arithmetic of the method runs in the
// kernels of lbsc_device.hip.
#include "lbsc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbsc_internal.h"

struct lbsc_ctx {
  lbsc_params p;
  lbsc::StepArgs a;
  lbsc_tuning tune;
  hipStream_t stream;
  char* buf;
  size_t bytes;
  void* lat[2];
  int cur;           // lattice holding the current state
  double* part;      // diagnostic partial sums
  double* dout;      // diagnostic results: 4 + nz doubles
  int64_t step;
  std::string err;
};

namespace {

thread_local std::string g_init_err;

constexpr size_t kAlign = 256;
// Largest padding between population arrays (elements); the state buffer is
// sized for it so the layout can be retuned in place.
constexpr long long kMaxPad = 65536;
constexpr long long kDefaultPad = 1088;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

size_t elem_size(const lbsc_params& p) { return p.precision == LBSC_F64 ? 8 : 4; }

int fail(std::string* where, int code, const std::string& msg) {
  if (where) *where = msg;
  return code;
}

// Checks a parameter set; returns LBSC_OK or LBSC_EINVAL with a message.
int check_params(const lbsc_params* p, std::string* msg) {
  if (!p) return fail(msg, LBSC_EINVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1)
    return fail(msg, LBSC_EINVAL, "box dimensions must be >= 1");
  if (p->nx > 1024) return fail(msg, LBSC_EINVAL, "nx > 1024 is not supported (full-row tiles)");
  const long long n = (long long)p->nx * p->ny * p->nz;
  if (n > 0x7fffffffLL) return fail(msg, LBSC_EINVAL, "more than 2^31 - 1 nodes");
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

lbsc::StepArgs make_args(const lbsc_params& p, const lbsc_tuning& t) {
  lbsc::StepArgs a;
  a.nx = p.nx;
  a.ny = p.ny;
  a.nz = p.nz;
  a.plane = p.nx * p.ny;
  a.n = (long long)p.nx * p.ny * p.nz;
  a.ps = (a.n + 63) / 64 * 64 + (t.pop_pad >= 0 ? t.pop_pad : kDefaultPad);
  const int rows = t.nodes_per_thread * t.threads / p.nx;  // rows the group can hold
  int by = t.block_y > 0 ? t.block_y : rows;
  if (by > rows) by = rows;
  if (by < 1) by = 1;
  if (by > p.ny) by = p.ny;
  // Four psi planes of (by + 2) rows must fit the 160 KB of LDS of a CU.
  while (by > 1 && 4LL * (by + 2) * p.nx * (long long)elem_size(p) > 160 * 1024) --by;
  a.by = by;
  a.ntiles_y = (p.ny + by - 1) / by;
  a.zchunk = t.z_chunk > 0 ? (t.z_chunk > p.nz ? p.nz : t.z_chunk) : p.nz;
  a.xcd_remap = t.xcd_remap;
  a.G = p.G;
  a.psi_rho0 = p.psi_rho0;
  a.tau = p.tau;
  a.omega = 1.0 / p.tau;
  a.s_bulk = p.s_bulk;
  a.s_ghost = p.s_ghost;
  a.rho_ref = p.precision == LBSC_F64 ? 0.0 : p.rho_ref;
  return a;
}

lbsc_tuning default_tuning(const lbsc_params& p) {
  lbsc_tuning t;
  // Two or more work-groups per CU overlap one group's loads with another's
  // collision; float64 needs twice the registers, so smaller groups.
  t.threads = p.precision == LBSC_F64 ? 256 : 512;
  while (t.threads < p.nx) t.threads *= 2;
  t.block_y = 0;
  t.xcd_remap = 1;
  t.pop_pad = -1;
  t.nodes_per_thread = 1;
  // Enough work-groups to fill 256 CUs a few times over, but long z-marches
  // so the two extra halo planes of each chunk stay a small fraction.
  const int by = std::max(1, std::min(p.ny, t.nodes_per_thread * t.threads / p.nx));
  const long long tiles = (p.ny + by - 1) / by;
  long long zc = (tiles * p.nz + 2047) / 2048;
  if (zc < 8) zc = 8;
  if (zc > 64) zc = 64;
  if (zc > p.nz) zc = p.nz;
  t.z_chunk = (int)zc;
  return t;
}

size_t lattice_bytes(const lbsc_params& p) {
  const long long n = (long long)p.nx * p.ny * p.nz;
  return align_up((size_t)lbsc::Q * (size_t)((n + 63) / 64 * 64 + kMaxPad) * elem_size(p));
}

size_t aux_bytes(const lbsc_params& p, const lbsc::StepArgs& a) {
  return align_up((size_t)lbsc::diag_blocks(a) * 8 * sizeof(double)) +
         align_up((size_t)(4 + p.nz) * sizeof(double));
}

int hip_fail(lbsc_ctx* c, hipError_t e, const char* what) {
  c->err = std::string(what) + ": " + hipGetErrorString(e);
  return LBSC_EHIP;
}

#define HIP_OR_FAIL(ctx, expr)                          \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return hip_fail(ctx, _e, #expr); \
  } while (0)

}  // namespace

extern "C" {

size_t lbsc_state_bytes(const lbsc_params* p) {
  if (check_params(p, nullptr) != LBSC_OK) return 0;
  const lbsc_tuning t = default_tuning(*p);
  const lbsc::StepArgs a = make_args(*p, t);
  return 2 * lattice_bytes(*p) + aux_bytes(*p, a);
}

int lbsc_init_fields(lbsc_ctx** out, const lbsc_params* p, const double* rho0_host,
                     void* dev_buf, size_t dev_bytes, void* hip_stream) {
  g_init_err.clear();
  if (!out) return fail(&g_init_err, LBSC_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_params(p, &g_init_err);
  if (rc != LBSC_OK) return rc;
  if (!rho0_host) return fail(&g_init_err, LBSC_EINVAL, "rho0_host is NULL");
  if (!dev_buf) return fail(&g_init_err, LBSC_EINVAL, "dev_buf is NULL");
  if (((uintptr_t)dev_buf) % kAlign != 0)
    return fail(&g_init_err, LBSC_EINVAL, "dev_buf must be 256-byte aligned");
  const size_t need = lbsc_state_bytes(p);
  if (dev_bytes < need)
    return fail(&g_init_err, LBSC_EINVAL,
                "dev_bytes " + std::to_string(dev_bytes) + " < lbsc_state_bytes " +
                    std::to_string(need));
  const long long n = (long long)p->nx * p->ny * p->nz;
  for (long long i = 0; i < n; ++i) {
    const double r = rho0_host[i];
    if (!(std::isfinite(r) && r > 0))
      return fail(&g_init_err, LBSC_EINVAL,
                  "rho0 must be finite and > 0 (index " + std::to_string(i) + ")");
  }
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, dev_buf) != hipSuccess || attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return fail(&g_init_err, LBSC_EINVAL, "dev_buf is not device memory");
  }

  lbsc_ctx* c = new (std::nothrow) lbsc_ctx();
  if (!c) return fail(&g_init_err, LBSC_ENOMEM, "context allocation failed");
  c->p = *p;
  c->tune = default_tuning(*p);
  c->a = make_args(*p, c->tune);
  c->stream = (hipStream_t)hip_stream;
  c->buf = (char*)dev_buf;
  c->bytes = dev_bytes;
  const size_t lb = lattice_bytes(*p);
  c->lat[0] = c->buf;
  c->lat[1] = c->buf + lb;
  c->part = (double*)(c->buf + 2 * lb);
  c->dout = (double*)(c->buf + 2 * lb + align_up((size_t)lbsc::diag_blocks(c->a) * 8 * 8));
  c->cur = 0;
  c->step = 0;

  // Stage rho0 in the second lattice (19 N values >= N doubles), then build
  // the state in the first.
  hipError_t e = hipMemcpyAsync(c->lat[1], rho0_host, (size_t)n * sizeof(double),
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = lbsc::launch_init(p->precision, c->lat[0], (const double*)c->lat[1],
                                             c->a, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    g_init_err = std::string("initialisation failed: ") + hipGetErrorString(e);
    delete c;
    return LBSC_EHIP;
  }
  *out = c;
  return LBSC_OK;
}

int lbsc_step(lbsc_ctx* c, int64_t nsteps) {
  if (!c) return LBSC_EINVAL;
  if (nsteps < 0) return fail(&c->err, LBSC_EINVAL, "nsteps must be >= 0");
  for (int64_t i = 0; i < nsteps; ++i) {
    hipError_t e = lbsc::launch_step(c->p.precision, c->p.collision, c->p.forcing,
                                     c->tune.threads, c->tune.nodes_per_thread, c->lat[c->cur],
                                     c->lat[c->cur ^ 1], c->a, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "step launch");
    c->cur ^= 1;
    c->step += 1;
  }
  return LBSC_OK;
}

int64_t lbsc_step_count(const lbsc_ctx* c) { return c ? c->step : -1; }

int lbsc_compute_moments(lbsc_ctx* c, double* rho_dev, double* u_dev, double* p_dev) {
  if (!c) return LBSC_EINVAL;
  if (!rho_dev) return fail(&c->err, LBSC_EINVAL, "rho_dev is required");
  hipError_t e = lbsc::launch_moments(c->p.precision, c->lat[c->cur], rho_dev, u_dev, p_dev, c->a,
                                      c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "moments launch");
  return LBSC_OK;
}

int lbsc_interface_diagnostics(lbsc_ctx* c, double rho_v, double rho_l, lbsc_diag* out,
                               double* r_of_z_host) {
  if (!c) return LBSC_EINVAL;
  if (!out) return fail(&c->err, LBSC_EINVAL, "out is NULL");
  if (!(std::isfinite(rho_v) && std::isfinite(rho_l) && rho_l > rho_v))
    return fail(&c->err, LBSC_EINVAL, "need finite rho_l > rho_v");
  const int nz = c->p.nz;
  hipError_t e = lbsc::launch_diagnostics(c->p.precision, c->lat[c->cur],
                                          (double*)c->lat[c->cur ^ 1], c->part, c->dout, rho_v,
                                          rho_l, c->a, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "diagnostics launch");
  std::vector<double> h(4 + (size_t)nz);
  HIP_OR_FAIL(c, hipMemcpyAsync(h.data(), c->dout, h.size() * sizeof(double),
                                hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  out->mass = h[0];
  out->mom[0] = h[1];
  out->mom[1] = h[2];
  out->mom[2] = h[3];
  out->reserved = 0;
  const double pi = 3.14159265358979323846;
  double rmin = INFINITY;
  int zmin = 0;
  for (int z = 0; z < nz; ++z) {
    const double r = std::sqrt(h[4 + z] / pi);
    if (r_of_z_host) r_of_z_host[z] = r;
    if (r < rmin) {
      rmin = r;
      zmin = z;
    }
  }
  out->r_min = rmin;
  out->z_argmin = zmin;
  if (!std::isfinite(h[0])) return fail(&c->err, LBSC_ENONFINITE, "mass is not finite");
  return LBSC_OK;
}

int lbsc_get_state(lbsc_ctx* c, void* host, size_t bytes, int64_t* step) {
  if (!c) return LBSC_EINVAL;
  const size_t need = (size_t)lbsc::Q * c->a.n * elem_size(c->p);
  if (!host || bytes != need)
    return fail(&c->err, LBSC_EINVAL, "host buffer must hold 19 * N values of the storage type");
  const size_t es = elem_size(c->p);
  hipError_t e = lbsc::launch_gather(c->p.precision, c->lat[c->cur], c->a.ps, c->lat[c->cur ^ 1],
                                     c->a.ps, c->a, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "gather launch");
  HIP_OR_FAIL(c, hipMemcpy2DAsync(host, c->a.n * es, c->lat[c->cur ^ 1], c->a.ps * es, c->a.n * es,
                                  lbsc::Q, hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  if (step) *step = c->step;
  return LBSC_OK;
}

int lbsc_set_state(lbsc_ctx* c, const void* host, size_t bytes, int64_t step) {
  if (!c) return LBSC_EINVAL;
  const size_t need = (size_t)lbsc::Q * c->a.n * elem_size(c->p);
  if (!host || bytes != need)
    return fail(&c->err, LBSC_EINVAL, "host buffer must hold 19 * N values of the storage type");
  if (step < 0) return fail(&c->err, LBSC_EINVAL, "step must be >= 0");
  const size_t es = elem_size(c->p);
  HIP_OR_FAIL(c, hipMemcpy2DAsync(c->lat[c->cur ^ 1], c->a.ps * es, host, c->a.n * es, c->a.n * es,
                                  lbsc::Q, hipMemcpyHostToDevice, c->stream));
  hipError_t e = lbsc::launch_scatter(c->p.precision, c->lat[c->cur ^ 1], c->a.ps, c->lat[c->cur],
                                      c->a.ps, c->a, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "scatter launch");
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->step = step;
  return LBSC_OK;
}

int lbsc_set_tuning(lbsc_ctx* c, const lbsc_tuning* t) {
  if (!c) return LBSC_EINVAL;
  if (!t) return fail(&c->err, LBSC_EINVAL, "tuning is NULL");
  lbsc_tuning n = default_tuning(c->p);
  if (t->threads) {
    if (t->threads != 256 && t->threads != 512 && t->threads != 1024)
      return fail(&c->err, LBSC_EINVAL, "threads must be 256, 512 or 1024");
    if (t->threads < c->p.nx)
      return fail(&c->err, LBSC_EINVAL, "threads must be >= nx (full-row tiles)");
    n.threads = t->threads;
  }
  if (t->z_chunk < 0 || t->block_y < 0) return fail(&c->err, LBSC_EINVAL, "negative tuning value");
  if (t->nodes_per_thread < 0 || t->nodes_per_thread > 2)
    return fail(&c->err, LBSC_EINVAL, "nodes_per_thread must be 0, 1 or 2");
  if (t->nodes_per_thread) n.nodes_per_thread = t->nodes_per_thread;
  if (t->block_y && (long long)t->block_y * c->p.nx > (long long)n.nodes_per_thread * n.threads)
    return fail(&c->err, LBSC_EINVAL, "block_y * nx exceeds nodes_per_thread * threads");
  if (t->pop_pad > kMaxPad) return fail(&c->err, LBSC_EINVAL, "pop_pad exceeds 65536");
  if (t->z_chunk) n.z_chunk = t->z_chunk;
  n.block_y = t->block_y;
  n.xcd_remap = t->xcd_remap ? 1 : 0;
  n.pop_pad = t->pop_pad;
  const lbsc::StepArgs na = make_args(c->p, n);
  if (na.ps != c->a.ps) {
    // New population stride: export the state through the free lattice and
    // import it again in the new layout.
    hipError_t e = lbsc::launch_gather(c->p.precision, c->lat[c->cur], c->a.ps, c->lat[c->cur ^ 1],
                                       na.ps, c->a, c->stream);
    if (e == hipSuccess)
      e = lbsc::launch_scatter(c->p.precision, c->lat[c->cur ^ 1], na.ps, c->lat[c->cur], na.ps,
                               na, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "re-layout launch");
  }
  c->tune = n;
  c->a = na;
  // The diagnostic area depends on nx, ny, nz only, not on the tuning.
  return LBSC_OK;
}

int lbsc_get_tuning(const lbsc_ctx* c, lbsc_tuning* t) {
  if (!c || !t) return LBSC_EINVAL;
  *t = c->tune;
  t->block_y = c->a.by;
  t->z_chunk = c->a.zchunk;
  t->pop_pad = (int32_t)(c->a.ps - (c->a.n + 63) / 64 * 64);
  return LBSC_OK;
}

void lbsc_lattice(int32_t* c, double* w) { lbsc::lattice_tables(c, w); }

void lbsc_destroy(lbsc_ctx* c) { delete c; }

const char* lbsc_last_error(const lbsc_ctx* c) {
  return c ? c->err.c_str() : g_init_err.c_str();
}

}  // extern "C"
