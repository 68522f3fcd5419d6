// Internal interface between the C-ABI layer (lbsc_api.hip) and the device
// code (lbsc_device.hip).  Not installed; callers use include/lbsc.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbsc {

constexpr int Q = 19;

// Everything a step kernel needs to know about the box and the physics.
struct StepArgs {
  int nx, ny, nz;
  int plane;          // nx * ny
  long long n;        // nodes
  long long ps;       // stride between populations (elements), >= n
  int by;             // rows per tile
  int ntiles_y;       // ceil(ny / by)
  int zchunk;         // planes per work-group
  int xcd_remap;      // 1: neighbouring tiles on one XCD
  double G, psi_rho0, tau, omega, s_bulk, s_ghost, rho_ref;
};

// One member of a batch as the device sees it: its geometry and physics and
// its two lattices.
struct BatchMember {
  StepArgs a;
  void* lat[2];
};

// A batched step: `ntiles` entries (member, tile row, z chunk, 0) in
// `tiles`; persistent = 1 runs `nsteps` steps in one cooperative launch with
// grid barriers (sync: 3 zeroed words), else one ordinary launch of one step.
struct BatchLaunch {
  int prec, coll, forc, threads, npt;
  const BatchMember* members;
  const int4* tiles;
  int ntiles;
  int parity;
  int remap;
  size_t lds;
  int persistent;
  int nsteps;
  unsigned* sync;
  unsigned spin_limit;
};

enum Coll { kBGK = 0, kMRT = 1 };
enum Forc { kGuo = 0, kShift = 1 };

// Launchers; all queue work on `s` and return the launch status.
hipError_t launch_init(int prec, void* lat, const double* rho0_dev, const StepArgs& a,
                       hipStream_t s);
hipError_t launch_step(int prec, int coll, int forc, int threads, int npt, const void* src,
                       void* dst, const StepArgs& a, hipStream_t s);
hipError_t launch_batch(const BatchLaunch& L, hipStream_t s);
hipError_t launch_moments(int prec, const void* lat, double* rho, double* u, double* p,
                          const StepArgs& a, hipStream_t s);
// Diagnostics: partials holds diag_blocks(a) * 8 doubles; out holds 4 + nz.
int diag_blocks(const StepArgs& a);
hipError_t launch_diagnostics(int prec, const void* lat, double* rho_scratch, double* partials,
                              double* out, double rho_v, double rho_l, const StepArgs& a,
                              hipStream_t s);
// State export/import between the pull layout and post-streaming values;
// strides are per population, in elements.
hipError_t launch_gather(int prec, const void* lat, long long ps_in, void* out, long long ps_out,
                         const StepArgs& a, hipStream_t s);
hipError_t launch_scatter(int prec, const void* in, long long ps_in, void* lat, long long ps_out,
                          const StepArgs& a, hipStream_t s);

// Velocity set and weights as the library orders them.
void lattice_tables(int32_t* c, double* w);

}  // namespace lbsc
