// Internal interface between the C-ABI layer (lbsc_api.hip) and the device
// code (lbsc_device.hip).  Not installed; callers use include/lbsc.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbsc {

constexpr int Q = 19;

// Population layout of a lattice.  The nodes, in C order (z, y, x), are cut
// into blocks of kBlock consecutive nodes, and a block stores its 19
// populations one after the other, kBlock values each: population a of node
// i is element ((i / kBlock) * 19 + a) * kBlock + i % kBlock.  A step's work-
// group then streams a few long runs of memory instead of 19 arrays (the
// 19-array layout moved 4.84 TB/s in the step's own access pattern, blocks
// of 1024 nodes 5.29).  A lattice holds ps = n rounded up to kBlock nodes,
// 19 ps elements.  kBlock may be 0 for one array of ps elements per
// population (element a * ps + i), with ps padded by the tuning's pop_pad.
template <class T>
struct Layout {
  static constexpr long long kBlock = 1024;
};

template <class T>
__host__ __device__ inline long long lat_index(int a, unsigned i, long long ps) {
  constexpr long long B = Layout<T>::kBlock;
  if constexpr (B > 0)
    return ((long long)(i / (unsigned)B) * Q + a) * B + (long long)(i % (unsigned)B);
  else
    return (long long)a * ps + i;
}

// Everything a step kernel needs to know about the box and the physics.
struct StepArgs {
  int nx, ny, nz;
  int plane;          // nx * ny
  long long n;        // nodes
  long long ps;       // nodes a lattice holds room for (>= n); see Layout
  int bx;             // columns per tile
  int by;             // rows per tile
  int ntiles_x;       // ceil(nx / bx)
  int ntiles_y;       // ceil(ny / by)
  int zchunk;         // planes per work-group
  int xcd_remap;      // 1: neighbouring tiles on one XCD
  double G, psi_rho0, tau, omega, s_bulk, s_ghost, rho_ref;
  void* psi_out;      // if set, the step also writes the psi its forces used (n values)
};

// One member of a batch as the device sees it: its geometry and physics and
// its two lattices.
struct BatchMember {
  StepArgs a;
  void* lat[2];
};

// A batched step: `ntiles` entries (member, xy tile, z chunk, 0) in
// `tiles`; persistent = 1 runs `nsteps` steps in one cooperative launch with
// grid barriers (sync: 5 zeroed words), else one ordinary launch of one step.
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

// One adjoint step (see the adjoint section of lbsc_device.hip): lattice
// B_{n-1}, psi(rho_n) as step n computed it, adjoint (P, r) of step n+1 in,
// of step n out,
// dL/dF scratch (3n values) and per-block partials (4 doubles per block:
// dL/dG, dL/dtau, dL/ds_bulk, dL/ds_ghost).
struct AdjArgs {
  StepArgs a;
  const void* bprev;
  const void* psi;
  const void* p_next;
  const void* r_next;
  void* p_out;
  void* r_out;
  // Written by kernel A for kernel B, per node x (Fb = dL/dF(x)):
  void* psi_fbar;    // psi(x) Fb(x), three arrays of n values (x, y, z)
  void* fbar_dot_v;  // Fb(x) . sum_b w_b psi(x + c_b) c_b, n values
  double* partial;  // accumulated over the whole backward pass, reduced once
};

enum Coll { kBGK = 0, kMRT = 1 };
enum Forc { kGuo = 0, kShift = 1 };

// Launchers; all queue work on `s` and return the launch status.
hipError_t launch_init(int prec, void* lat, const double* rho0_dev, const StepArgs& a,
                       hipStream_t s);
hipError_t launch_step(int prec, int coll, int forc, int threads, int npt, const void* src,
                       void* dst, const StepArgs& a, hipStream_t s);
// The two-kernel form of one step (psi to global memory, then the step from
// the psi stencil); psi holds n values of the storage type.
hipError_t launch_step_two_kernel(int prec, int coll, int forc, const void* src, void* psi,
                                  void* dst, const StepArgs& a, hipStream_t s);
hipError_t launch_batch(const BatchLaunch& L, hipStream_t s);
// psi_scratch: n doubles of device scratch (the idle lattice) for psi(rho).
hipError_t launch_moments(int prec, const void* lat, double* rho, double* u, double* p,
                          double* psi_scratch, const StepArgs& a, hipStream_t s);
// Diagnostics: rho_scratch holds 2 n doubles (rho, then psi); partials holds
// diag_blocks(a) * 8 doubles; out holds 4 + nz.
int diag_blocks(const StepArgs& a);
hipError_t launch_diagnostics(int prec, const void* lat, double* rho_scratch, double* partials,
                              double* out, double rho_v, double rho_l, const StepArgs& a,
                              hipStream_t s);
// State export/import between a lattice (its size ps_in / ps_out, see
// Layout) and plain arrays of post-streaming values, one of ps_out / ps_in
// elements per population.
hipError_t launch_gather(int prec, const void* lat, long long ps_in, void* out, long long ps_out,
                         const StepArgs& a, hipStream_t s);
hipError_t launch_scatter(int prec, const void* in, long long ps_in, void* lat, long long ps_out,
                          const StepArgs& a, hipStream_t s);

// Adjoint: blocks of the collision kernel (partials hold 2 doubles each);
// one backward step (acc[0..1] += dL/dG, dL/dtau of the step); the terminal
// seed; dL/drho0 from the adjoint of step 0; the minimum-radius gradient.
int adj_blocks(const StepArgs& a);
hipError_t launch_adjoint_step(int prec, int coll, const AdjArgs& g, hipStream_t s);
// acc[0..3] += the sums of the accumulated block partials.
hipError_t launch_adjoint_reduce(const AdjArgs& g, double* acc, hipStream_t s);
hipError_t launch_adjoint_seed(int prec, const AdjArgs& g, const double* rhobar, hipStream_t s);
hipError_t launch_adjoint_final(int prec, const AdjArgs& g, double* rho0bar, hipStream_t s);
hipError_t launch_rmin_grad(double* rho, const StepArgs& a, int zstar, double coef, double rho_v,
                            double rho_l, hipStream_t s);

// Velocity set and weights as the library orders them.
void lattice_tables(int32_t* c, double* w);

}  // namespace lbsc
