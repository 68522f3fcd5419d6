/*
 * lbsc -- D3Q19 pseudo-potential (Shan-Chen) lattice Boltzmann step on AMD
 * Instinct MI355X (gfx950).
 *
 * The method is the one of Chiappini, Xue, Falcucci and Sbragaglia,
 * "Hydrodynamic behavior of the Pseudo-Potential lattice Boltzmann method for
 * interfacial flows" (arXiv:1905.09554), Sec. 2:
 *   - lattice Boltzmann equation with D3Q19 populations f_a(x, t),
 *     collide at x then stream to x + c_a                    (Eq. LBE)
 *   - SRT (BGK, rate 1/tau) or MRT (M^-1 Lambda M) collision (collision cases)
 *   - equilibrium f^eq of Eq. local_eq, moments of Eq. momentum
 *   - Shan-Chen force F = -G psi(x) sum_a w_a psi(x + c_a) c_a  (Eq. SC_force)
 *     with psi = rho0 (1 - exp(-rho / rho0))
 *   - forcing: Guo-like, u^b = u + F/(2 rho) (Eq. barycentric) plus the Guo
 *     source term, or the SRT velocity shift u' = u + tau F / rho (Eq. vel_shift)
 *   - equation of state P = rho c_s^2 + c_s^2 G psi^2 / 2    (Eq. EOS_SC)
 * on a fully periodic box L_x x L_y x L_z holding a liquid ligament (Sec. 3),
 * with the minimum ligament radius as diagnostic (Sec. 4, Fig. 5).
 *
 * Conventions for every call
 *   - Every call returns an lbsc_status (0 on success) and never aborts.
 *   - Host arrays are owned by the caller and copied.  Device memory is owned
 *     by the caller and borrowed: the library never allocates or frees device
 *     memory.  One caller buffer of lbsc_state_bytes() bytes holds the whole
 *     state (two population lattices plus a small reduction area).
 *   - Arrays are C order [z][y][x] (x fastest); populations [a][z][y][x].
 *   - Work is queued on the caller's HIP stream, asynchronously, unless the
 *     call says it synchronises.
 *   - Outputs are float64 whatever the storage precision.
 *   - On error, lbsc_last_error() returns a message; a HIP error maps to
 *     LBSC_EHIP with the HIP error string in the message.
 *   - A context is used by one host thread at a time.
 */
#ifndef LBSC_H
#define LBSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbsc_ctx lbsc_ctx;

typedef enum lbsc_status {
  LBSC_OK = 0,
  LBSC_EINVAL = -1,     /* invalid argument: parameters, sizes, input field */
  LBSC_ENOMEM = -2,     /* host allocation failed */
  LBSC_EHIP = -3,       /* a HIP runtime call or kernel launch failed */
  LBSC_ENONFINITE = -4, /* the state holds NaN or Inf (diagnostics found it) */
  LBSC_ESTATE = -5      /* call not valid in the context's current state */
} lbsc_status;

/* Collision operator (Sec. 2, the SRT and MRT cases of Omega_coll). */
enum { LBSC_BGK = 0, LBSC_MRT = 1 };
/* Forcing: Guo-like with barycentric velocity (Eq. barycentric) or the SRT
 * velocity shift (Eq. vel_shift; BGK only). */
enum { LBSC_FORCING_GUO = 0, LBSC_FORCING_SHIFT = 1 };
/* Storage precision: float64 populations, or float32 populations stored
 * shifted as g_a = f_a - w_a rho_ref with float32 arithmetic. */
enum { LBSC_F64 = 0, LBSC_F32_SHIFTED = 1 };

typedef struct lbsc_params {
  int32_t nx, ny, nz;  /* periodic box, x fastest; each >= 1, nx*ny*nz < 2^31 */
  int32_t collision;   /* LBSC_BGK or LBSC_MRT                                */
  int32_t forcing;     /* LBSC_FORCING_GUO or LBSC_FORCING_SHIFT (BGK only)   */
  int32_t precision;   /* LBSC_F64 or LBSC_F32_SHIFTED                        */
  double G;            /* interaction strength G_0 of Eq. SC_force (finite)   */
  double psi_rho0;     /* rho_0 of psi (the paper fixes 1.0); > 0             */
  double tau;          /* BGK relaxation time; MRT shear rate is 1/tau; > 0.5 */
  double s_bulk;       /* MRT rate of the energy (bulk) row, in (0, 2)        */
  double s_ghost;      /* MRT rate of the non-hydrodynamic rows, in (0, 2)    */
  double rho_ref;      /* shift of the float32 storage (ignored for F64)      */
} lbsc_params;

/* Result of lbsc_interface_diagnostics. */
typedef struct lbsc_diag {
  double mass;     /* sum_x rho                                              */
  double mom[3];   /* sum_x (j + F/2) = sum_x rho u^b                         */
  double r_min;    /* min_z r(z), r(z) = sqrt(A(z)/pi)                        */
  int32_t z_argmin;/* smallest z at which r(z) = r_min                        */
  int32_t reserved;
} lbsc_diag;

/* Kernel launch shape and population layout; the autotuner picks these.
 * threads, z_chunk, block_y, nodes_per_thread, block_x: 0 means the default;
 * pop_pad < 0 means the default.  A tile of the fused step is block_x columns
 * by block_y rows (block_x * block_y <= nodes_per_thread * threads); the
 * default block_x is the whole row when the work-group holds at least
 * min_rows rows (4 for float64, for 1024-thread groups and for rows wider
 * than half the group; 2 otherwise) and 2 nx <= threads, else the widest
 * multiple of 64 whose tile and halo ring (2 (block_x + 2) + 2 block_y nodes)
 * fit the work-group.  lbsc_default_tuning gives the whole default on the
 * host.  The populations are stored in blocks of 1024 consecutive nodes,
 * each block holding its 19 populations one after the other; pop_pad, the
 * padding of a layout with one array per population, is then ignored. */
typedef struct lbsc_tuning {
  int32_t threads;     /* work-group size of the fused step: 256, 512, 1024   */
  int32_t z_chunk;     /* planes marched per work-group (>= 1)                */
  int32_t xcd_remap;   /* 1: map neighbouring tiles onto one XCD (L2), 0: off;
                          < 0: the default (1 for a single box, 0 for a
                          batch)                                            */
  int32_t block_y;     /* rows per tile; 0 = as many as the work-group holds  */
  int32_t pop_pad;     /* padding between population arrays, <= 65536 (only
                          for one array per population; see above)        */
  int32_t nodes_per_thread; /* interior nodes each thread carries: 1 or 2      */
  int32_t persistent;  /* 1: all steps of one lbsc_step call in one cooperative
                          launch with grid barriers; 0: one launch per step   */
  int32_t block_x;     /* columns per tile; 0 = the default above             */
  int32_t two_kernel;  /* 1: the two-kernel form of the step (psi written to
                          global memory by one kernel, read as a stencil by
                          the next), a baseline for the fused kernel; single
                          box with one launch per step only; 0: fused       */
} lbsc_tuning;

/* Bytes of device memory a context with these parameters needs: two
 * population lattices of 19 nx * ny * nz values in the storage precision
 * (with room for 65536 padding elements per population), plus a reduction
 * area and the psi field of the two-kernel form of the step (nx * ny * nz
 * values).  Returns 0 for invalid parameters. */
size_t lbsc_state_bytes(const lbsc_params* p);

/* Creates a context and sets the initial state f_a(x) = w_a rho0(x) (zero
 * momentum; in float32 storage g_a = w_a (rho0 - rho_ref)).
 *   rho0_host  nx*ny*nz float64 densities, host memory, copied; every value
 *              must be finite and > 0.
 *   dev_buf    device buffer of dev_bytes >= lbsc_state_bytes(p) bytes,
 *              256-byte aligned, borrowed for the context's lifetime.
 *   hip_stream hipStream_t to queue work on; NULL is the default stream.
 * Initial geometry: Sec. 3 (perturbed cylinder) with densities from
 * flat-interface runs.  Synchronises the stream before returning. */
int lbsc_init_fields(lbsc_ctx** out, const lbsc_params* p, const double* rho0_host,
                     void* dev_buf, size_t dev_bytes, void* hip_stream);

/* Advances the state by nsteps >= 0 time steps (Eq. LBE with the force of
 * Eq. SC_force), asynchronously on the context's stream. */
int lbsc_step(lbsc_ctx* c, int64_t nsteps);

/* Number of steps taken since the state was set. */
int64_t lbsc_step_count(const lbsc_ctx* c);

/* Moments of the current state into caller DEVICE buffers (float64):
 *   rho_dev  N values, rho = sum_a f_a (Eq. momentum); required
 *   u_dev    3N values [3][z][y][x], barycentric velocity u^b (Eq. barycentric),
 *            or NULL
 *   p_dev    N values, pressure of Eq. EOS_SC, or NULL
 * Asynchronous on the context's stream. */
int lbsc_compute_moments(lbsc_ctx* c, double* rho_dev, double* u_dev, double* p_dev);

/* Interface diagnostics of the current state (Sec. 4, minimum ligament
 * radius): liquid area per z-slice A(z) = sum_{x,y} clamp((rho - rho_v) /
 * (rho_l - rho_v), 0, 1), r(z) = sqrt(A(z)/pi), r_min and its z; total mass
 * and momentum.  All sums in float64 with a fixed reduction order (bitwise
 * reproducible).  r_of_z_host: nz doubles or NULL.  Synchronises the stream.
 * Returns LBSC_ENONFINITE if the mass is not finite. */
int lbsc_interface_diagnostics(lbsc_ctx* c, double rho_v, double rho_l, lbsc_diag* out,
                               double* r_of_z_host);

/* For callers that cannot allocate device memory at the time of the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): lbsc_interface_diagnostics with its reduction scratch -- the
 * per-block partial sums and the results -- in a static device array of the
 * library instead of the context's buffer.  Same arguments, kernels and
 * results (bitwise) as lbsc_interface_diagnostics; the density and psi fields
 * still use the context's idle lattice, as there.  Calls no hipMalloc,
 * hipFree or other allocating routine, and takes no host heap memory except
 * for the message of an error it returns.
 *   Limit: the array holds 16 MiB per GPU, for the life of the process; a box
 *   needs nz * ceil(nx * ny / 4096) * 64 bytes of partials plus
 *   (4 + nz) * 8 bytes of results (rounded up to 256 bytes), so e.g.
 *   672 x 672 x 1792 fits; larger boxes return LBSC_EINVAL.
 *   The context's device must be current (LBSC_EINVAL otherwise).
 *   Every call on one GPU shares that GPU's array: calls that overlap in
 *   time on one GPU (other host threads, other streams) race and must be
 *   serialised by the caller.  Each call writes every value it reads, so
 *   nothing needs clearing between calls.  Synchronises the stream. */
int lbsc_interface_diagnostics_static(lbsc_ctx* c, double rho_v, double rho_l, lbsc_diag* out,
                                      double* r_of_z_host);

/* Copies the post-streaming populations f_a(x) of the current time step to
 * host memory: 19*N values [a][z][y][x] in the storage precision (float64 f,
 * or float32 g = f - w rho_ref), bytes = 19*N*size.  *step receives the step
 * counter (may be NULL).  Synchronises the stream. */
int lbsc_get_state(lbsc_ctx* c, void* host, size_t bytes, int64_t* step);

/* Replaces the state by populations in the layout of lbsc_get_state and sets
 * the step counter; resuming from a saved state is bitwise identical to an
 * uninterrupted run.  Synchronises the stream. */
int lbsc_set_state(lbsc_ctx* c, const void* host, size_t bytes, int64_t step);

/* ---------------------------------------------------------------- batches
 * Many independent periodic boxes (e.g. ligaments of uneven radius and
 * wavenumber for a dispersion sweep, Sec. 4 and Fig. 3 of the paper) stepped
 * together: one launch per step covers the tiles of every member, or, with
 * lbsc_tuning.persistent = 1, one cooperative launch runs all steps of an
 * lbsc_step call with a grid-wide barrier between steps (bounded wait: a
 * barrier that does not complete within about a second makes lbsc_step return
 * LBSC_EHIP instead of hanging).  Members share precision, collision and
 * forcing; box size, G, tau, rates and rho_ref may differ.  Each member's
 * result is bitwise identical to running it alone.
 */

/* Device bytes for a batch of n members (params[n]); 0 if invalid. */
size_t lbsc_batch_state_bytes(int32_t n, const lbsc_params* params);

/* Creates a batch context.  rho0_host[i]: member i's nx*ny*nz float64
 * densities (host, copied, finite and > 0).  dev_buf: >=
 * lbsc_batch_state_bytes bytes, 256-byte aligned, borrowed.  The calls for a
 * single box (lbsc_step, lbsc_get_tuning, ...) act on the whole batch or, for
 * per-box outputs, on member 0.  Synchronises the stream. */
int lbsc_init_batch(lbsc_ctx** out, int32_t n, const lbsc_params* params,
                    const double* const* rho0_host, void* dev_buf, size_t dev_bytes,
                    void* hip_stream);

/* Number of members (1 for a context from lbsc_init_fields). */
int32_t lbsc_batch_size(const lbsc_ctx* c);

/* Per-member versions of lbsc_compute_moments, lbsc_interface_diagnostics,
 * lbsc_get_state and lbsc_set_state (same arguments and layouts; member is
 * 0-based; the step counter is shared by all members). */
int lbsc_member_moments(lbsc_ctx* c, int32_t member, double* rho_dev, double* u_dev,
                        double* p_dev);
int lbsc_member_diagnostics(lbsc_ctx* c, int32_t member, double rho_v, double rho_l,
                            lbsc_diag* out, double* r_of_z_host);
int lbsc_member_get_state(lbsc_ctx* c, int32_t member, void* host, size_t bytes);
int lbsc_member_set_state(lbsc_ctx* c, int32_t member, const void* host, size_t bytes);

/* ---------------------------------------------------------------- adjoint
 * Reverse-mode gradients of a loss of the final density with respect to the
 * initial density rho0, the interaction strength G (Eq. SC_force) and the
 * relaxation time tau (BGK rate, or MRT shear rate 1/tau), by a hand-written
 * adjoint of the step (Guo forcing, BGK or MRT, float64 or float32 storage;
 * parameter gradients accumulated in float64).  Memory is held down by
 * checkpointing: the forward saves the state every `segment` steps; the
 * backward recomputes one segment at a time, keeping its lattices, and runs
 * the adjoint steps through it.  Single boxes only.
 */

/* Workspace bytes for nsteps steps with checkpoints every segment steps
 * (about (nsteps/segment + segment + 3) lattices plus segment psi
 * fields, the psi(rho) each recomputed step's forces used); 0 if invalid. */
size_t lbsc_adjoint_workspace_bytes(const lbsc_params* p, int64_t nsteps, int32_t segment);

/* Runs nsteps steps from the initial state (step counter 0), saving a
 * checkpoint every `segment` steps in the caller's device workspace
 * (borrowed until the next lbsc_adjoint_forward).  Asynchronous. */
int lbsc_adjoint_forward(lbsc_ctx* c, int64_t nsteps, int32_t segment, void* workspace,
                         size_t bytes);

/* Loss gradient for the minimum ligament radius of the current state
 * (Sec. 4, Fig. 5): writes dr_min/drho (N doubles, device) into rhobar_dev;
 * *r_min receives r_min.  Nodes strictly between rho_v and rho_l on the
 * argmin slice carry 1/(2 pi r_min (rho_l - rho_v)), all others 0.
 * Synchronises the stream; LBSC_EINVAL if r_min = 0 (broken ligament). */
int lbsc_rmin_gradient(lbsc_ctx* c, double rho_v, double rho_l, double* rhobar_dev,
                       double* r_min);

/* Backward pass after lbsc_adjoint_forward (the state must not have moved):
 * rhobar_dev = dL/drho of the final state (N doubles, device); outputs
 * dL/drho0 into rho0bar_dev (N doubles, device) and dL/dG, dL/dtau on the
 * host.  The current state is left unchanged.  Synchronises the stream. */
int lbsc_adjoint_backward(lbsc_ctx* c, const double* rhobar_dev, double* rho0bar_dev,
                          double* dL_dG, double* dL_dtau);

/* Gradients of the last lbsc_adjoint_backward with respect to the MRT bulk
 * and ghost relaxation rates s_bulk and s_ghost of lbsc_params (the rates of
 * the d'Humieres rows other than the shear rows, Sec. 2 MRT paragraph; both
 * 0 for BGK).  dL/dtau covers the shear rates 1/tau only: a caller that ties
 * s_bulk to 1/tau, as the paper's rate set does, adds
 * dL/ds_bulk * (-1/tau^2) itself.  Host outputs, either may be NULL.
 * LBSC_ESTATE before the first backward pass. */
int lbsc_adjoint_rate_gradients(const lbsc_ctx* c, double* dL_ds_bulk, double* dL_ds_ghost);

/* Overrides the launch shape of the fused step (see lbsc_tuning). */
int lbsc_set_tuning(lbsc_ctx* c, const lbsc_tuning* t);
int lbsc_get_tuning(const lbsc_ctx* c, lbsc_tuning* t);

/* The launch shape a context for these n boxes starts with, as
 * lbsc_get_tuning would report it (for a single box: the effective tile,
 * chunk and padding).  Host only: needs no GPU and no context.  Returns
 * LBSC_EINVAL for invalid parameters or a NULL t. */
int lbsc_default_tuning(const lbsc_params* p, int32_t n, lbsc_tuning* t);

/* Lattice of the library: velocities c[19][3] (cx, cy, cz) and weights w[19]
 * in the population order used by lbsc_get_state.  Either may be NULL. */
void lbsc_lattice(int32_t* c, double* w);

/* Destroys a context (NULL is allowed); the device buffer is not freed. */
void lbsc_destroy(lbsc_ctx* c);

/* Message of the last error on this context; with c == NULL, the last error
 * of a failed lbsc_init_fields on this thread. */
const char* lbsc_last_error(const lbsc_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* LBSC_H */
