/*
 * The C ABI from plain C, without Python: reads an initial density field
 * (nz*ny*nx float64, C order) from a file, runs a D3Q19 BGK box of the
 * given size through lbsc_init_fields / lbsc_step /
 * lbsc_interface_diagnostics, and prints the mass and minimum radius before
 * and after.  The device buffer comes from hipMalloc; the library borrows it.
 *
 *   abi_step rho0.bin nx ny nz steps rho_v rho_l
 *
 * Exit status 0 when every call succeeds and the mass is conserved to
 * 1e-12 relative.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "lbsc.h"

static int check(int rc, lbsc_ctx* c, const char* what) {
  if (rc != LBSC_OK) {
    fprintf(stderr, "%s failed (%d): %s\n", what, rc, lbsc_last_error(c));
    return 1;
  }
  return 0;
}

int main(int argc, char** argv) {
  if (argc != 8) {
    fprintf(stderr, "usage: %s rho0.bin nx ny nz steps rho_v rho_l\n", argv[0]);
    return 2;
  }
  lbsc_params p;
  p.nx = atoi(argv[2]);
  p.ny = atoi(argv[3]);
  p.nz = atoi(argv[4]);
  p.collision = LBSC_BGK;
  p.forcing = LBSC_FORCING_GUO;
  p.precision = LBSC_F64;
  p.G = -5.0;
  p.psi_rho0 = 1.0;
  p.tau = 1.0;
  p.s_bulk = 1.0;
  p.s_ghost = 1.2;
  p.rho_ref = 1.0;
  const long long steps = atoll(argv[5]);
  const double rho_v = atof(argv[6]), rho_l = atof(argv[7]);
  const size_t n = (size_t)p.nx * p.ny * p.nz;

  double* rho0 = malloc(n * sizeof(double));
  double* r_of_z = malloc((size_t)p.nz * sizeof(double));
  FILE* fh = fopen(argv[1], "rb");
  if (!rho0 || !r_of_z || !fh || fread(rho0, sizeof(double), n, fh) != n) {
    fprintf(stderr, "cannot read %zu doubles from %s\n", n, argv[1]);
    return 2;
  }
  fclose(fh);

  const size_t bytes = lbsc_state_bytes(&p);
  if (bytes == 0) {
    fprintf(stderr, "invalid parameters\n");
    return 2;
  }
  void* buf = NULL;
  if (hipMalloc(&buf, bytes) != hipSuccess) {
    fprintf(stderr, "hipMalloc of %zu bytes failed\n", bytes);
    return 2;
  }
  lbsc_ctx* c = NULL;
  int bad = check(lbsc_init_fields(&c, &p, rho0, buf, bytes, NULL), NULL, "lbsc_init_fields");
  lbsc_diag d0, d1;
  if (!bad) bad = check(lbsc_interface_diagnostics(c, rho_v, rho_l, &d0, r_of_z), c, "diagnostics");
  if (!bad) bad = check(lbsc_step(c, steps), c, "lbsc_step");
  if (!bad) bad = check(lbsc_interface_diagnostics(c, rho_v, rho_l, &d1, r_of_z), c, "diagnostics");
  if (!bad) {
    printf("mass0 %.17g\nmass1 %.17g\nr_min0 %.17g\nr_min1 %.17g\nsteps %lld\n", d0.mass,
           d1.mass, d0.r_min, d1.r_min, (long long)lbsc_step_count(c));
    if (!(fabs(d1.mass - d0.mass) <= 1e-12 * d0.mass)) {
      fprintf(stderr, "mass not conserved: %.17g -> %.17g\n", d0.mass, d1.mass);
      bad = 1;
    }
  }
  lbsc_destroy(c);
  hipFree(buf);
  free(rho0);
  free(r_of_z);
  return bad;
}
