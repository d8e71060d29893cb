/* Drives every entry point of the oracle once, for an AddressSanitizer /
 * UndefinedBehaviorSanitizer build (test infrastructure).  Exit status 0
 * when every call returns the expected status. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "mclbm_oracle.h"

/* On failure: report, then leave through the function's clean-up label so
 * that the leak checker reports only real leaks. */
#define CHECK(cond)                                                     \
  do {                                                                  \
    if (!(cond)) {                                                      \
      fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      rc = 1;                                                           \
      goto done;                                                        \
    }                                                                   \
  } while (0)

static int run(int thermal_lattices, int flags, const char* ckpt) {
  mo_config c;
  mclbm_oracle_config_defaults(&c);
  c.nx = 13;
  c.ny = 9;
  /* the literal gravity reading drives a much stronger flow: keep it stable */
  c.Ra = (flags & 2) ? 1e3 : 2e4;
  c.phi0 = 0.02;
  c.dp = 40e-9;
  c.thermal_lattices = thermal_lattices;
  c.reading_flags = flags;
  const size_t nn = (size_t)c.nx * c.ny;
  int rc = 0;
  mo_state* o = NULL;
  double *m = NULL, *pops = NULL, *f = NULL;
  double* xi = malloc(nn * sizeof(double));
  for (size_t k = 0; k < nn; ++k) xi[k] = (double)((k * 7919) % 200) / 100.0 - 1.0;
  CHECK(mclbm_oracle_create(&c, xi, &o) == 0);
  CHECK(mclbm_oracle_step(o, 25) == 0);
  m = malloc(11 * nn * sizeof(double));
  CHECK(mclbm_oracle_read_moments(o, 2047, m, 11 * nn) == 0);
  CHECK(mclbm_oracle_read_moments(o, 2047, m, 10 * nn) != 0);
  const size_t np = (size_t)(thermal_lattices == 2 ? 36 : 27) * nn;
  pops = malloc(np * sizeof(double));
  CHECK(mclbm_oracle_read_populations(o, pops, np) == 0);
  CHECK(mclbm_oracle_write_populations(o, pops, np) == 0);
  double a, b, k, ru, rt;
  CHECK(mclbm_oracle_nusselt(o, &a, &b, &k) == 0 && isfinite(a));
  CHECK(mclbm_oracle_residual(o, &ru, &rt) == 0);
  double d[32];
  CHECK(mclbm_oracle_derived(o, d, 32) == 0);
  double in[16] = {0.98, 0.0, 0.0, 0.08, 0.0, 0.0, 0.1}, out[64];
  CHECK(mclbm_oracle_node_forces(o, in, out) == 0);
  CHECK(mclbm_oracle_checkpoint(o, ckpt) == 0);
  CHECK(mclbm_oracle_step(o, 3) == 0);
  CHECK(mclbm_oracle_restore(o, ckpt) == 0);
  CHECK(mclbm_oracle_time(o) == 25);
  if (thermal_lattices != 2) {
    f = calloc(4 * nn, sizeof(double));
    for (size_t q = 0; q < nn; ++q) f[3 * nn + q] = 0.02;
    CHECK(mclbm_oracle_load_fields(o, f, f + nn, f + 2 * nn, f + 3 * nn, NULL) == 0);
  }
  double eq[9], fo[9];
  mclbm_oracle_equilibrium(1.0, 0.01, -0.02, eq);
  mclbm_oracle_forcing(1e-5, 2e-5, fo);
done:
  mclbm_oracle_destroy(o);
  free(xi);
  free(m);
  free(pops);
  free(f);
  return rc;
}

int main(int argc, char** argv) {
  const char* ckpt = argc > 1 ? argv[1] : "driver.ckpt";
  mclbm_oracle_set_threads(2);
  for (int tl = 1; tl <= 2; ++tl)
    for (int flags = 0; flags < 8; flags += 7)
      if (run(tl, flags, ckpt)) return 1;
  int rc = 0;
  mo_config bad;
  mclbm_oracle_config_defaults(&bad);
  bad.nx = 2;
  mo_state* o = NULL;
  CHECK(mclbm_oracle_create(&bad, NULL, &o) != 0 && o == NULL);
  puts("oracle driver ok");
done:
  return rc;
}
