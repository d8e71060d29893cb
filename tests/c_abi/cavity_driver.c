/* A plain C program on the C ABI of libmclbm (include/mclbm.h) and the HIP
 * runtime only: allocate the device buffer, create a cavity, step it, read
 * Nu and moments back, and print one JSON line.  The GPU test that runs it
 * compares the line with the FP64 oracle.
 *
 * usage: cavity_driver nx ny Ra phi0 dp_nm steps steps_per_launch */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "mclbm.h"

static int check(int rc, const char* what) {
  if (rc != MCLBM_OK) fprintf(stderr, "%s failed: %d (%s)\n", what, rc, mclbm_last_error());
  return rc;
}

int main(int argc, char** argv) {
  if (argc != 8) {
    fprintf(stderr, "usage: %s nx ny Ra phi0 dp_nm steps steps_per_launch\n", argv[0]);
    return 2;
  }
  if (mclbm_abi_version() != MCLBM_ABI_VERSION) {
    fprintf(stderr, "library ABI %d, header ABI %d\n", mclbm_abi_version(), MCLBM_ABI_VERSION);
    return 2;
  }
  mclbm_config cfg;
  mclbm_config_defaults(&cfg);
  cfg.nx = atoi(argv[1]);
  cfg.ny = atoi(argv[2]);
  cfg.Ra = atof(argv[3]);
  cfg.phi0 = atof(argv[4]);
  cfg.dp_m = atof(argv[5]) * 1e-9;
  const long steps = atol(argv[6]);
  cfg.steps_per_launch = atoi(argv[7]);

  /* an invalid configuration is refused with a message */
  mclbm_config bad = cfg;
  bad.nx = 2;
  if (mclbm_device_bytes(&bad) != 0 || mclbm_last_error()[0] == '\0') {
    fprintf(stderr, "an invalid configuration was accepted\n");
    return 1;
  }

  const size_t bytes = mclbm_device_bytes(&cfg);
  if (bytes == 0) {
    check(MCLBM_EINVAL, "mclbm_device_bytes");
    return 1;
  }
  void* buf = NULL;
  if (hipMalloc(&buf, bytes) != hipSuccess) {
    fprintf(stderr, "hipMalloc of %zu bytes failed\n", bytes);
    return 1;
  }
  int rc = 0;
  mclbm_cavity* c = NULL;
  double* m = NULL;
  if (check(mclbm_create(&cfg, NULL, buf, bytes, NULL, &c), "mclbm_create")) {
    rc = 1;
    goto done;
  }
  if (check(mclbm_step(c, steps), "mclbm_step")) {
    rc = 1;
    goto done;
  }
  double nu_hot, nu_cold, nu_k;
  if (check(mclbm_nusselt(c, &nu_hot, &nu_cold, &nu_k), "mclbm_nusselt")) {
    rc = 1;
    goto done;
  }
  const size_t nn = (size_t)cfg.nx * cfg.ny;
  m = (double*)malloc(3 * nn * sizeof(double));
  const uint32_t mask = MCLBM_PHI | MCLBM_THETA | MCLBM_UX_NS;  /* written in bit order */
  if (!m || check(mclbm_read_moments(c, mask, m, 3 * nn), "mclbm_read_moments")) {
    rc = 1;
    goto done;
  }
  double phi_sum = 0.0, theta_abs = 0.0, ux_max = 0.0;
  for (size_t k = 0; k < nn; ++k) {
    phi_sum += m[k];
    theta_abs += fabs(m[nn + k]);
    if (fabs(m[2 * nn + k]) > ux_max) ux_max = fabs(m[2 * nn + k]);
  }
  printf("{\"time\": %lld, \"nu_hot\": %.17g, \"nu_cold\": %.17g, \"nu_hot_k\": %.17g, "
         "\"phi_sum\": %.17g, \"theta_abs_sum\": %.17g, \"ux_ns_max\": %.17g, \"device_bytes\": %zu}\n",
         (long long)mclbm_time(c), nu_hot, nu_cold, nu_k, phi_sum, theta_abs, ux_max, bytes);
done:
  free(m);
  if (c) mclbm_destroy(c);
  hipFree(buf);
  return rc;
}
