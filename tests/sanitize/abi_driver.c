/* Drives the host-only entry points of the HIP library (configuration
 * validation, size queries, derived constants, early argument checks of
 * mclbm_create, checkpoint-header parsing of good and damaged files) for an
 * AddressSanitizer / UndefinedBehaviorSanitizer build of the library's host
 * code (test infrastructure).  No call here touches a GPU.  Exit status 0
 * when every call returns the expected status. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mclbm.h"

static int failures = 0;
#define EXPECT(cond)                                                    \
  do {                                                                  \
    if (!(cond)) {                                                      \
      fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

static void hex(const void* p, size_t n, char* out) {
  static const char* d = "0123456789abcdef";
  const unsigned char* b = (const unsigned char*)p;
  for (size_t k = 0; k < n; ++k) {
    out[2 * k] = d[b[k] >> 4];
    out[2 * k + 1] = d[b[k] & 15];
  }
  out[2 * n] = '\0';
}

/* A checkpoint header line as the library writes it (the fields the reader
 * uses), followed by `tail`; `cfg_hex` / `xi_hex` may be overridden. */
static void write_ckpt(const char* path, const char* format, int version, const char* cfg_hex,
                       const char* xi_hex, const char* t_field, const char* tail) {
  FILE* fp = fopen(path, "wb");
  if (!fp) {
    ++failures;
    return;
  }
  fprintf(fp, "{\"format\": \"%s\", \"version\": %d, \"abi\": %d, %s\"config_hex\": \"%s\", \"xi_hex\": \"%s\", "
              "\"sections\": []}%s",
          format, version, MCLBM_ABI_VERSION, t_field, cfg_hex, xi_hex, tail);
  fclose(fp);
}

static void configs(void) {
  mclbm_config c;
  mclbm_config_defaults(&c);
  EXPECT(c.nx == 64 && c.ny == 64 && c.force_mask == MCLBM_F_ALL);
  EXPECT(mclbm_device_bytes(&c) > 0);
  EXPECT(mclbm_device_bytes(NULL) == 0);
  double d[MCLBM_D_COUNT + 4];
  EXPECT(mclbm_derive_constants(&c, d, MCLBM_D_COUNT) == MCLBM_OK);
  EXPECT(isfinite(d[MCLBM_D_DT]) && d[MCLBM_D_DT] > 0.0);
  EXPECT(mclbm_derive_constants(&c, d, MCLBM_D_COUNT - 1) != MCLBM_OK);
  EXPECT(mclbm_derive_constants(NULL, d, MCLBM_D_COUNT) != MCLBM_OK);
  EXPECT(mclbm_derive_constants(&c, NULL, 0) == MCLBM_EINVAL);  /* valid, but no room */

  /* invalid configurations, one field at a time */
  for (int k = 0; k < 16; ++k) {
    mclbm_config b = c;
    switch (k) {
      case 0: b.nx = 3; break;
      case 1: b.ny = 1 << 20; break;
      case 2: b.Ra = NAN; break;
      case 3: b.Ra = -1.0; break;
      case 4: b.Pr = 0.0; break;
      case 5: b.phi0 = 0.5; break;
      case 6: b.dp_m = -1e-9; break;
      case 7: b.tau_f = 0.5; break;
      case 8: b.storage = 7; break;
      case 9: b.block_x = 48; break;
      case 10: b.block_x = 256; b.block_y = 4; break;
      case 11: b.thermal_lattices = 3; break;
      case 12: b.reading_flags = 1u << 10; break;
      case 13: b.steps_per_launch = 3; break;
      case 14: b.force_mask = 1u << 7; break;
      case 15: b.dT_K = INFINITY; break;
    }
    EXPECT(mclbm_device_bytes(&b) == 0);
    EXPECT(strlen(mclbm_last_error()) > 0);
    EXPECT(mclbm_derive_constants(&b, d, MCLBM_D_COUNT) != MCLBM_OK);
  }

  /* batches: mixed storage types are rejected */
  mclbm_config two[2] = {c, c};
  EXPECT(mclbm_batch_device_bytes(two, 2) > 0);
  two[1].storage = MCLBM_FP16S;
  EXPECT(mclbm_batch_device_bytes(two, 2) == 0);
  EXPECT(mclbm_batch_device_bytes(two, 0) == 0);
  EXPECT(mclbm_batch_device_bytes(NULL, 1) == 0);

  /* create: argument checks that come before any device work */
  mclbm_cavity* cav = (mclbm_cavity*)0x1;
  EXPECT(mclbm_create(&c, NULL, NULL, 0, NULL, &cav) == MCLBM_EINVAL && cav == NULL);
  EXPECT(mclbm_create(&c, NULL, (void*)0x1000, mclbm_device_bytes(&c) - 1, NULL, &cav) == MCLBM_ENOMEM);
  EXPECT(mclbm_create(&c, NULL, (void*)0x1001, mclbm_device_bytes(&c), NULL, &cav) == MCLBM_EINVAL);
  EXPECT(mclbm_create(&c, NULL, (void*)0x1000, 1u << 30, NULL, NULL) == MCLBM_EINVAL);
  mclbm_config bad = c;
  bad.nx = 2;
  EXPECT(mclbm_create(&bad, NULL, (void*)0x1000, 1u << 30, NULL, &cav) == MCLBM_EINVAL);
  EXPECT(mclbm_residual_noalloc(NULL, NULL) == MCLBM_EINVAL);
  EXPECT(strlen(mclbm_version()) > 0 && mclbm_abi_version() == MCLBM_ABI_VERSION);
}

static void checkpoints(const char* dir) {
  char path[4096];
  snprintf(path, sizeof path, "%s/h.ckpt", dir);
  mclbm_config c;
  mclbm_config_defaults(&c);
  c.nx = 7;
  c.ny = 5;
  c.Ra = 2.5e4;
  c.block_x = c.block_y = 0;
  c.steps_per_launch = 0;
  static char cfg_hex[2 * sizeof(mclbm_config) + 1];
  hex(&c, sizeof c, cfg_hex);
  double xi[35];
  for (int k = 0; k < 35; ++k) xi[k] = (k % 7) / 3.5 - 1.0;
  static char xi_hex[2 * sizeof xi + 1];
  hex(xi, sizeof xi, xi_hex);

  mclbm_config got;
  int64_t t = -1;
  double xo[35];
  size_t n = 99;
  /* a good header, with and without the perturbation field */
  write_ckpt(path, "mclbm-checkpoint", 2, cfg_hex, xi_hex, "\"t\": 41, ", "\nraw");
  EXPECT(mclbm_checkpoint_info(path, &got, &t, xo, 35, &n) == MCLBM_OK);
  EXPECT(t == 41 && n == 35 && got.nx == 7 && got.ny == 5 && got.Ra == 2.5e4);
  EXPECT(memcmp(xo, xi, sizeof xi) == 0);
  EXPECT(mclbm_checkpoint_info(path, NULL, NULL, xo, 34, NULL) == MCLBM_EINVAL);
  EXPECT(mclbm_checkpoint_info(path, NULL, NULL, NULL, 0, NULL) == MCLBM_OK);
  write_ckpt(path, "mclbm-checkpoint", 2, cfg_hex, "", "\"t\": 0, ", "\n");
  EXPECT(mclbm_checkpoint_info(path, &got, &t, xo, 35, &n) == MCLBM_OK && n == 0 && t == 0);

  /* damaged headers */
  static char buf[2 * sizeof(mclbm_config) + 8];
  struct {
    const char *format, *cfg, *xi, *t, *tail;
    int version;
  } cases[12];
  int m = 0;
  cases[m++] = (typeof(cases[0])){"mclbm-checkpoinx", cfg_hex, xi_hex, "\"t\": 1, ", "\n", 2};
  cases[m++] = (typeof(cases[0])){"mclbm-checkpoint", cfg_hex, xi_hex, "\"t\": 1, ", "\n", 1};
  cases[m++] = (typeof(cases[0])){"mclbm-checkpoint", cfg_hex + 2, xi_hex, "\"t\": 1, ", "\n", 2};
  strcpy(buf, cfg_hex);
  buf[10] = 'g';
  cases[m++] = (typeof(cases[0])){"mclbm-checkpoint", buf, xi_hex, "\"t\": 1, ", "\n", 2};
  cases[m++] = (typeof(cases[0])){"mclbm-checkpoint", cfg_hex, xi_hex + 16, "\"t\": 1, ", "\n", 2};
  cases[m++] = (typeof(cases[0])){"mclbm-checkpoint", cfg_hex, xi_hex, "", "\n", 2};
  cases[m++] = (typeof(cases[0])){"mclbm-checkpoint", cfg_hex, xi_hex, "\"t\": -3, ", "\n", 2};
  cases[m++] = (typeof(cases[0])){"mclbm-checkpoint", cfg_hex, xi_hex, "\"t\": x, ", "\n", 2};
  cases[m++] = (typeof(cases[0])){"mclbm-checkpoint", "", xi_hex, "\"t\": 1, ", "\n", 2};
  for (int k = 0; k < m; ++k) {
    write_ckpt(path, cases[k].format, cases[k].version, cases[k].cfg, cases[k].xi, cases[k].t, cases[k].tail);
    t = 1234;
    EXPECT(mclbm_checkpoint_info(path, &got, &t, xo, 35, &n) == MCLBM_EINVAL);
    EXPECT(t == 1234);
  }
  /* a configuration that decodes but is invalid */
  mclbm_config inv = c;
  inv.nx = 1;
  hex(&inv, sizeof inv, buf);
  write_ckpt(path, "mclbm-checkpoint", 2, buf, "", "\"t\": 1, ", "\n");
  EXPECT(mclbm_checkpoint_info(path, &got, &t, xo, 35, &n) == MCLBM_EINVAL);
  /* empty file, a file without a newline, a missing file */
  FILE* fp = fopen(path, "wb");
  if (fp) fclose(fp);
  EXPECT(mclbm_checkpoint_info(path, &got, &t, xo, 35, &n) == MCLBM_EINVAL);
  fp = fopen(path, "wb");
  if (fp) {
    fputs("{\"format\": \"mclbm-checkpoint\", \"version\": 2", fp);
    fclose(fp);
  }
  EXPECT(mclbm_checkpoint_info(path, &got, &t, xo, 35, &n) == MCLBM_EINVAL);
  snprintf(path, sizeof path, "%s/missing.ckpt", dir);
  EXPECT(mclbm_checkpoint_info(path, &got, &t, xo, 35, &n) == MCLBM_EINVAL);
  EXPECT(mclbm_checkpoint_info(NULL, &got, &t, xo, 35, &n) == MCLBM_EINVAL);
  EXPECT(mclbm_restore(NULL, path) == MCLBM_EINVAL);
  EXPECT(mclbm_checkpoint(NULL, path) == MCLBM_EINVAL);
}

int main(int argc, char** argv) {
  configs();
  checkpoints(argc > 1 ? argv[1] : ".");
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("abi host driver ok\n");
  return 0;
}
