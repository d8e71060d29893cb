/*
 * FP64 CPU oracle for the multi-component lattice Boltzmann step
 * (three D2Q9 lattices: base fluid f, nanoparticle phase p, temperature g).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU baseline of the benchmark can check the HIP path against
 * a plain, slow, obviously correct implementation.  The product path never
 * links, loads or calls it.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * The algorithm follows the paper's Section 2.d (Eqs 18-36) with the slip
 * forces of Table 1 and the effective-property models of Eqs 7-11.  Where
 * the paper is garbled or silent, the reading taken is stated at the point of
 * use in mclbm_oracle.c.
 */
#ifndef MCLBM_ORACLE_H
#define MCLBM_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MO_OK = 0, MO_EINVAL = -1, MO_ENOMEM = -2, MO_EDIVERGED = -4
};

/* Boundary modes.  CAVITY is the paper's problem (Section 2.d, Fig 2a).
 * The two others exist only to pin the oracle against closed forms:
 * CHANNEL = periodic in x, no-slip walls in y (body-force Poiseuille flow);
 * PERIODIC = periodic in x and y (uniform two-phase drag relaxation). */
enum { MO_CAVITY = 0, MO_CHANNEL = 1, MO_PERIODIC = 2 };

/* Slip-force switches (Table 1): drag, Brownian, thermophoresis, Saffman,
 * Magnus+rotation, gravity. */
enum {
  MO_F_DRAG = 1, MO_F_BROWN = 2, MO_F_THERMO = 4, MO_F_SAFF = 8,
  MO_F_MAGROT = 16, MO_F_GRAV = 32, MO_F_ALL = 63
};

/* Moment field bits for mclbm_oracle_read_moments. */
enum {
  MO_RHO_F = 1, MO_UX_F = 2, MO_UY_F = 4, MO_PHI = 8, MO_UX_P = 16,
  MO_UY_P = 32, MO_THETA = 64, MO_UX_NS = 128, MO_UY_NS = 256,
  MO_THETA_F = 512, MO_THETA_P = 1024
};

typedef struct {
  double rho, cp, k, beta, mu, d_mol; /* SI units */
} mo_material;

typedef struct {
  int32_t nx, ny;
  double Ra, Pr, phi0, dp;       /* dp in metres */
  double tau_f;                  /* <= 0: automatic (Mach cap) */
  double dT, T0;                 /* kelvin */
  uint32_t force_mask;
  double force_scale[6];         /* drag, Brownian, thermo, Saffman, MR, gravity */
  double phi_perturb_amp;        /* amplitude multiplying the xi field */
  mo_material fluid, particle;
  /* test-only knobs */
  int32_t boundary;              /* MO_CAVITY / MO_CHANNEL / MO_PERIODIC */
  double body_force[2];          /* extra uniform force density on f */
  double u_f_init[2], u_p_init[2];
  /* 1 (0 means 1): one thermal lattice for the suspension; 2: Eq 19 for
   * each phase, the suspension temperature by Eq 33 */
  int32_t thermal_lattices;
  /* alternative readings: 1 literal Eq 10a ratio k_f/k_p, 2 gravity on the
   * particles only (no reference weight on the fluid), 4 one common
   * equilibrium velocity for f and p weighted by rho/tau */
  uint32_t reading_flags;
} mo_config;

/* Derived-constant slots returned by mclbm_oracle_derived. */
enum {
  MO_D_NU_L = 0, MO_D_ALPHA_L, MO_D_H, MO_D_DX, MO_D_DT, MO_D_G_L,
  MO_D_GRAV_L, MO_D_CK, MO_D_R, MO_D_TAU_F, MO_D_RHOC_RATIO,
  MO_D_BETA_RATIO, MO_D_RHO_F0, MO_D_RHO_P0, MO_D_NU_F, MO_D_ALPHA_F,
  MO_D_COUNT
};

/* Per-node diagnostics of mclbm_oracle_node_forces (inputs and outputs in
 * lattice units). */
enum {
  MO_IN_RHO_F = 0, MO_IN_JX_F, MO_IN_JY_F, MO_IN_RHO_P, MO_IN_JX_P,
  MO_IN_JY_P, MO_IN_THETA, MO_IN_DPHI_DX, MO_IN_DPHI_DY, MO_IN_DTH_DX,
  MO_IN_DTH_DY, MO_IN_COUNT
};
enum {
  MO_OUT_FFX = 0, MO_OUT_FFY, MO_OUT_FPX, MO_OUT_FPY, MO_OUT_TAU_P,
  MO_OUT_TAU_TH, MO_OUT_ABX, MO_OUT_ABY, MO_OUT_ATX, MO_OUT_ATY,
  MO_OUT_ASX, MO_OUT_ASY, MO_OUT_AMRX, MO_OUT_AMRY, MO_OUT_AGX, MO_OUT_AGY,
  MO_OUT_DX, MO_OUT_DY, MO_OUT_BETA_L, MO_OUT_KAPPA, MO_OUT_R_K,
  MO_OUT_R_MU, MO_OUT_COUNT
};

typedef struct mo_state mo_state;

void mclbm_oracle_config_defaults(mo_config* cfg);
/* xi: nx*ny values in [-1, 1] (row-major, x fastest) or NULL.  The initial
 * particle volume fraction is max(phi0 + phi_perturb_amp * xi, 0). */
int mclbm_oracle_create(const mo_config* cfg, const double* xi, mo_state** out);
int mclbm_oracle_step(mo_state* o, int64_t nsteps);
int64_t mclbm_oracle_time(const mo_state* o);
int mclbm_oracle_load_fields(mo_state* o, const double* ux, const double* uy,
                             const double* theta, const double* phi,
                             const double* rho_f);
int mclbm_oracle_read_moments(const mo_state* o, uint32_t mask, double* out,
                              size_t n_doubles);
int mclbm_oracle_write_populations(mo_state* o, const double* in,
                                   size_t n_doubles);
int mclbm_oracle_read_populations(const mo_state* o, double* out,
                                  size_t n_doubles); /* [3 or 4][9][ny][nx] */
int mclbm_oracle_nusselt(const mo_state* o, double* nu_hot, double* nu_cold,
                         double* nu_hot_k);
int mclbm_oracle_residual(mo_state* o, double* res_u, double* res_theta);
int mclbm_oracle_derived(const mo_state* o, double* out, int n);
void mclbm_oracle_equilibrium(double a, double ux, double uy, double out[9]);
void mclbm_oracle_forcing(double Fx, double Fy, double out[9]);
int mclbm_oracle_node_forces(const mo_state* o, const double* in, double* out);
int mclbm_oracle_checkpoint(mo_state* o, const char* path);
int mclbm_oracle_restore(mo_state* o, const char* path);
void mclbm_oracle_destroy(mo_state* o);
void mclbm_oracle_set_threads(int n);
int mclbm_oracle_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
