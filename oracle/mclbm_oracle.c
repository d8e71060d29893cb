/*
 * FP64 CPU oracle of the multi-component lattice Boltzmann model (MCLBM) for
 * buoyancy-driven flow of a nanosuspension in a differentially heated cavity.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product path.  Plain two-array
 * ("AB") layout, unshifted FP64 populations, one plain loop per algorithm
 * step, OpenMP over rows (which does not change any arithmetic).
 *
 * Per time step (Section 2.d):
 *   S1 moments (Eqs 29-31) -> S2 mixture velocity and mass fraction (Eqs 25,
 *   32) -> S3 local properties and relaxation times (Eqs 7-11, 22-24) ->
 *   S4 gradients of the previous step's (phi, theta) -> S5 slip forces
 *   (Table 1, Eqs 6, 20) -> S6 BGK collision with forcing (Eqs 18, 19,
 *   26-28) -> S7 streaming and walls (Eqs 34-36) -> S8 keep (phi, theta).
 *
 * Readings of passages that are garbled or silent in the paper are marked
 * "Reading:" where they are used.
 *
 * Parity status per part: the equilibrium, forcing, streaming, walls,
 * conduction limit, drag integrator and Nusselt definition are pinned by
 * closed forms and invariants in the tests.  Of the slip forces (Table 1,
 * under the stated readings): the Magnus term is pinned to the Magnus time
 * scale of Table 2 (rate v_M / d_p, against the slip), the rotation term to
 * Table 2's rotation time scale and the sphere's area-to-volume ratio, the
 * drag coefficient to the Schiller-Naumann law (its value at Re_d = 1 and
 * its slope), the thermophoretic coefficient to its continuum (k*) and
 * free-molecular (C_m) limits, and the settling force to Archimedes'
 * principle.  Parity unpinned: the absolute prefactors of the Brownian force
 * (the factors of D_B and v_B), of the Saffman lift (K_S / 4) and the
 * thermophoretic constants C_S and C_t; these are checked only through
 * directions and scaling laws (the paper prints no value that could fix
 * them).
 */
#include "mclbm_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- D2Q9 lattice, Eqs 21 and 28 -------------------------------------- */
/* Order of Eq 21: rest; theta = 0, 90, 180, 270 deg; then the diagonals at
 * 45, 135, 225, 315 deg. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double WGT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                              1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* ---- physical constants ------------------------------------------------ */
static const double KB = 1.380649e-23; /* Boltzmann constant, J/K */
static const double GRAV = 9.81;       /* m/s^2 */
static const double PI = 3.14159265358979323846;

/* Table 1 constants. */
static const double C_S = 1.17, C_T = 2.18, C_M = 1.14; /* thermophoresis */
static const double K_S = 81.2;                         /* Saffman lift */

/* Wall temperatures of the zero-mean theta = (T - T0)/dT. */
static const double TH_HOT = 0.5, TH_COLD = -0.5;

typedef struct {
  double nu_f, alpha_f, R, nu_L, alpha_L, tau_f, H, dx, dt, G_L, grav_L, Ck;
  double rhoc_ratio, beta_ratio, rho_f0, rho_p0;
  double s[6]; /* force switches times scales: D, B, T, S, MR, G */
} Setup;

struct mo_state {
  mo_config cfg;
  Setup s;
  int nx, ny;
  size_t nn;
  int64_t t;
  double *f, *p, *g;    /* [9][nn], populations after streaming */
  double *fs, *ps, *gs; /* [9][nn], populations after collision */
  double *g2, *g2s;     /* particle thermal lattice (two thermal lattices) */
  int two_t;            /* two thermal lattices */
  double *phi_prev, *th_prev, *phi_cur, *th_cur;
  double *snap_ux, *snap_uy, *snap_th;
};

void mclbm_oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int mclbm_oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void mclbm_oracle_config_defaults(mo_config* c) {
  memset(c, 0, sizeof(*c));
  c->nx = c->ny = 64;
  c->Ra = 1e3;
  c->Pr = 6.2;
  c->phi0 = 0.01;
  c->dp = 100e-9;
  c->tau_f = 0.8;
  c->dT = 10.0;
  c->T0 = 300.0;
  c->force_mask = MO_F_ALL;
  for (int k = 0; k < 6; ++k) c->force_scale[k] = 1.0;
  c->phi_perturb_amp = 1e-6;
  /* Reading: the paper names water and alumina but gives no property
   * values; a fixed textbook set at 300 K is used. */
  c->fluid.rho = 997.1;
  c->fluid.cp = 4179.0;
  c->fluid.k = 0.613;
  c->fluid.beta = 2.1e-4;
  c->fluid.mu = 8.9e-4;
  c->fluid.d_mol = 0.384e-9;
  c->particle.rho = 3970.0;
  c->particle.cp = 765.0;
  c->particle.k = 40.0;
  c->particle.beta = 8.5e-6;
  c->particle.mu = 0.0;
  c->particle.d_mol = 0.0;
  c->boundary = MO_CAVITY;
  c->thermal_lattices = 1;
}

/* ---- setup: lattice units from Ra, Pr, tau_f (Eqs 16, 22) -------------- */
static int derive_setup(const mo_config* c, Setup* s) {
  const double N = (double)c->nx; /* hot-to-cold wall distance in nodes */
  s->nu_f = c->fluid.mu / c->fluid.rho;
  s->alpha_f = s->nu_f / c->Pr;
  s->R = c->particle.rho / c->fluid.rho;
  if (c->tau_f > 0.0) {
    /* Eq 22 with c = dx/dt = 1, c_s^2 = 1/3: nu = (2 tau - 1)/6 */
    s->nu_L = (2.0 * c->tau_f - 1.0) / 6.0;
  } else {
    /* Reading: automatic viscosity keeps the free-fall velocity
     * sqrt(Ra nu alpha)/N at or below 0.1 of the lattice sound speed. */
    const double umax = 0.1 / sqrt(3.0);
    double nu = 0.1;
    const double ufree = nu * sqrt(c->Ra / c->Pr) / N;
    if (ufree > umax) nu = umax * N / sqrt(c->Ra / c->Pr);
    s->nu_L = nu;
  }
  s->tau_f = 3.0 * s->nu_L + 0.5;
  s->alpha_L = s->nu_L / c->Pr;
  /* Ra of the base fluid (Eq 16 with base-fluid properties) fixes the
   * physical height; Ra = 0 (pure conduction) uses a 1 cm cavity. */
  if (c->Ra > 0.0)
    s->H = cbrt(c->Ra * s->nu_f * s->alpha_f / (GRAV * c->fluid.beta * c->dT));
  else
    s->H = 0.01;
  s->dx = s->H / N;
  s->dt = s->nu_L * s->dx * s->dx / s->nu_f;
  /* g beta dT in lattice units follows from Eq 16 directly. */
  s->G_L = c->Ra * s->nu_L * s->alpha_L / (N * N * N);
  s->grav_L = GRAV * s->dt * s->dt / s->dx;
  /* Eq 10a/10b evaluated at T0.  Reading: the conductivity ratio is taken as
   * k_p/k_f (the printed k_f/k_p would make the enhancement vanish). */
  {
    const double Re = c->fluid.rho * KB * c->T0 /
                      (3.0 * PI * c->fluid.mu * c->fluid.mu * c->fluid.d_mol);
    /* alternative reading: the ratio as printed, k_f/k_p */
    const double kr = (c->reading_flags & 1u) ? c->fluid.k / c->particle.k
                                              : c->particle.k / c->fluid.k;
    s->Ck = 64.7 * pow(c->fluid.d_mol / c->dp, 0.369) * pow(kr, 0.7476) *
            pow(c->Pr, 0.995) * pow(Re, 1.2321);
  }
  s->rhoc_ratio = (c->particle.rho * c->particle.cp) /
                  (c->fluid.rho * c->fluid.cp);
  s->beta_ratio = c->particle.beta / c->fluid.beta;
  s->rho_f0 = 1.0 - c->phi0;
  s->rho_p0 = s->R * c->phi0;
  for (int k = 0; k < 6; ++k)
    s->s[k] = ((c->force_mask >> k) & 1u) ? c->force_scale[k] : 0.0;
  return MO_OK;
}

/* ---- Eq 26/27: second-order equilibrium E_i(a, u) ---------------------- */
static double equilibrium(int i, double a, double ux, double uy) {
  const double eu = EX[i] * ux + EY[i] * uy;
  const double uu = ux * ux + uy * uy;
  /* c_s^2 = 1/3 */
  return WGT[i] * a * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

void mclbm_oracle_equilibrium(double a, double ux, double uy, double out[9]) {
  for (int i = 0; i < 9; ++i) out[i] = equilibrium(i, a, ux, uy);
}

/* Reading of the forcing term of Eq 18: S_i = W_i e_i.F / c_s^2 so that its
 * first moment is F (the printed W_i F e_i gives F/3). */
static double forcing(int i, double Fx, double Fy) {
  return 3.0 * WGT[i] * (EX[i] * Fx + EY[i] * Fy);
}

void mclbm_oracle_forcing(double Fx, double Fy, double out[9]) {
  for (int i = 0; i < 9; ++i) out[i] = forcing(i, Fx, Fy);
}

/* ---- S3 + S5: properties and forces at one node ------------------------ */
typedef struct {
  double rho_f, jx_f, jy_f, rho_p, jx_p, jy_p, theta;
  double dphi_dx, dphi_dy, dth_dx, dth_dy;
} NodeIn;

typedef struct {
  double ux_f, uy_f, ux_p, uy_p, ux_ns, uy_ns;
  double tau_p, tau_th;
  double Ffx, Ffy, Fpx, Fpy;
  double aB[2], aT[2], aS[2], aMR[2], aG[2], D[2];
  double beta_L, kappa, r_k, r_mu;
} NodeOut;

static void node_physics(const mo_state* o, const NodeIn* in, NodeOut* r) {
  const Setup* s = &o->s;
  const mo_config* c = &o->cfg;
  memset(r, 0, sizeof(*r));

  /* S1: Eqs 29-30 per component.  Reading: the lattices carry partial
   * densities, rho_p~ = R phi. */
  const double rho_f = in->rho_f, rho_p = in->rho_p;
  const double uxf = in->jx_f / rho_f, uyf = in->jy_f / rho_f;
  const int empty = !(rho_p > 1e-12);
  const double uxp = empty ? uxf : in->jx_p / rho_p;
  const double uyp = empty ? uyf : in->jy_p / rho_p;
  const double phi = rho_p / s->R;

  /* S2: Eq 32 read as the mass-averaged velocity; Eq 25 mass fraction. */
  const double rho_m = rho_f + rho_p;
  const double uxn = (in->jx_f + in->jx_p) / rho_m;
  const double uyn = (in->jy_f + in->jy_p) / rho_m;
  const double rbar_p = rho_p / rho_m;

  /* S3: Eqs 7-11 as ratios to the base fluid. */
  const double phic = phi > 0.0 ? phi : 0.0;
  const double r_rho = 1.0 + phi * (s->R - 1.0);                /* Eq 7 */
  const double r_rhoc = 1.0 + phi * (s->rhoc_ratio - 1.0);      /* Eq 8 */
  const double r_beta = 1.0 + phi * (s->beta_ratio - 1.0);      /* Eq 9 */
  const double r_k = 1.0 + s->Ck * pow(phic, 0.764);            /* Eq 10a */
  const double r_mu = 1.0 + 4.93 * phi + 222.4 * phi * phi;     /* Eq 11 */
  /* Eq 23 solved for the particle relaxation time, nu_ns from Eq 11/7. */
  const double nu_ns = s->nu_L * r_mu / r_rho;
  double tau_p;
  if (rbar_p <= 1e-12) {
    tau_p = s->tau_f;
  } else {
    tau_p = (3.0 * nu_ns + 0.5 - (1.0 - rbar_p) * s->tau_f) / rbar_p;
    if (tau_p < 0.505) tau_p = 0.505;
    if (tau_p > 5.0) tau_p = 5.0;
  }
  /* Eq 24 with one thermal lattice for the suspension: alpha_ns =
   * alpha_f k_ns/k_f / ((rho cp)_ns/(rho cp)_f). */
  const double tau_th = 3.0 * s->alpha_L * r_k / r_rhoc + 0.5;

  /* S5: slip forces of Table 1, evaluated in SI units and converted.
   * Reading: each force is the force on one particle; the force density on
   * the particle lattice is n_p F = rho_p~ F/m_p (Eq 4 per mixture volume),
   * so every term below is an acceleration per particle mass. */
  const double vel = s->dx / s->dt;          /* lattice -> SI velocity */
  const double acc = s->dt * s->dt / s->dx;  /* SI -> lattice acceleration */
  const double d = c->dp;
  const double Vp = PI * d * d * d / 6.0, Ap = PI * d * d;
  const double mp = c->particle.rho * Vp;
  const double mu_ns = c->fluid.mu * r_mu;
  const double rho_ns = c->fluid.rho * r_rho;
  const double T = c->T0 + c->dT * in->theta;

  /* slip velocity w = v_f - v_p and its +90 degree rotation */
  const double wx = uxf - uxp, wy = uyf - uyp;
  const double wn = sqrt(wx * wx + wy * wy);
  const double wpx = wn > 0.0 ? -wy / wn : 0.0;
  const double wpy = wn > 0.0 ? wx / wn : 0.0;
  const double up_si = sqrt(uxp * uxp + uyp * uyp) * vel;
  /* shear rate of Table 1 (Saffman row): 8 v_p / H */
  const double gdot = 8.0 * up_si / s->H;

  double aB[2] = {0, 0}, aT[2] = {0, 0}, aS[2] = {0, 0};
  double aMR[2] = {0, 0}, aG[2] = {0, 0}, D[2] = {0, 0};
  double beta_L = 0.0, kappa = 0.0;
  double Fpx = 0.0, Fpy = 0.0, Ffx, Ffy;

  /* buoyancy on the fluid lattice (Eq 20), Boussinesq with beta_ns (Eq 9) */
  Ffx = c->body_force[0];
  Ffy = c->body_force[1] + rho_m * r_beta * s->G_L * in->theta;

  if (s->s[5] != 0.0 && !(c->reading_flags & 2u)) {
    /* Reading: the settling force of Table 1 (particles) is referenced to
     * the uniform initial suspension; the fluid carries the opposite
     * uniform weight so that the mixture feels only (phi - phi0).  The
     * alternative (flag 2) is Table 1 as printed: particles only. */
    Ffy += s->s[5] * s->rho_p0 * (1.0 - 1.0 / s->R) * s->grav_L;
  }

  if (!empty) {
    /* Brownian (Table 1).  Reading: directed down the concentration
     * gradient. */
    if (s->s[1] != 0.0) {
      const double DB = 2.0 * KB * T / (3.0 * PI * mu_ns * d);
      const double vB = 2.0 * KB * T / (PI * mu_ns * d * d);
      const double coef = c->particle.rho * DB * Ap * vB / mp; /* per grad */
      aB[0] = -s->s[1] * coef * (in->dphi_dx / s->dx) * acc;
      aB[1] = -s->s[1] * coef * (in->dphi_dy / s->dx) * acc;
    }
    /* Thermophoresis (Table 1).  Reading: F_T = mu_ns d_p v_T (a force),
     * with v_T as printed; directed down the temperature gradient. */
    if (s->s[2] != 0.0) {
      const double kstar = c->fluid.k * r_k / c->particle.k;
      const double Kn = c->fluid.d_mol / d;
      const double CT = 6.0 * PI * C_S * (kstar + C_T * Kn) /
                        ((1.0 + 3.0 * C_M * Kn) *
                         (1.0 + 2.0 * kstar + 2.0 * C_T * Kn));
      const double gTx = c->dT * in->dth_dx / s->dx; /* K/m */
      const double gTy = c->dT * in->dth_dy / s->dx;
      const double vTx = CT * (mu_ns / rho_ns) * gTx / T;
      const double vTy = CT * (mu_ns / rho_ns) * gTy / T;
      aT[0] = -s->s[2] * mu_ns * d * vTx / mp * acc;
      aT[1] = -s->s[2] * mu_ns * d * vTy / mp * acc;
    }
    /* Saffman lift (Table 1).  Reading: square root on (rho gdot / mu),
     * directed along the rotated slip. */
    if (s->s[3] != 0.0) {
      const double FS = (K_S / 4.0) * mu_ns * (wn * vel) * d * d *
                        sqrt(rho_ns * gdot / mu_ns);
      aS[0] = s->s[3] * FS / mp * wpx * acc;
      aS[1] = s->s[3] * FS / mp * wpy * acc;
    }
    /* Magnus + particle rotation (Table 1).  Reading: v_M = (v_f + v_p)/2,
     * mass rate m_p |v_M| / d_p from tau_M = d_p / v_M of Table 2; the
     * rotation term times the particle area, along the rotated slip. */
    if (s->s[4] != 0.0) {
      const double vMx = 0.5 * (uxf + uxp) * vel, vMy = 0.5 * (uyf + uyp) * vel;
      const double vMn = sqrt(vMx * vMx + vMy * vMy);
      const double mdot = mp * vMn / d;
      const double FMx = mdot * (uxp * vel - vMx);
      const double FMy = mdot * (uyp * vel - vMy);
      const double FR = mu_ns * c->particle.rho * gdot / rho_ns * Ap;
      aMR[0] = s->s[4] * (FMx + FR * wpx) / mp * acc;
      aMR[1] = s->s[4] * (FMy + FR * wpy) / mp * acc;
    }
    /* Gravity (Table 1): F_G = -V_p (rho_p - rho_f) g */
    if (s->s[5] != 0.0) {
      aG[1] = -s->s[5] * Vp * (c->particle.rho - c->fluid.rho) * GRAV / mp *
              acc;
    }
    const double aIx = aB[0] + aT[0] + aS[0] + aMR[0];
    const double aIy = aB[1] + aT[1] + aS[1] + aMR[1];
    /* Reading: the interaction forces act on the fluid as reactions
     * (Eq 20 extended from drag and Brownian to every particle-fluid
     * interaction); gravity is external. */
    Ffx -= rho_p * aIx;
    Ffy -= rho_p * aIy;
    Fpx = rho_p * (aIx + aG[0]);
    Fpy = rho_p * (aIy + aG[1]);
    /* Drag (Table 1): F_D = beta m_p (v_f - v_p) on the particles,
     * beta = 18 mu C_d Re_d / (24 rho_p d^2) with Schiller-Naumann C_d.
     * Reading: beta dt ~ 1e4 makes explicit forcing unstable, so the
     * coupled two-phase relative-velocity equation dw/dt = a_rel - kappa w
     * is integrated exactly over the step and the mean drag is applied. */
    if (s->s[0] != 0.0) {
      const double Red = c->particle.rho * d * (wn * vel) / mu_ns;
      const double beta = 18.0 * mu_ns * (1.0 + 0.15 * pow(Red, 0.687)) /
                          (c->particle.rho * d * d);
      beta_L = s->s[0] * beta * s->dt;
      kappa = beta_L * (1.0 + rho_p / rho_f);
      const double arx = Ffx / rho_f - Fpx / rho_p;
      const double ary = Ffy / rho_f - Fpy / rho_p;
      /* mean of w over the step: w_inf + (w - w_inf)(1 - e^-k)/k with
       * w_inf = a_rel / kappa */
      const double ph1 = -expm1(-kappa) / kappa;
      double ph2; /* (1 - ph1)/kappa, series for small kappa */
      if (kappa < 1e-4)
        ph2 = 0.5 - kappa / 6.0 + kappa * kappa / 24.0;
      else
        ph2 = (1.0 - ph1) / kappa;
      const double wmx = wx * ph1 + arx * ph2;
      const double wmy = wy * ph1 + ary * ph2;
      D[0] = rho_p * beta_L * wmx;
      D[1] = rho_p * beta_L * wmy;
      Fpx += D[0];
      Fpy += D[1];
      Ffx -= D[0];
      Ffy -= D[1];
    }
  }

  r->ux_f = uxf; r->uy_f = uyf; r->ux_p = uxp; r->uy_p = uyp;
  r->ux_ns = uxn; r->uy_ns = uyn;
  r->tau_p = tau_p; r->tau_th = tau_th;
  r->Ffx = Ffx; r->Ffy = Ffy; r->Fpx = Fpx; r->Fpy = Fpy;
  memcpy(r->aB, aB, sizeof aB); memcpy(r->aT, aT, sizeof aT);
  memcpy(r->aS, aS, sizeof aS); memcpy(r->aMR, aMR, sizeof aMR);
  memcpy(r->aG, aG, sizeof aG); memcpy(r->D, D, sizeof D);
  r->beta_L = beta_L; r->kappa = kappa; r->r_k = r_k; r->r_mu = r_mu;
}

/* ---- S4 helpers: previous-step fields with wall ghosts ----------------- */
static int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

static double phi_at(const mo_state* o, int x, int y) {
  const int nx = o->nx, ny = o->ny, b = o->cfg.boundary;
  if (b != MO_CAVITY) x = wrap(x, nx);
  if (b == MO_PERIODIC) y = wrap(y, ny);
  /* zero-flux walls: mirror ghost */
  if (x < 0) x = 0;
  if (x >= nx) x = nx - 1;
  if (y < 0) y = 0;
  if (y >= ny) y = ny - 1;
  return o->phi_prev[(size_t)y * nx + x];
}

static double theta_at(const mo_state* o, int x, int y) {
  const int nx = o->nx, ny = o->ny, b = o->cfg.boundary;
  if (b != MO_CAVITY) x = wrap(x, nx);
  if (b == MO_PERIODIC) y = wrap(y, ny);
  if (y < 0) y = 0;          /* adiabatic: mirror */
  if (y >= ny) y = ny - 1;
  /* isothermal: linear ghost through the wall value at half a spacing */
  if (x < 0) return 2.0 * TH_HOT - o->th_prev[(size_t)y * nx + 0];
  if (x >= nx) return 2.0 * TH_COLD - o->th_prev[(size_t)y * nx + nx - 1];
  return o->th_prev[(size_t)y * nx + x];
}

/* ---- create / destroy -------------------------------------------------- */
static void free_state(mo_state* o) {
  if (!o) return;
  free(o->f); free(o->p); free(o->g);
  free(o->fs); free(o->ps); free(o->gs);
  free(o->g2); free(o->g2s);
  free(o->phi_prev); free(o->th_prev); free(o->phi_cur); free(o->th_cur);
  free(o->snap_ux); free(o->snap_uy); free(o->snap_th);
  free(o);
}

void mclbm_oracle_destroy(mo_state* o) { free_state(o); }

/* Temperatures at node n: the fluid's (first thermal lattice), the
 * particles' (second thermal lattice, or the same one) and the
 * suspension's, by Eq 33 over the two lattices.  Reading of Eq 33: the
 * denominator carries the heat capacities as the numerator does (printed
 * without them, the expression is not a temperature), so theta_ns is the
 * average weighted by heat capacity per volume, (rho c_p)_f (1 - phi) and
 * (rho c_p)_p phi. */
static void node_temps(const mo_state* o, size_t n, double rho_p, double* th_f,
                       double* th_p, double* th_ns) {
  const size_t nn = o->nn;
  double tf = 0.0;
  for (int i = 0; i < 9; ++i) tf += o->g[i * nn + n];
  *th_f = tf;
  if (!o->two_t) {
    *th_p = tf;
    *th_ns = tf;
    return;
  }
  double tp = 0.0;
  for (int i = 0; i < 9; ++i) tp += o->g2[i * nn + n];
  double phi = rho_p / o->s.R;
  if (phi < 0.0) phi = 0.0;
  const double cf = 1.0 - phi, cp = o->s.rhoc_ratio * phi;
  *th_p = tp;
  *th_ns = (cf * tf + cp * tp) / (cf + cp);
}

static void node_moments(const mo_state* o, size_t n, double* rho_f,
                         double* jxf, double* jyf, double* rho_p, double* jxp,
                         double* jyp, double* th) {
  const size_t nn = o->nn;
  double a = 0, bx = 0, by = 0, c = 0, cx = 0, cy = 0;
  for (int i = 0; i < 9; ++i) {
    const double fi = o->f[i * nn + n], pi = o->p[i * nn + n];
    a += fi; bx += fi * EX[i]; by += fi * EY[i];
    c += pi; cx += pi * EX[i]; cy += pi * EY[i];
  }
  double tf, tp;
  node_temps(o, n, c, &tf, &tp, th);
  *rho_f = a; *jxf = bx; *jyf = by; *rho_p = c; *jxp = cx; *jyp = cy;
}

/* Lag fields of the first step and the residual snapshot, from the
 * populations of the initial state. */
static void init_lag_and_snapshot(mo_state* o) {
  const size_t nn = o->nn;
  for (size_t n = 0; n < nn; ++n) {
    double rf, jxf, jyf, rp, jxp, jyp, th;
    node_moments(o, n, &rf, &jxf, &jyf, &rp, &jxp, &jyp, &th);
    o->phi_prev[n] = rp / o->s.R;
    o->th_prev[n] = th;
    o->snap_ux[n] = (jxf + jxp) / (rf + rp);
    o->snap_uy[n] = (jyf + jyp) / (rf + rp);
    o->snap_th[n] = th;
  }
}

int mclbm_oracle_create(const mo_config* cfg, const double* xi,
                        mo_state** out) {
  if (!cfg || !out) return MO_EINVAL;
  *out = NULL;
  if (cfg->nx < 4 || cfg->ny < 4) return MO_EINVAL;
  if (!(cfg->Ra >= 0.0) || !(cfg->Pr > 0.0) || !(cfg->phi0 >= 0.0) ||
      !(cfg->phi0 <= 0.1) || !(cfg->dp > 0.0))
    return MO_EINVAL;
  if (cfg->tau_f > 0.0 && !(cfg->tau_f > 0.5)) return MO_EINVAL;
  if (cfg->thermal_lattices < 0 || cfg->thermal_lattices > 2) return MO_EINVAL;
  if (cfg->reading_flags & ~7u) return MO_EINVAL;
  mo_state* o = (mo_state*)calloc(1, sizeof(mo_state));
  if (!o) return MO_ENOMEM;
  o->cfg = *cfg;
  o->nx = cfg->nx;
  o->ny = cfg->ny;
  o->nn = (size_t)cfg->nx * (size_t)cfg->ny;
  derive_setup(cfg, &o->s);
  const size_t nn = o->nn;
  o->f = malloc(9 * nn * sizeof(double));
  o->p = malloc(9 * nn * sizeof(double));
  o->g = malloc(9 * nn * sizeof(double));
  o->two_t = cfg->thermal_lattices == 2;
  if (o->two_t) {
    o->g2 = malloc(9 * nn * sizeof(double));
    o->g2s = malloc(9 * nn * sizeof(double));
  }
  o->fs = malloc(9 * nn * sizeof(double));
  o->ps = malloc(9 * nn * sizeof(double));
  o->gs = malloc(9 * nn * sizeof(double));
  o->phi_prev = malloc(nn * sizeof(double));
  o->th_prev = malloc(nn * sizeof(double));
  o->phi_cur = malloc(nn * sizeof(double));
  o->th_cur = malloc(nn * sizeof(double));
  o->snap_ux = malloc(nn * sizeof(double));
  o->snap_uy = malloc(nn * sizeof(double));
  o->snap_th = malloc(nn * sizeof(double));
  if (!o->f || !o->p || !o->g || !o->fs || !o->ps || !o->gs || !o->phi_prev ||
      !o->th_prev || !o->phi_cur || !o->th_cur || !o->snap_ux ||
      !o->snap_uy || !o->snap_th || (o->two_t && (!o->g2 || !o->g2s))) {
    free_state(o);
    return MO_ENOMEM;
  }
  /* Initial state: equilibrium at the initial velocities (zero in the
   * cavity), rho_f~ = 1 - phi0, rho_p~ = R phi(x), theta = 0. */
  for (size_t n = 0; n < nn; ++n) {
    double phi = cfg->phi0;
    if (xi) phi += cfg->phi_perturb_amp * xi[n];
    if (phi < 0.0) phi = 0.0;
    const double rf = o->s.rho_f0, rp = o->s.R * phi;
    for (int i = 0; i < 9; ++i) {
      o->f[i * nn + n] = equilibrium(i, rf, cfg->u_f_init[0], cfg->u_f_init[1]);
      o->p[i * nn + n] = equilibrium(i, rp, cfg->u_p_init[0], cfg->u_p_init[1]);
      o->g[i * nn + n] = 0.0;
      if (o->two_t) o->g2[i * nn + n] = 0.0;
    }
  }
  init_lag_and_snapshot(o);
  o->t = 0;
  *out = o;
  return MO_OK;
}

/* Difference of a node field along x (dx = 1) or y (dx = 0): central
 * inside, one-sided at the first and last node. */
static double field_diff(const double* a, int nx, int ny, int x, int y, int along_x) {
  const int n = y * nx + x;
  if (along_x) {
    if (x == 0) return a[n + 1] - a[n];
    if (x == nx - 1) return a[n] - a[n - 1];
    return 0.5 * (a[n + 1] - a[n - 1]);
  }
  if (y == 0) return a[n + nx] - a[n];
  if (y == ny - 1) return a[n] - a[n - nx];
  return 0.5 * (a[n + nx] - a[n - nx]);
}

/* Warm start from given fields (fluid partial density rho_f, NULL: 1 - phi0
 * of the cold start; rho_p~ = R phi; the mixture velocity for both phases):
 * every node takes the second-order equilibria (Eqs 26-27) plus the
 * first-order non-equilibrium parts of the Chapman-Enskog expansion of the
 * BGK lattices (Eqs 18-19): -3 tau_f W_i rho_f (e_i e_i - I/3) : grad u on
 * the fluid lattice and -tau_theta W_i e_i . grad theta on the temperature
 * lattice (tau_theta of Eq 24 at the node's phi), with gradients by node
 * differences; the particle lattice takes its equilibrium.  Time restarts
 * at 0. */
int mclbm_oracle_load_fields(mo_state* o, const double* ux, const double* uy,
                             const double* theta, const double* phi,
                             const double* rho_f) {
  if (!o || !ux || !uy || !theta || !phi || o->two_t) return MO_EINVAL;
  const int nx = o->nx, ny = o->ny;
  const Setup* s = &o->s;
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      const size_t n = (size_t)y * nx + x, nn = o->nn;
      const double rf = rho_f ? rho_f[n] : s->rho_f0, rp = s->R * phi[n];
      const double dxux = field_diff(ux, nx, ny, x, y, 1), dyux = field_diff(ux, nx, ny, x, y, 0);
      const double dxuy = field_diff(uy, nx, ny, x, y, 1), dyuy = field_diff(uy, nx, ny, x, y, 0);
      const double dxth = field_diff(theta, nx, ny, x, y, 1), dyth = field_diff(theta, nx, ny, x, y, 0);
      const double phic = phi[n] > 0.0 ? phi[n] : 0.0;
      const double r_k = 1.0 + s->Ck * pow(phic, 0.764);
      const double r_rhoc = 1.0 + phi[n] * (s->rhoc_ratio - 1.0);
      const double tau_th = 3.0 * s->alpha_L * r_k / r_rhoc + 0.5;
      for (int i = 0; i < 9; ++i) {
        /* grad u contracted with e_i e_i - I/3 */
        const double qgu = (EX[i] * EX[i] - 1.0 / 3.0) * dxux + (EY[i] * EY[i] - 1.0 / 3.0) * dyuy +
                           EX[i] * EY[i] * (dxuy + dyux);
        o->f[i * nn + n] = equilibrium(i, rf, ux[n], uy[n]) - 3.0 * s->tau_f * WGT[i] * rf * qgu;
        o->p[i * nn + n] = equilibrium(i, rp, ux[n], uy[n]);
        o->g[i * nn + n] = equilibrium(i, theta[n], ux[n], uy[n]) -
                           tau_th * WGT[i] * (EX[i] * dxth + EY[i] * dyth);
      }
    }
  }
  init_lag_and_snapshot(o);
  o->t = 0;
  return MO_OK;
}

int64_t mclbm_oracle_time(const mo_state* o) { return o ? o->t : -1; }

/* ---- one time step ----------------------------------------------------- */
static void collide_all(mo_state* o) {
  const int nx = o->nx, ny = o->ny;
  const size_t nn = o->nn;
  const double tau_f = o->s.tau_f;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      const size_t n = (size_t)y * nx + x;
      NodeIn in;
      /* S1 */
      node_moments(o, n, &in.rho_f, &in.jx_f, &in.jy_f, &in.rho_p, &in.jx_p,
                   &in.jy_p, &in.theta);
      /* S4: central differences of the previous step's fields.  Reading:
       * the paper gives no stencil; the lag keeps the gradient independent
       * of the order in which nodes are updated. */
      in.dphi_dx = 0.5 * (phi_at(o, x + 1, y) - phi_at(o, x - 1, y));
      in.dphi_dy = 0.5 * (phi_at(o, x, y + 1) - phi_at(o, x, y - 1));
      in.dth_dx = 0.5 * (theta_at(o, x + 1, y) - theta_at(o, x - 1, y));
      in.dth_dy = 0.5 * (theta_at(o, x, y + 1) - theta_at(o, x, y - 1));
      NodeOut r;
      node_physics(o, &in, &r); /* S2, S3, S5 */
      /* S6: BGK collisions, Eqs 18-19 with equilibria of Eqs 26-27.
       * Reading: f and p relax to their own velocities; g to the mixture
       * velocity of Eq 32. */
      /* equilibrium velocities: each phase its own (R-4), or, as the
       * alternative reading (flag 4), one common velocity for both, the
       * average weighted by rho/tau (conserves the collision's momentum) */
      double uef[2] = {r.ux_f, r.uy_f}, uep[2] = {r.ux_p, r.uy_p};
      if (o->cfg.reading_flags & 4u) {
        const double wf = in.rho_f / tau_f, wp = in.rho_p > 1e-12 ? in.rho_p / r.tau_p : 0.0;
        for (int d = 0; d < 2; ++d) {
          const double uc = (wf * (d ? r.uy_f : r.ux_f) + wp * (d ? r.uy_p : r.ux_p)) / (wf + wp);
          uef[d] = uc;
          uep[d] = uc;
        }
      }
      for (int i = 0; i < 9; ++i) {
        const size_t k = i * nn + n;
        const double fi = o->f[k], pi = o->p[k];
        o->fs[k] = fi - (fi - equilibrium(i, in.rho_f, uef[0], uef[1])) / tau_f +
                   forcing(i, r.Ffx, r.Ffy);
        o->ps[k] = pi - (pi - equilibrium(i, in.rho_p, uep[0], uep[1])) / r.tau_p +
                   forcing(i, r.Fpx, r.Fpy);
      }
      if (!o->two_t) {
        for (int i = 0; i < 9; ++i) {
          const size_t k = i * nn + n;
          const double gi = o->g[k];
          o->gs[k] = gi - (gi - equilibrium(i, in.theta, r.ux_ns, r.uy_ns)) / r.tau_th;
        }
      } else {
        /* Eq 19 for each phase (reading of Eqs 18-19, "two equations"
         * each): the fluid's thermal lattice relaxes to the fluid velocity
         * with the base-fluid diffusivity (Eq 22 form), the particles' to
         * the particle velocity with the relaxation time that makes the
         * mass-weighted sum of Eq 24 equal tau_theta of the suspension
         * (clamped as tau_p), or the fluid's where there are no particles. */
        double th_f, th_p, th_ns;
        node_temps(o, n, in.rho_p, &th_f, &th_p, &th_ns);
        const double tau_tf = 3.0 * o->s.alpha_L + 0.5;
        double tau_tp = tau_tf;
        if (in.rho_p > 1e-12) {
          const double rbar_p = in.rho_p / (in.rho_f + in.rho_p);
          tau_tp = (r.tau_th - (1.0 - rbar_p) * tau_tf) / rbar_p;
          if (tau_tp < 0.505) tau_tp = 0.505;
          if (tau_tp > 5.0) tau_tp = 5.0;
        }
        for (int i = 0; i < 9; ++i) {
          const size_t k = i * nn + n;
          const double gi = o->g[k], hi = o->g2[k];
          o->gs[k] = gi - (gi - equilibrium(i, th_f, r.ux_f, r.uy_f)) / tau_tf;
          o->g2s[k] = hi - (hi - equilibrium(i, th_p, r.ux_p, r.uy_p)) / tau_tp;
        }
      }
      /* keep (phi, theta) of this step for the next step's gradients */
      o->phi_cur[n] = in.rho_p / o->s.R;
      o->th_cur[n] = in.theta;
    }
  }
}

/* S7: pull streaming with the walls of Eqs 34-36.
 * Reading: walls sit half-way between the last node and its ghost, so the
 * no-slip condition of Eq 34 becomes link-wise bounce-back and conserves the
 * mass of each component exactly; the isothermal condition of Eq 35 solved
 * for the unknown gives anti-bounce-back g_i = -g*_opp + 2 W_i theta_w; the
 * adiabatic condition of Eq 36 copies the unknown populations from the
 * adjacent row in the same direction, after the isothermal rule. */
static void stream_all(mo_state* o) {
  const int nx = o->nx, ny = o->ny, b = o->cfg.boundary;
  const size_t nn = o->nn;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      const size_t n = (size_t)y * nx + x;
      for (int i = 0; i < 9; ++i) {
        int sx = x - EX[i], sy = y - EY[i];
        if (b != MO_CAVITY) sx = wrap(sx, nx);
        if (b == MO_PERIODIC) sy = wrap(sy, ny);
        const int in_x = sx >= 0 && sx < nx, in_y = sy >= 0 && sy < ny;
        const size_t k = i * nn + n;
        if (in_x && in_y) {
          const size_t src = i * nn + (size_t)sy * nx + sx;
          o->f[k] = o->fs[src];
          o->p[k] = o->ps[src];
          o->g[k] = o->gs[src];
          if (o->two_t) o->g2[k] = o->g2s[src];
        } else {
          const size_t own = OPP[i] * nn + n;
          o->f[k] = o->fs[own];
          o->p[k] = o->ps[own];
          if (!in_x) {
            const double thw = sx < 0 ? TH_HOT : TH_COLD;
            o->g[k] = -o->gs[own] + 2.0 * WGT[i] * thw;
            if (o->two_t) o->g2[k] = -o->g2s[own] + 2.0 * WGT[i] * thw;
          } else {
            o->g[k] = NAN; /* crossing a y-wall only: set by the copy below */
            if (o->two_t) o->g2[k] = NAN;
          }
        }
      }
    }
  }
  if (b == MO_PERIODIC) return;
  /* adiabatic walls: unknowns of row 0 (e_y = +1) and of row ny-1
   * (e_y = -1) copied from rows 1 and ny-2 */
  for (int x = 0; x < nx; ++x) {
    for (int i = 0; i < 9; ++i) {
      for (int l = 0; l < 1 + o->two_t; ++l) {
        double* h = l == 0 ? o->g : o->g2;
        if (EY[i] == 1)
          h[i * nn + x] = h[i * nn + (size_t)nx + x];
        else if (EY[i] == -1)
          h[i * nn + (size_t)(ny - 1) * nx + x] = h[i * nn + (size_t)(ny - 2) * nx + x];
      }
    }
  }
}

int mclbm_oracle_step(mo_state* o, int64_t nsteps) {
  if (!o || nsteps < 0) return MO_EINVAL;
  for (int64_t s = 0; s < nsteps; ++s) {
    collide_all(o);
    stream_all(o);
    /* S8 */
    double* t1 = o->phi_prev; o->phi_prev = o->phi_cur; o->phi_cur = t1;
    double* t2 = o->th_prev; o->th_prev = o->th_cur; o->th_cur = t2;
    o->t += 1;
  }
  return MO_OK;
}

/* ---- outputs ----------------------------------------------------------- */
int mclbm_oracle_read_moments(const mo_state* o, uint32_t mask, double* out,
                              size_t n_doubles) {
  if (!o || !out) return MO_EINVAL;
  int nf = 0;
  for (int b = 0; b < 11; ++b) nf += (mask >> b) & 1u;
  if (mask >> 11) return MO_EINVAL;
  const size_t nn = o->nn;
  if (n_doubles < (size_t)nf * nn) return MO_EINVAL;
  for (size_t n = 0; n < nn; ++n) {
    double rf, jxf, jyf, rp, jxp, jyp, th, th_f, th_p, th_ns;
    node_moments(o, n, &rf, &jxf, &jyf, &rp, &jxp, &jyp, &th);
    node_temps(o, n, rp, &th_f, &th_p, &th_ns);
    const double uxf = jxf / rf, uyf = jyf / rf;
    const int empty = !(rp > 1e-12);
    const double v[11] = {rf,
                          uxf,
                          uyf,
                          rp / o->s.R,
                          empty ? uxf : jxp / rp,
                          empty ? uyf : jyp / rp,
                          th,
                          (jxf + jxp) / (rf + rp),
                          (jyf + jyp) / (rf + rp),
                          th_f,
                          th_p};
    int slot = 0;
    for (int b = 0; b < 11; ++b) {
      if ((mask >> b) & 1u) {
        out[(size_t)slot * nn + n] = v[b];
        ++slot;
      }
    }
  }
  return MO_OK;
}

int mclbm_oracle_read_populations(const mo_state* o, double* out,
                                  size_t n_doubles) {
  if (!o || !out || n_doubles < (size_t)(27 + 9 * o->two_t) * o->nn) return MO_EINVAL;
  memcpy(out, o->f, 9 * o->nn * sizeof(double));
  memcpy(out + 9 * o->nn, o->p, 9 * o->nn * sizeof(double));
  memcpy(out + 18 * o->nn, o->g, 9 * o->nn * sizeof(double));
  if (o->two_t) memcpy(out + 27 * o->nn, o->g2, 9 * o->nn * sizeof(double));
  return MO_OK;
}

/* Test knob: replace the populations (layout of read_populations); the lag
 * fields and the residual snapshot are taken from the new state. */
int mclbm_oracle_write_populations(mo_state* o, const double* in,
                                   size_t n_doubles) {
  if (!o || !in || n_doubles < (size_t)(27 + 9 * o->two_t) * o->nn) return MO_EINVAL;
  memcpy(o->f, in, 9 * o->nn * sizeof(double));
  memcpy(o->p, in + 9 * o->nn, 9 * o->nn * sizeof(double));
  memcpy(o->g, in + 18 * o->nn, 9 * o->nn * sizeof(double));
  if (o->two_t) memcpy(o->g2, in + 27 * o->nn, 9 * o->nn * sizeof(double));
  init_lag_and_snapshot(o);
  return MO_OK;
}

/* ---- checkpoint / resume (test infrastructure) ------------------------
 * One line of JSON (format "mclbm-checkpoint", version, step count, parity,
 * the configuration as raw bytes, the section sizes), then the FP64
 * sections: f, p, g[, g2], the lag fields and the residual snapshot. */
#define MO_CKPT_VERSION 1

static void hex_of(const void* p, size_t n, char* out) {
  static const char* d = "0123456789abcdef";
  const unsigned char* b = (const unsigned char*)p;
  for (size_t k = 0; k < n; ++k) {
    out[2 * k] = d[b[k] >> 4];
    out[2 * k + 1] = d[b[k] & 15];
  }
  out[2 * n] = 0;
}

static int ckpt_arrays(mo_state* o, double** arr, size_t* len) {
  const size_t nn = o->nn;
  int k = 0;
  arr[k] = o->f; len[k++] = 9 * nn;
  arr[k] = o->p; len[k++] = 9 * nn;
  arr[k] = o->g; len[k++] = 9 * nn;
  if (o->two_t) { arr[k] = o->g2; len[k++] = 9 * nn; }
  arr[k] = o->phi_prev; len[k++] = nn;
  arr[k] = o->th_prev; len[k++] = nn;
  arr[k] = o->snap_ux; len[k++] = nn;
  arr[k] = o->snap_uy; len[k++] = nn;
  arr[k] = o->snap_th; len[k++] = nn;
  return k;
}

int mclbm_oracle_checkpoint(mo_state* o, const char* path) {
  if (!o || !path) return MO_EINVAL;
  double* arr[9];
  size_t len[9];
  const int na = ckpt_arrays(o, arr, len);
  char* cfg = malloc(2 * sizeof(mo_config) + 1);
  if (!cfg) return MO_ENOMEM;
  hex_of(&o->cfg, sizeof(mo_config), cfg);
  FILE* fp = fopen(path, "wb");
  if (!fp) { free(cfg); return MO_EINVAL; }
  fprintf(fp, "{\"format\": \"mclbm-checkpoint\", \"version\": %d, \"payload\": \"fp64\", \"nx\": %d, \"ny\": %d, "
              "\"t\": %lld, \"parity\": %d, \"config_hex\": \"%s\", \"sections\": %d, \"doubles\": %zu}\n",
          MO_CKPT_VERSION, o->nx, o->ny, (long long)o->t, (int)(o->t & 1), cfg, na, 9 * (size_t)(na > 8 ? 4 : 3) * o->nn + 5 * o->nn);
  free(cfg);
  int ok = 1;
  for (int k = 0; k < na && ok; ++k) ok = fwrite(arr[k], sizeof(double), len[k], fp) == len[k];
  ok = (fclose(fp) == 0) && ok;
  return ok ? MO_OK : MO_EINVAL;
}

int mclbm_oracle_restore(mo_state* o, const char* path) {
  if (!o || !path) return MO_EINVAL;
  FILE* fp = fopen(path, "rb");
  if (!fp) return MO_EINVAL;
  size_t cap = 4096 + 2 * sizeof(mo_config), n = 0;
  char* h = malloc(cap + 1);
  if (!h) { fclose(fp); return MO_ENOMEM; }
  int ch;
  while ((ch = fgetc(fp)) != EOF && ch != '\n' && n < cap) h[n++] = (char)ch;
  h[n] = 0;
  char* cfg = malloc(2 * sizeof(mo_config) + 1);
  if (!cfg) { free(h); fclose(fp); return MO_ENOMEM; }
  hex_of(&o->cfg, sizeof(mo_config), cfg);
  int rc = MO_OK;
  long long t = -1;
  const char* tp = strstr(h, "\"t\": ");
  if (!strstr(h, "\"format\": \"mclbm-checkpoint\"") || !strstr(h, "\"payload\": \"fp64\"") || !tp ||
      !strstr(h, cfg))
    rc = MO_EINVAL;
  else
    t = strtoll(tp + 5, NULL, 10);
  free(cfg);
  free(h);
  if (rc != MO_OK || t < 0) { fclose(fp); return MO_EINVAL; }
  double* arr[9];
  size_t len[9];
  const int na = ckpt_arrays(o, arr, len);
  /* read into scratch first so that a short file leaves the state unchanged */
  size_t total = 0;
  for (int k = 0; k < na; ++k) total += len[k];
  double* tmp = malloc(total * sizeof(double));
  if (!tmp) { fclose(fp); return MO_ENOMEM; }
  const int ok = fread(tmp, sizeof(double), total, fp) == total && fgetc(fp) == EOF;
  fclose(fp);
  if (!ok) { free(tmp); return MO_EINVAL; }
  size_t off = 0;
  for (int k = 0; k < na; ++k) {
    memcpy(arr[k], tmp + off, len[k] * sizeof(double));
    off += len[k];
  }
  free(tmp);
  o->t = t;
  return MO_OK;
}

/* Average Nusselt number at the walls.  Reading: the paper plots the average
 * hot-wall Nu without printing its formula; the wall gradient is the
 * second-order one-sided difference through theta_w at half a spacing and
 * the two first nodes, (9 theta_0 - theta_1 - 8 theta_w)/3, which is exact
 * for linear profiles.  nu_hot_k weights it with k_ns/k_f at the first node. */
int mclbm_oracle_nusselt(const mo_state* o, double* nu_hot, double* nu_cold,
                         double* nu_hot_k) {
  if (!o) return MO_EINVAL;
  const int nx = o->nx, ny = o->ny;
  const size_t nn = o->nn;
  double sh = 0.0, sc = 0.0, sk = 0.0;
  int bad = 0;
  for (int y = 0; y < ny; ++y) {
    double th[4] = {0, 0, 0, 0};
    const int xs[4] = {0, 1, nx - 2, nx - 1};
    for (int q = 0; q < 4; ++q) {
      const size_t n = (size_t)y * nx + xs[q];
      double rq = 0.0, tf, tp;
      for (int i = 0; i < 9; ++i) rq += o->p[i * nn + n];
      node_temps(o, n, rq, &tf, &tp, &th[q]);
    }
    double rp = 0.0;
    for (int i = 0; i < 9; ++i) rp += o->p[i * nn + (size_t)y * nx];
    double phi = rp / o->s.R;
    if (phi < 0.0) phi = 0.0;
    const double r_k = 1.0 + o->s.Ck * pow(phi, 0.764);
    const double gh = -(double)nx * (9.0 * th[0] - th[1] - 8.0 * TH_HOT) / 3.0;
    const double gc = (double)nx * (9.0 * th[3] - th[2] - 8.0 * TH_COLD) / 3.0;
    sh += gh;
    sc += gc;
    sk += r_k * gh;
    if (!isfinite(gh) || !isfinite(gc)) bad = 1;
  }
  if (nu_hot) *nu_hot = sh / ny;
  if (nu_cold) *nu_cold = sc / ny;
  if (nu_hot_k) *nu_hot_k = sk / ny;
  return bad ? MO_EDIVERGED : MO_OK;
}

/* Relative L2 change of the mixture velocity and of theta since the last
 * call (or since the initial state), then the snapshot is replaced. */
int mclbm_oracle_residual(mo_state* o, double* res_u, double* res_theta) {
  if (!o) return MO_EINVAL;
  const size_t nn = o->nn;
  double du = 0.0, nu = 0.0, dth = 0.0, nth = 0.0;
  int bad = 0;
  for (size_t n = 0; n < nn; ++n) {
    double rf, jxf, jyf, rp, jxp, jyp, th;
    node_moments(o, n, &rf, &jxf, &jyf, &rp, &jxp, &jyp, &th);
    const double ux = (jxf + jxp) / (rf + rp), uy = (jyf + jyp) / (rf + rp);
    if (!isfinite(ux) || !isfinite(uy) || !isfinite(th)) bad = 1;
    du += (ux - o->snap_ux[n]) * (ux - o->snap_ux[n]) +
          (uy - o->snap_uy[n]) * (uy - o->snap_uy[n]);
    nu += ux * ux + uy * uy;
    dth += (th - o->snap_th[n]) * (th - o->snap_th[n]);
    nth += th * th;
    o->snap_ux[n] = ux;
    o->snap_uy[n] = uy;
    o->snap_th[n] = th;
  }
  if (res_u) *res_u = bad ? NAN : (nu > 0.0 ? sqrt(du / nu) : (du > 0.0 ? INFINITY : 0.0));
  if (res_theta)
    *res_theta = bad ? NAN : (nth > 0.0 ? sqrt(dth / nth) : (dth > 0.0 ? INFINITY : 0.0));
  return bad ? MO_EDIVERGED : MO_OK;
}

int mclbm_oracle_derived(const mo_state* o, double* out, int n) {
  if (!o || !out || n < MO_D_COUNT) return MO_EINVAL;
  const Setup* s = &o->s;
  out[MO_D_NU_L] = s->nu_L;
  out[MO_D_ALPHA_L] = s->alpha_L;
  out[MO_D_H] = s->H;
  out[MO_D_DX] = s->dx;
  out[MO_D_DT] = s->dt;
  out[MO_D_G_L] = s->G_L;
  out[MO_D_GRAV_L] = s->grav_L;
  out[MO_D_CK] = s->Ck;
  out[MO_D_R] = s->R;
  out[MO_D_TAU_F] = s->tau_f;
  out[MO_D_RHOC_RATIO] = s->rhoc_ratio;
  out[MO_D_BETA_RATIO] = s->beta_ratio;
  out[MO_D_RHO_F0] = s->rho_f0;
  out[MO_D_RHO_P0] = s->rho_p0;
  out[MO_D_NU_F] = s->nu_f;
  out[MO_D_ALPHA_F] = s->alpha_f;
  return MO_OK;
}

int mclbm_oracle_node_forces(const mo_state* o, const double* in,
                             double* out) {
  if (!o || !in || !out) return MO_EINVAL;
  NodeIn a;
  a.rho_f = in[MO_IN_RHO_F]; a.jx_f = in[MO_IN_JX_F]; a.jy_f = in[MO_IN_JY_F];
  a.rho_p = in[MO_IN_RHO_P]; a.jx_p = in[MO_IN_JX_P]; a.jy_p = in[MO_IN_JY_P];
  a.theta = in[MO_IN_THETA];
  a.dphi_dx = in[MO_IN_DPHI_DX]; a.dphi_dy = in[MO_IN_DPHI_DY];
  a.dth_dx = in[MO_IN_DTH_DX]; a.dth_dy = in[MO_IN_DTH_DY];
  NodeOut r;
  node_physics(o, &a, &r);
  out[MO_OUT_FFX] = r.Ffx; out[MO_OUT_FFY] = r.Ffy;
  out[MO_OUT_FPX] = r.Fpx; out[MO_OUT_FPY] = r.Fpy;
  out[MO_OUT_TAU_P] = r.tau_p; out[MO_OUT_TAU_TH] = r.tau_th;
  out[MO_OUT_ABX] = r.aB[0]; out[MO_OUT_ABY] = r.aB[1];
  out[MO_OUT_ATX] = r.aT[0]; out[MO_OUT_ATY] = r.aT[1];
  out[MO_OUT_ASX] = r.aS[0]; out[MO_OUT_ASY] = r.aS[1];
  out[MO_OUT_AMRX] = r.aMR[0]; out[MO_OUT_AMRY] = r.aMR[1];
  out[MO_OUT_AGX] = r.aG[0]; out[MO_OUT_AGY] = r.aG[1];
  out[MO_OUT_DX] = r.D[0]; out[MO_OUT_DY] = r.D[1];
  out[MO_OUT_BETA_L] = r.beta_L; out[MO_OUT_KAPPA] = r.kappa;
  out[MO_OUT_R_K] = r.r_k; out[MO_OUT_R_MU] = r.r_mu;
  return MO_OK;
}
