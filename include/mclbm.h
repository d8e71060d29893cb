/*
 * mclbm.h -- C ABI of the MI355X (gfx950) multi-component lattice Boltzmann
 * library: three coupled D2Q9 lattices (base fluid f, nanoparticle phase p,
 * temperature g) in a differentially heated cavity, after Savithiri, Dhar,
 * Pattamatta and Das, "Particle-fluid interactivity deteriorates buoyancy
 * driven thermal transport in nanosuspensions: a multi component lattice
 * Boltzmann approach" (arXiv:1511.04552).
 *
 * Conventions for every entry point:
 *   - All functions return an int status (MCLBM_OK = 0, negative = error)
 *     unless stated otherwise; mclbm_last_error() gives a thread-local
 *     message for the last failure on the calling thread.
 *   - No C++ exception crosses this boundary.
 *   - Device pointers are HIP device addresses on the current device; host
 *     pointers are plain host memory.  The library never allocates device
 *     memory: the caller passes one device buffer of mclbm_device_bytes()
 *     bytes, which the library borrows until mclbm_destroy().
 *   - All device work is enqueued on the stream given at creation
 *     (a hipStream_t, NULL = the legacy default stream).  Calls marked
 *     "async" return before the work completes; calls marked "sync" wait for
 *     the stream before returning.
 *   - A cavity handle is not thread-safe; distinct handles on distinct
 *     streams may be used concurrently.
 *
 * Lattice conventions (Section 2.d, Eqs 21 and 28): direction order rest,
 * E, N, W, S, NE, NW, SW, SE; lattice units dx = dt = 1, c_s^2 = 1/3;
 * nodes x = 0..nx-1 (hot wall at x = -1/2, cold wall at x = nx - 1/2),
 * y = 0..ny-1 (adiabatic walls at y = -1/2 and ny - 1/2); theta =
 * (T - T0)/dT with theta_hot = +1/2, theta_cold = -1/2.
 */
#ifndef MCLBM_H
#define MCLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCLBM_ABI_VERSION 4

enum mclbm_status {
  MCLBM_OK = 0,
  MCLBM_EINVAL = -1,      /* invalid argument or configuration */
  MCLBM_ENOMEM = -2,      /* device buffer smaller than mclbm_device_bytes */
  MCLBM_EHIP = -3,        /* a HIP runtime call failed (message kept) */
  MCLBM_EDIVERGED = -4,   /* a non-finite value was found at a sync point */
  MCLBM_ESTATE = -5,      /* call not allowed in the current state */
  MCLBM_EUNSUPPORTED = -6 /* valid request this build does not implement */
};

/* Storage type of the populations.  Populations are always stored as
 * deviations from the uniform reference state (f_i - W_i rho_ref); the
 * collision always computes in FP32 and reductions in FP64. */
enum mclbm_storage { MCLBM_FP32S = 0, MCLBM_FP16S = 1, MCLBM_BF16S = 2 };

/* Slip-force switches (Table 1 of the paper).  Buoyancy (Eq 20) is always
 * on and scales with Ra. */
enum mclbm_force {
  MCLBM_F_DRAG = 1, MCLBM_F_BROWN = 2, MCLBM_F_THERMO = 4, MCLBM_F_SAFF = 8,
  MCLBM_F_MAGROT = 16, MCLBM_F_GRAV = 32, MCLBM_F_ALL = 63
};

/* Alternative readings (reading_flags).  Each replaces one default reading
 * of a garbled or ambiguous passage by another:
 *   LITERAL_K_RATIO   Eq 10a with (k_f/k_p)^0.7476 as printed (default:
 *                     k_p/k_f, the printed form makes the enhancement vanish)
 *   LITERAL_GRAVITY   Table 1 gravity on the particles only (default: the
 *                     fluid carries the weight of the uniform suspension,
 *                     so the mixture feels only phi - phi0)
 *   COMMON_VELOCITY   f and p relax to one common velocity weighted by
 *                     rho/tau (default: each to its own, Eq 26 "u^sigma")
 *   GUO_FORCING, LITERAL_REACTIONS  reserved: MCLBM_EUNSUPPORTED */
enum mclbm_reading {
  MCLBM_R_LITERAL_K_RATIO = 1, MCLBM_R_LITERAL_GRAVITY = 2,
  MCLBM_R_COMMON_VELOCITY = 4, MCLBM_R_GUO_FORCING = 8,
  MCLBM_R_LITERAL_REACTIONS = 16
};

/* Moment fields (Eqs 29-32) for mclbm_read_moments / mclbm_export_moments.
 * Fields are written in increasing bit order, each nx*ny doubles, row-major
 * with x fastest. RHO_F is the fluid partial density, PHI the particle
 * volume fraction, *_NS the mass-averaged mixture velocity of Eq 32, THETA
 * the suspension temperature; THETA_F and THETA_P the temperatures of the
 * fluid and particle thermal lattices (equal to THETA with one thermal
 * lattice). */
enum mclbm_field {
  MCLBM_RHO_F = 1, MCLBM_UX_F = 2, MCLBM_UY_F = 4, MCLBM_PHI = 8,
  MCLBM_UX_P = 16, MCLBM_UY_P = 32, MCLBM_THETA = 64, MCLBM_UX_NS = 128,
  MCLBM_UY_NS = 256, MCLBM_ALL_FIELDS = 511, MCLBM_THETA_F = 512,
  MCLBM_THETA_P = 1024, MCLBM_FIELD_MASK = 2047, MCLBM_FIELD_COUNT = 11
};

/* Derived lattice constants (slots of mclbm_derived). */
enum mclbm_derived_slot {
  MCLBM_D_NU_L = 0, MCLBM_D_ALPHA_L, MCLBM_D_H, MCLBM_D_DX, MCLBM_D_DT,
  MCLBM_D_G_L, MCLBM_D_GRAV_L, MCLBM_D_CK, MCLBM_D_R, MCLBM_D_TAU_F,
  MCLBM_D_RHOC_RATIO, MCLBM_D_BETA_RATIO, MCLBM_D_RHO_F0, MCLBM_D_RHO_P0,
  MCLBM_D_NU_F, MCLBM_D_ALPHA_F, MCLBM_D_COUNT
};

typedef struct {
  double rho;   /* density, kg/m^3 */
  double cp;    /* specific heat, J/(kg K) */
  double k;     /* thermal conductivity, W/(m K) */
  double beta;  /* thermal expansion coefficient, 1/K */
  double mu;    /* dynamic viscosity, Pa s (fluid only) */
  double d_mol; /* molecular diameter, m (fluid only; also the mean free
                   path of the thermophoretic Knudsen number) */
} mclbm_material;

typedef struct {
  int32_t nx, ny;          /* nodes, each >= 4; Ra is based on nx */
  double Ra;               /* base-fluid Rayleigh number (Eq 16), >= 0 */
  double Pr;               /* base-fluid Prandtl number, > 0 */
  double phi0;             /* mean particle volume fraction, [0, 0.1] */
  double dp_m;             /* particle diameter, m, > 0 */
  double tau_f;            /* fluid relaxation time (Eq 22), > 0.5; <= 0:
                              automatic, free-fall velocity <= 0.1 c_s */
  double dT_K, T0_K;       /* wall temperature difference and mean, K */
  uint32_t force_mask;     /* MCLBM_F_* bits */
  double force_scale[6];   /* per-force multipliers in bit order (test knob) */
  double phi_perturb_amp;  /* initial phi = max(phi0 + amp * xi, 0) */
  mclbm_material fluid, particle;
  int32_t storage;         /* enum mclbm_storage */
  int32_t block_x, block_y;/* step-kernel workgroup shape; 0 = default
                              (256 x 1 when nx >= 256, else 64 x 1);
                              block_x in {32, 64, 128, 256} and
                              block_x * block_y in {64, 128, 256} */
  uint32_t reading_flags;  /* MCLBM_R_* alternatives to the default readings
                              of garbled passages; 0 = the defaults */
  int32_t thermal_lattices;/* 1 (default; 0 means 1): one thermal lattice
                              for the suspension.  2: Eq 19 for each phase
                              (fluid and particle temperatures), the
                              suspension temperature by Eq 33; FP32 storage
                              and single cavities only (MCLBM_EUNSUPPORTED
                              otherwise, also for mclbm_load_fields) */
  int32_t steps_per_launch;/* 0 (default) = automatic: 2 for FP32 storage
                              from 2^20 nodes and 256 columns on (where it
                              is faster), else 1.  1: one launch per step,
                              updated in place.  2: an even and the
                              following odd step in one launch, from one
                              population copy into a second one (device
                              bytes grow by one population array; 1.25x
                              instead of 2x the bytes of one step, the same
                              arithmetic); one thermal lattice only, and
                              in a batch populations below 2 GiB per cavity
                              (MCLBM_EUNSUPPORTED on request otherwise; the
                              automatic choice falls back to 1).  Above
                              2 GiB of populations the single cavity's
                              launches take 64-bit element offsets; the
                              two copies then need twice those bytes of
                              device memory (set 1 where they do not fit).  A batch
                              takes one schedule for all its cavities: 2
                              if every cavity asks for 2 (a batch mixing
                              2 with 0 or 1 is rejected), or if every
                              cavity leaves 0 and the batch holds FP32
                              cavities of 2^20 nodes in total that fill at
                              least 60 % of their 62-column strips; else 1.  A step
                              count or start that is odd takes single steps
                              where needed.  With FP32 storage the results
                              are bitwise those of single steps (16-bit
                              storage: the intermediate odd-step state is
                              kept in FP32, not rounded to storage) */
} mclbm_config;

typedef struct mclbm_cavity mclbm_cavity; /* opaque host-side handle */

/* Environment variables read when a cavity is created (none changes the
 * results; the tests use them to reach size-chosen paths on small
 * cavities):
 *   MCLBM_LOG=debug      one line on stderr per configuration with the
 *                        lattice constants and stability numbers
 *   MCLBM_INDEX64=1      64-bit element offsets (otherwise above 2 GiB of
 *                        populations), in both schedules of a single
 *                        cavity; a batch then steps one step per launch
 *   MCLBM_STREAMING=1    non-temporal population access of single steps
 *                        (otherwise above 160 MiB)
 *   MCLBM_POISON=1       race check: NaN-fill, before each launch, what it
 *                        writes and must not read first
 *   MCLBM_BAND2=<rows>   band height of two steps per launch (tuning)
 *   MCLBM_BANDMIX=<n>    dispatch interleave of those bands, 1 to 64 (1:
 *                        in order; otherwise about 150 / strips of 62
 *                        columns from 2^21 nodes on) (tuning)
 *   MCLBM_PLANE_PAD=<n>  elements of padding between population planes, a
 *                        multiple of 64 in [0, 2^20] (otherwise 4160 from
 *                        2^20 nodes on and for every member of a batch
 *                        whose FP32 working set exceeds 160 MiB, 0 below);
 *                        mclbm_copy_state needs the same pad on both
 *                        sides, checkpoints hold the planes without it */

/* Fill *cfg with the defaults: 64x64, Ra 1e3, Pr 6.2, phi0 0.01, dp 100 nm,
 * tau_f 0.8, dT 10 K, T0 300 K, all forces at scale 1, amplitude 1e-6,
 * water and alumina properties, FP32 storage, default block shape. */
void mclbm_config_defaults(mclbm_config* cfg);

/* Bytes of device memory a cavity with this configuration needs; 0 if the
 * configuration is invalid (see mclbm_last_error).  From 2^20 nodes on the
 * population planes are padded (MCLBM_PLANE_PAD), which adds a few hundred
 * KB. */
size_t mclbm_device_bytes(const mclbm_config* cfg);

/* Derived lattice constants of a configuration (host only, no device work):
 * MCLBM_D_COUNT doubles in enum mclbm_derived_slot order -- lattice
 * viscosity and diffusivity (Eq 22), cavity width H from Ra (Eq 16), dx,
 * dt, g beta dT and g in lattice units, the Eq 10a constant, density ratio,
 * relaxation time, heat-capacity and expansion ratios (Eqs 8-9), reference
 * partial densities, physical viscosity and diffusivity. */
int mclbm_derive_constants(const mclbm_config* cfg, double* out, int n);

/* Create a cavity on the device buffer dev_buf (>= mclbm_device_bytes,
 * 256-byte aligned) and enqueue its initial state on `stream`: fluid at rest,
 * uniform temperature theta = 0, populations at equilibrium (Eqs 26-27).
 * xi_host: NULL or nx*ny host doubles in [-1, 1] (row-major) scaling the
 * initial phi perturbation; it is copied.  Async.  The library keeps a
 * pointer to neither cfg nor xi_host. */
int mclbm_create(const mclbm_config* cfg, const double* xi_host,
                 void* dev_buf, size_t bytes, void* stream,
                 mclbm_cavity** out);

/* Change Ra, phi0 and dp (the parameters the paper sweeps, Section 3) and
 * restart from the initial state.  Allowed at any time; re-derives the
 * lattice constants.  Async.  MCLBM_EINVAL leaves the cavity unchanged. */
int mclbm_set_properties(mclbm_cavity* c, double Ra, double phi0,
                         double dp_m);

/* Restart from the initial state (time 0).  Async. */
int mclbm_reset(mclbm_cavity* c);

/* Warm start: restart at time 0 from given fields instead of the fluid at
 * rest.  The initial state of the method is an equilibrium one (Eqs 26-27);
 * here every node takes the equilibrium of the given fields instead, so a
 * prediction of the steady flow shortens the transient while the time
 * stepping, and so the steady state it converges to, are unchanged.
 *   dev_fields: device FP32, sy x sx x nc channel-last (row y, column x):
 *     mixture velocity u_x, u_y (lattice units), dimensionless temperature
 *     theta, particle volume fraction phi and, if nc == 5, the deviation of
 *     the fluid partial density rho_f~ from its cold-start value 1 - phi0
 *     (the pressure field), sampled at the cell centres of an sx x sy grid
 *     over the cavity (sx, sy >= 1, nc = 4 or 5);
 *   affine: NULL (identity) or 2 nc host doubles: channel c is taken as
 *     affine[c] * v + affine[nc + c].
 * Lattice node (x, y) samples position s_x = (x + 1/2) sx / nx - 1/2
 * (clamped to [0, sx - 1]; likewise y) bilinearly in FP64.  phi is clipped
 * at 0 and rescaled so that its lattice sum equals that of the cold start,
 * sum max(phi0 + A xi, 0) (the particle mass of the closed cavity is
 * conserved); if nothing is left it becomes uniform.  rho_f~ = 1 - phi0
 * plus the density deviation less its lattice mean (the fluid mass is
 * conserved too), rho_p~ = R phi, and both phases move with u.  Synchronous
 * on the cavity's stream.  A member of a batch (mclbm_batch_cavity) may be
 * loaded while the batch is at an even step count (MCLBM_ESTATE otherwise):
 * its time restarts at 0 and it keeps its active flag. */
int mclbm_load_fields(mclbm_cavity* c, const float* dev_fields, int32_t sx,
                      int32_t sy, int32_t nc, const double* affine);

/* Continue a run in another storage type: the state of src (populations,
 * converted from src's storage type and scale to dst's; the lag fields;
 * the adiabatic side buffer; the residual reference; the step count)
 * becomes dst's.  Both cavities must have the same configuration apart
 * from the storage type and the launch shape (MCLBM_EINVAL otherwise);
 * src must be at an even step count, and a dst that belongs to a batch
 * needs its batch at an even step count (MCLBM_ESTATE otherwise).  Used to
 * run the transient with 16-bit storage (Section 2.d's scheme is unchanged;
 * only the rounding of the stored populations differs) and finish in FP32.
 * Waits for src's stream, then enqueues on dst's and waits for it (sync). */
int mclbm_copy_state(mclbm_cavity* dst, const mclbm_cavity* src);

/* Advance nsteps >= 0 time steps (Eqs 18-36: collision with the slip
 * forces, streaming, walls).  Each step is one fused kernel launch, or with
 * two steps per launch (steps_per_launch) each pair from an even step
 * count is one launch and a leftover step a single one.  Async. */
int mclbm_step(mclbm_cavity* c, int64_t nsteps);

/* Periodic Nusselt numbers on the device (the average hot-wall Nu of
 * Section 2.d, Fig 3a, as mclbm_nusselt), with no host synchronisation per
 * record: while every > 0, each time mclbm_step brings the step count to a
 * multiple t of `every`, record k (k = 0, 1, ... since this call) is written
 * on the cavity's stream to dev_ring[4 (k mod capacity) ..]: nu_hot,
 * nu_cold, nu_hot_k and a flag (1.0 if a wall value was not finite, else
 * 0.0).  dev_ring: 4 capacity doubles of device memory, 8-byte aligned,
 * owned by the caller and borrowed until recording is switched off (every
 * = 0) or the cavity is destroyed.  With two steps per launch, a pair whose
 * odd step is a multiple of `every` runs as two single steps.  Not for
 * batch members (MCLBM_ESTATE). */
int mclbm_record_nusselt(mclbm_cavity* c, int32_t every, double* dev_ring, int32_t capacity);

/* Records written since the last mclbm_record_nusselt call (-1 for NULL);
 * the newest is in slot (count - 1) mod capacity. */
int64_t mclbm_nusselt_records(const mclbm_cavity* c);

/* Number of steps taken since the initial state. */
int64_t mclbm_time(const mclbm_cavity* c);

/* Moments (Eqs 29-32) of the current state as doubles into device memory
 * dev_out (n_doubles >= popcount(mask) * nx * ny).  Async. */
int mclbm_export_moments(mclbm_cavity* c, uint32_t mask, double* dev_out,
                         size_t n_doubles);

/* As mclbm_export_moments, into host memory.  Sync. */
int mclbm_read_moments(mclbm_cavity* c, uint32_t mask, double* host_out,
                       size_t n_doubles);

/* Populations of the current state after streaming, as doubles in host
 * memory: [lattice f,p,g(,g2)][direction][y][x], 27*nx*ny values (36*nx*ny
 * with two thermal lattices), the shift of the storage added back.  Sync.
 * For tests and checkpoints. */
int mclbm_read_populations(mclbm_cavity* c, double* host_out,
                           size_t n_doubles);

/* As mclbm_read_populations, into device memory dev_out
 * (n_doubles >= 27*nx*ny, or 36*nx*ny).  Async. */
int mclbm_export_populations(mclbm_cavity* c, double* dev_out,
                             size_t n_doubles);

/* Average Nusselt numbers of the current state, accumulated in FP64:
 * nu_hot = mean over y of -nx (9 theta(0,y) - theta(1,y) - 8 theta_hot)/3,
 * nu_cold the mirror image at the cold wall, nu_hot_k the hot-wall value
 * weighted with k_ns/k_f of Eq 10a at the first node.  Any pointer may be
 * NULL.  Sync.  Returns MCLBM_EDIVERGED if a wall value is not finite. */
int mclbm_nusselt(mclbm_cavity* c, double* nu_hot, double* nu_cold,
                  double* nu_hot_k);

/* Relative L2 change of the mixture velocity and of theta since the
 * previous call (or since the initial state), accumulated in FP64; the
 * current state becomes the new reference.  Sync.  Returns
 * MCLBM_EDIVERGED if any node is not finite. */
int mclbm_residual(mclbm_cavity* c, double* res_u, double* res_theta);

/* For callers that cannot allocate device memory or wait on the host (code
 * under HIP graph capture, tight serving loops): mclbm_residual with its
 * per-block FP64 partials in a library-owned static device array instead
 * of the cavity's buffer, and its result left in device memory instead of
 * being returned after a synchronisation.
 *   dev_out: device memory of 3 doubles, 8-byte aligned, written on the
 *     cavity's stream: [0] relative L2 change of the mixture velocity,
 *     [1] of theta (as mclbm_residual), [2] 1.0 if any node was not finite,
 *     else 0.0 (mclbm_residual's MCLBM_EDIVERGED).
 * The current state becomes the new reference, as in mclbm_residual.
 * Async; no device or host allocation, no synchronisation.  The cavity's
 * device must be current.  The static array holds MCLBM_NOALLOC_SCRATCH_BYTES
 * on every GPU the library runs on, until the process ends; larger cavities
 * (more than MCLBM_NOALLOC_MAX_NODES nodes) are rejected with MCLBM_EINVAL.
 * Every call on one GPU uses the same array: calls that overlap in time on
 * one GPU (different streams, or different host threads) race and must be
 * ordered by the caller.  Nothing in the array needs to start at zero. */
#define MCLBM_NOALLOC_SCRATCH_BYTES (4u << 20)
#define MCLBM_NOALLOC_MAX_NODES (((MCLBM_NOALLOC_SCRATCH_BYTES) / 40u) * 256u)
int mclbm_residual_noalloc(mclbm_cavity* c, double* dev_out);

/* Derived lattice constants, MCLBM_D_COUNT doubles (enum slots). */
int mclbm_derived(const mclbm_cavity* c, double* out, int n);

/* Checkpoint / resume.  mclbm_checkpoint writes the complete state to the
 * file `path`: one line of JSON (format "mclbm-checkpoint", version, the
 * configuration in readable form and as raw bytes, the derived constants,
 * the step count, parity, storage type and the byte size of each section),
 * then the raw sections: populations (storage format, both A-A parities
 * as stored, the planes without the padding between them), the two
 * lag-field buffers (likewise), the adiabatic side buffer and the
 * residual snapshot.  Sync.  A member of a batch may be checkpointed.
 * mclbm_restore reads such a file into a cavity created with the same
 * configuration apart from its launch shape (block_x, block_y and
 * steps_per_launch may differ; MCLBM_EINVAL otherwise, or for a damaged or
 * foreign file; the cavity is then unchanged); stepping then continues
 * bitwise as the checkpointed run would have (also after a change of
 * steps_per_launch with FP32 storage).  Not for batch members
 * (MCLBM_ESTATE).
 * Both return MCLBM_EHIP-free host errors as MCLBM_EINVAL with a message. */
int mclbm_checkpoint(mclbm_cavity* c, const char* path);
int mclbm_restore(mclbm_cavity* c, const char* path);

/* Inspect a checkpoint file without a cavity (host only, no device work):
 * the configuration it was written from (launch shape fields zeroed), its
 * step count and, if the cavity had one, its initial perturbation field, so
 * that a caller can create the matching cavity before mclbm_restore.  Any
 * output pointer may be NULL.  *n_xi receives nx*ny, or 0 if the cavity was
 * created without a field; xi_out (capacity xi_cap doubles) receives the
 * field when it is non-NULL (MCLBM_EINVAL if xi_cap < nx*ny).  A file that
 * is not a checkpoint of this format, or whose header is damaged (hex
 * fields of the wrong length or alphabet, an invalid configuration, no step
 * count), gives MCLBM_EINVAL and leaves the outputs unchanged. */
int mclbm_checkpoint_info(const char* path, mclbm_config* cfg_out, int64_t* t_out,
                          double* xi_out, size_t xi_cap, size_t* n_xi);

/* Release the handle.  Does not free dev_buf.  Waits for the stream. */
int mclbm_destroy(mclbm_cavity* c);

/* Thread-local message describing the last failure ("" if none). */
const char* mclbm_last_error(void);

/* ---- Batched parameter sweeps ------------------------------------------
 * A batch holds n independent cavities of uneven sizes and parameters (the
 * sweeps over Ra, phi and d_p of Section 3) in one device buffer.  One
 * kernel launch per time step updates every active cavity (one workgroup
 * per tile of every cavity); the step loop is replayed from a captured HIP
 * graph.  Many small cavities step instead one workgroup per cavity for up
 * to 256 steps per launch (mclbm_batch_set_per_cavity).  Every cavity gives
 * bitwise the same result as the same cavity created alone.  All cavities of
 * a batch share the storage type; each keeps its own workgroup shape.
 * With two steps per launch (steps_per_launch in mclbm_config), each launch
 * from an even step runs two steps of every active cavity (tiles of 62
 * columns by a band of rows per cavity), as the same cavity alone with two
 * steps per launch; otherwise one step per launch. */
typedef struct mclbm_batch mclbm_batch;

/* Bytes of device memory for a batch of n cavities; 0 if any configuration
 * is invalid or the storage types differ. */
size_t mclbm_batch_device_bytes(const mclbm_config* cfgs, int32_t n);

/* Create a batch on dev_buf (>= mclbm_batch_device_bytes, 256-byte aligned)
 * and enqueue every cavity's initial state on `stream`.  xis: NULL, or n
 * pointers each NULL or to nx*ny host doubles (as for mclbm_create).  Sync. */
int mclbm_batch_create(const mclbm_config* cfgs, int32_t n, const double* const* xis,
                       void* dev_buf, size_t bytes, void* stream, mclbm_batch** out);

/* Advance every active cavity by nsteps >= 0 steps.  Async. */
int mclbm_batch_step(mclbm_batch* b, int64_t nsteps);

/* Steps replayed per graph launch (an even number >= 2), or 0 to launch
 * every step directly.  Default 32.  With two steps per launch a replay of
 * an odd number of launches makes the next replay rewrite the batch's
 * device-side descriptors first (a synchronisation). */
int mclbm_batch_set_graph_steps(mclbm_batch* b, int32_t steps);

/* Mark cavities active (1) or dropped (0); dropped cavities stop stepping
 * and keep their state.  A dropped cavity may only rejoin when its step
 * count has the parity of the active ones.  Sync. */
int mclbm_batch_set_active(mclbm_batch* b, const int32_t* active);

/* Residual (as mclbm_residual) of every active cavity: out[2k], out[2k+1];
 * status[k] = 0 still running, 1 converged (both below tol; dropped),
 * 2 diverged (non-finite; dropped), 3 inactive.  tol <= 0 only reports.
 * Sync (once for the whole batch). */
int mclbm_batch_residual(mclbm_batch* b, double tol, double* out, int32_t* status);

/* Nusselt numbers (as mclbm_nusselt) of every cavity: out[3k .. 3k+2].
 * Non-finite values are reported as such.  Sync (once for the whole
 * batch). */
int mclbm_batch_nusselt(mclbm_batch* b, double* out);

/* Project-written autotuner: for every size class of the batch (cavities of
 * equal nx, ny) time `steps` steps, that class alone, with each candidate
 * workgroup shape (256x1, 128x2, 64x4, 32x8), or with two steps per launch
 * each band height of the two-step tiles (3, 4, 6, 8 rows); keep the
 * fastest per class.  Where the batch may step one workgroup per cavity
 * (mclbm_batch_set_per_cavity), time that and the tiles on the whole batch
 * and keep the faster.  Then restart every cavity from its initial state.
 * Neither changes any result.  Sync. */
int mclbm_batch_autotune(mclbm_batch* b, int32_t steps);

/* Schedule of many small cavities: with on = 1, every launch runs up to 256
 * steps (an even number, from an even step) of all active cavities, one
 * 1024-thread workgroup per cavity with a workgroup barrier between steps;
 * on = 0 returns to one launch per step over the tiles.  Results are
 * bitwise those of the tiles.  Needs one step per launch and cavities of at
 * most 128^2 nodes (MCLBM_EINVAL otherwise).  Default: on for batches of
 * cavities of at most 64^2 nodes that number at least
 * max(128, 256 * nodes / 64^2) of the largest; mclbm_batch_autotune times
 * both on the whole batch and keeps the faster.  Sync. */
int mclbm_batch_set_per_cavity(mclbm_batch* b, int32_t on);

/* 1 when the batch steps one workgroup per cavity, 0 over tiles, -1 for a
 * NULL batch. */
int32_t mclbm_batch_per_cavity(const mclbm_batch* b);

/* Tile of cavity idx: the workgroup shape (bx, by), or with two steps per
 * launch the strip width and band height (62, rows). */
int mclbm_batch_tile_shape(const mclbm_batch* b, int32_t idx, int32_t* bx, int32_t* by);

/* Restart every cavity from its initial state and reactivate it.  Sync. */
int mclbm_batch_reset(mclbm_batch* b);

/* Number of cavities; steps taken by cavity idx (-1 on bad arguments). */
int32_t mclbm_batch_size(const mclbm_batch* b);
int64_t mclbm_batch_time(const mclbm_batch* b, int32_t idx);

/* The cavity idx of the batch as a cavity handle owned by the batch (valid
 * until mclbm_batch_destroy): moments, populations, Nusselt, residual and
 * derived constants of that cavity.  Do not step, reset or destroy it. */
mclbm_cavity* mclbm_batch_cavity(mclbm_batch* b, int32_t idx);

/* Release the batch (waits for its stream).  Does not free dev_buf. */
int mclbm_batch_destroy(mclbm_batch* b);

/* Measurement helper: copy `bytes` (multiple of 16) from src to dst, both
 * device buffers, with a plain streaming kernel on `stream`.  Async.
 * Used to calibrate the achievable HBM bandwidth and the byte counters. */
int mclbm_copy_kernel(void* dst, const void* src, size_t bytes, void* stream);

/* Library version string and the ABI version. */
const char* mclbm_version(void);
int mclbm_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MCLBM_H */
