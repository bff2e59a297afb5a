/*
 * ecrpic.h -- C ABI of the MI355X (gfx950) ion PIC/MCC step of the ECRIS
 * model of Mironov et al., "Numerical model of Electron Cyclotron Resonance
 * Ion Source", Sec. II.
 *
 * The paper states the problem as: for a given magnetic configuration and
 * chamber (Sec. II, Table I), macro-particle ions and atoms are moved in the
 * field, collide (ion-ion Coulomb scattering, electron-impact ionisation,
 * charge exchange with atoms), are neutralised at the walls or leave through
 * the extraction aperture and are recycled at the gas inlet; the outputs are
 * the extracted charge-state distribution and gas flow (Sec. II, III.C) and
 * the density distributions (Sec. III.B).  The calls below follow that
 * statement: create a run, initialise its ions, advance N steps, read the
 * extracted-ion tallies and the density grid.
 *
 * Conventions
 *  - Every call returns ecr_status; 0 is success.  Nothing throws across the
 *    boundary.  ECR_EINVAL means a bad argument and leaves the run unchanged.
 *  - Units are SI (m, s, kg, T, m^-3, m^3/s, m^2, V/m); temperatures and
 *    energies carry an _eV suffix.
 *  - Device memory: the caller owns one device buffer (the arena) of at
 *    least ecr_footprint() bytes and a HIP stream; the library carves the
 *    arena and never allocates device memory itself.  Host buffers passed to
 *    read/get/set calls belong to the caller and are only used during the
 *    call.  ecr_destroy frees the host handle only.
 *  - ecr_step and ecr_init_ions are asynchronous on the run's stream; the
 *    read/get/set calls synchronise that stream.
 *  - A handle is not thread-safe; distinct handles may be used concurrently
 *    on distinct streams.
 */
#ifndef ECRPIC_H
#define ECRPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ECR_ABI_VERSION 7u
#define ECR_MAX_SPECIES 4
#define ECR_MAX_Q 32          /* charge-state slots per species: Q = 0..31 */
#define ECR_MAX_NION 4        /* electrons one ionisation may remove: Q -> Q+n, n = 1..4 */
#define ECR_FPT_BINS 32       /* log2 bins of first-passage times */
#define ECR_BIRTH_NONE 0xffffffffu /* birth step of an atom, or of an ion of unknown origin */

typedef enum {
  ECR_OK = 0,
  ECR_EINVAL = -1,   /* bad argument; nothing changed */
  ECR_ENOMEM = -2,   /* arena smaller than ecr_footprint() */
  ECR_EDEVICE = -3,  /* a HIP call failed; the run is now unusable except read/destroy */
  ECR_ESTATE = -4,   /* call not valid in the run's state */
  ECR_ENUMERIC = -5, /* anomalies counted (non-finite state, or per-step collision probability > 0.1) */
  ECR_EDT = -6,      /* time step too large for first-order Monte-Carlo collisions */
  ECR_EABI = -7      /* abi_version mismatch */
} ecr_status;

typedef enum { ECR_FP64 = 0, ECR_FP32_MIXED = 1 } ecr_precision;

/* process switches (process_mask) */
enum {
  ECR_P_PUSH = 1,     /* Boris push in the magnetic (and optional electric) field + wall/aperture loss */
  ECR_P_IONIZE = 2,   /* electron-impact ionisation Q -> Q+n (n = 1, and 2..4 where the species gives rates) */
  ECR_P_CX = 4,       /* charge exchange with the background neutral gas */
  ECR_P_COULOMB = 8,  /* ion-ion Coulomb scattering: Takizuka-Abe pairing, Nanbu angle */
  ECR_P_DEPOSIT = 16, /* cloud-in-cell density deposit */
  ECR_P_ALL = 31,     /* the five processes above: the fixed-background step */
  ECR_P_HEAT = 32,    /* electron-ion heating and diffusion kick (Sec. II): each ion that stays in the
                         chamber gets dV = D (R + delta) |R| / |R + delta| before ionisation and charge
                         exchange, D^2 = 3.715e-6 n_e lnL_ei Q^2 dt / (M_amu^2 sqrt(T_e)) (SI; the printed
                         formula's Q read as Q^2, the heating rate's stated charge law), R uniform in
                         [-1/2, 1/2]^3 (one draw of Philox stream 5); with ECR_FLAG_SELF_NE, n_e is the
                         cell's and delta the electron diamagnetic bias: the 9-point stencil of the cell
                         electron density in the ion's z plane (cells beyond the mesh: 0) times
                         -R_L / n_e(cell), R_L = 2.38e-6 sqrt(T_e) / (|B(cell centre)| hx); with the fixed
                         background, n_e and T_e are the zone's and delta = 0 */
  ECR_P_ELASTIC = 64  /* elastic ion-atom scattering on the background neutrals (Sec. II): isotropic in the
                         centre-of-mass frame of the ion and a Maxwellian neutral at T_n (Philox stream 6) */
};

/* density fields (bit f of deposit_mask enables field f) */
enum {
  ECR_F_ION_N = 0,  /* sum of CIC weights of ions (Q >= 1) */
  ECR_F_ION_Q = 1,  /* sum of Q x CIC weight of ions */
  ECR_F_ATOM_N = 2, /* sum of CIC weights of atoms (Q = 0) */
  ECR_F_ION_P = 3,  /* sum of CIC weight x M |v|^2 / 3 of ions, J: with no mean flow, the ion pressure
                       n k T (Sec. III.B) times the node volume; its own kernel, only when requested */
  ECR_N_FIELDS = 4
};

/* run flags */
enum {
  ECR_FLAG_EVENTS = 1, /* record each particle's event code of the last step */
  ECR_FLAG_SPLIT = 2,  /* the step as separate kernels (Coulomb pairing order, Coulomb collisions, push + loss +
                          MCC, deposit) instead of one kernel for the whole step, for per-kernel timing; the
                          results are the same (the density and the FP64 sums within atomic rounding).  Runs with
                          an electric field grid or a magnetic field map always run the separate kernels.  In
                          this form a Coulomb chunk of more than 1024 ions skips its collisions for the step and
                          the read calls report it (ECR_ENUMERIC); the one-kernel step has no such limit */
  ECR_FLAG_SELF_NE = 4, /* electron density = ion charge density of the particle's cell at the start of the
                          step (Sec. II: charge neutrality) instead of the fixed ne_in/ne_out background;
                          the zone still picks the rate table (warm inside, cold outside), and the
                          ionisation probability is n_e k_Q dt (ne_in/ne_out only bound the dt check) */
  ECR_FLAG_HEAT_ISOTROPIC = 8, /* the heating kick without its diamagnetic bias (delta = 0): the paper's
                                  ablation that switches off the plasma diffusion by e-i collisions (Sec. IV) */
  ECR_FLAG_SELF_N0 = 16, /* the neutral gas of charge exchange and elastic scattering is the tracked atoms (Sec. II):
                           n0 = weight x (atoms of the ion's species in its cell at the start of the step) / cell
                           volume, instead of the species' uniform n0_m3 (which then only bounds the dt check) */
  ECR_FLAG_CX_PARTNER = 32 /* needs ECR_FLAG_SELF_N0.  Every charge exchange takes its electron from a tracked atom
                              (Sec. II): at the end of the step, in each collision cell (the cell at the last sort),
                              the exchanges of species s ionise that many atoms of species s, picked in the order
                              of (word 3 of the particle's Philox stream-1 draw, id) among the cell's atoms that did
                              not become atoms in this step; each becomes a Q = 1 ion born in the step
                              (ECR_EV_CX_PARTNER).  A Q = 1 ion that exchanges becomes an atom with its own velocity;
                              Q >= 2 exchanges are as without the flag.  Exchanges left without an atom are counted
                              in cx_unmatched.  The density of the step is deposited before the partners change.
                              With this flag an atom's birth is the step it became one (walls, aperture, resonant
                              exchange) instead of ECR_BIRTH_NONE. */
};

/* event codes returned by ecr_event_log */
enum {
  ECR_EV_NONE = 0,
  ECR_EV_IONIZE = 1,
  ECR_EV_CX = 2,
  ECR_EV_WALL = 3,
  ECR_EV_EXTRACT = 4,
  ECR_EV_ELASTIC = 5,
  ECR_EV_CX_PARTNER = 6 /* an atom made a Q = 1 ion as the partner of an exchange (ECR_FLAG_CX_PARTNER) */
};

/* One ion species (the paper models argon, Sec. II; a second species is allowed). */
typedef struct {
  double mass_amu;
  int32_t z_max;                      /* highest charge state, <= 31 */
  uint32_t cx_forbidden_mask;         /* bit Q set: no charge exchange from Q (argon: Q = 2) */
  double fraction;                    /* share of particles; ids are assigned in order */
  double k_ion_in_m3s[ECR_MAX_Q];     /* ionisation rate Q -> Q+1 inside the ECR zone */
  double k_ion_out_m3s[ECR_MAX_Q];    /* same, outside the zone */
  double sigma_cx1_m2;                /* charge-exchange cross-section of Q = 1; Q scales it linearly */
  double n0_m3;                       /* background neutral density (charge-exchange target) */
  /* Sec. II, multiple ionisation: rate of Q -> Q+n for n = 2..ECR_MAX_NION ([n-2]); entries whose Q + n
     passes z_max are ignored.  One uniform picks among the channels n = 1..4, charge exchange and elastic
     scattering by running sums of their probabilities, in that order. */
  double k_ion_multi_in_m3s[ECR_MAX_NION - 1][ECR_MAX_Q];
  double k_ion_multi_out_m3s[ECR_MAX_NION - 1][ECR_MAX_Q];
  double sigma_el1_m2;                /* elastic ion-atom cross-section of Q = 1 (ECR_P_ELASTIC); Q scales it
                                         linearly, P_el = n0 (Q sigma_el1) |v| dt */
} ecr_species;

typedef struct {
  uint32_t abi_version;               /* ECR_ABI_VERSION */
  int32_t precision;                  /* ecr_precision */
  uint32_t process_mask;              /* ECR_P_* */
  uint32_t deposit_mask;              /* bits of ECR_F_* */
  uint32_t flags;                     /* ECR_FLAG_* */
  int32_t sort_every;                 /* steps between sorts by cell (>= 1) */
  uint64_t seed;                      /* Philox key */
  int64_t n_particles;                /* 0 .. 2^31-1 */
  double dt_s;
  int32_t nx, ny, nz;                 /* cells of the mesh over [-R0,R0]^2 x [-L/2,L/2] */
  int32_t n_species;                  /* 1 .. ECR_MAX_SPECIES */
  double R0_m, L_m;                   /* chamber radius and length; extraction flange at z = +L/2 */
  double r_ap_m;                      /* extraction aperture radius */
  double inlet_x_m, inlet_y_m;        /* gas inlet on the injection flange z = -L/2 */
  double B0_T, mirror_k, BH_T;        /* on-axis Bz = B0 (1 + k (2z/L)^2); hexapole BH at r = R0 */
  double zone_a_m, zone_c_m;          /* ECR zone: ellipsoid x^2/a^2 + y^2/a^2 + z^2/c^2 < 1 */
  double ne_in_m3, ne_out_m3;         /* electron density inside / outside the zone */
  double Ti0_eV;                      /* initial ion temperature */
  double T_wall_eV;                   /* wall re-emission temperature */
  double T_n_eV;                      /* neutral gas temperature (charge-exchange partners) */
  double dE_cx_eV;                    /* energy release of multiply-charged charge exchange */
  double lnL_ii;                      /* ion-ion Coulomb logarithm */
  double lnL_ei;                      /* electron-ion Coulomb logarithm (ECR_P_HEAT; the paper: 17) */
  double Te_in_eV, Te_out_eV;         /* electron temperature inside / outside the zone (ECR_P_HEAT; > 0) */
  double weight;                      /* real ions per macro-particle; 0: n_e,in V_zone / N */
  const double *efield_nodes;         /* host, [3][(nx+1)(ny+1)(nz+1)] V/m node field, or NULL (E = 0) */
  const double *bfield_nodes;         /* host, [3][(nx+1)(ny+1)(nz+1)] T node magnetic field (a field-solver map,
                                         as the paper's Superfish maps), node index ix + (nx+1)(iy + (ny+1) iz),
                                         interpolated trilinearly at the particle in place of the analytic
                                         B0/mirror_k/BH field, and at the cell centre for the heating kick;
                                         copied into the arena at create; or NULL (analytic field) */
  ecr_species species[ECR_MAX_SPECIES];
} ecr_params;

typedef struct {
  uint64_t extracted[ECR_MAX_SPECIES][ECR_MAX_Q]; /* left through the aperture, by charge at exit */
  uint64_t wall[ECR_MAX_SPECIES][ECR_MAX_Q];      /* neutralised at a wall, by charge at impact */
  uint64_t ionized[ECR_MAX_SPECIES][ECR_MAX_Q];   /* ionisation events, by charge before */
  uint64_t cx[ECR_MAX_SPECIES][ECR_MAX_Q];        /* charge-exchange events, by charge before */
  uint64_t cx_products[ECR_MAX_SPECIES];          /* untracked singly-charged products of Q >= 3 exchange */
  uint64_t recycled;                              /* particles returned at the gas inlet */
  uint64_t anomalies;
  int64_t steps;                                  /* steps since init_ions / set_state */
  double coul_dp[3];                              /* total momentum change in Coulomb collisions, kg m/s */
  double coul_de;                                 /* total kinetic-energy change in Coulomb collisions, J */
  double coul_e;                                  /* kinetic energy of the collision pools before, J */
  /* Diagnostics of the extracted ions and of the losses (Sec. III.B, III.D
   * and the power balance of Sec. II).  An ion's birth is the step in which
   * it was made from an atom (ionisation of Q = 0, or resonant Q = 1 charge
   * exchange, which hands the charge to the neutral partner), or step 0 for
   * the ions of ecr_init_ions; its first-passage time is (step of its
   * extraction - birth) steps.  Ions of unknown birth (set_state without
   * births) are counted in extracted but not here. */
  uint64_t fpt_n[ECR_MAX_SPECIES][ECR_MAX_Q];       /* extracted ions of known birth, by charge at exit */
  uint64_t fpt_sum[ECR_MAX_SPECIES][ECR_MAX_Q];     /* sum of their first-passage times, steps */
  uint64_t fpt_hist[ECR_MAX_SPECIES][ECR_FPT_BINS]; /* all charges: bin k counts times t with floor(log2 t) = k (t <= 1 in bin 0) */
  double extracted_r[ECR_MAX_SPECIES][ECR_MAX_Q];   /* sum of sqrt(x^2 + y^2) where the extracted ions cross the flange, m */
  double lost_ke[ECR_MAX_SPECIES];                  /* kinetic energy of the ions (Q >= 1) lost to the walls and the aperture, J */
  uint64_t ionized_n[ECR_MAX_SPECIES][ECR_MAX_NION];/* ionisation events by electrons removed ([n-1]) */
  uint64_t elastic[ECR_MAX_SPECIES][ECR_MAX_Q];     /* elastic ion-atom collisions, by charge */
  uint64_t cx_unmatched[ECR_MAX_SPECIES];           /* ECR_FLAG_CX_PARTNER: exchanges that found no atom in their cell */
} ecr_tallies;

/* Host particle arrays indexed by particle id (length n). */
typedef struct {
  double *x, *y, *z, *vx, *vy, *vz;
  uint8_t *q;        /* charge state */
  uint8_t *species;  /* get only (ignored by set: species follow the id order) */
  uint32_t *cell;    /* collision cell (cell of the last sort); set: may be NULL -> sorted at the next step */
  int64_t n;
  int64_t step;      /* step counter (Philox counter word 1) */
  uint32_t *birth;   /* birth step (ECR_BIRTH_NONE: atom or unknown); may be NULL (set: all unknown) */
} ecr_state_view;

typedef struct ecr_run ecr_run;

/* Device bytes a run with these parameters needs.  ECR_EINVAL on bad params. */
ecr_status ecr_footprint(const ecr_params *params, size_t *device_bytes);

/* Create a run of the ion model of Sec. II (its chamber, field, electron
 * background and species; Table I gives the paper's values) in a
 * caller-owned device arena of arena_bytes >= ecr_footprint() bytes (the
 * caller keeps ownership and must keep it alive until ecr_destroy), bound to
 * a caller-owned HIP stream (NULL: the null stream).  Copies params (and the
 * E-field nodes, if given) and uploads the derived tables (Boris factors,
 * per-step ionisation and exchange probabilities, Nanbu's A(s)).
 * ECR_EINVAL on bad parameters or a short arena, ECR_EABI on a foreign
 * abi_version, ECR_EDT if the per-step ionisation plus charge-exchange
 * probability can exceed 0.1 (the first-order Monte Carlo collision limit
 * of Sec. II), ECR_EDEVICE if the upload fails.  *out is set only on
 * ECR_OK. */
ecr_status ecr_create(const ecr_params *params, void *device_arena, size_t arena_bytes,
                      void *hip_stream, ecr_run **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * run as ecr_create, with the arena replaced by a static workspace of
 * 64 MiB that the library holds in device memory, one per GPU it runs on,
 * from the first call on that GPU until the process ends.  The call itself
 * allocates no device memory (no hipMalloc, no allocating library routine).
 * It binds the run to the current device's workspace and to hip_stream
 * (NULL: the null stream) and returns that device's one static handle.
 * A run whose ecr_footprint() exceeds the workspace is rejected with
 * ECR_ENOMEM and a message giving both sizes.  The workspace keeps the last
 * run's contents: the run is set up exactly as on an uninitialised arena
 * (tables uploaded, tallies and density zeroed; the particle state comes
 * from ecr_init_ions or ecr_set_state).  One static run per device at a
 * time: a second call while one is live returns ECR_ESTATE; ecr_destroy
 * releases the workspace for the next call (it waits for the run's stream).
 * Runs on one device that overlap in time would race on the workspace,
 * which is why the second call is refused.  Every other call takes the
 * handle as it takes one of ecr_create. */
ecr_status ecr_create_static(const ecr_params *params, void *hip_stream, ecr_run **out);

/* Initial ions: uniform in the ECR-zone ellipsoid, Maxwellian at Ti0, Q = 1
 * (Sec. II); zeroes tallies and density; step counter 0. */
ecr_status ecr_init_ions(ecr_run *run);

/* Advance n_steps time steps of Sec. II: the sort by cell every sort_every
 * steps; then, per step, the Coulomb block (Takizuka-Abe pairing within
 * each collision cell, Nanbu's scattering angle), the Boris push in the
 * magnetic field, wall and aperture loss, ionisation and charge exchange
 * with the background (Monte Carlo collisions), and the cloud-in-cell
 * deposit of the densities.  Asynchronous on the run's stream; launch
 * failures return ECR_EDEVICE with the HIP message in ecr_last_error. */
ecr_status ecr_step(ecr_run *run, int64_t n_steps);

/* Same as ecr_step(run, n_steps), with the same results, but every whole
 * sort period (sort_every steps starting at a step that is a multiple of
 * sort_every, the period's sort first) is replayed from a HIP graph that
 * the run captures on first use: one launch instead of ~3 per step.  Steps
 * outside whole periods, runs on the null stream and runs being profiled
 * are launched step by step as ecr_step does.  The run keeps at most two
 * graphs (one per sort buffer) until ecr_destroy.  Asynchronous. */
ecr_status ecr_step_graph(ecr_run *run, int64_t n_steps);

/* Advance several independent runs (the scans of Sec. III: one run per
 * gas-flow or power point) that share the stream hip_stream by n_steps
 * each, with the same results as ecr_step on each run.  Each step of all
 * the runs whose step is the default one (fused step, deposit of exactly
 * ECR_F_ION_N and ECR_F_ION_Q, no optional physics, not profiled) is one
 * kernel launch over the chunks of every such run (at most 32 runs per
 * launch), which reads each run's arguments from a job in the run's own
 * arena; other runs are stepped as ecr_step does.  When every run is at the
 * start of a sort period of the same length and n_steps covers it, the
 * period is replayed from a graph captured for that set of runs (captured
 * the second time the set comes up, kept until one of its runs is
 * destroyed).  ECR_EINVAL if a run is NULL, failed, uninitialised, bound to
 * another stream or listed twice.  Asynchronous. */
ecr_status ecr_step_batch(ecr_run *const *runs, int32_t n_runs, int64_t n_steps, void *hip_stream);

/* Tallies since the last init/set_state.  Synchronises.  ECR_ENUMERIC (with
 * the tallies filled in) when anomalies > 0. */
ecr_status ecr_read_tallies(ecr_run *run, ecr_tallies *host_out);

/* Time-integrated CIC deposit of one field: (nx+1)(ny+1)(nz+1) doubles in
 * x-fastest node order into host_out (caller-owned), plus the number of
 * deposited steps; divided by that number these are the time-averaged
 * distributions of Sec. III.B.  Synchronises.  ECR_EINVAL for a field
 * outside ECR_F_* or a NULL output. */
ecr_status ecr_read_density(ecr_run *run, uint32_t field, double *host_out, int64_t *steps_accum);

/* Particle state by id (checkpoint and parity).  Synchronises. */
ecr_status ecr_get_state(ecr_run *run, ecr_state_view *host_out);

/* Replace the particle state (by id), set the step counter, zero tallies and
 * density.  ECR_EINVAL if a charge state exceeds its species' z_max or a cell
 * is out of range.  Synchronises. */
ecr_status ecr_set_state(ecr_run *run, const ecr_state_view *host_in);

/* Event codes (ECR_EV_*) of the last step, by particle id; needs
 * ECR_FLAG_EVENTS (else ECR_ESTATE).  Synchronises. */
ecr_status ecr_event_log(ecr_run *run, uint8_t *host_out);

/* Macro-particle weight in use (real ions per macro-particle). */
ecr_status ecr_weight(const ecr_run *run, double *weight);

/* Per-kernel timing.  ecr_profile(run, mask): bit k of mask (1 << ECR_K_*)
 * brackets every launch of kernel kind k with HIP events on the run's
 * stream (-1: every kind; 0: off) and resets the counters;
 * ecr_kernel_times returns, per kind, the summed milliseconds and the launch
 * count since then.  Timed runs are stepped launch by launch (ecr_step_graph
 * does not replay graphs while any bit is set). */
enum {
  ECR_K_SORT = 0,       /* the sort by cell (count, scan, scatter, chunk table) */
  ECR_K_COULOMB = 1,    /* Coulomb pairing: pool order and pair lists */
  ECR_K_PUSH = 2,       /* push + wall/aperture + ionisation/charge exchange */
  ECR_K_DEPOSIT = 3,    /* deposit alone (ECR_FLAG_SPLIT) */
  ECR_K_FUSED = 4,      /* push + wall/aperture + ionisation/charge exchange + deposit in one kernel */
  ECR_K_COUL_PAIRS = 5, /* Coulomb scattering of the listed pairs */
  ECR_K_PARTNER = 6,    /* exchange partners (ECR_FLAG_CX_PARTNER) */
  ECR_K_STEP = 7,       /* the whole step in one kernel: Coulomb pairing and collisions, push, loss, MCC, deposit */
  ECR_N_KERNELS = 8
};
ecr_status ecr_profile(ecr_run *run, int32_t enable);
ecr_status ecr_kernel_times(ecr_run *run, double *ms_out, int64_t *launches_out);
/* Bracket only one launch in `stride` (>= 1, default 1) of each timed kind,
 * counted from the next ecr_profile call: sampled timing that leaves the
 * other launches without event packets.  ECR_EINVAL for stride < 1. */
ecr_status ecr_profile_stride(ecr_run *run, int32_t stride);

/* Message of the last error on this run (NULL run: of the calling thread). */
const char *ecr_last_error(const ecr_run *run);

ecr_status ecr_destroy(ecr_run *run);

/* Self-test entry points (device buffers, run on the given stream):
 * Philox4x32-10 of counters (c0 = i + ctr0, c1, c2, c3) for i < n with key
 * (seed lo, seed hi) into out[4*i..4*i+3]; and the binary64 quotient and
 * square root a[i]/b[i], sqrt(a[i]) into q[i], r[i]. */
ecr_status ecr_selftest_philox(uint64_t seed, uint32_t ctr0, uint32_t c1, uint32_t c2, uint32_t c3,
                               int64_t n, uint32_t *out_dev, void *hip_stream);
ecr_status ecr_selftest_divsqrt(const double *a_dev, const double *b_dev, int64_t n, double *q_dev,
                                double *r_dev, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
