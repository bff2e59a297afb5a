/*
 * ecr_oracle.h -- plain FP64 CPU oracle of the ion PIC/MCC step of the ECRIS
 * model (Mironov et al., "Numerical model of Electron Cyclotron Resonance Ion
 * Source", Sec. II).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a slow, obviously correct implementation.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant generator with the GPU library.
 *
 * Units are SI throughout (m, s, kg, T, m^-3, m^3/s, m^2); temperatures and
 * energies carry an _eV suffix.  Particle arrays are indexed by particle id.
 */
#ifndef ECR_ORACLE_H
#define ECR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXS 4   /* species */
#define ORC_MAXQ 32  /* charge-state slots per species, Q = 0..31 */
#define ORC_MAXN 4   /* electrons removed by one ionisation, n = 1..4 */
#define ORC_FPT_BINS 32            /* log2 bins of first-passage times */
#define ORC_BIRTH_NONE 0xFFFFFFFFu /* birth of an atom or of an ion of unknown origin */

/* process switches */
#define ORC_P_PUSH 1u      /* Boris push + wall/aperture boundary */
#define ORC_P_IONIZE 2u    /* electron-impact ionisation Q -> Q+1 */
#define ORC_P_CX 4u        /* charge exchange with background neutrals */
#define ORC_P_COULOMB 8u   /* ion-ion Coulomb scattering (TA pairing, Nanbu angle) */
#define ORC_P_DEPOSIT 16u  /* cloud-in-cell density deposit */
#define ORC_P_HEAT 32u     /* electron-ion heating kick, biased along the electron diamagnetic drift */
#define ORC_P_ELASTIC 64u  /* elastic ion-atom scattering on the background neutrals, isotropic */

/* deposit fields */
#define ORC_F_ION_N 0  /* sum of CIC weights of ions (Q >= 1) */
#define ORC_F_ION_Q 1  /* sum of Q * CIC weight of ions */
#define ORC_F_ATOM_N 2 /* sum of CIC weights of atoms (Q = 0) */
#define ORC_F_ION_P 3  /* sum of CIC weight * M |v|^2 / 3 of ions (J): ion pressure x cell volume */
#define ORC_NFIELDS 4

/* per-particle event codes of the last step */
#define ORC_EV_NONE 0
#define ORC_EV_IONIZE 1
#define ORC_EV_CX 2
#define ORC_EV_WALL 3
#define ORC_EV_EXTRACT 4
#define ORC_EV_ELASTIC 5
#define ORC_EV_CX_PARTNER 6 /* an atom made an ion as the partner of an exchange (cx_partner) */

typedef struct {
  double mass_amu;
  int32_t z_max;              /* highest charge state (<= 31) */
  uint32_t cx_forbidden_mask; /* bit Q set: no charge exchange from Q */
  double fraction;            /* share of the particles, assigned in id order */
  double k_in[ORC_MAXQ];      /* ionisation rate Q->Q+1 inside the zone, m^3/s */
  double k_out[ORC_MAXQ];     /* same, outside the zone */
  double sigma_cx1;           /* charge-exchange cross-section of Q=1, m^2 */
  double n0;                  /* background neutral density, m^-3 */
  double k_multi_in[ORC_MAXN - 1][ORC_MAXQ];  /* rate Q -> Q+n, n = 2..4 ([n-2]), inside the zone */
  double k_multi_out[ORC_MAXN - 1][ORC_MAXQ]; /* same, outside */
  double sigma_el1;           /* elastic ion-atom cross-section of Q=1, m^2 (Q scales it linearly) */
} orc_species;

typedef struct {
  uint64_t seed;
  int64_t n;                  /* number of macro-particles */
  double dt;
  int32_t sort_every;
  uint32_t process_mask;
  uint32_t deposit_mask;      /* bit f: deposit field f */
  int32_t nx, ny, nz;
  double R0, L, r_ap, inlet_x, inlet_y;
  double B0, mirror_k, BH;
  double zone_a, zone_c, ne_in, ne_out;
  double Ti0_eV, T_wall_eV, T_n_eV, dE_cx_eV, lnL, weight;
  const double *efield;       /* [3][(nx+1)(ny+1)(nz+1)] node field, V/m, or NULL */
  int32_t n_species;
  orc_species sp[ORC_MAXS];
  int32_t self_ne;            /* 1: electron density = ion charge density of the cell (Sec. II) */
  double lnL_ei;              /* electron-ion Coulomb logarithm (the paper: 17) */
  double Te_in_eV, Te_out_eV; /* electron temperature inside (warm) and outside (cold) the zone */
  const double *bfield;       /* [3][(nx+1)(ny+1)(nz+1)] node magnetic field, T, interpolated trilinearly
                                 in place of the analytic field; or NULL */
  int32_t heat_isotropic;     /* 1: the heating kick without its diamagnetic bias (Sec. IV ablation) */
  int32_t self_n0;            /* 1: the neutral density of charge exchange and elastic scattering is that of the
                                 tracked atoms of the species in the ion's cell, not the species' n0 */
  int32_t cx_partner;         /* 1 (needs self_n0): every charge exchange ionises a tracked atom of the ion's
                                 species and collision cell at the end of the step; a Q = 1 ion becomes an
                                 atom with its own velocity */
} orc_params;

typedef struct {
  uint64_t extracted[ORC_MAXS][ORC_MAXQ];
  uint64_t wall[ORC_MAXS][ORC_MAXQ];
  uint64_t ionized[ORC_MAXS][ORC_MAXQ];
  uint64_t cx[ORC_MAXS][ORC_MAXQ];
  uint64_t cx_products[ORC_MAXS];
  uint64_t recycled;
  uint64_t anomalies;
  int64_t steps;
  double coul_dp[3];  /* total momentum change from Coulomb collisions, kg m/s */
  double coul_de;     /* total kinetic-energy change, J */
  double coul_e;      /* total kinetic energy of the collision pools before, J */
  /* losses and extracted-ion diagnostics (Sec. II power balance, Sec. III.B
   * radial size, Sec. III.D first-passage times); an ion's birth is the step
   * in which it was made from an atom (ionisation of Q = 0, or resonant
   * Q = 1 charge exchange), step 0 for the initial ions */
  uint64_t fpt_n[ORC_MAXS][ORC_MAXQ];   /* extracted ions of known birth, by charge at exit */
  uint64_t fpt_sum[ORC_MAXS][ORC_MAXQ]; /* sum of (extraction step - birth) */
  uint64_t fpt_hist[ORC_MAXS][ORC_FPT_BINS]; /* bin floor(log2 t), t <= 1 in bin 0 */
  double extracted_r[ORC_MAXS][ORC_MAXQ];    /* sum of the crossing radius of extracted particles, m */
  double lost_ke[ORC_MAXS];             /* kinetic energy of ions (Q >= 1) lost to walls and aperture, J */
  uint64_t ionized_n[ORC_MAXS][ORC_MAXN];  /* ionisations by electrons removed ([n-1]) */
  uint64_t elastic[ORC_MAXS][ORC_MAXQ];    /* elastic ion-atom collisions, by charge */
  uint64_t cx_unmatched[ORC_MAXS];         /* cx_partner: exchanges that found no atom in their cell */
} orc_tallies;

typedef struct orc_sim orc_sim;

int orc_create(const orc_params *p, orc_sim **out);
void orc_destroy(orc_sim *s);
int orc_init_ions(orc_sim *s);
int orc_step(orc_sim *s, int64_t n_steps);
/* arrays indexed by particle id; cell may be NULL (then the next step sorts) */
/* birth may be NULL: every ion of unknown birth (ORC_BIRTH_NONE) */
int orc_set_state(orc_sim *s, int64_t step, const double *x, const double *y, const double *z,
                  const double *vx, const double *vy, const double *vz, const uint8_t *q,
                  const uint32_t *cell, const uint32_t *birth);
int orc_get_state(const orc_sim *s, int64_t *step, double *x, double *y, double *z, double *vx,
                  double *vy, double *vz, uint8_t *q, uint8_t *species, uint32_t *cell, uint32_t *birth);
int orc_get_tallies(const orc_sim *s, orc_tallies *t);
int orc_get_density(const orc_sim *s, int field, double *out, int64_t *steps);
int orc_get_events(const orc_sim *s, uint8_t *out);
double orc_weight(const orc_sim *s);
/* explicit particle ids (Philox counter word, pairing tie-break) and species */
int orc_set_ids(orc_sim *s, const uint32_t *ids, const uint8_t *species);
void orc_philox_fill(uint64_t seed, uint32_t ctr0, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
                     uint32_t *out);

/* unit entry points used by the pin tests */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double orc_u53(uint32_t a, uint32_t b);
void orc_field(const orc_sim *s, double x, double y, double z, double B[3]);
void orc_boris(const orc_sim *s, int species, int q, const double E[3], double x[3], double v[3]);
double orc_nanbu_A(const orc_sim *s, double sv);
double orc_nanbu_A_root(double sv);
double orc_nanbu_omc(const orc_sim *s, double sv, double u);
int orc_segment_exit(const orc_sim *s, const double x0[3], const double x1[3], double *f);
uint32_t orc_cell_of(const orc_sim *s, double x, double y, double z);

#ifdef __cplusplus
}
#endif
#endif
