/*
 * ecr_oracle.c -- plain FP64 CPU oracle of the ion PIC/MCC step of the ECRIS
 * model of Mironov et al., Sec. II ("The model description").
 *
 * TEST INFRASTRUCTURE ONLY: it exists to check the GPU library.  It is built
 * with -O2 -ffp-contract=off and no fast-math, keeps every particle in id
 * order, and does each step of the method in the order the method states,
 * with no blocking, fusion or reordering:
 *
 *   sort by cell (every sort_every steps) -> ion-ion Coulomb scattering
 *   (Takizuka-Abe pairing, Nanbu angle) -> Boris push in the minimum-B field
 *   -> wall / extraction-aperture loss with recycling -> electron-impact
 *   ionisation or charge exchange -> cloud-in-cell deposit.
 *
 * Where the paper leaves a detail open, the oracle takes one stated reading;
 * each one is named at the function that implements it.  Random numbers come
 * from Philox4x32-10 (Salmon et al., SC'11) keyed by the run seed, with the
 * counter (particle id, step, stream, call index), so that any implementation
 * of the same definition draws the same numbers.
 */
#include "ecr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* SI (CODATA 2018) constants */
#define E_CHARGE 1.602176634e-19
#define AMU 1.66053906660e-27
#define EPS0 8.8541878128e-12
#define PI 3.14159265358979323846
#define EPS_WALL 1e-9 /* re-emission offset from a wall, m */

/* Philox stream ids (third counter word) */
enum { S_INIT = 0, S_STEP = 1, S_COUL = 2, S_BND = 3, S_CX = 4, S_HEAT = 5, S_EL = 6 };

/* Nanbu A(s) table: nodes s = 2^e (1 + j/K) for e in [E_LO, E_HI], j in [0, K) */
#define A_E_LO (-20)
#define A_E_HI 2
#define A_K 128
#define A_NODES ((A_E_HI - A_E_LO + 1) * A_K + 1)
#define S_LO 9.5367431640625e-07 /* 2^-20: below, A = 1/s */
#define S_HI 8.0                 /* 2^3: at and above, isotropic scattering */

struct orc_sim {
  orc_params p;
  int64_t N;
  /* derived constants */
  double M[ORC_MAXS];                /* species mass, kg */
  double qmh[ORC_MAXS][ORC_MAXQ];    /* (Q e / M) dt / 2 */
  /* ionisation Q -> Q+n ([n-1]) per step [outside, inside]: probability with
   * the fixed background, rate x dt for self-consistent electrons */
  double pion[ORC_MAXS][2][ORC_MAXN][ORC_MAXQ];
  double kdt[ORC_MAXS][2][ORC_MAXN][ORC_MAXQ];
  double ccx[ORC_MAXS];              /* n0 sigma1 dt */
  double cel[ORC_MAXS];              /* n0 sigma_el1 dt */
  double sdt_cx[ORC_MAXS], sdt_el[ORC_MAXS]; /* sigma1 dt, sigma_el1 dt (neutrals from the tracked atoms) */
  int cxok[ORC_MAXS][ORC_MAXQ];
  double sig_w[ORC_MAXS], sig_n[ORC_MAXS], sig_i[ORC_MAXS], decx[ORC_MAXS];
  int64_t sp_end[ORC_MAXS];          /* particle ids [sp_end[s-1], sp_end[s]) are species s */
  double ia2, ic2, idx, idy, idz, hL, R0sq, rap2, nfac, Cs, w;
  double hx, hy, hz;                 /* cell sizes */
  double c1, c2, c3, c4;
  int nx1, ny1, nz1;
  int64_t ncell, nnode;
  double atab[A_NODES]; /* ln A at the nodes */
  /* particle state, indexed by position i; id[i] is the particle's id (its
   * Philox counter word and pairing tie-break), i unless set by orc_set_ids */
  uint32_t *id;
  double *x, *y, *z, *vx, *vy, *vz;
  uint8_t *q, *sp, *ev;
  uint32_t *cell;
  uint32_t *birth;  /* step the ion was made from an atom, or ORC_BIRTH_NONE */
  uint32_t *chg;    /* self-consistent electrons: ion charge per cell at the start of the step */
  uint32_t *atoms;  /* tracked neutrals: atoms per species and cell at the start of the step [s][cell] */
  uint32_t *cxreq;  /* cx_partner: exchanges of the step per species and collision cell [s][cell] */
  /* cell order */
  uint32_t *order, *cell_off;
  int64_t step;
  int need_sort;
  orc_tallies t;
  double *dens[ORC_NFIELDS];
  int64_t dens_steps;
  /* scratch for the Coulomb pools */
  uint32_t *pool;
  uint32_t *pkey;
};

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 and Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).       */
/* One round maps (c0,c1,c2,c3) with key (k0,k1) to                           */
/*   (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0));       */
/* the key is bumped by the Weyl constants before every round but the first. */
/* The 64-bit instance is built from the same macro and is checked against   */
/* an independent implementation in the tests.                               */
/* ------------------------------------------------------------------------ */
static void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}
#define PHILOX_BODY(T, MULHILO, M0, M1, W0, W1)                                 \
  T c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1]; \
  for (int r = 0; r < 10; r++) {                                                \
    T h0, l0, h1, l1;                                                           \
    if (r > 0) {                                                                \
      k0 += (T)(W0);                                                            \
      k1 += (T)(W1);                                                            \
    }                                                                           \
    MULHILO((T)(M0), c0, &h0, &l0);                                             \
    MULHILO((T)(M1), c2, &h1, &l1);                                             \
    T n0 = h1 ^ c1 ^ k0, n1 = l1, n2 = h0 ^ c3 ^ k1, n3 = l0;                   \
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;                                         \
  }                                                                             \
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  PHILOX_BODY(uint32_t, mulhilo32, 0xD2511F53u, 0xCD9E8D57u, 0x9E3779B9u, 0xBB67AE85u)
}
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  PHILOX_BODY(uint64_t, mulhilo64, 0xD2E7470EE14C6C93ull, 0xCA5A826395121157ull,
              0x9E3779B97F4A7C15ull, 0xBB67AE8584CAA73Bull)
}

/* uniform double in [0,1) from 27 + 26 random bits */
double orc_u53(uint32_t a, uint32_t b) {
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

static void draw(const orc_sim *s, uint32_t id, uint32_t step, uint32_t stream, uint32_t k,
                 uint32_t out[4]) {
  uint32_t ctr[4] = {id, step, stream, k};
  uint32_t key[2] = {(uint32_t)s->p.seed, (uint32_t)(s->p.seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

/* Box-Muller: two standard normals from two uniforms in [0,1) */
static void box_muller(double ua, double ub, double *n1, double *n2) {
  double r = sqrt(-2.0 * log(1.0 - ua));
  double th = 2.0 * PI * ub;
  *n1 = r * cos(th);
  *n2 = r * sin(th);
}

/* ------------------------------------------------------------------------ */
/* Magnetic field (Sec. II, hexapole formulas and the solenoid description). */
/* Solenoid: on-axis Bz(z) = B0 (1 + k (2z/L)^2), continued off axis to      */
/* second order (Br = -(r/2) dBz/dz, Bz(r,z) = Bz(z) - (r^2/4) d2Bz/dz2), so  */
/* the field is divergence- and curl-free.  Hexapole without edge effects:   */
/* Bx += BH sin(2 theta) R^2/R0^2 = (BH/R0^2) 2xy,                           */
/* By += BH cos(2 theta) R^2/R0^2 = (BH/R0^2)(x^2 - y^2).                    */
/* ------------------------------------------------------------------------ */
static void field_B(const orc_sim *s, double x, double y, double z, double *bx, double *by,
                    double *bz) {
  double xx = x * x, yy = y * y, zz = z * z, xy = x * y;
  *bx = s->c2 * xy - (s->c1 * x) * z;
  *by = s->c3 * (xx - yy) - (s->c1 * y) * z;
  *bz = (s->p.B0 + s->c1 * zz) - s->c4 * (xx + yy);
}

static void magnetic(const orc_sim *s, double x, double y, double z, double B[3]);

void orc_field(const orc_sim *s, double x, double y, double z, double B[3]) { magnetic(s, x, y, z, B); }

/* cell-in-cell index helpers on the box [-R0,R0]^2 x [-L/2,L/2] */
static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

uint32_t orc_cell_of(const orc_sim *s, double x, double y, double z) {
  int ix = clampi((int)floor((x + s->p.R0) * s->idx), 0, s->p.nx - 1);
  int iy = clampi((int)floor((y + s->p.R0) * s->idy), 0, s->p.ny - 1);
  int iz = clampi((int)floor((z + s->hL) * s->idz), 0, s->p.nz - 1);
  return (uint32_t)ix + (uint32_t)s->p.nx * ((uint32_t)iy + (uint32_t)s->p.ny * (uint32_t)iz);
}

/* CIC: lower node index along each axis and the fractional offset */
static void cic_axis(double pos, double origin, double inv_h, int ncell, int *i, double *t) {
  double f = (pos + origin) * inv_h;
  int k = clampi((int)floor(f), 0, ncell - 1);
  *i = k;
  *t = f - (double)k;
}

/* trilinear interpolation of a node vector field [3][nnode] at (x,y,z) */
static void gather_grid(const orc_sim *s, const double *grid, double x, double y, double z, double out[3]) {
  int ix, iy, iz;
  double tx, ty, tz;
  cic_axis(x, s->p.R0, s->idx, s->p.nx, &ix, &tx);
  cic_axis(y, s->p.R0, s->idy, s->p.ny, &iy, &ty);
  cic_axis(z, s->hL, s->idz, s->p.nz, &iz, &tz);
  double wx[2] = {1.0 - tx, tx}, wy[2] = {1.0 - ty, ty}, wz[2] = {1.0 - tz, tz};
  for (int c = 0; c < 3; c++) {
    const double *F = grid + (int64_t)c * s->nnode;
    double acc = 0.0;
    for (int dz = 0; dz < 2; dz++)
      for (int dy = 0; dy < 2; dy++)
        for (int dx = 0; dx < 2; dx++) {
          int64_t node = (int64_t)(ix + dx) + (int64_t)s->nx1 * ((iy + dy) + (int64_t)s->ny1 * (iz + dz));
          acc = acc + ((wx[dx] * wy[dy]) * wz[dz]) * F[node];
        }
    out[c] = acc;
  }
}

static void gather_E(const orc_sim *s, double x, double y, double z, double E[3]) {
  gather_grid(s, s->p.efield, x, y, z, E);
}

/* the run's magnetic field: a given node map (a field-solver output such as
 * the paper's Superfish maps), interpolated trilinearly, else the analytic
 * field above */
static void magnetic(const orc_sim *s, double x, double y, double z, double B[3]) {
  if (s->p.bfield) gather_grid(s, s->p.bfield, x, y, z, B);
  else field_B(s, x, y, z, &B[0], &B[1], &B[2]);
}

/* ------------------------------------------------------------------------ */
/* Boris push (standard leapfrog rotation): v- = v + hE; t = hB;             */
/* s = 2t/(1+t.t); v' = v- + v- x t; v+ = v- + v' x s; v = v+ + hE;          */
/* x += v dt, with h = (Q e / M) dt/2.  Q = 0 gives a straight line (atoms). */
/* ------------------------------------------------------------------------ */
static void boris(const orc_sim *s, double h, const double *E, double *x, double *y, double *z,
                  double *vx, double *vy, double *vz) {
  double B[3];
  magnetic(s, *x, *y, *z, B);
  double bx = B[0], by = B[1], bz = B[2];
  double vmx = *vx, vmy = *vy, vmz = *vz;
  if (E) {
    vmx = vmx + h * E[0];
    vmy = vmy + h * E[1];
    vmz = vmz + h * E[2];
  }
  double tx = h * bx, ty = h * by, tz = h * bz;
  double t2 = (tx * tx + ty * ty) + tz * tz;
  double f = 2.0 / (1.0 + t2);
  double sx = f * tx, sy = f * ty, sz = f * tz;
  double vpx = vmx + (vmy * tz - vmz * ty);
  double vpy = vmy + (vmz * tx - vmx * tz);
  double vpz = vmz + (vmx * ty - vmy * tx);
  double nvx = vmx + (vpy * sz - vpz * sy);
  double nvy = vmy + (vpz * sx - vpx * sz);
  double nvz = vmz + (vpx * sy - vpy * sx);
  if (E) {
    nvx = nvx + h * E[0];
    nvy = nvy + h * E[1];
    nvz = nvz + h * E[2];
  }
  *vx = nvx;
  *vy = nvy;
  *vz = nvz;
  *x = *x + nvx * s->p.dt;
  *y = *y + nvy * s->p.dt;
  *z = *z + nvz * s->p.dt;
}

void orc_boris(const orc_sim *s, int species, int q, const double E[3], double x[3], double v[3]) {
  boris(s, s->qmh[species][q], E, &x[0], &x[1], &x[2], &v[0], &v[1], &v[2]);
}

/* ------------------------------------------------------------------------ */
/* Nanbu's A(s): the root of coth(A) - 1/A = exp(-s).  The root is found by  */
/* bisection on a form of the equation that has no cancellation:             */
/*   s >= 1: N(A)/(A sinh A) = exp(-s), N(A) = A cosh A - sinh A summed as    */
/*           the all-positive series sum_k 2k A^(2k+1)/(2k+1)!  (A < 3), else */
/*           coth(A) - 1/A;                                                   */
/*   s <  1: 1/A - 2/expm1(2A) = -expm1(-s)  (this is 1 - (coth A - 1/A)).    */
/* ------------------------------------------------------------------------ */
static double langevin(double a) {
  if (a < 3.0) {
    double term = a * a * a / 3.0; /* k = 1: 2 a^3 / 3! */
    double sum = term;
    for (int k = 2; k < 60; k++) {
      /* term_k / term_{k-1} = (2k / (2k-2)) * a^2 / ((2k)(2k+1)) */
      term = term * (a * a) / ((double)(2 * k - 2) * (double)(2 * k + 1));
      sum += term;
      if (term < 1e-20 * sum) break;
    }
    return sum / (a * sinh(a));
  }
  return 1.0 / tanh(a) - 1.0 / a;
}

double orc_nanbu_A_root(double sv) {
  double lo, hi;
  if (sv >= 1.0) {
    double target = exp(-sv);
    lo = 0.0;
    hi = 3.5;
    for (int it = 0; it < 400; it++) {
      double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (langevin(mid) < target) lo = mid; else hi = mid;
    }
  } else {
    double target = -expm1(-sv);
    lo = 0.5;
    hi = 1.0 / sv + 2.0;
    for (int it = 0; it < 400; it++) {
      double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      double g = 1.0 / mid - 2.0 / expm1(2.0 * mid); /* decreasing in A */
      if (g > target) lo = mid; else hi = mid;
    }
  }
  return 0.5 * (lo + hi);
}

static void build_atab(orc_sim *s) {
  for (int e = A_E_LO; e <= A_E_HI; e++)
    for (int j = 0; j < A_K; j++) {
      double sv = ldexp(1.0 + (double)j / (double)A_K, e);
      s->atab[(e - A_E_LO) * A_K + j] = log(orc_nanbu_A_root(sv));
    }
  s->atab[A_NODES - 1] = log(orc_nanbu_A_root(S_HI));
}

/* A(s) on [2^-20, 8): ln A interpolated linearly in s between the table
 * nodes (ln A is close to linear in s at both ends: -ln s + s/2 for small s,
 * ln 3 - s for large s), then exponentiated. */
double orc_nanbu_A(const orc_sim *s, double sv) {
  int ex;
  double m = frexp(sv, &ex); /* sv = m 2^ex, m in [0.5, 1) */
  int e = ex - 1;            /* sv = (2m) 2^e, 2m in [1, 2) */
  double t = (2.0 * m - 1.0) * (double)A_K;
  int j = (int)t;
  double fr = t - (double)j;
  int i = (e - A_E_LO) * A_K + j;
  return exp(s->atab[i] + fr * (s->atab[i + 1] - s->atab[i]));
}

/* 1 - cos(chi) of Nanbu's scattering angle for a uniform u in [0,1):
 * cos chi = ln(exp(-A) + 2u sinh A)/A, rewritten as
 * 1 - cos chi = -log1p(u expm1(-2A)) / A, which cannot overflow. */
double orc_nanbu_omc(const orc_sim *s, double sv, double u) {
  double omc;
  if (sv >= S_HI) {
    omc = 2.0 * u; /* isotropic */
  } else {
    double A = (sv < S_LO) ? 1.0 / sv : orc_nanbu_A(s, sv);
    omc = -log1p(u * expm1(-2.0 * A)) / A;
  }
  if (omc < 0.0) omc = 0.0;
  if (omc > 2.0) omc = 2.0;
  return omc;
}

/* ------------------------------------------------------------------------ */
/* Setup                                                                      */
/* ------------------------------------------------------------------------ */
static int species_of(const orc_sim *s, int64_t id) {
  for (int k = 0; k < s->p.n_species; k++)
    if (id < s->sp_end[k]) return k;
  return s->p.n_species - 1;
}

int orc_create(const orc_params *p, orc_sim **out) {
  if (!p || !out) return -1;
  if (p->n < 0 || p->n > 0x7fffffff || p->n_species < 1 || p->n_species > ORC_MAXS) return -1;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->sort_every < 1 || !(p->dt > 0.0)) return -1;
  if ((p->process_mask & ORC_P_HEAT) && !(p->Te_in_eV > 0.0 && p->Te_out_eV > 0.0 && p->lnL_ei >= 0.0)) return -1;
  if (p->cx_partner && !p->self_n0) return -1; /* the partners are the tracked atoms */
  orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
  if (!s) return -2;
  s->p = *p;
  s->N = p->n;
  double dt = p->dt;
  int64_t acc = 0;
  for (int k = 0; k < p->n_species; k++) {
    const orc_species *sp = &p->sp[k];
    if (sp->z_max < 0 || sp->z_max >= ORC_MAXQ) { free(s); return -1; }
    s->M[k] = sp->mass_amu * AMU;
    for (int Q = 0; Q < ORC_MAXQ; Q++) {
      s->qmh[k][Q] = ((double)Q * E_CHARGE / s->M[k]) * (dt * 0.5);
      /* probability of one ionisation in dt: 1 - exp(-n_e k dt) */
      /* channel n only up to z_max; each channel 1 - exp(-n_e k dt) */
      for (int n = 1; n <= ORC_MAXN; n++) {
        double kin = n == 1 ? sp->k_in[Q] : sp->k_multi_in[n - 2][Q];
        double kout = n == 1 ? sp->k_out[Q] : sp->k_multi_out[n - 2][Q];
        int ok = Q + n <= sp->z_max;
        s->pion[k][1][n - 1][Q] = ok ? -expm1(-(p->ne_in * kin) * dt) : 0.0;
        s->pion[k][0][n - 1][Q] = ok ? -expm1(-(p->ne_out * kout) * dt) : 0.0;
        s->kdt[k][1][n - 1][Q] = ok ? kin * dt : 0.0;
        s->kdt[k][0][n - 1][Q] = ok ? kout * dt : 0.0;
      }
      s->cxok[k][Q] = (Q >= 1 && Q <= sp->z_max && !((sp->cx_forbidden_mask >> Q) & 1u));
    }
    s->ccx[k] = (sp->n0 * sp->sigma_cx1) * dt;
    s->cel[k] = (sp->n0 * sp->sigma_el1) * dt;
    s->sdt_cx[k] = sp->sigma_cx1 * dt;
    s->sdt_el[k] = sp->sigma_el1 * dt;
    s->sig_w[k] = sqrt(p->T_wall_eV * E_CHARGE / s->M[k]);
    s->sig_n[k] = sqrt(p->T_n_eV * E_CHARGE / s->M[k]);
    s->sig_i[k] = sqrt(p->Ti0_eV * E_CHARGE / s->M[k]);
    s->decx[k] = 4.0 * p->dE_cx_eV * E_CHARGE / s->M[k];
    if (k == p->n_species - 1) acc = p->n;
    else acc += (int64_t)floor(sp->fraction * (double)p->n + 0.5);
    if (acc > p->n) acc = p->n;
    s->sp_end[k] = acc;
  }
  s->ia2 = 1.0 / (p->zone_a * p->zone_a);
  s->ic2 = 1.0 / (p->zone_c * p->zone_c);
  s->idx = (double)p->nx / (2.0 * p->R0);
  s->idy = (double)p->ny / (2.0 * p->R0);
  s->idz = (double)p->nz / p->L;
  s->hL = 0.5 * p->L;
  s->R0sq = p->R0 * p->R0;
  s->rap2 = p->r_ap * p->r_ap;
  s->c1 = ((4.0 * p->mirror_k) * p->B0) / (p->L * p->L);
  s->c2 = (2.0 * p->BH) / (p->R0 * p->R0);
  s->c3 = p->BH / (p->R0 * p->R0);
  s->c4 = ((2.0 * p->mirror_k) * p->B0) / (p->L * p->L);
  /* macro-particle weight: quasi-neutral zone at t = 0 unless given */
  double vzone = (4.0 / 3.0) * PI * (p->zone_a * p->zone_a) * p->zone_c;
  s->w = (p->weight > 0.0) ? p->weight : (p->n > 0 ? p->ne_in * vzone / (double)p->n : 0.0);
  double vcell = ((2.0 * p->R0 / p->nx) * (2.0 * p->R0 / p->ny)) * (p->L / p->nz);
  s->nfac = s->w / vcell;
  s->hx = 2.0 * p->R0 / p->nx;
  s->hy = 2.0 * p->R0 / p->ny;
  s->hz = p->L / p->nz;
  s->Cs = p->lnL * (E_CHARGE * E_CHARGE) * (E_CHARGE * E_CHARGE) / (4.0 * PI * EPS0 * EPS0);
  s->nx1 = p->nx + 1;
  s->ny1 = p->ny + 1;
  s->nz1 = p->nz + 1;
  s->ncell = (int64_t)p->nx * p->ny * p->nz;
  s->nnode = (int64_t)s->nx1 * s->ny1 * s->nz1;
  build_atab(s);

  int64_t N = p->n;
  size_t nd = (size_t)(N > 0 ? N : 1);
  s->x = calloc(nd, 8); s->y = calloc(nd, 8); s->z = calloc(nd, 8);
  s->vx = calloc(nd, 8); s->vy = calloc(nd, 8); s->vz = calloc(nd, 8);
  s->q = calloc(nd, 1); s->sp = calloc(nd, 1); s->ev = calloc(nd, 1);
  s->cell = calloc(nd, 4); s->order = calloc(nd, 4); s->id = calloc(nd, 4);
  s->pool = calloc(nd, 4); s->pkey = calloc(nd, 4); s->birth = calloc(nd, 4);
  s->cell_off = calloc((size_t)s->ncell + 1, 4);
  s->chg = calloc((size_t)s->ncell, 4);
  s->atoms = calloc((size_t)s->ncell * ORC_MAXS, 4);
  s->cxreq = calloc((size_t)s->ncell * ORC_MAXS, 4);
  for (int f = 0; f < ORC_NFIELDS; f++) s->dens[f] = calloc((size_t)s->nnode, 8);
  if (!s->x || !s->y || !s->z || !s->vx || !s->vy || !s->vz || !s->q || !s->sp || !s->ev ||
      !s->cell || !s->order || !s->id || !s->pool || !s->pkey || !s->birth || !s->cell_off || !s->chg || !s->atoms || !s->cxreq || !s->dens[0] ||
      !s->dens[1] || !s->dens[2] || !s->dens[3]) {
    orc_destroy(s);
    return -2;
  }
  for (int64_t i = 0; i < N; i++) {
    s->sp[i] = (uint8_t)species_of(s, i);
    s->id[i] = (uint32_t)i;
  }
  s->need_sort = 1;
  *out = s;
  return 0;
}

void orc_destroy(orc_sim *s) {
  if (!s) return;
  free(s->x); free(s->y); free(s->z); free(s->vx); free(s->vy); free(s->vz);
  free(s->q); free(s->sp); free(s->ev); free(s->cell); free(s->order); free(s->id);
  free(s->pool); free(s->pkey); free(s->birth); free(s->cell_off); free(s->chg); free(s->atoms); free(s->cxreq);
  for (int f = 0; f < ORC_NFIELDS; f++) free(s->dens[f]);
  free(s);
}

double orc_weight(const orc_sim *s) { return s->w; }

static void zero_accumulators(orc_sim *s) {
  memset(&s->t, 0, sizeof(s->t));
  for (int f = 0; f < ORC_NFIELDS; f++) memset(s->dens[f], 0, (size_t)s->nnode * 8);
  s->dens_steps = 0;
}

/* ------------------------------------------------------------------------ */
/* Initial ions: uniform in the zone ellipsoid (rejection sampling in its    */
/* bounding box), Maxwellian velocities at Ti0, all Q = 1.                   */
/* ------------------------------------------------------------------------ */
int orc_init_ions(orc_sim *s) {
  double a = s->p.zone_a, c = s->p.zone_c;
  for (int64_t i = 0; i < s->N; i++) {
    uint32_t id = s->id[i];
    double px = 0.0, py = 0.0, pz = 0.0;
    for (uint32_t j = 0; j < 64; j++) {
      uint32_t A[4], B[4];
      draw(s, id, 0xFFFFFFFFu, S_INIT, 2 * j, A);
      draw(s, id, 0xFFFFFFFFu, S_INIT, 2 * j + 1, B);
      double u0 = orc_u53(A[0], A[1]), u1 = orc_u53(A[2], A[3]), u2 = orc_u53(B[0], B[1]);
      double tx = a * (2.0 * u0 - 1.0), ty = a * (2.0 * u1 - 1.0), tz = c * (2.0 * u2 - 1.0);
      if (((tx * tx) * s->ia2 + (ty * ty) * s->ia2) + (tz * tz) * s->ic2 < 1.0) {
        px = tx; py = ty; pz = tz;
        break;
      }
    }
    uint32_t C[4], D[4];
    draw(s, id, 0xFFFFFFFFu, S_INIT, 0x10000u, C);
    draw(s, id, 0xFFFFFFFFu, S_INIT, 0x10001u, D);
    double n0, n1, n2, ndis;
    box_muller(orc_u53(C[0], C[1]), orc_u53(C[2], C[3]), &n0, &n1);
    box_muller(orc_u53(D[0], D[1]), orc_u53(D[2], D[3]), &n2, &ndis);
    double sg = s->sig_i[s->sp[i]];
    s->x[i] = px; s->y[i] = py; s->z[i] = pz;
    s->vx[i] = sg * n0; s->vy[i] = sg * n1; s->vz[i] = sg * n2;
    s->q[i] = 1;
    s->birth[i] = 0;
    s->ev[i] = ORC_EV_NONE;
  }
  s->step = 0;
  s->need_sort = 1;
  zero_accumulators(s);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Sort by cell: counting sort, stable in particle id.  Each particle keeps  */
/* the cell it is sorted into as its collision cell until the next sort.     */
/* ------------------------------------------------------------------------ */
static void sort_from_cells(orc_sim *s) {
  memset(s->cell_off, 0, ((size_t)s->ncell + 1) * 4);
  for (int64_t i = 0; i < s->N; i++) s->cell_off[s->cell[i] + 1]++;
  for (int64_t c = 0; c < s->ncell; c++) s->cell_off[c + 1] += s->cell_off[c];
  uint32_t *fill = (uint32_t *)malloc(((size_t)s->ncell + 1) * 4);
  memcpy(fill, s->cell_off, ((size_t)s->ncell + 1) * 4);
  for (int64_t i = 0; i < s->N; i++) s->order[fill[s->cell[i]]++] = (uint32_t)i;
  free(fill);
}

static void sort_particles(orc_sim *s) {
  for (int64_t i = 0; i < s->N; i++) s->cell[i] = orc_cell_of(s, s->x[i], s->y[i], s->z[i]);
  sort_from_cells(s);
}

/* ------------------------------------------------------------------------ */
/* Ion-ion Coulomb scattering (Sec. II): Takizuka-Abe random pairing inside */
/* each collision cell, Nanbu's scattering angle with ln(Lambda) = 10.       */
/* Reading: one pool per cell of every ion with Q >= 1 (all species), put in */
/* random order by a 32-bit key drawn per particle and step (ties by id);    */
/* even pool: pairs (0,1),(2,3),...; odd pool: (0,1),(1,2),(2,0) with dt/2   */
/* each, in that order, then (3,4),...  The pool density is m w / V_cell.    */
/* Nanbu: s = lnL e^4 (Qa Qb)^2 n dt / (4 pi eps0^2 mu^2 g^3).               */
/* ------------------------------------------------------------------------ */
static uint32_t *g_sort_key, *g_sort_id; /* qsort comparator context (single-threaded oracle) */
static int cmp_pool(const void *a, const void *b) {
  uint32_t ia = *(const uint32_t *)a, ib = *(const uint32_t *)b;
  uint32_t ka = g_sort_key[ia], kb = g_sort_key[ib];
  if (ka != kb) return ka < kb ? -1 : 1;
  uint32_t da = g_sort_id[ia], db = g_sort_id[ib];
  return da < db ? -1 : (da > db ? 1 : 0);
}

static void coulomb_pair(orc_sim *s, uint32_t ia, uint32_t ib, double nc, double dtp) {
  uint32_t W[4];
  draw(s, s->id[ia], (uint32_t)s->step, S_COUL, 0, W);
  double u = orc_u53(W[0], W[1]), u2 = orc_u53(W[2], W[3]);
  double ux = s->vx[ia] - s->vx[ib];
  double uy = s->vy[ia] - s->vy[ib];
  double uz = s->vz[ia] - s->vz[ib];
  double g2 = (ux * ux + uy * uy) + uz * uz;
  if (g2 == 0.0) return;
  double g = sqrt(g2);
  double ma = s->M[s->sp[ia]], mb = s->M[s->sp[ib]];
  double mu = (ma * mb) / (ma + mb);
  double qq = (double)s->q[ia] * (double)s->q[ib];
  double num = ((s->Cs * (qq * qq)) * nc) * dtp;
  double den = (mu * mu) * (g2 * g);
  double sv = num / den;
  double omc = orc_nanbu_omc(s, sv, u);
  double sinchi = sqrt(omc * (2.0 - omc));
  double phi = 2.0 * PI * u2;
  double ca = sinchi * cos(phi), cb = sinchi * sin(phi);
  double uperp = sqrt(ux * ux + uy * uy);
  double dux, duy, duz;
  if (uperp > 0.0) {
    dux = (((ux / uperp) * uz) * ca - ((uy / uperp) * g) * cb) - ux * omc;
    duy = (((uy / uperp) * uz) * ca + ((ux / uperp) * g) * cb) - uy * omc;
    duz = -(uperp * ca) - uz * omc;
  } else {
    dux = g * ca;
    duy = g * cb;
    duz = -(g * omc);
  }
  double ra = mu / ma, rb = mu / mb;
  s->vx[ia] = s->vx[ia] + ra * dux;
  s->vy[ia] = s->vy[ia] + ra * duy;
  s->vz[ia] = s->vz[ia] + ra * duz;
  s->vx[ib] = s->vx[ib] - rb * dux;
  s->vy[ib] = s->vy[ib] - rb * duy;
  s->vz[ib] = s->vz[ib] - rb * duz;
}

static void pool_moments(const orc_sim *s, const uint32_t *pool, int64_t m, double mom[4]) {
  mom[0] = mom[1] = mom[2] = mom[3] = 0.0;
  for (int64_t k = 0; k < m; k++) {
    uint32_t i = pool[k];
    double M = s->M[s->sp[i]];
    mom[0] += M * s->vx[i];
    mom[1] += M * s->vy[i];
    mom[2] += M * s->vz[i];
    mom[3] += 0.5 * M * ((s->vx[i] * s->vx[i] + s->vy[i] * s->vy[i]) + s->vz[i] * s->vz[i]);
  }
}

static void coulomb(orc_sim *s) {
  /* per-particle pairing key of this step: word 2 of the STEP draw */
  for (int64_t i = 0; i < s->N; i++) {
    uint32_t W[4];
    draw(s, s->id[i], (uint32_t)s->step, S_STEP, 0, W);
    s->pkey[i] = W[2];
  }
  g_sort_key = s->pkey;
  g_sort_id = s->id;
  for (int64_t c = 0; c < s->ncell; c++) {
    int64_t m = 0;
    for (uint32_t k = s->cell_off[c]; k < s->cell_off[c + 1]; k++) {
      uint32_t i = s->order[k];
      if (s->q[i] >= 1) s->pool[m++] = i;
    }
    if (m < 2) continue;
    qsort(s->pool, (size_t)m, sizeof(uint32_t), cmp_pool);
    double before[4], after[4];
    pool_moments(s, s->pool, m, before);
    double nc = (double)m * s->nfac;
    int64_t start = 0;
    if (m % 2 == 1) {
      double h = 0.5 * s->p.dt;
      coulomb_pair(s, s->pool[0], s->pool[1], nc, h);
      coulomb_pair(s, s->pool[1], s->pool[2], nc, h);
      coulomb_pair(s, s->pool[2], s->pool[0], nc, h);
      start = 3;
    }
    for (int64_t k = start; k + 1 < m; k += 2) coulomb_pair(s, s->pool[k], s->pool[k + 1], nc, s->p.dt);
    pool_moments(s, s->pool, m, after);
    for (int d = 0; d < 3; d++) s->t.coul_dp[d] += after[d] - before[d];
    s->t.coul_de += after[3] - before[3];
    s->t.coul_e += before[3];
  }
}

/* ------------------------------------------------------------------------ */
/* Wall and aperture (Sec. II): the first crossing of the step's segment    */
/* x0 -> x1 with the flanges z = +-L/2 or the cylinder r = R0 wins (ties go  */
/* to the flange).  A crossing of z = +L/2 within r_ap of the axis is an     */
/* extraction: the particle is counted and returned at the gas inlet as an   */
/* atom.  Any other crossing neutralises it at the wall: full accommodation, */
/* cosine-law (flux-Maxwellian) re-emission at the wall temperature.         */
/* ------------------------------------------------------------------------ */
enum { X_NONE = 0, X_EXT_FLANGE = 1, X_INJ_FLANGE = 2, X_CYL = 3 };

static int segment_exit(const orc_sim *s, double x0, double y0, double z0, double x1, double y1,
                        double z1, double *fout) {
  double dx = x1 - x0, dy = y1 - y0, dz = z1 - z0;
  double best = 2.0;
  int kind = X_NONE;
  if (z1 > s->hL) {
    best = (s->hL - z0) / dz;
    kind = X_EXT_FLANGE;
  } else if (z1 < -s->hL) {
    best = (-s->hL - z0) / dz;
    kind = X_INJ_FLANGE;
  }
  if (x1 * x1 + y1 * y1 > s->R0sq) {
    double a = dx * dx + dy * dy;
    double b = x0 * dx + y0 * dy;
    double c = (x0 * x0 + y0 * y0) - s->R0sq;
    double D = b * b - a * c;
    if (D < 0.0) D = 0.0;
    double sq = sqrt(D);
    double f = (b > 0.0) ? (-c) / (b + sq) : (sq - b) / a;
    if (kind == X_NONE || f < best) {
      best = f;
      kind = X_CYL;
    }
  }
  if (best < 0.0) best = 0.0;
  if (best > 1.0) best = 1.0;
  *fout = best;
  return kind;
}

int orc_segment_exit(const orc_sim *s, const double x0[3], const double x1[3], double *f) {
  return segment_exit(s, x0[0], x0[1], x0[2], x1[0], x1[1], x1[2], f);
}

/* flux-Maxwellian re-emission about the inward normal n, tangents t1, t2 */
static void reemit(orc_sim *s, int64_t i, const double n[3], const double t1[3], const double t2[3]) {
  uint32_t W[4], V[4];
  draw(s, s->id[i], (uint32_t)s->step, S_BND, 0, W);
  draw(s, s->id[i], (uint32_t)s->step, S_BND, 1, V);
  double sg = s->sig_w[s->sp[i]];
  double vn = sg * sqrt(-2.0 * log(1.0 - orc_u53(W[0], W[1])));
  double na, nb;
  box_muller(orc_u53(W[2], W[3]), orc_u53(V[0], V[1]), &na, &nb);
  double sa = sg * na, sb = sg * nb;
  s->vx[i] = (vn * n[0] + sa * t1[0]) + sb * t2[0];
  s->vy[i] = (vn * n[1] + sa * t1[1]) + sb * t2[1];
  s->vz[i] = (vn * n[2] + sa * t1[2]) + sb * t2[2];
}

/* first-passage histogram bin: floor(log2 t), 0 for t <= 1 */
static int fpt_bin_of(uint32_t t) {
  int k = 0;
  while (t >= 2u) {
    t >>= 1;
    k++;
  }
  return k;
}

static int boundary(orc_sim *s, int64_t i, double x0, double y0, double z0) {
  double f;
  int kind = segment_exit(s, x0, y0, z0, s->x[i], s->y[i], s->z[i], &f);
  if (kind == X_NONE) return ORC_EV_NONE;
  int sp = s->sp[i], Q = s->q[i];
  double dx = s->x[i] - x0, dy = s->y[i] - y0, dz = s->z[i] - z0;
  double xc = x0 + f * dx, yc = y0 + f * dy, zc = z0 + f * dz;
  static const double ex[3] = {1, 0, 0}, ey[3] = {0, 1, 0}, pz[3] = {0, 0, 1}, mz[3] = {0, 0, -1};
  /* an ion lost to a wall or the aperture carries its kinetic energy out of
   * the plasma (power balance, Sec. II) and is an atom from now on */
  if (Q >= 1) {
    double v2 = (s->vx[i] * s->vx[i] + s->vy[i] * s->vy[i]) + s->vz[i] * s->vz[i];
    s->t.lost_ke[sp] += 0.5 * s->M[sp] * v2;
  }
  uint32_t born = s->birth[i];
  /* with exchange partners an atom remembers the step it became one, so
   * that a particle recycled in this step is not taken as a partner */
  s->birth[i] = s->p.cx_partner ? (uint32_t)s->step : ORC_BIRTH_NONE;
  if (kind == X_EXT_FLANGE && xc * xc + yc * yc <= s->rap2) {
    s->t.extracted[sp][Q]++;
    s->t.recycled++;
    /* radial size of the extracted beam (Sec. III.B) and first-passage time
     * from the ion's birth (Sec. III.D) */
    s->t.extracted_r[sp][Q] += sqrt(xc * xc + yc * yc);
    if (Q >= 1 && born != ORC_BIRTH_NONE) {
      uint32_t tp = (uint32_t)s->step - born;
      s->t.fpt_n[sp][Q]++;
      s->t.fpt_sum[sp][Q] += tp;
      s->t.fpt_hist[sp][fpt_bin_of(tp)]++;
    }
    s->q[i] = 0;
    s->x[i] = s->p.inlet_x;
    s->y[i] = s->p.inlet_y;
    s->z[i] = -s->hL + EPS_WALL;
    reemit(s, i, pz, ex, ey);
    return ORC_EV_EXTRACT;
  }
  s->t.wall[sp][Q]++;
  s->q[i] = 0;
  if (kind == X_EXT_FLANGE) {
    s->x[i] = xc; s->y[i] = yc; s->z[i] = s->hL - EPS_WALL;
    reemit(s, i, mz, ex, ey);
  } else if (kind == X_INJ_FLANGE) {
    s->x[i] = xc; s->y[i] = yc; s->z[i] = -s->hL + EPS_WALL;
    reemit(s, i, pz, ex, ey);
  } else {
    double rc = sqrt(xc * xc + yc * yc);
    double n[3] = {-xc / rc, -yc / rc, 0.0};
    double t1[3] = {yc / rc, -xc / rc, 0.0};
    double sc = (s->p.R0 - EPS_WALL) / rc;
    s->x[i] = xc * sc; s->y[i] = yc * sc; s->z[i] = zc;
    reemit(s, i, n, t1, pz);
  }
  return ORC_EV_WALL;
}

/* ------------------------------------------------------------------------ */
/* Electron-ion heating and diffusion (Sec. II): each step an ion's velocity */
/* gets the kick D (R + delta) |R| / |R + delta|.                            */
/*   D^2 = 3.715e-6 n_e lambda_ei Q^2 dt / (M^2 sqrt(T_e)), SI (n_e in m^-3, */
/*   dt in s, D in m/s), M in amu, T_e in eV.  The printed formula has Q     */
/*   inside the root; the text states a heating rate quadratic in Q, and     */
/*   with Q^2, SI units and R uniform in the cube [-1/2, 1/2]^3 (so that     */
/*   E|R|^2 = 1/4) the mean energy gain (1/8) M D^2 per step is the NRL      */
/*   electron-ion heating rate for T_i << T_e to within 2%: that reading.    */
/*   R: three uniforms of one draw of the heating stream, (w + 1/2) 2^-32 -  */
/*   1/2 each.                                                               */
/*   delta (x and y only): the 9-point stencil of n_e around the ion's cell  */
/*   in its z plane, times -R_L / n_e(cell), R_L = 2.38e-6 sqrt(T_e) /       */
/*   (|B| dX): the electron Larmor radius in units of the mesh step dX = hx, */
/*   |B| at the cell centre.  Cells beyond the mesh count as n_e = 0.        */
/* n_e and T_e are the ionisation's: with self-consistent electrons the     */
/* cell's ion charge density at the start of the step (no kick in a cell    */
/* without charge), else the zone's fixed background, which is uniform, so */
/* delta = 0; so does the isotropic-heating switch (the ablation of Sec.    */
/* IV).  Applied to ions that stay in the chamber, with their charge        */
/* before ionisation and charge exchange.                                    */
/* ------------------------------------------------------------------------ */
static double cell_ne(const orc_sim *s, int ix, int iy, int iz) {
  if (ix < 0 || ix >= s->p.nx || iy < 0 || iy >= s->p.ny) return 0.0;
  return s->nfac * (double)s->chg[(int64_t)ix + (int64_t)s->p.nx * ((int64_t)iy + (int64_t)s->p.ny * iz)];
}

static void heat_kick(orc_sim *s, int64_t i) {
  int sp = s->sp[i], Q = s->q[i];
  double x = s->x[i], y = s->y[i], z = s->z[i];
  int zone = (((x * x) * s->ia2 + (y * y) * s->ia2) + (z * z) * s->ic2) < 1.0;
  double Te = zone ? s->p.Te_in_eV : s->p.Te_out_eV;
  double ne, dlx = 0.0, dly = 0.0;
  if (s->p.self_ne) {
    uint32_t c = orc_cell_of(s, x, y, z);
    int ix = (int)(c % (uint32_t)s->p.nx);
    int iy = (int)((c / (uint32_t)s->p.nx) % (uint32_t)s->p.ny);
    int iz = (int)(c / ((uint32_t)s->p.nx * (uint32_t)s->p.ny));
    ne = cell_ne(s, ix, iy, iz);
    if (!(ne > 0.0)) return;
    double B[3];
    orc_field(s, -s->p.R0 + (ix + 0.5) * s->hx, -s->p.R0 + (iy + 0.5) * s->hy, -s->hL + (iz + 0.5) * s->hz, B);
    double bmag = sqrt((B[0] * B[0] + B[1] * B[1]) + B[2] * B[2]);
    if (bmag > 0.0 && !s->p.heat_isotropic) {
      double RL = (2.38e-6 * sqrt(Te)) / (bmag * s->hx);
      double gy = (-cell_ne(s, ix, iy + 1, iz) + cell_ne(s, ix, iy - 1, iz)) +
                  0.5 * (((-cell_ne(s, ix - 1, iy + 1, iz) - cell_ne(s, ix + 1, iy + 1, iz)) +
                          cell_ne(s, ix + 1, iy - 1, iz)) + cell_ne(s, ix - 1, iy - 1, iz));
      double gx = (-cell_ne(s, ix - 1, iy, iz) + cell_ne(s, ix + 1, iy, iz)) +
                  0.5 * (((-cell_ne(s, ix - 1, iy + 1, iz) + cell_ne(s, ix + 1, iy + 1, iz)) +
                          cell_ne(s, ix + 1, iy - 1, iz)) - cell_ne(s, ix - 1, iy - 1, iz));
      dlx = -(RL / ne) * gy;
      dly = -(RL / ne) * gx;
    }
  } else {
    ne = zone ? s->p.ne_in : s->p.ne_out;
    if (!(ne > 0.0)) return;
  }
  double A = s->p.sp[sp].mass_amu;
  double h = (((3.715e-6 * s->p.lnL_ei) * (double)(Q * Q)) * s->p.dt) / ((A * A) * sqrt(Te));
  double D = sqrt(ne * h);
  uint32_t W[4];
  draw(s, s->id[i], (uint32_t)s->step, S_HEAT, 0, W);
  const double two_m32 = 2.3283064365386962890625e-10; /* 2^-32 */
  double rx = ((double)W[0] + 0.5) * two_m32 - 0.5;
  double ry = ((double)W[1] + 0.5) * two_m32 - 0.5;
  double rz = ((double)W[2] + 0.5) * two_m32 - 0.5;
  double sx = rx + dlx, sy = ry + dly, sz = rz;
  double nr = sqrt((rx * rx + ry * ry) + rz * rz);
  double ns = sqrt((sx * sx + sy * sy) + sz * sz);
  if (!(ns > 0.0)) return;
  double f = (D * nr) / ns;
  s->vx[i] += f * sx;
  s->vy[i] += f * sy;
  s->vz[i] += f * sz;
}

/* ------------------------------------------------------------------------ */
/* Monte-Carlo collisions with electrons and neutrals (Sec. II).             */
/* One uniform u decides between the channels, taken in this order:         */
/*   ionisation Q -> Q+n, n = 1..4: P_n = 1 - exp(-n_e k_{Q,n} dt) with the  */
/*     zone's n_e and rates (channels that would pass z_max are closed);     */
/*   charge exchange: P_cx = n0 (Q sigma1) |v| dt (cross-section scaled      */
/*     linearly with Q, none for forbidden Q such as Ar2+);                  */
/*   elastic ion-atom scattering: P_el = n0 (Q sigma_el1) |v| dt;            */
/* u below the running sum of the channels up to one picks that channel.    */
/* Exchange is with a neutral drawn from a Maxwellian at T_n: Q = 1 takes    */
/* the neutral's velocity (resonant); Q >= 3 goes to Q-1 and the energy      */
/* release dE is shared equally in the centre-of-mass frame of the two       */
/* equal-mass partners.  Elastic scattering is isotropic in the centre-of-   */
/* mass frame of the ion and a neutral drawn the same way (its own stream):  */
/* the relative speed is kept and turned into a uniformly random direction. */
/* ------------------------------------------------------------------------ */
static void neutral_partner(const orc_sim *s, int64_t i, uint32_t stream, int sp, double w[3]) {
  uint32_t G[4], H[4];
  draw(s, s->id[i], (uint32_t)s->step, stream, 0, G);
  draw(s, s->id[i], (uint32_t)s->step, stream, 1, H);
  double n0, n1, n2, ndis;
  box_muller(orc_u53(G[0], G[1]), orc_u53(G[2], G[3]), &n0, &n1);
  box_muller(orc_u53(H[0], H[1]), orc_u53(H[2], H[3]), &n2, &ndis);
  double sg = s->sig_n[sp];
  w[0] = sg * n0; w[1] = sg * n1; w[2] = sg * n2;
}

/* v -> V_cm + (|g'|/2) n, n isotropic from call 2 of the stream; |g'|^2 = |v - w|^2 + extra */
static void cm_isotropic(orc_sim *s, int64_t i, uint32_t stream, const double w[3], double extra) {
  uint32_t I[4];
  draw(s, s->id[i], (uint32_t)s->step, stream, 2, I);
  double ct = 1.0 - 2.0 * orc_u53(I[0], I[1]);
  double st = sqrt(fmax(0.0, (1.0 - ct) * (1.0 + ct)));
  double ph = 2.0 * PI * orc_u53(I[2], I[3]);
  double nxv = st * cos(ph), nyv = st * sin(ph), nzv = ct;
  double gx = s->vx[i] - w[0], gy = s->vy[i] - w[1], gz = s->vz[i] - w[2];
  double g2 = (gx * gx + gy * gy) + gz * gz + extra;
  double hg = 0.5 * sqrt(g2);
  s->vx[i] = (s->vx[i] + w[0]) * 0.5 + hg * nxv;
  s->vy[i] = (s->vy[i] + w[1]) * 0.5 + hg * nyv;
  s->vz[i] = (s->vz[i] + w[2]) * 0.5 + hg * nzv;
}

static int mcc(orc_sim *s, int64_t i) {
  uint32_t W[4];
  draw(s, s->id[i], (uint32_t)s->step, S_STEP, 0, W);
  double u = orc_u53(W[0], W[1]);
  int sp = s->sp[i], Q = s->q[i];
  double x = s->x[i], y = s->y[i], z = s->z[i];
  int zone = (((x * x) * s->ia2 + (y * y) * s->ia2) + (z * z) * s->ic2) < 1.0;
  /* ionisation channels: the fixed background's 1 - exp(-n_e k dt), or
   * with self-consistent electrons n_e k dt, n_e = weight x (ion charge of
   * the cell at the start of the step) / cell volume */
  double cum[ORC_MAXN];
  double acc = 0.0;
  double ne = 0.0;
  if ((s->p.process_mask & ORC_P_IONIZE) && s->p.self_ne) ne = s->nfac * (double)s->chg[orc_cell_of(s, x, y, z)];
  for (int n = 1; n <= ORC_MAXN; n++) {
    double pn = 0.0;
    if (s->p.process_mask & ORC_P_IONIZE)
      pn = s->p.self_ne ? ne * s->kdt[sp][zone][n - 1][Q] : s->pion[sp][zone][n - 1][Q];
    acc = acc + pn;
    cum[n - 1] = acc;
  }
  double speed = sqrt((s->vx[i] * s->vx[i] + s->vy[i] * s->vy[i]) + s->vz[i] * s->vz[i]);
  /* neutral partners: the species' uniform n0, or with tracked neutrals
   * n0 = weight x (atoms of the species in the cell at the start of the
   * step) / cell volume */
  double ccx = s->ccx[sp], cel = s->cel[sp];
  if (s->p.self_n0 && (s->p.process_mask & (ORC_P_CX | ORC_P_ELASTIC))) {
    double n0c = s->nfac * (double)s->atoms[(int64_t)sp * s->ncell + orc_cell_of(s, x, y, z)];
    ccx = n0c * s->sdt_cx[sp];
    cel = n0c * s->sdt_el[sp];
  }
  double pc = 0.0;
  if ((s->p.process_mask & ORC_P_CX) && s->cxok[sp][Q]) pc = (ccx * (double)Q) * speed;
  double pe = 0.0;
  if (s->p.process_mask & ORC_P_ELASTIC) pe = (cel * (double)Q) * speed;
  double pt = acc + pc;
  double pall = pt + pe;
  if (pall > 0.1) s->t.anomalies++;
  for (int n = 1; n <= ORC_MAXN; n++) {
    if (u < cum[n - 1]) {
      s->t.ionized[sp][Q]++;
      s->t.ionized_n[sp][n - 1]++;
      if (Q == 0) s->birth[i] = (uint32_t)s->step; /* an ion is made from an atom */
      s->q[i] = (uint8_t)(Q + n);
      return ORC_EV_IONIZE;
    }
  }
  if (u < pt) {
    s->t.cx[sp][Q]++;
    if (s->p.cx_partner) {
      /* the electron comes from a tracked atom of the ion's collision cell,
       * chosen at the end of the step; a Q = 1 ion is now an atom and keeps
       * its velocity (resonant: no energy is released) */
      s->cxreq[(int64_t)sp * s->ncell + s->cell[i]]++;
      if (Q == 1) {
        s->q[i] = 0;
        s->birth[i] = (uint32_t)s->step;
        return ORC_EV_CX;
      }
    }
    /* resonant exchange hands the charge to the neutral: a new ion */
    if (Q == 1) s->birth[i] = (uint32_t)s->step;
    double w[3];
    neutral_partner(s, i, S_CX, sp, w);
    if (Q == 1) {
      s->vx[i] = w[0]; s->vy[i] = w[1]; s->vz[i] = w[2];
    } else {
      cm_isotropic(s, i, S_CX, w, s->decx[sp]);
      s->q[i] = (uint8_t)(Q - 1);
      s->t.cx_products[sp]++;
    }
    return ORC_EV_CX;
  }
  if (u < pall) {
    s->t.elastic[sp][Q]++;
    double w[3];
    neutral_partner(s, i, S_EL, sp, w);
    cm_isotropic(s, i, S_EL, w, 0.0);
    return ORC_EV_ELASTIC;
  }
  return ORC_EV_NONE;
}

/* ------------------------------------------------------------------------ */
/* Exchange partners (cx_partner): at the end of the step, in each collision */
/* cell, the exchanges of species s take tracked atoms of species s that     */
/* did not become atoms in this step, in the order of (key, id), key = word  */
/* 3 of the particle's STEP draw; each becomes a Q = 1 ion born in the step. */
/* Exchanges left without an atom are counted.                               */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint32_t group; /* species * ncell + cell */
  uint32_t key, id;
  int64_t i;
} partner_cand;

static int cmp_cand(const void *a, const void *b) {
  const partner_cand *x = a, *y = b;
  if (x->group != y->group) return x->group < y->group ? -1 : 1;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->id != y->id) return x->id < y->id ? -1 : 1;
  return 0;
}

static void match_partners(orc_sim *s) {
  int64_t nc = 0;
  for (int64_t i = 0; i < s->N; i++)
    if (s->q[i] == 0 && s->birth[i] != (uint32_t)s->step && s->cxreq[(int64_t)s->sp[i] * s->ncell + s->cell[i]])
      nc++;
  partner_cand *c = malloc(sizeof(partner_cand) * (size_t)(nc > 0 ? nc : 1));
  int64_t k = 0;
  for (int64_t i = 0; i < s->N; i++) {
    int64_t g = (int64_t)s->sp[i] * s->ncell + s->cell[i];
    if (s->q[i] == 0 && s->birth[i] != (uint32_t)s->step && s->cxreq[g]) {
      uint32_t W[4];
      draw(s, s->id[i], (uint32_t)s->step, S_STEP, 0, W);
      c[k].group = (uint32_t)g;
      c[k].key = W[3];
      c[k].id = s->id[i];
      c[k].i = i;
      k++;
    }
  }
  qsort(c, (size_t)nc, sizeof(partner_cand), cmp_cand);
  /* walk each group: its first cxreq[group] candidates become ions */
  for (int64_t a = 0; a < nc;) {
    int64_t b = a;
    while (b < nc && c[b].group == c[a].group) b++;
    uint32_t want = s->cxreq[c[a].group];
    for (int64_t t = a; t < b && (uint32_t)(t - a) < want; t++) {
      int64_t i = c[t].i;
      s->q[i] = 1;
      s->birth[i] = (uint32_t)s->step;
      s->ev[i] = ORC_EV_CX_PARTNER;
    }
    if ((int64_t)want > b - a) s->t.cx_unmatched[c[a].group / s->ncell] += (uint64_t)want - (uint64_t)(b - a);
    s->cxreq[c[a].group] = 0;
    a = b;
  }
  /* groups with requests and no candidate at all */
  for (int64_t g = 0; g < s->ncell * s->p.n_species; g++) {
    if (s->cxreq[g]) {
      s->t.cx_unmatched[g / s->ncell] += s->cxreq[g];
      s->cxreq[g] = 0;
    }
  }
  free(c);
}

/* ------------------------------------------------------------------------ */
/* Cloud-in-cell deposit on the (nx+1)(ny+1)(nz+1) node grid (the mesh of   */
/* Sec. II), accumulated over steps.                                         */
/* ------------------------------------------------------------------------ */
static void deposit(orc_sim *s) {
  uint32_t dm = s->p.deposit_mask;
  for (int64_t i = 0; i < s->N; i++) {
    int Q = s->q[i];
    int ion = Q >= 1;
    if (!((ion && (dm & 11u)) || (!ion && (dm & 4u)))) continue;
    /* ion pressure moment (Sec. III.B): with no mean flow, an ion of speed v
     * adds M v^2 / 3 = k T to n k T */
    double e = 0.0;
    if (ion && (dm & 8u)) {
      double v2 = (s->vx[i] * s->vx[i] + s->vy[i] * s->vy[i]) + s->vz[i] * s->vz[i];
      e = (s->M[s->sp[i]] * v2) / 3.0;
    }
    int ix, iy, iz;
    double tx, ty, tz;
    cic_axis(s->x[i], s->p.R0, s->idx, s->p.nx, &ix, &tx);
    cic_axis(s->y[i], s->p.R0, s->idy, s->p.ny, &iy, &ty);
    cic_axis(s->z[i], s->hL, s->idz, s->p.nz, &iz, &tz);
    double wx[2] = {1.0 - tx, tx}, wy[2] = {1.0 - ty, ty}, wz[2] = {1.0 - tz, tz};
    for (int dz = 0; dz < 2; dz++)
      for (int dy = 0; dy < 2; dy++)
        for (int dx = 0; dx < 2; dx++) {
          int64_t node = (int64_t)(ix + dx) + (int64_t)s->nx1 * ((iy + dy) + (int64_t)s->ny1 * (iz + dz));
          double w = (wx[dx] * wy[dy]) * wz[dz];
          if (ion) {
            if (dm & 1u) s->dens[ORC_F_ION_N][node] += w;
            if (dm & 2u) s->dens[ORC_F_ION_Q][node] += (double)Q * w;
            if (dm & 8u) s->dens[ORC_F_ION_P][node] += w * e;
          } else {
            s->dens[ORC_F_ATOM_N][node] += w;
          }
        }
  }
  s->dens_steps++;
}

/* ------------------------------------------------------------------------ */
/* One step: sort (every sort_every steps) -> Coulomb -> per particle push,  */
/* boundary, and (without a boundary event) heating kick and MCC ->         */
/* deposit.                                                                  */
/* ------------------------------------------------------------------------ */
int orc_step(orc_sim *s, int64_t n_steps) {
  uint32_t pm = s->p.process_mask;
  for (int64_t it = 0; it < n_steps; it++) {
    if (s->need_sort || s->step % s->p.sort_every == 0) {
      sort_particles(s);
      s->need_sort = 0;
    }
    if (pm & ORC_P_COULOMB) coulomb(s);
    if (s->p.self_ne) {
      /* electrons neutralise the ions cell by cell (Sec. II) */
      memset(s->chg, 0, (size_t)s->ncell * 4);
      for (int64_t i = 0; i < s->N; i++)
        if (s->q[i] >= 1) s->chg[orc_cell_of(s, s->x[i], s->y[i], s->z[i])] += s->q[i];
    }
    if (s->p.self_n0) {
      /* the tracked atoms are the neutral gas of the collisions */
      memset(s->atoms, 0, (size_t)s->ncell * ORC_MAXS * 4);
      for (int64_t i = 0; i < s->N; i++)
        if (s->q[i] == 0) s->atoms[(int64_t)s->sp[i] * s->ncell + orc_cell_of(s, s->x[i], s->y[i], s->z[i])]++;
    }
    for (int64_t i = 0; i < s->N; i++) {
      int ev = ORC_EV_NONE;
      if (pm & ORC_P_PUSH) {
        double x0 = s->x[i], y0 = s->y[i], z0 = s->z[i];
        double E[3];
        if (s->p.efield) gather_E(s, x0, y0, z0, E);
        boris(s, s->qmh[s->sp[i]][s->q[i]], s->p.efield ? E : NULL, &s->x[i], &s->y[i], &s->z[i],
              &s->vx[i], &s->vy[i], &s->vz[i]);
        ev = boundary(s, i, x0, y0, z0);
      }
      if (ev == ORC_EV_NONE && (pm & ORC_P_HEAT) && s->q[i] >= 1) heat_kick(s, i);
      if (ev == ORC_EV_NONE && (pm & (ORC_P_IONIZE | ORC_P_CX | ORC_P_ELASTIC))) ev = mcc(s, i);
      s->ev[i] = (uint8_t)ev;
      if (!(isfinite(s->x[i]) && isfinite(s->y[i]) && isfinite(s->z[i]) && isfinite(s->vx[i]) &&
            isfinite(s->vy[i]) && isfinite(s->vz[i])))
        s->t.anomalies++;
    }
    if (pm & ORC_P_DEPOSIT) deposit(s);
    if (s->p.cx_partner) match_partners(s);
    s->step++;
    s->t.steps++;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* State and accumulator access                                              */
/* ------------------------------------------------------------------------ */
int orc_set_state(orc_sim *s, int64_t step, const double *x, const double *y, const double *z,
                  const double *vx, const double *vy, const double *vz, const uint8_t *q,
                  const uint32_t *cell, const uint32_t *birth) {
  for (int64_t i = 0; i < s->N; i++) {
    if (q[i] > s->p.sp[s->sp[i]].z_max) return -1;
    if (cell && cell[i] >= (uint32_t)s->ncell) return -1;
    if (birth && q[i] >= 1 && birth[i] != ORC_BIRTH_NONE && (int64_t)birth[i] > step) return -1;
  }
  for (int64_t i = 0; i < s->N; i++) {
    s->x[i] = x[i]; s->y[i] = y[i]; s->z[i] = z[i];
    s->vx[i] = vx[i]; s->vy[i] = vy[i]; s->vz[i] = vz[i];
    s->q[i] = q[i];
    s->birth[i] = (birth && q[i] >= 1) ? birth[i] : ORC_BIRTH_NONE;
    s->ev[i] = ORC_EV_NONE;
  }
  s->step = step;
  if (cell) {
    memcpy(s->cell, cell, (size_t)s->N * 4);
    sort_from_cells(s);
    s->need_sort = 0;
  } else {
    s->need_sort = 1;
  }
  zero_accumulators(s);
  return 0;
}

int orc_get_state(const orc_sim *s, int64_t *step, double *x, double *y, double *z, double *vx,
                  double *vy, double *vz, uint8_t *q, uint8_t *species, uint32_t *cell, uint32_t *birth) {
  size_t n8 = (size_t)s->N * 8;
  if (step) *step = s->step;
  if (x) memcpy(x, s->x, n8);
  if (y) memcpy(y, s->y, n8);
  if (z) memcpy(z, s->z, n8);
  if (vx) memcpy(vx, s->vx, n8);
  if (vy) memcpy(vy, s->vy, n8);
  if (vz) memcpy(vz, s->vz, n8);
  if (q) memcpy(q, s->q, (size_t)s->N);
  if (species) memcpy(species, s->sp, (size_t)s->N);
  if (cell) memcpy(cell, s->cell, (size_t)s->N * 4);
  if (birth) memcpy(birth, s->birth, (size_t)s->N * 4);
  return 0;
}

/* Give the particles explicit ids and species: lets a test step a subset of
 * a larger run (whole collision cells) with the draws the full run makes. */
int orc_set_ids(orc_sim *s, const uint32_t *ids, const uint8_t *species) {
  for (int64_t i = 0; i < s->N; i++)
    if (species[i] >= s->p.n_species) return -1;
  for (int64_t i = 0; i < s->N; i++) {
    s->id[i] = ids[i];
    s->sp[i] = species[i];
  }
  return 0;
}

/* Philox4x32-10 of counters (ctr0 + i, c1, c2, c3), i < n, into out[4n] */
void orc_philox_fill(uint64_t seed, uint32_t ctr0, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
                     uint32_t *out) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int64_t i = 0; i < n; i++) {
    uint32_t ctr[4] = {ctr0 + (uint32_t)i, c1, c2, c3};
    orc_philox4x32_10(ctr, key, out + 4 * i);
  }
}

int orc_get_tallies(const orc_sim *s, orc_tallies *t) {
  *t = s->t;
  return 0;
}

int orc_get_density(const orc_sim *s, int field, double *out, int64_t *steps) {
  if (field < 0 || field >= ORC_NFIELDS) return -1;
  memcpy(out, s->dens[field], (size_t)s->nnode * 8);
  if (steps) *steps = s->dens_steps;
  return 0;
}

int orc_get_events(const orc_sim *s, uint8_t *out) {
  memcpy(out, s->ev, (size_t)s->N);
  return 0;
}
