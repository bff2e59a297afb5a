/* Drives every code path of the CPU oracle on a small run, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (host code only): init,
 * sorts, Coulomb pools (pairs and triplets), push with an E grid and a
 * magnetic map, walls and the aperture, ionisation Q -> Q+n, charge
 * exchange, elastic scattering, the heating kick with self-consistent
 * electrons, the tracked-neutral density and exchange partners (second
 * pass), all four density
 * fields, state round trips and a second species.  Prints the tallies' totals; exits non-zero on an API error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ecr_oracle.h"

static void species(orc_species *sp, double mass, int zmax, double frac) {
  memset(sp, 0, sizeof(*sp));
  sp->mass_amu = mass;
  sp->z_max = zmax;
  sp->cx_forbidden_mask = 1u << 2;
  sp->fraction = frac;
  for (int q = 0; q < zmax; q++) {
    sp->k_in[q] = 1e-13 * pow(0.6, q);
    sp->k_out[q] = 0.1 * sp->k_in[q];
    for (int n = 0; n < ORC_MAXN - 1; n++) sp->k_multi_in[n][q] = sp->k_multi_out[n][q] = 0.1 * sp->k_in[q];
  }
  sp->sigma_cx1 = 5e-19;
  sp->sigma_el1 = 3e-19;
  sp->n0 = 2e19;
}

int main(void) {
  const int nx = 8, ny = 8, nz = 16;
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  double *ef = malloc(sizeof(double) * 3 * nn), *bf = malloc(sizeof(double) * 3 * nn);
  for (int64_t i = 0; i < 3 * nn; i++) {
    ef[i] = 500.0 * sin(0.37 * (double)i);
    bf[i] = (i >= 2 * nn ? 0.5 : 0.0) + 0.02 * cos(0.11 * (double)i);
  }
  orc_params p;
  memset(&p, 0, sizeof(p));
  p.seed = 12345;
  p.n = 3001;
  p.dt = 5e-9;
  p.sort_every = 7;
  p.process_mask = ORC_P_PUSH | ORC_P_IONIZE | ORC_P_CX | ORC_P_COULOMB | ORC_P_DEPOSIT | ORC_P_HEAT | ORC_P_ELASTIC;
  p.deposit_mask = 15;
  p.nx = nx; p.ny = ny; p.nz = nz;
  p.R0 = 0.035; p.L = 0.3; p.r_ap = 0.01; p.inlet_x = 0.0175; p.inlet_y = 0.0;
  p.B0 = 0.5; p.mirror_k = 3.0; p.BH = 1.0;
  p.zone_a = 0.03; p.zone_c = 0.12; p.ne_in = 1e19; p.ne_out = 1e17;
  p.Ti0_eV = 30.0; p.T_wall_eV = 0.025; p.T_n_eV = 0.025; p.dE_cx_eV = 10.0; p.lnL = 10.0; p.weight = 4e11;
  p.efield = ef;
  p.n_species = 2;
  species(&p.sp[0], 39.948, 18, 0.6);
  species(&p.sp[1], 15.999, 8, 0.4);
  p.self_ne = 1;
  p.lnL_ei = 17.0; p.Te_in_eV = 1000.0; p.Te_out_eV = 5.0;
  for (int pass = 0; pass < 2; pass++) {
    p.bfield = pass ? bf : NULL;
    p.heat_isotropic = pass;
    p.self_n0 = pass;
    p.cx_partner = pass; /* exchange partners taken from the tracked atoms */
    /* the tracked atoms give about 1e18 m^-3 here: raise the cross-sections
     * so exchange and elastic scattering still occur, keeping n0 sigma */
    for (int k = 0; k < 2; k++) {
      p.sp[k].sigma_cx1 = pass ? 1e-17 : 5e-19;
      p.sp[k].sigma_el1 = pass ? 6e-18 : 3e-19;
      p.sp[k].n0 = pass ? 1e18 : 2e19;
    }
    orc_sim *s = NULL;
    if (orc_create(&p, &s) != 0) { fprintf(stderr, "create failed\n"); return 1; }
    if (orc_init_ions(s) != 0) return 1;
    if (orc_step(s, 40) != 0) return 1;
    /* state round trip, then more steps from the restored state */
    int64_t n = p.n, step;
    double *a = malloc(sizeof(double) * 6 * n);
    uint8_t *q = malloc(n), *spc = malloc(n);
    uint32_t *cell = malloc(4 * n), *birth = malloc(4 * n);
    orc_get_state(s, &step, a, a + n, a + 2 * n, a + 3 * n, a + 4 * n, a + 5 * n, q, spc, cell, birth);
    /* init makes ions only: in the tracked-neutral pass turn every third
     * particle into an atom, so that the cells hold atoms to collide with */
    if (pass)
      for (int64_t i = 0; i < n; i += 3) q[i] = 0;
    if (orc_set_state(s, step, a, a + n, a + 2 * n, a + 3 * n, a + 4 * n, a + 5 * n, q, cell, birth) != 0) return 1;
    if (orc_step(s, 23) != 0) return 1;
    orc_tallies t;
    orc_get_tallies(s, &t);
    double *d = malloc(sizeof(double) * nn);
    double dsum = 0.0;
    for (int f = 0; f < ORC_NFIELDS; f++) {
      int64_t st;
      if (orc_get_density(s, f, d, &st) != 0) return 1;
      for (int64_t i = 0; i < nn; i++) dsum += d[i];
    }
    uint64_t ion = 0, wall = 0, ext = 0, cx = 0, el = 0;
    for (int k = 0; k < ORC_MAXS; k++)
      for (int j = 0; j < ORC_MAXQ; j++) {
        ion += t.ionized[k][j]; wall += t.wall[k][j]; ext += t.extracted[k][j]; cx += t.cx[k][j]; el += t.elastic[k][j];
      }
    printf("pass %d: steps %lld ionized %llu wall %llu extracted %llu cx %llu elastic %llu density %.6g\n", pass,
           (long long)t.steps, (unsigned long long)ion, (unsigned long long)wall, (unsigned long long)ext,
           (unsigned long long)cx, (unsigned long long)el, dsum);
    free(a); free(q); free(spc); free(cell); free(birth); free(d);
    orc_destroy(s);
  }
  free(ef);
  free(bf);
  return 0;
}
