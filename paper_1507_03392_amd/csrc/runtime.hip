// runtime.hip -- host runtime behind the C ABI in ecrpic.h: parameter
// checks, derived tables, arena layout, the step loop, read-back, profiling.
//
// Device memory layout (one caller-owned arena, every region 256-B aligned):
//   SoA A and SoA B (double buffer for the sort): x y z vx vy vz (R each),
//   qs (u8), pid (u32); key, rank, cellid (u32 per slot); count and cell_off
//   (u32 per cell, +1); scan block sums; density grids (3 fields of FP64 per
//   node); accumulators (tallies, FP64 Coulomb moments, error bits); tables
//   (Boris factors, ionisation probabilities, Nanbu ln A); the first step of
//   a replayed graph (u32); the optional node E field; the optional per-slot
//   event log.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "ecr_kernels.hpp"
#include "ecrpic.h"

using namespace ecr;

namespace {

thread_local std::string g_thread_err;

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t soa[2][9];  // offsets of x y z vx vy vz qs pid birth in buffer A and B
  size_t key, rank, cellid, chunks, pairs, tris, moments, count, cell_off, bsum, dens, acc, tables, stepc, job, efield,
      bfield, evlog;
  size_t fchunks;  // chunk table of the fused step kernel
  size_t big;      // its oversized chunks: count, then indices
  size_t nbk;      // its ordering buckets per chunk (the per-slot ones reuse the sort's rank array)
  size_t scratch64;  // sort space of the pools that exceed the LDS (fused kernel)
  size_t chg[2];  // ion charge per cell, double-buffered (ECR_FLAG_SELF_NE)
  size_t cxreq;   // exchanges per species and collision cell (ECR_FLAG_CX_PARTNER)
  size_t cxchunk; // per Coulomb chunk: any of them in its cells
  size_t bden;    // |B| hx per cell (heating kick with self-consistent electrons)
  size_t total;
};

int64_t ncells(const ecr_params *p) { return (int64_t)p->nx * p->ny * p->nz; }
// FP64 moment slots of a run: the Coulomb kernels' and the fused step's
int64_t moment_slots(int64_t n) {
  const int64_t m = n > 0 ? n : 1;
  return std::max(coul_moment_slots(m), step_moment_slots(m));
}
int64_t nnodes(const ecr_params *p) { return (int64_t)(p->nx + 1) * (p->ny + 1) * (p->nz + 1); }
// the heating kick reads |B| hx per cell when n_e comes from the particles
bool needs_bden(const ecr_params *p) {
  return (p->process_mask & ECR_P_HEAT) && (p->flags & ECR_FLAG_SELF_NE);
}

Layout make_layout(const ecr_params *p) {
  Layout L{};
  const size_t N = (size_t)(p->n_particles > 0 ? p->n_particles : 1);
  const size_t rs = p->precision == ECR_FP32_MIXED ? 4 : 8;
  size_t o = 0;
  for (int b = 0; b < 2; ++b) {
    for (int k = 0; k < 6; ++k) {
      L.soa[b][k] = o;
      o = align_up(o + rs * N);
    }
    L.soa[b][6] = o;
    o = align_up(o + N);
    L.soa[b][7] = o;
    o = align_up(o + 4 * N);
    L.soa[b][8] = o;
    o = align_up(o + 4 * N);
  }
  L.key = o;
  o = align_up(o + 4 * N);
  L.rank = o;
  o = align_up(o + 4 * N);
  L.cellid = o;
  o = align_up(o + 4 * N);
  L.chunks = o;
  o = align_up(o + 4 * (size_t)(coul_nchunks((int64_t)N) + 2));
  L.fchunks = o;
  o = align_up(o + 4 * (size_t)(step_nchunks_max((int64_t)N) + 2));
  L.big = o;
  o = align_up(o + 4 * (size_t)(step_nchunks_max((int64_t)N) + 1));
  L.nbk = o;
  o = align_up(o + 4 * (size_t)(step_nchunks_max((int64_t)N) + 1));
  L.scratch64 = o;
  o = align_up(o + 8 * N);
  L.pairs = o;
  o = align_up(o + sizeof(CoulItem) * kCoulItems * (size_t)coul_nchunks((int64_t)N));
  L.tris = o;  // per-chunk (pairs, triplets) counts
  o = align_up(o + 8 * (size_t)coul_nchunks((int64_t)N));
  L.moments = o;
  o = align_up(o + 8 * 5 * (size_t)moment_slots((int64_t)N));
  L.count = o;
  o = align_up(o + 4 * (size_t)(ncells(p) + 1));
  L.cell_off = o;
  o = align_up(o + 4 * (size_t)(ncells(p) + 1));
  L.bsum = o;
  o = align_up(o + 4 * scan_blocksums_len(ncells(p)));
  L.dens = o;
  o = align_up(o + 8 * (size_t)ECR_N_FIELDS * (size_t)nnodes(p));
  L.acc = o;
  o = align_up(o + sizeof(DevAccum));
  L.tables = o;
  o = align_up(o + sizeof(Tables));
  L.stepc = o;
  o = align_up(o + 4);
  L.job = o;  // the batched step's two jobs (one per SoA buffer)
  o = align_up(o + 2 * sizeof(StepJob<double>));
  L.efield = o;
  if (p->efield_nodes) o = align_up(o + 8 * 3 * (size_t)nnodes(p));
  L.bfield = o;
  if (p->bfield_nodes) o = align_up(o + 8 * 3 * (size_t)nnodes(p));
  L.evlog = o;
  if (p->flags & ECR_FLAG_EVENTS) o = align_up(o + N);
  for (int b = 0; b < 2; ++b) {
    L.chg[b] = o;
    if (p->flags & (ECR_FLAG_SELF_NE | ECR_FLAG_SELF_N0))
      o = align_up(o + 4 * (size_t)ncells(p) * (size_t)(1 + p->n_species));
  }
  L.cxreq = o;
  if (p->flags & ECR_FLAG_CX_PARTNER) o = align_up(o + 4 * (size_t)ncells(p) * (size_t)p->n_species);
  L.cxchunk = o;
  if (p->flags & ECR_FLAG_CX_PARTNER) o = align_up(o + 4 * (size_t)(coul_nchunks((int64_t)N) + 1));
  L.bden = o;
  if (needs_bden(p)) o = align_up(o + 8 * (size_t)ncells(p));
  L.total = o + kAlign;  // slack so the arena base may be realigned
  return L;
}

// Nanbu's A(s): root of coth(A) - 1/A = exp(-s) by Newton's method on
// F(A) = ln(coth A - 1/A) + s, with coth A - 1/A evaluated without
// cancellation: for A < 2 from its odd power series (Bernoulli numbers
// through A^41), else directly.  Returns ln A.
double langevin_lib(double a, double *deriv) {
  // L(a) = coth a - 1/a; L'(a) = 1/a^2 - 1/sinh(a)^2
  double L, dL;
  if (a < 2.0) {
    // coth a - 1/a = sum_k 2^(2k) B_2k a^(2k-1) / (2k)!, convergent for
    // |a| < pi; the coefficients come from the Bernoulli numbers, computed once
    static double coef[24];
    static bool init = false;
    if (!init) {
      // B_2k via the recurrence sum_{j=0}^{m} C(m+1, j) B_j = 0
      double B[50] = {0};
      B[0] = 1.0;
      for (int m = 1; m < 50; ++m) {
        double s = 0.0, binom = 1.0;  // C(m+1, 0)
        for (int j = 0; j < m; ++j) {
          s += binom * B[j];
          binom = binom * (double)(m + 1 - j) / (double)(j + 1);
        }
        B[m] = -s / (double)(m + 1);
      }
      double fact = 1.0, pow2 = 1.0;
      for (int k = 1; k <= 24; ++k) {
        fact *= (double)(2 * k - 1) * (double)(2 * k);
        pow2 *= 4.0;
        coef[k - 1] = pow2 * B[2 * k] / fact;
      }
      init = true;
    }
    double a2 = a * a, p = a, sum = 0.0, dsum = 0.0;
    for (int k = 1; k <= 24; ++k) {
      sum += coef[k - 1] * p;                     // a^(2k-1)
      dsum += coef[k - 1] * (double)(2 * k - 1) * (p / a);
      p *= a2;
    }
    L = sum;
    dL = dsum;
  } else {
    L = 1.0 / tanh(a) - 1.0 / a;
    const double sh = sinh(a);
    dL = 1.0 / (a * a) - 1.0 / (sh * sh);
  }
  *deriv = dL;
  return L;
}

double nanbu_lnA_lib(double s) {
  // start from the asymptotes and polish with Newton on G(t) = ln L(e^t) + s, t = ln A
  double A = (s < 1.0) ? 1.0 / (-expm1(-s)) : 3.0 * exp(-s) + 1e-300;
  if (s >= 0.5 && s < 3.0) A = 1.0 / s;  // any start in range; Newton below is safeguarded
  double lo = 1e-6, hi = 2.0 / s + 4.0;
  double t = log(A);
  for (int it = 0; it < 200; ++it) {
    const double a = exp(t);
    double G, dG;
    if (s < 1.0) {
      // 1 - L(a) = 1/a - 2/expm1(2a), target 1 - exp(-s) = -expm1(-s); use the log of the complement
      const double e2 = expm1(2.0 * a);
      const double comp = 1.0 / a - 2.0 / e2;
      const double dcomp = -1.0 / (a * a) + 4.0 * (e2 + 1.0) / (e2 * e2);
      G = log(comp) - log(-expm1(-s));
      dG = dcomp / comp * a;
    } else {
      double dL;
      const double L = langevin_lib(a, &dL);
      G = log(L) + s;
      dG = dL / L * a;
    }
    if (G > 0.0) {  // s < 1: complement too large -> a too small; s >= 1: L too large -> a too large
      if (s < 1.0) lo = fmax(lo, a); else hi = fmin(hi, a);
    } else {
      if (s < 1.0) hi = fmin(hi, a); else lo = fmax(lo, a);
    }
    double tn = t - G / dG;
    if (!(tn > log(lo) && tn < log(hi))) tn = 0.5 * (log(lo) + log(hi));
    if (fabs(tn - t) <= 1e-17 * fmax(1.0, fabs(t))) {
      t = tn;
      break;
    }
    t = tn;
  }
  return t;
}

}  // namespace

struct ecr_run {
  ecr_params p;
  KParams kp;
  hipStream_t stream;
  char *base;
  Layout L;
  bool fp32;
  int64_t fcap;  // the fused step's chunk size (step_fcap)
  double weight;
  int64_t ncell, nnode;
  int64_t step;
  int64_t steps;
  int64_t dens_steps;
  bool need_sort;
  bool initialized;
  bool failed;
  int cur;  // which SoA buffer is current
  std::string err;
  // profiling: bit k set = launches of kernel kind k are bracketed by events
  uint32_t prof;
  int32_t prof_stride = 1;           // bracket one launch in prof_stride of each kind
  int64_t prof_seen[ECR_N_KERNELS];  // launches of each kind since ecr_profile
  double ms[ECR_N_KERNELS];
  int64_t launches[ECR_N_KERNELS];
  std::vector<hipEvent_t> free_events;
  struct Pending {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  // one sort period (sort_every steps, starting with its sort) captured as a
  // HIP graph, one per SoA buffer the period starts from
  hipGraphExec_t gexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [SoA buffer][charge grid]
  int chg_par = 0;  // charge grid of the current step (ECR_FLAG_SELF_NE)
  // a run of ecr_create_static: it lives in the library's static workspace
  // and handle of its device; ecr_destroy releases them instead of freeing
  bool is_static = false;
  bool live = false;
  uint64_t uid = 0;  // unique over the process: names the run in the batched graphs
};

namespace {

template <typename T>
T *at(ecr_run *r, size_t off) {
  return reinterpret_cast<T *>(r->base + off);
}

template <typename R>
Soa<R> soa(ecr_run *r, int b) {
  Soa<R> s;
  s.x = at<R>(r, r->L.soa[b][0]);
  s.y = at<R>(r, r->L.soa[b][1]);
  s.z = at<R>(r, r->L.soa[b][2]);
  s.vx = at<R>(r, r->L.soa[b][3]);
  s.vy = at<R>(r, r->L.soa[b][4]);
  s.vz = at<R>(r, r->L.soa[b][5]);
  s.qs = at<uint8_t>(r, r->L.soa[b][6]);
  s.pid = at<uint32_t>(r, r->L.soa[b][7]);
  s.birth = at<uint32_t>(r, r->L.soa[b][8]);
  return s;
}

ecr_status fail(ecr_run *r, ecr_status st, const std::string &msg) {
  if (r) r->err = msg; else g_thread_err = msg;
  return st;
}

ecr_status check_hip(ecr_run *r, hipError_t e, const char *what) {
  if (e == hipSuccess) return ECR_OK;
  r->failed = true;
  return fail(r, ECR_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

std::string validate(const ecr_params *p) {
  if (!p) return "params is NULL";
  if (p->abi_version != ECR_ABI_VERSION) return "abi_version mismatch";
  if (p->precision != ECR_FP64 && p->precision != ECR_FP32_MIXED) return "precision must be ECR_FP64 or ECR_FP32_MIXED";
  if (p->n_particles < 0 || p->n_particles > 0x7fffffffLL) return "n_particles out of range";
  if (!(p->dt_s > 0.0) || !isfinite(p->dt_s)) return "dt_s must be positive";
  if (p->sort_every < 1) return "sort_every must be >= 1";
  if (p->deposit_mask >= (1u << ECR_N_FIELDS)) return "deposit_mask has unknown bits";
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return "mesh dimensions must be >= 1";
  if ((int64_t)p->nx * p->ny * p->nz >= (1LL << 31) - 1) return "mesh too large";
  if ((int64_t)p->nx * p->ny * p->nz >= (1LL << 30)) return "mesh too large for 64-bit pairing keys";
  if (nnodes(p) >= (1LL << 31)) return "mesh has too many nodes";
  if (p->n_species < 1 || p->n_species > ECR_MAX_SPECIES) return "n_species must be 1..4";
  if (!(p->R0_m > 0.0) || !(p->L_m > 0.0)) return "R0_m and L_m must be positive";
  if (!(p->zone_a_m > 0.0) || !(p->zone_c_m > 0.0)) return "zone semi-axes must be positive";
  if (p->r_ap_m < 0.0) return "r_ap_m must be >= 0";
  if (p->inlet_x_m * p->inlet_x_m + p->inlet_y_m * p->inlet_y_m >= p->R0_m * p->R0_m) return "gas inlet outside the chamber";
  if (p->weight < 0.0 || p->lnL_ii < 0.0 || p->Ti0_eV < 0.0 || p->T_wall_eV < 0.0 || p->T_n_eV < 0.0)
    return "negative weight, Coulomb logarithm or temperature";
  if (p->ne_in_m3 < 0.0 || p->ne_out_m3 < 0.0) return "negative electron density";
  if (p->process_mask >= 128u) return "process_mask has unknown bits";
  if (p->flags >= 64u) return "flags has unknown bits";
  if ((p->flags & ECR_FLAG_CX_PARTNER) && !(p->flags & ECR_FLAG_SELF_N0))
    return "ECR_FLAG_CX_PARTNER needs ECR_FLAG_SELF_N0 (the partners are the tracked atoms)";
  if ((p->flags & ECR_FLAG_SELF_N0) && (int64_t)ncells(p) * (1 + p->n_species) >= (1LL << 32) - 1)
    return "mesh too large for the per-species atom grids";
  if ((p->process_mask & ECR_P_HEAT) &&
      !(p->Te_in_eV > 0.0 && p->Te_out_eV > 0.0 && isfinite(p->Te_in_eV) && isfinite(p->Te_out_eV)))
    return "the heating kick needs positive electron temperatures";
  if ((p->process_mask & ECR_P_HEAT) && !(p->lnL_ei >= 0.0)) return "negative electron-ion Coulomb logarithm";
  double fsum = 0.0;
  for (int s = 0; s < p->n_species; ++s) {
    const ecr_species &sp = p->species[s];
    if (!(sp.mass_amu > 0.0)) return "species mass must be positive";
    if (sp.z_max < 0 || sp.z_max >= ECR_MAX_Q) return "z_max must be 0..31";
    if (sp.fraction < 0.0) return "species fraction must be >= 0";
    if (sp.sigma_cx1_m2 < 0.0 || sp.n0_m3 < 0.0 || sp.sigma_el1_m2 < 0.0)
      return "negative cross-section or neutral density";
    for (int q = 0; q < ECR_MAX_Q; ++q) {
      if (sp.k_ion_in_m3s[q] < 0.0 || sp.k_ion_out_m3s[q] < 0.0) return "negative ionisation rate";
      for (int n = 0; n < ECR_MAX_NION - 1; ++n)
        if (sp.k_ion_multi_in_m3s[n][q] < 0.0 || sp.k_ion_multi_out_m3s[n][q] < 0.0) return "negative ionisation rate";
    }
    fsum += sp.fraction;
  }
  (void)fsum;
  return "";
}

// derived constants and tables, computed on the host in binary64
void derive(const ecr_params *p, KParams &K, Tables &T, double &weight) {
  memset(&K, 0, sizeof(K));
  memset(&T, 0, sizeof(T));
  const double dt = p->dt_s;
  K.R0 = p->R0_m;
  K.hL = 0.5 * p->L_m;
  K.R0sq = p->R0_m * p->R0_m;
  K.rap2 = p->r_ap_m * p->r_ap_m;
  K.inlet_x = p->inlet_x_m;
  K.inlet_y = p->inlet_y_m;
  K.idx = (double)p->nx / (2.0 * p->R0_m);
  K.idy = (double)p->ny / (2.0 * p->R0_m);
  K.idz = (double)p->nz / p->L_m;
  K.zone_a = p->zone_a_m;
  K.zone_c = p->zone_c_m;
  K.ia2 = 1.0 / (p->zone_a_m * p->zone_a_m);
  K.ic2 = 1.0 / (p->zone_c_m * p->zone_c_m);
  K.B0 = p->B0_T;
  const double L2 = p->L_m * p->L_m, R02 = p->R0_m * p->R0_m;
  K.c1 = ((4.0 * p->mirror_k) * p->B0_T) / L2;
  K.c2 = (2.0 * p->BH_T) / R02;
  K.c3 = p->BH_T / R02;
  K.c4 = ((2.0 * p->mirror_k) * p->B0_T) / L2;
  K.dt = dt;
  const double vzone = (4.0 / 3.0) * kPi * (p->zone_a_m * p->zone_a_m) * p->zone_c_m;
  weight = p->weight > 0.0 ? p->weight
                           : (p->n_particles > 0 ? p->ne_in_m3 * vzone / (double)p->n_particles : 0.0);
  const double vcell = ((2.0 * p->R0_m / p->nx) * (2.0 * p->R0_m / p->ny)) * (p->L_m / p->nz);
  K.nfac = weight / vcell;
  K.Cs = p->lnL_ii * (kE * kE) * (kE * kE) / (4.0 * kPi * kEps0 * kEps0);
  K.nion = 1;
  K.hx = 2.0 * p->R0_m / p->nx;
  K.hy = 2.0 * p->R0_m / p->ny;
  K.hz = p->L_m / p->nz;
  // heating kick: D^2 = n_e x (3.715e-6 lnL_ei Q^2 dt) / (M_amu^2 sqrt(T_e)), M in amu
  // and T_e in eV (Sec. II, the kick's charge law read as Q^2)
  const bool heat = (p->process_mask & ECR_P_HEAT) != 0;
  const double te[2] = {p->Te_out_eV, p->Te_in_eV};
  K.ne_zone[0] = p->ne_out_m3;
  K.ne_zone[1] = p->ne_in_m3;
  for (int z = 0; z < 2; ++z) K.rl_zone[z] = heat ? 2.38e-6 * sqrt(te[z]) : 0.0;
  int64_t end = 0;
  for (int s = 0; s < p->n_species; ++s) {
    const ecr_species &sp = p->species[s];
    const double M = sp.mass_amu * kAmu;
    K.mass[s] = M;
    K.sig_w[s] = sqrt(p->T_wall_eV * kE / M);
    K.sig_n[s] = sqrt(p->T_n_eV * kE / M);
    K.sig_i[s] = sqrt(p->Ti0_eV * kE / M);
    K.decx[s] = 4.0 * p->dE_cx_eV * kE / M;
    K.ccx[s] = (sp.n0_m3 * sp.sigma_cx1_m2) * dt;
    K.cel[s] = (sp.n0_m3 * sp.sigma_el1_m2) * dt;
    K.sdt_cx[s] = sp.sigma_cx1_m2 * dt;
    K.sdt_el[s] = sp.sigma_el1_m2 * dt;
    uint32_t ok = 0;
    for (int q = 0; q < kMaxQ; ++q) {
      T.qmh[s][q] = ((double)q * kE / M) * (dt * 0.5);
      if (q < sp.z_max) {
        T.pion[s][1][q] = -expm1(-(p->ne_in_m3 * sp.k_ion_in_m3s[q]) * dt);
        T.pion[s][0][q] = -expm1(-(p->ne_out_m3 * sp.k_ion_out_m3s[q]) * dt);
        T.kdt[s][1][q] = sp.k_ion_in_m3s[q] * dt;
        T.kdt[s][0][q] = sp.k_ion_out_m3s[q] * dt;
      }
      // Q -> Q+n, n >= 2, while Q + n stays within z_max
      for (int n = 2; n <= kMaxN; ++n) {
        if (q + n > sp.z_max) continue;
        const double kin = sp.k_ion_multi_in_m3s[n - 2][q], kout = sp.k_ion_multi_out_m3s[n - 2][q];
        T.pmul[s][1][n - 2][q] = -expm1(-(p->ne_in_m3 * kin) * dt);
        T.pmul[s][0][n - 2][q] = -expm1(-(p->ne_out_m3 * kout) * dt);
        T.kmul[s][1][n - 2][q] = kin * dt;
        T.kmul[s][0][n - 2][q] = kout * dt;
        if (kin > 0.0 || kout > 0.0) K.nion = K.nion > n ? K.nion : n;
      }
      if (q >= 1 && q <= sp.z_max && !((sp.cx_forbidden_mask >> q) & 1u)) ok |= 1u << q;
      if (heat)
        for (int z = 0; z < 2; ++z)
          T.dheat[s][z][q] = (((3.715e-6 * p->lnL_ei) * (double)(q * q)) * dt) /
                             ((sp.mass_amu * sp.mass_amu) * sqrt(te[z]));
    }
    K.cxok[s] = ok;
    if (s == p->n_species - 1) end = p->n_particles;
    else end += (int64_t)floor(sp.fraction * (double)p->n_particles + 0.5);
    if (end > p->n_particles) end = p->n_particles;
    K.sp_end[s] = end;
  }
  for (int a = 0; a < p->n_species; ++a)
    for (int b = 0; b < p->n_species; ++b) {
      const double ma = K.mass[a], mb = K.mass[b];
      K.mu[a][b] = (ma * mb) / (ma + mb);
      K.mra[a][b] = K.mu[a][b] / ma;
      K.mrb[a][b] = K.mu[a][b] / mb;
    }
  for (int e = kAeLo; e <= kAeHi; ++e)
    for (int j = 0; j < kAK; ++j) T.lnA[(e - kAeLo) * kAK + j] = nanbu_lnA_lib(ldexp(1.0 + (double)j / kAK, e));
  T.lnA[kANodes - 1] = nanbu_lnA_lib(kSHi);
  K.n = p->n_particles;
  K.ncell = (uint32_t)ncells(p);
  K.nnode = nnodes(p);
  K.nx = p->nx;
  K.ny = p->ny;
  K.nz = p->nz;
  K.nx1 = p->nx + 1;
  K.ny1 = p->ny + 1;
  K.nspecies = p->n_species;
  K.seed_lo = (uint32_t)p->seed;
  K.seed_hi = (uint32_t)(p->seed >> 32);
  K.pmask = p->process_mask;
  K.dmask = p->deposit_mask;
  K.flags = p->flags;
}

// largest per-step collision probability, with charge exchange bounded at a
// speed cap of 10 sqrt(2 T e / M), T = max(Ti0, T_wall, 10 eV)
double max_probability(const ecr_params *p, const KParams &K, const Tables &T) {
  double worst = 0.0;
  for (int s = 0; s < p->n_species; ++s) {
    const double Tm = fmax(fmax(p->Ti0_eV, p->T_wall_eV), 10.0);
    const double vcap = 10.0 * sqrt(2.0 * Tm * kE / K.mass[s]);
    for (int q = 0; q <= p->species[s].z_max; ++q)
      for (int z = 0; z < 2; ++z) {
        double pi = 0.0;
        if (p->process_mask & ECR_P_IONIZE) {
          pi = T.pion[s][z][q];
          for (int n = 0; n < kMaxN - 1; ++n) pi += T.pmul[s][z][n][q];
        }
        double pc = ((p->process_mask & ECR_P_CX) && ((K.cxok[s] >> q) & 1u)) ? K.ccx[s] * q * vcap : 0.0;
        double pe = (p->process_mask & ECR_P_ELASTIC) ? K.cel[s] * q * vcap : 0.0;
        worst = fmax(worst, pi + pc + pe);
      }
  }
  return worst;
}

// ---- profiling ----
hipEvent_t get_event(ecr_run *r) {
  if (!r->free_events.empty()) {
    hipEvent_t e = r->free_events.back();
    r->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void harvest(ecr_run *r) {
  if (r->pending.empty()) return;
  (void)hipStreamSynchronize(r->stream);
  for (auto &pd : r->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pd.a, pd.b) == hipSuccess) {
      r->ms[pd.kind] += ms;
      r->launches[pd.kind] += 1;
    }
    r->free_events.push_back(pd.a);
    r->free_events.push_back(pd.b);
  }
  r->pending.clear();
}

struct ProfScope {
  ecr_run *r;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(ecr_run *r_, int k) : r(r_), kind(k) {
    if ((r->prof >> kind) & 1u && r->prof_seen[kind]++ % r->prof_stride == 0) {
      a = get_event(r);
      b = get_event(r);
      (void)hipEventRecord(a, r->stream);
    }
  }
  ~ProfScope() {
    if (a) {
      (void)hipEventRecord(b, r->stream);
      r->pending.push_back({kind, a, b});
      if (r->pending.size() >= 4096) harvest(r);
    }
  }
};

// the whole step in one kernel: the default, for the analytic magnetic
// field without an electric field grid; ECR_FLAG_SPLIT (per-kernel timing)
// and the field grids run the step as separate kernels
bool fused(const ecr_run *r) {
  return !(r->p.flags & ECR_FLAG_SPLIT) && !r->p.efield_nodes && !r->kp.bmap;
}

template <typename R>
void do_sort(ecr_run *r, const uint32_t *given) {
  ProfScope ps(r, ECR_K_SORT);
  const int a = r->cur, b = 1 - r->cur;
  launch_sort<R>(r->kp, soa<R>(r, a), soa<R>(r, b), given, at<uint32_t>(r, r->L.key), at<uint32_t>(r, r->L.rank),
                 at<uint32_t>(r, r->L.count), at<uint32_t>(r, r->L.cell_off), at<uint32_t>(r, r->L.bsum),
                 at<uint32_t>(r, r->L.cellid), r->ncell, r->stream);
  if (r->kp.n > 0) {
    launch_coul_chunks(at<uint32_t>(r, r->L.cellid), at<uint32_t>(r, r->L.cell_off), r->kp.n,
                       at<uint32_t>(r, r->L.chunks), kCoulCap, r->stream);
    if (fused(r)) {
      launch_coul_chunks(at<uint32_t>(r, r->L.cellid), at<uint32_t>(r, r->L.cell_off), r->kp.n,
                         at<uint32_t>(r, r->L.fchunks), r->fcap, r->stream);
      // the per-slot buckets go into the sort's rank array, free until the next sort
      launch_step_prep(at<uint32_t>(r, r->L.cellid), at<uint32_t>(r, r->L.fchunks), r->kp.n, r->fcap,
                       at<uint32_t>(r, r->L.big), at<uint32_t>(r, r->L.rank), at<uint32_t>(r, r->L.nbk), r->stream);
    }
  }
  r->cur = b;
}

template <typename R>
void step_tail(ecr_run *r, StepArg stepw, bool grids);

// one step; sa gives the step number the kernels use (the host's counter in
// eager launches, a device word plus an offset inside a captured graph)
template <typename R>
void do_step(ecr_run *r, StepArg stepw) {
  const uint32_t pm = r->p.process_mask;
  if (r->need_sort || r->step % r->p.sort_every == 0) {
    do_sort<R>(r, nullptr);
    r->need_sort = false;
  }
  DevAccum *acc = at<DevAccum>(r, r->L.acc);
  const Tables *T = at<Tables>(r, r->L.tables);
  const bool grids = (r->p.flags & (ECR_FLAG_SELF_NE | ECR_FLAG_SELF_N0)) != 0;
  uint32_t *chg_cur = grids ? at<uint32_t>(r, r->L.chg[r->chg_par]) : nullptr;
  uint32_t *chg_next = grids ? at<uint32_t>(r, r->L.chg[1 - r->chg_par]) : nullptr;
  const int64_t chg_words = r->ncell * (1 + r->p.n_species);
  if (fused(r)) {
    if (grids) launch_fill_u32(chg_next, 0u, chg_words, r->stream);
    {
      ProfScope ps(r, ECR_K_STEP);
      launch_step<R>(r->kp, T, soa<R>(r, r->cur), at<uint32_t>(r, r->L.cellid), at<uint32_t>(r, r->L.fchunks),
                     at<uint32_t>(r, r->L.big), at<uint32_t>(r, r->L.rank), at<uint32_t>(r, r->L.nbk),
                     (r->p.flags & ECR_FLAG_EVENTS) ? at<uint8_t>(r, r->L.evlog) : nullptr,
                     acc, (pm & ECR_P_DEPOSIT) ? at<double>(r, r->L.dens) : nullptr, at<double>(r, r->L.moments),
                     at<uint64_t>(r, r->L.scratch64), stepw, chg_cur, chg_next, r->fcap, r->stream);
    }
    step_tail<R>(r, stepw, grids);
    return;
  }
  // the ordering kernel clears the next step's grids when it runs
  const bool fold = grids && (pm & ECR_P_COULOMB) && r->kp.n > 1;
  if (pm & ECR_P_COULOMB) {
    {
      ProfScope ps(r, ECR_K_COULOMB);
      launch_coul_order<R>(r->kp, soa<R>(r, r->cur), at<uint32_t>(r, r->L.cellid), at<uint32_t>(r, r->L.chunks), acc,
                           at<CoulItem>(r, r->L.pairs), at<uint2>(r, r->L.tris), stepw, fold ? chg_next : nullptr,
                           fold ? chg_words : 0, r->stream);
    }
    ProfScope ps(r, ECR_K_COUL_PAIRS);
    launch_coul_pairs<R>(r->kp, T, soa<R>(r, r->cur), at<uint32_t>(r, r->L.chunks), at<CoulItem>(r, r->L.pairs),
                         at<uint2>(r, r->L.tris), at<double>(r, r->L.moments), stepw, r->stream);
  }
  const bool dep = (pm & ECR_P_DEPOSIT) != 0;
  const bool split = (r->p.flags & ECR_FLAG_SPLIT) != 0;
  if (grids && !fold) launch_fill_u32(chg_next, 0u, chg_words, r->stream);
  {
    ProfScope ps(r, (dep && !split) ? ECR_K_FUSED : ECR_K_PUSH);
    launch_push<R>(r->kp, T, soa<R>(r, r->cur), r->p.efield_nodes ? at<double>(r, r->L.efield) : nullptr,
                   (r->p.flags & ECR_FLAG_EVENTS) ? at<uint8_t>(r, r->L.evlog) : nullptr, acc,
                   (dep && !split) ? at<double>(r, r->L.dens) : nullptr, stepw, chg_cur, chg_next, r->stream);
  }
  if (dep && split) {
    ProfScope ps(r, ECR_K_DEPOSIT);
    launch_deposit<R>(r->kp, soa<R>(r, r->cur), at<double>(r, r->L.dens), r->stream);
  }
  step_tail<R>(r, stepw, grids);
}

// after the push: the pressure moment, the exchange partners, the counters
template <typename R>
void step_tail(ecr_run *r, StepArg stepw, bool grids) {
  DevAccum *acc = at<DevAccum>(r, r->L.acc);
  const bool dep = (r->p.process_mask & ECR_P_DEPOSIT) != 0;
  if (grids) r->chg_par = 1 - r->chg_par;
  if (dep && (r->p.deposit_mask & (1u << ECR_F_ION_P))) {
    ProfScope ps(r, ECR_K_DEPOSIT);
    launch_deposit_pressure<R>(r->kp, soa<R>(r, r->cur), at<double>(r, r->L.dens), r->stream);
  }
  if (r->kp.cxreq) {
    ProfScope ps(r, ECR_K_PARTNER);
    // exchange partners, after the deposit; chg_par now names the grids of
    // the next step, which the partners' new charges update
    launch_cx_partner<R>(r->kp, soa<R>(r, r->cur), at<uint32_t>(r, r->L.chunks),
                         at<uint32_t>(r, r->L.chg[r->chg_par]),
                         (r->p.flags & ECR_FLAG_EVENTS) ? at<uint8_t>(r, r->L.evlog) : nullptr, acc, stepw,
                         r->stream);
  }
  if (dep) r->dens_steps++;
  r->step++;
  r->steps++;
}

// ---------------------------------------------------------------------------
// Batched stepping: the default steps of several runs on one stream in one
// launch per step (k_step_batch), each run's arguments read from its job in
// its own arena.  The jobs of both SoA buffers are written once, at init.
// ---------------------------------------------------------------------------
template <typename R>
StepJob<R> make_job(ecr_run *r, int b) {
  StepJob<R> J;
  J.P = r->kp;
  J.T = at<Tables>(r, r->L.tables);
  J.S = soa<R>(r, b);
  J.cellid = at<uint32_t>(r, r->L.cellid);
  J.chunk_lo = at<uint32_t>(r, r->L.fchunks);
  J.big = at<uint32_t>(r, r->L.big);
  J.bkinfo = at<uint32_t>(r, r->L.rank);
  J.nbk = at<uint32_t>(r, r->L.nbk);
  J.evlog = (r->p.flags & ECR_FLAG_EVENTS) ? at<uint8_t>(r, r->L.evlog) : nullptr;
  J.acc = at<DevAccum>(r, r->L.acc);
  J.dens = at<double>(r, r->L.dens);
  J.moments = at<double>(r, r->L.moments);
  J.scratch64 = at<uint64_t>(r, r->L.scratch64);
  return J;
}

template <typename R>
void write_jobs(ecr_run *r) {
  for (int b = 0; b < 2; ++b) launch_set_job<R>(make_job<R>(r, b), at<StepJob<R>>(r, r->L.job) + b, r->stream);
}

// a run whose step the batched kernel can take: the default fused step
bool batchable(const ecr_run *r) {
  const bool grids = (r->p.flags & (ECR_FLAG_SELF_NE | ECR_FLAG_SELF_N0)) != 0;
  return fused(r) && !r->prof && step_batchable(r->kp, (r->p.process_mask & ECR_P_DEPOSIT) != 0, grids);
}

// one step of the batchable runs rs (all of precision R), step numbers sa:
// each run's sort when due, one launch per kMaxBatch runs, then each run's tail
template <typename R>
void batch_step(const std::vector<ecr_run *> &rs, const std::vector<StepArg> &sa, hipStream_t st) {
  for (ecr_run *r : rs)
    if (r->need_sort || r->step % r->p.sort_every == 0) {
      do_sort<R>(r, nullptr);
      r->need_sort = false;
    }
  for (size_t k0 = 0; k0 < rs.size(); k0 += kMaxBatch) {
    StepBatch<R> B{};
    B.n = (int)std::min(rs.size() - k0, (size_t)kMaxBatch);
    B.wg0[0] = 0;
    for (int j = 0; j < B.n; ++j) {
      ecr_run *r = rs[k0 + j];
      B.job[j] = at<StepJob<R>>(r, r->L.job) + r->cur;
      B.stepw[j] = sa[k0 + j].base;
      B.step[j] = sa[k0 + j].off;
      B.wg0[j + 1] = B.wg0[j] + step_batch_wgs(r->kp.n, r->fcap);
    }
    launch_step_batch<R>(B, st);
  }
  for (size_t k = 0; k < rs.size(); ++k) step_tail<R>(rs[k], sa[k], false);
}

// one step of every run of a batch; base: each run's step counter word in
// a captured graph (offset off), else the host's counters
void batch_step_all(const std::vector<ecr_run *> &runs, hipStream_t st, bool captured, uint32_t off) {
  std::vector<ecr_run *> bd, bf;
  std::vector<StepArg> sd, sf;
  for (ecr_run *r : runs) {
    const StepArg a = captured ? StepArg{at<uint32_t>(r, r->L.stepc), off} : StepArg{nullptr, (uint32_t)r->step};
    if (!batchable(r)) {
      if (r->fp32) do_step<float>(r, a);
      else do_step<double>(r, a);
    } else if (r->fp32) {
      bf.push_back(r);
      sf.push_back(a);
    } else {
      bd.push_back(r);
      sd.push_back(a);
    }
  }
  if (!bd.empty()) batch_step<double>(bd, sd, st);
  if (!bf.empty()) batch_step<float>(bf, sf, st);
}

// sort periods of a set of runs captured as one graph, keyed by the runs'
// ids and the buffers they start from; kept until one of the runs is
// destroyed (or the cache is full)
struct BatchGraph {
  hipStream_t stream;
  std::vector<uint64_t> key;
  hipGraphExec_t ge;
};
std::mutex g_bgraph_mu;
std::vector<BatchGraph> g_bgraphs;
constexpr size_t kMaxBatchGraphs = 16;
// the keys of periods stepped eagerly: a set of runs is captured the second
// time one of its periods comes up (a batch whose members change at every
// period would otherwise pay a capture per period)
std::vector<std::vector<uint64_t>> g_bseen;
constexpr size_t kMaxBatchSeen = 64;

std::vector<uint64_t> batch_key(const std::vector<ecr_run *> &runs) {
  std::vector<uint64_t> k;
  for (ecr_run *r : runs) k.push_back(r->uid << 2 | (uint64_t)r->cur << 1 | (uint64_t)r->chg_par);
  return k;
}

hipError_t capture_batch_period(const std::vector<ecr_run *> &runs, hipStream_t st, int64_t K, hipGraphExec_t *out) {
  struct Saved {
    int64_t step, steps, dens;
    int cur, par;
    bool need;
  };
  std::vector<Saved> sv;
  for (ecr_run *r : runs) sv.push_back({r->step, r->steps, r->dens_steps, r->cur, r->chg_par, r->need_sort});
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  for (int64_t i = 0; i < K; ++i) batch_step_all(runs, st, true, (uint32_t)i);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(st, &g);
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  for (size_t k = 0; k < runs.size(); ++k) {
    ecr_run *r = runs[k];
    r->step = sv[k].step;
    r->steps = sv[k].steps;
    r->dens_steps = sv[k].dens;
    r->cur = sv[k].cur;
    r->chg_par = sv[k].par;
    r->need_sort = sv[k].need;
  }
  return e;
}

// drop the batched graphs that hold run r (its stream synchronised first)
void forget_batch_graphs(const ecr_run *r) {
  std::lock_guard<std::mutex> lock(g_bgraph_mu);
  for (size_t i = 0; i < g_bgraphs.size();) {
    bool has = false;
    for (uint64_t k : g_bgraphs[i].key) has |= (k >> 2) == r->uid;
    if (has) {
      (void)hipStreamSynchronize(g_bgraphs[i].stream);
      (void)hipGraphExecDestroy(g_bgraphs[i].ge);
      g_bgraphs.erase(g_bgraphs.begin() + i);
    } else {
      ++i;
    }
  }
}

// ion charge and atoms per cell of the state just set (ECR_FLAG_SELF_NE,
// ECR_FLAG_SELF_N0)
void build_charge_grid(ecr_run *r) {
  if (!(r->p.flags & (ECR_FLAG_SELF_NE | ECR_FLAG_SELF_N0))) return;
  r->chg_par = 0;
  uint32_t *g = at<uint32_t>(r, r->L.chg[0]);
  launch_fill_u32(g, 0u, r->ncell * (1 + r->p.n_species), r->stream);
  if (r->fp32) launch_charge_grid<float>(r->kp, soa<float>(r, r->cur), g, r->stream);
  else launch_charge_grid<double>(r->kp, soa<double>(r, r->cur), g, r->stream);
}

void zero_accumulators(ecr_run *r) {
  launch_fill_f64(at<double>(r, r->L.dens), 0.0, (int64_t)ECR_N_FIELDS * r->nnode, r->stream);
  launch_fill_u32(at<uint32_t>(r, r->L.acc), 0u, (int64_t)(sizeof(DevAccum) / 4), r->stream);
  launch_fill_f64(at<double>(r, r->L.moments), 0.0, 5 * moment_slots(r->kp.n), r->stream);
  if (r->kp.cxreq) {
    launch_fill_u32(r->kp.cxreq, 0u, r->ncell * r->p.n_species, r->stream);
    launch_fill_u32(r->kp.cxchunk, 0u, coul_nchunks(r->kp.n) + 1, r->stream);
  }
  r->steps = 0;
  r->dens_steps = 0;
}

}  // namespace

namespace {
template <typename R>
ecr_status get_state_t(ecr_run *r, ecr_state_view *v) {
  const int64_t n = r->kp.n;
  std::vector<R> buf[6];
  std::vector<uint8_t> qs(n);
  std::vector<uint32_t> pid(n), cell(n), birth(n);
  hipError_t e = hipSuccess;
  for (int k = 0; k < 6 && e == hipSuccess; ++k) {
    buf[k].resize(n);
    e = hipMemcpyAsync(buf[k].data(), r->base + r->L.soa[r->cur][k], sizeof(R) * n, hipMemcpyDeviceToHost, r->stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(qs.data(), r->base + r->L.soa[r->cur][6], n, hipMemcpyDeviceToHost, r->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(pid.data(), r->base + r->L.soa[r->cur][7], 4 * n, hipMemcpyDeviceToHost, r->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(cell.data(), r->base + r->L.cellid, 4 * n, hipMemcpyDeviceToHost, r->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(birth.data(), r->base + r->L.soa[r->cur][8], 4 * n, hipMemcpyDeviceToHost, r->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
  if (e != hipSuccess) return check_hip(r, e, "get_state");
  double *dst[6] = {v->x, v->y, v->z, v->vx, v->vy, v->vz};
  for (int64_t j = 0; j < n; ++j) {
    const uint32_t i = pid[j];
    if (i >= (uint32_t)n) return fail(r, ECR_ESTATE, "corrupt particle ids");
    for (int k = 0; k < 6; ++k)
      if (dst[k]) dst[k][i] = (double)buf[k][j];
    if (v->q) v->q[i] = qs[j] & 31;
    if (v->species) v->species[i] = qs[j] >> 5;
    if (v->cell) v->cell[i] = cell[j];
    if (v->birth) v->birth[i] = birth[j];
  }
  v->step = r->step;
  return ECR_OK;
}

template <typename R>
ecr_status set_state_t(ecr_run *r, const ecr_state_view *v) {
  const int64_t n = r->kp.n;
  std::vector<R> buf[6];
  const double *src[6] = {v->x, v->y, v->z, v->vx, v->vy, v->vz};
  std::vector<uint8_t> qs(n);
  std::vector<uint32_t> pid(n), birth(n);
  for (int64_t i = 0; i < n; ++i) {
    int s = r->kp.nspecies - 1;
    for (int k = r->kp.nspecies - 1; k >= 0; --k)
      if (i < r->kp.sp_end[k]) s = k;
    if (v->q[i] > r->p.species[s].z_max) return fail(r, ECR_EINVAL, "charge state above z_max");
    if (v->cell && v->cell[i] >= (uint32_t)r->ncell) return fail(r, ECR_EINVAL, "cell out of range");
    qs[i] = (uint8_t)(v->q[i] | (s << 5));
    pid[i] = (uint32_t)i;
    birth[i] = v->birth && v->q[i] >= 1 ? v->birth[i] : ECR_BIRTH_NONE;
    if (birth[i] != ECR_BIRTH_NONE && (int64_t)birth[i] > v->step)
      return fail(r, ECR_EINVAL, "birth step after the state's step");
  }
  for (int k = 0; k < 6; ++k) {
    buf[k].resize(n);
    for (int64_t i = 0; i < n; ++i) buf[k][i] = (R)src[k][i];
  }
  r->cur = 0;
  hipError_t e = hipSuccess;
  for (int k = 0; k < 6 && e == hipSuccess; ++k)
    e = hipMemcpyAsync(r->base + r->L.soa[0][k], buf[k].data(), sizeof(R) * n, hipMemcpyHostToDevice, r->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(r->base + r->L.soa[0][6], qs.data(), n, hipMemcpyHostToDevice, r->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(r->base + r->L.soa[0][7], pid.data(), 4 * n, hipMemcpyHostToDevice, r->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(r->base + r->L.soa[0][8], birth.data(), 4 * n, hipMemcpyHostToDevice, r->stream);
  // given collision cells (by id) are staged in buffer B's id array: the
  // sort's count pass reads them before its scatter overwrites buffer B
  if (e == hipSuccess && v->cell)
    e = hipMemcpyAsync(r->base + r->L.soa[1][7], v->cell, 4 * n, hipMemcpyHostToDevice, r->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
  if (e != hipSuccess) return check_hip(r, e, "set_state");
  return ECR_OK;
}
}  // namespace

extern "C" {

ecr_status ecr_footprint(const ecr_params *params, size_t *device_bytes) {
  const std::string v = validate(params);
  if (!v.empty()) return fail(nullptr, params && params->abi_version != ECR_ABI_VERSION ? ECR_EABI : ECR_EINVAL, v);
  if (!device_bytes) return fail(nullptr, ECR_EINVAL, "device_bytes is NULL");
  *device_bytes = make_layout(params).total;
  return ECR_OK;
}

}  // extern "C"

namespace {

// release what a run holds besides its arena: events and captured graphs
void release_run(ecr_run *r) {
  forget_batch_graphs(r);
  harvest(r);
  for (auto e : r->free_events) (void)hipEventDestroy(e);
  r->free_events.clear();
  for (auto &row : r->gexec)
    for (auto &g : row) {
      if (g) (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

// bind run r (fresh) to the arena at device_arena and upload its tables;
// params were validated and the arena checked by the caller
ecr_status init_run(ecr_run *r, const ecr_params *params, const Layout &L, const KParams &K, const Tables &T,
                    double w, void *device_arena, void *hip_stream) {
  r->p = *params;
  r->kp = K;
  r->stream = (hipStream_t)hip_stream;
  r->base = (char *)(((uintptr_t)device_arena + kAlign - 1) / kAlign * kAlign);
  r->L = L;
  r->fp32 = params->precision == ECR_FP32_MIXED;
  r->fcap = step_fcap(K.n, step_resident_wgs(r->fp32));
  r->weight = w;
  r->ncell = ncells(params);
  r->nnode = nnodes(params);
  r->cur = 0;
  r->need_sort = true;
  r->prof = 0u;
  for (int k = 0; k < ECR_N_KERNELS; ++k) r->prof_seen[k] = 0;
  for (int k = 0; k < ECR_N_KERNELS; ++k) {
    r->ms[k] = 0.0;
    r->launches[k] = 0;
  }
  hipError_t e = hipMemcpyAsync(at<Tables>(r, L.tables), &T, sizeof(Tables), hipMemcpyHostToDevice, r->stream);
  if (e == hipSuccess && params->efield_nodes)
    e = hipMemcpyAsync(at<double>(r, L.efield), params->efield_nodes, 8 * 3 * (size_t)r->nnode,
                       hipMemcpyHostToDevice, r->stream);
  if (e == hipSuccess && params->bfield_nodes)
    e = hipMemcpyAsync(at<double>(r, L.bfield), params->bfield_nodes, 8 * 3 * (size_t)r->nnode,
                       hipMemcpyHostToDevice, r->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
  if (e != hipSuccess) {
    g_thread_err = std::string("upload failed: ") + hipGetErrorString(e);
    return ECR_EDEVICE;
  }
  r->p.efield_nodes = params->efield_nodes ? (const double *)1 : nullptr;  // only its presence is kept
  r->p.bfield_nodes = nullptr;  // the kernels read the arena copy through kp.bmap
  r->kp.bmap = params->bfield_nodes ? at<double>(r, L.bfield) : nullptr;
  r->kp.cellid = at<uint32_t>(r, L.cellid);
  r->kp.cxreq = (params->flags & ECR_FLAG_CX_PARTNER) ? at<uint32_t>(r, L.cxreq) : nullptr;
  r->kp.cxchunk = (params->flags & ECR_FLAG_CX_PARTNER) ? at<uint32_t>(r, L.cxchunk) : nullptr;
  r->kp.cell_off = at<uint32_t>(r, L.cell_off);
  r->kp.bden = needs_bden(params) ? at<double>(r, L.bden) : nullptr;
  if (r->kp.bden) launch_cell_bden(r->kp, at<double>(r, L.bden), r->stream);
  zero_accumulators(r);
  static std::atomic<uint64_t> next_uid{1};
  r->uid = next_uid++;
  if (r->fp32) write_jobs<float>(r);
  else write_jobs<double>(r);
  return ECR_OK;
}

// checks shared by ecr_create and ecr_create_static: the parameters, and the
// derived constants and tables
ecr_status prepare(const ecr_params *params, Layout &L, KParams &K, Tables &T, double &w) {
  const std::string v = validate(params);
  if (!v.empty()) return fail(nullptr, params && params->abi_version != ECR_ABI_VERSION ? ECR_EABI : ECR_EINVAL, v);
  L = make_layout(params);
  derive(params, K, T, w);
  if (max_probability(params, K, T) >= 0.1)
    return fail(nullptr, ECR_EDT, "per-step ionisation + charge-exchange probability can reach 0.1: reduce dt_s");
  return ECR_OK;
}

// The static workspace of ecr_create_static: one array per GPU the library
// runs on (each device holds its own copy until the process ends), and one
// run handle per device.  In host code `scratch` only names the symbol; its
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kStaticArenaBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_base[kMaxDevices];
ecr_run g_static_run[kMaxDevices];

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticArenaBytes];

extern "C" {

ecr_status ecr_create(const ecr_params *params, void *device_arena, size_t arena_bytes, void *hip_stream,
                      ecr_run **out) {
  if (!out) return fail(nullptr, ECR_EINVAL, "out is NULL");
  *out = nullptr;
  Layout L;
  KParams K;
  Tables T;
  double w;
  // the arena is checked before the tables, so that a missing arena is
  // EINVAL whatever the parameters' probabilities
  {
    const std::string v = validate(params);
    if (!v.empty()) return fail(nullptr, params && params->abi_version != ECR_ABI_VERSION ? ECR_EABI : ECR_EINVAL, v);
    if (!device_arena) return fail(nullptr, ECR_EINVAL, "device_arena is NULL");
    if (arena_bytes < make_layout(params).total) return fail(nullptr, ECR_ENOMEM, "arena smaller than ecr_footprint()");
  }
  const ecr_status st = prepare(params, L, K, T, w);
  if (st != ECR_OK) return st;
  ecr_run *r = new ecr_run();
  const ecr_status si = init_run(r, params, L, K, T, w, device_arena, hip_stream);
  if (si != ECR_OK) {
    delete r;
    return si;
  }
  r->live = true;
  *out = r;
  return ECR_OK;
}

ecr_status ecr_create_static(const ecr_params *params, void *hip_stream, ecr_run **out) {
  if (!out) return fail(nullptr, ECR_EINVAL, "out is NULL");
  *out = nullptr;
  Layout L;
  KParams K;
  Tables T;
  double w;
  const ecr_status st = prepare(params, L, K, T, w);
  if (st != ECR_OK) return st;
  if (L.total > kStaticArenaBytes)
    return fail(nullptr, ECR_ENOMEM,
                "run needs " + std::to_string(L.total) + " bytes of device memory; the static workspace holds " +
                    std::to_string(kStaticArenaBytes) + " (create the run with ecr_create and an arena instead)");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(nullptr, ECR_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, ECR_EDEVICE, "device index beyond the static workspaces");
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_base[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(nullptr, ECR_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_static_base[dev] = p;
  }
  ecr_run *r = &g_static_run[dev];
  if (r->live) return fail(nullptr, ECR_ESTATE, "the static workspace of this device holds a run: ecr_destroy it first");
  *r = ecr_run();
  r->is_static = true;
  const ecr_status si = init_run(r, params, L, K, T, w, g_static_base[dev], hip_stream);
  if (si != ECR_OK) return si;
  r->live = true;
  *out = r;
  return ECR_OK;
}

ecr_status ecr_init_ions(ecr_run *r) {
  if (!r) return fail(nullptr, ECR_EINVAL, "run is NULL");
  if (r->failed) return fail(r, ECR_ESTATE, "run failed earlier");
  r->cur = 0;
  if (r->fp32) launch_init<float>(r->kp, soa<float>(r, 0), r->stream);
  else launch_init<double>(r->kp, soa<double>(r, 0), r->stream);
  if (r->p.flags & ECR_FLAG_EVENTS) launch_fill_u8(at<uint8_t>(r, r->L.evlog), 0, r->kp.n, r->stream);
  zero_accumulators(r);
  build_charge_grid(r);
  r->step = 0;
  r->need_sort = true;
  r->initialized = true;
  return check_hip(r, hipGetLastError(), "init_ions launch");
}

ecr_status ecr_step(ecr_run *r, int64_t n_steps) {
  if (!r) return fail(nullptr, ECR_EINVAL, "run is NULL");
  if (n_steps < 0) return fail(r, ECR_EINVAL, "n_steps < 0");
  if (r->failed) return fail(r, ECR_ESTATE, "run failed earlier");
  if (!r->initialized) return fail(r, ECR_ESTATE, "call ecr_init_ions or ecr_set_state first");
  for (int64_t i = 0; i < n_steps; ++i) {
    if (r->fp32) do_step<float>(r, StepArg{nullptr, (uint32_t)r->step});
    else do_step<double>(r, StepArg{nullptr, (uint32_t)r->step});
  }
  return check_hip(r, hipGetLastError(), "step launch");
}

namespace {

// capture one sort period starting from buffer r->cur; host counters are
// restored afterwards (capturing runs nothing)
hipError_t capture_period(ecr_run *r, hipGraphExec_t *out) {
  const int64_t K = r->p.sort_every;
  const int64_t step0 = r->step, steps0 = r->steps, dens0 = r->dens_steps;
  const int cur0 = r->cur, par0 = r->chg_par;
  const bool need0 = r->need_sort;
  const uint32_t *base = at<uint32_t>(r, r->L.stepc);
  hipError_t e = hipStreamBeginCapture(r->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  for (int64_t i = 0; i < K; ++i) {
    if (r->fp32) do_step<float>(r, StepArg{base, (uint32_t)i});
    else do_step<double>(r, StepArg{base, (uint32_t)i});
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(r->stream, &g);
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  r->step = step0;
  r->steps = steps0;
  r->dens_steps = dens0;
  r->cur = cur0;
  r->chg_par = par0;
  r->need_sort = need0;
  return e;
}

}  // namespace

ecr_status ecr_step_graph(ecr_run *r, int64_t n_steps) {
  if (!r) return fail(nullptr, ECR_EINVAL, "run is NULL");
  if (n_steps < 0) return fail(r, ECR_EINVAL, "n_steps < 0");
  if (r->failed) return fail(r, ECR_ESTATE, "run failed earlier");
  if (!r->initialized) return fail(r, ECR_ESTATE, "call ecr_init_ions or ecr_set_state first");
  const int64_t K = r->p.sort_every;
  const bool dep = (r->p.process_mask & ECR_P_DEPOSIT) != 0;
  while (n_steps > 0) {
    if (r->stream == nullptr || r->prof || r->step % K != 0 || n_steps < K || r->step + K > 0xffffffffLL) {
      // not at the start of a whole period (or nothing to capture on): one eager step
      const ecr_status st = ecr_step(r, 1);
      if (st != ECR_OK) return st;
      --n_steps;
      continue;
    }
    hipGraphExec_t &ge = r->gexec[r->cur][r->chg_par];
    if (!ge) {
      const hipError_t e = capture_period(r, &ge);
      if (e != hipSuccess) {
        ge = nullptr;
        return check_hip(r, e, "graph capture");
      }
    }
    launch_fill_u32(at<uint32_t>(r, r->L.stepc), (uint32_t)r->step, 1, r->stream);
    const hipError_t e = hipGraphLaunch(ge, r->stream);
    if (e != hipSuccess) return check_hip(r, e, "graph launch");
    r->step += K;
    r->steps += K;
    if (dep) r->dens_steps += K;
    r->cur = 1 - r->cur;  // the period's sort moved the state to the other buffer
    if ((r->p.flags & (ECR_FLAG_SELF_NE | ECR_FLAG_SELF_N0)) && (K & 1)) r->chg_par = 1 - r->chg_par;
    r->need_sort = false;
    n_steps -= K;
  }
  return check_hip(r, hipGetLastError(), "graph step");
}

ecr_status ecr_step_batch(ecr_run *const *runs, int32_t n_runs, int64_t n_steps, void *hip_stream) {
  if (!runs || n_runs < 0 || n_steps < 0) return fail(nullptr, ECR_EINVAL, "bad batch arguments");
  const hipStream_t st = (hipStream_t)hip_stream;
  std::vector<ecr_run *> rs;
  for (int32_t k = 0; k < n_runs; ++k) {
    ecr_run *r = runs[k];
    if (!r || r->failed || !r->initialized || r->stream != st)
      return fail(nullptr, ECR_EINVAL, "every run must be initialised and bound to the batch stream");
    for (ecr_run *q : rs)
      if (q == r) return fail(nullptr, ECR_EINVAL, "a run appears twice in the batch");
    rs.push_back(r);
  }
  if (rs.empty()) return ECR_OK;
  const int64_t K = rs[0]->p.sort_every;
  while (n_steps > 0) {
    bool aligned = st != nullptr && n_steps >= K;
    for (ecr_run *r : rs)
      aligned = aligned && r->p.sort_every == K && r->step % K == 0 && !r->prof && r->step + K <= 0xffffffffLL;
    if (!aligned) {
      // not at the start of a common sort period: one step, batched launches
      batch_step_all(rs, st, false, 0u);
      for (ecr_run *r : rs) {
        const ecr_status s2 = check_hip(r, hipGetLastError(), "batch step launch");
        if (s2 != ECR_OK) return s2;
      }
      --n_steps;
      continue;
    }
    const std::vector<uint64_t> key = batch_key(rs);
    hipGraphExec_t ge = nullptr;
    bool seen = false;
    {
      std::lock_guard<std::mutex> lock(g_bgraph_mu);
      for (const BatchGraph &g : g_bgraphs)
        if (g.stream == st && g.key == key) ge = g.ge;
      if (!ge) {
        // a set of runs is the same set whichever buffers its runs start from
        std::vector<uint64_t> ids;
        for (uint64_t k : key) ids.push_back(k >> 2);
        for (const auto &q : g_bseen) seen |= q == ids;
        if (!seen) {
          if (g_bseen.size() >= kMaxBatchSeen) g_bseen.erase(g_bseen.begin());
          g_bseen.push_back(ids);
        }
      }
    }
    if (!ge && !seen) {
      // first period of this set of runs: stepped eagerly, batched launches
      for (int64_t i = 0; i < K; ++i) batch_step_all(rs, st, false, 0u);
      for (ecr_run *r : rs) {
        const ecr_status s2 = check_hip(r, hipGetLastError(), "batch step launch");
        if (s2 != ECR_OK) return s2;
      }
      n_steps -= K;
      continue;
    }
    if (!ge) {
      const hipError_t e = capture_batch_period(rs, st, K, &ge);
      if (e != hipSuccess) return check_hip(rs[0], e, "batch graph capture");
      std::lock_guard<std::mutex> lock(g_bgraph_mu);
      if (g_bgraphs.size() >= kMaxBatchGraphs) {
        (void)hipStreamSynchronize(g_bgraphs.front().stream);
        (void)hipGraphExecDestroy(g_bgraphs.front().ge);
        g_bgraphs.erase(g_bgraphs.begin());
      }
      g_bgraphs.push_back({st, key, ge});
    }
    // every run's first step of the period into its counter word, then the period
    for (size_t k0 = 0; k0 < rs.size(); k0 += kMaxBatch) {
      SetWords w{};
      w.n = (int)std::min(rs.size() - k0, (size_t)kMaxBatch);
      for (int j = 0; j < w.n; ++j) {
        w.ptr[j] = at<uint32_t>(rs[k0 + j], rs[k0 + j]->L.stepc);
        w.val[j] = (uint32_t)rs[k0 + j]->step;
      }
      launch_set_words(w, st);
    }
    const hipError_t e = hipGraphLaunch(ge, st);
    if (e != hipSuccess) return check_hip(rs[0], e, "batch graph launch");
    for (ecr_run *r : rs) {
      r->step += K;
      r->steps += K;
      if (r->p.process_mask & ECR_P_DEPOSIT) r->dens_steps += K;
      r->cur = 1 - r->cur;
      if ((r->p.flags & (ECR_FLAG_SELF_NE | ECR_FLAG_SELF_N0)) && (K & 1)) r->chg_par = 1 - r->chg_par;
      r->need_sort = false;
    }
    n_steps -= K;
  }
  for (ecr_run *r : rs) {
    const ecr_status s2 = check_hip(r, hipGetLastError(), "batch step");
    if (s2 != ECR_OK) return s2;
  }
  return ECR_OK;
}

ecr_status ecr_read_tallies(ecr_run *r, ecr_tallies *out) {
  if (!r || !out) return fail(r, ECR_EINVAL, "NULL argument");
  DevAccum h;
  launch_sum_moments(at<double>(r, r->L.moments), moment_slots(r->kp.n), at<DevAccum>(r, r->L.acc),
                     r->stream);
  hipError_t e = hipMemcpyAsync(&h, at<DevAccum>(r, r->L.acc), sizeof(DevAccum), hipMemcpyDeviceToHost, r->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
  if (e != hipSuccess) return check_hip(r, e, "read_tallies");
  *out = h.t;
  out->steps = r->steps;
  if (h.err & ERR_COUL_OVERFLOW) {
    r->err = "a Coulomb chunk exceeded the LDS capacity; its cells were skipped";
    out->anomalies += 1;
  }
  if (out->anomalies > 0) return fail(r, ECR_ENUMERIC, r->err.empty() ? "anomalies counted" : r->err);
  return ECR_OK;
}

ecr_status ecr_read_density(ecr_run *r, uint32_t field, double *out, int64_t *steps_accum) {
  if (!r || !out) return fail(r, ECR_EINVAL, "NULL argument");
  if (field >= ECR_N_FIELDS) return fail(r, ECR_EINVAL, "field out of range");
  hipError_t e = hipMemcpyAsync(out, at<double>(r, r->L.dens) + (size_t)field * r->nnode, 8 * (size_t)r->nnode,
                                hipMemcpyDeviceToHost, r->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
  if (e != hipSuccess) return check_hip(r, e, "read_density");
  if (steps_accum) *steps_accum = r->dens_steps;
  return ECR_OK;
}


ecr_status ecr_get_state(ecr_run *r, ecr_state_view *v) {
  if (!r || !v) return fail(r, ECR_EINVAL, "NULL argument");
  if (v->n != r->kp.n) return fail(r, ECR_EINVAL, "view length differs from n_particles");
  if (!r->initialized) return fail(r, ECR_ESTATE, "no state yet");
  return r->fp32 ? get_state_t<float>(r, v) : get_state_t<double>(r, v);
}

ecr_status ecr_set_state(ecr_run *r, const ecr_state_view *v) {
  if (!r || !v) return fail(r, ECR_EINVAL, "NULL argument");
  if (r->failed) return fail(r, ECR_ESTATE, "run failed earlier");
  if (v->n != r->kp.n) return fail(r, ECR_EINVAL, "view length differs from n_particles");
  if (!v->x || !v->y || !v->z || !v->vx || !v->vy || !v->vz || !v->q) return fail(r, ECR_EINVAL, "NULL array");
  if (v->step < 0) return fail(r, ECR_EINVAL, "negative step");
  ecr_status st = r->fp32 ? set_state_t<float>(r, v) : set_state_t<double>(r, v);
  if (st != ECR_OK) return st;
  r->step = v->step;
  zero_accumulators(r);
  if (r->p.flags & ECR_FLAG_EVENTS) launch_fill_u8(at<uint8_t>(r, r->L.evlog), 0, r->kp.n, r->stream);
  if (v->cell) {
    // sort with the given collision cells, staged by set_state_t
    const uint32_t *stage = at<uint32_t>(r, r->L.soa[1][7]);
    if (r->fp32) do_sort<float>(r, stage);
    else do_sort<double>(r, stage);
    r->need_sort = false;
  } else {
    r->need_sort = true;
  }
  build_charge_grid(r);
  r->initialized = true;
  return check_hip(r, hipGetLastError(), "set_state");
}

ecr_status ecr_event_log(ecr_run *r, uint8_t *out) {
  if (!r || !out) return fail(r, ECR_EINVAL, "NULL argument");
  if (!(r->p.flags & ECR_FLAG_EVENTS)) return fail(r, ECR_ESTATE, "run created without ECR_FLAG_EVENTS");
  const int64_t n = r->kp.n;
  std::vector<uint8_t> ev(n);
  std::vector<uint32_t> pid(n);
  hipError_t e = hipMemcpyAsync(ev.data(), r->base + r->L.evlog, n, hipMemcpyDeviceToHost, r->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(pid.data(), r->base + r->L.soa[r->cur][7], 4 * n, hipMemcpyDeviceToHost, r->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
  if (e != hipSuccess) return check_hip(r, e, "event_log");
  for (int64_t j = 0; j < n; ++j) out[pid[j]] = ev[j];
  return ECR_OK;
}

ecr_status ecr_weight(const ecr_run *r, double *w) {
  if (!r || !w) return fail(nullptr, ECR_EINVAL, "NULL argument");
  *w = r->weight;
  return ECR_OK;
}

ecr_status ecr_profile(ecr_run *r, int32_t enable) {
  if (!r) return fail(nullptr, ECR_EINVAL, "run is NULL");
  harvest(r);
  r->prof = (uint32_t)enable & ((1u << ECR_N_KERNELS) - 1u);
  for (int k = 0; k < ECR_N_KERNELS; ++k) {
    r->ms[k] = 0.0;
    r->launches[k] = 0;
    r->prof_seen[k] = 0;
  }
  return ECR_OK;
}

ecr_status ecr_profile_stride(ecr_run *r, int32_t stride) {
  if (!r) return fail(nullptr, ECR_EINVAL, "run is NULL");
  if (stride < 1) return fail(r, ECR_EINVAL, "stride must be >= 1");
  r->prof_stride = stride;
  return ECR_OK;
}

ecr_status ecr_kernel_times(ecr_run *r, double *ms_out, int64_t *launches_out) {
  if (!r) return fail(nullptr, ECR_EINVAL, "run is NULL");
  harvest(r);
  for (int k = 0; k < ECR_N_KERNELS; ++k) {
    if (ms_out) ms_out[k] = r->ms[k];
    if (launches_out) launches_out[k] = r->launches[k];
  }
  return ECR_OK;
}

const char *ecr_last_error(const ecr_run *r) { return r ? r->err.c_str() : g_thread_err.c_str(); }

ecr_status ecr_destroy(ecr_run *r) {
  if (!r) return ECR_OK;
  if (r->is_static) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (r->live) {
      (void)hipStreamSynchronize(r->stream);  // nothing may still use the workspace
      release_run(r);
      r->live = false;
    }
    return ECR_OK;
  }
  release_run(r);
  delete r;
  return ECR_OK;
}

ecr_status ecr_selftest_philox(uint64_t seed, uint32_t ctr0, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
                               uint32_t *out_dev, void *hip_stream) {
  if (n < 0 || (n > 0 && !out_dev)) return fail(nullptr, ECR_EINVAL, "bad arguments");
  launch_selftest_philox(seed, ctr0, c1, c2, c3, n, out_dev, (hipStream_t)hip_stream);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? ECR_OK : fail(nullptr, ECR_EDEVICE, hipGetErrorString(e));
}

ecr_status ecr_selftest_divsqrt(const double *a_dev, const double *b_dev, int64_t n, double *q_dev, double *r_dev,
                                void *hip_stream) {
  if (n < 0 || (n > 0 && (!a_dev || !b_dev || !q_dev || !r_dev))) return fail(nullptr, ECR_EINVAL, "bad arguments");
  launch_selftest_divsqrt(a_dev, b_dev, n, q_dev, r_dev, (hipStream_t)hip_stream);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? ECR_OK : fail(nullptr, ECR_EDEVICE, hipGetErrorString(e));
}

}  // extern "C"
