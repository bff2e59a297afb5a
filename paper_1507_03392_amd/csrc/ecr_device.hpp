// ecr_device.hpp -- device-side building blocks of the ion PIC/MCC step
// (Mironov et al., Sec. II), shared by the gfx950 kernels of this library.
//
// Every function here is written for one particle in registers.  Arithmetic
// is templated on the storage/compute type R (double for the FP64 path,
// float for the FP32-mixed path); all accumulators stay double.  The library
// is compiled with -ffp-contract=off, so every expression below rounds once
// per operation in the order written; decisions (boundary crossings, the
// ionisation / charge-exchange draw, cell indices) use only + - * / sqrt and
// integer operations, which are correctly rounded on both CPU and GPU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ecr {

constexpr double kE = 1.602176634e-19;       // elementary charge, C
constexpr double kAmu = 1.66053906660e-27;   // atomic mass unit, kg
constexpr double kEps0 = 8.8541878128e-12;   // vacuum permittivity, F/m
constexpr double kPi = 3.14159265358979323846;
constexpr double kWallEps = 1e-9;            // re-emission offset from a wall, m

// Philox stream ids (counter word 2); word 0 = particle id, word 1 = step,
// word 3 = call index within the stream.
enum : uint32_t { S_INIT = 0, S_STEP = 1, S_COUL = 2, S_BND = 3, S_CX = 4, S_HEAT = 5, S_EL = 6 };
enum : uint8_t { EV_NONE = 0, EV_IONIZE = 1, EV_CX = 2, EV_WALL = 3, EV_EXTRACT = 4, EV_ELASTIC = 5, EV_CX_PARTNER = 6 };
enum : uint32_t { P_PUSH = 1, P_IONIZE = 2, P_CX = 4, P_COULOMB = 8, P_DEPOSIT = 16, P_HEAT = 32, P_ELASTIC = 64 };

// Nanbu A(s) table: ln A at s = 2^e (1 + j/K), e in [kAeLo, kAeHi], j in [0, K)
constexpr int kAeLo = -20;
constexpr int kAeHi = 2;
constexpr int kAK = 128;
constexpr int kANodes = (kAeHi - kAeLo + 1) * kAK + 1;
constexpr double kSLo = 9.5367431640625e-07;  // 2^-20: A = 1/s below
constexpr double kSHi = 8.0;                  // isotropic at and above

constexpr int kMaxS = 4;
constexpr int kMaxQ = 32;
constexpr int kMaxN = 4;  // electrons removed by one ionisation

// Run constants that every kernel reads (passed by value).
struct KParams {
  double R0, hL, R0sq, rap2, inlet_x, inlet_y;
  double idx, idy, idz, ia2, ic2, zone_a, zone_c;
  double B0, c1, c2, c3, c4;
  double dt, nfac, Cs;
  double hx, hy, hz;  // cell sizes
  // heating kick, [outside, inside] the zone: fixed-background n_e, and
  // 2.38e-6 sqrt(T_e) (the electron Larmor radius times |B|)
  double ne_zone[2], rl_zone[2];
  const double *bmap;  // device [3][nnode] node magnetic field (T), or null: the analytic field
  // exchange partners (ECR_FLAG_CX_PARTNER): the exchanges of the step per
  // species and collision cell [s][cell], a flag per Coulomb chunk holding
  // any, each slot's collision cell and each cell's first slot
  uint32_t *cxreq, *cxchunk;
  const uint32_t *cellid, *cell_off;
  // heating kick with self-consistent electrons: |B| x hx at each cell centre
  const double *bden;
  double mass[kMaxS], sig_w[kMaxS], sig_n[kMaxS], sig_i[kMaxS], decx[kMaxS], ccx[kMaxS];
  double cel[kMaxS];     // n0 sigma_el1 dt (elastic ion-atom scattering)
  double sdt_cx[kMaxS], sdt_el[kMaxS];  // sigma1 dt, sigma_el1 dt: neutrals from the tracked atoms
  int32_t nion;          // ionisation channels with a nonzero rate: 1 .. kMaxN
  // per species pair (a, b): reduced mass mu = ma mb / (ma + mb), mu / ma, mu / mb
  double mu[kMaxS][kMaxS], mra[kMaxS][kMaxS], mrb[kMaxS][kMaxS];
  uint32_t cxok[kMaxS];  // bit Q: charge exchange allowed from Q
  int64_t sp_end[kMaxS]; // ids [sp_end[s-1], sp_end[s]) are species s
  int64_t n, nnode;
  uint32_t ncell;  // nx ny nz: the stride of the cell grids' channels
  int32_t nx, ny, nz, nx1, ny1, nspecies;
  uint32_t seed_lo, seed_hi, pmask, dmask, flags;
};

// Device-resident tables.
// the step number of a launch: off alone, or *base + off when the launch
// sits in a replayed graph and reads its first step from device memory
struct StepArg {
  const uint32_t *base;
  uint32_t off;
  __device__ __forceinline__ uint32_t get() const { return base ? *base + off : off; }
};

struct Tables {
  double qmh[kMaxS][kMaxQ];      // (Q e / M) dt / 2
  double pion[kMaxS][2][kMaxQ];  // ionisation probability per step [outside, inside]
  double kdt[kMaxS][2][kMaxQ];   // rate x dt [outside, inside], for a cell's own electron density
  // the same for Q -> Q+n, n = 2..kMaxN ([n-2]); zero where Q + n passes z_max
  double pmul[kMaxS][2][kMaxN - 1][kMaxQ];
  double kmul[kMaxS][2][kMaxN - 1][kMaxQ];
  double dheat[kMaxS][2][kMaxQ]; // heating kick D^2 / n_e [outside, inside]
  double lnA[kANodes];           // ln A at the Nanbu table nodes
};

template <typename R>
struct Soa {
  R *x, *y, *z, *vx, *vy, *vz;
  uint8_t *qs;   // charge state in bits 0-4, species in bits 5-7
  uint32_t *pid;
  uint32_t *birth;  // step the ion was made from an atom (ECR_BIRTH_NONE: atom or unknown); touched on events only
};

constexpr uint32_t kBirthNone = 0xffffffffu;

// first-passage histogram bin of a time of t steps: floor(log2 t), 0 for t <= 1
__device__ __forceinline__ int fpt_bin(uint32_t t) { return t <= 1u ? 0 : 31 - __clz(t); }

__device__ __forceinline__ int q_of(uint8_t qs) { return qs & 31; }
__device__ __forceinline__ int sp_of(uint8_t qs) { return qs >> 5; }
__device__ __forceinline__ uint8_t make_qs(int q, int s) { return (uint8_t)(q | (s << 5)); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the key bumped by the Weyl constants between
// rounds.  The key is the run seed; it is uniform across a wavefront, so the
// key schedule runs on the scalar unit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint4 draw(const KParams &P, uint32_t id, uint32_t step, uint32_t stream,
                                      uint32_t k) {
  return philox(id, step, stream, k, P.seed_lo, P.seed_hi);
}

// uniform in [0,1) from 27 bits of a and 26 bits of b (exact in binary64)
__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ void sincos_r(double x, double *s, double *c) { sincos(x, s, c); }
__device__ __forceinline__ void sincos_r(float x, float *s, float *c) { sincosf(x, s, c); }
// sin(pi x), cos(pi x): exact argument reduction, for angles 2 pi u with u in [0,1)
__device__ __forceinline__ void sincospi_r(double x, double *s, double *c) { sincospi(x, s, c); }
__device__ __forceinline__ void sincospi_r(float x, float *s, float *c) { sincospif(x, s, c); }

// sin and cos of 2 pi u for u in [0, 1) (the azimuth of a collision, a
// continuous outcome): 4u = q + f exactly with q = rint(4u), f in [-1/2, 1/2],
// theta = f pi/2 in [-pi/4, pi/4]; Taylor polynomials in theta^2 through
// theta^17 (sine) and theta^18 (cosine), truncation below 5e-17; the quarter
// turn q mod 4 swaps and negates.  Within a few ulp of the exact values.
__device__ __forceinline__ void sincos_2pi(double u, double *sn, double *cs) {
  const double t = 4.0 * u;
  const double q = rint(t);
  const double th = (t - q) * 1.5707963267948966192;
  const double z = th * th;
  double ps = 1.0 / 355687428096000.0;
  ps = fma(ps, z, -1.0 / 1307674368000.0);
  ps = fma(ps, z, 1.0 / 6227020800.0);
  ps = fma(ps, z, -1.0 / 39916800.0);
  ps = fma(ps, z, 1.0 / 362880.0);
  ps = fma(ps, z, -1.0 / 5040.0);
  ps = fma(ps, z, 1.0 / 120.0);
  ps = fma(ps, z, -1.0 / 6.0);
  const double s = fma(th * z, ps, th);
  double pc = -1.0 / 6402373705728000.0;
  pc = fma(pc, z, 1.0 / 20922789888000.0);
  pc = fma(pc, z, -1.0 / 87178291200.0);
  pc = fma(pc, z, 1.0 / 479001600.0);
  pc = fma(pc, z, -1.0 / 3628800.0);
  pc = fma(pc, z, 1.0 / 40320.0);
  pc = fma(pc, z, -1.0 / 720.0);
  pc = fma(pc, z, 1.0 / 24.0);
  pc = fma(pc, z, -0.5);
  const double c = fma(z, pc, 1.0);
  const int k = (int)q & 3;
  const double a = (k & 1) ? c : s, b = (k & 1) ? s : c;
  *sn = (k & 2) ? -a : a;
  *cs = (k == 1 || k == 2) ? -b : b;
}
__device__ __forceinline__ void sincos_2pi(double u, float *sn, float *cs) { sincospif((float)(2.0 * u), sn, cs); }

// two standard normals from two uniforms
__device__ __forceinline__ void box_muller(double ua, double ub, double &n1, double &n2) {
  const double r = sqrt(-2.0 * log(1.0 - ua));
  const double th = 2.0 * kPi * ub;
  double s, c;
  sincos(th, &s, &c);
  n1 = r * c;
  n2 = r * s;
}

// ---------------------------------------------------------------------------
// Magnetic field (Sec. II): solenoid mirror Bz(z) = B0 (1 + k (2z/L)^2) on
// axis, continued off axis to second order (Br = -(r/2) dBz/dz,
// Bz -= (r^2/4) d2Bz/dz2), plus the analytic hexapole
// (BH/R0^2)(2xy, x^2 - y^2, 0).  c1 = 4 k B0/L^2, c2 = 2 BH/R0^2,
// c3 = BH/R0^2, c4 = 2 k B0/L^2.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void field_B(const KParams &P, R x, R y, R z, R &bx, R &by, R &bz) {
  const R c1 = (R)P.c1, c2 = (R)P.c2, c3 = (R)P.c3, c4 = (R)P.c4, B0 = (R)P.B0;
  const R xx = x * x, yy = y * y, zz = z * z, xy = x * y;
  bx = c2 * xy - (c1 * x) * z;
  by = c3 * (xx - yy) - (c1 * y) * z;
  bz = (B0 + c1 * zz) - c4 * (xx + yy);
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// lower node index and fractional offset of a coordinate on one mesh axis
template <typename R>
__device__ __forceinline__ void cic_axis(R pos, R origin, R inv_h, int ncell, int &i, R &t) {
  const R f = (pos + origin) * inv_h;
  const int k = clampi((int)floor(f), 0, ncell - 1);
  i = k;
  t = f - (R)k;
}

template <typename R>
__device__ __forceinline__ uint32_t cell_of(const KParams &P, R x, R y, R z) {
  const int ix = clampi((int)floor((x + (R)P.R0) * (R)P.idx), 0, P.nx - 1);
  const int iy = clampi((int)floor((y + (R)P.R0) * (R)P.idy), 0, P.ny - 1);
  const int iz = clampi((int)floor((z + (R)P.hL) * (R)P.idz), 0, P.nz - 1);
  return (uint32_t)ix + (uint32_t)P.nx * ((uint32_t)iy + (uint32_t)P.ny * (uint32_t)iz);
}

// trilinear gather of a node vector field [3][nnode] (the electric field,
// or a magnetic field map)
template <typename R>
__device__ __forceinline__ void gather_E(const KParams &P, const double *__restrict__ ef, R x, R y, R z,
                                         R E[3]) {
  int ix, iy, iz;
  R tx, ty, tz;
  cic_axis<R>(x, (R)P.R0, (R)P.idx, P.nx, ix, tx);
  cic_axis<R>(y, (R)P.R0, (R)P.idy, P.ny, iy, ty);
  cic_axis<R>(z, (R)P.hL, (R)P.idz, P.nz, iz, tz);
  const R wx[2] = {(R)1 - tx, tx}, wy[2] = {(R)1 - ty, ty}, wz[2] = {(R)1 - tz, tz};
  for (int c = 0; c < 3; ++c) {
    const double *F = ef + (int64_t)c * P.nnode;
    R acc = (R)0;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int64_t node = (int64_t)(ix + dx) + (int64_t)P.nx1 * ((iy + dy) + (int64_t)P.ny1 * (iz + dz));
          acc = acc + ((wx[dx] * wy[dy]) * wz[dz]) * (R)F[node];
        }
    E[c] = acc;
  }
}

// ---------------------------------------------------------------------------
// Boris push: v- = v + hE; t = hB; s = 2t/(1 + t.t); v' = v- + v- x t;
// v+ = v- + v' x s; v = v+ + hE; x += v dt with h = (Q e/M) dt/2.
// ---------------------------------------------------------------------------
// FLD: bit 0 an electric field grid, bit 1 a magnetic field map (P.bmap)
// in place of the analytic field
template <typename R, int FLD>
__device__ __forceinline__ void boris(const KParams &P, R h, const R E[3], R &x, R &y, R &z, R &vx, R &vy,
                                      R &vz) {
  R bx, by, bz;
  if (FLD & 2) {
    R B[3];
    gather_E<R>(P, P.bmap, x, y, z, B);
    bx = B[0];
    by = B[1];
    bz = B[2];
  } else {
    field_B<R>(P, x, y, z, bx, by, bz);
  }
  R vmx = vx, vmy = vy, vmz = vz;
  if (FLD & 1) {
    vmx = vmx + h * E[0];
    vmy = vmy + h * E[1];
    vmz = vmz + h * E[2];
  }
  const R tx = h * bx, ty = h * by, tz = h * bz;
  const R t2 = (tx * tx + ty * ty) + tz * tz;
  const R f = (R)2 / ((R)1 + t2);
  const R sx = f * tx, sy = f * ty, sz = f * tz;
  const R vpx = vmx + (vmy * tz - vmz * ty);
  const R vpy = vmy + (vmz * tx - vmx * tz);
  const R vpz = vmz + (vmx * ty - vmy * tx);
  R nvx = vmx + (vpy * sz - vpz * sy);
  R nvy = vmy + (vpz * sx - vpx * sz);
  R nvz = vmz + (vpx * sy - vpy * sx);
  if (FLD & 1) {
    nvx = nvx + h * E[0];
    nvy = nvy + h * E[1];
    nvz = nvz + h * E[2];
  }
  vx = nvx;
  vy = nvy;
  vz = nvz;
  const R dt = (R)P.dt;
  x = x + nvx * dt;
  y = y + nvy * dt;
  z = z + nvz * dt;
}

// ---------------------------------------------------------------------------
// First exit of the step's segment x0 -> x1 from the chamber: flange
// z = +L/2 (kind 1), flange z = -L/2 (kind 2) or cylinder r = R0 (kind 3);
// the smallest fraction wins, ties go to the flange.
// ---------------------------------------------------------------------------
enum : int { X_NONE = 0, X_EXT = 1, X_INJ = 2, X_CYL = 3 };

template <typename R>
__device__ __forceinline__ int segment_exit(const KParams &P, R x0, R y0, R z0, R x1, R y1, R z1, R &fout) {
  const R hL = (R)P.hL, R0sq = (R)P.R0sq;
  const R dx = x1 - x0, dy = y1 - y0, dz = z1 - z0;
  R best = (R)2;
  int kind = X_NONE;
  if (z1 > hL) {
    best = (hL - z0) / dz;
    kind = X_EXT;
  } else if (z1 < -hL) {
    best = (-hL - z0) / dz;
    kind = X_INJ;
  }
  if (x1 * x1 + y1 * y1 > R0sq) {
    const R a = dx * dx + dy * dy;
    const R b = x0 * dx + y0 * dy;
    const R c = (x0 * x0 + y0 * y0) - R0sq;
    R D = b * b - a * c;
    if (D < (R)0) D = (R)0;
    const R sq = sqrt(D);
    const R f = (b > (R)0) ? (-c) / (b + sq) : (sq - b) / a;
    if (kind == X_NONE || f < best) {
      best = f;
      kind = X_CYL;
    }
  }
  if (best < (R)0) best = (R)0;
  if (best > (R)1) best = (R)1;
  fout = best;
  return kind;
}

// ---------------------------------------------------------------------------
// Wall / aperture handling with recycling (Sec. II).  Returns the event code
// and updates the particle; tallies are counted by the caller.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void reemit(const KParams &P, uint32_t id, uint32_t step, int s, const R n[3],
                                       const R t1[3], const R t2[3], R &vx, R &vy, R &vz) {
  const uint4 W = draw(P, id, step, S_BND, 0);
  const uint4 V = draw(P, id, step, S_BND, 1);
  const double sg = P.sig_w[s];
  const double vn = sg * sqrt(-2.0 * log(1.0 - u53(W.x, W.y)));
  double na, nb;
  box_muller(u53(W.z, W.w), u53(V.x, V.y), na, nb);
  const R rvn = (R)vn, sa = (R)(sg * na), sb = (R)(sg * nb);
  vx = (rvn * n[0] + sa * t1[0]) + sb * t2[0];
  vy = (rvn * n[1] + sa * t1[1]) + sb * t2[1];
  vz = (rvn * n[2] + sa * t1[2]) + sb * t2[2];
}

// kind: from segment_exit; returns EV_WALL or EV_EXTRACT and sets q_new = 0
template <typename R>
// rc2: squared radius of the crossing point, set for an extraction
__device__ __forceinline__ uint8_t wall_event(const KParams &P, uint32_t id, uint32_t step, int s, int kind,
                                              R f, R x0, R y0, R z0, R &x, R &y, R &z, R &vx, R &vy, R &vz,
                                              R &rc2) {
  const R dx = x - x0, dy = y - y0, dz = z - z0;
  const R xc = x0 + f * dx, yc = y0 + f * dy, zc = z0 + f * dz;
  const R ex[3] = {(R)1, (R)0, (R)0}, ey[3] = {(R)0, (R)1, (R)0};
  const R pz[3] = {(R)0, (R)0, (R)1}, mz[3] = {(R)0, (R)0, (R)-1};
  const R hL = (R)P.hL, eps = (R)kWallEps;
  if (kind == X_EXT && xc * xc + yc * yc <= (R)P.rap2) {
    rc2 = xc * xc + yc * yc;
    x = (R)P.inlet_x;
    y = (R)P.inlet_y;
    z = -hL + eps;
    reemit<R>(P, id, step, s, pz, ex, ey, vx, vy, vz);
    return EV_EXTRACT;
  }
  if (kind == X_EXT) {
    x = xc;
    y = yc;
    z = hL - eps;
    reemit<R>(P, id, step, s, mz, ex, ey, vx, vy, vz);
  } else if (kind == X_INJ) {
    x = xc;
    y = yc;
    z = -hL + eps;
    reemit<R>(P, id, step, s, pz, ex, ey, vx, vy, vz);
  } else {
    const R rc = sqrt(xc * xc + yc * yc);
    const R n[3] = {-xc / rc, -yc / rc, (R)0};
    const R t1[3] = {yc / rc, -xc / rc, (R)0};
    const R sc = ((R)P.R0 - eps) / rc;
    x = xc * sc;
    y = yc * sc;
    z = zc;
    reemit<R>(P, id, step, s, n, t1, pz, vx, vy, vz);
  }
  return EV_WALL;
}

// ---------------------------------------------------------------------------
// Charge exchange outcome (Sec. II): a neutral drawn from a Maxwellian at
// T_n; Q = 1 takes its velocity (resonant), Q >= 3 goes to Q-1 with the
// energy release dE shared equally in the centre-of-mass frame.
// ---------------------------------------------------------------------------
// a background neutral for a collision: Maxwellian at T_n, from calls 0
// and 1 of the given stream
template <typename R>
__device__ __forceinline__ void neutral_partner(const KParams &P, uint32_t id, uint32_t step, uint32_t stream, int s,
                                                R &wx, R &wy, R &wz) {
  const uint4 G = draw(P, id, step, stream, 0);
  const uint4 H = draw(P, id, step, stream, 1);
  double n0, n1, n2, nd;
  box_muller(u53(G.x, G.y), u53(G.z, G.w), n0, n1);
  box_muller(u53(H.x, H.y), u53(H.z, H.w), n2, nd);
  const double sg = P.sig_n[s];
  wx = (R)(sg * n0);
  wy = (R)(sg * n1);
  wz = (R)(sg * n2);
}

// equal masses, isotropic in the centre-of-mass frame: v -> V + (|g'|/2) n,
// |g'|^2 = |v - w|^2 + extra, n from call 2 of the stream
template <typename R>
__device__ __forceinline__ void cm_isotropic(const KParams &P, uint32_t id, uint32_t step, uint32_t stream, R extra,
                                             R wx, R wy, R wz, R &vx, R &vy, R &vz) {
  const uint4 I = draw(P, id, step, stream, 2);
  const double ct = 1.0 - 2.0 * u53(I.x, I.y);
  const double st = sqrt(fmax(0.0, (1.0 - ct) * (1.0 + ct)));
  double sp, cp;
  sincos(2.0 * kPi * u53(I.z, I.w), &sp, &cp);
  const R nxv = (R)(st * cp), nyv = (R)(st * sp), nzv = (R)ct;
  const R gx = vx - wx, gy = vy - wy, gz = vz - wz;
  const R g2 = (gx * gx + gy * gy) + gz * gz + extra;
  const R hg = (R)0.5 * sqrt(g2);
  vx = (vx + wx) * (R)0.5 + hg * nxv;
  vy = (vy + wy) * (R)0.5 + hg * nyv;
  vz = (vz + wz) * (R)0.5 + hg * nzv;
}

// charge exchange with a background neutral (Sec. II): Q = 1 takes the
// neutral's velocity; Q >= 2 shares the release dE in the centre-of-mass frame
template <typename R>
__device__ __forceinline__ void cx_outcome(const KParams &P, uint32_t id, uint32_t step, int s, int Q, R &vx,
                                           R &vy, R &vz) {
  R wx, wy, wz;
  neutral_partner<R>(P, id, step, S_CX, s, wx, wy, wz);
  if (Q == 1) {
    vx = wx;
    vy = wy;
    vz = wz;
    return;
  }
  cm_isotropic<R>(P, id, step, S_CX, (R)P.decx[s], wx, wy, wz, vx, vy, vz);
}

// elastic ion-atom scattering, isotropic in the centre-of-mass frame (Sec. II)
template <typename R>
__device__ __forceinline__ void elastic_outcome(const KParams &P, uint32_t id, uint32_t step, int s, R &vx, R &vy,
                                                R &vz) {
  R wx, wy, wz;
  neutral_partner<R>(P, id, step, S_EL, s, wx, wy, wz);
  cm_isotropic<R>(P, id, step, S_EL, (R)0, wx, wy, wz, vx, vy, vz);
}

// ---------------------------------------------------------------------------
// Square root and log1p for continuous outcomes of a collision (never for a
// decision, which keeps the correctly rounded library operations).
// sqrt: the hardware reciprocal square root refined by two Goldschmidt
// steps (coupled iterations on the root and half its reciprocal), then one
// Newton correction of the root: within an ulp of the correctly rounded root
// at half the library's cost.  Zero, subnormal, huge and non-finite inputs
// take the library path.
// log1p(x) for x in (-1, 0]: y = 1 + x and its rounding error d = x - (y - 1)
// (exact: Sterbenz), y = m 2^e with m in [sqrt(1/2), sqrt(2)), and
// log m = 2 atanh(s), s = (m - 1)/(m + 1), summed as 2 s sum_k z^k/(2k+1),
// z = s^2 <= 0.0295, through k = 11 (truncation below 2^-60 relative);
// log1p x = e ln2 + log m + d/y.  Within 2 ulp of the correctly rounded
// value, at half the library's cost.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double sqrt_cont(double x) {
  if (!(x >= 0x1p-1000 && x <= 0x1p+1000)) return sqrt(x);
  const double h = __builtin_amdgcn_rsq(x);
  double g = x * h, hh = 0.5 * h;
  const double r = fma(-g, hh, 0.5);
  g = fma(g, r, g);
  hh = fma(hh, r, hh);
  const double d = fma(-g, g, x);
  return fma(d, hh, g);
}
__device__ __forceinline__ float sqrt_cont(float x) { return sqrtf(x); }

__device__ __forceinline__ double log1p_cont(double x) {
  const double y = 1.0 + x;
  const double d = x - (y - 1.0);
  int e;
  double m = frexp(y, &e);
  if (m < 0.70710678118654752440) {
    m = m + m;
    e -= 1;
  }
  const double f = m - 1.0;
  const double sv = f / (2.0 + f);
  const double z = sv * sv;
  double p = 2.0 / 23.0;
  p = fma(p, z, 2.0 / 21.0);
  p = fma(p, z, 2.0 / 19.0);
  p = fma(p, z, 2.0 / 17.0);
  p = fma(p, z, 2.0 / 15.0);
  p = fma(p, z, 2.0 / 13.0);
  p = fma(p, z, 2.0 / 11.0);
  p = fma(p, z, 2.0 / 9.0);
  p = fma(p, z, 2.0 / 7.0);
  p = fma(p, z, 2.0 / 5.0);
  p = fma(p, z, 2.0 / 3.0);
  // ln 2 = ln2_hi + ln2_lo, ln2_hi with its low 32 bits zero (e ln2_hi exact)
  constexpr double ln2_hi = 6.93147180369123816490e-01, ln2_lo = 1.90821492927058770002e-10;
  const double de = (double)e;
  const double lm = fma(sv * z, p, 2.0 * sv);
  return fma(de, ln2_hi, lm + fma(de, ln2_lo, d / y));
}

// ---------------------------------------------------------------------------
// Nanbu: 1 - cos(chi) = -log1p(u expm1(-2A))/A with A(s) from the table
// (ln A linear in s between nodes), A = 1/s below 2^-20, isotropic from 8.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double nanbu_A(const double *__restrict__ lnA, double sv) {
  int ex;
  const double m = frexp(sv, &ex);
  const int e = ex - 1;
  const double t = (2.0 * m - 1.0) * (double)kAK;
  const int j = (int)t;
  const double fr = t - (double)j;
  int i = (e - kAeLo) * kAK + j;
  i = i < 0 ? 0 : (i > kANodes - 2 ? kANodes - 2 : i);  // only a non-finite s can leave the range
  const double a = lnA[i], b = lnA[i + 1];
  return exp(a + fr * (b - a));
}

__device__ __forceinline__ double nanbu_omc(const double *__restrict__ lnA, double sv, double u) {
  double omc;
  if (sv >= kSHi) {
    omc = 2.0 * u;
  } else {
    const double A = (sv < kSLo) ? 1.0 / sv : nanbu_A(lnA, sv);
    // for A > 20, exp(-2A) < 5e-18 is below half an ulp of 1, so expm1(-2A)
    // rounds to -1 exactly: skip the call (most pairs of a cool plasma)
    const double em = A > 20.0 ? -1.0 : expm1(-2.0 * A);
    omc = -log1p_cont(u * em) / A;
  }
  omc = omc < 0.0 ? 0.0 : omc;
  omc = omc > 2.0 ? 2.0 : omc;
  return omc;
}

}  // namespace ecr
