// ecr_push.hpp -- per-particle device code of the ion step (Mironov et al.,
// Sec. II), shared by the push kernels and the fused step kernel: the
// electron-ion heating kick, the advance of one particle (push, wall and
// aperture loss, ionisation / charge exchange / elastic scattering), and the
// cloud-in-cell deposit of a staged tile through an LDS brick.
#pragma once

#include "ecr_kernels.hpp"
#include "ecr_wave.hpp"

namespace ecr {

constexpr int kP = 4;                // consecutive slots per lane
constexpr int kBlock = 256;          // lanes per workgroup
constexpr int kTile = kBlock * kP;   // slots per workgroup
constexpr int kBrickNodes = 1536;    // LDS brick capacity in nodes (x 3 fields)

// ---------------------------------------------------------------------------
// Electron-ion heating and diffusion (Sec. II): dV = D (R + delta) |R| /
// |R + delta| with D^2 = n_e x dheat[s][zone][Q] and R uniform in the cube
// [-1/2, 1/2]^3 (three words of one draw of the heating stream).  With the
// cell charge grid (self-consistent electrons) n_e is the ion's cell's and
// delta the electron diamagnetic bias: the 9-point stencil of the cell
// density in the ion's z plane (cells beyond the mesh count as empty) times
// -R_L / n_e(cell), R_L = 2.38e-6 sqrt(T_e) / (|B(cell centre)| hx); a cell
// without charge gives no kick.  With the fixed background, n_e is the
// zone's and, the background being uniform, delta = 0; ECR_FLAG_HEAT_ISOTROPIC
// also sets delta = 0 (the isotropic-heating ablation).  The kick is
// evaluated in binary64 whatever R; the neighbours' loads hit the cache
// lines the lanes of a cell share (slots are in cell order).
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void heat_kick(const KParams &P, const Tables *__restrict__ T, uint32_t id, uint32_t step,
                                          int s, int Q, R x, R y, R z, R &vx, R &vy, R &vz,
                                          const uint32_t *__restrict__ chg) {
  const int zone = (((x * x) * (R)P.ia2 + (y * y) * (R)P.ia2) + (z * z) * (R)P.ic2) < (R)1;
  double ne, dlx = 0.0, dly = 0.0;
  if (P.flags & ECR_FLAG_SELF_NE) {
    const int ix = clampi((int)floor((x + (R)P.R0) * (R)P.idx), 0, P.nx - 1);
    const int iy = clampi((int)floor((y + (R)P.R0) * (R)P.idy), 0, P.ny - 1);
    const int iz = clampi((int)floor((z + (R)P.hL) * (R)P.idz), 0, P.nz - 1);
    const uint32_t plane = (uint32_t)P.nx * (uint32_t)P.ny * (uint32_t)iz;
    auto nat = [&](int jx, int jy) -> double {
      if (jx < 0 || jx >= P.nx || jy < 0 || jy >= P.ny) return 0.0;
      return P.nfac * (double)chg[plane + (uint32_t)jx + (uint32_t)P.nx * (uint32_t)jy];
    };
    ne = nat(ix, iy);
    if (!(ne > 0.0)) return;
    // |B| at the cell centre times the cell size, tabulated per cell when
    // the run is created (cell_bden)
    const double den = P.bden[plane + (uint32_t)ix + (uint32_t)P.nx * (uint32_t)iy];
    if (den > 0.0 && !(P.flags & ECR_FLAG_HEAT_ISOTROPIC)) {
      const double rl = P.rl_zone[zone] / den;
      const double nmm = nat(ix - 1, iy - 1), nzm = nat(ix, iy - 1), npm = nat(ix + 1, iy - 1);
      const double nmz = nat(ix - 1, iy), npz = nat(ix + 1, iy);
      const double nmp = nat(ix - 1, iy + 1), nzp = nat(ix, iy + 1), npp = nat(ix + 1, iy + 1);
      const double gy = (-nzp + nzm) + 0.5 * (((-nmp - npp) + npm) + nmm);
      const double gx = (-nmz + npz) + 0.5 * (((-nmp + npp) + npm) - nmm);
      dlx = -(rl / ne) * gy;
      dly = -(rl / ne) * gx;
    }
  } else {
    ne = P.ne_zone[zone];
    if (!(ne > 0.0)) return;
  }
  const double D = sqrt(ne * T->dheat[s][zone][Q]);
  const uint4 W = draw(P, id, step, S_HEAT, 0);
  constexpr double k2m32 = 2.3283064365386962890625e-10;  // 2^-32
  const double rx = ((double)W.x + 0.5) * k2m32 - 0.5;
  const double ry = ((double)W.y + 0.5) * k2m32 - 0.5;
  const double rz = ((double)W.z + 0.5) * k2m32 - 0.5;
  const double sx = rx + dlx, sy = ry + dly, sz = rz;
  const double nr = sqrt((rx * rx + ry * ry) + rz * rz);
  const double ns = sqrt((sx * sx + sy * sy) + sz * sz);
  if (!(ns > 0.0)) return;
  const double f = (D * nr) / ns;
  vx = (R)((double)vx + f * sx);
  vy = (R)((double)vy + f * sy);
  vz = (R)((double)vz + f * sz);
}

// ---------------------------------------------------------------------------
// One particle: push -> wall/aperture -> heating kick -> ionisation (Q -> Q+n)
// / charge exchange / elastic ion-atom scattering.
// Tallies are rare events (~1e-4 per particle-step) and go straight to
// 64-bit global atomics; so do the loss diagnostics (first-passage times,
// crossing radius, lost kinetic energy), and the particle's birth step
// (birth[j]) is read or written only on such events.  Returns the event code.
// ---------------------------------------------------------------------------
// EXT: the kernel variant with the optional physics (self-consistent
// electrons, heating kick, multiple ionisation, elastic scattering); the
// default step runs the lean variant, which leaves those paths out of the
// code altogether
// the processes that consume the STEP draw's uniform
__device__ __forceinline__ bool needs_mcc_uniform(const KParams &P) {
  return (P.pmask & (P_IONIZE | P_CX | P_ELASTIC)) != 0;
}

// birth[j]: the particle's birth step; P.cellid[jc]: its collision cell.
// u: the particle's Monte-Carlo uniform of the step, u53 of words 0 and 1 of
// its STEP draw (the caller draws it once; its word 2 is the Coulomb pairing
// key of the same step)
template <typename R, int FLD, bool EXT>
__device__ __forceinline__ uint8_t advance(const KParams &P, const Tables *__restrict__ T,
                                           const double *__restrict__ ef, DevAccum *__restrict__ acc, uint32_t step,
                                           uint32_t id, int s, int &Q, R &x, R &y, R &z, R &vx, R &vy, R &vz,
                                           uint32_t *__restrict__ birth, int64_t j, int64_t jc,
                                           const uint32_t *__restrict__ chg, double u) {
  uint8_t ev = EV_NONE;
  if (P.pmask & P_PUSH) {
    const R x0 = x, y0 = y, z0 = z;
    const R h = (R)T->qmh[s][Q];
    R E[3] = {(R)0, (R)0, (R)0};
    if (FLD & 1) gather_E<R>(P, ef, x, y, z, E);
    boris<R, FLD>(P, h, E, x, y, z, vx, vy, vz);
    R f;
    const int kind = segment_exit<R>(P, x0, y0, z0, x, y, z, f);
    if (kind != X_NONE) {
      if (Q >= 1) {
        const double ke = 0.5 * P.mass[s] * (double)((vx * vx + vy * vy) + vz * vz);
        unsafeAtomicAdd(&acc->t.lost_ke[s], ke);
      }
      R rc2 = (R)0;
      ev = wall_event<R>(P, id, step, s, kind, f, x0, y0, z0, x, y, z, vx, vy, vz, rc2);
      if (ev == EV_EXTRACT) {
        atomicAdd((unsigned long long *)&acc->t.extracted[s][Q], 1ull);
        atomicAdd((unsigned long long *)&acc->t.recycled, 1ull);
        unsafeAtomicAdd(&acc->t.extracted_r[s][Q], (double)sqrt(rc2));
        const uint32_t b = birth[j];
        if (Q >= 1 && b != kBirthNone) {
          const uint32_t t = step - b;
          atomicAdd((unsigned long long *)&acc->t.fpt_n[s][Q], 1ull);
          atomicAdd((unsigned long long *)&acc->t.fpt_sum[s][Q], (unsigned long long)t);
          atomicAdd((unsigned long long *)&acc->t.fpt_hist[s][fpt_bin(t)], 1ull);
        }
      } else {
        atomicAdd((unsigned long long *)&acc->t.wall[s][Q], 1ull);
      }
      // now an atom; with exchange partners an atom's birth is the step it
      // became one, so that it is no partner in this step
      if (EXT && (P.flags & ECR_FLAG_CX_PARTNER)) birth[j] = step;
      else if (Q >= 1) birth[j] = kBirthNone;
      Q = 0;
    }
  }
  if (EXT && ev == EV_NONE && (P.pmask & P_HEAT) && Q >= 1)
    heat_kick<R>(P, T, id, step, s, Q, x, y, z, vx, vy, vz, chg);
  if (!EXT && ev == EV_NONE && (P.pmask & (P_IONIZE | P_CX))) {
    const int zone = (((x * x) * (R)P.ia2 + (y * y) * (R)P.ia2) + (z * z) * (R)P.ic2) < (R)1;
    // single ionisation with the fixed background, then charge exchange
    const double pi = (P.pmask & P_IONIZE) ? T->pion[s][zone][Q] : 0.0;
    double pc = 0.0;
    if ((P.pmask & P_CX) && ((P.cxok[s] >> Q) & 1u)) {
      const R sp2 = (vx * vx + vy * vy) + vz * vz;
      pc = (P.ccx[s] * (double)Q) * (double)sqrt(sp2);
    }
    const double pt = pi + pc;
    if (pt > 0.1) atomicAdd((unsigned long long *)&acc->t.anomalies, 1ull);
    if (u < pi) {
      atomicAdd((unsigned long long *)&acc->t.ionized[s][Q], 1ull);
      atomicAdd((unsigned long long *)&acc->t.ionized_n[s][0], 1ull);
      if (Q == 0) birth[j] = step;  // an ion is made from an atom
      Q = Q + 1;
      ev = EV_IONIZE;
    } else if (u < pt) {
      atomicAdd((unsigned long long *)&acc->t.cx[s][Q], 1ull);
      if (Q == 1) birth[j] = step;  // resonant exchange: the ion is the former neutral
      cx_outcome<R>(P, id, step, s, Q, vx, vy, vz);
      if (Q >= 2) {
        Q = Q - 1;
        atomicAdd((unsigned long long *)&acc->t.cx_products[s], 1ull);
      }
      ev = EV_CX;
    }
  }
  if (EXT && ev == EV_NONE && (P.pmask & (P_IONIZE | P_CX | P_ELASTIC))) {
    const int zone = (((x * x) * (R)P.ia2 + (y * y) * (R)P.ia2) + (z * z) * (R)P.ic2) < (R)1;
    // ionisation channels Q -> Q+n: the fixed background's tabulated
    // probabilities, or with ECR_FLAG_SELF_NE n_e k dt, n_e = weight x (ion
    // charge of the cell at the start of the step) / cell volume.  One
    // uniform picks the channel by running sums: ionisation n = 1..4, then
    // charge exchange, then elastic scattering.
    const bool self_ne = (P.flags & ECR_FLAG_SELF_NE) != 0;
    double pi = 0.0, ne = 0.0;
    if (P.pmask & P_IONIZE) {
      if (self_ne) {
        ne = P.nfac * (double)chg[cell_of<R>(P, x, y, z)];
        pi = ne * T->kdt[s][zone][Q];
      } else {
        pi = T->pion[s][zone][Q];
      }
    }
    double c2 = pi, c3 = pi, c4 = pi;  // running sums through n = 2, 3, 4
    if ((P.pmask & P_IONIZE) && P.nion > 1) {
      const double p2 = self_ne ? ne * T->kmul[s][zone][0][Q] : T->pmul[s][zone][0][Q];
      const double p3 = self_ne ? ne * T->kmul[s][zone][1][Q] : T->pmul[s][zone][1][Q];
      const double p4 = self_ne ? ne * T->kmul[s][zone][2][Q] : T->pmul[s][zone][2][Q];
      c2 = pi + p2;
      c3 = c2 + p3;
      c4 = c3 + p4;
    }
    const bool cxon = (P.pmask & P_CX) && ((P.cxok[s] >> Q) & 1u);
    const bool elon = (P.pmask & P_ELASTIC) != 0;
    double speed = 0.0;
    if (cxon || elon) {
      const R sp2 = (vx * vx + vy * vy) + vz * vz;
      speed = (double)sqrt(sp2);
    }
    // neutral partners: the species' uniform n0, or with ECR_FLAG_SELF_N0
    // weight x (atoms of the species in the cell at the start of the step) / cell volume
    double ccx = P.ccx[s], cel = P.cel[s];
    if ((P.flags & ECR_FLAG_SELF_N0) && (cxon || elon)) {
      const double n0c = P.nfac * (double)chg[(uint32_t)(1 + s) * P.ncell + cell_of<R>(P, x, y, z)];
      ccx = n0c * P.sdt_cx[s];
      cel = n0c * P.sdt_el[s];
    }
    double pc = 0.0;
    if (cxon) pc = (ccx * (double)Q) * speed;
    const double pt = c4 + pc;
    const double pall = elon ? pt + (cel * (double)Q) * speed : pt;
    if (pall > 0.1) atomicAdd((unsigned long long *)&acc->t.anomalies, 1ull);
    if (u < c4) {
      const int n = u < pi ? 1 : (u < c2 ? 2 : (u < c3 ? 3 : 4));
      atomicAdd((unsigned long long *)&acc->t.ionized[s][Q], 1ull);
      atomicAdd((unsigned long long *)&acc->t.ionized_n[s][n - 1], 1ull);
      if (Q == 0) birth[j] = step;  // an ion is made from an atom
      Q = Q + n;
      ev = EV_IONIZE;
    } else if (u < pt) {
      atomicAdd((unsigned long long *)&acc->t.cx[s][Q], 1ull);
      ev = EV_CX;
      if (P.flags & ECR_FLAG_CX_PARTNER) {
        // the electron comes from a tracked atom of the collision cell,
        // picked at the end of the step; a Q = 1 ion is an atom from now
        // on and keeps its velocity
        const uint32_t cc = P.cellid[jc];
        atomicAdd(&P.cxreq[(uint32_t)s * P.ncell + cc], 1u);
        // the chunk owning the cell: the one its first slot falls in
        P.cxchunk[P.cell_off[cc] / (uint32_t)kCoulCap] = 1u;
        if (Q == 1) {
          birth[j] = step;
          Q = 0;
        }
      }
      if (Q >= 1) {
        if (Q == 1) birth[j] = step;  // resonant exchange: the ion is the former neutral
        cx_outcome<R>(P, id, step, s, Q, vx, vy, vz);
        if (Q >= 2) {
          Q = Q - 1;
          atomicAdd((unsigned long long *)&acc->t.cx_products[s], 1ull);
        }
      }
    } else if (u < pall) {
      atomicAdd((unsigned long long *)&acc->t.elastic[s][Q], 1ull);
      elastic_outcome<R>(P, id, step, s, vx, vy, vz);
      ev = EV_ELASTIC;
    }
  }
  if (!(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(vx) && isfinite(vy) && isfinite(vz)))
    atomicAdd((unsigned long long *)&acc->t.anomalies, 1ull);
  return ev;
}

// ---------------------------------------------------------------------------
// Cloud-in-cell deposit of a tile onto the (nx+1)(ny+1)(nz+1) node grid:
// fields ion number (Q >= 1), ion charge (Q x weight) and atom number
// (Q = 0), as enabled by the deposit mask.
//
// The push works on coalesced slots (lane = slot, kP rounds of 256).  Its
// deposit inputs (lower node, fractional offsets, charge) are staged in LDS
// and read back transposed, so that lane l owns the kP consecutive slots
// kP*l .. kP*l+kP-1.  Consecutive slots share a cell almost always, so the
// lane sums their weights in registers and flushes a run only when the cell
// changes, into an LDS brick spanning the tile's nodes.  The lanes' last runs
// go through a segmented sum over the wavefront, so only the last lane of
// each run of equal cells touches the brick; the brick goes to HBM with one
// FP64 atomic per touched node.  A tile whose nodes do not fit the brick
// (one spanning two planes of cells) sends the same wavefront sums to HBM.
// ---------------------------------------------------------------------------
constexpr int kPad(int i) { return i + (i >> 2); }  // one pad slot every 4: fewer LDS bank conflicts
constexpr int kStage = kPad(kTile);

// unpadded: the push writes one slot per lane (consecutive addresses), and
// lane l reads its kP consecutive slots back with wide loads, both free of
// bank conflicts; 31 KB in binary64, so that five workgroups share a CU
// TILE: slots of a staged tile (kP per lane of the workgroup)
template <typename R, int TILE = kTile>
struct alignas(16) DepStage {
  R t[3][TILE];
  uint16_t c[3][TILE];
  uint8_t q[TILE];  // charge, or 0xFF: nothing to deposit
};

// the brick reuses the staging memory: as many doubles as binary64 staging holds
template <int TILE>
constexpr int dep_brick() {
  return (int)(sizeof(DepStage<double, TILE>) / sizeof(double));
}
constexpr int kDepBrick = dep_brick<kTile>();

template <typename R, int TILE = kTile>
union DepShared {
  DepStage<R, TILE> st;
  double brick[dep_brick<TILE>()];
};

// kP consecutive staged values of lane l (16-byte aligned: kP = 4)
__device__ __forceinline__ void lds_load4(const double *p, double o[4]) {
  const double2 a = reinterpret_cast<const double2 *>(p)[0], b = reinterpret_cast<const double2 *>(p)[1];
  o[0] = a.x;
  o[1] = a.y;
  o[2] = b.x;
  o[3] = b.y;
}
__device__ __forceinline__ void lds_load4(const float *p, float o[4]) {
  const float4 a = *reinterpret_cast<const float4 *>(p);
  o[0] = a.x;
  o[1] = a.y;
  o[2] = a.z;
  o[3] = a.w;
}

template <typename R>
struct DepIn {
  int ix[kP], iy[kP], iz[kP], q[kP];
  R tx[kP], ty[kP], tz[kP];
  bool on[kP];
};

// sum the runs of equal base node held by this lane; flush(node, field, corner, value)
// the last run of a lane, handed to the wavefront reduction (node -1: none)
struct DepRun {
  int64_t node;
  double a[8], b[8], c[8];
};

// CARRY: the lane's last run is returned in `last` instead of flushed
template <typename R, bool CARRY, typename NodeOf, typename Flush>
__device__ __forceinline__ void run_accumulate(const DepIn<R> &D, uint32_t dm, NodeOf nodeof, Flush flush,
                                               DepRun &last) {
  double a[8], b[8], c[8];
  int64_t cur = -1;
  bool has_ion = false, has_atom = false;
  for (int k = 0; k < 8; ++k) a[k] = b[k] = c[k] = 0.0;
  auto emit = [&]() {
    if (cur < 0) return;
    for (int k = 0; k < 8; ++k) {
      if (has_ion && (dm & 1u)) flush(cur, 0, k, a[k]);
      if (has_ion && (dm & 2u)) flush(cur, 1, k, b[k]);
      if (has_atom && (dm & 4u)) flush(cur, 2, k, c[k]);
    }
  };
#pragma unroll
  for (int p = 0; p < kP; ++p) {
    if (!D.on[p]) continue;
    const int64_t node = nodeof(D.ix[p], D.iy[p], D.iz[p]);
    if (node != cur) {
      emit();
      cur = node;
      has_ion = has_atom = false;
      for (int k = 0; k < 8; ++k) a[k] = b[k] = c[k] = 0.0;
    }
    const R wx[2] = {(R)1 - D.tx[p], D.tx[p]}, wy[2] = {(R)1 - D.ty[p], D.ty[p]};
    const R wz[2] = {(R)1 - D.tz[p], D.tz[p]};
    const bool ion = (dm & 4u) ? D.q[p] >= 1 : true;  // without the atom field only ions are staged
    const double qd = (double)D.q[p];
    int k = 0;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx, ++k) {
          const double w = (double)((wx[dx] * wy[dy]) * wz[dz]);
          if (ion) {
            a[k] += w;
            b[k] += qd * w;
          } else {
            c[k] += w;
          }
        }
    has_ion |= ion;
    has_atom |= !ion;
  }
  if (CARRY) {
    last.node = cur;
    for (int k = 0; k < 8; ++k) {
      last.a[k] = a[k];
      last.b[k] = b[k];
      last.c[k] = c[k];
    }
  } else {
    emit();
  }
}

// stage the deposit input of tile slot i (lane = slot layout)
// NQ: the deposit mask is known to hold exactly the ion number and ion
// charge fields (the default); the atom-field paths then compile away
template <typename R, bool NQ, int TILE = kTile>
__device__ __forceinline__ void stage_cic(const KParams &P, DepStage<R, TILE> &st, int i, R x, R y, R z, int q, int mn[3],
                                          int mx[3]) {
  int ix, iy, iz;
  R tx, ty, tz;
  cic_axis<R>(x, (R)P.R0, (R)P.idx, P.nx, ix, tx);
  cic_axis<R>(y, (R)P.R0, (R)P.idy, P.ny, iy, ty);
  cic_axis<R>(z, (R)P.hL, (R)P.idz, P.nz, iz, tz);
  const uint32_t dm = NQ ? 3u : P.dmask;
  const bool on = (q >= 1) ? (dm & 3u) != 0 : (dm & 4u) != 0;
  const int k = i;
  st.t[0][k] = tx;
  st.t[1][k] = ty;
  st.t[2][k] = tz;
  st.c[0][k] = (uint16_t)ix;
  st.c[1][k] = (uint16_t)iy;
  st.c[2][k] = (uint16_t)iz;
  st.q[k] = on ? (uint8_t)q : (uint8_t)0xFF;
  if (on) {
    mn[0] = min(mn[0], ix);
    mn[1] = min(mn[1], iy);
    mn[2] = min(mn[2], iz);
    mx[0] = max(mx[0], ix);
    mx[1] = max(mx[1], iy);
    mx[2] = max(mx[2], iz);
  }
}

// exact i / d for 0 <= i < 2^22 and 0 < d < 2^22 (d uniform, rcp = 1/d in
// binary32): the binary32 estimate is within one of the quotient
__device__ __forceinline__ int small_div(int i, int d, float rcp) {
  int q = (int)((float)i * rcp);
  q = (q + 1) * d <= i ? q + 1 : q;
  q = q * d > i ? q - 1 : q;
  return q;
}

// the box of base cells of a tile: each wavefront's last lane writes the
// wavefront's min / max into the wavefront's own six entries of box (6 ints
// per wavefront of the workgroup: no atomics, nothing to clear first);
// after a barrier every lane reduces them (uniform reads, scalar results)
__device__ __forceinline__ void box_publish(int *box, int mn[3], int mx[3]) {
  wave_box_last(mn, mx);
  if ((threadIdx.x & 63) == 63) {
    int *b = box + 6 * (threadIdx.x >> 6);
    for (int d = 0; d < 3; ++d) {
      b[d] = mn[d];
      b[3 + d] = mx[d];
    }
  }
}

template <int NT>
__device__ __forceinline__ void box_reduce(const int *box, int out[6]) {
  for (int d = 0; d < 6; ++d) out[d] = box[d];
  for (int w = 1; w < NT / 64; ++w)
    for (int d = 0; d < 3; ++d) {
      out[d] = min(out[d], box[6 * w + d]);
      out[3 + d] = max(out[3 + d], box[6 * w + 3 + d]);
    }
  for (int d = 0; d < 6; ++d) out[d] = __builtin_amdgcn_readfirstlane(out[d]);
}

// deposit a staged tile; every lane of the workgroup must call it.  G: the
// lanes' last runs are summed within groups of G lanes (G = 64: over the
// whole wavefront) before the run's last lane in the group flushes them
template <typename R, bool NQ, int G = 64, int NT = kBlock>
__device__ __forceinline__ void deposit_staged(const KParams &P, double *__restrict__ dens, DepShared<R, NT * kP> &sh,
                                               int *box, int mn[3], int mx[3]) {
  constexpr int kBrickCap = dep_brick<NT * kP>();
  const int tid = threadIdx.x;
  const uint32_t dm = NQ ? 3u : P.dmask;
  constexpr int kFields = NQ ? 2 : 3;  // brick fields
  box_publish(box, mn, mx);
  __syncthreads();  // staging and box complete
  static_assert(kP == 4, "the wide staging reads take four slots");
  DepIn<R> D;
  {
    const int k0 = tid * kP;
    lds_load4(&sh.st.t[0][k0], D.tx);
    lds_load4(&sh.st.t[1][k0], D.ty);
    lds_load4(&sh.st.t[2][k0], D.tz);
    const uint32_t q4 = *reinterpret_cast<const uint32_t *>(&sh.st.q[k0]);
    uint2 c4[3];
    for (int a = 0; a < 3; ++a) c4[a] = *reinterpret_cast<const uint2 *>(&sh.st.c[a][k0]);
#pragma unroll
    for (int p = 0; p < kP; ++p) {
      const uint8_t q = (uint8_t)(q4 >> (8 * p));
      D.on[p] = q != 0xFF;
      D.q[p] = q;
      const int sh16 = 16 * (p & 1);
      D.ix[p] = (int)(((p < 2 ? c4[0].x : c4[0].y) >> sh16) & 0xffffu);
      D.iy[p] = (int)(((p < 2 ? c4[1].x : c4[1].y) >> sh16) & 0xffffu);
      D.iz[p] = (int)(((p < 2 ? c4[2].x : c4[2].y) >> sh16) & 0xffffu);
    }
  }
  // the box is the same for every lane: keep it in scalar registers
  int bb[6];
  box_reduce<NT>(box, bb);
  const int x0 = bb[0], y0 = bb[1], z0 = bb[2];
  const bool any = bb[3] >= 0;
  const int bx = bb[3] - x0 + 2, by = bb[4] - y0 + 2, bz = bb[5] - z0 + 2;
  __syncthreads();  // staging read: the brick may now reuse it
  if (!any) return;
  const int64_t nodes = (int64_t)bx * by * bz;
  // the lanes' last runs: summed over runs of lanes (the whole wavefront,
  // or groups of G lanes), then the last lane of each run flushes
  auto flush_last = [&](DepRun &L, auto &&flush) {
    const int key = (int)L.node;
    int seg;
    bool tail;
    wave_runs(key, seg, tail);
    if constexpr (G == 64) {
      const SegSteps st = seg_steps(seg);
      const bool out = tail && key >= 0;
      for (int k = 0; k < 8; ++k) {
        if (dm & 1u) {
          const double v = seg_scan(st, L.a[k]);
          if (out && v != 0.0) flush(key, 0, k, v);
        }
        if (dm & 2u) {
          const double v = seg_scan(st, L.b[k]);
          if (out && v != 0.0) flush(key, 1, k, v);
        }
        if (dm & 4u) {
          const double v = seg_scan(st, L.c[k]);
          if (out && v != 0.0) flush(key, 2, k, v);
        }
      }
    } else {
      const GroupSteps<G> st = group_steps<G>(seg);
      const bool out = (tail || (threadIdx.x & (G - 1)) == G - 1) && key >= 0;
      for (int k = 0; k < 8; ++k) {
        if (dm & 1u) {
          const double v = group_scan<G>(st, L.a[k]);
          if (out && v != 0.0) flush(key, 0, k, v);
        }
        if (dm & 2u) {
          const double v = group_scan<G>(st, L.b[k]);
          if (out && v != 0.0) flush(key, 1, k, v);
        }
        if (dm & 4u) {
          const double v = group_scan<G>(st, L.c[k]);
          if (out && v != 0.0) flush(key, 2, k, v);
        }
      }
    }
  };
  if (nodes <= kBrickCap / kFields) {
    const int nb = (int)nodes;
    for (int i = tid; i < kFields * nb; i += NT) sh.brick[i] = 0.0;
    __syncthreads();
    double *br = sh.brick;
    // corner k of a cell is node base + dx + bx (dy + by dz)
    const int cyz = bx * by;
    auto to_brick = [&](int64_t base, int f, int k, double v) {
      const int dx = k & 1, dy = (k >> 1) & 1, dz = k >> 2;
      atomicAdd(&br[f * nb + (int)base + (dx + (dy ? bx : 0) + (dz ? cyz : 0))], v);
    };
    DepRun L;
    run_accumulate<R, true>(
        D, dm,
        [&](int ix, int iy, int iz) -> int64_t { return (int64_t)((ix - x0) + bx * ((iy - y0) + by * (iz - z0))); },
        to_brick, L);
    flush_last(L, to_brick);
    __syncthreads();
    const float rnb = 1.0f / (float)nb, rbx = 1.0f / (float)bx, rby = 1.0f / (float)by;
    for (int i = tid; i < kFields * nb; i += NT) {
      const double v = sh.brick[i];
      if (v != 0.0) {
        const int f = small_div(i, nb, rnb), li = i - f * nb;
        const int t = small_div(li, bx, rbx), lx = li - t * bx;
        const int lz = small_div(t, by, rby), ly = t - lz * by;
        const int64_t node = (int64_t)(x0 + lx) + (int64_t)P.nx1 * ((y0 + ly) + (int64_t)P.ny1 * (z0 + lz));
        unsafeAtomicAdd(&dens[(int64_t)f * P.nnode + node], v);
      }
    }
  } else {
    // a tile whose nodes do not fit the brick (typically one that spans two
    // planes of cells): runs go to HBM, still summed over the wavefront
    // first, so that the dense cells at either end take a few atomics each
    const int nx1 = P.nx1, ny1 = P.ny1;
    auto to_hbm = [&](int64_t base, int f, int k, double v) {
      const int dx = k & 1, dy = (k >> 1) & 1, dz = k >> 2;
      unsafeAtomicAdd(&dens[(int64_t)f * P.nnode + base + dx + (int64_t)nx1 * (dy + (int64_t)ny1 * dz)], v);
    };
    DepRun L;
    run_accumulate<R, true>(
        D, dm, [&](int ix, int iy, int iz) -> int64_t { return (int64_t)ix + (int64_t)nx1 * (iy + (int64_t)ny1 * iz); },
        to_hbm, L);
    flush_last(L, to_hbm);
  }
}


// a lane's contribution to the next step's cell grids (chg_next: the ion
// charge Q in channel 0, or one atom in its species' channel): lanes hold
// consecutive slots, mostly of one cell, so the last lane of each run of
// equal entries adds the run's sum with one atomic
__device__ __forceinline__ void add_charge(uint32_t *__restrict__ chg, uint32_t cell, uint32_t q) {
  int seg;
  bool tail;
  wave_runs((int64_t)cell, seg, tail);
  q = seg_scan(seg_steps(seg), q);
  if (tail && cell != 0xffffffffu && q != 0u) atomicAdd(&chg[cell], q);
}

// DEP: 0 no deposit, 1 deposit with the run's mask, 2 deposit of exactly the

}  // namespace ecr
