// ecr_coll.hpp -- one binary Coulomb collision (Mironov et al., Sec. II):
// Nanbu's scattering angle for the pair's s parameter with a constant
// Coulomb logarithm, and the Takizuka-Abe rotation of the relative velocity.
// Shared by the Coulomb kernels and the fused step kernel; the particles'
// velocities and charges are read and written through `Acc`, an accessor of
// either the global structure of arrays or a workgroup's LDS copy.
#pragma once

#include "ecr_kernels.hpp"

namespace ecr {

// velocities and charge states in the global structure of arrays
template <typename R>
struct SoaAcc {
  Soa<R> S;
  __device__ __forceinline__ R &vx(uint32_t i) const { return S.vx[i]; }
  __device__ __forceinline__ R &vy(uint32_t i) const { return S.vy[i]; }
  __device__ __forceinline__ R &vz(uint32_t i) const { return S.vz[i]; }
  __device__ __forceinline__ uint8_t qs(uint32_t i) const { return S.qs[i]; }
};

// one binary collision of slots ia, ib with time step dtp and pool density
// nc; acc gathers the momentum / energy change and the energy of the pool
// before (count_e0_*: count this member's energy)
template <typename R, typename Acc>
__device__ __forceinline__ void collide_acc(const KParams &P, const double *__restrict__ lnA, const Acc &S, uint32_t ia,
                                        uint32_t ib, uint32_t id_a, double nc, double dtp, uint32_t step,
                                        double acc[5], bool count_e0_a, bool count_e0_b) {
  const uint4 W = draw(P, id_a, step, S_COUL, 0);
  const double u = u53(W.x, W.y), u2 = u53(W.z, W.w);
  const R vax = S.vx(ia), vay = S.vy(ia), vaz = S.vz(ia);
  const R vbx = S.vx(ib), vby = S.vy(ib), vbz = S.vz(ib);
  const uint8_t qa = S.qs(ia), qb = S.qs(ib);
  const int sa = sp_of(qa), sb = sp_of(qb);
  const double ma = P.mass[sa], mb = P.mass[sb];
  const double ea = 0.5 * ma * (double)((vax * vax + vay * vay) + vaz * vaz);
  const double eb = 0.5 * mb * (double)((vbx * vbx + vby * vby) + vbz * vbz);
  if (count_e0_a) acc[4] += ea;
  if (count_e0_b) acc[4] += eb;
  const R ux = vax - vbx, uy = vay - vby, uz = vaz - vbz;
  const R g2 = (ux * ux + uy * uy) + uz * uz;
  if (g2 == (R)0) return;
  const R g = sqrt_cont(g2);
  const double mu = P.mu[sa][sb];  // (ma mb) / (ma + mb), tabulated on the host
  const double qq = (double)q_of(qa) * (double)q_of(qb);
  const double num = ((P.Cs * (qq * qq)) * nc) * dtp;
  const double den = (mu * mu) * ((double)g2 * (double)g);
  const double sv = num / den;
  const R omc = (R)nanbu_omc(lnA, sv, u);
  const R sinchi = sqrt_cont(omc * ((R)2 - omc));
  R sp, cp;
  sincos_2pi(u2, &sp, &cp);  // phi = 2 pi u2
  const R ca = sinchi * cp, cb = sinchi * sp;
  const R uperp = sqrt_cont(ux * ux + uy * uy);
  R dux, duy, duz;
  if (uperp > (R)0) {
    const R iu = (R)1 / uperp;
    const R cx = ux * iu, cy = uy * iu;  // within an ulp of ux/uperp, uy/uperp
    dux = ((cx * uz) * ca - (cy * g) * cb) - ux * omc;
    duy = ((cy * uz) * ca + (cx * g) * cb) - uy * omc;
    duz = -(uperp * ca) - uz * omc;
  } else {
    dux = g * ca;
    duy = g * cb;
    duz = -(g * omc);
  }
  const R ra = (R)P.mra[sa][sb], rb = (R)P.mrb[sa][sb];  // mu / ma, mu / mb
  const R nax = vax + ra * dux, nay = vay + ra * duy, naz = vaz + ra * duz;
  const R nbx = vbx - rb * dux, nby = vby - rb * duy, nbz = vbz - rb * duz;
  S.vx(ia) = nax;
  S.vy(ia) = nay;
  S.vz(ia) = naz;
  S.vx(ib) = nbx;
  S.vy(ib) = nby;
  S.vz(ib) = nbz;
  acc[0] += ma * (double)(nax - vax) + mb * (double)(nbx - vbx);
  acc[1] += ma * (double)(nay - vay) + mb * (double)(nby - vby);
  acc[2] += ma * (double)(naz - vaz) + mb * (double)(nbz - vbz);
  const double ea1 = 0.5 * ma * (double)((nax * nax + nay * nay) + naz * naz);
  const double eb1 = 0.5 * mb * (double)((nbx * nbx + nby * nby) + nbz * nbz);
  acc[3] += (ea1 - ea) + (eb1 - eb);
}

template <typename R>
__device__ __forceinline__ void collide(const KParams &P, const double *__restrict__ lnA, Soa<R> S, uint32_t ia,
                                        uint32_t ib, uint32_t id_a, double nc, double dtp, uint32_t step,
                                        double acc[5], bool count_e0_a, bool count_e0_b) {
  collide_acc<R>(P, lnA, SoaAcc<R>{S}, ia, ib, id_a, nc, dtp, step, acc, count_e0_a, count_e0_b);
}

}  // namespace ecr
