// k_coulomb.hip -- ion-ion Coulomb scattering (Mironov et al., Sec. II):
// Takizuka-Abe random pairing of the ions of each collision cell, Nanbu's
// scattering angle with a constant Coulomb logarithm.
//
// Pairing rule: the pool of a cell is every slot sorted into it at the last
// sort whose charge is Q >= 1; it is ordered by a 32-bit key drawn per
// particle and step (word 2 of the STEP draw), ties by particle id.  An even
// pool pairs (0,1),(2,3),...; an odd pool first does (0,1),(1,2),(2,0) with
// dt/2 each, in that order, then (3,4),...  Each pair draws its two uniforms
// from the COUL stream of its first member.
//
// GPU mapping: workgroup b owns the cells whose first slot lies in
// [b*kCoulCap, (b+1)*kCoulCap) (found by binary search on cell_off, so no
// chunk table is needed).  It sorts the composite keys
// (cell, not-in-pool, random key, id) of its slots in LDS with a bitonic
// network, which groups each pool in pairing order; pools are then found by
// binary search in the sorted keys, and one lane per pair (or per triplet)
// applies the collision to the velocities in HBM.  Pairs are disjoint, so no
// two lanes touch the same particle.
#include "ecr_kernels.hpp"

namespace ecr {

template <typename R>
struct PairAcc {
  double dp[3];
  double de;
  double e0;
};

// one binary collision of slots ia, ib with time step dtp and pool density nc
template <typename R>
__device__ __forceinline__ void collide(const KParams &P, const Tables *__restrict__ T, Soa<R> S, uint32_t ia,
                                        uint32_t ib, uint32_t id_a, double nc, double dtp, uint32_t step,
                                        double acc[5], bool count_e0_a, bool count_e0_b) {
  const uint4 W = draw(P, id_a, step, S_COUL, 0);
  const double u = u53(W.x, W.y), u2 = u53(W.z, W.w);
  const R vax = S.vx[ia], vay = S.vy[ia], vaz = S.vz[ia];
  const R vbx = S.vx[ib], vby = S.vy[ib], vbz = S.vz[ib];
  const uint8_t qa = S.qs[ia], qb = S.qs[ib];
  const double ma = P.mass[sp_of(qa)], mb = P.mass[sp_of(qb)];
  const double ea = 0.5 * ma * (double)((vax * vax + vay * vay) + vaz * vaz);
  const double eb = 0.5 * mb * (double)((vbx * vbx + vby * vby) + vbz * vbz);
  if (count_e0_a) acc[4] += ea;
  if (count_e0_b) acc[4] += eb;
  const R ux = vax - vbx, uy = vay - vby, uz = vaz - vbz;
  const R g2 = (ux * ux + uy * uy) + uz * uz;
  if (g2 == (R)0) return;
  const R g = sqrt(g2);
  const double mu = (ma * mb) / (ma + mb);
  const double qq = (double)q_of(qa) * (double)q_of(qb);
  const double num = ((P.Cs * (qq * qq)) * nc) * dtp;
  const double den = (mu * mu) * ((double)g2 * (double)g);
  const double sv = num / den;
  const R omc = (R)nanbu_omc(T->lnA, sv, u);
  const R sinchi = sqrt(omc * ((R)2 - omc));
  R sp, cp;
  sincos_r((R)(2.0 * kPi * u2), &sp, &cp);
  const R ca = sinchi * cp, cb = sinchi * sp;
  const R uperp = sqrt(ux * ux + uy * uy);
  R dux, duy, duz;
  if (uperp > (R)0) {
    dux = (((ux / uperp) * uz) * ca - ((uy / uperp) * g) * cb) - ux * omc;
    duy = (((uy / uperp) * uz) * ca + ((ux / uperp) * g) * cb) - uy * omc;
    duz = -(uperp * ca) - uz * omc;
  } else {
    dux = g * ca;
    duy = g * cb;
    duz = -(g * omc);
  }
  const R ra = (R)(mu / ma), rb = (R)(mu / mb);
  const R nax = vax + ra * dux, nay = vay + ra * duy, naz = vaz + ra * duz;
  const R nbx = vbx - rb * dux, nby = vby - rb * duy, nbz = vbz - rb * duz;
  S.vx[ia] = nax;
  S.vy[ia] = nay;
  S.vz[ia] = naz;
  S.vx[ib] = nbx;
  S.vy[ib] = nby;
  S.vz[ib] = nbz;
  acc[0] += ma * (double)(nax - vax) + mb * (double)(nbx - vbx);
  acc[1] += ma * (double)(nay - vay) + mb * (double)(nby - vby);
  acc[2] += ma * (double)(naz - vaz) + mb * (double)(nbz - vbz);
  const double ea1 = 0.5 * ma * (double)((nax * nax + nay * nay) + naz * naz);
  const double eb1 = 0.5 * mb * (double)((nbx * nbx + nby * nby) + nbz * nbz);
  acc[3] += (ea1 - ea) + (eb1 - eb);
}

__device__ __forceinline__ bool key_less(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

template <typename R>
__global__ void __launch_bounds__(256) k_coulomb(KParams P, const Tables *__restrict__ T, Soa<R> S,
                                                 const uint32_t *__restrict__ cellid,
                                                 const uint32_t *__restrict__ cell_off, int64_t ncell,
                                                 DevAccum *__restrict__ accum, uint32_t step) {
  __shared__ uint64_t skey[kCoulMaxE];
  __shared__ uint32_t sid[kCoulMaxE];
  __shared__ uint32_t sslot[kCoulMaxE];
  __shared__ int64_t srange[2];
  __shared__ double sred[5][4];
  const int tid = threadIdx.x, bs = blockDim.x;
  const int64_t n = P.n;
  if (tid == 0) {
    const int64_t b = blockIdx.x;
    const int64_t t_lo = b * kCoulCap;
    const int64_t t_hi = t_lo + kCoulCap < n ? t_lo + kCoulCap : n;
    // first cell whose start offset is >= target (cell_off has ncell+1 entries)
    int64_t lo = 0, hi = ncell + 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)cell_off[mid] < t_lo) lo = mid + 1; else hi = mid;
    }
    const int64_t c_lo = lo;
    lo = c_lo;
    hi = ncell + 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)cell_off[mid] < t_hi) lo = mid + 1; else hi = mid;
    }
    const int64_t c_hi = lo;
    srange[0] = c_lo <= ncell ? cell_off[c_lo] : n;
    srange[1] = c_hi <= ncell ? cell_off[c_hi] : n;
    if (t_hi >= n) srange[1] = n;
  }
  __syncthreads();
  const int64_t s_lo = srange[0];
  const int64_t ns = srange[1] - s_lo;
  if (ns <= 1) return;
  if (ns > kCoulMaxE) {
    if (tid == 0) atomicOr(&accum->err, ERR_COUL_OVERFLOW);
    return;
  }
  int p2 = 2;
  while (p2 < ns) p2 <<= 1;
  for (int i = tid; i < p2; i += bs) {
    if (i < ns) {
      const int64_t j = s_lo + i;
      const uint32_t id = S.pid[j];
      const bool pool = q_of(S.qs[j]) >= 1;
      const uint4 W = draw(P, id, step, S_STEP, 0);
      skey[i] = ((uint64_t)cellid[j] << 33) | ((uint64_t)(pool ? 0u : 1u) << 32) | (uint64_t)W.z;
      sid[i] = id;
      sslot[i] = (uint32_t)j;
    } else {
      skey[i] = ~0ull;
      sid[i] = 0xFFFFFFFFu;
      sslot[i] = 0;
    }
  }
  __syncthreads();
  // bitonic sort ascending on (key, id)
  for (int k = 2; k <= p2; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int i = tid; i < p2; i += bs) {
        const int l = i ^ jj;
        if (l > i) {
          const uint64_t ka = skey[i], kb = skey[l];
          const uint32_t ia = sid[i], ib = sid[l];
          const bool up = (i & k) == 0;
          const bool swap = up ? key_less(kb, ib, ka, ia) : key_less(ka, ia, kb, ib);
          if (swap) {
            skey[i] = kb;
            skey[l] = ka;
            sid[i] = ib;
            sid[l] = ia;
            const uint32_t t = sslot[i];
            sslot[i] = sslot[l];
            sslot[l] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = tid; i < ns; i += bs) {
    const uint64_t key = skey[i];
    if ((key >> 32) & 1ull) continue;  // atom: not in any pool
    const uint64_t cbase = (key >> 33) << 33;
    // pool start: first entry with key >= cbase; pool end: first with key >= cbase | 1<<32
    int lo = 0, hi = i;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (skey[mid] < cbase) lo = mid + 1; else hi = mid;
    }
    const int start = lo;
    const uint64_t cend = cbase | (1ull << 32);
    lo = i + 1;
    hi = (int)ns;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (skey[mid] < cend) lo = mid + 1; else hi = mid;
    }
    const int m = lo - start;
    const int r = i - start;
    if (m < 2) continue;
    const double nc = (double)m * P.nfac;
    if (m & 1) {
      if (r == 0) {
        const double h = 0.5 * P.dt;
        const uint32_t s0 = sslot[i], s1 = sslot[i + 1], s2 = sslot[i + 2];
        collide<R>(P, T, S, s0, s1, sid[i], nc, h, step, acc, true, true);
        collide<R>(P, T, S, s1, s2, sid[i + 1], nc, h, step, acc, false, true);
        collide<R>(P, T, S, s2, s0, sid[i + 2], nc, h, step, acc, false, false);
      } else if (r >= 3 && (r & 1)) {
        collide<R>(P, T, S, sslot[i], sslot[i + 1], sid[i], nc, P.dt, step, acc, true, true);
      }
    } else if (!(r & 1)) {
      collide<R>(P, T, S, sslot[i], sslot[i + 1], sid[i], nc, P.dt, step, acc, true, true);
    }
  }
  // workgroup reduction of the moment changes, then one atomic per quantity
  for (int q = 0; q < 5; ++q) {
    double v = acc[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((tid & 63) == 0) sred[q][tid >> 6] = v;
  }
  __syncthreads();
  if (tid < 5) {
    double v = 0.0;
    for (int w = 0; w < (bs + 63) / 64; ++w) v += sred[tid][w];
    if (v != 0.0) {
      double *dst = tid < 3 ? &accum->t.coul_dp[tid] : (tid == 3 ? &accum->t.coul_de : &accum->t.coul_e);
      atomicAdd(dst, v);
    }
  }
}

template <typename R>
void launch_coulomb(const KParams &P, const Tables *T, Soa<R> S, const uint32_t *cellid, const uint32_t *cell_off,
                    int64_t ncell, DevAccum *acc, uint32_t step, hipStream_t st) {
  if (P.n <= 1) return;
  const unsigned nb = (unsigned)((P.n + kCoulCap - 1) / kCoulCap);
  hipLaunchKernelGGL(k_coulomb<R>, dim3(nb), dim3(256), 0, st, P, T, S, cellid, cell_off, ncell, acc, step);
}

template void launch_coulomb<double>(const KParams &, const Tables *, Soa<double>, const uint32_t *,
                                     const uint32_t *, int64_t, DevAccum *, uint32_t, hipStream_t);
template void launch_coulomb<float>(const KParams &, const Tables *, Soa<float>, const uint32_t *, const uint32_t *,
                                    int64_t, DevAccum *, uint32_t, hipStream_t);

}  // namespace ecr
