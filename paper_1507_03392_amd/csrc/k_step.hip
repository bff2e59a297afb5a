// k_step.hip -- the whole ion step in one kernel (Mironov et al., Sec. II):
// Takizuka-Abe pairing and Nanbu scattering of the ions of each collision
// cell, then the push in the magnetic field, wall / aperture loss,
// ionisation or charge exchange, and the cloud-in-cell deposit.
//
// One workgroup (four wavefronts) owns a chunk of whole collision cells: the
// cells whose first sorted slot lies in [b*c, (b+1)*c), c the run's chunk
// size (step_fcap; the table is rebuilt at every sort).
// Cells never straddle chunks and nothing couples two cells within a step
// except the density grid and the tallies (atomics), so each chunk is
// stepped start to finish by its workgroup and the state is read once and
// written once:
//  1. lane = slot, four rounds of 256: charge, id and the slot's buckets
//     (tabulated per cell at the sort) are loaded; each particle's STEP
//     draw is made once: words 0-1 are its Monte-Carlo uniform (kept in
//     registers for step 6), word 2 its pairing key;
//  2. the pool of each cell (its ions) is ordered by (key, id) in LDS: a
//     cell of m slots gets 2^floor(log2 m) buckets on the top key bits, an
//     LDS histogram and scan place the members bucket by bucket, and a
//     member's exact position is its bucket offset plus the bucket mates of
//     smaller (key, id); pair leaders (and odd pools' triplet leaders)
//     write their work items to LDS, triplets first;
//  3. the velocities go to LDS;
//  4. the collisions in LDS, one binary collision per lane and iteration (a
//     pair is one, a triplet three in a row at dt/2 in its lane; triplets
//     one to a lane in the first wavefronts, whose spare lanes take pairs
//     three at a time); momentum and energy sums go to one slot per
//     wavefront of the chunk;
//  5-6. lane = slot again: positions are loaded, the velocities read back
//     from LDS, each particle is pushed,
//     tested against the walls and the aperture, and draws its ionisation /
//     exchange outcome from the uniform of step 1; the state is stored;
//  7. the deposit inputs are staged and deposited through an LDS brick.
// A chunk of more than kFMax slots (a cell crowded with atoms at the gas
// inlet, or any very populous cell) is taken by one of the kBigWG handler
// workgroups at the front of the grid, from a list made at the sort: cell
// by cell it sorts the pool's (key, slot) values with a bitonic network
// (in LDS, or in a global scratch array beyond its capacity; equal keys are
// then ordered by id), collides the pairs from global memory, and pushes
// and deposits the chunk tile by tile.  No cell size skips its collisions.
#include <stddef.h>

#include "ecr_coll.hpp"
#include "ecr_kernels.hpp"
#include "ecr_push.hpp"
#include "ecr_wave.hpp"

namespace ecr {

namespace {

// four wavefronts per workgroup (two per workgroup with chunks of 320 slots
// ran 7% slower at 2M ions: a chunk's 160 pairs leave more lanes idle in the
// collisions than 384 do)
constexpr int kFB = 256;                  // lanes per workgroup
constexpr int kFR = 4;                    // rounds of kFB slots
constexpr int kFMax = kFB * kFR;          // slots of a chunk on the fast path
constexpr int kFLead = kFR * (kFB / 64);  // (round, wavefront) entries
constexpr int kBigWG = 4;                 // handler workgroups of oversized chunks
static_assert(kFR == kP, "the deposit stages one tile of kP slots per lane: the chunk");
static_assert(kFMax > kFCap, "a chunk fits the fast path unless one of its cells is large");
static_assert(kFLead <= 64, "per-wave counts fit one wavefront");

// LDS layout in bytes.  Ordering (steps 1-2): the members' (key, id) by
// bucket, the bucket histogram, the members by pool position.  Collisions
// (steps 3-5): the velocities over the ordering arrays, the work items beyond
// both.  Ids and charges (steps 1-4) beyond all of these.  Deposit (steps
// 6-7): the staging and brick over everything.
constexpr int kBkeyOff = 0;
constexpr int kR1Off = kBkeyOff + 8 * kFMax;
static_assert(kR1Off + 4 * (kFMax + 2) >= kBkeyOff + 8 * (kFMax + 3), "a bucket's batch of four keys stays in the arrays");
constexpr int kOrdOff = kR1Off + 4 * (kFMax + 2);
constexpr int kOrdEnd = kOrdOff + 2 * kFMax;
constexpr int align16(int v) { return (v + 15) / 16 * 16; }
template <typename R>
constexpr int items_off() {
  return align16(3 * kFMax * (int)sizeof(R) > kOrdEnd ? 3 * kFMax * (int)sizeof(R) : kOrdEnd);
}
template <typename R>
constexpr int sid_off() {
  return items_off<R>() + 8 * (kFMax / 2);
}
template <typename R>
constexpr int sqs_off() {
  return sid_off<R>() + 4 * kFMax;
}
template <typename R>
constexpr int lds_bytes() {
  return align16(sqs_off<R>() + kFMax > (int)sizeof(DepShared<R, kFMax>) ? sqs_off<R>() + kFMax
                                                                         : (int)sizeof(DepShared<R, kFMax>));
}

// velocities and charges of the chunk's slots in LDS
template <typename R>
struct LdsAcc {
  R *v;            // [3][kFMax]
  const uint8_t *q;
  __device__ __forceinline__ R &vx(uint32_t i) const { return v[i]; }
  __device__ __forceinline__ R &vy(uint32_t i) const { return v[kFMax + i]; }
  __device__ __forceinline__ R &vz(uint32_t i) const { return v[2 * kFMax + i]; }
  __device__ __forceinline__ uint8_t qs(uint32_t i) const { return q[i]; }
};

// a work item: slots a, b, c (c: the third member of a triplet) relative to
// the chunk, the pool size m, and whether it is a triplet
__device__ __forceinline__ uint64_t make_item(uint32_t a, uint32_t b, uint32_t c, uint32_t m, bool tri) {
  return (uint64_t)a | ((uint64_t)b << 11) | ((uint64_t)c << 22) | ((uint64_t)m << 33) | ((uint64_t)tri << 44);
}

// the momentum / energy sums of a wavefront into its own moment slot (all
// lanes call it)
__device__ __forceinline__ void flush_moments(const double acc[5], double *__restrict__ slot) {
  for (int k = 0; k < 5; ++k) {
    const double v = wave_sum_last(acc[k]);
    if ((threadIdx.x & 63) == 63 && v != 0.0) slot[k] += v;
  }
}

// a workgroup sum (all lanes call it; red: kFB / 64 words)
__device__ __forceinline__ uint32_t wg_sum_u32(uint32_t v, uint32_t *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();  // red may still be read by the previous call
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t s = 0;
  for (int w = 0; w < kFB / 64; ++w) s += red[w];
  return s;
}

// push + wall/aperture + MCC + deposit of slots [t0, min(t0 + kFMax, hi)),
// lane = slot, every value loaded from global memory and the uniform drawn
// here (the oversized chunks' path)
template <typename R, int DEP, bool EXT>
__device__ __forceinline__ void push_tile_global(const KParams &P, const Tables *__restrict__ T, Soa<R> S,
                                                 uint8_t *__restrict__ evlog, DevAccum *__restrict__ acc,
                                                 double *__restrict__ dens, uint32_t step,
                                                 const uint32_t *__restrict__ chg_cur, uint32_t *__restrict__ chg_next,
                                                 int64_t t0, int64_t hi, DepShared<R, kFMax> &dsh, int *box) {
  int mn[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, mx[3] = {-1, -1, -1};
#pragma unroll
  for (int p = 0; p < kP; ++p) {
    const int i = threadIdx.x + p * kFB;
    const int64_t j = t0 + i;
    uint32_t ccell = 0xffffffffu, cq = 0u;
    if (j >= hi) {
      if (DEP) dsh.st.q[i] = 0xFF;
    } else {
      R x = S.x[j], y = S.y[j], z = S.z[j];
      R vx = S.vx[j], vy = S.vy[j], vz = S.vz[j];
      const uint8_t qs0 = S.qs[j];
      const uint32_t id = S.pid[j];
      int Q = q_of(qs0);
      const int s = sp_of(qs0);
      double u = 0.0;
      if (needs_mcc_uniform(P)) {
        const uint4 W = draw(P, id, step, S_STEP, 0);
        u = u53(W.x, W.y);
      }
      const uint8_t ev =
          advance<R, 0, EXT>(P, T, nullptr, acc, step, id, s, Q, x, y, z, vx, vy, vz, S.birth, j, j, chg_cur, u);
      S.x[j] = x;
      S.y[j] = y;
      S.z[j] = z;
      S.vx[j] = vx;
      S.vy[j] = vy;
      S.vz[j] = vz;
      S.qs[j] = make_qs(Q, s);
      if (evlog) evlog[j] = ev;
      if (EXT && chg_next) {
        const uint32_t c = cell_of<R>(P, x, y, z);
        ccell = Q >= 1 ? c : (uint32_t)(1 + s) * P.ncell + c;
        cq = Q >= 1 ? (uint32_t)Q : 1u;
      }
      if (DEP) stage_cic<R, DEP == 2, kFMax>(P, dsh.st, i, x, y, z, Q, mn, mx);
    }
    if (EXT && chg_next) add_charge(chg_next, ccell, cq);
  }
  if (DEP) deposit_staged<R, DEP == 2, 4, kFB>(P, dens, dsh, box, mn, mx);
}

// an oversized chunk [lo, hi), chunk index b, by one workgroup
template <typename R, int DEP, bool EXT>
__device__ __forceinline__ void big_chunk(const KParams &P, const Tables *__restrict__ T, Soa<R> S, const uint32_t *__restrict__ cellid,
                          int64_t lo, int64_t hi, int64_t b, uint8_t *__restrict__ evlog, DevAccum *__restrict__ acc,
                          double *__restrict__ dens, double *__restrict__ moments, uint64_t *__restrict__ scratch64,
                          uint32_t step, const uint32_t *__restrict__ chg_cur, uint32_t *__restrict__ chg_next,
                          unsigned char *lds, int *box, uint32_t *red, uint32_t *gcount) {
  const int tid = threadIdx.x;
  // (key, slot) values the LDS holds: the largest power of two that fits
  constexpr int kBigLds = lds_bytes<R>() / 8 >= 4096 ? 4096 : (lds_bytes<R>() / 8 >= 2048 ? 2048 : 1024);
  static_assert(kBigLds * 8 <= lds_bytes<R>(), "LDS sort buffer");
  double cacc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (P.pmask & P_COULOMB) {
    int64_t c_lo = lo;
    while (c_lo < hi) {  // uniform: every lane walks the same cells
      const uint32_t c = cellid[c_lo];
      int64_t c_hi = (int64_t)P.cell_off[c + 1];
      c_hi = c_hi < hi ? c_hi : hi;
      uint32_t cnt = 0;
      for (int64_t t = c_lo + tid; t < c_hi; t += kFB) cnt += q_of(S.qs[t]) >= 1 ? 1u : 0u;
      const uint32_t m = wg_sum_u32(cnt, red);
      if (m >= 2) {
        // the pool's (key << 32 | slot in chunk) values, in any order
        uint64_t *arr = m <= (uint32_t)kBigLds ? reinterpret_cast<uint64_t *>(lds) : scratch64 + c_lo;
        if (tid == 0) *gcount = 0u;
        __syncthreads();
        for (int64_t t = c_lo + tid; t < c_hi; t += kFB) {
          if (q_of(S.qs[t]) < 1) continue;
          const uint32_t k = draw(P, S.pid[t], step, S_STEP, 0).z;
          arr[atomicAdd(gcount, 1u)] = ((uint64_t)k << 32) | (uint32_t)(t - lo);
        }
        __syncthreads();
        // bitonic sort of arr[0..m) in ascending order; positions from m to
        // the next power of two hold +infinity virtually: every comparator
        // puts the smaller value at the lower position (the first stage of
        // each merge compares a position with its mirror in the block), so a
        // comparator that reaches past m never swaps
        uint32_t p2 = 1;
        while (p2 < m) p2 <<= 1;
        for (uint32_t k = 2; k <= p2; k <<= 1) {
          for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
            for (uint32_t t = tid; t < p2 / 2; t += kFB) {
              const uint32_t i = (t / jj) * 2 * jj + (t % jj);
              const uint32_t l = jj == (k >> 1) ? (i ^ (k - 1)) : i + jj;
              if (l < m) {
                const uint64_t x = arr[i], y = arr[l];
                if (y < x) {
                  arr[i] = y;
                  arr[l] = x;
                }
              }
            }
            __syncthreads();
          }
        }
        // equal 32-bit keys (rare) are ordered by particle id: the first
        // position of each run sorts the run by insertion
        for (uint32_t t = tid; t < m; t += kFB) {
          const uint32_t kt = (uint32_t)(arr[t] >> 32);
          if ((t == 0 || (uint32_t)(arr[t - 1] >> 32) != kt) && t + 1 < m && (uint32_t)(arr[t + 1] >> 32) == kt) {
            uint32_t e = t + 1;
            while (e < m && (uint32_t)(arr[e] >> 32) == kt) ++e;
            for (uint32_t x = t + 1; x < e; ++x) {
              const uint64_t v = arr[x];
              const uint32_t idv = S.pid[lo + (uint32_t)v];
              uint32_t y = x;
              while (y > t && S.pid[lo + (uint32_t)arr[y - 1]] > idv) {
                arr[y] = arr[y - 1];
                --y;
              }
              arr[y] = v;
            }
          }
        }
        __syncthreads();
        // the odd pool's triplet as item 0, then the pairs
        const bool odd = (m & 1u) != 0u;
        const uint32_t np = odd ? (m - 3u) / 2u : m / 2u;
        const uint32_t nit = np + (odd ? 1u : 0u);
        const double nc = (double)m * P.nfac;
        for (uint32_t it = tid; it < nit; it += kFB) {
          if (odd && it == 0) {
            const uint32_t a = (uint32_t)lo + (uint32_t)arr[0], bb = (uint32_t)lo + (uint32_t)arr[1];
            const uint32_t cc = (uint32_t)lo + (uint32_t)arr[2];
            const double h = 0.5 * P.dt;
            collide<R>(P, T->lnA, S, a, bb, S.pid[a], nc, h, step, cacc, true, true);
            collide<R>(P, T->lnA, S, bb, cc, S.pid[bb], nc, h, step, cacc, false, true);
            collide<R>(P, T->lnA, S, cc, a, S.pid[cc], nc, h, step, cacc, false, false);
          } else {
            const uint32_t pp = odd ? 3u + 2u * (it - 1u) : 2u * it;
            const uint32_t a = (uint32_t)lo + (uint32_t)arr[pp], bb = (uint32_t)lo + (uint32_t)arr[pp + 1];
            collide<R>(P, T->lnA, S, a, bb, S.pid[a], nc, P.dt, step, cacc, true, true);
          }
        }
        __syncthreads();  // the sort buffer is reused; the push reads the velocities
      }
      c_lo = c_hi;
    }
    flush_moments(cacc, moments + (b * (kFB / 64) + (tid >> 6)) * 5);
  }
  DepShared<R, kFMax> &dsh = *reinterpret_cast<DepShared<R, kFMax> *>(lds);
  for (int64_t t0 = lo; t0 < hi; t0 += kFMax) {
    push_tile_global<R, DEP, EXT>(P, T, S, evlog, acc, dens, step, chg_cur, chg_next, t0, hi, dsh, box);
    __syncthreads();  // the brick is read before the next tile stages over it
  }
}

}  // namespace

// workgroup wg of one run's step: wg < kBigWG handles the oversized chunks,
// wg = kBigWG + b steps chunk b
template <typename R, int DEP, bool EXT>
__device__ __forceinline__ void step_wg(const KParams &P, const Tables *__restrict__ T, Soa<R> S,
                                        const uint32_t *__restrict__ cellid, const uint32_t *__restrict__ chunk_lo,
                                        const uint32_t *__restrict__ big, const uint32_t *__restrict__ bkinfo,
                                        const uint32_t *__restrict__ nbk, uint8_t *__restrict__ evlog,
                                        DevAccum *__restrict__ acc, double *__restrict__ dens,
                                        double *__restrict__ moments, uint64_t *__restrict__ scratch64, StepArg sa,
                                        const uint32_t *__restrict__ chg_cur, uint32_t *__restrict__ chg_next,
                                        const uint32_t wg) {
  __shared__ __align__(16) unsigned char lds[lds_bytes<R>()];
  __shared__ uint32_t lead[kFLead], wsum[kFB / 64];
  __shared__ int box[6 * (kFB / 64)];
  const uint32_t step = sa.get();
  const int tid = threadIdx.x;
  if (wg < (unsigned)kBigWG) {
    __shared__ uint32_t gcount;
    const uint32_t nbig = big[0];
    for (uint32_t e = wg; e < nbig; e += kBigWG) {
      const uint32_t b = big[1 + e];
      big_chunk<R, DEP, EXT>(P, T, S, cellid, chunk_lo[b], chunk_lo[b + 1], b, evlog, acc, dens, moments, scratch64,
                             step, chg_cur, chg_next, lds, box, wsum, &gcount);
      __syncthreads();
    }
    return;
  }
  const int64_t b = (int64_t)wg - kBigWG;
  const int64_t lo = chunk_lo[b];
  const int nsl = (int)((int64_t)chunk_lo[b + 1] - lo);
  if (nsl <= 0 || nsl > kFMax) return;  // empty, or an oversized chunk (taken by a handler)
  // the chunk's arrays from its first slot: uniform bases, 32-bit offsets
  S.x += lo;
  S.y += lo;
  S.z += lo;
  S.vx += lo;
  S.vy += lo;
  S.vz += lo;
  S.qs += lo;
  S.pid += lo;
  S.birth += lo;
  bkinfo += lo;
  if (evlog) evlog += lo;
  const int lane = tid & 63, wv = tid >> 6;
  const int wvu = __builtin_amdgcn_readfirstlane(wv);
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const bool coul = (P.pmask & P_COULOMB) != 0 && nsl >= 2;
  const bool mcc = needs_mcc_uniform(P);
  uint64_t *bkey = reinterpret_cast<uint64_t *>(lds + kBkeyOff);
  uint32_t *hist = reinterpret_cast<uint32_t *>(lds + kR1Off);
  uint16_t *pord = reinterpret_cast<uint16_t *>(lds + kOrdOff);
  R *vs = reinterpret_cast<R *>(lds);
  uint64_t *items = reinterpret_cast<uint64_t *>(lds + items_off<R>());
  uint32_t *sid = reinterpret_cast<uint32_t *>(lds + sid_off<R>());
  uint8_t *sqs = lds + sqs_off<R>();

  // 1. load; one STEP draw per particle: uniform (words 0-1) and pairing key
  //    (word 2); the slot's buckets (first bucket, log2 of their number: its
  //    cell's, set at the sort)
  uint8_t qs[kFR];
  uint32_t id[kFR], key[kFR], bki[kFR];
  R vr[kFR][3];  // the velocities, loaded here so that their latency overlaps the ordering
  double u[kFR];
  bool pool[kFR];
  // every round's loads go out before any is used (indices clamped to the
  // chunk, so that no load waits behind a branch): ids, charges and bucket
  // words first, the velocities last, so that the draws and the ordering
  // wait only for the former (the memory counter drains in issue order) and
  // the velocities arrive during the ordering; the histogram is cleared
  // while they are in flight
  int jc[kFR];
#pragma unroll
  for (int k = 0; k < kFR; ++k) jc[k] = min(tid + k * kFB, nsl - 1);
#pragma unroll
  for (int k = 0; k < kFR; ++k) id[k] = S.pid[jc[k]];
#pragma unroll
  for (int k = 0; k < kFR; ++k) qs[k] = S.qs[jc[k]];
#pragma unroll
  for (int k = 0; k < kFR; ++k) bki[k] = coul ? bkinfo[jc[k]] : 0u;
#pragma unroll
  for (int k = 0; k < kFR; ++k) {
    vr[k][0] = S.vx[jc[k]];
    vr[k][1] = S.vy[jc[k]];
    vr[k][2] = S.vz[jc[k]];
  }
  const int nbuckets = coul ? (int)nbk[b] : 0;
  for (int i = tid; i <= nbuckets; i += kFB) hist[i] = 0u;
#pragma unroll
  for (int k = 0; k < kFR; ++k) {
    const int i = tid + k * kFB;
    const bool in = i < nsl;
    if (!in) {
      qs[k] = 0;
      id[k] = bki[k] = 0u;
    }
    key[k] = 0u;
    u[k] = 0.0;
    pool[k] = in && coul && q_of(qs[k]) >= 1;
    if (in && (mcc || pool[k])) {
      const uint4 W = draw(P, id[k], step, S_STEP, 0);
      u[k] = u53(W.x, W.y);
      key[k] = W.z;
    }
    if (coul && in) {
      sid[i] = id[k];
      sqs[i] = qs[k];
    }
  }
  int nitems = 0, ntri = 0;
  if (coul) {
    __syncthreads();
    // 2c. histogram of the pool members over their cell's buckets
    int bk[kFR], arr[kFR];
#pragma unroll
    for (int k = 0; k < kFR; ++k) {
      bk[k] = 0;
      arr[k] = 0;
      if (pool[k]) {
        const int lg = (int)(bki[k] >> 16);
        bk[k] = (int)(bki[k] & 0xffffu) + (lg ? (int)(key[k] >> (32 - lg)) : 0);
        arr[k] = (int)atomicAdd(&hist[bk[k]], 1u);
      }
    }
    __syncthreads();
    // 2d. bucket offsets; the members' (key, id) listed bucket by bucket
    (void)wg_exscan<kFB>(hist, nbuckets, wsum, true);  // hist[nbuckets] = pool total
#pragma unroll
    for (int k = 0; k < kFR; ++k)
      if (pool[k]) bkey[hist[bk[k]] + arr[k]] = ((uint64_t)key[k] << 32) | id[k];
    __syncthreads();
    // 2e. exact pool position: bucket offset + bucket mates of smaller (key, id)
    int pos[kFR], rr[kFR], mm[kFR];
#pragma unroll
    for (int k = 0; k < kFR; ++k) {
      pos[k] = rr[k] = mm[k] = 0;
      if (pool[k]) {
        const uint64_t me = ((uint64_t)key[k] << 32) | id[k];
        const int b0 = (int)hist[bk[k]], b1 = (int)hist[bk[k] + 1];
        // the bucket's first four entries in one batch of loads (a bucket
        // holds one or two members mostly; entries past its end are masked,
        // and b0 + 3 stays inside the histogram that follows the keys), the
        // rest one by one
        const uint64_t q0 = bkey[b0], q1 = bkey[b0 + 1], q2 = bkey[b0 + 2], q3 = bkey[b0 + 3];
        int rib = (q0 < me ? 1 : 0) + (b0 + 1 < b1 && q1 < me ? 1 : 0) + (b0 + 2 < b1 && q2 < me ? 1 : 0) +
                  (b0 + 3 < b1 && q3 < me ? 1 : 0);
        for (int t = b0 + 4; t < b1; ++t) rib += bkey[t] < me ? 1 : 0;
        pos[k] = b0 + rib;
        const int c0 = (int)(bki[k] & 0xffffu);
        const int pstart = (int)hist[c0];
        mm[k] = (int)hist[c0 + (1 << (bki[k] >> 16))] - pstart;
        rr[k] = pos[k] - pstart;
      }
    }
    // 2f. pool order, and the pair and triplet leaders per round and wave
#pragma unroll
    for (int k = 0; k < kFR; ++k)
      if (pool[k]) pord[pos[k]] = (uint16_t)(tid + k * kFB);
    const int nk = (nsl + kFB - 1) / kFB;  // rounds that hold slots
    int lt[kFR], li[kFR];
#pragma unroll
    for (int k = 0; k < kFR; ++k) {
      lt[k] = 0;
      li[k] = 0;
      if (k < nk) {  // uniform over the workgroup
        if (pool[k]) {
          const int m = mm[k], r = rr[k];
          if (m >= 2) {
            if ((m & 1) && r == 0) lt[k] = 2;                              // triplet
            else if ((m & 1) ? (r >= 3 && (r & 1)) : !(r & 1)) lt[k] = 1;  // pair
          }
        }
        const uint64_t bp = __ballot(lt[k] == 1), bt = __ballot(lt[k] == 2);
        li[k] = __popcll((lt[k] == 2 ? bt : bp) & below);
        if (lane == 0) lead[k * (kFB / 64) + wv] = (uint32_t)__popcll(bp) | ((uint32_t)__popcll(bt) << 16);
      }
    }
    __syncthreads();
    // 2g. work items, triplets first, each kind numbered in the slot order of
    //     its leaders
    const uint32_t c = lane < nk * (kFB / 64) ? lead[lane] : 0u;
    const uint32_t incl = wave_incl_scan(c), excl = incl - c;
    const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, kFLead - 1);
    const int np = (int)(tot & 0xffffu);
    ntri = (int)(tot >> 16);
    nitems = np + ntri;
#pragma unroll
    for (int k = 0; k < kFR; ++k) {
      const uint32_t before = (uint32_t)__builtin_amdgcn_readlane((int)excl, k * (kFB / 64) + wvu);
      if (lt[k]) {
        const int p = pos[k];
        const uint32_t a = pord[p], bb = pord[p + 1], cc = lt[k] == 2 ? pord[p + 2] : 0u;
        const int slot = lt[k] == 2 ? (int)(before >> 16) + li[k] : ntri + (int)(before & 0xffffu) + li[k];
        items[slot] = make_item(a, bb, cc, (uint32_t)mm[k], lt[k] == 2);
      }
    }
    __syncthreads();
  }
  // 3. the velocities into LDS (over the ordering arrays)
#pragma unroll
  for (int k = 0; k < kFR; ++k) {
    const int i = tid + k * kFB;
    if (i < nsl) {
      vs[i] = vr[k][0];
      vs[kFMax + i] = vr[k][1];
      vs[2 * kFMax + i] = vr[k][2];
    }
  }
  if (coul) {
    __syncthreads();
    // 4. collisions, one binary collision per lane and iteration: a triplet
    //    is three collisions in a row in its lane, a pair one.  The triplets
    //    fill the first wavefronts one to a lane, the spare lanes of the last
    //    of these take up to three pairs each, one after the other, and the
    //    other wavefronts take the remaining pairs round-robin, so a
    //    wavefront with a triplet runs three collisions.  (With more than
    //    three wavefronts of triplets, every item goes round-robin.)  Pairs
    //    are disjoint, so the order changes no particle.
    int first, count, stride;
    {
      const int np = nitems - ntri;
      if (ntri > kFB - 64) {
        first = tid;
        stride = kFB;
        count = tid < nitems ? (nitems - 1 - tid) / kFB + 1 : 0;
      } else {
        const int l3 = (ntri + 63) & ~63;         // lanes of the triplet wavefronts
        const int n3 = min(np, 3 * (l3 - ntri));  // pairs taken three to a lane
        if (tid < ntri) {
          first = tid;
          count = 1;
          stride = 1;
        } else if (tid < l3) {
          const int q = 3 * (tid - ntri);
          first = ntri + q;
          count = max(0, min(3, n3 - q));
          stride = 1;
        } else {
          const int q = tid - l3;
          stride = kFB - l3;
          first = ntri + n3 + q;
          count = q < np - n3 ? (np - n3 - 1 - q) / stride + 1 : 0;
        }
      }
    }
    // the lane's collisions: three per triplet item (items below ntri), one per pair
    int ncol = 0;
    for (int k = 0; k < count; ++k) ncol += first + k * stride < ntri ? 3 : 1;
    double cacc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const LdsAcc<R> A{vs, sqs};
    int k = 0, sub = 0;  // the lane's item, and the collision within a triplet
    for (int c = 0; c < ncol; ++c) {
      const uint64_t e = items[first + k * stride];
      const bool tri = ((e >> 44) & 1u) != 0;
      const uint32_t a = (uint32_t)(e & 0x7ff), bb = (uint32_t)((e >> 11) & 0x7ff);
      const uint32_t cc = (uint32_t)((e >> 22) & 0x7ff);
      // a triplet's collisions (a, b), (b, c), (c, a) at dt/2; the energy of
      // the pool before counts each member once
      const uint32_t ia = sub == 0 ? a : (sub == 1 ? bb : cc), ib = sub == 0 ? bb : (sub == 1 ? cc : a);
      const double nc = (double)((e >> 33) & 0x7ff) * P.nfac;
      collide_acc<R>(P, T->lnA, A, ia, ib, sid[ia], nc, tri ? 0.5 * P.dt : P.dt, step, cacc, sub == 0, sub < 2);
      if (tri && sub < 2) {
        ++sub;
      } else {
        sub = 0;
        ++k;
      }
    }
    flush_moments(cacc, moments + (b * (kFB / 64) + wv) * 5);
  }
  // 5-6. push + wall/aperture + MCC with the uniform of step 1, the
  // velocities read back from LDS; deposit staging.  The staging of slot i
  // (its fractional offsets) lies on exactly the LDS words of slot i's
  // velocity, and the same lane reads the one before it writes the other,
  // so the velocities need no copy; the staged cells and charges lie over
  // the work items and ids, dead after the collisions
  using Stage = DepStage<R, kFMax>;
  static_assert(offsetof(Stage, t) == 0 && sizeof(Stage::t) == 3 * kFMax * sizeof(R),
                "the staged offsets overlay the velocities slot by slot");
  DepShared<R, kFMax> &dsh = *reinterpret_cast<DepShared<R, kFMax> *>(lds);
  __syncthreads();  // collisions done (the staged cells go over the items)
  int mn[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, mx[3] = {-1, -1, -1};
  // every round's positions first (indices clamped to the chunk): one memory
  // latency for all rounds instead of one per round
  R xr[kFR][3];
#pragma unroll
  for (int k = 0; k < kFR; ++k) {
    const int j = min(tid + k * kFB, nsl - 1);
    xr[k][0] = S.x[j];
    xr[k][1] = S.y[j];
    xr[k][2] = S.z[j];
  }
#pragma unroll
  for (int k = 0; k < kFR; ++k) {
    const int i = tid + k * kFB;
    const int j = i;
    uint32_t ccell = 0xffffffffu, cq = 0u;
    if (i >= nsl) {
      if (DEP) dsh.st.q[i] = 0xFF;
    } else {
      R x = xr[k][0], y = xr[k][1], z = xr[k][2];
      R vx = vs[i], vy = vs[kFMax + i], vz = vs[2 * kFMax + i];
      int Q = q_of(qs[k]);
      const int s = sp_of(qs[k]);
      const uint8_t ev = advance<R, 0, EXT>(P, T, nullptr, acc, step, id[k], s, Q, x, y, z, vx, vy, vz, S.birth, j,
                                            lo + j, chg_cur, u[k]);
      S.x[j] = x;
      S.y[j] = y;
      S.z[j] = z;
      S.vx[j] = vx;
      S.vy[j] = vy;
      S.vz[j] = vz;
      S.qs[j] = make_qs(Q, s);
      if (evlog) evlog[j] = ev;
      if (EXT && chg_next) {
        const uint32_t c = cell_of<R>(P, x, y, z);
        ccell = Q >= 1 ? c : (uint32_t)(1 + s) * P.ncell + c;
        cq = Q >= 1 ? (uint32_t)Q : 1u;
      }
      if (DEP) stage_cic<R, DEP == 2, kFMax>(P, dsh.st, i, x, y, z, Q, mn, mx);
    }
    if (EXT && chg_next) add_charge(chg_next, ccell, cq);
  }
  // 7. deposit; the lanes' last runs summed within groups of four lanes
  // (groups of two: 110.8 us at 2M ions against 103.9; of eight: the same
  // time with 2% more instructions)
  if (DEP) deposit_staged<R, DEP == 2, 4, kFB>(P, dens, dsh, box, mn, mx);
}

template <typename R, int DEP, bool EXT>
__global__ void __launch_bounds__(kFB) __attribute__((amdgpu_waves_per_eu(4)))
k_step(KParams P, const Tables *__restrict__ T, Soa<R> S, const uint32_t *__restrict__ cellid,
       const uint32_t *__restrict__ chunk_lo, const uint32_t *__restrict__ big, const uint32_t *__restrict__ bkinfo,
       const uint32_t *__restrict__ nbk, uint8_t *__restrict__ evlog, DevAccum *__restrict__ acc,
       double *__restrict__ dens, double *__restrict__ moments, uint64_t *__restrict__ scratch64, StepArg sa,
       const uint32_t *__restrict__ chg_cur, uint32_t *__restrict__ chg_next) {
  step_wg<R, DEP, EXT>(P, T, S, cellid, chunk_lo, big, bkinfo, nbk, evlog, acc, dens, moments, scratch64, sa, chg_cur,
                       chg_next, blockIdx.x);
}

// one step of several runs in one launch: run j owns workgroups
// [wg0[j], wg0[j+1]) and reads its arguments from its job in device memory
template <typename R>
__global__ void __launch_bounds__(kFB) __attribute__((amdgpu_waves_per_eu(4))) k_step_batch(StepBatch<R> B) {
  const uint32_t wg = blockIdx.x;
  int j = 0;
  for (int t = 1; t < B.n; ++t) j = wg >= B.wg0[t] ? t : j;
  const StepJob<R> *__restrict__ J = B.job[j];
  step_wg<R, 2, false>(J->P, J->T, J->S, J->cellid, J->chunk_lo, J->big, J->bkinfo, J->nbk, J->evlog, J->acc,
                       J->dens, J->moments, J->scratch64, StepArg{B.stepw[j], B.step[j]}, nullptr, nullptr,
                       wg - B.wg0[j]);
}

// a run's job, passed by value, into device memory (one lane writes it)
template <typename R>
__global__ void k_set_job(StepJob<R> J, StepJob<R> *__restrict__ dst) {
  if (threadIdx.x == 0) *dst = J;
}

__global__ void k_set_words(SetWords w) {
  if ((int)threadIdx.x < w.n) *w.ptr[threadIdx.x] = w.val[threadIdx.x];
}

// Once per sort, for every chunk of the fast path: the buckets of each
// cell of the ordering (2^floor(log2 m) buckets for a cell of m slots,
// numbered cell after cell from the chunk's first slot), stored per slot as
// first bucket | log2(bucket count) << 16, and each chunk's bucket total.
// The cells of a slot range are fixed from one sort to the next; the step
// kernel only histograms its keys into them.
__global__ void __launch_bounds__(kFB) k_step_prep(const uint32_t *__restrict__ cellid,
                                                   const uint32_t *__restrict__ chunk_lo,
                                                   uint32_t *__restrict__ bkinfo, uint32_t *__restrict__ nbk) {
  __shared__ uint32_t cell[kFMax + 1];
  __shared__ uint16_t hd[kFMax], hcell[kFMax + 1];
  __shared__ uint32_t lead[kFLead], wsum[kFB / 64], nbs[kFMax + 1];
  const int64_t b = blockIdx.x;
  const int64_t lo = chunk_lo[b];
  const int nsl = (int)((int64_t)chunk_lo[b + 1] - lo);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wvu = __builtin_amdgcn_readfirstlane(wv);
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  if (nsl <= 0 || nsl > kFMax) {
    if (tid == 0) nbk[b] = 0u;
    return;
  }
  for (int i = tid; i < nsl; i += kFB) cell[i] = cellid[lo + i];
  __syncthreads();
  // heads of cells (ballots per round and wave, a scan of the counts), the
  // cell index of every slot, the first slot of every cell
  uint32_t fl[kFR];
  uint64_t hb[kFR];
#pragma unroll
  for (int k = 0; k < kFR; ++k) {
    const int i = tid + k * kFB;
    fl[k] = (i < nsl && (i == 0 || cell[i] != cell[i - 1])) ? 1u : 0u;
    hb[k] = __ballot(fl[k] != 0u);
    if (lane == 0) lead[k * (kFB / 64) + wv] = (uint32_t)__popcll(hb[k]);
  }
  __syncthreads();
  const uint32_t hc = lane < kFLead ? lead[lane] : 0u;
  const uint32_t hincl = wave_incl_scan(hc), hexcl = hincl - hc;
  const int nheads = __builtin_amdgcn_readlane((int)hincl, kFLead - 1);
#pragma unroll
  for (int k = 0; k < kFR; ++k) {
    const int i = tid + k * kFB;
    if (i < nsl) {
      const int h = __builtin_amdgcn_readlane((int)hexcl, k * (kFB / 64) + wvu) + (int)__popcll(hb[k] & below) +
                    (int)fl[k] - 1;
      hd[i] = (uint16_t)h;
      if (fl[k]) hcell[h] = (uint16_t)i;
    }
  }
  if (tid == 0) hcell[nheads] = (uint16_t)nsl;
  __syncthreads();
  // buckets per cell: 2^floor(log2(slots of the cell)), at most one per slot
  for (int h = tid; h < nheads; h += kFB) {
    const int m = hcell[h + 1] - hcell[h];
    const int lg = m <= 1 ? 0 : 31 - __clz(m);
    nbs[h] = 1u << lg;
  }
  __syncthreads();
  const uint32_t total = wg_exscan<kFB>(nbs, nheads, wsum);  // nbs: first bucket of each cell
  for (int i = tid; i < nsl; i += kFB) {
    const int h = hd[i];
    const uint32_t first = nbs[h];
    const uint32_t cnt = (h + 1 < nheads ? nbs[h + 1] : total) - first;
    bkinfo[lo + i] = first | ((uint32_t)(31 - __clz(cnt)) << 16);
  }
  if (tid == 0) nbk[b] = total;
}

// chunks of more than kFMax slots, listed once per sort: big[0] = count,
// big[1..] = chunk indices (any order)
__global__ void k_big_list(const uint32_t *__restrict__ chunk_lo, int64_t nchunks, uint32_t *__restrict__ big) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nchunks) return;
  if ((int64_t)chunk_lo[b + 1] - (int64_t)chunk_lo[b] > kFMax) big[1 + atomicAdd(&big[0], 1u)] = (uint32_t)b;
}

// the chunk size of a run: kFCap from 128 chunks up; a smaller run gets
// about 128 chunks of a power-of-two size (at least 64 slots), so that it
// still spreads over the CUs (and, its cells being sparsely filled, a
// chunk's deposit box fits the LDS brick more often).  Chunks smaller than
// kFCap cost more per particle where the GPU is full anyway (fewer pairs per
// workgroup, more fixed work per chunk), hence kFCap from 98 304 particles.
int64_t step_nchunks(int64_t n, int64_t cap) { return (n + cap - 1) / cap; }

// The last of the rounds in which the device's resident workgroups take the
// launch's workgroups is partly empty: chunks of kFCapLo slots instead of
// kFCap, where that fills the last round more, cut the idle share of it (at
// 2M particles on 1024 resident workgroups, 2722 workgroups fill 66% of the
// third round where 2609 fill 55%, and the step runs 1.3% faster; at 10M,
// 13025 fill 72% of the thirteenth where 13591 would fill 27%).
int64_t step_fcap(int64_t n, int64_t resident) {
  if (n < 128 * (int64_t)kFCap) {
    int64_t p = 64;
    while (2 * p <= n / 128 && 2 * p <= 512) p *= 2;
    return p;
  }
  if (resident <= 0) return kFCap;
  const auto fill = [&](int64_t cap) {
    const int64_t r = (step_nchunks(n, cap) + kBigWG) % resident;
    return r == 0 ? resident : r;  // workgroups in the last round
  };
  return fill(kFCapLo) > fill(kFCap) ? kFCapLo : kFCap;
}

int64_t step_nchunks_max(int64_t n) {
  return step_nchunks(n, n < 128 * (int64_t)kFCap ? step_fcap(n, 0) : (int64_t)kFCapLo);
}

int64_t step_moment_slots(int64_t n) { return step_nchunks_max(n) * (kFB / 64); }

int64_t step_resident_wgs(bool fp32) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const hipError_t e = fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_step<float, 2, false>, kFB, 0)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_step<double, 2, false>, kFB, 0);
  if (e != hipSuccess) return 0;
  return (int64_t)cus * per;
}

void launch_step_prep(const uint32_t *cellid, const uint32_t *chunk_lo, int64_t n, int64_t cap, uint32_t *big,
                      uint32_t *bkinfo,
                      uint32_t *nbk, hipStream_t st) {
  const int64_t nc = step_nchunks(n, cap);
  launch_fill_u32(big, 0u, 1, st);
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_big_list, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, chunk_lo, nc, big);
  hipLaunchKernelGGL(k_step_prep, dim3((unsigned)nc), dim3(kFB), 0, st, cellid, chunk_lo, bkinfo, nbk);
}

template <typename R, bool EXT>
static void launch_step_e(const KParams &P, const Tables *T, Soa<R> S, const uint32_t *cellid,
                          const uint32_t *chunk_lo, const uint32_t *big, const uint32_t *bkinfo, const uint32_t *nbk,
                          uint8_t *evlog, DevAccum *acc, double *dens,
                          double *moments, uint64_t *scratch64, StepArg step, const uint32_t *chg_cur,
                          uint32_t *chg_next, int64_t cap, hipStream_t st) {
  const dim3 g((unsigned)(kBigWG + step_nchunks(P.n, cap))), b(kFB);
  if (!dens)
    hipLaunchKernelGGL((k_step<R, 0, EXT>), g, b, 0, st, P, T, S, cellid, chunk_lo, big, bkinfo, nbk, evlog, acc, dens,
                       moments, scratch64, step, chg_cur, chg_next);
  else if ((P.dmask & 7u) == 3u)
    hipLaunchKernelGGL((k_step<R, 2, EXT>), g, b, 0, st, P, T, S, cellid, chunk_lo, big, bkinfo, nbk, evlog, acc, dens,
                       moments, scratch64, step, chg_cur, chg_next);
  else
    hipLaunchKernelGGL((k_step<R, 1, EXT>), g, b, 0, st, P, T, S, cellid, chunk_lo, big, bkinfo, nbk, evlog, acc, dens,
                       moments, scratch64, step, chg_cur, chg_next);
}

template <typename R>
void launch_step(const KParams &P, const Tables *T, Soa<R> S, const uint32_t *cellid, const uint32_t *chunk_lo,
                 const uint32_t *big, const uint32_t *bkinfo, const uint32_t *nbk, uint8_t *evlog, DevAccum *acc,
                 double *dens, double *moments,
                 uint64_t *scratch64, StepArg step, const uint32_t *chg_cur, uint32_t *chg_next, int64_t cap,
                 hipStream_t st) {
  if (P.n <= 0) return;
  const bool ext = chg_cur || chg_next || (P.pmask & (P_HEAT | P_ELASTIC)) || P.nion > 1;
  if (ext)
    launch_step_e<R, true>(P, T, S, cellid, chunk_lo, big, bkinfo, nbk, evlog, acc, dens, moments, scratch64, step,
                           chg_cur, chg_next, cap, st);
  else
    launch_step_e<R, false>(P, T, S, cellid, chunk_lo, big, bkinfo, nbk, evlog, acc, dens, moments, scratch64, step,
                            chg_cur, chg_next, cap, st);
}

bool step_batchable(const KParams &P, bool dens, bool grids) {
  return P.n > 0 && dens && (P.dmask & 7u) == 3u && !grids && !(P.pmask & (P_HEAT | P_ELASTIC)) && P.nion <= 1;
}

template <typename R>
void launch_step_batch(const StepBatch<R> &B, hipStream_t st) {
  if (B.n <= 0 || B.wg0[B.n] == 0) return;
  hipLaunchKernelGGL((k_step_batch<R>), dim3(B.wg0[B.n]), dim3(kFB), 0, st, B);
}

uint32_t step_batch_wgs(int64_t n, int64_t cap) { return (uint32_t)(kBigWG + step_nchunks(n, cap)); }

template <typename R>
void launch_set_job(const StepJob<R> &J, StepJob<R> *dst, hipStream_t st) {
  hipLaunchKernelGGL((k_set_job<R>), dim3(1), dim3(64), 0, st, J, dst);
}

void launch_set_words(const SetWords &w, hipStream_t st) {
  if (w.n > 0) hipLaunchKernelGGL(k_set_words, dim3(1), dim3(64), 0, st, w);
}

template void launch_step_batch<double>(const StepBatch<double> &, hipStream_t);
template void launch_step_batch<float>(const StepBatch<float> &, hipStream_t);
template void launch_set_job<double>(const StepJob<double> &, StepJob<double> *, hipStream_t);
template void launch_set_job<float>(const StepJob<float> &, StepJob<float> *, hipStream_t);

template void launch_step<double>(const KParams &, const Tables *, Soa<double>, const uint32_t *, const uint32_t *,
                                  const uint32_t *, const uint32_t *, const uint32_t *, uint8_t *, DevAccum *, double *,
                                  double *, uint64_t *, StepArg, const uint32_t *, uint32_t *, int64_t, hipStream_t);
template void launch_step<float>(const KParams &, const Tables *, Soa<float>, const uint32_t *, const uint32_t *,
                                 const uint32_t *, const uint32_t *, const uint32_t *, uint8_t *, DevAccum *, double *,
                                 double *, uint64_t *, StepArg, const uint32_t *, uint32_t *, int64_t, hipStream_t);

}  // namespace ecr
