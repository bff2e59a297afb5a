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
// Two kernels per step:
//  * k_coul_order: workgroup b owns the cells whose first slot lies in
//    [b*kCoulCap, (b+1)*kCoulCap) (slot ranges tabulated once per sort by
//    k_coul_chunks).  It first compacts the chunk's pool members (ions) into
//    LDS in slot order, so they are already grouped by cell, and the pool
//    order is found per cell without a general sort: a cell of m members
//    gets B = 2^floor(log2 m) buckets on the top bits of the uniform keys
//    (one or two members per bucket); an LDS histogram and scan place the
//    members bucket by bucket, and a member's exact position is its bucket
//    offset plus the number of bucket mates with a smaller (key, id).  Each
//    pair leader writes (slot a, slot b, pool size) into the chunk's own
//    region of the work list (pairs first, then the odd pools' triplets), and
//    the chunk's counts go to a per-chunk array: no global atomics.
//  * k_coul_pairs: one lane per pair (wavefront (b, y) takes pairs
//    64y..64y+63 of chunk b) and one lane per odd-pool triplet (a wavefront
//    gathers the triplets of kTriChunks chunks), with no LDS and no
//    barriers, so the long dependent FP64 chains and scattered loads of the
//    collisions are all in flight at once.  Pairs are disjoint, so no two
//    lanes touch one particle, and the item order does not change any
//    particle (it only regroups the FP64 momentum and energy sums).
#include "ecr_coll.hpp"
#include "ecr_kernels.hpp"
#include "ecr_wave.hpp"

namespace ecr {

// moment slots of a chunk: one per pair wavefront, one for triplets
constexpr int kMomentSlotsPerChunk = kCoulItems / 64 + 1;
// pair wavefronts per chunk (a chunk of 256 slots holds about 128 pairs)
constexpr int kPairRows = 2;
// chunks whose triplets are numbered together (about one odd pool per chunk
// where cells are populous, so one wavefront of 64 lanes takes them all)
constexpr int kTriChunks = 32;

constexpr int kCB = 256;               // lanes per ordering workgroup
constexpr int kEPT = kCoulMaxE / kCB;  // pool members per lane at most

struct CoulShared {
  uint64_t skey[kCoulMaxE];         // (key << 32) | slot of each pool member, in slot order
  uint32_t r1[kCoulMaxE + 2];       // member cells, then cell flags and scan scratch, then the bucket histogram
  uint16_t hd[kCoulMaxE];           // cell (head) index of each member
  uint16_t hcell[kCoulMaxE + 1];    // first member of each cell (steps 2-3), then its first bucket
  uint16_t ord[kCoulMaxE];          // members bucket by bucket
  uint32_t lead[kEPT * (kCB / 64)];  // leaders per (pass, wavefront): pairs | triplets << 16
  uint32_t wsum[kCB / 64];
  uint32_t grp[2][kEPT * (kCB / 64)];  // step 1's member counts per pass and wave, by group parity
};

// slot range of every chunk: the first slot of the first cell starting at or
// after b*cap (the cell holding that slot if it starts there, else the next
// one)
__global__ void k_coul_chunks(const uint32_t *__restrict__ cellid, const uint32_t *__restrict__ cell_off, int64_t n,
                              int64_t nchunks, int64_t cap, uint32_t *__restrict__ chunk_lo) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nchunks) return;
  const int64_t t = b * cap;
  if (t >= n) {
    chunk_lo[b] = (uint32_t)n;
    return;
  }
  const uint32_t c = cellid[t];
  const uint32_t st = cell_off[c];
  chunk_lo[b] = st == (uint32_t)t ? (uint32_t)t : cell_off[c + 1];
}

// the ordering of one chunk.  CMP: the chunk holds more than kCoulMaxE
// slots, so only its pool members (ions) are staged, compacted in slot
// order, with skey = (key << 32) | slot; else every slot is staged with
// skey = (key << 32) | id, atoms as entries in no pool.  Both give the same
// pool order and so the same work items.
template <typename R, bool CMP>
__device__ __forceinline__ void order_chunk(const KParams &P, Soa<R> S, const uint32_t *__restrict__ cellid,
                                            DevAccum *__restrict__ accum, CoulItem *__restrict__ items,
                                            uint2 *__restrict__ counts, uint32_t step, int64_t s_lo, int nsl,
                                            CoulShared &sh) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  // 1. the pool members (ions) of the chunk, compacted in slot order, with
  //    their pairing keys: skey = (key << 32) | slot, and the cell in r1.
  //    Atoms take no LDS, so a cell crowded with atoms (the gas inlet's,
  //    where recycled particles return) cannot overflow it; the capacity
  //    bounds the ions of a chunk
  constexpr int kLead = kEPT * (kCB / 64);  // (pass, wavefront) entries of a group
  static_assert(kLead <= 64, "per-wave counts fit one wavefront");
  const int wvu = __builtin_amdgcn_readfirstlane(wv);  // uniform over the wavefront
  int ns;  // entries: pool members (CMP), or every slot of the chunk
  bool pool[kEPT];
  uint32_t key[kEPT], myslot[kEPT], myid[kEPT];
  if constexpr (!CMP) {
    // a chunk that fits: every slot is an entry, (key << 32) | id in skey,
    // the cell in r1; atoms are entries that are in no pool
    ns = nsl;
#pragma unroll
    for (int k = 0; k < kEPT; ++k) {
      const int i = tid + k * kCB;
      pool[k] = false;
      key[k] = myslot[k] = myid[k] = 0u;
      if (i < ns) {
        const int64_t j = s_lo + i;
        const uint32_t id = S.pid[j];
        sh.r1[i] = cellid[j];
        pool[k] = q_of(S.qs[j]) >= 1;
        if (pool[k]) key[k] = draw(P, id, step, S_STEP, 0).z;
        sh.skey[i] = ((uint64_t)key[k] << 32) | id;
      }
    }
    __syncthreads();
  } else {
  uint32_t nm = 0;  // members so far, uniform over the workgroup
  // groups of kEPT passes of kCB slots (one group unless the chunk holds
  // more than kCoulMaxE slots): ballots, one barrier, then each member's
  // index from a scan of the per-wave counts
  for (int g0 = 0; g0 < nsl; g0 += kEPT * kCB) {
    uint32_t *gc = sh.grp[(g0 / (kEPT * kCB)) & 1];
    bool pl[kEPT];
    uint32_t cc[kEPT], kk[kEPT];
    uint64_t bm[kEPT];
#pragma unroll
    for (int k = 0; k < kEPT; ++k) {
      const int i = g0 + tid + k * kCB;
      pl[k] = false;
      cc[k] = kk[k] = 0u;
      if (i < nsl) {
        // the three loads issued together (one round of memory latency)
        const int64_t j = s_lo + i;
        const uint8_t qs = S.qs[j];
        const uint32_t id = S.pid[j];
        cc[k] = cellid[j];
        pl[k] = q_of(qs) >= 1;
        if (pl[k]) kk[k] = draw(P, id, step, S_STEP, 0).z;
      }
      bm[k] = __ballot(pl[k]);
      if (lane == 0) gc[k * (kCB / 64) + wv] = (uint32_t)__popcll(bm[k]);
    }
    __syncthreads();
    const uint32_t c = lane < kLead ? gc[lane] : 0u;
    const uint32_t incl = wave_incl_scan(c), excl = incl - c;
#pragma unroll
    for (int k = 0; k < kEPT; ++k) {
      const uint32_t m = nm + (uint32_t)__builtin_amdgcn_readlane((int)excl, k * (kCB / 64) + wvu) +
                         (uint32_t)__popcll(bm[k] & below);
      if (pl[k] && m < (uint32_t)kCoulMaxE) {
        sh.skey[m] = ((uint64_t)kk[k] << 32) | (uint32_t)(g0 + tid + k * kCB);
        sh.r1[m] = cc[k];
      }
    }
    nm += (uint32_t)__builtin_amdgcn_readlane((int)incl, kLead - 1);
  }
  if (nm <= 1u || nm > (uint32_t)kCoulMaxE) {
    if (tid == 0) {
      if (nm > (uint32_t)kCoulMaxE) atomicOr(&accum->err, ERR_COUL_OVERFLOW);
      counts[blockIdx.x] = make_uint2(0u, 0u);
    }
    return;
  }
  __syncthreads();  // the members are in LDS
  // from here on an index i counts the chunk's pool members (in slot order)
  ns = (int)nm;
  // each lane's members: key, slot, and the particle id (loaded now, used
  // by the work items at the end, so the load's latency is hidden)
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const int i = tid + k * kCB;
    pool[k] = i < ns;
    const uint64_t sk = pool[k] ? sh.skey[i] : 0ull;
    key[k] = (uint32_t)(sk >> 32);
    myslot[k] = (uint32_t)sk;
    myid[k] = pool[k] ? S.pid[s_lo + myslot[k]] : 0u;
  }
  }
  // one array serves twice: the cells' first entries are last read in step
  // 3, before the scan after which their first buckets are written (18.5 KB
  // of LDS in all, so eight workgroups share a CU)
  uint16_t *const hstart = sh.hcell, *const hbase = sh.hcell;
  // 2. cells of the members: heads (ballots per pass and wave, one
  //    barrier, a scan of the counts), cell index of every member, first
  //    member of every cell
  uint32_t fl[kEPT];
  uint64_t hb[kEPT];
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const int i = tid + k * kCB;
    fl[k] = (i < ns && (i == 0 || sh.r1[i] != sh.r1[i - 1])) ? 1u : 0u;
    hb[k] = __ballot(fl[k] != 0u);
    if (lane == 0) sh.lead[k * (kCB / 64) + wv] = (uint32_t)__popcll(hb[k]);
  }
  __syncthreads();
  const uint32_t hc = lane < kLead ? sh.lead[lane] : 0u;
  const uint32_t hincl = wave_incl_scan(hc), hexcl = hincl - hc;
  const int nheads = __builtin_amdgcn_readlane((int)hincl, kLead - 1);
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const int i = tid + k * kCB;
    if (i < ns) {
      const int h = __builtin_amdgcn_readlane((int)hexcl, k * (kCB / 64) + wvu) + (int)__popcll(hb[k] & below) +
                    (int)fl[k] - 1;
      sh.hd[i] = (uint16_t)h;
      if (fl[k]) hstart[h] = (uint16_t)i;
    }
  }
  if (tid == 0) hstart[nheads] = (uint16_t)ns;
  __syncthreads();
  // 3. buckets per cell: B = 2^floor(log2(members of the cell)), so at most
  //    one bucket per member
  for (int h = tid; h < nheads; h += kCB) {
    const int m = hstart[h + 1] - hstart[h];
    const int lg = m <= 1 ? 0 : 31 - __clz(m);
    sh.r1[h] = 1u << lg;
  }
  __syncthreads();
  const int nbuckets = (int)wg_exscan<kCB>(sh.r1, nheads, sh.wsum);
  for (int h = tid; h < nheads; h += kCB) hbase[h] = (uint16_t)sh.r1[h];
  if (tid == 0) hbase[nheads] = (uint16_t)nbuckets;
  __syncthreads();
  // 4-5. histogram of the pool members over their cell's buckets
  uint32_t *hist = sh.r1;
  for (int i = tid; i <= nbuckets; i += kCB) hist[i] = 0u;
  __syncthreads();
  int bk[kEPT], arr[kEPT];
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const int i = tid + k * kCB;
    bk[k] = 0;
    arr[k] = 0;
    if (i < ns && pool[k]) {
      const int h = sh.hd[i];
      const int lg = 31 - __clz(hbase[h + 1] - hbase[h]);  // the cell's 2^lg buckets
      bk[k] = hbase[h] + (lg ? (int)(key[k] >> (32 - lg)) : 0);
      arr[k] = (int)atomicAdd(&hist[bk[k]], 1u);
    }
  }
  __syncthreads();
  // 6-7. bucket offsets, members listed bucket by bucket
  const int npool = (int)wg_exscan<kCB>(hist, nbuckets, sh.wsum);
  if (tid == 0) hist[nbuckets] = (uint32_t)npool;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const int i = tid + k * kCB;
    if (i < ns && pool[k]) sh.ord[hist[bk[k]] + arr[k]] = (uint16_t)i;
  }
  __syncthreads();
  // 8. exact pool position: bucket offset + bucket mates with a smaller
  //    (key, id); equal keys (rare) fetch the two ids
  auto precedes = [&](uint64_t o, uint64_t me) -> int {
    const uint32_t ko = (uint32_t)(o >> 32), km = (uint32_t)(me >> 32);
    if (ko != km || o == me) return ko < km ? 1 : 0;  // (o == me: the member itself)
    return S.pid[s_lo + (uint32_t)o] < S.pid[s_lo + (uint32_t)me] ? 1 : 0;
  };
  int pos[kEPT], rr[kEPT], mm[kEPT];
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const int i = tid + k * kCB;
    pos[k] = rr[k] = mm[k] = 0;
    if (i < ns && pool[k]) {
      const uint64_t me = sh.skey[i];
      const int b0 = (int)hist[bk[k]], b1 = (int)hist[bk[k] + 1];
      int rib = 0;
      if constexpr (CMP) {
        for (int t = b0; t < b1; ++t) rib += precedes(sh.skey[sh.ord[t]], me);
      } else {
        for (int t = b0; t < b1; ++t) rib += sh.skey[sh.ord[t]] < me ? 1 : 0;
      }
      pos[k] = b0 + rib;
      const int h = sh.hd[i];
      const int pstart = (int)hist[hbase[h]];
      const int pend = (int)hist[hbase[h + 1]];
      mm[k] = pend - pstart;
      rr[k] = pos[k] - pstart;
    }
  }
  __syncthreads();
  // 9. pool order (element of every pool position), and the pair and
  //    triplet leaders counted per pass and wavefront for step 10 (one
  //    barrier for both)
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const int i = tid + k * kCB;
    if (i < ns && pool[k]) sh.ord[pos[k]] = (uint16_t)i;
  }
  const int nk = (ns + kCB - 1) / kCB;  // passes that hold members
  int lt[kEPT], li[kEPT];
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const int i = tid + k * kCB;
    lt[k] = 0;
    li[k] = 0;
    if (k < nk) {  // uniform over the workgroup
      if (i < ns && pool[k]) {
        const int m = mm[k], r = rr[k];
        if (m >= 2) {
          if ((m & 1) && r == 0) lt[k] = 2;                              // triplet
          else if ((m & 1) ? (r >= 3 && (r & 1)) : !(r & 1)) lt[k] = 1;  // pair
        }
      }
      const uint64_t bp = __ballot(lt[k] == 1), bt = __ballot(lt[k] == 2);
      li[k] = __popcll((lt[k] == 2 ? bt : bp) & below);
      if (lane == 0) sh.lead[k * (kCB / 64) + wv] = (uint32_t)__popcll(bp) | ((uint32_t)__popcll(bt) << 16);
    }
  }
  __syncthreads();
  // 10. pair leaders write their work items into the chunk's own list region:
  //     pairs first, then the odd pools' triplets, each numbered in the slot
  //     order of its leader, hence cell by cell: the chunk's first pair
  //     wavefront then takes the cells at its front and the second those at
  //     its back, so the two share few cache lines of the state (the items
  //     are disjoint, so their order does not change any particle)
  // exclusive scan of the leader counts in (pass, wavefront) order, which is
  // slot order; pairs and triplets side by side in one word (each at most
  // kCoulItems, so the low half never carries into the high one)
  const uint32_t c = lane < nk * (kCB / 64) ? sh.lead[lane] : 0u;
  const uint32_t incl = wave_incl_scan(c), excl = incl - c;
  const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, kLead - 1);
  const int np = (int)(tot & 0xffffu);
  uint32_t before[kEPT];
#pragma unroll
  for (int k = 0; k < kEPT; ++k) before[k] = (uint32_t)__builtin_amdgcn_readlane((int)excl, k * (kCB / 64) + wvu);
  CoulItem *out = items + (int64_t)blockIdx.x * kCoulItems;
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    if (lt[k]) {
      const int p = pos[k];
      CoulItem e;
      if constexpr (CMP) {
        e.a = (uint16_t)myslot[k];  // the leader is the member at pool position p
        e.b = (uint16_t)sh.skey[sh.ord[p + 1]];  // member -> its slot in the chunk
        e.c = lt[k] == 2 ? (uint16_t)sh.skey[sh.ord[p + 2]] : (uint16_t)0;
        e.id = myid[k];
      } else {
        e.a = sh.ord[p];
        e.b = sh.ord[p + 1];
        e.c = lt[k] == 2 ? sh.ord[p + 2] : (uint16_t)0;
        e.id = (uint32_t)sh.skey[e.a];
      }
      e.m = (uint16_t)mm[k];
      out[lt[k] == 1 ? (int)(before[k] & 0xffffu) + li[k] : np + (int)(before[k] >> 16) + li[k]] = e;
    }
  }
  if (tid == 0) counts[blockIdx.x] = make_uint2((uint32_t)np, tot >> 16);
}

template <typename R>
__global__ void __launch_bounds__(kCB) k_coul_order(KParams P, Soa<R> S, const uint32_t *__restrict__ cellid,
                                                    const uint32_t *__restrict__ chunk_lo,
                                                    DevAccum *__restrict__ accum, CoulItem *__restrict__ items,
                                                    uint2 *__restrict__ counts, StepArg sa,
                                                    uint32_t *__restrict__ zero, int64_t zero_n) {
  __shared__ CoulShared sh;
  const uint32_t step = sa.get();
  const int tid = threadIdx.x;
  if (zero) {
    // the next step's cell grids, cleared here, a slice per workgroup,
    // instead of by a kernel of their own (the push fills them afterwards)
    const int64_t per = (zero_n + gridDim.x - 1) / gridDim.x;
    const int64_t z0 = (int64_t)blockIdx.x * per, z1 = min(z0 + per, zero_n);
    for (int64_t t = z0 + tid; t < z1; t += kCB) zero[t] = 0u;
  }
  const int64_t s_lo = chunk_lo[blockIdx.x];
  const int nsl = (int)((int64_t)chunk_lo[blockIdx.x + 1] - s_lo);  // slots of the chunk
  if (nsl <= 1 || nsl > 0xffff) {  // no pool, or slots past the items' 16-bit fields
    if (tid == 0) {
      if (nsl > 0xffff) atomicOr(&accum->err, ERR_COUL_OVERFLOW);
      counts[blockIdx.x] = make_uint2(0u, 0u);
    }
    return;
  }
  if (nsl <= kCoulMaxE) order_chunk<R, false>(P, S, cellid, accum, items, counts, step, s_lo, nsl, sh);
  else order_chunk<R, true>(P, S, cellid, accum, items, counts, step, s_lo, nsl, sh);
}

// collisions, one per lane, so that every collision of the step is in
// flight at once.  Grid (nchunks, 1 + kPairRows), one wavefront per
// workgroup.  Row 0
// holds the triplet waves: the triplets of a group of kTriChunks chunks are
// numbered in chunk order, and wave k of the group (column k * ngroups + g
// for group g) runs numbers 64k..64k+63 (then 64(k + nw).. if the group has
// more), one triplet per lane, three dependent collisions each ((a,b),
// (b,c), (c,a) with dt/2).  The k = 0 waves, usually the only busy ones, thus
// sit side by side at the front, spread over the XCDs (consecutive
// workgroups go to different XCDs), and start before the pair waves;
// row 1 + y, column b takes pairs 64y..64y+63 of chunk b (then
// 64(y + kPairRows).. if the chunk has more).  Triplets and pairs touch
// disjoint particles.  At most 4 waves per SIMD: the triplet path alone
// would need a few more registers than that allows, for nothing.
template <typename R>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))
k_coul_pairs(KParams P, const Tables *__restrict__ T, Soa<R> S,
                                                   const uint32_t *__restrict__ chunk_lo,
                                                   const CoulItem *__restrict__ items,
                                                   const uint2 *__restrict__ counts, double *__restrict__ moments,
                                                   StepArg sa, int64_t nchunks) {
  const uint32_t step = sa.get();
  const int lane = (int)threadIdx.x;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (blockIdx.y == 0) {
    // triplet wave kw of the group starting at chunk b: lane j < kTriChunks
    // holds chunk b + j's first slot, pair count and inclusive triplet prefix
    const int64_t ngroups = (nchunks + kTriChunks - 1) / kTriChunks;
    const int64_t g = (int64_t)blockIdx.x % ngroups;
    const int kw = (int)((int64_t)blockIdx.x / ngroups);
    const int nw = (int)((nchunks - 1 - g) / ngroups) + 1;  // waves serving group g
    const int64_t b = g * kTriChunks;
    uint32_t my_lo = 0, my_np = 0, nt = 0;
    if (lane < kTriChunks && b + lane < nchunks) {
      my_lo = chunk_lo[b + lane];
      const int ns = (int)(chunk_lo[b + lane + 1] - my_lo);
      if (ns > 1) {  // else no pool (an overflowing chunk has zero counts, flagged by the ordering)
        const uint2 c = counts[b + lane];
        my_np = c.x;
        nt = c.y;
      }
    }
    static_assert(kTriChunks <= 64, "a group's chunks fit one wavefront");
    const uint32_t my_incl = wave_incl_scan(nt);  // lanes >= kTriChunks hold nt = 0
    const int total = __builtin_amdgcn_readlane((int)my_incl, kTriChunks - 1);
    if (kw * 64 >= total) return;
    const double h = 0.5 * P.dt;
    for (int q0 = kw * 64; q0 < total; q0 += 64 * nw) {
      const int q = q0 + lane;
      int c = 0;  // the lane's triplet is number q - incl[c-1] of chunk b + c
#pragma unroll
      for (int j = 0; j < kTriChunks; ++j) c += __builtin_amdgcn_readlane((int)my_incl, j) <= q ? 1 : 0;
      const int cc = c < kTriChunks ? c : kTriChunks - 1;  // c < kTriChunks when q < total
      const uint32_t prev = __shfl(my_incl, cc > 0 ? cc - 1 : 0, 64);
      const uint32_t lo = __shfl(my_lo, cc, 64), np = __shfl(my_np, cc, 64);
      if (q < total) {
        const CoulItem e = items[(b + c) * kCoulItems + np + ((uint32_t)q - (cc > 0 ? prev : 0u))];
        const double nc = (double)e.m * P.nfac;
        const uint32_t ia = lo + e.a, ib = lo + e.b, ic = lo + e.c;
        collide<R>(P, T->lnA, S, ia, ib, e.id, nc, h, step, acc, true, true);
        collide<R>(P, T->lnA, S, ib, ic, S.pid[ib], nc, h, step, acc, false, true);
        collide<R>(P, T->lnA, S, ic, ia, S.pid[ic], nc, h, step, acc, false, false);
      }
    }
    // each triplet wave owns the triplet slot of the chunk its column names
    double *slot = moments + ((int64_t)blockIdx.x * kMomentSlotsPerChunk + kMomentSlotsPerChunk - 1) * 5;
    for (int k = 0; k < 5; ++k) {
      const double v = wave_sum_last(acc[k]);
      if (lane == 63 && v != 0.0) slot[k] += v;
    }
    return;
  }
  const int64_t b = blockIdx.x;
  const int y = (int)blockIdx.y - 1;
  const int64_t s_lo = chunk_lo[b];
  const int ns = (int)((int64_t)chunk_lo[b + 1] - s_lo);
  if (ns <= 1) return;
  const int np = (int)counts[b].x;
  if (y * 64 >= np) return;
  // rows beyond kPairRows are folded onto these (rare: > 64 kPairRows pairs)
#pragma unroll 1
  for (int q = y * 64 + lane; q < np; q += 64 * kPairRows) {
    const CoulItem e = items[b * kCoulItems + q];
    collide<R>(P, T->lnA, S, (uint32_t)s_lo + e.a, (uint32_t)s_lo + e.b, e.id, (double)e.m * P.nfac, P.dt, step, acc,
               true, true);
  }
  // each pair wavefront owns one slot of the moment buffer: plain
  // read-add-write, no contended atomics (summed in a fixed order when
  // tallies are read)
  double *slot = moments + (b * kMomentSlotsPerChunk + y) * 5;
  for (int k = 0; k < 5; ++k) {
    const double v = wave_sum_last(acc[k]);
    if (lane == 63 && v != 0.0) slot[k] += v;
  }
}

// fixed-order sum of the per-wavefront moment slots into the tallies
__global__ void __launch_bounds__(256) k_sum_moments(const double *__restrict__ moments, int64_t nslots,
                                                     DevAccum *__restrict__ accum) {
  __shared__ double red[5][256];
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = threadIdx.x; i < nslots; i += 256)
    for (int k = 0; k < 5; ++k) s[k] += moments[i * 5 + k];
  for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    accum->t.coul_dp[0] = red[0][0];
    accum->t.coul_dp[1] = red[1][0];
    accum->t.coul_dp[2] = red[2][0];
    accum->t.coul_de = red[3][0];
    accum->t.coul_e = red[4][0];
  }
}

int64_t coul_moment_slots(int64_t n) { return ((n + kCoulCap - 1) / kCoulCap) * kMomentSlotsPerChunk; }

void launch_sum_moments(const double *moments, int64_t nslots, DevAccum *acc, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_moments, dim3(1), dim3(256), 0, st, moments, nslots, acc);
}

int64_t coul_nchunks(int64_t n) { return (n + kCoulCap - 1) / kCoulCap; }

void launch_coul_chunks(const uint32_t *cellid, const uint32_t *cell_off, int64_t n, uint32_t *chunk_lo, int64_t cap,
                        hipStream_t st) {
  const int64_t nc = (n + cap - 1) / cap;
  hipLaunchKernelGGL(k_coul_chunks, dim3((unsigned)((nc + 1 + 255) / 256)), dim3(256), 0, st, cellid, cell_off, n, nc,
                     cap, chunk_lo);
}

template <typename R>
void launch_coul_order(const KParams &P, Soa<R> S, const uint32_t *cellid, const uint32_t *chunk_lo, DevAccum *acc,
                       CoulItem *items, uint2 *counts, StepArg step, uint32_t *zero, int64_t zero_n,
                       hipStream_t st) {
  if (P.n <= 1) return;
  hipLaunchKernelGGL(k_coul_order<R>, dim3((unsigned)coul_nchunks(P.n)), dim3(kCB), 0, st, P, S, cellid, chunk_lo, acc,
                     items, counts, step, zero, zero_n);
}

template <typename R>
void launch_coul_pairs(const KParams &P, const Tables *T, Soa<R> S, const uint32_t *chunk_lo, const CoulItem *items,
                       const uint2 *counts, double *moments, StepArg step, hipStream_t st) {
  if (P.n <= 1) return;
  const int64_t nc = coul_nchunks(P.n);
  hipLaunchKernelGGL(k_coul_pairs<R>, dim3((unsigned)nc, 1 + kPairRows), dim3(64), 0, st, P, T, S, chunk_lo,
                     items, counts, moments, step, nc);
}

template void launch_coul_order<double>(const KParams &, Soa<double>, const uint32_t *, const uint32_t *, DevAccum *,
                                        CoulItem *, uint2 *, StepArg, uint32_t *, int64_t, hipStream_t);
template void launch_coul_order<float>(const KParams &, Soa<float>, const uint32_t *, const uint32_t *, DevAccum *,
                                       CoulItem *, uint2 *, StepArg, uint32_t *, int64_t, hipStream_t);
template void launch_coul_pairs<double>(const KParams &, const Tables *, Soa<double>, const uint32_t *,
                                        const CoulItem *, const uint2 *, double *, StepArg, hipStream_t);
template void launch_coul_pairs<float>(const KParams &, const Tables *, Soa<float>, const uint32_t *, const CoulItem *,
                                       const uint2 *, double *, StepArg, hipStream_t);

}  // namespace ecr
