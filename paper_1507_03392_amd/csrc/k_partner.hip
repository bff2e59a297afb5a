// k_partner.hip -- tracked exchange partners (Mironov et al., Sec. II: the
// atoms are tracked macro-particles, so a charge exchange takes its electron
// from one of them).
//
// After the push of a step with ECR_FLAG_CX_PARTNER, cxreq[s][c] holds the
// exchanges of species s whose ion sits in collision cell c (the cell at the
// last sort).  One workgroup per Coulomb chunk (the cells whose first sorted
// slot lies in [b*kCoulCap, (b+1)*kCoulCap)), so each cell has exactly one
// owner:
//  0. a chunk none of whose cells holds a request (the push flags the
//     others) returns at once;
//  1. every slot puts its cell in LDS; an atom that did not become one in
//     this step (birth != step) and whose species has requests in its cell
//     is a candidate and also puts (key, id) there, key = word 3 of its
//     stream-1 draw;
//  2. the first slot of each cell counts the cell's candidates of each
//     requesting species, adds the requests beyond them to cx_unmatched and
//     clears the requests for the next step;
//  3. a candidate whose rank by (key, id) among its cell's candidates of its
//     species is below the requests becomes a Q = 1 ion born in the step;
//     the next step's cell grids move one unit from the species' atom
//     channel to the ion charge channel of the cell it is in.
// The work is proportional to the requesting cells only; the default step
// never launches it.
//
// A chunk of more slots than the LDS holds (the gas inlet's cell gathers
// thousands of recycled atoms in long runs) takes the same decisions from
// global memory instead: cell by cell, for each requesting species, the
// workgroup picks the candidates of lowest (key, id) one at a time by
// minimum reductions over the cell, each bounded below by the previous
// pick.  The candidates of rank below the requests are the same ones, so
// the result does not depend on the path; the cost is one pass over the
// cell per request, and requests are rare.
#include "ecr_kernels.hpp"

namespace ecr {

namespace {

constexpr int kPB = 256;  // lanes per workgroup
// slots a chunk may hold: four times the Coulomb ordering's, since the
// candidates are atoms and the gas inlet's cell gathers recycled atoms
// (about 2000 at 2M ions after 50k steps); 53 KB of LDS, but a workgroup
// without requests returns after one load
constexpr int kPMaxE = 4 * kCoulMaxE;
constexpr int kPEPT = kPMaxE / kPB;  // slots per lane at most

struct PartnerShared {
  uint64_t kv[kPMaxE];    // (key << 32) | id of a candidate
  uint32_t cell[kPMaxE];  // collision cell of every slot of the chunk
  uint8_t spc[kPMaxE];    // species of a candidate, 0xFF for any other slot
};

// the smallest of the workgroup's 64-bit values (all lanes call it)
__device__ __forceinline__ uint64_t wg_min_u64(uint64_t v, uint64_t *red) {
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  __syncthreads();  // red may still be read by the previous call
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t m = red[0];
  for (int w = 1; w < kPB / 64; ++w) m = red[w] < m ? red[w] : m;
  return m;
}

// a chunk beyond the LDS capacity: every decision from global memory
template <typename R>
__device__ void partner_chunk_global(const KParams &P, Soa<R> S, int64_t s_lo, int64_t s_hi,
                                     uint32_t *__restrict__ chg, uint8_t *__restrict__ evlog,
                                     DevAccum *__restrict__ acc, uint32_t step, uint64_t *red) {
  const int tid = threadIdx.x;
  int64_t c_lo = s_lo;
  while (c_lo < s_hi) {  // uniform: every lane walks the same cells
    const uint32_t c = P.cellid[c_lo];
    const int64_t c_hi = (int64_t)P.cell_off[c + 1];
    for (int s = 0; s < P.nspecies; ++s) {
      const uint32_t r = P.cxreq[(uint32_t)s * P.ncell + c];
      if (r == 0u) continue;
      uint32_t got = 0u;
      uint64_t prev = 0ull;
      bool first = true;
      for (; got < r; ++got) {
        // the smallest (key, id) above the previous pick among the cell's
        // atoms of species s that did not become atoms in this step
        uint64_t best = ~0ull;
        for (int64_t j = c_lo + tid; j < c_hi; j += kPB) {
          const uint8_t qs = S.qs[j];
          if (q_of(qs) != 0 || sp_of(qs) != s || S.birth[j] == step) continue;
          const uint32_t id = S.pid[j];
          const uint64_t kv = ((uint64_t)draw(P, id, step, S_STEP, 0).w << 32) | id;
          if ((first || kv > prev) && kv < best) best = kv;
        }
        const uint64_t m = wg_min_u64(best, red);
        if (m == ~0ull) break;  // no candidate left (an id is below 2^31, so no real key is ~0)
        prev = m;
        first = false;
        // the owner of the pick converts it
        for (int64_t j = c_lo + tid; j < c_hi; j += kPB) {
          if (S.pid[j] != (uint32_t)m) continue;
          S.qs[j] = make_qs(1, s);
          S.birth[j] = step;
          if (evlog) evlog[j] = EV_CX_PARTNER;
          const uint32_t cc = cell_of<R>(P, S.x[j], S.y[j], S.z[j]);
          atomicAdd(&chg[cc], 1u);
          atomicSub(&chg[(uint32_t)(1 + s) * P.ncell + cc], 1u);
        }
      }
      __syncthreads();  // every lane has read the request before it is cleared
      if (tid == 0) {
        if (r > got) atomicAdd((unsigned long long *)&acc->t.cx_unmatched[s], (unsigned long long)(r - got));
        P.cxreq[(uint32_t)s * P.ncell + c] = 0u;
      }
    }
    c_lo = c_hi;
  }
}

}  // namespace

template <typename R>
__global__ void __launch_bounds__(kPB) k_cx_partner(KParams P, Soa<R> S, const uint32_t *__restrict__ chunk_lo,
                                                    uint32_t *__restrict__ chg, uint8_t *__restrict__ evlog,
                                                    DevAccum *__restrict__ acc, StepArg sa) {
  __shared__ PartnerShared sh;
  const uint32_t step = sa.get();
  const int tid = threadIdx.x;
  const int64_t s_lo = chunk_lo[blockIdx.x];
  const int ns = (int)((int64_t)chunk_lo[blockIdx.x + 1] - s_lo);
  if (ns <= 0 || P.cxchunk[blockIdx.x] == 0u) return;
  if (ns > kPMaxE) {
    __shared__ uint64_t red[kPB / 64];
    partner_chunk_global<R>(P, S, s_lo, s_lo + ns, chg, evlog, acc, step, red);
    __syncthreads();
    if (tid == 0) P.cxchunk[blockIdx.x] = 0u;
    return;
  }
  // 1. cells and candidates
  uint32_t want[kPEPT];
#pragma unroll
  for (int k = 0; k < kPEPT; ++k) {
    const int i = tid + k * kPB;
    want[k] = 0u;
    if (i < ns) {
      const int64_t j = s_lo + i;
      const uint32_t c = P.cellid[j];
      const uint8_t qs = S.qs[j];
      uint8_t sp = 0xFF;
      sh.cell[i] = c;
      if (q_of(qs) == 0 && S.birth[j] != step) {
        want[k] = P.cxreq[(uint32_t)sp_of(qs) * P.ncell + c];
        if (want[k]) {
          const uint32_t id = S.pid[j];
          sp = (uint8_t)sp_of(qs);
          sh.kv[i] = ((uint64_t)draw(P, id, step, S_STEP, 0).w << 32) | id;
        }
      }
      sh.spc[i] = sp;
    }
  }
  __syncthreads();
  if (tid == 0) P.cxchunk[blockIdx.x] = 0u;  // every lane has read it
  // 2. the first slot of a cell settles the cell's requests; it reads them
  //    first and walks the cell only when there are any (requests are
  //    rare, cells in the zone hold a hundred slots or more)
#pragma unroll
  for (int k = 0; k < kPEPT; ++k) {
    const int i = tid + k * kPB;
    if (i < ns && (i == 0 || sh.cell[i - 1] != sh.cell[i])) {
      const uint32_t c = sh.cell[i];
      uint32_t r[kMaxS];
      bool any = false;
#pragma unroll
      for (int s = 0; s < kMaxS; ++s) {
        r[s] = s < P.nspecies ? P.cxreq[(uint32_t)s * P.ncell + c] : 0u;
        any = any || r[s] != 0u;
      }
      if (any) {
        int e = i + 1;
        while (e < ns && sh.cell[e] == c) ++e;
#pragma unroll
        for (int s = 0; s < kMaxS; ++s) {
          if (r[s] == 0u) continue;
          uint32_t m = 0u;
          for (int t = i; t < e; ++t) m += sh.spc[t] == (uint8_t)s ? 1u : 0u;
          if (r[s] > m) atomicAdd((unsigned long long *)&acc->t.cx_unmatched[s], (unsigned long long)(r[s] - m));
          P.cxreq[(uint32_t)s * P.ncell + c] = 0u;
        }
      }
    }
  }
  // 3. the candidates of lowest (key, id) become ions
#pragma unroll
  for (int k = 0; k < kPEPT; ++k) {
    const int i = tid + k * kPB;
    if (i < ns && want[k]) {
      const uint32_t c = sh.cell[i];
      const uint8_t sp = sh.spc[i];
      const uint64_t me = sh.kv[i];
      int b = i;
      while (b > 0 && sh.cell[b - 1] == c) --b;
      uint32_t rank = 0u;
      for (int t = b; t < ns && sh.cell[t] == c; ++t) rank += (sh.spc[t] == sp && sh.kv[t] < me) ? 1u : 0u;
      if (rank < want[k]) {
        const int64_t j = s_lo + i;
        S.qs[j] = make_qs(1, sp);
        S.birth[j] = step;
        if (evlog) evlog[j] = EV_CX_PARTNER;
        const uint32_t cc = cell_of<R>(P, S.x[j], S.y[j], S.z[j]);
        atomicAdd(&chg[cc], 1u);
        atomicSub(&chg[(uint32_t)(1 + sp) * P.ncell + cc], 1u);
      }
    }
  }
}

template <typename R>
void launch_cx_partner(const KParams &P, Soa<R> S, const uint32_t *chunk_lo, uint32_t *chg, uint8_t *evlog,
                       DevAccum *acc, StepArg step, hipStream_t st) {
  if (P.n <= 0) return;
  hipLaunchKernelGGL(k_cx_partner<R>, dim3((unsigned)coul_nchunks(P.n)), dim3(kPB), 0, st, P, S, chunk_lo, chg,
                     evlog, acc, step);
}

template void launch_cx_partner<double>(const KParams &, Soa<double>, const uint32_t *, uint32_t *, uint8_t *,
                                        DevAccum *, StepArg, hipStream_t);
template void launch_cx_partner<float>(const KParams &, Soa<float>, const uint32_t *, uint32_t *, uint8_t *,
                                       DevAccum *, StepArg, hipStream_t);

}  // namespace ecr
