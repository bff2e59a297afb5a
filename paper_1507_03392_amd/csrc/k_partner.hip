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
    if (tid == 0) atomicOr(&acc->err, ERR_PARTNER_OVERFLOW);
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
