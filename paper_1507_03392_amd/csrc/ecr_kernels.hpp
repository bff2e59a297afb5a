// ecr_kernels.hpp -- launch entry points of the gfx950 kernels (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ecr_device.hpp"
#include "ecrpic.h"

namespace ecr {

// Coulomb chunking: a workgroup owns the cells whose first sorted slot falls
// in [b*kCoulCap, (b+1)*kCoulCap); it orders up to kCoulMaxE pool members
// (ions; atoms take no room) in LDS.
constexpr int kCoulCap = 256;
constexpr int kCoulMaxE = 1024;
// the fused step kernel's chunks: the cells whose first sorted slot falls in
// [b*cap, (b+1)*cap), cap = step_fcap(n, resident) (kFCap or kFCapLo from
// 98 304 particles up, whichever fills the last round of resident
// workgroups more; smaller runs get smaller chunks, down to 64 slots, so that
// they still spread over the CUs); a chunk of at most 1024 slots is stepped
// by its own workgroup, a larger one by a handler workgroup
constexpr int kFCap = 768;
constexpr int kFCapLo = 736;

static_assert(kBirthNone == ECR_BIRTH_NONE, "birth sentinel");

// Error bits raised by kernels (read back with the tallies).
enum : uint32_t { ERR_COUL_OVERFLOW = 1, ERR_PARTNER_OVERFLOW = 2 };

struct DevAccum {
  ecr_tallies t;           // steps field unused on the device
  uint32_t err;            // ERR_* bits
  uint32_t pad[63];
};

// one Coulomb work item of a chunk: chunk-relative slots a, b (and c for an
// odd pool's triplet), the pool size m and the id of a; a chunk owns
// kCoulItems items
struct CoulItem {
  uint16_t a, b, c, m;
  uint32_t id;
};
constexpr int kCoulItems = kCoulMaxE / 2;

template <typename R>
void launch_init(const KParams &P, Soa<R> S, hipStream_t st);

// push + wall/aperture + MCC; also deposits when dens != nullptr; with
// chg_cur, ionisation uses the cell's ion charge (self-consistent n_e) and
// the updated charges are summed per cell into chg_next (zeroed before)
template <typename R>
void launch_push(const KParams &P, const Tables *T, Soa<R> S, const double *ef, uint8_t *evlog,
                 DevAccum *acc, double *dens, StepArg step, const uint32_t *chg_cur, uint32_t *chg_next,
                 hipStream_t st);

// exchange partners (ECR_FLAG_CX_PARTNER): per Coulomb chunk, the atoms of
// each requesting collision cell become ions in (key, id) order; chg is the
// next step's cell grids, updated for the new charges; the requests are
// cleared
template <typename R>
void launch_cx_partner(const KParams &P, Soa<R> S, const uint32_t *chunk_lo, uint32_t *chg, uint8_t *evlog,
                       DevAccum *acc, StepArg step, hipStream_t st);

// |B| at every cell centre times hx, into bden[ncell] (once, at create)
void launch_cell_bden(const KParams &P, double *bden, hipStream_t st);

// ion charge per cell of the current state, added into chg (zeroed before)
template <typename R>
void launch_charge_grid(const KParams &P, Soa<R> S, uint32_t *chg, hipStream_t st);

template <typename R>
void launch_deposit(const KParams &P, Soa<R> S, double *dens, hipStream_t st);

// optional ion pressure moment (field ECR_F_ION_P)
template <typename R>
void launch_deposit_pressure(const KParams &P, Soa<R> S, double *dens, hipStream_t st);

// Coulomb chunk table: chunk b covers slots [chunk_lo[b], chunk_lo[b+1]),
// nchunks+1 entries, rebuilt after every sort
int64_t coul_nchunks(int64_t n);
void launch_coul_chunks(const uint32_t *cellid, const uint32_t *cell_off, int64_t n, uint32_t *chunk_lo, int64_t cap,
                        hipStream_t st);

// pairing (k_coul_order) then collisions (k_coul_pairs); items holds
// kCoulItems entries per chunk, counts one (pairs, triplets) per chunk
// moments: coul_moment_slots(n) x 5 doubles of per-wavefront momentum /
// energy sums, reduced into the tallies by launch_sum_moments.  The ordering
// kernel also clears zero[0..zero_n) (the next step's cell grids) when zero
// is given; it does nothing at all for n <= 1
template <typename R>
void launch_coul_order(const KParams &P, Soa<R> S, const uint32_t *cellid, const uint32_t *chunk_lo, DevAccum *acc,
                       CoulItem *items, uint2 *counts, StepArg step, uint32_t *zero, int64_t zero_n,
                       hipStream_t st);
template <typename R>
void launch_coul_pairs(const KParams &P, const Tables *T, Soa<R> S, const uint32_t *chunk_lo, const CoulItem *items,
                       const uint2 *counts, double *moments, StepArg step, hipStream_t st);
int64_t coul_moment_slots(int64_t n);
void launch_sum_moments(const double *moments, int64_t nslots, DevAccum *acc, hipStream_t st);

// the whole step in one kernel (Coulomb pairing and collisions, push,
// wall/aperture loss, MCC, deposit) over the chunks of the fused table
// (chunk_lo, step_nchunks(n, cap) + 1 entries for the chunk size cap of the
// table; big: the oversized chunks, made by
// launch_big_list at the sort); moments as for the Coulomb kernels;
// scratch64: n 64-bit words of sort space for pools beyond the LDS.  With
// chg_next, it must have been zeroed before.
// At each sort, launch_step_prep lists the oversized chunks (big) and
// tabulates the ordering's buckets of every other chunk: per slot
// (bkinfo[n]) first bucket | log2(bucket count) << 16 of its cell, per chunk
// (nbk[nchunks]) the bucket total.
// resident: the step workgroups the device holds at once (step_resident_wgs;
// 0 when unknown)
int64_t step_fcap(int64_t n, int64_t resident);
int64_t step_nchunks(int64_t n, int64_t cap);
// the most chunks step_fcap can give n particles (the tables' size)
int64_t step_nchunks_max(int64_t n);
int64_t step_resident_wgs(bool fp32);
// moment slots the fused step writes (one per wavefront of a chunk)
int64_t step_moment_slots(int64_t n);
void launch_step_prep(const uint32_t *cellid, const uint32_t *chunk_lo, int64_t n, int64_t cap, uint32_t *big,
                      uint32_t *bkinfo, uint32_t *nbk, hipStream_t st);
template <typename R>
void launch_step(const KParams &P, const Tables *T, Soa<R> S, const uint32_t *cellid, const uint32_t *chunk_lo,
                 const uint32_t *big, const uint32_t *bkinfo, const uint32_t *nbk, uint8_t *evlog, DevAccum *acc,
                 double *dens, double *moments, uint64_t *scratch64, StepArg step, const uint32_t *chg_cur,
                 uint32_t *chg_next, int64_t cap, hipStream_t st);

// Batched step: one launch steps several runs (each a default step: fused
// kernel, ion number and charge deposited, no optional physics).  A run's
// arguments sit in its job in device memory (written by launch_set_job,
// passed by value); the launch's list names each job, its step and its
// first workgroup (run j owns step_batch_wgs(n_j) workgroups from wg0[j]).
template <typename R>
struct StepJob {
  KParams P;
  const Tables *T;
  Soa<R> S;
  const uint32_t *cellid, *chunk_lo, *big, *bkinfo, *nbk;
  uint8_t *evlog;
  DevAccum *acc;
  double *dens, *moments;
  uint64_t *scratch64;
};
constexpr int kMaxBatch = 32;
template <typename R>
struct StepBatch {
  const StepJob<R> *job[kMaxBatch];
  const uint32_t *stepw[kMaxBatch];  // step = *stepw + step, or step alone when stepw is null
  uint32_t step[kMaxBatch];
  uint32_t wg0[kMaxBatch + 1];
  int n;
};
// a few 32-bit words set from the launch's arguments (the step counters
// read by captured graphs)
struct SetWords {
  uint32_t *ptr[kMaxBatch];
  uint32_t val[kMaxBatch];
  int n;
};
bool step_batchable(const KParams &P, bool dens, bool grids);
uint32_t step_batch_wgs(int64_t n, int64_t cap);
template <typename R>
void launch_step_batch(const StepBatch<R> &B, hipStream_t st);
template <typename R>
void launch_set_job(const StepJob<R> &J, StepJob<R> *dst, hipStream_t st);
void launch_set_words(const SetWords &w, hipStream_t st);

// sort by cell: keys either from positions or (given != nullptr) from given[pid]
template <typename R>
void launch_sort(const KParams &P, Soa<R> A, Soa<R> B, const uint32_t *given, uint32_t *key, uint32_t *rank,
                 uint32_t *count, uint32_t *cell_off, uint32_t *blocksums, uint32_t *cellid_out, int64_t ncell,
                 hipStream_t st);

size_t scan_blocksums_len(int64_t ncell);

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st);
void launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t st);
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t st);

void launch_selftest_philox(uint64_t seed, uint32_t ctr0, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
                            uint32_t *out, hipStream_t st);
void launch_selftest_divsqrt(const double *a, const double *b, int64_t n, double *q, double *r, hipStream_t st);

}  // namespace ecr
