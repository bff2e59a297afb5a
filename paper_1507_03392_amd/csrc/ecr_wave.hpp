// ecr_wave.hpp -- cross-lane building blocks of the gfx950 kernels: sums,
// scans, segmented sums and min/max over a 64-lane wavefront with DPP lane
// moves (row_shr 1, 2, 4, 8 inside each row of 16 lanes, then row_bcast 15
// and 31 across the rows; no LDS), and an exclusive scan over a workgroup.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ecr {

// Inclusive sums over a wavefront with DPP lane moves, no LDS: row_shr 1,
// 2, 4, 8 within each row of 16 lanes, then row_bcast 15 (the last lane of
// rows 0 and 2 into rows 1 and 3) and row_bcast 31 (lane 31 into rows 2
// and 3); a missing source adds zero.  Called by all 64 lanes; lane 63 ends
// with the wavefront's total.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  x += dpp_u32<0x111, 0xf>(x);
  x += dpp_u32<0x112, 0xf>(x);
  x += dpp_u32<0x114, 0xf>(x);
  x += dpp_u32<0x118, 0xf>(x);
  x += dpp_u32<0x142, 0xa>(x);
  x += dpp_u32<0x143, 0xc>(x);
  return x;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = dpp_u32<CTRL, ROWS>((uint32_t)u), hi = dpp_u32<CTRL, ROWS>((uint32_t)(u >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// the wavefront's total, in lane 63
__device__ __forceinline__ double wave_sum_last(double x) {
  x += dpp_f64<0x111, 0xf>(x);
  x += dpp_f64<0x112, 0xf>(x);
  x += dpp_f64<0x114, 0xf>(x);
  x += dpp_f64<0x118, 0xf>(x);
  x += dpp_f64<0x142, 0xa>(x);
  x += dpp_f64<0x143, 0xc>(x);
  return x;
}

// in-place exclusive scan of a[0..L) by a workgroup of NT lanes; returns the
// total, also stored in a[L] when store_total (wsum: NT / 64 words of LDS);
// a, a[L] included, is complete for every lane on return
template <int NT>
__device__ __forceinline__ uint32_t wg_exscan(uint32_t *a, int L, uint32_t *wsum, bool store_total = false) {
  const int tid = threadIdx.x;
  const int per = (L + NT - 1) / NT;
  const int b = tid * per, e = min(b + per, L);
  uint32_t s = 0;
  for (int i = b; i < e; ++i) s += a[i];
  const int lane = tid & 63, w = tid >> 6;
  const uint32_t x = wave_incl_scan(s);
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t woff = 0, tot = 0;
  for (int q = 0; q < NT / 64; ++q) {
    if (q < w) woff += wsum[q];
    tot += wsum[q];
  }
  uint32_t run = woff + x - s;
  for (int i = b; i < e; ++i) {
    const uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
  if (store_total && tid == 0) a[L] = tot;
  __syncthreads();
  return tot;
}


// Segmented sums over the lanes of a wavefront: lanes are in slot order, so
// equal run nodes form contiguous lane segments (a lane's earlier runs were
// flushed already).  Segmented inclusive sums over a wavefront with DPP lane moves, no LDS:
// row_shr 1, 2, 4, 8 within each row of 16 lanes, then row_bcast 15 (the
// last lane of rows 0 and 2 into rows 1 and 3) and row_bcast 31 (lane 31
// into rows 2 and 3).  seg is a run id, equal exactly on runs of
// consecutive lanes; a step adds the source lane's partial sum when the
// source exists and lies in the same run, so after the six steps the last
// lane of every run holds the run's total.  Called by all 64 lanes.
struct SegSteps {
  bool t[6];  // step i takes its source lane's partial sum
};

template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_move(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);  // disabled or missing source: old
}

__device__ __forceinline__ SegSteps seg_steps(int seg) {
  SegSteps s;  // seg >= 0, so the -1 of a missing source never matches
  s.t[0] = dpp_move<0x111, 0xf>(-1, seg) == seg;  // row_shr:1
  s.t[1] = dpp_move<0x112, 0xf>(-1, seg) == seg;  // row_shr:2
  s.t[2] = dpp_move<0x114, 0xf>(-1, seg) == seg;  // row_shr:4
  s.t[3] = dpp_move<0x118, 0xf>(-1, seg) == seg;  // row_shr:8
  s.t[4] = dpp_move<0x142, 0xa>(-1, seg) == seg;  // row_bcast:15 into rows 1, 3
  s.t[5] = dpp_move<0x143, 0xc>(-1, seg) == seg;  // row_bcast:31 into rows 2, 3
  return s;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move_d(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)dpp_move<CTRL, ROWS>(0, (int)(uint32_t)u);
  const uint32_t hi = (uint32_t)dpp_move<CTRL, ROWS>(0, (int)(uint32_t)(u >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double seg_scan(const SegSteps &s, double x) {
  double o;
  o = dpp_move_d<0x111, 0xf>(x);
  x = s.t[0] ? x + o : x;
  o = dpp_move_d<0x112, 0xf>(x);
  x = s.t[1] ? x + o : x;
  o = dpp_move_d<0x114, 0xf>(x);
  x = s.t[2] ? x + o : x;
  o = dpp_move_d<0x118, 0xf>(x);
  x = s.t[3] ? x + o : x;
  o = dpp_move_d<0x142, 0xa>(x);
  x = s.t[4] ? x + o : x;
  o = dpp_move_d<0x143, 0xc>(x);
  x = s.t[5] ? x + o : x;
  return x;
}

// (the moves run on every lane before the select: a move under a lane
// condition would read the lanes the condition turns off as missing)
__device__ __forceinline__ uint32_t seg_scan(const SegSteps &s, uint32_t x) {
  uint32_t o;
  o = (uint32_t)dpp_move<0x111, 0xf>(0, (int)x);
  x += s.t[0] ? o : 0u;
  o = (uint32_t)dpp_move<0x112, 0xf>(0, (int)x);
  x += s.t[1] ? o : 0u;
  o = (uint32_t)dpp_move<0x114, 0xf>(0, (int)x);
  x += s.t[2] ? o : 0u;
  o = (uint32_t)dpp_move<0x118, 0xf>(0, (int)x);
  x += s.t[3] ? o : 0u;
  o = (uint32_t)dpp_move<0x142, 0xa>(0, (int)x);
  x += s.t[4] ? o : 0u;
  o = (uint32_t)dpp_move<0x143, 0xc>(0, (int)x);
  x += s.t[5] ? o : 0u;
  return x;
}

// Segmented sums within aligned groups of G consecutive lanes (G = 2, 4, 8
// or 16, inside a row of 16), by log2 G row_shr steps: a group boundary acts
// as a run boundary, so after the steps a lane holds the sum over the lanes
// of its run from the later of the run's first lane and the group's first
// lane up to itself.  Cheaper than the whole-wavefront sums (fewer steps, no
// bcast rows); the last lane of each run within a group carries the partial
// sum that has to be flushed.
template <int G>
struct GroupSteps {
  bool t[4];
};

template <int G>
__device__ __forceinline__ GroupSteps<G> group_steps(int seg) {
  static_assert(G == 2 || G == 4 || G == 8 || G == 16, "groups inside a row of 16 lanes");
  const int gl = (int)(threadIdx.x & (G - 1));  // lane within the group
  GroupSteps<G> s;
  s.t[0] = dpp_move<0x111, 0xf>(-1, seg) == seg && gl >= 1;
  s.t[1] = G > 2 && dpp_move<0x112, 0xf>(-1, seg) == seg && gl >= 2;
  s.t[2] = G > 4 && dpp_move<0x114, 0xf>(-1, seg) == seg && gl >= 4;
  s.t[3] = G > 8 && dpp_move<0x118, 0xf>(-1, seg) == seg && gl >= 8;
  return s;
}

// a lane's double from the lane CTRL names (any value where there is none:
// the caller selects)
template <int CTRL>
__device__ __forceinline__ double dpp_take_d(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xf, 0xf, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <int G>
__device__ __forceinline__ double group_scan(const GroupSteps<G> &s, double x) {
  double o = dpp_take_d<0x111>(x);
  x = s.t[0] ? x + o : x;
  if (G > 2) {
    o = dpp_take_d<0x112>(x);
    x = s.t[1] ? x + o : x;
  }
  if (G > 4) {
    o = dpp_take_d<0x114>(x);
    x = s.t[2] ? x + o : x;
  }
  if (G > 8) {
    o = dpp_take_d<0x118>(x);
    x = s.t[3] ? x + o : x;
  }
  return x;
}

// the wavefront's cell-index bounding box (minima and maxima of three
// indices) by the same DPP moves, in lane 63; called by all 64 lanes
template <int CTRL, int ROWS>
__device__ __forceinline__ void box_step(int mn[3], int mx[3]) {
  for (int d = 0; d < 3; ++d) {
    const int a = dpp_move<CTRL, ROWS>(0x7fffffff, mn[d]), b = dpp_move<CTRL, ROWS>(-0x7fffffff - 1, mx[d]);
    mn[d] = min(mn[d], a);
    mx[d] = max(mx[d], b);
  }
}

__device__ __forceinline__ void wave_box_last(int mn[3], int mx[3]) {
  box_step<0x111, 0xf>(mn, mx);
  box_step<0x112, 0xf>(mn, mx);
  box_step<0x114, 0xf>(mn, mx);
  box_step<0x118, 0xf>(mn, mx);
  box_step<0x142, 0xa>(mn, mx);
  box_step<0x143, 0xc>(mn, mx);
}

// runs of equal keys over the wavefront: run ids, and whether this lane ends its run
__device__ __forceinline__ void wave_runs(int64_t key, int &seg, bool &tail) {
  const int lane = threadIdx.x & 63;
  // the previous lane's key by wave_shr:1 (lane 0 has none and heads a run)
  const uint32_t plo = (uint32_t)dpp_move<0x138, 0xf>(0, (int)(uint32_t)(uint64_t)key);
  const uint32_t phi = (uint32_t)dpp_move<0x138, 0xf>(0, (int)(uint32_t)((uint64_t)key >> 32));
  const int64_t kprev = (int64_t)(((uint64_t)phi << 32) | plo);
  const uint64_t heads = __ballot(lane == 0 || kprev != key);
  seg = __popcll(heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1)));
  tail = lane == 63 || ((heads >> (lane + 1)) & 1ull);
}


}  // namespace ecr
