// k_particles.hip -- per-particle kernels of the ion step (Mironov et al.,
// Sec. II): initial ions, and the kernel that pushes each particle, applies
// the wall / aperture loss, draws ionisation or charge exchange, and
// deposits it on the density mesh.
//
// Layout: structure of arrays in HBM, one lane per slot, so every load and
// store of a wavefront is 64 consecutive elements.  A workgroup covers a tile
// of kP x 256 slots.  Slots are in cell order (sorted every sort_every steps),
// which the deposit exploits (see deposit_staged): it takes the deposit from
// 16 contended global atomics per particle to a few per workgroup.
#include <type_traits>

#include "ecr_kernels.hpp"
#include "ecr_push.hpp"

namespace ecr {


// ---------------------------------------------------------------------------
// Initial ions: uniform in the ECR-zone ellipsoid by rejection sampling in
// its bounding box (at most 64 attempts, then the centre), Maxwellian
// velocity at Ti0, Q = 1, species by contiguous id ranges.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) k_init(KParams P, Soa<R> S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n) return;
  const uint32_t id = (uint32_t)i;
  const double a = P.zone_a, c = P.zone_c;
  int s = P.nspecies - 1;
  for (int k = P.nspecies - 1; k >= 0; --k)
    if (i < P.sp_end[k]) s = k;
  double px = 0.0, py = 0.0, pz = 0.0;
  for (uint32_t j = 0; j < 64; ++j) {
    const uint4 A = draw(P, id, 0xFFFFFFFFu, S_INIT, 2 * j);
    const uint4 B = draw(P, id, 0xFFFFFFFFu, S_INIT, 2 * j + 1);
    const double u0 = u53(A.x, A.y), u1 = u53(A.z, A.w), u2 = u53(B.x, B.y);
    const double tx = a * (2.0 * u0 - 1.0);
    const double ty = a * (2.0 * u1 - 1.0);
    const double tz = c * (2.0 * u2 - 1.0);
    if (((tx * tx) * P.ia2 + (ty * ty) * P.ia2) + (tz * tz) * P.ic2 < 1.0) {
      px = tx;
      py = ty;
      pz = tz;
      break;
    }
  }
  const uint4 C = draw(P, id, 0xFFFFFFFFu, S_INIT, 0x10000u);
  const uint4 D = draw(P, id, 0xFFFFFFFFu, S_INIT, 0x10001u);
  double n0, n1, n2, nd;
  box_muller(u53(C.x, C.y), u53(C.z, C.w), n0, n1);
  box_muller(u53(D.x, D.y), u53(D.z, D.w), n2, nd);
  const double sg = P.sig_i[s];
  S.x[i] = (R)px;
  S.y[i] = (R)py;
  S.z[i] = (R)pz;
  S.vx[i] = (R)(sg * n0);
  S.vy[i] = (R)(sg * n1);
  S.vz[i] = (R)(sg * n2);
  S.qs[i] = make_qs(1, s);
  S.pid[i] = id;
  S.birth[i] = 0u;  // created at step 0
}

// ---------------------------------------------------------------------------
// Push + wall/aperture + MCC (+ deposit): slot j = tile + tid + 256 p.
// ---------------------------------------------------------------------------
// ion number and charge fields
template <typename R, int FLD, int DEP, bool EXT>
__device__ __forceinline__ void push_tile(const KParams &P, const Tables *__restrict__ T, Soa<R> S,
                                          const double *__restrict__ ef, uint8_t *__restrict__ evlog,
                                          DevAccum *__restrict__ acc, double *__restrict__ dens, StepArg sa,
                                          const uint32_t *__restrict__ chg_cur, uint32_t *__restrict__ chg_next) {
  __shared__ DepShared<R> sh;
  const uint32_t step = sa.get();
  __shared__ int box[6 * (kBlock / 64)];
  int mn[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, mx[3] = {-1, -1, -1};
  const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
  for (int p = 0; p < kP; ++p) {
    const int i = threadIdx.x + p * kBlock;
    const int64_t j = base + i;
    uint32_t ccell = 0xffffffffu, cq = 0u;  // this lane's contribution to the next charge grid
    if (j >= P.n) {
      if (DEP) sh.st.q[i] = 0xFF;
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
          advance<R, FLD, EXT>(P, T, ef, acc, step, id, s, Q, x, y, z, vx, vy, vz, S.birth, j, j, chg_cur, u);
      S.x[j] = x;
      S.y[j] = y;
      S.z[j] = z;
      S.vx[j] = vx;
      S.vy[j] = vy;
      S.vz[j] = vz;
      S.qs[j] = make_qs(Q, s);
      if (evlog) evlog[j] = ev;
      if (EXT && chg_next) {
        // the next step's cell grids: ion charge in channel 0, atoms of
        // species s in channel 1 + s
        const uint32_t c = cell_of<R>(P, x, y, z);
        ccell = Q >= 1 ? c : (uint32_t)(1 + s) * P.ncell + c;
        cq = Q >= 1 ? (uint32_t)Q : 1u;
      }
      if (DEP) stage_cic<R, DEP == 2>(P, sh.st, i, x, y, z, Q, mn, mx);
    }
    if (EXT && chg_next) add_charge(chg_next, ccell, cq);  // all lanes together: run sums use shuffles
  }
  if (DEP) deposit_staged<R, DEP == 2>(P, dens, sh, box, mn, mx);
}

template <typename R, int FLD, int DEP, bool EXT>
__global__ void __launch_bounds__(kBlock) k_push(KParams P, const Tables *__restrict__ T, Soa<R> S,
                                                 const double *__restrict__ ef, uint8_t *__restrict__ evlog,
                                                 DevAccum *__restrict__ acc, double *__restrict__ dens,
                                                 StepArg sa, const uint32_t *__restrict__ chg_cur,
                                                 uint32_t *__restrict__ chg_next) {
  push_tile<R, FLD, DEP, EXT>(P, T, S, ef, evlog, acc, dens, sa, chg_cur, chg_next);
}

// the default binary64 step (no E field, ion number and charge deposit, no
// optional physics) held at five waves per SIMD: its 31 KB of LDS lets five
// workgroups share a CU, and the registers fit with a few spills on cold paths
// (measured 68 -> 65 us per launch at 2M ions)
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5)))
k_push_lean(KParams P, const Tables *__restrict__ T, Soa<double> S, const double *__restrict__ ef,
            uint8_t *__restrict__ evlog, DevAccum *__restrict__ acc, double *__restrict__ dens, StepArg sa,
            const uint32_t *__restrict__ chg_cur, uint32_t *__restrict__ chg_next) {
  push_tile<double, 0, 2, false>(P, T, S, ef, evlog, acc, dens, sa, chg_cur, chg_next);
}

// standalone deposit (same tile code), for per-kernel timing
template <typename R, bool NQ>
__global__ void __launch_bounds__(kBlock) k_deposit(KParams P, Soa<R> S, double *__restrict__ dens) {
  __shared__ DepShared<R> sh;
  __shared__ int box[6 * (kBlock / 64)];
  int mn[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, mx[3] = {-1, -1, -1};
  const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
  for (int p = 0; p < kP; ++p) {
    const int i = threadIdx.x + p * kBlock;
    const int64_t j = base + i;
    if (j < P.n) stage_cic<R, NQ>(P, sh.st, i, S.x[j], S.y[j], S.z[j], q_of(S.qs[j]), mn, mx);
    else sh.st.q[i] = 0xFF;
  }
  deposit_staged<R, NQ>(P, dens, sh, box, mn, mx);
}

// ---------------------------------------------------------------------------
// Ion pressure moment (optional field ECR_F_ION_P, Sec. III.B): every ion
// adds its CIC weights times M |v|^2 / 3.  The tile scheme of the number and
// charge deposit (lane = slot staging, transposed runs of 4 slots, wavefront
// segmented sums, LDS brick) with one field and a weight per particle.
// ---------------------------------------------------------------------------
template <typename R>
struct PStage {
  R t[3][kStage];
  uint16_t c[3][kStage];
  double e[kStage];  // M |v|^2 / 3, or < 0: nothing to deposit
};

template <typename R>
union PShared {
  PStage<R> st;
  double brick[3 * kBrickNodes];  // one field: three times the nodes of the number brick
};

template <typename R>
__global__ void __launch_bounds__(kBlock) k_deposit_pressure(KParams P, Soa<R> S, double *__restrict__ dens) {
  __shared__ PShared<R> sh;
  __shared__ int box[6 * (kBlock / 64)];
  const int tid = threadIdx.x;
  int mn[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, mx[3] = {-1, -1, -1};
  const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
  for (int p = 0; p < kP; ++p) {
    const int i = tid + p * kBlock;
    const int64_t j = base + i;
    const int k = kPad(i);
    sh.st.e[k] = -1.0;
    if (j < P.n) {
      const uint8_t qs = S.qs[j];
      if (q_of(qs) >= 1) {
        const R vx = S.vx[j], vy = S.vy[j], vz = S.vz[j];
        int ix, iy, iz;
        R tx, ty, tz;
        cic_axis<R>(S.x[j], (R)P.R0, (R)P.idx, P.nx, ix, tx);
        cic_axis<R>(S.y[j], (R)P.R0, (R)P.idy, P.ny, iy, ty);
        cic_axis<R>(S.z[j], (R)P.hL, (R)P.idz, P.nz, iz, tz);
        sh.st.t[0][k] = tx;
        sh.st.t[1][k] = ty;
        sh.st.t[2][k] = tz;
        sh.st.c[0][k] = (uint16_t)ix;
        sh.st.c[1][k] = (uint16_t)iy;
        sh.st.c[2][k] = (uint16_t)iz;
        sh.st.e[k] = (P.mass[sp_of(qs)] * (double)((vx * vx + vy * vy) + vz * vz)) / 3.0;
        mn[0] = min(mn[0], ix);
        mn[1] = min(mn[1], iy);
        mn[2] = min(mn[2], iz);
        mx[0] = max(mx[0], ix);
        mx[1] = max(mx[1], iy);
        mx[2] = max(mx[2], iz);
      }
    }
  }
  box_publish(box, mn, mx);
  __syncthreads();  // staging and box complete
  int ix[kP], iy[kP], iz[kP];
  R tx[kP], ty[kP], tz[kP];
  double e[kP];
#pragma unroll
  for (int p = 0; p < kP; ++p) {
    const int k = kPad(tid * kP + p);
    e[p] = sh.st.e[k];
    tx[p] = sh.st.t[0][k];
    ty[p] = sh.st.t[1][k];
    tz[p] = sh.st.t[2][k];
    ix[p] = sh.st.c[0][k];
    iy[p] = sh.st.c[1][k];
    iz[p] = sh.st.c[2][k];
  }
  int bb[6];
  box_reduce<kBlock>(box, bb);
  const int x0 = bb[0], y0 = bb[1], z0 = bb[2];
  const bool any = bb[3] >= 0;
  const int bx = bb[3] - x0 + 2, by = bb[4] - y0 + 2, bz = bb[5] - z0 + 2;
  __syncthreads();  // staging read: the brick may now reuse it
  if (!any) return;
  const int64_t nodes = (int64_t)bx * by * bz;
  const bool in_brick = nodes <= 3 * kBrickNodes;
  const int nb = (int)(in_brick ? nodes : 0);
  const int nx1 = P.nx1, ny1 = P.ny1;
  double *f3 = dens + (int64_t)ECR_F_ION_P * P.nnode;
  auto node_of = [&](int p) -> int64_t {
    return in_brick ? (int64_t)((ix[p] - x0) + bx * ((iy[p] - y0) + by * (iz[p] - z0)))
                    : (int64_t)ix[p] + (int64_t)nx1 * (iy[p] + (int64_t)ny1 * iz[p]);
  };
  auto flush = [&](int64_t nd, const double *a) {
    for (int k = 0; k < 8; ++k) {
      if (a[k] == 0.0) continue;
      const int dx = k & 1, dy = (k >> 1) & 1, dz = k >> 2;
      if (in_brick) atomicAdd(&sh.brick[(int)nd + dx + bx * (dy + by * dz)], a[k]);
      else unsafeAtomicAdd(&f3[nd + dx + (int64_t)nx1 * (dy + (int64_t)ny1 * dz)], a[k]);
    }
  };
  if (in_brick) {
    for (int i = tid; i < nb; i += kBlock) sh.brick[i] = 0.0;
    __syncthreads();
  }
  // this lane's runs of equal base node; the last one goes to the wavefront sum
  double a[8];
  int64_t cur = -1;
  for (int k = 0; k < 8; ++k) a[k] = 0.0;
#pragma unroll
  for (int p = 0; p < kP; ++p) {
    if (!(e[p] >= 0.0)) continue;
    const int64_t nd = node_of(p);
    if (nd != cur) {
      if (cur >= 0) flush(cur, a);
      cur = nd;
      for (int k = 0; k < 8; ++k) a[k] = 0.0;
    }
    const R wx[2] = {(R)1 - tx[p], tx[p]}, wy[2] = {(R)1 - ty[p], ty[p]}, wz[2] = {(R)1 - tz[p], tz[p]};
    int k = 0;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx, ++k) a[k] += (double)((wx[dx] * wy[dy]) * wz[dz]) * e[p];
  }
  const int64_t key = cur;
  int seg;
  bool tail;
  wave_runs(key, seg, tail);
  const SegSteps st = seg_steps(seg);
  for (int k = 0; k < 8; ++k) a[k] = seg_scan(st, a[k]);
  if (tail && key >= 0) flush(key, a);
  if (!in_brick) return;
  __syncthreads();
  for (int li = tid; li < nb; li += kBlock) {
    const double v = sh.brick[li];
    if (v != 0.0) {
      const int t = li / bx, lx = li - t * bx, lz = t / by, ly = t - lz * by;
      unsafeAtomicAdd(&f3[(int64_t)(x0 + lx) + (int64_t)nx1 * ((y0 + ly) + (int64_t)ny1 * (z0 + lz))], v);
    }
  }
}

static inline unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

template <typename R>
void launch_init(const KParams &P, Soa<R> S, hipStream_t st) {
  if (P.n <= 0) return;
  hipLaunchKernelGGL(k_init<R>, dim3(grid_for(P.n, 256)), dim3(256), 0, st, P, S);
}

template <typename R, int FLD, bool EXT>
static void launch_push_e(const KParams &P, const Tables *T, Soa<R> S, const double *ef, uint8_t *evlog,
                          DevAccum *acc, double *dens, StepArg step, const uint32_t *chg_cur, uint32_t *chg_next,
                          hipStream_t st) {
  const dim3 g(grid_for(P.n, kTile)), b(kBlock);
  if (!dens)
    hipLaunchKernelGGL((k_push<R, FLD, 0, EXT>), g, b, 0, st, P, T, S, ef, evlog, acc, dens, step, chg_cur,
                       chg_next);
  else if ((P.dmask & 7u) == 3u) {
    if constexpr (std::is_same<R, double>::value && FLD == 0 && !EXT)
      hipLaunchKernelGGL(k_push_lean, g, b, 0, st, P, T, S, ef, evlog, acc, dens, step, chg_cur, chg_next);
    else
      hipLaunchKernelGGL((k_push<R, FLD, 2, EXT>), g, b, 0, st, P, T, S, ef, evlog, acc, dens, step, chg_cur,
                         chg_next);
  } else {
    hipLaunchKernelGGL((k_push<R, FLD, 1, EXT>), g, b, 0, st, P, T, S, ef, evlog, acc, dens, step, chg_cur,
                       chg_next);
  }
}

template <typename R, bool EXT>
static void launch_push_v(const KParams &P, const Tables *T, Soa<R> S, const double *ef, uint8_t *evlog,
                          DevAccum *acc, double *dens, StepArg step, const uint32_t *chg_cur, uint32_t *chg_next,
                          hipStream_t st) {
  switch ((ef ? 1 : 0) | (P.bmap ? 2 : 0)) {
    case 0: launch_push_e<R, 0, EXT>(P, T, S, ef, evlog, acc, dens, step, chg_cur, chg_next, st); break;
    case 1: launch_push_e<R, 1, EXT>(P, T, S, ef, evlog, acc, dens, step, chg_cur, chg_next, st); break;
    case 2: launch_push_e<R, 2, EXT>(P, T, S, ef, evlog, acc, dens, step, chg_cur, chg_next, st); break;
    default: launch_push_e<R, 3, EXT>(P, T, S, ef, evlog, acc, dens, step, chg_cur, chg_next, st); break;
  }
}

template <typename R>
void launch_push(const KParams &P, const Tables *T, Soa<R> S, const double *ef, uint8_t *evlog, DevAccum *acc,
                 double *dens, StepArg step, const uint32_t *chg_cur, uint32_t *chg_next, hipStream_t st) {
  if (P.n <= 0) return;
  const bool ext = chg_cur || chg_next || (P.pmask & (P_HEAT | P_ELASTIC)) || P.nion > 1;
  if (ext)
    launch_push_v<R, true>(P, T, S, ef, evlog, acc, dens, step, chg_cur, chg_next, st);
  else
    launch_push_v<R, false>(P, T, S, ef, evlog, acc, dens, step, chg_cur, chg_next, st);
}

// ion charge and atoms per cell of the current state (the first step after init or set_state)
template <typename R>
__global__ void __launch_bounds__(256) k_charge_grid(KParams P, Soa<R> S, uint32_t *__restrict__ chg) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t cell = 0xffffffffu, q = 0u;
  if (j < P.n) {
    const uint8_t qs = S.qs[j];
    const int Q = q_of(qs);
    const uint32_t c = cell_of<R>(P, S.x[j], S.y[j], S.z[j]);
    cell = Q >= 1 ? c : (uint32_t)(1 + sp_of(qs)) * P.ncell + c;
    q = Q >= 1 ? (uint32_t)Q : 1u;
  }
  add_charge(chg, cell, q);  // all lanes together
}

template <typename R>
void launch_charge_grid(const KParams &P, Soa<R> S, uint32_t *chg, hipStream_t st) {
  if (P.n <= 0) return;
  hipLaunchKernelGGL(k_charge_grid<R>, dim3(grid_for(P.n, 256)), dim3(256), 0, st, P, S, chg);
}

template void launch_charge_grid<double>(const KParams &, Soa<double>, uint32_t *, hipStream_t);
template void launch_charge_grid<float>(const KParams &, Soa<float>, uint32_t *, hipStream_t);

// |B| at each cell centre times the cell size hx (the heating kick's
// electron Larmor radius divides by it): the analytic field, or the node
// map interpolated at the centre
__global__ void __launch_bounds__(256) k_cell_bden(KParams P, double *__restrict__ bden) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (int64_t)P.ncell) return;
  const int ix = (int)(c % P.nx), iy = (int)((c / P.nx) % P.ny), iz = (int)(c / ((int64_t)P.nx * P.ny));
  const double xc = -P.R0 + ((double)ix + 0.5) * P.hx, yc = -P.R0 + ((double)iy + 0.5) * P.hy;
  const double zc = -P.hL + ((double)iz + 0.5) * P.hz;
  double bx, by, bz;
  if (P.bmap) {
    double B[3];
    gather_E<double>(P, P.bmap, xc, yc, zc, B);
    bx = B[0];
    by = B[1];
    bz = B[2];
  } else {
    field_B<double>(P, xc, yc, zc, bx, by, bz);
  }
  const double bmag = sqrt((bx * bx + by * by) + bz * bz);
  bden[c] = bmag * P.hx;
}

void launch_cell_bden(const KParams &P, double *bden, hipStream_t st) {
  if (P.ncell == 0u) return;
  hipLaunchKernelGGL(k_cell_bden, dim3(grid_for((int64_t)P.ncell, 256)), dim3(256), 0, st, P, bden);
}

template <typename R>
void launch_deposit(const KParams &P, Soa<R> S, double *dens, hipStream_t st) {
  if (P.n <= 0) return;
  if ((P.dmask & 7u) == 3u)
    hipLaunchKernelGGL((k_deposit<R, true>), dim3(grid_for(P.n, kTile)), dim3(kBlock), 0, st, P, S, dens);
  else
    hipLaunchKernelGGL((k_deposit<R, false>), dim3(grid_for(P.n, kTile)), dim3(kBlock), 0, st, P, S, dens);
}

template <typename R>
void launch_deposit_pressure(const KParams &P, Soa<R> S, double *dens, hipStream_t st) {
  if (P.n <= 0) return;
  hipLaunchKernelGGL(k_deposit_pressure<R>, dim3(grid_for(P.n, kTile)), dim3(kBlock), 0, st, P, S, dens);
}

template void launch_deposit_pressure<double>(const KParams &, Soa<double>, double *, hipStream_t);
template void launch_deposit_pressure<float>(const KParams &, Soa<float>, double *, hipStream_t);
template void launch_init<double>(const KParams &, Soa<double>, hipStream_t);
template void launch_init<float>(const KParams &, Soa<float>, hipStream_t);
template void launch_push<double>(const KParams &, const Tables *, Soa<double>, const double *, uint8_t *, DevAccum *,
                                  double *, StepArg, const uint32_t *, uint32_t *, hipStream_t);
template void launch_push<float>(const KParams &, const Tables *, Soa<float>, const double *, uint8_t *, DevAccum *,
                                 double *, StepArg, const uint32_t *, uint32_t *, hipStream_t);
template void launch_deposit<double>(const KParams &, Soa<double>, double *, hipStream_t);
template void launch_deposit<float>(const KParams &, Soa<float>, double *, hipStream_t);

}  // namespace ecr
