// k_particles.hip -- per-particle kernels of the ion step (Mironov et al.,
// Sec. II): initial ions, the push / wall-aperture / Monte-Carlo-collision
// kernel, and the cloud-in-cell deposit.
//
// Layout: structure of arrays in HBM, one lane per particle slot, so every
// load and store of x, y, z, vx, vy, vz, qs and pid is a fully coalesced
// 64-lane access.  Slots are in cell order (sorted every sort_every steps),
// which keeps the deposit's atomics and the field-table reads local.
#include "ecr_kernels.hpp"

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
}

// ---------------------------------------------------------------------------
// Push -> wall/aperture -> ionisation / charge exchange, one particle per
// lane.  Tallies are rare events (~1e-4 per particle-step) and go straight
// to 64-bit global atomics.
// ---------------------------------------------------------------------------
template <typename R, bool HAS_E>
__global__ void __launch_bounds__(256) k_push(KParams P, const Tables *__restrict__ T, Soa<R> S,
                                              const double *__restrict__ ef, uint8_t *__restrict__ evlog,
                                              DevAccum *__restrict__ acc, uint32_t step) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P.n) return;
  R x = S.x[j], y = S.y[j], z = S.z[j];
  R vx = S.vx[j], vy = S.vy[j], vz = S.vz[j];
  const uint8_t qs0 = S.qs[j];
  const uint32_t id = S.pid[j];
  int Q = q_of(qs0);
  const int s = sp_of(qs0);
  uint8_t ev = EV_NONE;
  if (P.pmask & P_PUSH) {
    const R x0 = x, y0 = y, z0 = z;
    const R h = (R)T->qmh[s][Q];
    R E[3] = {(R)0, (R)0, (R)0};
    if (HAS_E) gather_E<R>(P, ef, x, y, z, E);
    boris<R, HAS_E>(P, h, E, x, y, z, vx, vy, vz);
    R f;
    const int kind = segment_exit<R>(P, x0, y0, z0, x, y, z, f);
    if (kind != X_NONE) {
      ev = wall_event<R>(P, id, step, s, kind, f, x0, y0, z0, x, y, z, vx, vy, vz);
      if (ev == EV_EXTRACT) {
        atomicAdd((unsigned long long *)&acc->t.extracted[s][Q], 1ull);
        atomicAdd((unsigned long long *)&acc->t.recycled, 1ull);
      } else {
        atomicAdd((unsigned long long *)&acc->t.wall[s][Q], 1ull);
      }
      Q = 0;
    }
  }
  if (ev == EV_NONE && (P.pmask & (P_IONIZE | P_CX))) {
    const uint4 W = draw(P, id, step, S_STEP, 0);
    const double u = u53(W.x, W.y);
    const int zone = (((x * x) * (R)P.ia2 + (y * y) * (R)P.ia2) + (z * z) * (R)P.ic2) < (R)1;
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
      Q = Q + 1;
      ev = EV_IONIZE;
    } else if (u < pt) {
      atomicAdd((unsigned long long *)&acc->t.cx[s][Q], 1ull);
      cx_outcome<R>(P, id, step, s, Q, vx, vy, vz);
      if (Q >= 2) {
        Q = Q - 1;
        atomicAdd((unsigned long long *)&acc->t.cx_products[s], 1ull);
      }
      ev = EV_CX;
    }
  }
  if (!(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(vx) && isfinite(vy) && isfinite(vz)))
    atomicAdd((unsigned long long *)&acc->t.anomalies, 1ull);
  S.x[j] = x;
  S.y[j] = y;
  S.z[j] = z;
  S.vx[j] = vx;
  S.vy[j] = vy;
  S.vz[j] = vz;
  S.qs[j] = make_qs(Q, s);
  if (evlog) evlog[j] = ev;
}

// ---------------------------------------------------------------------------
// Cloud-in-cell deposit of ion number, ion charge and atom number onto the
// (nx+1)(ny+1)(nz+1) node grid, FP64 global atomics.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) k_deposit(KParams P, Soa<R> S, double *__restrict__ dens) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P.n) return;
  const int Q = q_of(S.qs[j]);
  const bool ion = Q >= 1;
  const uint32_t dm = P.dmask;
  if (!((ion && (dm & 3u)) || (!ion && (dm & 4u)))) return;
  int ix, iy, iz;
  R tx, ty, tz;
  cic_axis<R>(S.x[j], (R)P.R0, (R)P.idx, P.nx, ix, tx);
  cic_axis<R>(S.y[j], (R)P.R0, (R)P.idy, P.ny, iy, ty);
  cic_axis<R>(S.z[j], (R)P.hL, (R)P.idz, P.nz, iz, tz);
  const R wx[2] = {(R)1 - tx, tx}, wy[2] = {(R)1 - ty, ty}, wz[2] = {(R)1 - tz, tz};
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int64_t node = (int64_t)(ix + dx) + (int64_t)P.nx1 * ((iy + dy) + (int64_t)P.ny1 * (iz + dz));
        const double w = (double)((wx[dx] * wy[dy]) * wz[dz]);
        if (ion) {
          if (dm & 1u) atomicAdd(&dens[node], w);
          if (dm & 2u) atomicAdd(&dens[P.nnode + node], (double)Q * w);
        } else {
          atomicAdd(&dens[2 * P.nnode + node], w);
        }
      }
}

static inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename R>
void launch_init(const KParams &P, Soa<R> S, hipStream_t st) {
  if (P.n <= 0) return;
  hipLaunchKernelGGL(k_init<R>, dim3(grid_for(P.n, 256)), dim3(256), 0, st, P, S);
}

template <typename R>
void launch_push(const KParams &P, const Tables *T, Soa<R> S, const double *ef, uint8_t *evlog, DevAccum *acc,
                 uint32_t step, hipStream_t st) {
  if (P.n <= 0) return;
  if (ef)
    hipLaunchKernelGGL((k_push<R, true>), dim3(grid_for(P.n, 256)), dim3(256), 0, st, P, T, S, ef, evlog, acc, step);
  else
    hipLaunchKernelGGL((k_push<R, false>), dim3(grid_for(P.n, 256)), dim3(256), 0, st, P, T, S, ef, evlog, acc,
                       step);
}

template <typename R>
void launch_deposit(const KParams &P, Soa<R> S, double *dens, hipStream_t st) {
  if (P.n <= 0) return;
  hipLaunchKernelGGL(k_deposit<R>, dim3(grid_for(P.n, 256)), dim3(256), 0, st, P, S, dens);
}

template void launch_init<double>(const KParams &, Soa<double>, hipStream_t);
template void launch_init<float>(const KParams &, Soa<float>, hipStream_t);
template void launch_push<double>(const KParams &, const Tables *, Soa<double>, const double *, uint8_t *, DevAccum *,
                                  uint32_t, hipStream_t);
template void launch_push<float>(const KParams &, const Tables *, Soa<float>, const double *, uint8_t *, DevAccum *,
                                 uint32_t, hipStream_t);
template void launch_deposit<double>(const KParams &, Soa<double>, double *, hipStream_t);
template void launch_deposit<float>(const KParams &, Soa<float>, double *, hipStream_t);

}  // namespace ecr
