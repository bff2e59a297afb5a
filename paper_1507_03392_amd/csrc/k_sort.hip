// k_sort.hip -- periodic sort of the particles by cell, plus fill and
// self-test kernels.
//
// Counting sort in three passes: (1) each slot computes its cell and claims
// a rank inside the cell from the cell's counter (one atomic per run of
// equal cells within a wavefront);
// (2) an exclusive scan of the counters gives cell_off (reduce per block of
// 1024 counters, scan of the block sums in one workgroup, scan within each
// block); (3) each slot scatters its record to cell_off[cell] + rank and
// stores its cell as its collision cell.  Within a cell the order is that of
// the atomic claims; nothing downstream depends on it except the summation
// order of the FP64 deposit (pairing order is fixed by keys, not slots).
#include "ecr_kernels.hpp"

namespace ecr {

constexpr int kScanBlock = 1024;  // counters per scan block (256 lanes x 4)

template <typename R>
__global__ void __launch_bounds__(256) k_sort_count(KParams P, Soa<R> A, const uint32_t *__restrict__ given,
                                                    uint32_t *__restrict__ key, uint32_t *__restrict__ rank,
                                                    uint32_t *__restrict__ count) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = j < P.n;
  const int lane = (int)(threadIdx.x & 63);
  uint32_t c = 0xffffffffu;
  if (valid) {
    c = given ? given[A.pid[j]] : cell_of<R>(P, A.x[j], A.y[j], A.z[j]);
    key[j] = c;
  }
  // slots are mostly in cell order already (the previous sort), so runs of
  // lanes share a cell: the first lane of each run claims the whole run with
  // one atomic and the others take consecutive ranks after it
  const uint32_t prev = __shfl_up(c, 1, 64);
  const bool head = lane == 0 || prev != c;
  const uint64_t hm = __ballot(head);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
  const int h = 63 - __clzll(hm & upto);  // first lane of my run
  const uint64_t after = hm & ~upto;
  const int next = after ? __builtin_ctzll(after) : 64;  // first lane of the next run
  uint32_t base = 0;
  if (head && valid) base = atomicAdd(&count[c], (uint32_t)(next - lane));
  base = __shfl(base, h, 64);
  if (valid) rank[j] = base + (uint32_t)(lane - h);
}

__global__ void __launch_bounds__(256) k_scan_reduce(const uint32_t *__restrict__ count, int64_t ncell,
                                                     uint32_t *__restrict__ blocksums) {
  __shared__ uint32_t sw[4];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  uint32_t v = 0;
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + threadIdx.x * 4 + k;
    if (i < ncell) v += count[i];
  }
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) blocksums[blockIdx.x] = sw[0] + sw[1] + sw[2] + sw[3];
}

// exclusive scan of nb block sums in place, one workgroup, 1024 per pass
__global__ void __launch_bounds__(256) k_scan_top(uint32_t *__restrict__ bsum, int64_t nb) {
  __shared__ uint32_t sw[4];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += kScanBlock) {
    uint32_t v[4];
    uint32_t tsum = 0;
    for (int k = 0; k < 4; ++k) {
      const int64_t i = base + threadIdx.x * 4 + k;
      v[k] = i < nb ? bsum[i] : 0u;
      tsum += v[k];
    }
    // inclusive scan of tsum across the workgroup
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = tsum;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) sw[w] = x;
    __syncthreads();
    uint32_t woff = 0;
    for (int q = 0; q < w; ++q) woff += sw[q];
    const uint32_t excl = carry + woff + x - tsum;
    uint32_t run = excl;
    for (int k = 0; k < 4; ++k) {
      const int64_t i = base + threadIdx.x * 4 + k;
      if (i < nb) bsum[i] = run;
      run += v[k];
    }
    __syncthreads();
    if (threadIdx.x == 255) carry = run;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_scan_down(const uint32_t *__restrict__ count, int64_t ncell,
                                                   const uint32_t *__restrict__ bsum, uint32_t *__restrict__ off,
                                                   uint32_t total) {
  __shared__ uint32_t sw[4];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  uint32_t v[4];
  uint32_t tsum = 0;
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + threadIdx.x * 4 + k;
    v[k] = i < ncell ? count[i] : 0u;
    tsum += v[k];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = tsum;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sw[w] = x;
  __syncthreads();
  uint32_t woff = 0;
  for (int q = 0; q < w; ++q) woff += sw[q];
  uint32_t run = bsum[blockIdx.x] + woff + x - tsum;
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + threadIdx.x * 4 + k;
    if (i < ncell) off[i] = run;
    run += v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) off[ncell] = total;
}

template <typename R>
__global__ void __launch_bounds__(256) k_sort_scatter(KParams P, Soa<R> A, Soa<R> B, const uint32_t *__restrict__ key,
                                                      const uint32_t *__restrict__ rank,
                                                      const uint32_t *__restrict__ off, uint32_t *__restrict__ cellid) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P.n) return;
  const uint32_t c = key[j];
  const int64_t d = (int64_t)off[c] + rank[j];
  B.x[d] = A.x[j];
  B.y[d] = A.y[j];
  B.z[d] = A.z[j];
  B.vx[d] = A.vx[j];
  B.vy[d] = A.vy[j];
  B.vz[d] = A.vz[j];
  B.qs[d] = A.qs[j];
  B.pid[d] = A.pid[j];
  B.birth[d] = A.birth[j];
  cellid[d] = c;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u8(uint8_t *p, uint8_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_f64(double *p, double v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

static unsigned fill_grid(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (unsigned)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(n)), dim3(256), 0, st, p, v, n);
}
void launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_fill_u8, dim3(fill_grid(n)), dim3(256), 0, st, p, v, n);
}
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_fill_f64, dim3(fill_grid(n)), dim3(256), 0, st, p, v, n);
}

size_t scan_blocksums_len(int64_t ncell) { return (size_t)((ncell + kScanBlock - 1) / kScanBlock) + 1; }

template <typename R>
void launch_sort(const KParams &P, Soa<R> A, Soa<R> B, const uint32_t *given, uint32_t *key, uint32_t *rank,
                 uint32_t *count, uint32_t *cell_off, uint32_t *blocksums, uint32_t *cellid_out, int64_t ncell,
                 hipStream_t st) {
  const unsigned gp = (unsigned)((P.n + 255) / 256);
  const unsigned nb = (unsigned)((ncell + kScanBlock - 1) / kScanBlock);
  launch_fill_u32(count, 0u, ncell, st);
  if (P.n > 0) hipLaunchKernelGGL(k_sort_count<R>, dim3(gp), dim3(256), 0, st, P, A, given, key, rank, count);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(256), 0, st, count, ncell, blocksums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, st, blocksums, (int64_t)nb);
  hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(256), 0, st, count, ncell, blocksums, cell_off, (uint32_t)P.n);
  if (P.n > 0) hipLaunchKernelGGL(k_sort_scatter<R>, dim3(gp), dim3(256), 0, st, P, A, B, key, rank, cell_off, cellid_out);
}

template void launch_sort<double>(const KParams &, Soa<double>, Soa<double>, const uint32_t *, uint32_t *, uint32_t *,
                                  uint32_t *, uint32_t *, uint32_t *, uint32_t *, int64_t, hipStream_t);
template void launch_sort<float>(const KParams &, Soa<float>, Soa<float>, const uint32_t *, uint32_t *, uint32_t *,
                                 uint32_t *, uint32_t *, uint32_t *, uint32_t *, int64_t, hipStream_t);

// ---------------------------------------------------------------------------
// self-test kernels
// ---------------------------------------------------------------------------
__global__ void k_selftest_philox(uint32_t k0, uint32_t k1, uint32_t ctr0, uint32_t c1, uint32_t c2, uint32_t c3,
                                  int64_t n, uint32_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint4 r = philox(ctr0 + (uint32_t)i, c1, c2, c3, k0, k1);
  out[4 * i + 0] = r.x;
  out[4 * i + 1] = r.y;
  out[4 * i + 2] = r.z;
  out[4 * i + 3] = r.w;
}

__global__ void k_selftest_divsqrt(const double *a, const double *b, int64_t n, double *q, double *r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  q[i] = a[i] / b[i];
  r[i] = sqrt(a[i]);
}

void launch_selftest_philox(uint64_t seed, uint32_t ctr0, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
                            uint32_t *out, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_selftest_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (uint32_t)seed,
                       (uint32_t)(seed >> 32), ctr0, c1, c2, c3, n, out);
}
void launch_selftest_divsqrt(const double *a, const double *b, int64_t n, double *q, double *r, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_selftest_divsqrt, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n, q, r);
}

}  // namespace ecr
