// ecr_kernels.hpp -- launch entry points of the gfx950 kernels (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ecr_device.hpp"
#include "ecrpic.h"

namespace ecr {

// Coulomb chunking: a workgroup owns the cells whose first sorted slot falls
// in [b*kCoulCap, (b+1)*kCoulCap); it sorts up to kCoulMaxE entries in LDS.
constexpr int kCoulCap = 512;
constexpr int kCoulMaxE = 2048;

// Error bits raised by kernels (read back with the tallies).
enum : uint32_t { ERR_COUL_OVERFLOW = 1 };

struct DevAccum {
  ecr_tallies t;        // steps field unused on the device
  uint32_t err;         // ERR_* bits
  uint32_t pad[63];
};

template <typename R>
void launch_init(const KParams &P, Soa<R> S, hipStream_t st);

template <typename R>
void launch_push(const KParams &P, const Tables *T, Soa<R> S, const double *ef, uint8_t *evlog,
                 DevAccum *acc, uint32_t step, hipStream_t st);

template <typename R>
void launch_deposit(const KParams &P, Soa<R> S, double *dens, hipStream_t st);

template <typename R>
void launch_coulomb(const KParams &P, const Tables *T, Soa<R> S, const uint32_t *cellid,
                    const uint32_t *cell_off, int64_t ncell, DevAccum *acc, uint32_t step, hipStream_t st);

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
