// Independent Philox4x32-10 for the oracle's pin: PyTorch's header-only
// at::Philox4_32 engine (ATen/core/PhiloxRNGEngine.h), compiled with g++.
// stdin: lines "c0 c1 c2 c3 k0 k1" (decimal 32-bit words); stdout: the four
// output words of that counter and key, one line each.  The engine's
// counter is (offset lo, offset hi, subsequence lo, subsequence hi) and its
// key (seed lo, seed hi); four calls return the block's words in order.
#include <ATen/core/PhiloxRNGEngine.h>

#include <cstdio>

int main() {
  unsigned long long c[4], k[2];
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    at::Philox4_32 e(k[0] | (k[1] << 32), c[2] | (c[3] << 32), c[0] | (c[1] << 32));
    const unsigned w0 = e(), w1 = e(), w2 = e(), w3 = e();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
