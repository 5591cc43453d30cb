// Test harness: Philox4x32-10 words from PyTorch's header-only engine, an
// implementation independent of the oracle's.  Reads lines
// "k0 k1 c0 c1 c2 c3" (hex) from stdin, prints the four output words (hex).
// The engine's state maps key = seed, counter = (offset_lo, offset_hi,
// subsequence_lo, subsequence_hi).
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>

int main() {
  unsigned k0, k1, c0, c1, c2, c3;
  while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    const uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
    const uint64_t offset = (uint64_t)c0 | ((uint64_t)c1 << 32);
    const uint64_t subseq = (uint64_t)c2 | ((uint64_t)c3 << 32);
    at::Philox4_32 e(seed, subseq, offset);
    const uint32_t w0 = e(), w1 = e(), w2 = e(), w3 = e();
    std::printf("%08x %08x %08x %08x\n", w0, w1, w2, w3);
  }
  return 0;
}
