// Independent Philox4x32-10 reference for the oracle's pin: calls PyTorch's
// header-only at::philox_engine (it is not copied here). Reads lines
// "k0 k1 c0 c1 c2 c3" and prints the four output words of each block.
//
// Mapping: philox_engine(seed, subsequence, offset) keys the block with
// (seed lo, seed hi) and starts at counter (offset lo, offset hi,
// subsequence lo, subsequence hi); four calls return the block's words.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>

int main() {
  unsigned long long k0, k1, c0, c1, c2, c3;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
    uint64_t subseq = (uint64_t)c2 | ((uint64_t)c3 << 32);
    uint64_t offset = (uint64_t)c0 | ((uint64_t)c1 << 32);
    at::philox_engine eng(seed, subseq, offset);
    uint32_t x0 = eng(), x1 = eng(), x2 = eng(), x3 = eng();
    std::printf("%u %u %u %u\n", x0, x1, x2, x3);
  }
  return 0;
}
