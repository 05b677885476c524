// Prints Philox4x32-10 blocks computed by PyTorch's own host-side engine
// (ATen/core/PhiloxRNGEngine.h), an implementation independent of the
// oracle's.  The engine's state maps onto a raw (counter, key) block as:
// key = seed, counter words 0-1 = offset, counter words 2-3 = subsequence.
// Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin, prints four hex words.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>

int main() {
  unsigned c[4], k[2];
  while (std::scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    uint64_t seed = (uint64_t)k[0] | ((uint64_t)k[1] << 32);
    uint64_t subseq = (uint64_t)c[2] | ((uint64_t)c[3] << 32);
    uint64_t offset = (uint64_t)c[0] | ((uint64_t)c[1] << 32);
    at::Philox4_32 eng(seed, subseq, offset);
    unsigned w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
    std::printf("%08x %08x %08x %08x\n", w0, w1, w2, w3);
  }
  return 0;
}
