// Reads lines "c0 c1 c2 c3 k0 k1" (hex) and prints Philox4x32-10 outputs from
// PyTorch's own engine (ATen/core/PhiloxRNGEngine.h), an implementation
// independent of this repository's.  Test infrastructure only.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    at::Philox4_32 e((static_cast<uint64_t>(k1) << 32) | k0,
                     (static_cast<uint64_t>(c3) << 32) | c2, 0);
    e.set_offset((static_cast<uint64_t>(c1) << 32) | c0);
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%08x %08x %08x %08x\n", a, b, c, d);
  }
  return 0;
}
