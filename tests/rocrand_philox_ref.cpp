// Host program for the Philox4x32-10 pin of the oracle's noise generator:
// the ten-round bijection of rocRAND's engine (an implementation of Salmon,
// Moraes, Dror and Shaw, SC'11, written independently of this repository)
// applied to (counter, key) blocks. Test infrastructure only.
//
// stdin: one block per line, "c0 c1 c2 c3 k0 k1" (decimal uint32);
// stdout: "o0 o1 o2 o3" for each block, in order.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

namespace {

// The engine keeps its ten-round function protected; a derived type exposes
// it without touching the engine's own counter and key handling.
struct Exposed : rocrand_device::philox4x32_10_engine {
  uint4 bijection(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

}  // namespace

int main() {
  Exposed e;
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    const uint4 o = e.bijection(make_uint4(c0, c1, c2, c3), make_uint2(k0, k1));
    std::printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
  }
  return 0;
}
