// Host-only probe: prints rocRAND's Philox4x32-10 block function for the
// (counter, key) pairs read from stdin, one "c0 c1 c2 c3 k0 k1" line each
// (hex).  Used by the test suite as an independent cross-check of the
// oracle's generator; it runs on the CPU and touches no GPU.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Probe : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  Probe p;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 r = p.block(make_uint4(c0, c1, c2, c3), make_uint2(k0, k1));
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
