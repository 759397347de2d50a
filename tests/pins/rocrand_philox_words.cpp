// Host-side pin for the oracle's Philox4x32-10: prints the raw output words of
// rocRAND's philox4x32_10 engine (header-only, host-callable) for a seed, a
// subsequence (= the method's stream word) and a list of counters.  The engine
// built with (seed, subsequence s, offset 4 c) holds key (seed lo, seed hi) and
// counter (c lo, c hi, s lo, s hi), so next4() returns Philox(counter, key).
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv) {
  if (argc < 4) return 2;
  unsigned long long seed = std::strtoull(argv[1], nullptr, 0);
  unsigned long long stream = std::strtoull(argv[2], nullptr, 0);
  for (int a = 3; a < argc; ++a) {
    unsigned long long c = std::strtoull(argv[a], nullptr, 0);
    rocrand_device::philox4x32_10_engine e(seed, stream, 4ull * c);
    uint4 r = e.next4();
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
