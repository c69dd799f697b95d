// Independent Philox4x32-10 for the oracle's pin test: rocRAND's host-side
// engine.  Reads lines "k0 k1 c0 c1 c2 c3" (hex) and prints the four output
// words.  rocRAND maps (seed, subsequence, offset) onto the Philox key and
// counter as key = seed, counter = (offset/4 as 64 bits, subsequence as 64
// bits), so each counter is reached through that mapping.
#include <cstdio>
#include <rocrand/rocrand_kernel.h>

int main() {
  unsigned k0, k1, c0, c1, c2, c3;
  while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
    unsigned long long subseq = ((unsigned long long)c3 << 32) | c2;
    unsigned long long ofs4 = ((unsigned long long)c1 << 32) | c0;
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, subseq, 0, &st);
    // offset counts 32-bit outputs: 4 per counter value; skip in pieces to
    // avoid overflow of 4*ofs4
    for (int i = 0; i < 4; ++i) skipahead(ofs4, &st);
    unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
    std::printf("%08x %08x %08x %08x\n", a, b, c, d);
  }
  return 0;
}
