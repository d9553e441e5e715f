// Host-side driver around rocRAND's Philox4x32-10 engine (an implementation
// independent of both the oracle and the GPU library).  Reads lines
// "x y z w k0 k1" (decimal u32) on stdin and prints the 4 output words of
// the block with counter (x, y, z, w) under key (k0, k1).
//
// The engine is reached through its public interface: seed = k0 | k1<<32,
// subsequence = z | w<<32 (the two high counter words), offset = 4*(x | y<<32)
// (whole blocks in the two low counter words).  Requires y < 2^30.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long x, y, z, w, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &x, &y, &z, &w, &k0, &k1) == 6) {
        if (y >= (1ull << 30)) return 2;
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long subseq = z | (w << 32);
        unsigned long long offset = 4ull * (x | (y << 32));
        rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
        uint4 o = e.next4();
        std::printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
