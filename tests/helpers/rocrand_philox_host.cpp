// Test helper: prints Philox4x32-10 blocks from the ROCm rocRAND engine, run on
// the host CPU.  rocRAND's engine with subsequence S and offset 4*O evaluates
// the block at counter (O lo, O hi, S lo, S hi) under key (seed lo, seed hi),
// which lets the tests compare the oracle's generator with an independent
// implementation.  Usage: rocrand_philox_host seed subsequence block_offset
#include <cstdio>
#include <cstdlib>
#include <rocrand/rocrand_philox4x32_10.h>

int main(int argc, char** argv)
{
    if (argc != 4) return 2;
    unsigned long long seed = std::strtoull(argv[1], nullptr, 0);
    unsigned long long sub = std::strtoull(argv[2], nullptr, 0);
    unsigned long long off = std::strtoull(argv[3], nullptr, 0);
    rocrand_device::philox4x32_10_engine eng(seed, sub, 4ull * off);
    for (int k = 0; k < 4; ++k) std::printf("%u\n", eng.next());
    return 0;
}
