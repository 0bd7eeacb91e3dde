// Test pin: prints Philox4x32-10 blocks from rocRAND's host-callable engine
// (a library implementation independent of the oracle and of the HIP library).
// Usage: rocrand_philox_blocks SEED SUBSEQUENCE FIRST COUNT
// Prints one line per block: four decimal 32-bit words, for the blocks at
// positions FIRST .. FIRST+COUNT-1 of the given subsequence.
#include <cstdio>
#include <cstdlib>
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>

int main(int argc, char** argv)
{
    if (argc != 5) {
        std::fprintf(stderr, "usage: %s SEED SUBSEQUENCE FIRST COUNT\n", argv[0]);
        return 2;
    }
    unsigned long long seed = std::strtoull(argv[1], nullptr, 0);
    unsigned long long subseq = std::strtoull(argv[2], nullptr, 0);
    unsigned long long first = std::strtoull(argv[3], nullptr, 0);
    unsigned long long count = std::strtoull(argv[4], nullptr, 0);
    for (unsigned long long j = 0; j < count; ++j) {
        rocrand_state_philox4x32_10 state;
        rocrand_init(seed, subseq, 4ull * (first + j), &state);
        uint4 r = rocrand4(&state);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
