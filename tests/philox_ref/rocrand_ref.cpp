// Host-side reference stream of rocRAND's Philox4x32-10 engine, used only by
// the test-suite to pin the CPU oracle's Philox implementation.  It calls the
// engine through rocRAND's public device/host API (rocrand_init + rocrand4);
// nothing of rocRAND is copied here.
//
// usage: rocrand_ref <seed> <subsequence> <offset> <count4>
// prints count4 lines "w0 w1 w2 w3" (decimal), the outputs of successive
// rocrand4() calls starting at the given position.
#include <cstdio>
#include <cstdlib>
#include <rocrand/rocrand_kernel.h>

int main(int argc, char** argv) {
    if (argc != 5) { std::fprintf(stderr, "usage\n"); return 2; }
    unsigned long long seed = std::strtoull(argv[1], nullptr, 0);
    unsigned long long subseq = std::strtoull(argv[2], nullptr, 0);
    unsigned long long offset = std::strtoull(argv[3], nullptr, 0);
    long count = std::strtol(argv[4], nullptr, 0);
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, subseq, offset, &st);
    for (long i = 0; i < count; ++i) {
        uint4 v = rocrand4(&st);
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
