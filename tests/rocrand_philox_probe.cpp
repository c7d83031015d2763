// Host-side driver of rocRAND's Philox4x32-10 engine, used only by the oracle's pin
// tests as an implementation of the published generator written independently of
// this repository.  Reads "seed subsequence offset" triples from stdin and prints the
// first four 32-bit outputs of each engine.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
    unsigned long long seed, sub, off;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
