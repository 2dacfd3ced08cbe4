// Prints Philox4x32-10 output blocks computed by rocRAND's header-only engine,
// run on the host.  Used only by the test suite as an independent reference
// for the oracle's Philox.  Reads lines "seed subsequence offset" from stdin
// (decimal, 64-bit) and prints the first four 32-bit outputs of each stream
// in hexadecimal.  rocRAND maps the subsequence to counter words 2-3 and
// offset/4 to counter words 0-1.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main() {
    unsigned long long seed, sub, off;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, off, &st);
        for (int i = 0; i < 4; ++i) std::printf("%08x ", rocrand(&st));
        std::printf("\n");
    }
    return 0;
}
