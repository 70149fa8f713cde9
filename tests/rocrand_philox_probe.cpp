// Host-only probe: runs rocRAND's Philox4x32-10 round function on
// (counter, key) lines read from stdin and prints the four output words.
// Used by the oracle's RNG pin test (a library implementation of the same
// published generator); built for the host by the test itself.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

struct Engine : rocrand_device::philox4x32_10_engine {
    uint4 rounds(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    Engine e;
    unsigned a[6];
    while (std::scanf("%x %x %x %x %x %x", &a[0], &a[1], &a[2], &a[3], &a[4], &a[5]) == 6) {
        uint4 c = {a[0], a[1], a[2], a[3]};
        uint2 k = {a[4], a[5]};
        uint4 r = e.rounds(c, k);
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
