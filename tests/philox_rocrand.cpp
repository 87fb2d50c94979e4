// Test helper, host only: the Philox4x32-10 block function of rocRAND (an
// implementation independent of this repository), so that the oracle's own
// Philox can be compared with it word for word.
//
// Reads lines "c0 c1 c2 c3 k0 k1" (hex words) on stdin and writes the four
// output words of the block for counter (c0, c1, c2, c3) and key (k0, k1),
// in hex, one line per input line.
#include <cstdio>

#include <rocrand/rocrand_philox4x32_10.h>

// ten_rounds is a protected member of rocRAND's engine: the block function
// proper, with no stream state around it
struct Block : rocrand_device::philox4x32_10_engine {
    uint4 operator()(uint4 ctr, uint2 key) { return ten_rounds(ctr, key); }
};

int main() {
    Block block;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        const uint4 y = block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", y.x, y.y, y.z, y.w);
    }
    return 0;
}
