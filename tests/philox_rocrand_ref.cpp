// Reference Philox4x32-10 words from rocRAND's engine (host build), used to pin
// the oracle's own Philox.  Reads lines "key0 key1 c0 c1 c2 c3" (hex) on stdin
// and prints the four output words of the block with that counter and key.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long blocks = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
        rocrand_device::philox4x32_10_engine e(seed, subseq, 0);
        // discard(n) advances by n words = n/4 blocks; split to avoid overflow of 4*blocks.
        for (int k = 0; k < 4; ++k) e.discard(4ull * (blocks >> 2));
        e.discard(4ull * (blocks & 3ull));
        uint4 r = e.next4();
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
