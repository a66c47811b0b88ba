// Host-side reader of rocRAND's Philox4x32-10 engine, used to pin the oracle's
// Philox to an implementation it shares no code with.  Reads lines
// "seed c0 c1 c2 c3" on stdin and prints the 4 output words of the block whose
// key is seed and whose counter is (c0, c1, c2, c3).  rocRAND's engine keeps
// the counter's high 64 bits as the subsequence and counts offsets in words
// (4 per block), so engine(seed, c2 | c3 << 32, 4 * c0) sits at counter
// (c0, 0, c2, c3); four discards of c1 << 32 words then add c1 << 32 blocks,
// which moves it to (c0, c1, c2, c3) without overflowing the 64-bit offset.
// next4() returns that block.  Runs on the host only.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long seed, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
        rocrand_device::philox4x32_10_engine eng(seed, c2 | (c3 << 32), 4ull * c0);
        for (int k = 0; k < 4; ++k) eng.discard(c1 << 32);
        uint4 v = eng.next4();
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
