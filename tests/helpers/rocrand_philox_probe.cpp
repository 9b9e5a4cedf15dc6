// Host-side probe of rocRAND's Philox4x32-10 engine (the library's own
// header, called through its public engine API, not copied).  Test helper:
// it gives the oracle's and the device path's Philox an independent pin.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>

extern "C" void rocrand_philox_block(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    // The engine keys on the 64-bit seed (k0 low, k1 high), puts the
    // subsequence in counter words 2-3 and offset/4 in counter words 0-1.
    const unsigned long long seed = (unsigned long long)key[0] | ((unsigned long long)key[1] << 32);
    const unsigned long long subseq = (unsigned long long)ctr[2] | ((unsigned long long)ctr[3] << 32);
    const unsigned long long block = (unsigned long long)ctr[0] | ((unsigned long long)ctr[1] << 32);
    rocrand_device::philox4x32_10_engine eng(seed, subseq, 4ull * block);
    uint4 r = eng.next4();
    out[0] = r.x; out[1] = r.y; out[2] = r.z; out[3] = r.w;
}
