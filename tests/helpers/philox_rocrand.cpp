// Host-only helper for the oracle's Philox pin: prints rocRAND's
// philox4x32_10 output for a given counter and key.  rocRAND addresses the
// counter through (subsequence, offset): words 2,3 are the subsequence and
// words 0,1 the offset in blocks of four outputs, so word 1 must stay below
// 2^30 for the offset to fit 64 bits.
// usage: philox_rocrand c0 c1 c2 c3 k0 k1   (hex words)
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv)
{
    if (argc != 7) return 2;
    unsigned c[4], k[2];
    for (int i = 0; i < 4; i++) c[i] = (unsigned)strtoul(argv[1 + i], 0, 16);
    for (int i = 0; i < 2; i++) k[i] = (unsigned)strtoul(argv[5 + i], 0, 16);
    rocrand_state_philox4x32_10 st;
    unsigned long long seed = ((unsigned long long)k[1] << 32) | k[0];
    unsigned long long sub = ((unsigned long long)c[3] << 32) | c[2];
    unsigned long long off = 4ULL * (((unsigned long long)c[1] << 32) | c[0]);
    rocrand_init(seed, sub, off, &st);
    uint4 v = rocrand4(&st);
    printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
    return 0;
}
