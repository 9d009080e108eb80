/* Multi-threaded fill with counter-based SplitMix64 uniforms (input generation
 * only; no part of the diffusion method).  Value i of the stream keyed by k0
 * is lo + (hi - lo) * (mix(k0 ^ (start + i)) >> 11) * 2^-53, identical to the
 * numpy form in workloads/__init__.py. */
#include <stdint.h>

static inline uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

void splitmix_uniform(uint64_t k0, uint64_t unused, int64_t start, int64_t count,
                      double lo, double hi, double* out)
{
    (void)unused;
    const double scale = 1.0 / 9007199254740992.0; /* 2^-53 */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        uint64_t k = mix64(k0 ^ (uint64_t)(start + i));
        out[i] = lo + (hi - lo) * ((double)(k >> 11) * scale);
    }
}
