// Device-side field set-up: seeded uniform fields and the Gaussian initial
// profile, written directly into HBM (no host staging), for grids larger
// than host memory comfortably holds (e.g. 1500^3 x 8 in FP64 = 216 GB).
//
// The uniform values come from the counter-based SplitMix64 generator
// (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
// OOPSLA 2014), implemented here from its published finaliser: for stream
// key k and element index i, key_i = mix(k ^ i) and U_i = (key_i >> 11) 2^-53
// in [0, 1); k = mix(seed ^ (stream << 56)).  The Gaussian profile is the
// paper's initial condition of the end-to-end run (Sec. 5.3): a blob centred
// in the domain in voxel-centre coordinates (voxel i at i + 1/2).
#include "internal.hpp"

namespace bfvm {

__host__ __device__ inline uint64_t splitmix_mix(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double unit_uniform(uint64_t k0, uint64_t i)
{
    return (double)(splitmix_mix(k0 ^ i) >> 11) * 0x1p-53;
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill_uniform(T* __restrict__ u, int64_t n, uint64_t k0, double lo, double hi)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        u[i] = (T)(lo + (hi - lo) * unit_uniform(k0, (uint64_t)i));
}

// u[(z, y, x, s)] = peak * exp(-d^2 / (2 sigma^2)) + noise * U_i, with d the
// distance of the voxel centre from (cx, cy, cz) in voxel units
template <typename T>
__global__ __launch_bounds__(256) void k_fill_gaussian(T* __restrict__ u, int64_t nx, int64_t ny, int64_t nz, int S,
                                                       double cx, double cy, double cz, double inv2s2,
                                                       double peak, double noise, uint64_t k0)
{
    const int64_t n = nx * ny * nz * S;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t v = i / S;
        const int64_t x = v % nx, y = (v / nx) % ny, z = v / (nx * ny);
        const double dx = (double)x + 0.5 - cx, dy = (double)y + 0.5 - cy, dz = (double)z + 0.5 - cz;
        const double g = peak * exp(-(dx * dx + dy * dy + dz * dz) * inv2s2);
        u[i] = (T)(g + noise * unit_uniform(k0, (uint64_t)i));
    }
}

static unsigned fill_blocks(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 65536 ? (b < 1 ? 1 : b) : 65536);
}

hipError_t launch_fill_uniform(int dtype, void* u, int64_t n, uint64_t seed, uint32_t stream, double lo, double hi,
                               hipStream_t st)
{
    const uint64_t k0 = splitmix_mix(seed ^ ((uint64_t)stream << 56));
    if (dtype == DT_F64)
        hipLaunchKernelGGL(k_fill_uniform<double>, dim3(fill_blocks(n)), dim3(256), 0, st, static_cast<double*>(u),
                           n, k0, lo, hi);
    else
        hipLaunchKernelGGL(k_fill_uniform<float>, dim3(fill_blocks(n)), dim3(256), 0, st, static_cast<float*>(u), n,
                           k0, lo, hi);
    return hipGetLastError();
}

hipError_t launch_fill_gaussian(int dtype, void* u, int64_t nx, int64_t ny, int64_t nz, int S, double cx, double cy,
                                double cz, double sigma, double peak, double noise, uint64_t seed, uint32_t stream,
                                hipStream_t st)
{
    const uint64_t k0 = splitmix_mix(seed ^ ((uint64_t)stream << 56));
    const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
    const int64_t n = nx * ny * nz * S;
    if (dtype == DT_F64)
        hipLaunchKernelGGL(k_fill_gaussian<double>, dim3(fill_blocks(n)), dim3(256), 0, st, static_cast<double*>(u),
                           nx, ny, nz, S, cx, cy, cz, inv2s2, peak, noise, k0);
    else
        hipLaunchKernelGGL(k_fill_gaussian<float>, dim3(fill_blocks(n)), dim3(256), 0, st, static_cast<float*>(u), nx,
                           ny, nz, S, cx, cy, cz, inv2s2, peak, noise, k0);
    return hipGetLastError();
}

}  // namespace bfvm
