// Sparse stages of the LOD step and the adjoint's reductions (gfx950).
//
//   source      u <- (u + P) * invQ at merged source entries, with
//               P = dt*sum S*rho and invQ = 1/(1 + dt*sum(S+U)) built in FP64
//               on the host (production and uptake by cells, Sec. 5.3)
//   dirichlet   u[e] <- value at active Dirichlet entries (Sec. 2, 7 stages)
//   adjoint     transposes: mask (zero at Dirichlet entries), source
//               (multiply by invQ), and the second stage of the
//               per-substrate sums sum y*(L_N x) and sum y*x behind dL/dD
//               and dL/dlambda (the transposed sweeps form the per-line sums)
#include "internal.hpp"

namespace bfvm {

template <typename T>
__global__ void k_source(T* u, const int64_t* __restrict__ vox, const double* __restrict__ P,
                         const double* __restrict__ invQ, int64_t m, int S)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m * S) return;
    const int64_t k = t / S;
    const int s = (int)(t - k * S);
    const int64_t e = vox[k] * S + s;
    u[e] = (T)(((double)u[e] + P[t]) * invQ[t]);
}

template <typename T>
__global__ void k_source_transpose(T* g, const int64_t* __restrict__ vox,
                                   const double* __restrict__ invQ, int64_t m, int S)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m * S) return;
    const int64_t k = t / S;
    const int s = (int)(t - k * S);
    const int64_t e = vox[k] * S + s;
    g[e] = (T)((double)g[e] * invQ[t]);
}

template <typename T>
__global__ void k_dirichlet(T* u, const int64_t* __restrict__ elem, const double* __restrict__ val,
                            int64_t cnt)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < cnt) u[elem[t]] = (T)val[t];
}

template <typename T>
__global__ void k_mask(T* g, const int64_t* __restrict__ elem, int64_t cnt)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < cnt) g[elem[t]] = (T)0;
}

static unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

#define DISPATCH_T(dtype, CALL)                    \
    switch (dtype) {                               \
        case DT_F64: { using T = double; CALL; break; } \
        case DT_F32:                               \
        case DT_F32_FAST: { using T = float; CALL; break; } \
        default: return hipErrorInvalidValue;      \
    }

hipError_t launch_source(int dtype, void* u, const int64_t* vox, const double* P, const double* invQ,
                         int64_t m, int32_t S, hipStream_t st)
{
    if (m == 0) return hipSuccess;
    DISPATCH_T(dtype, hipLaunchKernelGGL(k_source<T>, dim3(blocks_for(m * S, 256)), dim3(256), 0, st,
                                         static_cast<T*>(u), vox, P, invQ, m, S));
    return hipGetLastError();
}

hipError_t launch_source_transpose(int dtype, void* g, const int64_t* vox, const double* invQ,
                                   int64_t m, int32_t S, hipStream_t st)
{
    if (m == 0) return hipSuccess;
    DISPATCH_T(dtype, hipLaunchKernelGGL(k_source_transpose<T>, dim3(blocks_for(m * S, 256)), dim3(256),
                                         0, st, static_cast<T*>(g), vox, invQ, m, S));
    return hipGetLastError();
}

hipError_t launch_dirichlet(int dtype, void* u, const int64_t* elem, const double* val, int64_t cnt,
                            hipStream_t st)
{
    if (cnt == 0) return hipSuccess;
    DISPATCH_T(dtype, hipLaunchKernelGGL(k_dirichlet<T>, dim3(blocks_for(cnt, 256)), dim3(256), 0, st,
                                         static_cast<T*>(u), elem, val, cnt));
    return hipGetLastError();
}

hipError_t launch_mask(int dtype, void* g, const int64_t* elem, int64_t cnt, hipStream_t st)
{
    if (cnt == 0) return hipSuccess;
    DISPATCH_T(dtype, hipLaunchKernelGGL(k_mask<T>, dim3(blocks_for(cnt, 256)), dim3(256), 0, st,
                                         static_cast<T*>(g), elem, cnt));
    return hipGetLastError();
}

// ------------------------------------------------------ adjoint reductions

// Second stage of the per-line sums formed inside the transposed sweeps:
// block (s, a) adds the pairs of the lines L = s, s + S, s + 2S, ... of axis
// a, thread t taking every 256th of them in order, then a fixed-order tree:
// deterministic.
struct LineParts {
    const double* p[3];
    int64_t n[3];
};

__global__ __launch_bounds__(256) void k_adj_line_final(LineParts lp, int S, double* __restrict__ out)
{
    __shared__ double s0[256], s1[256];
    const int s = blockIdx.x, a = blockIdx.y;
    const double* part = lp.p[a];
    const int64_t n = lp.n[a];
    double a0 = 0.0, a1 = 0.0;
    for (int64_t L = s + (int64_t)S * threadIdx.x; L < n; L += (int64_t)S * 256) {
        a0 += part[2 * L + 0];
        a1 += part[2 * L + 1];
    }
    s0[threadIdx.x] = a0;
    s1[threadIdx.x] = a1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[((int64_t)a * S + s) * 2 + 0] = s0[0];
        out[((int64_t)a * S + s) * 2 + 1] = s1[0];
    }
}

hipError_t launch_adjoint_line_final(double* const part[3], const int64_t nlines[3], int S, double* out,
                                     hipStream_t st)
{
    LineParts lp;
    for (int a = 0; a < 3; ++a) {
        lp.p[a] = part[a];
        lp.n[a] = nlines[a];
    }
    hipLaunchKernelGGL(k_adj_line_final, dim3((unsigned)S, 3), dim3(256), 0, st, lp, S, out);
    return hipGetLastError();
}

}  // namespace bfvm
