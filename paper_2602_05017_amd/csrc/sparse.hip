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

// The per-line sums formed inside the transposed sweeps (pairs part[2 L],
// part[2 L + 1]; line L holds substrate L % S) added per (axis, substrate)
// in two stages, each in a fixed order (deterministic):
//   chunks: block (b, a) takes lines [b C, b C + C) of axis a (C a multiple
//     of S); thread t < T = S floor(256 / S) adds the lines b C + t, + T, ...
//     (all of substrate t % S), coalesced; then thread s < S adds the
//     threads s, s + S, ... in order and writes the chunk's pair of
//     substrate s over line b C + s, inside the block's own chunk (S > 256:
//     thread t adds substrates t, t + 256, ... line by line);
//   final: block (s, a) adds the chunks' pairs of substrate s, thread t
//     taking every 256th chunk in order, then a fixed-order tree.
// A single stage of S x 3 blocks, each walking every S-th line of an axis,
// left most CUs idle: 0.54 ms for the 3 x 2^20 lines of a 512^3 x 4 grid,
// against 0.025 ms for the two stages.
struct LineParts {
    double* p[3];
    int64_t n[3];
    int64_t C[3];   // lines per chunk
};

__global__ __launch_bounds__(256) void k_adj_line_chunks(LineParts lp, int S)
{
    __shared__ double s0[256], s1[256];
    const int a = blockIdx.y;
    double* part = lp.p[a];
    const int64_t L0 = (int64_t)blockIdx.x * lp.C[a];
    if (L0 >= lp.n[a]) return;
    const int64_t L1 = min(L0 + lp.C[a], lp.n[a]);
    const int t = threadIdx.x;
    if (S <= 256) {
        const int T = S * (256 / S);
        double a0 = 0.0, a1 = 0.0;
        if (t < T)
            for (int64_t L = L0 + t; L < L1; L += T) {
                a0 += part[2 * L + 0];
                a1 += part[2 * L + 1];
            }
        s0[t] = a0;
        s1[t] = a1;
        __syncthreads();   // every read of the chunk is done
        if (t < S) {
            double b0 = 0.0, b1 = 0.0;
            for (int u = t; u < T; u += S) {
                b0 += s0[u];
                b1 += s1[u];
            }
            part[2 * (L0 + t) + 0] = b0;
            part[2 * (L0 + t) + 1] = b1;
        }
    } else {
        // only this thread reads the lines of its substrates
        for (int ss = t; ss < S; ss += 256) {
            double b0 = 0.0, b1 = 0.0;
            for (int64_t L = L0 + ss; L < L1; L += S) {
                b0 += part[2 * L + 0];
                b1 += part[2 * L + 1];
            }
            part[2 * (L0 + ss) + 0] = b0;
            part[2 * (L0 + ss) + 1] = b1;
        }
    }
}

__global__ __launch_bounds__(256) void k_adj_line_final(LineParts lp, int S, double* __restrict__ out)
{
    __shared__ double s0[256], s1[256];
    const int s = blockIdx.x, a = blockIdx.y;
    const double* part = lp.p[a];
    const int64_t C = lp.C[a];
    const int64_t nb = (lp.n[a] + C - 1) / C;
    double a0 = 0.0, a1 = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += 256) {
        const int64_t L = b * C + s;
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
    int64_t gmax = 1;
    for (int a = 0; a < 3; ++a) {
        lp.p[a] = part[a];
        lp.n[a] = nlines[a];
        // about 512 chunks per axis; whole rows of S lines each
        const int64_t rows = nlines[a] / S;
        const int64_t R = std::max<int64_t>(1, (rows + 511) / 512);
        lp.C[a] = R * S;
        gmax = std::max<int64_t>(gmax, (nlines[a] + lp.C[a] - 1) / lp.C[a]);
    }
    hipLaunchKernelGGL(k_adj_line_chunks, dim3((unsigned)gmax, 3), dim3(256), 0, st, lp, S);
    hipLaunchKernelGGL(k_adj_line_final, dim3((unsigned)S, 3), dim3(256), 0, st, lp, S, out);
    return hipGetLastError();
}

}  // namespace bfvm
