// The x sweep of one x-slab: one process's share of the distributed solver
// (Sec. 3.2).  The distributed form splits the domain along x into slabs,
// one per process.  Along x, the forward elimination runs slab after slab,
// each slab handing the eliminated values of its last x-plane to the next;
// the backward substitution then runs back, each slab handing the solution
// values of its first x-plane to the previous.  The systems (the (y, z,
// substrate) lines) are processed in blocks, so that while one slab works
// on a block the next works on the block before it.
//
// On one GPU this is the per-process part: two kernels over a block of
// lines [l0, l1) of a slab [x0, x1) of an nx-voxel grid, stored as the
// slab's own array [nz][ny][m][S] (m = x1 - x0, x fastest, then substrate
// innermost as in the whole field):
//   forward:  d' over the slab from the field values, with the carry
//             d'_{x0-1} of each line coming in (none at x0 = 0); d' replaces
//             the field values; out: d'_{x1-1} of each line;
//   backward: x over the slab from d', with x_{x1} of each line coming in
//             (none at x1 = nx); x replaces d'; out: x_{x0} of each line.
// Chained over the slabs (forward slab 0, 1, ...; backward slab P-1, ...,
// 0) they give the whole-line solve of the x sweep, up to rounding order.
// Each element is read and written once in each direction: 4 element moves
// per sweep, against 2 for a whole-line tile (the values wait in memory
// between the directions, while the other slabs work).
//
// Tiles as the x rows of kind 3: lpw consecutive lines (line L is row L / S,
// substrate L % S) x K segments of M, the carries between segments by the
// leader scan with the incoming carry as its initial value.  The forward
// kernel puts slot j at slab position j (padding past m); the backward
// kernel puts it at j - (K*M - m) (padding before 0), so that in either
// direction the incoming carry enters the line's first real slot and the
// padding (coefficient 0) lies past the line's far end.  The slab's window
// [x0, x1) of the Thomas constants is staged in LDS per block.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.hpp"
#include "seg_solver.hpp"

namespace bfvm {

namespace {

// window [x0, x0 + m) of the [n][S] table in [s][segment][k] layout with a
// segment stride of M + 1 and substrate stride SPw; slot j holds position
// j - shift of the window (0 outside it)
template <typename C, int M>
__device__ __forceinline__ void stage_window(C* tab, const C* __restrict__ invd, int x0, int m, int S, int K,
                                             int SPw, int shift)
{
    const int KM = K * M;
    for (int e = threadIdx.x; e < S * KM; e += blockDim.x) {
        const int s = e / KM, j = e - s * KM, i = j - shift;
        tab[s * SPw + (j / M) * (M + 1) + j % M] = (i >= 0 && i < m) ? invd[(int64_t)(x0 + i) * S + s] : (C)0;
    }
}

template <typename T, typename C, int M, bool FWD>
__global__ __launch_bounds__(1024) void k_xslab(T* slab, int m, int S, int64_t l0, int64_t nlines,
                                                const C* __restrict__ invd, const C* __restrict__ rr, int x0,
                                                int lpw, int SPw, const C* __restrict__ cin, C* __restrict__ cout)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int K = blockDim.x / lpw;
    const int A = K * lpw;
    C* sF = reinterpret_cast<C*>(smem);
    C* sG = sF + A;
    C* tab = sG + A;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int line = lane % lpw;
    const int seg = wave * (64 / lpw) + lane / lpw;
    const int slot = seg * lpw + line;
    const int64_t q = (int64_t)blockIdx.x * lpw + line;   // line within the block of lines
    const bool valid = q < nlines;
    const int64_t qa = valid ? q : nlines - 1;
    const int64_t L = l0 + qa;
    const int64_t row = L / S;
    const int s = (int)(L - row * S);
    const int shift = FWD ? 0 : K * M - m;
    const int i0 = seg * M - shift;                         // slab position of slot 0 of the segment
    const int64_t rowbase = row * (int64_t)m * S + s;
    C v[M];
    // the loads at a raised wave priority, so that a wave loading its tile
    // is not held behind another block's solve on its SIMD (125-voxel slab
    // of the 1000^3 x 4 FP64 cube: 3.40 -> 3.29 ms; the batched tiles were
    // 2% slower with it, the headline z sweep 2% faster)
    __builtin_amdgcn_s_setprio(2);
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int i = std::min(std::max(i0 + k, 0), m - 1);   // padding: clamped, in bounds
        v[k] = (C)slab[rowbase + (int64_t)i * S];
    }
    __builtin_amdgcn_s_setprio(0);
    stage_window<C, M>(tab, invd, x0, m, S, K, SPw, shift);
    __syncthreads();
    const LdsCoef<C> coef{tab + s * SPw + seg * (M + 1), (C)0};
    const C r = rr[s];
    const C init = cin ? cin[qa] : (C)0;
    C f, G;
    if constexpr (FWD) {
        seg_forward<C, M, false>(v, r, coef, f, G);
        sF[slot] = f;
        sG[slot] = G;
        __syncthreads();
        if ((int)threadIdx.x < lpw) carry_scan(sF, sG, K, lpw, (int)threadIdx.x, false, init);
        __syncthreads();
        seg_fwd_correct<C, M, false>(v, r, coef, sF[slot]);
    } else {
        seg_bwd_local<C, M, false>(v, r, coef, f, G);
        sF[slot] = f;
        sG[slot] = G;
        __syncthreads();
        if ((int)threadIdx.x < lpw) carry_scan(sF, sG, K, lpw, (int)threadIdx.x, true, init);
        __syncthreads();
        seg_last<C, M>(v, r, coef, sF[slot]);
    }
    // store the real slots; the value handed on: d'_{m-1} (forward) or x_0
    // (backward), from the thread holding that slot
    const int edge = FWD ? m - 1 : 0;
    C out = (C)0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int i = i0 + k;
        if (valid && i >= 0 && i < m) slab[rowbase + (int64_t)i * S] = (T)v[k];
        if (i == edge) out = v[k];
    }
    if (valid && edge >= i0 && edge < i0 + M) cout[q] = out;
}

}  // namespace

// M and segments for an m-voxel slab line, lpw lines per tile (as the kind-3
// x rows); 0 if m is beyond the kernels' reach.  Measured on the 125-voxel
// slab of the 1000^3 x 4 FP64 cube (forward + backward over 16 blocks):
// M = 8 in 32-line tiles 3.41 ms, M = 16 3.72 ms, M = 4 3.65 ms, M = 8 in
// 64-line tiles 3.52 ms.
int xslab_plan(int64_t m, int* M, int* K, int* lpw)
{
    if (m < 1 || m > 2048) return 0;
    *M = m >= 192 ? 32 : 8;
    const int segs = (int)((m + *M - 1) / *M);
    *lpw = segs <= 16 ? 32 : 16;
    const int spw = 64 / *lpw;
    *K = (segs + spw - 1) / spw * spw;
    return *K * *lpw <= 1024 ? 1 : 0;
}

size_t xslab_lds(int M, int K, int lpw, int S, int cs)
{
    const int SPw = K * (M + 1) + 1;
    return (size_t)(2 * K * lpw) * cs + (size_t)S * SPw * cs;
}

template <typename T, typename C>
static hipError_t launch_xslab_t(bool fwd, void* slab, int64_t m, int S, int64_t l0, int64_t nlines, const void* invd,
                                 const void* r, int64_t x0, const void* cin, void* cout, hipStream_t st)
{
    int M = 0, K = 0, lpw = 0;
    if (!xslab_plan(m, &M, &K, &lpw)) return hipErrorInvalidValue;
    const int SPw = K * (M + 1) + 1;
    const size_t lds = xslab_lds(M, K, lpw, S, sizeof(C));
    const dim3 grid((unsigned)((nlines + lpw - 1) / lpw)), block((unsigned)(K * lpw));
    T* sp = static_cast<T*>(slab);
    const C* cf = static_cast<const C*>(invd);
    const C* rr = static_cast<const C*>(r);
    const C* ci = static_cast<const C*>(cin);
    C* co = static_cast<C*>(cout);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, block, lds, st, sp, (int)m, S, l0, nlines, cf, rr, (int)x0, lpw, SPw, ci, co);
    };
    if (M == 8) fwd ? go(k_xslab<T, C, 8, true>) : go(k_xslab<T, C, 8, false>);
    else fwd ? go(k_xslab<T, C, 32, true>) : go(k_xslab<T, C, 32, false>);
    return hipGetLastError();
}

hipError_t launch_xslab(int dtype, bool fwd, void* slab, int64_t m, int S, int64_t l0, int64_t nlines,
                        const void* invd, const void* r, int64_t x0, const void* cin, void* cout, hipStream_t st)
{
    if (nlines == 0) return hipSuccess;
    switch (dtype) {
        case DT_F64: return launch_xslab_t<double, double>(fwd, slab, m, S, l0, nlines, invd, r, x0, cin, cout, st);
        case DT_F32: return launch_xslab_t<float, double>(fwd, slab, m, S, l0, nlines, invd, r, x0, cin, cout, st);
        case DT_F32_FAST:
            return launch_xslab_t<float, float>(fwd, slab, m, S, l0, nlines, invd, r, x0, cin, cout, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bfvm
