// Thomas sweeps of the LOD diffusion-decay step on gfx950.
//
// One sweep solves, for every grid line along one axis and every substrate,
// the constant-coefficient tridiagonal system of App. A (off-diagonals -r,
// diagonal 1+r+beta at the ends, 1+2r+beta inside) with the Thomas algorithm
// (Sec. 2, Algorithm 1; Sec. 2.1 Eq. 2).  Lines are independent, so the GPU
// parallelises across lines (Sec. 2 and Sec. 3.3: parallelism across
// systems, not within one).  With invd_i = 1/denom_i and alpha_i = r*invd_i
// (note -c'_i = alpha_i), Thomas is
//     forward   t_i = invd_i * (d_i + r * t_{i-1})          (t_{-1} = 0)
//     backward  x_i = t_i + alpha_i * x_{i+1}                (x_n = 0)
// and the transposed solve (A = L U: solve U^T w = g, then L^T y = w) is
//     forward   w_i = g_i + alpha_{i-1} * w_{i-1}
//     backward  y_i = invd_i * (w_i + r * y_{i+1}).
// Both passes are first-order linear recurrences, so a line can be cut into
// segments: each segment is solved with a zero carry, and the true carry of
// segment j follows from an affine scan over the segments before it
// (forward) or after it (backward), using the segment's last (first) local
// value and the product of its recurrence coefficients.  The local result is
// then corrected by carry * (running product of coefficients).  This keeps a
// whole line on chip in registers between the two passes, so every element
// is read from HBM once and written once per sweep.
//
// Kernels:
//   k_sweep_line         one thread per line, both passes through memory
//                        (simple fallback: 2 reads + 2 writes per element)
//   k_sweep_seg_strided  y and z: lanes over neighbouring lines (coalesced,
//                        substrate-innermost layout), waves over segments
//   k_sweep_seg_xtile    x: rows of nx*S contiguous elements staged through
//                        LDS (coalesced load/store), lanes over segments
#include "internal.hpp"

#include <algorithm>

namespace bfvm {

AxisGeom axis_geom(int axis, int64_t nx, int64_t ny, int64_t nz, int32_t S)
{
    AxisGeom g;
    g.S = S;
    if (axis == 0) {
        g.n = nx; g.inner = S; g.outer = nz * ny; g.stride = S; g.outer_stride = nx * S;
    } else if (axis == 1) {
        g.n = ny; g.inner = nx * S; g.outer = nz; g.stride = nx * S; g.outer_stride = ny * nx * S;
    } else {
        g.n = nz; g.inner = ny * nx * S; g.outer = 1; g.stride = ny * nx * S;
        g.outer_stride = ny * nx * S * nz;
    }
    return g;
}

// ------------------------------------------------------------ kind 0 (line)

template <typename T, typename C, bool TR>
__global__ __launch_bounds__(256) void k_sweep_line(const T* in, T* out, AxisGeom g,
                                                    const C* __restrict__ invd,
                                                    const C* __restrict__ rr)
{
    const int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= g.inner * g.outer) return;
    const int64_t o = L / g.inner;
    const int64_t p = L - o * g.inner;
    const int S = g.S;
    const int s = (int)(p % S);
    const int64_t base = o * g.outer_stride + p;
    const int64_t n = g.n, st = g.stride;
    const C r = rr[s];
    if (!TR) {
        C t = 0;
        for (int64_t i = 0; i < n; ++i) {
            t = invd[i * S + s] * ((C)in[base + i * st] + r * t);
            out[base + i * st] = (T)t;
        }
        C x = 0;
        for (int64_t i = n - 1; i >= 0; --i) {
            x = (C)out[base + i * st] + r * invd[i * S + s] * x;
            out[base + i * st] = (T)x;
        }
    } else {
        C w = 0;
        for (int64_t i = 0; i < n; ++i) {
            const C a = i > 0 ? r * invd[(i - 1) * S + s] : (C)0;
            w = (C)in[base + i * st] + a * w;
            out[base + i * st] = (T)w;
        }
        C y = 0;
        for (int64_t i = n - 1; i >= 0; --i) {
            y = invd[i * S + s] * ((C)out[base + i * st] + r * y);
            out[base + i * st] = (T)y;
        }
    }
}

// ------------------------------------------------ segment solver (registers)
//
// Shared by both segmented kernels.  v[0..cnt) holds the segment's inputs
// (elements i0 .. i0+cnt-1 of line `line`, substrate s); on return it holds
// the final solution.  sF/sG are LDS arrays of [K][nl] carry terms, indexed
// [segment * nl + line].  Every thread of the block must call this (it
// contains barriers); threads without a valid segment pass cnt = 0.

template <typename C, int M, bool TR>
__device__ __forceinline__ void solve_segment(C (&v)[M], int cnt, int64_t i0, int seg, int K,
                                              int line, int nl, int s, int S, C r,
                                              const C* __restrict__ invd, C* sF, C* sG,
                                              bool writer)
{
    // forward pass with zero carry; G = product of the forward coefficients
    C f = 0, G = 1;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        if (k < cnt) {
            const int64_t i = i0 + k;
            const C b = invd[i * S + s];
            if (!TR) {
                f = b * (v[k] + r * f);
                G *= r * b;
            } else {
                const C a = i > 0 ? r * invd[(i - 1) * S + s] : (C)0;
                f = v[k] + a * f;
                G *= a;
            }
            v[k] = f;
        }
    }
    if (writer) {
        sF[seg * nl + line] = f;
        sG[seg * nl + line] = G;
    }
    __syncthreads();
    C carry = 0;
    for (int j = 0; j < seg; ++j) carry = sF[j * nl + line] + sG[j * nl + line] * carry;
    // forward correction: t_i = f_i + (prod of coefficients up to i) * carry
    C c = carry;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        if (k < cnt) {
            const int64_t i = i0 + k;
            const C a = !TR ? r * invd[i * S + s] : (i > 0 ? r * invd[(i - 1) * S + s] : (C)0);
            c = a * c;
            v[k] += c;
        }
    }
    __syncthreads();   // all forward carries read before the arrays are reused
    // backward pass with zero carry; GB = product of alpha over the segment
    C bw = 0, GB = 1;
#pragma unroll
    for (int k = M - 1; k >= 0; --k) {
        if (k < cnt) {
            const int64_t i = i0 + k;
            const C b = invd[i * S + s];
            const C a = r * b;
            if (!TR)
                bw = v[k] + a * bw;
            else
                bw = b * (v[k] + r * bw);
            GB *= a;
            v[k] = bw;
        }
    }
    if (writer) {
        sF[seg * nl + line] = bw;
        sG[seg * nl + line] = GB;
    }
    __syncthreads();
    C X = 0;
    for (int j = K - 1; j > seg; --j) X = sF[j * nl + line] + sG[j * nl + line] * X;
    C e = X;
#pragma unroll
    for (int k = M - 1; k >= 0; --k) {
        if (k < cnt) {
            const int64_t i = i0 + k;
            e = r * invd[i * S + s] * e;
            v[k] += e;
        }
    }
}

// --------------------------------------------------- kind 1 (strided, y / z)
//
// Block = lpw neighbouring lines x K segments; blockDim = K * lpw.  Lane l of
// wave w handles line (l % lpw) and segment (w * (64/lpw) + l / lpw), so a
// wave's load of element k touches 64/lpw runs of lpw consecutive elements.
// blockIdx.x: line tile, blockIdx.y: outer index.

template <typename T, typename C, int M, bool TR>
__global__ __launch_bounds__(1024) void k_sweep_seg_strided(const T* in, T* out, AxisGeom g,
                                                            const C* __restrict__ invd,
                                                            const C* __restrict__ rr, int lpw)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int K = blockDim.x / lpw;
    C* sF = reinterpret_cast<C*>(smem);
    C* sG = sF + K * lpw;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int line = lane % lpw;
    const int seg = wave * (64 / lpw) + lane / lpw;
    const int64_t p = (int64_t)blockIdx.x * lpw + line;
    const bool valid = p < g.inner;
    const int S = g.S;
    const int s = valid ? (int)(p % S) : 0;
    const int64_t i0 = (int64_t)seg * M;
    const int64_t rem = g.n - i0;
    const int cnt = (valid && rem > 0) ? (rem < M ? (int)rem : M) : 0;
    const int64_t st = g.stride;
    const int64_t base = (int64_t)blockIdx.y * g.outer_stride + p + i0 * st;
    const C r = rr[s];
    C v[M];
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = k < cnt ? (C)in[base + k * st] : (C)0;
    solve_segment<C, M, TR>(v, cnt, i0, seg, K, line, lpw, s, S, r, invd, sF, sG, true);
#pragma unroll
    for (int k = 0; k < M; ++k)
        if (k < cnt) out[base + k * st] = (T)v[k];
}

// ------------------------------------------------------- kind 2 (x, LDS tile)
//
// Block = R rows (one row = the nx*S contiguous elements of one (y, z)).
// The rows are loaded into LDS with coalesced accesses in a padded layout:
// element (i, s) of row r sits at r*RS + (i/M)*SB + (i%M)*S + s, with
// SB = M*S + pad chosen so that the lanes of a wave (s fastest, then
// segment) hit distinct banks.  Thread t = (r*K + j)*S + s solves segment j
// of line (r, s) from registers, writes it back, and the block stores the
// rows with coalesced accesses.

struct FastDiv {   // q / d for q < 2^24, d < 2^16: (q * m) >> 40
    uint64_t m;
    __host__ __device__ FastDiv() : m(1) {}
    __host__ __device__ explicit FastDiv(uint32_t d) : m(((1ull << 40) + d - 1) / d) {}
    __device__ __forceinline__ uint32_t div(uint32_t q) const { return (uint32_t)(((uint64_t)q * m) >> 40); }
};

template <typename T, typename C, int M, bool TR>
__global__ __launch_bounds__(1024) void k_sweep_seg_xtile(const T* in, T* out, AxisGeom g,
                                                          const C* __restrict__ invd,
                                                          const C* __restrict__ rr, int R, int K,
                                                          int SB, uint32_t tile_bytes,
                                                          FastDiv divL, FastDiv divMS)
{
    extern __shared__ __align__(16) unsigned char smem[];
    T* tile = reinterpret_cast<T*>(smem);
    const int S = g.S;
    const int nl = R * S;
    C* sF = reinterpret_cast<C*>(smem + tile_bytes);
    C* sG = sF + K * nl;
    const uint32_t L = (uint32_t)(g.n * S);          // row length
    const uint32_t MS = (uint32_t)(M * S);
    const uint32_t RS = (uint32_t)(K * SB);           // tile row stride
    const int64_t o0 = (int64_t)blockIdx.x * R;
    const int nrows = (int)min((int64_t)R, g.outer - o0);
    const uint32_t tot = (uint32_t)nrows * L;
    const T* src = in + o0 * (int64_t)L;
    T* dst = out + o0 * (int64_t)L;

    for (uint32_t e = threadIdx.x; e < tot; e += blockDim.x) {
        const uint32_t rw = divL.div(e);
        const uint32_t q = e - rw * L;
        const uint32_t sg = divMS.div(q);
        tile[rw * RS + sg * SB + (q - sg * MS)] = src[e];
    }
    __syncthreads();

    const int t = threadIdx.x;
    const bool active = t < nl * K;
    const int s = t % S;
    const int j = (t / S) % K;
    const int rw = t / (S * K);
    const bool valid = active && rw < nrows;
    const int64_t i0 = (int64_t)j * M;
    const int64_t rem = g.n - i0;
    const int cnt = (valid && rem > 0) ? (rem < M ? (int)rem : M) : 0;
    const C r = rr[s];
    T* my = tile + rw * RS + j * SB + s;
    C v[M];
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = k < cnt ? (C)my[k * S] : (C)0;
    solve_segment<C, M, TR>(v, cnt, i0, j, K, active ? rw * S + s : 0, nl, s, S, r, invd, sF, sG,
                            active);
#pragma unroll
    for (int k = 0; k < M; ++k)
        if (k < cnt) my[k * S] = (T)v[k];
    __syncthreads();

    for (uint32_t e = threadIdx.x; e < tot; e += blockDim.x) {
        const uint32_t rw2 = divL.div(e);
        const uint32_t q = e - rw2 * L;
        const uint32_t sg = divMS.div(q);
        dst[e] = tile[rw2 * RS + sg * SB + (q - sg * MS)];
    }
}

// ---------------------------------------------------------------- planning

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

static const int kMaxLDS = 64 * 1024;

// padded segment block (elements of T) for the x tile
static int xtile_sb(int M, int S, int esize)
{
    const int words = esize == 8 ? 16 : 32;   // bank period in elements
    int pad = ((S - M * S) % words + words) % words;
    return M * S + pad;
}

static size_t xtile_lds(int M, int S, int R, int K, int esize, int csize, uint32_t* tile_bytes)
{
    size_t tb = (size_t)R * K * xtile_sb(M, S, esize) * esize;
    tb = (tb + 15) & ~(size_t)15;
    if (tile_bytes) *tile_bytes = (uint32_t)tb;
    return tb + 2 * (size_t)K * R * S * csize;
}

static int compute_size(int dtype) { return dtype == DT_F32_FAST ? 4 : 8; }

std::string check_plan(const SweepPlan& p, const AxisGeom& g, int dtype)
{
    const int es = (int)dtype_size(dtype), cs = compute_size(dtype);
    if (p.kind == PLAN_LINE) return "";
    if (p.m != 4 && p.m != 8 && p.m != 16 && p.m != 32) return "m must be 4, 8, 16 or 32";
    if (p.kind == PLAN_SEG_STRIDED) {
        if (p.lpw != 16 && p.lpw != 32 && p.lpw != 64) return "lpw must be 16, 32 or 64";
        if (p.w < 1 || p.w > 16) return "w must be in [1, 16]";
        if (g.outer > 65535) return "too many outer blocks for the strided kernel";
        const int64_t K = (int64_t)p.w * 64 / p.lpw;
        if (K * p.m < g.n) return "too few segments for the line length";
        if (2 * K * p.lpw * cs > kMaxLDS) return "LDS too large";
        return "";
    }
    if (p.kind == PLAN_SEG_XTILE) {
        if (g.inner != g.S) return "the LDS tile kernel only runs the x axis";
        const int64_t K = ceil_div(g.n, p.m);
        if (p.lpw < 1) return "rows per block must be >= 1";
        const int64_t threads = K * g.S * p.lpw;
        if (threads > 1024) return "more than 1024 threads per block";
        if ((int64_t)p.w * 64 < threads) return "w too small for the rows";
        if (p.w > 16) return "w must be <= 16";
        // FastDiv is exact while (index < 2^24) and index * divisor <= 2^40
        const int64_t L = g.n * g.S, tot = L * p.lpw;
        if (tot >= (1 << 24) || tot * L > (1ll << 40)) return "tile too long";
        if (xtile_lds(p.m, g.S, p.lpw, (int)K, es, cs, nullptr) > (size_t)kMaxLDS) return "LDS too large";
        return "";
    }
    return "unknown plan kind";
}

SweepPlan default_plan(int axis, const AxisGeom& g, int dtype)
{
    SweepPlan p;
    const int es = (int)dtype_size(dtype);
    if (axis == 0) {
        const int big[] = {16, 8, 32, 4}, mid[] = {8, 4, 16, 32}, small[] = {4, 8, 16, 32};
        const int* ms = g.n >= 512 ? big : (g.n >= 64 ? mid : small);
        for (int mi = 0; mi < 4; ++mi) {
            const int M = ms[mi];
            const int64_t K = ceil_div(g.n, M);
            const int64_t per_row = K * g.S;
            if (per_row > 1024) continue;
            int64_t R = std::max<int64_t>(1, 256 / per_row);
            R = std::min<int64_t>(R, g.outer);
            SweepPlan c;
            c.kind = PLAN_SEG_XTILE;
            c.m = M;
            c.lpw = (int)R;
            c.w = (int)ceil_div(R * per_row, 64);
            while (c.lpw > 1 && !check_plan(c, g, dtype).empty()) {
                c.lpw /= 2;
                c.w = (int)ceil_div((int64_t)c.lpw * per_row, 64);
            }
            if (check_plan(c, g, dtype).empty()) return c;
        }
        return p;   // kind 0
    }
    const int lpw = es == 8 ? 16 : 32;
    const int spw = 64 / lpw;
    const int ms[] = {16, 8, 32, 4};
    for (int M : ms) {
        if (M == 16 && g.n < 128) continue;
        int64_t K = ceil_div(g.n, M);
        K = ceil_div(K, spw) * spw;
        SweepPlan c;
        c.kind = PLAN_SEG_STRIDED;
        c.m = M;
        c.lpw = lpw;
        c.w = (int)(K * lpw / 64);
        if (check_plan(c, g, dtype).empty()) return c;
    }
    return p;
}

// --------------------------------------------------------------- launching

template <typename T, typename C, bool TR, int M>
static hipError_t launch_seg(const SweepPlan& p, const AxisGeom& g, const T* in, T* out,
                             const C* invd, const C* r, hipStream_t st)
{
    if (p.kind == PLAN_SEG_STRIDED) {
        const int threads = p.w * 64;
        const int K = threads / p.lpw;
        dim3 grid((unsigned)ceil_div(g.inner, p.lpw), (unsigned)g.outer);
        size_t lds = 2 * (size_t)K * p.lpw * sizeof(C);
        hipLaunchKernelGGL((k_sweep_seg_strided<T, C, M, TR>), grid, dim3(threads), lds, st, in, out,
                           g, invd, r, p.lpw);
    } else {
        const int K = (int)ceil_div(g.n, M);
        const int SB = xtile_sb(M, g.S, (int)sizeof(T));
        uint32_t tile_bytes = 0;
        size_t lds = xtile_lds(M, g.S, p.lpw, K, (int)sizeof(T), (int)sizeof(C), &tile_bytes);
        dim3 grid((unsigned)ceil_div(g.outer, p.lpw));
        hipLaunchKernelGGL((k_sweep_seg_xtile<T, C, M, TR>), grid, dim3(p.w * 64), lds, st, in, out,
                           g, invd, r, p.lpw, K, SB, tile_bytes, FastDiv((uint32_t)(g.n * g.S)),
                           FastDiv((uint32_t)(M * g.S)));
    }
    return hipGetLastError();
}

template <typename T, typename C, bool TR>
static hipError_t launch_typed(const SweepPlan& p, const AxisGeom& g, const void* in, void* out,
                               const void* invd, const void* r, hipStream_t st)
{
    const T* i = static_cast<const T*>(in);
    T* o = static_cast<T*>(out);
    const C* cf = static_cast<const C*>(invd);
    const C* rr = static_cast<const C*>(r);
    if (p.kind == PLAN_LINE) {
        const int64_t lines = g.inner * g.outer;
        hipLaunchKernelGGL((k_sweep_line<T, C, TR>), dim3((unsigned)ceil_div(lines, 256)), dim3(256), 0,
                           st, i, o, g, cf, rr);
        return hipGetLastError();
    }
    switch (p.m) {
        case 4: return launch_seg<T, C, TR, 4>(p, g, i, o, cf, rr, st);
        case 8: return launch_seg<T, C, TR, 8>(p, g, i, o, cf, rr, st);
        case 16: return launch_seg<T, C, TR, 16>(p, g, i, o, cf, rr, st);
        case 32: return launch_seg<T, C, TR, 32>(p, g, i, o, cf, rr, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep(int dtype, bool transposed, const SweepPlan& plan, const AxisGeom& g,
                        const void* in, void* out, const void* invd, const void* r, hipStream_t st)
{
    if (g.inner * g.outer == 0) return hipSuccess;
    switch (dtype) {
        case DT_F64:
            return transposed ? launch_typed<double, double, true>(plan, g, in, out, invd, r, st)
                              : launch_typed<double, double, false>(plan, g, in, out, invd, r, st);
        case DT_F32:
            return transposed ? launch_typed<float, double, true>(plan, g, in, out, invd, r, st)
                              : launch_typed<float, double, false>(plan, g, in, out, invd, r, st);
        case DT_F32_FAST:
            return transposed ? launch_typed<float, float, true>(plan, g, in, out, invd, r, st)
                              : launch_typed<float, float, false>(plan, g, in, out, invd, r, st);
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace bfvm
