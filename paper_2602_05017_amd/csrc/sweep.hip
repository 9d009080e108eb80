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
#include "seg_solver.hpp"

#include <algorithm>

namespace bfvm {

AxisGeom axis_geom(int axis, int64_t nx, int64_t ny, int64_t nz, int32_t S)
{
    AxisGeom g;
    g.S = S;
    g.axis = axis;
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

AxisGeom slab_geom(int axis, int64_t nx, int64_t ny, int64_t nz, int32_t S, int64_t x0, int64_t x1)
{
    AxisGeom g;
    g.S = S;
    g.axis = axis;
    g.inner = (x1 - x0) * S;
    g.p0 = x0 * S;
    if (axis == 1) {   // lines (z, x in slab, s) along y
        g.n = ny; g.outer = nz; g.stride = nx * S; g.outer_stride = ny * nx * S;
    } else {           // lines (y, x in slab, s) along z
        g.n = nz; g.outer = ny; g.stride = ny * nx * S; g.outer_stride = nx * S;
    }
    return g;
}

AxisGeom zslab_geom(int axis, int64_t nx, int64_t ny, int64_t nz, int32_t S, int64_t z0, int64_t z1)
{
    AxisGeom g = axis_geom(axis, nx, ny, z1 - z0, S);
    g.axis = axis;
    if (axis == 0)      // rows (z, y) of the slab: lines start after z0*ny rows
        g.p0 = z0 * ny * S;
    else                // y lines of planes z0 .. z1-1
        g.o0 = z0;
    return g;
}

// ------------------------------------------------------------ kind 0 (line)

// RED (transposed sweeps only): then sum y (L_N xf) and y xf along the
// line, written to part[2 L] with L the thread's line index.
template <typename T, typename C, bool TR, bool RED>
__global__ __launch_bounds__(256) void k_sweep_line(const T* in, T* out, AxisGeom g,
                                                    const C* __restrict__ invd,
                                                    const C* __restrict__ rr,
                                                    const T* __restrict__ xf, double* __restrict__ part)
{
    const int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= g.inner * g.outer) return;
    const int64_t o = L / g.inner;
    const int64_t p = g.p0 + (L - o * g.inner);
    const int S = g.S;
    const int s = (int)(p % S);
    const int64_t base = (g.o0 + o) * g.outer_stride + p;
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
        if constexpr (RED) {
            double a0 = 0.0, a1 = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                const double xc = (double)xf[base + i * st];
                double lx = 0.0;
                if (i > 0) lx += xc - (double)xf[base + (i - 1) * st];
                if (i < n - 1) lx += xc - (double)xf[base + (i + 1) * st];
                const double yi = (double)out[base + i * st];
                a0 += yi * lx;
                a1 += yi * xc;
            }
            part[2 * L + 0] = a0;
            part[2 * L + 1] = a1;
        }
    }
}

// --------------------------------------------------- kind 1 (strided, y / z)
//
// Block = lpw neighbouring lines x K segments; blockDim = K * lpw.  Lane l of
// wave w handles line (l % lpw) and segment (w * (64/lpw) + l / lpw), so a
// wave's load of element k touches 64/lpw runs of lpw consecutive elements.
// Grid: (line tiles, outer index), visited in the XCD-aware order of xcd_tile.

// Copy the [n][S] coefficient table into LDS for K*M slots in [s][seg][k]
// layout: slot (i, s) at s*SP + (i/M)*MP + i%M, with MP = M + 1 and SP chosen
// by the host so that the (substrate, segment) pairs of a wave fall in
// distinct banks; slots i >= n get 0.  A thread's M coefficients are then
// contiguous and read with immediate offsets.
template <typename C, int M>
__device__ __forceinline__ void stage_table(C* tab, const C* __restrict__ invd, uint32_t n, uint32_t KM,
                                            uint32_t S, uint32_t SP, FastDiv divS)
{
    constexpr int UNR = 8;
    const uint32_t tot = KM * S;
    const uint32_t nS = n * S;
    for (uint32_t e0 = threadIdx.x; e0 < tot; e0 += UNR * blockDim.x) {
        C buf[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const uint32_t e = e0 + u * blockDim.x;
            buf[u] = e < nS ? invd[e] : (C)0;
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const uint32_t e = e0 + u * blockDim.x;
            if (e < tot) {
                const uint32_t i = divS.div(e);
                const uint32_t sub = e - i * S;
                tab[sub * SP + (i / M) * (M + 1) + (i % M)] = buf[u];
            }
        }
    }
}

// Rows of M + 1 slots per substrate built in LDS from the exact compressed
// table comp ([s][H + 2]: head slots, interior constant, last slot): the nh
// segments that overlap the head, one row of the interior constant (shared
// by every other segment before the last slot's), the segment holding slot
// n - 1, and a zero row for segments past the line end (left out where no
// segment lies past it: zero = false).  Every thread of the block takes
// part; the caller synchronises before use.
template <int M>
struct CompRows {
    int nh, tseg, SPr;
    __device__ __forceinline__ CompRows(int H, int n, bool zero = true)
        : nh((H + M - 1) / M), tseg((n - 1) / M), SPr((nh + 2 + (zero ? 1 : 0)) * (M + 1)) {}
    __device__ __forceinline__ int row(int seg) const
    {
        return seg < nh ? seg : (seg == tseg ? nh + 1 : (seg > tseg ? nh + 2 : nh));
    }
};

template <typename C, int M>
__device__ __forceinline__ void build_comp_rows(C* tab, const C* __restrict__ comp, int H, int n, int S,
                                                const CompRows<M>& cr)
{
    constexpr int RW = M + 1;
    const int nm1 = n - 1;
    for (int e = threadIdx.x; e < S * cr.SPr; e += blockDim.x) {
        const int ss = e / cr.SPr, q = e - ss * cr.SPr, row = q / RW, k = q - row * RW;
        const C* cp = comp + ss * (H + 2);
        const int i = row < cr.nh ? row * M + k : cr.tseg * M + k;
        C val = (C)0;
        if (k < M && row != cr.nh + 2) {
            if (row == cr.nh) val = cp[H];
            else val = i < H ? cp[i] : (i < nm1 ? cp[H] : (i == nm1 ? cp[H + 1] : (C)0));
        }
        tab[e] = val;
    }
}

// AX (0, 1, 2) only names the axis in the kernel symbol, so that profiles
// report the x, y and z sweeps separately.
// COEF: where the Thomas constants come from: 0 the global [n][S] table,
// 1 its LDS copy in [s][segment][k] layout, 2 rows built in LDS from the
// exact compressed table comp ([s][H + 2]: head, interior constant, last
// slot), so that a segment inside the constant interior needs no table.
// RED (transposed sweeps only): also form the reverse step's per-line sums
// from y and the forward sweep's output xf (seg_adjoint_sums), written to
// part[2 L], L = by * inner + p.
template <typename T, typename C, int M, bool TR, int COEF, bool XROWS, int AX, bool RED>
__global__ __launch_bounds__(1024) void k_sweep_seg_strided(const T* in, T* out, AxisGeom g,
                                                            const C* __restrict__ invd,
                                                            const C* __restrict__ rr, int lpw, int SP,
                                                            FastDiv divS, const C* __restrict__ comp, int H,
                                                            const T* __restrict__ xf, double* __restrict__ part)
{
    uint32_t bx, by;
    xcd_tile(bx, by);
    extern __shared__ __align__(16) unsigned char smem[];
    const int K = blockDim.x / lpw;
    C* sc = reinterpret_cast<C*>(smem);
    C* tab = sc + 4 * scan_slots(K, lpw, (int)blockDim.x, false);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int line = lane % lpw;
    const int seg = wave * (64 / lpw) + lane / lpw;
    const int64_t p = (int64_t)bx * lpw + line;
    const bool valid = p < g.inner;
    const int64_t pa = valid ? p : g.inner - 1;          // clamped line for padding loads
    const int S = g.S;
    const int s = (int)((g.p0 + pa) % S);
    const int64_t i0 = (int64_t)seg * M;
    const int64_t last = g.n - 1 - i0;                    // slots k > last are padding
    const int cnt = !valid || last < 0 ? 0 : (last >= M ? M : (int)last + 1);
    const int64_t st = g.stride;
    // XROWS: the x axis run through this kernel; line pa is substrate pa % S of
    // row pa / S, whose elements are S apart inside the row's n*S run
    const int64_t line0 = XROWS ? ((g.p0 + pa) / S) * (g.n * S) + (pa % S)
                                : (g.o0 + (int64_t)by) * g.outer_stride + g.p0 + pa;
    const int64_t base = line0 + i0 * st;
    C v[M];
    // FP64 z lines (a 32 MB stride on 1000^3 x 4) stream through once per
    // sweep: loads and stores carry the non-temporal hint.  Measured on that
    // grid: z 3% faster; y 4% slower, FP32 and the x rows (whose loads reuse
    // cache lines across k) slower, so only this case uses it.
    constexpr bool NT = sizeof(T) == 8 && AX == 2;
    // z tiles run at a raised wave priority, highest while they issue their
    // loads, one lower through the solve and back to the lowest for the
    // stores, so that a wave loading its tile is not held behind the other
    // block's solve.  1000^3 x 4: FP64 z 12.80 -> 12.56 ms with the loads
    // alone raised, 12.43-12.46 ms so; FP32 storage z 7.89 -> 7.69 ms, FP32
    // arithmetic 6.97 -> 6.73 ms (1-3% slower with the loads alone raised).
    // Raised through the stores as well, FP64 z took 14.1 ms.  y with FP32
    // arithmetic (32-line tiles) gains too: 5.65-5.75 -> 5.32-5.48 ms; FP64 y
    // and x lost 1-2.5%, FP32-storage y in 16-line tiles 10%.
    constexpr bool PRI = AX == 2 || (AX == 1 && sizeof(C) == 4);
    if constexpr (PRI) __builtin_amdgcn_s_setprio(2);
    if (NT) {
#pragma unroll
        for (int k = 0; k < M; ++k) v[k] = (C)__builtin_nontemporal_load(&in[base + (k <= last ? k : last) * st]);
    } else {
#pragma unroll
        for (int k = 0; k < M; ++k) v[k] = (C)in[base + (k <= last ? k : last) * st];
    }
    if constexpr (PRI) __builtin_amdgcn_s_setprio(1);
    const C r = rr[s];
    const C prev = (TR && i0 > 0 && last >= 0) ? invd[(i0 - 1) * S + s] : (C)0;
    if (COEF == 1) {
        stage_table<C, M>(tab, invd, (uint32_t)g.n, (uint32_t)(K * M), (uint32_t)S, (uint32_t)SP, divS);
        __syncthreads();
        LdsCoef<C> coef{tab + s * SP + seg * (M + 1), prev};
        solve_segment<C, M, TR, false>(v, seg, K, line, lpw, r, coef, sc, true);
    } else if (COEF == 2) {
        const CompRows<M> cr(H, (int)g.n);
        build_comp_rows<C, M>(tab, comp, H, (int)g.n, S, cr);
        __syncthreads();
        LdsCoef<C> coef{tab + s * cr.SPr + cr.row(seg) * (M + 1), prev};
        solve_segment<C, M, TR, false>(v, seg, K, line, lpw, r, coef, sc, true);
    } else {
        GlobalCoef<C> coef{invd + (last >= 0 ? i0 * S + s : s), S, (int)(last < M ? last : M), prev};
        solve_segment<C, M, TR, false>(v, seg, K, line, lpw, r, coef, sc, true);
    }
    // An opaque store pointer makes the compiler recompute the M addresses
    // here instead of keeping the load addresses live through the solve.
    T* op = out + base;
    asm volatile("" : "+v"(op));
    if constexpr (PRI) __builtin_amdgcn_s_setprio(0);
    if (NT) {
        if (cnt == M) {
#pragma unroll
            for (int k = 0; k < M; ++k) __builtin_nontemporal_store((T)v[k], &op[k * st]);
        } else {
#pragma unroll
            for (int k = 0; k < M; ++k)
                if (k < cnt) __builtin_nontemporal_store((T)v[k], &op[k * st]);
        }
    } else if (cnt == M) {
#pragma unroll
        for (int k = 0; k < M; ++k) op[k * st] = (T)v[k];
    } else {
#pragma unroll
        for (int k = 0; k < M; ++k)
            if (k < cnt) op[k * st] = (T)v[k];
    }
    if constexpr (RED) {
        double a0 = 0.0, a1 = 0.0;
        if (cnt > 0) seg_adjoint_sums<C, M, NT>(v, xf + base, st, (int)last, i0 > 0, a0, a1);
        const int64_t p_first = (int64_t)bx * lpw;
        line_sums_store<C>(a0, a1, seg, K, line, lpw, sc, false, true, part,
                           (int64_t)by * g.inner + p_first, (int)min((int64_t)lpw, g.inner - p_first));
    }
}

// A segment's cnt real values to p[k * st].  The opaque pointer makes the
// compiler form the M addresses here instead of keeping the load addresses
// live through the solve; it stays a global pointer, so the stores are
// global stores, counted by the memory counter only (a flat store would
// also hold up every later wait for LDS accesses).
template <typename T, typename C, int M>
__device__ __forceinline__ void store_seg(const C (&v)[M], T* gp, int64_t st, int cnt)
{
    auto p = (__attribute__((address_space(1))) T*)gp;
    asm volatile("" : "+v"(p));
    if (cnt == M) {
#pragma unroll
        for (int k = 0; k < M; ++k) p[k * st] = (T)v[k];
    } else {
#pragma unroll
        for (int k = 0; k < M; ++k)
            if (k < cnt) p[k * st] = (T)v[k];
    }
}

// ------------------------------- reverse step: z recomputation + z transposed
//
// The z axis of the reverse step in one pass.  The reverse step needs the
// forward z sweep's output x (before the step's last Dirichlet overwrite)
// only for the parameter sums of the transposed z sweep, which runs first.
// Here each block recomputes x for its tile in registers (the forward solve
// of zin, the y sweep's output with the Dirichlet values applied), then
// solves the transposed system on the gradient in place, and forms the
// sums y.(L_N x) and y.x from the two register arrays: x is never written
// to memory or read back, so the reverse step moves 13 element values per
// voxel-substrate instead of 15.  x enters the sums rounded to the storage
// type, the value the two-kernel form reads back from its workspace; the
// x values next to a segment come from the neighbouring segments through
// LDS.  Tiles as kind 1 (lanes over neighbouring lines, waves over
// segments), with M values of x and M of y per thread; COEF 1 (LDS copy of
// the table) or 2 (compressed rows).
//
// DMA: the block's gradient tile ([n planes][lpw lines] of T, from byte gb_off
// of the block's LDS) is fetched straight into LDS with 16-byte global-to-LDS
// loads issued before the forward solve, so the gradient is in flight while x
// is recomputed instead of being requested after it; the solves then use two
// carry arrays instead of four, and the x end values and the sums go through
// the tile's space once it has been read.  Needs 16-byte aligned rows and
// lines that fill whole 16-byte chunks (checked by the launcher).
template <typename T, typename C, int M, int COEF, int UNR, bool DMA>
__global__ __launch_bounds__(512, 4) void k_adj_z_fused(const T* zin, T* grad, AxisGeom g,
                                                        const C* __restrict__ invd, const C* __restrict__ rr,
                                                        int lpw, int SP, FastDiv divS, const C* __restrict__ comp,
                                                        int H, double* __restrict__ part, int gb_off)
{
    uint32_t bx, by;
    xcd_tile(bx, by);
    extern __shared__ __align__(16) unsigned char smem[];
    const int K = blockDim.x / lpw;
    C* sc = reinterpret_cast<C*>(smem);
    C* tab = sc + (DMA ? 2 : 4) * scan_slots(K, lpw, (int)blockDim.x, false);
    T* gb = reinterpret_cast<T*>(smem + gb_off);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int line = lane % lpw;
    const int seg = wave * (64 / lpw) + lane / lpw;
    const int64_t p = (int64_t)bx * lpw + line;
    const bool valid = p < g.inner;
    const int64_t pa = valid ? p : g.inner - 1;   // clamped line for padding loads
    const int S = g.S;
    const int s = (int)((g.p0 + pa) % S);
    const int64_t i0 = (int64_t)seg * M;
    const int64_t last = g.n - 1 - i0;            // slots k > last are padding
    const int cnt = !valid || last < 0 ? 0 : (last >= M ? M : (int)last + 1);
    const int64_t st = g.stride;
    const int64_t base = (g.o0 + (int64_t)by) * g.outer_stride + g.p0 + pa + i0 * st;
    const C r = rr[s];
    const C prev = (i0 > 0 && last >= 0) ? invd[(i0 - 1) * S + s] : (C)0;
    const int64_t p_first = (int64_t)bx * lpw;
    C x[M], y[M];
#pragma unroll
    for (int k = 0; k < M; ++k) x[k] = (C)zin[base + (k <= last ? k : last) * st];
    // the leader scans load UNR segments' terms ahead (not 8): the x values
    // stay live through the second solve
    auto solve_both = [&](const auto& coef) {
        using Cf = std::decay_t<decltype(coef)>;
        if constexpr (DMA) {
            // the x values first (the compiler's own wait before their use
            // would otherwise count the tile's loads too)
            wait_vm();
            fetch_tile_lds<T, M>(gb, grad + (g.o0 + (int64_t)by) * g.outer_stride + g.p0 + p_first,
                              [](int l) { return (int64_t)l; }, st, (int)g.n, lpw, g.inner - p_first);
        }
        solve_segment<C, M, false, false, Cf, UNR, DMA>(x, seg, K, line, lpw, r, coef, sc, true);
        int lastv = (int)(last < M ? last : M);
        if constexpr (DMA) {
            // this wave's chunks have landed once its memory counter is 0,
            // every wave's after the barrier
            wait_vm();
            __syncthreads();
            const T* gr = gb + (int)(pa - p_first);
#pragma unroll
            for (int k = 0; k < M; ++k) y[k] = (C)gr[((int)i0 + (k <= lastv ? k : lastv)) * lpw];
        } else {
            // opaque pointer and bound: the gradient's addresses are formed
            // here instead of being kept live through the first solve
            const T* gp = grad + base;
            asm volatile("" : "+v"(gp), "+v"(lastv));
#pragma unroll
            for (int k = 0; k < M; ++k) y[k] = (C)gp[(k <= lastv ? k : lastv) * st];
        }
        solve_segment<C, M, true, false, Cf, UNR, DMA>(y, seg, K, line, lpw, r, coef, sc, true);
    };
    if constexpr (COEF == 1) {
        stage_table<C, M>(tab, invd, (uint32_t)g.n, (uint32_t)(K * M), (uint32_t)S, (uint32_t)SP, divS);
        __syncthreads();
        solve_both(LdsCoef<C>{tab + s * SP + seg * (M + 1), prev});
    } else {
        const CompRows<M> cr(H, (int)g.n);
        build_comp_rows<C, M>(tab, comp, H, (int)g.n, S, cr);
        __syncthreads();
        solve_both(LdsCoef<C>{tab + s * cr.SPr + cr.row(seg) * (M + 1), prev});
    }
    // stored before the sums (after them, with x and y both live through the
    // exchange, the kernel spills 17-19 VGPRs); the barriers below order LDS
    // only, so the stores stay in flight through them
    store_seg<T, C, M>(y, grad + base, st, cnt);
    // x at the segment's ends for the neighbouring segments (the carry
    // arrays hold at least two doubles per slot)
    const int slot = seg * lpw + line;
    C* sums = DMA ? reinterpret_cast<C*>(gb) : sc;   // room for two doubles per slot
    double* xfirst = reinterpret_cast<double*>(sums);
    double* xlast = xfirst + K * lpw;
    lds_sync();   // the solves' last reads of the carry arrays are done
    xfirst[slot] = (double)(T)x[0];
    xlast[slot] = (double)(T)x[M - 1];
    lds_sync();
    const bool left = i0 > 0 && last >= 0;
    double xl = left ? xlast[slot - lpw] : 0.0;
    double a0 = 0.0, a1 = 0.0;
    if (cnt > 0) {
        double xc = (double)(T)x[0];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const double xn = k + 1 < M ? (double)(T)x[k + 1] : (k + 1 <= last ? xfirst[slot + lpw] : 0.0);
            double lx = 0.0;
            if (k > 0 || left) lx += xc - xl;
            if (k + 1 <= last) lx += xc - xn;
            if (k <= last) {
                a0 += (double)y[k] * lx;
                a1 += (double)y[k] * xc;
            }
            xl = xc;
            xc = xn;
        }
    }
    line_sums_store<C, true>(a0, a1, seg, K, line, lpw, sums, false, true, part, (int64_t)by * g.inner + p_first,
                             (int)min((int64_t)lpw, g.inner - p_first));
}

// ------------------------- reverse step: transposed sweep, sums from an LDS tile
//
// The transposed sweep of y (or z) lines of up to 512 voxels with the
// reverse step's per-line sums y.(L_N x) and y.x, x being the forward
// output xf on the same lines (in the storage type).  The strided kernel
// reads x after its solve, so those loads start only when the solve ends;
// here the block fetches its x tile into LDS with global-to-LDS loads issued
// before the solve (fetch_tile_lds), in flight while it runs, and the sums
// read x and its neighbours from LDS.  Tiles as k_adj_z_fused: M = 16, K =
// the power of two >= n/16 (at least 8) segments, 512/K neighbouring lines,
// two blocks per CU; the solve's barriers order LDS only and its scans use
// two carry arrays; the sums go through the tile's space once it is read.
// XROWS: x lines (line L = substrate L % S of row L / S, its elements S
// apart in the row's n*S run; g.inner = rows * S, one outer index), the
// tile's lpw lines being lpw / S whole rows.
template <typename T, typename C, int M, int COEF, bool XROWS>
__global__ __launch_bounds__(512, 4) void k_adj_tr_tile(const T* in, T* out, AxisGeom g, const C* __restrict__ invd,
                                                        const C* __restrict__ rr, int lpw, int SP, FastDiv divS,
                                                        const C* __restrict__ comp, int H, const T* __restrict__ xf,
                                                        double* __restrict__ part, int gb_off)
{
    uint32_t bx, by;
    xcd_tile(bx, by);
    extern __shared__ __align__(16) unsigned char smem[];
    const int K = blockDim.x / lpw;
    C* sc = reinterpret_cast<C*>(smem);
    C* tab = sc + 2 * scan_slots(K, lpw, (int)blockDim.x, false);
    T* gb = reinterpret_cast<T*>(smem + gb_off);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int line = lane % lpw;
    const int seg = wave * (64 / lpw) + lane / lpw;
    const int64_t p = (int64_t)bx * lpw + line;
    const bool valid = p < g.inner;
    const int64_t pa = valid ? p : g.inner - 1;   // clamped line for padding loads
    const int S = g.S;
    const int s = (int)((g.p0 + pa) % S);
    const int64_t i0 = (int64_t)seg * M;
    const int64_t last = g.n - 1 - i0;            // slots k > last are padding
    const int cnt = !valid || last < 0 ? 0 : (last >= M ? M : (int)last + 1);
    const int64_t st = g.stride;
    const int64_t p_first = (int64_t)bx * lpw;
    const int64_t nS = g.n * S;
    // first element of the tile's first line, and of line pa
    const int64_t row0 = XROWS ? (int64_t)divS.div((uint32_t)p_first) * nS
                               : (g.o0 + (int64_t)by) * g.outer_stride + g.p0 + p_first;
    const int64_t base = (XROWS ? (int64_t)divS.div((uint32_t)pa) * nS + s : row0 + (pa - p_first)) + i0 * st;
    const C r = rr[s];
    const C prev = (i0 > 0 && last >= 0) ? invd[(i0 - 1) * S + s] : (C)0;
    C y[M];
#pragma unroll
    for (int k = 0; k < M; ++k) y[k] = (C)in[base + (k <= last ? k : last) * st];
    auto solve = [&](const auto& coef) {
        using Cf = std::decay_t<decltype(coef)>;
        wait_vm();   // the gradient values first, then the x tile in flight
        if constexpr (XROWS)
            fetch_tile_lds<T, M>(gb, xf + row0, [&](int l) {
                const int r = (int)divS.div((uint32_t)l);
                return (int64_t)r * nS + (l - r * S);
            }, st,
                              (int)g.n, lpw, g.inner - p_first);
        else
            fetch_tile_lds<T, M>(gb, xf + row0, [](int l) { return (int64_t)l; }, st, (int)g.n, lpw, g.inner - p_first);
        solve_segment<C, M, true, false, Cf, 8, true>(y, seg, K, line, lpw, r, coef, sc, true);
    };
    if constexpr (COEF == 1) {
        stage_table<C, M>(tab, invd, (uint32_t)g.n, (uint32_t)(K * M), (uint32_t)S, (uint32_t)SP, divS);
        __syncthreads();
        solve(LdsCoef<C>{tab + s * SP + seg * (M + 1), prev});
    } else {
        const CompRows<M> cr(H, (int)g.n);
        build_comp_rows<C, M>(tab, comp, H, (int)g.n, S, cr);
        __syncthreads();
        solve(LdsCoef<C>{tab + s * cr.SPr + cr.row(seg) * (M + 1), prev});
    }
    wait_vm();
    __syncthreads();   // every wave's part of the x tile has landed
    double a0 = 0.0, a1 = 0.0;
    if (cnt > 0) {
        const T* xr = gb + (int)(pa - p_first);
        const int ib = (int)i0, lst = (int)last;
        const bool left = ib > 0;
        double xl = left ? (double)xr[(ib - 1) * lpw] : 0.0;
        double xc = (double)xr[ib * lpw];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const double xn = k + 1 <= lst ? (double)xr[(ib + k + 1) * lpw] : 0.0;
            double lx = 0.0;
            if (k > 0 || left) lx += xc - xl;
            if (k + 1 <= lst) lx += xc - xn;
            if (k <= lst) {
                a0 += (double)y[k] * lx;
                a1 += (double)y[k] * xc;
            }
            xl = xc;
            xc = xn;
        }
    }
    line_sums_store<C>(a0, a1, seg, K, line, lpw, reinterpret_cast<C*>(gb), false, true, part,
                       (int64_t)by * g.inner + p_first, (int)min((int64_t)lpw, g.inner - p_first));
    // the stores last: the barriers above would otherwise wait for them
    store_seg<T, C, M>(y, out + base, st, cnt);
}

// ------------------------------------------ kind 5 (y/z, lines in two parts)
//
// For lines longer than one block's K = blockDim/lpw segments of M cover
// (K*M < n <= 2*K*M).  The block takes each line in two parts: a head of
// K0 = ceil(n/M) - K full segments (h0 = K0*M elements) and a tail of the
// other n - h0 <= K*M, cut into segments at the same positions as a kind-1
// block of K0 + K segments would cut the line.  Three passes:
//   A. head: load, keep a copy in LDS in the storage type, forward
//      elimination and forward carry scan; the carry leaving the head (the
//      eliminated value at h0 - 1) is kept per line;
//   B. tail: load, full solve with that carry entering its forward scan;
//      the backward carry leaving it (x at h0) is kept per line; store;
//   C. head again from its LDS copy: the same elimination and forward scan,
//      then the backward pass with the tail's carry entering it; store.
// Every element is read from and written to memory once; the head's
// forward elimination runs twice.  A 512-thread block of this kind leaves
// room for a second one on the CU, where the kind-1 block of 2K segments
// (1024 threads) holds a CU alone and the CU issues no loads while it
// scans.  In passes A and C the segments past the head are idle and pass
// every carry through unchanged (f = 0, G = 1; bw = 0, GB = 1), so the scans
// take the same steps, in the same order, as the kind-1 block's.  The
// backward carry terms reuse the forward carry arrays: a thread reads its
// own forward carry before it writes its own backward term.  The Thomas
// constants come from rows built in LDS from the exact compressed table (as
// in kind 1 with COEF = 2).  Two blocks per CU also need at most 128 VGPRs
// (4 waves per SIMD): the backward correction is fused with the stores
// (seg_last_store), which keeps the M = 32 FP64 form at 128 without spills.
// seg_last fused with the store: each value is stored (slots k < cnt) as
// soon as its backward correction is added, last slot first
template <typename T, typename C, int M, typename Coef>
__device__ __forceinline__ void seg_last_store(const C (&v)[M], C r, const Coef& coef, C X, T* op, int64_t st,
                                               int cnt)
{
    C e = X;
#pragma unroll
    for (int k = M - 1; k >= 0; --k) {
        e = r * coef(k) * e;
        if (k < cnt) op[k * st] = (T)(v[k] + e);
    }
}

// XROWS: the x axis, every (row, substrate) one line whose elements lie S
// apart inside the row's n*S run (as in kind 3); AX only names the axis.
template <typename T, typename C, int M, bool XROWS, int AX>
__global__ __launch_bounds__(512, 4) void k_sweep_seg_halves(const T* in, T* out, AxisGeom g,
                                                          const C* __restrict__ rr, int lpw, int K0,
                                                          const C* __restrict__ comp, int H)
{
    uint32_t bx, by;
    xcd_tile(bx, by);
    extern __shared__ __align__(16) unsigned char smem[];
    const int K = blockDim.x / lpw;
    const int A = K * lpw;
    C* sF = reinterpret_cast<C*>(smem);
    C* sG = sF + A;
    C* ini = sG + A;   // [line]: forward carry into the tail; [lpw + line]: backward carry into the head
    C* tab = ini + 2 * lpw;
    const int n = (int)g.n;
    // no segment lies past the last slot's: the tail ends with it
    const CompRows<M> cr(H, n, false);
    T* raw = reinterpret_cast<T*>(tab + g.S * cr.SPr);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int line = lane % lpw;
    const int seg = wave * (64 / lpw) + lane / lpw;
    const int slot = seg * lpw + line;
    const bool leader = (int)threadIdx.x < lpw;
    const int64_t p = (int64_t)bx * lpw + line;
    const bool valid = p < g.inner;
    const int64_t pa = valid ? p : g.inner - 1;   // clamped line for padding loads
    const int S = g.S;
    const int s = (int)((g.p0 + pa) % S);
    const int64_t st = g.stride;
    const int64_t line0 = XROWS ? ((g.p0 + pa) / S) * (g.n * S) + (pa % S)
                                : (g.o0 + (int64_t)by) * g.outer_stride + g.p0 + pa;
    const bool head = seg < K0;
    const C r = rr[s];
    build_comp_rows<C, M>(tab, comp, H, n, S, cr);
    // the coefficient row of global segment gs
    auto with_coef = [&](int gs, auto&& fn) {
        const LdsCoef<C> cf{tab + s * cr.SPr + cr.row(gs) * (M + 1), (C)0};
        fn(cf);
    };
    // LDS copy of the head: value k of segment seg in row seg*M + (k ^ (seg & 3))
    // of lpw values, so that the segments one wave holds use distinct banks
    auto raw_at = [&](int k) -> T& { return raw[(seg * M + (k ^ (seg & 3))) * lpw + line]; };
    C v[M];
    C f, G;
    // ---- A: head, forward elimination and scan
    if (head) {
        const T* ip = in + line0 + (int64_t)seg * M * st;
        T t[M];
#pragma unroll
        for (int k = 0; k < M; ++k) t[k] = ip[k * st];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            raw_at(k) = t[k];
            v[k] = (C)t[k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < M; ++k) v[k] = (C)0;
    }
    __syncthreads();   // the coefficient rows are built
    with_coef(seg, [&](const auto& cf) { seg_forward<C, M, false>(v, r, cf, f, G); });
    if (!head) {
        f = 0;
        G = 1;
    }
    sF[slot] = f;
    sG[slot] = G;
    __syncthreads();
    if (leader) carry_scan(sF, sG, K, lpw, (int)threadIdx.x, false, (C)0, ini);
    __syncthreads();
    // ---- B: tail, full solve
    {
        const int64_t i0 = (int64_t)K0 * M + (int64_t)seg * M;
        const int64_t last = g.n - 1 - i0;   // slots k > last are padding
        const int cnt = !valid || last < 0 ? 0 : (last >= M ? M : (int)last + 1);
        const int64_t base = line0 + i0 * st;
#pragma unroll
        for (int k = 0; k < M; ++k) v[k] = (C)in[base + (k <= last ? k : last) * st];
        with_coef(K0 + seg, [&](const auto& cf) {
            seg_forward<C, M, false>(v, r, cf, f, G);
            sF[slot] = f;
            sG[slot] = G;
            __syncthreads();
            if (leader) carry_scan(sF, sG, K, lpw, (int)threadIdx.x, false, ini[threadIdx.x]);
            __syncthreads();
            const C carry = sF[slot];
            C bw, GB;
            seg_middle<C, M, false>(v, r, cf, carry, bw, GB);
            sF[slot] = bw;
            sG[slot] = GB;
            __syncthreads();
            if (leader) carry_scan(sF, sG, K, lpw, (int)threadIdx.x, true, (C)0, ini + lpw);
            __syncthreads();
            T* op = out + base;
            asm volatile("" : "+v"(op));
            seg_last_store<T, C, M>(v, r, cf, sF[slot], op, st, cnt);
        });
    }
    // ---- C: head again from LDS, full solve with the tail's carry
    if (head) {
        // an opaque row pointer: the addresses are recomputed here rather
        // than kept live from pass A
        const T* rp = raw + seg * M * lpw + line;
        asm volatile("" : "+v"(rp));
#pragma unroll
        for (int k = 0; k < M; ++k) v[k] = (C)rp[(k ^ (seg & 3)) * lpw];
    } else {
#pragma unroll
        for (int k = 0; k < M; ++k) v[k] = (C)0;
    }
    with_coef(seg, [&](const auto& cf) {
        seg_forward<C, M, false>(v, r, cf, f, G);
        if (!head) {
            f = 0;
            G = 1;
        }
        __syncthreads();   // every thread has read its backward carry of pass B
        sF[slot] = f;
        sG[slot] = G;
        __syncthreads();
        if (leader) carry_scan(sF, sG, K, lpw, (int)threadIdx.x, false);
        __syncthreads();
        const C carry = sF[slot];
        C bw, GB;
        seg_middle<C, M, false>(v, r, cf, carry, bw, GB);
        if (!head) {
            bw = 0;
            GB = 1;
        }
        sF[slot] = bw;
        sG[slot] = GB;
        __syncthreads();
        if (leader) carry_scan(sF, sG, K, lpw, (int)threadIdx.x, true, ini[lpw + threadIdx.x]);
        __syncthreads();
        T* op = out + line0 + (int64_t)seg * M * st;
        asm volatile("" : "+v"(op));
        seg_last_store<T, C, M>(v, r, cf, sF[slot], op, st, head && valid ? M : 0);
    });
}

// ------------------------------------------------------- kind 2 (x, LDS tile)
//
// Block = R rows (one row = the nx*S contiguous elements of one (y, z)).
// The rows are loaded into LDS with coalesced 16-byte accesses in a padded
// layout: element (i, s) of row r sits at r*RS + (i/M)*SB + (i%M)*S + s, with
// SB = M*S + pad chosen so that the lanes of a wave (s fastest, then
// segment) hit distinct banks.  Thread t = (r*K + j)*S + s solves segment j
// of line (r, s) from registers, writes it back, and the block stores the
// rows with coalesced accesses.

// Load `tot` elements of src (consecutive rows) into the padded LDS tile.
// Loads are issued UNR at a time per thread so that many are in flight before
// the first LDS write waits for its data; indices past the end are clamped so
// every load stays in bounds.
template <typename T, int M>
__device__ __forceinline__ void xtile_load_rows(T* tile, const T* src, uint32_t tot, uint32_t L, uint32_t MS,
                                                uint32_t RS, int SB, FastDiv divL, FastDiv divMS, bool vec)
{
    constexpr int UNR = 8;
    if (vec) {
        // 16-byte chunks: a chunk never straddles a segment block (M*S, SB and
        // L are multiples of the chunk) and both sides are 16-byte aligned
        using V = typename Vec16<T>::type;
        constexpr uint32_t VW = 16 / sizeof(T);
        const V* srcv = reinterpret_cast<const V*>(src);
        const uint32_t nch = tot / VW;
        for (uint32_t c0 = threadIdx.x; c0 < nch; c0 += UNR * blockDim.x) {
            V buf[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const uint32_t c = c0 + u * blockDim.x;
                buf[u] = srcv[c < nch ? c : 0];
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const uint32_t c = c0 + u * blockDim.x;
                if (c < nch) {
                    const uint32_t e = c * VW;
                    const uint32_t rw = divL.div(e);
                    const uint32_t q = e - rw * L;
                    const uint32_t sg = divMS.div(q);
                    *reinterpret_cast<V*>(tile + rw * RS + sg * SB + (q - sg * MS)) = buf[u];
                }
            }
        }
    } else {
        for (uint32_t e0 = threadIdx.x; e0 < tot; e0 += UNR * blockDim.x) {
            T buf[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const uint32_t e = e0 + u * blockDim.x;
                buf[u] = src[e < tot ? e : 0];
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const uint32_t e = e0 + u * blockDim.x;
                if (e < tot) {
                    const uint32_t rw = divL.div(e);
                    const uint32_t q = e - rw * L;
                    const uint32_t sg = divMS.div(q);
                    tile[rw * RS + sg * SB + (q - sg * MS)] = buf[u];
                }
            }
        }
    }
}

// RED (transposed sweeps only): after y has been stored, the forward sweep's
// output xf of the same rows is staged through the tile as well, and the
// reverse step's per-line sums are written to part[2 L], L = row * S + s.
template <typename T, typename C, int M, bool TR, bool RED>
__global__ __launch_bounds__(512) void k_sweep_seg_xtile(const T* in, T* out, AxisGeom g,
                                                         const C* __restrict__ invd,
                                                         const C* __restrict__ rr, int R, int K,
                                                         int SB, uint32_t tile_bytes,
                                                         FastDiv divL, FastDiv divMS, bool vec,
                                                         const T* __restrict__ xf, double* __restrict__ part)
{
    extern __shared__ __align__(16) unsigned char smem[];
    T* tile = reinterpret_cast<T*>(smem);
    const int S = g.S;
    const int nl = R * S;
    C* sc = reinterpret_cast<C*>(smem + tile_bytes);
    const uint32_t L = (uint32_t)(g.n * S);          // row length
    const uint32_t MS = (uint32_t)(M * S);
    const uint32_t RS = (uint32_t)(K * SB);           // tile row stride
    const int64_t o0 = (int64_t)blockIdx.x * R;
    const int nrows = (int)min((int64_t)R, g.outer - o0);
    const uint32_t tot = (uint32_t)nrows * L;
    const T* src = in + o0 * (int64_t)L;
    T* dst = out + o0 * (int64_t)L;

    xtile_load_rows<T, M>(tile, src, tot, L, MS, RS, SB, divL, divMS, vec);
    __syncthreads();

    const int t = threadIdx.x;
    const bool active = t < nl * K;
    const int s = t % S;
    const int j = (t / S) % K;
    const int rw = active ? t / (S * K) : 0;
    const bool valid = active && rw < nrows;
    const int64_t i0 = (int64_t)j * M;
    const int64_t last = g.n - 1 - i0;                // slots k > last are padding
    const int cnt = valid ? (last >= M ? M : (int)last + 1) : 0;
    const C r = rr[s];
    // padding slots read the segment's last real element (row 0 for threads
    // without a row), so every LDS read below is of initialised data
    const int rws = valid ? rw : 0;
    T* my = tile + rws * RS + j * SB + s;
    RegCoef<C, M> coef;
    coef.prev = (TR && i0 > 0) ? invd[(i0 - 1) * S + s] : (C)0;
    const C* cf = invd + i0 * S + s;
    C v[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        coef.b[k] = k <= last ? cf[(k <= last ? k : 0) * S] : (C)0;
        v[k] = (C)my[(k <= last ? k : last) * S];
    }
    solve_segment<C, M, TR, true>(v, j, K, active ? rw * S + s : 0, nl, r, coef, sc, active);
    asm volatile("" : "+v"(my));
    if (cnt == M) {
#pragma unroll
        for (int k = 0; k < M; ++k) my[k * S] = (T)v[k];
    } else {
#pragma unroll
        for (int k = 0; k < M; ++k)
            if (k < cnt) my[k * S] = (T)v[k];
    }
    __syncthreads();

    if (vec) {
        using V = typename Vec16<T>::type;
        constexpr uint32_t VW = 16 / sizeof(T);
        V* dstv = reinterpret_cast<V*>(dst);
        for (uint32_t c = threadIdx.x; c < tot / VW; c += blockDim.x) {
            const uint32_t e = c * VW;
            const uint32_t rw2 = divL.div(e);
            const uint32_t q = e - rw2 * L;
            const uint32_t sg = divMS.div(q);
            dstv[c] = *reinterpret_cast<const V*>(tile + rw2 * RS + sg * SB + (q - sg * MS));
        }
    } else {
        for (uint32_t e = threadIdx.x; e < tot; e += blockDim.x) {
            const uint32_t rw2 = divL.div(e);
            const uint32_t q = e - rw2 * L;
            const uint32_t sg = divMS.div(q);
            dst[e] = tile[rw2 * RS + sg * SB + (q - sg * MS)];
        }
    }
    if constexpr (RED) {
        __syncthreads();   // the stores above have read the tile
        xtile_load_rows<T, M>(tile, xf + o0 * (int64_t)L, tot, L, MS, RS, SB, divL, divMS, vec);
        __syncthreads();
        double a0 = 0.0, a1 = 0.0;
        if (cnt > 0) {
            // the segment's x values in the tile; x_{i0-1} is slot M-1 of segment j-1
            const T* xs = tile + rw * RS + j * SB + s;
            const T* xl = xs - SB + (M - 1) * S;
            double xm = i0 > 0 ? (double)*xl : 0.0;
            double xc = (double)xs[0];
#pragma unroll
            for (int k = 0; k < M; ++k) {
                // x_{i0+k+1}: slot k+1 of this segment, or slot 0 of segment j+1
                const T* nx = k + 1 < M ? xs + (k + 1) * S : xs + SB;
                const double xn = k + 1 <= last ? (double)*nx : 0.0;
                double lx = 0.0;
                if (k > 0 || i0 > 0) lx += xc - xm;
                if (k + 1 <= last) lx += xc - xn;
                if (k <= last) {
                    a0 += (double)v[k] * lx;
                    a1 += (double)v[k] * xc;
                }
                xm = xc;
                xc = xn;
            }
        }
        line_sums_store<C>(a0, a1, j, K, active ? rw * S + s : 0, nl, sc, true, active, part, o0 * S, nrows * S);
    }
}

// ------------------------------------- kind 4 (x, LDS tile, pipelined rows)
//
// The layout and per-thread work of kind 2, in a persistent loop: block b
// handles row tiles b, b + gridDim.x, ...  A thread's line and segment are
// the same in every tile, so its M coefficients are loaded once.  The next
// tile's rows are loaded into registers (P 16-byte chunks per thread) right
// after the current tile has been written to LDS, so those loads are in
// flight while the current tile is solved and stored.  Requires the 16-byte
// conditions of kind 2 and P * blockDim.x chunks >= R * nx * S / (16 / e).
template <typename T, typename C, int M, bool TR, int P>
__global__ __launch_bounds__(512) void k_sweep_seg_xpipe(const T* in, T* out, AxisGeom g,
                                                         const C* __restrict__ invd,
                                                         const C* __restrict__ rr, int R, int K,
                                                         int SB, uint32_t tile_bytes,
                                                         FastDiv divL, FastDiv divMS)
{
    // a native 16-byte vector type keeps the prefetch buffer in registers
    constexpr uint32_t VW = 16 / sizeof(T);
    typedef T V __attribute__((ext_vector_type(VW)));
    extern __shared__ __align__(16) unsigned char smem[];
    T* tile = reinterpret_cast<T*>(smem);
    const int S = g.S;
    const int nl = R * S;
    C* sc = reinterpret_cast<C*>(smem + tile_bytes);
    const uint32_t L = (uint32_t)(g.n * S);          // row length
    const uint32_t MS = (uint32_t)(M * S);
    const uint32_t RS = (uint32_t)(K * SB);           // tile row stride
    const int64_t ntiles = (g.outer + R - 1) / R;

    const int t = threadIdx.x;
    const bool active = t < nl * K;
    const int s = t % S;
    const int j = (t / S) % K;
    const int rw = active ? t / (S * K) : 0;
    const int64_t i0 = (int64_t)j * M;
    const int64_t last = g.n - 1 - i0;                // slots k > last are padding
    const C r = rr[s];
    RegCoef<C, M> coef;
    coef.prev = (TR && i0 > 0) ? invd[(i0 - 1) * S + s] : (C)0;
    const C* cf = invd + i0 * S + s;
#pragma unroll
    for (int k = 0; k < M; ++k) coef.b[k] = k <= last ? cf[(k <= last ? k : 0) * S] : (C)0;

    // Chunk slots past the tile's end load and store the tile's last chunk:
    // the duplicate LDS writes carry the same data as the owner's, and the
    // loop stays branch-free so the prefetch buffer stays in registers.
    // LDS offsets of the thread's P chunks in a full tile (the same in every
    // full tile; the last tile may be partial and recomputes them)
    const uint32_t nch_full = (uint32_t)R * L / VW;
    uint32_t offs[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
        const uint32_t c0 = t + u * blockDim.x;
        const uint32_t c = c0 < nch_full ? c0 : nch_full - 1;
        const uint32_t e = c * VW;
        const uint32_t rw2 = divL.div(e);
        const uint32_t q = e - rw2 * L;
        const uint32_t sg = divMS.div(q);
        offs[u] = rw2 * RS + sg * SB + (q - sg * MS);
    }
    V buf[P];
    int64_t ti = blockIdx.x;
    if (ti < ntiles) {
        const int64_t o0 = ti * R;
        const uint32_t nch = (uint32_t)min((int64_t)R, g.outer - o0) * L / VW;
        const V* srcv = reinterpret_cast<const V*>(in + o0 * (int64_t)L);
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const uint32_t c = t + u * blockDim.x;
            buf[u] = srcv[c < nch ? c : nch - 1];
        }
    }
    for (; ti < ntiles; ti += gridDim.x) {
        const int64_t o0 = ti * R;
        const int nrows = (int)min((int64_t)R, g.outer - o0);
        const uint32_t nch = (uint32_t)nrows * L / VW;
        const bool full = nrows == R;
        __syncthreads();   // the previous tile's stores have finished reading the LDS tile
        if (full) {
#pragma unroll
            for (int u = 0; u < P; ++u) *reinterpret_cast<V*>(tile + offs[u]) = buf[u];
        } else {
#pragma unroll
            for (int u = 0; u < P; ++u) {
                const uint32_t c0 = t + u * blockDim.x;
                const uint32_t c = c0 < nch ? c0 : nch - 1;
                const uint32_t e = c * VW;
                const uint32_t rw2 = divL.div(e);
                const uint32_t q = e - rw2 * L;
                const uint32_t sg = divMS.div(q);
                *reinterpret_cast<V*>(tile + rw2 * RS + sg * SB + (q - sg * MS)) = buf[u];
            }
        }
        __syncthreads();
        const int64_t tn = ti + gridDim.x;
        if (tn < ntiles) {   // next tile's rows: in flight during the solve below
            const int64_t on = tn * R;
            const uint32_t nchn = (uint32_t)min((int64_t)R, g.outer - on) * L / VW;
            const V* srcv = reinterpret_cast<const V*>(in + on * (int64_t)L);
#pragma unroll
            for (int u = 0; u < P; ++u) {
                const uint32_t c = t + u * blockDim.x;
                buf[u] = srcv[c < nchn ? c : nchn - 1];
            }
        }
        const bool valid = active && rw < nrows;
        const int cnt = valid ? (last >= M ? M : (int)last + 1) : 0;
        // padding slots read the segment's last real element (row 0 for
        // threads without a row), so every LDS read is of initialised data
        const int rws = valid ? rw : 0;
        T* my = tile + rws * RS + j * SB + s;
        C v[M];
#pragma unroll
        for (int k = 0; k < M; ++k) v[k] = (C)my[(k <= last ? k : last) * S];
        // LDS-only barriers in the solve: the next tile's loads above stay in
        // flight through it instead of being waited for at its first barrier
        // (1000^3 x 4 FP32 storage x 6.60 -> 6.50 ms)
        solve_segment<C, M, TR, true, RegCoef<C, M>, 8, true>(v, j, K, active ? rw * S + s : 0, nl, r, coef, sc,
                                                              active);
        if (cnt == M) {
#pragma unroll
            for (int k = 0; k < M; ++k) my[k * S] = (T)v[k];
        } else {
#pragma unroll
            for (int k = 0; k < M; ++k)
                if (k < cnt) my[k * S] = (T)v[k];
        }
        __syncthreads();
        V* dstv = reinterpret_cast<V*>(out + o0 * (int64_t)L);
        if (full) {
#pragma unroll
            for (int u = 0; u < P; ++u) {
                const uint32_t c = t + u * blockDim.x;
                if (c < nch) dstv[c] = *reinterpret_cast<const V*>(tile + offs[u]);
            }
        } else {
            for (uint32_t c = t; c < nch; c += blockDim.x) {
                const uint32_t e = c * VW;
                const uint32_t rw2 = divL.div(e);
                const uint32_t q = e - rw2 * L;
                const uint32_t sg = divMS.div(q);
                dstv[c] = *reinterpret_cast<const V*>(tile + rw2 * RS + sg * SB + (q - sg * MS));
            }
        }
    }
}

// ---------------------------------------------------------------- planning

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// LDS a workgroup may use: the current device's limit (160 KB per workgroup
// on gfx950), or 64 KB where it cannot be queried (no device).
static int64_t max_lds()
{
    static int64_t cached = -1;
    if (cached < 0) {
        int dev = 0, v = 0;
        cached = 64 * 1024;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > cached)
            cached = v;
    }
    return cached;
}

// padded segment block (elements of T) for the x tile
static int xtile_sb(int M, int S, int esize)
{
    const int words = esize == 8 ? 16 : 32;   // bank period in elements
    int pad = ((S - M * S) % words + words) % words;
    return M * S + pad;
}

static size_t xtile_lds(int M, int S, int R, int K, int esize, int csize, int threads, uint32_t* tile_bytes)
{
    size_t tb = (size_t)R * K * xtile_sb(M, S, esize) * esize;
    tb = (tb + 15) & ~(size_t)15;
    if (tile_bytes) *tile_bytes = (uint32_t)tb;
    return tb + 4 * (size_t)scan_slots(K, R * S, threads, true) * csize;
}

// 16-byte chunks each thread of a kind-4 block prefetches per row tile, and
// the compiled prefetch depth that covers it (0: none fits)
static int xpipe_need(const AxisGeom& g, int R, int threads, int es)
{
    const int64_t nch = (int64_t)R * g.n * g.S * es / 16;
    return (int)ceil_div(nch, threads);
}
static int xpipe_depth(int need) { return need <= 2 ? 2 : (need <= 4 ? 4 : (need <= 8 ? 8 : 0)); }

static int compute_size(int dtype) { return dtype == DT_F32_FAST ? 4 : 8; }

// LDS of a kind-5 block: two carry arrays of K*lpw and two per-line carries
// (compute type), the coefficient rows (ctab bytes) and the head's copy,
// K0*M rows of lpw values (storage type)
size_t halves_lds(int K, int lpw, int K0, int M, int es, int cs, size_t ctab)
{
    return (size_t)(2 * K * lpw + 2 * lpw) * cs + ctab + (size_t)K0 * M * lpw * es;
}

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
        if (4 * (int64_t)scan_slots((int)K, p.lpw, p.w * 64, false) * cs > max_lds()) return "LDS too large";
        return "";
    }
    if (p.kind == PLAN_SEG_HALVES) {
        if (p.lpw != 16 && p.lpw != 32 && p.lpw != 64) return "lpw must be 16, 32 or 64";
        if (p.w < 1 || p.w > 8) return "w must be in [1, 8]";
        if (g.axis == 0 && ceil_div(g.outer * g.S, p.lpw) >= (1ll << 31)) return "too many lines";
        if (g.axis != 0 && g.outer > 65535) return "too many outer blocks for the strided kernel";
        const int64_t K = (int64_t)p.w * 64 / p.lpw;
        if (K * p.m >= g.n) return "the line fits one part: use kind 1";
        if (2 * K * p.m < g.n) return "too few segments for the line length";
        const int64_t K0 = ceil_div(g.n, p.m) - K;
        if (halves_lds((int)K, p.lpw, (int)K0, p.m, es, cs, 0) > (size_t)max_lds()) return "LDS too large";
        return "";
    }
    if (p.kind == PLAN_SEG_XROWS) {
        if (g.inner != g.S) return "the row-line kernel only runs the x axis";
        if (p.lpw != 16 && p.lpw != 32 && p.lpw != 64) return "lpw must be 16, 32 or 64";
        if (p.w < 1 || p.w > 16) return "w must be in [1, 16]";
        const int64_t K = (int64_t)p.w * 64 / p.lpw;
        if (K * p.m < g.n) return "too few segments for the line length";
        if (ceil_div(g.outer * g.S, p.lpw) >= (1ll << 31)) return "too many lines";
        // the coefficient table itself need not fit: the launch then uses the
        // compressed rows or the global table
        if (4 * (int64_t)scan_slots((int)K, p.lpw, p.w * 64, false) * cs > max_lds()) return "LDS too large";
        if (K * p.m * g.S >= (1 << 24)) return "line too long";
        return "";
    }
    if (p.kind == PLAN_SEG_XPIPE) {
        if (g.inner != g.S) return "the pipelined LDS tile kernel only runs the x axis";
        if (p.m != 8 && p.m != 16) return "m must be 8 or 16 for the pipelined LDS tile kernel";
        const int64_t K = ceil_div(g.n, p.m);
        if (p.lpw < 1) return "rows per block must be >= 1";
        const int64_t threads = K * g.S * p.lpw;
        if (threads > 512) return "more than 512 threads per block";
        if ((int64_t)p.w * 64 < threads) return "w too small for the rows";
        if (p.w > 8) return "w must be <= 8";
        const int VW = 16 / es;
        if ((p.m * g.S) % VW || xtile_sb(p.m, g.S, es) % VW || (g.n * g.S) % VW)
            return "rows must split into 16-byte chunks";
        const int64_t L = g.n * g.S, tot = L * p.lpw;
        if (tot >= (1 << 24) || tot * L > (1ll << 40)) return "tile too long";
        if (!xpipe_depth(xpipe_need(g, p.lpw, p.w * 64, es))) return "row tile too long for the register prefetch";
        if (xtile_lds(p.m, g.S, p.lpw, (int)K, es, cs, p.w * 64, nullptr) > (size_t)max_lds()) return "LDS too large";
        return "";
    }
    if (p.kind == PLAN_SEG_XTILE) {
        if (g.inner != g.S) return "the LDS tile kernel only runs the x axis";
        const int64_t K = ceil_div(g.n, p.m);
        if (p.lpw < 1) return "rows per block must be >= 1";
        const int64_t threads = K * g.S * p.lpw;
        if (threads > 512) return "more than 512 threads per block";
        if ((int64_t)p.w * 64 < threads) return "w too small for the rows";
        if (p.w > 8) return "w must be <= 8";
        // FastDiv is exact while (index < 2^24) and index * divisor <= 2^40
        const int64_t L = g.n * g.S, tot = L * p.lpw;
        if (tot >= (1 << 24) || tot * L > (1ll << 40)) return "tile too long";
        if (xtile_lds(p.m, g.S, p.lpw, (int)K, es, cs, p.w * 64, nullptr) > (size_t)max_lds()) return "LDS too large";
        return "";
    }
    return "unknown plan kind";
}

SweepPlan default_plan(int axis, const AxisGeom& g, int dtype)
{
    SweepPlan p;
    const int es = (int)dtype_size(dtype), cs = compute_size(dtype);
    if (axis == 0) {
        // One or two substrates per row: the strided row kernel would read
        // pieces of 8-16 bytes of each row per instruction, so rows go
        // through one-wave LDS tiles of R rows with coalesced loads (measured
        // 21-49% faster on 256^3 and 500^3 grids of 1 and 2 substrates)
        // FP64 rows of two substrates from 384 voxels on: the pipelined row
        // tiles with M = 8 and as many rows as fit 512 threads (500^3 x 2:
        // 0.73 ms against 0.94 ms for the one-wave tiles)
        if (es == 8 && g.S == 2 && g.n >= 384) {
            const int64_t per_row = ceil_div(g.n, 8) * g.S;
            if (per_row <= 512) {
                int64_t R = 1;
                while (R * 2 * per_row <= 512) R *= 2;
                SweepPlan c;
                c.kind = PLAN_SEG_XPIPE;
                c.m = 8;
                c.lpw = (int)R;
                c.w = (int)ceil_div(R * per_row, 64);
                if (check_plan(c, g, dtype).empty()) return c;
            }
        }
        if (g.S <= 2 && g.n >= 64) {
            const int M = g.n >= 256 ? 16 : 8;
            const int64_t per_row = ceil_div(g.n, M) * g.S;
            if (per_row <= 64) {
                int64_t R = 1;
                while (R * 2 * per_row <= 64) R *= 2;
                SweepPlan c;
                c.kind = PLAN_SEG_XTILE;
                c.m = M;
                c.lpw = (int)std::min<int64_t>(R, g.outer);
                c.w = 1;
                if (check_plan(c, g, dtype).empty()) return c;
            }
        }
        // FP32 storage on long rows: the strided kernel's loads would touch
        // 16-byte pieces of each row per instruction, so rows go through LDS
        // with coalesced 16-byte loads, in the pipelined row-tile kernel
        // (from 512 voxels: two rows per tile where they fit 512 threads; on
        // 1000^3 x 4, FP32 arithmetic 6.77 -> 6.36 ms, FP64 arithmetic 6.63
        // -> 6.52 ms in alternating runs)
        if (es == 4 && g.n >= 256) {
            SweepPlan c;
            c.kind = PLAN_SEG_XPIPE;
            c.m = 16;
            const int64_t per_row = ceil_div(g.n, 16) * g.S;
            c.lpw = (g.n >= 512 && 2 * per_row <= 512) ? 2 : 1;
            c.w = (int)ceil_div(c.lpw * per_row, 64);
            if (check_plan(c, g, dtype).empty()) return c;
            c.lpw = 1;
            c.w = (int)ceil_div(per_row, 64);
            if (check_plan(c, g, dtype).empty()) return c;
        }
        // FP32 rows of 1025..2048 voxels: every (row, substrate) as a line
        // taken in two parts (kind 5), two 512-thread blocks per CU where
        // their LDS fits, as for y and z below.  Measured: 2000^3 x 8 FP32 x
        // 157.2 -> 137.5 ms; FP64 rows gain nothing (1500^3 x 8: 76.4 ms as
        // kind 3, 76.7 ms as kind 5) and keep kind 3.
        if (es == 4 && g.n > 1024 && g.n <= 2048) {
            SweepPlan c;
            c.kind = PLAN_SEG_HALVES;
            c.m = 32;
            c.lpw = 16;
            c.w = 8;
            const int K = 32, K0 = (int)ceil_div(g.n, 32) - K;
            const size_t ctab = (size_t)g.S * 4 * 33 * cs;
            if (check_plan(c, g, dtype).empty() && halves_lds(K, 16, K0, 32, es, cs, ctab) <= (size_t)max_lds() / 2)
                return c;
        }
        // preferred: every (row, substrate) as a line of the strided kernel;
        // 32 lines per tile where 16 segments or fewer cover a line (measured
        // 5-11% faster than 16 on 256^3 and 500^3 x 8)
        {
            const int pm[] = {32, 16, 8, 4};
            for (int M : pm) {
                if (M == 32 && g.n < 192) continue;
                if (M == 16 && g.n < 128) continue;
                if (M == 8 && g.n < 16) continue;
                const int lpw = ceil_div(g.n, M) <= 16 ? 32 : 16, spw = 64 / lpw;
                int64_t K = ceil_div(ceil_div(g.n, M), spw) * spw;
                SweepPlan c;
                c.kind = PLAN_SEG_XROWS;
                c.m = M;
                c.lpw = lpw;
                c.w = (int)(K * lpw / 64);
                if (check_plan(c, g, dtype).empty()) return c;
            }
        }
        const int big[] = {16, 8, 32, 4}, mid[] = {8, 4, 16, 32}, small[] = {4, 8, 16, 32};
        const int* ms = g.n >= 512 ? big : (g.n >= 64 ? mid : small);
        for (int mi = 0; mi < 4; ++mi) {
            const int M = ms[mi];
            const int64_t K = ceil_div(g.n, M);
            const int64_t per_row = K * g.S;
            if (per_row > 512) continue;
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
    // Lines of 1025..2048: the kind-1 tile of such a line is a block of up
    // to 1024 threads, alone on its CU, which issues no loads while it
    // scans; kind 5 takes the line in two parts with 512 threads (16 lines,
    // M = 32), two blocks per CU, where their LDS fits (coefficient rows
    // for a head of up to two segments assumed; a longer head falls back
    // at launch).  Measured: 2000^3 x 8 FP32 y 144 -> 127 ms, z 167 -> 130
    // ms; 1500^3 x 8 FP64 y 78.4 -> 77.3 ms, z 110.5 -> 95.1 ms.
    if (g.n > 1024 && g.n <= 2048) {
        SweepPlan c;
        c.kind = PLAN_SEG_HALVES;
        c.m = 32;
        c.lpw = 16;
        c.w = 8;
        const int K = 32, K0 = (int)ceil_div(g.n, 32) - K;
        const size_t ctab = (size_t)g.S * 4 * 33 * cs;
        if (check_plan(c, g, dtype).empty() && halves_lds(K, 16, K0, 32, es, cs, ctab) <= (size_t)max_lds() / 2)
            return c;
    }
    // FP32 arithmetic on long y and z lines: 32-line tiles (a full 128-byte
    // line per row; with FP32 registers the 1024-thread tile still leaves
    // room for its waves): z 7.66 -> 7.00 ms on 1000^3 x 4, y faster too.
    // FP32 storage with FP64 arithmetic keeps 16-line tiles (two 512-thread
    // blocks per CU): y 7.17-7.21 ms with 32 lines, 6.16-6.17 ms with 16 on
    // 1000^3 x 4 (z was 15% slower with 32); FP64 lines keep 16 as well.
    if (es == 4 && cs == 4 && g.n >= 512) {
        SweepPlan c;
        c.kind = PLAN_SEG_STRIDED;
        c.m = 32;
        c.lpw = 32;
        c.w = (int)(ceil_div(ceil_div(g.n, 32), 2) * 2 * 32 / 64);
        if (check_plan(c, g, dtype).empty()) return c;
    }
    // Lines of 192..1024: M = 32, K = the power of two >= n / 32 segments
    // (8, 16 or 32) and as many lines per tile as fill 512 threads (64, 32
    // or 16).  Fewer segments per line shorten the carry scan and wider
    // tiles read longer runs per row: measured 3-33% faster than 16-line
    // tiles of M = 16 on 256^3 and 500^3 (most for FP32); on 1000^3 this is
    // the 16-line M = 32 tile.
    if (g.n >= 192 && g.n <= 1024) {
        int64_t K = 8;
        while (K * 32 < g.n) K *= 2;
        SweepPlan c;
        c.kind = PLAN_SEG_STRIDED;
        c.m = 32;
        c.lpw = (int)(512 / K);
        c.w = 8;
        if (check_plan(c, g, dtype).empty()) return c;
    }
    const int lpw = 16;
    const int spw = 64 / lpw;
    const int big[] = {32, 16, 8, 4}, mid[] = {16, 32, 8, 4}, small[] = {8, 4, 16, 32};
    const int* ms = g.n >= 512 ? big : (g.n >= 128 ? mid : small);
    for (int mi = 0; mi < 4; ++mi) {
        const int M = ms[mi];
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

template <typename T, typename C, bool TR, int M, int P>
static hipError_t launch_xpipe_p(const SweepPlan& p, const AxisGeom& g, const T* in, T* out, const C* invd,
                                 const C* r, hipStream_t st)
{
    const int K = (int)ceil_div(g.n, M);
    const int SB = xtile_sb(M, g.S, (int)sizeof(T));
    uint32_t tile_bytes = 0;
    const size_t lds = xtile_lds(M, g.S, p.lpw, K, (int)sizeof(T), (int)sizeof(C), p.w * 64, &tile_bytes);
    const int threads = p.w * 64;
    auto kern = k_sweep_seg_xpipe<T, C, M, TR, P>;
    int dev = 0, cus = 0, occ = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, threads, lds) != hipSuccess || occ < 1) occ = 1;
    const int64_t ntiles = ceil_div(g.outer, p.lpw);
    const unsigned blocks = (unsigned)std::min<int64_t>(ntiles, (int64_t)cus * occ);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), lds, st, in, out, g, invd, r, p.lpw, K, SB, tile_bytes,
                       FastDiv((uint32_t)(g.n * g.S)), FastDiv((uint32_t)(M * g.S)));
    return hipGetLastError();
}

template <typename T, typename C, bool TR, int M>
static hipError_t launch_xpipe(const SweepPlan& p, const AxisGeom& g, const T* in, T* out, const C* invd,
                               const C* r, hipStream_t st)
{
    if constexpr (M == 8 || M == 16) {
        switch (xpipe_depth(xpipe_need(g, p.lpw, p.w * 64, (int)sizeof(T)))) {
            case 2: return launch_xpipe_p<T, C, TR, M, 2>(p, g, in, out, invd, r, st);
            case 4: return launch_xpipe_p<T, C, TR, M, 4>(p, g, in, out, invd, r, st);
            case 8: return launch_xpipe_p<T, C, TR, M, 8>(p, g, in, out, invd, r, st);
            default: break;
        }
    }
    return hipErrorInvalidValue;
}

template <typename T, typename C, bool TR, int M, bool RED>
static hipError_t launch_seg(const SweepPlan& p, const AxisGeom& g, const T* in, T* out,
                             const C* invd, const C* r, const C* comp, int compH, hipStream_t st,
                             const T* xf, double* part)
{
    if (p.kind == PLAN_SEG_HALVES) {
        // Runs as the kind-1 (x: kind-3) plan with as few segments as cover
        // the line (at most twice this plan's: one block of up to 1024
        // threads per CU) where this kernel does not apply: the transposed
        // sweeps, a grid without compressed coefficient rows, or LDS beyond
        // half the CU's, which would leave no room for a second block.
        const int threads = p.w * 64;
        const int K = threads / p.lpw;
        const int K0 = (int)(ceil_div(g.n, M) - K);
        const int nh = compH >= 0 ? (compH + M - 1) / M : 0;
        const bool comp_ok = comp && compH >= 0 && (g.n - 1) / M >= nh;
        const size_t ctab = (size_t)g.S * (nh + 2) * (M + 1) * sizeof(C);   // no zero row
        const size_t lds = halves_lds(K, p.lpw, K0, M, (int)sizeof(T), (int)sizeof(C), ctab);
        if (TR || RED || !comp_ok || lds > (size_t)max_lds() / 2) {
            SweepPlan q = p;
            q.kind = g.axis == 0 ? PLAN_SEG_XROWS : PLAN_SEG_STRIDED;
            const int spw = 64 / p.lpw;
            q.w = (int)(ceil_div(ceil_div(g.n, M), spw) * spw * p.lpw / 64);
            return launch_seg<T, C, TR, M, RED>(q, g, in, out, invd, r, comp, compH, st, xf, part);
        }
        if constexpr (!TR && !RED) {
            if (g.axis == 0) {   // every (row, substrate) of the x axis is one line
                AxisGeom gg = g;
                gg.inner = g.outer * g.S;
                gg.outer = 1;
                hipLaunchKernelGGL((k_sweep_seg_halves<T, C, M, true, 0>), dim3((unsigned)ceil_div(gg.inner, p.lpw)),
                                   dim3(threads), lds, st, in, out, gg, r, p.lpw, K0, comp, compH);
            } else {
                dim3 grid((unsigned)ceil_div(g.inner, p.lpw), (unsigned)g.outer);
                if (g.axis == 2)
                    hipLaunchKernelGGL((k_sweep_seg_halves<T, C, M, false, 2>), grid, dim3(threads), lds, st, in,
                                       out, g, r, p.lpw, K0, comp, compH);
                else
                    hipLaunchKernelGGL((k_sweep_seg_halves<T, C, M, false, 1>), grid, dim3(threads), lds, st, in,
                                       out, g, r, p.lpw, K0, comp, compH);
            }
        }
        return hipGetLastError();
    }
    if (p.kind == PLAN_SEG_STRIDED || p.kind == PLAN_SEG_XROWS) {
        const bool xrows = p.kind == PLAN_SEG_XROWS;
        AxisGeom gg = g;
        if (xrows) {            // every (row, substrate) of the x axis is one line
            gg.inner = g.outer * g.S;
            gg.outer = 1;
        }
        const int threads = p.w * 64;
        const int K = threads / p.lpw;
        dim3 grid((unsigned)ceil_div(gg.inner, p.lpw), (unsigned)gg.outer);
        const size_t scan = 4 * (size_t)scan_slots(K, p.lpw, threads, false) * sizeof(C);
        // [s][seg][k] table: segment stride M + 1 (odd), substrate stride SP with
        // SP = spw (mod bank period), so the spw segments x S substrates a wave
        // touches at once land in distinct banks
        const int period = sizeof(C) == 8 ? 16 : 32;
        const int spw = 64 / p.lpw;
        const int KM1 = K * (M + 1);
        const int SP = KM1 + (((spw - KM1) % period) + period) % period;
        const size_t tab = (size_t)g.S * SP * sizeof(C);
        const int64_t KMS = (int64_t)K * M * g.S;
        const bool lds_tab = scan + tab <= (size_t)max_lds() && KMS < (1 << 24) && KMS * g.S <= (1ll << 40);
        // The exact compressed table replaces a full table that would not fit,
        // or that would take more than 48 KB of LDS (fewer workgroups per CU).
        // It is also taken for FP32 storage and for the x rows, where the
        // smaller per-block staging measured faster on 1000^3 x 4 (FP32 y 4%,
        // z 3%, FP64 x rows 0.6%); FP64 y was even and FP64 z 4% slower.
        // compressed rows: head segments, constant, last slot's segment, zero;
        // usable when the head segments end before the last slot's segment
        const int nh = compH >= 0 ? (compH + M - 1) / M : 0;
        const bool comp_ok = comp && compH >= 0 && (g.n - 1) / M >= nh;
        const size_t ctab = comp_ok ? (size_t)g.S * (nh + 3) * (M + 1) * sizeof(C) : 0;
        const bool use_comp = ctab > 0 && scan + ctab <= (size_t)max_lds() &&
                              (!lds_tab || tab > (48u << 10) || sizeof(T) == 4 || xrows);
        const bool zaxis = g.axis == 2;
        const FastDiv dS((uint32_t)g.S);
        if (xrows && use_comp)
            hipLaunchKernelGGL((k_sweep_seg_strided<T, C, M, TR, 2, true, 0, RED>), grid, dim3(threads), scan + ctab,
                               st, in, out, gg, invd, r, p.lpw, SP, dS, comp, compH, xf, part);
        else if (xrows && lds_tab)
            hipLaunchKernelGGL((k_sweep_seg_strided<T, C, M, TR, 1, true, 0, RED>), grid, dim3(threads), scan + tab,
                               st, in, out, gg, invd, r, p.lpw, SP, dS, comp, compH, xf, part);
        else if (xrows)
            hipLaunchKernelGGL((k_sweep_seg_strided<T, C, M, TR, 0, true, 0, RED>), grid, dim3(threads), scan, st,
                               in, out, gg, invd, r, p.lpw, SP, dS, comp, compH, xf, part);
        else if (use_comp && zaxis)
            hipLaunchKernelGGL((k_sweep_seg_strided<T, C, M, TR, 2, false, 2, RED>), grid, dim3(threads),
                               scan + ctab, st, in, out, gg, invd, r, p.lpw, SP, dS, comp, compH, xf, part);
        else if (use_comp)
            hipLaunchKernelGGL((k_sweep_seg_strided<T, C, M, TR, 2, false, 1, RED>), grid, dim3(threads),
                               scan + ctab, st, in, out, gg, invd, r, p.lpw, SP, dS, comp, compH, xf, part);
        else if (lds_tab && zaxis)
            hipLaunchKernelGGL((k_sweep_seg_strided<T, C, M, TR, 1, false, 2, RED>), grid, dim3(threads),
                               scan + tab, st, in, out, gg, invd, r, p.lpw, SP, dS, comp, compH, xf, part);
        else if (lds_tab)
            hipLaunchKernelGGL((k_sweep_seg_strided<T, C, M, TR, 1, false, 1, RED>), grid, dim3(threads),
                               scan + tab, st, in, out, gg, invd, r, p.lpw, SP, dS, comp, compH, xf, part);
        else
            hipLaunchKernelGGL((k_sweep_seg_strided<T, C, M, TR, 0, false, 1, RED>), grid, dim3(threads), scan, st,
                               in, out, gg, invd, r, p.lpw, SP, dS, comp, compH, xf, part);
    } else {
        const int K = (int)ceil_div(g.n, M);
        const int SB = xtile_sb(M, g.S, (int)sizeof(T));
        uint32_t tile_bytes = 0;
        size_t lds = xtile_lds(M, g.S, p.lpw, K, (int)sizeof(T), (int)sizeof(C), p.w * 64, &tile_bytes);
        dim3 grid((unsigned)ceil_div(g.outer, p.lpw));
        const int64_t VW = 16 / sizeof(T);
        const bool vec = (M * g.S) % VW == 0 && SB % VW == 0 && (g.n * g.S) % VW == 0 &&
                         (reinterpret_cast<uintptr_t>(in) % 16) == 0 && (reinterpret_cast<uintptr_t>(out) % 16) == 0;
        // kind 4 needs 16-byte aligned fields; otherwise (and for the reverse
        // step's fused sums) its plan runs as kind 2
        if (!RED && p.kind == PLAN_SEG_XPIPE && vec) return launch_xpipe<T, C, TR, M>(p, g, in, out, invd, r, st);
        const bool vx = vec && (!RED || (reinterpret_cast<uintptr_t>(xf) % 16) == 0);
        hipLaunchKernelGGL((k_sweep_seg_xtile<T, C, M, TR, RED>), grid, dim3(p.w * 64), lds, st, in, out,
                           g, invd, r, p.lpw, K, SB, tile_bytes, FastDiv((uint32_t)(g.n * g.S)),
                           FastDiv((uint32_t)(M * g.S)), vx, xf, part);
    }
    return hipGetLastError();
}

template <typename T, typename C, bool TR, bool RED>
static hipError_t launch_typed(const SweepPlan& p, const AxisGeom& g, const void* in, void* out,
                               const void* invd, const void* r, const void* comp, int compH, hipStream_t st,
                               const AdjSums& red)
{
    const T* i = static_cast<const T*>(in);
    T* o = static_cast<T*>(out);
    const C* cf = static_cast<const C*>(invd);
    const C* rr = static_cast<const C*>(r);
    const C* cc = static_cast<const C*>(comp);
    const T* xf = static_cast<const T*>(red.x);
    if (p.kind == PLAN_LINE) {
        const int64_t lines = g.inner * g.outer;
        hipLaunchKernelGGL((k_sweep_line<T, C, TR, RED>), dim3((unsigned)ceil_div(lines, 256)), dim3(256), 0,
                           st, i, o, g, cf, rr, xf, red.part);
        return hipGetLastError();
    }
    switch (p.m) {
        case 4: return launch_seg<T, C, TR, 4, RED>(p, g, i, o, cf, rr, cc, compH, st, xf, red.part);
        case 8: return launch_seg<T, C, TR, 8, RED>(p, g, i, o, cf, rr, cc, compH, st, xf, red.part);
        case 16: return launch_seg<T, C, TR, 16, RED>(p, g, i, o, cf, rr, cc, compH, st, xf, red.part);
        case 32: return launch_seg<T, C, TR, 32, RED>(p, g, i, o, cf, rr, cc, compH, st, xf, red.part);
        default: return hipErrorInvalidValue;
    }
}

constexpr int kAdjZUnr = 1;

// z lines of up to 512 voxels: M = 16 values of x and of y per thread, K =
// the power of two >= n/16 segments (at least 8), 512/K lines per tile
static int adj_z_fused_k(int64_t n)
{
    if (n < 1 || n > 512) return 0;
    int K = 8;
    while ((int64_t)K * 16 < n) K *= 2;
    return K;
}

template <typename T, typename C>
static hipError_t launch_adj_z_fused_t(const AxisGeom& g, const void* zin, void* grad, const void* invd,
                                       const void* r, const void* comp, int compH, double* part, hipStream_t st)
{
    constexpr int M = 16;
    const int K = adj_z_fused_k(g.n);
    const int lpw = 512 / K;
    const int threads = 512;
    const size_t scan = 4 * (size_t)scan_slots(K, lpw, threads, false) * sizeof(C);
    const int period = sizeof(C) == 8 ? 16 : 32;
    const int spw = 64 / lpw;
    const int KM1 = K * (M + 1);
    const int SP = KM1 + (((spw - KM1) % period) + period) % period;
    const size_t tab = (size_t)g.S * SP * sizeof(C);
    const int64_t KMS = (int64_t)K * M * g.S;
    const bool lds_tab = scan + tab <= (size_t)max_lds() && KMS < (1 << 24) && KMS * g.S <= (1ll << 40);
    const int nh = compH >= 0 ? (compH + M - 1) / M : 0;
    const bool comp_ok = comp && compH >= 0 && (g.n - 1) / M >= nh;
    const size_t ctab = comp_ok ? (size_t)g.S * (nh + 3) * (M + 1) * sizeof(C) : 0;
    const bool use_comp = ctab > 0 && scan + ctab <= (size_t)max_lds() && (!lds_tab || tab > (48u << 10));
    int coefk = use_comp ? 2 : (lds_tab ? 1 : 0);
    if (!coefk) return hipErrorNotSupported;
    // gradient tile through LDS (DMA form) where the rows are 16-byte aligned
    // and two blocks still fit a CU; the compressed rows leave it more room
    constexpr int E = 16 / (int)sizeof(T);
    const bool dma_ok = (g.stride * (int64_t)sizeof(T)) % 16 == 0 &&
                        (g.outer == 1 || (g.outer_stride * (int64_t)sizeof(T)) % 16 == 0) && g.p0 == 0 &&
                        g.o0 == 0 && g.inner % E == 0 && reinterpret_cast<uintptr_t>(grad) % 16 == 0;
    // the tile of K*M planes (also room for the x end values and the sums,
    // two doubles per slot)
    const size_t gbytes = (size_t)K * M * lpw * sizeof(T);
    auto gb_at = [&](int ck) { return (scan / 2 + (ck == 2 ? ctab : tab) + 15) & ~(size_t)15; };
    const size_t half = (size_t)max_lds() / 2;
    bool dma = false;
    if (dma_ok) {
        if (gb_at(coefk) + gbytes <= half) dma = true;
        else if (coefk == 1 && ctab > 0 && gb_at(2) + gbytes <= half) { coefk = 2; dma = true; }
    }
    const int gb_off = dma ? (int)gb_at(coefk) : 0;
    const size_t lds = dma ? gb_at(coefk) + gbytes : scan + (coefk == 2 ? ctab : tab);
    const dim3 grid((unsigned)ceil_div(g.inner, lpw), (unsigned)g.outer);
    const FastDiv dS((uint32_t)g.S);
    const T* zi = static_cast<const T*>(zin);
    T* gr = static_cast<T*>(grad);
    const C* cf = static_cast<const C*>(invd);
    const C* rr = static_cast<const C*>(r);
    const C* cc = static_cast<const C*>(comp);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(threads), lds, st, zi, gr, g, cf, rr, lpw, SP, dS, cc, compH, part, gb_off);
    };
    if (coefk == 2) dma ? go(k_adj_z_fused<T, C, M, 2, kAdjZUnr, true>) : go(k_adj_z_fused<T, C, M, 2, kAdjZUnr, false>);
    else dma ? go(k_adj_z_fused<T, C, M, 1, kAdjZUnr, true>) : go(k_adj_z_fused<T, C, M, 1, kAdjZUnr, false>);
    return hipGetLastError();
}

bool adj_z_fusable(int dtype, const AxisGeom& g, const void* comp, int compH)
{
    if (g.axis != 2 || g.p0 != 0 || g.o0 != 0 || g.outer > 65535 || !adj_z_fused_k(g.n)) return false;
    const int K = adj_z_fused_k(g.n);
    const int cs = compute_size(dtype);
    const size_t scan = 4 * (size_t)scan_slots(K, 512 / K, 512, false) * cs;
    const int64_t KMS = (int64_t)K * 16 * g.S;
    const bool lds_tab = scan + (size_t)g.S * (K * 17 + 32) * cs <= (size_t)max_lds() && KMS < (1 << 24) &&
                         KMS * g.S <= (1ll << 40);
    const int nh = compH >= 0 ? (compH + 15) / 16 : 0;
    const bool comp_ok = comp && compH >= 0 && (g.n - 1) / 16 >= nh &&
                         scan + (size_t)g.S * (nh + 3) * 17 * cs <= (size_t)max_lds();
    return lds_tab || comp_ok;
}

hipError_t launch_adj_z_fused(int dtype, const AxisGeom& g, const void* zin, void* grad, const void* invd,
                              const void* r, const void* comp, int compH, double* part, hipStream_t st)
{
    if (g.inner * g.outer == 0) return hipSuccess;
    if (!adj_z_fusable(dtype, g, comp, compH)) return hipErrorNotSupported;
    switch (dtype) {
        case DT_F64: return launch_adj_z_fused_t<double, double>(g, zin, grad, invd, r, comp, compH, part, st);
        case DT_F32: return launch_adj_z_fused_t<float, double>(g, zin, grad, invd, r, comp, compH, part, st);
        case DT_F32_FAST: return launch_adj_z_fused_t<float, float>(g, zin, grad, invd, r, comp, compH, part, st);
        default: return hipErrorInvalidValue;
    }
}

// Transposed sweep with the sums from an LDS x tile (k_adj_tr_tile), the
// reverse step's form of that sweep where it applies: lines of up to 512
// voxels, two blocks per CU within the LDS, and tile rows of whole 16-byte
// chunks, 16-byte aligned: for y and z lines, lines filling whole chunks;
// for x lines (as rows of S substrates), S a multiple of the values per
// chunk and the tiles whole rows.  It replaces the strided kernel of the
// axis's plan (kind 1, or kind 5, whose transposed sweeps run as kind 1; x
// rows: kind 3), whose per-thread access pattern it keeps; the row-tile
// kinds for x (2, 4) keep their own kernels.  Elsewhere
// hipErrorNotSupported before any launch: the caller runs the plan's kernel.
template <typename T, typename C>
static hipError_t launch_adj_tr_tile_t(int kind, const AxisGeom& g0, const void* in, void* out, const void* invd,
                                       const void* r, const void* comp, int compH, const void* xf, double* part,
                                       hipStream_t st)
{
    constexpr int M = 16;
    constexpr int64_t E = 16 / (int64_t)sizeof(T), es = sizeof(T);
    const int K = adj_z_fused_k(g0.n);
    if (!K || g0.p0 != 0 || g0.o0 != 0 || reinterpret_cast<uintptr_t>(xf) % 16) return hipErrorNotSupported;
    if (g0.axis == 0 ? kind != PLAN_SEG_XROWS : kind != PLAN_SEG_STRIDED && kind != PLAN_SEG_HALVES)
        return hipErrorNotSupported;
    const int lpw = 512 / K;
    const bool xrows = g0.axis == 0;
    AxisGeom g = g0;
    if (xrows) {
        // every (row, substrate) a line: one outer index over rows * S lines
        const int64_t lines = g0.inner * g0.outer;
        if (g0.S % E || lpw % g0.S || (g0.n * g0.S * es) % 16 || lines >= (1ll << 31) ||
            lines * g0.S > (1ll << 40))
            return hipErrorNotSupported;
        g.inner = lines;
        g.outer = 1;
    } else if (g.outer > 65535 || (g.stride * es) % 16 || (g.outer > 1 && (g.outer_stride * es) % 16) ||
               g.inner % E) {
        return hipErrorNotSupported;
    }
    const int threads = 512;
    const size_t scan2 = 2 * (size_t)scan_slots(K, lpw, threads, false) * sizeof(C);
    const int period = sizeof(C) == 8 ? 16 : 32;
    const int spw = 64 / lpw;
    const int KM1 = K * (M + 1);
    const int SP = KM1 + (((spw - KM1) % period) + period) % period;
    const size_t tab = (size_t)g.S * SP * sizeof(C);
    const int64_t KMS = (int64_t)K * M * g.S;
    const bool tab_ok = KMS < (1 << 24) && KMS * g.S <= (1ll << 40);
    const int nh = compH >= 0 ? (compH + M - 1) / M : 0;
    const bool comp_ok = comp && compH >= 0 && (g.n - 1) / M >= nh;
    const size_t ctab = comp_ok ? (size_t)g.S * (nh + 3) * (M + 1) * sizeof(C) : 0;
    const size_t gbytes = (size_t)K * M * lpw * sizeof(T);   // also room for the sums
    const size_t half = (size_t)max_lds() / 2;
    auto gb_at = [&](size_t coefb) { return (scan2 + coefb + 15) & ~(size_t)15; };
    // the compressed rows where they fit (less to stage), else the table
    int coefk = 0;
    if (ctab > 0 && gb_at(ctab) + gbytes <= half) coefk = 2;
    else if (tab_ok && gb_at(tab) + gbytes <= half) coefk = 1;
    if (!coefk) return hipErrorNotSupported;
    const size_t at = gb_at(coefk == 2 ? ctab : tab);
    const dim3 grid((unsigned)ceil_div(g.inner, lpw), (unsigned)g.outer);
    const FastDiv dS((uint32_t)g.S);
    const T* ip = static_cast<const T*>(in);
    T* op = static_cast<T*>(out);
    const C* cf = static_cast<const C*>(invd);
    const C* rr = static_cast<const C*>(r);
    const C* cc = static_cast<const C*>(comp);
    const T* xp = static_cast<const T*>(xf);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(threads), at + gbytes, st, ip, op, g, cf, rr, lpw, SP, dS, cc, compH, xp,
                           part, (int)at);
    };
    if (xrows) coefk == 2 ? go(k_adj_tr_tile<T, C, M, 2, true>) : go(k_adj_tr_tile<T, C, M, 1, true>);
    else coefk == 2 ? go(k_adj_tr_tile<T, C, M, 2, false>) : go(k_adj_tr_tile<T, C, M, 1, false>);
    return hipGetLastError();
}

template <typename T, typename C>
static hipError_t launch_dir(bool transposed, const SweepPlan& plan, const AxisGeom& g, const void* in, void* out,
                             const void* invd, const void* r, const void* comp, int compH, hipStream_t st,
                             const AdjSums& red)
{
    if (!transposed) return launch_typed<T, C, false, false>(plan, g, in, out, invd, r, comp, compH, st, red);
    if (red.part) {
        const hipError_t e =
            launch_adj_tr_tile_t<T, C>(plan.kind, g, in, out, invd, r, comp, compH, red.x, red.part, st);
        if (e != hipErrorNotSupported) return e;
        return launch_typed<T, C, true, true>(plan, g, in, out, invd, r, comp, compH, st, red);
    }
    return launch_typed<T, C, true, false>(plan, g, in, out, invd, r, comp, compH, st, red);
}

hipError_t launch_sweep(int dtype, bool transposed, const SweepPlan& plan, const AxisGeom& g,
                        const void* in, void* out, const void* invd, const void* r, const void* comp, int compH,
                        hipStream_t st, const AdjSums& red)
{
    if (g.inner * g.outer == 0) return hipSuccess;
    if (red.part && (!transposed || !red.x || g.p0 != 0 || g.o0 != 0)) return hipErrorInvalidValue;
    switch (dtype) {
        case DT_F64: return launch_dir<double, double>(transposed, plan, g, in, out, invd, r, comp, compH, st, red);
        case DT_F32: return launch_dir<float, double>(transposed, plan, g, in, out, invd, r, comp, compH, st, red);
        case DT_F32_FAST:
            return launch_dir<float, float>(transposed, plan, g, in, out, invd, r, comp, compH, st, red);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bfvm
