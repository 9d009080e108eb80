// Register-segmented Thomas solver shared by the sweep kernels and the
// batched multi-domain engine (see sweep.hip for the method).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bfvm {

// ------------------------------------------------ segment solver (registers)
//
// A block solves nl lines, each cut into K segments of M elements held in
// the registers of one thread.  The segment carries travel through 4 LDS
// arrays of [K][nl] values (forward local value, forward coefficient
// product, backward local value, backward coefficient product), indexed
// [segment * nl + line].  They are resolved by one leader thread per line
// (threads 0..nl-1), which walks the K segments in order with all LDS loads
// issued ahead of the dependent multiply-add chain and leaves each segment's
// incoming carry in place of its local value (or, where it fits, by the
// lane-parallel scan below).

// init: the carry entering the first segment in scan order; last (if not
// null): where the carry leaving the last segment is written, at last[line].
// UNR: segments whose LDS terms are loaded ahead of their multiply-adds.
template <typename C, int UNR = 8>
__device__ __forceinline__ void carry_scan(C* val, const C* prod, int K, int nl, int line, bool reverse,
                                           C init = 0, C* last = nullptr)
{
    C c = init;
    if (!reverse) {
        int j = 0;
        for (; j + UNR <= K; j += UNR) {
            C f[UNR], g[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) { f[u] = val[(j + u) * nl + line]; g[u] = prod[(j + u) * nl + line]; }
#pragma unroll
            for (int u = 0; u < UNR; ++u) { val[(j + u) * nl + line] = c; c = f[u] + g[u] * c; }
        }
        for (; j < K; ++j) {
            const C f = val[j * nl + line], g = prod[j * nl + line];
            val[j * nl + line] = c;
            c = f + g * c;
        }
    } else {
        int j = K - 1;
        for (; j - UNR >= -1; j -= UNR) {
            C f[UNR], g[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) { f[u] = val[(j - u) * nl + line]; g[u] = prod[(j - u) * nl + line]; }
#pragma unroll
            for (int u = 0; u < UNR; ++u) { val[(j - u) * nl + line] = c; c = f[u] + g[u] * c; }
        }
        for (; j >= 0; --j) {
            const C f = val[j * nl + line], g = prod[j * nl + line];
            val[j * nl + line] = c;
            c = f + g * c;
        }
    }
    if (last) last[line] = c;
}

// Lane-parallel form of the same scan.  When a line's K segments fit one
// group of KP lanes (KP = the power of two >= K, at most 64) and the block
// has KP lanes for each of its nl lines, lane q of group l takes segment q
// (in scan order) of line l and the groups run a log2(KP)-step inclusive
// scan of the affine maps c -> f + g c through DPP lane moves (no LDS round
// trip per step); one more shift turns it into the exclusive carries.  The
// LDS arrays are then laid out line-major, [line * (KP + 1) + segment], so
// that both the writers (lanes over lines) and the scan (lanes over
// segments) touch distinct banks.  Kernels choose the scan at compile time
// (par).  Measured on 1000^3 x 4: the lane-parallel scan takes the FP32 LDS
// row tiles from 8.1 to 6.6 ms per sweep and the batched step from 5.38 to
// 5.20 ms; the strided tiles of long y/z lines keep the leader scan (the
// lane-parallel one was even for FP64 and 1-3% slower for FP32).
__host__ __device__ inline int scan_kp(int K, int nl, int threads, bool par)
{
    int kp = 1;
    while (kp < K) kp <<= 1;
    return (par && kp <= 64 && nl * kp <= threads) ? kp : 0;
}

// values per carry array: the lane-parallel or the serial layout
__host__ __device__ inline int scan_slots(int K, int nl, int threads, bool par)
{
    const int kp = scan_kp(K, nl, threads, par);
    return kp ? nl * (kp + 1) : K * nl;
}

// DPP lane moves (gfx9 encodings): row_shr:n = 0x110 + n within 16-lane
// rows, row_bcast:15 = 0x142 (lane 15 of each row to the next row),
// row_bcast:31 = 0x143 (lane 31 to rows 2 and 3), wave_shr:1 = 0x138.
// Lanes without a source, or outside the row mask, keep their own value.
template <int CTRL, int RM>
__device__ __forceinline__ int dpp32(int x)
{
    return __builtin_amdgcn_update_dpp(x, x, CTRL, RM, 0xf, false);
}
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_mov(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = dpp32<CTRL, RM>((int)b), hi = dpp32<CTRL, RM>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL, int RM>
__device__ __forceinline__ float dpp_mov(float x)
{
    return __int_as_float(dpp32<CTRL, RM>(__float_as_int(x)));
}

template <typename C>
__device__ __forceinline__ void carry_scan_par(C* val, const C* prod, int K, int KP, int nl, bool reverse)
{
    const int t = threadIdx.x;
    const int line = t / KP;
    const int q = t - line * KP;                 // position in scan order
    const int j = reverse ? K - 1 - q : q;       // segment
    const bool real = line < nl && q < K;
    const int at = line * (KP + 1) + j;
    C f = 0, g = 1;                              // identity map for idle lanes
    if (real) {
        f = val[at];
        g = prod[at];
    }
    // groups of KP lanes are aligned to KP (a power of two <= 64): inside a
    // 16-lane row the steps 1, 2, 4, 8 scan each row (or each smaller group);
    // row_bcast:15 then joins rows 0|1 and 2|3, row_bcast:31 rows 0-1|2-3
    const int r16 = q & 15;
#define BFVM_SCAN_STEP(D)                                                         \
    if (KP > D) {                                                                 \
        const C fo = dpp_mov<0x110 + D, 0xf>(f), go = dpp_mov<0x110 + D, 0xf>(g); \
        if (r16 >= D) {                                                           \
            f = f + g * fo;                                                       \
            g = g * go;                                                           \
        }                                                                         \
    }
    BFVM_SCAN_STEP(1)
    BFVM_SCAN_STEP(2)
    BFVM_SCAN_STEP(4)
    BFVM_SCAN_STEP(8)
#undef BFVM_SCAN_STEP
    if (KP >= 32) {
        const C fo = dpp_mov<0x142, 0xa>(f), go = dpp_mov<0x142, 0xa>(g);
        if ((t >> 4) & 1) {
            f = f + g * fo;
            g = g * go;
        }
    }
    if (KP == 64) {
        const C fo = dpp_mov<0x143, 0xc>(f), go = dpp_mov<0x143, 0xc>(g);
        if ((t >> 5) & 1) {
            f = f + g * fo;
            g = g * go;
        }
    }
    C c = dpp_mov<0x138, 0xf>(f);
    if (q == 0) c = 0;
    if (real) val[at] = c;
}

// Ragged tails.  A line of n elements is covered by K segments of M; the
// slots past the end (i >= n) are padding: their coefficient invd is 0 and
// their input is any finite value (a clamped, in-bounds load).  With invd = 0
// a padding slot yields exactly 0 in both passes and multiplies every carry
// crossing it by 0, so it changes no real element, in the Thomas solve and
// in the transposed solve alike.  Every segment therefore runs the same
// guard-free code; only the final stores are guarded.

// Coefficient accessors: coef(k) = invd of slot i0 + k of the thread's
// segment (0 when i0 + k >= n), prev = invd of slot i0 - 1 (0 when i0 = 0).
template <typename C>
struct LdsCoef {        // the block's zero-padded LDS copy, [s][segment][k] layout
    const C* p;                // &tab[s*SP + seg*MP]: the M slots are contiguous
    C prev;
    __device__ __forceinline__ C operator()(int k) const { return p[k]; }
};

template <typename C>
struct GlobalCoef {     // the global [n][S] table, masked past the line end
    const C* __restrict__ p;   // &invd[i0*S + s] (clamped into the table)
    int S;
    int last;                  // n - 1 - i0
    C prev;
    __device__ __forceinline__ C operator()(int k) const
    {
        return k <= last ? p[(k <= last ? k : 0) * S] : (C)0;
    }
};

template <typename C, int M>
struct RegCoef {        // the segment's M values held in registers
    C b[M];
    C prev;
    __device__ __forceinline__ C operator()(int k) const { return b[k]; }
};

// Workgroup barrier for LDS traffic only: the wave's own LDS accesses are
// complete (lgkmcnt 0) before it, and the compiler moves no memory access
// across it.  Unlike __syncthreads it does not wait for the wave's global
// loads in flight, so global-to-LDS loads can continue through it; their
// target is read only after an explicit wait for them and a barrier.
__device__ __forceinline__ void lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// 16 bytes per lane from global memory straight into LDS (no registers):
// lane l's bytes land at wave_base + 16 * l; wave_base is the same for the
// whole wave.  Counted by the wave's vector-memory counter like a load.
__device__ __forceinline__ void load_lds16(const void* src, void* wave_base)
{
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)wave_base, 16, 0, 0);
}

// The block's tile [K*M planes][lpw lines] of T (lines of its tile
// contiguous, planes st apart; K*M*lpw = 512*M, the block's 512 threads
// times M) into LDS at gb with 16-byte global-to-LDS loads, which take no
// registers: chunk c = plane * lpw/E + part of the plane's row (E = 16 /
// sizeof(T) values), Q = M * sizeof(T) / 16 chunks per thread, a wave's
// instruction filling 64 consecutive ones (lane l at 16 * l bytes past its
// base).  Every lane issues every load: planes past the line end and chunks
// past the last line read a clamped chunk, so the count in flight is fixed
// and a later wait for values loaded before these counts them exactly.
// Tile line l (a multiple of E) starts at src0 + lineoff(l) at plane 0, its
// E lines contiguous; nlines = lines from the tile's first to the last line
// of the grid (at least E, a multiple of E).  The tile is complete once the
// wave's memory counter is 0 and then, for every wave's part, after a
// barrier.
template <typename T, int M, typename F>
__device__ __forceinline__ void fetch_tile_lds(T* gb, const T* src0, F lineoff, int64_t st, int n, int lpw,
                                               int64_t nlines)
{
    constexpr int E = 16 / (int)sizeof(T);
    constexpr int Q = M * (int)sizeof(T) / 16;
    static_assert(Q * 16 == M * (int)sizeof(T), "whole chunks per thread");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int chs = __builtin_ctz((unsigned)(lpw / E));   // chunks per row: a power of two
    const int64_t cmax = nlines / E - 1;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = (q * (int)(blockDim.x >> 6) + wave) * 64;
        const int c = j + lane;
        const int pl = min(c >> chs, n - 1);
        const int cc = (int)min((int64_t)(c & ((1 << chs) - 1)), cmax);
        load_lds16(src0 + lineoff(cc * E) + pl * st, gb + (int64_t)j * E);
    }
}

// vmcnt(0) alone: the wave's vector-memory loads (and global-to-LDS loads)
// are complete
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// The three register phases of a segment.
// forward pass with zero carry; G = product of the forward coefficients
template <typename C, int M, bool TR, typename Coef>
__device__ __forceinline__ void seg_forward(C (&v)[M], C r, const Coef& coef, C& f, C& G)
{
    f = 0;
    G = 1;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const C b = coef(k);
        if (!TR) {
            f = b * (v[k] + r * f);
            G *= r * b;
        } else {
            const C a = r * (k > 0 ? coef(k - 1) : coef.prev);
            f = v[k] + a * f;
            G *= a;
        }
        v[k] = f;
    }
}

// forward correction t_i = f_i + (prod of coefficients up to i) * carry
template <typename C, int M, bool TR, typename Coef>
__device__ __forceinline__ void seg_fwd_correct(C (&v)[M], C r, const Coef& coef, C carry)
{
    C c = carry;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const C a = r * (!TR ? coef(k) : (k > 0 ? coef(k - 1) : coef.prev));
        c = a * c;
        v[k] += c;
    }
}

// the backward pass with zero carry; GB = product of alpha over the segment
template <typename C, int M, bool TR, typename Coef>
__device__ __forceinline__ void seg_bwd_local(C (&v)[M], C r, const Coef& coef, C& bw, C& GB)
{
    bw = 0;
    GB = 1;
#pragma unroll
    for (int k = M - 1; k >= 0; --k) {
        const C b = coef(k);
        const C a = r * b;
        if (!TR)
            bw = v[k] + a * bw;
        else
            bw = b * (v[k] + r * bw);
        GB *= a;
        v[k] = bw;
    }
}

// the two together (the middle of a whole-line solve)
template <typename C, int M, bool TR, typename Coef>
__device__ __forceinline__ void seg_middle(C (&v)[M], C r, const Coef& coef, C carry, C& bw, C& GB)
{
    seg_fwd_correct<C, M, TR>(v, r, coef, carry);
    // Re-read the coefficients below instead of keeping all M of them live
    // across both loops (they are cheap LDS/L1 reads; registers are not).
    asm volatile("" ::: "memory");
    seg_bwd_local<C, M, TR>(v, r, coef, bw, GB);
}

// backward correction x_i = b_i + (prod of alpha from i to the segment end) * X
template <typename C, int M, typename Coef>
__device__ __forceinline__ void seg_last(C (&v)[M], C r, const Coef& coef, C X)
{
    C e = X;
#pragma unroll
    for (int k = M - 1; k >= 0; --k) {
        e = r * coef(k) * e;
        v[k] += e;
    }
}

// Solve one segment held in v (see the file comment).  sc points to 4 LDS
// arrays of scan_slots(K, nl, blockDim.x, PAR) carry terms each.  Every
// thread of the block calls this (it holds barriers and shuffles); writer =
// the thread owns a (segment, line) slot.
// UNR: see carry_scan (fewer registers for the leader scan where a kernel
// holds more than one segment's values).  ASYNC: the block has
// global-to-LDS loads in flight during the solve; its barriers order LDS
// only (lds_sync), and with the leader scan the backward terms reuse the
// forward arrays (2 arrays instead of 4): every thread reads its own
// forward carry before it writes its own backward term.
template <typename C, int M, bool TR, bool PAR, typename Coef, int UNR = 8, bool ASYNC = false>
__device__ __forceinline__ void solve_segment(C (&v)[M], int seg, int K, int line, int nl, C r,
                                              const Coef& coef, C* sc, bool writer)
{
    auto sync = [] {
        if constexpr (ASYNC) lds_sync();
        else __syncthreads();
    };
    const int KP = scan_kp(K, nl, (int)blockDim.x, PAR);
    const int A = KP ? nl * (KP + 1) : K * nl;
    C* sF = sc;
    C* sG = sc + A;
    C* sB = ASYNC && !PAR ? sF : sc + 2 * A;
    C* sH = ASYNC && !PAR ? sG : sc + 3 * A;
    const int slot = KP ? line * (KP + 1) + seg : seg * nl + line;
    C f, G;
    seg_forward<C, M, TR>(v, r, coef, f, G);
    if (writer) {
        sF[slot] = f;
        sG[slot] = G;
    }
    sync();
    if (KP) carry_scan_par(sF, sG, K, KP, nl, false);
    else if ((int)threadIdx.x < nl) carry_scan<C, UNR>(sF, sG, K, nl, threadIdx.x, false);
    sync();
    const C carry = writer ? sF[slot] : (C)0;
    C bw, GB;
    seg_middle<C, M, TR>(v, r, coef, carry, bw, GB);
    if (writer) {
        sB[slot] = bw;
        sH[slot] = GB;
    }
    sync();
    if (KP) carry_scan_par(sB, sH, K, KP, nl, true);
    else if ((int)threadIdx.x < nl) carry_scan<C, UNR>(sB, sH, K, nl, threadIdx.x, true);
    sync();
    const C X = writer ? sB[slot] : (C)0;
    seg_last<C, M>(v, r, coef, X);
}

// ------------------------------------------- reverse-step sums (adjoint)
//
// The reverse step needs, per substrate and axis, sum y^T (L_N x) and
// sum y^T x, where y is the transposed sweep's output and x the forward
// sweep's output on the same lines, and (L_N x)_i = [i > 0](x_i - x_{i-1})
// + [i < n-1](x_i - x_{i+1}) is the zero-flux Laplacian.  A transposed sweep
// holds y in registers, so it forms the sums itself: each thread streams x
// along its segment (with the one neighbour on each side), then the
// segments of a line are added in order in LDS and the line's two sums are
// written, one pair per line.  Padding slots have y = 0 and add nothing.

// Sums of one segment: x_{i0 + k} at xp[k * st] for the real slots k <= last
// (last >= 0); x_{i0 - 1} at xp[-st] when i0 > 0.  The loads run eight at a
// time behind a compiler barrier, so they do not all become live at once
// beside the M values of y.
template <typename C, int M, bool NT, typename T>
__device__ __forceinline__ void seg_adjoint_sums(const C (&y)[M], const T* xp, int64_t st, int last, bool left,
                                                 double& a0, double& a1)
{
    auto ld = [&](int64_t off) -> double {
        if constexpr (NT) return (double)__builtin_nontemporal_load(&xp[off]);
        else return (double)xp[off];
    };
    double xl = left ? ld(-st) : 0.0;
    double xc = ld(0);
    a0 = 0.0;
    a1 = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        if ((k & 7) == 0) asm volatile("" ::: "memory");
        const double xn = ld((int64_t)(k + 1 <= last ? k + 1 : last) * st);
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

// Adds the (a0, a1) of every (segment, line) slot of the block in segment
// order and writes each valid line's pair to out[2 L], L = L0 + line.  The
// carry arrays sc of solve_segment are reused (they hold at least 2 doubles
// per slot in either layout), so this must follow the solve; every thread
// of the block calls it.  LDSB: its barriers order LDS only (lds_sync), so
// global stores issued before it stay in flight.
template <typename C, bool LDSB = false>
__device__ __forceinline__ void line_sums_store(double a0, double a1, int seg, int K, int line, int nl, C* sc,
                                                bool par, bool writer, double* out, int64_t L0, int nvalid)
{
    const int KP = scan_kp(K, nl, (int)blockDim.x, par);
    const int A = KP ? nl * (KP + 1) : K * nl;
    double* s0 = reinterpret_cast<double*>(sc);
    double* s1 = s0 + A;
    auto sync = [] {
        if constexpr (LDSB) lds_sync();
        else __syncthreads();
    };
    sync();   // the solve's last reads of the carry arrays are done
    if (writer) {
        const int slot = KP ? line * (KP + 1) + seg : seg * nl + line;
        s0[slot] = a0;
        s1[slot] = a1;
    }
    sync();
    const int l = (int)threadIdx.x;
    if (l < nl && l < nvalid) {
        double b0 = 0.0, b1 = 0.0;
        for (int j = 0; j < K; ++j) {
            const int sl = KP ? l * (KP + 1) + j : j * nl + l;
            b0 += s0[sl];
            b1 += s1[sl];
        }
        out[2 * (L0 + l) + 0] = b0;
        out[2 * (L0 + l) + 1] = b1;
    }
}

template <typename T> struct Vec16;
template <> struct Vec16<double> { using type = double2; };
template <> struct Vec16<float> { using type = float4; };

struct FastDiv {   // q / d for q * d <= 2^40: (q * m) >> 40
    uint64_t m;
    __host__ __device__ FastDiv() : m(1) {}
    __host__ __device__ explicit FastDiv(uint32_t d) : m(((1ull << 40) + d - 1) / d) {}
    __device__ __forceinline__ uint32_t div(uint32_t q) const { return (uint32_t)(((uint64_t)q * m) >> 40); }
};

// XCD-aware tile order.  The dispatcher hands workgroups to the eight XCDs
// round-robin in launch order (block L goes to XCD L % 8), and each XCD has
// its own L2.  Giving XCD x the contiguous tile range
// [x*per + min(x, rem), ...) instead makes neighbouring tiles - which share
// cache lines and pages when a tile row is narrower than a 128-byte line -
// run on the same XCD at about the same time.  The map is a bijection of
// [0, gridDim.x * gridDim.y).
__device__ __forceinline__ void xcd_tile(uint32_t& bx, uint32_t& by)
{
    const uint32_t gx = gridDim.x;
    const uint32_t nb = gx * gridDim.y;
    const uint32_t L = blockIdx.y * gx + blockIdx.x;
    const uint32_t x = L % 8u, q = L / 8u;
    const uint32_t per = nb / 8u, rem = nb % 8u;
    const uint32_t t = x * per + (x < rem ? x : rem) + q;
    by = t / gx;
    bx = t - by * gx;
}


}  // namespace bfvm
