// Batched multi-domain stepping: many independent grids of uneven size,
// substrate count and storage type advanced together, one captured hipGraph
// replay per step.
//
// Each domain's step is a linear chain of stages (source, Dirichlet, x sweep,
// Dirichlet, y sweep, Dirichlet, z sweep, Dirichlet; the adjoint step adds
// copies, masks and transposed sweeps that also form the parameter sums).
// Every stage is cut into
// work items (tiles of lines for sweeps, ranges for the sparse stages).
//
// Grouped mode (the default): one kernel launch per stage covers that stage
// of EVERY domain, one block per item, so the order of the launches is the
// order of the stages and no block ever waits for another.  A sweep stage is
// split into one launch per (storage type, elements-per-thread) class, so
// each launch runs a kernel compiled for exactly that register shape; the
// lines per tile may differ between domains of a class.  A step is at most
// 4 + 3 x (number of classes) launches, captured once and replayed.  The
// launches of each storage type form an independent chain on a stream of its
// own, so the chains of FP64 and FP32 domains overlap on the device.
//
// Domains the grouped kernels cannot take (lines over 256 voxels, more than
// 2048 coefficient-table entries on an axis, more than 256 substrates or
// 2^31 elements) join the same graph through their own grid's kernels (the
// single-grid sweeps, plain schedule, the grid's plans and, for the reverse
// step, the grid's workspace), on one more chain of their own.
//
// Persistent mode (switched off): ONE launch per step whose blocks take the
// items of all stages from an atomic queue and wait, through per-(domain,
// stage) completion counters, for the previous stage of their own domain.
// On gfx950 its dependency waits did not complete, both with the counters in
// ordinary device memory and in uncached memory; until the cause is known,
// bfvm_batch_set_mode refuses it.  The scheduler is kept below unchanged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "internal.hpp"
#include "seg_solver.hpp"
#include "batch_program.hpp"

namespace bfvm {

// ------------------------------------------------------------ device work

struct SweepShape {
    int64_t n, inner, outer, stride, outer_stride;
    bool xrows;
    int64_t row_len;
};

__device__ __forceinline__ SweepShape sweep_shape(const BDomain& d, int axis)
{
    SweepShape q;
    const int64_t S = d.S;
    q.xrows = axis == 0;
    q.row_len = d.nx * S;
    if (axis == 0) {
        q.n = d.nx; q.inner = d.ny * d.nz * S; q.outer = 1; q.stride = S; q.outer_stride = 0;
    } else if (axis == 1) {
        q.n = d.ny; q.inner = d.nx * S; q.outer = d.nz; q.stride = d.nx * S; q.outer_stride = d.ny * d.nx * S;
    } else {
        q.n = d.nz; q.inner = d.nx * d.ny * S; q.outer = 1; q.stride = d.nx * d.ny * S; q.outer_stride = 0;
    }
    return q;
}

// One tile of lpw lines (all K = blockDim/lpw segments), as in the strided
// sweep kernel, with coefficients read from the [n][S] table invd (global,
// or the block's LDS copy of it).  Split into the thread's tile geometry,
// the load of its M values (in storage precision) and the solve + store, so
// that a loop over tiles can load the next tile while it solves this one.
// Element indices are signed 32-bit (a batched domain has < 2^31 elements):
// a padding slot's index base + last * st, with last < 0, is then the line's
// last element, computed without leaving the domain.
__device__ __forceinline__ int lpw_log2(int lpw) { return 31 - __clz(lpw); }

struct TileSpot {
    int base;        // element index of the thread's first slot
    int last;        // n - 1 - i0: slots k > last are padding
    int cnt;         // slots to store
    int s;           // substrate
};

__device__ __forceinline__ TileSpot tile_spot(const SweepShape& q, int S, const FastDiv& dS, int lpw, int M,
                                              uint32_t ox, uint32_t oy)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int line = lane & (lpw - 1);   // lpw is 16, 32 or 64
    const int seg = wave * (64 >> lpw_log2(lpw)) + (lane >> lpw_log2(lpw));
    const uint32_t inner = (uint32_t)q.inner;
    const uint32_t p = (uint32_t)ox * lpw + line;
    const bool valid = p < inner;
    const uint32_t pa = valid ? p : inner - 1;
    TileSpot t;
    const uint32_t row = dS.div(pa);   // pa * S < 2^39: exact
    t.s = (int)(pa - row * (uint32_t)S);
    const int i0 = seg * M;
    t.last = (int)q.n - 1 - i0;
    t.cnt = !valid || t.last < 0 ? 0 : (t.last >= M ? M : t.last + 1);
    const int line0 = q.xrows ? (int)(row * (uint32_t)q.row_len) + t.s
                              : (int)oy * (int)q.outer_stride + (int)pa;
    t.base = line0 + i0 * (int)q.stride;
    return t;
}

template <typename T, int M>
__device__ __forceinline__ void tile_load(const T* in, const TileSpot& t, int st, T (&raw)[M])
{
#pragma unroll
    for (int k = 0; k < M; ++k) raw[k] = in[t.base + (k <= t.last ? k : t.last) * st];
}

template <typename T, typename C, int M, bool TR>
__device__ __forceinline__ void tile_solve_store(T* out, const TileSpot& t, int st, const T (&raw)[M], int S,
                                                 int lpw, const C* __restrict__ invd, const C* __restrict__ rr,
                                                 C* sc, C (&v)[M])
{
    const int K = blockDim.x / lpw;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int line = lane & (lpw - 1);   // lpw is 16, 32 or 64
    const int seg = wave * (64 >> lpw_log2(lpw)) + (lane >> lpw_log2(lpw));
    const int i0 = seg * M;
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = (C)raw[k];
    const C r = rr[t.s];
    RegCoef<C, M> coef;
    coef.prev = (TR && i0 > 0 && t.last >= 0) ? invd[(i0 - 1) * S + t.s] : (C)0;
    const C* cf = invd + (t.last >= 0 ? i0 * S + t.s : t.s);
#pragma unroll
    for (int k = 0; k < M; ++k) coef.b[k] = k <= t.last ? cf[(k <= t.last ? k : 0) * S] : (C)0;
    solve_segment<C, M, TR, true>(v, seg, K, line, lpw, r, coef, sc, true);
    T* op = out + t.base;
    asm volatile("" : "+v"(op));
#pragma unroll
    for (int k = 0; k < M; ++k)
        if (k < t.cnt) op[k * st] = (T)v[k];
}

// The reverse step's parameter sums of one transposed tile (y in v, the
// forward output x streamed from xf): per-line sums in segment order, then
// added into acc[2 s], acc[2 s + 1] by substrate in line order.  Every
// thread of the block calls this; lsum holds 2 doubles per line of the tile.
template <typename T, typename C, int M>
__device__ __forceinline__ void tile_sums(const C (&v)[M], const TileSpot& t, const SweepShape& q, int S,
                                          const FastDiv& dS, int lpw, uint32_t ox, const T* __restrict__ xf, C* sc,
                                          double* lsum, double* acc)
{
    const int K = blockDim.x / lpw;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int line = lane & (lpw - 1);   // lpw is 16, 32 or 64
    const int seg = wave * (64 >> lpw_log2(lpw)) + (lane >> lpw_log2(lpw));
    double a0 = 0.0, a1 = 0.0;
    if (t.cnt > 0) seg_adjoint_sums<C, M, false>(v, xf + t.base, (int64_t)q.stride, t.last, seg > 0, a0, a1);
    const int KP = scan_kp(K, lpw, (int)blockDim.x, true);
    const int A = KP ? lpw * (KP + 1) : K * lpw;
    double* s0 = reinterpret_cast<double*>(sc);
    double* s1 = s0 + A;
    __syncthreads();   // the solve's last reads of the carry arrays are done
    const int slot = KP ? line * (KP + 1) + seg : seg * lpw + line;
    s0[slot] = a0;
    s1[slot] = a1;
    __syncthreads();
    const uint32_t p0 = ox * (uint32_t)lpw;
    const int nvalid = (int)min((int64_t)lpw, q.inner - (int64_t)p0);
    const int l = (int)threadIdx.x;
    if (l < nvalid) {
        double b0 = 0.0, b1 = 0.0;
        for (int j = 0; j < K; ++j) {
            const int sl = KP ? l * (KP + 1) + j : j * lpw + l;
            b0 += s0[sl];
            b1 += s1[sl];
        }
        lsum[2 * l + 0] = b0;
        lsum[2 * l + 1] = b1;
    }
    __syncthreads();
    // line p0 + l belongs to substrate (p0 + l) % S
    const int ph = (int)(p0 - dS.div(p0) * (uint32_t)S);
    for (int sub = (int)threadIdx.x; sub < S; sub += (int)blockDim.x) {
        double b0 = acc[2 * sub + 0], b1 = acc[2 * sub + 1];
        for (int l2 = (sub - ph + S) % S; l2 < nvalid; l2 += S) {
            b0 += lsum[2 * l2 + 0];
            b1 += lsum[2 * l2 + 1];
        }
        acc[2 * sub + 0] = b0;
        acc[2 * sub + 1] = b1;
    }
}

// One tile; for transposed tiles also the parameter sums (xf, lsum, acc).
template <typename T, typename C, int M, bool TR>
__device__ __forceinline__ void batch_tile(const T* in, T* out, const SweepShape& q, int S, const FastDiv& dS,
                                           int lpw, uint32_t ox, uint32_t oy, const C* __restrict__ invd,
                                           const C* __restrict__ rr, C* sc, const T* __restrict__ xf, double* lsum,
                                           double* acc)
{
    const TileSpot t = tile_spot(q, S, dS, lpw, M, ox, oy);
    T raw[M];
    tile_load<T, M>(in, t, (int)q.stride, raw);
    C v[M];
    tile_solve_store<T, C, M, TR>(out, t, (int)q.stride, raw, S, lpw, invd, rr, sc, v);
    if constexpr (TR) tile_sums<T, C, M>(v, t, q, S, dS, lpw, ox, xf, sc, lsum, acc);
}

// acc: 2 * S doubles of the item's parameter sums (transposed items)
template <typename T, typename C, bool TR>
__device__ void batch_sweep_item(const BDomain& d, const BItem& it, C* sc, double* lsum, double* acc,
                                 double* partials)
{
    const SweepShape q = sweep_shape(d, it.axis);
    const int lpw = it.lpw;
    const int64_t tpo = (q.inner + lpw - 1) / lpw;   // tiles per outer index
    const T* in = static_cast<const T*>(d.buf[it.in]);
    T* out = static_cast<T*>(d.buf[it.out]);
    const T* xf = TR ? static_cast<const T*>(d.buf[it.xb]) : nullptr;
    const C* invd = static_cast<const C*>(d.invd[it.axis]);
    const C* rr = static_cast<const C*>(d.r[it.axis]);
    if (TR)
        for (int sub = threadIdx.x; sub < d.S; sub += blockDim.x) acc[2 * sub] = acc[2 * sub + 1] = 0.0;
    const FastDiv dS((uint32_t)d.S);
    // tile t = oy * tpo + ox, stepped without a division per tile
    uint32_t oy = (uint32_t)(it.a0 / tpo), ox = (uint32_t)(it.a0 - (int64_t)oy * tpo);
    for (int64_t t = it.a0; t < it.a1; ++t) {
        if (it.m == 4)
            batch_tile<T, C, 4, TR>(in, out, q, d.S, dS, lpw, ox, oy, invd, rr, sc, xf, lsum, acc);
        else
            batch_tile<T, C, 8, TR>(in, out, q, d.S, dS, lpw, ox, oy, invd, rr, sc, xf, lsum, acc);
        if (++ox == (uint32_t)tpo) {
            ox = 0;
            ++oy;
        }
    }
    if (TR)
        for (int sub = threadIdx.x; sub < d.S; sub += blockDim.x) {
            partials[it.slot + 2 * sub + 0] = acc[2 * sub + 0];
            partials[it.slot + 2 * sub + 1] = acc[2 * sub + 1];
        }
}

template <typename T>
__device__ void batch_sparse_item(const BDomain& d, const BItem& it)
{
    const int S = d.S;
    switch (it.type) {
        case ST_SRC: {
            // entry indices are below nsrc * S <= the domain's elements < 2^31
            T* u = static_cast<T*>(d.buf[it.out]);
            for (int64_t t = it.a0 + threadIdx.x; t < it.a1; t += blockDim.x) {
                const uint32_t k = (uint32_t)t / (uint32_t)S;
                const int64_t e = d.src_vox[k] * S + ((uint32_t)t - k * (uint32_t)S);
                u[e] = (T)(((double)u[e] + d.src_P[t]) * d.src_invQ[t]);
            }
            break;
        }
        case ST_SRC_T: {
            T* g = static_cast<T*>(d.buf[it.out]);
            for (int64_t t = it.a0 + threadIdx.x; t < it.a1; t += blockDim.x) {
                const uint32_t k = (uint32_t)t / (uint32_t)S;
                const int64_t e = d.src_vox[k] * S + ((uint32_t)t - k * (uint32_t)S);
                g[e] = (T)((double)g[e] * d.src_invQ[t]);
            }
            break;
        }
        case ST_DIR: {
            T* u = static_cast<T*>(d.buf[it.out]);
            for (int64_t t = it.a0 + threadIdx.x; t < it.a1; t += blockDim.x) u[d.dir_elem[t]] = (T)d.dir_val[t];
            break;
        }
        case ST_MASK: {
            T* g = static_cast<T*>(d.buf[it.out]);
            for (int64_t t = it.a0 + threadIdx.x; t < it.a1; t += blockDim.x) g[d.dir_elem[t]] = (T)0;
            break;
        }
        case ST_COPY: {
            const T* a = static_cast<const T*>(d.buf[it.in]);
            T* b = static_cast<T*>(d.buf[it.out]);
            for (int64_t t = it.a0 + threadIdx.x; t < it.a1; t += blockDim.x) b[t] = a[t];
            break;
        }
        default: break;
    }
}


// ------------------------------------------------------------ grouped mode

// One block per item of one sweep stage (one storage type and M).
// The axis's [n][S] coefficient table (n*S <= kBatchTab) is copied to LDS
// once per item, so the tiles read their coefficients from LDS instead of
// issuing as many global loads as they load field values.

// At most 128 VGPRs (four waves per SIMD), so that two 512-thread blocks
// fit per CU, except the transposed M = 16 tiles.  Measured on 96 uneven
// domains: the forward M = 16 tiles at 128 VGPRs (a few spilled) instead of
// 136 took the step from 5.21 to 4.78 ms; the transposed ones (45 spilled)
// made the reverse step 8% slower, so they keep one block per CU.
// Transposed items also form the reverse step's parameter sums of their
// tiles from the y they hold and the forward output x (buffer it.xb), and
// write the item's 2 S sums to partials[it.slot].
template <typename T, typename C, int M, bool TR>
__global__ __launch_bounds__(kBatchThreads, (TR && M > 8) ? 2 : 4) void k_group_sweep(const BDomain* __restrict__ doms,
                                                                                      const BItem* __restrict__ items,
                                                                                      double* __restrict__ partials)
{
    // carry arrays, lane-parallel layout: lpw * (K + 1) = 512 + lpw <= 576 slots each
    __shared__ __align__(16) C sc[4 * (kBatchThreads + 64)];
    __shared__ __align__(16) C tab[kBatchTab];
    __shared__ double lsum[TR ? 2 * 64 : 1];
    __shared__ double acc[TR ? 2 * kMaxBatchSub : 1];
    const BItem it = items[blockIdx.x];
    const BDomain& d = doms[it.dom];
    const SweepShape q = sweep_shape(d, it.axis);
    const int lpw = it.lpw;
    const int64_t tpo = (q.inner + lpw - 1) / lpw;   // tiles per outer index
    const T* in = static_cast<const T*>(d.buf[it.in]);
    T* out = static_cast<T*>(d.buf[it.out]);
    const T* xf = TR ? static_cast<const T*>(d.buf[it.xb]) : nullptr;
    const C* invd = static_cast<const C*>(d.invd[it.axis]);
    const C* rr = static_cast<const C*>(d.r[it.axis]);
    const int nS = (int)(q.n * d.S);   // <= kBatchTab (checked when the batch is created)
    for (int e = threadIdx.x; e < nS; e += blockDim.x) tab[e] = invd[e];
    if (TR)
        for (int sub = threadIdx.x; sub < d.S; sub += blockDim.x) acc[2 * sub] = acc[2 * sub + 1] = 0.0;
    __syncthreads();
    const FastDiv dS((uint32_t)d.S);
    // tile t = oy * tpo + ox, stepped without a division per tile
    uint32_t oy = (uint32_t)(it.a0 / tpo), ox = (uint32_t)(it.a0 - (int64_t)oy * tpo);
    for (int64_t t = it.a0; t < it.a1; ++t) {
        batch_tile<T, C, M, TR>(in, out, q, d.S, dS, lpw, ox, oy, tab, rr, sc, xf, lsum, acc);
        if (++ox == (uint32_t)tpo) {
            ox = 0;
            ++oy;
        }
    }
    if (TR)
        for (int sub = threadIdx.x; sub < d.S; sub += blockDim.x) {
            partials[it.slot + 2 * sub + 0] = acc[2 * sub + 0];
            partials[it.slot + 2 * sub + 1] = acc[2 * sub + 1];
        }
}

// One block per item of one sparse stage (source, Dirichlet, mask, copy) of
// one storage type.
__global__ __launch_bounds__(kBatchThreads) void k_group_sparse(const BDomain* __restrict__ doms,
                                                                const BItem* __restrict__ items)
{
    const BItem it = items[blockIdx.x];
    const BDomain& d = doms[it.dom];
    if (d.dtype == DT_F64) batch_sparse_item<double>(d, it);
    else batch_sparse_item<float>(d, it);
}

// ------------------------------------------------- persistent mode (off)

__global__ void k_batch_reset(uint32_t* counters, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        counters[i] = 0;
}

// counters[0] = queue head, counters[1] = error flag, counters[2 + c] = stage
// counters; all in uncached device memory (see CounterPool).
// At least 4 waves per SIMD (two 512-thread blocks per CU): every variant
// must fit 128 VGPRs.
__global__ __launch_bounds__(kBatchThreads, 4) void k_batch(const BDomain* __restrict__ doms,
                                                         const BItem* __restrict__ items, int64_t nitems,
                                                         uint32_t* counters, double* partials,
                                                         uint64_t limit_ticks)
{
    __shared__ __align__(16) double sc[4 * (kBatchThreads + 64)];   // carry arrays
    __shared__ double lsum[2 * 64];
    __shared__ double acc[2 * kMaxBatchSub];
    __shared__ int64_t s_item;
    uint32_t* head = counters;
    uint32_t* err = counters + 1;
    uint32_t* cnt = counters + 2;
    for (;;) {
        if (threadIdx.x == 0)
            s_item = (int64_t)__hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int64_t idx = s_item;
        __syncthreads();
        if (idx >= nitems) break;
        const BItem it = items[idx];
        if (threadIdx.x == 0 && it.dep >= 0) {
            // Wait (bounded in wall-clock time) for the previous stage of this
            // domain.  The counters live in uncached memory, so plain polls
            // read memory; one acquire fence follows a successful wait.  Once
            // any wait has failed, no block waits again.
            const uint64_t t0 = wall_clock64();
            bool ok = true;
            while (__hip_atomic_load(&cnt[it.dep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < it.need) {
                if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = false; break; }
                __builtin_amdgcn_s_sleep(2);
                if (wall_clock64() - t0 > limit_ticks) {
                    __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = false;
                    break;
                }
            }
            if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        const BDomain& d = doms[it.dom];
        if (it.type == ST_SWEEP || it.type == ST_SWEEP_T) {
            const bool tr = it.type == ST_SWEEP_T;
            if (d.dtype == DT_F64) {
                if (tr) batch_sweep_item<double, double, true>(d, it, sc, lsum, acc, partials);
                else batch_sweep_item<double, double, false>(d, it, sc, lsum, acc, partials);
            } else if (d.dtype == DT_F32) {
                if (tr) batch_sweep_item<float, double, true>(d, it, sc, lsum, acc, partials);
                else batch_sweep_item<float, double, false>(d, it, sc, lsum, acc, partials);
            } else {
                float* scf = reinterpret_cast<float*>(sc);
                if (tr) batch_sweep_item<float, float, true>(d, it, scf, lsum, acc, partials);
                else batch_sweep_item<float, float, false>(d, it, scf, lsum, acc, partials);
            }
        } else {
            if (d.dtype == DT_F64) batch_sparse_item<double>(d, it);
            else batch_sparse_item<float>(d, it);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            // publish the item's writes (L2 write-back), then count it
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(&cnt[it.done], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}


}  // namespace bfvm

// ===================================================================== host

using namespace bfvm;

namespace {

int bfail(int code, const std::string& msg)
{
    set_error(msg);
    return code;
}

#define BHIP(expr, what)                                                                   \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess) return bfail(BFVM_EDEVICE, std::string(what) + ": " + hipGetErrorString(_e)); \
    } while (0)

// The single-launch persistent mode is switched off: on gfx950 its
// dependency waits did not complete (see the file header).  Its scheduler is
// kept so that it can be re-enabled once the cause is known.
constexpr bool kPersistentModeEnabled = false;

struct Program : ProgramLayout {
    BItem* d_items = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // members outside the grouped kernels' limits, run with their own grid's
    // launches: one step (forward program) or one reverse step (adjoint)
    std::vector<int32_t> big;
    bool reverse = false;
};

void drop_graph(Program& P)
{
    if (P.exec) (void)hipGraphExecDestroy(P.exec);
    if (P.graph) (void)hipGraphDestroy(P.graph);
    P.exec = nullptr;
    P.graph = nullptr;
}

void free_program(Program& P)
{
    drop_graph(P);
    if (P.d_items) (void)hipFree(P.d_items);
    P.d_items = nullptr;
    P.items.clear();
    P.launches.clear();
    P.big.clear();
}

// Whether the grouped kernels can take a domain: lines of at most
// kMaxBatchLine voxels (K = 512 / 16 segments of at most 16 elements), an
// [n][S] coefficient table of at most kBatchTab entries per axis (staged in
// LDS), at most kMaxBatchSub substrates (the reverse step's per-substrate
// sums are kept in LDS) and 32-bit element offsets.
bool group_fits(bfvm_grid g)
{
    for (int a = 0; a < 3; ++a) {
        const int64_t n = a == 0 ? g->nx : (a == 1 ? g->ny : g->nz);
        if (n > kMaxBatchLine || n * g->S > kBatchTab) return false;
    }
    return g->S <= kMaxBatchSub && g->nelem() < (1ll << 31);
}

}  // namespace

struct bfvm_batch_s {
    std::vector<bfvm_grid> grids;
    std::vector<uint64_t> gens;       // each grid's setter count when its descriptor was last read
    std::vector<BDomain> doms;        // host copy of the descriptors
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // side streams and events of the per-storage-type chains (grouped mode);
    // side[2] carries the members the grouped kernels cannot take
    hipStream_t side[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[3] = {nullptr, nullptr, nullptr};
    std::vector<uint8_t> large;       // 1: member runs its own grid's launches
    int mode = BFVM_BATCH_GROUPED;
    BDomain* d_doms = nullptr;
    int64_t chunk_elems = 1 << 14;    // work per item
    int blocks = 0;                   // persistent grid size
    uint64_t wait_ticks = 0;          // bound of one dependency wait (wall-clock ticks)
    Program fwd;                      // one step of every domain
    Program adj;                      // one reverse step of adj_subset
    std::vector<int32_t> adj_subset;
    double* d_partials = nullptr;
    int64_t partials_cap = 0;
    uint32_t* d_counters = nullptr;   // persistent mode only
    int64_t counters_cap = 0;
    void* work_mem = nullptr;         // adjoint workspace of the subset
};

namespace {

void build_program(bfvm_batch b, const std::vector<int32_t>& which, const std::vector<Stage>& prog, Program& P)
{
    build_layout(b->doms, b->chunk_elems, which, prog, P);
}

// Counters that blocks of one launch use to hand work to each other must be
// coherent across the GPU's XCDs while the kernel runs, so they are taken
// from uncached device memory.  Uncached allocations are never freed (a
// freed uncached block can corrupt later allocations): they come from a
// grow-only, process-lifetime bump pool.  Persistent mode only.
struct CounterPool {
    uint32_t* chunk = nullptr;
    size_t used = 0, cap = 0;
};

int counters_from_pool(int64_t n, uint32_t** out)
{
    static CounterPool pool;
    const size_t need = ((size_t)n * sizeof(uint32_t) + 255) & ~(size_t)255;
    if (!pool.chunk || pool.used + need > pool.cap) {
        const size_t cap = std::max<size_t>(need, (size_t)4 << 20);
        void* p = nullptr;
        BHIP(hipExtMallocWithFlags(&p, cap, hipDeviceMallocUncached), "uncached counter allocation");
        pool.chunk = static_cast<uint32_t*>(p);   // any previous chunk stays allocated
        pool.used = 0;
        pool.cap = cap;
    }
    *out = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(pool.chunk) + pool.used);
    pool.used += need;
    return BFVM_OK;
}

int ensure_counters(bfvm_batch b, int64_t n)
{
    if (b->counters_cap >= n) return BFVM_OK;
    drop_graph(b->fwd);   // captured programs hold the old pointer
    drop_graph(b->adj);
    uint32_t* c = nullptr;
    if (int st = counters_from_pool(n, &c)) return st;
    b->d_counters = c;
    b->counters_cap = n;
    return BFVM_OK;
}

int upload_doms(bfvm_batch b)
{
    BHIP(hipMemcpyAsync(b->d_doms, b->doms.data(), sizeof(BDomain) * b->doms.size(), hipMemcpyHostToDevice,
                        b->stream), "upload descriptors");
    BHIP(hipStreamSynchronize(b->stream), "sync");
    return BFVM_OK;
}

int upload_program(bfvm_batch b, Program& P)
{
    drop_graph(P);
    if (P.d_items) (void)hipFree(P.d_items);
    P.d_items = nullptr;
    BHIP(hipMalloc((void**)&P.d_items, sizeof(BItem) * std::max<size_t>(1, P.items.size())), "hipMalloc items");
    if (!P.items.empty())
        BHIP(hipMemcpy(P.d_items, P.items.data(), sizeof(BItem) * P.items.size(), hipMemcpyHostToDevice),
             "upload items");
    if (b->mode == BFVM_BATCH_PERSISTENT) return ensure_counters(b, 2 + P.ncounters);
    return BFVM_OK;
}

int build_forward(bfvm_batch b)
{
    // the tile plans, the chunk size or the mode may have changed: the
    // adjoint program is rebuilt on its next call as well
    free_program(b->adj);
    b->adj_subset.clear();
    std::vector<int32_t> small, big;
    for (size_t i = 0; i < b->doms.size(); ++i) (b->large[i] ? big : small).push_back((int32_t)i);
    build_program(b, small, forward_program(), b->fwd);
    b->fwd.big = big;
    b->fwd.reverse = false;
    return upload_program(b, b->fwd);
}

template <typename T, typename C, bool TR>
void launch_group_sweep(int M, int64_t n, hipStream_t s, const BDomain* d, const BItem* it, double* partials)
{
    const dim3 grid((unsigned)n), block(kBatchThreads);
    switch (M) {
        case 4: hipLaunchKernelGGL((k_group_sweep<T, C, 4, TR>), grid, block, 0, s, d, it, partials); break;
        case 8: hipLaunchKernelGGL((k_group_sweep<T, C, 8, TR>), grid, block, 0, s, d, it, partials); break;
        case 12: hipLaunchKernelGGL((k_group_sweep<T, C, 12, TR>), grid, block, 0, s, d, it, partials); break;
        default: hipLaunchKernelGGL((k_group_sweep<T, C, 16, TR>), grid, block, 0, s, d, it, partials); break;
    }
}

// enqueue one run of a program on the batch stream
int enqueue_program(bfvm_batch b, const Program& P)
{
    if (b->mode == BFVM_BATCH_PERSISTENT) {
        if (!P.big.empty()) return bfail(BFVM_ESTATE, "the persistent mode takes no members beyond the grouped limits");
        const int64_t nreset = 2 + P.ncounters;
        hipLaunchKernelGGL(k_batch_reset, dim3((unsigned)std::min<int64_t>((nreset + 255) / 256, 1024)), dim3(256),
                           0, b->stream, b->d_counters, nreset);
        BHIP(hipGetLastError(), "batch reset kernel");
        hipLaunchKernelGGL(k_batch, dim3(b->blocks), dim3(kBatchThreads), 0, b->stream, b->d_doms, P.d_items,
                           (int64_t)P.items.size(), b->d_counters, b->d_partials, b->wait_ticks);
        BHIP(hipGetLastError(), "batch kernel");
        return BFVM_OK;
    }
    // Every launch covers domains of one storage type only, and every item
    // touches its own domain's buffers (and its own reduction slots), so the
    // launches of each storage type form an independent chain.  The chains
    // run on their own streams, forked from and joined back into the batch
    // stream (also under graph capture, where they become parallel branches),
    // so that one chain's small or draining launches overlap the other's.
    int chain_of[3] = {-1, -1, -1};
    int nchain = 0;
    for (const Launch& L : P.launches)
        if (chain_of[L.dtype] < 0) chain_of[L.dtype] = nchain++;
    const hipStream_t cs[3] = {b->stream, b->side[0], b->side[1]};
    const bool big = !P.big.empty();
    if (nchain > 1 || big) BHIP(hipEventRecord(b->ev_fork, b->stream), "fork event");
    for (int c = 1; c < nchain; ++c) BHIP(hipStreamWaitEvent(cs[c], b->ev_fork, 0), "fork wait");
    // Members beyond the grouped kernels' limits run their own grid's
    // kernels (plain schedule, the grid's plans), one after another on a
    // chain of their own beside the grouped chains.
    if (big) {
        BHIP(hipStreamWaitEvent(b->side[2], b->ev_fork, 0), "fork wait");
        for (int32_t i : P.big) {
            bfvm_grid g = b->grids[i];
            const BDomain& d = b->doms[i];
            int st;
            if (!P.reverse) {
                st = enqueue_step(g, d.buf[0], b->side[2]);
            } else {
                OnStream on(g, b->side[2]);
                st = adjoint_enqueue(g, d.buf[0], d.buf[1], g->work, g->red_partials, g->red_out);
            }
            if (st) return st;
        }
    }
    for (const Launch& L : P.launches) {
        const BItem* it = P.d_items + L.off;
        const hipStream_t s = cs[chain_of[L.dtype]];
        double* pt = b->d_partials;
        if (!L.sweep) {
            hipLaunchKernelGGL(k_group_sparse, dim3((unsigned)L.count), dim3(kBatchThreads), 0, s, b->d_doms, it);
        } else if (L.dtype == BFVM_F64) {
            if (L.tr) launch_group_sweep<double, double, true>(L.M, L.count, s, b->d_doms, it, pt);
            else launch_group_sweep<double, double, false>(L.M, L.count, s, b->d_doms, it, pt);
        } else if (L.dtype == BFVM_F32) {
            if (L.tr) launch_group_sweep<float, double, true>(L.M, L.count, s, b->d_doms, it, pt);
            else launch_group_sweep<float, double, false>(L.M, L.count, s, b->d_doms, it, pt);
        } else {
            if (L.tr) launch_group_sweep<float, float, true>(L.M, L.count, s, b->d_doms, it, pt);
            else launch_group_sweep<float, float, false>(L.M, L.count, s, b->d_doms, it, pt);
        }
        BHIP(hipGetLastError(), "grouped stage kernel");
    }
    for (int c = 1; c < nchain; ++c) {
        BHIP(hipEventRecord(b->ev_join[c - 1], cs[c]), "join event");
        BHIP(hipStreamWaitEvent(b->stream, b->ev_join[c - 1], 0), "join wait");
    }
    if (big) {
        BHIP(hipEventRecord(b->ev_join[2], b->side[2]), "join event");
        BHIP(hipStreamWaitEvent(b->stream, b->ev_join[2], 0), "join wait");
    }
    return BFVM_OK;
}

int capture(bfvm_batch b, Program& P)
{
    drop_graph(P);
    BHIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    int st = enqueue_program(b, P);
    hipGraph_t graph = nullptr;
    hipError_t ee = hipStreamEndCapture(b->stream, &graph);
    if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (ee != hipSuccess) return bfail(BFVM_EDEVICE, std::string("end capture: ") + hipGetErrorString(ee));
    P.graph = graph;
    BHIP(hipGraphInstantiate(&P.exec, graph, nullptr, nullptr, 0), "graph instantiate");
    return BFVM_OK;
}

// wait for the batch stream; in persistent mode also check the error flag
int finish(bfvm_batch b)
{
    if (b->mode == BFVM_BATCH_PERSISTENT) {
        uint32_t flag = 0;
        BHIP(hipMemcpyAsync(&flag, b->d_counters + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, b->stream),
             "read flag");
        BHIP(hipStreamSynchronize(b->stream), "sync");
        if (flag) return bfail(BFVM_EDEVICE, "batch dependency wait exceeded its time limit (2 s)");
        return BFVM_OK;
    }
    BHIP(hipStreamSynchronize(b->stream), "sync");
    return BFVM_OK;
}

int refresh_from_grids(bfvm_batch b)
{
    for (size_t i = 0; i < b->grids.size(); ++i) {
        bfvm_grid g = b->grids[i];
        BDomain& d = b->doms[i];
        d.dtype = g->dtype;
        d.S = g->S;
        d.nx = g->nx;
        d.ny = g->ny;
        d.nz = g->nz;
        const bool f32c = g->dtype == BFVM_F32_FAST;
        for (int a = 0; a < 3; ++a) {
            d.invd[a] = f32c ? (const void*)g->invd32[a] : (const void*)g->invd64[a];
            d.r[a] = f32c ? (const void*)g->r32[a] : (const void*)g->r64[a];
        }
        d.src_vox = g->src_vox;
        d.src_P = g->src_P;
        d.src_invQ = g->src_invQ;
        d.nsrc = g->nsrc;
        d.dir_elem = g->dir_elem;
        d.dir_val = g->dir_val;
        d.ndir = g->ndir;
        b->gens[i] = g->gen;
    }
    return BFVM_OK;
}

// A member grid's setters free and reallocate its coefficient tables and
// source / Dirichlet lists (and may change their lengths), which the device
// descriptors and the captured programs point to.  Before every call that
// runs work, re-read any grid whose setter count moved, then rebuild the
// programs; the graphs are captured again on their next run.
int sync_grids(bfvm_batch b)
{
    bool moved = false;
    for (size_t i = 0; i < b->grids.size(); ++i) moved |= b->grids[i]->gen != b->gens[i];
    if (!moved) return BFVM_OK;
    refresh_from_grids(b);
    if (int st = upload_doms(b)) return st;
    return build_forward(b);
}

}  // namespace

// ====================================================================== ABI

extern "C" {

int bfvm_batch_create(bfvm_batch* out, int32_t ndomains, const bfvm_grid* grids, void* const* fields, void* stream)
{
    if (!out) return bfail(BFVM_EINVAL, "out is NULL");
    *out = nullptr;
    if (ndomains < 1 || !grids || !fields) return bfail(BFVM_EINVAL, "need >= 1 grid and field");
    for (int32_t i = 0; i < ndomains; ++i) {
        if (!grids[i] || !fields[i]) return bfail(BFVM_EINVAL, "NULL grid or field");
        if (!grids[i]->have_params) return bfail(BFVM_ESTATE, "every grid needs set_params first");
        // a member beyond the grouped limits runs with its grid's own
        // reverse-step workspace, so that grid may hold one member only
        if (!group_fits(grids[i]))
            for (int32_t j = 0; j < ndomains; ++j)
                if (j != i && grids[j] == grids[i])
                    return bfail(BFVM_EINVAL, "a grid beyond the grouped limits appears twice in the batch");
    }
    bfvm_batch b = new (std::nothrow) bfvm_batch_s();
    if (!b) return bfail(BFVM_ENOMEM, "host allocation failed");
    b->stream = static_cast<hipStream_t>(stream);
    if (!b->stream) {   // the legacy null stream cannot be captured into a graph
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return bfail(BFVM_EDEVICE, "hipStreamCreateWithFlags");
        }
        b->own_stream = true;
    }
    for (int c = 0; c < 3; ++c) {   // default priority, like the batch stream
        if (hipStreamCreateWithFlags(&b->side[c], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->ev_join[c], hipEventDisableTiming) != hipSuccess) {
            bfvm_batch_destroy(b);
            return bfail(BFVM_EDEVICE, "side stream or event creation");
        }
    }
    if (hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess) {
        bfvm_batch_destroy(b);
        return bfail(BFVM_EDEVICE, "fork event creation");
    }
    b->grids.assign(grids, grids + ndomains);
    b->gens.assign(ndomains, 0);
    b->large.resize(ndomains);
    for (int32_t i = 0; i < ndomains; ++i) b->large[i] = group_fits(grids[i]) ? 0 : 1;
    b->doms.resize(ndomains);
    std::memset(b->doms.data(), 0, sizeof(BDomain) * ndomains);
    refresh_from_grids(b);
    for (int32_t i = 0; i < ndomains; ++i) {
        b->doms[i].buf[0] = fields[i];
        default_batch_plan(b->doms[i], b->mode);
    }
    int dev = 0, cus = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch, kBatchThreads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    b->blocks = cus * per_cu;
    int rate_khz = 0;   // wall_clock64() frequency
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || rate_khz <= 0)
        rate_khz = 100000;
    b->wait_ticks = (uint64_t)rate_khz * 1000ull * 2ull;   // 2 s per dependency wait
    int st = BFVM_OK;
    hipError_t e = hipMalloc((void**)&b->d_doms, sizeof(BDomain) * ndomains);
    if (e != hipSuccess) st = bfail(BFVM_ENOMEM, "hipMalloc descriptors");
    if (!st) st = upload_doms(b);
    if (!st) st = build_forward(b);
    if (st) {
        bfvm_batch_destroy(b);
        return st;
    }
    *out = b;
    return BFVM_OK;
}

int bfvm_batch_destroy(bfvm_batch b)
{
    if (!b) return BFVM_OK;
    (void)hipStreamSynchronize(b->stream);
    free_program(b->fwd);
    free_program(b->adj);
    if (b->d_doms) (void)hipFree(b->d_doms);
    if (b->d_partials) (void)hipFree(b->d_partials);
    // d_counters is a slice of the uncached pool: never freed
    if (b->work_mem) (void)hipFree(b->work_mem);
    for (int c = 0; c < 3; ++c) {
        if (b->side[c]) {
            (void)hipStreamSynchronize(b->side[c]);
            (void)hipStreamDestroy(b->side[c]);
        }
        if (b->ev_join[c]) (void)hipEventDestroy(b->ev_join[c]);
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return BFVM_OK;
}

int bfvm_batch_set_mode(bfvm_batch b, int32_t mode)
{
    if (!b) return bfail(BFVM_EINVAL, "batch is NULL");
    if (mode != BFVM_BATCH_GROUPED && mode != BFVM_BATCH_PERSISTENT) return bfail(BFVM_EINVAL, "unknown mode");
    if (mode == BFVM_BATCH_PERSISTENT && !kPersistentModeEnabled)
        return bfail(BFVM_EOFF, "the single-launch persistent mode is switched off: its cross-block "
                                "dependency waits did not complete on gfx950");
    if (mode == b->mode) return BFVM_OK;
    b->mode = mode;
    for (auto& d : b->doms) default_batch_plan(d, mode);
    if (int st = upload_doms(b)) return st;
    return build_forward(b);
}

int bfvm_batch_set_fields(bfvm_batch b, int32_t which, void* const* ptrs)
{
    if (!b) return bfail(BFVM_EINVAL, "batch is NULL");
    if ((which != 0 && which != 1) || !ptrs) return bfail(BFVM_EINVAL, "which must be 0 (field) or 1 (gradient)");
    for (size_t i = 0; i < b->doms.size(); ++i)
        if (which == 0 && !ptrs[i]) return bfail(BFVM_EINVAL, "NULL field");
    // the grouped kernels read the pointers from the device descriptors;
    // the launches of members beyond the grouped limits carry them as
    // kernel arguments, so their graphs are captured again
    bool recapture = false;
    for (size_t i = 0; i < b->doms.size(); ++i) {
        recapture |= b->large[i] && b->doms[i].buf[which] != ptrs[i];
        b->doms[i].buf[which] = ptrs[i];
    }
    if (recapture) {
        drop_graph(b->fwd);
        drop_graph(b->adj);
    }
    return upload_doms(b);
}

int bfvm_batch_step(bfvm_batch b, int64_t nsteps)
{
    if (!b) return bfail(BFVM_EINVAL, "batch is NULL");
    if (nsteps < 0) return bfail(BFVM_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return BFVM_OK;
    if (int st = sync_grids(b)) return st;
    if (!b->fwd.exec)
        if (int st = capture(b, b->fwd)) return st;
    for (int64_t t = 0; t < nsteps; ++t) BHIP(hipGraphLaunch(b->fwd.exec, b->stream), "graph launch");
    return finish(b);
}

int bfvm_batch_step_eager(bfvm_batch b, int64_t nsteps)
{
    if (!b) return bfail(BFVM_EINVAL, "batch is NULL");
    if (nsteps < 0) return bfail(BFVM_EINVAL, "nsteps must be >= 0");
    if (int st = sync_grids(b)) return st;
    for (int64_t t = 0; t < nsteps; ++t)
        if (int st = enqueue_program(b, b->fwd)) return st;
    return finish(b);
}

int bfvm_batch_step_adjoint(bfvm_batch b, int32_t count, const int32_t* subset, double* grad_D, double* grad_lambda)
{
    if (!b) return bfail(BFVM_EINVAL, "batch is NULL");
    if (count < 1 || !subset || !grad_D || !grad_lambda) return bfail(BFVM_EINVAL, "bad subset or NULL");
    for (int32_t i = 0; i < count; ++i) {
        if (subset[i] < 0 || subset[i] >= (int32_t)b->doms.size()) return bfail(BFVM_ERANGE, "domain index");
        if (!b->doms[subset[i]].buf[1]) return bfail(BFVM_ESTATE, "set the gradient buffers first");
        for (int32_t j = 0; j < i; ++j)
            if (subset[j] == subset[i]) return bfail(BFVM_EINVAL, "repeated domain in subset");
    }
    if (int st = sync_grids(b)) return st;
    std::vector<int32_t> sub(subset, subset + count);
    if (sub != b->adj_subset) {
        // (re)build the adjoint program: workspace, items, partials, graph.
        // Members beyond the grouped limits run their grid's own reverse
        // step, in the grid's own workspace.
        free_program(b->adj);
        b->adj_subset.clear();
        if (b->work_mem) (void)hipFree(b->work_mem);
        b->work_mem = nullptr;
        std::vector<int32_t> small, big;
        for (int32_t i : sub) (b->large[i] ? big : small).push_back(i);
        for (int32_t i : big)
            if (int st = ensure_adjoint_workspace(b->grids[i])) return st;
        size_t total = 0;
        std::vector<size_t> off(small.size());
        for (size_t i = 0; i < small.size(); ++i) {
            const BDomain& d = b->doms[small[i]];
            off[i] = total;
            total += 3 * (size_t)(d.nx * d.ny * d.nz * d.S) * dtype_size(d.dtype);
            total = (total + 255) & ~(size_t)255;
        }
        if (total) BHIP(hipMalloc(&b->work_mem, total), "hipMalloc adjoint workspace");
        for (size_t i = 0; i < small.size(); ++i) {
            BDomain& d = b->doms[small[i]];
            const size_t nb = (size_t)(d.nx * d.ny * d.nz * d.S) * dtype_size(d.dtype);
            for (int k = 0; k < 3; ++k) d.buf[2 + k] = static_cast<char*>(b->work_mem) + off[i] + k * nb;
        }
        if (int st = upload_doms(b)) return st;
        build_program(b, small, adjoint_program(), b->adj);
        b->adj.big = big;
        b->adj.reverse = true;
        if (b->partials_cap < b->adj.npartials) {
            drop_graph(b->fwd);   // the forward graph holds the old partials pointer
            if (b->d_partials) (void)hipFree(b->d_partials);
            b->d_partials = nullptr;
            BHIP(hipMalloc((void**)&b->d_partials, sizeof(double) * std::max<int64_t>(1, b->adj.npartials)),
                 "hipMalloc partials");
            b->partials_cap = b->adj.npartials;
        }
        if (int st = upload_program(b, b->adj)) return st;
        b->adj_subset = sub;
    }
    if (!b->adj.exec)
        if (int st = capture(b, b->adj)) return st;
    BHIP(hipGraphLaunch(b->adj.exec, b->stream), "graph launch");
    if (int st = finish(b)) return st;
    std::vector<double> part(b->adj.npartials);
    if (!part.empty())
        BHIP(hipMemcpy(part.data(), b->d_partials, sizeof(double) * part.size(), hipMemcpyDeviceToHost),
             "read partials");
    // per domain of the subset (in subset order), per axis: sums in item order
    std::map<int32_t, int> pos;
    int64_t base = 0;
    std::vector<int64_t> first(count);
    for (int32_t i = 0; i < count; ++i) {
        pos[sub[i]] = i;
        first[i] = base;
        base += b->doms[sub[i]].S;
    }
    std::vector<double> Gr(base * 3, 0.0), Gb(base * 3, 0.0);
    for (const BItem& it : b->adj.items) {
        if (it.type != ST_SWEEP_T) continue;
        const int i = pos[it.dom];
        const int S = b->doms[it.dom].S;
        for (int s = 0; s < S; ++s) {
            Gr[(first[i] + s) * 3 + it.axis] += part[it.slot + 2 * s + 0];
            Gb[(first[i] + s) * 3 + it.axis] += part[it.slot + 2 * s + 1];
        }
    }
    for (int32_t i = 0; i < count; ++i) {
        bfvm_grid g = b->grids[sub[i]];
        if (b->large[sub[i]]) {
            // the grid's own reverse step left its sums in its red_out
            if (int st = adjoint_accumulate(g, g->red_out, b->stream, grad_D + first[i], grad_lambda + first[i]))
                return st;
            continue;
        }
        for (int s = 0; s < g->S; ++s)
            for (int a = 0; a < 3; ++a) {
                grad_D[first[i] + s] += -Gr[(first[i] + s) * 3 + a] * g->dt / (g->h[a] * g->h[a]);
                grad_lambda[first[i] + s] += -Gb[(first[i] + s) * 3 + a] * g->dt / 3.0;
            }
    }
    return BFVM_OK;
}

int bfvm_batch_get_plan(bfvm_batch b, int32_t domain, int32_t axis, int32_t* m, int32_t* lpw)
{
    if (!b || !m || !lpw) return bfail(BFVM_EINVAL, "NULL");
    if (domain < 0 || domain >= (int32_t)b->doms.size() || axis < 0 || axis > 2)
        return bfail(BFVM_ERANGE, "domain or axis");
    if (b->large[domain])
        return bfail(BFVM_ESTATE, "the domain runs its own grid's kernels: query its plan with bfvm_get_plan");
    *m = b->doms[domain].M[axis];
    *lpw = b->doms[domain].lpw[axis];
    return BFVM_OK;
}

int bfvm_batch_set_plan(bfvm_batch b, int32_t domain, int32_t axis, int32_t m, int32_t lpw)
{
    if (!b) return bfail(BFVM_EINVAL, "batch is NULL");
    if (domain < 0 || domain >= (int32_t)b->doms.size() || axis < 0 || axis > 2)
        return bfail(BFVM_ERANGE, "domain or axis");
    if (b->large[domain])
        return bfail(BFVM_ESTATE, "the domain runs its own grid's kernels: set its plan with bfvm_set_plan");
    if (m != 4 && m != 8 && m != 12 && m != 16) return bfail(BFVM_EINVAL, "m must be 4, 8, 12 or 16");
    if (m > max_m_for_mode(b->mode)) return bfail(BFVM_EINVAL, "m too large for the batch mode");
    if (lpw != 16 && lpw != 32 && lpw != 64) return bfail(BFVM_EINVAL, "lpw must be 16, 32 or 64");
    BDomain& d = b->doms[domain];
    if (!plan_fits(axis_len(d, axis), m, lpw)) return bfail(BFVM_EINVAL, "too few segments for the line length");
    if (int st = sync_grids(b)) return st;
    d.M[axis] = m;
    d.lpw[axis] = lpw;
    if (int st = upload_doms(b)) return st;
    return build_forward(b);
}

int bfvm_batch_info(bfvm_batch b, int64_t* items, int32_t* launches, int64_t* chunk_elems)
{
    if (!b || !items || !launches || !chunk_elems) return bfail(BFVM_EINVAL, "NULL");
    *items = (int64_t)b->fwd.items.size();
    *launches = b->mode == BFVM_BATCH_PERSISTENT ? 2 : (int32_t)b->fwd.launches.size();
    *chunk_elems = b->chunk_elems;
    return BFVM_OK;
}

}  // extern "C"

// ================================================================ autotuner
//
// Tunes, for the batch at hand, (1) the tile shape of every (axis, line
// length, substrate count, storage type) class: lines per tile lpw in
// {16, 32, 64} with the smallest elements-per-thread M in {4, 8, 12, 16} that
// still covers the line (K = 512 / lpw segments of M), and (2) the work
// per item.  Coordinate descent: for each axis, each lpw candidate is
// applied to every domain where it fits and the whole batch step is timed;
// then each chunk size.  Results are cached in a small JSON file keyed by
// the GPU architecture and the class, and reused when every class of the
// batch is present.

namespace {

std::string class_key(const BDomain& d, int axis)
{
    std::ostringstream o;
    o << axis << ":" << axis_len(d, axis) << ":" << d.S << ":" << d.dtype;
    return o.str();
}

double time_steps(bfvm_batch b, int reps, int* st)
{
    hipEvent_t e0, e1;
    *st = BFVM_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        *st = bfail(BFVM_EDEVICE, "event create");
        return 1e30;
    }
    *st = enqueue_program(b, b->fwd);   // warm-up
    (void)hipEventRecord(e0, b->stream);
    for (int r = 0; r < reps && !*st; ++r) *st = enqueue_program(b, b->fwd);
    (void)hipEventRecord(e1, b->stream);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!*st) *st = finish(b);
    return ms / reps;
}

// minimal JSON cache: {"arch": "...", "chunk": N, "plans": {"key": [M, lpw], ...}}
bool load_cache(const std::string& path, const std::string& arch, int64_t* chunk,
                std::map<std::string, std::pair<int, int>>* plans)
{
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    if (t.find("\"arch\": \"" + arch + "\"") == std::string::npos) return false;
    size_t c = t.find("\"chunk\": ");
    if (c == std::string::npos) return false;
    *chunk = std::atoll(t.c_str() + c + 9);
    size_t p = t.find("\"plans\": {");
    if (p == std::string::npos) return false;
    p += 10;
    while (true) {
        const size_t q0 = t.find('"', p);
        if (q0 == std::string::npos) break;
        const size_t q1 = t.find('"', q0 + 1);
        const size_t b0 = t.find('[', q1);
        const size_t b1 = t.find(']', b0);
        if (q1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos) break;
        int m = 0, l = 0;
        if (std::sscanf(t.c_str() + b0, "[%d, %d]", &m, &l) == 2) (*plans)[t.substr(q0 + 1, q1 - q0 - 1)] = {m, l};
        p = b1 + 1;
    }
    return *chunk > 0;
}

void save_cache(const std::string& path, const std::string& arch, int64_t chunk,
                const std::map<std::string, std::pair<int, int>>& plans)
{
    std::ofstream f(path);
    if (!f) return;
    f << "{\"arch\": \"" << arch << "\", \"chunk\": " << chunk << ", \"plans\": {";
    bool first = true;
    for (auto& kv : plans) {
        f << (first ? "" : ", ") << "\"" << kv.first << "\": [" << kv.second.first << ", " << kv.second.second << "]";
        first = false;
    }
    f << "}}\n";
}

bool plan_ok(int mode, int64_t n, int m, int lpw)
{
    bool known_m = false;
    for (int k : kBatchM) known_m |= (k == m && m <= max_m_for_mode(mode));
    return known_m && (lpw == 16 || lpw == 32 || lpw == 64) && plan_fits(n, m, lpw);
}

}  // namespace

extern "C" int bfvm_batch_autotune(bfvm_batch b, const char* cache_path, double* best_ms)
{
    if (!b || !best_ms) return bfail(BFVM_EINVAL, "NULL");
    if (int st = sync_grids(b)) return st;
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    arch += b->mode == BFVM_BATCH_PERSISTENT ? "/persistent" : "/grouped";
    std::map<std::string, std::pair<int, int>> cached;
    int64_t chunk = 0;
    int st = BFVM_OK;
    if (cache_path && load_cache(cache_path, arch, &chunk, &cached)) {
        bool all = true;
        for (size_t i = 0; i < b->doms.size(); ++i)
            for (int a = 0; a < 3 && !b->large[i]; ++a) {
                const BDomain& d = b->doms[i];
                auto it = cached.find(class_key(d, a));
                if (it == cached.end() || !plan_ok(b->mode, axis_len(d, a), it->second.first, it->second.second))
                    all = false;
            }
        if (all) {
            for (size_t i = 0; i < b->doms.size(); ++i)
                for (int a = 0; a < 3 && !b->large[i]; ++a) {
                    BDomain& d = b->doms[i];
                    const auto pl = cached[class_key(d, a)];
                    d.M[a] = pl.first;
                    d.lpw[a] = pl.second;
                }
            b->chunk_elems = chunk;
            if ((st = upload_doms(b)) || (st = build_forward(b))) return st;
            *best_ms = time_steps(b, 3, &st);
            return st;
        }
    }
    if ((st = build_forward(b))) return st;
    double best = time_steps(b, 3, &st);
    if (st) return st;
    const int lps[] = {16, 32, 64};
    for (int a = 0; a < 3; ++a) {
        std::vector<BDomain> keep = b->doms;
        for (int l : lps) {
            std::vector<BDomain> trial = keep;
            for (size_t i = 0; i < trial.size(); ++i) {
                if (b->large[i]) continue;
                BDomain& d = trial[i];
                const int m = smallest_m(axis_len(d, a), l, max_m_for_mode(b->mode));
                if (m) {
                    d.M[a] = m;
                    d.lpw[a] = l;
                }
            }
            b->doms = trial;
            if ((st = upload_doms(b)) || (st = build_forward(b))) return st;
            const double t = time_steps(b, 3, &st);
            if (st) return st;
            if (t < best) {
                best = t;
                keep = trial;
            }
        }
        b->doms = keep;
    }
    const int64_t chunks[] = {1 << 12, 1 << 13, 1 << 14, 1 << 15, 1 << 16, 1 << 17};
    int64_t best_chunk = b->chunk_elems;
    for (int64_t c : chunks) {
        b->chunk_elems = c;
        if ((st = upload_doms(b)) || (st = build_forward(b))) return st;
        const double t = time_steps(b, 3, &st);
        if (st) return st;
        if (t < best) {
            best = t;
            best_chunk = c;
        }
    }
    b->chunk_elems = best_chunk;
    if ((st = upload_doms(b)) || (st = build_forward(b))) return st;
    if (cache_path) {
        for (size_t i = 0; i < b->doms.size(); ++i)
            for (int a = 0; a < 3 && !b->large[i]; ++a) cached[class_key(b->doms[i], a)] = {b->doms[i].M[a], b->doms[i].lpw[a]};
        save_cache(cache_path, arch, best_chunk, cached);
    }
    *best_ms = best;
    return BFVM_OK;
}
