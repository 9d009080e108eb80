// Plan autotuning for one grid.  A measurement utility around the method,
// not part of it: every valid plan of a candidate set is timed on the
// caller's field with HIP events on the grid's stream, and each axis keeps
// its fastest plan.  The candidates span the kernels of every plan kind:
// LDS row tiles (plain and pipelined) and row lines for x, strided tiles of
// 16, 32 or 64 lines for y and z, each with 8, 16 or 32 elements per
// thread and as few segments as cover the line, and for y and z lines too
// long for one 512-thread block the two-part tiles.
#include <algorithm>
#include <string>
#include <vector>

#include "internal.hpp"

namespace {

int tune_fail(int code, const std::string& msg)
{
    bfvm::set_error(msg);
    return code;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

std::vector<bfvm::SweepPlan> candidates(int axis, const bfvm::AxisGeom& g)
{
    std::vector<bfvm::SweepPlan> out;
    auto add = [&](int kind, int m, int64_t w, int64_t lpw) {
        bfvm::SweepPlan p;
        p.kind = kind;
        p.m = m;
        p.w = (int)w;
        p.lpw = (int)lpw;
        out.push_back(p);
    };
    if (axis == 0) {
        for (int M : {8, 16, 32}) {
            const int64_t per_row = cdiv(g.n, M) * g.S;
            for (int64_t R : {1, 2, 4, 8, 16}) {
                if (per_row * R > 512) break;
                const int64_t w = cdiv(per_row * R, 64);
                add(bfvm::PLAN_SEG_XTILE, M, w, R);
                if (M != 32) add(bfvm::PLAN_SEG_XPIPE, M, w, R);
            }
        }
        for (int M : {8, 16, 32})
            for (int lpw : {16, 32}) {
                const int spw = 64 / lpw;
                const int64_t K = cdiv(cdiv(g.n, M), spw) * spw;
                if (K * lpw / 64 <= 16) add(bfvm::PLAN_SEG_XROWS, M, K * lpw / 64, lpw);
            }
    } else {
        for (int M : {8, 16, 32})
            for (int lpw : {16, 32, 64}) {
                const int spw = 64 / lpw;
                const int64_t K = cdiv(cdiv(g.n, M), spw) * spw;
                if (K * lpw / 64 <= 16) add(bfvm::PLAN_SEG_STRIDED, M, K * lpw / 64, lpw);
            }
        // lines in two parts, 512-thread blocks
        for (int M : {16, 32})
            for (int lpw : {16, 32}) {
                const int64_t K = 512 / lpw;
                if (K * M < g.n && 2 * K * M >= g.n) add(bfvm::PLAN_SEG_HALVES, M, 8, lpw);
            }
    }
    return out;
}

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

int bfvm_autotune(bfvm_grid g, void* field, int32_t reps, float* best_ms)
{
    if (!g) return tune_fail(BFVM_EINVAL, "grid is NULL");
    if (!field) return tune_fail(BFVM_EINVAL, "field is NULL");
    if (reps < 1 || reps > 100) return tune_fail(BFVM_EINVAL, "reps must be in [1, 100]");
    if (!g->have_params) return tune_fail(BFVM_ESTATE, "set_params must come before autotune");
    Events ev;
    if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess)
        return tune_fail(BFVM_EDEVICE, "hipEventCreate");
    for (int axis = 0; axis < 3; ++axis) {
        const bfvm::AxisGeom geo = bfvm::axis_geom(axis, g->nx, g->ny, g->nz, g->S);
        const bfvm::SweepPlan keep = g->plan[axis];
        std::vector<bfvm::SweepPlan> cand = candidates(axis, geo);
        cand.insert(cand.begin(), keep);
        bfvm::SweepPlan best = keep;
        float best_t = 0.0f;
        bool have = false;
        for (const bfvm::SweepPlan& c : cand) {
            if (!bfvm::check_plan(c, geo, g->dtype).empty()) continue;
            g->plan[axis] = c;
            int st = bfvm_sweep(g, field, axis);   // warm-up (and the first use of the kernel)
            if (st) {
                g->plan[axis] = keep;
                return st;
            }
            if (hipEventRecord(ev.a, g->stream) != hipSuccess) return tune_fail(BFVM_EDEVICE, "hipEventRecord");
            for (int r = 0; r < reps && !st; ++r) st = bfvm_sweep(g, field, axis);
            if (st) {
                g->plan[axis] = keep;
                return st;
            }
            float ms = 0.0f;
            if (hipEventRecord(ev.b, g->stream) != hipSuccess || hipEventSynchronize(ev.b) != hipSuccess ||
                hipEventElapsedTime(&ms, ev.a, ev.b) != hipSuccess) {
                g->plan[axis] = keep;
                return tune_fail(BFVM_EDEVICE, "event timing");
            }
            ms /= (float)reps;
            if (!have || ms < best_t) {
                best = c;
                best_t = ms;
                have = true;
            }
        }
        g->plan[axis] = best;
        if (best_ms) best_ms[axis] = best_t;
    }
    return BFVM_OK;
}

// ------------------------------------------------------ field placement
//
// The sweep rate of one field depends on where its allocation lands in
// device memory: on 1000^3 x 4 FP64 fields allocated side by side, the same
// step took 38.4-38.6 ms on most allocations and 34.8-35.9 ms on one or two
// of five, and each allocation kept its rate when measured again.  A
// streaming in-place multiply ran at the same rate on all of them, so the
// difference lies in how the sweeps' many concurrent row and plane streams
// map onto the memory, not in the bytes moved.  The allocation is therefore
// chosen by measurement: candidates are allocated side by side, each is
// timed on one x, y and z sweep set, and the fastest is kept.

namespace {

// device memory to leave free while candidates are held
size_t placement_reserve(size_t total) { return std::max<size_t>(total / 16, (size_t)4 << 30); }

}  // namespace

int bfvm_field_alloc(bfvm_grid g, int32_t candidates, void** field, float* cand_ms)
{
    if (!g) return tune_fail(BFVM_EINVAL, "grid is NULL");
    if (!field) return tune_fail(BFVM_EINVAL, "field is NULL");
    *field = nullptr;
    if (candidates < 1 || candidates > 16) return tune_fail(BFVM_EINVAL, "candidates must be in [1, 16]");
    if (!g->have_params) return tune_fail(BFVM_ESTATE, "set_params must come before field_alloc");
    if (cand_ms)
        for (int i = 0; i < candidates; ++i) cand_ms[i] = -1.0f;
    const size_t bytes = (size_t)g->nelem() * bfvm::dtype_size(g->dtype);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return tune_fail(BFVM_EDEVICE, "hipMemGetInfo");
    const size_t reserve = placement_reserve(total_b);
    int n = candidates;
    while (n > 1 && (free_b < reserve || (size_t)n * bytes > free_b - reserve)) --n;
    std::vector<void*> bufs;
    for (int i = 0; i < n; ++i) {
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            break;
        }
        bufs.push_back(p);
    }
    if (bufs.empty()) return tune_fail(BFVM_ENOMEM, "device allocation of the field failed");
    auto release_all_but = [&](size_t keep) {
        (void)hipStreamSynchronize(g->stream);
        for (size_t i = 0; i < bufs.size(); ++i)
            if (i != keep) (void)hipFree(bufs[i]);
    };
    if (bufs.size() == 1) {
        *field = bufs[0];
        return BFVM_OK;
    }
    Events ev;
    if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess) {
        release_all_but(bufs.size());
        return tune_fail(BFVM_EDEVICE, "hipEventCreate");
    }
    size_t best = 0;
    float best_t = 0.0f;
    for (size_t i = 0; i < bufs.size(); ++i) {
        // bounded values (each sweep is a contraction), one warm-up set, one timed set
        hipError_t e = bfvm::launch_fill_uniform(g->dtype, bufs[i], g->nelem(), 7, 0, 0.0, 1.0, g->stream);
        int st = e == hipSuccess ? BFVM_OK : tune_fail(BFVM_EDEVICE, "fill kernel");
        for (int a = 0; a < 3 && !st; ++a) st = bfvm_sweep(g, bufs[i], a);
        if (!st && hipEventRecord(ev.a, g->stream) != hipSuccess) st = tune_fail(BFVM_EDEVICE, "hipEventRecord");
        for (int a = 0; a < 3 && !st; ++a) st = bfvm_sweep(g, bufs[i], a);
        float ms = 0.0f;
        if (!st && (hipEventRecord(ev.b, g->stream) != hipSuccess || hipEventSynchronize(ev.b) != hipSuccess ||
                    hipEventElapsedTime(&ms, ev.a, ev.b) != hipSuccess))
            st = tune_fail(BFVM_EDEVICE, "event timing");
        if (st) {
            release_all_but(bufs.size());
            return st;
        }
        if (cand_ms) cand_ms[i] = ms;
        if (i == 0 || ms < best_t) {
            best = i;
            best_t = ms;
        }
    }
    release_all_but(best);
    *field = bufs[best];
    return BFVM_OK;
}

int bfvm_field_free(void* field)
{
    if (!field) return BFVM_OK;
    hipError_t e = hipFree(field);
    if (e != hipSuccess) return tune_fail(BFVM_EDEVICE, std::string("hipFree: ") + hipGetErrorString(e));
    return BFVM_OK;
}
