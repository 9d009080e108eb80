// C ABI of the gfx950 diffusion-decay library: grid object, FP64 coefficient
// precompute, argument validation, step composition, adjoint step, timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace bfvm;

namespace bfvm {
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace bfvm

namespace {

int fail(int code, const std::string& msg)
{
    set_error(msg);
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(BFVM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                           \
    do {                                              \
        hipError_t _e = (expr);                       \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

template <typename P>
void dfree(P*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

template <typename P>
int dalloc_copy(P*& dst, const P* src, size_t count, hipStream_t st)
{
    dfree(dst);
    if (count == 0) return BFVM_OK;
    hipError_t e = hipMalloc((void**)&dst, count * sizeof(P));
    if (e != hipSuccess) {
        dst = nullptr;
        return fail(e == hipErrorOutOfMemory ? BFVM_ENOMEM : BFVM_EDEVICE,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    HIP_TRY(hipMemcpyAsync(dst, src, count * sizeof(P), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    return BFVM_OK;
}

bool finite_nonneg(const double* a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i]) || a[i] < 0.0) return false;
    return true;
}

// Thomas constants of the zero-flux matrix of one (axis, substrate):
// b_i = 1 + r + beta at both ends, 1 + 2r + beta inside, 1 + beta for n = 1,
// off-diagonals -r; denom_1 = b_1, denom_i = b_i - r^2 / denom_{i-1}
// (= b_i - a_i c'_{i-1} of App. A with a_i = -r, c'_{i-1} = -r / denom_{i-1}).
// Writes invd[i*S + s] = 1 / denom_i.
void thomas_constants(int64_t n, double r, double beta, int S, int s, double* invd)
{
    double prev_inv = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double diag = n == 1 ? 1.0 + beta
                                   : ((i == 0 || i == n - 1) ? 1.0 + r + beta : 1.0 + 2.0 * r + beta);
        const double denom = i == 0 ? diag : diag - r * r * prev_inv;
        prev_inv = 1.0 / denom;
        invd[i * S + s] = prev_inv;
    }
}

// Head length H of the exact compressed form of an axis's [n][S] table: the
// smallest H such that, for every substrate, slots H .. n-2 all equal slot H
// bit for bit; -1 when there is none short enough to pay (H + 2 >= n or
// H > kCompHeadMax).
const int kCompHeadMax = 512;

int comp_head(const std::vector<double>& invd, int64_t n, int S)
{
    if (n < 4) return -1;
    int H = 0;
    for (int s = 0; s < S; ++s) {
        int64_t h = n - 2;   // walk back from the last interior slot while equal to it
        const double c = invd[(n - 2) * S + s];
        while (h > 0 && invd[(h - 1) * S + s] == c) --h;
        H = std::max<int>(H, (int)h);
    }
    return (H + 2 < n && H <= kCompHeadMax) ? H : -1;
}

int merge_sources(bfvm_grid g)
{
    const int S = g->S;
    const int64_t cnt = (int64_t)g->raw_vox.size();
    std::vector<int64_t> order(cnt);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return g->raw_vox[a] < g->raw_vox[b]; });
    std::vector<int64_t> vox;
    std::vector<double> P, invQ;
    for (int64_t t = 0; t < cnt;) {
        const int64_t v = g->raw_vox[order[t]];
        std::vector<double> ps(S, 0.0), qs(S, 0.0);
        for (; t < cnt && g->raw_vox[order[t]] == v; ++t) {
            const int64_t k = order[t];
            for (int s = 0; s < S; ++s) {
                ps[s] += g->raw_sec[k * S + s] * g->raw_sat[k * S + s];
                qs[s] += g->raw_sec[k * S + s] + g->raw_upt[k * S + s];
            }
        }
        vox.push_back(v);
        for (int s = 0; s < S; ++s) {
            P.push_back(g->dt * ps[s]);
            invQ.push_back(1.0 / (1.0 + g->dt * qs[s]));
        }
    }
    int st;
    if ((st = dalloc_copy(g->src_vox, vox.data(), vox.size(), g->stream)) != BFVM_OK) return st;
    if ((st = dalloc_copy(g->src_P, P.data(), P.size(), g->stream)) != BFVM_OK) return st;
    if ((st = dalloc_copy(g->src_invQ, invQ.data(), invQ.size(), g->stream)) != BFVM_OK) return st;
    g->nsrc = (int64_t)vox.size();
    return BFVM_OK;
}

// ---------------------------------------------------------------- timing
void time_begin(bfvm_grid g, int stage, hipEvent_t* a)
{
    *a = nullptr;
    if (!g->timing) return;
    if (g->ev_pool.size() < 2) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            if (hipEventCreate(&e) == hipSuccess) g->ev_pool.push_back(e);
        }
    }
    if (g->ev_pool.size() < 2) return;
    *a = g->ev_pool.back();
    g->ev_pool.pop_back();
    (void)hipEventRecord(*a, g->stream);
    (void)stage;
}

void time_end(bfvm_grid g, int stage, hipEvent_t a, int64_t elems = 0)
{
    if (!g->timing || !a) return;
    g->stage_elems[stage] += elems;
    hipEvent_t b = g->ev_pool.back();
    g->ev_pool.pop_back();
    (void)hipEventRecord(b, g->stream);
    g->pending.push_back({stage, a, b});
}

void time_harvest(bfvm_grid g)
{
    if (g->pending.empty()) return;
    (void)hipStreamSynchronize(g->stream);
    for (auto& p : g->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g->stage_ms[p.stage] += ms;
            g->stage_count[p.stage] += 1;
        }
        g->ev_pool.push_back(p.a);
        g->ev_pool.push_back(p.b);
    }
    g->pending.clear();
}

// ------------------------------------------------------------ stage runs
int run_source(bfvm_grid g, void* u)
{
    if (g->nsrc == 0) return BFVM_OK;
    hipEvent_t a;
    time_begin(g, 0, &a);
    hipError_t e = launch_source(g->dtype, u, g->src_vox, g->src_P, g->src_invQ, g->nsrc, g->S, g->stream);
    time_end(g, 0, a);
    return e == hipSuccess ? BFVM_OK : hip_fail(e, "source kernel");
}

int run_dirichlet(bfvm_grid g, void* u)
{
    if (g->ndir == 0) return BFVM_OK;
    hipEvent_t a;
    time_begin(g, 1, &a);
    hipError_t e = launch_dirichlet(g->dtype, u, g->dir_elem, g->dir_val, g->ndir, g->stream);
    time_end(g, 1, a);
    return e == hipSuccess ? BFVM_OK : hip_fail(e, "dirichlet kernel");
}

int run_sweep_geo(bfvm_grid g, int axis, const AxisGeom& geo, const void* in, void* out, bool transposed,
                  const AdjSums& red = AdjSums())
{
    const bool f32c = g->dtype == BFVM_F32_FAST;
    const void* invd = f32c ? (const void*)g->invd32[axis] : (const void*)g->invd64[axis];
    const void* r = f32c ? (const void*)g->r32[axis] : (const void*)g->r64[axis];
    const void* comp = f32c ? (const void*)g->comp32[axis] : (const void*)g->comp64[axis];
    hipEvent_t a;
    time_begin(g, 2 + axis, &a);
    hipError_t e = launch_sweep(g->dtype, transposed, g->plan[axis], geo, in, out, invd, r, comp, g->comp_H[axis],
                                g->stream, red);
    time_end(g, 2 + axis, a, geo.n * geo.inner * geo.outer);
    return e == hipSuccess ? BFVM_OK : hip_fail(e, "sweep kernel");
}

int run_sweep(bfvm_grid g, int axis, const void* in, void* out, bool transposed, const AdjSums& red = AdjSums())
{
    return run_sweep_geo(g, axis, axis_geom(axis, g->nx, g->ny, g->nz, g->S), in, out, transposed, red);
}

// ------------------------------------------------------- fused schedules
// Slab size target for the fused schedules: a slab fits the 256 MB
// memory-side cache, so the second sweep of a pair could read the first
// sweep's output from it.  Measured on the 1000^3 x 4 grid, the smaller
// launches cost more than the reuse saves, so the automatic choice is the
// plain schedule; the fused ones stay selectable.
const int64_t kSlabTarget = 128ll << 20;

bool slab_plans_ok(bfvm_grid g)
{
    return g->plan[1].kind == PLAN_SEG_STRIDED && g->plan[2].kind == PLAN_SEG_STRIDED && g->nz <= 65535 &&
           g->ny <= 65535;
}

// resolved schedule and slab width
void resolve_schedule(bfvm_grid g, int* sched, int64_t* w)
{
    const int64_t col = g->ny * g->nz * (int64_t)g->S * (int64_t)dtype_size(g->dtype);
    int sc = g->schedule;
    if (sc < 0) sc = 0;
    if (sc == 1 && !slab_plans_ok(g)) sc = 0;
    if (sc == 2 && !(g->plan[0].kind == PLAN_SEG_XROWS && g->plan[1].kind == PLAN_SEG_STRIDED)) sc = 0;
    if (sc == 2) {
        const int64_t plane = g->nx * g->ny * (int64_t)g->S * (int64_t)dtype_size(g->dtype);
        int64_t wz = g->slab_w > 0 ? g->slab_w : std::max<int64_t>(1, kSlabTarget / std::max<int64_t>(plane, 1));
        *sched = sc;
        *w = std::min<int64_t>(wz, g->nz);
        return;
    }
    int64_t ww = g->slab_w;
    if (ww <= 0) {
        ww = std::max<int64_t>(1, kSlabTarget / std::max<int64_t>(col, 1));
        // prefer slabs whose width * S fills whole 16-line tiles
        for (int64_t c = ww; c >= 1; --c)
            if ((c * g->S) % 16 == 0) { ww = c; break; }
    }
    *sched = sc;
    *w = std::min<int64_t>(std::max<int64_t>(ww, 1), g->nx);
}

// Dirichlet entries regrouped by x-slab of width w (device copy)
int build_dir_slabs(bfvm_grid g, int64_t w)
{
    if (g->dir_slab_w == w && !g->dir_slab_off.empty()) return BFVM_OK;
    const int64_t nslab = (g->nx + w - 1) / w;
    const int S = g->S;
    int sc;
    int64_t wr;
    resolve_schedule(g, &sc, &wr);
    const bool zs = sc == 2;
    const int64_t nsl = zs ? (g->nz + w - 1) / w : nslab;
    std::vector<std::vector<int64_t>> idx(nsl);
    for (size_t i = 0; i < g->dir_elem_h.size(); ++i) {
        const int64_t v = g->dir_elem_h[i] / S;
        const int64_t c = zs ? v / (g->nx * g->ny) : v % g->nx;
        idx[c / w].push_back((int64_t)i);
    }
    std::vector<int64_t> el, off(nsl + 1, 0);
    std::vector<double> val;
    for (int64_t k = 0; k < nsl; ++k) {
        for (int64_t i : idx[k]) {
            el.push_back(g->dir_elem_h[i]);
            val.push_back(g->dir_val_h[i]);
        }
        off[k + 1] = (int64_t)el.size();
    }
    int st;
    if ((st = dalloc_copy(g->dir_elem_slab, el.data(), el.size(), g->stream))) return st;
    if ((st = dalloc_copy(g->dir_val_slab, val.data(), val.size(), g->stream))) return st;
    g->dir_slab_off = off;
    g->dir_slab_w = w;
    return BFVM_OK;
}

// Rebuild the per-slab Dirichlet lists when the resolved schedule is the
// fused one (called by the setters, so that a step never allocates).
int refresh_dir_slabs(bfvm_grid g)
{
    int sc;
    int64_t w;
    resolve_schedule(g, &sc, &w);
    if (sc != 1 && sc != 2) return BFVM_OK;
    return build_dir_slabs(g, w);
}

int run_dirichlet_slab(bfvm_grid g, void* u, int64_t k)
{
    const int64_t a0 = g->dir_slab_off[k], a1 = g->dir_slab_off[k + 1];
    if (a1 == a0) return BFVM_OK;
    hipEvent_t a;
    time_begin(g, 1, &a);
    hipError_t e = launch_dirichlet(g->dtype, u, g->dir_elem_slab + a0, g->dir_val_slab + a0, a1 - a0, g->stream);
    time_end(g, 1, a);
    return e == hipSuccess ? BFVM_OK : hip_fail(e, "dirichlet kernel");
}

// One step with x and y back to back on z-slabs: Src, Dir, then per z-slab
// X, Dir (slab entries), Y, then Dir, Z, Dir.  Rows and y lines stay inside
// a z-slab, so this is again the plain composition.
int run_step_zfused(bfvm_grid g, void* field, int64_t w)
{
    int st;
    if ((st = run_source(g, field))) return st;
    if ((st = run_dirichlet(g, field))) return st;
    int64_t k = 0;
    for (int64_t z0 = 0; z0 < g->nz; z0 += w, ++k) {
        const int64_t z1 = std::min(g->nz, z0 + w);
        if ((st = run_sweep_geo(g, 0, zslab_geom(0, g->nx, g->ny, g->nz, g->S, z0, z1), field, field, false)))
            return st;
        if ((st = run_dirichlet_slab(g, field, k))) return st;
        if ((st = run_sweep_geo(g, 1, zslab_geom(1, g->nx, g->ny, g->nz, g->S, z0, z1), field, field, false)))
            return st;
    }
    if ((st = run_dirichlet(g, field))) return st;
    if ((st = run_sweep(g, 2, field, field, false))) return st;
    return run_dirichlet(g, field);
}

// One step: Src, Dir, X, Dir, then per x-slab Y, Dir (slab entries), Z, then
// Dir.  Every Dirichlet entry is still overwritten after its y sweep and
// before its z sweep, and the y and z lines of a slab never leave it, so the
// result is that of Src, Dir, X, Dir, Y, Dir, Z, Dir.
int run_step_fused(bfvm_grid g, void* field, int64_t w)
{
    int st;
    if ((st = run_source(g, field))) return st;
    if ((st = run_dirichlet(g, field))) return st;
    if ((st = run_sweep(g, 0, field, field, false))) return st;
    if ((st = run_dirichlet(g, field))) return st;
    int64_t k = 0;
    for (int64_t x0 = 0; x0 < g->nx; x0 += w, ++k) {
        const int64_t x1 = std::min(g->nx, x0 + w);
        if ((st = run_sweep_geo(g, 1, slab_geom(1, g->nx, g->ny, g->nz, g->S, x0, x1), field, field, false)))
            return st;
        if ((st = run_dirichlet_slab(g, field, k))) return st;
        if ((st = run_sweep_geo(g, 2, slab_geom(2, g->nx, g->ny, g->nz, g->S, x0, x1), field, field, false)))
            return st;
    }
    return run_dirichlet(g, field);
}

int check_grid(bfvm_grid g)
{
    if (!g) return fail(BFVM_EINVAL, "grid is NULL");
    return BFVM_OK;
}

}  // namespace

namespace bfvm {

// per-line sums of the three axes: 2 doubles per line, axis by axis
int64_t adjoint_partials_count(bfvm_grid g)
{
    int64_t n = 0;
    for (int a = 0; a < 3; ++a) n += 2 * axis_lines(axis_geom(a, g->nx, g->ny, g->nz, g->S));
    return n;
}

// One plain-schedule step (source, then Dirichlet and a sweep per axis, then
// Dirichlet) on the grid's stream.
int run_plain_step(bfvm_grid g, void* field)
{
    int st;
    if ((st = run_source(g, field))) return st;
    for (int a = 0; a < 3; ++a) {
        if ((st = run_dirichlet(g, field))) return st;
        if ((st = run_sweep(g, a, field, field, false))) return st;
    }
    return run_dirichlet(g, field);
}

int enqueue_step(bfvm_grid g, void* field, hipStream_t s)
{
    OnStream on(g, s);
    return run_plain_step(g, field);
}

int ensure_adjoint_workspace(bfvm_grid g)
{
    const size_t bytes = (size_t)g->nelem() * dtype_size(g->dtype);
    for (int a = 0; a < 3; ++a) {
        if (!g->work[a]) {
            hipError_t e = hipMalloc(&g->work[a], bytes);
            if (e != hipSuccess) {
                g->work[a] = nullptr;
                return fail(BFVM_ENOMEM, std::string("adjoint workspace: ") + hipGetErrorString(e));
            }
        }
    }
    // per-line sums of the three axes side by side, summed by one final launch
    const int64_t np = adjoint_partials_count(g);
    if (!g->red_partials || g->red_count < np) {
        dfree(g->red_partials);
        HIP_TRY(hipMalloc((void**)&g->red_partials, sizeof(double) * np), "hipMalloc partials");
        g->red_count = np;
    }
    if (!g->red_out) HIP_TRY(hipMalloc((void**)&g->red_out, sizeof(double) * 2 * g->S * 3), "hipMalloc red_out");
    return BFVM_OK;
}

// The device part of one reverse step, enqueued on the grid's stream into
// caller-provided workspace: work[3] field buffers, partials
// (adjoint_partials_count doubles), red_out (6 S doubles, see
// adjoint_accumulate).  Allocates nothing and never waits for the device.
int adjoint_enqueue(bfvm_grid g, const void* field_in, void* grad, void* const work[3], double* partials,
                    double* red_out)
{
    const size_t bytes = (size_t)g->nelem() * dtype_size(g->dtype);
    const int S = g->S;
    hipStream_t st = g->stream;
    int rc;
    const bool f32c = g->dtype == BFVM_F32_FAST;
    const AxisGeom zgeo = axis_geom(2, g->nx, g->ny, g->nz, S);
    const void* zcomp = f32c ? (const void*)g->comp32[2] : (const void*)g->comp64[2];
    // The z recomputation and the z transposed sweep run as one kernel where
    // it applies: the z output is formed and consumed in registers.
    const bool fuse_z = adj_z_fusable(g->dtype, zgeo, zcomp, g->comp_H[2]);
    // forward recomputation: work[a] = output of sweep a (before the following
    // Dirichlet overwrite).  Without Dirichlet entries sweep a reads work[a-1]
    // directly; with them it runs on an overwritten copy, so that work[a-1]
    // keeps the sweep output the reduction needs.  Without sources either,
    // nothing changes the state before the x sweep, which then reads field_in
    // itself instead of a copy.
    if (g->nsrc == 0 && g->ndir == 0) {
        if ((rc = run_sweep(g, 0, field_in, work[0], false))) return rc;
    } else {
        HIP_TRY(hipMemcpyAsync(work[0], field_in, bytes, hipMemcpyDeviceToDevice, st), "copy");
        if ((rc = run_source(g, work[0]))) return rc;
        if ((rc = run_dirichlet(g, work[0]))) return rc;
        if ((rc = run_sweep(g, 0, work[0], work[0], false))) return rc;
    }
    // the fused z pass reads the y output with the Dirichlet values applied:
    // work[1] itself, or an overwritten copy in work[2]
    const void* zin = work[1];
    for (int a = 1; a < 3; ++a) {
        if (a == 2 && fuse_z) {
            if (g->ndir > 0) {
                HIP_TRY(hipMemcpyAsync(work[2], work[1], bytes, hipMemcpyDeviceToDevice, st), "copy");
                if ((rc = run_dirichlet(g, work[2]))) return rc;
                zin = work[2];
            }
            break;
        }
        if (g->ndir > 0) {
            HIP_TRY(hipMemcpyAsync(work[a], work[a - 1], bytes, hipMemcpyDeviceToDevice, st), "copy");
            if ((rc = run_dirichlet(g, work[a]))) return rc;
            if ((rc = run_sweep(g, a, work[a], work[a], false))) return rc;
        } else if ((rc = run_sweep(g, a, work[a - 1], work[a], false))) {
            return rc;
        }
    }
    // reverse: Dir^T, Z^T, Dir^T, Y^T, Dir^T, X^T, Dir^T, Src^T.  Each
    // transposed sweep also forms its per-line sums of y^T (L_N x) and y^T x
    // from the y it holds and the forward output x = work[a].
    double* part[3];
    int64_t nlines[3];
    int64_t off = 0;
    for (int a = 0; a < 3; ++a) {
        part[a] = partials + off;
        nlines[a] = axis_lines(axis_geom(a, g->nx, g->ny, g->nz, S));
        off += 2 * nlines[a];
    }
    for (int a = 2; a >= 0; --a) {
        hipError_t e = launch_mask(g->dtype, grad, g->dir_elem, g->ndir, st);
        if (e != hipSuccess) return hip_fail(e, "mask kernel");
        if (a == 2 && fuse_z) {
            const void* invd = f32c ? (const void*)g->invd32[2] : (const void*)g->invd64[2];
            const void* r = f32c ? (const void*)g->r32[2] : (const void*)g->r64[2];
            hipEvent_t t0;
            time_begin(g, 4, &t0);
            e = launch_adj_z_fused(g->dtype, zgeo, zin, grad, invd, r, zcomp, g->comp_H[2], part[2], st);
            time_end(g, 4, t0, zgeo.n * zgeo.inner * zgeo.outer);
            if (e != hipSuccess) return hip_fail(e, "fused z reverse kernel");
            continue;
        }
        AdjSums red;
        red.x = work[a];
        red.part = part[a];
        if ((rc = run_sweep(g, a, grad, grad, true, red))) return rc;
    }
    hipError_t ef = launch_adjoint_line_final(part, nlines, S, red_out, st);
    if (ef != hipSuccess) return hip_fail(ef, "adjoint reduction");
    hipError_t e = launch_mask(g->dtype, grad, g->dir_elem, g->ndir, st);
    if (e != hipSuccess) return hip_fail(e, "mask kernel");
    e = launch_source_transpose(g->dtype, grad, g->src_vox, g->src_invQ, g->nsrc, S, st);
    if (e != hipSuccess) return hip_fail(e, "source transpose kernel");
    return BFVM_OK;
}

// Reads red_out[(a*S + s)*2 + {0, 1}], the sums of y^T (L_N x) and y^T x, in
// chunks of substrates through a stack buffer (after the work before it on
// stream st) and adds dL/dD and dL/dlambda into grad_D, grad_lambda:
// dL/dr_a = -sum y^T L_N x, dL/dbeta = -sum y^T x, dr_a/dD = dt/h_a^2 and
// dbeta/dlambda = dt/3.  Allocates nothing.
int adjoint_accumulate(bfvm_grid g, const double* red_out, hipStream_t st, double* grad_D, double* grad_lambda)
{
    const int S = g->S;
    constexpr int kChunk = 64;
    double buf[3][2 * kChunk];
    for (int s0 = 0; s0 < S; s0 += kChunk) {
        const int cnt = std::min(kChunk, S - s0);
        for (int a = 0; a < 3; ++a)
            HIP_TRY(hipMemcpyAsync(buf[a], red_out + 2 * ((int64_t)a * S + s0), sizeof(double) * 2 * cnt,
                                   hipMemcpyDeviceToHost, st),
                    "copy reductions");
        HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
        for (int k = 0; k < cnt; ++k)
            for (int a = 0; a < 3; ++a) {
                grad_D[s0 + k] += -buf[a][2 * k + 0] * g->dt / (g->h[a] * g->h[a]);
                grad_lambda[s0 + k] += -buf[a][2 * k + 1] * g->dt / 3.0;
            }
    }
    return BFVM_OK;
}

int adjoint_step_into(bfvm_grid g, const void* field_in, void* grad, void* const work[3], double* partials,
                      double* red_out, double* grad_D, double* grad_lambda)
{
    if (int rc = adjoint_enqueue(g, field_in, grad, work, partials, red_out)) return rc;
    return adjoint_accumulate(g, red_out, g->stream, grad_D, grad_lambda);
}

}  // namespace bfvm

// ======================================================================= ABI

extern "C" {

const char* bfvm_version(void) { return "bfvm-gfx950 0.1"; }

const char* bfvm_status_string(int status)
{
    switch (status) {
        case BFVM_OK: return "ok";
        case BFVM_EINVAL: return "invalid argument";
        case BFVM_ERANGE: return "index out of range";
        case BFVM_ESTATE: return "call out of order";
        case BFVM_EDEVICE: return "HIP device error";
        case BFVM_ENOMEM: return "out of memory";
        case BFVM_EOFF: return "feature switched off";
        case BFVM_EIO: return "file I/O error";
        default: return "unknown status";
    }
}

const char* bfvm_last_error(void) { return g_last_error.c_str(); }

int bfvm_create(bfvm_grid* out, int64_t nx, int64_t ny, int64_t nz, int32_t nsub, double hx, double hy,
                double hz, int32_t dtype, void* stream)
{
    if (!out) return fail(BFVM_EINVAL, "out is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail(BFVM_EINVAL, "grid sizes must be >= 1");
    if (nsub < 1) return fail(BFVM_EINVAL, "nsub must be >= 1");
    const double h[3] = {hx, hy, hz};
    for (double v : h)
        if (!std::isfinite(v) || v <= 0.0) return fail(BFVM_EINVAL, "spacings must be finite and > 0");
    if (dtype != BFVM_F64 && dtype != BFVM_F32 && dtype != BFVM_F32_FAST)
        return fail(BFVM_EINVAL, "unknown dtype");
    // every element index must fit in int64 and every line in the kernels' ranges
    const double total = (double)nx * (double)ny * (double)nz * (double)nsub;
    if (total > 9.0e18) return fail(BFVM_EINVAL, "grid too large");
    bfvm_grid g = new (std::nothrow) bfvm_grid_s();
    if (!g) return fail(BFVM_ENOMEM, "host allocation failed");
    g->nx = nx;
    g->ny = ny;
    g->nz = nz;
    g->S = nsub;
    g->h[0] = hx;
    g->h[1] = hy;
    g->h[2] = hz;
    g->dtype = dtype;
    g->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&g->device) != hipSuccess) g->device = 0;
    for (int a = 0; a < 3; ++a)
        g->plan[a] = default_plan(a, axis_geom(a, nx, ny, nz, nsub), dtype);
    (void)refresh_dir_slabs(g);   // no entries yet: empty lists, no allocation
    *out = g;
    return BFVM_OK;
}

int bfvm_destroy(bfvm_grid g)
{
    if (!g) return BFVM_OK;
    (void)hipStreamSynchronize(g->stream);
    for (int a = 0; a < 3; ++a) {
        dfree(g->invd64[a]);
        dfree(g->r64[a]);
        dfree(g->invd32[a]);
        dfree(g->r32[a]);
        dfree(g->comp64[a]);
        dfree(g->comp32[a]);
        if (g->work[a]) (void)hipFree(g->work[a]);
    }
    dfree(g->src_vox);
    dfree(g->src_P);
    dfree(g->src_invQ);
    dfree(g->dir_elem);
    dfree(g->dir_val);
    dfree(g->dir_elem_slab);
    dfree(g->dir_val_slab);
    dfree(g->red_partials);
    dfree(g->red_out);
    for (auto& p : g->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : g->ev_pool) (void)hipEventDestroy(e);
    for (int b = 0; b < 2; ++b) {
        if (g->io_buf[b]) (void)hipHostFree(g->io_buf[b]);
        if (g->io_ev[b]) (void)hipEventDestroy(g->io_ev[b]);
    }
    delete g;
    return BFVM_OK;
}

int bfvm_set_stream(bfvm_grid g, void* stream)
{
    if (int st = check_grid(g)) return st;
    g->stream = static_cast<hipStream_t>(stream);
    return BFVM_OK;
}

int bfvm_set_params(bfvm_grid g, const double* D, const double* lambda, double dt)
{
    if (int st = check_grid(g)) return st;
    if (!D || !lambda) return fail(BFVM_EINVAL, "D and lambda must not be NULL");
    if (!std::isfinite(dt) || dt <= 0.0) return fail(BFVM_EINVAL, "dt must be finite and > 0");
    if (!finite_nonneg(D, g->S)) return fail(BFVM_EINVAL, "D must be finite and >= 0");
    if (!finite_nonneg(lambda, g->S)) return fail(BFVM_EINVAL, "lambda must be finite and >= 0");
    const int S = g->S;
    const int64_t ns[3] = {g->nx, g->ny, g->nz};
    // build all tables on the host before touching device state
    std::vector<double> invd[3], r[3];
    std::vector<float> invd32[3], r32[3];
    for (int a = 0; a < 3; ++a) {
        invd[a].assign((size_t)(ns[a] * S), 0.0);
        r[a].assign(S, 0.0);
        for (int s = 0; s < S; ++s) {
            r[a][s] = dt * D[s] / (g->h[a] * g->h[a]);
            const double beta = dt * lambda[s] / 3.0;
            thomas_constants(ns[a], r[a][s], beta, S, s, invd[a].data());
        }
        invd32[a].assign(invd[a].begin(), invd[a].end());
        r32[a].assign(r[a].begin(), r[a].end());
    }
    // exact compressed tables, [s][H + 2]
    int compH[3];
    std::vector<double> comp[3];
    std::vector<float> comp32[3];
    for (int a = 0; a < 3; ++a) {
        compH[a] = comp_head(invd[a], ns[a], S);
        if (compH[a] < 0) continue;
        const int H = compH[a];
        comp[a].resize((size_t)S * (H + 2));
        for (int s = 0; s < S; ++s) {
            for (int i = 0; i < H; ++i) comp[a][(size_t)s * (H + 2) + i] = invd[a][(size_t)i * S + s];
            comp[a][(size_t)s * (H + 2) + H] = invd[a][(size_t)H * S + s];
            comp[a][(size_t)s * (H + 2) + H + 1] = invd[a][(size_t)(ns[a] - 1) * S + s];
        }
        comp32[a].assign(comp[a].begin(), comp[a].end());
    }
    ++g->gen;
    for (int a = 0; a < 3; ++a) {
        int st;
        if ((st = dalloc_copy(g->invd64[a], invd[a].data(), invd[a].size(), g->stream))) return st;
        if ((st = dalloc_copy(g->r64[a], r[a].data(), r[a].size(), g->stream))) return st;
        if ((st = dalloc_copy(g->invd32[a], invd32[a].data(), invd32[a].size(), g->stream))) return st;
        if ((st = dalloc_copy(g->r32[a], r32[a].data(), r32[a].size(), g->stream))) return st;
        g->comp_H[a] = -1;
        if ((st = dalloc_copy(g->comp64[a], comp[a].data(), comp[a].size(), g->stream))) return st;
        if ((st = dalloc_copy(g->comp32[a], comp32[a].data(), comp32[a].size(), g->stream))) return st;
        g->comp_H[a] = compH[a];
    }
    g->D.assign(D, D + S);
    g->lambda.assign(lambda, lambda + S);
    g->dt = dt;
    g->have_params = true;
    if (!g->raw_vox.empty()) return merge_sources(g);
    return BFVM_OK;
}

int bfvm_set_sources(bfvm_grid g, int64_t count, const int64_t* voxel, const double* secretion,
                     const double* saturation, const double* uptake)
{
    if (int st = check_grid(g)) return st;
    if (count < 0) return fail(BFVM_EINVAL, "count must be >= 0");
    if (!g->have_params) return fail(BFVM_ESTATE, "set_params must come before set_sources");
    if (count > 0 && (!voxel || !secretion || !saturation || !uptake))
        return fail(BFVM_EINVAL, "source arrays must not be NULL");
    const int S = g->S;
    const int64_t V = g->nvox();
    for (int64_t k = 0; k < count; ++k)
        if (voxel[k] < 0 || voxel[k] >= V) return fail(BFVM_ERANGE, "source voxel index out of range");
    if (count > 0 && (!finite_nonneg(secretion, count * S) || !finite_nonneg(saturation, count * S) ||
                      !finite_nonneg(uptake, count * S)))
        return fail(BFVM_EINVAL, "source rates must be finite and >= 0");
    ++g->gen;
    g->raw_vox.assign(voxel, voxel + count);
    g->raw_sec.assign(secretion, secretion + count * S);
    g->raw_sat.assign(saturation, saturation + count * S);
    g->raw_upt.assign(uptake, uptake + count * S);
    if (count == 0) {
        g->nsrc = 0;
        dfree(g->src_vox);
        dfree(g->src_P);
        dfree(g->src_invQ);
        return BFVM_OK;
    }
    return merge_sources(g);
}

int bfvm_set_dirichlet(bfvm_grid g, int64_t count, const int64_t* voxel, const double* value,
                       const uint8_t* active)
{
    if (int st = check_grid(g)) return st;
    if (count < 0) return fail(BFVM_EINVAL, "count must be >= 0");
    if (count > 0 && (!voxel || !value || !active)) return fail(BFVM_EINVAL, "Dirichlet arrays must not be NULL");
    const int S = g->S;
    const int64_t V = g->nvox();
    for (int64_t k = 0; k < count; ++k)
        if (voxel[k] < 0 || voxel[k] >= V) return fail(BFVM_ERANGE, "Dirichlet voxel index out of range");
    for (int64_t i = 0; i < count * S; ++i)
        if (active[i] && !std::isfinite(value[i])) return fail(BFVM_EINVAL, "Dirichlet values must be finite");
    // last active entry of each (voxel, substrate) wins
    std::vector<std::pair<int64_t, int64_t>> ent;   // (element, list position)
    for (int64_t k = 0; k < count; ++k)
        for (int s = 0; s < S; ++s)
            if (active[k * S + s]) ent.push_back({voxel[k] * S + s, k * S + s});
    std::stable_sort(ent.begin(), ent.end(),
                     [](const std::pair<int64_t, int64_t>& a, const std::pair<int64_t, int64_t>& b) {
                         return a.first < b.first;
                     });
    std::vector<int64_t> elem;
    std::vector<double> val;
    for (size_t i = 0; i < ent.size(); ++i) {
        if (i + 1 < ent.size() && ent[i + 1].first == ent[i].first) continue;   // a later entry wins
        elem.push_back(ent[i].first);
        val.push_back(value[ent[i].second]);
    }
    ++g->gen;
    int st;
    if ((st = dalloc_copy(g->dir_elem, elem.data(), elem.size(), g->stream))) return st;
    if ((st = dalloc_copy(g->dir_val, val.data(), val.size(), g->stream))) return st;
    g->ndir = (int64_t)elem.size();
    g->dir_elem_h = elem;
    g->dir_val_h = val;
    g->dir_slab_w = 0;
    g->dir_slab_off.clear();
    return refresh_dir_slabs(g);
}

int bfvm_step(bfvm_grid g, void* field, int64_t nsteps)
{
    if (int st = check_grid(g)) return st;
    if (!field) return fail(BFVM_EINVAL, "field is NULL");
    if (nsteps < 0) return fail(BFVM_EINVAL, "nsteps must be >= 0");
    if (!g->have_params) return fail(BFVM_ESTATE, "set_params must come before step");
    int sched;
    int64_t w;
    resolve_schedule(g, &sched, &w);
    if (sched == 1 || sched == 2) {
        if (g->dir_slab_w != w || g->dir_slab_off.empty())
            return fail(BFVM_ESTATE, "per-slab Dirichlet lists are stale");
        for (int64_t t = 0; t < nsteps; ++t)
            if (int st = sched == 1 ? run_step_fused(g, field, w) : run_step_zfused(g, field, w)) return st;
        return BFVM_OK;
    }
    for (int64_t t = 0; t < nsteps; ++t)
        if (int st = bfvm::run_plain_step(g, field)) return st;
    return BFVM_OK;
}

int bfvm_sweep(bfvm_grid g, void* field, int32_t axis)
{
    if (int st = check_grid(g)) return st;
    if (!field) return fail(BFVM_EINVAL, "field is NULL");
    if (axis < 0 || axis > 2) return fail(BFVM_EINVAL, "axis must be 0, 1 or 2");
    if (!g->have_params) return fail(BFVM_ESTATE, "set_params must come before sweep");
    return run_sweep(g, axis, field, field, false);
}

namespace {

int xslab_run(bfvm_grid g, bool fwd, void* slab, int64_t x0, int64_t x1, int64_t l0, int64_t l1, const void* cin,
              void* cout)
{
    if (int st = check_grid(g)) return st;
    if (!g->have_params) return fail(BFVM_ESTATE, "set_params must come before the slab sweeps");
    if (!slab || !cout) return fail(BFVM_EINVAL, "slab or carry_out is NULL");
    if (x0 < 0 || x1 <= x0 || x1 > g->nx) return fail(BFVM_EINVAL, "need 0 <= x0 < x1 <= nx");
    const int64_t nl = g->ny * g->nz * (int64_t)g->S;
    if (l0 < 0 || l1 <= l0 || l1 > nl) return fail(BFVM_EINVAL, "need 0 <= l0 < l1 <= ny * nz * S");
    const bool edge = fwd ? x0 == 0 : x1 == g->nx;
    if (edge != (cin == nullptr))
        return fail(BFVM_EINVAL, fwd ? "carry_in must be NULL exactly when x0 == 0"
                                     : "carry_in must be NULL exactly when x1 == nx");
    int M = 0, K = 0, lpw = 0;
    if (!xslab_plan(x1 - x0, &M, &K, &lpw)) return fail(BFVM_EINVAL, "slab longer than 2048");
    const bool f32c = g->dtype == BFVM_F32_FAST;
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, g->device) != hipSuccess)
        return fail(BFVM_EDEVICE, "hipDeviceGetAttribute");
    if (xslab_lds(M, K, lpw, g->S, f32c ? 4 : 8) > (size_t)lds_max)
        return fail(BFVM_EINVAL, "the slab's constants do not fit the LDS");
    const void* invd = f32c ? (const void*)g->invd32[0] : (const void*)g->invd64[0];
    const void* r = f32c ? (const void*)g->r32[0] : (const void*)g->r64[0];
    hipEvent_t a;
    time_begin(g, 2, &a);
    hipError_t e = launch_xslab(g->dtype, fwd, slab, x1 - x0, g->S, l0, l1 - l0, invd, r, x0, cin, cout, g->stream);
    time_end(g, 2, a, (x1 - x0) * (l1 - l0));
    return e == hipSuccess ? BFVM_OK : hip_fail(e, "slab sweep kernel");
}

}  // namespace

int bfvm_xslab_forward(bfvm_grid g, void* slab, int64_t x0, int64_t x1, int64_t l0, int64_t l1, const void* carry_in,
                       void* carry_out)
{
    return xslab_run(g, true, slab, x0, x1, l0, l1, carry_in, carry_out);
}

int bfvm_xslab_backward(bfvm_grid g, void* slab, int64_t x0, int64_t x1, int64_t l0, int64_t l1,
                        const void* carry_in, void* carry_out)
{
    return xslab_run(g, false, slab, x0, x1, l0, l1, carry_in, carry_out);
}

int bfvm_step_adjoint(bfvm_grid g, const void* field_in, void* grad, double* grad_D, double* grad_lambda)
{
    if (int st = check_grid(g)) return st;
    if (!field_in || !grad || !grad_D || !grad_lambda) return fail(BFVM_EINVAL, "NULL pointer");
    if (!g->have_params) return fail(BFVM_ESTATE, "set_params must come before step_adjoint");
    // workspace: three sweep outputs, reduction partials and results
    if (int st = bfvm::ensure_adjoint_workspace(g)) return st;
    return bfvm::adjoint_step_into(g, field_in, grad, g->work, g->red_partials, g->red_out, grad_D, grad_lambda);
}

int bfvm_device_bytes(bfvm_grid g, int64_t* bytes)
{
    if (int st = check_grid(g)) return st;
    if (!bytes) return fail(BFVM_EINVAL, "NULL pointer");
    int64_t total = 0;
    auto add = [&](const void* p) {
        if (!p) return;
        void* base = nullptr;
        size_t size = 0;
        if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) == hipSuccess) total += (int64_t)size;
    };
    for (int a = 0; a < 3; ++a) {
        add(g->invd64[a]);
        add(g->r64[a]);
        add(g->invd32[a]);
        add(g->r32[a]);
        add(g->comp64[a]);
        add(g->comp32[a]);
        add(g->work[a]);
    }
    for (const void* p : {(const void*)g->src_vox, (const void*)g->src_P, (const void*)g->src_invQ,
                          (const void*)g->dir_elem, (const void*)g->dir_val, (const void*)g->dir_elem_slab,
                          (const void*)g->dir_val_slab, (const void*)g->red_partials, (const void*)g->red_out})
        add(p);
    *bytes = total;
    return BFVM_OK;
}

int bfvm_fill_uniform(bfvm_grid g, void* field, uint64_t seed, uint32_t stream, double lo, double hi)
{
    if (int st = check_grid(g)) return st;
    if (!field) return fail(BFVM_EINVAL, "NULL field");
    if (!std::isfinite(lo) || !std::isfinite(hi) || hi < lo) return fail(BFVM_EINVAL, "bounds must be finite, lo <= hi");
    hipError_t e = launch_fill_uniform(g->dtype, field, g->nelem(), seed, stream, lo, hi, g->stream);
    return e == hipSuccess ? BFVM_OK : hip_fail(e, "fill kernel");
}

int bfvm_fill_gaussian(bfvm_grid g, void* field, double cx, double cy, double cz, double sigma, double peak,
                       double noise, uint64_t seed, uint32_t stream)
{
    if (int st = check_grid(g)) return st;
    if (!field) return fail(BFVM_EINVAL, "NULL field");
    for (double v : {cx, cy, cz, sigma, peak, noise})
        if (!std::isfinite(v)) return fail(BFVM_EINVAL, "non-finite argument");
    if (!(sigma > 0)) return fail(BFVM_EINVAL, "sigma must be > 0");
    hipError_t e = launch_fill_gaussian(g->dtype, field, g->nx, g->ny, g->nz, g->S, cx, cy, cz, sigma, peak, noise,
                                        seed, stream, g->stream);
    return e == hipSuccess ? BFVM_OK : hip_fail(e, "fill kernel");
}

int bfvm_read_field(bfvm_grid g, const void* field, void* host_dst)
{
    if (int st = check_grid(g)) return st;
    if (!field || !host_dst) return fail(BFVM_EINVAL, "NULL pointer");
    const size_t bytes = (size_t)g->nelem() * dtype_size(g->dtype);
    HIP_TRY(hipMemcpyAsync(host_dst, field, bytes, hipMemcpyDeviceToHost, g->stream), "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
    return BFVM_OK;
}

int bfvm_timing_enable(bfvm_grid g, int32_t enable)
{
    if (int st = check_grid(g)) return st;
    if (!enable) time_harvest(g);
    g->timing = enable != 0;
    return BFVM_OK;
}

int bfvm_timing_read(bfvm_grid g, int32_t stage, double* total_ms, int64_t* launches)
{
    if (int st = check_grid(g)) return st;
    if (stage < 0 || stage > 4 || !total_ms || !launches) return fail(BFVM_EINVAL, "bad stage or NULL");
    time_harvest(g);
    *total_ms = g->stage_ms[stage];
    *launches = g->stage_count[stage];
    return BFVM_OK;
}

int bfvm_timing_reset(bfvm_grid g)
{
    if (int st = check_grid(g)) return st;
    time_harvest(g);
    for (int i = 0; i < 5; ++i) {
        g->stage_ms[i] = 0;
        g->stage_count[i] = 0;
        g->stage_elems[i] = 0;
    }
    return BFVM_OK;
}

int bfvm_timing_elements(bfvm_grid g, int32_t stage, int64_t* elements)
{
    if (int st = check_grid(g)) return st;
    if (stage < 0 || stage > 4 || !elements) return fail(BFVM_EINVAL, "bad stage or NULL");
    time_harvest(g);
    *elements = g->stage_elems[stage];
    return BFVM_OK;
}

int bfvm_set_schedule(bfvm_grid g, int32_t schedule, int64_t slab_width)
{
    if (int st = check_grid(g)) return st;
    if (schedule < -1 || schedule > 2) return fail(BFVM_EINVAL, "schedule must be -1, 0, 1 or 2");
    if (slab_width < 0) return fail(BFVM_EINVAL, "slab_width must be >= 0");
    g->schedule = schedule;
    g->slab_w = slab_width;
    g->dir_slab_w = 0;
    g->dir_slab_off.clear();
    return refresh_dir_slabs(g);
}

int bfvm_get_schedule(bfvm_grid g, int32_t* schedule, int64_t* slab_width)
{
    if (int st = check_grid(g)) return st;
    if (!schedule || !slab_width) return fail(BFVM_EINVAL, "NULL pointer");
    int sc;
    int64_t w;
    resolve_schedule(g, &sc, &w);
    *schedule = sc;
    *slab_width = w;
    return BFVM_OK;
}

int bfvm_get_plan(bfvm_grid g, int32_t axis, int32_t* kind, int32_t* m, int32_t* w, int32_t* lpw)
{
    if (int st = check_grid(g)) return st;
    if (axis < 0 || axis > 2 || !kind || !m || !w || !lpw) return fail(BFVM_EINVAL, "bad axis or NULL");
    *kind = g->plan[axis].kind;
    *m = g->plan[axis].m;
    *w = g->plan[axis].w;
    *lpw = g->plan[axis].lpw;
    return BFVM_OK;
}

int bfvm_set_plan(bfvm_grid g, int32_t axis, int32_t kind, int32_t m, int32_t w, int32_t lpw)
{
    if (int st = check_grid(g)) return st;
    if (axis < 0 || axis > 2) return fail(BFVM_EINVAL, "axis must be 0, 1 or 2");
    SweepPlan p;
    p.kind = kind;
    p.m = m;
    p.w = w;
    p.lpw = lpw;
    if ((kind == PLAN_SEG_XTILE || kind == PLAN_SEG_XROWS) && axis != 0)
        return fail(BFVM_EINVAL, "plan kinds 2 and 3 only run the x axis");
    const std::string why = check_plan(p, axis_geom(axis, g->nx, g->ny, g->nz, g->S), g->dtype);
    if (!why.empty()) return fail(BFVM_EINVAL, "plan does not fit: " + why);
    g->plan[axis] = p;
    g->dir_slab_w = 0;
    g->dir_slab_off.clear();
    return refresh_dir_slabs(g);
}

}  // extern "C"
