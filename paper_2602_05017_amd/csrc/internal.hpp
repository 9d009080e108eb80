// Internal declarations of the gfx950 diffusion-decay library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "bfvm.h"

namespace bfvm {

// Thread-local error text behind bfvm_last_error().
void set_error(const std::string& msg);

// ----------------------------------------------------------------- geometry
//
// A sweep along axis a sees the field as [outer][n][inner]: line (o, p) has
// elements  o*outer_stride + p + i*stride,  i = 0..n-1, p in [0, inner),
// and belongs to substrate p % S.
//   x: outer = nz*ny, n = nx, inner = S,          stride = S
//   y: outer = nz,    n = ny, inner = nx*S,       stride = nx*S
//   z: outer = 1,     n = nz, inner = ny*nx*S,    stride = ny*nx*S
struct AxisGeom {
    int64_t n;
    int64_t inner;
    int64_t outer;
    int64_t stride;
    int64_t outer_stride;
    int32_t S;
    int64_t p0 = 0;   // offset of line 0 inside the inner range (a multiple of S)
    int64_t o0 = 0;   // offset of outer index 0
    int32_t axis = 0; // 0 x, 1 y, 2 z (names the kernel instance in profiles)
};

AxisGeom axis_geom(int axis, int64_t nx, int64_t ny, int64_t nz, int32_t S);
// The y (axis 1) or z (axis 2) lines of the x-slab [x0, x1): both stay inside
// the slab, so the two sweeps can run back to back on one slab.
AxisGeom slab_geom(int axis, int64_t nx, int64_t ny, int64_t nz, int32_t S, int64_t x0, int64_t x1);
// The x (axis 0) or y (axis 1) lines of the z-slab [z0, z1).
AxisGeom zslab_geom(int axis, int64_t nx, int64_t ny, int64_t nz, int32_t S, int64_t z0, int64_t z1);

// Launch plan of one sweep (see bfvm_get_plan in bfvm.h).
enum PlanKind {
    PLAN_LINE = 0,
    PLAN_SEG_STRIDED = 1,
    PLAN_SEG_XTILE = 2,
    PLAN_SEG_XROWS = 3,
    PLAN_SEG_XPIPE = 4,
    PLAN_SEG_HALVES = 5
};

struct SweepPlan {
    int32_t kind = PLAN_LINE;
    int32_t m = 0;     // elements per thread (segmented kernels)
    int32_t w = 0;     // waves per workgroup
    int32_t lpw = 0;   // lines per wave (strided) / rows per workgroup (x tile)
};

// Device coefficient tables of one axis: invd[i*S + s] = 1/denom_i of
// substrate s, r[s] = dt*D_s/h_a^2.  Compute type C (double or float).
template <typename C>
struct Coefs {
    const C* invd;
    const C* r;
};

// Storage/arithmetic combinations.
enum DType { DT_F64 = BFVM_F64, DT_F32 = BFVM_F32, DT_F32_FAST = BFVM_F32_FAST };

inline size_t dtype_size(int dt) { return dt == DT_F64 ? 8 : 4; }

// Validate a plan for an axis; returns empty string when it fits.
std::string check_plan(const SweepPlan& p, const AxisGeom& g, int dtype);
// Default plan for an axis.
SweepPlan default_plan(int axis, const AxisGeom& g, int dtype);

// The reverse step's per-line sums, formed inside a transposed sweep: for
// line L of the axis, part[2 L] = sum_i y_i (L_N x)_i and part[2 L + 1] =
// sum_i y_i x_i, with y the sweep's output, x the forward sweep's output on
// the same lines (field layout) and L_N the zero-flux Laplacian.  Lines are
// numbered L = o * inner + p (AxisGeom order; for x, row * S + s), so line L
// belongs to substrate L % S.
struct AdjSums {
    const void* x = nullptr;
    double* part = nullptr;   // nullptr: no sums
};
inline int64_t axis_lines(const AxisGeom& g) { return g.inner * g.outer; }

// Enqueue one sweep (forward Thomas, or transposed solve when transposed) of
// field `in` into `out` (may alias) on `stream`.  coefs point to double or
// float tables matching the dtype's compute type.
// comp / comp_H: the axis's exact compressed coefficient table (comp_H < 0: none)
// red: with red.part set (transposed whole-field sweeps only), also write
// the per-line sums.
hipError_t launch_sweep(int dtype, bool transposed, const SweepPlan& plan, const AxisGeom& g,
                        const void* in, void* out, const void* invd, const void* r,
                        const void* comp, int comp_H, hipStream_t stream, const AdjSums& red = AdjSums());

// Sparse stages.
hipError_t launch_source(int dtype, void* u, const int64_t* vox, const double* P,
                         const double* invQ, int64_t m, int32_t S, hipStream_t stream);
hipError_t launch_source_transpose(int dtype, void* g, const int64_t* vox, const double* invQ,
                                   int64_t m, int32_t S, hipStream_t stream);
hipError_t launch_dirichlet(int dtype, void* u, const int64_t* elem, const double* val,
                            int64_t cnt, hipStream_t stream);
hipError_t launch_mask(int dtype, void* g, const int64_t* elem, int64_t cnt, hipStream_t stream);

// The reverse step's z axis in one pass (sweep.hip): the forward z sweep of
// zin recomputed in registers, the transposed z sweep of grad in place and
// the per-line parameter sums part[2 L] (as the RED transposed sweep writes
// them).  adj_z_fusable: whether this geometry takes it (z lines of up to
// 512 voxels, the coefficient table or compressed rows in LDS).
bool adj_z_fusable(int dtype, const AxisGeom& g, const void* comp, int compH);
hipError_t launch_adj_z_fused(int dtype, const AxisGeom& g, const void* zin, void* grad, const void* invd,
                              const void* r, const void* comp, int compH, double* part, hipStream_t stream);

// One x-slab's forward or backward share of the x sweep (slab.hip); see
// bfvm_xslab_forward.  xslab_plan: M, segments and lines per tile for an
// m-voxel slab line (0 beyond reach); xslab_lds: the block's LDS bytes.
int xslab_plan(int64_t m, int* M, int* K, int* lpw);
size_t xslab_lds(int M, int K, int lpw, int S, int cs);
hipError_t launch_xslab(int dtype, bool fwd, void* slab, int64_t m, int S, int64_t l0, int64_t nlines,
                        const void* invd, const void* r, int64_t x0, const void* cin, void* cout, hipStream_t st);

// Second stage of the per-line sums: out[(a*S + s)*2 + {0,1}] = the sum over
// the lines L = s (mod S) of axis a (part[a], nlines[a] lines), in line order.
hipError_t launch_adjoint_line_final(double* const part[3], const int64_t nlines[3], int S, double* out,
                                     hipStream_t stream);

// Device-side field set-up (fill.hip).
hipError_t launch_fill_uniform(int dtype, void* u, int64_t n, uint64_t seed, uint32_t stream, double lo, double hi,
                               hipStream_t st);
hipError_t launch_fill_gaussian(int dtype, void* u, int64_t nx, int64_t ny, int64_t nz, int S, double cx, double cy,
                                double cz, double sigma, double peak, double noise, uint64_t seed, uint32_t stream,
                                hipStream_t st);

}  // namespace bfvm

struct bfvm_grid_s;

namespace bfvm {
// One reverse step (bfvm_step_adjoint) into caller-provided workspace, shared
// by the allocating and the allocation-free entry points (grid.cpp):
// adjoint_enqueue puts the device work on the grid's stream,
// adjoint_accumulate reads the parameter sums back and adds them to the
// caller's gradients, adjoint_step_into does both.
int64_t adjoint_partials_count(bfvm_grid_s* g);
int adjoint_enqueue(bfvm_grid_s* g, const void* field_in, void* grad, void* const work[3], double* partials,
                    double* red_out);
int adjoint_accumulate(bfvm_grid_s* g, const double* red_out, hipStream_t st, double* grad_D, double* grad_lambda);
int adjoint_step_into(bfvm_grid_s* g, const void* field_in, void* grad, void* const work[3], double* partials,
                      double* red_out, double* grad_D, double* grad_lambda);
// the grid's own reverse-step workspace (work, red_partials, red_out),
// allocated on first use
int ensure_adjoint_workspace(bfvm_grid_s* g);
// one step of the plain schedule on the grid's stream / on stream s
int run_plain_step(bfvm_grid_s* g, void* field);
int enqueue_step(bfvm_grid_s* g, void* field, hipStream_t s);
}  // namespace bfvm

// --------------------------------------------------------------- grid object
struct bfvm_grid_s {
    int64_t nx = 0, ny = 0, nz = 0;
    int32_t S = 0;
    double h[3] = {0, 0, 0};
    int32_t dtype = BFVM_F64;
    hipStream_t stream = nullptr;
    int device = 0;

    bool have_params = false;
    double dt = 0.0;
    // bumped by every setter that may reallocate the device tables or lists
    // below (set_params, set_sources, set_dirichlet); a batch holding this
    // grid compares it before each call and re-reads the grid when it moved
    uint64_t gen = 0;
    std::vector<double> D, lambda;

    // coefficient tables per axis (device): double and float copies
    double* invd64[3] = {nullptr, nullptr, nullptr};
    double* r64[3] = {nullptr, nullptr, nullptr};
    float* invd32[3] = {nullptr, nullptr, nullptr};
    float* r32[3] = {nullptr, nullptr, nullptr};
    // exact compressed coefficient tables, [s][H + 2] (head, constant, last);
    // comp_H[a] < 0: the axis has none (the full table is used)
    double* comp64[3] = {nullptr, nullptr, nullptr};
    float* comp32[3] = {nullptr, nullptr, nullptr};
    int comp_H[3] = {-1, -1, -1};

    // merged sources (device)
    int64_t nsrc = 0;
    int64_t* src_vox = nullptr;
    double* src_P = nullptr;
    double* src_invQ = nullptr;
    // raw source list (host copy, re-merged when dt changes)
    std::vector<int64_t> raw_vox;
    std::vector<double> raw_sec, raw_sat, raw_upt;

    // Dirichlet (device), deduplicated active entries
    int64_t ndir = 0;
    int64_t* dir_elem = nullptr;
    double* dir_val = nullptr;
    std::vector<int64_t> dir_elem_h;   // host copies (sorted by element)
    std::vector<double> dir_val_h;

    bfvm::SweepPlan plan[3];

    // step schedule: 0 = three full sweeps; 1 = x sweep, then y and z back to
    // back on x-slabs of slab_w columns; 2 = x and y back to back on z-slabs
    // of slab_w planes, then the z sweep (slab_w = 0: chosen automatically)
    int32_t schedule = -1;   // -1 = automatic
    int64_t slab_w = 0;
    // Dirichlet entries sorted by x-slab (for the fused schedule): slab k owns
    // dir entries [dir_slab_off[k], dir_slab_off[k+1])
    int64_t dir_slab_w = 0;
    std::vector<int64_t> dir_slab_off;
    int64_t* dir_elem_slab = nullptr;
    double* dir_val_slab = nullptr;

    // adjoint workspace
    void* work[3] = {nullptr, nullptr, nullptr};
    double* red_partials = nullptr;   // per-line sums of the reverse step
    int64_t red_count = 0;            // doubles allocated at red_partials
    double* red_out = nullptr;

    // pinned host buffers and events of the .npy field I/O (io.cpp)
    void* io_buf[2] = {nullptr, nullptr};
    hipEvent_t io_ev[2] = {nullptr, nullptr};

    // stage timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    struct Pending { int stage; hipEvent_t a, b; };
    std::vector<Pending> pending;
    double stage_ms[5] = {0, 0, 0, 0, 0};
    int64_t stage_count[5] = {0, 0, 0, 0, 0};
    int64_t stage_elems[5] = {0, 0, 0, 0, 0};

    int64_t nvox() const { return nx * ny * nz; }
    int64_t nelem() const { return nx * ny * nz * (int64_t)S; }
};

namespace bfvm {
// While alive, the grid's stage launches go to stream s with its stage
// timers off (a batch enqueues the members its grouped kernels cannot take
// this way, on one of its own streams); the grid's stream and timers are
// restored on destruction.
struct OnStream {
    bfvm_grid_s* g;
    hipStream_t keep;
    bool timing;
    OnStream(bfvm_grid_s* g_, hipStream_t s) : g(g_), keep(g_->stream), timing(g_->timing)
    {
        g->stream = s;
        g->timing = false;
    }
    ~OnStream()
    {
        g->stream = keep;
        g->timing = timing;
    }
    OnStream(const OnStream&) = delete;
    OnStream& operator=(const OnStream&) = delete;
};
}  // namespace bfvm
