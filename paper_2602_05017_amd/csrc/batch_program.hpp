// Host-side description of a batch program: the per-domain stage chains of
// one step (or one reverse step) cut into work items, in the order the
// kernels take them, with the grouped mode's launches and the persistent
// mode's dependency counters.  Plain C++ (no HIP): the library builds its
// programs with it, and a CPU test builds the same programs to check the
// persistent scheduler's protocol.
#pragma once

#include <algorithm>
#include <cstdint>
#include <utility>
#include <vector>

#include "bfvm.h"

namespace bfvm {

enum StageType : int32_t {
    ST_SRC = 0,      // u <- (u + P) * invQ at source entries
    ST_DIR = 1,      // u <- value at Dirichlet entries
    ST_SWEEP = 2,    // Thomas sweep along axis
    ST_SWEEP_T = 3,  // transposed sweep along axis
    ST_MASK = 4,     // g <- 0 at Dirichlet entries
    ST_SRC_T = 5,    // g <- g * invQ at source entries
    ST_COPY = 6,     // buffer out <- buffer in
};

constexpr int kBatchThreads = 512;
constexpr int64_t kSparseChunk = 2048;   // source / Dirichlet entries per item
constexpr int kBatchTab = 2048;   // line length x substrates, per axis
// elements per thread M in {4, 8} and at most 512/16 = 32 segments per line
constexpr int64_t kMaxBatchLine = 256;
constexpr int kNumBuf = 5;   // 0 field, 1 gradient, 2..4 adjoint workspace
// substrates per domain: the reverse step's per-substrate sums of an item
// are kept in LDS
constexpr int kMaxBatchSub = 256;

struct BDomain {
    int32_t dtype;
    int32_t S;
    int64_t nx, ny, nz;
    void* buf[kNumBuf];
    const void* invd[3];
    const void* r[3];
    const int64_t* src_vox;
    const double* src_P;
    const double* src_invQ;
    int64_t nsrc;
    const int64_t* dir_elem;
    const double* dir_val;
    int64_t ndir;
    int32_t M[3];
    int32_t lpw[3];
};

struct BItem {
    int32_t dom;
    int32_t type;
    int32_t axis;
    int32_t in, out;
    int32_t xb;        // SWEEP_T: buffer of the forward output x for the parameter sums
    int32_t done;      // counter incremented when the item completes
    int32_t dep;       // counter to wait for (-1: none)
    uint32_t need;     // value of counter dep that means "stage complete"
    int32_t m, lpw;    // sweeps: elements per thread and lines per tile
    int64_t a0, a1;    // range (tiles, entries, elements or voxels)
    int64_t slot;      // SWEEP_T: offset of the item's 2*S parameter sums
};

struct Stage {
    int32_t type, axis, in, out;
    int32_t xb = -1;   // SWEEP_T: buffer of the forward output for the parameter sums
};

// One kernel launch of the grouped mode: the items [off, off + count) of one
// stage (sweeps: one (storage type, M) class of that stage), one block each.
struct Launch {
    int32_t sweep;     // 1: k_group_sweep, 0: k_group_sparse
    int32_t dtype, M;
    bool tr;
    int64_t off, count;
};

// Items, launches and counter counts of one program.
struct ProgramLayout {
    std::vector<BItem> items;        // stage-major
    std::vector<Launch> launches;    // grouped mode, in program order
    int64_t ncounters = 0;           // persistent mode
    int64_t npartials = 0;
};

inline int64_t tiles_of(const BDomain& d, int axis, int lpw)
{
    int64_t inner, outer;
    if (axis == 0) { inner = d.ny * d.nz * d.S; outer = 1; }
    else if (axis == 1) { inner = d.nx * d.S; outer = d.nz; }
    else { inner = d.nx * d.ny * d.S; outer = 1; }
    return (inner + lpw - 1) / lpw * outer;
}

inline int64_t axis_len(const BDomain& d, int axis) { return axis == 0 ? d.nx : (axis == 1 ? d.ny : d.nz); }

inline bool plan_fits(int64_t n, int M, int lpw) { return (int64_t)(kBatchThreads / lpw) * M >= n; }

// M = 12 fills the lines of 65..96 voxels that an 8-segment tile would
// otherwise hold as 128 slots of 16: 96-domain step 4.70 -> 4.44 ms with
// {4, 8, 12, 16}; adding 6 and 10 (38 launches per step instead of 26) gave
// 4.47 ms
constexpr int kBatchM[] = {4, 8, 12, 16};

// smallest supported elements-per-thread whose K = 512 / lpw segments cover n
inline int smallest_m(int64_t n, int lpw, int max_m)
{
    for (int m : kBatchM)
        if (m <= max_m && plan_fits(n, m, lpw)) return m;
    return 0;
}

inline int max_m_for_mode(int mode) { return mode == BFVM_BATCH_PERSISTENT ? 8 : 16; }

// Tile shape of a sweep stage: the domain's plan, except that a transposed
// sweep of M = 12 or 16 runs as M = 8 with half the lines per tile (at
// least 16) where those segments still cover the line.  The transposed
// M = 12 and 16 tiles need 168 and 203 VGPRs, one 512-thread block per CU;
// at M = 8 (128) two fit.
inline void tile_shape(const BDomain& d, int axis, bool transposed, int* m, int* lpw)
{
    *m = d.M[axis];
    *lpw = d.lpw[axis];
    if (transposed && *m > 8) {
        const int l = std::max(16, *lpw / 2);
        if (plan_fits(axis_len(d, axis), 8, l)) {
            *m = 8;
            *lpw = l;
        }
    }
}

// default per-axis plan: the most lines per tile (widest coalesced rows)
// whose segments of at most 8 elements still cover the line (16 only if
// the autotuner finds it faster: it doubles the registers per thread)
inline void default_batch_plan(BDomain& d, int mode)
{
    (void)mode;
    for (int a = 0; a < 3; ++a) {
        const int64_t n = axis_len(d, a);
        for (int l : {64, 32, 16}) {
            const int m = smallest_m(n, l, 8);
            if (m) {
                d.M[a] = m;
                d.lpw[a] = l;
                break;
            }
        }
    }
}

// Build a program (per-domain stage chains) over domains `which`: items in
// stage-major order, the grouped launches, and the persistent mode's
// counters: one per non-empty (domain, stage); each item increments its
// stage's counter (done) and waits until the counter of its domain's
// previous non-empty stage (dep) reaches that stage's item count (need).
// Stage-major order puts every item after all items it depends on.
inline void build_layout(const std::vector<BDomain>& doms, int64_t chunk_elems, const std::vector<int32_t>& which,
                  const std::vector<Stage>& prog, ProgramLayout& P)
{
    P.items.clear();
    P.launches.clear();
    const int ns = (int)prog.size();
    std::vector<std::vector<std::vector<BItem>>> per(which.size(), std::vector<std::vector<BItem>>(ns));
    int64_t partials = 0;
    for (int k = 0; k < ns; ++k) {
        const Stage& sg = prog[k];
        for (size_t wi = 0; wi < which.size(); ++wi) {
            const BDomain& d = doms[which[wi]];
            const int64_t nel = d.nx * d.ny * d.nz * d.S;
            int64_t total = 0, chunk = 1;
            int tm = 0, tl = 0;
            if (sg.type == ST_SWEEP || sg.type == ST_SWEEP_T) tile_shape(d, sg.axis, sg.type == ST_SWEEP_T, &tm, &tl);
            switch (sg.type) {
                // scattered sparse entries: small items, so that a launch has
                // blocks for every CU and each thread few dependent accesses
                case ST_SRC: case ST_SRC_T: total = d.nsrc * d.S; chunk = kSparseChunk; break;
                case ST_DIR: case ST_MASK: total = d.ndir; chunk = kSparseChunk; break;
                // a domain without Dirichlet entries needs no copy between the
                // recomputed sweeps: its y and z sweeps read the previous
                // sweep's buffer and write their own (out of place, below);
                // without sources either, its x sweep reads the state itself
                case ST_COPY:
                    total = (d.ndir == 0 && (sg.in != 0 || d.nsrc == 0)) ? 0 : nel;
                    chunk = chunk_elems;
                    break;
                default: {
                    total = tiles_of(d, sg.axis, tl);
                    const int64_t per_tile = (int64_t)tl * axis_len(d, sg.axis);
                    chunk = std::max<int64_t>(1, chunk_elems / std::max<int64_t>(per_tile, 1));
                }
            }
            for (int64_t a0 = 0; a0 < total; a0 += chunk) {
                BItem it{};
                it.dom = which[wi];
                it.type = sg.type;
                it.axis = sg.axis;
                it.in = sg.in;
                it.out = sg.out;
                it.xb = sg.xb;
                it.m = tm;
                it.lpw = tl;
                if (sg.type == ST_SWEEP && sg.in == sg.out && sg.in >= 2 && d.ndir == 0) {
                    if (sg.in >= 3) it.in = sg.in - 1;
                    else if (d.nsrc == 0) it.in = 0;
                }
                it.a0 = a0;
                it.a1 = std::min(total, a0 + chunk);
                if (sg.type == ST_SWEEP_T) {
                    it.slot = partials;
                    partials += 2 * d.S;
                }
                per[wi][k].push_back(it);
            }
        }
    }
    // persistent mode: one counter per non-empty (domain, stage); an item
    // waits for the previous non-empty stage of its domain
    int64_t nc = 0;
    for (size_t wi = 0; wi < which.size(); ++wi) {
        int32_t prev = -1;
        uint32_t prev_need = 0;
        for (int k = 0; k < ns; ++k) {
            if (per[wi][k].empty()) continue;
            const int32_t c = (int32_t)nc++;
            for (auto& it : per[wi][k]) {
                it.done = c;
                it.dep = prev;
                it.need = prev_need;
            }
            prev = c;
            prev_need = (uint32_t)per[wi][k].size();
        }
    }
    // stage-major order; within a sweep stage grouped by (storage type, M)
    for (int k = 0; k < ns; ++k) {
        const Stage& sg = prog[k];
        const bool sweep = sg.type == ST_SWEEP || sg.type == ST_SWEEP_T;
        std::vector<std::pair<int, int>> classes;   // (dtype, M) in first-seen order
        for (size_t wi = 0; wi < which.size(); ++wi) {
            if (per[wi][k].empty()) continue;
            const BDomain& d = doms[which[wi]];
            const std::pair<int, int> c{d.dtype, sweep ? per[wi][k].front().m : 0};
            if (std::find(classes.begin(), classes.end(), c) == classes.end()) classes.push_back(c);
        }
        for (const auto& c : classes) {
            Launch L{};
            L.sweep = sweep ? 1 : 0;
            L.dtype = c.first;
            L.M = c.second;
            L.tr = sg.type == ST_SWEEP_T;
            L.off = (int64_t)P.items.size();
            for (size_t wi = 0; wi < which.size(); ++wi) {
                const BDomain& d = doms[which[wi]];
                if (per[wi][k].empty()) continue;
                if (sweep && (d.dtype != c.first || per[wi][k].front().m != c.second)) continue;
                if (!sweep && d.dtype != c.first) continue;
                for (auto& it : per[wi][k]) P.items.push_back(it);
            }
            L.count = (int64_t)P.items.size() - L.off;
            if (L.count) P.launches.push_back(L);
        }
    }
    P.ncounters = nc;
    P.npartials = partials;
}

inline std::vector<Stage> forward_program()
{
    return {{ST_SRC, 0, 0, 0},   {ST_DIR, 0, 0, 0}, {ST_SWEEP, 0, 0, 0}, {ST_DIR, 0, 0, 0},
            {ST_SWEEP, 1, 0, 0}, {ST_DIR, 0, 0, 0}, {ST_SWEEP, 2, 0, 0}, {ST_DIR, 0, 0, 0}};
}

// adjoint of one step: recompute the sweep outputs into buffers 2, 3, 4 from
// the state in buffer 0, then run the transposed stages on the gradient (1);
// each transposed sweep also forms its axis's parameter sums from the
// forward output of that axis (buffer 4, 3, 2 for z, y, x).  Written for
// domains with Dirichlet entries (each sweep runs on an overwritten copy, so
// the previous sweep's output stays intact for the sums); build_program
// drops the two inner copies of a domain without Dirichlet entries and runs
// its y and z sweeps 2 -> 3 and 3 -> 4; without sources either, it also
// drops the first copy and runs the x sweep 0 -> 2.
inline std::vector<Stage> adjoint_program()
{
    return {{ST_COPY, 0, 0, 2},       {ST_SRC, 0, 2, 2},    {ST_DIR, 0, 2, 2},          {ST_SWEEP, 0, 2, 2},
            {ST_COPY, 0, 2, 3},       {ST_DIR, 0, 3, 3},    {ST_SWEEP, 1, 3, 3},        {ST_COPY, 0, 3, 4},
            {ST_DIR, 0, 4, 4},        {ST_SWEEP, 2, 4, 4},  {ST_MASK, 0, 1, 1},         {ST_SWEEP_T, 2, 1, 1, 4},
            {ST_MASK, 0, 1, 1},       {ST_SWEEP_T, 1, 1, 1, 3}, {ST_MASK, 0, 1, 1},     {ST_SWEEP_T, 0, 1, 1, 2},
            {ST_MASK, 0, 1, 1},       {ST_SRC_T, 0, 1, 1}};
}

}  // namespace bfvm
