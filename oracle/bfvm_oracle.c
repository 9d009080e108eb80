/*
 * Plain FP64 CPU oracle for the BioFVM-B diffusion-decay time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and is
 * loaded by the test-suite, by the smoke check and by the CPU-baseline leg of
 * the benchmark.  The GPU library never links, includes or calls it, and it
 * shares no code, header or table with the GPU path.
 *
 * It is deliberately slow and literal: IEEE double, divisions written as
 * divisions (build with -ffp-contract=off, no fast-math), one loop nest per
 * stage of the method.  Lines are visited "across lines" (the inner loop runs
 * over neighbouring systems, as in the vectorised x/y solvers of Sec. 3.3,
 * Algorithms 2 and 3), which only changes the order in which independent
 * systems are touched, never the arithmetic inside one system.
 *
 * Field layout: u[((z*ny + y)*nx + x)*S + s]  (substrate innermost, then x).
 *
 * Method, by step (paper section / equation):
 *   O1  r = dt*D_s/h_a^2, beta = dt*lambda_s/3            (App. A, coefficients a_i, b_i, c_i)
 *   O2  tridiagonal A: off-diagonals -r, diagonal 1+r+beta at both ends and
 *       1+2r+beta inside; 1+beta when the line has one voxel (App. A, b_i)
 *   O3  Thomas factors denom_i and c'_i                     (App. A, eqs. for constant_c and denom)
 *   O4  forward elimination / back substitution of one line (Sec. 2, TDMA; Sec. 2.1 Eq. 2)
 *   O5  bulk source/sink, implicit                          (Sec. 5.3, production and uptake by cells)
 *   O6  Dirichlet overwrite                                 (Sec. 2, the 7-stage solver)
 *   O7  x, y and z sweeps                                   (Sec. 2, Algorithm 1)
 *   O8  one step = Src, Dir, X, Dir, Y, Dir, Z, Dir         (Sec. 2, the 7-stage solver)
 *   O9  adjoint of O8 (reverse order, transposed Thomas) with per-substrate
 *       gradients of D and lambda (not in the paper; derived from O2)
 *
 * Readings where the paper is silent or garbled:
 *   - App. A writes the system as "a_i + b_i x_i + c_i = d_i" with a_i = +r;
 *     the symmetric zero-flux finite-volume matrix has -r on both
 *     off-diagonals, and the "+r" is the constant of the forward axpy.
 *   - The four Dirichlet applications are interleaved with the three sweeps
 *     (before x, y, z and after z); the source term is applied once per step
 *     before the first Dirichlet application.
 *   - Source entries: u <- (u + dt*sum(S*rho)) / (1 + dt*sum(S+U)), duplicate
 *     voxels merged additively.
 *   - Dirichlet entries are applied in list order; an inactive entry does
 *     nothing, so the last active entry of a (voxel, substrate) wins.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-5)

/* Number of OpenMP threads the sweeps use (reported with CPU timings). */
int oracle_threads(void) { return omp_get_max_threads(); }

/* Thread count for the following calls (baseline timing at one thread and at
 * all host threads); n < 1 leaves it unchanged. */
void oracle_set_threads(int n)
{
    if (n >= 1) omp_set_num_threads(n);
}

/* ---------------------------------------------------------------- O1-O3 */

/* Thomas factors of the (n x n) matrix of O2 with parameters r, beta.
 * denom[0..n-1]; cprime[0..n-2] (cprime[n-1] is set to 0, it is never used). */
void oracle_factor(int64_t n, double r, double beta, double* denom, double* cprime)
{
    for (int64_t i = 0; i < n; ++i) {
        double b;
        if (n == 1)
            b = 1.0 + beta;
        else if (i == 0 || i == n - 1)
            b = 1.0 + r + beta;
        else
            b = 1.0 + 2.0 * r + beta;
        double a = -r;     /* sub-diagonal entry of row i   */
        double c = -r;     /* super-diagonal entry of row i */
        if (i == 0)
            denom[i] = b;
        else
            denom[i] = b - a * cprime[i - 1];
        cprime[i] = (i < n - 1) ? c / denom[i] : 0.0;
    }
}

/* --------------------------------------------------------------- O4, O7 */

/* The field seen as [outer][n][inner]: line (o, j) has elements
 * u[(o*n + i)*inner + j], i = 0..n-1, and belongs to substrate j % S.
 *   x sweep: outer = nz*ny, n = nx, inner = S
 *   y sweep: outer = nz,    n = ny, inner = nx*S
 *   z sweep: outer = 1,     n = nz, inner = ny*nx*S                        */
static void axis_view(int axis, int64_t nx, int64_t ny, int64_t nz, int64_t S,
                      int64_t* outer, int64_t* n, int64_t* inner)
{
    if (axis == 0) { *outer = nz * ny; *n = nx; *inner = S; }
    else if (axis == 1) { *outer = nz; *n = ny; *inner = nx * S; }
    else { *outer = 1; *n = nz; *inner = ny * nx * S; }
}

#define JBLOCK 512

/* Solve every line of one axis in place with precomputed factors
 * denom[s*n + i], cprime[s*n + i]. */
static void sweep_with_factors(double* u, int64_t outer, int64_t n, int64_t inner, int64_t S,
                               const double* r, const double* denom, const double* cprime)
{
    int64_t nblk = (inner + JBLOCK - 1) / JBLOCK;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t o = 0; o < outer; ++o) {
        for (int64_t jb = 0; jb < nblk; ++jb) {
            int64_t j0 = jb * JBLOCK;
            int64_t j1 = j0 + JBLOCK < inner ? j0 + JBLOCK : inner;
            double* base = u + o * n * inner;
            /* forward elimination */
            for (int64_t j = j0; j < j1; ++j) {
                int64_t s = j % S;
                base[j] = base[j] / denom[s * n + 0];
            }
            for (int64_t i = 1; i < n; ++i) {
                for (int64_t j = j0; j < j1; ++j) {
                    int64_t s = j % S;
                    base[i * inner + j] = (base[i * inner + j] + r[s] * base[(i - 1) * inner + j])
                                          / denom[s * n + i];
                }
            }
            /* back substitution */
            for (int64_t i = n - 2; i >= 0; --i) {
                for (int64_t j = j0; j < j1; ++j) {
                    int64_t s = j % S;
                    base[i * inner + j] = base[i * inner + j] - cprime[s * n + i] * base[(i + 1) * inner + j];
                }
            }
        }
    }
}

static int factors_for_axis(int axis, int64_t nx, int64_t ny, int64_t nz, int64_t S,
                            const double* h, const double* D, const double* lambda, double dt,
                            double* r, double** denom, double** cprime)
{
    int64_t outer, n, inner;
    axis_view(axis, nx, ny, nz, S, &outer, &n, &inner);
    *denom = (double*)malloc(sizeof(double) * (size_t)(n * S));
    *cprime = (double*)malloc(sizeof(double) * (size_t)(n * S));
    if (!*denom || !*cprime) {
        free(*denom);
        free(*cprime);
        return ORACLE_ENOMEM;
    }
    for (int64_t s = 0; s < S; ++s) {
        r[s] = dt * D[s] / (h[axis] * h[axis]);       /* O1 */
        double beta = dt * lambda[s] / 3.0;            /* O1 */
        oracle_factor(n, r[s], beta, *denom + s * n, *cprime + s * n);
    }
    return ORACLE_OK;
}

/* One sweep (axis 0 = x, 1 = y, 2 = z) of every line and substrate, in place. */
int oracle_sweep(double* u, int64_t nx, int64_t ny, int64_t nz, int32_t nsub,
                 const double* h, const double* D, const double* lambda, double dt, int32_t axis)
{
    if (!u || nx < 1 || ny < 1 || nz < 1 || nsub < 1 || axis < 0 || axis > 2)
        return ORACLE_EINVAL;
    int64_t S = nsub, outer, n, inner;
    axis_view(axis, nx, ny, nz, S, &outer, &n, &inner);
    double* r = (double*)malloc(sizeof(double) * (size_t)S);
    double *denom = NULL, *cprime = NULL;
    if (!r) return ORACLE_ENOMEM;
    int st = factors_for_axis(axis, nx, ny, nz, S, h, D, lambda, dt, r, &denom, &cprime);
    if (st == ORACLE_OK)
        sweep_with_factors(u, outer, n, inner, S, r, denom, cprime);
    free(r);
    free(denom);
    free(cprime);
    return st;
}

/* ------------------------------------------------------------------ O5 */

typedef struct {
    const int64_t* voxel;
    int64_t idx;
} src_key;

static int cmp_src_key(const void* a, const void* b)
{
    const src_key* ka = (const src_key*)a;
    const src_key* kb = (const src_key*)b;
    int64_t va = ka->voxel[ka->idx], vb = kb->voxel[kb->idx];
    if (va != vb) return va < vb ? -1 : 1;
    return ka->idx < kb->idx ? -1 : (ka->idx > kb->idx);
}

/* Merged source terms: for every distinct voxel, P = dt*sum_k S_k*rho_k and
 * Q = 1 + dt*sum_k (S_k + U_k), per substrate.  Returns the number of
 * distinct voxels; mvox[m], P[m*S + s], Q[m*S + s] are allocated here. */
static int64_t merge_sources(int64_t count, int64_t S, const int64_t* voxel,
                             const double* secretion, const double* saturation, const double* uptake,
                             double dt, int64_t** mvox, double** P, double** Q)
{
    src_key* keys = (src_key*)malloc(sizeof(src_key) * (size_t)(count > 0 ? count : 1));
    *mvox = (int64_t*)malloc(sizeof(int64_t) * (size_t)(count > 0 ? count : 1));
    *P = (double*)malloc(sizeof(double) * (size_t)(count > 0 ? count * S : 1));
    *Q = (double*)malloc(sizeof(double) * (size_t)(count > 0 ? count * S : 1));
    if (!keys || !*mvox || !*P || !*Q) {
        free(keys); free(*mvox); free(*P); free(*Q);
        return -1;
    }
    for (int64_t k = 0; k < count; ++k) { keys[k].voxel = voxel; keys[k].idx = k; }
    qsort(keys, (size_t)count, sizeof(src_key), cmp_src_key);
    int64_t m = -1;
    int64_t last = -1;
    for (int64_t t = 0; t < count; ++t) {
        int64_t k = keys[t].idx;
        if (voxel[k] != last) {
            ++m;
            last = voxel[k];
            (*mvox)[m] = last;
            for (int64_t s = 0; s < S; ++s) { (*P)[m * S + s] = 0.0; (*Q)[m * S + s] = 0.0; }
        }
        for (int64_t s = 0; s < S; ++s) {
            (*P)[m * S + s] += secretion[k * S + s] * saturation[k * S + s];
            (*Q)[m * S + s] += secretion[k * S + s] + uptake[k * S + s];
        }
    }
    free(keys);
    for (int64_t i = 0; i <= m; ++i)
        for (int64_t s = 0; s < S; ++s) {
            (*P)[i * S + s] = dt * (*P)[i * S + s];
            (*Q)[i * S + s] = 1.0 + dt * (*Q)[i * S + s];
        }
    return m + 1;
}

int oracle_source(double* u, int32_t nsub, int64_t count, const int64_t* voxel,
                  const double* secretion, const double* saturation, const double* uptake, double dt)
{
    if (count < 0 || nsub < 1) return ORACLE_EINVAL;
    if (count == 0) return ORACLE_OK;
    int64_t S = nsub;
    int64_t* mvox; double *P, *Q;
    int64_t m = merge_sources(count, S, voxel, secretion, saturation, uptake, dt, &mvox, &P, &Q);
    if (m < 0) return ORACLE_ENOMEM;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t s = 0; s < S; ++s) {
            double* p = u + mvox[i] * S + s;
            *p = (*p + P[i * S + s]) / Q[i * S + s];
        }
    free(mvox); free(P); free(Q);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ O6 */

int oracle_dirichlet(double* u, int32_t nsub, int64_t count, const int64_t* voxel,
                     const double* value, const uint8_t* active)
{
    if (count < 0 || nsub < 1) return ORACLE_EINVAL;
    int64_t S = nsub;
    for (int64_t k = 0; k < count; ++k)
        for (int64_t s = 0; s < S; ++s)
            if (active[k * S + s])
                u[voxel[k] * S + s] = value[k * S + s];
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ O8 */

/* nsteps full LOD steps in place.  h[3] = (hx, hy, hz); D, lambda: [nsub]. */
int oracle_step(double* u, int64_t nx, int64_t ny, int64_t nz, int32_t nsub,
                const double* h, const double* D, const double* lambda, double dt,
                int64_t nsrc, const int64_t* src_voxel, const double* secretion,
                const double* saturation, const double* uptake,
                int64_t ndir, const int64_t* dir_voxel, const double* dir_value, const uint8_t* dir_active,
                int64_t nsteps)
{
    if (!u || nx < 1 || ny < 1 || nz < 1 || nsub < 1 || nsteps < 0) return ORACLE_EINVAL;
    int64_t S = nsub;
    double* r[3] = {NULL, NULL, NULL};
    double* denom[3] = {NULL, NULL, NULL};
    double* cprime[3] = {NULL, NULL, NULL};
    int st = ORACLE_OK;
    for (int a = 0; a < 3 && st == ORACLE_OK; ++a) {
        r[a] = (double*)malloc(sizeof(double) * (size_t)S);
        if (!r[a]) { st = ORACLE_ENOMEM; break; }
        st = factors_for_axis(a, nx, ny, nz, S, h, D, lambda, dt, r[a], &denom[a], &cprime[a]);
    }
    int64_t m = 0;
    int64_t* mvox = NULL; double *P = NULL, *Q = NULL;
    if (st == ORACLE_OK && nsrc > 0) {
        m = merge_sources(nsrc, S, src_voxel, secretion, saturation, uptake, dt, &mvox, &P, &Q);
        if (m < 0) { st = ORACLE_ENOMEM; m = 0; }
    }
    for (int64_t t = 0; t < nsteps && st == ORACLE_OK; ++t) {
        for (int64_t i = 0; i < m; ++i)                       /* Src */
            for (int64_t s = 0; s < S; ++s) {
                double* p = u + mvox[i] * S + s;
                *p = (*p + P[i * S + s]) / Q[i * S + s];
            }
        for (int a = 0; a < 3; ++a) {
            oracle_dirichlet(u, nsub, ndir, dir_voxel, dir_value, dir_active);   /* Dir */
            int64_t outer, n, inner;
            axis_view(a, nx, ny, nz, S, &outer, &n, &inner);
            sweep_with_factors(u, outer, n, inner, S, r[a], denom[a], cprime[a]); /* X, Y, Z */
        }
        oracle_dirichlet(u, nsub, ndir, dir_voxel, dir_value, dir_active);       /* Dir */
    }
    for (int a = 0; a < 3; ++a) { free(r[a]); free(denom[a]); free(cprime[a]); }
    free(mvox); free(P); free(Q);
    return st;
}

/* ------------------------------------------------------------------ O9 */

/* Transposed Thomas solve of one line (A = L U with L lower bidiagonal
 * (diag denom, sub -r) and U unit upper bidiagonal (super c')): solve
 * U^T w = g, then L^T y = w.  In place on g (elements g[i*inner]). */
static void transposed_solve(double* g, int64_t inner, int64_t n, double r,
                             const double* denom, const double* cprime)
{
    for (int64_t i = 1; i < n; ++i)
        g[i * inner] = g[i * inner] - cprime[i - 1] * g[(i - 1) * inner];
    g[(n - 1) * inner] = g[(n - 1) * inner] / denom[n - 1];
    for (int64_t i = n - 2; i >= 0; --i)
        g[i * inner] = (g[i * inner] + r * g[(i + 1) * inner]) / denom[i];
}

/* Adjoint of one sweep: g <- A^{-T} g along every line, and per substrate
 *   Gr[s] -= sum over lines of y^T (L_N x),  Gb[s] -= sum over lines of y^T x,
 * where x is the sweep's forward output and L_N the zero-flux Laplacian. */
static void sweep_adjoint(double* g, const double* x, int64_t outer, int64_t n, int64_t inner, int64_t S,
                          const double* r, const double* denom, const double* cprime,
                          double* Gr, double* Gb)
{
    for (int64_t o = 0; o < outer; ++o) {
        for (int64_t j = 0; j < inner; ++j) {
            int64_t s = j % S;
            double* gl = g + o * n * inner + j;
            const double* xl = x + o * n * inner + j;
            transposed_solve(gl, inner, n, r[s], denom + s * n, cprime + s * n);
            double yLx = 0.0, yx = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                double Lx;
                if (n == 1) Lx = 0.0;
                else if (i == 0) Lx = xl[0] - xl[inner];
                else if (i == n - 1) Lx = xl[i * inner] - xl[(i - 1) * inner];
                else Lx = 2.0 * xl[i * inner] - xl[(i - 1) * inner] - xl[(i + 1) * inner];
                yLx += gl[i * inner] * Lx;
                yx += gl[i * inner] * xl[i * inner];
            }
            Gr[s] -= yLx;
            Gb[s] -= yx;
        }
    }
}

static void dirichlet_mask(double* g, int64_t S, int64_t count, const int64_t* voxel, const uint8_t* active)
{
    for (int64_t k = 0; k < count; ++k)
        for (int64_t s = 0; s < S; ++s)
            if (active[k * S + s]) g[voxel[k] * S + s] = 0.0;
}

/* One reverse step.  u_in: the field at the start of the forward step;
 * g: on entry dL/du after the step, on exit dL/du before it;
 * gD, gL: [nsub] accumulators, incremented by this step's dL/dD, dL/dlambda. */
int oracle_adjoint_step(const double* u_in, double* g, double* gD, double* gL,
                        int64_t nx, int64_t ny, int64_t nz, int32_t nsub,
                        const double* h, const double* D, const double* lambda, double dt,
                        int64_t nsrc, const int64_t* src_voxel, const double* secretion,
                        const double* saturation, const double* uptake,
                        int64_t ndir, const int64_t* dir_voxel, const double* dir_value, const uint8_t* dir_active)
{
    if (!u_in || !g || nx < 1 || ny < 1 || nz < 1 || nsub < 1) return ORACLE_EINVAL;
    int64_t S = nsub, V = nx * ny * nz, N = V * S;
    double* xs[3];
    double* r[3] = {NULL, NULL, NULL};
    double* denom[3] = {NULL, NULL, NULL};
    double* cprime[3] = {NULL, NULL, NULL};
    double* Gr = (double*)calloc((size_t)(3 * S), sizeof(double));
    double* Gb = (double*)calloc((size_t)(3 * S), sizeof(double));
    double* w = (double*)malloc(sizeof(double) * (size_t)N);
    for (int a = 0; a < 3; ++a) xs[a] = (double*)malloc(sizeof(double) * (size_t)N);
    int st = (Gr && Gb && w && xs[0] && xs[1] && xs[2]) ? ORACLE_OK : ORACLE_ENOMEM;
    for (int a = 0; a < 3 && st == ORACLE_OK; ++a) {
        r[a] = (double*)malloc(sizeof(double) * (size_t)S);
        if (!r[a]) { st = ORACLE_ENOMEM; break; }
        st = factors_for_axis(a, nx, ny, nz, S, h, D, lambda, dt, r[a], &denom[a], &cprime[a]);
    }
    int64_t m = 0;
    int64_t* mvox = NULL; double *P = NULL, *Q = NULL;
    if (st == ORACLE_OK && nsrc > 0) {
        m = merge_sources(nsrc, S, src_voxel, secretion, saturation, uptake, dt, &mvox, &P, &Q);
        if (m < 0) { st = ORACLE_ENOMEM; m = 0; }
    }
    if (st == ORACLE_OK) {
        /* forward recomputation, keeping each sweep's output */
        memcpy(w, u_in, sizeof(double) * (size_t)N);
        for (int64_t i = 0; i < m; ++i)
            for (int64_t s = 0; s < S; ++s) {
                double* p = w + mvox[i] * S + s;
                *p = (*p + P[i * S + s]) / Q[i * S + s];
            }
        for (int a = 0; a < 3; ++a) {
            oracle_dirichlet(w, nsub, ndir, dir_voxel, dir_value, dir_active);
            int64_t outer, n, inner;
            axis_view(a, nx, ny, nz, S, &outer, &n, &inner);
            sweep_with_factors(w, outer, n, inner, S, r[a], denom[a], cprime[a]);
            memcpy(xs[a], w, sizeof(double) * (size_t)N);
        }
        /* reverse: Dir^T, Z^T, Dir^T, Y^T, Dir^T, X^T, Dir^T, Src^T */
        for (int a = 2; a >= 0; --a) {
            dirichlet_mask(g, S, ndir, dir_voxel, dir_active);
            int64_t outer, n, inner;
            axis_view(a, nx, ny, nz, S, &outer, &n, &inner);
            sweep_adjoint(g, xs[a], outer, n, inner, S, r[a], denom[a], cprime[a], Gr + a * S, Gb + a * S);
        }
        dirichlet_mask(g, S, ndir, dir_voxel, dir_active);
        for (int64_t i = 0; i < m; ++i)
            for (int64_t s = 0; s < S; ++s)
                g[mvox[i] * S + s] = g[mvox[i] * S + s] / Q[i * S + s];
        /* dr_a/dD = dt/h_a^2, dbeta/dlambda = dt/3 */
        for (int64_t s = 0; s < S; ++s) {
            for (int a = 0; a < 3; ++a) {
                gD[s] += dt / (h[a] * h[a]) * Gr[a * S + s];
                gL[s] += dt / 3.0 * Gb[a * S + s];
            }
        }
    }
    for (int a = 0; a < 3; ++a) { free(xs[a]); free(r[a]); free(denom[a]); free(cprime[a]); }
    free(Gr); free(Gb); free(w);
    free(mvox); free(P); free(Q);
    return st;
}
