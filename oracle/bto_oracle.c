/*
 * FP64 CPU oracle for the per-block Boundary Termination Optimization (BTO)
 * path.  TEST INFRASTRUCTURE ONLY: nothing in the product library links,
 * loads or calls this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header or table with
 * the HIP library.
 *
 * What it computes, one particle at a time, in the order the method states it:
 *
 *  - Seeds on a uniform lattice, one per s^3 grid points (the 1:X data
 *    reduction, Section 2.3 and Section 4.1): coordinate off + s*m per axis.
 *  - One classic fourth-order Runge-Kutta step per simulation cycle
 *    (Section 2.2: in situ a particle advances one step before the field
 *    changes; Section 3.1: RK4 advection), with the velocity sampled
 *    trilinearly in space from the cycle's uniform grid and linearly in time
 *    between cycles n and n+1 (stage times t_n, t_n+h/2, t_n+h/2, t_n+h).
 *  - Boundary termination (Section 3.1): a particle whose trajectory reaches
 *    the block boundary during the interval is terminated; the interval's
 *    flow map F_{t0}^{t}(x0) (Section 2.1) is kept only for the others.
 *
 * Readings where the paper leaves the detail open (each listed with the
 * design notes):
 *  - the block is the closed box [0, n_d - 1] in cell units; points on a face
 *    are inside;
 *  - every RK4 stage point y2, y3, y4 and the step's end point are tested, in
 *    that order, and the first one outside terminates the particle in that
 *    step: flag TERMINATED, exit step n (0-based), end position = the last
 *    inside position x_n;
 *  - a non-finite velocity sample (tested right after each stage sample)
 *    flags the particle INVALID at that step, position likewise frozen;
 *  - a seed outside the box is TERMINATED at exit step 0;
 *  - the sampling cell is i_d = min(floor(p_d), n_d - 2), f_d = p_d - i_d;
 *  - the location where a terminated trajectory leaves the block (stored on
 *    the boundary, which the paper's conclusion names as future work) is
 *    taken as the point where the straight segment from the last inside
 *    position x_n to the first outside point (the stage or end point that
 *    triggered the termination) meets the box surface; seeds outside the box
 *    from the start have none.
 *
 * Grid values are handed in through a fetch callback (dense arrays of
 * f64/f32/f16/bf16 are decoded exactly by orc_dense_fetch).
 *
 * Derivatives (for the adjoint pins): the forward tangent Phi = dx_N/dx_0
 * carried through the same stages, and the discrete adjoint (reverse sweep of
 * the same stages) giving dL/dx_0 and dL/dV for L = sum_i w_i . x_i(T).
 * Both use the sampler's analytic gradient on the cell chosen by the
 * floor/clamp rule above.
 *
 * Compile: gcc -O2 -fopenmp -ffp-contract=off (no contraction, no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_VALID = 0, ORC_TERMINATED = 1, ORC_INVALID = 2 };
enum { ORC_LINEAR = 0, ORC_FROZEN = 1 };

typedef void (*orc_fetch_fn)(void *user, int32_t c, int32_t i, int32_t j, int32_t k, double out[3]);

typedef struct {
    int32_t n[3];          /* grid points per axis (>= 2)                       */
    int32_t n_steps;       /* N: steps in the interval (N+1 cycles)             */
    const double *times;   /* N+1 strictly increasing cycle times               */
    int32_t mode;          /* ORC_LINEAR or ORC_FROZEN                          */
    int32_t first_cycle;   /* fetch cycle index of times[0]                     */
    orc_fetch_fn fetch;
    void *user;
} orc_problem;

/* ------------------------------------------------------------------------ */
/* Dense grids: exact decoding of the stored values.                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n[3];
    int32_t dtype;               /* 0 f64, 1 f32, 2 binary16 bits, 3 bfloat16 bits */
    const void *const *grids;    /* one (nz, ny, nx, 3) array per cycle             */
} orc_dense;

static double dec_f16(uint16_t b)
{
    const int s = b >> 15, e = (b >> 10) & 31, m = b & 1023;
    double v;
    if (e == 0) v = ldexp((double)m, -24);
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = ldexp((double)(1024 + m), e - 25);
    return s ? -v : v;
}

static double dec_bf16(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

void orc_dense_fetch(void *user, int32_t c, int32_t i, int32_t j, int32_t k, double out[3])
{
    const orc_dense *D = (const orc_dense *)user;
    const size_t idx = 3 * ((size_t)i + (size_t)D->n[0] * ((size_t)j + (size_t)D->n[1] * (size_t)k));
    const void *g = D->grids[c];
    for (int d = 0; d < 3; ++d) {
        switch (D->dtype) {
        case 0: out[d] = ((const double *)g)[idx + d]; break;
        case 1: out[d] = (double)((const float *)g)[idx + d]; break;
        case 2: out[d] = dec_f16(((const uint16_t *)g)[idx + d]); break;
        default: out[d] = dec_bf16(((const uint16_t *)g)[idx + d]); break;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Seed lattice.                                                             */
/* ------------------------------------------------------------------------ */
int64_t orc_lattice_count(const int32_t n[3], int32_t s, const double off[3], int32_t m_out[3])
{
    int64_t P = 1;
    for (int d = 0; d < 3; ++d) {
        const int32_t m = (off[d] > n[d] - 1) ? 0 : (int32_t)floor((n[d] - 1 - off[d]) / s) + 1;
        if (m_out) m_out[d] = m;
        P *= m;
    }
    return P;
}

/* Seed id = lattice linear index, x fastest. */
void orc_seed_lattice(const int32_t n[3], int32_t s, const double off[3], double *out)
{
    int32_t m[3];
    orc_lattice_count(n, s, off, m);
    int64_t id = 0;
    for (int32_t c = 0; c < m[2]; ++c)
        for (int32_t b = 0; b < m[1]; ++b)
            for (int32_t a = 0; a < m[0]; ++a, ++id) {
                out[3 * id + 0] = off[0] + (double)s * a;
                out[3 * id + 1] = off[1] + (double)s * b;
                out[3 * id + 2] = off[2] + (double)s * c;
            }
}

/* ------------------------------------------------------------------------ */
/* Trilinear sampling in space, linear in time.                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t cell[3];
    double f[3];
} orc_cell;

static void locate(const int32_t n[3], const double p[3], orc_cell *L)
{
    for (int d = 0; d < 3; ++d) {
        double fl = floor(p[d]);
        int32_t i = (int32_t)fl;
        if (i > n[d] - 2) i = n[d] - 2;
        if (i < 0) i = 0; /* only reached for points the caller already rejected */
        L->cell[d] = i;
        L->f[d] = p[d] - (double)i;
    }
}

/* weight of corner (a,b,c) and its derivative along each axis */
static void corner_weight(const orc_cell *L, int a, int b, int c, double *w, double dw[3])
{
    const double wx = a ? L->f[0] : 1.0 - L->f[0];
    const double wy = b ? L->f[1] : 1.0 - L->f[1];
    const double wz = c ? L->f[2] : 1.0 - L->f[2];
    const double sx = a ? 1.0 : -1.0, sy = b ? 1.0 : -1.0, sz = c ? 1.0 : -1.0;
    *w = wx * wy * wz;
    if (dw) {
        dw[0] = sx * wy * wz;
        dw[1] = wx * sy * wz;
        dw[2] = wx * wy * sz;
    }
}

/* T(V_c, p) and, if grad != NULL, dT/dp (grad[r*3+col] = d v_r / d p_col). */
static void trilinear(const orc_problem *P, int32_t c, const orc_cell *L, double v[3], double *grad)
{
    v[0] = v[1] = v[2] = 0.0;
    if (grad) memset(grad, 0, 9 * sizeof(double));
    for (int cc = 0; cc < 2; ++cc)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                double V[3], w, dw[3];
                P->fetch(P->user, P->first_cycle + c, L->cell[0] + a, L->cell[1] + b, L->cell[2] + cc, V);
                corner_weight(L, a, b, cc, &w, grad ? dw : NULL);
                for (int r = 0; r < 3; ++r) {
                    v[r] += w * V[r];
                    if (grad)
                        for (int q = 0; q < 3; ++q) grad[3 * r + q] += dw[q] * V[r];
                }
            }
}

/* S(p, n, theta): theta in {0, 1/2, 1}; FROZEN mode always reads cycle n. */
static void sample(const orc_problem *P, int32_t n, double theta, const double p[3], double v[3], double *grad)
{
    orc_cell L;
    locate(P->n, p, &L);
    if (P->mode == ORC_FROZEN || theta == 0.0) {
        trilinear(P, n, &L, v, grad);
        return;
    }
    if (theta == 1.0) {
        trilinear(P, n + 1, &L, v, grad);
        return;
    }
    double v0[3], v1[3], g0[9], g1[9];
    trilinear(P, n, &L, v0, grad ? g0 : NULL);
    trilinear(P, n + 1, &L, v1, grad ? g1 : NULL);
    for (int r = 0; r < 3; ++r) v[r] = (1.0 - theta) * v0[r] + theta * v1[r];
    if (grad)
        for (int q = 0; q < 9; ++q) grad[q] = (1.0 - theta) * g0[q] + theta * g1[q];
}

int orc_sample(const orc_problem *P, int32_t n, double theta, const double p[3], double v[3], double grad[9])
{
    sample(P, n, theta, p, v, grad);
    return 0;
}

static int inside(const int32_t n[3], const double p[3])
{
    for (int d = 0; d < 3; ++d)
        if (!(p[d] >= 0.0 && p[d] <= (double)(n[d] - 1))) return 0;
    return 1;
}

static double face_distance(const int32_t n[3], const double p[3])
{
    double m = INFINITY;
    for (int d = 0; d < 3; ++d) {
        double a = fabs(p[d]), b = fabs((double)(n[d] - 1) - p[d]);
        if (a < m) m = a;
        if (b < m) m = b;
    }
    return m;
}

static int finite3(const double v[3])
{
    return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
}

static void matmul3(const double A[9], const double B[9], double C[9])
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}

static uint64_t mix(uint64_t h, int64_t v)
{
    h ^= (uint64_t)v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    return h * 0x100000001b3ull;
}

/* ------------------------------------------------------------------------ */
/* One particle through the interval.                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    double x[3];
    int flag;
    int32_t exit;
    double margin;
    uint64_t sig;      /* hash of every stage's sampling cell */
    double phi[9];     /* tangent dx/dx0                        */
    double *stages;    /* optional: 4 stage points per step (N x 4 x 3) */
    double face[3];    /* exit point on the box surface (NaN unless terminated in a step) */
    double face_cond;  /* |y - x|_inf / |y_a - x_a| of that segment (NaN likewise) */
} orc_track;

/* Where the segment from the inside point x to the outside point y first meets
 * the box [0, n-1]^3: the smallest fraction tau over the violated faces (ties
 * to the lowest axis), that axis set exactly to its face value.  cond is the
 * factor by which errors in x and y can grow in the exit point. */
static void exit_face(const int32_t n[3], const double x[3], const double y[3], double f[3], double *cond)
{
    double tau = INFINITY, fv = 0.0;
    int axis = -1;
    for (int d = 0; d < 3; ++d) {
        const double hi = (double)(n[d] - 1);
        double t = INFINITY, v = 0.0;
        if (y[d] < 0.0) {
            t = (0.0 - x[d]) / (y[d] - x[d]);
            v = 0.0;
        } else if (y[d] > hi) {
            t = (hi - x[d]) / (y[d] - x[d]);
            v = hi;
        }
        if (t < tau) {
            tau = t;
            axis = d;
            fv = v;
        }
    }
    double span = 0.0;
    for (int d = 0; d < 3; ++d) {
        f[d] = x[d] + tau * (y[d] - x[d]);
        const double hi = (double)(n[d] - 1);
        if (f[d] < 0.0) f[d] = 0.0;
        if (f[d] > hi) f[d] = hi;
        if (fabs(y[d] - x[d]) > span) span = fabs(y[d] - x[d]);
    }
    f[axis] = fv;
    *cond = span / fabs(y[axis] - x[axis]);
}

static const double STAGE_THETA[4] = {0.0, 0.5, 0.5, 1.0};

static void advect_one(const orc_problem *P, const double x0[3], int want_phi, orc_track *T)
{
    const int32_t N = P->n_steps;
    double x[3] = {x0[0], x0[1], x0[2]};
    double phi[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    uint64_t sig = 0xcbf29ce484222325ull;
    double margin = face_distance(P->n, x);
    T->face[0] = T->face[1] = T->face[2] = NAN;
    T->face_cond = NAN;
    int flag = ORC_VALID;
    int32_t exit = N;
    if (!inside(P->n, x)) {
        flag = ORC_TERMINATED;
        exit = 0;
    }
    for (int32_t s = 0; s < N && flag == ORC_VALID; ++s) {
        const double h = P->times[s + 1] - P->times[s];
        const double a[4] = {0.0, 0.5 * h, 0.5 * h, h};
        double y[4][3], k[4][3], G[4][9], dy[4][9];
        int event = ORC_VALID;
        for (int st = 0; st < 4; ++st) {
            if (st == 0) {
                memcpy(y[0], x, sizeof x);
                if (want_phi) memcpy(dy[0], phi, sizeof phi);
            } else {
                for (int d = 0; d < 3; ++d) y[st][d] = x[d] + a[st] * k[st - 1][d];
                const double fd = face_distance(P->n, y[st]);
                if (fd < margin) margin = fd;
                if (!inside(P->n, y[st])) {
                    event = ORC_TERMINATED;
                    exit_face(P->n, x, y[st], T->face, &T->face_cond);
                    break;
                }
                if (want_phi) {
                    double Gd[9];
                    matmul3(G[st - 1], dy[st - 1], Gd);
                    for (int q = 0; q < 9; ++q) dy[st][q] = phi[q] + a[st] * Gd[q];
                }
            }
            if (T->stages) memcpy(T->stages + ((size_t)s * 4 + st) * 3, y[st], 3 * sizeof(double));
            orc_cell L;
            locate(P->n, y[st], &L);
            for (int d = 0; d < 3; ++d) sig = mix(sig, L.cell[d]);
            sample(P, s, STAGE_THETA[st], y[st], k[st], want_phi ? G[st] : NULL);
            if (!finite3(k[st])) { event = ORC_INVALID; break; }
        }
        if (event == ORC_VALID) {
            double xn[3];
            for (int d = 0; d < 3; ++d)
                xn[d] = x[d] + (h / 6.0) * (k[0][d] + 2.0 * k[1][d] + 2.0 * k[2][d] + k[3][d]);
            const double fd = face_distance(P->n, xn);
            if (fd < margin) margin = fd;
            if (!inside(P->n, xn)) {
                event = ORC_TERMINATED;
                exit_face(P->n, x, xn, T->face, &T->face_cond);
            } else {
                if (want_phi) {
                    double Gd[4][9];
                    for (int st = 0; st < 4; ++st) matmul3(G[st], dy[st], Gd[st]);
                    for (int q = 0; q < 9; ++q)
                        phi[q] = phi[q] + (h / 6.0) * (Gd[0][q] + 2.0 * Gd[1][q] + 2.0 * Gd[2][q] + Gd[3][q]);
                }
                memcpy(x, xn, sizeof x);
            }
        }
        if (event != ORC_VALID) {
            flag = event;
            exit = s;
        }
    }
    memcpy(T->x, x, sizeof x);
    T->flag = flag;
    T->exit = exit;
    T->margin = margin;
    T->sig = sig;
    memcpy(T->phi, phi, sizeof phi);
}

/* Threads of one call: nthreads if positive, else the OpenMP default.  Passed
 * to the call's own parallel region (num_threads), so no call changes the
 * thread count of later calls. */
static int call_threads(int32_t nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? (int)nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* Flow map of P seeds: end position, flag, exit step; optional face margin,
 * stage-cell signature and tangent Phi (row-major dx_end/dx0). */
int orc_flowmap(const orc_problem *P, int64_t np, const double *seeds, double *end, uint8_t *flag,
                int32_t *exit_step, double *margin, uint64_t *cellsig, double *jac, double *face,
                double *face_cond, int32_t nthreads)
{
    if (!P || !P->times || !P->fetch || P->n_steps < 0) return -1;
    for (int d = 0; d < 3; ++d)
        if (P->n[d] < 2) return -1;
    for (int32_t s = 0; s < P->n_steps; ++s)
        if (!(P->times[s + 1] > P->times[s])) return -1;
    const int nt = call_threads(nthreads);
    (void)nt;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt)
    for (int64_t p = 0; p < np; ++p) {
        orc_track T;
        T.stages = NULL;
        advect_one(P, seeds + 3 * p, jac != NULL, &T);
        memcpy(end + 3 * p, T.x, 3 * sizeof(double));
        flag[p] = (uint8_t)T.flag;
        exit_step[p] = T.exit;
        if (margin) margin[p] = T.margin;
        if (cellsig) cellsig[p] = T.sig;
        if (jac) memcpy(jac + 9 * p, T.phi, 9 * sizeof(double));
        if (face) memcpy(face + 3 * p, T.face, 3 * sizeof(double));
        if (face_cond) face_cond[p] = T.face_cond;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint of the interval for L = sum_p cot_p . x_p(T) over VALID  */
/* particles (terminated and invalid particles contribute nothing).          */
/* grad_grid (optional): N+1 dense FP64 grids (nz, ny, nx, 3) that receive   */
/* dL/dV_c; when given the sweep runs on one thread.                         */
/* ------------------------------------------------------------------------ */
static void scatter_grid(const orc_problem *P, double *const *gg, int32_t c, const double y[3], double coef,
                         const double lam[3])
{
    if (!gg || coef == 0.0) return;
    orc_cell L;
    locate(P->n, y, &L);
    double *g = gg[c];
    for (int cc = 0; cc < 2; ++cc)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                double w;
                corner_weight(&L, a, b, cc, &w, NULL);
                const size_t idx = 3 * ((size_t)(L.cell[0] + a) +
                                        (size_t)P->n[0] * ((size_t)(L.cell[1] + b) + (size_t)P->n[1] * (size_t)(L.cell[2] + cc)));
                for (int r = 0; r < 3; ++r) g[idx + r] += coef * w * lam[r];
            }
}

static void matTvec(const double G[9], const double v[3], double out[3])
{
    for (int q = 0; q < 3; ++q) out[q] = G[q] * v[0] + G[3 + q] * v[1] + G[6 + q] * v[2];
}

int orc_adjoint(const orc_problem *P, int64_t np, const double *seeds, const double *cot, double *grad_seed,
                double *const *grad_grid, int32_t nthreads)
{
    if (!P || !P->times || !P->fetch || P->n_steps < 0) return -1;
    const int32_t N = P->n_steps;
    const int nt = grad_grid ? 1 : call_threads(nthreads);
    (void)nt;
#pragma omp parallel num_threads(nt)
    {
        double *stages = (double *)malloc(sizeof(double) * 12 * (size_t)(N > 0 ? N : 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < np; ++p) {
            orc_track T;
            T.stages = stages;
            advect_one(P, seeds + 3 * p, 0, &T);
            double lam[3] = {0, 0, 0};
            if (T.flag == ORC_VALID) {
                memcpy(lam, cot + 3 * p, sizeof lam);
                for (int32_t s = N - 1; s >= 0; --s) {
                    const double h = P->times[s + 1] - P->times[s];
                    const double *y = stages + (size_t)s * 12;
                    double G[4][9], kk[3];
                    for (int st = 0; st < 4; ++st) sample(P, s, STAGE_THETA[st], y + 3 * st, kk, G[st]);
                    double lk[4][3], ly[4][3];
                    for (int r = 0; r < 3; ++r) lk[3][r] = (h / 6.0) * lam[r];
                    matTvec(G[3], lk[3], ly[3]);
                    for (int r = 0; r < 3; ++r) lk[2][r] = (h / 3.0) * lam[r] + h * ly[3][r];
                    matTvec(G[2], lk[2], ly[2]);
                    for (int r = 0; r < 3; ++r) lk[1][r] = (h / 3.0) * lam[r] + (0.5 * h) * ly[2][r];
                    matTvec(G[1], lk[1], ly[1]);
                    for (int r = 0; r < 3; ++r) lk[0][r] = (h / 6.0) * lam[r] + (0.5 * h) * ly[1][r];
                    matTvec(G[0], lk[0], ly[0]);
                    if (grad_grid) {
                        for (int st = 0; st < 4; ++st) {
                            const double th = (P->mode == ORC_FROZEN) ? 0.0 : STAGE_THETA[st];
                            scatter_grid(P, grad_grid, s, y + 3 * st, 1.0 - th, lk[st]);
                            scatter_grid(P, grad_grid, s + 1, y + 3 * st, th, lk[st]);
                        }
                    }
                    for (int r = 0; r < 3; ++r) lam[r] = lam[r] + ly[0][r] + ly[1][r] + ly[2][r] + ly[3][r];
                }
            }
            memcpy(grad_seed + 3 * p, lam, sizeof lam);
        }
        free(stages);
    }
    return 0;
}
