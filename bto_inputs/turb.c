/*
 * Input generator: divergence-free random Fourier-mode turbulence on a block's
 * grid, evaluated in FP64.  Input preparation only (no advection arithmetic).
 *
 *   u(g, t_c) = sum_m a_m * Re( e^{i kx_m gx} e^{i ky_m gy} e^{i kz_m gz} e^{i psi_m(c)} )
 *
 * The per-axis exponentials and the per-cycle phase factors are tables built
 * once by the caller; every grid value is then a fixed sequence of FP64
 * multiplies and adds, written out below in one order and compiled without
 * contraction (-ffp-contract=off), so that the whole-grid routine and the
 * single-point routine return bit-identical values.
 *
 * Layout: tables are mode-major (table[m * n_axis + index]); the grid is
 * (nz, ny, nx, 3) with x fastest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny, nz, M, C;
    const double *exr, *exi, *eyr, *eyi, *ezr, *ezi; /* M x n_axis            */
    const double *pr, *pi;                           /* C x M (cycle-major)   */
    const double *amp;                               /* M x 3                 */
    int32_t dtype; /* storage rounding for turb_fetch: 0 f64, 1 f32, 2 f16, 3 bf16 */
} turb_tables;

/* Round-to-nearest-even to `bits` significant bits with a minimum exponent
 * `emin` (values below 2^emin are rounded on the fixed quantum 2^(emin-bits+1)). */
static double round_sig(double x, int bits, int emin)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    double m = frexp(x, &e);           /* x = m 2^e, 0.5 <= |m| < 1 */
    int ex = e - 1;                    /* x = 1.m 2^ex               */
    if (ex < emin) ex = emin;
    int q = ex - (bits - 1);           /* quantum exponent           */
    (void)m;
    return ldexp(rint(ldexp(x, -q)), q);
}

static double store_round(double x, int dtype)
{
    switch (dtype) {
    case 1: return (double)(float)x;
    case 2: return round_sig(x, 11, -14);   /* binary16 */
    case 3: return round_sig(x, 8, -126);   /* bfloat16 */
    default: return x;
    }
}

static inline void mode_factor(const turb_tables *T, int m, int c, int j, int k,
                               double *cr, double *ci)
{
    const double yr = T->eyr[(size_t)m * T->ny + j], yi = T->eyi[(size_t)m * T->ny + j];
    const double zr = T->ezr[(size_t)m * T->nz + k], zi = T->ezi[(size_t)m * T->nz + k];
    const double tr = yr * zr - yi * zi;
    const double ti = yr * zi + yi * zr;
    const double qr = T->pr[(size_t)c * T->M + m], qi = T->pi[(size_t)c * T->M + m];
    *cr = tr * qr - ti * qi;
    *ci = tr * qi + ti * qr;
}

/* Whole grid of cycle c into out (nz*ny*nx*3 doubles). */
void turb_grid(const turb_tables *T, int32_t c, double *out)
{
    const int nx = T->nx, ny = T->ny, nz = T->nz, M = T->M;
#pragma omp parallel
    {
        double *ax = (double *)malloc(sizeof(double) * 3 * (size_t)nx);
        double *ay = ax + nx, *az = ay + nx;
#pragma omp for schedule(static)
        for (long row = 0; row < (long)ny * nz; ++row) {
            const int j = (int)(row % ny), k = (int)(row / ny);
            memset(ax, 0, sizeof(double) * 3 * (size_t)nx);
            for (int m = 0; m < M; ++m) {
                double cr, ci;
                mode_factor(T, m, c, j, k, &cr, &ci);
                const double a0 = T->amp[3 * m], a1 = T->amp[3 * m + 1], a2 = T->amp[3 * m + 2];
                const double *xr = T->exr + (size_t)m * nx, *xi = T->exi + (size_t)m * nx;
                for (int i = 0; i < nx; ++i) {
                    const double re = xr[i] * cr - xi[i] * ci;
                    ax[i] += a0 * re;
                    ay[i] += a1 * re;
                    az[i] += a2 * re;
                }
            }
            double *o = out + (size_t)row * nx * 3;
            for (int i = 0; i < nx; ++i) {
                o[3 * i] = ax[i];
                o[3 * i + 1] = ay[i];
                o[3 * i + 2] = az[i];
            }
        }
        free(ax);
    }
}

/* One grid point, same operations in the same order as turb_grid. */
void turb_point(const turb_tables *T, int32_t c, int32_t i, int32_t j, int32_t k, double out[3])
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int m = 0; m < T->M; ++m) {
        double cr, ci;
        mode_factor(T, m, c, j, k, &cr, &ci);
        const double re = T->exr[(size_t)m * T->nx + i] * cr - T->exi[(size_t)m * T->nx + i] * ci;
        s0 += T->amp[3 * m] * re;
        s1 += T->amp[3 * m + 1] * re;
        s2 += T->amp[3 * m + 2] * re;
    }
    out[0] = s0;
    out[1] = s1;
    out[2] = s2;
}

/* Fetch callback for consumers that read grid values one point at a time:
 * the point's value rounded to the table's storage precision, returned as the
 * exact FP64 value of the stored number. */
void turb_fetch(void *user, int32_t c, int32_t i, int32_t j, int32_t k, double out[3])
{
    const turb_tables *T = (const turb_tables *)user;
    turb_point(T, c, i, j, k, out);
    for (int d = 0; d < 3; ++d) out[d] = store_round(out[d], T->dtype);
}

/* Round an FP64 array in place to a storage precision (for checking the
 * generator's rounding against independent conversions). */
void turb_store_round(double *x, int64_t n, int32_t dtype)
{
    for (int64_t t = 0; t < n; ++t) x[t] = store_round(x[t], dtype);
}
