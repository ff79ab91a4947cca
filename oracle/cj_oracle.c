/*
 * Plain FP64 CPU reference ("oracle") for the Chebyshev-Jacobi method (CJM)
 * on the 2D finite-difference Poisson problem.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; it is used by the tests, by the smoke check and by the
 * benchmark's CPU-baseline leg.  It shares no code, header or table with the
 * GPU library.
 *
 * What it computes (Adsuara et al., "Speeding up a few orders of magnitude
 * the Jacobi method: high order Chebyshev-Jacobi over GPUs", §2.1):
 *
 *   - the discrete Laplacian, exactly as printed: the classical 5-point
 *     stencil (Table "tab:ste2", Cartesian), the 9-point first-family stencil
 *     with alpha = 2/3 (Eq. "9-points") and the 17-point second-family stencil
 *     with alpha = 2/3 (Eq. "17-points");
 *   - the system A u = f with A = -Delta_h, homogeneous Dirichlet data;
 *   - one weighted Jacobi sweep  u <- u + omega * D^{-1} (f - A u), where D is
 *     the (scalar) centre coefficient of A;
 *   - the residual f - A u and its squared 2-norm.
 *
 * The cycle loop, the weights and the stopping rule live in cjm.py; this file
 * only holds the O(N^2) loops so that the oracle finishes large samples in
 * seconds.  Floating point: IEEE double, round to nearest, no fast-math, no
 * contraction (built with -ffp-contract=off).
 *
 * Layout used by every routine here: a padded array of (nx+4) x (ny+4)
 * doubles, row-major with x fastest, holding grid nodes i = -1 .. nx+2 and
 * j = -1 .. ny+2.  Interior unknowns are 1 <= i <= nx, 1 <= j <= ny; the ring
 * i in {0, nx+1}, j in {0, ny+1} holds the Dirichlet value 0; the outer ring
 * i in {-1, nx+2}, j in {-1, ny+2} is read only by the 17-point stencil and
 * holds the odd reflection of the interior (u(-1,j) = -u(1,j),
 * u(nx+2,j) = -u(nx,j), likewise in y; corners take both flips).  The paper
 * does not say how the second ring is closed; odd reflection about the
 * Dirichlet node keeps every sine mode an exact eigenvector, which is what
 * makes the printed kappa_min closed form exact.
 */
#include <math.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(p, nx, i, j) \
    (p)[(size_t)((j) + 1) * (size_t)((nx) + 4) + (size_t)((i) + 1)]

struct tap { int di, dj; double c; };

/* 5-point: (1/h^2)[u(i-1,j) + u(i+1,j) + u(i,j-1) + u(i,j+1) - 4 u(i,j)]. */
static const struct tap TAPS5[] = {
    {-1, 0, 1.0}, {1, 0, 1.0}, {0, -1, 1.0}, {0, 1, 1.0}, {0, 0, -4.0}};

/* 9-point, alpha = 2/3: (1/(6h^2))[4 (W + E + S + N) + (SW + NE + NW + SE) - 20 C],
 * terms in the order the equation prints them. */
static const struct tap TAPS9[] = {
    {-1, 0, 4.0}, {1, 0, 4.0}, {0, -1, 4.0}, {0, 1, 4.0},
    {-1, -1, 1.0}, {1, 1, 1.0}, {-1, 1, 1.0}, {1, -1, 1.0},
    {0, 0, -20.0}};

/* 17-point, alpha = 2/3: (1/(72h^2))[ -4 u(i-2,j) + 64 u(i-1,j) + 64 u(i+1,j) - 4 u(i+2,j)
 *   - 4 u(i,j-2) + 64 u(i,j-1) + 64 u(i,j+1) - 4 u(i,j+2)
 *   - u(i-2,j-2) + 16 u(i-1,j-1) + 16 u(i+1,j+1) - u(i+2,j+2)
 *   - u(i-2,j+2) + 16 u(i-1,j+1) + 16 u(i+1,j-1) - u(i+2,j-2) - 300 u(i,j) ]. */
static const struct tap TAPS17[] = {
    {-2, 0, -4.0}, {-1, 0, 64.0}, {1, 0, 64.0}, {2, 0, -4.0},
    {0, -2, -4.0}, {0, -1, 64.0}, {0, 1, 64.0}, {0, 2, -4.0},
    {-2, -2, -1.0}, {-1, -1, 16.0}, {1, 1, 16.0}, {2, 2, -1.0},
    {-2, 2, -1.0}, {-1, 1, 16.0}, {1, -1, 16.0}, {2, -2, -1.0},
    {0, 0, -300.0}};

/* Returns the tap list and the prefactor denominator s (Laplacian = (1/(s h^2)) sum c u). */
static int taps_for(int stencil, const struct tap** t, double* s)
{
    switch (stencil) {
    case 5:  *t = TAPS5;  *s = 1.0;  return (int)(sizeof TAPS5 / sizeof TAPS5[0]);
    case 9:  *t = TAPS9;  *s = 6.0;  return (int)(sizeof TAPS9 / sizeof TAPS9[0]);
    case 17: *t = TAPS17; *s = 72.0; return (int)(sizeof TAPS17 / sizeof TAPS17[0]);
    default: return 0;
    }
}

/* Number of taps of a stencil (0 if unknown); lets the caller check the tables. */
int cjo_ntaps(int stencil)
{
    const struct tap* t; double s;
    return taps_for(stencil, &t, &s);
}

/* Copies tap k of a stencil out: (di, dj, c) and the prefactor denominator s. */
int cjo_tap(int stencil, int k, int* di, int* dj, double* c, double* s)
{
    const struct tap* t; int n = taps_for(stencil, &t, s);
    if (k < 0 || k >= n) return -1;
    *di = t[k].di; *dj = t[k].dj; *c = t[k].c;
    return 0;
}

/* Sets the Dirichlet ring to zero and the outer ring to the odd reflection of
 * the interior (see the layout note above).  Must be called after every change
 * of the interior and before the next stencil evaluation. */
void cjo_fill_ring(int nx, int ny, double* u)
{
    for (int j = 0; j <= ny + 1; ++j) { AT(u, nx, 0, j) = 0.0; AT(u, nx, nx + 1, j) = 0.0; }
    for (int i = 0; i <= nx + 1; ++i) { AT(u, nx, i, 0) = 0.0; AT(u, nx, i, ny + 1) = 0.0; }
    for (int j = 0; j <= ny + 1; ++j) {
        AT(u, nx, -1, j) = -AT(u, nx, 1, j);
        AT(u, nx, nx + 2, j) = -AT(u, nx, nx, j);
    }
    for (int i = -1; i <= nx + 2; ++i) {
        AT(u, nx, i, -1) = -AT(u, nx, i, 1);
        AT(u, nx, i, ny + 2) = -AT(u, nx, i, ny);
    }
}

/* Discrete Laplacian Delta_h u at interior node (i, j). */
static double laplacian(const struct tap* t, int nt, double s, double h,
                        int nx, const double* u, int i, int j)
{
    double acc = 0.0;
    for (int k = 0; k < nt; ++k) acc += t[k].c * AT(u, nx, i + t[k].di, j + t[k].dj);
    return acc / (s * h * h);
}

/* out = A u = -Delta_h u on the interior; out is unpadded nx*ny, x fastest. */
int cjo_apply(int nx, int ny, int stencil, double h, const double* u, double* out)
{
    const struct tap* t; double s; int nt = taps_for(stencil, &t, &s);
    if (nt == 0) return -1;
#pragma omp parallel for schedule(static)
    for (int j = 1; j <= ny; ++j)
        for (int i = 1; i <= nx; ++i)
            out[(size_t)(j - 1) * nx + (i - 1)] = -laplacian(t, nt, s, h, nx, u, i, j);
    return 0;
}

/* One weighted Jacobi sweep on the interior nodes of the region
 * [i0, i1] x [j0, j1] (inclusive, clipped to the interior):
 *     uout(i,j) = uin(i,j) + omega * r(i,j) / D,   r = f - A uin,
 * with D = -c_centre / (s h^2) the diagonal of A.  f is unpadded nx*ny.
 * Nodes outside the region are not written. */
int cjo_sweep(int nx, int ny, int stencil, double h, const double* f,
              const double* uin, double* uout, double omega,
              int i0, int i1, int j0, int j1)
{
    const struct tap* t; double s; int nt = taps_for(stencil, &t, &s);
    if (nt == 0) return -1;
    double centre = 0.0;
    for (int k = 0; k < nt; ++k) if (t[k].di == 0 && t[k].dj == 0) centre = t[k].c;
    const double D = -centre / (s * h * h);
    if (i0 < 1) i0 = 1;
    if (j0 < 1) j0 = 1;
    if (i1 > nx) i1 = nx;
    if (j1 > ny) j1 = ny;
#pragma omp parallel for schedule(static)
    for (int j = j0; j <= j1; ++j)
        for (int i = i0; i <= i1; ++i) {
            const double r = f[(size_t)(j - 1) * nx + (i - 1)]
                           + laplacian(t, nt, s, h, nx, uin, i, j);
            AT(uout, nx, i, j) = AT(uin, nx, i, j) + omega * r / D;
        }
    return 0;
}

/* Sum over the interior of (f - A u)^2, accumulated serially in row-major
 * order (j outer, i inner) so that the result does not depend on threading. */
double cjo_residual_sumsq(int nx, int ny, int stencil, double h,
                          const double* f, const double* u)
{
    const struct tap* t; double s; int nt = taps_for(stencil, &t, &s);
    if (nt == 0) return NAN;
    double acc = 0.0;
    for (int j = 1; j <= ny; ++j)
        for (int i = 1; i <= nx; ++i) {
            const double r = f[(size_t)(j - 1) * nx + (i - 1)]
                           + laplacian(t, nt, s, h, nx, u, i, j);
            acc += r * r;
        }
    return acc;
}

/* cjo_residual_sumsq of the unevaluated sum hi + lo (a double-double
 * iterate, both padded), in x87 extended precision (long double, 64-bit
 * significand) throughout: the pair sum, the taps in the printed order, the
 * division by s h^2, and the serial sum of squares. */
double cjo_residual_sumsq_ext(int nx, int ny, int stencil, double h,
                              const double* f, const double* hi, const double* lo)
{
    const struct tap* t; double s; int nt = taps_for(stencil, &t, &s);
    if (nt == 0) return NAN;
    const long double den = (long double)s * (long double)h * (long double)h;
    long double acc = 0.0L;
    for (int j = 1; j <= ny; ++j)
        for (int i = 1; i <= nx; ++i) {
            long double lap = 0.0L;
            for (int k = 0; k < nt; ++k) {
                const long double v = (long double)AT(hi, nx, i + t[k].di, j + t[k].dj)
                                    + (long double)AT(lo, nx, i + t[k].di, j + t[k].dj);
                lap += (long double)t[k].c * v;
            }
            const long double r = (long double)f[(size_t)(j - 1) * nx + (i - 1)] + lap / den;
            acc += r * r;
        }
    return (double)acc;
}

/* Sum of squares of n doubles, accumulated serially in storage order. */
double cjo_sumsq(size_t n, const double* x)
{
    double acc = 0.0;
    for (size_t k = 0; k < n; ++k) acc += x[k] * x[k];
    return acc;
}

/* Number of OpenMP threads the sweeps run on (1 when built without OpenMP). */
int cjo_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
