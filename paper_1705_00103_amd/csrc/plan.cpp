// Host planner of libcj.so: spectral bounds, cycle length and the ordered
// Chebyshev weights of the Chebyshev-Jacobi method (§2.1 of the paper).
#include <cmath>
#include <string>
#include <vector>

#include "cj_internal.h"

namespace cj {
namespace {

constexpr double kPi = 3.14159265358979323846;

double sq_sin(double a) {
    const double s = std::sin(a);
    return s * s;
}

// Smallest eigenvalue of D^{-1} A: the paper's closed forms (§2.1) evaluated
// with N = n + 1 intervals per axis.  The 5-point form is the stencil symbol
// at the (1, 1) sine mode.
double kappa_min(int stencil, int nx, int ny) {
    const double Nx = nx + 1.0, Ny = ny + 1.0;
    const double hx = kPi / (2.0 * Nx), hy = kPi / (2.0 * Ny);   // pi / 2N
    const double fx = kPi / Nx, fy = kPi / Ny;                   // pi / N
    switch (stencil) {
    case 5:
        return sq_sin(hx) + sq_sin(hy);
    case 9:
        return 0.8 * (sq_sin(hx) + sq_sin(hy)) + 0.2 * (sq_sin(hx + hy) + sq_sin(hx - hy));
    case 17: {
        const double ring1 = sq_sin(hx) + sq_sin(hy);
        const double ring2 = sq_sin(fx) + sq_sin(fy);
        const double diag1 = sq_sin(hx + hy) + sq_sin(hx - hy);
        const double diag2 = sq_sin(fx + fy) + sq_sin(fx - fy);
        return (64.0 * ring1 - 4.0 * ring2 + 16.0 * diag1 - diag2) / 75.0;
    }
    default:
        return NAN;
    }
}

// Supremum of the symbol of D^{-1} A (reached at the (pi, pi) mode).
double kappa_max(int stencil) {
    switch (stencil) {
    case 5: return 2.0;
    case 9: return 8.0 / 5.0;
    case 17: return 128.0 / 75.0;
    default: return NAN;
    }
}

// ln cosh(x), x >= 0, without overflow.
double log_cosh(double x) { return x + std::log1p(std::exp(-2.0 * x)) - std::log(2.0); }

// Cycles of length M that the per-cycle bound 1 / cosh(M beta) needs to reach tol.
long long cycles_for(long long M, double beta, double tol) {
    if (tol >= 1.0) return 1;
    const double c = std::ceil(std::log(1.0 / tol) / log_cosh((double)M * beta));
    return c < 1.0 ? 1 : (long long)c;
}

// theta values of the recursive symmetric-pair order for M = 2^p: each
// doubling step m -> 2m replaces every entry s by the pair (s, 4m - s).
std::vector<int> pair_order(int M) {
    std::vector<int> th(1, 1);
    for (int m = 1; m < M; m *= 2) {
        std::vector<int> next(2 * (size_t)m);
        for (int k = 0; k < m; ++k) {
            next[2 * (size_t)k] = th[k];
            next[2 * (size_t)k + 1] = 4 * m - th[k];
        }
        th.swap(next);
    }
    return th;
}

// Argument checks and the fields every schedule shares.
bool common_fields(int stencil, int nx, int ny, double tol, double h, int M_request, Schedule* s,
                   std::string* err) {
    if (stencil != 5 && stencil != 9 && stencil != 17) {
        *err = "stencil must be 5, 9 or 17";
        return false;
    }
    if (nx < 1 || ny < 1 || nx > (1 << 20) || ny > (1 << 20)) {
        *err = "nx and ny must lie in [1, 2^20]";
        return false;
    }
    if (!(tol > 0.0) || !std::isfinite(tol)) {
        *err = "tol must be a finite positive number";
        return false;
    }
    if (!(h >= 0.0) || !std::isfinite(h)) {
        *err = "h must be >= 0 (0 selects the default)";
        return false;
    }
    if (M_request < 0 || M_request > (1 << 24) || (M_request & (M_request - 1)) != 0) {
        *err = "M must be 0 (automatic) or a power of two <= 2^24";
        return false;
    }
    s->stencil = stencil;
    s->nx = nx;
    s->ny = ny;
    s->tol = tol;
    s->h = h > 0.0 ? h : 1.0 / (double)(nx > ny ? nx + 1 : ny + 1);
    s->kmin = kappa_min(stencil, nx, ny);
    s->kmax = kappa_max(stencil);
    s->beta = std::acosh((s->kmax + s->kmin) / (s->kmax - s->kmin));
    return true;
}

}  // namespace

bool make_schedule(int stencil, int nx, int ny, double tol, double h, int M_request,
                   Schedule* s, std::string* err) {
    if (!common_fields(stencil, nx, ny, tol, h, M_request, s, err)) return false;
    if (M_request > 0) {
        s->M = M_request;
        s->cycles_pred = (int)cycles_for(M_request, s->beta, tol);
    } else {
        long long bestM = 1, bestC = cycles_for(1, s->beta, tol);
        for (int p = 1; p <= 24 && bestC > 1; ++p) {
            const long long M = 1LL << p;
            const long long c = cycles_for(M, s->beta, tol);
            if (c * M < bestC * bestM) {
                bestM = M;
                bestC = c;
            }
            if (c == 1) break;
        }
        s->M = (int)bestM;
        s->cycles_pred = (int)bestC;
    }
    s->rho = std::exp(-log_cosh((double)s->M * s->beta));
    const std::vector<int> th = pair_order(s->M);
    const double sum = s->kmax + s->kmin, dif = s->kmax - s->kmin;
    s->w.resize(s->M);
    for (int k = 0; k < s->M; ++k)
        s->w[k] = 2.0 / (sum - dif * std::cos((double)th[k] * kPi / (2.0 * s->M)));
    return true;
}

// Plain Jacobi (omega = 1, the paper's reference method): the weights are all
// one and M is only the interval between residual checks.  n_J sweeps meet tol
// under the bound (1 - kappa_min)^n; by default M is the largest power of two
// not above n_J / 32, so that the last check overshoots by at most ~3%.
bool make_jacobi_schedule(int stencil, int nx, int ny, double tol, double h, int M_request, Schedule* s,
                          std::string* err) {
    if (!common_fields(stencil, nx, ny, tol, h, M_request, s, err)) return false;
    const double per_sweep = -std::log1p(-s->kmin);
    long long nj = 1;
    if (tol < 1.0) {
        const double c = std::ceil(std::log(1.0 / tol) / per_sweep);
        nj = c < 1.0 ? 1 : (c > 4e18 ? (long long)4e18 : (long long)c);
    }
    long long M = M_request;
    if (M == 0) {
        M = 1;
        const long long target = nj / 32 > 1 ? nj / 32 : 1;
        while (2 * M <= target && M < (1LL << 24)) M *= 2;
    }
    const long long checks = (nj + M - 1) / M;
    if (checks > (1LL << 30)) {
        *err = "Jacobi would need more than 2^30 residual checks at this M and tol";
        return false;
    }
    s->M = (int)M;
    s->cycles_pred = (int)checks;
    s->rho = std::exp(-(double)M * per_sweep);
    s->w.assign((size_t)M, 1.0);
    return true;
}

}  // namespace cj
