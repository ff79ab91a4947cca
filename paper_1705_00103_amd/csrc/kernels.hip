// HIP kernels of libcj.so for gfx950 (MI355X): stage-in/out, the weighted
// Chebyshev-Jacobi sweep (one sweep per launch, or K sweeps per launch with
// temporal blocking), the residual norm, the stencil apply, and the FP32 /
// FP64 pieces of iterative refinement.
//
// All kernels work on the padded, pitched layout described in cj_internal.h.
// A single sweep is HBM-bound (24 bytes in FP64, 12 in FP32, and 8-16 flops
// per grid-point update), so the kernels are organised around memory
// traffic: one wave64 lane per grid column, marching up the rows of its tile
// and keeping the (2R+1) rows of the stencil window in registers, so that
// every value of u is fetched from HBM once per sweep and the row re-reads of
// the window hit registers.  Row loads of a wave are 64 consecutive elements,
// aligned on the interior.  The temporally blocked kernel performs K updates
// per HBM pass; it is bound by FP64 latency, instruction issue and its LDS
// exchange instead.
//
// Arithmetic is written with explicit fma and compiled with
// -ffp-contract=off, so that every kernel that evaluates the update in a
// given precision performs exactly the same operations in the same order and
// produces the same bits.
#include <hip/hip_runtime.h>

#include <mutex>

#include "cj_internal.h"

namespace cj {
namespace {

// ------------------------------------------------------------ element types

template <typename T> __device__ __forceinline__ T fmat(T a, T b, T c);
template <> __device__ __forceinline__ double fmat<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <> __device__ __forceinline__ float fmat<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// c ? a : b as a per-lane select.  The empty asm makes b a value every lane
// has computed, so the compiler cannot move b's computation into a branch
// taken only by the lanes that need it (which would split the blocked
// kernel's row step into one exec-masked region per level).
template <typename T>
__device__ __forceinline__ T select_lane(bool c, T a, T b) {
    asm volatile("" : "+v"(b));
    return c ? a : b;
}

template <typename T>
__device__ __forceinline__ size_t at(int pitch, int x, int y) {
    return (size_t)(y + 1) * (size_t)pitch + (size_t)(x + xoff_of(sizeof(T)));
}

// ------------------------------------------------------------ stencils
// The update in normalised form.  With c_hat = c / |c_centre| and
// g = D^{-1} f (D = |c_centre| / (s h^2)):
//     t = sum over neighbours of c_hat * u_nbr
//     r = (g + t) - u            (= D^{-1} (f - A u))
//     u' = u + omega * r
// c_hat (from the stencil equations of §2.1 and Table tab:ste2):
//     5-point : 1/4 on the four axis neighbours
//     9-point : 4/20 axis, 1/20 diagonal
//     17-point: 64/300 axis ring 1, -4/300 axis ring 2,
//               16/300 diagonal ring 1, -1/300 diagonal ring 2.
// Every coefficient multiplies a centre value or a symmetric pair of one
// window row, so a row y + dy enters as its summary
//     C = u(x, y + dy),  P_k = u(x - k, y + dy) + u(x + k, y + dy),  k = 1..R,
// and t = scale * S, S an integer-weighted sum of the summaries
// s[dy + R] = {C, P_1, .., P_R} (the weights differ from c_hat / scale by
// powers of two, so scale * weight is exactly the rounded c_hat):
//     5-point : scale 1/4,   S = P_1[0] + (C[-1] + C[+1])
//     9-point : scale 1/20,  S = fma(4, P_1[0] + (C[-1] + C[+1]), P_1[-1] + P_1[+1])
//     17-point: scale 1/300, S = fma(16, P_1[-1] + P_1[+1], fma(-4, P_2[0] + (C[-2] + C[+2]),
//                                fma(64, P_1[0] + (C[-1] + C[+1]), -(P_2[-2] + P_2[+2]))))
// and r = fma(scale, S, g) - u: the scale rides on the fma that adds g
// (9-point: 8 FP64 operations per update with the pair sums and the update,
// 17-point 14).  The temporally blocked kernel keeps only the summaries of its
// window rows (R + 1 values instead of 2R + 1) and forms each pair sum once
// per row; every kernel evaluates r through these functions, so all produce
// the same bits.

template <int ST> struct Stencil;

template <> struct Stencil<5> {
    static constexpr int R = 1;
    static constexpr double scale = 0.25;
    template <typename T> __device__ static __forceinline__ T combine(const T (&s)[3][2]) {
        return s[1][1] + (s[0][0] + s[2][0]);
    }
};

template <> struct Stencil<9> {
    static constexpr int R = 1;
    static constexpr double scale = 1.0 / 20.0;
    template <typename T> __device__ static __forceinline__ T combine(const T (&s)[3][2]) {
        const T axis = s[1][1] + (s[0][0] + s[2][0]);
        const T diag = s[0][1] + s[2][1];
        return fmat<T>(T(4), axis, diag);
    }
};

template <> struct Stencil<17> {
    static constexpr int R = 2;
    static constexpr double scale = 1.0 / 300.0;
    template <typename T> __device__ static __forceinline__ T combine(const T (&s)[5][3]) {
        const T axis1 = s[2][1] + (s[1][0] + s[3][0]);
        const T axis2 = s[2][2] + (s[0][0] + s[4][0]);
        const T diag1 = s[1][1] + s[3][1];
        const T diag2 = s[0][2] + s[4][2];
        return fmat<T>(T(16), diag1, fmat<T>(T(-4), axis2, fmat<T>(T(64), axis1, -diag2)));
    }
};

// r = fma(scale, S, g) - u from the window summaries, with u the centre value.
template <typename T, int ST>
__device__ __forceinline__ T summary_residual(const T (&s)[2 * Stencil<ST>::R + 1][Stencil<ST>::R + 1], T g, T u) {
    return fmat<T>(T(Stencil<ST>::scale), Stencil<ST>::template combine<T>(s), g) - u;
}

// Summary {C, P_1, .., P_R} of one window row (its 2R + 1 values around x).
template <typename T, int R>
__device__ __forceinline__ void row_summary(const T (&row)[2 * R + 1], T (&sm)[R + 1]) {
    sm[0] = row[R];
#pragma unroll
    for (int k = 1; k <= R; ++k) sm[k] = row[R - k] + row[R + k];
}

// r and t of a full window, v[dy + R][dx + R] = u(x + dx, y + dy).
template <typename T, int ST>
__device__ __forceinline__ T window_residual(const T (&v)[2 * Stencil<ST>::R + 1][2 * Stencil<ST>::R + 1], T g) {
    constexpr int R = Stencil<ST>::R;
    T sm[2 * R + 1][R + 1];
#pragma unroll
    for (int r = 0; r < 2 * R + 1; ++r) row_summary<T, R>(v[r], sm[r]);
    return summary_residual<T, ST>(sm, g, v[R][R]);
}

template <typename T, int ST>
__device__ __forceinline__ T neighbour_sum(const T (&v)[2 * Stencil<ST>::R + 1][2 * Stencil<ST>::R + 1]) {
    constexpr int R = Stencil<ST>::R;
    T sm[2 * R + 1][R + 1];
#pragma unroll
    for (int r = 0; r < 2 * R + 1; ++r) row_summary<T, R>(v[r], sm[r]);
    return T(Stencil<ST>::scale) * Stencil<ST>::template combine<T>(sm);
}

// ------------------------------------------------------------ accurate residual
// The refinement's outer residual r = g - D^{-1}A u decides how far the FP64
// iterate can be corrected, so it is evaluated with error-free transformations.
// D^{-1}A u = (W u - sum_k w_k u_k) / W with the integer weights of the stencil
// (W = 4, 20, 300; w_k = 1; 4 and 1; 64, -4, 16 and -1).  Each w_k u_k is exact
// (w_k is a power of two), W u is split exactly by an fma, and the terms are
// summed with TwoSum (Knuth) carrying the compensation, so the difference of
// magnitude ~ |g| W is formed to about a unit in its own last place instead of
// in the last place of W |u|.  Then r = fma(-1/W, D, g).  The order of the
// terms is fixed, so the result is deterministic.

__device__ __forceinline__ void acc_two_sum(double& s, double& c, double x) {
    const double t = s + x;
    const double z = t - s;
    c += (s - (t - z)) + (x - z);
    s = t;
}

// Integer weight w_k of the neighbour (dx, dy) in D^{-1}A u = (W u - sum_k w_k u_k) / W.
template <int ST>
__device__ __forceinline__ constexpr double stencil_weight(int dx, int dy) {
    const int ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy;
    if (ST == 5) return (ax + ay == 1) ? 1.0 : 0.0;
    if (ST == 9) return (ax + ay == 1) ? 4.0 : (ax == 1 && ay == 1) ? 1.0 : 0.0;
    if (ax + ay == 1) return 64.0;
    if ((ax == 2 && ay == 0) || (ax == 0 && ay == 2)) return -4.0;
    if (ax == 1 && ay == 1) return 16.0;
    if (ax == 2 && ay == 2) return -1.0;
    return 0.0;
}

template <int ST> constexpr double stencil_centre = ST == 5 ? 4.0 : ST == 9 ? 20.0 : 300.0;

// W u - sum_k w_k u_k of a window in plain FP64, fixed order: the low part
// of a double-double iterate, whose rounding errors are far below those of
// the high part's exact evaluation.
template <int ST>
__device__ __forceinline__ double plain_scaled_operator(
    const double (&v)[2 * Stencil<ST>::R + 1][2 * Stencil<ST>::R + 1]) {
    constexpr int R = Stencil<ST>::R;
    double t = 0.0;
#pragma unroll
    for (int dy = -R; dy <= R; ++dy)
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) {
            const double w = stencil_weight<ST>(dx, dy);
            if (w != 0.0) t = __builtin_fma(w, v[dy + R][dx + R], t);
        }
    return __builtin_fma(stencil_centre<ST>, v[R][R], -t);
}

// With DD the iterate is hi + lo (v holds hi); dlo = plain_scaled_operator
// of lo joins the compensation term before the final rounding.
template <int ST, bool DD = false>
__device__ __forceinline__ double accurate_residual(const double (&v)[2 * Stencil<ST>::R + 1][2 * Stencil<ST>::R + 1],
                                                    double g, double dlo = 0.0) {
    constexpr int R = Stencil<ST>::R;
    constexpr double W = stencil_centre<ST>;
    const double u = v[R][R];
    double s = W * u;
    double c = __builtin_fma(W, u, -s);      // W u = s + c exactly
#pragma unroll
    for (int dy = -R; dy <= R; ++dy) {
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) {
            const double w = stencil_weight<ST>(dx, dy);
            if (w != 0.0) acc_two_sum(s, c, -w * v[dy + R][dx + R]);
        }
    }
    if (DD) c += dlo;
    return __builtin_fma(-1.0 / W, s + c, g);
}

// Hardware dispatches workgroup b to XCD b % 8.  Give every XCD a contiguous
// range of tiles (row-major over the grid), so that vertically adjacent tiles,
// which share halo rows, usually run on the same XCD and share its L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int xcd = b & 7, slot = b >> 3;
    return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// Sum over the workgroup (blockDim.x = 64 * waves, waves <= 8), fixed order.
// The result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double ws[8];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) ws[wave] = v;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        tot = ws[0];
        for (int k = 1; k < nw; ++k) tot += ws[k];
    }
    return tot;
}

// Stores u'(x, y) with a streaming (non-temporal) store: the new iterate is not
// read again before it has left the caches.  REFL (17-point stencil with
// homogeneous data): the odd reflections on the outer ring are kept up to date
// as well.  Without it every node outside the interior holds data that the
// sweeps never change.
template <typename T, int ST, bool REFL>
__device__ __forceinline__ void store_update(T* __restrict__ uout, int pitch, int nx, int ny, int x, int y, T un) {
    __builtin_nontemporal_store(un, uout + at<T>(pitch, x, y));
    if (ST == 17 && REFL) {
        if (x == 1) uout[at<T>(pitch, -1, y)] = -un;
        if (x == nx) uout[at<T>(pitch, nx + 2, y)] = -un;
        if (y == 1) {
            uout[at<T>(pitch, x, -1)] = -un;
            if (x == 1) uout[at<T>(pitch, -1, -1)] = un;
            if (x == nx) uout[at<T>(pitch, nx + 2, -1)] = un;
        }
        if (y == ny) {
            uout[at<T>(pitch, x, ny + 2)] = -un;
            if (x == 1) uout[at<T>(pitch, -1, ny + 2)] = un;
            if (x == nx) uout[at<T>(pitch, nx + 2, ny + 2)] = un;
        }
    }
}

// ------------------------------------------------------------ sweep / residual
// One lane per column x of a tile of width blockDim.x and `rows` rows.  The
// lane keeps the window rows y-R .. y+R in registers and loads one new row
// (2R+1 columns) per output row.  WRITE: store the update; NORM: accumulate
// r^2 of the input iterate (FP64 only).

template <typename T, int ST, bool WRITE, bool NORM, bool REFL>
__global__ __launch_bounds__(256) void sweep_kernel(const T* __restrict__ uin, T* __restrict__ uout,
                                                    const T* __restrict__ g, const T* __restrict__ w, int widx,
                                                    int nx, int ny, int pitch, int tiles_x, int rows,
                                                    double* __restrict__ part) {
    constexpr int R = Stencil<ST>::R;
    constexpr int W = 2 * R + 1;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int x = tx * (int)blockDim.x + (int)threadIdx.x + 1;
    const bool active = x <= nx;
    const int xl = active ? x : nx;   // idle lanes load a valid column and store nothing
    const int y0 = ty * rows + 1;
    const int y1 = min(y0 + rows, ny + 1);
    const T omega = WRITE ? w[widx] : T(0);

    T v[W][W];
#pragma unroll
    for (int r = 1; r < W; ++r) {
        const T* p = uin + at<T>(pitch, xl - R, y0 - R + r - 1);
#pragma unroll
        for (int c = 0; c < W; ++c) v[r][c] = p[c];
    }
    double acc = 0.0;
#pragma unroll 4
    for (int y = y0; y < y1; ++y) {
#pragma unroll
        for (int r = 0; r < W - 1; ++r)
#pragma unroll
            for (int c = 0; c < W; ++c) v[r][c] = v[r + 1][c];
        const T* p = uin + at<T>(pitch, xl - R, y + R);
#pragma unroll
        for (int c = 0; c < W; ++c) v[W - 1][c] = p[c];
        const T gv = __builtin_nontemporal_load(g + at<T>(pitch, xl, y));
        const T uc = v[R][R];
        const T res = window_residual<T, ST>(v, gv);
        if (NORM) acc = fmat<double>((double)res, (double)res, acc);
        if (WRITE && active) store_update<T, ST, REFL>(uout, pitch, nx, ny, x, y, fmat<T>(omega, res, uc));
    }
    if (NORM) {
        if (!active) acc = 0.0;
        const double tot = block_sum(acc);
        if (threadIdx.x == 0) part[tile] = tot;
    }
}

// ------------------------------------------------------------ temporal blocking
// K consecutive weighted sweeps in one launch.  A workgroup of 256 lanes owns a
// strip of 256 columns and marches up the rows of its tile; level s (the
// iterate after s sweeps) trails level s-1 by R+1 rows, so that each level
// only needs rows of the level below that were finished in an earlier step:
// one barrier per row step suffices.  Level 0 comes from HBM (the row and its
// x +- R neighbours), levels 1..K-1 are exchanged between lanes through LDS,
// and every lane keeps a register window of 2R+1 row summaries per level
// (see Stencil), each row tagged with the lane's value of g on that row (the
// g a level used for a row is the g the next level needs on it).  Only level
// K is written back, so one launch moves one read of u and g and one write of
// u per grid point and performs K updates per point.
// Outputs shrink by R columns per level on each side of the strip
// (256 - 2KR output columns) and the tiles overlap in y by KR rows.
// The row loop is unrolled by a multiple of the window height W = 2R+1 (and
// of the prefetch depth) so that the window rotation is a compile-time
// renaming of registers.  Where the halo reaches the domain boundary a
// variant closes the levels >= 1: with REFL (17-point, homogeneous data) by
// the Dirichlet zeros and the odd reflections of the level below, in every
// wave of the workgroup (a halo that crosses only an x-boundary skips the
// closure of rows); otherwise the outside nodes that interior nodes read keep,
// at every level, the value level 0 loaded for them (the boundary data), and
// only the wave holding such a column and the row blocks reaching such a row
// run that variant (see sweepk_tile).  Interior workgroups skip both.  The closures are per-lane selects
// (select_lane), not branches: a branch would cut the row step into one
// region per level and serialise the levels (edge workgroups took 1.4x as
// long as interior ones at 8192^2, 9-point K = 10).
// Every update evaluates exactly the expression of sweep_kernel on exactly the
// same values, so K sweeps here give the same bits as K launches of it.

template <typename T, int ST, int K>
struct March {
    static constexpr int R = Stencil<ST>::R;
    static constexpr int W = 2 * R + 1;
    static constexpr int SW = strip_lanes(R, K, sizeof(T));   // lanes = strip columns
    static constexpr int WOUT = SW - 2 * K * R;
    // level-0 rows are fetched PD row steps ahead (a row step is shorter than
    // the HBM latency under load).  Measured at 8192^2: 3-row windows gain
    // from 3 steps in FP32 and 2 in FP64 (9-point K = 8: 75.3 -> 70.1 us per
    // sweep; 3 steps in FP64 lose: K = 10 57.0 -> 61.5); 5-row windows take
    // two (17-point K = 4: 137.1 -> 132.3 us against one step).
    static constexpr int PD = (R == 2) ? 2 : sizeof(T) == 4 ? 3 : 2;
    // the row loop is unrolled by U steps, a multiple of both W (window slot
    // J % W) and PD (prefetch slot J % PD), so that both rotations are static
    static constexpr int U = (W % PD == 0) ? W : W * PD;
    static_assert(PD >= 1 && PD <= 3, "prefetch depth");
    // Window rows are kept as their summaries {C, P_1 .. P_R}: fewer
    // registers than the 2R + 1 values, and each pair sum is formed once.
    // Measured at 8192^2, FP64: this lets 9-point K = 10 and 17-point K = 4 run
    // at two waves per SIMD (9-point 73.4 -> 68.6 us per sweep, 17-point
    // 182.6 -> 152.5 us).
    static constexpr int NV = R + 1;
    T win[K][W][NV];      // [level][physical row slot][row summary]
    T gw[K][W];       // g of the lane's column on each window row
    T own[K];         // the lane's value on the row a level produced in this step
    T gused[K];       // the g it used
    T pre[PD][W];     // prefetched level-0 rows
    T pg[PD];         // and their g
    int lcol[W];      // level-0 load columns (clamped), with the layout offset
    int xsrc[W];      // exchange source lanes for the x +- R neighbours
    int xsgn[W];      // 1, 0 (Dirichlet column) or -1 (reflection), REFL edge workgroups only
};

// One row step with compile-time phase J = t mod U.  Level 0 enters window
// slot J % W at the start of the step; level s >= 1 enters that slot at its
// end.  The level-0 row of this step was prefetched PD steps earlier into
// prefetch slot J % PD, which this step refills with the row PD steps ahead.
template <typename T, int ST, int K, bool NORM, bool REFL, bool EDGE, bool EY, int J>
__device__ __forceinline__ void march_step(March<T, ST, K>& S, T (*xch)[March<T, ST, K>::W][March<T, ST, K>::SW],
                                           const T* __restrict__ uin, T* __restrict__ uout, const T* __restrict__ g,
                                           const T (&om)[K], int t, int ybase, int x, int xg, bool out_col, int Y0,
                                           int Y1, int nx, int ny, int pitch, double& acc) {
    constexpr int R = Stencil<ST>::R;
    constexpr int W = 2 * R + 1;
    constexpr int PD = March<T, ST, K>::PD;
    constexpr int P = J % PD;     // prefetch slot of this phase
    constexpr int JW = J % W;     // window slot of this phase
    const int tid = threadIdx.x;
    const int yl = ybase + t;
    row_summary<T, R>(S.pre[P], S.win[0][JW]);
    S.gw[0][JW] = S.pg[P];
    {   // prefetch the level-0 row PD steps ahead, and its g
        const int yr = min(max(yl + PD, -1), ny + 2);
        const T* rowp = uin + (size_t)(yr + 1) * (size_t)pitch;
#pragma unroll
        for (int c = 0; c < W; ++c) S.pre[P][c] = rowp[S.lcol[c]];
        S.pg[P] = __builtin_nontemporal_load(g + at<T>(pitch, xg, yr));
    }
#pragma unroll
    for (int s = 1; s <= K; ++s) {
        const int Y = yl - (s - 1) - s * R;   // row produced by level s in this step
        // logical window row r (0 = oldest) of level s-1 sits in physical slot
        // (JW + 1 + r) % W for level 0 (filled this step) and (JW + r) % W above
        T sm[W][R + 1];
        T gv;
#pragma unroll
        for (int r = 0; r < W; ++r) {
            const int ph = (s == 1) ? (JW + 1 + r) % W : (JW + r) % W;
#pragma unroll
            for (int k = 0; k <= R; ++k) sm[r][k] = S.win[s - 1][ph][k];
            if (r == R) gv = S.gw[s - 1][ph];
        }
        if (REFL && EDGE && EY && s > 1 && (Y - R < 1 || Y + R > ny)) {
            // rows beyond the interior: Dirichlet zeros, second ring by odd reflection
#pragma unroll
            for (int r = 0; r < W; ++r) {
                const int q = Y - R + r;
                if (q == 0 || q == ny + 1) {
#pragma unroll
                    for (int k = 0; k <= R; ++k) sm[r][k] = T(0);
                } else if (R == 2 && q == -1 && r + 2 < W) {
#pragma unroll
                    for (int k = 0; k <= R; ++k) sm[r][k] = -sm[r + 2][k];
                } else if (R == 2 && q == ny + 2 && r >= 2) {
#pragma unroll
                    for (int k = 0; k <= R; ++k) sm[r][k] = -sm[r - 2][k];
                }
            }
        }
        const T uc = sm[R][0];
        const T res = summary_residual<T, ST>(sm, gv, uc);
        T un = fmat<T>(om[s - 1], res, uc);
        // boundary data: a node outside the interior keeps its value
        if (!REFL && EDGE) un = select_lane<T>(x < 1 || x > nx || Y < 1 || Y > ny, uc, un);
        if (NORM && s == 1 && out_col && Y >= Y0 && Y < Y1) acc = fmat<double>((double)res, (double)res, acc);
        if (s < K) {
            xch[s - 1][JW][tid] = un;
            S.own[s] = un;
            S.gused[s] = gv;
        } else if (out_col && Y >= Y0 && Y < Y1) {
            store_update<T, ST, REFL>(uout, pitch, nx, ny, x, Y, un);
        }
    }
    if (K > 1) {
        __syncthreads();
#pragma unroll
        for (int s = 1; s < K; ++s) {
            T row[W];
#pragma unroll
            for (int c = 0; c < W; ++c) {
                if (c == R) {
                    row[c] = S.own[s];
                } else {
                    const T e = xch[s - 1][JW][S.xsrc[c]];
                    if (REFL && EDGE)
                        row[c] = select_lane<T>(S.xsgn[c] == 0, T(0), S.xsgn[c] < 0 ? -e : e);
                    else
                        row[c] = e;
                }
            }
            row_summary<T, R>(row, S.win[s][JW]);
            S.gw[s][JW] = S.gused[s];
        }
    }
}

// Row steps t + J, t + J + 1, ..., t + UU - 1 (compile-time phases).
template <typename T, int ST, int K, bool NORM, bool REFL, bool EDGE, bool EY, int J, int UU>
__device__ __forceinline__ void march_steps(March<T, ST, K>& S, T (*xch)[March<T, ST, K>::W][March<T, ST, K>::SW],
                                            const T* __restrict__ uin, T* __restrict__ uout,
                                            const T* __restrict__ g, const T (&om)[K], int t, int ybase, int x,
                                            int xg, bool out_col, int Y0, int Y1, int nx, int ny, int pitch,
                                            double& acc) {
    march_step<T, ST, K, NORM, REFL, EDGE, EY, J>(S, xch, uin, uout, g, om, t + J, ybase, x, xg, out_col, Y0, Y1, nx, ny,
                                              pitch, acc);
    if constexpr (J + 1 < UU)
        march_steps<T, ST, K, NORM, REFL, EDGE, EY, J + 1, UU>(S, xch, uin, uout, g, om, t, ybase, x, xg, out_col, Y0, Y1,
                                                       nx, ny, pitch, acc);
}

// Row-step blocks b0 .. b1 - 1 (a block is U row steps), UF blocks per pass
// (b1 - b0 a multiple of UF).  At the end of a pass the registers the loop
// carries wait for the loads and the store still in flight, so a longer pass
// waits less often.
template <typename T, int ST, int K, bool NORM, bool REFL, bool EDGE, bool EY, int UF = 1>
__device__ __forceinline__ void march(March<T, ST, K>& S, T (*xch)[March<T, ST, K>::W][March<T, ST, K>::SW],
                                      const T* __restrict__ uin, T* __restrict__ uout, const T* __restrict__ g,
                                      const T (&om)[K], int ybase, int b0, int b1, int x, int xg, bool out_col, int Y0,
                                      int Y1, int nx, int ny, int pitch, double& acc) {
    constexpr int U = March<T, ST, K>::U;
    for (int t = b0 * U; t < b1 * U; t += U * UF)
        march_steps<T, ST, K, NORM, REFL, EDGE, EY, 0, U * UF>(S, xch, uin, uout, g, om, t, ybase, x, xg, out_col, Y0, Y1, nx,
                                                   ny, pitch, acc);
}

// The blocked sweeps of one tile (strip sx, row tile sy = tile / strips_x).
// UF: blocks of U row steps per pass of the loop without boundary selects.
template <typename T, int ST, int K, bool NORM, bool REFL, int UF>
__device__ __forceinline__ void sweepk_tile(const T* __restrict__ uin, T* __restrict__ uout, const T* __restrict__ g,
                                            const T* __restrict__ w, int widx, int nx, int ny, int pitch,
                                            int strips_x, int rows, int tile, double* __restrict__ part) {
    using MS = March<T, ST, K>;
    constexpr int R = MS::R;
    constexpr int W = MS::W;
    constexpr int WOUT = MS::WOUT;
    constexpr int SW = MS::SW;
    __shared__ T xch[K > 1 ? K - 1 : 1][W][SW];

    const int tid = threadIdx.x;
    const int sx = tile % strips_x, sy = tile / strips_x;
    const int X0 = sx * WOUT + 1;
    const int x = X0 - K * R + tid;
    const int Y0 = sy * rows + 1;
    const int Y1 = min(Y0 + rows, ny + 1);
    const bool out_col = tid >= K * R && tid < K * R + WOUT && x >= 1 && x <= nx;
    const int xg = min(max(x, 1), nx);     // column for g (only interior columns matter)
    // Does the halo of this workgroup reach beyond the interior?  (uniform)
    const bool edge_x = (X0 - K * R < 1) || (X0 - K * R + SW - 1 > nx);
    const bool edge_y = (Y0 - K * R < 1) || (Y1 - 1 + K * R > ny);

    MS S;
#pragma unroll
    for (int c = 0; c < W; ++c) {
        S.lcol[c] = min(max(x - R + c, -1), nx + 2) + xoff_of(sizeof(T));
        const int dx = c - R, col = x + dx;
        int idx = tid + dx, sg = 1;
        if (REFL) {
            if (col == 0 || col == nx + 1) sg = 0;
            else if (col == -1) { idx = tid + dx + 2; sg = -1; }
            else if (col == nx + 2) { idx = tid + dx - 2; sg = -1; }
        }
        S.xsrc[c] = min(max(idx, 0), SW - 1);
        S.xsgn[c] = sg;
    }
    T om[K];
#pragma unroll
    for (int s = 0; s < K; ++s) om[s] = w[widx + s];
#pragma unroll
    for (int s = 0; s < K; ++s) {
#pragma unroll
        for (int r = 0; r < W; ++r) {
            S.gw[s][r] = T(0);
#pragma unroll
            for (int k = 0; k < MS::NV; ++k) S.win[s][r][k] = T(0);
        }
    }
    const int ybase = Y0 - K * R;   // level-0 row entering at step 0
#pragma unroll
    for (int q = 0; q < MS::PD; ++q) {
        const int yr = min(max(ybase + q, -1), ny + 2);
        const T* rowp = uin + (size_t)(yr + 1) * (size_t)pitch;
#pragma unroll
        for (int c = 0; c < W; ++c) S.pre[q][c] = rowp[S.lcol[c]];
        S.pg[q] = __builtin_nontemporal_load(g + at<T>(pitch, xg, yr));
    }
    double acc = 0.0;
    const int steps = (Y1 - Y0) + 2 * K * R + K - 1;
    constexpr int U = MS::U;
    const int nb = (steps + U - 1) / U;   // blocks of U row steps (rows past the tile are not stored)
    if constexpr (REFL) {
        // The closure of rows runs only in the blocks where some level s >= 2
        // reads a window row outside 1 .. ny (rows Y - R .. Y + R around the
        // row Y that level s produces), the closure of columns in every wave of
        // a workgroup whose halo crosses an x-boundary, and neither elsewhere.
        // The loops run one after another over (possibly empty) ranges of
        // blocks, as below.
        int bh = 0, bt = nb;   // blocks [0, bh) and [bt, nb) close the rows
        if (edge_y) {
            const int lo = 1 + R - ybase + (K - 1) + K * R;  // first block whose lowest row is >= 1 + R
            bh = lo <= 0 ? 0 : min((lo + U - 1) / U, nb);
            const int hi = ny - R - ybase - U + 1 + R;       // blocks b <= hi / U keep their rows <= ny - R
            bt = hi < 0 ? 0 : min(hi / U + 1, nb);
            bt = max(bt, bh);
        }
        const int bm = edge_x ? bt : bh;   // columns closed in [bh, bm), nothing in [bm, bt)
        march<T, ST, K, NORM, REFL, true, true>(S, xch, uin, uout, g, om, ybase, 0, bh, x, xg, out_col, Y0, Y1, nx, ny,
                                                pitch, acc);
        march<T, ST, K, NORM, REFL, true, false>(S, xch, uin, uout, g, om, ybase, bh, bm, x, xg, out_col, Y0, Y1, nx,
                                                 ny, pitch, acc);
        march<T, ST, K, NORM, REFL, false, false>(S, xch, uin, uout, g, om, ybase, bm, bt, x, xg, out_col, Y0, Y1, nx,
                                                  ny, pitch, acc);
        march<T, ST, K, NORM, REFL, true, true>(S, xch, uin, uout, g, om, ybase, bt, nb, x, xg, out_col, Y0, Y1, nx, ny,
                                                pitch, acc);
    } else {
        // The outside nodes that an interior node reads are the columns 0 and
        // nx + 1 and the rows 0 and ny + 1; every other outside node may take
        // any value.  So the boundary selects run only in the wave that holds
        // column 0 or nx + 1 (the others take the variant without selects: the
        // choice is per wave, and every wave still meets one barrier per row
        // step), and, where the halo reaches a y-boundary, only in the blocks
        // that produce a row outside 1 .. ny at some level: level s produces
        // row ybase + t - (s - 1) - sR in step t.  A selected node keeps the
        // same value in every variant, so the variants give the same bits.
        // The loops run one after another over (possibly empty) ranges of
        // blocks; an alternative between two loops would make the compiler
        // spill the register window where they join.
        int bh = 0, bt = nb;   // blocks [0, bh) and [bt, nb) take the selects
        if (__ballot(x == 0 || x == nx + 1) != 0) {
            // The wave with the selects has the longest row step; at the
            // default priority the older wave on its SIMD issues first, and the
            // whole workgroup waits for the younger one at every barrier.
            __builtin_amdgcn_s_setprio(2);
            bt = 0;   // everything in the last loop, where fewer values are live
        } else if (edge_y) {
            const int lo = 1 - ybase + (K - 1) + K * R;      // first block whose lowest row is >= 1
            bh = lo <= 0 ? 0 : min((lo + U - 1) / U, nb);
            const int hi = ny - ybase - U + 1 + R;           // blocks b <= hi / U keep their rows <= ny
            bt = hi < 0 ? 0 : min(hi / U + 1, nb);
            bt = max(bt, bh);
        }
        // The loop without selects takes UF blocks per pass; a block left
        // over runs in the last loop, whose selects keep every interior
        // node's update.
        bt = bh + (bt - bh) / UF * UF;
        march<T, ST, K, NORM, REFL, true, true>(S, xch, uin, uout, g, om, ybase, 0, bh, x, xg, out_col, Y0, Y1, nx, ny,
                                                pitch, acc);
        march<T, ST, K, NORM, REFL, false, false, UF>(S, xch, uin, uout, g, om, ybase, bh, bt, x, xg, out_col, Y0, Y1,
                                                      nx, ny, pitch, acc);
        march<T, ST, K, NORM, REFL, true, true>(S, xch, uin, uout, g, om, ybase, bt, nb, x, xg, out_col, Y0, Y1, nx, ny,
                                                pitch, acc);
    }
    if (NORM) {
        const double tot = block_sum(acc);
        if (threadIdx.x == 0) part[tile] = tot;
    }
}

template <typename T, int ST, int K, bool NORM, bool REFL>
__global__ __launch_bounds__((March<T, ST, K>::SW)) void sweepk_kernel(const T* __restrict__ uin, T* __restrict__ uout,
                                                     const T* __restrict__ g, const T* __restrict__ w, int widx,
                                                     int nx, int ny, int pitch, int strips_x, int rows,
                                                     double* __restrict__ part) {
    // 12 row steps per pass (FP64 blocks are 6 steps, FP32 blocks 3)
    sweepk_tile<T, ST, K, NORM, REFL, sizeof(T) == 4 ? 4 : 2>(uin, uout, g, w, widx, nx, ny, pitch, strips_x, rows,
                                                              xcd_tile(blockIdx.x, gridDim.x), part);
}

// ------------------------------------------------------------ batched problems
// Many independent problems advance together: one launch runs K FP32 sweeps of
// every problem on the work list; workgroup b (mapped XCD-contiguously) takes
// work item b = (problem, tile).  A problem's current inner cycle began at
// super-step cycle_start; launch j = step - cycle_start of the cycle reads
// the correction buffer d[j & 1], writes d[(j + 1) & 1] and uses the weights
// w32[jK .. jK + K - 1].

template <int ST, int K>
__global__ __launch_bounds__(256) void batch_sweepk_kernel(const BatchProblem* __restrict__ probs,
                                                           const BatchItem* __restrict__ work, int step) {
    const BatchItem it = work[xcd_tile(blockIdx.x, gridDim.x)];
    const BatchProblem& pb = probs[it.prob];
    const int j = step - pb.cycle_start;
    const float* uin = (j & 1) ? pb.d2 : pb.d1;
    float* uout = (j & 1) ? pb.d1 : pb.d2;
    // one block per pass: the batch's many short tiles lost 5% with 12-step
    // passes (582 against 613 ms for 512 problems)
    sweepk_tile<float, ST, K, false, ST == 17, 1>(uin, uout, pb.r32, pb.w32, j * K, pb.nx, pb.ny, pb.pitch32,
                                                  pb.strips_x, pb.rows_k, it.tile, nullptr);
}

// Cycle end of one problem, per tile of the single-sweep geometry: u += d
// (interior; the 17-point outer ring follows by reflection, the Dirichlet ring
// stays zero).
template <int ST>
__global__ __launch_bounds__(256) void batch_correct_kernel(const BatchProblem* __restrict__ probs,
                                                            const BatchItem* __restrict__ work) {
    const BatchItem it = work[xcd_tile(blockIdx.x, gridDim.x)];
    const BatchProblem& pb = probs[it.prob];
    const float* d = pb.dcur ? pb.d2 : pb.d1;
    const int tx = it.tile % pb.tiles_x, ty = it.tile / pb.tiles_x;
    const int x = tx * 256 + (int)threadIdx.x + 1;
    if (x > pb.nx) return;
    const int y0 = ty * pb.rows + 1;
    const int y1 = min(y0 + pb.rows, pb.ny + 1);
    for (int y = y0; y < y1; ++y) {
        const double un = pb.u[at<double>(pb.pitch, x, y)] + (double)d[at<float>(pb.pitch32, x, y)];
        store_update<double, ST, ST == 17>(pb.u, pb.pitch, pb.nx, pb.ny, x, y, un);
    }
}

// Residual of one problem for its next inner solve, per tile (accurate_residual,
// as the single-problem refinement): r32 <- (float)r,
// the correction buffer d[dnext] <- 0 (with its reflected ring), partial sums
// of r^2 into part[work index].
template <int ST>
__global__ __launch_bounds__(256) void batch_residual_kernel(const BatchProblem* __restrict__ probs,
                                                             const BatchItem* __restrict__ work,
                                                             double* __restrict__ part) {
    constexpr int R = Stencil<ST>::R;
    constexpr int W = 2 * R + 1;
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const BatchItem it = work[b];
    const BatchProblem& pb = probs[it.prob];
    float* dz = pb.dnext ? pb.d2 : pb.d1;
    const int nx = pb.nx, ny = pb.ny, pitch = pb.pitch, pitch32 = pb.pitch32;
    const int tx = it.tile % pb.tiles_x, ty = it.tile / pb.tiles_x;
    const int x = tx * 256 + (int)threadIdx.x + 1;
    const bool active = x <= nx;
    const int xl = active ? x : nx;
    const int y0 = ty * pb.rows + 1;
    const int y1 = min(y0 + pb.rows, ny + 1);
    double v[W][W];
#pragma unroll
    for (int r = 1; r < W; ++r) {
        const double* p = pb.u + at<double>(pitch, xl - R, y0 - R + r - 1);
#pragma unroll
        for (int c = 0; c < W; ++c) v[r][c] = p[c];
    }
    double acc = 0.0;
    for (int y = y0; y < y1; ++y) {
#pragma unroll
        for (int r = 0; r < W - 1; ++r)
#pragma unroll
            for (int c = 0; c < W; ++c) v[r][c] = v[r + 1][c];
        const double* p = pb.u + at<double>(pitch, xl - R, y + R);
#pragma unroll
        for (int c = 0; c < W; ++c) v[W - 1][c] = p[c];
        const double gv = pb.g[at<double>(pitch, xl, y)];
        const double res = accurate_residual<ST>(v, gv);
        acc = fmat<double>(res, res, acc);
        if (active) {
            __builtin_nontemporal_store((float)res, pb.r32 + at<float>(pitch32, x, y));
            store_update<float, ST, ST == 17>(dz, pitch32, nx, ny, x, y, 0.0f);
        }
    }
    if (!active) acc = 0.0;
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) part[b] = tot;
}

// out[s] <- sum of part[seg[s] .. seg[s + 1]) in a fixed order; one workgroup per segment.
__global__ __launch_bounds__(256) void segmented_reduce_kernel(const double* __restrict__ part,
                                                               const int* __restrict__ seg,
                                                               double* __restrict__ out) {
    const int s = blockIdx.x;
    double acc = 0.0;
    for (int k = seg[s] + (int)threadIdx.x; k < seg[s + 1]; k += blockDim.x) acc += part[k];
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) out[s] = tot;
}

// ------------------------------------------------------------ iterative refinement
// Residual of the FP64 iterate for the inner solve: r = g - D^{-1}A u in
// FP64 (accurate_residual), stored in the inner precision TR (rounded to
// FP32, or kept in FP64) into r32; the correction d32 (also TR) is reset to
// zero (with its reflected ring for REFL); per-tile partial sums of r^2 in
// FP64.  With DD the iterate is the double-double hi + lo (u = hi), lo in
// the same layout.

template <int ST, bool REFL, bool DD, typename TR>
__global__ __launch_bounds__(256) void ir_residual_kernel(const double* __restrict__ u,
                                                          const double* __restrict__ lo,
                                                          const double* __restrict__ g, TR* __restrict__ r32,
                                                          TR* __restrict__ d32, int nx, int ny, int pitch,
                                                          int pitch32, int tiles_x, int rows,
                                                          double* __restrict__ part) {
    constexpr int R = Stencil<ST>::R;
    constexpr int W = 2 * R + 1;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int x = tx * (int)blockDim.x + (int)threadIdx.x + 1;
    const bool active = x <= nx;
    const int xl = active ? x : nx;
    const int y0 = ty * rows + 1;
    const int y1 = min(y0 + rows, ny + 1);
    double v[W][W], vl[DD ? W : 1][W];
#pragma unroll
    for (int r = 1; r < W; ++r) {
        const size_t o = at<double>(pitch, xl - R, y0 - R + r - 1);
#pragma unroll
        for (int c = 0; c < W; ++c) v[r][c] = u[o + c];
        if constexpr (DD) {
#pragma unroll
            for (int c = 0; c < W; ++c) vl[r][c] = lo[o + c];
        }
    }
    double acc = 0.0;
    for (int y = y0; y < y1; ++y) {
#pragma unroll
        for (int r = 0; r < W - 1; ++r)
#pragma unroll
            for (int c = 0; c < W; ++c) v[r][c] = v[r + 1][c];
        const size_t o = at<double>(pitch, xl - R, y + R);
#pragma unroll
        for (int c = 0; c < W; ++c) v[W - 1][c] = u[o + c];
        double dlo = 0.0;
        if constexpr (DD) {
#pragma unroll
            for (int r = 0; r < W - 1; ++r)
#pragma unroll
                for (int c = 0; c < W; ++c) vl[r][c] = vl[r + 1][c];
#pragma unroll
            for (int c = 0; c < W; ++c) vl[W - 1][c] = lo[o + c];
            dlo = plain_scaled_operator<ST>(vl);
        }
        const double gv = g[at<double>(pitch, xl, y)];
        const double res = accurate_residual<ST, DD>(v, gv, dlo);
        acc = fmat<double>(res, res, acc);
        if (active) {
            __builtin_nontemporal_store((TR)res, r32 + at<TR>(pitch32, x, y));
            store_update<TR, ST, REFL>(d32, pitch32, nx, ny, x, y, TR(0));
        }
    }
    if (!active) acc = 0.0;
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) part[tile] = tot;
}

// u += d over the whole padded frame (rows and columns -1 .. n+2): the
// Dirichlet ring of d is zero and its outer ring holds the reflection of its
// interior (homogeneous 17-point data) or zero (boundary data), so u keeps
// its boundary exactly.
template <typename TD>
__global__ __launch_bounds__(256) void ir_correct_kernel(double* __restrict__ u, const TD* __restrict__ d,
                                                         int nx, int ny, int pitch, int pitchd, int bx) {
    const int x = (int)(blockIdx.x % bx) * 256 + (int)threadIdx.x - 1;
    const int y = (int)(blockIdx.x / bx) - 1;
    if (x > nx + 2 || y > ny + 2) return;
    double* p = u + at<double>(pitch, x, y);
    *p = *p + (double)d[at<TD>(pitchd, x, y)];
}

// (hi, lo) += d over the whole padded frame, as a double-double: TwoSum of
// hi and d, its error added to lo, and the pair renormalised by a second
// TwoSum so that |lo| <= ulp(hi) / 2.  Round-to-nearest is symmetric, so the
// reflected rings of hi, lo and d stay odd reflections of the interior.
template <typename TD>
__global__ __launch_bounds__(256) void ir_correct_dd_kernel(double* __restrict__ hi, double* __restrict__ lo,
                                                            const TD* __restrict__ d, int nx, int ny, int pitch,
                                                            int pitch32, int bx) {
    const int x = (int)(blockIdx.x % bx) * 256 + (int)threadIdx.x - 1;
    const int y = (int)(blockIdx.x / bx) - 1;
    if (x > nx + 2 || y > ny + 2) return;
    const size_t i = at<double>(pitch, x, y);
    const double a = hi[i], b = (double)d[at<TD>(pitch32, x, y)];
    const double s = a + b;
    const double z = s - a;
    const double e = ((a - (s - z)) + (b - z)) + lo[i];
    const double h = s + e;
    const double z2 = h - s;
    hi[i] = h;
    lo[i] = (s - (h - z2)) + (e - z2);
}

// dst = (Tout) src over the whole padded frame.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void convert_kernel(const Tin* __restrict__ src, Tout* __restrict__ dst, int nx,
                                                      int ny, int pitch_in, int pitch_out, int bx) {
    const int x = (int)(blockIdx.x % bx) * 256 + (int)threadIdx.x - 1;
    const int y = (int)(blockIdx.x / bx) - 1;
    if (x > nx + 2 || y > ny + 2) return;
    dst[at<Tout>(pitch_out, x, y)] = (Tout)src[at<Tin>(pitch_in, x, y)];
}

// ------------------------------------------------------------ stage in / out

// Interior of A <- u, of G <- scale * f (zero when f is NULL); of B <- u, or
// zero when u carries a frame of width fg > 0 (B then holds the zero interior
// inside the boundary data, whose residual norm is the norm of the lifted
// right-hand side).  u is nx x ny (fg = 0) or (nx + 2fg) x (ny + 2fg).
__global__ __launch_bounds__(256) void stage_in_kernel(const double* __restrict__ f, const double* __restrict__ u,
                                                       double scale, double* __restrict__ A, double* __restrict__ B,
                                                       double* __restrict__ G, int nx, int ny, int pitch,
                                                       int tiles_x, int rows, double* __restrict__ part, int fg) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int x = tx * (int)blockDim.x + (int)threadIdx.x + 1;
    const int y0 = ty * rows + 1;
    const int y1 = min(y0 + rows, ny + 1);
    double acc = 0.0;
    if (x <= nx) {
        const size_t ustride = (size_t)nx + 2 * (size_t)fg;
        for (int y = y0; y < y1; ++y) {
            const size_t src = (size_t)(y - 1) * (size_t)nx + (size_t)(x - 1);
            const size_t usrc = (size_t)(y - 1 + fg) * ustride + (size_t)(x - 1 + fg);
            const size_t dst = at<double>(pitch, x, y);
            const double uv = u[usrc];
            const double gv = f ? scale * f[src] : 0.0;
            A[dst] = uv;
            B[dst] = fg ? 0.0 : uv;
            G[dst] = gv;
            acc = fmat<double>(gv, gv, acc);
        }
    }
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) part[tile] = tot;
}

// Ring values: index k enumerates the 2-wide padded ring around the interior.
// fg = 0: homogeneous data, the Dirichlet ring zero and the outer ring the odd
// reflection of u (nx x ny).  fg > 0: u is (nx + 2fg) x (ny + 2fg) and carries
// the boundary data in a frame of width fg; ring nodes beyond it are zero.
__global__ __launch_bounds__(256) void ring_kernel(const double* __restrict__ u, double* __restrict__ A,
                                                   double* __restrict__ B, double* __restrict__ G, int nx, int ny,
                                                   int pitch, int fg) {
    const int W = nx + 4;                 // stored columns -1 .. nx+2
    const int n_rows = 4 * W;             // rows -1, 0, ny+1, ny+2
    const int n_cols = 4 * ny;            // columns -1, 0, nx+1, nx+2 for rows 1..ny
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_rows + n_cols) return;
    int x, y;
    if (k < n_rows) {
        const int band = k / W;
        x = k % W - 1;
        y = band == 0 ? -1 : band == 1 ? 0 : band == 2 ? ny + 1 : ny + 2;
    } else {
        const int q = k - n_rows;
        const int band = q / ny;
        y = q % ny + 1;
        x = band == 0 ? -1 : band == 1 ? 0 : band == 2 ? nx + 1 : nx + 2;
    }
    double val = 0.0;
    if (fg > 0) {
        if (x >= 1 - fg && x <= nx + fg && y >= 1 - fg && y <= ny + fg)
            val = u[(size_t)(y - 1 + fg) * ((size_t)nx + 2 * (size_t)fg) + (size_t)(x - 1 + fg)];
    } else {
        // odd reflection about the Dirichlet nodes 0 and n + 1
        double sgn = 1.0;
        int xs = x, ys = y;
        if (xs < 0) { xs = -xs; sgn = -sgn; }
        if (xs > nx + 1) { xs = 2 * (nx + 1) - xs; sgn = -sgn; }
        if (ys < 0) { ys = -ys; sgn = -sgn; }
        if (ys > ny + 1) { ys = 2 * (ny + 1) - ys; sgn = -sgn; }
        if (xs >= 1 && xs <= nx && ys >= 1 && ys <= ny)
            val = sgn * u[(size_t)(ys - 1) * (size_t)nx + (size_t)(xs - 1)];
    }
    const size_t d = at<double>(pitch, x, y);
    A[d] = val;
    B[d] = val;
    G[d] = 0.0;
}

// Row-wise kernels use a 1D grid of bx blocks per row: block b covers row
// b / bx + 1, columns (b % bx) * 256 + 1 ...
// (u with a frame of width fg: its interior only.)
__global__ __launch_bounds__(256) void stage_out_kernel(const double* __restrict__ A, double* __restrict__ u,
                                                        int nx, int ny, int pitch, int bx, int fg) {
    const int x = (int)(blockIdx.x % bx) * 256 + (int)threadIdx.x + 1;
    const int y = (int)(blockIdx.x / bx) + 1;
    if (x > nx || y > ny) return;
    u[(size_t)(y - 1 + fg) * ((size_t)nx + 2 * (size_t)fg) + (size_t)(x - 1 + fg)] = A[at<double>(pitch, x, y)];
}

// ------------------------------------------------------------ whole solve in one workgroup
// Small grids (5- and 9-point): one workgroup of 1024 lanes holds the padded
// grid (rows and columns -1 .. n + 2) in LDS and runs the whole FP64 solve in
// one launch, with the stopping rule of the host loop: at every cycle end the
// residual of the iterate (a read-only pass, summed per lane in row order and
// reduced in a fixed order), then the test, then M sweeps.  A sweep computes
// the new values of a lane's nodes into registers from the LDS values,
// waits at a barrier, and writes them back (an in-place Jacobi step: every
// new value depends on old values only).  Each update is the expression of
// sweep_kernel (window_residual, then fma(omega, r, u)) on the same values, so
// the iterate has the same bits as the launched kernels; only the residual's
// summation order differs.  Lane mapping: wave w covers columns
// 1 + (w mod wx) * 64 + lane and the band w / wx of `band` rows; waves past
// the last band only join the barriers.  Three instantiations by the band
// height BR they allow: up to 4 and up to 8 rows keep each lane's g in
// registers for the whole solve; up to 16 rows read g again each sweep (L2),
// which the 128-register budget of 1024-lane workgroups would otherwise spill.
// out: [0] status (0 ok, 1 stagnated, -4 max cycles, -5 not finite),
// [1] cycles, [2] last relative residual, [3] floor estimate.

constexpr int kLdsSolveLanes = 1024;
constexpr int kLdsSolveRows = 16;      // rows of a lane's band at most
constexpr int kLdsSolveShortRows = 4;  // bands up to this height take the short variant
constexpr int kLdsSolveMidRows = 8;    // and up to this height the middle one (g also in registers)

// A double from lane - 1 (from_lower) or lane + 1 of the wave (whole-wave DPP
// shifts); the first (last) lane gets 0.
__device__ __forceinline__ double dpp_from_lower(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x138, 0xf, 0xf, true);        // wave_shr:1
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double dpp_from_upper(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x130, 0xf, 0xf, true);        // wave_shl:1
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int ST, int BR>
__global__ __launch_bounds__(1024) void lds_solve_kernel(double* __restrict__ A, const double* __restrict__ G,
                                                         const double* __restrict__ w, int M, int nx, int ny,
                                                         int pitch, int wx, int band, double gnorm, double tol,
                                                         int cycles_pred, int max_cycles,
                                                         double* __restrict__ out) {
    constexpr int R = Stencil<ST>::R;
    static_assert(R == 1, "5- and 9-point stencils");
    extern __shared__ double lds[];
    const int P = nx + 4;                     // LDS row: columns -1 .. nx + 2
    double* red = lds + (size_t)(ny + 4) * P; // 16 wave sums, then the decision
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int x = 1 + (wave % wx) * 64 + lane;
    const int y0 = 1 + (wave / wx) * band;
    const int y1 = min(y0 + band, ny + 1);
    const bool in_band = wave / wx < 16 / wx && y0 <= ny;  // uniform per wave
    const bool active = in_band && x <= nx;
    // each lane holds its column's value of a row (lanes past the grid the
    // ring column nx + 1, which the last interior lane needs from its
    // neighbour); x - 1 and x + 1 come from the neighbouring lanes, across
    // wave edges from LDS
    const int xc = min(x, nx + 1);
    const int xg = min(x, nx);
    auto lat = [&](int xx, int yy) { return (size_t)(yy + 1) * P + (xx + 1); };
    // summary {C, P_1} of row yy from the lane's value c there, as row_summary forms it
    auto summarise = [&](double c, int yy, double (&sm)[2]) {
        double l = dpp_from_lower(c), r = dpp_from_upper(c);
        if (lane == 0) l = lds[lat(xc - 1, yy)];
        if (lane == 63) r = lds[lat(min(xc + 1, nx + 2), yy)];
        sm[0] = c;
        sm[1] = l + r;
    };
    // r of the band's rows in order, handed to body(k, r, u) (rows held as a
    // rolling window of summaries; the next row's value and g are loaded one
    // row ahead)
    // Bands of at most kLdsSolveMidRows rows keep their g in registers for
    // the whole solve; taller bands read it again each sweep (from L2) so as
    // not to spill.
    constexpr bool kGInRegs = BR <= kLdsSolveMidRows;
    double greg[kGInRegs ? BR : 1];
    if constexpr (kGInRegs) {
#pragma unroll
        for (int k = 0; k < BR; ++k)
            greg[k] = (in_band && y0 + k < y1) ? G[at<double>(pitch, xg, y0 + k)] : 0.0;
    }
    auto band_rows = [&](auto&& body) {
        double sm[3][2];
        summarise(lds[lat(xc, y0 - 1)], y0 - 1, sm[1]);
        summarise(lds[lat(xc, y0)], y0, sm[2]);
        double cn = lds[lat(xc, y0 + 1)];
        double gn = 0.0;
        if constexpr (!kGInRegs) gn = G[at<double>(pitch, xg, y0)];
#pragma unroll
        for (int k = 0; k < BR; ++k) {
            if (y0 + k < y1) {
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    sm[r][0] = sm[r + 1][0];
                    sm[r][1] = sm[r + 1][1];
                }
                summarise(cn, y0 + k + 1, sm[2]);
                double g;
                if constexpr (kGInRegs) {
                    g = greg[k];
                } else {
                    g = gn;
                }
                if (y0 + k + 1 < y1) {
                    cn = lds[lat(xc, y0 + k + 2)];
                    if constexpr (!kGInRegs) gn = G[at<double>(pitch, xg, y0 + k + 1)];
                }
                body(k, summary_residual<double, ST>(sm, g, sm[1][0]), sm[1][0]);
            }
        }
    };
    for (int i = tid; i < (ny + 4) * P; i += kLdsSolveLanes) {
        const int yy = i / P - 1, xx = i % P - 1;
        lds[i] = A[at<double>(pitch, xx, yy)];
    }
    __syncthreads();

    auto residual_sum = [&]() {
        double acc = 0.0;
        if (in_band)
            band_rows([&](int, double res, double) {
                if (active) acc = fmat<double>(res, res, acc);
            });
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) red[wave] = acc;
        __syncthreads();
        double tot = 0.0;
        if (tid == 0) {
            tot = red[0];
            for (int k = 1; k < kLdsSolveLanes / 64; ++k) tot += red[k];
        }
        return tot;
    };

    double prev = 0.0, rr = 0.0;
    int c = 0, status = 0;
    for (;;) {
        const double r2 = residual_sum();
        if (tid == 0) {
            rr = __builtin_sqrt(r2) / gnorm;
            int stop = 1;
            if (!(rr - rr == 0.0)) {
                status = -5;
            } else if (rr <= tol) {
                status = 0;
            } else if (c >= 1 && c >= cycles_pred && rr > 0.5 * prev) {
                status = 1;
                out[3] = rr < prev ? rr : prev;
            } else if (c >= max_cycles) {
                status = -4;
            } else {
                stop = 0;
            }
            red[16] = stop ? 1.0 : 0.0;
            prev = rr;
        }
        __syncthreads();
        const bool stop = red[16] != 0.0;
        __syncthreads();   // every lane has read the decision before the slots are reused
        if (stop) break;
        for (int j = 0; j < M; ++j) {
            const double omega = w[j];
            double un[BR];
            if (in_band)
                band_rows([&](int k, double res, double u) { un[k] = fmat<double>(omega, res, u); });
            __syncthreads();
            if (active) {
#pragma unroll
                for (int k = 0; k < BR; ++k)
                    if (y0 + k < y1) lds[lat(x, y0 + k)] = un[k];
            }
            __syncthreads();
        }
        ++c;
    }
    for (int i = tid; i < nx * ny; i += kLdsSolveLanes) {
        const int yy = i / nx + 1, xx = i % nx + 1;
        A[at<double>(pitch, xx, yy)] = lds[lat(xx, yy)];
    }
    if (tid == 0) {
        out[0] = (double)status;
        out[1] = (double)c;
        out[2] = rr;
    }
}

// ------------------------------------------------------------ reduction / apply

__global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
    double acc = 0.0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) acc += part[k];
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) out[0] = tot;
}

template <int ST>
__global__ __launch_bounds__(256) void apply_kernel(const double* __restrict__ A, double dscale,
                                                    double* __restrict__ au, int nx, int ny, int pitch, int bx) {
    constexpr int R = Stencil<ST>::R;
    constexpr int W = 2 * R + 1;
    const int x = (int)(blockIdx.x % bx) * 256 + (int)threadIdx.x + 1;
    const int y = (int)(blockIdx.x / bx) + 1;
    if (x > nx || y > ny) return;
    double v[W][W];
#pragma unroll
    for (int r = 0; r < W; ++r)
#pragma unroll
        for (int c = 0; c < W; ++c) v[r][c] = A[at<double>(pitch, x - R + c, y - R + r)];
    au[(size_t)(y - 1) * (size_t)nx + (size_t)(x - 1)] = dscale * (v[R][R] - neighbour_sum<double, ST>(v));
}

// ------------------------------------------------------------ allocation-free residual
// The relative residual of cj_residual read straight from the caller's arrays,
// with no staging copy: window values come from u itself (homogeneous data:
// zero on the Dirichlet ring and the odd reflection beyond it; boundary data:
// the frame array), g = scale * f is formed as stage-in forms it, and the
// per-tile partial sums follow the same tiles, rows and orders as the staged
// path (r^2 as the residual kernel sums it; the denominator as stage-in sums
// g^2 or, with a frame, as the residual kernel sums the residual of the zero
// interior), so both paths reduce the same partial sums in the same order.

// Value at node (x, y), -R <= x - 1, of the caller's u: fg = 0, the nx x ny
// interior with the homogeneous ring (zero at 0 and n + 1, odd reflection at
// -1 and n + 2); fg > 0, the (nx + 2 fg) x (ny + 2 fg) frame array, with the
// interior read as zero when zero_interior is set.
__device__ __forceinline__ double user_node(const double* __restrict__ u, int nx, int ny, int fg, int x, int y,
                                            bool zero_interior) {
    if (fg > 0) {
        if (zero_interior && x >= 1 && x <= nx && y >= 1 && y <= ny) return 0.0;
        return u[(size_t)(y - 1 + fg) * ((size_t)nx + 2 * (size_t)fg) + (size_t)(x - 1 + fg)];
    }
    double sgn = 1.0;
    if (x < 0) { x = -x; sgn = -sgn; }
    if (x > nx + 1) { x = 2 * (nx + 1) - x; sgn = -sgn; }
    if (y < 0) { y = -y; sgn = -sgn; }
    if (y > ny + 1) { y = 2 * (ny + 1) - y; sgn = -sgn; }
    if (x < 1 || x > nx || y < 1 || y > ny) return 0.0;
    return sgn * u[(size_t)(y - 1) * (size_t)nx + (size_t)(x - 1)];
}

template <int ST, bool FRAME>
__global__ __launch_bounds__(256) void residual_noalloc_kernel(const double* __restrict__ f,
                                                               const double* __restrict__ u, double scale, int nx,
                                                               int ny, int tiles_x, int rows,
                                                               double* __restrict__ part_r,
                                                               double* __restrict__ part_d) {
    constexpr int R = Stencil<ST>::R;
    constexpr int W = 2 * R + 1;
    constexpr int FG = FRAME ? R : 0;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int x = tx * (int)blockDim.x + (int)threadIdx.x + 1;
    const bool active = x <= nx;
    const int xl = active ? x : nx;   // idle lanes read a valid column; their sums are dropped
    const int y0 = ty * rows + 1;
    const int y1 = min(y0 + rows, ny + 1);
    double v[W][W], v0[FRAME ? W : 1][W];
#pragma unroll
    for (int r = 1; r < W; ++r)
#pragma unroll
        for (int c = 0; c < W; ++c) {
            v[r][c] = user_node(u, nx, ny, FG, xl - R + c, y0 - R + r - 1, false);
            if (FRAME) v0[r][c] = user_node(u, nx, ny, FG, xl - R + c, y0 - R + r - 1, true);
        }
    double acc = 0.0, accd = 0.0;
    for (int y = y0; y < y1; ++y) {
#pragma unroll
        for (int r = 0; r < W - 1; ++r)
#pragma unroll
            for (int c = 0; c < W; ++c) {
                v[r][c] = v[r + 1][c];
                if (FRAME) v0[r][c] = v0[r + 1][c];
            }
#pragma unroll
        for (int c = 0; c < W; ++c) {
            v[W - 1][c] = user_node(u, nx, ny, FG, xl - R + c, y + R, false);
            if (FRAME) v0[W - 1][c] = user_node(u, nx, ny, FG, xl - R + c, y + R, true);
        }
        const double gv = scale * f[(size_t)(y - 1) * (size_t)nx + (size_t)(xl - 1)];
        const double res = window_residual<double, ST>(v, gv);
        acc = fmat<double>(res, res, acc);
        if constexpr (FRAME) {
            const double res0 = window_residual<double, ST>(v0, gv);
            accd = fmat<double>(res0, res0, accd);
        } else {
            accd = fmat<double>(gv, gv, accd);
        }
    }
    if (!active) {
        acc = 0.0;
        accd = 0.0;
    }
    const double tr = block_sum(acc);
    __syncthreads();   // thread 0 has read block_sum's shared slots before they are reused
    const double td = block_sum(accd);
    if (threadIdx.x == 0) {
        part_r[tile] = tr;
        part_d[tile] = td;
    }
}

// out[0] <- sqrt(sum part_r) / sqrt(sum part_d) (0 when the second sum is 0),
// each sum in reduce_kernel's order.
__global__ __launch_bounds__(256) void ratio_kernel(const double* __restrict__ part_r,
                                                    const double* __restrict__ part_d, int n,
                                                    double* __restrict__ out) {
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        a += part_r[k];
        b += part_d[k];
    }
    const double r2 = block_sum(a);
    __syncthreads();
    const double d2 = block_sum(b);
    if (threadIdx.x == 0) out[0] = d2 == 0.0 ? 0.0 : __builtin_sqrt(r2) / __builtin_sqrt(d2);
}

// The 17-point stencil has two kernel families: REFL for homogeneous data
// (reflected outer ring) and one for boundary data in a frame (L.frame > 0).
// The 5- and 9-point kernels read only the Dirichlet ring, which is data in
// both cases.
template <typename T, int ST, bool WRITE, bool NORM>
hipError_t launch_tile(const Layout& L, const Tiles& Tl, const T* uin, T* uout, const T* g, const T* w, int widx,
                       double* part, hipStream_t s) {
    if (ST == 17 && L.frame == 0)
        hipLaunchKernelGGL((sweep_kernel<T, ST, WRITE, NORM, true>), dim3(Tl.count()), dim3(Tl.width), 0, s, uin,
                           uout, g, w, widx, L.nx, L.ny, L.pitch, Tl.tiles_x, Tl.rows, part);
    else
        hipLaunchKernelGGL((sweep_kernel<T, ST, WRITE, NORM, false>), dim3(Tl.count()), dim3(Tl.width), 0, s, uin,
                           uout, g, w, widx, L.nx, L.ny, L.pitch, Tl.tiles_x, Tl.rows, part);
    return hipGetLastError();
}

template <typename T, int ST, int K, bool NORM>
void launch_k_refl(const Layout& L, const Tiles& Tl, const T* uin, T* uout, const T* g, const T* w, int widx,
                   double* part, hipStream_t s) {
    if (ST == 17 && L.frame == 0)
        hipLaunchKernelGGL((sweepk_kernel<T, ST, K, NORM, true>), dim3(Tl.count()), dim3(March<T, ST, K>::SW), 0, s, uin, uout, g,
                           w, widx, L.nx, L.ny, L.pitch, Tl.tiles_x, Tl.rows, part);
    else
        hipLaunchKernelGGL((sweepk_kernel<T, ST, K, NORM, false>), dim3(Tl.count()), dim3(March<T, ST, K>::SW), 0, s, uin, uout, g,
                           w, widx, L.nx, L.ny, L.pitch, Tl.tiles_x, Tl.rows, part);
}

template <typename T, int ST, int K>
hipError_t launch_k(const Layout& L, const Tiles& Tl, const T* uin, T* uout, const T* g, const T* w, int widx,
                    double* part, hipStream_t s) {
    if (part)
        launch_k_refl<T, ST, K, true>(L, Tl, uin, uout, g, w, widx, part, s);
    else
        launch_k_refl<T, ST, K, false>(L, Tl, uin, uout, g, w, widx, part, s);
    return hipGetLastError();
}

int frame_blocks(const Layout& L, int* bx) {
    *bx = (L.nx + 4 + 255) / 256;
    return *bx * (L.ny + 4);
}

}  // namespace

// ------------------------------------------------------------ launchers

hipError_t launch_stage_in(const Layout& L, const Tiles& T, const double* f, const double* u, double scale,
                           double* A, double* B, double* G, double* part, hipStream_t stream) {
    hipLaunchKernelGGL(stage_in_kernel, dim3(T.count()), dim3(T.width), 0, stream, f, u, scale, A, B, G, L.nx,
                       L.ny, L.pitch, T.tiles_x, T.rows, part, L.frame);
    return hipGetLastError();
}

hipError_t launch_ring(const Layout& L, const double* u, double* A, double* B, double* G, hipStream_t stream) {
    const int n = 4 * (L.nx + 4) + 4 * L.ny;
    hipLaunchKernelGGL(ring_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, u, A, B, G, L.nx, L.ny, L.pitch,
                       L.frame);
    return hipGetLastError();
}

hipError_t launch_stage_out(const Layout& L, const double* A, double* u, hipStream_t stream) {
    const int bx = (L.nx + 255) / 256;
    hipLaunchKernelGGL(stage_out_kernel, dim3(bx * L.ny), dim3(256), 0, stream, A, u, L.nx, L.ny, L.pitch, bx,
                       L.frame);
    return hipGetLastError();
}

namespace {
template <typename T>
hipError_t sweep_dispatch(int stencil, const Layout& L, const Tiles& Tl, const T* uin, T* uout, const T* g,
                          const T* w, int widx, double* part, hipStream_t stream) {
    const bool norm = part != nullptr;
    if (norm && sizeof(T) != sizeof(double)) return hipErrorInvalidValue;
    switch (stencil) {
    case 5:
        return norm ? launch_tile<T, 5, true, true>(L, Tl, uin, uout, g, w, widx, part, stream)
                    : launch_tile<T, 5, true, false>(L, Tl, uin, uout, g, w, widx, part, stream);
    case 9:
        return norm ? launch_tile<T, 9, true, true>(L, Tl, uin, uout, g, w, widx, part, stream)
                    : launch_tile<T, 9, true, false>(L, Tl, uin, uout, g, w, widx, part, stream);
    case 17:
        return norm ? launch_tile<T, 17, true, true>(L, Tl, uin, uout, g, w, widx, part, stream)
                    : launch_tile<T, 17, true, false>(L, Tl, uin, uout, g, w, widx, part, stream);
    default:
        return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_sweep(int stencil, const Layout& L, const Tiles& Tl, const double* uin, double* uout,
                        const double* g, const double* w, int widx, double* part, hipStream_t stream) {
    return sweep_dispatch<double>(stencil, L, Tl, uin, uout, g, w, widx, part, stream);
}

hipError_t launch_sweep(int stencil, const Layout& L, const Tiles& Tl, const float* uin, float* uout,
                        const float* g, const float* w, int widx, double* part, hipStream_t stream) {
    return sweep_dispatch<float>(stencil, L, Tl, uin, uout, g, w, widx, part, stream);
}

bool sweepk_supported(int stencil, int K, int elem_bytes) {
    if (elem_bytes == 4) {
        if (stencil == 17) return K == 2 || K == 3 || K == 4;
        return K == 2 || K == 4 || K == 8;
    }
    if (stencil == 17) return K == 2 || K == 3 || K == 4;
    return K == 2 || K == 3 || K == 4 || K == 6 || K == 8 || K == 10;
}

hipError_t launch_sweepk(int stencil, int K, const Layout& L, const Tiles& Tl, const double* uin,
                                 double* uout, const double* g, const double* w, int widx, double* part,
                                 hipStream_t stream) {
#define CJ_K_CASE(ST, KK) \
    if (stencil == ST && K == KK) return launch_k<double, ST, KK>(L, Tl, uin, uout, g, w, widx, part, stream);
    CJ_K_CASE(5, 2) CJ_K_CASE(5, 3) CJ_K_CASE(5, 4) CJ_K_CASE(5, 6) CJ_K_CASE(5, 8)
    CJ_K_CASE(9, 2) CJ_K_CASE(9, 3) CJ_K_CASE(9, 4) CJ_K_CASE(9, 6) CJ_K_CASE(9, 8) CJ_K_CASE(9, 10)
    CJ_K_CASE(5, 10) CJ_K_CASE(17, 2) CJ_K_CASE(17, 3) CJ_K_CASE(17, 4)
#undef CJ_K_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_sweepk(int stencil, int K, const Layout& L, const Tiles& Tl, const float* uin, float* uout,
                                const float* g, const float* w, int widx, double* part, hipStream_t stream) {
    if (part) return hipErrorInvalidValue;
#define CJ_K_CASE(ST, KK) \
    if (stencil == ST && K == KK) return launch_k<float, ST, KK>(L, Tl, uin, uout, g, w, widx, nullptr, stream);
    CJ_K_CASE(5, 2) CJ_K_CASE(5, 4) CJ_K_CASE(5, 8)
    CJ_K_CASE(9, 2) CJ_K_CASE(9, 4) CJ_K_CASE(9, 8)
    CJ_K_CASE(17, 2) CJ_K_CASE(17, 3) CJ_K_CASE(17, 4)
#undef CJ_K_CASE
    return hipErrorInvalidValue;
}

namespace {
template <typename T, int ST, int K>
hipError_t occupancy_k(bool refl, int* blocks) {
    if (ST == 17 && refl)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sweepk_kernel<T, ST, K, false, true>,
                                                           March<T, ST, K>::SW, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sweepk_kernel<T, ST, K, false, false>,
                                                           March<T, ST, K>::SW, 0);
}
}  // namespace

hipError_t sweepk_blocks_per_cu(int stencil, int K, int elem_bytes, bool refl, int* blocks) {
    *blocks = 0;
    if (elem_bytes == 8) {
#define CJ_K_CASE(ST, KK) \
        if (stencil == ST && K == KK) return occupancy_k<double, ST, KK>(refl, blocks);
        CJ_K_CASE(5, 2) CJ_K_CASE(5, 3) CJ_K_CASE(5, 4) CJ_K_CASE(5, 6) CJ_K_CASE(5, 8)
        CJ_K_CASE(9, 2) CJ_K_CASE(9, 3) CJ_K_CASE(9, 4) CJ_K_CASE(9, 6) CJ_K_CASE(9, 8) CJ_K_CASE(9, 10)
        CJ_K_CASE(5, 10) CJ_K_CASE(17, 2) CJ_K_CASE(17, 3) CJ_K_CASE(17, 4)
#undef CJ_K_CASE
    } else {
#define CJ_K_CASE(ST, KK) \
        if (stencil == ST && K == KK) return occupancy_k<float, ST, KK>(refl, blocks);
        CJ_K_CASE(5, 2) CJ_K_CASE(5, 4) CJ_K_CASE(5, 8)
        CJ_K_CASE(9, 2) CJ_K_CASE(9, 4) CJ_K_CASE(9, 8)
        CJ_K_CASE(17, 2) CJ_K_CASE(17, 3) CJ_K_CASE(17, 4)
#undef CJ_K_CASE
    }
    return hipErrorInvalidValue;
}

hipError_t launch_residual(int stencil, const Layout& L, const Tiles& T, const double* u, const double* g,
                           double* part, hipStream_t stream) {
    switch (stencil) {
    case 5: return launch_tile<double, 5, false, true>(L, T, u, nullptr, g, nullptr, 0, part, stream);
    case 9: return launch_tile<double, 9, false, true>(L, T, u, nullptr, g, nullptr, 0, part, stream);
    case 17: return launch_tile<double, 17, false, true>(L, T, u, nullptr, g, nullptr, 0, part, stream);
    default: return hipErrorInvalidValue;
    }
}

namespace {

template <typename TR>
hipError_t ir_residual_launch(int stencil, const Layout& L, const Layout& LR, const Tiles& T, const double* u,
                              const double* lo, const double* g, TR* r, TR* d, double* part, hipStream_t stream) {
    const dim3 grid(T.count()), block(T.width);
#define CJ_IR_CASE(ST, REFL)                                                                                    \
        if (lo)                                                                                                 \
            hipLaunchKernelGGL((ir_residual_kernel<ST, REFL, true, TR>), grid, block, 0, stream, u, lo, g, r,  \
                               d, L.nx, L.ny, L.pitch, LR.pitch, T.tiles_x, T.rows, part);                      \
        else                                                                                                    \
            hipLaunchKernelGGL((ir_residual_kernel<ST, REFL, false, TR>), grid, block, 0, stream, u, lo, g, r, \
                               d, L.nx, L.ny, L.pitch, LR.pitch, T.tiles_x, T.rows, part);
    switch (stencil) {
    case 5: CJ_IR_CASE(5, false) break;
    case 9: CJ_IR_CASE(9, false) break;
    case 17:
        if (L.frame == 0) {
            CJ_IR_CASE(17, true)
        } else {
            CJ_IR_CASE(17, false)
        }
        break;
    default: return hipErrorInvalidValue;
    }
#undef CJ_IR_CASE
    return hipGetLastError();
}

template <typename TD>
hipError_t ir_correct_launch(const Layout& L, const Layout& LD, double* u, double* lo, const TD* d,
                             hipStream_t stream) {
    int bx = 0;
    const int nb = frame_blocks(L, &bx);
    if (lo)
        hipLaunchKernelGGL((ir_correct_dd_kernel<TD>), dim3(nb), dim3(256), 0, stream, u, lo, d, L.nx, L.ny,
                           L.pitch, LD.pitch, bx);
    else
        hipLaunchKernelGGL((ir_correct_kernel<TD>), dim3(nb), dim3(256), 0, stream, u, d, L.nx, L.ny, L.pitch,
                           LD.pitch, bx);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ir_residual(int stencil, const Layout& L, const Layout& L32, const Tiles& T, const double* u,
                              const double* lo, const double* g, float* r32, float* d32, double* part,
                              hipStream_t stream) {
    return ir_residual_launch<float>(stencil, L, L32, T, u, lo, g, r32, d32, part, stream);
}

hipError_t launch_ir_residual(int stencil, const Layout& L, const Tiles& T, const double* u, const double* lo,
                              const double* g, double* r, double* d, double* part, hipStream_t stream) {
    return ir_residual_launch<double>(stencil, L, L, T, u, lo, g, r, d, part, stream);
}

hipError_t launch_ir_correct(const Layout& L, const Layout& L32, double* u, double* lo, const float* d,
                             hipStream_t stream) {
    return ir_correct_launch<float>(L, L32, u, lo, d, stream);
}

hipError_t launch_ir_correct(const Layout& L, double* u, double* lo, const double* d, hipStream_t stream) {
    return ir_correct_launch<double>(L, L, u, lo, d, stream);
}

hipError_t launch_to_f32(const Layout& L, const Layout& L32, const double* src, float* dst, hipStream_t stream) {
    int bx = 0;
    const int nb = frame_blocks(L, &bx);
    hipLaunchKernelGGL((convert_kernel<double, float>), dim3(nb), dim3(256), 0, stream, src, dst, L.nx, L.ny,
                       L.pitch, L32.pitch, bx);
    return hipGetLastError();
}

hipError_t launch_from_f32(const Layout& L, const Layout& L32, const float* src, double* dst, hipStream_t stream) {
    int bx = 0;
    const int nb = frame_blocks(L, &bx);
    hipLaunchKernelGGL((convert_kernel<float, double>), dim3(nb), dim3(256), 0, stream, src, dst, L.nx, L.ny,
                       L32.pitch, L.pitch, bx);
    return hipGetLastError();
}

hipError_t launch_batch_sweepk(int stencil, int K, const BatchProblem* probs, const BatchItem* work, int n_items,
                               int step, hipStream_t stream) {
    if (n_items <= 0) return hipSuccess;
#define CJ_BK_CASE(ST, KK)                                                                                   \
    if (stencil == ST && K == KK) {                                                                        \
        hipLaunchKernelGGL((batch_sweepk_kernel<ST, KK>), dim3(n_items), dim3(256), 0, stream, probs, work, \
                           step);                                                                          \
        return hipGetLastError();                                                                          \
    }
    CJ_BK_CASE(5, 2) CJ_BK_CASE(5, 4) CJ_BK_CASE(5, 8)
    CJ_BK_CASE(9, 2) CJ_BK_CASE(9, 4) CJ_BK_CASE(9, 8)
    CJ_BK_CASE(17, 2) CJ_BK_CASE(17, 3) CJ_BK_CASE(17, 4)
#undef CJ_BK_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_batch_correct(int stencil, const BatchProblem* probs, const BatchItem* work, int n_items,
                                hipStream_t stream) {
    if (n_items <= 0) return hipSuccess;
    switch (stencil) {
    case 5: hipLaunchKernelGGL(batch_correct_kernel<5>, dim3(n_items), dim3(256), 0, stream, probs, work); break;
    case 9: hipLaunchKernelGGL(batch_correct_kernel<9>, dim3(n_items), dim3(256), 0, stream, probs, work); break;
    case 17: hipLaunchKernelGGL(batch_correct_kernel<17>, dim3(n_items), dim3(256), 0, stream, probs, work); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_residual(int stencil, const BatchProblem* probs, const BatchItem* work, int n_items,
                                 double* part, hipStream_t stream) {
    if (n_items <= 0) return hipSuccess;
    switch (stencil) {
    case 5:
        hipLaunchKernelGGL(batch_residual_kernel<5>, dim3(n_items), dim3(256), 0, stream, probs, work, part);
        break;
    case 9:
        hipLaunchKernelGGL(batch_residual_kernel<9>, dim3(n_items), dim3(256), 0, stream, probs, work, part);
        break;
    case 17:
        hipLaunchKernelGGL(batch_residual_kernel<17>, dim3(n_items), dim3(256), 0, stream, probs, work, part);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_segmented_reduce(const double* part, const int* seg, int n_seg, double* out, hipStream_t stream) {
    if (n_seg <= 0) return hipSuccess;
    hipLaunchKernelGGL(segmented_reduce_kernel, dim3(n_seg), dim3(256), 0, stream, part, seg, out);
    return hipGetLastError();
}

bool lds_solve_fits(int stencil, int nx, int ny, int* wx, int* band, size_t* lds_bytes) {
    if (stencil != 5 && stencil != 9) return false;
    const int w = (nx + 63) / 64;
    if (w > kLdsSolveLanes / 64) return false;
    const int bands = (kLdsSolveLanes / 64) / w;
    const int b = (ny + bands - 1) / bands;
    if (b > kLdsSolveRows) return false;
    const size_t bytes = ((size_t)(nx + 4) * (size_t)(ny + 4) + 17) * sizeof(double);
    if (bytes > 160 * 1024) return false;
    if (wx) *wx = w;
    if (band) *band = b;
    if (lds_bytes) *lds_bytes = bytes;
    return true;
}

hipError_t launch_lds_solve(int stencil, const Layout& L, double* A, const double* G, const double* w, int M,
                            double gnorm, double tol, int cycles_pred, int max_cycles, double* out,
                            hipStream_t stream) {
    int wx = 0, band = 0;
    size_t bytes = 0;
    if (!lds_solve_fits(stencil, L.nx, L.ny, &wx, &band, &bytes) || L.frame > 1) return hipErrorInvalidValue;
    const int br = band <= kLdsSolveShortRows ? kLdsSolveShortRows
                 : band <= kLdsSolveMidRows ? kLdsSolveMidRows : kLdsSolveRows;
    const void* fn = nullptr;
    if (stencil == 5)
        fn = br == kLdsSolveShortRows ? (const void*)lds_solve_kernel<5, kLdsSolveShortRows>
           : br == kLdsSolveMidRows ? (const void*)lds_solve_kernel<5, kLdsSolveMidRows>
                                    : (const void*)lds_solve_kernel<5, kLdsSolveRows>;
    else
        fn = br == kLdsSolveShortRows ? (const void*)lds_solve_kernel<9, kLdsSolveShortRows>
           : br == kLdsSolveMidRows ? (const void*)lds_solve_kernel<9, kLdsSolveMidRows>
                                    : (const void*)lds_solve_kernel<9, kLdsSolveRows>;
    // the dynamic LDS limit is a property of the function on the current
    // device: set it at every launch (one host call per solve), so that every
    // device the library runs on gets it
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
#define CJ_LDS_SOLVE(ST, BR)                                                                                  \
    hipLaunchKernelGGL((lds_solve_kernel<ST, BR>), dim3(1), dim3(kLdsSolveLanes), bytes, stream, A, G, w, M, \
                       L.nx, L.ny, L.pitch, wx, band, gnorm, tol, cycles_pred, max_cycles, out)
    if (stencil == 5) {
        if (br == kLdsSolveShortRows) CJ_LDS_SOLVE(5, kLdsSolveShortRows);
        else if (br == kLdsSolveMidRows) CJ_LDS_SOLVE(5, kLdsSolveMidRows);
        else CJ_LDS_SOLVE(5, kLdsSolveRows);
    } else {
        if (br == kLdsSolveShortRows) CJ_LDS_SOLVE(9, kLdsSolveShortRows);
        else if (br == kLdsSolveMidRows) CJ_LDS_SOLVE(9, kLdsSolveMidRows);
        else CJ_LDS_SOLVE(9, kLdsSolveRows);
    }
#undef CJ_LDS_SOLVE
    return hipGetLastError();
}

hipError_t launch_reduce(const double* part, int n, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, stream, part, n, out);
    return hipGetLastError();
}

hipError_t launch_apply(int stencil, const Layout& L, const double* A, double dscale, double* au,
                        hipStream_t stream) {
    const int bx = (L.nx + 255) / 256;
    const dim3 grid(bx * L.ny), block(256);
    switch (stencil) {
    case 5: hipLaunchKernelGGL(apply_kernel<5>, grid, block, 0, stream, A, dscale, au, L.nx, L.ny, L.pitch, bx); break;
    case 9: hipLaunchKernelGGL(apply_kernel<9>, grid, block, 0, stream, A, dscale, au, L.nx, L.ny, L.pitch, bx); break;
    case 17:
        hipLaunchKernelGGL(apply_kernel<17>, grid, block, 0, stream, A, dscale, au, L.nx, L.ny, L.pitch, bx);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

Layout make_layout(int nx, int ny, int elem_bytes, int frame) {
    Layout L;
    L.frame = frame;
    L.nx = nx;
    L.ny = ny;
    L.elem_bytes = elem_bytes;
    const int line = 128 / elem_bytes;                // elements per 128-byte line
    int pitch = nx + xoff_of(elem_bytes) + 3;         // columns up to x = nx + 2
    pitch = (pitch + line - 1) / line * line;         // 128-byte rows
    if (((long long)pitch * elem_bytes) % 4096 == 0) pitch += line;   // avoid 4 KB-multiple row strides
    L.pitch = pitch;
    L.elems = (size_t)(ny + 4) * (size_t)pitch;
    return L;
}

Tiles make_tiles_k(int nx, int ny, int K, int R, int rows_request, int elem_bytes) {
    Tiles T;
    T.width = strip_lanes(R, K, elem_bytes) - 2 * K * R;   // output columns per strip
    T.tiles_x = (nx + T.width - 1) / T.width;
    int rows = rows_request > 0 ? rows_request : 128;
    if (rows_request <= 0)
        while (rows > 16 && (long long)T.tiles_x * ((ny + rows - 1) / rows) < 2048) rows /= 2;
    if (rows > ny) rows = ny;
    T.rows = rows;
    T.tiles_y = (ny + rows - 1) / rows;
    return T;
}

Tiles make_tiles(int nx, int ny, int rows_request) {
    Tiles T;
    T.width = nx >= 256 ? 256 : ((nx + 63) / 64) * 64;
    T.tiles_x = (nx + T.width - 1) / T.width;
    int rows = rows_request > 0 ? rows_request : 16;
    if (rows_request <= 0)
        while (rows > 4 && (long long)T.tiles_x * ((ny + rows - 1) / rows) < 2048) rows /= 2;
    if (rows > ny) rows = ny;
    T.rows = rows;
    T.tiles_y = (ny + rows - 1) / rows;
    return T;
}

}  // namespace cj

// Scratch of cj_residual_noalloc: the per-tile partial sums of the residual
// (first kNoallocMaxTiles doubles) and of the denominator (the next ones).
// Every device the library runs on holds its own copy until the process ends;
// host code reaches it only through the address hipGetSymbolAddress gives on
// that device.
static __device__ __align__(256) double scratch[2 * cj::kNoallocMaxTiles];

namespace cj {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(double** out) {
    *out = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<double*>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

hipError_t launch_residual_noalloc(int stencil, int nx, int ny, bool frame, const Tiles& T, double scale,
                                   const double* f, const double* u, double* out, hipStream_t stream) {
    if (T.count() > kNoallocMaxTiles || T.count() < 1) return hipErrorInvalidValue;
    double* s = nullptr;
    const hipError_t e = noalloc_scratch(&s);
    if (e != hipSuccess) return e;
    double* pr = s;
    double* pd = s + kNoallocMaxTiles;
    const dim3 grid(T.count()), block(T.width);
#define CJ_NA_CASE(ST)                                                                                         \
    if (frame)                                                                                                 \
        hipLaunchKernelGGL((residual_noalloc_kernel<ST, true>), grid, block, 0, stream, f, u, scale, nx, ny,  \
                           T.tiles_x, T.rows, pr, pd);                                                         \
    else                                                                                                       \
        hipLaunchKernelGGL((residual_noalloc_kernel<ST, false>), grid, block, 0, stream, f, u, scale, nx, ny, \
                           T.tiles_x, T.rows, pr, pd);
    switch (stencil) {
    case 5: CJ_NA_CASE(5) break;
    case 9: CJ_NA_CASE(9) break;
    case 17: CJ_NA_CASE(17) break;
    default: return hipErrorInvalidValue;
    }
#undef CJ_NA_CASE
    hipLaunchKernelGGL(ratio_kernel, dim3(1), dim3(256), 0, stream, pr, pd, T.count(), out);
    return hipGetLastError();
}

}  // namespace cj
