// HIP kernels of libcj.so for gfx950 (MI355X): stage-in/out, the weighted
// Chebyshev-Jacobi sweep, the residual norm and the stencil apply.
//
// All kernels work on the padded, pitched layout described in cj_internal.h.
// The sweep is HBM-bound (24 bytes and 8-24 flops per grid-point update), so
// the kernels are organised around memory traffic: one wave64 lane per grid
// column, marching up the rows of its tile and keeping the (2R+1) rows of the
// stencil window in registers, so that every value of u is fetched from HBM
// once per sweep and the row re-reads of the window hit registers.  Row loads
// of a wave are 64 consecutive doubles (512 B), aligned on the interior.
//
// Arithmetic is written with explicit fma() and compiled with
// -ffp-contract=off, so that every kernel that evaluates the update performs
// exactly the same operations in the same order and produces the same bits.
#include <hip/hip_runtime.h>

#include "cj_internal.h"

namespace cj {
namespace {

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

template <int ST> struct Stencil;
template <> struct Stencil<5>  { static constexpr int R = 1; };
template <> struct Stencil<9>  { static constexpr int R = 1; };
template <> struct Stencil<17> { static constexpr int R = 2; };

// v[dy + R][dx + R] holds u(x + dx, y + dy).  Returns t.
template <int ST>
__device__ __forceinline__ double neighbour_sum(const double (&v)[2 * Stencil<ST>::R + 1][2 * Stencil<ST>::R + 1]);

template <>
__device__ __forceinline__ double neighbour_sum<5>(const double (&v)[3][3]) {
    const double axis = (v[1][0] + v[1][2]) + (v[0][1] + v[2][1]);
    return 0.25 * axis;
}

template <>
__device__ __forceinline__ double neighbour_sum<9>(const double (&v)[3][3]) {
    const double axis = (v[1][0] + v[1][2]) + (v[0][1] + v[2][1]);
    const double diag = (v[0][0] + v[2][2]) + (v[2][0] + v[0][2]);
    return fma(0.2, axis, 0.05 * diag);
}

template <>
__device__ __forceinline__ double neighbour_sum<17>(const double (&v)[5][5]) {
    const double axis1 = (v[2][1] + v[2][3]) + (v[1][2] + v[3][2]);
    const double axis2 = (v[2][0] + v[2][4]) + (v[0][2] + v[4][2]);
    const double diag1 = (v[1][1] + v[3][3]) + (v[3][1] + v[1][3]);
    const double diag2 = (v[0][0] + v[4][4]) + (v[4][0] + v[0][4]);
    constexpr double a1 = 64.0 / 300.0, a2 = -4.0 / 300.0;
    constexpr double d1 = 16.0 / 300.0, d2 = -1.0 / 300.0;
    return fma(a1, axis1, fma(a2, axis2, fma(d1, diag1, d2 * diag2)));
}

__device__ __forceinline__ size_t at(int pitch, int x, int y) {
    return (size_t)(y + 1) * (size_t)pitch + (size_t)(x + kXOff);
}

// Hardware dispatches workgroup b to XCD b % 8.  Give every XCD a contiguous
// range of tiles (row-major over the grid), so that vertically adjacent tiles,
// which share halo rows, usually run on the same XCD and share its L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int xcd = b & 7, slot = b >> 3;
    return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// Sum over the workgroup (blockDim.x = 64 * waves, waves <= 4), fixed order.
// The result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double ws[4];
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

// ------------------------------------------------------------ sweep / residual
// One lane per column x of a tile of width blockDim.x and `rows` rows.  The
// lane keeps the window rows y-R .. y+R in registers and loads one new row
// (2R+1 columns) per output row.  WRITE: store the update; NORM: accumulate
// r^2 of the input iterate.

template <int ST, bool WRITE, bool NORM>
__global__ __launch_bounds__(256) void sweep_kernel(
    const double* __restrict__ uin, double* __restrict__ uout, const double* __restrict__ g,
    const double* __restrict__ w, int widx, int nx, int ny, int pitch, int tiles_x, int rows,
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
    const double omega = WRITE ? w[widx] : 0.0;

    double v[W][W];
#pragma unroll
    for (int r = 1; r < W; ++r) {
        const double* p = uin + at(pitch, xl - R, y0 - R + r - 1);
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
        const double* p = uin + at(pitch, xl - R, y + R);
#pragma unroll
        for (int c = 0; c < W; ++c) v[W - 1][c] = p[c];
        const double gv = g[at(pitch, xl, y)];
        const double uc = v[R][R];
        const double res = (gv + neighbour_sum<ST>(v)) - uc;
        if (NORM) acc = fma(res, res, acc);
        if (WRITE && active) {
            const double un = fma(omega, res, uc);
            uout[at(pitch, x, y)] = un;
            if (ST == 17) {
                // keep the outer ring the odd reflection of the new iterate
                if (x == 1) uout[at(pitch, -1, y)] = -un;
                if (x == nx) uout[at(pitch, nx + 2, y)] = -un;
                if (y == 1) {
                    uout[at(pitch, x, -1)] = -un;
                    if (x == 1) uout[at(pitch, -1, -1)] = un;
                    if (x == nx) uout[at(pitch, nx + 2, -1)] = un;
                }
                if (y == ny) {
                    uout[at(pitch, x, ny + 2)] = -un;
                    if (x == 1) uout[at(pitch, -1, ny + 2)] = un;
                    if (x == nx) uout[at(pitch, nx + 2, ny + 2)] = un;
                }
            }
        }
    }
    if (NORM) {
        if (!active) acc = 0.0;
        const double tot = block_sum(acc);
        if (threadIdx.x == 0) part[tile] = tot;
    }
}

// ------------------------------------------------------------ stage in / out

__global__ __launch_bounds__(256) void stage_in_kernel(
    const double* __restrict__ f, const double* __restrict__ u, double scale, double* __restrict__ A,
    double* __restrict__ B, double* __restrict__ G, int nx, int ny, int pitch, int tiles_x, int rows,
    double* __restrict__ part) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int x = tx * (int)blockDim.x + (int)threadIdx.x + 1;
    const int y0 = ty * rows + 1;
    const int y1 = min(y0 + rows, ny + 1);
    double acc = 0.0;
    if (x <= nx) {
        for (int y = y0; y < y1; ++y) {
            const size_t src = (size_t)(y - 1) * (size_t)nx + (size_t)(x - 1);
            const size_t dst = at(pitch, x, y);
            const double uv = u[src];
            const double gv = scale * f[src];
            A[dst] = uv;
            B[dst] = uv;
            G[dst] = gv;
            acc = fma(gv, gv, acc);
        }
    }
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) part[tile] = tot;
}

// Ring values: index k enumerates the 2-wide frame around the interior.
__global__ __launch_bounds__(256) void ring_kernel(const double* __restrict__ u, double* __restrict__ A,
                                                   double* __restrict__ B, double* __restrict__ G,
                                                   int nx, int ny, int pitch) {
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
    // odd reflection about the Dirichlet nodes 0 and n + 1
    double sgn = 1.0;
    int xs = x, ys = y;
    if (xs < 0) { xs = -xs; sgn = -sgn; }
    if (xs > nx + 1) { xs = 2 * (nx + 1) - xs; sgn = -sgn; }
    if (ys < 0) { ys = -ys; sgn = -sgn; }
    if (ys > ny + 1) { ys = 2 * (ny + 1) - ys; sgn = -sgn; }
    double val = 0.0;
    if (xs >= 1 && xs <= nx && ys >= 1 && ys <= ny)
        val = sgn * u[(size_t)(ys - 1) * (size_t)nx + (size_t)(xs - 1)];
    const size_t d = at(pitch, x, y);
    A[d] = val;
    B[d] = val;
    G[d] = 0.0;
}

// Row-wise kernels use a 1D grid of bx blocks per row: block b covers row
// b / bx + 1, columns (b % bx) * 256 + 1 ...
__global__ __launch_bounds__(256) void stage_out_kernel(const double* __restrict__ A, double* __restrict__ u,
                                                        int nx, int ny, int pitch, int bx) {
    const int x = (int)(blockIdx.x % bx) * 256 + (int)threadIdx.x + 1;
    const int y = (int)(blockIdx.x / bx) + 1;
    if (x > nx || y > ny) return;
    u[(size_t)(y - 1) * (size_t)nx + (size_t)(x - 1)] = A[at(pitch, x, y)];
}

// ------------------------------------------------------------ reduction / apply

__global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ part, int n,
                                                     double* __restrict__ out) {
    double acc = 0.0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) acc += part[k];
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) out[0] = tot;
}

template <int ST>
__global__ __launch_bounds__(256) void apply_kernel(const double* __restrict__ A, double dscale,
                                                    double* __restrict__ au, int nx, int ny, int pitch,
                                                    int bx) {
    constexpr int R = Stencil<ST>::R;
    constexpr int W = 2 * R + 1;
    const int x = (int)(blockIdx.x % bx) * 256 + (int)threadIdx.x + 1;
    const int y = (int)(blockIdx.x / bx) + 1;
    if (x > nx || y > ny) return;
    double v[W][W];
#pragma unroll
    for (int r = 0; r < W; ++r)
#pragma unroll
        for (int c = 0; c < W; ++c) v[r][c] = A[at(pitch, x - R + c, y - R + r)];
    au[(size_t)(y - 1) * (size_t)nx + (size_t)(x - 1)] = dscale * (v[R][R] - neighbour_sum<ST>(v));
}

template <int ST, bool WRITE, bool NORM>
hipError_t launch_tile(const Layout& L, const Tiles& T, const double* uin, double* uout, const double* g,
                       const double* w, int widx, double* part, hipStream_t s) {
    hipLaunchKernelGGL((sweep_kernel<ST, WRITE, NORM>), dim3(T.count()), dim3(T.width), 0, s, uin, uout, g, w,
                       widx, L.nx, L.ny, L.pitch, T.tiles_x, T.rows, part);
    return hipGetLastError();
}

}  // namespace

// ------------------------------------------------------------ launchers

hipError_t launch_stage_in(const Layout& L, const Tiles& T, const double* f, const double* u, double scale,
                           double* A, double* B, double* G, double* part, hipStream_t stream) {
    hipLaunchKernelGGL(stage_in_kernel, dim3(T.count()), dim3(T.width), 0, stream, f, u, scale, A, B, G, L.nx,
                       L.ny, L.pitch, T.tiles_x, T.rows, part);
    return hipGetLastError();
}

hipError_t launch_ring(const Layout& L, const double* u, double* A, double* B, double* G, hipStream_t stream) {
    const int n = 4 * (L.nx + 4) + 4 * L.ny;
    hipLaunchKernelGGL(ring_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, u, A, B, G, L.nx, L.ny,
                       L.pitch);
    return hipGetLastError();
}

hipError_t launch_stage_out(const Layout& L, const double* A, double* u, hipStream_t stream) {
    const int bx = (L.nx + 255) / 256;
    hipLaunchKernelGGL(stage_out_kernel, dim3(bx * L.ny), dim3(256), 0, stream, A, u, L.nx, L.ny, L.pitch, bx);
    return hipGetLastError();
}

hipError_t launch_sweep(int stencil, const Layout& L, const Tiles& T, const double* uin, double* uout,
                        const double* g, const double* w, int widx, double* part, hipStream_t stream) {
    const bool norm = part != nullptr;
    switch (stencil) {
    case 5:
        return norm ? launch_tile<5, true, true>(L, T, uin, uout, g, w, widx, part, stream)
                    : launch_tile<5, true, false>(L, T, uin, uout, g, w, widx, part, stream);
    case 9:
        return norm ? launch_tile<9, true, true>(L, T, uin, uout, g, w, widx, part, stream)
                    : launch_tile<9, true, false>(L, T, uin, uout, g, w, widx, part, stream);
    case 17:
        return norm ? launch_tile<17, true, true>(L, T, uin, uout, g, w, widx, part, stream)
                    : launch_tile<17, true, false>(L, T, uin, uout, g, w, widx, part, stream);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_residual(int stencil, const Layout& L, const Tiles& T, const double* u, const double* g,
                           double* part, hipStream_t stream) {
    switch (stencil) {
    case 5: return launch_tile<5, false, true>(L, T, u, nullptr, g, nullptr, 0, part, stream);
    case 9: return launch_tile<9, false, true>(L, T, u, nullptr, g, nullptr, 0, part, stream);
    case 17: return launch_tile<17, false, true>(L, T, u, nullptr, g, nullptr, 0, part, stream);
    default: return hipErrorInvalidValue;
    }
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

Layout make_layout(int nx, int ny) {
    Layout L;
    L.nx = nx;
    L.ny = ny;
    int pitch = nx + kXOff + 3;             // columns up to x = nx + 2
    pitch = (pitch + 15) & ~15;             // 128-byte rows
    if ((pitch & 511) == 0) pitch += 16;    // avoid 4 KB-multiple row strides
    L.pitch = pitch;
    L.elems = (size_t)(ny + 4) * (size_t)pitch;
    return L;
}

Tiles make_tiles(int nx, int ny, int rows_request) {
    Tiles T;
    T.width = nx >= 256 ? 256 : ((nx + 63) / 64) * 64;
    T.tiles_x = (nx + T.width - 1) / T.width;
    int rows = rows_request > 0 ? rows_request : 64;
    if (rows_request <= 0)
        while (rows > 4 && (long long)T.tiles_x * ((ny + rows - 1) / rows) < 2048) rows /= 2;
    if (rows > ny) rows = ny;
    T.rows = rows;
    T.tiles_y = (ny + rows - 1) / rows;
    return T;
}

}  // namespace cj
