// Internal declarations shared by the host runtime and the kernel launchers of
// libcj.so.  Not part of the public ABI (see include/cj.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>
#include <vector>

namespace cj {

// ---------------------------------------------------------------- plan (host)

struct Schedule {
    int stencil = 9;
    int nx = 0, ny = 0;
    double tol = 0.0, h = 0.0;
    double kmin = 0.0, kmax = 0.0, beta = 0.0, rho = 0.0;
    int M = 0, cycles_pred = 0;
    std::vector<double> w;   // M weights in applied order
};

// Fills s from (stencil, nx, ny, tol, h, M_request); returns false with a message on bad input.
bool make_schedule(int stencil, int nx, int ny, double tol, double h, int M_request,
                   Schedule* s, std::string* err);

// Plain Jacobi: all weights 1, M = the interval between residual checks
// (0: automatic), cycles_pred = the predicted number of checks.
bool make_jacobi_schedule(int stencil, int nx, int ny, double tol, double h, int M_request,
                          Schedule* s, std::string* err);

// ---------------------------------------------------------------- device layout

// Padded, pitched storage of a grid function: node (x, y) for
// -1 <= x <= nx + 2, -1 <= y <= ny + 2 lives at (y + 1) * pitch + (x + xoff),
// xoff = 128 / element_bytes - 1, which puts the first interior column x = 1
// on a 128-byte boundary.  The ring x in {0, nx+1}, y in {0, ny+1} holds the
// Dirichlet data; the outer ring x in {-1, nx+2}, y in {-1, ny+2} is read by
// the 17-point stencil only.  frame = 0 (homogeneous data): the ring holds
// zeros and the outer ring the odd reflection of the interior.  frame = G > 0:
// the caller's u carries the boundary data in a frame of width G (1: 5/9-point,
// 2: 17-point) and both rings hold data that no sweep changes.
__host__ __device__ constexpr int xoff_of(int elem_bytes) { return 128 / elem_bytes - 1; }

struct Layout {
    int nx = 0, ny = 0;
    int elem_bytes = 8;
    int pitch = 0;          // elements per stored row
    size_t elems = 0;       // elements per padded array
    int frame = 0;          // width of the caller's boundary frame (0: homogeneous data)
};

Layout make_layout(int nx, int ny, int elem_bytes, int frame = 0);

// Launch geometry of the tile kernels (sweeps, residual, stage-in).
struct Tiles {
    int width = 256;        // columns per workgroup = threads per workgroup (multiple of 64)
    int rows = 64;          // rows per workgroup
    int tiles_x = 0, tiles_y = 0;
    int count() const { return tiles_x * tiles_y; }
};

Tiles make_tiles(int nx, int ny, int rows_request);

// Lanes of the temporally blocked kernel's workgroup, one per column of its
// strip.  FP64 radius-1 stencils at K >= 10 (the large-grid default) take 512
// lanes, one workgroup per CU: half the strip overlap of 256 lanes (2KR
// columns of 512), measured 5-6% faster per sweep at 8192^2; the 17-point
// kernel lost 9% that way, and smaller K serve grids where wider strips would
// leave CUs idle.
__host__ __device__ constexpr int strip_lanes(int R, int K, int elem_bytes) {
    return (elem_bytes == 8 && R == 1 && K >= 10) ? 512 : 256;
}

// Geometry of the temporally blocked kernel: strips of strip_lanes - 2KR
// output columns (tiles_x strips) by tiles of `rows` output rows.
Tiles make_tiles_k(int nx, int ny, int K, int R, int rows_request, int elem_bytes);

// ---------------------------------------------------------------- batches
// Device descriptor of one problem of a batch (FP32 inner sweeps inside FP64
// refinement).  u and g are FP64 padded arrays (layout pitch), r32, d1, d2
// FP32 padded arrays (pitch32).  Tile geometry: single-sweep tiles of 256
// columns x rows (tiles_x per row band) for the residual and correction;
// blocked strips (strips_x) x rows_k for the sweeps.
struct BatchProblem {
    double* u;
    const double* g;
    float* r32;
    float* d1;
    float* d2;
    const float* w32;      // weights of the current inner cycle
    int nx, ny, pitch, pitch32;
    int tiles_x, rows;     // single-sweep geometry
    int strips_x, rows_k;  // blocked geometry
    int cycle_start;       // super-step at which the current inner cycle began
    int dcur;              // buffer (0: d1, 1: d2) holding the finished correction
    int dnext;             // buffer the next inner cycle starts from (zeroed by the residual)
    int pad_;
};

// One work item: a tile of a problem.
struct BatchItem {
    int prob;
    int tile;
};

// ---------------------------------------------------------------- launchers
// Every launcher enqueues on `stream` and returns the launch status.

// Interior of A <- u (user layout; with L.frame > 0 the interior of u's frame
// layout), of B <- u (L.frame > 0: zero), of G <- scale * f (f == nullptr:
// zero); per-tile partial sums of G^2 into part[0 .. tiles.count()).
hipError_t launch_stage_in(const Layout& L, const Tiles& T, const double* f, const double* u,
                           double scale, double* A, double* B, double* G, double* part,
                           hipStream_t stream);

// Ring of A, B (L.frame = 0: zeros and the reflection of u; else the frame
// values of u) and of G (zeros).
hipError_t launch_ring(const Layout& L, const double* u, double* A, double* B, double* G,
                       hipStream_t stream);

// u (user layout; L.frame > 0: the interior of the frame layout) <- interior of A.
hipError_t launch_stage_out(const Layout& L, const double* A, double* u, hipStream_t stream);

// One weighted sweep uout <- uin + w[widx] * r(uin), r = g - D^{-1} A uin in
// normalised form.  If part != nullptr, per-tile partial sums of r^2 of uin go
// to part[0 .. tiles.count()).
hipError_t launch_sweep(int stencil, const Layout& L, const Tiles& T, const double* uin,
                        double* uout, const double* g, const double* w, int widx,
                        double* part, hipStream_t stream);
// The same sweep in FP32 (part must be nullptr).
hipError_t launch_sweep(int stencil, const Layout& L, const Tiles& T, const float* uin,
                        float* uout, const float* g, const float* w, int widx,
                        double* part, hipStream_t stream);

// K sweeps in one launch (weights w[widx .. widx+K-1]), bit-identical to K
// launch_sweep calls.  If part != nullptr, per-tile partial sums of r^2 of uin
// go to part[0 .. tiles.count()).  T must come from make_tiles_k.
bool sweepk_supported(int stencil, int K, int elem_bytes);
hipError_t launch_sweepk(int stencil, int K, const Layout& L, const Tiles& T, const double* uin, double* uout,
                         const double* g, const double* w, int widx, double* part, hipStream_t stream);
// Workgroups of the blocked kernel (stencil, K, element size, 17-point
// reflection) resident per CU at once, from the HIP occupancy calculator.
hipError_t sweepk_blocks_per_cu(int stencil, int K, int elem_bytes, bool refl, int* blocks);
// The same in FP32 (part must be nullptr).
hipError_t launch_sweepk(int stencil, int K, const Layout& L, const Tiles& T, const float* uin, float* uout,
                         const float* g, const float* w, int widx, double* part, hipStream_t stream);

// Iterative refinement: r32 <- (float)(g - D^{-1}A u) and d32 <- 0 (interior
// and reflected ring), per-tile partials of r^2 (FP64) into part.  L32 is the
// FP32 layout of the same grid; T the single-sweep tile geometry.  With lo
// non-null the iterate is the double-double u + lo (lo in the layout L).
hipError_t launch_ir_residual(int stencil, const Layout& L, const Layout& L32, const Tiles& T, const double* u,
                              const double* lo, const double* g, float* r32, float* d32, double* part,
                              hipStream_t stream);
// The same with an FP64 inner solve: r and d in the FP64 layout L.
hipError_t launch_ir_residual(int stencil, const Layout& L, const Tiles& T, const double* u, const double* lo,
                              const double* g, double* r, double* d, double* part, hipStream_t stream);
// u += (double)d over the padded frame; with lo non-null, (u, lo) += d as a
// double-double.
hipError_t launch_ir_correct(const Layout& L, const Layout& L32, double* u, double* lo, const float* d,
                             hipStream_t stream);
// u += d (FP64, layout L); with lo non-null, (u, lo) += d as a double-double.
hipError_t launch_ir_correct(const Layout& L, double* u, double* lo, const double* d, hipStream_t stream);
// Padded-frame conversions between the FP64 and FP32 layouts.
hipError_t launch_to_f32(const Layout& L, const Layout& L32, const double* src, float* dst, hipStream_t stream);
hipError_t launch_from_f32(const Layout& L, const Layout& L32, const float* src, double* dst, hipStream_t stream);

// Per-tile partial sums of r^2 of u (read-only).
hipError_t launch_residual(int stencil, const Layout& L, const Tiles& T, const double* u,
                           const double* g, double* part, hipStream_t stream);

// Batched launches over a work list of n_items (problem, tile) items.
hipError_t launch_batch_sweepk(int stencil, int K, const BatchProblem* probs, const BatchItem* work, int n_items,
                               int step, hipStream_t stream);
hipError_t launch_batch_correct(int stencil, const BatchProblem* probs, const BatchItem* work, int n_items,
                                hipStream_t stream);
hipError_t launch_batch_residual(int stencil, const BatchProblem* probs, const BatchItem* work, int n_items,
                                 double* part, hipStream_t stream);
// out[s] <- sum of part[seg[s] .. seg[s+1]) for s < n_seg, fixed order.
hipError_t launch_segmented_reduce(const double* part, const int* seg, int n_seg, double* out, hipStream_t stream);

// Whole FP64 solve of a small 5- or 9-point grid in one workgroup with the
// padded grid in LDS: A (padded iterate, staged, rings included) holds the
// answer afterwards; out[0..3] <- status (0 ok, 1 stagnated, -4 max cycles,
// -5 not finite), cycles, last relative residual, floor estimate.
// lds_solve_fits: whether the grid fits (columns <= 1024, 16 rows per lane,
// padded grid <= 160 KiB), with its lane mapping.
bool lds_solve_fits(int stencil, int nx, int ny, int* wx, int* band, size_t* lds_bytes);
hipError_t launch_lds_solve(int stencil, const Layout& L, double* A, const double* G, const double* w, int M,
                            double gnorm, double tol, int cycles_pred, int max_cycles, double* out,
                            hipStream_t stream);

// out[0] <- sum of part[0 .. n) in a fixed order (one workgroup).
hipError_t launch_reduce(const double* part, int n, double* out, hipStream_t stream);

// Allocation-free relative residual (cj_residual_noalloc): out[0] (device)
// <- ||f - A u|| / ||f|| (frame: over the lifted right-hand side) read from
// the caller's f and u, with the per-tile partial sums in the library's
// static per-device scratch array; T the plan's single-sweep tiles, at most
// kNoallocMaxTiles of them (else hipErrorInvalidValue).
constexpr int kNoallocMaxTiles = 65536;
hipError_t launch_residual_noalloc(int stencil, int nx, int ny, bool frame, const Tiles& T, double scale,
                                   const double* f, const double* u, double* out, hipStream_t stream);

// au (user layout) <- dscale * (u - sum c_hat u_nbr) = A u, with dscale = D.
hipError_t launch_apply(int stencil, const Layout& L, const double* A, double dscale,
                        double* au, hipStream_t stream);

}  // namespace cj
