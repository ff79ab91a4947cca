// Host runtime and C ABI of libcj.so (declared in include/cj.h).
//
// A plan holds the schedule (host, FP64) and, after the first device call, a
// device workspace: two padded iterates A and B (ping-pong), the padded
// scaled right-hand side G = D^{-1} f, the weights, the per-tile reduction
// partials and a pinned 8-byte host slot for the cycle-end residual.  Plans
// with FP32 sweeps also hold the FP32 residual, two FP32 corrections and the
// FP32 inner weights.
//
// FP64 solve loop: the residual of the iterate reached at a cycle end is
// produced by the first launch of the next cycle (the sweep forms r anyway),
// so the norm costs no extra pass over HBM.  The host waits for that 8-byte
// value once per cycle and decides; if it stops, the launch's input (still
// intact in the other buffer) is the answer.
//
// Refinement loop (FP32 sweeps): r = g - D^{-1}A u is formed in FP64 and
// rounded to FP32; one inner cycle of FP32 weighted sweeps approximately
// solves D^{-1}A d = r from d = 0; u += d in FP64; repeat until the FP64
// residual meets tol.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <iterator>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <new>
#include <string>
#include <vector>

#include "../../include/cj.h"
#include "cj_internal.h"

namespace {

thread_local std::string g_last_error;

cj_status fail(cj_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

#define CJ_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(CJ_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

// Stencil facts used by the runtime: |c_centre| / s, where A = -(1/(s h^2)) sum c u.
double centre_over_s(int stencil) {
    switch (stencil) {
    case 5: return 4.0;            // (1/h^2)[..., -4]
    case 9: return 20.0 / 6.0;     // (1/(6h^2))[..., -20]
    case 17: return 300.0 / 72.0;  // (1/(72h^2))[..., -300]
    default: return NAN;
    }
}

int radius(int stencil) { return stencil == 17 ? 2 : 1; }

// Refinement plans switch their inner cycles from FP32 to FP64 above this
// value of eps32 * kappa_max / kappa_min (CJ_INNER_AUTO).
constexpr double kInnerF64Above = 4.0;

// The single-workgroup solve is chosen automatically where it measured faster
// than the launched cycles: bands of at most 4 rows per lane; of at most 8 for
// the 5-point stencil, and for the 9-point one on grids of at most 4096 points
// (its g stays in registers up to 8 rows).
bool lds_auto(int stencil, int band, long long points) {
    if (band <= 4) return true;
    return band <= 8 && (stencil == 5 || points <= 4096);
}

}  // namespace

struct cj_plan_s {
    cj::Schedule s;       // the FP64 schedule (and the kappa bounds)
    cj::Schedule sin;     // the inner schedule of the FP32 sweeps (refinement plans)
    // FP32 weights of the inner cycles of length sin.M, sin.M / 2, ..., 1 (the
    // refinement halves its inner cycle when an outer step contracts poorly),
    // concatenated; the cycle of length m starts at w32_offset(m).
    std::vector<float> w32_all;
    size_t w32_offset(int m) const { return 2 * (size_t)sin.M - 2 * (size_t)m; }
    cj_options opt;
    int precision = CJ_PRECISION_F64;
    int max_cycles = 0;
    cj::Layout L;         // FP64 arrays
    cj::Layout L32;       // FP32 arrays (refinement plans)
    cj::Tiles T;          // single-sweep, stage-in and residual kernels
    cj::Tiles TK;         // temporally blocked kernel, FP64 (K > 1)
    cj::Tiles TK32;       // temporally blocked kernel, FP32 (K32 > 1)
    int K = 1;            // FP64 sweeps per launch
    int K32 = 1;          // FP32 sweeps per launch
    double D = 0.0;       // diagonal of A: |c_centre| / (s h^2)
    // device state
    int device = -1;
    double* A = nullptr;
    double* B = nullptr;
    double* G = nullptr;
    double* W = nullptr;
    double* part = nullptr;
    double* scalar = nullptr;
    double* host_slot = nullptr;   // pinned
    float* R32 = nullptr;
    float* D1 = nullptr;
    float* D2 = nullptr;
    float* W32 = nullptr;
    // double-double solves of FP64 plans (allocated by the first one): the
    // FP64 inner right-hand side and the two iterates of the correction
    double* R64 = nullptr;
    double* E1 = nullptr;
    double* E2 = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};   // bracket the plain sweeps of a cycle
    // The plain launches of an FP64 cycle (all but the first, norm-fused one),
    // captured once as a graph on a private stream and replayed every cycle.
    bool use_graph = false;
    // Small 5- and 9-point FP64 grids: the whole solve in one workgroup with
    // the grid in LDS (launch_lds_solve).
    bool use_lds = false;
    // Tile height of the blocked kernels: chosen on the device at the first
    // solve (tune_rows) unless the options fix it.
    bool tune_rows = false;
    bool rows_tuned = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    long long graph_launches = 0;
    // Refinement plans whose inner cycles run in FP64: chosen when
    // eps32 * kappa_max / kappa_min is large (cj_plan_ex), where FP32 cycles
    // contract too little per outer step.
    bool inner_f64 = false;
    bool mixed() const { return precision == CJ_PRECISION_F32_REFINE; }
    bool f32_inner() const { return mixed() && !inner_f64; }
    size_t workspace_bytes() const {
        size_t b = 3 * L.elems * sizeof(double) + (size_t)s.M * sizeof(double) +
                   ((size_t)n_partials() + 64) * sizeof(double);
        if (f32_inner()) b += 3 * L32.elems * sizeof(float) + w32_all.size() * sizeof(float);
        if (inner_f64) b += 3 * L.elems * sizeof(double);
        return b;
    }
    int n_partials() const {
        int n = T.count();
        if (TK.count() > n) n = TK.count();
        if (tune_rows && K > 1) {
            // room for the flattest tile the first solve may choose
            const bool small = (long long)s.nx * s.ny <= (1LL << 18);
            const int R = s.stencil == 17 ? 2 : 1;
            for (int eb : {4, 8}) {
                const int m = cj::make_tiles_k(s.nx, s.ny, K, R, small ? 1 : kTuneRows[0], eb).count();
                if (m > n) n = m;
            }
        }
        return n;
    }
    static constexpr int kTuneRows[10] = {16, 24, 32, 48, 64, 96, 128, 160, 192, 256};
};

namespace {

void release(cj_plan_s* p) {
    if (p->device >= 0) {
        int cur = -1;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(p->device);
        for (void* d : {(void*)p->A, (void*)p->B, (void*)p->G, (void*)p->W, (void*)p->part, (void*)p->scalar,
                        (void*)p->R32, (void*)p->D1, (void*)p->D2, (void*)p->W32, (void*)p->R64, (void*)p->E1,
                        (void*)p->E2})
            if (d) (void)hipFree(d);
        if (p->host_slot) (void)hipHostFree(p->host_slot);
        for (hipEvent_t& e : p->ev)
            if (e) (void)hipEventDestroy(e);
        if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
        if (cur >= 0) (void)hipSetDevice(cur);
    }
    p->A = p->B = p->G = p->W = p->part = p->scalar = p->host_slot = nullptr;
    p->R32 = p->D1 = p->D2 = p->W32 = nullptr;
    p->R64 = p->E1 = p->E2 = nullptr;
    p->ev[0] = p->ev[1] = nullptr;
    p->graph_exec = nullptr;
    p->graph = nullptr;
    p->cap_stream = nullptr;
    p->device = -1;
}

// Binds the plan to the current device on first use and allocates the workspace.
cj_status ensure_device(cj_plan_s* p, hipStream_t stream) {
    int dev = -1;
    CJ_HIP(hipGetDevice(&dev));
    if (p->device >= 0) {
        if (dev != p->device)
            return fail(CJ_ERR_DEVICE, "plan was first used on device " + std::to_string(p->device) +
                                           ", current device is " + std::to_string(dev));
        return CJ_OK;
    }
    p->device = dev;
    const size_t bytes = p->L.elems * sizeof(double);
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc((void**)&p->A, bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&p->B, bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&p->G, bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&p->W, (size_t)p->s.M * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&p->part, (size_t)p->n_partials() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&p->scalar, 64 * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->host_slot, 64 * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreate(&p->ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&p->ev[1]);
    if (p->f32_inner()) {
        const size_t b32 = p->L32.elems * sizeof(float);
        if (e == hipSuccess) e = hipMalloc((void**)&p->R32, b32);
        if (e == hipSuccess) e = hipMalloc((void**)&p->D1, b32);
        if (e == hipSuccess) e = hipMalloc((void**)&p->D2, b32);
        if (e == hipSuccess) e = hipMalloc((void**)&p->W32, p->w32_all.size() * sizeof(float));
    }
    if (e != hipSuccess) {
        release(p);
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? CJ_ERR_NOMEM : CJ_ERR_HIP,
                    std::string("workspace allocation: ") + hipGetErrorString(e));
    }
    CJ_HIP(hipMemcpyAsync(p->W, p->s.w.data(), (size_t)p->s.M * sizeof(double), hipMemcpyHostToDevice, stream));
    if (p->f32_inner()) {
        // the corrections' Dirichlet rings stay zero for the life of the plan
        CJ_HIP(hipMemsetAsync(p->D1, 0, p->L32.elems * sizeof(float), stream));
        CJ_HIP(hipMemsetAsync(p->D2, 0, p->L32.elems * sizeof(float), stream));
        CJ_HIP(hipMemsetAsync(p->R32, 0, p->L32.elems * sizeof(float), stream));
        CJ_HIP(hipMemcpyAsync(p->W32, p->w32_all.data(), p->w32_all.size() * sizeof(float), hipMemcpyHostToDevice,
                              stream));
    }
    return CJ_OK;
}

cj_status check_ptr(const void* ptr, const char* name) {
    if (ptr == nullptr) return fail(CJ_ERR_ARG, std::string(name) + " is NULL");
    if (reinterpret_cast<uintptr_t>(ptr) % 8 != 0) return fail(CJ_ERR_ARG, std::string(name) + " is not 8-byte aligned");
    return CJ_OK;
}

// Sum of the per-tile partials, copied to the host (waits on the stream).
cj_status read_sum(cj_plan_s* p, int n, hipStream_t stream, double* out) {
    CJ_HIP(cj::launch_reduce(p->part, n, p->scalar, stream));
    CJ_HIP(hipMemcpyAsync(p->host_slot, p->scalar, sizeof(double), hipMemcpyDeviceToHost, stream));
    CJ_HIP(hipStreamSynchronize(stream));
    *out = p->host_slot[0];
    return CJ_OK;
}

// Stage-in of f and u (f may be NULL: G = 0).  Returns the squared norm the
// relative residual is measured against: sum of G^2 for homogeneous data; with
// a boundary frame, the squared residual of the zero interior inside the frame
// (B holds it after stage-in), i.e. of the lifted right-hand side.
cj_status stage_in(cj_plan_s* p, const double* f, const double* u, hipStream_t stream, double* g2) {
    const double scale = p->s.h * p->s.h / centre_over_s(p->s.stencil);   // D^{-1}
    CJ_HIP(cj::launch_ring(p->L, u, p->A, p->B, p->G, stream));
    CJ_HIP(cj::launch_stage_in(p->L, p->T, f, u, scale, p->A, p->B, p->G, p->part, stream));
    if (p->L.frame > 0 && f) CJ_HIP(cj::launch_residual(p->s.stencil, p->L, p->T, p->B, p->G, p->part, stream));
    return read_sum(p, p->T.count(), stream, g2);
}

// Enqueues sweeps [first, first + n) of a cyclic schedule of length M with
// device weights w, on layout L with right-hand side g, starting from *cur,
// in launches of K sweeps; where a launch would run past the end of the cycle
// or of the range, the k < K sweeps left run as one blocked launch of depth k
// if there is one, else as single sweeps.  If norm_parts != nullptr (FP64 only) the
// first launch also produces the residual partials of its input and
// *norm_parts receives their count.  *launches counts the launches.
template <typename T>
cj_status enqueue_sweeps(cj_plan_s* p, int M, int K, const cj::Layout& L, const cj::Tiles& TK, const T* g,
                         const T* w, long long first, long long n, T** cur, T** nxt, hipStream_t stream,
                         int* norm_parts = nullptr, long long* launches = nullptr) {
    bool norm = norm_parts != nullptr;
    while (n > 0) {
        const int w0 = (int)(first % M);
        long long k = K;
        if (k > n) k = n;
        if (k > M - w0) k = M - w0;
        double* part = norm ? p->part : nullptr;
        if (k == K && K > 1) {
            CJ_HIP(cj::launch_sweepk(p->s.stencil, K, L, TK, *cur, *nxt, g, w, w0, part, stream));
            if (norm) *norm_parts = TK.count();
        } else if (k > 1 && !norm && cj::sweepk_supported(p->s.stencil, (int)k, L.elem_bytes)) {
            const cj::Tiles Tk =
                cj::make_tiles_k(L.nx, L.ny, (int)k, radius(p->s.stencil), p->opt.tile_rows, L.elem_bytes);
            CJ_HIP(cj::launch_sweepk(p->s.stencil, (int)k, L, Tk, *cur, *nxt, g, w, w0, nullptr, stream));
        } else {
            k = 1;
            CJ_HIP(cj::launch_sweep(p->s.stencil, L, p->T, *cur, *nxt, g, w, w0, part, stream));
            if (norm) *norm_parts = p->T.count();
        }
        norm = false;
        if (launches) ++*launches;
        std::swap(*cur, *nxt);
        first += k;
        n -= k;
    }
    return CJ_OK;
}

cj_status enqueue_f64(cj_plan_s* p, long long first, long long n, double** cur, double** nxt, hipStream_t stream,
                      int* norm_parts = nullptr, long long* launches = nullptr) {
    return enqueue_sweeps<double>(p, p->s.M, p->K, p->L, p->TK, p->G, p->W, first, n, cur, nxt, stream, norm_parts,
                                  launches);
}

// FP32 sweeps of the inner cycle of length m.
cj_status enqueue_f32(cj_plan_s* p, int m, long long first, long long n, float** cur, float** nxt,
                      hipStream_t stream, long long* launches = nullptr) {
    return enqueue_sweeps<float>(p, m, p->K32, p->L32, p->TK32, p->R32, p->W32 + p->w32_offset(m), first, n, cur,
                                 nxt, stream, nullptr, launches);
}

// Captures the plain launches of one FP64 cycle (sweeps k0 .. M-1, starting
// from buffer B) into p->graph_exec.  The cycle has M/K launches in all; with
// M/K even the captured part has an odd count and ends in A, where the next
// cycle starts, so the same graph serves every cycle.
cj_status capture_cycle(cj_plan_s* p, long long k0) {
    if (p->graph_exec) return CJ_OK;
    CJ_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    CJ_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    double* cur = p->B;
    double* nxt = p->A;
    long long launches = 0;
    cj_status st = enqueue_f64(p, k0, p->s.M - k0, &cur, &nxt, p->cap_stream, nullptr, &launches);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (st != CJ_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(CJ_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    p->graph = g;
    CJ_HIP(hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0));
    p->graph_launches = launches;
    if (cur != p->A) return fail(CJ_ERR_HIP, "captured cycle does not end in the start buffer");
    return CJ_OK;
}

// Tile-height tuner of the blocked kernels (FP64 plans: TK, refinement plans:
// TK32).  Candidates: 64 .. 256 rows, and the heights that make the tile count
// fill whole rounds of the workgroups the device holds at once (the launch
// then has no partly idle last round).  Each candidate runs one warm-up launch and one timed launch
// of K sweeps from the first iterate buffer into the second (the FP64 plan
// reads A, whose iterate stays intact, and writes B, which the solve
// overwrites before reading; refinement plans use the correction buffers,
// which the solve resets).  The fastest height is kept for the life of the
// plan.  Every tile geometry gives the same bits, so this changes speed only.
cj_status tune_tile_rows(cj_plan_s* p, hipStream_t stream) {
    if (!p->tune_rows || p->rows_tuned) return CJ_OK;
    p->rows_tuned = true;
    const bool mixed = p->f32_inner();
    const int K = mixed ? p->K32 : p->K;
    if (K <= 1) return CJ_OK;
    const int R = radius(p->s.stencil);
    const int eb = mixed ? (int)sizeof(float) : (int)sizeof(double);
    const int nx = p->s.nx, ny = p->s.ny;
    long long slots = 0;   // workgroups of the blocked kernel the device holds at once
    int cus = 0;
    {
        const cj::Layout& Lk = mixed ? p->L32 : p->L;
        int per_cu = 0;
        const bool refl = p->s.stencil == 17 && Lk.frame == 0;
        if (cj::sweepk_blocks_per_cu(p->s.stencil, K, Lk.elem_bytes, refl, &per_cu) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess)
            slots = (long long)per_cu * cus;
        (void)hipGetLastError();
    }
    if ((long long)nx * ny <= (1LL << 18)) {
        // small grids: a launch costs the latency of its row pipeline, rounds x
        // (rows + 2KR + K - 1) row steps, with the device far from full; a
        // workgroup that shares its CU steps slower, so a round is one
        // workgroup per CU.  Take the height that minimises that (no timing
        // launches).
        if (cus <= 0) return CJ_OK;
        const long long per_round = cus;
        const int strips = cj::make_tiles_k(nx, ny, K, R, 1, eb).tiles_x;
        long long best_cost = -1;
        int best_rows = 0;
        for (int rows = 1; rows <= 128 && rows <= ny; ++rows) {
            const long long tiles = (long long)strips * ((ny + rows - 1) / rows);
            const long long cost = ((tiles + per_round - 1) / per_round) * (rows + 2 * K * R + K - 1);
            if (best_cost < 0 || cost < best_cost) {
                best_cost = cost;
                best_rows = rows;
            }
        }
        (mixed ? p->TK32 : p->TK) = cj::make_tiles_k(nx, ny, K, R, best_rows, eb);
        return CJ_OK;
    }
    // candidates: a fixed ladder, plus the heights whose tile count just fills
    // r rounds of the workgroups the device holds at once (r = 1 .. 8)
    std::vector<int> cand(std::begin(cj_plan_s::kTuneRows), std::end(cj_plan_s::kTuneRows));
    {
        if (slots > 0) {
            const int strips = cj::make_tiles_k(nx, ny, K, R, cj_plan_s::kTuneRows[0], eb).tiles_x;
            for (int r = 1; r <= 8; ++r) {
                const long long ty = r * slots / strips;
                if (ty < 1) continue;
                const long long rows = (ny + ty - 1) / ty;
                if (rows >= cj_plan_s::kTuneRows[0] && rows <= 2048) cand.push_back((int)rows);
            }
        }
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    }
    cj::Tiles best = mixed ? p->TK32 : p->TK;
    float best_ms = -1.0f;
    for (int rows : cand) {
        if (rows > ny) break;
        const cj::Tiles Tc = cj::make_tiles_k(nx, ny, K, R, rows, eb);
        float ms = -1.0f;   // the faster of two launches
        for (int rep = 0; rep < 2; ++rep) {
            float t = 0.0f;
            CJ_HIP(hipEventRecord(p->ev[0], stream));
            if (mixed)
                CJ_HIP(cj::launch_sweepk(p->s.stencil, K, p->L32, Tc, p->D1, p->D2, p->R32, p->W32, 0, nullptr,
                                         stream));
            else
                CJ_HIP(cj::launch_sweepk(p->s.stencil, K, p->L, Tc, p->A, p->B, p->G, p->W, 0, nullptr, stream));
            CJ_HIP(hipEventRecord(p->ev[1], stream));
            CJ_HIP(hipEventSynchronize(p->ev[1]));
            CJ_HIP(hipEventElapsedTime(&t, p->ev[0], p->ev[1]));
            if (ms < 0.0f || t < ms) ms = t;
        }
        if (best_ms < 0.0f || ms < best_ms) {
            best_ms = ms;
            best = Tc;
        }
    }
    if (mixed)
        p->TK32 = best;
    else
        p->TK = best;
    return CJ_OK;
}

// The whole FP64 solve of a small grid in one workgroup (launch_lds_solve);
// the answer is in A.
cj_status solve_lds(cj_plan_s* p, double gnorm, hipStream_t stream, cj_result* r) {
    CJ_HIP(hipEventRecord(p->ev[0], stream));
    CJ_HIP(cj::launch_lds_solve(p->s.stencil, p->L, p->A, p->G, p->W, p->s.M, gnorm, p->s.tol, p->s.cycles_pred,
                                p->max_cycles, p->scalar, stream));
    CJ_HIP(hipEventRecord(p->ev[1], stream));
    CJ_HIP(hipMemcpyAsync(p->host_slot, p->scalar, 4 * sizeof(double), hipMemcpyDeviceToHost, stream));
    CJ_HIP(hipStreamSynchronize(stream));
    float ms = 0.0f;
    CJ_HIP(hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
    const int code = (int)p->host_slot[0];
    r->cycles = (int)p->host_slot[1];
    r->sweeps = (long long)r->cycles * p->s.M;
    r->rel_residual = p->host_slot[2];
    r->sweep_seconds = 1e-3 * (double)ms;
    r->sweep_launches = 1;
    switch (code) {
    case 0: return CJ_OK;
    case 1:
        r->floor_estimate = p->host_slot[3];
        g_last_error = "residual stagnated above tol (FP64 floor)";
        return CJ_STAGNATED;
    case -4: return fail(CJ_ERR_NOT_CONVERGED, "max_cycles reached");
    default: return fail(CJ_ERR_NONFINITE, "residual is not finite (u has a NaN or Inf)");
    }
}

// The FP64 CJM loop (see the file comment).  On return *out_buf is the buffer
// holding the answer.
cj_status solve_f64(cj_plan_s* p, double gnorm, hipStream_t stream, cj_result* r, double** out_buf) {
    if (p->use_lds) {
        *out_buf = p->A;
        return solve_lds(p, gnorm, stream, r);
    }
    cj_status st;
    double* cur = p->A;
    double* nxt = p->B;
    const long long M = p->s.M;
    double prev = 0.0;
    cj_status outcome = CJ_OK;
    int c = 0;
    bool timed = false;   // events ev[0], ev[1] bracket the previous cycle's plain launches
    long long timed_launches = 0;
    // the launch that also yields the norm is a single launch (K sweeps, or one
    // sweep when the cycle is shorter than K), so that its input stays intact
    const long long k0 = p->K <= M ? p->K : 1;
    for (;;) {
        int nparts = 0;
        if ((st = enqueue_f64(p, 0, k0, &cur, &nxt, stream, &nparts)) != CJ_OK) return st;
        double r2 = 0.0;
        if ((st = read_sum(p, nparts, stream, &r2)) != CJ_OK) return st;
        if (timed) {
            float ms = 0.0f;
            CJ_HIP(hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
            r->sweep_seconds += 1e-3 * (double)ms;
            r->sweep_launches += timed_launches;
            timed = false;
        }
        const double rr = std::sqrt(r2) / gnorm;
        r->rel_residual = rr;
        bool stop = true;
        if (!std::isfinite(rr)) {
            outcome = fail(CJ_ERR_NONFINITE, "residual is not finite (u has a NaN or Inf)");
        } else if (rr <= p->s.tol) {
            outcome = CJ_OK;
        } else if (c >= 1 && c >= p->s.cycles_pred && rr > 0.5 * prev) {
            outcome = CJ_STAGNATED;
            r->floor_estimate = rr < prev ? rr : prev;
            g_last_error = "residual stagnated above tol (FP64 floor)";
        } else if (c >= p->max_cycles) {
            outcome = fail(CJ_ERR_NOT_CONVERGED, "max_cycles reached");
        } else {
            stop = false;
        }
        if (stop) {
            std::swap(cur, nxt);   // the answer is the input of the launch just made
            break;
        }
        prev = rr;
        if (M > k0) {
            timed_launches = 0;
            const bool graph_ok = p->use_graph && k0 == p->K && cur == p->B;
            if (graph_ok && (st = capture_cycle(p, k0)) != CJ_OK) return st;
            CJ_HIP(hipEventRecord(p->ev[0], stream));
            if (graph_ok) {
                CJ_HIP(hipGraphLaunch(p->graph_exec, stream));
                timed_launches = p->graph_launches;
                std::swap(cur, nxt);   // the graph ends in A (see capture_cycle)
            } else {
                if ((st = enqueue_f64(p, k0, M - k0, &cur, &nxt, stream, nullptr, &timed_launches)) != CJ_OK)
                    return st;
            }
            CJ_HIP(hipEventRecord(p->ev[1], stream));
            timed = true;
        }
        ++c;
    }
    r->cycles = c;
    r->sweeps = (long long)c * M;
    *out_buf = cur;
    return outcome;
}

// The refinement loop (see the file comment).  The answer is always in A.
// The inner cycle starts at the plan's length and is halved (down to 16)
// after an outer step that contracts the residual by less than 1/2: FP32
// rounding, amplified by the growth of the partial products inside long
// cycles, can spoil a long inner cycle while a shorter one still contracts.
// Two consecutive outer steps that reduce the residual by less than 10% stop
// the solve as stagnated.  With lo non-null the iterate is the double-double
// A + lo (lo in A's layout, zero on entry).  An FP64 plan (double-double
// only) corrects with one FP64 cycle of its own schedule per outer step
// instead, on the buffers R64, E1 and E2.
cj_status solve_refine(cj_plan_s* p, double gnorm, hipStream_t stream, cj_result* r, double* lo) {
    const bool f64 = !p->f32_inner();
    cj_status st;
    int m = p->sin.M;
    double prev = 0.0;
    cj_status outcome = CJ_OK;
    int k = 0, fails = 0;
    long long sweeps = 0;
    for (;;) {
        if (f64)
            CJ_HIP(cj::launch_ir_residual(p->s.stencil, p->L, p->T, p->A, lo, p->G, p->R64, p->E1, p->part, stream));
        else
            CJ_HIP(cj::launch_ir_residual(p->s.stencil, p->L, p->L32, p->T, p->A, lo, p->G, p->R32, p->D1, p->part,
                                          stream));
        double r2 = 0.0;
        if ((st = read_sum(p, p->T.count(), stream, &r2)) != CJ_OK) return st;
        if (k > 0) {
            float ms = 0.0f;
            CJ_HIP(hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
            r->sweep_seconds += 1e-3 * (double)ms;
        }
        const double rr = std::sqrt(r2) / gnorm;
        r->rel_residual = rr;
        const double q = k >= 1 ? rr / prev : 0.0;   // contraction of the last outer step
        fails = (k >= 1 && q > 0.9) ? fails + 1 : 0;
        bool stop = true;
        if (!std::isfinite(rr)) {
            outcome = fail(CJ_ERR_NONFINITE, "residual is not finite (u has a NaN or Inf)");
        } else if (rr <= p->s.tol) {
            outcome = CJ_OK;
        } else if (fails >= 2) {
            // the FP64 floor, or the limit eps32 * cond(D^{-1}A) of the FP32 inner solve
            outcome = CJ_STAGNATED;
            r->floor_estimate = rr < prev ? rr : prev;
            g_last_error = "refinement stagnated above tol";
        } else if (k >= p->max_cycles) {
            outcome = fail(CJ_ERR_NOT_CONVERGED, "max_cycles (outer steps) reached");
        } else {
            stop = false;
        }
        if (stop) break;
        prev = rr;
        long long launches = 0;
        if (f64) {
            double* cur = p->E1;
            double* nxt = p->E2;
            CJ_HIP(hipEventRecord(p->ev[0], stream));
            if ((st = enqueue_sweeps<double>(p, p->s.M, p->K, p->L, p->TK, p->R64, p->W, 0, p->s.M, &cur, &nxt,
                                             stream, nullptr, &launches)) != CJ_OK)
                return st;
            CJ_HIP(hipEventRecord(p->ev[1], stream));
            sweeps += p->s.M;
            CJ_HIP(cj::launch_ir_correct(p->L, p->A, lo, cur, stream));
        } else {
            if (k >= 1 && q > 0.5 && m > 16) m /= 2;
            float* cur = p->D1;
            float* nxt = p->D2;
            CJ_HIP(hipEventRecord(p->ev[0], stream));
            if ((st = enqueue_f32(p, m, 0, m, &cur, &nxt, stream, &launches)) != CJ_OK) return st;
            CJ_HIP(hipEventRecord(p->ev[1], stream));
            sweeps += m;
            CJ_HIP(cj::launch_ir_correct(p->L, p->L32, p->A, lo, cur, stream));
        }
        r->sweep_launches += launches;
        ++k;
    }
    r->cycles = k;
    r->sweeps = sweeps;
    return outcome;
}

// cj_solve, and cj_solve_dd with u_lo non-null (refinement plans only).
cj_status solve_common(cj_plan_t p, const double* f, double* u, double* u_lo, void* stream_, cj_result* res) {
    const auto t0 = std::chrono::steady_clock::now();
    cj_result r{};
    auto finish = [&](cj_status s) {
        r.status = s;
        r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (res) *res = r;
        return s;
    };
    if (!p) return finish(fail(CJ_ERR_ARG, "plan is NULL"));
    cj_status st;
    if ((st = check_ptr(f, "f")) != CJ_OK || (st = check_ptr(u, "u")) != CJ_OK) return finish(st);
    const bool dd = u_lo != nullptr;
    const size_t u_bytes = (size_t)(p->s.nx + 2 * p->L.frame) * (size_t)(p->s.ny + 2 * p->L.frame) * sizeof(double);
    if (dd) {
        if (p->opt.method != CJ_METHOD_CHEBYSHEV)
            return finish(fail(CJ_ERR_ARG, "cj_solve_dd needs a Chebyshev-Jacobi plan"));
        if ((st = check_ptr(u_lo, "u_lo")) != CJ_OK) return finish(st);
        const char* lo_b = reinterpret_cast<const char*>(u_lo);
        const char* u_b = reinterpret_cast<const char*>(u);
        const char* f_b = reinterpret_cast<const char*>(f);
        const size_t f_bytes = (size_t)p->s.nx * (size_t)p->s.ny * sizeof(double);
        if ((lo_b < u_b + u_bytes && u_b < lo_b + u_bytes) || (lo_b < f_b + f_bytes && f_b < lo_b + u_bytes))
            return finish(fail(CJ_ERR_ARG, "u_lo overlaps u or f"));
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if ((st = ensure_device(p, stream)) != CJ_OK) return finish(st);
    // FP64 correction cycles (double-double solves of FP64 plans, refinement
    // plans with FP64 inner cycles) need the inner right-hand side and two
    // correction iterates
    if ((dd || p->mixed()) && !p->f32_inner() && !p->R64) {
        const size_t bytes = p->L.elems * sizeof(double);
        hipError_t e = hipMalloc((void**)&p->R64, bytes);
        if (e == hipSuccess) e = hipMalloc((void**)&p->E1, bytes);
        if (e == hipSuccess) e = hipMalloc((void**)&p->E2, bytes);
        // the corrections' Dirichlet rings stay zero for the life of the plan
        if (e == hipSuccess) e = hipMemsetAsync(p->R64, 0, bytes, stream);
        if (e == hipSuccess) e = hipMemsetAsync(p->E1, 0, bytes, stream);
        if (e == hipSuccess) e = hipMemsetAsync(p->E2, 0, bytes, stream);
        if (e != hipSuccess) {
            for (double** b : {&p->R64, &p->E1, &p->E2}) {
                if (*b) (void)hipFree(*b);
                *b = nullptr;
            }
            (void)hipGetLastError();
            return finish(fail(e == hipErrorOutOfMemory ? CJ_ERR_NOMEM : CJ_ERR_HIP,
                               std::string("double-double workspace: ") + hipGetErrorString(e)));
        }
    }

    double g2 = 0.0;
    if ((st = stage_in(p, f, u, stream, &g2)) != CJ_OK) return finish(st);
    if (!std::isfinite(g2)) return finish(fail(CJ_ERR_NONFINITE, "f has a NaN or Inf"));
    if (g2 == 0.0) {
        // zero (lifted) right-hand side: the solution is the zero interior,
        // which B holds with a frame
        hipError_t e = p->L.frame > 0
                           ? cj::launch_stage_out(p->L, p->B, u, stream)
                           : hipMemsetAsync(u, 0, (size_t)p->s.nx * (size_t)p->s.ny * sizeof(double), stream);
        if (e == hipSuccess && dd) e = hipMemsetAsync(u_lo, 0, u_bytes, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return finish(fail(CJ_ERR_HIP, hipGetErrorString(e)));
        return finish(CJ_OK);
    }
    const double gnorm = std::sqrt(g2);
    double* answer = p->A;
    cj_status outcome;
    if ((st = tune_tile_rows(p, stream)) != CJ_OK) return finish(st);
    // the refinement does not use the second iterate B: it holds the low
    // parts of a double-double iterate, zero over the whole padded frame
    if (dd) {
        const hipError_t e = hipMemsetAsync(p->B, 0, p->L.elems * sizeof(double), stream);
        if (e != hipSuccess) return finish(fail(CJ_ERR_HIP, hipGetErrorString(e)));
    }
    if (p->mixed() || dd)
        outcome = solve_refine(p, gnorm, stream, &r, dd ? p->B : nullptr);
    else
        outcome = solve_f64(p, gnorm, stream, &r, &answer);
    if (outcome == CJ_ERR_HIP) return finish(outcome);
    hipError_t e = cj::launch_stage_out(p->L, answer, u, stream);
    if (e == hipSuccess && dd) e = hipMemsetAsync(u_lo, 0, u_bytes, stream);
    if (e == hipSuccess && dd) e = cj::launch_stage_out(p->L, p->B, u_lo, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return finish(fail(CJ_ERR_HIP, hipGetErrorString(e)));
    return finish(outcome);
}

}  // namespace

extern "C" {

void cj_options_init(cj_options* opt) {
    if (opt) std::memset(opt, 0, sizeof(*opt));
}

cj_status cj_plan_ex(int nx, int ny, int stencil, int bc, double tol, const cj_options* opt, cj_plan_t* out) {
    if (out == nullptr) return fail(CJ_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (bc != CJ_BC_DIRICHLET0 && bc != CJ_BC_DIRICHLET_FRAME)
        return fail(CJ_ERR_ARG, "bc must be CJ_BC_DIRICHLET0 or CJ_BC_DIRICHLET_FRAME");
    cj_options o;
    cj_options_init(&o);
    if (opt) o = *opt;
    for (int r : o.reserved)
        if (r != 0) return fail(CJ_ERR_ARG, "reserved option fields must be zero");
    if (o.method != CJ_METHOD_CHEBYSHEV && o.method != CJ_METHOD_JACOBI)
        return fail(CJ_ERR_ARG, "method must be CJ_METHOD_CHEBYSHEV or CJ_METHOD_JACOBI");
    const bool jacobi = o.method == CJ_METHOD_JACOBI;
    if (jacobi && o.precision != CJ_PRECISION_F64) return fail(CJ_ERR_ARG, "CJ_METHOD_JACOBI runs in FP64 only");
    if (o.max_cycles < 0 || o.sweeps_per_launch < 0 || o.tile_rows < 0 || o.inner_M < 0)
        return fail(CJ_ERR_ARG, "negative option");
    if (o.precision != CJ_PRECISION_F64 && o.precision != CJ_PRECISION_F32_REFINE)
        return fail(CJ_ERR_ARG, "precision must be CJ_PRECISION_F64 or CJ_PRECISION_F32_REFINE");
    const bool mixed = o.precision == CJ_PRECISION_F32_REFINE;
    if (o.inner_precision != CJ_INNER_AUTO && o.inner_precision != CJ_INNER_F32 &&
        o.inner_precision != CJ_INNER_F64)
        return fail(CJ_ERR_ARG, "inner_precision must be CJ_INNER_AUTO, CJ_INNER_F32 or CJ_INNER_F64");
    if (!mixed && o.inner_precision != CJ_INNER_AUTO)
        return fail(CJ_ERR_ARG, "inner_precision applies to CJ_PRECISION_F32_REFINE plans only");
    // Inner cycles of a refinement plan: FP32 unless forced to FP64 or, when
    // automatic, eps32 * kappa_max / kappa_min exceeds kInnerF64Above (the
    // FP32 cycle then solves the correction equation to little better than
    // its own rounding: at 16384^2, 9-point, the product is 8.6 and FP32
    // outer steps contract by about 0.45 each, stagnating at 4.2e-10, where
    // FP64 cycles meet 1e-10 in the same time; at 8192^2, 2.2, FP32 cycles
    // still reach 1e-10 in 20% less time than FP64 ones).
    bool inner_f64 = false;
    if (mixed) {
        // the bounds do not depend on the tolerance or the cycle length
        cj::Schedule probe;
        std::string perr;
        if (!cj::make_schedule(stencil, nx, ny, 0.5, o.h, 1, &probe, &perr)) return fail(CJ_ERR_ARG, perr);
        const double eps32 = 1.1920928955078125e-07;   // 2^-23
        inner_f64 = o.inner_precision == CJ_INNER_F64 ||
                    (o.inner_precision == CJ_INNER_AUTO && eps32 * probe.kmax / probe.kmin > kInnerF64Above);
    }
    const int elem = (mixed && !inner_f64) ? 4 : 8;
    if (o.sweeps_per_launch > 1 && !cj::sweepk_supported(stencil, o.sweeps_per_launch, elem))
        return fail(CJ_ERR_ARG, "sweeps_per_launch not available for this stencil and precision "
                                "(FP64: 5/9-point 1, 2, 3, 4, 6, 8, 10, 17-point 1, 2, 3, 4; "
                                "FP32: 5/9-point 1, 2, 4, 8, 17-point 1, 2, 3, 4)");
    if (!mixed && o.inner_M != 0) return fail(CJ_ERR_ARG, "inner_M applies to CJ_PRECISION_F32_REFINE plans only");
    cj_plan_s* p = new (std::nothrow) cj_plan_s();
    if (!p) return fail(CJ_ERR_NOMEM, "host allocation");
    std::string err;
    const bool sched_ok = jacobi ? cj::make_jacobi_schedule(stencil, nx, ny, tol, o.h, o.M, &p->s, &err)
                                 : cj::make_schedule(stencil, nx, ny, tol, o.h, o.M, &p->s, &err);
    if (!sched_ok ||
        (mixed && !cj::make_schedule(stencil, nx, ny, tol, o.h, o.inner_M > 0 ? o.inner_M : o.M, &p->sin, &err))) {
        delete p;
        return fail(CJ_ERR_ARG, err);
    }
    if (inner_f64) {
        // FP64 inner cycles: the plan's FP64 schedule is the inner one (its
        // cycle length is inner_M when given)
        p->s = p->sin;
    } else if (mixed) {
        // inner weight table: cycles of length sin.M, sin.M / 2, ..., 1
        p->w32_all.assign(2 * (size_t)p->sin.M, 0.0f);
        for (int m = p->sin.M; m >= 1; m /= 2) {
            cj::Schedule sm;
            if (!cj::make_schedule(stencil, nx, ny, tol, o.h, m, &sm, &err)) {
                delete p;
                return fail(CJ_ERR_ARG, err);
            }
            for (int j = 0; j < m; ++j) p->w32_all[p->w32_offset(m) + j] = (float)sm.w[j];
        }
    }
    p->opt = o;
    p->precision = o.precision;
    p->inner_f64 = inner_f64;
    p->max_cycles = o.max_cycles > 0 ? o.max_cycles : (mixed ? 50 : p->s.cycles_pred + 4);
    const int R = radius(stencil);
    const int frame = bc == CJ_BC_DIRICHLET_FRAME ? R : 0;
    p->L = cj::make_layout(nx, ny, 8, frame);
    // default depths from measurements at 8192^2 on MI355X, us per sweep: FP64
    // 5- and 9-point K = 10 on grids above 2^22 points (9-point 60.4, K = 8: 62.6;
    // 5-point 56.5, K = 8: 58.7), K = 8 on smaller ones, where a cycle of whole
    // K-launches replays as one graph; 17-point K = 4 (132.3; K = 5 no longer
    // fits two waves per SIMD).  FP32: K = 8, 17-point K = 4.
    if (mixed && !inner_f64) {
        // the corrections have zero boundary data in the same frame geometry
        p->L32 = cj::make_layout(nx, ny, 4, frame);
        p->K = 1;
        p->K32 = o.sweeps_per_launch > 0 ? o.sweeps_per_launch : (stencil == 17 ? 4 : 8);
        p->T = cj::make_tiles(nx, ny, p->K32 == 1 ? o.tile_rows : 0);
        if (p->K32 > 1) p->TK32 = cj::make_tiles_k(nx, ny, p->K32, R, o.tile_rows, sizeof(float));
    } else {
        const bool large = (long long)nx * ny > (1LL << 22);
        p->K = o.sweeps_per_launch > 0 ? o.sweeps_per_launch : (stencil == 17 ? 4 : large ? 10 : 8);
        p->T = cj::make_tiles(nx, ny, p->K == 1 ? o.tile_rows : 0);
        if (p->K > 1) p->TK = cj::make_tiles_k(nx, ny, p->K, R, o.tile_rows, sizeof(double));
    }
    p->D = centre_over_s(stencil) / (p->s.h * p->s.h);
    // the tile height is chosen at the first solve, once the device is known:
    // measured on grids above 2^18 points (it depends on how many workgroups
    // fit per CU and on the grid; at 2048^2 the static rule's 16-row tiles spend
    // more row steps filling the level pipeline than producing), from a cost
    // model on smaller ones
    p->tune_rows = o.tile_rows == 0 && (p->f32_inner() ? p->K32 : p->K) > 1;
    if (o.graph < -1 || o.graph > 1) {
        delete p;
        return fail(CJ_ERR_ARG, "graph must be -1, 0 or 1");
    }
    if (o.single_workgroup < -1 || o.single_workgroup > 1) {
        delete p;
        return fail(CJ_ERR_ARG, "single_workgroup must be -1, 0 or 1");
    }
    {
        int band = 0;
        const bool fits = !mixed && cj::lds_solve_fits(stencil, nx, ny, nullptr, &band, nullptr);
        if (o.single_workgroup == 1 && !fits) {
            delete p;
            return fail(CJ_ERR_ARG, "single_workgroup = 1 needs an FP64 5- or 9-point plan whose padded grid fits "
                                    "in LDS (at most 1024 columns, 16 rows per lane, 160 KiB)");
        }
        // on by default only where one workgroup beat the launched cycles
        // (one CU's FP64 and LDS rates fall behind the whole chip's beyond)
        p->use_lds = fits && (o.single_workgroup == 1 ||
                              (o.single_workgroup == 0 && lds_auto(stencil, band, (long long)nx * ny)));
    }
    {
        // graphs need whole K-launches per cycle with an even launch count
        const bool shape_ok = !mixed && p->K > 1 && p->s.M % p->K == 0 && (p->s.M / p->K) % 2 == 0;
        const bool small = (long long)nx * ny <= (1LL << 22);
        p->use_graph = shape_ok && (o.graph == 1 || (o.graph == 0 && small));
    }
    *out = p;
    return CJ_OK;
}

cj_status cj_plan(int nx, int ny, int stencil, int bc, double tol, cj_plan_t* out) {
    return cj_plan_ex(nx, ny, stencil, bc, tol, nullptr, out);
}

cj_status cj_plan_info(cj_plan_t p, double* kmin, double* kmax, int* M, int* cycles_pred,
                       const double** weights_host, size_t* workspace_bytes) {
    if (!p) return fail(CJ_ERR_ARG, "plan is NULL");
    const cj::Schedule& s = p->f32_inner() ? p->sin : p->s;
    if (kmin) *kmin = s.kmin;
    if (kmax) *kmax = s.kmax;
    if (M) *M = s.M;
    if (cycles_pred) *cycles_pred = s.cycles_pred;
    if (weights_host) *weights_host = s.w.data();
    if (workspace_bytes) *workspace_bytes = p->workspace_bytes();
    return CJ_OK;
}

cj_status cj_plan_launch_info(cj_plan_t p, int* sweeps_per_launch, int* tile_rows, int* workgroups) {
    if (!p) return fail(CJ_ERR_ARG, "plan is NULL");
    const int K = p->f32_inner() ? p->K32 : p->K;
    const cj::Tiles& T = K > 1 ? (p->f32_inner() ? p->TK32 : p->TK) : p->T;
    if (sweeps_per_launch) *sweeps_per_launch = K;
    if (tile_rows) *tile_rows = T.rows;
    if (workgroups) *workgroups = T.count();
    return CJ_OK;
}

cj_status cj_solve(cj_plan_t p, const double* f, double* u, void* stream, cj_result* res) {
    return solve_common(p, f, u, nullptr, stream, res);
}

cj_status cj_solve_dd(cj_plan_t p, const double* f, double* u, double* u_lo, void* stream, cj_result* res) {
    if (!u_lo) {
        cj_result r{};
        const cj_status s = fail(CJ_ERR_ARG, "u_lo is NULL");
        r.status = s;
        if (res) *res = r;
        return s;
    }
    return solve_common(p, f, u, u_lo, stream, res);
}

cj_status cj_sweeps(cj_plan_t p, const double* f, double* u, long long n_sweeps, void* stream_) {
    if (!p) return fail(CJ_ERR_ARG, "plan is NULL");
    if (n_sweeps < 0) return fail(CJ_ERR_ARG, "n_sweeps < 0");
    cj_status st;
    if ((st = check_ptr(f, "f")) != CJ_OK || (st = check_ptr(u, "u")) != CJ_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if ((st = ensure_device(p, stream)) != CJ_OK) return st;
    double g2 = 0.0;
    if ((st = stage_in(p, f, u, stream, &g2)) != CJ_OK) return st;
    double* answer = p->A;
    if (p->f32_inner()) {
        // the plan's working precision: u and g rounded to FP32, FP32 sweeps
        // (both iterates carry the boundary: B's ring equals A's)
        CJ_HIP(cj::launch_to_f32(p->L, p->L32, p->A, p->D1, stream));
        CJ_HIP(cj::launch_to_f32(p->L, p->L32, p->B, p->D2, stream));
        CJ_HIP(cj::launch_to_f32(p->L, p->L32, p->G, p->R32, stream));
        float* cur = p->D1;
        float* nxt = p->D2;
        if ((st = enqueue_f32(p, p->sin.M, 0, n_sweeps, &cur, &nxt, stream)) != CJ_OK) return st;
        CJ_HIP(cj::launch_from_f32(p->L, p->L32, cur, p->A, stream));
        // the refinement needs the corrections' rings zero again
        CJ_HIP(hipMemsetAsync(p->D1, 0, p->L32.elems * sizeof(float), stream));
        CJ_HIP(hipMemsetAsync(p->D2, 0, p->L32.elems * sizeof(float), stream));
    } else {
        double* nxt = p->B;
        if ((st = enqueue_f64(p, 0, n_sweeps, &answer, &nxt, stream)) != CJ_OK) return st;
    }
    CJ_HIP(cj::launch_stage_out(p->L, answer, u, stream));
    CJ_HIP(hipStreamSynchronize(stream));
    return CJ_OK;
}

cj_status cj_residual(cj_plan_t p, const double* f, const double* u, void* stream_, double* rel_residual) {
    if (!p) return fail(CJ_ERR_ARG, "plan is NULL");
    if (!rel_residual) return fail(CJ_ERR_ARG, "rel_residual is NULL");
    cj_status st;
    if ((st = check_ptr(f, "f")) != CJ_OK || (st = check_ptr(u, "u")) != CJ_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if ((st = ensure_device(p, stream)) != CJ_OK) return st;
    double g2 = 0.0, r2 = 0.0;
    if ((st = stage_in(p, f, u, stream, &g2)) != CJ_OK) return st;
    CJ_HIP(cj::launch_residual(p->s.stencil, p->L, p->T, p->A, p->G, p->part, stream));
    if ((st = read_sum(p, p->T.count(), stream, &r2)) != CJ_OK) return st;
    *rel_residual = g2 == 0.0 ? 0.0 : std::sqrt(r2) / std::sqrt(g2);
    if (!std::isfinite(*rel_residual)) return fail(CJ_ERR_NONFINITE, "f or u has a NaN or Inf");
    return CJ_OK;
}

cj_status cj_residual_noalloc(cj_plan_t p, const double* f, const double* u, double* rel_residual,
                              void* stream_) {
    if (!p) return fail(CJ_ERR_ARG, "plan is NULL");
    cj_status st;
    if ((st = check_ptr(f, "f")) != CJ_OK || (st = check_ptr(u, "u")) != CJ_OK ||
        (st = check_ptr(rel_residual, "rel_residual")) != CJ_OK)
        return st;
    if (p->T.count() > cj::kNoallocMaxTiles)
        return fail(CJ_ERR_ARG, "the grid has " + std::to_string(p->T.count()) +
                                    " residual tiles; cj_residual_noalloc holds partial sums for at most " +
                                    std::to_string(cj::kNoallocMaxTiles));
    const double scale = p->s.h * p->s.h / centre_over_s(p->s.stencil);   // D^{-1}, as stage-in applies it
    const hipError_t e = cj::launch_residual_noalloc(p->s.stencil, p->s.nx, p->s.ny, p->L.frame > 0, p->T, scale, f,
                                                     u, rel_residual, static_cast<hipStream_t>(stream_));
    if (e != hipSuccess) return fail(CJ_ERR_HIP, std::string("cj_residual_noalloc: ") + hipGetErrorString(e));
    return CJ_OK;
}

cj_status cj_apply(cj_plan_t p, const double* u, double* au, void* stream_) {
    if (!p) return fail(CJ_ERR_ARG, "plan is NULL");
    cj_status st;
    if ((st = check_ptr(u, "u")) != CJ_OK || (st = check_ptr(au, "au")) != CJ_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if ((st = ensure_device(p, stream)) != CJ_OK) return st;
    double g2 = 0.0;
    // stage u in (f is not needed; G is unused here)
    if ((st = stage_in(p, nullptr, u, stream, &g2)) != CJ_OK) return st;
    CJ_HIP(cj::launch_apply(p->s.stencil, p->L, p->A, p->D, au, stream));
    CJ_HIP(hipStreamSynchronize(stream));
    return CJ_OK;
}

void cj_plan_destroy(cj_plan_t p) {
    if (!p) return;
    release(p);
    delete p;
}

const char* cj_status_string(int s) {
    switch (s) {
    case CJ_OK: return "CJ_OK";
    case CJ_STAGNATED: return "CJ_STAGNATED";
    case CJ_ERR_ARG: return "CJ_ERR_ARG";
    case CJ_ERR_NOMEM: return "CJ_ERR_NOMEM";
    case CJ_ERR_HIP: return "CJ_ERR_HIP";
    case CJ_ERR_NOT_CONVERGED: return "CJ_ERR_NOT_CONVERGED";
    case CJ_ERR_NONFINITE: return "CJ_ERR_NONFINITE";
    case CJ_ERR_DEVICE: return "CJ_ERR_DEVICE";
    default: return "CJ_UNKNOWN_STATUS";
    }
}

const char* cj_last_error(void) { return g_last_error.c_str(); }

// Lets the batch module report through cj_last_error (not part of the public header).
void cj_internal_set_error(const char* msg) { g_last_error = msg ? msg : ""; }

}  // extern "C"
