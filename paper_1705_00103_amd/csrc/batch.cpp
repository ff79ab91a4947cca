// Batched solves (C ABI cj_batch_*, declared in include/cj.h): many
// independent Poisson problems of uneven size, each with its own schedule,
// advance together in FP32 sweeps inside FP64 refinement.
//
// Super-step loop.  Every super-step is one launch per stencil group that runs
// K FP32 sweeps of every active problem (one workgroup per (problem, tile)
// work item).  A problem whose inner cycle ends in that super-step joins the
// cycle-end set E; for E, two more batched launches add the correction to u
// (FP64) and form the next FP64 residual (rounded to FP32, plus per-tile
// partial norms), a segmented reduction gives each problem's residual norm,
// and one small device-to-host copy brings those norms back.  The host then
// decides for each problem of E exactly as the single-problem refinement does
// (converged, stagnated, or the next inner cycle, halved when the last outer
// step contracted by less than 1/2) and rebuilds the work list when problems
// leave.  Between cycle ends the host only enqueues launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/cj.h"
#include "cj_internal.h"

namespace {

double centre_over_s(int stencil) {
    switch (stencil) {
    case 5: return 4.0;
    case 9: return 20.0 / 6.0;
    case 17: return 300.0 / 72.0;
    default: return NAN;
    }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// Set through cj_last_error's storage in runtime.cpp.
extern "C" void cj_internal_set_error(const char* msg);

namespace {

cj_status bfail(cj_status s, const std::string& msg) {
    cj_internal_set_error(msg.c_str());
    return s;
}

#define CJB_HIP(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return bfail(CJ_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

struct Prob {
    int nx = 0, ny = 0, stencil = 9;
    double tol = 0.0, h = 0.0;
    cj::Schedule s;                 // longest inner cycle (its M) and the kappa bounds
    std::vector<float> w32;         // weights of the cycles M, M/2, ..., mmin
    int mmin = 16;
    size_t w_offset(int m) const { return 2 * (size_t)s.M - 2 * (size_t)m; }
    cj::Layout L, L32;
    cj::Tiles T;                    // single-sweep geometry (residual, correction, stage-in)
    cj::Tiles TK;                   // blocked geometry (sweeps)
    int K = 8;
    size_t off_u = 0, off_g = 0, off_r = 0, off_d1 = 0, off_d2 = 0, off_w = 0;   // bytes into the slab
    // run state
    bool active = false;
    int m = 0, j = 0, outer = 0, fails = 0;
    double g2 = 0.0, prev = 0.0, rr = 0.0, floor_est = 0.0;
    long long sweeps = 0;
    cj_status status = CJ_OK;
};

}  // namespace

struct cj_batch_s {
    std::vector<Prob> P;
    cj_options opt;
    int max_outer = 50;
    int Kreq = 0;
    // device
    int device = -1;
    char* slab = nullptr;
    size_t slab_bytes = 0;
    cj::BatchProblem* d_probs = nullptr;
    cj::BatchItem* d_work = nullptr;     // sweep work list
    cj::BatchItem* d_work2 = nullptr;    // cycle-end work list
    double* d_part = nullptr;
    int* d_seg = nullptr;
    double* d_norm = nullptr;
    size_t cap_items = 0, cap_parts = 0;
    // pinned host mirrors
    cj::BatchProblem* h_probs = nullptr;
    cj::BatchItem* h_work = nullptr;
    cj::BatchItem* h_work2 = nullptr;
    int* h_seg = nullptr;
    double* h_norm = nullptr;
};

namespace {

void batch_release(cj_batch_s* b) {
    if (b->device >= 0) {
        int cur = -1;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(b->device);
        for (void* d : {(void*)b->slab, (void*)b->d_probs, (void*)b->d_work, (void*)b->d_work2, (void*)b->d_part,
                        (void*)b->d_seg, (void*)b->d_norm})
            if (d) (void)hipFree(d);
        for (void* h : {(void*)b->h_probs, (void*)b->h_work, (void*)b->h_work2, (void*)b->h_seg, (void*)b->h_norm})
            if (h) (void)hipHostFree(h);
        if (cur >= 0) (void)hipSetDevice(cur);
    }
    b->slab = nullptr;
    b->d_probs = nullptr;
    b->d_work = b->d_work2 = nullptr;
    b->d_part = b->d_norm = nullptr;
    b->d_seg = nullptr;
    b->h_probs = nullptr;
    b->h_work = b->h_work2 = nullptr;
    b->h_seg = nullptr;
    b->h_norm = nullptr;
    b->device = -1;
}

cj_status batch_device(cj_batch_s* b, hipStream_t stream) {
    int dev = -1;
    CJB_HIP(hipGetDevice(&dev));
    if (b->device >= 0) {
        if (dev != b->device) return bfail(CJ_ERR_DEVICE, "batch was first used on another device");
        return CJ_OK;
    }
    b->device = dev;
    const size_t n = b->P.size();
    size_t items = 0;
    for (const Prob& p : b->P) items += (size_t)std::max(p.T.count(), p.TK.count());
    b->cap_items = items;
    b->cap_parts = items;
    hipError_t e = hipMalloc((void**)&b->slab, b->slab_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_probs, n * sizeof(cj::BatchProblem));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_work, items * sizeof(cj::BatchItem));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_work2, items * sizeof(cj::BatchItem));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_part, items * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_seg, (n + 1) * sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_norm, n * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_probs, n * sizeof(cj::BatchProblem), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_work, items * sizeof(cj::BatchItem), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_work2, items * sizeof(cj::BatchItem), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_seg, (n + 1) * sizeof(int), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_norm, n * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        batch_release(b);
        (void)hipGetLastError();
        return bfail(e == hipErrorOutOfMemory ? CJ_ERR_NOMEM : CJ_ERR_HIP,
                     std::string("batch workspace allocation: ") + hipGetErrorString(e));
    }
    // corrections start and stay zero on their Dirichlet rings; upload the weight tables
    CJB_HIP(hipMemsetAsync(b->slab, 0, b->slab_bytes, stream));
    for (const Prob& p : b->P)
        CJB_HIP(hipMemcpyAsync(b->slab + p.off_w, p.w32.data(), p.w32.size() * sizeof(float), hipMemcpyHostToDevice,
                               stream));
    CJB_HIP(hipStreamSynchronize(stream));
    for (size_t i = 0; i < n; ++i) {
        const Prob& p = b->P[i];
        cj::BatchProblem& d = b->h_probs[i];
        std::memset(&d, 0, sizeof(d));
        d.u = reinterpret_cast<double*>(b->slab + p.off_u);
        d.g = reinterpret_cast<const double*>(b->slab + p.off_g);
        d.r32 = reinterpret_cast<float*>(b->slab + p.off_r);
        d.d1 = reinterpret_cast<float*>(b->slab + p.off_d1);
        d.d2 = reinterpret_cast<float*>(b->slab + p.off_d2);
        d.w32 = reinterpret_cast<const float*>(b->slab + p.off_w);
        d.nx = p.nx;
        d.ny = p.ny;
        d.pitch = p.L.pitch;
        d.pitch32 = p.L32.pitch;
        d.tiles_x = p.T.tiles_x;
        d.rows = p.T.rows;
        d.strips_x = p.TK.tiles_x;
        d.rows_k = p.TK.rows;
    }
    return CJ_OK;
}

cj_status upload_probs(cj_batch_s* b, hipStream_t stream) {
    CJB_HIP(hipMemcpyAsync(b->d_probs, b->h_probs, b->P.size() * sizeof(cj::BatchProblem), hipMemcpyHostToDevice,
                           stream));
    return CJ_OK;
}

// Cycle-end work for the problems in E: optional correction, then the residual
// and per-problem norms (copied to h_norm; waits on the stream).
cj_status cycle_end(cj_batch_s* b, const std::vector<int>& E, bool correct, hipStream_t stream) {
    if (E.empty()) return CJ_OK;
    for (int st : {5, 9, 17}) {
        // work list of the single-sweep tiles of E's problems with this stencil
        size_t n = 0;
        for (int i : E)
            if (b->P[i].stencil == st)
                for (int t = 0; t < b->P[i].T.count(); ++t) b->h_work2[n++] = cj::BatchItem{i, t};
        if (n == 0) continue;
        CJB_HIP(hipMemcpyAsync(b->d_work2, b->h_work2, n * sizeof(cj::BatchItem), hipMemcpyHostToDevice, stream));
        if (correct) CJB_HIP(cj::launch_batch_correct(st, b->d_probs, b->d_work2, (int)n, stream));
        // partials of this group land at the group's offsets; the segments below
        // index them in the same order
        CJB_HIP(cj::launch_batch_residual(st, b->d_probs, b->d_work2, (int)n, b->d_part, stream));
        // segments for this group
        int nseg = 0, pos = 0;
        std::vector<int> ids;
        for (int i : E)
            if (b->P[i].stencil == st) {
                b->h_seg[nseg++] = pos;
                pos += b->P[i].T.count();
                ids.push_back(i);
            }
        b->h_seg[nseg] = pos;
        CJB_HIP(hipMemcpyAsync(b->d_seg, b->h_seg, (nseg + 1) * sizeof(int), hipMemcpyHostToDevice, stream));
        CJB_HIP(cj::launch_segmented_reduce(b->d_part, b->d_seg, nseg, b->d_norm, stream));
        CJB_HIP(hipMemcpyAsync(b->h_norm, b->d_norm, nseg * sizeof(double), hipMemcpyDeviceToHost, stream));
        CJB_HIP(hipStreamSynchronize(stream));
        for (int k = 0; k < nseg; ++k) b->P[ids[k]].rr = std::sqrt(b->h_norm[k]) / std::sqrt(b->P[ids[k]].g2);
    }
    return CJ_OK;
}

// The refinement decision for one problem after a residual (mirrors the
// single-problem loop).  Returns true if it continues with another inner cycle.
bool decide(cj_batch_s* b, Prob& p) {
    const double rr = p.rr;
    const double q = p.outer >= 1 ? rr / p.prev : 0.0;
    p.fails = (p.outer >= 1 && q > 0.9) ? p.fails + 1 : 0;
    if (!std::isfinite(rr)) {
        p.status = CJ_ERR_NONFINITE;
    } else if (rr <= p.tol) {
        p.status = CJ_OK;
    } else if (p.fails >= 2) {
        p.status = CJ_STAGNATED;
        p.floor_est = rr < p.prev ? rr : p.prev;
    } else if (p.outer >= b->max_outer) {
        p.status = CJ_ERR_NOT_CONVERGED;
    } else {
        if (p.outer >= 1 && q > 0.5 && p.m > p.mmin) p.m /= 2;
        p.prev = rr;
        return true;
    }
    return false;
}

}  // namespace

extern "C" {

cj_status cj_batch_create(int n, const int* nx, const int* ny, const int* stencil, const double* tol,
                          const cj_options* opt, cj_batch_t* out) {
    if (!out) return bfail(CJ_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || !nx || !ny || !stencil || !tol) return bfail(CJ_ERR_ARG, "n >= 1 and non-NULL arrays required");
    cj_options o;
    cj_options_init(&o);
    if (opt) o = *opt;
    for (int r : o.reserved)
        if (r != 0) return bfail(CJ_ERR_ARG, "reserved option fields must be zero");
    if (o.precision != CJ_PRECISION_F32_REFINE)
        return bfail(CJ_ERR_ARG, "batches run FP32 sweeps inside FP64 refinement: set precision = "
                                 "CJ_PRECISION_F32_REFINE");
    if (o.M != 0 || o.inner_M != 0 || o.h != 0.0)
        return bfail(CJ_ERR_ARG, "M, inner_M and h are per problem and automatic in a batch (must be 0)");
    if (o.max_cycles < 0 || o.tile_rows < 0) return bfail(CJ_ERR_ARG, "negative option");
    const int Kreq = o.sweeps_per_launch;
    if (Kreq != 0 && Kreq != 2 && Kreq != 4 && Kreq != 8)
        return bfail(CJ_ERR_ARG, "batch sweeps_per_launch must be 0 (automatic), 2, 4 or 8");
    cj_batch_s* b = new (std::nothrow) cj_batch_s();
    if (!b) return bfail(CJ_ERR_NOMEM, "host allocation");
    b->opt = o;
    b->Kreq = Kreq;
    b->max_outer = o.max_cycles > 0 ? o.max_cycles : 50;
    b->P.resize(n);
    size_t off = 0;
    std::string err;
    for (int i = 0; i < n; ++i) {
        Prob& p = b->P[i];
        p.nx = nx[i];
        p.ny = ny[i];
        p.stencil = stencil[i];
        p.tol = tol[i];
        const int R = p.stencil == 17 ? 2 : 1;
        const int kdef = p.stencil == 17 ? 4 : 8;
        p.K = Kreq ? std::min(Kreq, kdef) : kdef;
        if (!cj::make_schedule(p.stencil, p.nx, p.ny, p.tol, 0.0, 0, &p.s, &err)) {
            delete b;
            return bfail(CJ_ERR_ARG, "problem " + std::to_string(i) + ": " + err);
        }
        p.h = p.s.h;
        p.mmin = std::max(16, p.K);
        if (p.s.M < p.mmin && !cj::make_schedule(p.stencil, p.nx, p.ny, p.tol, 0.0, p.mmin, &p.s, &err)) {
            delete b;
            return bfail(CJ_ERR_ARG, err);
        }
        p.w32.assign(2 * (size_t)p.s.M, 0.0f);
        for (int m = p.s.M; m >= p.mmin; m /= 2) {
            cj::Schedule sm;
            if (!cj::make_schedule(p.stencil, p.nx, p.ny, p.tol, 0.0, m, &sm, &err)) {
                delete b;
                return bfail(CJ_ERR_ARG, err);
            }
            for (int k = 0; k < m; ++k) p.w32[p.w_offset(m) + k] = (float)sm.w[k];
        }
        p.L = cj::make_layout(p.nx, p.ny, 8);
        p.L32 = cj::make_layout(p.nx, p.ny, 4);
        p.T = cj::make_tiles(p.nx, p.ny, 16);
        p.T.width = 256;   // batched single-sweep kernels use 256-lane tiles
        p.T.tiles_x = (p.nx + 255) / 256;
        p.TK = cj::make_tiles_k(p.nx, p.ny, p.K, R, o.tile_rows > 0 ? o.tile_rows : 64);
        p.off_u = off;  off += align256(p.L.elems * sizeof(double));
        p.off_g = off;  off += align256(p.L.elems * sizeof(double));
        p.off_r = off;  off += align256(p.L32.elems * sizeof(float));
        p.off_d1 = off; off += align256(p.L32.elems * sizeof(float));
        p.off_d2 = off; off += align256(p.L32.elems * sizeof(float));
        p.off_w = off;  off += align256(p.w32.size() * sizeof(float));
    }
    b->slab_bytes = off;
    *out = b;
    return CJ_OK;
}

cj_status cj_batch_info(cj_batch_t b, int i, int* M, int* sweeps_per_launch, size_t* workspace_bytes) {
    if (!b) return bfail(CJ_ERR_ARG, "batch is NULL");
    if (i < 0 || i >= (int)b->P.size()) return bfail(CJ_ERR_ARG, "problem index out of range");
    if (M) *M = b->P[i].s.M;
    if (sweeps_per_launch) *sweeps_per_launch = b->P[i].K;
    if (workspace_bytes) *workspace_bytes = b->slab_bytes;
    return CJ_OK;
}

cj_status cj_batch_solve(cj_batch_t b, const double* const* f, double* const* u, void* stream_, cj_result* results,
                         cj_batch_stats* stats) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!b) return bfail(CJ_ERR_ARG, "batch is NULL");
    if (!f || !u) return bfail(CJ_ERR_ARG, "f and u arrays are required");
    const int n = (int)b->P.size();
    for (int i = 0; i < n; ++i) {
        if (!f[i] || !u[i]) return bfail(CJ_ERR_ARG, "problem " + std::to_string(i) + ": NULL f or u");
        if (reinterpret_cast<uintptr_t>(f[i]) % 8 || reinterpret_cast<uintptr_t>(u[i]) % 8)
            return bfail(CJ_ERR_ARG, "problem " + std::to_string(i) + ": misaligned f or u");
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    cj_status st;
    if ((st = batch_device(b, stream)) != CJ_OK) return st;

    // ---- stage-in: every problem's u and g = D^{-1} f, with sums of g^2
    {
        int pos = 0;
        for (int i = 0; i < n; ++i) {
            Prob& p = b->P[i];
            double* du = reinterpret_cast<double*>(b->slab + p.off_u);
            double* dg = reinterpret_cast<double*>(b->slab + p.off_g);
            const double scale = p.h * p.h / centre_over_s(p.stencil);
            CJB_HIP(cj::launch_ring(p.L, u[i], du, du, dg, stream));
            CJB_HIP(cj::launch_stage_in(p.L, p.T, f[i], u[i], scale, du, du, dg, b->d_part + pos, stream));
            b->h_seg[i] = pos;
            pos += p.T.count();
        }
        b->h_seg[n] = pos;
        CJB_HIP(hipMemcpyAsync(b->d_seg, b->h_seg, (n + 1) * sizeof(int), hipMemcpyHostToDevice, stream));
        CJB_HIP(cj::launch_segmented_reduce(b->d_part, b->d_seg, n, b->d_norm, stream));
        CJB_HIP(hipMemcpyAsync(b->h_norm, b->d_norm, n * sizeof(double), hipMemcpyDeviceToHost, stream));
        CJB_HIP(hipStreamSynchronize(stream));
    }
    std::vector<int> E;
    for (int i = 0; i < n; ++i) {
        Prob& p = b->P[i];
        p.g2 = b->h_norm[i];
        p.active = false;
        p.outer = p.fails = 0;
        p.sweeps = 0;
        p.prev = p.rr = p.floor_est = 0.0;
        p.m = p.s.M;
        if (!std::isfinite(p.g2)) {
            p.status = CJ_ERR_NONFINITE;
        } else if (p.g2 == 0.0) {
            p.status = CJ_OK;
            CJB_HIP(hipMemsetAsync(u[i], 0, (size_t)p.nx * (size_t)p.ny * sizeof(double), stream));
        } else {
            E.push_back(i);
        }
        cj::BatchProblem& d = b->h_probs[i];
        d.dnext = 0;
        d.dcur = 0;
        d.cycle_start = 0;
        d.w32 = reinterpret_cast<const float*>(b->slab + p.off_w + p.w_offset(p.m) * sizeof(float));
    }
    // ---- initial residuals
    CJB_HIP(hipStreamSynchronize(stream));
    if ((st = upload_probs(b, stream)) != CJ_OK) return st;
    if ((st = cycle_end(b, E, false, stream)) != CJ_OK) return st;
    int step = 0;
    long long launches = 0;
    int supersteps = 0;
    for (int i : E) {
        Prob& p = b->P[i];
        if (decide(b, p)) {
            p.active = true;
            p.j = 0;
            cj::BatchProblem& d = b->h_probs[i];
            d.cycle_start = step;
            d.w32 = reinterpret_cast<const float*>(b->slab + p.off_w + p.w_offset(p.m) * sizeof(float));
        }
    }
    if ((st = upload_probs(b, stream)) != CJ_OK) return st;

    // ---- super-steps
    std::vector<size_t> group_n(3, 0);
    const int stencils[3] = {5, 9, 17};
    bool rebuild = true;
    for (;;) {
        bool any = false;
        for (const Prob& p : b->P) any = any || p.active;
        if (!any) break;
        if (rebuild) {
            // sweep work list: per stencil group, items of active problems, contiguous
            size_t pos = 0;
            for (int gi = 0; gi < 3; ++gi) {
                const size_t start = pos;
                for (int i = 0; i < n; ++i) {
                    const Prob& p = b->P[i];
                    if (!p.active || p.stencil != stencils[gi]) continue;
                    for (int t = 0; t < p.TK.count(); ++t) b->h_work[pos++] = cj::BatchItem{i, t};
                }
                group_n[gi] = pos - start;
            }
            CJB_HIP(hipMemcpyAsync(b->d_work, b->h_work, pos * sizeof(cj::BatchItem), hipMemcpyHostToDevice, stream));
            rebuild = false;
        }
        size_t base = 0;
        for (int gi = 0; gi < 3; ++gi) {
            if (group_n[gi] == 0) continue;
            // the K of a group: all its problems share it (depends on the stencil only)
            int K = 0;
            for (const Prob& p : b->P)
                if (p.stencil == stencils[gi]) {
                    K = p.K;
                    break;
                }
            CJB_HIP(cj::launch_batch_sweepk(stencils[gi], K, b->d_probs, b->d_work + base, (int)group_n[gi], step,
                                            stream));
            ++launches;
            base += group_n[gi];
        }
        ++step;
        ++supersteps;
        E.clear();
        for (int i = 0; i < n; ++i) {
            Prob& p = b->P[i];
            if (!p.active) continue;
            ++p.j;
            if (p.j * p.K == p.m) E.push_back(i);
        }
        if (E.empty()) continue;
        for (int i : E) {
            Prob& p = b->P[i];
            p.sweeps += p.m;
            p.outer += 1;
            b->h_probs[i].dcur = p.j & 1;   // launch j-1 wrote d[j & 1]
        }
        if ((st = upload_probs(b, stream)) != CJ_OK) return st;
        if ((st = cycle_end(b, E, true, stream)) != CJ_OK) return st;
        for (int i : E) {
            Prob& p = b->P[i];
            if (decide(b, p)) {
                p.j = 0;
                cj::BatchProblem& d = b->h_probs[i];
                d.cycle_start = step;
                d.w32 = reinterpret_cast<const float*>(b->slab + p.off_w + p.w_offset(p.m) * sizeof(float));
            } else {
                p.active = false;
                rebuild = true;
            }
        }
        if ((st = upload_probs(b, stream)) != CJ_OK) return st;
    }
    // ---- stage-out
    for (int i = 0; i < n; ++i) {
        Prob& p = b->P[i];
        if (p.g2 == 0.0 || !std::isfinite(p.g2)) continue;
        CJB_HIP(cj::launch_stage_out(p.L, reinterpret_cast<double*>(b->slab + p.off_u), u[i], stream));
    }
    CJB_HIP(hipStreamSynchronize(stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    cj_status worst = CJ_OK;
    for (int i = 0; i < n; ++i) {
        const Prob& p = b->P[i];
        if (results) {
            cj_result& r = results[i];
            std::memset(&r, 0, sizeof(r));
            r.status = p.status;
            r.cycles = p.outer;
            r.sweeps = p.sweeps;
            r.rel_residual = p.rr;
            r.floor_estimate = p.status == CJ_STAGNATED ? p.floor_est : 0.0;
            r.seconds = secs;
        }
        if (p.status != CJ_OK && worst == CJ_OK) worst = p.status;
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->supersteps = supersteps;
        stats->launches = launches;
        long long pts = 0;
        for (const Prob& p : b->P) pts += (long long)p.nx * p.ny;
        stats->points = pts;
        stats->seconds = secs;
        double upd = 0.0;
        for (const Prob& p : b->P) upd += (double)p.nx * p.ny * (double)p.sweeps;
        stats->updates = upd;
    }
    return worst == CJ_STAGNATED ? CJ_STAGNATED : (worst == CJ_OK ? CJ_OK : worst);
}

void cj_batch_destroy(cj_batch_t b) {
    if (!b) return;
    batch_release(b);
    delete b;
}

}  // extern "C"
