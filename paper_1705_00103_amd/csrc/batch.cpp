// Batched and served solves (C ABI cj_batch_* and cj_server_*, declared in
// include/cj.h): many independent Poisson problems of uneven size, each with
// its own schedule, advance together in FP32 sweeps inside FP64 refinement.
//
// Both APIs drive one engine.  Problems live in a device pool (the HBM
// budget); a problem is admitted when its arrays fit in the pool and leaves
// when it is finished, freeing its space for the next.
//
// Engine step (one "super-step"):
//   1. admit queued problems that fit: allocate, stage u and g = D^{-1} f in;
//   2. one launch per stencil group runs K FP32 sweeps of every active problem
//      (one workgroup per (problem, tile) work item), repeated up to the first
//      inner-cycle end among the active problems (the server: at most 32
//      times, so that arrivals are admitted soon);
//   3. problems whose inner cycle ended (set E), and the newly admitted ones,
//      get their correction u += d and their next FP64 residual (rounded to
//      FP32, plus per-tile partial norms) in batched launches; one segmented
//      reduction yields every norm needed (|g|^2 of the new ones, |r|^2 of E
//      and the new ones) and one small device-to-host copy brings them back;
//   4. the host decides for each of them exactly as the single-problem
//      refinement does (converged, stagnated, or another inner cycle, halved
//      when the last outer step contracted by less than 1/2); finished
//      problems are staged out and their pool space is released.
// Between cycle ends and admissions a step only enqueues its launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/cj.h"
#include "cj_internal.h"

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

double centre_over_s(int stencil) {
    switch (stencil) {
    case 5: return 4.0;
    case 9: return 20.0 / 6.0;
    case 17: return 300.0 / 72.0;
    default: return NAN;
    }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum class State { Queued, New, Active, Done };

// One problem: its host plan (schedules, layouts, geometry, pool footprint)
// and its run state.
struct Problem {
    long long ticket = 0;
    int nx = 0, ny = 0, stencil = 9;
    double tol = 0.0, h = 0.0;
    const double* f = nullptr;
    double* u = nullptr;
    cj::Schedule s;                 // longest inner cycle (its M) and the kappa bounds
    std::vector<float> w32;         // FP32 weights of the cycles M, M/2, ..., mmin
    int mmin = 16, K = 8;
    size_t w_offset(int m) const { return 2 * (size_t)s.M - 2 * (size_t)m; }
    cj::Layout L, L32;
    cj::Tiles T;                    // single-sweep geometry (stage-in, residual, correction), 256-lane tiles
    cj::Tiles TK;                   // blocked geometry (sweeps)
    size_t bytes = 0;               // pool footprint
    size_t off_u = 0, off_g = 0, off_r = 0, off_d1 = 0, off_d2 = 0, off_w = 0;   // within the block
    // placement
    size_t block = 0;
    int slot = -1;
    // run state
    State state = State::Queued;
    int m = 0, j = 0, outer = 0, fails = 0;
    double g2 = 0.0, prev = 0.0, rr = 0.0, floor_est = 0.0;
    long long sweeps = 0;
    cj_status status = CJ_OK;
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
};

// Builds the host plan of a problem; K from the requested depth (0: automatic).
cj_status plan_problem(Problem& p, int Kreq, int tile_rows) {
    std::string err;
    if (!cj::make_schedule(p.stencil, p.nx, p.ny, p.tol, 0.0, 0, &p.s, &err)) return bfail(CJ_ERR_ARG, err);
    const int R = p.stencil == 17 ? 2 : 1;
    const int kdef = p.stencil == 17 ? 4 : 8;
    p.K = Kreq ? std::min(Kreq, kdef) : kdef;
    p.h = p.s.h;
    p.mmin = std::max(16, p.K);
    if (p.s.M < p.mmin && !cj::make_schedule(p.stencil, p.nx, p.ny, p.tol, 0.0, p.mmin, &p.s, &err))
        return bfail(CJ_ERR_ARG, err);
    p.w32.assign(2 * (size_t)p.s.M, 0.0f);
    for (int m = p.s.M; m >= p.mmin; m /= 2) {
        cj::Schedule sm;
        if (!cj::make_schedule(p.stencil, p.nx, p.ny, p.tol, 0.0, m, &sm, &err)) return bfail(CJ_ERR_ARG, err);
        for (int k = 0; k < m; ++k) p.w32[p.w_offset(m) + k] = (float)sm.w[k];
    }
    p.L = cj::make_layout(p.nx, p.ny, 8);
    p.L32 = cj::make_layout(p.nx, p.ny, 4);
    p.T = cj::make_tiles(p.nx, p.ny, 16);
    p.T.width = 256;
    p.T.tiles_x = (p.nx + 255) / 256;
    p.TK = cj::make_tiles_k(p.nx, p.ny, p.K, R, tile_rows > 0 ? tile_rows : 64, sizeof(float));
    size_t off = 0;
    p.off_u = off;  off += align256(p.L.elems * sizeof(double));
    p.off_g = off;  off += align256(p.L.elems * sizeof(double));
    p.off_r = off;  off += align256(p.L32.elems * sizeof(float));
    p.off_d1 = off; off += align256(p.L32.elems * sizeof(float));
    p.off_d2 = off; off += align256(p.L32.elems * sizeof(float));
    p.off_w = off;  off += align256(p.w32.size() * sizeof(float));
    p.bytes = off;
    return CJ_OK;
}

// First-fit allocator over [0, size) of the device pool.
struct PoolAlloc {
    std::map<size_t, size_t> free_;   // offset -> length
    size_t size = 0, used = 0;
    void reset(size_t n) {
        free_.clear();
        size = n;
        used = 0;
        if (n) free_[0] = n;
    }
    bool alloc(size_t n, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, roff = it->first + n;
                free_.erase(it);
                if (rest) free_[roff] = rest;
                used += n;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n) {
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

template <typename T>
struct DevBuf {   // device array with a pinned host mirror, grown at sync points
    T* d = nullptr;
    T* h = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n) {
        if (n <= cap) return hipSuccess;
        const size_t c = std::max<size_t>(n, cap + cap / 2 + 16);
        if (d) (void)hipFree(d);
        if (h) (void)hipHostFree(h);
        d = nullptr;
        h = nullptr;
        cap = 0;
        hipError_t e = hipMalloc((void**)&d, c * sizeof(T));
        if (e == hipSuccess) e = hipHostMalloc((void**)&h, c * sizeof(T), hipHostMallocDefault);
        if (e == hipSuccess) cap = c;
        return e;
    }
    void release() {
        if (d) (void)hipFree(d);
        if (h) (void)hipHostFree(h);
        d = nullptr;
        h = nullptr;
        cap = 0;
    }
};

const int kStencils[3] = {5, 9, 17};

class Engine {
public:
    cj_options opt{};
    int max_outer = 50;
    int Kreq = 0;
    size_t budget = 0;
    int device = -1;
    int cus = 0;                      // compute units of the device (0: unknown)
    char* pool = nullptr;
    PoolAlloc alloc;
    std::vector<Problem*> slots;      // descriptor index -> problem (nullptr: free)
    std::deque<Problem*> queue;       // submitted, not admitted (FIFO; a later one that fits may pass)
    std::vector<Problem*> live;       // admitted, not finished
    DevBuf<cj::BatchProblem> probs;
    DevBuf<cj::BatchItem> work, work2;
    DevBuf<int> seg;
    DevBuf<double> norm;
    double* part = nullptr;
    size_t part_cap = 0;
    // Autotuner of a batch (all problems known up front, depth and tile height
    // automatic): before the first inner cycle it times (K, tile rows) per
    // stencil group on the problems themselves and keeps the fastest per sweep.
    bool autotune = false;
    bool tuned = false;
    int tuned_K[3] = {0, 0, 0};
    int tuned_rows[3] = {0, 0, 0};
    int step_no = 0;
    // Most super-steps one engine step enqueues (0: no limit).  A step runs up
    // to the first inner-cycle end among the active problems, where the host
    // has something to decide; the server caps it so that new arrivals are
    // admitted soon, a batch (all problems known up front) does not.
    int max_supersteps = 0;
    bool rebuild = true;
    size_t group_size[3] = {0, 0, 0};
    long long launches = 0, supersteps = 0;
    double updates = 0.0;

    ~Engine() { release(); }

    void release() {
        if (device >= 0) {
            int cur = -1;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(device);
            if (pool) (void)hipFree(pool);
            if (part) (void)hipFree(part);
            probs.release();
            work.release();
            work2.release();
            seg.release();
            norm.release();
            if (cur >= 0) (void)hipSetDevice(cur);
        }
        pool = nullptr;
        part = nullptr;
        part_cap = 0;
        device = -1;
    }

    cj_status bind() {
        int dev = -1;
        CJB_HIP(hipGetDevice(&dev));
        if (device >= 0) {
            if (dev != device) return bfail(CJ_ERR_DEVICE, "engine was first used on another device");
            return CJ_OK;
        }
        hipError_t e = hipMalloc((void**)&pool, budget);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            pool = nullptr;
            return bfail(e == hipErrorOutOfMemory ? CJ_ERR_NOMEM : CJ_ERR_HIP,
                         std::string("pool allocation: ") + hipGetErrorString(e));
        }
        device = dev;
        alloc.reset(budget);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            cus = 0;
        }
        return CJ_OK;
    }

    bool idle() const { return queue.empty() && live.empty(); }

    cj::BatchProblem& desc(const Problem* p) { return probs.h[p->slot]; }

    const float* wptr(const Problem* p) const {
        return reinterpret_cast<const float*>(pool + p->block + p->off_w + p->w_offset(p->m) * sizeof(float));
    }

    // Descriptors go up with a wait, so that the pinned mirror can be edited
    // again as soon as this returns.
    cj_status upload_probs(hipStream_t stream) {
        if (slots.empty()) return CJ_OK;
        CJB_HIP(hipMemcpyAsync(probs.d, probs.h, slots.size() * sizeof(cj::BatchProblem), hipMemcpyHostToDevice,
                               stream));
        CJB_HIP(hipStreamSynchronize(stream));
        return CJ_OK;
    }

    int take_slot(Problem* p) {
        for (size_t i = 0; i < slots.size(); ++i)
            if (!slots[i]) {
                slots[i] = p;
                return (int)i;
            }
        slots.push_back(p);
        return (int)slots.size() - 1;
    }

    // Admits queued problems that fit in the pool (FIFO order; a later one may
    // pass one that does not fit yet) and enqueues their stage-in.
    cj_status admit(hipStream_t stream, std::vector<Problem*>* fresh) {
        for (auto it = queue.begin(); it != queue.end();) {
            Problem* p = *it;
            size_t off = 0;
            if (!alloc.alloc(p->bytes, &off)) {
                ++it;
                continue;
            }
            p->block = off;
            p->slot = take_slot(p);
            p->state = State::New;
            p->t_admit = now_s();
            fresh->push_back(p);
            live.push_back(p);
            it = queue.erase(it);
        }
        if (fresh->empty()) return CJ_OK;
        if (probs.cap < slots.size()) {
            // growing the descriptor array: keep the entries of the live problems
            std::vector<cj::BatchProblem> keep(probs.h, probs.h + probs.cap);
            CJB_HIP(hipStreamSynchronize(stream));
            if (probs.ensure(slots.size()) != hipSuccess) return bfail(CJ_ERR_NOMEM, "descriptor allocation");
            std::copy(keep.begin(), keep.end(), probs.h);
        }
        for (Problem* p : *fresh) {
            char* base = pool + p->block;
            // the corrections start zero and their Dirichlet rings stay zero
            CJB_HIP(hipMemsetAsync(base + p->off_r, 0, p->off_w - p->off_r, stream));
            CJB_HIP(hipMemcpyAsync(base + p->off_w, p->w32.data(), p->w32.size() * sizeof(float),
                                   hipMemcpyHostToDevice, stream));
            cj::BatchProblem& d = desc(p);
            std::memset(&d, 0, sizeof(d));
            d.u = reinterpret_cast<double*>(base + p->off_u);
            d.g = reinterpret_cast<const double*>(base + p->off_g);
            d.r32 = reinterpret_cast<float*>(base + p->off_r);
            d.d1 = reinterpret_cast<float*>(base + p->off_d1);
            d.d2 = reinterpret_cast<float*>(base + p->off_d2);
            d.nx = p->nx;
            d.ny = p->ny;
            d.pitch = p->L.pitch;
            d.pitch32 = p->L32.pitch;
            d.tiles_x = p->T.tiles_x;
            d.rows = p->T.rows;
            d.strips_x = p->TK.tiles_x;
            d.rows_k = p->TK.rows;
            p->m = p->s.M;
            p->j = p->outer = p->fails = 0;
            p->sweeps = 0;
            p->prev = p->rr = p->floor_est = p->g2 = 0.0;
            d.w32 = wptr(p);
        }
        return CJ_OK;
    }

    cj_status ensure_part(size_t n, hipStream_t stream) {
        if (n <= part_cap) return CJ_OK;
        CJB_HIP(hipStreamSynchronize(stream));
        if (part) (void)hipFree(part);
        part = nullptr;
        part_cap = 0;
        const size_t c = std::max<size_t>(n, 1024);
        CJB_HIP(hipMalloc((void**)&part, c * sizeof(double)));
        part_cap = c;
        return CJ_OK;
    }

    // The refinement decision (mirrors the single-problem loop).  True: continue.
    bool decide(Problem& p) {
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
        } else if (p.outer >= max_outer) {
            p.status = CJ_ERR_NOT_CONVERGED;
        } else {
            if (p.outer >= 1 && q > 0.5 && p.m > p.mmin) p.m /= 2;
            p.prev = rr;
            return true;
        }
        return false;
    }

    static int group_of(int stencil) { return stencil == 5 ? 0 : stencil == 9 ? 1 : 2; }

    void set_rows(Problem* p, int rows) {
        p->TK = cj::make_tiles_k(p->nx, p->ny, p->K, p->stencil == 17 ? 2 : 1, rows, sizeof(float));
        desc(p).strips_x = p->TK.tiles_x;
        desc(p).rows_k = p->TK.rows;
    }

    // A new blocked depth for a problem at the start of a cycle (its cycle
    // lengths, at least 16, are multiples of every depth used here).
    void set_depth(Problem* p, int K) {
        p->K = K;
        set_rows(p, p->TK.rows);
    }

    // Work list of the active problems' blocked tiles, grouped by stencil.
    cj_status build_work(hipStream_t stream) {
        size_t n = 0;
        for (Problem* p : live)
            if (p->state == State::Active) n += p->TK.count();
        if (work.cap < n) {
            CJB_HIP(hipStreamSynchronize(stream));
            if (work.ensure(n) != hipSuccess) return bfail(CJ_ERR_NOMEM, "work list allocation");
        }
        size_t pos = 0;
        for (int gi = 0; gi < 3; ++gi) {
            const size_t start = pos;
            for (Problem* p : live)
                if (p->state == State::Active && p->stencil == kStencils[gi])
                    for (int t = 0; t < p->TK.count(); ++t) work.h[pos++] = cj::BatchItem{p->slot, t};
            group_size[gi] = pos - start;
        }
        CJB_HIP(hipMemcpyAsync(work.d, work.h, pos * sizeof(cj::BatchItem), hipMemcpyHostToDevice, stream));
        CJB_HIP(hipStreamSynchronize(stream));
        return CJ_OK;
    }

    // The batch autotuner.  Every active problem is at the start of its first
    // inner cycle: its correction d1 is zero and d2 is free.  For each stencil
    // group and each (K, tile rows) candidate it times two super-steps of the
    // group's problems (two launches), which read d1, write d2, then d1, and
    // scores the time per sweep; the fastest is kept
    // for the rest of the batch's life (cj_batch_stats reports it).  d1 and d2
    // are zeroed afterwards.  Tiles only partition the grids and a K-sweep
    // launch gives the bits of K single sweeps, so the choice changes speed
    // only.
    cj_status tune(hipStream_t stream) {
        static const int kK[3] = {8, 4, 2};
        static const int kRows[4] = {16, 32, 64, 128};
        hipEvent_t e0 = nullptr, e1 = nullptr;
        CJB_HIP(hipEventCreate(&e0));
        CJB_HIP(hipEventCreate(&e1));
        cj_status st = CJ_OK;
        for (int gi = 0; gi < 3 && st == CJ_OK; ++gi) {
            std::vector<Problem*> grp;
            for (Problem* p : live)
                if (p->state == State::Active && p->stencil == kStencils[gi]) grp.push_back(p);
            if (grp.empty()) continue;
            float best = -1.0f;
            int bestK = grp[0]->K, bestRows = grp[0]->TK.rows;
            for (int K : kK) {
                if (kStencils[gi] == 17 && K > 4) continue;
                for (int rows : kRows) {
                    for (Problem* p : grp) {
                        p->K = K;
                        set_rows(p, rows);
                        desc(p).cycle_start = step_no;
                    }
                    if ((st = upload_probs(stream)) != CJ_OK) break;
                    if ((st = build_work(stream)) != CJ_OK) break;
                    size_t base = 0;
                    for (int g = 0; g < gi; ++g) base += group_size[g];
                    const int n_items = (int)group_size[gi];
                    float ms = 0.0f;
                    hipError_t e = hipEventRecord(e0, stream);
                    for (int k = 0; k < 2 && e == hipSuccess; ++k)
                        e = cj::launch_batch_sweepk(kStencils[gi], K, probs.d, work.d + base, n_items, step_no + k,
                                                    stream);
                    if (e == hipSuccess) e = hipEventRecord(e1, stream);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                    if (e != hipSuccess) {
                        st = bfail(CJ_ERR_HIP, std::string("batch autotuner: ") + hipGetErrorString(e));
                        break;
                    }
                    const float per_sweep = ms / (2.0f * (float)K);
                    if (best < 0.0f || per_sweep < best) {
                        best = per_sweep;
                        bestK = K;
                        bestRows = rows;
                    }
                }
                if (st != CJ_OK) break;
            }
            tuned_K[gi] = bestK;
            tuned_rows[gi] = bestRows;
            for (Problem* p : grp) {
                char* base = pool + p->block;
                if (st == CJ_OK && hipMemsetAsync(base + p->off_d1, 0, p->off_w - p->off_d1, stream) != hipSuccess)
                    st = bfail(CJ_ERR_HIP, "batch autotuner: clearing the corrections");
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != CJ_OK) return st;
        tuned = true;
        return CJ_OK;
    }

    // One engine step (see the file comment).  Finished problems are appended to *done.
    cj_status step(hipStream_t stream, std::vector<Problem*>* done) {
        cj_status st;
        if ((st = bind()) != CJ_OK) return st;
        std::vector<Problem*> fresh;
        if ((st = admit(stream, &fresh)) != CJ_OK) return st;
        // stage-in of the admitted problems; their partials go first in `part`
        size_t n_in = 0, n_res = 0;
        for (Problem* p : fresh) n_in += p->T.count();
        for (Problem* p : live) n_res += p->T.count();
        if ((st = ensure_part(n_in + n_res, stream)) != CJ_OK) return st;
        {
            size_t pos = 0;
            for (Problem* p : fresh) {
                char* base = pool + p->block;
                double* du = reinterpret_cast<double*>(base + p->off_u);
                double* dg = reinterpret_cast<double*>(base + p->off_g);
                const double scale = p->h * p->h / centre_over_s(p->stencil);
                CJB_HIP(cj::launch_ring(p->L, p->u, du, du, dg, stream));
                CJB_HIP(cj::launch_stage_in(p->L, p->T, p->f, p->u, scale, du, du, dg, part + pos, stream));
                pos += p->T.count();
            }
        }
        // batched sweeps of the active problems
        int n_ss = 0;
        bool any_active = false;
        for (Problem* p : live) any_active = any_active || p->state == State::Active;
        if (any_active) {
            if (rebuild) {
                bool all_fresh = true;   // every active problem is at the start of its first cycle
                for (Problem* p : live)
                    if (p->state == State::Active && (p->j != 0 || p->outer != 0)) all_fresh = false;
                if (autotune && !tuned && all_fresh && (st = tune(stream)) != CJ_OK) return st;
                if (autotune && tuned) {
                    for (Problem* p : live)
                        if (p->state == State::Active) {
                            const int gi = group_of(p->stencil);
                            if (p->j == 0 && p->K != tuned_K[gi]) set_depth(p, tuned_K[gi]);
                            if (p->TK.rows != std::min(tuned_rows[gi], p->ny)) set_rows(p, tuned_rows[gi]);
                        }
                    if ((st = upload_probs(stream)) != CJ_OK) return st;
                } else if (opt.tile_rows == 0) {
                    // Tile height from the load: 64 rows while the active problems
                    // have at least 2048 tiles (the device is full and taller tiles
                    // waste less on their pipeline fill), shorter (down to 16) when
                    // few problems run, so that a lone small problem still spreads
                    // over many CUs.  Below that a launch costs the latency of its
                    // row pipeline, rounds x (rows + 2KR + K - 1) row steps with one
                    // workgroup per CU per round; the height from {16, 8, 4, 2, 1}
                    // that minimises it is taken.  Tiles only partition the grid:
                    // results do not depend on the height.
                    auto active_tiles = [&](int r) {
                        long long tiles = 0;
                        for (Problem* p : live)
                            if (p->state == State::Active)
                                tiles += cj::make_tiles_k(p->nx, p->ny, p->K, p->stencil == 17 ? 2 : 1, r, sizeof(float)).count();
                        return tiles;
                    };
                    int rows = 64;
                    for (; rows > 16; rows /= 2)
                        if (active_tiles(rows) >= 2048) break;
                    if (rows == 16 && cus > 0 && active_tiles(16) < 2048) {
                        int fill = 0;
                        for (Problem* p : live)
                            if (p->state == State::Active)
                                fill = std::max(fill, 2 * p->K * (p->stencil == 17 ? 2 : 1) + p->K - 1);
                        long long best = -1;
                        for (int r = 16; r >= 1; r /= 2) {
                            const long long cost = ((active_tiles(r) + cus - 1) / cus) * (r + fill);
                            if (best < 0 || cost < best) {
                                best = cost;
                                rows = r;
                            }
                        }
                    }
                    for (Problem* p : live)
                        if (p->state == State::Active && p->TK.rows != std::min(rows, p->ny)) {
                            p->TK = cj::make_tiles_k(p->nx, p->ny, p->K, p->stencil == 17 ? 2 : 1, rows, sizeof(float));
                            desc(p).strips_x = p->TK.tiles_x;
                            desc(p).rows_k = p->TK.rows;
                        }
                    if ((st = upload_probs(stream)) != CJ_OK) return st;
                }
                if ((st = build_work(stream)) != CJ_OK) return st;
                rebuild = false;
            }
            // super-steps until the first cycle end among the active problems
            n_ss = 0;
            for (Problem* p : live)
                if (p->state == State::Active) {
                    const int left = p->m / p->K - p->j;
                    if (n_ss == 0 || left < n_ss) n_ss = left;
                }
            if (n_ss < 1) n_ss = 1;
            if (max_supersteps > 0 && n_ss > max_supersteps) n_ss = max_supersteps;
            int Kg[3] = {0, 0, 0};
            for (int gi = 0; gi < 3; ++gi)
                for (Problem* p : live)
                    if (p->state == State::Active && p->stencil == kStencils[gi]) {
                        Kg[gi] = p->K;   // one depth per stencil group
                        break;
                    }
            for (int k = 0; k < n_ss; ++k) {
                size_t base = 0;
                for (int gi = 0; gi < 3; ++gi) {
                    if (group_size[gi] == 0) continue;
                    CJB_HIP(cj::launch_batch_sweepk(kStencils[gi], Kg[gi], probs.d, work.d + base,
                                                    (int)group_size[gi], step_no, stream));
                    ++launches;
                    base += group_size[gi];
                }
                ++step_no;
                ++supersteps;
            }
        }
        // cycle ends
        std::vector<Problem*> R;
        for (Problem* p : live) {
            if (p->state != State::Active) continue;
            p->j += n_ss;
            if (p->j * p->K == p->m) {
                R.push_back(p);
                p->sweeps += p->m;
                updates += (double)p->nx * p->ny * p->m;
                p->outer += 1;
                desc(p).dcur = p->j & 1;   // launch j-1 wrote d[j & 1]
            }
        }
        if (R.empty() && fresh.empty()) return CJ_OK;
        const size_t n_ends = R.size();
        R.insert(R.end(), fresh.begin(), fresh.end());
        if ((st = upload_probs(stream)) != CJ_OK) return st;
        // work list of R's single-sweep tiles per stencil group
        size_t n2 = 0;
        for (Problem* p : R) n2 += p->T.count();
        if (work2.cap < n2) {
            CJB_HIP(hipStreamSynchronize(stream));
            if (work2.ensure(n2) != hipSuccess) return bfail(CJ_ERR_NOMEM, "work list allocation");
        }
        std::vector<Problem*> order;   // R in the order of their residual partials
        std::pair<size_t, size_t> grp[3];
        size_t pos = 0;
        for (int gi = 0; gi < 3; ++gi) {
            const size_t start = pos;
            for (Problem* p : R)
                if (p->stencil == kStencils[gi]) {
                    for (int t = 0; t < p->T.count(); ++t) work2.h[pos++] = cj::BatchItem{p->slot, t};
                    order.push_back(p);
                }
            grp[gi] = std::make_pair(start, pos - start);
        }
        CJB_HIP(hipMemcpyAsync(work2.d, work2.h, pos * sizeof(cj::BatchItem), hipMemcpyHostToDevice, stream));
        for (int gi = 0; gi < 3; ++gi) {
            const size_t start = grp[gi].first, cnt = grp[gi].second;
            if (cnt == 0) continue;
            // the correction of a fresh problem adds its zero d: exact, and keeps one work list
            if (n_ends > 0)
                CJB_HIP(cj::launch_batch_correct(kStencils[gi], probs.d, work2.d + start, (int)cnt, stream));
            CJB_HIP(cj::launch_batch_residual(kStencils[gi], probs.d, work2.d + start, (int)cnt,
                                              part + n_in + start, stream));
        }
        // segments: |g|^2 of the fresh ones (stage-in partials), then |r|^2 of `order`
        const size_t nseg = fresh.size() + order.size();
        if (seg.cap < nseg + 1 || norm.cap < nseg) {
            CJB_HIP(hipStreamSynchronize(stream));
            if (seg.ensure(nseg + 1) != hipSuccess || norm.ensure(nseg) != hipSuccess)
                return bfail(CJ_ERR_NOMEM, "segment allocation");
        }
        {
            int s = 0, p0 = 0;
            for (Problem* p : fresh) {
                seg.h[s++] = p0;
                p0 += p->T.count();
            }
            for (Problem* p : order) {
                seg.h[s++] = p0;
                p0 += p->T.count();
            }
            seg.h[s] = p0;
        }
        CJB_HIP(hipMemcpyAsync(seg.d, seg.h, (nseg + 1) * sizeof(int), hipMemcpyHostToDevice, stream));
        CJB_HIP(cj::launch_segmented_reduce(part, seg.d, (int)nseg, norm.d, stream));
        CJB_HIP(hipMemcpyAsync(norm.h, norm.d, nseg * sizeof(double), hipMemcpyDeviceToHost, stream));
        CJB_HIP(hipStreamSynchronize(stream));
        for (size_t k = 0; k < fresh.size(); ++k) fresh[k]->g2 = norm.h[k];
        for (size_t k = 0; k < order.size(); ++k) {
            Problem* p = order[k];
            p->rr = std::sqrt(norm.h[fresh.size() + k]) / std::sqrt(p->g2);
        }
        // decisions
        for (Problem* p : R) {
            bool cont = false;
            if (p->state == State::New && !std::isfinite(p->g2)) {
                p->status = CJ_ERR_NONFINITE;
            } else if (p->state == State::New && p->g2 == 0.0) {
                p->status = CJ_OK;
                p->rr = 0.0;
                CJB_HIP(hipMemsetAsync(p->u, 0, (size_t)p->nx * (size_t)p->ny * sizeof(double), stream));
            } else {
                cont = decide(*p);
            }
            if (cont) {
                if (p->state == State::New) rebuild = true;
                p->state = State::Active;
                p->j = 0;
                cj::BatchProblem& d = desc(p);
                d.cycle_start = step_no;
                d.w32 = wptr(p);
            } else {
                if (p->state == State::Active) rebuild = true;
                if (p->g2 != 0.0 && std::isfinite(p->g2))
                    CJB_HIP(cj::launch_stage_out(p->L, reinterpret_cast<double*>(pool + p->block + p->off_u), p->u,
                                                 stream));
                slots[p->slot] = nullptr;
                alloc.release(p->block, p->bytes);
                live.erase(std::find(live.begin(), live.end(), p));
                p->state = State::Done;
                p->t_done = now_s();
                done->push_back(p);
            }
        }
        // the wait here also completes the stage-outs before results are reported
        return upload_probs(stream);
    }

    // Drops every queued and live problem (after an error), leaving the engine reusable.
    void reset_run() {
        queue.clear();
        for (Problem* p : live) {
            slots[p->slot] = nullptr;
            alloc.release(p->block, p->bytes);
        }
        live.clear();
        rebuild = true;
    }
};

cj_status engine_options(const cj_options* opt, cj_options* o, int* Kreq) {
    cj_options_init(o);
    if (opt) *o = *opt;
    for (int r : o->reserved)
        if (r != 0) return bfail(CJ_ERR_ARG, "reserved option fields must be zero");
    if (o->precision != CJ_PRECISION_F32_REFINE)
        return bfail(CJ_ERR_ARG, "batched and served solves run FP32 sweeps inside FP64 refinement: set precision "
                                 "= CJ_PRECISION_F32_REFINE");
    if (o->method != CJ_METHOD_CHEBYSHEV) return bfail(CJ_ERR_ARG, "batched and served solves use CJ_METHOD_CHEBYSHEV");
    if (o->single_workgroup != 0) return bfail(CJ_ERR_ARG, "single_workgroup applies to single FP64 plans");
    if (o->inner_precision != CJ_INNER_AUTO && o->inner_precision != CJ_INNER_F32)
        return bfail(CJ_ERR_ARG, "batched and served solves run FP32 inner cycles (inner_precision 0 or CJ_INNER_F32)");
    if (o->M != 0 || o->inner_M != 0 || o->h != 0.0)
        return bfail(CJ_ERR_ARG, "M, inner_M and h are per problem and automatic here (must be 0)");
    if (o->max_cycles < 0 || o->tile_rows < 0) return bfail(CJ_ERR_ARG, "negative option");
    *Kreq = o->sweeps_per_launch;
    if (*Kreq != 0 && *Kreq != 2 && *Kreq != 4 && *Kreq != 8)
        return bfail(CJ_ERR_ARG, "sweeps_per_launch must be 0 (automatic), 2, 4 or 8 here");
    return CJ_OK;
}

cj_status check_problem(int nx, int ny, int stencil, double tol) {
    if (stencil != 5 && stencil != 9 && stencil != 17) return bfail(CJ_ERR_ARG, "stencil must be 5, 9 or 17");
    if (nx < 1 || ny < 1 || nx > (1 << 20) || ny > (1 << 20)) return bfail(CJ_ERR_ARG, "nx, ny out of range");
    if (!(tol > 0.0) || !std::isfinite(tol)) return bfail(CJ_ERR_ARG, "tol must be a finite positive number");
    return CJ_OK;
}

void fill_result(const Problem& p, cj_result* r) {
    std::memset(r, 0, sizeof(*r));
    r->status = p.status;
    r->cycles = p.outer;
    r->sweeps = p.sweeps;
    r->rel_residual = p.rr;
    r->floor_estimate = p.status == CJ_STAGNATED ? p.floor_est : 0.0;
    r->seconds = p.t_done - p.t_submit;
}

}  // namespace

struct cj_batch_s {
    Engine eng;
    std::vector<Problem> P;
    size_t total_bytes = 0;
};

struct cj_server_s {
    Engine eng;
    hipStream_t stream = nullptr;
    long long next_ticket = 1;
    std::map<long long, Problem*> all;   // submitted and not yet reported
};

extern "C" {

// ------------------------------------------------------------------ batches

cj_status cj_batch_create(int n, const int* nx, const int* ny, const int* stencil, const double* tol,
                          const cj_options* opt, cj_batch_t* out) {
    if (!out) return bfail(CJ_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || !nx || !ny || !stencil || !tol) return bfail(CJ_ERR_ARG, "n >= 1 and non-NULL arrays required");
    cj_options o;
    int Kreq = 0;
    cj_status st;
    if ((st = engine_options(opt, &o, &Kreq)) != CJ_OK) return st;
    cj_batch_s* b = new (std::nothrow) cj_batch_s();
    if (!b) return bfail(CJ_ERR_NOMEM, "host allocation");
    b->eng.opt = o;
    b->eng.autotune = Kreq == 0 && o.tile_rows == 0;
    b->eng.Kreq = Kreq;
    b->eng.max_outer = o.max_cycles > 0 ? o.max_cycles : 50;
    b->P.resize(n);
    for (int i = 0; i < n; ++i) {
        Problem& p = b->P[i];
        st = check_problem(nx[i], ny[i], stencil[i], tol[i]);
        if (st == CJ_OK) {
            p.nx = nx[i];
            p.ny = ny[i];
            p.stencil = stencil[i];
            p.tol = tol[i];
            st = plan_problem(p, Kreq, o.tile_rows);
        }
        if (st != CJ_OK) {
            const std::string why = cj_last_error();
            delete b;
            return bfail(st, "problem " + std::to_string(i) + ": " + why);
        }
        p.ticket = i;
        b->total_bytes += p.bytes;
    }
    b->eng.budget = b->total_bytes;
    *out = b;
    return CJ_OK;
}

cj_status cj_batch_info(cj_batch_t b, int i, int* M, int* sweeps_per_launch, size_t* workspace_bytes) {
    if (!b) return bfail(CJ_ERR_ARG, "batch is NULL");
    if (i < 0 || i >= (int)b->P.size()) return bfail(CJ_ERR_ARG, "problem index out of range");
    if (M) *M = b->P[i].s.M;
    if (sweeps_per_launch) *sweeps_per_launch = b->P[i].K;
    if (workspace_bytes) *workspace_bytes = b->total_bytes;
    return CJ_OK;
}

cj_status cj_batch_solve(cj_batch_t b, const double* const* f, double* const* u, void* stream_, cj_result* results,
                         cj_batch_stats* stats) {
    const double t0 = now_s();
    if (!b) return bfail(CJ_ERR_ARG, "batch is NULL");
    if (!f || !u) return bfail(CJ_ERR_ARG, "f and u arrays are required");
    const int n = (int)b->P.size();
    for (int i = 0; i < n; ++i) {
        if (!f[i] || !u[i]) return bfail(CJ_ERR_ARG, "problem " + std::to_string(i) + ": NULL f or u");
        if (reinterpret_cast<uintptr_t>(f[i]) % 8 || reinterpret_cast<uintptr_t>(u[i]) % 8)
            return bfail(CJ_ERR_ARG, "problem " + std::to_string(i) + ": misaligned f or u");
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    Engine& E = b->eng;
    E.launches = E.supersteps = 0;
    E.updates = 0.0;
    for (int i = 0; i < n; ++i) {
        Problem& p = b->P[i];
        p.f = f[i];
        p.u = u[i];
        p.state = State::Queued;
        p.status = CJ_OK;
        p.t_submit = t0;
        E.queue.push_back(&p);
    }
    std::vector<Problem*> done;
    cj_status st;
    while (!E.idle()) {
        if ((st = E.step(stream, &done)) != CJ_OK) {
            E.reset_run();
            return st;
        }
    }
    const double secs = now_s() - t0;
    cj_status worst = CJ_OK;
    for (int i = 0; i < n; ++i) {
        const Problem& p = b->P[i];
        if (results) {
            fill_result(p, &results[i]);
            results[i].seconds = secs;
        }
        if (p.status != CJ_OK && worst == CJ_OK) worst = p.status;
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->supersteps = (int)E.supersteps;
        stats->launches = E.launches;
        long long pts = 0;
        for (const Problem& p : b->P) pts += (long long)p.nx * p.ny;
        stats->points = pts;
        stats->updates = E.updates;
        stats->seconds = secs;
        for (const Problem& p : b->P) {
            const int gi = Engine::group_of(p.stencil);
            stats->sweeps_per_launch[gi] = p.K;
            stats->tile_rows[gi] = std::max(stats->tile_rows[gi], p.TK.rows);
        }
    }
    return worst;
}

void cj_batch_destroy(cj_batch_t b) { delete b; }

// ------------------------------------------------------------------ server

cj_status cj_server_create(const cj_options* opt, size_t hbm_budget_bytes, void* stream, cj_server_t* out) {
    if (!out) return bfail(CJ_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (hbm_budget_bytes < ((size_t)1 << 20)) return bfail(CJ_ERR_ARG, "HBM budget below 1 MiB");
    cj_options o;
    int Kreq = 0;
    cj_status st;
    if ((st = engine_options(opt, &o, &Kreq)) != CJ_OK) return st;
    cj_server_s* s = new (std::nothrow) cj_server_s();
    if (!s) return bfail(CJ_ERR_NOMEM, "host allocation");
    s->eng.opt = o;
    s->eng.Kreq = Kreq;
    s->eng.max_outer = o.max_cycles > 0 ? o.max_cycles : 50;
    s->eng.budget = align256(hbm_budget_bytes);
    s->eng.max_supersteps = 32;   // admissions wait at most this many super-steps
    s->stream = static_cast<hipStream_t>(stream);
    *out = s;
    return CJ_OK;
}

cj_status cj_server_submit(cj_server_t s, int nx, int ny, int stencil, double tol, const double* f, double* u,
                           long long* ticket) {
    if (!s || !ticket) return bfail(CJ_ERR_ARG, "server and ticket are required");
    if (!f || !u || reinterpret_cast<uintptr_t>(f) % 8 || reinterpret_cast<uintptr_t>(u) % 8)
        return bfail(CJ_ERR_ARG, "f and u must be non-NULL, 8-byte aligned device pointers");
    cj_status st;
    if ((st = check_problem(nx, ny, stencil, tol)) != CJ_OK) return st;
    Problem* p = new (std::nothrow) Problem();
    if (!p) return bfail(CJ_ERR_NOMEM, "host allocation");
    p->nx = nx;
    p->ny = ny;
    p->stencil = stencil;
    p->tol = tol;
    if ((st = plan_problem(*p, s->eng.Kreq, s->eng.opt.tile_rows)) != CJ_OK) {
        delete p;
        return st;
    }
    if (p->bytes > s->eng.budget) {
        delete p;
        return bfail(CJ_ERR_NOMEM, "request needs more device memory than the whole HBM budget");
    }
    p->f = f;
    p->u = u;
    p->ticket = s->next_ticket++;
    p->t_submit = now_s();
    s->eng.queue.push_back(p);
    s->all[p->ticket] = p;
    *ticket = p->ticket;
    return CJ_OK;
}

cj_status cj_server_step(cj_server_t s, long long* done_tickets, cj_result* done_results, int max_done,
                         int* n_done) {
    if (!s || !n_done) return bfail(CJ_ERR_ARG, "server and n_done are required");
    *n_done = 0;
    if (max_done < 0 || (max_done > 0 && (!done_tickets || !done_results)))
        return bfail(CJ_ERR_ARG, "done arrays are required when max_done > 0");
    std::vector<Problem*> done;
    cj_status st = CJ_OK;
    if (!s->eng.idle()) st = s->eng.step(s->stream, &done);
    if (st != CJ_OK) {
        // fail every request that was in flight; report them as errors
        for (Problem* p : s->eng.live) {
            p->status = st;
            p->state = State::Done;
            p->t_done = now_s();
        }
        for (Problem* p : s->eng.queue) {
            p->status = st;
            p->state = State::Done;
            p->t_done = now_s();
        }
        s->eng.reset_run();
    }
    int k = 0;
    for (auto it = s->all.begin(); it != s->all.end() && k < max_done;) {
        Problem* p = it->second;
        if (p->state != State::Done) {
            ++it;
            continue;
        }
        done_tickets[k] = p->ticket;
        fill_result(*p, &done_results[k]);
        ++k;
        delete p;
        it = s->all.erase(it);
    }
    *n_done = k;
    return st;
}

cj_status cj_server_stats(cj_server_t s, int* active, int* queued, size_t* bytes_in_use) {
    if (!s) return bfail(CJ_ERR_ARG, "server is NULL");
    if (active) *active = (int)s->eng.live.size();
    if (queued) *queued = (int)s->eng.queue.size();
    if (bytes_in_use) *bytes_in_use = s->eng.alloc.used;
    return CJ_OK;
}

void cj_server_destroy(cj_server_t s) {
    if (!s) return;
    if (s->stream && s->eng.device >= 0) (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->all) delete kv.second;
    delete s;
}

}  // extern "C"
