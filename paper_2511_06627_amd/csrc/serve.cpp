// Serving: CGLS solves advanced one step at a time, with the signal
// contractions of several requests merged into shared launches.
//
// A state walks the same schedule as mpi3d_solve (restarts, iterations,
// clamps, refinement sweeps), one step per mpi3d_batch_step.  A batch step
// groups the given states by (line class, step kind, precision); inside a
// group every per-request kernel (projections, reductions, vector updates,
// float64 scalars) runs as before, while the two signal contractions -- the
// bulk of the work -- run once for the whole group with one job per request.
// Merged launches use a time split fixed per line class, and a line's
// arithmetic depends only on its own data and the class tables, so a
// request's iterates are bitwise the same whether it runs alone or batched.

#include <mutex>
#include <new>
#include <vector>

#include "internal.h"

using namespace mpi3d;

namespace {

enum StepKind { STEP_NONE = 0, STEP_RESTART = 1, STEP_ITER = 2 };

#define TRY(expr)                                   \
    do {                                            \
        hipError_t _e = (expr);                     \
        if (_e != hipSuccess) return MPI3D_EDEVICE; \
    } while (0)

#define TRYRC(expr)               \
    do {                          \
        int _rc = (expr);         \
        if (_rc) return _rc;      \
    } while (0)

}  // namespace

struct mpi3d_state {
    const mpi3d_plan *pl;
    mpi3d_solve_opts o;
    Cgls cg;
    bool need_restart = true;
    bool first = true;
    bool done = false;
    int it = 0;       // FP32 iterations done
    int sweep = 0;    // MIXED sweeps done
    int inner = 0;    // iterations done in the current sweep
    int steps = 0;    // batch steps taken

    StepKind next(int *prec) const
    {
        if (done) return STEP_NONE;
        if (need_restart) {
            *prec = MPI3D_FP32;
            return STEP_RESTART;
        }
        *prec = o.precision;
        return STEP_ITER;
    }

    // bookkeeping after an iteration; may enqueue the nonnegativity clamp
    int after_iter(hipStream_t st)
    {
        if (o.precision == MPI3D_FP32) {
            ++it;
            const bool last = it == o.iters;
            if (o.clamp_every > 0 && (it % o.clamp_every == 0 || last)) {
                TRY(launch_clamp(cg.x, pl->nvox, st));
                if (!last) need_restart = true;
            }
            if (last) done = true;
        } else {
            ++inner;
            if (inner == o.inner_iters) {
                TRYRC(cg.finish_sweep(o.clamp_every > 0, st));
                inner = 0;
                ++sweep;
                if (sweep == o.refine_sweeps) done = true;
                else need_restart = true;
            }
        }
        return MPI3D_OK;
    }

    void after_restart()
    {
        need_restart = false;
        first = false;
        if (o.precision == MPI3D_FP32 && o.iters == 0) done = true;
    }
};

extern "C" int mpi3d_state_create(const mpi3d_plan *pl, const float *b, float *x, const mpi3d_solve_opts *o, void *ws,
                                  size_t ws_bytes, mpi3d_state **out)
{
    if (!out) return MPI3D_EINVAL;
    *out = nullptr;
    if (!pl || !b || !x || !ws) return MPI3D_EINVAL;
    TRYRC(validate_opts(pl, o));
    if (o->solver != MPI3D_SOLVER_CGLS) return MPI3D_ENOTSUP;   // states step CGLS schedules
    if ((uintptr_t)ws & 255) return MPI3D_EINVAL;
    if (ws_bytes < pl->solve_ws_bytes) return MPI3D_ENOMEM;
    mpi3d_state *s = new (std::nothrow) mpi3d_state();
    if (!s) return MPI3D_ENOMEM;
    s->pl = pl;
    s->o = *o;
    s->cg.init(pl, b, x, ws, o->lambda, nullptr);
    s->cg.serve = true;
    if (o->precision == MPI3D_MIXED) {
        s->cg.pb = s->cg.w.xb;
        s->cg.corr = true;
    }
    *out = s;
    return MPI3D_OK;
}

extern "C" void mpi3d_state_destroy(mpi3d_state *s) { delete s; }

extern "C" int mpi3d_state_progress(const mpi3d_state *s, int32_t *iters_done, int32_t *done)
{
    if (!s) return MPI3D_EINVAL;
    if (iters_done) *iters_done = s->cg.step;
    if (done) *done = s->done ? 1 : 0;
    return MPI3D_OK;
}

namespace {

// One step for a group of states of one line class, kind and precision.
int run_group(mpi3d_state *const *g, int n, StepKind kind, int prec, hipStream_t st)
{
    LineJob jobs[kMaxJobs];
    if (kind == STEP_RESTART) {
        int nf = 0;
        for (int i = 0; i < n; ++i) {
            mpi3d_state *s = g[i];
            const bool xz = s->first && s->o.x0_is_zero;
            if (xz) TRY(launch_fill(s->cg.x, s->pl->nvox, 0.f, st));
            TRYRC(s->cg.restart_a(xz, st));
            if (!xz) jobs[nf++] = LineJob{s->pl, s->cg.w.rt, s->pl->nup, &s->cg.w};
        }
        if (nf) TRYRC(sig_forward_jobs(MPI3D_FP32, jobs, nf, true, st));
        for (int i = 0; i < n; ++i) {
            mpi3d_state *s = g[i];
            TRYRC(s->cg.restart_b(s->first && s->o.x0_is_zero, st));
            jobs[i] = LineJob{s->pl, s->cg.r, s->pl->nb2, &s->cg.w};
        }
        TRYRC(sig_adjoint_jobs(MPI3D_FP32, jobs, n, true, st));
        for (int i = 0; i < n; ++i) {
            TRYRC(g[i]->cg.restart_c(st));
            g[i]->after_restart();
        }
        return MPI3D_OK;
    }
    for (int i = 0; i < n; ++i) {
        mpi3d_state *s = g[i];
        TRYRC(s->cg.iter_a(prec, st));
        jobs[i] = LineJob{s->pl, s->cg.w.rt, s->pl->nup, &s->cg.w};
    }
    TRYRC(sig_forward_jobs(prec, jobs, n, true, st));
    for (int i = 0; i < n; ++i) {
        mpi3d_state *s = g[i];
        TRYRC(s->cg.iter_b(prec, st));
        jobs[i] = LineJob{s->pl, s->cg.r, s->pl->nb2, &s->cg.w};
    }
    TRYRC(sig_adjoint_jobs(prec, jobs, n, true, st));
    for (int i = 0; i < n; ++i) {
        TRYRC(g[i]->cg.iter_c(prec, st));
        TRYRC(g[i]->after_iter(st));
    }
    return MPI3D_OK;
}

}  // namespace

namespace {

// Groups of one batch step touch disjoint states (each request owns its
// data, volume and workspace; plan tables are only read), so they may run
// concurrently: group g goes to stream g % kServeStreams of the step, stream
// 0 being the caller's and the others a per-device pool of non-blocking
// streams at the default priority.  The pool streams first wait for the
// caller's stream (an event recorded at the step's start) and the caller's
// stream then waits for each of them (an event recorded after its last
// group), so to the caller the step is ordered on `stream` as before.  Small
// requests, whose launches fill few CUs, then overlap with other classes.
constexpr int kServeStreams = 4;

struct StreamPool {
    bool ready = false, failed = false;
    hipStream_t s[kServeStreams - 1] = {};
    hipEvent_t start = nullptr;
    hipEvent_t done[kServeStreams - 1] = {};
};

std::mutex g_pool_mu;
StreamPool g_pools[64];

// The current device's pool (created on first use), or null when it cannot
// be created: the step then runs on the caller's stream alone.
StreamPool *stream_pool(int dev)
{
    if (dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    StreamPool &p = g_pools[dev];
    if (p.failed) return nullptr;
    if (!p.ready) {
        bool ok = hipEventCreateWithFlags(&p.start, hipEventDisableTiming) == hipSuccess;
        for (int k = 0; ok && k < kServeStreams - 1; ++k)
            ok = hipStreamCreateWithFlags(&p.s[k], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&p.done[k], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            p.failed = true;
            return nullptr;
        }
        p.ready = true;
    }
    return &p;
}

}  // namespace

extern "C" int mpi3d_batch_step(mpi3d_state *const *states, int32_t n, void *stream)
{
    if (n < 0 || (n > 0 && !states)) return MPI3D_EINVAL;
    if (n == 0) return MPI3D_OK;
    const int dev = states[0] ? states[0]->pl->device : -1;
    for (int i = 0; i < n; ++i) {
        if (!states[i]) return MPI3D_EINVAL;
        if (states[i]->pl->device != dev) return MPI3D_EINVAL;
        for (int j = 0; j < i; ++j)
            if (states[j] == states[i]) return MPI3D_EINVAL;   // a state steps once per call
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != dev) (void)hipSetDevice(dev);
    hipStream_t st = (hipStream_t)stream;

    // the step's groups: states of one line class, step kind and precision
    struct Group {
        std::vector<mpi3d_state *> s;
        StepKind kind;
        int prec;
    };
    std::vector<Group> groups;
    std::vector<char> taken(n, 0);
    for (int i = 0; i < n; ++i) {
        if (taken[i]) continue;
        int prec_i = 0;
        const StepKind kind = states[i]->next(&prec_i);
        taken[i] = 1;
        if (kind == STEP_NONE) continue;
        Group g{{states[i]}, kind, prec_i};
        for (int j = i + 1; j < n && (int)g.s.size() < kMaxJobs; ++j) {
            if (taken[j]) continue;
            int prec_j = 0;
            const StepKind kj = states[j]->next(&prec_j);
            if (kj == kind && prec_j == prec_i && states[j]->pl->line_key == states[i]->pl->line_key) {
                g.s.push_back(states[j]);
                taken[j] = 1;
            }
        }
        groups.push_back(std::move(g));
    }

    StreamPool *pool = groups.size() > 1 ? stream_pool(dev) : nullptr;
    const int nst = pool ? std::min<int>(kServeStreams, (int)groups.size()) : 1;
    int rc = MPI3D_OK;
    if (nst > 1) {
        if (hipEventRecord(pool->start, st) != hipSuccess) rc = MPI3D_EDEVICE;
        for (int k = 1; rc == MPI3D_OK && k < nst; ++k)
            if (hipStreamWaitEvent(pool->s[k - 1], pool->start, 0) != hipSuccess) rc = MPI3D_EDEVICE;
    }
    for (size_t gi = 0; gi < groups.size() && rc == MPI3D_OK; ++gi) {
        Group &g = groups[gi];
        const int k = (int)(gi % nst);
        rc = run_group(g.s.data(), (int)g.s.size(), g.kind, g.prec, k == 0 ? st : pool->s[k - 1]);
        for (mpi3d_state *s : g.s) ++s->steps;
    }
    // join: the caller's stream waits for every pool stream used (also after
    // a failure, so nothing enqueued stays unordered)
    for (int k = 1; k < nst; ++k) {
        if (hipEventRecord(pool->done[k - 1], pool->s[k - 1]) != hipSuccess ||
            hipStreamWaitEvent(st, pool->done[k - 1], 0) != hipSuccess)
            rc = rc ? rc : MPI3D_EDEVICE;
    }
    if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
    return rc;
}
