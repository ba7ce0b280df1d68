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

    std::vector<char> taken(n, 0);
    int rc = MPI3D_OK;
    for (int i = 0; i < n && rc == MPI3D_OK; ++i) {
        if (taken[i]) continue;
        int prec_i = 0;
        const StepKind kind = states[i]->next(&prec_i);
        taken[i] = 1;
        if (kind == STEP_NONE) continue;
        mpi3d_state *group[kMaxJobs];
        int ng = 0;
        group[ng++] = states[i];
        for (int j = i + 1; j < n && ng < kMaxJobs; ++j) {
            if (taken[j]) continue;
            int prec_j = 0;
            const StepKind kj = states[j]->next(&prec_j);
            if (kj == kind && prec_j == prec_i && states[j]->pl->line_key == states[i]->pl->line_key) {
                group[ng++] = states[j];
                taken[j] = 1;
            }
        }
        rc = run_group(group, ng, kind, prec_i, st);
        for (int k = 0; k < ng; ++k) ++group[k]->steps;
    }
    if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
    return rc;
}
