// Operator and solver entry points of the C ABI.
//
// A x   = A_DC-per-line( P x )          (Sec. 3.3 definition of A, eq. modelF1)
// A^T y = P^T( Re(A_DC^H y) per line )
// CGLS on eq. nummodel with T = I; see include/mpi3d.h for the recurrences.

#include <algorithm>
#include <cstring>
#include <new>

#include "internal.h"

using namespace mpi3d;

namespace {

struct OpWs {
    float *rt;        // projections [L][nup]
    float *part;      // split partials
    double *norm;     // spare norm partials
    float *rowscale;  // [L] mixed per-line scales
    uint16_t *xb;     // mixed bf16 shadow of a volume
};

OpWs carve_op(const mpi3d_plan *pl, void *ws)
{
    char *b = (char *)ws;
    OpWs w;
    w.rt = (float *)(b + pl->ws_rt);
    w.part = (float *)(b + pl->ws_part);
    w.norm = (double *)(b + pl->ws_norm);
    w.rowscale = (float *)(b + pl->ws_rowscale);
    w.xb = (uint16_t *)(b + pl->ws_xb);
    return w;
}

SigArgs sig_args(const mpi3d_plan *pl)
{
    SigArgs a{};
    a.kf = pl->kf; a.ff = pl->ff; a.fa = pl->fa; a.ka = pl->ka;
    a.kf16 = pl->kf16; a.ff16 = pl->ff16; a.fa16 = pl->fa16; a.ka16 = pl->ka16;
    a.band_scale = pl->band_scale;
    a.nu = pl->nu; a.nup = pl->nup; a.nb2 = pl->nb2; a.nbp2 = pl->nbp2; a.nct = pl->nct;
    a.nchunks = pl->nchunks; a.cps = pl->cps; a.nsplit = pl->nsplit; a.ngroups = pl->ngroups; a.gct = pl->gct;
    return a;
}

int check_prec(const mpi3d_plan *pl, int32_t precision)
{
    if (precision != MPI3D_FP32 && precision != MPI3D_MIXED) return MPI3D_EINVAL;
    if (!(pl->precisions & (1 << precision))) return MPI3D_EINVAL;
    return MPI3D_OK;
}

inline int herr(hipError_t e) { return e == hipSuccess ? MPI3D_OK : MPI3D_EDEVICE; }

#define TRY(expr)                                   \
    do {                                            \
        hipError_t _e = (expr);                     \
        if (_e != hipSuccess) return MPI3D_EDEVICE; \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        hipGetDevice(&prev);
        if (prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) hipSetDevice(prev);
    }
};

}  // namespace

namespace mpi3d {

// Lines (stride in_stride) -> data (interleaved complex, L x nb), optionally
// out = b_sub - A_DC rho, with float64 partial norms of `out`.
int signal_forward(const mpi3d_plan *pl, int prec, const float *rho, int in_stride, float *out, const float *b_sub,
                   double *norm_parts, int *nnorm, const OpWs &w, hipStream_t st)
{
    SigArgs a = sig_args(pl);
    a.njobs = 1;
    a.jobs[0].in = rho;
    a.jobs[0].in_stride = in_stride;
    a.jobs[0].part = w.part;
    a.jobs[0].part_stride = pl->L * pl->nbp2;
    a.jobs[0].row_scale = w.rowscale;
    a.jobs[0].rows = (int)pl->L;
    a.jobs[0].tile0 = 0;
    a.total_tiles = (int)((pl->L + kRowsPerBlock - 1) / kRowsPerBlock);
    if (prec == MPI3D_MIXED) TRY(launch_row_scale(pl->L, pl->nu, in_stride, rho, nullptr, w.rowscale, st));
    TRY(launch_sig_fwd(pl, prec, a, st));
    const bool mixed = prec == MPI3D_MIXED;
    TRY(launch_reduce_fwd(pl->L, pl->nb2, pl->nbp2, pl->nsplit, pl->L * pl->nbp2, w.part, mixed ? w.rowscale : nullptr,
                          mixed ? pl->col_scale : nullptr, b_sub, out, norm_parts, nnorm, st));
    return MPI3D_OK;
}

// Data -> lines (stride out_stride): Re(A_DC^H y).
int signal_adjoint(const mpi3d_plan *pl, int prec, const float *y, float *rho, int out_stride, const OpWs &w,
                   hipStream_t st)
{
    SigArgs a = sig_args(pl);
    a.njobs = 1;
    a.jobs[0].in = y;
    a.jobs[0].in_stride = pl->nb2;
    a.jobs[0].part = w.part;
    a.jobs[0].part_stride = pl->L * pl->nup;
    a.jobs[0].row_scale = w.rowscale;
    a.jobs[0].rows = (int)pl->L;
    a.jobs[0].tile0 = 0;
    a.total_tiles = (int)((pl->L + kRowsPerBlock - 1) / kRowsPerBlock);
    if (prec == MPI3D_MIXED) TRY(launch_row_scale(pl->L, pl->nb2, pl->nb2, y, pl->band_scale, w.rowscale, st));
    TRY(launch_sig_adj(pl, prec, a, st));
    const bool mixed = prec == MPI3D_MIXED;
    TRY(launch_reduce_lines_strided(pl->L, pl->nu, pl->nup, out_stride, pl->nsplit * pl->ngroups, pl->L * pl->nup,
                                    w.part, mixed ? w.rowscale : nullptr, mixed ? pl->adj_scale16 : 1.0f, rho, st));
    return MPI3D_OK;
}

// xb: bf16 copy of x for the mixed path (null: convert x into the workspace)
int apply_forward(const mpi3d_plan *pl, int prec, const float *x, float *out, const float *b_sub, double *norm_parts,
                  int *nnorm, const OpWs &w, hipStream_t st, const uint16_t *xb = nullptr)
{
    if (prec == MPI3D_MIXED) {
        if (!xb) {
            TRY(launch_to_bf16(pl->nvox, x, w.xb, st));
            xb = w.xb;
        }
        TRY(launch_project(pl, nullptr, xb, w.rt, st));
    } else {
        TRY(launch_project(pl, x, nullptr, w.rt, st));
    }
    return signal_forward(pl, prec, w.rt, pl->nup, out, b_sub, norm_parts, nnorm, w, st);
}

int apply_adjoint(const mpi3d_plan *pl, int prec, const float *y, float *xo, const float *x_sub, double lambda,
                  double *norm_parts, int *nparts, const OpWs &w, hipStream_t st)
{
    int rc = signal_adjoint(pl, prec, y, w.rt, pl->nup, w, st);
    if (rc) return rc;
    TRY(launch_backproject(pl, w.rt, xo, x_sub, lambda, norm_parts, nparts, st));
    return MPI3D_OK;
}

}  // namespace mpi3d

extern "C" int mpi3d_forward(const mpi3d_plan *pl, int32_t precision, const float *x, float *b, void *ws,
                             size_t ws_bytes, void *stream)
{
    if (!pl || !x || !b || !ws) return MPI3D_EINVAL;
    if (int rc = check_prec(pl, precision)) return rc;
    if (ws_bytes < pl->op_ws_bytes) return MPI3D_ENOMEM;
    if ((uintptr_t)ws & 255) return MPI3D_EINVAL;
    DeviceGuard dg(pl->device);
    OpWs w = carve_op(pl, ws);
    return apply_forward(pl, precision, x, b, nullptr, nullptr, nullptr, w, (hipStream_t)stream);
}

extern "C" int mpi3d_adjoint(const mpi3d_plan *pl, int32_t precision, const float *b, float *x, void *ws,
                             size_t ws_bytes, void *stream)
{
    if (!pl || !x || !b || !ws) return MPI3D_EINVAL;
    if (int rc = check_prec(pl, precision)) return rc;
    if (ws_bytes < pl->op_ws_bytes) return MPI3D_ENOMEM;
    if ((uintptr_t)ws & 255) return MPI3D_EINVAL;
    DeviceGuard dg(pl->device);
    OpWs w = carve_op(pl, ws);
    return apply_adjoint(pl, precision, b, x, nullptr, 0.0, nullptr, nullptr, w, (hipStream_t)stream);
}

extern "C" int mpi3d_project(const mpi3d_plan *pl, const float *x, float *rho, void *stream)
{
    if (!pl || !x || !rho) return MPI3D_EINVAL;
    DeviceGuard dg(pl->device);
    return herr(launch_project_strided(pl, x, rho, pl->nu, (hipStream_t)stream));
}

extern "C" int mpi3d_backproject(const mpi3d_plan *pl, const float *rho, float *x, void *stream)
{
    if (!pl || !x || !rho) return MPI3D_EINVAL;
    DeviceGuard dg(pl->device);
    return herr(launch_backproject_strided(pl, rho, pl->nu, x, nullptr, 0.0, nullptr, nullptr, (hipStream_t)stream));
}

extern "C" int mpi3d_signal_fwd(const mpi3d_plan *pl, int32_t precision, const float *rho, float *b, void *ws,
                                size_t ws_bytes, void *stream)
{
    if (!pl || !rho || !b || !ws) return MPI3D_EINVAL;
    if (int rc = check_prec(pl, precision)) return rc;
    if (ws_bytes < pl->op_ws_bytes) return MPI3D_ENOMEM;
    if ((uintptr_t)ws & 255) return MPI3D_EINVAL;
    DeviceGuard dg(pl->device);
    OpWs w = carve_op(pl, ws);
    return signal_forward(pl, precision, rho, pl->nu, b, nullptr, nullptr, nullptr, w, (hipStream_t)stream);
}

extern "C" int mpi3d_signal_adj(const mpi3d_plan *pl, int32_t precision, const float *b, float *rho, void *ws,
                                size_t ws_bytes, void *stream)
{
    if (!pl || !rho || !b || !ws) return MPI3D_EINVAL;
    if (int rc = check_prec(pl, precision)) return rc;
    if (ws_bytes < pl->op_ws_bytes) return MPI3D_ENOMEM;
    if ((uintptr_t)ws & 255) return MPI3D_EINVAL;
    DeviceGuard dg(pl->device);
    OpWs w = carve_op(pl, ws);
    return signal_adjoint(pl, precision, b, rho, pl->nu, w, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// CGLS
// ---------------------------------------------------------------------------
namespace mpi3d {

struct Cgls {
    const mpi3d_plan *pl;
    const float *b;
    float *x, *r, *q, *s, *p;
    double *scal, *parts_q, *parts_p, *parts_s;
    double *hist;
    uint16_t *pb = nullptr;     // bf16 shadow of p for the mixed operator
    OpWs w;
    double lambda;
    int nq = 0, np = 0, ns = 0;
    int step = 0;
    bool started = false;

    int init(const mpi3d_plan *plan, const float *b_, float *x_, void *ws, double lam, double *h)
    {
        pl = plan;
        b = b_;
        x = x_;
        lambda = lam;
        hist = h;
        char *base = (char *)ws;
        w = carve_op(pl, base + pl->sw_op);
        r = (float *)(base + pl->sw_r);
        q = (float *)(base + pl->sw_q);
        s = (float *)(base + pl->sw_s);
        p = (float *)(base + pl->sw_p);
        scal = (double *)(base + pl->sw_scal);
        parts_q = (double *)(base + pl->sw_parts);
        parts_p = parts_q + kMaxNormParts;
        parts_s = parts_p + kMaxNormParts;
        return MPI3D_OK;
    }

    // r = b - A32 x (or b when x is known zero), s = A32^T r - lambda x,
    // gamma = |s|^2, p = s.
    int restart(hipStream_t st, bool x_zero)
    {
        const long ndata = 2 * pl->L * pl->nb;
        if (!started) TRY(launch_scal_init(scal, st));
        if (x_zero) {
            TRY(launch_copy(r, b, ndata, st));
        } else {
            int rc = apply_forward(pl, MPI3D_FP32, x, r, b, nullptr, nullptr, w, st);
            if (rc) return rc;
        }
        int rc = apply_adjoint(pl, MPI3D_FP32, r, s, x, lambda, parts_s, &ns, w, st);
        if (rc) return rc;
        TRY(launch_beta(scal, parts_s, ns, 1, started ? 0 : 1, hist, step, st));
        TRY(launch_update_p2(p, s, pb, pl->nvox, scal, parts_p, &np, 1, st));
        started = true;
        return MPI3D_OK;
    }

    int iterate(int prec, hipStream_t st)
    {
        const long ndata = 2 * pl->L * pl->nb;
        int rc = apply_forward(pl, prec, p, q, nullptr, parts_q, &nq, w, st, prec == MPI3D_MIXED ? pb : nullptr);
        if (rc) return rc;
        TRY(launch_alpha(scal, parts_q, nq, parts_p, np, lambda, hist, step, st));
        TRY(launch_update_xr2(x, p, r, q, pl->nvox, ndata, scal, st));
        rc = apply_adjoint(pl, prec, r, s, x, lambda, parts_s, &ns, w, st);
        if (rc) return rc;
        TRY(launch_beta(scal, parts_s, ns, 0, 0, hist, step, st));
        TRY(launch_update_p2(p, s, pb, pl->nvox, scal, parts_p, &np, 0, st));
        ++step;
        return MPI3D_OK;
    }
};

int validate_opts(const mpi3d_plan *pl, const mpi3d_solve_opts *o)
{
    if (!o) return MPI3D_EINVAL;
    if (!(o->lambda >= 0.0)) return MPI3D_EINVAL;
    if (o->clamp_every < 0) return MPI3D_EINVAL;
    if (check_prec(pl, o->precision)) return MPI3D_EINVAL;
    if (o->precision == MPI3D_FP32 && o->iters < 0) return MPI3D_EINVAL;
    if (o->precision == MPI3D_MIXED && (o->refine_sweeps < 1 || o->inner_iters < 1)) return MPI3D_EINVAL;
    return MPI3D_OK;
}

}  // namespace mpi3d

extern "C" int mpi3d_solve(const mpi3d_plan *pl, const float *b, float *x, const mpi3d_solve_opts *o, void *ws,
                           size_t ws_bytes, double *hist, mpi3d_solve_report *report, void *stream)
{
    if (!pl || !b || !x || !ws) return MPI3D_EINVAL;
    if (int rc = validate_opts(pl, o)) return rc;
    if (ws_bytes < pl->solve_ws_bytes) return MPI3D_ENOMEM;
    if ((uintptr_t)ws & 255) return MPI3D_EINVAL;
    DeviceGuard dg(pl->device);
    hipStream_t st = (hipStream_t)stream;
    Cgls cg;
    cg.init(pl, b, x, ws, o->lambda, hist);
    if (o->precision == MPI3D_MIXED) cg.pb = cg.w.xb;
    bool xz = o->x0_is_zero != 0;
    if (xz) TRY(launch_fill(x, pl->nvox, 0.f, st));
    int rc = MPI3D_OK;
    if (o->precision == MPI3D_FP32) {
        rc = cg.restart(st, xz);
        for (int it = 0; !rc && it < o->iters; ++it) {
            rc = cg.iterate(MPI3D_FP32, st);
            const bool last = it + 1 == o->iters;
            if (!rc && o->clamp_every > 0 && ((it + 1) % o->clamp_every == 0 || last)) {
                TRY(launch_clamp(x, pl->nvox, st));
                if (!last) rc = cg.restart(st, false);
            }
        }
    } else {
        for (int sw = 0; !rc && sw < o->refine_sweeps; ++sw) {
            rc = cg.restart(st, xz && sw == 0);
            for (int it = 0; !rc && it < o->inner_iters; ++it) rc = cg.iterate(MPI3D_MIXED, st);
            if (!rc && o->clamp_every > 0) TRY(launch_clamp(x, pl->nvox, st));
        }
    }
    if (rc) return rc;
    if (report) {
        double sc[16];
        TRY(hipMemcpyAsync(sc, cg.scal, sizeof(double) * scal_slots(), hipMemcpyDeviceToHost, st));
        TRY(hipStreamSynchronize(st));
        report->iters_done = cg.step;
        report->gamma = sc[scal_slot_gamma()];
        report->gamma0 = sc[scal_slot_gamma0()];
        report->status = sc[scal_slot_bad()] != 0.0 ? MPI3D_ENONFINITE : MPI3D_OK;
    }
    return MPI3D_OK;
}

extern "C" int mpi3d_time_kernel(const mpi3d_plan *pl, int32_t kernel, int32_t precision, int32_t repeats, float *x,
                                 const float *b, void *ws, size_t ws_bytes, void *stream, float *avg_ms)
{
    if (!pl || !x || !b || !ws || !avg_ms || repeats < 1 || kernel < 0 || kernel > 3) return MPI3D_EINVAL;
    if (int rc = check_prec(pl, precision)) return rc;
    if (ws_bytes < pl->op_ws_bytes) return MPI3D_ENOMEM;
    if ((uintptr_t)ws & 255) return MPI3D_EINVAL;
    DeviceGuard dg(pl->device);
    hipStream_t st = (hipStream_t)stream;
    OpWs w = carve_op(pl, ws);
    hipEvent_t e0, e1;
    TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MPI3D_EDEVICE;
    }
    SigArgs a = sig_args(pl);
    a.njobs = 1;
    a.jobs[0].row_scale = w.rowscale;
    a.jobs[0].rows = (int)pl->L;
    a.jobs[0].tile0 = 0;
    a.jobs[0].part = w.part;
    a.total_tiles = (int)((pl->L + kRowsPerBlock - 1) / kRowsPerBlock);
    if (kernel == 2) {
        a.jobs[0].in = w.rt;
        a.jobs[0].in_stride = pl->nup;
        a.jobs[0].part_stride = pl->L * pl->nbp2;
    } else if (kernel == 3) {
        a.jobs[0].in = b;
        a.jobs[0].in_stride = pl->nb2;
        a.jobs[0].part_stride = pl->L * pl->nup;
    }
    hipError_t err = hipEventRecord(e0, st);
    for (int i = 0; err == hipSuccess && i < repeats; ++i) {
        switch (kernel) {
        case 0: err = launch_project(pl, x, nullptr, w.rt, st); break;
        case 1: err = launch_backproject(pl, w.rt, x, nullptr, 0.0, nullptr, nullptr, st); break;
        case 2: err = launch_sig_fwd(pl, precision, a, st); break;
        default: err = launch_sig_adj(pl, precision, a, st); break;
        }
    }
    if (err == hipSuccess) err = hipEventRecord(e1, st);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return MPI3D_EDEVICE;
    *avg_ms = ms / repeats;
    return MPI3D_OK;
}
