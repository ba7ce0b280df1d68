// Operator and solver entry points of the C ABI.
//
// A x   = A_DC-per-line( P x )          (Sec. 3.3 definition of A, eq. modelF1)
// A^T y = P^T( Re(A_DC^H y) per line )
// CGLS on eq. nummodel with T = I; see include/mpi3d.h for the recurrences.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

using namespace mpi3d;

namespace {

inline int herr(hipError_t e) { return e == hipSuccess ? MPI3D_OK : MPI3D_EDEVICE; }

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

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        (void)hipGetDevice(&prev);
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) (void)hipSetDevice(prev);
    }
};

int ws_ok(const void *ws, size_t bytes, size_t need)
{
    if (!ws) return MPI3D_EINVAL;
    if ((uintptr_t)ws & 255) return MPI3D_EINVAL;
    if (bytes < need) return MPI3D_ENOMEM;
    return MPI3D_OK;
}

}  // namespace

namespace mpi3d {

OpWs carve_op(const mpi3d_plan *pl, void *ws)
{
    char *b = (char *)ws;
    OpWs w;
    w.rt = (float *)(b + pl->ws_rt);
    w.part = (float *)(b + pl->ws_part);
    w.norm = (double *)(b + pl->ws_norm);
    w.rowscale = (float *)(b + pl->ws_rowscale);
    w.xb = (uint16_t *)(b + pl->ws_xb);
    w.in16 = (uint16_t *)(b + pl->ws_in16);
    w.rtb = (uint16_t *)(b + pl->ws_rtb);
    w.rtsc = (float *)(b + pl->ws_rtsc);
    w.sig = (float *)(b + pl->ws_sig);
    w.fac = (float *)(b + pl->ws_fac);
    return w;
}

int check_prec(const mpi3d_plan *pl, int32_t precision)
{
    if (precision != MPI3D_FP32 && precision != MPI3D_MIXED && precision != MPI3D_PRECOMPOSED) return MPI3D_EINVAL;
    if (!(pl->precisions & (1 << precision))) return MPI3D_EINVAL;
    return MPI3D_OK;
}

static SigArgs sig_args(const mpi3d_plan *pl, int prec, bool serve)
{
    const mpi3d_plan::SigCfg &c = sig_cfg(pl, prec);
    SigArgs a{};
    a.ff = pl->ff; a.fa = pl->fa;
    a.ff16 = pl->ff16; a.fa16 = pl->fa16;
    a.band_scale = pl->band_scale;
    a.nu = pl->nu; a.nup = pl->nup; a.nb2 = pl->nb2; a.nbp2 = pl->nbp2; a.nct = pl->nct;
    if (fused_pass(pl, prec)) {   // virtual lines of (R + 1) nup samples, every one of them used
        a.nu = a.nup = pl->nupf;
        a.fused = 1;
    }
    a.nchunks = pl->nchunks;
    a.cps = serve ? c.serve_cps : c.cps;
    a.nsplit = serve ? c.serve_nsplit : c.nsplit;
    a.ngroups = c.ngroups; a.gct = c.gct; a.pairs = c.pairs;
    a.tail_c0 = serve ? 0 : c.tail_c0;
    a.tail_tpb = serve ? 0 : c.tail_tpb;
    return a;
}

static int nsplit_of(const mpi3d_plan *pl, int prec, bool serve)
{
    const mpi3d_plan::SigCfg &c = sig_cfg(pl, prec);
    return serve ? c.serve_nsplit : c.nsplit;
}
static int rows_per_block(const mpi3d_plan *pl, int prec) { return kRowsPerWave * sig_cfg(pl, prec).pairs; }

// The FP32 signal stage of plans with the band DFT factored over drive cycles.
static bool fac_on(const mpi3d_plan *pl, int prec) { return prec == MPI3D_FP32 && pl->fac.on; }

// Split partial-sum blocks the reductions add: forward (nbp2 columns a line),
// adjoint (nup or nupf columns a line).
static int fwd_parts(const mpi3d_plan *pl, int prec, bool serve)
{
    if (fac_on(pl, prec)) return pl->fac.psplit;
    return (fused_pass(pl, prec) ? 1 : pl->n_passes) * nsplit_of(pl, prec, serve);
}
static int adj_parts(const mpi3d_plan *pl, int prec, bool serve)
{
    if (fac_on(pl, prec)) return pl->fac.nsplit_adj;
    return (fused_pass(pl, prec) ? 1 : pl->n_passes) * nsplit_of(pl, prec, serve) * sig_cfg(pl, prec).ngroups;
}

static FacArgs fac_args(const LineJob &lj)
{
    const mpi3d_plan *pj = lj.pl;
    const mpi3d_plan::Fac &f = pj->fac;
    const mpi3d_plan::LineGroup &lg = pj->groups[0];
    FacArgs a{};
    a.job.in = lj.in;
    a.job.in_stride = lj.in_stride;
    a.job.part = lj.w->part;
    a.job.part_stride = pj->L * pj->nup;
    a.job.kf = f.kf;
    a.job.ka = f.ka;
    a.job.rows = lg.rows;
    a.job.map_per = lg.per;
    a.job.map_nz = lg.gnz;
    a.job.map_off = lg.off;
    a.job.map_step = lg.step;
    a.ef = f.ef; a.ea = f.ea; a.wf = f.wf; a.wa = f.wa;
    a.uq = f.uq; a.ubin = f.ubin; a.qbin = f.qbin; a.qsteps = f.qsteps;
    a.y = lj.w->fac;
    a.ylines = (lg.rows + 31) / 32 * 32;
    a.nu = pj->nu; a.nup = pj->nup; a.nbp2 = pj->nbp2;
    a.P = f.P; a.Pp = f.Pp; a.cj = f.cj;
    a.yc = 2 * f.zst; a.zst = f.zst; a.R = f.R; a.U = f.U; a.rct = f.rct;
    a.nsplit = f.nsplit; a.nsplit_adj = f.nsplit_adj; a.usplit = f.usplit; a.nzstage = f.nzstage;
    a.psplit = f.psplit; a.zsplit = f.zsplit;
    a.fwd_part_stride = pj->L * pj->nbp2;
    a.tiles = (lg.rows + 31) / 32;
    return a;
}

// The kernel jobs of one line job: one per line group (trajectory class of a
// raster, or x- and z-drive lines) and tensor-PSF pass.  Group g holds the
// lines of its map (class c: the lines (m, k) with k % n_classes == c; dual
// drive: the x-drive lines, then the z-drive lines) and its PSF tables.  Pass
// e = 0..coup uses the group's table e and writes the block of split partial
// sums of pass e: forward, it reads the symmetric line sums sigma_e (w->sig,
// or the lines themselves without coupling); adjoint, every pass reads the
// data and the reduction hands pass e of line l to lines l - e and l + e.
static void line_jobs(const LineJob &lj, int prec, bool fwd, bool serve, std::vector<SigJob> &out)
{
    const mpi3d_plan *pj = lj.pl;
    const bool fz = fused_pass(pj, prec);
    const long part_stride = pj->L * (fwd ? pj->nbp2 : (fz ? pj->nupf : pj->nup));
    const long pass_stride =
        (long)nsplit_of(pj, prec, serve) * (fwd ? 1 : sig_cfg(pj, prec).ngroups) * part_stride;
    const bool sym = fwd && pj->n_passes > 1;
    for (int gi = 0; gi < pj->n_line_groups; ++gi) {
        const mpi3d_plan::LineGroup &lg = pj->groups[gi];
        if (fz) {
            // one job: the group's R + 1 tables concatenated; forward input the
            // virtual lines of symmetric sums, adjoint input the data
            SigJob sj{};
            sj.in = fwd ? (const void *)lj.w->sig : (const void *)lj.in;
            sj.in_stride = fwd ? pj->nupf : lj.in_stride;
            sj.part = lj.w->part;
            sj.part_stride = part_stride;
            const size_t ko = (size_t)gi * pj->n_passes * pj->k_elems;
            sj.kf = pj->kff + ko;
            sj.ka = pj->kaf + ko;
            sj.rows = lg.rows;
            sj.map_per = lg.per;
            sj.map_nz = lg.gnz;
            sj.map_off = lg.off;
            sj.map_step = lg.step;
            out.push_back(sj);
            continue;
        }
        for (int e = 0; e <= lg.coup; ++e) {
            SigJob sj{};
            sj.in = sym ? (const void *)(lj.w->sig + (size_t)e * pj->L * pj->nup) : (const void *)lj.in;
            sj.in_stride = sym ? pj->nup : lj.in_stride;
            sj.in16 = lj.w->in16 + (sym ? (size_t)e * pj->L * pj->in16_cols : 0);
            sj.in16_stride = pj->in16_cols;
            sj.part = lj.w->part + e * pass_stride;
            sj.part_stride = part_stride;
            sj.row_scale = lj.w->rowscale;
            const size_t ko = (size_t)(lg.table + e) * pj->k_elems;
            sj.kf = pj->kf + ko;
            sj.ka = pj->ka + ko;
            sj.kf16 = pj->kf16 ? pj->kf16 + ko : nullptr;
            sj.ka16 = pj->ka16 ? pj->ka16 + ko : nullptr;
            sj.rows = lg.rows;
            sj.map_per = lg.per;
            sj.map_nz = lg.gnz;
            sj.map_off = lg.off;
            sj.map_step = lg.step;
            out.push_back(sj);
        }
    }
}

// The tensor PSF's passes as the reductions of one precision see them (a
// fused FP32 forward has a single pass; its adjoint holds every pass in each
// line of its partial sums).
static RowPasses row_passes(const mpi3d_plan *pl, bool fwd, int prec)
{
    RowPasses rp{};
    rp.npass = pl->n_passes;
    rp.nz = pl->nz;
    rp.zbase = pl->drive_axes == 2 ? pl->Lx : pl->L;
    rp.nzc = pl->nu;
    rp.rx = pl->groups[0].coup;
    rp.rz = pl->drive_axes == 2 ? pl->groups[1].coup : 0;
    rp.lines = pl->L;
    rp.pitch = fwd ? pl->nbp2 : pl->nup;
    rp.fwd = fwd ? 1 : 0;
    if (fused_pass(pl, prec)) {
        if (fwd) {
            rp.npass = 1;
        } else {
            rp.pitch = pl->nupf;
            rp.pass_cols = pl->nup;
        }
    }
    return rp;
}

// Mixed signal stage input: per-line scales into w.rowscale and the scaled
// lines as fp16 into w.in16 (forward: projections over n_u columns, zero to
// nup; adjoint: band-scaled data over 2nb columns, zero to nbp2).
static hipError_t row_scale16(const mpi3d_plan *pj, bool fwd, const float *in, int in_stride, const OpWs &w,
                              hipStream_t st)
{
    if (fwd && pj->n_passes > 1)   // every pass's symmetric line sums
        return launch_row_scale(pj->n_passes * pj->L, pj->nu, pj->nup, w.sig, nullptr, w.rowscale, w.in16, pj->nup,
                                pj->in16_cols, st);
    if (fwd)
        return launch_row_scale(pj->L, pj->nu, in_stride, in, nullptr, w.rowscale, w.in16, pj->nup, pj->in16_cols,
                                st);
    return launch_row_scale(pj->L, pj->nb2, in_stride, in, pj->band_scale, w.rowscale, w.in16, pj->nbp2,
                            pj->in16_cols, st);
}

static int sig_jobs(bool fwd, int prec, const LineJob *jobs, int n, bool serve, hipStream_t st)
{
    if (n < 1) return MPI3D_EINVAL;
    const mpi3d_plan *pl = jobs[0].pl;
    if (fac_on(pl, prec)) {
        // one factored stage per line job (its own phase sums in its workspace)
        for (int j = 0; j < n; ++j) {
            if (jobs[j].pl->line_key != pl->line_key || !jobs[j].pl->fac.on) return MPI3D_EINVAL;
            TRY(fwd ? launch_fac_fwd(fac_args(jobs[j]), st) : launch_fac_adj(fac_args(jobs[j]), st));
        }
        return MPI3D_OK;
    }
    SigArgs a = sig_args(pl, prec, serve);
    const int rpb = rows_per_block(pl, prec);
    int tiles = 0, nj = 0;
    auto flush = [&]() -> int {
        if (nj == 0) return MPI3D_OK;
        a.njobs = nj;
        a.total_tiles = tiles;
        TRY(fwd ? launch_sig_fwd(pl, prec, a, st) : launch_sig_adj(pl, prec, a, st));
        nj = 0;
        tiles = 0;
        return MPI3D_OK;
    };
    std::vector<SigJob> kj;
    for (int j = 0; j < n; ++j) {
        const mpi3d_plan *pj = jobs[j].pl;
        if (pj->line_key != pl->line_key) return MPI3D_EINVAL;
        if (fwd && pj->n_passes > 1) {
            // tensor PSF: the symmetric line sums the forward reads -- blocks
            // per pass, or (fused) one virtual line of R + 1 sums per line
            const bool fz = fused_pass(pj, prec);
            TRY(launch_sym_lines(jobs[j].in, jobs[j].in_stride, pj->nu, pj->nup, row_passes(pj, true, MPI3D_MIXED),
                                 jobs[j].w->sig, fz ? pj->nup : pj->L * pj->nup, fz ? pj->nupf : pj->nup, st));
        }
        if (prec == MPI3D_MIXED) {
            // per-line power-of-two scales and the scaled fp16 operand lines
            TRY(row_scale16(pj, fwd, jobs[j].in, jobs[j].in_stride, *jobs[j].w, st));
        }
        kj.clear();
        line_jobs(jobs[j], prec, fwd, serve, kj);
        for (SigJob &sj : kj) {
            if (nj == kMaxJobs) TRYRC(flush());
            sj.tile0 = tiles;
            tiles += (sj.rows + rpb - 1) / rpb;
            a.jobs[nj++] = sj;
        }
    }
    return flush();
}

int sig_forward_jobs(int prec, const LineJob *jobs, int n, bool serve, hipStream_t st)
{
    return sig_jobs(true, prec, jobs, n, serve, st);
}
int sig_adjoint_jobs(int prec, const LineJob *jobs, int n, bool serve, hipStream_t st)
{
    return sig_jobs(false, prec, jobs, n, serve, st);
}

// Split sums -> data: out = c_A * sum (or b_sub - c_A * sum), float64 norms.
static int reduce_forward(const mpi3d_plan *pl, int prec, const OpWs &w, bool serve, float *out, const float *b_sub,
                          double *norm_parts, int *nnorm, hipStream_t st)
{
    const bool mixed = prec == MPI3D_MIXED;
    TRY(launch_reduce_fwd(pl->L, pl->nb2, pl->nbp2, fwd_parts(pl, prec, serve), pl->L * pl->nbp2, w.part,
                          mixed ? w.rowscale : nullptr, mixed ? pl->col_scale : nullptr, pl->op_scale, b_sub, out,
                          norm_parts, nnorm, st, row_passes(pl, true, prec)));
    return MPI3D_OK;
}

// Split sums -> lines (stride out_stride): c_A * Re(A_DC^H y).
static int reduce_adjoint(const mpi3d_plan *pl, int prec, const OpWs &w, bool serve, float *out, int out_stride,
                          hipStream_t st)
{
    const bool mixed = prec == MPI3D_MIXED;
    const double scale = pl->op_scale * (mixed ? (double)pl->adj_scale16 : 1.0);
    const bool fz = fused_pass(pl, prec);
    const int pitch = fz ? pl->nupf : pl->nup;   // floats per line of the partial sums
    TRY(launch_reduce_lines_strided(pl->L, pl->nu, pitch, out_stride, adj_parts(pl, prec, serve),
                                    pl->L * pitch, w.part, mixed ? w.rowscale : nullptr, scale, out, st,
                                    row_passes(pl, false, prec)));
    return MPI3D_OK;
}

// The adjoint's second half after the signal contraction: the split sums
// reduced to lines, then P^T into xo with the optional epilogue
// (xo = acc + x_add - lambda x_sub, float64 norm partials).  The mixed
// operator's lines are fp16 with a power-of-two scale per line (its
// backprojection's 16-bit gathers); with the dual drive they are reduced in
// fp32 first so the z-drive lines can be folded in.
static int lines_to_volume(const mpi3d_plan *pl, int prec, const OpWs &w, bool serve, float *xo, const float *x_sub,
                           double lambda, double *parts, int *nparts, hipStream_t st, const float *x_add = nullptr)
{
    if (prec == MPI3D_MIXED) {
        const RowPasses rp = row_passes(pl, false, prec);
        if (pl->drive_axes == 2) {
            TRYRC(reduce_adjoint(pl, prec, w, serve, w.rt, pl->nup, st));
            TRY(launch_fold_zlines(pl, w.rt, st));
            TRY(launch_lines16(pl->Lx, pl->nu, pl->nup, 0, 0, nullptr, nullptr, 1.0, rp, w.rt, w.rtb, w.rtsc, st));
        } else {
            TRY(launch_lines16(pl->L, pl->nu, pl->nup, adj_parts(pl, prec, serve), pl->L * pl->nup, w.part,
                               w.rowscale, pl->op_scale * (double)pl->adj_scale16, rp,
                               nullptr, w.rtb, w.rtsc, st));
        }
        TRY(launch_backproject16(pl, w.rtb, w.rtsc, xo, x_sub, lambda, parts, nparts, st, x_add));
        return MPI3D_OK;
    }
    TRYRC(reduce_adjoint(pl, prec, w, serve, w.rt, pl->nup, st));
    TRY(launch_backproject(pl, w.rt, xo, x_sub, lambda, parts, nparts, st, x_add));
    return MPI3D_OK;
}

// P x into the workspace lines; the mixed path gathers from a bf16 copy
// (xb, or x converted into the workspace when xb is null).
static int project_into(const mpi3d_plan *pl, int prec, const float *x, const uint16_t *xb, const OpWs &w,
                        hipStream_t st)
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
    return MPI3D_OK;
}

// Precomposed signal stage: data[l] = c_A G_t rho(l) for every line l, or
// lines[l] = c_A sum G_t^T data(l), as float32 MFMA GEMMs (gemm.hip) over
// runs of lines.  One GEMM per line group
// and z-row offset: a group of consecutive lines is one GEMM; a raster class
// (every second z-row) and a tensor-PSF offset (rows shifted within each
// angle) are batched over the angles with the rows' own strides.  Offset 0
// runs first with beta = 0 and covers every line; the other offsets add.
struct GemmRun {
    int n;              // lines per angle (or all lines)
    long in0, out0;     // first input / output line
    int in_step, out_step;   // lines between consecutive rows
    int batch;          // angles (1: one plain GEMM)
    long batch_lines;   // lines between the angles' first rows
    int table;
    float beta;
};

static void gemm_runs(const mpi3d_plan *pl, bool fwd, std::vector<GemmRun> &runs)
{
    for (int gi = 0; gi < pl->n_line_groups; ++gi) {
        const mpi3d_plan::LineGroup &lg = pl->groups[gi];
        const int R = lg.coup;
        for (int k = 0; k <= 2 * R; ++k) {
            const int d = k == 0 ? 0 : (k <= R ? k : R - k);   // 0, 1..R, -1..-R
            GemmRun r{};
            r.table = lg.table + (d < 0 ? -d : d);
            r.beta = d == 0 ? 0.f : 1.f;
            if (lg.gnz == 0 && d == 0) {        // consecutive lines
                r.n = lg.rows;
                r.in0 = r.out0 = lg.off;
                r.in_step = r.out_step = 1;
                r.batch = 1;
            } else if (d == 0) {                // raster class: rows off, off + step, ... of each angle
                r.n = lg.per;
                r.in0 = r.out0 = lg.off;
                r.in_step = r.out_step = lg.step;
                r.batch = pl->M;
                r.batch_lines = lg.gnz;
            } else {                            // tensor offset d: line k reads line k + d of its angle
                // (x-drive: z-rows; z-drive: detector columns).  Forward: out
                // lines [lo, hi) read lines lo + d ...; adjoint: out lines k'
                // gather data lines k' - d
                const int per = lg.cper;
                const int lo = fwd ? std::max(0, -d) : std::max(0, d);
                const int hi = fwd ? std::min(per, per - d) : std::min(per, per + d);
                r.n = hi - lo;
                r.out0 = lg.cbase + lo;
                r.in0 = lg.cbase + (fwd ? lo + d : lo - d);
                r.in_step = r.out_step = 1;
                r.batch = pl->M;
                r.batch_lines = per;
            }
            if (r.n > 0) runs.push_back(r);
        }
    }
}

static int gemm_signal(const mpi3d_plan *pl, bool fwd, const float *in, int ld_in, float *out, int ld_out,
                       hipStream_t st)
{
    if (!pl->gt || !pl->gta) return MPI3D_EINVAL;
    std::vector<GemmRun> runs;
    gemm_runs(pl, fwd, runs);
    for (const GemmRun &r : runs) {
        LineGemm g{};
        // forward: data (2nb per line) = lines (n_u) x G^T [n_up][2nb];
        // adjoint: lines (n_u per line) = data (2nb) x G [2nb][n_up]
        g.a = in;
        g.lda = ld_in;
        g.w = (fwd ? pl->gt : pl->gta) + (size_t)r.table * pl->gt_elems;
        g.ldw = fwd ? pl->nb2 : pl->nup;
        g.c = out;
        g.ldc = ld_out;
        g.n = r.n;
        g.m = fwd ? pl->nb2 : pl->nu;
        g.k = fwd ? pl->nu : pl->nb2;
        g.batch = r.batch;
        g.in0 = r.in0;
        g.out0 = r.out0;
        g.batch_lines = r.batch_lines;
        g.in_step = r.in_step;
        g.out_step = r.out_step;
        g.alpha = (float)pl->op_scale;
        g.beta = r.beta;
        TRY(launch_line_gemm(g, st));
    }
    return MPI3D_OK;
}

static int gemm_signal_fwd(const mpi3d_plan *pl, const float *lines, int ld_in, float *data, hipStream_t st)
{
    return gemm_signal(pl, true, lines, ld_in, data, pl->nb2, st);
}

static int gemm_signal_adj(const mpi3d_plan *pl, const float *data, float *lines, int ld_out, hipStream_t st)
{
    return gemm_signal(pl, false, data, pl->nb2, lines, ld_out, st);
}

static int apply_forward(const mpi3d_plan *pl, int prec, const float *x, float *out, const OpWs &w, hipStream_t st)
{
    if (prec == MPI3D_PRECOMPOSED) {
        TRY(launch_project(pl, x, nullptr, w.rt, st));
        return gemm_signal_fwd(pl, w.rt, pl->nup, out, st);
    }
    TRYRC(project_into(pl, prec, x, nullptr, w, st));
    LineJob j{pl, w.rt, pl->nup, &w};
    TRYRC(sig_forward_jobs(prec, &j, 1, false, st));
    return reduce_forward(pl, prec, w, false, out, nullptr, nullptr, nullptr, st);
}

static int apply_adjoint(const mpi3d_plan *pl, int prec, const float *y, float *xo, const OpWs &w, hipStream_t st)
{
    if (prec == MPI3D_PRECOMPOSED) {
        // the pad columns n_u..n_up of the lines stay as the projection left them (zero)
        TRY(launch_fill(w.rt, pl->L * pl->nup, 0.f, st));
        TRYRC(gemm_signal_adj(pl, y, w.rt, pl->nup, st));
        TRY(launch_backproject(pl, w.rt, xo, nullptr, 0.0, nullptr, nullptr, st));
        return MPI3D_OK;
    }
    LineJob j{pl, y, pl->nb2, &w};
    TRYRC(sig_adjoint_jobs(prec, &j, 1, false, st));
    return lines_to_volume(pl, prec, w, false, xo, nullptr, 0.0, nullptr, nullptr, st);
}

// ---- CGLS -------------------------------------------------------------------

void Cgls::init(const mpi3d_plan *plan, const float *b_, float *x_, void *ws, double lam, double *h)
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
    parts_p = parts_q + pl->max_parts;
    parts_s = parts_p + pl->max_parts;
    const bool mixed = (pl->precisions & (1 << MPI3D_MIXED)) != 0;
    d = mixed ? (float *)(base + pl->sw_d) : nullptr;
    g0 = mixed ? (float *)(base + pl->sw_g) : nullptr;
}

int Cgls::restart_a(bool x_zero, hipStream_t st)
{
    if (!started) TRY(launch_scal_init(scal, st));
    if (x_zero) {
        TRY(launch_copy(r, b, 2 * pl->L * pl->nb, st));
        return MPI3D_OK;
    }
    return project_into(pl, MPI3D_FP32, x, nullptr, w, st);
}

int Cgls::restart_b(bool x_zero, hipStream_t st)
{
    if (x_zero) return MPI3D_OK;
    return reduce_forward(pl, MPI3D_FP32, w, serve, r, b, nullptr, nullptr, st);
}

int Cgls::restart_c(hipStream_t st)
{
    float *grad = corr ? g0 : s;
    TRYRC(lines_to_volume(pl, MPI3D_FP32, w, serve, grad, x, lambda, parts_s, &ns, st));
    TRY(launch_beta(scal, parts_s, ns, 1, started ? 0 : 1, hist, step, st));
    TRY(launch_update_p2(p, grad, pb, pl->nvox, scal, parts_p, &np, 1, st));
    if (corr) {
        TRY(launch_fill(d, pl->nvox, 0.f, st));
        TRY(launch_fill(r, 2 * pl->L * pl->nb, 0.f, st));
    }
    started = true;
    return MPI3D_OK;
}

int Cgls::finish_sweep(bool clamp, hipStream_t st)
{
    if (corr) TRY(launch_add_to(x, d, pl->nvox, clamp ? 1 : 0, st));
    else if (clamp) TRY(launch_clamp(x, pl->nvox, st));
    return MPI3D_OK;
}

int Cgls::iter_a(int prec, hipStream_t st)
{
    return project_into(pl, prec, p, prec == MPI3D_MIXED ? pb : nullptr, w, st);
}

int Cgls::iter_b(int prec, hipStream_t st)
{
    TRYRC(reduce_forward(pl, prec, w, serve, q, nullptr, parts_q, &nq, st));
    TRY(launch_alpha(scal, parts_q, nq, parts_p, np, lambda, hist, step, st));
    TRY(launch_update_xr2(corr ? d : x, p, r, q, pl->nvox, 2 * pl->L * pl->nb, scal, st));
    return MPI3D_OK;
}

int Cgls::iter_c(int prec, hipStream_t st)
{
    TRYRC(lines_to_volume(pl, prec, w, serve, s, corr ? d : x, lambda, parts_s, &ns, st, corr ? g0 : nullptr));
    TRY(launch_beta(scal, parts_s, ns, 0, 0, hist, step, st));
    TRY(launch_update_p2(p, s, pb, pl->nvox, scal, parts_p, &np, 0, st));
    ++step;
    return MPI3D_OK;
}

int Cgls::restart(bool x_zero, hipStream_t st)
{
    TRYRC(restart_a(x_zero, st));
    if (!x_zero) {
        LineJob j{pl, w.rt, pl->nup, &w};
        TRYRC(sig_forward_jobs(MPI3D_FP32, &j, 1, serve, st));
    }
    TRYRC(restart_b(x_zero, st));
    LineJob j{pl, r, pl->nb2, &w};
    TRYRC(sig_adjoint_jobs(MPI3D_FP32, &j, 1, serve, st));
    return restart_c(st);
}

int Cgls::iterate(int prec, hipStream_t st)
{
    TRYRC(iter_a(prec, st));
    LineJob jf{pl, w.rt, pl->nup, &w};
    TRYRC(sig_forward_jobs(prec, &jf, 1, serve, st));
    TRYRC(iter_b(prec, st));
    LineJob ja{pl, r, pl->nb2, &w};
    TRYRC(sig_adjoint_jobs(prec, &ja, 1, serve, st));
    return iter_c(prec, st);
}

// ||A||_2 by power iteration on A^T A with the FP32 operator, from the
// constant unit vector.  Each iteration records |A^T A v| (v of unit norm) in
// float64 on the device; every 10 iterations the host reads the records and
// stops once the estimate moved by at most 10 * rtol (relative) over the last
// 10.  The estimate of lambda_max is nondecreasing, so it approaches ||A||^2
// from below.
int power_norm(const mpi3d_plan *pl, const OpWs &w, float *v, float *z, float *y, double *norms, double *parts,
               double rtol, int max_iters, hipStream_t st, double *norm_out, int *iters_out)
{
    std::vector<double> host(max_iters);
    int rc = MPI3D_OK, done = 0;
    double est = 0.0;
    if (launch_fill(v, pl->nvox, (float)(1.0 / std::sqrt((double)pl->nvox)), st) != hipSuccess) rc = MPI3D_EDEVICE;
    for (int k = 0; rc == MPI3D_OK && k < max_iters; ++k) {
        rc = apply_forward(pl, MPI3D_FP32, v, y, w, st);
        LineJob j{pl, y, pl->nb2, &w};
        if (rc == MPI3D_OK) rc = sig_adjoint_jobs(MPI3D_FP32, &j, 1, false, st);
        int np = 0;
        if (rc == MPI3D_OK) rc = lines_to_volume(pl, MPI3D_FP32, w, false, z, nullptr, 0.0, parts, &np, st);
        if (rc == MPI3D_OK && (launch_norm_record(parts, np, norms, k, st) != hipSuccess ||
                               launch_scale_by(v, z, pl->nvox, norms, k, st) != hipSuccess))
            rc = MPI3D_EDEVICE;
        if (rc != MPI3D_OK) break;
        if ((k + 1) % 10 == 0 || k + 1 == max_iters) {
            if (hipMemcpyAsync(host.data(), norms, sizeof(double) * (k + 1), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                rc = MPI3D_EDEVICE;
                break;
            }
            est = host[k];
            done = k + 1;
            if (!std::isfinite(est) || !(est > 0.0)) {
                rc = MPI3D_ENONFINITE;
                break;
            }
            if (k + 1 >= 20 && std::fabs(est - host[k - 10]) <= 10.0 * rtol * est) break;
        }
    }
    if (rc != MPI3D_OK) return rc;
    *norm_out = std::sqrt(est);
    *iters_out = done;
    return MPI3D_OK;
}

// ||A||_2 of the operator without its global scale (the c_A that makes
// ||A||_2 = 1, Sec. 3.3), in a temporary allocation (plan creation only).
int estimate_op_norm(mpi3d_plan *pl, double rtol, int max_iters, double *norm_out, int *iters_out)
{
    const double keep = pl->op_scale;
    pl->op_scale = 1.0;
    size_t o = 0;
    auto put = [&](size_t bytes) { o = (o + 255) & ~(size_t)255; size_t r = o; o += bytes; return r; };
    const size_t o_ws = put(pl->op_ws_bytes);
    const size_t o_v = put(sizeof(float) * pl->nvox);
    const size_t o_z = put(sizeof(float) * pl->nvox);
    const size_t o_y = put(sizeof(float) * 2 * pl->L * pl->nb);
    const size_t o_n = put(sizeof(double) * max_iters);
    const size_t o_p = put(sizeof(double) * pl->max_parts);
    char *buf = nullptr;
    if (hipMalloc(&buf, o) != hipSuccess) {
        pl->op_scale = keep;
        return MPI3D_ENOMEM;
    }
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        (void)hipFree(buf);
        pl->op_scale = keep;
        return MPI3D_EDEVICE;
    }
    const int rc = power_norm(pl, carve_op(pl, buf + o_ws), (float *)(buf + o_v), (float *)(buf + o_z),
                              (float *)(buf + o_y), (double *)(buf + o_n), (double *)(buf + o_p), rtol, max_iters, st,
                              norm_out, iters_out);
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    (void)hipFree(buf);
    pl->op_scale = keep;
    return rc;
}

// ||T^T T||_2 of the finite differences, closed form: the Kronecker sum of 1D
// reflecting second differences, whose largest eigenvalue per axis of n
// points is 2 - 2 cos(pi (n - 1) / n).
static double fd_normal_norm(const mpi3d_plan *pl)
{
    double t = 0.0;
    for (int n : {pl->nx, pl->ny, pl->nz})
        if (n > 1) t += 2.0 - 2.0 * std::cos(M_PI * (n - 1) / n);
    return t;
}

// The paper's solver (eq. iters): gradient steps of fixed length tau with the
// momentum weight (k-1)/(k+2), each followed by the projection onto x >= 0.
// Four volumes rotate: x_k, x_{k-1}, the momentum point y and the gradient
// g (which the update overwrites with the next y).
static int momentum_solve(const mpi3d_plan *pl, const float *b, float *x, const mpi3d_solve_opts *o, char *ws,
                          double *hist, mpi3d_solve_report *report, hipStream_t st)
{
    OpWs w = carve_op(pl, ws + pl->sw_op);
    float *r = (float *)(ws + pl->sw_r);
    double *scal = (double *)(ws + pl->sw_scal);
    double *parts = (double *)(ws + pl->sw_parts);
    float *bufs[3] = {(float *)(ws + pl->sw_s), (float *)(ws + pl->sw_p), (float *)(ws + pl->sw_v)};
    const double tt = o->reg == MPI3D_REG_FD ? fd_normal_norm(pl) : 1.0;
    double tau = o->tau;
    if (!(tau > 0.0)) {
        // ||A^T A||_2 by power iteration in the workspace (q holds A v)
        double nrm = 0.0;
        int its = 0;
        TRYRC(power_norm(pl, w, bufs[0], bufs[1], (float *)(ws + pl->sw_q), parts + pl->max_parts, parts, 1e-7,
                         std::min(1000, pl->max_parts), st, &nrm, &its));
        tau = 1.0 / (nrm * nrm + o->lambda * tt);
    }
    TRY(launch_scal_init(scal, st));
    float *xk = x, *xprev = bufs[0], *y = bufs[1], *g = bufs[2];
    if (o->x0_is_zero) TRY(launch_fill(x, pl->nvox, 0.f, st));
    TRY(launch_copy(xprev, x, pl->nvox, st));
    TRY(launch_copy(y, x, pl->nvox, st));
    for (int k = 1; k <= o->iters; ++k) {
        // r = b - A y ; g = A^T r = -(A^T (A y - b))
        TRYRC(project_into(pl, MPI3D_FP32, y, nullptr, w, st));
        LineJob jf{pl, w.rt, pl->nup, &w};
        TRYRC(sig_forward_jobs(MPI3D_FP32, &jf, 1, false, st));
        TRYRC(reduce_forward(pl, MPI3D_FP32, w, false, r, b, nullptr, nullptr, st));
        LineJob ja{pl, r, pl->nb2, &w};
        TRYRC(sig_adjoint_jobs(MPI3D_FP32, &ja, 1, false, st));
        TRYRC(lines_to_volume(pl, MPI3D_FP32, w, false, g, nullptr, 0.0, nullptr, nullptr, st));
        // x_{k+1} into x_{k-1}'s buffer, y_{k+1} over g; beta of step k+1
        const float beta = (float)((double)k / (double)(k + 3));
        int np = 0;
        TRY(launch_momentum(y, g, xk, xprev, g, pl->nx, pl->ny, pl->nz, (float)tau, (float)(tau * o->lambda), beta,
                            o->reg == MPI3D_REG_FD ? 1 : 0, o->clamp_every > 0 ? 1 : 0, parts, &np, st));
        TRY(launch_step_norm(scal, parts, np, k == 1 ? 1 : 0, st));
        float *xn = xprev;
        xprev = xk;
        xk = xn;
        float *yn = g;
        g = y;
        y = yn;
    }
    if (xk != x) TRY(launch_copy(x, xk, pl->nvox, st));
    if (report) {
        double sc[16];
        TRY(hipMemcpyAsync(sc, scal, sizeof(double) * scal_slots(), hipMemcpyDeviceToHost, st));
        TRY(hipStreamSynchronize(st));
        report->iters_done = o->iters;
        report->gamma = sc[scal_slot_gamma()];
        report->gamma0 = sc[scal_slot_gamma0()];
        report->status = sc[scal_slot_bad()] != 0.0 ? MPI3D_ENONFINITE : MPI3D_OK;
    }
    (void)hist;
    return MPI3D_OK;
}

int forward_ws(const mpi3d_plan *pl, int prec, const float *x, float *b, void *ws, hipStream_t st)
{
    OpWs w = carve_op(pl, ws);
    return apply_forward(pl, prec, x, b, w, st);
}

int validate_opts(const mpi3d_plan *pl, const mpi3d_solve_opts *o)
{
    if (!o) return MPI3D_EINVAL;
    if (!(o->lambda >= 0.0)) return MPI3D_EINVAL;
    if (o->clamp_every < 0) return MPI3D_EINVAL;
    if (check_prec(pl, o->precision)) return MPI3D_EINVAL;
    if (o->precision == MPI3D_FP32 && o->iters < 0) return MPI3D_EINVAL;
    if (o->precision == MPI3D_MIXED && (o->refine_sweeps < 1 || o->inner_iters < 1)) return MPI3D_EINVAL;
    if (o->precision == MPI3D_MIXED && !(pl->precisions & (1 << MPI3D_FP32))) return MPI3D_EINVAL;
    if (o->precision == MPI3D_PRECOMPOSED) return MPI3D_ENOTSUP;
    if (o->solver != MPI3D_SOLVER_CGLS && o->solver != MPI3D_SOLVER_MOMENTUM) return MPI3D_EINVAL;
    if (o->reg != MPI3D_REG_IDENTITY && o->reg != MPI3D_REG_FD) return MPI3D_EINVAL;
    if (o->solver == MPI3D_SOLVER_CGLS && o->reg != MPI3D_REG_IDENTITY) return MPI3D_ENOTSUP;
    if (o->solver == MPI3D_SOLVER_MOMENTUM && o->precision != MPI3D_FP32) return MPI3D_ENOTSUP;
    if (!std::isfinite(o->tau)) return MPI3D_EINVAL;
    return MPI3D_OK;
}

}  // namespace mpi3d

// ---- operator entry points ---------------------------------------------------

extern "C" int mpi3d_forward(const mpi3d_plan *pl, int32_t precision, const float *x, float *b, void *ws,
                             size_t ws_bytes, void *stream)
{
    if (!pl || !x || !b) return MPI3D_EINVAL;
    TRYRC(check_prec(pl, precision));
    TRYRC(ws_ok(ws, ws_bytes, pl->op_ws_bytes));
    DeviceGuard dg(pl->device);
    OpWs w = carve_op(pl, ws);
    return apply_forward(pl, precision, x, b, w, (hipStream_t)stream);
}

extern "C" int mpi3d_adjoint(const mpi3d_plan *pl, int32_t precision, const float *b, float *x, void *ws,
                             size_t ws_bytes, void *stream)
{
    if (!pl || !x || !b) return MPI3D_EINVAL;
    TRYRC(check_prec(pl, precision));
    TRYRC(ws_ok(ws, ws_bytes, pl->op_ws_bytes));
    DeviceGuard dg(pl->device);
    OpWs w = carve_op(pl, ws);
    return apply_adjoint(pl, precision, b, x, w, (hipStream_t)stream);
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
    if (!pl || !rho || !b) return MPI3D_EINVAL;
    TRYRC(check_prec(pl, precision));
    TRYRC(ws_ok(ws, ws_bytes, pl->op_ws_bytes));
    DeviceGuard dg(pl->device);
    hipStream_t st = (hipStream_t)stream;
    if (precision == MPI3D_PRECOMPOSED) return gemm_signal_fwd(pl, rho, pl->nu, b, st);
    OpWs w = carve_op(pl, ws);
    LineJob j{pl, rho, pl->nu, &w};
    TRYRC(sig_forward_jobs(precision, &j, 1, false, st));
    return reduce_forward(pl, precision, w, false, b, nullptr, nullptr, nullptr, st);
}

extern "C" int mpi3d_signal_adj(const mpi3d_plan *pl, int32_t precision, const float *b, float *rho, void *ws,
                                size_t ws_bytes, void *stream)
{
    if (!pl || !rho || !b) return MPI3D_EINVAL;
    TRYRC(check_prec(pl, precision));
    TRYRC(ws_ok(ws, ws_bytes, pl->op_ws_bytes));
    DeviceGuard dg(pl->device);
    hipStream_t st = (hipStream_t)stream;
    if (precision == MPI3D_PRECOMPOSED) return gemm_signal_adj(pl, b, rho, pl->nu, st);
    OpWs w = carve_op(pl, ws);
    LineJob j{pl, b, pl->nb2, &w};
    TRYRC(sig_adjoint_jobs(precision, &j, 1, false, st));
    return reduce_adjoint(pl, precision, w, false, rho, pl->nu, st);
}

// ---- solve -------------------------------------------------------------------

extern "C" int mpi3d_solve(const mpi3d_plan *pl, const float *b, float *x, const mpi3d_solve_opts *o, void *ws,
                           size_t ws_bytes, double *hist, mpi3d_solve_report *report, void *stream)
{
    if (!pl || !b || !x) return MPI3D_EINVAL;
    TRYRC(validate_opts(pl, o));
    TRYRC(ws_ok(ws, ws_bytes, pl->solve_ws_bytes));
    DeviceGuard dg(pl->device);
    hipStream_t st = (hipStream_t)stream;
    if (o->solver == MPI3D_SOLVER_MOMENTUM) return momentum_solve(pl, b, x, o, (char *)ws, hist, report, st);
    Cgls cg;
    cg.init(pl, b, x, ws, o->lambda, hist);
    if (o->precision == MPI3D_MIXED) {
        cg.pb = cg.w.xb;
        cg.corr = true;
    }
    bool xz = o->x0_is_zero != 0;
    if (xz) TRY(launch_fill(x, pl->nvox, 0.f, st));
    if (o->precision == MPI3D_FP32) {
        TRYRC(cg.restart(xz, st));
        for (int it = 0; it < o->iters; ++it) {
            TRYRC(cg.iterate(MPI3D_FP32, st));
            const bool last = it + 1 == o->iters;
            if (o->clamp_every > 0 && ((it + 1) % o->clamp_every == 0 || last)) {
                TRY(launch_clamp(x, pl->nvox, st));
                if (!last) TRYRC(cg.restart(false, st));
            }
        }
    } else {
        for (int sw = 0; sw < o->refine_sweeps; ++sw) {
            TRYRC(cg.restart(xz && sw == 0, st));
            for (int it = 0; it < o->inner_iters; ++it) TRYRC(cg.iterate(MPI3D_MIXED, st));
            TRYRC(cg.finish_sweep(o->clamp_every > 0, st));
        }
    }
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

// ---- benchmark support ----------------------------------------------------------

extern "C" int mpi3d_time_kernel(const mpi3d_plan *pl, int32_t kernel, int32_t precision, int32_t repeats, float *x,
                                 const float *b, void *ws, size_t ws_bytes, void *stream, float *avg_ms)
{
    if (!pl || !x || !b || !avg_ms || repeats < 1 || kernel < 0 || kernel > 7) return MPI3D_EINVAL;
    TRYRC(check_prec(pl, precision));
    if (kernel >= 4 && !fac_on(pl, precision)) return MPI3D_EINVAL;
    TRYRC(ws_ok(ws, ws_bytes, pl->op_ws_bytes));
    DeviceGuard dg(pl->device);
    hipStream_t st = (hipStream_t)stream;
    OpWs w = carve_op(pl, ws);
    hipEvent_t e0, e1;
    TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MPI3D_EDEVICE;
    }
    // signal kernels: the first launch of a signal stage (every line, one job
    // per trajectory class and z-row offset, up to the job table's size)
    SigArgs a = sig_args(pl, precision, false);
    {
        const bool fwd = kernel == 2;
        const LineJob lj{pl, fwd ? w.rt : b, fwd ? pl->nup : pl->nb2, &w};
        std::vector<SigJob> kj;
        line_jobs(lj, precision, fwd, false, kj);
        a.njobs = std::min((int)kj.size(), kMaxJobs);
        a.total_tiles = 0;
        const int rpb = rows_per_block(pl, precision);
        for (int c = 0; c < a.njobs; ++c) {
            kj[c].tile0 = a.total_tiles;
            a.total_tiles += (kj[c].rows + rpb - 1) / rpb;
            a.jobs[c] = kj[c];
        }
    }
    // the factored band DFT's stages and kernels (FP32 plans that take it)
    const FacArgs fwd_fac = fac_on(pl, precision) ? fac_args(LineJob{pl, w.rt, pl->nup, &w}) : FacArgs{};
    const FacArgs adj_fac = fac_on(pl, precision) ? fac_args(LineJob{pl, b, pl->nb2, &w}) : FacArgs{};
    const bool mixed = precision == MPI3D_MIXED;
    hipError_t err = mixed && kernel == 0 ? launch_to_bf16(pl->nvox, x, w.xb, st) : hipSuccess;
    // the mixed signal kernels read fp16 operand lines: prepared once, untimed
    if (err == hipSuccess && mixed && kernel >= 2)
        err = row_scale16(pl, kernel == 2, kernel == 2 ? w.rt : b, kernel == 2 ? pl->nup : pl->nb2, w, st);
    if (err == hipSuccess) err = hipEventRecord(e0, st);
    for (int i = 0; err == hipSuccess && i < repeats; ++i) {
        switch (kernel) {
        case 0: err = mixed ? launch_project(pl, nullptr, w.xb, w.rt, st) : launch_project(pl, x, nullptr, w.rt, st);
            break;
        case 1:
            err = mixed ? launch_backproject16(pl, w.rtb, w.rtsc, x, nullptr, 0.0, nullptr, nullptr, st)
                        : launch_backproject(pl, w.rt, x, nullptr, 0.0, nullptr, nullptr, st);
            break;
        case 2:
            if (precision == MPI3D_PRECOMPOSED)
                err = gemm_signal_fwd(pl, w.rt, pl->nup, w.part, st) == MPI3D_OK ? hipSuccess : hipErrorUnknown;
            else if (fac_on(pl, precision))
                err = launch_fac_fwd(fwd_fac, st);
            else
                err = launch_sig_fwd(pl, precision, a, st);
            break;
        case 3:
            if (precision == MPI3D_PRECOMPOSED)
                err = gemm_signal_adj(pl, b, w.rt, pl->nup, st) == MPI3D_OK ? hipSuccess : hipErrorUnknown;
            else if (fac_on(pl, precision))
                err = launch_fac_adj(adj_fac, st);
            else
                err = launch_sig_adj(pl, precision, a, st);
            break;
        case 4: err = launch_fac_part(fwd_fac, kFacFwdInner, st); break;
        case 5: err = launch_fac_part(fwd_fac, kFacFwdOuter, st); break;
        case 6: err = launch_fac_part(adj_fac, kFacAdjOuter, st); break;
        default: err = launch_fac_part(adj_fac, kFacAdjInner, st); break;
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
