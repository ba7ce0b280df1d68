// Internal declarations of libmpi3d: plan layout, kernel argument blocks and
// the launch functions each .hip file provides.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <cstddef>
#include <cstdint>

#include "../../include/mpi3d.h"

namespace mpi3d {

// ---------------------------------------------------------------------------
// Fixed tiling constants of the signal kernels.
//   A pair of waves owns 32 FFL lines (one 32-row MFMA tile); a block of 4
//   pairs owns 128 lines.  Time is consumed in chunks of 32 samples (one MFMA tile of
//   the time dimension).  Columns of the band table come in tiles of 32.
// ---------------------------------------------------------------------------
constexpr int kRowsPerWave = 32;                      // lines per wave pair
constexpr int kWaves = 4;                             // wave pairs per block (two waves per SIMD)
constexpr int kRowsPerBlock = kRowsPerWave * kWaves;
constexpr int kSigThreads = 2 * 64 * kWaves;          // 8 waves
// Wide blocks: 2 wave pairs (one wave per SIMD, so each wave may hold up to
// 512 registers) with up to 22 column tiles per pair, for band tables that
// would otherwise need two column groups and repeat the first contraction.
constexpr int kWidePairs = 2;
constexpr int kChunk = 32;
constexpr int kColTile = 32;
constexpr int kMaxJobs = 16;

// Norm partial slots: every kernel that emits float64 partial sums writes at
// most this many, one per block.
constexpr int kMaxNormParts = 4096;
constexpr int kFwdThreads = 1024;                     // forward projection block
// Rays a forward-projection thread owns: 4 with one slice per texel, 2 with
// two (twice the accumulators and LDS operands per sample).
constexpr int fwd_rays_per_thread(int slices) { return slices == 1 ? 4 : 2; }
// Texels per LDS row of a staged slice: the grid row with a zero border on
// both sides, rounded up to an odd count so that rays a row apart fall in
// different LDS banks.
constexpr int proj_pitch(int nx) { return (nx + 2) | 1; }

// One batch segment of FFL lines sharing the same line tables.
struct SigJob {
    // fwd: projections [lines][nup], or one tensor-PSF pass's symmetric line
    // sums (f32); adj: data [lines][2nb] (f32)
    const void *in;
    float *part;           // partial sums per line, see kernels
    float *row_scale;      // mixed: per-line power-of-two scale (row_scale kernel)
    const float *kf, *ka;  // this job's PSF tables (fp32; its lines' trajectory class)
    const __half *kf16, *ka16;   // (fp16)
    int rows;              // FFL lines of this job
    int tile0;             // first block-row tile of this job in the launch
    int in_stride;         // floats between consecutive input lines
    // mixed: the input lines scaled and rounded to fp16 by the row_scale
    // kernel (bits), zero-padded; input line il starts at in16 + il * in16_stride
    const uint16_t *in16;
    int in16_stride;
    long part_stride;      // floats between consecutive split (x group) partial blocks
    // Job row r is line (r / map_per) * map_nz + map_off + map_step * (r % map_per)
    // of the buffers above (identity: map_per >= rows, map_off 0, map_step 1).
    int map_per, map_nz, map_off, map_step;
};

__host__ __device__ inline long job_line(const SigJob &j, int r)
{
    const int g = r / j.map_per;
    return (long)g * j.map_nz + j.map_off + (long)j.map_step * (r - g * j.map_per);
}

// The band DFT factored over drive cycles (FP32 scans with one PSF table and
// one line group): time t = n1 + P n2 with n1 < P, n2 < C, T = C P, C a
// multiple of 32.  The R distinct residues q of the kept bins mod C take
// 2 zst columns (re/im per residue, zst = R rounded up to 4) of the phase
// sums Y (forward) and Z (adjoint), per 32-line tile [P][2 zst][32 lines]
// floats in the workspace (plus one spare line of P 2 zst floats).  The
// forward's outer sum runs over units of at most 16 bins of one residue; the
// adjoint's over each residue's bins, at most kQMax.
constexpr int kFacWavesFwd = 8;     // waves (32-line tiles) per block of the forward line-tile kernel
                                    // (two per SIMD: one hides the other's wait at the chunk barrier)
constexpr int kFacWavesAdj = 8;     // and of the adjoint line-tile kernel
constexpr int kQMax = 24;           // bins per residue (adjoint outer sum, register operands)
constexpr int kFacInWaves = 8;      // waves of the adjoint outer sum; wave w takes residues w + 8 i
constexpr int kMaxFacSplit = 4;     // forward outer-sum blocks per line tile (40 units each)

struct FacArgs {
    SigJob job;              // input lines, partial sums (part, part_stride), row map; kf / ka: the PSF
                             // tables with their time rows in chunk order (n1, 32-cycle block)
    const float *ef, *ea;    // residue DFT: forward B operand, adjoint A operand (swizzled)
    const float *wf, *wa;    // outer sums: forward per unit, adjoint per residue and 16-phase stage
    const int *uq;           // [U] residue of unit u
    const int *ubin;         // [U][16] bins of unit u (-1: none)
    const int *qbin;         // [R][kQMax] bins of residue q (-1: none)
    const int *qsteps;       // [R] bins of residue q rounded up to 4
    float *y;                // phase sums Y or Z per 32-line tile, [P][yc][32 lines] (for Z the
                             // columns are [re/im][zst]); ylines = 32 tiles; then a spare row of
                             // P yc floats taking the stores that carry nothing
    int ylines;
    int nu, nup, nbp2;
    int P, Pp, cj;           // phases, phases rounded up to 8, 32-cycle blocks per phase (C / 32)
    int yc, zst, R, U, rct;  // yc = 2 zst; rct: 32-column tiles of the residue DFT (1 or 2)
    int nsplit, nsplit_adj;  // phase ranges of the forward and adjoint line-tile kernels
    int usplit;              // unit split of the forward outer sum
    int psplit, zsplit;      // stage ranges of the forward outer sum (partial sums each) and of the
                             // adjoint outer sum (disjoint phases of Z)
    long fwd_part_stride;    // floats between the forward outer sum's partial-sum blocks
    int nzstage;             // 16-phase stages of the adjoint outer sum
    int tiles;               // 32-line tiles of the job
};

struct SigArgs {
    // tables (device); the PSF tables are per job
    const float *ff, *fa;                         // fp32 swizzled DFT tables
    const __half *ff16, *fa16;                    // fp16 swizzled DFT tables
    const float *band_scale;                      // [nbp2] adjoint per-column scale (mixed)
    int nu, nup, nb2, nbp2, nct;                  // sizes (nup, nbp2 padded to 32)
    int nchunks, cps, nsplit, ngroups, gct;       // chunking and column groups
    int pairs;                                    // wave pairs per block (kWaves or kWidePairs)
    int fused;                                    // FP32 tensor PSF in one pass: nup is (R + 1) n_up
    int tail_c0, tail_tpb;                        // FP32 tail split (0: none), see block_work
    int total_tiles;
    int njobs;
    SigJob jobs[kMaxJobs];
};

// ---------------------------------------------------------------------------
// Projection argument block.
// ---------------------------------------------------------------------------
// Forward projection launch: slices per staged texel, row bands, blocks.
struct FwdConfig {
    int slices, band_rows, n_bands, blocks;
};

struct ProjArgs {
    float *rt;                  // projections [M][nz][nup]
    const float *rt_in;         // adjoint input projections [M][nz][nup]
    float *xo;                  // adjoint output volume
    const float *x_sub;         // adjoint epilogue: out = acc + x_add - lambda * x_sub (null = none)
    const float *x_add;         // (null = none)
    double *norm_parts;         // adjoint epilogue: per-block sum of out^2 (null = none)
    double lambda;
    const float2 *cs;           // [M] (cos, sin)
    const float *ax;            // [M][nu] forward x-coordinate bases
    const float *ay;            // [M][nu] forward y-coordinate bases
    int nx, ny, nz, M, nu, nup, nr;
    int band_rows, n_bands;
    int kz, n_zgroups, tiles_x, tiles_y, adj_chunk;
    float half_nr, half_nu, cx, cy;
};

}  // namespace mpi3d

// The plan.  Host copy of the geometry plus device tables and the layout of
// the caller's workspaces.
struct mpi3d_plan {
    int device;
    int nx, ny, nz, M, nu, nt, nr, nb;
    int harm_lo, harm_hi, half_band;
    double P, a, w, op_scale;
    int norm_iters;               // power iterations that set op_scale (0: given)
    int precisions;
    // padded sizes
    int nup;        // n_u padded to 64
    int ntp;        // n_t padded to 32
    int nb2;        // 2*nb real columns
    int nbp2;       // nb2 padded to 32
    int nct;        // nbp2 / 32
    long L;         // lines: the x-drive lines, then the z-drive lines (dual drive)
    long Lx, Lz;    // x-drive lines M*nz; z-drive lines M*nu (0 unless dual drive)
    int drive_axes;
    double a_z;     // z-drive amplitude
    long nvox;
    // signal kernel configuration, per precision: sc[0] FP32 (and the
    // precomposed variant's unused slot), sc[1] MIXED
    struct SigCfg {
        int pairs;                 // wave pairs per block
        int ngroups, gct;          // column groups per line tile, 32-wide column tiles per group
        int cps, nsplit;           // time chunks per split, splits (a tail counting as one)
        int tail_c0, tail_tpb;     // FP32: tail split over chunks [tail_c0, nchunks), tail_tpb tiles a block (0: none)
        int serve_cps, serve_nsplit;   // fixed time split of merged serving launches
    } sc[2];
    // FP32 tensor PSF in one fused pass per line group: the forward's first
    // contraction runs over the R + 1 symmetric line sums of a line laid end
    // to end (a virtual line of nupf = (R + 1) nup samples) against the
    // group's R + 1 tables concatenated per time chunk (kff, kaf: tables
    // table_g .. table_g + R), so the band DFT runs once; the adjoint's second
    // contraction writes all R + 1 offsets of a line at once.  Wide blocks;
    // scf is its launch configuration.
    bool fused = false;
    int nupf = 0;
    SigCfg scf{};
    float *kff = nullptr, *kaf = nullptr;   // [group][chunk][nupf x 32] swizzled like kf / ka
    int nchunks;
    // FP32 band DFT factored over drive cycles (see FacArgs): chosen at plan
    // time when it pays; tables in the plan's allocation
    struct Fac {
        bool on = false;
        int C, P, Pp, cj, R, zst, U, rct, nsplit, nsplit_adj, usplit, psplit, zsplit, nzstage;
        float *kf, *ka, *ef, *ea, *wf, *wa;
        int *uq, *ubin, *qbin, *qsteps;
    } fac;
    uint64_t line_key;             // equal keys <=> identical line tables
    // projection configuration
    mpi3d::FwdConfig fwd32, fwd16;  // forward projection, fp32 and bf16 gathers
    int kz, adj_chunk;
    int max_parts;                 // float64 norm partials a launch may write (>= kMaxNormParts)
    // device tables (one allocation)
    void *tables;
    size_t table_bytes;
    float2 *cs;
    float *ax, *ay;
    // PSF tables kf, ka (kf16, ka16): n_ktab consecutive copies of k_elems
    // elements: one per trajectory class (two under a raster), or per line
    // offset 0..R of each line group under the tensor PSF
    float *kf, *ff, *fa, *ka;
    __half *kf16, *ff16, *fa16, *ka16;
    int n_classes, psf_rows, n_ktab;
    // Line groups of one signal stage, each with its own PSF tables: the
    // trajectory classes of a raster, or the x- and z-drive lines.  Group g's
    // job row r is line (r / per) * gnz + off + step * (r % per).  Under the
    // tensor PSF a group's lines couple to the lines within `coup` of them
    // among the `cper` lines of their angle (x-drive: the z-rows; z-drive: the
    // detector columns), the group's lines starting at `cbase`.  The PSF entry
    // of offset d depends on |d| only (table `table + |d|`), so the signal
    // stage runs one pass per e = 0..coup: pass e contracts table e with the
    // symmetric sums sigma_e(l) = rho(l + e) + rho(l - e) (sigma_0 = rho; a
    // line outside the angle counts as zero), and its adjoint pass hands
    // line l's result to lines l + e and l - e in the reduction.
    struct LineGroup {
        int rows, per, gnz, off, step, table;
        int coup, cper;
        long cbase;
    } groups[2];
    int n_line_groups;
    int pass_r;                   // largest coupling range of the groups
    int n_passes;                 // blocks of split partial sums: pass_r + 1 (e = 0..pass_r)
    size_t k_elems;
    double raster_sweep;
    float *col_scale;     // [nbp2] mixed forward output scale per column
    float *band_scale;    // [nbp2] mixed adjoint input scale per column
    float adj_scale16;    // mixed adjoint output scale
    float *gt = nullptr;  // precomposed: n_ktab line matrices G^T [n_up][2 nb] (row-major)
    float *gta = nullptr; // and their transposes G [2 nb][n_up] (the adjoint's operand)
    size_t gt_elems = 0;  // floats per line matrix
    // operator workspace layout (bytes from ws base)
    size_t ws_rt, ws_part, ws_norm, ws_rowscale, ws_xb, ws_in16, ws_rtb, ws_rtsc, ws_sig, ws_fac, op_ws_bytes;
    int in16_cols;        // halves per fp16 operand line: max(nup, nbp2)
    // solver workspace layout
    size_t sw_op, sw_r, sw_q, sw_s, sw_p, sw_scal, sw_parts, sw_d, sw_g, sw_v, solve_ws_bytes;
};

namespace mpi3d {

// Launchers (return hipError_t of the launch).
// The operator's projection into the workspace lines rt [L][nup]: the x-drive
// lines, then (dual drive) the z-drive lines transposed from them.
hipError_t launch_project(const mpi3d_plan *pl, const float *x, const uint16_t *xb, float *rt,
                          hipStream_t st);
// The operator's backprojection of the workspace lines rt: with the dual drive
// the z-drive lines are first added, transposed, into the x-drive lines (rt
// is modified).
hipError_t launch_backproject(const mpi3d_plan *pl, float *rt, float *xo, const float *x_sub,
                              double lambda, double *norm_parts, int *nparts, hipStream_t st,
                              const float *x_add = nullptr);
// The mixed operator's backprojection: gathers from fp16 lines rtb [Lx][nup]
// with per-line inverse scales rtsc [Lx] (two z-slices per 32-bit LDS word);
// weights and sums in fp32; same epilogue.
hipError_t launch_backproject16(const mpi3d_plan *pl, const uint16_t *rtb, const float *rtsc, float *xo,
                                const float *x_sub, double lambda, double *norm_parts, int *nparts, hipStream_t st,
                                const float *x_add = nullptr);
// Dual drive: fold the z-drive lines of the fp32 lines rt into the x-drive lines.
hipError_t launch_fold_zlines(const mpi3d_plan *pl, float *rt, hipStream_t st);
hipError_t launch_sig_fwd(const mpi3d_plan *pl, int precision, SigArgs &a, hipStream_t st);
hipError_t launch_sig_adj(const mpi3d_plan *pl, int precision, SigArgs &a, hipStream_t st);
int sig_fwd_supported(int nup, int gct, int precision, int pairs);
int sig_adj_supported(int nup, int gct, int precision, int pairs);
int sig_fused_supported(int nupf, int gct);
// Factored band DFT (sigfac.hip): forward writes Y then the job's partial
// sums (psplit blocks of nbp2 columns); adjoint writes Z then nsplit_adj
// splits of nup-column partial sums.
int fac_supported(int nup, int rct, int zst, int cj);
hipError_t launch_fac_fwd(const FacArgs &a, hipStream_t st);
hipError_t launch_fac_adj(const FacArgs &a, hipStream_t st);
// one kernel of those stages: forward PSF contraction + residue DFT, forward
// outer sum, adjoint outer sum, adjoint residue DFT + PSF contraction
enum { kFacFwdInner = 0, kFacFwdOuter = 1, kFacAdjOuter = 2, kFacAdjInner = 3 };
hipError_t launch_fac_part(const FacArgs &a, int part, hipStream_t st);

// Precomposed signal stage (gemm.hip): C[i][j] = alpha sum_q A_i[q] W[q][j]
// (+ beta C[i][j] when beta != 0) for i < n, j < m, q < k, over `batch`
// blocks of rows: row i of block b reads line in0 + b batch_lines +
// i in_step of a (stride lda floats) and writes line out0 + b batch_lines +
// i out_step of c (stride ldc); W is row-major with row stride ldw.
struct LineGemm {
    const float *a;
    long lda;
    const float *w;
    int ldw;
    float *c;
    long ldc;
    int n, m, k;
    int batch;
    long in0, out0, batch_lines;
    int in_step, out_step;
    float alpha, beta;
};
hipError_t launch_line_gemm(const LineGemm &g, hipStream_t st);

// Reductions and vector kernels (vec.hip).  The split reductions sum nparts
// partial blocks; rp describes the tensor PSF's passes among them (npass
// blocks of nparts / npass, pass e = 0..npass-1 for offset e; npass = 1: no
// coupling).  Forward: line l's value is the sum of its passes e <= its
// group's coupling range.  Adjoint: line l collects pass 0 of line l and
// pass e of lines l - e and l + e of its angle.  Row scales (mixed path) are
// those of the lines each pass read: forward [npass][lines], adjoint [lines].
struct RowPasses {
    int npass, nz;         // passes; x-drive lines per angle
    long zbase;            // first z-drive line (lines when there are none)
    int nzc, rx, rz;       // z-drive lines per angle; coupling ranges of x- and z-drive lines
    long lines;            // lines per pass
    int pitch;             // floats between consecutive lines of a partial block
    int fwd;               // 1: forward reduction, 0: adjoint
    int pass_cols;         // fused adjoint (FP32): pass e is columns e pass_cols .. of each line
                           // of every partial block (0: passes are blocks of their own)
};
// The forward passes' inputs: sig[e][l] = rho(l + e) + rho(l - e) within l's
// angle (sig[0] = rho), over nup columns (zero past nu), for e = 0..npass-1
// (zero beyond the line's coupling range); rho has stride in_stride.
// Layout: sig[e][l] starts at e * pass_stride + l * line_stride (passes:
// L nup and nup; the fused pass: nup and (R + 1) nup, a virtual line per l).
hipError_t launch_sym_lines(const float *rho, int in_stride, int nu, int nup, RowPasses rp, float *sig,
                            long pass_stride, long line_stride, hipStream_t st);
hipError_t launch_reduce_fwd(long rows, int nb2, int nbp2, int nparts, long part_stride, const float *part,
                             const float *row_scale, const float *col_scale, double scale, const float *b_sub,
                             float *out, double *norm_parts, int *nnorm, hipStream_t st, RowPasses rp);
hipError_t launch_reduce_lines_strided(long rows, int nu, int nup, int out_stride, int nparts, long part_stride,
                                       const float *part, const float *row_scale, double scale, float *out,
                                       hipStream_t st, RowPasses rp);
// The mixed adjoint's lines [rows][nup] as fp16 with a power-of-two scale per
// line (out16 holds v * s, inv_scale[row] = 1/s), formed from the split sums
// as the reduction above does, or from fp32 lines (lines_in, stride nup).
hipError_t launch_lines16(long rows, int nu, int nup, int nparts, long part_stride, const float *part,
                          const float *row_scale, double scale, RowPasses rp, const float *lines_in, uint16_t *out16,
                          float *inv_scale, hipStream_t st);
hipError_t launch_to_bf16(long n, const float *x, uint16_t *xb, hipStream_t st);
// Per-line power-of-two scales of the fp16 contractions; with out16, also
// the scaled lines rounded to fp16 ([rows][out16_stride] halves, columns
// ncols..out16_cols-1 zero).
hipError_t launch_row_scale(long rows, int ncols, int in_stride, const float *in, const float *col_scale, float *out,
                            uint16_t *out16, int out16_cols, int out16_stride, hipStream_t st);

// CGLS scalar and vector steps.  `scal` holds the solve's float64 scalars.
int scal_slots();
int scal_slot_bad();
int scal_slot_gamma();
int scal_slot_gamma0();
hipError_t launch_scal_init(double *scal, hipStream_t st);
hipError_t launch_alpha(double *scal, const double *parts_q, int nq, const double *parts_p, int np, double lambda,
                        double *hist, int step, hipStream_t st);
hipError_t launch_beta(double *scal, const double *parts_s, int ns, int restart, int first, double *hist, int step,
                       hipStream_t st);
hipError_t launch_update_xr2(float *x, const float *p, float *r, const float *q, long nvox, long ndata,
                             const double *scal, hipStream_t st);
hipError_t launch_update_p2(float *p, const float *s, uint16_t *pb, long n, const double *scal, double *parts_p,
                            int *np_out, int init, hipStream_t st);
hipError_t launch_clamp(float *x, long n, hipStream_t st);
hipError_t launch_fill(float *x, long n, float v, hipStream_t st);
hipError_t launch_copy(float *dst, const float *src, long n, hipStream_t st);
hipError_t launch_norm_record(const double *parts, int n, double *norms, int k, hipStream_t st);
hipError_t launch_scale_by(float *v, const float *z, long n, const double *norms, int k, hipStream_t st);
hipError_t launch_add_to(float *x, const float *d, long n, int clamp, hipStream_t st);
hipError_t launch_momentum(const float *y, const float *g, const float *x, float *x_new, float *y_new, int nx,
                           int ny, int nz, float tau, float taulam, float beta, int fd, int nonneg, double *parts,
                           int *nparts, hipStream_t st);
hipError_t launch_step_norm(double *scal, const double *parts, int n, int first, hipStream_t st);

// Strided projection launchers (public stage entry points use stride n_u).
hipError_t launch_project_strided(const mpi3d_plan *pl, const float *x, float *rt, int out_stride, hipStream_t st);
hipError_t launch_backproject_strided(const mpi3d_plan *pl, const float *rt, int in_stride, float *xo,
                                      const float *x_sub, double lambda, double *norm_parts, int *nparts,
                                      hipStream_t st, const float *x_add = nullptr);

}  // namespace mpi3d

// ---------------------------------------------------------------------------
// Operator and CGLS building blocks shared by the solve and serving paths
// (api.cpp).
// ---------------------------------------------------------------------------
namespace mpi3d {

inline const mpi3d_plan::SigCfg &sig_cfg(const mpi3d_plan *pl, int prec)
{
    if (prec == MPI3D_MIXED) return pl->sc[1];
    return pl->fused ? pl->scf : pl->sc[0];
}
inline bool fused_pass(const mpi3d_plan *pl, int prec) { return pl->fused && prec != MPI3D_MIXED; }

struct OpWs {
    float *rt;        // projections [L][nup]
    float *part;      // split partial sums
    double *norm;     // spare norm partials
    float *rowscale;  // [n_passes][L] per-line scales of the fp16 path (adjoint: [L])
    uint16_t *xb;     // bf16 copy of a volume (mixed path)
    uint16_t *in16;   // [n_passes][L][in16_cols] fp16 operand lines of the mixed signal stage
    float *sig;       // [n_passes][L][nup] tensor PSF: the passes' symmetric line sums (forward)
    uint16_t *rtb;    // [L][nup] fp16 lines of the mixed adjoint (its backprojection gathers)
    float *rtsc;      // [L] their per-line inverse scales
    float *fac;       // phase sums of the factored band DFT (FP32): ceil(L / 32) tiles of
                      // [P][2 zst][32 lines], then a spare line of P 2 zst floats
};
OpWs carve_op(const mpi3d_plan *pl, void *ws);
int check_prec(const mpi3d_plan *pl, int32_t precision);

// One request's lines in a merged signal launch.
struct LineJob {
    const mpi3d_plan *pl;
    const float *in;      // fwd: projections, adj: data
    int in_stride;
    const OpWs *w;
};
// Signal contraction over the lines of n line jobs whose plans have equal line
// tables (line_key), in as few launches as the kernel's job table allows (a
// line job takes one kernel job per trajectory class); `serve` selects the
// fixed time split of merged serving launches.
int sig_forward_jobs(int prec, const LineJob *jobs, int n, bool serve, hipStream_t st);
int sig_adjoint_jobs(int prec, const LineJob *jobs, int n, bool serve, hipStream_t st);

// CGLS state of one solve, advanced in phases so several solves can share the
// signal launches between them (see serve.cpp).  Scalars stay on the device.
struct Cgls {
    const mpi3d_plan *pl = nullptr;
    const float *b = nullptr;
    float *x = nullptr, *r = nullptr, *q = nullptr, *s = nullptr, *p = nullptr;
    double *scal = nullptr, *parts_q = nullptr, *parts_p = nullptr, *parts_s = nullptr;
    double *hist = nullptr;
    uint16_t *pb = nullptr;     // bf16 shadow of p for the mixed operator
    // correction form (mixed refinement): within a sweep x stays fixed and
    // CGLS runs on the correction d, min |A~ d - r0|^2 + lambda |x + d|^2,
    // with r holding -A~ d and the gradient s = g0 + A~^T r - lambda d, where
    // g0 = A^T r0 - lambda x comes from the FP32 operator at the sweep start.
    bool corr = false;
    float *d = nullptr, *g0 = nullptr;
    OpWs w{};
    double lambda = 0.0;
    int nq = 0, np = 0, ns = 0;
    int step = 0;
    bool started = false;
    bool serve = false;         // class-fixed time split (merged launches)

    void init(const mpi3d_plan *plan, const float *b_, float *x_, void *ws, double lam, double *h);
    // restart: r = b - A32 x (or b when x is zero), s = A32^T r - lambda x,
    // gamma = |s|^2, p = s.  Phases around the two signal launches:
    int restart_a(bool x_zero, hipStream_t st);       // projection of x (or r = b)
    int restart_b(bool x_zero, hipStream_t st);       // r = b - (A x)
    int restart_c(hipStream_t st);                    // s (or g0), gamma, p; corr: d = 0, r = 0
    int finish_sweep(bool clamp, hipStream_t st);     // corr: x += d (then clamp); else clamp
    // one iteration: q = A p; alpha; x, r; s = A^T r - lambda x; beta; p
    int iter_a(int prec, hipStream_t st);             // projection of p
    int iter_b(int prec, hipStream_t st);             // q, alpha, x += alpha p, r -= alpha q
    int iter_c(int prec, hipStream_t st);             // s, beta, p
    // whole steps, no merging
    int restart(bool x_zero, hipStream_t st);
    int iterate(int prec, hipStream_t st);
};
int validate_opts(const mpi3d_plan *pl, const mpi3d_solve_opts *o);
// b = A x with the operator workspace at ws (op_ws_bytes, 256-byte aligned).
int forward_ws(const mpi3d_plan *pl, int prec, const float *x, float *b, void *ws, hipStream_t st);
// Records the device address of the no-allocation entry point's scratch array
// on `device` (which must be current); idempotent.
int scratch_setup(int device);
int estimate_op_norm(mpi3d_plan *pl, double rtol, int max_iters, double *norm_out, int *iters_out);
// ||A||_2 with the plan's current scale, by power iteration in caller buffers:
// v, z volumes, y data, norms (max_iters doubles), parts (max_parts doubles),
// w an operator workspace.
int power_norm(const mpi3d_plan *pl, const OpWs &w, float *v, float *z, float *y, double *norms, double *parts,
               double rtol, int max_iters, hipStream_t st, double *norm_out, int *iters_out);

}  // namespace mpi3d
