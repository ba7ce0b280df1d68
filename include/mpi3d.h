/*
 * mpi3d.h -- C ABI of libmpi3d.so: the compressed 3D field-free-line (FFL)
 * MPI forward operator A, its adjoint A^T and the Tikhonov solve, on one
 * AMD Instinct MI355X (gfx950).
 *
 * The operator (paper Sec. 3.3, the definition of A; eq. modelF1):
 *
 *   A = blockdiag(A_DC, ..., A_DC) [P_theta1; ...; P_thetaM]
 *
 *   P_theta   parallel-beam projection of the volume along the FFL direction
 *             rotated by theta about z (Sec. 2.2, eq. qtheta, eq. ptheta2,
 *             eq. ptheta1): unit-step bilinear ray sums inside each z-slice.
 *   A_DC      compressed FFL signal model S D_Gamma F V E H B (eq. DCmodel):
 *             per FFL line, the time signal
 *               s_n = c_A v_n sum_p rho_theta[p] L'((xi_n - u_p)/w) / w
 *             (eq. reals0 with the collinear PSF of Appendix B eq. PSF,
 *             xi_n = a sin(2 pi P n / T), v_n = xi'), followed by the unitary
 *             DFT of Appendix A (+i sign, T^{-1/2}) restricted to the kept
 *             harmonic bands (eq. bcompress) and the receive transfer
 *             function D_Gamma on those bins.
 *
 * and the objective solved (Sec. 3.3, eq. nummodel, with T = I):
 *
 *   min_x ||A x - b||^2 + lambda ||x||^2.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Status: 0 on success, a negative MPI3D_E* code otherwise.  Functions
 *   never throw, abort or print.  Argument errors are detected on the host
 *   before anything is enqueued (MPI3D_EINVAL); a HIP error surfaces as
 *   MPI3D_EDEVICE.
 * - Pointers named *_dev are device pointers on the plan's device; all other
 *   pointers are host pointers.  The caller owns every buffer it passes; the
 *   library keeps no caller pointer beyond the call, except that a serving
 *   state (mpi3d_state_create) keeps b, x and the workspace until destroyed.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   Work is enqueued asynchronously on it; the call returns before the GPU
 *   finishes unless stated otherwise.
 * - No entry point allocates device memory except mpi3d_plan_create (its
 *   tables).  Operator and solver scratch comes from a caller workspace whose
 *   size mpi3d_plan_query reports, so an HBM footprint is known up front
 *   (mpi3d_forward_noalloc uses the library's static scratch array instead).
 * - Layouts.  Volume x: float32 [nz][ny][nx], x index fastest.  Data b:
 *   complex64 as interleaved float pairs (re, im), [n_angles][nz][n_bins];
 *   kept bins ordered harmonic-major, offset-minor (see mpi3d_geometry).
 *   The volume is real, so the adjoint returns Re(A^H b) (the exact transpose
 *   in the real inner product <u, v> = Re(u^H v)).
 * - Thread safety.  A plan is read-only after creation and may be used from
 *   several host threads and streams at once, provided each concurrent call
 *   has its own workspace.
 */
#ifndef MPI3D_H
#define MPI3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MPI3D_OK = 0,
    MPI3D_EINVAL = -1,     /* bad argument (sizes, pointers, bins, precision) */
    MPI3D_ENOMEM = -2,     /* device allocation failed (plan tables), or workspace too small */
    MPI3D_EDEVICE = -3,    /* a HIP runtime call failed */
    MPI3D_ENOTSUP = -4,    /* geometry outside the compiled kernel variants */
    MPI3D_ENONFINITE = -5  /* a solver norm became NaN or infinite */
};

/* Operator precision.  FP32: projection in fp32, signal contractions on fp32
 * MFMA; with one PSF table and one line group the plan may factor the band
 * DFT over drive cycles (Appendix A's sum regrouped exactly over t = n1 + P n2,
 * T = C P: a C-point DFT at the residues of the kept bins mod C, then a P-point
 * sum per bin; mpi3d_plan_info.dft_cycles), when that needs less MFMA work --
 * the same operator with the sums in another order.  MIXED: the projection gathers a bf16 copy of the volume, the
 * backprojection fp16 lines with a power-of-two scale per line, and the
 * signal contractions run on fp16 MFMA with fp32 accumulation, per-line
 * power-of-two scaling and per-harmonic-band scaling.  PRECOMPOSED:
 * the lines of one PSF table share one trajectory, so A_DC = S D_Gamma F V E H B
 * is one real 2n_bins x n_u matrix G per table (per raster sweep direction,
 * tensor-PSF row offset, or drive axis); the plan forms G = F^T K once in
 * float64 on the host, and the signal stage becomes float32 MFMA GEMMs of
 * the projections with each G (or its transpose), batched over the angles
 * where a table's lines are strided or shifted -- the same operator without
 * forming time signals, about (n_t (n_u + 2 n_bins)) / (2 n_bins n_u) times
 * fewer flops.  PRECOMPOSED serves mpi3d_forward, mpi3d_adjoint,
 * mpi3d_signal_* and mpi3d_time_kernel; mpi3d_solve and serving states reject
 * it (MPI3D_ENOTSUP). */
enum { MPI3D_FP32 = 0, MPI3D_MIXED = 1, MPI3D_PRECOMPOSED = 2 };

/*
 * Scan geometry and physics (copied at plan creation).
 *
 * Volume grid: voxel (i, j, k) centred at (i - (nx-1)/2, j - (ny-1)/2) in the
 * xy-plane of slice k; the FFL rotates about z (Sec. 2.2), so FFL line
 * (m, k) of angle m reads slice k.  Detector samples u_p = p - (n_u-1)/2.
 * Ray samples: unit steps y_q = q - (n_r-1)/2, n_r the smallest integer
 * >= sqrt(nx^2 + ny^2) with the parity of ny.
 *
 * Kept bins: omega_{k,d} = floor(k * drive_cycles + 1/2) + d for
 * k = harm_lo..harm_hi and d = -half_band..half_band, stored k-major; they
 * must be distinct and inside (0, n_t/2), else MPI3D_EINVAL.
 */
typedef struct {
    int32_t nx, ny, nz;          /* volume size in voxels, each >= 2 */
    int32_t n_angles;            /* M >= 1 */
    const double *theta_rad;     /* host, n_angles FFL angles; NULL = m*pi/M */
    int32_t n_u;                 /* fast-axis samples per line; 0 = nx */
    int32_t n_t;                 /* time samples per FFL line T, >= 32 */
    double drive_cycles;         /* drive periods per line P (> 0) */
    double drive_amp;            /* drive amplitude a in voxels; 0 = n_u/2 */
    double psf_width;            /* PSF scale w = H_sat/G0 in voxels (> 0) */
    int32_t harm_lo, harm_hi;    /* kept harmonics, 1 <= harm_lo <= harm_hi */
    int32_t half_band;           /* D >= 0: bins omega_k - D .. omega_k + D */
    const float *rx_filter;      /* host, 2*n_bins floats (re, im) of D_Gamma on
                                    the kept bins; NULL = 1 */
    double op_scale;             /* c_A, the global signal scale (> 0); 0 = estimate it
                                    at plan creation so that ||A||_2 = 1 (Sec. 3.3): power
                                    iteration on A^T A with the FP32 operator on the device,
                                    from the constant vector, until the estimate of ||A||^2
                                    moves by at most 1e-6 (relative) over 10 iterations,
                                    at most 1000 iterations */
    int32_t precisions;          /* bit mask of (1 << MPI3D_FP32) | (1 << MPI3D_MIXED) |
                                    (1 << MPI3D_PRECOMPOSED): which operator variants get
                                    tables; 0 = FP32 only */
    double raster_sweep;         /* S, the focus-field shift over one FFL line in voxels
                                    (finite; 0 = none).  The zig-zag raster of Sec. 3.1:
                                    during line (m, k) the line centre moves at constant
                                    speed, c_n = +-S (n/T - 1/2), forward (+) when z-row k
                                    is even and backward (-) when it is odd, the same
                                    sequence for every angle (Sec. 2.2), so
                                    xi_n = a sin(2 pi P n/T) + c_n and v_n = xi' gains
                                    +-S/T.  With S != 0 and nz >= 2 the plan holds two
                                    PSF tables (and two precomposed line matrices) */
    int32_t psf_rows;            /* R >= 0: lines coupled by the tensor PSF on each side
                                    (Appendix B eq. PSF in the xz-plane of the 2D FFL model
                                    of Sec. 2.2, in-plane gradient of equal magnitude on both
                                    axes).  x-drive line (m, k) also sees the z-rows k' of
                                    angle m with |k - k'| <= min(R, nz - 1) through the xx
                                    entry h(du, dz) = L'(r/w)/w du^2/r^2 + L(r/w) dz^2/r^3,
                                    r = |(du, dz)|, dz = k - k'; with drive_axes = 2, z-drive
                                    line (m, p) also sees the detector columns p' with
                                    |p - p'| <= min(R, n_u - 1) through the zz entry, the same
                                    function with the drive axis exchanged (along-drive
                                    offset xi_z - z_k, transverse offset p - p').  0 = the
                                    collinear PSF.  h depends on |dz| only, so the time-domain
                                    path runs R + 1 signal passes over symmetric line sums
                                    (MPI3D_PRECOMPOSED: one GEMM per offset); with
                                    raster_sweep != 0 it is MPI3D_ENOTSUP */
    int32_t drive_axes;          /* 1 (or 0): the x-drive scan.  2: every angle is also
                                    scanned with the drive and receive coil along z
                                    (Sec. 3.1): the z-drive scan of angle m has one line
                                    per detector column p, across the z-rows k at
                                    z_k = k - (nz-1)/2, same PSF, time grid and bins.
                                    Its n_angles * n_u lines follow the x-drive lines in
                                    b: line n_angles*nz + m*n_u + p.  Needs nz <= n_u;
                                    with raster_sweep != 0 it is MPI3D_ENOTSUP */
    double drive_amp_z;          /* z-drive amplitude in voxels; 0 = nz/2 */
} mpi3d_geometry;

typedef struct mpi3d_plan mpi3d_plan;

/* Sizes a caller needs to allocate buffers for a plan. */
typedef struct {
    int64_t n_vox;              /* nx*ny*nz floats in a volume */
    int64_t n_lines;            /* FFL lines: n_angles*nz, plus n_angles*n_u z-drive lines
                                   with drive_axes = 2 */
    int64_t n_bins;             /* kept bins per line */
    int64_t n_data_floats;      /* 2*n_lines*n_bins floats in b */
    int64_t n_proj_floats;      /* n_angles*nz*n_u floats in a projection (mpi3d_project) */
    int64_t op_ws_bytes;        /* workspace of mpi3d_forward/adjoint/signal_* */
    int64_t solve_ws_bytes;     /* workspace of mpi3d_solve / a serving state */
    int64_t table_bytes;        /* device memory held by the plan itself */
    int64_t history_doubles;    /* per iteration doubles written to a solve history */
    int32_t n_r;                /* ray samples per projection ray */
    int32_t norm_iters;         /* power iterations that estimated op_scale; 0 = given */
    double op_scale;            /* c_A in use */
    int32_t dft_cycles;         /* FP32 band DFT factored over blocks of this many drive-cycle
                                   samples C (T = C P: a C-point sum at the residues of the kept
                                   bins mod C, then a P-point sum per bin); 0 = one dense
                                   contraction over all T samples */
    int32_t dft_residues;       /* distinct residues of the kept bins mod C (0 when dense) */
} mpi3d_plan_info;

/* Validates the geometry, builds the FP64 host tables (angles, trajectory,
 * PSF kernel, bins, twiddles, receive filter, band scales), and uploads them
 * to `device`.  *out receives the plan; the plan owns its tables. */
int mpi3d_plan_create(const mpi3d_geometry *geom, int device, mpi3d_plan **out);
void mpi3d_plan_destroy(mpi3d_plan *plan);
int mpi3d_plan_query(const mpi3d_plan *plan, mpi3d_plan_info *info);

/* b_dev = A x_dev (complex64, interleaved).  `precision` is MPI3D_FP32 or
 * MPI3D_MIXED (the latter needs the plan to hold the mixed tables).  ws_dev:
 * at least op_ws_bytes of device memory, 256-byte aligned. */
int mpi3d_forward(const mpi3d_plan *plan, int32_t precision, const float *x_dev, float *b_dev,
                  void *ws_dev, size_t ws_bytes, void *stream);

/* No-allocation forward, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  b_dev = A x_dev as mpi3d_forward computes it (same kernels,
 * same order, the same bits), with the operator workspace taken from a static
 * device array of MPI3D_NOALLOC_SCRATCH_BYTES per GPU that the library holds
 * until the process ends; the call allocates nothing.  Plans whose
 * op_ws_bytes exceed that size get MPI3D_ENOMEM (nothing is enqueued).  All
 * three precisions are served.  Every call on one GPU uses that GPU's one
 * array: calls that overlap on a GPU (concurrent streams or host threads)
 * race and must be serialised by the
 * caller; consecutive calls on one stream are safe.  The array keeps the last
 * call's contents, none of which a later call reads before writing it. */
#define MPI3D_NOALLOC_SCRATCH_BYTES (128ull << 20)
int mpi3d_forward_noalloc(const mpi3d_plan *plan, int32_t precision, const float *x_dev, float *b_dev,
                          void *stream);

/* x_dev = A^T b_dev = Re(A^H b_dev).  Same workspace rule as mpi3d_forward. */
int mpi3d_adjoint(const mpi3d_plan *plan, int32_t precision, const float *b_dev, float *x_dev,
                  void *ws_dev, size_t ws_bytes, void *stream);

/* Stage entry points, the operator's factors one at a time (FP32 only):
 *   project      rho_dev[n_angles][nz][n_u] = P x_dev          (eq. ptheta1)
 *   backproject  x_dev = P^T rho_dev
 *   signal_fwd   b_dev = A_DC rho_dev, line by line           (eq. DCmodel)
 *   signal_adj   rho_dev = Re(A_DC^H b_dev)
 * signal_* take and give all n_lines lines of n_u floats (with drive_axes = 2
 * the z-drive lines use their first nz floats; the rest must be zero on input
 * and are zero on output).  signal_* need op_ws_bytes of workspace;
 * project/backproject need none. */
int mpi3d_project(const mpi3d_plan *plan, const float *x_dev, float *rho_dev, void *stream);
int mpi3d_backproject(const mpi3d_plan *plan, const float *rho_dev, float *x_dev, void *stream);
int mpi3d_signal_fwd(const mpi3d_plan *plan, int32_t precision, const float *rho_dev, float *b_dev,
                     void *ws_dev, size_t ws_bytes, void *stream);
int mpi3d_signal_adj(const mpi3d_plan *plan, int32_t precision, const float *b_dev, float *rho_dev,
                     void *ws_dev, size_t ws_bytes, void *stream);

/*
 * Tikhonov least squares by CGLS (the solver of eq. nummodel; T = I):
 *   r = b - A x, s = A^T r - lambda x, p = s, gamma = |s|^2, then per
 *   iteration q = A p, alpha = gamma / (|q|^2 + lambda |p|^2),
 *   x += alpha p, r -= alpha q, s = A^T r - lambda x, beta = |s|^2 / gamma,
 *   p = s + beta p.
 * Inner products, alpha, beta and norms are float64 on the device; no host
 * synchronisation happens between iterations.
 *
 * Variants selected by the options:
 *   clamp_every > 0   after every clamp_every iterations (and after the last)
 *                     x <- max(x, 0) and CGLS restarts from it (the paper's
 *                     nonnegativity, Sec. 3.3 after eq. iters).
 *   precision MIXED   iterative refinement: refine_sweeps sweeps.  A sweep
 *                     forms r0 = b - A x and g0 = A^T r0 - lambda x with the
 *                     FP32 operator, runs inner_iters CGLS iterations with the
 *                     mixed operator A~ on the correction d of
 *                       min |A~ d - r0|^2 + lambda |x + d|^2   (d = 0 at the start),
 *                     whose gradient is g0 - A~^T A~ d - lambda d (A~ only ever
 *                     acts on d and its residual, never on r0, so its error
 *                     shrinks with the correction), then sets x += d (and
 *                     clamps at 0 when clamp_every > 0).
 *
 * solver MOMENTUM selects the paper's own iteration instead (eq. iters):
 *   y = x_k + (k-1)/(k+2) (x_k - x_{k-1}),
 *   x_{k+1} = P(y - tau [A^T (A y - b) + lambda T^T T y]),   k = 1..iters,
 * P = clamp at 0 when clamp_every > 0 (every iteration), else identity; FP32
 * operator only.  reg selects T: IDENTITY, or FD -- forward differences along
 * x, y and z with no term across the volume boundary, so T^T T is the 7-point
 * Laplacian with reflecting ends (FD is available with MOMENTUM only).
 * tau > 0 is used as given; tau <= 0 asks for the paper's
 * tau = 1/(||A^T A||_2 + lambda ||T^T T||_2), with ||A^T A||_2 from power
 * iteration on the device in the solve workspace (up to 1000 FP32 A^T A
 * applications, host-synchronised every 10) and ||T^T T||_2 in closed form.
 * The report's gamma0 / gamma are |x_2 - y_1|^2 and the last step's
 * |x_{k+1} - y|^2; no history is written.
 */
enum { MPI3D_SOLVER_CGLS = 0, MPI3D_SOLVER_MOMENTUM = 1 };
enum { MPI3D_REG_IDENTITY = 0, MPI3D_REG_FD = 1 };
typedef struct {
    double lambda;          /* Tikhonov weight (>= 0) */
    int32_t iters;          /* FP32: total iterations (>= 0) */
    int32_t clamp_every;    /* 0 = never clamp */
    int32_t precision;      /* MPI3D_FP32 or MPI3D_MIXED */
    int32_t refine_sweeps;  /* MIXED only: number of sweeps (>= 1) */
    int32_t inner_iters;    /* MIXED only: CGLS iterations per sweep (>= 1) */
    int32_t x0_is_zero;     /* 1: ignore x_dev on entry and start from 0 */
    int32_t solver;         /* MPI3D_SOLVER_CGLS or MPI3D_SOLVER_MOMENTUM */
    int32_t reg;            /* MPI3D_REG_IDENTITY or MPI3D_REG_FD (MOMENTUM only) */
    double tau;             /* MOMENTUM step; <= 0: the paper's 1/(||A^T A|| + lambda ||T^T T||) */
} mpi3d_solve_opts;

typedef struct {
    int32_t iters_done;     /* CGLS iterations run */
    int32_t status;         /* MPI3D_OK or MPI3D_ENONFINITE */
    double gamma0;          /* |A^T b - lambda x0|^2 at the first start */
    double gamma;           /* |A^T r - lambda x|^2 at the end (inner operator) */
} mpi3d_solve_report;

/* x_dev: in = x0 (unless x0_is_zero), out = solution.  ws_dev: at least
 * solve_ws_bytes.  history_dev: NULL, or device doubles of length
 * history_doubles * (iterations + restarts + 1) receiving per-iteration
 * (gamma, delta, alpha, beta) records.  report: NULL, or a host struct filled
 * after the call synchronises the stream (only then does the call block). */
int mpi3d_solve(const mpi3d_plan *plan, const float *b_dev, float *x_dev, const mpi3d_solve_opts *opts,
                void *ws_dev, size_t ws_bytes, double *history_dev, mpi3d_solve_report *report,
                void *stream);

/*
 * Serving: one CGLS solve per state, advanced one iteration at a time so a
 * scheduler can interleave requests that arrive while others run.  A state
 * keeps its plan, b, x and workspace (all caller-owned) until destroyed; its
 * vectors and float64 scalars stay on the device for its whole life.
 *
 * mpi3d_batch_step runs one iteration (or the restart step that opens a
 * refinement sweep) of every state in `states`, sharing kernel launches
 * between states whose plans have the same line geometry (n_u, n_t, bins,
 * psf, drive): their FFL lines are concatenated into one launch.  Each
 * line's arithmetic does not depend on which other states share the launch,
 * so a request's result is bitwise the same alone or batched.  Groups of
 * different line geometry, step kind or precision touch disjoint states and
 * run on up to four streams: `stream` and a per-device pool of non-blocking
 * streams created on first use (default priority), which wait for `stream`
 * at the step's start and which `stream` waits for at its end, so the step
 * is ordered on `stream`.  Steps on one device must not overlap.  States run
 * CGLS schedules (solver MOMENTUM is MPI3D_ENOTSUP here).
 */
typedef struct mpi3d_state mpi3d_state;
int mpi3d_state_create(const mpi3d_plan *plan, const float *b_dev, float *x_dev,
                       const mpi3d_solve_opts *opts, void *ws_dev, size_t ws_bytes, mpi3d_state **out);
int mpi3d_batch_step(mpi3d_state *const *states, int32_t n_states, void *stream);
/* Host-side progress of a state: steps enqueued so far and whether the
 * schedule is complete (results final once the stream reaches that point). */
int mpi3d_state_progress(const mpi3d_state *state, int32_t *iters_done, int32_t *done);
void mpi3d_state_destroy(mpi3d_state *state);

/*
 * Benchmark support.  Enqueues `repeats` back-to-back launches of one kernel
 * of the operator on `stream` between two HIP events, synchronises, and
 * stores the mean time per launch (milliseconds) in *avg_ms.
 *   kernel 0  projection            reads x_dev, writes the workspace (MIXED:
 *                                   x_dev is first converted to bf16 once,
 *                                   outside the timed launches, and the bf16
 *                                   gather variant is timed)
 *   kernel 1  backprojection        reads the workspace, writes x_dev
 *   kernel 2  signal forward contraction (time signal + band DFT), reads
 *             the workspace's projections (an FP32 plan that factors the band
 *             DFT over drive cycles, dft_cycles > 0: its two launches,
 *             kernels 4 and 5)
 *   kernel 3  signal adjoint contraction, reads b_dev (factored: kernels 6
 *             and 7)
 *             (MIXED, kernels 2 and 3: the per-line scales and fp16 operand
 *             lines are prepared once, outside the timed launches)
 *   kernels 4-7, FP32 plans with dft_cycles > 0 only (else MPI3D_EINVAL):
 *   kernel 4  forward PSF contraction + C-point residue DFT (writes the
 *             workspace's phase sums)
 *   kernel 5  forward P-point outer sum per bin (reads the phase sums)
 *   kernel 6  adjoint outer sum (reads b_dev, writes the phase sums)
 *   kernel 7  adjoint residue DFT + PSF contraction (reads the phase sums)
 * The kernels' work does not depend on the values they read.  x_dev holds
 * n_vox floats, b_dev n_data_floats, ws_dev op_ws_bytes.
 */
int mpi3d_time_kernel(const mpi3d_plan *plan, int32_t kernel, int32_t precision, int32_t repeats, float *x_dev,
                      const float *b_dev, void *ws_dev, size_t ws_bytes, void *stream, float *avg_ms);

/* Static description of a status code. */
const char *mpi3d_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* MPI3D_H */
