// Split reductions of the signal kernels and the CGLS vector/scalar steps.
//
// Every float64 norm is formed the same way: each block sums its elements'
// squares in float64 (fixed per-thread order, then a fixed tree), writes one
// partial, and a single-block scalar kernel adds the partials in index
// order.  Results therefore do not depend on timing, and the CGLS scalars
// (Sec. 3.3 solve of eq. nummodel; see the header for the recurrences) stay
// on the device: no host round trip per iteration.

#include <cmath>

#include "internal.h"

namespace mpi3d {

namespace {

constexpr int kThreads = 256;
constexpr int kVecBlocks = 1024;   // grid of the grid-stride vector kernels

__device__ __forceinline__ double block_sum(double v, double *red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kThreads / 64; ++i) t += red[i];
    return t;  // valid in thread 0
}

// sum_s pp[s * stride] in float64, in split order; four loads in flight
__device__ __forceinline__ double sum_splits(const float *__restrict__ pp, int n, long stride)
{
    double v = 0.0;
    int s = 0;
    for (; s + 4 <= n; s += 4) {
        const float a0 = pp[(long)s * stride], a1 = pp[(long)(s + 1) * stride];
        const float a2 = pp[(long)(s + 2) * stride], a3 = pp[(long)(s + 3) * stride];
        v += (double)a0;
        v += (double)a1;
        v += (double)a2;
        v += (double)a3;
    }
    for (; s < n; ++s) v += (double)pp[(long)s * stride];
    return v;
}

// Sum of the split partials of one output element, undoing the mixed path's
// per-line scale.  Without row coupling: the sum, divided by the line's own
// scale.  With the tensor PSF's passes (npass blocks of nparts / npass
// splits, pass e for offset e): forward, the line's passes e up to its
// coupling range, each divided by the scale of the symmetric sum that pass
// read (row_scale[e * lines + row]); adjoint, pass 0 of the line itself and
// pass e of the lines e before and after it within its angle, each divided
// by the scale of that line's data (row_scale[line]).  In pass order.
__device__ __forceinline__ double sum_unscaled(const float *__restrict__ pp, int nparts, long stride, long row,
                                               const float *__restrict__ row_scale, RowPasses rp)
{
    if (rp.npass <= 1) {
        const double v = sum_splits(pp, nparts, stride);
        return row_scale ? v / (double)row_scale[row] : v;
    }
    // passes: blocks of nparts / npass splits; the fused adjoint: every split
    // holds all passes, pass e at column offset e pass_cols of each line
    const int per = rp.pass_cols ? nparts : nparts / rp.npass;
    const long pass_off = rp.pass_cols ? (long)rp.pass_cols : (long)per * stride;
    const bool zl = row >= rp.zbase;
    const int nline = zl ? rp.nzc : rp.nz;
    const int R = min(zl ? rp.rz : rp.rx, rp.npass - 1);
    const int k = (int)(zl ? (row - rp.zbase) % rp.nzc : row % rp.nz);
    double v = 0.0;
    for (int e = 0; e <= R; ++e) {
        const float *pe = pp + (long)e * pass_off;
        if (rp.fwd) {
            const double t = sum_splits(pe, per, stride);
            v += row_scale ? t / (double)row_scale[(long)e * rp.lines + row] : t;
            continue;
        }
        for (int sg = e == 0 ? 1 : -1; sg <= 1; sg += 2) {
            const int d = sg * e;
            if (k + d < 0 || k + d >= nline) continue;
            const double t = sum_splits(pe + (long)d * rp.pitch, per, stride);
            v += row_scale ? t / (double)row_scale[row + d] : t;
        }
    }
    return v;
}

// out[row][c] = sign * sum_s part[s][row][c] * col_scale[c] / row_scale[row] (+ b_sub)
__global__ __launch_bounds__(kThreads) void reduce_fwd_kernel(long rows, int nb2, int nbp2, int nparts,
                                                               long part_stride, const float *__restrict__ part,
                                                               const float *__restrict__ row_scale,
                                                               const float *__restrict__ col_scale, double scale,
                                                               const float *__restrict__ b_sub, float *out,
                                                               double *norm_parts, RowPasses rp)
{
    __shared__ double red[kThreads / 64];
    const long n = rows * nb2;
    double sq = 0.0;
    for (long idx = (long)blockIdx.x * kThreads + threadIdx.x; idx < n; idx += (long)gridDim.x * kThreads) {
        const long row = idx / nb2;
        const int c = (int)(idx - row * nb2);
        const double v0 = sum_unscaled(part + row * nbp2 + c, nparts, part_stride, row, row_scale, rp);
        double v = v0 * scale;
        if (col_scale) v *= (double)col_scale[c];
        if (b_sub) v = (double)b_sub[idx] - v;
        const float o = (float)v;
        out[idx] = o;
        sq += (double)o * (double)o;
    }
    if (norm_parts) {
        const double t = block_sum(sq, red);
        if (threadIdx.x == 0) norm_parts[blockIdx.x] = t;
    }
}

// out[row][p] = scale * sum_s part[s][row][p] / row_scale[row]   (p < nu)
__global__ __launch_bounds__(kThreads) void reduce_lines_kernel(long rows, int nu, int nup, int out_stride,
                                                                 int nparts, long part_stride,
                                                                 const float *__restrict__ part,
                                                                 const float *__restrict__ row_scale, double scale,
                                                                 float *out, RowPasses rp)
{
    const long n = rows * out_stride;
    for (long idx = (long)blockIdx.x * kThreads + threadIdx.x; idx < n; idx += (long)gridDim.x * kThreads) {
        const long row = idx / out_stride;
        const int p = (int)(idx - row * out_stride);
        float o = 0.f;
        if (p < nu) {
            double v = sum_unscaled(part + row * nup + p, nparts, part_stride, row, row_scale, rp);
            v *= scale;
            o = (float)v;
        }
        out[idx] = o;
    }
}

// The tensor PSF's forward pass inputs: sig[e][row] = rho(row + e) +
// rho(row - e) for the lines of row's angle (rows outside it count as zero;
// sig[0] = rho), zero for e beyond the row's coupling range and for columns
// past nu.
__global__ __launch_bounds__(kThreads) void sym_lines_kernel(const float *__restrict__ rho, int in_stride, int nu,
                                                              int nup, RowPasses rp, float *__restrict__ sig,
                                                              long pass_stride, long line_stride)
{
    const long n = (long)rp.npass * rp.lines * nup;
    for (long idx = (long)blockIdx.x * kThreads + threadIdx.x; idx < n; idx += (long)gridDim.x * kThreads) {
        const int p = (int)(idx % nup);
        const long t = idx / nup;
        const long row = t % rp.lines;
        const int e = (int)(t / rp.lines);
        const long o = e * pass_stride + row * line_stride + p;
        float v = 0.f;
        if (p < nu) {
            if (e == 0) {
                v = rho[row * in_stride + p];
            } else {
                const bool zl = row >= rp.zbase;
                const int nline = zl ? rp.nzc : rp.nz;
                const int R = zl ? rp.rz : rp.rx;
                const int k = (int)(zl ? (row - rp.zbase) % rp.nzc : row % rp.nz);
                if (e <= R) {
                    if (k + e < nline) v += rho[(row + e) * in_stride + p];
                    if (k - e >= 0) v += rho[(row - e) * in_stride + p];
                }
            }
        }
        sig[o] = v;
    }
}

// The mixed adjoint's lines as 16-bit operands of its backprojection: one
// wave per line forms the line's values -- the split sums as reduce_lines
// does, or (lines_in) fp32 lines already formed -- and a power-of-two scale
// s with max |v| s in [0.5, 1) (1 for a zero line; capped like the signal
// kernels' row scales), then writes fp16(v s) over nup columns (zero past
// nu) and 1/s.  Per-line scaling gives every line fp16's relative precision
// whatever its size.
constexpr int kLineSlots = 4;     // nup <= 256: at most 4 values per lane
__global__ __launch_bounds__(kThreads) void lines16_kernel(long rows, int nu, int nup, int nparts, long part_stride,
                                                            const float *__restrict__ part,
                                                            const float *__restrict__ row_scale, double scale,
                                                            RowPasses rp, const float *__restrict__ lines_in,
                                                            uint16_t *__restrict__ out16, float *__restrict__ inv_scale)
{
    const int lane = threadIdx.x & 63;
    const long row = (long)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (row >= rows) return;
    float v[kLineSlots];
    float m = 0.f;
#pragma unroll
    for (int j = 0; j < kLineSlots; ++j) {
        const int p = lane + 64 * j;
        float o = 0.f;
        if (p < nu) {
            if (lines_in) {
                o = lines_in[row * nup + p];
            } else {
                const double t = sum_unscaled(part + row * nup + p, nparts, part_stride, row, row_scale, rp);
                o = (float)(t * scale);
            }
        }
        v[j] = o;
        m = fmaxf(m, fabsf(o));
    }
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    float s = 1.f;
    if (m > 0.f && isfinite(m)) {
        int e;
        frexpf(m, &e);
        s = ldexpf(1.f, min(-e, 120));
    }
    if (lane == 0) inv_scale[row] = 1.f / s;
#pragma unroll
    for (int j = 0; j < kLineSlots; ++j) {
        const int p = lane + 64 * j;
        if (p < nup) out16[row * nup + p] = __builtin_bit_cast(uint16_t, (_Float16)(v[j] * s));
    }
}

// Power-of-two line scales for the fp16 contractions: for each row,
// s = 2^-e with max_c |in[row][c] * col_scale[c]| in [2^(e-1), 2^e), so the
// scaled row's largest entry lies in [0.5, 1); 1 for an all-zero row.  With
// out16 the row is also written as the fp16 operand the signal kernels read,
// (in[row][c] * col_scale[c]) * s rounded to nearest, zero from column ncols
// to out16_cols.  One wave per row.
__global__ __launch_bounds__(kThreads) void row_scale_kernel(long rows, int ncols, int in_stride,
                                                              const float *__restrict__ in,
                                                              const float *__restrict__ col_scale, float *out,
                                                              uint16_t *__restrict__ out16, int out16_cols,
                                                              int out16_stride)
{
    const int lane = threadIdx.x & 63;
    const long row = (long)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (row >= rows) return;
    const float *p = in + row * in_stride;
    float m = 0.f;
    for (int c = lane; c < ncols; c += 64) m = fmaxf(m, fabsf(col_scale ? p[c] * col_scale[c] : p[c]));
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    float s = 1.f;
    if (m > 0.f && isfinite(m)) {
        // 2^-e brings the row maximum into [0.5, 1); capped so that rows
        // of subnormal size get a finite scale (and a normal 1/scale)
        int e;
        frexpf(m, &e);
        s = ldexpf(1.f, min(-e, 120));
    }
    if (lane == 0) out[row] = s;
    if (!out16) return;
    uint16_t *q = out16 + row * out16_stride;
    for (int c = lane; c < out16_cols; c += 64) {
        const float v = c < ncols ? (col_scale ? p[c] * col_scale[c] : p[c]) * s : 0.f;
        const _Float16 hv = (_Float16)v;
        q[c] = __builtin_bit_cast(uint16_t, hv);
    }
}

// Scalar slots (doubles) of one solve.
enum { S_GAMMA = 0, S_DELTA, S_ALPHA, S_BETA, S_BAD, S_GAMMA0, S_STEP, S_NSLOTS };

__device__ double sum_parts(const double *parts, int n, double *red)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) v += parts[i];
    return block_sum(v, red);
}

// delta = |q|^2 + lambda |p|^2, alpha = gamma / delta
__global__ __launch_bounds__(kThreads) void alpha_kernel(double *scal, const double *parts_q, int nq,
                                                          const double *parts_p, int np, double lambda,
                                                          double *hist, int step)
{
    __shared__ double red[kThreads / 64];
    const double qq = sum_parts(parts_q, nq, red);
    __syncthreads();
    const double pp = sum_parts(parts_p, np, red);
    if (threadIdx.x == 0) {
        const double delta = qq + lambda * pp;
        const double alpha = scal[S_GAMMA] / delta;
        scal[S_DELTA] = delta;
        scal[S_ALPHA] = alpha;
        if (!isfinite(alpha)) scal[S_BAD] = 1.0;
        if (hist) {
            hist[4 * step + 0] = scal[S_GAMMA];
            hist[4 * step + 1] = delta;
            hist[4 * step + 2] = alpha;
        }
    }
}

// gamma' = |s|^2; beta = gamma'/gamma (restart: beta = 0, and on the first
// start gamma0 = gamma')
__global__ __launch_bounds__(kThreads) void beta_kernel(double *scal, const double *parts_s, int ns, int restart,
                                                         int first, double *hist, int step)
{
    __shared__ double red[kThreads / 64];
    const double g = sum_parts(parts_s, ns, red);
    if (threadIdx.x == 0) {
        double beta = 0.0;
        if (!restart) beta = g / scal[S_GAMMA];
        if (first) scal[S_GAMMA0] = g;
        scal[S_GAMMA] = g;
        scal[S_BETA] = beta;
        if (!isfinite(g) || !isfinite(beta)) scal[S_BAD] = 1.0;
        if (hist && !restart) hist[4 * step + 3] = beta;
    }
}

__global__ __launch_bounds__(kThreads) void update_xr_kernel(float *__restrict__ x, const float *__restrict__ p,
                                                              float *__restrict__ r, const float *__restrict__ q,
                                                              long nvox, long ndata, const double *scal)
{
    const double alpha = scal[S_ALPHA];
    const float af = (float)alpha;
    const long n = nvox + ndata;
    for (long idx = (long)blockIdx.x * kThreads + threadIdx.x; idx < n; idx += (long)gridDim.x * kThreads) {
        if (idx < nvox) x[idx] = fmaf(af, p[idx], x[idx]);
        else {
            const long j = idx - nvox;
            r[j] = fmaf(-af, q[j], r[j]);
        }
    }
}

// p = s + beta p (beta from scal), optional bf16 shadow, partial |p|^2
__global__ __launch_bounds__(kThreads) void update_p_kernel(float *__restrict__ p, const float *__restrict__ s,
                                                             uint16_t *pb, long n, const double *scal,
                                                             double *parts_p, int init)
{
    __shared__ double red[kThreads / 64];
    const float bf = (float)scal[S_BETA];
    double sq = 0.0;
    for (long idx = (long)blockIdx.x * kThreads + threadIdx.x; idx < n; idx += (long)gridDim.x * kThreads) {
        const float v = init ? s[idx] : fmaf(bf, p[idx], s[idx]);
        p[idx] = v;
        sq += (double)v * (double)v;
        if (pb) {
            // round to nearest even bf16
            uint32_t u = __float_as_uint(v);
            u += 0x7fffu + ((u >> 16) & 1u);
            pb[idx] = (uint16_t)(u >> 16);
        }
    }
    const double t = block_sum(sq, red);
    if (threadIdx.x == 0) parts_p[blockIdx.x] = t;
}

__global__ __launch_bounds__(kThreads) void to_bf16_kernel(long n, const float *x, uint16_t *xb)
{
    for (long idx = (long)blockIdx.x * kThreads + threadIdx.x; idx < n; idx += (long)gridDim.x * kThreads) {
        uint32_t u = __float_as_uint(x[idx]);
        u += 0x7fffu + ((u >> 16) & 1u);
        xb[idx] = (uint16_t)(u >> 16);
    }
}

__global__ __launch_bounds__(kThreads) void clamp_kernel(float *x, long n)
{
    for (long idx = (long)blockIdx.x * kThreads + threadIdx.x; idx < n; idx += (long)gridDim.x * kThreads)
        x[idx] = fmaxf(x[idx], 0.f);
}

// x = x + d (refinement sweep end), optionally clamped at 0
__global__ __launch_bounds__(kThreads) void add_to_kernel(float *__restrict__ x, const float *__restrict__ d, long n,
                                                           int clamp)
{
    for (long idx = (long)blockIdx.x * kThreads + threadIdx.x; idx < n; idx += (long)gridDim.x * kThreads) {
        const float v = x[idx] + d[idx];
        x[idx] = clamp ? fmaxf(v, 0.f) : v;
    }
}

__global__ __launch_bounds__(kThreads) void fill_kernel(float *x, long n, float v)
{
    for (long idx = (long)blockIdx.x * kThreads + threadIdx.x; idx < n; idx += (long)gridDim.x * kThreads)
        x[idx] = v;
}

__global__ __launch_bounds__(kThreads) void copy_kernel(float *dst, const float *src, long n)
{
    for (long idx = (long)blockIdx.x * kThreads + threadIdx.x; idx < n; idx += (long)gridDim.x * kThreads)
        dst[idx] = src[idx];
}

// One step of the paper's iteration (eq. iters) after g = A^T (b - A y):
//   x_new = P(y + tau g - tau lambda T^T T y),  P = clamp at 0 when nonneg
//   y_new = x_new + beta (x_new - x)            (the next momentum point)
// T^T T y is the 7-point finite-difference Laplacian with no term across the
// volume boundary (fd = 1) or y itself (fd = 0).  y_new may alias g: every
// thread reads g only at its own voxel before writing y_new there.  A block
// partial of |x_new - y|^2 (the step) goes to parts.
__global__ __launch_bounds__(kThreads) void momentum_kernel(const float *__restrict__ y, const float *g,
                                                             const float *__restrict__ x, float *__restrict__ x_new,
                                                             float *y_new, int nx, int ny, int nz, float tau,
                                                             float taulam, float beta, int fd, int nonneg,
                                                             double *parts)
{
    __shared__ double red[kThreads / 64];
    const long n = (long)nx * ny * nz;
    const long sxy = (long)nx * ny;
    double sq = 0.0;
    for (long idx = (long)blockIdx.x * kThreads + threadIdx.x; idx < n; idx += (long)gridDim.x * kThreads) {
        const float yc = y[idx];
        float ty = yc;
        if (fd) {
            const int i = (int)(idx % nx);
            const int j = (int)((idx / nx) % ny);
            const int k = (int)(idx / sxy);
            float acc = 0.f;
            if (i > 0) acc += yc - y[idx - 1];
            if (i + 1 < nx) acc += yc - y[idx + 1];
            if (j > 0) acc += yc - y[idx - nx];
            if (j + 1 < ny) acc += yc - y[idx + nx];
            if (k > 0) acc += yc - y[idx - sxy];
            if (k + 1 < nz) acc += yc - y[idx + sxy];
            ty = acc;
        }
        float v = fmaf(tau, g[idx], fmaf(-taulam, ty, yc));
        if (nonneg) v = fmaxf(v, 0.f);
        const float xo = x[idx];
        x_new[idx] = v;
        y_new[idx] = fmaf(beta, v - xo, v);
        const double dv = (double)v - (double)yc;
        sq += dv * dv;
    }
    const double t = block_sum(sq, red);
    if (threadIdx.x == 0) parts[blockIdx.x] = t;
}

// scal[S_GAMMA] = sum of the step partials (and S_GAMMA0 on the first step)
__global__ __launch_bounds__(kThreads) void step_norm_kernel(double *scal, const double *parts, int n, int first)
{
    __shared__ double red[kThreads / 64];
    const double t = sum_parts(parts, n, red);
    if (threadIdx.x == 0) {
        scal[S_GAMMA] = t;
        if (first) scal[S_GAMMA0] = t;
        if (!isfinite(t)) scal[S_BAD] = 1.0;
    }
}

// Power iteration on A^T A: norms[k] = |z| from the partials of |z|^2.
__global__ __launch_bounds__(kThreads) void norm_record_kernel(const double *parts, int n, double *norms, int k)
{
    __shared__ double red[kThreads / 64];
    const double t = sum_parts(parts, n, red);
    if (threadIdx.x == 0) norms[k] = sqrt(t);
}

// v = z / norms[k]
__global__ __launch_bounds__(kThreads) void scale_by_kernel(float *__restrict__ v, const float *__restrict__ z, long n,
                                                             const double *norms, int k)
{
    const float inv = (float)(1.0 / norms[k]);
    for (long idx = (long)blockIdx.x * kThreads + threadIdx.x; idx < n; idx += (long)gridDim.x * kThreads)
        v[idx] = z[idx] * inv;
}

__global__ void scal_init_kernel(double *scal)
{
    if (threadIdx.x < S_NSLOTS) scal[threadIdx.x] = 0.0;
}

int grid_for(long n, int cap = kVecBlocks)
{
    long b = (n + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

constexpr int kReduceBlocks = kMaxNormParts;   // the split reductions want many loads in flight

}  // namespace

int scal_slots() { return S_NSLOTS; }
int scal_slot_bad() { return S_BAD; }
int scal_slot_gamma() { return S_GAMMA; }
int scal_slot_gamma0() { return S_GAMMA0; }

hipError_t launch_reduce_fwd(long rows, int nb2, int nbp2, int nparts, long part_stride, const float *part,
                             const float *row_scale, const float *col_scale, double scale, const float *b_sub,
                             float *out, double *norm_parts, int *nnorm, hipStream_t st, RowPasses rp)
{
    const int g = grid_for(rows * nb2, kReduceBlocks);
    if (nnorm) *nnorm = g;
    hipLaunchKernelGGL(reduce_fwd_kernel, dim3(g), dim3(kThreads), 0, st, rows, nb2, nbp2, nparts, part_stride,
                       part, row_scale, col_scale, scale, b_sub, out, norm_parts, rp);
    return hipGetLastError();
}

hipError_t launch_reduce_lines_strided(long rows, int nu, int nup, int out_stride, int nparts, long part_stride,
                                       const float *part, const float *row_scale, double scale, float *out,
                                       hipStream_t st, RowPasses rp)
{
    const int g = grid_for(rows * out_stride, kReduceBlocks);
    hipLaunchKernelGGL(reduce_lines_kernel, dim3(g), dim3(kThreads), 0, st, rows, nu, nup, out_stride, nparts,
                       part_stride, part, row_scale, scale, out, rp);
    return hipGetLastError();
}

hipError_t launch_lines16(long rows, int nu, int nup, int nparts, long part_stride, const float *part,
                          const float *row_scale, double scale, RowPasses rp, const float *lines_in, uint16_t *out16,
                          float *inv_scale, hipStream_t st)
{
    if (nup > 64 * kLineSlots) return hipErrorInvalidValue;
    const long blocks = (rows + kThreads / 64 - 1) / (kThreads / 64);
    hipLaunchKernelGGL(lines16_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, st, rows, nu, nup, nparts,
                       part_stride, part, row_scale, scale, rp, lines_in, out16, inv_scale);
    return hipGetLastError();
}



hipError_t launch_sym_lines(const float *rho, int in_stride, int nu, int nup, RowPasses rp, float *sig,
                            long pass_stride, long line_stride, hipStream_t st)
{
    const int g = grid_for((long)rp.npass * rp.lines * nup, kReduceBlocks);
    hipLaunchKernelGGL(sym_lines_kernel, dim3(g), dim3(kThreads), 0, st, rho, in_stride, nu, nup, rp, sig,
                       pass_stride, line_stride);
    return hipGetLastError();
}

hipError_t launch_row_scale(long rows, int ncols, int in_stride, const float *in, const float *col_scale, float *out,
                            uint16_t *out16, int out16_cols, int out16_stride, hipStream_t st)
{
    const long blocks = (rows + kThreads / 64 - 1) / (kThreads / 64);
    hipLaunchKernelGGL(row_scale_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, st, rows, ncols, in_stride, in,
                       col_scale, out, out16, out16_cols, out16_stride);
    return hipGetLastError();
}

hipError_t launch_to_bf16(long n, const float *x, uint16_t *xb, hipStream_t st)
{
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n)), dim3(kThreads), 0, st, n, x, xb);
    return hipGetLastError();
}

hipError_t launch_alpha(double *scal, const double *parts_q, int nq, const double *parts_p, int np, double lambda,
                        double *hist, int step, hipStream_t st)
{
    hipLaunchKernelGGL(alpha_kernel, dim3(1), dim3(kThreads), 0, st, scal, parts_q, nq, parts_p, np, lambda, hist,
                       step);
    return hipGetLastError();
}

hipError_t launch_beta(double *scal, const double *parts_s, int ns, int restart, int first, double *hist, int step,
                       hipStream_t st)
{
    hipLaunchKernelGGL(beta_kernel, dim3(1), dim3(kThreads), 0, st, scal, parts_s, ns, restart, first, hist, step);
    return hipGetLastError();
}

hipError_t launch_update_xr2(float *x, const float *p, float *r, const float *q, long nvox, long ndata,
                             const double *scal, hipStream_t st)
{
    hipLaunchKernelGGL(update_xr_kernel, dim3(grid_for(nvox + ndata)), dim3(kThreads), 0, st, x, p, r, q, nvox,
                       ndata, scal);
    return hipGetLastError();
}

hipError_t launch_update_p2(float *p, const float *s, uint16_t *pb, long n, const double *scal, double *parts_p,
                            int *np_out, int init, hipStream_t st)
{
    const int g = grid_for(n);
    if (np_out) *np_out = g;
    hipLaunchKernelGGL(update_p_kernel, dim3(g), dim3(kThreads), 0, st, p, s, pb, n, scal, parts_p, init);
    return hipGetLastError();
}

hipError_t launch_scal_init(double *scal, hipStream_t st)
{
    hipLaunchKernelGGL(scal_init_kernel, dim3(1), dim3(64), 0, st, scal);
    return hipGetLastError();
}

hipError_t launch_clamp(float *x, long n, hipStream_t st)
{
    hipLaunchKernelGGL(clamp_kernel, dim3(grid_for(n)), dim3(kThreads), 0, st, x, n);
    return hipGetLastError();
}

hipError_t launch_fill(float *x, long n, float v, hipStream_t st)
{
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(kThreads), 0, st, x, n, v);
    return hipGetLastError();
}

hipError_t launch_copy(float *dst, const float *src, long n, hipStream_t st)
{
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(kThreads), 0, st, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_add_to(float *x, const float *d, long n, int clamp, hipStream_t st)
{
    hipLaunchKernelGGL(add_to_kernel, dim3(grid_for(n)), dim3(kThreads), 0, st, x, d, n, clamp);
    return hipGetLastError();
}

hipError_t launch_momentum(const float *y, const float *g, const float *x, float *x_new, float *y_new, int nx,
                           int ny, int nz, float tau, float taulam, float beta, int fd, int nonneg, double *parts,
                           int *nparts, hipStream_t st)
{
    const long n = (long)nx * ny * nz;
    const int b = grid_for(n);
    if (nparts) *nparts = b;
    hipLaunchKernelGGL(momentum_kernel, dim3(b), dim3(kThreads), 0, st, y, g, x, x_new, y_new, nx, ny, nz, tau,
                       taulam, beta, fd, nonneg, parts);
    return hipGetLastError();
}

hipError_t launch_step_norm(double *scal, const double *parts, int n, int first, hipStream_t st)
{
    hipLaunchKernelGGL(step_norm_kernel, dim3(1), dim3(kThreads), 0, st, scal, parts, n, first);
    return hipGetLastError();
}

hipError_t launch_norm_record(const double *parts, int n, double *norms, int k, hipStream_t st)
{
    hipLaunchKernelGGL(norm_record_kernel, dim3(1), dim3(kThreads), 0, st, parts, n, norms, k);
    return hipGetLastError();
}

hipError_t launch_scale_by(float *v, const float *z, long n, const double *norms, int k, hipStream_t st)
{
    hipLaunchKernelGGL(scale_by_kernel, dim3(grid_for(n)), dim3(kThreads), 0, st, v, z, n, norms, k);
    return hipGetLastError();
}

}  // namespace mpi3d
