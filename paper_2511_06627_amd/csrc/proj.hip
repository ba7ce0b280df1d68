// Parallel-beam projection P_theta and its transpose on gfx950.
//
// Forward (Sec. 2.2, eq. ptheta2 / eq. ptheta1): for FFL angle m, z-slice k
// and detector sample p,
//   rho_theta[m][k][p] = sum_q bilerp(x[k]; u_p cos t + y_q sin t, -u_p sin t + y_q cos t)
// with unit-step ray samples y_q and zero outside the grid.
//
//   One block = one z-slice and a group of angles.  The slice is staged in
//   LDS with a one-voxel zero border (a band of rows at a time when a whole
//   slice does not fit in 160 KB), read once from HBM with coalesced row
//   loads and reused by every ray of every angle in the group.  Each thread
//   owns a few rays and walks the exact range of samples that fall in the
//   staged band, so no sample is read outside the tile and no ray sum needs
//   a cross-thread reduction.
//
// Adjoint (exact transpose, gather form, no atomics): every voxel collects,
// for each angle, the bilinear weights of the <= 3 x 3 ray samples whose
// 2x2 footprint covers it -- the same weights the forward pass uses --
// summed per ray into <= 3 ray weights.  Those weights do not depend on z,
// so one block covers a 16x16 voxel tile for a group of kz slices and reuses
// the weights kz times; the projections it needs for one angle (kz lines x
// <= 32 rays) are staged in LDS.  The epilogue optionally forms
// out = acc + x_add - lambda * x_sub and a float64 partial sum of out^2 (CGLS).

#include <type_traits>

#include "internal.h"

namespace mpi3d {

namespace {

// blockIdx -> logical block so that consecutive logical blocks share an XCD
// (blocks are dealt to the 8 XCDs round-robin).
__device__ __forceinline__ int xcd_logical(int bid, int nblocks)
{
    const int nx = 8;
    int xcd = bid % nx, slot = bid / nx;
    int per = nblocks / nx, rem = nblocks % nx;
    // XCD x receives per + (x < rem) blocks
    return xcd * per + min(xcd, rem) + slot;
}

constexpr int kFwdThreads = 1024;
constexpr int kMaxRaysPerThread = 4;

// Staged slice element (LDS column col = grid column col - 1):
//  fp32 path: the voxel value;
//  bf16 path (the mixed operator's gathers): a pair-packed word, low half the
//  bf16 voxel and high half its right neighbour, so the two horizontal
//  neighbours of a bilinear sample arrive in one 32-bit LDS read.
__device__ __forceinline__ void corners(const float *l0, int W, float &v00, float &v10, float &v01, float &v11)
{
    v00 = l0[0];
    v10 = l0[1];
    v01 = l0[W];
    v11 = l0[W + 1];
}
__device__ __forceinline__ void corners(const uint32_t *l0, int W, float &v00, float &v10, float &v01, float &v11)
{
    const uint32_t a = l0[0], b = l0[W];
    v00 = __uint_as_float(a << 16);
    v10 = __uint_as_float(a & 0xffff0000u);
    v01 = __uint_as_float(b << 16);
    v11 = __uint_as_float(b & 0xffff0000u);
}

// One bilinear sample of the staged band.  Branch-free: a sample whose 2x2
// footprint lies outside the band reads a safe LDS address and contributes 0.
template <typename T>
__device__ __forceinline__ float sample(const T *lds, int W, int nx, int nbase, int jb0, float bx, float by,
                                        float s, float c, float y)
{
    const float fx = fmaf(y, s, bx), fy = fmaf(y, c, by);
    const float ix = floorf(fx), iy = floorf(fy);
    int i0 = (int)ix, j0 = (int)iy - jb0;
    const bool ok = (unsigned)i0 <= (unsigned)nx && (unsigned)j0 < (unsigned)nbase;
    i0 = ok ? i0 : 0;
    j0 = ok ? j0 : 0;
    const float wx = fx - ix, wy = fy - iy;
    float v00, v10, v01, v11;
    corners(lds + j0 * W + i0, W, v00, v10, v01, v11);
    const float top = fmaf(wx, v10 - v00, v00);
    const float bot = fmaf(wx, v11 - v01, v01);
    return ok ? fmaf(wy, bot - top, top) : 0.f;
}

__device__ __forceinline__ uint32_t bf16_at(const uint16_t *slice, int nx, int ny, int gj, int gi)
{
    return (gj >= 0 && gj < ny && gi >= 0 && gi < nx) ? (uint32_t)slice[(size_t)gj * nx + gi] : 0u;
}

// T = float: the fp32 path (reads x).  T = uint32_t: the bf16 path (reads the
// bf16 copy xb, stages pair-packed words); weights and sums stay fp32.
template <typename T>
__global__ __launch_bounds__(kFwdThreads) void proj_fwd_kernel(ProjArgs a, int out_stride)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *lds = reinterpret_cast<T *>(lds_raw);
    const int nb = gridDim.x;
    const int lb = xcd_logical(blockIdx.x, nb);
    const int k = lb / a.n_angle_groups;
    const int mg = lb % a.n_angle_groups;
    // angles split as evenly as possible over the groups
    const int m0 = (mg * a.M) / a.n_angle_groups;
    const int m1 = ((mg + 1) * a.M) / a.n_angle_groups;
    const int W = a.nx + 2;
    const int tid = threadIdx.x;
    const int nrays = (m1 - m0) * a.nu;

    float acc[kMaxRaysPerThread];
#pragma unroll
    for (int i = 0; i < kMaxRaysPerThread; ++i) acc[i] = 0.f;

    const float *slice = a.x ? a.x + (size_t)k * a.nx * a.ny : nullptr;
    const uint16_t *sliceb = a.xb ? a.xb + (size_t)k * a.nx * a.ny : nullptr;
    for (int band = 0; band < a.n_bands; ++band) {
        const int jb0 = -1 + band * a.band_rows;               // first base row
        const int jb1 = min(jb0 + a.band_rows, a.ny);          // one past last base row
        const int nbase = jb1 - jb0;
        const int rows = nbase + 1;                            // LDS rows: grid rows jb0..jb1
        __syncthreads();
        for (int idx = tid; idx < rows * W; idx += kFwdThreads) {
            int r = idx / W, col = idx - r * W;
            int gj = jb0 + r, gi = col - 1;
            if constexpr (std::is_same<T, float>::value) {
                float v = 0.f;
                if (gj >= 0 && gj < a.ny && gi >= 0 && gi < a.nx) v = slice[(size_t)gj * a.nx + gi];
                lds[idx] = v;
            } else {
                lds[idx] = bf16_at(sliceb, a.nx, a.ny, gj, gi) | (bf16_at(sliceb, a.nx, a.ny, gj, gi + 1) << 16);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kMaxRaysPerThread; ++i) {
            const int ray = tid + kFwdThreads * i;
            if (ray >= nrays) continue;
            const int m = m0 + ray / a.nu, p = ray % a.nu;
            const float2 csv = a.cs[m];
            const float c = csv.x, s = csv.y;
            const float bx = a.ax[(size_t)m * a.nu + p];
            const float by = a.ay[(size_t)m * a.nu + p];
            // sample coordinates: fx = bx + y s in LDS columns (column 0 is grid
            // column -1), fy = by + y c in grid rows, y = q - (nr-1)/2.  A sample
            // belongs to this band when its base row floor(fy) is in [jb0, jb1);
            // fy does not depend on the band, so every sample lands in exactly
            // one band.  Samples with floor(fx) outside [0, nx] touch no voxel.
            // The q range below is a slightly widened superset; the exact test
            // is per sample.
            float ylo = -a.half_nr, yhi = a.half_nr;
            if (s > 0.f) {
                ylo = fmaxf(ylo, (0.f - bx) / s);
                yhi = fminf(yhi, ((float)(a.nx + 1) - bx) / s);
            }
            if (c > 0.f) {
                ylo = fmaxf(ylo, ((float)jb0 - by) / c);
                yhi = fminf(yhi, ((float)jb1 - by) / c);
            } else if (c < 0.f) {
                ylo = fmaxf(ylo, ((float)jb1 - by) / c);
                yhi = fminf(yhi, ((float)jb0 - by) / c);
            }
            const int q0 = max(0, (int)floorf(ylo + a.half_nr) - 1);
            const int q1 = min(a.nr - 1, (int)ceilf(yhi + a.half_nr) + 1);
            // four independent partial sums keep several LDS reads in flight
            float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
            int q = q0;
            for (; q + 3 <= q1; q += 4) {
                const float y = (float)q - a.half_nr;
                s0 += sample(lds, W, a.nx, nbase, jb0, bx, by, s, c, y);
                s1 += sample(lds, W, a.nx, nbase, jb0, bx, by, s, c, y + 1.f);
                s2 += sample(lds, W, a.nx, nbase, jb0, bx, by, s, c, y + 2.f);
                s3 += sample(lds, W, a.nx, nbase, jb0, bx, by, s, c, y + 3.f);
            }
            for (; q <= q1; ++q) s0 += sample(lds, W, a.nx, nbase, jb0, bx, by, s, c, (float)q - a.half_nr);
            acc[i] += (s0 + s1) + (s2 + s3);
        }
    }
#pragma unroll
    for (int i = 0; i < kMaxRaysPerThread; ++i) {
        const int ray = tid + kFwdThreads * i;
        if (ray >= nrays) continue;
        const int m = m0 + ray / a.nu, p = ray % a.nu;
        a.rt[((size_t)m * a.nz + k) * out_stride + p] = acc[i];
    }
    // zero the padding columns of the lines this block owns
    if (out_stride > a.nu) {
        const int pad = out_stride - a.nu;
        const int nm = m1 - m0;
        for (int idx = tid; idx < nm * pad; idx += kFwdThreads) {
            const int m = m0 + idx / pad, p = a.nu + idx % pad;
            a.rt[((size_t)m * a.nz + k) * out_stride + p] = 0.f;
        }
    }
}

constexpr int kTile = 16;
constexpr int kPW = 32;     // staged rays per angle per tile
constexpr int kMaxKz = 32;

__device__ __forceinline__ float hat(float t) { return fmaxf(0.f, 1.f - fabsf(t)); }

__global__ __launch_bounds__(256) void proj_adj_kernel(ProjArgs a, int in_stride)
{
    __shared__ float gs[kMaxKz * kPW];
    __shared__ double red[256 / 64];
    const int nb = gridDim.x;
    const int lb = xcd_logical(blockIdx.x, nb);
    const int zg = lb / (a.tiles_x * a.tiles_y);
    const int tile = lb % (a.tiles_x * a.tiles_y);
    const int tx0 = (tile % a.tiles_x) * kTile, ty0 = (tile / a.tiles_x) * kTile;
    const int k0 = zg * a.kz;
    const int kn = min(a.kz, a.nz - k0);
    const int tid = threadIdx.x;
    const int i = tx0 + (tid % kTile), j = ty0 + (tid / kTile);
    const bool valid = i < a.nx && j < a.ny;
    const float X = (float)i - a.cx, Y = (float)j - a.cy;
    const float X0 = (float)tx0 - a.cx, Y0 = (float)ty0 - a.cy;
    const float X1 = X0 + (float)(kTile - 1), Y1 = Y0 + (float)(kTile - 1);

    float acc[kMaxKz];
#pragma unroll
    for (int kk = 0; kk < kMaxKz; ++kk) acc[kk] = 0.f;

    for (int m = 0; m < a.M; ++m) {
        const float2 csv = a.cs[m];
        const float c = csv.x, s = csv.y;
        // detector index range of the tile (u is linear in X, Y: extremes at corners)
        const float u00 = X0 * c - Y0 * s, u10 = X1 * c - Y0 * s, u01 = X0 * c - Y1 * s, u11 = X1 * c - Y1 * s;
        const float umin = fminf(fminf(u00, u10), fminf(u01, u11)) + a.half_nu;
        const int p_lo = (int)floorf(umin) - 2;   // margin for rounding between u and umin
        __syncthreads();
        for (int idx = tid; idx < kMaxKz * kPW; idx += 256) {
            const int kk = idx / kPW, pp = idx % kPW;
            const int p = p_lo + pp;
            float v = 0.f;
            if (kk < kn && p >= 0 && p < a.nu) v = a.rt_in[((size_t)m * a.nz + k0 + kk) * in_stride + p];
            gs[idx] = v;
        }
        __syncthreads();
        if (!valid) continue;
        // voxel position in (detector, ray-sample) index coordinates
        const float u = fmaf(X, c, -Y * s) + a.half_nu;
        const float yv = fmaf(X, s, Y * c) + a.half_nr;
        const float pc = rintf(u), qc = rintf(yv);
        float w[3];
#pragma unroll
        for (int dp = 0; dp < 3; ++dp) {
            const float pf = pc + (float)(dp - 1);
            const float du = pf - u;
            float wp = 0.f;
#pragma unroll
            for (int dq = 0; dq < 3; ++dq) {
                const float qf = qc + (float)(dq - 1);
                const float dy = qf - yv;
                const float dX = fmaf(du, c, dy * s);
                const float dY = fmaf(dy, c, -du * s);
                const bool qok = qf >= 0.f && qf <= (float)(a.nr - 1);
                wp += qok ? hat(dX) * hat(dY) : 0.f;
            }
            const bool pok = pf >= 0.f && pf <= (float)(a.nu - 1);
            w[dp] = pok ? wp : 0.f;
        }
        const int off = min(max((int)pc - 1 - p_lo, 0), kPW - 3);  // in range by construction
        const float *g0 = gs + off;
#pragma unroll
        for (int kk = 0; kk < kMaxKz; ++kk) {
            if (kk < kn) {
                const float *gk = g0 + kk * kPW;
                acc[kk] = fmaf(w[0], gk[0], fmaf(w[1], gk[1], fmaf(w[2], gk[2], acc[kk])));
            }
        }
    }

    double sq = 0.0;
    if (valid) {
#pragma unroll
        for (int kk = 0; kk < kMaxKz; ++kk) {
            if (kk < kn) {
                const size_t idx = ((size_t)(k0 + kk) * a.ny + j) * a.nx + i;
                float v = acc[kk];
                if (a.x_sub || a.x_add) {
                    double t = (double)v;
                    if (a.x_add) t += (double)a.x_add[idx];
                    if (a.x_sub) t -= a.lambda * (double)a.x_sub[idx];
                    v = (float)t;
                }
                a.xo[idx] = v;
                sq += (double)v * (double)v;
            }
        }
    }
    if (a.norm_parts) {
        // block sum in float64, fixed order
        for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
        if ((tid & 63) == 0) red[tid >> 6] = sq;
        __syncthreads();
        if (tid == 0) a.norm_parts[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

}  // namespace

static ProjArgs base_args(const mpi3d_plan *pl)
{
    ProjArgs a{};
    a.cs = pl->cs;
    a.ax = pl->ax;
    a.ay = pl->ay;
    a.nx = pl->nx; a.ny = pl->ny; a.nz = pl->nz; a.M = pl->M; a.nu = pl->nu; a.nup = pl->nup; a.nr = pl->nr;
    a.angles_per_block = pl->angles_per_block;
    a.n_angle_groups = pl->n_angle_groups;
    a.band_rows = pl->band_rows;
    a.n_bands = pl->n_bands;
    a.kz = pl->kz;
    a.n_zgroups = (pl->nz + pl->kz - 1) / pl->kz;
    a.tiles_x = (pl->nx + kTile - 1) / kTile;
    a.tiles_y = (pl->ny + kTile - 1) / kTile;
    a.half_nr = 0.5f * (float)(pl->nr - 1);
    a.half_nu = 0.5f * (float)(pl->nu - 1);
    a.cx = 0.5f * (float)(pl->nx - 1);
    a.cy = 0.5f * (float)(pl->ny - 1);
    return a;
}

template <typename T>
static hipError_t launch_fwd(const mpi3d_plan *pl, const float *x, const uint16_t *xb, float *rt, int out_stride,
                             hipStream_t st)
{
    ProjArgs a = base_args(pl);
    a.x = x;
    a.xb = xb;
    a.rt = rt;
    const int blocks = pl->nz * a.n_angle_groups;
    const size_t lds = (size_t)(a.band_rows + 1) * (pl->nx + 2) * sizeof(T);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)proj_fwd_kernel<T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(proj_fwd_kernel<T>, dim3(blocks), dim3(kFwdThreads), lds, st, a, out_stride);
    return hipGetLastError();
}

hipError_t launch_project_strided(const mpi3d_plan *pl, const float *x, float *rt, int out_stride, hipStream_t st)
{
    return launch_fwd<float>(pl, x, nullptr, rt, out_stride, st);
}

// xb non-null: gather from the bf16 copy (mixed path)
hipError_t launch_project(const mpi3d_plan *pl, const float *x, const uint16_t *xb, float *rt, hipStream_t st)
{
    if (xb) return launch_fwd<uint32_t>(pl, nullptr, xb, rt, pl->nup, st);
    return launch_fwd<float>(pl, x, nullptr, rt, pl->nup, st);
}

hipError_t launch_backproject_strided(const mpi3d_plan *pl, const float *rt, int in_stride, float *xo,
                                      const float *x_sub, double lambda, double *norm_parts, int *nparts,
                                      hipStream_t st, const float *x_add)
{
    ProjArgs a = base_args(pl);
    a.rt_in = rt;
    a.xo = xo;
    a.x_sub = x_sub;
    a.x_add = x_add;
    a.lambda = lambda;
    a.norm_parts = norm_parts;
    const int blocks = a.tiles_x * a.tiles_y * a.n_zgroups;
    if (nparts) *nparts = blocks;
    if (norm_parts && blocks > kMaxNormParts) return hipErrorInvalidValue;
    hipLaunchKernelGGL(proj_adj_kernel, dim3(blocks), dim3(256), 0, st, a, in_stride);
    return hipGetLastError();
}

hipError_t launch_backproject(const mpi3d_plan *pl, const float *rt, float *xo, const float *x_sub, double lambda,
                              double *norm_parts, int *nparts, hipStream_t st, const float *x_add)
{
    return launch_backproject_strided(pl, rt, pl->nup, xo, x_sub, lambda, norm_parts, nparts, st, x_add);
}

}  // namespace mpi3d
