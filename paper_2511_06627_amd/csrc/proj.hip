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

// A sample known to lie kEdge inside the staged band (no test): fx in LDS
// columns, fyb in band rows.  floor() via fract, exact for positive values;
// the element index iy * W + ix is formed exactly in float.
constexpr float kEdge = 1.0f / 64.0f;
constexpr float kRange = 1.0f / 1024.0f;

template <typename T>
__device__ __forceinline__ float sample_in(const T *lds, int W, float bx, float byb, float s, float c, float y)
{
    const float fx = fmaf(y, s, bx), fy = fmaf(y, c, byb);
    const float wx = __builtin_amdgcn_fractf(fx), wy = __builtin_amdgcn_fractf(fy);
    const int e = (int)fmaf(fy - wy, (float)W, fx - wx);
    float v00, v10, v01, v11;
    corners(lds + e, W, v00, v10, v01, v11);
    const float top = fmaf(wx, v10 - v00, v00);
    const float bot = fmaf(wx, v11 - v01, v01);
    return fmaf(wy, bot - top, top);
}

// Four consecutive interior samples y, y+1, y+2, y+3: all LDS reads are
// issued before any is used.
template <typename T>
__device__ __forceinline__ float sample_in4(const T *lds, int W, float bx, float byb, float s, float c, float y)
{
    float wx[4], wy[4], v[4][4];
    int e[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float fx = fmaf(y + (float)j, s, bx), fy = fmaf(y + (float)j, c, byb);
        wx[j] = __builtin_amdgcn_fractf(fx);
        wy[j] = __builtin_amdgcn_fractf(fy);
        e[j] = (int)fmaf(fy - wy[j], (float)W, fx - wx[j]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) corners(lds + e[j], W, v[j][0], v[j][1], v[j][2], v[j][3]);
    float r[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float top = fmaf(wx[j], v[j][1] - v[j][0], v[j][0]);
        const float bot = fmaf(wx[j], v[j][3] - v[j][2], v[j][2]);
        r[j] = fmaf(wy[j], bot - top, top);
    }
    return (r[0] + r[1]) + (r[2] + r[3]);
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
    // The (slice, angle) units k * M + m are dealt to the blocks in equal
    // contiguous ranges: a block stages each slice its range touches once and
    // projects that slice for its angles there.
    const long U = (long)a.nz * a.M;
    const long u0 = (long)lb * U / nb, u1 = (long)(lb + 1) * U / nb;
    const int W = a.nx + 2;
    const int tid = threadIdx.x;
    for (long ku = u0; ku < u1;) {
        const int k = (int)(ku / a.M);
        const int m0 = (int)(ku - (long)k * a.M);
        const int m1 = (int)min((long)a.M, u1 - (long)k * a.M);
        ku = (long)k * a.M + m1;
        const int nrays = (m1 - m0) * a.nu;
        float acc[kMaxRaysPerThread];
#pragma unroll
        for (int r = 0; r < kMaxRaysPerThread; ++r) acc[r] = 0.f;
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
                // [q0, q1] is a widened superset of the samples in the band (each
                // checked exactly): the edges are moved out by kRange in fx and fy,
                // beyond the rounding of fx and fy themselves, so a ray that runs
                // along a band edge (|c| tiny, fy rounding onto the edge row) keeps
                // all its samples; inside it, [qa, qb] holds samples
                // at least kEdge away from every edge in both coordinates, which
                // need no test: there the band-relative row fy - jb0 lies in
                // [kEdge, nbase - kEdge] and fx in [kEdge, nx + 1 - kEdge].
                const float byb = by - (float)jb0;
                float ylo = -a.half_nr, yhi = a.half_nr;
                float ilo = -a.half_nr, ihi = a.half_nr;
                if (s > 0.f) {
                    ylo = fmaxf(ylo, (-kRange - bx) / s);
                    yhi = fminf(yhi, ((float)(a.nx + 1) + kRange - bx) / s);
                    ilo = fmaxf(ilo, (kEdge - bx) / s);
                    ihi = fminf(ihi, ((float)(a.nx + 1) - kEdge - bx) / s);
                } else if (bx < kEdge || bx > (float)(a.nx + 1) - kEdge) {
                    ihi = ilo - 2.f;
                }
                if (c > 0.f) {
                    ylo = fmaxf(ylo, ((float)jb0 - kRange - by) / c);
                    yhi = fminf(yhi, ((float)jb1 + kRange - by) / c);
                    ilo = fmaxf(ilo, (kEdge - byb) / c);
                    ihi = fminf(ihi, ((float)nbase - kEdge - byb) / c);
                } else if (c < 0.f) {
                    ylo = fmaxf(ylo, ((float)jb1 + kRange - by) / c);
                    yhi = fminf(yhi, ((float)jb0 - kRange - by) / c);
                    ilo = fmaxf(ilo, ((float)nbase - kEdge - byb) / c);
                    ihi = fminf(ihi, (kEdge - byb) / c);
                } else if (byb < kEdge || byb > (float)nbase - kEdge) {
                    ihi = ilo - 2.f;
                }
                const int q0 = max(0, (int)floorf(ylo + a.half_nr) - 1);
                const int q1 = min(a.nr - 1, (int)ceilf(yhi + a.half_nr) + 1);
                int qa = max(q0, (int)ceilf(ilo + a.half_nr));
                int qb = min(q1, (int)floorf(ihi + a.half_nr));
                if (qa > qb) {   // no interior: every sample checked
                    qa = q1 + 1;
                    qb = q1;
                }
                float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
                for (int q = q0; q < qa; ++q) s0 += sample(lds, W, a.nx, nbase, jb0, bx, by, s, c, (float)q - a.half_nr);
                // interior, four samples at a time with their LDS reads in flight together
                int q = qa;
                for (; q + 3 <= qb; q += 4) s3 += sample_in4(lds, W, bx, byb, s, c, (float)q - a.half_nr);
                for (; q <= qb; ++q) s1 += sample_in(lds, W, bx, byb, s, c, (float)q - a.half_nr);
                for (q = max(qb + 1, qa); q <= q1; ++q)
                    s2 += sample(lds, W, a.nx, nbase, jb0, bx, by, s, c, (float)q - a.half_nr);
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
}

constexpr int kTile = 16;
constexpr int kPW = 32;     // staged rays per angle per tile

__device__ __forceinline__ float hat(float t) { return fmaxf(0.f, 1.f - fabsf(t)); }

// First staged detector index of angle (c, s) for the tile whose voxel-centre
// corners are (X0, Y0) .. (X0 + 15, Y0 + 15): u is linear in X and Y, so its
// minimum over the tile is at a corner; 2 rays of margin absorb the rounding
// between that minimum and any voxel's own u.
__device__ __forceinline__ int tile_p_lo(float c, float s, float X0, float Y0, float half_nu)
{
    const float X1 = X0 + (float)(kTile - 1), Y1 = Y0 + (float)(kTile - 1);
    const float u00 = X0 * c - Y0 * s, u10 = X1 * c - Y0 * s, u01 = X0 * c - Y1 * s, u11 = X1 * c - Y1 * s;
    return (int)floorf(fminf(fminf(u00, u10), fminf(u01, u11)) + half_nu) - 2;
}

// One block: a 16 x 16 voxel tile times KZ slices.  Angles are taken in
// chunks of a.adj_chunk: all lines a chunk needs (per angle KZ lines x 32
// rays) are staged in LDS in one pass, then every voxel accumulates the
// chunk's angles without further barriers.
template <int KZ>
__global__ __launch_bounds__(256) void proj_adj_kernel(ProjArgs a, int in_stride)
{
    extern __shared__ __align__(16) float gs[];   // [chunk][KZ][kPW], then p_lo per angle
    __shared__ double red[256 / 64];
    int *plo = reinterpret_cast<int *>(gs + (size_t)a.adj_chunk * KZ * kPW);
    const int nb = gridDim.x;
    const int lb = xcd_logical(blockIdx.x, nb);
    const int zg = lb / (a.tiles_x * a.tiles_y);
    const int tile = lb % (a.tiles_x * a.tiles_y);
    const int tx0 = (tile % a.tiles_x) * kTile, ty0 = (tile / a.tiles_x) * kTile;
    const int k0 = zg * KZ;
    const int kn = min(KZ, a.nz - k0);
    const int tid = threadIdx.x;
    const int i = tx0 + (tid % kTile), j = ty0 + (tid / kTile);
    const bool valid = i < a.nx && j < a.ny;
    const float X = (float)i - a.cx, Y = (float)j - a.cy;
    const float X0 = (float)tx0 - a.cx, Y0 = (float)ty0 - a.cy;

    float acc[KZ];
#pragma unroll
    for (int kk = 0; kk < KZ; ++kk) acc[kk] = 0.f;

    for (int mb = 0; mb < a.M; mb += a.adj_chunk) {
        const int mc = min(a.adj_chunk, a.M - mb);
        __syncthreads();                       // the previous chunk is consumed
        if (tid < mc) {
            const float2 csv = a.cs[mb + tid];
            plo[tid] = tile_p_lo(csv.x, csv.y, X0, Y0, a.half_nu);
        }
        __syncthreads();
        for (int idx = tid; idx < mc * KZ * kPW; idx += 256) {
            const int mm = idx / (KZ * kPW);
            const int rem = idx - mm * (KZ * kPW);
            const int kk = rem / kPW, pp = rem % kPW;
            const int p = plo[mm] + pp;
            float v = 0.f;
            if (kk < kn && p >= 0 && p < a.nu) v = a.rt_in[((size_t)(mb + mm) * a.nz + k0 + kk) * in_stride + p];
            gs[idx] = v;
        }
        __syncthreads();
        if (!valid) continue;
        for (int mm = 0; mm < mc; ++mm) {
            const float2 csv = a.cs[mb + mm];
            const float c = csv.x, s = csv.y;
            // voxel position in (detector, ray-sample) index coordinates
            const float u = fmaf(X, c, -Y * s) + a.half_nu;
            const float yv = fmaf(X, s, Y * c) + a.half_nr;
            const float pc = rintf(u), qc = rintf(yv);
            // displacement from the voxel to sample (pc + dp, qc + dq) in grid
            // coordinates: (dX0 + dp c + dq s, dY0 + dq c - dp s)
            const float du = pc - u, dy = qc - yv;
            const float dX0 = fmaf(du, c, dy * s), dY0 = fmaf(dy, c, -du * s);
            float w[3];
#pragma unroll
            for (int dp = 0; dp < 3; ++dp) {
                const float pf = pc + (float)(dp - 1);
                float wp = 0.f;
#pragma unroll
                for (int dq = 0; dq < 3; ++dq) {
                    const float qf = qc + (float)(dq - 1);
                    const float dX = fmaf((float)(dq - 1), s, fmaf((float)(dp - 1), c, dX0));
                    const float dY = fmaf((float)(dq - 1), c, fmaf((float)(1 - dp), s, dY0));
                    const bool qok = qf >= 0.f && qf <= (float)(a.nr - 1);
                    wp += qok ? hat(dX) * hat(dY) : 0.f;
                }
                const bool pok = pf >= 0.f && pf <= (float)(a.nu - 1);
                w[dp] = pok ? wp : 0.f;
            }
            const int off = min(max((int)pc - 1 - plo[mm], 0), kPW - 3);  // in range by construction
            const float *g0 = gs + (size_t)mm * KZ * kPW + off;
#pragma unroll
            for (int kk = 0; kk < KZ; ++kk) {
                const float *gk = g0 + kk * kPW;
                acc[kk] = fmaf(w[0], gk[0], fmaf(w[1], gk[1], fmaf(w[2], gk[2], acc[kk])));
            }
        }
    }

    double sq = 0.0;
    if (valid) {
#pragma unroll
        for (int kk = 0; kk < KZ; ++kk) {
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
    a.band_rows = pl->band_rows;
    a.n_bands = pl->n_bands;
    a.kz = pl->kz;
    a.adj_chunk = pl->adj_chunk;
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
    const int blocks = pl->fwd_blocks;
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
    if (norm_parts && blocks > pl->max_parts) return hipErrorInvalidValue;
    const size_t lds = sizeof(float) * (size_t)a.adj_chunk * a.kz * kPW + sizeof(int) * a.adj_chunk;
    switch (a.kz) {
    case 8: hipLaunchKernelGGL(proj_adj_kernel<8>, dim3(blocks), dim3(256), lds, st, a, in_stride); break;
    case 16: hipLaunchKernelGGL(proj_adj_kernel<16>, dim3(blocks), dim3(256), lds, st, a, in_stride); break;
    case 32: hipLaunchKernelGGL(proj_adj_kernel<32>, dim3(blocks), dim3(256), lds, st, a, in_stride); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_backproject(const mpi3d_plan *pl, const float *rt, float *xo, const float *x_sub, double lambda,
                              double *norm_parts, int *nparts, hipStream_t st, const float *x_add)
{
    return launch_backproject_strided(pl, rt, pl->nup, xo, x_sub, lambda, norm_parts, nparts, st, x_add);
}

}  // namespace mpi3d
