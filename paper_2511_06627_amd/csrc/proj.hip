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

#include "device.h"

namespace mpi3d {

namespace {

// A ray sample's 2x2 footprint is the same in every z-slice, so a unit of
// work may cover NS consecutive slices k0 .. k0 + NS - 1 whose values share
// one staged texel (LDS column col = grid column col - 1): every address and
// bilinear weight is then formed once for all of them.  Texel types:
//  float    fp32, one slice;
//  float2   fp32, two slices {x[k0], x[k0 + 1]} (when a slice pair fits in LDS
//           in one band: row bands split the rays of a wave unevenly);
//  uint32_t bf16 (the mixed operator's gathers), two slices: low half the
//           bf16 voxel of k0, high half that of k0 + 1.
// A missing last slice (odd nz) is staged as zeros and never stored.
template <typename T>
struct Texel;
template <>
struct Texel<float> {
    static constexpr int NS = 1;
    using V = float;
};
template <>
struct Texel<float2> {
    static constexpr int NS = 2;
    using V = float;
};
template <>
struct Texel<uint32_t> {
    static constexpr int NS = 2;
    using V = uint16_t;
};

__device__ __forceinline__ void load(const float *p, float (&v)[1]) { v[0] = *p; }

__device__ __forceinline__ void load(const float2 *p, float (&v)[2])
{
    const float2 q = *p;
    v[0] = q.x;
    v[1] = q.y;
}

__device__ __forceinline__ void load(const uint32_t *p, float (&v)[2])
{
    const uint32_t w = *p;
    v[0] = __uint_as_float(w << 16);
    v[1] = __uint_as_float(w & 0xffff0000u);
}

// The 2x2 footprint whose corner (0,0) is the texel at p: t[0] = (0,0),
// t[1] = (1,0), t[2] = (0,1), t[3] = (1,1).
template <typename T, int NS>
__device__ __forceinline__ void fetch(const T *p, int W, float (&t)[4][NS])
{
    load(p, t[0]);
    load(p + 1, t[1]);
    load(p + W, t[2]);
    load(p + W + 1, t[3]);
}

// Staging.  LDS row r of a band holds grid row jb0 + r and LDS column col
// holds grid column col - 1; columns 0 and nx + 1 .. W - 1 are zero borders,
// written once per block.  A thread stages runs of VW consecutive voxels of
// one row (VW = 4 where every row start is aligned to a VW-voxel vector load,
// else 1), U runs at a time with all their global loads issued before the
// first LDS store: a band then costs a few memory latencies, not one per
// texel.
template <typename V, int VW>
struct Run {
    V v[VW];
};

template <typename V, int VW>
__device__ __forceinline__ Run<V, VW> load_run(const V *p)
{
    Run<V, VW> r;
    if constexpr (VW == 1) {
        r.v[0] = *p;
    } else {
        typedef V vec __attribute__((ext_vector_type(VW)));
        const vec q = *reinterpret_cast<const vec *>(p);
#pragma unroll
        for (int j = 0; j < VW; ++j) r.v[j] = q[j];
    }
    return r;
}

// The texel of voxel j of the runs a (slice k0) and b (slice k0 + 1); a
// run not in the grid (ia / ib false) contributes zeros.
template <typename T, typename V, int VW>
__device__ __forceinline__ T make_texel(const Run<V, VW> &ra, const Run<V, VW> &rb, bool ia, bool ib, int j)
{
    if constexpr (std::is_same_v<T, float>) {
        return ia ? ra.v[j] : 0.f;
    } else if constexpr (std::is_same_v<T, float2>) {
        return make_float2(ia ? ra.v[j] : 0.f, ib ? rb.v[j] : 0.f);
    } else {
        return (ia ? (uint32_t)ra.v[j] : 0u) | ((ib ? (uint32_t)rb.v[j] : 0u) << 16);
    }
}

// Stages LDS rows 0 .. rows - 1 (grid rows jb0 ..) of the slice group (s0,
// s1; s1 is read only where has1), LDS columns 1 .. nx.  Thread tid starts
// at run (r0, c0) of the row-major run order and steps by kFwdThreads runs,
// (dr, dc) rows and runs at a time.
template <typename T, int VW, int U>
__device__ __forceinline__ void stage_band(T *lds, const typename Texel<T>::V *s0, const typename Texel<T>::V *s1,
                                           bool has1, int nx, int ny, int W, int jb0, int rows, int r0, int c0,
                                           int dr, int dc, int tid)
{
    using V = typename Texel<T>::V;
    constexpr int NS = Texel<T>::NS;
    const int runs = nx / VW;
    const int total = rows * runs;
    int r = r0, c = c0;
    for (int e0 = tid; e0 < total; e0 += U * kFwdThreads) {
        Run<V, VW> ra[U], rb[U];
        int dst[U];
        bool in[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int gj = jb0 + r;
            const bool live = e0 + u * kFwdThreads < total;
            in[u] = live && (unsigned)gj < (unsigned)ny;
            // out-of-grid runs load row 0 of the slice (in bounds) and are dropped
            const size_t off = (size_t)(in[u] ? gj : 0) * nx + (size_t)c * VW;
            ra[u] = load_run<V, VW>(s0 + off);
            if constexpr (NS == 2) rb[u] = load_run<V, VW>((has1 ? s1 : s0) + off);
            dst[u] = live ? r * W + 1 + c * VW : -1;
            c += dc;
            r += dr;
            if (c >= runs) {
                c -= runs;
                ++r;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (dst[u] < 0) continue;
#pragma unroll
            for (int j = 0; j < VW; ++j) lds[dst[u] + j] = make_texel<T, V, VW>(ra[u], rb[u], in[u], in[u] && has1, j);
        }
    }
}

// Adds the bilinear interpolant of the footprint t at fractional offsets
// (wx, wy) to acc.  One slice: the three-lerp form.  Two slices: the corner
// weights (1-wx)(1-wy), wx(1-wy), (1-wx)wy, wx wy, formed once in five
// operations and shared.
template <int NS>
__device__ __forceinline__ void accum(float (&acc)[NS], const float (&t)[4][NS], float wx, float wy)
{
    if constexpr (NS == 1) {
        const float top = fmaf(wx, t[1][0] - t[0][0], t[0][0]);
        const float bot = fmaf(wx, t[3][0] - t[2][0], t[2][0]);
        acc[0] += fmaf(wy, bot - top, top);
    } else {
        const float w11 = wx * wy, w10 = wx - w11, w01 = wy - w11, w00 = (1.f - wx) - w01;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            acc[k] = fmaf(t[0][k], w00, acc[k]);
            acc[k] = fmaf(t[1][k], w10, acc[k]);
            acc[k] = fmaf(t[2][k], w01, acc[k]);
            acc[k] = fmaf(t[3][k], w11, acc[k]);
        }
    }
}

// One bilinear sample of the staged band, tested.  Branch-free: a sample whose
// 2x2 footprint lies outside the band reads a safe LDS address with zero
// weights.
template <typename T, int NS>
__device__ __forceinline__ void sample(const T *lds, int W, int nx, int nbase, int jb0, float bx, float by, float s,
                                       float c, float y, float (&acc)[NS])
{
    const float fx = fmaf(y, s, bx), fy = fmaf(y, c, by);
    const float ix = floorf(fx), iy = floorf(fy);
    int i0 = (int)ix, j0 = (int)iy - jb0;
    const bool ok = (unsigned)i0 <= (unsigned)nx && (unsigned)j0 < (unsigned)nbase;
    i0 = ok ? i0 : 0;
    j0 = ok ? j0 : 0;
    float t[4][NS];
    fetch(lds + j0 * W + i0, W, t);
    float v[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) v[k] = 0.f;
    accum(v, t, fx - ix, fy - iy);
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] += ok ? v[k] : 0.f;
}

// Samples known to lie kEdge inside the staged band need no test: there fx
// (in LDS columns) and fyb (in band rows) are positive, so floor is the
// truncating conversion of the value and the fraction is fract().
constexpr float kEdge = 1.0f / 64.0f;
constexpr float kRange = 1.0f / 1024.0f;

// The texel at (column fx, band row fyb), both positive.  Wb = W * sizeof(T).
template <typename T>
__device__ __forceinline__ const T *texel_at(const T *lds, unsigned Wb, float fx, float fyb)
{
    const unsigned off = __umul24((unsigned)fyb, Wb) + (unsigned)fx * (unsigned)sizeof(T);
    return reinterpret_cast<const T *>(reinterpret_cast<const unsigned char *>(lds) + off);
}

// Four consecutive interior samples y, y+1, y+2, y+3: all LDS reads are
// issued before any is used.
template <typename T, int NS>
__device__ __forceinline__ void sample_in4(const T *lds, int W, unsigned Wb, float bx, float byb, float s, float c,
                                           float y, float (&acc)[NS])
{
    float wx[4], wy[4];
    const T *p[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float fx = fmaf(y + (float)j, s, bx), fy = fmaf(y + (float)j, c, byb);
        wx[j] = __builtin_amdgcn_fractf(fx);
        wy[j] = __builtin_amdgcn_fractf(fy);
        p[j] = texel_at(lds, Wb, fx, fy);
    }
    float t[4][4][NS];
#pragma unroll
    for (int j = 0; j < 4; ++j) fetch(p[j], W, t[j]);
#pragma unroll
    for (int j = 0; j < 4; ++j) accum(acc, t[j], wx[j], wy[j]);
}

template <typename T, int NS>
__device__ __forceinline__ void sample_in(const T *lds, int W, unsigned Wb, float bx, float byb, float s, float c,
                                          float y, float (&acc)[NS])
{
    const float fx = fmaf(y, s, bx), fy = fmaf(y, c, byb);
    float t[4][NS];
    fetch(texel_at(lds, Wb, fx, fy), W, t);
    accum(acc, t, __builtin_amdgcn_fractf(fx), __builtin_amdgcn_fractf(fy));
}

// T: the texel type above; weights and sums are fp32.
template <typename T>
__global__ __launch_bounds__(kFwdThreads) void proj_fwd_kernel(ProjArgs a, const typename Texel<T>::V *vol,
                                                               int out_stride)
{
    using V = typename Texel<T>::V;
    constexpr int NS = Texel<T>::NS;
    constexpr int kMaxRaysPerThread = fwd_rays_per_thread(NS);
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *lds = reinterpret_cast<T *>(lds_raw);
    const int nb = gridDim.x;
    const int lb = xcd_logical(blockIdx.x, nb);
    // The (slice group, angle) units g * M + m are dealt to the blocks in equal
    // contiguous ranges: a block stages each slice group its range touches
    // once and projects that group for its angles there.
    const int ng = (a.nz + NS - 1) / NS;
    const long U = (long)ng * a.M;
    const long u0 = (long)lb * U / nb, u1 = (long)(lb + 1) * U / nb;
    const int W = proj_pitch(a.nx);
    const unsigned Wb = (unsigned)(W * sizeof(T));
    const int tid = threadIdx.x;
    // zero borders of every LDS row a band uses
    const int border = W - a.nx;
    for (int idx = tid; idx < (a.band_rows + 1) * border; idx += kFwdThreads) {
        const int r = idx / border, b = idx - r * border;
        lds[r * W + (b == 0 ? 0 : a.nx + b)] = T{};
    }
    // run positions of this thread for the vector (4 voxels) and scalar stagings
    const bool vec = a.nx % 4 == 0 && reinterpret_cast<uintptr_t>(vol) % (4 * sizeof(V)) == 0;
    const int v_runs = max(1, a.nx / 4), s_runs = a.nx;
    const int v_r0 = tid / v_runs, v_c0 = tid - v_r0 * v_runs, v_dr = kFwdThreads / v_runs,
              v_dc = kFwdThreads - v_dr * v_runs;
    const int s_r0 = tid / s_runs, s_c0 = tid - s_r0 * s_runs, s_dr = kFwdThreads / s_runs,
              s_dc = kFwdThreads - s_dr * s_runs;
    for (long ku = u0; ku < u1;) {
        const int g = (int)(ku / a.M);
        const int m0 = (int)(ku - (long)g * a.M);
        const int m1 = (int)min((long)a.M, u1 - (long)g * a.M);
        ku = (long)g * a.M + m1;
        const int k0 = NS * g;
        const int ns = min(NS, a.nz - k0);     // slices present in the group
        const int nrays = (m1 - m0) * a.nu;
        float acc[kMaxRaysPerThread][NS];
#pragma unroll
        for (int r = 0; r < kMaxRaysPerThread; ++r)
#pragma unroll
            for (int k = 0; k < NS; ++k) acc[r][k] = 0.f;
        const V *s0 = vol + (size_t)k0 * a.nx * a.ny;
        const V *s1 = s0 + (size_t)(ns > 1 ? a.nx * a.ny : 0);
        for (int band = 0; band < a.n_bands; ++band) {
            const int jb0 = -1 + band * a.band_rows;               // first base row
            const int jb1 = min(jb0 + a.band_rows, a.ny);          // one past last base row
            const int nbase = jb1 - jb0;
            const int rows = nbase + 1;                            // LDS rows: grid rows jb0..jb1
            __syncthreads();
            if (vec)
                stage_band<T, 4, (NS == 2 && sizeof(V) == 4 ? 4 : 8)>(lds, s0, s1, ns > 1, a.nx, a.ny, W, jb0, rows,
                                                                       v_r0, v_c0, v_dr, v_dc, tid);
            else
                stage_band<T, 1, 8>(lds, s0, s1, ns > 1, a.nx, a.ny, W, jb0, rows, s_r0, s_c0, s_dr, s_dc, tid);
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
                // all its samples; inside it, [qa, qb] holds samples at least kEdge
                // away from every edge in both coordinates, which need no test:
                // there the band-relative row fy - jb0 lies in [kEdge, nbase - kEdge]
                // and fx in [kEdge, nx + 1 - kEdge].  The bounds are solved with one
                // reciprocal per direction; its relative error (a few ulp, so below
                // 1e-4 samples over any ray) is far inside both margins.
                const float byb = by - (float)jb0;
                float ylo = -a.half_nr, yhi = a.half_nr;
                float ilo = -a.half_nr, ihi = a.half_nr;
                if (s > 0.f) {
                    const float rs = 1.f / s;
                    ylo = fmaxf(ylo, (-kRange - bx) * rs);
                    yhi = fminf(yhi, ((float)(a.nx + 1) + kRange - bx) * rs);
                    ilo = fmaxf(ilo, (kEdge - bx) * rs);
                    ihi = fminf(ihi, ((float)(a.nx + 1) - kEdge - bx) * rs);
                } else if (bx < kEdge || bx > (float)(a.nx + 1) - kEdge) {
                    ihi = ilo - 2.f;
                }
                if (c != 0.f) {
                    const float rc = 1.f / c;
                    const float e0 = ((float)jb0 - kRange - by) * rc, e1 = ((float)jb1 + kRange - by) * rc;
                    const float i0 = (kEdge - byb) * rc, i1 = ((float)nbase - kEdge - byb) * rc;
                    ylo = fmaxf(ylo, fminf(e0, e1));
                    yhi = fminf(yhi, fmaxf(e0, e1));
                    ilo = fmaxf(ilo, fminf(i0, i1));
                    ihi = fminf(ihi, fmaxf(i0, i1));
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
                float sa[NS], sb[NS];
#pragma unroll
                for (int k = 0; k < NS; ++k) sa[k] = sb[k] = 0.f;
                for (int q = q0; q < qa; ++q) sample(lds, W, a.nx, nbase, jb0, bx, by, s, c, (float)q - a.half_nr, sa);
                // interior, four samples at a time with their LDS reads in flight together
                int q = qa;
                for (; q + 3 <= qb; q += 4) sample_in4(lds, W, Wb, bx, byb, s, c, (float)q - a.half_nr, sb);
                for (; q <= qb; ++q) sample_in(lds, W, Wb, bx, byb, s, c, (float)q - a.half_nr, sb);
                for (q = max(qb + 1, qa); q <= q1; ++q)
                    sample(lds, W, a.nx, nbase, jb0, bx, by, s, c, (float)q - a.half_nr, sa);
#pragma unroll
                for (int k = 0; k < NS; ++k) acc[i][k] += sa[k] + sb[k];
            }
        }
#pragma unroll
        for (int i = 0; i < kMaxRaysPerThread; ++i) {
            const int ray = tid + kFwdThreads * i;
            if (ray >= nrays) continue;
            const int m = m0 + ray / a.nu, p = ray % a.nu;
            float *o = a.rt + ((size_t)m * a.nz + k0) * out_stride + p;
#pragma unroll
            for (int k = 0; k < NS; ++k)
                if (k < ns) o[(size_t)k * out_stride] = acc[i][k];
        }
        // zero the padding columns of the lines this block owns
        if (out_stride > a.nu) {
            const int pad = out_stride - a.nu;
            const int nl = (m1 - m0) * ns;
            for (int idx = tid; idx < nl * pad; idx += kFwdThreads) {
                const int l = idx / pad;
                const int m = m0 + l / ns, k = k0 + l % ns, p = a.nu + idx % pad;
                a.rt[((size_t)m * a.nz + k) * out_stride + p] = 0.f;
            }
        }
    }
}

constexpr int kTile = 16;
constexpr int kPW = 32;     // staged rays per angle per tile
constexpr int kAdjStage = 8;   // staged entries per thread per round of loads

// The fp16 values in the low and high halves of a 32-bit word, as fp32.
__device__ __forceinline__ float half_lo(uint32_t w)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
}
__device__ __forceinline__ float half_hi(uint32_t w)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
}

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
// chunk's angles without further barriers.  H: the lines are fp16 with a
// power-of-two scale per line (the mixed operator's gathers); a staged 32-bit
// word holds the values of two consecutive z-slices, so one LDS read serves
// both, and each line's inverse scale multiplies its three-sample sum.
// Weights and sums are fp32.
template <int KZ, bool H>
__device__ __forceinline__ void adj_body(const ProjArgs &a, const uint16_t *__restrict__ rtb,
                                         const float *__restrict__ rtsc, int in_stride)
{
    // LDS: staged lines [chunk][KZ][kPW] floats, or [chunk][KZ/2][kPW] words
    // and the lines' inverse scales [chunk][KZ]; then p_lo per angle
    extern __shared__ __align__(16) float gs[];
    __shared__ double red[256 / 64];
    constexpr int KW = H ? KZ / 2 : KZ;           // staged rows per angle
    uint32_t *gw = reinterpret_cast<uint32_t *>(gs);
    float *isc = gs + (size_t)a.adj_chunk * KW * kPW;
    int *plo = reinterpret_cast<int *>(isc + (H ? (size_t)a.adj_chunk * KZ : 0));
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
        if constexpr (H) {
            for (int idx = tid; idx < mc * KZ; idx += 256) {
                const int mm = idx / KZ, kk = idx - mm * KZ;
                isc[idx] = kk < kn ? rtsc[(size_t)(mb + mm) * a.nz + k0 + kk] : 0.f;
            }
        }
        __syncthreads();
        if constexpr (H) {
            for (int idx = tid; idx < mc * KW * kPW; idx += 256) {
                const int mm = idx / (KW * kPW);
                const int rem = idx - mm * (KW * kPW);
                const int kw = rem / kPW, pp = rem % kPW;
                const int p = plo[mm] + pp;
                const bool pin = p >= 0 && p < a.nu;
                const int kk = 2 * kw;
                const size_t base = ((size_t)(mb + mm) * a.nz + k0 + kk) * in_stride + p;
                const uint32_t lo = (kk < kn && pin) ? (uint32_t)rtb[base] : 0u;
                const uint32_t hi = (kk + 1 < kn && pin) ? (uint32_t)rtb[base + in_stride] : 0u;
                gw[idx] = lo | (hi << 16);
            }
        } else {
            // kAdjStage entries per thread at a time, all loads issued before
            // the first LDS store (an entry outside the lines reads line 0 and
            // stores zero).  Stores are unconditional so the loads stay
            // together: a slot past the end repeats the last entry, value
            // included.
            const int total = mc * KW * kPW;
            for (int idx0 = tid; idx0 < total; idx0 += 256 * kAdjStage) {
                float v[kAdjStage];
                bool ok[kAdjStage];
#pragma unroll
                for (int u = 0; u < kAdjStage; ++u) {
                    const int idx = min(idx0 + 256 * u, total - 1);
                    const int mm = idx / (KW * kPW);
                    const int rem = idx - mm * (KW * kPW);
                    const int kw = rem / kPW, pp = rem % kPW;
                    const int p = plo[mm] + pp;
                    const size_t base = ((size_t)(mb + mm) * a.nz + k0 + kw) * in_stride + p;
                    ok[u] = p >= 0 && p < a.nu && kw < kn;
                    v[u] = a.rt_in[ok[u] ? base : 0];
                }
#pragma unroll
                for (int u = 0; u < kAdjStage; ++u) gs[min(idx0 + 256 * u, total - 1)] = ok[u] ? v[u] : 0.f;
            }
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
            if constexpr (H) {
                const uint32_t *g0 = gw + (size_t)mm * KW * kPW + off;
                const float *sc = isc + (size_t)mm * KZ;
#pragma unroll
                for (int kw = 0; kw < KW; ++kw) {
                    const uint32_t *gk = g0 + kw * kPW;
                    const uint32_t v0 = gk[0], v1 = gk[1], v2 = gk[2];
                    const float lo = fmaf(w[0], half_lo(v0), fmaf(w[1], half_lo(v1), w[2] * half_lo(v2)));
                    const float hi = fmaf(w[0], half_hi(v0), fmaf(w[1], half_hi(v1), w[2] * half_hi(v2)));
                    acc[2 * kw] = fmaf(lo, sc[2 * kw], acc[2 * kw]);
                    acc[2 * kw + 1] = fmaf(hi, sc[2 * kw + 1], acc[2 * kw + 1]);
                }
            } else {
                const float *g0 = gs + (size_t)mm * KZ * kPW + off;
#pragma unroll
                for (int kk = 0; kk < KZ; ++kk) {
                    const float *gk = g0 + kk * kPW;
                    acc[kk] = fmaf(w[0], gk[0], fmaf(w[1], gk[1], fmaf(w[2], gk[2], acc[kk])));
                }
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

template <int KZ>
__global__ __launch_bounds__(256) void proj_adj_kernel(ProjArgs a, int in_stride)
{
    adj_body<KZ, false>(a, nullptr, nullptr, in_stride);
}

template <int KZ>
__global__ __launch_bounds__(256) void proj_adj_f16(ProjArgs a, const uint16_t *rtb, const float *rtsc, int in_stride)
{
    adj_body<KZ, true>(a, rtb, rtsc, in_stride);
}

// Dual drive: z-drive line (m, p) of the workspace (line Lx + m*nu + p) holds
// column p of the projections of angle m across the z-rows, zero beyond nz.
// One block moves a 32 x 32 tile (rows k, columns p) of one angle through LDS
// so both the read and the write are row-contiguous.
constexpr int kTr = 32;

__global__ __launch_bounds__(256) void zlines_kernel(float *rt, int nz, int nu, int nup, long Lx)
{
    __shared__ float tile[kTr][kTr + 1];
    const int m = blockIdx.z, k0 = blockIdx.y * kTr, p0 = blockIdx.x * kTr;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
    for (int j = ty; j < kTr; j += 8) {
        const int k = k0 + j, p = p0 + tx;
        tile[j][tx] = (k < nz && p < nu) ? rt[((size_t)m * nz + k) * nup + p] : 0.f;
    }
    __syncthreads();
    for (int j = ty; j < kTr; j += 8) {
        const int p = p0 + j, k = k0 + tx;
        if (p < nu && k < nup) rt[(size_t)(Lx + (long)m * nu + p) * nup + k] = tile[tx][j];
    }
}

// Transpose of zlines_kernel, added: x-drive line (m, k), column p gains
// element k of z-drive line (m, p).
__global__ __launch_bounds__(256) void fold_zlines_kernel(float *rt, int nz, int nu, int nup, long Lx)
{
    __shared__ float tile[kTr][kTr + 1];
    const int m = blockIdx.z, k0 = blockIdx.y * kTr, p0 = blockIdx.x * kTr;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int j = ty; j < kTr; j += 8) {
        const int p = p0 + j, k = k0 + tx;
        tile[j][tx] = (p < nu && k < nz) ? rt[(size_t)(Lx + (long)m * nu + p) * nup + k] : 0.f;
    }
    __syncthreads();
    for (int j = ty; j < kTr; j += 8) {
        const int k = k0 + j, p = p0 + tx;
        if (k < nz && p < nu) rt[((size_t)m * nz + k) * nup + p] += tile[tx][j];
    }
}

}  // namespace

static hipError_t launch_zlines(const mpi3d_plan *pl, float *rt, bool fold, hipStream_t st)
{
    // z-drive lines have nup entries (nz used), so the tiles cover nup rows k
    // when writing them and nz when folding back
    const int krows = fold ? pl->nz : pl->nup;
    const dim3 grid((pl->nu + kTr - 1) / kTr, (krows + kTr - 1) / kTr, pl->M);
    if (fold)
        hipLaunchKernelGGL(fold_zlines_kernel, grid, dim3(256), 0, st, rt, pl->nz, pl->nu, pl->nup, pl->Lx);
    else
        hipLaunchKernelGGL(zlines_kernel, grid, dim3(256), 0, st, rt, pl->nz, pl->nu, pl->nup, pl->Lx);
    return hipGetLastError();
}

static ProjArgs base_args(const mpi3d_plan *pl)
{
    ProjArgs a{};
    a.cs = pl->cs;
    a.ax = pl->ax;
    a.ay = pl->ay;
    a.nx = pl->nx; a.ny = pl->ny; a.nz = pl->nz; a.M = pl->M; a.nu = pl->nu; a.nup = pl->nup; a.nr = pl->nr;
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
static hipError_t launch_fwd(const mpi3d_plan *pl, const typename Texel<T>::V *vol, const FwdConfig &fc, float *rt,
                             int out_stride, hipStream_t st)
{
    ProjArgs a = base_args(pl);
    a.rt = rt;
    a.band_rows = fc.band_rows;
    a.n_bands = fc.n_bands;
    const size_t lds = (size_t)(fc.band_rows + 1) * proj_pitch(pl->nx) * sizeof(T);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)proj_fwd_kernel<T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(proj_fwd_kernel<T>, dim3(fc.blocks), dim3(kFwdThreads), lds, st, a, vol, out_stride);
    return hipGetLastError();
}

static hipError_t launch_fwd32(const mpi3d_plan *pl, const float *x, float *rt, int out_stride, hipStream_t st)
{
    if (pl->fwd32.slices == 2) return launch_fwd<float2>(pl, x, pl->fwd32, rt, out_stride, st);
    return launch_fwd<float>(pl, x, pl->fwd32, rt, out_stride, st);
}

hipError_t launch_project_strided(const mpi3d_plan *pl, const float *x, float *rt, int out_stride, hipStream_t st)
{
    return launch_fwd32(pl, x, rt, out_stride, st);
}

// xb non-null: gather from the bf16 copy (mixed path)
hipError_t launch_project(const mpi3d_plan *pl, const float *x, const uint16_t *xb, float *rt, hipStream_t st)
{
    hipError_t e = xb ? launch_fwd<uint32_t>(pl, xb, pl->fwd16, rt, pl->nup, st) : launch_fwd32(pl, x, rt, pl->nup, st);
    if (e == hipSuccess && pl->drive_axes == 2) e = launch_zlines(pl, rt, false, st);
    return e;
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

hipError_t launch_fold_zlines(const mpi3d_plan *pl, float *rt, hipStream_t st)
{
    return pl->drive_axes == 2 ? launch_zlines(pl, rt, true, st) : hipSuccess;
}

hipError_t launch_backproject16(const mpi3d_plan *pl, const uint16_t *rtb, const float *rtsc, float *xo,
                                const float *x_sub, double lambda, double *norm_parts, int *nparts, hipStream_t st,
                                const float *x_add)
{
    ProjArgs a = base_args(pl);
    a.xo = xo;
    a.x_sub = x_sub;
    a.x_add = x_add;
    a.lambda = lambda;
    a.norm_parts = norm_parts;
    const int blocks = a.tiles_x * a.tiles_y * a.n_zgroups;
    if (nparts) *nparts = blocks;
    if (norm_parts && blocks > pl->max_parts) return hipErrorInvalidValue;
    const size_t lds = sizeof(uint32_t) * (size_t)a.adj_chunk * (a.kz / 2) * kPW +
                       sizeof(float) * (size_t)a.adj_chunk * a.kz + sizeof(int) * a.adj_chunk;
    switch (a.kz) {
    case 8: hipLaunchKernelGGL(proj_adj_f16<8>, dim3(blocks), dim3(256), lds, st, a, rtb, rtsc, pl->nup); break;
    case 16: hipLaunchKernelGGL(proj_adj_f16<16>, dim3(blocks), dim3(256), lds, st, a, rtb, rtsc, pl->nup); break;
    case 32: hipLaunchKernelGGL(proj_adj_f16<32>, dim3(blocks), dim3(256), lds, st, a, rtb, rtsc, pl->nup); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_backproject(const mpi3d_plan *pl, float *rt, float *xo, const float *x_sub, double lambda,
                              double *norm_parts, int *nparts, hipStream_t st, const float *x_add)
{
    if (pl->drive_axes == 2) {
        hipError_t e = launch_zlines(pl, rt, true, st);
        if (e != hipSuccess) return e;
    }
    return launch_backproject_strided(pl, rt, pl->nup, xo, x_sub, lambda, norm_parts, nparts, st, x_add);
}

}  // namespace mpi3d
