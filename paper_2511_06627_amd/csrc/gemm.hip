// The precomposed-line signal stage as fp32 MFMA GEMMs (gfx950
// v_mfma_f32_32x32x2_f32).
//
// When every line of a scan shares one trajectory, the signal chain of a
// line is one fixed linear map G = F^T K (2nb x n_u; eq. DCmodel with the PSF
// kernel of eq. stheta1 folded in), formed once per plan in FP64:
//   forward   data[l][c]  = alpha sum_p lines[l][p] G^T[p][c]  (+ beta data[l][c])
//   adjoint   lines[l][p] = alpha sum_c data[l][c]  G[c][p]    (+ beta lines[l][p])
// Both are C[i][j] = alpha sum_k A_i[k] W[k][j] + beta C[i][j] over a run of
// lines: row i reads line in0 + b batch_lines + i in_step and writes line
// out0 + b batch_lines + i out_step (b < batch: the angles of a raster class
// or a tensor-PSF offset), W row-major with row stride ldw.
//
// One block computes a 32 x 32 tile of C; its four waves take interleaved
// blocks of 8 k-indices (wave w: blocks w, w + 4, ...), and their partial
// tiles are added through LDS in wave order, so the result does not depend
// on timing.  Within a block of 8, lane half h takes k = k0 + 4h + t at MFMA
// step t = 0..3: a lane reads four consecutive entries of its own row of A
// and four rows of W at its column (coalesced across the wave), the next
// block's values loaded before this block's products.  A 32x32 MFMA result
// register s of lane l holds row 8(s/4) + 4(l/32) + s%4, column l%32.

#include "device.h"

namespace mpi3d {

namespace {

#define MFMA32(a, b, c) __builtin_amdgcn_mfma_f32_32x32x2f32((a), (b), (c), 0, 0, 0)

constexpr int kGemmWaves = 4;

struct Operands {
    float a[4], w[4];
};

// The four A entries kb .. kb + 3 of a row: one 16-byte load (VA = 4: rows
// 16-byte aligned), two 8-byte loads (VA = 2: rows 8-byte aligned) or four
// (VA = 1) where all four lie inside the row, entry by entry at its end.
template <int VA>
__device__ __forceinline__ Operands gemm_load(const LineGemm &g, const float *arow, const float *wcol, bool iok,
                                              bool jok, int kb)
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    Operands o;
    if (VA > 1 && iok && kb + 3 < g.k) {
        if constexpr (VA == 4) {
            const f4 v = *reinterpret_cast<const f4 *>(arow + kb);
            o.a[0] = v[0], o.a[1] = v[1], o.a[2] = v[2], o.a[3] = v[3];
        } else {
            const f2 v0 = *reinterpret_cast<const f2 *>(arow + kb), v1 = *reinterpret_cast<const f2 *>(arow + kb + 2);
            o.a[0] = v0[0], o.a[1] = v0[1], o.a[2] = v1[0], o.a[3] = v1[1];
        }
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) o.a[t] = (iok && kb + t < g.k) ? arow[kb + t] : 0.f;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) o.w[t] = (jok && kb + t < g.k) ? wcol[(long)(kb + t) * g.ldw] : 0.f;
    return o;
}

template <int VA>
__global__ __launch_bounds__(64 * kGemmWaves) void line_gemm_kernel(LineGemm g)
{
    __shared__ float part[kGemmWaves - 1][16][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, r = lane & 31;
    const int tiles_j = (g.m + 31) / 32;
    const int ti = (int)(blockIdx.x / tiles_j), tj = (int)(blockIdx.x % tiles_j);
    const long b = blockIdx.y;
    const long in_base = g.in0 + b * g.batch_lines, out_base = g.out0 + b * g.batch_lines;
    const int i = ti * 32 + r;                        // this lane's row of A
    const bool iok = i < g.n;
    const float *arow = g.a + (in_base + (long)(iok ? i : 0) * g.in_step) * g.lda;
    const int j = tj * 32 + r;                        // this lane's column of W and C
    const bool jok = j < g.m;
    const float *wcol = g.w + (jok ? j : 0);

    f32x16 acc = 0.f;
    int k0 = 8 * wave;
    Operands cur = gemm_load<VA>(g, arow, wcol, iok, jok, k0 + 4 * h);
    for (; k0 < g.k; k0 += 8 * kGemmWaves) {
        const Operands nxt = gemm_load<VA>(g, arow, wcol, iok, jok, k0 + 8 * kGemmWaves + 4 * h);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc = MFMA32(cur.a[t], cur.w[t], acc);
        cur = nxt;
    }
    if (wave > 0) {
#pragma unroll
        for (int s = 0; s < 16; ++s) part[wave - 1][s][lane] = acc[s];
    }
    __syncthreads();
    if (wave > 0 || !jok) return;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int row = ti * 32 + 8 * (s / 4) + 4 * h + (s % 4);
        float v = acc[s];
#pragma unroll
        for (int w = 0; w < kGemmWaves - 1; ++w) v += part[w][s][lane];
        if (row >= g.n) continue;
        float *o = g.c + (out_base + (long)row * g.out_step) * g.ldc + j;
        v *= g.alpha;
        *o = g.beta != 0.f ? fmaf(g.beta, *o, v) : v;
    }
}

}  // namespace

hipError_t launch_line_gemm(const LineGemm &g, hipStream_t st)
{
    if (g.n <= 0 || g.batch <= 0) return hipSuccess;
    if (g.m <= 0 || g.k <= 0 || g.batch > 65535) return hipErrorInvalidValue;
    const long blocks = (long)((g.n + 31) / 32) * ((g.m + 31) / 32);   // one 32 x 32 tile each
    if (blocks > 0x7fffffffL) return hipErrorInvalidValue;
    // A's rows are 16- (8-) byte aligned when its base and row stride are
    const uintptr_t base = (uintptr_t)g.a;
    const dim3 grid((unsigned)blocks, (unsigned)g.batch);
    if (base % 16 == 0 && g.lda % 4 == 0)
        hipLaunchKernelGGL(line_gemm_kernel<4>, grid, dim3(64 * kGemmWaves), 0, st, g);
    else if (base % 8 == 0 && g.lda % 2 == 0)
        hipLaunchKernelGGL(line_gemm_kernel<2>, grid, dim3(64 * kGemmWaves), 0, st, g);
    else
        hipLaunchKernelGGL(line_gemm_kernel<1>, grid, dim3(64 * kGemmWaves), 0, st, g);
    return hipGetLastError();
}

}  // namespace mpi3d
