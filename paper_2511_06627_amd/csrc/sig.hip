// Compressed signal model A_DC on fp32 MFMA (gfx950 v_mfma_f32_32x32x2_f32).
//
// Forward, per FFL line (eq. stheta1 with eq. DCmodel):
//   s[t]  = sum_p rho_theta[p] K[t][p]       K = c_A v_t L'((xi_t - u_p)/w)/w
//   b[c]  = sum_t s[t] F[t][c]               F = Re/Im of D e^{+2 pi i omega t/T}/sqrt(T)
// Adjoint (the exact real transpose):
//   g[t]  = sum_c y[c] F[t][c]
//   r[p]  = sum_t g[t] K[t][p]
//
// Both are two chained contractions whose intermediate is the time signal of
// the line.  The time signal never leaves the chip: a wave owns 32 lines and
// walks time in chunks of 32 samples; the first contraction produces the
// 32 x 32 (time x line) tile in MFMA accumulators, and those same registers
// feed the second contraction as its A operand -- the result layout of the
// 32x32 MFMA holds, in register s of lane l, line l%32 at time
// 8(s/4) + 4(l/32) + s%4, which is exactly an A-operand column pair, so the
// tables of the second contraction are stored with their time index permuted
// to match.  All tables are pre-swizzled so every operand fetch is one
// coalesced 16-byte load per lane.
//
// Time is split across blocks (fixed chunk ranges per split) so that a scan
// with few lines still fills 256 CUs; each block writes fp32 partial sums of
// its split, and a reduction kernel adds the splits in a fixed order.  A
// line's arithmetic is independent of the other lines in its block, which is
// what makes batching requests bitwise invariant.

#include "internal.h"

namespace mpi3d {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ int xcd_logical(int bid, int nblocks)
{
    const int nx = 8;
    int xcd = bid % nx, slot = bid / nx;
    int per = nblocks / nx, rem = nblocks % nx;
    return xcd * per + min(xcd, rem) + slot;
}

struct BlockPos {
    int job, row0, split, group;
};

__device__ __forceinline__ BlockPos locate(const SigArgs &a)
{
    BlockPos bp;
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int tile = lb % a.total_tiles;
    const int sg = lb / a.total_tiles;
    bp.group = sg % a.ngroups;
    bp.split = sg / a.ngroups;
    int jb = 0;
    for (int j = 1; j < a.njobs; ++j)
        if (tile >= a.jobs[j].tile0) jb = j;
    bp.job = jb;
    bp.row0 = (tile - a.jobs[jb].tile0) * kRowsPerBlock + (threadIdx.x >> 6) * kRowsPerWave;
    return bp;
}

#define MFMA32(a, b, c) __builtin_amdgcn_mfma_f32_32x32x2f32((a), (b), (c), 0, 0, 0)

template <int NUP, int G>
__global__ __launch_bounds__(256, 1) void sig_fwd_f32(SigArgs a)
{
    const BlockPos bp = locate(a);
    const SigJob job = a.jobs[bp.job];
    if (bp.row0 >= job.rows) return;
    const int lane = threadIdx.x & 63, h = lane >> 5;
    const int r = bp.row0 + (lane & 31);
    const bool rok = r < job.rows;

    // B operand of the first contraction: rho_theta[r][2 st + h], kept for the whole block
    float R[NUP / 2];
    {
        const float *rin = (const float *)job.in + (size_t)(rok ? r : 0) * job.in_stride + h;
#pragma unroll
        for (int st = 0; st < NUP / 2; ++st) R[st] = (rok && 2 * st + h < a.nu) ? rin[2 * st] : 0.f;
    }
    f32x16 acc[G];
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g] = 0.f;

    const int ct0 = bp.group * a.gct;
    const int nctg = min(a.gct, a.nct - ct0);
    const int c0 = bp.split * a.cps, c1 = min(c0 + a.cps, a.nchunks);
    const f32x4 *kf = (const f32x4 *)a.kf;
    const f32x4 *ff = (const f32x4 *)a.ff;
    for (int c = c0; c < c1; ++c) {
        // time signal tile S^T[t][line] = sum_p K[t][p] rho[line][p]
        f32x16 S = 0.f;
        const f32x4 *kp = kf + (size_t)c * (NUP / 8) * 64 + lane;
#pragma unroll
        for (int st4 = 0; st4 < NUP / 8; ++st4) {
            const f32x4 kv = kp[st4 * 64];
            S = MFMA32(kv[0], R[4 * st4 + 0], S);
            S = MFMA32(kv[1], R[4 * st4 + 1], S);
            S = MFMA32(kv[2], R[4 * st4 + 2], S);
            S = MFMA32(kv[3], R[4 * st4 + 3], S);
        }
        // bands: acc[line][col] += sum_t S[line][t] F[t][col]
        const f32x4 *fp = ff + ((size_t)c * a.nct + ct0) * 4 * 64 + lane;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            f32x4 fv[G];
#pragma unroll
            for (int g = 0; g < G; ++g) fv[g] = (g < nctg) ? fp[(g * 4 + s4) * 64] : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int g = 0; g < G; ++g)
                    if (g < nctg) acc[g] = MFMA32(S[4 * s4 + e], fv[g][e], acc[g]);
        }
    }
    float *out = job.part + (size_t)bp.split * job.part_stride;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        if (g >= nctg) continue;
        const int col = (ct0 + g) * 32 + (lane & 31);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int row = bp.row0 + 8 * (j / 4) + 4 * h + (j % 4);
            if (row < job.rows) out[(size_t)row * a.nbp2 + col] = acc[g][j];
        }
    }
}

template <int NUP, int G>
__global__ __launch_bounds__(256, 1) void sig_adj_f32(SigArgs a)
{
    const BlockPos bp = locate(a);
    const SigJob job = a.jobs[bp.job];
    if (bp.row0 >= job.rows) return;
    const int lane = threadIdx.x & 63, h = lane >> 5;
    const int r = bp.row0 + (lane & 31);
    const bool rok = r < job.rows;
    const int ct0 = bp.group * a.gct;
    const int nctg = min(a.gct, a.nct - ct0);
    const int colbase = ct0 * 32;

    // B operand of the first contraction: y[r][colbase + 2 st + h]
    float Y[16 * G];
    {
        const float *yin = (const float *)job.in + (size_t)(rok ? r : 0) * job.in_stride + colbase + h;
#pragma unroll
        for (int st = 0; st < 16 * G; ++st) {
            const int col = colbase + 2 * st + h;
            Y[st] = (rok && col < a.nb2 && st < 16 * nctg) ? yin[2 * st] : 0.f;
        }
    }
    f32x16 racc[NUP / 32];
#pragma unroll
    for (int pt = 0; pt < NUP / 32; ++pt) racc[pt] = 0.f;

    const int c0 = bp.split * a.cps, c1 = min(c0 + a.cps, a.nchunks);
    const f32x4 *fa = (const f32x4 *)a.fa;
    const f32x4 *ka = (const f32x4 *)a.ka;
    for (int c = c0; c < c1; ++c) {
        // time tile G^T[t][line] = sum_col F[t][col] y[line][col]
        f32x16 Gt = 0.f;
        const f32x4 *fp = fa + ((size_t)c * (a.nbp2 / 8) + colbase / 8) * 64 + lane;
#pragma unroll
        for (int st4 = 0; st4 < 4 * G; ++st4) {
            if (st4 < 4 * nctg) {
                const f32x4 fv = fp[st4 * 64];
                Gt = MFMA32(fv[0], Y[4 * st4 + 0], Gt);
                Gt = MFMA32(fv[1], Y[4 * st4 + 1], Gt);
                Gt = MFMA32(fv[2], Y[4 * st4 + 2], Gt);
                Gt = MFMA32(fv[3], Y[4 * st4 + 3], Gt);
            }
        }
        // racc[line][p] += sum_t G[line][t] K[t][p]
        const f32x4 *kp = ka + (size_t)c * (NUP / 32) * 4 * 64 + lane;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            f32x4 kv[NUP / 32];
#pragma unroll
            for (int pt = 0; pt < NUP / 32; ++pt) kv[pt] = kp[(pt * 4 + s4) * 64];
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int pt = 0; pt < NUP / 32; ++pt) racc[pt] = MFMA32(Gt[4 * s4 + e], kv[pt][e], racc[pt]);
        }
    }
    float *out = job.part + (size_t)(bp.split * a.ngroups + bp.group) * job.part_stride;
#pragma unroll
    for (int pt = 0; pt < NUP / 32; ++pt) {
        const int col = pt * 32 + (lane & 31);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int row = bp.row0 + 8 * (j / 4) + 4 * h + (j % 4);
            if (row < job.rows) out[(size_t)row * NUP + col] = racc[pt][j];
        }
    }
}

typedef void (*SigKernel)(SigArgs);

constexpr int kNups[] = {32, 64, 128, 192, 256};
constexpr int kGs[] = {5, 8, 11, 14};

template <int NUP, int G>
SigKernel pick_fwd() { return sig_fwd_f32<NUP, G>; }
template <int NUP, int G>
SigKernel pick_adj() { return sig_adj_f32<NUP, G>; }

int g_slot(int gct)
{
    for (int i = 0; i < 4; ++i)
        if (gct <= kGs[i]) return i;
    return -1;
}
int nup_slot(int nup)
{
    for (int i = 0; i < 5; ++i)
        if (nup == kNups[i]) return i;
    return -1;
}

#define ROW(NUP, F) {F<NUP, 5>, F<NUP, 8>, F<NUP, 11>, F<NUP, 14>}
const SigKernel kFwd[5][4] = {ROW(32, sig_fwd_f32), ROW(64, sig_fwd_f32), ROW(128, sig_fwd_f32),
                              ROW(192, sig_fwd_f32), ROW(256, sig_fwd_f32)};
const SigKernel kAdj[5][4] = {ROW(32, sig_adj_f32), ROW(64, sig_adj_f32), ROW(128, sig_adj_f32),
                              ROW(192, sig_adj_f32), ROW(256, sig_adj_f32)};
#undef ROW

}  // namespace

// fp16 variants live in sig16.hip
hipError_t launch_sig_fwd16(const mpi3d_plan *pl, SigArgs &a, hipStream_t st);
hipError_t launch_sig_adj16(const mpi3d_plan *pl, SigArgs &a, hipStream_t st);
int sig16_supported(int nup, int gct);

int sig_fwd_supported(int nup, int gct, int precision)
{
    if (precision == MPI3D_MIXED) return sig16_supported(nup, gct);
    return nup_slot(nup) >= 0 && g_slot(gct) >= 0;
}
int sig_adj_supported(int nup, int gct, int precision) { return sig_fwd_supported(nup, gct, precision); }

hipError_t launch_sig_fwd(const mpi3d_plan *pl, int precision, SigArgs &a, hipStream_t st)
{
    if (precision == MPI3D_MIXED) return launch_sig_fwd16(pl, a, st);
    const int ns = nup_slot(pl->nup), gs = g_slot(pl->gct);
    if (ns < 0 || gs < 0) return hipErrorInvalidValue;
    const int blocks = a.total_tiles * a.nsplit * a.ngroups;
    hipLaunchKernelGGL(kFwd[ns][gs], dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_sig_adj(const mpi3d_plan *pl, int precision, SigArgs &a, hipStream_t st)
{
    if (precision == MPI3D_MIXED) return launch_sig_adj16(pl, a, st);
    const int ns = nup_slot(pl->nup), gs = g_slot(pl->gct);
    if (ns < 0 || gs < 0) return hipErrorInvalidValue;
    const int blocks = a.total_tiles * a.nsplit * a.ngroups;
    hipLaunchKernelGGL(kAdj[ns][gs], dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace mpi3d
