// Mixed-precision signal model: the same two chained contractions as sig.hip
// (time signal, then band DFT; and the transpose), on fp16 MFMA
// (gfx950 v_mfma_f32_32x32x16_f16) with fp32 accumulation.
//
// Scaling keeps every fp16 operand near unit magnitude:
//  * tables: K and F carry power-of-two scales ks, fs (max entry in [0.5, 1));
//  * per line: the projection row (forward) or the data row (adjoint) is
//    scaled by a power of two so its largest entry is in [0.5, 1) (computed
//    beforehand by the row_scale kernel) and the split reduction undoes it
//    in fp32;
//  * per harmonic band (adjoint): data columns of band b are multiplied by a
//    plan-fixed power of two bs_b that lifts weak high harmonics toward unit
//    size, and the matching F columns by 1/bs_b, so the band's products keep
//    fp16's relative precision instead of sinking into subnormals.
// The first contraction's fp32 result (the time tile, |.| <= n_u or 2 n_b)
// is rounded to fp16 once to feed the second.
//
// Layout and wave-pair structure follow sig.hip: a 32x32x16 MFMA result
// register j of lane l holds time 8(j/4) + 4(l/32) + j%4, so eight result
// registers form one fp16 A operand whose k index maps to time
// 16 h + 8(e/4) + 4(l/32) + e%4, and the second contraction's tables are
// stored with that permutation.

#include "internal.h"

namespace mpi3d {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

namespace {

// Table loads kept in flight per wave.  The ring slot of stream element i is
// i % ring, and the stream restarts every chunk, so the ring size must divide
// the per-chunk stream length: the largest divisor of it not above a cap.
constexpr int ring_size(int nl, int cap)
{
    for (int r = cap; r > 1; --r)
        if (nl % r == 0) return r;
    return 1;
}

__device__ __forceinline__ int xcd_logical(int bid, int nblocks)
{
    const int nx = 8;
    int xcd = bid % nx, slot = bid / nx;
    int per = nblocks / nx, rem = nblocks % nx;
    return xcd * per + min(xcd, rem) + slot;
}

struct BlockPos {
    int job, row0, split, group, half, pair;
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
    const int w = threadIdx.x >> 6;
    bp.pair = w >> 1;
    bp.half = w & 1;
    bp.row0 = (tile - a.jobs[jb].tile0) * kRowsPerBlock + bp.pair * kRowsPerWave;
    return bp;
}

#define MFMA16(a, b, c) __builtin_amdgcn_mfma_f32_32x32x16_f16((a), (b), (c), 0, 0, 0)

__device__ __forceinline__ f32x16 pair_sum(float *xs, int parity, int pair, int half, int lane, const f32x16 &mine)
{
    float *slot = xs + ((parity * kWaves + pair) * 2) * 16 * 64;
    float *own = slot + half * 16 * 64;
    const float *other = slot + (1 - half) * 16 * 64;
#pragma unroll
    for (int j = 0; j < 16; ++j) own[j * 64 + lane] = mine[j];
    __syncthreads();
    f32x16 r;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const float o = other[j * 64 + lane];
        r[j] = half == 0 ? mine[j] + o : o + mine[j];
    }
    return r;
}

__device__ __forceinline__ f16x8 to_f16x8(const f32x16 &v, int base)
{
    f16x8 r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = (_Float16)v[base + e];
    return r;
}

template <int NUP, int GH>
__global__ __launch_bounds__(kSigThreads) void sig_fwd_f16(SigArgs a)
{
    __shared__ float xs[2 * kWaves * 2 * 16 * 64];
    const BlockPos bp = locate(a);
    const SigJob job = a.jobs[bp.job];
    const int lane = threadIdx.x & 63, h = lane >> 5;
    const int r = bp.row0 + (lane & 31);
    const bool rok = r < job.rows;
    constexpr int NKS = NUP / 32;         // fp16 K steps per half (16 detector samples each)
    constexpr int NF = 2 * GH;            // F loads per chunk (two 16-sample halves per tile)
    constexpr int NL = NKS + NF;
    constexpr int kRing = ring_size(NL, 12);
    static_assert(NL % kRing == 0, "ring size must divide the stream");

    // this wave's half of the line, scaled by the line's power-of-two scale
    // (row_scale kernel), as fp16 B operands
    const float *rin = (const float *)job.in + (size_t)(rok ? r : 0) * job.in_stride;
    const float rs = rok ? job.row_scale[r] : 1.f;
    f16x8 R[NKS];
    {
        const int p0 = bp.half * (NUP / 2);
#pragma unroll
        for (int st = 0; st < NKS; ++st)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int p = p0 + 16 * st + 8 * h + e;
                R[st][e] = (_Float16)((rok && p < a.nu) ? rin[p] * rs : 0.f);
            }
    }
    f32x16 acc[GH];
#pragma unroll
    for (int g = 0; g < GH; ++g) acc[g] = 0.f;

    const int ctb = bp.group * 2 * GH + bp.half * GH;
    const int kst0 = bp.half * NKS;
    const int c0 = bp.split * a.cps, c1 = min(c0 + a.cps, a.nchunks);
    const f16x8 *kf = (const f16x8 *)a.kf16 + lane;
    const f16x8 *ff = (const f16x8 *)a.ff16 + lane;
    auto load = [&](int cc, int i) -> f16x8 {
        if (i < NKS) return kf[((size_t)cc * (NUP / 16) + kst0 + i) * 64];
        const int j = i - NKS, hh = j / GH, g = j % GH;
        return ff[(((size_t)cc * a.nct + ctb + g) * 2 + hh) * 64];
    };
    f16x8 ring[kRing];
    const int cfirst = min(c0, a.nchunks - 1);
#pragma unroll
    for (int d = 0; d < kRing; ++d) ring[d] = load(cfirst, d);

    for (int c = c0; c < c1; ++c) {
        const int cnext = min(c + 1, c1 - 1);
        f32x16 S = 0.f;
        f16x8 S16[2];
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const f16x8 v = ring[i % kRing];
            ring[i % kRing] = (i + kRing < NL) ? load(c, i + kRing) : load(cnext, i + kRing - NL);
            if (i < NKS) {
                S = MFMA16(v, R[i], S);
                // keep this load's issue point: later ring slots stay in flight
                __builtin_amdgcn_sched_barrier(0);
            } else {
                if (i == NKS) {
                    const f32x16 Sf = pair_sum(xs, c & 1, bp.pair, bp.half, lane, S);
                    S16[0] = to_f16x8(Sf, 0);
                    S16[1] = to_f16x8(Sf, 8);
                }
                const int j = i - NKS, hh = j / GH, g = j % GH;
                acc[g] = MFMA16(S16[hh], v, acc[g]);
            }
        }
    }
    if (bp.row0 >= job.rows) return;
    float *out = job.part + (size_t)bp.split * job.part_stride;
#pragma unroll
    for (int g = 0; g < GH; ++g) {
        const int col = (ctb + g) * 32 + (lane & 31);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int row = bp.row0 + 8 * (j / 4) + 4 * h + (j % 4);
            if (row < job.rows) out[(size_t)row * a.nbp2 + col] = acc[g][j];
        }
    }
}

template <int NUP, int GH>
__global__ __launch_bounds__(kSigThreads) void sig_adj_f16(SigArgs a)
{
    __shared__ float xs[2 * kWaves * 2 * 16 * 64];
    const BlockPos bp = locate(a);
    const SigJob job = a.jobs[bp.job];
    const int lane = threadIdx.x & 63, h = lane >> 5;
    const int r = bp.row0 + (lane & 31);
    const bool rok = r < job.rows;
    constexpr int PTH = NUP / 64;
    constexpr int NF = 2 * GH;            // fp16 F steps per chunk (16 columns each)
    constexpr int NK = 2 * PTH;           // K loads per chunk
    constexpr int NL = NF + NK;
    constexpr int kRing = ring_size(NL, 12);
    static_assert(NL % kRing == 0, "ring size must divide the stream");
    const int colbase = (bp.group * 2 * GH + bp.half * GH) * 32;
    const int pt0 = bp.half * PTH;

    // the line's power-of-two scale over the band-scaled row (row_scale kernel)
    const float *yin = (const float *)job.in + (size_t)(rok ? r : 0) * job.in_stride;
    const float ys = rok ? job.row_scale[r] : 1.f;
    f16x8 Y[NF];
#pragma unroll
    for (int st = 0; st < NF; ++st)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int col = colbase + 16 * st + 8 * h + e;
            Y[st][e] = (_Float16)((rok && col < a.nb2) ? yin[col] * a.band_scale[col] * ys : 0.f);
        }
    f32x16 racc[PTH];
#pragma unroll
    for (int pt = 0; pt < PTH; ++pt) racc[pt] = 0.f;

    const int c0 = bp.split * a.cps, c1 = min(c0 + a.cps, a.nchunks);
    const f16x8 *fa = (const f16x8 *)a.fa16 + lane;
    const f16x8 *ka = (const f16x8 *)a.ka16 + lane;
    auto load = [&](int cc, int i) -> f16x8 {
        if (i < NF) return fa[((size_t)cc * (a.nbp2 / 16) + colbase / 16 + i) * 64];
        const int j = i - NF, hh = j / PTH, pt = j % PTH;
        return ka[(((size_t)cc * (NUP / 32) + pt0 + pt) * 2 + hh) * 64];
    };
    f16x8 ring[kRing];
    const int cfirst = min(c0, a.nchunks - 1);
#pragma unroll
    for (int d = 0; d < kRing; ++d) ring[d] = load(cfirst, d);

    for (int c = c0; c < c1; ++c) {
        const int cnext = min(c + 1, c1 - 1);
        f32x16 Gt = 0.f;
        f16x8 G16[2];
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const f16x8 v = ring[i % kRing];
            ring[i % kRing] = (i + kRing < NL) ? load(c, i + kRing) : load(cnext, i + kRing - NL);
            if (i < NF) {
                Gt = MFMA16(v, Y[i], Gt);
                // keep this load's issue point: later ring slots stay in flight
                __builtin_amdgcn_sched_barrier(0);
            } else {
                if (i == NF) {
                    const f32x16 Gf = pair_sum(xs, c & 1, bp.pair, bp.half, lane, Gt);
                    G16[0] = to_f16x8(Gf, 0);
                    G16[1] = to_f16x8(Gf, 8);
                }
                const int j = i - NF, hh = j / PTH, pt = j % PTH;
                racc[pt] = MFMA16(G16[hh], v, racc[pt]);
            }
        }
    }
    if (bp.row0 >= job.rows) return;
    float *out = job.part + (size_t)(bp.split * a.ngroups + bp.group) * job.part_stride;
#pragma unroll
    for (int pt = 0; pt < PTH; ++pt) {
        const int col = (pt0 + pt) * 32 + (lane & 31);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int row = bp.row0 + 8 * (j / 4) + 4 * h + (j % 4);
            if (row < job.rows) out[(size_t)row * NUP + col] = racc[pt][j];
        }
    }
}

typedef void (*SigKernel)(SigArgs);

constexpr int kNups[] = {64, 128, 192, 256};
constexpr int kGHs[] = {3, 4, 6, 7};

int gh_slot(int gct)
{
    for (int i = 0; i < 4; ++i)
        if (gct == 2 * kGHs[i]) return i;
    return -1;
}
int nup_slot(int nup)
{
    for (int i = 0; i < 4; ++i)
        if (nup == kNups[i]) return i;
    return -1;
}

#define ROW(NUP, F) {F<NUP, 3>, F<NUP, 4>, F<NUP, 6>, F<NUP, 7>}
const SigKernel kFwd[4][4] = {ROW(64, sig_fwd_f16), ROW(128, sig_fwd_f16), ROW(192, sig_fwd_f16),
                              ROW(256, sig_fwd_f16)};
const SigKernel kAdj[4][4] = {ROW(64, sig_adj_f16), ROW(128, sig_adj_f16), ROW(192, sig_adj_f16),
                              ROW(256, sig_adj_f16)};
#undef ROW

}  // namespace

int sig16_supported(int nup, int gct) { return nup_slot(nup) >= 0 && gh_slot(gct) >= 0; }

hipError_t launch_sig_fwd16(const mpi3d_plan *pl, SigArgs &a, hipStream_t st)
{
    const int ns = nup_slot(pl->nup), gs = gh_slot(pl->gct);
    if (ns < 0 || gs < 0 || !pl->kf16) return hipErrorInvalidValue;
    const int blocks = a.total_tiles * a.nsplit * a.ngroups;
    hipLaunchKernelGGL(kFwd[ns][gs], dim3(blocks), dim3(kSigThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_sig_adj16(const mpi3d_plan *pl, SigArgs &a, hipStream_t st)
{
    const int ns = nup_slot(pl->nup), gs = gh_slot(pl->gct);
    if (ns < 0 || gs < 0 || !pl->ka16) return hipErrorInvalidValue;
    const int blocks = a.total_tiles * a.nsplit * a.ngroups;
    hipLaunchKernelGGL(kAdj[ns][gs], dim3(blocks), dim3(kSigThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace mpi3d
