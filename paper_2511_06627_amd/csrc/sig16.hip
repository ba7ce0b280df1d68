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

#include "device.h"

namespace mpi3d {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

namespace {

#define MFMA16(a, b, c) __builtin_amdgcn_mfma_f32_32x32x16_f16((a), (b), (c), 0, 0, 0)

__device__ __forceinline__ f16x8 to_f16x8(const f32x16 &v, int base)
{
    f16x8 r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = (_Float16)v[base + e];
    return r;
}

// N products whose table operands come from LDS: fragment j is read WIN
// products ahead of its use, and a scheduling barrier after every product
// keeps that distance, so an LDS read's latency is covered by the products
// in between instead of stalling the one that needs it.
template <int N, int WIN, class Frag, class Prod>
__device__ __forceinline__ void lds_pipelined(Frag frag, Prod prod)
{
    constexpr int W = WIN < N ? WIN : N;
    f16x8 w[W];
#pragma unroll
    for (int j = 0; j < W; ++j) w[j] = frag(j);
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const f16x8 f = w[j % W];
        if (j + W < N) w[j % W] = frag(j + W);
        prod(j, f);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Per-chunk table staging.  The block copies each time chunk's table slices
// (GEMM1's and GEMM2's) from HBM/L2 into LDS once, with every thread moving a
// few 16-byte units; the waves then read their operand fragments from LDS.
// Without it each of the four pairs would fetch the same slices itself.  A
// slice is loaded into registers two chunks before it is used and written to
// LDS during the chunk before.
//   A slice (GEMM1 operands), double-buffered: chunk c+1 is written before the
//     pair barrier of chunk c, whose GEMM1 no longer reads that buffer (it
//     last served chunk c-1, finished before the barrier of chunk c-1).
//   B slice (GEMM2 operands), double-buffered: chunk c+1 is written after the
//     pair barrier of chunk c; that buffer last served GEMM2 of chunk c-1,
//     which every wave finished before reaching the barrier of chunk c.
// The barrier of chunk c+1 then publishes both before they are read.
template <int UNITS>
struct Slice {
    static constexpr int kPer = (UNITS + kSigThreads - 1) / kSigThreads;
    f16x8 v[kPer];
    __device__ __forceinline__ void load(const f16x8 *src, int tid)
    {
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int u = tid + j * kSigThreads;
            if (u < UNITS) v[j] = src[u];
        }
    }
    __device__ __forceinline__ void store(f16x8 *dst, int tid) const
    {
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int u = tid + j * kSigThreads;
            if (u < UNITS) dst[u] = v[j];
        }
    }
};

constexpr int kXsBytes = 2 * kWaves * 2 * 16 * 64 * (int)sizeof(float);

template <int NUP, int GH>
constexpr int sig16_lds_bytes()
{
    return kXsBytes + 2 * 16 * (4 * NUP + 256 * GH);
}

template <int NUP, int GH>
__global__ __launch_bounds__(kSigThreads) void sig_fwd_f16(SigArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    float *xs = reinterpret_cast<float *>(smem);
    constexpr int UA = 4 * NUP;           // K slice: NUP/16 fragments of 64 lanes
    constexpr int UB = 256 * GH;          // F slice of the group: 2 GH tiles x 2 halves
    f16x8 *la = reinterpret_cast<f16x8 *>(smem + kXsBytes);
    f16x8 *lb = la + 2 * UA;
    const BlockPos bp = locate(a);
    const SigJob job = a.jobs[bp.job];
    const int tid = threadIdx.x;
    const int lane = tid & 63, h = lane >> 5;
    const int r = bp.row0 + (lane & 31);
    const bool rok = r < job.rows;
    // input line of this lane's row (-1: past the job's rows, zero input)
    const long il = rok ? job_line(job, r) : -1;
    const bool iok = il >= 0;
    constexpr int NKS = NUP / 32;         // fp16 K steps per half (16 detector samples each)

    // this wave's half of the line as fp16 B operands: the line scaled by its
    // power-of-two scale and rounded by the row_scale kernel (zero past n_u)
    f16x8 R[NKS];
    {
        const f16x8 *rin = (const f16x8 *)(job.in16 + (size_t)(iok ? il : 0) * job.in16_stride +
                                           bp.half * (NUP / 2) + 8 * h);
#pragma unroll
        for (int st = 0; st < NKS; ++st) R[st] = iok ? rin[2 * st] : f16x8(0);
        // complete these loads here: inside the time loop the only memory
        // loads in flight are then the next chunk's table slices, which the
        // first contraction does not wait for
#pragma unroll
        for (int st = 0; st < NKS; ++st) asm volatile("" ::"v"(R[st]));
    }
    f32x16 acc[GH];
#pragma unroll
    for (int g = 0; g < GH; ++g) acc[g] = 0.f;

    const int c0 = bp.split * a.cps, c1 = min(c0 + a.cps, a.nchunks);
    const f16x8 *kg = (const f16x8 *)job.kf16;
    const f16x8 *fg = (const f16x8 *)a.ff16 + (size_t)bp.group * UB;
    const size_t fstride = (size_t)a.nct * 128;
    // table slices in registers: chunk c + 1 (loaded during chunk c - 1,
    // stored to LDS during chunk c) and chunk c + 2 (loaded during chunk c),
    // so a load has a whole chunk to arrive
    Slice<UA> sa, sa2;
    Slice<UB> sb, sb2;
    if (c0 < c1) {
        sa.load(kg + (size_t)c0 * UA, tid);
        sb.load(fg + (size_t)c0 * fstride, tid);
        sa.store(la + (c0 & 1) * UA, tid);
        sb.store(lb + (c0 & 1) * UB, tid);
    }
    if (c0 + 1 < c1) {
        sa.load(kg + (size_t)(c0 + 1) * UA, tid);
        sb.load(fg + (size_t)(c0 + 1) * fstride, tid);
    }
    __syncthreads();
    const int ka0 = bp.half * NKS * 64 + lane;           // this wave's first K fragment
    const int fb0 = bp.half * GH * 128 + lane;           // this wave's first F fragment

    // one chunk: (ra, rb) hold chunk c + 1's slices, (na, nb) receive c + 2's;
    // the loop alternates the two register sets, so no slice is copied
    auto chunk = [&](int c, Slice<UA> &ra, Slice<UB> &rb, Slice<UA> &na, Slice<UB> &nb) {
        const int buf = c & 1;
        const bool more = c + 1 < c1;
        const int cn = min(c + 2, c1 - 1);               // loaded whether needed or not: no branch
        na.load(kg + (size_t)cn * UA, tid);
        nb.load(fg + (size_t)cn * fstride, tid);
        const f16x8 *ka = la + buf * UA + ka0;
        f32x16 S = 0.f;
        // GH = 7 leaves no registers for eight fragments in flight at NUP = 256
        lds_pipelined<NKS, GH >= 7 ? 4 : 8>([&](int i) { return ka[i * 64]; },
                                            [&](int i, const f16x8 &f) { S = MFMA16(f, R[i], S); });
        if (more) ra.store(la + (buf ^ 1) * UA, tid);
        const f32x16 Sf = pair_sum<kWaves>(xs, buf, bp.pair, bp.half, lane, S);
        if (more) rb.store(lb + (buf ^ 1) * UB, tid);
        const f16x8 S16[2] = {to_f16x8(Sf, 0), to_f16x8(Sf, 8)};
        const f16x8 *fb = lb + buf * UB + fb0;
        lds_pipelined<2 * GH, 4>([&](int j) { return fb[((j % GH) * 2 + j / GH) * 64]; },
                                 [&](int j, const f16x8 &f) { acc[j % GH] = MFMA16(S16[j / GH], f, acc[j % GH]); });
    };
    int c = c0;
    for (; c + 1 < c1; c += 2) {
        chunk(c, sa, sb, sa2, sb2);
        chunk(c + 1, sa2, sb2, sa, sb);
    }
    if (c < c1) chunk(c, sa, sb, sa2, sb2);
    if (bp.row0 >= job.rows) return;
    long ln[16];   // buffer lines of this lane's 16 result rows
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int row = bp.row0 + 8 * (j / 4) + 4 * h + (j % 4);
        ln[j] = row < job.rows ? job_line(job, row) : 0;
    }
    float *out = job.part + (size_t)bp.split * job.part_stride;
    const int ctb = bp.group * 2 * GH + bp.half * GH;
#pragma unroll
    for (int g = 0; g < GH; ++g) {
        const int col = (ctb + g) * 32 + (lane & 31);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int row = bp.row0 + 8 * (j / 4) + 4 * h + (j % 4);
            if (row < job.rows) out[(size_t)ln[j] * a.nbp2 + col] = acc[g][j];
        }
    }
}

template <int NUP, int GH>
__global__ __launch_bounds__(kSigThreads) void sig_adj_f16(SigArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    float *xs = reinterpret_cast<float *>(smem);
    constexpr int UA = 256 * GH;          // F slice of the group (GEMM1)
    constexpr int UB = 4 * NUP;           // K slice (GEMM2)
    f16x8 *la = reinterpret_cast<f16x8 *>(smem + kXsBytes);
    f16x8 *lb = la + 2 * UA;
    const BlockPos bp = locate(a);
    const SigJob job = a.jobs[bp.job];
    const int tid = threadIdx.x;
    const int lane = tid & 63, h = lane >> 5;
    const int r = bp.row0 + (lane & 31);
    const bool rok = r < job.rows;
    // input line of this lane's row (-1: past the job's rows, zero input)
    const long il = rok ? job_line(job, r) : -1;
    const bool iok = il >= 0;
    constexpr int PTH = NUP / 64;
    constexpr int NF = 2 * GH;            // fp16 F steps per chunk (16 columns each)
    const int colbase = (bp.group * 2 * GH + bp.half * GH) * 32;
    const int pt0 = bp.half * PTH;

    // this wave's bins of the line as fp16 B operands: the band-scaled row
    // times the line's power-of-two scale, rounded by the row_scale kernel
    // (zero past 2 nb)
    f16x8 Y[NF];
    {
        const f16x8 *yin = (const f16x8 *)(job.in16 + (size_t)(iok ? il : 0) * job.in16_stride + colbase + 8 * h);
#pragma unroll
        for (int st = 0; st < NF; ++st) Y[st] = iok ? yin[2 * st] : f16x8(0);
        // complete these loads before the time loop (see sig_fwd_f16)
#pragma unroll
        for (int st = 0; st < NF; ++st) asm volatile("" ::"v"(Y[st]));
    }
    f32x16 racc[PTH];
#pragma unroll
    for (int pt = 0; pt < PTH; ++pt) racc[pt] = 0.f;

    const int c0 = bp.split * a.cps, c1 = min(c0 + a.cps, a.nchunks);
    const size_t fstride = (size_t)a.nct * 128;
    const f16x8 *fg = (const f16x8 *)a.fa16 + (size_t)bp.group * UA;
    const f16x8 *kg = (const f16x8 *)job.ka16;
    // table slices in registers two chunks ahead (see sig_fwd_f16)
    Slice<UA> sa, sa2;
    Slice<UB> sb, sb2;
    if (c0 < c1) {
        sa.load(fg + (size_t)c0 * fstride, tid);
        sb.load(kg + (size_t)c0 * UB, tid);
        sa.store(la + (c0 & 1) * UA, tid);
        sb.store(lb + (c0 & 1) * UB, tid);
    }
    if (c0 + 1 < c1) {
        sa.load(fg + (size_t)(c0 + 1) * fstride, tid);
        sb.load(kg + (size_t)(c0 + 1) * UB, tid);
    }
    __syncthreads();
    const int fa0 = bp.half * NF * 64 + lane;            // this wave's first F fragment
    const int kb0 = pt0 * 128 + lane;                    // this wave's first K fragment

    // one chunk, alternating two register sets of slices (see sig_fwd_f16)
    auto chunk = [&](int c, Slice<UA> &ra, Slice<UB> &rb, Slice<UA> &na, Slice<UB> &nb) {
        const int buf = c & 1;
        const bool more = c + 1 < c1;
        const int cn = min(c + 2, c1 - 1);               // loaded whether needed or not: no branch
        na.load(fg + (size_t)cn * fstride, tid);
        nb.load(kg + (size_t)cn * UB, tid);
        const f16x8 *fa = la + buf * UA + fa0;
        f32x16 Gt = 0.f;
        lds_pipelined<NF, 6>([&](int i) { return fa[i * 64]; }, [&](int i, const f16x8 &f) { Gt = MFMA16(f, Y[i], Gt); });
        if (more) ra.store(la + (buf ^ 1) * UA, tid);
        const f32x16 Gf = pair_sum<kWaves>(xs, buf, bp.pair, bp.half, lane, Gt);
        if (more) rb.store(lb + (buf ^ 1) * UB, tid);
        const f16x8 G16[2] = {to_f16x8(Gf, 0), to_f16x8(Gf, 8)};
        const f16x8 *kb = lb + buf * UB + kb0;
        lds_pipelined<2 * PTH, 4>([&](int j) { return kb[((j % PTH) * 2 + j / PTH) * 64]; },
                                  [&](int j, const f16x8 &f) { racc[j % PTH] = MFMA16(G16[j / PTH], f, racc[j % PTH]); });
    };
    int c = c0;
    for (; c + 1 < c1; c += 2) {
        chunk(c, sa, sb, sa2, sb2);
        chunk(c + 1, sa2, sb2, sa, sb);
    }
    if (c < c1) chunk(c, sa, sb, sa2, sb2);
    if (bp.row0 >= job.rows) return;
    long ln[16];   // buffer lines of this lane's 16 result rows
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int row = bp.row0 + 8 * (j / 4) + 4 * h + (j % 4);
        ln[j] = row < job.rows ? job_line(job, row) : 0;
    }
    float *out = job.part + (size_t)(bp.split * a.ngroups + bp.group) * job.part_stride;
#pragma unroll
    for (int pt = 0; pt < PTH; ++pt) {
        const int col = (pt0 + pt) * 32 + (lane & 31);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int row = bp.row0 + 8 * (j / 4) + 4 * h + (j % 4);
            if (row < job.rows) out[(size_t)ln[j] * NUP + col] = racc[pt][j];
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

#define LROW(NUP) {sig16_lds_bytes<NUP, 3>(), sig16_lds_bytes<NUP, 4>(), sig16_lds_bytes<NUP, 6>(), \
                   sig16_lds_bytes<NUP, 7>()}
const int kLds[4][4] = {LROW(64), LROW(128), LROW(192), LROW(256)};
#undef LROW

#define ROW(NUP, F) {F<NUP, 3>, F<NUP, 4>, F<NUP, 6>, F<NUP, 7>}
const SigKernel kFwd[4][4] = {ROW(64, sig_fwd_f16), ROW(128, sig_fwd_f16), ROW(192, sig_fwd_f16),
                              ROW(256, sig_fwd_f16)};
const SigKernel kAdj[4][4] = {ROW(64, sig_adj_f16), ROW(128, sig_adj_f16), ROW(192, sig_adj_f16),
                              ROW(256, sig_adj_f16)};
#undef ROW

}  // namespace

int sig16_supported(int nup, int gct, int pairs)
{
    return pairs == kWaves && nup_slot(nup) >= 0 && gh_slot(gct) >= 0;
}

// Dynamic LDS above 64 KB has to be allowed per kernel.
static hipError_t allow_lds(const void *kernel, int bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t launch_sig_fwd16(const mpi3d_plan *pl, SigArgs &a, hipStream_t st)
{
    const int ns = nup_slot(pl->nup), gs = gh_slot(a.gct);
    if (ns < 0 || gs < 0 || a.pairs != kWaves || !pl->kf16) return hipErrorInvalidValue;
    hipError_t e = allow_lds((const void *)kFwd[ns][gs], kLds[ns][gs]);
    if (e != hipSuccess) return e;
    const int blocks = a.total_tiles * a.nsplit * a.ngroups;
    hipLaunchKernelGGL(kFwd[ns][gs], dim3(blocks), dim3(kSigThreads), kLds[ns][gs], st, a);
    return hipGetLastError();
}

hipError_t launch_sig_adj16(const mpi3d_plan *pl, SigArgs &a, hipStream_t st)
{
    const int ns = nup_slot(pl->nup), gs = gh_slot(a.gct);
    if (ns < 0 || gs < 0 || a.pairs != kWaves || !pl->ka16) return hipErrorInvalidValue;
    hipError_t e = allow_lds((const void *)kAdj[ns][gs], kLds[ns][gs]);
    if (e != hipSuccess) return e;
    const int blocks = a.total_tiles * a.nsplit * a.ngroups;
    hipLaunchKernelGGL(kAdj[ns][gs], dim3(blocks), dim3(kSigThreads), kLds[ns][gs], st, a);
    return hipGetLastError();
}

}  // namespace mpi3d
