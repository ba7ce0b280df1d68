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
// the line, and the time signal never leaves the chip.  Time is walked in
// chunks of 32 samples.  The first contraction leaves a 32 x 32 (time x line)
// tile in MFMA result registers; the 32x32 MFMA result layout holds, in
// register s of lane l, line l%32 at time 8(s/4) + 4(l/32) + s%4, which is an
// A-operand column pair of the next MFMA, so those registers feed the second
// contraction directly and its tables are stored with the time index permuted
// to match.  Every table is pre-swizzled so an operand fetch is one coalesced
// 16-byte load per lane.
//
// Wave pairs.  A block is 8 waves = 4 pairs (two waves per SIMD; wide
// blocks: 4 waves = 2 pairs, one wave per SIMD, whose waves hold up to 22
// column tiles and a deeper load ring); a pair owns 32 lines.  The two
// waves of a pair split the reduction of the first contraction (half the
// detector samples, or half the bins) and the output columns of the second,
// and swap their partial time tiles through LDS once per chunk: no work is
// duplicated, and each wave holds only half of the per-line operand and half
// of the accumulators, which leaves registers for a ring of table loads kept
// eight deep in flight.
//
// Time is also split across blocks (fixed chunk ranges) so a scan with few
// lines still fills 256 CUs; blocks write fp32 partial sums per split and a
// reduction kernel adds the splits in a fixed order.  A line's arithmetic does
// not depend on the other lines of its block, which makes batching requests
// bitwise invariant.

#include "device.h"

namespace mpi3d {

typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

// Table loads kept in flight per wave.  The ring slot of stream element i is
// i % ring, and the stream restarts every chunk, so the ring size must divide
// the per-chunk stream length: the largest divisor of it not above a cap, or,
// when that is below half the cap, the cap itself with the stream padded to
// a multiple of it by slots that load nothing.
constexpr int ring_div(int nl, int cap)
{
    for (int r = cap; r > 1; --r)
        if (nl % r == 0) return r;
    return 1;
}
constexpr int ring_size(int nl, int cap) { return 2 * ring_div(nl, cap) >= cap ? ring_div(nl, cap) : cap; }
constexpr int padded_stream(int nl, int ring) { return (nl + ring - 1) / ring * ring; }

#define MFMA32(a, b, c) __builtin_amdgcn_mfma_f32_32x32x2f32((a), (b), (c), 0, 0, 0)

// Forward.  Per pair: GEMM1 over this wave's half of the detector samples,
// pair exchange, GEMM2 over this wave's GH column tiles.  PAIRS wave pairs
// per block: kWaves (two waves per SIMD), or kWidePairs for the wide column
// groups (one wave per SIMD, up to 512 registers per wave).
template <int NUP, int GH, int PAIRS>
__device__ __forceinline__ void fwd_tile(const SigArgs &a, const BlockPos &bp, int c0, int c1, float *xs)
{
    const SigJob job = a.jobs[bp.job];
    const int lane = threadIdx.x & 63, h = lane >> 5;
    const int r = bp.row0 + (lane & 31);
    const bool rok = r < job.rows;
    // input line of this lane's row (-1: past the job's rows, zero input)
    const long il = rok ? job_line(job, r) : -1;
    const bool iok = il >= 0;
    constexpr int NK = NUP / 16;          // K float4 loads per chunk (this half)
    constexpr int NF = 4 * GH;            // F float4 loads per chunk
    constexpr int NL = NK + NF;
    constexpr int kRing = ring_size(NL, PAIRS == kWidePairs ? 16 : 8);
    constexpr int NLP = padded_stream(NL, kRing);        // stream slots per chunk (NL used)

    // B operand of GEMM1: rho[r][p0 + 2 st + h], p0 = half * NUP/2
    float R[NUP / 4];
    {
        const int p0 = bp.half * (NUP / 2);
        const float *rin = (const float *)job.in + (size_t)(iok ? il : 0) * job.in_stride + p0 + h;
#pragma unroll
        for (int st = 0; st < NUP / 4; ++st) R[st] = (iok && p0 + 2 * st + h < a.nu) ? rin[2 * st] : 0.f;
    }
    f32x16 acc[GH];
#pragma unroll
    for (int g = 0; g < GH; ++g) acc[g] = 0.f;

    const int ctb = bp.group * 2 * GH + bp.half * GH;     // first column tile of this wave
    const int kst0 = bp.half * (NUP / 16);                 // first K float4 step of this half
    const f32x4 *kf = (const f32x4 *)job.kf + lane;
    const f32x4 *ff = (const f32x4 *)a.ff + lane;
    auto load = [&](int cc, int i) -> f32x4 {
        if (i < NK) return kf[((size_t)cc * (NUP / 8) + kst0 + i) * 64];
        const int j = i - NK, s4 = j / GH, g = j % GH;
        return ff[(((size_t)cc * a.nct + ctb + g) * 4 + s4) * 64];
    };
    f32x4 ring[kRing];
    const int cfirst = min(c0, a.nchunks - 1);
#pragma unroll
    for (int d = 0; d < kRing; ++d) ring[d] = d < NL ? load(cfirst, d) : f32x4{};

    for (int c = c0; c < c1; ++c) {
        const int cnext = min(c + 1, c1 - 1);
        f32x16 S = 0.f;
        f32x16 Sf;
#pragma unroll
        for (int i = 0; i < NLP; ++i) {
            const f32x4 v = ring[i % kRing];
            const int nx = i + kRing;                    // the stream slot this ring slot takes next
            if (nx < NLP) {
                if (nx < NL) ring[i % kRing] = load(c, nx);
            } else if (nx - NLP < NL) {
                ring[i % kRing] = load(cnext, nx - NLP);
            }
            if (i >= NL) continue;                       // a padding slot
            if (i < NK) {
                S = MFMA32(v[0], R[4 * i + 0], S);
                S = MFMA32(v[1], R[4 * i + 1], S);
                S = MFMA32(v[2], R[4 * i + 2], S);
                S = MFMA32(v[3], R[4 * i + 3], S);
                // a long PSF-table stream (the fused tensor pass's 48 and more
                // loads per chunk) keeps its loads in flight as well
                if constexpr (PAIRS == kWidePairs && NK >= 32) __builtin_amdgcn_sched_barrier(0);
            } else {
                if (i == NK) Sf = pair_sum<PAIRS>(xs, c & 1, bp.pair, bp.half, lane, S);
                const int j = i - NK, s4 = j / GH, g = j % GH;
                acc[g] = MFMA32(Sf[4 * s4 + 0], v[0], acc[g]);
                acc[g] = MFMA32(Sf[4 * s4 + 1], v[1], acc[g]);
                acc[g] = MFMA32(Sf[4 * s4 + 2], v[2], acc[g]);
                acc[g] = MFMA32(Sf[4 * s4 + 3], v[3], acc[g]);
                // one wave per SIMD: keep this load's issue point so the
                // ring's later slots stay in flight through the long stream
                if constexpr (PAIRS == kWidePairs) __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    if (bp.row0 >= job.rows) return;
    long ln[16];   // buffer lines of this lane's 16 result rows
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int row = bp.row0 + 8 * (j / 4) + 4 * h + (j % 4);
        ln[j] = row < job.rows ? job_line(job, row) : 0;
    }
    float *out = job.part + (size_t)bp.split * job.part_stride;
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

template <int NUP, int GH, int PAIRS>
__global__ __launch_bounds__(128 * PAIRS) void sig_fwd_f32(SigArgs a)
{
    __shared__ __align__(16) float xs[2 * PAIRS * 2 * 16 * 64];
    const BlockWork bw = block_work(a);
    for (int k = 0; k < bw.ntiles; ++k) {
        if (k) __syncthreads();   // the previous tile's last exchange is read
        fwd_tile<NUP, GH, PAIRS>(a, tile_pos(a, bw.tile0 + k, bw.slot, bw.group), bw.c0, bw.c1, xs);
    }
}

// Adjoint.  Per pair: GEMM1 over this wave's GH column tiles (half the bins of
// the group), pair exchange, GEMM2 over this wave's half of the detector tiles.
template <int NUP, int GH, int PAIRS>
__device__ __forceinline__ void adj_tile(const SigArgs &a, const BlockPos &bp, int c0, int c1, float *xs)
{
    const SigJob job = a.jobs[bp.job];
    const int lane = threadIdx.x & 63, h = lane >> 5;
    const int r = bp.row0 + (lane & 31);
    const bool rok = r < job.rows;
    // input line of this lane's row (-1: past the job's rows, zero input)
    const long il = rok ? job_line(job, r) : -1;
    const bool iok = il >= 0;
    constexpr int PTH = NUP / 64;         // detector tiles per half
    constexpr int NF = 4 * GH;            // F float4 loads per chunk (GEMM1)
    constexpr int NK = 4 * PTH;           // K float4 loads per chunk (GEMM2)
    constexpr int NL = NF + NK;
    constexpr int kRing = ring_size(NL, PAIRS == kWidePairs ? 16 : 8);
    constexpr int NLP = padded_stream(NL, kRing);        // stream slots per chunk (NL used)
    const int colbase = (bp.group * 2 * GH + bp.half * GH) * 32;   // first column of this wave
    const int pt0 = bp.half * PTH;

    // B operand of GEMM1: y[r][colbase + 2 st + h]
    float Y[16 * GH];
    {
        const float *yin = (const float *)job.in + (size_t)(iok ? il : 0) * job.in_stride + colbase + h;
#pragma unroll
        for (int st = 0; st < 16 * GH; ++st) {
            const int col = colbase + 2 * st + h;
            Y[st] = (iok && col < a.nb2) ? yin[2 * st] : 0.f;
        }
    }
    f32x16 racc[PTH];
#pragma unroll
    for (int pt = 0; pt < PTH; ++pt) racc[pt] = 0.f;

    const f32x4 *fa = (const f32x4 *)a.fa + lane;
    const f32x4 *ka = (const f32x4 *)job.ka + lane;
    auto load = [&](int cc, int i) -> f32x4 {
        if (i < NF) return fa[((size_t)cc * (a.nbp2 / 8) + colbase / 8 + i) * 64];
        const int j = i - NF, s4 = j / PTH, pt = j % PTH;
        return ka[(((size_t)cc * (NUP / 32) + pt0 + pt) * 4 + s4) * 64];
    };
    f32x4 ring[kRing];
    const int cfirst = min(c0, a.nchunks - 1);
#pragma unroll
    for (int d = 0; d < kRing; ++d) ring[d] = d < NL ? load(cfirst, d) : f32x4{};

    for (int c = c0; c < c1; ++c) {
        const int cnext = min(c + 1, c1 - 1);
        f32x16 Gt = 0.f;
        f32x16 Gf;
#pragma unroll
        for (int i = 0; i < NLP; ++i) {
            const f32x4 v = ring[i % kRing];
            const int nx = i + kRing;                    // the stream slot this ring slot takes next
            if (nx < NLP) {
                if (nx < NL) ring[i % kRing] = load(c, nx);
            } else if (nx - NLP < NL) {
                ring[i % kRing] = load(cnext, nx - NLP);
            }
            if (i >= NL) continue;                       // a padding slot
            if (i < NF) {
                Gt = MFMA32(v[0], Y[4 * i + 0], Gt);
                Gt = MFMA32(v[1], Y[4 * i + 1], Gt);
                Gt = MFMA32(v[2], Y[4 * i + 2], Gt);
                Gt = MFMA32(v[3], Y[4 * i + 3], Gt);
                // keep this load's issue point: later ring slots stay in flight
                __builtin_amdgcn_sched_barrier(0);
            } else {
                if (i == NF) Gf = pair_sum<PAIRS>(xs, c & 1, bp.pair, bp.half, lane, Gt);
                const int j = i - NF, s4 = j / PTH, pt = j % PTH;
                racc[pt] = MFMA32(Gf[4 * s4 + 0], v[0], racc[pt]);
                racc[pt] = MFMA32(Gf[4 * s4 + 1], v[1], racc[pt]);
                racc[pt] = MFMA32(Gf[4 * s4 + 2], v[2], racc[pt]);
                racc[pt] = MFMA32(Gf[4 * s4 + 3], v[3], racc[pt]);
                // one wave per SIMD: the PSF-table stream too keeps its loads in flight
                if constexpr (PAIRS == kWidePairs) __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
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

template <int NUP, int GH, int PAIRS>
__global__ __launch_bounds__(128 * PAIRS) void sig_adj_f32(SigArgs a)
{
    __shared__ __align__(16) float xs[2 * PAIRS * 2 * 16 * 64];
    const BlockWork bw = block_work(a);
    for (int k = 0; k < bw.ntiles; ++k) {
        if (k) __syncthreads();   // the previous tile's last exchange is read
        adj_tile<NUP, GH, PAIRS>(a, tile_pos(a, bw.tile0 + k, bw.slot, bw.group), bw.c0, bw.c1, xs);
    }
}

typedef void (*SigKernel)(SigArgs);

constexpr int kNups[] = {64, 128, 192, 256};
constexpr int kGHs[] = {3, 4, 6, 7};        // kWaves pairs per block
constexpr int kGHw[] = {8, 9, 10, 11};      // kWidePairs pairs per block

int gh_slot(int gct, int pairs)
{
    const int *gh = pairs == kWidePairs ? kGHw : kGHs;
    for (int i = 0; i < 4; ++i)
        if (gct == 2 * gh[i]) return i;
    return -1;
}
int nup_slot(int nup)
{
    for (int i = 0; i < 4; ++i)
        if (nup == kNups[i]) return i;
    return -1;
}

#define ROW(NUP, F) {F<NUP, 3, kWaves>, F<NUP, 4, kWaves>, F<NUP, 6, kWaves>, F<NUP, 7, kWaves>}
#define ROWW(NUP, F) {F<NUP, 8, kWidePairs>, F<NUP, 9, kWidePairs>, F<NUP, 10, kWidePairs>, F<NUP, 11, kWidePairs>}
const SigKernel kFwd[4][4] = {ROW(64, sig_fwd_f32), ROW(128, sig_fwd_f32), ROW(192, sig_fwd_f32),
                              ROW(256, sig_fwd_f32)};
const SigKernel kAdj[4][4] = {ROW(64, sig_adj_f32), ROW(128, sig_adj_f32), ROW(192, sig_adj_f32),
                              ROW(256, sig_adj_f32)};
const SigKernel kFwdW[4][4] = {ROWW(64, sig_fwd_f32), ROWW(128, sig_fwd_f32), ROWW(192, sig_fwd_f32),
                               ROWW(256, sig_fwd_f32)};
const SigKernel kAdjW[4][4] = {ROWW(64, sig_adj_f32), ROWW(128, sig_adj_f32), ROWW(192, sig_adj_f32),
                               ROWW(256, sig_adj_f32)};
// Fused tensor-PSF passes (FP32): the first contraction runs over all R + 1
// symmetric line sums of a line at once (a virtual line of (R + 1) n_up
// samples), in wide blocks for the registers.
constexpr int kNupF[] = {192, 256, 384, 512, 768};
constexpr int kGHf[] = {7, 8};
#define ROWF(NUP, F) {F<NUP, 7, kWidePairs>, F<NUP, 8, kWidePairs>}
const SigKernel kFwdF[5][2] = {ROWF(192, sig_fwd_f32), ROWF(256, sig_fwd_f32), ROWF(384, sig_fwd_f32),
                               ROWF(512, sig_fwd_f32), ROWF(768, sig_fwd_f32)};
const SigKernel kAdjF[5][2] = {ROWF(192, sig_adj_f32), ROWF(256, sig_adj_f32), ROWF(384, sig_adj_f32),
                               ROWF(512, sig_adj_f32), ROWF(768, sig_adj_f32)};
#undef ROW
#undef ROWW
#undef ROWF

int fused_slots(int nupf, int gct, int *ns, int *gs)
{
    *ns = *gs = -1;
    for (int i = 0; i < 5; ++i)
        if (nupf == kNupF[i]) *ns = i;
    for (int i = 0; i < 2; ++i)
        if (gct == 2 * kGHf[i]) *gs = i;
    return *ns >= 0 && *gs >= 0;
}

}  // namespace

int sig_fused_supported(int nupf, int gct)
{
    int ns, gs;
    return fused_slots(nupf, gct, &ns, &gs);
}

// fp16 variants live in sig16.hip
hipError_t launch_sig_fwd16(const mpi3d_plan *pl, SigArgs &a, hipStream_t st);
hipError_t launch_sig_adj16(const mpi3d_plan *pl, SigArgs &a, hipStream_t st);
int sig16_supported(int nup, int gct, int pairs);

int sig_fwd_supported(int nup, int gct, int precision, int pairs)
{
    if (precision == MPI3D_MIXED) return sig16_supported(nup, gct, pairs);
    return (pairs == kWaves || pairs == kWidePairs) && nup_slot(nup) >= 0 && gh_slot(gct, pairs) >= 0;
}
int sig_adj_supported(int nup, int gct, int precision, int pairs)
{
    return sig_fwd_supported(nup, gct, precision, pairs);
}

static hipError_t launch32(const SigKernel (&narrow)[4][4], const SigKernel (&wide)[4][4],
                           const SigKernel (&fused)[5][2], SigArgs &a, hipStream_t st)
{
    SigKernel k = nullptr;
    if (a.fused) {
        int ns, gs;
        if (a.pairs != kWidePairs || !fused_slots(a.nup, a.gct, &ns, &gs)) return hipErrorInvalidValue;
        k = fused[ns][gs];
    } else {
        const int ns = nup_slot(a.nup), gs = gh_slot(a.gct, a.pairs);
        if (ns < 0 || gs < 0) return hipErrorInvalidValue;
        k = a.pairs == kWidePairs ? wide[ns][gs] : narrow[ns][gs];
    }
    // main splits (one tile each), then the tail blocks (tail_tpb tiles each)
    int blocks = a.total_tiles * a.nsplit * a.ngroups;
    if (a.tail_c0 > 0) {
        if (a.tail_tpb < 1 || a.nsplit < 2 || a.tail_c0 != (a.nsplit - 1) * a.cps || a.tail_c0 >= a.nchunks)
            return hipErrorInvalidValue;
        blocks = (a.total_tiles * (a.nsplit - 1) + (a.total_tiles + a.tail_tpb - 1) / a.tail_tpb) * a.ngroups;
    }
    hipLaunchKernelGGL(k, dim3(blocks), dim3(128 * a.pairs), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_sig_fwd(const mpi3d_plan *pl, int precision, SigArgs &a, hipStream_t st)
{
    if (precision == MPI3D_MIXED) return launch_sig_fwd16(pl, a, st);
    return launch32(kFwd, kFwdW, kFwdF, a, st);
}

hipError_t launch_sig_adj(const mpi3d_plan *pl, int precision, SigArgs &a, hipStream_t st)
{
    if (precision == MPI3D_MIXED) return launch_sig_adj16(pl, a, st);
    return launch32(kAdj, kAdjW, kAdjF, a, st);
}

}  // namespace mpi3d
