// The band DFT factored over drive cycles (FP32, gfx950 v_mfma_f32_32x32x2_f32).
//
// The kept bins omega_j (eq. bcompress) are integers, so with time t = n1 + P n2
// (n1 < P, n2 < C, T = C P) the DFT phase splits exactly:
//   omega_j t = omega_j n1 + (omega_j mod C) T n2 / C   (mod T),
// and the band DFT of a line's time signal s (Appendix A, eq. DCmodel)
//   b[j] = sum_t s[t] D_j e^{+2 pi i omega_j t / T} / sqrt(T)
// becomes two short sums: a C-point DFT over the drive cycles at the R
// distinct residues r_q of the kept bins mod C,
//   Y_q[n1] = sum_n2 s[n1 + P n2] e^{+2 pi i r_q n2 / C},
// then, per bin, a P-point sum over the phase within a cycle,
//   b[j] = sum_n1 G_j[n1] Y_q(j)[n1],   G_j[n1] = D_j e^{+2 pi i omega_j n1 / T} / sqrt(T).
// When the harmonics are bunched (R small against the 2 nb kept columns) this
// replaces the T x 2nb contraction by T x 2R and P x 4nb ones.  The adjoint is
// the exact transpose of both steps.
//
// Forward: fac_fwd_kernel runs the PSF contraction of a line tile chunk by
// chunk (a chunk: 32 cycles n2 of one phase n1, PSF tables with their time
// rows in that order) and feeds each 32 x 32 (time x line) result straight
// into the residue DFT (table E), storing the phase sums Y once the C cycles
// of a phase are in; fac_fwd_out_kernel then forms b per line tile from
// LDS-staged Y, one 32-column MFMA tile per unit of at most 16 bins of one
// residue.  Adjoint: fac_adj_in_kernel forms the phase sums Z from the data,
// fac_adj_kernel runs the residue DFT's transpose and the PSF contraction's
// transpose, accumulating the lines over its phases (split partial sums
// added in a fixed order afterwards).  Y and Z are laid out per 32-line tile
// as [phase][column][line] (Y's columns 2q + re/im, Z's re/im zst + q), the
// order of an MFMA result's lines.
//
// MFMA operand conventions as in sig.hip: lane l supplies A[l % 32][l / 32]
// and B[l / 32][l % 32]; result register s of lane l holds row
// 8(s/4) + 4(l/32) + s%4, column l%32.  Every table is pre-swizzled so a lane
// fetches the operands of four consecutive MFMA steps with one 16-byte load.

#include "device.h"

namespace mpi3d {

typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

#define MFMA32(a, b, c) __builtin_amdgcn_mfma_f32_32x32x2f32((a), (b), (c), 0, 0, 0)

// Wave position of the two line-tile kernels: a block of WAVES waves covers
// WAVES consecutive 32-line tiles for one of nsplit ranges of phases n1;
// consecutive logical blocks share a range, so they share the PSF table chunks
// in their XCD's L2.
struct FacPos {
    int tile, n1a, n1b, split;
};

template <int WAVES>
__device__ __forceinline__ FacPos fac_pos(const FacArgs &a, int nsplit)
{
    const int nb = gridDim.x;
    const int lb = xcd_logical(blockIdx.x, nb);
    const int tgroups = (a.tiles + WAVES - 1) / WAVES;
    FacPos p;
    p.split = lb / tgroups;
    p.tile = (lb - p.split * tgroups) * WAVES + (int)(threadIdx.x >> 6);
    p.n1a = (int)((long)p.split * a.P / nsplit);
    p.n1b = (int)((long)(p.split + 1) * a.P / nsplit);
    return p;
}

// Forward, per wave: 32 lines, phases [n1a, n1b).  Chunk c = n1 CJ + j holds
// the times n1 + P (32 j + i), i < 32.  The block's waves walk the same
// phases, so each PSF-table chunk is staged once per block in LDS (two
// buffers: chunk c + 1 is stored while chunk c is used, chunk c + 2 already
// requested into registers; one barrier a chunk), and the residue DFT table
// sits in LDS for the whole launch.  A wave past the last tile still stages.
// Y is laid out per line tile as [phase][column][32 lines] (lines past the
// job hold the results of zero lines): a lane's 16 results of a column are
// four 16-byte runs of lines.  Each phase's stores are unconditional; columns
// past yc go to the spare row's first 8 floats.
template <int NUP, int RCT, int CJ>
__global__ __launch_bounds__(64 * kFacWavesFwd) void fac_fwd_kernel(FacArgs a)
{
    // LDS: two PSF-table chunk buffers (NK x 64 16-byte words each), then the
    // residue DFT table (CJ x NE x 64 words)
    extern __shared__ __align__(16) f32x4 lk[];
    const FacPos fp = fac_pos<kFacWavesFwd>(a, a.nsplit);
    if (fp.n1a >= fp.n1b) return;                 // the whole block
    const bool active = fp.tile < a.tiles;        // a wave past the last tile still stages
    const SigJob &job = a.job;
    const int tid = threadIdx.x, lane = tid & 63, h = lane >> 5;
    const int row0 = fp.tile * 32;
    const int r = row0 + (lane & 31);
    const long il = active && r < job.rows ? job_line(job, r) : -1;
    constexpr int NK = NUP / 8;           // PSF-table words per lane per chunk
    constexpr int NE = 4 * RCT;           // E-table words per lane per chunk
    constexpr int CW = NK * 64;           // words per chunk
    constexpr int KPT = CW / (64 * kFacWavesFwd);   // chunk words a thread stages
    f32x4 *ebuf = lk + 2 * CW;

    // B operand of the PSF contraction: rho[r][2 st + h]
    float R[NUP / 2];
    {
        const float *rin = (const float *)job.in + (size_t)(il >= 0 ? il : 0) * job.in_stride + h;
#pragma unroll
        for (int st = 0; st < NUP / 2; ++st) R[st] = (il >= 0 && 2 * st + h < a.nu) ? rin[2 * st] : 0.f;
    }
    // this lane's column of residue tile g in the wave's Y tile, or the spare row
    float *ycol[RCT];
    int ystep[RCT], jstep[RCT];
#pragma unroll
    for (int g = 0; g < RCT; ++g) {
        const int col = 32 * g + (lane & 31);
        const bool ok = col < a.yc;
        ycol[g] = a.y + (ok ? ((size_t)fp.tile * a.P * a.yc + col) * 32 : (size_t)a.ylines * a.P * a.yc) + 4 * h;
        ystep[g] = ok ? a.yc * 32 : 0;   // per phase
        jstep[g] = ok ? 8 : 0;           // per run of 4 lines
    }

    const f32x4 *kf = (const f32x4 *)job.kf;
    const f32x4 *ef = (const f32x4 *)a.ef;
    for (int idx = tid; idx < CJ * NE * 64; idx += 64 * kFacWavesFwd) ebuf[idx] = ef[idx];
    const int c0 = fp.n1a * CJ, c1 = fp.n1b * CJ;
    f32x4 pk[KPT];
    auto chunk_load = [&](int cc) {
#pragma unroll
        for (int k = 0; k < KPT; ++k) pk[k] = kf[(size_t)cc * CW + tid + 64 * kFacWavesFwd * k];
    };
    auto chunk_store = [&](int buf) {
#pragma unroll
        for (int k = 0; k < KPT; ++k) lk[buf * CW + tid + 64 * kFacWavesFwd * k] = pk[k];
    };
    chunk_load(c0);
    chunk_store(c0 & 1);
    if (c0 + 1 < c1) chunk_load(c0 + 1);
    f32x16 acc[RCT];
#pragma unroll
    for (int g = 0; g < RCT; ++g) acc[g] = 0.f;
    __syncthreads();

    for (int n1 = fp.n1a; n1 < fp.n1b; ++n1) {
#pragma unroll
        for (int j = 0; j < CJ; ++j) {
            const int c = n1 * CJ + j;
            if (active) {
                const f32x4 *kb = lk + (c & 1) * CW + lane;
                f32x16 S = 0.f;
#pragma unroll
                for (int i = 0; i < NK; ++i) {
                    const f32x4 v = kb[i * 64];
                    S = MFMA32(v[0], R[4 * i + 0], S);
                    S = MFMA32(v[1], R[4 * i + 1], S);
                    S = MFMA32(v[2], R[4 * i + 2], S);
                    S = MFMA32(v[3], R[4 * i + 3], S);
                }
                const f32x4 *eb = ebuf + j * NE * 64 + lane;
#pragma unroll
                for (int jj = 0; jj < NE; ++jj) {
                    const f32x4 v = eb[jj * 64];
                    const int g = jj / 4, s4 = jj % 4;
                    acc[g] = MFMA32(S[4 * s4 + 0], v[0], acc[g]);
                    acc[g] = MFMA32(S[4 * s4 + 1], v[1], acc[g]);
                    acc[g] = MFMA32(S[4 * s4 + 2], v[2], acc[g]);
                    acc[g] = MFMA32(S[4 * s4 + 3], v[3], acc[g]);
                }
            }
            // chunk c + 1 goes to the buffer chunk c - 1 left (read by every
            // wave before the last barrier); chunk c + 2 is requested
            if (c + 1 < c1) {
                chunk_store((c + 1) & 1);
                if (c + 2 < c1) chunk_load(c + 2);
            }
            __syncthreads();
        }
        if (active) {
#pragma unroll
            for (int g = 0; g < RCT; ++g) {
                float *d = ycol[g] + (size_t)n1 * ystep[g];
#pragma unroll
                for (int J = 0; J < 4; ++J)
                    *reinterpret_cast<f32x4 *>(d + J * jstep[g]) =
                        f32x4{acc[g][4 * J], acc[g][4 * J + 1], acc[g][4 * J + 2], acc[g][4 * J + 3]};
                acc[g] = 0.f;
            }
        }
    }
}

// Forward outer sum, one block of kOutWaves waves per 32-line tile, unit
// split and stage range (partial sums ps).  A stage of kOutStage phases of the
// tile's Y ([phase][column][32 lines]) is one contiguous block of memory, moved
// straight to LDS in that order by global_load_lds (16 bytes a lane, no
// registers; pieces of phases past P read phase P - 1, whose table entries are
// zero), and a lane's A operands for a stage are 8 single reads (one per
// phase) that the wave spreads over all 64 banks (32 consecutive lines per
// half-wave, the halves 32 floats apart).  With three buffers (two where three
// do not fit) stages s + 1 and s + 2 are in flight while stage s's products
// run.  Block barriers here carry no memory fence: a fence would wait for
// every stage in flight; each wave instead waits for its own loads of the next
// stage (vmcnt) and its LDS reads (lgkmcnt) before the barrier.  Wave w takes
// units us + usplit (w + kOutWaves i).
constexpr int kOutStage = 8;
constexpr int kOutWaves = 8;
constexpr int kUnitsPerWave = 5;

constexpr int fac_out_bufs(int zst) { return 3 * kOutStage * 2 * zst * 32 * 4 <= 160 * 1024 ? 3 : 2; }

// s_waitcnt vmcnt(n) lgkmcnt(0) (expcnt not waited for), n < 64
template <int N>
__device__ __forceinline__ void wait_vm_lgkm()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | ((N >> 4) << 14));
}

__device__ __forceinline__ void block_barrier_nofence() { asm volatile("s_barrier" ::: "memory"); }

// 16 bytes a lane from src to LDS at dst + 16 lane (dst wave-uniform).  A
// function of its own: written inside the kernel template, this gfx950-only
// form made the host pass drop the kernel's launch stubs without a message.
__device__ __forceinline__ void dma16(const float *src, float *dst) { __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0); }

template <int ZST>
__global__ __launch_bounds__(64 * kOutWaves) void fac_fwd_out_kernel(FacArgs a)
{
    extern __shared__ __align__(16) float ys[];
    constexpr int yc = 2 * ZST, NBUF = fac_out_bufs(ZST);
    constexpr int bufsz = kOutStage * yc * 32;              // floats of a stage
    constexpr int RPW = bufsz / (4 * 64 * kOutWaves);       // 64-piece runs a wave moves per stage
    static_assert(bufsz % (4 * 64 * kOutWaves) == 0, "whole runs");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5;
    const int tile = blockIdx.x, us = blockIdx.y, nus = gridDim.y, ps = blockIdx.z;
    const SigJob &job = a.job;
    const int row0 = tile * 32;
    // run k of wave w moves floats 4 (64 (kOutWaves k + w) + lane) .. + 3 of the stage
    int pph[RPW], poff[RPW];
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int f = 4 * (64 * (kOutWaves * k + wave) + lane);
        pph[k] = f / (yc * 32);
        poff[k] = f - pph[k] * (yc * 32);
    }
    const float *yt = a.y + (size_t)tile * a.P * yc * 32;
    auto stage_dma = [&](int stg, int buf) {
#pragma unroll
        for (int k = 0; k < RPW; ++k) {
            const int n1 = min(stg * kOutStage + pph[k], a.P - 1);
            dma16(yt + (size_t)n1 * yc * 32 + poff[k], ys + buf * bufsz + 256 * (kOutWaves * k + wave));
        }
    };
    f32x16 acc[kUnitsPerWave];
#pragma unroll
    for (int i = 0; i < kUnitsPerWave; ++i) acc[i] = 0.f;
    int uu[kUnitsPerWave], aoff[kUnitsPerWave];
#pragma unroll
    for (int i = 0; i < kUnitsPerWave; ++i) {
        uu[i] = us + nus * (wave + kOutWaves * i);
        const int q = a.uq[uu[i] < a.U ? uu[i] : 0];   // unconditional: the five loads overlap
        const int col = 2 * (uu[i] < a.U ? q : 0) + h;
        aoff[i] = col * 32 + (lane & 31);
    }
    // this block's stages [s0, s1): range ps of psplit
    const int nst = (a.P + kOutStage - 1) / kOutStage;
    const int s0 = (int)((long)ps * nst / a.psplit), s1 = (int)((long)(ps + 1) * nst / a.psplit);
    // table operands of stage n1s / kOutStage for this wave's units
    auto table_load = [&](int n1s, f32x4 (&b0)[kUnitsPerWave], f32x4 (&b1)[kUnitsPerWave]) {
#pragma unroll
        for (int i = 0; i < kUnitsPerWave; ++i) {
            const int u = uu[i] < a.U ? uu[i] : 0;
            const f32x4 *w = (const f32x4 *)a.wf + ((size_t)u * (a.Pp / 4) + n1s / 4) * 64 + lane;
            b0[i] = w[0];
            b1[i] = w[64];
        }
    };
    f32x4 b0[kUnitsPerWave], b1[kUnitsPerWave], n0[kUnitsPerWave], n1v[kUnitsPerWave];
    table_load(s0 * kOutStage, b0, b1);
    __builtin_amdgcn_sched_barrier(0);   // ahead of the stage loads: in by the first wait
    // stages s0 .. s0 + NBUF - 2 requested (stage numbers past the range
    // repeat its last stage, so every wait below counts the same loads)
#pragma unroll
    for (int k = 0; k < NBUF - 1; ++k) stage_dma(min(s0 + k, s1 - 1), (s0 + k) % NBUF);
    wait_vm_lgkm<(NBUF - 2) * RPW>();   // stage s0 is in
    block_barrier_nofence();
    for (int stg = s0; stg < s1; ++stg) {
        const int n1s = stg * kOutStage;
        table_load(min(n1s + kOutStage, (s1 - 1) * kOutStage), n0, n1v);
        __builtin_amdgcn_sched_barrier(0);
        // stage stg + NBUF - 1 to the buffer stage stg - 1 left (every wave is
        // past its products: the barrier at the end of the last stage)
        stage_dma(min(stg + NBUF - 1, s1 - 1), (stg + NBUF - 1) % NBUF);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < kUnitsPerWave; ++i) {
            if (uu[i] >= a.U) break;
            const float *src = ys + (stg % NBUF) * bufsz + aoff[i];
            float av[kOutStage];
#pragma unroll
            for (int k = 0; k < kOutStage; ++k) av[k] = src[k * yc * 32];
            acc[i] = MFMA32(av[0], b0[i][0], acc[i]);
            acc[i] = MFMA32(av[1], b0[i][1], acc[i]);
            acc[i] = MFMA32(av[2], b0[i][2], acc[i]);
            acc[i] = MFMA32(av[3], b0[i][3], acc[i]);
            acc[i] = MFMA32(av[4], b1[i][0], acc[i]);
            acc[i] = MFMA32(av[5], b1[i][1], acc[i]);
            acc[i] = MFMA32(av[6], b1[i][2], acc[i]);
            acc[i] = MFMA32(av[7], b1[i][3], acc[i]);
        }
#pragma unroll
        for (int i = 0; i < kUnitsPerWave; ++i) {
            b0[i] = n0[i];
            b1[i] = n1v[i];
        }
        // stage stg + 1 is in (only the NBUF - 2 later stages' loads may be
        // outstanding), and this wave's LDS reads are done
        wait_vm_lgkm<(NBUF - 2) * RPW>();
        block_barrier_nofence();
    }
    // the repeated last-stage loads still in flight land before the block
    // ends and its LDS is handed to another block
    wait_vm_lgkm<0>();
    // column l%32 of unit u: bin slot col/2, re/im col%2
#pragma unroll
    for (int i = 0; i < kUnitsPerWave; ++i) {
        const int u = uu[i];
        if (u >= a.U) break;
        const int col = lane & 31;
        const int jb = a.ubin[u * 16 + col / 2];
        if (jb < 0) continue;
        const int oc = 2 * jb + (col & 1);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int row = row0 + 8 * (j / 4) + 4 * h + (j % 4);
            if (row < job.rows) job.part[ps * a.fwd_part_stride + (size_t)job_line(job, row) * a.nbp2 + oc] = acc[i][j];
        }
    }
}

// Adjoint outer sum: Z from the data, one block of kInWaves waves per 32-line
// tile and stage range; stages of 16 phases (a 32-column MFMA tile: phase
// col/2, re/im col%2).  Z is laid out per line tile as [phase][re/im][q][32
// lines], the MFMA result's own order: a lane's 16 results for residue q are
// four runs of four consecutive lines, written as 16-byte stores straight from
// the accumulator (no LDS, no barriers).  Wave w takes residue slots
// w + kInWaves i (the plan numbers the residues so the waves' bin counts
// balance); slots in [R, zst) are written as zeros, and slots past zst and
// phases past P go to the spare row, so every stage issues the same stores and
// its products wait for its own table loads, never for earlier stores.  The
// data operands (the bins of the wave's residues, up to kQMax steps each) stay
// in registers, and each stage's table operands are requested during the
// stage before.
constexpr int kZStage = 16;
constexpr int kWaitVmcnt0 = 0x0f70;   // s_waitcnt vmcnt(0), expcnt and lgkmcnt not waited for
constexpr int kInWaves = kFacInWaves;
constexpr int kResPerWave = 3;

__global__ __launch_bounds__(64 * kInWaves) void fac_adj_in_kernel(FacArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5;
    const int tile = blockIdx.x, zsp = blockIdx.y;
    const SigJob &job = a.job;
    const int row0 = tile * 32;
    const int r = row0 + (lane & 31);
    const long il = r < job.rows ? job_line(job, r) : -1;
    const int zst = a.zst;
    int qq[kResPerWave], qs[kResPerWave];
#pragma unroll
    for (int i = 0; i < kResPerWave; ++i) {
        qq[i] = wave + kInWaves * i;
        qs[i] = qq[i] < a.R ? a.qsteps[qq[i]] : 0;
    }
    // A operands: y[r][2 qbin[q][st] + h].  Per residue the bin numbers are
    // requested together, then the data (clamped addresses, masked values), so
    // the loads overlap instead of each data load waiting for its bin number.
    float Yv[kResPerWave][kQMax];
    {
        const float *yin = (const float *)job.in + (size_t)(il >= 0 ? il : 0) * job.in_stride + h;
#pragma unroll
        for (int i = 0; i < kResPerWave; ++i) {
            const int *qb = a.qbin + (qq[i] < a.R ? qq[i] : 0) * kQMax;
            int jb[kQMax];
#pragma unroll
            for (int st = 0; st < kQMax; ++st) jb[st] = qb[st];
#pragma unroll
            for (int st = 0; st < kQMax; ++st) {
                const bool ok = qq[i] < a.R && il >= 0 && jb[st] >= 0;
                const float v = yin[2 * (jb[st] >= 0 ? jb[st] : 0)];
                Yv[i][st] = ok ? v : 0.f;
            }
        }
    }
    // this block's stages [s0, s1): range zsp of zsplit
    const int nst = (a.P + kZStage - 1) / kZStage;
    const int s0 = (int)((long)zsp * nst / a.zsplit), s1 = (int)((long)(zsp + 1) * nst / a.zsplit);
    // table operands of stage stg for this wave's residues
    auto table_load = [&](int stg, f32x4 (&b)[kResPerWave][kQMax / 4]) {
#pragma unroll
        for (int i = 0; i < kResPerWave; ++i) {
            const int q = qq[i] < a.R ? qq[i] : 0;
            const f32x4 *w = (const f32x4 *)a.wa + ((size_t)(q * a.nzstage + stg) * (kQMax / 4)) * 64 + lane;
#pragma unroll
            for (int s4 = 0; s4 < kQMax / 4; ++s4) b[i][s4] = w[s4 * 64];
        }
    };
    // this tile's Z, and the spare row (phase 0) for the stores that carry nothing
    float *const zt = a.y + (size_t)tile * 32 * a.P * 2 * zst + 4 * h;
    float *const spare = a.y + (size_t)a.ylines * a.P * 2 * zst + 4 * h;
    const int col = lane & 31, n1l = col >> 1, cr = col & 1;
    f32x4 b[kResPerWave][kQMax / 4], bn[kResPerWave][kQMax / 4];
    table_load(s0, b);
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);   // (so no stage waits for an earlier stage's stores)
    for (int stg = s0; stg < s1; ++stg) {
        table_load(min(stg + 1, s1 - 1), bn);   // the next stage's, during this one
        const int n1 = stg * kZStage + n1l;
#pragma unroll
        for (int i = 0; i < kResPerWave; ++i) {
            f32x16 acc = 0.f;
            if (qq[i] < a.R) {
#pragma unroll
                for (int s4 = 0; s4 < kQMax / 4; ++s4) {
                    if (4 * s4 >= qs[i]) break;
                    acc = MFMA32(Yv[i][4 * s4 + 0], b[i][s4][0], acc);
                    acc = MFMA32(Yv[i][4 * s4 + 1], b[i][s4][1], acc);
                    acc = MFMA32(Yv[i][4 * s4 + 2], b[i][s4][2], acc);
                    acc = MFMA32(Yv[i][4 * s4 + 3], b[i][s4][3], acc);
                }
            }
            // lines 8 J + 4 h .. + 3 of column (n1, re/im cr), residue slot qq[i];
            // the stores that carry nothing all go to the spare row's first 8 floats
            const bool real = n1 < a.P && qq[i] < zst;
            float *d = real ? zt + ((size_t)(n1 * 2 + cr) * zst + qq[i]) * 32 : spare;
            const int js = real ? 8 : 0;
#pragma unroll
            for (int J = 0; J < 4; ++J)
                *reinterpret_cast<f32x4 *>(d + js * J) = f32x4{acc[4 * J], acc[4 * J + 1], acc[4 * J + 2], acc[4 * J + 3]};
        }
#pragma unroll
        for (int i = 0; i < kResPerWave; ++i)
#pragma unroll
            for (int s4 = 0; s4 < kQMax / 4; ++s4) b[i][s4] = bn[i][s4];
    }
}

// Adjoint, per wave: 32 lines, phases [n1a, n1b): for each chunk the residue
// DFT's transpose (A = E[time n2][col], B = Z[line][col]) then the PSF
// contraction's transpose into the lines; split partial sums per phase range.
// The PSF-table chunks are staged once per block in LDS as in the forward,
// the residue DFT table sits in LDS, and the next phase's Z operands are
// requested before its CJ chunks.
template <int NUP, int ZST, int CJ>
__global__ __launch_bounds__(64 * kFacWavesAdj) void fac_adj_kernel(FacArgs a)
{
    extern __shared__ __align__(16) f32x4 lk[];
    const FacPos fp = fac_pos<kFacWavesAdj>(a, a.nsplit_adj);
    if (fp.n1a >= fp.n1b) return;                 // the whole block
    const bool active = fp.tile < a.tiles;        // a wave past the last tile still stages
    const SigJob &job = a.job;
    const int tid = threadIdx.x, lane = tid & 63, h = lane >> 5;
    const int row0 = fp.tile * 32;
    const int r = row0 + (lane & 31);
    constexpr int PT = NUP / 32;          // detector tiles
    constexpr int NE = ZST / 4;           // E-table words per lane per chunk
    constexpr int NK = 4 * PT;            // PSF-table words per lane per chunk
    constexpr int CW = NK * 64;           // words per chunk
    constexpr int KPT = CW / (64 * kFacWavesAdj);
    constexpr int ZC = 2 * ZST;
    f32x4 *ebuf = lk + 2 * CW;

    f32x16 racc[PT];
#pragma unroll
    for (int pt = 0; pt < PT; ++pt) racc[pt] = 0.f;
    const f32x4 *ka = (const f32x4 *)job.ka;
    const f32x4 *ea = (const f32x4 *)a.ea;
    for (int idx = tid; idx < CJ * NE * 64; idx += 64 * kFacWavesAdj) ebuf[idx] = ea[idx];
    // B operand of the residue DFT's transpose: Z of this line tile, laid out
    // [phase][re/im][q][32 lines]: line r, half h, columns st < ZST (lines past
    // the job hold zeros).  A lane's ZST values of a phase are single floats
    // 128 bytes apart; the wave's loads of one st are two 128-byte runs.
    const float *zrow = a.y + (size_t)(active ? fp.tile : 0) * 32 * a.P * ZC + h * ZST * 32 + (lane & 31);
    auto zload = [&](int n1, float (&zb)[ZST]) {
#pragma unroll
        for (int st = 0; st < ZST; ++st) zb[st] = zrow[(size_t)n1 * ZC * 32 + st * 32];
    };
    const int c0 = fp.n1a * CJ, c1 = fp.n1b * CJ;
    f32x4 pk[KPT];
    auto chunk_load = [&](int cc) {
#pragma unroll
        for (int k = 0; k < KPT; ++k) pk[k] = ka[(size_t)cc * CW + tid + 64 * kFacWavesAdj * k];
    };
    auto chunk_store = [&](int buf) {
#pragma unroll
        for (int k = 0; k < KPT; ++k) lk[buf * CW + tid + 64 * kFacWavesAdj * k] = pk[k];
    };
    float zb[ZST], zn[ZST];
    zload(fp.n1a, zb);
    chunk_load(c0);
    chunk_store(c0 & 1);
    if (c0 + 1 < c1) chunk_load(c0 + 1);
    __syncthreads();

    for (int n1 = fp.n1a; n1 < fp.n1b; ++n1) {
        zload(min(n1 + 1, fp.n1b - 1), zn);   // the next phase's operands
#pragma unroll
        for (int j = 0; j < CJ; ++j) {
            const int c = n1 * CJ + j;
            if (active) {
                const f32x4 *eb = ebuf + j * NE * 64 + lane;
                f32x16 G = 0.f;
#pragma unroll
                for (int i = 0; i < NE; ++i) {
                    const f32x4 v = eb[i * 64];
                    G = MFMA32(v[0], zb[4 * i + 0], G);
                    G = MFMA32(v[1], zb[4 * i + 1], G);
                    G = MFMA32(v[2], zb[4 * i + 2], G);
                    G = MFMA32(v[3], zb[4 * i + 3], G);
                }
                const f32x4 *kb = lk + (c & 1) * CW + lane;
#pragma unroll
                for (int jj = 0; jj < NK; ++jj) {
                    const int s4 = jj / PT, pt = jj % PT;
                    const f32x4 v = kb[(pt * 4 + s4) * 64];
                    racc[pt] = MFMA32(G[4 * s4 + 0], v[0], racc[pt]);
                    racc[pt] = MFMA32(G[4 * s4 + 1], v[1], racc[pt]);
                    racc[pt] = MFMA32(G[4 * s4 + 2], v[2], racc[pt]);
                    racc[pt] = MFMA32(G[4 * s4 + 3], v[3], racc[pt]);
                }
            }
            // chunk c + 1 goes to the buffer chunk c - 1 left (read by every
            // wave before the last barrier); chunk c + 2 is requested
            if (c + 1 < c1) {
                chunk_store((c + 1) & 1);
                if (c + 2 < c1) chunk_load(c + 2);
            }
            __syncthreads();
        }
#pragma unroll
        for (int st = 0; st < ZST; ++st) zb[st] = zn[st];
    }
    if (!active) return;
    float *out = job.part + (size_t)fp.split * job.part_stride;
#pragma unroll
    for (int pt = 0; pt < PT; ++pt) {
        const int col = pt * 32 + (lane & 31);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int row = row0 + 8 * (j / 4) + 4 * h + (j % 4);
            if (row < job.rows) out[(size_t)job_line(job, row) * NUP + col] = racc[pt][j];
        }
    }
}

typedef void (*FacKernel)(FacArgs);
struct FacOut {
    FacKernel fn;
    int nbuf;
};
#define FAC_OUT(Z) {fac_fwd_out_kernel<Z>, fac_out_bufs(Z)}
const FacOut kFacFwdOut[8] = {FAC_OUT(4),  FAC_OUT(8),  FAC_OUT(12), FAC_OUT(16),
                              FAC_OUT(20), FAC_OUT(24), FAC_OUT(28), FAC_OUT(32)};
#undef FAC_OUT
constexpr int kFacNups[] = {64, 128, 192, 256};
#define FAC_FWD_ROW(NUP)                                                                                     \
    {{fac_fwd_kernel<NUP, 1, 1>, fac_fwd_kernel<NUP, 1, 2>}, {fac_fwd_kernel<NUP, 2, 1>, fac_fwd_kernel<NUP, 2, 2>}}
const FacKernel kFacFwd[4][2][2] = {FAC_FWD_ROW(64), FAC_FWD_ROW(128), FAC_FWD_ROW(192), FAC_FWD_ROW(256)};
#undef FAC_FWD_ROW
#define FAC_ADJ_Z(NUP, Z) {fac_adj_kernel<NUP, Z, 1>, fac_adj_kernel<NUP, Z, 2>}
#define FAC_ADJ_ROW(NUP)                                                                                     \
    {FAC_ADJ_Z(NUP, 4), FAC_ADJ_Z(NUP, 8), FAC_ADJ_Z(NUP, 12), FAC_ADJ_Z(NUP, 16), FAC_ADJ_Z(NUP, 20),         \
     FAC_ADJ_Z(NUP, 24), FAC_ADJ_Z(NUP, 28), FAC_ADJ_Z(NUP, 32)}
const FacKernel kFacAdj[4][8][2] = {FAC_ADJ_ROW(64), FAC_ADJ_ROW(128), FAC_ADJ_ROW(192), FAC_ADJ_ROW(256)};
#undef FAC_ADJ_ROW
#undef FAC_ADJ_Z

int fac_nup_slot(int nup)
{
    for (int i = 0; i < 4; ++i)
        if (kFacNups[i] == nup) return i;
    return -1;
}

}  // namespace

int fac_supported(int nup, int rct, int zst, int cj)
{
    return fac_nup_slot(nup) >= 0 && rct >= 1 && rct <= 2 && zst >= 4 && zst <= 32 && zst % 4 == 0 && cj >= 1 &&
           cj <= 2;
}

static bool fac_args_ok(const FacArgs &a)
{
    return a.tiles > 0 && a.P > 0 && a.cj > 0 && a.nsplit >= 1 && a.nsplit <= a.P && a.nsplit_adj >= 1 &&
           a.nsplit_adj <= a.P && a.yc % 4 == 0 &&
           a.yc == 2 * a.zst && a.yc <= 32 * a.rct && a.R <= kInWaves * kResPerWave && a.R <= a.zst && a.yc <= 64 &&
           a.Pp % kOutStage == 0 && a.Pp >= a.P && a.nzstage * kZStage >= a.P &&
           fac_supported(a.nup, a.rct, a.zst, a.cj) && a.job.rows <= a.tiles * 32 &&
           a.ylines >= a.tiles * 32 && (long)(a.ylines + 1) * a.P * a.yc < 0x7fffffffL && a.psplit >= 1 &&
           a.psplit <= (a.P + kOutStage - 1) / kOutStage && a.zsplit >= 1 && a.zsplit <= a.nzstage;
}

hipError_t launch_fac_part(const FacArgs &a, int part, hipStream_t st)
{
    if (a.job.rows <= 0) return hipSuccess;
    if (!fac_args_ok(a) || part < 0 || part > 3) return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    switch (part) {
    case kFacFwdInner: {
        const size_t lds = 16 * 64 * (size_t)(2 * a.nup / 8 + a.cj * 4 * a.rct);
        const FacKernel k = kFacFwd[fac_nup_slot(a.nup)][a.rct - 1][a.cj - 1];
        if (lds > 64 * 1024) {
            e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k, dim3((a.tiles + kFacWavesFwd - 1) / kFacWavesFwd * a.nsplit), dim3(64 * kFacWavesFwd),
                           lds, st, a);
        break;
    }
    case kFacFwdOuter: {
        if (a.usplit < 1 || a.usplit > kMaxFacSplit || a.U > kOutWaves * kUnitsPerWave * a.usplit)
            return hipErrorInvalidValue;
        const FacOut &k = kFacFwdOut[a.zst / 4 - 1];
        const size_t lds = sizeof(float) * (size_t)k.nbuf * kOutStage * 2 * a.zst * 32;
        if (lds > 64 * 1024) {
            e = hipFuncSetAttribute((const void *)k.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k.fn, dim3(a.tiles, a.usplit, a.psplit), dim3(64 * kOutWaves), lds, st, a);
        break;
    }
    case kFacAdjOuter:
        hipLaunchKernelGGL(fac_adj_in_kernel, dim3(a.tiles, a.zsplit), dim3(64 * kInWaves), 0, st, a);
        break;
    default: {
        const size_t lds = 16 * 64 * (size_t)(2 * a.nup / 8 + a.cj * a.zst / 4);
        const FacKernel k = kFacAdj[fac_nup_slot(a.nup)][a.zst / 4 - 1][a.cj - 1];
        if (lds > 64 * 1024) {
            e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k, dim3((a.tiles + kFacWavesAdj - 1) / kFacWavesAdj * a.nsplit_adj), dim3(64 * kFacWavesAdj),
                           lds, st, a);
        break;
    }
    }
    return hipGetLastError();
}

hipError_t launch_fac_fwd(const FacArgs &a, hipStream_t st)
{
    hipError_t e = launch_fac_part(a, kFacFwdInner, st);
    return e == hipSuccess ? launch_fac_part(a, kFacFwdOuter, st) : e;
}

hipError_t launch_fac_adj(const FacArgs &a, hipStream_t st)
{
    hipError_t e = launch_fac_part(a, kFacAdjOuter, st);
    return e == hipSuccess ? launch_fac_part(a, kFacAdjInner, st) : e;
}

}  // namespace mpi3d
