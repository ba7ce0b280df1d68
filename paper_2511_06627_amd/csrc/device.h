// Device helpers shared by the kernel sources (proj.hip, sig.hip, sig16.hip).
#pragma once

#include "internal.h"

namespace mpi3d {

typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

// blockIdx -> logical block so that consecutive logical blocks share an XCD
// (blocks are dealt to the 8 XCDs round-robin; XCD x receives
// nblocks / 8 + (x < nblocks % 8) of them).
__device__ __forceinline__ int xcd_logical(int bid, int nblocks)
{
    const int nx = 8;
    int xcd = bid % nx, slot = bid / nx;
    int per = nblocks / nx, rem = nblocks % nx;
    return xcd * per + min(xcd, rem) + slot;
}

// Where a signal-kernel block and wave sit: the block covers a.pairs *
// kRowsPerWave lines (a tile) of one job, for one time split and one column
// group; wave w is half w & 1 of pair w >> 1, which owns kRowsPerWave lines
// from row0.
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
    bp.row0 = (tile - a.jobs[jb].tile0) * (a.pairs * kRowsPerWave) + bp.pair * kRowsPerWave;
    return bp;
}

// The work of an FP32 signal-kernel block: tiles tile0 .. tile0 + ntiles - 1
// of column group `group` over time chunks [c0, c1), written to partial-sum
// slot `slot`.  The first total_tiles x main splits x ngroups logical blocks
// take one tile and one split of cps chunks each; with a tail (tail_c0 > 0,
// the main splits covering [0, tail_c0)), the remaining blocks take tail_tpb
// tiles each over [tail_c0, nchunks) into the last slot, so every block does
// about the same number of chunks on 256 CUs.
struct BlockWork {
    int tile0, ntiles, group, slot, c0, c1;
};

__device__ __forceinline__ BlockWork block_work(const SigArgs &a)
{
    BlockWork w;
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int msplit = a.tail_c0 > 0 ? a.nsplit - 1 : a.nsplit;
    const int nmain = a.total_tiles * msplit * a.ngroups;
    if (lb < nmain) {
        w.tile0 = lb % a.total_tiles;
        w.ntiles = 1;
        const int sg = lb / a.total_tiles;
        w.group = sg % a.ngroups;
        w.slot = sg / a.ngroups;
        w.c0 = w.slot * a.cps;
        w.c1 = min(w.c0 + a.cps, a.tail_c0 > 0 ? a.tail_c0 : a.nchunks);
    } else {
        const int tb = lb - nmain;
        w.group = tb % a.ngroups;
        w.tile0 = (tb / a.ngroups) * a.tail_tpb;
        w.ntiles = min(a.tail_tpb, a.total_tiles - w.tile0);
        w.slot = msplit;
        w.c0 = a.tail_c0;
        w.c1 = a.nchunks;
    }
    return w;
}

// The position of this wave in tile `tile` (see locate).
__device__ __forceinline__ BlockPos tile_pos(const SigArgs &a, int tile, int slot, int group)
{
    BlockPos bp;
    bp.group = group;
    bp.split = slot;
    int jb = 0;
    for (int j = 1; j < a.njobs; ++j)
        if (tile >= a.jobs[j].tile0) jb = j;
    bp.job = jb;
    const int w = threadIdx.x >> 6;
    bp.pair = w >> 1;
    bp.half = w & 1;
    bp.row0 = (tile - a.jobs[jb].tile0) * (a.pairs * kRowsPerWave) + bp.pair * kRowsPerWave;
    return bp;
}

// Swap partial time tiles within a pair: write mine, barrier, read the
// partner's, and return lo + hi (the same operand order on both waves).  xs
// holds two parities x PAIRS pairs x 2 halves x 16 x 64 floats.
template <int PAIRS>
__device__ __forceinline__ f32x16 pair_sum(float *xs, int parity, int pair, int half, int lane, const f32x16 &mine)
{
    // 16-byte words, word q of lane l at q * 64 + l: four 128-bit LDS
    // accesses each way, consecutive lanes on consecutive words
    typedef float f32x4v __attribute__((ext_vector_type(4)));
    f32x4v *slot = reinterpret_cast<f32x4v *>(xs) + ((parity * PAIRS + pair) * 2) * 4 * 64;
    f32x4v *own = slot + half * 4 * 64;
    const f32x4v *other = slot + (1 - half) * 4 * 64;
#pragma unroll
    for (int q = 0; q < 4; ++q) own[q * 64 + lane] = f32x4v{mine[4 * q], mine[4 * q + 1], mine[4 * q + 2], mine[4 * q + 3]};
    __syncthreads();
    f32x16 r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const f32x4v o = other[q * 64 + lane];
#pragma unroll
        for (int e = 0; e < 4; ++e) r[4 * q + e] = half == 0 ? mine[4 * q + e] + o[e] : o[e] + mine[4 * q + e];
    }
    return r;
}

}  // namespace

}  // namespace mpi3d
