// Plan creation: validation, float64 host tables, upload, workspace layout,
// and the operator entry points of the C ABI (forward, adjoint, stages).
//
// Tables follow the paper's factors:
//   cos/sin of the FFL angles           Sec. 2.2, eq. qtheta
//   ray-sample coordinate bases          eq. ptheta2 (unit-step Riemann sum)
//   PSF kernel K[n][p]                   eq. reals0 + Appendix B eq. PSF
//       = v_n L'((xi_n - u_p)/w) / w, xi_n = a sin(2 pi P n / T), v = xi'
//       (the global scale c_A is applied in fp64 when split sums are reduced,
//       so scans that differ only in c_A share identical line tables)
//   band DFT F[n][2j], F[n][2j+1]        Appendix A (+i, 1/sqrt(T)) on the kept
//       = Re/Im(D_j e^{+2 pi i (omega_j n mod T)/T}) / sqrt(T)   bins (eq. bcompress,
//                                        eq. DCmodel)
// All table values are computed in float64 and rounded once.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "internal.h"

using namespace mpi3d;

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// L'(x) = 1/x^2 - 1/sinh^2 x.  For |x| < 0.5 the Maclaurin series
// sum_{n>=1} 2^{2n} B_{2n} (2n-1) x^{2n-2} / (2n)! (Bernoulli numbers B_{2n});
// for larger |x| the closed form, written with e^{-2|x|} so nothing overflows.
double langevin_deriv(double x)
{
    x = std::fabs(x);
    if (x < 0.5) {
        static const double bern[] = {1.0 / 6, -1.0 / 30, 1.0 / 42, -1.0 / 30, 5.0 / 66, -691.0 / 2730,
                                      7.0 / 6, -3617.0 / 510, 43867.0 / 798, -174611.0 / 330};
        double coef[10];
        double fact = 1.0, pow4 = 1.0;
        for (int n = 1; n <= 10; ++n) {
            fact *= (2.0 * n - 1) * (2.0 * n);
            pow4 *= 4.0;
            coef[n - 1] = pow4 * bern[n - 1] * (2.0 * n - 1) / fact;
        }
        double x2 = x * x, acc = 0.0;
        for (int n = 9; n >= 0; --n) acc = acc * x2 + coef[n];
        return acc;
    }
    double e = std::exp(-2.0 * x);
    return 1.0 / (x * x) - 4.0 * e / ((1.0 - e) * (1.0 - e));
}

// L(x) = coth x - 1/x.  For |x| < 0.5 the Maclaurin series
// sum_{n>=1} 2^{2n} B_{2n} x^{2n-1} / (2n)!; for larger |x| the closed form,
// where the two terms differ by at least 8% and nothing cancels badly.
double langevin(double x)
{
    const double ax = std::fabs(x);
    if (ax < 0.5) {
        static const double bern[] = {1.0 / 6, -1.0 / 30, 1.0 / 42, -1.0 / 30, 5.0 / 66, -691.0 / 2730,
                                      7.0 / 6, -3617.0 / 510, 43867.0 / 798, -174611.0 / 330};
        double coef[10];
        double fact = 1.0, pow4 = 1.0;
        for (int n = 1; n <= 10; ++n) {
            fact *= (2.0 * n - 1) * (2.0 * n);
            pow4 *= 4.0;
            coef[n - 1] = pow4 * bern[n - 1] / fact;
        }
        double x2 = x * x, acc = 0.0;
        for (int n = 9; n >= 0; --n) acc = acc * x2 + coef[n];
        return x * acc;
    }
    return 1.0 / std::tanh(x) - 1.0 / x;
}

// xx entry of the tensor PSF at in-plane offset (du, dz), dz != 0, with the
// gradient magnitude equal on both axes: L'(r/w)/w du^2/r^2 + L(r/w) dz^2/r^3.
double psf_xx(double du, double dz, double w)
{
    const double r2 = du * du + dz * dz, r = std::sqrt(r2);
    return langevin_deriv(r / w) / w * (du * du / r2) + langevin(r / w) * (dz * dz / (r2 * r));
}

// double -> fp16, rounded once (clang's _Float16 conversion is correctly rounded)
inline _Float16 to_f16(double v) { return (_Float16)v; }

int round_up(int v, int m) { return (v + m - 1) / m * m; }
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Ray samples: smallest n >= sqrt(nx^2 + ny^2) with the parity of ny.
int ray_count(int nx, int ny)
{
    long d2 = (long)nx * nx + (long)ny * ny;
    int n = (int)std::floor(std::sqrt((double)d2));
    while ((long)n * n < d2) ++n;
    while (n > 0 && (long)(n - 1) * (n - 1) >= d2) --n;
    if ((n - ny) % 2) ++n;
    return n;
}

// Column groups of one precision's signal kernels for a band table of nct0
// 32-wide column tiles.  A pair covers 2 GH tiles of one group.  Narrow
// blocks (4 pairs, two waves per SIMD) hold at most 14 tiles per pair; wide
// blocks (2 pairs, one wave per SIMD: FP32 only) up to 22, so a table of 15 to
// 22 tiles needs one group instead of two -- each extra group repeats the
// first contraction (the time signal) for its lines.  Tables are zero-padded
// to the group width, so the kernels need no per-tile guards.
void column_groups(int nct0, bool fp32, mpi3d_plan::SigCfg &c)
{
    static const int widths[] = {6, 8, 12, 14};
    if (fp32 && nct0 > 14 && nct0 <= 22) {
        c.pairs = kWidePairs;
        c.ngroups = 1;
        c.gct = (nct0 + 1) / 2 * 2;
        return;
    }
    c.pairs = kWaves;
    c.ngroups = (nct0 + 13) / 14;
    const int want = (nct0 + c.ngroups - 1) / c.ngroups;
    c.gct = 0;
    for (int wdt : widths)
        if (!c.gct && wdt >= want) c.gct = wdt;
}

// Choose the T-split of one precision: (line tiles x splits x groups) blocks,
// one block resident per CU (narrow blocks need about 250 VGPRs a wave at two
// waves per SIMD, wide ones more than 256 at one).  Cost in seconds: rounds of
// blocks times chunks per block times one block's time per chunk, at the
// per-CU MFMA rate measured on MI355X (FP32 about 4.3e11 flop/s, fp16 about
// 2.3e12), plus each split's partial sums written and read back by the
// reduction at about 5 TB/s.
void choose_split(const mpi3d_plan *pl, bool fp32, mpi3d_plan::SigCfg &c, int nup, int passes)
{
    const int slots = 256;
    const int rows = kRowsPerWave * c.pairs;
    const long tiles = (pl->L + rows - 1) / rows;
    const double rate = fp32 ? 4.3e11 : 2.3e12;
    const double t_chunk = (double)rows * kChunk * 2.0 * (nup + kColTile * c.gct) / rate;
    const double split_bytes = 8.0 * passes * pl->L * std::max<double>(pl->nbp2, (double)c.ngroups * nup);
    int best_s = 1;
    double best = 1e30;
    for (int s = 1; s <= pl->nchunks; ++s) {
        int cps = (pl->nchunks + s - 1) / s;
        int used = (pl->nchunks + cps - 1) / cps;  // splits actually non-empty
        long blocks = tiles * used * c.ngroups;
        long rounds = (blocks + slots - 1) / slots;
        double cost = (double)rounds * cps * t_chunk + used * split_bytes / 5e12;
        if (cost < best * (1.0 - 1e-9)) {
            best = cost;
            best_s = used;
        }
    }
    c.cps = (pl->nchunks + best_s - 1) / best_s;
    c.nsplit = (pl->nchunks + c.cps - 1) / c.cps;
    c.tail_c0 = c.tail_tpb = 0;
    // FP32 wide blocks (one per CU): a tail split can even the load when the
    // tiles times the splits leave CUs idle -- s splits of w chunks per tile,
    // and the remaining r = nchunks - s w chunks of every tile gathered
    // tail_tpb tiles to a block, all in one round of blocks
    if (fp32 && c.pairs == kWidePairs) {
        const long per_group = slots / c.ngroups;
        for (int w = (int)((tiles * pl->nchunks + per_group - 1) / per_group); w < pl->nchunks; ++w) {
            const int s = pl->nchunks / w, r = pl->nchunks - s * w;
            if (r == 0) continue;
            const int tpb = std::max(1, w / r);
            const long blocks = (tiles * s + (tiles + tpb - 1) / tpb) * c.ngroups;
            if (blocks > slots) continue;
            const double cost = std::max(w, tpb * r) * t_chunk + (s + 1) * split_bytes / 5e12;
            if (cost < best * (1.0 - 1e-9)) {
                best = cost;
                c.cps = w;
                c.nsplit = s + 1;
                c.tail_c0 = s * w;
                c.tail_tpb = tpb;
            }
        }
    }
    // Serving launches merge the lines of several requests, so their time
    // split must not depend on the line count: a fixed split per line class.
    c.serve_nsplit = std::min(pl->nchunks, 16);
    c.serve_cps = (pl->nchunks + c.serve_nsplit - 1) / c.serve_nsplit;
    c.serve_nsplit = (pl->nchunks + c.serve_cps - 1) / c.serve_cps;
}

template <class T>
T *carve(char *base, size_t &off, size_t count)
{
    off = align256(off);
    T *p = reinterpret_cast<T *>(base + off);
    off += count * sizeof(T);
    return p;
}

}  // namespace

extern "C" const char *mpi3d_strerror(int status)
{
    switch (status) {
    case MPI3D_OK: return "ok";
    case MPI3D_EINVAL: return "invalid argument";
    case MPI3D_ENOMEM: return "out of device memory or workspace too small";
    case MPI3D_EDEVICE: return "HIP runtime error";
    case MPI3D_ENOTSUP: return "geometry not supported by the compiled kernels";
    case MPI3D_ENONFINITE: return "non-finite value in a solver norm";
    default: return "unknown status";
    }
}

extern "C" int mpi3d_plan_create(const mpi3d_geometry *g, int device, mpi3d_plan **out)
{
    if (!g || !out) return MPI3D_EINVAL;
    *out = nullptr;
    if (g->nx < 2 || g->ny < 2 || g->nz < 1 || g->n_angles < 1 || g->n_t < 32) return MPI3D_EINVAL;
    if (g->nx > 4096 || g->ny > 4096 || g->nz > 65535 || g->n_angles > 4096 || g->n_t > (1 << 22)) return MPI3D_EINVAL;
    int nu = g->n_u ? g->n_u : g->nx;
    if (nu < 2 || nu > 256) return MPI3D_ENOTSUP;
    if (!(g->drive_cycles > 0) || !(g->psf_width > 0) || !(g->op_scale >= 0)) return MPI3D_EINVAL;
    if (!(g->drive_amp >= 0)) return MPI3D_EINVAL;
    if (!std::isfinite(g->raster_sweep)) return MPI3D_EINVAL;
    const int n_classes = (g->raster_sweep != 0.0 && g->nz >= 2) ? 2 : 1;
    if (g->harm_lo < 1 || g->harm_hi < g->harm_lo || g->half_band < 0) return MPI3D_EINVAL;
    int precisions = g->precisions ? g->precisions : (1 << MPI3D_FP32);
    if (precisions & ~((1 << MPI3D_FP32) | (1 << MPI3D_MIXED) | (1 << MPI3D_PRECOMPOSED))) return MPI3D_EINVAL;
    // tensor PSF line coupling: every precision, without a raster
    if (g->psf_rows < 0) return MPI3D_EINVAL;
    const int psf_rows = std::min(g->psf_rows, g->nz - 1);
    if (psf_rows > 0 && n_classes > 1) return MPI3D_ENOTSUP;
    // dual drive: z-drive lines across the z-rows, as many entries as the
    // x-drive lines hold (nz <= n_u); under the tensor PSF they couple across
    // the detector columns of their angle
    const int drive_axes = g->drive_axes == 2 ? 2 : 1;
    if (g->drive_axes < 0 || g->drive_axes > 2 || !(g->drive_amp_z >= 0)) return MPI3D_EINVAL;
    if (drive_axes == 2 && (g->nz > nu || n_classes > 1)) return MPI3D_ENOTSUP;
    const int psf_cols = drive_axes == 2 && g->psf_rows > 0 ? std::min(g->psf_rows, nu - 1) : 0;
    const int n_ktab = drive_axes == 2 ? (psf_rows + 1) + (psf_cols + 1) : n_classes * (psf_rows + 1);

    // kept bins, validated
    std::vector<long> bins;
    for (int k = g->harm_lo; k <= g->harm_hi; ++k) {
        long c = (long)std::floor(k * g->drive_cycles + 0.5);
        for (int d = -g->half_band; d <= g->half_band; ++d) bins.push_back(c + d);
    }
    for (size_t i = 0; i < bins.size(); ++i) {
        if (bins[i] <= 0 || bins[i] >= g->n_t / 2) return MPI3D_EINVAL;
        if (i && bins[i] <= bins[i - 1]) return MPI3D_EINVAL;  // increasing => distinct
    }
    if (bins.size() > 2048) return MPI3D_ENOTSUP;

    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return MPI3D_EINVAL;

    mpi3d_plan *pl = new (std::nothrow) mpi3d_plan();
    if (!pl) return MPI3D_ENOMEM;
    pl->device = device;
    pl->nx = g->nx; pl->ny = g->ny; pl->nz = g->nz; pl->M = g->n_angles;
    pl->nu = nu; pl->nt = g->n_t; pl->nr = ray_count(g->nx, g->ny);
    pl->nb = (int)bins.size();
    pl->harm_lo = g->harm_lo; pl->harm_hi = g->harm_hi; pl->half_band = g->half_band;
    pl->P = g->drive_cycles;
    pl->a = g->drive_amp > 0 ? g->drive_amp : nu / 2.0;
    pl->w = g->psf_width;
    pl->op_scale = g->op_scale;
    pl->precisions = precisions;
    pl->n_classes = n_classes;
    pl->psf_rows = psf_rows;
    pl->n_ktab = n_ktab;
    pl->pass_r = std::max(psf_rows, psf_cols);
    pl->n_passes = pl->pass_r + 1;
    pl->raster_sweep = g->raster_sweep;
    pl->nup = round_up(nu, 64);
    pl->ntp = round_up(g->n_t, kChunk);
    pl->nb2 = 2 * pl->nb;
    pl->nbp2 = round_up(pl->nb2, kColTile);
    pl->nct = pl->nbp2 / kColTile;
    pl->drive_axes = drive_axes;
    pl->a_z = g->drive_amp_z > 0 ? g->drive_amp_z : g->nz / 2.0;
    pl->Lx = (long)pl->M * pl->nz;
    pl->Lz = drive_axes == 2 ? (long)pl->M * nu : 0;
    pl->L = pl->Lx + pl->Lz;
    // line groups of a signal stage (each with its own PSF tables)
    if (n_classes > 1) {
        pl->n_line_groups = n_classes;
        for (int c = 0; c < n_classes; ++c) {
            const int per = (pl->nz - c + n_classes - 1) / n_classes;
            pl->groups[c] = {pl->M * per, per, pl->nz, c, n_classes, c, 0, pl->nz, 0};
        }
    } else if (drive_axes == 2) {
        pl->n_line_groups = 2;
        pl->groups[0] = {(int)pl->Lx, (int)pl->Lx, 0, 0, 1, 0, psf_rows, pl->nz, 0};
        pl->groups[1] = {(int)pl->Lz, (int)pl->Lz, 0, (int)pl->Lx, 1, psf_rows + 1, psf_cols, nu, pl->Lx};
    } else {
        pl->n_line_groups = 1;
        pl->groups[0] = {(int)pl->L, (int)std::max<long>(1, pl->L), 0, 0, 1, 0, psf_rows, pl->nz, 0};
    }
    pl->nvox = (long)pl->nx * pl->ny * pl->nz;
    pl->nchunks = pl->ntp / kChunk;

    // Column groups and time splits per precision; the band tables hold the
    // larger of the two paddings.
    {
        const int nct0 = pl->nct;
        column_groups(nct0, true, pl->sc[0]);
        column_groups(nct0, false, pl->sc[1]);
        pl->nct = pl->sc[0].ngroups * pl->sc[0].gct;
        if (precisions & (1 << MPI3D_MIXED)) pl->nct = std::max(pl->nct, pl->sc[1].ngroups * pl->sc[1].gct);
        // FP32 tensor PSF in one fused pass, where a kernel fits: every line
        // group coupled over the same R, a virtual line of a compiled width,
        // the band table in one wide group of 14 or 16 column tiles
        bool same_r = pl->pass_r > 0;
        for (int gi = 0; gi < pl->n_line_groups; ++gi) same_r = same_r && pl->groups[gi].coup == pl->pass_r;
        const int nupf = (pl->pass_r + 1) * pl->nup, gctf = 2 * std::max(7, (nct0 + 1) / 2);
        if (same_r && nct0 <= 16 && sig_fused_supported(nupf, gctf)) {
            pl->fused = true;
            pl->nupf = nupf;
            pl->scf = mpi3d_plan::SigCfg{kWidePairs, 1, gctf, 0, 0, 0, 0, 0, 0};
            pl->nct = std::max(pl->nct, gctf);
        }
        pl->nbp2 = pl->nct * kColTile;
    }
    {
        const mpi3d_plan::SigCfg &c0 = pl->sc[0], &c1 = pl->sc[1];
        if (!sig_fwd_supported(pl->nup, c0.gct, MPI3D_FP32, c0.pairs) ||
            !sig_adj_supported(pl->nup, c0.gct, MPI3D_FP32, c0.pairs) ||
            ((precisions & (1 << MPI3D_MIXED)) && (!sig_fwd_supported(pl->nup, c1.gct, MPI3D_MIXED, c1.pairs) ||
                                                   !sig_adj_supported(pl->nup, c1.gct, MPI3D_MIXED, c1.pairs)))) {
            delete pl;
            return MPI3D_ENOTSUP;
        }
    }
    choose_split(pl, true, pl->sc[0], pl->nup, pl->n_passes);
    choose_split(pl, false, pl->sc[1], pl->nup, pl->n_passes);
    if (pl->fused) choose_split(pl, true, pl->scf, pl->nupf, 1);

    // projection configuration
    {
        // Forward: a staged texel holds one or two slices (4 bytes: one fp32
        // slice or two bf16 slices; 8 bytes: two fp32 slices); a slice group
        // too large for 160 KB of LDS is staged in row bands (LDS rows =
        // band_rows + 1).  The fp32 path takes slice pairs only when a pair
        // fits in one band, since a band edge splits a wave's rays unevenly.
        // The ceil(nz / slices) * M (slice group, angle) units are split into
        // equal contiguous ranges, one per block (a block holds kFwdThreads *
        // fwd_rays_per_thread rays, nu per unit), in whole rounds of 256
        // blocks.
        auto fwd_config = [&](int slices, int texel_bytes, mpi3d::FwdConfig &fc) {
            const size_t lds = 160 * 1024;
            const int bases = pl->ny + 1;           // base rows -1 .. ny-1
            const int max_rows = (int)(lds / ((size_t)mpi3d::proj_pitch(pl->nx) * texel_bytes)) - 1;
            if (max_rows < 2) return false;
            fc.slices = slices;
            fc.n_bands = (bases + max_rows - 1) / max_rows;
            fc.band_rows = (bases + fc.n_bands - 1) / fc.n_bands;
            const long units = (long)((pl->nz + slices - 1) / slices) * pl->M;
            const long umax = std::max<long>(1, kFwdThreads * fwd_rays_per_thread(slices) / pl->nu);
            long nb = (units + umax - 1) / umax;
            nb = ((nb + 255) / 256) * 256;
            fc.blocks = (int)std::min(nb, units);
            return true;
        };
        if (!fwd_config(2, 8, pl->fwd32) || pl->fwd32.n_bands > 1) {
            if (!fwd_config(1, 4, pl->fwd32)) { delete pl; return MPI3D_ENOTSUP; }
        }
        if (!fwd_config(2, 4, pl->fwd16)) { delete pl; return MPI3D_ENOTSUP; }
        // Backprojection: 16 x 16 voxel tiles times kz slices per block.  The
        // ray weights are formed once per voxel and angle and reused over kz
        // slices, so take the largest kz that still gives about three blocks
        // per CU; angles are staged in LDS in chunks of at most 40 KB.
        const long tiles = (long)((pl->nx + 15) / 16) * ((pl->ny + 15) / 16);
        pl->kz = 8;
        for (int kz : {32, 16}) {
            if (tiles * ((pl->nz + kz - 1) / kz) >= 768) {
                pl->kz = kz;
                break;
            }
        }
        const int chunk_max = std::max(1, (40 * 1024) / (pl->kz * 32 * (int)sizeof(float)));
        const int nchunk = (pl->M + chunk_max - 1) / chunk_max;
        pl->adj_chunk = (pl->M + nchunk - 1) / nchunk;
        const long adj_blocks = tiles * ((pl->nz + pl->kz - 1) / pl->kz);
        pl->max_parts = (int)std::max<long>(kMaxNormParts, adj_blocks);
    }

    // ---- float64 host tables ------------------------------------------------
    const int M = pl->M, NU = pl->nu, NUP = pl->nup, T = pl->nt, TP = pl->ntp, NB = pl->nb;
    const int NBP2 = pl->nbp2, NCT = pl->nct, NC = pl->nchunks;
    std::vector<double> theta(M);
    for (int m = 0; m < M; ++m) theta[m] = g->theta_rad ? g->theta_rad[m] : m * kPi / M;
    for (int m = 0; m < M; ++m)
        if (!std::isfinite(theta[m])) { delete pl; return MPI3D_EINVAL; }
    const double cx = 0.5 * (pl->nx - 1), cy = 0.5 * (pl->ny - 1), cu = 0.5 * (NU - 1);

    std::vector<float2> cs(M);
    std::vector<float> ax((size_t)M * NU), ay((size_t)M * NU);
    for (int m = 0; m < M; ++m) {
        double c = std::cos(theta[m]), s = std::sin(theta[m]);
        cs[m] = make_float2((float)c, (float)s);
        for (int p = 0; p < NU; ++p) {
            double up = p - cu;
            // sample (p, q) sits at x = u_p c + y_q s, y = -u_p s + y_q c; the
            // kernels add y_q times (s, c) to these bases (LDS column 0 holds
            // grid column -1, hence the +1).
            ax[(size_t)m * NU + p] = (float)(up * c + cx + 1.0);
            ay[(size_t)m * NU + p] = (float)(-up * s + cy);
        }
    }

    // PSF kernel K[n][p] of every table (n < T, p < NU; zero padding
    // elsewhere).  Line group g's tables are table_g + d, d = 0..coup_g: for
    // trajectory class c (class 1 being the raster's backward sweep,
    // xi_n = a sin(phi_n) + dir S (n/T - 1/2), v_n = a phi' cos(phi_n) + dir S/T)
    // and line offset d of the tensor PSF, d = 0 being the collinear
    // L'(du/w)/w.  The z-drive group's tables use amplitude a_z and the
    // centred z-rows as samples (zero beyond nz); its offsets are detector
    // columns, the tensor entry's transverse offset.
    const size_t KE = (size_t)TP * NUP;
    pl->k_elems = KE;
    std::vector<double> K(KE * n_ktab, 0.0);
    {
        const double om = 2.0 * kPi * pl->P / T;
        for (int tb = 0; tb < n_ktab; ++tb) {
            const bool zt = drive_axes == 2 && tb > psf_rows;
            const int cl = zt ? 0 : tb / (psf_rows + 1);
            const int d = zt ? tb - (psf_rows + 1) : tb % (psf_rows + 1);
            const double dir = cl == 0 ? 1.0 : -1.0, S = pl->raster_sweep;
            const double amp = zt ? pl->a_z : pl->a, centre = zt ? 0.5 * (pl->nz - 1) : cu;
            const int npts = zt ? pl->nz : NU;
            double *Kc = &K[KE * tb];
            for (int n = 0; n < T; ++n) {
                double ph = om * n;
                double xi = amp * std::sin(ph) + dir * S * ((double)n / T - 0.5);
                double v = amp * om * std::cos(ph) + dir * S / T;
                for (int p = 0; p < npts; ++p) {
                    const double du = xi - (p - centre);
                    Kc[(size_t)n * NUP + p] =
                        v * (d == 0 ? langevin_deriv(du / pl->w) / pl->w : psf_xx(du, (double)d, pl->w));
                }
            }
        }
    }
    // band DFT F[n][c] (real columns: 2j = Re, 2j+1 = Im)
    std::vector<double> F((size_t)TP * NBP2, 0.0);
    {
        const double inv = 1.0 / std::sqrt((double)T);
        for (int j = 0; j < NB; ++j) {
            double dre = 1.0, dim = 0.0;
            if (g->rx_filter) { dre = g->rx_filter[2 * j]; dim = g->rx_filter[2 * j + 1]; }
            if (!std::isfinite(dre) || !std::isfinite(dim)) { delete pl; return MPI3D_EINVAL; }
            for (int n = 0; n < T; ++n) {
                long ph = (long)(((unsigned long long)bins[j] * (unsigned long long)n) % (unsigned long long)T);
                double a = 2.0 * kPi * (double)ph / T;
                double c = std::cos(a), s = std::sin(a);
                F[(size_t)n * NBP2 + 2 * j] = (dre * c - dim * s) * inv;
                F[(size_t)n * NBP2 + 2 * j + 1] = (dre * s + dim * c) * inv;
            }
        }
    }

    // precomposed line matrices Gt[p][c] = sum_n K[n][p] F[n][c] (the whole
    // A_DC of one line, c_A aside), one per PSF table, float64 accumulation
    const bool precomp = precisions & (1 << MPI3D_PRECOMPOSED);
    std::vector<float> gt;
    pl->gt_elems = (size_t)NUP * 2 * NB;
    if (precomp) {
        const int NB2 = 2 * NB;
        gt.resize(pl->gt_elems * n_ktab);
        std::vector<double> acc(pl->gt_elems);
        for (int tb = 0; tb < n_ktab; ++tb) {
            std::fill(acc.begin(), acc.end(), 0.0);
            const double *Kc = &K[KE * tb];
            for (int n = 0; n < T; ++n) {
                const double *fr = &F[(size_t)n * NBP2];
                for (int p = 0; p < NU; ++p) {
                    const double k = Kc[(size_t)n * NUP + p];
                    double *row = &acc[(size_t)p * NB2];
                    for (int c = 0; c < NB2; ++c) row[c] += k * fr[c];
                }
            }
            for (size_t i = 0; i < acc.size(); ++i) gt[pl->gt_elems * tb + i] = (float)acc[i];
        }
    }

    // ---- band DFT factored over drive cycles (FP32) --------------------------
    // t = n1 + P n2 (T = C P, C = 32 or 64): the kept bin omega_j
    // contributes e^{2 pi i omega_j n1 / T} e^{2 pi i (omega_j mod C) n2 / C},
    // so the forward first sums each phase n1's C cycles against the R distinct
    // residues (omega_j mod C), then each bin's P phases.  Taken when its MFMA
    // work per line, T (n_up + 32 rct) + 64 P U, is under 3/4 of the dense
    // T (n_up + nbp2); C minimises it.
    std::vector<float> fkf, fka, fef, fea, fwf, fwa;
    std::vector<int> fuq, fubin, fqbin, fqsteps;
    if ((precisions & (1 << MPI3D_FP32)) && !pl->fused && pl->n_passes == 1 && pl->n_line_groups == 1 &&
        n_ktab == 1 && T % 32 == 0) {
        double best = 0.75 * (double)T * (NUP + NBP2);
        int bestC = 0;
        for (int C = 32; C <= T && C <= 64; C += 32) {
            if (T % C) continue;
            std::vector<int> cnt(C, 0);
            for (int j = 0; j < NB; ++j) ++cnt[bins[j] % C];
            int R = 0, U = 0, mx = 0;
            for (int r = 0; r < C; ++r)
                if (cnt[r]) {
                    ++R;
                    U += (cnt[r] + 15) / 16;
                    mx = std::max(mx, cnt[r]);
                }
            const int zst = (R + 3) / 4 * 4, rct = (2 * zst + 31) / 32;
            const int P = T / C;
            if (R > 24 || mx > kQMax || U > 40 * kMaxFacSplit || !fac_supported(NUP, rct, zst, C / 32) ||
                (double)((pl->L + 31) / 32 * 32 + 1) * P * 2 * zst >= 2147483647.0)
                continue;
            const double cost = (double)T * (NUP + 32 * rct) + 64.0 * (P + 7) / 8 * 8 * U;
            if (cost < best) {
                best = cost;
                bestC = C;
            }
        }
        if (bestC) {
            mpi3d_plan::Fac &f = pl->fac;
            f.on = true;
            f.C = bestC;
            f.P = T / bestC;
            f.Pp = (f.P + 7) / 8 * 8;
            f.cj = bestC / 32;
            f.nzstage = (f.P + 15) / 16;
            // Residue order: the adjoint outer sum's wave w takes residues
            // w, w + 8, w + 16 (so waves w < R % 8 take one more when 8 does
            // not divide R) and spends a step per bin, so residues are dealt
            // largest first to the least loaded wave with room, and numbered
            // by (wave, turn).  Units: a residue's bins (ascending) 16 at a time.
            std::vector<int> cnt(bestC, 0), byc;
            for (int j = 0; j < NB; ++j) ++cnt[bins[j] % bestC];
            for (int r = 0; r < bestC; ++r)
                if (cnt[r]) byc.push_back(r);
            std::stable_sort(byc.begin(), byc.end(), [&](int x, int y) { return cnt[x] > cnt[y]; });
            const int nw = kFacInWaves, nr = (int)byc.size();
            std::vector<std::vector<int>> wres(nw);
            std::vector<int> load(nw, 0), room(nw);
            for (int w = 0; w < nw; ++w) room[w] = nr / nw + (w < nr % nw ? 1 : 0);
            for (int r : byc) {
                int best = -1;
                for (int w = 0; w < nw; ++w)
                    if ((int)wres[w].size() < room[w] && (best < 0 || load[w] < load[best])) best = w;
                wres[best].push_back(r);
                load[best] += (cnt[r] + 3) / 4 * 4;
            }
            std::vector<int> slot(bestC, -1), res(byc.size(), -1);
            for (int w = 0; w < nw; ++w)
                for (size_t i = 0; i < wres[w].size(); ++i) {
                    const int q = w + nw * (int)i;
                    res[q] = wres[w][i];
                    slot[wres[w][i]] = q;
                }
            f.R = (int)res.size();
            f.zst = (f.R + 3) / 4 * 4;
            f.rct = (2 * f.zst + 31) / 32;
            std::vector<std::vector<int>> qb(f.R);
            for (int j = 0; j < NB; ++j) qb[slot[bins[j] % bestC]].push_back(j);
            fqbin.assign((size_t)f.R * kQMax, -1);
            fqsteps.assign(f.R, 0);
            for (int q = 0; q < f.R; ++q) {
                for (size_t i = 0; i < qb[q].size(); ++i) fqbin[(size_t)q * kQMax + i] = qb[q][i];
                fqsteps[q] = ((int)qb[q].size() + 3) / 4 * 4;
                for (size_t i0 = 0; i0 < qb[q].size(); i0 += 16) {
                    fuq.push_back(q);
                    for (size_t i = 0; i < 16; ++i) fubin.push_back(i0 + i < qb[q].size() ? qb[q][i0 + i] : -1);
                }
            }
            f.U = (int)fuq.size();
            f.usplit = (f.U + 39) / 40;
            // the outer sums' blocks: one per line tile (and unit split); small
            // scans also split the phase stages so about 256 blocks run
            const long tiles = (pl->L + 31) / 32;
            f.psplit = (int)std::max<long>(1, std::min<long>({4, 256 / (tiles * f.usplit), (f.P + 7) / 8}));
            f.zsplit = (int)std::max<long>(1, std::min<long>({4, 256 / tiles, (f.P + 15) / 16}));
            // phase ranges of the line-tile kernels (8 tiles a block, one block a
            // CU): the fewest splits within 2% of the best time, counted as
            // rounds of 256 blocks times the phases of the longest range
            auto splits = [&](int waves) {
                const long tgroups = ((pl->L + 31) / 32 + waves - 1) / waves;
                auto per_phase = [&](int ns) {
                    return (double)((tgroups * ns + 255) / 256) * (double)((f.P + ns - 1) / ns) / f.P;
                };
                double pbest = 1e30;
                for (int ns = 1; ns <= std::min(f.P, 64); ++ns) pbest = std::min(pbest, per_phase(ns));
                int ns = 1;
                while (ns < std::min(f.P, 64) && per_phase(ns) > 1.02 * pbest) ++ns;
                return ns;
            };
            f.nsplit = splits(kFacWavesFwd);
            f.nsplit_adj = splits(kFacWavesAdj);
            // tables
            const int C = bestC, P = f.P, CJ = f.cj, ZST = f.zst, RCT = f.rct, YC = 2 * ZST;
            auto tperm = [](int s2, int h) { return 8 * (s2 / 4) + 4 * h + (s2 % 4); };
            auto tof = [&](int c, int i) { return (c / CJ) + P * (32 * (c % CJ) + i); };   // chunk row -> time
            const double *K0 = &K[0];
            fkf.assign(KE, 0.f);
            fka.assign(KE, 0.f);
            for (int c = 0; c < P * CJ; ++c) {
                for (int st = 0; st < NUP / 2; ++st)
                    for (int l = 0; l < 64; ++l)
                        fkf[(((size_t)c * (NUP / 8) + st / 4) * 64 + l) * 4 + st % 4] =
                            (float)K0[(size_t)tof(c, l % 32) * NUP + 2 * st + l / 32];
                for (int pt = 0; pt < NUP / 32; ++pt)
                    for (int s2 = 0; s2 < 16; ++s2)
                        for (int l = 0; l < 64; ++l)
                            fka[((((size_t)c * (NUP / 32) + pt) * 4 + s2 / 4) * 64 + l) * 4 + s2 % 4] =
                                (float)K0[(size_t)tof(c, tperm(s2, l / 32)) * NUP + 32 * pt + l % 32];
            }
            // E[n2][2q] = cos, E[n2][2q + 1] = sin of 2 pi (r_q n2 mod C) / C
            auto E = [&](int n2, int col) -> double {
                if (col >= 2 * f.R) return 0.0;
                const long ph = (long)res[col / 2] * n2 % C;
                const double a = 2.0 * kPi * (double)ph / C;
                return col % 2 ? std::sin(a) : std::cos(a);
            };
            fef.assign((size_t)C * 32 * RCT, 0.f);
            for (int j = 0; j < CJ; ++j)
                for (int g2 = 0; g2 < RCT; ++g2)
                    for (int s2 = 0; s2 < 16; ++s2)
                        for (int l = 0; l < 64; ++l)
                            fef[((((size_t)j * RCT + g2) * 4 + s2 / 4) * 64 + l) * 4 + s2 % 4] =
                                (float)E(32 * j + tperm(s2, l / 32), 32 * g2 + l % 32);
            fea.assign((size_t)C * YC, 0.f);
            for (int j = 0; j < CJ; ++j)
                for (int st = 0; st < ZST; ++st)
                    for (int l = 0; l < 64; ++l)
                        fea[(((size_t)j * (ZST / 4) + st / 4) * 64 + l) * 4 + st % 4] =
                            (float)E(32 * j + l % 32, 2 * st + l / 32);
            // G_j[n1] = D_j e^{2 pi i (omega_j n1 mod T) / T} / sqrt(T)
            const double inv = 1.0 / std::sqrt((double)T);
            auto G = [&](int j, int n1, double &gr, double &gi) {
                double dre = 1.0, dim = 0.0;
                if (g->rx_filter) { dre = g->rx_filter[2 * j]; dim = g->rx_filter[2 * j + 1]; }
                const long ph = (long)(((unsigned long long)bins[j] * (unsigned long long)n1) % (unsigned long long)T);
                const double a = 2.0 * kPi * (double)ph / T;
                gr = (dre * std::cos(a) - dim * std::sin(a)) * inv;
                gi = (dre * std::sin(a) + dim * std::cos(a)) * inv;
            };
            // forward outer B operand: k = (n1 = st, re/im of Y = l / 32), column
            // l % 32 = (bin slot, re/im of b)
            fwf.assign((size_t)f.U * f.Pp * 64, 0.f);
            for (int u = 0; u < f.U; ++u)
                for (int st = 0; st < P; ++st)
                    for (int l = 0; l < 64; ++l) {
                        const int col = l % 32, jb = fubin[(size_t)u * 16 + col / 2];
                        if (jb < 0) continue;
                        double gr, gi;
                        G(jb, st, gr, gi);
                        const int cy = l / 32, cb = col % 2;
                        const double v = cb == 0 ? (cy == 0 ? gr : -gi) : (cy == 0 ? gi : gr);
                        fwf[(((size_t)u * (f.Pp / 4) + st / 4) * 64 + l) * 4 + st % 4] = (float)v;
                    }
            // adjoint outer B operand: k = (bin slot st, re/im of the data =
            // l / 32), column l % 32 = (phase stg 16 + col / 2, re/im of Z)
            fwa.assign((size_t)f.R * f.nzstage * kQMax * 64, 0.f);
            for (int q = 0; q < f.R; ++q)
                for (int stg = 0; stg < f.nzstage; ++stg)
                    for (int st = 0; st < kQMax; ++st)
                        for (int l = 0; l < 64; ++l) {
                            const int jb = fqbin[(size_t)q * kQMax + st], col = l % 32, n1 = 16 * stg + col / 2;
                            if (jb < 0 || n1 >= P) continue;
                            double gr, gi;
                            G(jb, n1, gr, gi);
                            const int cd = l / 32, cz = col % 2;
                            const double v = cz == 0 ? (cd == 0 ? gr : gi) : (cd == 0 ? -gi : gr);
                            fwa[((((size_t)q * f.nzstage + stg) * (kQMax / 4) + st / 4) * 64 + l) * 4 + st % 4] =
                                (float)v;
                        }
        }
    }

    // ---- table layout in one device allocation -----------------------------
    bool mixed = precisions & (1 << MPI3D_MIXED);
    size_t off = 0;
    char *nullbase = nullptr;
    size_t o_cs, o_ax, o_ay, o_kf, o_ff, o_fa, o_ka, o_kf16 = 0, o_ff16 = 0, o_fa16 = 0, o_ka16 = 0, o_cols = 0, o_bands = 0;
    auto place = [&](size_t bytes) { off = align256(off); size_t o = off; off += bytes; return o; };
    o_cs = place(sizeof(float2) * M);
    o_ax = place(sizeof(float) * M * NU);
    o_ay = place(sizeof(float) * M * NU);
    o_kf = place(sizeof(float) * KE * n_ktab);
    o_ff = place(sizeof(float) * (size_t)TP * NBP2);
    o_fa = place(sizeof(float) * (size_t)TP * NBP2);
    o_ka = place(sizeof(float) * KE * n_ktab);
    const size_t KEF = KE * pl->n_passes * pl->n_line_groups;   // fused tables, all groups
    const size_t o_kff = pl->fused ? place(sizeof(float) * KEF) : 0;
    const size_t o_kaf = pl->fused ? place(sizeof(float) * KEF) : 0;
    const size_t o_gt = precomp ? place(sizeof(float) * gt.size()) : 0;
    const size_t o_gta = precomp ? place(sizeof(float) * gt.size()) : 0;
    const bool fac = pl->fac.on;
    const size_t o_fkf = fac ? place(sizeof(float) * fkf.size()) : 0;
    const size_t o_fka = fac ? place(sizeof(float) * fka.size()) : 0;
    const size_t o_fef = fac ? place(sizeof(float) * fef.size()) : 0;
    const size_t o_fea = fac ? place(sizeof(float) * fea.size()) : 0;
    const size_t o_fwf = fac ? place(sizeof(float) * fwf.size()) : 0;
    const size_t o_fwa = fac ? place(sizeof(float) * fwa.size()) : 0;
    const size_t o_fuq = fac ? place(sizeof(int) * fuq.size()) : 0;
    const size_t o_fubin = fac ? place(sizeof(int) * fubin.size()) : 0;
    const size_t o_fqbin = fac ? place(sizeof(int) * fqbin.size()) : 0;
    const size_t o_fqsteps = fac ? place(sizeof(int) * fqsteps.size()) : 0;
    if (mixed) {
        o_kf16 = place(sizeof(__half) * KE * n_ktab);
        o_ff16 = place(sizeof(__half) * (size_t)TP * NBP2);
        o_fa16 = place(sizeof(__half) * (size_t)TP * NBP2);
        o_ka16 = place(sizeof(__half) * KE * n_ktab);
        o_cols = place(sizeof(float) * NBP2);
        o_bands = place(sizeof(float) * NBP2);
    }
    (void)nullbase;
    pl->table_bytes = align256(off);

    // Swizzled fp32 tables: every MFMA operand a lane needs for 4 consecutive
    // steps is one 16-byte load, and a wave's 64 loads are contiguous.
    //  kf: fwd GEMM1 A operand  K[t = 32c + l%32][p = 2st + l/32]    [c][st/4][l][st%4]
    //  ff: fwd GEMM2 B operand  F[t = 32c + tperm(s, l/32)][32ct + l%32]  [c][ct][s/4][l][s%4]
    //  fa: adj GEMM1 A operand  F[t = 32c + l%32][col = 2st + l/32]  [c][st/4][l][st%4]
    //  ka: adj GEMM2 B operand  K[t = 32c + tperm(s, l/32)][32pt + l%32]  [c][pt][s/4][l][s%4]
    // tperm(s, h) = 8(s/4) + 4h + s%4 is the time index that the 32x32 MFMA
    // result layout leaves in register s of lane half h.
    std::vector<float> kf(KE * n_ktab), ff((size_t)TP * NBP2), fa((size_t)TP * NBP2), ka(KE * n_ktab);
    auto tperm = [](int s, int h) { return 8 * (s / 4) + 4 * h + (s % 4); };
    for (int cl = 0; cl < n_ktab; ++cl)
        for (int c = 0; c < NC; ++c) {
            const double *Kc = &K[KE * cl];
            float *kfc = &kf[KE * cl], *kac = &ka[KE * cl];
            for (int st = 0; st < NUP / 2; ++st)
                for (int l = 0; l < 64; ++l)
                    kfc[(((size_t)c * (NUP / 8) + st / 4) * 64 + l) * 4 + st % 4] =
                        (float)Kc[(size_t)(32 * c + l % 32) * NUP + 2 * st + l / 32];
            for (int pt = 0; pt < NUP / 32; ++pt)
                for (int s = 0; s < 16; ++s)
                    for (int l = 0; l < 64; ++l)
                        kac[((((size_t)c * (NUP / 32) + pt) * 4 + s / 4) * 64 + l) * 4 + s % 4] =
                            (float)Kc[(size_t)(32 * c + tperm(s, l / 32)) * NUP + 32 * pt + l % 32];
        }
    for (int c = 0; c < NC; ++c) {
        for (int ct = 0; ct < NCT; ++ct)
            for (int s = 0; s < 16; ++s)
                for (int l = 0; l < 64; ++l)
                    ff[((((size_t)c * NCT + ct) * 4 + s / 4) * 64 + l) * 4 + s % 4] =
                        (float)F[(size_t)(32 * c + tperm(s, l / 32)) * NBP2 + 32 * ct + l % 32];
        for (int st = 0; st < NBP2 / 2; ++st)
            for (int l = 0; l < 64; ++l)
                fa[(((size_t)c * (NBP2 / 8) + st / 4) * 64 + l) * 4 + st % 4] =
                    (float)F[(size_t)(32 * c + l % 32) * NBP2 + 2 * st + l / 32];
    }

    // Mixed (fp16) tables with power-of-two scales.
    std::vector<_Float16> kf16, ff16, fa16, ka16;
    std::vector<float> col_scale, band_scale;
    if (mixed) {
        double kmax = 0, fmax = 0;
        for (double v : K) kmax = std::max(kmax, std::fabs(v));
        for (double v : F) fmax = std::max(fmax, std::fabs(v));
        int ek, ef;
        std::frexp(kmax > 0 ? kmax : 1.0, &ek);
        std::frexp(fmax > 0 ? fmax : 1.0, &ef);
        double ks = std::ldexp(1.0, -ek), fs = std::ldexp(1.0, -ef);  // scaled max in [0.5, 1)
        // Per-band adjoint scale: a band's share of the operator, measured as
        // its response to a unit source at each of a few detector positions.
        std::vector<double> bnorm(NB / (2 * pl->half_band + 1), 0.0);
        int nbands = (int)bnorm.size(), bw = 2 * pl->half_band + 1;
        for (int probe = 0; probe < 3 * n_ktab; ++probe) {
            const int p = (probe % 3 + 1) * NU / 4;
            const double *Kc = &K[KE * (probe / 3)];
            for (int j = 0; j < NB; ++j) {
                double re = 0, im = 0;
                for (int n = 0; n < T; ++n) {
                    double kv = Kc[(size_t)n * NUP + p];
                    re += kv * F[(size_t)n * NBP2 + 2 * j];
                    im += kv * F[(size_t)n * NBP2 + 2 * j + 1];
                }
                bnorm[j / bw] = std::max(bnorm[j / bw], std::sqrt(re * re + im * im));
            }
        }
        double bmax = *std::max_element(bnorm.begin(), bnorm.end());
        col_scale.assign(NBP2, (float)(1.0 / (ks * fs)));
        pl->adj_scale16 = (float)(1.0 / (ks * fs));
        band_scale.assign(NBP2, 1.0f);
        std::vector<double> fcol(NBP2, fs);
        for (int b = 0; b < nbands; ++b) {
            double rel = bnorm[b] > 0 && bmax > 0 ? bnorm[b] / bmax : 1.0;
            int e;
            std::frexp(rel, &e);                       // rel in [2^(e-1), 2^e)
            double bs = std::ldexp(1.0, std::min(-(e - 1), 14));  // lifts the band to [1, 2) x max
            for (int d = 0; d < bw; ++d)
                for (int h = 0; h < 2; ++h) {
                    int col = 2 * (b * bw + d) + h;
                    band_scale[col] = (float)bs;
                    fcol[col] = fs / bs;
                }
        }
        // fp16 layouts (8 halves per lane per MFMA step, 32x32x16):
        //  kf16: fwd GEMM1 A: K[t = 32c + l%32][p = 16st + 8(l/32) + e]          [c][st][l][e]
        //  ff16: fwd GEMM2 B: F[t = 32c + 16h + tperm16(e, l/32)][32ct + l%32]   [c][ct][h][l][e]
        //  fa16: adj GEMM1 A: F[t = 32c + l%32][col = 16st + 8(l/32) + e]        [c][st][l][e]
        //  ka16: adj GEMM2 B: K[t = 32c + 16h + tperm16(e, l/32)][32pt + l%32]   [c][pt][h][l][e]
        // tperm16(e, h) = 8(e/4) + 4h + e%4.
        auto tp16 = [](int e, int h) { return 8 * (e / 4) + 4 * h + (e % 4); };
        kf16.resize(KE * n_ktab);
        ff16.resize((size_t)TP * NBP2);
        fa16.resize((size_t)TP * NBP2);
        ka16.resize(KE * n_ktab);
        for (int cl = 0; cl < n_ktab; ++cl)
            for (int c = 0; c < NC; ++c) {
                const double *Kc = &K[KE * cl];
                _Float16 *kfc = &kf16[KE * cl], *kac = &ka16[KE * cl];
                for (int st = 0; st < NUP / 16; ++st)
                    for (int l = 0; l < 64; ++l)
                        for (int e2 = 0; e2 < 8; ++e2)
                            kfc[(((size_t)c * (NUP / 16) + st) * 64 + l) * 8 + e2] =
                                to_f16(Kc[(size_t)(32 * c + l % 32) * NUP + 16 * st + 8 * (l / 32) + e2] * ks);
                for (int pt = 0; pt < NUP / 32; ++pt)
                    for (int h = 0; h < 2; ++h)
                        for (int l = 0; l < 64; ++l)
                            for (int e2 = 0; e2 < 8; ++e2)
                                kac[((((size_t)c * (NUP / 32) + pt) * 2 + h) * 64 + l) * 8 + e2] = to_f16(
                                    Kc[(size_t)(32 * c + 16 * h + tp16(e2, l / 32)) * NUP + 32 * pt + l % 32] * ks);
            }
        for (int c = 0; c < NC; ++c) {
            for (int ct = 0; ct < NCT; ++ct)
                for (int h = 0; h < 2; ++h)
                    for (int l = 0; l < 64; ++l)
                        for (int e2 = 0; e2 < 8; ++e2)
                            ff16[((((size_t)c * NCT + ct) * 2 + h) * 64 + l) * 8 + e2] = to_f16(
                                F[(size_t)(32 * c + 16 * h + tp16(e2, l / 32)) * NBP2 + 32 * ct + l % 32] * fs);
            for (int st = 0; st < NBP2 / 16; ++st)
                for (int l = 0; l < 64; ++l)
                    for (int e2 = 0; e2 < 8; ++e2) {
                        int col = 16 * st + 8 * (l / 32) + e2;
                        fa16[(((size_t)c * (NBP2 / 16) + st) * 64 + l) * 8 + e2] =
                            to_f16(F[(size_t)(32 * c + l % 32) * NBP2 + col] * fcol[col]);
                    }
        }
        // undo factors applied to the adjoint: result = acc / (fs * ks * row_scale)
        (void)ef;
    }

    // ---- upload ------------------------------------------------------------
    e = hipMalloc(&pl->tables, pl->table_bytes);
    if (e != hipSuccess) { delete pl; return MPI3D_ENOMEM; }
    char *tb = (char *)pl->tables;
    pl->cs = (float2 *)(tb + o_cs);
    pl->ax = (float *)(tb + o_ax);
    pl->ay = (float *)(tb + o_ay);
    pl->kf = (float *)(tb + o_kf);
    pl->ff = (float *)(tb + o_ff);
    pl->fa = (float *)(tb + o_fa);
    pl->ka = (float *)(tb + o_ka);
    bool ok = hipMemcpy(pl->cs, cs.data(), sizeof(float2) * M, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(pl->ax, ax.data(), sizeof(float) * ax.size(), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(pl->ay, ay.data(), sizeof(float) * ay.size(), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(pl->kf, kf.data(), sizeof(float) * kf.size(), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(pl->ff, ff.data(), sizeof(float) * ff.size(), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(pl->fa, fa.data(), sizeof(float) * fa.size(), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(pl->ka, ka.data(), sizeof(float) * ka.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (pl->fused) {
        // group g's tables table_g .. table_g + R side by side per time chunk:
        // a chunk of kf / ka holds NUP x 32 floats for detector samples (kf:
        // 8 per float4 step, ka: 32 per column tile) in the order the kernels
        // walk them, so concatenating the chunks of consecutive offsets is the
        // layout of one table of NUP (R + 1) samples
        std::vector<float> kff(KEF), kaf(KEF);
        const size_t CB = (size_t)NUP * 32;   // floats per chunk of one table
        const int NP = pl->n_passes;
        for (int gi = 0; gi < pl->n_line_groups; ++gi)
            for (int c = 0; c < NC; ++c)
                for (int e2 = 0; e2 < NP; ++e2) {
                    const size_t src = (size_t)(pl->groups[gi].table + e2) * KE + c * CB;
                    const size_t dst = ((size_t)gi * NP * NC + (size_t)c * NP + e2) * CB;
                    std::copy(&kf[src], &kf[src] + CB, &kff[dst]);
                    std::copy(&ka[src], &ka[src] + CB, &kaf[dst]);
                }
        pl->kff = (float *)(tb + o_kff);
        pl->kaf = (float *)(tb + o_kaf);
        ok = ok && hipMemcpy(pl->kff, kff.data(), sizeof(float) * KEF, hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(pl->kaf, kaf.data(), sizeof(float) * KEF, hipMemcpyHostToDevice) == hipSuccess;
    }
    if (fac) {
        mpi3d_plan::Fac &f = pl->fac;
        auto up = [&](auto *&dst, size_t o, const auto &v) {
            dst = reinterpret_cast<std::remove_reference_t<decltype(dst)>>(tb + o);
            ok = ok && hipMemcpy(dst, v.data(), sizeof(v[0]) * v.size(), hipMemcpyHostToDevice) == hipSuccess;
        };
        up(f.kf, o_fkf, fkf);
        up(f.ka, o_fka, fka);
        up(f.ef, o_fef, fef);
        up(f.ea, o_fea, fea);
        up(f.wf, o_fwf, fwf);
        up(f.wa, o_fwa, fwa);
        up(f.uq, o_fuq, fuq);
        up(f.ubin, o_fubin, fubin);
        up(f.qbin, o_fqbin, fqbin);
        up(f.qsteps, o_fqsteps, fqsteps);
    }
    if (precomp) {
        pl->gt = (float *)(tb + o_gt);
        pl->gta = (float *)(tb + o_gta);
        // G = (G^T)^T per table, [2nb][n_up]: the adjoint GEMM's operand rows
        std::vector<float> gta(gt.size());
        const size_t NB2 = 2 * (size_t)NB;
        for (int tb2 = 0; tb2 < n_ktab; ++tb2)
            for (size_t p = 0; p < (size_t)NUP; ++p)
                for (size_t c = 0; c < NB2; ++c)
                    gta[pl->gt_elems * tb2 + c * NUP + p] = gt[pl->gt_elems * tb2 + p * NB2 + c];
        ok = ok && hipMemcpy(pl->gt, gt.data(), sizeof(float) * gt.size(), hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(pl->gta, gta.data(), sizeof(float) * gta.size(), hipMemcpyHostToDevice) == hipSuccess;
    }
    if (mixed) {
        pl->kf16 = (__half *)(tb + o_kf16);
        pl->ff16 = (__half *)(tb + o_ff16);
        pl->fa16 = (__half *)(tb + o_fa16);
        pl->ka16 = (__half *)(tb + o_ka16);
        pl->col_scale = (float *)(tb + o_cols);
        pl->band_scale = (float *)(tb + o_bands);
        ok = ok && hipMemcpy(pl->kf16, kf16.data(), sizeof(_Float16) * kf16.size(), hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(pl->ff16, ff16.data(), sizeof(_Float16) * ff16.size(), hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(pl->fa16, fa16.data(), sizeof(_Float16) * fa16.size(), hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(pl->ka16, ka16.data(), sizeof(_Float16) * ka16.size(), hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(pl->col_scale, col_scale.data(), sizeof(float) * NBP2, hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(pl->band_scale, band_scale.data(), sizeof(float) * NBP2, hipMemcpyHostToDevice) == hipSuccess;
    }
    if (!ok) {
        (void)hipFree(pl->tables);
        delete pl;
        return MPI3D_EDEVICE;
    }

    // ---- workspace layouts -------------------------------------------------
    {
        size_t o = 0;
        auto put = [&](size_t bytes) { o = align256(o); size_t r = o; o += bytes; return r; };
        pl->ws_rt = put(sizeof(float) * pl->L * pl->nup);
        size_t parts = 0;   // split partial sums: forward [splits][L][nbp2], adjoint [splits][groups][L][nup]
        for (const mpi3d_plan::SigCfg &c : pl->sc)
            parts = std::max(parts, (size_t)std::max(c.nsplit, c.serve_nsplit) *
                                        std::max<size_t>(pl->nbp2, (size_t)c.ngroups * pl->nup));
        size_t part_floats = (size_t)pl->n_passes * pl->L * parts;
        if (pl->fused)   // one pass; adjoint lines of nupf
            part_floats = std::max(part_floats, (size_t)pl->L * std::max(pl->scf.nsplit, pl->scf.serve_nsplit) *
                                                    std::max<size_t>(pl->nbp2, (size_t)pl->nupf));
        if (pl->fac.on)   // adjoint: nsplit blocks of nup-column lines; forward: psplit of nbp2 columns
            part_floats = std::max(part_floats, (size_t)std::max(pl->fac.nsplit_adj, pl->fac.psplit) * pl->L *
                                                    std::max(pl->nup, pl->nbp2));
        pl->ws_part = put(sizeof(float) * part_floats);
        pl->ws_norm = put(sizeof(double) * pl->max_parts);
        // per tensor-PSF pass: the forward's symmetric line sums, their
        // scales and fp16 operands (one block each without coupling)
        const size_t np = pl->n_passes;
        pl->ws_rowscale = put(sizeof(float) * np * pl->L);
        pl->ws_xb = put(mixed ? sizeof(uint16_t) * pl->nvox : 0);
        pl->in16_cols = std::max(pl->nup, pl->nbp2);
        pl->ws_in16 = put(mixed ? sizeof(uint16_t) * np * pl->L * pl->in16_cols : 0);
        pl->ws_rtb = put(mixed ? sizeof(uint16_t) * pl->L * pl->nup : 0);
        pl->ws_rtsc = put(mixed ? sizeof(float) * pl->L : 0);
        pl->ws_sig = put(np > 1 ? sizeof(float) * np * pl->L * pl->nup : 0);
        pl->ws_fac = put(pl->fac.on ? sizeof(float) * ((pl->L + 31) / 32 * 32 + 1) * pl->fac.P * 2 * pl->fac.zst : 0);
        pl->op_ws_bytes = align256(o);
    }
    {
        size_t o = 0;
        auto put = [&](size_t bytes) { o = align256(o); size_t r = o; o += bytes; return r; };
        long ndata = 2 * pl->L * pl->nb;
        pl->sw_op = put(pl->op_ws_bytes);
        pl->sw_r = put(sizeof(float) * ndata);
        pl->sw_q = put(sizeof(float) * ndata);
        pl->sw_s = put(sizeof(float) * pl->nvox);
        pl->sw_p = put(sizeof(float) * pl->nvox);
        pl->sw_scal = put(sizeof(double) * 64);
        pl->sw_parts = put(sizeof(double) * 3 * pl->max_parts);
        pl->sw_d = put(mixed ? sizeof(float) * pl->nvox : 0);   // refinement correction
        pl->sw_g = put(mixed ? sizeof(float) * pl->nvox : 0);   // FP32 gradient at the sweep start
        pl->sw_v = put(sizeof(float) * pl->nvox);                 // momentum solver: fourth volume
        pl->solve_ws_bytes = align256(o);
    }
    {
        // FNV-1a over the parameters that determine the line tables
        uint64_t h = 1469598103934665603ull;
        auto mix = [&](const void *p, size_t n) {
            const unsigned char *c = (const unsigned char *)p;
            for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
        };
        int ints[] = {pl->nu, pl->nup, pl->nt, pl->harm_lo, pl->harm_hi, pl->half_band, pl->nbp2,
                      pl->sc[0].pairs, pl->sc[0].ngroups, pl->sc[0].gct, pl->sc[1].pairs, pl->sc[1].ngroups,
                      pl->sc[1].gct, precisions, n_classes, psf_rows, drive_axes, drive_axes == 2 ? pl->nz : 0,
                      pl->fused ? pl->nupf : 0, pl->fused ? pl->scf.gct : 0, pl->fac.on ? pl->fac.C : 0};
        double dbl[] = {pl->P, pl->a, pl->w, pl->raster_sweep, drive_axes == 2 ? pl->a_z : 0.0};
        mix(ints, sizeof(ints));
        mix(dbl, sizeof(dbl));
        if (g->rx_filter) mix(g->rx_filter, sizeof(float) * 2 * pl->nb);
        pl->line_key = h;
    }
    // the no-allocation entry point's scratch address on this device (a
    // failure here is reported by that entry point itself)
    (void)scratch_setup(device);
    pl->norm_iters = 0;
    if (g->op_scale == 0.0) {
        // c_A = 1 / ||A||_2, estimated on the device
        double nrm = 0.0;
        int its = 0;
        const int rc = estimate_op_norm(pl, 1e-7, 1000, &nrm, &its);
        if (rc != MPI3D_OK) {
                (void)hipFree(pl->tables);
            delete pl;
            return rc;
        }
        pl->op_scale = 1.0 / nrm;
        pl->norm_iters = its;
    }
    *out = pl;
    return MPI3D_OK;
}

extern "C" void mpi3d_plan_destroy(mpi3d_plan *pl)
{
    if (!pl) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(pl->device);
    (void)hipFree(pl->tables);
    (void)hipSetDevice(prev);
    delete pl;
}

extern "C" int mpi3d_plan_query(const mpi3d_plan *pl, mpi3d_plan_info *info)
{
    if (!pl || !info) return MPI3D_EINVAL;
    info->n_vox = pl->nvox;
    info->n_lines = pl->L;
    info->n_bins = pl->nb;
    info->n_data_floats = 2 * pl->L * pl->nb;
    info->n_proj_floats = pl->Lx * pl->nu;
    info->op_ws_bytes = (int64_t)pl->op_ws_bytes;
    info->solve_ws_bytes = (int64_t)pl->solve_ws_bytes;
    info->table_bytes = (int64_t)pl->table_bytes;
    info->history_doubles = 4;
    info->n_r = pl->nr;
    info->norm_iters = pl->norm_iters;
    info->op_scale = pl->op_scale;
    info->dft_cycles = pl->fac.on ? pl->fac.C : 0;
    info->dft_residues = pl->fac.on ? pl->fac.R : 0;
    return MPI3D_OK;
}
