// mpi3d_forward_noalloc: the forward operator for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  Its operator workspace -- the projected
// lines, the signal kernels' split partial sums, the mixed path's bf16 volume,
// per-line scales and fp16 operand lines -- is a file-scope device array of
// fixed size instead of a caller buffer.  The kernels and their order are
// those of mpi3d_forward with a caller workspace, so the results are the same
// bit for bit.
//
// Host code never uses the array's name as an address: its device address on
// each GPU comes from hipGetSymbolAddress, taken once per device with that
// device current (at plan creation, or on the entry point's first call there)
// and kept in a per-device table.

#include <mutex>

#include "internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)MPI3D_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];   // device address of `scratch` on each device; null until set up

struct CurrentDevice {
    int prev = -1;
    explicit CurrentDevice(int dev)
    {
        (void)hipGetDevice(&prev);
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~CurrentDevice()
    {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

namespace mpi3d {

// With `device` current: record the device address of the scratch array.
int scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return MPI3D_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return MPI3D_OK;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MPI3D_EDEVICE;
    g_scratch_ptr[device] = p;
    return MPI3D_OK;
}

}  // namespace mpi3d

extern "C" int mpi3d_forward_noalloc(const mpi3d_plan *pl, int32_t precision, const float *x, float *b, void *stream)
{
    if (!pl || !x || !b) return MPI3D_EINVAL;
    const int rc = mpi3d::check_prec(pl, precision);
    if (rc) return rc;
    if (pl->op_ws_bytes > kScratchBytes) return MPI3D_ENOMEM;
    if (pl->device < 0 || pl->device >= kMaxDevices) return MPI3D_EINVAL;
    CurrentDevice cd(pl->device);
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        ws = g_scratch_ptr[pl->device];
    }
    if (!ws) {
        const int s = mpi3d::scratch_setup(pl->device);
        if (s) return s;
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        ws = g_scratch_ptr[pl->device];
    }
    return mpi3d::forward_ws(pl, precision, x, b, ws, (hipStream_t)stream);
}
