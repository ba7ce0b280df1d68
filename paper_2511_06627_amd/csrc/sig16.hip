// Mixed-precision (fp16 MFMA) signal kernels: not built yet.
#include "internal.h"

namespace mpi3d {

int sig16_supported(int, int) { return 0; }
hipError_t launch_sig_fwd16(const mpi3d_plan *, SigArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_sig_adj16(const mpi3d_plan *, SigArgs &, hipStream_t) { return hipErrorInvalidValue; }

}  // namespace mpi3d
