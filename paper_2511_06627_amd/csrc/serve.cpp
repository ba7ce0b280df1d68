// Serving states: not built yet.
#include "internal.h"

extern "C" int mpi3d_state_create(const mpi3d_plan *, const float *, float *, const mpi3d_solve_opts *, void *, size_t,
                                  mpi3d_state **out)
{
    if (out) *out = nullptr;
    return MPI3D_ENOTSUP;
}
extern "C" int mpi3d_batch_step(mpi3d_state *const *, int32_t, void *) { return MPI3D_ENOTSUP; }
extern "C" int mpi3d_state_progress(const mpi3d_state *, int32_t *, int32_t *) { return MPI3D_ENOTSUP; }
extern "C" void mpi3d_state_destroy(mpi3d_state *) {}
