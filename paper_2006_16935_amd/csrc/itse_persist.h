// Host interface of the persistent batch kernel (itse_persist.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "itse_internal.h"

namespace itse {

// One group of equal (n, schedule) lattices of a batch, as the persistent kernel
// sees it: the (lattice, state) jobs, the lattices, the tiles of each pass.
struct PersistGroup {
    int n, variant, kmax;
    int gram;                 // the step runs the projection/Gram pass
    int njobs, nlats;
    int nb_plane, nb_cols, nb_gram;
    int nq_fin;               // finalisation sums a lattice of the group can need
    const JobRef *jobs, *lats;
};

constexpr int PERSIST_GROUPS = 8;

struct PersistPlan {
    int ngroups;
    PersistGroup g[PERSIST_GROUPS];
};

// (n, precision, schedule variant) the persistent kernel has tiles for.
bool persist_shape_ok(int n, int prec, int variant);
int persist_nb_plane(int n, int variant);
int persist_nb_cols(int n, int variant);
// Workgroups the GPU keeps resident for the kernel (the cooperative grid).
hipError_t persist_grid(int *blocks);
// One cooperative launch stepping every lattice of the plan (in device memory)
// nsteps times.
hipError_t persist_launch(const PersistPlan *plan_dev, int nsteps, int blocks, hipStream_t s);

}  // namespace itse
