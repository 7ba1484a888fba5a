// Persistent batched stepping: every pass of every lattice of a batch, for a
// chunk of steps, in one cooperative launch.
//
// The grid holds as many workgroups as the GPU keeps resident.  For each step it
// takes the passes in order (forward plane pass, column pass, inverse plane pass,
// projection/Gram pass when a lattice needs it, finalisation sums, finalisation
// tail); within a pass each workgroup runs the tiles (lattice, state, sub-plane or
// column chunk) with index blockIdx.x, blockIdx.x + gridDim.x, ... of all the
// batch's lattices, and a grid-wide barrier separates the passes.  A tile is the
// same code with the same data mapping as in the pass's own kernel (the same
// schedule and state-count instance), so every lattice's results are bitwise
// those of its step alone.
//
// Scope: FP32 lattices of real states with the transform kinetic terms, N in
// {32, 48, 64, 96} under the schedules whose plane and column workgroups both
// have 256 threads (variants 1 and 2), at most two states, without position
// moments or per-state projection axes.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "itse_fin.h"
#include "itse_internal.h"
#include "itse_pass.h"
#include "itse_persist.h"

namespace itse {

namespace {

constexpr int PBT = 256;  // threads per workgroup of the persistent kernel

// The (N, schedule variant) pairs the kernel runs, and their LDS needs.
template <int N, int V>
constexpr int plane_lds() {
    using G = Geo<float, N, V>;
    return G::PLANE_ELEMS * 8 + N * 8 + NQR * (G::NTP / 64) * 8;
}
template <int N, int V>
constexpr int cols_lds() {
    using G = Geo<float, N, V>;
    return N * G::CS * 8 + N * 8 + N * 8 + NQC * (G::NTC / 64) * 8;
}
template <int N, int V>
constexpr bool uniform_256() {
    return Geo<float, N, V>::NTP == PBT && Geo<float, N, V>::NTC == PBT;
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int LDS_BYTES =
    cmax(cmax(cmax(plane_lds<32, 1>(), cols_lds<32, 1>()),
              cmax(cmax(plane_lds<48, 1>(), cols_lds<48, 1>()), cmax(plane_lds<48, 2>(), cols_lds<48, 2>()))),
         cmax(cmax(cmax(plane_lds<64, 1>(), cols_lds<64, 1>()), cmax(plane_lds<64, 2>(), cols_lds<64, 2>())),
              cmax(cmax(plane_lds<96, 1>(), cols_lds<96, 1>()), cmax(plane_lds<96, 2>(), cols_lds<96, 2>()))));
static_assert(uniform_256<32, 1>() && uniform_256<48, 1>() && uniform_256<48, 2>() && uniform_256<64, 1>() &&
                  uniform_256<64, 2>() && uniform_256<96, 1>() && uniform_256<96, 2>(),
              "plane and column workgroups of 256 threads");
static_assert(NT == PBT, "the projection/Gram pass runs 256 threads");

enum PPass { PP_FWD = 0, PP_COLS, PP_INV, PP_GRAM, PP_FSUM, PP_FTAIL };

// tiles of a pass for one group
__device__ __forceinline__ int group_tiles(const PersistGroup &g, int pass) {
    switch (pass) {
    case PP_FWD:
    case PP_INV: return g.njobs * g.nb_plane;
    case PP_COLS: return g.njobs * g.nb_cols;
    case PP_GRAM: return g.gram ? g.nlats * g.nb_gram : 0;
    case PP_FSUM: return g.nlats * g.nq_fin;
    default: return g.nlats;
    }
}

// Calls f.template operator()<N, V>() for a group's (n, variant).
template <typename F>
__device__ __forceinline__ void by_shape(int n, int v, F &&f) {
    if (n == 32) f.template operator()<32, 1>();
    else if (n == 48) (v == 1 ? f.template operator()<48, 1>() : f.template operator()<48, 2>());
    else if (n == 64) (v == 1 ? f.template operator()<64, 1>() : f.template operator()<64, 2>());
    else (v == 1 ? f.template operator()<96, 1>() : f.template operator()<96, 2>());
}

struct TileRun {
    const PersistGroup &g;
    int pass, t;
    char *lds;
    template <int N, int V>
    __device__ __forceinline__ void operator()() const {
        using G = Geo<float, N, V>;
        C2<float> *big = (C2<float> *)lds;
        if (pass == PP_FWD || pass == PP_INV) {
            const int jb = t / G::NB_PLANE, spb = t % G::NB_PLANE;
            C2<float> *tw = big + G::PLANE_ELEMS;
            double *red = (double *)(tw + N);
            if (pass == PP_FWD) {
                if (g.kmax <= 1) plane_fwd_tile<float, N, V, 1>(g.jobs, spb, jb, big, tw);
                else plane_fwd_tile<float, N, V, 4>(g.jobs, spb, jb, big, tw);
            } else {
                if (g.kmax <= 1) plane_inv_tile<float, N, V, false, 1>(g.jobs, spb, jb, INV_UPDATE, big, tw, red);
                else plane_inv_tile<float, N, V, false, 4>(g.jobs, spb, jb, INV_UPDATE, big, tw, red);
            }
        } else if (pass == PP_COLS) {
            const int jy = t / G::NB_COLS, blk = t % G::NB_COLS;
            C2<float> *tw = big + N * G::CS;
            double *ktab = (double *)(tw + N);
            double *red = ktab + N;
            columns_tile<float, N, V>(g.jobs, blk, jy, COL_KIN, 1, nullptr, big, tw, ktab, red);
        } else {
            const int ly = t / g.nb_gram, bx = t % g.nb_gram;
            double *red = (double *)lds;
            if (g.kmax <= 1) project_gram_vec_tile<float, 1, N>(g.lats, bx, g.nb_gram, ly, 0, 1, red);
            else project_gram_vec_tile<float, 2, N>(g.lats, bx, g.nb_gram, ly, 0, 1, red);
        }
    }
};

// Three workgroups per CU (the LDS of the largest tile allows three): at most 168
// VGPRs, which the largest tile (the two-state projection/Gram tile) fits.
__global__ void __launch_bounds__(PBT) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_batch_persistent(const PersistPlan *__restrict__ plan, int nsteps) {
    __shared__ __attribute__((aligned(16))) char lds[LDS_BYTES > (int)sizeof(FinTailLds) ? LDS_BYTES
                                                                                     : (int)sizeof(FinTailLds)];
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    const int ngroups = plan->ngroups;
    for (int s = 0; s < nsteps; ++s) {
#pragma unroll 1
        for (int p = 0; p < 6; ++p) {
            int total = 0;
            for (int k = 0; k < ngroups; ++k) total += group_tiles(plan->g[k], p);
            if (total == 0) continue;  // uniform over the grid
            for (int it = blockIdx.x; it < total; it += gridDim.x) {
                // the group of tile `it` and its index within the group
                int k = 0, t = it;
                while (t >= group_tiles(plan->g[k], p)) t -= group_tiles(plan->g[k++], p);
                const PersistGroup &g = plan->g[k];
                __syncthreads();  // the previous tile's readers of the LDS are done
                if (p == PP_FSUM) {
                    fin_sums_tile<PBT>(g.lats, t % g.nq_fin, t / g.nq_fin, FIN_STEP, (double *)lds);
                } else if (p == PP_FTAIL) {
                    fin_tail_tile(g.lats, t, FIN_STEP, *(FinTailLds *)lds);
                } else {
                    by_shape(g.n, g.variant, TileRun{g, p, t, lds});
                }
            }
            // the pass's global writes, visible to every workgroup (on every XCD) after
            // the barrier
            __threadfence();
            grid.sync();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
    }
}

}  // namespace

bool persist_shape_ok(int n, int prec, int variant) {
    if (prec != ITSE_FP32) return false;
    if (n == 32) return variant == 1;
    return (n == 48 || n == 64 || n == 96) && (variant == 1 || variant == 2);
}

int persist_nb_plane(int n, int variant) { return Launch<float>::schedule(n, variant).nb_rows; }
int persist_nb_cols(int n, int variant) { return Launch<float>::schedule(n, variant).nb_cols; }

hipError_t persist_grid(int *blocks) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persistent, PBT, 0);
    if (e != hipSuccess) return e;
    *blocks = cus * per_cu;
    return *blocks > 0 ? hipSuccess : hipErrorInvalidConfiguration;
}

hipError_t persist_launch(const PersistPlan *plan_dev, int nsteps, int blocks, hipStream_t s) {
    const PersistPlan *p = plan_dev;
    int ns = nsteps;
    void *args[] = {&p, &ns};
    return hipLaunchCooperativeKernel((const void *)k_batch_persistent, dim3(blocks), dim3(PBT), args, 0, s);
}

}  // namespace itse
