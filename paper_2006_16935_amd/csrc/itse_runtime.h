// Host-side runtime structures shared by the runtime translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "itse_internal.h"

#define ITSE_GRAPH_CHUNK 16

namespace itse {

// Optional work of a step: the one-state-at-a-time projection (states projected
// along different axes), the fused projection + Gram pass (any projection, or
// Gram-Schmidt of more than one state), and the position moments (the kernel
// instance that sums them).  A step without the first two only launches the
// transform passes and the finalisation.
enum StepNeeds { NEED_PROJECT = 1, NEED_GRAM = 2, NEED_MOMENTS = 4 };

// A set of jobs of equal (n, precision, schedule) stepped by the same launches.
struct Group {
    int n = 0, prec = 0, variant = 0;
    const JobRef *jobs = nullptr;  // device array of (lattice, state)
    int njobs = 0;
    const JobRef *lats = nullptr;  // device array of (lattice, 0)
    int nlats = 0;
    int kmax = 1;                  // largest number of states among the lattices
    int needs = NEED_PROJECT | NEED_GRAM | NEED_MOMENTS;  // optional work of a step
    bool fdtd = false;             // H_K^(0): one stencil pass instead of the transforms
    bool cplx = false;             // complex lattices (jobs: every lattice's state 0, then every state 1)
    int nb_cplx = 0;               // complex lattices: workgroups of the separate complex update
};

itse_status fail(itse_status st, const char *fmt, ...);
int step_needs(const LatDev &opts, int nstates);
hipError_t enqueue_step(const Group &g, hipStream_t s);
hipError_t enqueue_eval(const Group &g, hipStream_t s);
itse_status capture_steps(hipStream_t cap, const std::vector<Group> &groups, int nsteps,
                          std::vector<hipStream_t> &branch, hipGraphExec_t *out);
bool prec_supported(int n, int prec);
Sched prec_schedule(int n, int prec, int variant);
int schedule_variant_for(int n, int prec, int nstates);
double max_symbol(const itse_desc &d);
itse_status norm_host(itse_lattice *L, int i, double *out);
hipError_t launch_check_potential(const LatDev *lat, int prec, hipStream_t s);

}  // namespace itse

struct itse_lattice {
    itse_desc d{};
    int device = 0;                 // HIP device current at create
    hipStream_t stream = nullptr;
    itse_alloc_fn alloc = nullptr;
    itse_free_fn freefn = nullptr;
    void *alloc_user = nullptr;
    std::vector<void *> allocations;
    itse::LatDev host{};            // host mirror of the device record
    itse::LatDev *dev = nullptr;    // device record
    itse::JobRef *jobs_dev = nullptr;  // [MAXK] (lattice, state i)
    itse::JobRef *lat_dev = nullptr;   // [1] (lattice, 0)
    void **tmp_ptrs_dev = nullptr;     // [MAXK] all pointing at tmp
    void *tmp = nullptr;               // N^3 scratch in the lattice precision
    void *staging = nullptr;
    size_t staging_bytes = 0;
    itse::Sched sched{};
    int variant = 0;
    long long steps_host = 0;
    itse_step_opts opts{};
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph1 = nullptr;
    hipGraphExec_t graphN = nullptr;
    int graph_needs = -1;              // optional passes captured in graph1 / graphN
    itse_lattice *shadow = nullptr;    // FP64 twin for polish
    void *snap[ITSE_SNAPSHOTS] = {};   // snapshot ring of state 0
    void **snap_ptr_dev = nullptr;     // [ITSE_SNAPSHOTS] device copies of snap[]
    int snap_count = 0, snap_newest = -1;
    itse_lattice *snapx = nullptr;     // estimates of the snapshot-overlap extraction
    double *ana = nullptr;             // analysis partial sums (device)
    size_t ana_bytes = 0;
    void *mom_spec = nullptr;          // half spectrum for the momentum-space analysis
    void *cur_raw(int i) const { return itse::state_buf(host, steps_host, 0, i); }
    void *stage_buf(size_t bytes);
    ~itse_lattice();
};
