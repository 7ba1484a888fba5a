// Batched stepping of independent lattices and schedule selection.
//
// A batch groups its lattices by (n, precision, schedule); every pass of the
// step is one launch per group whose grid covers all (lattice, state) jobs of
// the group.  A chunk of steps for all groups is captured once into a HIP graph
// (groups on parallel branches) and replayed with a single graph launch.  The
// per-job computation is the same code with the same workgroup->data mapping as
// a lone lattice, so results are bitwise identical alone and in a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "itse_internal.h"
#include "itse_persist.h"
#include "itse_runtime.h"

using namespace itse;

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(ITSE_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                  \
    } while (0)

struct itse_batch {
    std::vector<itse_lattice *> lats;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    std::vector<hipStream_t> branch;
    std::vector<Group> groups;
    std::vector<std::vector<itse_lattice *>> members;  // lattices of each group
    std::vector<void *> dev_arrays;
    hipGraphExec_t graph1 = nullptr, graphN = nullptr;
    std::vector<hipEvent_t> evs;
    bool persistent = false;     // step through the persistent kernel
    int persist_blocks = 0;      // its cooperative grid
    PersistPlan pplan{};         // host copy of the plan
    PersistPlan *pplan_dev = nullptr;
};

// ------------------------------------------------------------------------------------
// Schedule registry (selected by itse_autotune / itse_schedule_set)
// ------------------------------------------------------------------------------------
// keyed by (n, precision, one-state lattice or not): the best schedule of a bare
// one-state step differs from that of a multi-state step
static std::mutex g_sched_mu;
static std::map<std::tuple<int, int, int>, int> g_sched;

namespace itse {
int schedule_variant_for(int n, int prec, int nstates) {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    auto it = g_sched.find({n, prec, nstates == 1 ? 1 : 0});
    return it == g_sched.end() ? 0 : it->second;
}
}  // namespace itse

static itse_status check_variant(int n, int precision, int variant) {
    if (!prec_supported(n, precision)) return fail(ITSE_EINVAL, "n = %d not supported", n);
    const int nv = precision == ITSE_FP32 ? Launch<float>::variants(n) : Launch<double>::variants(n);
    if (variant < 0 || variant >= nv) return fail(ITSE_EINVAL, "variant %d of %d", variant, nv);
    return ITSE_OK;
}

extern "C" itse_status itse_schedule_set(int n, int precision, int variant) {
    itse_status st = check_variant(n, precision, variant);
    if (st) return st;
    std::lock_guard<std::mutex> lk(g_sched_mu);
    g_sched[{n, precision, 0}] = variant;
    g_sched[{n, precision, 1}] = variant;
    return ITSE_OK;
}

extern "C" itse_status itse_schedule_set_states(int n, int precision, int nstates, int variant) {
    itse_status st = check_variant(n, precision, variant);
    if (st) return st;
    if (nstates < 1 || nstates > MAXK) return fail(ITSE_EINVAL, "nstates = %d", nstates);
    std::lock_guard<std::mutex> lk(g_sched_mu);
    g_sched[{n, precision, nstates == 1 ? 1 : 0}] = variant;
    return ITSE_OK;
}

extern "C" itse_status itse_schedule_get(int n, int precision, char *json, size_t len) {
    if (!prec_supported(n, precision)) return fail(ITSE_EINVAL, "n = %d not supported", n);
    const int v = schedule_variant_for(n, precision, 2);
    const int v1 = schedule_variant_for(n, precision, 1);
    Sched s = prec_schedule(n, precision, v);
    if (json && len) {
        snprintf(json, len,
                 "{\"n\": %d, \"precision\": %d, \"variant\": %d, \"variants\": %d, \"split\": %d, "
                 "\"plane_waves\": %d, \"cols_per_wg\": %d, \"cols_waves\": %d, \"wg_plane\": %d, "
                 "\"wg_cols\": %d, \"lds_plane\": %d, \"lds_cols\": %d, \"variant_one_state\": %d}",
                 n, precision, v, precision == ITSE_FP32 ? Launch<float>::variants(n) : Launch<double>::variants(n),
                 s.split, s.nwp, s.cols_w, s.nwc, s.nb_rows, s.nb_cols, s.lds_plane, s.lds_cols, v1);
    }
    return ITSE_OK;
}

// ------------------------------------------------------------------------------------
// Batches
// ------------------------------------------------------------------------------------
static void batch_release(itse_batch *b) {
    if (b->graph1) (void)hipGraphExecDestroy(b->graph1);
    if (b->graphN) (void)hipGraphExecDestroy(b->graphN);
    for (void *p : b->dev_arrays) (void)hipFree(p);
    for (auto s : b->branch) (void)hipStreamDestroy(s);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (auto e : b->evs) (void)hipEventDestroy(e);
}

extern "C" itse_status itse_batch_create(int count, itse_lattice *const *lats, void *stream, itse_batch **out) {
    if (!out || (count > 0 && !lats)) return fail(ITSE_EINVAL, "null argument");
    if (count <= 0) return fail(ITSE_EINVAL, "empty batch");
    *out = nullptr;
    for (int a = 0; a < count; ++a) {
        if (!lats[a]) return fail(ITSE_EINVAL, "lattice %d is null", a);
        for (int b = 0; b < a; ++b)
            if (lats[a] == lats[b]) return fail(ITSE_EINVAL, "lattice %d appears twice", a);
    }
    itse_batch *B = new itse_batch();
    B->stream = (hipStream_t)stream;
    B->lats.assign(lats, lats + count);
    auto bail = [&](itse_status st) {
        batch_release(B);
        delete B;
        return st;
    };
    // group by (n, precision, variant, kind: bit0 H_K^(0), bit1 complex), keeping
    // input order within a group
    std::map<std::tuple<int, int, int, int>, std::vector<itse_lattice *>> by;
    std::vector<std::tuple<int, int, int, int>> order;
    for (auto *L : B->lats) {
        auto key = std::make_tuple(L->d.n, L->d.precision, L->variant,
                                   (L->d.kin == ITSE_KIN_FDTD ? 1 : 0) | (L->host.cplx ? 2 : 0));
        if (!by.count(key)) order.push_back(key);
        by[key].push_back(L);
    }
    // largest groups first (sites x states): they start first and bound the step
    auto lat_work = [](const itse_lattice *L) { return (long long)L->d.n * L->d.n * L->d.n * L->d.nstates; };
    auto group_work = [&](const std::vector<itse_lattice *> &m) {
        long long w = 0;
        for (auto *L : m) w += lat_work(L);
        return w;
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](const auto &x, const auto &y) { return group_work(by[x]) > group_work(by[y]); });
    for (auto &key : order) {
        auto &members = by[key];
        std::vector<JobRef> jobs, lrefs;
        if (std::get<3>(key) & 2) {
            // complex lattices: every lattice's real part, then every imaginary part
            for (int i = 0; i < 2; ++i)
                for (auto *L : members) jobs.push_back(JobRef{L->dev, i, 0});
            for (auto *L : members) lrefs.push_back(JobRef{L->dev, 0, 0});
        } else {
            for (auto *L : members) {
                for (int i = 0; i < L->d.nstates; ++i) jobs.push_back(JobRef{L->dev, i, 0});
                lrefs.push_back(JobRef{L->dev, 0, 0});
            }
        }
        JobRef *dj = nullptr, *dl = nullptr;
        if (hipMalloc(&dj, jobs.size() * sizeof(JobRef)) != hipSuccess ||
            hipMalloc(&dl, lrefs.size() * sizeof(JobRef)) != hipSuccess)
            return bail(fail(ITSE_ENOMEM, "batch job arrays"));
        B->dev_arrays.push_back(dj);
        B->dev_arrays.push_back(dl);
        if (hipMemcpy(dj, jobs.data(), jobs.size() * sizeof(JobRef), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(dl, lrefs.data(), lrefs.size() * sizeof(JobRef), hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(ITSE_EDEVICE, "batch job upload"));
        Group g;
        g.n = std::get<0>(key);
        g.prec = std::get<1>(key);
        g.variant = std::get<2>(key);
        g.fdtd = (std::get<3>(key) & 1) != 0;
        g.cplx = (std::get<3>(key) & 2) != 0;
        g.nb_cplx = members[0]->host.nb_cplx;
        g.jobs = dj;
        g.njobs = (int)jobs.size();
        g.lats = dl;
        g.nlats = (int)lrefs.size();
        for (auto *L : members) g.kmax = std::max(g.kmax, L->d.nstates);
        B->groups.push_back(g);
        B->members.push_back(members);
    }
    if (hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(ITSE_EDEVICE, "stream create"));
    const int nbr = (int)std::min<size_t>(B->groups.size(), 8);
    for (int i = 0; i < nbr; ++i) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(ITSE_EDEVICE, "stream create"));
        B->branch.push_back(s);
    }
    *out = B;
    return ITSE_OK;
}

extern "C" itse_status itse_batch_set_persistent(itse_batch *B, int on) {
    if (!B) return fail(ITSE_EINVAL, "null batch");
    if (!on) {
        B->persistent = false;
        return ITSE_OK;
    }
    if (B->groups.size() > (size_t)PERSIST_GROUPS)
        return fail(ITSE_EINVAL, "persistent batches hold at most %d groups of equal shape", PERSIST_GROUPS);
    PersistPlan pl{};
    pl.ngroups = (int)B->groups.size();
    for (size_t gi = 0; gi < B->groups.size(); ++gi) {
        const Group &g = B->groups[gi];
        if (g.fdtd || g.cplx || g.kmax > 2 || !persist_shape_ok(g.n, g.prec, g.variant))
            return fail(ITSE_EINVAL,
                        "the persistent kernel takes FP32 transform lattices of real states, N in {32, 48, 64, "
                        "96} under schedule variants with 256-thread plane and column workgroups (1, or 2 "
                        "where N has it), at most two states (group n = %d, precision %d, variant %d, "
                        "%d states)",
                        g.n, g.prec, g.variant, g.kmax);
        PersistGroup &q = pl.g[gi];
        q.n = g.n;
        q.variant = g.variant;
        q.kmax = g.kmax;
        q.gram = 0;
        q.njobs = g.njobs;
        q.nlats = g.nlats;
        q.nb_plane = persist_nb_plane(g.n, g.variant);
        q.nb_cols = persist_nb_cols(g.n, g.variant);
        q.nb_gram = pg_blocks(g.n);
        q.nq_fin = g.kmax * NQR + g.kmax * (g.kmax + 1) / 2;  // rows, Gram (no moments)
        q.jobs = g.jobs;
        q.lats = g.lats;
    }
    int blocks = 0;
    hipError_t e = persist_grid(&blocks);
    if (e != hipSuccess) return fail(ITSE_EDEVICE, "persistent grid: %s", hipGetErrorString(e));
    if (!B->pplan_dev) {
        void *p = nullptr;
        if (hipMalloc(&p, sizeof(PersistPlan)) != hipSuccess) return fail(ITSE_ENOMEM, "persistent plan");
        B->pplan_dev = (PersistPlan *)p;
        B->dev_arrays.push_back(p);
    }
    B->pplan = pl;
    B->persist_blocks = blocks;
    B->persistent = true;
    return ITSE_OK;
}

extern "C" itse_status itse_batch_step(itse_batch *B, int nsteps) {
    if (!B) return fail(ITSE_EINVAL, "null batch");
    if (nsteps < 0) return fail(ITSE_EINVAL, "nsteps < 0");
    if (nsteps == 0) return ITSE_OK;
    // order after earlier work on each lattice's own stream
    for (auto *L : B->lats) {
        if (L->stream == B->stream) continue;
        hipEvent_t ev;
        HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIPCHK(hipEventRecord(ev, L->stream));
        HIPCHK(hipStreamWaitEvent(B->stream, ev, 0));
        HIPCHK(hipEventDestroy(ev));
    }
    // passes each group launches, from the members' current options; a change
    // since the graphs were captured captures them again
    bool changed = false;
    for (size_t gi = 0; gi < B->groups.size(); ++gi) {
        int needs = 0;
        for (auto *L : B->members[gi]) needs |= step_needs(L->host, L->d.nstates);
        if (needs != B->groups[gi].needs) changed = true;
        B->groups[gi].needs = needs;
    }
    // cached graphs of an older set of passes are dropped here, before either path,
    // so that a change made while stepping persistently is not missed later
    if (changed && (B->graph1 || B->graphN)) {
        HIPCHK(hipStreamSynchronize(B->stream));
        if (B->graph1) HIPCHK(hipGraphExecDestroy(B->graph1));
        if (B->graphN) HIPCHK(hipGraphExecDestroy(B->graphN));
        B->graph1 = B->graphN = nullptr;
    }
    // the persistent kernel, when the steps need no per-state projection pass and no
    // position moments (else the graph path)
    bool persist = B->persistent;
    for (size_t gi = 0; gi < B->groups.size() && persist; ++gi) {
        if (B->groups[gi].needs & (NEED_PROJECT | NEED_MOMENTS)) persist = false;
        B->pplan.g[gi].gram = (B->groups[gi].needs & NEED_GRAM) ? 1 : 0;
    }
    if (persist) {
        HIPCHK(hipMemcpyAsync(B->pplan_dev, &B->pplan, sizeof(PersistPlan), hipMemcpyHostToDevice, B->stream));
        hipError_t e = persist_launch(B->pplan_dev, nsteps, B->persist_blocks, B->stream);
        if (e != hipSuccess) return fail(ITSE_EDEVICE, "persistent batch launch: %s", hipGetErrorString(e));
        hipEvent_t done;
        HIPCHK(hipEventCreateWithFlags(&done, hipEventDisableTiming));
        HIPCHK(hipEventRecord(done, B->stream));
        for (auto *L : B->lats) {
            if (L->stream != B->stream) HIPCHK(hipStreamWaitEvent(L->stream, done, 0));
            L->steps_host += nsteps;
        }
        HIPCHK(hipEventDestroy(done));
        return ITSE_OK;
    }
    const int chunk = ITSE_GRAPH_CHUNK;
    if (nsteps >= chunk && !B->graphN) {
        itse_status st = capture_steps(B->cap, B->groups, chunk, B->branch, &B->graphN);
        if (st) return st;
    }
    if (!B->graph1) {
        itse_status st = capture_steps(B->cap, B->groups, 1, B->branch, &B->graph1);
        if (st) return st;
    }
    int left = nsteps;
    while (left >= chunk) {
        HIPCHK(hipGraphLaunch(B->graphN, B->stream));
        left -= chunk;
    }
    while (left-- > 0) HIPCHK(hipGraphLaunch(B->graph1, B->stream));
    hipEvent_t done;
    HIPCHK(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    HIPCHK(hipEventRecord(done, B->stream));
    for (auto *L : B->lats) {
        if (L->stream != B->stream) HIPCHK(hipStreamWaitEvent(L->stream, done, 0));
        L->steps_host += nsteps;
    }
    HIPCHK(hipEventDestroy(done));
    return ITSE_OK;
}

extern "C" itse_status itse_batch_destroy(itse_batch *B) {
    if (!B) return ITSE_OK;
    (void)hipStreamSynchronize(B->stream);
    batch_release(B);
    delete B;
    return ITSE_OK;
}

// ------------------------------------------------------------------------------------
// Autotuning: time every schedule variant for (n, precision) on a scratch lattice.
// ------------------------------------------------------------------------------------
// Mean time (ms) of a step of a lattice of `nstates` states under schedule
// variant v: synthetic states, parity +, -, - and Gram-Schmidt every step for
// several states (every kernel of a step runs), the bare step for one state.
// Time `count` lattices of (n, precision) with `nstates` states stepped under
// schedule v (one lattice: itse_step; several: one batch).  Mean ms per step.
static itse_status time_variant(int n, int precision, int v, int nstates, void *stream, float *out_ms,
                                int count = 1) {
    {
        std::lock_guard<std::mutex> lk(g_sched_mu);
        g_sched[{n, precision, nstates == 1 ? 1 : 0}] = v;
    }
    itse_desc d{};
    d.n = n;
    d.a = 0.1;
    d.mass = 1.0;
    d.kin = ITSE_KIN_REL_LAT;
    d.subtract_rest_mass = 1;
    d.dtau = 0.025;
    d.precision = precision;
    d.center = ITSE_CENTER_ORIGIN;
    d.nstates = nstates;
    std::vector<itse_lattice *> lats(count, nullptr);
    itse_batch *B = nullptr;
    itse_status st = ITSE_OK;
    const size_t n3 = (size_t)n * n * n;
    std::vector<double> psi(n3);
    itse_step_opts o{};
    o.ortho_every = nstates > 1 ? 1 : 0;
    if (nstates > 1) {
        o.parity[0] = 1;
        for (int i = 1; i < nstates; ++i) o.parity[i] = -1;
    }
    for (int i = 0; i < ITSE_MAX_STATES; ++i) o.axes[i] = 7;
    for (int c = 0; c < count && !st; ++c) {
        st = itse_create(&d, stream, nullptr, nullptr, nullptr, &lats[c]);
        for (int i = 0; i < d.nstates && !st; ++i) {
            for (size_t e = 0; e < n3; ++e) psi[e] = std::sin(0.37 * (double)(e % 100003) * (i + 1)) + 0.1 * i;
            st = itse_set_state(lats[c], i, psi.data(), ITSE_DTYPE_F64, 0);
        }
        if (!st) st = itse_set_step_opts(lats[c], &o);
    }
    if (!st && count > 1) st = itse_batch_create(count, lats.data(), stream, &B);
    auto steps = [&](int k) { return B ? itse_batch_step(B, k) : itse_step(lats[0], k, nullptr); };
    if (!st) st = steps(3);
    // steps per trial, and the fastest of three trials: the schedules of a size can
    // lie within a percent of each other (host-side setup of the lattices costs
    // more than these steps)
    const int reps = n >= 192 ? 30 : 60;
    float ms = 1e30f;
    for (int trial = 0; trial < 3 && !st; ++trial) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipError_t he = hipEventCreate(&e0);
        if (he == hipSuccess) he = hipEventCreate(&e1);
        if (he == hipSuccess) he = hipEventRecord(e0, (hipStream_t)stream);
        if (he == hipSuccess) st = steps(reps);
        if (he == hipSuccess && !st) he = hipEventRecord(e1, (hipStream_t)stream);
        if (he == hipSuccess && !st) he = hipEventSynchronize(e1);
        float t = 0.f;
        if (he == hipSuccess && !st) he = hipEventElapsedTime(&t, e0, e1);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (he != hipSuccess && !st) st = fail(ITSE_EDEVICE, "autotune timing: %s", hipGetErrorString(he));
        if (!st) ms = std::min(ms, t);
    }
    for (auto *L : lats)
        if (L && !st) st = itse_sync(L);
    if (B) itse_batch_destroy(B);
    for (auto *L : lats)
        if (L) itse_destroy(L);
    *out_ms = ms / reps;
    return st;
}

extern "C" itse_status itse_autotune(int n, int precision, void *stream, char *json, size_t len) {
    if (!prec_supported(n, precision)) return fail(ITSE_EINVAL, "n = %d not supported", n);
    const int nv = precision == ITSE_FP32 ? Launch<float>::variants(n) : Launch<double>::variants(n);
    std::string rep = "{\"n\": " + std::to_string(n) + ", \"precision\": " + std::to_string(precision);
    int best[2] = {0, 0};
    for (int one = 0; one < 2; ++one) {
        rep += one ? ", \"times_ms_one_state\": [" : ", \"times_ms\": [";
        float best_ms = 1e30f;
        for (int v = 0; v < nv; ++v) {
            float ms = 0.f;
            itse_status st = time_variant(n, precision, v, one ? 1 : 3, stream, &ms);
            if (st) return st;
            rep += (v ? ", " : "") + std::to_string(ms);
            if (ms < best_ms) {
                best_ms = ms;
                best[one] = v;
            }
        }
        rep += "]";
        std::lock_guard<std::mutex> lk(g_sched_mu);
        g_sched[{n, precision, one}] = best[one];
    }
    rep += ", \"best\": " + std::to_string(best[0]) + ", \"best_one_state\": " + std::to_string(best[1]) + "}";
    if (json && len) snprintf(json, len, "%s", rep.c_str());
    return ITSE_OK;
}

extern "C" itse_status itse_autotune_batch(int n, int precision, int count, int nstates, void *stream, char *json,
                                           size_t len) {
    if (!prec_supported(n, precision)) return fail(ITSE_EINVAL, "n = %d not supported", n);
    if (count < 1) return fail(ITSE_EINVAL, "count = %d", count);
    if (nstates < 1 || nstates > MAXK) return fail(ITSE_EINVAL, "nstates = %d", nstates);
    const int nv = precision == ITSE_FP32 ? Launch<float>::variants(n) : Launch<double>::variants(n);
    std::string rep = "{\"n\": " + std::to_string(n) + ", \"precision\": " + std::to_string(precision) +
                      ", \"count\": " + std::to_string(count) + ", \"nstates\": " + std::to_string(nstates) +
                      ", \"times_ms\": [";
    int best = 0;
    float best_ms = 1e30f;
    for (int v = 0; v < nv; ++v) {
        float ms = 0.f;
        itse_status st = time_variant(n, precision, v, nstates, stream, &ms, count);
        if (st) return st;
        rep += (v ? ", " : "") + std::to_string(ms);
        if (ms < best_ms) {
            best_ms = ms;
            best = v;
        }
    }
    rep += "], \"best\": " + std::to_string(best) + "}";
    {
        std::lock_guard<std::mutex> lk(g_sched_mu);
        g_sched[{n, precision, nstates == 1 ? 1 : 0}] = best;
    }
    if (json && len) snprintf(json, len, "%s", rep.c_str());
    return ITSE_OK;
}
