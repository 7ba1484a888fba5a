// Serving: eigensolve requests admitted by HBM footprint and stepped together.
//
// Requests wait in arrival order; the head of the queue is admitted when its
// footprint fits the budget beside the live requests and a slot is free (strict
// arrival order, so a large request is never overtaken indefinitely).  Live
// requests advance together, one chunk of steps per progress call, through a
// batch (one graph launch per chunk; membership changes rebuild the batch).  A
// request's arrays, sums and step sequence are its own, so its results are the
// same alone and in any mix.  After each chunk the energies are compared with
// those of the previous chunk; a request completes when every state moved by at
// most tol (relative to |E| if asked), or at its step limit, and its device
// memory is released at once.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "itse_internal.h"
#include "itse_runtime.h"

using namespace itse;

namespace {

struct Pending {
    uint64_t id = 0;
    itse_request req{};                    // pointers cleared; data below
    std::vector<char> potential;           // N^3 values of potential_dtype
    std::vector<std::vector<char>> states; // nstates arrays of state_dtype
    double t_submit = 0.0;
};

struct Live {
    Pending p;
    itse_lattice *lat = nullptr;
    size_t bytes = 0;
    double t_admit = 0.0;
    long long steps = 0;
    bool has_prev = false;
    double prev[ITSE_MAX_STATES] = {};
};

size_t dtype_size(int dt) { return dt == ITSE_DTYPE_F32 ? 4 : 8; }

}  // namespace

struct itse_server {
    size_t budget = 0;
    int max_slots = 0;
    int chunk = 0;
    hipStream_t stream = nullptr;
    uint64_t next_id = 1;
    std::deque<Pending> queue;
    std::vector<Live> live;
    std::deque<itse_result> done;
    struct Kept {
        int dtype = ITSE_DTYPE_F64;
        std::vector<std::vector<char>> states;
    };
    std::map<uint64_t, Kept> kept;  // final states of requests that asked for them
    size_t in_use = 0;
    itse_batch *batch = nullptr;
    bool dirty = true;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

extern "C" itse_status itse_server_create(size_t hbm_budget, int max_slots, int chunk, void *hip_stream,
                                          itse_server **out) {
    if (!out) return fail(ITSE_EINVAL, "null argument");
    *out = nullptr;
    if (hbm_budget == 0 || max_slots < 1 || chunk < 1) return fail(ITSE_EINVAL, "budget, slots and chunk must be > 0");
    itse_server *s = new itse_server();
    s->budget = hbm_budget;
    s->max_slots = max_slots;
    s->chunk = chunk;
    s->stream = (hipStream_t)hip_stream;
    *out = s;
    return ITSE_OK;
}

static void retire(itse_server *s, size_t k, itse_status status, bool converged) {
    Live &L = s->live[k];
    itse_result r{};
    r.id = L.p.id;
    r.status = status;
    r.converged = converged ? 1 : 0;
    r.steps = L.steps;
    for (int i = 0; i < L.p.req.desc.nstates; ++i) {
        itse_obs o{};
        if (status == ITSE_OK && itse_observe(L.lat, i, &o) == ITSE_OK) r.energy[i] = o.energy;
        else r.energy[i] = NAN;
    }
    r.t_submit = L.p.t_submit;
    r.t_admit = L.t_admit;
    if (status == ITSE_OK && L.p.req.keep_states) {
        const size_t n3 = (size_t)L.p.req.desc.n * L.p.req.desc.n * L.p.req.desc.n;
        const int dt = L.p.req.state_dtype;
        std::vector<std::vector<char>> st(L.p.req.desc.nstates, std::vector<char>(n3 * dtype_size(dt)));
        for (int i = 0; i < L.p.req.desc.nstates; ++i)
            if (itse_get_state(L.lat, i, st[i].data(), dt, 0) != ITSE_OK) r.status = ITSE_EDEVICE;
        s->kept[r.id] = itse_server::Kept{dt, std::move(st)};
    }
    itse_destroy(L.lat);
    s->in_use -= L.bytes;
    r.t_done = s->now();
    s->done.push_back(r);
    s->live.erase(s->live.begin() + (long)k);
    s->dirty = true;
}

extern "C" itse_status itse_server_destroy(itse_server *s) {
    if (!s) return ITSE_OK;
    if (s->batch) itse_batch_destroy(s->batch);
    for (auto &L : s->live) itse_destroy(L.lat);
    delete s;
    return ITSE_OK;
}

extern "C" itse_status itse_server_submit(itse_server *s, const itse_request *req, uint64_t *id) {
    if (!s || !req || !req->potential || !req->states) return fail(ITSE_EINVAL, "null argument");
    const itse_desc &d = req->desc;
    if (d.nstates < 1 || d.nstates > ITSE_MAX_STATES) return fail(ITSE_EINVAL, "nstates = %d", d.nstates);
    if (d.complex_psi) return fail(ITSE_EINVAL, "the server takes real states only (complex_psi = 0)");
    if ((req->potential_dtype != ITSE_DTYPE_F32 && req->potential_dtype != ITSE_DTYPE_F64) ||
        (req->state_dtype != ITSE_DTYPE_F32 && req->state_dtype != ITSE_DTYPE_F64))
        return fail(ITSE_EINVAL, "dtype");
    if (!(req->tol >= 0.0) || req->max_steps < 1) return fail(ITSE_EINVAL, "tol >= 0 and max_steps >= 1 needed");
    for (int i = 0; i < d.nstates; ++i)
        if (!req->states[i]) return fail(ITSE_EINVAL, "state %d is null", i);
    if (!prec_supported(d.n, d.precision)) return fail(ITSE_EINVAL, "n = %d not supported", d.n);
    if (d.a > 0 && d.mass > 0 && d.dtau * max_symbol(d) > 1.95)
        return fail(ITSE_EUNSTABLE, "dtau * max T(k) = %.4f > 1.95", d.dtau * max_symbol(d));
    const size_t fp = itse_footprint_bytes(&d);
    if (fp > s->budget) return fail(ITSE_ENOMEM, "request needs %zu bytes, budget is %zu", fp, s->budget);
    Pending p;
    p.id = s->next_id++;
    p.req = *req;
    p.req.potential = nullptr;
    p.req.states = nullptr;
    const size_t n3 = (size_t)d.n * d.n * d.n;
    const size_t pb = n3 * dtype_size(req->potential_dtype), sb = n3 * dtype_size(req->state_dtype);
    p.potential.assign((const char *)req->potential, (const char *)req->potential + pb);
    p.states.resize(d.nstates);
    for (int i = 0; i < d.nstates; ++i)
        p.states[i].assign((const char *)req->states[i], (const char *)req->states[i] + sb);
    p.t_submit = s->now();
    if (id) *id = p.id;
    s->queue.push_back(std::move(p));
    return ITSE_OK;
}

// Create the lattice of the queue head and upload its inputs.
static itse_status admit_head(itse_server *s) {
    Pending &p = s->queue.front();
    Live L;
    itse_status st = itse_create(&p.req.desc, s->stream, nullptr, nullptr, nullptr, &L.lat);
    if (!st) st = itse_set_potential(L.lat, p.potential.data(), p.req.potential_dtype, 0);
    for (int i = 0; i < p.req.desc.nstates && !st; ++i)
        st = itse_set_state(L.lat, i, p.states[i].data(), p.req.state_dtype, 0);
    if (!st) st = itse_set_step_opts(L.lat, &p.req.opts);
    if (st) {
        itse_result r{};
        r.id = p.id;
        r.status = st;
        r.t_submit = p.t_submit;
        r.t_admit = r.t_done = s->now();
        for (int i = 0; i < ITSE_MAX_STATES; ++i) r.energy[i] = NAN;
        s->done.push_back(r);
        if (L.lat) itse_destroy(L.lat);
        s->queue.pop_front();
        return ITSE_OK;  // reported through the result
    }
    L.bytes = itse_footprint_bytes(&p.req.desc);
    L.t_admit = s->now();
    p.potential.clear();
    p.potential.shrink_to_fit();
    p.states.clear();
    L.p = std::move(p);
    s->queue.pop_front();
    s->in_use += L.bytes;
    s->live.push_back(std::move(L));
    s->dirty = true;
    return ITSE_OK;
}

extern "C" itse_status itse_server_progress(itse_server *s, int *live, int *queued) {
    if (!s) return fail(ITSE_EINVAL, "null server");
    // admission in arrival order
    while (!s->queue.empty() && (int)s->live.size() < s->max_slots) {
        const size_t fp = itse_footprint_bytes(&s->queue.front().req.desc);
        if (s->in_use + fp > s->budget) break;
        itse_status st = admit_head(s);
        if (st) return st;
    }
    if (!s->live.empty()) {
        if (s->dirty) {
            if (s->batch) {
                itse_batch_destroy(s->batch);
                s->batch = nullptr;
            }
            std::vector<itse_lattice *> lats;
            for (auto &L : s->live) lats.push_back(L.lat);
            itse_status st = itse_batch_create((int)lats.size(), lats.data(), s->stream, &s->batch);
            if (st) return st;
            s->dirty = false;
        }
        itse_status st = itse_batch_step(s->batch, s->chunk);
        if (st) return st;
        if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(ITSE_EDEVICE, "stream synchronise failed");
        for (size_t k = 0; k < s->live.size();) {
            Live &L = s->live[k];
            L.steps += s->chunk;
            const int K = L.p.req.desc.nstates;
            double e[ITSE_MAX_STATES];
            itse_status est = ITSE_OK;
            for (int i = 0; i < K && !est; ++i) {
                itse_obs o{};
                est = itse_observe(L.lat, i, &o);
                e[i] = o.energy;
            }
            if (est) {
                retire(s, k, est, false);
                continue;
            }
            bool conv = L.has_prev;
            for (int i = 0; i < K && conv; ++i) {
                const double scale = L.p.req.tol_relative ? std::fabs(e[i]) : 1.0;
                if (!(std::fabs(e[i] - L.prev[i]) <= L.p.req.tol * scale)) conv = false;
            }
            for (int i = 0; i < K; ++i) L.prev[i] = e[i];
            L.has_prev = true;
            if (conv || L.steps >= L.p.req.max_steps) {
                retire(s, k, ITSE_OK, conv);
                continue;
            }
            ++k;
        }
    }
    if (live) *live = (int)s->live.size();
    if (queued) *queued = (int)s->queue.size();
    return ITSE_OK;
}

extern "C" itse_status itse_server_poll(itse_server *s, itse_result *out, int max, int *n_out) {
    if (!s || !n_out || (max > 0 && !out)) return fail(ITSE_EINVAL, "null argument");
    int n = 0;
    while (n < max && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    *n_out = n;
    return ITSE_OK;
}

extern "C" itse_status itse_server_state(itse_server *s, uint64_t id, int i, void *out, int dtype) {
    if (!s || !out) return fail(ITSE_EINVAL, "null argument");
    auto it = s->kept.find(id);
    if (it == s->kept.end()) return fail(ITSE_ENOTFOUND, "no kept states for request %llu", (unsigned long long)id);
    if (i < 0 || i >= (int)it->second.states.size()) return fail(ITSE_EINVAL, "state index %d", i);
    if (dtype != ITSE_DTYPE_F32 && dtype != ITSE_DTYPE_F64) return fail(ITSE_EINVAL, "dtype");
    const std::vector<char> &src = it->second.states[i];
    const int sdt = it->second.dtype;
    if (sdt == dtype) {
        std::memcpy(out, src.data(), src.size());
    } else {
        const size_t count = src.size() / dtype_size(sdt);
        for (size_t e = 0; e < count; ++e) {
            const double v = sdt == ITSE_DTYPE_F32 ? (double)((const float *)src.data())[e]
                                                   : ((const double *)src.data())[e];
            if (dtype == ITSE_DTYPE_F32) ((float *)out)[e] = (float)v;
            else ((double *)out)[e] = v;
        }
    }
    return ITSE_OK;
}

extern "C" itse_status itse_server_release(itse_server *s, uint64_t id) {
    if (!s) return fail(ITSE_EINVAL, "null server");
    s->kept.erase(id);
    return ITSE_OK;
}

extern "C" size_t itse_server_bytes_in_use(const itse_server *s) { return s ? s->in_use : 0; }
