// Host runtime of the imaginary-time eigensolver: lattice objects, the C ABI of
// include/itse.h, the finalisation kernel (fixed-order FP64 sums, Gram-Schmidt
// coefficients by Cholesky of the Gram matrix), step sequencing, HIP graph
// capture and batched stepping of many lattices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "itse_internal.h"
#include "itse_fin.h"
#include "itse_pass.h"
#include "itse_runtime.h"

using namespace itse;

// ------------------------------------------------------------------------------------
// Errors
// ------------------------------------------------------------------------------------
static thread_local std::string g_err;

namespace itse {
itse_status fail(itse_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}
}  // namespace itse

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(ITSE_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                  \
    } while (0)

extern "C" const char *itse_last_error(void) { return g_err.c_str(); }
extern "C" const char *itse_version(void) { return "itse 0.1 (gfx950)"; }

// ------------------------------------------------------------------------------------
// Finalisation kernels: the step's sums, then observables and coefficients.
// ------------------------------------------------------------------------------------
namespace itse {

__global__ void __launch_bounds__(FIN_NT) k_fin_sums(const JobRef *__restrict__ lats, int mode) {
    __shared__ double red[FIN_NT / 64];
    fin_sums_tile<FIN_NT>(lats, blockIdx.x, blockIdx.y, mode, red);
}

__global__ void __launch_bounds__(64) k_fin_tail(const JobRef *__restrict__ lats, int mode) {
    __shared__ FinTailLds sh;
    fin_tail_tile(lats, blockIdx.x, mode, sh);
}

// Device-side check of 1 + dtau min(V)/2 > 0 and finiteness (for device-provided V).
template <typename R>
__global__ void __launch_bounds__(NT) k_check_potential(const LatDev *lp) {
    const LatDev &L = *lp;
    const size_t n3 = (size_t)L.n * L.n * L.n;
    const R *v = (const R *)L.v;
    int bad = 0;
    for (size_t s = (size_t)blockIdx.x * NT + threadIdx.x; s < n3; s += (size_t)gridDim.x * NT) {
        const double x = (double)v[s];
        if (!isfinite(x)) bad |= 1;
        else if (1.0 + L.h * x <= 0.0) bad |= 4;
    }
    if (bad) atomicOr((int *)&lp->error, bad);
}

hipError_t launch_finalize(const JobRef *lats, int nlats, int mode, hipStream_t s) {
    if (nlats <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fin_sums, dim3(FIN_QMAX, nlats), dim3(FIN_NT), 0, s, lats, mode);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fin_tail, dim3(nlats), dim3(64), 0, s, lats, mode);
    return hipGetLastError();
}

hipError_t launch_check_potential(const LatDev *lat, int prec, hipStream_t s) {
    if (prec == ITSE_FP32)
        hipLaunchKernelGGL(k_check_potential<float>, dim3(256), dim3(NT), 0, s, lat);
    else
        hipLaunchKernelGGL(k_check_potential<double>, dim3(256), dim3(NT), 0, s, lat);
    return hipGetLastError();
}

}  // namespace itse

// ------------------------------------------------------------------------------------
// Per-precision dispatch helpers
// ------------------------------------------------------------------------------------
namespace itse {

static size_t real_bytes(int prec) { return prec == ITSE_FP32 ? 4 : 8; }

bool prec_supported(int n, int prec) {
    return prec == ITSE_FP32 ? Launch<float>::supported(n) : Launch<double>::supported(n);
}

Sched prec_schedule(int n, int prec, int variant) {
    return prec == ITSE_FP32 ? Launch<float>::schedule(n, variant) : Launch<double>::schedule(n, variant);
}

// Host-side kinetic tables and stability bound (FP64).
static void kinetic_axis_table(const itse_desc &d, std::vector<double> &tab) {
    const int n = d.n;
    tab.resize(n);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        const int m = (2 * i <= n) ? i : i - n;
        const double k = 2.0 * pi * (double)m / (double)n;
        const double s = std::sin(0.5 * k);
        switch (d.kin) {
        case ITSE_KIN_NR_CONT: tab[i] = k * k / (2.0 * d.a * d.a * d.mass); break;
        case ITSE_KIN_FDTD:  // bounded by the periodic stencil's symbol
        case ITSE_KIN_NR_LAT: tab[i] = 4.0 * s * s / (2.0 * d.a * d.a * d.mass); break;
        case ITSE_KIN_REL_LAT: tab[i] = 4.0 * s * s / (d.a * d.a); break;
        default: tab[i] = k * k / (d.a * d.a); break;
        }
    }
}

double max_symbol(const itse_desc &d) {
    std::vector<double> tab;
    kinetic_axis_table(d, tab);
    const double mx = *std::max_element(tab.begin(), tab.end());
    const double s = 3.0 * mx;
    if (d.kin == ITSE_KIN_NR_CONT || d.kin == ITSE_KIN_NR_LAT || d.kin == ITSE_KIN_FDTD) return s;
    const double e = std::sqrt(s + d.mass * d.mass);
    return d.subtract_rest_mass ? s / (e + d.mass) : e;
}

// ------------------------------------------------------------------------------------
// Twiddle tables, shared per (device, n, precision)
// ------------------------------------------------------------------------------------
static std::mutex g_tw_mu;
static std::map<std::tuple<int, int, int>, void *> g_tw;

static itse_status twiddles(int n, int prec, void **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_tw_mu);
    auto key = std::make_tuple(dev, n, prec);
    auto it = g_tw.find(key);
    if (it != g_tw.end()) {
        *out = it->second;
        return ITSE_OK;
    }
    const double pi = 3.14159265358979323846;
    std::vector<double> d(2 * n);
    for (int e = 0; e < n; ++e) {
        const double ang = -2.0 * pi * (double)e / (double)n;
        d[2 * e] = std::cos(ang);
        d[2 * e + 1] = std::sin(ang);
    }
    void *p = nullptr;
    HIPCHK(hipMalloc(&p, 2 * n * real_bytes(prec)));
    if (prec == ITSE_FP32) {
        // each entry: of the float pairs within one ulp of (cos, sin) (each
        // component rounded down or up), the one whose magnitude is closest to 1,
        // ties to the nearest pair.  Plain rounding to nearest leaves magnitude
        // errors whose mean over a table is negative (a few 1e-9 to 2e-8 per
        // transform), which biases energies formed through the transforms; the
        // closest-to-unit choice leaves a mean of either sign a few times smaller
        std::vector<float> f(2 * n);
        for (int e = 0; e < n; ++e) {
            const double c = d[2 * e], sv = d[2 * e + 1];
            float cand_c[2], cand_s[2];
            auto around = [](double x, float out[2]) {
                const float r = (float)x;
                out[0] = (double)r <= x ? r : std::nextafter(r, -INFINITY);
                out[1] = (double)r >= x ? r : std::nextafter(r, INFINITY);
            };
            around(c, cand_c);
            around(sv, cand_s);
            double best_norm = 1e300, best_dist = 1e300;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    const double cc = cand_c[a], ss = cand_s[b];
                    const double nerr = std::fabs(cc * cc + ss * ss - 1.0);
                    const double dist = std::fabs(cc - c) + std::fabs(ss - sv);
                    if (nerr < best_norm || (nerr == best_norm && dist < best_dist)) {
                        best_norm = nerr;
                        best_dist = dist;
                        f[2 * e] = cand_c[a];
                        f[2 * e + 1] = cand_s[b];
                    }
                }
        }
        HIPCHK(hipMemcpy(p, f.data(), f.size() * 4, hipMemcpyHostToDevice));
    } else {
        HIPCHK(hipMemcpy(p, d.data(), d.size() * 8, hipMemcpyHostToDevice));
    }
    g_tw[key] = p;
    *out = p;
    return ITSE_OK;
}

// ------------------------------------------------------------------------------------
// Kernel sequences
// ------------------------------------------------------------------------------------
template <typename R>
static hipError_t seq_forward_kin(const Group &g, int inv_mode, hipStream_t s) {
    if (g.fdtd) return Launch<R>::fdtd(g.n, g.kmax, inv_mode, g.jobs, g.njobs, s);
    hipError_t e;
    if ((e = Launch<R>::plane_fwd(g.n, g.variant, g.kmax, g.jobs, g.njobs, s)) != hipSuccess) return e;
    if ((e = Launch<R>::columns(g.n, g.variant, COL_KIN, 1, g.jobs, g.njobs, nullptr, s)) != hipSuccess) return e;
    return Launch<R>::plane_inv(g.n, g.variant, inv_mode, (g.needs & NEED_MOMENTS) ? 1 : 0, g.kmax, g.jobs, g.njobs,
                                s);
}

int step_needs(const LatDev &o, int nstates) {
    int m = 0;
    if (o.proj_mode == 2) m |= NEED_PROJECT;
    if (o.proj_mode != 0 || (nstates > 1 && o.ortho_every > 0)) m |= NEED_GRAM;
    if (o.moments) m |= NEED_MOMENTS;
    return m;
}

// Complex lattices: the transforms and the complex update.  Transform lattices
// without position moments: both parts forward, the real parts' inverse pass
// writing K Re psi to kbuf, then the imaginary parts' inverse pass, which applies
// the complex update to both parts.  Otherwise (H_K^(0), or moments, whose sums
// leave no registers for the fused update): K psi of both parts to kbuf, then the
// separate complex update.
static bool cplx_fused(const Group &g) { return !g.fdtd && !(g.needs & NEED_MOMENTS); }

template <typename R>
static hipError_t seq_cplx_update(const Group &g, hipStream_t s) {
    hipError_t e;
    if (!cplx_fused(g)) {
        if ((e = seq_forward_kin<R>(g, INV_KBUF, s)) != hipSuccess) return e;
        return Launch<R>::complex_update(g.n, g.nb_cplx, g.lats, g.nlats, INV_UPDATE, s);
    }
    if ((e = Launch<R>::plane_fwd(g.n, g.variant, g.kmax, g.jobs, g.njobs, s)) != hipSuccess) return e;
    if ((e = Launch<R>::columns(g.n, g.variant, COL_KIN, 1, g.jobs, g.njobs, nullptr, s)) != hipSuccess) return e;
    if ((e = Launch<R>::plane_inv(g.n, g.variant, INV_KBUF, 0, g.kmax, g.jobs, g.nlats, s)) != hipSuccess) return e;
    return Launch<R>::plane_inv_cplx(g.n, g.variant, g.jobs + g.nlats, g.nlats, s);
}

template <typename R>
static hipError_t seq_step(const Group &g, hipStream_t s) {
    hipError_t e;
    if (g.cplx) {
        // projection (both parts, same sign and axes) with the norm in the Gram pass
        if ((e = seq_cplx_update<R>(g, s)) != hipSuccess) return e;
        if ((g.needs & NEED_GRAM) &&
            (e = Launch<R>::project_gram(g.n, g.kmax, g.lats, g.nlats, 0, 1, s)) != hipSuccess)
            return e;
        return launch_finalize(g.lats, g.nlats, FIN_STEP, s);
    }
    if ((e = seq_forward_kin<R>(g, INV_UPDATE, s)) != hipSuccess) return e;
    if ((g.needs & NEED_PROJECT) && (e = Launch<R>::project(g.n, g.jobs, g.njobs, 0, 0, 1, s)) != hipSuccess)
        return e;
    if ((g.needs & NEED_GRAM) &&
        (e = Launch<R>::project_gram(g.n, g.kmax, g.lats, g.nlats, 0, 1, s)) != hipSuccess)
        return e;
    return launch_finalize(g.lats, g.nlats, FIN_STEP, s);
}

hipError_t enqueue_step(const Group &g, hipStream_t s) {
    return g.prec == ITSE_FP32 ? seq_step<float>(g, s) : seq_step<double>(g, s);
}

hipError_t enqueue_eval(const Group &g, hipStream_t s) {
    const int mode = g.cplx ? INV_KBUF : INV_EVAL;
    hipError_t e = g.prec == ITSE_FP32 ? seq_forward_kin<float>(g, mode, s) : seq_forward_kin<double>(g, mode, s);
    if (e == hipSuccess && g.cplx)
        e = g.prec == ITSE_FP32 ? Launch<float>::complex_update(g.n, g.nb_cplx, g.lats, g.nlats, INV_EVAL, s)
                                : Launch<double>::complex_update(g.n, g.nb_cplx, g.lats, g.nlats, INV_EVAL, s);
    if (e != hipSuccess) return e;
    return launch_finalize(g.lats, g.nlats, FIN_EVAL, s);
}

}  // namespace itse

// ------------------------------------------------------------------------------------
// Lattice object
// ------------------------------------------------------------------------------------
itse_lattice::~itse_lattice() {}

namespace itse {

// Current raw array of state i on the device (the device flips buffers every step).
static void *cur_state(itse_lattice *L, int i) { return L->cur_raw(i); }

void *lat_alloc(itse_lattice *L, size_t bytes) {
    void *p = nullptr;
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    if (L->alloc) {
        p = L->alloc(bytes, L->alloc_user);
    } else {
        if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    }
    if (p) L->allocations.push_back(p);
    return p;
}

void lat_free_all(itse_lattice *L) {
    for (void *p : L->allocations) {
        if (L->freefn) L->freefn(p, L->alloc_user);
        else if (!L->alloc) (void)hipFree(p);
    }
    L->allocations.clear();
}

itse_status upload_latdev(itse_lattice *L) {
    HIPCHK(hipMemcpyAsync(L->dev, &L->host, sizeof(LatDev), hipMemcpyHostToDevice, L->stream));
    return ITSE_OK;
}

// Write only the option fields (ortho_every .. paxes) to the device copy.
itse_status upload_opts(itse_lattice *L) {
    const size_t off = offsetof(LatDev, ortho_every);
    const size_t len = offsetof(LatDev, coef) - off;
    HIPCHK(hipMemcpyAsync((char *)L->dev + off, (char *)&L->host + off, len, hipMemcpyHostToDevice, L->stream));
    return ITSE_OK;
}

itse_status upload_field(itse_lattice *L, size_t off, size_t len) {
    HIPCHK(hipMemcpyAsync((char *)L->dev + off, (char *)&L->host + off, len, hipMemcpyHostToDevice, L->stream));
    return ITSE_OK;
}

itse_status set_identity_coef(itse_lattice *L) {
    for (int j = 0; j < MAXK; ++j)
        for (int i = 0; i < MAXK; ++i) L->host.coef[j][i] = (i == j) ? 1.0 : 0.0;
    return upload_field(L, offsetof(LatDev, coef), sizeof(L->host.coef));
}

itse_status check_device_error(itse_lattice *L) {
    int err = 0;
    HIPCHK(hipMemcpyAsync(&err, (char *)L->dev + offsetof(LatDev, error), sizeof(int), hipMemcpyDeviceToHost,
                          L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
    if (err) {
        int zero = 0;
        HIPCHK(hipMemcpy((char *)L->dev + offsetof(LatDev, error), &zero, sizeof(int), hipMemcpyHostToDevice));
        if (err & 4) return fail(ITSE_EUNSTABLE, "potential violates 1 + dtau min(V)/2 > 0");
        if (err & 2) return fail(ITSE_ENONFINITE, "Gram matrix not positive definite (states linearly dependent)");
        return fail(ITSE_ENONFINITE, "non-finite value in a reduction (NaN/Inf in state or potential)");
    }
    return ITSE_OK;
}

Group single_group(itse_lattice *L) {
    Group g;
    g.n = L->d.n;
    g.prec = L->d.precision;
    g.variant = L->variant;
    g.jobs = L->jobs_dev;
    g.njobs = L->d.nstates;
    g.lats = L->lat_dev;
    g.nlats = 1;
    g.kmax = L->d.nstates;
    g.needs = step_needs(L->host, L->d.nstates);
    g.fdtd = L->d.kin == ITSE_KIN_FDTD;
    g.cplx = L->host.cplx != 0;
    g.nb_cplx = L->host.nb_cplx;
    return g;
}

Group state_group(itse_lattice *L, int i) {
    Group g = single_group(L);
    g.jobs = L->jobs_dev + i;
    g.njobs = 1;
    return g;
}

// Replace the lazy representation by materialised states: psi_i = sum_(j<=i) coef[j][i] u_j
// is formed in the scratch array and copied over u_i, highest state first (psi_i only
// reads u_0..u_i), then coef = identity.
itse_status materialise(itse_lattice *L) {
    const int K = L->d.nstates;
    const size_t bytes = (size_t)L->d.n * L->d.n * L->d.n * real_bytes(L->d.precision);
    for (int i = K - 1; i >= 0; --i) {
        hipError_t e = L->d.precision == ITSE_FP32
                           ? Launch<float>::combine(L->d.n, L->jobs_dev + i, 1, L->tmp_ptrs_dev, L->stream)
                           : Launch<double>::combine(L->d.n, L->jobs_dev + i, 1, L->tmp_ptrs_dev, L->stream);
        if (e != hipSuccess) return fail(ITSE_EDEVICE, "combine launch: %s", hipGetErrorString(e));
        HIPCHK(hipMemcpyAsync(cur_state(L, i), L->tmp, bytes, hipMemcpyDeviceToDevice, L->stream));
    }
    return set_identity_coef(L);
}

}  // namespace itse

extern "C" size_t itse_footprint_bytes(const itse_desc *d) {
    if (!d || d->n < 1) return 0;
    const size_t w = real_bytes(d->precision);
    const size_t n = (size_t)d->n, n3 = n * n * n;
    const bool cplx = d->complex_psi == 1;
    const size_t K = cplx ? 2 : (size_t)std::max(1, std::min(d->nstates, MAXK));
    const size_t spec = spec_bytes(d->n, d->precision);
    size_t arena = 0;
    int rows_max = 0;
    if (prec_supported(d->n, d->precision)) {
        const int nv = d->precision == ITSE_FP32 ? Launch<float>::variants(d->n) : Launch<double>::variants(d->n);
        for (int v = 0; v < nv; ++v) {
            Sched s = prec_schedule(d->n, d->precision, v);
            if (d->kin == ITSE_KIN_FDTD)
                s.nb_rows = d->precision == ITSE_FP32 ? Launch<float>::fdtd_blocks(d->n)
                                                      : Launch<double>::fdtd_blocks(d->n);
            const size_t a = (size_t)MAXK * ((size_t)s.nb_rows * NQR + (size_t)s.nb_cols * NQC + s.nb_proj) * 8 +
                             (size_t)s.nb_gram * (MAXK * (MAXK + 1) / 2) * 8;
            arena = std::max(arena, a);
            rows_max = std::max(rows_max, s.nb_rows);
        }
    }
    const size_t hist = (size_t)HIST_CAP * MAXK * sizeof(ObsDev);
    // per state: two raw arrays u_i (current, next) and the half spectrum; shared: potential, scratch array,
    // staging for a host upload in the other precision (n^3 doubles), partial sums, history
    // complex lattices also: Im V, K Re psi and K Im psi, the complex-update partials
    const size_t cx = cplx ? 3 * n3 * w + (size_t)std::max(flat_blocks(d->n), rows_max) * NQX * 8 : 0;
    return K * (2 * n3 * w + spec) + n3 * w + n3 * w + n3 * 8 + arena + hist + sizeof(LatDev) + 8192 + n * 8 + cx;
}

static bool valid_n(int n) {
    if (n < 8 || n > 256) return false;
    int m = n;
    while (m % 2 == 0) m /= 2;
    while (m % 3 == 0) m /= 3;
    return m == 1;
}

extern "C" itse_status itse_create(const itse_desc *d, void *hip_stream, itse_alloc_fn alloc, itse_free_fn free_fn,
                                   void *alloc_user, itse_lattice **out) {
    if (!d || !out) return fail(ITSE_EINVAL, "null argument");
    *out = nullptr;
    if (!valid_n(d->n)) return fail(ITSE_EINVAL, "n = %d: need 8 <= n <= 256 with prime factors 2 and 3", d->n);
    if (!(d->a > 0) || !(d->mass > 0) || !(d->dtau > 0) || !std::isfinite(d->a) || !std::isfinite(d->mass) ||
        !std::isfinite(d->dtau))
        return fail(ITSE_EINVAL, "a, mass and dtau must be finite and > 0");
    if (d->kin < 0 || d->kin > 4) return fail(ITSE_EINVAL, "kin = %d", d->kin);
    if (d->precision != ITSE_FP32 && d->precision != ITSE_FP64) return fail(ITSE_EINVAL, "precision");
    if (d->center != ITSE_CENTER_CELL && d->center != ITSE_CENTER_ORIGIN) return fail(ITSE_EINVAL, "center");
    if (d->nstates < 1 || d->nstates > MAXK) return fail(ITSE_EINVAL, "nstates = %d (1..%d)", d->nstates, MAXK);
    if (d->complex_psi != 0 && d->complex_psi != 1) return fail(ITSE_EINVAL, "complex_psi = %d", d->complex_psi);
    if (d->complex_psi && d->nstates != 1) return fail(ITSE_EINVAL, "complex_psi needs nstates = 1");
    if (!prec_supported(d->n, d->precision)) return fail(ITSE_EINVAL, "n = %d not built", d->n);
    const double tmax = max_symbol(*d);
    if (d->dtau * tmax > 1.95)
        return fail(ITSE_EUNSTABLE, "dtau * max T(k) = %.4f > 1.95 (step map would amplify the highest modes)",
                    d->dtau * tmax);

    itse_lattice *L = new itse_lattice();
    L->d = *d;
    if (d->complex_psi) L->d.nstates = 2;  // Re psi and Im psi
    L->stream = (hipStream_t)hip_stream;
    HIPCHK(hipGetDevice(&L->device));
    L->alloc = alloc;
    L->freefn = free_fn;
    L->alloc_user = alloc_user;
    L->variant = schedule_variant_for(d->n, d->precision, L->d.nstates);
    L->sched = prec_schedule(d->n, d->precision, L->variant);
    if (d->kin == ITSE_KIN_FDTD)
        L->sched.nb_rows = d->precision == ITSE_FP32 ? Launch<float>::fdtd_blocks(d->n)
                                                     : Launch<double>::fdtd_blocks(d->n);
    const int n = d->n, K = L->d.nstates;
    const size_t w = real_bytes(d->precision);
    const size_t n3 = (size_t)n * n * n;
    const size_t spec = spec_bytes(n, d->precision);
    auto cleanup = [&](itse_status st) {
        lat_free_all(L);
        delete L;
        return st;
    };
    LatDev &H = L->host;
    std::memset(&H, 0, sizeof(H));
    H.n = n;
    H.nstates = K;
    H.kin = d->kin;
    H.sub = d->subtract_rest_mass ? 1 : 0;
    H.center = d->center;
    H.prec = d->precision;
    H.a = d->a;
    H.mass = d->mass;
    H.dtau = d->dtau;
    H.h = 0.5 * d->dtau;
    for (int i = 0; i < K; ++i) {
        H.ub[0][i] = lat_alloc(L, n3 * w);
        H.ub[1][i] = lat_alloc(L, n3 * w);
        H.spec[i] = lat_alloc(L, spec);
        if (!H.ub[0][i] || !H.ub[1][i] || !H.spec[i]) return cleanup(fail(ITSE_ENOMEM, "state buffers (%zu bytes)", n3 * w));
    }
    H.v = lat_alloc(L, n3 * w);
    L->tmp = lat_alloc(L, n3 * w);
    H.nb_rows = L->sched.nb_rows;
    H.nb_cols = L->sched.nb_cols;
    H.nb_proj = L->sched.nb_proj;
    H.nb_gram = L->sched.nb_gram;
    H.pg_chunks = pg_chunks(n);
    H.part_rows = (double *)lat_alloc(L, (size_t)MAXK * H.nb_rows * NQR * 8);
    H.part_cols = (double *)lat_alloc(L, (size_t)MAXK * H.nb_cols * NQC * 8);
    H.part_proj = (double *)lat_alloc(L, (size_t)MAXK * H.nb_proj * 8);
    H.part_gram = (double *)lat_alloc(L, (size_t)H.nb_gram * (MAXK * (MAXK + 1) / 2) * 8);
    H.hist = (ObsDev *)lat_alloc(L, (size_t)HIST_CAP * MAXK * sizeof(ObsDev));
    if (d->complex_psi) {
        H.cplx = 1;
        H.nb_cplx = d->kin == ITSE_KIN_FDTD ? flat_blocks(n) : H.nb_rows;
        H.vi = lat_alloc(L, n3 * w);
        H.kbuf = lat_alloc(L, 2 * n3 * w);
        H.part_cplx = (double *)lat_alloc(L, (size_t)H.nb_cplx * NQX * 8);
        if (!H.vi || !H.kbuf || !H.part_cplx) return cleanup(fail(ITSE_ENOMEM, "complex-state buffers"));
    }
    double *ktab = (double *)lat_alloc(L, (size_t)n * 8);
    L->dev = (LatDev *)lat_alloc(L, sizeof(LatDev));
    L->jobs_dev = (JobRef *)lat_alloc(L, sizeof(JobRef) * MAXK);
    L->lat_dev = (JobRef *)lat_alloc(L, sizeof(JobRef));
    L->tmp_ptrs_dev = (void **)lat_alloc(L, sizeof(void *) * MAXK);
    if (!H.v || !L->tmp || !H.part_rows || !H.part_cols || !H.part_proj || !H.part_gram || !H.hist || !ktab ||
        !L->dev || !L->jobs_dev || !L->lat_dev || !L->tmp_ptrs_dev)
        return cleanup(fail(ITSE_ENOMEM, "lattice buffers"));
    H.ktab = ktab;
    void *tw = nullptr;
    itse_status st = twiddles(n, d->precision, &tw);
    if (st) return cleanup(st);
    H.tw = tw;
    H.ortho_every = 1;
    H.moments = 0;
    for (int i = 0; i < MAXK; ++i) {
        H.psign[i] = 0;
        H.paxes[i] = 7;
    }
    for (int j = 0; j < MAXK; ++j)
        for (int i = 0; i < MAXK; ++i) H.coef[j][i] = (i == j) ? 1.0 : 0.0;
    H.step = 0;
    H.error = 0;
    L->opts.ortho_every = 1;
    L->opts.moments = 0;
    for (int i = 0; i < MAXK; ++i) {
        L->opts.parity[i] = 0;
        L->opts.axes[i] = 7;
    }

    std::vector<double> tab;
    kinetic_axis_table(*d, tab);
    std::vector<JobRef> jobs(MAXK);
    std::vector<void *> tmps(MAXK, nullptr);
    for (int i = 0; i < MAXK; ++i) {
        jobs[i].lat = L->dev;
        jobs[i].state = i;
        jobs[i].pad_ = 0;
        tmps[i] = L->tmp;
    }
    JobRef lj{L->dev, 0, 0};
    auto s = L->stream;
#define CK(expr)                                                                                  \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return cleanup(fail(ITSE_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_))); \
    } while (0)
    CK(hipMemcpyAsync(ktab, tab.data(), n * 8, hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(L->jobs_dev, jobs.data(), sizeof(JobRef) * MAXK, hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(L->lat_dev, &lj, sizeof(JobRef), hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(L->tmp_ptrs_dev, tmps.data(), sizeof(void *) * MAXK, hipMemcpyHostToDevice, s));
    for (int i = 0; i < K; ++i) {
        CK(hipMemsetAsync(H.ub[0][i], 0, n3 * w, s));
        CK(hipMemsetAsync(H.ub[1][i], 0, n3 * w, s));
    }
    CK(hipMemsetAsync(H.v, 0, n3 * w, s));
    if (H.vi) CK(hipMemsetAsync(H.vi, 0, n3 * w, s));
    CK(hipMemsetAsync(H.hist, 0, (size_t)HIST_CAP * MAXK * sizeof(ObsDev), s));
    CK(hipMemcpyAsync(L->dev, &H, sizeof(LatDev), hipMemcpyHostToDevice, s));
    CK(hipStreamSynchronize(s));
#undef CK
    *out = L;
    return ITSE_OK;
}

extern "C" itse_status itse_destroy(itse_lattice *L) {
    if (!L) return ITSE_OK;
    (void)hipStreamSynchronize(L->stream);
    if (L->graph1) (void)hipGraphExecDestroy(L->graph1);
    if (L->graphN) (void)hipGraphExecDestroy(L->graphN);
    if (L->cap_stream) (void)hipStreamDestroy(L->cap_stream);
    if (L->shadow) itse_destroy(L->shadow);
    if (L->snapx) itse_destroy(L->snapx);
    lat_free_all(L);
    delete L;
    return ITSE_OK;
}

extern "C" itse_status itse_set_stream(itse_lattice *L, void *stream) {
    if (!L) return fail(ITSE_EINVAL, "null lattice");
    HIPCHK(hipStreamSynchronize(L->stream));
    L->stream = (hipStream_t)stream;
    return ITSE_OK;
}

namespace itse {
// Copy N^3 values of dtype `dtype` from host/device into a lattice buffer of the lattice precision.
static itse_status copy_in(itse_lattice *L, const void *src, int dtype, int on_device, void *dst) {
    const size_t n3 = (size_t)L->d.n * L->d.n * L->d.n;
    const int prec = L->d.precision;
    const size_t sw = dtype == ITSE_DTYPE_F32 ? 4 : 8;
    const bool same = (dtype == ITSE_DTYPE_F32) == (prec == ITSE_FP32);
    if (same) {
        HIPCHK(hipMemcpyAsync(dst, src, n3 * sw, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                              L->stream));
        if (!on_device) HIPCHK(hipStreamSynchronize(L->stream));
        return ITSE_OK;
    }
    const void *dsrc = src;
    void *staging = nullptr;
    if (!on_device) {
        staging = L->stage_buf(n3 * sw);
        if (!staging) return fail(ITSE_ENOMEM, "staging buffer");
        HIPCHK(hipMemcpyAsync(staging, src, n3 * sw, hipMemcpyHostToDevice, L->stream));
        dsrc = staging;
    }
    hipError_t e = prec == ITSE_FP32 ? Launch<float>::convert_in(dsrc, dtype, dst, n3, L->stream)
                                     : Launch<double>::convert_in(dsrc, dtype, dst, n3, L->stream);
    if (e != hipSuccess) return fail(ITSE_EDEVICE, "convert: %s", hipGetErrorString(e));
    if (!on_device) HIPCHK(hipStreamSynchronize(L->stream));
    return ITSE_OK;
}
}  // namespace itse

void *itse_lattice::stage_buf(size_t bytes) {
    if (staging && staging_bytes >= bytes) return staging;
    staging = itse::lat_alloc(this, bytes);
    staging_bytes = staging ? bytes : 0;
    return staging;
}

extern "C" itse_status itse_set_potential(itse_lattice *L, const void *v, int dtype, int on_device) {
    if (!L || !v) return fail(ITSE_EINVAL, "null argument");
    if (dtype != ITSE_DTYPE_F32 && dtype != ITSE_DTYPE_F64) return fail(ITSE_EINVAL, "dtype");
    const size_t n3 = (size_t)L->d.n * L->d.n * L->d.n;
    if (!on_device) {
        double vmin = 0.0;
        for (size_t s = 0; s < n3; ++s) {
            const double x = dtype == ITSE_DTYPE_F32 ? (double)((const float *)v)[s] : ((const double *)v)[s];
            if (!std::isfinite(x)) return fail(ITSE_ENONFINITE, "potential has a non-finite value at site %zu", s);
            if (s == 0 || x < vmin) vmin = x;
        }
        if (1.0 + 0.5 * L->d.dtau * vmin <= 0.0)
            return fail(ITSE_EUNSTABLE, "1 + dtau min(V)/2 = %.4g <= 0", 1.0 + 0.5 * L->d.dtau * vmin);
    }
    itse_status st = copy_in(L, v, dtype, on_device, L->host.v);
    if (st) return st;
    if (on_device) {
        hipError_t e = launch_check_potential(L->dev, L->d.precision, L->stream);
        if (e != hipSuccess) return fail(ITSE_EDEVICE, "check_potential: %s", hipGetErrorString(e));
    }
    return ITSE_OK;
}

extern "C" itse_status itse_set_potential_imag(itse_lattice *L, const void *v, int dtype, int on_device) {
    if (!L || !v) return fail(ITSE_EINVAL, "null argument");
    if (!L->host.cplx) return fail(ITSE_ESTATE, "imaginary potential on a lattice of real states");
    if (dtype != ITSE_DTYPE_F32 && dtype != ITSE_DTYPE_F64) return fail(ITSE_EINVAL, "dtype");
    const size_t n3 = (size_t)L->d.n * L->d.n * L->d.n;
    if (!on_device)
        for (size_t s = 0; s < n3; ++s) {
            const double x = dtype == ITSE_DTYPE_F32 ? (double)((const float *)v)[s] : ((const double *)v)[s];
            if (!std::isfinite(x)) return fail(ITSE_ENONFINITE, "Im V has a non-finite value at site %zu", s);
        }
    return copy_in(L, v, dtype, on_device, L->host.vi);
}

extern "C" itse_status itse_set_state(itse_lattice *L, int i, const void *psi, int dtype, int on_device) {
    if (!L || !psi) return fail(ITSE_EINVAL, "null argument");
    if (i < 0 || i >= L->d.nstates) return fail(ITSE_EINVAL, "state index %d", i);
    if (dtype != ITSE_DTYPE_F32 && dtype != ITSE_DTYPE_F64) return fail(ITSE_EINVAL, "dtype");
    itse_status st = materialise(L);
    if (st) return st;
    return copy_in(L, psi, dtype, on_device, cur_state(L, i));
}

extern "C" itse_status itse_get_state(itse_lattice *L, int i, void *out, int dtype, int on_device) {
    if (!L || !out) return fail(ITSE_EINVAL, "null argument");
    if (i < 0 || i >= L->d.nstates) return fail(ITSE_EINVAL, "state index %d", i);
    if (dtype != ITSE_DTYPE_F32 && dtype != ITSE_DTYPE_F64) return fail(ITSE_EINVAL, "dtype");
    const size_t n3 = (size_t)L->d.n * L->d.n * L->d.n;
    const int prec = L->d.precision;
    hipError_t e = prec == ITSE_FP32 ? Launch<float>::combine(L->d.n, L->jobs_dev + i, 1, L->tmp_ptrs_dev, L->stream)
                                     : Launch<double>::combine(L->d.n, L->jobs_dev + i, 1, L->tmp_ptrs_dev, L->stream);
    if (e != hipSuccess) return fail(ITSE_EDEVICE, "combine: %s", hipGetErrorString(e));
    const size_t dw = dtype == ITSE_DTYPE_F32 ? 4 : 8;
    const bool same = (dtype == ITSE_DTYPE_F32) == (prec == ITSE_FP32);
    const void *src = L->tmp;
    if (!same) {
        void *stg = L->stage_buf(n3 * dw);
        if (!stg) return fail(ITSE_ENOMEM, "staging buffer");
        e = prec == ITSE_FP32 ? Launch<float>::convert_out(L->tmp, stg, dtype, n3, L->stream)
                              : Launch<double>::convert_out(L->tmp, stg, dtype, n3, L->stream);
        if (e != hipSuccess) return fail(ITSE_EDEVICE, "convert: %s", hipGetErrorString(e));
        src = stg;
    }
    HIPCHK(hipMemcpyAsync(out, src, n3 * dw, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, L->stream));
    if (!on_device) HIPCHK(hipStreamSynchronize(L->stream));
    return ITSE_OK;
}

extern "C" itse_status itse_set_step_opts(itse_lattice *L, const itse_step_opts *o) {
    if (!L || !o) return fail(ITSE_EINVAL, "null argument");
    if (o->ortho_every < 0) return fail(ITSE_EINVAL, "ortho_every < 0");
    for (int i = 0; i < MAXK; ++i) {
        if (o->parity[i] < -1 || o->parity[i] > 1) return fail(ITSE_EINVAL, "parity[%d] = %d", i, o->parity[i]);
        if (o->parity[i] != 0 && (o->axes[i] < 1 || o->axes[i] > 7))
            return fail(ITSE_EINVAL, "axes[%d] = %d", i, o->axes[i]);
    }
    L->opts = *o;
    L->host.ortho_every = o->ortho_every;
    L->host.moments = o->moments ? 1 : 0;
    // a complex lattice: never orthogonalised; parity[0] / axes[0] project both parts
    itse_step_opts eff = *o;
    if (L->host.cplx) {
        L->host.ortho_every = 0;
        for (int i = 1; i < MAXK; ++i) {
            eff.parity[i] = i == 1 ? o->parity[0] : 0;
            eff.axes[i] = i == 1 ? o->axes[0] : 7;
        }
    }
    int mode = 0, paxes = 0;
    for (int i = 0; i < MAXK; ++i) {
        L->host.psign[i] = i < L->d.nstates ? eff.parity[i] : 0;
        L->host.paxes[i] = eff.parity[i] ? eff.axes[i] : 7;
        if (L->host.psign[i] != 0) {
            if (mode == 0) {
                mode = 1;
                paxes = L->host.paxes[i];
            } else if (L->host.paxes[i] != paxes) {
                mode = 2;
            }
        }
    }
    L->host.proj_mode = mode;
    L->host.proj_axes = paxes;
    return upload_opts(L);
}

namespace itse {
static bool graphs_enabled() {
    const char *e = getenv("ITSE_GRAPHS");
    return !(e && e[0] == '0');
}

// Capture `nsteps` step sequences of group set `groups` into an executable graph.
itse_status capture_steps(hipStream_t cap, const std::vector<Group> &groups, int nsteps,
                          std::vector<hipStream_t> &branch, hipGraphExec_t *out) {
    HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    std::vector<hipEvent_t> evs;
    if (groups.size() == 1) {
        for (int s = 0; s < nsteps && err == hipSuccess; ++s) err = enqueue_step(groups[0], cap);
    } else {
        // fork: each group on its own branch stream, joined at the end
        hipEvent_t fork = nullptr;
        err = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        if (err == hipSuccess) {
            evs.push_back(fork);
            err = hipEventRecord(fork, cap);
        }
        for (size_t g = 0; g < groups.size() && err == hipSuccess; ++g) {
            hipStream_t bs = branch[g % branch.size()];
            err = hipStreamWaitEvent(bs, fork, 0);
            for (int s = 0; s < nsteps && err == hipSuccess; ++s) err = enqueue_step(groups[g], bs);
            hipEvent_t join = nullptr;
            if (err == hipSuccess) err = hipEventCreateWithFlags(&join, hipEventDisableTiming);
            if (err == hipSuccess) {
                evs.push_back(join);
                err = hipEventRecord(join, bs);
            }
            if (err == hipSuccess) err = hipStreamWaitEvent(cap, join, 0);
        }
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cap, &graph);
    for (auto ev : evs) (void)hipEventDestroy(ev);
    if (err != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(ITSE_EDEVICE, "launch during capture: %s", hipGetErrorString(err));
    }
    if (e2 != hipSuccess) return fail(ITSE_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    hipError_t e3 = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return fail(ITSE_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e3));
    return ITSE_OK;
}
}  // namespace itse

extern "C" itse_status itse_step(itse_lattice *L, int nsteps, const itse_step_opts *opts) {
    if (!L) return fail(ITSE_EINVAL, "null lattice");
    if (nsteps < 0) return fail(ITSE_EINVAL, "nsteps < 0");
    if (opts) {
        itse_status st = itse_set_step_opts(L, opts);
        if (st) return st;
    }
    if (nsteps == 0) return ITSE_OK;
    Group g = single_group(L);
    if (!graphs_enabled()) {
        for (int s = 0; s < nsteps; ++s) {
            hipError_t e = enqueue_step(g, L->stream);
            if (e != hipSuccess) return fail(ITSE_EDEVICE, "step launch: %s", hipGetErrorString(e));
        }
        L->steps_host += nsteps;
        return ITSE_OK;
    }
    if (!L->cap_stream) HIPCHK(hipStreamCreateWithFlags(&L->cap_stream, hipStreamNonBlocking));
    if (L->graph_needs != g.needs) {
        // the options changed which passes a step launches: capture again
        HIPCHK(hipStreamSynchronize(L->stream));
        if (L->graph1) HIPCHK(hipGraphExecDestroy(L->graph1));
        if (L->graphN) HIPCHK(hipGraphExecDestroy(L->graphN));
        L->graph1 = L->graphN = nullptr;
        L->graph_needs = g.needs;
    }
    std::vector<hipStream_t> br{L->cap_stream};
    const int chunk = ITSE_GRAPH_CHUNK;
    if (nsteps >= chunk && !L->graphN) {
        itse_status st = capture_steps(L->cap_stream, {g}, chunk, br, &L->graphN);
        if (st) return st;
    }
    if (!L->graph1) {
        itse_status st = capture_steps(L->cap_stream, {g}, 1, br, &L->graph1);
        if (st) return st;
    }
    int left = nsteps;
    while (left >= chunk) {
        HIPCHK(hipGraphLaunch(L->graphN, L->stream));
        left -= chunk;
    }
    while (left > 0) {
        HIPCHK(hipGraphLaunch(L->graph1, L->stream));
        --left;
    }
    L->steps_host += nsteps;
    return ITSE_OK;
}

extern "C" itse_status itse_evaluate(itse_lattice *L, int moments) {
    if (!L) return fail(ITSE_EINVAL, "null lattice");
    const int saved = L->host.moments;
    L->host.moments = moments ? 1 : 0;
    itse_status st = upload_field(L, offsetof(LatDev, moments), sizeof(int));
    if (st) return st;
    hipError_t e = enqueue_eval(single_group(L), L->stream);
    if (e != hipSuccess) return fail(ITSE_EDEVICE, "evaluate launch: %s", hipGetErrorString(e));
    L->host.moments = saved;
    return upload_field(L, offsetof(LatDev, moments), sizeof(int));
}

extern "C" itse_status itse_observe(itse_lattice *L, int i, itse_obs *out) {
    if (!L || !out) return fail(ITSE_EINVAL, "null argument");
    if (i < 0 || i >= (L->host.cplx ? 1 : L->d.nstates)) return fail(ITSE_EINVAL, "state index %d", i);
    ObsDev o;
    HIPCHK(hipMemcpyAsync(&o, (char *)L->dev + offsetof(LatDev, obs) + i * sizeof(ObsDev), sizeof(ObsDev),
                          hipMemcpyDeviceToHost, L->stream));
    itse_status st = check_device_error(L);
    static_assert(sizeof(ObsDev) == sizeof(itse_obs), "observable layout");
    std::memcpy(out, &o, sizeof(o));
    return st;
}

extern "C" itse_status itse_history(itse_lattice *L, int count, itse_obs *out) {
    if (!L || (!out && count > 0)) return fail(ITSE_EINVAL, "null argument");
    if (count < 0 || count > HIST_CAP || count > L->steps_host)
        return fail(ITSE_EINVAL, "count %d (steps taken %lld, capacity %d)", count, L->steps_host, HIST_CAP);
    const int K = L->host.cplx ? 1 : L->d.nstates;  // records per step
    std::vector<ObsDev> all((size_t)HIST_CAP * MAXK);
    HIPCHK(hipMemcpyAsync(all.data(), L->host.hist, all.size() * sizeof(ObsDev), hipMemcpyDeviceToHost, L->stream));
    itse_status st = check_device_error(L);
    const long long last = L->steps_host;  // steps 0..last-1 recorded
    for (int c = 0; c < count; ++c) {
        const long long step = last - count + c;
        const size_t slot = (size_t)(step % HIST_CAP);
        for (int i = 0; i < K; ++i) std::memcpy(&out[(size_t)c * K + i], &all[slot * MAXK + i], sizeof(itse_obs));
    }
    return st;
}

extern "C" long long itse_step_count(const itse_lattice *L) { return L ? L->steps_host : -1; }

extern "C" itse_status itse_sync(itse_lattice *L) {
    if (!L) return fail(ITSE_EINVAL, "null lattice");
    return check_device_error(L);
}

namespace itse {
// Sum per-block partials on the host in the same fixed order the device uses.
static double host_fixed_sum(const std::vector<double> &p, int count, int stride, int off) {
    std::vector<double> red(NT, 0.0);
    for (int t = 0; t < NT; ++t)
        for (int b = t; b < count; b += NT) red[t] += p[(size_t)b * stride + off];
    for (int s = NT / 2; s > 0; s >>= 1)
        for (int t = 0; t < s; ++t) red[t] += red[t + s];
    return red[0];
}

static itse_status gram_host(itse_lattice *L, double G[MAXK][MAXK]) {
    constexpr int NG = MAXK * (MAXK + 1) / 2;
    const int K = L->d.nstates;
    hipError_t e = L->d.precision == ITSE_FP32
                       ? Launch<float>::project_gram(L->d.n, K, L->lat_dev, 1, 1, 0, L->stream)
                       : Launch<double>::project_gram(L->d.n, K, L->lat_dev, 1, 1, 0, L->stream);
    if (e != hipSuccess) return fail(ITSE_EDEVICE, "gram: %s", hipGetErrorString(e));
    std::vector<double> part((size_t)L->host.nb_gram * NG);
    HIPCHK(hipMemcpyAsync(part.data(), L->host.part_gram, part.size() * 8, hipMemcpyDeviceToHost, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
    for (int l = 0; l < K; ++l)
        for (int j = 0; j <= l; ++j) {
            const double s = host_fixed_sum(part, L->host.nb_gram, NG, l * (l + 1) / 2 + j);
            G[j][l] = G[l][j] = s;
        }
    return ITSE_OK;
}
}  // namespace itse

extern "C" itse_status itse_orthogonalise(itse_lattice *L, int i) {
    if (L && L->host.cplx) return fail(ITSE_ESTATE, "%s: real states only", "itse_orthogonalise");
    if (!L) return fail(ITSE_EINVAL, "null lattice");
    if (i < 0 || i >= L->d.nstates) return fail(ITSE_EINVAL, "state index %d", i);
    itse_status st = materialise(L);
    if (st) return st;
    double G[MAXK][MAXK] = {};
    if (L->d.nstates == 1) {
        // one state: only the norm
        G[0][0] = 0.0;
    }
    // the Gram kernel needs nstates >= 2; for one state compute the norm via a forced projection-free sum
    if (L->d.nstates >= 2) {
        st = gram_host(L, G);
        if (st) return st;
    } else {
        st = norm_host(L, 0, &G[0][0]);
        if (st) return st;
    }
    // Cholesky of the leading (i+1)x(i+1) block; column i of R^{-1}
    double Rm[MAXK][MAXK] = {};
    for (int j = 0; j <= i; ++j)
        for (int c = j; c <= i; ++c) {
            double s = G[j][c];
            for (int l = 0; l < j; ++l) s -= Rm[l][j] * Rm[l][c];
            if (c == j) {
                if (!(s > 0.0)) return fail(ITSE_ENONFINITE, "state %d lies in the span of the lower states", i);
                Rm[j][j] = std::sqrt(s);
            } else {
                Rm[j][c] = s / Rm[j][j];
            }
        }
    double M[MAXK] = {};
    M[i] = 1.0 / Rm[i][i];
    for (int j = i - 1; j >= 0; --j) {
        double s = 0.0;
        for (int l = j + 1; l <= i; ++l) s += Rm[j][l] * M[l];
        M[j] = -s / Rm[j][j];
    }
    for (int j = 0; j < MAXK; ++j) L->host.coef[j][i] = j <= i ? M[j] : 0.0;
    return upload_field(L, offsetof(LatDev, coef), sizeof(L->host.coef));
}

namespace itse {
itse_status norm_host(itse_lattice *L, int i, double *out) {
    // sum of squares of u_i via the projection kernel's partials with sign +1 on axes 0
    // is not available; use the combine-free path: copy to host and sum in FP64.
    const size_t n3 = (size_t)L->d.n * L->d.n * L->d.n;
    std::vector<double> h(n3);
    itse_status st = itse_get_state(L, i, h.data(), ITSE_DTYPE_F64, 0);
    if (st) return st;
    double acc = 0.0;
    for (size_t s = 0; s < n3; ++s) acc += h[s] * h[s];
    *out = acc;
    return ITSE_OK;
}
}  // namespace itse

extern "C" itse_status itse_project_parity(itse_lattice *L, int i, int sign, int axes, double *weight) {
    if (L && L->host.cplx) return fail(ITSE_ESTATE, "%s: real states only", "itse_project_parity");
    if (!L) return fail(ITSE_EINVAL, "null lattice");
    if (i < 0 || i >= L->d.nstates) return fail(ITSE_EINVAL, "state index %d", i);
    if (sign != 1 && sign != -1) return fail(ITSE_EINVAL, "sign must be +1 or -1");
    if (axes < 1 || axes > 7) return fail(ITSE_EINVAL, "axes must be in 1..7");
    itse_status st = materialise(L);
    if (st) return st;
    double before = 0.0;
    st = norm_host(L, i, &before);
    if (st) return st;
    hipError_t e = L->d.precision == ITSE_FP32
                       ? Launch<float>::project(L->d.n, L->jobs_dev + i, 1, sign, axes, 0, L->stream)
                       : Launch<double>::project(L->d.n, L->jobs_dev + i, 1, sign, axes, 0, L->stream);
    if (e != hipSuccess) return fail(ITSE_EDEVICE, "project: %s", hipGetErrorString(e));
    std::vector<double> part(L->host.nb_proj);
    HIPCHK(hipMemcpyAsync(part.data(), L->host.part_proj + (size_t)i * L->host.nb_proj, part.size() * 8,
                          hipMemcpyDeviceToHost, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
    const double after = host_fixed_sum(part, L->host.nb_proj, 1, 0);
    if (weight) *weight = before > 0 ? after / before : 0.0;
    if (!(after > 0.0)) return fail(ITSE_ENONFINITE, "projection of state %d vanishes", i);
    for (int j = 0; j < MAXK; ++j) L->host.coef[j][i] = (j == i) ? 1.0 / std::sqrt(after) : 0.0;
    return upload_field(L, offsetof(LatDev, coef), sizeof(L->host.coef));
}

extern "C" itse_status itse_apply_kinetic(itse_lattice *L, int i, void *out) {
    if (!L || !out) return fail(ITSE_EINVAL, "null argument");
    if (i < 0 || i >= L->d.nstates) return fail(ITSE_EINVAL, "state index %d", i);
    L->host.kout = out;
    itse_status st = upload_field(L, offsetof(LatDev, kout), sizeof(void *));
    if (st) return st;
    Group g = state_group(L, i);
    hipError_t e = L->d.precision == ITSE_FP32 ? seq_forward_kin<float>(g, INV_KOUT, L->stream)
                                               : seq_forward_kin<double>(g, INV_KOUT, L->stream);
    if (e != hipSuccess) return fail(ITSE_EDEVICE, "kinetic launch: %s", hipGetErrorString(e));
    return ITSE_OK;
}

extern "C" itse_status itse_spectrum(itse_lattice *L, int i, void *out) {
    if (!L || !out) return fail(ITSE_EINVAL, "null argument");
    if (i < 0 || i >= L->d.nstates) return fail(ITSE_EINVAL, "state index %d", i);
    Group g = state_group(L, i);
    hipError_t e;
    if (L->d.precision == ITSE_FP32) {
        e = Launch<float>::plane_fwd(g.n, g.variant, g.kmax, g.jobs, 1, L->stream);
        if (e == hipSuccess) e = Launch<float>::columns(g.n, g.variant, COL_FWD, 0, g.jobs, 1, out, L->stream);
    } else {
        e = Launch<double>::plane_fwd(g.n, g.variant, g.kmax, g.jobs, 1, L->stream);
        if (e == hipSuccess) e = Launch<double>::columns(g.n, g.variant, COL_FWD, 0, g.jobs, 1, out, L->stream);
    }
    if (e != hipSuccess) return fail(ITSE_EDEVICE, "spectrum launch: %s", hipGetErrorString(e));
    return ITSE_OK;
}

extern "C" itse_status itse_polish(itse_lattice *L, int i, itse_obs *out) {
    if (L && L->host.cplx) return fail(ITSE_ESTATE, "%s: real states only", "itse_polish");
    if (!L || !out) return fail(ITSE_EINVAL, "null argument");
    if (i < 0 || i >= L->d.nstates) return fail(ITSE_EINVAL, "state index %d", i);
    if (L->d.precision == ITSE_FP64) {
        itse_status st = itse_evaluate(L, 1);
        if (st) return st;
        return itse_observe(L, i, out);
    }
    if (!L->shadow) {
        itse_desc d = L->d;
        d.precision = ITSE_FP64;
        d.nstates = 1;
        itse_status st = itse_create(&d, L->stream, L->alloc, L->freefn, L->alloc_user, &L->shadow);
        if (st) return st;
    }
    itse_lattice *S = L->shadow;
    itse_set_stream(S, L->stream);
    // potential and state: FP32 values widened exactly to FP64
    itse_status st = itse_set_potential(S, L->host.v, ITSE_DTYPE_F32, 1);
    if (st) return st;
    hipError_t e = Launch<float>::combine(L->d.n, L->jobs_dev + i, 1, L->tmp_ptrs_dev, L->stream);
    if (e != hipSuccess) return fail(ITSE_EDEVICE, "combine: %s", hipGetErrorString(e));
    st = itse_set_state(S, 0, L->tmp, ITSE_DTYPE_F32, 1);
    if (st) return st;
    st = itse_evaluate(S, 1);
    if (st) return st;
    return itse_observe(S, 0, out);
}

// ------------------------------------------------------------------------------------
// Analysis of a state (box normalisation, radius, parity weights; momentum space)
// ------------------------------------------------------------------------------------
static double *ana_scratch(itse_lattice *L, size_t doubles) {
    const size_t bytes = doubles * sizeof(double);
    if (L->ana && L->ana_bytes >= bytes) return L->ana;
    L->ana = (double *)lat_alloc(L, bytes);
    L->ana_bytes = L->ana ? bytes : 0;
    return L->ana;
}

// The analysis kernels (partial sums per workgroup, then their fixed-order sum)
// into the workspace buf of at least analyse_doubles(n) doubles; results to out.
static size_t analyse_doubles(const itse_lattice *L) {
    const int n = L->d.n;
    return (L->d.precision == ITSE_FP32 ? Launch<float>::analyse_parts(n) : Launch<double>::analyse_parts(n)) + NAQ;
}

static itse_status analyse_checks(itse_lattice *L, int i, double min_sep_edge, itse_analysis *out,
                                  const char *who) {
    if (L && L->host.cplx) return fail(ITSE_ESTATE, "%s: real states only", who);
    if (!L || !out) return fail(ITSE_EINVAL, "null argument");
    if (i < 0 || i >= L->d.nstates) return fail(ITSE_EINVAL, "state index %d", i);
    if (!(min_sep_edge >= 0.0 && min_sep_edge < 1.0)) return fail(ITSE_EINVAL, "min_sep_edge = %g", min_sep_edge);
    return ITSE_OK;
}

static itse_status analyse_into(itse_lattice *L, int i, double min_sep_edge, double *buf, itse_analysis *out) {
    const int n = L->d.n;
    const size_t np = analyse_doubles(L) - NAQ;
    const double half = (1.0 - min_sep_edge) * n * L->d.a / 2.0;
    hipError_t e = L->d.precision == ITSE_FP32
                       ? Launch<float>::analyse(n, L->jobs_dev + i, half, buf, buf + np, L->stream)
                       : Launch<double>::analyse(n, L->jobs_dev + i, half, buf, buf + np, L->stream);
    if (e != hipSuccess) return fail(ITSE_EDEVICE, "analyse: %s", hipGetErrorString(e));
    double q[NAQ];
    HIPCHK(hipMemcpyAsync(q, buf + np, sizeof q, hipMemcpyDeviceToHost, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
    if (!(q[NA_NORM] > 0.0) || !std::isfinite(q[NA_NORM])) return fail(ITSE_ENONFINITE, "no weight in the box");
    out->box_norm2 = q[NA_NORM];
    out->rho_box = q[NA_RHO] / q[NA_NORM];
    out->w_plus = q[NA_PPLUS] / q[NA_NORM];
    out->w_minus = q[NA_PMINUS] / q[NA_NORM];
    out->w_minus_axis[0] = q[NA_PE1] / q[NA_NORM];
    out->w_minus_axis[1] = q[NA_PE2] / q[NA_NORM];
    out->w_minus_axis[2] = q[NA_PE3] / q[NA_NORM];
    return ITSE_OK;
}

extern "C" itse_status itse_analyse(itse_lattice *L, int i, double min_sep_edge, itse_analysis *out) {
    itse_status st = analyse_checks(L, i, min_sep_edge, out, "itse_analyse");
    if (st) return st;
    double *buf = ana_scratch(L, analyse_doubles(L));
    if (!buf) return fail(ITSE_ENOMEM, "analysis sums");
    return analyse_into(L, i, min_sep_edge, buf, out);
}

// ------------------------------------------------------------------------------------
// The analysis without allocation: its workspace is a file-scope device array,
// one copy per GPU, sized for the largest supported lattice (n = 256: 256 x 8
// workgroups x 7 partial sums + 7 totals, 112 KiB).  Every kernel writes each
// slot it later reads (the partial sums, then the totals), so nothing needs
// clearing between calls.  Calls on one GPU share the array: calls that overlap
// on one GPU (different streams, or threads) race and must be ordered by the
// caller.
// ------------------------------------------------------------------------------------
constexpr size_t ANA_SCRATCH_DOUBLES = (size_t)256 * ANA_CHUNKS * NAQ + NAQ;
static __device__ __align__(256) double scratch[ANA_SCRATCH_DOUBLES];

static std::mutex g_scratch_mu;
static std::map<int, double *> g_scratch_ptr;  // device -> address of `scratch` on it

// Address of the workspace on the lattice's device, looked up once per device with
// that device current (the name of the array is a host-side stand-in, not a device
// address).
static itse_status scratch_on(int device, double **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return ITSE_OK;
    }
    int cur = 0;
    HIPCHK(hipGetDevice(&cur));
    if (cur != device) HIPCHK(hipSetDevice(device));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) HIPCHK(hipSetDevice(cur));
    if (e != hipSuccess || !p) return fail(ITSE_EDEVICE, "workspace address on device %d: %s", device,
                                           hipGetErrorString(e));
    g_scratch_ptr[device] = (double *)p;
    *out = (double *)p;
    return ITSE_OK;
}

extern "C" itse_status itse_analyse_noalloc(itse_lattice *L, int i, double min_sep_edge, itse_analysis *out) {
    itse_status st = analyse_checks(L, i, min_sep_edge, out, "itse_analyse_noalloc");
    if (st) return st;
    const size_t need = analyse_doubles(L);
    if (need > ANA_SCRATCH_DOUBLES)
        return fail(ITSE_EINVAL, "itse_analyse_noalloc: n = %d needs %zu workspace doubles, the limit is %zu",
                    L->d.n, need, ANA_SCRATCH_DOUBLES);
    double *buf = nullptr;
    st = scratch_on(L->device, &buf);
    if (st) return st;
    return analyse_into(L, i, min_sep_edge, buf, out);
}

extern "C" itse_status itse_momentum_radial(itse_lattice *L, int i, int nbins, double *count, double *p, double *psi,
                                            double *y) {
    if (L && L->host.cplx) return fail(ITSE_ESTATE, "itse_momentum_radial: real states only");
    if (!L) return fail(ITSE_EINVAL, "null lattice");
    if (i < 0 || i >= L->d.nstates) return fail(ITSE_EINVAL, "state index %d", i);
    if (nbins < 1 || nbins > MOM_MAXBINS) return fail(ITSE_EINVAL, "nbins = %d (1..%d)", nbins, MOM_MAXBINS);
    const int n = L->d.n;
    if (!L->mom_spec) {
        const size_t h = (size_t)n / 2 + 1;
        L->mom_spec = lat_alloc(L, (size_t)n * n * h * 2 * real_bytes(L->d.precision));
        if (!L->mom_spec) return fail(ITSE_ENOMEM, "momentum-space spectrum");
    }
    itse_status st = itse_spectrum(L, i, L->mom_spec);
    if (st) return st;
    const size_t w = 3 * (size_t)nbins + 1, np = (size_t)n * w;
    double *buf = ana_scratch(L, np + w);
    if (!buf) return fail(ITSE_ENOMEM, "momentum histograms");
    hipError_t e = L->d.precision == ITSE_FP32
                       ? Launch<float>::momentum_bins(n, L->mom_spec, nbins, buf, buf + np, L->stream)
                       : Launch<double>::momentum_bins(n, L->mom_spec, nbins, buf, buf + np, L->stream);
    if (e != hipSuccess) return fail(ITSE_EDEVICE, "momentum bins: %s", hipGetErrorString(e));
    std::vector<double> q(w);
    HIPCHK(hipMemcpyAsync(q.data(), buf + np, w * sizeof(double), hipMemcpyDeviceToHost, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
    const double pi = 3.14159265358979323846;
    const double dp = 2.0 * pi / (n * L->d.a);
    const double total = q[3 * nbins];
    if (!(total > 0.0) || !std::isfinite(total)) return fail(ITSE_ENONFINITE, "zero or non-finite spectrum");
    const double scale = 1.0 / std::sqrt(dp * dp * dp * total);
    for (int b = 0; b < nbins; ++b) {
        const double c = q[3 * b];
        const double pm = c > 0.0 ? q[3 * b + 1] / c * dp : 0.0;
        const double fm = c > 0.0 ? q[3 * b + 2] / c * scale : 0.0;
        if (count) count[b] = c;
        if (p) p[b] = pm;
        if (psi) psi[b] = fm;
        if (y) y[b] = std::sqrt(4.0 * pi) * pm * fm;
    }
    return ITSE_OK;
}

// ------------------------------------------------------------------------------------
// Snapshot-overlap extraction of excited states (section "The iterative procedure")
// ------------------------------------------------------------------------------------
extern "C" itse_status itse_snapshot_push(itse_lattice *L) {
    if (L && L->host.cplx) return fail(ITSE_ESTATE, "%s: real states only", "itse_snapshot_push");
    if (!L) return fail(ITSE_EINVAL, "null lattice");
    const size_t n3 = (size_t)L->d.n * L->d.n * L->d.n;
    if (!L->snap[0]) {
        void *ptrs[ITSE_SNAPSHOTS];
        for (int k = 0; k < ITSE_SNAPSHOTS; ++k) {
            L->snap[k] = lat_alloc(L, n3 * real_bytes(L->d.precision));
            if (!L->snap[k]) return fail(ITSE_ENOMEM, "snapshot ring");
            ptrs[k] = L->snap[k];
        }
        L->snap_ptr_dev = (void **)lat_alloc(L, sizeof ptrs);
        if (!L->snap_ptr_dev) return fail(ITSE_ENOMEM, "snapshot ring");
        HIPCHK(hipMemcpyAsync(L->snap_ptr_dev, ptrs, sizeof ptrs, hipMemcpyHostToDevice, L->stream));
    }
    // the slot after the newest one (the oldest once the ring is full)
    const int slot = (L->snap_newest + 1) % ITSE_SNAPSHOTS;
    hipError_t e = L->d.precision == ITSE_FP32
                       ? Launch<float>::combine(L->d.n, L->jobs_dev, 1, L->snap_ptr_dev + slot, L->stream)
                       : Launch<double>::combine(L->d.n, L->jobs_dev, 1, L->snap_ptr_dev + slot, L->stream);
    if (e != hipSuccess) return fail(ITSE_EDEVICE, "snapshot: %s", hipGetErrorString(e));
    L->snap_newest = slot;
    L->snap_count = std::min(L->snap_count + 1, ITSE_SNAPSHOTS);
    return ITSE_OK;
}

extern "C" itse_status itse_snapshot_count(const itse_lattice *L, int *count) {
    if (!L || !count) return fail(ITSE_EINVAL, "null argument");
    *count = L->snap_count;
    return ITSE_OK;
}

extern "C" itse_status itse_snapshot_clear(itse_lattice *L) {
    if (!L) return fail(ITSE_EINVAL, "null lattice");
    L->snap_count = 0;
    L->snap_newest = -1;
    return ITSE_OK;
}

extern "C" itse_status itse_snapshot_extract(itse_lattice *L, itse_obs *out, int *n_out, void *states_out, int dtype,
                                             int on_device) {
    if (L && L->host.cplx) return fail(ITSE_ESTATE, "itse_snapshot_extract: real states only");
    if (!L || !out || !n_out) return fail(ITSE_EINVAL, "null argument");
    if (states_out && dtype != ITSE_DTYPE_F32 && dtype != ITSE_DTYPE_F64) return fail(ITSE_EINVAL, "dtype");
    const int ne = 1 + L->snap_count;
    // a lattice of the same description holding the current state and the
    // snapshots, newest first, as its states 0 .. ne-1
    if (L->snapx && L->snapx->d.nstates != ne) {
        itse_destroy(L->snapx);
        L->snapx = nullptr;
    }
    if (!L->snapx) {
        itse_desc d = L->d;
        d.nstates = ne;
        itse_status st = itse_create(&d, L->stream, L->alloc, L->freefn, L->alloc_user, &L->snapx);
        if (st) return st;
    }
    itse_lattice *X = L->snapx;
    itse_status st = itse_set_stream(X, L->stream);
    if (st) return st;
    const int wdt = L->d.precision == ITSE_FP32 ? ITSE_DTYPE_F32 : ITSE_DTYPE_F64;
    if ((st = itse_set_potential(X, L->host.v, wdt, 1))) return st;
    hipError_t e = L->d.precision == ITSE_FP32
                       ? Launch<float>::combine(L->d.n, L->jobs_dev, 1, L->tmp_ptrs_dev, L->stream)
                       : Launch<double>::combine(L->d.n, L->jobs_dev, 1, L->tmp_ptrs_dev, L->stream);
    if (e != hipSuccess) return fail(ITSE_EDEVICE, "combine: %s", hipGetErrorString(e));
    if ((st = itse_set_state(X, 0, L->tmp, wdt, 1))) return st;
    for (int k = 0; k < L->snap_count; ++k) {
        const int slot = ((L->snap_newest - k) % ITSE_SNAPSHOTS + ITSE_SNAPSHOTS) % ITSE_SNAPSHOTS;
        if ((st = itse_set_state(X, 1 + k, L->snap[slot], wdt, 1))) return st;
    }
    // Gram-Schmidt in that order: estimate e is snapshot e minus its projections
    // on estimates 0 .. e-1, normalised
    for (int k = 0; k < ne; ++k)
        if ((st = itse_orthogonalise(X, k))) return st;
    if ((st = itse_evaluate(X, 1))) return st;
    for (int k = 0; k < ne; ++k)
        if ((st = itse_observe(X, k, &out[k]))) return st;
    *n_out = ne;
    if (states_out) {
        const size_t n3 = (size_t)L->d.n * L->d.n * L->d.n;
        const size_t sw = dtype == ITSE_DTYPE_F32 ? 4 : 8;
        for (int k = 0; k < ne; ++k)
            if ((st = itse_get_state(X, k, (char *)states_out + (size_t)k * n3 * sw, dtype, on_device))) return st;
    }
    return ITSE_OK;
}

// ------------------------------------------------------------------------------------
// Per-pass profiling (eager launches bracketed by events)
// ------------------------------------------------------------------------------------
namespace itse {
template <typename R>
static hipError_t launch_pass(const Group &g, int p, hipStream_t s) {
    switch (p) {
    case 0: return Launch<R>::plane_fwd(g.n, g.variant, g.kmax, g.jobs, g.njobs, s);
    case 1: return Launch<R>::columns(g.n, g.variant, COL_KIN, 1, g.jobs, g.njobs, nullptr, s);
    case 2: {
        const int mom = (g.needs & NEED_MOMENTS) ? 1 : 0;
        if (g.cplx && cplx_fused(g)) {
            // the real parts' pass, then the imaginary parts' pass with the complex update
            hipError_t e = Launch<R>::plane_inv(g.n, g.variant, INV_KBUF, 0, g.kmax, g.jobs, g.nlats, s);
            return e != hipSuccess ? e : Launch<R>::plane_inv_cplx(g.n, g.variant, g.jobs + g.nlats, g.nlats, s);
        }
        const int mode = g.cplx ? INV_KBUF : INV_UPDATE;
        return g.fdtd ? Launch<R>::fdtd(g.n, g.kmax, mode, g.jobs, g.njobs, s)
                      : Launch<R>::plane_inv(g.n, g.variant, mode, mom, g.kmax, g.jobs, g.njobs, s);
    }
    case 3:
        // the separate complex update takes the slot of the per-state projection
        if (g.cplx && !cplx_fused(g))
            return Launch<R>::complex_update(g.n, g.nb_cplx, g.lats, g.nlats, INV_UPDATE, s);
        return (g.needs & NEED_PROJECT) ? Launch<R>::project(g.n, g.jobs, g.njobs, 0, 0, 1, s) : hipSuccess;
    case 4:
        return (g.needs & NEED_GRAM) ? Launch<R>::project_gram(g.n, g.kmax, g.lats, g.nlats, 0, 1, s) : hipSuccess;
    default: return launch_finalize(g.lats, g.nlats, FIN_STEP, s);
    }
}
static const char *pass_names[] = {"k_plane_fwd", "k_columns", "k_plane_inv", "k_project", "k_project_gram",
                                   "k_finalize"};
constexpr int NPASS = 6;
}  // namespace itse

extern "C" itse_status itse_profile_step(itse_lattice *L, int nsteps, double *ms_out, int *npass, char *names,
                                         size_t names_len) {
    if (!L || !npass || (*npass > 0 && !ms_out)) return fail(ITSE_EINVAL, "null argument");
    if (nsteps < 1) return fail(ITSE_EINVAL, "nsteps < 1");
    Group g = single_group(L);
    // passes a step of these options does not launch are reported as 0
    bool launched[NPASS];
    for (int p = 0; p < NPASS; ++p)
        launched[p] = !((p == 3 && !(g.needs & NEED_PROJECT) && !(g.cplx && !cplx_fused(g))) ||
                        (p == 4 && !(g.needs & NEED_GRAM)) || (p < 2 && g.fdtd));
    std::vector<hipEvent_t> ev((size_t)nsteps * (NPASS + 1));
    for (auto &e : ev) HIPCHK(hipEventCreate(&e));
    for (int s = 0; s < nsteps; ++s) {
        HIPCHK(hipEventRecord(ev[(size_t)s * (NPASS + 1)], L->stream));
        for (int p = 0; p < NPASS; ++p) {
            if (!launched[p]) continue;
            hipError_t e = L->d.precision == ITSE_FP32 ? launch_pass<float>(g, p, L->stream)
                                                       : launch_pass<double>(g, p, L->stream);
            if (e != hipSuccess) return fail(ITSE_EDEVICE, "pass %d: %s", p, hipGetErrorString(e));
            HIPCHK(hipEventRecord(ev[(size_t)s * (NPASS + 1) + p + 1], L->stream));
        }
    }
    HIPCHK(hipStreamSynchronize(L->stream));
    L->steps_host += nsteps;
    const int cap = *npass;
    for (int p = 0; p < NPASS && p < cap; ++p) {
        double acc = 0.0;
        if (launched[p]) {
            int prev = p;  // the event recorded before this pass
            while (prev > 0 && !launched[prev - 1]) --prev;
            for (int s = 0; s < nsteps; ++s) {
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, ev[(size_t)s * (NPASS + 1) + prev],
                                           ev[(size_t)s * (NPASS + 1) + p + 1]));
                acc += ms;
            }
        }
        ms_out[p] = acc / nsteps;
    }
    *npass = NPASS;
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (names && names_len) {
        std::string js = "[";
        for (int p = 0; p < NPASS; ++p)
            js += std::string(p ? ", " : "") + "\"" +
                  (p == 2 && g.fdtd ? "k_fdtd" : p == 3 && g.cplx && !cplx_fused(g) ? "k_complex_update" : pass_names[p]) +
                  "\"";
        js += "]";
        snprintf(names, names_len, "%s", js.c_str());
    }
    return check_device_error(L);
}
