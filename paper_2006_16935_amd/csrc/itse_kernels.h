// Device code for the imaginary-time step: LDS-staged Stockham transforms,
// the fused update + FP64 reductions, reflection projection and Gram sums.
// Included once per precision (itse_f32.hip, itse_f64.hip).
//
// Transform conventions follow the paper's FFT / IFFT definitions (section
// "Kinetic terms"): forward sum_x psi exp(-i k.x), inverse with exp(+i k.x),
// both unnormalised; the 1/N^3 is folded into the kinetic symbol.
#pragma once

#include "itse_internal.h"

namespace itse {

template <typename R>
struct C2 {
    R x, y;
};

template <typename R>
__device__ __forceinline__ C2<R> cadd(C2<R> a, C2<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ C2<R> csub(C2<R> a, C2<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ C2<R> cmul(C2<R> a, C2<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by SIGN * i
template <int SIGN, typename R>
__device__ __forceinline__ C2<R> mul_si(C2<R> a) {
    return SIGN > 0 ? C2<R>{-a.y, a.x} : C2<R>{a.y, -a.x};
}

// ---------------------------------------------------------------------------
// Small DFT kernels (radix 2, 3, 4) with exponent sign SIGN.
// ---------------------------------------------------------------------------
template <int RAD, int SIGN, typename R>
__device__ __forceinline__ void dft_small(C2<R> *a) {
    if constexpr (RAD == 2) {
        C2<R> t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    } else if constexpr (RAD == 4) {
        C2<R> s0 = cadd(a[0], a[2]), d0 = csub(a[0], a[2]);
        C2<R> s1 = cadd(a[1], a[3]), d1 = mul_si<SIGN>(csub(a[1], a[3]));
        a[0] = cadd(s0, s1);
        a[2] = csub(s0, s1);
        a[1] = cadd(d0, d1);
        a[3] = csub(d0, d1);
    } else {
        static_assert(RAD == 3, "radix");
        // w = exp(SIGN 2 pi i / 3) = -1/2 + SIGN i sqrt(3)/2
        const R half_sqrt3 = (R)0.86602540378443864676372317075294;
        C2<R> t1 = cadd(a[1], a[2]);
        C2<R> t2 = {a[0].x - (R)0.5 * t1.x, a[0].y - (R)0.5 * t1.y};
        C2<R> d = csub(a[1], a[2]);
        C2<R> r = mul_si<SIGN>(C2<R>{half_sqrt3 * d.x, half_sqrt3 * d.y});
        a[0] = cadd(a[0], t1);
        a[1] = cadd(t2, r);
        a[2] = csub(t2, r);
    }
}

constexpr int next_radix(int rem) { return rem % 4 == 0 ? 4 : (rem % 2 == 0 ? 2 : 3); }

// One Stockham (autosort, decimation in time) stage over NL lines of length N
// held in LDS.  P = product of the radices already applied.  Element e of line l
// is at buf[l*ls + e*es].  Butterfly j reads x[j + m N/RAD] (m < RAD), twiddles
// input m by w^(k m N/(P RAD)) with k = j mod P, and writes output q to
// (j - k) RAD + k + q P.  LINE_FAST selects which index varies fastest over
// the threads (chosen so that consecutive lanes touch consecutive LDS words).
template <typename R, int N, int P, int RAD, int NL, int SIGN, bool LINE_FAST>
__device__ __forceinline__ void stockham_stage(C2<R> *buf, int ls, int es, const C2<R> *tw, int tid) {
    constexpr int M = N / RAD;
    constexpr int TASKS = NL * M;
    constexpr int TPT = (TASKS + NT - 1) / NT;
    C2<R> v[TPT][RAD];
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const int task = tid + t * NT;
        if (TASKS % NT == 0 || task < TASKS) {
            const int line = LINE_FAST ? task % NL : task / M;
            const int j = LINE_FAST ? task / NL : task % M;
            const int k = j % P;
            const C2<R> *b = buf + line * ls;
#pragma unroll
            for (int m = 0; m < RAD; ++m) {
                C2<R> a = b[(j + m * M) * es];
                if (P > 1 && m > 0) {
                    C2<R> w = tw[k * m * (N / (P * RAD))];
                    if (SIGN > 0) w.y = -w.y;
                    a = cmul(a, w);
                }
                v[t][m] = a;
            }
            dft_small<RAD, SIGN>(v[t]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const int task = tid + t * NT;
        if (TASKS % NT == 0 || task < TASKS) {
            const int line = LINE_FAST ? task % NL : task / M;
            const int j = LINE_FAST ? task / NL : task % M;
            const int k = j % P;
            C2<R> *b = buf + line * ls;
#pragma unroll
            for (int q = 0; q < RAD; ++q) b[((j - k) * RAD + k + q * P) * es] = v[t][q];
        }
    }
    __syncthreads();
}

template <typename R, int N, int P, int NL, int SIGN, bool LINE_FAST>
__device__ __forceinline__ void stockham(C2<R> *buf, int ls, int es, const C2<R> *tw, int tid) {
    if constexpr (P < N) {
        constexpr int RAD = next_radix(N / P);
        stockham_stage<R, N, P, RAD, NL, SIGN, LINE_FAST>(buf, ls, es, tw, tid);
        stockham<R, N, P * RAD, NL, SIGN, LINE_FAST>(buf, ls, es, tw, tid);
    }
}

// ---------------------------------------------------------------------------
// Fixed-order workgroup sums (deterministic).
// ---------------------------------------------------------------------------
template <int Q>
__device__ __forceinline__ void block_reduce_store(double (&acc)[Q], double *dst, double *lds) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < Q; ++q) lds[q * NT + tid] = acc[q];
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (tid < s) {
#pragma unroll
            for (int q = 0; q < Q; ++q) lds[q * NT + tid] += lds[q * NT + tid + s];
        }
        __syncthreads();
    }
    if (tid < Q) dst[tid] = lds[tid * NT];
}

// Coordinate of index idx about the potential centre (same convention as the
// potential generator: cell centre (n-1)/2, or origin with minimum image).
__device__ __forceinline__ double site_coord(int idx, int n, int center, double a) {
    if (center == ITSE_CENTER_CELL) return ((double)idx - 0.5 * (double)(n - 1)) * a;
    return (double)((2 * idx <= n) ? idx : idx - n) * a;
}

__device__ __forceinline__ int mirror_idx(int idx, int n, int center) {
    return center == ITSE_CENTER_CELL ? n - 1 - idx : (idx == 0 ? 0 : n - idx);
}

// Kinetic symbol from the sum of the three per-axis table entries (FP64).
__device__ __forceinline__ double kin_symbol(int kin, int sub, double mass, double s) {
    if (kin == ITSE_KIN_NR_CONT || kin == ITSE_KIN_NR_LAT) return s;
    const double e = sqrt(s + mass * mass);
    return sub ? s / (e + mass) : e;
}

// ---------------------------------------------------------------------------
// Schedules.
// ---------------------------------------------------------------------------
constexpr int largest_divisor_le(int total, int cap) {
    int best = 1;
    for (int d = 1; d <= cap && d <= total; ++d)
        if (total % d == 0) best = d;
    return best;
}
template <int N>
struct RowSched {
    static constexpr int RP = largest_divisor_le(N * N / 2, (2048 / N) > 0 ? 2048 / N : 1);
    static constexpr int LS = N + 1;  // padded line stride in LDS
    static constexpr int NB = (N * N / 2) / RP;
};
template <typename R>
struct ColW {
    static constexpr int W = sizeof(R) == 4 ? 16 : 8;
};
template <typename R, int N, int W>
struct ColSched {
    static constexpr int NCOLS = N * (N / 2 + 1);
    static constexpr int NB = (NCOLS + W - 1) / W;
};

// ---------------------------------------------------------------------------
// Pass 1 (row pairs along x3): current state phi_i = sum_j coef[j][i] u_j is
// formed in FP64 and stored, then two real rows (x2 = 2p, 2p+1) are packed as one
// complex row, transformed along x3, and split into the two half spectra.
// ---------------------------------------------------------------------------
template <typename R, int N>
__global__ void __launch_bounds__(NT) k_rows_fwd(const JobRef *__restrict__ jobs) {
    using RS = RowSched<N>;
    constexpr int RP = RS::RP, LS = RS::LS, H = N / 2 + 1;
    __shared__ C2<R> buf[RP * LS];
    __shared__ C2<R> tw[N];
    const JobRef job = jobs[blockIdx.y];
    const LatDev &L = *job.lat;
    const int i = job.state;
    const int tid = threadIdx.x;
    const C2<R> *twg = (const C2<R> *)L.tw;
    for (int e = tid; e < N; e += NT) tw[e] = twg[e];
    double c[MAXK];
#pragma unroll
    for (int j = 0; j < MAXK; ++j) c[j] = (j <= i) ? L.coef[j][i] : 0.0;
    R *phi = (R *)L.phi[i];
    const int q0 = blockIdx.x * RP;
    for (int e = tid; e < RP * N; e += NT) {
        const int r = e / N, z = e % N;
        const int q = q0 + r, x = q / (N / 2), p = q % (N / 2);
        const size_t off0 = ((size_t)x * N + 2 * p) * N + z, off1 = off0 + N;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int j = 0; j < MAXK; ++j) {
            if (j <= i && c[j] != 0.0) {
                const R *u = (const R *)L.u[j];
                s0 += c[j] * (double)u[off0];
                s1 += c[j] * (double)u[off1];
            }
        }
        const R a0 = (R)s0, a1 = (R)s1;
        phi[off0] = a0;
        phi[off1] = a1;
        buf[r * LS + z] = C2<R>{a0, a1};
    }
    __syncthreads();
    stockham<R, N, 1, RP, -1, false>(buf, LS, 1, tw, tid);
    C2<R> *spec = (C2<R> *)L.spec[i];
    for (int e = tid; e < RP * 2 * H; e += NT) {
        const int r = e / (2 * H), t = e % (2 * H);
        const int row = t / H, k = t % H;
        const C2<R> ck = buf[r * LS + k];
        const C2<R> cm = buf[r * LS + (N - k) % N];
        C2<R> out;
        if (row == 0) out = C2<R>{(R)0.5 * (ck.x + cm.x), (R)0.5 * (ck.y - cm.y)};
        else out = C2<R>{(R)0.5 * (ck.y + cm.y), (R)0.5 * (cm.x - ck.x)};
        const int q = q0 + r, x = q / (N / 2), p = q % (N / 2);
        spec[((size_t)x * N + 2 * p + row) * H + k] = out;
    }
}

// ---------------------------------------------------------------------------
// Strided-axis pass: W adjacent columns of the half spectrum, transformed along
// x2 (axis 1) or x1 (axis 0).  COL_KIN does forward, multiply by T(k)/N^3 (FP64
// symbol, FP64 product), inverse, all in LDS; with `moments` it also sums the
// momentum-space norm and <psi|P psi> for the parity weight.
// ---------------------------------------------------------------------------
template <typename R, int N, int W, int MODE>
__global__ void __launch_bounds__(NT) k_cols(const JobRef *__restrict__ jobs, int axis, int moments) {
    constexpr int H = N / 2 + 1, LSW = W + 1;
    constexpr int NCOLS = N * H;
    __shared__ C2<R> buf[N * LSW];
    __shared__ C2<R> tw[N];
    __shared__ double ktab[MODE == COL_KIN ? N : 1];
    __shared__ double red[NQC * NT];
    const JobRef job = jobs[blockIdx.y];
    const LatDev &L = *job.lat;
    const int i = job.state;
    const int tid = threadIdx.x;
    const C2<R> *twg = (const C2<R> *)L.tw;
    for (int e = tid; e < N; e += NT) tw[e] = twg[e];
    if constexpr (MODE == COL_KIN)
        for (int e = tid; e < N; e += NT) ktab[e] = L.ktab[e];
    C2<R> *spec = (C2<R> *)L.spec[i];
    const size_t S = axis == 0 ? (size_t)NCOLS : (size_t)H;
    const int c0 = blockIdx.x * W;
    for (int e = tid; e < N * W; e += NT) {
        const int n = e / W, w = e % W, c = c0 + w;
        C2<R> val = {(R)0, (R)0};
        if (c < NCOLS) {
            const size_t base = axis == 0 ? (size_t)c : (size_t)(c / H) * NCOLS + (c % H);
            val = spec[base + n * S];
        }
        buf[n * LSW + w] = val;
    }
    __syncthreads();
    if constexpr (MODE == COL_FWD || MODE == COL_KIN) stockham<R, N, 1, W, -1, true>(buf, 1, LSW, tw, tid);
    if constexpr (MODE == COL_INV) stockham<R, N, 1, W, +1, true>(buf, 1, LSW, tw, tid);
    if constexpr (MODE == COL_KIN) {
        const double inv_n3 = 1.0 / ((double)N * (double)N * (double)N);
        const bool mom = moments && L.moments;
        double acc[NQC] = {0.0, 0.0};
        for (int e = tid; e < N * W; e += NT) {
            const int n = e / W, w = e % W, c = c0 + w;
            if (c >= NCOLS) continue;
            const int ky = c / H, kz = c % H;
            C2<R> val = buf[n * LSW + w];
            if (mom) {
                // weight 2 for the interior of the half spectrum (its mirror is implied)
                const double wt = (kz == 0 || 2 * kz == N) ? 1.0 : 2.0;
                const double re = (double)val.x, im = (double)val.y;
                acc[CQ_NORM] += wt * (re * re + im * im);
                // <psi|P psi> = sum_k e^{i kappa} conj(psi_k)^2 / N^3; kappa = k1+k2+k3
                // for the off-grid centre (x -> N-1-x), 0 for the origin
                double pr = re * re - im * im, pi = -2.0 * re * im;
                if (L.center == ITSE_CENTER_CELL) {
                    const int m = (n + ky + kz) % N;
                    double sn, cs;
                    sincospi(2.0 * (double)m / (double)N, &sn, &cs);
                    const double tr = cs * pr - sn * pi;
                    pr = tr;
                }
                acc[CQ_PAR] += wt * pr;
            }
            const double t = kin_symbol(L.kin, L.sub, L.mass, ktab[n] + ktab[ky] + ktab[kz]) * inv_n3;
            val.x = (R)((double)val.x * t);
            val.y = (R)((double)val.y * t);
            buf[n * LSW + w] = val;
        }
        if (mom) block_reduce_store<NQC>(acc, L.part_cols + ((size_t)i * L.nb_cols + blockIdx.x) * NQC, red);
        __syncthreads();
        stockham<R, N, 1, W, +1, true>(buf, 1, LSW, tw, tid);
    }
    for (int e = tid; e < N * W; e += NT) {
        const int n = e / W, w = e % W, c = c0 + w;
        if (c < NCOLS) {
            const size_t base = axis == 0 ? (size_t)c : (size_t)(c / H) * NCOLS + (c % H);
            spec[base + n * S] = buf[n * LSW + w];
        }
    }
}

// ---------------------------------------------------------------------------
// Pass 3 (row pairs along x3): rebuild the packed complex row from the two half
// spectra, inverse transform -> H_K phi for rows 2p and 2p+1, then the update
//   u = ((1 - h V) phi - dtau H_K phi) / (1 + h V)      (= A phi - B dtau H_K phi)
// with FP64 partial sums of <phi|phi>, <phi|K phi>, <phi|V phi>, <u|u> and moments.
// ---------------------------------------------------------------------------
template <typename R, int N>
__global__ void __launch_bounds__(NT) k_rows_inv(const JobRef *__restrict__ jobs, int mode) {
    using RS = RowSched<N>;
    constexpr int RP = RS::RP, LS = RS::LS, H = N / 2 + 1;
    __shared__ C2<R> buf[RP * LS];
    __shared__ C2<R> tw[N];
    __shared__ double red[NQR * NT];
    const JobRef job = jobs[blockIdx.y];
    const LatDev &L = *job.lat;
    const int i = job.state;
    const int tid = threadIdx.x;
    const C2<R> *twg = (const C2<R> *)L.tw;
    for (int e = tid; e < N; e += NT) tw[e] = twg[e];
    const C2<R> *spec = (const C2<R> *)L.spec[i];
    const int q0 = blockIdx.x * RP;
    for (int e = tid; e < RP * N; e += NT) {
        const int r = e / N, k = e % N;
        const int q = q0 + r, x = q / (N / 2), p = q % (N / 2);
        const size_t row0 = ((size_t)x * N + 2 * p) * H, row1 = row0 + H;
        const bool direct = 2 * k <= N;
        const int kk = direct ? k : N - k;
        C2<R> A = spec[row0 + kk], B = spec[row1 + kk];
        if (!direct) {
            A.y = -A.y;
            B.y = -B.y;
        } else if (k == 0 || 2 * k == N) {
            A.y = (R)0;
            B.y = (R)0;
        }
        buf[r * LS + k] = C2<R>{A.x - B.y, A.y + B.x};
    }
    __syncthreads();
    stockham<R, N, 1, RP, +1, false>(buf, LS, 1, tw, tid);
    const R *phi = (const R *)L.phi[i];
    const R *v = (const R *)L.v;
    R *u = (R *)L.u[i];
    R *kout = (R *)L.kout;
    const R h = (R)L.h, dt = (R)L.dtau;
    const bool mom = L.moments != 0;
    double acc[NQR];
#pragma unroll
    for (int q = 0; q < NQR; ++q) acc[q] = 0.0;
    for (int e = tid; e < RP * N; e += NT) {
        const int r = e / N, z = e % N;
        const int q = q0 + r, x = q / (N / 2), p = q % (N / 2);
        const C2<R> kp = buf[r * LS + z];
#pragma unroll
        for (int row = 0; row < 2; ++row) {
            const int y = 2 * p + row;
            const size_t off = ((size_t)x * N + y) * N + z;
            const R kv = row == 0 ? kp.x : kp.y;
            const R ph = phi[off];
            const R vv = v[off];
            const R hv = h * vv;
            const R un = (ph * ((R)1 - hv) - dt * kv) / ((R)1 + hv);
            if (mode == INV_UPDATE) u[off] = un;
            else if (mode == INV_KOUT) kout[off] = kv;
            const double pd = (double)ph;
            acc[RQ_PP] += pd * pd;
            acc[RQ_PK] += pd * (double)kv;
            acc[RQ_VPP] += (double)vv * pd * pd;
            acc[RQ_UU] += (double)un * (double)un;
            if (mom) {
                const double cx = site_coord(x, N, L.center, L.a);
                const double cy = site_coord(y, N, L.center, L.a);
                const double cz = site_coord(z, N, L.center, L.a);
                const double w2 = pd * pd;
                acc[RQ_X] += cx * w2;
                acc[RQ_Y] += cy * w2;
                acc[RQ_Z] += cz * w2;
                acc[RQ_R2] += (cx * cx + cy * cy + cz * cz) * w2;
            }
        }
    }
    block_reduce_store<NQR>(acc, L.part_rows + ((size_t)i * L.nb_rows + blockIdx.x) * NQR, red);
}

// ---------------------------------------------------------------------------
// Reflection projection of u_i in place: u <- (u + sign u o R)/2.  Each site
// pair {s, R s} is handled by the one thread owning the smaller index, so the
// in-place update is race-free.  Partial sums of |P u|^2.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(NT) k_project(const JobRef *__restrict__ jobs, int force_sign, int force_axes) {
    __shared__ double red[NT];
    const JobRef job = jobs[blockIdx.y];
    const LatDev &L = *job.lat;
    const int i = job.state;
    const int sign = force_sign ? force_sign : L.psign[i];
    if (sign == 0) return;  // uniform over the workgroup
    const int axes = force_sign ? force_axes : L.paxes[i];
    const int n = L.n;
    const size_t n3 = (size_t)n * n * n;
    R *u = (R *)L.u[i];
    double acc[1] = {0.0};
    const size_t base = (size_t)blockIdx.x * NT * FLAT_SPT;
    for (int t = 0; t < FLAT_SPT; ++t) {
        const size_t s = base + (size_t)t * NT + threadIdx.x;
        if (s >= n3) break;
        const int x = (int)(s / ((size_t)n * n)), y = (int)((s / n) % n), z = (int)(s % n);
        const int rx = (axes & 1) ? mirror_idx(x, n, L.center) : x;
        const int ry = (axes & 2) ? mirror_idx(y, n, L.center) : y;
        const int rz = (axes & 4) ? mirror_idx(z, n, L.center) : z;
        const size_t m = ((size_t)rx * n + ry) * n + rz;
        if (m < s) continue;
        if (m == s) {
            const R val = sign > 0 ? u[s] : (R)0;
            u[s] = val;
            acc[0] += (double)val * (double)val;
        } else {
            const R a = u[s], b = u[m];
            const R pa = (R)0.5 * (a + (R)sign * b);
            const R pb = (R)sign * pa;
            u[s] = pa;
            u[m] = pb;
            acc[0] += 2.0 * (double)pa * (double)pa;
        }
    }
    block_reduce_store<1>(acc, L.part_proj + (size_t)i * L.nb_proj + blockIdx.x, red);
}

// ---------------------------------------------------------------------------
// Gram sums <u_j|u_l>, j <= l < nstates, for one lattice per blockIdx.y.  Runs
// only on steps that orthogonalise (or when forced).
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(NT) k_gram(const JobRef *__restrict__ lats, int force) {
    constexpr int NG = MAXK * (MAXK + 1) / 2;
    __shared__ double red[NT];
    const LatDev &L = *lats[blockIdx.y].lat;
    const int K = L.nstates;
    if (K < 2) return;
    if (!force) {
        if (L.ortho_every <= 0 || ((L.step + 1) % L.ortho_every) != 0) return;
    }
    const int n = L.n;
    const size_t n3 = (size_t)n * n * n;
    double acc[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) acc[g] = 0.0;
    const size_t base = (size_t)blockIdx.x * NT * FLAT_SPT;
    for (int t = 0; t < FLAT_SPT; ++t) {
        const size_t s = base + (size_t)t * NT + threadIdx.x;
        if (s >= n3) break;
        double val[MAXK];
#pragma unroll
        for (int j = 0; j < MAXK; ++j) val[j] = j < K ? (double)((const R *)L.u[j])[s] : 0.0;
        int g = 0;
#pragma unroll
        for (int l = 0; l < MAXK; ++l)
#pragma unroll
            for (int j = 0; j <= l; ++j) {
                acc[g] += val[j] * val[l];
                ++g;
            }
    }
    // reduce each used slot in turn (fixed order)
    const int ng_used = K * (K + 1) / 2;
    double *dst = L.part_gram + (size_t)blockIdx.x * NG;
    int g = 0;
    for (int l = 0; l < MAXK; ++l)
        for (int j = 0; j <= l; ++j, ++g) {
            if (l >= K) continue;
            red[threadIdx.x] = acc[g];
            __syncthreads();
            for (int st = NT / 2; st > 0; st >>= 1) {
                if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
                __syncthreads();
            }
            if (threadIdx.x == 0) dst[g] = red[0];
            __syncthreads();
        }
    (void)ng_used;
}

// out_i = sum_j coef[j][i] u_j (materialise the current state i), FP64 combination.
template <typename R>
__global__ void __launch_bounds__(NT) k_combine(const JobRef *__restrict__ jobs, void *const *outs) {
    const JobRef job = jobs[blockIdx.y];
    const LatDev &L = *job.lat;
    const int i = job.state;
    const int n = L.n;
    const size_t n3 = (size_t)n * n * n;
    R *out = (R *)outs[blockIdx.y];
    const size_t base = (size_t)blockIdx.x * NT * FLAT_SPT;
    for (int t = 0; t < FLAT_SPT; ++t) {
        const size_t s = base + (size_t)t * NT + threadIdx.x;
        if (s >= n3) break;
        double acc = 0.0;
        for (int j = 0; j <= i; ++j) {
            const double c = L.coef[j][i];
            if (c != 0.0) acc += c * (double)((const R *)L.u[j])[s];
        }
        out[s] = (R)acc;
    }
}

template <typename S, typename D>
__global__ void __launch_bounds__(NT) k_convert(const S *__restrict__ src, D *__restrict__ dst, size_t count) {
    const size_t stride = (size_t)gridDim.x * NT;
    for (size_t s = (size_t)blockIdx.x * NT + threadIdx.x; s < count; s += stride) dst[s] = (D)src[s];
}

}  // namespace itse
