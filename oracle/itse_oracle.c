/*
 * FP64 CPU oracle for the imaginary-time Schroedinger eigensolver step
 * (arXiv:2006.16935, "The Relativistic Schroedinger Equation through FFTW 3").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the HIP
 * path is checked against.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it; the product library never links or calls it, and
 * it shares no code, header or table with the product.
 *
 * Everything is double precision.  Complex arithmetic uses C99 `double complex`.
 * Transforms are complex-to-complex over the whole N^3 lattice (no real-input
 * tricks), unnormalised, with the sign convention of the paper's FFT / IFFT
 * definitions (section "Kinetic terms"): forward = exp(-i k.x), inverse = exp(+i k.x).
 *
 * Pins: each function below is checked by tests/test_oracle_*.py against values
 * fixed by the paper or by mathematics (naive DFT, numpy's FFT, analytic
 * derivatives, the lattice Laplacian stencil, separable 1D eigensolves, the
 * paper's printed relativistic-oscillator energy).  See the header comment of
 * each test module.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* Lattice description: NUM, A, MASS, KINTERM, EPS of the paper's parameter list. */
typedef struct {
    int n;
    double a;
    double mass;
    double dtau;
    int kin;            /* 0: H_K^(0) finite differences, Dirichlet box; 1: H_K^(1), 2: H_K^(2),
                           3: H_K^(3), 4: relativistic with k^2 */
    int subtract_rest;  /* relativistic forms: 1 -> sqrt(p^2+m^2) - m */
    int center;         /* 0: off-grid cell centre (N-1)/2, 1: lattice origin */
} orc_lattice;

/* Observables of one state (pre-update), all FP64. */
typedef struct {
    double energy, kinetic, potential, norm2, x, y, z, r2, parity_even;
} orc_obs;

static const double ORC_PI = 3.14159265358979323846264338327950288;

static int valid_length(int n)
{
    if (n < 2) return 0;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

/* ------------------------------------------------------------------------------ */
/* 1D transform.  Unnormalised DFT  y_k = sum_j x_j exp(sign * 2 pi i j k / len).  */
/* Lengths up to 16 use the definition directly; longer lengths split by radix 2  */
/* (else 3) in decimation-in-time Cooley-Tukey form and recurse.                  */
/* ------------------------------------------------------------------------------ */

/* Root of unity table for the top-level length `ntw`: tw[e] = exp(-2 pi i e / ntw). */
static cplx *make_roots(int ntw)
{
    cplx *tw = (cplx *)malloc(sizeof(cplx) * (size_t)ntw);
    if (!tw) return NULL;
    for (int e = 0; e < ntw; ++e) {
        double ang = -2.0 * ORC_PI * (double)e / (double)ntw;
        tw[e] = cos(ang) + I * sin(ang);
    }
    return tw;
}

/* exp(sign * 2 pi i e / len) for len dividing ntw. */
static inline cplx root(const cplx *tw, int ntw, int len, long e, int sign)
{
    long r = e % len;
    cplx w = tw[r * (ntw / len)];
    return sign > 0 ? conj(w) : w;
}

static void dft_definition(const cplx *x, cplx *y, int len, const cplx *tw, int ntw, int sign)
{
    for (int k = 0; k < len; ++k) {
        cplx acc = 0.0;
        for (int j = 0; j < len; ++j) acc += x[j] * root(tw, ntw, len, (long)j * k, sign);
        y[k] = acc;
    }
}

/* In-place transform of contiguous x[0..len); scratch must hold len values. */
static void fft_recursive(cplx *x, int len, cplx *scratch, const cplx *tw, int ntw, int sign)
{
    if (len <= 16 || (len % 2 != 0 && len % 3 != 0)) {
        dft_definition(x, scratch, len, tw, ntw, sign);
        memcpy(x, scratch, sizeof(cplx) * (size_t)len);
        return;
    }
    int p = (len % 2 == 0) ? 2 : 3;
    int m = len / p;
    /* decimate: sub-sequence r holds x[r], x[r+p], x[r+2p], ... */
    for (int r = 0; r < p; ++r)
        for (int j = 0; j < m; ++j) scratch[r * m + j] = x[j * p + r];
    /* transform each sub-sequence; the original x is free to serve as scratch */
    for (int r = 0; r < p; ++r) fft_recursive(scratch + r * m, m, x + r * m, tw, ntw, sign);
    /* combine: X[k + q m] = sum_r w_len^{r (k + q m)} Y_r[k] */
    for (int q = 0; q < p; ++q)
        for (int k = 0; k < m; ++k) {
            cplx acc = 0.0;
            for (int r = 0; r < p; ++r)
                acc += scratch[r * m + k] * root(tw, ntw, len, (long)r * (k + q * m), sign);
            x[k + q * m] = acc;
        }
}

/* `count` contiguous lines of length `len`, interleaved re/im doubles. */
int orc_fft_lines(int len, int count, double *data, int sign)
{
    if (len < 1 || count < 0 || !data || (sign != 1 && sign != -1)) return ORC_EINVAL;
    cplx *tw = make_roots(len);
    if (!tw) return ORC_ENOMEM;
    cplx *lines = (cplx *)data;
    int err = 0;
#pragma omp parallel
    {
        cplx *scratch = (cplx *)malloc(sizeof(cplx) * (size_t)len);
        if (!scratch) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static)
            for (int c = 0; c < count; ++c) fft_recursive(lines + (size_t)c * len, len, scratch, tw, len, sign);
            free(scratch);
        }
    }
    free(tw);
    return err ? ORC_ENOMEM : ORC_OK;
}

/* Unnormalised 3D transform of an N^3 complex array [x][y][z] (z fastest),
 * applied axis by axis: z, then y, then x. */
int orc_fft3d(int n, double *data, int sign)
{
    if (n < 1 || !data || (sign != 1 && sign != -1)) return ORC_EINVAL;
    cplx *tw = make_roots(n);
    if (!tw) return ORC_ENOMEM;
    cplx *f = (cplx *)data;
    const size_t nn = (size_t)n * n;
    int err = 0;
    for (int axis = 2; axis >= 0; --axis) {
        size_t stride = axis == 2 ? 1 : (axis == 1 ? (size_t)n : nn);
#pragma omp parallel
        {
            cplx *line = (cplx *)malloc(sizeof(cplx) * (size_t)n);
            cplx *scratch = (cplx *)malloc(sizeof(cplx) * (size_t)n);
            if (!line || !scratch) {
#pragma omp atomic write
                err = 1;
            } else {
#pragma omp for schedule(static)
                for (long l = 0; l < (long)nn; ++l) {
                    /* the two indices other than `axis` */
                    size_t i0 = (size_t)l / n, i1 = (size_t)l % n;
                    size_t base;
                    if (axis == 2) base = i0 * nn + i1 * n;
                    else if (axis == 1) base = i0 * nn + i1;
                    else base = i0 * n + i1;
                    for (int t = 0; t < n; ++t) line[t] = f[base + t * stride];
                    fft_recursive(line, n, scratch, tw, n, sign);
                    for (int t = 0; t < n; ++t) f[base + t * stride] = line[t];
                }
            }
            free(line);
            free(scratch);
        }
    }
    free(tw);
    return err ? ORC_ENOMEM : ORC_OK;
}

/* ------------------------------------------------------------------------------ */
/* Kinetic symbol T(k)  (paper, equations HK1, HK2, HK3 and the eigenmode set).   */
/* ------------------------------------------------------------------------------ */

/* k_l = 2 pi m / N with m = n if 2n <= N else n - N (momenta in (-pi, pi]). */
static double lattice_k(int idx, int n)
{
    int m = (2 * idx <= n) ? idx : idx - n;
    return 2.0 * ORC_PI * (double)m / (double)n;
}

static double symbol_value(const orc_lattice *L, double kx, double ky, double kz)
{
    const double a = L->a, m = L->mass;
    if (L->kin == 1) {
        /* H_K^(1): sum k_l^2 / (2 A^2 M) */
        return (kx * kx + ky * ky + kz * kz) / (2.0 * a * a * m);
    }
    if (L->kin == 2) {
        /* H_K^(2): 4 sum sin^2(k_l/2) / (2 A^2 M) */
        double s = sin(0.5 * kx) * sin(0.5 * kx) + sin(0.5 * ky) * sin(0.5 * ky) +
                   sin(0.5 * kz) * sin(0.5 * kz);
        return 4.0 * s / (2.0 * a * a * m);
    }
    double p2;
    if (L->kin == 3) {
        /* H_K^(3): (1/A) sqrt(4 sum sin^2(k_l/2) + (A M)^2) = sqrt(p^2 + M^2),
         * p^2 = (4/A^2) sum sin^2(k_l/2) */
        double s = sin(0.5 * kx) * sin(0.5 * kx) + sin(0.5 * ky) * sin(0.5 * ky) +
                   sin(0.5 * kz) * sin(0.5 * kz);
        p2 = 4.0 * s / (a * a);
    } else {
        /* relativistic analogue of H_K^(1): p^2 = sum k_l^2 / A^2 */
        p2 = (kx * kx + ky * ky + kz * kz) / (a * a);
    }
    double e = sqrt(p2 + m * m);
    if (L->subtract_rest) {
        /* sqrt(p^2+m^2) - m written without cancellation */
        return p2 / (e + m);
    }
    return e;
}

static int lattice_ok(const orc_lattice *L)
{
    return L && L->n >= 2 && L->a > 0.0 && L->mass > 0.0 && L->kin >= 0 && L->kin <= 4 &&
           (L->center == 0 || L->center == 1);
}

/* Full FP64 symbol on the N^3 momentum grid, same index layout as the spectrum
 * (the transform-based kinds 1..4 only). */
int orc_kinetic_symbol(const orc_lattice *L, double *T)
{
    if (!lattice_ok(L) || L->kin == 0 || !T) return ORC_EINVAL;
    const int n = L->n;
#pragma omp parallel for schedule(static)
    for (int ix = 0; ix < n; ++ix)
        for (int iy = 0; iy < n; ++iy)
            for (int iz = 0; iz < n; ++iz)
                T[((size_t)ix * n + iy) * n + iz] =
                    symbol_value(L, lattice_k(ix, n), lattice_k(iy, n), lattice_k(iz, n));
    return ORC_OK;
}

/* H_K^(0) (paper, equation HK0): the finite-difference kinetic term with Dirichlet
 * boundaries.  Read with the normalisation of its momentum-space form
 * (4/A^2) sin^2(k/2) / (2M) per axis, i.e.
 *   H psi(x) = (1/(2 M A^2)) sum over the six neighbours y of (psi(x) - psi(y)),
 * where psi vanishes outside the N^3 box (the neighbours beyond a face are zero). */
static void apply_fdtd(const orc_lattice *L, const double *psi, double *out)
{
    const int n = L->n;
    const double c = 1.0 / (2.0 * L->mass * L->a * L->a);
#pragma omp parallel for schedule(static)
    for (int ix = 0; ix < n; ++ix)
        for (int iy = 0; iy < n; ++iy)
            for (int iz = 0; iz < n; ++iz) {
                const size_t s = ((size_t)ix * n + iy) * n + iz;
                const double p = psi[s];
                double acc = 0.0;
                acc += p - (ix > 0 ? psi[s - (size_t)n * n] : 0.0);
                acc += p - (ix < n - 1 ? psi[s + (size_t)n * n] : 0.0);
                acc += p - (iy > 0 ? psi[s - n] : 0.0);
                acc += p - (iy < n - 1 ? psi[s + n] : 0.0);
                acc += p - (iz > 0 ? psi[s - 1] : 0.0);
                acc += p - (iz < n - 1 ? psi[s + 1] : 0.0);
                out[s] = c * acc;
            }
}

/* K psi = IFFT[ T(k) FFT[psi] ] / N^3 for a real psi (result is real); H_K^(0)
 * by its stencil. */
static int apply_kinetic_with(const orc_lattice *L, const double *T, const double *psi, double *out,
                              cplx *work)
{
    if (L->kin == 0) {
        apply_fdtd(L, psi, out);
        return ORC_OK;
    }
    const size_t n3 = (size_t)L->n * L->n * L->n;
    for (size_t s = 0; s < n3; ++s) work[s] = psi[s];
    int st = orc_fft3d(L->n, (double *)work, -1);
    if (st) return st;
    const double inv = 1.0 / (double)n3;
    for (size_t s = 0; s < n3; ++s) work[s] *= T[s] * inv;
    st = orc_fft3d(L->n, (double *)work, +1);
    if (st) return st;
    for (size_t s = 0; s < n3; ++s) out[s] = creal(work[s]);
    return ORC_OK;
}

int orc_apply_kinetic(const orc_lattice *L, const double *psi, double *out)
{
    if (!lattice_ok(L) || !valid_length(L->n) || !psi || !out) return ORC_EINVAL;
    const size_t n3 = (size_t)L->n * L->n * L->n;
    double *T = (double *)malloc(sizeof(double) * n3);
    cplx *work = (cplx *)malloc(sizeof(cplx) * n3);
    int st = ORC_ENOMEM;
    if (T && work) {
        if (L->kin != 0) orc_kinetic_symbol(L, T);
        st = apply_kinetic_with(L, T, psi, out, work);
    }
    free(T);
    free(work);
    return st;
}

/* ------------------------------------------------------------------------------ */
/* Sums.  Each x-plane is summed in index order, then the plane sums are added in */
/* index order; the result does not depend on the number of threads.              */
/* ------------------------------------------------------------------------------ */

typedef double (*site_fn)(const void *ctx, size_t s, int ix, int iy, int iz);

static double lattice_sum(int n, site_fn f, const void *ctx)
{
    double *plane = (double *)malloc(sizeof(double) * (size_t)n);
    if (!plane) return NAN;
#pragma omp parallel for schedule(static)
    for (int ix = 0; ix < n; ++ix) {
        double acc = 0.0;
        for (int iy = 0; iy < n; ++iy) {
            double row = 0.0;
            for (int iz = 0; iz < n; ++iz) row += f(ctx, ((size_t)ix * n + iy) * n + iz, ix, iy, iz);
            acc += row;
        }
        plane[ix] = acc;
    }
    double total = 0.0;
    for (int ix = 0; ix < n; ++ix) total += plane[ix];
    free(plane);
    return total;
}

typedef struct {
    const double *p, *q, *w;  /* sum p q (w) */
} dot_ctx;

static double dot_site(const void *c, size_t s, int ix, int iy, int iz)
{
    (void)ix; (void)iy; (void)iz;
    const dot_ctx *d = (const dot_ctx *)c;
    return d->w ? d->p[s] * d->w[s] * d->q[s] : d->p[s] * d->q[s];
}

static double dot(int n, const double *p, const double *q, const double *w)
{
    dot_ctx c = {p, q, w};
    return lattice_sum(n, dot_site, &c);
}

/* Signed physical coordinate relative to the potential centre. */
static double coord(const orc_lattice *L, int idx)
{
    if (L->center == 0) return ((double)idx - 0.5 * (double)(L->n - 1)) * L->a;
    int m = (2 * idx <= L->n) ? idx : idx - L->n;
    return (double)m * L->a;
}

static int mirror(const orc_lattice *L, int idx)
{
    return L->center == 0 ? L->n - 1 - idx : (L->n - idx) % L->n;
}

typedef struct {
    const orc_lattice *L;
    const double *p;
    int what; /* 0: x, 1: y, 2: z, 3: r^2, 4: psi . (R psi) over all axes */
} moment_ctx;

static double moment_site(const void *c, size_t s, int ix, int iy, int iz)
{
    const moment_ctx *m = (const moment_ctx *)c;
    const orc_lattice *L = m->L;
    double w = m->p[s] * m->p[s];
    switch (m->what) {
    case 0: return coord(L, ix) * w;
    case 1: return coord(L, iy) * w;
    case 2: return coord(L, iz) * w;
    case 3: {
        double x = coord(L, ix), y = coord(L, iy), z = coord(L, iz);
        return (x * x + y * y + z * z) * w;
    }
    default: {
        int n = L->n;
        size_t r = ((size_t)mirror(L, ix) * n + mirror(L, iy)) * n + mirror(L, iz);
        return m->p[s] * m->p[r];
    }
    }
}

static double moment(const orc_lattice *L, const double *p, int what)
{
    moment_ctx c = {L, p, what};
    return lattice_sum(L->n, moment_site, &c);
}

/* Observables of psi given K psi: Rayleigh-quotient energy, its kinetic and
 * potential parts, the norm, <x>, <y>, <z>, <r^2> about the potential centre and
 * the weight of the even-parity projection 1/2 (1 + <psi|P psi>/<psi|psi>). */
static void observables(const orc_lattice *L, const double *psi, const double *kpsi, const double *v,
                        orc_obs *o)
{
    const int n = L->n;
    double nn = dot(n, psi, psi, NULL);
    double kk = dot(n, psi, kpsi, NULL);
    double vv = dot(n, psi, psi, v);
    o->norm2 = nn;
    o->kinetic = kk / nn;
    o->potential = vv / nn;
    o->energy = (kk + vv) / nn;
    o->x = moment(L, psi, 0) / nn;
    o->y = moment(L, psi, 1) / nn;
    o->z = moment(L, psi, 2) / nn;
    o->r2 = moment(L, psi, 3) / nn;
    o->parity_even = 0.5 * (1.0 + moment(L, psi, 4) / nn);
}

int orc_observe(const orc_lattice *L, int nstates, const double *psi, const double *v, orc_obs *out)
{
    if (!lattice_ok(L) || !valid_length(L->n) || nstates < 1 || !psi || !v || !out) return ORC_EINVAL;
    const size_t n3 = (size_t)L->n * L->n * L->n;
    double *T = (double *)malloc(sizeof(double) * n3);
    double *kpsi = (double *)malloc(sizeof(double) * n3);
    cplx *work = (cplx *)malloc(sizeof(cplx) * n3);
    int st = ORC_ENOMEM;
    if (T && kpsi && work) {
        if (L->kin != 0) orc_kinetic_symbol(L, T);
        st = ORC_OK;
        for (int i = 0; i < nstates && !st; ++i) {
            st = apply_kinetic_with(L, T, psi + i * n3, kpsi, work);
            if (!st) observables(L, psi + i * n3, kpsi, v, &out[i]);
        }
    }
    free(T);
    free(kpsi);
    free(work);
    return st;
}

/* ------------------------------------------------------------------------------ */
/* Reflection projection  P psi = 1/2 (psi(r) + sign psi(R r)),  R reflecting the  */
/* axes set in `axes` (bit 0: x1, bit 1: x2, bit 2: x3; 7 = inversion, the paper's */
/* parity projection; 4 and 2 = the INITSYMMETRY options along x3 and x2).         */
/* ------------------------------------------------------------------------------ */
int orc_project(const orc_lattice *L, double *psi, int sign, int axes)
{
    if (!lattice_ok(L) || !psi || (sign != 1 && sign != -1) || axes < 1 || axes > 7) return ORC_EINVAL;
    const int n = L->n;
    const size_t n3 = (size_t)n * n * n;
    double *src = (double *)malloc(sizeof(double) * n3);
    if (!src) return ORC_ENOMEM;
    memcpy(src, psi, sizeof(double) * n3);
#pragma omp parallel for schedule(static)
    for (int ix = 0; ix < n; ++ix)
        for (int iy = 0; iy < n; ++iy)
            for (int iz = 0; iz < n; ++iz) {
                int rx = (axes & 1) ? mirror(L, ix) : ix;
                int ry = (axes & 2) ? mirror(L, iy) : iy;
                int rz = (axes & 4) ? mirror(L, iz) : iz;
                size_t s = ((size_t)ix * n + iy) * n + iz;
                size_t r = ((size_t)rx * n + ry) * n + rz;
                psi[s] = 0.5 * (src[s] + (double)sign * src[r]);
            }
    free(src);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------ */
/* Gram-Schmidt: state i loses its components along the already orthonormal      */
/* states 0..i-1 (modified Gram-Schmidt, one projection at a time), then is       */
/* normalised so that sum |psi|^2 = 1 over the full lattice.                      */
/* ------------------------------------------------------------------------------ */
static void orthonormalise_one(int n, double *states, int i, int deflate)
{
    const size_t n3 = (size_t)n * n * n;
    double *pi = states + i * n3;
    if (deflate)
        for (int j = 0; j < i; ++j) {
            const double *pj = states + j * n3;
            double c = dot(n, pj, pi, NULL);
#pragma omp parallel for schedule(static)
            for (long s = 0; s < (long)n3; ++s) pi[s] -= c * pj[s];
        }
    double nrm = sqrt(dot(n, pi, pi, NULL));
#pragma omp parallel for schedule(static)
    for (long s = 0; s < (long)n3; ++s) pi[s] /= nrm;
}

int orc_orthonormalise(int n, int nstates, double *states)
{
    if (n < 1 || nstates < 1 || !states) return ORC_EINVAL;
    for (int i = 0; i < nstates; ++i) orthonormalise_one(n, states, i, 1);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------ */
/* The imaginary-time step (paper, equation iter_proced and the A, B factors):    */
/*   psi(tau + dtau) = A psi(tau) - B dtau H_K psi(tau),                          */
/*   A = (1 - dtau V/2) / (1 + dtau V/2),  B = 1 / (1 + dtau V/2).                */
/* Per step, for every state in order: observables of the current state, the      */
/* update, then the optional reflection projection.  After all states: Gram-      */
/* Schmidt in state order when (global step + 1) is a multiple of ortho_every,    */
/* and normalisation of every state.                                              */
/* ------------------------------------------------------------------------------ */
int orc_step(const orc_lattice *L, int nstates, double *psi, const double *v, int nsteps,
             long long step0, int ortho_every, const int *par_sign, const int *par_axes,
             orc_obs *obs_out)
{
    if (!lattice_ok(L) || !valid_length(L->n) || nstates < 1 || !psi || !v || nsteps < 0 ||
        L->dtau <= 0.0)
        return ORC_EINVAL;
    const int n = L->n;
    const size_t n3 = (size_t)n * n * n;
    double *T = (double *)malloc(sizeof(double) * n3);
    double *kpsi = (double *)malloc(sizeof(double) * n3);
    cplx *work = (cplx *)malloc(sizeof(cplx) * n3);
    int st = ORC_OK;
    if (!T || !kpsi || !work) st = ORC_ENOMEM;
    if (!st && L->kin != 0) orc_kinetic_symbol(L, T);
    const double h = 0.5 * L->dtau;
    for (int step = 0; step < nsteps && !st; ++step) {
        for (int i = 0; i < nstates && !st; ++i) {
            double *p = psi + i * n3;
            st = apply_kinetic_with(L, T, p, kpsi, work);
            if (st) break;
            if (obs_out) observables(L, p, kpsi, v, &obs_out[(size_t)step * nstates + i]);
#pragma omp parallel for schedule(static)
            for (long s = 0; s < (long)n3; ++s) {
                double A = (1.0 - h * v[s]) / (1.0 + h * v[s]);
                double B = 1.0 / (1.0 + h * v[s]);
                p[s] = A * p[s] - B * L->dtau * kpsi[s];
            }
            if (par_sign && par_sign[i] != 0) {
                int axes = par_axes ? par_axes[i] : 7;
                st = orc_project(L, p, par_sign[i], axes);
            }
        }
        if (st) break;
        long long global = step0 + step;
        int deflate = ortho_every > 0 && ((global + 1) % ortho_every == 0);
        for (int i = 0; i < nstates; ++i) orthonormalise_one(n, psi, i, deflate);
    }
    free(T);
    free(kpsi);
    free(work);
    return st;
}

/* ------------------------------------------------------------------------------ */
/* Certification of an eigenpair of the step map L = A - B dtau H_K.  With        */
/* D = 1 + dtau V / 2, D L is symmetric, so lambda = <psi|D L psi>/<psi|D psi> is */
/* the Rayleigh quotient of the generalised problem and                           */
/*   resid = ||L psi - lambda psi||_D / ||psi||_D                                 */
/* measures how far psi is from the map's fixed point.  Also returns the energy   */
/* Rayleigh quotient of psi.                                                      */
/* ------------------------------------------------------------------------------ */
int orc_certify(const orc_lattice *L, const double *psi, const double *v, double *lambda,
                double *resid, double *energy)
{
    if (!lattice_ok(L) || !valid_length(L->n) || !psi || !v || L->dtau <= 0.0) return ORC_EINVAL;
    const int n = L->n;
    const size_t n3 = (size_t)n * n * n;
    double *T = (double *)malloc(sizeof(double) * n3);
    double *kpsi = (double *)malloc(sizeof(double) * n3);
    double *lp = (double *)malloc(sizeof(double) * n3);
    double *d = (double *)malloc(sizeof(double) * n3);
    cplx *work = (cplx *)malloc(sizeof(cplx) * n3);
    int st = ORC_ENOMEM;
    if (T && kpsi && lp && d && work) {
        if (L->kin != 0) orc_kinetic_symbol(L, T);
        st = apply_kinetic_with(L, T, psi, kpsi, work);
        if (!st) {
            const double h = 0.5 * L->dtau;
            for (size_t s = 0; s < n3; ++s) {
                d[s] = 1.0 + h * v[s];
                double A = (1.0 - h * v[s]) / d[s];
                double B = 1.0 / d[s];
                lp[s] = A * psi[s] - B * L->dtau * kpsi[s];
            }
            double num = dot(n, psi, lp, d);
            double den = dot(n, psi, psi, d);
            double lam = num / den;
            for (size_t s = 0; s < n3; ++s) lp[s] -= lam * psi[s];
            double rr = dot(n, lp, lp, d);
            if (lambda) *lambda = lam;
            if (resid) *resid = sqrt(rr / den);
            if (energy) {
                double nn = dot(n, psi, psi, NULL);
                *energy = (dot(n, psi, kpsi, NULL) + dot(n, psi, psi, v)) / nn;
            }
        }
    }
    free(T);
    free(kpsi);
    free(lp);
    free(d);
    free(work);
    return st;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
