// Finalisation of a step (sums of the per-workgroup partials, then observables
// and coefficients) as tile functions, shared by its kernels and the persistent
// batch kernel.
#pragma once

#include "itse_internal.h"
#include "itse_pass.h"

namespace itse {

constexpr int FIN_NT = 512;  // threads of the sums kernel (the order of its sums)
// Largest number of sums one lattice needs: rows and columns of every state, Gram.
constexpr int FIN_QMAX = MAXK * (NQR + NQC) + MAXK * (MAXK + 1) / 2;

// Which sums a finalisation forms: K * NQR row sums, K * NQC column sums (when
// moments are on), when Gram sums exist the K (K + 1) / 2 Gram entries, and for
// complex lattices the NQX sums of the complex update.  Gram sums of the updated
// (and projected) arrays exist on orthogonalisation steps and whenever states are
// projected (their diagonal then gives the norms).  A complex lattice (K = 2: the
// real and imaginary parts) is never orthogonalised.
struct FinLayout {
    bool ortho_step, have_gram;
    int q_rows, q_cols, q_gram, q_cplx, total;
};

__device__ __forceinline__ FinLayout fin_layout(const LatDev &L, int mode) {
    FinLayout f;
    const int K = L.nstates;
    f.ortho_step = (mode == FIN_STEP) && !L.cplx && K > 1 && L.ortho_every > 0 &&
                   ((L.step + 1) % L.ortho_every) == 0;
    f.have_gram = (mode == FIN_STEP) && (f.ortho_step || L.proj_mode != 0);
    f.q_rows = K * NQR;
    // the parity weight comes from the column pass (Parseval), which H_K^(0)
    // lattices do not run
    f.q_cols = (L.moments && L.kin != ITSE_KIN_FDTD) ? K * NQC : 0;
    f.q_gram = f.have_gram ? K * (K + 1) / 2 : 0;
    f.q_cplx = L.cplx ? NQX : 0;
    f.total = f.q_rows + f.q_cols + f.q_gram + f.q_cplx;
    return f;
}

// Finalisation, first part: workgroup (q, lattice) forms sum number q of the
// lattice from the per-workgroup partials of the step's passes, in a fixed order
// (that of FIN_NT threads: thread v adds up to 8 partials per round, then wave and
// workgroup sums), and stores it in the lattice record.  NTH threads run it, each
// standing for FIN_NT / NTH of the FIN_NT (the sums are the same for either).
// red: FIN_NT / 64 doubles of LDS.
template <int NTH>
__device__ __forceinline__ void fin_sums_tile(const JobRef *__restrict__ lats, int q, int ly, int mode, double *red) {
    constexpr int NG = MAXK * (MAXK + 1) / 2;
    constexpr int VPT = FIN_NT / NTH;  // virtual threads per thread
    static_assert(FIN_NT % NTH == 0 && NTH % 64 == 0, "whole virtual waves");
    LatDev &L = *lats[ly].lat;
    const FinLayout f = fin_layout(L, mode);
    if (q >= f.total) return;
    const double *p;
    int count, stride;
    if (q < f.q_rows) {
        const int i = q / NQR, c = q % NQR;
        p = L.part_rows + (size_t)i * L.nb_rows * NQR + c;
        count = L.nb_rows;
        stride = NQR;
    } else if (q < f.q_rows + f.q_cols) {
        const int t = q - f.q_rows, i = t / NQC, c = t % NQC;
        p = L.part_cols + (size_t)i * L.nb_cols * NQC + c;
        count = L.nb_cols;
        stride = NQC;
    } else if (q < f.q_rows + f.q_cols + f.q_gram) {
        const int slot = q - f.q_rows - f.q_cols;  // l (l + 1) / 2 + j
        p = L.part_gram + slot;
        count = L.nb_gram;
        stride = NG;
    } else {
        p = L.part_cplx + (q - f.q_rows - f.q_cols - f.q_gram);
        count = L.nb_cplx;
        stride = NQX;
    }
    // up to 8 loads in flight per virtual thread, added in a fixed order
    double acc[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        acc[u] = 0.0;
        const int vt = threadIdx.x + u * NTH;
        for (int b0 = 0; b0 < count; b0 += 8 * FIN_NT) {
            double v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int b = b0 + t * FIN_NT + vt;
                v[t] = b < count ? p[(size_t)b * stride] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) acc[u] += v[t];
        }
    }
    // the workgroup sum of FIN_NT virtual threads: wave sums (virtual wave w + 4 u of
    // thread u's copy), then the FIN_NT / 64 wave sums in order
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const double sw = wave_sum(acc[u]);
        if (lane == 0) red[u * (NTH / 64) + wv] = sw;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < FIN_NT / 64; ++w) t += red[w];
        L.fin_sums[q] = t;
    }
}

// Finalisation, second kernel (one wave per lattice): the observables of the
// states at the start of the step (lane i: state i), and on step finalisation
// the coefficients of the new states in terms of the raw updated arrays:
// Gram-Schmidt in state order as G = R^T R (Cholesky, R upper triangular), new
// states U R^{-1}, or the normalisation alone.  A non-finite or non-positive sum
// sets the lattice's error flags and keeps the previous coefficients.
// LDS of the tail: sums, the coefficient matrix, R and the error flags of the lanes.
struct FinTailLds {
    double sums[FIN_QMAX];
    double M[MAXK][MAXK];
    double Rm[MAXK][MAXK];
    int errs[64];
};

// The tail for lattice ly, run by the threads of one workgroup: threads 0..63 do the
// work (one wave's lanes), any further threads only take the barriers.
__device__ __forceinline__ void fin_tail_tile(const JobRef *__restrict__ lats, int ly, int mode, FinTailLds &sh) {
    LatDev &L = *lats[ly].lat;
    const FinLayout f = fin_layout(L, mode);
    const int K = L.nstates;
    const int lane = threadIdx.x;
    double *sums = sh.sums;
    auto &M = sh.M;
    auto &Rm = sh.Rm;
    int *errs = sh.errs;
    for (int t = lane; t < f.total; t += 64)
        if (lane < 64) sums[t] = L.fin_sums[t];
    __syncthreads();
    int err = 0;
    // a complex lattice: one observable record from the sums of both parts
    const int nobs = L.cplx ? 1 : K;
    if (L.cplx && lane == 0) {
        for (int c = 0; c < NQR; ++c) sums[c] += sums[NQR + c];
        if (f.q_cols)
            for (int c = 0; c < NQC; ++c) sums[f.q_rows + c] += sums[f.q_rows + NQC + c];
    }
    __syncthreads();
    const double *xs = sums + f.q_rows + f.q_cols + f.q_gram;  // complex-update sums
    if (lane < nobs) {
        const double *rows = sums + lane * NQR;
        const double *cols = sums + f.q_rows + lane * NQC;
        ObsDev o;
        const double pp = rows[RQ_PP];
        o.step = L.step;
        o.norm2 = pp;
        o.kinetic = rows[RQ_PK] / pp;
        o.potential = rows[RQ_VPP] / pp;
        o.energy = (rows[RQ_PK] + rows[RQ_VPP]) / pp;
        if (L.moments) {
            o.x = rows[RQ_X] / pp;
            o.y = rows[RQ_Y] / pp;
            o.z = rows[RQ_Z] / pp;
            o.r2 = rows[RQ_R2] / pp;
            o.parity_even = f.q_cols ? 0.5 * (1.0 + cols[CQ_PAR] / cols[CQ_NORM]) : -1.0;
        } else {
            o.x = o.y = o.z = o.r2 = 0.0;
            o.parity_even = -1.0;
        }
        o.energy_imag = L.cplx ? xs[XQ_VIPP] / pp : 0.0;
        if (!isfinite(o.energy) || !isfinite(o.energy_imag) || !isfinite(pp) || pp <= 0.0) err |= 1;
        L.obs[lane] = o;
        if (mode == FIN_STEP && L.hist) L.hist[(size_t)(L.step % HIST_CAP) * MAXK + lane] = o;
    }
    if (mode == FIN_STEP && lane == 0) {
        const double *gram = sums + f.q_rows + f.q_cols;
        for (int j = 0; j < MAXK; ++j)
            for (int i = 0; i < MAXK; ++i) M[j][i] = 0.0;
        bool done = false;
        if (f.ortho_step) {
            bool ok = true;
            for (int j = 0; j < K && ok; ++j) {
                for (int i = j; i < K; ++i) {
                    double s = gram[i * (i + 1) / 2 + j];
                    for (int l = 0; l < j; ++l) s -= Rm[l][j] * Rm[l][i];
                    if (i == j) {
                        if (!(s > 0.0) || !isfinite(s)) {
                            ok = false;
                            break;
                        }
                        Rm[j][j] = sqrt(s);
                    } else {
                        Rm[j][i] = s / Rm[j][j];
                    }
                }
            }
            if (ok) {
                for (int i = 0; i < K; ++i) {
                    M[i][i] = 1.0 / Rm[i][i];
                    for (int j = i - 1; j >= 0; --j) {
                        double s = 0.0;
                        for (int l = j + 1; l <= i; ++l) s += Rm[j][l] * M[l][i];
                        M[j][i] = -s / Rm[j][j];
                    }
                }
                done = true;
            } else {
                err |= 2;
            }
        }
        if (!done && L.cplx) {
            // |psi'|^2 summed over both parts; one coefficient for both
            const double nn = f.have_gram ? gram[0] + gram[2] : xs[XQ_UU];
            if (!(nn > 0.0) || !isfinite(nn)) err |= 1;
            M[0][0] = M[1][1] = 1.0 / sqrt(nn);
        } else if (!done) {
            for (int i = 0; i < K; ++i) {
                const double nn = f.have_gram ? gram[i * (i + 1) / 2 + i] : sums[i * NQR + RQ_UU];
                if (!(nn > 0.0) || !isfinite(nn)) err |= 1;
                M[i][i] = 1.0 / sqrt(nn);
            }
        }
    }
    __syncthreads();
    // one coefficient per lane
    static_assert(MAXK * MAXK == 64, "one coefficient per lane");
    const double mv = (mode == FIN_STEP && lane < 64) ? M[lane / MAXK][lane % MAXK] : 0.0;
    if (!isfinite(mv)) err |= 1;
    if (lane < 64) errs[lane] = err;
    __syncthreads();
    int all = 0;
    for (int t = 0; t < 64; ++t) all |= errs[t];
    if (mode == FIN_STEP && !all && lane < 64) L.coef[lane / MAXK][lane % MAXK] = mv;
    if (lane == 0) {
        L.error |= all;
        if (mode == FIN_STEP) L.step += 1;
    }
}

}  // namespace itse
