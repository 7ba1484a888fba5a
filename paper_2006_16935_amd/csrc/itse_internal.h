// Internal declarations shared by the host runtime and the per-precision kernel
// translation units.  Not part of the public ABI (include/itse.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/itse.h"

namespace itse {

constexpr int MAXK = ITSE_MAX_STATES;
constexpr int NT = 256;           // threads per workgroup for every kernel here
constexpr int HIST_CAP = 4096;    // steps of observables kept on the device

// Reduction slots of the inverse (update) pass, per workgroup.
enum RowQ { RQ_PP = 0, RQ_PK, RQ_VPP, RQ_UU, RQ_X, RQ_Y, RQ_Z, RQ_R2, NQR };
// Reduction slots of the momentum-space pass (parity weight via Parseval).
enum ColQ { CQ_NORM = 0, CQ_PAR, NQC };

// Modes of the inverse (update) pass.
// INV_KBUF: K psi_i written to L.kbuf + i N^3 (complex lattices).
enum InvMode { INV_UPDATE = 0, INV_EVAL = 1, INV_KOUT = 2, INV_KBUF = 3 };
// Reduction slots of the complex update kernel, per workgroup.
enum CplxQ { XQ_VIPP = 0, XQ_UU, NQX };
// Modes of the column pass.
enum ColMode { COL_FWD = 0, COL_KIN = 2 };
// Modes of the finalisation kernel.
enum FinMode { FIN_STEP = 0, FIN_EVAL = 1, FIN_NORM_ONLY = 2 };

// Device-resident observables record (mirrors itse_obs).
struct ObsDev {
    long long step;
    double energy, kinetic, potential, norm2, x, y, z, r2, parity_even, energy_imag;
};

// Everything the kernels need to know about one lattice.  Lives in device
// memory; the host writes the constant part at create and the options part
// before steps; the finalisation kernel writes the dynamic part.
struct LatDev {
    // shape and physics
    int n, nstates, kin, sub, center, prec;
    double a, mass, dtau, h;
    // buffers (element type follows prec)
    // raw states: two buffers per state, ub[(step + 0) & 1] holds the current raw
    // arrays, ub[(step + 1) & 1] receives the update (so that the lazily combined
    // current states stay readable while other states' updates are written)
    void *ub[2][MAXK];
    void *spec[MAXK];    // half spectra
    void *v;             // potential
    const void *tw;      // twiddle table exp(-2 pi i e / n), n entries, prec
    const double *ktab;  // per-axis kinetic term, n entries, FP64
    void *kout;          // output of H_K psi for the kinetic-only mode
    // complex lattices (cplx = 1): states 0 and 1 hold Re psi and Im psi with
    // coef[0][0] = coef[1][1], vi the imaginary part of the potential, kbuf
    // 2 N^3 values receiving K Re psi and K Im psi
    int cplx;
    void *vi;
    void *kbuf;
    double *part_cplx;   // [nb_cplx][NQX]
    int nb_cplx;         // transform lattices: nb_rows (one partial per imaginary-part
                         // plane workgroup); H_K^(0) lattices: flat_blocks(n)
    // reduction arena
    double *part_rows;   // [MAXK][nb_rows][NQR]
    double *part_cols;   // [MAXK][nb_cols][NQC]
    double *part_proj;   // [MAXK][nb_proj]
    double *part_gram;   // [nb_gram][MAXK*(MAXK+1)/2]
    int nb_rows, nb_cols, nb_proj, nb_gram;
    int pg_chunks;            // workgroups per plane of the projection/Gram kernel
    // options
    int ortho_every, moments;
    int psign[MAXK], paxes[MAXK];
    int proj_mode;            // 0 no projection, 1 all projected states share proj_axes, 2 mixed axes
    int proj_axes;
    // dynamic state
    double coef[MAXK][MAXK];  // current state i = sum_j coef[j][i] u[j]
    long long step;
    int error;                // bit0 non-finite, bit1 Gram not positive definite, bit2 unstable V
    double fin_sums[MAXK * (NQR + NQC) + MAXK * (MAXK + 1) / 2];
    ObsDev obs[MAXK];
    ObsDev *hist;             // [HIST_CAP][MAXK]
};

// Raw state array j of the current step (which = 0) or of the step being formed
// (which = 1).
__host__ __device__ inline void *state_buf(const LatDev &L, long long step, int which, int j) {
    return L.ub[(int)((step + which) & 1)][j];
}

struct JobRef {
    LatDev *lat;
    int state;
    int pad_;
};

// Kernel schedule for one (n, precision, variant).
struct Sched {
    int split;     // sub-planes per plane (y = r + split * j)
    int nwp;       // waves per plane-pass workgroup
    int cols_w;    // kz columns per column-pass workgroup
    int nwc;       // waves per column-pass workgroup
    int nb_rows, nb_cols, nb_proj, nb_gram;  // partial-sum blocks per state
    int lds_plane, lds_cols;                 // LDS bytes of the two kinds of workgroup
};

// Per-precision launchers (defined in itse_f32.hip / itse_f64.hip).
template <typename R>
struct Launch {
    static bool supported(int n);
    static Sched schedule(int n, int variant);
    static int variants(int n);
    // Passes over a group of jobs sharing n; jobs is a device array of njobs entries.
    // kmax: the largest number of states among the jobs' lattices
    static hipError_t plane_fwd(int n, int variant, int kmax, const JobRef *jobs, int njobs, hipStream_t s);
    static hipError_t columns(int n, int variant, int mode, int moments, const JobRef *jobs, int njobs, void *out,
                              hipStream_t s);
    // moments: some job's lattice sums position moments (else they are left at zero)
    static hipError_t plane_inv(int n, int variant, int mode, int moments, int kmax, const JobRef *jobs, int njobs,
                                hipStream_t s);
    static hipError_t project(int n, const JobRef *jobs, int njobs, int force_sign, int force_axes, int which,
                              hipStream_t s);
    static hipError_t project_gram(int n, int kmax, const JobRef *lats, int nlats, int force, int which,
                                   hipStream_t s);
    static hipError_t combine(int n, const JobRef *jobs, int njobs, void *const *outs, hipStream_t s);
    // complex lattices: the imaginary parts' inverse pass with the complex update
    // (jobs: state 1 of each lattice; after the real parts' pass in mode INV_KBUF;
    // without position moments)
    static hipError_t plane_inv_cplx(int n, int variant, const JobRef *jobs, int njobs, hipStream_t s);
    // complex lattices: the separate complex update after the transforms in mode
    // INV_KBUF (mode INV_UPDATE or INV_EVAL); nb workgroups per lattice, the
    // lattices' nb_cplx
    static hipError_t complex_update(int n, int nb, const JobRef *lats, int nlats, int mode, hipStream_t s);
    // H_K^(0) lattices: stencil, update and sums in one pass (modes of plane_inv)
    static hipError_t fdtd(int n, int kmax, int mode, const JobRef *jobs, int njobs, hipStream_t s);
    static int fdtd_blocks(int n);
    // analysis of one job's state: parts holds analyse_parts(n) doubles, out NAQ
    static hipError_t analyse(int n, const JobRef *job, double half, double *parts, double *out, hipStream_t s);
    static size_t analyse_parts(int n);
    // radial binning of a standard-layout half spectrum: parts holds
    // n * (3 nbins + 1) doubles, out 3 nbins + 1
    static hipError_t momentum_bins(int n, const void *spec, int nbins, double *parts, double *out, hipStream_t s);
    static hipError_t convert_in(const void *src, int src_dtype, void *dst, size_t count, hipStream_t s);
    static hipError_t convert_out(const void *src, void *dst, int dst_dtype, size_t count, hipStream_t s);
};

hipError_t launch_finalize(const JobRef *lats, int nlats, int mode, hipStream_t s);
hipError_t launch_check_potential(const LatDev *lat, int prec, hipStream_t s);

// Workgroups of the flat kernels (Gram sums, combination): a fixed count per n,
// so that the partial-sum layout and the summation order do not change.
// Row stride (complex values) of the stored half spectra along kz: N/2 + 1 rounded
// up to whole 128-byte lines.
template <typename R>
__host__ __device__ constexpr int spec_row_stride(int n) {
    constexpr int per_line = 128 / (2 * (int)sizeof(R));
    return ((n / 2 + 1 + per_line - 1) / per_line) * per_line;
}
inline size_t spec_bytes(int n, int prec) {
    const size_t hs = prec == ITSE_FP32 ? spec_row_stride<float>(n) : spec_row_stride<double>(n);
    const size_t w = prec == ITSE_FP32 ? 4 : 8;
    return (size_t)n * n * hs * 2 * w;
}

// Units per plane of the projection/Gram kernel (about 4096 sites each), and its
// workgroups (at most 2048, each taking units in a stride; one partial each).
inline int pg_chunks(int n) {
    const int c = n * n / 4096;
    return c < 1 ? 1 : c;
}
inline int pg_blocks(int n) {
    const int u = n * pg_chunks(n);
    return u < 2048 ? u : 2048;
}

inline int flat_blocks(int n) {
    const long long n3 = (long long)n * n * n;
    const long long b = (n3 + 4 * NT - 1) / (4 * NT);
    return (int)(b < 1024 ? b : 1024);
}

}  // namespace itse
