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
enum InvMode { INV_UPDATE = 0, INV_EVAL = 1, INV_KOUT = 2 };
// Modes of the strided-axis transform pass.
enum ColMode { COL_FWD = 0, COL_INV = 1, COL_KIN = 2 };
// Modes of the finalisation kernel.
enum FinMode { FIN_STEP = 0, FIN_EVAL = 1, FIN_NORM_ONLY = 2 };

// Device-resident observables record (mirrors itse_obs).
struct ObsDev {
    long long step;
    double energy, kinetic, potential, norm2, x, y, z, r2, parity_even;
};

// Everything the kernels need to know about one lattice.  Lives in device
// memory; the host writes the constant part at create and the options part
// before steps; the finalisation kernel writes the dynamic part.
struct LatDev {
    // shape and physics
    int n, nstates, kin, sub, center, prec;
    double a, mass, dtau, h;
    // buffers (element type follows prec)
    void *u[MAXK];       // raw states after the last update
    void *phi[MAXK];     // current states (materialised at the start of a step)
    void *spec[MAXK];    // half spectra
    void *v;             // potential
    const void *tw;      // twiddle table exp(-2 pi i e / n), n entries, prec
    const double *ktab;  // per-axis kinetic term, n entries, FP64
    void *kout;          // output of H_K psi for the kinetic-only mode
    // reduction arena
    double *part_rows;   // [MAXK][nb_rows][NQR]
    double *part_cols;   // [MAXK][nb_cols][NQC]
    double *part_proj;   // [MAXK][nb_proj]
    double *part_gram;   // [nb_gram][MAXK*(MAXK+1)/2]
    int nb_rows, nb_cols, nb_proj, nb_gram;
    // options
    int ortho_every, moments;
    int psign[MAXK], paxes[MAXK];
    // dynamic state
    double coef[MAXK][MAXK];  // current state i = sum_j coef[j][i] u[j]
    long long step;
    int error;                // bit0 non-finite, bit1 Gram not positive definite, bit2 unstable V
    int pad_;
    ObsDev obs[MAXK];
    ObsDev *hist;             // [HIST_CAP][MAXK]
};

struct JobRef {
    LatDev *lat;
    int state;
    int pad_;
};

// Kernel schedule for one (n, precision).
struct Sched {
    int rows_rp;   // row pairs per workgroup in the row passes
    int cols_w;    // columns per workgroup in the strided passes
    int nb_rows, nb_cols, nb_proj, nb_gram;
};

// Per-precision launchers (defined in itse_f32.hip / itse_f64.hip).
template <typename R>
struct Launch {
    static bool supported(int n);
    static Sched schedule(int n, int variant);
    static int variants(int n);
    // Passes over a group of jobs sharing n; jobs is a device array of njobs entries.
    static hipError_t rows_fwd(int n, int variant, const JobRef *jobs, int njobs, hipStream_t s);
    static hipError_t cols(int n, int variant, int mode, int axis, int moments, const JobRef *jobs,
                           int njobs, hipStream_t s);
    static hipError_t rows_inv(int n, int variant, int mode, const JobRef *jobs, int njobs,
                               hipStream_t s);
    static hipError_t project(int n, const JobRef *jobs, int njobs, int force_sign, int force_axes,
                              hipStream_t s);
    static hipError_t gram(int n, const JobRef *lats, int nlats, int force, hipStream_t s);
    static hipError_t combine(int n, const JobRef *jobs, int njobs, void *const *outs, hipStream_t s);
    static hipError_t convert_in(const void *src, int src_dtype, void *dst, size_t count, hipStream_t s);
    static hipError_t convert_out(const void *src, void *dst, int dst_dtype, size_t count, hipStream_t s);
};

hipError_t launch_finalize(const JobRef *lats, int nlats, int mode, hipStream_t s);
hipError_t launch_check_potential(const LatDev *lat, int prec, hipStream_t s);

// Number of sites per thread in the flat (projection, Gram) kernels.
constexpr int FLAT_SPT = 4;

inline int flat_blocks(int n) {
    long long n3 = (long long)n * n * n;
    long long per = (long long)NT * FLAT_SPT;
    return (int)((n3 + per - 1) / per);
}

}  // namespace itse
