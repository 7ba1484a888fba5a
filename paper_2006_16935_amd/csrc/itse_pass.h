// Device code of the three-pass imaginary-time step (included once per
// precision by itse_f32.hip / itse_f64.hip).
//
// The step applies, per state, psi' = A psi - B dtau H_K psi with
// H_K psi = IFFT[T(k) FFT[psi]] / N^3 (the paper's equation iter_proced and its
// kinetic terms H_K^(1..3)).  The 3D transform is split over three passes that
// each read and write HBM once:
//
//   P1 (plane, forward)  sub-plane (x, r) = rows y = r + S j of plane x:
//                        R2C along z (two real rows packed as one complex row),
//                        complex FFT of length M = N/S along j.
//   P2 (columns)         for (y', kz-chunk): radix-S combination of the S
//                        sub-spectra (completing the y transform), FFT along x,
//                        multiply by T(k)/N^3 (symbol evaluated in FP64 and rounded
//                        once to the lattice precision), inverse FFT along x,
//                        inverse radix-S split.
//   P3 (plane, inverse)  length-M inverse FFT along j, C2R along z, then the
//                        update and FP64 partial sums of <psi|psi>, <psi|K psi>,
//                        <psi|V psi>, <psi'|psi'> (and moments).
//
// The split of the y axis: with y = r + S j and ky = ky' + M q,
//   X[ky' + M q] = sum_r w_S^(r q) w_N^(r ky') S_r[ky'],  S_r[ky'] = sum_j x_(r+Sj) w_M^(j ky'),
// and the inverse mirrors it.  Spectrum storage per state: S sub-spectra
// [r][x][ky'][kz], kz = 0..N/2 (private to these passes).
//
// Current states are kept lazily: psi_i = sum_(j<=i) coef[j][i] u_j, formed in
// FP64 from the raw updated arrays u_j on every load (normalisation and
// Gram-Schmidt cost no extra pass).
#pragma once

#include <type_traits>

#include "itse_fft.h"
#include "itse_internal.h"

namespace itse {

// Pointers into device memory that the compiler should address as global memory
// (global_load/store instead of flat accesses, which also count against the LDS
// wait counter).
#if defined(__HIP_DEVICE_COMPILE__)
#define ITSE_GLOBAL __attribute__((address_space(1)))
#else
#define ITSE_GLOBAL
#endif
template <typename T>
__device__ __forceinline__ ITSE_GLOBAL T *gmem(T *p) {
    return (ITSE_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ const ITSE_GLOBAL T *gmem(const T *p) {
    return (const ITSE_GLOBAL T *)p;
}

// Workgroup index remapped so that consecutive indices run on one XCD: the
// hardware hands workgroup b to XCD b mod 8, so XCD k gets the contiguous range
// [k nb/8, (k+1) nb/8) in dispatch order (a tail of nb mod 8 keeps its index).
__device__ __forceinline__ int xcd_local_index(int b, int nb) {
    const int full = nb & ~7;
    if (b >= full) return b;
    return (b & 7) * (full >> 3) + (b >> 3);
}

// Workgroup order of the plane passes: the jobs of one sub-plane are dispatched
// 8 workgroups apart, so that they run on the same XCD (the hardware hands
// workgroup b to XCD b mod 8) at nearly the same time and share the sub-plane's
// rows of the lower states and of V in that XCD's L2.  With NB % 8 == 0 the grid
// is (8 nj, NB / 8): x = job * 8 + (sub-plane mod 8), y = sub-plane / 8; else
// (NB, nj).  Returns the sub-plane and sets the job index (no division).
template <int NB>
__device__ __forceinline__ int plane_block(int &job) {
    if constexpr (NB % 8 == 0) {
        job = blockIdx.x >> 3;
        return blockIdx.y * 8 + (blockIdx.x & 7);
    }
    job = blockIdx.y;
    return blockIdx.x;
}
template <int NB>
inline dim3 plane_grid(int njobs) {
    return NB % 8 == 0 ? dim3(8 * njobs, NB / 8) : dim3(NB, njobs);
}

// ---------------------------------------------------------------------------
// Schedules: split factor S (sub-planes per plane), waves per workgroup in the
// plane passes (NWP) and the column pass (NWC), kz columns per column-pass
// workgroup (W).  Variant V selects among
// the alternatives the autotuner times.
// ---------------------------------------------------------------------------
template <typename R, int N, int V>
struct Plan;

#define ITSE_PLAN(RT, NN, VV, S_, NWP_, W_, NWC_)                 \
    template <>                                                   \
    struct Plan<RT, NN, VV> {                                     \
        static constexpr int S = S_, NWP = NWP_, W = W_, NWC = NWC_; \
    };

// Column-pass chunks of W complex values are 128 bytes (W = 16 FP32, 8 FP64) from
// N = 48 up, so that the strided reads along x fetch whole cache lines.
// FP32: variant 0 is the default.
ITSE_PLAN(float, 8, 0, 1, 1, 5, 1)
ITSE_PLAN(float, 12, 0, 1, 1, 7, 1)
ITSE_PLAN(float, 16, 0, 1, 2, 9, 1)
ITSE_PLAN(float, 24, 0, 1, 2, 13, 1)
ITSE_PLAN(float, 32, 0, 1, 4, 17, 1)
ITSE_PLAN(float, 48, 0, 1, 4, 16, 1)
ITSE_PLAN(float, 64, 0, 1, 4, 16, 1)
ITSE_PLAN(float, 96, 0, 1, 4, 16, 2)
// the batch sizes: column workgroups of four waves (one kz chunk of W = 20 at
// N = 32: the whole half row), and the y axis split in two (twice the plane
// workgroups, for batches of few lattices).  N = 32 variant 2 and N = 96 variant
// 3: plane workgroups of two and three waves, so that each wave owns a whole
// number of 64-lane rounds of four-value chunks (64 and 192 chunks; four waves
// own 32 and 144)
ITSE_PLAN(float, 32, 1, 1, 4, 20, 4)
ITSE_PLAN(float, 32, 2, 1, 2, 20, 4)
ITSE_PLAN(float, 48, 1, 1, 4, 16, 4)
ITSE_PLAN(float, 48, 2, 2, 4, 16, 4)
ITSE_PLAN(float, 64, 1, 1, 4, 16, 4)
ITSE_PLAN(float, 64, 2, 2, 4, 16, 4)
ITSE_PLAN(float, 96, 1, 1, 4, 16, 4)
ITSE_PLAN(float, 96, 2, 2, 4, 16, 4)
ITSE_PLAN(float, 96, 3, 2, 3, 16, 4)
ITSE_PLAN(float, 128, 0, 1, 8, 16, 2)
ITSE_PLAN(float, 128, 1, 2, 4, 16, 4)
ITSE_PLAN(float, 192, 0, 2, 8, 16, 8)
ITSE_PLAN(float, 256, 0, 4, 8, 16, 16)
ITSE_PLAN(float, 256, 1, 2, 8, 16, 8)
ITSE_PLAN(float, 256, 2, 4, 8, 8, 8)
ITSE_PLAN(float, 256, 3, 4, 8, 4, 4)
ITSE_PLAN(float, 256, 4, 8, 4, 4, 8)
// variant 5: variant 2's layout (S = 4), forward pass and column pass; the inverse
// plane pass on the sub-planes of variant 4 (see PassVariants)
ITSE_PLAN(float, 256, 5, 4, 8, 8, 8)
// FP64
ITSE_PLAN(double, 8, 0, 1, 1, 5, 1)
ITSE_PLAN(double, 12, 0, 1, 1, 7, 1)
ITSE_PLAN(double, 16, 0, 1, 2, 9, 1)
ITSE_PLAN(double, 24, 0, 1, 2, 13, 1)
ITSE_PLAN(double, 32, 0, 1, 4, 17, 1)
ITSE_PLAN(double, 48, 0, 1, 4, 8, 1)
ITSE_PLAN(double, 64, 0, 1, 4, 8, 1)
ITSE_PLAN(double, 96, 0, 1, 4, 8, 2)
ITSE_PLAN(double, 128, 0, 2, 4, 8, 2)
ITSE_PLAN(double, 192, 0, 4, 4, 8, 8)
ITSE_PLAN(double, 256, 0, 4, 8, 8, 8)
ITSE_PLAN(double, 256, 1, 8, 4, 4, 8)
#undef ITSE_PLAN

// The schedules each pass of variant V runs: the forward plane pass under FWD, the
// column pass under COLS (whose split S fixes the layout of the sub-spectra; FWD
// writes it), the inverse plane pass under INV.  SPLIT_INV: the inverse pass
// computes on twice as many sub-planes as the layout has; each of its workgroups
// takes one half of a layout sub-plane's rows, joined to the layout by a radix-2
// step of the y transform as the rows are loaded.  It then holds half a layout
// sub-plane in LDS, while the column pass keeps the layout's longer row pieces.
template <typename R, int N, int V>
struct PassVariants {
    static constexpr int FWD = V, COLS = V, INV = V;
    static constexpr bool SPLIT_INV = false;
};
// 256^3 FP32: the layout of variant 2 (S = 4), the inverse pass under variant 4 (S = 8)
template <>
struct PassVariants<float, 256, 5> {
    static constexpr int FWD = 2, COLS = 2, INV = 4;
    static constexpr bool SPLIT_INV = true;
};

template <typename R, int N, int V>
struct Geo {
    using PL = Plan<R, N, V>;
    static constexpr int S = PL::S, NWP = PL::NWP, W = PL::W, NWC = PL::NWC;
    static constexpr int H = N / 2 + 1;
    static constexpr int M = N / S;
    static constexpr int PAIRS = M / 2;
    static_assert(M % 2 == 0, "sub-planes hold pairs of rows");
    static_assert(PAIRS % NWP == 0, "pairs split evenly over waves");
    static_assert((N / 2) % NWP == 0, "columns split evenly over waves");
    static constexpr int PPW = PAIRS / NWP;     // row pairs per wave
    static constexpr int CPW = (N / 2) / NWP;   // kz columns per wave (the kz = N/2 column extra)
    // Row stride of the plane layout: room for a padded z transform in two rows
    // (2 HP >= span), and HP = 8 mod 16 (FP32) or 4 mod 8 (FP64) so that the
    // rows fall on different banks.
    static constexpr int SPANZ = WaveFft<R, N, 1, -1, false, 1>::SPAN;
    static constexpr int HMIN = (SPANZ + 1) / 2 > H ? (SPANZ + 1) / 2 : H;
    static constexpr int HMOD = sizeof(R) == 4 ? 16 : 8;
    static constexpr int HOFF = sizeof(R) == 4 ? 8 : 4;
    static constexpr int HP = HMIN + ((HOFF - HMIN % HMOD) + HMOD) % HMOD;
    static constexpr int LSZ = 2 * HP;
    static constexpr int PLANE_ELEMS = M * HP;
    static constexpr int NTP = 64 * NWP;
    // plane workgroups that fit one CU's 160 KiB of LDS (at most 4), and the waves
    // per SIMD they need (caps the registers so that they do fit)
    static constexpr int LDS_PLANE = PLANE_ELEMS * (int)sizeof(C2<R>) + N * (int)sizeof(C2<R>) + 64 * NQR;
    static constexpr int WG_FIT = 163840 / LDS_PLANE;
    static constexpr int WG_CU = WG_FIT >= 4 ? 4 : WG_FIT >= 2 ? WG_FIT : 1;
    static constexpr int WPE = (WG_CU * NWP + 3) / 4 > 1 ? (WG_CU * NWP + 3) / 4 : 1;
    // Column pass
    static constexpr int NCH = (H + W - 1) / W;      // kz chunks
    // Row stride of the stored sub-spectra: H rounded up to whole 128-byte lines,
    // so that the column pass's chunks of W values start on a line.
    static constexpr int HS = spec_row_stride<R>(N);
    static constexpr int LINES = S * W;              // x lines per column workgroup
    static_assert(LINES % NWC == 0, "lines split evenly over waves");
    static constexpr int LPWC = LINES / NWC;
    // Row stride (x) of the column layout: the smallest CS >= LINES with
    // CS = 4 (mod 8).  Consecutive rows then start 8 x odd banks apart (FP32; 16 x odd
    // for FP64), so 8 (4) successive rows fall on distinct groups of banks, which
    // spreads both the butterfly accesses (a few lines x 16 rows) and the row-wise
    // load/store accesses over all banks.
    static constexpr int CS = LINES + ((4 - LINES % 8) + 8) % 8;
    static constexpr int NTC = 64 * NWC;
    // column workgroups that fit one CU's LDS (at most 4) and the waves per SIMD they need
    static constexpr int LDS_COLS = N * CS * (int)sizeof(C2<R>) + N * (int)sizeof(C2<R>) + N * 8 + 64 * NQC;
    static constexpr int WGC_CU = (163840 / LDS_COLS) >= 4 ? 4 : (163840 / LDS_COLS) < 1 ? 1 : (163840 / LDS_COLS);
    static constexpr int WPEC = (WGC_CU * NWC + 3) / 4 > 1 ? (WGC_CU * NWC + 3) / 4 : 1;
    static constexpr int NB_PLANE = N * S;           // plane workgroups per state
    static constexpr int NB_COLS = M * NCH;          // column workgroups per state
};

// Coordinate of index idx about the potential centre (cell centre (n-1)/2, or
// origin with minimum image).
__device__ __forceinline__ double site_coord(int idx, int n, int center, double a) {
    if (center == ITSE_CENTER_CELL) return ((double)idx - 0.5 * (double)(n - 1)) * a;
    return (double)((2 * idx <= n) ? idx : idx - n) * a;
}

__device__ __forceinline__ int mirror_idx(int idx, int n, int center) {
    return center == ITSE_CENTER_CELL ? n - 1 - idx : (idx == 0 ? 0 : n - idx);
}

// Kinetic symbol forms: the table sum itself (non-relativistic kinds),
// sqrt(p^2 + m^2), and sqrt(p^2 + m^2) - m written as p^2 / (sqrt(p^2 + m^2) + m).
enum SymKind { SYM_SUM = 0, SYM_REL = 1, SYM_REL_SUB = 2 };

// T / N^3 for the table sum s.  FP64 lattices: correctly rounded FP64 operations.
// FP32 lattices: T evaluated in FP64 and rounded once to FP32.  The square root
// and the reciprocal start from the FP32 hardware estimates (about 1e-7 relative)
// and take one Newton-Raphson step in FP64 (y <- y (3 - x y^2)/2 for x^-1/2,
// q <- q (2 - d q) for 1/d), which squares the relative error to ~1e-14, far
// below FP32's half ulp; T then carries only the one rounding to FP32, with no
// bias from the estimates (an error in T enters the energy at first order).
template <typename R, int KIND>
__device__ __forceinline__ R symbol_scaled(double s, double mass, double inv_n3) {
    if constexpr (sizeof(R) == 4) {
        double t = s;
        if constexpr (KIND != SYM_SUM) {
            const double x = s + mass * mass;
            double y = (double)__builtin_amdgcn_rsqf((float)x);
            y = y * (1.5 - 0.5 * x * y * y);
            const double e = x * y;
            if constexpr (KIND == SYM_REL) {
                t = e;
            } else {
                const double d = e + mass;
                double q = (double)__builtin_amdgcn_rcpf((float)d);
                q = q * (2.0 - d * q);
                t = s * q;
            }
        }
        return (R)(t * inv_n3);
    } else {
        double t = s;
        if constexpr (KIND != SYM_SUM) {
            const double e = sqrt(s + mass * mass);
            t = KIND == SYM_REL ? e : s / (e + mass);
        }
        return t * inv_n3;
    }
}

// Multiply one x line of the column layout (stride CS) by T(kx, ky, kz) / N^3 at
// kx = kx0, kx0 + KSTEP, ...; `cl` is the line's table sum over ky and kz.
template <typename R, int KIND, int N, int KSTEP, int CS>
__device__ __forceinline__ void multiply_line(C2<R> *line, const double *ktab, int kx0, double cl, double mass,
                                              double inv_n3) {
    constexpr int NE = N / KSTEP;
#pragma unroll
    for (int k = 0; k < NE; ++k) {
        const int kx = kx0 + KSTEP * k;
        const R t = symbol_scaled<R, KIND>(ktab[kx] + cl, mass, inv_n3);
        C2<R> v = line[kx * CS];
        v.x *= t;
        v.y *= t;
        line[kx * CS] = v;
    }
}

// a / b: times the hardware reciprocal for FP32 lattices (about 1 ulp, below the
// transforms' rounding), correctly rounded division for FP64 lattices.
template <typename R>
__device__ __forceinline__ R div_fast(R a, R b) {
    if constexpr (sizeof(R) == 4) return a * __builtin_amdgcn_rcpf(b);
    else return a / b;
}

// Wave-level fixed-order sum of a double over the 64 lanes (lane 0 gets it).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// The thread's index within its workgroup, hidden from loop-invariant code motion:
// a tile run inside a loop over tiles (the persistent batch kernel) then forms its
// per-thread addresses inside each tile, instead of hoisting them all before the
// loop where they would stay live across every tile's transforms.
__device__ __forceinline__ int tile_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    __builtin_assume(t >= 0 && t < 1024);
    return t;
}

// Fixed-order workgroup sums of Q doubles; thread 0 writes dst[0..Q).
template <int Q, int NTH>
__device__ __forceinline__ void block_sums(double (&acc)[Q], double *dst, double *lds) {
    constexpr int NWV = NTH / 64;
    const int tid = tile_tid(), lane = tid & 63, wv = tid >> 6;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const double s = wave_sum(acc[q]);
        if (lane == 0) lds[q * NWV + wv] = s;
    }
    __syncthreads();
    if (tid < Q) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NWV; ++w) s += lds[tid * NWV + w];
        dst[tid] = s;
    }
}

// Lattice fields used by the passes, copied out of the device record once; KM
// bounds the number of states of the lattices a launch serves (i < KM).
template <typename R, int KM = MAXK>
struct LatView {
    const ITSE_GLOBAL R *u[KM];
    double c[KM];
    int i;
};

template <typename R, int KM>
__device__ __forceinline__ void load_view(LatView<R, KM> &vw, const LatDev &L, int i) {
    vw.i = i;
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        vw.u[j] = gmem((const R *)state_buf(L, L.step, 0, j));
        vw.c[j] = (j <= i) ? L.coef[j][i] : 0.0;
    }
}

// Destination of K psi_i in the modes that write it.
template <typename R>
__device__ __forceinline__ R *kout_ptr(const LatDev &L, int mode, int i) {
    return mode == INV_KBUF ? (R *)L.kbuf + (size_t)i * L.n * L.n * L.n : (R *)L.kout;
}

// Current state psi_i at flat offset off: sum_(j<=i) coef[j][i] u_j in FP64,
// rounded once to the storage precision.
template <typename R, int KM>
__device__ __forceinline__ R lazy_psi(const LatView<R, KM> &vw, size_t off) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < KM; ++j)
        if (j <= vw.i && vw.c[j] != 0.0) s += vw.c[j] * (double)vw.u[j][off];
    return (R)s;
}

// 16-byte vector of R (4 floats or 2 doubles): one global load or store.
template <typename R>
constexpr int VLEN = 16 / (int)sizeof(R);
template <typename R>
using Vec = R __attribute__((ext_vector_type(VLEN<R>)));

// Raw loads of lazy_combine: the rows y0 and y1 of every array u_j (j <= i, c_j
// != 0) over G chunks, all issued before any of them is used.
template <typename R, int G, int KM>
struct LazyRaw {
    Vec<R> v0[KM][G], v1[KM][G];
};

template <typename R, int G, int KM>
__device__ __forceinline__ void lazy_issue(const LatView<R, KM> &vw, const size_t (&o0)[G], const size_t (&o1)[G],
                                           const bool (&ok)[G], LazyRaw<R, G, KM> &raw) {
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        if (j > vw.i || vw.c[j] == 0.0) continue;
#pragma unroll
        for (int t = 0; t < G; ++t) {
            if (ok[t]) {
                raw.v0[j][t] = *(const ITSE_GLOBAL Vec<R> *)(vw.u[j] + o0[t]);
                raw.v1[j][t] = *(const ITSE_GLOBAL Vec<R> *)(vw.u[j] + o1[t]);
            }
        }
    }
}

// psi = sum_(j<=i) c_j u_j of the raw loads, in FP64, rounded once.
template <typename R, int G, int KM>
__device__ __forceinline__ void lazy_combine(const LatView<R, KM> &vw, const LazyRaw<R, G, KM> &raw,
                                             R (&p0)[G][VLEN<R>], R (&p1)[G][VLEN<R>]) {
    constexpr int VL = VLEN<R>;
    double a0[G][VL], a1[G][VL];
#pragma unroll
    for (int t = 0; t < G; ++t)
#pragma unroll
        for (int k = 0; k < VL; ++k) a0[t][k] = a1[t][k] = 0.0;
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        if (j > vw.i || vw.c[j] == 0.0) continue;
        const double c = vw.c[j];
#pragma unroll
        for (int t = 0; t < G; ++t)
#pragma unroll
            for (int k = 0; k < VL; ++k) {
                a0[t][k] += c * (double)raw.v0[j][t][k];
                a1[t][k] += c * (double)raw.v1[j][t][k];
            }
    }
#pragma unroll
    for (int t = 0; t < G; ++t)
#pragma unroll
        for (int k = 0; k < VL; ++k) {
            p0[t][k] = (R)a0[t][k];
            p1[t][k] = (R)a1[t][k];
        }
}

// Current states of rows y0 and y1 of plane x over G chunks of VLEN consecutive
// z (chunk t of the calling lane starts at z0[t]): psi = sum_(j<=i) c_j u_j in
// FP64, rounded once.  All loads of one array are issued before any use.
template <typename R, int G, int KM>
__device__ __forceinline__ void lazy_rows(const LatView<R, KM> &vw, const size_t (&o0)[G], const size_t (&o1)[G],
                                          const bool (&ok)[G], R (&p0)[G][VLEN<R>], R (&p1)[G][VLEN<R>]) {
    constexpr int VL = VLEN<R>;
    double a0[G][VL], a1[G][VL];
#pragma unroll
    for (int t = 0; t < G; ++t)
#pragma unroll
        for (int k = 0; k < VL; ++k) a0[t][k] = a1[t][k] = 0.0;
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        if (j > vw.i) break;
        const double c = vw.c[j];
        if (c == 0.0) continue;
        Vec<R> v0[G], v1[G];
#pragma unroll
        for (int t = 0; t < G; ++t) {
            if (ok[t]) {
                v0[t] = *(const ITSE_GLOBAL Vec<R> *)(vw.u[j] + o0[t]);
                v1[t] = *(const ITSE_GLOBAL Vec<R> *)(vw.u[j] + o1[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < G; ++t)
#pragma unroll
            for (int k = 0; k < VL; ++k) {
                a0[t][k] += c * (double)v0[t][k];
                a1[t][k] += c * (double)v1[t][k];
            }
    }
#pragma unroll
    for (int t = 0; t < G; ++t)
#pragma unroll
        for (int k = 0; k < VL; ++k) {
            p0[t][k] = (R)a0[t][k];
            p1[t][k] = (R)a1[t][k];
        }
}

// Chunks of the row pairs a wave owns: PPW pairs x N/VLEN chunks, taken by the 64
// lanes in groups of G per lane.
template <typename R, int N, int PPW, int GMAX>
struct PairChunks {
    static constexpr int VL = VLEN<R>;
    static constexpr int CPR = N / VL;                 // chunks per row
    static constexpr int TOTAL = PPW * CPR;            // chunks per wave
    static constexpr int PER_LANE = (TOTAL + 63) / 64;
    static constexpr int G = PER_LANE < GMAX ? PER_LANE : GMAX;
    static constexpr int GROUPS = (PER_LANE + G - 1) / G;
    static_assert(N % VLEN<R> == 0, "rows hold whole vectors");
};

// Copy of a contiguous global block of E complex values into LDS rows of length
// RL with stride RS, all loads of the calling thread issued first (up to 16
// 16-byte loads per thread in one batch: one memory round trip).
// FP32 rows copied two values per thread (16-byte accesses): needs even strides
// and, for rows of odd length, one slot of padding after each row in both layouts
// (it receives the padding value of the other side, which nothing reads).
template <typename R, int RL, int GS, int RS>
constexpr bool PAIR_ROWS = sizeof(R) == 4 && GS % 2 == 0 && RS % 2 == 0 && RL + RL % 2 <= GS && RL + RL % 2 <= RS;

template <typename R, int E, int RL, int GS, int RS, int NTH>
__device__ __forceinline__ void block_load_rows(const C2<R> *src_, C2<R> *dst, int tid) {
    if constexpr (PAIR_ROWS<R, RL, GS, RS>) {
        using F4 = float __attribute__((ext_vector_type(4)));
        static_assert(E % RL == 0, "whole rows");
        constexpr int RP = (RL + 1) / 2, EP = E / RL * RP;
        constexpr int T = (EP + NTH - 1) / NTH;
        constexpr int TB = T < 16 ? T : 16;
        const ITSE_GLOBAL F4 *src = (const ITSE_GLOBAL F4 *)gmem(src_);
        F4 *d4 = (F4 *)dst;
#pragma unroll
        for (int t0 = 0; t0 < T; t0 += TB) {
            F4 v[TB];
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                const int e = tid + (t0 + t) * NTH;
                const int ee = (EP % NTH == 0 || e < EP) ? e : EP - 1;
                if (t0 + t < T) v[t] = src[(ee / RP) * (GS / 2) + ee % RP];
            }
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                const int e = tid + (t0 + t) * NTH;
                if (t0 + t < T && (EP % NTH == 0 || e < EP)) d4[(e / RP) * (RS / 2) + e % RP] = v[t];
            }
        }
        return;
    }
    const ITSE_GLOBAL C2<R> *src = gmem(src_);
    constexpr int T = (E + NTH - 1) / NTH;
    constexpr int TB0 = 64 / (int)sizeof(C2<R>);  // values in 64 bytes: 8 (FP32), 4 (FP64)
    constexpr int TB = T < 4 * TB0 ? T : 4 * TB0;
#pragma unroll
    for (int t0 = 0; t0 < T; t0 += TB) {
        C2<R> v[TB];
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            // out-of-range threads load the last element (valid) and store nothing
            const int e = tid + (t0 + t) * NTH;
            const int ee = (E % NTH == 0 || e < E) ? e : E - 1;
            if (t0 + t < T) v[t] = src[(ee / RL) * GS + ee % RL];
        }
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            const int e = tid + (t0 + t) * NTH;
            if (t0 + t < T && (E % NTH == 0 || e < E)) dst[(e / RL) * RS + e % RL] = v[t];
        }
    }
}

template <typename R, int E, int RL, int GS, int RS, int NTH>
__device__ __forceinline__ void block_store_rows(const C2<R> *src, C2<R> *dst_, int tid) {
    if constexpr (PAIR_ROWS<R, RL, GS, RS>) {
        using F4 = float __attribute__((ext_vector_type(4)));
        static_assert(E % RL == 0, "whole rows");
        constexpr int RP = (RL + 1) / 2, EP = E / RL * RP;
        constexpr int T = (EP + NTH - 1) / NTH;
        ITSE_GLOBAL F4 *d4 = (ITSE_GLOBAL F4 *)gmem(dst_);
        const F4 *s4 = (const F4 *)src;
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int e = tid + t * NTH;
            if (EP % NTH == 0 || e < EP) d4[(e / RP) * (GS / 2) + e % RP] = s4[(e / RP) * (RS / 2) + e % RP];
        }
        return;
    }
    ITSE_GLOBAL C2<R> *dst = gmem(dst_);
    constexpr int T = (E + NTH - 1) / NTH;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int e = tid + t * NTH;
        if (E % NTH == 0 || e < E) dst[(e / RL) * GS + e % RL] = src[(e / RL) * RS + e % RL];
    }
}

// The inverse pass's input rows when its y split is twice the layout's: rows k and
// k + M of layout sub-spectrum (x, r_L) (M = half its rows, RL values each, row stride
// GS) give row k of half t: e^(+2 pi i t k / 2M) (X[k] + (-1)^t X[k + M]), the first
// radix-2 step of the inverse y transform over the layout's 2M rows (its rows
// 2 j + t, which are the rows y = r_L + S_L (2 j + t) of the finer split's
// sub-plane r_L + S_L t); the factor is twiddle k * TWS of the table (TWS = N / 2M).
// Stored in LDS rows of stride RS; FP32 pairs of values per 16-byte access.
template <typename R, int M, int RL, int GS, int RS, int TWS, int NTH>
__device__ __forceinline__ void block_load_rows_split(const C2<R> *src_, C2<R> *dst, int t, const C2<R> *tw,
                                                      int tid) {
    static_assert(PAIR_ROWS<R, RL, GS, RS>, "FP32 rows copied in pairs");
    using F4 = float __attribute__((ext_vector_type(4)));
    constexpr int RP = (RL + 1) / 2, EP = M * RP;
    constexpr int T = (EP + NTH - 1) / NTH;
    constexpr int TB = T < 8 ? T : 8;
    const ITSE_GLOBAL F4 *src = (const ITSE_GLOBAL F4 *)gmem(src_);
    F4 *d4 = (F4 *)dst;
#pragma unroll
    for (int t0 = 0; t0 < T; t0 += TB) {
        F4 va[TB], vb[TB];
#pragma unroll
        for (int q = 0; q < TB; ++q) {
            const int e = tid + (t0 + q) * NTH;
            const int ee = (EP % NTH == 0 || e < EP) ? e : EP - 1;
            if (t0 + q < T) {
                va[q] = src[(ee / RP) * (GS / 2) + ee % RP];
                vb[q] = src[(ee / RP + M) * (GS / 2) + ee % RP];
            }
        }
#pragma unroll
        for (int q = 0; q < TB; ++q) {
            const int e = tid + (t0 + q) * NTH;
            if (t0 + q < T && (EP % NTH == 0 || e < EP)) {
                const int k = e / RP;
                C2<R> a0{va[q].x, va[q].y}, a1{va[q].z, va[q].w};
                const C2<R> b0{vb[q].x, vb[q].y}, b1{vb[q].z, vb[q].w};
                if (t == 0) {
                    a0 = cadd(a0, b0);
                    a1 = cadd(a1, b1);
                } else {
                    a0 = tw_mul<+1>(csub(a0, b0), tw, k * TWS);
                    a1 = tw_mul<+1>(csub(a1, b1), tw, k * TWS);
                }
                d4[k * (RS / 2) + e % RP] = F4{a0.x, a0.y, a1.x, a1.y};
            }
        }
    }
}

// ---------------------------------------------------------------------------
// P1: forward plane pass.  Sub-plane x * S + r and job from plane_block.
// ---------------------------------------------------------------------------
// The passes are written as tile functions (one workgroup's work: the tile's
// indices and its LDS arrays are arguments), called by their own kernels and by
// the persistent batch kernel.
template <typename R, int N, int V, int KM>
__device__ __forceinline__ void plane_fwd_tile(const JobRef *__restrict__ jobs, int spb, int jb, C2<R> *buf,
                                               C2<R> *tw) {
    using G = Geo<R, N, V>;
    constexpr int S = G::S, M = G::M, H = G::H, HP = G::HP, LSZ = G::LSZ, PPW = G::PPW, CPW = G::CPW;
    const JobRef job = jobs[jb];
    const LatDev &L = *job.lat;
    const int tid = tile_tid(), lane = tid & 63, wv = tid >> 6;
    const int x = spb / S, r = spb % S;
    const C2<R> *twg = (const C2<R> *)L.tw;
    for (int e = tid; e < N; e += G::NTP) tw[e] = twg[e];
    LatView<R, KM> vw;
    load_view(vw, L, job.state);
    C2<R> *spec = (C2<R> *)L.spec[job.state];

    // rows of this wave's pairs -> packed complex rows (z along the line)
    const int p0 = wv * PPW;
    {
        // FP64 lattices whose plane's LDS keeps the pass at two waves per SIMD or
        // fewer (registers for a round's raw arrays): every array's loads of a round
        // issued before any is used, one memory round trip per round.  Otherwise one
        // array after another (FP32 under schedule 1 at 256^3 measured 2 % slower
        // up front).
        constexpr bool UPFRONT = sizeof(R) == 8 && G::WPE <= 2 && KM <= 4;
        using PC = PairChunks<R, N, PPW, KM <= 4 ? 4 : 2>;
        constexpr int VL = PC::VL, G = PC::G;
#pragma unroll 1
        for (int gi = 0; gi < PC::GROUPS; ++gi) {
            size_t o0[G], o1[G];
            bool ok[G];
            int lp[G];
#pragma unroll
            for (int t = 0; t < G; ++t) {
                const int c = lane + 64 * (gi * G + t);
                ok[t] = c < PC::TOTAL;
                const int pl = ok[t] ? c / PC::CPR : 0, z = ok[t] ? (c % PC::CPR) * VL : 0;
                const int p = p0 + pl;
                const int y0 = r + S * (2 * p);
                o0[t] = ((size_t)x * N + y0) * N + z;
                o1[t] = o0[t] + (size_t)S * N;
                lp[t] = p * LSZ + z;
            }
            R v0[G][VL], v1[G][VL];
            if constexpr (UPFRONT) {
                LazyRaw<R, G, KM> raw;
                lazy_issue<R, G>(vw, o0, o1, ok, raw);
                lazy_combine<R, G>(vw, raw, v0, v1);
            } else {
                lazy_rows<R, G>(vw, o0, o1, ok, v0, v1);
            }
#pragma unroll
            for (int t = 0; t < G; ++t)
                if (ok[t]) {
#pragma unroll
                    for (int k = 0; k < VL; ++k) buf[lp[t] + k] = C2<R>{v0[t][k], v1[t][k]};
                }
        }
    }
    __syncthreads();  // twiddles
    WaveFft<R, N, PPW, -1, false, 1>::run(buf + p0 * LSZ, LSZ, 1, tw, lane);
    // unpack each pair into two half spectra, in place: rows 2p, 2p+1 of the plane layout
    constexpr int TU = (H + 63) / 64;
    for (int pl = 0; pl < PPW; ++pl) {
        C2<R> *zl = buf + (p0 + pl) * LSZ;
        C2<R> a0[TU], a1[TU];
#pragma unroll
        for (int t = 0; t < TU; ++t) {
            const int k = lane + 64 * t;
            if (k < H) {
                const C2<R> ck = zl[k];
                const C2<R> cm = zl[(N - k) % N];
                a0[t] = C2<R>{(R)0.5 * (ck.x + cm.x), (R)0.5 * (ck.y - cm.y)};
                a1[t] = C2<R>{(R)0.5 * (ck.y + cm.y), (R)0.5 * (cm.x - ck.x)};
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int t = 0; t < TU; ++t) {
            const int k = lane + 64 * t;
            if (k < H) {
                zl[k] = a0[t];
                zl[HP + k] = a1[t];
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // transform along j (rows) for this wave's kz columns, the kz = N/2 column by the last wave
    WaveFft<R, M, CPW, -1, true, S>::run(buf + wv * CPW, 1, HP, tw, lane);
    if (wv == G::NWP - 1) WaveFft<R, M, 1, -1, true, S>::run(buf + N / 2, 1, HP, tw, lane);
    __syncthreads();
    block_store_rows<R, M * H, H, G::HS, HP, G::NTP>(buf, spec + ((size_t)r * N + x) * M * G::HS, tid);
}

// Sub-plane and job of a plane-pass workgroup.  SPLIT (inverse pass): the two
// halves of a layout sub-plane run as two jobs eight workgroups apart, both on one
// XCD at nearly the same time, so that the second finds the layout rows they share
// in L2.
template <int NB, int S, bool SPLIT>
__device__ __forceinline__ int plane_tile(int &jb) {
    if constexpr (SPLIT) {
        constexpr int SL = S / 2;
        int jt;
        const int spl = plane_block<NB / 2>(jt);
        jb = jt >> 1;
        return (spl / SL) * S + spl % SL + SL * (jt & 1);
    } else {
        return plane_block<NB>(jb);
    }
}

template <typename R, int N, int V, int KM>
__global__ void __launch_bounds__((Geo<R, N, V>::NTP)) __attribute__((amdgpu_waves_per_eu(Geo<R, N, V>::WPE)))
k_plane_fwd(const JobRef *__restrict__ jobs) {
    using G = Geo<R, N, V>;
    __shared__ __attribute__((aligned(16))) C2<R> buf[G::PLANE_ELEMS];
    __shared__ C2<R> tw[N];
    int jb;
    const int spb = plane_block<G::NB_PLANE>(jb);
    plane_fwd_tile<R, N, V, KM>(jobs, spb, jb, buf, tw);
}

// ---------------------------------------------------------------------------
// P2: column pass.  grid.x = ky' * NCH + chunk, grid.y = job.
// mode COL_KIN: forward x transform, kinetic multiply (+ parity-weight sums
// when moments are on), inverse, back to sub-spectra.
// mode COL_FWD: forward x transform only, stored in the standard layout
// [kx][ky][kz] at `out` (for the spectrum query).
// ---------------------------------------------------------------------------
template <typename R, int N, int V>
__device__ __forceinline__ void columns_tile(const JobRef *__restrict__ jobs, int blk, int jy, int mode, int moments,
                                             C2<R> *__restrict__ out, C2<R> *buf, C2<R> *tw, double *ktab,
                                             double *red) {
    using G = Geo<R, N, V>;
    constexpr int S = G::S, M = G::M, H = G::H, W = G::W, CS = G::CS, LPW = G::LPWC, NTC = G::NTC;
    const JobRef job = jobs[jy];
    const LatDev &L = *job.lat;
    const int i = job.state;
    const int tid = tile_tid(), lane = tid & 63, wv = tid >> 6;
    const int kyp = blk / G::NCH, kz0 = (blk % G::NCH) * W;
    const C2<R> *twg = (const C2<R> *)L.tw;
    for (int e = tid; e < N; e += NTC) {
        tw[e] = twg[e];
        ktab[e] = L.ktab[e];
    }
    __syncthreads();
    ITSE_GLOBAL C2<R> *spec = gmem((C2<R> *)L.spec[i]);
    constexpr int HS = G::HS;
    const size_t sub = (size_t)N * M * HS;  // one sub-spectrum
    // load S sub-spectra values (all loads of the thread first), combine over r ->
    // S full-y columns ky = ky' + M q
    if constexpr (sizeof(R) == 4 && W % 2 == 0) {
        // FP32: two kz per thread, one 16-byte load per sub-spectrum (rows are
        // padded, so the pair at kz = N/2 stays in the row; its upper half is
        // padding and is replaced by zero)
        constexpr int W2 = W / 2;
        constexpr int T = (N * W2 + NTC - 1) / NTC;
        using F4 = float __attribute__((ext_vector_type(4)));
        // every load unconditional (out-of-range threads and chunks read offset 0),
        // the values masked where they are used: all loads in flight before the
        // first wait
        F4 v[T][S];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int e = tid + t * NTC;
            const int xx = e / W2, kz = kz0 + 2 * (e % W2);
            const bool ok = ((N * W2) % NTC == 0 || e < N * W2) && kz < H;
            const size_t base = ok ? ((size_t)xx * M + kyp) * HS + kz : 0;
#pragma unroll
            for (int rr = 0; rr < S; ++rr) v[t][rr] = *(const ITSE_GLOBAL F4 *)(spec + rr * sub + base);
        }
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int e = tid + t * NTC;
            if ((N * W2) % NTC != 0 && e >= N * W2) continue;
            const int xx = e / W2, w = 2 * (e % W2), kz = kz0 + w;
            // kz >= H: no data; kz + 1 = H: the pair's upper half is row padding
            const bool oka = kz < H, okb = kz + 1 < H;
            C2<R> a[S], b[S];
#pragma unroll
            for (int rr = 0; rr < S; ++rr) {
                a[rr] = oka ? C2<R>{v[t][rr].x, v[t][rr].y} : C2<R>{(R)0, (R)0};
                b[rr] = okb ? C2<R>{v[t][rr].z, v[t][rr].w} : C2<R>{(R)0, (R)0};
                if (rr > 0) {
                    a[rr] = tw_mul<-1>(a[rr], tw, rr * kyp);
                    b[rr] = tw_mul<-1>(b[rr], tw, rr * kyp);
                }
            }
            Dft<S, -1, R>::run(a);
            Dft<S, -1, R>::run(b);
#pragma unroll
            for (int q = 0; q < S; ++q) *(F4 *)&buf[xx * CS + q * W + w] = F4{a[q].x, a[q].y, b[q].x, b[q].y};
        }
    } else {
        constexpr int T = (N * W + NTC - 1) / NTC;
        // unconditional loads (offset 0 when out of range), masked at their use
        C2<R> v[T][S];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int e = tid + t * NTC;
            const int xx = e / W, kz = kz0 + e % W;
            const bool ok = ((N * W) % NTC == 0 || e < N * W) && kz < H;
            const size_t base = ok ? ((size_t)xx * M + kyp) * HS + kz : 0;
#pragma unroll
            for (int rr = 0; rr < S; ++rr) v[t][rr] = spec[rr * sub + base];
        }
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int e = tid + t * NTC;
            if ((N * W) % NTC != 0 && e >= N * W) continue;
            const int xx = e / W, w = e % W;
            if (kz0 + w >= H)
#pragma unroll
                for (int rr = 0; rr < S; ++rr) v[t][rr] = C2<R>{(R)0, (R)0};
#pragma unroll
            for (int rr = 1; rr < S; ++rr) v[t][rr] = tw_mul<-1>(v[t][rr], tw, rr * kyp);
            Dft<S, -1, R>::run(v[t]);
#pragma unroll
            for (int q = 0; q < S; ++q) buf[xx * CS + q * W + w] = v[t][q];
        }
    }
    __syncthreads();
    const int l0 = wv * LPW;
    if (mode == COL_FWD) {
        WaveFft<R, N, LPW, -1, true, 1>::run(buf + l0, 1, CS, tw, lane);
        __syncthreads();
        for (int e = tid; e < N * S * W; e += NTC) {
            const int xx = e / (S * W), l = e % (S * W), q = l / W, w = l % W, kz = kz0 + w;
            if (kz < H) gmem(out)[((size_t)xx * N + kyp + M * q) * H + kz] = buf[xx * CS + l];
        }
        return;
    }
    // forward transform along x, then the kinetic multiply T(kx, ky, kz) / N^3 on this
    // wave's lines (with the momentum-space parity sums when moments are on), then
    // the inverse transform along x
    const double inv_n3 = 1.0 / ((double)N * (double)N * (double)N);
    const bool mom = moments && L.moments;
    const int kin = L.kin, rest = L.sub, center = L.center;
    const double mass = L.mass;
    const int kind = kin == ITSE_KIN_NR_CONT || kin == ITSE_KIN_NR_LAT ? SYM_SUM : rest ? SYM_REL_SUB : SYM_REL;
    double acc[NQC] = {0.0, 0.0};
    using Pair = WaveFftPair<R, N, LPW, true, 1>;
    bool fused = false;
    if constexpr (Pair::OK) {
        if (!mom) {
            // square lengths: the multiply between the last forward and the first
            // inverse stage, in registers
            auto run = [&](auto kc) {
                constexpr int KIND = decltype(kc)::value;
                Pair::run(buf + l0, 1, CS, tw, lane, [&](int line, int j, C2<R>(&v)[Pair::G]) {
                    const int l = l0 + line, kz = kz0 + l % W;
                    if (kz >= H) return;
                    const double cl = ktab[kyp + M * (l / W)] + ktab[kz];
#pragma unroll
                    for (int q = 0; q < Pair::G; ++q) {
                        const R t = symbol_scaled<R, KIND>(ktab[j + Pair::G * q] + cl, mass, inv_n3);
                        v[q].x *= t;
                        v[q].y *= t;
                    }
                });
            };
            if (kind == SYM_SUM) run(std::integral_constant<int, SYM_SUM>{});
            else if (kind == SYM_REL) run(std::integral_constant<int, SYM_REL>{});
            else run(std::integral_constant<int, SYM_REL_SUB>{});
            fused = true;
        }
    }
    if (!fused) {
        WaveFft<R, N, LPW, -1, true, 1>::run(buf + l0, 1, CS, tw, lane);
        // the same symbol evaluation as the line-wise paths (table sum over ky, kz
        // first, then kx)
        auto multiply = [&](int kx, int ky, int kz, C2<R> &val) {
            const double ssum = ktab[kx] + (ktab[ky] + ktab[kz]);
            const R t = kind == SYM_SUM  ? symbol_scaled<R, SYM_SUM>(ssum, mass, inv_n3)
                        : kind == SYM_REL ? symbol_scaled<R, SYM_REL>(ssum, mass, inv_n3)
                                          : symbol_scaled<R, SYM_REL_SUB>(ssum, mass, inv_n3);
            val.x *= t;
            val.y *= t;
        };
        if (!mom) {
            if constexpr (64 % LPW == 0 && N % (64 / LPW) == 0) {
                // each lane keeps one line (fixed ky, kz) and steps through kx
                const int l = l0 + lane % LPW, kz = kz0 + l % W;
                const double cl = ktab[kyp + M * (l / W)] + ktab[kz < H ? kz : 0];
                if (kz < H) {
                    if (kind == SYM_SUM)
                        multiply_line<R, SYM_SUM, N, 64 / LPW, CS>(buf + l, ktab, lane / LPW, cl, mass, inv_n3);
                    else if (kind == SYM_REL)
                        multiply_line<R, SYM_REL, N, 64 / LPW, CS>(buf + l, ktab, lane / LPW, cl, mass, inv_n3);
                    else
                        multiply_line<R, SYM_REL_SUB, N, 64 / LPW, CS>(buf + l, ktab, lane / LPW, cl, mass, inv_n3);
                }
            } else {
#pragma unroll 1
                for (int e = lane; e < N * LPW; e += 64) {
                    const int kx = e / LPW, l = l0 + e % LPW, q = l / W, kz = kz0 + l % W;
                    if (kz >= H) continue;
                    C2<R> val = buf[kx * CS + l];
                    multiply(kx, kyp + M * q, kz, val);
                    buf[kx * CS + l] = val;
                }
            }
        } else {
#pragma unroll 1
            for (int e = lane; e < N * LPW; e += 64) {
                const int kx = e / LPW, l = l0 + e % LPW, q = l / W, kz = kz0 + l % W;
                if (kz >= H) continue;
                const int ky = kyp + M * q;
                C2<R> val = buf[kx * CS + l];
                // weight 2 for the interior of the half spectrum (its mirror is implied)
                const double wt = (kz == 0 || 2 * kz == N) ? 1.0 : 2.0;
                const double re = (double)val.x, im = (double)val.y;
                acc[CQ_NORM] += wt * (re * re + im * im);
                // <psi|P psi> = sum_k e^{i kappa} conj(psi_k)^2 / N^3 with kappa = 2 pi (kx+ky+kz)/N
                // for the off-grid centre (x -> N-1-x), kappa = 0 for the origin
                double pr = re * re - im * im;
                const double pim = -2.0 * re * im;
                if (center == ITSE_CENTER_CELL) {
                    const int mm = (kx + ky + kz) % N;
                    double sn, cs;
                    sincospi(2.0 * (double)mm / (double)N, &sn, &cs);
                    pr = cs * pr - sn * pim;
                }
                acc[CQ_PAR] += wt * pr;
                multiply(kx, ky, kz, val);
                buf[kx * CS + l] = val;
            }
        }
        __builtin_amdgcn_wave_barrier();
        WaveFft<R, N, LPW, +1, true, 1>::run(buf + l0, 1, CS, tw, lane);
    }
    if (mom) block_sums<NQC, NTC>(acc, L.part_cols + ((size_t)i * L.nb_cols + blk) * NQC, red);
    __syncthreads();
    if constexpr (sizeof(R) == 4 && W % 2 == 0) {
        // FP32: two kz per thread, 16-byte stores (8 bytes at kz = N/2)
        using F4 = float __attribute__((ext_vector_type(4)));
        constexpr int W2 = W / 2;
        for (int e = tid; e < N * W2; e += NTC) {
            const int xx = e / W2, w = 2 * (e % W2), kz = kz0 + w;
            if (kz >= H) continue;
            C2<R> a[S], b[S];
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const F4 f = *(const F4 *)&buf[xx * CS + q * W + w];
                a[q] = C2<R>{f.x, f.y};
                b[q] = C2<R>{f.z, f.w};
            }
            Dft<S, +1, R>::run(a);
            Dft<S, +1, R>::run(b);
            const size_t base = ((size_t)xx * M + kyp) * HS + kz;
#pragma unroll
            for (int rr = 0; rr < S; ++rr) {
                C2<R> x0 = a[rr], x1 = b[rr];
                if (rr > 0) {
                    x0 = tw_mul<+1>(x0, tw, rr * kyp);
                    x1 = tw_mul<+1>(x1, tw, rr * kyp);
                }
                if (kz + 1 < H) *(ITSE_GLOBAL F4 *)(spec + rr * sub + base) = F4{x0.x, x0.y, x1.x, x1.y};
                else spec[rr * sub + base] = x0;
            }
        }
        return;
    }
    for (int e = tid; e < N * W; e += NTC) {
        const int xx = e / W, w = e % W, kz = kz0 + w;
        if (kz >= H) continue;
        C2<R> v[S];
#pragma unroll
        for (int q = 0; q < S; ++q) v[q] = buf[xx * CS + q * W + w];
        Dft<S, +1, R>::run(v);
        const size_t base = ((size_t)xx * M + kyp) * HS + kz;
#pragma unroll
        for (int rr = 0; rr < S; ++rr) {
            C2<R> a = v[rr];
            if (rr > 0) a = tw_mul<+1>(a, tw, rr * kyp);
            spec[rr * sub + base] = a;
        }
    }
}

template <typename R, int N, int V>
__global__ void __launch_bounds__((Geo<R, N, V>::NTC)) __attribute__((amdgpu_waves_per_eu(Geo<R, N, V>::WPEC)))
k_columns(const JobRef *__restrict__ jobs, int mode, int moments, C2<R> *__restrict__ out) {
    using G = Geo<R, N, V>;
    __shared__ __attribute__((aligned(16))) C2<R> buf[N * G::CS];
    __shared__ C2<R> tw[N];
    __shared__ double ktab[N];
    __shared__ double red[NQC * (G::NTC / 64)];
    // consecutive chunks of one ky' row share cache lines: keep them on one XCD
    columns_tile<R, N, V>(jobs, xcd_local_index(blockIdx.x, gridDim.x), blockIdx.y, mode, moments, out, buf, tw,
                          ktab, red);
}

// ---------------------------------------------------------------------------
// P3: inverse plane pass + update.  Sub-plane x * S + r and job from plane_block.
// mode INV_UPDATE: u_i <- ((1 - h V) psi - dtau K psi) / (1 + h V)   (= A psi - B dtau K psi)
// mode INV_EVAL: sums only; INV_KOUT: K psi written to L.kout; INV_KBUF: K psi_i
// written to L.kbuf + i N^3.
// ---------------------------------------------------------------------------
// MOM: position moments summed (the lattices' moments flag); without them the
// update loop has the registers to take two chunks per load round.
// CPX: the imaginary part (state 1) of complex lattices, after the real part's
// pass has written K Re psi to kbuf: with Re psi = c u_0, Im psi = c u_1 and
// V = Vr + i Vi it applies the complex map ((1 - h V) psi - dtau K psi)/(1 + h V)
// and writes both parts' new arrays; besides its own row sums it forms
// sum Vi |psi|^2 and sum |psi'|^2 (the complex-update sums).
template <typename R, int N, int V, bool MOM, int KM, bool CPX = false, bool SPLIT = false>
__device__ __forceinline__ void plane_inv_tile(const JobRef *__restrict__ jobs, int spb, int jb, int mode, C2<R> *buf,
                                               C2<R> *tw, double *red) {
    using G = Geo<R, N, V>;
    constexpr int S = G::S, M = G::M, H = G::H, HP = G::HP, LSZ = G::LSZ, PPW = G::PPW, CPW = G::CPW;
    constexpr int NTP = G::NTP;
    const JobRef job = jobs[jb];
    const LatDev &L = *job.lat;
    const int i = job.state;
    const int tid = tile_tid(), lane = tid & 63, wv = tid >> 6;
    const int x = spb / S, r = spb % S;
    const C2<R> *twg = (const C2<R> *)L.tw;
    for (int e = tid; e < N; e += NTP) tw[e] = twg[e];
    if constexpr (SPLIT) {
        // layout of S / 2 sub-spectra of 2 M rows: this workgroup's rows are half
        // r / (S / 2) of layout sub-plane (x, r mod S / 2)
        static_assert(S % 2 == 0, "the layout's split is half of this pass's");
        constexpr int SL = S / 2;
        __syncthreads();  // the twiddle table
        block_load_rows_split<R, M, H, G::HS, HP, SL, NTP>(
            (const C2<R> *)L.spec[i] + ((size_t)(r % SL) * N + x) * (2 * M) * G::HS, buf, r / SL, tw, tid);
    } else {
        block_load_rows<R, M * H, H, G::HS, HP, NTP>((const C2<R> *)L.spec[i] + ((size_t)r * N + x) * M * G::HS,
                                                     buf, tid);
    }
    __syncthreads();
    WaveFft<R, M, CPW, +1, true, S>::run(buf + wv * CPW, 1, HP, tw, lane);
    if (wv == G::NWP - 1) WaveFft<R, M, 1, +1, true, S>::run(buf + N / 2, 1, HP, tw, lane);
    __syncthreads();
    // pack rows 2p, 2p+1 (half spectra along z) into one complex row, in place
    const int p0 = wv * PPW;
    constexpr int TK = (N + 63) / 64;
    for (int pl = 0; pl < PPW; ++pl) {
        C2<R> *zl = buf + (p0 + pl) * LSZ;
        C2<R> zz[TK];
#pragma unroll
        for (int t = 0; t < TK; ++t) {
            const int k = lane + 64 * t;
            if (N % 64 == 0 || k < N) {
                const bool direct = 2 * k <= N;
                const int kk = direct ? k : N - k;
                C2<R> A = zl[kk], B = zl[HP + kk];
                if (!direct) {
                    A.y = -A.y;
                    B.y = -B.y;
                } else if (k == 0 || 2 * k == N) {
                    A.y = (R)0;
                    B.y = (R)0;
                }
                zz[t] = C2<R>{A.x - B.y, A.y + B.x};
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int t = 0; t < TK; ++t) {
            const int k = lane + 64 * t;
            if (N % 64 == 0 || k < N) zl[k] = zz[t];
        }
        __builtin_amdgcn_wave_barrier();
    }
    WaveFft<R, N, PPW, +1, false, 1>::run(buf + p0 * LSZ, LSZ, 1, tw, lane);
    // update of this wave's rows
    LatView<R, KM> vw;
    load_view(vw, L, i);
    const ITSE_GLOBAL R *v = gmem((const R *)L.v);
    ITSE_GLOBAL R *u = gmem((R *)state_buf(L, L.step, 1, i));
    ITSE_GLOBAL R *kout = gmem(kout_ptr<R>(L, mode, i));
    const R h = (R)L.h, dt = (R)L.dtau;
    const bool mom = MOM && L.moments != 0;
    const int center = L.center;
    const double a = L.a;
    double acc[NQR];
#pragma unroll
    for (int q = 0; q < NQR; ++q) acc[q] = 0.0;
    // UPFRONT (FP32 lattices and FP64 from N = 128; no moments, no complex part, up to
    // four states): every global load of a round (V and the lazy combination's
    // arrays) is issued before any of them is used, one memory round trip per round;
    // the registers then allow two chunks per round for one state, and for more
    // where the plane's LDS keeps the pass at two waves per SIMD or fewer (256
    // VGPRs); one otherwise.  Otherwise the arrays load one after another (each
    // array's loads issued together), two chunks per round without moments.
    constexpr bool UPFRONT = (sizeof(R) == 4 || N >= 128) && !MOM && !CPX && KM <= 4;
    using PC = PairChunks<R, N, PPW, UPFRONT ? ((KM == 1 || G::WPE <= 2) ? 2 : 1) : ((MOM || CPX) ? 1 : 2)>;
    constexpr int VL = PC::VL, GG = PC::G;
    const double cx = site_coord(x, N, center, a);
    // CPX: the real part's raw array and K psi, Im V, the real part's new array
    const double c0 = CPX ? L.coef[0][0] : 0.0;
    const ITSE_GLOBAL R *u0c = gmem((const R *)state_buf(L, L.step, 0, 0));
    const ITSE_GLOBAL R *krc = gmem((const R *)L.kbuf);
    const ITSE_GLOBAL R *vic = gmem((const R *)L.vi);
    ITSE_GLOBAL R *w0c = gmem((R *)state_buf(L, L.step, 1, 0));
    double xacc[NQX] = {0.0, 0.0};
#pragma unroll 1
    for (int gi = 0; gi < PC::GROUPS; ++gi) {
        size_t o0[GG], o1[GG];
        bool ok[GG];
        int lp[GG], yy[GG], zz0[GG];
#pragma unroll
        for (int t = 0; t < GG; ++t) {
            const int c = lane + 64 * (gi * GG + t);
            ok[t] = c < PC::TOTAL;
            const int pl = ok[t] ? c / PC::CPR : 0, z = ok[t] ? (c % PC::CPR) * VL : 0;
            const int p = p0 + pl;
            yy[t] = r + S * (2 * p);
            zz0[t] = z;
            o0[t] = ((size_t)x * N + yy[t]) * N + z;
            o1[t] = o0[t] + (size_t)S * N;
            lp[t] = p * LSZ + z;
        }
        R ph[2][GG][VL];
        if constexpr (!UPFRONT) lazy_rows<R, GG>(vw, o0, o1, ok, ph[0], ph[1]);
        Vec<R> vv[2][GG];
        Vec<R> xr[2][GG], xk[2][GG], xi[2][GG];  // CPX: u_0, K Re psi, Im V
#pragma unroll
        for (int t = 0; t < GG; ++t)
            if (ok[t]) {
                vv[0][t] = *(const ITSE_GLOBAL Vec<R> *)(v + o0[t]);
                vv[1][t] = *(const ITSE_GLOBAL Vec<R> *)(v + o1[t]);
                if constexpr (CPX) {
                    xr[0][t] = *(const ITSE_GLOBAL Vec<R> *)(u0c + o0[t]);
                    xr[1][t] = *(const ITSE_GLOBAL Vec<R> *)(u0c + o1[t]);
                    xk[0][t] = *(const ITSE_GLOBAL Vec<R> *)(krc + o0[t]);
                    xk[1][t] = *(const ITSE_GLOBAL Vec<R> *)(krc + o1[t]);
                    xi[0][t] = *(const ITSE_GLOBAL Vec<R> *)(vic + o0[t]);
                    xi[1][t] = *(const ITSE_GLOBAL Vec<R> *)(vic + o1[t]);
                }
            }
        if constexpr (UPFRONT) {
            LazyRaw<R, GG, KM> raw;
            lazy_issue<R, GG>(vw, o0, o1, ok, raw);
            lazy_combine<R, GG>(vw, raw, ph[0], ph[1]);
        }
#pragma unroll
        for (int t = 0; t < GG; ++t) {
            if (!ok[t]) continue;
            Vec<R> un[2], kv[2], unr[2];
#pragma unroll
            for (int k = 0; k < VL; ++k) {
                const C2<R> kp = buf[lp[t] + k];
                kv[0][k] = kp.x;
                kv[1][k] = kp.y;
            }
#pragma unroll
            for (int row = 0; row < 2; ++row) {
                const double cy = site_coord(yy[t] + row * S, N, center, a);
#pragma unroll
                for (int k = 0; k < VL; ++k) {
                    const R p_ = ph[row][t][k];
                    const R vr = vv[row][t][k];
                    const R kr = kv[row][k];
                    const R hv = h * vr;
                    R unv;
                    if constexpr (CPX) {
                        // p_ = Im psi, kr = K Im psi; the real part from u_0 and kbuf
                        const R pr = (R)(c0 * (double)xr[row][t][k]);
                        const R hi = h * xi[row][t][k];
                        const R nr = pr * ((R)1 - hv) + hi * p_ - dt * xk[row][t][k];
                        const R ni = p_ * ((R)1 - hv) - hi * pr - dt * kr;
                        const R dr = (R)1 + hv;
                        const R inv = div_fast<R>((R)1, dr * dr + hi * hi);
                        const R ur = (nr * dr + ni * hi) * inv;
                        unv = (ni * dr - nr * hi) * inv;
                        unr[row][k] = ur;
                        xacc[XQ_VIPP] += (double)xi[row][t][k] * ((double)pr * (double)pr + (double)p_ * (double)p_);
                        xacc[XQ_UU] += (double)ur * (double)ur + (double)unv * (double)unv;
                    } else {
                        unv = div_fast<R>(p_ * ((R)1 - hv) - dt * kr, (R)1 + hv);
                    }
                    un[row][k] = unv;
                    const double pd = (double)p_;
                    acc[RQ_PP] += pd * pd;
                    acc[RQ_PK] += pd * (double)kr;
                    acc[RQ_VPP] += (double)vr * pd * pd;
                    acc[RQ_UU] += (double)unv * (double)unv;
                    if (mom) {
                        const double cz = site_coord(zz0[t] + k, N, center, a);
                        const double w2 = pd * pd;
                        acc[RQ_X] += cx * w2;
                        acc[RQ_Y] += cy * w2;
                        acc[RQ_Z] += cz * w2;
                        acc[RQ_R2] += (cx * cx + cy * cy + cz * cz) * w2;
                    }
                }
            }
            if (mode == INV_UPDATE) {
                *(ITSE_GLOBAL Vec<R> *)(u + o0[t]) = un[0];
                *(ITSE_GLOBAL Vec<R> *)(u + o1[t]) = un[1];
                if constexpr (CPX) {
                    *(ITSE_GLOBAL Vec<R> *)(w0c + o0[t]) = unr[0];
                    *(ITSE_GLOBAL Vec<R> *)(w0c + o1[t]) = unr[1];
                }
            } else if (mode >= INV_KOUT) {
                *(ITSE_GLOBAL Vec<R> *)(kout + o0[t]) = kv[0];
                *(ITSE_GLOBAL Vec<R> *)(kout + o1[t]) = kv[1];
            }
        }
    }
    block_sums<NQR, NTP>(acc, L.part_rows + ((size_t)i * L.nb_rows + spb) * NQR, red);
    if constexpr (CPX) {
        __syncthreads();
        block_sums<NQX, NTP>(xacc, L.part_cplx + (size_t)spb * NQX, red);
    }
}

template <typename R, int N, int V, bool MOM, int KM, bool CPX = false, bool SPLIT = false>
__global__ void __launch_bounds__((Geo<R, N, V>::NTP)) __attribute__((amdgpu_waves_per_eu(Geo<R, N, V>::WPE)))
k_plane_inv(const JobRef *__restrict__ jobs, int mode) {
    using G = Geo<R, N, V>;
    __shared__ __attribute__((aligned(16))) C2<R> buf[G::PLANE_ELEMS];
    __shared__ C2<R> tw[N];
    __shared__ double red[NQR * (G::NTP / 64)];
    int jb;
    const int spb = plane_tile<G::NB_PLANE, G::S, SPLIT>(jb);
    plane_inv_tile<R, N, V, MOM, KM, CPX, SPLIT>(jobs, spb, jb, mode, buf, tw, red);
}

// ---------------------------------------------------------------------------
// H_K^(0) step (the paper's equation HK0: finite differences, Dirichlet walls):
// K psi(x) = (1 / (2 M A^2)) sum over the six neighbours y of (psi(x) - psi(y)),
// psi vanishing outside the N^3 box, fused with the update and the FP64 sums of
// P3 (same modes, same partial-sum layout).  One pass over the lattice.
//
// Workgroup = a tile of TY full rows (y0 .. y0 + TY) and XS planes (x0 .. x0 + XS)
// of one job; it marches along x.  Each thread owns one 16-byte vector of VL
// consecutive z in the tile's plane; its values at x - 1, x, x + 1 stay in
// registers, the plane x with one halo row on each side goes through LDS for the
// y and z neighbours.  The halo rows and V are loaded one iteration before their
// use; the centre rows one iteration before their use up to three states, and in
// the iteration of their use with more (see AHEAD below).
// ---------------------------------------------------------------------------
constexpr int fd_rows(int n, int gpr) {
    int best = 1;
    for (int t = 1; t <= n; ++t)
        if (n % t == 0 && t * gpr <= NT) best = t;
    return best;
}
constexpr int fd_segments(int n, int tiles) {
    int best = 1;
    for (int sg = 1; sg <= n; ++sg)
        if (n % sg == 0 && n / sg >= 16 && tiles * sg <= 1024) best = sg;
    return best;
}

template <typename R, int N>
struct FdGeo {
    static constexpr int VL = VLEN<R>;
    static constexpr int GPR = N / VL;                      // vectors per row
    static constexpr int TY = fd_rows(N, GPR);              // rows per tile
    static constexpr int TILES = N / TY;
    static constexpr int NSEG = fd_segments(N, TILES);      // x segments
    static constexpr int XS = N / NSEG;
    static constexpr int NB = TILES * NSEG;                 // workgroups per state
    static constexpr int TV = TY * GPR;                     // vectors per plane tile
    static_assert(N % VL == 0 && TV <= NT, "tile fits the workgroup");
};

// psi = sum_(j<=i) c_j u_j at one vector (FP64 combination, rounded once); KM
// bounds the number of states (i < KM).  Split into the loads and the
// combination, so that a caller can issue the loads early and combine only when
// the values are needed (the combination waits for them).
template <typename R, int KM>
__device__ __forceinline__ void lazy_vec_load(const LatView<R, KM> &vw, size_t off, bool ok, Vec<R> (&u)[KM]) {
#pragma unroll
    for (int j = 0; j < KM; ++j) u[j] = (j <= vw.i && ok) ? *(const ITSE_GLOBAL Vec<R> *)(vw.u[j] + off) : Vec<R>{};
}

template <typename R, int KM>
__device__ __forceinline__ Vec<R> lazy_vec_combine(const LatView<R, KM> &vw, const Vec<R> (&u)[KM], bool ok) {
    constexpr int VL = VLEN<R>;
    Vec<R> out;
#pragma unroll
    for (int k = 0; k < VL; ++k) {
        double a = 0.0;
#pragma unroll
        for (int j = 0; j < KM; ++j)
            if (j <= vw.i && vw.c[j] != 0.0) a += vw.c[j] * (double)u[j][k];
        out[k] = ok ? (R)a : (R)0;
    }
    return out;
}

template <typename R, int KM>
__device__ __forceinline__ Vec<R> lazy_vec(const LatView<R, KM> &vw, size_t off, bool ok) {
    Vec<R> u[KM];
    lazy_vec_load<R, KM>(vw, off, ok, u);
    return lazy_vec_combine<R, KM>(vw, u, ok);
}

template <typename R, int N, int KM>
__global__ void __launch_bounds__(NT) k_fdtd(const JobRef *__restrict__ jobs, int mode) {
    using G = FdGeo<R, N>;
    constexpr int VL = G::VL, GPR = G::GPR, TY = G::TY, XS = G::XS, TV = G::TV;
    __shared__ __attribute__((aligned(16))) R pl[(TY + 2) * N];
    __shared__ double red[NQR * (NT / 64)];
    // flat grid over (segment, tile, job), the job fastest, in XCD-contiguous
    // ranges: the jobs of one tile (which read the same lower states' arrays and V)
    // and neighbouring tiles (which share halo rows) run on the same XCD at nearly
    // the same time, so the repeated reads come from its L2
    const int nj = (int)(gridDim.x / G::NB);
    const int b = xcd_local_index(blockIdx.x, G::NB * nj);
    const int jb = b % nj, wg = b / nj;
    const int tile = wg % G::TILES, seg = wg / G::TILES;
    const int y0 = tile * TY, x0 = seg * XS;
    const JobRef job = jobs[jb];
    const LatDev &L = *job.lat;
    const int i = job.state;
    LatView<R, KM> vw;
    load_view(vw, L, i);
    const ITSE_GLOBAL R *v = gmem((const R *)L.v);
    ITSE_GLOBAL R *u = gmem((R *)state_buf(L, L.step, 1, i));
    ITSE_GLOBAL R *kout = gmem(kout_ptr<R>(L, mode, i));
    const R h = (R)L.h, dt = (R)L.dtau;
    const R cK = (R)(1.0 / (2.0 * L.mass * L.a * L.a));
    const bool mom = L.moments != 0;
    const int center = L.center;
    const double a = L.a;
    const int t = threadIdx.x;
    const bool own = t < TV;
    const int row = own ? t / GPR : 0, g = own ? t % GPR : 0;
    const int y = y0 + row, z0 = g * VL;
    // halo vectors: threads t < 2 GPR load row y0 - 1 (first GPR) or y0 + TY
    const bool hal = t < 2 * GPR;
    const int hrow = hal ? t / GPR : 0, hg = hal ? t % GPR : 0;
    const int hy = hrow == 0 ? y0 - 1 : y0 + TY;
    const bool hin = hal && hy >= 0 && hy < N;
    auto off = [&](int xx, int yy, int zz) { return ((size_t)xx * N + yy) * N + zz; };
    // the planes before the first and after the last are outside the box for
    // x0 = 0 and x0 + XS = N, else real planes of the lattice.
    //
    // Instances of up to three states load the centre rows two planes ahead (plane
    // xx + 2 in iteration xx, combined after the stencil, so that the loads' latency
    // overlaps it).  With four or more the raw loads held across the stencil cost a
    // wave per SIMD: their centre rows are loaded one plane ahead and combined at
    // once.
    constexpr bool AHEAD = KM <= 3;
    Vec<R> pm = lazy_vec<R, KM>(vw, off(x0 > 0 ? x0 - 1 : 0, y, z0), own && x0 > 0);
    Vec<R> pc = lazy_vec<R, KM>(vw, off(x0, y, z0), own);
    Vec<R> pn = AHEAD ? lazy_vec<R, KM>(vw, off(x0 + 1 < N ? x0 + 1 : 0, y, z0), own && x0 + 1 < N) : Vec<R>{};
    Vec<R> hc = lazy_vec<R, KM>(vw, off(x0, hin ? hy : 0, hg * VL), hin);
    Vec<R> vc = own ? *(const ITSE_GLOBAL Vec<R> *)(v + off(x0, y, z0)) : Vec<R>{};
    double acc[NQR];
#pragma unroll
    for (int q = 0; q < NQR; ++q) acc[q] = 0.0;
    const double cy = site_coord(y, N, center, a);
    // the first planes' loads complete here: otherwise the compiler's wait for V
    // inside the loop (a value loaded before it) also waits for the loads that the
    // loop issues ahead
    // (CDNA s_waitcnt immediate: vmcnt in bits 3:0 and 15:14 = 0, expcnt in bits 6:4
    // = 7 and lgkmcnt in bits 11:8 = 15, i.e. wait for vector memory only)
    if constexpr (AHEAD) __builtin_amdgcn_s_waitcnt(0x0f70);
#pragma unroll 1
    for (int xx = x0; xx < x0 + XS; ++xx) {
        // loads for the next iteration: plane xx + 1's halo rows and V, and the
        // centre rows of plane xx + 2 (AHEAD) or of plane xx + 1 (needed now);
        // planes from N on are outside the box (zero)
        const bool more = xx + 1 < x0 + XS;
        const bool n2 = more && xx + 2 < N;
        Vec<R> rn[KM], rh[KM];
        if constexpr (AHEAD) {
            lazy_vec_load<R, KM>(vw, off(n2 ? xx + 2 : 0, y, z0), own && n2, rn);
        } else {
            const bool nx = xx + 1 < N;
            pn = lazy_vec<R, KM>(vw, off(nx ? xx + 1 : 0, y, z0), own && nx);
        }
        const bool hnext = hin && more;
        lazy_vec_load<R, KM>(vw, off(hnext ? xx + 1 : 0, hin ? hy : 0, hg * VL), hnext, rh);
        Vec<R> hn{};
        if constexpr (!AHEAD) hn = lazy_vec_combine<R, KM>(vw, rh, hnext);
        const Vec<R> vn = (own && more) ? *(const ITSE_GLOBAL Vec<R> *)(v + off(xx + 1, y, z0)) : Vec<R>{};
        // plane xx with its halo rows into LDS
        if (own) *(Vec<R> *)&pl[(row + 1) * N + z0] = pc;
        if (hal) *(Vec<R> *)&pl[(hrow == 0 ? 0 : TY + 1) * N + hg * VL] = hc;
        __syncthreads();
        Vec<R> un{}, kv{};
        if (own) {
            const Vec<R> ym = *(const Vec<R> *)&pl[row * N + z0];
            const Vec<R> yp = *(const Vec<R> *)&pl[(row + 2) * N + z0];
            const R zl = z0 > 0 ? pl[(row + 1) * N + z0 - 1] : (R)0;
            const R zr = z0 + VL < N ? pl[(row + 1) * N + z0 + VL] : (R)0;
            const double cx = site_coord(xx, N, center, a);
#pragma unroll
            for (int k = 0; k < VL; ++k) {
                const R left = k > 0 ? pc[k - 1] : zl;
                const R right = k + 1 < VL ? pc[k + 1] : zr;
                const R p_ = pc[k];
                const R kr = cK * ((R)6 * p_ - pm[k] - pn[k] - ym[k] - yp[k] - left - right);
                const R vr = vc[k];
                const R hv = h * vr;
                const R unv = div_fast<R>(p_ * ((R)1 - hv) - dt * kr, (R)1 + hv);
                un[k] = unv;
                kv[k] = kr;
                const double pd = (double)p_;
                acc[RQ_PP] += pd * pd;
                acc[RQ_PK] += pd * (double)kr;
                acc[RQ_VPP] += (double)vr * pd * pd;
                acc[RQ_UU] += (double)unv * (double)unv;
                if (mom) {
                    const double cz = site_coord(z0 + k, N, center, a);
                    const double w2 = pd * pd;
                    acc[RQ_X] += cx * w2;
                    acc[RQ_Y] += cy * w2;
                    acc[RQ_Z] += cz * w2;
                    acc[RQ_R2] += (cx * cx + cy * cy + cz * cz) * w2;
                }
            }
            if constexpr (!AHEAD) {
                if (mode == INV_UPDATE) *(ITSE_GLOBAL Vec<R> *)(u + off(xx, y, z0)) = un;
                else if (mode >= INV_KOUT) *(ITSE_GLOBAL Vec<R> *)(kout + off(xx, y, z0)) = kv;
            }
        }
        if constexpr (AHEAD) {
            // the next iteration's values (this waits for the loads), then this
            // plane's stores, so that the wait does not include their completion
            pm = pc;
            pc = pn;
            pn = lazy_vec_combine<R, KM>(vw, rn, own && n2);
            hc = lazy_vec_combine<R, KM>(vw, rh, hnext);
            vc = vn;
            // keeps the stores below the combination (the compiler would hoist them)
            asm volatile("" ::"v"(pn), "v"(hc), "v"(vc) : "memory");
            if (own) {
                if (mode == INV_UPDATE) *(ITSE_GLOBAL Vec<R> *)(u + off(xx, y, z0)) = un;
                else if (mode >= INV_KOUT) *(ITSE_GLOBAL Vec<R> *)(kout + off(xx, y, z0)) = kv;
            }
            __syncthreads();
        } else {
            __syncthreads();
            pm = pc;
            pc = pn;
            hc = hn;
            vc = vn;
        }
    }
    block_sums<NQR, NT>(acc, L.part_rows + ((size_t)i * L.nb_rows + wg) * NQR, red);
}

// ---------------------------------------------------------------------------
// Reflection projection of u_i in place: u <- (u + sign u o R)/2, R reflecting
// the axes in `axes`; `which` = 1 projects the freshly updated arrays of a step,
// 0 the current ones.  One workgroup per plane x and job; the plane is paired
// with its mirror plane (the workgroup of the larger index exits), each site
// pair {s, R s} is handled by one thread.  Partial sums of |P u|^2 per plane.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(NT) k_project(const JobRef *__restrict__ jobs, int force_sign,
                                                int force_axes, int which) {
    __shared__ double red[NT / 64];
    const JobRef job = jobs[blockIdx.y];
    const LatDev &L = *job.lat;
    const int i = job.state;
    const int sign = force_sign ? force_sign : (L.proj_mode == 2 ? L.psign[i] : 0);
    const int axes = force_sign ? force_axes : L.paxes[i];
    const int n = L.n, center = L.center;
    const int x = blockIdx.x;
    const int xm = (axes & 1) ? mirror_idx(x, n, center) : x;
    double acc[1] = {0.0};
    double *dst = L.part_proj + (size_t)i * L.nb_proj + x;
    if (sign == 0) return;  // uniform over the workgroup
    if (xm < x) {
        if (threadIdx.x == 0) *dst = 0.0;
        return;
    }
    ITSE_GLOBAL R *u = gmem((R *)state_buf(L, L.step, which, i));
    const size_t n2 = (size_t)n * n;
    ITSE_GLOBAL R *pa_ = u + (size_t)x * n2;
    ITSE_GLOBAL R *pb_ = u + (size_t)xm * n2;
    const R sg = (R)sign;
#pragma unroll 4
    for (int e = threadIdx.x; e < (int)n2; e += NT) {
        const int y = e / n, z = e % n;
        const int ym = (axes & 2) ? mirror_idx(y, n, center) : y;
        const int zm = (axes & 4) ? mirror_idx(z, n, center) : z;
        const int m = ym * n + zm;
        if (xm == x && m < e) continue;
        if (xm == x && m == e) {
            const R val = sign > 0 ? pa_[e] : (R)0;
            pa_[e] = val;
            acc[0] += (double)val * (double)val;
        } else {
            const R a = pa_[e], b = pb_[m];
            const R pa = (R)0.5 * (a + sg * b);
            pa_[e] = pa;
            pb_[m] = sg * pa;
            acc[0] += 2.0 * (double)pa * (double)pa;
        }
    }
    block_sums<1, NT>(acc, dst, red);
}

// ---------------------------------------------------------------------------
// Reflection projection of every projected state together with the Gram sums
// <P u_j|P u_l>, j <= l < K, of all states (one lattice per blockIdx.y, KM >= K).
// Used when all projected states reflect the same axes (proj_mode 1): sites are
// taken in mirror pairs {s, R s}, each array is read and (if projected) written
// once, and the Gram sums of the projected values come for free.  With
// proj_mode 2 (different axes) the projections were done by k_project and this
// kernel only sums; with `force` it sums the current arrays without projecting
// (orthogonalisation on request).  Workgroup (plane x, chunk): planes are paired
// with their mirror plane (the larger index contributes zeros).
// ---------------------------------------------------------------------------
template <typename R, int KM>
__global__ void __launch_bounds__(NT) k_project_gram(const JobRef *__restrict__ lats, int force, int which) {
    constexpr int NG = MAXK * (MAXK + 1) / 2;
    constexpr int NGK = KM * (KM + 1) / 2;
    __shared__ double red[NGK * (NT / 64)];
    const LatDev &L = *lats[blockIdx.y].lat;
    const int K = L.nstates;
    const bool ortho = force || (K > 1 && L.ortho_every > 0 && ((L.step + 1) % L.ortho_every) == 0);
    const bool do_proj = !force && L.proj_mode == 1;
    if (!(ortho || (!force && L.proj_mode != 0)) || K > KM) return;  // finalize reads nothing then
    const int n = L.n, center = L.center;
    const int chunks = L.pg_chunks;
    const int axes = do_proj ? L.proj_axes : 0;
    double acc[NGK];
#pragma unroll
    for (int g = 0; g < NGK; ++g) acc[g] = 0.0;
    // threads along z (rows of n sites, NT / n rows at a time), rows [y0, y1) of plane x
    const int rpi = NT / n;
    const int z = threadIdx.x % n, ry = threadIdx.x / n;
    // units (plane x, chunk of rows), strided over the workgroups
    for (int unit = blockIdx.x; unit < n * chunks; unit += gridDim.x) {
        const int x = unit / chunks, ch = unit % chunks;
        const int xm = (axes & 1) ? mirror_idx(x, n, center) : x;
        if (xm >= x && ry < rpi) {
            const size_t n2 = (size_t)n * n;
            ITSE_GLOBAL R *ua[KM];
            ITSE_GLOBAL R *ub[KM];
            R sg[KM];
#pragma unroll
            for (int j = 0; j < KM; ++j) {
                ITSE_GLOBAL R *u = gmem((R *)state_buf(L, L.step, which, j < K ? j : 0));
                ua[j] = u + (size_t)x * n2;
                ub[j] = u + (size_t)xm * n2;
                sg[j] = (do_proj && j < K) ? (R)L.psign[j] : (R)0;
            }
            const int rpc = (n + chunks - 1) / chunks;
            const int y0 = ch * rpc, y1 = y0 + rpc < n ? y0 + rpc : n;
            const int zm = (axes & 4) ? mirror_idx(z, n, center) : z;
            // rows in batches of RB, the loads of the next batch issued before the stores
            // of the current one (stores and loads share the memory wait counter)
            constexpr int RB = 4;
            const int nrows = y0 + ry < y1 ? (y1 - (y0 + ry) + rpi - 1) / rpi : 0;
            const int nbatch = (nrows + RB - 1) / RB;
            R ca[RB][KM], cb[RB][KM];
            auto load_batch = [&](int bi, R (&la)[RB][KM], R (&lb)[RB][KM]) {
#pragma unroll
                for (int t = 0; t < RB; ++t) {
                    const int k = bi * RB + t;
                    const int y = y0 + ry + k * rpi;
                    const int ym = (axes & 2) ? mirror_idx(y, n, center) : y;
                    const bool ok = k < nrows;
                    const int e = ok ? y * n + z : 0, m = ok ? ym * n + zm : 0;
#pragma unroll
                    for (int j = 0; j < KM; ++j) {
                        la[t][j] = (ok && j < K) ? ua[j][e] : (R)0;
                        lb[t][j] = (ok && j < K) ? ub[j][m] : (R)0;
                    }
                }
            };
            if (nbatch > 0) load_batch(0, ca, cb);
            for (int bi = 0; bi < nbatch; ++bi) {
                R na[RB][KM], nb[RB][KM];
                if (bi + 1 < nbatch) load_batch(bi + 1, na, nb);
#pragma unroll
                for (int t = 0; t < RB; ++t) {
                    const int k = bi * RB + t;
                    if (k >= nrows) continue;
                    const int y = y0 + ry + k * rpi;
                    const int ym = (axes & 2) ? mirror_idx(y, n, center) : y;
                    const int e = y * n + z, m = ym * n + zm;
                    const bool self = xm == x && m == e;
                    if (xm == x && m < e) continue;
                    double va[KM], vb[KM];
#pragma unroll
                    for (int j = 0; j < KM; ++j) {
                        va[j] = vb[j] = 0.0;
                        if (j < K) {
                            const R a = ca[t][j];
                            const R b = self ? a : cb[t][j];
                            R pa = a, pb = b;
                            if (sg[j] != (R)0) {
                                if (self) {
                                    pa = pb = sg[j] > (R)0 ? a : (R)0;
                                } else {
                                    pa = (R)0.5 * (a + sg[j] * b);
                                    pb = sg[j] * pa;
                                }
                                ua[j][e] = pa;
                                if (!self) ub[j][m] = pb;
                            }
                            va[j] = (double)pa;
                            vb[j] = self ? 0.0 : (double)pb;
                        }
                    }
                    int g = 0;
#pragma unroll
                    for (int l = 0; l < KM; ++l)
#pragma unroll
                        for (int j = 0; j <= l; ++j) acc[g++] += va[j] * va[l] + vb[j] * vb[l];
                }
                if (bi + 1 < nbatch) {
#pragma unroll
                    for (int t = 0; t < RB; ++t)
#pragma unroll
                        for (int j = 0; j < KM; ++j) {
                            ca[t][j] = na[t][j];
                            cb[t][j] = nb[t][j];
                        }
                }
            }
        }
    }
    // slot layout l (l + 1) / 2 + j, the same for every KM
    block_sums<NGK, NT>(acc, L.part_gram + (size_t)blockIdx.x * NG, red);
}

// ---------------------------------------------------------------------------
// The same projection and Gram sums with 16-byte accesses, for rows of at most
// 64 vectors (GPR = N / VLEN groups of VLEN consecutive z per row).  Workgroup
// (plane x, chunk) with x <= mirror(x) takes the row pairs {A = (x, y),
// B = (xm, ym)} of its rows.  Lane g of a row slot holds group g of A and group
// GPR - 1 - g of B (group g when z is not reflected), so the mirror of each site
// is in the lane's other vector, except for origin centring (z -> -z mod N), where
// element 0 pairs with element 0 of the neighbouring lane's other vector.  A row
// pair is read completely before it is written; a pair that is its own mirror
// (x = xm, y = ym) is written and summed on its A side only.
// ---------------------------------------------------------------------------
template <typename R, int KM, int N>
__device__ __forceinline__ void project_gram_vec_tile(const JobRef *__restrict__ lats, int bx, int gx, int ly,
                                                      int force, int which, double *red) {
    constexpr int NG = MAXK * (MAXK + 1) / 2;
    constexpr int NGK = KM * (KM + 1) / 2;
    constexpr int VL = VLEN<R>;
    constexpr int GPR = N / VL;                 // vectors per row
    constexpr int RPW = 64 / GPR;               // row slots per wave
    constexpr int NWV = NT / 64;
    constexpr int RB = 2;                       // row pairs in flight per slot
    static_assert(N % VL == 0 && GPR <= 64, "rows of at most 64 vectors");
    const LatDev &L = *lats[ly].lat;
    const int K = L.nstates;
    const bool ortho = force || (K > 1 && L.ortho_every > 0 && ((L.step + 1) % L.ortho_every) == 0);
    const bool do_proj = !force && L.proj_mode == 1;
    if (!(ortho || (!force && L.proj_mode != 0)) || K > KM) return;  // finalize reads nothing then
    const int center = L.center;
    const int chunks = L.pg_chunks;
    const int axes = do_proj ? L.proj_axes : 0;
    const bool zr = (axes & 4) != 0;
    const bool origin_z = zr && center != ITSE_CENTER_CELL;
    double acc[NGK];
#pragma unroll
    for (int g = 0; g < NGK; ++g) acc[g] = 0.0;
    const int tid = tile_tid(), lane = tid & 63, wv = tid >> 6;
    const int slot = lane / GPR, g = lane % GPR;
    const int gb = zr ? GPR - 1 - g : g;
    const int src_prev = slot * GPR + (g + GPR - 1) % GPR;  // lane holding group g - 1
    const int src_next = slot * GPR + (g + 1) % GPR;        // lane holding group g + 1
    ITSE_GLOBAL R *uj[KM];
    R sg[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        uj[j] = gmem((R *)state_buf(L, L.step, which, j < K ? j : 0));
        sg[j] = (do_proj && j < K) ? (R)L.psign[j] : (R)0;
    }
    const int rpc = (N + chunks - 1) / chunks;
    constexpr int SLOTS = NWV * RPW;
    // units (plane x, chunk of rows), strided over the workgroups (uniform per
    // workgroup, so every lane of a wave reaches the shuffles below)
    for (int unit = bx; unit < N * chunks; unit += gx) {
        const int x = unit / chunks, ch = unit % chunks;
        const int xm = (axes & 1) ? mirror_idx(x, N, center) : x;
        const int y0 = ch * rpc, y1 = y0 + rpc < N ? y0 + rpc : N;
        const bool active = xm >= x && slot < RPW;
        // row slots of the workgroup step through the chunk's rows together
        for (int yb = y0; yb < y1; yb += SLOTS * RB) {
            Vec<R> va[RB][KM], vb[RB][KM];
            size_t oa[RB], ob[RB];
            bool ok[RB], self[RB];
#pragma unroll
            for (int t = 0; t < RB; ++t) {
                const int y = yb + (t * NWV + wv) * RPW + slot;
                const int ym = (axes & 2) ? mirror_idx(y < N ? y : 0, N, center) : y;
                ok[t] = active && y < y1 && (xm != x || y <= ym);
                self[t] = xm == x && y == ym;
                oa[t] = ok[t] ? ((size_t)x * N + y) * N + (size_t)g * VL : 0;
                ob[t] = ok[t] ? ((size_t)xm * N + ym) * N + (size_t)gb * VL : 0;
                // unconditional loads (inactive lanes read offset 0, states j >= K
                // read u_0), the values masked afterwards: straight-line code, so
                // every load of the round is in flight before the first wait
#pragma unroll
                for (int j = 0; j < KM; ++j) {
                    const Vec<R> la = *(const ITSE_GLOBAL Vec<R> *)(uj[j] + oa[t]);
                    const Vec<R> lb = *(const ITSE_GLOBAL Vec<R> *)(uj[j] + ob[t]);
                    const bool use = ok[t] && j < K;
                    va[t][j] = use ? la : Vec<R>{};
                    vb[t][j] = use ? lb : Vec<R>{};
                }
            }
#pragma unroll
            for (int t = 0; t < RB; ++t) {
                double da[KM][VL], db[KM][VL];
#pragma unroll
                for (int j = 0; j < KM; ++j) {
                    // mirror values of this lane's A and B sites
                    R ma[VL], mb[VL];
                    if (origin_z) {
                        const R b0 = __shfl(vb[t][j][0], src_prev, 64);
                        const R a0 = __shfl(va[t][j][0], src_next, 64);
                        ma[0] = b0;
                        mb[0] = a0;
#pragma unroll
                        for (int k = 1; k < VL; ++k) {
                            ma[k] = vb[t][j][VL - k];
                            mb[k] = va[t][j][VL - k];
                        }
                    } else if (zr) {
#pragma unroll
                        for (int k = 0; k < VL; ++k) {
                            ma[k] = vb[t][j][VL - 1 - k];
                            mb[k] = va[t][j][VL - 1 - k];
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < VL; ++k) {
                            ma[k] = vb[t][j][k];
                            mb[k] = va[t][j][k];
                        }
                    }
                    Vec<R> pa = va[t][j], pb = vb[t][j];
                    if (sg[j] != (R)0) {
#pragma unroll
                        for (int k = 0; k < VL; ++k) {
                            pa[k] = (R)0.5 * (va[t][j][k] + sg[j] * ma[k]);
                            pb[k] = (R)0.5 * (vb[t][j][k] + sg[j] * mb[k]);
                        }
                        if (ok[t]) {
                            *(ITSE_GLOBAL Vec<R> *)(uj[j] + oa[t]) = pa;
                            if (!self[t]) *(ITSE_GLOBAL Vec<R> *)(uj[j] + ob[t]) = pb;
                        }
                    }
                    const bool use_b = ok[t] && !self[t];
#pragma unroll
                    for (int k = 0; k < VL; ++k) {
                        da[j][k] = ok[t] && j < K ? (double)pa[k] : 0.0;
                        db[j][k] = use_b && j < K ? (double)pb[k] : 0.0;
                    }
                }
                int q = 0;
#pragma unroll
                for (int l = 0; l < KM; ++l)
#pragma unroll
                    for (int j = 0; j <= l; ++j) {
#pragma unroll
                        for (int k = 0; k < VL; ++k) acc[q] += da[j][k] * da[l][k] + db[j][k] * db[l][k];
                        ++q;
                    }
            }
        }
    }
    // slot layout l (l + 1) / 2 + j, the same for every KM
    block_sums<NGK, NT>(acc, L.part_gram + (size_t)bx * NG, red);
}

template <typename R, int KM, int N>
__global__ void __launch_bounds__(NT) k_project_gram_vec(const JobRef *__restrict__ lats, int force, int which) {
    __shared__ double red[KM * (KM + 1) / 2 * (NT / 64)];
    project_gram_vec_tile<R, KM, N>(lats, blockIdx.x, gridDim.x, blockIdx.y, force, which, red);
}

// out_i = sum_j coef[j][i] u_j (materialise the current state i), FP64 combination.
template <typename R>
__global__ void __launch_bounds__(NT) k_combine(const JobRef *__restrict__ jobs, void *const *outs) {
    const JobRef job = jobs[blockIdx.y];
    const LatDev &L = *job.lat;
    LatView<R> vw;
    load_view(vw, L, job.state);
    const int n = L.n;
    const size_t n3 = (size_t)n * n * n;
    R *out = (R *)outs[blockIdx.y];
    for (size_t s = (size_t)blockIdx.x * NT + threadIdx.x; s < n3; s += (size_t)gridDim.x * NT)
        out[s] = lazy_psi(vw, s);
}

// ---------------------------------------------------------------------------
// Complex update (complex lattices; runs after the transform passes in mode
// INV_KBUF have written K Re psi and K Im psi to kbuf).  With psi = Re + i Im,
// Re = c u_0, Im = c u_1 (c = coef[0][0] = coef[1][1], the FP64 product rounded
// once as in the passes), V = Vr + i Vi and h = dtau / 2, the map of equation
// iter_proced with complex A and B:
//   psi' = A psi - B dtau K psi = ((1 - h V) psi - dtau K psi) / (1 + h V),
// written to the raw arrays of the next step.  FP64 partial sums per workgroup:
// sum Vi |psi|^2 and sum |psi'|^2 (mode INV_EVAL: sums only).  Grid
// (nb_cplx, lattices); each thread takes two 16-byte vectors per round in a
// stride over the lattice (all loads of a round issued before use).
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(NT) k_complex_update(const JobRef *__restrict__ lats, int mode) {
    constexpr int VL = VLEN<R>;
    constexpr int U = 2;
    __shared__ double red[NQX * (NT / 64)];
    const LatDev &L = *lats[blockIdx.y].lat;
    const size_t n3 = (size_t)L.n * L.n * L.n;
    const size_t nv = n3 / VL;
    const double c = L.coef[0][0];
    const ITSE_GLOBAL R *u0 = gmem((const R *)state_buf(L, L.step, 0, 0));
    const ITSE_GLOBAL R *u1 = gmem((const R *)state_buf(L, L.step, 0, 1));
    ITSE_GLOBAL R *w0 = gmem((R *)state_buf(L, L.step, 1, 0));
    ITSE_GLOBAL R *w1 = gmem((R *)state_buf(L, L.step, 1, 1));
    const ITSE_GLOBAL R *kr = gmem((const R *)L.kbuf);
    const ITSE_GLOBAL R *ki = kr + n3;
    const ITSE_GLOBAL R *vr = gmem((const R *)L.v);
    const ITSE_GLOBAL R *vi = gmem((const R *)L.vi);
    const R h = (R)L.h, dt = (R)L.dtau;
    const size_t stride = (size_t)gridDim.x * NT;
    double acc[NQX] = {0.0, 0.0};
    for (size_t q0 = (size_t)blockIdx.x * NT + threadIdx.x; q0 < nv; q0 += U * stride) {
        Vec<R> a0[U], a1[U], k0[U], k1[U], p0[U], p1[U];
        bool ok[U];
#pragma unroll
        for (int t = 0; t < U; ++t) {
            const size_t q = q0 + t * stride;
            ok[t] = q < nv;
            if (ok[t]) {
                const size_t o = q * VL;
                a0[t] = *(const ITSE_GLOBAL Vec<R> *)(u0 + o);
                a1[t] = *(const ITSE_GLOBAL Vec<R> *)(u1 + o);
                k0[t] = *(const ITSE_GLOBAL Vec<R> *)(kr + o);
                k1[t] = *(const ITSE_GLOBAL Vec<R> *)(ki + o);
                p0[t] = *(const ITSE_GLOBAL Vec<R> *)(vr + o);
                p1[t] = *(const ITSE_GLOBAL Vec<R> *)(vi + o);
            }
        }
#pragma unroll
        for (int t = 0; t < U; ++t) {
            if (!ok[t]) continue;
            Vec<R> n0, n1;
#pragma unroll
            for (int k = 0; k < VL; ++k) {
                const R pr = (R)(c * (double)a0[t][k]), pi = (R)(c * (double)a1[t][k]);
                const R hr = h * p0[t][k], hi = h * p1[t][k];
                // numerator (1 - h V) psi - dtau K psi, denominator d = 1 + h V
                const R nr = pr * ((R)1 - hr) + hi * pi - dt * k0[t][k];
                const R ni = pi * ((R)1 - hr) - hi * pr - dt * k1[t][k];
                const R dr = (R)1 + hr;
                const R inv = div_fast<R>((R)1, dr * dr + hi * hi);
                const R ur = (nr * dr + ni * hi) * inv, ui = (ni * dr - nr * hi) * inv;
                n0[k] = ur;
                n1[k] = ui;
                const double m2 = (double)pr * (double)pr + (double)pi * (double)pi;
                acc[XQ_VIPP] += (double)p1[t][k] * m2;
                acc[XQ_UU] += (double)ur * (double)ur + (double)ui * (double)ui;
            }
            if (mode == INV_UPDATE) {
                const size_t o = (q0 + t * stride) * VL;
                *(ITSE_GLOBAL Vec<R> *)(w0 + o) = n0;
                *(ITSE_GLOBAL Vec<R> *)(w1 + o) = n1;
            }
        }
    }
    block_sums<NQX, NT>(acc, L.part_cplx + (size_t)blockIdx.x * NQX, red);
}

// ---------------------------------------------------------------------------
// Analysis of state psi_i (one job): box normalisation, average radius and parity
// weights in the effective volume |c_l| <= half (sections "Finite volume
// normalization" and "Parity projection").  Workgroup (plane x, chunk of rows);
// per site of the box: psi at the site and at its seven reflections (R1, R2, R4
// reflect x, y, z; combinations by bits), FP64 partial sums in the order
// NA_NORM .. NA_PE3.
// ---------------------------------------------------------------------------
enum AnaQ { NA_NORM = 0, NA_RHO, NA_PPLUS, NA_PMINUS, NA_PE1, NA_PE2, NA_PE3, NAQ };
constexpr int ANA_CHUNKS = 8;

template <typename R>
__global__ void __launch_bounds__(NT) k_analyse(const JobRef *__restrict__ job_, double half, double *parts) {
    __shared__ double red[NAQ * (NT / 64)];
    const JobRef job = *job_;
    const LatDev &L = *job.lat;
    LatView<R> vw;
    load_view(vw, L, job.state);
    const int n = L.n, center = L.center;
    const double a = L.a;
    const int x = blockIdx.x / ANA_CHUNKS, ch = blockIdx.x % ANA_CHUNKS;
    const int rpc = (n + ANA_CHUNKS - 1) / ANA_CHUNKS;
    const int y0 = ch * rpc, y1 = y0 + rpc < n ? y0 + rpc : n;
    const double lim = half * (1.0 + 1e-12);
    double acc[NAQ];
#pragma unroll
    for (int q = 0; q < NAQ; ++q) acc[q] = 0.0;
    const double cx = site_coord(x, n, center, a);
    if (fabs(cx) <= lim) {
        const int mx = mirror_idx(x, n, center);
        for (int e = threadIdx.x; e < (y1 - y0) * n; e += NT) {
            const int y = y0 + e / n, z = e % n;
            const double cy = site_coord(y, n, center, a), cz = site_coord(z, n, center, a);
            if (fabs(cy) > lim || fabs(cz) > lim) continue;
            const int my = mirror_idx(y, n, center), mz = mirror_idx(z, n, center);
            auto at = [&](int xx, int yy, int zz) {
                return (double)lazy_psi(vw, ((size_t)xx * n + yy) * n + zz);
            };
            const double v0 = at(x, y, z), v1 = at(mx, y, z), v2 = at(x, my, z), v3 = at(mx, my, z);
            const double v4 = at(x, y, mz), v5 = at(mx, y, mz), v6 = at(x, my, mz), v7 = at(mx, my, mz);
            const double rho = sqrt(cx * cx + cy * cy + cz * cz) / a;
            const double pp = 0.5 * (v0 + v7), pm = 0.5 * (v0 - v7);
            const double e1 = 0.25 * (v0 + v6 - v1 - v7), e2 = 0.25 * (v0 + v5 - v2 - v7);
            const double e3 = 0.25 * (v0 + v3 - v4 - v7);
            acc[NA_NORM] += v0 * v0;
            acc[NA_RHO] += rho * v0 * v0;
            acc[NA_PPLUS] += pp * pp;
            acc[NA_PMINUS] += pm * pm;
            acc[NA_PE1] += e1 * e1;
            acc[NA_PE2] += e2 * e2;
            acc[NA_PE3] += e3 * e3;
        }
    }
    block_sums<NAQ, NT>(acc, parts + (size_t)blockIdx.x * NAQ, red);
}

// Radial binning of a half spectrum in the standard layout [kx][ky][kz] (kz <= N/2)
// for the momentum-space wave-function: bin b = round(|m|) of the integer momentum
// m on the eigenmode set; per bin the number of momenta, the sum of |m| and of
// |F(m)| over the full spectrum (interior kz count twice: F(-m) = conj F(m)), and
// the total sum of |F|^2.  One workgroup per kx; LDS histograms (FP64 atomics),
// then per-workgroup partials [nbins][3] + 1.
// ---------------------------------------------------------------------------
constexpr int MOM_MAXBINS = 512;

template <typename R>
__global__ void __launch_bounds__(NT) k_momentum_bins(const C2<R> *__restrict__ spec, int n, int nbins,
                                                      double *parts) {
    __shared__ double hist[3 * MOM_MAXBINS];
    __shared__ double red[NT / 64];
    const int h = n / 2 + 1, kx = blockIdx.x;
    for (int b = threadIdx.x; b < 3 * nbins; b += NT) hist[b] = 0.0;
    __syncthreads();
    const int mx = 2 * kx <= n ? kx : kx - n;
    double f2[1] = {0.0};
    for (int e = threadIdx.x; e < n * h; e += NT) {
        const int ky = e / h, kz = e % h;
        const int my = 2 * ky <= n ? ky : ky - n;
        const double w = (kz == 0 || 2 * kz == n) ? 1.0 : 2.0;
        const double mag2 = (double)(mx * mx + my * my + kz * kz);
        const C2<R> f = spec[((size_t)kx * n + ky) * h + kz];
        const double af2 = (double)f.x * (double)f.x + (double)f.y * (double)f.y;
        f2[0] += w * af2;
        const double mag = sqrt(mag2);
        const int b = (int)floor(mag + 0.5);
        if (b < nbins) {
            atomicAdd(&hist[3 * b], w);
            atomicAdd(&hist[3 * b + 1], w * mag);
            atomicAdd(&hist[3 * b + 2], w * sqrt(af2));
        }
    }
    __syncthreads();
    double *out = parts + (size_t)kx * (3 * nbins + 1);
    for (int b = threadIdx.x; b < 3 * nbins; b += NT) out[b] = hist[b];
    block_sums<1, NT>(f2, out + 3 * nbins, red);
}

// Fixed-order sums of `count` partial records of `width` doubles (one workgroup;
// R only makes one instance per precision's translation unit).
template <typename R>
__global__ void __launch_bounds__(NT) k_sum_records(const double *__restrict__ parts, int count, int width,
                                                    double *out) {
    for (int q = threadIdx.x; q < width; q += NT) {
        double s = 0.0;
        for (int b = 0; b < count; ++b) s += parts[(size_t)b * width + q];
        out[q] = s;
    }
}

template <typename S, typename D>
__global__ void __launch_bounds__(NT) k_convert(const S *__restrict__ src, D *__restrict__ dst, size_t count) {
    const size_t stride = (size_t)gridDim.x * NT;
    for (size_t s = (size_t)blockIdx.x * NT + threadIdx.x; s < count; s += stride) dst[s] = (D)src[s];
}

}  // namespace itse
