// FFT building blocks for gfx950: complex arithmetic, small DFTs held in
// registers (radix 2, 3, 4, 6, 8, 12, 16), and Stockham stages over lines held
// in LDS and owned by one wavefront.
//
// Transform convention (the paper's FFT / IFFT of section "Kinetic terms"):
// forward X[k] = sum_n x[n] exp(-2 pi i n k / L), inverse with exp(+2 pi i n k / L),
// both unnormalised.  SIGN = -1 is the forward transform, +1 the inverse.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

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
template <typename R>
__device__ __forceinline__ C2<R> cconj(C2<R> a) { return {a.x, -a.y}; }
// multiply by SIGN * i
template <int SIGN, typename R>
__device__ __forceinline__ C2<R> mul_si(C2<R> a) {
    return SIGN > 0 ? C2<R>{-a.y, a.x} : C2<R>{a.y, -a.x};
}

// The rotation constants of the FP32 butterflies (cos and sin of multiples of
// pi/8 and pi/6) are carried as unevaluated sums hi + lo of two floats (hi the
// float nearest to the value, lo the float nearest to the rest).  With one float
// per constant the rotations would not be unitary, in a systematic way: the floats
// nearest to cos(pi/8), sin(pi/8), sqrt(1/2) and sqrt(3)/2 all lie below those
// values, so every radix-8, -12 and -16 butterfly would shrink the modes it
// rotates (by about 5e-8 per transform at N = 256), and the kinetic energy
// <psi|H_K psi> formed through the transforms would come out low by a few 1e-7
// relative.  a (hi + lo) = a hi + a lo costs one rounding more than a plain
// product and carries no such bias.  The twiddle tables hold one float pair per
// entry, chosen among the neighbours of (cos, sin) for the magnitude closest to 1
// (see the table set-up).  FP64 transforms use one double per constant (their
// bias is at the 1e-16 level).

// a * (w + wl) in FP32: the low part's product first, then the high part's, fused.
__device__ __forceinline__ C2<float> cmul2(C2<float> a, C2<float> w, C2<float> wl) {
    const float lr = a.x * wl.x - a.y * wl.y;
    const float li = a.x * wl.y + a.y * wl.x;
    return {__builtin_fmaf(a.x, w.x, __builtin_fmaf(-a.y, w.y, lr)),
            __builtin_fmaf(a.x, w.y, __builtin_fmaf(a.y, w.x, li))};
}

// a times table twiddle e, conjugated for SIGN > 0.
template <int SIGN, typename R>
__device__ __forceinline__ C2<R> tw_mul(C2<R> a, const C2<R> *tw, int e) {
    C2<R> w = tw[e];
    if (SIGN > 0) w.y = -w.y;
    return cmul(a, w);
}

// cos(2 pi e / R) for R in {16, 12} (R = 8, 6, 4, 3, 2 map onto these).  The
// values are the exact trigonometric constants rounded to double.
__host__ __device__ constexpr double unit_cos(int R, int e) {
    const double c16[16] = {1.0,
                            0.92387953251128675613,
                            0.70710678118654752440,
                            0.38268343236508977173,
                            0.0,
                            -0.38268343236508977173,
                            -0.70710678118654752440,
                            -0.92387953251128675613,
                            -1.0,
                            -0.92387953251128675613,
                            -0.70710678118654752440,
                            -0.38268343236508977173,
                            0.0,
                            0.38268343236508977173,
                            0.70710678118654752440,
                            0.92387953251128675613};
    const double c12[12] = {1.0,  0.86602540378443864676,  0.5,  0.0, -0.5, -0.86602540378443864676,
                            -1.0, -0.86602540378443864676, -0.5, 0.0, 0.5,  0.86602540378443864676};
    e = ((e % R) + R) % R;
    if (16 % R == 0) return c16[e * (16 / R)];
    return c12[e * (12 / R)];
}
// Twiddle exp(SIGN 2 pi i e / R) applied to a, with the trivial angles
// (multiples of pi/2) done without multiplications.
template <int R, int E, int SIGN, typename T>
__device__ __forceinline__ C2<T> twiddle_c(C2<T> a) {
    constexpr int e = ((E % R) + R) % R;
    if constexpr (e == 0) {
        return a;
    } else if constexpr (4 * e == R) {
        return mul_si<SIGN>(a);
    } else if constexpr (2 * e == R) {
        return C2<T>{-a.x, -a.y};
    } else if constexpr (4 * e == 3 * R) {
        return mul_si<-SIGN>(a);
    } else {
        // R in {6, 8, 12, 16} here
        constexpr int RR = (R == 6) ? 12 : R;
        constexpr int EE = (R == 6) ? 2 * e : e;
        constexpr double c = unit_cos(RR, EE);
        constexpr double s = SIGN * unit_cos(RR, EE - RR / 4);
        if constexpr (sizeof(T) == 4) {
            constexpr float ch = (float)c, sh = (float)s;
            constexpr float cl = (float)(c - (double)ch), sl = (float)(s - (double)sh);
            return cmul2(a, C2<T>{ch, sh}, C2<T>{cl, sl});
        } else {
            const C2<T> w{(T)c, (T)s};
            return cmul(a, w);
        }
    }
}

// ---------------------------------------------------------------------------
// Small DFTs in registers: a[0..R) -> X[0..R) in natural order.
// ---------------------------------------------------------------------------
template <int RAD, int SIGN, typename T>
struct Dft;

template <int SIGN, typename T>
struct Dft<1, SIGN, T> {
    static __device__ __forceinline__ void run(C2<T> *) {}
};

template <int SIGN, typename T>
struct Dft<2, SIGN, T> {
    static __device__ __forceinline__ void run(C2<T> *a) {
        const C2<T> t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    }
};

template <int SIGN, typename T>
struct Dft<3, SIGN, T> {
    static __device__ __forceinline__ void run(C2<T> *a) {
        // w = exp(SIGN 2 pi i / 3) = -1/2 + SIGN i sqrt(3)/2
        constexpr double hs3 = 0.86602540378443864676;
        const C2<T> t1 = cadd(a[1], a[2]);
        const C2<T> t2 = {a[0].x - (T)0.5 * t1.x, a[0].y - (T)0.5 * t1.y};
        const C2<T> d = csub(a[1], a[2]);
        C2<T> hd;
        if constexpr (sizeof(T) == 4) {
            constexpr float hh = (float)hs3, hl = (float)(hs3 - (double)hh);
            hd = C2<T>{__builtin_fmaf(hh, d.x, hl * d.x), __builtin_fmaf(hh, d.y, hl * d.y)};
        } else {
            hd = C2<T>{(T)hs3 * d.x, (T)hs3 * d.y};
        }
        const C2<T> r = mul_si<SIGN>(hd);
        a[0] = cadd(a[0], t1);
        a[1] = cadd(t2, r);
        a[2] = csub(t2, r);
    }
};

template <int SIGN, typename T>
struct Dft<4, SIGN, T> {
    static __device__ __forceinline__ void run(C2<T> *a) {
        const C2<T> s0 = cadd(a[0], a[2]), d0 = csub(a[0], a[2]);
        const C2<T> s1 = cadd(a[1], a[3]), d1 = mul_si<SIGN>(csub(a[1], a[3]));
        a[0] = cadd(s0, s1);
        a[2] = csub(s0, s1);
        a[1] = cadd(d0, d1);
        a[3] = csub(d0, d1);
    }
};

// Composite size R = R1 * R2 by one Cooley-Tukey split in registers:
// n = R2 n1 + n2, k = k1 + R1 k2,
// X[k1 + R1 k2] = sum_n2 w_R2^(n2 k2) w_R^(n2 k1) sum_n1 a[R2 n1 + n2] w_R1^(n1 k1).
template <int R1, int R2, int SIGN, typename T>
struct DftSplit {
    static constexpr int R = R1 * R2;
    template <int N2, int K1>
    static __device__ __forceinline__ void tw_one(C2<T> (&b)[R2][R1]) {
        b[N2][K1] = twiddle_c<R, N2 * K1, SIGN>(b[N2][K1]);
    }
    template <int N2, int... K1s>
    static __device__ __forceinline__ void tw_row(C2<T> (&b)[R2][R1], std::integer_sequence<int, K1s...>) {
        (tw_one<N2, K1s>(b), ...);
    }
    template <int... N2s>
    static __device__ __forceinline__ void tw_all(C2<T> (&b)[R2][R1], std::integer_sequence<int, N2s...>) {
        (tw_row<N2s>(b, std::make_integer_sequence<int, R1>{}), ...);
    }
    static __device__ __forceinline__ void run(C2<T> *a) {
        C2<T> b[R2][R1];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) b[n2][n1] = a[R2 * n1 + n2];
            Dft<R1, SIGN, T>::run(b[n2]);
        }
        tw_all(b, std::make_integer_sequence<int, R2>{});
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            C2<T> c[R2];
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) c[n2] = b[n2][k1];
            Dft<R2, SIGN, T>::run(c);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) a[k1 + R1 * k2] = c[k2];
        }
    }
};

template <int SIGN, typename T>
struct Dft<6, SIGN, T> : DftSplit<3, 2, SIGN, T> {};
template <int SIGN, typename T>
struct Dft<8, SIGN, T> : DftSplit<4, 2, SIGN, T> {};
template <int SIGN, typename T>
struct Dft<12, SIGN, T> : DftSplit<4, 3, SIGN, T> {};
template <int SIGN, typename T>
struct Dft<16, SIGN, T> : DftSplit<4, 4, SIGN, T> {};

// ---------------------------------------------------------------------------
// Radix plans: the radix of the first stage of a length-L transform whose
// remaining length is REM.  Large radices first (fewer LDS round trips).
// ---------------------------------------------------------------------------
constexpr bool plan_ok(int L) {
    if (L == 1) return true;
    const int rads[7] = {16, 12, 8, 6, 4, 3, 2};
    for (int i = 0; i < 7; ++i)
        if (L % rads[i] == 0 && plan_ok(L / rads[i])) return true;
    return false;
}
constexpr int stage_radix(int rem) {
    if (rem <= 16 && (rem == 16 || rem == 12 || rem == 8 || rem == 6 || rem == 4 || rem == 3 || rem == 2))
        return rem;
    // prefer 16, then 12, 8: keep the remainder a valid single radix when possible
    const int rads[7] = {16, 12, 8, 6, 4, 3, 2};
    for (int i = 0; i < 7; ++i) {
        const int r = rads[i];
        if (rem % r == 0) {
            const int q = rem / r;
            if (q == 16 || q == 12 || q == 8 || q == 6 || q == 4 || q == 3 || q == 2) return r;
        }
    }
    for (int i = 0; i < 7; ++i)
        if (rem % rads[i] == 0) return rads[i];
    return 1;
}
constexpr int num_stages(int L) {
    int s = 0;
    for (int rem = L; rem > 1; rem /= stage_radix(rem)) ++s;
    return s;
}

// ---------------------------------------------------------------------------
// One Stockham (autosort, decimation in time) stage of radix RAD over LPW lines
// of length L owned by the calling wavefront.  P = product of the radices
// already applied.  Element e of local line l is at buf[l*LS + padded(e)*ES], with
// layout MR for the reads of this stage and MW for its writes (see padded()).  Butterfly j
// (< L/RAD) reads x[j + m L/RAD] (m < RAD), twiddles input m by
// w_L^(k m L/(P RAD)) with k = j mod P, and writes output q to
// (j - k) RAD + k + q P.  Twiddles come from tw[] = w_N^e (N = L * TWS), with
// SIGN applied by conjugation.  LINE_FAST: consecutive lanes take consecutive
// lines (for element-strided layouts), else consecutive butterflies.
//
// All reads of the stage finish before any write of the wavefront (the values
// are in registers), and no other wavefront touches these lines, so no
// workgroup barrier is needed.
// ---------------------------------------------------------------------------
// Slot of element e in the layout between the two stages of a two-stage
// transform with first radix G (e = hi G + lo, lo < G):
//  MODE 0: natural, slot e;
//  MODE 1: one gap after every G elements, slot e + hi (contiguous lines);
//  MODE 2: lo rotated by hi, slot hi G + (lo + hi) mod G (element-strided lines:
//          the first stage's writes, at fixed lo and hi varying over the lanes,
//          and the second stage's reads, at fixed hi and lo varying, both fall on
//          distinct rows mod G, hence on different banks; no extra storage).
template <int MODE, int G>
__device__ __forceinline__ int padded(int e) {
    if constexpr (MODE == 0) {
        return e;
    } else if constexpr (MODE == 1) {
        return e + e / G;
    } else {
        const int hi = e / G, lo = e - hi * G;
        const int r = lo + hi % G;
        return hi * G + (r >= G ? r - G : r);
    }
}

template <typename R, int L, int P, int RAD, int LPW, int SIGN, bool LINE_FAST, int TWS, int MR, int MW, int G>
__device__ __forceinline__ void wave_stage(C2<R> *__restrict__ buf, int LS, int ES,
                                           const C2<R> *__restrict__ tw, int lane) {
    constexpr int B = L / RAD;
    constexpr int TASKS = LPW * B;
    constexpr int TPT = (TASKS + 63) / 64;
    C2<R> v[TPT][RAD];
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const int task = lane + 64 * t;
        if (TASKS % 64 == 0 || task < TASKS) {
            const int line = LINE_FAST ? task % LPW : task / B;
            const int j = LINE_FAST ? task / LPW : task % B;
            const int k = j % P;
            const C2<R> *b = buf + line * LS;
#pragma unroll
            for (int m = 0; m < RAD; ++m) {
                C2<R> a = b[padded<MR, G>(j + m * B) * ES];
                if (P > 1 && m > 0) a = tw_mul<SIGN>(a, tw, (k * m * (L / (P * RAD))) * TWS);
                v[t][m] = a;
            }
            Dft<RAD, SIGN, R>::run(v[t]);
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const int task = lane + 64 * t;
        if (TASKS % 64 == 0 || task < TASKS) {
            const int line = LINE_FAST ? task % LPW : task / B;
            const int j = LINE_FAST ? task / LPW : task % B;
            const int k = j % P;
            C2<R> *b = buf + line * LS;
#pragma unroll
            for (int q = 0; q < RAD; ++q) b[padded<MW, G>((j - k) * RAD + k + q * P) * ES] = v[t][q];
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// Whole transform: successive stages from P = 1.  For a two-stage plan the
// intermediate layout is changed so that the first stage's stride-RAD1 writes do
// not fall on one bank: one gap per RAD1 elements on contiguous lines (the line
// then needs L + L/RAD1 slots), a rotation on element-strided lines.  Input and
// output are in natural order.
template <typename R, int L, int LPW, int SIGN, bool LINE_FAST, int TWS>
struct WaveFft {
    static constexpr int R1 = stage_radix(L);
    static constexpr bool TWO = num_stages(L) == 2;
    static constexpr int MODE = !TWO ? 0 : (LINE_FAST ? 2 : 1);   // intermediate layout
    static constexpr int SPAN = MODE == 1 ? L + L / R1 : L;       // slots a line needs
    template <int P>
    static __device__ __forceinline__ void from(C2<R> *buf, int LS, int ES, const C2<R> *tw, int lane) {
        if constexpr (P < L) {
            constexpr int RAD = stage_radix(L / P);
            static_assert(RAD > 1, "length must factor into 2, 3");
            constexpr int MR = (TWO && P > 1) ? MODE : 0;
            constexpr int MW = (TWO && P == 1) ? MODE : 0;
            wave_stage<R, L, P, RAD, LPW, SIGN, LINE_FAST, TWS, MR, MW, R1>(buf, LS, ES, tw, lane);
            from<P * RAD>(buf, LS, ES, tw, lane);
        }
    }
    static __device__ __forceinline__ void run(C2<R> *buf, int LS, int ES, const C2<R> *tw, int lane) {
        from<1>(buf, LS, ES, tw, lane);
    }
};

// Forward transform, a pointwise map of the spectrum, and inverse transform of
// LPW lines of a two-stage length L = G * G.  The last forward stage leaves in
// the lane of butterfly j the outputs j + G q (q < G), which are exactly the
// inputs of the inverse transform's first butterfly j; so the map and these two
// stages run in registers, with no pass through LDS between them.
// map(line, j, v) receives v[q] = X[j + G q] of local line `line`.
template <typename R, int L, int LPW, bool LINE_FAST, int TWS>
struct WaveFftPair {
    static constexpr int G = stage_radix(L);
    static constexpr bool OK = num_stages(L) == 2 && G * G == L;
    static constexpr int MODE = LINE_FAST ? 2 : 1;
    static constexpr int SPAN = MODE == 1 ? L + L / G : L;
    template <typename F>
    static __device__ __forceinline__ void run(C2<R> *buf, int LS, int ES, const C2<R> *tw, int lane, F &&map) {
        static_assert(OK, "square two-stage lengths only");
        constexpr int B = G;
        constexpr int TASKS = LPW * B;
        constexpr int TPT = (TASKS + 63) / 64;
        wave_stage<R, L, 1, G, LPW, -1, LINE_FAST, TWS, 0, MODE, G>(buf, LS, ES, tw, lane);
        C2<R> v[TPT][G];
#pragma unroll
        for (int t = 0; t < TPT; ++t) {
            const int task = lane + 64 * t;
            if (TASKS % 64 == 0 || task < TASKS) {
                const int line = LINE_FAST ? task % LPW : task / B;
                const int j = LINE_FAST ? task / LPW : task % B;
                const C2<R> *b = buf + line * LS;
                // second forward stage (P = G): input m twiddled by w_L^(j m)
#pragma unroll
                for (int m = 0; m < G; ++m) {
                    C2<R> a = b[padded<MODE, G>(j + m * B) * ES];
                    if (m > 0) a = tw_mul<-1>(a, tw, (j * m) * TWS);
                    v[t][m] = a;
                }
                Dft<G, -1, R>::run(v[t]);
                map(line, j, v[t]);
                // first inverse stage (P = 1): no twiddles
                Dft<G, +1, R>::run(v[t]);
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int t = 0; t < TPT; ++t) {
            const int task = lane + 64 * t;
            if (TASKS % 64 == 0 || task < TASKS) {
                const int line = LINE_FAST ? task % LPW : task / B;
                const int j = LINE_FAST ? task / LPW : task % B;
                C2<R> *b = buf + line * LS;
#pragma unroll
                for (int q = 0; q < G; ++q) b[padded<MODE, G>(j * G + q) * ES] = v[t][q];
            }
        }
        __builtin_amdgcn_wave_barrier();
        wave_stage<R, L, G, G, LPW, +1, LINE_FAST, TWS, MODE, 0, G>(buf, LS, ES, tw, lane);
    }
};

}  // namespace itse
