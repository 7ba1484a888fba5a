// Host-side launchers for one precision; included by itse_f32.hip and itse_f64.hip.
#pragma once

#include "itse_pass.h"

namespace itse {

// Lattice sizes with compiled passes, and the schedule variants of each.
#define ITSE_FOR_EACH_N(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256)

template <typename R, int N>
struct NVariants {
    static constexpr int value = 1;
};
template <>
struct NVariants<float, 32> {
    static constexpr int value = 3;
};
template <>
struct NVariants<float, 48> {
    static constexpr int value = 3;
};
template <>
struct NVariants<float, 64> {
    static constexpr int value = 3;
};
template <>
struct NVariants<float, 96> {
    static constexpr int value = 4;
};
template <>
struct NVariants<float, 128> {
    static constexpr int value = 2;
};
template <>
struct NVariants<float, 256> {
    static constexpr int value = 6;
};
template <>
struct NVariants<double, 256> {
    static constexpr int value = 2;
};

template <typename R, int N, int V>
static Sched sched_of() {
    using PV = PassVariants<R, N, V>;
    using G = Geo<R, N, PV::COLS>;
    Sched s{};
    s.split = G::S;
    s.nwp = G::NWP;
    s.cols_w = G::W;
    s.nwc = G::NWC;
    // one partial-sum block per inverse plane-pass workgroup
    s.nb_rows = Geo<R, N, PV::INV>::NB_PLANE;
    s.nb_cols = G::NB_COLS;
    s.nb_proj = N;
    s.nb_gram = pg_blocks(N);
    s.lds_plane = (int)(G::PLANE_ELEMS * sizeof(C2<R>) + N * sizeof(C2<R>));
    s.lds_cols = (int)(N * G::CS * sizeof(C2<R>) + N * sizeof(C2<R>) + N * sizeof(double));
    return s;
}

// Calls F.template operator()<N, V>() for the runtime (n, variant).
template <typename R, typename F>
static hipError_t dispatch(int n, int variant, F f) {
    switch (n) {
#define ITSE_CASE(NN)                                                                  \
    case NN:                                                                           \
        if (variant == 0 || NVariants<R, NN>::value == 1) return f.template operator()<NN, 0>(); \
        if constexpr (NVariants<R, NN>::value > 1)                                     \
            if (variant == 1) return f.template operator()<NN, 1>();                   \
        if constexpr (NVariants<R, NN>::value > 2)                                     \
            if (variant == 2) return f.template operator()<NN, 2>();                   \
        if constexpr (NVariants<R, NN>::value > 3)                                     \
            if (variant == 3) return f.template operator()<NN, 3>();                   \
        if constexpr (NVariants<R, NN>::value > 4)                                     \
            if (variant == 4) return f.template operator()<NN, 4>();                   \
        if constexpr (NVariants<R, NN>::value > 5)                                     \
            if (variant == 5) return f.template operator()<NN, 5>();                   \
        return hipErrorInvalidValue;
        ITSE_FOR_EACH_N(ITSE_CASE)
#undef ITSE_CASE
    default:
        return hipErrorInvalidValue;
    }
}

template <typename R>
bool Launch<R>::supported(int n) {
    switch (n) {
#define ITSE_CASE(NN) case NN:
        ITSE_FOR_EACH_N(ITSE_CASE)
#undef ITSE_CASE
        return true;
    default:
        return false;
    }
}

template <typename R>
int Launch<R>::variants(int n) {
    switch (n) {
#define ITSE_CASE(NN) \
    case NN:          \
        return NVariants<R, NN>::value;
        ITSE_FOR_EACH_N(ITSE_CASE)
#undef ITSE_CASE
    default:
        return 0;
    }
}

template <typename R>
struct SchedF {
    Sched *o;
    template <int N, int V>
    hipError_t operator()() {
        *o = sched_of<R, N, V>();
        return hipSuccess;
    }
};

template <typename R>
Sched Launch<R>::schedule(int n, int variant) {
    Sched out{};
    (void)dispatch<R>(n, variant, SchedF<R>{&out});
    return out;
}

// Bound on the number of states of the lattices a plane-pass launch serves: the
// instance with the smallest bound >= kmax (1, 4 or MAXK).
template <typename F>
static hipError_t with_state_bound(int kmax, F f) {
    if (kmax <= 1) return f(std::integral_constant<int, 1>{});
    if (kmax <= 4) return f(std::integral_constant<int, 4>{});
    return f(std::integral_constant<int, MAXK>{});
}

// Grid of the inverse plane pass: with SPLIT, half as many sub-planes (the
// layout's) and each job twice (its two halves; see plane_tile).
template <int NB, bool SPLIT>
inline dim3 split_grid(int njobs) {
    return SPLIT ? plane_grid<NB / 2>(2 * njobs) : plane_grid<NB>(njobs);
}

template <typename R>
struct PlaneFwdF {
    int kmax;
    const JobRef *jobs;
    int njobs;
    hipStream_t s;
    template <int N, int V0>
    hipError_t operator()() {
        using PV = PassVariants<R, N, V0>;
        constexpr int V = PV::FWD;
        using G = Geo<R, N, V>;
        static_assert(G::S == Geo<R, N, PV::COLS>::S, "the forward pass writes the column pass's layout");
        return with_state_bound(kmax, [&](auto kc) {
            constexpr int KM = decltype(kc)::value;
            hipLaunchKernelGGL((k_plane_fwd<R, N, V, KM>), plane_grid<G::NB_PLANE>(njobs), dim3(G::NTP), 0, s, jobs);
            return hipGetLastError();
        });
    }
};

template <typename R>
hipError_t Launch<R>::plane_fwd(int n, int variant, int kmax, const JobRef *jobs, int njobs, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    return dispatch<R>(n, variant, PlaneFwdF<R>{kmax, jobs, njobs, s});
}

template <typename R>
struct ColumnsF {
    int mode, moments;
    const JobRef *jobs;
    int njobs;
    void *out;
    hipStream_t s;
    template <int N, int V0>
    hipError_t operator()() {
        constexpr int V = PassVariants<R, N, V0>::COLS;
        using G = Geo<R, N, V>;
        hipLaunchKernelGGL((k_columns<R, N, V>), dim3(G::NB_COLS, njobs), dim3(G::NTC), 0, s, jobs, mode, moments,
                           (C2<R> *)out);
        return hipGetLastError();
    }
};

template <typename R>
hipError_t Launch<R>::columns(int n, int variant, int mode, int moments, const JobRef *jobs, int njobs, void *out,
                              hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    return dispatch<R>(n, variant, ColumnsF<R>{mode, moments, jobs, njobs, out, s});
}

template <typename R>
struct PlaneInvF {
    int mode, mom, kmax;
    const JobRef *jobs;
    int njobs;
    hipStream_t s;
    template <int N, int V0>
    hipError_t operator()() {
        using PV = PassVariants<R, N, V0>;
        constexpr int V = PV::INV;
        using G = Geo<R, N, V>;
        static_assert(PV::SPLIT_INV ? G::S == 2 * Geo<R, N, PV::COLS>::S : G::S == Geo<R, N, PV::COLS>::S,
                      "the inverse pass reads the column pass's layout");
        return with_state_bound(kmax, [&](auto kc) {
            constexpr int KM = decltype(kc)::value;
            const dim3 grid = split_grid<G::NB_PLANE, PV::SPLIT_INV>(njobs);
            if (mom)
                hipLaunchKernelGGL((k_plane_inv<R, N, V, true, KM, false, PV::SPLIT_INV>), grid, dim3(G::NTP), 0, s,
                                   jobs, mode);
            else
                hipLaunchKernelGGL((k_plane_inv<R, N, V, false, KM, false, PV::SPLIT_INV>), grid, dim3(G::NTP), 0, s,
                                   jobs, mode);
            return hipGetLastError();
        });
    }
};

template <typename R>
hipError_t Launch<R>::plane_inv(int n, int variant, int mode, int moments, int kmax, const JobRef *jobs, int njobs,
                                hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    return dispatch<R>(n, variant, PlaneInvF<R>{mode, moments, kmax, jobs, njobs, s});
}

template <typename R>
struct PlaneInvCplxF {
    const JobRef *jobs;
    int njobs;
    hipStream_t s;
    template <int N, int V0>
    hipError_t operator()() {
        using PV = PassVariants<R, N, V0>;
        constexpr int V = PV::INV;
        using G = Geo<R, N, V>;
        const dim3 grid = split_grid<G::NB_PLANE, PV::SPLIT_INV>(njobs);
        hipLaunchKernelGGL((k_plane_inv<R, N, V, false, 4, true, PV::SPLIT_INV>), grid, dim3(G::NTP), 0, s, jobs,
                           (int)INV_UPDATE);
        return hipGetLastError();
    }
};

template <typename R>
hipError_t Launch<R>::plane_inv_cplx(int n, int variant, const JobRef *jobs, int njobs, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    return dispatch<R>(n, variant, PlaneInvCplxF<R>{jobs, njobs, s});
}

template <typename R>
hipError_t Launch<R>::project(int n, const JobRef *jobs, int njobs, int force_sign, int force_axes, int which,
                              hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_project<R>), dim3(n, njobs), dim3(NT), 0, s, jobs, force_sign, force_axes, which);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::project_gram(int n, int kmax, const JobRef *lats, int nlats, int force, int which,
                                   hipStream_t s) {
    if (nlats <= 0) return hipSuccess;
    const dim3 grid(pg_blocks(n), nlats);
    if (kmax <= 4 && n / VLEN<R> <= 64) {
        // 16-byte form (rows of at most 64 vectors, up to four states)
        auto vec = [&](auto nc) -> hipError_t {
            constexpr int NN = decltype(nc)::value;
            if constexpr (NN % VLEN<R> == 0 && NN / VLEN<R> <= 64) {
                if (kmax <= 1)
                    hipLaunchKernelGGL((k_project_gram_vec<R, 1, NN>), grid, dim3(NT), 0, s, lats, force, which);
                else if (kmax <= 2)
                    hipLaunchKernelGGL((k_project_gram_vec<R, 2, NN>), grid, dim3(NT), 0, s, lats, force, which);
                else if (kmax <= 3)
                    hipLaunchKernelGGL((k_project_gram_vec<R, 3, NN>), grid, dim3(NT), 0, s, lats, force, which);
                else
                    hipLaunchKernelGGL((k_project_gram_vec<R, 4, NN>), grid, dim3(NT), 0, s, lats, force, which);
                return hipGetLastError();
            }
            return hipErrorInvalidValue;
        };
        switch (n) {
#define ITSE_CASE(NN) \
    case NN: return vec(std::integral_constant<int, NN>{});
            ITSE_FOR_EACH_N(ITSE_CASE)
#undef ITSE_CASE
        default: return hipErrorInvalidValue;
        }
    }
    if (kmax <= 1) hipLaunchKernelGGL((k_project_gram<R, 1>), grid, dim3(NT), 0, s, lats, force, which);
    else if (kmax <= 2) hipLaunchKernelGGL((k_project_gram<R, 2>), grid, dim3(NT), 0, s, lats, force, which);
    else if (kmax <= 3) hipLaunchKernelGGL((k_project_gram<R, 3>), grid, dim3(NT), 0, s, lats, force, which);
    else if (kmax <= 4) hipLaunchKernelGGL((k_project_gram<R, 4>), grid, dim3(NT), 0, s, lats, force, which);
    else hipLaunchKernelGGL((k_project_gram<R, MAXK>), grid, dim3(NT), 0, s, lats, force, which);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::fdtd(int n, int kmax, int mode, const JobRef *jobs, int njobs, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    auto go = [&](auto nc) -> hipError_t {
        constexpr int NN = decltype(nc)::value;
        const dim3 grid(FdGeo<R, NN>::NB * njobs);
        if (kmax <= 1) hipLaunchKernelGGL((k_fdtd<R, NN, 1>), grid, dim3(NT), 0, s, jobs, mode);
        else if (kmax <= 2) hipLaunchKernelGGL((k_fdtd<R, NN, 2>), grid, dim3(NT), 0, s, jobs, mode);
        else if (kmax <= 3) hipLaunchKernelGGL((k_fdtd<R, NN, 3>), grid, dim3(NT), 0, s, jobs, mode);
        else if (kmax <= 4) hipLaunchKernelGGL((k_fdtd<R, NN, 4>), grid, dim3(NT), 0, s, jobs, mode);
        else hipLaunchKernelGGL((k_fdtd<R, NN, MAXK>), grid, dim3(NT), 0, s, jobs, mode);
        return hipGetLastError();
    };
    switch (n) {
#define ITSE_CASE(NN) \
    case NN: return go(std::integral_constant<int, NN>{});
        ITSE_FOR_EACH_N(ITSE_CASE)
#undef ITSE_CASE
    default:
        return hipErrorInvalidValue;
    }
}

template <typename R>
int Launch<R>::fdtd_blocks(int n) {
    switch (n) {
#define ITSE_CASE(NN) \
    case NN: return FdGeo<R, NN>::NB;
        ITSE_FOR_EACH_N(ITSE_CASE)
#undef ITSE_CASE
    default:
        return 0;
    }
}

template <typename R>
size_t Launch<R>::analyse_parts(int n) {
    return (size_t)n * ANA_CHUNKS * NAQ;
}

template <typename R>
hipError_t Launch<R>::analyse(int n, const JobRef *job, double half, double *parts, double *out, hipStream_t s) {
    hipLaunchKernelGGL((k_analyse<R>), dim3(n * ANA_CHUNKS), dim3(NT), 0, s, job, half, parts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sum_records<R>), dim3(1), dim3(NT), 0, s, (const double *)parts, n * ANA_CHUNKS, (int)NAQ,
                       out);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::momentum_bins(int n, const void *spec, int nbins, double *parts, double *out, hipStream_t s) {
    if (nbins < 1 || nbins > MOM_MAXBINS) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_momentum_bins<R>), dim3(n), dim3(NT), 0, s, (const C2<R> *)spec, n, nbins, parts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sum_records<R>), dim3(1), dim3(NT), 0, s, (const double *)parts, n, 3 * nbins + 1, out);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::combine(int n, const JobRef *jobs, int njobs, void *const *outs, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_combine<R>), dim3(flat_blocks(n), njobs), dim3(NT), 0, s, jobs, outs);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::complex_update(int n, int nb, const JobRef *lats, int nlats, int mode, hipStream_t s) {
    if (nlats <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_complex_update<R>), dim3(nb, nlats), dim3(NT), 0, s, lats, mode);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::convert_in(const void *src, int src_dtype, void *dst, size_t count, hipStream_t s) {
    const int blocks = (int)((count + NT - 1) / NT < 65536 ? (count + NT - 1) / NT : 65536);
    if (count == 0) return hipSuccess;
    if (src_dtype == ITSE_DTYPE_F32)
        hipLaunchKernelGGL((k_convert<float, R>), dim3(blocks), dim3(NT), 0, s, (const float *)src, (R *)dst, count);
    else
        hipLaunchKernelGGL((k_convert<double, R>), dim3(blocks), dim3(NT), 0, s, (const double *)src, (R *)dst,
                           count);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::convert_out(const void *src, void *dst, int dst_dtype, size_t count, hipStream_t s) {
    const int blocks = (int)((count + NT - 1) / NT < 65536 ? (count + NT - 1) / NT : 65536);
    if (count == 0) return hipSuccess;
    if (dst_dtype == ITSE_DTYPE_F32)
        hipLaunchKernelGGL((k_convert<R, float>), dim3(blocks), dim3(NT), 0, s, (const R *)src, (float *)dst, count);
    else
        hipLaunchKernelGGL((k_convert<R, double>), dim3(blocks), dim3(NT), 0, s, (const R *)src, (double *)dst,
                           count);
    return hipGetLastError();
}

}  // namespace itse
