// Host-side launchers for one precision; included by itse_f32.hip and itse_f64.hip.
#pragma once

#include "itse_kernels.h"

namespace itse {

#define ITSE_FOR_EACH_N(X) \
    X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)

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
    return supported(n) ? 1 : 0;
}

template <typename R>
Sched Launch<R>::schedule(int n, int variant) {
    (void)variant;
    Sched s{};
    switch (n) {
#define ITSE_CASE(NN)                                                      \
    case NN:                                                               \
        s.rows_rp = RowSched<NN>::RP;                                      \
        s.cols_w = ColW<R>::W;                                             \
        s.nb_rows = RowSched<NN>::NB;                                      \
        s.nb_cols = ColSched<R, NN, ColW<R>::W>::NB;                       \
        break;
        ITSE_FOR_EACH_N(ITSE_CASE)
#undef ITSE_CASE
    default:
        break;
    }
    s.nb_proj = flat_blocks(n);
    s.nb_gram = flat_blocks(n);
    return s;
}

template <typename R>
hipError_t Launch<R>::rows_fwd(int n, int variant, const JobRef *jobs, int njobs, hipStream_t s) {
    (void)variant;
    if (njobs <= 0) return hipSuccess;
    switch (n) {
#define ITSE_CASE(NN)                                                                            \
    case NN:                                                                                     \
        hipLaunchKernelGGL((k_rows_fwd<R, NN>), dim3(RowSched<NN>::NB, njobs), dim3(NT), 0, s, jobs); \
        break;
        ITSE_FOR_EACH_N(ITSE_CASE)
#undef ITSE_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R, int NN>
static void launch_cols_n(int mode, int axis, int moments, const JobRef *jobs, int njobs, hipStream_t s) {
    constexpr int W = ColW<R>::W;
    const dim3 grid(ColSched<R, NN, W>::NB, njobs);
    if (mode == COL_FWD)
        hipLaunchKernelGGL((k_cols<R, NN, W, COL_FWD>), grid, dim3(NT), 0, s, jobs, axis, moments);
    else if (mode == COL_INV)
        hipLaunchKernelGGL((k_cols<R, NN, W, COL_INV>), grid, dim3(NT), 0, s, jobs, axis, moments);
    else
        hipLaunchKernelGGL((k_cols<R, NN, W, COL_KIN>), grid, dim3(NT), 0, s, jobs, axis, moments);
}

template <typename R>
hipError_t Launch<R>::cols(int n, int variant, int mode, int axis, int moments, const JobRef *jobs, int njobs,
                           hipStream_t s) {
    (void)variant;
    if (njobs <= 0) return hipSuccess;
    switch (n) {
#define ITSE_CASE(NN)                                                  \
    case NN:                                                           \
        launch_cols_n<R, NN>(mode, axis, moments, jobs, njobs, s);     \
        break;
        ITSE_FOR_EACH_N(ITSE_CASE)
#undef ITSE_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::rows_inv(int n, int variant, int mode, const JobRef *jobs, int njobs, hipStream_t s) {
    (void)variant;
    if (njobs <= 0) return hipSuccess;
    switch (n) {
#define ITSE_CASE(NN)                                                                                   \
    case NN:                                                                                            \
        hipLaunchKernelGGL((k_rows_inv<R, NN>), dim3(RowSched<NN>::NB, njobs), dim3(NT), 0, s, jobs, mode); \
        break;
        ITSE_FOR_EACH_N(ITSE_CASE)
#undef ITSE_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::project(int n, const JobRef *jobs, int njobs, int force_sign, int force_axes,
                              hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_project<R>), dim3(flat_blocks(n), njobs), dim3(NT), 0, s, jobs, force_sign,
                       force_axes);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::gram(int n, const JobRef *lats, int nlats, int force, hipStream_t s) {
    if (nlats <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_gram<R>), dim3(flat_blocks(n), nlats), dim3(NT), 0, s, lats, force);
    return hipGetLastError();
}

template <typename R>
hipError_t Launch<R>::combine(int n, const JobRef *jobs, int njobs, void *const *outs, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_combine<R>), dim3(flat_blocks(n), njobs), dim3(NT), 0, s, jobs, outs);
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
