// pass_dispatch.hpp -- launch of the line-pass kernel variants.
//
// The kernels are instantiated per (field type T, solve type S), chunk size,
// mode, tile and the full-line / material-index / fused-output flags; those
// instantiations dominate the build, so they live in translation units of
// their own (kern_inst.hip, compiled once per part) and the rest of the
// library calls them through the functions declared here.
#pragma once
#include <hip/hip_runtime.h>

#include "batch_kernels.hpp"
#include "pass_kernels.hpp"

namespace fdtd {

// Dispatch results.
enum { DISPATCH_OK = 0, DISPATCH_NOT_BUILT = 1 };

// One single-grid x-line pass of mode MODE (FUND, CONV_LOD, CONV_ADI,
// FUND_REF): chunk M (8 or 16), full lines, material index, fused output.
template <typename T, typename S, int MODE>
int dispatch_x_m(int M, bool full, bool mat, bool fin, dim3 g, dim3 b, hipStream_t st, const PassArgs<T, S>& a);

// One single-grid y/z-line pass of mode MODE and variant {M, TX, NT}.
template <typename T, typename S, int MODE>
int dispatch_yz_m(int M, int TX, int NT, bool full, bool mat, bool fin, dim3 g, dim3 b, size_t lds, hipStream_t st,
                  const PassArgs<T, S>& a);

// Plans with a permeability map (MU variants, modes FUND, CONV_LOD,
// CONV_ADI): x lines with 8-slot chunks, y/z lines of the variants
// kYzMuF32 / kYzMuF64; no material index.
template <typename T, typename S, int MODE>
int dispatch_x_mu_m(int M, bool full, bool fin, dim3 g, dim3 b, hipStream_t st, const PassArgs<T, S>& a);
template <typename T, typename S, int MODE>
int dispatch_yz_mu_m(int M, int TX, int NT, bool full, bool fin, dim3 g, dim3 b, size_t lds, hipStream_t st,
                     const PassArgs<T, S>& a);

// One batched launch of mode MODE (FUND, FUND_REF).  kind 0: x lines alone
// (chunk M); 1: y/z lines of variant {M, TX, NT}; 2: a whole sub-step, y/z
// lines of that variant with the x lines (8-slot chunks) from table entry ex0
// on.
template <typename T, typename S, int MODE>
int dispatch_batch_m(int kind, int M, int TX, int NT, bool mat, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                     const PassArgs<T, S>* tab, const int2* items, int ex0);

// Refined solves exist for FP32 solves only.
template <typename S> struct HasRef { static constexpr bool v = sizeof(S) == 4; };

template <typename T, typename S>
inline int dispatch_x(int kmode, int M, bool full, bool mat, bool fin, dim3 g, dim3 b, hipStream_t st,
                      const PassArgs<T, S>& a) {
    switch (kmode) {
        case FUND: return dispatch_x_m<T, S, FUND>(M, full, mat, fin, g, b, st, a);
        case CONV_LOD: return dispatch_x_m<T, S, CONV_LOD>(M, full, mat, fin, g, b, st, a);
        case CONV_ADI: return dispatch_x_m<T, S, CONV_ADI>(M, full, mat, fin, g, b, st, a);
        case FUND_REF:
            if constexpr (HasRef<S>::v) return dispatch_x_m<T, S, FUND_REF>(M, full, mat, fin, g, b, st, a);
            break;
    }
    return DISPATCH_NOT_BUILT;
}

template <typename T, typename S>
inline int dispatch_yz(int kmode, int M, int TX, int NT, bool full, bool mat, bool fin, dim3 g, dim3 b, size_t lds,
                       hipStream_t st, const PassArgs<T, S>& a) {
    switch (kmode) {
        case FUND: return dispatch_yz_m<T, S, FUND>(M, TX, NT, full, mat, fin, g, b, lds, st, a);
        case CONV_LOD: return dispatch_yz_m<T, S, CONV_LOD>(M, TX, NT, full, mat, fin, g, b, lds, st, a);
        case CONV_ADI: return dispatch_yz_m<T, S, CONV_ADI>(M, TX, NT, full, mat, fin, g, b, lds, st, a);
        case FUND_REF:
            if constexpr (HasRef<S>::v) return dispatch_yz_m<T, S, FUND_REF>(M, TX, NT, full, mat, fin, g, b, lds, st, a);
            break;
    }
    return DISPATCH_NOT_BUILT;
}

template <typename T, typename S>
inline int dispatch_x_mu(int kmode, int M, bool full, bool fin, dim3 g, dim3 b, hipStream_t st,
                         const PassArgs<T, S>& a) {
    switch (kmode) {
        case FUND: return dispatch_x_mu_m<T, S, FUND>(M, full, fin, g, b, st, a);
        case CONV_LOD: return dispatch_x_mu_m<T, S, CONV_LOD>(M, full, fin, g, b, st, a);
        case CONV_ADI: return dispatch_x_mu_m<T, S, CONV_ADI>(M, full, fin, g, b, st, a);
    }
    return DISPATCH_NOT_BUILT;
}

template <typename T, typename S>
inline int dispatch_yz_mu(int kmode, int M, int TX, int NT, bool full, bool fin, dim3 g, dim3 b, size_t lds,
                          hipStream_t st, const PassArgs<T, S>& a) {
    switch (kmode) {
        case FUND: return dispatch_yz_mu_m<T, S, FUND>(M, TX, NT, full, fin, g, b, lds, st, a);
        case CONV_LOD: return dispatch_yz_mu_m<T, S, CONV_LOD>(M, TX, NT, full, fin, g, b, lds, st, a);
        case CONV_ADI: return dispatch_yz_mu_m<T, S, CONV_ADI>(M, TX, NT, full, fin, g, b, lds, st, a);
    }
    return DISPATCH_NOT_BUILT;
}

template <typename T, typename S>
inline int dispatch_batch(int kmode, int kind, int M, int TX, int NT, bool mat, dim3 grid, dim3 block, size_t lds,
                          hipStream_t st, const PassArgs<T, S>* tab, const int2* items, int ex0) {
    if (kmode == FUND) return dispatch_batch_m<T, S, FUND>(kind, M, TX, NT, mat, grid, block, lds, st, tab, items, ex0);
    if constexpr (HasRef<S>::v) {
        if (kmode == FUND_REF)
            return dispatch_batch_m<T, S, FUND_REF>(kind, M, TX, NT, mat, grid, block, lds, st, tab, items, ex0);
    }
    return DISPATCH_NOT_BUILT;
}

#ifdef FDTD_DISPATCH_IMPL

// Refined solves are built for FP32: x lines with 8-slot chunks, y/z lines
// with 8- or 16-slot chunks.
template <typename S, int M> struct HasRefX { static constexpr bool v = sizeof(S) == 4 && M == 8; };
template <typename S, int M> struct HasRefYZ { static constexpr bool v = sizeof(S) == 4 && (M == 8 || M == 16); };

template <typename T, typename S, int M, int MODE, bool FULL, bool MAT>
void launch_x_fin(bool fin, dim3 g, dim3 b, hipStream_t st, const PassArgs<T, S>& a) {
    if (fin) hipLaunchKernelGGL((pass_x_kernel<T, S, M, MODE, FULL, MAT, true>), g, b, 0, st, a);
    else hipLaunchKernelGGL((pass_x_kernel<T, S, M, MODE, FULL, MAT, false>), g, b, 0, st, a);
}
template <typename T, typename S, int M, int MODE>
int launch_x(bool full, bool mat, bool fin, dim3 g, dim3 b, hipStream_t st, const PassArgs<T, S>& a) {
    if constexpr (MODE == FUND_REF && !HasRefX<S, M>::v) {
        return DISPATCH_NOT_BUILT;
    } else {
        if (full) {
            if (mat) launch_x_fin<T, S, M, MODE, true, true>(fin, g, b, st, a);
            else launch_x_fin<T, S, M, MODE, true, false>(fin, g, b, st, a);
        } else {
            if (mat) launch_x_fin<T, S, M, MODE, false, true>(fin, g, b, st, a);
            else launch_x_fin<T, S, M, MODE, false, false>(fin, g, b, st, a);
        }
        return DISPATCH_OK;
    }
}

template <typename T, typename S, int MODE>
int dispatch_x_m(int M, bool full, bool mat, bool fin, dim3 g, dim3 b, hipStream_t st, const PassArgs<T, S>& a) {
    if (M == 8) return launch_x<T, S, 8, MODE>(full, mat, fin, g, b, st, a);
    if (M == 16) return launch_x<T, S, 16, MODE>(full, mat, fin, g, b, st, a);
    return DISPATCH_NOT_BUILT;
}

template <typename T, typename S, int M, int TX, int NT, int MODE, bool FULL, bool MAT>
void launch_yz_fin(bool fin, dim3 g, dim3 b, size_t lds, hipStream_t st, const PassArgs<T, S>& a) {
    if (fin) hipLaunchKernelGGL((pass_yz_kernel<T, S, M, MODE, TX, NT, FULL, MAT, true>), g, b, lds, st, a);
    else hipLaunchKernelGGL((pass_yz_kernel<T, S, M, MODE, TX, NT, FULL, MAT, false>), g, b, lds, st, a);
}
template <typename T, typename S, int M, int TX, int NT, int MODE>
int launch_yz(bool full, bool mat, bool fin, dim3 g, dim3 b, size_t lds, hipStream_t st, const PassArgs<T, S>& a) {
    if constexpr (MODE == FUND_REF && !HasRefYZ<S, M>::v) {
        return DISPATCH_NOT_BUILT;
    } else {
        if (full) {
            if (mat) launch_yz_fin<T, S, M, TX, NT, MODE, true, true>(fin, g, b, lds, st, a);
            else launch_yz_fin<T, S, M, TX, NT, MODE, true, false>(fin, g, b, lds, st, a);
        } else {
            if (mat) launch_yz_fin<T, S, M, TX, NT, MODE, false, true>(fin, g, b, lds, st, a);
            else launch_yz_fin<T, S, M, TX, NT, MODE, false, false>(fin, g, b, lds, st, a);
        }
        return DISPATCH_OK;
    }
}

// The y/z variants {M, TX, NT} built per solve precision (the lists the
// autotuner draws from, kYzF32 and kYzF64).
template <typename T, typename S, int MODE>
int dispatch_yz_m(int M, int TX, int NT, bool full, bool mat, bool fin, dim3 g, dim3 b, size_t lds, hipStream_t st,
                  const PassArgs<T, S>& a) {
#define CASE_YZ(MM, TT, NN) \
    if (M == MM && TX == TT && NT == NN) return launch_yz<T, S, MM, TT, NN, MODE>(full, mat, fin, g, b, lds, st, a);
    if constexpr (sizeof(S) == 4) {
        CASE_YZ(16, 32, 1024) CASE_YZ(16, 16, 512) CASE_YZ(8, 16, 1024) CASE_YZ(32, 16, 512) CASE_YZ(8, 32, 512)
    } else {
        CASE_YZ(16, 16, 512) CASE_YZ(8, 8, 512) CASE_YZ(8, 16, 1024)
    }
#undef CASE_YZ
    return DISPATCH_NOT_BUILT;
}

// Permeability-map variants (the fused output form only for the
// fundamental forms).
template <typename T, typename S, int MODE>
int dispatch_x_mu_m(int M, bool full, bool fin, dim3 g, dim3 b, hipStream_t st, const PassArgs<T, S>& a) {
    if (M != 8 || (fin && MODE != FUND)) return DISPATCH_NOT_BUILT;
    if constexpr (MODE == FUND) {
        if (fin) {
            if (full) hipLaunchKernelGGL((pass_x_kernel<T, S, 8, MODE, true, false, true, true>), g, b, 0, st, a);
            else hipLaunchKernelGGL((pass_x_kernel<T, S, 8, MODE, false, false, true, true>), g, b, 0, st, a);
            return DISPATCH_OK;
        }
    }
    if (full) hipLaunchKernelGGL((pass_x_kernel<T, S, 8, MODE, true, false, false, true>), g, b, 0, st, a);
    else hipLaunchKernelGGL((pass_x_kernel<T, S, 8, MODE, false, false, false, true>), g, b, 0, st, a);
    return DISPATCH_OK;
}

template <typename T, typename S, int M, int TX, int NT, int MODE>
int launch_yz_mu(bool full, bool fin, dim3 g, dim3 b, size_t lds, hipStream_t st, const PassArgs<T, S>& a) {
    if (fin && MODE != FUND) return DISPATCH_NOT_BUILT;
    if constexpr (MODE == FUND) {
        if (fin) {
            if (full)
                hipLaunchKernelGGL((pass_yz_kernel<T, S, M, MODE, TX, NT, true, false, true, true>), g, b, lds, st, a);
            else
                hipLaunchKernelGGL((pass_yz_kernel<T, S, M, MODE, TX, NT, false, false, true, true>), g, b, lds, st, a);
            return DISPATCH_OK;
        }
    }
    if (full) hipLaunchKernelGGL((pass_yz_kernel<T, S, M, MODE, TX, NT, true, false, false, true>), g, b, lds, st, a);
    else hipLaunchKernelGGL((pass_yz_kernel<T, S, M, MODE, TX, NT, false, false, false, true>), g, b, lds, st, a);
    return DISPATCH_OK;
}

template <typename T, typename S, int MODE>
int dispatch_yz_mu_m(int M, int TX, int NT, bool full, bool fin, dim3 g, dim3 b, size_t lds, hipStream_t st,
                     const PassArgs<T, S>& a) {
#define CASE_YZ_MU(MM, TT, NN) \
    if (M == MM && TX == TT && NT == NN) return launch_yz_mu<T, S, MM, TT, NN, MODE>(full, fin, g, b, lds, st, a);
    if constexpr (sizeof(S) == 4) {
        CASE_YZ_MU(16, 16, 512) CASE_YZ_MU(8, 16, 512) CASE_YZ_MU(8, 8, 512)
    } else {
        CASE_YZ_MU(8, 16, 512) CASE_YZ_MU(8, 8, 512)
    }
#undef CASE_YZ_MU
    return DISPATCH_NOT_BUILT;
}

template <typename T, typename S, int MODE>
int dispatch_batch_m(int kind, int M, int TX, int NT, bool mat, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                        const PassArgs<T, S>* tab, const int2* items, int ex0) {
    if (kind == 2) {
        // fused sub-step: x lines with 8-slot chunks inside the y/z launch
#define CASE_SUB(MM, TT, NN)                                                                                         \
    if (M == MM && TX == TT && NN == NT) {                                                                           \
        if constexpr (MODE != FUND_REF || MM == 8 || (MM == 16 && NN == 512)) {                                                                 \
            if (mat)                                                                                                 \
                hipLaunchKernelGGL((pass_sub_batch_kernel<T, S, 8, MM, MODE, TT, NN, true>), grid, block, lds, st,  \
                                   tab, items, ex0);                                                                 \
            else                                                                                                     \
                hipLaunchKernelGGL((pass_sub_batch_kernel<T, S, 8, MM, MODE, TT, NN, false>), grid, block, lds, st, \
                                   tab, items, ex0);                                                                 \
            return DISPATCH_OK;                                                                                      \
        }                                                                                                            \
        return DISPATCH_NOT_BUILT;                                                                                   \
    }
        if constexpr (sizeof(S) == 4) {
            CASE_SUB(8, 16, 1024) CASE_SUB(8, 32, 512) CASE_SUB(16, 32, 1024) CASE_SUB(16, 16, 512)
        } else {
            CASE_SUB(8, 8, 512) CASE_SUB(8, 16, 1024) CASE_SUB(16, 16, 512)
        }
#undef CASE_SUB
        return DISPATCH_NOT_BUILT;
    }
    if (kind == 0) {
        if (M == 8) {
            if (mat) hipLaunchKernelGGL((pass_x_batch_kernel<T, S, 8, MODE, true>), grid, block, 0, st, tab, items);
            else hipLaunchKernelGGL((pass_x_batch_kernel<T, S, 8, MODE, false>), grid, block, 0, st, tab, items);
            return DISPATCH_OK;
        }
        if constexpr (MODE != FUND_REF) {
            if (M == 16) {
                if (mat) hipLaunchKernelGGL((pass_x_batch_kernel<T, S, 16, MODE, true>), grid, block, 0, st, tab, items);
                else hipLaunchKernelGGL((pass_x_batch_kernel<T, S, 16, MODE, false>), grid, block, 0, st, tab, items);
                return DISPATCH_OK;
            }
        }
        return DISPATCH_NOT_BUILT;
    }
#define CASE_YZB(MM, TT, NN)                                                                                      \
    if (M == MM && TX == TT && NT == NN) {                                                                        \
        if constexpr (MODE != FUND_REF || MM == 8 || (MM == 16 && NN == 512)) {                                                              \
            if (mat)                                                                                              \
                hipLaunchKernelGGL((pass_yz_batch_kernel<T, S, MM, MODE, TT, NN, true>), grid, block, lds, st, tab, \
                                   items);                                                                        \
            else                                                                                                  \
                hipLaunchKernelGGL((pass_yz_batch_kernel<T, S, MM, MODE, TT, NN, false>), grid, block, lds, st,    \
                                   tab, items);                                                                   \
            return DISPATCH_OK;                                                                                   \
        }                                                                                                         \
        return DISPATCH_NOT_BUILT;                                                                                \
    }
    if constexpr (sizeof(S) == 4) {
        CASE_YZB(16, 32, 1024) CASE_YZB(16, 16, 512) CASE_YZB(8, 16, 1024) CASE_YZB(32, 16, 512) CASE_YZB(8, 32, 512)
    } else {
        CASE_YZB(16, 16, 512) CASE_YZB(8, 8, 512) CASE_YZB(8, 16, 1024)
    }
#undef CASE_YZB
    return DISPATCH_NOT_BUILT;
}

#endif  // FDTD_DISPATCH_IMPL

}  // namespace fdtd
