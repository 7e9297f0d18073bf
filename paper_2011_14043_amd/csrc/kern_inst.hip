// kern_inst.hip -- instantiations of the line-pass kernels, one part per
// compilation (-DFDTD_PART=n, n = 0 .. FDTD_NPARTS-1), so that the parts build
// in parallel.  Each part instantiates the dispatch functions of
// pass_dispatch.hpp for one field/solve type pair and one mode.
#define FDTD_DISPATCH_IMPL
#include "pass_dispatch.hpp"

#ifndef FDTD_PART
#define FDTD_PART 0
#endif

namespace fdtd {

#define FDTD_SINGLE(T, S, MODE)                                                                                    \
    template int dispatch_x_m<T, S, MODE>(int, bool, bool, bool, dim3, dim3, hipStream_t, const PassArgs<T, S>&); \
    template int dispatch_yz_m<T, S, MODE>(int, int, int, bool, bool, bool, dim3, dim3, size_t, hipStream_t,    \
                                           const PassArgs<T, S>&);
#define FDTD_MU(T, S, MODE)                                                                                   \
    template int dispatch_x_mu_m<T, S, MODE>(int, bool, bool, dim3, dim3, hipStream_t, const PassArgs<T, S>&); \
    template int dispatch_yz_mu_m<T, S, MODE>(int, int, int, bool, bool, dim3, dim3, size_t, hipStream_t,      \
                                              const PassArgs<T, S>&);
#define FDTD_BATCH(T, S, MODE)                                                                                 \
    template int dispatch_batch_m<T, S, MODE>(int, int, int, int, bool, dim3, dim3, size_t, hipStream_t,     \
                                              const PassArgs<T, S>*, const int2*, int);

#if FDTD_PART == 0
FDTD_SINGLE(float, float, FUND)
#elif FDTD_PART == 1
FDTD_SINGLE(float, float, CONV_LOD)
#elif FDTD_PART == 2
FDTD_SINGLE(float, float, CONV_ADI)
#elif FDTD_PART == 3
FDTD_SINGLE(float, float, FUND_REF)
#elif FDTD_PART == 4
FDTD_SINGLE(double, double, FUND)
#elif FDTD_PART == 5
FDTD_SINGLE(double, double, CONV_LOD)
#elif FDTD_PART == 6
FDTD_SINGLE(double, double, CONV_ADI)
#elif FDTD_PART == 7
FDTD_SINGLE(float, double, FUND)
#elif FDTD_PART == 8
FDTD_SINGLE(float, double, CONV_LOD)
#elif FDTD_PART == 9
FDTD_SINGLE(float, double, CONV_ADI)
#elif FDTD_PART == 10
FDTD_BATCH(float, float, FUND)
#elif FDTD_PART == 11
FDTD_BATCH(float, float, FUND_REF)
#elif FDTD_PART == 12
FDTD_BATCH(double, double, FUND)
#elif FDTD_PART == 13
FDTD_BATCH(float, double, FUND)
#elif FDTD_PART == 14
FDTD_MU(float, float, FUND)
FDTD_MU(float, float, CONV_LOD)
FDTD_MU(float, float, CONV_ADI)
#elif FDTD_PART == 15
FDTD_MU(double, double, FUND)
FDTD_MU(double, double, CONV_LOD)
FDTD_MU(double, double, CONV_ADI)
#elif FDTD_PART == 16
FDTD_MU(float, double, FUND)
FDTD_MU(float, double, CONV_LOD)
FDTD_MU(float, double, CONV_ADI)
#else
#error "FDTD_PART out of range"
#endif

}  // namespace fdtd
