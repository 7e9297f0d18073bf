// batch_kernels.hpp -- line passes over many independent grids in one launch.
//
// A launch runs one or more line passes of every grid of a batch (up to all
// three pair passes of a sub-step).  Its blocks take work items (table entry,
// block of that entry's pass) from a list in device memory; the pass
// arguments of each grid and pair come from a table in device memory.  The
// bodies are the single-grid ones of pass_kernels.hpp.
#pragma once
#include "pass_kernels.hpp"

namespace fdtd {

// Batched x lines: block b runs work item items[remap(b)] = (entry of tab,
// block of that entry's pass); one launch covers the passes of many grids.
template <typename T, typename S, int M, int MODE, bool MAT>
__global__ void __launch_bounds__(256) pass_x_batch_kernel(const PassArgs<T, S>* tab, const int2* items) {
    __shared__ CoefTab<S> ctab[MAT ? 256 : 1];
    const int2 it = items[xcd_remap(blockIdx.x, gridDim.x)];   // neighbouring items on one XCD
    const PassArgs<T, S> a = tab[it.x];
    if constexpr (MAT) load_coef_table<T, S, MODE>(ctab, a);
    pass_x_body<T, S, M, MODE, false, MAT>(a, it.y, ctab);
}

// Batched y/z lines: block b runs work item items[remap(b)] = (entry e of
// tab, item index q).  The block has blockDim.x = TX * Pmax threads; entry e
// has P <= Pmax chunks per line, so the block splits into floor(Pmax/P)
// sub-blocks of TX * P threads, which run the virtual blocks
// q * floor(Pmax/P) + sub of that entry; leftover threads idle.
template <typename T, typename S, int M, int MODE, int TX, int NT, bool MAT>
__device__ __forceinline__ void yz_batch_item(const PassArgs<T, S>& a, int q, const CoefTab<S>* ctab) {
    extern __shared__ unsigned char smem_raw[];
    const int sub_n = TX * a.P;
    const int spb = blockDim.x / sub_n;          // whole sub-blocks per block
    const int sub = threadIdx.x / sub_n;         // sub == spb: leftover threads (Pmax not a multiple of P)
    const bool partial = sub >= spb;
    const int vb = q * spb + (partial ? 0 : sub);
    // LDS holds ceil(Pmax / P) sub-block areas (the launch sizes it so), so the
    // leftover threads have an area of their own; they never store.
    constexpr int ROWS = (MODE == FUND_REF) ? 13 : 9;   // rows of P (TX + 1) per area
    S* sm = reinterpret_cast<S*>(smem_raw) + (size_t)sub * ROWS * a.P * (TX + 1);
    const bool valid = !partial && vb < a.nblk;
    pass_yz_body<T, S, M, MODE, TX, NT, false, MAT>(a, valid ? vb : 0, threadIdx.x - sub * sub_n, sm, ctab, valid);
}

template <typename T, typename S, int M, int MODE, int TX, int NT, bool MAT>
__global__ void __launch_bounds__(NT) pass_yz_batch_kernel(const PassArgs<T, S>* tab, const int2* items) {
    __shared__ CoefTab<S> ctab[MAT ? 256 : 1];
    const int2 it = items[xcd_remap(blockIdx.x, gridDim.x)];   // neighbouring tiles on one XCD
    const PassArgs<T, S> a = tab[it.x];
    if constexpr (MAT) load_coef_table<T, S, MODE>(ctab, a);
    yz_batch_item<T, S, M, MODE, TX, NT, MAT>(a, it.y, ctab);
}

// All pair passes of a sub-step in one launch.  Items whose entry is below ex0
// are y/z-line blocks as above; the others are x-line blocks of blockDim.x / 64
// waves (their table entries count blocks of that size).  The two kinds are
// interleaved in the work list, so every XCD's share holds both.
template <typename T, typename S, int MX, int M, int MODE, int TX, int NT, bool MAT>
__global__ void __launch_bounds__(NT) pass_sub_batch_kernel(const PassArgs<T, S>* tab, const int2* items, int ex0) {
    __shared__ CoefTab<S> ctab[MAT ? 256 : 1];
    const int2 it = items[xcd_remap(blockIdx.x, gridDim.x)];
    const PassArgs<T, S> a = tab[it.x];
    if constexpr (MAT) load_coef_table<T, S, MODE>(ctab, a);
    if (it.x < ex0) yz_batch_item<T, S, M, MODE, TX, NT, MAT>(a, it.y, ctab);
    else pass_x_body<T, S, MX, MODE, false, MAT>(a, it.y, ctab);
}

}  // namespace fdtd
