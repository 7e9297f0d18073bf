// batch_kernels.hpp -- line passes over many independent grids in one launch.
//
// A launch runs one line pass of every grid of a batch.  Its blocks take work
// items (grid, block of that grid's pass) from a list in device memory; the
// pass arguments of each grid come from a table in device memory.  The bodies
// are the single-grid ones of pass_kernels.hpp.
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
__global__ void __launch_bounds__(NT) pass_yz_batch_kernel(const PassArgs<T, S>* tab, const int2* items) {
    __shared__ CoefTab<S> ctab[MAT ? 256 : 1];
    extern __shared__ unsigned char smem_raw[];
    const int2 it = items[xcd_remap(blockIdx.x, gridDim.x)];   // neighbouring tiles on one XCD
    const PassArgs<T, S> a = tab[it.x];
    if constexpr (MAT) load_coef_table<T, S, MODE>(ctab, a);
    const int sub_n = TX * a.P;
    const int spb = blockDim.x / sub_n;          // whole sub-blocks per block
    const int sub = threadIdx.x / sub_n;         // sub == spb: leftover threads (Pmax not a multiple of P)
    const bool partial = sub >= spb;
    const int vb = it.y * spb + (partial ? 0 : sub);
    // LDS holds ceil(Pmax / P) sub-block areas (the launch sizes it so), so the
    // leftover threads have an area of their own; they never store.
    constexpr int ROWS = (MODE == FUND_REF) ? 13 : 9;   // rows of P (TX + 1) per area
    S* sm = reinterpret_cast<S*>(smem_raw) + (size_t)sub * ROWS * a.P * (TX + 1);
    const bool valid = !partial && vb < a.nblk;
    pass_yz_body<T, S, M, MODE, TX, NT, false, MAT>(a, valid ? vb : 0, threadIdx.x - sub * sub_n, sm, ctab, valid);
}

}  // namespace fdtd
