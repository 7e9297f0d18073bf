// order4_kernels.hpp -- line passes with fourth-order staggered differences.
//
// The closing remark of Sec. III-A leaves the difference operators of the
// updating equations open (higher order, optimized, compact).  With a 4-point
// staggered first difference
//     d_w f = [wi (f[+1/2] - f[-1/2]) + wo (f[+3/2] - f[-3/2])] / dw,
// wi = 1 - 3 wo (fourth order: wo = -1/24, wi = 27/24; a parameter-optimized
// operator takes another outer weight wo),
// in both the implicit line equation and the explicit H update, the
// fundamental pass of a pair (E, H) along w keeps its form:
//   r_j  = 2 sigma_j (U_e,j + pre) + kap (D U_h)_j
//   solve (diag(sigma) + D^T D) V = r        (symmetric, positive definite)
//   U_h  += q (D V)                           (H samples j + 1/2)
//   U_e   = V - U_e - post
// with D the dimensionless 4-point difference (weights -wo, -wi, wi, wo)
// folded onto image samples across the PEC walls (tangential E odd, H even),
// so that D^T is minus the H-to-E difference and the sub-step stays an exact
// Cayley factor.  The system couples each unknown to three neighbours on
// either side (band 3).
//
// One thread solves one line: an LDL^T sweep forward, then a backward sweep
// that forms V and writes the new E and H.  The forward sweep stores, per
// row, only the forward-substituted right side divided by its pivot (y), and
// at the start of every segment of K rows the recurrence state of the
// factorization (the last three pivots and the three multipliers of the
// previous two rows that the next row needs: six words); the backward sweep
// takes each segment's state, factors its K rows
// again into registers (the factors depend on the medium only) and then runs
// the back substitution over them.  So the work area takes 1 + 6/K words per
// slot instead of the four (three multipliers and y) a stored factorization
// needs.  With FP32 solves both sweeps issue a segment's loads together
// before its rows run (the recurrences are serial, so a lane would otherwise
// wait on memory once per row); FP64 solves load per row (a segment's values
// in registers would cost occupancy).  K = 8.  Work-area
// arrays are indexed [slot][line] so that the lanes of a wave store and load
// consecutive words.
// With a material index the medium term Ks eps_r comes from a per-material
// table in LDS (one byte per slot read, the same values as from eps_r).
// Lanes hold neighbouring lines, so every field access is coalesced (x lines
// on a transposed copy, below).
//
// Rows near the walls (the first and last three unknowns) have the folded
// coefficients, computed on the host per line length; the other rows have
// the interior band {2 wi^2 + 2 wo^2, 2 wi wo - wi^2, -2 wi wo, -wo^2}
// ((1460, -783, 54, -1) / 576 for the fourth-order weights).
#pragma once
#include <hip/hip_runtime.h>

#include "line_solver.hpp"   // recip
#include "pass_kernels.hpp"  // PassArgs (line geometry, coefficients, source)

namespace fdtd {

template <typename T, typename S>
struct Pass4Args {
    PassArgs<T, S> p;     // pair arrays (Ein == Eout, Hin == Hout), line geometry, coefficients, source
    S* scr;               // work area: y (n_w * nlines), then the recurrence state at each segment
                          // start (nseg * 6 * nlines, nseg = segments of the kernel's length)
    long long nlines;
    // band of rows 1..3 (lo) and n-3..n-1 (hi): {A_jj, A_j,j-1, A_j,j-2, A_j,j-3}
    double blo[3][4], bhi[3][4];
    double bin[4];        // band of the other rows
    double wi, wo;        // inner and outer weights of the difference
};

// Entries of row j (1 <= j <= n-1) of D^T D: {A_jj, A_j,j-1, A_j,j-2, A_j,j-3}.
template <typename T, typename S>
__device__ __forceinline__ void band_row4(const Pass4Args<T, S>& a, int j, int n, S (&b)[4]) {
    if (j <= 3) {
#pragma unroll
        for (int t = 0; t < 4; ++t) b[t] = S(a.blo[j - 1][t]);
    } else if (j >= n - 3) {
#pragma unroll
        for (int t = 0; t < 4; ++t) b[t] = S(a.bhi[j - (n - 3)][t]);
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) b[t] = S(a.bin[t]);
    }
}

// Recurrence state of the LDL^T factorization at a row: D_{j-1}, D_{j-2},
// D_{j-3} and L_{j-1,j-2}, L_{j-1,j-3}, L_{j-2,j-3}.
template <typename S>
struct Ldl4 {
    S D1, D2, D3, L11, L12, L21;
};

template <typename S>
__device__ __forceinline__ Ldl4<S> ldl4_start() {
    return Ldl4<S>{S(1), S(1), S(1), S(0), S(0), S(0)};
}

// Row j of the factorization (band b, diagonal dgj): multipliers L_{j,j-1},
// L_{j,j-2}, L_{j,j-3}, pivot D_j; advances the state to row j + 1.  The
// forward and the backward sweep both call this, so they get the same factors.
template <typename S>
__device__ __forceinline__ void ldl4_row(Ldl4<S>& f, const S (&b)[4], S dgj, S& l1, S& l2, S& l3, S& Dj) {
    l3 = b[3] * recip(f.D3);
    l2 = (b[2] - l3 * f.L21 * f.D3) * recip(f.D2);
    l1 = (b[1] - l3 * f.L12 * f.D3 - l2 * f.L11 * f.D2) * recip(f.D1);
    Dj = dgj - (l3 * l3 * f.D3 + l2 * l2 * f.D2 + l1 * l1 * f.D1);
    f.D3 = f.D2;
    f.D2 = f.D1;
    f.D1 = Dj;
    f.L21 = f.L11;
    f.L12 = l2;
    f.L11 = l1;
}

// State of segment s of a line in the work area (6 arrays of nlines words).
template <typename S>
__device__ __forceinline__ void ldl4_save(S* ck, long long NL, long long line, const Ldl4<S>& f) {
    ck[line] = f.D1;
    ck[NL + line] = f.D2;
    ck[2 * NL + line] = f.D3;
    ck[3 * NL + line] = f.L11;
    ck[4 * NL + line] = f.L12;
    ck[5 * NL + line] = f.L21;
}
template <typename S>
__device__ __forceinline__ Ldl4<S> ldl4_load(const S* ck, long long NL, long long line) {
    return Ldl4<S>{ck[line], ck[NL + line], ck[2 * NL + line], ck[3 * NL + line], ck[4 * NL + line],
                   ck[5 * NL + line]};
}

// Ks eps_r of each material (LDS), when the plan has a material index.
template <typename T, typename S>
__device__ __forceinline__ void load_ks_table(S* ktab, const PassArgs<T, S>& a) {
    if (!a.mat) return;
    for (int m = int(threadIdx.x); m < 256; m += int(blockDim.x))
        ktab[m] = S(a.Ks * double(m < a.nmat ? a.mat_eps[m] : 1.0f));
    __syncthreads();
}

// Segment length of the kernel (factors of a segment held in registers).
template <typename S>
__host__ __device__ constexpr int seg4() { return 8; }

// Work-area words of one pass over nlines lines of n cells: y (n per line)
// and the factorization state (6 words) at the start of each segment of K
// rows (rows 1 .. n-1).  The kernel's indexing and the host's allocation both
// use this.
__host__ __device__ constexpr long long work4_words(int n, long long nlines, int K) {
    return ((long long)n + 6LL * ((n - 1 + K - 1) / K)) * nlines;
}

// Pointer type of the pass kernel's arrays: restrict-qualified (R) or plain.
template <typename V, bool R> struct Ptr4 { using type = V* __restrict__; };
template <typename V> struct Ptr4<V, false> { using type = V*; };

// One fundamental pass of the fourth-order operator over the lines of `a`
// (FIN: the output form u = U_old + U_new, as the second-order FIN passes).
template <typename T, typename S, bool FIN>
__global__ void __launch_bounds__(128) pass4_kernel(Pass4Args<T, S> A) {
    constexpr int K = seg4<S>();
    // FP32 solves: a segment's loads are issued together before its rows run,
    // so a lane waits for memory once per segment rather than once per row.
    // FP64 solves load per row, from plain pointers that keep each load at
    // its row: a segment's values in registers cost more in occupancy than
    // the waits (a 512^3 y/z pass: 2.60 ms batched with K = 4, 2.22 ms per
    // row with K = 8).  Both forms compute the same rows in the same order.
    constexpr bool kBatch = sizeof(S) == 4;
    using TP = typename Ptr4<T, kBatch>::type;
    using SP = typename Ptr4<S, kBatch>::type;
    const PassArgs<T, S>& a = A.p;
    __shared__ S ktab[256];
    load_ks_table<T, S>(ktab, a);
    const long long line = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (line >= A.nlines) return;
    const int ia = a.a_lo + int(line % a.na), ib = a.b_lo + int(line / a.na);
    const long long base = (long long)ia * a.sa + (long long)ib * a.sb;
    const long long sw = a.sw;
    const int n = a.n_w;   // cells along the line: unknowns 1 .. n-1, H samples 0 .. n-1
    TP E = a.Eout;
    TP H = a.Hout;
    const long long NL = A.nlines;
    SP sy = A.scr;
    SP ck = sy + (long long)n * NL;
    const bool src_line = ia == a.src_a && ib == a.src_b;
    const S pre = src_line ? (a.src_pre_dev ? S(*a.src_pre_dev) : a.src_pre) : S(0);
    const S post = src_line ? (a.src_post_dev ? S(*a.src_post_dev) : a.src_post) : S(0);
    auto Hat = [&](int q) -> S {   // H sample q (0 .. n-1), even images across the walls
        q = q < 0 ? -1 - q : (q > n - 1 ? 2 * n - 1 - q : q);
        return S(H[base + q * sw]);
    };
    auto kes = [&](int j) -> S {   // Ks eps_r at unknown j
        const long long o = base + j * sw;
        return a.mat ? ktab[a.mat[o]] : S(a.Ks * double(a.eps[o]));
    };
    const int nseg = (n - 1 + K - 1) / K;   // segments of K rows from row 1
    // ---- forward: LDL^T and forward substitution ----------------------------
    // window: H_{j-2}, H_{j-1}, H_j; forward-substituted z of the previous
    // three rows
    S h0 = Hat(-1), h1 = Hat(0), h2 = Hat(1);
    Ldl4<S> f = ldl4_start<S>();
    S z1 = S(0), z2 = S(0), z3 = S(0);
    for (int s = 0; s < nseg; ++s) {
        const int j0 = 1 + s * K;
        S ev[K], hv[K], mv[K];
        if constexpr (kBatch) {
#pragma unroll
            for (int t = 0; t < K; ++t) {
                const int j = j0 + t;
                if (j < n) {
                    ev[t] = S(E[base + j * sw]);
                    hv[t] = Hat(j + 1);
                    mv[t] = kes(j);
                }
            }
        }
        ldl4_save(ck + (long long)s * 6 * NL, NL, line, f);
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const int j = j0 + t;
            if (j >= n) continue;
            if constexpr (!kBatch) {
                ev[t] = S(E[base + j * sw]);
                hv[t] = Hat(j + 1);
                mv[t] = kes(j);
            }
            const S hn = hv[t];
            const S dhs = S(A.wi) * (h2 - h1) + S(A.wo) * (hn - h0);
            S hterm = dhs * a.kap_hi;
            if constexpr (sizeof(S) == 4) hterm = fused(dhs, a.kap_lo, hterm);
            S b[4];
            band_row4<T, S>(A, j, n, b);
            // diagonal sigma + (D^T D)_jj, and sigma taken back from it
            // (exact), so that the diagonal and the right side see one medium
            // (as the second-order FP32 passes do with 2 + sigma)
            const S dgj = b[0] + mv[t];
            const S sig = dgj - b[0];
            const S r = S(2) * sig * (ev[t] + ((src_line && j == a.src_j) ? pre : S(0))) + hterm;
            S l1, l2, l3, Dj;
            ldl4_row(f, b, dgj, l1, l2, l3, Dj);
            const S zj = r - (l1 * z1 + l2 * z2 + l3 * z3);
            sy[(long long)j * NL + line] = zj * recip(Dj);
            z3 = z2; z2 = z1; z1 = zj;
            h0 = h1; h1 = h2; h2 = hn;
        }
    }
    // ---- backward: V, then the new E_j and H_{j+1} --------------------------
    // V_j = y_j - L_{j+1,j} V_{j+1} - L_{j+2,j} V_{j+2} - L_{j+3,j} V_{j+3}:
    // v1..v3 = V_{j+1..j+3} (0 past the last unknown), m11 = l1_{j+1},
    // m21, m22 = l2_{j+1}, l2_{j+2}, m31, m32, m33 = l3_{j+1}, l3_{j+2}, l3_{j+3}
    S v1 = S(0), v2 = S(0), v3 = S(0);
    S m11 = S(0), m21 = S(0), m22 = S(0), m31 = S(0), m32 = S(0), m33 = S(0);
    S vlast = S(0);   // V_{n-1}: its odd image is V_{n+1}
    // new H sample from its old value and V_{hq-1} .. V_{hq+2}: U_h += q (D V)
    auto new_h = [&](T old, S vm1, S v0, S vp1, S vp2) -> T {
        const S dv = S(A.wi) * (vp1 - v0) + S(A.wo) * (vp2 - vm1);
        const T nh = T(fused(a.q, dv, S(old)));
        return FIN ? T(double(nh) + double(old)) : nh;
    };
    for (int s = nseg - 1; s >= 0; --s) {
        const int j0 = 1 + s * K;
        // (FP32) the segment's loads, then its factors again from its saved
        // state
        Ldl4<S> g = ldl4_load(ck + (long long)s * 6 * NL, NL, line);
        S yv[K], mv[K], f1[K], f2[K], f3[K];
        T ev[K], hv[K];
        if constexpr (kBatch) {
#pragma unroll
            for (int t = 0; t < K; ++t) {
                const int j = j0 + t;
                if (j < n) {
                    yv[t] = sy[(long long)j * NL + line];
                    ev[t] = E[base + j * sw];
                    if (j + 1 <= n - 1) hv[t] = H[base + (j + 1) * sw];
                    mv[t] = kes(j);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const int j = j0 + t;
            if (j < n) {
                if constexpr (!kBatch) mv[t] = kes(j);
                S b[4];
                band_row4<T, S>(A, j, n, b);
                S Dj;
                ldl4_row(g, b, b[0] + mv[t], f1[t], f2[t], f3[t], Dj);
            }
        }
#pragma unroll
        for (int t = K - 1; t >= 0; --t) {
            const int j = j0 + t;
            if (j >= n) continue;
            if constexpr (!kBatch) {
                yv[t] = sy[(long long)j * NL + line];
                ev[t] = E[base + j * sw];
                if (j + 1 <= n - 1) hv[t] = H[base + (j + 1) * sw];
            }
            const S vj = yv[t] - ((m11 * v1 + m22 * v2) + m33 * v3);
            if (j == n - 1) vlast = vj;
            // H_{j+1} (j + 1 <= n - 1): V_j .. V_{j+3}; V_n = 0 (wall, the window's
            // zero), V_{n+1} = -V_{n-1} (needed at j = n - 2)
            if (j + 1 <= n - 1) H[base + (j + 1) * sw] = new_h(hv[t], vj, v1, v2, (j == n - 2) ? -vlast : v3);
            const bool at_src = src_line && j == a.src_j;
            const T old = ev[t];
            const T ne = T(vj - S(old) - (at_src ? post : S(0)));
            E[base + j * sw] = FIN ? T(double(ne) + double(old) + (at_src ? a.fsrc : 0.0)) : ne;
            m33 = m32; m32 = m31; m31 = f3[t];
            m22 = m21; m21 = f2[t];
            m11 = f1[t];
            v3 = v2; v2 = v1; v1 = vj;
        }
    }
    // here v1..v3 = V_1..V_3 (0 at or past the wall, except the image V_{n+1})
    H[base + sw] = new_h(H[base + sw], S(0), v1, v2, (n == 2) ? -vlast : v3);   // H_1: V_0 .. V_3
    H[base] = new_h(H[base], -v1, S(0), v1, v2);                                // H_0: V_-1 = -V_1 .. V_2
}

// x lines (the contiguous axis) run through the same kernel on a transposed
// copy of their pair: with x the slow axis inside each z plane, a line's
// slots lie a row pitch apart and neighbouring lanes (consecutive y) read
// consecutive words, as on the y and z lines.  The copy is made before the
// pass and moved back after it (transpose_planes_kernel); the medium's copy
// is made once per plan.  One-thread-per-line sweeps straight over x rows
// would read each 128-byte line piecemeal, many lanes apart in time.
//
// dst[p][c][r] = src[p][r][c] for r < R, c < C and every plane p: rows of
// src are columns of dst.  Square tiles through LDS, 256 threads: every wave
// load reads consecutive elements of a src row, every wave store writes
// consecutive elements of a dst row.  Tiles of 64 for 1- and 4-byte elements,
// 32 for 8-byte ones (a 64-tile of doubles takes 33 KB of LDS per block,
// which measured slower).  Whole tiles of 4-byte elements move 16 bytes per
// access (rows and planes of both layouts are multiples of 16 bytes, tile
// corners multiples of the tile): 236 against 276 us per 512^3 array; tiles at
// the edges of a plane and other element sizes move one element per access
// (for doubles, 16-byte accesses measured 430 against 408 us).
template <typename V>
__host__ __device__ constexpr int tr_tile() { return sizeof(V) == 8 ? 32 : 64; }

template <typename V>
struct Vec16 {   // 16-byte vector of 4-byte V
    using type = float4;
    static constexpr int n = 4;
};

template <typename V>
__global__ void __launch_bounds__(256) transpose_planes_kernel(const V* __restrict__ src, long long sp,
                                                               long long srow, V* __restrict__ dst, long long dp,
                                                               long long drow, int R, int C) {
    constexpr int TT = tr_tile<V>(), RS = 256 / TT;   // RS rows per pass of the block
    __shared__ V tile[TT][TT + 1];
    const int c0 = int(blockIdx.x) * TT, r0 = int(blockIdx.y) * TT;
    const long long pl = blockIdx.z;
    const V* s = src + pl * sp;
    V* d = dst + pl * dp;
    if constexpr (sizeof(V) == 4) {
        if (r0 + TT <= R && c0 + TT <= C) {
            using W = typename Vec16<V>::type;
            constexpr int VN = Vec16<V>::n, VR = TT / VN, VS = 256 / VR;   // vectors per row, rows per pass
            const int vc = int(threadIdx.x) % VR, vr = int(threadIdx.x) / VR;
#pragma unroll
            for (int m = 0; m < TT; m += VS) {
                const W w = *reinterpret_cast<const W*>(s + (long long)(r0 + vr + m) * srow + c0 + vc * VN);
                const V* e = reinterpret_cast<const V*>(&w);
#pragma unroll
                for (int q = 0; q < VN; ++q) tile[vr + m][vc * VN + q] = e[q];
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < TT; m += VS) {
                W w;
                V* e = reinterpret_cast<V*>(&w);
#pragma unroll
                for (int q = 0; q < VN; ++q) e[q] = tile[vc * VN + q][vr + m];
                *reinterpret_cast<W*>(d + (long long)(c0 + vr + m) * drow + r0 + vc * VN) = w;
            }
            return;
        }
    }
    const int tx = int(threadIdx.x) % TT, ty = int(threadIdx.x) / TT;
#pragma unroll
    for (int m = 0; m < TT; m += RS) {
        const int r = r0 + ty + m, c = c0 + tx;
        if (r < R && c < C) tile[ty + m][tx] = s[(long long)r * srow + c];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < TT; m += RS) {
        const int c = c0 + ty + m, r = r0 + tx;
        if (r < R && c < C) d[(long long)c * drow + r] = tile[tx][ty + m];
    }
}

// Grid of transpose_planes_kernel<V> over planes of R x C.
template <typename V>
static dim3 transpose_grid(int R, int C, int planes) {
    constexpr int TT = tr_tile<V>();
    return dim3((unsigned)((C + TT - 1) / TT), (unsigned)((R + TT - 1) / TT), (unsigned)planes);
}

}  // namespace fdtd
