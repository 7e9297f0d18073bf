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
// One thread solves one line: an LDL^T sweep forward (the three multipliers
// of each row and the forward-substituted right side divided by its pivot go
// to a work area, one array per quantity, indexed [slot][line] so that the
// lanes of a wave store and load consecutive words), then the backward sweep
// forms V from the work area and writes the new E and H.  Lanes hold
// neighbouring lines, so for y and z lines every field access is coalesced;
// x lines read their rows with a stride between lanes.
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
    S* scr;               // work area: 4 arrays of n_w * nlines (l1, l2, l3, y)
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

// One fundamental pass of the fourth-order operator over the lines of `a`
// (FIN: the output form u = U_old + U_new, as the second-order FIN passes).
template <typename T, typename S, bool FIN>
__global__ void __launch_bounds__(128) pass4_kernel(Pass4Args<T, S> A) {
    const PassArgs<T, S>& a = A.p;
    const long long line = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (line >= A.nlines) return;
    const int ia = a.a_lo + int(line % a.na), ib = a.b_lo + int(line / a.na);
    const long long base = (long long)ia * a.sa + (long long)ib * a.sb;
    const long long sw = a.sw;
    const int n = a.n_w;   // cells along the line: unknowns 1 .. n-1, H samples 0 .. n-1
    T* E = a.Eout;
    T* H = a.Hout;
    const float* eps = a.eps;
    const long long NL = A.nlines;
    S* s1 = A.scr;
    S* s2 = s1 + (long long)n * NL;
    S* s3 = s2 + (long long)n * NL;
    S* sy = s3 + (long long)n * NL;
    const bool src_line = ia == a.src_a && ib == a.src_b;
    const S pre = src_line ? (a.src_pre_dev ? S(*a.src_pre_dev) : a.src_pre) : S(0);
    const S post = src_line ? (a.src_post_dev ? S(*a.src_post_dev) : a.src_post) : S(0);
    auto Hat = [&](int q) -> S {   // H sample q (0 .. n-1), even images across the walls
        q = q < 0 ? -1 - q : (q > n - 1 ? 2 * n - 1 - q : q);
        return S(H[base + q * sw]);
    };
    // ---- forward: LDL^T and forward substitution ----------------------------
    // window: H_{j-2}, H_{j-1}, H_j (H_{j+1} loaded per row); previous rows'
    // pivots D, forward-substituted z and multipliers
    S h0 = Hat(-1), h1 = Hat(0), h2 = Hat(1);
    S D1 = S(1), D2 = S(1), D3 = S(1);          // D_{j-1}, D_{j-2}, D_{j-3}
    S z1 = S(0), z2 = S(0), z3 = S(0);          // z_{j-1}, z_{j-2}, z_{j-3}
    S L11 = S(0), L12 = S(0), L21 = S(0);       // L_{j-1,j-2}, L_{j-1,j-3}, L_{j-2,j-3}
    for (int j = 1; j < n; ++j) {
        const S hn = Hat(j + 1);
        const S dhs = S(A.wi) * (h2 - h1) + S(A.wo) * (hn - h0);
        S hterm = dhs * a.kap_hi;
        if constexpr (sizeof(S) == 4) hterm = fused(dhs, a.kap_lo, hterm);
        S b[4];
        band_row4<T, S>(A, j, n, b);
        // diagonal sigma + (D^T D)_jj, and sigma taken back from it (exact),
        // so that the diagonal and the right side see one medium (as the
        // second-order FP32 passes do with 2 + sigma)
        const S dgj = b[0] + S(a.Ks * double(eps[base + j * sw]));
        const S sig = dgj - b[0];
        const S ue = S(E[base + j * sw]);
        const S r = S(2) * sig * (ue + ((src_line && j == a.src_j) ? pre : S(0))) + hterm;
        // L_{j,j-3}, L_{j,j-2}, L_{j,j-1}, D_j
        const S l3 = b[3] * recip(D3);
        const S l2 = (b[2] - l3 * L21 * D3) * recip(D2);
        const S l1 = (b[1] - l3 * L12 * D3 - l2 * L11 * D2) * recip(D1);
        const S Dj = dgj - (l3 * l3 * D3 + l2 * l2 * D2 + l1 * l1 * D1);
        const S zj = r - (l1 * z1 + l2 * z2 + l3 * z3);
        const long long o = (long long)j * NL + line;
        s1[o] = l1;
        s2[o] = l2;
        s3[o] = l3;
        sy[o] = zj * recip(Dj);
        // shift the windows
        D3 = D2; D2 = D1; D1 = Dj;
        z3 = z2; z2 = z1; z1 = zj;
        L21 = L11; L12 = l2; L11 = l1;
        h0 = h1; h1 = h2; h2 = hn;
    }
    // ---- backward: V, then the new E_j and H_{j+1} --------------------------
    // V_j = y_j - L_{j+1,j} V_{j+1} - L_{j+2,j} V_{j+2} - L_{j+3,j} V_{j+3}:
    // v1..v3 = V_{j+1..j+3} (0 past the last unknown), m11 = l1_{j+1},
    // m21, m22 = l2_{j+1}, l2_{j+2}, m31, m32, m33 = l3_{j+1}, l3_{j+2}, l3_{j+3}
    S v1 = S(0), v2 = S(0), v3 = S(0);
    S m11 = S(0), m21 = S(0), m22 = S(0), m31 = S(0), m32 = S(0), m33 = S(0);
    S vlast = S(0);   // V_{n-1}: its odd image is V_{n+1}
    // H sample hq: U_h += q (D V)_hq from V_{hq-1} .. V_{hq+2}
    auto store_h = [&](int hq, S vm1, S v0, S vp1, S vp2) {
        const S dv = S(A.wi) * (vp1 - v0) + S(A.wo) * (vp2 - vm1);
        const T old = H[base + hq * sw];
        const T nh = T(fused(a.q, dv, S(old)));
        H[base + hq * sw] = FIN ? T(double(nh) + double(old)) : nh;
    };
    for (int j = n - 1; j >= 1; --j) {
        const long long o = (long long)j * NL + line;
        const S l1 = s1[o], l2 = s2[o], l3 = s3[o], yj = sy[o];
        const S vj = yj - ((m11 * v1 + m22 * v2) + m33 * v3);
        if (j == n - 1) vlast = vj;
        // H_{j+1} (j + 1 <= n - 1): V_j .. V_{j+3}; V_n = 0 (wall, the window's
        // zero), V_{n+1} = -V_{n-1} (needed at j = n - 2)
        if (j + 1 <= n - 1) store_h(j + 1, vj, v1, v2, (j == n - 2) ? -vlast : v3);
        const bool at_src = src_line && j == a.src_j;
        const T old = E[base + j * sw];
        const T ne = T(vj - S(old) - (at_src ? post : S(0)));
        E[base + j * sw] = FIN ? T(double(ne) + double(old) + (at_src ? a.fsrc : 0.0)) : ne;
        m33 = m32; m32 = m31; m31 = l3;
        m22 = m21; m21 = l2;
        m11 = l1;
        v3 = v2; v2 = v1; v1 = vj;
    }
    // here v1..v3 = V_1..V_3 (0 at or past the wall, except the image V_{n+1})
    store_h(1, S(0), v1, v2, (n == 2) ? -vlast : v3);   // H_1: V_0 .. V_3
    store_h(0, -v1, S(0), v1, v2);                      // H_0: V_-1 = -V_1 .. V_2
}

// x lines (the contiguous axis): the same sweeps, with the fields staged
// through LDS so that HBM sees whole rows.  A block is one wave holding 64
// consecutive lines; tiles of X4_TS slots of all 64 rows are loaded row by
// row (64 / X4_TS rows per wave instruction, X4_TS contiguous words each), each lane
// then runs its own line's recurrences from LDS, and the backward sweep writes
// its results into the tile, which is stored row by row.  The H tile of the
// E slots [t0, t0 + X4_TS) covers H samples t0 + 1 .. t0 + X4_TS: the sample
// that E_j's row completes in the backward sweep is H_{j+1}.
constexpr int X4_TS = 8;

template <typename T, typename S, bool FIN>
__global__ void __launch_bounds__(64) pass4_x_kernel(Pass4Args<T, S> A) {
    const PassArgs<T, S>& a = A.p;
    constexpr int TS = X4_TS, LD = X4_TS + 1;
    __shared__ T tE[64 * LD];
    __shared__ T tH[64 * LD];
    __shared__ float tP[64 * LD];
    const int lane = threadIdx.x;
    const long long L0 = (long long)blockIdx.x * 64;
    const long long line = L0 + lane;
    const bool live = line < A.nlines;
    const int n = a.n_w;
    T* E = a.Eout;
    T* H = a.Hout;
    auto base_of = [&](long long ln) -> long long {
        const int ia = a.a_lo + int(ln % a.na), ib = a.b_lo + int(ln / a.na);
        return (long long)ia * a.sa + (long long)ib * a.sb;
    };
    const long long base = live ? base_of(line) : 0;
    const int ia = a.a_lo + int(line % a.na), ib = a.b_lo + int(line / a.na);
    const bool src_line = live && ia == a.src_a && ib == a.src_b;
    const S pre = src_line ? (a.src_pre_dev ? S(*a.src_pre_dev) : a.src_pre) : S(0);
    const S post = src_line ? (a.src_post_dev ? S(*a.src_post_dev) : a.src_post) : S(0);
    const long long NL = A.nlines;
    S* s1 = A.scr;
    S* s2 = s1 + (long long)n * NL;
    S* s3 = s2 + (long long)n * NL;
    S* sy = s3 + (long long)n * NL;
    // tile transfer: 64 / TS rows per wave instruction, rows r = m (64 / TS) +
    // lane / TS, slot t0 + lane % TS of E and eps, t0 + 1 + lane % TS of H;
    // `store` writes E slots [elo, ehi] and H samples [hlo, hhi] back
    constexpr int RPI = 64 / TS;
    const int half = lane / TS, col = lane % TS;
    auto load_tile = [&](int t0, bool with_eps) {
        for (int m = 0; m < TS; ++m) {
            const int r = RPI * m + half;
            const long long ln = L0 + r;
            if (ln >= NL) continue;
            const long long b = base_of(ln);
            const int je = t0 + col, jh = t0 + 1 + col;
            if (je <= n) {
                tE[r * LD + col] = E[b + je];
                if (with_eps) tP[r * LD + col] = a.eps[b + je];
            }
            if (jh <= n - 1) tH[r * LD + col] = H[b + jh];
        }
        __syncthreads();
    };
    auto store_tile = [&](int t0, int elo, int ehi, int hlo, int hhi) {
        __syncthreads();
        for (int m = 0; m < TS; ++m) {
            const int r = RPI * m + half;
            const long long ln = L0 + r;
            if (ln >= NL) continue;
            const long long b = base_of(ln);
            const int je = t0 + col, jh = t0 + 1 + col;
            if (je >= elo && je <= ehi) E[b + je] = tE[r * LD + col];
            if (jh >= hlo && jh <= hhi) H[b + jh] = tH[r * LD + col];
        }
        __syncthreads();
    };
    const int ntiles = (n + TS - 1) / TS;   // tiles of E slots 0 .. n-1
    // ---- forward ------------------------------------------------------------
    const S H0 = live ? S(H[base]) : S(0);
    S h0 = H0, h1 = H0, h2 = S(0);
    S D1 = S(1), D2 = S(1), D3 = S(1);
    S z1 = S(0), z2 = S(0), z3 = S(0);
    S L11 = S(0), L12 = S(0), L21 = S(0);
    for (int tt = 0; tt < ntiles; ++tt) {
        const int t0 = tt * TS;
        load_tile(t0, true);
        if (tt == 0) h2 = S(tH[lane * LD + 0]);   // H_1 (n >= 2)
        const int jlo = t0 < 1 ? 1 : t0, jhi = (t0 + TS - 1 < n - 1) ? t0 + TS - 1 : n - 1;
        if (live) {
            for (int j = jlo; j <= jhi; ++j) {
                const int c = j - t0;
                const S hn = (j + 1 <= n - 1) ? S(tH[lane * LD + c]) : h2;   // H_{j+1}; image H_{n-1}
                const S dhs = S(A.wi) * (h2 - h1) + S(A.wo) * (hn - h0);
                S hterm = dhs * a.kap_hi;
                if constexpr (sizeof(S) == 4) hterm = fused(dhs, a.kap_lo, hterm);
                S b[4];
                band_row4<T, S>(A, j, n, b);
                const S dgj = b[0] + S(a.Ks * double(tP[lane * LD + c]));
                const S sig = dgj - b[0];
                const S ue = S(tE[lane * LD + c]);
                const S r = S(2) * sig * (ue + ((src_line && j == a.src_j) ? pre : S(0))) + hterm;
                const S l3 = b[3] * recip(D3);
                const S l2 = (b[2] - l3 * L21 * D3) * recip(D2);
                const S l1 = (b[1] - l3 * L12 * D3 - l2 * L11 * D2) * recip(D1);
                const S Dj = dgj - (l3 * l3 * D3 + l2 * l2 * D2 + l1 * l1 * D1);
                const S zj = r - (l1 * z1 + l2 * z2 + l3 * z3);
                const long long o = (long long)j * NL + line;
                s1[o] = l1;
                s2[o] = l2;
                s3[o] = l3;
                sy[o] = zj * recip(Dj);
                D3 = D2; D2 = D1; D1 = Dj;
                z3 = z2; z2 = z1; z1 = zj;
                L21 = L11; L12 = l2; L11 = l1;
                h0 = h1; h1 = h2; h2 = hn;
            }
        }
        __syncthreads();
    }
    // ---- backward -----------------------------------------------------------
    S v1 = S(0), v2 = S(0), v3 = S(0);
    S m11 = S(0), m21 = S(0), m22 = S(0), m31 = S(0), m32 = S(0), m33 = S(0);
    S vlast = S(0);
    auto new_h = [&](S old, S vm1, S v0, S vp1, S vp2) -> T {
        const S dv = S(A.wi) * (vp1 - v0) + S(A.wo) * (vp2 - vm1);
        const T nh = T(fused(a.q, dv, old));
        return FIN ? T(double(nh) + double(T(old))) : nh;
    };
    for (int tt = ntiles - 1; tt >= 0; --tt) {
        const int t0 = tt * TS;
        load_tile(t0, false);
        const int jlo = t0 < 1 ? 1 : t0, jhi = (t0 + TS - 1 < n - 1) ? t0 + TS - 1 : n - 1;
        if (live) {
            for (int j = jhi; j >= jlo; --j) {
                const int c = j - t0;
                const long long o = (long long)j * NL + line;
                const S l1 = s1[o], l2 = s2[o], l3 = s3[o], yj = sy[o];
                const S vj = yj - ((m11 * v1 + m22 * v2) + m33 * v3);
                if (j == n - 1) vlast = vj;
                if (j + 1 <= n - 1)
                    tH[lane * LD + c] = new_h(S(tH[lane * LD + c]), vj, v1, v2, (j == n - 2) ? -vlast : v3);
                const bool at_src = src_line && j == a.src_j;
                const T old = tE[lane * LD + c];
                const T ne = T(vj - S(old) - (at_src ? post : S(0)));
                tE[lane * LD + c] = FIN ? T(double(ne) + double(old) + (at_src ? a.fsrc : 0.0)) : ne;
                m33 = m32; m32 = m31; m31 = l3;
                m22 = m21; m21 = l2;
                m11 = l1;
                v3 = v2; v2 = v1; v1 = vj;
            }
            if (tt == 0) {
                // H_1 (tile column 0) from V_0 = 0 .. V_3
                tH[lane * LD + 0] = new_h(S(tH[lane * LD + 0]), S(0), v1, v2, (n == 2) ? -vlast : v3);
            }
        }
        // E slots [jlo, jhi]; H samples t0+1 .. t0+TS below n (H_1 only in the lowest tile, done above)
        store_tile(t0, jlo, jhi, t0 + 1, (t0 + TS < n - 1) ? t0 + TS : n - 1);
    }
    if (live) H[base] = new_h(H0, -v1, S(0), v1, v2);   // H_0: V_-1 = -V_1 .. V_2
}

}  // namespace fdtd
