// pass_kernels.hpp -- the fused line pass ("pair pass") kernels.
//
// One pass updates one (E, H) pair of operator X along its axis w (eq. (AMat)):
//   A: (Ex,Hz) y, (Ey,Hx) z, (Ez,Hy) x;   B: (Ex,Hy) z, (Ey,Hz) x, (Ez,Hx) y.
// Along every grid line of w the E samples sit at integer positions j (PEC
// walls at j = 0 and j = n), the H samples at j + 1/2 (stored at j).
//
// Mode FUND (the fundamental update of Sec. III, in the link scaling of
// Sec. II-E, U = auxiliary of the LOD1 iteration):
//   r_j  = 2 sigma_j (U_e,j + pre) + kap (U_h,j - U_h,j-1)
//   solve -V_{j-1} + (2 + sigma_j) V_j - V_{j+1} = r_j
//   U_h,j += q (V_{j+1} - V_j)                      (fasterADIbbh/ddh, fastestLOD2ex)
//   U_e,j  = V_j - U_e,j - post                     (fasterADIcc, fastLOD2.bbE)
// with sigma_j = eps_j mu dw^2 / theta^2, kap = 2 s mu dw / theta, q = s theta/(mu dw):
// this is 1/2 V - (b d / 2) d_w^2 V = U_e + s b d_w U_h multiplied by 2 sigma.
//
// Mode CONV_LOD (original LOD/SS formulae (orgLOD), (orgSS2), (orgLOD2)):
//   (1 - b d d_w^2) E' = E + 2 s b d_w H + b d d_w^2 E,  H' = H + s d d_w (E + E')
// multiplied by sigma.
//
// Mode CONV_ADI (original ADI (clsADI)): as CONV_LOD with the cross terms of
// the explicit operator Y != X:
//   (1 - b d d_w^2) E' = E + s b d_w H + s2 b d_t H2 + s s3 b d d_w d_e E3,
//   H' = H + s3 d d_e E3 + s d d_w E',
// read from the previous state and written to the other buffer set.  With
// H* = H + s3 d d_e E3 the right side is E + s b d_w H* + s2 b d_t H2, so the
// kernel forms H* once per H sample and uses it in both equations.
#pragma once
#include <hip/hip_runtime.h>
#include "line_solver.hpp"

namespace fdtd {

enum Mode { FUND = 0, CONV_LOD = 1, CONV_ADI = 2 };

template <typename T, typename S>
struct PassArgs {
    const T* Ein;
    const T* Hin;
    T* Eout;
    T* Hout;
    const T* H2;          // CONV_ADI: H component of Y's E row (shifted along t)
    const T* E3;          // CONV_ADI: E component of Y's H row (shifted along e)
    const float* eps;     // relative permittivity at node index (node layout)
    long long sw;         // stride along the line
    long long sa, sb;     // strides of the transverse line indices a, b
    long long s_t, s_e;   // CONV_ADI: strides along t and e
    int n_w;              // slots per line: 0 .. n_w-1 (slot 0 = wall)
    int a_lo, na, b_lo, nb;
    int P;                // chunks per line (power of two <= 64)
    double Ks;            // sigma = Ks * eps_r
    S kap_hi, kap_lo;     // coefficient of the H difference (double-float if S = float)
    S q;                  // H update coefficient
    S cH2, hE3;           // CONV_ADI cross-term coefficients
    long long src;        // offset of the source sample in E (or -1)
    S src_pre, src_post;
};

template <int MODE> struct ModeCE { static constexpr int v = (MODE == FUND) ? -1 : 0; };
template <int MODE> struct ModeCH { static constexpr int v = (MODE == CONV_LOD) ? 1 : 0; };

template <typename S> __device__ __forceinline__ S make_sigma(double Ks, float eps) {
    return S(Ks * double(eps));
}

// Right side and diagonal of one slot.  ue_m/ue_p: U_e at j-1, j+1 (CONV_LOD);
// uh_m: U_h at j-1; x2: CONV_ADI cross contribution (already scaled).
template <typename T, typename S, int MODE>
__device__ __forceinline__ void slot_rhs(const PassArgs<T, S>& a, bool dirichlet, bool is_src, float eps,
                                         S ue, S uh, S uh_m, S ue_m, S ue_p, S x2, S& dg, S& r) {
    if (dirichlet) {
        dg = Big<S>::v;
        r = S(0);
        return;
    }
    const S sig = make_sigma<S>(a.Ks, eps);
    dg = S(2) + sig;
    const S dh = uh - uh_m;
    const S hterm = dh * a.kap_hi + dh * a.kap_lo;
    const S e0 = is_src ? ue + a.src_pre : ue;
    if constexpr (MODE == FUND) {
        r = S(2) * sig * e0 + hterm;
    } else if constexpr (MODE == CONV_LOD) {
        r = sig * e0 + hterm + ((ue_p + ue_m) - S(2) * ue);
    } else {
        r = sig * e0 + hterm + x2;
    }
}

// ----------------------------------------------------------------------------
// x lines: contiguous axis.  One line per segment of P lanes of a wave; lane
// `ls` owns slots [ls*M, ls*M+M).  Rows are 128-byte aligned, so chunks are
// loaded with 16-byte vector loads.  The separator system is solved with
// cross-lane PCR (no LDS, no barrier).
// ----------------------------------------------------------------------------
template <typename T, int M>
__device__ __forceinline__ void load_row_chunk(const T* p, int j0, int lim, T (&v)[M]) {
    if (j0 + M <= lim) {
        constexpr int V = 16 / sizeof(T);
        static_assert(M % V == 0, "chunk must be a multiple of 16 bytes");
        using V16 = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
        const V16* q = reinterpret_cast<const V16*>(p + j0);
#pragma unroll
        for (int b = 0; b < M / V; ++b) {
            V16 x = q[b];
            const T* xs = reinterpret_cast<const T*>(&x);
#pragma unroll
            for (int e = 0; e < V; ++e) v[b * V + e] = xs[e];
        }
    } else {
#pragma unroll
        for (int i = 0; i < M; ++i) v[i] = (j0 + i < lim) ? p[j0 + i] : T(0);
    }
}

template <typename T, int M>
__device__ __forceinline__ void load_row_chunk_f(const float* p, int j0, int lim, float (&v)[M]) {
    if (j0 + M <= lim) {
        const float4* q = reinterpret_cast<const float4*>(p + j0);
#pragma unroll
        for (int b = 0; b < M / 4; ++b) {
            float4 x = q[b];
            v[4 * b] = x.x; v[4 * b + 1] = x.y; v[4 * b + 2] = x.z; v[4 * b + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < M; ++i) v[i] = (j0 + i < lim) ? p[j0 + i] : 1.0f;
    }
}

template <typename T, int M>
__device__ __forceinline__ void store_row_chunk(T* p, int j0, int lo, int hi, const T (&v)[M]) {
    if (j0 >= lo && j0 + M <= hi) {
        constexpr int V = 16 / sizeof(T);
        using V16 = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
        V16* q = reinterpret_cast<V16*>(p + j0);
#pragma unroll
        for (int b = 0; b < M / V; ++b) {
            V16 x;
            T* xs = reinterpret_cast<T*>(&x);
#pragma unroll
            for (int e = 0; e < V; ++e) xs[e] = v[b * V + e];
            q[b] = x;
        }
    } else {
#pragma unroll
        for (int i = 0; i < M; ++i)
            if (j0 + i >= lo && j0 + i < hi) p[j0 + i] = v[i];
    }
}

template <typename T, typename S, int M, int MODE>
__global__ void __launch_bounds__(256) pass_x_kernel(PassArgs<T, S> a) {
    constexpr int CE = ModeCE<MODE>::v, CH = ModeCH<MODE>::v;
    const int P = a.P;
    const int lane = threadIdx.x & 63;
    const int ls = lane & (P - 1);
    const long long line = ((long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * (64 / P) + lane / P;
    const long long nlines = (long long)a.na * a.nb;
    const bool live = line < nlines;
    const long long L = live ? line : 0;
    const int ia = a.a_lo + int(L % a.na), ib = a.b_lo + int(L / a.na);
    const long long base = ia * a.sa + ib * a.sb;
    const int n = a.n_w;
    const int j0 = ls * M;

    S ue[M], uh[M];
    float ep[M];
    {
        T te[M], th[M];
        load_row_chunk<T, M>(a.Ein + base, j0, n + 1, te);
        load_row_chunk<T, M>(a.Hin + base, j0, n, th);
#pragma unroll
        for (int i = 0; i < M; ++i) { ue[i] = S(te[i]); uh[i] = S(th[i]); }
    }
    load_row_chunk_f<T, M>(a.eps + base, j0, n, ep);
    const S uh_prev = (j0 > 0) ? S(a.Hin[base + j0 - 1]) : S(0);
    S ue_prev = S(0), ue_next = S(0);
    if constexpr (MODE == CONV_LOD) {
        ue_prev = (j0 > 0) ? S(a.Ein[base + j0 - 1]) : S(0);
        ue_next = (j0 + M <= n) ? S(a.Ein[base + j0 + M]) : S(0);
    }
    S x2[M];
    S uh_m_eff = uh_prev;
    if constexpr (MODE == CONV_ADI) {
        S D[M + 1];
#pragma unroll
        for (int i = -1; i < M; ++i) {
            const int j = j0 + i;
            D[i + 1] = (j >= 0 && j < n) ? S(a.E3[base + j + a.s_e]) - S(a.E3[base + j]) : S(0);
        }
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const int j = j0 + i;
            const S h2 = (j >= 1 && j < n) ? S(a.H2[base + j]) - S(a.H2[base + j - a.s_t]) : S(0);
            x2[i] = a.cH2 * h2;
            uh[i] += a.hE3 * D[i + 1];
        }
        uh_m_eff += a.hE3 * D[0];
    }

    S dg[M], r[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int j = j0 + i;
        const bool dir = (j == 0) || (j >= n);
        const bool is_src = (a.src >= 0) && (base + j == a.src);
        const S um = (i == 0) ? uh_m_eff : uh[i - 1];
        const S em = (i == 0) ? ue_prev : ue[i - 1];
        const S epv = (i == M - 1) ? ue_next : ue[i + 1];
        slot_rhs<T, S, MODE>(a, dir, is_src, ep[i], ue[i], uh[i], um, em, epv,
                             (MODE == CONV_ADI) ? x2[i] : S(0), dg[i], r[i]);
    }
    Chunk<S, M> c;
    chunk_eliminate<S, M, CE, CH>(dg, r, ue, uh, a.q, c);

    // Separator system across the P lanes of the line.  Every lane executes
    // every shuffle (a lane must not read from a lane that skipped it).
    const bool has_next = ls + 1 < P;
    const S a0n_r = __shfl_down(c.a0, 1, P), g0n_r = __shfl_down(c.g0, 1, P), y0n_r = __shfl_down(c.y0, 1, P);
    const S a0n = has_next ? a0n_r : S(0), g0n = has_next ? g0n_r : S(0), y0n = has_next ? y0n_r : S(0);
    const S Sl = pcr_wave<S>(separator_row<S>(c.aL, c.gL, c.yL, c.dgS, c.rS, a0n, g0n, y0n), ls, P);
    const S Sp_r = __shfl_up(Sl, 1, P), Sn_r = __shfl_down(Sl, 1, P);
    const S Sp = (ls > 0) ? Sp_r : S(0);
    const S Sn = has_next ? Sn_r : S(0);
    const S xn = y0n + a0n * Sl + g0n * Sn;

    S eo[M], ho[M];
    chunk_finish<S, M, CE, CH>(c, Sp, Sl, xn, ue_next, a.q, eo, ho);
    T te[M], th[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int j = j0 + i;
        S e = eo[i];
        if (MODE == FUND && a.src >= 0 && base + j == a.src) e -= a.src_post;
        if (j == 0 || j >= n) e = S(0);
        te[i] = T(e);
        th[i] = T(ho[i]);
    }
    if (live) {
        store_row_chunk<T, M>(a.Eout + base, j0, 1, n, te);
        store_row_chunk<T, M>(a.Hout + base, j0, 0, n, th);
    }
}

// ----------------------------------------------------------------------------
// y and z lines: strided axis.  A block holds TX consecutive x positions (the
// transverse index a) times P chunks; thread t = tx + TX p.  Loads and stores
// are coalesced across tx.  The separator rows go through LDS to segments of P
// consecutive lanes, are reduced by cross-lane PCR, and S returns through LDS.
// ----------------------------------------------------------------------------
template <typename T, typename S, int M, int MODE, int TX, int NT>
__global__ void __launch_bounds__(NT) pass_yz_kernel(PassArgs<T, S> a) {
    constexpr int CE = ModeCE<MODE>::v, CH = ModeCH<MODE>::v;
    extern __shared__ unsigned char smem_raw[];
    S* sm = reinterpret_cast<S*>(smem_raw);
    const int P = a.P;
    const int t = threadIdx.x;
    const int tx = t % TX, p = t / TX;
    constexpr int LD = TX + 1;                   // padded row (bank conflicts)
    S* ep_ = sm;                                 // [8][P][LD]
    S* sb_ = sm + 8 * P * LD;                    // [P][LD]
    auto EP = [&](int k, int pp, int xx) -> S& { return ep_[(k * P + pp) * LD + xx]; };
    auto SB = [&](int pp, int xx) -> S& { return sb_[pp * LD + xx]; };

    const int ia = blockIdx.x * TX + tx;
    const int ib = a.b_lo + blockIdx.y;
    const bool live = ia >= a.a_lo && ia < a.a_lo + a.na;
    const long long base = (long long)(live ? ia : a.a_lo) * a.sa + (long long)ib * a.sb;
    const int n = a.n_w;
    const int j0 = p * M;
    const long long sw = a.sw;

    S ue[M], uh[M], x2[M];
    float ep[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int j = j0 + i;
        const bool in = j < n;
        ue[i] = in ? S(a.Ein[base + j * sw]) : S(0);
        uh[i] = in ? S(a.Hin[base + j * sw]) : S(0);
        ep[i] = in ? a.eps[base + j * sw] : 1.0f;
    }
    const S uh_prev = (j0 > 0 && j0 <= n) ? S(a.Hin[base + (j0 - 1) * sw]) : S(0);
    S ue_prev = S(0), ue_next = S(0);
    if constexpr (MODE == CONV_LOD) {
        ue_prev = (j0 > 0 && j0 <= n) ? S(a.Ein[base + (j0 - 1) * sw]) : S(0);
        ue_next = (j0 + M <= n) ? S(a.Ein[base + (j0 + M) * sw]) : S(0);
    }
    S uh_m_eff = uh_prev;
    if constexpr (MODE == CONV_ADI) {
        S D[M + 1];
#pragma unroll
        for (int i = -1; i < M; ++i) {
            const int j = j0 + i;
            D[i + 1] = (j >= 0 && j < n) ? S(a.E3[base + j * sw + a.s_e]) - S(a.E3[base + j * sw]) : S(0);
        }
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const int j = j0 + i;
            const S h2 = (j >= 1 && j < n) ? S(a.H2[base + j * sw]) - S(a.H2[base + j * sw - a.s_t]) : S(0);
            x2[i] = a.cH2 * h2;
            uh[i] += a.hE3 * D[i + 1];
        }
        uh_m_eff += a.hE3 * D[0];
    }

    S dg[M], r[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int j = j0 + i;
        const bool dir = (j == 0) || (j >= n);
        const bool is_src = (a.src >= 0) && (base + j * sw == a.src);
        const S um = (i == 0) ? uh_m_eff : uh[i - 1];
        const S em = (i == 0) ? ue_prev : ue[i - 1];
        const S epv = (i == M - 1) ? ue_next : ue[i + 1];
        slot_rhs<T, S, MODE>(a, dir, is_src, ep[i], ue[i], uh[i], um, em, epv,
                             (MODE == CONV_ADI) ? x2[i] : S(0), dg[i], r[i]);
    }
    Chunk<S, M> c;
    chunk_eliminate<S, M, CE, CH>(dg, r, ue, uh, a.q, c);

    EP(0, p, tx) = c.a0; EP(1, p, tx) = c.g0; EP(2, p, tx) = c.y0;
    EP(3, p, tx) = c.aL; EP(4, p, tx) = c.gL; EP(5, p, tx) = c.yL;
    EP(6, p, tx) = c.dgS; EP(7, p, tx) = c.rS;
    __syncthreads();
    {
        // re-index: line = t / P, chunk = t % P (P consecutive lanes per line)
        const int pl = t % P, xl = t / P;
        const bool hn = pl + 1 < P;
        const int pn = hn ? pl + 1 : pl;
        Row<S> w = separator_row<S>(EP(3, pl, xl), EP(4, pl, xl), EP(5, pl, xl), EP(6, pl, xl), EP(7, pl, xl),
                                    hn ? EP(0, pn, xl) : S(0), hn ? EP(1, pn, xl) : S(0), hn ? EP(2, pn, xl) : S(0));
        const S Sv = pcr_wave<S>(w, pl, P);
        SB(pl, xl) = Sv;
    }
    __syncthreads();
    const S Sl = SB(p, tx);
    const S Sp = (p > 0) ? SB(p - 1, tx) : S(0);
    const bool hn = p + 1 < P;
    const int pn = hn ? p + 1 : p;
    const S Sn = hn ? SB(pn, tx) : S(0);
    const S xn = hn ? EP(2, pn, tx) + EP(0, pn, tx) * Sl + EP(1, pn, tx) * Sn : S(0);

    S eo[M], ho[M];
    chunk_finish<S, M, CE, CH>(c, Sp, Sl, xn, ue_next, a.q, eo, ho);
    if (!live) return;
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int j = j0 + i;
        if (j >= n) break;
        S e = eo[i];
        if (MODE == FUND && a.src >= 0 && base + j * sw == a.src) e -= a.src_post;
        if (j >= 1) a.Eout[base + j * sw] = T(e);
        a.Hout[base + j * sw] = T(ho[i]);
    }
}

}  // namespace fdtd
