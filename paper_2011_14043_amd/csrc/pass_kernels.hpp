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
//
// Memory access: every wave addresses its data through buffer resources whose
// 64-bit base is wave-uniform (SGPRs) and whose size is the rest of the
// array; a lane adds one 32-bit byte offset and each slot of a line adds a
// uniform scalar offset, so the per-slot address arithmetic costs no vector
// instructions, and loads past the end of an array return 0.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

#include "line_solver.hpp"
#include "xcd.hpp"

namespace fdtd {

// FUND_REF: the fundamental update with one step of iterative refinement of
// every tridiagonal solve (FP32 solves without their fixed rounding bias).
enum Mode { FUND = 0, CONV_LOD = 1, CONV_ADI = 2, FUND_REF = 3 };
template <int MODE> struct IsFund { static constexpr bool v = MODE == FUND || MODE == FUND_REF; };

template <typename T, typename S>
struct PassArgs {
    const T* Ein;
    const T* Hin;
    T* Eout;
    T* Hout;
    const T* H2;          // CONV_ADI: H component of Y's E row (shifted along t)
    const T* E3;          // CONV_ADI: E component of Y's H row (shifted along e)
    const float* eps;     // relative permittivity at node index (node layout)
    const float* mu;      // MU variants: relative permeability at node index (node layout)
    const unsigned char* mat;   // MAT variants: material index at node index (node layout)
    const float* mat_eps;       // MAT variants: eps_r of each material (<= 256 entries)
    int nmat;
    long long sw;         // stride along the line (elements)
    long long sa, sb;     // strides of the transverse line indices a, b
    long long s_t, s_e;   // CONV_ADI: strides along t and e
    long long comp;       // elements per component array
    int n_w;              // slots per line: 0 .. n_w-1 (slot 0 = wall)
    int a_lo, na, b_lo, nb;
    int P;                // chunks per line (power of two <= 64)
    int ntx;              // y/z lines: x tiles per row of blocks
    int nblk;             // number of blocks in the (1-D) grid
    int remap;            // 1: XCD-aware block order
    double Ks;            // sigma = Ks * eps_r
    S kap_hi, kap_lo;     // coefficient of the H difference (double-float if S = float)
    S q;                  // H update coefficient
    S cH2, hE3;           // CONV_ADI cross-term coefficients
    int src_a, src_b, src_j;   // source sample in line coordinates (src_a < 0: none)
    S src_pre, src_post;
    const double* src_pre_dev;  // if set, the value of src_pre is read from device memory
    const double* src_post_dev; // if set, the value of src_post is read from device memory
    double fsrc;          // FIN passes: added to E at the source sample (the g/2 the pass subtracts)
    // FIN passes (the last pass of a run over its pair) store the run's output:
    // with fin_add, u = U_old + U_new (fundamental ADI), else U_new; to Eout,
    // Hout with pitches of their own (the caller's arrays, or the state's):
    // along the transverse axes a, b and along the line, and the elements per
    // component.
    int fin_add;
    long long sa_o, sb_o, sw_o, comp_o;
};

// Output form of one slot in a FIN pass (the last B sub-step of a fundamental
// ADI run): the field v of that sub-step, u = U_old + U_new (Sec. II-E link),
// with U_new rounded as the state would store it, U_old as loaded, summed in
// FP64 and rounded once to the field type; at the source sample the g/2 the
// pass subtracted is added back.
template <typename T, typename S>
__device__ __forceinline__ void fin_value(const PassArgs<T, S>& a, T& oe, T& oh, T ue_old, T uh_old, bool at_src) {
    oe = T(double(oe) + double(ue_old) + (at_src ? a.fsrc : 0.0));
    oh = T(double(oh) + double(uh_old));
}


template <int MODE> struct ModeCE { static constexpr int v = IsFund<MODE>::v ? -1 : 0; };
template <int MODE> struct ModeCH { static constexpr int v = (MODE == CONV_LOD) ? 1 : 0; };

// ---------------------------------------------------------------------------
// buffer addressing
// ---------------------------------------------------------------------------
using Rsrc = __amdgpu_buffer_rsrc_t;
using V4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(Rsrc(), 0, 0, 0));
using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(Rsrc(), 0, 0, 0));

// Buffer resource for array `arr` (n_elem elements of `esz` bytes) starting at
// element `off` (may be past the end: then every access returns 0).
__device__ __forceinline__ Rsrc make_rsrc(const void* arr, long long off, long long n_elem, int esz) {
    const long long rem = (n_elem - off) * esz;
    const unsigned nr = rem <= 0 ? 0u : (rem > 0xFFFFFFFFll ? 0xFFFFFFFFu : (unsigned)rem);
    const char* p = static_cast<const char*>(arr) + off * esz;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(p), (short)0, (int)nr, 0x00020000);
}
template <typename T> struct Buf;
template <> struct Buf<float> {
    static __device__ __forceinline__ float ld(Rsrc r, int vo, int so) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    static __device__ __forceinline__ void st(float v, Rsrc r, int vo, int so) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, 0);
    }
};
template <> struct Buf<double> {
    static __device__ __forceinline__ double ld(Rsrc r, int vo, int so) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
    static __device__ __forceinline__ void st(double v, Rsrc r, int vo, int so) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, vo, so, 0);
    }
};

// Contiguous chunk of M elements at byte offset vo (16-byte aligned).
template <typename T, int M>
__device__ __forceinline__ void ld_chunk(Rsrc r, int vo, T (&v)[M]) {
    constexpr int V = 16 / sizeof(T);
    static_assert(M % V == 0, "chunk must be a multiple of 16 bytes");
#pragma unroll
    for (int b = 0; b < M / V; ++b) {
        const V4 x = __builtin_amdgcn_raw_buffer_load_b128(r, vo + 16 * b, 0, 0);
        if constexpr (sizeof(T) == 4) {
            const float4 f = __builtin_bit_cast(float4, x);
            v[4 * b] = f.x; v[4 * b + 1] = f.y; v[4 * b + 2] = f.z; v[4 * b + 3] = f.w;
        } else {
            const double2 f = __builtin_bit_cast(double2, x);
            v[2 * b] = f.x; v[2 * b + 1] = f.y;
        }
    }
}
template <typename T, int M>
__device__ __forceinline__ void st_chunk(Rsrc r, int vo, const T (&v)[M]) {
    constexpr int V = 16 / sizeof(T);
#pragma unroll
    for (int b = 0; b < M / V; ++b) {
        V4 x;
        if constexpr (sizeof(T) == 4) {
            x = __builtin_bit_cast(V4, make_float4(v[4 * b], v[4 * b + 1], v[4 * b + 2], v[4 * b + 3]));
        } else {
            x = __builtin_bit_cast(V4, make_double2(v[2 * b], v[2 * b + 1]));
        }
        __builtin_amdgcn_raw_buffer_store_b128(x, r, vo + 16 * b, 0, 0);
    }
}

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Per-slot coefficients of the scaled system: c multiplies U_e on the right
// side (2 sigma for FUND, sigma for the original forms), d = 2 + sigma is the
// diagonal.
template <typename S>
struct SlotCoef { S c, d; };
// M consecutive material bytes at byte offset vo (8-byte aligned).
template <int M>
__device__ __forceinline__ void ld_bytes(Rsrc r, int vo, unsigned (&id)[M]) {
    static_assert(M % 8 == 0, "byte chunk must be a multiple of 8");
#pragma unroll
    for (int b = 0; b < M / 8; ++b) {
        const V2 x = __builtin_amdgcn_raw_buffer_load_b64(r, vo + 8 * b, 0, 0);
#pragma unroll
        for (int e = 0; e < 8; ++e) id[8 * b + e] = (x[e / 4] >> (8 * (e % 4))) & 0xFFu;
    }
}

// ---------------------------------------------------------------------------
// per-slot right-hand side
// ---------------------------------------------------------------------------
// sigma of a slot.  In FP32 the diagonal 2 + sigma is rounded to the spacing
// of numbers near 2, which is coarse relative to a sigma << 1 (large time
// steps); sigma is therefore returned as fl(2 + sigma) - 2 (exact), so the
// diagonal and the right-hand side use the same value and every sub-step
// stays an exact Cayley factor of a (very slightly) perturbed medium instead
// of losing energy coherently step after step.
template <typename S>
__device__ __forceinline__ S make_sigma(double Ks, float eps) {
    if constexpr (sizeof(S) == 4) return (2.0f + float(Ks) * eps) - 2.0f;
    else return Ks * double(eps);
}
// Refined solves take sigma as it is: the rounded diagonal only shapes the
// factors, and the residual of the refinement step is formed with sigma itself
// (rhs c = 2 sigma exactly), so no fixed perturbation of the medium remains.
template <typename S, int MODE>
__device__ __forceinline__ SlotCoef<S> coef_of(double Ks, float eps) {
    const S sig = (MODE == FUND_REF) ? S(Ks * double(eps)) : make_sigma<S>(Ks, eps);
    return SlotCoef<S>{IsFund<MODE>::v ? sig + sig : sig, S(2) + sig};
}
// Material-index variants keep a per-material table in LDS, filled once per
// block.  FP32 solves store the coefficients themselves (one LDS read per
// slot, no per-slot arithmetic); FP64 solves store eps_r and form the
// coefficients per slot, which costs less than 16-byte table reads.
template <typename S>
using CoefTab = typename std::conditional<sizeof(S) == 4, SlotCoef<float>, float>::type;
template <typename T, typename S, int MODE>
__device__ __forceinline__ void load_coef_table(CoefTab<S>* tab, const PassArgs<T, S>& a) {
    for (int k = threadIdx.x; k < 256; k += blockDim.x) {
        const float e = k < a.nmat ? a.mat_eps[k] : 1.0f;
        if constexpr (sizeof(S) == 4) tab[k] = coef_of<S, MODE>(a.Ks, e);
        else tab[k] = e;
    }
    __syncthreads();
}
template <typename T, typename S, int MODE>
__device__ __forceinline__ SlotCoef<S> coef_from_tab(const PassArgs<T, S>& a, const CoefTab<S>* tab, unsigned id) {
    if constexpr (sizeof(S) == 4) return tab[id];
    else return coef_of<S, MODE>(a.Ks, tab[id]);
}

// rhs and diagonal of one slot; x2 = CONV_ADI cross term (scaled)
template <typename T, typename S, int MODE>
__device__ __forceinline__ void slot_rhs(const PassArgs<T, S>& a, SlotCoef<S> sc, S ue, S uh, S uh_m, S ue_m, S ue_p,
                                         S x2, S& dg, S& r) {
    dg = sc.d;
    const S dh = uh - uh_m;
    S hterm = dh * a.kap_hi;
    if constexpr (sizeof(S) == 4) hterm = __builtin_fmaf(dh, a.kap_lo, hterm);
    if constexpr (IsFund<MODE>::v) {
        r = sc.c * ue + hterm;
    } else if constexpr (MODE == CONV_LOD) {
        r = sc.c * ue + hterm + ((ue_p + ue_m) - S(2) * ue);
    } else {
        r = sc.c * ue + hterm + x2;
    }
}

// MU variants (variable permeability): rhs, diagonal and right-side
// coefficient c of one slot with m = mu0/mu at the H samples below (mlo) and
// above (mhi) it; eps_r from the FP32 map.  In FP32 sigma is taken as
// fl(m_lo + m_hi + sigma) - (m_lo + m_hi), so that the diagonal and the right
// side use one value (as make_sigma does for unit off-diagonals).
template <typename T, typename S, int MODE>
__device__ __forceinline__ void slot_rhs_mu(const PassArgs<T, S>& a, float eps, S mlo, S mhi, S ue, S uh, S uh_m,
                                            S ue_m, S ue_p, S x2, S& dg, S& r, S& c) {
    const S dsum = mlo + mhi;
    S sig;
    if constexpr (sizeof(S) == 4) {
        sig = S(a.Ks) * eps;
        dg = dsum + sig;
        sig = dg - dsum;
    } else {
        sig = a.Ks * double(eps);
        dg = dsum + sig;
    }
    c = IsFund<MODE>::v ? sig + sig : sig;
    const S dh = uh - uh_m;
    S hterm = dh * a.kap_hi;
    if constexpr (sizeof(S) == 4) hterm = __builtin_fmaf(dh, a.kap_lo, hterm);
    if constexpr (IsFund<MODE>::v) {
        r = c * ue + hterm;
    } else if constexpr (MODE == CONV_LOD) {
        r = c * ue + hterm + (mhi * (ue_p - ue) - mlo * (ue - ue_m));
    } else {
        r = c * ue + hterm + x2;
    }
}

// Source term at slot si of this chunk (rhs: 2 sigma pre or sigma pre).
// sigma is recovered from the diagonal: dg - 2 is exact.
template <typename T, typename S, int MODE, int M>
__device__ __forceinline__ void add_source(const PassArgs<T, S>& a, int si, const S (&dg)[M], S (&r)[M]) {
    const S pre = a.src_pre_dev ? S(*a.src_pre_dev) : a.src_pre;
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const S sig = dg[i] - S(2);
        const S coef = IsFund<MODE>::v ? sig + sig : sig;
        r[i] += (i == si) ? coef * pre : S(0);
    }
}

// The same with the right-side coefficients c of the slots given (MU variants).
template <typename T, typename S, int M>
__device__ __forceinline__ void add_source_c(const PassArgs<T, S>& a, int si, const S (&c)[M], S (&r)[M]) {
    const S pre = a.src_pre_dev ? S(*a.src_pre_dev) : a.src_pre;
#pragma unroll
    for (int i = 0; i < M; ++i) r[i] += (i == si) ? c[i] * pre : S(0);
}

// ---------------------------------------------------------------------------
// x lines: contiguous axis.  One line per segment of P lanes of a wave; lane
// `ls` owns slots [ls*M, ls*M+M), loaded with 16-byte buffer loads (rows are
// 128-byte aligned).  The separator system is solved with cross-lane PCR.
// FULL: P*M == n_w (no slot beyond the line).
// ---------------------------------------------------------------------------
// Body of one block of x-line work: block `blk` of the pass described by `a`
// (lines blk * waves * 64/P ...); ctab = the per-material coefficients in LDS (MAT).
// FIN: fin_lds = 64 * M elements of T per wave of the block (LDS).
template <typename T, typename S, int M, int MODE, bool FULL, bool MAT, bool FIN = false, bool MU = false>
__device__ __forceinline__ void pass_x_body(const PassArgs<T, S>& a, int blk, const CoefTab<S>* ctab,
                                            T* fin_lds = nullptr) {
    static_assert(!(MU && (MAT || MODE == FUND_REF)), "MU variants read eps_r maps and solve without refinement");
    constexpr int CE = ModeCE<MODE>::v, CH = ModeCH<MODE>::v;
    constexpr int ES = (int)sizeof(T);
    const int P = a.P;
    const int lane = threadIdx.x & 63;
    const int ls = lane & (P - 1);
    const int wave = wave_uniform(threadIdx.x >> 6);
    const long long nlines = (long long)a.na * a.nb;
    const long long raw0 = ((long long)blk * (blockDim.x >> 6) + wave) * (64 / P);
    const long long line = raw0 + lane / P;
    const bool live = line < nlines;
    const long long line0 = raw0 < nlines ? raw0 : nlines - 1;   // wave base line (clamped)
    const long long L = live ? line : line0;
    const int ia = a.a_lo + int(L % a.na), ib = a.b_lo + int(L / a.na);
    const long long wbase = (long long)(a.a_lo + int(line0 % a.na)) * a.sa + (long long)(a.b_lo + int(line0 / a.na)) * a.sb;
    const long long base = (long long)ia * a.sa + (long long)ib * a.sb;
    const int n = a.n_w;
    const int j0 = ls * M;
    const int lel = int(base - wbase) + j0;           // element offset of the chunk from the wave base
    const int vo = lel * ES, vo_e = lel * 4;
    const Rsrc rE = make_rsrc(a.Ein, wbase, a.comp, ES), rH = make_rsrc(a.Hin, wbase, a.comp, ES);
    const Rsrc rP = make_rsrc(a.eps, wbase, a.comp, 4);
    const Rsrc rMu = make_rsrc(a.mu, wbase, a.comp, 4);

    S ue[M], uh[M];
    SlotCoef<S> sc[M];
    unsigned idp[(M + 3) / 4] = {};   // refined solves: material indices, 4 per word
    float eps_s[M], mur_s[M];         // MU: eps_r and mu_r per slot
    {
        T te[M], th[M];
        if (!FULL && j0 >= n) {
            // chunk past the end of its line (power-of-two padding): no loads
#pragma unroll
            for (int i = 0; i < M; ++i) {
                te[i] = T(0); th[i] = T(0); sc[i] = SlotCoef<S>{S(0), S(2)};
                eps_s[i] = 1.0f; mur_s[i] = 1.0f;
            }
        } else {
            ld_chunk<T, M>(rE, vo, te);
            ld_chunk<T, M>(rH, vo, th);
            if constexpr (MAT) {
                unsigned id[M];
                ld_bytes<M>(make_rsrc(a.mat, wbase, a.comp, 1), lel, id);
#pragma unroll
                for (int i = 0; i < M; ++i) sc[i] = coef_from_tab<T, S, MODE>(a, ctab, id[i]);
#pragma unroll
                for (int i = 0; i < M; ++i) idp[i >> 2] |= id[i] << (8 * (i & 3));
            } else if constexpr (MU) {
                ld_chunk<float, M>(rP, vo_e, eps_s);
                ld_chunk<float, M>(rMu, vo_e, mur_s);
            } else {
                float ep[M];
                ld_chunk<float, M>(rP, vo_e, ep);
#pragma unroll
                for (int i = 0; i < M; ++i) sc[i] = coef_of<S, MODE>(a.Ks, ep[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const bool in = FULL || j0 + i < n;
            ue[i] = in ? S(te[i]) : S(0);
            uh[i] = in ? S(th[i]) : S(0);
        }
    }
    const bool first = j0 == 0;
    const bool beyond = j0 > n;
    const int vo_prev = (first || beyond) ? vo : vo - ES;
    const S uh_prev = (first || beyond) ? S(0) : S(Buf<T>::ld(rH, vo_prev, 0));
    // MU: m = mu0/mu at the H samples of the chunk's slots (0 past the line)
    // and at the one before it
    S mm[M], m_prev = S(0);
    if constexpr (MU) {
#pragma unroll
        for (int i = 0; i < M; ++i) mm[i] = (FULL || j0 + i < n) ? recip(S(mur_s[i])) : S(0);
        m_prev = (first || beyond) ? S(0) : recip(S(Buf<float>::ld(rMu, vo_e - 4, 0)));
    }
    S ue_prev = S(0), ue_next = S(0);
    if constexpr (MODE == CONV_LOD) {
        ue_prev = (first || beyond) ? S(0) : S(Buf<T>::ld(rE, vo_prev, 0));
        ue_next = (j0 + M <= n) ? S(Buf<T>::ld(rE, vo, M * ES)) : S(0);   // slot n (wall) exists
    }
    S x2[M];
    S uh_m_eff = uh_prev;
    if constexpr (MODE == CONV_ADI) {
        const Rsrc r3 = make_rsrc(a.E3, wbase, a.comp, ES);
        const Rsrc r2 = make_rsrc(a.H2, wbase, a.comp, ES);
        const Rsrc r2m = make_rsrc(a.H2, wbase - a.s_t, a.comp, ES);   // the t-1 neighbour rows
        const int se = (int)(a.s_e * ES);
        T e3a[M], e3b[M], h2a[M], h2b[M];
        ld_chunk<T, M>(r3, vo, e3a);
        ld_chunk<T, M>(r3, vo + se, e3b);
        ld_chunk<T, M>(r2, vo, h2a);
        ld_chunk<T, M>(r2m, vo, h2b);
        S D[M + 1];
        D[0] = (first || beyond) ? S(0) : S(Buf<T>::ld(r3, vo_prev, se)) - S(Buf<T>::ld(r3, vo_prev, 0));
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const bool in = FULL || j0 + i < n;
            D[i + 1] = in ? S(e3b[i]) - S(e3a[i]) : S(0);
            x2[i] = in ? a.cH2 * (S(h2a[i]) - S(h2b[i])) : S(0);
            uh[i] += (MU ? a.hE3 * mm[i] : a.hE3) * D[i + 1];
        }
        uh_m_eff += (MU ? a.hE3 * m_prev : a.hE3) * D[0];
    }

    S dg[M], r[M], cc[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const S um = (i == 0) ? uh_m_eff : uh[i - 1];
        const S em = (i == 0) ? ue_prev : ue[i - 1];
        const S epv = (i == M - 1) ? ue_next : ue[i + 1];
        if constexpr (MU)
            slot_rhs_mu<T, S, MODE>(a, eps_s[i], (i == 0) ? m_prev : mm[i - 1], mm[i], ue[i], uh[i], um, em, epv,
                                    (MODE == CONV_ADI) ? x2[i] : S(0), dg[i], r[i], cc[i]);
        else
            slot_rhs<T, S, MODE>(a, sc[i], ue[i], uh[i], um, em, epv, (MODE == CONV_ADI) ? x2[i] : S(0), dg[i], r[i]);
        if (!FULL) {
            const bool out = j0 + i >= n;
            dg[i] = out ? Big<S>::v : dg[i];
            r[i] = out ? S(0) : r[i];
        }
    }
    dg[0] = first ? Big<S>::v : dg[0];   // the wall at slot 0
    r[0] = first ? S(0) : r[0];
    // point source (one sample of one line): wave-uniform branch
    const int si = (ia == a.src_a && ib == a.src_b && live) ? a.src_j - j0 : -1;
    const bool src_here = si >= 0 && si < M;
    const bool src_wave = __ballot(src_here) != 0;
    if (MODE != FUND_REF && __builtin_expect(src_wave, 0)) {
        if constexpr (MU) add_source_c<T, S, M>(a, src_here ? si : -1, cc, r);
        else add_source<T, S, MODE, M>(a, src_here ? si : -1, dg, r);
    }
    // separator system across the P lanes of the line (all lanes shuffle):
    // own last interior slot (aL, gL, yL), separator row (dgS, rS), and the
    // next chunk's first slot (a0n, g0n, y0; zero past the line).  Returns
    // S_l, S_{l-1} and the next chunk's first value.
    const bool has_next = ls + 1 < P;
    auto separators = [&](S aL, S gL, S yL, S dgS, S rS, S a0n, S g0n, S y0, S& Sl, S& Sp, S& xn) {
        const S y0n_r = __shfl_down(y0, 1, P);
        const S y0n = has_next ? y0n_r : S(0);
        Sl = pcr_wave<S>(separator_row<S>(aL, gL, yL, dgS, rS, a0n, g0n, y0n), ls, P);
        const S Sp_r = __shfl_up(Sl, 1, P), Sn_r = __shfl_down(Sl, 1, P);
        Sp = (ls > 0) ? Sp_r : S(0);
        const S Sn = has_next ? Sn_r : S(0);
        xn = fused(g0n, Sn, fused(a0n, Sl, y0n));
    };

    S eo[M], ho[M];
    if constexpr (MODE == FUND_REF) {
        // refined solve: first solve, residual with the unrounded sigma, and
        // a correction solve with the same pivots (right sides recomputed
        // from the fields instead of kept in registers)
        unsigned fixed = first ? 1u : 0u;   // rows with no unknown: the wall, slots past the line
        if (!FULL) {
#pragma unroll
            for (int i = 0; i < M; ++i) fixed |= (j0 + i >= n) ? (1u << i) : 0u;
        }
        const S pre = src_wave ? (a.src_pre_dev ? S(*a.src_pre_dev) : a.src_pre) : S(0);
        // coefficients: from the LDS table again (material index) rather than kept
        auto coef = [&](int i) -> SlotCoef<S> {
            if constexpr (MAT) {
                if (!FULL && j0 >= n) return SlotCoef<S>{S(0), S(2)};
                return coef_from_tab<T, S, MODE>(a, ctab, (idp[i >> 2] >> (8 * (i & 3))) & 0xFFu);
            } else {
                return sc[i];
            }
        };
        auto rhs = [&](int i, S c) -> S {
            const S dh = uh[i] - ((i == 0) ? uh_m_eff : uh[i - 1]);
            S rr = fused(c, ue[i], fused(dh, a.kap_lo, dh * a.kap_hi));
            rr = (src_here && i == si) ? fused(c, pre, rr) : rr;
            return ((fixed >> i) & 1u) ? S(0) : rr;
        };
        S g[M - 1], d[M];
#pragma unroll
        for (int i = 0; i < M - 1; ++i) {
            const SlotCoef<S> sci = coef(i);
            const S dgi = ((fixed >> i) & 1u) ? Big<S>::v : sci.d;
            g[i] = recip(i == 0 ? dgi : dgi - g[i - 1]);
            d[i] = rhs(i, sci.c);
        }
        const S y0 = rsweep<S, M>(g, d);
        S a0, pL;
        rinfluence<S, M>(g, a0, pL);
        const SlotCoef<S> scS = coef(M - 1);
        const S dgS = ((fixed >> (M - 1)) & 1u) ? Big<S>::v : scS.d;
        const S a0n_r = __shfl_down(a0, 1, P), g0n_r = __shfl_down(pL, 1, P);
        const S a0n = has_next ? a0n_r : S(0), g0n = has_next ? g0n_r : S(0);
        S Sl, Sp, xn;
        separators(pL, g[M - 2], d[M - 2], dgS, rhs(M - 1, scS.c), a0n, g0n, y0, Sl, Sp, xn);
        rvalues<S, M>(g, d, Sp, Sl);
#pragma unroll
        for (int i = 0; i < M; ++i) asm volatile("" : "+v"(uh[i]));
        S rho[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const SlotCoef<S> sci = coef(i);
            const S vm = (i == 0) ? Sp : d[i - 1];
            const S vp = (i == M - 1) ? xn : d[i + 1];
            const S res = fused(S(-0.5) * sci.c, d[i], rhs(i, sci.c)) + ((vm - d[i]) + (vp - d[i]));
            rho[i] = ((fixed >> i) & 1u) ? S(0) : res;
            eo[i] = d[i] - ue[i];
            ho[i] = fused(a.q, vp - d[i], uh[i]);
        }
        // first outputs and the residual are final here (see the y/z lines)
#pragma unroll
        for (int i = 0; i < M; ++i) asm volatile("" : "+v"(eo[i]), "+v"(ho[i]), "+v"(rho[i]));
        const S rS = rho[M - 1];
        const S y0c = rsweep<S, M>(g, rho);
        S dSl, dSp, dxn;
        separators(pL, g[M - 2], rho[M - 2], dgS, rS, a0n, g0n, y0c, dSl, dSp, dxn);
        rvalues<S, M>(g, rho, dSp, dSl);
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const S dn = (i == M - 1) ? dxn : rho[i + 1];
            eo[i] += rho[i];
            ho[i] = fused(a.q, dn - rho[i], ho[i]);
        }
    } else if constexpr (MU) {
        ChunkMu<S, M> c;
        chunk_eliminate_mu<S, M, CE, CH>(dg, r, ue, uh, mm, m_prev, a.q, c);
        const S a0n_r = __shfl_down(c.a0, 1, P), g0n_r = __shfl_down(c.g0, 1, P);
        const S a0n = has_next ? a0n_r : S(0), g0n = has_next ? g0n_r : S(0);
        S Sl, Sp, xs;
        separators(c.aL, c.gL, c.yL, c.dgS, c.rS, a0n, g0n, c.y0, Sl, Sp, xs);
        chunk_finish_mu<S, M, CE, CH>(c, Sp, Sl, xs, ue_next, eo, ho);
    } else {
        Chunk<S, M> c;
        chunk_eliminate<S, M, CE, CH>(dg, r, ue, uh, a.q, c);
        const S a0n_r = __shfl_down(c.a0, 1, P), g0n_r = __shfl_down(c.g0, 1, P);
        const S a0n = has_next ? a0n_r : S(0), g0n = has_next ? g0n_r : S(0);
        S Sl, Sp, xn;
        separators(c.aL, c.gL, c.yL, c.dgS, c.rS, a0n, g0n, c.y0, Sl, Sp, xn);
        chunk_finish<S, M, CE, CH>(c, Sp, Sl, xn, ue_next, a.q, eo, ho);
    }
    eo[0] = first ? S(0) : eo[0];
    if (IsFund<MODE>::v && __builtin_expect(src_wave, 0)) {
        const S post = a.src_post_dev ? S(*a.src_post_dev) : a.src_post;
#pragma unroll
        for (int i = 0; i < M; ++i) eo[i] -= (src_here && i == si) ? post : S(0);
    }
    T te[M], th[M];
#pragma unroll
    for (int i = 0; i < M; ++i) { te[i] = T(eo[i]); th[i] = T(ho[i]); }
    if constexpr (FIN) {
        // the run's output: U_old of this thread's own slots is loaded again
        // (the output may overwrite them), with the chunk's aligned loads
        if (live && a.fin_add && (FULL || j0 < n)) {
            T oe[M], oh[M];
            ld_chunk<T, M>(rE, vo, oe);
            ld_chunk<T, M>(rH, vo, oh);
#pragma unroll
            for (int i = 0; i < M; ++i)
                if (FULL || j0 + i < n) fin_value<T, S>(a, te[i], th[i], oe[i], oh[i], src_here && i == si);
        }
        if (first) te[0] = T(0);   // the wall
        // Output pitches: the caller's rows need not be aligned, so the wave's
        // outputs go through LDS (lane l holds slots l*M .. l*M+M-1 of the
        // wave's 64/P lines, line by line) and each store instruction writes
        // 64 consecutive samples of a row rather than one sample per lane,
        // M samples apart.  Every thread of the block reaches the barriers
        // (lanes past the last line store nothing).
        T* tile = fin_lds + wave * 64 * M;
        const int PM = P * M;
#pragma unroll
        for (int arr = 0; arr < 2; ++arr) {
            T* out = arr == 0 ? a.Eout : a.Hout;
#pragma unroll
            for (int i = 0; i < M; ++i) tile[lane * M + i] = arr == 0 ? te[i] : th[i];
            __syncthreads();
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int f = lane + 64 * m;
                const int lw = f / PM, slot = f - lw * PM;
                const long long ln = raw0 + lw;
                if (ln < nlines && slot < n) {
                    const int ja = a.a_lo + int(ln % a.na), jb = a.b_lo + int(ln / a.na);
                    out[(long long)ja * a.sa_o + (long long)jb * a.sb_o + slot] = tile[f];
                }
            }
            __syncthreads();
        }
        return;
    }
    if (!live) return;
    const Rsrc wE = make_rsrc(a.Eout, wbase, a.comp, ES), wH = make_rsrc(a.Hout, wbase, a.comp, ES);
    if (FULL || j0 + M <= n) {
        st_chunk<T, M>(wE, vo, te);
        st_chunk<T, M>(wH, vo, th);
    } else {
#pragma unroll
        for (int i = 0; i < M; ++i) {
            if (j0 + i < n) {
                Buf<T>::st(te[i], wE, vo, i * ES);
                Buf<T>::st(th[i], wH, vo, i * ES);
            }
        }
    }
}

// FIN: the last pass of a run over its pair stores the run's output, with the
// output pitches: u = U_old + U_new with fin_add (output processing of the
// last B sub-step of a fundamental ADI run), else U_new (a separate
// instantiation, so the other passes carry none of its registers).
// MU: variable permeability (eps_r and mu_r maps, no material index).
template <typename T, typename S, int M, int MODE, bool FULL, bool MAT, bool FIN, bool MU = false>
__global__ void __launch_bounds__(256) pass_x_kernel(PassArgs<T, S> a) {
    __shared__ CoefTab<S> ctab[MAT ? 256 : 1];
    __shared__ T fin_lds[FIN ? 256 * M : 1];   // FIN: the outputs of each wave (at most 4 waves)
    if constexpr (MAT) load_coef_table<T, S, MODE>(ctab, a);
    pass_x_body<T, S, M, MODE, FULL, MAT, FIN, MU>(a, a.remap ? xcd_remap(blockIdx.x, a.nblk) : int(blockIdx.x),
                                                   ctab, fin_lds);
}

// ---------------------------------------------------------------------------
// y and z lines: strided axis.  A block holds TX consecutive x positions (the
// transverse index a) times P chunks; thread t = tx + TX p.  Loads and stores
// are coalesced across tx.  The separator rows go through LDS to segments of P
// consecutive lanes, are reduced by cross-lane PCR, and S returns through LDS.
// FULL: P*M == n_w.
// ---------------------------------------------------------------------------
// Body of one (virtual) block of TX * P threads: thread t, block index blk of
// the pass (blk < a.nblk when valid; an invalid block computes nothing and
// stores nothing but takes part in the barriers), LDS area sm of
// 9 P (TX+1) elements (13 P (TX+1) for refined solves, whose second
// separator exchange has areas of its own).  TX * P must be a multiple of 64
// (whole waves).
template <typename T, typename S, int M, int MODE, int TX, int NT, bool FULL, bool MAT, bool FIN = false,
          bool MU = false>
__device__ __forceinline__ void pass_yz_body(const PassArgs<T, S>& a, int blk, int t, S* sm, const CoefTab<S>* ctab,
                                             bool valid) {
    static_assert(!(MU && (MAT || MODE == FUND_REF)), "MU variants read eps_r maps and solve without refinement");
    constexpr int CE = ModeCE<MODE>::v, CH = ModeCH<MODE>::v;
    constexpr int ES = (int)sizeof(T);
    constexpr int CPW = 64 / TX;                  // chunks per wave
    const int P = a.P;
    const int tx = t % TX, p = t / TX;
    constexpr int LD = TX + 1;                   // padded row (bank conflicts)
    S* ep_ = sm;                                 // [8][P][LD]
    S* sb_ = sm + 8 * P * LD;                    // [P][LD]
    auto EP = [&](int k, int pp, int xx) -> S& { return ep_[(k * P + pp) * LD + xx]; };
    auto SB = [&](int pp, int xx) -> S& { return sb_[pp * LD + xx]; };
    // refined solves, second exchange: y_0, y_{M-2}, rS in [3][P][LD], S in [P][LD]
    S* ep2_ = sm + 9 * P * LD;
    S* sb2_ = sm + 12 * P * LD;
    auto EPs = [&](int set, int k, int pp, int xx) -> S& {
        if (set && (k == 2 || k == 5 || k == 7)) return ep2_[((k == 2 ? 0 : (k == 5 ? 1 : 2)) * P + pp) * LD + xx];
        return EP(k, pp, xx);
    };
    auto SBs = [&](int set, int pp, int xx) -> S& { return set ? sb2_[pp * LD + xx] : SB(pp, xx); };

    const int tile0 = (blk % a.ntx) * TX;
    const int ib = a.b_lo + blk / a.ntx;
    const int ia = tile0 + tx;
    const bool live = valid && ia >= a.a_lo && ia < a.a_lo + a.na;
    const int wave = wave_uniform(t >> 6);
    const int pw0 = wave * CPW;                  // first chunk of this wave
    const int n = a.n_w;
    const int j0 = p * M;
    const long long sw = a.sw;
    // wave base: line (tile0, ib), slot pw0*M; lane element offset tx + (p-pw0)*M*sw
    const long long wbase = (long long)tile0 * a.sa + (long long)ib * a.sb + (long long)pw0 * M * sw;
    const int swb = (int)(sw * ES), swf = (int)(sw * 4);
    const int lel = tx + (p - pw0) * M * (int)sw;
    const int vo = lel * ES, vo_e = lel * 4;
    const Rsrc rE = make_rsrc(a.Ein, wbase, a.comp, ES), rH = make_rsrc(a.Hin, wbase, a.comp, ES);
    const Rsrc rP = make_rsrc(a.eps, wbase, a.comp, 4);

    S ue[M], uh[M], x2[M];
    unsigned id[M];      // MAT: material index per slot
    float epf[M];        // else: eps_r per slot
    float mur_s[M];      // MU: mu_r per slot
    const Rsrc rM = make_rsrc(a.mat, wbase, a.comp, 1);
    const Rsrc rMu = make_rsrc(a.mu, wbase, a.comp, 4);
    T te[M], th[M];
    if (!FULL && j0 >= n) {
        // chunk past the end of its line (power-of-two padding): no loads
#pragma unroll
        for (int i = 0; i < M; ++i) {
            te[i] = T(0); th[i] = T(0); id[i] = 0u; epf[i] = 1.0f; mur_s[i] = 1.0f;
        }
    } else {
#pragma unroll
        for (int i = 0; i < M; ++i) {
            te[i] = Buf<T>::ld(rE, vo, i * swb);
            th[i] = Buf<T>::ld(rH, vo, i * swb);
            if constexpr (MAT) id[i] = __builtin_amdgcn_raw_buffer_load_b8(rM, lel, i * (int)sw, 0);
            else epf[i] = Buf<float>::ld(rP, vo_e, i * swf);
            if constexpr (MU) mur_s[i] = Buf<float>::ld(rMu, vo_e, i * swf);
        }
    }
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const bool in = FULL || j0 + i < n;
        ue[i] = in ? S(te[i]) : S(0);
        uh[i] = in ? S(th[i]) : S(0);
    }
    const bool first = (p == 0);
    const bool beyond = j0 > n;                   // chunk entirely past the far wall
    // slot j0-1 through resources based one slot earlier (offsets stay >= 0)
    const Rsrc rHm = make_rsrc(a.Hin, wbase - sw, a.comp, ES);
    const S uh_prev = (first || beyond) ? S(0) : S(Buf<T>::ld(rHm, vo, 0));
    // MU: m = mu0/mu at the H samples of the chunk's slots (0 past the line)
    // and at the one before it
    S mm[M], m_prev = S(0);
    if constexpr (MU) {
#pragma unroll
        for (int i = 0; i < M; ++i) mm[i] = (FULL || j0 + i < n) ? recip(S(mur_s[i])) : S(0);
        const Rsrc rMum = make_rsrc(a.mu, wbase - sw, a.comp, 4);
        m_prev = (first || beyond) ? S(0) : recip(S(Buf<float>::ld(rMum, vo_e, 0)));
    }
    S ue_prev = S(0), ue_next = S(0);
    if constexpr (MODE == CONV_LOD) {
        const Rsrc rEm = make_rsrc(a.Ein, wbase - sw, a.comp, ES);
        ue_prev = (first || beyond) ? S(0) : S(Buf<T>::ld(rEm, vo, 0));
        ue_next = (j0 + M <= n) ? S(Buf<T>::ld(rE, vo, M * swb)) : S(0);
    }
    S uh_m_eff = uh_prev;
    if constexpr (MODE == CONV_ADI) {
        const Rsrc r3 = make_rsrc(a.E3, wbase, a.comp, ES), r3m = make_rsrc(a.E3, wbase - sw, a.comp, ES);
        const Rsrc r2 = make_rsrc(a.H2, wbase, a.comp, ES), r2t = make_rsrc(a.H2, wbase - a.s_t, a.comp, ES);
        const int se = (int)(a.s_e * ES);
        S D[M + 1];
        D[0] = (first || beyond) ? S(0) : S(Buf<T>::ld(r3m, vo, se)) - S(Buf<T>::ld(r3m, vo, 0));
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const bool in = FULL || j0 + i < n;
            const S d = S(Buf<T>::ld(r3, vo, i * swb + se)) - S(Buf<T>::ld(r3, vo, i * swb));
            const S h2 = S(Buf<T>::ld(r2, vo, i * swb)) - S(Buf<T>::ld(r2t, vo, i * swb));
            D[i + 1] = in ? d : S(0);
            x2[i] = in ? a.cH2 * h2 : S(0);
            uh[i] += (MU ? a.hE3 * mm[i] : a.hE3) * D[i + 1];
        }
        uh_m_eff += (MU ? a.hE3 * m_prev : a.hE3) * D[0];
    }

    S dg[M], r[M], cc[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const S um = (i == 0) ? uh_m_eff : uh[i - 1];
        const S em = (i == 0) ? ue_prev : ue[i - 1];
        const S epv = (i == M - 1) ? ue_next : ue[i + 1];
        if constexpr (MU) {
            slot_rhs_mu<T, S, MODE>(a, epf[i], (i == 0) ? m_prev : mm[i - 1], mm[i], ue[i], uh[i], um, em, epv,
                                    (MODE == CONV_ADI) ? x2[i] : S(0), dg[i], r[i], cc[i]);
        } else {
            const SlotCoef<S> sci = MAT ? coef_from_tab<T, S, MODE>(a, ctab, id[i]) : coef_of<S, MODE>(a.Ks, epf[i]);
            slot_rhs<T, S, MODE>(a, sci, ue[i], uh[i], um, em, epv, (MODE == CONV_ADI) ? x2[i] : S(0), dg[i], r[i]);
        }
        if (!FULL) {
            const bool out = j0 + i >= n;
            dg[i] = out ? Big<S>::v : dg[i];
            r[i] = out ? S(0) : r[i];
        }
    }
    dg[0] = first ? Big<S>::v : dg[0];
    r[0] = first ? S(0) : r[0];
    const int si = (ia == a.src_a && ib == a.src_b && live) ? a.src_j - j0 : -1;
    const bool src_here = si >= 0 && si < M;
    const bool src_wave = __ballot(src_here) != 0;
    if (MODE != FUND_REF && __builtin_expect(src_wave, 0)) {
        if constexpr (MU) add_source_c<T, S, M>(a, src_here ? si : -1, cc, r);
        else add_source<T, S, MODE, M>(a, src_here ? si : -1, dg, r);
    }
    // Separator system: every chunk's end values go through LDS (slots
    // 0-2: first interior slot alpha, gamma, y; 3-5: last interior slot;
    // 6, 7: separator diagonal and right side), the P chunks of a line are
    // reduced on P consecutive lanes, and S returns through LDS.
    auto separators = [&](int set) {
        __syncthreads();
        {
            // re-index: line = t / P, chunk = t % P (P consecutive lanes per line)
            const int pl = t % P, xl = t / P;
            const bool hn = pl + 1 < P;
            const int pn = hn ? pl + 1 : pl;
            Row<S> w = separator_row<S>(EPs(set, 3, pl, xl), EPs(set, 4, pl, xl), EPs(set, 5, pl, xl),
                                        EPs(set, 6, pl, xl), EPs(set, 7, pl, xl), hn ? EPs(set, 0, pn, xl) : S(0),
                                        hn ? EPs(set, 1, pn, xl) : S(0), hn ? EPs(set, 2, pn, xl) : S(0));
            const S Sv = pcr_wave<S>(w, pl, P);
            SBs(set, pl, xl) = Sv;
        }
        __syncthreads();
    };
    const bool hn = p + 1 < P;
    const int pn = hn ? p + 1 : p;
    // S_l, S_{l-1} and the next chunk's first value, after separators(set)
    auto read_separators = [&](int set, S& Sl, S& Sp, S& xn) {
        Sl = SBs(set, p, tx);
        Sp = first ? S(0) : SBs(set, p - 1, tx);
        const S Sn = hn ? SBs(set, pn, tx) : S(0);
        xn = hn ? fused(EPs(set, 1, pn, tx), Sn, fused(EPs(set, 0, pn, tx), Sl, EPs(set, 2, pn, tx))) : S(0);
    };

    S eo[M], ho[M];
    if constexpr (MODE == FUND_REF) {
        // refined solve (see the x lines); material indices packed 4 per word
        unsigned fixed = first ? 1u : 0u;   // rows with no unknown: the wall, slots past the line
        if (!FULL) {
#pragma unroll
            for (int i = 0; i < M; ++i) fixed |= (j0 + i >= n) ? (1u << i) : 0u;
        }
        unsigned idp[(M + 3) / 4];
        if constexpr (MAT) {
#pragma unroll
            for (int k = 0; k < (M + 3) / 4; ++k) {
                unsigned w = 0;
#pragma unroll
                for (int e = 0; e < 4 && 4 * k + e < M; ++e) w |= id[4 * k + e] << (8 * e);
                idp[k] = w;
            }
        }
        auto coef = [&](int i) -> SlotCoef<S> {
            if constexpr (MAT) return coef_from_tab<T, S, MODE>(a, ctab, (idp[i >> 2] >> (8 * (i & 3))) & 0xFFu);
            else return coef_of<S, MODE>(a.Ks, epf[i]);
        };
        const S pre = src_wave ? (a.src_pre_dev ? S(*a.src_pre_dev) : a.src_pre) : S(0);
        auto rhs = [&](int i, S c) -> S {
            const S dh = uh[i] - ((i == 0) ? uh_m_eff : uh[i - 1]);
            S rr = fused(c, ue[i], fused(dh, a.kap_lo, dh * a.kap_hi));
            rr = (src_here && i == si) ? fused(c, pre, rr) : rr;
            return ((fixed >> i) & 1u) ? S(0) : rr;
        };
        S g[M - 1], d[M];
#pragma unroll
        for (int i = 0; i < M - 1; ++i) {
            const SlotCoef<S> sci = coef(i);
            const S dgi = ((fixed >> i) & 1u) ? Big<S>::v : sci.d;
            g[i] = recip(i == 0 ? dgi : dgi - g[i - 1]);
            d[i] = rhs(i, sci.c);
        }
        const S y0 = rsweep<S, M>(g, d);
        S a0, pL;
        rinfluence<S, M>(g, a0, pL);
        const SlotCoef<S> scS = coef(M - 1);
        EP(0, p, tx) = a0; EP(1, p, tx) = pL; EP(2, p, tx) = y0;
        EP(3, p, tx) = pL; EP(4, p, tx) = g[M - 2]; EP(5, p, tx) = d[M - 2];
        EP(6, p, tx) = ((fixed >> (M - 1)) & 1u) ? Big<S>::v : scS.d;
        EP(7, p, tx) = rhs(M - 1, scS.c);
        separators(0);
        S Sl, Sp, xn;
        read_separators(0, Sl, Sp, xn);
        rvalues<S, M>(g, d, Sp, Sl);
        // the right sides are formed again from the fields (an opaque copy,
        // so that the first ones are not kept live across the barriers)
#pragma unroll
        for (int i = 0; i < M; ++i) asm volatile("" : "+v"(uh[i]));
        S rho[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const SlotCoef<S> sci = coef(i);
            const S vm = (i == 0) ? Sp : d[i - 1];
            const S vp = (i == M - 1) ? xn : d[i + 1];
            const S res = fused(S(-0.5) * sci.c, d[i], rhs(i, sci.c)) + ((vm - d[i]) + (vp - d[i]));
            rho[i] = ((fixed >> i) & 1u) ? S(0) : res;
            eo[i] = d[i] - ue[i];
            ho[i] = fused(a.q, vp - d[i], uh[i]);
        }
        // keep the compiler from re-deriving the first outputs after the
        // barriers below (that would hold V and the fields live instead)
#pragma unroll
        for (int i = 0; i < M; ++i) asm volatile("" : "+v"(eo[i]), "+v"(ho[i]), "+v"(rho[i]));
        const S rS = rho[M - 1];
        const S y0c = rsweep<S, M>(g, rho);
        EPs(1, 2, p, tx) = y0c; EPs(1, 5, p, tx) = rho[M - 2]; EPs(1, 7, p, tx) = rS;
        separators(1);
        S dSl, dSp, dxn;
        read_separators(1, dSl, dSp, dxn);
        rvalues<S, M>(g, rho, dSp, dSl);
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const S dn = (i == M - 1) ? dxn : rho[i + 1];
            eo[i] += rho[i];
            ho[i] = fused(a.q, dn - rho[i], ho[i]);
        }
    } else if constexpr (MU) {
        // first and last interior values scaled by their off-diagonals (see
        // ChunkMu): the exchange and xn (= m[M-1] times the next chunk's
        // first value) as for unit off-diagonals
        ChunkMu<S, M> c;
        chunk_eliminate_mu<S, M, CE, CH>(dg, r, ue, uh, mm, m_prev, a.q, c);
        EP(0, p, tx) = c.a0; EP(1, p, tx) = c.g0; EP(2, p, tx) = c.y0;
        EP(3, p, tx) = c.aL; EP(4, p, tx) = c.gL; EP(5, p, tx) = c.yL;
        EP(6, p, tx) = c.dgS; EP(7, p, tx) = c.rS;
        separators(0);
        S Sl, Sp, xs;
        read_separators(0, Sl, Sp, xs);
        chunk_finish_mu<S, M, CE, CH>(c, Sp, Sl, xs, ue_next, eo, ho);
    } else {
        Chunk<S, M> c;
        chunk_eliminate<S, M, CE, CH>(dg, r, ue, uh, a.q, c);
        EP(0, p, tx) = c.a0; EP(1, p, tx) = c.g0; EP(2, p, tx) = c.y0;
        EP(3, p, tx) = c.aL; EP(4, p, tx) = c.gL; EP(5, p, tx) = c.yL;
        EP(6, p, tx) = c.dgS; EP(7, p, tx) = c.rS;
        separators(0);
        S Sl, Sp, xn;
        read_separators(0, Sl, Sp, xn);
        chunk_finish<S, M, CE, CH>(c, Sp, Sl, xn, ue_next, a.q, eo, ho);
    }
    eo[0] = first ? S(0) : eo[0];
    if (IsFund<MODE>::v && __builtin_expect(src_wave, 0)) {
        const S post = a.src_post_dev ? S(*a.src_post_dev) : a.src_post;
#pragma unroll
        for (int i = 0; i < M; ++i) eo[i] -= (src_here && i == si) ? post : S(0);
    }
    if (!live) return;
    T ot[M], oh[M];   // the values stored
#pragma unroll
    for (int i = 0; i < M; ++i) { ot[i] = T(eo[i]); oh[i] = T(ho[i]); }
    long long wb = wbase, ncomp = a.comp;
    int vs = vo, sws = swb;
    if constexpr (FIN) {
        // the run's output (see the x lines)
        if (a.fin_add) {
#pragma unroll
            for (int i = 0; i < M; ++i) {
                if (FULL || j0 + i < n) {
                    fin_value<T, S>(a, ot[i], oh[i], Buf<T>::ld(rE, vo, i * swb), Buf<T>::ld(rH, vo, i * swb),
                                    src_here && i == si);
                }
            }
        }
        if (first) ot[0] = T(0);   // the wall
        wb = (long long)tile0 * a.sa_o + (long long)ib * a.sb_o + (long long)pw0 * M * a.sw_o;
        vs = (tx + (p - pw0) * M * (int)a.sw_o) * ES;
        sws = (int)(a.sw_o * ES);
        ncomp = a.comp_o;
    }
    const Rsrc wE = make_rsrc(a.Eout, wb, ncomp, ES), wH = make_rsrc(a.Hout, wb, ncomp, ES);
#pragma unroll
    for (int i = 0; i < M; ++i) {
        if (FULL || j0 + i < n) {
            Buf<T>::st(ot[i], wE, vs, i * sws);
            Buf<T>::st(oh[i], wH, vs, i * sws);
        }
    }
}

// Waves per SIMD the register allocation must allow: FP32 solves with 8-slot
// chunks (modes without the cross-term arrays) fit in 64 VGPRs, so two
// 1024-thread blocks share a CU and one block's loads overlap the other's LDS
// phase.
template <typename S, int M, int MODE, int NT, bool MU>
struct YzOcc {
    static constexpr int v =
        (sizeof(S) == 4 && M <= 8 && NT == 1024 && MODE != CONV_ADI && MODE != FUND_REF && !MU) ? 8 : 1;
};

// MU: variable permeability (eps_r and mu_r maps, no material index).
template <typename T, typename S, int M, int MODE, int TX, int NT, bool FULL, bool MAT, bool FIN, bool MU = false>
__global__ void __launch_bounds__(NT, (YzOcc<S, M, MODE, NT, MU>::v)) pass_yz_kernel(PassArgs<T, S> a) {
    __shared__ CoefTab<S> ctab[MAT ? 256 : 1];
    if constexpr (MAT) load_coef_table<T, S, MODE>(ctab, a);
    extern __shared__ unsigned char smem_raw[];
    pass_yz_body<T, S, M, MODE, TX, NT, FULL, MAT, FIN, MU>(
        a, a.remap ? xcd_remap(blockIdx.x, a.nblk) : int(blockIdx.x), threadIdx.x, reinterpret_cast<S*>(smem_raw),
        ctab, true);
}

}  // namespace fdtd
