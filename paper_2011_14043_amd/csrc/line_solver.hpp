// line_solver.hpp -- register-resident tridiagonal line solver for gfx950.
//
// Every implicit update of the method reduces, per grid line of the solve axis
// w, to the scaled tridiagonal system
//
//     -V[j-1] + (2 + sigma[j]) V[j] - V[j+1] = r[j],   j = 0 .. n-1,
//
// (the fundamental equation 1/2 E~ - (b d / 2) d_w^2 E~ = e + s b d_w h of
// Sec. III-A, and the original (I - theta X) systems, multiplied by
// 2 sigma or sigma, sigma = 1/(p q), p = b/dw, q = d/dw).  It is strictly
// diagonally dominant, so no pivoting is needed.  PEC walls (Dirichlet V = 0)
// are rows whose diagonal is BIG = 2^100: they decouple from their neighbours
// below working precision in FP32 and FP64.
//
// A line is split into P chunks of M consecutive slots, one chunk per thread.
// The last slot of each chunk is a separator S_l.  The M-1 interior slots of
// chunk l depend only on S_{l-1} and S_l:
//     x_i = y_i + alpha_i S_{l-1} + gamma_i S_l,
// with y = T^{-1} r, alpha = T^{-1} e_0, gamma = T^{-1} e_{M-2} from one LU
// sweep of the chunk (Thomas' forward elimination with running products).
// Eliminating the interiors leaves a P x P tridiagonal system in the separators
// (a Schur complement, again diagonally dominant), solved by parallel cyclic
// reduction across the P threads.  Each thread then finishes its own slots.
// No per-slot data leaves the registers; HBM sees only the line's inputs and
// outputs once.
#pragma once
#include <hip/hip_runtime.h>

namespace fdtd {

template <typename T> struct Big;
template <> struct Big<float> { static constexpr float v = 1.2676506e30f; };   // 2^100
template <> struct Big<double> { static constexpr double v = 1.2676506002282294e30; };

// a * b + c with one rounding.  Written out where the result must not depend
// on which multiply-adds the compiler chooses to fuse (that choice can differ
// between kernels that inline the same code).
__device__ __forceinline__ float fused(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fused(double a, double b, double c) { return __builtin_fma(a, b, c); }
// a * b rounded once and never fused into a later addition (an FMA with a zero
// addend): a product that several expressions use then rounds the same way in
// every kernel, whichever uses the compiler would otherwise have fused.
__device__ __forceinline__ float sealed_mul(float a, float b) { return __builtin_fmaf(a, b, 0.0f); }
__device__ __forceinline__ double sealed_mul(double a, double b) { return __builtin_fma(a, b, 0.0); }

// Reciprocal of a positive normal number (pivots, diagonals): the hardware
// estimate refined by Newton-Raphson steps r <- r + r (1 - x r), one for FP32
// and two for FP64 (each step squares the relative error), which ends within
// about an ulp without the scaling and fix-up steps of an IEEE division.
__device__ __forceinline__ float recip(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

// Per-thread state of one chunk after local elimination, folded with the
// outputs so that 4 words per slot stay live:
//   W[i] = y_i + CE * ue_i,   Z[i] = uh_i + q * (y_{i+1} - y_i + CH (ue_{i+1} - ue_i))
// for interior slots; slot M-1 (the separator) keeps ue, uh.
template <typename T, int M>
struct Chunk {
    T W[M], Z[M], al[M], ga[M];
    T a0, g0, y0;   // alpha_0, gamma_0, y_0   (needed by the previous chunk)
    T aL, gL, yL;   // alpha_{M-2}, gamma_{M-2}, y_{M-2}
    T dgS, rS;      // separator row: diagonal and right side
};

// Local elimination of one chunk.  CE = -1: E' = V - U_e (fundamental);
// CE = 0: E' = V (original forms).  CH = 1 adds U_e to the H difference
// (original LOD family: H' = H + q d_w(E + E')).
template <typename T, int M, int CE, int CH>
__device__ __forceinline__ void chunk_eliminate(const T (&dg)[M], const T (&r)[M], const T (&ue)[M],
                                                const T (&uh)[M], T q, Chunk<T, M>& c) {
    static_assert(M >= 2, "chunk needs an interior slot and a separator");
    T g[M - 1], d[M - 1], p[M - 1];
    g[0] = recip(dg[0]);
    d[0] = r[0] * g[0];
    p[0] = g[0];
#pragma unroll
    for (int i = 1; i < M - 1; ++i) {
        g[i] = recip(dg[i] - g[i - 1]);
        d[i] = (r[i] + d[i - 1]) * g[i];
        p[i] = p[i - 1] * g[i];
    }
    T y = d[M - 2], a = p[M - 2], gm = g[M - 2];
    c.yL = y; c.aL = a; c.gL = gm;
    c.W[M - 2] = y + T(CE) * ue[M - 2];
    c.Z[M - 2] = uh[M - 2] + q * ((T(0) - y) + T(CH) * (ue[M - 1] - ue[M - 2]));
    c.al[M - 2] = a;
    c.ga[M - 2] = gm;
#pragma unroll
    for (int i = M - 3; i >= 0; --i) {
        const T yi = d[i] + g[i] * y;
        const T ai = p[i] + g[i] * a;
        const T gi = g[i] * gm;
        c.W[i] = yi + T(CE) * ue[i];
        c.Z[i] = uh[i] + q * ((y - yi) + T(CH) * (ue[i + 1] - ue[i]));
        c.al[i] = ai;
        c.ga[i] = gi;
        y = yi; a = ai; gm = gi;
    }
    c.y0 = y; c.a0 = a; c.g0 = gm;
    c.W[M - 1] = ue[M - 1];
    c.Z[M - 1] = uh[M - 1];
    c.al[M - 1] = T(0);
    c.ga[M - 1] = T(1);
    c.dgS = dg[M - 1];
    c.rS = r[M - 1];
}

// Separator row l from chunk l (own) and chunk l+1 (next; zeros past the end).
template <typename T>
struct Row { T A, B, C, D; };

template <typename T>
__device__ __forceinline__ Row<T> separator_row(T aL, T gL, T yL, T dgS, T rS, T a0n, T g0n, T y0n) {
    Row<T> w;
    w.A = -aL;
    w.B = dgS - gL - a0n;
    w.C = -g0n;
    w.D = rS + yL + y0n;
    return w;
}

// Parallel cyclic reduction over segments of `P` consecutive lanes of a wave
// (P a power of two <= 64; lane's position in its segment is `ls`).  Rows
// outside the segment are identity rows.  Returns S_ls.
template <typename T>
__device__ __forceinline__ T pcr_wave(Row<T> w, int ls, int P) {
    for (int s = 1; s < P; s <<= 1) {
        const T Am = __shfl_up(w.A, s, P), Bm = __shfl_up(w.B, s, P);
        const T Cm = __shfl_up(w.C, s, P), Dm = __shfl_up(w.D, s, P);
        const T Ap = __shfl_down(w.A, s, P), Bp = __shfl_down(w.B, s, P);
        const T Cp = __shfl_down(w.C, s, P), Dp = __shfl_down(w.D, s, P);
        const bool hm = ls - s >= 0, hp = ls + s < P;
        const T k1 = hm ? w.A * recip(Bm) : T(0);
        const T k2 = hp ? w.C * recip(Bp) : T(0);
        Row<T> n;
        n.A = hm ? -k1 * Am : T(0);
        n.C = hp ? -k2 * Cp : T(0);
        const T b1 = hm ? fused(-k1, Cm, w.B) : w.B;
        const T d1 = hm ? fused(-k1, Dm, w.D) : w.D;
        n.B = hp ? fused(-k2, Ap, b1) : b1;
        n.D = hp ? fused(-k2, Dp, d1) : d1;
        w = n;
    }
    return sealed_mul(w.D, recip(w.B));
}

// Final values of one chunk given S_{l-1} (Sp), S_l (S) and the first slot of
// chunk l+1 (xn, with its U_e value uen for CH = 1).  Writes E' and H' for
// slot i into eo[i], ho[i].
template <typename T, int M, int CE, int CH>
__device__ __forceinline__ void chunk_finish(const Chunk<T, M>& c, T Sp, T S, T xn, T uen, T q,
                                             T (&eo)[M], T (&ho)[M]) {
#pragma unroll
    for (int i = 0; i < M - 1; ++i) {
        eo[i] = c.W[i] + c.al[i] * Sp + c.ga[i] * S;
        ho[i] = c.Z[i] + q * ((c.al[i + 1] - c.al[i]) * Sp + (c.ga[i + 1] - c.ga[i]) * S);
    }
    eo[M - 1] = S + T(CE) * c.W[M - 1];
    ho[M - 1] = c.Z[M - 1] + q * ((xn - S) + T(CH) * (uen - c.W[M - 1]));
}

// ---------------------------------------------------------------------------
// Variable permeability.  With mu varying along the line the scaled system is
//     -m[j-1] V[j-1] + (sigma[j] + m[j-1] + m[j]) V[j] - m[j] V[j+1] = r[j],
// m[j] = mu0 / mu at the H sample j + 1/2 (stored at slot j): symmetric,
// strictly diagonally dominant, off-diagonals that differ from row to row.
// A chunk's interior system T (rows 0..M-2) has lower off-diagonals
// m[i-1] (m[-1] = mp, the H sample before the chunk) and upper ones m[i]:
//     x_i = y_i + ah_i (mp S_{l-1}) + gh_i (m[M-2] S_l),
// y = T^-1 r, ah = T^-1 e_0, gh = T^-1 e_{M-2} (Thomas' sweeps with the
// off-diagonals).  The separator row of chunk l,
//     -m[M-2] x_{M-2} + dg S_l - m[M-1] x'_0 = r,
// takes the same form as with unit off-diagonals once chunk l stores
// m[M-2] times its last interior values and chunk l+1 stores mp' = m[M-1]
// times its first ones (ChunkMu below): separator_row and the PCR are shared.
// ---------------------------------------------------------------------------
template <typename T, int M>
struct ChunkMu : Chunk<T, M> {
    T qv[M];        // H update coefficient per slot (q0 m[i])
    T q0;
    T mp, mL;       // m[-1], m[M-2]
};

// Local elimination of one chunk with off-diagonals m (see above); q0 is the
// H update coefficient for mu = mu0.  Stores a0, g0, y0 (first interior slot)
// times mp and aL, gL, yL (last interior slot) times m[M-2].
template <typename T, int M, int CE, int CH>
__device__ __forceinline__ void chunk_eliminate_mu(const T (&dg)[M], const T (&r)[M], const T (&ue)[M],
                                                   const T (&uh)[M], const T (&m)[M], T mp, T q0,
                                                   ChunkMu<T, M>& c) {
    static_assert(M >= 2, "chunk needs an interior slot and a separator");
    T g[M - 1], d[M - 1], p[M - 1];
    g[0] = recip(dg[0]);
    d[0] = r[0] * g[0];
    p[0] = g[0];
#pragma unroll
    for (int i = 1; i < M - 1; ++i) {
        const T l = m[i - 1];
        g[i] = recip(dg[i] - l * l * g[i - 1]);
        d[i] = fused(l, d[i - 1], r[i]) * g[i];
        p[i] = l * p[i - 1] * g[i];
    }
#pragma unroll
    for (int i = 0; i < M; ++i) c.qv[i] = q0 * m[i];
    c.q0 = q0;
    c.mp = mp;
    c.mL = m[M - 2];
    T y = d[M - 2], a = p[M - 2], gm = g[M - 2];
    c.yL = c.mL * y; c.aL = c.mL * mp * a; c.gL = c.mL * c.mL * gm;
    c.W[M - 2] = y + T(CE) * ue[M - 2];
    c.Z[M - 2] = uh[M - 2] + c.qv[M - 2] * ((T(0) - y) + T(CH) * (ue[M - 1] - ue[M - 2]));
    c.al[M - 2] = a;
    c.ga[M - 2] = gm;
#pragma unroll
    for (int i = M - 3; i >= 0; --i) {
        const T e = m[i] * g[i];
        const T yi = fused(e, y, d[i]);
        const T ai = fused(e, a, p[i]);
        const T gi = e * gm;
        c.W[i] = yi + T(CE) * ue[i];
        c.Z[i] = uh[i] + c.qv[i] * ((y - yi) + T(CH) * (ue[i + 1] - ue[i]));
        c.al[i] = ai;
        c.ga[i] = gi;
        y = yi; a = ai; gm = gi;
    }
    c.y0 = mp * y; c.a0 = mp * mp * a; c.g0 = mp * c.mL * gm;
    c.W[M - 1] = ue[M - 1];
    c.Z[M - 1] = uh[M - 1];
    c.al[M - 1] = T(0);
    c.ga[M - 1] = T(0);
    c.dgS = dg[M - 1];
    c.rS = r[M - 1];
}

// Final values of a ChunkMu given S_{l-1} (Sp), S_l (S) and xs = m[M-1] times
// the first value of chunk l+1 (what the separator exchange yields from the
// scaled first-slot values), with that slot's U_e value uen for CH = 1.
template <typename T, int M, int CE, int CH>
__device__ __forceinline__ void chunk_finish_mu(const ChunkMu<T, M>& c, T Sp, T S, T xs, T uen, T (&eo)[M],
                                                T (&ho)[M]) {
    const T sp = c.mp * Sp, sl = c.mL * S;
#pragma unroll
    for (int i = 0; i < M - 1; ++i) eo[i] = c.W[i] + c.al[i] * sp + c.ga[i] * sl;
#pragma unroll
    for (int i = 0; i < M - 2; ++i)
        ho[i] = c.Z[i] + c.qv[i] * ((c.al[i + 1] - c.al[i]) * sp + (c.ga[i + 1] - c.ga[i]) * sl);
    ho[M - 2] = c.Z[M - 2] + c.qv[M - 2] * ((S - c.al[M - 2] * sp) - c.ga[M - 2] * sl);
    eo[M - 1] = S + T(CE) * c.W[M - 1];
    // q[M-1] (x'_0 - S) = q0 xs - q[M-1] S
    ho[M - 1] = c.Z[M - 1] + ((c.q0 * xs - c.qv[M - 1] * S) + c.qv[M - 1] * (T(CH) * (uen - c.W[M - 1])));
}

// ---------------------------------------------------------------------------
// Refined solves.  The coefficients of the elimination (pivots, influence
// vectors, the separator system) depend only on the medium, so in FP32 their
// rounding is the same at every time step: a fixed perturbation of the
// operator, whose phase error grows linearly with the step count.  One step of
// iterative refinement in working precision -- the residual rho = r - T V,
// then a second solve T dV = rho with the same factors -- takes that bias to
// second order; what is left is rounding that changes from step to step.
// ---------------------------------------------------------------------------
// A refined chunk keeps only the inverse pivots g of its interior rows.  With
// p_k = g_0 ... g_k (p_{-1} = 1), the values the separator rows need follow
// from forward sweeps alone:  alpha_{M-2} = gamma_0 = p_{M-2},
// gamma_{M-2} = g_{M-2},  alpha_0 = sum_k p_{k-1} p_k,  y_{M-2} = d_{M-2} and
// y_0 = sum_k p_{k-1} d_k  (d: the forward-swept right side), since
// alpha_i = p_i + g_i alpha_{i+1} and y_i = d_i + g_i y_{i+1}.

// Forward sweep of the interior rows 0..M-2 in place (d holds the right side
// on entry): d_i <- (d_i + d_{i-1}) g_i.  Returns y_0.
template <typename T, int M>
__device__ __forceinline__ T rsweep(const T (&g)[M - 1], T (&d)[M]) {
    d[0] = sealed_mul(d[0], g[0]);
    T p = g[0], y0 = d[0];
#pragma unroll
    for (int i = 1; i < M - 1; ++i) {
        d[i] = sealed_mul(d[i] + d[i - 1], g[i]);
        y0 = fused(p, d[i], y0);
        p = p * g[i];
    }
    return y0;
}

// alpha_0 and p_{M-2} of the interior rows.
template <typename T, int M>
__device__ __forceinline__ void rinfluence(const T (&g)[M - 1], T& a0, T& pL) {
    T p = g[0], a = g[0];
#pragma unroll
    for (int i = 1; i < M - 1; ++i) {
        const T pn = p * g[i];
        a = fused(p, pn, a);
        p = pn;
    }
    a0 = a;
    pL = p;
}

// Slot values from the forward-swept d once the separators S_{l-1} (Sp) and
// S_l (S) are known, in place: the interior rows see Sp in row 0 and S in row
// M-2, i.e. d_k + Sp p_k, then the backward sweep; V[M-1] = S.
template <typename T, int M>
__device__ __forceinline__ void rvalues(const T (&g)[M - 1], T (&V)[M], T Sp, T S) {
    T p = g[0];
    V[0] = fused(Sp, p, V[0]);
#pragma unroll
    for (int i = 1; i < M - 1; ++i) {
        p = p * g[i];
        V[i] = fused(Sp, p, V[i]);
    }
    V[M - 1] = S;
#pragma unroll
    for (int i = M - 2; i >= 0; --i) V[i] = fused(g[i], V[i + 1], V[i]);
}

}  // namespace fdtd
