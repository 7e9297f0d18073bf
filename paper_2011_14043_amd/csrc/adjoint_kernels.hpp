// adjoint_kernels.hpp -- reverse-mode gradient of a probe objective of the
// fundamental ADI with respect to eps_r.
//
// Forward, in the link scaling of Sec. II-E, every sub-step with operator X
// and half-span theta maps the state U^m to
//     W = U^m + h,   V = 2 (I - theta X)^{-1} W,   U^{m+1} = V - W,
// h = half the source term of the sub-step (one Ez sample); V of every B
// sub-step is the physical field u^{n+1}.  The objective is
//     J = dt * sum_n |E(u^{n+1})|^2 at the probe node.
// X = M^{-1} K with M = diag(eps, mu) and K skew-symmetric (eq. (AMat) on the
// Yee grid), so (I - theta X)^{-T} = M (I + theta X)^{-1} M^{-1}: in the
// variables lam^ = M^{-1} lam the transposed solve is the forward sub-step
// with theta -> -theta.  Reverse sub-step (run by the line passes):
//     lam^_V = lam^ + seed,   seed = 2 dt V_probe / eps_probe (B sub-steps),
//     out    = 2 (I + theta X)^{-1} lam^_V - lam^     (FUND pass, pre = seed)
// and, since theta X V = V - 2W = U^{m+1} - U^m - h on the E rows,
//     dJ/d eps_i += -(1/2) (lam^_i + out_i) (U^{m+1} - U^m - h)_i.
// The input processing U^0 = 1/2 u^0 + dt/4 B u^0 adds
//     dJ/d eps_i += -lam^_i(U^0) (U^0 - u^0/2)_i.
// eps_r of a cell enters the Ex, Ey, Ez samples stored at its node index, so
// dJ/d eps_r(cell) = eps0 * (sum of the three).
#pragma once
#include <hip/hip_runtime.h>
#include "aux_kernels.hpp"

namespace fdtd {

// Design cells [i0, i0+bi) x [j0, j0+bj) x [k0, k0+bk); compact arrays are
// [bk][bj][bi], x fastest.
struct Box { int i0, j0, k0, bi, bj, bk; };

__device__ __forceinline__ long long box_node(const Box& b, const Dims& d, long long idx) {
    const int i = b.i0 + int(idx % b.bi);
    const int j = b.j0 + int((idx / b.bi) % b.bj);
    const int k = b.k0 + int(idx / ((long long)b.bi * b.bj));
    return (long long)k * d.plane + (long long)j * d.px + i;
}

// Record the E samples of the design cells of state s into rec ([3][nb], may
// be NULL) and the three E samples of the probe node into prb (FP64).  With J
// (a B sub-step of the forward sweep): J += dt |V|^2 for the probe field
// V = prb + prb_old (+ h_ez on Ez where the source sits on the probe node).
template <typename T>
__global__ void record_kernel(FieldPtrs<T> s, Dims d, Box b, T* rec, long long probe_off, double* prb,
                              const double* prb_old, double h_ez, double dt, double* J) {
    const long long nb = (long long)b.bi * b.bj * b.bk;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx == 0 && prb) {
        double acc = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double v = double(s.c[c][probe_off]);
            prb[c] = v;
            if (J) {
                const double w = v + prb_old[c] + (c == 2 ? h_ez : 0.0);
                acc += w * w;
            }
        }
        if (J) *J += dt * acc;
    }
    if (!rec || idx >= nb) return;
    const long long so = box_node(b, d, idx);
#pragma unroll
    for (int c = 0; c < 3; ++c) rec[c * nb + idx] = s.c[c][so];
}

// Gradient terms of one adjoint state lam, in FP64:
//     grad[idx] += scale sum_c lam_c (rec[m+1] - rec[m] - h)_c
// for m = m1, then m = m2 (either < 0: none), rec[m] = the record [3][nb] of
// sub-step state m, h = h1 (h2) on the Ez sample of box cell src_idx (-1:
// none).  With seed (one thread): the adjoint seed of a B sub-step,
// seed_c = 2 dt V_c / eps_abs, V = prb_new + prb_old (+ h_seed on Ez).
template <typename T>
__global__ void grad_acc_kernel(FieldPtrs<T> lam, Dims d, Box b, const T* rec, int m1, double h1, int m2,
                                double h2, long long src_idx, double scale, double* grad, double* seed,
                                const double* prb_old, const double* prb_new, double h_seed, const float* eps,
                                long long probe_off, double eps0, double dt) {
    const long long nb = (long long)b.bi * b.bj * b.bk;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (seed && idx == 0) {
        const double e = eps0 * double(eps[probe_off]);
        for (int c = 0; c < 3; ++c) {
            const double v = prb_new[c] + prb_old[c] + (c == 2 ? h_seed : 0.0);
            seed[c] = 2.0 * dt * v / e;
        }
    }
    if (idx >= nb) return;
    const long long so = box_node(b, d, idx);
    double l[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) l[c] = double(lam.c[c][so]);
    double g = grad[idx];
    for (int t = 0; t < 2; ++t) {
        const int m = t == 0 ? m1 : m2;
        if (m < 0) continue;
        const double h = t == 0 ? h1 : h2;
        const T* r = rec + (size_t)m * 3 * nb;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double dv = double(r[(3 + c) * nb + idx]) - double(r[c * nb + idx]) -
                              ((c == 2 && idx == src_idx) ? h : 0.0);
            acc += l[c] * dv;
        }
        g += scale * acc;
    }
    grad[idx] = g;
}

// Input-processing term: grad[idx] += scale * sum_c lam_c (U0 - u0/2)_c with
// U0 from the record rec0 and u0 the caller's initial field.
template <typename T>
__global__ void grad_link_kernel(FieldPtrs<T> lam, FieldPtrs<T> u0, Dims d, Box b, const T* rec0, double scale,
                                 double* grad) {
    const long long nb = (long long)b.bi * b.bj * b.bk;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nb) return;
    const int i = b.i0 + int(idx % b.bi);
    const int j = b.j0 + int((idx / b.bi) % b.bj);
    const int k = b.k0 + int(idx / ((long long)b.bi * b.bj));
    const long long so = (long long)k * d.plane + (long long)j * d.px + i;
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double u = double(phys<T>(u0, c, i, j, k, d));
        acc += double(lam.c[c][so]) * (double(rec0[c * nb + idx]) - 0.5 * u);
    }
    grad[idx] += scale * acc;
}

}  // namespace fdtd
