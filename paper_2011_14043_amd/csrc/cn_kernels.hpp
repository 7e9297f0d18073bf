// cn_kernels.hpp -- Crank-Nicolson without factorization (Sec. II-E), device side
//
// The fundamental form of the classical scheme,
//     [1/2 I - dt/4 (A + B)] v = u^n ,   u^{n+1} = v - u^n ,
// is one global system per step.  With theta = dt/2, (A + B) u = (eps^-1 C_H(H),
// -mu^-1 C_E(E)), where C_H is the curl of H at the E samples and C_E the curl
// of E at the H samples (C_H = C_E^T on the PEC Yee grid), the H rows give
//     v_H = 2 u_H - theta mu^-1 C_E(v_E)
// and the E rows become the symmetric positive definite system
//     S v_E = eps v_E + theta^2 C_H(mu^-1 C_E(v_E)) = 2 eps u_E + 2 theta C_H(u_H),
// solved by conjugate gradients with the diagonal of S as preconditioner.  The
// initial guess v_E = 2 u_E has the residual 2 theta C_H(u_H - theta mu^-1
// C_E(u_E)), so no product with S is needed to start.  Finally
//     u_E^{n+1} = v_E - u_E^n ,   u_H^{n+1} = u_H^n - theta mu^-1 C_E(v_E).
//
// The product S p evaluates the curls of p at the H samples inside the kernel
// that forms S p, so an iteration moves p, q, x, r and eps_r only (and mu_r
// with a permeability map).
//
// Every kernel walks the nodes with a grid-stride loop over a fixed grid of
// kCnBlocks blocks, so the dot products (per-block partials, then one fixed-
// order tree per sum) are deterministic.  Non-dynamic E samples of the work
// vectors are kept at 0, which is what the curls of E read on the walls.
//
// Part of the single translation unit of libfdtd.so: included by fdtd.hip.
#pragma once

namespace fdtd {

constexpr int kCnBlocks = 1024;   // blocks of every grid-stride kernel (= partials per dot product)
constexpr int kCnThreads = 256;

// Scalars of the iteration in device memory: r.z of the current and the next
// iteration (by parity), p.q, r.r and b.b.
enum CnScalar { kRz0 = 0, kRz1 = 1, kPq = 2, kRr = 3, kBb = 4, kCnScalars = 8 };

struct CnArgs {
    Dims d;
    double rdx, rdy, rdz;       // reciprocal cell sizes
    double eps0, rmu0, theta;   // theta = dt / 2
    const float* eps;           // eps_r per node (state layout)
    const float* mu;            // mu_r per node (state layout), or NULL (mu = mu0)
    double* u[6];               // state: Ex Ey Ez Hx Hy Hz
    double* x[3];               // v_E
    double* r[3];               // residual
    double* p[3];               // search direction
    double* q[3];               // S p
    double* w[3];               // u_H - theta mu^-1 C_E(u_E) at the H samples (start of a step)
    double* partial;            // 3 x kCnBlocks
    double* scal;               // kCnScalars
    long long src_off;          // state offset of the source's Ez sample (< 0: none)
    double src_g;               // its term g of this step: eps g joins b and r at that sample
};

// Curl of H at E sample c (0..2) of node offset so; caller checks the E sample is dynamic.
__device__ __forceinline__ double curl_h(const double* const h[3], int c, long long so, const CnArgs& a) {
    const long long sy = a.d.px, sz = a.d.plane;
    switch (c) {
        case 0: return (h[2][so] - h[2][so - sy]) * a.rdy - (h[1][so] - h[1][so - sz]) * a.rdz;
        case 1: return (h[0][so] - h[0][so - sz]) * a.rdz - (h[2][so] - h[2][so - 1]) * a.rdx;
        default: return (h[1][so] - h[1][so - 1]) * a.rdx - (h[0][so] - h[0][so - sy]) * a.rdy;
    }
}

// Curl of E at H sample c (0..2 = Hx Hy Hz); caller checks the H sample is dynamic.
__device__ __forceinline__ double curl_e(const double* const e[3], int c, long long so, const CnArgs& a) {
    const long long sy = a.d.px, sz = a.d.plane;
    switch (c) {
        case 0: return (e[2][so + sy] - e[2][so]) * a.rdy - (e[1][so + sz] - e[1][so]) * a.rdz;
        case 1: return (e[0][so + sz] - e[0][so]) * a.rdz - (e[2][so + 1] - e[2][so]) * a.rdx;
        default: return (e[1][so + 1] - e[1][so]) * a.rdx - (e[0][so + sy] - e[0][so]) * a.rdy;
    }
}

// 1/mu of the H samples stored at node offset so (mu_r of that node).
__device__ __forceinline__ double rmu_at(const CnArgs& a, long long so) {
    return a.mu ? a.rmu0 / double(a.mu[so]) : a.rmu0;
}

// Diagonal of S at E sample c of node so: eps + theta^2 sum over the four H
// samples around it of mu^-1 / h^2 (h the spacing of the curl it enters).
__device__ __forceinline__ double s_diag(int c, long long so, double eps, const CnArgs& a) {
    const long long sy = a.d.px, sz = a.d.plane;
    const double m0 = rmu_at(a, so);
    double t;
    if (c == 0) t = (m0 + rmu_at(a, so - sy)) * a.rdy * a.rdy + (m0 + rmu_at(a, so - sz)) * a.rdz * a.rdz;
    else if (c == 1) t = (m0 + rmu_at(a, so - sz)) * a.rdz * a.rdz + (m0 + rmu_at(a, so - 1)) * a.rdx * a.rdx;
    else t = (m0 + rmu_at(a, so - 1)) * a.rdx * a.rdx + (m0 + rmu_at(a, so - sy)) * a.rdy * a.rdy;
    return eps + a.theta * a.theta * t;
}

// One partial per block for each of NV sums (fixed-order tree).
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double* partial) {
    __shared__ double red[NV][kCnThreads];
#pragma unroll
    for (int m = 0; m < NV; ++m) red[m][threadIdx.x] = v[m];
    __syncthreads();
    for (int s = kCnThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int m = 0; m < NV; ++m) red[m][threadIdx.x] += red[m][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int m = 0; m < NV; ++m) partial[m * kCnBlocks + blockIdx.x] = red[m][0];
}

#define CN_NODES(a)                                                                            \
    const long long nn_ = (long long)((a).d.nx + 1) * ((a).d.ny + 1) * ((a).d.nz + 1);         \
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < nn_;          \
         idx += (long long)gridDim.x * blockDim.x)

// w = u_H - theta mu^-1 C_E(u_E) at the dynamic H samples (0 elsewhere).
__global__ void __launch_bounds__(kCnThreads) cn_start_h_kernel(CnArgs a) {
    const double* e[3] = {a.u[0], a.u[1], a.u[2]};
    CN_NODES(a) {
        const Node nd = node_of(unsigned(idx), a.d);
        const long long so = (long long)nd.k * a.d.plane + (long long)nd.j * a.d.px + nd.i;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            a.w[c][so] = is_dynamic(3 + c, nd.i, nd.j, nd.k, a.d)
                             ? a.u[3 + c][so] - a.theta * rmu_at(a, so) * curl_e(e, c, so, a) : 0.0;
    }
}

// x = 2 u_E, r = 2 theta C_H(w), p = r / diag(S); sums r.z, r.r and b.b with
// b = 2 eps u_E + 2 theta C_H(u_H).  A source term g (added as g/2 to u_E in
// the fundamental form) adds eps g to b and r at its Ez sample.
__global__ void __launch_bounds__(kCnThreads) cn_start_e_kernel(CnArgs a) {
    const double* w[3] = {a.w[0], a.w[1], a.w[2]};
    const double* h[3] = {a.u[3], a.u[4], a.u[5]};
    double acc[3] = {0.0, 0.0, 0.0};
    CN_NODES(a) {
        const Node nd = node_of(unsigned(idx), a.d);
        const long long so = (long long)nd.k * a.d.plane + (long long)nd.j * a.d.px + nd.i;
        const double eps = a.eps0 * double(a.eps[so]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double xv = 0.0, rv = 0.0, pv = 0.0;
            if (is_dynamic(c, nd.i, nd.j, nd.k, a.d)) {
                const double ue = a.u[c][so];
                const double gs = (c == 2 && so == a.src_off) ? eps * a.src_g : 0.0;
                xv = 2.0 * ue;
                rv = 2.0 * a.theta * curl_h(w, c, so, a) + gs;
                pv = rv / s_diag(c, so, eps, a);
                const double bv = 2.0 * eps * ue + 2.0 * a.theta * curl_h(h, c, so, a) + gs;
                acc[0] += rv * pv;
                acc[1] += rv * rv;
                acc[2] += bv * bv;
            }
            a.x[c][so] = xv;
            a.r[c][so] = rv;
            a.p[c][so] = pv;
        }
    }
    block_partials<3>(acc, a.partial);
}

// q = S p = eps p + theta^2 C_H(mu^-1 C_E(p)); sum p.q.  The H values come from
// the curls of p at the four H samples around each E sample, formed here (the
// stencil reads of p hit the caches), so no H-side vector goes through HBM.
__global__ void __launch_bounds__(kCnThreads) cn_apply_kernel(CnArgs a) {
    const double* e[3] = {a.p[0], a.p[1], a.p[2]};
    const long long sy = a.d.px, sz = a.d.plane;
    const double t2 = a.theta * a.theta;
    // mu^-1 C_E(p) at the H sample of component c stored at node o
    auto mce = [&](int c, long long o) { return rmu_at(a, o) * curl_e(e, c, o, a); };
    double acc[1] = {0.0};
    CN_NODES(a) {
        const Node nd = node_of(unsigned(idx), a.d);
        const long long so = (long long)nd.k * a.d.plane + (long long)nd.j * a.d.px + nd.i;
        const double eps = a.eps0 * double(a.eps[so]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double qv = 0.0;
            if (is_dynamic(c, nd.i, nd.j, nd.k, a.d)) {
                // the four H samples around a dynamic E sample are dynamic
                double ch;
                if (c == 0)
                    ch = (mce(2, so) - mce(2, so - sy)) * a.rdy - (mce(1, so) - mce(1, so - sz)) * a.rdz;
                else if (c == 1)
                    ch = (mce(0, so) - mce(0, so - sz)) * a.rdz - (mce(2, so) - mce(2, so - 1)) * a.rdx;
                else
                    ch = (mce(1, so) - mce(1, so - 1)) * a.rdx - (mce(0, so) - mce(0, so - sy)) * a.rdy;
                const double pv = a.p[c][so];
                qv = eps * pv + t2 * ch;
                acc[0] += pv * qv;
            }
            a.q[c][so] = qv;
        }
    }
    block_partials<1>(acc, a.partial);
}

// alpha = r.z / p.q;  x += alpha p;  r -= alpha q;  sums r.z (next) and r.r.
__global__ void __launch_bounds__(kCnThreads) cn_update_kernel(CnArgs a, int par) {
    const double rz = a.scal[par], pq = a.scal[kPq];
    const double alpha = pq != 0.0 ? rz / pq : 0.0;
    double acc[2] = {0.0, 0.0};
    CN_NODES(a) {
        const Node nd = node_of(unsigned(idx), a.d);
        const long long so = (long long)nd.k * a.d.plane + (long long)nd.j * a.d.px + nd.i;
        const double eps = a.eps0 * double(a.eps[so]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (!is_dynamic(c, nd.i, nd.j, nd.k, a.d)) continue;
            a.x[c][so] += alpha * a.p[c][so];
            const double rv = a.r[c][so] - alpha * a.q[c][so];
            a.r[c][so] = rv;
            acc[0] += rv * rv / s_diag(c, so, eps, a);
            acc[1] += rv * rv;
        }
    }
    block_partials<2>(acc, a.partial);
}

// beta = r.z (new) / r.z (old);  p = r / diag(S) + beta p.
__global__ void __launch_bounds__(kCnThreads) cn_direction_kernel(CnArgs a, int par) {
    const double rz_new = a.scal[par], rz_old = a.scal[par ^ 1];
    const double beta = rz_old != 0.0 ? rz_new / rz_old : 0.0;
    CN_NODES(a) {
        const Node nd = node_of(unsigned(idx), a.d);
        const long long so = (long long)nd.k * a.d.plane + (long long)nd.j * a.d.px + nd.i;
        const double eps = a.eps0 * double(a.eps[so]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (!is_dynamic(c, nd.i, nd.j, nd.k, a.d)) continue;
            a.p[c][so] = a.r[c][so] / s_diag(c, so, eps, a) + beta * a.p[c][so];
        }
    }
}

// u_E = v_E - u_E;  u_H = u_H - theta mu^-1 C_E(v_E)  (dynamic samples only).
__global__ void __launch_bounds__(kCnThreads) cn_finish_kernel(CnArgs a) {
    const double* e[3] = {a.x[0], a.x[1], a.x[2]};
    CN_NODES(a) {
        const Node nd = node_of(unsigned(idx), a.d);
        const long long so = (long long)nd.k * a.d.plane + (long long)nd.j * a.d.px + nd.i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (is_dynamic(c, nd.i, nd.j, nd.k, a.d)) a.u[c][so] = a.x[c][so] - a.u[c][so];
            if (is_dynamic(3 + c, nd.i, nd.j, nd.k, a.d))
                a.u[3 + c][so] -= a.theta * rmu_at(a, so) * curl_e(e, c, so, a);
        }
    }
}

// ---------------------------------------------------------------------------
// Classical form, [I - theta (A + B)] u^{n+1} = [I + theta (A + B)] u^n + g:
// the right side f is formed explicitly, then the same elimination of H gives
//     S u_E^{n+1} = eps f_E + theta C_H(f_H),   u_H^{n+1} = f_H - theta mu^-1 C_E(u_E^{n+1}),
// solved from the guess u_E^{n+1} = u_E^n.
// ---------------------------------------------------------------------------

// f_E = u_E + theta eps^-1 C_H(u_H) (+ g at the source) into r; f_H =
// u_H - theta mu^-1 C_E(u_E) into w (0 off the dynamic samples).
__global__ void __launch_bounds__(kCnThreads) cn_conv_rhs_kernel(CnArgs a) {
    const double* e[3] = {a.u[0], a.u[1], a.u[2]};
    const double* h[3] = {a.u[3], a.u[4], a.u[5]};
    CN_NODES(a) {
        const Node nd = node_of(unsigned(idx), a.d);
        const long long so = (long long)nd.k * a.d.plane + (long long)nd.j * a.d.px + nd.i;
        const double eps = a.eps0 * double(a.eps[so]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double fe = 0.0;
            if (is_dynamic(c, nd.i, nd.j, nd.k, a.d)) {
                fe = a.u[c][so] + a.theta * curl_h(h, c, so, a) / eps;
                if (c == 2 && so == a.src_off) fe += a.src_g;
            }
            a.r[c][so] = fe;
            a.w[c][so] = is_dynamic(3 + c, nd.i, nd.j, nd.k, a.d)
                             ? a.u[3 + c][so] - a.theta * rmu_at(a, so) * curl_e(e, c, so, a) : 0.0;
        }
    }
}

// b = eps f_E + theta C_H(f_H) into r (f_E is read at the own node only);
// x = p = u_E; sum b.b.
__global__ void __launch_bounds__(kCnThreads) cn_conv_start_kernel(CnArgs a) {
    const double* w[3] = {a.w[0], a.w[1], a.w[2]};
    double acc[1] = {0.0};
    CN_NODES(a) {
        const Node nd = node_of(unsigned(idx), a.d);
        const long long so = (long long)nd.k * a.d.plane + (long long)nd.j * a.d.px + nd.i;
        const double eps = a.eps0 * double(a.eps[so]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double bv = 0.0, xv = 0.0;
            if (is_dynamic(c, nd.i, nd.j, nd.k, a.d)) {
                bv = eps * a.r[c][so] + a.theta * curl_h(w, c, so, a);
                xv = a.u[c][so];
                acc[0] += bv * bv;
            }
            a.r[c][so] = bv;
            a.x[c][so] = xv;
            a.p[c][so] = xv;
        }
    }
    block_partials<1>(acc, a.partial);
}

// r = b - S x (q holds S x), p = r / diag(S); sums r.z and r.r.
__global__ void __launch_bounds__(kCnThreads) cn_conv_resid_kernel(CnArgs a) {
    double acc[2] = {0.0, 0.0};
    CN_NODES(a) {
        const Node nd = node_of(unsigned(idx), a.d);
        const long long so = (long long)nd.k * a.d.plane + (long long)nd.j * a.d.px + nd.i;
        const double eps = a.eps0 * double(a.eps[so]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (!is_dynamic(c, nd.i, nd.j, nd.k, a.d)) continue;
            const double rv = a.r[c][so] - a.q[c][so];
            const double pv = rv / s_diag(c, so, eps, a);
            a.r[c][so] = rv;
            a.p[c][so] = pv;
            acc[0] += rv * pv;
            acc[1] += rv * rv;
        }
    }
    block_partials<2>(acc, a.partial);
}

// u_E = x;  u_H = f_H - theta mu^-1 C_E(x)  (dynamic samples only).
__global__ void __launch_bounds__(kCnThreads) cn_conv_finish_kernel(CnArgs a) {
    const double* e[3] = {a.x[0], a.x[1], a.x[2]};
    CN_NODES(a) {
        const Node nd = node_of(unsigned(idx), a.d);
        const long long so = (long long)nd.k * a.d.plane + (long long)nd.j * a.d.px + nd.i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (is_dynamic(c, nd.i, nd.j, nd.k, a.d)) a.u[c][so] = a.x[c][so];
            if (is_dynamic(3 + c, nd.i, nd.j, nd.k, a.d))
                a.u[3 + c][so] = a.w[c][so] - a.theta * rmu_at(a, so) * curl_e(e, c, so, a);
        }
    }
}

// scal[slot[m]] = sum of the m-th partial array (block m, fixed-order tree).
struct CnSlots { int s[3]; };
__global__ void __launch_bounds__(kCnThreads) cn_reduce_kernel(const double* partial, double* scal, CnSlots slots) {
    __shared__ double red[kCnThreads];
    const double* src = partial + (size_t)blockIdx.x * kCnBlocks;
    double v = 0.0;
    for (int b = threadIdx.x; b < kCnBlocks; b += kCnThreads) v += src[b];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kCnThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) scal[slots.s[blockIdx.x]] = red[0];
}

#undef CN_NODES

}  // namespace fdtd
