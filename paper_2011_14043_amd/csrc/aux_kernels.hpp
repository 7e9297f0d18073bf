// aux_kernels.hpp -- input/output processing and FP64 energy reductions.
//
// Caller layout: dense (nz+1, ny+1, nx+1) arrays.  State layout: the same
// nodes with rows padded to `px` elements (128-byte aligned rows).
#pragma once
#include <hip/hip_runtime.h>

namespace fdtd {

struct Dims {
    int nx, ny, nz;
    long long px, plane, comp;   // state: row pitch, plane pitch, component pitch
    long long cplane, ccomp;     // caller: plane pitch, component size (nx+1)(ny+1)(nz+1)
};

// Node (i, j, k) of flat node index idx (x fastest).  Node counts stay below
// 2^32 (at most 1025^3), so 32-bit division suffices.
struct Node { int i, j, k; };
__device__ __forceinline__ Node node_of(unsigned idx, const Dims& d) {
    const unsigned nx1 = unsigned(d.nx + 1), ny1 = unsigned(d.ny + 1);
    const unsigned t = idx / nx1;
    return Node{int(idx - t * nx1), int(t % ny1), int(t / ny1)};
}

// Is component c (0..5 = Ex Ey Ez Hx Hy Hz) dynamic / inside the box at node (i, j, k)?
__device__ __forceinline__ bool is_dynamic(int c, int i, int j, int k, const Dims& d) {
    switch (c) {
        case 0: return i < d.nx && j >= 1 && j < d.ny && k >= 1 && k < d.nz;
        case 1: return i >= 1 && i < d.nx && j < d.ny && k >= 1 && k < d.nz;
        case 2: return i >= 1 && i < d.nx && j >= 1 && j < d.ny && k < d.nz;
        case 3: return i >= 1 && i < d.nx && j < d.ny && k < d.nz;
        case 4: return i < d.nx && j >= 1 && j < d.ny && k < d.nz;
        default: return i < d.nx && j < d.ny && k >= 1 && k < d.nz;
    }
}
__device__ __forceinline__ bool in_extent(int c, int i, int j, int k, const Dims& d) {
    switch (c) {
        case 0: return i < d.nx;
        case 1: return j < d.ny;
        case 2: return k < d.nz;
        case 3: return j < d.ny && k < d.nz;
        case 4: return i < d.nx && k < d.nz;
        default: return i < d.nx && j < d.ny;
    }
}

template <typename T>
struct FieldPtrs { const T* c[6]; };
template <typename T>
struct FieldPtrsW { T* c[6]; };

// Physical sample of the caller's field: E is 0 off its dynamic set, H 0 off its extent.
template <typename T>
__device__ __forceinline__ T phys(const FieldPtrs<T>& f, int c, int i, int j, int k, const Dims& d) {
    if (i < 0 || j < 0 || k < 0 || i > d.nx || j > d.ny || k > d.nz) return T(0);
    const bool ok = (c < 3) ? is_dynamic(c, i, j, k, d) : in_extent(c, i, j, k, d);
    return ok ? f.c[c][(long long)k * d.cplane + (long long)j * (d.nx + 1) + i] : T(0);
}

struct AuxCoef {
    double eps0, mu0;
    double rmu0, rdx, rdy, rdz;   // 1/mu0, 1/dx, 1/dy, 1/dz (formed on the host)
    double link;                  // ADI: dt/4 (state = 1/2 u + dt/4 B u); 0 for a plain copy
};

// (B u)_c at a node, operator B of eq. (AMat) with Yee central differences.
// inv_eps = 1/(eps0 eps_r) at the node.
template <typename T, typename F>
__device__ __forceinline__ double apply_B(F get, int c, int i, int j, int k, double inv_eps, const AuxCoef& q) {
    switch (c) {
        case 0: return -inv_eps * (double(get(4, i, j, k)) - double(get(4, i, j, k - 1))) * q.rdz;   // -dHy/dz
        case 1: return -inv_eps * (double(get(5, i, j, k)) - double(get(5, i - 1, j, k))) * q.rdx;   // -dHz/dx
        case 2: return -inv_eps * (double(get(3, i, j, k)) - double(get(3, i, j - 1, k))) * q.rdy;   // -dHx/dy
        case 3: return -q.rmu0 * (double(get(2, i, j + 1, k)) - double(get(2, i, j, k))) * q.rdy;    // -dEz/dy
        case 4: return -q.rmu0 * (double(get(0, i, j, k + 1)) - double(get(0, i, j, k))) * q.rdz;    // -dEx/dz
        default: return -q.rmu0 * (double(get(1, i + 1, j, k)) - double(get(1, i, j, k))) * q.rdx;   // -dEy/dx
    }
}

// Input processing: caller fields -> state.  link != 0: the ADI/LOD1 link
// U = (1/2 I + dt/4 B) u (Sec. II-E); else U = u.  Non-dynamic E -> 0.
template <typename T>
__global__ void load_state_kernel(FieldPtrs<T> f, FieldPtrsW<T> s, const float* eps, Dims d, AuxCoef k_) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nn = (long long)(d.nx + 1) * (d.ny + 1) * (d.nz + 1);
    if (idx >= nn) return;
    const Node nd = node_of(unsigned(idx), d);
    const int i = nd.i, j = nd.j, k = nd.k;
    const long long so = (long long)k * d.plane + (long long)j * d.px + i;
    auto get = [&](int c, int ii, int jj, int kk) { return phys<T>(f, c, ii, jj, kk, d); };
    const double inv_eps = 1.0 / (k_.eps0 * double(eps[so]));
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const double u = double(get(c, i, j, k));
        double v = u;
        if (k_.link != 0.0) {
            const bool dyn = is_dynamic(c, i, j, k, d);
            const double bu = dyn ? apply_B<T>(get, c, i, j, k, inv_eps, k_) : 0.0;
            v = 0.5 * u + k_.link * bu;
        }
        s.c[c][so] = T(v);
    }
}

// Output processing: state (and, for ADI, the state before the last B
// sub-step) -> caller fields.  ADI: u = U_old + U_new (+ src_add at the Ez
// sample of the source, where the sub-step subtracted g/2), the v of the last
// B sub-step; else u = U.  Entries outside the box are not written.
template <typename T>
__global__ void store_state_kernel(FieldPtrs<T> s, FieldPtrs<T> s_old, FieldPtrsW<T> f, Dims d, int add_old,
                                   long long src_off, double src_add) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nn = (long long)(d.nx + 1) * (d.ny + 1) * (d.nz + 1);
    if (idx >= nn) return;
    const Node nd = node_of(unsigned(idx), d);
    const int i = nd.i, j = nd.j, k = nd.k;
    const long long so = (long long)k * d.plane + (long long)j * d.px + i;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        if (!in_extent(c, i, j, k, d)) continue;
        T v;
        if (c < 3 && !is_dynamic(c, i, j, k, d)) v = T(0);
        else if (add_old) {
            const double extra = (c == 2 && so == src_off) ? src_add : 0.0;
            v = T(double(s.c[c][so]) + double(s_old.c[c][so]) + extra);
        } else v = s.c[c][so];
        f.c[c][idx] = v;
    }
}

// Energy sum eps |E|^2 + mu |H|^2 over all samples of a state, FP64, first
// stage: one partial per block (fixed order => deterministic).
// link != 0 (original ADI): evaluated on (1/2 I + dt/4 B) u.
template <typename T>
__global__ void __launch_bounds__(256) energy_partial_kernel(FieldPtrs<T> s, const float* eps, Dims d, AuxCoef k_,
                                                             double* partial) {
    __shared__ double red[256];
    const long long nn = (long long)(d.nx + 1) * (d.ny + 1) * (d.nz + 1);
    double acc = 0.0;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < nn;
         idx += (long long)gridDim.x * blockDim.x) {
        const Node nd = node_of(unsigned(idx), d);
        const int i = nd.i, j = nd.j, k = nd.k;
        const long long so = (long long)k * d.plane + (long long)j * d.px + i;
        const double ew = k_.eps0 * double(eps[so]);
        if (k_.link == 0.0) {
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const double u = double(s.c[c][so]);
                acc += (c < 3 ? ew : k_.mu0) * u * u;
            }
        } else {
            auto get = [&](int c, int ii, int jj, int kk) -> T {
                if (ii < 0 || jj < 0 || kk < 0 || ii > d.nx || jj > d.ny || kk > d.nz) return T(0);
                return s.c[c][(long long)kk * d.plane + (long long)jj * d.px + ii];
            };
            const double inv_eps = 1.0 / ew;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const double u = double(get(c, i, j, k));
                const bool dyn = is_dynamic(c, i, j, k, d);
                const double bu = dyn ? apply_B<T>(get, c, i, j, k, inv_eps, k_) : 0.0;
                const double v = 0.5 * u + k_.link * bu;
                acc += (c < 3 ? ew : k_.mu0) * v * v;
            }
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) red[threadIdx.x] += red[threadIdx.x + s2];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Weighted squared distance of two field sets in the caller's layout, FP64,
// first stage: per block, sum eps |E_a - E_b|^2 + mu |H_a - H_b|^2 and
// sum eps |E_b|^2 + mu |H_b|^2 over the samples inside each component's
// extent (eps of the sample's owning node), into partial[b] and
// partial[gridDim.x + b] (fixed order => deterministic).
template <typename T>
__global__ void __launch_bounds__(256) diff_partial_kernel(FieldPtrs<T> fa, FieldPtrs<T> fb, const float* eps, Dims d,
                                                           AuxCoef k_, double* partial) {
    __shared__ double red[2][256];
    const long long nn = (long long)(d.nx + 1) * (d.ny + 1) * (d.nz + 1);
    double num = 0.0, den = 0.0;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < nn;
         idx += (long long)gridDim.x * blockDim.x) {
        const Node nd = node_of(unsigned(idx), d);
        const long long so = (long long)nd.k * d.plane + (long long)nd.j * d.px + nd.i;
        const double ew = k_.eps0 * double(eps[so]);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            if (!in_extent(c, nd.i, nd.j, nd.k, d)) continue;
            const double w = c < 3 ? ew : k_.mu0;
            const double vb = double(fb.c[c][idx]);
            const double dv = double(fa.c[c][idx]) - vb;
            num += w * dv * dv;
            den += w * vb * vb;
        }
    }
    red[0][threadIdx.x] = num;
    red[1][threadIdx.x] = den;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s2];
            red[1][threadIdx.x] += red[1][threadIdx.x + s2];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = red[0][0];
        partial[gridDim.x + blockIdx.x] = red[1][0];
    }
}

// Second stage: one thread sums the partials in index order.
__global__ void energy_final_kernel(const double* partial, int n, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < n; ++b) s += partial[b];
        *out = s;
    }
}

}  // namespace fdtd
