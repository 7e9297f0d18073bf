// aux_kernels.hpp -- input/output processing and FP64 energy reductions.
//
// Caller layout: dense (nz+1, ny+1, nx+1) arrays.  State layout: the same
// nodes with rows padded to `px` elements (128-byte aligned rows).
#pragma once
#include <hip/hip_runtime.h>

#include "line_solver.hpp"   // recip
#include "xcd.hpp"

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
    int fin_form;                 // energy of a fundamental ADI state in output form (static H
                                  // still hold 1/2 u, i.e. their link value)
    int order;                    // 4: the 4-point differences (apply_B4); else second order
    double wo;                    // order 4: outer weight of the 4-point difference
};

// (B u)_c at a node, operator B of eq. (AMat) with Yee central differences.
// inv_eps = 1/(eps0 eps_r), inv_mu = 1/(mu0 mu_r) at the node.
template <typename T, typename F>
__device__ __forceinline__ double apply_B(F get, int c, int i, int j, int k, double inv_eps, double inv_mu,
                                          const AuxCoef& q) {
    switch (c) {
        case 0: return -inv_eps * (double(get(4, i, j, k)) - double(get(4, i, j, k - 1))) * q.rdz;   // -dHy/dz
        case 1: return -inv_eps * (double(get(5, i, j, k)) - double(get(5, i - 1, j, k))) * q.rdx;   // -dHz/dx
        case 2: return -inv_eps * (double(get(3, i, j, k)) - double(get(3, i, j - 1, k))) * q.rdy;   // -dHx/dy
        case 3: return -inv_mu * (double(get(2, i, j + 1, k)) - double(get(2, i, j, k))) * q.rdy;    // -dEz/dy
        case 4: return -inv_mu * (double(get(0, i, j, k + 1)) - double(get(0, i, j, k))) * q.rdz;    // -dEx/dz
        default: return -inv_mu * (double(get(1, i + 1, j, k)) - double(get(1, i, j, k))) * q.rdx;   // -dEy/dx
    }
}

// (B u)_c at a node with the 4-point staggered differences, weights
// (-wo, -wi, wi, wo), wi = 1 - 3 wo (fourth order: (1, -27, 27, -1) / 24),
// over the four partner samples along the pair's axis
// (B pairs: Ex-Hy along z, Ey-Hz along x, Ez-Hx along y), folded across a PEC
// wall onto image samples: H even (stored index -1 -> 0, n -> n-1), E odd
// (position -p -> -E_p, n + p -> -E_{n-p}; E on a wall is 0).  `get` returns
// the physical sample (0 for E off its dynamic set).
template <typename F>
__device__ __forceinline__ double apply_B4(F get, int c, int i, int j, int k, double inv_eps, double inv_mu,
                                           const AuxCoef& q, const Dims& d) {
    const double wi = 1.0 - 3.0 * q.wo;
    const double w[4] = {-q.wo, -wi, wi, q.wo};
    const int axis = (c == 1 || c == 5) ? 0 : ((c == 2 || c == 3) ? 1 : 2);
    const int partner = c < 3 ? (c == 0 ? 4 : (c == 1 ? 5 : 3)) : (c == 3 ? 2 : (c == 4 ? 0 : 1));
    const int n = axis == 0 ? d.nx : (axis == 1 ? d.ny : d.nz);
    const int pos = axis == 0 ? i : (axis == 1 ? j : k);
    const double rh = axis == 0 ? q.rdx : (axis == 1 ? q.rdy : q.rdz);
    auto at = [&](int p) -> double {
        return double(axis == 0 ? get(partner, p, j, k) : (axis == 1 ? get(partner, i, p, k) : get(partner, i, j, p)));
    };
    double s = 0.0;
    if (c < 3) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            int qh = pos - 2 + t;
            qh = qh < 0 ? -1 - qh : (qh > n - 1 ? 2 * n - 1 - qh : qh);
            s += w[t] * at(qh);
        }
        return -inv_eps * s * rh;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        int pe = pos - 1 + t;
        double sg = 1.0;
        if (pe < 0) { pe = -pe; sg = -1.0; }
        else if (pe > n) { pe = 2 * n - pe; sg = -1.0; }
        s += sg * w[t] * at(pe);
    }
    return -inv_mu * s * rh;
}

// Input processing with the fourth-order differences: U = 1/2 u + link (B u)
// (the ADI link of Sec. II-E) in FP64, one thread per node (once per run).
// Non-dynamic E -> 0, static normal H -> 1/2 u.  The same values as
// apply_B4 over `phys` (same sums in the same order), with the index
// arithmetic and the set tests written out per component: a dynamic E's
// partner H samples (even images) are always inside the H extent, and a
// dynamic H's partner E is read only where it is dynamic (odd images, 0 on
// the walls).
template <typename T>
__global__ void load_state4_kernel(FieldPtrs<T> f, FieldPtrsW<T> s, const float* eps, const float* mu, Dims d,
                                   AuxCoef k_) {
    // caller offset of the node; consecutive blocks in one L2 (XCD-aware
    // order), so the neighbouring rows the y differences read were fetched there
    const long long co = (long long)xcd_remap(int(blockIdx.x), int(gridDim.x)) * blockDim.x + threadIdx.x;
    const long long nn = (long long)(d.nx + 1) * (d.ny + 1) * (d.nz + 1);
    if (co >= nn) return;
    const Node nd = node_of(unsigned(co), d);
    const int i = nd.i, j = nd.j, k = nd.k;
    const long long so = (long long)k * d.plane + (long long)j * d.px + i;
    const long long sx = 1, sy = d.nx + 1, sz = d.cplane;   // caller strides
    const double inv_eps = 1.0 / (k_.eps0 * double(eps[so]));
    const double inv_mu = 1.0 / (k_.mu0 * (mu ? double(mu[so]) : 1.0));
    const double wi = 1.0 - 3.0 * k_.wo;
    const double w[4] = {-k_.wo, -wi, wi, k_.wo};
    const bool ilo = i < d.nx, iin = i >= 1 && i < d.nx;
    const bool jlo = j < d.ny, jin = j >= 1 && j < d.ny;
    const bool klo = k < d.nz, kin = k >= 1 && k < d.nz;
    const bool dyn[6] = {ilo && jin && kin, iin && jlo && kin, iin && jin && klo,
                         iin && jlo && klo, ilo && jin && klo, ilo && jlo && kin};
    const bool ext[3] = {jlo && klo, ilo && klo, ilo && jlo};   // H extents
    // sum over the partner H along an axis: positions pos-2 .. pos+1, even images
    auto sum_h = [&](const T* h, int pos, int n, long long st) -> double {
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            int q = pos - 2 + t;
            q = q < 0 ? -1 - q : (q > n - 1 ? 2 * n - 1 - q : q);
            acc += w[t] * double(h[co + (long long)(q - pos) * st]);
        }
        return acc;
    };
    // sum over the partner E along an axis: positions pos-1 .. pos+2, odd
    // images; E at 0 and n (the walls) is 0, as is E whose other indices
    // leave its dynamic set (the caller passes e_ok = false then)
    auto sum_e = [&](const T* e, int pos, int n, long long st) -> double {
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            int q = pos - 1 + t;
            double sg = 1.0;
            if (q < 0) { q = -q; sg = -1.0; }
            else if (q > n) { q = 2 * n - q; sg = -1.0; }
            const double v = (q >= 1 && q <= n - 1) ? double(e[co + (long long)(q - pos) * st]) : 0.0;
            acc += sg * w[t] * v;
        }
        return acc;
    };
    const double L = k_.link;
    // E: U = 1/2 E - L/eps d_w H  (dynamic samples; else 0)
    s.c[0][so] = T(dyn[0] ? 0.5 * double(f.c[0][co]) + L * (-inv_eps * sum_h(f.c[4], k, d.nz, sz) * k_.rdz) : 0.0);
    s.c[1][so] = T(dyn[1] ? 0.5 * double(f.c[1][co]) + L * (-inv_eps * sum_h(f.c[5], i, d.nx, sx) * k_.rdx) : 0.0);
    s.c[2][so] = T(dyn[2] ? 0.5 * double(f.c[2][co]) + L * (-inv_eps * sum_h(f.c[3], j, d.ny, sy) * k_.rdy) : 0.0);
    // H: U = 1/2 H - L/mu d_w E  (dynamic samples; static H in the extent: 1/2 H; else 0)
    {
        const double u = ext[0] ? double(f.c[3][co]) : 0.0;
        s.c[3][so] = T(dyn[3] ? 0.5 * u + L * (-inv_mu * sum_e(f.c[2], j, d.ny, sy) * k_.rdy) : 0.5 * u);
    }
    {
        const double u = ext[1] ? double(f.c[4][co]) : 0.0;
        s.c[4][so] = T(dyn[4] ? 0.5 * u + L * (-inv_mu * sum_e(f.c[0], k, d.nz, sz) * k_.rdz) : 0.5 * u);
    }
    {
        const double u = ext[2] ? double(f.c[5][co]) : 0.0;
        s.c[5][so] = T(dyn[5] ? 0.5 * u + L * (-inv_mu * sum_e(f.c[1], i, d.nx, sx) * k_.rdx) : 0.5 * u);
    }
}

// Row kernels: block b covers the node row r = (j, k) = (r mod (ny+1), r div
// (ny+1)) and its threads loop over i, so j and k, the row offsets and the
// (j, k) parts of the extent and dynamic tests are uniform per block.  Rows
// are handed out XCD-aware (r = xcd_remap(b)): neighbouring rows, which share
// the input kernel's stencil rows and the caller layout's unaligned 128-byte
// lines, run in one L2.
constexpr int kRowThreads = 128;
inline dim3 row_grid(const Dims& d) { return dim3((unsigned)((d.ny + 1) * (d.nz + 1))); }

// Input processing: caller fields -> state.  link != 0: the ADI/LOD1 link
// U = (1/2 I + dt/4 B) u (Sec. II-E); else U = u.  Non-dynamic E -> 0.
// Row kernel (row_grid, kRowThreads threads), arithmetic in A (the solve
// precision: FP32 plans form the link in FP32, one more rounding than the
// stored value already has).  Each dynamic E takes the difference of its
// partner H across its own position, each dynamic H that of its partner E
// (B of eq. (AMat)); E off its dynamic set is 0, also where it enters a
// difference.  mu: mu_r in the state layout, or NULL (mu = mu0).
template <typename T, typename A = double>
__global__ void __launch_bounds__(kRowThreads) load_state_kernel(FieldPtrs<T> f, FieldPtrsW<T> s, const float* eps,
                                                                 const float* mu, Dims d, AuxCoef k_) {
    const int r = xcd_remap(int(blockIdx.x), int(gridDim.x));
    const int j = r % (d.ny + 1), k = r / (d.ny + 1);
    const long long nx1 = d.nx + 1;
    const long long srow = (long long)k * d.plane + (long long)j * d.px;
    const long long crow = (long long)k * d.cplane + (long long)j * nx1;
    const A L = A(k_.link), half = A(0.5);
    const A rdx = A(k_.rdx), rdy = A(k_.rdy), rdz = A(k_.rdz), cmu = L * A(k_.rmu0);
    // (j, k) parts of the dynamic sets (uniform per block)
    const bool jin = j >= 1 && j < d.ny, kin = k >= 1 && k < d.nz, jlo = j < d.ny, klo = k < d.nz;
    const bool jin1 = j + 1 < d.ny, kin1 = k + 1 < d.nz;   // E at j+1 (Ez) / k+1 (Ex) dynamic
    const T* Ex = f.c[0] + crow; const T* Ey = f.c[1] + crow; const T* Ez = f.c[2] + crow;
    const T* Hx = f.c[3] + crow; const T* Hy = f.c[4] + crow; const T* Hz = f.c[5] + crow;
    for (int i = int(threadIdx.x); i <= d.nx; i += kRowThreads) {
        const long long so = srow + i;
        const bool ilo = i < d.nx, iin = i >= 1 && i < d.nx, iin1 = i + 1 < d.nx;
        A u[6];
        u[0] = (ilo && jin && kin) ? A(Ex[i]) : A(0);
        u[1] = (iin && jlo && kin) ? A(Ey[i]) : A(0);
        u[2] = (iin && jin && klo) ? A(Ez[i]) : A(0);
        u[3] = (jlo && klo) ? A(Hx[i]) : A(0);
        u[4] = (ilo && klo) ? A(Hy[i]) : A(0);
        u[5] = (ilo && jlo) ? A(Hz[i]) : A(0);
        if (k_.link == 0.0) {
#pragma unroll
            for (int c = 0; c < 6; ++c) s.c[c][so] = T(u[c]);
            continue;
        }
        const A ce = L * recip(A(k_.eps0) * A(eps[so]));   // dt/4 / eps
        A v[6];
        // E: U = 1/2 E - (dt/4)/eps d_w H   (dynamic samples; else 0)
        v[0] = u[0];
        if (ilo && jin && kin) v[0] = fused(-ce, (A(Hy[i]) - A(Hy[i - d.cplane])) * rdz, half * u[0]);
        v[1] = u[1];
        if (iin && jlo && kin) v[1] = fused(-ce, (A(Hz[i]) - A(Hz[i - 1])) * rdx, half * u[1]);
        v[2] = u[2];
        if (iin && jin && klo) v[2] = fused(-ce, (A(Hx[i]) - A(Hx[i - nx1])) * rdy, half * u[2]);
        // H: U = 1/2 H - (dt/4)/mu d_w E   (dynamic samples; static normal H: 1/2 H)
        const A cm = mu ? cmu * recip(A(mu[so])) : cmu;
        v[3] = half * u[3];
        if (iin && jlo && klo) {
            const A ez1 = (iin && jin1) ? A(Ez[i + nx1]) : A(0);
            v[3] = fused(-cm, (ez1 - u[2]) * rdy, v[3]);
        }
        v[4] = half * u[4];
        if (ilo && jin && klo) {
            const A ex1 = (ilo && jin && kin1) ? A(Ex[i + d.cplane]) : A(0);
            v[4] = fused(-cm, (ex1 - u[0]) * rdz, v[4]);
        }
        v[5] = half * u[5];
        if (ilo && jlo && kin) {
            const A ey1 = (iin1 && jlo && kin) ? A(Ey[i + 1]) : A(0);
            v[5] = fused(-cm, (ey1 - u[1]) * rdx, v[5]);
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) s.c[c][so] = T(v[c]);
    }
}

// Output processing: state -> caller fields, one thread per node of a row
// (grid as load_state_kernel).  E off its dynamic set is 0; H normal to a wall
// (static) is doubled when static_twice (a fundamental ADI state keeps it as
// 1/2 u, the link value); entries outside the box are not written.  The state
// of a fundamental ADI run is in output form here (u = U_old + U_new, stored
// by the passes of the last B sub-step); the other schemes' state is u.
template <typename T>
__global__ void __launch_bounds__(kRowThreads) store_out_kernel(FieldPtrs<T> s, FieldPtrsW<T> f, Dims d,
                                                                int static_twice) {
    const int r = xcd_remap(int(blockIdx.x), int(gridDim.x));
    const int j = r % (d.ny + 1), k = r / (d.ny + 1);
    const long long srow = (long long)k * d.plane + (long long)j * d.px;
    const long long crow = (long long)k * d.cplane + (long long)j * (d.nx + 1);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const T* src = s.c[c] + srow;
        T* dst = f.c[c] + crow;
        for (int i = int(threadIdx.x); i <= d.nx; i += kRowThreads) {
            if (!in_extent(c, i, j, k, d)) continue;
            const bool dyn = is_dynamic(c, i, j, k, d);
            T v = src[i];
            if (c < 3) v = dyn ? v : T(0);
            else if (static_twice && !dyn) v = v + v;
            dst[i] = v;
        }
    }
}

// The samples of a run's output that no line pass writes, when the last
// passes of the run store straight into the caller's fields: E off its dynamic
// set (0) and static H (the state's value, doubled when static_twice), all on
// the walls.  Blocks [0, nface): one row on a y or z wall each (all i);
// the rest: one thread per row off those walls, for its two x-wall samples.
template <typename T>
__global__ void __launch_bounds__(kRowThreads) store_faces_kernel(FieldPtrs<T> s, FieldPtrsW<T> f, Dims d,
                                                                  int static_twice, int nface) {
    auto put = [&](int c, int i, int j, int k) {
        if (!in_extent(c, i, j, k, d) || is_dynamic(c, i, j, k, d)) return;
        T* dst = f.c[c] + (long long)k * d.cplane + (long long)j * (d.nx + 1) + i;
        if (c < 3) {
            *dst = T(0);
        } else {
            const T v = s.c[c][(long long)k * d.plane + (long long)j * d.px + i];
            *dst = static_twice ? T(v + v) : v;
        }
    };
    if (int(blockIdx.x) < nface) {
        int fb = int(blockIdx.x), j, k;
        if (fb < 2 * (d.nz + 1)) {
            j = (fb & 1) ? d.ny : 0;
            k = fb >> 1;
        } else {
            fb -= 2 * (d.nz + 1);
            k = (fb & 1) ? d.nz : 0;
            j = 1 + (fb >> 1);
        }
#pragma unroll
        for (int c = 0; c < 6; ++c)
            for (int i = int(threadIdx.x); i <= d.nx; i += kRowThreads) put(c, i, j, k);
        return;
    }
    const long long r = (long long)(int(blockIdx.x) - nface) * kRowThreads + threadIdx.x;
    if (r >= (long long)(d.ny + 1) * (d.nz + 1)) return;
    const int j = int(r % (d.ny + 1)), k = int(r / (d.ny + 1));
    if (j == 0 || j == d.ny || k == 0 || k == d.nz) return;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        put(c, 0, j, k);
        put(c, d.nx, j, k);
    }
}

// Output processing of the batched ADI: state (and the state before the last
// B sub-step) -> caller fields: u = U_old + U_new, the v of the last B
// sub-step (Sec. II-E link); else u = U.  Entries outside the box are not
// written.
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
// link != 0 (original ADI): evaluated on (1/2 I + dt/4 B) u.  mu: mu_r in
// the state layout, or NULL.
template <typename T>
__global__ void __launch_bounds__(256) energy_partial_kernel(FieldPtrs<T> s, const float* eps, const float* mu, Dims d,
                                                             AuxCoef k_, double* partial) {
    __shared__ double red[256];
    const long long nn = (long long)(d.nx + 1) * (d.ny + 1) * (d.nz + 1);
    double acc = 0.0;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < nn;
         idx += (long long)gridDim.x * blockDim.x) {
        const Node nd = node_of(unsigned(idx), d);
        const int i = nd.i, j = nd.j, k = nd.k;
        const long long so = (long long)k * d.plane + (long long)j * d.px + i;
        const double ew = k_.eps0 * double(eps[so]);
        const double mw = mu ? k_.mu0 * double(mu[so]) : k_.mu0;
        if (k_.link == 0.0) {
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const double u = double(s.c[c][so]);
                acc += (c < 3 ? ew : mw) * u * u;
            }
        } else {
            auto get = [&](int c, int ii, int jj, int kk) -> T {
                if (ii < 0 || jj < 0 || kk < 0 || ii > d.nx || jj > d.ny || kk > d.nz) return T(0);
                return s.c[c][(long long)kk * d.plane + (long long)jj * d.px + ii];
            };
            const double inv_eps = recip(ew), inv_mu = recip(mw);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const double u = double(get(c, i, j, k));
                const bool dyn = is_dynamic(c, i, j, k, d);
                const double bu = !dyn ? 0.0
                                  : (k_.order == 4 ? apply_B4(get, c, i, j, k, inv_eps, inv_mu, k_, d)
                                                   : apply_B<T>(get, c, i, j, k, inv_eps, inv_mu, k_));
                const double v = (k_.fin_form && c >= 3 && !dyn) ? u : 0.5 * u + k_.link * bu;
                acc += (c < 3 ? ew : mw) * v * v;
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
// extent (eps and mu of the sample's owning node; mu NULL: mu0), into
// partial[b] and partial[gridDim.x + b] (fixed order => deterministic).
template <typename T>
__global__ void __launch_bounds__(256) diff_partial_kernel(FieldPtrs<T> fa, FieldPtrs<T> fb, const float* eps,
                                                           const float* mu, Dims d, AuxCoef k_, double* partial) {
    __shared__ double red[2][256];
    const long long nn = (long long)(d.nx + 1) * (d.ny + 1) * (d.nz + 1);
    double num = 0.0, den = 0.0;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < nn;
         idx += (long long)gridDim.x * blockDim.x) {
        const Node nd = node_of(unsigned(idx), d);
        const long long so = (long long)nd.k * d.plane + (long long)nd.j * d.px + nd.i;
        const double ew = k_.eps0 * double(eps[so]);
        const double mw = mu ? k_.mu0 * double(mu[so]) : k_.mu0;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            if (!in_extent(c, nd.i, nd.j, nd.k, d)) continue;
            const double w = c < 3 ? ew : mw;
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
