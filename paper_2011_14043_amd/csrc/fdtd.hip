// fdtd.hip -- plan, scheme tables and the C ABI of libfdtd.so.
//
// Schemes (Sec. II of the paper) as sequences of sub-steps; each sub-step
// applies the Cayley factor of A or B with half-span theta through three
// fused line passes, one per (E, H) pair of the operator (eq. (AMat)):
//   ADI  (fasterADI) in the link scaling of Sec. II-E:  A dt/2, B dt/2,
//        input U = (1/2 I + dt/4 B) u, output u = V of the last B sub-step;
//   LOD1 (fastLOD):   A dt/2, B dt/2;
//   SS2  (fastSS2):   A dt/4, B dt/2, A dt/4;
//   LOD2 (fastLOD2):  A dt/2, B dt/2 on the n+1/4 levels, input B dt/4
//        (fastLOD2i), output B -dt/4 (fastLOD2o).
// The original forms (clsADI), (orgLOD), (orgSS2), (orgLOD2) run the same
// sequences with the original right-hand sides (modes CONV_*).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fdtd.h"
#include "adjoint_kernels.hpp"
#include "aux_kernels.hpp"
#include "batch_kernels.hpp"
#include "pass_kernels.hpp"

namespace fdtd {

static constexpr double kEps0 = 8.8541878128e-12;
static constexpr double kMu0 = 1.25663706212e-6;

// Pairs of eq. (AMat): E component, H component, line axis, e axis, t axis, sign.
// Components 0..5 = Ex Ey Ez Hx Hy Hz; axes 0..2 = x y z.
struct PairDef { int ce, ch, w, e, t, s; };
static const PairDef kPairs[2][3] = {
    {{0, 5, 1, 0, 2, +1}, {1, 3, 2, 1, 0, +1}, {2, 4, 0, 2, 1, +1}},   // A
    {{0, 4, 2, 0, 1, -1}, {1, 5, 0, 1, 2, -1}, {2, 3, 1, 2, 0, -1}},   // B
};

struct SubStep { int op; double theta_frac; double t_frac; };
struct SchemeDef { int nsub; SubStep sub[3]; };
static const SchemeDef kSchemes[4] = {
    {2, {{0, 0.5, 0.25}, {1, 0.5, 0.75}, {0, 0, 0}}},          // ADI
    {2, {{0, 0.5, 0.25}, {1, 0.5, 0.75}, {0, 0, 0}}},          // LOD1
    {3, {{0, 0.25, 0.125}, {1, 0.5, 0.5}, {0, 0.25, 0.875}}},  // SS2
    {2, {{0, 0.5, 0.5}, {1, 0.5, 1.0}, {0, 0, 0}}},            // LOD2
};

// Kernel configuration of the passes along one line axis.
//   x lines: M (slots per lane), wpb (waves per block), remap
//   y/z lines: M (slots per thread), TX (x positions per block),
//              NT (block-size bound of the instantiation), remap
struct KCfg { int M, TX, NT, wpb, remap; };

// Instantiated y/z-line variants {M, TX, NT} by solve precision.
static const int kYzF32[][3] = {{16, 32, 1024}, {16, 16, 512}, {8, 16, 1024}, {32, 16, 512}, {8, 32, 512}};
static const int kYzF64[][3] = {{16, 16, 512}, {8, 8, 512}, {8, 16, 1024}};

struct Timing {
    int per_launch = 0;           // 0: off; k >= 1: every launch of every k-th main-loop step
    hipEvent_t main0 = nullptr, main1 = nullptr;
    std::vector<hipEvent_t> ev;   // pairs
    std::vector<int> fam;         // family of each pair (0 = yz lines, 1 = x lines)
    size_t used = 0;
};

// Batch plans (fdtd_plan_batch): one pass of every grid of the batch per
// launch.  For each (operator, pair, theta) the batch keeps a device table of
// the grids' pass arguments and a work list of (grid, block) items.
struct BatchPass {
    int op = 0, k = 0;
    double frac = 0.0;        // theta = frac * dt of each grid
    void* tab = nullptr;      // device PassArgs<T, S>[ngrids]
    void* items = nullptr;    // device int2[nitems]
    int nitems = 0;
    int Pmax = 1;             // y/z lines: largest chunk count (block = TX * Pmax)
    size_t lds = 0;           // y/z lines: dynamic LDS per block
};
struct Batch {
    std::vector<fdtd_plan_s*> subs;
    bool mat = false;         // every grid has a material index
    std::vector<BatchPass> passes;
    hipStream_t cap = nullptr;        // private stream for graph capture
    hipStream_t fork[2] = {nullptr, nullptr};   // capture branches: the three pair passes of a
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};   // sub-step are independent and run side by side
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;    // time steps of the main iteration
    // A batch larger than kGroupBytes is split into groups of consecutive
    // grids, each a batch plan of its own (it owns its grids); the plan then
    // only delegates, and a run steps one group after the other.
    std::vector<fdtd_plan_s*> groups;
    std::vector<int> first;           // first grid of each group
};

}  // namespace fdtd

struct fdtd_plan_s {
    fdtd_desc d;
    hipStream_t stream;
    int device;
    fdtd::Dims dims;
    size_t esz;
    void* state = nullptr;    // 6 (or 12 for original ADI) arrays, padded layout
    void* snap = nullptr;     // ADI: state before the last B sub-step
    float* eps = nullptr;     // node layout, padded
    unsigned char* mat = nullptr;   // material index per node (if <= 256 distinct eps_r)
    float* mat_eps = nullptr;       // eps_r per material
    int nmat = 0;
    double* partial = nullptr;
    int npartial = 0;
    double* energy_dev = nullptr;
    int energy_cap = 0;
    void* gbuf = nullptr;     // adjoint: checkpoints, records, adjoint state (grown on demand)
    size_t gcap = 0;
    long long step = 0;
    fdtd::Timing tm;
    fdtd::KCfg cfg[3];        // per line axis x, y, z
    int tuned = 0;
    int refine = 0;           // FDTD_F32_REFINE: fundamental passes refine each solve once
    double last_main_ms = 0.0;
    double fam_ms[2] = {0, 0};
    int fam_n[2] = {0, 0};
    fdtd::Batch* batch = nullptr;   // batch plan: the grids and their tables
    unsigned magic = 0xFD7DFD7Du;
};

namespace fdtd {

static fdtd_status from_hip(hipError_t e) {
    if (e == hipSuccess) return FDTD_OK;
    if (e == hipErrorOutOfMemory) return FDTD_ENOMEM;
    return FDTD_EDEVICE;
}
#define HIPCHK(x)                                       \
    do {                                                \
        hipError_t e_ = (x);                            \
        if (e_ != hipSuccess) return from_hip(e_);      \
    } while (0)

static int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

template <typename T>
static T* comp_ptr(fdtd_plan_s* p, int set, int c) {
    return reinterpret_cast<T*>(p->state) + (size_t)(set * 6 + c) * p->dims.comp;
}

static long long axis_stride(const Dims& d, int ax) { return ax == 0 ? 1 : (ax == 1 ? d.px : d.plane); }
static int axis_cells(const Dims& d, int ax) { return ax == 0 ? d.nx : (ax == 1 ? d.ny : d.nz); }
static double axis_h(const fdtd_desc& d, int ax) { return ax == 0 ? d.dx : (ax == 1 ? d.dy : d.dz); }

// ---------------------------------------------------------------------------
// kernel launch helpers (variants: full lines, material-index eps_r)
// ---------------------------------------------------------------------------
template <typename T, typename S, int M, int MODE>
static void launch_x(bool full, bool mat, dim3 g, dim3 b, hipStream_t st, const PassArgs<T, S>& a) {
    if (full) {
        if (mat) hipLaunchKernelGGL((pass_x_kernel<T, S, M, MODE, true, true>), g, b, 0, st, a);
        else hipLaunchKernelGGL((pass_x_kernel<T, S, M, MODE, true, false>), g, b, 0, st, a);
    } else {
        if (mat) hipLaunchKernelGGL((pass_x_kernel<T, S, M, MODE, false, true>), g, b, 0, st, a);
        else hipLaunchKernelGGL((pass_x_kernel<T, S, M, MODE, false, false>), g, b, 0, st, a);
    }
}
// Refined solves are built for FP32: x lines with 8-slot chunks, y/z lines
// with 8- or 16-slot chunks.
template <typename S, int M> struct HasRefX { static constexpr bool v = sizeof(S) == 4 && M == 8; };
template <typename S, int M> struct HasRefYZ { static constexpr bool v = sizeof(S) == 4 && (M == 8 || M == 16); };
template <typename T, typename S, int M>
static bool launch_x_mode(int mode, bool full, bool mat, dim3 g, dim3 b, hipStream_t st, const PassArgs<T, S>& a) {
    if (mode == FUND) launch_x<T, S, M, FUND>(full, mat, g, b, st, a);
    else if (mode == CONV_LOD) launch_x<T, S, M, CONV_LOD>(full, mat, g, b, st, a);
    else if (mode == CONV_ADI) launch_x<T, S, M, CONV_ADI>(full, mat, g, b, st, a);
    else if constexpr (HasRefX<S, M>::v) launch_x<T, S, M, FUND_REF>(full, mat, g, b, st, a);
    else return false;
    return true;
}
template <typename T, typename S, int M, int TX, int NT, int MODE>
static void launch_yz(bool full, bool mat, dim3 g, dim3 b, size_t lds, hipStream_t st, const PassArgs<T, S>& a) {
    if (full) {
        if (mat) hipLaunchKernelGGL((pass_yz_kernel<T, S, M, MODE, TX, NT, true, true>), g, b, lds, st, a);
        else hipLaunchKernelGGL((pass_yz_kernel<T, S, M, MODE, TX, NT, true, false>), g, b, lds, st, a);
    } else {
        if (mat) hipLaunchKernelGGL((pass_yz_kernel<T, S, M, MODE, TX, NT, false, true>), g, b, lds, st, a);
        else hipLaunchKernelGGL((pass_yz_kernel<T, S, M, MODE, TX, NT, false, false>), g, b, lds, st, a);
    }
}
template <typename T, typename S, int M, int TX, int NT>
static bool launch_yz_mode(int mode, bool full, bool mat, dim3 g, dim3 b, size_t lds, hipStream_t st,
                           const PassArgs<T, S>& a) {
    if (mode == FUND) launch_yz<T, S, M, TX, NT, FUND>(full, mat, g, b, lds, st, a);
    else if (mode == CONV_LOD) launch_yz<T, S, M, TX, NT, CONV_LOD>(full, mat, g, b, lds, st, a);
    else if (mode == CONV_ADI) launch_yz<T, S, M, TX, NT, CONV_ADI>(full, mat, g, b, lds, st, a);
    else if constexpr (HasRefYZ<S, M>::v) launch_yz<T, S, M, TX, NT, FUND_REF>(full, mat, g, b, lds, st, a);
    else return false;
    return true;
}

// ---------------------------------------------------------------------------
// one line pass
// ---------------------------------------------------------------------------
// Right-hand-side injection of one sub-step at the E samples stored at node
// (i, j, k): component c (bit c of mask) gets `pre` added to its state before
// the solve (FUND; the conventional forms add it to the right-hand side) and
// `post` subtracted from the FUND output.  pre_dev (device, 3 doubles),
// if set, supplies the pre values instead.
struct Inject {
    int i = 0, j = 0, k = 0;
    unsigned mask = 0;
    double pre[3] = {0, 0, 0}, post[3] = {0, 0, 0};
    const double* pre_dev = nullptr;
};

// The physical source of a sub-step with source term g (fdtd_source).
static Inject source_inject(const fdtd_plan_s* p, const fdtd_source* src, double g, int mode) {
    Inject in;
    if (!src || g == 0.0) return in;
    in.i = src->i; in.j = src->j; in.k = src->k;
    in.mask = 4u;   // Ez
    if (mode == FUND) {
        in.pre[2] = 0.5 * g;
        in.post[2] = (p->d.scheme == FDTD_ADI) ? 0.5 * g : 0.0;
    } else {
        in.pre[2] = g;
    }
    return in;
}

// Coefficients of the input/output and energy kernels (reciprocals formed here).
static AuxCoef aux_coef(const fdtd_desc& d, double link) {
    return AuxCoef{kEps0, kMu0, 1.0 / kMu0, 1.0 / d.dx, 1.0 / d.dy, 1.0 / d.dz, link};
}

template <typename T>
static T* set_ptr(fdtd_plan_s* p, int set) {
    return reinterpret_cast<T*>(p->state) + (size_t)set * 6 * p->dims.comp;
}

// Launch shape of one pass.
struct PassShape {
    int w = 0;            // line axis
    dim3 grid, block;
    size_t lds = 0;
    bool full = false;    // every line fills its P*M slots exactly
    bool mat = false;     // material-index variant
};

// Arguments and launch shape of the pass of pair k of operator op (half-span
// theta, mode) from state set `set_in` to `set_out` of plan p, with the plan's
// kernel configuration for the line axis.
template <typename T, typename S>
static void build_pass(fdtd_plan_s* p, int op, int k, double theta, int mode, T* set_in, T* set_out,
                       const Inject* inj, PassArgs<T, S>& a, PassShape& sh) {
    const PairDef& pd = kPairs[op][k];
    const Dims& d = p->dims;
    std::memset(&a, 0, sizeof(a));
    const size_t cs = (size_t)d.comp;
    a.Ein = set_in + pd.ce * cs;
    a.Hin = set_in + pd.ch * cs;
    a.Eout = set_out + pd.ce * cs;
    a.Hout = set_out + pd.ch * cs;
    a.eps = p->eps;
    a.mat = p->mat;
    a.mat_eps = p->mat_eps;
    a.nmat = p->nmat;
    sh.mat = p->mat != nullptr;
    sh.w = pd.w;
    a.sw = axis_stride(d, pd.w);
    a.n_w = axis_cells(d, pd.w);
    const double h = axis_h(p->d, pd.w);
    const double mu = kMu0;
    const double s = double(pd.s);
    a.Ks = kEps0 * mu * h * h / (theta * theta);
    const double qd = s * theta / (mu * h);
    double kap = (mode == CONV_ADI) ? s * mu * h / theta : 2.0 * s * mu * h / theta;
    a.q = S(qd);
    a.kap_hi = S(kap);
    a.kap_lo = (sizeof(S) == 4) ? S(kap - double(S(kap))) : S(0);
    if (mode == CONV_ADI) {
        // Y = the other operator; H2 = partner of E in Y, E3 = partner of H in Y
        const int yo = 1 - op;
        int h2 = -1, e3 = -1;
        for (int m = 0; m < 3; ++m) {
            if (kPairs[yo][m].ce == pd.ce) h2 = kPairs[yo][m].ch;
            if (kPairs[yo][m].ch == pd.ch) e3 = kPairs[yo][m].ce;
        }
        const double sy = (op == 0) ? -1.0 : 1.0;
        const double ht = axis_h(p->d, pd.t), he = axis_h(p->d, pd.e);
        a.H2 = set_in + h2 * cs;
        a.E3 = set_in + e3 * cs;
        a.s_t = axis_stride(d, pd.t);
        a.s_e = axis_stride(d, pd.e);
        a.cH2 = S(sy * h * h * mu / (ht * theta));
        a.hE3 = S(sy * theta / (mu * he));
    }
    a.comp = d.comp;
    a.src_a = a.src_b = a.src_j = -1;
    int src_idx[3] = {0, 0, 0};
    const bool has_src = inj && ((inj->mask >> pd.ce) & 1u);
    if (has_src) {
        src_idx[0] = inj->i; src_idx[1] = inj->j; src_idx[2] = inj->k;
        a.src_pre = S(inj->pre[pd.ce]);
        a.src_post = S(inj->post[pd.ce]);
        a.src_pre_dev = inj->pre_dev ? inj->pre_dev + pd.ce : nullptr;
    }
    const int ne = axis_cells(d, pd.e), nt = axis_cells(d, pd.t);
    const KCfg& cf = p->cfg[pd.w];
    a.remap = cf.remap;
    if (pd.w == 0) {
        // x lines: a = y (fast), b = z (slow), so that line order is memory
        // order and every line of a wave lies after the wave's first line.
        // The e axis starts at 0, the t axis at 1 (t = 0 is a PEC wall plane).
        a.sa = axis_stride(d, 1);
        a.sb = axis_stride(d, 2);
        if (pd.e == 1) { a.a_lo = 0; a.na = d.ny; a.b_lo = 1; a.nb = d.nz - 1; }
        else { a.a_lo = 1; a.na = d.ny - 1; a.b_lo = 0; a.nb = d.nz; }
        if (has_src) { a.src_a = src_idx[1]; a.src_b = src_idx[2]; a.src_j = src_idx[0]; }
        const int M = cf.M;
        a.P = next_pow2((a.n_w + M - 1) / M);
        const long long nlines = (long long)a.na * a.nb;
        const long long lines_per_block = (long long)cf.wpb * (64 / a.P);
        a.nblk = (int)((nlines + lines_per_block - 1) / lines_per_block);
        sh.grid = dim3((unsigned)a.nblk);
        sh.block = dim3(64 * cf.wpb);
        sh.lds = 0;
    } else {
        // y/z lines: a = x axis (lanes), b = the other transverse axis
        const int other = (pd.e == 0) ? pd.t : pd.e;
        a.sa = 1;
        a.sb = axis_stride(d, other);
        if (pd.e == 0) { a.a_lo = 0; a.na = d.nx; a.b_lo = 1; a.nb = nt - 1; }
        else { a.a_lo = 1; a.na = d.nx - 1; a.b_lo = 0; a.nb = ne; }
        if (has_src) { a.src_a = src_idx[0]; a.src_b = src_idx[other]; a.src_j = src_idx[pd.w]; }
        const int M = cf.M, TX = cf.TX;
        a.P = next_pow2((a.n_w + M - 1) / M);
        a.ntx = (a.a_lo + a.na + TX - 1) / TX;
        a.nblk = a.ntx * a.nb;
        sh.block = dim3(TX * a.P);
        sh.grid = dim3((unsigned)a.nblk);
        sh.lds = (size_t)9 * a.P * (TX + 1) * sizeof(S);
    }
    sh.full = a.P * cf.M == a.n_w;
}

template <typename T, typename S>
static fdtd_status launch_pass(fdtd_plan_s* p, int op, int k, double theta, int mode, T* set_in, T* set_out,
                               const Inject* inj, bool timed) {
    PassArgs<T, S> a;
    PassShape sh;
    build_pass<T, S>(p, op, k, theta, mode, set_in, set_out, inj, a, sh);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        Timing& tm = p->tm;
        if (tm.used + 2 > tm.ev.size()) {
            for (int m = 0; m < 64; ++m) {
                hipEvent_t ev;
                HIPCHK(hipEventCreate(&ev));
                tm.ev.push_back(ev);
            }
        }
        e0 = tm.ev[tm.used];
        e1 = tm.ev[tm.used + 1];
        tm.fam.push_back(sh.w == 0 ? 1 : 0);
        tm.used += 2;
        HIPCHK(hipEventRecord(e0, p->stream));
    }
    const KCfg& cf = p->cfg[sh.w];
    const int kmode = (mode == FUND && p->refine) ? FUND_REF : mode;
    bool built = true;
    if (sh.w == 0) {
        if (cf.M == 8) built = launch_x_mode<T, S, 8>(kmode, sh.full, sh.mat, sh.grid, sh.block, p->stream, a);
        else built = launch_x_mode<T, S, 16>(kmode, sh.full, sh.mat, sh.grid, sh.block, p->stream, a);
    } else {
        const int M = cf.M, TX = cf.TX, NT = cf.NT;
        const size_t lds = kmode == FUND_REF ? sh.lds / 9 * 13 : sh.lds;   // refined: second exchange areas
#define CASE_YZ(MM, TT, NN)                                                                                    \
    if (M == MM && TX == TT && NT == NN) {                                                                     \
        built = launch_yz_mode<T, S, MM, TT, NN>(kmode, sh.full, sh.mat, sh.grid, sh.block, lds, p->stream, a); \
    } else
        if constexpr (sizeof(S) == 4) {
            CASE_YZ(16, 32, 1024) CASE_YZ(16, 16, 512) CASE_YZ(8, 16, 1024) CASE_YZ(32, 16, 512) CASE_YZ(8, 32, 512)
            return FDTD_EUNSUPPORTED;
        } else {
            CASE_YZ(16, 16, 512) CASE_YZ(8, 8, 512) CASE_YZ(8, 16, 1024) return FDTD_EUNSUPPORTED;
        }
#undef CASE_YZ
    }
    if (!built) return FDTD_EUNSUPPORTED;
    HIPCHK(hipGetLastError());
    if (timed) HIPCHK(hipEventRecord(e1, p->stream));
    return FDTD_OK;
}

template <typename T, typename S>
static fdtd_status substep(fdtd_plan_s* p, int op, double theta, int mode, int& cur, const Inject* inj,
                           bool timed) {
    const int out = (mode == CONV_ADI) ? 1 - cur : cur;
    for (int k = 0; k < 3; ++k) {
        fdtd_status st = launch_pass<T, S>(p, op, k, theta, mode, set_ptr<T>(p, cur), set_ptr<T>(p, out), inj, timed);
        if (st != FDTD_OK) return st;
    }
    cur = out;
    return FDTD_OK;
}

// ---------------------------------------------------------------------------
// kernel configurations and the autotuner
// ---------------------------------------------------------------------------
static bool cfg_valid(const fdtd_plan_s* p, int axis, const KCfg& c) {
    const int n = axis_cells(p->dims, axis);
    if (c.remap != 0 && c.remap != 1) return false;
    if (p->refine && (axis == 0 ? c.M != 8 : c.M > 16)) return false;   // refined solves built
    if (axis == 0) {
        if (c.M != 8 && c.M != 16) return false;
        if (c.wpb < 1 || c.wpb > 4) return false;
        return next_pow2((n + c.M - 1) / c.M) <= 64;
    }
    // FP64 conventional ADI (two extra arrays per pass) exceeds the register
    // budget of the 1024-thread FP64 variant
    if (p->d.dtype == FDTD_F64 && p->d.scheme == FDTD_ADI && p->d.form == FDTD_CONVENTIONAL && c.NT == 1024)
        return false;
    bool inst = false;
    if (p->d.dtype == FDTD_F32) {
        for (const auto& v : kYzF32) inst = inst || (v[0] == c.M && v[1] == c.TX && v[2] == c.NT);
    } else {
        for (const auto& v : kYzF64) inst = inst || (v[0] == c.M && v[1] == c.TX && v[2] == c.NT);
    }
    if (!inst) return false;
    const int P = next_pow2((n + c.M - 1) / c.M);
    return P <= 64 && c.TX * P <= c.NT;
}

// Candidates: y/z lines only in the XCD-aware order (the plain order reads
// the z pass's material lines once per XCD; the time difference is noise,
// the traffic is not); x lines in both orders.
static std::vector<KCfg> cfg_candidates(const fdtd_plan_s* p, int axis) {
    std::vector<KCfg> out;
    for (int remap = 1; remap >= (axis == 0 ? 0 : 1); --remap) {
        if (axis == 0) {
            for (int M : {8, 16})
                for (int wpb : {4, 2, 1}) {
                    KCfg c{M, 0, 0, wpb, remap};
                    if (cfg_valid(p, axis, c)) out.push_back(c);
                }
        } else if (p->d.dtype == FDTD_F32) {
            for (const auto& v : kYzF32) {
                KCfg c{v[0], v[1], v[2], 0, remap};
                if (cfg_valid(p, axis, c)) out.push_back(c);
            }
        } else {
            for (const auto& v : kYzF64) {
                KCfg c{v[0], v[1], v[2], 0, remap};
                if (cfg_valid(p, axis, c)) out.push_back(c);
            }
        }
    }
    return out;
}

// Untuned default: the first valid entry of the preference order.
static void default_cfg(fdtd_plan_s* p) {
    for (int axis = 0; axis < 3; ++axis) {
        std::vector<KCfg> pref;
        if (axis == 0) {
            pref = {{8, 0, 0, 4, 1}, {16, 0, 0, 4, 1}};
        } else if (p->d.dtype == FDTD_F32) {
            pref = {{16, 16, 512, 0, 1}, {16, 32, 1024, 0, 1}, {32, 16, 512, 0, 1}, {8, 16, 1024, 0, 1},
                    {8, 32, 512, 0, 1}};
        } else {
            pref = {{16, 16, 512, 0, 1}, {8, 8, 512, 0, 1}};
        }
        for (const KCfg& c : pref)
            if (cfg_valid(p, axis, c)) { p->cfg[axis] = c; break; }
    }
}

template <typename T, typename S>
static fdtd_status autotune_impl(fdtd_plan_s* p, int reps, double* best_ms) {
    const bool adi = p->d.scheme == FDTD_ADI, conv = p->d.form == FDTD_CONVENTIONAL;
    const int mode = conv ? (adi ? CONV_ADI : CONV_LOD) : FUND;
    const double theta = 0.5 * p->d.dt;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    fdtd_status st = FDTD_OK;
    for (int axis = 0; axis < 3 && st == FDTD_OK; ++axis) {
        int k = 0;
        while (kPairs[0][k].w != axis) ++k;
        const std::vector<KCfg> cand = cfg_candidates(p, axis);
        KCfg best = p->cfg[axis];
        float tbest = 1e30f;
        // two rounds over the candidates; each keeps its best time (clock
        // and neighbour noise only ever add time)
        for (int round = 0; round < 2 * (int)cand.size() && st == FDTD_OK; ++round) {
            const KCfg& c = cand[round % cand.size()];
            p->cfg[axis] = c;
            T* s0 = set_ptr<T>(p, 0);
            T* s1 = set_ptr<T>(p, conv && adi ? 1 : 0);
            st = launch_pass<T, S>(p, 0, k, theta, mode, s0, s1, nullptr, false);
            if (st != FDTD_OK) break;
            if (hipEventRecord(e0, p->stream) != hipSuccess) { st = FDTD_EDEVICE; break; }
            for (int r = 0; r < reps && st == FDTD_OK; ++r)
                st = launch_pass<T, S>(p, 0, k, theta, mode, s0, s1, nullptr, false);
            if (st != FDTD_OK) break;
            if (hipEventRecord(e1, p->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                st = FDTD_EDEVICE;
                break;
            }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < tbest) { tbest = ms; best = c; }
        }
        p->cfg[axis] = best;
        if (best_ms) best_ms[axis] = tbest / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == FDTD_OK) p->tuned = 1;
    return st;
}

// Text cache of tuned configurations: one line per key
//   {"key": "<nx>,<ny>,<nz>,<dtype>,<scheme>,<form>", "cfg": [[M,TX,NT,wpb,remap],[...],[...]]}
static std::string tune_key(const fdtd_plan_s* p) {
    char b[160];
    std::snprintf(b, sizeof(b), "%d,%d,%d,%d,%d,%d", p->d.nx, p->d.ny, p->d.nz, p->d.dtype, p->d.scheme, p->d.form);
    return b;
}

static bool tune_cache_lookup(fdtd_plan_s* p, const char* path) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    const std::string key = tune_key(p);
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        char k[160];
        KCfg c[3];
        if (std::sscanf(line, " {\"key\": \"%159[^\"]\", \"cfg\": [[%d,%d,%d,%d,%d],[%d,%d,%d,%d,%d],[%d,%d,%d,%d,%d]]}", k,
                        &c[0].M, &c[0].TX, &c[0].NT, &c[0].wpb, &c[0].remap, &c[1].M, &c[1].TX, &c[1].NT, &c[1].wpb,
                        &c[1].remap, &c[2].M, &c[2].TX, &c[2].NT, &c[2].wpb, &c[2].remap) != 16)
            continue;
        if (key != k) continue;
        if (cfg_valid(p, 0, c[0]) && cfg_valid(p, 1, c[1]) && cfg_valid(p, 2, c[2])) {
            for (int a = 0; a < 3; ++a) p->cfg[a] = c[a];
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

static void tune_cache_store(const fdtd_plan_s* p, const char* path) {
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    const KCfg* c = p->cfg;
    std::fprintf(f, "{\"key\": \"%s\", \"cfg\": [[%d,%d,%d,%d,%d],[%d,%d,%d,%d,%d],[%d,%d,%d,%d,%d]]}\n",
                 tune_key(p).c_str(), c[0].M, c[0].TX, c[0].NT, c[0].wpb, c[0].remap, c[1].M, c[1].TX, c[1].NT,
                 c[1].wpb, c[1].remap, c[2].M, c[2].TX, c[2].NT, c[2].wpb, c[2].remap);
    std::fclose(f);
}

static double source_value(const fdtd_source* src, double theta, double t) {
    if (!src) return 0.0;
    const double x = (t - src->t0) / src->tau;
    return theta * src->amp * std::exp(-x * x) * std::sin(2.0 * M_PI * src->f0 * (t - src->t0));
}

template <typename T>
static FieldPtrs<T> state_ptrs(fdtd_plan_s* p, int set) {
    FieldPtrs<T> f;
    for (int c = 0; c < 6; ++c) f.c[c] = comp_ptr<T>(p, set, c);
    return f;
}
template <typename T>
static FieldPtrsW<T> state_ptrs_w(fdtd_plan_s* p, int set) {
    FieldPtrsW<T> f;
    for (int c = 0; c < 6; ++c) f.c[c] = comp_ptr<T>(p, set, c);
    return f;
}

template <typename T>
static fdtd_status energy_into(fdtd_plan_s* p, int set, double* dst) {
    AuxCoef k = aux_coef(p->d, 0.0);
    if (p->d.scheme == FDTD_ADI && p->d.form == FDTD_CONVENTIONAL) k.link = 0.25 * p->d.dt;
    hipLaunchKernelGGL((energy_partial_kernel<T>), dim3(p->npartial), dim3(256), 0, p->stream,
                       state_ptrs<T>(p, set), p->eps, p->dims, k, p->partial);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(64), 0, p->stream, p->partial, p->npartial, dst);
    HIPCHK(hipGetLastError());
    return FDTD_OK;
}

template <typename T, typename S>
static fdtd_status run_impl(fdtd_plan_s* p, void* const E[3], void* const H[3], int nsteps, const fdtd_source* src,
                            double* energy, int every) {
    const fdtd_desc& d = p->d;
    const Dims& dm = p->dims;
    const bool adi = d.scheme == FDTD_ADI;
    const bool conv = d.form == FDTD_CONVENTIONAL;
    const int mode = conv ? (adi ? CONV_ADI : CONV_LOD) : FUND;
    const long long nn = (long long)(dm.nx + 1) * (dm.ny + 1) * (dm.nz + 1);
    const unsigned gblocks = (unsigned)((nn + 255) / 256);
    FieldPtrs<T> caller;
    FieldPtrsW<T> caller_w;
    for (int c = 0; c < 3; ++c) {
        caller.c[c] = static_cast<const T*>(E[c]);
        caller.c[3 + c] = static_cast<const T*>(H[c]);
        caller_w.c[c] = static_cast<T*>(E[c]);
        caller_w.c[3 + c] = static_cast<T*>(H[c]);
    }
    const int nrec = energy ? nsteps / every + 1 : 0;
    if (nrec > p->energy_cap) {
        if (p->energy_dev) HIPCHK(hipFree(p->energy_dev));
        p->energy_dev = nullptr;
        HIPCHK(hipMalloc(&p->energy_dev, sizeof(double) * nrec));
        p->energy_cap = nrec;
    }
    // input processing
    const AuxCoef kin = aux_coef(d, (adi && !conv) ? 0.25 * d.dt : 0.0);
    hipLaunchKernelGGL((load_state_kernel<T>), dim3(gblocks), dim3(256), 0, p->stream, caller, state_ptrs_w<T>(p, 0),
                       p->eps, dm, kin);
    HIPCHK(hipGetLastError());
    int cur = 0;
    if (adi && conv) {
        HIPCHK(hipMemcpyAsync(comp_ptr<T>(p, 1, 0), comp_ptr<T>(p, 0, 0), sizeof(T) * dm.comp * 6,
                              hipMemcpyDeviceToDevice, p->stream));
    }
    if (d.scheme == FDTD_LOD2) {
        fdtd_status st = substep<T, S>(p, 1, 0.25 * d.dt, mode, cur, nullptr, false);
        if (st != FDTD_OK) return st;
    }
    const SchemeDef& sd = kSchemes[d.scheme];
    Timing& tm = p->tm;
    tm.used = 0;
    tm.fam.clear();
    if (!tm.main0) {
        HIPCHK(hipEventCreate(&tm.main0));
        HIPCHK(hipEventCreate(&tm.main1));
    }
    HIPCHK(hipEventRecord(tm.main0, p->stream));
    if (energy) {
        fdtd_status st = energy_into<T>(p, cur, p->energy_dev);
        if (st != FDTD_OK) return st;
    }
    double last_b_g = 0.0;   // source term of the last B sub-step (ADI output correction)
    for (int n = 0; n < nsteps; ++n) {
        const long long nglob = p->step + n;
        for (int u = 0; u < sd.nsub; ++u) {
            const SubStep& ss = sd.sub[u];
            const double theta = ss.theta_frac * d.dt;
            const double g = source_value(src, theta, (double(nglob) + ss.t_frac) * d.dt);
            if (adi && !conv && n == nsteps - 1 && ss.op == 1) {
                HIPCHK(hipMemcpyAsync(p->snap, comp_ptr<T>(p, cur, 0), sizeof(T) * dm.comp * 6,
                                      hipMemcpyDeviceToDevice, p->stream));
            }
            const Inject inj = source_inject(p, src, g, mode);
            const bool timed = tm.per_launch > 0 && n % tm.per_launch == 0;
            fdtd_status st = substep<T, S>(p, ss.op, theta, mode, cur, &inj, timed);
            if (st != FDTD_OK) return st;
            if (ss.op == 1) last_b_g = g;
        }
        if (energy && (n + 1) % every == 0) {
            fdtd_status st = energy_into<T>(p, cur, p->energy_dev + (n + 1) / every);
            if (st != FDTD_OK) return st;
        }
    }
    HIPCHK(hipEventRecord(tm.main1, p->stream));
    // output processing
    if (nsteps > 0) {
        if (d.scheme == FDTD_LOD2) {
            fdtd_status st = substep<T, S>(p, 1, -0.25 * d.dt, mode, cur, nullptr, false);
            if (st != FDTD_OK) return st;
        }
        const bool add_old = adi && !conv;
        FieldPtrs<T> old;
        for (int c = 0; c < 6; ++c) old.c[c] = reinterpret_cast<const T*>(p->snap ? p->snap : p->state) + (size_t)c * dm.comp;
        const long long src_off = src ? (long long)src->k * dm.plane + (long long)src->j * dm.px + src->i : -1;
        hipLaunchKernelGGL((store_state_kernel<T>), dim3(gblocks), dim3(256), 0, p->stream, state_ptrs<T>(p, cur),
                           old, caller_w, dm, add_old ? 1 : 0, src_off, 0.5 * last_b_g);
        HIPCHK(hipGetLastError());
    }
    p->step += nsteps;
    if (energy) {
        HIPCHK(hipMemcpyAsync(energy, p->energy_dev, sizeof(double) * nrec, hipMemcpyDeviceToHost, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
        for (int m = 0; m < nrec; ++m)
            if (!std::isfinite(energy[m])) return FDTD_ENONFINITE;
    }
    return FDTD_OK;
}

// ---------------------------------------------------------------------------
// adjoint gradient of the probe objective (fundamental ADI)
// ---------------------------------------------------------------------------
static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

template <typename T, typename S>
static fdtd_status grad_impl(fdtd_plan_s* p, void* const E[3], void* const H[3], int nsteps, const fdtd_source* src,
                             const int probe[3], const int* dbox, int K, double* J_out, double* grad_out) {
    const fdtd_desc& d = p->d;
    const Dims& dm = p->dims;
    const double theta = 0.5 * d.dt;
    const bool want = grad_out != nullptr;
    FieldPtrs<T> caller;
    for (int c = 0; c < 3; ++c) {
        caller.c[c] = static_cast<const T*>(E[c]);
        caller.c[3 + c] = static_cast<const T*>(H[c]);
    }
    Box b{0, 0, 0, 1, 1, 1};
    if (want) b = Box{dbox[0], dbox[2], dbox[4], dbox[1] - dbox[0], dbox[3] - dbox[2], dbox[5] - dbox[4]};
    const long long nb = (long long)b.bi * b.bj * b.bk;
    const int nseg = want ? (nsteps + K - 1) / K : 0;
    const int nrec = want ? 2 * std::min(K, std::max(nsteps, 1)) + 1 : 0;
    const size_t ssz = sizeof(T) * 6 * (size_t)dm.comp;
    // scratch layout: scalars | probe records | design records | adjoint state | checkpoints
    const size_t o_prb = 256;
    const size_t o_rec = o_prb + align256(sizeof(double) * 3 * std::max(nrec, 2));
    const size_t o_adj = o_rec + align256(sizeof(T) * 3 * (size_t)nb * nrec);
    const size_t o_ckp = o_adj + (want ? align256(ssz) : 0);
    const size_t need = o_ckp + (size_t)nseg * align256(ssz);
    if (need > p->gcap) {
        if (p->gbuf) HIPCHK(hipFree(p->gbuf));
        p->gbuf = nullptr;
        p->gcap = 0;
        HIPCHK(hipMalloc(&p->gbuf, need));
        p->gcap = need;
    }
    char* g0 = static_cast<char*>(p->gbuf);
    double* Jd = reinterpret_cast<double*>(g0);
    double* seed = Jd + 1;
    double* prb = reinterpret_cast<double*>(g0 + o_prb);
    T* rec = reinterpret_cast<T*>(g0 + o_rec);
    T* adj = want ? reinterpret_cast<T*>(g0 + o_adj) : nullptr;
    auto ckpt = [&](int sidx) { return reinterpret_cast<T*>(g0 + o_ckp + (size_t)sidx * align256(ssz)); };
    auto recp = [&](int m) { return rec + (size_t)m * 3 * nb; };
    const long long probe_off = (long long)probe[2] * dm.plane + (long long)probe[1] * dm.px + probe[0];
    const bool src_at_probe = src && src->i == probe[0] && src->j == probe[1] && src->k == probe[2];
    long long src_idx = -1;
    if (want && src && src->i >= b.i0 && src->i < b.i0 + b.bi && src->j >= b.j0 && src->j < b.j0 + b.bj &&
        src->k >= b.k0 && src->k < b.k0 + b.bk)
        src_idx = ((long long)(src->k - b.k0) * b.bj + (src->j - b.j0)) * b.bi + (src->i - b.i0);
    const unsigned rblocks = (unsigned)std::max<long long>(1, (nb + 255) / 256);
    const long long nn = (long long)(dm.nx + 1) * (dm.ny + 1) * (dm.nz + 1);
    const unsigned gblocks = (unsigned)((nn + 255) / 256);
    T* st0 = set_ptr<T>(p, 0);
    auto fptrs = [&](T* base) {
        FieldPtrs<T> f;
        for (int c = 0; c < 6; ++c) f.c[c] = base + (size_t)c * dm.comp;
        return f;
    };
    auto record = [&](T* dst, double* pdst) -> fdtd_status {
        hipLaunchKernelGGL((record_kernel<T>), dim3(dst ? rblocks : 1), dim3(256), 0, p->stream, fptrs(st0), dm, b,
                           dst, probe_off, pdst);
        HIPCHK(hipGetLastError());
        return FDTD_OK;
    };
    auto fwd_sub = [&](int op, long long glob, double tf, double* g_out) -> fdtd_status {
        const double g = source_value(src, theta, (double(glob) + tf) * d.dt);
        *g_out = g;
        const Inject inj = source_inject(p, src, g, FUND);
        int cur = 0;
        return substep<T, S>(p, op, theta, FUND, cur, &inj, false);
    };
#define GCHK(x)                                   \
    do {                                          \
        fdtd_status s_ = (x);                     \
        if (s_ != FDTD_OK) return s_;             \
    } while (0)

    // forward sweep: J, checkpoints every K steps
    const AuxCoef kin = aux_coef(d, 0.25 * d.dt);
    hipLaunchKernelGGL((load_state_kernel<T>), dim3(gblocks), dim3(256), 0, p->stream, caller, state_ptrs_w<T>(p, 0),
                       p->eps, dm, kin);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemsetAsync(Jd, 0, 256, p->stream));
    for (int n = 0; n < nsteps; ++n) {
        if (want && n % K == 0) HIPCHK(hipMemcpyAsync(ckpt(n / K), st0, ssz, hipMemcpyDeviceToDevice, p->stream));
        const long long glob = p->step + n;
        double gA, gB;
        GCHK(fwd_sub(0, glob, 0.25, &gA));
        GCHK(record(nullptr, prb));
        GCHK(fwd_sub(1, glob, 0.75, &gB));
        GCHK(record(nullptr, prb + 3));
        hipLaunchKernelGGL(probe_kernel, dim3(1), dim3(64), 0, p->stream, prb, prb + 3,
                           src_at_probe ? 0.5 * gB : 0.0, p->eps, probe_off, kEps0, d.dt, Jd, nullptr);
        HIPCHK(hipGetLastError());
    }
    if (want) {
        HIPCHK(hipMemsetAsync(adj, 0, ssz, p->stream));
        HIPCHK(hipMemsetAsync(grad_out, 0, sizeof(double) * nb, p->stream));
        const FieldPtrs<T> lam = fptrs(adj);
        const double scale = -0.5 * kEps0;
        auto acc = [&](int m, double g) -> fdtd_status {
            hipLaunchKernelGGL((grad_acc_kernel<T>), dim3(rblocks), dim3(256), 0, p->stream, lam, dm, b, recp(m),
                               recp(m + 1), src_idx, 0.5 * g, scale, grad_out);
            HIPCHK(hipGetLastError());
            return FDTD_OK;
        };
        auto adj_sub = [&](int op, const Inject* inj) -> fdtd_status {
            for (int k = 0; k < 3; ++k) GCHK((launch_pass<T, S>(p, op, k, -theta, FUND, adj, adj, inj, false)));
            return FDTD_OK;
        };
        Inject seed_inj;
        seed_inj.i = probe[0]; seed_inj.j = probe[1]; seed_inj.k = probe[2];
        seed_inj.mask = 7u;
        seed_inj.pre_dev = seed;
        std::vector<double> gs(2 * (size_t)K);
        for (int sg = nseg - 1; sg >= 0; --sg) {
            const int n0 = sg * K, L = std::min(nsteps, n0 + K) - n0;
            // recompute the segment from its checkpoint, recording every sub-step state
            HIPCHK(hipMemcpyAsync(st0, ckpt(sg), ssz, hipMemcpyDeviceToDevice, p->stream));
            GCHK(record(recp(0), prb));
            for (int q = 0; q < L; ++q) {
                const long long glob = p->step + n0 + q;
                GCHK(fwd_sub(0, glob, 0.25, &gs[2 * q]));
                GCHK(record(recp(2 * q + 1), prb + 3 * (2 * q + 1)));
                GCHK(fwd_sub(1, glob, 0.75, &gs[2 * q + 1]));
                GCHK(record(recp(2 * q + 2), prb + 3 * (2 * q + 2)));
            }
            // reverse sub-steps
            for (int q = L - 1; q >= 0; --q) {
                const int mB = 2 * q + 1, mA = 2 * q;
                const double gB = gs[mB], gA = gs[mA];
                hipLaunchKernelGGL(probe_kernel, dim3(1), dim3(64), 0, p->stream, prb + 3 * mB, prb + 3 * (mB + 1),
                                   src_at_probe ? 0.5 * gB : 0.0, p->eps, probe_off, kEps0, d.dt, nullptr, seed);
                HIPCHK(hipGetLastError());
                GCHK(acc(mB, gB));
                GCHK(adj_sub(1, &seed_inj));
                GCHK(acc(mB, gB));
                GCHK(acc(mA, gA));
                GCHK(adj_sub(0, nullptr));
                GCHK(acc(mA, gA));
            }
        }
        if (nsteps > 0) {
            hipLaunchKernelGGL((grad_link_kernel<T>), dim3(rblocks), dim3(256), 0, p->stream, lam, caller, dm, b,
                               recp(0), -kEps0, grad_out);
            HIPCHK(hipGetLastError());
        }
    }
#undef GCHK
    HIPCHK(hipMemcpyAsync(J_out, Jd, sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    return std::isfinite(*J_out) ? FDTD_OK : FDTD_ENONFINITE;
}

// ---------------------------------------------------------------------------
// batch plans
// ---------------------------------------------------------------------------
static void batch_clear(Batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    for (BatchPass& bp : b->passes) {
        if (bp.tab) (void)hipFree(bp.tab);
        if (bp.items) (void)hipFree(bp.items);
    }
    b->passes.clear();
}

// Chunks per line of a grid in a batched pass: a power of two (the separator
// solve runs over segments of P lanes), for y/z lines at least 64/TX so that a
// sub-block of TX * P threads is whole waves.  (Chunk counts rounded only to
// a multiple of 64/TX, with a serial separator solve, were measured slower.)
static int batch_P(const fdtd_plan_s* g, int axis, const KCfg& c) {
    const int P = next_pow2((axis_cells(g->dims, axis) + c.M - 1) / c.M);
    return axis == 0 ? P : std::max(P, 64 / c.TX);
}

static bool batch_cfg_valid(const fdtd_plan_s* p, int axis, const KCfg& c) {
    // refined batched passes: 8-slot chunks (the 16-slot y/z variant does not fit
    // its registers with the batch addressing)
    if (p->refine && c.M != 8) return false;
    int Pmax = 1;
    for (const fdtd_plan_s* g : p->batch->subs) {
        if (!cfg_valid(g, axis, c)) return false;
        Pmax = std::max(Pmax, batch_P(g, axis, c));
    }
    if (Pmax > 64) return false;
    return axis == 0 || c.TX * Pmax <= c.NT;
}

static void batch_default_cfg(fdtd_plan_s* p) {
    for (int axis = 0; axis < 3; ++axis) {
        std::vector<KCfg> pref;
        if (axis == 0) pref = {{8, 0, 0, 4, 0}, {16, 0, 0, 4, 0}};
        else if (p->d.dtype == FDTD_F32) pref = {{8, 16, 1024, 0, 0}, {16, 32, 1024, 0, 0}, {16, 16, 512, 0, 0}, {32, 16, 512, 0, 0}};
        else pref = {{8, 8, 512, 0, 0}, {16, 16, 512, 0, 0}};
        for (const KCfg& c : pref)
            if (batch_cfg_valid(p, axis, c)) { p->cfg[axis] = c; break; }
    }
}

// The table of pass (op, k) with theta = frac * dt for every grid (built on
// first use with the current kernel configuration).
template <typename T, typename S>
static fdtd_status batch_pass(fdtd_plan_s* p, int op, int k, double frac, const BatchPass** out) {
    Batch* b = p->batch;
    for (const BatchPass& bp : b->passes)
        if (bp.op == op && bp.k == k && bp.frac == frac) { *out = &bp; return FDTD_OK; }
    const int w = kPairs[op][k].w;
    const KCfg& cf = p->cfg[w];
    const int n = (int)b->subs.size();
    std::vector<PassArgs<T, S>> tab(n);
    int Pmax = 1;
    for (int g = 0; g < n; ++g) {
        fdtd_plan_s* sub = b->subs[g];
        sub->cfg[w] = cf;
        PassShape sh;
        build_pass<T, S>(sub, op, k, frac * sub->d.dt, FUND, set_ptr<T>(sub, 0), set_ptr<T>(sub, 0), nullptr,
                         tab[g], sh);
        tab[g].P = batch_P(sub, w, cf);
        tab[g].remap = 0;
        Pmax = std::max(Pmax, tab[g].P);
    }
    std::vector<int2> items;
    int lds_rows = 0;   // y/z: sub-block areas x chunks, the most any grid needs
    for (int g = 0; g < n; ++g) {
        const int per = (w == 0) ? 1 : Pmax / tab[g].P;   // virtual blocks per block
        const int nit = (tab[g].nblk + per - 1) / per;
        for (int q = 0; q < nit; ++q) items.push_back(make_int2(g, q));
        if (w != 0) lds_rows = std::max(lds_rows, ((Pmax + tab[g].P - 1) / tab[g].P) * tab[g].P);
    }
    BatchPass bp;
    bp.op = op; bp.k = k; bp.frac = frac; bp.Pmax = Pmax;
    bp.lds = (size_t)(p->refine ? 13 : 9) * lds_rows * (cf.TX + 1) * sizeof(S);
    bp.nitems = (int)items.size();
    HIPCHK(hipMalloc(&bp.tab, sizeof(PassArgs<T, S>) * n));
    hipError_t e = hipMalloc(&bp.items, sizeof(int2) * items.size());
    if (e == hipSuccess) e = hipMemcpy(bp.tab, tab.data(), sizeof(PassArgs<T, S>) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bp.items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(bp.tab);
        if (bp.items) (void)hipFree(bp.items);
        return from_hip(e);
    }
    b->passes.push_back(bp);
    *out = &b->passes.back();
    return FDTD_OK;
}

template <typename T, typename S, int MODE>
static fdtd_status batch_launch_mode(fdtd_plan_s* p, const BatchPass& bp, hipStream_t st) {
    const int w = kPairs[bp.op][bp.k].w;
    const KCfg& cf = p->cfg[w];
    const bool mat = p->batch->mat;
    const auto* tab = static_cast<const PassArgs<T, S>*>(bp.tab);
    const auto* items = static_cast<const int2*>(bp.items);
    const dim3 grid((unsigned)bp.nitems);
    if (w == 0) {
        const dim3 block(64 * cf.wpb);
        if (cf.M == 8) {
            if (mat) hipLaunchKernelGGL((pass_x_batch_kernel<T, S, 8, MODE, true>), grid, block, 0, st, tab, items);
            else hipLaunchKernelGGL((pass_x_batch_kernel<T, S, 8, MODE, false>), grid, block, 0, st, tab, items);
        } else if constexpr (MODE != FUND_REF) {
            if (mat) hipLaunchKernelGGL((pass_x_batch_kernel<T, S, 16, MODE, true>), grid, block, 0, st, tab, items);
            else hipLaunchKernelGGL((pass_x_batch_kernel<T, S, 16, MODE, false>), grid, block, 0, st, tab, items);
        } else {
            return FDTD_EUNSUPPORTED;
        }
    } else {
        const int M = cf.M, TX = cf.TX, NT = cf.NT;
        const dim3 block(TX * bp.Pmax);
        const size_t lds = bp.lds;
#define CASE_YZB(MM, TT, NN)                                                                                  \
    if (M == MM && TX == TT && NT == NN) {                                                                    \
        if constexpr (MODE != FUND_REF || MM == 8) {                                                          \
            if (mat)                                                                                          \
                hipLaunchKernelGGL((pass_yz_batch_kernel<T, S, MM, MODE, TT, NN, true>), grid, block, lds, st, tab, items); \
            else                                                                                              \
                hipLaunchKernelGGL((pass_yz_batch_kernel<T, S, MM, MODE, TT, NN, false>), grid, block, lds, st, tab, items); \
        } else {                                                                                              \
            return FDTD_EUNSUPPORTED;                                                                         \
        }                                                                                                     \
    } else
        if constexpr (sizeof(S) == 4) {
            CASE_YZB(16, 32, 1024) CASE_YZB(16, 16, 512) CASE_YZB(8, 16, 1024) CASE_YZB(32, 16, 512) CASE_YZB(8, 32, 512)
            return FDTD_EUNSUPPORTED;
        } else {
            CASE_YZB(16, 16, 512) CASE_YZB(8, 8, 512) CASE_YZB(8, 16, 1024) return FDTD_EUNSUPPORTED;
        }
#undef CASE_YZB
    }
    HIPCHK(hipGetLastError());
    return FDTD_OK;
}
template <typename T, typename S>
static fdtd_status batch_launch(fdtd_plan_s* p, const BatchPass& bp, hipStream_t st) {
    if constexpr (sizeof(S) == 4) {
        if (p->refine) return batch_launch_mode<T, S, FUND_REF>(p, bp, st);
    }
    return batch_launch_mode<T, S, FUND>(p, bp, st);
}

// One sub-step (operator op, theta = frac * dt) of every grid: three launches.
template <typename T, typename S>
static fdtd_status batch_substep(fdtd_plan_s* p, int op, double frac, hipStream_t st) {
    for (int k = 0; k < 3; ++k) {
        const BatchPass* bp = nullptr;
        fdtd_status s = batch_pass<T, S>(p, op, k, frac, &bp);
        if (s != FDTD_OK) return s;
        s = batch_launch<T, S>(p, *bp, st);
        if (s != FDTD_OK) return s;
    }
    return FDTD_OK;
}

template <typename T, typename S>
static fdtd_status batch_tables(fdtd_plan_s* p) {
    const SchemeDef& sd = kSchemes[p->d.scheme];
    for (int u = 0; u < sd.nsub; ++u)
        for (int k = 0; k < 3; ++k) {
            const BatchPass* bp = nullptr;
            fdtd_status s = batch_pass<T, S>(p, sd.sub[u].op, k, sd.sub[u].theta_frac, &bp);
            if (s != FDTD_OK) return s;
        }
    if (p->d.scheme == FDTD_LOD2)
        for (double f : {0.25, -0.25})
            for (int k = 0; k < 3; ++k) {
                const BatchPass* bp = nullptr;
                fdtd_status s = batch_pass<T, S>(p, 1, k, f, &bp);
                if (s != FDTD_OK) return s;
            }
    return FDTD_OK;
}

// Time steps per captured graph.  A graph launch costs tens of microseconds
// of host time and separates consecutive replays on the device, so one graph
// holds several steps; a run replays it floor(steps / kGraphSteps) times and
// launches the remaining steps directly.
constexpr int kGraphSteps = 8;

// Per-step working set (fields and medium) above which a batch is stepped in
// groups.  A group runs all its steps before the next one starts, so its
// arrays stay in the 256 MB MALL (AMD Infinity Cache) from pass to pass
// instead of cycling through it: 21 of the 64 test cavities (130 MB) step at
// 38 G cell-updates/s, all 64 (308 MB) at 31.
constexpr size_t kGroupBytes = size_t(128) << 20;

// Capture kGraphSteps time steps of the main iteration (all sub-steps) as a graph.
template <typename T, typename S>
static fdtd_status batch_graph(fdtd_plan_s* p) {
    Batch* b = p->batch;
    if (b->exec) return FDTD_OK;
    const SchemeDef& sd = kSchemes[p->d.scheme];
    // The three pair passes of a sub-step update disjoint arrays: capture them
    // as parallel branches (fork on events, join before the next sub-step).
    HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    fdtd_status st = FDTD_OK;
    auto branch = [&](int k, hipStream_t str, int op, double frac) -> fdtd_status {
        const BatchPass* bp = nullptr;
        fdtd_status s2 = batch_pass<T, S>(p, op, k, frac, &bp);
        return s2 == FDTD_OK ? batch_launch<T, S>(p, *bp, str) : s2;
    };
    for (int v = 0; v < kGraphSteps * sd.nsub && st == FDTD_OK; ++v) {
        const int u = v % sd.nsub;
        const int op = sd.sub[u].op;
        const double frac = sd.sub[u].theta_frac;
        if (hipEventRecord(b->ev[0], b->cap) != hipSuccess || hipStreamWaitEvent(b->fork[0], b->ev[0], 0) != hipSuccess ||
            hipStreamWaitEvent(b->fork[1], b->ev[0], 0) != hipSuccess) {
            st = FDTD_EDEVICE;
            break;
        }
        st = branch(0, b->cap, op, frac);
        if (st == FDTD_OK) st = branch(1, b->fork[0], op, frac);
        if (st == FDTD_OK) st = branch(2, b->fork[1], op, frac);
        if (st == FDTD_OK &&
            (hipEventRecord(b->ev[1], b->fork[0]) != hipSuccess || hipEventRecord(b->ev[2], b->fork[1]) != hipSuccess ||
             hipStreamWaitEvent(b->cap, b->ev[1], 0) != hipSuccess || hipStreamWaitEvent(b->cap, b->ev[2], 0) != hipSuccess))
            st = FDTD_EDEVICE;
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (st != FDTD_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    HIPCHK(e);
    b->graph = g;
    HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return FDTD_OK;
}

template <typename T, typename S>
static fdtd_status run_batch_impl(fdtd_plan_s* p, void* const* E, void* const* H, int nsteps) {
    Batch* b = p->batch;
    const fdtd_desc& d = p->d;
    const bool adi = d.scheme == FDTD_ADI;
    const int n = (int)b->subs.size();
    auto caller = [&](int g) {
        FieldPtrs<T> f;
        for (int c = 0; c < 3; ++c) {
            f.c[c] = static_cast<const T*>(E[3 * g + c]);
            f.c[3 + c] = static_cast<const T*>(H[3 * g + c]);
        }
        return f;
    };
    fdtd_status st = batch_tables<T, S>(p);
    if (st != FDTD_OK) return st;
    for (int g = 0; g < n; ++g) {
        fdtd_plan_s* sub = b->subs[g];
        const Dims& dm = sub->dims;
        const long long nn = (long long)(dm.nx + 1) * (dm.ny + 1) * (dm.nz + 1);
        const AuxCoef kin = aux_coef(sub->d, adi ? 0.25 * sub->d.dt : 0.0);
        hipLaunchKernelGGL((load_state_kernel<T>), dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, p->stream,
                           caller(g), state_ptrs_w<T>(sub, 0), sub->eps, dm, kin);
        HIPCHK(hipGetLastError());
    }
    if (d.scheme == FDTD_LOD2) {
        st = batch_substep<T, S>(p, 1, 0.25, p->stream);
        if (st != FDTD_OK) return st;
    }
    const int nmain = nsteps > 0 ? (adi ? nsteps - 1 : nsteps) : 0;   // steps of the plain main iteration
    const int ngraph = nmain / kGraphSteps;
    if (ngraph > 0) {
        st = batch_graph<T, S>(p);
        if (st != FDTD_OK) return st;
    }
    Timing& tm = p->tm;
    tm.used = 0;
    tm.fam.clear();
    if (!tm.main0) {
        HIPCHK(hipEventCreate(&tm.main0));
        HIPCHK(hipEventCreate(&tm.main1));
    }
    HIPCHK(hipEventRecord(tm.main0, p->stream));
    for (int m = 0; m < ngraph; ++m) HIPCHK(hipGraphLaunch(b->exec, p->stream));
    {
        const SchemeDef& sd = kSchemes[d.scheme];
        for (int m = ngraph * kGraphSteps; m < nmain; ++m)
            for (int u = 0; u < sd.nsub; ++u) {
                st = batch_substep<T, S>(p, sd.sub[u].op, sd.sub[u].theta_frac, p->stream);
                if (st != FDTD_OK) return st;
            }
    }
    if (adi && nsteps > 0) {
        // last step: the state before the B sub-step is kept for the output
        st = batch_substep<T, S>(p, 0, 0.5, p->stream);
        if (st != FDTD_OK) return st;
        for (fdtd_plan_s* sub : b->subs)
            HIPCHK(hipMemcpyAsync(sub->snap, sub->state, sizeof(T) * sub->dims.comp * 6, hipMemcpyDeviceToDevice,
                                  p->stream));
        st = batch_substep<T, S>(p, 1, 0.5, p->stream);
        if (st != FDTD_OK) return st;
    }
    HIPCHK(hipEventRecord(tm.main1, p->stream));
    if (nsteps > 0) {
        if (d.scheme == FDTD_LOD2) {
            st = batch_substep<T, S>(p, 1, -0.25, p->stream);
            if (st != FDTD_OK) return st;
        }
        for (int g = 0; g < n; ++g) {
            fdtd_plan_s* sub = b->subs[g];
            const Dims& dm = sub->dims;
            const long long nn = (long long)(dm.nx + 1) * (dm.ny + 1) * (dm.nz + 1);
            FieldPtrsW<T> out;
            for (int c = 0; c < 3; ++c) {
                out.c[c] = static_cast<T*>(E[3 * g + c]);
                out.c[3 + c] = static_cast<T*>(H[3 * g + c]);
            }
            FieldPtrs<T> old;
            for (int c = 0; c < 6; ++c)
                old.c[c] = reinterpret_cast<const T*>(adi ? sub->snap : sub->state) + (size_t)c * dm.comp;
            hipLaunchKernelGGL((store_state_kernel<T>), dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, p->stream,
                               state_ptrs<T>(sub, 0), old, out, dm, adi ? 1 : 0, -1LL, 0.0);
            HIPCHK(hipGetLastError());
        }
    }
    p->step += nsteps;
    return FDTD_OK;
}

template <typename T, typename S>
static fdtd_status batch_autotune_impl(fdtd_plan_s* p, int reps, double* best_ms) {
    Batch* b = p->batch;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    fdtd_status st = FDTD_OK;
    for (int axis = 0; axis < 3 && st == FDTD_OK; ++axis) {
        int k = 0;
        while (kPairs[0][k].w != axis) ++k;
        std::vector<KCfg> cand;
        if (axis == 0) {
            for (int M : {8, 16})
                for (int wpb : {4, 2, 1}) cand.push_back(KCfg{M, 0, 0, wpb, 0});
        } else if (p->d.dtype == FDTD_F32) {
            for (const auto& v : kYzF32) cand.push_back(KCfg{v[0], v[1], v[2], 0, 0});
        } else {
            for (const auto& v : kYzF64) cand.push_back(KCfg{v[0], v[1], v[2], 0, 0});
        }
        KCfg best = p->cfg[axis];
        float tbest = 1e30f;
        for (const KCfg& c : cand) {
            if (!batch_cfg_valid(p, axis, c)) continue;
            p->cfg[axis] = c;
            batch_clear(b);
            const BatchPass* bp = nullptr;
            st = batch_pass<T, S>(p, 0, k, 0.5, &bp);
            if (st == FDTD_OK) st = batch_launch<T, S>(p, *bp, p->stream);
            if (st != FDTD_OK) break;
            if (hipEventRecord(e0, p->stream) != hipSuccess) { st = FDTD_EDEVICE; break; }
            for (int r = 0; r < reps && st == FDTD_OK; ++r) st = batch_launch<T, S>(p, *bp, p->stream);
            if (st != FDTD_OK) break;
            if (hipEventRecord(e1, p->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                st = FDTD_EDEVICE;
                break;
            }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < tbest) { tbest = ms; best = c; }
        }
        p->cfg[axis] = best;
        if (best_ms) best_ms[axis] = tbest / reps;
    }
    batch_clear(b);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == FDTD_OK) p->tuned = 1;
    return st;
}

// Wrap single-grid plans (their ownership passes to the result; on failure
// they are destroyed) into one batch plan.
static fdtd_status batch_from_subs(const fdtd_desc& d0, const std::vector<fdtd_plan_s*>& subs, void* hip_stream,
                                   fdtd_plan_s** out);

}  // namespace fdtd

using namespace fdtd;

static bool plan_ok(fdtd_plan_t p) { return p != nullptr && p->magic == 0xFD7DFD7Du; }

extern "C" {

const char* fdtd_strerror(fdtd_status s) {
    switch (s) {
        case FDTD_OK: return "ok";
        case FDTD_EINVAL: return "invalid argument";
        case FDTD_ENOMEM: return "device out of memory";
        case FDTD_EDEVICE: return "HIP runtime error";
        case FDTD_EUNSUPPORTED: return "not supported by this library";
        case FDTD_ENONFINITE: return "non-finite energy after stepping";
    }
    return "unknown status";
}

fdtd_status fdtd_plan(const fdtd_desc* d, void* hip_stream, fdtd_plan_t* out) {
    if (!d || !out) return FDTD_EINVAL;
    *out = nullptr;
    if (d->nx < 2 || d->ny < 2 || d->nz < 2) return FDTD_EINVAL;
    if (!(d->dt > 0) || !(d->dx > 0) || !(d->dy > 0) || !(d->dz > 0)) return FDTD_EINVAL;
    if (!std::isfinite(d->dt) || !std::isfinite(d->dx) || !std::isfinite(d->dy) || !std::isfinite(d->dz))
        return FDTD_EINVAL;
    if (d->scheme < 0 || d->scheme > 3 || d->form < 0 || d->form > 1 || d->dtype < 0 || d->dtype > 3)
        return FDTD_EINVAL;
    if (d->boundary != 0) return FDTD_EUNSUPPORTED;
    if (d->mu_r != nullptr) return FDTD_EUNSUPPORTED;
    const bool refine = d->dtype == FDTD_F32_REFINE;
    if (refine && d->form != FDTD_FUNDAMENTAL) return FDTD_EUNSUPPORTED;
    const int nmax = std::max(d->nx, std::max(d->ny, d->nz));
    // register budget (refined solves: 8-slot chunks on at most 64 lanes)
    if (nmax > (d->dtype == FDTD_F32 ? 1024 : 512)) return FDTD_EUNSUPPORTED;
    const long long ncells = (long long)d->nx * d->ny * d->nz;
    std::vector<float> eps_host;
    if (d->eps_r) {
        eps_host.resize(ncells);
        if (hipMemcpy(eps_host.data(), d->eps_r, sizeof(float) * ncells, hipMemcpyDefault) != hipSuccess)
            return FDTD_EINVAL;
        for (long long c = 0; c < ncells; ++c)
            if (!(eps_host[c] > 0.0f) || !std::isfinite(eps_host[c])) return FDTD_EINVAL;
    }
    fdtd_plan_s* p = new (std::nothrow) fdtd_plan_s();
    if (!p) return FDTD_ENOMEM;
    p->d = *d;
    p->d.eps_r = nullptr;
    if (refine) {
        p->refine = 1;
        p->d.dtype = FDTD_F32;   // FP32 storage and arithmetic; only the fundamental passes differ
    }
    p->stream = static_cast<hipStream_t>(hip_stream);
    (void)hipGetDevice(&p->device);
    p->esz = d->dtype == FDTD_F64 ? 8 : 4;
    Dims& dm = p->dims;
    dm.nx = d->nx; dm.ny = d->ny; dm.nz = d->nz;
    const int align = d->dtype == FDTD_F64 ? 16 : 32;   // 128-byte rows
    dm.px = ((d->nx + 1 + align - 1) / align) * align;
    dm.plane = dm.px * (d->ny + 1);
    dm.comp = dm.plane * (d->nz + 1);
    dm.cplane = (long long)(d->nx + 1) * (d->ny + 1);
    dm.ccomp = dm.cplane * (d->nz + 1);
    const int sets = (d->scheme == FDTD_ADI && d->form == FDTD_CONVENTIONAL) ? 2 : 1;
    auto fail = [&](fdtd_status st) {
        if (p->state) (void)hipFree(p->state);
        if (p->snap) (void)hipFree(p->snap);
        if (p->eps) (void)hipFree(p->eps);
        if (p->partial) (void)hipFree(p->partial);
        if (p->mat) (void)hipFree(p->mat);
        if (p->mat_eps) (void)hipFree(p->mat_eps);
        delete p;
        return st;
    };
    if (std::getenv("FDTD_TEST_FAIL_ALLOC")) return fail(FDTD_ENOMEM);
    hipError_t e;
    if ((e = hipMalloc(&p->state, p->esz * dm.comp * 6 * sets)) != hipSuccess) return fail(from_hip(e));
    if ((e = hipMemset(p->state, 0, p->esz * dm.comp * 6 * sets)) != hipSuccess) return fail(from_hip(e));
    if (d->scheme == FDTD_ADI && d->form == FDTD_FUNDAMENTAL) {
        if ((e = hipMalloc(&p->snap, p->esz * dm.comp * 6)) != hipSuccess) return fail(from_hip(e));
    }
    // eps_r at node indices (owned index, clamped to the last cell), padded rows
    std::vector<float> en((size_t)dm.comp, 1.0f);
    for (int k = 0; k <= d->nz; ++k)
        for (int j = 0; j <= d->ny; ++j)
            for (int i = 0; i <= d->nx; ++i) {
                const int kk = std::min(k, d->nz - 1), jj = std::min(j, d->ny - 1), ii = std::min(i, d->nx - 1);
                en[(size_t)k * dm.plane + (size_t)j * dm.px + i] =
                    eps_host.empty() ? 1.0f : eps_host[((size_t)kk * d->ny + jj) * d->nx + ii];
            }
    if ((e = hipMalloc(&p->eps, sizeof(float) * dm.comp)) != hipSuccess) return fail(from_hip(e));
    if ((e = hipMemcpy(p->eps, en.data(), sizeof(float) * dm.comp, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(from_hip(e));
    // Piecewise-constant media: at most 256 distinct eps_r values are stored as
    // a one-byte material index per node (the passes then read 17 instead of
    // 20 bytes per FP32 slot); the table of values lives in LDS.
    if (!std::getenv("FDTD_NO_MATERIAL_INDEX")) {
        std::vector<float> uniq(eps_host.begin(), eps_host.end());
        uniq.push_back(1.0f);
        std::sort(uniq.begin(), uniq.end());
        uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
        if (uniq.size() <= 256) {
            std::vector<unsigned char> idx((size_t)dm.comp);
            for (size_t m = 0; m < idx.size(); ++m)
                idx[m] = (unsigned char)(std::lower_bound(uniq.begin(), uniq.end(), en[m]) - uniq.begin());
            p->nmat = (int)uniq.size();
            if ((e = hipMalloc(&p->mat, (size_t)dm.comp)) != hipSuccess) return fail(from_hip(e));
            if ((e = hipMemcpy(p->mat, idx.data(), (size_t)dm.comp, hipMemcpyHostToDevice)) != hipSuccess)
                return fail(from_hip(e));
            if ((e = hipMalloc(&p->mat_eps, sizeof(float) * 256)) != hipSuccess) return fail(from_hip(e));
            if ((e = hipMemcpy(p->mat_eps, uniq.data(), sizeof(float) * uniq.size(), hipMemcpyHostToDevice)) !=
                hipSuccess)
                return fail(from_hip(e));
        }
    }
    default_cfg(p);
    p->npartial = 1024;
    if ((e = hipMalloc(&p->partial, sizeof(double) * p->npartial)) != hipSuccess) return fail(from_hip(e));
    *out = p;
    return FDTD_OK;
}

fdtd_status fdtd_run(fdtd_plan_t p, void* const E[3], void* const H[3], int nsteps, const fdtd_source* src,
                     double* energy, int energy_every) {
    if (!plan_ok(p) || p->batch || !E || !H || nsteps < 0) return FDTD_EINVAL;
    for (int c = 0; c < 3; ++c)
        if (!E[c] || !H[c]) return FDTD_EINVAL;
    if (energy && energy_every < 1) return FDTD_EINVAL;
    if (src) {
        if (src->i < 1 || src->i >= p->d.nx || src->j < 1 || src->j >= p->d.ny || src->k < 0 || src->k >= p->d.nz)
            return FDTD_EINVAL;
        if (!(src->tau > 0) || !std::isfinite(src->f0) || !std::isfinite(src->t0) || !std::isfinite(src->amp))
            return FDTD_EINVAL;
    }
    int dev_now = -1;
    (void)hipGetDevice(&dev_now);
    if (dev_now != p->device) (void)hipSetDevice(p->device);
    fdtd_status st;
    if (p->d.dtype == FDTD_F32) st = run_impl<float, float>(p, E, H, nsteps, src, energy, energy_every);
    else if (p->d.dtype == FDTD_F64) st = run_impl<double, double>(p, E, H, nsteps, src, energy, energy_every);
    else st = run_impl<float, double>(p, E, H, nsteps, src, energy, energy_every);
    if (dev_now != p->device) (void)hipSetDevice(dev_now);
    return st;
}

fdtd_status fdtd_step(fdtd_plan_t p, void* const E[3], void* const H[3], const fdtd_source* src) {
    return fdtd_run(p, E, H, 1, src, nullptr, 1);
}

fdtd_status fdtd_set_step(fdtd_plan_t p, long long n) {
    if (!plan_ok(p) || n < 0) return FDTD_EINVAL;
    p->step = n;
    return FDTD_OK;
}

fdtd_status fdtd_set_timing(fdtd_plan_t p, int per_launch) {
    if (!plan_ok(p) || per_launch < 0) return FDTD_EINVAL;
    p->tm.per_launch = per_launch;
    if (p->batch)
        for (fdtd_plan_s* c : p->batch->groups) c->tm.per_launch = per_launch;
    return FDTD_OK;
}

fdtd_status fdtd_last_timing(fdtd_plan_t p, double* main_ms, double* fam_ms_avg, int* fam_launches) {
    if (!plan_ok(p)) return FDTD_EINVAL;
    if (p->batch && !p->batch->groups.empty()) {
        double tot = 0.0;
        for (fdtd_plan_s* c : p->batch->groups) {
            double m = 0.0;
            const fdtd_status st = fdtd_last_timing(c, &m, nullptr, nullptr);
            if (st != FDTD_OK) return st;
            tot += m;
        }
        if (main_ms) *main_ms = tot;
        for (int f = 0; f < 2; ++f) {
            if (fam_ms_avg) fam_ms_avg[f] = 0.0;
            if (fam_launches) fam_launches[f] = 0;
        }
        return FDTD_OK;
    }
    HIPCHK(hipStreamSynchronize(p->stream));
    float ms = 0.0f;
    if (p->tm.main0) HIPCHK(hipEventElapsedTime(&ms, p->tm.main0, p->tm.main1));
    if (main_ms) *main_ms = ms;
    double tot[2] = {0, 0};
    int cnt[2] = {0, 0};
    for (size_t m = 0; m < p->tm.fam.size(); ++m) {
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, p->tm.ev[2 * m], p->tm.ev[2 * m + 1]));
        tot[p->tm.fam[m]] += t;
        cnt[p->tm.fam[m]] += 1;
    }
    for (int f = 0; f < 2; ++f) {
        if (fam_ms_avg) fam_ms_avg[f] = cnt[f] ? tot[f] / cnt[f] : 0.0;
        if (fam_launches) fam_launches[f] = cnt[f];
    }
    return FDTD_OK;
}

fdtd_status fdtd_autotune(fdtd_plan_t p, int reps, double* best_ms) {
    if (!plan_ok(p) || reps < 1) return FDTD_EINVAL;
    if (p->batch && !p->batch->groups.empty()) {
        // each group tunes for its own grids; best_ms: one pass over all groups
        double tot[3] = {0, 0, 0};
        for (fdtd_plan_s* c : p->batch->groups) {
            double b3[3] = {0, 0, 0};
            const fdtd_status st = fdtd_autotune(c, reps, b3);
            if (st != FDTD_OK) return st;
            for (int a = 0; a < 3; ++a) tot[a] += b3[a];
        }
        for (int a = 0; a < 3; ++a) p->cfg[a] = p->batch->groups[0]->cfg[a];
        if (best_ms)
            for (int a = 0; a < 3; ++a) best_ms[a] = tot[a];
        p->tuned = 1;
        return FDTD_OK;
    }
    const char* cache = p->batch ? nullptr : std::getenv("FDTD_TUNE_CACHE");
    if (cache && *cache && tune_cache_lookup(p, cache)) {
        p->tuned = 2;
        if (best_ms) best_ms[0] = best_ms[1] = best_ms[2] = 0.0;
        return FDTD_OK;
    }
    int dev_now = -1;
    (void)hipGetDevice(&dev_now);
    if (dev_now != p->device) (void)hipSetDevice(p->device);
    fdtd_status st;
    if (p->batch) {
        if (p->d.dtype == FDTD_F32) st = batch_autotune_impl<float, float>(p, reps, best_ms);
        else if (p->d.dtype == FDTD_F64) st = batch_autotune_impl<double, double>(p, reps, best_ms);
        else st = batch_autotune_impl<float, double>(p, reps, best_ms);
    } else if (p->d.dtype == FDTD_F32) st = autotune_impl<float, float>(p, reps, best_ms);
    else if (p->d.dtype == FDTD_F64) st = autotune_impl<double, double>(p, reps, best_ms);
    else st = autotune_impl<float, double>(p, reps, best_ms);
    if (dev_now != p->device) (void)hipSetDevice(dev_now);
    if (st == FDTD_OK && cache && *cache) tune_cache_store(p, cache);
    return st;
}

fdtd_status fdtd_get_kernel_config(fdtd_plan_t p, int axis, fdtd_kernel_config* c) {
    if (!plan_ok(p) || axis < 0 || axis > 2 || !c) return FDTD_EINVAL;
    const KCfg& k = p->cfg[axis];
    c->chunk = k.M;
    c->tile_x = axis == 0 ? 0 : k.TX;
    c->block_threads = axis == 0 ? 64 * k.wpb : k.NT;
    c->remap = k.remap;
    return FDTD_OK;
}

fdtd_status fdtd_set_kernel_config(fdtd_plan_t p, int axis, const fdtd_kernel_config* c) {
    if (!plan_ok(p) || axis < 0 || axis > 2 || !c) return FDTD_EINVAL;
    KCfg k{c->chunk, axis == 0 ? 0 : c->tile_x, axis == 0 ? 0 : c->block_threads,
           axis == 0 ? c->block_threads / 64 : 0, c->remap};
    if (axis == 0 && c->block_threads % 64 != 0) return FDTD_EINVAL;
    if (p->batch && !p->batch->groups.empty()) {
        for (fdtd_plan_s* g : p->batch->groups)
            if (!batch_cfg_valid(g, axis, k)) return FDTD_EINVAL;
        for (fdtd_plan_s* g : p->batch->groups) {
            const fdtd_status st = fdtd_set_kernel_config(g, axis, c);
            if (st != FDTD_OK) return st;
        }
    } else if (p->batch) {
        if (!batch_cfg_valid(p, axis, k)) return FDTD_EINVAL;
        (void)hipStreamSynchronize(p->stream);
        batch_clear(p->batch);
    } else if (!cfg_valid(p, axis, k)) {
        return FDTD_EINVAL;
    }
    p->cfg[axis] = k;
    return FDTD_OK;
}

fdtd_status fdtd_grad_eps(fdtd_plan_t p, void* const E[3], void* const H[3], int nsteps, const fdtd_source* src,
                          int probe_i, int probe_j, int probe_k, const int* design_box, int ckpt_every,
                          double* J_out, double* grad_out) {
    if (!plan_ok(p) || p->batch || !E || !H || nsteps < 0 || !J_out) return FDTD_EINVAL;
    for (int c = 0; c < 3; ++c)
        if (!E[c] || !H[c]) return FDTD_EINVAL;
    const fdtd_desc& d = p->d;
    if (probe_i < 1 || probe_i >= d.nx || probe_j < 1 || probe_j >= d.ny || probe_k < 1 || probe_k >= d.nz)
        return FDTD_EINVAL;
    if (src) {
        if (src->i < 1 || src->i >= d.nx || src->j < 1 || src->j >= d.ny || src->k < 0 || src->k >= d.nz)
            return FDTD_EINVAL;
        if (!(src->tau > 0) || !std::isfinite(src->f0) || !std::isfinite(src->t0) || !std::isfinite(src->amp))
            return FDTD_EINVAL;
    }
    if (grad_out) {
        if (!design_box || ckpt_every < 1) return FDTD_EINVAL;
        const int* b = design_box;
        if (b[0] < 0 || b[1] <= b[0] || b[1] > d.nx || b[2] < 0 || b[3] <= b[2] || b[3] > d.ny || b[4] < 0 ||
            b[5] <= b[4] || b[5] > d.nz)
            return FDTD_EINVAL;
    }
    if (d.scheme != FDTD_ADI || d.form != FDTD_FUNDAMENTAL) return FDTD_EUNSUPPORTED;
    const int probe[3] = {probe_i, probe_j, probe_k};
    int dev_now = -1;
    (void)hipGetDevice(&dev_now);
    if (dev_now != p->device) (void)hipSetDevice(p->device);
    fdtd_status st;
    if (d.dtype == FDTD_F32)
        st = grad_impl<float, float>(p, E, H, nsteps, src, probe, design_box, ckpt_every, J_out, grad_out);
    else if (d.dtype == FDTD_F64)
        st = grad_impl<double, double>(p, E, H, nsteps, src, probe, design_box, ckpt_every, J_out, grad_out);
    else
        st = grad_impl<float, double>(p, E, H, nsteps, src, probe, design_box, ckpt_every, J_out, grad_out);
    if (dev_now != p->device) (void)hipSetDevice(dev_now);
    return st;
}

fdtd_status fdtd_plan_batch(const fdtd_desc* d, int n, void* hip_stream, fdtd_plan_t* out) {
    if (!d || !out || n < 1) return FDTD_EINVAL;
    *out = nullptr;
    for (int g = 0; g < n; ++g) {
        if (d[g].scheme != d[0].scheme || d[g].form != d[0].form || d[g].dtype != d[0].dtype) return FDTD_EINVAL;
        if (d[g].scheme < 0 || d[g].scheme > 3 || d[g].form < 0 || d[g].form > 1 || d[g].dtype < 0 || d[g].dtype > 3)
            return FDTD_EINVAL;
    }
    if (d[0].form != FDTD_FUNDAMENTAL) return FDTD_EUNSUPPORTED;
    std::vector<fdtd_plan_s*> subs;
    fdtd_status st = FDTD_OK;
    for (int g = 0; g < n && st == FDTD_OK; ++g) {
        fdtd_plan_t sub = nullptr;
        st = fdtd_plan(&d[g], hip_stream, &sub);
        if (st == FDTD_OK) subs.push_back(sub);
    }
    if (st != FDTD_OK) {
        for (fdtd_plan_s* sub : subs) (void)fdtd_destroy(sub);
        return st;
    }
    // per-step working set of each grid: six field arrays and the medium
    std::vector<size_t> bytes(n);
    size_t total = 0;
    for (int g = 0; g < n; ++g) {
        bytes[g] = (size_t)subs[g]->dims.comp * (6 * subs[g]->esz + (subs[g]->mat ? 1 : 4));
        total += bytes[g];
    }
    const int ngroups = (int)std::min<size_t>((size_t)n, (total + kGroupBytes - 1) / kGroupBytes);
    if (ngroups <= 1) return batch_from_subs(d[0], subs, hip_stream, out);
    // consecutive grids, about total / ngroups bytes per group
    fdtd_plan_s* p = new (std::nothrow) fdtd_plan_s();
    Batch* b = p ? new (std::nothrow) Batch() : nullptr;
    if (!b) {
        delete p;
        for (fdtd_plan_s* sub : subs) (void)fdtd_destroy(sub);
        return FDTD_ENOMEM;
    }
    p->batch = b;
    p->d = d[0];
    p->d.eps_r = nullptr;
    if (d[0].dtype == FDTD_F32_REFINE) {
        p->refine = 1;
        p->d.dtype = FDTD_F32;
    }
    p->stream = static_cast<hipStream_t>(hip_stream);
    (void)hipGetDevice(&p->device);
    p->esz = d[0].dtype == FDTD_F64 ? 8 : 4;
    const double target = double(total) / ngroups;
    int g0 = 0;
    double acc = 0.0;
    for (int g = 0; g < n && st == FDTD_OK; ++g) {
        acc += double(bytes[g]);
        const bool last = g == n - 1;
        const int left = ngroups - (int)b->groups.size() - 1;   // groups still to open after this one
        if (last || (acc >= target * (b->groups.size() + 1) && n - 1 - g >= left && left > 0)) {
            std::vector<fdtd_plan_s*> part(subs.begin() + g0, subs.begin() + g + 1);
            fdtd_plan_s* child = nullptr;
            st = batch_from_subs(d[0], part, hip_stream, &child);
            if (st == FDTD_OK) {
                b->groups.push_back(child);
                b->first.push_back(g0);
            } else {
                for (int k = g + 1; k < n; ++k) (void)fdtd_destroy(subs[k]);   // part is freed by batch_from_subs
            }
            g0 = g + 1;
        }
    }
    if (st != FDTD_OK) {
        for (fdtd_plan_s* c : b->groups) (void)fdtd_destroy(c);
        delete b;
        delete p;
        return st;
    }
    for (int ax = 0; ax < 3; ++ax) p->cfg[ax] = b->groups[0]->cfg[ax];
    *out = p;
    return FDTD_OK;
}

fdtd_status fdtd_run_batch(fdtd_plan_t p, void* const* E, void* const* H, int nsteps) {
    if (!plan_ok(p) || !p->batch || !E || !H || nsteps < 0) return FDTD_EINVAL;
    if (!p->batch->groups.empty()) {
        const Batch* b = p->batch;
        const fdtd_plan_s* last = b->groups.back();
        const size_t n = (size_t)b->first.back() + last->batch->subs.size();
        for (size_t m = 0; m < 3 * n; ++m)
            if (!E[m] || !H[m]) return FDTD_EINVAL;
        // one group after the other, each through all its steps
        for (size_t gi = 0; gi < b->groups.size(); ++gi) {
            const fdtd_status st = fdtd_run_batch(b->groups[gi], E + 3 * b->first[gi], H + 3 * b->first[gi], nsteps);
            if (st != FDTD_OK) return st;
        }
        p->step += nsteps;
        return FDTD_OK;
    }
    const size_t n = p->batch->subs.size();
    for (size_t m = 0; m < 3 * n; ++m)
        if (!E[m] || !H[m]) return FDTD_EINVAL;
    int dev_now = -1;
    (void)hipGetDevice(&dev_now);
    if (dev_now != p->device) (void)hipSetDevice(p->device);
    fdtd_status st;
    if (p->d.dtype == FDTD_F32) st = run_batch_impl<float, float>(p, E, H, nsteps);
    else if (p->d.dtype == FDTD_F64) st = run_batch_impl<double, double>(p, E, H, nsteps);
    else st = run_batch_impl<float, double>(p, E, H, nsteps);
    if (dev_now != p->device) (void)hipSetDevice(dev_now);
    return st;
}

fdtd_status fdtd_destroy(fdtd_plan_t p) {
    if (!plan_ok(p)) return FDTD_EINVAL;
    (void)hipStreamSynchronize(p->stream);
    if (p->batch) {
        for (fdtd_plan_s* c : p->batch->groups) (void)fdtd_destroy(c);
        batch_clear(p->batch);
        for (fdtd_plan_s* sub : p->batch->subs) (void)fdtd_destroy(sub);
        if (p->batch->cap) (void)hipStreamDestroy(p->batch->cap);
        for (hipStream_t f : p->batch->fork)
            if (f) (void)hipStreamDestroy(f);
        for (hipEvent_t e : p->batch->ev)
            if (e) (void)hipEventDestroy(e);
        delete p->batch;
        p->batch = nullptr;
    }
    if (p->state) (void)hipFree(p->state);
    if (p->snap) (void)hipFree(p->snap);
    if (p->eps) (void)hipFree(p->eps);
    if (p->partial) (void)hipFree(p->partial);
    if (p->energy_dev) (void)hipFree(p->energy_dev);
    if (p->mat) (void)hipFree(p->mat);
    if (p->mat_eps) (void)hipFree(p->mat_eps);
    if (p->gbuf) (void)hipFree(p->gbuf);
    for (hipEvent_t e : p->tm.ev) (void)hipEventDestroy(e);
    if (p->tm.main0) (void)hipEventDestroy(p->tm.main0);
    if (p->tm.main1) (void)hipEventDestroy(p->tm.main1);
    p->magic = 0;
    delete p;
    return FDTD_OK;
}

}  // extern "C"

namespace fdtd {
static fdtd_status batch_from_subs(const fdtd_desc& d0, const std::vector<fdtd_plan_s*>& subs, void* hip_stream,
                                   fdtd_plan_s** out) {
    *out = nullptr;
    fdtd_plan_s* p = new (std::nothrow) fdtd_plan_s();
    if (p) p->batch = new (std::nothrow) Batch();
    if (!p || !p->batch) {
        delete p;
        for (fdtd_plan_s* sub : subs) (void)fdtd_destroy(sub);
        return FDTD_ENOMEM;
    }
    p->d = d0;
    p->d.eps_r = nullptr;
    if (d0.dtype == FDTD_F32_REFINE) {
        p->refine = 1;
        p->d.dtype = FDTD_F32;
    }
    p->stream = static_cast<hipStream_t>(hip_stream);
    (void)hipGetDevice(&p->device);
    p->esz = d0.dtype == FDTD_F64 ? 8 : 4;
    p->batch->subs = subs;
    fdtd_status st = FDTD_OK;
    if (hipStreamCreateWithFlags(&p->batch->cap, hipStreamNonBlocking) != hipSuccess) st = FDTD_EDEVICE;
    for (int f = 0; f < 2 && st == FDTD_OK; ++f)
        if (hipStreamCreateWithFlags(&p->batch->fork[f], hipStreamNonBlocking) != hipSuccess) st = FDTD_EDEVICE;
    for (int f = 0; f < 3 && st == FDTD_OK; ++f)
        if (hipEventCreateWithFlags(&p->batch->ev[f], hipEventDisableTiming) != hipSuccess) st = FDTD_EDEVICE;
    if (st != FDTD_OK) {
        (void)fdtd_destroy(p);   // destroys the grids, streams and events
        return st;
    }
    bool mat = true;
    for (const fdtd_plan_s* sub : p->batch->subs) mat = mat && sub->mat != nullptr;
    p->batch->mat = mat;
    batch_default_cfg(p);
    *out = p;
    return FDTD_OK;
}
}  // namespace fdtd
