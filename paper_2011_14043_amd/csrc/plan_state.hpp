// plan_state.hpp -- plan state: physical constants, scheme tables, kernel configurations, batch
// bookkeeping and the plan object
//
// Part of the single translation unit of libfdtd.so: included by fdtd.hip
// after the kernel headers and the headers before it in fdtd.hip.
#pragma once

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

// Does an FDTD_F32 plan of `d` (scheme already mapped to a line-pass scheme)
// refine its solves?  Wherever refined passes are built: fundamental forms, at
// most 512 cells per axis, unit permeability.  Plain FP32 solves carry two
// fixed roundings at every step: of the diagonal 2 + sigma (a relative
// perturbation of up to 1.2e-7 / sigma of the medium, whose phase error grows
// linearly with the step count: 3e-4 after 1000 steps at sigma = 0.12) and of
// the medium-only factors (an amplification slightly off unit modulus,
// whatever sigma: 4e-5 to 6e-5 after 1000 steps at sigma = 12 as at 0.48).
// One refinement step removes both for 1 % to 3 % of the step time.
static bool f32_refine_wanted(const fdtd_desc& d, bool has_mu) {
    if (d.form != FDTD_FUNDAMENTAL || has_mu) return false;
    return std::max(d.nx, std::max(d.ny, d.nz)) <= 512;
}

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
// Plans with a permeability map (per-row off-diagonals, more registers per
// slot): x lines with 8-slot chunks; these y/z variants (16-slot chunks for
// FP32 solves only).
static const int kYzMuF32[][3] = {{16, 16, 512}, {8, 16, 512}, {8, 8, 512}};
static const int kYzMuF64[][3] = {{8, 16, 512}, {8, 8, 512}};

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
    int op = 0;
    int mask = 0;             // pairs k of operator op in this launch (bit k): the x pair, y/z
                              // pairs of one kernel configuration, or all three (fused)
    int w = 0;                // line axis of the first pair (selects the configuration); a fused
                              // launch has its y/z pairs first
    int ex0 = -1;             // fused launch: first x-line entry of tab; -1 otherwise
    int threads = 0;          // threads per block
    double frac = 0.0;        // theta = frac * dt of each grid
    void* tab = nullptr;      // device PassArgs<T, S>[ngrids x pairs in mask], pair-major
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
    void* snap = nullptr;     // grid of an ADI batch: state before the last B sub-step
    float* eps = nullptr;     // node layout, padded
    float* mu = nullptr;      // mu_r in node layout (plans with a permeability map; else NULL)
    int order = 2;            // accuracy order of the staggered differences (fdtd_set_order: 2 or 4)
    double stencil_wo = -1.0 / 24.0;   // order 4: outer weight of the 4-point difference (fdtd_set_stencil)
    void* scr4 = nullptr;     // order 4: line-solve work area, 3 pairs x scr4_region words (solve type)
    size_t scr4_region = 0;   // words per pair: y and the factorization state at segment starts
    void* tr4 = nullptr;      // order 4, x lines: the pair (E, H) transposed, x the slow axis of a plane
    void* tr4_med = nullptr;  // the medium in that layout (material index, else eps_r), made once
    long long tr4_pitch = 0;  // row pitch (elements) of that layout: ny + 1 padded to 128 bytes
    long long tr4_plane = 0;  // plane size: (nx + 1) rows
    unsigned char* mat = nullptr;   // material index per node (if <= 256 distinct eps_r)
    // Crank-Nicolson plans: 15 work components (x, r, p, q on E; w on H),
    // 3 x 1024 partial sums, scalars; CG controls and the last run's statistics
    double* cg = nullptr;
    double* cg_partial = nullptr;
    double* cg_scal = nullptr;
    double cg_tol = 1e-12;
    int cg_maxit = 500;
    long long cg_iters = 0;
    double cg_rel = 0.0;
    float* mat_eps = nullptr;       // eps_r per material
    int nmat = 0;
    double* partial = nullptr;
    int npartial = 0;
    double* energy_dev = nullptr;
    int energy_cap = 0;
    double* diff_dev = nullptr;   // fdtd_diff_norm: 2 x npartial partials and 2 results (on first use)
    void* gbuf = nullptr;     // adjoint: checkpoints, records, adjoint state (grown on demand)
    size_t gcap = 0;
    long long step = 0;
    fdtd::Timing tm;
    fdtd::KCfg cfg[3];        // per line axis x, y, z
    int tuned = 0;
    int refine = 0;           // FP32 fundamental passes refine each solve once (FDTD_F32_REFINE, or
                              // FDTD_F32 where refined passes are built)
    int req_dtype = 0;        // the dtype the caller asked for (d.dtype holds the storage/solve kind)
    double last_main_ms = 0.0;
    double fam_ms[2] = {0, 0};
    int fam_n[2] = {0, 0};
    fdtd::Batch* batch = nullptr;   // batch plan: the grids and their tables
    // Single-grid runs: main-iteration steps captured as a HIP graph of
    // graph_steps steps (0, the default: no graphs), replayed on the plan's
    // stream.  The
    // source values of every sub-step of a run are computed on the host into
    // the pinned table src_host, copied once to src_dev, and each replay
    // first copies its window of src_dev into src_win, which the captured
    // passes read.
    int graph_steps = 0;
    hipStream_t gstream = nullptr;        // private capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    long long gkey[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // what the captured graph depends on
    double* src_dev = nullptr;            // [steps][sub-steps][pre xyz, post xyz]
    double* src_win = nullptr;            // one graph's window of src_dev
    double* src_host = nullptr;           // pinned staging of src_dev
    size_t src_cap = 0;                   // doubles in src_dev and src_host
    hipEvent_t src_copied = nullptr;      // the last staging copy has been read
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

}  // namespace fdtd
