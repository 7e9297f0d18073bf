// fdtd.hip -- the C ABI of libfdtd.so.  The plan state, pass launches,
// autotuner, run loop, adjoint gradient and batch plans live in the headers
// included below, in that order; the line-pass kernels are instantiated in
// kern_inst.hip (pass_dispatch.hpp).
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
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/fdtd.h"
#include "adjoint_kernels.hpp"
#include "aux_kernels.hpp"
#include "cn_kernels.hpp"
#include "order4_kernels.hpp"
#include "pass_dispatch.hpp"
#include "plan_state.hpp"
#include "pass_launch.hpp"
#include "autotune.hpp"
#include "run_loop.hpp"
#include "adjoint_grad.hpp"
#include "batch_plan.hpp"
#include "cn_solver.hpp"

using namespace fdtd;

// Live plans.  A handle is looked up here before it is dereferenced, so a
// destroyed (or never created) handle is rejected with FDTD_EINVAL instead of
// being read.  The set and its lock are never destroyed, so calls made while
// the process ends (finalizers of a binding) still find them.
static std::mutex& plans_mu() {
    static std::mutex* m = new std::mutex();
    return *m;
}
static std::unordered_set<const fdtd_plan_s*>& plans() {
    static auto* s = new std::unordered_set<const fdtd_plan_s*>();
    return *s;
}
static void plan_register(const fdtd_plan_s* p) {
    std::lock_guard<std::mutex> lock(plans_mu());
    plans().insert(p);
}
static void plan_unregister(const fdtd_plan_s* p) {
    std::lock_guard<std::mutex> lock(plans_mu());
    plans().erase(p);
}
static bool plan_ok(fdtd_plan_t p) {
    if (p == nullptr) return false;
    std::lock_guard<std::mutex> lock(plans_mu());
    return plans().count(p) != 0 && p->magic == 0xFD7DFD7Du;
}

// ---------------------------------------------------------------------------
// fdtd_diff_norm and its variant without allocation
// ---------------------------------------------------------------------------
// Device work area of fdtd_diff_norm_noalloc: the partial sums of the
// two-stage reduction and its two results.  Each GPU the library runs on
// holds one copy until the process ends; in host code its address is taken
// per device with hipGetSymbolAddress (scratch_ptr), never from the name.
constexpr int kScratchDoubles = 2 * 1024 + 2;   // 16,400 bytes
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static double* g_scratch[kMaxDevices];   // per device, resolved on first use
static std::mutex g_scratch_mu;

// Address of `scratch` on device `dev` (which must be current).
static fdtd_status scratch_ptr(int dev, double** out) {
    if (dev < 0 || dev >= kMaxDevices) return FDTD_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FDTD_EDEVICE;
        g_scratch[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch[dev];
    return FDTD_OK;
}

// Blocks of the first reduction stage of fdtd_diff_norm: one per 256 nodes,
// at most the plan's npartial (1024).
static int diff_blocks(const fdtd_plan_s* p) {
    const long long nn = (long long)(p->dims.nx + 1) * (p->dims.ny + 1) * (p->dims.nz + 1);
    return (int)std::min<long long>(p->npartial, (nn + 255) / 256);
}
static int diff_work_doubles(const fdtd_plan_s* p) { return 2 * p->npartial + 2; }

// The reduction of fdtd_diff_norm with device work area `work` (2 npartial + 2
// doubles): per-block partials, then the two sums in fixed order.
static fdtd_status diff_norm_impl(fdtd_plan_s* p, void* const Ea[3], void* const Ha[3], void* const Eb[3],
                                  void* const Hb[3], double* out, double* work) {
    const int nb = diff_blocks(p);
    const AuxCoef k = aux_coef(p->d, 0.0);
    auto launch = [&](auto tag) -> fdtd_status {
        using T = decltype(tag);
        FieldPtrs<T> fa, fb;
        for (int c = 0; c < 3; ++c) {
            fa.c[c] = static_cast<const T*>(Ea[c]);
            fa.c[3 + c] = static_cast<const T*>(Ha[c]);
            fb.c[c] = static_cast<const T*>(Eb[c]);
            fb.c[3 + c] = static_cast<const T*>(Hb[c]);
        }
        hipLaunchKernelGGL((diff_partial_kernel<T>), dim3(nb), dim3(256), 0, p->stream, fa, fb, p->eps, p->mu, p->dims, k,
                           work);
        HIPCHK(hipGetLastError());
        return FDTD_OK;
    };
    const fdtd_status st = p->d.dtype == FDTD_F64 ? launch(double()) : launch(float());
    if (st != FDTD_OK) return st;
    double* res = work + 2 * p->npartial;
    for (int m = 0; m < 2; ++m) {
        hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(64), 0, p->stream, work + m * nb, nb, res + m);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(out, res, sizeof(double) * 2, hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    return std::isfinite(out[0]) && std::isfinite(out[1]) ? FDTD_OK : FDTD_ENONFINITE;
}

extern "C" {

const char* fdtd_strerror(fdtd_status s) {
    switch (s) {
        case FDTD_OK: return "ok";
        case FDTD_EINVAL: return "invalid argument";
        case FDTD_ENOMEM: return "device out of memory";
        case FDTD_EDEVICE: return "HIP runtime error";
        case FDTD_EUNSUPPORTED: return "not supported by this library";
        case FDTD_ENONFINITE: return "non-finite energy after stepping";
        case FDTD_ENOTCONVERGED: return "iterative solve not converged";
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
    if (d->scheme < 0 || d->scheme > 6 || d->form < 0 || d->form > 1 || d->dtype < 0 || d->dtype > 4)
        return FDTD_EINVAL;
    const bool cn = d->scheme == FDTD_CRANK_NICOLSON;
    if (cn && d->dtype != FDTD_F64) return FDTD_EUNSUPPORTED;
    // D'Yakonov and Douglas-Gunn: the fundamental ADI iteration (Sec. II-E)
    fdtd_desc as_adi;
    if (d->scheme == FDTD_DYAKONOV || d->scheme == FDTD_DOUGLAS_GUNN) {
        if (d->form != FDTD_FUNDAMENTAL) return FDTD_EUNSUPPORTED;
        as_adi = *d;
        as_adi.scheme = FDTD_ADI;
        d = &as_adi;
    }
    if (d->boundary != 0) return FDTD_EUNSUPPORTED;
    if (d->dtype == FDTD_F32_REFINE && d->form != FDTD_FUNDAMENTAL) return FDTD_EUNSUPPORTED;
    const int nmax = std::max(d->nx, std::max(d->ny, d->nz));
    // register budget (refined solves: 8-slot chunks on at most 64 lanes)
    const bool f32_any = d->dtype == FDTD_F32 || d->dtype == FDTD_F32_PLAIN;
    if (nmax > (f32_any ? 1024 : 512)) return FDTD_EUNSUPPORTED;
    const long long ncells = (long long)d->nx * d->ny * d->nz;
    // eps_r, mu_r per cell (host or device pointers), each > 0 and finite
    auto read_map = [&](const float* src, std::vector<float>& dst) -> bool {
        dst.resize(ncells);
        if (hipMemcpy(dst.data(), src, sizeof(float) * ncells, hipMemcpyDefault) != hipSuccess) return false;
        for (long long c = 0; c < ncells; ++c)
            if (!(dst[c] > 0.0f) || !std::isfinite(dst[c])) return false;
        return true;
    };
    std::vector<float> eps_host, mu_host;
    if (d->eps_r && !read_map(d->eps_r, eps_host)) return FDTD_EINVAL;
    if (d->mu_r) {
        if (!read_map(d->mu_r, mu_host)) return FDTD_EINVAL;
        // a map of ones is unit permeability: the plan runs the mu = mu0 passes
        if (std::all_of(mu_host.begin(), mu_host.end(), [](float v) { return v == 1.0f; })) mu_host.clear();
    }
    const bool has_mu = !mu_host.empty();
    // Variable permeability: line passes with per-row off-diagonals (8-slot
    // chunks, at most 512 cells per axis, no refinement)
    if (has_mu && (d->dtype == FDTD_F32_REFINE || nmax > 512)) return FDTD_EUNSUPPORTED;
    fdtd_plan_s* p = new (std::nothrow) fdtd_plan_s();
    if (!p) return FDTD_ENOMEM;
    p->d = *d;
    p->d.eps_r = nullptr;
    p->d.mu_r = nullptr;
    p->req_dtype = d->dtype;
    if (d->dtype == FDTD_F32_REFINE || (d->dtype == FDTD_F32 && !cn && f32_refine_wanted(*d, has_mu))) {
        p->refine = 1;
        p->d.dtype = FDTD_F32;   // FP32 storage and arithmetic; only the fundamental passes differ
    } else if (d->dtype == FDTD_F32_PLAIN) {
        p->d.dtype = FDTD_F32;
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
        if (p->mu) (void)hipFree(p->mu);
        if (p->partial) (void)hipFree(p->partial);
        if (p->mat) (void)hipFree(p->mat);
        if (p->mat_eps) (void)hipFree(p->mat_eps);
        if (p->cg) (void)hipFree(p->cg);
        if (p->cg_partial) (void)hipFree(p->cg_partial);
        if (p->cg_scal) (void)hipFree(p->cg_scal);
        delete p;
        return st;
    };
    if (std::getenv("FDTD_TEST_FAIL_ALLOC")) return fail(FDTD_ENOMEM);
    hipError_t e;
    if ((e = hipMalloc(&p->state, p->esz * dm.comp * 6 * sets)) != hipSuccess) return fail(from_hip(e));
    if ((e = hipMemset(p->state, 0, p->esz * dm.comp * 6 * sets)) != hipSuccess) return fail(from_hip(e));
    // eps_r (and mu_r) at node indices (owned index, clamped to the last
    // cell), padded rows
    auto node_map = [&](const std::vector<float>& cells) {
        std::vector<float> nm((size_t)dm.comp, 1.0f);
        for (int k = 0; k <= d->nz; ++k)
            for (int j = 0; j <= d->ny; ++j)
                for (int i = 0; i <= d->nx; ++i) {
                    const int kk = std::min(k, d->nz - 1), jj = std::min(j, d->ny - 1), ii = std::min(i, d->nx - 1);
                    nm[(size_t)k * dm.plane + (size_t)j * dm.px + i] =
                        cells.empty() ? 1.0f : cells[((size_t)kk * d->ny + jj) * d->nx + ii];
                }
        return nm;
    };
    const std::vector<float> en = node_map(eps_host);
    if ((e = hipMalloc(&p->eps, sizeof(float) * dm.comp)) != hipSuccess) return fail(from_hip(e));
    if ((e = hipMemcpy(p->eps, en.data(), sizeof(float) * dm.comp, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(from_hip(e));
    if (has_mu) {
        const std::vector<float> mn = node_map(mu_host);
        if ((e = hipMalloc(&p->mu, sizeof(float) * dm.comp)) != hipSuccess) return fail(from_hip(e));
        if ((e = hipMemcpy(p->mu, mn.data(), sizeof(float) * dm.comp, hipMemcpyHostToDevice)) != hipSuccess)
            return fail(from_hip(e));
    }
    // Piecewise-constant media: at most 256 distinct eps_r values are stored as
    // a one-byte material index per node (the passes then read 17 instead of
    // 20 bytes per FP32 slot); the table of values lives in LDS.  Plans with a
    // permeability map read both maps instead.
    if (!has_mu && !std::getenv("FDTD_NO_MATERIAL_INDEX")) {
        // distinct values, sorted; the scan stops at the 257th
        std::vector<float> uniq{1.0f};
        float last = 1.0f;
        for (float v : eps_host) {
            if (v == last) continue;   // runs of one value (boxes) cost one comparison
            last = v;
            auto it = std::lower_bound(uniq.begin(), uniq.end(), v);
            if (it != uniq.end() && *it == v) continue;
            uniq.insert(it, v);
            if (uniq.size() > 256) break;
        }
        if (uniq.size() <= 256) {
            std::vector<unsigned char> idx((size_t)dm.comp);
            float lv = uniq[0];
            unsigned char li = 0;
            for (size_t m = 0; m < idx.size(); ++m) {
                if (en[m] != lv) {
                    lv = en[m];
                    li = (unsigned char)(std::lower_bound(uniq.begin(), uniq.end(), lv) - uniq.begin());
                }
                idx[m] = li;
            }
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
    if (cn) {
        const size_t bytes = sizeof(double) * 15 * (size_t)dm.comp;
        if ((e = hipMalloc(&p->cg, bytes)) != hipSuccess) return fail(from_hip(e));
        if ((e = hipMemset(p->cg, 0, bytes)) != hipSuccess) return fail(from_hip(e));
        if ((e = hipMalloc(&p->cg_partial, sizeof(double) * 3 * kCnBlocks)) != hipSuccess) return fail(from_hip(e));
        if ((e = hipMalloc(&p->cg_scal, sizeof(double) * kCnScalars)) != hipSuccess) return fail(from_hip(e));
        if ((e = hipMemset(p->cg_scal, 0, sizeof(double) * kCnScalars)) != hipSuccess) return fail(from_hip(e));
    }
    plan_register(p);
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
    if (p->cg) st = cn_run_impl(p, E, H, nsteps, src, energy, energy_every);
    else if (p->d.dtype == FDTD_F32) st = run_impl<float, float>(p, E, H, nsteps, src, energy, energy_every);
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

fdtd_status fdtd_set_graph(fdtd_plan_t p, int steps) {
    if (!plan_ok(p) || p->batch || steps < 0 || steps > 64) return FDTD_EINVAL;
    if (p->cg) return FDTD_EUNSUPPORTED;   // Crank-Nicolson: no line passes
    if (steps != p->graph_steps) {
        (void)hipStreamSynchronize(p->stream);
        graph_clear(p);
        p->graph_steps = steps;
    }
    return FDTD_OK;
}

// Storage and solve kind of a plan's order-4 passes.  They have no refined
// solves, and plain FP32 solves of their band-3 systems drift linearly with
// the step count (after 1000 steps at 128^3: up to 1.4e-3 at CFL 10 and
// 1.6e-4 at CFL 5 or 1.3e-4 at CFL 1, against 1.4e-6 with FP64 solves), so FDTD_F32, the
// library's choice for FP32 fields, solves them in FP64; FDTD_F32_PLAIN keeps
// FP32 solves.
static int order4_dtype(const fdtd_plan_s* p) {
    return p->req_dtype == FDTD_F32 ? int(FDTD_F32_F64SOLVE) : p->d.dtype;
}

fdtd_status fdtd_set_order(fdtd_plan_t p, int order) {
    if (!plan_ok(p) || p->batch || (order != 2 && order != 4)) return FDTD_EINVAL;
    if (order == p->order) return FDTD_OK;
    if (order == 4) {
        // fundamental forms of the line-pass schemes, unit permeability, no
        // refined solves
        if (p->cg || p->d.form != FDTD_FUNDAMENTAL || p->mu || p->req_dtype == FDTD_F32_REFINE)
            return FDTD_EUNSUPPORTED;
        if (!p->scr4) {
            // per pair pass: the work area of the kernel (y and the
            // factorization state at segment starts) for the largest of the
            // three line families (at most (n + 1)^2 lines of each)
            const bool fsolve = order4_dtype(p) == FDTD_F32;
            const size_t ssz = fsolve ? sizeof(float) : sizeof(double);
            const int K = fsolve ? seg4<float>() : seg4<double>();
            const long long n1[3] = {p->d.nx + 1LL, p->d.ny + 1LL, p->d.nz + 1LL};
            size_t region = 0;
            for (int w = 0; w < 3; ++w)
                region = std::max(region, (size_t)work4_words(int(n1[w] - 1), n1[(w + 1) % 3] * n1[(w + 2) % 3], K));
            if (hipMalloc(&p->scr4, ssz * 3 * region) != hipSuccess) {
                p->scr4 = nullptr;
                return FDTD_ENOMEM;
            }
            p->scr4_region = region;
        }
        if (!p->tr4) {
            // x lines run on a transposed copy of their pair: planes of nx + 1
            // rows of ny + 1 samples (rows padded to 128 bytes); the medium's
            // copy is made here, once
            const Dims& dm = p->dims;
            const long long align = p->esz == 8 ? 16 : 32;
            const long long pitch = ((dm.ny + 1 + align - 1) / align) * align;
            const long long plane = (long long)(dm.nx + 1) * pitch;
            const size_t compt = (size_t)plane * (dm.nz + 1);
            const size_t msz = p->mat ? 1 : sizeof(float);
            if (hipMalloc(&p->tr4, 2 * compt * p->esz) != hipSuccess) {
                p->tr4 = nullptr;
                return FDTD_ENOMEM;
            }
            if (hipMalloc(&p->tr4_med, compt * msz) != hipSuccess) {
                (void)hipFree(p->tr4);
                p->tr4 = p->tr4_med = nullptr;
                return FDTD_ENOMEM;
            }
            p->tr4_pitch = pitch;
            p->tr4_plane = plane;
            if (p->mat)
                hipLaunchKernelGGL((transpose_planes_kernel<unsigned char>),
                                   transpose_grid<unsigned char>(dm.ny + 1, dm.nx + 1, dm.nz + 1), dim3(256), 0,
                                   p->stream, p->mat,
                                   dm.plane, (long long)dm.px, static_cast<unsigned char*>(p->tr4_med), plane, pitch,
                                   dm.ny + 1, dm.nx + 1);
            else
                hipLaunchKernelGGL((transpose_planes_kernel<float>), transpose_grid<float>(dm.ny + 1, dm.nx + 1, dm.nz + 1),
                                   dim3(256), 0, p->stream, p->eps, dm.plane,
                                   (long long)dm.px, static_cast<float*>(p->tr4_med), plane, pitch, dm.ny + 1,
                                   dm.nx + 1);
            if (hipGetLastError() != hipSuccess || hipStreamSynchronize(p->stream) != hipSuccess) return FDTD_EDEVICE;
        }
    }
    (void)hipStreamSynchronize(p->stream);
    graph_clear(p);
    p->order = order;
    p->d.dtype = order == 4 ? order4_dtype(p) : (p->req_dtype == FDTD_F64 || p->req_dtype == FDTD_F32_F64SOLVE
                                                      ? p->req_dtype
                                                      : int(FDTD_F32));
    // refined solves exist for the second-order passes only
    p->refine = (order == 2 && (p->req_dtype == FDTD_F32_REFINE ||
                                (p->req_dtype == FDTD_F32 && f32_refine_wanted(p->d, p->mu != nullptr))))
                    ? 1
                    : 0;
    return FDTD_OK;
}

fdtd_status fdtd_set_stencil(fdtd_plan_t p, double outer) {
    if (!plan_ok(p) || p->batch || !std::isfinite(outer) || std::fabs(outer) > 0.25) return FDTD_EINVAL;
    if (p->order != 4) return FDTD_EUNSUPPORTED;
    if (outer == p->stencil_wo) return FDTD_OK;
    (void)hipStreamSynchronize(p->stream);
    graph_clear(p);
    p->stencil_wo = outer;
    return FDTD_OK;
}

fdtd_status fdtd_stencil_optimized(double theta_max, double* outer) {
    if (!outer || !(theta_max > 0.0) || !(theta_max <= M_PI)) return FDTD_EINVAL;
    // b = -<e0, g> / <g, g> over [0, theta_max], e0 = 2 sin(t/2) - t,
    // g = 2 sin(3t/2) - 6 sin(t/2): composite 8-point Gauss-Legendre rule on
    // 64 panels (the integrands are smooth)
    static const double x8[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
    static const double w8[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
    const int panels = 64;
    const double hp = theta_max / panels;
    double num = 0.0, den = 0.0;
    for (int m = 0; m < panels; ++m) {
        const double c = (m + 0.5) * hp;
        for (int t = 0; t < 8; ++t) {
            const double th = c + 0.5 * hp * (t < 4 ? -x8[t] : x8[t - 4]);
            const double wt = 0.5 * hp * w8[t < 4 ? t : t - 4];
            const double e0 = 2.0 * std::sin(0.5 * th) - th;
            const double g = 2.0 * std::sin(1.5 * th) - 6.0 * std::sin(0.5 * th);
            num += wt * e0 * g;
            den += wt * g * g;
        }
    }
    *outer = -num / den;
    return FDTD_OK;
}

fdtd_status fdtd_get_refined(fdtd_plan_t p, int* refined) {
    if (!plan_ok(p) || !refined) return FDTD_EINVAL;
    *refined = p->refine;
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
    if (p->cg) return FDTD_EUNSUPPORTED;   // Crank-Nicolson: no line passes
    if (p->order == 4) {
        // one launch shape (a thread per line): nothing to tune
        p->tuned = 1;
        if (best_ms) best_ms[0] = best_ms[1] = best_ms[2] = 0.0;
        return FDTD_OK;
    }
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
    if (p->cg) return FDTD_EUNSUPPORTED;
    const KCfg& k = p->cfg[axis];
    c->chunk = k.M;
    c->tile_x = axis == 0 ? 0 : k.TX;
    c->block_threads = axis == 0 ? 64 * k.wpb : k.NT;
    c->remap = k.remap;
    return FDTD_OK;
}

fdtd_status fdtd_set_kernel_config(fdtd_plan_t p, int axis, const fdtd_kernel_config* c) {
    if (!plan_ok(p) || axis < 0 || axis > 2 || !c) return FDTD_EINVAL;
    if (p->cg) return FDTD_EUNSUPPORTED;
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
        if (d[g].scheme < 0 || d[g].scheme > 6 || d[g].form < 0 || d[g].form > 1 || d[g].dtype < 0 || d[g].dtype > 4)
            return FDTD_EINVAL;
    }
    if (d[0].form != FDTD_FUNDAMENTAL || d[0].scheme == FDTD_CRANK_NICOLSON) return FDTD_EUNSUPPORTED;
    // D'Yakonov and Douglas-Gunn batches step as ADI (no sources in a batch)
    std::vector<fdtd_desc> as_adi;
    if (d[0].scheme == FDTD_DYAKONOV || d[0].scheme == FDTD_DOUGLAS_GUNN) {
        as_adi.assign(d, d + n);
        for (fdtd_desc& x : as_adi) x.scheme = FDTD_ADI;
        d = as_adi.data();
    }
    std::vector<fdtd_plan_s*> subs;
    fdtd_status st = FDTD_OK;
    for (int g = 0; g < n && st == FDTD_OK; ++g) {
        fdtd_plan_t sub = nullptr;
        st = fdtd_plan(&d[g], hip_stream, &sub);
        if (st == FDTD_OK) subs.push_back(sub);
    }
    // batched passes take unit permeability
    for (const fdtd_plan_s* sub : subs)
        if (sub->mu) st = FDTD_EUNSUPPORTED;
    if (st != FDTD_OK) {
        for (fdtd_plan_s* sub : subs) (void)fdtd_destroy(sub);
        return st;
    }
    // one launch serves every grid: an FDTD_F32 batch refines all its grids'
    // solves if any grid needs it (refinement never loses accuracy)
    bool any_refine = false;
    for (const fdtd_plan_s* sub : subs) any_refine = any_refine || sub->refine;
    for (fdtd_plan_s* sub : subs) sub->refine = any_refine ? 1 : 0;
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
    p->d = subs[0]->d;
    p->req_dtype = d[0].dtype;
    p->refine = any_refine ? 1 : 0;
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
    plan_register(p);
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

fdtd_status fdtd_diff_norm(fdtd_plan_t p, void* const Ea[3], void* const Ha[3], void* const Eb[3],
                           void* const Hb[3], double* out) {
    if (!plan_ok(p) || p->batch || !Ea || !Ha || !Eb || !Hb || !out) return FDTD_EINVAL;
    for (int c = 0; c < 3; ++c)
        if (!Ea[c] || !Ha[c] || !Eb[c] || !Hb[c]) return FDTD_EINVAL;
    int dev_now = -1;
    (void)hipGetDevice(&dev_now);
    if (dev_now != p->device) (void)hipSetDevice(p->device);
    fdtd_status st = FDTD_OK;
    if (!p->diff_dev && hipMalloc(&p->diff_dev, sizeof(double) * diff_work_doubles(p)) != hipSuccess)
        st = FDTD_ENOMEM;
    if (st == FDTD_OK) st = diff_norm_impl(p, Ea, Ha, Eb, Hb, out, p->diff_dev);
    if (dev_now != p->device) (void)hipSetDevice(dev_now);
    return st;
}

fdtd_status fdtd_diff_norm_noalloc(fdtd_plan_t p, void* const Ea[3], void* const Ha[3], void* const Eb[3],
                                   void* const Hb[3], double* out) {
    if (!plan_ok(p) || p->batch || !Ea || !Ha || !Eb || !Hb || !out) return FDTD_EINVAL;
    for (int c = 0; c < 3; ++c)
        if (!Ea[c] || !Ha[c] || !Eb[c] || !Hb[c]) return FDTD_EINVAL;
    if (diff_work_doubles(p) > kScratchDoubles) return FDTD_EINVAL;   // never: at most 2 * 1024 + 2
    int dev_now = -1;
    (void)hipGetDevice(&dev_now);
    if (dev_now != p->device) (void)hipSetDevice(p->device);
    double* work = nullptr;
    fdtd_status st = scratch_ptr(p->device, &work);
    if (st == FDTD_OK) st = diff_norm_impl(p, Ea, Ha, Eb, Hb, out, work);
    if (dev_now != p->device) (void)hipSetDevice(dev_now);
    return st;
}

fdtd_status fdtd_set_cg(fdtd_plan_t p, double tol, int maxit) {
    if (!plan_ok(p) || !(tol > 0.0 && tol < 1.0) || maxit < 1) return FDTD_EINVAL;
    if (!p->cg) return FDTD_EUNSUPPORTED;
    p->cg_tol = tol;
    p->cg_maxit = maxit;
    return FDTD_OK;
}

fdtd_status fdtd_last_cg(fdtd_plan_t p, long long* iterations, double* rel_residual) {
    if (!plan_ok(p)) return FDTD_EINVAL;
    if (!p->cg) return FDTD_EUNSUPPORTED;
    if (iterations) *iterations = p->cg_iters;
    if (rel_residual) *rel_residual = p->cg_rel;
    return FDTD_OK;
}

fdtd_status fdtd_destroy(fdtd_plan_t p) {
    if (!plan_ok(p)) return FDTD_EINVAL;
    plan_unregister(p);
    (void)hipStreamSynchronize(p->stream);
    if (p->batch) {
        for (fdtd_plan_s* c : p->batch->groups) (void)fdtd_destroy(c);
        batch_clear(p->batch);
        for (fdtd_plan_s* sub : p->batch->subs) (void)fdtd_destroy(sub);
        if (p->batch->cap) (void)hipStreamDestroy(p->batch->cap);
        delete p->batch;
        p->batch = nullptr;
    }
    graph_clear(p);
    if (p->gstream) (void)hipStreamDestroy(p->gstream);
    if (p->src_copied) (void)hipEventDestroy(p->src_copied);
    if (p->src_dev) (void)hipFree(p->src_dev);
    if (p->src_win) (void)hipFree(p->src_win);
    if (p->src_host) (void)hipHostFree(p->src_host);
    if (p->state) (void)hipFree(p->state);
    if (p->snap) (void)hipFree(p->snap);
    if (p->eps) (void)hipFree(p->eps);
    if (p->mu) (void)hipFree(p->mu);
    if (p->scr4) (void)hipFree(p->scr4);
    if (p->tr4) (void)hipFree(p->tr4);
    if (p->tr4_med) (void)hipFree(p->tr4_med);
    if (p->partial) (void)hipFree(p->partial);
    if (p->energy_dev) (void)hipFree(p->energy_dev);
    if (p->mat) (void)hipFree(p->mat);
    if (p->mat_eps) (void)hipFree(p->mat_eps);
    if (p->gbuf) (void)hipFree(p->gbuf);
    if (p->cg) (void)hipFree(p->cg);
    if (p->cg_partial) (void)hipFree(p->cg_partial);
    if (p->cg_scal) (void)hipFree(p->cg_scal);
    if (p->diff_dev) (void)hipFree(p->diff_dev);
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
    plan_register(p);   // from here on fdtd_destroy releases it
    p->d = subs[0]->d;   // storage/solve kind as normalized by fdtd_plan
    p->req_dtype = d0.dtype;
    p->refine = subs[0]->refine;   // equal for all grids (fdtd_plan_batch)
    p->stream = static_cast<hipStream_t>(hip_stream);
    (void)hipGetDevice(&p->device);
    p->esz = d0.dtype == FDTD_F64 ? 8 : 4;
    p->batch->subs = subs;
    fdtd_status st = FDTD_OK;
    if (hipStreamCreateWithFlags(&p->batch->cap, hipStreamNonBlocking) != hipSuccess) st = FDTD_EDEVICE;
    if (st != FDTD_OK) {
        (void)fdtd_destroy(p);   // destroys the grids and the stream
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
