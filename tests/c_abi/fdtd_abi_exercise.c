/*
 * fdtd_abi_exercise.c -- every entry point of include/fdtd.h, called from
 * plain C, for the host-sanitized build of the library (host code compiled
 * with AddressSanitizer and UndefinedBehaviorSanitizer; device code as in the
 * product build).  The program checks status codes and that results are
 * finite; the numerics are checked elsewhere against the oracle.
 *
 *   fdtd_abi_exercise host   argument checks that return before any device
 *                            work (runs without a GPU)
 *   fdtd_abi_exercise        those, then plans, runs, graphs, timing, kernel
 *                            configurations, the autotuner and its cache,
 *                            permeability maps, fourth-order and optimized
 *                            stencils, Crank-Nicolson, the adjoint gradient,
 *                            distances (allocating and not) and batches, with
 *                            the error paths of each
 *
 * Prints one JSON line {"checks": n, "failures": m}; exit status 0 when every
 * check holds, 1 otherwise, 2 on a setup error (HIP allocation or copy).  The
 * leak check runs before the end of main, which then ends the process
 * directly.
 */
#define _POSIX_C_SOURCE 200809L
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <sanitizer/lsan_interface.h>

#include "fdtd.h"

static int nchk = 0, nfail = 0;

#define EXPECT(expr, want)                                                                              \
    do {                                                                                                \
        const fdtd_status s_ = (expr);                                                                  \
        ++nchk;                                                                                         \
        if (s_ != (want)) {                                                                             \
            ++nfail;                                                                                    \
            fprintf(stderr, "line %d: %s -> %s, expected %s\n", __LINE__, #expr, fdtd_strerror(s_),     \
                    fdtd_strerror(want));                                                               \
        }                                                                                               \
    } while (0)

#define TRUE(cond)                                                            \
    do {                                                                      \
        ++nchk;                                                               \
        if (!(cond)) {                                                        \
            ++nfail;                                                          \
            fprintf(stderr, "line %d: %s does not hold\n", __LINE__, #cond);  \
        }                                                                     \
    } while (0)

#define SETUP(call)                                                                   \
    do {                                                                              \
        if ((call) != hipSuccess) {                                                   \
            fprintf(stderr, "line %d: %s failed\n", __LINE__, #call);                 \
            exit(2);                                                                  \
        }                                                                             \
    } while (0)

static unsigned long long lcg = 0x9E3779B97F4A7C15ull;
static double unif(void) {   /* xorshift64, in [-1, 1) */
    lcg ^= lcg << 13;
    lcg ^= lcg >> 7;
    lcg ^= lcg << 17;
    return (double)(lcg >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static const double C0 = 299792458.0;
static const double PI = 3.14159265358979323846;

static fdtd_desc desc(int nx, int ny, int nz, double cfl, int scheme, int form, int dtype) {
    fdtd_desc d;
    const double h = 1e-3;
    d.nx = nx; d.ny = ny; d.nz = nz;
    d.dx = h; d.dy = h; d.dz = h;
    d.dt = cfl / (C0 * sqrt(3.0 / (h * h)));
    d.scheme = scheme; d.form = form; d.dtype = dtype;
    d.eps_r = NULL; d.mu_r = NULL;
    d.boundary = 0;
    return d;
}

/* ------------------------------------------------------------------ host */

static void host_checks(void) {
    fdtd_plan_t p = NULL;
    fdtd_desc d = desc(8, 8, 8, 2.0, FDTD_ADI, FDTD_FUNDAMENTAL, FDTD_F32);
    double b = 0.0;

    for (int s = -7; s <= 1; ++s) TRUE(fdtd_strerror((fdtd_status)s) != NULL);

    EXPECT(fdtd_plan(NULL, NULL, &p), FDTD_EINVAL);
    EXPECT(fdtd_plan(&d, NULL, NULL), FDTD_EINVAL);
    EXPECT(fdtd_plan_batch(NULL, 1, NULL, &p), FDTD_EINVAL);
    EXPECT(fdtd_plan_batch(&d, 0, NULL, &p), FDTD_EINVAL);
    EXPECT(fdtd_run(NULL, NULL, NULL, 1, NULL, NULL, 1), FDTD_EINVAL);
    EXPECT(fdtd_step(NULL, NULL, NULL, NULL), FDTD_EINVAL);
    EXPECT(fdtd_run_batch(NULL, NULL, NULL, 1), FDTD_EINVAL);
    EXPECT(fdtd_set_step(NULL, 0), FDTD_EINVAL);
    EXPECT(fdtd_set_graph(NULL, 2), FDTD_EINVAL);
    EXPECT(fdtd_set_order(NULL, 4), FDTD_EINVAL);
    EXPECT(fdtd_set_stencil(NULL, -0.05), FDTD_EINVAL);
    EXPECT(fdtd_get_refined(NULL, NULL), FDTD_EINVAL);
    EXPECT(fdtd_set_timing(NULL, 1), FDTD_EINVAL);
    EXPECT(fdtd_last_timing(NULL, NULL, NULL, NULL), FDTD_EINVAL);
    EXPECT(fdtd_get_kernel_config(NULL, 0, NULL), FDTD_EINVAL);
    EXPECT(fdtd_set_kernel_config(NULL, 0, NULL), FDTD_EINVAL);
    EXPECT(fdtd_autotune(NULL, 1, NULL), FDTD_EINVAL);
    EXPECT(fdtd_grad_eps(NULL, NULL, NULL, 1, NULL, 1, 1, 1, NULL, 1, NULL, NULL), FDTD_EINVAL);
    EXPECT(fdtd_diff_norm(NULL, NULL, NULL, NULL, NULL, NULL), FDTD_EINVAL);
    EXPECT(fdtd_diff_norm_noalloc(NULL, NULL, NULL, NULL, NULL, NULL), FDTD_EINVAL);
    EXPECT(fdtd_set_cg(NULL, 1e-10, 10), FDTD_EINVAL);
    EXPECT(fdtd_last_cg(NULL, NULL, NULL), FDTD_EINVAL);
    EXPECT(fdtd_destroy(NULL), FDTD_EINVAL);

    /* descriptors rejected before any device work */
    {
        struct { int field, value, want; } bad[] = {
            {0, 1, FDTD_EINVAL},  {1, 0, FDTD_EINVAL},  {2, -3, FDTD_EINVAL}, {3, 8, FDTD_EINVAL},
            {3, -1, FDTD_EINVAL}, {4, 2, FDTD_EINVAL},  {5, 7, FDTD_EINVAL},  {5, 5, FDTD_EINVAL},
            {6, 1, FDTD_EUNSUPPORTED}, {0, 2000, FDTD_EUNSUPPORTED},
        };
        for (size_t n = 0; n < sizeof bad / sizeof bad[0]; ++n) {
            fdtd_desc e = d;
            switch (bad[n].field) {
                case 0: e.nx = bad[n].value; break;
                case 1: e.ny = bad[n].value; break;
                case 2: e.nz = bad[n].value; break;
                case 3: e.scheme = bad[n].value; break;
                case 4: e.form = bad[n].value; break;
                case 5: e.dtype = bad[n].value; break;
                default: e.boundary = bad[n].value; break;
            }
            p = (fdtd_plan_t)&e;   /* must come back NULL */
            EXPECT(fdtd_plan(&e, NULL, &p), (fdtd_status)bad[n].want);
            TRUE(p == NULL);
        }
        fdtd_desc e = d;
        e.dt = 0.0;
        EXPECT(fdtd_plan(&e, NULL, &p), FDTD_EINVAL);
        e.dt = NAN;
        EXPECT(fdtd_plan(&e, NULL, &p), FDTD_EINVAL);
        e = d;
        e.dz = INFINITY;
        EXPECT(fdtd_plan(&e, NULL, &p), FDTD_EINVAL);
        e = desc(8, 8, 8, 2.0, FDTD_DYAKONOV, FDTD_CONVENTIONAL, FDTD_F32);
        EXPECT(fdtd_plan(&e, NULL, &p), FDTD_EUNSUPPORTED);
        e = desc(8, 8, 8, 2.0, FDTD_CRANK_NICOLSON, FDTD_FUNDAMENTAL, FDTD_F32);
        EXPECT(fdtd_plan(&e, NULL, &p), FDTD_EUNSUPPORTED);
        e = desc(8, 8, 8, 2.0, FDTD_ADI, FDTD_CONVENTIONAL, FDTD_F32_REFINE);
        EXPECT(fdtd_plan(&e, NULL, &p), FDTD_EUNSUPPORTED);
        e = desc(8, 600, 8, 2.0, FDTD_ADI, FDTD_FUNDAMENTAL, FDTD_F64);
        EXPECT(fdtd_plan(&e, NULL, &p), FDTD_EUNSUPPORTED);
    }

    /* forced allocation failure */
    setenv("FDTD_TEST_FAIL_ALLOC", "1", 1);
    EXPECT(fdtd_plan(&d, NULL, &p), FDTD_ENOMEM);
    TRUE(p == NULL);
    unsetenv("FDTD_TEST_FAIL_ALLOC");

    /* the least-squares outer weight */
    EXPECT(fdtd_stencil_optimized(0.0, &b), FDTD_EINVAL);
    EXPECT(fdtd_stencil_optimized(-1.0, &b), FDTD_EINVAL);
    EXPECT(fdtd_stencil_optimized(4.0, &b), FDTD_EINVAL);
    EXPECT(fdtd_stencil_optimized(NAN, &b), FDTD_EINVAL);
    EXPECT(fdtd_stencil_optimized(1.0, NULL), FDTD_EINVAL);
    EXPECT(fdtd_stencil_optimized(PI / 2, &b), FDTD_OK);
    TRUE(b < -0.0515 && b > -0.0519);
    EXPECT(fdtd_stencil_optimized(1e-3, &b), FDTD_OK);
    TRUE(fabs(b + 1.0 / 24.0) < 1e-6);   /* small bands: the fourth-order weight */
}

/* ---------------------------------------------------------------- device */

typedef struct {
    void* E[3];
    void* H[3];
    size_t n;
    int esz;
} fset;

static void fset_alloc(fset* f, int nx, int ny, int nz, int esz) {
    f->n = (size_t)(nx + 1) * (ny + 1) * (nz + 1);
    f->esz = esz;
    void* host = malloc(f->n * (size_t)esz);
    if (!host) exit(2);
    for (int c = 0; c < 6; ++c) {
        const double scale = c < 3 ? 1.0 : 1.0 / 377.0;
        for (size_t i = 0; i < f->n; ++i) {
            const double v = unif() * scale;
            if (esz == 8) ((double*)host)[i] = v;
            else ((float*)host)[i] = (float)v;
        }
        void** dst = c < 3 ? &f->E[c] : &f->H[c - 3];
        SETUP(hipMalloc(dst, f->n * (size_t)esz));
        SETUP(hipMemcpy(*dst, host, f->n * (size_t)esz, hipMemcpyHostToDevice));
    }
    free(host);
}

static void fset_copy(fset* dst, const fset* src) {
    for (int c = 0; c < 3; ++c) {
        SETUP(hipMemcpy(dst->E[c], src->E[c], src->n * (size_t)src->esz, hipMemcpyDeviceToDevice));
        SETUP(hipMemcpy(dst->H[c], src->H[c], src->n * (size_t)src->esz, hipMemcpyDeviceToDevice));
    }
}

static void fset_free(fset* f) {
    for (int c = 0; c < 3; ++c) {
        (void)hipFree(f->E[c]);
        (void)hipFree(f->H[c]);
    }
}

/* every sample of the six arrays is finite */
static int fset_finite(const fset* f) {
    void* host = malloc(f->n * (size_t)f->esz);
    int ok = host != NULL;
    for (int c = 0; c < 6 && ok; ++c) {
        SETUP(hipMemcpy(host, c < 3 ? f->E[c] : f->H[c - 3], f->n * (size_t)f->esz, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < f->n && ok; ++i)
            ok = f->esz == 8 ? isfinite(((double*)host)[i]) : isfinite(((float*)host)[i]);
    }
    free(host);
    return ok;
}

static int elem_size(int dtype) { return dtype == FDTD_F64 ? 8 : 4; }

static float* random_map(int nx, int ny, int nz, float lo, float hi) {
    const size_t n = (size_t)nx * ny * nz;
    float* m = (float*)malloc(sizeof(float) * n);
    if (!m) exit(2);
    for (size_t c = 0; c < n; ++c) m[c] = lo + (hi - lo) * (float)(0.5 * (unif() + 1.0));
    return m;
}

static fdtd_source source_for(const fdtd_desc* d) {
    fdtd_source s;
    s.i = d->nx / 2; s.j = d->ny / 2; s.k = d->nz / 2;
    s.f0 = 1.0 / (12.0 * d->dt); s.tau = 3.0 * d->dt; s.t0 = 2.0 * d->dt; s.amp = 1e3;
    return s;
}

static int all_finite(const double* v, int n) {
    for (int m = 0; m < n; ++m)
        if (!isfinite(v[m]) || !(v[m] > 0.0)) return 0;
    return 1;
}

/* Every scheme x form x dtype: plan, a run with an energy trace, graph
 * replays, a step, the step counter, the refined flag. */
static void scheme_sweep(void) {
    const int nx = 13, ny = 11, nz = 9;
    float* eps = random_map(nx, ny, nz, 1.0f, 6.0f);
    for (int s = FDTD_ADI; s <= FDTD_DOUGLAS_GUNN; ++s)
        for (int f = FDTD_FUNDAMENTAL; f <= FDTD_CONVENTIONAL; ++f)
            for (int t = FDTD_F32; t <= FDTD_F32_PLAIN; ++t) {
                fdtd_desc d = desc(nx, ny, nz, 4.0, s, f, t);
                d.eps_r = eps;   /* host pointer */
                const int unsupported = (f == FDTD_CONVENTIONAL && (s == FDTD_DYAKONOV || s == FDTD_DOUGLAS_GUNN)) ||
                                        (f == FDTD_CONVENTIONAL && t == FDTD_F32_REFINE);
                fdtd_plan_t p = NULL;
                EXPECT(fdtd_plan(&d, NULL, &p), unsupported ? FDTD_EUNSUPPORTED : FDTD_OK);
                if (unsupported || !p) continue;
                fset u;
                fset_alloc(&u, nx, ny, nz, elem_size(t));
                const fdtd_source src = source_for(&d);
                double energy[4];
                int refined = -1;
                EXPECT(fdtd_get_refined(p, &refined), FDTD_OK);
                TRUE(refined == 0 || refined == 1);
                EXPECT(fdtd_run(p, u.E, u.H, 3, &src, energy, 1), FDTD_OK);
                TRUE(all_finite(energy, 4));
                EXPECT(fdtd_set_graph(p, 2), FDTD_OK);
                EXPECT(fdtd_run(p, u.E, u.H, 5, &src, NULL, 1), FDTD_OK);
                EXPECT(fdtd_step(p, u.E, u.H, NULL), FDTD_OK);
                EXPECT(fdtd_set_step(p, 0), FDTD_OK);
                EXPECT(fdtd_set_graph(p, 0), FDTD_OK);
                EXPECT(fdtd_run(p, u.E, u.H, 2, &src, NULL, 1), FDTD_OK);
                SETUP(hipDeviceSynchronize());
                TRUE(fset_finite(&u));
                EXPECT(fdtd_destroy(p), FDTD_OK);
                fset_free(&u);
            }
    free(eps);
}

/* A destroyed handle is rejected, not read (the sanitizer would report a
 * read of the freed plan). */
static void destroyed_handle(void) {
    fdtd_desc d = desc(9, 8, 7, 3.0, FDTD_ADI, FDTD_FUNDAMENTAL, FDTD_F32);
    fdtd_plan_t p = NULL;
    EXPECT(fdtd_plan(&d, NULL, &p), FDTD_OK);
    if (!p) return;
    fset u;
    fset_alloc(&u, d.nx, d.ny, d.nz, 4);
    EXPECT(fdtd_run(p, u.E, u.H, 1, NULL, NULL, 1), FDTD_OK);
    EXPECT(fdtd_destroy(p), FDTD_OK);
    EXPECT(fdtd_run(p, u.E, u.H, 1, NULL, NULL, 1), FDTD_EINVAL);
    EXPECT(fdtd_set_step(p, 0), FDTD_EINVAL);
    EXPECT(fdtd_set_order(p, 4), FDTD_EINVAL);
    EXPECT(fdtd_destroy(p), FDTD_EINVAL);
    fdtd_plan_t q = NULL;
    fdtd_desc e[2] = {desc(9, 8, 7, 3.0, FDTD_ADI, FDTD_FUNDAMENTAL, FDTD_F32),
                      desc(7, 9, 8, 3.0, FDTD_ADI, FDTD_FUNDAMENTAL, FDTD_F32)};
    EXPECT(fdtd_plan_batch(e, 2, NULL, &q), FDTD_OK);
    if (q) {
        EXPECT(fdtd_destroy(q), FDTD_OK);
        EXPECT(fdtd_run_batch(q, u.E, u.H, 1), FDTD_EINVAL);
        EXPECT(fdtd_destroy(q), FDTD_EINVAL);
    }
    SETUP(hipDeviceSynchronize());
    fset_free(&u);
}

/* Argument errors on a valid plan; the plan stays usable. */
static void run_errors(void) {
    fdtd_desc d = desc(10, 9, 8, 3.0, FDTD_ADI, FDTD_FUNDAMENTAL, FDTD_F32);
    fdtd_plan_t p = NULL;
    EXPECT(fdtd_plan(&d, NULL, &p), FDTD_OK);
    if (!p) return;
    fset u;
    fset_alloc(&u, d.nx, d.ny, d.nz, 4);
    double energy[3];
    fdtd_source src = source_for(&d);
    void* Ebad[3] = {u.E[0], NULL, u.E[2]};
    EXPECT(fdtd_run(p, u.E, u.H, -1, NULL, NULL, 1), FDTD_EINVAL);
    EXPECT(fdtd_run(p, u.E, u.H, 2, NULL, energy, 0), FDTD_EINVAL);
    EXPECT(fdtd_run(p, Ebad, u.H, 2, NULL, NULL, 1), FDTD_EINVAL);
    EXPECT(fdtd_run(p, NULL, u.H, 2, NULL, NULL, 1), FDTD_EINVAL);
    src.i = 0;
    EXPECT(fdtd_run(p, u.E, u.H, 2, &src, NULL, 1), FDTD_EINVAL);
    src = source_for(&d);
    src.k = d.nz;
    EXPECT(fdtd_run(p, u.E, u.H, 2, &src, NULL, 1), FDTD_EINVAL);
    src = source_for(&d);
    src.tau = 0.0;
    EXPECT(fdtd_run(p, u.E, u.H, 2, &src, NULL, 1), FDTD_EINVAL);
    src = source_for(&d);
    src.amp = INFINITY;
    EXPECT(fdtd_run(p, u.E, u.H, 2, &src, NULL, 1), FDTD_EINVAL);
    EXPECT(fdtd_set_graph(p, 65), FDTD_EINVAL);
    EXPECT(fdtd_set_graph(p, -1), FDTD_EINVAL);
    EXPECT(fdtd_set_step(p, -1), FDTD_EINVAL);
    EXPECT(fdtd_set_order(p, 3), FDTD_EINVAL);
    EXPECT(fdtd_set_stencil(p, -0.05), FDTD_EUNSUPPORTED);   /* second-order plan */
    EXPECT(fdtd_get_refined(p, NULL), FDTD_EINVAL);
    EXPECT(fdtd_set_cg(p, 1e-10, 10), FDTD_EUNSUPPORTED);
    EXPECT(fdtd_last_cg(p, NULL, NULL), FDTD_EUNSUPPORTED);
    EXPECT(fdtd_run_batch(p, u.E, u.H, 1), FDTD_EINVAL);
    src = source_for(&d);
    EXPECT(fdtd_run(p, u.E, u.H, 0, &src, energy, 1), FDTD_OK);
    TRUE(all_finite(energy, 1));
    EXPECT(fdtd_run(p, u.E, u.H, 2, &src, energy, 1), FDTD_OK);
    TRUE(all_finite(energy, 3));
    EXPECT(fdtd_destroy(p), FDTD_OK);
    fset_free(&u);
}

/* Fundamental and conventional ADI give the same fields; fdtd_diff_norm and
 * fdtd_diff_norm_noalloc give the same sums. */
static void forms_and_distances(void) {
    const int nx = 16, ny = 12, nz = 14;
    fdtd_plan_t p[2] = {NULL, NULL};
    fset u[2];
    float* eps = random_map(nx, ny, nz, 1.0f, 9.0f);
    float* eps_d = NULL;
    SETUP(hipMalloc((void**)&eps_d, sizeof(float) * nx * ny * nz));
    SETUP(hipMemcpy(eps_d, eps, sizeof(float) * nx * ny * nz, hipMemcpyHostToDevice));
    fset_alloc(&u[0], nx, ny, nz, 8);
    fset_alloc(&u[1], nx, ny, nz, 8);
    fset_copy(&u[1], &u[0]);
    for (int f = 0; f < 2; ++f) {
        fdtd_desc d = desc(nx, ny, nz, 6.0, FDTD_ADI, f, FDTD_F64);
        d.eps_r = eps_d;   /* device pointer */
        EXPECT(fdtd_plan(&d, NULL, &p[f]), FDTD_OK);
    }
    if (p[0] && p[1]) {
        const fdtd_desc d = desc(nx, ny, nz, 6.0, FDTD_ADI, 0, FDTD_F64);
        const fdtd_source src = source_for(&d);
        double a[2] = {0, 0}, b[2] = {1, 1};
        EXPECT(fdtd_run(p[0], u[0].E, u[0].H, 6, &src, NULL, 1), FDTD_OK);
        EXPECT(fdtd_run(p[1], u[1].E, u[1].H, 6, &src, NULL, 1), FDTD_OK);
        EXPECT(fdtd_diff_norm(p[0], u[0].E, u[0].H, u[1].E, u[1].H, a), FDTD_OK);
        EXPECT(fdtd_diff_norm_noalloc(p[0], u[0].E, u[0].H, u[1].E, u[1].H, b), FDTD_OK);
        TRUE(a[0] == b[0] && a[1] == b[1]);
        TRUE(a[1] > 0.0 && sqrt(a[0] / a[1]) < 1e-12);
        EXPECT(fdtd_diff_norm(p[0], u[0].E, u[0].H, u[1].E, u[1].H, NULL), FDTD_EINVAL);
    }
    for (int f = 0; f < 2; ++f) {
        if (p[f]) EXPECT(fdtd_destroy(p[f]), FDTD_OK);
        fset_free(&u[f]);
    }
    (void)hipFree(eps_d);
    free(eps);
}

static void crank_nicolson(void) {
    for (int f = 0; f < 2; ++f) {
        fdtd_desc d = desc(9, 8, 10, 4.0, FDTD_CRANK_NICOLSON, f, FDTD_F64);
        fdtd_plan_t p = NULL;
        EXPECT(fdtd_plan(&d, NULL, &p), FDTD_OK);
        if (!p) continue;
        fset u;
        fset_alloc(&u, d.nx, d.ny, d.nz, 8);
        const fdtd_source src = source_for(&d);
        double energy[3], res = -1.0;
        long long it = -1;
        fdtd_kernel_config kc;
        EXPECT(fdtd_set_cg(p, 0.0, 10), FDTD_EINVAL);
        EXPECT(fdtd_set_cg(p, 1e-10, 0), FDTD_EINVAL);
        EXPECT(fdtd_set_cg(p, 1e-11, 300), FDTD_OK);
        EXPECT(fdtd_run(p, u.E, u.H, 2, &src, energy, 1), FDTD_OK);
        TRUE(all_finite(energy, 3));
        EXPECT(fdtd_last_cg(p, &it, &res), FDTD_OK);
        TRUE(it > 0 && res >= 0.0 && res < 1e-10);
        EXPECT(fdtd_set_graph(p, 2), FDTD_EUNSUPPORTED);
        EXPECT(fdtd_autotune(p, 1, NULL), FDTD_EUNSUPPORTED);
        EXPECT(fdtd_get_kernel_config(p, 0, &kc), FDTD_EUNSUPPORTED);
        EXPECT(fdtd_set_order(p, 4), FDTD_EUNSUPPORTED);
        EXPECT(fdtd_destroy(p), FDTD_OK);
        fset_free(&u);
    }
}

static void permeability(void) {
    const int nx = 12, ny = 10, nz = 11;
    float* mu = random_map(nx, ny, nz, 1.0f, 3.0f);
    float* eps = random_map(nx, ny, nz, 1.0f, 4.0f);
    float* ones = (float*)malloc(sizeof(float) * nx * ny * nz);
    float* mu_d = NULL;
    if (!ones) exit(2);
    for (int c = 0; c < nx * ny * nz; ++c) ones[c] = 1.0f;
    SETUP(hipMalloc((void**)&mu_d, sizeof(float) * nx * ny * nz));
    SETUP(hipMemcpy(mu_d, mu, sizeof(float) * nx * ny * nz, hipMemcpyHostToDevice));
    const int cases[][3] = {{FDTD_ADI, FDTD_FUNDAMENTAL, FDTD_F64}, {FDTD_ADI, FDTD_CONVENTIONAL, FDTD_F32_PLAIN},
                            {FDTD_LOD1, FDTD_FUNDAMENTAL, FDTD_F32}, {FDTD_SS2, FDTD_CONVENTIONAL, FDTD_F32_F64SOLVE},
                            {FDTD_CRANK_NICOLSON, FDTD_FUNDAMENTAL, FDTD_F64}};
    for (size_t n = 0; n < sizeof cases / sizeof cases[0]; ++n) {
        fdtd_desc d = desc(nx, ny, nz, 5.0, cases[n][0], cases[n][1], cases[n][2]);
        d.eps_r = eps;
        d.mu_r = mu_d;
        fdtd_plan_t p = NULL;
        EXPECT(fdtd_plan(&d, NULL, &p), FDTD_OK);
        if (!p) continue;
        fset u;
        fset_alloc(&u, nx, ny, nz, elem_size(cases[n][2]));
        double energy[4];
        const fdtd_source src = source_for(&d);
        EXPECT(fdtd_run(p, u.E, u.H, 3, &src, energy, 1), FDTD_OK);
        TRUE(all_finite(energy, 4));
        if (cases[n][0] != FDTD_CRANK_NICOLSON) EXPECT(fdtd_set_order(p, 4), FDTD_EUNSUPPORTED);
        EXPECT(fdtd_destroy(p), FDTD_OK);
        fset_free(&u);
    }
    fdtd_desc d = desc(nx, ny, nz, 5.0, FDTD_ADI, FDTD_FUNDAMENTAL, FDTD_F32_REFINE);
    fdtd_plan_t p = NULL;
    d.mu_r = mu_d;
    EXPECT(fdtd_plan(&d, NULL, &p), FDTD_EUNSUPPORTED);
    d.mu_r = ones;   /* all ones: unit permeability, refined solves allowed */
    EXPECT(fdtd_plan(&d, NULL, &p), FDTD_OK);
    if (p) EXPECT(fdtd_destroy(p), FDTD_OK);
    mu[5] = -1.0f;
    d.mu_r = mu;
    EXPECT(fdtd_plan(&d, NULL, &p), FDTD_EINVAL);
    (void)hipFree(mu_d);
    free(mu);
    free(eps);
    free(ones);
}

static void fourth_order(void) {
    const int nx = 14, ny = 12, nz = 13;
    const int types[4] = {FDTD_F32, FDTD_F64, FDTD_F32_F64SOLVE, FDTD_F32_PLAIN};
    for (int it = 0; it < 4; ++it) {
        const int t = types[it];
        fdtd_desc d = desc(nx, ny, nz, 8.0, FDTD_ADI, FDTD_FUNDAMENTAL, t);
        fdtd_plan_t p = NULL;
        double b = 0.0, energy[4];
        int refined = -1;
        EXPECT(fdtd_plan(&d, NULL, &p), FDTD_OK);
        if (!p) continue;
        fset u;
        fset_alloc(&u, nx, ny, nz, elem_size(t));
        const fdtd_source src = source_for(&d);
        EXPECT(fdtd_set_stencil(p, -0.05), FDTD_EUNSUPPORTED);
        EXPECT(fdtd_set_order(p, 4), FDTD_OK);
        EXPECT(fdtd_get_refined(p, &refined), FDTD_OK);
        TRUE(refined == 0);   /* order 4: no refined solves (FDTD_F32: FP64 solves) */
        EXPECT(fdtd_run(p, u.E, u.H, 3, &src, energy, 1), FDTD_OK);
        TRUE(all_finite(energy, 4));
        EXPECT(fdtd_stencil_optimized(PI / 2, &b), FDTD_OK);
        EXPECT(fdtd_set_stencil(p, b), FDTD_OK);
        EXPECT(fdtd_set_stencil(p, 0.3), FDTD_EINVAL);
        EXPECT(fdtd_set_stencil(p, NAN), FDTD_EINVAL);
        EXPECT(fdtd_set_graph(p, 2), FDTD_OK);
        EXPECT(fdtd_run(p, u.E, u.H, 5, &src, NULL, 1), FDTD_OK);
        EXPECT(fdtd_run(p, u.E, u.H, 3, &src, energy, 1), FDTD_OK);
        TRUE(all_finite(energy, 4));
        EXPECT(fdtd_set_order(p, 2), FDTD_OK);
        EXPECT(fdtd_get_refined(p, &refined), FDTD_OK);
        TRUE(refined == (t == FDTD_F32));   /* FDTD_F32: refined again */
        EXPECT(fdtd_run(p, u.E, u.H, 2, &src, NULL, 1), FDTD_OK);
        SETUP(hipDeviceSynchronize());
        TRUE(fset_finite(&u));
        EXPECT(fdtd_destroy(p), FDTD_OK);
        fset_free(&u);
    }
    fdtd_desc d = desc(nx, ny, nz, 8.0, FDTD_LOD1, FDTD_CONVENTIONAL, FDTD_F64);
    fdtd_plan_t p = NULL;
    EXPECT(fdtd_plan(&d, NULL, &p), FDTD_OK);
    if (p) {
        EXPECT(fdtd_set_order(p, 4), FDTD_EUNSUPPORTED);
        EXPECT(fdtd_destroy(p), FDTD_OK);
    }
}

static void timing_configs_autotune(void) {
    fdtd_desc d = desc(40, 36, 34, 5.0, FDTD_ADI, FDTD_FUNDAMENTAL, FDTD_F32);
    fdtd_plan_t p = NULL, q = NULL;
    EXPECT(fdtd_plan(&d, NULL, &p), FDTD_OK);
    if (!p) return;
    fset u;
    fset_alloc(&u, d.nx, d.ny, d.nz, 4);
    double main_ms = -1.0, avg[2] = {-1, -1}, best[3] = {-1, -1, -1};
    int launches[2] = {-1, -1};
    EXPECT(fdtd_set_timing(p, -1), FDTD_EINVAL);
    EXPECT(fdtd_set_timing(p, 1), FDTD_OK);
    EXPECT(fdtd_run(p, u.E, u.H, 2, NULL, NULL, 1), FDTD_OK);
    EXPECT(fdtd_last_timing(p, &main_ms, avg, launches), FDTD_OK);
    TRUE(main_ms > 0.0 && avg[0] > 0.0 && avg[1] > 0.0 && launches[0] == 8 && launches[1] == 4);
    EXPECT(fdtd_set_timing(p, 0), FDTD_OK);
    EXPECT(fdtd_last_timing(p, NULL, NULL, NULL), FDTD_OK);

    for (int axis = 0; axis < 3; ++axis) {
        fdtd_kernel_config c, bad;
        EXPECT(fdtd_get_kernel_config(p, axis, &c), FDTD_OK);
        EXPECT(fdtd_set_kernel_config(p, axis, &c), FDTD_OK);
        bad = c;
        bad.chunk = 7;
        EXPECT(fdtd_set_kernel_config(p, axis, &bad), FDTD_EINVAL);
        EXPECT(fdtd_set_kernel_config(p, axis, NULL), FDTD_EINVAL);
    }
    {
        fdtd_kernel_config c;
        EXPECT(fdtd_get_kernel_config(p, 3, &c), FDTD_EINVAL);
        EXPECT(fdtd_get_kernel_config(p, 0, NULL), FDTD_EINVAL);
    }

    /* autotuner, then a second plan of the same kind from the cache */
    const char* tmp = getenv("TMPDIR");
    char path[512];
    snprintf(path, sizeof path, "%s/fdtd_abi_exercise_tune_%ld.jsonl", tmp && *tmp ? tmp : "/tmp", (long)getpid());
    unlink(path);
    setenv("FDTD_TUNE_CACHE", path, 1);
    EXPECT(fdtd_autotune(p, 0, best), FDTD_EINVAL);
    EXPECT(fdtd_autotune(p, 2, best), FDTD_OK);
    TRUE(best[0] > 0.0 && best[1] > 0.0 && best[2] > 0.0);
    EXPECT(fdtd_plan(&d, NULL, &q), FDTD_OK);
    if (q) {
        double cached[3] = {-1, -1, -1};
        fdtd_kernel_config a, b;
        EXPECT(fdtd_autotune(q, 2, cached), FDTD_OK);
        TRUE(cached[0] == 0.0 && cached[1] == 0.0 && cached[2] == 0.0);
        for (int axis = 0; axis < 3; ++axis) {
            EXPECT(fdtd_get_kernel_config(p, axis, &a), FDTD_OK);
            EXPECT(fdtd_get_kernel_config(q, axis, &b), FDTD_OK);
            TRUE(memcmp(&a, &b, sizeof a) == 0);
        }
        EXPECT(fdtd_run(q, u.E, u.H, 2, NULL, NULL, 1), FDTD_OK);
        EXPECT(fdtd_destroy(q), FDTD_OK);
    }
    unsetenv("FDTD_TUNE_CACHE");
    unlink(path);
    EXPECT(fdtd_run(p, u.E, u.H, 2, NULL, NULL, 1), FDTD_OK);
    SETUP(hipDeviceSynchronize());
    TRUE(fset_finite(&u));
    EXPECT(fdtd_destroy(p), FDTD_OK);
    fset_free(&u);
}

static void adjoint(void) {
    const int nx = 8, ny = 7, nz = 9;
    float* eps = random_map(nx, ny, nz, 1.0f, 5.0f);
    const int box[6] = {1, 7, 0, 7, 2, 9};
    const size_t nb = (size_t)6 * 7 * 7;
    double* grad = NULL;
    SETUP(hipMalloc((void**)&grad, sizeof(double) * nb));
    for (int s = FDTD_ADI; s <= FDTD_DOUGLAS_GUNN; ++s) {
        fdtd_desc d = desc(nx, ny, nz, 3.0, s, FDTD_FUNDAMENTAL, FDTD_F64);
        d.eps_r = eps;
        fdtd_plan_t p = NULL;
        EXPECT(fdtd_plan(&d, NULL, &p), FDTD_OK);
        if (!p) continue;
        fset u;
        fset_alloc(&u, nx, ny, nz, 8);
        const fdtd_source src = source_for(&d);
        const int supported = s == FDTD_ADI || s == FDTD_DYAKONOV || s == FDTD_DOUGLAS_GUNN;
        double J = -1.0, J2 = -2.0;
        EXPECT(fdtd_grad_eps(p, u.E, u.H, 6, &src, 4, 3, 4, box, 2, &J, grad),
               supported ? FDTD_OK : FDTD_EUNSUPPORTED);
        if (supported) {
            double* g = (double*)malloc(sizeof(double) * nb);
            if (!g) exit(2);
            SETUP(hipMemcpy(g, grad, sizeof(double) * nb, hipMemcpyDeviceToHost));
            int ok = isfinite(J) && J > 0.0;
            for (size_t c = 0; c < nb; ++c) ok = ok && isfinite(g[c]);
            TRUE(ok);
            free(g);
            EXPECT(fdtd_grad_eps(p, u.E, u.H, 6, &src, 4, 3, 4, NULL, 0, &J2, NULL), FDTD_OK);
            TRUE(fabs(J2 - J) <= 1e-12 * J);
            EXPECT(fdtd_grad_eps(p, u.E, u.H, 6, &src, 0, 3, 4, box, 2, &J2, grad), FDTD_EINVAL);
            EXPECT(fdtd_grad_eps(p, u.E, u.H, 6, &src, 4, 3, 4, box, 0, &J2, grad), FDTD_EINVAL);
            EXPECT(fdtd_grad_eps(p, u.E, u.H, 6, &src, 4, 3, 4, NULL, 2, &J2, grad), FDTD_EINVAL);
            EXPECT(fdtd_grad_eps(p, u.E, u.H, 6, &src, 4, 3, 4, box, 2, NULL, grad), FDTD_EINVAL);
            const int bad_box[6] = {0, 9, 0, 7, 0, 9};
            EXPECT(fdtd_grad_eps(p, u.E, u.H, 6, &src, 4, 3, 4, bad_box, 2, &J2, grad), FDTD_EINVAL);
        }
        EXPECT(fdtd_destroy(p), FDTD_OK);
        fset_free(&u);
    }
    (void)hipFree(grad);
    free(eps);
}

static void batches(void) {
    const int dims[3][3] = {{10, 9, 8}, {12, 11, 7}, {9, 13, 10}};
    fdtd_desc d[3];
    float* eps[3];
    fset u[3];
    void *E[9], *H[9];
    for (int g = 0; g < 3; ++g) {
        d[g] = desc(dims[g][0], dims[g][1], dims[g][2], 4.0, FDTD_ADI, FDTD_FUNDAMENTAL, FDTD_F32);
        eps[g] = random_map(dims[g][0], dims[g][1], dims[g][2], 1.0f, 4.0f);
        d[g].eps_r = eps[g];
        fset_alloc(&u[g], dims[g][0], dims[g][1], dims[g][2], 4);
        for (int c = 0; c < 3; ++c) {
            E[3 * g + c] = u[g].E[c];
            H[3 * g + c] = u[g].H[c];
        }
    }
    fdtd_plan_t p = NULL;
    EXPECT(fdtd_plan_batch(d, 3, NULL, &p), FDTD_OK);
    if (p) {
        double main_ms = -1.0, dist[2];
        fdtd_kernel_config c;
        double J = 0.0;
        EXPECT(fdtd_autotune(p, 2, NULL), FDTD_OK);
        EXPECT(fdtd_get_kernel_config(p, 1, &c), FDTD_OK);
        EXPECT(fdtd_set_kernel_config(p, 1, &c), FDTD_OK);
        EXPECT(fdtd_set_timing(p, 1), FDTD_OK);
        EXPECT(fdtd_run_batch(p, E, H, 11), FDTD_OK);
        EXPECT(fdtd_last_timing(p, &main_ms, NULL, NULL), FDTD_OK);
        TRUE(main_ms > 0.0);
        EXPECT(fdtd_run_batch(p, E, H, -1), FDTD_EINVAL);
        EXPECT(fdtd_run_batch(p, NULL, H, 1), FDTD_EINVAL);
        EXPECT(fdtd_run(p, E, H, 1, NULL, NULL, 1), FDTD_EINVAL);
        EXPECT(fdtd_set_graph(p, 2), FDTD_EINVAL);
        EXPECT(fdtd_set_order(p, 4), FDTD_EINVAL);
        EXPECT(fdtd_diff_norm(p, E, H, E, H, dist), FDTD_EINVAL);
        EXPECT(fdtd_diff_norm_noalloc(p, E, H, E, H, dist), FDTD_EINVAL);
        EXPECT(fdtd_grad_eps(p, E, H, 1, NULL, 2, 2, 2, NULL, 1, &J, NULL), FDTD_EINVAL);
        SETUP(hipDeviceSynchronize());
        for (int g = 0; g < 3; ++g) TRUE(fset_finite(&u[g]));
        EXPECT(fdtd_destroy(p), FDTD_OK);
    }
    {
        fdtd_desc e[2] = {d[0], d[1]};
        e[1].scheme = FDTD_LOD1;
        EXPECT(fdtd_plan_batch(e, 2, NULL, &p), FDTD_EINVAL);
        e[0].form = e[1].form = FDTD_CONVENTIONAL;
        e[1].scheme = FDTD_ADI;
        EXPECT(fdtd_plan_batch(e, 2, NULL, &p), FDTD_EUNSUPPORTED);
    }
    for (int g = 0; g < 3; ++g) {
        fset_free(&u[g]);
        free(eps[g]);
    }
}

int main(int argc, char** argv) {
    const int host_only = argc > 1 && strcmp(argv[1], "host") == 0;
    host_checks();
    if (!host_only) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
            fprintf(stderr, "no GPU\n");
            return 2;
        }
        scheme_sweep();
        run_errors();
        destroyed_handle();
        forms_and_distances();
        crank_nicolson();
        permeability();
        fourth_order();
        timing_configs_autotune();
        adjoint();
        batches();
        SETUP(hipDeviceSynchronize());
    }
    printf("{\"checks\": %d, \"failures\": %d}\n", nchk, nfail);
    fflush(stdout);
    fflush(stderr);
    /* The leak check runs here, and the process ends without the HIP runtime's
     * teardown at exit: that teardown frees runtime memory after the
     * sanitizer's own hooks into the HSA runtime are gone, which the sanitizer
     * reports as an internal error of its own. */
    __lsan_do_leak_check();
    _exit(nfail ? 1 : 0);
}
