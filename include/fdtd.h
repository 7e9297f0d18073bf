/*
 * fdtd.h -- C ABI of the MI355X implicit FDTD library (libfdtd.so).
 *
 * Time-steps Maxwell's equations for a lossless isotropic medium in a PEC
 * box on a Yee grid with the unconditionally stable splitting schemes of
 * E. L. Tan, "Fundamental Schemes for Efficient Unconditionally Stable
 * Implicit FDTD Methods" (arXiv 2011.14043):
 *   ADI   -- Sec. II-A, eq. (clsADI) / fundamental (fasterADI)
 *   LOD1  -- Sec. II-B, eq. (orgLOD)  / fundamental (fastLOD)   (== SS1)
 *   SS2   -- Sec. II-C, eq. (orgSS2)  / fundamental (fastSS2)
 *   LOD2  -- Sec. II-D, eq. (orgLOD2) / fundamental (fastLOD2), with the
 *            input/output processing (orgLOD2i/o), (fastLOD2i/o)
 *   D'Yakonov, Douglas-Gunn -- Sec. II-E, eqs. (orgDY) / (fastDY) and the
 *            delta formulation / (fastDGo), fundamental form only
 * using the operators A, B of eq. (AMat) with b = dt/(2 eps), d = dt/(2 mu)
 * (eq. (bd)) and second-order central differences on Yee cells (Sec. III).
 * "Fundamental" runs the matrix-operator-free right-hand sides of Sec. III;
 * "conventional" runs the original splitting formulae with the same line
 * solver, for comparison (Table I).
 *
 * Field layout (caller's arrays).  Each of Ex, Ey, Ez, Hx, Hy, Hz is a dense
 * row-major device array of shape (nz+1, ny+1, nx+1), index [k][j][i], x
 * fastest, element type double for FDTD_F64, else float.  The entry
 * [k][j][i] of a component is its Yee sample nearest to node (i, j, k):
 * Ex (i+1/2, j, k), Ey (i, j+1/2, k), Ez (i, j, k+1/2), Hx (i, j+1/2, k+1/2),
 * Hy (i+1/2, j, k+1/2), Hz (i+1/2, j+1/2, k), in units of dx, dy, dz.
 * Entries outside the box are ignored on input and left untouched on output;
 * E tangential to a wall is treated as 0 on input and written as 0 on output;
 * H normal to a wall is static and passed through.
 *
 * Every call returns an fdtd_status (0 = OK); no C++ exception crosses the
 * ABI.  Arguments are validated before any device work; on an error other
 * than FDTD_ENONFINITE the plan and the caller's buffers are unchanged.
 * A plan is not re-entrant; distinct plans are independent.
 */
#ifndef FDTD_H
#define FDTD_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtd_plan_s* fdtd_plan_t;

typedef enum {
    FDTD_OK = 0,
    FDTD_EINVAL = -1,        /* bad argument (NULL, sizes, time step, cell index ...) */
    FDTD_ENOMEM = -2,        /* device allocation failed                             */
    FDTD_EDEVICE = -3,       /* HIP runtime error                                    */
    FDTD_EUNSUPPORTED = -4,  /* valid request the library does not implement         */
    FDTD_ENONFINITE = -5,    /* NaN/Inf found in the energy after stepping           */
    FDTD_ENOTCONVERGED = -6  /* an iterative solve stopped at its iteration limit    */
                             /* above its tolerance (Crank-Nicolson plans)           */
} fdtd_status;

/* FDTD_DYAKONOV and FDTD_DOUGLAS_GUNN (Sec. II-E) take the fundamental form
 * only (else FDTD_EUNSUPPORTED).  The paper gives these splittings without a
 * nonhomogeneous term; a source follows the ADI convention (see
 * fdtd_source).  Their fundamental
 * forms are the iteration of (fasterADI) with other variables: (fastDY) is
 * it with u in place of u~ = 2u and the input v^{-1/2} = (1/2 I - dt/4 B) u^0,
 * and (fastDGo) reads the delta formulation's increments off u~.  Both give
 * the Peaceman-Rachford fields u^n, and the ADI plan already iterates in the
 * variables of (fastDY) (state v^n = (1/2 I + dt/4 B) u^n, field
 * u^{n+1} = v^{n+1/2} + v^{n+1}), so these plans run the fundamental ADI
 * passes, input and output processing unchanged: same fields, energy trace,
 * kernels and cost.  Batches and fdtd_grad_eps accept them too. */
/* FDTD_CRANK_NICOLSON (Sec. II-E, closing part) is the unfactorized scheme in
 * its fundamental form, [1/2 I - dt/4 (A + B)] u^{n+1/2} = u^n,
 * u^{n+1} = u^{n+1/2} - u^n: one global sparse system per step instead of line
 * solves.  With theta = dt/2 the H rows are eliminated, leaving for E the
 * symmetric positive definite system eps v + theta^2 C_H(mu^-1 C_E(v)) =
 * 2 eps u_E + 2 theta C_H(u_H) (C_E, C_H the discrete curls), which each step
 * solves by conjugate gradients with the diagonal as preconditioner, started
 * from v = 2 u_E, to the relative residual of fdtd_set_cg.  The conventional
 * form is the classical [I - dt/2 (A + B)] u^{n+1} = [I + dt/2 (A + B)] u^n:
 * its right side f is formed explicitly, and the same system
 * S u_E^{n+1} = eps f_E + theta C_H(f_H) is solved from the guess u_E^n.
 * FDTD_F64 only (else FDTD_EUNSUPPORTED); no batches, adjoint or kernel
 * configuration (no line passes).  A source adds one term per step (see
 * fdtd_source).  fdtd_run returns
 * FDTD_ENOTCONVERGED, with every step done, if some step ended at the
 * iteration limit above the tolerance.  A Crank-Nicolson run synchronizes
 * the plan's stream: the host reads the residual every fourth iteration.
 * The plan holds 15 more FP64 arrays of the state's size (CG work vectors). */
typedef enum {
    FDTD_ADI = 0, FDTD_LOD1 = 1 /* == SS1 */, FDTD_SS2 = 2, FDTD_LOD2 = 3,
    FDTD_DYAKONOV = 4, FDTD_DOUGLAS_GUNN = 5, FDTD_CRANK_NICOLSON = 6
} fdtd_scheme;
typedef enum { FDTD_FUNDAMENTAL = 0, FDTD_CONVENTIONAL = 1 } fdtd_form;
/* Precision.  FDTD_F64 uses FP64 for fields and solves.  FDTD_F32_F64SOLVE
 * keeps fields in FP32 (FP32 HBM traffic) but forms every right-hand side,
 * tridiagonal solve and update in FP64 registers, rounding once per stored
 * value.  FDTD_F32_PLAIN keeps fields in FP32 and solves in FP32.
 * FDTD_F32_REFINE is FDTD_F32_PLAIN with one step of iterative refinement of
 * every tridiagonal solve (the residual r - T V formed with the unrounded
 * sigma, and a second solve with the same factors, all in FP32), which
 * removes the fixed rounding bias of the FP32 factors and of 2 + sigma;
 * fundamental forms only (else FDTD_EUNSUPPORTED), nx, ny, nz <= 512.
 * FDTD_F32 (FP32 fields and arithmetic) refines wherever refined passes are
 * built (fundamental forms, nx, ny, nz <= 512, no permeability map) and runs
 * as FDTD_F32_PLAIN elsewhere: the line systems are
 * -V[j-1] + (2 + sigma) V[j] - V[j+1] = r with sigma = eps mu dw^2 / theta^2
 * (Sec. III-A multiplied by 2 sigma), and plain FP32 solves round both 2 +
 * sigma (FP32 spaces numbers near 2 by 2.4e-7: a relative perturbation of
 * the medium of up to 1.2e-7 / sigma) and the medium-only factors the same
 * way at every step, so their error grows linearly with the step count
 * (after 1000 steps: 3e-4 at sigma = 0.12, 4e-5 to 6e-5 at sigma >= 0.48 and
 * at sigma = 12); refined solves stay near 1e-5, for 1 % to 3 % of the step
 * time.  fdtd_get_refined tells which. */
typedef enum { FDTD_F32 = 0, FDTD_F64 = 1, FDTD_F32_F64SOLVE = 2, FDTD_F32_REFINE = 3,
               FDTD_F32_PLAIN = 4 } fdtd_dtype;

typedef struct {
    int nx, ny, nz;            /* cells per axis, each >= 2                               */
    double dt;                 /* time step [s], > 0 (any size: the schemes are           */
                               /* unconditionally stable)                                 */
    double dx, dy, dz;         /* cell sizes [m], > 0                                     */
    int scheme;                /* fdtd_scheme                                             */
    int form;                  /* fdtd_form                                               */
    int dtype;                 /* fdtd_dtype; nx, ny, nz <= 1024 (FDTD_F32,               */
                               /* FDTD_F32_PLAIN), <= 512 else                            */
    const float* eps_r;        /* relative permittivity per cell, (nz, ny, nx) row-major, */
                               /* x fastest, > 0; host or device pointer, copied by       */
                               /* fdtd_plan (may be freed afterwards).  NULL means 1.     */
                               /* The E sample stored at [k][j][i] uses cell [k][j][i].   */
    const float* mu_r;         /* relative permeability per cell (eq. (bd): d = dt/(2 mu)),*/
                               /* layout, ownership and checks as eps_r; NULL means 1.    */
                               /* The H sample stored at [k][j][i] uses cell [k][j][i].   */
                               /* A map that is not all ones: line passes with per-row    */
                               /* off-diagonals (each axis <= 512, no FDTD_F32_REFINE,    */
                               /* not in fdtd_plan_batch: FDTD_EUNSUPPORTED); FDTD_F32     */
                               /* then solves plainly.                                    */
    int boundary;              /* 0 = PEC on all faces (the only value)                   */
} fdtd_desc;

/* Ez point source in cell (i, j, k) (1 <= i < nx, 1 <= j < ny, 0 <= k < nz).
 * The paper omits nonhomogeneous terms (Sec. II); the library adds, in every
 * sub-step written as (I - theta X) u' = (I + theta Y) u + g, the vector g
 * with the single entry  theta * amp * p(t_k)  at that Ez sample, where
 * p(t) = exp(-((t - t0)/tau)^2) sin(2 pi f0 (t - t0)) and t_k is the middle
 * of the sub-step's time interval (ADI, LOD1: n+1/4, n+3/4; SS2: n+1/8, n+1/2,
 * n+7/8; LOD2: n+1/2, n+1; Crank-Nicolson, one term per step with
 * theta = dt/2: n+1/2; times dt, n counted from the plan's step counter).
 * The fundamental forms add the same term so that both forms agree; the
 * D'Yakonov and Douglas-Gunn plans take ADI's. */
typedef struct { int i, j, k; double f0, tau, t0, amp; } fdtd_source;

/* Create a plan: validates `d`, copies eps_r, allocates the internal state
 * (6 arrays; 12 for conventional ADI) and scratch on the current device.
 * `hip_stream` (hipStream_t or NULL for the default stream) is used by every
 * later call.  The step counter starts at 0. */
fdtd_status fdtd_plan(const fdtd_desc* d, void* hip_stream, fdtd_plan_t* out);

/* *refined (host) = 1 if the plan's FP32 line solves are refined
 * (FDTD_F32_REFINE, or FDTD_F32 where refined passes are built), else 0. */
fdtd_status fdtd_get_refined(fdtd_plan_t p, int* refined);

/* Accuracy order of the staggered first differences d_w of the updating
 * equations (Sec. III-A; its closing remark leaves the difference operators
 * open: higher order, optimized, compact): 2 (the Yee differences, the
 * default) or 4, the fourth-order staggered difference
 *   d_w f = (f[-3/2] - 27 f[-1/2] + 27 f[+1/2] - f[+3/2]) / (24 dw),
 * used in every implicit line equation, explicit H update and input/output
 * operator.  Near a PEC wall the stencil reaches image samples across it
 * (tangential E odd about the wall, tangential H even), which keeps A and B
 * skew-adjoint in the energy norm, so the schemes remain unconditionally
 * stable and energy-conserving; each line system then couples every E
 * sample to three neighbours on either side (symmetric positive definite,
 * solved by one thread per line).  Order 4: single-grid plans of the
 * fundamental forms (ADI, LOD1, SS2, LOD2, D'Yakonov, Douglas-Gunn) with unit
 * permeability and without FDTD_F32_REFINE (else FDTD_EUNSUPPORTED).  The
 * order-4 passes have no refined solves, and plain FP32 solves of their band-3
 * systems drift linearly with the step count (after 1000 steps at 128^3: up
 * to 1.4e-3 at CFL 10, 1.6e-4 at CFL 5, 1.3e-4 at CFL 1); FDTD_F32 plans
 * therefore solve them in FP64 with FP32 fields, as FDTD_F32_F64SOLVE (1.4e-6
 * after 1000 steps), and FDTD_F32_PLAIN plans in FP32, the faster choice.
 * fdtd_set_order(p, 2) restores the plan's second-order passes (FDTD_F32:
 * refined again where built).  The plan allocates its order-4 work areas once
 * (FDTD_ENOMEM): about five arrays of one field component's size in the solve
 * precision, two in the field precision and a copy of the medium.  Batch plans:
 * FDTD_EINVAL.  Synchronizes the plan's stream; takes effect at the next
 * run. */
fdtd_status fdtd_set_order(fdtd_plan_t p, int order);

/* Parameter-optimized operators (the closing remark of Sec. III-A names them
 * without giving one).  The order-4 plans' difference is the 4-point
 * staggered difference with outer weight b = `outer`:
 *   d_w f = [(1 - 3b)(f[+1/2] - f[-1/2]) + b (f[+3/2] - f[-3/2])] / dw,
 * exact on quadratics for every b, fourth order at b = -1/24 (the default);
 * the wall images and the line solve are those of fdtd_set_order, so the
 * schemes stay unconditionally stable and energy-conserving for every b.  A
 * cavity mode of wavenumber k sees K(k) dw = 2 (1 - 3b) sin(k dw/2) +
 * 2 b sin(3 k dw/2).  Order-4 plans only (else FDTD_EUNSUPPORTED);
 * |outer| <= 0.25 (else FDTD_EINVAL).  Synchronizes the plan's stream; takes
 * effect at the next run. */
fdtd_status fdtd_set_stencil(fdtd_plan_t p, double outer);

/* The outer weight b that minimizes the squared error of the modified
 * wavenumber over a band: the integral over theta = k dw in [0, theta_max] of
 * (K(k) dw - theta)^2, least squares in b (host computation, 64 x 8-point
 * Gauss-Legendre quadrature).  0 < theta_max <= pi (theta_max = pi/2: four
 * samples per wavelength), else FDTD_EINVAL; `outer`: host double.  A narrow
 * band gives the fourth-order -1/24. */
fdtd_status fdtd_stencil_optimized(double theta_max, double* outer);

/* Advance the caller's fields by `nsteps` >= 0 full time steps:
 *   input processing (ADI: u^0 -> (1/2 I + dt/4 B) u^0, the link of
 *   Sec. II-E; LOD2: (fastLOD2i)/(orgLOD2i)), nsteps main iterations, output
 *   processing (ADI: the field v of the last B sub-step; LOD2:
 *   (fastLOD2o)/(orgLOD2o)).  Without an energy trace, the line passes of the
 *   last sub-step (LOD2: of the output processing) store the output straight
 *   into E, H, and a small kernel writes the wall samples no pass writes.
 * E[3] = {Ex, Ey, Ez}, H[3] = {Hx, Hy, Hz}: device pointers, read on entry and
 * overwritten on return (the same arrays may be reused by the next call).
 * `src` may be NULL.  If `energy` is non-NULL (host array of
 * nsteps/energy_every + 1 doubles, energy_every >= 1), energy[m] receives the
 * FP64 energy sum eps |E|^2 + mu |H|^2 over all samples of the main-iteration
 * state at step m*energy_every (ADI: the state (1/2 I + dt/4 B) u, whose
 * energy the scheme conserves); the call then synchronizes the stream and
 * returns FDTD_ENONFINITE if any value is not finite.  Without `energy` the
 * call is asynchronous on the plan's stream.  The step counter advances by
 * nsteps. */
fdtd_status fdtd_run(fdtd_plan_t p, void* const E[3], void* const H[3], int nsteps,
                     const fdtd_source* src, double* energy, int energy_every);

/* fdtd_run with nsteps = 1 and no energy. */
fdtd_status fdtd_step(fdtd_plan_t p, void* const E[3], void* const H[3], const fdtd_source* src);

/* Captured graphs of a single-grid plan (else FDTD_EINVAL): fdtd_run replays
 * a HIP graph of `steps` main-iteration steps (1 <= steps <= 64) for the
 * steps before its last one, and launches the rest directly; 0 (the default)
 * launches every step directly.  The graph is a chain of the passes on one
 * stream, for callers that want the launches recorded; it runs at the speed
 * of direct launches.  Runs with an energy trace or per-launch
 * timing never use graphs.  The graph is captured on the first run that
 * uses it and again when the source cell or a kernel configuration changes;
 * the source terms of a run are computed on the host (as for direct
 * launches), copied to the device once per run, and each replay reads its
 * window of them, so replays and direct launches give the same fields bit for
 * bit.  Crank-Nicolson plans: FDTD_EUNSUPPORTED. */
fdtd_status fdtd_set_graph(fdtd_plan_t p, int steps);

/* Set the plan's step counter (the source time origin). */
fdtd_status fdtd_set_step(fdtd_plan_t p, long long n);

/* Timing of the most recent fdtd_run (synchronizes the plan's stream).
 * main_ms: milliseconds between HIP events recorded on the plan's stream
 * around the main iterations (input processing and the LOD2 output sub-step
 * excluded; the last main-iteration passes store the output).
 * fdtd_set_timing(p, k), k >= 1, before the run: HIP events bracket every
 * line pass of every k-th main-iteration step (steps 0, k, 2k, ...; k = 1:
 * every step) on the plan's stream, and pass_ms_avg[f] / pass_launches[f]
 * give the mean duration [ms] and count of the bracketed launches of family
 * f (0 = y/z-line passes, 1 = x-line passes); k = 0 (the default): no
 * per-launch events, both are 0.  k < 0: FDTD_EINVAL.  Either output pointer
 * may be NULL (arrays of 2).  Each event pair adds a few microseconds between
 * launches. */
fdtd_status fdtd_set_timing(fdtd_plan_t p, int per_launch);
fdtd_status fdtd_last_timing(fdtd_plan_t p, double* main_ms, double* pass_ms_avg, int* pass_launches);

/* Kernel configuration of the line passes along one axis (0 = x, 1 = y, 2 = z):
 *   chunk          slots of a line held by one thread (8, 16 or 32)
 *   tile_x         y/z lines: consecutive x positions per block (8, 16, 32); 0 for x
 *   block_threads  x lines: threads per block (64, 128, 256); for a batch
 *                  plan also 0: the x lines run inside the y/z launch of their
 *                  sub-step, in its blocks, when chunk is 8 and y and z share
 *                  a configuration built for it; otherwise in blocks of 256;
 *                  y/z lines: block-size bound of the variant (256, 512, 1024)
 *   remap          1 = XCD-aware block order, 0 = plain order
 * Every configuration computes the same result up to rounding order.
 * fdtd_set_kernel_config returns FDTD_EINVAL for a variant that is not built
 * or does not fit the axis length. */
typedef struct { int chunk, tile_x, block_threads, remap; } fdtd_kernel_config;
fdtd_status fdtd_get_kernel_config(fdtd_plan_t p, int axis, fdtd_kernel_config* c);
fdtd_status fdtd_set_kernel_config(fdtd_plan_t p, int axis, const fdtd_kernel_config* c);

/* Autotuner: times every valid configuration of the A-operator pass of each
 * axis (`reps` launches each, HIP events on the plan's stream, on the plan's
 * internal state, whose contents it overwrites) and keeps the fastest.  If
 * the environment variable FDTD_TUNE_CACHE names a file, a cached choice for
 * the same (nx, ny, nz, dtype, scheme, form) is used instead of timing, and a
 * new choice is appended to the file (one JSON object per line).  A batch
 * plan then also times a pair of sub-steps with the tuned configurations
 * against one launch per sub-step (x lines fused, y and z both in the tuned
 * y or z configuration) and keeps the faster; it uses no cache.
 * best_ms (host array of 3, may be NULL) receives the best mean launch time
 * per axis (0 when taken from the cache).  Synchronizes the stream. */
fdtd_status fdtd_autotune(fdtd_plan_t p, int reps, double* best_ms);

/* Gradient of a probe objective with respect to eps_r (fundamental ADI,
 * D'Yakonov and Douglas-Gunn plans only, else FDTD_EUNSUPPORTED).
 *   J = dt * sum_{n=1..nsteps} (Ex^2 + Ey^2 + Ez^2)(u^n) at the E samples stored
 *   at the probe node (probe_i, probe_j, probe_k), 1 <= probe_* < n_*,
 * where u^n are the fields fdtd_run would return after n steps from the
 * caller's E, H (read only here, not modified) with source `src` (may be
 * NULL), source times counted from the plan's step counter (unchanged).
 * J_out (host) receives J, accumulated in FP64.  If grad_out is non-NULL it
 * receives dJ/d eps_r for the design cells
 *   design_box = {i0, i1, j0, j1, k0, k1}: cells i0 <= i < i1, ... (host array,
 *   0 <= i0 < i1 <= nx, likewise for y, z),
 * as a device FP64 array [k1-k0][j1-j0][i1-i0], x fastest, overwritten.
 * Method: the adjoint of the ADI time stepping in the link scaling of
 * Sec. II-E.  The transpose of a sub-step's Cayley factor is the same factor
 * with theta -> -theta in the variables scaled by diag(eps, mu)^-1 (X = M^-1 K
 * with K skew-symmetric for eq. (AMat) on the Yee grid), so the reverse sweep
 * runs the fundamental line passes of Sec. III backwards in time; the
 * gradient terms are accumulated in FP64 on the device.  The forward sweep
 * stores the state every `ckpt_every` >= 1 steps; the reverse sweep
 * recomputes each segment from its checkpoint (about two forward runs plus
 * one adjoint run in total; device memory about (nsteps/ckpt_every + 1)
 * states plus (2 ckpt_every + 1) x 3 design-box arrays, kept by the plan for
 * reuse and released by fdtd_destroy).  With grad_out NULL only the forward
 * sweep runs and design_box, ckpt_every are ignored.  The internal state is
 * overwritten.  Synchronizes the plan's stream; FDTD_ENONFINITE if J is not
 * finite. */
fdtd_status fdtd_grad_eps(fdtd_plan_t p, void* const E[3], void* const H[3], int nsteps,
                          const fdtd_source* src, int probe_i, int probe_j, int probe_k,
                          const int* design_box, int ckpt_every, double* J_out, double* grad_out);

/* FP64 distance of two field sets on a single-grid plan's grid (else
 * FDTD_EINVAL for a batch plan):
 *   out[0] = sum eps |Ea - Eb|^2 + mu |Ha - Hb|^2,  out[1] = sum eps |Eb|^2 + mu |Hb|^2
 * over the samples inside each component's extent, eps = eps0 eps_r of the
 * sample's owning cell (as in the energy trace), mu = mu0 mu_r likewise; so
 * sqrt(out[0] / out[1]) is the energy-weighted relative L2 distance of Ea, Ha
 * from Eb, Hb.  Ea, Ha, Eb, Hb: device arrays in the caller's field layout and
 * the plan's element type (read only); out: host array of 2.  Two-stage
 * reduction in a fixed order (deterministic); synchronizes the plan's stream;
 * FDTD_ENONFINITE if a sum is not finite.  The first call allocates 16 KB of
 * device memory kept by the plan. */
fdtd_status fdtd_diff_norm(fdtd_plan_t p, void* const Ea[3], void* const Ha[3], void* const Eb[3],
                           void* const Hb[3], double* out);

/* fdtd_diff_norm without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, result and errors as fdtd_diff_norm
 * (and bit for bit the same out[]); its work area -- at most 2 x 1024
 * partial sums and the 2 results, 16,400 bytes -- is a static device array
 * of the library, one per GPU, held until the process ends (no grid size
 * needs more: the first reduction stage takes at most 1024 blocks).  Every
 * call on a GPU shares that array, so calls that overlap on one GPU (other
 * host threads, other streams) race; calls in sequence are independent
 * (each writes every value it reads).  Calls no hipMalloc or hipFree. */
fdtd_status fdtd_diff_norm_noalloc(fdtd_plan_t p, void* const Ea[3], void* const Ha[3], void* const Eb[3],
                                   void* const Hb[3], double* out);

/* Conjugate-gradient controls of a Crank-Nicolson plan (else
 * FDTD_EUNSUPPORTED): stop when |r| <= tol |b| (0 < tol < 1, checked every
 * fourth iteration) or after maxit >= 1 iterations.  Defaults 1e-12, 500. */
fdtd_status fdtd_set_cg(fdtd_plan_t p, double tol, int maxit);

/* Conjugate-gradient iterations summed over the steps of the last fdtd_run of
 * a Crank-Nicolson plan, and the largest final |r| / |b| among those steps
 * (host pointers, either may be NULL). */
fdtd_status fdtd_last_cg(fdtd_plan_t p, long long* iterations, double* rel_residual);

/* Batch of independent grids stepped together (fundamental forms only, else
 * FDTD_EUNSUPPORTED).  d[0..n-1] describe the grids (each validated as by
 * fdtd_plan; sizes, dt, dx, dy, dz and eps_r may differ; scheme, form and
 * dtype must be equal, else FDTD_EINVAL; Crank-Nicolson: FDTD_EUNSUPPORTED).
 * Every line pass of a sub-step runs as ONE launch over all grids; the y-
 * and z-line passes share that launch when their kernel configurations
 * agree, and by default (x block_threads 0) the x-line pass joins it, so a
 * sub-step is one launch.  The plan keeps a device table of the grids' pass
 * arguments and a work list of (table entry, block) items, and eight time
 * steps of the main iteration are captured once as a HIP graph (on a private
 * stream) and replayed on `hip_stream` (remaining steps are launched
 * directly).  When the fields and media of all grids exceed 128 MiB, the
 * grids are split into groups of consecutive grids of about equal size
 * (each below that bound when possible), and fdtd_run_batch steps one group
 * through all `nsteps` before the next, so that a group's arrays stay in the
 * 256 MB on-die cache between passes; each group is then batched as above.
 * Per-grid state and eps_r as in
 * fdtd_plan.  fdtd_autotune, fdtd_get/set_kernel_config (a configuration
 * must fit every grid), fdtd_set_timing/fdtd_last_timing (main_ms only) and
 * fdtd_destroy accept a batch plan; fdtd_run, fdtd_step and fdtd_grad_eps
 * return FDTD_EINVAL for it. */
fdtd_status fdtd_plan_batch(const fdtd_desc* d, int n, void* hip_stream, fdtd_plan_t* out);

/* Advance every grid of a batch plan by `nsteps` >= 0 steps, with the input
 * and output processing of fdtd_run and no source.  E and H are host arrays
 * of 3n device pointers: E[3g + c] is component c (x, y, z) of grid g, with
 * the layout of fdtd_run, read on entry and overwritten on return.
 * Asynchronous on the plan's stream. */
fdtd_status fdtd_run_batch(fdtd_plan_t p, void* const* E, void* const* H, int nsteps);

/* Destroy a plan: synchronizes its stream and releases everything it holds.
 * Every call checks its handle against the library's live plans before using
 * it, so a destroyed handle is rejected with FDTD_EINVAL rather than read
 * (until a later plan happens to receive the same address). */
fdtd_status fdtd_destroy(fdtd_plan_t p);
const char* fdtd_strerror(fdtd_status s);

#ifdef __cplusplus
}
#endif
#endif /* FDTD_H */
