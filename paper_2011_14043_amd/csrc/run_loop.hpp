// run_loop.hpp -- the main iteration of a single-grid plan: input processing, time
// steps with source and energy trace, output processing
//
// Part of the single translation unit of libfdtd.so: included by fdtd.hip
// after the kernel headers and the headers before it in fdtd.hip.
#pragma once

namespace fdtd {

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

// Energy of the main-iteration state (ADI: of (1/2 I + dt/4 B) u, the
// fundamental state itself, the conventional one through the link).
// fin_form: a fundamental ADI state in output form (after the last B
// sub-step of a run), whose energy is taken through the link as well.
template <typename T>
static fdtd_status energy_into(fdtd_plan_s* p, int set, double* dst, bool fin_form = false) {
    AuxCoef k = aux_coef(p->d, 0.0);
    if (p->d.scheme == FDTD_ADI && (p->d.form == FDTD_CONVENTIONAL || fin_form)) k.link = 0.25 * p->d.dt;
    k.fin_form = fin_form ? 1 : 0;
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
    hipLaunchKernelGGL((load_state_kernel<T, S>), row_grid(dm), dim3(kRowThreads), 0, p->stream, caller, state_ptrs_w<T>(p, 0),
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
    // Output processing of the fundamental ADI rides on the passes of the
    // run's last B sub-step: they store u = U_old + U_new (the v of that
    // sub-step, with g/2 added back at the source) instead of U_new, so the
    // state before it need not be kept; store_out_kernel copies the state to
    // the caller.  The other schemes' state is u after their last sub-step.
    const bool fin_adi = adi && !conv;
    Fin fin{0.0};
    for (int n = 0; n < nsteps; ++n) {
        const long long nglob = p->step + n;
        for (int u = 0; u < sd.nsub; ++u) {
            const SubStep& ss = sd.sub[u];
            const double theta = ss.theta_frac * d.dt;
            const double g = source_value(src, theta, (double(nglob) + ss.t_frac) * d.dt);
            const Inject inj = source_inject(p, src, g, mode);
            const bool timed = tm.per_launch > 0 && n % tm.per_launch == 0;
            const bool last = fin_adi && n == nsteps - 1 && u == sd.nsub - 1;
            if (last) fin.src = src ? 0.5 * g : 0.0;
            fdtd_status st = substep<T, S>(p, ss.op, theta, mode, cur, &inj, timed, last ? &fin : nullptr);
            if (st != FDTD_OK) return st;
        }
        if (energy && (n + 1) % every == 0) {
            fdtd_status st = energy_into<T>(p, cur, p->energy_dev + (n + 1) / every, fin_adi && n == nsteps - 1);
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
        hipLaunchKernelGGL((store_out_kernel<T>), row_grid(dm), dim3(kRowThreads), 0, p->stream, state_ptrs<T>(p, cur),
                           caller_w, dm, fin_adi ? 1 : 0);
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

}  // namespace fdtd
