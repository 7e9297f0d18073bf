// cn_solver.hpp -- host side of the Crank-Nicolson plans (Sec. II-E): the
// conjugate-gradient loop of each step around the kernels of cn_kernels.hpp
//
// Part of the single translation unit of libfdtd.so: included by fdtd.hip
// after the kernel headers and the headers before it in fdtd.hip.
#pragma once

namespace fdtd {

constexpr int kCgCheck = 4;   // iterations between two reads of the residual on the host

static CnArgs cn_args(fdtd_plan_s* p) {
    CnArgs a;
    a.d = p->dims;
    a.rdx = 1.0 / p->d.dx;
    a.rdy = 1.0 / p->d.dy;
    a.rdz = 1.0 / p->d.dz;
    a.eps0 = kEps0;
    a.rmu0 = 1.0 / kMu0;
    a.theta = 0.5 * p->d.dt;
    a.eps = p->eps;
    a.mu = p->mu;
    for (int c = 0; c < 6; ++c) a.u[c] = comp_ptr<double>(p, 0, c);
    const size_t n = (size_t)p->dims.comp;
    for (int c = 0; c < 3; ++c) {
        a.x[c] = p->cg + (0 + c) * n;
        a.r[c] = p->cg + (3 + c) * n;
        a.p[c] = p->cg + (6 + c) * n;
        a.q[c] = p->cg + (9 + c) * n;
        a.w[c] = p->cg + (12 + c) * n;
    }
    a.partial = p->cg_partial;
    a.scal = p->cg_scal;
    a.src_off = -1;
    a.src_g = 0.0;
    return a;
}

static fdtd_status cn_reduce(fdtd_plan_s* p, int m, CnSlots s) {
    hipLaunchKernelGGL(cn_reduce_kernel, dim3(m), dim3(kCnThreads), 0, p->stream, p->cg_partial, p->cg_scal, s);
    HIPCHK(hipGetLastError());
    return FDTD_OK;
}

#define CN_LAUNCH(kernel, ...)                                                                         \
    do {                                                                                               \
        hipLaunchKernelGGL(kernel, dim3(kCnBlocks), dim3(kCnThreads), 0, p->stream, __VA_ARGS__);      \
        HIPCHK(hipGetLastError());                                                                     \
    } while (0)

// One Crank-Nicolson step on the plan's state.  Adds the iterations to
// *iters and returns the final relative residual |r| / |b| in *rel.
static fdtd_status cn_step(fdtd_plan_s* p, const CnArgs& a, long long* iters, double* rel) {
    const bool conv = p->d.form == FDTD_CONVENTIONAL;
    fdtd_status st;
    if (conv) {   // classical form: explicit right side, guess u_E, residual by one product
        CN_LAUNCH(cn_conv_rhs_kernel, a);
        CN_LAUNCH(cn_conv_start_kernel, a);
        if ((st = cn_reduce(p, 1, CnSlots{{kBb, 0, 0}})) != FDTD_OK) return st;
        CN_LAUNCH(cn_apply_kernel, a);
        CN_LAUNCH(cn_conv_resid_kernel, a);
        st = cn_reduce(p, 2, CnSlots{{kRz0, kRr, 0}});
    } else {
        CN_LAUNCH(cn_start_h_kernel, a);
        CN_LAUNCH(cn_start_e_kernel, a);
        st = cn_reduce(p, 3, CnSlots{{kRz0, kRr, kBb}});
    }
    if (st != FDTD_OK) return st;
    double host[2] = {0.0, 0.0};   // r.r, b.b
    int it = 0;
    *rel = 0.0;
    while (it < p->cg_maxit) {
        if (it > 0) CN_LAUNCH(cn_direction_kernel, a, it & 1);
        CN_LAUNCH(cn_apply_kernel, a);
        if ((st = cn_reduce(p, 1, CnSlots{{kPq, 0, 0}})) != FDTD_OK) return st;
        CN_LAUNCH(cn_update_kernel, a, it & 1);
        if ((st = cn_reduce(p, 2, CnSlots{{(it & 1) ? kRz0 : kRz1, kRr, 0}})) != FDTD_OK) return st;
        ++it;
        if (it % kCgCheck == 0 || it == p->cg_maxit) {
            HIPCHK(hipMemcpyAsync(host, p->cg_scal + kRr, sizeof(host), hipMemcpyDeviceToHost, p->stream));
            HIPCHK(hipStreamSynchronize(p->stream));
            if (!std::isfinite(host[0]) || !std::isfinite(host[1])) return FDTD_ENONFINITE;
            *rel = host[1] > 0.0 ? std::sqrt(host[0] / host[1]) : 0.0;
            if (*rel <= p->cg_tol) break;
        }
    }
    *iters += it;
    if (conv) CN_LAUNCH(cn_conv_finish_kernel, a);
    else CN_LAUNCH(cn_finish_kernel, a);
    return *rel <= p->cg_tol ? FDTD_OK : FDTD_ENOTCONVERGED;
}

#undef CN_LAUNCH

static fdtd_status cn_run_impl(fdtd_plan_s* p, void* const E[3], void* const H[3], int nsteps,
                               const fdtd_source* src, double* energy, int every) {
    const Dims& dm = p->dims;
    const long long nn = (long long)(dm.nx + 1) * (dm.ny + 1) * (dm.nz + 1);
    const unsigned gblocks = (unsigned)((nn + 255) / 256);
    FieldPtrs<double> caller;
    FieldPtrsW<double> caller_w;
    for (int c = 0; c < 3; ++c) {
        caller.c[c] = static_cast<const double*>(E[c]);
        caller.c[3 + c] = static_cast<const double*>(H[c]);
        caller_w.c[c] = static_cast<double*>(E[c]);
        caller_w.c[3 + c] = static_cast<double*>(H[c]);
    }
    const int nrec = energy ? nsteps / every + 1 : 0;
    if (nrec > p->energy_cap) {
        if (p->energy_dev) HIPCHK(hipFree(p->energy_dev));
        p->energy_dev = nullptr;
        HIPCHK(hipMalloc(&p->energy_dev, sizeof(double) * nrec));
        p->energy_cap = nrec;
    }
    hipLaunchKernelGGL((load_state_kernel<double>), row_grid(p->dims), dim3(kRowThreads), 0, p->stream, caller,
                       state_ptrs_w<double>(p, 0), p->eps, p->mu, dm, aux_coef(p->d, 0.0));
    HIPCHK(hipGetLastError());
    Timing& tm = p->tm;
    tm.used = 0;
    tm.fam.clear();
    if (!tm.main0) {
        HIPCHK(hipEventCreate(&tm.main0));
        HIPCHK(hipEventCreate(&tm.main1));
    }
    HIPCHK(hipEventRecord(tm.main0, p->stream));
    fdtd_status st = FDTD_OK;
    if (energy && (st = energy_into<double>(p, 0, p->energy_dev)) != FDTD_OK) return st;
    CnArgs a = cn_args(p);
    if (src) a.src_off = (long long)src->k * dm.plane + (long long)src->j * dm.px + src->i;
    p->cg_iters = 0;
    p->cg_rel = 0.0;
    fdtd_status conv = FDTD_OK;
    for (int n = 0; n < nsteps; ++n) {
        // one source term per step, at its middle (theta = dt / 2)
        a.src_g = source_value(src, 0.5 * p->d.dt, (double(p->step + n) + 0.5) * p->d.dt);
        double rel = 0.0;
        st = cn_step(p, a, &p->cg_iters, &rel);
        p->cg_rel = std::max(p->cg_rel, rel);
        if (st == FDTD_ENOTCONVERGED) conv = st;
        else if (st != FDTD_OK) return st;
        if (energy && (n + 1) % every == 0 && (st = energy_into<double>(p, 0, p->energy_dev + (n + 1) / every)) != FDTD_OK)
            return st;
    }
    HIPCHK(hipEventRecord(tm.main1, p->stream));
    if (nsteps > 0) {
        hipLaunchKernelGGL((store_state_kernel<double>), dim3(gblocks), dim3(256), 0, p->stream,
                           state_ptrs<double>(p, 0), state_ptrs<double>(p, 0), caller_w, dm, 0, -1LL, 0.0);
        HIPCHK(hipGetLastError());
    }
    p->step += nsteps;
    if (energy) {
        HIPCHK(hipMemcpyAsync(energy, p->energy_dev, sizeof(double) * nrec, hipMemcpyDeviceToHost, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
        for (int m = 0; m < nrec; ++m)
            if (!std::isfinite(energy[m])) return FDTD_ENONFINITE;
    }
    return conv;
}

}  // namespace fdtd
