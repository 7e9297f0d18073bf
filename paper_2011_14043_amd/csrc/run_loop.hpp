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
    k.order = p->order;
    k.wo = p->stencil_wo;
    hipLaunchKernelGGL((energy_partial_kernel<T>), dim3(p->npartial), dim3(256), 0, p->stream,
                       state_ptrs<T>(p, set), p->eps, p->mu, p->dims, k, p->partial);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(64), 0, p->stream, p->partial, p->npartial, dst);
    HIPCHK(hipGetLastError());
    return FDTD_OK;
}

// Input processing into state set 0: U = 1/2 u + link B u (link = dt/4 for
// the ADI link of Sec. II-E), else U = u; with the plan's difference order.
template <typename T, typename S>
static fdtd_status load_state(fdtd_plan_s* p, const FieldPtrs<T>& caller, double link) {
    AuxCoef kin = aux_coef(p->d, link);
    kin.order = p->order;
    kin.wo = p->stencil_wo;
    if (p->order == 4 && link != 0.0) {
        const long long nn = (long long)(p->dims.nx + 1) * (p->dims.ny + 1) * (p->dims.nz + 1);
        hipLaunchKernelGGL((load_state4_kernel<T>), dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, p->stream, caller,
                           state_ptrs_w<T>(p, 0), p->eps, p->mu, p->dims, kin);
    } else {
        hipLaunchKernelGGL((load_state_kernel<T, S>), row_grid(p->dims), dim3(kRowThreads), 0, p->stream, caller,
                           state_ptrs_w<T>(p, 0), p->eps, p->mu, p->dims, kin);
    }
    HIPCHK(hipGetLastError());
    return FDTD_OK;
}

// ---------------------------------------------------------------------------
// captured step graphs (single-grid runs)
// ---------------------------------------------------------------------------
static void graph_clear(fdtd_plan_s* p) {
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->gexec = nullptr;
    p->graph = nullptr;
}

// What a captured graph depends on: steps per graph, the source cell, the
// kernel configuration of the three line axes.
static void graph_key(const fdtd_plan_s* p, const fdtd_source* src, long long (&k)[8]) {
    k[0] = p->graph_steps;
    k[1] = src ? 1 : 0;
    k[2] = src ? src->i : -1;
    k[3] = src ? src->j : -1;
    k[4] = src ? src->k : -1;
    for (int a = 0; a < 3; ++a) {
        const KCfg& c = p->cfg[a];
        k[5 + a] = (long long)c.M | ((long long)c.TX << 8) | ((long long)c.NT << 16) | ((long long)c.wpb << 32) |
                   ((long long)c.remap << 40);
    }
}

// Source terms of sub-step u of main step n of a run (host, as the eager
// loop computes them): pre and post of the Ez sample.
static void source_terms(fdtd_plan_s* p, const fdtd_source* src, int mode, long long nglob, int u, double* pre,
                         double* post) {
    const SubStep& ss = kSchemes[p->d.scheme].sub[u];
    const double theta = ss.theta_frac * p->d.dt;
    const Inject inj = source_inject(p, src, source_value(src, theta, (double(nglob) + ss.t_frac) * p->d.dt), mode);
    *pre = inj.pre[2];
    *post = inj.post[2];
}

// Capture graph_steps main-iteration steps (all sub-steps, state set 0 in,
// set 0 out) on the plan's private stream; with a source, the passes read
// their pre/post values from src_win.
template <typename T, typename S>
static fdtd_status graph_capture(fdtd_plan_s* p, const fdtd_source* src, int mode) {
    // replays of the old graph may still be queued: let them finish before its
    // executable (kernel arguments included) is released
    if (p->gexec) HIPCHK(hipStreamSynchronize(p->stream));
    graph_clear(p);
    const SchemeDef& sd = kSchemes[p->d.scheme];
    const int K = p->graph_steps;
    if (!p->gstream) HIPCHK(hipStreamCreateWithFlags(&p->gstream, hipStreamNonBlocking));
    if (src && !p->src_win) HIPCHK(hipMalloc(&p->src_win, sizeof(double) * 6 * 3 * 64));
    if ((size_t)K * sd.nsub * 6 > 6 * 3 * 64) return FDTD_EINVAL;
    hipStream_t user = p->stream;
    p->stream = p->gstream;
    fdtd_status st = FDTD_OK;
    if (hipStreamBeginCapture(p->gstream, hipStreamCaptureModeThreadLocal) != hipSuccess) st = FDTD_EDEVICE;
    int cur = 0;
    for (int q = 0; q < K && st == FDTD_OK; ++q) {
        for (int u = 0; u < sd.nsub && st == FDTD_OK; ++u) {
            const SubStep& ss = sd.sub[u];
            Inject inj;
            if (src) {
                inj.i = src->i; inj.j = src->j; inj.k = src->k;
                inj.mask = 4u;   // Ez
                inj.pre_dev = p->src_win + (size_t)(q * sd.nsub + u) * 6;
                inj.post_dev = inj.pre_dev + 3;
            }
            // The three pair passes of a sub-step are captured as a chain on
            // the capture stream.  (They write disjoint arrays and could run as
            // parallel branches forked and joined on events; that form was
            // faster on small grids but is not used: a process that replayed
            // such graphs ended once in an abort whose cause was not found.)
            const int out = (mode == CONV_ADI) ? 1 - cur : cur;
            for (int k = 0; k < 3 && st == FDTD_OK; ++k)
                st = launch_pass<T, S>(p, ss.op, k, ss.theta_frac * p->d.dt, mode, set_ptr<T>(p, cur),
                                       set_ptr<T>(p, out), src ? &inj : nullptr, false);
            cur = out;
        }
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->gstream, &g);
    p->stream = user;
    if (st != FDTD_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return st != FDTD_OK ? st : from_hip(e);
    }
    p->graph = g;
    HIPCHK(hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0));
    graph_key(p, src, p->gkey);
    return FDTD_OK;
}

// Main steps [0, ngraph * graph_steps) of a run as graph replays.
template <typename T, typename S>
static fdtd_status run_graphs(fdtd_plan_s* p, const fdtd_source* src, int mode, int ngraph) {
    const SchemeDef& sd = kSchemes[p->d.scheme];
    const int K = p->graph_steps;
    const size_t per_graph = (size_t)K * sd.nsub * 6;
    if (src) {
        // the source terms of the covered steps, once per run
        const size_t need = (size_t)ngraph * per_graph;
        if (need > p->src_cap) {
            if (p->src_copied) HIPCHK(hipEventSynchronize(p->src_copied));
            if (p->src_dev) HIPCHK(hipFree(p->src_dev));
            if (p->src_host) HIPCHK(hipHostFree(p->src_host));
            p->src_dev = nullptr;
            p->src_host = nullptr;
            p->src_cap = 0;
            HIPCHK(hipMalloc(&p->src_dev, sizeof(double) * need));
            HIPCHK(hipHostMalloc(&p->src_host, sizeof(double) * need, hipHostMallocDefault));
            p->src_cap = need;
        }
        if (!p->src_copied) HIPCHK(hipEventCreateWithFlags(&p->src_copied, hipEventDisableTiming));
        HIPCHK(hipEventSynchronize(p->src_copied));   // the previous run's copy has read the staging
        double* h = p->src_host;
        for (int n = 0; n < ngraph * K; ++n)
            for (int u = 0; u < sd.nsub; ++u) {
                double* r = h + ((size_t)n * sd.nsub + u) * 6;
                r[0] = r[1] = r[3] = r[4] = 0.0;
                source_terms(p, src, mode, p->step + n, u, &r[2], &r[5]);
            }
        HIPCHK(hipMemcpyAsync(p->src_dev, h, sizeof(double) * need, hipMemcpyHostToDevice, p->stream));
        HIPCHK(hipEventRecord(p->src_copied, p->stream));
    }
    long long key[8];
    graph_key(p, src, key);
    if (!p->gexec || std::memcmp(key, p->gkey, sizeof(key)) != 0) {
        fdtd_status st = graph_capture<T, S>(p, src, mode);
        if (st != FDTD_OK) return st;
    }
    for (int m = 0; m < ngraph; ++m) {
        if (src)
            HIPCHK(hipMemcpyAsync(p->src_win, p->src_dev + (size_t)m * per_graph, sizeof(double) * per_graph,
                                  hipMemcpyDeviceToDevice, p->stream));
        HIPCHK(hipGraphLaunch(p->gexec, p->stream));
    }
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
    {
        const fdtd_status st = load_state<T, S>(p, caller, (adi && !conv) ? 0.25 * d.dt : 0.0);
        if (st != FDTD_OK) return st;
    }
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
    // state before it need not be kept.  The other schemes' output is U_new of
    // their last sub-step (LOD2: of the output processing sub-step).  Unless
    // an energy trace reads the final state (or the passes are the in-place
    // fourth-order ones, or conventional with a permeability map), the last
    // passes store the output straight into the caller's arrays and
    // store_faces_kernel writes the wall samples no pass writes; else the
    // state takes it and store_out_kernel copies it.
    const bool fin_adi = adi && !conv;
    const bool lod2 = d.scheme == FDTD_LOD2;
    // The last passes of a run are FIN instantiations wherever those are built
    // (second-order passes except conventional ones with a permeability map;
    // fourth-order ones for ADI only), whether the output goes to the caller
    // or to the state, so both destinations get the same arithmetic.
    const bool fin_last = fin_adi || (p->order == 2 && !(p->mu && conv));
    const bool direct = !energy && p->order == 2 && !(p->mu && conv);
    Fin fin;
    fin.add = fin_adi;
    if (direct) {
        fin.E = E;
        fin.H = H;
    }
    // Steps before the last one run as replays of a captured graph of
    // graph_steps steps (no energy trace or per-launch timing), the rest
    // directly.
    const int ngraph = (p->graph_steps > 0 && !energy && tm.per_launch == 0) ? (nsteps - 1) / p->graph_steps : 0;
    if (ngraph > 0) {
        fdtd_status st = run_graphs<T, S>(p, src, mode, ngraph);
        if (st != FDTD_OK) return st;
    }
    for (int n = ngraph * p->graph_steps; n < nsteps; ++n) {
        const long long nglob = p->step + n;
        for (int u = 0; u < sd.nsub; ++u) {
            const SubStep& ss = sd.sub[u];
            const double theta = ss.theta_frac * d.dt;
            const double g = source_value(src, theta, (double(nglob) + ss.t_frac) * d.dt);
            const Inject inj = source_inject(p, src, g, mode);
            const bool timed = tm.per_launch > 0 && n % tm.per_launch == 0;
            const bool last = fin_last && !lod2 && n == nsteps - 1 && u == sd.nsub - 1;
            if (last) fin.src = (fin_adi && src) ? 0.5 * g : 0.0;
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
        if (lod2) {
            fdtd_status st = substep<T, S>(p, 1, -0.25 * d.dt, mode, cur, nullptr, false, fin_last ? &fin : nullptr);
            if (st != FDTD_OK) return st;
        }
        if (direct) {
            const int nface = 2 * (dm.nz + 1) + 2 * (dm.ny - 1);
            const long long rows = (long long)(dm.ny + 1) * (dm.nz + 1);
            const unsigned nblk = (unsigned)(nface + (rows + kRowThreads - 1) / kRowThreads);
            hipLaunchKernelGGL((store_faces_kernel<T>), dim3(nblk), dim3(kRowThreads), 0, p->stream,
                               state_ptrs<T>(p, cur), caller_w, dm, fin_adi ? 1 : 0, nface);
        } else
            hipLaunchKernelGGL((store_out_kernel<T>), row_grid(dm), dim3(kRowThreads), 0, p->stream,
                               state_ptrs<T>(p, cur), caller_w, dm, fin_adi ? 1 : 0);
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
