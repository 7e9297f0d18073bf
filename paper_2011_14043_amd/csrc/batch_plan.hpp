// batch_plan.hpp -- batch plans: pass tables and work lists, launches, captured step
// graphs, groups sized to the MALL, batch autotuning
//
// Part of the single translation unit of libfdtd.so: included by fdtd.hip
// after the kernel headers and the headers before it in fdtd.hip.
#pragma once

namespace fdtd {

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

// x lines of a batch with no block size of their own (wpb = 0) run inside
// the y/z launch of their sub-step, in blocks of its size (fused launch);
// where that launch is not available they run alone in blocks of 4 waves.
static KCfg x_alone_cfg(const fdtd_plan_s* p) {
    KCfg c = p->cfg[0];
    if (c.wpb == 0) c.wpb = 4;
    return c;
}

static bool refined_batch_cfg(int axis, const KCfg& c) {
    return c.M == 8 || (axis != 0 && c.M == 16 && c.NT == 512);
}

static bool batch_cfg_valid(const fdtd_plan_s* p, int axis, const KCfg& c0) {
    KCfg c = c0;
    if (axis == 0 && c.wpb == 0) c.wpb = 4;
    // refined batched passes: 8-slot chunks, or 16-slot y/z chunks in blocks of
    // at most 512 threads (136 VGPRs with the batch addressing; a 1024-thread
    // bound would cap them at 128)
    if (p->refine && !refined_batch_cfg(axis, c)) return false;
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
        if (axis == 0) pref = {{8, 0, 0, 0, 0}, {16, 0, 0, 4, 0}};   // 8-slot chunks fused where possible
        else if (p->d.dtype == FDTD_F32) pref = {{8, 16, 1024, 0, 0}, {16, 32, 1024, 0, 0}, {16, 16, 512, 0, 0}, {32, 16, 512, 0, 0}};
        else pref = {{8, 8, 512, 0, 0}, {16, 16, 512, 0, 0}};
        for (const KCfg& c : pref)
            if (batch_cfg_valid(p, axis, c)) { p->cfg[axis] = c; break; }
    }
}

// y and z lines share a kernel; their passes can run as one launch when the
// two axes have the same configuration.
static bool yz_same_cfg(const fdtd_plan_s* p) {
    return p->cfg[1].M == p->cfg[2].M && p->cfg[1].TX == p->cfg[2].TX && p->cfg[1].NT == p->cfg[2].NT;
}

// Kernel configurations {M, TX, NT} of the y/z lines with a fused launch (x
// lines with 8-slot chunks), by solve precision.
static const int kSubF32[][3] = {{8, 16, 1024}, {8, 32, 512}, {16, 32, 1024}, {16, 16, 512}};
static const int kSubF64[][3] = {{8, 8, 512}, {8, 16, 1024}, {16, 16, 512}};

static bool same_kcfg(const KCfg& a, const KCfg& b) {
    return a.M == b.M && a.TX == b.TX && a.NT == b.NT && a.wpb == b.wpb && a.remap == b.remap;
}

static bool fused_ok(const fdtd_plan_s* p) {
    if (p->cfg[0].wpb != 0 || p->cfg[0].M != 8 || !yz_same_cfg(p)) return false;
    const KCfg& c = p->cfg[1];
    if (p->refine && !refined_batch_cfg(1, c)) return false;
    if (p->d.dtype == FDTD_F32) {
        for (const auto& v : kSubF32)
            if (v[0] == c.M && v[1] == c.TX && v[2] == c.NT) return true;
    } else {
        for (const auto& v : kSubF64)
            if (v[0] == c.M && v[1] == c.TX && v[2] == c.NT) return true;
    }
    return false;
}

// Launches of one sub-step with operator op: all three pairs in one launch
// when the x lines are fused (above); otherwise the x-line pair alone, and
// the y- and z-line pairs together when they share a configuration (else one
// each).
static int substep_masks(const fdtd_plan_s* p, int op, int (&masks)[3]) {
    if (fused_ok(p)) {
        masks[0] = 7;
        return 1;
    }
    int yz = 0, n = 0;
    for (int k = 0; k < 3; ++k) {
        if (kPairs[op][k].w == 0) masks[n++] = 1 << k;
        else yz |= 1 << k;
    }
    if (yz_same_cfg(p)) {
        masks[n++] = yz;
    } else {
        for (int k = 0; k < 3; ++k)
            if (yz & (1 << k)) masks[n++] = 1 << k;
    }
    return n;
}

// The table of the passes (op, k in mask) with theta = frac * dt for every grid
// (built on first use with the current kernel configuration).  Entry
// j * ngrids + g is the j-th pair of the mask (y/z pairs first) on grid g; a
// work item (entry, block) names one block of one of them.
template <typename T, typename S>
static fdtd_status batch_pass(fdtd_plan_s* p, int op, int mask, double frac, const BatchPass** out) {
    Batch* b = p->batch;
    for (const BatchPass& bp : b->passes)
        if (bp.op == op && bp.mask == mask && bp.frac == frac) { *out = &bp; return FDTD_OK; }
    int ks[3], nk = 0, nyz = 0;
    for (int x = 0; x < 2; ++x)
        for (int k = 0; k < 3; ++k)
            if ((mask & (1 << k)) && (kPairs[op][k].w == 0) == (x == 1)) ks[nk++] = k;
    for (int j = 0; j < nk; ++j) nyz += kPairs[op][ks[j]].w != 0;
    if (nk == 0) return FDTD_EINVAL;
    const bool fused = nyz > 0 && nyz < nk;
    if (fused && (nk != 3 || !fused_ok(p))) return FDTD_EINVAL;
    const int w = kPairs[op][ks[0]].w;
    const KCfg cf = w == 0 ? x_alone_cfg(p) : p->cfg[w];
    for (int j = 1; j < nyz; ++j) {   // one launch needs one y/z kernel configuration
        const KCfg& c2 = p->cfg[kPairs[op][ks[j]].w];
        if (c2.M != cf.M || c2.TX != cf.TX || c2.NT != cf.NT) return FDTD_EINVAL;
    }
    if (nyz == 0 && nk > 1) return FDTD_EINVAL;
    const int n = (int)b->subs.size();
    const int ne = n * nk;
    std::vector<PassArgs<T, S>> tab(ne);
    int Pmax = 1;   // y/z entries: block = TX * Pmax threads
    auto build = [&](int j, const KCfg& c) {
        const int wj = kPairs[op][ks[j]].w;
        for (int g = 0; g < n; ++g) {
            fdtd_plan_s* sub = b->subs[g];
            PassArgs<T, S>& a = tab[j * n + g];
            sub->cfg[wj] = c;
            PassShape sh;
            build_pass<T, S>(sub, op, ks[j], frac * sub->d.dt, FUND, set_ptr<T>(sub, 0), set_ptr<T>(sub, 0), nullptr,
                             a, sh);
            a.P = batch_P(sub, wj, c);
            a.remap = 0;
            if (wj != 0) Pmax = std::max(Pmax, a.P);
        }
    };
    for (int j = 0; j < nyz; ++j) build(j, p->cfg[kPairs[op][ks[j]].w]);
    const int threads = nyz > 0 ? cf.TX * Pmax : 64 * cf.wpb;
    if (nyz < nk) {   // the x pair: blocks of `threads` threads
        KCfg cx = x_alone_cfg(p);
        cx.wpb = threads / 64;
        build(nyz, cx);
    }
    std::vector<int2> iyz, ix;
    int lds_rows = 0;   // y/z: sub-block areas x chunks, the most any entry needs
    for (int e = 0; e < ne; ++e) {
        const bool yz = e < nyz * n;
        const int per = yz ? Pmax / tab[e].P : 1;   // virtual blocks per block
        const int nit = (tab[e].nblk + per - 1) / per;
        for (int q = 0; q < nit; ++q) (yz ? iyz : ix).push_back(make_int2(e, q));
        if (yz) lds_rows = std::max(lds_rows, ((Pmax + tab[e].P - 1) / tab[e].P) * tab[e].P);
    }
    // Interleave the two kinds in proportion: each XCD runs a contiguous
    // range of the list.
    std::vector<int2> items;
    items.reserve(iyz.size() + ix.size());
    for (size_t u = 0, v = 0; u < iyz.size() || v < ix.size();) {
        if (v >= ix.size() || (u < iyz.size() && u * ix.size() <= v * iyz.size())) items.push_back(iyz[u++]);
        else items.push_back(ix[v++]);
    }
    BatchPass bp;
    bp.op = op; bp.mask = mask; bp.w = w; bp.frac = frac; bp.Pmax = Pmax;
    bp.ex0 = fused ? nyz * n : -1;
    bp.threads = threads;
    bp.lds = (size_t)(p->refine ? 13 : 9) * lds_rows * (cf.TX + 1) * sizeof(S);
    bp.nitems = (int)items.size();
    HIPCHK(hipMalloc(&bp.tab, sizeof(PassArgs<T, S>) * ne));
    hipError_t e = hipMalloc(&bp.items, sizeof(int2) * items.size());
    if (e == hipSuccess) e = hipMemcpy(bp.tab, tab.data(), sizeof(PassArgs<T, S>) * ne, hipMemcpyHostToDevice);
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

template <typename T, typename S>
static fdtd_status batch_launch(fdtd_plan_s* p, const BatchPass& bp, hipStream_t st) {
    const KCfg& cf = p->cfg[bp.w];
    const int kmode = (sizeof(S) == 4 && p->refine) ? FUND_REF : FUND;
    const int kind = bp.ex0 >= 0 ? 2 : (bp.w == 0 ? 0 : 1);
    if (kind == 2 && p->cfg[0].M != 8) return FDTD_EINVAL;
    const int r = dispatch_batch<T, S>(kmode, kind, cf.M, cf.TX, cf.NT, p->batch->mat, dim3((unsigned)bp.nitems),
                                       dim3(bp.threads), kind == 0 ? 0 : bp.lds, st,
                                       static_cast<const PassArgs<T, S>*>(bp.tab), static_cast<const int2*>(bp.items),
                                       bp.ex0);
    if (r != DISPATCH_OK) return FDTD_EUNSUPPORTED;
    HIPCHK(hipGetLastError());
    return FDTD_OK;
}

// One sub-step (operator op, theta = frac * dt) of every grid: one, two or three launches.
template <typename T, typename S>
static fdtd_status batch_substep(fdtd_plan_s* p, int op, double frac, hipStream_t st) {
    int masks[3];
    const int nl = substep_masks(p, op, masks);
    for (int l = 0; l < nl; ++l) {
        const BatchPass* bp = nullptr;
        fdtd_status s = batch_pass<T, S>(p, op, masks[l], frac, &bp);
        if (s != FDTD_OK) return s;
        s = batch_launch<T, S>(p, *bp, st);
        if (s != FDTD_OK) return s;
    }
    return FDTD_OK;
}

template <typename T, typename S>
static fdtd_status batch_tables(fdtd_plan_s* p) {
    const SchemeDef& sd = kSchemes[p->d.scheme];
    int masks[3];
    for (int u = 0; u < sd.nsub; ++u) {
        const int nl = substep_masks(p, sd.sub[u].op, masks);
        for (int l = 0; l < nl; ++l) {
            const BatchPass* bp = nullptr;
            fdtd_status s = batch_pass<T, S>(p, sd.sub[u].op, masks[l], sd.sub[u].theta_frac, &bp);
            if (s != FDTD_OK) return s;
        }
    }
    if (p->d.scheme == FDTD_LOD2)
        for (double f : {0.25, -0.25}) {
            const int nl = substep_masks(p, 1, masks);
            for (int l = 0; l < nl; ++l) {
                const BatchPass* bp = nullptr;
                fdtd_status s = batch_pass<T, S>(p, 1, masks[l], f, &bp);
                if (s != FDTD_OK) return s;
            }
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
    // The launches of every sub-step (one when the sub-step is fused, else
    // one per group of passes) are captured as a chain on the capture stream,
    // as the single-grid graphs are (no branches forked and joined on events).
    HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    fdtd_status st = FDTD_OK;
    for (int v = 0; v < kGraphSteps * sd.nsub && st == FDTD_OK; ++v) {
        const int u = v % sd.nsub;
        const int op = sd.sub[u].op;
        const double frac = sd.sub[u].theta_frac;
        int masks[3];
        const int nl = substep_masks(p, op, masks);
        for (int l = 0; l < nl && st == FDTD_OK; ++l) {
            const BatchPass* bp = nullptr;
            st = batch_pass<T, S>(p, op, masks[l], frac, &bp);
            if (st == FDTD_OK) st = batch_launch<T, S>(p, *bp, b->cap);
        }
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
    if (adi && nsteps > 0) {   // the state before the last B sub-step (output processing)
        for (fdtd_plan_s* sub : b->subs)
            if (!sub->snap) HIPCHK(hipMalloc(&sub->snap, sizeof(T) * sub->dims.comp * 6));
    }
    for (int g = 0; g < n; ++g) {
        fdtd_plan_s* sub = b->subs[g];
        const Dims& dm = sub->dims;
        const long long nn = (long long)(dm.nx + 1) * (dm.ny + 1) * (dm.nz + 1);
        const AuxCoef kin = aux_coef(sub->d, adi ? 0.25 * sub->d.dt : 0.0);
        hipLaunchKernelGGL((load_state_kernel<T, S>), row_grid(dm), dim3(kRowThreads), 0, p->stream,
                           caller(g), state_ptrs_w<T>(sub, 0), sub->eps, sub->mu, dm, kin);
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
            st = batch_pass<T, S>(p, 0, 1 << k, 0.5, &bp);
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
    // Joint choice: the configurations tuned above with separate launches, or
    // one launch per sub-step (x lines fused) with both y and z in the y or in
    // the z configuration; timed over sub-step pairs launched on the stream.
    if (st == FDTD_OK) {
        const KCfg tuned[3] = {p->cfg[0], p->cfg[1], p->cfg[2]};
        std::vector<std::array<KCfg, 3>> cand = {{tuned[0], tuned[1], tuned[2]}};
        for (int src = 1; src <= 2; ++src) {
            if (src == 2 && same_kcfg(tuned[1], tuned[2])) break;
            const KCfg c0{8, 0, 0, 0, tuned[0].remap}, cy = tuned[src];
            if (!batch_cfg_valid(p, 0, c0) || !batch_cfg_valid(p, 1, cy) || !batch_cfg_valid(p, 2, cy)) continue;
            p->cfg[0] = c0;
            p->cfg[1] = p->cfg[2] = cy;
            if (fused_ok(p)) cand.push_back({c0, cy, cy});
        }
        int ibest = 0;
        float tbest = 1e30f;
        for (size_t i = 0; i < cand.size() && cand.size() > 1 && st == FDTD_OK; ++i) {
            for (int a = 0; a < 3; ++a) p->cfg[a] = cand[i][a];
            batch_clear(b);
            float ms = 0.0f;
            for (int r = 0; r <= reps && st == FDTD_OK; ++r) {   // r = 0: build the tables, warm up
                if (r == 1 && hipEventRecord(e0, p->stream) != hipSuccess) st = FDTD_EDEVICE;
                if (st == FDTD_OK) st = batch_substep<T, S>(p, 0, 0.5, p->stream);
                if (st == FDTD_OK) st = batch_substep<T, S>(p, 1, 0.5, p->stream);
            }
            if (st != FDTD_OK) break;
            if (hipEventRecord(e1, p->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                st = FDTD_EDEVICE;
                break;
            }
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < tbest) { tbest = ms; ibest = (int)i; }
        }
        for (int a = 0; a < 3; ++a) p->cfg[a] = cand[ibest][a];
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
