// pass_launch.hpp -- one line pass: kernel variant dispatch, source injection, pass
// arguments, launch and sub-step
//
// Part of the single translation unit of libfdtd.so: included by fdtd.hip
// after the kernel headers and the headers before it in fdtd.hip.
#pragma once

namespace fdtd {

// ---------------------------------------------------------------------------
// one line pass
// ---------------------------------------------------------------------------
// Right-hand-side injection of one sub-step at the E samples stored at node
// (i, j, k): component c (bit c of mask) gets `pre` added to its state before
// the solve (FUND; the conventional forms add it to the right-hand side) and
// `post` subtracted from the FUND output.  pre_dev / post_dev (device, 3
// doubles each), if set, supply the pre / post values instead (captured
// graphs, adjoint seeds).
struct Inject {
    int i = 0, j = 0, k = 0;
    unsigned mask = 0;
    double pre[3] = {0, 0, 0}, post[3] = {0, 0, 0};
    const double* pre_dev = nullptr;
    const double* post_dev = nullptr;
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

// The last passes of a run store its output.  Fundamental ADI (add): u =
// U_old + U_new, the output processing fused into the passes of the last B
// sub-step; other schemes: U_new.  With E and H set, straight into the
// caller's arrays (their own pitches), else in place in the state.
struct Fin {
    double src = 0.0;             // g/2 of this sub-step, added back at the source sample (add)
    bool add = true;
    void* const* E = nullptr;     // caller's E, H (or NULL: the state)
    void* const* H = nullptr;
};

// Coefficients of the input/output and energy kernels (reciprocals formed here).
static AuxCoef aux_coef(const fdtd_desc& d, double link) {
    return AuxCoef{kEps0, kMu0, 1.0 / kMu0, 1.0 / d.dx, 1.0 / d.dy, 1.0 / d.dz, link, 0};
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
    bool mu = false;      // permeability-map variant
};

// Arguments and launch shape of the pass of pair k of operator op (half-span
// theta, mode) from state set `set_in` to `set_out` of plan p, with the plan's
// kernel configuration for the line axis.
template <typename T, typename S>
static void build_pass(fdtd_plan_s* p, int op, int k, double theta, int mode, T* set_in, T* set_out,
                       const Inject* inj, PassArgs<T, S>& a, PassShape& sh, const Fin* fin = nullptr) {
    const PairDef& pd = kPairs[op][k];
    const Dims& d = p->dims;
    std::memset(&a, 0, sizeof(a));
    const size_t cs = (size_t)d.comp;
    a.Ein = set_in + pd.ce * cs;
    a.Hin = set_in + pd.ch * cs;
    a.Eout = set_out + pd.ce * cs;
    a.Hout = set_out + pd.ch * cs;
    a.eps = p->eps;
    a.mu = p->mu;
    sh.mu = p->mu != nullptr;
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
        a.src_post_dev = inj->post_dev ? inj->post_dev + pd.ce : nullptr;
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
    a.sa_o = a.sa;
    a.sb_o = a.sb;
    a.sw_o = a.sw;
    a.comp_o = a.comp;
    if (fin) {
        a.fsrc = fin->add ? fin->src : 0.0;
        a.fin_add = fin->add ? 1 : 0;
        if (fin->E) {
            // the caller's arrays: x fastest, rows of nx+1, planes of cplane
            auto cstride = [&](int ax) -> long long {
                return ax == 0 ? 1 : (ax == 1 ? (long long)(d.nx + 1) : d.cplane);
            };
            a.Eout = static_cast<T*>(fin->E[pd.ce]);
            a.Hout = static_cast<T*>(fin->H[pd.ch - 3]);
            a.sw_o = cstride(pd.w);
            if (pd.w == 0) {
                a.sa_o = cstride(1);
                a.sb_o = cstride(2);
            } else {
                a.sa_o = 1;
                a.sb_o = cstride((pd.e == 0) ? pd.t : pd.e);
            }
            a.comp_o = d.ccomp;
        }
    }
}

// Weights of the 4-point difference with outer weight wo, for the samples at
// -3/2, -1/2, +1/2, +3/2: {-wo, -wi, wi, wo} with wi = 1 - 3 wo.
static void stencil4_weights(double wo, double w[4]) {
    const double wi = 1.0 - 3.0 * wo;
    w[0] = -wo;
    w[1] = -wi;
    w[2] = wi;
    w[3] = wo;
}

// Band of D^T D (the 4-point difference D with weights w, folded onto the wall
// images) for a line of n cells: rows 1..3 (lo) and n-3..n-1 (hi), entries
// {A_jj, A_j,j-1, A_j,j-2, A_j,j-3}, 0 where a column is not an unknown.
static void band4_rows(int n, const double w[4], double lo[3][4], double hi[3][4]) {
    auto coef = [n, w](int h, int p) {   // D[h][p]: H sample h, E unknown p
        double c = 0.0;
        for (int t = 0; t < 4; ++t) {
            int q = h - 1 + t;
            double sg = 1.0;
            if (q < 0) { q = -q; sg = -1.0; }
            else if (q > n) { q = 2 * n - q; sg = -1.0; }
            if (q == p && q >= 1 && q <= n - 1) c += sg * w[t];
        }
        return c;
    };
    auto A = [&](int j, int k) {
        double s = 0.0;
        for (int h = std::max(0, std::max(j, k) - 2); h <= std::min(n - 1, std::min(j, k) + 1); ++h)
            s += coef(h, j) * coef(h, k);
        return s;
    };
    for (int r = 0; r < 3; ++r)
        for (int t = 0; t < 4; ++t) {
            const int jl = r + 1, jh = n - 3 + r;
            lo[r][t] = (jl <= n - 1 && jl - t >= 1) ? A(jl, jl - t) : 0.0;
            hi[r][t] = (jh >= 1 && jh - t >= 1) ? A(jh, jh - t) : 0.0;
        }
}

// A fourth-order pass (pair k of operator op, fundamental form, in place).
template <typename T, typename S>
static fdtd_status launch_pass4(fdtd_plan_s* p, int op, int k, double theta, T* set, const Inject* inj,
                                const Fin* fin) {
    Pass4Args<T, S> a4;
    PassShape sh;
    build_pass<T, S>(p, op, k, theta, FUND, set, set, inj, a4.p, sh, fin);
    a4.nlines = (long long)a4.p.na * a4.p.nb;
    // the kernel's work area must fit the pass's region
    if ((size_t)work4_words(a4.p.n_w, a4.nlines, seg4<S>()) > p->scr4_region) return FDTD_EINVAL;
    a4.scr = reinterpret_cast<S*>(p->scr4) + (size_t)k * p->scr4_region;
    double w[4];
    stencil4_weights(p->stencil_wo, w);
    band4_rows(a4.p.n_w, w, a4.blo, a4.bhi);
    a4.wi = w[2];
    a4.wo = w[3];
    // interior rows: A_jj = sum w_t^2, A_j,j-1 = sum w_t w_t+1, ...
    for (int t = 0; t < 4; ++t) {
        double sum = 0.0;
        for (int u = 0; u + t < 4; ++u) sum += w[u] * w[u + t];
        a4.bin[t] = sum;
    }
    const Dims& d = p->dims;
    T* const Es = a4.p.Eout;   // the pair in the state (in place: Ein == Eout)
    T* const Hs = a4.p.Hout;
    const dim3 tb(256);
    const dim3 to_t = transpose_grid<T>(d.ny + 1, d.nx + 1, d.nz + 1);     // rows y, columns x
    const dim3 from_t = transpose_grid<T>(d.nx + 1, d.ny + 1, d.nz + 1);   // rows x, columns y
    if (sh.w == 0) {
        // x lines: on the transposed copy (x the slow axis of each plane), so
        // that lanes (consecutive y) read consecutive words
        if (!p->tr4) return FDTD_EINVAL;
        T* const Et = static_cast<T*>(p->tr4);
        T* const Ht = Et + (size_t)p->tr4_plane * (d.nz + 1);
        hipLaunchKernelGGL((transpose_planes_kernel<T>), to_t, tb, 0, p->stream, Es, d.plane,
                           (long long)d.px, Et, p->tr4_plane, p->tr4_pitch, d.ny + 1, d.nx + 1);
        hipLaunchKernelGGL((transpose_planes_kernel<T>), to_t, tb, 0, p->stream, Hs, d.plane,
                           (long long)d.px, Ht, p->tr4_plane, p->tr4_pitch, d.ny + 1, d.nx + 1);
        a4.p.Ein = a4.p.Eout = Et;
        a4.p.Hin = a4.p.Hout = Ht;
        a4.p.sa = 1;
        a4.p.sb = p->tr4_plane;
        a4.p.sw = p->tr4_pitch;
        if (p->mat) a4.p.mat = static_cast<const unsigned char*>(p->tr4_med);
        else a4.p.eps = static_cast<const float*>(p->tr4_med);
    }
    const dim3 grid((unsigned)((a4.nlines + 127) / 128)), block(128);
    if (fin) hipLaunchKernelGGL((pass4_kernel<T, S, true>), grid, block, 0, p->stream, a4);
    else hipLaunchKernelGGL((pass4_kernel<T, S, false>), grid, block, 0, p->stream, a4);
    if (sh.w == 0) {
        hipLaunchKernelGGL((transpose_planes_kernel<T>), from_t, tb, 0, p->stream, a4.p.Eout, p->tr4_plane,
                           p->tr4_pitch, Es, d.plane, (long long)d.px, d.nx + 1, d.ny + 1);
        hipLaunchKernelGGL((transpose_planes_kernel<T>), from_t, tb, 0, p->stream, a4.p.Hout, p->tr4_plane,
                           p->tr4_pitch, Hs, d.plane, (long long)d.px, d.nx + 1, d.ny + 1);
    }
    return FDTD_OK;
}

template <typename T, typename S>
static fdtd_status launch_pass(fdtd_plan_s* p, int op, int k, double theta, int mode, T* set_in, T* set_out,
                               const Inject* inj, bool timed, const Fin* fin = nullptr) {
    PassArgs<T, S> a;
    PassShape sh;
    build_pass<T, S>(p, op, k, theta, mode, set_in, set_out, inj, a, sh, fin);
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
    const bool fused = fin != nullptr;
    int r;
    if (p->order == 4) {
        // fourth-order differences: fundamental forms, in place (set_in == set_out)
        if (mode != FUND || set_in != set_out) return FDTD_EUNSUPPORTED;
        fdtd_status st = launch_pass4<T, S>(p, op, k, theta, set_out, inj, fin);
        if (st != FDTD_OK) return st;
        r = DISPATCH_OK;
    } else if (sh.mu) {
        r = sh.w == 0 ? dispatch_x_mu<T, S>(kmode, cf.M, sh.full, fused, sh.grid, sh.block, p->stream, a)
                      : dispatch_yz_mu<T, S>(kmode, cf.M, cf.TX, cf.NT, sh.full, fused, sh.grid, sh.block, sh.lds,
                                             p->stream, a);
    } else if (sh.w == 0) {
        r = dispatch_x<T, S>(kmode, cf.M, sh.full, sh.mat, fused, sh.grid, sh.block, p->stream, a);
    } else {
        const size_t lds = kmode == FUND_REF ? sh.lds / 9 * 13 : sh.lds;   // refined: second exchange areas
        r = dispatch_yz<T, S>(kmode, cf.M, cf.TX, cf.NT, sh.full, sh.mat, fused, sh.grid, sh.block, lds, p->stream, a);
    }
    if (r != DISPATCH_OK) return FDTD_EUNSUPPORTED;
    HIPCHK(hipGetLastError());
    if (timed) HIPCHK(hipEventRecord(e1, p->stream));
    return FDTD_OK;
}

template <typename T, typename S>
static fdtd_status substep(fdtd_plan_s* p, int op, double theta, int mode, int& cur, const Inject* inj,
                           bool timed, const Fin* fin = nullptr) {
    const int out = (mode == CONV_ADI) ? 1 - cur : cur;
    for (int k = 0; k < 3; ++k) {
        fdtd_status st =
            launch_pass<T, S>(p, op, k, theta, mode, set_ptr<T>(p, cur), set_ptr<T>(p, out), inj, timed, fin);
        if (st != FDTD_OK) return st;
    }
    cur = out;
    return FDTD_OK;
}

}  // namespace fdtd
