// adjoint_grad.hpp -- adjoint gradient of the probe objective with checkpoints and
// segment recomputation (fundamental ADI)
//
// Part of the single translation unit of libfdtd.so: included by fdtd.hip
// after the kernel headers and the headers before it in fdtd.hip.
#pragma once

namespace fdtd {

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
    // records of state set 0; with J, the probe energy of the B sub-step whose
    // A-side record is pold
    auto record = [&](T* dst, double* pdst, const double* pold = nullptr, double h = 0.0,
                      double* J = nullptr) -> fdtd_status {
        hipLaunchKernelGGL((record_kernel<T>), dim3(dst ? rblocks : 1), dim3(256), 0, p->stream, fptrs(st0), dm, b,
                           dst, probe_off, pdst, pold, h, d.dt, J);
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
    {
        const fdtd_status st = load_state<T, S>(p, caller, 0.25 * d.dt);
        if (st != FDTD_OK) return st;
    }
    HIPCHK(hipMemsetAsync(Jd, 0, 256, p->stream));
    for (int n = 0; n < nsteps; ++n) {
        if (want && n % K == 0) HIPCHK(hipMemcpyAsync(ckpt(n / K), st0, ssz, hipMemcpyDeviceToDevice, p->stream));
        const long long glob = p->step + n;
        double gA, gB;
        GCHK(fwd_sub(0, glob, 0.25, &gA));
        GCHK(record(nullptr, prb));
        GCHK(fwd_sub(1, glob, 0.75, &gB));
        GCHK(record(nullptr, prb + 3, prb, src_at_probe ? 0.5 * gB : 0.0, Jd));   // J += dt |V|^2
    }
    if (want) {
        HIPCHK(hipMemsetAsync(adj, 0, ssz, p->stream));
        HIPCHK(hipMemsetAsync(grad_out, 0, sizeof(double) * nb, p->stream));
        const FieldPtrs<T> lam = fptrs(adj);
        const double scale = -0.5 * kEps0;
        // the gradient terms m1, m2 (< 0: none) of the current adjoint state, with
        // their sub-steps' source terms g1, g2; with mseed >= 0 also the seed of
        // B sub-step mseed (records mseed and mseed + 1, source term gseed)
        auto acc = [&](int m1, double g1, int m2, double g2, int mseed = -1, double gseed = 0.0) -> fdtd_status {
            hipLaunchKernelGGL((grad_acc_kernel<T>), dim3(rblocks), dim3(256), 0, p->stream, lam, dm, b, rec, m1,
                               0.5 * g1, m2, 0.5 * g2, src_idx, scale, grad_out, mseed >= 0 ? seed : nullptr,
                               prb + 3 * std::max(mseed, 0), prb + 3 * (std::max(mseed, 0) + 1),
                               src_at_probe ? 0.5 * gseed : 0.0, p->eps, probe_off, kEps0, d.dt);
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
            // reverse sub-steps: before the B sub-step of step q, the terms of the
            // state between steps q + 1 and q (the A term of step q + 1, the B
            // term of step q) and the seed of step q; between its sub-steps the
            // B and A terms; after step 0 of the segment its A term
            for (int q = L - 1; q >= 0; --q) {
                const int mB = 2 * q + 1, mA = 2 * q;
                const double gB = gs[mB], gA = gs[mA];
                GCHK(acc(q < L - 1 ? mA + 2 : -1, q < L - 1 ? gs[mA + 2] : 0.0, mB, gB, mB, gB));
                GCHK(adj_sub(1, &seed_inj));
                GCHK(acc(mB, gB, mA, gA));
                GCHK(adj_sub(0, nullptr));
            }
            if (L > 0) GCHK(acc(0, gs[0], -1, 0.0));
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

}  // namespace fdtd
