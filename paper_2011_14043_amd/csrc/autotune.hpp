// autotune.hpp -- kernel configurations of the line passes and the autotuner (with its
// text cache)
//
// Part of the single translation unit of libfdtd.so: included by fdtd.hip
// after the kernel headers and the headers before it in fdtd.hip.
#pragma once

namespace fdtd {

// ---------------------------------------------------------------------------
// kernel configurations and the autotuner
// ---------------------------------------------------------------------------
static bool cfg_valid(const fdtd_plan_s* p, int axis, const KCfg& c) {
    const int n = axis_cells(p->dims, axis);
    if (c.remap != 0 && c.remap != 1) return false;
    if (p->refine && (axis == 0 ? c.M != 8 : c.M > 16)) return false;   // refined solves built
    if (axis == 0) {
        if (c.M != 8 && c.M != 16) return false;
        if (p->mu && c.M != 8) return false;
        if (c.wpb < 1 || c.wpb > 4) return false;
        return next_pow2((n + c.M - 1) / c.M) <= 64;
    }
    // FP64 conventional ADI (two extra arrays per pass) exceeds the register
    // budget of the 1024-thread FP64 variant
    if (p->d.dtype == FDTD_F64 && p->d.scheme == FDTD_ADI && p->d.form == FDTD_CONVENTIONAL && c.NT == 1024)
        return false;
    bool inst = false;
    if (p->mu) {
        if (p->d.dtype == FDTD_F32) {
            for (const auto& v : kYzMuF32) inst = inst || (v[0] == c.M && v[1] == c.TX && v[2] == c.NT);
        } else {
            for (const auto& v : kYzMuF64) inst = inst || (v[0] == c.M && v[1] == c.TX && v[2] == c.NT);
        }
    } else if (p->d.dtype == FDTD_F32) {
        for (const auto& v : kYzF32) inst = inst || (v[0] == c.M && v[1] == c.TX && v[2] == c.NT);
    } else {
        for (const auto& v : kYzF64) inst = inst || (v[0] == c.M && v[1] == c.TX && v[2] == c.NT);
    }
    if (!inst) return false;
    const int P = next_pow2((n + c.M - 1) / c.M);
    return P <= 64 && c.TX * P <= c.NT;
}

// Candidates: y/z lines only in the XCD-aware order (the plain order reads
// the z pass's material lines once per XCD; the time difference is noise,
// the traffic is not); x lines in both orders.
static std::vector<KCfg> cfg_candidates(const fdtd_plan_s* p, int axis) {
    std::vector<KCfg> out;
    for (int remap = 1; remap >= (axis == 0 ? 0 : 1); --remap) {
        if (axis == 0) {
            for (int M : {8, 16})
                for (int wpb : {4, 2, 1}) {
                    KCfg c{M, 0, 0, wpb, remap};
                    if (cfg_valid(p, axis, c)) out.push_back(c);
                }
        } else if (p->mu && p->d.dtype == FDTD_F32) {
            for (const auto& v : kYzMuF32) {
                KCfg c{v[0], v[1], v[2], 0, remap};
                if (cfg_valid(p, axis, c)) out.push_back(c);
            }
        } else if (p->mu) {
            for (const auto& v : kYzMuF64) {
                KCfg c{v[0], v[1], v[2], 0, remap};
                if (cfg_valid(p, axis, c)) out.push_back(c);
            }
        } else if (p->d.dtype == FDTD_F32) {
            for (const auto& v : kYzF32) {
                KCfg c{v[0], v[1], v[2], 0, remap};
                if (cfg_valid(p, axis, c)) out.push_back(c);
            }
        } else {
            for (const auto& v : kYzF64) {
                KCfg c{v[0], v[1], v[2], 0, remap};
                if (cfg_valid(p, axis, c)) out.push_back(c);
            }
        }
    }
    return out;
}

// Untuned default: the first valid entry of the preference order.
static void default_cfg(fdtd_plan_s* p) {
    for (int axis = 0; axis < 3; ++axis) {
        std::vector<KCfg> pref;
        if (axis == 0) {
            pref = {{8, 0, 0, 4, 1}, {16, 0, 0, 4, 1}};
        } else if (p->mu) {
            pref = {{16, 16, 512, 0, 1}, {8, 16, 512, 0, 1}, {8, 8, 512, 0, 1}};
        } else if (p->d.dtype == FDTD_F32) {
            pref = {{16, 16, 512, 0, 1}, {16, 32, 1024, 0, 1}, {32, 16, 512, 0, 1}, {8, 16, 1024, 0, 1},
                    {8, 32, 512, 0, 1}};
        } else {
            pref = {{16, 16, 512, 0, 1}, {8, 8, 512, 0, 1}};
        }
        for (const KCfg& c : pref)
            if (cfg_valid(p, axis, c)) { p->cfg[axis] = c; break; }
    }
}

template <typename T, typename S>
static fdtd_status autotune_impl(fdtd_plan_s* p, int reps, double* best_ms) {
    const bool adi = p->d.scheme == FDTD_ADI, conv = p->d.form == FDTD_CONVENTIONAL;
    const int mode = conv ? (adi ? CONV_ADI : CONV_LOD) : FUND;
    const double theta = 0.5 * p->d.dt;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    fdtd_status st = FDTD_OK;
    for (int axis = 0; axis < 3 && st == FDTD_OK; ++axis) {
        int k = 0;
        while (kPairs[0][k].w != axis) ++k;
        const std::vector<KCfg> cand = cfg_candidates(p, axis);
        KCfg best = p->cfg[axis];
        float tbest = 1e30f;
        // two rounds over the candidates; each keeps its best time (clock
        // and neighbour noise only ever add time)
        for (int round = 0; round < 2 * (int)cand.size() && st == FDTD_OK; ++round) {
            const KCfg& c = cand[round % cand.size()];
            p->cfg[axis] = c;
            T* s0 = set_ptr<T>(p, 0);
            T* s1 = set_ptr<T>(p, conv && adi ? 1 : 0);
            st = launch_pass<T, S>(p, 0, k, theta, mode, s0, s1, nullptr, false);
            if (st != FDTD_OK) break;
            if (hipEventRecord(e0, p->stream) != hipSuccess) { st = FDTD_EDEVICE; break; }
            for (int r = 0; r < reps && st == FDTD_OK; ++r)
                st = launch_pass<T, S>(p, 0, k, theta, mode, s0, s1, nullptr, false);
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
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == FDTD_OK) p->tuned = 1;
    return st;
}

// Text cache of tuned configurations: one line per key
//   {"key": "<nx>,<ny>,<nz>,<dtype>,<scheme>,<form>,<refine>", "cfg": [[M,TX,NT,wpb,remap],[...],[...]]}
static std::string tune_key(const fdtd_plan_s* p) {
    char b[160];
    std::snprintf(b, sizeof(b), "%d,%d,%d,%d,%d,%d,%d%s", p->d.nx, p->d.ny, p->d.nz, p->d.dtype, p->d.scheme,
                  p->d.form, p->refine, p->mu ? ",mu" : "");
    return b;
}

static bool tune_cache_lookup(fdtd_plan_s* p, const char* path) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    const std::string key = tune_key(p);
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        char k[160];
        KCfg c[3];
        if (std::sscanf(line, " {\"key\": \"%159[^\"]\", \"cfg\": [[%d,%d,%d,%d,%d],[%d,%d,%d,%d,%d],[%d,%d,%d,%d,%d]]}", k,
                        &c[0].M, &c[0].TX, &c[0].NT, &c[0].wpb, &c[0].remap, &c[1].M, &c[1].TX, &c[1].NT, &c[1].wpb,
                        &c[1].remap, &c[2].M, &c[2].TX, &c[2].NT, &c[2].wpb, &c[2].remap) != 16)
            continue;
        if (key != k) continue;
        if (cfg_valid(p, 0, c[0]) && cfg_valid(p, 1, c[1]) && cfg_valid(p, 2, c[2])) {
            for (int a = 0; a < 3; ++a) p->cfg[a] = c[a];
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

static void tune_cache_store(const fdtd_plan_s* p, const char* path) {
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    const KCfg* c = p->cfg;
    std::fprintf(f, "{\"key\": \"%s\", \"cfg\": [[%d,%d,%d,%d,%d],[%d,%d,%d,%d,%d],[%d,%d,%d,%d,%d]]}\n",
                 tune_key(p).c_str(), c[0].M, c[0].TX, c[0].NT, c[0].wpb, c[0].remap, c[1].M, c[1].TX, c[1].NT,
                 c[1].wpb, c[1].remap, c[2].M, c[2].TX, c[2].NT, c[2].wpb, c[2].remap);
    std::fclose(f);
}

}  // namespace fdtd
