/*
 * fdtd_abi_check.c -- the library used from plain C through include/fdtd.h
 * and the HIP runtime's C API only (no Python, no torch).
 *
 * A 24 x 20 x 22 PEC box, random-box eps_r, deterministic pseudo-random
 * fields, CFL 6, FP64: 20 steps of fundamental ADI (Sec. II-A, (fasterADI))
 * with the energy trace, and the same 20 steps of conventional ADI
 * ((clsADI)).  Checks that the trace is conserved (the fundamental ADI
 * invariant) and that the two forms give the same fields (fdtd_diff_norm).
 * Prints one JSON line; exit status 0 when both hold, 1 otherwise, 2 on an
 * API error.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "fdtd.h"

#define NX 24
#define NY 20
#define NZ 22
#define STEPS 20

static unsigned long long lcg = 88172645463325252ull;
static double unif(void) {   /* xorshift64, in [-1, 1) */
    lcg ^= lcg << 13;
    lcg ^= lcg >> 7;
    lcg ^= lcg << 17;
    return (double)(lcg >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static int check(fdtd_status s, const char* what) {
    if (s != FDTD_OK) {
        fprintf(stderr, "%s: %s\n", what, fdtd_strerror(s));
        return 1;
    }
    return 0;
}

int main(void) {
    const size_t nn = (size_t)(NX + 1) * (NY + 1) * (NZ + 1);
    const size_t ncell = (size_t)NX * NY * NZ;
    const double h = 1e-3, c0 = 299792458.0;
    const double dt = 6.0 / (c0 * sqrt(3.0 / (h * h)));
    float* eps_h = (float*)malloc(sizeof(float) * ncell);
    double* f_h = (double*)malloc(sizeof(double) * nn);
    double* energy = (double*)malloc(sizeof(double) * (STEPS + 1));
    void *f[2][6], *eps_d = NULL;
    fdtd_plan_t plan[2] = {NULL, NULL};
    int rc = 2;
    if (!eps_h || !f_h || !energy) return 2;
    for (size_t c = 0; c < ncell; ++c) {   /* two slabs of dielectric */
        const size_t k = c / ((size_t)NX * NY);
        eps_h[c] = k < NZ / 3 ? 4.0f : (k < 2 * NZ / 3 ? 1.0f : 9.5f);
    }
    if (hipMalloc(&eps_d, sizeof(float) * ncell) != hipSuccess) return 2;
    if (hipMemcpy(eps_d, eps_h, sizeof(float) * ncell, hipMemcpyHostToDevice) != hipSuccess) return 2;
    for (int s = 0; s < 2; ++s)
        for (int c = 0; c < 6; ++c) {
            if (hipMalloc(&f[s][c], sizeof(double) * nn) != hipSuccess) return 2;
            for (size_t i = 0; i < nn; ++i) f_h[i] = unif() * (c < 3 ? 1.0 : 1.0 / 377.0);
            if (hipMemcpy(f[s][c], f_h, sizeof(double) * nn, hipMemcpyHostToDevice) != hipSuccess) return 2;
        }
    /* the conventional run starts from the same fields as the fundamental one */
    for (int c = 0; c < 6; ++c)
        if (hipMemcpy(f[1][c], f[0][c], sizeof(double) * nn, hipMemcpyDeviceToDevice) != hipSuccess) return 2;
    for (int s = 0; s < 2; ++s) {
        fdtd_desc d;
        d.nx = NX; d.ny = NY; d.nz = NZ;
        d.dt = dt; d.dx = h; d.dy = h; d.dz = h;
        d.scheme = FDTD_ADI;
        d.form = s == 0 ? FDTD_FUNDAMENTAL : FDTD_CONVENTIONAL;
        d.dtype = FDTD_F64;
        d.eps_r = (const float*)eps_d;
        d.mu_r = NULL;
        d.boundary = 0;
        if (check(fdtd_plan(&d, NULL, &plan[s]), "fdtd_plan")) goto done;
    }
    if (check(fdtd_run(plan[0], &f[0][0], &f[0][3], STEPS, NULL, energy, 1), "fdtd_run (fundamental)")) goto done;
    if (check(fdtd_run(plan[1], &f[1][0], &f[1][3], STEPS, NULL, NULL, 1), "fdtd_run (conventional)")) goto done;
    if (hipDeviceSynchronize() != hipSuccess) goto done;
    {
        double dist[2];
        double drift = 0.0;
        if (check(fdtd_diff_norm(plan[0], &f[0][0], &f[0][3], &f[1][0], &f[1][3], dist), "fdtd_diff_norm")) goto done;
        for (int m = 1; m <= STEPS; ++m) drift = fmax(drift, fabs(energy[m] / energy[0] - 1.0));
        const double rel = sqrt(dist[0] / dist[1]);
        printf("{\"energy_drift\": %.3e, \"fundamental_vs_conventional\": %.3e}\n", drift, rel);
        rc = (drift < 1e-12 && rel < 1e-12) ? 0 : 1;
    }
done:
    for (int s = 0; s < 2; ++s) {
        if (plan[s]) fdtd_destroy(plan[s]);
        for (int c = 0; c < 6; ++c) (void)hipFree(f[s][c]);
    }
    (void)hipFree(eps_d);
    free(eps_h);
    free(f_h);
    free(energy);
    return rc;
}
