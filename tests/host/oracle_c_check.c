/*
 * The oracle's C code (oracle/sweep.c, oracle/cpu_sweep.c) exercised under the
 * address and undefined-behaviour sanitizers by tests/test_host_schedule.py.
 * The values are pinned elsewhere (against NumPy and dense solves in the
 * Python tests); here: the block sweep on random block systems with upwind
 * cycles satisfies its own equations, and the compiled hex sweep gives the
 * same bits for 1, 2 and 4 threads.  Prints "ok" and exits 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_sweep(int64_t E, int k, int F, const double* D, const int64_t* nbr, const double* Cpl,
                 const double* rhs, double* psi);
int cpu_sweep_hex(int nx, int ny, int nz, const double* h, const double* sigma_t, const double* sigma_s,
                  const double* q, const double* phi, int M, const double* omega, const double* w,
                  double* psi, double* phi_out, int threads);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static double urand(void) {   /* xorshift64*, uniform in [0, 1) */
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (double)((state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static int check_block_sweep(int64_t E, int k, int F) {
    double* D = malloc(sizeof(double) * E * k * k);
    double* C = malloc(sizeof(double) * E * F * k * k);
    int64_t* nbr = malloc(sizeof(int64_t) * E * F);
    double* rhs = malloc(sizeof(double) * E * k);
    double* psi = malloc(sizeof(double) * E * k);
    for (int64_t e = 0; e < E; ++e) {
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) D[(e * k + a) * k + b] = (a == b ? 4.0 + urand() : 0.5 * (urand() - 0.5));
        for (int f = 0; f < F; ++f) {
            const double r = urand();
            nbr[e * F + f] = r < 0.3 ? -1 : (int64_t)(urand() * (double)E);
            if (nbr[e * F + f] == e) nbr[e * F + f] = -1;
            for (int a = 0; a < k * k; ++a) C[(e * F + f) * k * k + a] = 0.2 * (urand() - 0.5);
        }
        for (int a = 0; a < k; ++a) rhs[e * k + a] = urand() - 0.5;
    }
    /* a planted three-element cycle */
    nbr[0 * F + 0] = 1; nbr[1 * F + 0] = 2; nbr[2 * F + 0] = 0;
    const int cyc = oracle_sweep(E, k, F, D, nbr, C, rhs, psi);
    double worst = 0.0;
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < k; ++a) {
            double r = -rhs[e * k + a];
            for (int b = 0; b < k; ++b) r += D[(e * k + a) * k + b] * psi[e * k + b];
            for (int f = 0; f < F; ++f) {
                const int64_t u = nbr[e * F + f];
                if (u < 0) continue;
                for (int b = 0; b < k; ++b) r += C[((e * F + f) * k + a) * k + b] * psi[u * k + b];
            }
            if (fabs(r) > worst) worst = fabs(r);
        }
    free(D); free(C); free(nbr); free(rhs); free(psi);
    if (cyc < 1 || !(worst <= 1e-10)) {
        printf("FAIL block sweep: cycles %d, residual %.3e\n", cyc, worst);
        return 1;
    }
    return 0;
}

static int check_hex_sweep(void) {
    const int nx = 5, ny = 4, nz = 6, M = 6;
    const int64_t E = (int64_t)nx * ny * nz, N = 8 * E;
    const double h[3] = {0.2, 0.25, 1.0 / 6.0};
    double *st = malloc(sizeof(double) * E), *ss = malloc(sizeof(double) * E), *q = malloc(sizeof(double) * E);
    double* phi = malloc(sizeof(double) * N);
    double om[3 * 6], w[6];
    for (int64_t e = 0; e < E; ++e) { st[e] = 0.5 + 2.0 * urand(); ss[e] = 0.5 * st[e]; q[e] = urand(); }
    for (int64_t i = 0; i < N; ++i) phi[i] = urand();
    for (int m = 0; m < M; ++m) {
        double v[3] = {urand() - 0.5, urand() - 0.5, urand() - 0.5};
        if (m == 4) v[1] = 0.0;           /* a direction along a face: no flux through it */
        const double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        for (int d = 0; d < 3; ++d) om[3 * m + d] = v[d] / n;
        w[m] = 4.0 * M_PI / M;
    }
    double* ref = malloc(sizeof(double) * M * N);
    double* out = malloc(sizeof(double) * M * N);
    double *pr = malloc(sizeof(double) * N), *po = malloc(sizeof(double) * N);
    int bad = cpu_sweep_hex(nx, ny, nz, h, st, ss, q, phi, M, om, w, ref, pr, 1) != 0;
    for (int64_t i = 0; i < M * N; ++i) if (!isfinite(ref[i])) bad = 1;
    for (int th = 2; th <= 4 && !bad; th *= 2) {
        bad |= cpu_sweep_hex(nx, ny, nz, h, st, ss, q, phi, M, om, w, out, po, th) != 0;
        bad |= memcmp(ref, out, sizeof(double) * M * N) != 0 || memcmp(pr, po, sizeof(double) * N) != 0;
    }
    free(st); free(ss); free(q); free(phi); free(ref); free(out); free(pr); free(po);
    if (bad) { printf("FAIL hex sweep: thread counts differ or non-finite values\n"); return 1; }
    return 0;
}

int main(void) {
    if (check_block_sweep(400, 4, 4) || check_block_sweep(200, 8, 6) || check_block_sweep(50, 3, 2)) return 1;
    if (check_hex_sweep()) return 1;
    printf("ok\n");
    return 0;
}
