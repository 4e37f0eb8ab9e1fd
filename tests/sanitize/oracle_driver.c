/* Drives every entry point of the FP64 oracle on small systems, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer: the sanitizers report
 * any out-of-bounds access, leak or undefined operation, and the driver checks
 * a few results the oracle's own tests pin (the cell list finds the all-pairs
 * set, momentum is conserved without propulsion and friction, binning counts
 * every particle).  Exit status 0 when every check holds. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/oracle.h"

static int fails = 0;
#define CHECK(c, msg) do { if (!(c)) { fprintf(stderr, "FAIL: %s\n", msg); ++fails; } } while (0)

static uint64_t lcg = 0x9E3779B97F4A7C15ull;
static double urand(void) {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

static void run_case(int64_t n_agents, double L, double r_c, double bond_l, double f_sp,
                     double gamma_s) {
    oracle_params p;
    memset(&p, 0, sizeof p);
    p.n_agents = n_agents; p.L = L; p.r_c = r_c; p.A = 25.0; p.gamma = 4.5; p.kT = 1.0;
    p.kappa = 1000.0; p.bond_l = bond_l; p.f_sp = f_sp; p.gamma_s = gamma_s; p.mass = 1.0;
    p.dt = 0.005; p.seed = 77; p.w_exp = 2.0;
    const int64_t n = 2 * n_agents;
    double* x = malloc(sizeof(double) * 2 * n);
    double* v = malloc(sizeof(double) * 2 * n);
    double* F = malloc(sizeof(double) * 2 * n);
    double* F2 = malloc(sizeof(double) * 2 * n);
    double* parts = malloc(sizeof(double) * 6 * n);
    double* scale = malloc(sizeof(double) * n);
    for (int64_t k = 0; k < n_agents; ++k) {
        const double cx = L * urand(), cy = L * urand(), th = 6.283185307179586 * urand();
        x[4 * k + 0] = oracle_wrap(cx + 0.5 * bond_l * cos(th), L);
        x[4 * k + 1] = oracle_wrap(cy + 0.5 * bond_l * sin(th), L);
        x[4 * k + 2] = oracle_wrap(cx - 0.5 * bond_l * cos(th), L);
        x[4 * k + 3] = oracle_wrap(cy - 0.5 * bond_l * sin(th), L);
    }
    for (int64_t i = 0; i < 2 * n; ++i) v[i] = urand() - 0.5;

    /* pair sets: the cell list equals the all-pairs search; a short buffer
     * reports the size it needs */
    int64_t need_b = 0, need_c = 0, need_s = 0, small[2];
    CHECK(oracle_pairs_brute(&p, x, NULL, 0, &need_b) == (need_b ? -1 : 0), "pairs_brute size query");
    CHECK(oracle_pairs_cells(&p, x, small, 1, &need_s) == (need_s <= 1 ? need_s : -1), "pairs_cells short buffer");
    int64_t* pb = malloc(sizeof(int64_t) * 2 * (need_b + 1));
    int64_t* pc = malloc(sizeof(int64_t) * 2 * (need_b + 1));
    const int64_t nb = oracle_pairs_brute(&p, x, pb, need_b, NULL);
    const int64_t ncl = oracle_pairs_cells(&p, x, pc, need_b, &need_c);
    CHECK(nb == need_b && ncl == nb && need_c == nb, "pair counts");
    CHECK(nb < 1 || memcmp(pb, pc, sizeof(int64_t) * 2 * nb) == 0, "pair sets");

    /* forces by both routes, bitwise; parts, scales and a subset */
    CHECK(oracle_forces(&p, x, v, 3, F, 0) == 0, "forces brute");
    CHECK(oracle_forces(&p, x, v, 3, F2, 1) == 0, "forces cells");
    CHECK(memcmp(F, F2, sizeof(double) * 2 * n) == 0, "forces bitwise");
    CHECK(oracle_force_parts(&p, x, v, 3, parts, scale, 1) == 0, "force parts");
    int64_t idx[3] = {0, n - 1, n / 2};
    double Fs[6];
    CHECK(oracle_forces_subset(&p, x, v, 3, idx, 3, Fs) == 0, "forces subset");
    for (int k = 0; k < 3; ++k)
        CHECK(Fs[2 * k] == F[2 * idx[k]] && Fs[2 * k + 1] == F[2 * idx[k] + 1], "subset equals full");

    /* stepping with reductions */
    double pk[3 * 4], mk[3];
    int64_t step = 3;
    oracle_momentum_ke(&p, v, mk);
    CHECK(oracle_step(&p, x, v, F, &step, 20, 1, 5, pk) == 0 && step == 23, "step");
    if (f_sp == 0.0 && gamma_s == 0.0)
        CHECK(fabs(pk[9] - mk[0]) <= 1e-12 * (1.0 + fabs(mk[0])) &&
              fabs(pk[10] - mk[1]) <= 1e-12 * (1.0 + fabs(mk[1])), "momentum conserved");

    /* binning and the filtered field */
    float* xf = malloc(sizeof(float) * 2 * n);
    float* vf = malloc(sizeof(float) * 2 * n);
    for (int64_t i = 0; i < 2 * n; ++i) {
        xf[i] = (float)x[i];
        if (xf[i] >= (float)L) xf[i] = 0.0f;
        vf[i] = (float)v[i];
    }
    const int64_t nc = oracle_n_cells_side(&p);
    int32_t* cs = malloc(sizeof(int32_t) * (nc * nc + 1));
    int32_t* ids = malloc(sizeof(int32_t) * n);
    CHECK(oracle_bin(&p, xf, cs, ids) >= 0 && cs[nc * nc] == n, "binning counts every particle");
    for (int mode = 0; mode < 2; ++mode)
        for (int k = 0; k < 2; ++k) {
            const int M = 7;
            double u[2 * 49];
            int32_t cnt[49];
            CHECK(oracle_bin_velocity(&p, xf, vf, M, k ? 2.5 * L / M : 0.0, mode, u, cnt) == 0, "bin_velocity");
            if (k == 0) {
                int64_t tot = 0;
                for (int b = 0; b < 49; ++b) tot += cnt[b];
                CHECK(tot == (mode ? n_agents : n), "plain bins count every contributor");
            }
        }
    CHECK(oracle_bin_velocity(&p, xf, vf, 0, 0.0, 0, NULL, NULL) != 0, "bin_velocity rejects M = 0");

    /* generators */
    uint32_t w4[4], w2[2];
    const uint32_t c4[4] = {1, 2, 3, 4}, k2[2] = {5, 6}, c2[2] = {7, 8};
    oracle_philox4x32_10(c4, k2, w4);
    oracle_philox2x32_10(c2, 9u, w2);
    oracle_pair_words(&p, 3, 1, 12345, w4);
    const double a = oracle_pair_alpha(&p, 1, 3, 12345);
    CHECK(isfinite(a) && a == oracle_pair_alpha(&p, 3, 1, 12345), "alpha symmetric");

    free(x); free(v); free(F); free(F2); free(parts); free(scale); free(pb); free(pc);
    free(xf); free(vf); free(cs); free(ids);
}

int main(void) {
    run_case(60, 10.0, 1.0, 0.5, 1.0, 0.5);
    run_case(40, 8.0, 1.0, 0.5, 0.0, 0.0);    /* momentum conserved */
    run_case(1, 3.0, 1.0, 0.5, 1.0, 0.5);     /* one agent, the smallest grid */
    run_case(50, 12.0, 0.5, 1.0, 1.0, 0.1);   /* bond longer than the cutoff */
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("oracle driver: all checks passed\n");
    return 0;
}
