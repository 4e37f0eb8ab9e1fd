/*
 * oracle.c -- plain FP64 CPU reference for the self-propelled soft-core
 * dumbbell DPD model of Hinz, Panchenko, Kim & Fried (arXiv:1310.0998).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  It shares no
 * code with the HIP engine.  Build with -ffp-contract=off so that every
 * expression is evaluated exactly as written.
 *
 * Readings of the paper taken here (where it is silent or ambiguous):
 *   - e^{ij} = (r^i - r^j)/r as in the formula of Sec. 2.1 (so a positive A
 *     pushes i away from j), not the "from i to j" of the prose;
 *   - alpha^{ij} is Gaussian N(0,1) by default (uniform of unit variance as an
 *     option), symmetric in (i, j) and fresh every step;
 *   - the generator is Philox (Salmon et al., SC'11) keyed on
 *     (min id, max id, step, seed);
 *   - the bonded partner feels no C/D/R pair force (Sec. 2.2);
 *   - f_sp is the total propulsion per agent, split f_sp/2 on each particle
 *     by default (head-only as an option) (Sec. 2.3);
 *   - the director is n = (r_head - r_tail)/|...|, head = particle 2k;
 *   - velocity-dependent forces at step n+1 use the half-step velocity
 *     u = v_n + dt/(2m) F_n (standard velocity-Verlet, Sec. 5);
 *   - strict cutoff r < r_c; coincident particles (r = 0) do not interact.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------- */
/* Philox: a Feistel-like network whose S-box is a 32x32->64 multiply, with a
 * Weyl-sequence key schedule (Salmon, Moraes, Dror & Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11).                                       */

static void mul_hi_lo(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
    uint64_t prod = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(prod >> 32);
    *lo = (uint32_t)(prod & 0xffffffffu);
}

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;  /* round multipliers */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;  /* key increments    */
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint32_t hi0, lo0, hi1, lo1;
        mul_hi_lo(M0, x0, &hi0, &lo0);
        mul_hi_lo(M1, x2, &hi1, &lo1);
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void oracle_philox2x32_10(const uint32_t ctr[2], uint32_t key, uint32_t out[2]) {
    const uint32_t M = 0xD256D193u, W = 0x9E3779B9u;
    uint32_t x0 = ctr[0], x1 = ctr[1], k = key;
    for (int round = 0; round < 10; ++round) {
        uint32_t hi, lo;
        mul_hi_lo(M, x0, &hi, &lo);
        uint32_t y0 = hi ^ k ^ x1;
        uint32_t y1 = lo;
        x0 = y0; x1 = y1;
        k += W;
    }
    out[0] = x0; out[1] = x1;
}

void oracle_pair_words(const oracle_params* p, int64_t i, int64_t j, int64_t step,
                       uint32_t out[4]) {
    uint32_t a = (uint32_t)(i < j ? i : j);
    uint32_t b = (uint32_t)(i < j ? j : i);
    uint32_t s = (uint32_t)((uint64_t)step & 0xffffffffu);
    uint32_t seed_lo = (uint32_t)(p->seed & 0xffffffffu);
    uint32_t seed_hi = (uint32_t)(p->seed >> 32);
    if (p->rng_kind == 0) {
        uint32_t ctr[4] = {a, b, s, 0u};
        uint32_t key[2] = {seed_lo, seed_hi};
        oracle_philox4x32_10(ctr, key, out);
    } else {
        /* Two-word counter holds the pair; the step is folded into the key by an
         * odd multiplier, so for a fixed seed every step has its own key. */
        uint32_t ctr[2] = {a, b};
        uint32_t key = seed_lo ^ (seed_hi * 0x85EBCA6Bu) ^ (s * 0xC2B2AE35u);
        uint32_t w[2];
        oracle_philox2x32_10(ctr, key, w);
        out[0] = w[0]; out[1] = w[1]; out[2] = 0u; out[3] = 0u;
    }
}

/* 23 random bits -> (2n+1)/2^24, strictly inside (0, 1) and exact in FP32. */
static double unit_open(uint32_t w) {
    return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0);
}

double oracle_pair_alpha(const oracle_params* p, int64_t i, int64_t j, int64_t step) {
    uint32_t w[4];
    oracle_pair_words(p, i, j, step, w);
    double u0 = unit_open(w[0]);
    if (p->noise_kind == 1)
        return sqrt(3.0) * (2.0 * u0 - 1.0);
    double u1 = unit_open(w[1]);
    /* Box-Muller (cosine branch) */
    const double two_pi = 6.283185307179586476925286766559;
    return sqrt(-2.0 * log(u0)) * cos(two_pi * u1);
}

/* ------------------------------------------------------------------------- */
double oracle_minimg(double d, double L) {
    return d - L * rint(d / L);
}

double oracle_wrap(double y, double L) {
    double z = y - L * floor(y / L);
    if (z >= L) z -= L;
    if (z < 0.0) z += L;
    return z;
}

/* DPD pair force on i from j (Eqs. 2.2-2.4). */
int oracle_pair_force(const oracle_params* p, const double d[2], const double dv[2],
                      double alpha, double f[2], double* parts) {
    double r2 = d[0] * d[0] + d[1] * d[1];
    f[0] = 0.0; f[1] = 0.0;
    if (parts) for (int k = 0; k < 6; ++k) parts[k] = 0.0;
    if (!(r2 > 0.0) || !(r2 < p->r_c * p->r_c)) return 0;
    double r = sqrt(r2);
    double e0 = d[0] / r, e1 = d[1] / r;          /* unit vector (r_i - r_j)/r */
    double w = 1.0 - r / p->r_c;                  /* Eq. 2.4                    */
    double g = dv[0] * e0 + dv[1] * e1;           /* (v_i - v_j) . e           */
    double sigma = sqrt(2.0 * p->gamma * p->kT);
    double sC = p->A * w;                         /* conservative magnitude     */
    double sD, sR;                                /* dissipative, random        */
    if (p->w_exp == 2.0) {                        /* Eq. 2.3 as printed         */
        sD = -p->gamma * w * w * g;
        sR = sigma * w * alpha / sqrt(p->dt);
    } else {
        /* dissipative weight w^s, random weight w^(s/2): the first is the
           square of the second, as fluctuation-dissipation requires */
        sD = -p->gamma * pow(w, p->w_exp) * g;
        sR = sigma * pow(w, 0.5 * p->w_exp) * alpha / sqrt(p->dt);
    }
    double s = (sC + sD) + sR;
    f[0] = s * e0;
    f[1] = s * e1;
    if (parts) {
        parts[0] = sC * e0; parts[1] = sC * e1;
        parts[2] = sD * e0; parts[3] = sD * e1;
        parts[4] = sR * e0; parts[5] = sR * e1;
    }
    return 1;
}

/* ------------------------------------------------------------------------- */
/* Neighbour search.  The definition is brute force; the cell list reaches the
 * same set faster.  Either way each particle's partners come back sorted.    */

typedef struct cells_t {
    int64_t nc;        /* cells per side               */
    double inv_w;      /* nc / L                       */
    int64_t* start;    /* nc*nc + 1                    */
    int64_t* members;  /* particle indices, cell order */
} cells_t;

int64_t oracle_n_cells_side(const oracle_params* p) {
    if (!(p->L > 0.0) || !(p->r_c > 0.0)) return -1;
    return (int64_t)floor(p->L / p->r_c);
}

static int64_t cell_coord(double x, double inv_w, int64_t nc) {
    int64_t c = (int64_t)floor(x * inv_w);
    if (c > nc - 1) c = nc - 1;
    if (c < 0) c = 0;
    return c;
}

static int cells_build(const oracle_params* p, const double* x, cells_t* cl) {
    int64_t n = 2 * p->n_agents;
    cl->nc = oracle_n_cells_side(p);
    if (cl->nc < 3) return -1;
    cl->inv_w = (double)cl->nc / p->L;
    int64_t ncell = cl->nc * cl->nc;
    cl->start = (int64_t*)calloc((size_t)(ncell + 1), sizeof(int64_t));
    cl->members = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t* key = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t* fill = (int64_t*)calloc((size_t)ncell, sizeof(int64_t));
    if (!cl->start || !cl->members || !key || !fill) {
        free(cl->start); free(cl->members); free(key); free(fill);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t cx = cell_coord(x[2 * i], cl->inv_w, cl->nc);
        int64_t cy = cell_coord(x[2 * i + 1], cl->inv_w, cl->nc);
        key[i] = cy * cl->nc + cx;
        cl->start[key[i] + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) cl->start[c + 1] += cl->start[c];
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = key[i];
        cl->members[cl->start[c] + fill[c]] = i;
        fill[c] += 1;
    }
    free(key);
    free(fill);
    return 0;
}

static void cells_free(cells_t* cl) {
    free(cl->start);
    free(cl->members);
}

static int cmp_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

/* Is (i, j) an interacting pair?  Writes the minimum-image separation. */
static int pair_interacts(const oracle_params* p, const double* x, int64_t i, int64_t j,
                          double d[2]) {
    if (j == i || j == (i ^ 1)) return 0;
    d[0] = oracle_minimg(x[2 * i] - x[2 * j], p->L);
    d[1] = oracle_minimg(x[2 * i + 1] - x[2 * j + 1], p->L);
    double r2 = d[0] * d[0] + d[1] * d[1];
    return (r2 > 0.0) && (r2 < p->r_c * p->r_c);
}

typedef struct vec_t { int64_t* a; int64_t n, cap; } vec_t;

static int vec_push(vec_t* v, int64_t x) {
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 64;
        int64_t* na = (int64_t*)realloc(v->a, (size_t)nc * sizeof(int64_t));
        if (!na) return -1;
        v->a = na; v->cap = nc;
    }
    v->a[v->n++] = x;
    return 0;
}

/* Sorted interacting partners of i.  cl == NULL means brute force. */
static int partners_of(const oracle_params* p, const double* x, const cells_t* cl,
                       int64_t i, vec_t* out) {
    int64_t n = 2 * p->n_agents;
    double d[2];
    out->n = 0;
    if (!cl) {
        for (int64_t j = 0; j < n; ++j)
            if (pair_interacts(p, x, i, j, d) && vec_push(out, j)) return -1;
        return 0;
    }
    int64_t nc = cl->nc;
    int64_t cx = cell_coord(x[2 * i], cl->inv_w, nc);
    int64_t cy = cell_coord(x[2 * i + 1], cl->inv_w, nc);
    for (int64_t dy = -1; dy <= 1; ++dy) {
        for (int64_t dx = -1; dx <= 1; ++dx) {
            int64_t c = ((cy + dy + nc) % nc) * nc + ((cx + dx + nc) % nc);
            for (int64_t t = cl->start[c]; t < cl->start[c + 1]; ++t) {
                int64_t j = cl->members[t];
                if (pair_interacts(p, x, i, j, d) && vec_push(out, j)) return -1;
            }
        }
    }
    if (out->n > 1) qsort(out->a, (size_t)out->n, sizeof(int64_t), cmp_i64);
    return 0;
}

static int64_t pairs_common(const oracle_params* p, const double* x, int use_cells,
                            int64_t* pairs, int64_t cap, int64_t* n_needed) {
    int64_t n = 2 * p->n_agents;
    cells_t cl;
    if (use_cells && cells_build(p, x, &cl)) return -1;
    vec_t nb = {0, 0, 0};
    int64_t count = 0;
    int err = 0;
    for (int64_t i = 0; i < n && !err; ++i) {
        if (partners_of(p, x, use_cells ? &cl : NULL, i, &nb)) { err = 1; break; }
        for (int64_t t = 0; t < nb.n; ++t) {
            int64_t j = nb.a[t];
            if (j <= i) continue;
            if (count < cap) { pairs[2 * count] = i; pairs[2 * count + 1] = j; }
            count++;
        }
    }
    free(nb.a);
    if (use_cells) cells_free(&cl);
    if (err) return -1;
    if (n_needed) *n_needed = count;
    return count <= cap ? count : -1;
}

int64_t oracle_pairs_brute(const oracle_params* p, const double* x,
                           int64_t* pairs, int64_t cap, int64_t* n_needed) {
    return pairs_common(p, x, 0, pairs, cap, n_needed);
}

int64_t oracle_pairs_cells(const oracle_params* p, const double* x,
                           int64_t* pairs, int64_t cap, int64_t* n_needed) {
    return pairs_common(p, x, 1, pairs, cap, n_needed);
}

/* ------------------------------------------------------------------------- */
/* Per-agent forces on particle i (Eqs. 2.5-2.7) and Stokes friction. */
static void agent_forces(const oracle_params* p, const double* x, const double* v,
                         int64_t i, double fb[2], double fsp[2], double fs[2]) {
    int64_t j = i ^ 1;                              /* bonded partner */
    double d0 = oracle_minimg(x[2 * i] - x[2 * j], p->L);
    double d1 = oracle_minimg(x[2 * i + 1] - x[2 * j + 1], p->L);
    double r = sqrt(d0 * d0 + d1 * d1);
    /* bond: -dV_H/dr_i with V_H = kappa (r - l)^2 / 2 */
    double cb = -p->kappa * (r - p->bond_l) / r;
    fb[0] = cb * d0; fb[1] = cb * d1;
    /* director n = (r_head - r_tail)/|r_head - r_tail|; d points from the
     * partner to i, so n = +d/r on the head (even i) and -d/r on the tail. */
    double sgn = (i % 2 == 0) ? 1.0 : -1.0;
    double share;
    if (p->sp_split == 0) share = 0.5;
    else share = (i % 2 == 0) ? 1.0 : 0.0;
    double csp = share * p->f_sp * sgn / r;
    fsp[0] = csp * d0; fsp[1] = csp * d1;
    fs[0] = -p->gamma_s * v[2 * i];
    fs[1] = -p->gamma_s * v[2 * i + 1];
}

/* Total force on particle i; optionally the three pair parts and the scale. */
static int force_on(const oracle_params* p, const double* x, const double* v,
                    const cells_t* cl, int64_t step, int64_t i, vec_t* nb,
                    double F[2], double parts_out[6], double* scale_out) {
    if (partners_of(p, x, cl, i, nb)) return -1;
    double acc[2] = {0.0, 0.0};
    double parts[6] = {0, 0, 0, 0, 0, 0};
    double scale = 0.0;
    for (int64_t t = 0; t < nb->n; ++t) {
        int64_t j = nb->a[t];
        double d[2], dv[2], f[2], pp[6];
        d[0] = oracle_minimg(x[2 * i] - x[2 * j], p->L);
        d[1] = oracle_minimg(x[2 * i + 1] - x[2 * j + 1], p->L);
        dv[0] = v[2 * i] - v[2 * j];
        dv[1] = v[2 * i + 1] - v[2 * j + 1];
        double alpha = oracle_pair_alpha(p, i, j, step);
        oracle_pair_force(p, d, dv, alpha, f, pp);
        acc[0] += f[0]; acc[1] += f[1];
        for (int k = 0; k < 6; ++k) parts[k] += pp[k];
        scale += sqrt(f[0] * f[0] + f[1] * f[1]);
    }
    double fb[2], fsp[2], fs[2];
    agent_forces(p, x, v, i, fb, fsp, fs);
    F[0] = acc[0] + fb[0] + fsp[0] + fs[0];
    F[1] = acc[1] + fb[1] + fsp[1] + fs[1];
    scale += sqrt(fb[0] * fb[0] + fb[1] * fb[1]) + sqrt(fsp[0] * fsp[0] + fsp[1] * fsp[1]) +
             sqrt(fs[0] * fs[0] + fs[1] * fs[1]);
    if (parts_out) for (int k = 0; k < 6; ++k) parts_out[k] = parts[k];
    if (scale_out) *scale_out = scale;
    return 0;
}

static int forces_impl(const oracle_params* p, const double* x, const double* v,
                       int64_t step, const int64_t* idx, int64_t n_idx, double* F,
                       double* parts, double* scale, int method) {
    cells_t cl;
    const cells_t* clp = NULL;
    if (method == 1) {
        if (cells_build(p, x, &cl)) return -1;
        clp = &cl;
    }
    int err = 0;
#pragma omp parallel reduction(| : err)
    {
        vec_t nb = {0, 0, 0};
#pragma omp for schedule(static)
        for (int64_t t = 0; t < n_idx; ++t) {
            int64_t i = idx ? idx[t] : t;
            double pp[6], sc;
            if (force_on(p, x, v, clp, step, i, &nb, &F[2 * t], pp, &sc)) { err = 1; continue; }
            if (parts) for (int k = 0; k < 6; ++k) parts[6 * t + k] = pp[k];
            if (scale) scale[t] = sc;
        }
        free(nb.a);
    }
    if (clp) cells_free(&cl);
    return err ? -1 : 0;
}

int oracle_forces(const oracle_params* p, const double* x, const double* v,
                  int64_t step, double* F, int method) {
    return forces_impl(p, x, v, step, NULL, 2 * p->n_agents, F, NULL, NULL, method);
}

int oracle_forces_subset(const oracle_params* p, const double* x, const double* v,
                         int64_t step, const int64_t* idx, int64_t n_idx, double* F) {
    return forces_impl(p, x, v, step, idx, n_idx, F, NULL, NULL, 1);
}

int oracle_force_parts(const oracle_params* p, const double* x, const double* v,
                       int64_t step, double* out, double* scale, int method) {
    int64_t n = 2 * p->n_agents;
    double* F = (double*)malloc((size_t)(2 * (n > 0 ? n : 1)) * sizeof(double));
    if (!F) return -1;
    int rc = forces_impl(p, x, v, step, NULL, n, F, out, scale, method);
    free(F);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Compensated (Kahan) sums of momentum and kinetic energy. */
void oracle_momentum_ke(const oracle_params* p, const double* v, double out[3]) {
    int64_t n = 2 * p->n_agents;
    double s[3] = {0, 0, 0}, c[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        double terms[3];
        terms[0] = p->mass * v[2 * i];
        terms[1] = p->mass * v[2 * i + 1];
        terms[2] = 0.5 * p->mass * (v[2 * i] * v[2 * i] + v[2 * i + 1] * v[2 * i + 1]);
        for (int k = 0; k < 3; ++k) {
            double y = terms[k] - c[k];
            double t = s[k] + y;
            c[k] = (t - s[k]) - y;
            s[k] = t;
        }
    }
    out[0] = s[0]; out[1] = s[1]; out[2] = s[2];
}

/* Velocity-Verlet (Sec. 5): half kick, drift with periodic wrap, force at the
 * new position with the half-step velocity, second half kick. */
int oracle_step(const oracle_params* p, double* x, double* v, double* F,
                int64_t* step, int64_t n, int method, int64_t every, double* pk) {
    int64_t np = 2 * p->n_agents;
    double h = p->dt / (2.0 * p->mass);
    double* u = (double*)malloc((size_t)(2 * (np > 0 ? np : 1)) * sizeof(double));
    if (!u) return -1;
    int64_t rec = 0;
    for (int64_t s = 0; s < n; ++s) {
        for (int64_t i = 0; i < 2 * np; ++i) u[i] = v[i] + h * F[i];
        for (int64_t i = 0; i < 2 * np; ++i) x[i] = oracle_wrap(x[i] + p->dt * u[i], p->L);
        *step += 1;
        if (forces_impl(p, x, u, *step, NULL, np, F, NULL, NULL, method)) { free(u); return -1; }
        for (int64_t i = 0; i < 2 * np; ++i) v[i] = u[i] + h * F[i];
        if (pk && every > 0 && (s + 1) % every == 0) {
            oracle_momentum_ke(p, v, &pk[3 * rec]);
            rec++;
        }
    }
    free(u);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Cell binning of FP32 positions, ordered by (cell, id). */
int64_t oracle_bin(const oracle_params* p, const float* x, int32_t* cell_start,
                   int32_t* ids) {
    int64_t n = 2 * p->n_agents;
    int64_t nc = oracle_n_cells_side(p);
    if (nc < 1) return -1;
    double inv_w = (double)nc / p->L;
    int64_t ncell = nc * nc;
    int64_t* key = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t* fill = (int64_t*)calloc((size_t)ncell, sizeof(int64_t));
    if (!key || !fill) { free(key); free(fill); return -1; }
    for (int64_t c = 0; c <= ncell; ++c) cell_start[c] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t cx = cell_coord((double)x[2 * i], inv_w, nc);
        int64_t cy = cell_coord((double)x[2 * i + 1], inv_w, nc);
        key[i] = cy * nc + cx;
        cell_start[key[i] + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) cell_start[c + 1] += cell_start[c];
    /* ascending id within each cell: visit ids in order */
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = key[i];
        ids[cell_start[c] + fill[c]] = (int32_t)i;
        fill[c] += 1;
    }
    free(key);
    free(fill);
    return nc;
}

/* ------------------------------------------------------------------------- */
/* Filtered and projected velocity field (Sec. 5.4). */
int oracle_bin_velocity(const oracle_params* p, const float* x, const float* v,
                        int32_t M, double eps, int32_t mode, double* u_out,
                        int32_t* n_out) {
    if (M < 1 || (mode != 0 && mode != 1)) return -1;
    int64_t np = 2 * p->n_agents;
    int64_t nsrc = (mode == 0) ? np : p->n_agents;
    double L = p->L;
    double dxm = L / (double)M;
    int64_t nbin = (int64_t)M * M;
    double* sum = (double*)calloc((size_t)(2 * nbin), sizeof(double));
    int64_t* cnt = (int64_t*)calloc((size_t)nbin, sizeof(int64_t));
    if (!sum || !cnt) { free(sum); free(cnt); return -1; }
    for (int64_t s = 0; s < nsrc; ++s) {
        double px, py, vx, vy;
        if (mode == 0) {
            px = x[2 * s]; py = x[2 * s + 1];
            vx = v[2 * s]; vy = v[2 * s + 1];
        } else {
            int64_t h = 2 * s, t = 2 * s + 1;
            double dx = (double)x[2 * h] - (double)x[2 * t];
            double dy = (double)x[2 * h + 1] - (double)x[2 * t + 1];
            if (dx >= 0.5 * L) dx -= L; else if (dx < -0.5 * L) dx += L;
            if (dy >= 0.5 * L) dy -= L; else if (dy < -0.5 * L) dy += L;
            px = (double)x[2 * t] + 0.5 * dx;
            py = (double)x[2 * t + 1] + 0.5 * dy;
            if (px < 0.0) px += L; else if (px >= L) px -= L;
            if (py < 0.0) py += L; else if (py >= L) py -= L;
            vx = 0.5 * ((double)v[2 * h] + (double)v[2 * t]);
            vy = 0.5 * ((double)v[2 * h + 1] + (double)v[2 * t + 1]);
        }
        if (eps <= 0.0) {
            /* eps = dx: each grid point owns the square [i dx, (i+1) dx) */
            double inv = (double)M / L;
            int64_t bx = (int64_t)floor(px * inv); if (bx > M - 1) bx = M - 1; if (bx < 0) bx = 0;
            int64_t by = (int64_t)floor(py * inv); if (by > M - 1) by = M - 1; if (by < 0) by = 0;
            int64_t b = by * M + bx;
            sum[2 * b] += vx; sum[2 * b + 1] += vy; cnt[b] += 1;
            continue;
        }
        double half = 0.5 * eps;
        /* candidate grid indices per axis, then the exact window test */
        int64_t lo[2], hi[2];
        double pos[2] = {px, py};
        for (int a = 0; a < 2; ++a) {
            lo[a] = (int64_t)floor((pos[a] - half) / dxm) - 1;
            hi[a] = (int64_t)floor((pos[a] + half) / dxm) + 1;
            if (hi[a] - lo[a] + 1 > M) { lo[a] = 0; hi[a] = M - 1; }
        }
        for (int64_t jy = lo[1]; jy <= hi[1]; ++jy) {
            int64_t gy = ((jy % M) + M) % M;
            double ym = ((double)gy + 0.5) * dxm;
            double ddy = py - ym;
            if (ddy >= 0.5 * L) ddy -= L; else if (ddy < -0.5 * L) ddy += L;
            if (!(ddy >= -half && ddy < half)) continue;
            for (int64_t jx = lo[0]; jx <= hi[0]; ++jx) {
                int64_t gx = ((jx % M) + M) % M;
                double xm = ((double)gx + 0.5) * dxm;
                double ddx = px - xm;
                if (ddx >= 0.5 * L) ddx -= L; else if (ddx < -0.5 * L) ddx += L;
                if (!(ddx >= -half && ddx < half)) continue;
                int64_t b = gy * M + gx;
                sum[2 * b] += vx; sum[2 * b + 1] += vy; cnt[b] += 1;
            }
        }
    }
    for (int64_t b = 0; b < nbin; ++b) {
        n_out[b] = (int32_t)cnt[b];
        if (cnt[b] > 0) {
            u_out[2 * b] = sum[2 * b] / (double)cnt[b];
            u_out[2 * b + 1] = sum[2 * b + 1] / (double)cnt[b];
        } else {
            u_out[2 * b] = 0.0;
            u_out[2 * b + 1] = 0.0;
        }
    }
    free(sum);
    free(cnt);
    return 0;
}
