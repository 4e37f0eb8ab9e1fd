/*
 * oracle.h -- plain FP64 CPU reference ("oracle") for the self-propelled
 * soft-core dumbbell DPD model (Hinz, Panchenko, Kim & Fried, arXiv:1310.0998).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code: only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code with the HIP engine.
 *
 * Everything here is FP64, written for obviousness rather than speed:
 *   - forces are the all-pairs sum of the DPD pair force (Sec. 2.1, Eqs. 2.2-2.4)
 *     under the minimum-image convention, with the bonded partner excluded
 *     (Sec. 2.2), plus the harmonic bond (Eq. 2.5), self-propulsion and Stokes
 *     friction (Sec. 2.3, Eqs. 2.6-2.7);
 *   - a cell list is offered only as a faster way to reach exactly the same
 *     pair set; each particle sums its pairs in ascending partner id, so both
 *     routes give bit-identical forces;
 *   - time stepping is velocity-Verlet (Sec. 5, first paragraph);
 *   - the filtered/projected field u_M follows Sec. 5.4, Eqs. 5.8-5.10.
 *
 * Particle 2k is the head and 2k+1 the tail of agent k.  Arrays of vectors are
 * interleaved (x0, y0, x1, y1, ...).
 */
#ifndef DPD_ORACLE_H
#define DPD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oracle_params {
    int64_t  n_agents;   /* agents; particles N = 2 n_agents                       */
    double   L;          /* side of the periodic square box                        */
    double   r_c;        /* pair cutoff radius (Eq. 2.2)                           */
    double   A;          /* conservative amplitude (Eq. 2.3, first line)           */
    double   gamma;      /* pair friction (Eq. 2.3, second line)                   */
    double   kT;         /* thermal energy (Eq. 2.3, third line)                   */
    double   kappa;      /* bond stiffness (Eq. 2.5)                               */
    double   bond_l;     /* bond rest length (Eq. 2.5)                             */
    double   f_sp;       /* self-propulsion force per agent (Eq. 2.6)              */
    double   gamma_s;    /* Stokes friction per particle (Eq. 2.6)                 */
    double   mass;       /* particle mass (Eq. 2.1)                                */
    double   dt;         /* time step                                              */
    uint64_t seed;       /* key of the counter-based noise generator               */
    int32_t  noise_kind; /* 0: Gaussian alpha, 1: uniform alpha of unit variance   */
    int32_t  rng_kind;   /* 0: Philox4x32-10, 1: Philox2x32-10                     */
    int32_t  sp_split;   /* 0: f_sp/2 on each particle, 1: all of f_sp on the head */
    int32_t  pad_;
    double   w_exp;      /* exponent s of the dissipative weight w^s; the random
                            weight is w^(s/2) and the conservative one stays w
                            (s = 2: Eq. 2.3 as printed; other s: the change of
                            exponent that Sec. 6 proposes)                       */
} oracle_params;

/* ---- counter-based generator (Salmon, Moraes, Dror & Shaw, SC'11) ---------- */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void oracle_philox2x32_10(const uint32_t ctr[2], uint32_t key, uint32_t out[2]);
/* Raw words used for the pair (i, j) at `step`; symmetric in (i, j).
 * Writes 4 words for rng_kind 0, 2 words (rest zero) for rng_kind 1. */
void oracle_pair_words(const oracle_params* p, int64_t i, int64_t j, int64_t step,
                       uint32_t out[4]);
/* The random number alpha^{ij} of Eq. 2.3 (third line). */
double oracle_pair_alpha(const oracle_params* p, int64_t i, int64_t j, int64_t step);

/* ---- single-pair force (Eqs. 2.2-2.4) --------------------------------------
 * d = x_i - x_j (already minimum-imaged), dv = v_i - v_j.
 * Writes the force on i into f and returns 1 if 0 < |d| < r_c, else writes 0
 * and returns 0.  The three parts are also returned when parts != NULL as
 * [fC_x, fC_y, fD_x, fD_y, fR_x, fR_y]. */
int oracle_pair_force(const oracle_params* p, const double d[2], const double dv[2],
                      double alpha, double f[2], double* parts);

/* ---- pair sets -------------------------------------------------------------
 * Interacting pairs (i < j, j != partner(i), 0 < r^2 < r_c^2), lexicographically
 * sorted, written as (i, j) int64 pairs.  Returns the number of pairs, or -1 if
 * cap is too small (the count is then still returned in *n_needed). */
int64_t oracle_pairs_brute(const oracle_params* p, const double* x,
                           int64_t* pairs, int64_t cap, int64_t* n_needed);
int64_t oracle_pairs_cells(const oracle_params* p, const double* x,
                           int64_t* pairs, int64_t cap, int64_t* n_needed);

/* ---- total force on every particle -----------------------------------------
 * F(x, v, step): pair forces + bond + propulsion + Stokes friction, where the
 * velocity-dependent terms use the v passed in.  method 0: all pairs,
 * method 1: cell list (requires floor(L/r_c) >= 3).  Returns 0 or -1. */
int oracle_forces(const oracle_params* p, const double* x, const double* v,
                  int64_t step, double* F, int method);
/* Same, but only for the particles listed in idx (F holds n_idx vectors). */
int oracle_forces_subset(const oracle_params* p, const double* x, const double* v,
                         int64_t step, const int64_t* idx, int64_t n_idx, double* F);
/* Pair-force part only, split per particle into the three DPD terms:
 * out[6*i + 0..5] = sum over partners of (fC, fD, fR).  Also returns the
 * per-particle scale S_i = sum_j |f_ij| + |F_bond| + |F_sp| + |F_S| in scale
 * (may be NULL).  method as above. */
int oracle_force_parts(const oracle_params* p, const double* x, const double* v,
                       int64_t step, double* out, double* scale, int method);

/* ---- velocity-Verlet stepping (Sec. 5) -------------------------------------
 * State (x, v, F) at step *step; F must equal F(x, v, *step) on entry (use
 * oracle_forces to initialise).  Advances n steps:
 *   u = v + dt/(2m) F;  x <- wrap(x + dt u);  step += 1;  F <- F(x, u, step);
 *   v = u + dt/(2m) F.
 * If pk != NULL and every > 0, after each `every` steps writes
 * (P_x, P_y, KE) into pk (3 doubles per record).  Returns 0 or -1. */
int oracle_step(const oracle_params* p, double* x, double* v, double* F,
                int64_t* step, int64_t n, int method, int64_t every, double* pk);

/* Total momentum and kinetic energy, compensated summation. out = (Px, Py, KE). */
void oracle_momentum_ke(const oracle_params* p, const double* v, double out[3]);

/* ---- cell binning reference -------------------------------------------------
 * Positions are FP32 (the engine's storage type).  n_c = floor(L / r_c),
 * inv_w = n_c / L (FP64), cell = min(n_c - 1, floor(x * inv_w)) per axis,
 * cell index = cy * n_c + cx.  Outputs cell_start[n_c^2 + 1] and the particle
 * ids ordered by (cell, id).  Returns n_c, or -1 on bad input. */
int64_t oracle_bin(const oracle_params* p, const float* x, int32_t* cell_start,
                   int32_t* ids);
int64_t oracle_n_cells_side(const oracle_params* p);

/* ---- filtered and projected velocity field (Sec. 5.4, Eqs. 5.8-5.10) --------
 * Grid points x_M = ((i + 1/2) dx, (j + 1/2) dx), dx = L / M.  A particle
 * (mode 0) or agent centre of mass (mode 1) at x contributes to grid point
 * (i, j) iff d = minimg(x - x_M) has both components in [-eps/2, eps/2).
 * eps <= 0 means eps = dx (non-overlapping bins).  Positions and velocities are
 * FP32 inputs.  u_out[2*(j*M+i) + c] is the mean velocity, n_out[j*M+i] the
 * number of contributors (u = 0 where n = 0).  Returns 0 or -1. */
int oracle_bin_velocity(const oracle_params* p, const float* x, const float* v,
                        int32_t M, double eps, int32_t mode, double* u_out,
                        int32_t* n_out);

/* Minimum-image wrap of a separation component, and periodic wrap of a position. */
double oracle_minimg(double d, double L);
double oracle_wrap(double y, double L);

int oracle_num_threads(void);
/* OpenMP threads of the following calls (n > 0; ignored without OpenMP). */
void oracle_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
