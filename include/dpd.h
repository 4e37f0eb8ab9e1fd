/*
 * dpd.h -- C ABI of the MI355X DPD engine for self-propelled soft-core
 * dumbbells (Hinz, Panchenko, Kim & Fried, arXiv:1310.0998).
 *
 * The model (Sec. 2 of the paper): particle 2k is the head and 2k+1 the tail of
 * agent k.  Each particle feels
 *   - the DPD pair force f_C + f_D + f_R from every non-bonded particle within
 *     r_c (Eqs. 2.2-2.4), with e = (r_i - r_j)/r, w = 1 - r/r_c and the random
 *     number alpha^{ij} drawn from a counter-based generator keyed on
 *     (min id, max id, step, seed), so that f_ij = -f_ji exactly;
 *   - the harmonic bond V = kappa (r - l)^2 / 2 to its partner (Eq. 2.5), whose
 *     other pair forces are switched off (Sec. 2.2);
 *   - the self-propulsion f_sp n^k of its agent, n^k = (r_head - r_tail)/|...|
 *     (Eqs. 2.6-2.7), split f_sp/2 per particle or all on the head;
 *   - Stokes friction -gamma_s v (Eq. 2.6);
 * in a 2-D periodic square box of side L, advanced by velocity-Verlet (Sec. 5):
 *   u = v + dt/(2m) F;  x <- wrap(x + dt u);  F <- F(x, u, step + 1);
 *   v = u + dt/(2m) F.
 *
 * Conventions for every entry point:
 *   - Vector arrays are N x 2 FP32 (x0, y0, x1, y1, ...) in particle-id order,
 *     N = 2 n_agents, contiguous, in device memory of the current HIP device.
 *   - The caller owns every buffer and the workspace; the library allocates no
 *     device memory and frees nothing it was given.
 *   - All device work is enqueued on the stream given to dpd_create and is
 *     asynchronous unless stated otherwise; outputs are valid once the stream
 *     has been synchronised.  One handle per stream; a handle is not
 *     thread-safe.
 *   - Return value: DPD_OK (0) or a negative DPD_E* code; dpd_last_error gives
 *     the message.  No exception crosses the ABI and the library never aborts.
 *   - Device-side failures (non-finite state, a bonded partner beyond the
 *     neighbour stencil, a velocity too large for the binned field) set a flag
 *     that the next synchronising call (dpd_sync, dpd_get_state, dpd_forces,
 *     dpd_get_cells) reports.
 */
#ifndef DPD_H
#define DPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPD_OK          0
#define DPD_EINVAL     -1  /* bad argument or parameter                          */
#define DPD_EWORKSPACE -2  /* workspace missing, misaligned or too small          */
#define DPD_EHIP       -3  /* a HIP runtime call failed, or an internal device
                              check of the cell binning did (inconsistent counts,
                              a scan whose look-back exceeded its poll limit)    */
#define DPD_ENONFINITE -4  /* a non-finite position, velocity or force appeared   */
#define DPD_ESTATE     -5  /* call needs a state set by dpd_set_state first       */
#define DPD_EBOND      -6  /* a bond grew beyond the cell stencil (1.25 bond_l <= cell width) */
#define DPD_ERANGE     -7  /* a velocity exceeded the binned-field range          */

/* Model and engine parameters; physics constants in the units of the caller
 * (e.g. the nondimensional units of Sec. 3).  All fields are read once, by
 * dpd_workspace_bytes / dpd_create / dpd_rng_words. */
typedef struct dpd_params {
    int64_t  n_agents;   /* agents, >= 1; particles N = 2 n_agents <= 2^30           */
    double   L;          /* box side, exactly representable in FP32, >= 3 r_c         */
    double   r_c;        /* pair cutoff (Eq. 2.2), > 0; cells per side
                            n_c = floor(L / (r_c + skin)), >= 3.  A bond that can
                            reach beyond the 3 x 3 cell stencil (1.25 bond_l >
                            r_c + skin) has its partner read by particle id
                            (not with a skin)                                         */
    double   A;          /* conservative amplitude (Eq. 2.3), >= 0                    */
    double   gamma;      /* pair friction (Eq. 2.3), >= 0                             */
    double   kT;         /* thermal energy (Eq. 2.3), >= 0; sigma = sqrt(2 gamma kT)  */
    double   kappa;      /* bond stiffness (Eq. 2.5), >= 0                            */
    double   bond_l;     /* bond rest length (Eq. 2.5), >= 0                          */
    double   f_sp;       /* total self-propulsion per agent (Eq. 2.6)                 */
    double   gamma_s;    /* Stokes friction per particle (Eq. 2.6), >= 0              */
    double   mass;       /* particle mass (Eq. 2.1), > 0                              */
    double   dt;         /* time step, > 0                                            */
    uint64_t seed;       /* key of the noise generator                                */
    int32_t  noise_kind; /* 0: Gaussian alpha (Box-Muller); 1: uniform sqrt(3)(2u-1)  */
    int32_t  rng_kind;   /* 0: Philox4x32-10 on (min id, max id, step, 0), key = seed;
                            1: Philox2x32-10 on (min id, max id), key folds seed and step */
    int32_t  sp_split;   /* 0: f_sp/2 on head and tail; 1: f_sp on the head only      */
    int32_t  bin_M_max;  /* largest grid side dpd_bin_velocity will be asked for (0: 256) */
    int32_t  tile;       /* pair-kernel tile side in cells, 1..8 (0: 8 x 7 cells at one
                            particle per cell, the sides scaled by 1 / (particles per
                            cell), or by its square root with a skin)                */
    float    skin;       /* Verlet skin (>= 0, in units of length).  0: the cell list
                            is rebuilt every step with cells of width >= r_c.  > 0:
                            cells are >= r_c + skin wide and a rebuild also stores,
                            per tile, every pair closer than r_c + skin; later steps
                            test only those pairs, until some particle has moved more
                            than skin / 2 since the rebuild, which triggers the next
                            one (checked on the device, every step).  Results are
                            bitwise the same for every skin. */
    float    w_exp;      /* exponent s of the dissipative weight: f_D uses w^s and
                            f_R uses w^(s/2), so that the fluctuation-dissipation
                            balance of Eq. 2.3 holds for every s; f_C keeps w.
                            0 means 2 (Eq. 2.3 as printed); other values, in
                            (0, 8], are the change of exponent Sec. 6 proposes. */
    int32_t  reserved[1];
} dpd_params;

typedef struct dpd_handle dpd_handle;

/* Bytes of device workspace that dpd_create needs for these parameters.
 * Returns DPD_EINVAL for invalid parameters (message via dpd_last_error(NULL)). */
int dpd_workspace_bytes(const dpd_params* p, size_t* bytes);

/* Validate p, carve `workspace` (device memory, 256-byte aligned, at least
 * dpd_workspace_bytes bytes, owned by the caller and kept alive until
 * dpd_destroy) and bind the handle to `stream` (a hipStream_t; NULL = the null
 * stream).  Enqueues the clearing of internal counters on the stream.
 * Errors: DPD_EINVAL, DPD_EWORKSPACE, DPD_EHIP. */
int dpd_create(const dpd_params* p, void* workspace, size_t bytes, void* stream,
               dpd_handle** out);

/* Release the handle (host memory only; the workspace stays the caller's). */
void dpd_destroy(dpd_handle* h);

/* Message of the last failure on h, or of the last failed call without a
 * handle when h is NULL.  Never NULL. */
const char* dpd_last_error(const dpd_handle* h);

/* Set the state at `step` from x (positions in [0, L)^2; values outside are
 * wrapped) and v, both device N x 2 FP32 in id order.  If F is NULL the force
 * F(x, v, step) is evaluated (Eqs. 2.1-2.7 with the velocity v); otherwise F
 * (device N x 2, id order) is taken as the force of that state, which makes a
 * checkpoint taken with dpd_get_state resume bit-exactly.
 * Errors: DPD_EINVAL (NULL pointers), DPD_EHIP; non-finite inputs are reported
 * by the next synchronising call as DPD_ENONFINITE. */
int dpd_set_state(dpd_handle* h, const float* x, const float* v, int64_t step,
                  const float* F);

/* Copy the state out in id order: x, v, F device N x 2 FP32 (any may be NULL),
 * *step (host, may be NULL).  Synchronises the stream.
 * Errors: DPD_ESTATE, DPD_EHIP, device flags. */
int dpd_get_state(dpd_handle* h, float* x, float* v, float* F, int64_t* step);

/* Force F(x, v, step) of the current state (pair + bond + propulsion + Stokes,
 * velocity-dependent terms with the stored v), device N x 2 FP32, id order.
 * Does not change the state.  Synchronises the stream.
 * Errors: DPD_ESTATE, DPD_EINVAL, DPD_EHIP, device flags. */
int dpd_forces(dpd_handle* h, float* F_out);

/* Advance n_steps >= 0 velocity-Verlet steps (Sec. 5), rebinning the cell list
 * every step.  If reduce_every > 0 and pk_out != NULL, after every
 * reduce_every-th step the FP64 totals (P_x, P_y, KE) = (sum m v_x, sum m v_y,
 * sum m |v|^2 / 2) are written to device pk_out[3 r .. 3 r + 2], r = 0, 1, ...
 * (pk_out holds 3 * floor(n_steps / reduce_every) doubles; for a batch, record
 * r holds the totals of every replica q at pk_out[3 (r R + q) ..]).  With a
 * graph chunk set (dpd_set_graph_chunk) whole chunks are replayed from captured
 * graphs when reduce_every is 0 or a multiple of the chunk; the results are
 * bitwise those of the launches one by one.  Asynchronous.
 * Errors: DPD_ESTATE, DPD_EINVAL, DPD_EHIP. */
int dpd_step(dpd_handle* h, int32_t n_steps, int32_t reduce_every, double* pk_out);

/* Filtered and projected velocity field u_M (Sec. 5.4, Eqs. 5.8-5.10) of the
 * current state on an M x M grid (1 <= M <= bin_M_max), grid points
 * x_M = ((i + 1/2) L/M, (j + 1/2) L/M).  A contributor at x belongs to grid
 * point (i, j) iff the minimum-image d = x - x_M has both components in
 * [-eps/2, eps/2); eps <= 0 means non-overlapping bins of side L/M, each grid
 * point owning [i L/M, (i+1) L/M) x [j L/M, (j+1) L/M).  mode 0: particles and
 * their velocities; mode 1: agent centres of mass (minimum-image midpoints)
 * and (v_head + v_tail)/2.  u_out: device M*M*2 FP32, element (j*M + i)*2 + c,
 * the mean velocity (0 where nothing contributes); n_out: device M*M int32
 * contributor counts.  Sums are exact in 64-bit fixed point (scale 2^S with
 * S = min(32, 46 - ceil(log2(contributors + 1))), |v| <= 2^16), so the result
 * is independent of the order of contributions.  For a batch, replica q's
 * field follows at u_out + 2 q M M and n_out + q M M (each on its own box).
 * Asynchronous; a velocity beyond 2^16 is reported by the next synchronising
 * call as DPD_ERANGE.
 * Errors: DPD_ESTATE, DPD_EINVAL, DPD_EHIP. */
int dpd_bin_velocity(dpd_handle* h, int32_t M, double eps, int32_t mode,
                     float* u_out, int32_t* n_out);

/* dpd_bin_velocity with a window width of its own for every replica of a
 * batch: eps[r] (host array of the batch's replica count) for replica r, with
 * the meaning of eps above.  Each replica's field is binned once.
 * Errors: as dpd_bin_velocity. */
int dpd_bin_velocity_reps(dpd_handle* h, int32_t M, const double* eps, int32_t mode,
                          float* u_out, int32_t* n_out);

/* Velocity correlation function of the agents (Sec. 5.3, Eqs. 5.5-5.6), as
 * pair sums by separation.  Agent k's centre of mass is the minimum-image
 * midpoint of its head 2k and tail 2k+1 (wrapped into [0, L)) and its velocity
 * V_k = (v_2k + v_2k+1) / 2, in FP64 from the FP32 state.  For every bin
 * b < n_bins of width dr, over the pairs k < l whose minimum-image separation
 * r has floor(r / dr) = b:
 *   sums[b]   = sum of round(2^20 V_k . V_l) (exact integer sums, any order),
 *   counts[b] = number of pairs.
 * The caller forms g(r_b) = (sums[b] 2^-20 / counts[b] - |<V>|^2) /
 * (<|V|^2> - |<V>|^2) with the means over agents (Eq. 5.6), taken from the
 * velocities left in work.
 *   x, v: device N x 2 FP32 in id order, N = 2 n_agents (1 <= n_agents <= 2^29);
 *   work: device FP64 scratch of 4 n_agents + 1 values, caller's; on return
 *         work[0 .. 2n) holds the centres (x, y per agent) and
 *         work[2n .. 4n) the velocities V;
 *   sums, counts: device int64[n_bins], 1 <= n_bins <= 1024, caller's;
 *   stream: a hipStream_t (NULL = the null stream).
 * O(n_agents^2) pairs on the GPU.  Synchronises the stream.
 * Errors: DPD_EINVAL; DPD_ERANGE if some |V_k . V_l| reached 4096 (the sums
 * would lose exactness); DPD_EHIP. */
int dpd_agent_vcf(const float* x, const float* v, int64_t n_agents, double L, double dr,
                  int32_t n_bins, double* work, long long* sums, long long* counts, void* stream);

/* Wait for the stream and return the first device-side failure since the last
 * synchronising call (clearing it), or DPD_OK. */
int dpd_sync(dpd_handle* h);

/* ---- batches of replicas, captured step chunks, tile schedules ------------- */

/* A batch of n_rep independent systems, e.g. the points of a parameter sweep
 * over area fraction and the two friction coefficients (Sec. 5, Sec. 5.1):
 * p[0 .. n_rep-1] are their parameters (any sizes, boxes and constants; skin
 * must be 0), each system keeping its own ids 0 .. N_q - 1 and its own noise
 * key.  The batch's per-step kernels cover every replica in one launch each;
 * each replica's
 * trajectory is bitwise the one of a handle made for it alone.  All state
 * arrays of the entry points above are the replicas' arrays concatenated in
 * replica order (replica q's N_q x 2 block follows replica q - 1's);
 * dpd_get_cells returns the concatenated cell lists (replica q's cells follow
 * replica q - 1's, slots counted over the batch).  A handle made by dpd_create
 * is a batch of one.  Errors as dpd_workspace_bytes / dpd_create. */
int dpd_batch_workspace_bytes(const dpd_params* p, int32_t n_rep, size_t* bytes);
int dpd_create_batch(const dpd_params* p, int32_t n_rep, void* workspace, size_t bytes,
                     void* stream, dpd_handle** out);

/* Replay dpd_step in chunks of `steps` (even, <= 4096; 0: off) launches
 * captured once into a HIP graph (on a stream of the handle's own; replayed on
 * the handle's stream), which removes the host's per-launch cost.  Not used
 * with a Verlet skin or while profiling.  Errors: DPD_EINVAL. */
int dpd_set_graph_chunk(dpd_handle* h, int32_t steps);

/* Pair-kernel schedule: tiles of tile_x x tile_y cells (1..8, clamped per
 * replica to n_c - 2), or tile_x = tile_y = 0 for every replica's default
 * tile (see dpd_params.tile), and the tile order (0: each of the 8 XCDs takes a
 * band of consecutive tiles; 1: launch order).  The workspace holds the tiles
 * of the schedules dpd_autotune tries and of the one the handle was made with;
 * smaller tiles are refused.  The results do not depend on the schedule.
 * dpd_get_schedule reports replica 0's tile.  Not with a Verlet skin.
 * Errors: DPD_EINVAL. */
int dpd_set_schedule(dpd_handle* h, int32_t tile_x, int32_t tile_y, int32_t tile_order);
int dpd_get_schedule(dpd_handle* h, int32_t* tile_x, int32_t* tile_y, int32_t* tile_order);

/* Time trial_steps steps of the current state under each candidate schedule
 * (every replica's default tile scaled by 1, 0.85, 0.7 and 0.55; the same
 * 8 x 7, 8 x 8, 6 x 6 and 4 x 4 tiles for all; both tile orders), keep the
 * fastest and restore the state exactly as it was (state, step, no prepared
 * step).  In a batch, replicas that still have more than 2 % of their tiles
 * over the tile kernel's LDS capacities (dense clusters) then move, round by
 * round while the step gets faster, to finer tiles (down to the default tile
 * scaled by 0.3), so replicas can end with tiles of different scales; the
 * batch workspace holds those tilings.  The choice holds for states like the
 * one timed: cell occupancy changes along a run (a random start relaxes within
 * a few hundred steps, and propelled agents cluster), so tune on a state of
 * the kind the run will see, and again as it changes.
 * Outputs (host, any may be NULL): replica 0's tile and the tile order of the
 * chosen schedule, and its time per step in ms.  Synchronises the stream.
 * Not with a Verlet skin.  Errors: DPD_ESTATE, DPD_EINVAL, DPD_EHIP, device
 * flags; after DPD_EHIP the state and schedule are those of the failed trial. */
int dpd_autotune(dpd_handle* h, int32_t trial_steps, int32_t* tile_x, int32_t* tile_y,
                 int32_t* tile_order, double* best_ms);

/* ---- one call that allocates nothing ---------------------------------------- */

/* For callers that cannot allocate device memory or pass a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the force F(x, v, step) of dpd_forces (pair + bond + propulsion
 * + Stokes, Eqs. 2.1-2.7) for one system given directly by its state, with the
 * library's own static device scratch as the workspace.
 *   p: parameters as for dpd_create (skin and bin_M_max are ignored);
 *   x, v: device N x 2 FP32 in id order (caller's, read only);
 *   F_out: device N x 2 FP32 in id order (caller's, written);
 *   stream: a hipStream_t (NULL = the null stream).
 * The scratch is a fixed 32 MiB per device (about 250k particles at one
 * particle per cell); larger systems are refused with DPD_EWORKSPACE before
 * any device work.  It calls no hipMalloc or hipFree and creates no stream or
 * event.  Every call on a device shares that device's scratch and clears what
 * must start at zero: calls that overlap on one device (other streams or
 * threads) race.  Synchronises the stream; the results are bitwise those of
 * dpd_create + dpd_set_state + dpd_forces.
 * Errors: DPD_EINVAL, DPD_EWORKSPACE, DPD_EHIP, device flags. */
int dpd_forces_noalloc(const dpd_params* p, const float* x, const float* v, int64_t step,
                       float* F_out, void* stream);

/* ---- diagnostics used by tests and the benchmark --------------------------- */

/* The cell list of the current state: cell_start_out device int32[n_c^2 + 1]
 * (first slot of each cell, row-major cells cy * n_c + cx with
 * c = min(n_c - 1, floor(x * n_c / L)) per axis in FP64), ids_out device
 * int32[N] (particle ids ordered by (cell, id)).  With a Verlet skin it is the
 * list of the last rebuild: n_c cells per side (dpd_cells_per_side), binned
 * from the positions of that step (no particle has moved more than skin / 2
 * since).  Synchronises the stream. */
int dpd_get_cells(dpd_handle* h, int32_t* cell_start_out, int32_t* ids_out);

/* Cells per side of the cell list for p (n_c = floor(L / (r_c + skin)), the
 * skin being 0 unless set), or a negative error code. */
int64_t dpd_cells_per_side(const dpd_params* p);

/* The generator output for n pairs (i[k], j[k]) at `step` with p's seed,
 * rng_kind and noise_kind: words_out device uint32[4 n] (unused words zero),
 * alpha_out device float[n] (may be NULL).  i, j device int32[n].  Enqueued on
 * `stream`; synchronises it. */
int dpd_rng_words(const dpd_params* p, const int32_t* i, const int32_t* j, int64_t step,
                  int32_t n, uint32_t* words_out, float* alpha_out, void* stream);

/* Bracket every 8th launch of the fused pair kernel (the first, ninth, ...
 * after switching on) with HIP events on the handle's stream (on != 0), or stop
 * doing so (on == 0).  Only a sample is bracketed because an event record
 * between two kernels costs a few microseconds of GPU time. */
int dpd_set_profiling(dpd_handle* h, int32_t on);

/* Total device time (ms) and number of the bracketed launches of the fused
 * pair kernel since profiling was switched on.  Synchronises the stream. */
int dpd_pair_kernel_time(dpd_handle* h, double* ms_total, int64_t* launches);

/* Number of steps since dpd_create that rebuilt the cell list under a Verlet
 * skin (skin > 0: the first step of a dpd_step call after dpd_create,
 * dpd_set_state, dpd_forces or a windowed / centre-of-mass dpd_bin_velocity,
 * and every step after one on which some particle had moved more than skin / 2
 * since the last rebuild); 0 without a skin.  Synchronises the stream. */
int dpd_cell_list_rebuilds(dpd_handle* h, int64_t* rebuilds);

/* Plain device-to-device copy of `bytes` (multiple of 16) by a simple
 * streaming kernel, for calibrating hardware byte counters.  Enqueued on
 * `stream`. */
int dpd_copy_kernel(const void* src, void* dst, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DPD_H */
