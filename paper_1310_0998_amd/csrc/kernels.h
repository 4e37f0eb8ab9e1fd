// kernels.h -- HIP kernels of the DPD engine (gfx950).
//
// One step of the hot path runs four kinds of kernel on the caller's stream:
//   k_pair<STEP>  fused: stage a tile of cells plus a one-cell halo in LDS,
//                 DPD pair forces (Eqs. 2.2-2.4, bonded partner excluded),
//                 bond + propulsion + Stokes (Eqs. 2.5-2.7), second half kick,
//                 next step's half kick + drift + FP64 wrap, new cell key and
//                 its atomic rank in the new cell;
//   k_scan_*      exclusive scan of the per-cell counts -> cell_start;
//   k_scatter     slot = cell_start[key] + rank;
//   k_cell_sort   order every cell's members by particle id,
// so that the particle order is always (cell, id), bit-identical to a plain
// counting sort, and every sum below runs in a fixed order.
#pragma once

#include "device.h"

namespace dpd {

constexpr int kBlock = 256;  // threads per block of the streaming kernels

// Pair kernel: one wavefront per tile of up to kTileX x kTileY cells.
constexpr int kTileX = 8, kTileY = 7;                // default tile (cells)
constexpr int kTileMax = 8;                          // largest tile side
constexpr int kLocMax = (kTileMax + 2) * (kTileMax + 2);  // tile + halo cells
// Capacities of a tile in LDS, about 4-5 standard deviations above what an
// 8 x 7 tile holds at one particle per cell (56 tile particles, 90 staged, about
// 100 kept pairs); a tile over any of them goes to the global-memory kernel
// (the same results bit for bit).  Small capacities keep the LDS of a
// wavefront near 6 KB, so that about 25 wavefronts fit on a CU.
constexpr int kCap = 128;   // staged particles (tile + halo); indices fit a byte, 0xFF = none
constexpr int kTP = 96;     // tile particles
constexpr int kEcap = 192;  // kept pairs per tile
constexpr int kItems = kCap / kWave;  // staged particles per lane
constexpr int kLcap = 512;  // listed pairs per tile (Verlet skin)

// What a rebuild stores per tile for the steps that follow it (Verlet skin):
// the staged set (global slot and tile index of every staged particle, in the
// canonical order of the rebuild), the tile particles' staged indices and
// bonded partners, and every tile pair closer than r_c + skin (staged index of
// the tile particle << 8 | staged index of the other).
struct TileRec {
    int ntile, total, nlist, valid;
    int slot[kCap];
    unsigned char tix[kCap];
    unsigned char tslot[kTP];
    unsigned char partner[kTP];
    unsigned short pairs[kLcap];
};
constexpr size_t kRecStride = (sizeof(TileRec) + 255) / 256 * 256;

enum PairMode { MODE_STEP = 0, MODE_FINAL = 1, MODE_FORCES = 2 };

struct PairArgs {
    const int* cs;      // cell_start of the current (cell, id) order
    const int* src;     // sorted slot -> index in the input buffers
    const float2* xin;
    const float2* uin;  // velocity the forces use
    const int* idin;
    float2* xout;       // STEP: next position; FINAL/FORCES: position
    float2* uout;       // STEP: next half-step velocity; FINAL: v; FORCES: input velocity
    int* idout;
    int* keyout;        // STEP: new cell key (index into the cells of the whole batch)
    int* rankout;       // STEP: rank of the particle within its new cell
    int* count;         // STEP: per-cell counters (atomically incremented)
    float2* Fout;       // FINAL/FORCES: total force
    float2* pxout;      // FINAL, if not null: also the next step's drifted position,
    float2* puout;      //   half-step velocity and id (as k_kick_drift would make them),
    int* pidout;        //   with keyout, rankout and count as in STEP
    double* red;        // 3 doubles per tile (sum v_x, sum v_y, sum |v|^2) or null
    unsigned* status;
    int* ovf_count;     // tiles handed to the global-memory kernel (cleared by the cell-count scan)
    int* ovf_list;      // their tile indices
    // Verlet skin (all null without it)
    const int* rebuild; // nonzero: this step rebuilds the cell list (null: always)
    unsigned char* rec; // tile records, kRecStride bytes each
    float2* xref;       // position of every slot at the last rebuild
    int* moved;         // set when a particle has moved more than skin / 2 since then
    int* count_clear;   // STEP: the counter array this step's binning consumed, cleared
                        // tile by tile (null: none)
    uint32_t step;      // step number of the force evaluation (mod 2^32), or its
                        // offset from *step_base when that is set
    const uint32_t* step_base;  // null, or the step before a replayed graph chunk
    // a batch of replicas: the parameters of each, the replica of each tile of
    // the concatenated tile list, and the number of tiles
    const DevParams* reps;
    const int* tile_rep;
    int nt_total;
    int tile_order;     // 0: bands of consecutive tiles per XCD; 1: launch order
    // bonds longer than the cell stencil reaches (far_bond): index in the input
    // buffers of the particle with id i of the replica at pbase, at pos_of_id[pbase + i]
    const int* pos_of_id;
    // STEP, and FINAL with pxout: the same map for the buffers this launch
    // writes (the next step's input), or null
    int* pos_out;
};

// ---- small helpers ----------------------------------------------------------

// The pair kernels take (DevParams, PairArgs, int) by value; the kernel-argument
// segment holds them in that order at their natural alignment.  Reading an
// argument again from that segment behind a compiler barrier gives the same
// values in fresh scalar registers: the compiler can then no longer keep the
// first copies live from the prologue to the last phase, which overflows the
// scalar registers and spills them into vector-register lanes (one vector
// instruction per spill and per reload).
constexpr int kArgOffPairArgs =
    (int)((sizeof(DevParams) + alignof(PairArgs) - 1) / alignof(PairArgs) * alignof(PairArgs));

template <class T>
__device__ __forceinline__ T kernel_arg_again(int offset) {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const char __attribute__((address_space(4)))* seg_ptr;
    typedef const T __attribute__((address_space(4)))* arg_ptr;
    seg_ptr p = (seg_ptr)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return *(arg_ptr)(p + offset);
#else
    (void)offset;  // the host pass only parses device code
    return T{};
#endif
}

__device__ __forceinline__ int wrap_cell(int c, int nc) {
    c += (c < 0) ? nc : 0;
    return c - ((c >= nc) ? nc : 0);
}

// Exclusive scan of vals[0..n) in LDS by a 256-thread block (n <= 512);
// vals[n] receives the total, which is also returned.
__device__ int block_scan_excl_512(int* vals, int n, int* s_wave) {
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    const int a = (2 * t < n) ? vals[2 * t] : 0;
    const int b = (2 * t + 1 < n) ? vals[2 * t + 1] : 0;
    const int s = a + b;
    int incl = s;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) s_wave[w] = incl;
    __syncthreads();
    int wofs = 0;
    for (int k = 0; k < w; ++k) wofs += s_wave[k];
    const int total = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    const int excl = wofs + incl - s;
    if (2 * t < n) vals[2 * t] = excl;
    if (2 * t + 1 < n) vals[2 * t + 1] = excl + a;
    if (t == 0) vals[n] = total;
    __syncthreads();
    return total;
}

// Sum of three doubles over a 256-thread block in a fixed order; result valid
// in thread 0.
__device__ void block_sum3(double v[3], double (*s_red)[3]) {
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) v[k] += __shfl_down(v[k], o, kWave);
    }
    if (lane == 0) {
        s_red[w][0] = v[0]; s_red[w][1] = v[1]; s_red[w][2] = v[2];
    }
    __syncthreads();
    if (t == 0) {
        for (int k = 0; k < 3; ++k)
            v[k] = ((s_red[0][k] + s_red[1][k]) + s_red[2][k]) + s_red[3][k];
    }
}

// r_c^2 - |d|^2 by two fused multiply-adds: accurate to ~1e-8 absolute near the
// cutoff, where 1 - r/r_c would lose most of its digits.
__device__ __forceinline__ float cutoff_gap(const DevParams& P, float dx, float dy) {
    return fmaf(-dy, dy, fmaf(-dx, dx, P.rc2));
}

// The pair interacts iff 0 < |d| < r_c: q = r_c^2 - |d|^2 > 0 and r2 = |d|^2 > 0
// (q alone cannot tell a coincident pair from one a few ulps apart).
__device__ __forceinline__ bool interacts(float q, float r2) { return q > 0.f && r2 > 0.f; }

// DPD pair force on i from j (Eqs. 2.2-2.4) added to (fx, fy); d = x_i - x_j,
// r2 = |d|^2 and q = r_c^2 - |d|^2 with interacts(q, r2).  The weight
// w = 1 - r/r_c (Eq. 2.4) is evaluated as q / (r_c (r_c + r)).  Every
// operation is symmetric under (i, j, d) -> (j, i, -d), so the force on j is
// bitwise the negation.  WEXP = false compiles the printed weights (w, w^2)
// only; with WEXP the exponent P.w_half is applied when it is not 1.
template <bool WEXP = true>
__device__ __forceinline__ void add_pair_force(const DevParams& P, float dx, float dy,
                                               float q, float r2, float2 ui, float2 uj, int idi,
                                               int idj, uint32_t step, float& fx,
                                               float& fy) {
    const float rinv = rsqrtf(r2);
    const float r = r2 * rinv;
    const float w = q * __builtin_amdgcn_rcpf(fmaf(r, P.rc, P.rc2));
    const float ex = dx * rinv, ey = dy * rinv;
    const float g = (ui.x - uj.x) * ex + (ui.y - uj.y) * ey;
    const uint32_t a = (uint32_t)min(idi, idj), b = (uint32_t)max(idi, idj);
    const float alpha = alpha_from_words(P.noise_kind, pair_words2(P, a, b, step));
    // random weight w^(s/2) and dissipative weight its square (s = 2: w and w^2)
    float wr = w;
    if (WEXP && P.w_half != 1.0f) wr = exp2f(P.w_half * log2f(w));
    const float s = P.A * w - P.gamma * wr * wr * g + P.sigma_rdt * wr * alpha;
    fx += s * ex;
    fy += s * ey;
}

// Bond stretch r - l for the separation d = (dx + dx_lo, dy + dy_lo).  r^2 is
// formed without rounding error (two-product and two-sum, the lo parts to
// first order), and r - l = (r^2 - l^2) / (r + l), so the stiff bond force
// kappa (r - l) keeps FP32 relative accuracy even though r itself is only
// known to one FP32 ulp.
__device__ __forceinline__ float bond_stretch(const DevParams& P, float dx, float dx_lo, float dy,
                                              float dy_lo, float& r) {
#pragma clang fp contract(off)
    const float px = dx * dx, ex = fmaf(2.0f * dx, dx_lo, fmaf(dx, dx, -px));
    const float py = dy * dy, ey = fmaf(2.0f * dy, dy_lo, fmaf(dy, dy, -py));
    const float s = px + py;
    const float bp = s - px;
    const float es = (px - (s - bp)) + (py - bp);
    const float lo = (es + ex) + ey;
    const float num = (s - P.bond_l2_hi) + (lo - P.bond_l2_lo);
    r = __builtin_amdgcn_sqrtf(s);
    return num * __builtin_amdgcn_rcpf(r + P.bond_l);
}

// Bond to the partner (Eq. 2.5), propulsion along n = (r_head - r_tail)/|.|
// (Eqs. 2.6-2.7) and Stokes friction (Eq. 2.6) on particle i at xi.
__device__ __forceinline__ void add_agent_force(const DevParams& P, float2 xi, float2 xp,
                                                float2 ui, int idi, float& fx, float& fy) {
    float lx, ly;
    const float dx = minimg_sub2(xi.x, xp.x, P, lx);
    const float dy = minimg_sub2(xi.y, xp.y, P, ly);
    float r;
    const float stretch = bond_stretch(P, dx, lx, dy, ly, r);
    const float rinv = __builtin_amdgcn_rcpf(r);
    const float cb = -P.kappa * stretch * rinv;
    const float csp = ((idi & 1) ? -P.sp_tail : P.sp_head) * rinv;
    fx += (cb + csp) * dx - P.gamma_s * ui.x;
    fy += (cb + csp) * dy - P.gamma_s * ui.y;
}

// Pair-force sums are kept in 64-bit fixed point with 32 fractional bits.
// Integer addition is associative, so a particle's total does not depend on
// the order its pairs are added in, and the force on j from a pair is exactly
// the negation of the force on i.  One term is rounded to 2^-32 (~2e-10);
// |F| must stay below 2^31 (a non-finite force is flagged separately).
constexpr double kFixScale = 4294967296.0;        // 2^32
constexpr double kFixInv = 1.0 / 4294967296.0;    // 2^-32

__device__ __forceinline__ long long to_fixed(float f) {
    const double d = rint((double)f * kFixScale);   // exact: f has 24 significant bits
    const double hi = floor(d * kFixInv);
    const double lo = fma(hi, -kFixScale, d);       // exact, in [0, 2^32)
    return (long long)(((unsigned long long)(unsigned)(int)hi << 32) | (unsigned long long)(unsigned)lo);
}

__device__ __forceinline__ float from_fixed(long long q) {
    return (float)((double)q * kFixInv);            // (double)q exact for |q| < 2^53
}

// With a Verlet skin: the position at the last rebuild is recorded (or read),
// and a particle whose next position is more than skin / 2 from it asks for a
// rebuild before the next force evaluation.
__device__ __forceinline__ bool moved_too_far(const DevParams& P, const PairArgs& a, int g,
                                              float2 xi, float2 xn, bool rebuilt) {
    float2 xr;
    if (rebuilt) {
        a.xref[g] = xi;
        xr = xi;
    } else {
        xr = a.xref[g];
    }
    const float dx = minimg_sub(xn.x, xr.x, P), dy = minimg_sub(xn.y, xr.y, P);
    return !(fmaf(dx, dx, dy * dy) <= P.half_skin2);
}

// Finish one particle: kicks, drift, key and outputs at sorted slot g.  SKIN:
// the displacement test of a Verlet skin is compiled in (it also needs a.moved).
template <int MODE, bool SKIN>
__device__ __forceinline__ void finish_particle(const DevParams& P, const PairArgs& a, int g,
                                                float2 xi, float2 ui, int idi, float fx,
                                                float fy, double rv[3], bool reduce,
                                                bool rebuilt = true) {
    const float2 F = make_float2(fx, fy);
    if (MODE == MODE_FORCES) {
        a.xout[g] = xi;
        a.uout[g] = ui;
        a.idout[g] = idi;
        a.Fout[g] = F;
        if (!finite2(F)) atomicOr(a.status, kStatusNonFinite);
        return;
    }
    // half kicks as explicit fused multiply-adds, so that every kernel that kicks
    // (this one, k_kick_drift) rounds them identically
    const float2 v = make_float2(fmaf(P.h, fx, ui.x), fmaf(P.h, fy, ui.y));
    if (reduce) {
        rv[0] += (double)v.x;
        rv[1] += (double)v.y;
        rv[2] += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
    }
    if (MODE == MODE_FINAL) {
        a.xout[g] = xi;
        a.uout[g] = v;
        a.idout[g] = idi;
        a.Fout[g] = F;
        bool bad = !finite2(v) || !finite2(F);
        if (a.pxout) {  // start the next call's first step: half kick, drift, key, rank
            const float2 un = make_float2(fmaf(P.h, fx, v.x), fmaf(P.h, fy, v.y));
            const float2 xn = make_float2(drift_wrap(xi.x, un.x, P), drift_wrap(xi.y, un.y, P));
            const int key = cell_key(xn, P) + P.cbase;
            a.pxout[g] = xn;
            a.puout[g] = un;
            a.pidout[g] = idi;
            a.keyout[g] = key;
            a.rankout[g] = atomicAdd(&a.count[key], 1);
            if (a.pos_out && (unsigned)idi < (unsigned)P.N) a.pos_out[P.pbase + idi] = g;
            bad |= !finite2(xn) || !finite2(un);
            if (SKIN && a.moved && moved_too_far(P, a, g, xi, xn, rebuilt)) atomicOr(a.moved, 1);
        }
        if (bad) atomicOr(a.status, kStatusNonFinite);
        return;
    }
    const float2 un = make_float2(fmaf(P.h, fx, v.x), fmaf(P.h, fy, v.y));
    const float2 xn = make_float2(drift_wrap(xi.x, un.x, P), drift_wrap(xi.y, un.y, P));
    const int key = cell_key(xn, P) + P.cbase;
    const int rank = atomicAdd(&a.count[key], 1);
    a.xout[g] = xn;
    a.uout[g] = un;
    a.idout[g] = idi;
    a.keyout[g] = key;
    a.rankout[g] = rank;
    if (a.pos_out && (unsigned)idi < (unsigned)P.N) a.pos_out[P.pbase + idi] = g;
    if (!finite2(xn) || !finite2(un)) atomicOr(a.status, kStatusNonFinite);
    if (SKIN && a.moved && moved_too_far(P, a, g, xi, xn, rebuilt)) atomicOr(a.moved, 1);
}

// ---- wavefront helpers ----------------------------------------------------------

__device__ __forceinline__ int wave_scan_excl(int v, int& total) {
    const int lane = threadIdx.x & (kWave - 1);
    int incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
    }
    total = __shfl(incl, kWave - 1, kWave);
    return incl - v;
}

// Inclusive prefix sum and prefix maximum over the 64 lanes with DPP lane
// moves (no LDS round trip): within rows of 16 lanes by shifts of 1, 2, 4 and
// 8, then each row combines the last lane of the rows before it (row_bcast of
// lanes 15 and 31).  The shifts set bound_ctrl: a lane whose source lies
// before the start of its row reads 0, which must be the identity of the
// operation; every lane is written, so each shift step is one DPP-sourced add
// or max.  The broadcasts write only the rows of their mask; the other rows
// keep the combined value's 0 operand, the identity again.
__device__ __forceinline__ int wave_incl_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// The maximum's identity is INT_MIN: a lane the DPP move leaves out keeps it
// (no bound_ctrl), so every step folds into one DPP-sourced max as well.
__device__ __forceinline__ int wave_incl_max(int v) {
    constexpr int kLow = (int)0x80000000u;
    v = max(v, __builtin_amdgcn_update_dpp(kLow, v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(kLow, v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(kLow, v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(kLow, v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(kLow, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(kLow, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return v;
}

// Exclusive prefix sum over the lanes; total = the sum of all 64.  The
// exclusive value is the inclusive one of the lane before (wave_shr:1, lane 0
// reads 0), which keeps each shift step of the inclusive scan a single
// DPP-sourced add (written as incl - v, the compiler rebuilds the difference
// from the shifted values and keeps every one of them).
__device__ __forceinline__ int wave_excl_sum(int v, int& total) {
    const int incl = wave_incl_sum(v);
    total = __builtin_amdgcn_readlane(incl, kWave - 1);
    return __builtin_amdgcn_update_dpp(0, incl, 0x138, 0xf, 0xf, true);  // wave_shr:1
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}

// lanes below this one whose bit is set in mask
__device__ __forceinline__ int lanes_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Local cell lc -> (ly, lx) on a local grid W cells wide, by multiply-shift
// (exact for lc < 128 and W <= 10, wmul = ceil(2^16 / W)); the operands are
// far below 2^24, so the 24-bit multiplies (full rate) give the exact products.
__device__ __forceinline__ void local_xy(int lc, int wmul, int W, int& ly, int& lx) {
    ly = (int)(__umul24((unsigned)lc, (unsigned)wmul) >> 16);
    lx = lc - (int)__umul24((unsigned)ly, (unsigned)W);
}

// Cell origin and size of tile t (row-major tiles of tile_x x tile_y cells).
struct TileGeom {
    int cx0, cy0, tw, th;
};

__device__ __forceinline__ TileGeom tile_geom(const DevParams& P, int t) {
    TileGeom g;
    const int ty = (int)(((double)t + 0.5) * P.inv_ntx), tx = t - ty * P.ntx;
    g.cx0 = tx * P.tile_x;
    g.cy0 = ty * P.tile_y;
    g.tw = min(P.tile_x, P.nc - g.cx0);
    g.th = min(P.tile_y, P.nc - g.cy0);
    return g;
}

// Fixed-order sum of the per-lane partials of a 64-lane tile into red[3 t].
__device__ __forceinline__ void tile_reduce(const PairArgs& a, int t, double rv[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) rv[k] += __shfl_down(rv[k], o, kWave);
    }
    if (threadIdx.x == 0) {
        a.red[3 * t + 0] = rv[0];
        a.red[3 * t + 1] = rv[1];
        a.red[3 * t + 2] = rv[2];
    }
}

// Phase B of the pair kernel: the forces of the kept pairs s_pair[0 .. E), added
// in fixed point to the tile particles (the first of each pair, and the second
// if it is in the tile).  Returns whether a force was not finite.
template <bool WEXP>
__device__ __forceinline__ bool pair_sums(const DevParams& P, uint32_t step, bool edge, int E,
                                          const unsigned short* s_pair, const float4* s_rec,
                                          const float2* s_u, long long (*s_acc)[2]) {
    bool bad = false;
    for (int e = threadIdx.x; e < E; e += kWave) {
        const int w = s_pair[e];
        const int so = w >> 8, j = w & 0xFF;
        const float4 ro = s_rec[so], rj = s_rec[j];
        const int k = __float_as_int(ro.w);
        const float dx = edge ? minimg_sub(ro.x, rj.x, P) : ro.x - rj.x;
        const float dy = edge ? minimg_sub(ro.y, rj.y, P) : ro.y - rj.y;
        float fx = 0.f, fy = 0.f;
        add_pair_force<WEXP>(P, dx, dy, cutoff_gap(P, dx, dy), fmaf(dx, dx, dy * dy), s_u[so], s_u[j],
                             __float_as_int(ro.z), __float_as_int(rj.z), step, fx, fy);
        bad |= !(__builtin_isfinite(fx) && __builtin_isfinite(fy));
        const long long qx = to_fixed(fx), qy = to_fixed(fy);
        atomicAdd((unsigned long long*)&s_acc[k][0], (unsigned long long)qx);
        atomicAdd((unsigned long long*)&s_acc[k][1], (unsigned long long)qy);
        const int tj = __float_as_int(rj.w);
        if (tj != 0xFF) {
            atomicAdd((unsigned long long*)&s_acc[tj][0], (unsigned long long)(-qx));
            atomicAdd((unsigned long long*)&s_acc[tj][1], (unsigned long long)(-qy));
        }
    }
    return bad;
}

// The fused pair / agent / integrator kernel: one 64-lane wavefront per tile of
// up to kTileMax x kTileMax cells, the tile and a one-cell halo staged in LDS.
// On a step that rebuilds the cell list (every step without a Verlet skin):
//   S  stage: cell counts from cell_start (one scan gives the staged and the
//      tile offsets of every local cell); each staged particle is gathered
//      through src and placed at its rank by id within its cell, so the LDS
//      order is the canonical (cell, id) order;
//   A  every tile particle tests the staged particles of its half stencil and
//      keeps a pair if the other particle is in the halo or comes later in the
//      canonical order, so each pair within the tile is kept once; kept pairs
//      are compacted by ballot; the bonded partner is recorded.  With a skin,
//      the pairs closer than r_c + skin also go to the tile's record.
// On a step between rebuilds (Verlet skin), instead:
//   L  the staged set is read back from the tile's record (the data already
//      sits in the order of the rebuild), and only the recorded pairs are
//      tested;
// and then on every step:
//   B  one force evaluation per kept pair (Eqs. 2.2-2.4), added in fixed point
//      to the first particle and subtracted from the second (Newton's third
//      law) with LDS integer atomics - exact, so the order does not matter;
//   C  every tile particle adds its agent forces and finishes the step.
// A tile that overflows an LDS capacity (CAP staged particles, TP tile
// particles, ECAP kept pairs) is left to k_pair_overflow (returns false).
// SKIN compiles the Verlet-skin code (records, list steps, displacement test)
// in; without it the kernel carries none of it.  BATCH: the tiles of all
// replicas of a batch form one launch; each wavefront reads its replica's
// parameters from a.reps (the kernel argument P is then unused).
template <int MODE, bool SKIN, bool BATCH, int CAP, int TP, int ECAP>
__device__ __forceinline__ bool pair_tile(DevParams P, PairArgs a, int reduce, int gtile) {
    constexpr int kItemsT = CAP / kWave;  // staged particles per lane
    static_assert(CAP % kWave == 0 && CAP <= 255 && TP <= 255, "tile capacities");
    __shared__ unsigned char s_ofs[kLocMax + 1];  // first staged index of each local cell
    __shared__ int s_gbeg[kLocMax];          // first global slot of each local cell
    __shared__ unsigned char s_tofs[kLocMax];  // first tile index of each local cell
    __shared__ unsigned char s_lcell[CAP];  // local cell of each staged index
    __shared__ float4 s_rec[CAP];           // x, y, id, tile index (0xFF: halo)
    __shared__ float2 s_u[CAP];
    __shared__ int s_slot[SKIN ? CAP : 1];  // global slot of each staged index (skin only)
    __shared__ unsigned char s_tslot[TP];   // tile index -> staged index
    __shared__ unsigned char s_partner[TP]; // tile index -> staged index of the partner
    __shared__ unsigned short s_pair[ECAP]; // kept pair: staged index of the tile particle << 8 | other
    // one buffer, three lifetimes: ids in arrival order while staging, the
    // candidate list of phase A, fixed-point force sums after
    constexpr int kPhaseBytes = TP * 16;
    static_assert(kPhaseBytes >= CAP * 4, "phase buffer too small");
    __shared__ __align__(16) unsigned char s_phase[kPhaseBytes];
    int* s_tmpid = reinterpret_cast<int*>(s_phase);                       // [CAP]
    constexpr int kCand = kPhaseBytes / 2;  // candidate pairs of phase A
    long long (*s_acc)[2] = reinterpret_cast<long long (*)[2]>(s_phase);  // [TP][2]

    if constexpr (BATCH) {
        P = a.reps[a.tile_rep[gtile]];
        a.cs += P.cbase;
    }
    const int tile = BATCH ? gtile - P.tbase : gtile;
    const TileGeom G = tile_geom(P, tile);
    const int cx0 = G.cx0, cy0 = G.cy0, tw = G.tw, th = G.th;
    const int W = tw + 2, nloc = W * (th + 2);
    // local cell -> (lx, ly) by multiply-shift: exact for lc < 128 and W <= 10
    const int wmul = (cx0 + tw == P.nc) ? P.wmul_last : P.wmul_full;
    const bool edge = (cx0 == 0) || (cx0 + tw >= P.nc) || (cy0 == 0) || (cy0 + th >= P.nc);
    const int lane = threadIdx.x;
    const bool rebuild = !SKIN || (MODE == MODE_FORCES) || a.rebuild == nullptr || *a.rebuild != 0;
    const bool keep_list = SKIN && MODE != MODE_FORCES;
    TileRec* R = SKIN ? reinterpret_cast<TileRec*>(a.rec + (size_t)tile * kRecStride) : nullptr;
    if (a.count_clear) {  // the counters this step's binning consumed: this tile's cells
        const int row = lane >> 3, col = lane & 7;  // tile sides <= kTileMax = 8
        if (col < tw && row < th) a.count_clear[P.cbase + (cy0 + row) * P.nc + cx0 + col] = 0;
    }

    int ntile = 0, E = 0;
    bool ok = false;
    if (rebuild) {
        // ---- S1: counts of the two local cells 2*lane and 2*lane + 1
        int cnt[2] = {0, 0};
        bool tcell[2] = {false, false};
        bool big = false;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int lc = 2 * lane + h;
            if (lc < nloc) {
                int ly, lx;
                local_xy(lc, wmul, W, ly, lx);
                // the periodic wrap only matters for tiles at the box edge
                const int gy = cy0 - 1 + ly, gx = cx0 - 1 + lx;
                const int c = edge ? (int)__umul24((unsigned)wrap_cell(gy, P.nc), (unsigned)P.nc) +
                                         wrap_cell(gx, P.nc)
                                   : (int)__umul24((unsigned)gy, (unsigned)P.nc) + gx;
                const int b = a.cs[c];
                const int n = a.cs[c + 1] - b;
                s_gbeg[lc] = b;
                big |= (n > CAP) || (n < 0);
                cnt[h] = min(max(n, 0), CAP);
                tcell[h] = (lx >= 1 && lx <= tw && ly >= 1 && ly <= th);
            }
        }
        // staged counts in the low 16 bits, tile counts in the high 16 (each <= 100 * CAP)
        const int v0 = cnt[0] + (tcell[0] ? cnt[0] << 16 : 0);
        const int v1 = cnt[1] + (tcell[1] ? cnt[1] << 16 : 0);
        int tot;
        const int ex = wave_excl_sum(v0 + v1, tot);
        const int total = tot & 0xFFFF;
        ntile = tot >> 16;
        const bool fits = !__any(big) && total <= CAP && ntile <= TP;
        // (offsets are only used when the tile fits, i.e. below CAP <= 255)
        if (2 * lane < nloc) {
            s_ofs[2 * lane] = (unsigned char)(ex & 0xFF);
            s_tofs[2 * lane] = (unsigned char)min(ex >> 16, 255);
        }
        if (2 * lane + 1 < nloc) {
            s_ofs[2 * lane + 1] = (unsigned char)((ex + v0) & 0xFF);
            s_tofs[2 * lane + 1] = (unsigned char)min((ex + v0) >> 16, 255);
        }
        if (lane == 0) s_ofs[nloc] = (unsigned char)(total & 0xFF);
        // S2 (first half): every staged index is "no cell start" (0xFF) ...
        for (int q = lane; q < CAP; q += kWave) s_lcell[q] = 0xFF;
        __syncthreads();

        if (fits) {
            // ---- S2: staged index -> local cell.  ... except the first staged
            // index of each non-empty cell, which is marked with its cell; cells
            // follow each other in staged order, so the running maximum of the
            // marks is the cell of every staged index.
            if (cnt[0] > 0) s_lcell[ex & 0xFF] = (unsigned char)(2 * lane);
            if (cnt[1] > 0) s_lcell[(ex + v0) & 0xFF] = (unsigned char)(2 * lane + 1);
            __syncthreads();
            // ---- S3: gather in arrival order, by the lane that found the cell
            // (every slot load is issued before the loads that depend on it)
            float2 xq[kItemsT], uq[kItemsT];
            int idq[kItemsT], lcq[kItemsT], pq[kItemsT];
            {
                int carry = -1;
#pragma unroll
                for (int r = 0; r < kItemsT; ++r) {
                    const int q = r * kWave + lane;
                    const int m = s_lcell[q];
                    lcq[r] = max(wave_incl_max(m == 0xFF ? -1 : m), carry);
                    carry = __builtin_amdgcn_readlane(lcq[r], kWave - 1);
                }
            }
#pragma unroll
            for (int r = 0; r < kItemsT; ++r) {
                const int q = r * kWave + lane;
                pq[r] = P.pbase;
                if (q < total) {
                    const int lc = lcq[r];
                    s_lcell[q] = (unsigned char)lc;
                    pq[r] = a.src[s_gbeg[lc] + (q - s_ofs[lc])];
                }
            }
#pragma unroll
            for (int r = 0; r < kItemsT; ++r) {
                const int q = r * kWave + lane;
                idq[r] = 0;
                xq[r] = make_float2(0.f, 0.f);
                uq[r] = make_float2(0.f, 0.f);
                if (q < total) {
                    int p = pq[r];
                    if ((unsigned)(p - P.pbase) >= (unsigned)P.N) {  // outside this system
                        atomicOr(a.status, kStatusBinning);
                        p = P.pbase;
                    }
                    idq[r] = a.idin[p];
                    xq[r] = a.xin[p];
                    uq[r] = a.uin[p];
                    s_tmpid[q] = idq[r];
                }
            }
            __syncthreads();
            // ---- S4: place every particle at its rank by id within its cell
#pragma unroll
            for (int r = 0; r < kItemsT; ++r) {
                const int q = r * kWave + lane;
                if (q < total) {
                    const int lc = lcq[r];
                    const int b = s_ofs[lc], e = s_ofs[lc + 1];
                    int rank = 0;
                    for (int t = b; t < e; ++t) rank += (s_tmpid[t] < idq[r]) ? 1 : 0;
                    const int qs = b + rank;
                    int ly, lx;
                local_xy(lc, wmul, W, ly, lx);
                    int ti = 0xFF;
                    if (lx >= 1 && lx <= tw && ly >= 1 && ly <= th) {
                        ti = s_tofs[lc] + rank;
                        s_tslot[ti] = (unsigned char)qs;
                        s_partner[ti] = 0xFF;
                    }
                    const int g = s_gbeg[lc] + rank;
                    s_rec[qs] = make_float4(xq[r].x, xq[r].y, __int_as_float(idq[r]), __int_as_float(ti));
                    s_u[qs] = uq[r];
                    if constexpr (SKIN) s_slot[qs] = g;
                    if (keep_list) {
                        R->slot[qs] = g;
                        R->tix[qs] = (unsigned char)ti;
                    }
                }
            }
            __syncthreads();
            // ---- A: the candidates of the tile's half stencil, tested as one
            // flat list.  A tile particle's candidates are up to three ranges of
            // staged indices:
            //   own row: the rest of the own cell and the cell to the right (from
            //            the left neighbour on when that is a halo cell);
            //   row above: the three cells of the stencil;
            //   row below: its three cells where they include halo cells (first
            //            tile row, first or last tile column).
            // A1: each tile particle finds its ranges, and a wavefront scan of
            // their lengths gives its offset in the list; A2: it writes its
            // candidates there (staged index of the particle << 8 | staged index of
            // the candidate); A3: the list is tested 64 candidates at a time, every
            // lane busy.  A pair is kept if the other particle is in the halo or
            // later in the canonical order, so each pair inside the tile is kept
            // once and each tile-halo pair once, from the tile side.  Kept pairs
            // are compacted by ballot; a bonded pair records each member as the
            // other's partner.  The list lives in the staging buffer (free until
            // the force sums).
            unsigned short* s_cand = reinterpret_cast<unsigned short*>(s_phase);  // [kCand]
            const int rounds = (ntile + kWave - 1) / kWave;
            int T = 0;
            for (int r = 0; r < rounds; ++r) {
                const int k = r * kWave + lane;
                int si = 0, b0 = 0, n0 = 0, bu = 0, nu = 0, bd = 0, nd = 0;
                if (k < ntile) {
                    si = s_tslot[k];
                    const int lc = s_lcell[si];
                    int ly, lx;
                local_xy(lc, wmul, W, ly, lx);
                    const int me = ly * W + lx - 1, up = me + W;
                    b0 = (lx == 1) ? s_ofs[me] : si + 1;
                    n0 = s_ofs[me + 3] - b0;
                    bu = s_ofs[up];
                    nu = s_ofs[up + 3] - bu;
                    if (ly == 1 || lx == 1 || lx == tw) {
                        const int dn = me - W;
                        bd = s_ofs[dn];
                        nd = s_ofs[dn + 3] - bd;
                    }
                }
                int tot;
                const int pos = T + wave_excl_sum(n0 + nu + nd, tot);
                if (T + tot <= kCand) {
                    // staged indices are below 256, so (si << 8) | j == (si << 8) + j
                    // (loops of a few trips: kept simple, one 2-byte write each)
                    unsigned short* dst = s_cand + pos;
                    const int w0 = (si << 8) + b0;
#pragma clang loop unroll(disable) vectorize(disable)
                    for (int t = 0; t < n0; ++t) dst[t] = (unsigned short)(w0 + t);
                    dst += n0;
                    const int wu = (si << 8) + bu;
#pragma clang loop unroll(disable) vectorize(disable)
                    for (int t = 0; t < nu; ++t) dst[t] = (unsigned short)(wu + t);
                    dst += nu;
                    const int wd = (si << 8) + bd;
#pragma clang loop unroll(disable) vectorize(disable)
                    for (int t = 0; t < nd; ++t) dst[t] = (unsigned short)(wd + t);
                }
                T += tot;
            }
            __syncthreads();
            const bool fits_cand = T <= kCand;
            int EL = 0;
            if (fits_cand) {
                for (int f0 = 0; f0 < T; f0 += kWave) {
                    const int f = f0 + lane;
                    bool keep = false, lk = false;
                    unsigned short w = 0;
                    if (f < T) {
                        w = s_cand[f];
                        const int si = w >> 8, j = w & 0xFF;
                        const float4 ri = s_rec[si], rj = s_rec[j];
                        const int tj = __float_as_int(rj.w);
                        const bool mine = (tj == 0xFF) || (j > si);
                        const bool isp = mine && ((__float_as_int(ri.z) ^ __float_as_int(rj.z)) == 1);
                        if (isp) {
                            s_partner[__float_as_int(ri.w)] = (unsigned char)j;
                            if (tj != 0xFF) s_partner[tj] = (unsigned char)si;
                        }
                        const float dx = edge ? minimg_sub(ri.x, rj.x, P) : ri.x - rj.x;
                        const float dy = edge ? minimg_sub(ri.y, rj.y, P) : ri.y - rj.y;
                        const float r2 = fmaf(dx, dx, dy * dy);
                        keep = mine && !isp && interacts(cutoff_gap(P, dx, dy), r2);
                        if (keep_list) lk = mine && !isp && r2 > 0.f && r2 < P.list_rc2;
                    }
                    const unsigned long long msk = __ballot(keep);
                    const int nk = __popcll(msk);
                    if (E + nk <= ECAP) {
                        if (keep) s_pair[E + lanes_below(msk)] = w;
                    }
                    E += nk;
                    if (keep_list) {
                        const unsigned long long ml = __ballot(lk);
                        const int nl = __popcll(ml);
                        if (EL + nl <= kLcap) {
                            if (lk) R->pairs[EL + lanes_below(ml)] = w;
                        }
                        EL += nl;
                    }
                }
            }
            __syncthreads();
            ok = fits_cand && (E <= ECAP) && (!keep_list || EL <= kLcap);
            if (keep_list) {
                for (int k = lane; k < ntile; k += kWave) {
                    R->tslot[k] = s_tslot[k];
                    R->partner[k] = s_partner[k];
                }
                if (lane == 0) {
                    R->ntile = ntile;
                    R->total = total;
                    R->nlist = EL;
                    R->valid = ok ? 1 : 0;
                }
            }
        } else if (keep_list && lane == 0) {
            R->valid = 0;
        }
    } else if constexpr (SKIN) {
        // ---- L: between rebuilds: the staged set and the pair list of the record
        const int valid = R->valid;
        if (valid) {
            ntile = min(R->ntile, TP);
            const int total = min(R->total, CAP), nlist = min(R->nlist, kLcap);
            for (int q = lane; q < total; q += kWave) {
                int g = R->slot[q];
                if ((unsigned)(g - P.pbase) >= (unsigned)P.N) {
                    atomicOr(a.status, kStatusBinning);
                    g = P.pbase;
                }
                const float2 xg = a.xin[g];
                s_rec[q] = make_float4(xg.x, xg.y, __int_as_float(a.idin[g]), __int_as_float((int)R->tix[q]));
                s_u[q] = a.uin[g];
                s_slot[q] = g;
            }
            for (int k = lane; k < ntile; k += kWave) {
                s_tslot[k] = R->tslot[k];
                s_partner[k] = R->partner[k];
            }
            __syncthreads();
            for (int e0 = 0; e0 < nlist; e0 += kWave) {
                const int e = e0 + lane;
                bool keep = false;
                unsigned short w = 0;
                if (e < nlist) {
                    w = R->pairs[e];
                    const float4 ri = s_rec[w >> 8], rj = s_rec[w & 0xFF];
                    const float dx = edge ? minimg_sub(ri.x, rj.x, P) : ri.x - rj.x;
                    const float dy = edge ? minimg_sub(ri.y, rj.y, P) : ri.y - rj.y;
                    keep = interacts(cutoff_gap(P, dx, dy), fmaf(dx, dx, dy * dy));
                }
                const unsigned long long msk = __ballot(keep);
                const int nk = __popcll(msk);
                if (E + nk <= ECAP) {
                    if (keep) s_pair[E + lanes_below(msk)] = w;
                }
                E += nk;
            }
            __syncthreads();
            ok = E <= ECAP;
        }
    }

    double rv[3] = {0.0, 0.0, 0.0};
    if (!ok) return false;  // over an LDS capacity
    for (int k = lane; k < ntile; k += kWave) {
        s_acc[k][0] = 0;
        s_acc[k][1] = 0;
    }
    __syncthreads();
    // ---- B: one force per kept pair, exact fixed-point sums (the weight
    // exponent is tested once, outside the loop)
    const bool bad = P.w_half == 1.0f
        ? pair_sums<false>(P, a.step, edge, E, s_pair, s_rec, s_u, s_acc)
        : pair_sums<true>(P, a.step, edge, E, s_pair, s_rec, s_u, s_acc);
    if (bad) atomicOr(a.status, kStatusNonFinite);
    __syncthreads();

    // ---- C: agent forces and integration, tile particles in canonical order
    // (the parameters and pointers this phase uses, read again: see
    // kernel_arg_again; a batch's parameters come from its replica table)
    if constexpr (!BATCH) P = kernel_arg_again<DevParams>(0);
    a = kernel_arg_again<PairArgs>(kArgOffPairArgs);
    const int rounds = (ntile + kWave - 1) / kWave;
    for (int r = 0; r < rounds; ++r) {
        const int k = r * kWave + lane;
        if (k >= ntile) continue;
        const int si = s_tslot[k];
        const float4 ri = s_rec[si];
        const float2 xi = make_float2(ri.x, ri.y), ui = s_u[si];
        const int idi = __float_as_int(ri.z);
        float fx = from_fixed(s_acc[k][0]), fy = from_fixed(s_acc[k][1]);
        const int jp = s_partner[k];
        if (jp != 0xFF) {
            const float4 rp = s_rec[jp];
            add_agent_force(P, xi, make_float2(rp.x, rp.y), ui, idi, fx, fy);
        } else if (P.far_bond) {
            // the partner lies beyond the staged cells: read it by id
            int pp = a.pos_of_id[P.pbase + (idi ^ 1)];
            if ((unsigned)(pp - P.pbase) >= (unsigned)P.N) {
                atomicOr(a.status, kStatusBinning);
                pp = P.pbase;
            }
            add_agent_force(P, xi, a.xin[pp], ui, idi, fx, fy);
        } else {
            atomicOr(a.status, kStatusBond);
            fx -= P.gamma_s * ui.x;
            fy -= P.gamma_s * ui.y;
        }
        int g;
        if constexpr (SKIN) {
            g = s_slot[si];
        } else {
            const int lc = s_lcell[si];
            g = s_gbeg[lc] + (si - s_ofs[lc]);
        }
        // inconsistent cell data (flagged when the gather found an index outside
        // the system) must not turn into a store outside the system's slots
        g = min(max(g, P.pbase), P.pbase + P.N - 1);
        finish_particle<MODE, SKIN>(P, a, g, xi, ui, idi, fx, fy, rv, reduce != 0, rebuild);
    }
    if (reduce) tile_reduce(a, gtile, rv);
    return true;
}

// The fast pair kernel: one wavefront per tile with the small capacities; a
// tile over one of them is listed for k_pair_overflow.
template <int MODE, bool SKIN, bool BATCH>
__global__ __launch_bounds__(kWave) void k_pair(DevParams P, PairArgs a, int reduce) {
    // XCD-aware tile order: blocks are dealt round-robin to the 8 XCDs, so give
    // each XCD a contiguous band of tiles (neighbouring halos share its L2).
    const int nt = BATCH ? a.nt_total : P.ntx * P.nty;
    const int bid = blockIdx.x;
    int gtile = bid;
    if (a.tile_order == 0) {
        const int xcd = bid & 7, kk = bid >> 3;
        const int per = nt >> 3, rem = nt & 7;
        gtile = xcd * per + min(xcd, rem) + kk;
    }
    if (a.step_base) a.step += *a.step_base;
    if (!pair_tile<MODE, SKIN, BATCH, kCap, kTP, kEcap>(P, a, reduce, gtile) && threadIdx.x == 0)
        a.ovf_list[atomicAdd(a.ovf_count, 1)] = gtile;
}

// Slow path for a tile that overflows an LDS capacity (dense clusters), one
// 64-lane wavefront per tile.  The members of the tile's cells are numbered
// in canonical order (cells in turn, each cell's members by id; a scan of the
// cell counts gives each cell's first number) and dealt to the lanes in that
// order, so that both sparse tiles (many cells, few members each) and dense
// ones (one cell, many members) keep the lanes busy, and every lane's velocity
// sums run over the same particles in the same order from run to run.  A
// first pass gives each member, taken in slot order, its canonical number (its
// cell's first number plus the members of the cell with a smaller id) and
// records the slot under that number in LDS, kOvfWindow numbers at a time.
// Each member sums its pairs over the full 3x3 stencil straight from global
// memory.  The sums are fixed point, so the result is bitwise the fast path's.
// REBUILT is a template parameter, not a runtime flag: the lanes' loops here
// diverge, and a wave-uniform flag tested inside them was compiled into a lane
// mask taken under one loop's exec mask and reused under another's, which sent
// some lanes down the wrong side of the test.  The velocity sums are always
// accumulated (the caller decides whether to store them).
constexpr int kOvfWindow = 2048;
// Candidates (and cell members) the global path loads at a time per lane.
constexpr int kGlobBatch = 4;
template <int MODE, bool REBUILT>
__device__ void tile_global(const DevParams& P, const PairArgs& a, int cx0, int cy0, int tw,
                            int th, double rv[3]) {
    // between rebuilds (Verlet skin) the data already sits in the cell order of
    // the last rebuild: slot g holds particle g
    __shared__ int s_pre[kTileMax * kTileMax + 1];  // first member number of each tile cell
    __shared__ int s_beg[kTileMax * kTileMax];      // its first global slot
    __shared__ int s_slot[kOvfWindow];              // global slot of canonical number w0 + i
    const int nc = P.nc, ncell = tw * th, lane = threadIdx.x;
    int cnt = 0;
    if (lane < ncell) {
        const int c = (cy0 + lane / tw) * nc + cx0 + lane % tw;
        const int b = a.cs[c];
        cnt = max(a.cs[c + 1] - b, 0);
        s_beg[lane] = b;
    }
    int tot;
    const int ex = wave_scan_excl(cnt, tot);
    if (lane < ncell) s_pre[lane] = ex;
    if (lane == 0) s_pre[ncell] = tot;
    __syncthreads();
    // the tile cell of member number t: the last with s_pre <= t (not empty)
    auto cell_of = [&](int t) {
        int lo = 0, hi = ncell - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_pre[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    };
    for (int w0 = 0; w0 < tot; w0 += kOvfWindow) {
        const int w1 = min(tot, w0 + kOvfWindow);
        // canonical numbers of the members, taken in slot order
        for (int t = lane; t < tot; t += kWave) {
            const int lo = cell_of(t);
            const int b = s_beg[lo], e = b + (s_pre[lo + 1] - s_pre[lo]);
            const int g = b + (t - s_pre[lo]);
            int p = REBUILT ? a.src[g] : g;
            if ((unsigned)(p - P.pbase) >= (unsigned)P.N) {  // outside this system
                atomicOr(a.status, kStatusBinning);
                p = P.pbase;
            }
            const int idi = a.idin[p];
            int r = 0;  // members of the cell with a smaller id (ids are distinct)
            for (int g1 = b; g1 < e; g1 += kGlobBatch) {
                // a batch of members at a time: their loads are independent
                int pv[kGlobBatch];
#pragma unroll
                for (int k = 0; k < kGlobBatch; ++k) {
                    int p1 = g1 + k < e ? (REBUILT ? a.src[g1 + k] : g1 + k) : P.pbase;
                    if ((unsigned)(p1 - P.pbase) >= (unsigned)P.N) p1 = P.pbase;
                    pv[k] = p1;
                }
#pragma unroll
                for (int k = 0; k < kGlobBatch; ++k)
                    r += (g1 + k < e && a.idin[pv[k]] < idi) ? 1 : 0;
            }
            const int tc = s_pre[lo] + r;
            if (tc >= w0 && tc < w1) s_slot[tc - w0] = g;
        }
        __syncthreads();
        for (int tc = w0 + lane; tc < w1; tc += kWave) {
            const int lo = cell_of(tc);
            const int gx = cx0 + lo % tw, gy = cy0 + lo / tw;
            const int b = s_beg[lo], e = b + (s_pre[lo + 1] - s_pre[lo]);
            const int r = tc - s_pre[lo];  // canonical rank in the cell: output slot b + r
            int g = s_slot[tc - w0];
            g = (g >= b && g < e) ? g : b;  // a valid slot of the cell even on corrupt input
            int p = REBUILT ? a.src[g] : g;
            if ((unsigned)(p - P.pbase) >= (unsigned)P.N) p = P.pbase;
            const int idi = a.idin[p];
            const float2 xi = a.xin[p], ui = a.uin[p];
            const int pid = idi ^ 1;
            long long qx = 0, qy = 0;
            bool found = false, bad = false;
            float2 xpart = xi;
            for (int oy = -1; oy <= 1; ++oy) {
                for (int ox = -1; ox <= 1; ++ox) {
                    const int c2 = wrap_cell(gy + oy, nc) * nc + wrap_cell(gx + ox, nc);
                    const int b2 = a.cs[c2], e2 = a.cs[c2 + 1];
                    for (int g2 = b2; g2 < e2; g2 += kGlobBatch) {
                        // a batch of candidates at a time, in slot order: the
                        // loads of a batch are independent and overlap (the
                        // fixed-point sums do not depend on the order anyway)
                        int qv[kGlobBatch], idv[kGlobBatch];
                        float2 xv[kGlobBatch], uv[kGlobBatch];
#pragma unroll
                        for (int k = 0; k < kGlobBatch; ++k) {
                            int q = g2 + k < e2 ? (REBUILT ? a.src[g2 + k] : g2 + k) : P.pbase;
                            if ((unsigned)(q - P.pbase) >= (unsigned)P.N) q = P.pbase;
                            qv[k] = q;
                        }
#pragma unroll
                        for (int k = 0; k < kGlobBatch; ++k) {
                            idv[k] = a.idin[qv[k]];
                            xv[k] = a.xin[qv[k]];
                            uv[k] = a.uin[qv[k]];
                        }
#pragma unroll
                        for (int k = 0; k < kGlobBatch; ++k) {
                            if (g2 + k >= e2 || g2 + k == g) continue;
                            const int idj = idv[k];
                            const float2 xj = xv[k];
                            if (idj == pid) {
                                found = true;
                                xpart = xj;
                                continue;
                            }
                            const float dx = minimg_sub(xi.x, xj.x, P);
                            const float dy = minimg_sub(xi.y, xj.y, P);
                            const float gap = cutoff_gap(P, dx, dy);
                            const float r2 = fmaf(dx, dx, dy * dy);
                            if (interacts(gap, r2)) {
                                float fx = 0.f, fy = 0.f;
                                add_pair_force(P, dx, dy, gap, r2, ui, uv[k], idi, idj, a.step, fx, fy);
                                bad |= !(__builtin_isfinite(fx) && __builtin_isfinite(fy));
                                qx += to_fixed(fx);
                                qy += to_fixed(fy);
                            }
                        }
                    }
                }
            }
            if (bad) atomicOr(a.status, kStatusNonFinite);
            float fx = from_fixed(qx), fy = from_fixed(qy);
            if (!found && P.far_bond) {  // the partner lies beyond the stencil: by id
                int pp = a.pos_of_id[P.pbase + pid];
                if ((unsigned)(pp - P.pbase) >= (unsigned)P.N) {
                    atomicOr(a.status, kStatusBinning);
                    pp = P.pbase;
                }
                xpart = a.xin[pp];
                found = true;
            }
            if (found) {
                add_agent_force(P, xi, xpart, ui, idi, fx, fy);
            } else {
                atomicOr(a.status, kStatusBond);
                fx -= P.gamma_s * ui.x;
                fy -= P.gamma_s * ui.y;
            }
            finish_particle<MODE, true>(P, a, b + r, xi, ui, idi, fx, fy, rv, true, REBUILT);
        }
        __syncthreads();  // s_slot is rewritten for the next window, s_pre for the next tile
    }
}

// The tiles k_pair left over, one 64-lane wavefront per listed tile (same
// results bit for bit).  Launched right after k_pair with a fixed grid; with an
// empty list every wavefront exits at once.  RETRY (handles without a Verlet
// skin): a listed tile is first run through the tile body with the large LDS
// capacities, which holds tiles up to about twice the usual load (the uneven
// cells of a random start, denser systems); only tiles over those go to the
// global-memory path.
constexpr int kCapBig = 192, kTPBig = 128, kEcapBig = 384;

template <int MODE, bool REBUILT, bool BATCH, bool RETRY>
__device__ __forceinline__ void overflow_tiles(const DevParams& P0, const PairArgs& a0, int n,
                                               int reduce) {
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int gtile = a0.ovf_list[i];
        if constexpr (RETRY) {
            if (pair_tile<MODE, false, BATCH, kCapBig, kTPBig, kEcapBig>(P0, a0, reduce, gtile)) continue;
        }
        DevParams P = P0;
        PairArgs a = a0;
        if constexpr (BATCH) {
            P = a.reps[a.tile_rep[gtile]];
            a.cs += P.cbase;
        }
        const TileGeom G = tile_geom(P, BATCH ? gtile - P.tbase : gtile);
        double rv[3] = {0.0, 0.0, 0.0};
        tile_global<MODE, REBUILT>(P, a, G.cx0, G.cy0, G.tw, G.th, rv);
        if (reduce) tile_reduce(a, gtile, rv);
    }
}

template <int MODE, bool BATCH, bool RETRY>
__global__ __launch_bounds__(kWave) void k_pair_overflow(DevParams P, PairArgs a, int reduce) {
    const int n = *a.ovf_count;
    if (a.step_base) a.step += *a.step_base;
    if (MODE == MODE_FORCES || a.rebuild == nullptr || *a.rebuild != 0)
        overflow_tiles<MODE, true, BATCH, RETRY>(P, a, n, reduce);
    else
        overflow_tiles<MODE, false, BATCH, false>(P, a, n, reduce);
}

// ---- binning ------------------------------------------------------------------

// Input state in id order -> buffer (x wrapped into the box, v, id) plus cell
// key and atomic rank.
__global__ void k_load_input(DevParams P, const float2* __restrict__ x, const float2* __restrict__ v,
                             float2* xo, float2* uo, int* ido, int* key, int* rank, int* count,
                             unsigned* status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.N) return;
    const float2 xi = x[i], vi = v[i];
    if (!finite2(xi) || !finite2(vi)) atomicOr(status, kStatusNonFinite);
    const float2 xw = make_float2(drift_wrap(xi.x, 0.f, P), drift_wrap(xi.y, 0.f, P));
    const int k = cell_key(xw, P) + P.cbase;
    xo[i] = xw;
    uo[i] = vi;
    ido[i] = i;
    key[i] = k;
    rank[i] = atomicAdd(&count[k], 1);
}

// Positions (any order) -> cell key and atomic rank.
__global__ void k_key_rank(DevParams P, const float2* __restrict__ x, int* key, int* rank,
                           int* count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.N) return;
    const int k = cell_key(x[i], P) + P.cbase;
    key[i] = k;
    rank[i] = atomicAdd(&count[k], 1);
}

// Exclusive scan of the per-cell counts -> cell_start in one pass over chunks
// of 4 ROWS kScanThreads cells (decoupled look-back: Merrill & Garland,
// "Single-pass parallel prefix scan with decoupled look-back", NVIDIA tech.
// report 2016).
// Each block draws a ticket from a counter, so the chunks are taken in order
// and a block only ever waits for chunks taken before its own, whose blocks are
// already running.  A block publishes its chunk's sum at once, then its
// prefix: it adds up the sums published to its left until it meets a chunk
// whose inclusive prefix is known, publishes its own inclusive prefix and
// writes its cell_start values.  The last block writes the grand total to
// cell_start[n] and resets the ticket counter.  With `clear` the block also
// zeroes its counts for the next binning (the stepping path leaves that to the
// pair kernel, tile by tile).
//
// A chunk is ROWS rows of kScanThreads groups of 4 cells in row-major order,
// thread t holding group t of every row: each load and store of a wavefront
// covers 1 KB of consecutive cells.  The chunks are large (ROWS = 4: a few
// hundred for millions of cells, about one per compute unit; ROWS = 1 below
// kScanSmallCells cells, so that a small grid still spreads over tens of
// blocks) and one wavefront reads kScanWindow descriptors per round of the
// look-back: the blocks run side by side and publish their sums at about the
// same time, so a round that reaches back over every earlier chunk at once
// keeps the look-back to one round trip.
//
// A descriptor is one 64-bit word, written and read whole: bits 0-31 the
// value, bit 32 set when the value is the inclusive prefix (clear: the chunk's
// own sum), bits 33-63 the launch's epoch.  A descriptor of another epoch is
// not yet written in this launch, so no descriptor is ever cleared; the
// counter word holds the epoch in its high half and the next ticket in its
// low half (all zero at creation: the first launch has epoch 1).  The sums are
// exact integers, so the result is the same as any other order of addition.
// A look-back that waits past kScanSpin polls sets kStatusScan and goes on,
// which ends the kernel in any case.
//
// The launch also clears the pair kernel's tile overflow counter and, with a
// Verlet skin, the displacement flag the coming pair launch sets
// (`moved_clear`) and counts the rebuilds; the scan itself runs only on
// rebuild steps (`rebuild` null: always).
constexpr int kScanThreads = 1024;
constexpr int kScanLook = 4;                    // descriptors per lane and round
constexpr int kScanWindow = kWave * kScanLook;  // chunks per round of the look-back
// grids up to this many cells scan in chunks of one row (at most kScanWindow
// chunks, so one look-back round still reaches the first)
constexpr long long kScanSmallCells = (long long)kScanWindow * kScanThreads * 4;
__host__ __device__ constexpr int scan_rows(long long cells) { return cells <= kScanSmallCells ? 1 : 4; }
constexpr int kScanSpin = 1 << 20;

__device__ __forceinline__ uint64_t scan_desc(uint32_t epoch, bool inclusive, uint32_t v) {
    return ((uint64_t)(epoch & 0x7FFFFFFFu) << 33) | ((uint64_t)inclusive << 32) | v;
}

template <int ROWS>
__global__ __launch_bounds__(kScanThreads) void k_scan(int* count, int n, int clear, int* cs,
                                                       unsigned long long* desc,
                                                       unsigned long long* ticket,
                                                       unsigned* status, int* ovf_count,
                                                       const int* rebuild, int* moved_clear,
                                                       int* rebuilds) {
    constexpr int kWaves = kScanThreads / kWave;
    constexpr int kTile = kScanThreads * 4 * ROWS;  // cells per chunk
    __shared__ int s_wave[ROWS][kWaves];
    __shared__ uint32_t s_ticket[2];
    __shared__ int s_prefix;
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    if (blockIdx.x == 0 && t == 0) {
        *ovf_count = 0;
        if (moved_clear) {
            *moved_clear = 0;
            if (rebuild && *rebuild) atomicAdd(rebuilds, 1);
        }
    }
    if (rebuild && *rebuild == 0) return;
    if (t == 0) {
        const unsigned long long old = atomicAdd(ticket, 1ull);
        s_ticket[0] = (uint32_t)old;
        s_ticket[1] = (uint32_t)(old >> 32) + 1u;
    }
    __syncthreads();
    const int chunk = (int)s_ticket[0];
    const uint32_t epoch = s_ticket[1];
    const uint32_t etag = epoch & 0x7FFFFFFFu;
    if (chunk == (int)gridDim.x - 1 && t == 0)  // every ticket of this launch is taken
        __hip_atomic_store(ticket, (unsigned long long)epoch << 32, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);

    // group t of every row: 4 consecutive cells
    const int base = chunk * kTile;
    int4 v[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        const int c = base + (k * kScanThreads + t) * 4;
        if (c + 4 <= n) {
            v[k] = *reinterpret_cast<const int4*>(count + c);
        } else {  // the ragged end: c + 3 >= n
            v[k] = make_int4(c < n ? count[c] : 0, c + 1 < n ? count[c + 1] : 0,
                             c + 2 < n ? count[c + 2] : 0, 0);
        }
    }
    // exclusive prefix of every group within the chunk
    int ex[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        const int g = (v[k].x + v[k].y) + (v[k].z + v[k].w);
        int incl = g;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += y;
        }
        if (lane == kWave - 1) s_wave[k][w] = incl;
        ex[k] = incl - g;
    }
    __syncthreads();
    int agg = 0;
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        int wofs = 0, row = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) {
            wofs += (q < w) ? s_wave[k][q] : 0;
            row += s_wave[k][q];
        }
        ex[k] += agg + wofs;
        agg += row;
    }

    if (w == 0) {
        if (lane == 0)
            __hip_atomic_store(desc + chunk, scan_desc(epoch, chunk == 0, (uint32_t)agg),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t prefix = 0;
        int p = chunk - 1;  // nearest chunk not yet added
        bool timed_out = false;
        while (p >= 0) {
            // lane l looks at chunks p - kScanLook l - j, j = 0 .. kScanLook - 1
            // (nearest first); left of chunk 0 reads as an inclusive 0
            uint64_t d[kScanLook];
#pragma unroll
            for (int j = 0; j < kScanLook; ++j) {
                const int q = p - kScanLook * lane - j;
                d[j] = (q >= 0) ? __hip_atomic_load(desc + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                : scan_desc(epoch, true, 0u);
            }
            for (int spin = 0;;) {  // poll the ones not yet written in this launch
                bool ready = true;
#pragma unroll
                for (int j = 0; j < kScanLook; ++j) ready = ready && (uint32_t)(d[j] >> 33) == etag;
                if (ready) break;
                if (++spin >= kScanSpin) {
                    timed_out = true;
#pragma unroll
                    for (int j = 0; j < kScanLook; ++j)
                        if ((uint32_t)(d[j] >> 33) != etag) d[j] = scan_desc(epoch, true, 0u);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
#pragma unroll
                for (int j = 0; j < kScanLook; ++j) {
                    const int q = p - kScanLook * lane - j;
                    if ((uint32_t)(d[j] >> 33) != etag)  // q >= 0 here
                        d[j] = __hip_atomic_load(desc + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            // this lane's sum up to and including its nearest inclusive prefix
            uint32_t all = 0, upto = 0;
            bool has = false;
#pragma unroll
            for (int j = 0; j < kScanLook; ++j) {
                all += (uint32_t)d[j];
                if (!has) upto += (uint32_t)d[j];
                has = has || ((d[j] >> 32) & 1u);
            }
            const uint64_t with_incl = __ballot(has);
            uint32_t x = all;
            if (with_incl) {
                const int first = __builtin_ctzll(with_incl);  // nearest lane with one
                x = (lane < first) ? all : (lane == first ? upto : 0u);
            }
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
            prefix += x;
            if (with_incl) break;
            p -= kScanWindow;
        }
        if (__ballot(timed_out) && lane == 0) atomicOr(status, kStatusScan);
        if (lane == 0) {
            if (chunk > 0)
                __hip_atomic_store(desc + chunk, scan_desc(epoch, true, prefix + (uint32_t)agg),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_prefix = (int)prefix;
        }
    }
    __syncthreads();
    const int pre = s_prefix;
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        const int c = base + (k * kScanThreads + t) * 4;
        const int o = pre + ex[k];
        const int4 r = make_int4(o, o + v[k].x, o + v[k].x + v[k].y, o + v[k].x + v[k].y + v[k].z);
        if (c + 4 <= n) {
            *reinterpret_cast<int4*>(cs + c) = r;
            if (clear) *reinterpret_cast<int4*>(count + c) = make_int4(0, 0, 0, 0);
        } else {
            if (c < n) cs[c] = r.x;
            if (c + 1 < n) cs[c + 1] = r.y;
            if (c + 2 < n) cs[c + 2] = r.z;
            if (clear) {
                if (c < n) count[c] = 0;
                if (c + 1 < n) count[c + 1] = 0;
                if (c + 2 < n) count[c + 2] = 0;
            }
        }
    }
    if (chunk == (int)gridDim.x - 1 && t == 0) cs[n] = pre + agg;
}

__global__ void k_scatter(int N, const int* __restrict__ key, const int* __restrict__ rank,
                          const int* __restrict__ cs, int* src, const int* rebuild) {
    if (rebuild && *rebuild == 0) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x)
        src[cs[key[i]] + rank[i]] = i;
}

// Bonds longer than the cell stencil reaches: pos[pbase + id] = index in the
// input buffers of every particle, its replica found by bisection of the
// replicas' first slots (reps null: a single system).  Runs with the binning
// that consumes those buffers (rebuild as for k_scatter).
__global__ void k_pos_of_id(int N, const int* __restrict__ id, const DevParams* __restrict__ reps,
                            int R, int* pos, const int* rebuild) {
    if (rebuild && *rebuild == 0) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        int base = 0;
        if (reps) {
            // a wavefront's lanes hold consecutive indices: bisect once for the
            // first active lane (uniform, so in scalar registers), then each
            // lane steps on past replicas that end before its own index
            const int i0 = __builtin_amdgcn_readfirstlane(i);
            int lo = 0, hi = R - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (reps[mid].pbase <= i0) lo = mid;
                else hi = mid - 1;
            }
            while (lo + 1 < R && reps[lo + 1].pbase <= i) ++lo;
            base = reps[lo].pbase;
        }
        pos[base + id[i]] = i;
    }
}

// Order each cell's slots by particle id.  Cells hold about one particle:
// two or three members are sorted in registers, larger cells in place.
__device__ __forceinline__ void cswap(int& sa, int& ia, int& sb, int& ib) {
    if (ia > ib) {
        const int s0 = sa, i0 = ia;
        sa = sb; ia = ib;
        sb = s0; ib = i0;
    }
}

__global__ void k_cell_sort(int n_cells, const int* __restrict__ cs, int* src,
                            const int* __restrict__ id) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const int b = cs[c], e = cs[c + 1];
    const int n = e - b;
    if (n < 2) return;
    if (n == 2) {
        int s0 = src[b], s1 = src[b + 1];
        int i0 = id[s0], i1 = id[s1];
        if (i0 > i1) {
            src[b] = s1;
            src[b + 1] = s0;
        }
        return;
    }
    if (n == 3) {
        int s0 = src[b], s1 = src[b + 1], s2 = src[b + 2];
        int i0 = id[s0], i1 = id[s1], i2 = id[s2];
        cswap(s0, i0, s1, i1);
        cswap(s1, i1, s2, i2);
        cswap(s0, i0, s1, i1);
        src[b] = s0;
        src[b + 1] = s1;
        src[b + 2] = s2;
        return;
    }
    for (int k = b + 1; k < e; ++k) {
        const int s0 = src[k], i0 = id[s0];
        int m = k - 1;
        while (m >= b && id[src[m]] > i0) {
            src[m + 1] = src[m];
            --m;
        }
        src[m + 1] = s0;
    }
}

// Resume: state in sorted order from the binned input plus a given force (id order).
__global__ void k_gather_state(int N, const int* __restrict__ src, const float2* __restrict__ xi,
                               const float2* __restrict__ ui, const int* __restrict__ idi,
                               const float2* __restrict__ Fin, float2* xo, float2* vo, int* ido,
                               float2* Fo, unsigned* status) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    const int p = src[g];
    const int id = idi[p];
    const float2 F = Fin[id];
    if (!finite2(F)) atomicOr(status, kStatusNonFinite);
    xo[g] = xi[p];
    vo[g] = ui[p];
    ido[g] = id;
    Fo[g] = F;
}

// First half kick and drift of a dpd_step call, from the stored state.
__global__ void k_kick_drift(DevParams P, const float2* __restrict__ x, const float2* __restrict__ v,
                             const float2* __restrict__ F, const int* __restrict__ id, float2* xo,
                             float2* uo, int* ido, int* key, int* rank, int* count,
                             unsigned* status, int* pos) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= P.N) return;
    const float2 f = F[g], vv = v[g], xx = x[g];
    const float2 u = make_float2(fmaf(P.h, f.x, vv.x), fmaf(P.h, f.y, vv.y));
    const float2 xn = make_float2(drift_wrap(xx.x, u.x, P), drift_wrap(xx.y, u.y, P));
    const int k = cell_key(xn, P) + P.cbase;
    const int idg = id[g];
    xo[g] = xn;
    uo[g] = u;
    ido[g] = idg;
    // far bonds: the id -> index map of the buffers written (indices of the
    // whole batch)
    if (pos && (unsigned)idg < (unsigned)P.N) pos[P.pbase + idg] = P.pbase + g;
    key[g] = k;
    rank[g] = atomicAdd(&count[k], 1);
    if (!finite2(xn) || !finite2(u)) atomicOr(status, kStatusNonFinite);
}

// Fixed-order sum of the per-tile partials -> (P_x, P_y, KE), in two stages:
// k_reduce_part sums fixed consecutive ranges of tiles (one block each), then
// k_reduce_final sums the block results.
constexpr int kRedParts = 256;

__global__ __launch_bounds__(kBlock) void k_reduce_part(const double* __restrict__ red, int n_tiles,
                                                        double* part) {
    __shared__ double s_red[kBlock / kWave][3];
    const int per = (n_tiles + gridDim.x - 1) / gridDim.x;
    const int t0 = blockIdx.x * per, t1 = min(n_tiles, t0 + per);
    double v[3] = {0.0, 0.0, 0.0};
    for (int t = t0 + threadIdx.x; t < t1; t += kBlock) {
        v[0] += red[3 * t + 0];
        v[1] += red[3 * t + 1];
        v[2] += red[3 * t + 2];
    }
    block_sum3(v, s_red);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = v[0];
        part[3 * blockIdx.x + 1] = v[1];
        part[3 * blockIdx.x + 2] = v[2];
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce_final(const double* __restrict__ part,
                                                         int n_parts, double mass, double* out) {
    __shared__ double s_red[kBlock / kWave][3];
    double v[3] = {0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < n_parts; t += kBlock) {
        v[0] += part[3 * t + 0];
        v[1] += part[3 * t + 1];
        v[2] += part[3 * t + 2];
    }
    block_sum3(v, s_red);
    if (threadIdx.x == 0) {
        out[0] = mass * v[0];
        out[1] = mass * v[1];
        out[2] = 0.5 * mass * v[2];
    }
}

// Per replica of a batch: (P_x, P_y, KE) of its tiles, summed in a fixed order
// by one block per replica.
__global__ __launch_bounds__(kBlock) void k_reduce_reps(const double* __restrict__ red,
                                                        const DevParams* __restrict__ reps,
                                                        double* out) {
    __shared__ double s_red[kBlock / kWave][3];
    const DevParams& P = reps[blockIdx.x];
    const int t0 = P.tbase, t1 = P.tbase + P.ntx * P.nty;
    double v[3] = {0.0, 0.0, 0.0};
    for (int t = t0 + threadIdx.x; t < t1; t += kBlock) {
        v[0] += red[3 * t + 0];
        v[1] += red[3 * t + 1];
        v[2] += red[3 * t + 2];
    }
    block_sum3(v, s_red);
    if (threadIdx.x == 0) {
        out[3 * blockIdx.x + 0] = P.mass_d * v[0];
        out[3 * blockIdx.x + 1] = P.mass_d * v[1];
        out[3 * blockIdx.x + 2] = 0.5 * P.mass_d * v[2];
    }
}

// Sorted order -> id order.
__global__ void k_unpermute(int N, const int* __restrict__ id, const float2* __restrict__ a,
                            float2* out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    out[id[g]] = a[g];
}

// ---- filtered and projected velocity field (Sec. 5.4) -------------------------

struct BinArgs {
    const float2* x;   // id order
    const float2* v;   // id order
    long long* acc;    // M*M*3: sum q_x, sum q_y, count
    unsigned* status;
    int n_src;         // particles (mode 0) or agents (mode 1)
    int mode;
    int M;
    double L;
    double inv_dx;     // M / L
    double dx;         // L / M
    double eps;        // window width, <= 0 for plain bins
    double qscale;     // fixed-point scale 2^S
    double vmax;       // velocities beyond this cannot be summed exactly
};

__device__ __forceinline__ int clamp_floor(double y, int n) {
    double f = floor(y);
    f = fmin(fmax(f, 0.0), (double)(n - 1));
    return (int)f;
}

__global__ void k_bin_accum(BinArgs b) {
#pragma clang fp contract(off)
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= b.n_src) return;
    double px, py, vx, vy;
    const double L = b.L;
    if (b.mode == 0) {
        px = (double)b.x[s].x;
        py = (double)b.x[s].y;
        vx = (double)b.v[s].x;
        vy = (double)b.v[s].y;
    } else {
        const float2 xh = b.x[2 * s], xt = b.x[2 * s + 1];
        const float2 vh = b.v[2 * s], vt = b.v[2 * s + 1];
        double dx = (double)xh.x - (double)xt.x;
        double dy = (double)xh.y - (double)xt.y;
        if (dx >= 0.5 * L) dx -= L; else if (dx < -0.5 * L) dx += L;
        if (dy >= 0.5 * L) dy -= L; else if (dy < -0.5 * L) dy += L;
        px = (double)xt.x + 0.5 * dx;
        py = (double)xt.y + 0.5 * dy;
        if (px < 0.0) px += L; else if (px >= L) px -= L;
        if (py < 0.0) py += L; else if (py >= L) py -= L;
        vx = 0.5 * ((double)vh.x + (double)vt.x);
        vy = 0.5 * ((double)vh.y + (double)vt.y);
    }
    if (!(px >= 0.0 && px < L) || !(py >= 0.0 && py < L)) {
        atomicOr(b.status, kStatusNonFinite);
        return;
    }
    if (!(fabs(vx) <= b.vmax) || !(fabs(vy) <= b.vmax)) {
        atomicOr(b.status, kStatusRange);
        return;
    }
    const long long qx = llrint(vx * b.qscale), qy = llrint(vy * b.qscale);
    const int M = b.M;
    if (b.eps <= 0.0) {
        const int bx = clamp_floor(px * b.inv_dx, M), by = clamp_floor(py * b.inv_dx, M);
        const int k = by * M + bx;
        atomicAdd((unsigned long long*)&b.acc[3 * k + 0], (unsigned long long)qx);
        atomicAdd((unsigned long long*)&b.acc[3 * k + 1], (unsigned long long)qy);
        atomicAdd((unsigned long long*)&b.acc[3 * k + 2], 1ull);
        return;
    }
    const double half = 0.5 * b.eps;
    long long lo[2], hi[2];
    const double pos[2] = {px, py};
    for (int ax = 0; ax < 2; ++ax) {
        lo[ax] = (long long)floor((pos[ax] - half) / b.dx) - 1;
        hi[ax] = (long long)floor((pos[ax] + half) / b.dx) + 1;
        if (hi[ax] - lo[ax] + 1 > M) {
            lo[ax] = 0;
            hi[ax] = M - 1;
        }
    }
    for (long long jy = lo[1]; jy <= hi[1]; ++jy) {
        const int gy = (int)(((jy % M) + M) % M);
        const double ym = ((double)gy + 0.5) * b.dx;
        double ddy = py - ym;
        if (ddy >= 0.5 * L) ddy -= L; else if (ddy < -0.5 * L) ddy += L;
        if (!(ddy >= -half && ddy < half)) continue;
        for (long long jx = lo[0]; jx <= hi[0]; ++jx) {
            const int gx = (int)(((jx % M) + M) % M);
            const double xm = ((double)gx + 0.5) * b.dx;
            double ddx = px - xm;
            if (ddx >= 0.5 * L) ddx -= L; else if (ddx < -0.5 * L) ddx += L;
            if (!(ddx >= -half && ddx < half)) continue;
            const int k = gy * M + gx;
            atomicAdd((unsigned long long*)&b.acc[3 * k + 0], (unsigned long long)qx);
            atomicAdd((unsigned long long*)&b.acc[3 * k + 1], (unsigned long long)qy);
            atomicAdd((unsigned long long*)&b.acc[3 * k + 2], 1ull);
        }
    }
}

// Plain bins of particle velocities from the canonical state.  Block (q, j)
// owns bins [q M/Q, (q+1) M/Q) of grid row j.  The cells that can hold those
// bins (one cell of margin on each side) are, row by row, contiguous in the
// (cell, id) order; the block sums the particles whose bin it owns into LDS
// fixed-point accumulators and writes the bins' means and counts.  No global
// atomics; the sums are exact, so the result is bitwise that of k_bin_accum +
// k_bin_finalize.
struct BinRowArgs {
    const float2* x;   // canonical order
    const float2* v;
    const int* cs;     // cell_start of that order
    float2* u;
    int* n;
    unsigned* status;
    int M;
    int Q;             // column parts per grid row
    int nc;
    double L;
    double inv_dx;     // M / L
    double qscale;
    double vmax;
};

constexpr int kBinRowBlock = 256;

// Up to two ranges [lo, hi] of cell indices modulo nc covering [a, b] (b - a + 1 < nc).
__device__ __forceinline__ int wrapped_ranges(long long a, long long b, int nc, int lo[2], int hi[2]) {
    if (b - a + 1 >= nc) {
        lo[0] = 0; hi[0] = nc - 1;
        return 1;
    }
    if (a < 0) {
        lo[0] = (int)(a + nc); hi[0] = nc - 1;
        lo[1] = 0; hi[1] = (int)b;
        return 2;
    }
    if (b >= nc) {
        lo[0] = (int)a; hi[0] = nc - 1;
        lo[1] = 0; hi[1] = (int)(b - nc);
        return 2;
    }
    lo[0] = (int)a; hi[0] = (int)b;
    return 1;
}

__global__ __launch_bounds__(kBinRowBlock) void k_bin_rows(BinRowArgs b) {
#pragma clang fp contract(off)
    extern __shared__ long long s_bin[];  // 3 per owned bin: sum q_x, sum q_y, count
    const int M = b.M, Q = b.Q, nc = b.nc;
    const int j = blockIdx.y, q = blockIdx.x;
    const int i0 = (int)((long long)q * M / Q), i1 = (int)((long long)(q + 1) * M / Q);
    const int nb = i1 - i0;
    for (int i = threadIdx.x; i < 3 * nb; i += blockDim.x) s_bin[i] = 0;
    __syncthreads();
    int rlo[2], rhi[2], clo[2], chi[2];
    const int nr = wrapped_ranges((long long)j * nc / M - 1, ((long long)(j + 1) * nc + M - 1) / M, nc, rlo, rhi);
    const int ncr = wrapped_ranges((long long)i0 * nc / M - 1, ((long long)i1 * nc + M - 1) / M, nc, clo, chi);
    for (int ra = 0; ra < nr; ++ra) {
        for (int row = rlo[ra]; row <= rhi[ra]; ++row) {
            const long long rb = (long long)row * nc;
            for (int ca = 0; ca < ncr; ++ca) {
                const int g0 = b.cs[rb + clo[ca]], g1 = b.cs[rb + chi[ca] + 1];
                for (int g = g0 + threadIdx.x; g < g1; g += blockDim.x) {
                    const float2 xx = b.x[g];
                    const double py = (double)xx.y, px = (double)xx.x;
                    if (clamp_floor(py * b.inv_dx, M) != j) continue;
                    const int bx = clamp_floor(px * b.inv_dx, M);
                    if (bx < i0 || bx >= i1) continue;
                    if (!(px >= 0.0 && px < b.L) || !(py >= 0.0 && py < b.L)) {
                        atomicOr(b.status, kStatusNonFinite);
                        continue;
                    }
                    const float2 vv = b.v[g];
                    const double vx = (double)vv.x, vy = (double)vv.y;
                    if (!(fabs(vx) <= b.vmax) || !(fabs(vy) <= b.vmax)) {
                        atomicOr(b.status, kStatusRange);
                        continue;
                    }
                    const int k = bx - i0;
                    atomicAdd((unsigned long long*)&s_bin[3 * k + 0], (unsigned long long)llrint(vx * b.qscale));
                    atomicAdd((unsigned long long*)&s_bin[3 * k + 1], (unsigned long long)llrint(vy * b.qscale));
                    atomicAdd((unsigned long long*)&s_bin[3 * k + 2], 1ull);
                }
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        const long long c = s_bin[3 * i + 2];
        const long long k = (long long)j * M + i0 + i;
        b.n[k] = (int)c;
        if (c > 0) {
            const double inv = 1.0 / (b.qscale * (double)c);
            b.u[k] = make_float2((float)((double)s_bin[3 * i + 0] * inv),
                                 (float)((double)s_bin[3 * i + 1] * inv));
        } else {
            b.u[k] = make_float2(0.f, 0.f);
        }
    }
}

__global__ void k_bin_finalize(int nbin, const long long* __restrict__ acc, double qscale,
                               float2* u, int* n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nbin) return;
    const long long c = acc[3 * k + 2];
    n[k] = (int)c;
    if (c > 0) {
        const double inv = 1.0 / (qscale * (double)c);
        u[k] = make_float2((float)((double)acc[3 * k + 0] * inv), (float)((double)acc[3 * k + 1] * inv));
    } else {
        u[k] = make_float2(0.f, 0.f);
    }
}

// ---- velocity correlation of the agents (Sec. 5.3) ----------------------------

// Agent centres of mass and velocities in FP64 from the FP32 state in id
// order: d = x_head - x_tail under the minimum image, centre = (x_tail + d/2)
// wrapped into [0, L), V = (v_head + v_tail) / 2.  work holds the centres
// [n][2], then the velocities [n][2].
__global__ void k_agent_com(int n, double L, const float2* __restrict__ x, const float2* __restrict__ v,
                            double* work) {
#pragma clang fp contract(off)
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float2 xh = x[2 * k], xt = x[2 * k + 1], vh = v[2 * k], vt = v[2 * k + 1];
    double c[2];
    const double h[2] = {(double)xh.x, (double)xh.y}, t[2] = {(double)xt.x, (double)xt.y};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        double d = h[a] - t[a];
        d = d - L * rint(d / L);
        double y = t[a] + 0.5 * d;
        y = y - L * floor(y / L);
        c[a] = y;
    }
    work[2 * k] = c[0];
    work[2 * k + 1] = c[1];
    work[2 * n + 2 * k] = 0.5 * ((double)vh.x + (double)vt.x);
    work[2 * n + 2 * k + 1] = 0.5 * ((double)vh.y + (double)vt.y);
}

// Pair sums of V_k . V_l over the pairs k < l binned by their minimum-image
// separation, floor(r / dr) < nb, and the pair counts.  A block of 256 threads
// takes the 256 x 256 pairs of one tile of the upper triangle (row tile
// blockIdx.y, column tile blockIdx.x >= blockIdx.y; lower tiles exit), the
// column tile staged in LDS.  The separation and the bin follow the plain
// FP64 sequence d - L rint(d / L), sqrt(dx dx + dy dy), floor(r / dr); every
// dot product enters in 64-bit fixed point (scale 2^20, exact integer sums, so
// the result does not depend on the order), the block's bins then go to the
// global sums with integer atomics.
constexpr int kVcfTile = 256;
constexpr int kVcfMaxBins = 1024;
constexpr double kVcfScale = 1048576.0;  // 2^20

__global__ __launch_bounds__(kVcfTile) void k_vcf_pairs(int n, double L, double dr, int nb,
                                                        const double* __restrict__ work,
                                                        long long* sums, long long* counts,
                                                        unsigned* status) {
#pragma clang fp contract(off)
    if (blockIdx.x < blockIdx.y) return;
    __shared__ double s_pos[kVcfTile][2];
    __shared__ double s_vel[kVcfTile][2];
    __shared__ long long s_sum[kVcfMaxBins];
    __shared__ int s_cnt[kVcfMaxBins];
    const int t = threadIdx.x;
    for (int b = t; b < nb; b += kVcfTile) {
        s_sum[b] = 0;
        s_cnt[b] = 0;
    }
    const int l0 = blockIdx.x * kVcfTile, k = blockIdx.y * kVcfTile + t;
    const double* pos = work;
    const double* vel = work + 2 * (size_t)n;
    if (l0 + t < n) {
        s_pos[t][0] = pos[2 * (l0 + t)];
        s_pos[t][1] = pos[2 * (l0 + t) + 1];
        s_vel[t][0] = vel[2 * (l0 + t)];
        s_vel[t][1] = vel[2 * (l0 + t) + 1];
    }
    __syncthreads();
    bool big = false;
    if (k < n) {
        const double px = pos[2 * k], py = pos[2 * k + 1];
        const double vx = vel[2 * k], vy = vel[2 * k + 1];
        const int lend = min(kVcfTile, n - l0);
        for (int j = 0; j < lend; ++j) {
            if (l0 + j <= k) continue;
            double dx = s_pos[j][0] - px;
            double dy = s_pos[j][1] - py;
            dx = dx - L * rint(dx / L);
            dy = dy - L * rint(dy / L);
            const double r = sqrt(dx * dx + dy * dy);
            const double bf = floor(r / dr);
            if (!(bf < (double)nb)) continue;
            const int b = (int)bf;
            const double dot = s_vel[j][0] * vx + s_vel[j][1] * vy;
            big |= !(fabs(dot) < 4096.0);
            atomicAdd((unsigned long long*)&s_sum[b], (unsigned long long)llrint(dot * kVcfScale));
            atomicAdd(&s_cnt[b], 1);
        }
    }
    if (big) atomicOr(status, kStatusRange);
    __syncthreads();
    for (int b = t; b < nb; b += kVcfTile) {
        if (s_cnt[b]) {
            atomicAdd((unsigned long long*)&sums[b], (unsigned long long)s_sum[b]);
            atomicAdd((unsigned long long*)&counts[b], (unsigned long long)s_cnt[b]);
        }
    }
}

// ---- diagnostics -------------------------------------------------------------

__global__ void k_rng_words(DevParams P, const int* __restrict__ i, const int* __restrict__ j,
                            uint32_t step, int n, uint4* words, float* alpha) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t a = (uint32_t)min(i[k], j[k]), b = (uint32_t)max(i[k], j[k]);
    uint4 w;
    uint2 w2;
    if (P.rng_kind == 0) {
        w = philox4x32_10(make_uint4(a, b, step, 0u), P.seed_lo, P.seed_hi);
        w2 = make_uint2(w.x, w.y);
    } else {
        w2 = pair_words2(P, a, b, step);
        w = make_uint4(w2.x, w2.y, 0u, 0u);
    }
    words[k] = w;
    if (alpha) alpha[k] = alpha_from_words(P.noise_kind, w2);
}

__global__ void k_fill_i32(int* p, int v, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Advance the step before the next replay of a captured chunk of steps.
__global__ void k_add_u32(unsigned* p, unsigned v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) p[0] += v;
}

__global__ void k_copy16(const uint4* __restrict__ a, uint4* __restrict__ b, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        b[i] = a[i];
}

}  // namespace dpd
