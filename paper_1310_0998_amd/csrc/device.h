// device.h -- constants and small device functions shared by the engine's
// kernels: launch parameters, the counter-based noise generator, periodic
// wrap and cell keys.  Written for gfx950 (64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpd {

constexpr int kWave = 64;

// Device-side status bits (reported by the next synchronising host call).
constexpr unsigned kStatusNonFinite = 1u;
constexpr unsigned kStatusBond = 2u;
constexpr unsigned kStatusRange = 4u;
constexpr unsigned kStatusBinning = 8u;  // cell counts inconsistent with N (internal error)
constexpr unsigned kStatusScan = 16u;    // the cell scan's look-back waited too long (internal error)

// Everything a kernel needs to know about the model, by value.
struct DevParams {
    int N;            // particles
    int nc;           // cells per side
    int n_cells;      // nc * nc
    int tile_x;       // pair-kernel tile width (cells)
    int tile_y;       // pair-kernel tile height (cells)
    int ntx, nty;     // tiles per side
    int wmul_full;    // ceil(2^16 / (tile_x + 2)): local cell -> row by multiply-shift
    int wmul_last;    // the same for the narrower last tile column
    double inv_ntx;   // 1 / ntx: tile row = floor((tile + 1/2) / ntx) by one multiply
    int skin_on;      // Verlet skin in use
    float list_rc2;   // (r_c + skin)^2, rounded up: pairs kept in the tile lists
    float half_skin2; // (skin / 2)^2, rounded down: displacement that forces a rebuild
    int noise_kind;   // 0 Gaussian, 1 uniform
    int rng_kind;     // 0 Philox4x32-10, 1 Philox2x32-10
    float L;          // box side (FP32)
    float halfL;
    float rc;         // r_c
    float rc2;        // r_c^2
    float inv_rc;     // 1 / r_c
    float A;
    float gamma;
    float sigma_rdt;  // sqrt(2 gamma kT) / sqrt(dt)
    float kappa;
    float bond_l;
    float bond_l2_hi; // l^2 as a sum of two floats (hi + lo)
    float bond_l2_lo;
    float sp_head;    // share of f_sp on the head, times f_sp
    float sp_tail;    // share of f_sp on the tail, times f_sp
    float gamma_s;
    float h;          // dt / (2 m)
    double L_d;       // box side (FP64)
    double dt_d;      // time step (FP64)
    double inv_w;     // nc / L (FP64): cell = floor(x * inv_w)
    uint32_t seed_lo, seed_hi;
    // a replica of a batch: its first particle slot, cell and tile in the
    // concatenated arrays of the batch (all 0 for a single system), its mass
    int pbase, cbase, tbase;
    double mass_d;
    float w_half;     // half the exponent of the dissipative weight (1: Eq. 2.3)
    int far_bond;     // a bond may reach beyond the 3 x 3 cell stencil: the partner
                      // is then read by id (PairArgs::pos_of_id)
};

// ---- Philox (Salmon, Moraes, Dror & Shaw, SC'11) ---------------------------
// A Feistel-like network whose nonlinearity is the 32x32 -> 64 multiply; the
// key advances by a Weyl sequence between rounds.

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ uint2 philox2x32_10(uint2 c, uint32_t k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p = (uint64_t)0xD256D193u * (uint64_t)c.x;
        c = make_uint2((uint32_t)(p >> 32) ^ k ^ c.y, (uint32_t)p);
        k += 0x9E3779B9u;
    }
    return c;
}

// Two raw words for the pair (a = min id, b = max id) at step s.
__device__ __forceinline__ uint2 pair_words2(const DevParams& P, uint32_t a, uint32_t b,
                                             uint32_t s) {
    if (P.rng_kind == 0) {
        const uint4 w = philox4x32_10(make_uint4(a, b, s, 0u), P.seed_lo, P.seed_hi);
        return make_uint2(w.x, w.y);
    }
    const uint32_t key = P.seed_lo ^ (P.seed_hi * 0x85EBCA6Bu) ^ (s * 0xC2B2AE35u);
    return philox2x32_10(make_uint2(a, b), key);
}

// 23 random bits -> (2n + 1) / 2^24, inside (0, 1), exact in FP32: the bits
// become the mantissa of 1 + n 2^-23 in [1, 2), and subtracting 1 - 2^-24 from
// it is exact (the two are within a factor of 2 of each other).
__device__ __forceinline__ float unit_open(uint32_t w) {
    return __uint_as_float((w >> 9) | 0x3F800000u) - 0.999999940395355224609375f;
}

// alpha^{ij}: Gaussian by Box-Muller (cosine branch) or uniform of unit variance.
// The Gaussian uses the hardware base-2 logarithm, square root and cosine of
// 2 pi times the argument directly (-2 ln u0 = -2 ln 2 log2 u0): measured over
// every uniform the generator produces, they give alpha within 1.5e-6 of its
// FP64 value.
__device__ __forceinline__ float alpha_from_words(int noise_kind, uint2 w) {
    const float u0 = unit_open(w.x);
    if (noise_kind == 1) return 1.7320508075688772f * (2.0f * u0 - 1.0f);
    const float u1 = unit_open(w.y);
    return __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u0)) *
           __builtin_amdgcn_cosf(u1);
}

// ---- periodic geometry ------------------------------------------------------

// Cell coordinate of an FP32 position: min(nc - 1, floor(x * nc / L)) in FP64.
// The clamp runs in FP64 before the conversion, so any input (NaN included)
// yields a cell inside the grid.
__device__ __forceinline__ int cell_coord(float x, const DevParams& P) {
    double c = floor((double)x * P.inv_w);
    c = fmin(fmax(c, 0.0), (double)(P.nc - 1));
    return (int)c;
}

__device__ __forceinline__ int cell_key(float2 x, const DevParams& P) {
    // cell coordinates and nc are below 2^24 and the key below 2^31: the 24-bit
    // multiply gives the exact product
    return (int)__umul24((unsigned)cell_coord(x.y, P), (unsigned)P.nc) + cell_coord(x.x, P);
}

// x + dt u evaluated and wrapped into [0, L) in FP64, then rounded to FP32
// (a value that rounds up to L becomes 0).
__device__ __forceinline__ float drift_wrap(float x, float u, const DevParams& P) {
    double y = (double)x + P.dt_d * (double)u;
    if (y < 0.0 || y >= P.L_d) {
        y = y - P.L_d * floor(y / P.L_d);
        if (y >= P.L_d) y -= P.L_d;
        if (y < 0.0) y += P.L_d;
    }
    float f = (float)y;
    return f >= P.L ? 0.0f : f;
}

// Minimum-image separation component with the shift applied to the operand
// near L, which keeps the shift exact (x - L is exact for x >= L/2).
__device__ __forceinline__ float minimg_sub(float xi, float xj, const DevParams& P) {
    float d = xi - xj;
    if (d > P.halfL) d = (xi - P.L) - xj;
    else if (d < -P.halfL) d = xi - (xj - P.L);
    return d;
}

// Minimum-image separation as an unevaluated sum hi + lo of two floats (the
// rounding error of the final subtraction by Knuth's two-sum), for the stiff
// bond whose force needs |d| beyond FP32 resolution.
__device__ __forceinline__ float minimg_sub2(float xi, float xj, const DevParams& P, float& lo) {
#pragma clang fp contract(off)
    float a = xi, b = xj;
    const float d0 = xi - xj;
    if (d0 > P.halfL) a = xi - P.L;        // exact: xi >= L/2
    else if (d0 < -P.halfL) b = xj - P.L;  // exact: xj >= L/2
    const float s = a - b;
    const float bb = s - a;
    lo = (a - (s - bb)) + (-b - bb);
    return s;
}

__device__ __forceinline__ bool finite2(float2 a) {
    return __builtin_isfinite(a.x) && __builtin_isfinite(a.y);
}

}  // namespace dpd
