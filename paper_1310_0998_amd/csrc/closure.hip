// closure.hip -- the learned closure of include/closure.h: a periodic
// convolutional network on the binned velocity field (Sec. 5.4), its training
// kernels (forward, loss, input and weight gradients, Adam) and its rollout.
//
// Layout: every field is NHWC ([pixel][channel], pixel = (b M + j) M + i).
// Convolution l maps c_in(l) channels to c_out(l): 3 x 3 taps with periodic
// wrap, weights W_l[tap][c][o] (FP32 master), bias b_l[o].
//
// Forward and input-gradient convolutions are implicit GEMMs on the matrix
// cores: one 64-lane wavefront computes 16 pixels x 16 output channels per
// accumulator, running over K = 9 c_in.  The LDS-staged forward kernel and
// the input-gradient kernel take K in chunks of 32 (v_mfma_f32_16x16x32_bf16,
// 8 values per lane); the general forward kernels for other shapes take
// chunks of 16 (v_mfma_f32_16x16x16_bf16, 4 consecutive channels of one tap
// per lane, one 8-byte load).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/closure.h"
#include "../../include/dpd.h"
#include "device.h"

namespace nn {

constexpr int kWaveN = 64;
constexpr int kThreads = 256;      // 4 wavefronts per block
constexpr int kWgPix = 256;        // pixels per block of the weight-gradient sums
constexpr int kWgStage = 8;        // pixels staged in LDS at a time
constexpr int kMaxC = 32;          // largest channel count
constexpr int kWgOutMax = 9 * kMaxC * kMaxC + kMaxC;  // weights + biases of one layer
constexpr int kWgPerThread = (kWgOutMax + kThreads - 1) / kThreads;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (NaN stays NaN).
__device__ __forceinline__ unsigned short to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float from_bf16(unsigned short h) {
    return __uint_as_float((unsigned)h << 16);
}

// One convolution's shapes.
struct Conv {
    int cin, cout;      // channels in, out
    int K, Kpad;        // 9 cin, rounded up to 16
    int cout16;         // cout rounded up to 16 (output-channel tiles)
    int cout4;          // cout rounded up to 4 (channels of the BF16 output gradient)
    int Kb, Kbpad;      // 9 cout4, rounded up to 16
    int cin16;          // cin rounded up to 16
};

// ---- parameters -----------------------------------------------------------------

// Master W[tap][c][o] -> Wf[o][tap cin + c] (forward B operand, rows padded to
// cout16 and Kpad) and Wb[c][tap cout4 + o] (input-gradient B operand).
__global__ void k_cast_weights(Conv cv, const float* __restrict__ W, unsigned short* Wf,
                               unsigned short* Wb) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int nf = cv.cout16 * cv.Kpad;
    if (t < nf) {
        const int o = t / cv.Kpad, k = t % cv.Kpad;
        float w = 0.f;
        if (o < cv.cout && k < cv.K) w = W[k * cv.cout + o];  // k = tap cin + c
        Wf[t] = to_bf16(w);
    }
    const int nb = cv.cin16 * cv.Kbpad;
    if (Wb && t < nb) {
        const int c = t / cv.Kbpad, k = t % cv.Kbpad;
        float w = 0.f;
        if (c < cv.cin && k < cv.Kb) {
            const int tap = k / cv.cout4, o = k % cv.cout4;
            if (o < cv.cout) w = W[(tap * cv.cin + c) * cv.cout + o];
        }
        Wb[t] = to_bf16(w);
    }
}

// ---- forward ---------------------------------------------------------------------

// First activation: (u_x, u_y, conditions...) rounded to BF16.
__global__ void k_input(int npix, int M2, int cin, const float* __restrict__ u,
                        const float* __restrict__ cond, unsigned short* X) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const int b = p / M2;
    X[(size_t)p * cin + 0] = to_bf16(u[2 * (size_t)p + 0]);
    X[(size_t)p * cin + 1] = to_bf16(u[2 * (size_t)p + 1]);
    for (int c = 2; c < cin; ++c) X[(size_t)p * cin + c] = to_bf16(cond[(size_t)b * (cin - 2) + c - 2]);
}

// Pixel index of (pixel p, tap) shifted by +(dx, dy) (sign = 1) or -(dx, dy)
// (sign = -1) with periodic wrap.
__device__ __forceinline__ int shifted(int p, int tap, int sign, int M) {
    const int M2 = M * M;
    const int b = p / M2, r = p - b * M2;
    const int y = r / M, x = r - y * M;
    const int dy = sign * (tap / 3 - 1), dx = sign * (tap % 3 - 1);
    int ny = y + dy, nx = x + dx;
    ny += (ny < 0) ? M : 0;
    ny -= (ny >= M) ? M : 0;
    nx += (nx < 0) ? M : 0;
    nx -= (nx >= M) ? M : 0;
    return b * M2 + ny * M + nx;
}

// Z = conv(X, W) + b on 16-pixel tiles, one wavefront each.  Hidden layers
// write relu(Z) in BF16 (the next activation); the last writes pred = u + Z.
template <bool LAST>
__global__ __launch_bounds__(kThreads) void k_conv_fwd(Conv cv, int M, int npix,
                                                        const unsigned short* __restrict__ X,
                                                        const unsigned short* __restrict__ Wf,
                                                        const float* __restrict__ bias,
                                                        unsigned short* Xnext,
                                                        const float* __restrict__ u, float* pred) {
    const int tile = blockIdx.x * (kThreads / kWaveN) + threadIdx.x / kWaveN;
    if (tile * 16 >= npix) return;
    const int lane = threadIdx.x & (kWaveN - 1), r16 = lane & 15, g = lane >> 4;
    const int pa = tile * 16 + r16;  // pixel of this lane's A row
    const int nct = cv.cout16 / 16;  // 1 or 2
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < cv.Kpad; k0 += 16) {
        const int k = k0 + 4 * g;
        bf16x4 a = {0, 0, 0, 0};
        if (k < cv.K) {
            const int tap = k / cv.cin, c = k - tap * cv.cin;
            const int q = shifted(pa, tap, 1, M);
            a = *reinterpret_cast<const bf16x4*>(X + (size_t)q * cv.cin + c);
        }
        const bf16x4 b0 = *reinterpret_cast<const bf16x4*>(Wf + (size_t)r16 * cv.Kpad + k);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b0, acc0, 0, 0, 0);
        if (nct > 1) {
            const bf16x4 b1 = *reinterpret_cast<const bf16x4*>(Wf + (size_t)(16 + r16) * cv.Kpad + k);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b1, acc1, 0, 0, 0);
        }
    }
    // D[row 4 g + i][column r16]: pixel tile 16 + 4 g + i, channel ct 16 + r16
    for (int ct = 0; ct < nct; ++ct) {
        const int o = ct * 16 + r16;
        if (o >= cv.cout) continue;
        const f32x4 acc = ct == 0 ? acc0 : acc1;
        const float bo = bias[o];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int p = tile * 16 + 4 * g + i;
            const float z = acc[i] + bo;
            if (LAST)
                pred[2 * (size_t)p + o] = u[2 * (size_t)p + o] + z;
            else
                Xnext[(size_t)p * cv.cout + o] = to_bf16(fmaxf(z, 0.f));
        }
    }
}

// The same convolution for c_in = CIN in {4, 16, 32}.  At CIN >= 16 every
// chunk of 16 K values lies within one tap; at CIN = 4 a lane group's 4 K
// values are the 4 channels of one tap (K = 36, padded to 48 with zero
// activations).  A wavefront keeps its lanes' weight operands in registers and
// computes kConvTPW consecutive 16-pixel tiles with them; per tile the
// neighbour pixels are found once and all activation loads are issued before
// the matrix-core chain, the next tile's loads overlapping this tile's
// products (same products, same accumulation order as k_conv_fwd).  NCT:
// output-channel tiles (cout16 / 16).
constexpr int kConvTPW = 4;
template <int CIN, int NCT, bool LAST>
__global__ __launch_bounds__(kThreads) void k_conv_fwd_c(Conv cv, int M, int npix,
                                                          const unsigned short* __restrict__ X,
                                                          const unsigned short* __restrict__ Wf,
                                                          const float* __restrict__ bias,
                                                          unsigned short* Xnext,
                                                          const float* __restrict__ u, float* pred) {
    static_assert((CIN == 4 || CIN % 16 == 0) && (NCT == 1 || NCT == 2), "unsupported shape");
    constexpr int CH = CIN >= 16 ? CIN / 16 : 1;  // chunks per tap (CIN >= 16)
    constexpr int NK = CIN >= 16 ? 9 * CH : 3;    // chunks of 16 K values (K = 36 padded to 48 at CIN = 4)
    const int wave = blockIdx.x * (kThreads / kWaveN) + threadIdx.x / kWaveN;
    const int ntile = npix / 16;
    if (wave * kConvTPW >= ntile) return;
    const int lane = threadIdx.x & (kWaveN - 1), r16 = lane & 15, g = lane >> 4;
    bf16x4 wb[NCT][NK];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
        for (int i = 0; i < NK; ++i)
            wb[ct][i] = *reinterpret_cast<const bf16x4*>(Wf + (size_t)(ct * 16 + r16) * cv.Kpad + i * 16 + 4 * g);
    float bo[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
        const int o = ct * 16 + r16;
        bo[ct] = o < cv.cout ? bias[o] : 0.f;
    }
    const int M2 = M * M;
    // activation operands of tile t: the NK chunks of its 16 pixels
    auto load = [&](int t, bf16x4 (&dst)[NK]) {
        const int pa = t * 16 + r16;
        const int b = pa / M2, rr = pa - b * M2;
        const int y = rr / M, x = rr - y * M;
        const int ys[3] = {y == 0 ? M - 1 : y - 1, y, y == M - 1 ? 0 : y + 1};
        const int xs[3] = {x == 0 ? M - 1 : x - 1, x, x == M - 1 ? 0 : x + 1};
        if constexpr (CIN == 4) {
            // chunk i, lane group g: the 4 channels of tap 4 i + g (zero past tap 8)
#pragma unroll
            for (int i = 0; i < NK; ++i) {
                const int tap = 4 * i + g;
                dst[i] = bf16x4{0, 0, 0, 0};
                if (tap < 9) {
                    const int ty = tap / 3, tx = tap - 3 * ty;
                    const int yy = ty == 0 ? ys[0] : (ty == 1 ? ys[1] : ys[2]);
                    const int xx = tx == 0 ? xs[0] : (tx == 1 ? xs[1] : xs[2]);
                    const size_t q = (size_t)b * M2 + yy * M + xx;
                    dst[i] = *reinterpret_cast<const bf16x4*>(X + q * 4);
                }
            }
        } else {
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const size_t q = (size_t)b * M2 + ys[tap / 3] * M + xs[tap % 3];
#pragma unroll
                for (int h = 0; h < CH; ++h)
                    dst[tap * CH + h] = *reinterpret_cast<const bf16x4*>(X + q * CIN + h * 16 + 4 * g);
            }
        }
    };
    bf16x4 a[2][NK];
    load(wave * kConvTPW, a[0]);
#pragma unroll
    for (int tt = 0; tt < kConvTPW; ++tt) {
        const int tile = wave * kConvTPW + tt;
        if (tile >= ntile) break;
        // the next tile's loads are in flight while this one's products run
        if (tt + 1 < kConvTPW && tile + 1 < ntile) load(tile + 1, a[(tt + 1) & 1]);
        f32x4 acc[NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < NK; ++i)
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[tt & 1][i], wb[ct][i], acc[ct], 0, 0, 0);
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            const int o = ct * 16 + r16;
            if (o >= cv.cout) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = tile * 16 + 4 * g + i;
                const float z = acc[ct][i] + bo[ct];
                if (LAST)
                    pred[2 * (size_t)p + o] = u[2 * (size_t)p + o] + z;
                else
                    Xnext[(size_t)p * cv.cout + o] = to_bf16(fmaxf(z, 0.f));
            }
        }
    }
}

// The convolution for CIN in {4, 16, 32} on grids with M in {16, 32, 64}, with
// its operands staged in LDS: a block of 4 wavefronts computes kLdsPix
// consecutive pixels (kLdsPix / M whole rows of one field).  It stages those
// rows and one halo row on each side (periodic), all M columns, and the
// layer's BF16 weights; both layouts are padded by 8 elements per pixel or
// output channel so that the 16 pixels (or channels) a matrix-core operand
// load spans fall in different LDS banks.  Each wavefront then computes
// kLdsPix / 64 tiles from LDS, with its weight operands held in registers.
// Same products as k_conv_fwd, accumulated over K in chunks of 32.
constexpr int kLdsPix = 128;
template <int CIN, int NCT, bool LAST>
__global__ __launch_bounds__(kThreads) void k_conv_fwd_l(Conv cv, int M, int npix,
                                                          const unsigned short* __restrict__ X,
                                                          const unsigned short* __restrict__ Wf,
                                                          const float* __restrict__ bias,
                                                          unsigned short* Xnext,
                                                          const float* __restrict__ u, float* pred) {
    static_assert((CIN == 4 || CIN == 16 || CIN == 32) && (NCT == 1 || NCT == 2), "unsupported shape");
    // K = 9 CIN in chunks of 32 for v_mfma_f32_16x16x32_bf16: lane group g holds
    // the K values 8 g .. 8 g + 7 of a chunk (K index = tap CIN + channel):
    //   CIN = 32: one tap per chunk, channels 8 g .. 8 g + 7;
    //   CIN = 16: taps 2 i (g = 0, 1) and 2 i + 1 (g = 2, 3), channels 8 (g & 1) ..;
    //   CIN = 4:  taps 8 i + 2 g and 8 i + 2 g + 1, 4 channels each.
    // Taps past 8 contribute zeros (the padding of K to a multiple of 32).
    constexpr int NK = (9 * CIN + 31) / 32;
    constexpr int K = NK * 32;                  // weights per output channel, padding included
    // staged elements per pixel: 4 channels at CIN = 4 (16 consecutive pixels
    // then fill consecutive banks), else padded by 8
    constexpr int XS = CIN == 4 ? 4 : CIN + 8;
    constexpr int WS = K + 8;  // staged elements per output channel
    constexpr int kRowsMax = kLdsPix / 16 + 2;  // staged rows at M = 16
    __shared__ __align__(16) unsigned short sx[kRowsMax * 16 * XS > (kLdsPix / 64 + 2) * 64 * XS
                                                   ? kRowsMax * 16 * XS
                                                   : (kLdsPix / 64 + 2) * 64 * XS];
    __shared__ __align__(16) unsigned short sw[NCT * 16 * WS];
    const int p0 = blockIdx.x * kLdsPix;
    if (p0 >= npix) return;
    const int M2 = M * M, R = kLdsPix / M;
    const int b = p0 / M2, y0 = (p0 - b * M2) / M;
    // stage rows y0 - 1 .. y0 + R (periodic) in 16-byte vectors (8-byte ones,
    // a pixel each, at CIN = 4)
    if constexpr (CIN == 4) {
        const int npx = (R + 2) * M;
        for (int pix = threadIdx.x; pix < npx; pix += kThreads) {
            const int rr = pix / M, xx = pix - rr * M;
            int yy = y0 - 1 + rr;
            yy += (yy < 0) ? M : 0;
            yy -= (yy >= M) ? M : 0;
            *reinterpret_cast<uint2*>(sx + pix * XS) =
                *reinterpret_cast<const uint2*>(X + ((size_t)b * M2 + (size_t)yy * M + xx) * 4);
        }
    } else {
        const int nvec = (R + 2) * M * CIN / 8;
        for (int t = threadIdx.x; t < nvec; t += kThreads) {
            const int e = t * 8, pix = e / CIN, c = e - pix * CIN;  // staged pixel, channel
            const int rr = pix / M, xx = pix - rr * M;
            int yy = y0 - 1 + rr;
            yy += (yy < 0) ? M : 0;
            yy -= (yy >= M) ? M : 0;
            const uint4 v = *reinterpret_cast<const uint4*>(X + (((size_t)b * M2 + (size_t)yy * M + xx) * CIN + c));
            *reinterpret_cast<uint4*>(sx + pix * XS + c) = v;
        }
    }
    // the weights of the NCT * 16 output channels (rows of Wf, Kpad long, then
    // zeros up to K)
    const int wvec = NCT * 16 * K / 8;
    for (int t = threadIdx.x; t < wvec; t += kThreads) {
        const int e = t * 8, o = e / K, k = e - o * K;
        uint4 w = make_uint4(0u, 0u, 0u, 0u);
        if (k < cv.Kpad) w = *reinterpret_cast<const uint4*>(Wf + (size_t)o * cv.Kpad + k);
        *reinterpret_cast<uint4*>(sw + o * WS + k) = w;
    }
    __syncthreads();
    const int wave = threadIdx.x / kWaveN, lane = threadIdx.x & (kWaveN - 1);
    const int r16 = lane & 15, g = lane >> 4;
    bf16x8 wb[NCT][NK];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
        for (int i = 0; i < NK; ++i)
            wb[ct][i] = *reinterpret_cast<const bf16x8*>(sw + (ct * 16 + r16) * WS + i * 32 + 8 * g);
    float bo[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
        const int o = ct * 16 + r16;
        bo[ct] = o < cv.cout ? bias[o] : 0.f;
    }
    constexpr int TPW = kLdsPix / 16 / (kThreads / kWaveN);
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
        const int tile = (p0 >> 4) + wave * TPW + tt;
        const int lp = (wave * TPW + tt) * 16 + r16;  // pixel within the block
        const int ly = lp / M, x = lp - ly * M;
        const int xs[3] = {x == 0 ? M - 1 : x - 1, x, x == M - 1 ? 0 : x + 1};
        // staged pixel of tap t (staged row ly + dy + 1)
        auto tap_pix = [&](int t) {
            const int ty = t / 3, tx = t - 3 * ty;
            return (ly + ty) * M + (tx == 0 ? xs[0] : (tx == 1 ? xs[1] : xs[2]));
        };
        bf16x8 a[NK];
#pragma unroll
        for (int i = 0; i < NK; ++i) {
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if constexpr (CIN == 32) {
                v = *reinterpret_cast<const uint4*>(sx + tap_pix(i) * XS + 8 * g);
            } else if constexpr (CIN == 16) {
                const int t = 2 * i + (g >> 1);
                if (t < 9) v = *reinterpret_cast<const uint4*>(sx + tap_pix(t) * XS + 8 * (g & 1));
            } else {
                const int t = 8 * i + 2 * g;
                if (t < 9) {
                    const uint2 lo = *reinterpret_cast<const uint2*>(sx + tap_pix(t) * XS);
                    v.x = lo.x;
                    v.y = lo.y;
                }
                if (t + 1 < 9) {
                    const uint2 hi = *reinterpret_cast<const uint2*>(sx + tap_pix(t + 1) * XS);
                    v.z = hi.x;
                    v.w = hi.y;
                }
            }
            a[i] = __builtin_bit_cast(bf16x8, v);
        }
        f32x4 acc[NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < NK; ++i)
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], wb[ct][i], acc[ct], 0, 0, 0);
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            const int o = ct * 16 + r16;
            if (o >= cv.cout) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = tile * 16 + 4 * g + i;
                const float z = acc[ct][i] + bo[ct];
                if (LAST)
                    pred[2 * (size_t)p + o] = u[2 * (size_t)p + o] + z;
                else
                    Xnext[(size_t)p * cv.cout + o] = to_bf16(fmaxf(z, 0.f));
            }
        }
    }
}

// ---- the whole network of a rollout step -------------------------------------
// All L convolutions of a network with c_in = 4 and width 32 in one kernel, on
// fields of side M in {32, 64}.  A block of kBandWaves wavefronts owns a band
// of R = kBandPix / M output rows of one field.  It stages the input rows of
// the band plus L rows on each side (periodic), then computes each layer on
// the rows the layers after it need - the band plus one row more on each side
// per layer still to come - with the activations kept in LDS; only the input
// X_1 and the prediction touch global memory.  Every output element is the
// same sequence of matrix-core operations as in k_conv_fwd_l (K in chunks of
// 32, the same operand layout, bias, ReLU and BF16 rounding), so the result
// is bitwise that of the layer-by-layer kernels.  The halo rows are computed
// by both neighbouring bands: 1.34x the matrix-core work of the layer-by-layer
// kernels at M = 64, L = 4, in exchange for no intermediate global traffic and
// one launch instead of L.
constexpr int kBandPix = 512;    // output pixels per band
constexpr int kBandWaves = 8;
constexpr int kBandMaxL = 4;
constexpr int kBandXS = 40;      // staged elements per pixel of a 32-channel activation
constexpr int kNoiseAhead = 8;   // rollout steps whose noise is drawn in one pass

struct BandNet {
    const unsigned short* wf[kBandMaxL];  // BF16 weights [cout16][kpad]
    const float* bias[kBandMaxL];
    int kpad[kBandMaxL];
    int cout[kBandMaxL];
};

// What the last layer of a rollout step writes: u <- (u + z) + noise (in
// place), its copy into save (if not null) and its BF16 values into channels
// 0 and 1 of the next input (4 channels per pixel; the others stay).
struct BandOut {
    float* u;
    const float* noise;   // this step's noise, same layout as u
    float* save;
    unsigned short* xnext;
};

// The weight operands of one layer for this lane (rows of Wf, kpad long, zeros
// up to NK 32) and the biases of the output channels it holds: loaded a layer
// ahead, so that their latency overlaps the layer before.
template <int NCT, int NK>
struct BandW {
    bf16x8 w[NCT][NK];
    float bo[NCT][4];
};

template <int NCT, int NK>
__device__ __forceinline__ void band_weights(BandW<NCT, NK>& W, const unsigned short* __restrict__ Wf,
                                             int kpad, const float* __restrict__ bias, int cout) {
    const int lane = threadIdx.x & (kWaveN - 1), r16 = lane & 15, g = lane >> 4;
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
        const int o = ct * 16 + r16;
#pragma unroll
        for (int i = 0; i < NK; ++i) {
            const int k = i * 32 + 8 * g;
            uint4 w = make_uint4(0u, 0u, 0u, 0u);
            if (k < kpad) w = *reinterpret_cast<const uint4*>(Wf + (size_t)o * kpad + k);
            W.w[ct][i] = __builtin_bit_cast(bf16x8, w);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int oc = ct * 16 + 4 * g + i;
            W.bo[ct][i] = oc < cout ? bias[oc] : 0.f;
        }
    }
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two FP32 values to packed BF16, round to nearest even (v_cvt_pk_bf16_f32).
__device__ __forceinline__ unsigned pack_bf16(float lo, float hi) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){lo, hi}, bf16x2));
}

// A hidden layer of the band: rows_out rows of M output pixels from the
// staged input (rows_out + 2 rows, XSI elements per pixel).  The matrix cores
// take the weights as the first operand and the activations as the second,
// so each lane ends with four consecutive output channels of one pixel, and
// writes them, ReLU and BF16 applied, as one 8-byte store into sout
// (kBandXS elements per pixel).
template <int M, int CIN, int NCT, int ROWS>
__device__ __forceinline__ void band_layer(const unsigned short* sin, unsigned short* sout,
                                           const BandW<NCT, (9 * CIN + 31) / 32>& W) {
    constexpr int NK = (9 * CIN + 31) / 32;
    constexpr int XSI = CIN == 4 ? 4 : kBandXS;
    constexpr int ntile = ROWS * M / 16, trips = (ntile + kBandWaves - 1) / kBandWaves;
    const int wave = threadIdx.x / kWaveN, lane = threadIdx.x & (kWaveN - 1);
    const int r16 = lane & 15, g = lane >> 4;
    // a known trip count, unrolled by two: the loads of one tile can overlap
    // the matrix-core work of the one before
#pragma unroll 2
    for (int j = 0; j < trips; ++j) {
        const int t = wave + kBandWaves * j;
        if (ntile % kBandWaves != 0 && t >= ntile) break;
        const int lp = t * 16 + r16;  // this lane's pixel
        const int ly = lp / M, x = lp - ly * M;
        const int xs[3] = {x == 0 ? M - 1 : x - 1, x, x == M - 1 ? 0 : x + 1};
        auto tap_pix = [&](int tp) {
            const int ty = tp / 3, tx = tp - 3 * ty;
            return (ly + ty) * M + (tx == 0 ? xs[0] : (tx == 1 ? xs[1] : xs[2]));
        };
        bf16x8 a[NK];
#pragma unroll
        for (int i = 0; i < NK; ++i) {
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if constexpr (CIN == 32) {
                v = *reinterpret_cast<const uint4*>(sin + tap_pix(i) * XSI + 8 * g);
            } else {
                const int tp = 8 * i + 2 * g;
                if (tp < 9) {
                    const uint2 lo = *reinterpret_cast<const uint2*>(sin + tap_pix(tp) * XSI);
                    v.x = lo.x;
                    v.y = lo.y;
                }
                if (tp + 1 < 9) {
                    const uint2 hi = *reinterpret_cast<const uint2*>(sin + tap_pix(tp + 1) * XSI);
                    v.z = hi.x;
                    v.w = hi.y;
                }
            }
            a[i] = __builtin_bit_cast(bf16x8, v);
        }
        f32x4 acc[NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < NK; ++i)
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.w[ct][i], a[i], acc[ct], 0, 0, 0);
        // acc[ct][i]: output channel ct 16 + 4 g + i of pixel lp
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            float z[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) z[i] = fmaxf(acc[ct][i] + W.bo[ct][i], 0.f);
            *reinterpret_cast<uint2*>(sout + lp * kBandXS + ct * 16 + 4 * g) =
                make_uint2(pack_bf16(z[0], z[1]), pack_bf16(z[2], z[3]));
        }
    }
}

// The last layer (32 -> 2 channels) of the band: R rows, kLastTPW tiles per
// wavefront.  u and the noise of this lane's pixels were loaded at the start
// of the kernel (ul, nl; lanes of group 0 hold output channels 0 and 1), so
// the layer does not wait on global memory:
// u <- (u + z) + noise, the same roundings as the prediction followed by
// k_noise or k_colour_out; the field is updated in place (each value is read
// and written by this lane only), copied to save, and its BF16 values go to
// channels 0 and 1 of the next input.
constexpr int kLastTPW = kBandPix / 16 / kBandWaves;

template <int M>
__device__ __forceinline__ void band_last(const unsigned short* sin, const BandW<1, 9>& W, size_t pix0,
                                          const float2 (&ul)[kLastTPW], const float2 (&nl)[kLastTPW],
                                          const BandOut& out) {
    const int wave = threadIdx.x / kWaveN, lane = threadIdx.x & (kWaveN - 1);
    const int r16 = lane & 15, g = lane >> 4;
#pragma unroll
    for (int j = 0; j < kLastTPW; ++j) {
        const int t = wave + kBandWaves * j;
        const int lp = t * 16 + r16;
        const int ly = lp / M, x = lp - ly * M;
        const int xs[3] = {x == 0 ? M - 1 : x - 1, x, x == M - 1 ? 0 : x + 1};
        bf16x8 a[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int ty = i / 3, tx = i - 3 * ty;
            const int pix = (ly + ty) * M + (tx == 0 ? xs[0] : (tx == 1 ? xs[1] : xs[2]));
            a[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(sin + pix * kBandXS + 8 * g));
        }
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 9; ++i) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.w[0][i], a[i], acc, 0, 0, 0);
        if (g == 0) {
            const size_t p = pix0 + (size_t)lp;
            const float vx = (ul[j].x + (acc[0] + W.bo[0][0])) + nl[j].x;
            const float vy = (ul[j].y + (acc[1] + W.bo[0][1])) + nl[j].y;
            *reinterpret_cast<float2*>(out.u + 2 * p) = make_float2(vx, vy);
            if (out.save) *reinterpret_cast<float2*>(out.save + 2 * p) = make_float2(vx, vy);
            *reinterpret_cast<unsigned*>(out.xnext + 4 * p) = (unsigned)to_bf16(vx) | ((unsigned)to_bf16(vy) << 16);
        }
    }
}

template <int L, int M>
__global__ __launch_bounds__(kBandWaves * kWaveN) void k_net_band(BandNet net,
                                                                  const unsigned short* __restrict__ X,
                                                                  BandOut out) {
    static_assert(L >= 2 && L <= kBandMaxL, "2 to 4 layers");
    static_assert(M == 32 || M == 64, "M in {32, 64}");
    constexpr int R = kBandPix / M, bands = M / R, M2 = M * M;
    // input band: R + 2 L rows of 4 channels; layer l writes R + 2 (L - 1 - l)
    // rows, the even layers into sa, the odd ones into sb
    __shared__ __align__(16) unsigned short sx[(R + 2 * L) * M * 4];
    __shared__ __align__(16) unsigned short sa[(R + 2 * (L - 1)) * M * kBandXS];
    __shared__ __align__(16) unsigned short sb[L >= 3 ? (R + 2 * (L - 2)) * M * kBandXS : 8];
    const int b = blockIdx.x / bands, y0 = (blockIdx.x - b * bands) * R;
    const size_t pix0 = (size_t)b * M2 + (size_t)y0 * M;
    // the last layer's u and noise (lanes of group 0), loaded a layer or more
    // ahead of it
    float2 ul[kLastTPW], nl[kLastTPW];
    auto load_last = [&]() {
        const int wave = threadIdx.x / kWaveN, lane = threadIdx.x & (kWaveN - 1);
#pragma unroll
        for (int j = 0; j < kLastTPW; ++j) {
            ul[j] = nl[j] = make_float2(0.f, 0.f);
            if (lane < 16) {
                const size_t p = pix0 + (size_t)((wave + kBandWaves * j) * 16 + lane);
                ul[j] = *reinterpret_cast<const float2*>(out.u + 2 * p);
                nl[j] = *reinterpret_cast<const float2*>(out.noise + 2 * p);
            }
        }
    };
    BandW<2, 2> w0;
    band_weights(w0, net.wf[0], net.kpad[0], net.bias[0], net.cout[0]);
    constexpr int npx = (R + 2 * L) * M;
    for (int pix = threadIdx.x; pix < npx; pix += kBandWaves * kWaveN) {
        const int rr = pix / M, xx = pix - rr * M;
        int yy = y0 - L + rr;
        yy += (yy < 0) ? M : 0;
        yy -= (yy >= M) ? M : 0;
        *reinterpret_cast<uint2*>(sx + pix * 4) =
            *reinterpret_cast<const uint2*>(X + ((size_t)b * M2 + (size_t)yy * M + xx) * 4);
    }
    if constexpr (L == 2) {
        BandW<1, 9> w1;
        band_weights(w1, net.wf[1], net.kpad[1], net.bias[1], net.cout[1]);
        load_last();
        __syncthreads();
        band_layer<M, 4, 2, R + 2>(sx, sa, w0);
        __syncthreads();
        band_last<M>(sa, w1, pix0, ul, nl, out);
    } else if constexpr (L == 3) {
        BandW<2, 9> w1;
        band_weights(w1, net.wf[1], net.kpad[1], net.bias[1], net.cout[1]);
        load_last();
        __syncthreads();
        band_layer<M, 4, 2, R + 4>(sx, sa, w0);
        __syncthreads();
        BandW<1, 9> w2;
        band_weights(w2, net.wf[2], net.kpad[2], net.bias[2], net.cout[2]);
        band_layer<M, 32, 2, R + 2>(sa, sb, w1);
        __syncthreads();
        band_last<M>(sb, w2, pix0, ul, nl, out);
    } else {
        // registers: the weights of the next layer are loaded while the
        // current one runs, except during layer 1, where two tiles' operands
        // and both 32-channel weight sets would not fit
        BandW<2, 9> w1;
        band_weights(w1, net.wf[1], net.kpad[1], net.bias[1], net.cout[1]);
        __syncthreads();
        band_layer<M, 4, 2, R + 6>(sx, sa, w0);
        __syncthreads();
        band_layer<M, 32, 2, R + 4>(sa, sb, w1);
        BandW<2, 9> w2;
        band_weights(w2, net.wf[2], net.kpad[2], net.bias[2], net.cout[2]);
        __syncthreads();
        BandW<1, 9> w3;
        band_weights(w3, net.wf[3], net.kpad[3], net.bias[3], net.cout[3]);
        load_last();
        band_layer<M, 32, 2, R + 2>(sb, sa, w2);
        __syncthreads();
        band_last<M>(sa, w3, pix0, ul, nl, out);
    }
}

// ---- loss --------------------------------------------------------------------------

// d = pred - target; loss partials sum d^2 (FP64, per block); the gradient of
// the mean, 2 d / n, in FP32 ([p][2]) and BF16 ([p][4], channels 2, 3 zero).
__global__ __launch_bounds__(kThreads) void k_loss(int npix, const float* __restrict__ pred,
                                                    const float* __restrict__ target, float inv_n2,
                                                    float* dZ, unsigned short* dZb, double* part) {
    __shared__ double s[kThreads / kWaveN];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (p < npix) {
        const float d0 = pred[2 * (size_t)p] - target[2 * (size_t)p];
        const float d1 = pred[2 * (size_t)p + 1] - target[2 * (size_t)p + 1];
        e = (double)d0 * d0 + (double)d1 * d1;
        const float g0 = inv_n2 * d0, g1 = inv_n2 * d1;
        dZ[2 * (size_t)p] = g0;
        dZ[2 * (size_t)p + 1] = g1;
        dZb[4 * (size_t)p + 0] = to_bf16(g0);
        dZb[4 * (size_t)p + 1] = to_bf16(g1);
        dZb[4 * (size_t)p + 2] = 0;
        dZb[4 * (size_t)p + 3] = 0;
    }
    for (int o = kWaveN / 2; o > 0; o >>= 1) e += __shfl_down(e, o, kWaveN);
    if ((threadIdx.x & (kWaveN - 1)) == 0) s[threadIdx.x / kWaveN] = e;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((s[0] + s[1]) + s[2]) + s[3];
}

__global__ __launch_bounds__(kThreads) void k_loss_final(int nparts, const double* __restrict__ part,
                                                          double inv_n, double* loss) {
    __shared__ double s[kThreads];
    double e = 0.0;
    for (int k = threadIdx.x; k < nparts; k += kThreads) e += part[k];
    s[threadIdx.x] = e;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) *loss = s[0] * inv_n;
}

// ---- input gradient ------------------------------------------------------------

// dX[q][c] = sum_{tap, o} dZ[q - off(tap)][o] W[tap][c][o] on the matrix cores,
// then through the ReLU of the layer below: dZ_below = dX where X[q][c] > 0
// (X is this layer's input, the ReLU output below), in FP32 and BF16.
__global__ __launch_bounds__(kThreads) void k_conv_bwd(Conv cv, int M, int npix,
                                                        const unsigned short* __restrict__ dZb,
                                                        const unsigned short* __restrict__ Wb,
                                                        const unsigned short* __restrict__ X,
                                                        float* dZprev, unsigned short* dZprevb) {
    const int tile = blockIdx.x * (kThreads / kWaveN) + threadIdx.x / kWaveN;
    if (tile * 16 >= npix) return;
    const int lane = threadIdx.x & (kWaveN - 1), r16 = lane & 15, g = lane >> 4;
    const int qa = tile * 16 + r16;
    const int nct = cv.cin16 / 16;
    // K = 9 cout4 in chunks of 32 (v_mfma_f32_16x16x32_bf16): lane group g
    // holds K values k0 + 8 g .. + 7 as two runs of 4, each inside one tap
    // (cout4 is a multiple of 4); values past Kb (and past the row of Wb)
    // are zeros
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < cv.Kbpad; k0 += 32) {
        bf16x4 ah[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, bh0[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}},
               bh1[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            const int k = k0 + 8 * g + 4 * hf;
            if (k < cv.Kb) {
                const int tap = k / cv.cout4, o = k - tap * cv.cout4;
                const int p = shifted(qa, tap, -1, M);
                ah[hf] = *reinterpret_cast<const bf16x4*>(dZb + (size_t)p * cv.cout4 + o);
            }
            if (k < cv.Kbpad) {
                bh0[hf] = *reinterpret_cast<const bf16x4*>(Wb + (size_t)r16 * cv.Kbpad + k);
                if (nct > 1) bh1[hf] = *reinterpret_cast<const bf16x4*>(Wb + (size_t)(16 + r16) * cv.Kbpad + k);
            }
        }
        const bf16x8 a = __builtin_bit_cast(bf16x8, __builtin_shufflevector(ah[0], ah[1], 0, 1, 2, 3, 4, 5, 6, 7));
        const bf16x8 b0 = __builtin_bit_cast(bf16x8, __builtin_shufflevector(bh0[0], bh0[1], 0, 1, 2, 3, 4, 5, 6, 7));
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc0, 0, 0, 0);
        if (nct > 1) {
            const bf16x8 b1 = __builtin_bit_cast(bf16x8, __builtin_shufflevector(bh1[0], bh1[1], 0, 1, 2, 3, 4, 5, 6, 7));
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc1, 0, 0, 0);
        }
    }
    for (int ct = 0; ct < nct; ++ct) {
        const int c = ct * 16 + r16;
        if (c >= cv.cin) continue;
        const f32x4 acc = ct == 0 ? acc0 : acc1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = tile * 16 + 4 * g + i;
            const bool on = from_bf16(X[(size_t)q * cv.cin + c]) > 0.f;
            const float d = on ? acc[i] : 0.f;
            dZprev[(size_t)q * cv.cin + c] = d;
            dZprevb[(size_t)q * cv.cin + c] = to_bf16(d);
        }
    }
}

// ---- weight gradient -----------------------------------------------------------

// Per block of kWgPix pixels: part[block][o] = sum_p X[p + off(tap)][c] dZ[p][o']
// for o = (tap cin + c) cout + o' (the layout of W), then the bias sums
// sum_p dZ[p][o'] at o = 9 cin cout + o'.  Pixels are taken in order, so the
// sums are reproducible.
__global__ __launch_bounds__(kThreads) void k_wgrad_part(Conv cv, int M, int npix,
                                                          const unsigned short* __restrict__ X,
                                                          const float* __restrict__ dZ,
                                                          float* part) {
    __shared__ float xs[kWgStage][9 * kMaxC];
    __shared__ float zs[kWgStage][kMaxC];
    const int nW = cv.K * cv.cout, nO = nW + cv.cout;
    float acc[kWgPerThread];
#pragma unroll
    for (int j = 0; j < kWgPerThread; ++j) acc[j] = 0.f;
    const int p0 = blockIdx.x * kWgPix;
    const int p1 = min(npix, p0 + kWgPix);
    for (int pb = p0; pb < p1; pb += kWgStage) {
        const int np = min(kWgStage, p1 - pb);
        for (int t = threadIdx.x; t < np * cv.K; t += kThreads) {
            const int pp = t / cv.K, k = t - pp * cv.K;
            const int tap = k / cv.cin, c = k - tap * cv.cin;
            xs[pp][k] = from_bf16(X[(size_t)shifted(pb + pp, tap, 1, M) * cv.cin + c]);
        }
        for (int t = threadIdx.x; t < np * cv.cout; t += kThreads) {
            const int pp = t / cv.cout, o = t - pp * cv.cout;
            zs[pp][o] = dZ[(size_t)(pb + pp) * cv.cout + o];
        }
        __syncthreads();
        for (int pp = 0; pp < np; ++pp) {
#pragma unroll
            for (int j = 0; j < kWgPerThread; ++j) {
                const int o = threadIdx.x + j * kThreads;
                if (o < nW) {
                    const int k = o / cv.cout, oo = o - k * cv.cout;
                    acc[j] = fmaf(xs[pp][k], zs[pp][oo], acc[j]);
                } else if (o < nO) {
                    acc[j] += zs[pp][o - nW];
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < kWgPerThread; ++j) {
        const int o = threadIdx.x + j * kThreads;
        if (o < nO) part[(size_t)blockIdx.x * nO + o] = acc[j];
    }
}

// grad[o] = sum over the blocks in order of part[block][o].
__global__ void k_wgrad_reduce(int nO, int nblocks, const float* __restrict__ part, float* grad) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= nO) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * nO + o];
    grad[o] = s;
}

// ---- optimiser and rollout -----------------------------------------------------

__global__ void k_adam(int n, float* w, float* m, float* v, const float* __restrict__ g, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// u_next = pred + sigma_c alpha, alpha Gaussian by Box-Muller from
// Philox4x32-10 with counter (point, component, step, 0) and the seed as key
// (point = b M^2 + pixel over a batch).  Also writes u_next rounded to BF16
// into channels 0 and 1 of the next forward pass's input X (cin channels per
// pixel; the condition channels stay as they are), and u_next to `save` too
// when that is not null (a saved step of a rollout).
__global__ void k_noise(int n, const float* __restrict__ pred, float s0, float s1, uint32_t step,
                        uint32_t k0, uint32_t k1, float* unext, int cin, unsigned short* X,
                        float* save) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;  // t = 2 point + component
    if (t >= n) return;
    const uint4 w = dpd::philox4x32_10(make_uint4((uint32_t)(t >> 1), (uint32_t)(t & 1), step, 0u), k0, k1);
    const float alpha = dpd::alpha_from_words(0, make_uint2(w.x, w.y));
    const float v = pred[t] + ((t & 1) ? s1 : s0) * alpha;
    unext[t] = v;
    if (save) save[t] = v;
    X[(size_t)(t >> 1) * cin + (t & 1)] = to_bf16(v);
}

constexpr int kColourMaxM = 64;  // largest grid side of a filtered rollout

// ---- coloured rollout noise -----------------------------------------------------
// noise = s_c (h * w) for the periodic convolution *, computed as
// IDFT(DFT(h) DFT(w)) with FP32 direct DFTs of length M along rows and columns
// (O(M^3) per field instead of O(M^4)); twiddles tw[m] = e^{-2 pi i m / M}
// from an LDS table.  One block per (row or column, field), 2 M threads:
// thread t = 2 index + component.  All sums run in a fixed order.

__device__ __forceinline__ void twiddle_table(int M, float2* tw) {
    for (int m = threadIdx.x; m < M; m += blockDim.x) {
        float sn, cs;
        sincospif(2.0f * (float)m / (float)M, &sn, &cs);
        tw[m] = make_float2(cs, -sn);
    }
}

// Hhat[l][k] = sum_{j,i} h[j][i] tw[(l j + k i) mod M], once per rollout.
__global__ __launch_bounds__(kThreads) void k_filter_hat(int M, const float* __restrict__ h, float2* Hhat) {
    __shared__ float2 tw[kColourMaxM];
    twiddle_table(M, tw);
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * M) return;
    const int l = t / M, k = t - l * M;
    float re = 0.f, im = 0.f;
    for (int j = 0; j < M; ++j)
        for (int i = 0; i < M; ++i) {
            const float2 e = tw[(l * j + k * i) % M];
            const float v = h[j * M + i];
            re = fmaf(v, e.x, re);
            im = fmaf(v, e.y, im);
        }
    Hhat[t] = make_float2(re, im);
}

// Row j of field b at step step0 + q (blockIdx.y = q B + b): white numbers
// w[j][i][c] = alpha(b M^2 + j M + i, c, step) (Philox4x32-10 and Box-Muller,
// as k_noise), then A[q B + b][j][k][c] = sum_i w[j][i][c] tw[k i mod M] for
// k <= M / 2 (the rest of a real field's spectrum is conjugate to it).
__global__ void k_colour_rows(int M, int B, uint32_t step0, uint32_t k0, uint32_t k1, float2* A) {
    __shared__ float2 tw[kColourMaxM];
    __shared__ float sw[2 * kColourMaxM];
    const int j = blockIdx.x, bq = blockIdx.y, t = threadIdx.x;
    const int q = bq / B, b = bq - q * B;
    const uint32_t step = step0 + (uint32_t)q;
    twiddle_table(M, tw);
    const uint32_t point = (uint32_t)(((size_t)b * M + j) * M + (t >> 1));
    const uint4 r = dpd::philox4x32_10(make_uint4(point, (uint32_t)(t & 1), step, 0u), k0, k1);
    sw[t] = dpd::alpha_from_words(0, make_uint2(r.x, r.y));
    __syncthreads();
    const int k = t >> 1, c = t & 1;
    if (k > M / 2) return;
    float re = 0.f, im = 0.f;
    for (int i = 0, m = 0; i < M; ++i) {  // m = k i mod M
        const float2 e = tw[m];
        const float v = sw[2 * i + c];
        re = fmaf(v, e.x, re);
        im = fmaf(v, e.y, im);
        m += k;
        m -= (m >= M) ? M : 0;
    }
    A[(((size_t)bq * M + j) * M + k) * 2 + c] = make_float2(re, im);
}

// Column k <= M / 2 of field b: the column DFT, times Hhat, and the inverse
// column DFT (without its 1/M), in place: A[b][j][k][c] <- sum_l conj(tw[l j])
// Hhat[l][k] sum_j' A[b][j'][k][c] tw[l j'].
__global__ void k_colour_cols(int M, const float2* __restrict__ Hhat, float2* A) {
    __shared__ float2 tw[kColourMaxM];
    __shared__ float2 sa[2 * kColourMaxM], sb[2 * kColourMaxM];
    const int k = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
    const int q = t >> 1, c = t & 1;
    twiddle_table(M, tw);
    float2* col = A + ((size_t)b * M * M + k) * 2 + c;  // + 2 M row
    sa[t] = col[(size_t)2 * M * q];
    __syncthreads();
    float re = 0.f, im = 0.f;  // forward: l = q
    for (int jj = 0, m = 0; jj < M; ++jj) {  // m = q jj mod M
        const float2 e = tw[m], z = sa[2 * jj + c];
        re = fmaf(z.x, e.x, fmaf(-z.y, e.y, re));
        im = fmaf(z.y, e.x, fmaf(z.x, e.y, im));
        m += q;
        m -= (m >= M) ? M : 0;
    }
    const float2 hh = Hhat[q * M + k];
    sb[t] = make_float2(re * hh.x - im * hh.y, re * hh.y + im * hh.x);
    __syncthreads();
    re = 0.f;
    im = 0.f;  // inverse: j = q
    for (int l = 0, m = 0; l < M; ++l) {  // m = l q mod M
        const float2 e = tw[m], z = sb[2 * l + c];
        re = fmaf(z.x, e.x, fmaf(z.y, e.y, re));
        im = fmaf(z.y, e.x, fmaf(-z.x, e.y, im));
        m += q;
        m -= (m >= M) ? M : 0;
    }
    col[(size_t)2 * M * q] = make_float2(re, im);
}

// Row j of field b: the inverse row DFT's real part over M^2 is the noise;
// u_next = pred + s_c noise, also written to the next input X (and to `save`)
// as in k_noise.
// h and w are real, so the filtered spectrum is Hermitian and so is each row
// of its inverse column transform: C[j][M - k] = conj(C[j][k]) fills the
// columns past M / 2.
__global__ void k_colour_out(int M, const float2* __restrict__ A, const float* __restrict__ pred,
                             float s0, float s1, float* unext, int cin, unsigned short* X,
                             float* save) {
    __shared__ float2 tw[kColourMaxM];
    __shared__ float2 sa[2 * kColourMaxM];
    const int j = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
    twiddle_table(M, tw);
    {
        const int k = t >> 1, c = t & 1;
        const int kk = k <= M / 2 ? k : M - k;
        const float2 z = A[(((size_t)b * M + j) * M + kk) * 2 + c];
        sa[t] = k <= M / 2 ? z : make_float2(z.x, -z.y);
    }
    __syncthreads();
    const int i = t >> 1, c = t & 1;
    float re = 0.f;
    for (int k = 0, m = 0; k < M; ++k) {  // m = k i mod M
        const float2 e = tw[m], z = sa[2 * k + c];
        re = fmaf(z.x, e.x, fmaf(z.y, e.y, re));
        m += i;
        m -= (m >= M) ? M : 0;
    }
    const float inv = 1.0f / (float)(M * M);
    const size_t p = ((size_t)b * M + j) * M + i;
    const float v = pred[2 * p + c] + (c ? s1 : s0) * (re * inv);
    unext[2 * p + c] = v;
    if (save) save[2 * p + c] = v;
    X[p * cin + c] = to_bf16(v);
}

// The noise of S steps ahead, for the rollout kernel that adds it: noise[q][t]
// = s_c alpha(t / 2, c, step0 + q) (t = 2 point + component; as k_noise) and,
// filtered, noise[q B + b][p][c] = s_c (the inverse row transform's real part
// over M^2) (as k_colour_out); the sums are the same as there.
__global__ void k_noise_steps(int nf, int S, uint32_t step0, uint32_t k0, uint32_t k1, float s0, float s1,
                              float* noise) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)nf * S) return;
    const int q = (int)(t / nf), tt = (int)(t - (long long)q * nf);
    const uint4 w = dpd::philox4x32_10(make_uint4((uint32_t)(tt >> 1), (uint32_t)(tt & 1), step0 + (uint32_t)q, 0u),
                                       k0, k1);
    const float alpha = dpd::alpha_from_words(0, make_uint2(w.x, w.y));
    noise[t] = ((tt & 1) ? s1 : s0) * alpha;
}

__global__ void k_colour_noise(int M, const float2* __restrict__ A, float s0, float s1, float* noise) {
    __shared__ float2 tw[kColourMaxM];
    __shared__ float2 sa[2 * kColourMaxM];
    const int j = blockIdx.x, bq = blockIdx.y, t = threadIdx.x;
    twiddle_table(M, tw);
    {
        const int k = t >> 1, c = t & 1;
        const int kk = k <= M / 2 ? k : M - k;
        const float2 z = A[(((size_t)bq * M + j) * M + kk) * 2 + c];
        sa[t] = k <= M / 2 ? z : make_float2(z.x, -z.y);
    }
    __syncthreads();
    const int i = t >> 1, c = t & 1;
    float re = 0.f;
    for (int k = 0, m = 0; k < M; ++k) {  // m = k i mod M
        const float2 e = tw[m], z = sa[2 * k + c];
        re = fmaf(z.x, e.x, fmaf(z.y, e.y, re));
        m += i;
        m -= (m >= M) ? M : 0;
    }
    const float inv = 1.0f / (float)(M * M);
    noise[(((size_t)bq * M + j) * M + i) * 2 + c] = (c ? s1 : s0) * (re * inv);
}

// The same three passes for the rollout's noise drawn ahead, with each
// length-M transform (M = kRadixP Q, a power of two) in two stages instead
// of M-term sums: for n = Q n1 + n2 and k = k1 + P k2,
//   X[k1 + P k2] = sum_{n2 < Q} W^(P n2 k2) [W^(n2 k1) sum_{n1 < P} x[Q n1 + n2] W^(Q n1 k1)],
// W = e^{-2 pi i / M} (conjugated for the inverse transforms): P + Q + 1
// complex products per output instead of M.  Stage outputs go through LDS.
constexpr int kRadixP = 8;

// The product of z and w (inv: of z and conj(w)).
__device__ __forceinline__ float2 cmul(float2 z, float2 w, bool inv) {
    if (inv) w.y = -w.y;
    return make_float2(z.x * w.x - z.y * w.y, z.x * w.y + z.y * w.x);
}

// Stage 1 for slot idx = n2 P + k1 of component c: x holds M complex values
// [n][c] (or M real values [n][c] with REAL).
template <bool REAL>
__device__ __forceinline__ float2 radix_stage1(const void* xv, int c, int idx, int M, const float2* tw, bool inv) {
    const int Q = M / kRadixP, n2 = idx / kRadixP, k1 = idx - n2 * kRadixP;
    float re = 0.f, im = 0.f;
#pragma unroll
    for (int n1 = 0; n1 < kRadixP; ++n1) {
        float2 e = tw[(Q * n1 * k1) & (M - 1)];
        if (inv) e.y = -e.y;
        if constexpr (REAL) {
            const float v = reinterpret_cast<const float*>(xv)[2 * (Q * n1 + n2) + c];
            re = fmaf(v, e.x, re);
            im = fmaf(v, e.y, im);
        } else {
            const float2 z = reinterpret_cast<const float2*>(xv)[2 * (Q * n1 + n2) + c];
            re = fmaf(z.x, e.x, fmaf(-z.y, e.y, re));
            im = fmaf(z.y, e.x, fmaf(z.x, e.y, im));
        }
    }
    return cmul(make_float2(re, im), tw[(n2 * k1) & (M - 1)], inv);
}

// Stage 2 for output k (k1 = k mod P, k2 = k / P) of component c from the
// stage-1 values y [n2 P + k1][c].
__device__ __forceinline__ float2 radix_stage2(const float2* y, int c, int k, int M, const float2* tw, bool inv) {
    const int Q = M / kRadixP, k1 = k & (kRadixP - 1), k2 = k / kRadixP;
    float re = 0.f, im = 0.f;
    for (int n2 = 0; n2 < Q; ++n2) {
        float2 e = tw[(kRadixP * n2 * k2) & (M - 1)];
        if (inv) e.y = -e.y;
        const float2 z = y[2 * (n2 * kRadixP + k1) + c];
        re = fmaf(z.x, e.x, fmaf(-z.y, e.y, re));
        im = fmaf(z.y, e.x, fmaf(z.x, e.y, im));
    }
    return make_float2(re, im);
}

constexpr int kColGroupThreads = 1024;  // threads of a filtered-noise block

// The filtered noise of k_colour_rows, k_colour_cols and k_colour_noise by
// two-stage transforms, one field-step per block, with the half spectrum
// [j][k <= M/2][c] held in LDS between the passes: white numbers and the
// forward row transforms; the forward column transforms, the filter and the
// inverse column transforms; the inverse row transforms of the
// Hermitian-extended rows, real part over M^2, times s_c.  The block takes
// G = kColGroupThreads / (2 M) rows or columns at a time.  In the column pass
// thread t owns component t & 1 of row (t >> 1) / G of column (t >> 1) mod G,
// and every column's 2 M values are padded by one in LDS, so that the columns
// a wavefront works on fall on different banks.  Only the noise goes to
// global memory.
__global__ __launch_bounds__(kColGroupThreads) void k_colour_fused_r(int M, int B, uint32_t step0,
                                                                     uint32_t k0, uint32_t k1,
                                                                     const float2* __restrict__ Hhat,
                                                                     float s0, float s1, float* noise) {
    constexpr int kHalfMax = kColourMaxM / 2 + 1;
    __shared__ float2 tw[kColourMaxM];
    __shared__ float2 S[kColourMaxM * kHalfMax * 2];
    __shared__ float rw[kColGroupThreads];
    __shared__ float2 ry[kColGroupThreads];
    __shared__ float2 sa[kColGroupThreads + kColGroupThreads / 4], sy[kColGroupThreads + kColGroupThreads / 4];
    const int G = kColGroupThreads / (2 * M), CS = 2 * M + 1, H = M / 2 + 1;
    const int bq = blockIdx.x, t = threadIdx.x;
    const int q = bq / B, b = bq - q * B;
    twiddle_table(M, tw);
    {  // rows: white numbers, forward transform, half spectrum into S
        const int g = t / (2 * M), lt = t - g * 2 * M, idx = lt >> 1, c = lt & 1;
        float* w = rw + g * 2 * M;
        float2* y = ry + g * 2 * M;
        for (int j0 = 0; j0 < M; j0 += G) {
            const int j = j0 + g;
            const uint32_t point = (uint32_t)(((size_t)b * M + j) * M + idx);
            const uint4 r = dpd::philox4x32_10(make_uint4(point, (uint32_t)c, step0 + (uint32_t)q, 0u), k0, k1);
            w[lt] = dpd::alpha_from_words(0, make_uint2(r.x, r.y));
            __syncthreads();
            y[lt] = radix_stage1<true>(w, c, idx, M, tw, false);
            __syncthreads();
            if (idx <= M / 2) S[(j * H + idx) * 2 + c] = radix_stage2(y, c, idx, M, tw, false);
        }
    }
    __syncthreads();
    {  // columns k <= M / 2: forward transform, times Hhat, inverse, in place
        const int c = t & 1, g = (t >> 1) % G, idx = (t >> 1) / G;
        float2* ca = sa + g * CS;
        float2* cy = sy + g * CS;
        for (int kb = 0; kb < H; kb += G) {
            const int k = kb + g;
            const bool valid = k < H;
            ca[2 * idx + c] = valid ? S[(idx * H + k) * 2 + c] : make_float2(0.f, 0.f);
            __syncthreads();
            cy[2 * idx + c] = radix_stage1<false>(ca, c, idx, M, tw, false);
            __syncthreads();
            const float2 hh = valid ? Hhat[idx * M + k] : make_float2(0.f, 0.f);
            ca[2 * idx + c] = cmul(radix_stage2(cy, c, idx, M, tw, false), hh, false);  // l = idx
            __syncthreads();
            cy[2 * idx + c] = radix_stage1<false>(ca, c, idx, M, tw, true);
            __syncthreads();
            const float2 out = radix_stage2(cy, c, idx, M, tw, true);  // j = idx
            if (valid) S[(idx * H + k) * 2 + c] = out;
        }
    }
    __syncthreads();
    {  // rows: Hermitian extension, inverse transform, real part over M^2, times s_c
        const int g = t / (2 * M), lt = t - g * 2 * M, idx = lt >> 1, c = lt & 1;
        float2* x = sa + g * 2 * M;
        float2* y = sy + g * 2 * M;
        const float inv = 1.0f / (float)(M * M);
        for (int j0 = 0; j0 < M; j0 += G) {
            const int j = j0 + g;
            const int kk = idx <= M / 2 ? idx : M - idx;
            const float2 z = S[(j * H + kk) * 2 + c];
            x[lt] = idx <= M / 2 ? z : make_float2(z.x, -z.y);
            __syncthreads();
            y[lt] = radix_stage1<false>(x, c, idx, M, tw, true);
            __syncthreads();
            const float re = radix_stage2(y, c, idx, M, tw, true).x;  // i = idx
            noise[(((size_t)bq * M + j) * M + idx) * 2 + c] = (c ? s1 : s0) * (re * inv);
        }
    }
}

// ---- field statistics ------------------------------------------------------------

// Row transforms A[f][j][k][c] = sum_i u[f][j][i][c] e^{-2 pi i k i / M}
// (complex, FP32), one thread per (field, row, k).
__global__ void k_dft_rows(int nf, int M, const float* __restrict__ u, float2* A) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)nf * M * M) return;
    const int k = (int)(t % M);
    const long long fj = t / M;  // field * M + row
    const float* row = u + fj * M * 2;
    float re0 = 0.f, im0 = 0.f, re1 = 0.f, im1 = 0.f;
    for (int i = 0; i < M; ++i) {
        float s, c;
        sincospif(2.0f * (float)((k * i) % M) / (float)M, &s, &c);  // exact angle index
        const float a0 = row[2 * i], a1 = row[2 * i + 1];
        re0 = fmaf(a0, c, re0);
        im0 = fmaf(-a0, s, im0);
        re1 = fmaf(a1, c, re1);
        im1 = fmaf(-a1, s, im1);
    }
    A[(fj * M + k) * 2 + 0] = make_float2(re0, im0);
    A[(fj * M + k) * 2 + 1] = make_float2(re1, im1);
}

// Column transforms and power: P[l][k] = sum_f sum_c |sum_j A[f][j][k][c]
// e^{-2 pi i l j / M}|^2 / M^4, summed over the fields in order (FP64), one
// thread per (l, k).
__global__ void k_dft_cols_power(int nf, int M, const float2* __restrict__ A, double* P) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * M) return;
    const int l = t / M, k = t % M;
    double acc = 0.0;
    for (int f = 0; f < nf; ++f) {
        float re0 = 0.f, im0 = 0.f, re1 = 0.f, im1 = 0.f;
        for (int j = 0; j < M; ++j) {
            float s, c;
            sincospif(2.0f * (float)((l * j) % M) / (float)M, &s, &c);
            const float2 a0 = A[(((long long)f * M + j) * M + k) * 2 + 0];
            const float2 a1 = A[(((long long)f * M + j) * M + k) * 2 + 1];
            // (a.x + i a.y)(c - i s)
            re0 += a0.x * c + a0.y * s;
            im0 += a0.y * c - a0.x * s;
            re1 += a1.x * c + a1.y * s;
            im1 += a1.y * c - a1.x * s;
        }
        acc += (double)re0 * re0 + (double)im0 * im0 + (double)re1 * re1 + (double)im1 * im1;
    }
    const double M2 = (double)M * M;
    P[t] = acc / (M2 * M2);
}

__global__ void k_zero(float* p, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

}  // namespace nn

// ======================================================================= host

namespace {

using namespace nn;

thread_local std::string g_nn_error = "no error";

std::string nfmt(const char* f, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, f);
    vsnprintf(buf, sizeof buf, f, ap);
    va_end(ap);
    return buf;
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
int up(int x, int m) { return (x + m - 1) / m * m; }
int blocks(long long n, int b = kThreads) { return (int)((n + b - 1) / b); }

struct Net {
    dpd_nn_params p;
    std::vector<Conv> conv;
    std::vector<size_t> woff, boff;  // parameter offsets of W_l and b_l
    long long nparam = 0;
    size_t total = 0;
    // workspace offsets
    size_t o_w, o_m, o_v, o_g, o_pred, o_dz[2], o_dzb[2], o_part, o_lpart, o_loss, o_u;
    std::vector<size_t> o_x, o_wf, o_wb;
};

int plan(const dpd_nn_params* p, Net* n, std::string* err) {
    if (!p) { *err = "params is NULL"; return DPD_EINVAL; }
    if (p->M < 4 || p->M > 256 || p->M % 4) { *err = "M must be a multiple of 4 in [4, 256]"; return DPD_EINVAL; }
    if (p->c_in < 4 || p->c_in > kMaxC || p->c_in % 4) { *err = "c_in must be a multiple of 4 in [4, 32]"; return DPD_EINVAL; }
    if (p->width != 16 && p->width != 32) { *err = "width must be 16 or 32"; return DPD_EINVAL; }
    if (p->layers < 1 || p->layers > 8) { *err = "layers must be in [1, 8]"; return DPD_EINVAL; }
    if (p->max_batch < 1 || (long long)p->max_batch * p->M * p->M > (1LL << 26)) {
        *err = "max_batch must be >= 1 with max_batch M^2 <= 2^26";
        return DPD_EINVAL;
    }
    n->p = *p;
    n->conv.clear();
    n->woff.clear();
    n->boff.clear();
    long long off = 0;
    for (int l = 0; l < p->layers; ++l) {
        Conv c;
        c.cin = l == 0 ? p->c_in : p->width;
        c.cout = l == p->layers - 1 ? 2 : p->width;
        c.K = 9 * c.cin;
        c.Kpad = up(c.K, 16);
        c.cout16 = up(c.cout, 16);
        c.cout4 = up(c.cout, 4);
        c.Kb = 9 * c.cout4;
        c.Kbpad = up(c.Kb, 16);
        c.cin16 = up(c.cin, 16);
        n->conv.push_back(c);
        n->woff.push_back((size_t)off);
        off += (long long)c.K * c.cout;
        n->boff.push_back((size_t)off);
        off += c.cout;
    }
    n->nparam = off;
    const size_t npix = (size_t)p->max_batch * p->M * p->M;
    const size_t P = (size_t)off;
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o = al256(o + b); return r; };
    n->o_w = take(P * 4);
    n->o_m = take(P * 4);
    n->o_v = take(P * 4);
    n->o_g = take(P * 4);
    n->o_pred = take(npix * 2 * 4);
    const int cmax = std::max(p->width, 4);
    for (int k = 0; k < 2; ++k) {
        n->o_dz[k] = take(npix * cmax * 4);
        n->o_dzb[k] = take(npix * cmax * 2);
    }
    const size_t nwb = (npix + kWgPix - 1) / kWgPix;
    n->o_part = take(nwb * kWgOutMax * 4);
    n->o_lpart = take(((npix + kThreads - 1) / kThreads) * 8);
    n->o_loss = take(8);
    n->o_u = take(npix * 2 * 4 * 2);  // rollout fields and their predictions
    n->o_x.clear();
    n->o_wf.clear();
    n->o_wb.clear();
    for (const Conv& c : n->conv) {
        n->o_x.push_back(take(npix * c.cin * 2));
        n->o_wf.push_back(take((size_t)c.cout16 * c.Kpad * 2));
        n->o_wb.push_back(take((size_t)c.cin16 * c.Kbpad * 2));
    }
    n->total = o;
    return DPD_OK;
}

}  // namespace

struct dpd_nn {
    Net net;
    hipStream_t stream;
    char* ws;
    int adam_t;
    std::string err;
};

namespace {

int nfail(dpd_nn* h, int code, const std::string& m) {
    if (h) h->err = m;
    g_nn_error = m;
    return code;
}

#define NCHK(h, expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return nfail((h), DPD_EHIP, nfmt("%s: %s", #expr, hipGetErrorString(e_))); \
    } while (0)

#define NLAUNCH(h)                                                                        \
    do {                                                                                  \
        hipError_t e_ = hipGetLastError();                                                \
        if (e_ != hipSuccess)                                                             \
            return nfail((h), DPD_EHIP, nfmt("kernel launch: %s", hipGetErrorString(e_))); \
    } while (0)

template <class T>
T* at(dpd_nn* h, size_t off) { return reinterpret_cast<T*>(h->ws + off); }

// BF16 weight layouts from the master weights.
int cast_weights(dpd_nn* h) {
    const Net& n = h->net;
    for (size_t l = 0; l < n.conv.size(); ++l) {
        const Conv& c = n.conv[l];
        const int nt = std::max(c.cout16 * c.Kpad, c.cin16 * c.Kbpad);
        hipLaunchKernelGGL(k_cast_weights, dim3(blocks(nt)), dim3(kThreads), 0, h->stream, c,
                           (const float*)at<float>(h, n.o_w + 4 * n.woff[l]),
                           at<unsigned short>(h, n.o_wf[l]), at<unsigned short>(h, n.o_wb[l]));
    }
    NLAUNCH(h);
    return DPD_OK;
}

// Forward pass of B fields: activations stay in the workspace, pred -> out.
// With prepared = true the BF16 weights and the first activation are already
// in place (a rollout's later steps).
int forward(dpd_nn* h, const float* u, const float* cond, int B, float* pred, bool prepared = false) {
    const Net& n = h->net;
    const int M = n.p.M, M2 = M * M, npix = B * M2;
    if (!prepared) {
        int rc = cast_weights(h);
        if (rc) return rc;
        hipLaunchKernelGGL(k_input, dim3(blocks(npix)), dim3(kThreads), 0, h->stream, npix, M2,
                           n.p.c_in, u, cond, at<unsigned short>(h, n.o_x[0]));
    }
    const int ntile = npix / 16;
    const int grid = (ntile + 3) / 4;
    for (size_t l = 0; l < n.conv.size(); ++l) {
        const Conv& c = n.conv[l];
        const unsigned short* X = at<unsigned short>(h, n.o_x[l]);
        const unsigned short* Wf = at<unsigned short>(h, n.o_wf[l]);
        const float* b = at<float>(h, n.o_w + 4 * n.boff[l]);
        const bool last = l + 1 == n.conv.size();
        unsigned short* Xn = last ? nullptr : at<unsigned short>(h, n.o_x[l + 1]);
        const float* uu = last ? u : nullptr;
        float* pp = last ? pred : nullptr;
        auto kern = last ? k_conv_fwd<true> : k_conv_fwd<false>;
        int g = grid;
        if (c.cin == 32 || c.cin == 16 || c.cin == 4) {
            const int nct = c.cout16 / 16;
            if (c.cin == 4)
                kern = last ? (nct == 1 ? k_conv_fwd_c<4, 1, true> : k_conv_fwd_c<4, 2, true>)
                            : (nct == 1 ? k_conv_fwd_c<4, 1, false> : k_conv_fwd_c<4, 2, false>);
            else if (c.cin == 32)
                kern = last ? (nct == 1 ? k_conv_fwd_c<32, 1, true> : k_conv_fwd_c<32, 2, true>)
                            : (nct == 1 ? k_conv_fwd_c<32, 1, false> : k_conv_fwd_c<32, 2, false>);
            else
                kern = last ? (nct == 1 ? k_conv_fwd_c<16, 1, true> : k_conv_fwd_c<16, 2, true>)
                            : (nct == 1 ? k_conv_fwd_c<16, 1, false> : k_conv_fwd_c<16, 2, false>);
            const int waves = (ntile + kConvTPW - 1) / kConvTPW;
            g = (waves + kThreads / kWaveN - 1) / (kThreads / kWaveN);
            if ((c.cin == 32 || c.cin == 16 || c.cin == 4) && (M == 16 || M == 32 || M == 64) &&
                npix % kLdsPix == 0) {
                if (c.cin == 4)
                    kern = last ? (nct == 1 ? k_conv_fwd_l<4, 1, true> : k_conv_fwd_l<4, 2, true>)
                                : (nct == 1 ? k_conv_fwd_l<4, 1, false> : k_conv_fwd_l<4, 2, false>);
                else if (c.cin == 32)
                    kern = last ? (nct == 1 ? k_conv_fwd_l<32, 1, true> : k_conv_fwd_l<32, 2, true>)
                                : (nct == 1 ? k_conv_fwd_l<32, 1, false> : k_conv_fwd_l<32, 2, false>);
                else
                    kern = last ? (nct == 1 ? k_conv_fwd_l<16, 1, true> : k_conv_fwd_l<16, 2, true>)
                                : (nct == 1 ? k_conv_fwd_l<16, 1, false> : k_conv_fwd_l<16, 2, false>);
                g = npix / kLdsPix;
            }
        }
        hipLaunchKernelGGL(kern, dim3(g), dim3(kThreads), 0, h->stream, c, M, npix, X, Wf, b, Xn, uu, pp);
    }
    NLAUNCH(h);
    return DPD_OK;
}

// The forward pass of a rollout step as one kernel (k_net_band) where the
// network's shape allows it: c_in = 4, width 32, 2 to 4 layers, M in {32, 64}.
// Needs the BF16 weights and the first input in place, as forward(prepared).
bool band_fits(const Net& n) {
    return n.p.c_in == 4 && n.p.width == 32 && n.p.layers >= 2 && n.p.layers <= kBandMaxL &&
           (n.p.M == 32 || n.p.M == 64);
}

// One rollout step of the whole network as one kernel: reads the BF16 input
// X, writes u <- (u + net) + noise, save and the next input Xn.
int band_step(dpd_nn* h, int B, const unsigned short* X, unsigned short* Xn, float* u, const float* noise,
              float* save) {
    const Net& n = h->net;
    BandNet bn = {};
    for (int l = 0; l < n.p.layers; ++l) {
        bn.wf[l] = at<unsigned short>(h, n.o_wf[l]);
        bn.bias[l] = at<float>(h, n.o_w + 4 * n.boff[l]);
        bn.kpad[l] = n.conv[l].Kpad;
        bn.cout[l] = n.conv[l].cout;
    }
    const BandOut out = {u, noise, save, Xn};
    const int M = n.p.M, L = n.p.layers, grid = B * (M * M / kBandPix);
    auto kern = M == 64 ? (L == 2 ? k_net_band<2, 64> : (L == 3 ? k_net_band<3, 64> : k_net_band<4, 64>))
                        : (L == 2 ? k_net_band<2, 32> : (L == 3 ? k_net_band<3, 32> : k_net_band<4, 32>));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBandWaves * kWaveN), 0, h->stream, bn, X, out);
    NLAUNCH(h);
    return DPD_OK;
}

int gradient(dpd_nn* h, const float* u, const float* cond, const float* target, int B,
             float* grad, double* loss) {
    const Net& n = h->net;
    const int M = n.p.M, M2 = M * M, npix = B * M2;
    float* pred = at<float>(h, n.o_pred);
    int rc = forward(h, u, cond, B, pred);
    if (rc) return rc;
    const int nlb = blocks(npix);
    double* lpart = at<double>(h, n.o_lpart);
    hipLaunchKernelGGL(k_loss, dim3(nlb), dim3(kThreads), 0, h->stream, npix, (const float*)pred,
                       target, (float)(2.0 / (2.0 * npix)), at<float>(h, n.o_dz[0]),
                       at<unsigned short>(h, n.o_dzb[0]), lpart);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kThreads), 0, h->stream, nlb,
                       (const double*)lpart, 1.0 / (2.0 * npix), loss);
    NLAUNCH(h);
    const int ntile = npix / 16;
    const int grid = (ntile + 3) / 4;
    const int nwb = (npix + kWgPix - 1) / kWgPix;
    float* part = at<float>(h, n.o_part);
    int cur = 0;  // dZ of layer l sits in buffer cur
    for (int l = (int)n.conv.size() - 1; l >= 0; --l) {
        const Conv& c = n.conv[l];
        const int nO = c.K * c.cout + c.cout;
        hipLaunchKernelGGL(k_wgrad_part, dim3(nwb), dim3(kThreads), 0, h->stream, c, M, npix,
                           (const unsigned short*)at<unsigned short>(h, n.o_x[l]),
                           (const float*)at<float>(h, n.o_dz[cur]), part);
        hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks(nO)), dim3(kThreads), 0, h->stream, nO, nwb,
                           (const float*)part, grad + n.woff[l]);
        if (l > 0) {
            hipLaunchKernelGGL(k_conv_bwd, dim3(grid), dim3(kThreads), 0, h->stream, c, M, npix,
                               (const unsigned short*)at<unsigned short>(h, n.o_dzb[cur]),
                               (const unsigned short*)at<unsigned short>(h, n.o_wb[l]),
                               (const unsigned short*)at<unsigned short>(h, n.o_x[l]),
                               at<float>(h, n.o_dz[1 - cur]), at<unsigned short>(h, n.o_dzb[1 - cur]));
            cur = 1 - cur;
        }
        NLAUNCH(h);
    }
    return DPD_OK;
}

int adam(dpd_nn* h, const float* grad, float lr, float b1, float b2, float eps) {
    const Net& n = h->net;
    h->adam_t += 1;
    const float c1 = (float)(1.0 - std::pow((double)b1, h->adam_t));
    const float c2 = (float)(1.0 - std::pow((double)b2, h->adam_t));
    hipLaunchKernelGGL(k_adam, dim3(blocks(n.nparam)), dim3(kThreads), 0, h->stream, (int)n.nparam,
                       at<float>(h, n.o_w), at<float>(h, n.o_m), at<float>(h, n.o_v), grad, lr, b1,
                       b2, eps, c1, c2);
    NLAUNCH(h);
    return DPD_OK;
}

int check_batch(dpd_nn* h, int B) {
    if (B < 1 || B > h->net.p.max_batch)
        return nfail(h, DPD_EINVAL, nfmt("B = %d outside [1, %d]", B, h->net.p.max_batch));
    return DPD_OK;
}

}  // namespace

extern "C" {

int dpd_nn_param_count(const dpd_nn_params* p, int64_t* count) {
    Net n;
    std::string e;
    int rc = plan(p, &n, &e);
    if (rc) return nfail(nullptr, rc, e);
    if (!count) return nfail(nullptr, DPD_EINVAL, "count is NULL");
    *count = n.nparam;
    return DPD_OK;
}

int dpd_nn_workspace_bytes(const dpd_nn_params* p, size_t* bytes) {
    Net n;
    std::string e;
    int rc = plan(p, &n, &e);
    if (rc) return nfail(nullptr, rc, e);
    if (!bytes) return nfail(nullptr, DPD_EINVAL, "bytes is NULL");
    *bytes = n.total;
    return DPD_OK;
}

int dpd_nn_create(const dpd_nn_params* p, void* workspace, size_t bytes, void* stream,
                  dpd_nn** out) {
    try {
        if (!out) return nfail(nullptr, DPD_EINVAL, "out is NULL");
        *out = nullptr;
        Net n;
        std::string e;
        int rc = plan(p, &n, &e);
        if (rc) return nfail(nullptr, rc, e);
        if (!workspace || ((uintptr_t)workspace & 255u))
            return nfail(nullptr, DPD_EWORKSPACE, "workspace is NULL or not 256-byte aligned");
        if (bytes < n.total)
            return nfail(nullptr, DPD_EWORKSPACE, nfmt("workspace has %zu bytes, needs %zu", bytes, n.total));
        dpd_nn* h = new (std::nothrow) dpd_nn();
        if (!h) return nfail(nullptr, DPD_EINVAL, "out of host memory");
        h->net = n;
        h->stream = (hipStream_t)stream;
        h->ws = (char*)workspace;
        h->adam_t = 0;
        h->err = "no error";
        for (size_t off : {n.o_w, n.o_m, n.o_v, n.o_g})
            hipLaunchKernelGGL(k_zero, dim3(blocks(n.nparam)), dim3(kThreads), 0, h->stream,
                               at<float>(h, off), (long long)n.nparam);
        hipError_t le = hipGetLastError();
        if (le != hipSuccess) {
            delete h;
            return nfail(nullptr, DPD_EHIP, nfmt("kernel launch: %s", hipGetErrorString(le)));
        }
        *out = h;
        return DPD_OK;
    } catch (...) {
        return nfail(nullptr, DPD_EINVAL, "internal error");
    }
}

void dpd_nn_destroy(dpd_nn* nn) { delete nn; }

const char* dpd_nn_last_error(const dpd_nn* nn) { return nn ? nn->err.c_str() : g_nn_error.c_str(); }

int dpd_nn_set_weights(dpd_nn* nn, const float* w) {
    if (!nn) return nfail(nullptr, DPD_EINVAL, "handle is NULL");
    if (!w) return nfail(nn, DPD_EINVAL, "w is NULL");
    const Net& n = nn->net;
    NCHK(nn, hipMemcpyAsync(at<float>(nn, n.o_w), w, 4 * (size_t)n.nparam, hipMemcpyDeviceToDevice,
                            nn->stream));
    for (size_t off : {n.o_m, n.o_v})
        hipLaunchKernelGGL(k_zero, dim3(blocks(n.nparam)), dim3(kThreads), 0, nn->stream,
                           at<float>(nn, off), (long long)n.nparam);
    NLAUNCH(nn);
    nn->adam_t = 0;
    return DPD_OK;
}

int dpd_nn_get_weights(dpd_nn* nn, float* w) {
    if (!nn) return nfail(nullptr, DPD_EINVAL, "handle is NULL");
    if (!w) return nfail(nn, DPD_EINVAL, "w is NULL");
    NCHK(nn, hipMemcpyAsync(w, at<float>(nn, nn->net.o_w), 4 * (size_t)nn->net.nparam,
                            hipMemcpyDeviceToDevice, nn->stream));
    return DPD_OK;
}

int dpd_nn_forward(dpd_nn* nn, const float* u, const float* cond, int32_t B, float* pred) {
    if (!nn) return nfail(nullptr, DPD_EINVAL, "handle is NULL");
    int rc = check_batch(nn, B);
    if (rc) return rc;
    if (!u || !pred || (!cond && nn->net.p.c_in > 2)) return nfail(nn, DPD_EINVAL, "NULL field");
    try {
        return forward(nn, u, cond, B, pred);
    } catch (...) {
        return nfail(nn, DPD_EINVAL, "internal error");
    }
}

int dpd_nn_gradient(dpd_nn* nn, const float* u, const float* cond, const float* target,
                    int32_t B, float* grad, double* loss) {
    if (!nn) return nfail(nullptr, DPD_EINVAL, "handle is NULL");
    int rc = check_batch(nn, B);
    if (rc) return rc;
    if (!u || !target || !grad || (!cond && nn->net.p.c_in > 2)) return nfail(nn, DPD_EINVAL, "NULL argument");
    try {
        return gradient(nn, u, cond, target, B, grad, loss);
    } catch (...) {
        return nfail(nn, DPD_EINVAL, "internal error");
    }
}

int dpd_nn_adam(dpd_nn* nn, const float* grad, float lr, float beta1, float beta2, float eps) {
    if (!nn) return nfail(nullptr, DPD_EINVAL, "handle is NULL");
    if (!grad) return nfail(nn, DPD_EINVAL, "grad is NULL");
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return nfail(nn, DPD_EINVAL, "need lr >= 0, 0 <= beta < 1, eps > 0");
    return adam(nn, grad, lr, beta1, beta2, eps);
}

int dpd_nn_train_step(dpd_nn* nn, const float* u, const float* cond, const float* target,
                      int32_t B, float lr, float beta1, float beta2, float eps, double* loss) {
    if (!nn) return nfail(nullptr, DPD_EINVAL, "handle is NULL");
    float* g = at<float>(nn, nn->net.o_g);
    int rc = dpd_nn_gradient(nn, u, cond, target, B, g, loss);
    if (rc) return rc;
    return dpd_nn_adam(nn, g, lr, beta1, beta2, eps);
}

int dpd_nn_rollout(dpd_nn* nn, const float* u0, const float* cond, int32_t B, int32_t steps,
                   const float* noise_std, const float* noise_filter, uint64_t seed,
                   int32_t save_every, float* traj) {
    if (!nn) return nfail(nullptr, DPD_EINVAL, "handle is NULL");
    if (!u0 || !noise_std || (!cond && nn->net.p.c_in > 2)) return nfail(nn, DPD_EINVAL, "NULL argument");
    if (B < 1 || B > nn->net.p.max_batch) return nfail(nn, DPD_EINVAL, "need 1 <= B <= max_batch");
    if (steps < 0 || save_every < 1) return nfail(nn, DPD_EINVAL, "need steps >= 0, save_every >= 1");
    if (steps / save_every > 0 && !traj) return nfail(nn, DPD_EINVAL, "traj is NULL");
    if (!std::isfinite(noise_std[0]) || !std::isfinite(noise_std[1]) || noise_std[0] < 0.f || noise_std[1] < 0.f)
        return nfail(nn, DPD_EINVAL, "noise_std must be finite and >= 0");
    if (noise_filter && (nn->net.p.M > kColourMaxM || B > 65535))
        return nfail(nn, DPD_EINVAL, nfmt("a noise filter needs M <= %d and B <= 65535", kColourMaxM));
    try {
        const Net& n = nn->net;
        const int M2 = n.p.M * n.p.M, nf = 2 * M2 * B;
        float* ucur = at<float>(nn, n.o_u);
        float* pred = ucur + nf;
        unsigned short* X0 = at<unsigned short>(nn, n.o_x[0]);
        NCHK(nn, hipMemcpyAsync(ucur, u0, 4 * (size_t)nf, hipMemcpyDeviceToDevice, nn->stream));
        // weights in BF16 and the first input, once; each step's noise kernel
        // then writes the next input's field channels
        int rc = cast_weights(nn);
        if (rc) return rc;
        hipLaunchKernelGGL(k_input, dim3(blocks(B * M2)), dim3(kThreads), 0, nn->stream, B * M2, M2,
                           n.p.c_in, (const float*)ucur, cond, X0);
        NLAUNCH(nn);
        const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
        if (band_fits(n)) {
            // the whole network per step as one kernel, which also adds the
            // noise; the noise of up to S steps is drawn ahead in one pass.
            // Buffers free during a rollout: noise [S][B][M][M][2] in dz[1],
            // DFT(h) in dzb[0], the second input buffer (the kernel reads one,
            // writes the other) in dzb[1]
            const int cmax = std::max(n.p.width, 4);
            const int S = std::max(1, std::min(std::min(kNoiseAhead, cmax / 4), 65535 / B));
            float* noise = at<float>(nn, n.o_dz[1]);
            float2* Hh = at<float2>(nn, n.o_dzb[0]);
            unsigned short* X1 = at<unsigned short>(nn, n.o_dzb[1]);
            hipLaunchKernelGGL(k_input, dim3(blocks(B * M2)), dim3(kThreads), 0, nn->stream, B * M2, M2,
                               n.p.c_in, (const float*)ucur, cond, X1);
            if (noise_filter)
                hipLaunchKernelGGL(k_filter_hat, dim3(blocks(M2)), dim3(kThreads), 0, nn->stream, n.p.M,
                                   noise_filter, Hh);
            NLAUNCH(nn);
            unsigned short *Xc = X0, *Xo = X1;
            for (int s = 1; s <= steps; ++s) {
                const int q = (s - 1) % S;
                if (q == 0) {
                    const int ns = std::min(S, steps - s + 1);
                    if (noise_filter) {  // M is 32 or 64: two-stage transforms, one block per field-step
                        hipLaunchKernelGGL(k_colour_fused_r, dim3(B * ns), dim3(kColGroupThreads), 0,
                                           nn->stream, n.p.M, B, (uint32_t)s, k0, k1, (const float2*)Hh,
                                           noise_std[0], noise_std[1], noise);
                    } else {
                        hipLaunchKernelGGL(k_noise_steps, dim3(blocks((long long)nf * ns)), dim3(kThreads), 0,
                                           nn->stream, nf, ns, (uint32_t)s, k0, k1, noise_std[0],
                                           noise_std[1], noise);
                    }
                    NLAUNCH(nn);
                }
                float* save = (s % save_every == 0) ? traj + (size_t)(s / save_every - 1) * nf : nullptr;
                rc = band_step(nn, B, Xc, Xo, ucur, noise + (size_t)q * nf, save);
                if (rc) return rc;
                std::swap(Xc, Xo);
            }
            return DPD_OK;
        }
        // filtered noise: DFT(h) once; the fields' spectra in a free buffer
        float2* Aw = at<float2>(nn, n.o_dz[0]);  // [B][M][M][2] complex
        float2* Hh = at<float2>(nn, n.o_dz[1]);  // [M][M] complex
        if (noise_filter) {
            hipLaunchKernelGGL(k_filter_hat, dim3(blocks(M2)), dim3(kThreads), 0, nn->stream, n.p.M,
                               noise_filter, Hh);
            NLAUNCH(nn);
        }
        for (int s = 1; s <= steps; ++s) {
            rc = forward(nn, ucur, nullptr, B, pred, true);
            if (rc) return rc;
            float* save = (s % save_every == 0) ? traj + (size_t)(s / save_every - 1) * nf : nullptr;
            if (noise_filter) {
                hipLaunchKernelGGL(k_colour_rows, dim3(n.p.M, B), dim3(2 * n.p.M), 0, nn->stream, n.p.M, B,
                                   (uint32_t)s, k0, k1, Aw);
                hipLaunchKernelGGL(k_colour_cols, dim3(n.p.M / 2 + 1, B), dim3(2 * n.p.M), 0, nn->stream,
                                   n.p.M, (const float2*)Hh, Aw);
                hipLaunchKernelGGL(k_colour_out, dim3(n.p.M, B), dim3(2 * n.p.M), 0, nn->stream, n.p.M,
                                   (const float2*)Aw, (const float*)pred, noise_std[0], noise_std[1],
                                   ucur, n.p.c_in, X0, save);
            } else {
                hipLaunchKernelGGL(k_noise, dim3(blocks(nf)), dim3(kThreads), 0, nn->stream, nf,
                                   (const float*)pred, noise_std[0], noise_std[1], (uint32_t)s, k0,
                                   k1, ucur, n.p.c_in, X0, save);
            }
            NLAUNCH(nn);
        }
        return DPD_OK;
    } catch (...) {
        return nfail(nn, DPD_EINVAL, "internal error");
    }
}

int dpd_field_power(const float* u, int32_t nfields, int32_t M, float* work, double* power,
                    void* stream) {
    if (!u || !work || !power) return nfail(nullptr, DPD_EINVAL, "NULL argument");
    if (nfields < 1 || M < 2 || M > 4096 || (long long)nfields * M * M > (1LL << 28))
        return nfail(nullptr, DPD_EINVAL, "need nfields >= 1, 2 <= M <= 4096, nfields M^2 <= 2^28");
    hipStream_t s = (hipStream_t)stream;
    const long long n = (long long)nfields * M * M;
    hipLaunchKernelGGL(k_dft_rows, dim3((unsigned)blocks(n)), dim3(kThreads), 0, s, (int)nfields,
                       (int)M, u, (float2*)work);
    hipLaunchKernelGGL(k_dft_cols_power, dim3(blocks((long long)M * M)), dim3(kThreads), 0, s,
                       (int)nfields, (int)M, (const float2*)work, power);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return nfail(nullptr, DPD_EHIP, nfmt("kernel launch: %s", hipGetErrorString(e)));
    return DPD_OK;
}

int dpd_nn_sync(dpd_nn* nn) {
    if (!nn) return nfail(nullptr, DPD_EINVAL, "handle is NULL");
    NCHK(nn, hipStreamSynchronize(nn->stream));
    return DPD_OK;
}

}  // extern "C"
