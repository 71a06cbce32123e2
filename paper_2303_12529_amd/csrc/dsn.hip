// DevelSet-Net (Sec. III-B): UNet forward with the level-set head and the
// optional modulation head, backward of L_0 (and of L_m), Adam, and the
// resampling between the fine grid and the network grid, on the gfx950 BF16
// matrix cores.  The C ABI is in
// include/dsn.h.
//
// Activations are channels-last BF16 views (pointer, channel stride): the
// encoder's skip outputs are written straight into the upper half of the
// decoder's concatenation buffers, whose lower half receives the up
// convolution.  A 3x3 convolution is an implicit GEMM C[co][pixel] =
// sum_{tap, ci} W[co][tap][ci] X[pixel + tap][ci] on 16x16x32 BF16 matrix
// instructions (weights as the A operand, so each lane stores four
// consecutive channels of one pixel); the same kernel computes the input
// gradient with flipped, transposed weights.  A flag makes a convolution read
// its input through a nearest 2x upsampling, so the upsampled tensor is never
// written.  Weight gradients are a GEMM over pixels, split into pixel ranges
// whose FP32 partials are summed in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/dsn.h"

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return fail(DSN_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

__device__ __forceinline__ f4 mfma_b(bf8 a, bf8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf8 bf8_zero() {
    bf8 z;
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.f;
    return z;
}

// Channels-last BF16 tensor view: element (pixel, c) at p[pixel * stride + c].
struct View {
    __bf16 *p;
    int C, stride;
};

// --------------------------------------------------------------------------
// First convolution (one input channel), VALU: thread = pixel, all output
// channels in groups of 8 (one 16-byte store each); the weights and biases
// as FP32 in LDS (dynamic, Cout x 10 floats), read as broadcasts.  Pixel
// coordinates from 32-bit divisions (npix < 2^31, checked on the host).
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_conv_first(const float *__restrict__ x, int B, int H, int W,
                                                     const __bf16 *__restrict__ w, const float *__restrict__ bias,
                                                     View y) {
    extern __shared__ float wsh[];                 // [Cout][9] then [Cout] biases
    const int C = y.C;
    for (int i = threadIdx.x; i < C * 10; i += 256) wsh[i] = i < C * 9 ? (float)w[i] : bias[i - C * 9];
    __syncthreads();
    const unsigned npix = (unsigned)B * H * W;
    const unsigned pix = blockIdx.x * 256u + threadIdx.x;
    if (pix >= npix) return;
    const unsigned r = pix / (unsigned)W;
    const int xx = (int)(pix - r * W);
    const unsigned b = r / (unsigned)H;
    const int yy = (int)(r - b * H);
    float in[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int sy = yy + t / 3 - 1, sx = xx + t % 3 - 1;
        in[t] = (sy >= 0 && sy < H && sx >= 0 && sx < W) ? x[((size_t)b * H + sy) * W + sx] : 0.f;
    }
    __bf16 *dst = y.p + (size_t)pix * y.stride;
    for (int g = 0; g < C / 8; ++g) {
        bf8 out;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int co = 8 * g + e;
            float acc = wsh[C * 9 + co];
#pragma unroll
            for (int t = 0; t < 9; ++t) acc = fmaf(wsh[co * 9 + t], in[t], acc);
            out[e] = (__bf16)fmaxf(acc, 0.f);
        }
        *reinterpret_cast<bf8 *>(dst + 8 * g) = out;
    }
}

// --------------------------------------------------------------------------
// 3x3 convolution, implicit GEMM on the BF16 matrix cores.
//   out[pixel][co] = act(bias[co] + sum_{tap, ci} w[co][tap][ci] x[src(pixel, tap)][ci])
// Block: 4 waves as WPX (pixels) x WCO (channels); wave tile CB x PB matrix
// blocks of 16 channels x 16 pixels: per 32-deep step a wave loads CB weight
// and PB input fragments straight from global memory for CB x PB
// matrix-core steps (used for small images; larger ones take k_conv_lds).
// Every output sums taps, then input channels in steps of 32.  UP: x has
// half the resolution and is read through a nearest 2x upsampling.
// Requirements (checked on the host): Cin % 32 == 0, Cout % (16 CB WCO) == 0,
// 16-byte aligned views.
// --------------------------------------------------------------------------
template <int WPX, int WCO, int CB, int PB, bool UP>
__global__ __launch_bounds__(256) void k_conv(View x, int B, int H, int W, const __bf16 *__restrict__ w,
                                              int Cin, const float *__restrict__ bias, int relu, View y,
                                              View mask) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int wp = wave % WPX, wc = wave / WPX;
    const long long npix = (long long)B * H * W;
    const long long px0 = ((long long)blockIdx.x * WPX + wp) * (16 * PB);
    const int co0 = (blockIdx.y * WCO + wc) * (16 * CB);
    const int Hin = UP ? H / 2 : H, Win = UP ? W / 2 : W;
    int pb_b[PB], pb_y[PB], pb_x[PB];
    bool pb_ok[PB];
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
        const long long pix = px0 + 16 * pb + l16;
        pb_ok[pb] = pix < npix;
        const long long pc = pb_ok[pb] ? pix : 0;
        pb_x[pb] = (int)(pc % W);
        const long long r = pc / W;
        pb_y[pb] = (int)(r % H);
        pb_b[pb] = (int)(r / H);
    }
    f4 acc[CB][PB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) acc[cb][pb] = f4{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < 9; ++t) {
        const int dy = t / 3 - 1, dx = t % 3 - 1;
        const __bf16 *src[PB];
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) {
            const int sy = pb_y[pb] + dy, sx = pb_x[pb] + dx;
            const bool ok = pb_ok[pb] && sy >= 0 && sy < H && sx >= 0 && sx < W;
            const int iy = UP ? (sy >> 1) : sy, ix = UP ? (sx >> 1) : sx;
            src[pb] = ok ? x.p + (((size_t)pb_b[pb] * Hin + iy) * Win + ix) * x.stride + 8 * lq : nullptr;
        }
        const __bf16 *wt[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) wt[cb] = w + ((size_t)(co0 + 16 * cb + l16) * 9 + t) * Cin + 8 * lq;
        for (int ci0 = 0; ci0 < Cin; ci0 += 32) {
            bf8 a[CB], bv[PB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) a[cb] = *reinterpret_cast<const bf8 *>(wt[cb] + ci0);
#pragma unroll
            for (int pb = 0; pb < PB; ++pb)
                bv[pb] = src[pb] ? *reinterpret_cast<const bf8 *>(src[pb] + ci0) : bf8_zero();
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int pb = 0; pb < PB; ++pb) acc[cb][pb] = mfma_b(a[cb], bv[pb], acc[cb][pb]);
        }
    }
    // register i of acc[cb][pb]: channel co0 + 16 cb + 4 lq + i, pixel px0 + 16 pb + l16
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
        const long long pix = px0 + 16 * pb + l16;
        if (pix >= npix) continue;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int c = co0 + 16 * cb + 4 * lq;
            bf4 o;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float v = acc[cb][pb][i] + (bias ? bias[c + i] : 0.f);
                if (relu) v = fmaxf(v, 0.f);
                o[i] = (__bf16)v;
            }
            if (mask.p) {
                const bf4 m = *reinterpret_cast<const bf4 *>(mask.p + pix * mask.stride + c);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (!((float)m[i] > 0.f)) o[i] = (__bf16)0.f;
            }
            *reinterpret_cast<bf4 *>(y.p + pix * y.stride + c) = o;
        }
    }
}

// --------------------------------------------------------------------------
// 3x3 convolution with LDS-staged operands.  Block: an 8 x 32 pixel tile of
// one image x TC (64 or 32) output channels; per 32-channel input chunk it
// stages the tile's input pixels with a one-pixel halo (zero outside the
// image; through the nearest 2x upsampling when UP) and the TC x 9 x 32
// weights in LDS.  Wave w: the 16-pixel column strip w & 1 of the tile x 32
// output channels, over all 8 rows (TC = 64: channels 32 (w >> 1) on) or
// over rows 4 (w >> 1) .. + 3 (TC = 32).  Per chunk the wave keeps its 9 x 2
// weight operands in registers and walks down its rows: each halo row's
// three shifted input operands are read once and serve the three output
// rows whose taps touch it.  Pixel and channel strides of 40 and 296
// elements make the 16-byte reads of 8 consecutive lanes hit distinct
// banks.  Every output sums input-channel chunks, then taps in order.
// --------------------------------------------------------------------------
constexpr int CL_TY = 8, CL_TX = 32;
constexpr int CL_XS = 40;                         // LDS elements per staged pixel
constexpr int CL_WS = 9 * 32 + 8;                 // LDS elements per staged output channel
constexpr int CL_NPX = (CL_TY + 2) * (CL_TX + 2);

template <bool UP, int TC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_conv_lds(
    View x, int B, int H, int W, const __bf16 *__restrict__ w, int Cin, const float *__restrict__ bias, int relu,
    View y, View mask) {
    constexpr int RW = TC == 64 ? 8 : 4;          // output rows per wave
    __shared__ __attribute__((aligned(16))) __bf16 Xs[CL_NPX * CL_XS];
    __shared__ __attribute__((aligned(16))) __bf16 Ws[TC * CL_WS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int strip = wave & 1;
    const int cw = TC == 64 ? 32 * (wave >> 1) : 0, row0 = TC == 64 ? 0 : 4 * (wave >> 1);
    const int ntx = (W + CL_TX - 1) / CL_TX, nty = (H + CL_TY - 1) / CL_TY;
    const int tix = blockIdx.x % ntx, rest = blockIdx.x / ntx;
    const int tiy = rest % nty, b = rest / nty;
    const int x0 = tix * CL_TX, y0 = tiy * CL_TY, co0 = blockIdx.y * TC;
    const int Hin = UP ? H / 2 : H, Win = UP ? W / 2 : W;
    constexpr int XU = (CL_NPX * 4 + 255) / 256;  // 16-byte input units per thread
    constexpr int WU = (TC * 36 + 255) / 256;     // 16-byte weight units per thread
    f4 acc[RW][2];
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r][0] = acc[r][1] = f4{0.f, 0.f, 0.f, 0.f};
    // the input chunk's loads: the next chunk's are in flight while the
    // current one is multiplied
    bf8 xv[XU];
    auto fetch_x = [&](int ci0) {
#pragma unroll
        for (int u = 0; u < XU; ++u) {
            const int e = threadIdx.x + 256 * u;
            xv[u] = bf8_zero();
            if (e < CL_NPX * 4) {
                const int px = e >> 2, seg = e & 3;
                const int gy = y0 + px / (CL_TX + 2) - 1, gx = x0 + px % (CL_TX + 2) - 1;
                if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
                    const int sy = UP ? (gy >> 1) : gy, sx = UP ? (gx >> 1) : gx;
                    xv[u] = *reinterpret_cast<const bf8 *>(x.p + (((size_t)b * Hin + sy) * Win + sx) * x.stride +
                                                           ci0 + 8 * seg);
                }
            }
        }
    };
    fetch_x(0);
    for (int ci0 = 0; ci0 < Cin; ci0 += 32) {
        bf8 wv[WU];
#pragma unroll
        for (int u = 0; u < WU; ++u) {
            const int e = threadIdx.x + 256 * u;
            if (e < TC * 36) {
                const int col = e / 36, rem = e % 36;
                wv[u] = *reinterpret_cast<const bf8 *>(w + ((size_t)(co0 + col) * 9 + rem / 4) * Cin + ci0 +
                                                       8 * (rem % 4));
            }
        }
        __syncthreads();                              // the previous chunk's reads are done
#pragma unroll
        for (int u = 0; u < XU; ++u) {
            const int e = threadIdx.x + 256 * u;
            if (e < CL_NPX * 4) *reinterpret_cast<bf8 *>(&Xs[(e >> 2) * CL_XS + 8 * (e & 3)]) = xv[u];
        }
#pragma unroll
        for (int u = 0; u < WU; ++u) {
            const int e = threadIdx.x + 256 * u;
            if (e < TC * 36) {
                const int col = e / 36, rem = e % 36;
                *reinterpret_cast<bf8 *>(&Ws[col * CL_WS + (rem / 4) * 32 + 8 * (rem % 4)]) = wv[u];
            }
        }
        __syncthreads();
        if (ci0 + 32 < Cin) fetch_x(ci0 + 32);
        bf8 a[9][2];
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
                a[t][cb] = *reinterpret_cast<const bf8 *>(&Ws[(cw + 16 * cb + l16) * CL_WS + t * 32 + 8 * lq]);
        // the three column shifts of halo row hr (of the wave's rows)
        const __bf16 *xcol = Xs + (16 * strip + l16) * CL_XS + 8 * lq;
        bf8 bw[3][3];
        auto load_row = [&](int hr, bf8(&o)[3]) {
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
                o[dx] = *reinterpret_cast<const bf8 *>(xcol + ((row0 + hr) * (CL_TX + 2) + dx) * CL_XS);
        };
        load_row(0, bw[0]);
        load_row(1, bw[1]);
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            load_row(r + 2, bw[(r + 2) % 3]);
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        acc[r][cb] = mfma_b(a[3 * dy + dx][cb], bw[(r + dy) % 3][dx], acc[r][cb]);
        }
    }
    // register i of acc[r][cb]: channel co0 + cw + 16 cb + 4 lq + i, pixel (row row0 + r, column 16 strip + l16)
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int gy = y0 + row0 + r, gx = x0 + 16 * strip + l16;
        if (gy >= H || gx >= W) continue;
        const long long pix = ((long long)b * H + gy) * W + gx;
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const int c = co0 + cw + 16 * cb + 4 * lq;
            bf4 o;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float v = acc[r][cb][i] + (bias ? bias[c + i] : 0.f);
                if (relu) v = fmaxf(v, 0.f);
                o[i] = (__bf16)v;
            }
            if (mask.p) {
                const bf4 m = *reinterpret_cast<const bf4 *>(mask.p + pix * mask.stride + c);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (!((float)m[i] > 0.f)) o[i] = (__bf16)0.f;
            }
            *reinterpret_cast<bf4 *>(y.p + pix * y.stride + c) = o;
        }
    }
}

// --------------------------------------------------------------------------
// Weight gradient over spatial tiles, all nine taps per block:
//   part[s][co][tap][ci] = sum over the pixels of split s of
//                          dz[pixel][co] x[pixel + tap offset][ci]
// A block owns TCO output x TCI input channels and a range of 8 x 32 pixel
// tiles of the batch.  Per tile, dz is staged channel-major (Zs[co][pixel])
// and x as the tile plus a one-pixel halo (Xs[ci][halo row][7 + halo
// column], zero outside the image, through the nearest 2x upsampling when
// UP), by 16-byte loads of 8 channels scattered into LDS; the next tile's
// loads are in flight while the current one is multiplied.  A GEMM over
// pixels: each wave owns 32 co x 16 ci and, per output row, reads its two dz
// operands (8 consecutive pixels of one channel per lane) once and takes
// them against the x operands of the three halo rows that the row's taps
// touch, at the three column shifts.  The shifted operands come from three
// aligned 16-byte reads per halo row and lane plus 32-bit funnel shifts; a
// halo row's operands stay in registers for the three output rows that use
// it.  Channel strides padded to 264 and 488 elements keep the lanes'
// 16-byte reads on distinct banks.  FP32 accumulation; the partials of the
// splits are summed in a fixed order afterwards.
// With bpart, the blocks of the first input-channel tile also sum dz over
// their pixels (the bias gradient) by products with a vector of ones: the
// waves of a row of the block take the output rows in turn and write
// bpart[split][wave column][co].
// --------------------------------------------------------------------------
constexpr int WT_TY = 8, WT_TX = 32, WT_HR = WT_TY + 2, WT_HC = WT_TX + 2, WT_XS = 48;
constexpr int WT_ZST = WT_TY * WT_TX + 8;        // dz channel stride (elements)
constexpr int WT_XST = WT_HR * WT_XS + 8;        // x channel stride (elements)

// elements 1..8 of the 16-element sequence lo | hi
__device__ __forceinline__ bf8 bf8_next(bf8 lo, bf8 hi) {
    const u4 a = *reinterpret_cast<const u4 *>(&lo), b = *reinterpret_cast<const u4 *>(&hi);
    u4 o;
    o[0] = __builtin_amdgcn_alignbit(a[1], a[0], 16);
    o[1] = __builtin_amdgcn_alignbit(a[2], a[1], 16);
    o[2] = __builtin_amdgcn_alignbit(a[3], a[2], 16);
    o[3] = __builtin_amdgcn_alignbit(b[0], a[3], 16);
    return *reinterpret_cast<const bf8 *>(&o);
}

// elements 7..14 of the 16-element sequence lo | hi
__device__ __forceinline__ bf8 bf8_prev(bf8 lo, bf8 hi) {
    const u4 a = *reinterpret_cast<const u4 *>(&lo), b = *reinterpret_cast<const u4 *>(&hi);
    u4 o;
    o[0] = __builtin_amdgcn_alignbit(b[0], a[3], 16);
    o[1] = __builtin_amdgcn_alignbit(b[1], b[0], 16);
    o[2] = __builtin_amdgcn_alignbit(b[2], b[1], 16);
    o[3] = __builtin_amdgcn_alignbit(b[3], b[2], 16);
    return *reinterpret_cast<const bf8 *>(&o);
}

template <int TCO, int TCI, bool UP>
__global__ __launch_bounds__((TCO / 32) * (TCI / 16) * 64) __attribute__((amdgpu_waves_per_eu(TCO * TCI > 1024 ? 2 : 1))) void k_wgrad_tile(View dz, View x, int B, int H, int W,
                                                                          int Cin, int Cout, int tiles_per_split,
                                                                          float *__restrict__ part,
                                                                          float *__restrict__ bpart) {
    constexpr int NWC = TCI / 16, NT = (TCO / 32) * NWC * 64;
    constexpr int ZE = WT_TY * WT_TX * (TCO / 8), XE = WT_HR * WT_HC * (TCI / 8);
    constexpr int ZL = (ZE + NT - 1) / NT, XL = (XE + NT - 1) / NT;     // 16-byte loads per thread
    __shared__ __attribute__((aligned(16))) __bf16 Zs[TCO * WT_ZST];
    __shared__ __attribute__((aligned(16))) __bf16 Xs[TCI * WT_XST];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int wco = (wave / NWC) * 32, wci = (wave % NWC) * 16;
    const int co_t = blockIdx.x * TCO, ci_t = blockIdx.y * TCI;
    const int ntx = (W + WT_TX - 1) / WT_TX, nty = (H + WT_TY - 1) / WT_TY;
    const long long ntiles = (long long)B * nty * ntx;
    const long long t0 = (long long)blockIdx.z * tiles_per_split;
    const long long t1 = t0 + tiles_per_split < ntiles ? t0 + tiles_per_split : ntiles;
    const int Hin = UP ? H / 2 : H, Win = UP ? W / 2 : W;
    bf8 zv[ZL], xv[XL];
    auto fetch = [&](long long tile) {
        const int tx = (int)(tile % ntx);
        const long long rest = tile / ntx;
        const int ty = (int)(rest % nty), b = (int)(rest / nty);
        const int x0 = tx * WT_TX, y0 = ty * WT_TY;
#pragma unroll
        for (int u = 0; u < ZL; ++u) {
            const int e = threadIdx.x + NT * u;
            zv[u] = bf8_zero();
            if (ZE % NT == 0 || e < ZE) {
                const int p = e % (WT_TY * WT_TX), g = e / (WT_TY * WT_TX);
                const int yy = y0 + p / WT_TX, xx = x0 + p % WT_TX;
                if (yy < H && xx < W)
                    zv[u] = *reinterpret_cast<const bf8 *>(dz.p + (((size_t)b * H + yy) * W + xx) * dz.stride +
                                                           co_t + 8 * g);
            }
        }
#pragma unroll
        for (int u = 0; u < XL; ++u) {
            const int e = threadIdx.x + NT * u;
            xv[u] = bf8_zero();
            if (XE % NT == 0 || e < XE) {
                const int hp = e % (WT_HR * WT_HC), g = e / (WT_HR * WT_HC);
                const int gy = y0 + hp / WT_HC - 1, gx = x0 + hp % WT_HC - 1;
                if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
                    const int sy = UP ? (gy >> 1) : gy, sx = UP ? (gx >> 1) : gx;
                    xv[u] = *reinterpret_cast<const bf8 *>(x.p + (((size_t)b * Hin + sy) * Win + sx) * x.stride +
                                                           ci_t + 8 * g);
                }
            }
        }
    };
    f4 acc[9][2], accb[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t][0] = acc[t][1] = f4{0.f, 0.f, 0.f, 0.f};
    const bool with_b = bpart != nullptr && blockIdx.y == 0;
    bf8 ones;
#pragma unroll
    for (int k = 0; k < 8; ++k) ones[k] = (__bf16)1.f;
    if (t0 < t1) fetch(t0);
    const __bf16 *xrow = Xs + (wci + l16) * WT_XST + 8 * lq;
    const __bf16 *zrow0 = Zs + (wco + l16) * WT_ZST + 8 * lq;
    const __bf16 *zrow1 = zrow0 + 16 * WT_ZST;
    for (long long tile = t0; tile < t1; ++tile) {
        __syncthreads();                                   // the previous tile's reads are done
#pragma unroll
        for (int u = 0; u < ZL; ++u) {
            const int e = threadIdx.x + NT * u;
            if (ZE % NT == 0 || e < ZE) {
                const int p = e % (WT_TY * WT_TX), g = e / (WT_TY * WT_TX);
#pragma unroll
                for (int k = 0; k < 8; ++k) Zs[(8 * g + k) * WT_ZST + p] = zv[u][k];
            }
        }
#pragma unroll
        for (int u = 0; u < XL; ++u) {
            const int e = threadIdx.x + NT * u;
            if (XE % NT == 0 || e < XE) {
                const int hp = e % (WT_HR * WT_HC), g = e / (WT_HR * WT_HC);
                const int pos = (hp / WT_HC) * WT_XS + hp % WT_HC + 7;
#pragma unroll
                for (int k = 0; k < 8; ++k) Xs[(8 * g + k) * WT_XST + pos] = xv[u][k];
            }
        }
        __syncthreads();
        if (tile + 1 < t1) fetch(tile + 1);
        // x operands of halo row hr at the column shifts -1, 0, +1
        bf8 rows[3][3];
        auto load_row = [&](int hr, bf8(&op)[3]) {
            const bf8 c0 = *reinterpret_cast<const bf8 *>(xrow + hr * WT_XS);
            const bf8 c1 = *reinterpret_cast<const bf8 *>(xrow + hr * WT_XS + 8);
            const bf8 c2 = *reinterpret_cast<const bf8 *>(xrow + hr * WT_XS + 16);
            op[0] = bf8_prev(c0, c1);
            op[1] = c1;
            op[2] = bf8_next(c1, c2);
        };
        load_row(0, rows[0]);
        load_row(1, rows[1]);
#pragma unroll
        for (int r = 0; r < WT_TY; ++r) {
            load_row(r + 2, rows[(r + 2) % 3]);
            const bf8 a0 = *reinterpret_cast<const bf8 *>(zrow0 + r * WT_TX);
            const bf8 a1 = *reinterpret_cast<const bf8 *>(zrow1 + r * WT_TX);
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const bf8 bo = rows[(r + dy) % 3][dx];
                    acc[3 * dy + dx][0] = mfma_b(a0, bo, acc[3 * dy + dx][0]);
                    acc[3 * dy + dx][1] = mfma_b(a1, bo, acc[3 * dy + dx][1]);
                }
            if (with_b && r % NWC == wave % NWC) {
                accb[0] = mfma_b(a0, ones, accb[0]);
                accb[1] = mfma_b(a1, ones, accb[1]);
            }
        }
    }
    if (with_b && l16 == 0) {
        float *bd = bpart + ((size_t)blockIdx.z * NWC + wave % NWC) * Cout;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) bd[co_t + wco + 16 * h + 4 * lq + i] = accb[h][i];
    }
    // register i of acc[t][h]: co = wco + 16 h + 4 lq + i, ci = wci + l16
    float *dst = part + (size_t)blockIdx.z * Cout * 9 * Cin;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = co_t + wco + 16 * h + 4 * lq + i, ci = ci_t + wci + l16;
                dst[((size_t)co * 9 + t) * Cin + ci] = acc[t][h][i];
            }
}

// First layer (one input channel): part[s][co][tap] over a pixel range and,
// after the S x C x 9 weight partials, the bias partials part[S C 9 + s C +
// co].  Thread = (8 channels, pixel): one 16-byte dz load and the nine
// neighbouring inputs (FP32, cached reads) per pixel, 80 FMAs into FP32
// registers; then a shuffle tree over the wave's pixel lanes and the four
// waves in order.  C in {8, 16, 32, 64}.
__global__ __launch_bounds__(256) void k_wgrad_first(View dz, const float *__restrict__ x, int B, int H, int W,
                                                      long long pix_per_split, float *__restrict__ part) {
    const int C = dz.C, G = C / 8;
    __shared__ float red[4][8][81];
    const int s = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = threadIdx.x % G, ph = threadIdx.x / G, nph = 256 / G;
    const long long npix = (long long)B * H * W;
    const long long p_lo = (long long)s * pix_per_split;
    const long long p_hi = p_lo + pix_per_split < npix ? p_lo + pix_per_split : npix;
    float acc[8][10];
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int k = 0; k < 10; ++k) acc[e][k] = 0.f;
    // the thread's pixels advance by nph: (b, yy, xx) stepped instead of
    // divided out per pixel
    long long pix = p_lo + ph;
    int xx = 0, yy = 0, b = 0;
    if (pix < p_hi) {
        xx = (int)(pix % W);
        const long long r = pix / W;
        yy = (int)(r % H);
        b = (int)(r / H);
    }
    for (; pix < p_hi; pix += nph) {
        const bf8 d = *reinterpret_cast<const bf8 *>(dz.p + pix * dz.stride + 8 * g);
        float xv[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int sy = yy + t / 3 - 1, sx = xx + t % 3 - 1;
            xv[t] = (sy >= 0 && sy < H && sx >= 0 && sx < W) ? x[((size_t)b * H + sy) * W + sx] : 0.f;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float de = (float)d[e];
#pragma unroll
            for (int t = 0; t < 9; ++t) acc[e][t] = fmaf(de, xv[t], acc[e][t]);
            acc[e][9] += de;
        }
        xx += nph;
        while (xx >= W) {
            xx -= W;
            if (++yy == H) {
                yy = 0;
                ++b;
            }
        }
    }
    // lanes lane, lane ^ G, ... hold the same channels
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            float v = acc[e][k];
            for (int o = G; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
            acc[e][k] = v;
        }
    if (lane < G) {
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
            for (int k = 0; k < 10; ++k) red[wave][lane][e * 10 + k] = acc[e][k];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < C * 10; i += 256) {
        const int co = i / 10, k = i % 10;
        const int gg = co / 8, e = co % 8;
        const float v = ((red[0][gg][e * 10 + k] + red[1][gg][e * 10 + k]) + red[2][gg][e * 10 + k]) +
                        red[3][gg][e * 10 + k];
        if (k < 9) part[((size_t)s * C + co) * 9 + k] = v;
        else part[(size_t)gridDim.x * C * 9 + (size_t)s * C + co] = v;
    }
}

// out[j] = sum_s part[s][j] in a fixed order (FP64 accumulation).  Block:
// OUT outputs x (256 / OUT) groups of partials s = g, g + 256/OUT, ...; the
// group sums are added in group order.
template <int OUT>
__global__ __launch_bounds__(256) void k_reduce_splits(const float *__restrict__ part, int S, long long n,
                                                       float *__restrict__ out) {
    constexpr int GRP = 256 / OUT;
    __shared__ double red[GRP][OUT + 1];
    const int o = threadIdx.x % OUT, g = threadIdx.x / OUT;
    const long long j = (long long)blockIdx.x * OUT + o;
    double v = 0.0;
    if (j < n)
        for (int s = g; s < S; s += GRP) v += part[(size_t)s * n + j];
    red[g][o] = v;
    __syncthreads();
    if (g == 0 && j < n) {
        double t = 0.0;
        for (int q = 0; q < GRP; ++q) t += red[q][o];
        out[j] = (float)t;
    }
}

// many outputs: 16 per block; few (biases, the head): one per block, all
// 256 threads on its partials
// The same sums for n % 4 == 0 and 16-byte aligned partials: a block of 1024
// threads takes QB consecutive 4-float groups (16-byte loads) x 1024 / QB
// phases over the splits; each thread adds its splits in order in FP64, then
// the phases are added by a halving tree.  QB shrinks for short vectors so that the
// splits spread over more threads (and more blocks).
__global__ __launch_bounds__(1024) void k_reduce_splits4(const float *__restrict__ part, int S, long long n, int QB,
                                                         float *__restrict__ out) {
    __shared__ double red[4096];
    const long long nq = n / 4;
    const int qi = threadIdx.x % QB, ph = threadIdx.x / QB, P = 1024 / QB;
    const long long q = (long long)blockIdx.x * QB + qi;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (q < nq) {
#pragma unroll 4
        for (int s = ph; s < S; s += P) {
            const float4 f = *reinterpret_cast<const float4 *>(part + (size_t)s * n + 4 * q);
            v[0] += f.x;
            v[1] += f.y;
            v[2] += f.z;
            v[3] += f.w;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) red[threadIdx.x * 4 + k] = v[k];
    // phases: a halving tree (P is a power of two)
    for (int h = P / 2; h > 0; h >>= 1) {
        __syncthreads();
        if (ph < h)
#pragma unroll
            for (int k = 0; k < 4; ++k) red[threadIdx.x * 4 + k] += red[(threadIdx.x + h * QB) * 4 + k];
    }
    __syncthreads();
    if (ph == 0 && q < nq)
#pragma unroll
        for (int k = 0; k < 4; ++k) out[4 * q + k] = (float)red[qi * 4 + k];
}

void reduce_splits(const float *part, int S, long long n, float *out, hipStream_t st) {
    if (n % 4 == 0 && reinterpret_cast<uintptr_t>(part) % 16 == 0) {
        const long long nq = n / 4;
        int QB = 64;
        while (QB > 1 && (nq + QB - 1) / QB < 512) QB /= 2;
        k_reduce_splits4<<<(unsigned)((nq + QB - 1) / QB), 1024, 0, st>>>(part, S, n, QB, out);
    } else if (n >= 4096) {
        k_reduce_splits<16><<<(unsigned)((n + 15) / 16), 256, 0, st>>>(part, S, n, out);
    } else {
        k_reduce_splits<1><<<(unsigned)n, 256, 0, st>>>(part, S, n, out);
    }
}

// --------------------------------------------------------------------------
// Pooling, upsampling, ReLU gradient (thread = pixel x 8 channels).
// --------------------------------------------------------------------------
__global__ void k_maxpool(View x, int B, int H, int W, View y) {
    const int groups = x.C / 8;
    const int Ho = H / 2, Wo = W / 2;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)B * Ho * Wo * groups;
    if (id >= n) return;
    const long long po = id / groups;
    const int g = (int)(id - po * groups);
    const int xo = (int)(po % Wo);
    const long long r = po / Wo;
    const int yo = (int)(r % Ho), b = (int)(r / Ho);
    bf8 m;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const size_t pi = ((size_t)b * H + 2 * yo + k / 2) * W + 2 * xo + k % 2;
        const bf8 v = *reinterpret_cast<const bf8 *>(x.p + pi * x.stride + 8 * g);
        if (k == 0) {
            m = v;
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) m[e] = (float)v[e] > (float)m[e] ? v[e] : m[e];
        }
    }
    *reinterpret_cast<bf8 *>(y.p + po * y.stride + 8 * g) = m;
}

// dx (view holding the skip gradient) += gradient routed to the first
// maximum (row-major order) of each 2x2 window.
template <bool MASK>
__global__ void k_maxpool_bwd(View x, int B, int H, int W, View dy, View dx) {
    const int groups = x.C / 8;
    const int Ho = H / 2, Wo = W / 2;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)B * Ho * Wo * groups;
    if (id >= n) return;
    const long long po = id / groups;
    const int g = (int)(id - po * groups);
    const int xo = (int)(po % Wo);
    const long long r = po / Wo;
    const int yo = (int)(r % Ho), b = (int)(r / Ho);
    bf8 v[4];
    size_t pi[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        pi[k] = ((size_t)b * H + 2 * yo + k / 2) * W + 2 * xo + k % 2;
        v[k] = *reinterpret_cast<const bf8 *>(x.p + pi[k] * x.stride + 8 * g);
    }
    int arg[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        int a = 0;
        float best = (float)v[0][e];
#pragma unroll
        for (int k = 1; k < 4; ++k)
            if ((float)v[k][e] > best) {
                best = (float)v[k][e];
                a = k;
            }
        arg[e] = a;
    }
    const bf8 d = *reinterpret_cast<const bf8 *>(dy.p + po * dy.stride + 8 * g);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        __bf16 *q = dx.p + pi[k] * dx.stride + 8 * g;
        bf8 cur = *reinterpret_cast<const bf8 *>(q);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if (arg[e] == k) cur[e] = (__bf16)((float)cur[e] + (float)d[e]);
            if (MASK && !((float)v[k][e] > 0.f)) cur[e] = (__bf16)0.f;
        }
        *reinterpret_cast<bf8 *>(q) = cur;
    }
}

// Gradient of the nearest 2x upsampling: dx[half pixel] = sum of its 4 children.
__global__ void k_upsample_bwd(View dy, int B, int H, int W, View dx, View mask) {
    const int groups = dx.C / 8;
    const int Ho = H / 2, Wo = W / 2;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)B * Ho * Wo * groups;
    if (id >= n) return;
    const long long po = id / groups;
    const int g = (int)(id - po * groups);
    const int xo = (int)(po % Wo);
    const long long r = po / Wo;
    const int yo = (int)(r % Ho), b = (int)(r / Ho);
    float s[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const size_t pi = ((size_t)b * H + 2 * yo + k / 2) * W + 2 * xo + k % 2;
        const bf8 v = *reinterpret_cast<const bf8 *>(dy.p + pi * dy.stride + 8 * g);
#pragma unroll
        for (int e = 0; e < 8; ++e) s[e] += (float)v[e];
    }
    bf8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = (__bf16)s[e];
    if (mask.p) {
        const bf8 m = *reinterpret_cast<const bf8 *>(mask.p + po * mask.stride + 8 * g);
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (!((float)m[e] > 0.f)) o[e] = (__bf16)0.f;
    }
    *reinterpret_cast<bf8 *>(dx.p + po * dx.stride + 8 * g) = o;
}

// d <- d . [y > 0] (in place), same shape views.
__global__ void k_relu_bwd(View d, View y, long long npix) {
    const int groups = d.C / 8;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= npix * groups) return;
    const long long pix = id / groups;
    const int g = (int)(id - pix * groups);
    __bf16 *q = d.p + pix * d.stride + 8 * g;
    bf8 dv = *reinterpret_cast<const bf8 *>(q);
    const bf8 yv = *reinterpret_cast<const bf8 *>(y.p + pix * y.stride + 8 * g);
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if (!((float)yv[e] > 0.f)) dv[e] = (__bf16)0.f;
    *reinterpret_cast<bf8 *>(q) = dv;
}

// --------------------------------------------------------------------------
// Head (1x1 convolution to one channel) and the loss.
// --------------------------------------------------------------------------
__global__ void k_head(View x, long long npix, const __bf16 *__restrict__ w, const float *__restrict__ bias,
                       const __bf16 *__restrict__ wm, const float *__restrict__ bm, float *__restrict__ out,
                       float *__restrict__ out_m) {
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= npix) return;
    float acc = bias[0], accm = out_m ? bm[0] : 0.f;
    for (int c = 0; c < x.C; c += 8) {
        const bf8 v = *reinterpret_cast<const bf8 *>(x.p + pix * x.stride + c);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            acc = fmaf((float)w[c + e], (float)v[e], acc);
            if (out_m) accm = fmaf((float)wm[c + e], (float)v[e], accm);
        }
    }
    out[pix] = acc;
    if (out_m) out_m[pix] = accm;
}

// approximated Heaviside of the modulation branch and its derivative
__device__ __forceinline__ float ahf(float z) { return 0.5f * (1.f + (2.f / 3.14159265358979f) * atanf(z / DSN_EPS_AHF)); }
__device__ __forceinline__ float ahf_grad(float z) {
    return (1.f / 3.14159265358979f) * DSN_EPS_AHF / (DSN_EPS_AHF * DSN_EPS_AHF + z * z);
}

// g = (2/B)(out - t); with the modulation head also gm = (2/B)(H(out_m) - t_m)
// H'(out_m) (0 without t_m); dx[pixel][c] = g w[c] + gm wm[c]; per-block
// partials of both losses (FP64) and of both heads' gradients (FP32):
// gpart[block][h][C + 1] = {sum_p g_h x[p][c], sum_p g_h}.
__global__ __launch_bounds__(256) void k_head_bwd(View x, long long npix, int B, const __bf16 *__restrict__ w,
                                                   const __bf16 *__restrict__ wm, const float *__restrict__ out,
                                                   const float *__restrict__ out_m, const float *__restrict__ tgt,
                                                   const float *__restrict__ tgt_m, View dx, int relu_mask,
                                                   double *__restrict__ loss_part, float *__restrict__ gpart) {
    const int C = x.C;                      // <= 64, a multiple of 8
    const int NH = out_m ? 2 : 1;
    __shared__ double lw[2][4];
    __shared__ float gw[2][4][65];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long pix = (long long)blockIdx.x * 256 + threadIdx.x;
    double l = 0.0, lm = 0.0;
    float g = 0.f, gm = 0.f;
    bf8 v[8];
    if (pix < npix) {
        const float d = out[pix] - tgt[pix];
        l = (double)d * d;
        g = 2.f / (float)B * d;
        if (out_m && tgt_m) {
            const float z = out_m[pix], hm = ahf(z) - tgt_m[pix];
            lm = (double)hm * hm;
            gm = 2.f / (float)B * hm * ahf_grad(z);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (8 * k >= C) break;
            const int c = 8 * k;
            v[k] = *reinterpret_cast<const bf8 *>(x.p + pix * x.stride + c);
            bf8 o;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                o[e] = (__bf16)(g * (float)w[c + e] + (out_m ? gm * (float)wm[c + e] : 0.f));
                if (relu_mask && !((float)v[k][e] > 0.f)) o[e] = (__bf16)0.f;
            }
            *reinterpret_cast<bf8 *>(dx.p + pix * dx.stride + c) = o;
        }
    }
    // per-block sums in a fixed order: a shuffle tree in each wave, then the
    // four waves in wave order
    double l0 = l, l1 = lm;
    for (int o = 32; o > 0; o >>= 1) {
        l0 += __shfl_xor(l0, o, 64);
        l1 += __shfl_xor(l1, o, 64);
    }
    if (lane == 0) {
        lw[0][wave] = l0;
        lw[1][wave] = l1;
    }
    for (int h = 0; h < NH; ++h) {
        const float gh = pix < npix ? (h == 0 ? g : gm) : 0.f;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (8 * k >= C) break;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                float t = pix < npix ? gh * (float)v[k][e] : 0.f;
                for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
                if (lane == 0) gw[h][wave][8 * k + e] = t;
            }
        }
        float t = gh;
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        if (lane == 0) gw[h][wave][C] = t;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NH * (C + 1); i += 256) {
        const int h = i / (C + 1), c = i - (i / (C + 1)) * (C + 1);
        gpart[((size_t)blockIdx.x * NH + h) * (C + 1) + c] =
            ((gw[h][0][c] + gw[h][1][c]) + gw[h][2][c]) + gw[h][3][c];
    }
    if (threadIdx.x == 0) {
        loss_part[2 * blockIdx.x] = ((lw[0][0] + lw[0][1]) + lw[0][2]) + lw[0][3];
        loss_part[2 * blockIdx.x + 1] = ((lw[1][0] + lw[1][1]) + lw[1][2]) + lw[1][3];
    }
}

__global__ void k_loss_finish(const double *__restrict__ part, int n, int B, double *__restrict__ loss) {
    __shared__ double red[2][256];
    double s0 = 0.0, s1 = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        s0 += part[2 * i];
        s1 += part[2 * i + 1];
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = 0.0, t1 = 0.0;
        for (int i = 0; i < 256; ++i) {
            t0 += red[0][i];
            t1 += red[1][i];
        }
        loss[0] = t0 / B;
        loss[1] = t1 / B;
    }
}

// --------------------------------------------------------------------------
// Parameters: BF16 working copies, flipped/transposed copies for the input
// gradient, Adam.
// --------------------------------------------------------------------------
__global__ void k_fill_f32(float *__restrict__ a, long long n, float v) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        a[i] = v;
}

__global__ void k_to_bf16(const float *__restrict__ a, long long n, __bf16 *__restrict__ b) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (__bf16)a[i];
}

// wt[ci][tap][co] = w[co][8 - tap][ci]
__global__ void k_flip_transpose(const __bf16 *__restrict__ w, int Cout, int Cin, __bf16 *__restrict__ wt) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)Cout * 9 * Cin;
    if (i >= n) return;
    const int co = (int)(i % Cout);
    const long long r = i / Cout;
    const int t = (int)(r % 9), ci = (int)(r / 9);
    wt[i] = w[((size_t)co * 9 + (8 - t)) * Cin + ci];
}

__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, long long n, float lr, float b1, float b2, float eps,
                       float c1, float c2, __bf16 *__restrict__ pb) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    pb[i] = (__bf16)pi;
}

// --------------------------------------------------------------------------
// Resampling between the fine grid (4H x 4W) and the network grid (H x W).
// --------------------------------------------------------------------------
__global__ void k_prepare(const unsigned char *__restrict__ tgt, const float *__restrict__ phi,
                          const float *__restrict__ mgt, int B, int H, int W, float *__restrict__ x,
                          float *__restrict__ t, float *__restrict__ tm) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)B * H * W) return;
    const int xx = (int)(id % W);
    const long long r = id / W;
    const int yy = (int)(r % H), b = (int)(r / H);
    const int W4 = 4 * W, H4 = 4 * H;
    int cnt = 0;
    double s = 0.0, sm = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 4; ++c) {
            const size_t q = ((size_t)b * H4 + 4 * yy + a) * W4 + 4 * xx + c;
            cnt += tgt[q] != 0;
            if (phi) s += phi[q];
            if (mgt) sm += mgt[q];
        }
    x[id] = (float)cnt * (1.f / 16.f);
    if (phi) t[id] = (float)(s / 16.0 / (double)DSN_SCALE);
    if (mgt) tm[id] = (float)(sm / 16.0);
}

// phi0 = clip(100 x bilinear 4x upsampling): fine pixel i samples the network
// coordinate (i + 1/2)/4 - 1/2, clamped to [0, n - 1].
__global__ void k_phi0(const float *__restrict__ out, int B, int H, int W, float lo, float hi, int is_mod,
                       float *__restrict__ phi0) {
    const int W4 = 4 * W, H4 = 4 * H;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)B * H4 * W4) return;
    const int xx = (int)(id % W4);
    const long long r = id / W4;
    const int yy = (int)(r % H4), b = (int)(r / H4);
    const float ty = fminf(fmaxf((yy + 0.5f) * 0.25f - 0.5f, 0.f), (float)(H - 1));
    const float tx = fminf(fmaxf((xx + 0.5f) * 0.25f - 0.5f, 0.f), (float)(W - 1));
    const int y0 = (int)ty, x0 = (int)tx;
    const int y1 = min(y0 + 1, H - 1), x1 = min(x0 + 1, W - 1);
    const float fy = ty - y0, fx = tx - x0;
    const float *o = out + (size_t)b * H * W;
    // phi_0: 100 x bilinear of the prediction, clipped; modulation: bilinear
    // of H_eps of the prediction
    auto val = [&](int yy_, int xx_) {
        const float v = o[(size_t)yy_ * W + xx_];
        return is_mod ? ahf(v) : v;
    };
    const float top = val(y0, x0) * (1.f - fx) + val(y0, x1) * fx;
    const float bot = val(y1, x0) * (1.f - fx) + val(y1, x1) * fx;
    const float v = top * (1.f - fy) + bot * fy;
    phi0[id] = is_mod ? v : fminf(fmaxf(DSN_SCALE * v, lo), hi);
}

inline unsigned grid1(long long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// The same convolution for 32 input channels (one chunk), persistent: the
// block's weights are staged once and kept in registers, and the block walks
// tiles blockIdx.x, blockIdx.x + gridDim.x, ... with the next tile's input
// loads in flight while the current tile is multiplied.
template <bool UP, int TC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_conv_lds32(
    View x, int B, int H, int W, const __bf16 *__restrict__ w, const float *__restrict__ bias, int relu, View y,
    View mask) {
    constexpr int RW = TC == 64 ? 8 : 4;
    __shared__ __attribute__((aligned(16))) __bf16 Xs[CL_NPX * CL_XS];
    __shared__ __attribute__((aligned(16))) __bf16 Ws[TC * CL_WS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int strip = wave & 1;
    const int cw = TC == 64 ? 32 * (wave >> 1) : 0, row0 = TC == 64 ? 0 : 4 * (wave >> 1);
    const int ntx = (W + CL_TX - 1) / CL_TX, nty = (H + CL_TY - 1) / CL_TY;
    const int ntiles = B * nty * ntx;
    const int co0 = blockIdx.y * TC;
    const int Hin = UP ? H / 2 : H, Win = UP ? W / 2 : W;
    constexpr int XU = (CL_NPX * 4 + 255) / 256;
    for (int e = threadIdx.x; e < TC * 36; e += 256) {
        const int col = e / 36, rem = e % 36;
        *reinterpret_cast<bf8 *>(&Ws[col * CL_WS + (rem / 4) * 32 + 8 * (rem % 4)]) =
            *reinterpret_cast<const bf8 *>(w + ((size_t)(co0 + col) * 9 + rem / 4) * 32 + 8 * (rem % 4));
    }
    __syncthreads();
    bf8 a[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
            a[t][cb] = *reinterpret_cast<const bf8 *>(&Ws[(cw + 16 * cb + l16) * CL_WS + t * 32 + 8 * lq]);
    bf8 xv[XU];
    auto fetch = [&](int tile) {
        const int tix = tile % ntx, rest = tile / ntx;
        const int tiy = rest % nty, b = rest / nty;
        const int x0 = tix * CL_TX, y0 = tiy * CL_TY;
#pragma unroll
        for (int u = 0; u < XU; ++u) {
            const int e = threadIdx.x + 256 * u;
            xv[u] = bf8_zero();
            if (e < CL_NPX * 4) {
                const int px = e >> 2, seg = e & 3;
                const int gy = y0 + px / (CL_TX + 2) - 1, gx = x0 + px % (CL_TX + 2) - 1;
                if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
                    const int sy = UP ? (gy >> 1) : gy, sx = UP ? (gx >> 1) : gx;
                    xv[u] = *reinterpret_cast<const bf8 *>(x.p + (((size_t)b * Hin + sy) * Win + sx) * x.stride +
                                                           8 * seg);
                }
            }
        }
    };
    if ((int)blockIdx.x < ntiles) fetch(blockIdx.x);
    const __bf16 *xcol = Xs + (16 * strip + l16) * CL_XS + 8 * lq;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        __syncthreads();                              // the previous tile's reads are done
#pragma unroll
        for (int u = 0; u < XU; ++u) {
            const int e = threadIdx.x + 256 * u;
            if (e < CL_NPX * 4) *reinterpret_cast<bf8 *>(&Xs[(e >> 2) * CL_XS + 8 * (e & 3)]) = xv[u];
        }
        __syncthreads();
        if (tile + (int)gridDim.x < ntiles) fetch(tile + gridDim.x);
        f4 acc[RW][2];
#pragma unroll
        for (int r = 0; r < RW; ++r) acc[r][0] = acc[r][1] = f4{0.f, 0.f, 0.f, 0.f};
        bf8 bw[3][3];
        auto load_row = [&](int hr, bf8(&o)[3]) {
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
                o[dx] = *reinterpret_cast<const bf8 *>(xcol + ((row0 + hr) * (CL_TX + 2) + dx) * CL_XS);
        };
        load_row(0, bw[0]);
        load_row(1, bw[1]);
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            load_row(r + 2, bw[(r + 2) % 3]);
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        acc[r][cb] = mfma_b(a[3 * dy + dx][cb], bw[(r + dy) % 3][dx], acc[r][cb]);
        }
        const int tix = tile % ntx, rest = tile / ntx;
        const int tiy = rest % nty, b = rest / nty;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int gy = tiy * CL_TY + row0 + r, gx = tix * CL_TX + 16 * strip + l16;
            if (gy >= H || gx >= W) continue;
            const long long pix = ((long long)b * H + gy) * W + gx;
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const int c = co0 + cw + 16 * cb + 4 * lq;
                bf4 o;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float v = acc[r][cb][i] + (bias ? bias[c + i] : 0.f);
                    if (relu) v = fmaxf(v, 0.f);
                    o[i] = (__bf16)v;
                }
                if (mask.p) {
                    const bf4 m = *reinterpret_cast<const bf4 *>(mask.p + pix * mask.stride + c);
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (!((float)m[i] > 0.f)) o[i] = (__bf16)0.f;
                }
                *reinterpret_cast<bf4 *>(y.p + pix * y.stride + c) = o;
            }
        }
    }
}

// Kernel of a 3x3 convolution: the LDS-staged tiles from 8 x 32 pixels up,
// register tiles of 32 x 32 per wave (operands straight from global memory)
// for smaller images.
template <bool UP>
void launch_conv_tiles(View x, int B, int H, int W, const __bf16 *w, int Cin, const float *bias, int relu, int Cout,
                       View y, View mask, hipStream_t st) {
    if (H >= CL_TY && W >= CL_TX) {
        const long long tiles = (long long)B * ((H + CL_TY - 1) / CL_TY) * ((W + CL_TX - 1) / CL_TX);
        if (Cin == 32) {
            // two resident blocks per compute unit
            const unsigned nb = (unsigned)std::min<long long>(tiles, 512);
            if (Cout % 64 == 0)
                k_conv_lds32<UP, 64><<<dim3(nb, Cout / 64), 256, 0, st>>>(x, B, H, W, w, bias, relu, y, mask);
            else
                k_conv_lds32<UP, 32><<<dim3(nb, Cout / 32), 256, 0, st>>>(x, B, H, W, w, bias, relu, y, mask);
            return;
        }
        if (Cout % 64 == 0)
            k_conv_lds<UP, 64><<<dim3((unsigned)tiles, Cout / 64), 256, 0, st>>>(x, B, H, W, w, Cin, bias, relu, y,
                                                                                mask);
        else
            k_conv_lds<UP, 32><<<dim3((unsigned)tiles, Cout / 32), 256, 0, st>>>(x, B, H, W, w, Cin, bias, relu, y,
                                                                                mask);
        return;
    }
    const long long npix = (long long)B * H * W;
    if (Cout % 64 == 0)
        k_conv<2, 2, 2, 2, UP><<<dim3(grid1(npix, 64), Cout / 64), 256, 0, st>>>(x, B, H, W, w, Cin, bias, relu, y,
                                                                                mask);
    else
        k_conv<4, 1, 2, 2, UP><<<dim3(grid1(npix, 128), Cout / 32), 256, 0, st>>>(x, B, H, W, w, Cin, bias, relu, y,
                                                                                 mask);
}

// mask (or a NULL view): the output is zeroed where mask <= 0, the backward
// of a ReLU whose output is mask, fused into the producer of the gradient
void launch_conv(View x, int B, int H, int W, const __bf16 *w, int Cin, const float *bias, int relu, int Cout, bool up,
                 View y, View mask, hipStream_t st) {
    if (up) launch_conv_tiles<true>(x, B, H, W, w, Cin, bias, relu, Cout, y, mask, st);
    else launch_conv_tiles<false>(x, B, H, W, w, Cin, bias, relu, Cout, y, mask, st);
}

}  // namespace

// ---------------------------------------------------------------- host side

struct dsn_layer {
    int cin, cout;
    long long w_off, b_off;   // offsets in the flat parameter vector
};

struct dsn_ctx {
    int H, W, base, maxB, modulation;
    hipStream_t stream;
    int C[DSN_LEVELS], h[DSN_LEVELS], w[DSN_LEVELS];
    long long np[DSN_LEVELS];          // pixels per level at max batch
    std::vector<dsn_layer> L;          // parameter order
    long long n_params;
    float *p = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    __bf16 *pb = nullptr, *pt = nullptr;   // BF16 weights, flipped/transposed copies
    int step = 0;
    // activations
    float *x_in = nullptr;                 // forward input [B][H][W] (caller's, kept)
    __bf16 *act_a[DSN_LEVELS] = {}, *cat[DSN_LEVELS] = {}, *pool[DSN_LEVELS] = {}, *bott = nullptr;
    __bf16 *dec_a[DSN_LEVELS] = {}, *dec_b[DSN_LEVELS] = {};
    float *out = nullptr;                  // forward output [B][H][W] (caller's, kept)
    float *out_m = nullptr;                // modulation output of the last forward (caller's) or NULL
    int fwdB = 0;
    // gradients
    __bf16 *gA[DSN_LEVELS] = {}, *gB[DSN_LEVELS] = {}, *gcat[DSN_LEVELS] = {};
    float *part = nullptr;
    long long part_cap = 0;
    double *lpart = nullptr;
    float *hpart = nullptr;
    float *net_x = nullptr, *net_out = nullptr, *net_out_m = nullptr;   // predict scratch
    std::vector<void *> allocs;
};

namespace {

// layer indices: enc l a = 2l, enc l b = 2l + 1; dec l: 8 + 3 (2 - l) + {0 up, 1 a, 2 b}; head 17;
// modulation head 18.  Only the layers before the heads are 3x3 convolutions.
inline int enc_a(int l) { return 2 * l; }
inline int enc_b(int l) { return 2 * l + 1; }
inline int dec_up(int l) { return 2 * DSN_LEVELS + 3 * (DSN_LEVELS - 2 - l); }
inline int dec_a_i(int l) { return dec_up(l) + 1; }
inline int dec_b_i(int l) { return dec_up(l) + 2; }
inline int head_i() { return 2 * DSN_LEVELS + 3 * (DSN_LEVELS - 1); }
inline int head_m_i() { return head_i() + 1; }

View view(__bf16 *p, int C, int stride) { return View{p, C, stride}; }

int splits_for(long long npix) {
    long long s = npix / 4096;
    return (int)std::max(1LL, std::min(256LL, s));
}

// Splits of the tiled weight gradient: about 1024 blocks in all, each over
// a range of whole 8 x 32 tiles, with at most WG_PART_MAX floats of partials.
constexpr long long WG_PART_MAX = 32LL << 20;

long long wgrad_tiles(int B, int H, int W) {
    return (long long)B * ((H + WT_TY - 1) / WT_TY) * ((W + WT_TX - 1) / WT_TX);
}

// at most this many splits for B images (and so for any smaller batch)
long long wgrad_tile_split_bound(int B, int H, int W, int Cin, int Cout) {
    const int tco = Cout % 64 == 0 ? 64 : 32, tci = Cin % 64 == 0 ? 64 : 32;
    const long long gxy = (long long)(Cout / tco) * (Cin / tci);
    long long S = (1024 + gxy - 1) / gxy;
    S = std::min(S, std::max(1LL, WG_PART_MAX / ((long long)Cout * 9 * Cin)));
    return std::max(1LL, std::min(S, wgrad_tiles(B, H, W)));
}

int wgrad_tile_splits(int B, int H, int W, int Cin, int Cout, long long *tiles_per_split) {
    const long long ntiles = wgrad_tiles(B, H, W);
    const long long tps = (ntiles + wgrad_tile_split_bound(B, H, W, Cin, Cout) - 1) /
                          wgrad_tile_split_bound(B, H, W, Cin, Cout);
    *tiles_per_split = tps;
    return (int)((ntiles + tps - 1) / tps);
}

// dW (cout x 9 x cin) and db (cout) of a 3x3 layer, through cap floats of
// partials at part.  hipErrorInvalidValue when the partials do not fit.
long long wgrad_part_floats(long long S, int Cin, int Cout) {
    const int nwc = (Cin % 64 == 0 ? 64 : 32) / 16;
    return S * Cout * 9 * Cin + S * nwc * Cout;
}

hipError_t launch_wgrad_tile(View dz, View x, int B, int H, int W, int Cin, int Cout, bool up, float *part,
                             long long cap, float *dw, float *db, hipStream_t st) {
    long long tps = 0;
    const int S = wgrad_tile_splits(B, H, W, Cin, Cout, &tps);
    if (wgrad_part_floats(S, Cin, Cout) > cap) return hipErrorInvalidValue;
    const int tco = Cout % 64 == 0 ? 64 : 32, tci = Cin % 64 == 0 ? 64 : 32;
    const dim3 grid(Cout / tco, Cin / tci, S);
    const int tp = (int)tps;
    float *bpart = part + (size_t)S * Cout * 9 * Cin;
#define WG(A, Bq)                                                                                        \
    if (up) k_wgrad_tile<A, Bq, true><<<grid, (A / 32) * (Bq / 16) * 64, 0, st>>>(dz, x, B, H, W, Cin, Cout, tp, part, bpart); \
    else k_wgrad_tile<A, Bq, false><<<grid, (A / 32) * (Bq / 16) * 64, 0, st>>>(dz, x, B, H, W, Cin, Cout, tp, part, bpart)
    if (tco == 64 && tci == 64) WG(64, 64);
    else if (tco == 64) WG(64, 32);
    else if (tci == 64) WG(32, 64);
    else WG(32, 32);
#undef WG
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    reduce_splits(part, S, (long long)Cout * 9 * Cin, dw, st);
    reduce_splits(bpart, S * (tci / 16), Cout, db, st);
    return hipGetLastError();
}

template <typename T>
hipError_t dalloc(dsn_ctx *c, T **p, size_t n) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
    if (e == hipSuccess) {
        c->allocs.push_back(q);
        *p = static_cast<T *>(q);
    }
    return e;
}

void free_all(dsn_ctx *c) {
    for (void *q : c->allocs) (void)hipFree(q);
    c->allocs.clear();
}

int conv(dsn_ctx *c, View x, int B, int l, int layer_i, bool up, bool transposed, int relu, View y,
         View mask = View{}) {
    // forward: weights pb[layer] [cout][9][cin]; input gradient: pt[layer] [cin][9][cout]
    const dsn_layer &ly = c->L[layer_i];
    const int Cin = transposed ? ly.cout : ly.cin, Cout = transposed ? ly.cin : ly.cout;
    const __bf16 *w = (transposed ? c->pt : c->pb) + ly.w_off;
    const float *bias = transposed ? nullptr : c->p + ly.b_off;
    if (Cin % 32 || Cout % 32 || x.C != Cin || y.C != Cout) return fail(DSN_EINVAL, "conv shape mismatch");
    launch_conv(x, B, c->h[l], c->w[l], w, Cin, bias, relu, Cout, up, y, mask, c->stream);
    HIPCHK(hipGetLastError());
    return DSN_OK;
}

// weight and bias gradients of a 3x3 layer (input view x, output gradient dz)
int wgrad(dsn_ctx *c, View dz, View x, int B, int l, int layer_i, bool up) {
    const dsn_layer &ly = c->L[layer_i];
    const hipError_t e = launch_wgrad_tile(dz, x, B, c->h[l], c->w[l], ly.cin, ly.cout, up, c->part, c->part_cap,
                                           c->grad + ly.w_off, c->grad + ly.b_off, c->stream);
    if (e == hipErrorInvalidValue) return fail(DSN_EINVAL, "weight-gradient scratch too small");
    HIPCHK(e);
    return DSN_OK;
}

// First layer's weight gradient: ranges of 4096 pixels (up to 2048 blocks)
// while the partials (S x C x 10 floats) fit cap; ranges of splits_for()
// otherwise.
int first_layer_splits(long long npix, int C, long long cap) {
    int S = (int)std::max(1LL, std::min(2048LL, npix / 4096));
    if ((long long)S * C * 10 > cap) S = splits_for(npix);
    return S;
}

// dw [C][9] and db [C] of the first layer from S range partials in part
hipError_t launch_wgrad_first(View dz, const float *x, int B, int H, int W, int S, float *part, float *dw, float *db,
                              hipStream_t st) {
    const long long np = (long long)B * H * W;
    const long long pps = (np + S - 1) / S;
    k_wgrad_first<<<S, 256, 0, st>>>(dz, x, B, H, W, pps, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    reduce_splits(part, S, (long long)dz.C * 9, dw, st);
    reduce_splits(part + (size_t)S * dz.C * 9, S, dz.C, db, st);
    return hipGetLastError();
}

// Head backward over npix pixels of the features x: the input gradient dx,
// the losses (d_loss[2], averaged over B) and the heads' weight and bias
// gradients (gw [heads][C + 1]) from per-block partials in lpart / hpart.
// relu_mask: dx is also zeroed where x <= 0 (the backward of the ReLU that
// produced x)
hipError_t launch_head_bwd(View x, long long npix, int B, const __bf16 *w, const __bf16 *wm, const float *out,
                           const float *out_m, const float *tgt, const float *tgt_m, View dx, int relu_mask,
                           double *lpart, float *hpart, double *d_loss, float *gw, hipStream_t st) {
    const unsigned nblk = grid1(npix);
    k_head_bwd<<<nblk, 256, 0, st>>>(x, npix, B, w, wm, out, out_m, tgt, tgt_m, dx, relu_mask, lpart, hpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_loss_finish<<<1, 256, 0, st>>>(lpart, (int)nblk, B, d_loss);
    reduce_splits(hpart, (int)nblk, (out_m ? 2 : 1) * (x.C + 1), gw, st);
    return hipGetLastError();
}

int check_ctx(const dsn_ctx *c) { return c ? DSN_OK : fail(DSN_EINVAL, "context is NULL"); }

int check_ptr(const void *p, const char *name) {
    if (!p) return fail(DSN_EINVAL, "%s is NULL", name);
    if (reinterpret_cast<uintptr_t>(p) % 16) return fail(DSN_EINVAL, "%s is not 16-byte aligned", name);
    return DSN_OK;
}

}  // namespace

extern "C" const char *dsn_last_error(void) { return g_err.c_str(); }

extern "C" int dsn_create(dsn_ctx **out, int H, int W, int base, int maxB, int modulation, void *stream) {
    if (!out) return fail(DSN_EINVAL, "out is NULL");
    *out = nullptr;
    if (H < 8 || W < 8 || H % 8 || W % 8 || H > 2048 || W > 2048)
        return fail(DSN_EINVAL, "H and W must be multiples of 8 in [8, 2048]");
    if (base != 32 && base != 64) return fail(DSN_EINVAL, "base must be 32 or 64");
    if (maxB < 1) return fail(DSN_EINVAL, "max_batch must be >= 1");
    if ((long long)maxB * H * W >= (1LL << 31)) return fail(DSN_EINVAL, "max_batch H W must be below 2^31");
    if (modulation != 0 && modulation != 1) return fail(DSN_EINVAL, "modulation must be 0 or 1");
    dsn_ctx *c = new (std::nothrow) dsn_ctx();
    if (!c) return fail(DSN_ENOMEM, "out of host memory");
    c->H = H;
    c->W = W;
    c->base = base;
    c->maxB = maxB;
    c->modulation = modulation;
    c->stream = static_cast<hipStream_t>(stream);
    for (int l = 0; l < DSN_LEVELS; ++l) {
        c->C[l] = base << l;
        c->h[l] = H >> l;
        c->w[l] = W >> l;
        c->np[l] = (long long)maxB * c->h[l] * c->w[l];
    }
    // parameter table
    long long off = 0;
    auto add = [&](int cin, int cout, int taps) {
        dsn_layer ly{cin, cout, off, off + (long long)cout * taps * cin};
        off = ly.b_off + cout;
        c->L.push_back(ly);
    };
    int prev = 1;
    for (int l = 0; l < DSN_LEVELS; ++l) {
        add(prev, c->C[l], 9);
        add(c->C[l], c->C[l], 9);
        prev = c->C[l];
    }
    for (int l = DSN_LEVELS - 2; l >= 0; --l) {
        add(c->C[l + 1], c->C[l], 9);
        add(2 * c->C[l], c->C[l], 9);
        add(c->C[l], c->C[l], 9);
    }
    add(c->C[0], 1, 1);
    if (modulation) add(c->C[0], 1, 1);
    c->n_params = off;
    // scratch for split weight gradients: the largest S * Cout * 9 * Cin
    long long cap = 0;
    for (int i = 0; i < head_i(); ++i) {
        int l = 0;
        if (i < 2 * DSN_LEVELS) l = (int)i / 2;
        else l = DSN_LEVELS - 2 - (int)(i - 2 * DSN_LEVELS) / 3;
        const long long S = splits_for(c->np[l]);
        cap = std::max(cap, S * c->L[i].cout * 9 * std::max(c->L[i].cin, 1) + S * c->L[i].cout);
        if (c->L[i].cin % 32 == 0 && c->L[i].cout % 32 == 0) {
            const long long St = wgrad_tile_split_bound(maxB, c->h[l], c->w[l], c->L[i].cin, c->L[i].cout);
            cap = std::max(cap, wgrad_part_floats(St, c->L[i].cin, c->L[i].cout));
        }
    }
    c->part_cap = cap;
    hipError_t e = hipSuccess;
    const long long n = c->n_params;
    if (e == hipSuccess) e = dalloc(c, &c->p, n);
    if (e == hipSuccess) e = dalloc(c, &c->m, n);
    if (e == hipSuccess) e = dalloc(c, &c->v, n);
    if (e == hipSuccess) e = dalloc(c, &c->grad, n);
    if (e == hipSuccess) e = dalloc(c, &c->pb, n);
    if (e == hipSuccess) e = dalloc(c, &c->pt, n);
    if (e == hipSuccess) e = dalloc(c, &c->part, cap);
    for (int l = 0; l < DSN_LEVELS && e == hipSuccess; ++l) {
        const long long np = c->np[l];
        const int C = c->C[l];
        e = dalloc(c, &c->act_a[l], np * C);
        if (e == hipSuccess && l < DSN_LEVELS - 1) e = dalloc(c, &c->cat[l], np * 2 * C);
        if (e == hipSuccess && l < DSN_LEVELS - 1) e = dalloc(c, &c->pool[l], c->np[l + 1] * C);
        if (e == hipSuccess && l < DSN_LEVELS - 1) e = dalloc(c, &c->dec_a[l], np * C);
        if (e == hipSuccess && l < DSN_LEVELS - 1) e = dalloc(c, &c->dec_b[l], np * C);
        if (e == hipSuccess && l < DSN_LEVELS - 1) e = dalloc(c, &c->gcat[l], np * 2 * C);
        if (e == hipSuccess) e = dalloc(c, &c->gA[l], np * 2 * C);
        if (e == hipSuccess) e = dalloc(c, &c->gB[l], np * 2 * C);
    }
    if (e == hipSuccess) e = dalloc(c, &c->bott, c->np[DSN_LEVELS - 1] * c->C[DSN_LEVELS - 1]);
    const long long nblk = (c->np[0] + 255) / 256;
    if (e == hipSuccess) e = dalloc(c, &c->lpart, 2 * nblk);
    if (e == hipSuccess) e = dalloc(c, &c->hpart, nblk * 2 * (c->C[0] + 1));
    if (e == hipSuccess) e = dalloc(c, &c->net_x, c->np[0]);
    if (e == hipSuccess) e = dalloc(c, &c->net_out, c->np[0]);
    if (e == hipSuccess && modulation) e = dalloc(c, &c->net_out_m, c->np[0]);
    if (e == hipSuccess) e = hipMemsetAsync(c->p, 0, n * sizeof(float), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->pb, 0, n * sizeof(__bf16), c->stream);
    if (e != hipSuccess) {
        free_all(c);
        delete c;
        return fail(e == hipErrorOutOfMemory ? DSN_ENOMEM : DSN_EDEVICE, "dsn_create: %s", hipGetErrorString(e));
    }
    *out = c;
    return DSN_OK;
}

extern "C" int dsn_destroy(dsn_ctx *c) {
    if (!c) return fail(DSN_EINVAL, "context is NULL");
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
    return DSN_OK;
}

extern "C" long long dsn_num_params(const dsn_ctx *c) { return c ? c->n_params : -1; }

extern "C" int dsn_set_params(dsn_ctx *c, const float *d) {
    int r;
    if ((r = check_ctx(c)) || (r = check_ptr(d, "d_params"))) return r;
    const long long n = c->n_params;
    HIPCHK(hipMemcpyAsync(c->p, d, n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    k_to_bf16<<<grid1(n), 256, 0, c->stream>>>(c->p, n, c->pb);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemsetAsync(c->m, 0, n * sizeof(float), c->stream));
    HIPCHK(hipMemsetAsync(c->v, 0, n * sizeof(float), c->stream));
    c->step = 0;
    return DSN_OK;
}

extern "C" int dsn_get_params(const dsn_ctx *c, float *d) {
    int r;
    if ((r = check_ctx(c)) || (r = check_ptr(d, "d_params"))) return r;
    HIPCHK(hipMemcpyAsync(d, c->p, c->n_params * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    return DSN_OK;
}

extern "C" int dsn_forward(dsn_ctx *c, const float *d_x, int B, float *d_out, float *d_out_m) {
    int r;
    if ((r = check_ctx(c)) || (r = check_ptr(d_x, "d_x")) || (r = check_ptr(d_out, "d_out"))) return r;
    if (d_out_m && (r = check_ptr(d_out_m, "d_out_m"))) return r;
    if (d_out_m && !c->modulation) return fail(DSN_EINVAL, "d_out_m given but the network has no modulation head");
    if (B < 1 || B > c->maxB) return fail(DSN_EINVAL, "B must be in [1, %d]", c->maxB);
    const int NL = DSN_LEVELS;
    // encoder
    {
        const dsn_layer &ly = c->L[enc_a(0)];
        const long long npix = (long long)B * c->h[0] * c->w[0];
        k_conv_first<<<grid1(npix), 256, (size_t)c->C[0] * 10 * sizeof(float), c->stream>>>(
            d_x, B, c->h[0], c->w[0], c->pb + ly.w_off, c->p + ly.b_off, view(c->act_a[0], c->C[0], c->C[0]));
        HIPCHK(hipGetLastError());
    }
    for (int l = 0; l < NL; ++l) {
        const int C = c->C[l];
        if (l > 0) {
            if ((r = conv(c, view(c->pool[l - 1], c->C[l - 1], c->C[l - 1]), B, l, enc_a(l), false, false, 1,
                          view(c->act_a[l], C, C))))
                return r;
        }
        View yb = l < NL - 1 ? view(c->cat[l] + C, C, 2 * C) : view(c->bott, C, C);
        if ((r = conv(c, view(c->act_a[l], C, C), B, l, enc_b(l), false, false, 1, yb))) return r;
        if (l < NL - 1) {
            const long long n = (long long)B * c->h[l + 1] * c->w[l + 1] * (C / 8);
            k_maxpool<<<grid1(n), 256, 0, c->stream>>>(yb, B, c->h[l], c->w[l], view(c->pool[l], C, C));
            HIPCHK(hipGetLastError());
        }
    }
    // decoder
    for (int l = NL - 2; l >= 0; --l) {
        const int C = c->C[l], C1 = c->C[l + 1];
        View below = l == NL - 2 ? view(c->bott, C1, C1) : view(c->dec_b[l + 1], C1, C1);
        if ((r = conv(c, below, B, l, dec_up(l), true, false, 1, view(c->cat[l], C, 2 * C)))) return r;
        if ((r = conv(c, view(c->cat[l], 2 * C, 2 * C), B, l, dec_a_i(l), false, false, 1, view(c->dec_a[l], C, C))))
            return r;
        if ((r = conv(c, view(c->dec_a[l], C, C), B, l, dec_b_i(l), false, false, 1, view(c->dec_b[l], C, C))))
            return r;
    }
    const dsn_layer &hd = c->L[head_i()];
    const long long npix = (long long)B * c->h[0] * c->w[0];
    const dsn_layer &hm = c->L[c->modulation ? head_m_i() : head_i()];
    k_head<<<grid1(npix), 256, 0, c->stream>>>(view(c->dec_b[0], c->C[0], c->C[0]), npix, c->pb + hd.w_off,
                                               c->p + hd.b_off, c->pb + hm.w_off, c->p + hm.b_off, d_out, d_out_m);
    HIPCHK(hipGetLastError());
    c->x_in = const_cast<float *>(d_x);
    c->out = d_out;
    c->out_m = d_out_m;
    c->fwdB = B;
    return DSN_OK;
}

extern "C" int dsn_backward(dsn_ctx *c, const float *d_target, const float *d_target_m, int B, double *d_loss,
                            float *d_grad) {
    int r;
    if ((r = check_ctx(c)) || (r = check_ptr(d_target, "d_target"))) return r;
    if (d_target_m && (r = check_ptr(d_target_m, "d_target_m"))) return r;
    if (d_target_m && !c->out_m) return fail(DSN_EINVAL, "d_target_m needs a forward pass with d_out_m");
    if (!d_loss) return fail(DSN_EINVAL, "d_loss is NULL");
    if (d_grad && (r = check_ptr(d_grad, "d_grad"))) return r;
    if (B != c->fwdB || !c->out) return fail(DSN_EINVAL, "backward needs a forward pass with the same batch");
    const int NL = DSN_LEVELS;
    // flipped/transposed weights for the input gradients
    for (int i = 0; i < head_i(); ++i) {
        const dsn_layer &ly = c->L[i];
        const long long n = (long long)ly.cout * 9 * ly.cin;
        k_flip_transpose<<<grid1(n), 256, 0, c->stream>>>(c->pb + ly.w_off, ly.cout, ly.cin, c->pt + ly.w_off);
        HIPCHK(hipGetLastError());
    }
    // head and loss
    const int C0 = c->C[0];
    const long long np0 = (long long)B * c->h[0] * c->w[0];
    const dsn_layer &hd = c->L[head_i()];
    // the modulation head takes part only when its target is given; otherwise
    // its gradient is zero and L_m is reported as 0
    const int with_m = d_target_m != nullptr;
    const dsn_layer &hm = c->L[c->modulation ? head_m_i() : head_i()];
    // hpart [nblk][heads][C0 + 1] -> each head's weights then bias; the two
    // heads are adjacent in the flat vector
    // every ReLU's backward is fused into the kernel that produces the
    // gradient of its output (a mask by the stored activation)
    HIPCHK(launch_head_bwd(view(c->dec_b[0], C0, C0), np0, B, c->pb + hd.w_off, c->pb + hm.w_off, c->out,
                           with_m ? c->out_m : nullptr, d_target, d_target_m, view(c->gA[0], C0, C0), 1, c->lpart,
                           c->hpart, d_loss, c->grad + hd.w_off, c->stream));
    if (c->modulation && !with_m) {
        k_fill_f32<<<1, 256, 0, c->stream>>>(c->grad + hm.w_off, C0 + 1, 0.f);
        HIPCHK(hipGetLastError());
    }
    // decoder, bottom-up in the backward order
    for (int l = 0; l <= NL - 2; ++l) {
        const int C = c->C[l], C1 = c->C[l + 1];
        View gy = view(c->gA[l], C, C);                        // d(dec_b pre-activation)
        if ((r = wgrad(c, gy, view(c->dec_a[l], C, C), B, l, dec_b_i(l), false))) return r;
        View ga = view(c->gB[l], C, C);
        if ((r = conv(c, gy, B, l, dec_b_i(l), false, true, 0, ga, view(c->dec_a[l], C, C)))) return r;
        if ((r = wgrad(c, ga, view(c->cat[l], 2 * C, 2 * C), B, l, dec_a_i(l), false))) return r;
        // both halves of the concatenation are ReLU outputs (up-convolution,
        // skip): the mask covers all 2C channels
        View gc = view(c->gcat[l], 2 * C, 2 * C);
        if ((r = conv(c, ga, B, l, dec_a_i(l), false, true, 0, gc, view(c->cat[l], 2 * C, 2 * C)))) return r;
        View gu = view(c->gcat[l], C, 2 * C);                  // d(up-convolution pre-activation)
        View below = l == NL - 2 ? view(c->bott, C1, C1) : view(c->dec_b[l + 1], C1, C1);
        if ((r = wgrad(c, gu, below, B, l, dec_up(l), true))) return r;
        View gfull = view(c->gA[l], C1, C1);                   // gradient of the upsampled input
        if ((r = conv(c, gu, B, l, dec_up(l), false, true, 0, gfull))) return r;
        const long long n = (long long)B * c->h[l + 1] * c->w[l + 1] * (C1 / 8);
        k_upsample_bwd<<<grid1(n), 256, 0, c->stream>>>(gfull, B, c->h[l], c->w[l], view(c->gA[l + 1], C1, C1),
                                                        below);
        HIPCHK(hipGetLastError());
    }
    // encoder, top-down
    for (int l = NL - 1; l >= 0; --l) {
        const int C = c->C[l];
        const long long np = (long long)B * c->h[l] * c->w[l];
        View yb, gyb;
        if (l == NL - 1) {
            yb = view(c->bott, C, C);
            gyb = view(c->gA[l], C, C);
        } else {
            yb = view(c->cat[l] + C, C, 2 * C);
            gyb = view(c->gcat[l] + C, C, 2 * C);
            // add the pooled path's gradient (held in gA[l + 1]) to the skip's
            // (already masked) and mask the sum by yb
            const long long n = (long long)B * c->h[l + 1] * c->w[l + 1] * (C / 8);
            k_maxpool_bwd<true><<<grid1(n), 256, 0, c->stream>>>(yb, B, c->h[l], c->w[l], view(c->gA[l + 1], C, C),
                                                               gyb);
            HIPCHK(hipGetLastError());
        }
        if ((r = wgrad(c, gyb, view(c->act_a[l], C, C), B, l, enc_b(l), false))) return r;
        View ga = view(c->gB[l], C, C);
        if ((r = conv(c, gyb, B, l, enc_b(l), false, true, 0, ga, view(c->act_a[l], C, C)))) return r;
        if (l > 0) {
            const int Cp = c->C[l - 1];
            if ((r = wgrad(c, ga, view(c->pool[l - 1], Cp, Cp), B, l, enc_a(l), false))) return r;
            // gradient of the pooled input, kept in gA[l] for the level above
            if ((r = conv(c, ga, B, l, enc_a(l), false, true, 0, view(c->gA[l], Cp, Cp)))) return r;
        } else {
            const dsn_layer &ly = c->L[enc_a(0)];
            const int S = first_layer_splits(np, ly.cout, c->part_cap);
            HIPCHK(launch_wgrad_first(ga, c->x_in, B, c->h[0], c->w[0], S, c->part, c->grad + ly.w_off,
                                      c->grad + ly.b_off, c->stream));
        }
    }
    if (d_grad)
        HIPCHK(hipMemcpyAsync(d_grad, c->grad, c->n_params * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    return DSN_OK;
}

extern "C" int dsn_adam_step(dsn_ctx *c, float lr, float b1, float b2, float eps) {
    int r;
    if ((r = check_ctx(c))) return r;
    if (!(lr >= 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
        return fail(DSN_EINVAL, "bad Adam hyperparameters");
    c->step += 1;
    const float c1 = 1.f - std::pow(b1, (float)c->step), c2 = 1.f - std::pow(b2, (float)c->step);
    k_adam<<<grid1(c->n_params), 256, 0, c->stream>>>(c->p, c->m, c->v, c->grad, c->n_params, lr, b1, b2, eps, c1,
                                                      c2, c->pb);
    HIPCHK(hipGetLastError());
    return DSN_OK;
}

extern "C" int dsn_prepare(dsn_ctx *c, const unsigned char *d_target, const float *d_phi_gt, const float *d_m_gt,
                           int B, float *d_x, float *d_t, float *d_t_m) {
    int r;
    if ((r = check_ctx(c)) || (r = check_ptr(d_target, "d_target")) || (r = check_ptr(d_x, "d_x"))) return r;
    if (d_phi_gt && ((r = check_ptr(d_phi_gt, "d_phi_gt")) || (r = check_ptr(d_t, "d_t")))) return r;
    if (d_m_gt && ((r = check_ptr(d_m_gt, "d_m_gt")) || (r = check_ptr(d_t_m, "d_t_m")))) return r;
    if (B < 1) return fail(DSN_EINVAL, "B must be >= 1");
    k_prepare<<<grid1((long long)B * c->H * c->W), 256, 0, c->stream>>>(d_target, d_phi_gt, d_m_gt, B, c->H, c->W,
                                                                        d_x, d_t, d_t_m);
    HIPCHK(hipGetLastError());
    return DSN_OK;
}

extern "C" int dsn_predict(dsn_ctx *c, const unsigned char *d_target, int B, float lo, float hi, float *d_phi0,
                           float *d_m0) {
    int r;
    if ((r = check_ctx(c)) || (r = check_ptr(d_target, "d_target")) || (r = check_ptr(d_phi0, "d_phi0"))) return r;
    if (d_m0 && (r = check_ptr(d_m0, "d_m0"))) return r;
    if (d_m0 && !c->modulation) return fail(DSN_EINVAL, "d_m0 given but the network has no modulation head");
    if (B < 1 || B > c->maxB) return fail(DSN_EINVAL, "B must be in [1, %d]", c->maxB);
    if (!(lo < hi)) return fail(DSN_EINVAL, "d_lower must be below d_upper");
    if ((r = dsn_prepare(c, d_target, nullptr, nullptr, B, c->net_x, nullptr, nullptr))) return r;
    if ((r = dsn_forward(c, c->net_x, B, c->net_out, d_m0 ? c->net_out_m : nullptr))) return r;
    const long long n = (long long)B * 16 * c->H * c->W;
    k_phi0<<<grid1(n), 256, 0, c->stream>>>(c->net_out, B, c->H, c->W, lo, hi, 0, d_phi0);
    HIPCHK(hipGetLastError());
    if (d_m0) {
        k_phi0<<<grid1(n), 256, 0, c->stream>>>(c->net_out_m, B, c->H, c->W, 0.f, 1.f, 1, d_m0);
        HIPCHK(hipGetLastError());
    }
    return DSN_OK;
}

// ---------------------------------------------------------------- single operations

namespace {

int op_conv(View x, int N, int H, int W, int Cin, bool up, const __bf16 *w, const float *b, int Cout, int relu,
            View y, hipStream_t st, View mask = View{}) {
    launch_conv(x, N, H, W, w, Cin, b, relu, Cout, up, y, mask, st);
    HIPCHK(hipGetLastError());
    return DSN_OK;
}

int op_check(const void *a, const void *b, int N, int H, int W, int Cin, int Cout, bool up) {
    int r;
    // the kernels read both operands with 16-byte vector loads
    if ((r = check_ptr(a, "first operand")) || (r = check_ptr(b, "second operand"))) return r;
    if (N < 1 || H < 1 || W < 1) return fail(DSN_EINVAL, "bad N, H, W");
    if (up && (H % 2 || W % 2)) return fail(DSN_EINVAL, "up needs even H and W");
    if (Cin % 32 || Cout % 32 || Cin < 32 || Cout < 32 || Cin > 1024 || Cout > 1024)
        return fail(DSN_EINVAL, "channel counts must be multiples of 32 in [32, 1024]");
    return DSN_OK;
}

}  // namespace

extern "C" int dsn_op_conv3x3(const void *d_x, int N, int H, int W, int Cin, int up, const void *d_w,
                              const float *d_b, int Cout, int relu, void *d_y, void *stream) {
    int r;
    if ((r = op_check(d_x, d_w, N, H, W, Cin, Cout, up)) || (r = check_ptr(d_y, "d_y"))) return r;
    return op_conv(View{(__bf16 *)d_x, Cin, Cin}, N, H, W, Cin, up, (const __bf16 *)d_w, d_b, Cout, relu ? 1 : 0,
                   View{(__bf16 *)d_y, Cout, Cout}, static_cast<hipStream_t>(stream));
}

extern "C" int dsn_op_conv3x3_dgrad(const void *d_dy, int N, int H, int W, int Cout, const void *d_w, int Cin,
                                    const void *d_mask, void *d_dx, void *stream) {
    int r;
    if ((r = op_check(d_dy, d_w, N, H, W, Cin, Cout, false)) || (r = check_ptr(d_dx, "d_dx"))) return r;
    if (d_mask && (r = check_ptr(d_mask, "d_mask"))) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    __bf16 *wt = nullptr;
    const long long n = (long long)Cout * 9 * Cin;
    HIPCHK(hipMalloc(&wt, n * sizeof(__bf16)));
    k_flip_transpose<<<grid1(n), 256, 0, st>>>((const __bf16 *)d_w, Cout, Cin, wt);
    hipError_t e = hipGetLastError();
    r = e == hipSuccess ? op_conv(View{(__bf16 *)d_dy, Cout, Cout}, N, H, W, Cout, false, wt, nullptr, Cin, 0,
                                  View{(__bf16 *)d_dx, Cin, Cin}, st, View{(__bf16 *)d_mask, Cin, Cin})
                        : fail(DSN_EDEVICE, "k_flip_transpose: %s", hipGetErrorString(e));
    (void)hipStreamSynchronize(st);
    (void)hipFree(wt);
    return r;
}

extern "C" int dsn_op_conv3x3_wgrad(const void *d_dz, const void *d_x, int N, int H, int W, int Cin, int up,
                                    int Cout, float *d_dw, float *d_db, void *stream) {
    int r;
    if ((r = op_check(d_dz, d_x, N, H, W, Cin, Cout, up)) || (r = check_ptr(d_dw, "d_dw")) ||
        (r = check_ptr(d_db, "d_db")))
        return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    long long tps = 0;
    const long long cap = wgrad_part_floats(wgrad_tile_splits(N, H, W, Cin, Cout, &tps), Cin, Cout);
    float *part = nullptr;
    HIPCHK(hipMalloc(&part, (size_t)cap * sizeof(float)));
    View dz{(__bf16 *)d_dz, Cout, Cout}, x{(__bf16 *)d_x, Cin, Cin};
    hipError_t e = launch_wgrad_tile(dz, x, N, H, W, Cin, Cout, up != 0, part, cap, d_dw, d_db, st);
    (void)hipStreamSynchronize(st);
    (void)hipFree(part);
    if (e != hipSuccess) return fail(DSN_EDEVICE, "weight gradient: %s", hipGetErrorString(e));
    return DSN_OK;
}

namespace {

bool c_ok_first(int C) { return C >= 8 && C <= 64 && C % 8 == 0 && 256 % C == 0; }

}  // namespace

extern "C" int dsn_op_conv_first(const float *d_x, int N, int H, int W, const void *d_w, const float *d_b, int Cout,
                                 void *d_y, void *stream) {
    int r;
    if ((r = check_ptr(d_x, "d_x")) || (r = check_ptr(d_w, "d_w")) || (r = check_ptr(d_b, "d_b")) ||
        (r = check_ptr(d_y, "d_y")))
        return r;
    if (N < 1 || H < 1 || W < 1) return fail(DSN_EINVAL, "bad N, H, W");
    if (Cout < 8 || Cout > 1024 || Cout % 8) return fail(DSN_EINVAL, "Cout must be a multiple of 8 in [8, 1024]");
    const long long npix = (long long)N * H * W;
    if (npix >= (1LL << 31)) return fail(DSN_EINVAL, "N H W must be below 2^31");
    k_conv_first<<<grid1(npix), 256, (size_t)Cout * 10 * sizeof(float), static_cast<hipStream_t>(stream)>>>(
        d_x, N, H, W, (const __bf16 *)d_w, d_b, View{(__bf16 *)d_y, Cout, Cout});
    HIPCHK(hipGetLastError());
    return DSN_OK;
}

extern "C" int dsn_op_wgrad_first(const void *d_dz, const float *d_x, int N, int H, int W, int C, float *d_dw,
                                  float *d_db, void *stream) {
    int r;
    if ((r = check_ptr(d_dz, "d_dz")) || (r = check_ptr(d_x, "d_x")) || (r = check_ptr(d_dw, "d_dw")) ||
        (r = check_ptr(d_db, "d_db")))
        return r;
    if (N < 1 || H < 1 || W < 1) return fail(DSN_EINVAL, "bad N, H, W");
    if (!c_ok_first(C)) return fail(DSN_EINVAL, "C must be 8, 16, 32 or 64");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const long long npix = (long long)N * H * W;
    const int S = first_layer_splits(npix, C, 1LL << 62);
    float *part = nullptr;
    HIPCHK(hipMalloc(&part, (size_t)S * C * 10 * sizeof(float)));
    hipError_t e = launch_wgrad_first(View{(__bf16 *)d_dz, C, C}, d_x, N, H, W, S, part, d_dw, d_db, st);
    (void)hipStreamSynchronize(st);
    (void)hipFree(part);
    if (e != hipSuccess) return fail(DSN_EDEVICE, "first-layer weight gradient: %s", hipGetErrorString(e));
    return DSN_OK;
}

extern "C" int dsn_op_head_bwd(const void *d_x, long long npix, int C, int B, const void *d_w, const void *d_wm,
                               const float *d_out, const float *d_out_m, const float *d_t, const float *d_t_m,
                               int relu_mask, void *d_dx, double *d_loss, float *d_gw, void *stream) {
    int r;
    if ((r = check_ptr(d_x, "d_x")) || (r = check_ptr(d_w, "d_w")) || (r = check_ptr(d_out, "d_out")) ||
        (r = check_ptr(d_t, "d_t")) || (r = check_ptr(d_dx, "d_dx")) || (r = check_ptr(d_loss, "d_loss")) ||
        (r = check_ptr(d_gw, "d_gw")))
        return r;
    const int nm = (d_wm != nullptr) + (d_out_m != nullptr) + (d_t_m != nullptr);
    if (nm != 0 && nm != 3) return fail(DSN_EINVAL, "d_wm, d_out_m and d_t_m are given together or not at all");
    if (nm == 3 && ((r = check_ptr(d_wm, "d_wm")) || (r = check_ptr(d_out_m, "d_out_m")) ||
                    (r = check_ptr(d_t_m, "d_t_m"))))
        return r;
    if (npix < 1 || B < 1) return fail(DSN_EINVAL, "npix and B must be >= 1");
    if (C < 8 || C > 64 || C % 8) return fail(DSN_EINVAL, "C must be a multiple of 8 in [8, 64]");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const long long nblk = grid1(npix);
    double *lpart = nullptr;
    float *hpart = nullptr;
    HIPCHK(hipMalloc(&lpart, (size_t)nblk * 2 * sizeof(double)));
    hipError_t e = hipMalloc(&hpart, (size_t)nblk * 2 * (C + 1) * sizeof(float));
    if (e == hipSuccess)
        e = launch_head_bwd(View{(__bf16 *)d_x, C, C}, npix, B, (const __bf16 *)d_w, (const __bf16 *)d_wm, d_out,
                            d_out_m, d_t, d_t_m, View{(__bf16 *)d_dx, C, C}, relu_mask != 0, lpart, hpart, d_loss,
                            d_gw, st);
    (void)hipStreamSynchronize(st);
    (void)hipFree(lpart);
    if (hpart) (void)hipFree(hpart);
    if (e != hipSuccess) return fail(DSN_EDEVICE, "head backward: %s", hipGetErrorString(e));
    return DSN_OK;
}

extern "C" int dsn_op_maxpool2_bwd(const void *d_x, int N, int H, int W, int C, const void *d_dy, int relu_mask,
                                   void *d_dx, void *stream) {
    int r;
    if ((r = check_ptr(d_x, "d_x")) || (r = check_ptr(d_dy, "d_dy")) || (r = check_ptr(d_dx, "d_dx"))) return r;
    if (N < 1 || H < 2 || W < 2 || H % 2 || W % 2) return fail(DSN_EINVAL, "need N >= 1 and even H, W >= 2");
    if (C < 8 || C % 8 || C > 2048) return fail(DSN_EINVAL, "C must be a multiple of 8 in [8, 2048]");
    const long long n = (long long)N * (H / 2) * (W / 2) * (C / 8);
    const View x{(__bf16 *)d_x, C, C}, dy{(__bf16 *)d_dy, C, C}, dx{(__bf16 *)d_dx, C, C};
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (relu_mask) k_maxpool_bwd<true><<<grid1(n), 256, 0, st>>>(x, N, H, W, dy, dx);
    else k_maxpool_bwd<false><<<grid1(n), 256, 0, st>>>(x, N, H, W, dy, dx);
    HIPCHK(hipGetLastError());
    return DSN_OK;
}

extern "C" int dsn_op_upsample2_bwd(const void *d_dy, int N, int H, int W, int C, const void *d_mask, void *d_dx,
                                    void *stream) {
    int r;
    if ((r = check_ptr(d_dy, "d_dy")) || (r = check_ptr(d_dx, "d_dx"))) return r;
    if (d_mask && (r = check_ptr(d_mask, "d_mask"))) return r;
    if (N < 1 || H < 2 || W < 2 || H % 2 || W % 2) return fail(DSN_EINVAL, "need N >= 1 and even H, W >= 2");
    if (C < 8 || C % 8 || C > 2048) return fail(DSN_EINVAL, "C must be a multiple of 8 in [8, 2048]");
    const long long n = (long long)N * (H / 2) * (W / 2) * (C / 8);
    k_upsample_bwd<<<grid1(n), 256, 0, static_cast<hipStream_t>(stream)>>>(View{(__bf16 *)d_dy, C, C}, N, H, W,
                                                                            View{(__bf16 *)d_dx, C, C},
                                                                            View{(__bf16 *)d_mask, C, C});
    HIPCHK(hipGetLastError());
    return DSN_OK;
}

extern "C" int dsn_op_relu_bwd(void *d_d, const void *d_y, long long npix, int C, void *stream) {
    int r;
    if ((r = check_ptr(d_d, "d_d")) || (r = check_ptr(d_y, "d_y"))) return r;
    if (npix < 1) return fail(DSN_EINVAL, "npix must be >= 1");
    if (C < 8 || C % 8 || C > 2048) return fail(DSN_EINVAL, "C must be a multiple of 8 in [8, 2048]");
    k_relu_bwd<<<grid1(npix * (C / 8)), 256, 0, static_cast<hipStream_t>(stream)>>>(
        View{(__bf16 *)d_d, C, C}, View{(__bf16 *)d_y, C, C}, npix);
    HIPCHK(hipGetLastError());
    return DSN_OK;
}
