// Split-BF16 ("BF16x3") forms of the SOCS image and adjoint GEMMs.
//
// Every FP32 operand x is split as x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (round to nearest even); a product is approximated by
// hi*hi + hi*lo + lo*hi with FP32 accumulation (the lo*lo term, ~2^-16
// relative, is dropped).  The three products are laid end to end along the
// inner dimension, so one GEMM with K = 3 KP (padded to a multiple of 32)
// computes them on the 16x16x32 BF16 matrix cores:
//   A-side segments: [hi | hi | lo],   B-side segments: [hi | lo | hi].
// KP is a multiple of 8, so each lane's 8-element k-group lies in one segment.
//
// 16x16x32 BF16 operand convention: lane l supplies A[m = l%16][k = 8(l/16)+e]
// and B[k = 8(l/16)+e][n = l%16], e = 0..7; accumulator register i of lane l
// is C[m = 4(l/16) + i][n = l%16] (as for the FP32 16x16x4 form).
//
// The operations are those of k_litho.hip (Sec. II-B forward imaging,
// Sec. III-A adjoint); only the arithmetic of the two dense contractions
// changes.  The adjoint recomputes the fields (cheap at BF16 rate) instead of
// streaming them from HBM.
#include "ilt_internal.h"
#include "ilt_device.h"

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma_b(bf8 a, bf8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Two products a b split at once: the packed hi pair is rounded once, the
// FP32 values of its halves are read back by shifts of the packed word, and
// lo = bf16(a b - hi) takes the residual of the exact product (one FMA).
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split2(float a0, float b0, float a1, float b1, unsigned &hp, unsigned &lp) {
    hp = __builtin_bit_cast(unsigned, __builtin_convertvector(f2v{a0 * b0, a1 * b1}, bf2));
    const float h0 = __builtin_bit_cast(float, hp << 16), h1 = __builtin_bit_cast(float, hp & 0xFFFF0000u);
    lp = __builtin_bit_cast(unsigned, __builtin_convertvector(f2v{fmaf(a0, b0, -h0), fmaf(a1, b1, -h1)}, bf2));
}

__device__ __forceinline__ bf8 bf8_zero() {
    bf8 z;
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.f;
    return z;
}

// Order of the 8-wide k-groups of the concatenated inner dimension.  Step st
// of a contraction (32 wide) gives lane l the group of segment p, first row
// r0; B-side operands live in registers, and slot() says which register
// holds the B data of step st.  The first NF steps take hi rows of segment 0
// and the next NF steps the same rows of segment 2, whose B-side data (hi) is
// identical, so they share registers: NS - NF registers per operand instead
// of NS.  The remaining groups (tails of segments 0 and 2, all of segment 1,
// then zero padding, p = 3) fill the last steps in that order.
// A-side reads hi for p = 0, 1 and lo for p = 2; B-side reads hi for p = 0, 2
// and lo for p = 1.
template <int KP>
struct kmap {
    static constexpr int KP8 = KP / 8;
    static constexpr int NF = KP8 / 4;
    static constexpr int NS = (3 * KP8 + 3) / 4;
    static constexpr int NSL = NS - NF;
    static constexpr int R = KP8 - 4 * NF;
    __device__ static constexpr int slot(int st) { return st < NF ? st : st - NF; }
    // step whose groups are loaded into register slot sl
    __device__ static constexpr int load_step(int sl) { return sl < NF ? sl : sl + NF; }
    __device__ static __forceinline__ void group(int st, int lq, int &p, int &r0) {
        int rb;
        if (st < NF) {
            p = 0;
            rb = 4 * st + lq;
        } else if (st < 2 * NF) {
            p = 2;
            rb = 4 * (st - NF) + lq;
        } else {
            const int idx = 4 * (st - 2 * NF) + lq;
            if (idx < R) {
                p = 0;
                rb = 4 * NF + idx;
            } else if (idx < 2 * R) {
                p = 2;
                rb = 4 * NF + idx - R;
            } else if (idx < 2 * R + KP8) {
                p = 1;
                rb = idx - 2 * R;
            } else {
                p = 3;
                rb = 0;
            }
        }
        r0 = 8 * rb;
    }
};

// B-side (L) operands of one wave's 16-row block y..y+15 for both parts.
template <int KP>
__device__ __forceinline__ void load_l_operands(const __bf16 *__restrict__ tlhl, int Np, size_t y, int lq,
                                                bf8 (&b1)[kmap<KP>::NSL], bf8 (&b2)[kmap<KP>::NSL]) {
#pragma unroll
    for (int sl = 0; sl < kmap<KP>::NSL; ++sl) {
        int p, r0;
        kmap<KP>::group(kmap<KP>::load_step(sl), lq, p, r0);
        if (p >= 3) {
            b1[sl] = bf8_zero();
            b2[sl] = bf8_zero();
        } else {
            const int hl = (p == 1);
            b1[sl] = *reinterpret_cast<const bf8 *>(tlhl + ((0 * (size_t)Np + y) * 2 + hl) * KP + r0);
            b2[sl] = *reinterpret_cast<const bf8 *>(tlhl + ((1 * (size_t)Np + y) * 2 + hl) * KP + r0);
        }
    }
}

// XCD-aware tile order: hardware places consecutive blocks round-robin on the
// 8 XCDs; remap so that the blocks an XCD receives cover all row tiles of the
// same column tiles, which then share that XCD's L2 for their Y_j tiles.
__device__ __forceinline__ void xcd_tile(int b, int nblk, int NY, int NX, int remap, int &ty, int &tx, int &ts) {
    int L = b;
    if (remap && (nblk & 7) == 0) L = (b & 7) * (nblk >> 3) + (b >> 3);
    ty = L % NY;
    const int rest = L / NY;
    tx = rest % NX;
    ts = rest / NX;
}

// --------------------------------------------------------------------------
// Image, split-BF16: out[set] = sum_j |A^H Y_j|^2 over 128 x 64 block tiles;
// wave tile 32 rows x 64 columns; E^T orientation (m = x, n = y, k = r).
// The L-side operands (B, per wave) stay in registers; each Y_j tile
// (64 columns x [hi|lo] rows, 16-byte k-groups) is staged in LDS,
// double-buffered, shared by the four waves.
// --------------------------------------------------------------------------
template <int KP>
__global__ __launch_bounds__(256, 2) void k_image_b3(const __bf16 *__restrict__ tlhl, const __bf16 *__restrict__ Yhl,
                                                      int nj, int N, int Np, int set_lo, int nsets, int remap,
                                                      float *__restrict__ out) {
    constexpr int NS = kmap<KP>::NS, NSL = kmap<KP>::NSL;
    constexpr int RW = 2 * KP + 8;                 // LDS row (one column x), bf16
    __shared__ __attribute__((aligned(16))) __bf16 Ys[2][64][RW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int NX = Np / 64, NY = Np / 128;
    int ty, tx, ts;
    xcd_tile(blockIdx.x, gridDim.x, NY, NX, remap, ty, tx, ts);
    const int s = set_lo + ts;
    const int x0 = tx * 64;
    const int yw = ty * 128 + wave * 32;

    bf8 b1[2][NSL], b2[2][NSL];
#pragma unroll
    for (int yb = 0; yb < 2; ++yb) load_l_operands<KP>(tlhl, Np, (size_t)yw + 16 * yb + l16, lq, b1[yb], b2[yb]);
    f4 accI[4][2];
#pragma unroll
    for (int xb = 0; xb < 4; ++xb)
#pragma unroll
        for (int yb = 0; yb < 2; ++yb) accI[xb][yb] = f4{0.f, 0.f, 0.f, 0.f};

    // Y_j tile: rows x0 .. x0 + 63 of [hi|lo] (2 KP / 8 units of 16 bytes,
    // one pad unit per LDS row), copied global -> LDS by the memory unit; the
    // copy of Y_{j+1} runs while Y_j is contracted.  Per-lane source offsets
    // are formed once (wave w copies the 64-unit groups w, w + 4, ...; a pad
    // unit copies its row's first unit, never read).
    constexpr int RWU = RW / 8, NYI = RWU, NYT = (NYI + 3) / 4;
    int yoff[NYT];
#pragma unroll
    for (int t = 0; t < NYT; ++t) {
        const int U = 64 * (wave + 4 * t) + lane;
        const int row = U / RWU, col = U - (U / RWU) * RWU;
        yoff[t] = (x0 + row) * 2 * KP + (col < RWU - 1 ? col : 0) * 8;
    }
    auto copy_y = [&](int jj, int bb) {
        const __bf16 *src = Yhl + (size_t)(s * nj + jj) * Np * 2 * KP;
#pragma unroll
        for (int t = 0; t < NYT; ++t)
            if (wave + 4 * t < NYI) ilt_dev::lds_dma16(src + yoff[t], &Ys[bb][0][0] + 512 * (wave + 4 * t));
    };
    copy_y(0, 0);
    ilt_dev::wait_copies();
    __syncthreads();
    for (int j = 0; j < nj; ++j) {
        const int buf = j & 1;
        if (j + 1 < nj) copy_y(j + 1, buf ^ 1);
        // two halves of the 64 columns keep only half the field accumulators
        // live; the Y operands of step t + 1 are read from LDS before the
        // products of step t issue (scheduling barriers keep that order)
        auto read_a = [&](int t, bf8 (&a)[2]) {
            const int xh = t / NS, st = t - (t / NS) * NS;
            int p, r0;
            kmap<KP>::group(st, lq, p, r0);
            const int off = (p == 2 ? KP : 0) + r0;
#pragma unroll
            for (int xl = 0; xl < 2; ++xl)
                a[xl] = (p >= 3) ? bf8_zero() : *reinterpret_cast<const bf8 *>(&Ys[buf][16 * (2 * xh + xl) + l16][off]);
        };
        f4 er[2][2], ei[2][2];
        bf8 an[2];
        read_a(0, an);
#pragma unroll
        for (int t = 0; t < 2 * NS; ++t) {
            const int xh = t / NS, st = t - (t / NS) * NS;
            if (st == 0) {
#pragma unroll
                for (int xl = 0; xl < 2; ++xl)
#pragma unroll
                    for (int yb = 0; yb < 2; ++yb) {
                        er[xl][yb] = f4{0.f, 0.f, 0.f, 0.f};
                        ei[xl][yb] = f4{0.f, 0.f, 0.f, 0.f};
                    }
            }
            const bf8 a[2] = {an[0], an[1]};
            if (t + 1 < 2 * NS) read_a(t + 1, an);
            __builtin_amdgcn_sched_barrier(0);
            const int sl = kmap<KP>::slot(st);
#pragma unroll
            for (int xl = 0; xl < 2; ++xl)
#pragma unroll
                for (int yb = 0; yb < 2; ++yb) {
                    er[xl][yb] = mfma_b(a[xl], b1[yb][sl], er[xl][yb]);
                    ei[xl][yb] = mfma_b(a[xl], b2[yb][sl], ei[xl][yb]);
                }
            __builtin_amdgcn_sched_barrier(0);
            if (st == NS - 1) {
#pragma unroll
                for (int xl = 0; xl < 2; ++xl)
#pragma unroll
                    for (int yb = 0; yb < 2; ++yb)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            accI[2 * xh + xl][yb][i] = fmaf(er[xl][yb][i], er[xl][yb][i],
                                                            fmaf(ei[xl][yb][i], ei[xl][yb][i], accI[2 * xh + xl][yb][i]));
            }
        }
        // this wave's copy of Y_{j+1} has landed, and every wave is done with
        // buffer buf before it is refilled
        ilt_dev::wait_copies();
        __syncthreads();
    }
    float *o = out + (size_t)ts * N * N;
#pragma unroll
    for (int xb = 0; xb < 4; ++xb)
#pragma unroll
        for (int yb = 0; yb < 2; ++yb) {
            const int y = yw + 16 * yb + l16;
            const int x = x0 + 16 * xb + 4 * lq;
            if (y < N) {
                if ((N % 4) == 0 && x + 3 < N) {
                    *reinterpret_cast<f4 *>(o + (size_t)y * N + x) = accI[xb][yb];
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (x + i < N) o[(size_t)y * N + x + i] = accI[xb][yb][i];
                }
            }
        }
}

// --------------------------------------------------------------------------
// Adjoint, split-BF16, fields recomputed.  Block = (128-row tile, range of
// 32-column chunks, kernel j, set); wave w owns rows 32w..32w+31 of the tile.
// Per chunk the four waves share, through LDS, the Y_j chunk (hi|lo rows),
// the B3 chunk (stored in matrix-core fragment order) and the G tile.  They
// are copied global -> LDS by the memory unit without register staging; Y_j
// and B3 are double-buffered so that chunk c+1 arrives while chunk c is
// contracted, the G tile is read into registers first and then refilled.
// Each wave:
//   (a) E^T = Y_j^T L^T                split-BF16 GEMM, K = 3 KP padded; the
//       L-side operands of the wave's rows stay in registers
//   (b) X = G . E                       FP32
//   (c) Z += X B3                       X split in registers; its 8 values per
//       lane (columns 4(l/16)+i of both 16-column blocks) form one k-group,
//       matching the fragment order of the B3 table
// real part first, then imaginary part.  Then the FP32 window contraction;
// the four waves' W contributions (same kernel j) are summed in a fixed
// order into the block's partial.
//
// The copies are issued from inline assembly, so the compiler neither
// counts them nor waits for them: every wave waits for its own copies
// (vmcnt 0) and then meets the others at a barrier before reading them.
// --------------------------------------------------------------------------
using ilt_dev::lds_dma16;
using ilt_dev::wait_copies;

// G[y][x..x+3] (x a multiple of 4), zero outside the N x N image, for N % 4 != 0
__device__ __forceinline__ f4 load_g4_any(const float *__restrict__ G, int N, int y, int x) {
    const bool ok = y < N && x < N;
    const int yc = ok ? y : 0, xc = ok ? x : 0;
    f4 v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int xi = xc + i < N ? xc + i : N - 1;
        v[i] = (ok && x + i < N) ? G[(size_t)yc * N + xi] : 0.f;
    }
    return v;
}

template <int KP, int FB, int MIX, bool A4>
__global__ __launch_bounds__(256, 2) void k_adjoint_b3(const __bf16 *__restrict__ tlhl,
                                                        const __bf16 *__restrict__ tbf,
                                                        const float *__restrict__ ta4,
                                                        const __bf16 *__restrict__ Yhl, const float *__restrict__ G,
                                                        size_t g_set_stride, const float2 *__restrict__ coef, int K,
                                                        int P, int N, int Np, int AP, int set_lo, int xsplit,
                                                        float *__restrict__ Wpart) {
    constexpr int NS = kmap<KP>::NS, NSL = kmap<KP>::NSL;
    constexpr int NZ = 32 * FB + 16 * MIX, NB = NZ / 16;
    constexpr int RWU = 2 * KP / 8 + 1;            // 16-byte units per LDS row of Y (one pad unit)
    constexpr int NYI = (32 * RWU + 63) / 64;      // 64-unit copies per Y chunk
    constexpr int NBI = 2 * NB * 2;                // 64-unit copies per B3 chunk
    constexpr int GRU = 9;                         // 16-byte units per LDS row of G (one pad unit)
    constexpr int NGI = 128 * GRU / 64;            // 64-unit copies per G tile
    __shared__ u4 Yc[2][NYI * 64];
    __shared__ u4 Bc[2][NBI * 64];
    // G tile during the chunk loop, the window accumulator W afterwards
    __shared__ u4 GWs[128 * GRU];
    static_assert(sizeof(GWs) >= ILT_MAX_P * ILT_MAX_P * sizeof(float2), "W fits the G tile");
    const float *Gs = reinterpret_cast<const float *>(GWs);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int ytile = blockIdx.x / xsplit, xs = blockIdx.x - ytile * xsplit;
    const int j = blockIdx.y, srel = blockIdx.z, s = set_lo + srel;
    const int yt0 = ytile * 128, y0 = yt0 + 32 * wave;
    const int nchunk = (N + 31) / 32;
    const int c_lo = xs * nchunk / xsplit, c_hi = (xs + 1) * nchunk / xsplit;

    bf8 b1[2][NSL], b2[2][NSL];
#pragma unroll
    for (int yb = 0; yb < 2; ++yb) load_l_operands<KP>(tlhl, Np, (size_t)y0 + 16 * yb + l16, lq, b1[yb], b2[yb]);

    f4 accZ[2][NB];
#pragma unroll
    for (int yb = 0; yb < 2; ++yb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) accZ[yb][nb] = f4{0.f, 0.f, 0.f, 0.f};

    const __bf16 *Yj = Yhl + (size_t)(s * K + j) * Np * 2 * KP;
    const float *Gsrc = G + (size_t)s * g_set_stride;
    // Y_j and B3 of chunk c_ -> buffer bb; pad units and rows past the chunk
    // copy a valid in-chunk unit (never read back)
    // The copies' per-lane source offsets within a chunk do not depend on
    // the chunk: they are formed once (wave w copies the 64-unit groups
    // w, w + 4, ...).
    constexpr int NYT = (NYI + 3) / 4, NGT = (NGI + 3) / 4;
    int yoff[NYT], goff[NGT];
#pragma unroll
    for (int t = 0; t < NYT; ++t) {
        const int U = 64 * (wave + 4 * t) + lane;
        int row = U / RWU, col = U - row * RWU;
        if (row > 31) row = 31;
        if (col >= RWU - 1) col = 0;
        yoff[t] = row * 2 * KP + col * 8;
    }
    auto g_unit = [&](int U, int x0_) {         // G element offset of unit U for chunk column x0_
        const int row = U / GRU, col = U - row * GRU;
        const int y = min(yt0 + row, N - 1);
        return y * N + min(x0_ + 4 * (col < GRU - 1 ? col : 0), N - 4);
    };
#pragma unroll
    for (int t = 0; t < NGT; ++t) goff[t] = g_unit(64 * (wave + 4 * t) + lane, 0);
    auto copy_yb = [&](int c_, int bb) {
        const __bf16 *src = Yj + (size_t)c_ * 32 * 2 * KP;
#pragma unroll
        for (int t = 0; t < NYT; ++t)
            if (wave + 4 * t < NYI) lds_dma16(src + yoff[t], &Yc[bb][64 * (wave + 4 * t)]);
        for (int i = wave; i < NBI; i += 4)
            lds_dma16(tbf + ((size_t)c_ * NBI * 64 + 64 * i + lane) * 8, &Bc[bb][64 * i]);
    };
    // G rows yt0.., columns 32 c_.. (clamped into the image; values outside it
    // are masked when read).  Only a chunk that reaches past the image needs
    // the clamp of the column.
    auto copy_g = [&](int c_) {
        const int x0_ = c_ * 32;
        const bool inside = x0_ + 32 <= N;
#pragma unroll
        for (int t = 0; t < NGT; ++t)
            if (wave + 4 * t < NGI) {
                const int U = 64 * (wave + 4 * t) + lane;
                lds_dma16(Gsrc + (inside ? goff[t] + x0_ : g_unit(U, x0_)), &GWs[64 * (wave + 4 * t)]);
            }
    };
    if (c_lo < c_hi) {
        copy_yb(c_lo, 0);
        if (A4) copy_g(c_lo);
    }
    wait_copies();
    __syncthreads();
    for (int c = c_lo, it = 0; c < c_hi; ++c, ++it) {
        const int bb = it & 1;
        const int x0 = c * 32;
        f4 gv[2][2];
#pragma unroll
        for (int xb = 0; xb < 2; ++xb)
#pragma unroll
            for (int yb = 0; yb < 2; ++yb) {
                const int yy = 32 * wave + 16 * yb + l16, xx = 16 * xb + 4 * lq;
                if constexpr (A4) {
                    const f4 v = *reinterpret_cast<const f4 *>(&Gs[yy * (4 * GRU) + xx]);
                    gv[xb][yb] = (yt0 + yy < N && x0 + xx < N) ? v : f4{0.f, 0.f, 0.f, 0.f};
                } else {
                    gv[xb][yb] = load_g4_any(Gsrc, N, yt0 + yy, x0 + xx);
                }
            }
        if (c + 1 < c_hi) {
            if (A4) {
                __syncthreads();   // every wave holds its G values before the tile is refilled
                copy_g(c + 1);
            }
            copy_yb(c + 1, bb ^ 1);
        }
        const u4 *Yb = Yc[bb];
        const u4 *Bb = Bc[bb];
#pragma unroll
        for (int part = 0; part < 2; ++part) {
            // (a) E^T for this part; register i of e[xb][yb] is column
            // 16 xb + 4 lq + i, row 16 yb + l16 of the wave's 32 x 32 block
            f4 e[2][2];
#pragma unroll
            for (int xb = 0; xb < 2; ++xb)
#pragma unroll
                for (int yb = 0; yb < 2; ++yb) e[xb][yb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < NS; ++st) {
                int p, r0;
                kmap<KP>::group(st, lq, p, r0);
                const int sl = kmap<KP>::slot(st);
                // zero padding of the inner dimension (p = 3) goes in as zero
                // operands: the matrix instructions must run with every lane active
                const bool pad = p >= 3;
                const int ua = pad ? 0 : ((p == 2 ? KP : 0) + r0) / 8;
#pragma unroll
                for (int xb = 0; xb < 2; ++xb) {
                    const bf8 a = pad ? bf8_zero() : __builtin_bit_cast(bf8, Yb[(16 * xb + l16) * RWU + ua]);
#pragma unroll
                    for (int yb = 0; yb < 2; ++yb)
                        e[xb][yb] = mfma_b(a, part ? b2[yb][sl] : b1[yb][sl], e[xb][yb]);
                }
            }
            // (b) X = G . E, split
            // (element 2 m + q of a row's 8 values: column block m / 2, register 2 (m % 2) + q)
            bf8 xh[2], xl[2];
#pragma unroll
            for (int yb = 0; yb < 2; ++yb) {
                unsigned hw[4], lw[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int xb = m >> 1, i = 2 * (m & 1);
                    split2(e[xb][yb][i], gv[xb][yb][i], e[xb][yb][i + 1], gv[xb][yb][i + 1], hw[m], lw[m]);
                }
                xh[yb] = __builtin_bit_cast(bf8, u4{hw[0], hw[1], hw[2], hw[3]});
                xl[yb] = __builtin_bit_cast(bf8, u4{lw[0], lw[1], lw[2], lw[3]});
            }
            // (c) Z[y][n] += sum_x X[y][x] B3[x][n]: every column block's B3
            // operands first, then the three split products pass by pass, so
            // that 2 NB independent accumulators separate dependent steps
            // (each accumulator still adds hi.hi, hi.lo, lo.hi in that order)
            bf8 bh[NB], bl[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                bh[nb] = __builtin_bit_cast(bf8, Bb[((part * NB + nb) * 2 + 0) * 64 + lane]);
                bl[nb] = __builtin_bit_cast(bf8, Bb[((part * NB + nb) * 2 + 1) * 64 + lane]);
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int yb = 0; yb < 2; ++yb) accZ[yb][nb] = mfma_b(xh[yb], bh[nb], accZ[yb][nb]);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int yb = 0; yb < 2; ++yb) accZ[yb][nb] = mfma_b(xh[yb], bl[nb], accZ[yb][nb]);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int yb = 0; yb < 2; ++yb) accZ[yb][nb] = mfma_b(xl[yb], bh[nb], accZ[yb][nb]);
        }
        // the next chunk's copies have landed (this wave's), and every wave is
        // done with buffer bb before it is refilled
        wait_copies();
        __syncthreads();
    }
    float *dst = Wpart + ((size_t)(srel * gridDim.x + blockIdx.x) * gridDim.y + j) * P * P * 2;
    ilt_dev::adjoint_tail<FB, MIX>(accZ, true, j, s, K, P, Np, AP, y0, ta4, coef,
                                   reinterpret_cast<float2 *>(GWs), dst);
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_image_b3(ilt_ctx *c, int set_lo, int set_hi, float *out) {
    const int nblk = (c->Np / 64) * (c->Np / 128) * (set_hi - set_lo);
    switch (c->KP) {
#define IMGB(KP_) case KP_: k_image_b3<KP_><<<nblk, 256, 0, c->stream>>>(c->tlhl, c->Yhl, c->K, c->N, c->Np, set_lo, set_hi - set_lo, c->xcd_remap, out); break;
        IMGB(8) IMGB(24) IMGB(40) IMGB(72)
#undef IMGB
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Column chunks are split over two blocks once there are enough of them, so
// that a 2048-pixel clip gives three full rounds of blocks on 256 CUs; the
// tuner may pick 1 to ILT_B3_MAX_XSPLIT instead.
static int adjoint_b3_xsplit(const ilt_ctx *c) {
    if (c->b3_xsplit > 0) return c->b3_xsplit;
    return (c->N + 31) / 32 >= 8 ? 2 : 1;
}

int adjoint_b3_max_parts(const ilt_ctx *c, int nsets) {
    return nsets * ((c->N + 127) / 128) * ILT_B3_MAX_XSPLIT * c->K;
}

int adjoint_b3_parts(const ilt_ctx *c, int nsets) {
    return nsets * ((c->N + 127) / 128) * adjoint_b3_xsplit(c) * c->K;
}

hipError_t launch_adjoint_b3(ilt_ctx *c, const float *G, size_t g_set_stride, int set_lo, int set_hi) {
    const int xsplit = adjoint_b3_xsplit(c);
    if ((size_t)adjoint_b3_parts(c, set_hi - set_lo) * c->P * c->P * 2 > (size_t)c->n_wpart) return hipErrorInvalidValue;
    dim3 grid((c->N + 127) / 128 * xsplit, c->K, set_hi - set_lo);
#define ADJB(KP_, FB_, MIX_)                                                                                   \
    do {                                                                                                       \
        if ((c->N & 3) == 0 && (reinterpret_cast<uintptr_t>(G) & 15) == 0)                                    \
            k_adjoint_b3<KP_, FB_, MIX_, true><<<grid, 256, 0, c->stream>>>(                                   \
                c->tlhl, c->tbhl, c->ta4, c->Yhl, G, g_set_stride, c->coef, c->K, c->P, c->N, c->Np, c->AP,     \
                set_lo, xsplit, c->Wpart);                                                                     \
        else                                                                                                   \
            k_adjoint_b3<KP_, FB_, MIX_, false><<<grid, 256, 0, c->stream>>>(                                  \
                c->tlhl, c->tbhl, c->ta4, c->Yhl, G, g_set_stride, c->coef, c->K, c->P, c->N, c->Np, c->AP,     \
                set_lo, xsplit, c->Wpart);                                                                     \
    } while (0)
    const int KPv = c->KP, FBv = c->FB, MIXv = c->MIX;
    if (KPv == 8 && FBv == 0 && MIXv == 1) ADJB(8, 0, 1);
    else if (KPv == 24 && FBv == 0 && MIXv == 1) ADJB(24, 0, 1);
    else if (KPv == 24 && FBv == 1 && MIXv == 0) ADJB(24, 1, 0);
    else if (KPv == 40 && FBv == 1 && MIXv == 0) ADJB(40, 1, 0);
    else if (KPv == 40 && FBv == 1 && MIXv == 1) ADJB(40, 1, 1);
    else if (KPv == 72 && FBv == 1 && MIXv == 1) ADJB(72, 1, 1);
    else if (KPv == 72 && FBv == 2 && MIXv == 0) ADJB(72, 2, 0);
    else if (KPv == 72 && FBv == 2 && MIXv == 1) ADJB(72, 2, 1);
    else return hipErrorInvalidValue;
#undef ADJB
    return hipGetLastError();
}
