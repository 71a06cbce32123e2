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

__device__ __forceinline__ void split(float x, __bf16 &hi, __bf16 &lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

__device__ __forceinline__ bf8 bf8_zero() {
    bf8 z;
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.f;
    return z;
}

// k-group g (8 wide) of the concatenated inner dimension: segment p = g / (KP/8)
// and first row r0.  A-side reads hi for p = 0, 1 and lo for p = 2; B-side
// reads hi for p = 0, 2 and lo for p = 1; p >= 3 is zero padding.
template <int KP>
__device__ __forceinline__ void kgroup(int g, int &p, int &r0) {
    constexpr int KP8 = KP / 8;
    p = g / KP8;
    r0 = (g - p * KP8) * 8;
}

// --------------------------------------------------------------------------
// Split and transpose the window-row operands:
//   Y  [set][j][KP][Np] fp32   ->   Yhl [set][j][Np][2][KP] bf16 (hi row, lo row)
// Block: 64 columns x 4 groups of 8 rows.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_split_rows(const float *__restrict__ Y, int KP, int Np, int nj, int set_lo,
                                                    __bf16 *__restrict__ Yhl) {
    const int j = blockIdx.y, s = set_lo + blockIdx.z;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int rg = threadIdx.x >> 6;
    const float *src = Y + ((size_t)(s * nj + j) * KP) * Np + x;
    __bf16 *dst = Yhl + (((size_t)(s * nj + j) * Np) + x) * 2 * KP;
    for (int g = rg; g < KP / 8; g += 4) {
        bf8 h, l;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            __bf16 a, b;
            split(src[(size_t)(8 * g + e) * Np], a, b);
            h[e] = a;
            l[e] = b;
        }
        *reinterpret_cast<bf8 *>(dst + 8 * g) = h;
        *reinterpret_cast<bf8 *>(dst + KP + 8 * g) = l;
    }
}

// XCD-aware tile order: hardware places consecutive blocks round-robin on the
// 8 XCDs; remap so that the blocks an XCD receives cover all row tiles of the
// same column tiles, which then share that XCD's L2 for their Y_j tiles.
__device__ __forceinline__ void xcd_tile(int b, int nblk, int NY, int NX, int &ty, int &tx, int &ts) {
    int L = b;
    if ((nblk & 7) == 0) L = (b & 7) * (nblk >> 3) + (b >> 3);
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
__global__ __launch_bounds__(256, KP > 40 ? 1 : 2) void k_image_b3(const __bf16 *__restrict__ tlhl, const __bf16 *__restrict__ Yhl,
                                                      int nj, int N, int Np, int set_lo, int nsets,
                                                      float *__restrict__ out) {
    constexpr int KC = (3 * KP + 31) / 32 * 32;
    constexpr int NS = KC / 32;
    constexpr int RW = 2 * KP + 8;                 // LDS row (one column x), bf16
    constexpr int NV = (64 * 2 * KP / 8 + 255) / 256;
    __shared__ __attribute__((aligned(16))) __bf16 Ys[2][64][RW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int NX = Np / 64, NY = Np / 128;
    int ty, tx, ts;
    xcd_tile(blockIdx.x, gridDim.x, NY, NX, ty, tx, ts);
    const int s = set_lo + ts;
    const int x0 = tx * 64;
    const int yw = ty * 128 + wave * 32;

    bf8 b1[2][NS], b2[2][NS];
#pragma unroll
    for (int yb = 0; yb < 2; ++yb)
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            int p, r0;
            kgroup<KP>(4 * st + lq, p, r0);
            if (p >= 3) {
                b1[yb][st] = bf8_zero();
                b2[yb][st] = bf8_zero();
            } else {
                const int hl = (p == 1);
                const size_t y = yw + 16 * yb + l16;
                b1[yb][st] = *reinterpret_cast<const bf8 *>(tlhl + ((0 * (size_t)Np + y) * 2 + hl) * KP + r0);
                b2[yb][st] = *reinterpret_cast<const bf8 *>(tlhl + ((1 * (size_t)Np + y) * 2 + hl) * KP + r0);
            }
        }
    f4 accI[4][2];
#pragma unroll
    for (int xb = 0; xb < 4; ++xb)
#pragma unroll
        for (int yb = 0; yb < 2; ++yb) accI[xb][yb] = f4{0.f, 0.f, 0.f, 0.f};

    u4 pre[NV];
#define B3_FETCH(jj)                                                                                     \
    do {                                                                                                 \
        const __bf16 *src_ = Yhl + (((size_t)(s * nj + (jj)) * Np) + x0) * 2 * KP;                     \
        _Pragma("unroll") for (int v = 0; v < NV; ++v) {                                                 \
            const int e = threadIdx.x + 256 * v;                                                         \
            if (e < 64 * 2 * KP / 8) pre[v] = *reinterpret_cast<const u4 *>(src_ + (size_t)e * 8);       \
        }                                                                                                \
    } while (0)
#define B3_STASH(bb)                                                                                     \
    do {                                                                                                 \
        _Pragma("unroll") for (int v = 0; v < NV; ++v) {                                                 \
            const int e = threadIdx.x + 256 * v;                                                         \
            if (e < 64 * 2 * KP / 8) {                                                                   \
                const int xx = e / (2 * KP / 8), q = e % (2 * KP / 8);                                   \
                *reinterpret_cast<u4 *>(&Ys[(bb)][xx][q * 8]) = pre[v];                                  \
            }                                                                                            \
        }                                                                                                \
    } while (0)
    B3_FETCH(0);
    B3_STASH(0);
    __syncthreads();
    for (int j = 0; j < nj; ++j) {
        const int buf = j & 1;
        if (j + 1 < nj) B3_FETCH(j + 1);
        // two halves of the 64 columns keep only half the field accumulators live
#pragma unroll
        for (int xh = 0; xh < 2; ++xh) {
            f4 er[2][2], ei[2][2];
#pragma unroll
            for (int xl = 0; xl < 2; ++xl)
#pragma unroll
                for (int yb = 0; yb < 2; ++yb) {
                    er[xl][yb] = f4{0.f, 0.f, 0.f, 0.f};
                    ei[xl][yb] = f4{0.f, 0.f, 0.f, 0.f};
                }
#pragma unroll
            for (int st = 0; st < NS; ++st) {
                int p, r0;
                kgroup<KP>(4 * st + lq, p, r0);
                const int off = (p == 2 ? KP : 0) + r0;
#pragma unroll
                for (int xl = 0; xl < 2; ++xl) {
                    const int xb = 2 * xh + xl;
                    bf8 a = (p >= 3) ? bf8_zero() : *reinterpret_cast<const bf8 *>(&Ys[buf][16 * xb + l16][off]);
#pragma unroll
                    for (int yb = 0; yb < 2; ++yb) {
                        er[xl][yb] = mfma_b(a, b1[yb][st], er[xl][yb]);
                        ei[xl][yb] = mfma_b(a, b2[yb][st], ei[xl][yb]);
                    }
                }
            }
#pragma unroll
            for (int xl = 0; xl < 2; ++xl)
#pragma unroll
                for (int yb = 0; yb < 2; ++yb)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        accI[2 * xh + xl][yb][i] = fmaf(er[xl][yb][i], er[xl][yb][i],
                                                        fmaf(ei[xl][yb][i], ei[xl][yb][i], accI[2 * xh + xl][yb][i]));
        }
        if (j + 1 < nj) B3_STASH(buf ^ 1);
        __syncthreads();
    }
#undef B3_FETCH
#undef B3_STASH
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
// Adjoint, split-BF16, fields recomputed.  Block = (32-row tile, 4 kernels,
// set); per 32-column chunk, each wave:
//   (a) E^T = Y_j^T L^T                split-BF16 GEMM, K = 3 KP padded
//   (b) X = G . E                       FP32, G tile from LDS
//   (c) Z += X B3                       X split in registers; its 8 values per
//       lane (columns 4(l/16)+i of both 16-column blocks) form one k-group,
//       and the B3 rows are read in the same order
// then the FP32 window contraction and W partial of the plain path.
// --------------------------------------------------------------------------
template <int KP, int FB, int MIX>
__global__ __launch_bounds__(256, 2) void k_adjoint_b3(const __bf16 *__restrict__ tlhl,
                                                        const __bf16 *__restrict__ tbhl,
                                                        const float *__restrict__ ta4,
                                                        const __bf16 *__restrict__ Yhl, const float *__restrict__ G,
                                                        size_t g_set_stride, const float2 *__restrict__ coef, int K,
                                                        int P, int N, int Np, int AP, int set_lo,
                                                        float *__restrict__ Wpart) {
    constexpr int KC = (3 * KP + 31) / 32 * 32;
    constexpr int NS = KC / 32;
    constexpr int RW = 2 * KP + 8;
    constexpr int NZ = 32 * FB + 16 * MIX, NB = NZ / 16;
    constexpr int BW = 32 + 8;                     // B3 chunk row (bf16)
    constexpr int NBV = (2 * 2 * NZ * 4 + 255) / 256;
    __shared__ __attribute__((aligned(16))) __bf16 Ls[2][32][RW];
    __shared__ __attribute__((aligned(16))) __bf16 Bt[2][2][NZ][BW];
    __shared__ __attribute__((aligned(16))) float Gs[32][36];
    __shared__ float2 Ws[ILT_MAX_P * ILT_MAX_P];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int ytile = blockIdx.x, kg = blockIdx.y, srel = blockIdx.z, s = set_lo + srel;
    const int y0 = ytile * 32;
    const int j = kg * 4 + wave;
    const bool jok = j < K;

    // L operands of the block's 32 rows (both parts, hi and lo)
    for (int e = threadIdx.x; e < 2 * 32 * (2 * KP / 8); e += 256) {
        const int part = e / (32 * (2 * KP / 8));
        const int rem = e % (32 * (2 * KP / 8));
        const int yy = rem / (2 * KP / 8), q = rem % (2 * KP / 8);
        *reinterpret_cast<u4 *>(&Ls[part][yy][q * 8]) =
            *reinterpret_cast<const u4 *>(tlhl + ((size_t)part * Np + y0 + yy) * 2 * KP + q * 8);
    }

    f4 accZ[2][NB];
#pragma unroll
    for (int yb = 0; yb < 2; ++yb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) accZ[yb][nb] = f4{0.f, 0.f, 0.f, 0.f};

    const __bf16 *Yj = Yhl + (size_t)(s * K + (jok ? j : 0)) * Np * 2 * KP;
    const float *Gsrc = G + (size_t)s * g_set_stride;
    const int nchunk = (N + 31) / 32;
    for (int c = 0; c < nchunk; ++c) {
        const int x0 = c * 32;
        __syncthreads();
#pragma unroll
        for (int v = 0; v < NBV; ++v) {
            const int e = threadIdx.x + 256 * v;
            if (e < 2 * 2 * NZ * 4) {
                const int row = e >> 2, q = e & 3;        // row = (part, hl, n)
                const int part = row / (2 * NZ), hl = (row / NZ) & 1, n = row % NZ;
                *reinterpret_cast<u4 *>(&Bt[part][hl][n][q * 8]) =
                    *reinterpret_cast<const u4 *>(tbhl + ((size_t)(part * 2 + hl) * NZ + n) * Np + x0 + q * 8);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int e = threadIdx.x + 256 * v;
            const int yy = e >> 5, xx = e & 31;
            const int gy = y0 + yy, gx = x0 + xx;
            Gs[yy][xx] = (gy < N && gx < N) ? Gsrc[(size_t)gy * N + gx] : 0.f;
        }
        __syncthreads();
        if (!jok) continue;
        // (a) fields of this chunk, E^T blocks (xb = 16-column block, yb = 16-row block)
        f4 er[2][2], ei[2][2];
#pragma unroll
        for (int xb = 0; xb < 2; ++xb)
#pragma unroll
            for (int yb = 0; yb < 2; ++yb) {
                er[xb][yb] = f4{0.f, 0.f, 0.f, 0.f};
                ei[xb][yb] = f4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            int p, r0;
            kgroup<KP>(4 * st + lq, p, r0);
            // zero padding of the inner dimension (p >= 3) goes in as zero
            // operands: the matrix instructions must run with every lane active
            const bool pad = p >= 3;
            const int offA = pad ? 0 : (p == 2 ? KP : 0) + r0;
            const int offB = pad ? 0 : (p == 1 ? KP : 0) + r0;
            bf8 bb1[2], bb2[2];
#pragma unroll
            for (int yb = 0; yb < 2; ++yb) {
                bb1[yb] = pad ? bf8_zero() : *reinterpret_cast<const bf8 *>(&Ls[0][16 * yb + l16][offB]);
                bb2[yb] = pad ? bf8_zero() : *reinterpret_cast<const bf8 *>(&Ls[1][16 * yb + l16][offB]);
            }
#pragma unroll
            for (int xb = 0; xb < 2; ++xb) {
                const bf8 a = pad ? bf8_zero()
                                  : *reinterpret_cast<const bf8 *>(Yj + (size_t)(x0 + 16 * xb + l16) * 2 * KP + offA);
#pragma unroll
                for (int yb = 0; yb < 2; ++yb) {
                    er[xb][yb] = mfma_b(a, bb1[yb], er[xb][yb]);
                    ei[xb][yb] = mfma_b(a, bb2[yb], ei[xb][yb]);
                }
            }
        }
        // (b) X = G . E; register i of (xb, yb) is column 16 xb + 4 lq + i, row 16 yb + l16
#pragma unroll
        for (int xb = 0; xb < 2; ++xb)
#pragma unroll
            for (int yb = 0; yb < 2; ++yb) {
                const f4 g4 = *reinterpret_cast<const f4 *>(&Gs[16 * yb + l16][16 * xb + 4 * lq]);
                er[xb][yb] *= g4;
                ei[xb][yb] *= g4;
            }
        // (c) Z[y][n] += sum_x X[y][x] B3[x][n]: one k-group per part = the
        // lane's 8 columns {4lq+i} of block 0 then block 1
#pragma unroll
        for (int part = 0; part < 2; ++part) {
            bf8 xh[2], xl[2];
#pragma unroll
            for (int yb = 0; yb < 2; ++yb)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float v = part ? ei[e >> 2][yb][e & 3] : er[e >> 2][yb][e & 3];
                    __bf16 h, l;
                    split(v, h, l);
                    xh[yb][e] = h;
                    xl[yb][e] = l;
                }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int n = 16 * nb + l16;
                bf8 bh, bl;
                {
                    const uint2 h0 = *reinterpret_cast<const uint2 *>(&Bt[part][0][n][4 * lq]);
                    const uint2 h1 = *reinterpret_cast<const uint2 *>(&Bt[part][0][n][16 + 4 * lq]);
                    const uint2 l0 = *reinterpret_cast<const uint2 *>(&Bt[part][1][n][4 * lq]);
                    const uint2 l1 = *reinterpret_cast<const uint2 *>(&Bt[part][1][n][16 + 4 * lq]);
                    u4 th = {h0.x, h0.y, h1.x, h1.y}, tl = {l0.x, l0.y, l1.x, l1.y};
                    bh = __builtin_bit_cast(bf8, th);
                    bl = __builtin_bit_cast(bf8, tl);
                }
#pragma unroll
                for (int yb = 0; yb < 2; ++yb) {
                    accZ[yb][nb] = mfma_b(xh[yb], bh, accZ[yb][nb]);
                    accZ[yb][nb] = mfma_b(xh[yb], bl, accZ[yb][nb]);
                    accZ[yb][nb] = mfma_b(xl[yb], bh, accZ[yb][nb]);
                }
            }
        }
    }
    float *dst = Wpart + ((size_t)(srel * gridDim.x + ytile) * gridDim.y + kg) * P * P * 2;
    ilt_dev::adjoint_tail<FB, MIX>(accZ, jok, j, s, K, P, Np, AP, y0, ta4, coef, Ws, dst);
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_split_rows(ilt_ctx *c, int set_lo, int set_hi) {
    dim3 grid(c->Np / 64, c->K, set_hi - set_lo);
    k_split_rows<<<grid, 256, 0, c->stream>>>(c->Y, c->KP, c->Np, c->K, set_lo, c->Yhl);
    return hipGetLastError();
}

hipError_t launch_image_b3(ilt_ctx *c, int set_lo, int set_hi, float *out) {
    const int nblk = (c->Np / 64) * (c->Np / 128) * (set_hi - set_lo);
    switch (c->KP) {
#define IMGB(KP_) case KP_: k_image_b3<KP_><<<nblk, 256, 0, c->stream>>>(c->tlhl, c->Yhl, c->K, c->N, c->Np, set_lo, set_hi - set_lo, out); break;
        IMGB(8) IMGB(24) IMGB(40) IMGB(72)
#undef IMGB
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_b3(ilt_ctx *c, const float *G, size_t g_set_stride, int set_lo, int set_hi) {
    dim3 grid((c->N + 31) / 32, (c->K + 3) / 4, set_hi - set_lo);
#define ADJB(KP_, FB_, MIX_)                                                                                  \
    k_adjoint_b3<KP_, FB_, MIX_><<<grid, 256, 0, c->stream>>>(c->tlhl, c->tbhl, c->ta4, c->Yhl, G, g_set_stride, \
                                                              c->coef, c->K, c->P, c->N, c->Np, c->AP, set_lo,  \
                                                              c->Wpart)
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
