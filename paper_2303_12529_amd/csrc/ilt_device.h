// Device helpers shared by the FP32 and split-BF16 adjoint kernels.
#pragma once
#include "ilt_internal.h"

namespace ilt_dev {

// --------------------------------------------------------------------------
// Global -> LDS copies issued from inline assembly: the compiler neither
// counts them nor waits for them, so every wave waits for its own copies
// (wait_copies) and then meets the others at a barrier before reading them.
// --------------------------------------------------------------------------
__device__ __forceinline__ unsigned lds_offset(const void *p) {
    return (unsigned)(size_t)(const __attribute__((address_space(3))) void *)p;
}

// global -> LDS copy of 16 bytes per lane: lane l's bytes land at
// lds + 16 l (lds wave-uniform); M0 is restored afterwards
__device__ __forceinline__ void lds_dma16(const void *g, const void *lds) {
    const unsigned base = __builtin_amdgcn_readfirstlane(lds_offset(lds));
    unsigned saved;
    asm volatile(
        "s_mov_b32 %0, m0\n\t"
        "s_mov_b32 m0, %2\n\t"
        "global_load_lds_dwordx4 %1, off\n\t"
        "s_mov_b32 m0, %0"
        : "=&s"(saved)
        : "v"(g), "s"(base)
        : "memory");
}

// wait for every outstanding memory operation of this wave, the copies
// included; as a compiler-visible wait it also retires the compiler's own
// pending loads, so that none of its waits land inside the chunk loop
__device__ __forceinline__ void wait_copies() { __builtin_amdgcn_s_waitcnt(0); }

// --------------------------------------------------------------------------
// Adjoint, shared tail: (d) V = A4 Z over each wave's 32 rows y0.., then
// W_part += c_j conj(H_j) . V, summed over the four waves in a fixed order.
// --------------------------------------------------------------------------
template <int FB, int MIX>
__device__ __forceinline__ void adjoint_tail(const f4 (&accZ)[2][2 * FB + MIX], bool jok, int j, int s, int K, int P,
                                             int Np, int AP, int y0, const float *__restrict__ ta4,
                                             const float2 *__restrict__ coef, float2 *Ws,
                                             float *__restrict__ dst) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int AB = AP / 16;
    for (int e = threadIdx.x; e < P * P; e += 256) Ws[e] = make_float2(0.f, 0.f);
    __syncthreads();
    const float2 *cj = coef + ((size_t)s * K + (jok ? j : 0)) * P * P;
    for (int ab = 0; ab < AB; ++ab) {
        // full column blocks: real in block bb, imaginary in block FB + bb
        f4 vr[FB + MIX], vi[FB + MIX];
#pragma unroll
        for (int bb = 0; bb < FB + MIX; ++bb) {
            vr[bb] = f4{0.f, 0.f, 0.f, 0.f};
            vi[bb] = f4{0.f, 0.f, 0.f, 0.f};
        }
        if (jok) {
#pragma unroll
            for (int yb = 0; yb < 2; ++yb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int y = y0 + 16 * yb + 4 * lq + i;
                    const float car = ta4[(size_t)y * AP + 16 * ab + l16];
                    const float cai = ta4[((size_t)Np + y) * AP + 16 * ab + l16];
#pragma unroll
                    for (int bb = 0; bb < FB; ++bb) {
                        vr[bb] = mfma4(car, accZ[yb][bb][i], vr[bb]);
                        vi[bb] = mfma4(cai, accZ[yb][bb][i], vi[bb]);
                    }
#pragma unroll
                    for (int bb = 0; bb < FB; ++bb) {
                        vr[bb] = mfma4(-cai, accZ[yb][bb + FB][i], vr[bb]);
                        vi[bb] = mfma4(car, accZ[yb][bb + FB][i], vi[bb]);
                    }
                    if (MIX) {
                        // shared block: vr <- Ar Z, vi <- Ai Z (combined across lanes below)
                        vr[FB] = mfma4(car, accZ[yb][2 * FB][i], vr[FB]);
                        vi[FB] = mfma4(cai, accZ[yb][2 * FB][i], vi[FB]);
                    }
                }
            if (MIX) {
                // lanes l16 < 8 hold real columns, l16 >= 8 the imaginary ones:
                // V_re = (Ar Z_re) - (Ai Z_im), V_im = (Ar Z_im) + (Ai Z_re)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float q1 = vr[FB][i], q2 = vi[FB][i];
                    const float q1o = __shfl_xor(q1, 8), q2o = __shfl_xor(q2, 8);
                    vr[FB][i] = q1 - q2o;
                    vi[FB][i] = q1o + q2;
                }
            }
        }
        for (int w = 0; w < 4; ++w) {
            if (wave == w && jok) {
#pragma unroll
                for (int bb = 0; bb < FB + MIX; ++bb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int a = 16 * ab + 4 * lq + i;
                        const int b = bb < FB ? 16 * bb + l16 : (l16 < 8 ? 16 * FB + l16 : P);
                        if (a < P && b < P) {
                            const float2 c = cj[a * P + b];
                            const float xr = vr[bb][i], xi = vi[bb][i];
                            float2 cur = Ws[a * P + b];
                            cur.x += c.x * xr - c.y * xi;
                            cur.y += c.x * xi + c.y * xr;
                            Ws[a * P + b] = cur;
                        }
                    }
            }
            __syncthreads();
        }
    }
    for (int e = threadIdx.x; e < P * P; e += 256) {
        dst[2 * e] = Ws[e].x;
        dst[2 * e + 1] = Ws[e].y;
    }
}

// (c) for one 16-column block xb of a 32-column chunk: Z += (G . E) B3.
// The B3 operands of step i + 1 are read from LDS before the products of
// step i are issued (scheduling barriers keep that order), so each step's
// 4 NB products cover the next step's LDS latency.
template <int NB>
__device__ __forceinline__ void adjoint_rows(f4 (&accZ)[2][NB], const f4 (&er)[2], const f4 (&ei)[2],
                                             const float *Bre, const float *Bim, int ldb, int xb, int lq,
                                             int l16) {
    float br[2][NB], bi[2][NB];
    auto fetch = [&](int i, float (&r)[NB], float (&m)[NB]) {
        const int xr = 16 * xb + 4 * lq + i;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            r[nb] = Bre[xr * ldb + 16 * nb + l16];
            m[nb] = Bim[xr * ldb + 16 * nb + l16];
        }
    };
    fetch(0, br[0], bi[0]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i + 1 < 4) fetch(i + 1, br[(i + 1) & 1], bi[(i + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int yb = 0; yb < 2; ++yb) accZ[yb][nb] = mfma4(er[yb][i], br[i & 1][nb], accZ[yb][nb]);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int yb = 0; yb < 2; ++yb) accZ[yb][nb] = mfma4(ei[yb][i], bi[i & 1][nb], accZ[yb][nb]);
        __builtin_amdgcn_sched_barrier(0);
    }
}


// (c) as above with the B3 operands in fragment order: the tile holds, per
// 16-column half xb, column block nb and part (re, im), 64 lanes x 4 rows,
// so one 16-byte read gives a lane its operands of all four steps; the
// products are issued in the same order, so the sums are the same.
template <int NB>
__device__ __forceinline__ void adjoint_rows_frag(f4 (&accZ)[2][NB], const f4 (&er)[2], const f4 (&ei)[2],
                                                  const float *Bt, int xb, int lane) {
    f4 br[NB], bi[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        br[nb] = *reinterpret_cast<const f4 *>(Bt + ((((xb * NB + nb) * 2 + 0) * 64 + lane) * 4));
        bi[nb] = *reinterpret_cast<const f4 *>(Bt + ((((xb * NB + nb) * 2 + 1) * 64 + lane) * 4));
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int yb = 0; yb < 2; ++yb) accZ[yb][nb] = mfma4(er[yb][i], br[nb][i], accZ[yb][nb]);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int yb = 0; yb < 2; ++yb) accZ[yb][nb] = mfma4(ei[yb][i], bi[nb][i], accZ[yb][nb]);
    }
}

}  // namespace ilt_dev
