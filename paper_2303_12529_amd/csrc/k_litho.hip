// SOCS imaging and its adjoint on gfx950 matrix cores (FP32 MFMA 16x16x4).
//
// Paper: Sec. II-B (Hopkins model approximated by the sum of coherent
// systems, I = sum_k w_k |M (*) h_k|^2 with N_k = 24 kernels) and Sec. III-A
// (the ILT gradient: dL/dM through the rotated kernel H' and the conjugate
// H*).  The paper computes these convolutions with its own FFT; here every
// transform is a pruned DFT on the P x P pass-band window written as a
// dense GEMM, because only P^2 of the N^2 frequencies are non-zero:
//
//   spectrum   S = A M A^T            (N x N -> P x P)
//   rows       Y_k = c_k (H_k . S) conj(A)      (P x P -> P x N), c_k = sqrt(w_k)/N^2
//   image      I = sum_k |A^H Y_k|^2             (P x N -> N x N, fused |.|^2)
//   adjoint    V_k = A (G . E_k) A^T, W = sum_k c_k conj(H_k) . V_k
//   gradient   g = 2 Re(A^H W conj(A))
//
// Layouts of the tables and workspaces are described in ilt_internal.h.
#include "ilt_internal.h"

namespace {

__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// --------------------------------------------------------------------------
// Spectrum, first half: T1[y][n] = sum_x M[y][x] tb0[x][n]  (row transform).
// One block per 16-row band; 8 waves split the x range; the 8 partial
// accumulators are summed in a fixed order through LDS.
// src_is_phi: M = [phi <= 0]; else M = src (real mask).
// --------------------------------------------------------------------------
template <int NZ>
__global__ __launch_bounds__(512) void k_spectrum_rows(const float *__restrict__ src, int src_is_phi,
                                                       const float *__restrict__ tb, int N, int Np,
                                                       float *__restrict__ t1) {
    constexpr int NB = NZ / 16;
    __shared__ float red[8][16][NZ + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int y0 = blockIdx.x * 16;
    const int span = Np / 8;
    const int xa = wave * span;
    f4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = f4{0.f, 0.f, 0.f, 0.f};
    const int y = y0 + l16;
    const bool yok = y < N;
    for (int x = xa; x < xa + span; x += 4) {
        const int xx = x + lq;
        float m = 0.f;
        if (yok && xx < N) {
            const float v = src[(size_t)y * N + xx];
            m = src_is_phi ? (v <= 0.f ? 1.f : 0.f) : v;
        }
        const float *brow = tb + (size_t)xx * NZ + l16;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma4(m, brow[nb * 16], acc[nb]);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[wave][4 * lq + i][nb * 16 + l16] = acc[nb][i];
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * NZ; e += 512) {
        const int r = e / NZ, n = e % NZ;
        float s = 0.f;
#pragma unroll
        for (int w = 0; w < 8; ++w) s += red[w][r][n];
        t1[((size_t)blockIdx.x * 16 + r) * NZ + n] = s;
    }
}

// Spectrum, second half: S[a][b] = sum_y A[a][y] T1[y][b] (complex), in FP64.
// One block per window row a; four y-quarters reduced in a fixed order.
__global__ __launch_bounds__(256) void k_spectrum_cols(const float *__restrict__ t1,
                                                       const float *__restrict__ ar,
                                                       const float *__restrict__ ai, int P, int N,
                                                       int Np, int NZ, int ZO, float2 *__restrict__ S) {
    __shared__ double sr[4][64], si[4][64];
    const int a = blockIdx.x;
    const int b = threadIdx.x & 63, q = threadIdx.x >> 6;
    double accr = 0.0, acci = 0.0;
    if (b < P) {
        const int per = (N + 3) / 4;
        const int ylo = q * per, yhi = min(N, ylo + per);
        for (int y = ylo; y < yhi; ++y) {
            const double c = ar[(size_t)a * Np + y], s = ai[(size_t)a * Np + y];
            const double tr = t1[(size_t)y * NZ + b], ti = t1[(size_t)y * NZ + ZO + b];
            accr += c * tr - s * ti;
            acci += c * ti + s * tr;
        }
    }
    sr[q][b] = accr;
    si[q][b] = acci;
    __syncthreads();
    if (q == 0 && b < P) {
        const double r = ((sr[0][b] + sr[1][b]) + sr[2][b]) + sr[3][b];
        const double i = ((si[0][b] + si[1][b]) + si[2][b]) + si[3][b];
        S[a * P + b] = make_float2((float)r, (float)i);
    }
}

// --------------------------------------------------------------------------
// Window -> rows: out[j][r][x] = scale_j * sum_b U_j[a][b] conj(A[b][x]),
// U_j = H_j . S (or U = S when H is null); rows r = a (real), P + a (imag).
// Grid (Np/64, n_j, n_sets); each thread owns one x and a strided set of a.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_window_rows(const float2 *__restrict__ H, size_t h_set_stride,
                                                     const float2 *__restrict__ S,
                                                     const float *__restrict__ scale, size_t sc_set_stride,
                                                     float scale_c, const float *__restrict__ ar,
                                                     const float *__restrict__ ai, int P, int KP, int Np,
                                                     int nj, int set_lo, float *__restrict__ out) {
    __shared__ float2 U[ILT_MAX_P * ILT_MAX_P];
    const int j = blockIdx.y, s = set_lo + blockIdx.z;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int ag = threadIdx.x >> 6;
    const float sc = scale ? scale[s * sc_set_stride + j] : scale_c;
    for (int e = threadIdx.x; e < P * P; e += 256) {
        float2 u = S[e];
        if (H) {
            const float2 h = H[s * h_set_stride + (size_t)j * P * P + e];
            u = make_float2(h.x * u.x - h.y * u.y, h.x * u.y + h.y * u.x);
        }
        U[e] = u;
    }
    __syncthreads();
    float *o = out + ((size_t)(s * nj + j) * KP) * Np;
    for (int a = ag; a < P; a += 4) {
        float yr = 0.f, yi = 0.f;
        for (int b = 0; b < P; ++b) {
            const float c = ar[(size_t)b * Np + x], sn = ai[(size_t)b * Np + x];
            const float2 u = U[a * P + b];
            // u * conj(A) = (ur + i ui)(c - i sn)
            yr = fmaf(u.x, c, fmaf(u.y, sn, yr));
            yi = fmaf(u.y, c, fmaf(-u.x, sn, yi));
        }
        o[(size_t)a * Np + x] = sc * yr;
        o[(size_t)(P + a) * Np + x] = sc * yi;
    }
}

// --------------------------------------------------------------------------
// Image: E_j = A^H Y_j per 16x16 block with Re E = L1 Y, Im E = L2 Y.
//   MODE 0: out = sum_j |E_j|^2      (aerial image of one kernel set)
//   MODE 1: out = Re E_0             (gradient back-transform), plus the
//           block maximum of |out| into maxpart[block].
// Block = 4 waves; block tile = 128 rows x 64 columns; wave tile = 32 x 64.
// The image-side operands L1, L2 of a wave stay in registers for all j; the
// Y_j tile of each j is staged through LDS and shared by the four waves.
// --------------------------------------------------------------------------
template <int KP, int MODE>
__global__ __launch_bounds__(256) void k_image(const float *__restrict__ tl, const float *__restrict__ Y,
                                               int nj, int N, int Np, int set_lo,
                                               float *__restrict__ out, double *__restrict__ maxpart) {
    constexpr int KS = KP / 4;
    constexpr int LDW = 64 + 16;
    __shared__ float Ys[KP][LDW];
    __shared__ float wmax[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int s = set_lo + blockIdx.z;
    const int x0 = blockIdx.x * 64;
    const int yw = blockIdx.y * 128 + wave * 32;

    float a1[2][KS], a2[2][KS];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            a1[mb][ks] = tl[(size_t)(4 * ks + lq) * Np + yw + 16 * mb + l16];
            a2[mb][ks] = tl[(size_t)(KP + 4 * ks + lq) * Np + yw + 16 * mb + l16];
        }
    f4 accI[2][4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) accI[mb][nb] = f4{0.f, 0.f, 0.f, 0.f};

    for (int j = 0; j < nj; ++j) {
        const float *Yj = Y + ((size_t)(s * nj + j) * KP) * Np + x0;
        for (int e = threadIdx.x; e < KP * 16; e += 256) {
            const int r = e >> 4, c4 = (e & 15) * 4;
            const float4 v = *reinterpret_cast<const float4 *>(Yj + (size_t)r * Np + c4);
            Ys[r][c4 + 0] = v.x;
            Ys[r][c4 + 1] = v.y;
            Ys[r][c4 + 2] = v.z;
            Ys[r][c4 + 3] = v.w;
        }
        __syncthreads();
        f4 er[2][4], ei[2][4];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                er[mb][nb] = f4{0.f, 0.f, 0.f, 0.f};
                ei[mb][nb] = f4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                const float b = Ys[4 * ks + lq][16 * nb + l16];
#pragma unroll
                for (int mb = 0; mb < 2; ++mb) {
                    er[mb][nb] = mfma4(a1[mb][ks], b, er[mb][nb]);
                    if (MODE == 0) ei[mb][nb] = mfma4(a2[mb][ks], b, ei[mb][nb]);
                }
            }
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (MODE == 0)
                        accI[mb][nb][i] = fmaf(er[mb][nb][i], er[mb][nb][i],
                                               fmaf(ei[mb][nb][i], ei[mb][nb][i], accI[mb][nb][i]));
                    else
                        accI[mb][nb][i] += er[mb][nb][i];
                }
        __syncthreads();
    }
    float m = 0.f;
    float *o = out + (size_t)blockIdx.z * N * N;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int y = yw + 16 * mb + 4 * lq + i, x = x0 + 16 * nb + l16;
                if (y < N && x < N) {
                    const float v = accI[mb][nb][i];
                    o[(size_t)y * N + x] = v;
                    if (MODE == 1) m = (v != v) ? INFINITY : fmaxf(m, fabsf(v));
                }
            }
    if (MODE == 1) {
        m = wave_max(m);
        if (lane == 0) wmax[wave] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            const float r = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
            maxpart[blockIdx.y * gridDim.x + blockIdx.x] = (double)r;
        }
    }
}

// --------------------------------------------------------------------------
// Adjoint, fused with recomputation of the fields.
// Block = (32-row tile, group of 4 kernels, set); wave w handles kernel
// j = 4*group + w.  For each 32-column chunk:
//   (a) E^T chunk = Y_j^T L^T     (A-operand streamed from Y_j, B in registers)
//   (b) X = G . E                 (G tile staged in LDS)
//   (c) Z += X B3                 (accumulator layout of (a) is fed straight
//                                  in as the A-operand; B3 chunk in LDS)
// after all chunks:
//   (d) V = A4 Z (window rows), W_part += c_j conj(H_j) . V, summed over the
//       four waves in a fixed order and written per block.
// --------------------------------------------------------------------------
template <int KP, int ZO>
__global__ __launch_bounds__(256) void k_adjoint(const float *__restrict__ tl, const float *__restrict__ tb,
                                                 const float *__restrict__ ta4, const float *__restrict__ Y,
                                                 const float *__restrict__ G, size_t g_set_stride,
                                                 const float2 *__restrict__ coef, int K, int P, int N,
                                                 int Np, int set_lo, float *__restrict__ Wpart) {
    constexpr int NZ = 2 * ZO, NB = NZ / 16, KS = KP / 4, AB = ZO / 16, AP = ZO;
    constexpr int LDB = NZ + 4;
    __shared__ float Gs[32][33];
    __shared__ float Bs[2][32][LDB];
    __shared__ float2 Ws[ILT_MAX_P * ILT_MAX_P];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int ytile = blockIdx.x, kg = blockIdx.y, srel = blockIdx.z, s = set_lo + srel;
    const int y0 = ytile * 32;
    const int j = kg * 4 + wave;
    const bool jok = j < K;

    float b1[2][KS], b2[2][KS];
#pragma unroll
    for (int yb = 0; yb < 2; ++yb)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            b1[yb][ks] = tl[(size_t)(4 * ks + lq) * Np + y0 + 16 * yb + l16];
            b2[yb][ks] = tl[(size_t)(KP + 4 * ks + lq) * Np + y0 + 16 * yb + l16];
        }
    f4 accZ[2][NB];
#pragma unroll
    for (int yb = 0; yb < 2; ++yb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) accZ[yb][nb] = f4{0.f, 0.f, 0.f, 0.f};

    const float *Yj = Y + ((size_t)(s * K + (jok ? j : 0)) * KP) * Np;
    const float *Gsrc = G + (size_t)s * g_set_stride;
    const int xend = (N + 31) & ~31;
    for (int x0 = 0; x0 < xend; x0 += 32) {
        for (int e = threadIdx.x; e < 32 * 32; e += 256) {
            const int yy = e >> 5, xx = e & 31;
            const int gy = y0 + yy, gx = x0 + xx;
            Gs[yy][xx] = (gy < N && gx < N) ? Gsrc[(size_t)gy * N + gx] : 0.f;
        }
        for (int e = threadIdx.x; e < 2 * 32 * (NZ / 4); e += 256) {
            const int part = e / (32 * (NZ / 4));
            const int rem = e % (32 * (NZ / 4));
            const int xx = rem / (NZ / 4), c4 = (rem % (NZ / 4)) * 4;
            const float4 v = *reinterpret_cast<const float4 *>(tb + ((size_t)part * Np + x0 + xx) * NZ + c4);
            Bs[part][xx][c4 + 0] = v.x;
            Bs[part][xx][c4 + 1] = v.y;
            Bs[part][xx][c4 + 2] = v.z;
            Bs[part][xx][c4 + 3] = v.w;
        }
        __syncthreads();
        if (jok) {
#pragma unroll
            for (int xb = 0; xb < 2; ++xb) {
                f4 er[2], ei[2];
#pragma unroll
                for (int yb = 0; yb < 2; ++yb) {
                    er[yb] = f4{0.f, 0.f, 0.f, 0.f};
                    ei[yb] = f4{0.f, 0.f, 0.f, 0.f};
                }
                const float *yrow = Yj + x0 + 16 * xb + l16;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const float a = yrow[(size_t)(4 * ks + lq) * Np];
#pragma unroll
                    for (int yb = 0; yb < 2; ++yb) {
                        er[yb] = mfma4(a, b1[yb][ks], er[yb]);
                        ei[yb] = mfma4(a, b2[yb][ks], ei[yb]);
                    }
                }
                // (b) multiply by G; er/ei register i holds E[y = 16yb + l16][x = 16xb + 4lq + i]
#pragma unroll
                for (int yb = 0; yb < 2; ++yb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float gv = Gs[16 * yb + l16][16 * xb + 4 * lq + i];
                        er[yb][i] *= gv;
                        ei[yb][i] *= gv;
                    }
                // (c) Z[y][n] += sum_x X[y][x] B3[x][n]
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int xr = 16 * xb + 4 * lq + i;
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        const float br = Bs[0][xr][16 * nb + l16];
                        const float bi = Bs[1][xr][16 * nb + l16];
#pragma unroll
                        for (int yb = 0; yb < 2; ++yb) {
                            accZ[yb][nb] = mfma4(er[yb][i], br, accZ[yb][nb]);
                            accZ[yb][nb] = mfma4(ei[yb][i], bi, accZ[yb][nb]);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }

    for (int e = threadIdx.x; e < P * P; e += 256) Ws[e] = make_float2(0.f, 0.f);
    __syncthreads();
    // (d) V[a][b] = sum_y A[a][y] Z[y][b]
    f4 vr[AB][AB], vi[AB][AB];
#pragma unroll
    for (int ab = 0; ab < AB; ++ab)
#pragma unroll
        for (int bb = 0; bb < AB; ++bb) {
            vr[ab][bb] = f4{0.f, 0.f, 0.f, 0.f};
            vi[ab][bb] = f4{0.f, 0.f, 0.f, 0.f};
        }
    if (jok) {
#pragma unroll
        for (int yb = 0; yb < 2; ++yb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int y = y0 + 16 * yb + 4 * lq + i;
#pragma unroll
                for (int ab = 0; ab < AB; ++ab) {
                    const float car = ta4[(size_t)y * AP + 16 * ab + l16];
                    const float cai = ta4[((size_t)Np + y) * AP + 16 * ab + l16];
#pragma unroll
                    for (int bb = 0; bb < AB; ++bb) {
                        const float zr = accZ[yb][bb][i];
                        const float zi = accZ[yb][bb + ZO / 16][i];
                        vr[ab][bb] = mfma4(car, zr, vr[ab][bb]);
                        vr[ab][bb] = mfma4(-cai, zi, vr[ab][bb]);
                        vi[ab][bb] = mfma4(cai, zr, vi[ab][bb]);
                        vi[ab][bb] = mfma4(car, zi, vi[ab][bb]);
                    }
                }
            }
    }
    const float2 *cj = coef + ((size_t)s * K + (jok ? j : 0)) * P * P;
    for (int w = 0; w < 4; ++w) {
        if (wave == w && jok) {
#pragma unroll
            for (int ab = 0; ab < AB; ++ab)
#pragma unroll
                for (int bb = 0; bb < AB; ++bb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int a = 16 * ab + 4 * lq + i, b = 16 * bb + l16;
                        if (a < P && b < P) {
                            const float2 c = cj[a * P + b];
                            const float xr = vr[ab][bb][i], xi = vi[ab][bb][i];
                            float2 cur = Ws[a * P + b];
                            cur.x += c.x * xr - c.y * xi;
                            cur.y += c.x * xi + c.y * xr;
                            Ws[a * P + b] = cur;
                        }
                    }
        }
        __syncthreads();
    }
    float *dst = Wpart + ((size_t)(srel * gridDim.x + ytile) * gridDim.y + kg) * P * P * 2;
    for (int e = threadIdx.x; e < P * P; e += 256) {
        dst[2 * e] = Ws[e].x;
        dst[2 * e + 1] = Ws[e].y;
    }
}

// W[a][b] = sum over all adjoint partials, in FP64, fixed order.
__global__ __launch_bounds__(256) void k_window_sum(const float *__restrict__ Wpart, int nparts, int P,
                                                    float2 *__restrict__ W) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= P * P) return;
    double r = 0.0, i = 0.0;
    for (int p = 0; p < nparts; ++p) {
        r += Wpart[((size_t)p * P * P + e) * 2];
        i += Wpart[((size_t)p * P * P + e) * 2 + 1];
    }
    W[e] = make_float2((float)r, (float)i);
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_spectrum(ilt_ctx *c, const float *src, int src_is_phi) {
    const int nyb = c->Np / 16;
    switch (c->NZ) {
        case 32: k_spectrum_rows<32><<<nyb, 512, 0, c->stream>>>(src, src_is_phi, c->tb, c->N, c->Np, c->t1); break;
        case 64: k_spectrum_rows<64><<<nyb, 512, 0, c->stream>>>(src, src_is_phi, c->tb, c->N, c->Np, c->t1); break;
        case 96: k_spectrum_rows<96><<<nyb, 512, 0, c->stream>>>(src, src_is_phi, c->tb, c->N, c->Np, c->t1); break;
        default: return hipErrorInvalidValue;
    }
    k_spectrum_cols<<<c->P, 256, 0, c->stream>>>(c->t1, c->ar, c->ai, c->P, c->N, c->Np, c->NZ, c->ZO, c->S);
    return hipGetLastError();
}

hipError_t launch_make_Y(ilt_ctx *c, int set_lo, int set_hi) {
    dim3 grid(c->Np / 64, c->K, set_hi - set_lo);
    k_window_rows<<<grid, 256, 0, c->stream>>>(c->H, (size_t)c->K * c->P * c->P, c->S, c->sw, (size_t)c->K,
                                               1.f, c->ar, c->ai, c->P, c->KP, c->Np, c->K, set_lo, c->Y);
    return hipGetLastError();
}

template <int MODE>
static hipError_t image_dispatch(ilt_ctx *c, const float *Y, int nj, int set_lo, int nsets, float *out,
                                 double *maxpart) {
    dim3 grid(c->Np / 64, c->Np / 128, nsets);
    switch (c->KP) {
        case 8: k_image<8, MODE><<<grid, 256, 0, c->stream>>>(c->tl, Y, nj, c->N, c->Np, set_lo, out, maxpart); break;
        case 24: k_image<24, MODE><<<grid, 256, 0, c->stream>>>(c->tl, Y, nj, c->N, c->Np, set_lo, out, maxpart); break;
        case 40: k_image<40, MODE><<<grid, 256, 0, c->stream>>>(c->tl, Y, nj, c->N, c->Np, set_lo, out, maxpart); break;
        case 72: k_image<72, MODE><<<grid, 256, 0, c->stream>>>(c->tl, Y, nj, c->N, c->Np, set_lo, out, maxpart); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_image_to(ilt_ctx *c, int set_lo, int set_hi, float *out) {
    return image_dispatch<0>(c, c->Y, c->K, set_lo, set_hi - set_lo, out, nullptr);
}

hipError_t launch_adjoint(ilt_ctx *c, const float *G, size_t g_set_stride, int set_lo, int set_hi) {
    dim3 grid((c->N + 31) / 32, (c->K + 3) / 4, set_hi - set_lo);
#define ADJ(KP_, ZO_)                                                                                  \
    k_adjoint<KP_, ZO_><<<grid, 256, 0, c->stream>>>(c->tl, c->tb, c->ta4, c->Y, G, g_set_stride, c->coef, \
                                                     c->K, c->P, c->N, c->Np, set_lo, c->Wpart)
    if (c->KP == 8 && c->ZO == 16) ADJ(8, 16);
    else if (c->KP == 24 && c->ZO == 16) ADJ(24, 16);
    else if (c->KP == 40 && c->ZO == 16) ADJ(40, 16);
    else if (c->KP == 40 && c->ZO == 32) ADJ(40, 32);
    else if (c->KP == 72 && c->ZO == 32) ADJ(72, 32);
    else if (c->KP == 72 && c->ZO == 48) ADJ(72, 48);
    else return hipErrorInvalidValue;
#undef ADJ
    return hipGetLastError();
}

hipError_t launch_window_sum(ilt_ctx *c, int set_lo, int set_hi) {
    const int nparts = (set_hi - set_lo) * ((c->N + 31) / 32) * ((c->K + 3) / 4);
    k_window_sum<<<(c->P * c->P + 255) / 256, 256, 0, c->stream>>>(c->Wpart, nparts, c->P, c->W);
    return hipGetLastError();
}

hipError_t launch_gradient(ilt_ctx *c, float *g_out, double *maxpart) {
    // Tg = 2 W conj(A) in the row layout, then g = Re(A^H Tg)
    dim3 grid(c->Np / 64, 1, 1);
    k_window_rows<<<grid, 256, 0, c->stream>>>(nullptr, 0, c->W, nullptr, 0, 2.f, c->ar, c->ai, c->P, c->KP,
                                               c->Np, 1, 0, c->Tg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return image_dispatch<1>(c, c->Tg, 1, 0, 1, g_out, maxpart);
}
