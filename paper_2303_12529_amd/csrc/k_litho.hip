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
// Matrix-core operand conventions (16x16x4 FP32): lane l supplies
// A[m = l%16][k = l/16] and B[k = l/16][n = l%16]; accumulator register i of
// lane l holds C[m = 4(l/16) + i][n = l%16].  The image kernel computes E^T
// (m = x, n = y), so register i of lane l is E[y = l%16][x = 4(l/16) + i]:
// exactly the A-operand the adjoint's row transform needs (k = x), and the
// field fragments are stored and reloaded in that native layout.
#include "ilt_internal.h"
#include "ilt_device.h"

namespace {

__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// --------------------------------------------------------------------------
// Spectrum.  Block = one 16-row band x one of gridDim.y column ranges, 8
// waves splitting the range:
//   T1[y][n] = sum_x M[y][x] tb0[x][n]        (matrix cores; M = [phi<=0] or src)
//   Spart[band][a][b] = sum_{y in band} A[a][y] T1[y][b]
// The band product is a 16-deep complex GEMM on the matrix cores too: per
// 16 x 16 output tile, S_re = [Ar | -Ai] [T1_re; T1_im] and
// S_im = [Ar | Ai] [T1_im; T1_re], the B operands gathered from the band's
// T1 columns of the window layout.  Band partials are FP32 (16-term sums);
// they are summed over the bands in FP64.
// Each lane loads four consecutive columns of its row as one float4 and uses
// them in four consecutive k-steps; the B-operand rows follow the same
// (x = 4(l/16) + e) order, so the sum is unchanged.  The column table comes
// in fragment order ([x/16][NZ/16][lane][e]): one 16-byte load per column
// block gives a lane its B operands of those four steps.
// --------------------------------------------------------------------------
// PR: window rows (the twiddles ar, ai), P: window columns (the table tb);
// PR = P but for the difference window of a real image, whose columns
// Db >= 0 suffice (the others are conjugates, k_conj_fill).
template <int FB, int MIX>
__global__ __launch_bounds__(512) void k_spectrum_band(const float *__restrict__ src, size_t src_stride,
                                                       int src_is_phi, const float *__restrict__ tb,
                                                       const float *__restrict__ ar, const float *__restrict__ ai,
                                                       int PR, int P, int N, int Np, float2 *__restrict__ Spart) {
    // grid.z: independent images src + z src_stride, partials in their own range
    src += blockIdx.z * src_stride;
    Spart += (size_t)blockIdx.z * gridDim.x * gridDim.y * PR * P;
    constexpr int NZ = 32 * FB + 16 * MIX;
    constexpr int NB = NZ / 16;
    constexpr int PW = 2 * ILT_MAX_P - 1;          // >= every window's row count
    __shared__ float red[4][16][NZ + 1];
    __shared__ float twr[PW][17], twi[PW][17];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int y0 = blockIdx.x * 16;
    const int span = Np / (8 * gridDim.y);
    const int xa = blockIdx.y * (Np / gridDim.y) + wave * span;
    f4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = f4{0.f, 0.f, 0.f, 0.f};
    const int y = y0 + l16;
    const bool yok = y < N;
    const bool vec = (N % 4) == 0;
    for (int x = xa; x < xa + span; x += 16) {
        const int xx = x + 4 * lq;
        float m[4] = {0.f, 0.f, 0.f, 0.f};
        if (yok) {
            if (vec && xx + 3 < N) {
                const float4 v = *reinterpret_cast<const float4 *>(src + (size_t)y * N + xx);
                m[0] = v.x; m[1] = v.y; m[2] = v.z; m[3] = v.w;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (xx + e < N) m[e] = src[(size_t)y * N + xx + e];
            }
            if (src_is_phi) {
#pragma unroll
                for (int e = 0; e < 4; ++e) m[e] = m[e] <= 0.f ? 1.f : 0.f;
            }
        }
        f4 bv[NB];
        const f4 *bsrc = reinterpret_cast<const f4 *>(tb) + (size_t)(x / 16) * NB * 64 + lane;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) bv[nb] = bsrc[nb * 64];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma4(m[e], bv[nb][e], acc[nb]);
        }
    }
    // sum of the 8 waves' partials in a fixed order, through half as much
    // LDS: waves 4..7 store, waves 0..3 add theirs (w + (w + 4)), then the
    // four pair sums are added in order
    if (wave >= 4) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int i = 0; i < 4; ++i) red[wave - 4][4 * lq + i][nb * 16 + l16] = acc[nb][i];
    }
    __syncthreads();
    if (wave < 4) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float &r = red[wave][4 * lq + i][nb * 16 + l16];
                r = acc[nb][i] + r;
            }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * NZ; e += 512) {
        const int r = e / NZ, n = e % NZ;
        red[0][r][n] = ((red[0][r][n] + red[1][r][n]) + red[2][r][n]) + red[3][r][n];
    }
    __syncthreads();
    // the band's 16 twiddle columns of every window row, once per block
    for (int e = threadIdx.x; e < PR * 16; e += 512) {
        const int a = e / 16, r = e % 16;
        const int yy = min(y0 + r, N - 1);
        twr[a][r] = ar[(size_t)a * Np + yy];
        twi[a][r] = ai[(size_t)a * Np + yy];
    }
    __syncthreads();
    // band partial of S = A T1 (rows of the band beyond the image hold T1 = 0)
    float2 *dst = Spart + ((size_t)blockIdx.x * gridDim.y + blockIdx.y) * PR * P;
    const int TA = (PR + 15) / 16, TC = (P + 15) / 16;
    for (int t = wave; t < TA * TC; t += 8) {
        const int ta = t / TC, tc = t - (t / TC) * TC;
        const int a = 16 * ta + l16, b = 16 * tc + l16;
        const bool aok = a < PR, bok = b < P;
        const int cre = bok ? win_re(b, FB) : 0, cim = bok ? win_im(b, FB) : 0;
        f4 sre = f4{0.f, 0.f, 0.f, 0.f}, sim = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int r = 4 * ks + lq;
            const float cw = aok ? twr[a][r] : 0.f, sw = aok ? twi[a][r] : 0.f;
            const float tre = red[0][r][cre], tim = red[0][r][cim];
            sre = mfma4(cw, tre, sre);
            sre = mfma4(-sw, tim, sre);
            sim = mfma4(cw, tim, sim);
            sim = mfma4(sw, tre, sim);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ao = 16 * ta + 4 * lq + i;
            if (ao < PR && bok) dst[ao * P + b] = make_float2(sre[i], sim[i]);
        }
    }
}

// Deterministic sum of n complex partial arrays: out[e] = sum_p part[p][e].
// Block = 16 outputs x 64 partial groups; groups combined in a fixed order.
// grid.y: independent sums (part + y nparts n -> out + y n).
template <typename T2>
__global__ __launch_bounds__(1024) void k_psum(const T2 *__restrict__ part, int nparts, int n,
                                               float2 *__restrict__ out) {
    part += (size_t)blockIdx.y * nparts * n;
    out += (size_t)blockIdx.y * n;
    __shared__ double sr[64][17], si[64][17];
    const int o = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int e = blockIdx.x * 16 + o;
    double r = 0.0, i = 0.0;
    if (e < n)
        for (int p = g; p < nparts; p += 64) {
            const T2 v = part[(size_t)p * n + e];
            r += (double)v.x;
            i += (double)v.y;
        }
    sr[g][o] = r;
    si[g][o] = i;
    __syncthreads();
    if (g == 0 && e < n) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < 64; ++q) {
            a += sr[q][o];
            b += si[q][o];
        }
        out[e] = make_float2((float)a, (float)b);
    }
}

// --------------------------------------------------------------------------
// Window -> rows: out[j][r][x] = scale_j * sum_b U_j[a][b] conj(A[b][x]),
// U_j = H_j . S (or U = S when H is null); rows r = a (real), PR + a (imag).
// The window has PR rows of P columns (PR = P but for the image spectrum's
// half window; H is used only with PR = P).
// Grid (Np/COLS, ceil(n_j/JB), n_sets); COLS columns x 256/COLS row groups
// per block, JB kernels per block; each thread keeps the twiddles of its
// column in registers and reuses them for the block's JB kernels.
// --------------------------------------------------------------------------
template <int COLS, int JB, int WS = ILT_MAX_P>
__global__ __launch_bounds__(256) void k_window_rows(const float2 *__restrict__ H, const float2 *__restrict__ S,
                                                     const float *__restrict__ scale, float scale_c,
                                                     const float *__restrict__ ar, const float *__restrict__ ai,
                                                     int P, int PR, int KP, int Np, int nj, int set_lo,
                                                     float *__restrict__ out, int zs, size_t s_cs, size_t out_cs) {
    constexpr int RG = 256 / COLS;
    __shared__ float2 U[JB][WS * WS];
    // grid.z = clips x zs window slices; every clip has its own S and out
    const int clip = blockIdx.z / zs;
    S += clip * s_cs;
    out += clip * out_cs;
    const int j0 = blockIdx.y * JB, s = set_lo + (blockIdx.z - clip * zs);
    const int x = blockIdx.x * COLS + (threadIdx.x % COLS);
    const int ag = threadIdx.x / COLS;
    const int jn = min(JB, nj - j0);
    // U_j = H_j . S (or S itself): a thread's loads are issued before any
    // product is stored
    constexpr int UPT = (WS * WS + 255) / 256;
    for (int jj = 0; jj < jn; ++jj) {
        float2 sv[UPT], hv[UPT];
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            const int e = threadIdx.x + 256 * u;
            if (e < PR * P) {
                sv[u] = S[e];
                if (H) hv[u] = H[((size_t)s * nj + j0 + jj) * P * P + e];
            }
        }
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            const int e = threadIdx.x + 256 * u;
            if (e < PR * P) {
                float2 v = sv[u];
                if (H) v = make_float2(hv[u].x * v.x - hv[u].y * v.y, hv[u].x * v.y + hv[u].y * v.x);
                U[jj][e] = v;
            }
        }
    }
    float cr[WS], ci[WS];
#pragma unroll
    for (int b = 0; b < WS; ++b) {
        cr[b] = b < P ? ar[(size_t)b * Np + x] : 0.f;
        ci[b] = b < P ? ai[(size_t)b * Np + x] : 0.f;
    }
    __syncthreads();
    for (int jj = 0; jj < jn; ++jj) {
        const int j = j0 + jj;
        const float sc = scale ? scale[(size_t)s * nj + j] : scale_c;
        float *o = out + ((size_t)(s * nj + j) * KP) * Np;
        for (int a = ag; a < PR; a += RG) {
            float yr = 0.f, yi = 0.f;
#pragma unroll
            for (int b = 0; b < WS; ++b) {
                if (b < P) {
                    const float2 u = U[jj][a * P + b];
                    // u * conj(A) = (ur + i ui)(c - i sn)
                    yr = fmaf(u.x, cr[b], fmaf(u.y, ci[b], yr));
                    yi = fmaf(u.y, cr[b], fmaf(-u.x, ci[b], yi));
                }
            }
            o[(size_t)a * Np + x] = sc * yr;
            o[(size_t)(PR + a) * Np + x] = sc * yi;
        }
    }
}

// --------------------------------------------------------------------------
// Window -> rows for every kernel on the matrix cores.  With U_j = H_j . S
// and conj(A) = Ar - i Ai, the rows of Y_j are
//   [Re; Im](U_j conj(A)) = C_j [Ar; Ai],  C_j = [[Ur, Ui], [Ui, -Ur]],
// a (2P x 2P) x (2P x N) real GEMM whose right operand is the image-side
// table tl (part 0 holds [Ar; Ai] in rows [0, 2P)).  Block = (128-column
// range, kernel j, set): the scaled C_j is built in LDS, each wave takes 32
// columns (two 16-column tiles) of every 16-row tile of C_j.
// SPLIT: write the split-BF16 form instead, Yhl [set][j][Np][hi | lo][KP]
// with hi = bf16(y), lo = bf16(y - hi) (rows [2P, KP) zero).
// --------------------------------------------------------------------------
template <int KP, bool SPLIT>
__global__ __launch_bounds__(256) void k_make_y(const float2 *__restrict__ H, const float2 *__restrict__ S,
                                                const float *__restrict__ scale, const float *__restrict__ tl,
                                                int P, int Np, int nj, int set_lo, float *__restrict__ out,
                                                __bf16 *__restrict__ outhl, int zs, size_t s_cs, size_t y_cs) {
    constexpr int MT = (KP + 15) / 16;            // 16-row tiles of C (>= 2P rows)
    constexpr int LDC = KP + 4;
    __shared__ float C[16 * MT][LDC];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    // grid.z = clips x sets; every clip has its own S and Y (FP32 form)
    const int clip = blockIdx.z / zs;
    S += clip * s_cs;
    if (out) out += clip * y_cs;
    const int j = blockIdx.y, s = set_lo + (blockIdx.z - clip * zs);
    const float sc = scale[(size_t)s * nj + j];
    const int x0 = blockIdx.x * 128 + wave * 32;
    // all of the wave's tl operands are requested first (2 KP / 4 values),
    // so that their latency overlaps the construction of C
    float bt[KP / 4][2];
#pragma unroll
    for (int ks = 0; ks < KP / 4; ++ks)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) bt[ks][nt] = tl[(size_t)(4 * ks + lq) * Np + x0 + 16 * nt + l16];
    const float2 *Hj = H + (size_t)(s * nj + j) * P * P;
    // pad rows and columns of C are zero
    for (int e = threadIdx.x; e < 16 * MT * KP; e += 256) {
        const int m = e / KP, k = e - (e / KP) * KP;
        if (m >= 2 * P || k >= 2 * P) C[m][k] = 0.f;
    }
    // each U entry fills four places of C; the loads of a thread's entries
    // are issued together (P^2 <= 5 x 256)
    constexpr int UPT = (ILT_MAX_P * ILT_MAX_P + 255) / 256;
    float2 hv[UPT], sv[UPT];
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
        const int e = threadIdx.x + 256 * u;
        hv[u] = e < P * P ? Hj[e] : make_float2(0.f, 0.f);
        sv[u] = e < P * P ? S[e] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
        const int e = threadIdx.x + 256 * u;
        if (e < P * P) {
            const int a = e / P, b = e - (e / P) * P;
            const float ur = sc * (hv[u].x * sv[u].x - hv[u].y * sv[u].y);
            const float ui = sc * (hv[u].x * sv[u].y + hv[u].y * sv[u].x);
            C[a][b] = ur;
            C[a][P + b] = ui;
            C[P + a][b] = ui;
            C[P + a][P + b] = -ur;
        }
    }
    __syncthreads();
    f4 acc[MT][2];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KP / 4; ++ks) {
        const int k = 4 * ks + lq;
        float b[2] = {bt[ks][0], bt[ks][1]}, a[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) a[mt] = C[16 * mt + l16][k];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = mfma4(a[mt], b[nt], acc[mt][nt]);
    }
    if (SPLIT) {
        // four consecutive rows per lane: 8 bytes of hi and 8 of lo per column
        typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int r0 = 16 * mt + 4 * lq;
            if (r0 >= KP) continue;
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                const int x = x0 + 16 * nt + l16;
                bf4 h, l;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float v = acc[mt][nt][i];
                    h[i] = (__bf16)v;
                    l[i] = (__bf16)(v - (float)h[i]);
                }
                __bf16 *d = outhl + (((size_t)(s * nj + j) * Np) + x) * 2 * KP + r0;
                *reinterpret_cast<bf4 *>(d) = h;
                *reinterpret_cast<bf4 *>(d + KP) = l;
            }
        }
        return;
    }
    float *o = out + ((size_t)(s * nj + j) * KP) * Np;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * mt + 4 * lq + i;
                if (r < 2 * P) o[(size_t)r * Np + x0 + 16 * nt + l16] = acc[mt][nt][i];
            }
}

// --------------------------------------------------------------------------
// Image: per 16x16 block, E_j^T = Y_j^T L^T with Re E = L1 Y, Im E = L2 Y.
//   MODE 0: out = sum_j |E_j|^2      (aerial image of one kernel set)
//   MODE 2: out = Re E_0             (an image from its window rows)
//   MODE 1: out = Re E_0             (gradient back-transform), plus the
//           block maximum of |out| into maxpart[block].
//   STORE:  also write every E_j fragment to Est in the accumulator layout
//           [set][j][y/16][x/16][re|im][lane][4].
// Block = 4 waves; block tile = 128 rows x 64 columns; wave tile = 32 x 64.
// The image-side operands (L rows of the wave's 32 y) stay in registers as
// B-operands; each Y_j tile (KP x 64) is staged in LDS, double-buffered
// (the next j copied global -> LDS by the memory unit), and shared by the
// four waves.
// --------------------------------------------------------------------------
template <int KP, int MODE, bool STORE>
__global__ __launch_bounds__(256, 2) void k_image(const float *__restrict__ tl, const float *__restrict__ Y,
                                               int nj, int N, int Np, int set_lo, float *__restrict__ out,
                                               double *__restrict__ maxpart, float *__restrict__ Est, int zs,
                                               size_t y_cs, size_t out_cs, size_t max_cs, size_t est_cs) {
    constexpr int KS = KP / 4;
    constexpr int LDW = 64 + 16;
    // Y_j tiles, KP rows of LDW floats (16 data units of 16 bytes + 4 pad
    // units), rounded up to whole 64-unit copies
    constexpr int RU = LDW / 4, NYI = (KP * RU + 63) / 64, NYT = (NYI + 3) / 4;
    constexpr int NBUF = MODE == 0 ? 2 : 1;        // MODE 1, 2: one tile (nj = 1)
    __shared__ __align__(16) float Ysm[NBUF][NYI * 256];
    __shared__ float wmax[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    // grid.z = clips x sets; every clip has its own Y, output, maxima and fields
    const int clip = blockIdx.z / zs, zr = blockIdx.z - clip * zs;
    Y += clip * y_cs;
    out += clip * out_cs;
    if (MODE == 1) maxpart += clip * max_cs;
    if (STORE) Est += clip * est_cs;
    const int s = set_lo + zr;
    const int x0 = blockIdx.x * 64;
    const int yw = blockIdx.y * 128 + wave * 32;
    const int NB16 = Np / 16;

    float b1[2][KS], b2[2][KS];
#pragma unroll
    for (int yb = 0; yb < 2; ++yb)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            b1[yb][ks] = tl[(size_t)(4 * ks + lq) * Np + yw + 16 * yb + l16];
            if (MODE == 0) b2[yb][ks] = tl[(size_t)(KP + 4 * ks + lq) * Np + yw + 16 * yb + l16];
        }
    f4 accI[4][2];
#pragma unroll
    for (int xb = 0; xb < 4; ++xb)
#pragma unroll
        for (int yb = 0; yb < 2; ++yb) accI[xb][yb] = f4{0.f, 0.f, 0.f, 0.f};

    // copied global -> LDS by the memory unit, the copy of Y_{j+1} in flight
    // while Y_j is contracted; per-lane source offsets formed once (wave w
    // copies the 64-unit groups w, w + 4, ...; pad units and the units past
    // the last row copy a valid unit and are never read)
    int yoff[NYT];
#pragma unroll
    for (int t = 0; t < NYT; ++t) {
        const int U = 64 * (wave + 4 * t) + lane;
        const int row = min(U / RU, KP - 1), col = U - (U / RU) * RU;
        yoff[t] = row * Np + (col < 16 ? 4 * col : 0);
    }
    auto copy_y = [&](int jj, int bb) {
        const float *src = Y + ((size_t)(s * nj + jj) * KP) * Np + x0;
#pragma unroll
        for (int t = 0; t < NYT; ++t)
            if (wave + 4 * t < NYI) ilt_dev::lds_dma16(src + yoff[t], &Ysm[bb][256 * (wave + 4 * t)]);
    };
    copy_y(0, 0);
    ilt_dev::wait_copies();
    __syncthreads();
    for (int j = 0; j < nj; ++j) {
        const int buf = NBUF == 2 ? (j & 1) : 0;
        if (NBUF == 2 && j + 1 < nj) copy_y(j + 1, buf ^ 1);
        f4 er[4][2], ei[4][2];
#pragma unroll
        for (int xb = 0; xb < 4; ++xb)
#pragma unroll
            for (int yb = 0; yb < 2; ++yb) {
                er[xb][yb] = f4{0.f, 0.f, 0.f, 0.f};
                ei[xb][yb] = f4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
            for (int xb = 0; xb < 4; ++xb) {
                const float a = Ysm[buf][(4 * ks + lq) * LDW + 16 * xb + l16];
#pragma unroll
                for (int yb = 0; yb < 2; ++yb) {
                    er[xb][yb] = mfma4(a, b1[yb][ks], er[xb][yb]);
                    if (MODE == 0) ei[xb][yb] = mfma4(a, b2[yb][ks], ei[xb][yb]);
                }
            }
        }
        // this wave's copy of Y_{j+1} has landed (waited for before the field
        // stores are issued, so that the wait does not cover them)
        ilt_dev::wait_copies();
        if (STORE) {
#pragma unroll
            for (int xb = 0; xb < 4; ++xb)
#pragma unroll
                for (int yb = 0; yb < 2; ++yb) {
                    const size_t blk = (((size_t)(s * nj + j) * NB16 + (yw / 16 + yb)) * NB16 + (x0 / 16 + xb));
                    float *dst = Est + blk * 512 + lane * 4;
                    __builtin_nontemporal_store(er[xb][yb], reinterpret_cast<f4 *>(dst));
                    __builtin_nontemporal_store(ei[xb][yb], reinterpret_cast<f4 *>(dst + 256));
                }
        }
#pragma unroll
        for (int xb = 0; xb < 4; ++xb)
#pragma unroll
            for (int yb = 0; yb < 2; ++yb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (MODE == 0)
                        accI[xb][yb][i] = fmaf(er[xb][yb][i], er[xb][yb][i],
                                               fmaf(ei[xb][yb][i], ei[xb][yb][i], accI[xb][yb][i]));
                    else
                        accI[xb][yb][i] += er[xb][yb][i];
                }
        // every wave is done with buffer buf before it is refilled
        __syncthreads();
    }
    float m = 0.f;
    float *o = out + (size_t)zr * N * N;
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
                if (MODE == 1)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (x + i < N) {
                            const float v = accI[xb][yb][i];
                            m = (v != v) ? INFINITY : fmaxf(m, fabsf(v));
                        }
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
// Adjoint from stored fields.  Block = (32-row tile, group of 4 kernels,
// set); wave w handles kernel j = 4*group + w and walks its columns in
// 32-column chunks:
//   X = G . E_j    (E_j fragments read in accumulator layout, G from LDS)
//   Z += X B3      (E fragments are the A-operand as loaded; B3 from LDS)
// then the shared tail.  grid.y = kernel groups x column ranges: a block
// walks its range of chunks only (its partial W is summed with the others').
//
// The B3 operands come from a table in fragment order ([chunk][16-column
// half][column block][re|im][lane][4 rows]), so that one 16-byte LDS read
// gives a lane its operands of four matrix-core steps.
//
// Pipeline, one barrier per chunk: the B3 operands and G tile of chunk c + 1
// are copied global -> LDS (no registers) into the other half of
// double-buffered tiles, and the E fragments of the next 16-column half are
// loaded into registers, while the current half is multiplied.  Both are
// issued only after the compiler's wait for the current half's fragments,
// so that its waits never cover them; the chunk ends with a full wait and
// the barrier.  G tiles are copied with clamped coordinates and masked when
// read (N % 4 == 0), else staged through registers.  The tail's W
// accumulator reuses the two B3 tiles.
// --------------------------------------------------------------------------
template <int FB, int MIX, bool A4>
__global__ __launch_bounds__(256, 2) void k_adjoint_st(const float *__restrict__ tba, const float *__restrict__ ta4,
                                                    const float *__restrict__ Est, const float *__restrict__ G,
                                                    size_t g_set_stride, const float2 *__restrict__ coef, int K,
                                                    int P, int N, int Np, int AP, int set_lo,
                                                    float *__restrict__ Wpart, int zs, size_t est_cs, size_t g_cs,
                                                    size_t wp_cs) {
    constexpr int NZ = 32 * FB + 16 * MIX, NB = NZ / 16;
    constexpr int BU = 4 * NB * 64;                   // 16-byte units of one B3 tile, fragment order
    constexpr int WU = (int)((sizeof(float2) * ILT_MAX_P * ILT_MAX_P + 2047) / 2048) * 64;   // W: 16-byte units per tile
    constexpr int BUA = BU > WU ? BU : WU;            // tile size in LDS
    constexpr int GU = 320;                           // G tile [32][36] = 288 units, padded to 5 x 64
    static_assert(BU % 64 == 0, "B3 tile must be whole wave copies");
    static_assert((size_t)2 * BUA * 16 >= sizeof(float2) * ILT_MAX_P * ILT_MAX_P, "W accumulator must fit the B3 tiles");
    __shared__ __align__(16) float Bs[2][BUA * 4];
    __shared__ __align__(16) float Gs[2][GU * 4];
    float2 *Ws = reinterpret_cast<float2 *>(&Bs[0][0]);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int kgroups = (K + 3) / 4;
    const int ytile = blockIdx.x, kg = blockIdx.y % kgroups, xs = blockIdx.y / kgroups;
    // grid.z = clips x sets; every clip has its own fields, G and partials
    const int clip = blockIdx.z / zs;
    Est += clip * est_cs;
    G += clip * g_cs;
    Wpart += clip * wp_cs;
    const int srel = blockIdx.z - clip * zs, s = set_lo + srel;
    const int y0 = ytile * 32;
    const int j = kg * 4 + wave;
    const bool jok = j < K;
    const int NB16 = Np / 16;
    const float *Gsrc = G + (size_t)s * g_set_stride;
    const float *Ej = Est + (size_t)(s * K + (jok ? j : 0)) * NB16 * NB16 * 512;
    const int nchunk = (N + 31) / 32;
    const int xsplit = gridDim.y / kgroups;
    const int c_begin = xs * nchunk / xsplit, c_end = (xs + 1) * nchunk / xsplit;

    f4 accZ[2][NB];
#pragma unroll
    for (int yb = 0; yb < 2; ++yb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) accZ[yb][nb] = f4{0.f, 0.f, 0.f, 0.f};

    // The G copies' per-lane source offsets do not depend on the chunk: they
    // are formed once (wave w copies the 64-unit groups w, w + 4, ...).
    constexpr int NBI = (BU / 64 + 3) / 4, NGI = (GU / 64 + 3) / 4;
    int grow[NGI], gcol[NGI];
#pragma unroll
    for (int t = 0; t < NGI; ++t) {
        const int U = 64 * (wave + 4 * t) + lane;
        const int row = U / 9, c4 = U - (U / 9) * 9;
        const bool data = U < 288 && c4 < 8;
        grow[t] = min(y0 + (data ? row : 0), N - 1) * N;
        gcol[t] = data ? 4 * c4 : 0;
    }
    // B3 operands of chunk c (contiguous in the fragment-ordered table) into tile bb
    auto copy_b = [&](int c, int bb) {
        const float *src = tba + (size_t)c * BU * 4;
#pragma unroll
        for (int t = 0; t < NBI; ++t)
            if (wave + 4 * t < BU / 64)
                ilt_dev::lds_dma16(src + (size_t)(64 * (wave + 4 * t) + lane) * 4, &Bs[bb][256 * (wave + 4 * t)]);
    };
    // G rows y0.., columns x0.. into tile bb, coordinates clamped into the image
    auto copy_g = [&](int c, int bb) {
        const int x0 = c * 32;
#pragma unroll
        for (int t = 0; t < NGI; ++t)
            if (wave + 4 * t < GU / 64)
                ilt_dev::lds_dma16(Gsrc + grow[t] + min(x0 + gcol[t], N - 4), &Gs[bb][256 * (wave + 4 * t)]);
    };
    // N % 4 != 0: G staged through registers, 4 values per thread
    float gr[4];
    auto load_g_regs = [&](int c) {
        const int x0 = c * 32;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int e = threadIdx.x + 256 * v;
            const int gy = y0 + (e >> 5), gx = x0 + (e & 31);
            gr[v] = (gy < N && gx < N) ? Gsrc[(size_t)gy * N + gx] : 0.f;
        }
    };
    auto store_g_regs = [&](int bb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int e = threadIdx.x + 256 * v;
            Gs[bb][(e >> 5) * 36 + (e & 31)] = gr[v];
        }
    };
    auto load_half = [&](int c, int xb, f4 (&e_)[2][2]) {
#pragma unroll
        for (int yb = 0; yb < 2; ++yb) {
            const float *src = Ej + (((size_t)(ytile * 2 + yb) * NB16) + (c * 2 + xb)) * 512 + lane * 4;
            e_[yb][0] = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(src));
            e_[yb][1] = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(src + 256));
        }
    };
    // X = G . E for one 16-column half (G masked outside the image)
    auto form_x = [&](int c, int bb, int xb, const f4 (&e_)[2][2], f4 (&er)[2], f4 (&ei)[2]) {
        const int gx = c * 32 + 16 * xb + 4 * lq;
#pragma unroll
        for (int yb = 0; yb < 2; ++yb) {
            const float4 gv = *reinterpret_cast<const float4 *>(&Gs[bb][(16 * yb + l16) * 36 + 16 * xb + 4 * lq]);
            f4 g4 = f4{gv.x, gv.y, gv.z, gv.w};
            if (A4) {
                const bool rin = y0 + 16 * yb + l16 < N;
#pragma unroll
                for (int i = 0; i < 4; ++i) g4[i] = (rin && gx + i < N) ? g4[i] : 0.f;
            }
            er[yb] = e_[yb][0] * g4;
            ei[yb] = e_[yb][1] * g4;
        }
    };

    f4 ea[2][2], eb[2][2];
    if (c_begin < c_end) {
        copy_b(c_begin, 0);
        if (A4) copy_g(c_begin, 0);
        else {
            load_g_regs(c_begin);
            store_g_regs(0);
        }
        if (jok) load_half(c_begin, 0, ea);
    }
    ilt_dev::wait_copies();
    __syncthreads();
    for (int c = c_begin; c < c_end; ++c) {
        const int bb = (c - c_begin) & 1;
        const bool more = c + 1 < c_end;
        if (jok) load_half(c, 1, eb);
        if (jok) {
            f4 er[2], ei[2];
            form_x(c, bb, 0, ea, er, ei);
            ilt_dev::adjoint_rows_frag<NB>(accZ, er, ei, &Bs[bb][0], 0, lane);
        }
        f4 er[2], ei[2];
        if (jok) form_x(c, bb, 1, eb, er, ei);
        ilt_dev::wait_copies();                        // eb has landed; nothing issued later is waited for
        if (more) {
            copy_b(c + 1, bb ^ 1);
            if (A4) copy_g(c + 1, bb ^ 1);
            else load_g_regs(c + 1);
            if (jok) load_half(c + 1, 0, ea);
        }
        if (jok) ilt_dev::adjoint_rows_frag<NB>(accZ, er, ei, &Bs[bb][0], 1, lane);
        if (!A4 && more) store_g_regs(bb ^ 1);
        ilt_dev::wait_copies();
        __syncthreads();
    }
    float *dst = Wpart + ((size_t)(srel * gridDim.x + ytile) * gridDim.y + blockIdx.y) * P * P * 2;
    ilt_dev::adjoint_tail<FB, MIX>(accZ, jok, j, s, K, P, Np, AP, y0, ta4, coef, Ws, dst);
}

// --------------------------------------------------------------------------
// Adjoint with the fields recomputed (no field store; half the matrix-core
// throughput of the stored form but no N^2 K workspace):
//   (a) E^T chunk = Y_j^T L^T     (A-operand streamed from Y_j, B in registers)
//   (b) X = G . E                 (G tile staged in LDS)
//   (c) Z += X B3                 then the shared tail.
// --------------------------------------------------------------------------
template <int KP, int FB, int MIX>
__global__ __launch_bounds__(256, 2) void k_adjoint_rc(const float *__restrict__ tl, const float *__restrict__ tb,
                                                    const float *__restrict__ ta4, const float *__restrict__ Y,
                                                    const float *__restrict__ G, size_t g_set_stride,
                                                    const float2 *__restrict__ coef, int K, int P, int N, int Np,
                                                    int AP, int set_lo, float *__restrict__ Wpart, int zs,
                                                    size_t y_cs, size_t g_cs, size_t wp_cs) {
    constexpr int NZ = 32 * FB + 16 * MIX, NB = NZ / 16, KS = KP / 4;
    constexpr int LDB = NZ + 4;
    __shared__ float Gs[32][33];
    __shared__ float Bs[2][32][LDB];
    __shared__ float2 Ws[ILT_MAX_P * ILT_MAX_P];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    // grid.z = clips x sets; every clip has its own Y, G and partials
    const int clip = blockIdx.z / zs;
    Y += clip * y_cs;
    G += clip * g_cs;
    Wpart += clip * wp_cs;
    const int ytile = blockIdx.x, kg = blockIdx.y, srel = blockIdx.z - clip * zs, s = set_lo + srel;
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
            *reinterpret_cast<float4 *>(&Bs[part][xx][c4]) =
                *reinterpret_cast<const float4 *>(tb + ((size_t)part * Np + x0 + xx) * NZ + c4);
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
#pragma unroll
                for (int yb = 0; yb < 2; ++yb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float gv = Gs[16 * yb + l16][16 * xb + 4 * lq + i];
                        er[yb][i] *= gv;
                        ei[yb][i] *= gv;
                    }
                ilt_dev::adjoint_rows<NB>(accZ, er, ei, &Bs[0][0][0], &Bs[1][0][0], LDB, xb, lq, l16);
            }
        }
        __syncthreads();
    }
    float *dst = Wpart + ((size_t)(srel * gridDim.x + ytile) * gridDim.y + kg) * P * P * 2;
    ilt_dev::adjoint_tail<FB, MIX>(accZ, jok, j, s, K, P, Np, AP, y0, ta4, coef, Ws, dst);
}

// --------------------------------------------------------------------------
// G-window adjoint (exact): with U_k = H_k . S on the window and Ghat the
// DFT of G at the difference frequencies D in [-(P-1), P-1]^2,
//   V_k(f') = sum_f U_k(f) Ghat(f' - f),
//   W = sum over (set, k) of (w_k / N^4) conj(H_k(f')) V_k(f').
// All kernels of a set share Ghat, so the correlation is one GEMM per set,
// V[f'][k] = sum_f T[f'][f] U[f][k], with the Toeplitz-block-Toeplitz
// T[f'][f] = Ghat(a' - a, b' - b) read from Ghat in LDS, on the FP32 matrix
// cores (the precision of the field adjoint); partial sums over ranges of f,
// the weighting by conj(H_k) and the sums over k and sets are FP64.  U holds
// real and imaginary parts as separate columns, so the complex product is
// two real products per operand pair.
// --------------------------------------------------------------------------

// U operand: row f of the window (row-major, zero rows up to Fpad, a
// multiple of 4), columns [Re U_0 .. Re U_{K-1} | Im U_0 .. Im U_{K-1} | 0]
// (NC = 2K rounded up to 16).
__global__ __launch_bounds__(256) void k_gwindow_U(const float2 *__restrict__ H, const float2 *__restrict__ S, int P,
                                                   int K, int NC, int Fpad, int set_lo, float *__restrict__ U) {
    const int srel = blockIdx.y, s = set_lo + srel;
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= Fpad * NC) return;
    const int f = id / NC, col = id - (id / NC) * NC;
    double v = 0.0;
    if (f < P * P && col < 2 * K) {
        const int k = col < K ? col : col - K;
        const float2 h = H[((size_t)s * K + k) * P * P + f], sv = S[f];
        v = col < K ? (double)h.x * sv.x - (double)h.y * sv.y : (double)h.x * sv.y + (double)h.y * sv.x;
    }
    U[(size_t)srel * Fpad * NC + id] = (float)v;
}

// --------------------------------------------------------------------------
// Image spectrum on the difference window, the TCC form of the SOCS sum:
//   Ihat[D] = sum_k sw_k^2 sum_f U_k[f + D] conj(U_k[f]),  U_k = H_k . S,
// D = (Da, Db) in [-(P-1), P-1]^2 (stored at D + P - 1), sw_k^2 = w_k / N^4,
// so that I(r) = sum_D Ihat[D] exp(+2 pi i D.r / N) is the SOCS image.
// Ihat[-D] = conj(Ihat[D]) (I is real), so only the rows Da >= 0 are formed
// (the image uses them alone).  Block = (pair of rows Da and P - 1 - Da,
// kernel k, set), so that every block sums P + 1 window rows whatever Da
// (the middle row of an odd P is alone).  The work items (Da, window row a,
// column pair Db = 2 j - (P-1) and the next one) are spread over all 256
// threads; U_k sits in LDS with P - 1 zero columns on each side, so that
// every shifted read is in range and the items run the same loop, the
// shifted factor sliding along the row in registers.  Each item's products
// (P terms per column) are summed in FP32 and kept in registers until U
// is read no more, then stored in U's place in LDS (29 KB per block, five
// blocks per CU); the rows of a column are then summed in FP64 in the
// order a = 0, 1, ..., and the kernels' partials in FP64 afterwards, in a
// fixed order.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_hopkins_ihat(const float2 *__restrict__ H, const float2 *__restrict__ S,
                                                      const float *__restrict__ sw, int P, int K, int set_lo,
                                                      double2 *__restrict__ part) {
    constexpr int WMAX = 3 * ILT_MAX_P - 1, NI = (ILT_MAX_P + 1) * ILT_MAX_P, NQ = (NI + 255) / 256;
    static_assert(2 * NI <= ILT_MAX_P * WMAX, "the item sums must fit in the U storage");
    __shared__ float4 L4[(ILT_MAX_P * WMAX + 1) / 2];
    float2 *U = reinterpret_cast<float2 *>(L4);
    float4 *R = L4;                                        // after U: [item row][pair], (re, im) of both columns
    const int Q = 2 * P - 1, PP = P * P, W = 3 * P - 1;    // one more zero column for the pair's second
    const int k = blockIdx.y, srel = blockIdx.z, s = set_lo + srel;
    const int da0 = blockIdx.x, da1 = P - 1 - blockIdx.x;  // da1 >= da0 (grid.x = ceil(P / 2))
    const int n0 = P - da0, n1 = da1 > da0 ? P - da1 : 0;  // window rows of each Da
    for (int e = threadIdx.x; e < P * W; e += 256) U[e] = make_float2(0.f, 0.f);
    __syncthreads();
    const float2 *Hk = H + ((size_t)s * K + k) * PP;
    for (int f = threadIdx.x; f < PP; f += 256) {
        const int a = f / P, b = f - (f / P) * P;
        const float2 h = Hk[f], sv = S[f];
        U[a * W + (P - 1) + b] = make_float2(h.x * sv.x - h.y * sv.y, h.x * sv.y + h.y * sv.x);
    }
    __syncthreads();
    // item i = r P + j: r < n0 is window row a = r of Da = da0, else a = r - n0
    // of da1; columns t0 = 2 j, t0 + 1 (index Db + P - 1), whose read of
    // U[a + Da][b + Db] is at column b + t0 of the padded row
    float4 acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = (int)threadIdx.x + 256 * q;
        if (i >= (n0 + n1) * P) break;
        const int r = i / P, j = i - (i / P) * P;
        const int a = r < n0 ? r : r - n0, da = r < n0 ? da0 : da1, t0 = 2 * j;
        const float2 *xs = &U[(a + da) * W + t0], *ys = &U[a * W + (P - 1)];
        float re0 = 0.f, im0 = 0.f, re1 = 0.f, im1 = 0.f;
        float2 x0 = xs[0];
        for (int b = 0; b < P; ++b) {
            const float2 x1 = xs[b + 1], y = ys[b];        // x conj(y)
            re0 = fmaf(x0.x, y.x, fmaf(x0.y, y.y, re0));
            im0 = fmaf(x0.y, y.x, fmaf(-x0.x, y.y, im0));
            re1 = fmaf(x1.x, y.x, fmaf(x1.y, y.y, re1));
            im1 = fmaf(x1.y, y.x, fmaf(-x1.x, y.y, im1));
            x0 = x1;
        }
        acc[q] = make_float4(re0, im0, re1, im1);
    }
    __syncthreads();                                       // U is read no more
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = (int)threadIdx.x + 256 * q;
        if (i < (n0 + n1) * P) R[i] = acc[q];
    }
    __syncthreads();
    const int t = threadIdx.x < Q ? threadIdx.x : threadIdx.x - Q, half = threadIdx.x < Q ? 0 : 1;
    if (threadIdx.x >= 2 * Q || (half && n1 == 0)) return;
    const int r0 = half ? n0 : 0, nr = half ? n1 : n0, j = t >> 1;
    double re = 0.0, im = 0.0;
    for (int a = 0; a < nr; ++a) {
        const float4 v = R[(r0 + a) * P + j];
        re += (double)(t & 1 ? v.z : v.x);
        im += (double)(t & 1 ? v.w : v.y);
    }
    const double w2 = (double)sw[(size_t)s * K + k] * (double)sw[(size_t)s * K + k];
    part[(((size_t)srel * K + k) * P + (half ? da1 : da0)) * Q + t] = make_double2(w2 * re, w2 * im);
}

// Block-wide copy global -> LDS with UNR independent loads in flight per
// thread (a plain copy loop waits for each load before the next).
template <int UNR, typename T>
__device__ __forceinline__ void stage_to_lds(T *dst, const T *__restrict__ src, int n) {
    for (int base = 0; base < n; base += 256 * UNR) {
        T v[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int e = base + u * 256 + (int)threadIdx.x;
            if (e < n) v[u] = src[e];
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int e = base + u * 256 + (int)threadIdx.x;
            if (e < n) dst[e] = v[u];
        }
    }
}

// Block: 4 waves, wave w = a 16-row tile of f' (v_mfma_f32_16x16x4: lane l
// holds A[l%16][l/16], B[l/16][l%16] and C[4(l/16) + i][l%16] in item i).
// grid.y splits the sum over f into ranges of 4-row chunks whose rows of U
// are staged in LDS after Ghat (the host sizes the ranges to fit), grid.z =
// set.  Epilogue: V_re = T_re U_re - T_im U_im, V_im = T_re U_im + T_im U_re,
// times (w_k / N^4) conj(H_k(f')), summed over k in a fixed order ->
// Wpart[range][set][f'].
template <int NT>
__global__ __launch_bounds__(256) void k_gwindow_mm(const float2 *__restrict__ Ghat, const float *__restrict__ U,
                                                    const float2 *__restrict__ H, const float *__restrict__ sw, int P,
                                                    int K, int Fpad, int set_lo, double2 *__restrict__ Wpart) {
    constexpr int NC = 16 * NT;
    constexpr int SMEM = GWIN_LDS_FLOATS;                   // 64 KB
    constexpr int WPR = (SMEM / (32 * NC)) < 4 ? SMEM / (32 * NC) : 4;   // epilogue waves per round
    static_assert(2 * (2 * ILT_MAX_P - 1) * (2 * ILT_MAX_P - 1) + 4 * 16 * 8 <= SMEM,
                  "Ghat and one chunk of U do not fit");
    static_assert(WPR >= 1, "epilogue tile does not fit");
    __shared__ float smem[SMEM];
    const int srel = blockIdx.z, s = set_lo + srel, Q = 2 * P - 1, PP = P * P;
    float2 *Gs = reinterpret_cast<float2 *>(smem);
    stage_to_lds<10>(Gs, Ghat + (size_t)s * Q * Q, Q * Q);
    const int nchunk = Fpad / 4, per = (nchunk + gridDim.y - 1) / gridDim.y;
    const int t0 = blockIdx.y * per, t1 = min(nchunk, t0 + per);
    float *Us = smem + 2 * Q * Q;
    stage_to_lds<12>(Us, U + ((size_t)srel * Fpad + 4 * t0) * NC, (t1 > t0 ? t1 - t0 : 0) * 4 * NC);
    __syncthreads();

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, kq = lane >> 4;
    const int m0 = (blockIdx.x * 4 + w) * 16;
    const int fp = m0 + r;
    const bool fp_ok = fp < PP;
    const int a2 = fp_ok ? fp / P : 0, b2 = fp_ok ? fp - (fp / P) * P : 0;

    // the epilogue's conj(H_k(f')) and weights, fetched before the main loop
    // (lane: row rr of the tile, kernels k = q, q + 4, ...; K <= 8 NT)
    const int rr = lane >> 2, q = lane & 3, fo = m0 + rr;
    float2 hv[2 * NT];
    float sv[2 * NT];
#pragma unroll
    for (int u = 0; u < 2 * NT; ++u) {
        const int k = q + 4 * u;
        hv[u] = make_float2(0.f, 0.f);
        sv[u] = 0.f;
        if (fo < PP && k < K) {
            hv[u] = H[((size_t)s * K + k) * PP + fo];
            sv[u] = sw[(size_t)s * K + k];
        }
    }

    f4 pre[NT], pim[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) pre[j] = pim[j] = f4{0.f, 0.f, 0.f, 0.f};
    if (m0 < PP && t0 < t1) {                               // wave-uniform
        int f = 4 * t0 + kq, a = f / P, b = f - (f / P) * P;
        const float *urow = Us + kq * NC + r;
        for (int t = t0; t < t1; ++t) {
            float2 g = make_float2(0.f, 0.f);
            if (fp_ok && f < PP) g = Gs[(a2 - a + P - 1) * Q + (b2 - b + P - 1)];
            float bv[NT];
#pragma unroll
            for (int j = 0; j < NT; ++j) bv[j] = urow[16 * j];
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                pre[j] = mfma4(g.x, bv[j], pre[j]);
                pim[j] = mfma4(g.y, bv[j], pim[j]);
            }
            f += 4;
            urow += 4 * NC;
            b += 4;
            while (b >= P) {
                b -= P;
                ++a;
            }
        }
    }
    __syncthreads();                                        // LDS free again

    // epilogue in rounds of WPR waves: E[row][col][re-part, im-part]
    for (int w0 = 0; w0 < 4; w0 += WPR) {
        float *E = smem + (size_t)(w - w0) * 32 * NC;
        const bool mine = w >= w0 && w < w0 + WPR;
        if (mine) {
#pragma unroll
            for (int j = 0; j < NT; ++j) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    *reinterpret_cast<float2 *>(E + ((4 * kq + i) * NC + 16 * j + r) * 2) = make_float2(pre[j][i], pim[j][i]);
            }
        }
        __syncthreads();
        if (mine) {
            double wr = 0.0, wi = 0.0;
            if (fo < PP) {
                const float *er = E + rr * NC * 2;
#pragma unroll
                for (int u = 0; u < 2 * NT; ++u) {
                    const int k = q + 4 * u;
                    if (k < K) {
                        const double vre = (double)er[2 * k] - (double)er[2 * (K + k) + 1];
                        const double vim = (double)er[2 * (K + k)] + (double)er[2 * k + 1];
                        const double sc = (double)sv[u] * (double)sv[u];
                        wr += sc * ((double)hv[u].x * vre + (double)hv[u].y * vim);
                        wi += sc * ((double)hv[u].x * vim - (double)hv[u].y * vre);
                    }
                }
            }
            wr += __shfl_xor(wr, 1, 64);
            wi += __shfl_xor(wi, 1, 64);
            wr += __shfl_xor(wr, 2, 64);
            wi += __shfl_xor(wi, 2, 64);
            if (q == 0 && fo < PP)
                Wpart[((size_t)blockIdx.y * gridDim.z + srel) * PP + fo] = make_double2(wr, wi);
        }
        __syncthreads();
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers

// Pruned spectrum of src (or of [src <= 0]) on a window of side Pw with the
// given column tables, summed into out [Pw][Pw].
static hipError_t spectrum_to(ilt_ctx *c, const float *src, int src_is_phi, int FBw, int MIXw, const float *tbw,
                              const float *arw, const float *aiw, int PRw, int Pw, float2 *out, int nimg = 1,
                              size_t src_stride = 0, int xs_nimg = 0) {
    // xs_nimg: the image count whose column split to use (0: nimg); the
    // clips of one sequence keep the single-image split, so that each
    // clip's sums group exactly as in a solve of that clip alone
    const int nband = c->Np / 16;
    const int xs = spectrum_xsplit(c, xs_nimg > 0 ? xs_nimg : nimg);
#define SPEC(FB_, MIX_)                                                                                    \
    k_spectrum_band<FB_, MIX_><<<dim3(nband, xs, nimg), 512, 0, c->stream>>>(src, src_stride, src_is_phi, tbw, \
                                                                            arw, aiw, PRw, Pw, c->N, c->Np, c->Spart)
    if (FBw == 0 && MIXw == 1) SPEC(0, 1);
    else if (FBw == 1 && MIXw == 0) SPEC(1, 0);
    else if (FBw == 1 && MIXw == 1) SPEC(1, 1);
    else if (FBw == 2 && MIXw == 0) SPEC(2, 0);
    else if (FBw == 2 && MIXw == 1) SPEC(2, 1);
    else if (FBw == 3 && MIXw == 0) SPEC(3, 0);
    else if (FBw == 3 && MIXw == 1) SPEC(3, 1);
    else if (FBw == 4 && MIXw == 0) SPEC(4, 0);
    else if (FBw == 4 && MIXw == 1) SPEC(4, 1);
    else return hipErrorInvalidValue;
#undef SPEC
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int n = PRw * Pw;
    k_psum<float2><<<dim3((n + 15) / 16, nimg), 1024, 0, c->stream>>>(c->Spart, nband * xs, n, out);
    return hipGetLastError();
}

// Spectrum of a real image on the (2P-1)^2 difference window from its
// columns Db >= 0 (half [img][Q][P]): S(Da, Db) = conj(S(-Da, -Db)).
__global__ __launch_bounds__(128) void k_conj_fill(const float2 *__restrict__ half, int P, float2 *__restrict__ full) {
    const int Q = 2 * P - 1, r = blockIdx.x, cix = threadIdx.x;
    if (cix >= Q) return;
    const float2 *h = half + (size_t)blockIdx.y * Q * P;
    float2 v;
    if (cix >= P - 1) {
        v = h[(size_t)r * P + (cix - (P - 1))];
    } else {
        v = h[(size_t)(Q - 1 - r) * P + (Q - 1 - cix - (P - 1))];
        v.y = -v.y;
    }
    full[(size_t)blockIdx.y * Q * Q + (size_t)r * Q + cix] = v;
}

hipError_t launch_spectrum(ilt_ctx *c, const float *src, int src_is_phi) {
    return spectrum_to(c, src, src_is_phi, c->FB, c->MIX, c->tbs, c->ar, c->ai, c->P, c->P, c->S, c->ncur,
                       cs_npix(c), 1);
}

hipError_t launch_make_Y(ilt_ctx *c, int set_lo, int set_hi) {
    const int zs = set_hi - set_lo;
    dim3 grid(c->Np / 128, c->K, zs * c->ncur);
    const size_t scs = (size_t)c->P * c->P, ycs = cs_y(c);
    // the split-BF16 form reads only the split rows, written here directly
    const bool split = c->precision == ILT_BF16X3;
    switch (c->KP) {
#define MKY(KP_)                                                                                               \
    case KP_:                                                                                                  \
        if (split)                                                                                             \
            k_make_y<KP_, true><<<grid, 256, 0, c->stream>>>(c->H, c->S, c->sw, c->tl, c->P, c->Np, c->K, set_lo, \
                                                             nullptr, c->Yhl, zs, scs, ycs);                   \
        else                                                                                                   \
            k_make_y<KP_, false><<<grid, 256, 0, c->stream>>>(c->H, c->S, c->sw, c->tl, c->P, c->Np, c->K,      \
                                                              set_lo, c->Y, nullptr, zs, scs, ycs);            \
        break;
        MKY(8) MKY(24) MKY(40) MKY(72)
#undef MKY
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// y_cs, out_cs: the clip strides of Y and out; maxima and fields step by the
// clip's partials and field store
template <int MODE, bool STORE>
static hipError_t image_dispatch(ilt_ctx *c, const float *Y, int nj, int set_lo, int nsets, float *out,
                                 double *maxpart, size_t y_cs, size_t out_cs) {
    dim3 grid(c->Np / 64, c->Np / 128, nsets * c->ncur);
    const size_t mcs = (size_t)c->n_part, ecs = cs_est(c);
    switch (c->KP) {
#define IMG(KP_) case KP_: k_image<KP_, MODE, STORE><<<grid, 256, 0, c->stream>>>(c->tl, Y, nj, c->N, c->Np, set_lo, out, maxpart, c->Est, nsets, y_cs, out_cs, mcs, ecs); break;
        IMG(8) IMG(24) IMG(40) IMG(72)
#undef IMG
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_image_to(ilt_ctx *c, int set_lo, int set_hi, float *out, int store_fields) {
    // out: the sets' images of the first clip; clips step by n_sets images
    const size_t ocs = (size_t)c->n_sets * cs_npix(c);
    if (store_fields && c->Est)
        return image_dispatch<0, true>(c, c->Y, c->K, set_lo, set_hi - set_lo, out, nullptr, cs_y(c), ocs);
    return image_dispatch<0, false>(c, c->Y, c->K, set_lo, set_hi - set_lo, out, nullptr, cs_y(c), ocs);
}

hipError_t launch_adjoint(ilt_ctx *c, const float *G, size_t g_set_stride, int set_lo, int set_hi, int fields_stored) {
    // grid.z = clips x sets; G steps by n_sets images per clip, the W
    // partials by the clip's share
    const int zs = set_hi - set_lo;
    dim3 grid((c->N + 31) / 32, (c->K + 3) / 4, zs * c->ncur);
    const size_t gcs = (size_t)c->n_sets * cs_npix(c);
    if (fields_stored) {
        if (!c->Est) return hipErrorInvalidValue;
        grid.y *= adjoint_st_xsplit(c);
        const size_t wcs = (size_t)grid.x * grid.y * zs * c->P * c->P * 2;
        if (wcs * c->ncur > (size_t)c->n_wpart * c->nb) return hipErrorInvalidValue;
#define ADJS(FB_, MIX_)                                                                                        \
    do {                                                                                                        \
        if ((c->N & 3) == 0 && (reinterpret_cast<uintptr_t>(G) & 15) == 0)                                     \
            k_adjoint_st<FB_, MIX_, true><<<grid, 256, 0, c->stream>>>(c->tba, c->ta4, c->Est, G, g_set_stride,   \
                                                                      c->coef, c->K, c->P, c->N, c->Np, c->AP, \
                                                                      set_lo, c->Wpart, zs, cs_est(c), gcs, wcs); \
        else                                                                                                    \
            k_adjoint_st<FB_, MIX_, false><<<grid, 256, 0, c->stream>>>(c->tba, c->ta4, c->Est, G, g_set_stride,  \
                                                                       c->coef, c->K, c->P, c->N, c->Np, c->AP, \
                                                                       set_lo, c->Wpart, zs, cs_est(c), gcs, wcs); \
    } while (0)
        if (c->FB == 0 && c->MIX == 1) ADJS(0, 1);
        else if (c->FB == 1 && c->MIX == 0) ADJS(1, 0);
        else if (c->FB == 1 && c->MIX == 1) ADJS(1, 1);
        else if (c->FB == 2 && c->MIX == 0) ADJS(2, 0);
        else if (c->FB == 2 && c->MIX == 1) ADJS(2, 1);
        else return hipErrorInvalidValue;
#undef ADJS
        return hipGetLastError();
    }
    const size_t wcs = (size_t)grid.x * grid.y * zs * c->P * c->P * 2;
    if (wcs * c->ncur > (size_t)c->n_wpart * c->nb) return hipErrorInvalidValue;
#define ADJ(KP_, FB_, MIX_)                                                                                 \
    k_adjoint_rc<KP_, FB_, MIX_><<<grid, 256, 0, c->stream>>>(c->tl, c->tb, c->ta4, c->Y, G, g_set_stride,  \
                                                              c->coef, c->K, c->P, c->N, c->Np, c->AP, set_lo, \
                                                              c->Wpart, zs, cs_y(c), gcs, wcs)
    const int KPv = c->KP, FBv = c->FB, MIXv = c->MIX;
    if (KPv == 8 && FBv == 0 && MIXv == 1) ADJ(8, 0, 1);
    else if (KPv == 24 && FBv == 0 && MIXv == 1) ADJ(24, 0, 1);
    else if (KPv == 24 && FBv == 1 && MIXv == 0) ADJ(24, 1, 0);
    else if (KPv == 40 && FBv == 1 && MIXv == 0) ADJ(40, 1, 0);
    else if (KPv == 40 && FBv == 1 && MIXv == 1) ADJ(40, 1, 1);
    else if (KPv == 72 && FBv == 1 && MIXv == 1) ADJ(72, 1, 1);
    else if (KPv == 72 && FBv == 2 && MIXv == 0) ADJ(72, 2, 0);
    else if (KPv == 72 && FBv == 2 && MIXv == 1) ADJ(72, 2, 1);
    else return hipErrorInvalidValue;
#undef ADJ
    return hipGetLastError();
}

hipError_t launch_window_sum(ilt_ctx *c, int set_lo, int set_hi) {
    const int nparts = c->precision == ILT_BF16X3 ? adjoint_b3_parts(c, set_hi - set_lo)
                                                  : adjoint_fp32_parts(c, set_hi - set_lo);
    const int n = c->P * c->P;
    // one sum per clip (the clips' partials lie one after another)
    k_psum<float2><<<dim3((n + 15) / 16, c->ncur), 1024, 0, c->stream>>>(
        reinterpret_cast<const float2 *>(c->Wpart), nparts, n, c->W);
    return hipGetLastError();
}

hipError_t launch_gradient(ilt_ctx *c, float *g_out, double *maxpart) {
    // Tg = 2 W conj(A) in the row layout, then g = Re(A^H Tg)
    // one transform only: narrow column tiles so that the launch covers the chip
    dim3 grid(c->Np / 16, 1, c->ncur);
    k_window_rows<16, 1><<<grid, 256, 0, c->stream>>>(nullptr, c->W, nullptr, 2.f, c->ar, c->ai, c->P, c->P, c->KP, c->Np,
                                                      1, 0, c->Tg, 1, (size_t)c->P * c->P, cs_tg(c));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return image_dispatch<1, false>(c, c->Tg, 1, 0, 1, g_out, maxpart, cs_tg(c), cs_npix(c));
}

// TCC-form image (ILT_FLAG_HOPKINS_FORWARD): the sets' spectra on the rows
// Da >= 0 of the difference window, then for each set its window rows
// R = Ihat conj(A_Q) over those rows and the image
//   I = Re R_0 + 2 Re sum_{Da > 0} exp(+2 pi i Da y / N) R_Da,
// since R_{-Da} = conj(R_Da) (Ihat(-D) = conj(Ihat(D))): the image-side
// table tlH holds the rows Da >= 0 with the factor 2, so the image kernel
// contracts 2P rows, not 2(2P-1) (a set's rows are one window slice of the
// row kernel and one image of the image kernel).
hipError_t launch_hopkins_spectrum(ilt_ctx *c, int set_lo, int set_hi) {
    if (!c->hop) return hipErrorInvalidValue;
    const int P = c->P, Q = c->Q, ns = set_hi - set_lo;
    k_hopkins_ihat<<<dim3((P + 1) / 2, c->K, ns), 256, 0, c->stream>>>(c->H, c->S, c->sw, P, c->K, set_lo, c->Ipart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_psum<double2><<<dim3((P * Q + 15) / 16, ns), 1024, 0, c->stream>>>(c->Ipart, c->K, P * Q, c->Ihat);
    return hipGetLastError();
}

hipError_t launch_hopkins_image(ilt_ctx *c, int set_lo, int set_hi, float *out) {
    if (!c->hop) return hipErrorInvalidValue;
    const int P = c->P, Q = c->Q, ns = set_hi - set_lo;
    (void)set_lo;
    k_window_rows<16, 1, 2 * ILT_MAX_P - 1><<<dim3(c->Np / 16, 1, ns), 256, 0, c->stream>>>(
        nullptr, c->Ihat, nullptr, 1.f, c->arQ, c->aiQ, Q, P,
        c->KP, c->Np, 1, 0, c->Tq, 1, (size_t)P * Q, (size_t)c->KP * c->Np);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid(c->Np / 64, c->Np / 128, ns);
    switch (c->KP) {
#define HIMG(KP_) case KP_: k_image<KP_, 2, false><<<grid, 256, 0, c->stream>>>(c->tlQ, c->Tq, 1, c->N, c->Np, 0, out, nullptr, nullptr, ns, 0, 0, 0, 0); break;
        HIMG(8) HIMG(24) HIMG(40) HIMG(72)
#undef HIMG
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_gwindow(ilt_ctx *c, const float *G, size_t g_set_stride, int set_lo, int set_hi) {
    if (!c->gwin) return hipErrorInvalidValue;
    const int Q = c->Q;
    // the spectra of every set's G in one launch (one pass over the tables)
    {
        // the columns f >= 0 (the layout of P), then the others by symmetry
        hipError_t e = spectrum_to(c, G + (size_t)set_lo * g_set_stride, 0, c->FB, c->MIX, c->tbQ, c->arQ, c->aiQ,
                                   Q, c->P, c->Ghalf + (size_t)set_lo * Q * c->P, set_hi - set_lo, g_set_stride);
        if (e != hipSuccess) return e;
        k_conj_fill<<<dim3(Q, set_hi - set_lo), 128, 0, c->stream>>>(c->Ghalf + (size_t)set_lo * Q * c->P, c->P,
                                                                     c->Ghat + (size_t)set_lo * Q * Q);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int n = c->P * c->P, ns = set_hi - set_lo, NT = gwin_ntiles(c->K), NC = 16 * NT;
    const int Fpad = (n + 3) / 4 * 4;
    k_gwindow_U<<<dim3((Fpad * NC + 255) / 256, ns), 256, 0, c->stream>>>(c->H, c->S, c->P, c->K, NC, Fpad, set_lo,
                                                                         c->Ugw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((gwin_ftiles(c->P) + 3) / 4, c->gw_groups, ns);
    switch (NT) {
#define GWMM(NT_)                                                                                              \
    case NT_:                                                                                                  \
        k_gwindow_mm<NT_><<<grid, 256, 0, c->stream>>>(c->Ghat, c->Ugw, c->H, c->sw, c->P, c->K, Fpad, set_lo, \
                                                      c->Vpart);                                               \
        break;
        GWMM(1) GWMM(2) GWMM(3) GWMM(4) GWMM(5) GWMM(6) GWMM(7) GWMM(8)
#undef GWMM
    default: return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_psum<double2><<<(n + 15) / 16, 1024, 0, c->stream>>>(c->Vpart, c->gw_groups * ns, n, c->W);
    return hipGetLastError();
}
