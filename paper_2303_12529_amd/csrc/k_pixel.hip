// Pixel-wise kernels: resist and loss, reductions, the level-set step and the
// exact squared EDT.  All reductions are two-stage with a fixed order (block
// partials, then one block), so results are bitwise reproducible.
#include <algorithm>
#include <cmath>

#include "ilt_internal.h"

namespace {

constexpr int RB = 256;           // threads per reduction block
constexpr int MAX_RBLK = 2048;    // cap on reduction blocks

static_assert(RB == 256, "block reductions combine four waves");

// Block reductions in a fixed order: a shuffle tree inside each wave, then
// the four wave results in wave order; every thread receives the result.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return r;
}

// Per-thread sums over the partials b = threadIdx.x, +RB, ... (NQ values per
// partial), with the loads of UNR partials in flight at a time; the additions
// happen in the order of the plain strided loop, so the sums are the same.
template <int NQ, int UNR>
__device__ __forceinline__ void thread_partial_sums(const double *__restrict__ part, int nblk, double (&v)[NQ]) {
    for (int b0 = threadIdx.x; b0 < nblk; b0 += RB * UNR) {
        double t[UNR][NQ];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int b = b0 + RB * u;
#pragma unroll
            for (int q = 0; q < NQ; ++q) t[u][q] = b < nblk ? part[(size_t)b * NQ + q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u)
            if (b0 + RB * u < nblk) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) v[q] += t[u][q];
            }
    }
}

__device__ __forceinline__ double block_max(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    __syncthreads();
    return r;
}

// --------------------------------------------------------------------------
// Resist (Sec. III-A): per corner Z = 1/(1+exp(-sigma_z (d I_s - I_th))),
// loss += omega (Z - Zt)^2, G_s += omega 2 sigma_z d (Z - Zt) Z (1 - Z);
// binary print (Sec. II-B) for L2 (corner 0) and PVBand (corners 1, 2).
// Block b covers a contiguous pixel range; partials {loss, l2, pvb, nonfinite}.
// --------------------------------------------------------------------------
// One pixel of the resist: loss, G contributions and the print decisions.
// The sigmoid's reciprocal is the hardware one (1 ulp); print counts are
// integers per thread, the loss an FP64 sum.
//
// Corner layouts: CL = 0 any (corners' sets chosen at run time), CL = 1 one
// corner on set 0, CL = 2 three corners on sets 0, 0, 1 (nominal, outer,
// inner).  The fixed layouts index the sets at compile time.
constexpr int corner_count(int CL) { return CL == 1 ? 1 : CL == 2 ? 3 : 4; }
constexpr int corner_set(int CL, int c) { return CL == 2 ? (c == 2 ? 1 : 0) : 0; }

template <int CL>
__device__ __forceinline__ void resist_pixel(const resist_args &ra, float zt, const float (&ii)[ILT_MAX_SETS],
                                             float (&gs)[ILT_MAX_SETS], double &loss, unsigned &l2, unsigned &pvb,
                                             unsigned &bad) {
    float lp = 0.f;
    bool print[4] = {false, false, false, false};
#pragma unroll
    for (int q = 0; q < ILT_MAX_SETS; ++q) gs[q] = 0.f;
#pragma unroll
    for (int c = 0; c < corner_count(CL); ++c) {
        if (CL != 0 || c < ra.n_corners) {
            const float d = ra.dose[c];
            float iv = 0.f;
            if (CL != 0) {
                iv = ii[corner_set(CL, c)];
            } else {
#pragma unroll
                for (int q = 0; q < ILT_MAX_SETS; ++q)
                    if (q == ra.cset[c]) iv = ii[q];
            }
            const float di = d * iv;
            const float z = __builtin_amdgcn_rcpf(1.f + expf(-ra.sigma_z * (di - ra.i_th)));
            const float r = z - zt;
            lp = fmaf(ra.omega[c] * r, r, lp);
            const float gv = ra.omega[c] * 2.f * ra.sigma_z * d * r * (z * (1.f - z));
            if (CL != 0) {
                gs[corner_set(CL, c)] += gv;
            } else {
#pragma unroll
                for (int q = 0; q < ILT_MAX_SETS; ++q)
                    if (q == ra.cset[c]) gs[q] += gv;
            }
            print[c] = di >= ra.i_th;
        }
    }
    loss += (double)lp;
    bad += !isfinite(lp);
    l2 += print[0] != (zt != 0.f);
    if (CL == 2 || (CL == 0 && ra.n_corners >= 3)) pvb += print[1] != print[2];
}

// sets a corner layout reads
__device__ __forceinline__ bool layout_uses(int CL, const resist_args &ra, int q) {
    return CL == 1 ? q == 0 : CL == 2 ? q < 2 : ra.set_used[q] != 0;
}

// Four consecutive pixels per thread and step (16-byte loads and stores);
// block b covers quads [b chunk, (b + 1) chunk).  Needs npix % 4 == 0 (every
// set's image then starts 16-byte aligned).
template <int CL>
__global__ __launch_bounds__(RB) void k_resist4(const float *__restrict__ I, size_t set_stride,
                                               const uint8_t *__restrict__ target, resist_args ra,
                                               size_t npix, size_t chunk, float *__restrict__ G,
                                               double *__restrict__ part) {
    __shared__ double sh[RB];
    const size_t nq = npix / 4;
    const size_t lo = (size_t)blockIdx.x * chunk;
    const size_t hi = min(nq, lo + chunk);
    double loss = 0.0;
    unsigned l2 = 0, pvb = 0, bad = 0;
    // the loads of RU consecutive steps are issued together
    constexpr int RU = 4;
    for (size_t base = lo + threadIdx.x; base < hi; base += (size_t)RB * RU) {
      uchar4 tq[RU];
      float4 ivq[RU][ILT_MAX_SETS];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const size_t q4 = base + (size_t)u * RB;
        tq[u] = make_uchar4(0, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < ILT_MAX_SETS; ++q) ivq[u][q] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (q4 < hi) {
            tq[u] = *reinterpret_cast<const uchar4 *>(target + 4 * q4);
#pragma unroll
            for (int q = 0; q < ILT_MAX_SETS; ++q)
                if (layout_uses(CL, ra, q)) ivq[u][q] = *reinterpret_cast<const float4 *>(I + (size_t)q * set_stride + 4 * q4);
        }
      }
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const size_t q4 = base + (size_t)u * RB;
        if (q4 >= hi) break;
        const size_t p = 4 * q4;
        const uchar4 t4 = tq[u];
        const float4 (&iv)[ILT_MAX_SETS] = ivq[u];
        float g4[ILT_MAX_SETS][4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const unsigned char tb = e == 0 ? t4.x : e == 1 ? t4.y : e == 2 ? t4.z : t4.w;
            float ii[ILT_MAX_SETS], gs[ILT_MAX_SETS];
#pragma unroll
            for (int q = 0; q < ILT_MAX_SETS; ++q)
                ii[q] = e == 0 ? iv[q].x : e == 1 ? iv[q].y : e == 2 ? iv[q].z : iv[q].w;
            resist_pixel<CL>(ra, tb ? 1.f : 0.f, ii, gs, loss, l2, pvb, bad);
#pragma unroll
            for (int q = 0; q < ILT_MAX_SETS; ++q) g4[q][e] = gs[q];
        }
#pragma unroll
        for (int q = 0; q < ILT_MAX_SETS; ++q)
            if (layout_uses(CL, ra, q))
                *reinterpret_cast<float4 *>(G + (size_t)q * set_stride + p) =
                    make_float4(g4[q][0], g4[q][1], g4[q][2], g4[q][3]);
      }
    }
    loss = block_sum(loss, sh);
    const double l2s = block_sum((double)l2, sh);
    const double pvbs = block_sum((double)pvb, sh);
    const double bads = block_sum((double)bad, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 4 + 0] = loss;
        part[blockIdx.x * 4 + 1] = l2s;
        part[blockIdx.x * 4 + 2] = pvbs;
        part[blockIdx.x * 4 + 3] = bads;
    }
}

// Any npix: one pixel per thread and step; block b covers pixels
// [b chunk, (b + 1) chunk).
__global__ __launch_bounds__(RB) void k_resist1(const float *__restrict__ I, size_t set_stride,
                                                const uint8_t *__restrict__ target, resist_args ra,
                                                size_t npix, size_t chunk, float *__restrict__ G,
                                                double *__restrict__ part) {
    __shared__ double sh[RB];
    const size_t lo = (size_t)blockIdx.x * chunk;
    const size_t hi = min(npix, lo + chunk);
    double loss = 0.0;
    unsigned l2 = 0, pvb = 0, bad = 0;
    for (size_t p = lo + threadIdx.x; p < hi; p += RB) {
        float ii[ILT_MAX_SETS], gs[ILT_MAX_SETS];
#pragma unroll
        for (int q = 0; q < ILT_MAX_SETS; ++q) ii[q] = ra.set_used[q] ? I[(size_t)q * set_stride + p] : 0.f;
        resist_pixel<0>(ra, target[p] ? 1.f : 0.f, ii, gs, loss, l2, pvb, bad);
#pragma unroll
        for (int q = 0; q < ILT_MAX_SETS; ++q)
            if (ra.set_used[q]) G[(size_t)q * set_stride + p] = gs[q];
    }
    loss = block_sum(loss, sh);
    const double l2s = block_sum((double)l2, sh);
    const double pvbs = block_sum((double)pvb, sh);
    const double bads = block_sum((double)bad, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 4 + 0] = loss;
        part[blockIdx.x * 4 + 1] = l2s;
        part[blockIdx.x * 4 + 2] = pvbs;
        part[blockIdx.x * 4 + 3] = bads;
    }
}

__global__ __launch_bounds__(RB) void k_finish_resist(const double *__restrict__ part, int nblk,
                                                      double *__restrict__ scal, double *__restrict__ stats4) {
    __shared__ double sh[RB];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    thread_partial_sums<4, 8>(part, nblk, v);
    for (int q = 0; q < 4; ++q) v[q] = block_sum(v[q], sh);
    if (threadIdx.x == 0) {
        scal[SC_LOSS] = v[0];
        scal[SC_L2] = v[1];
        scal[SC_PVB] = v[2];
        scal[SC_NONFIN] = v[3];
        if (stats4)
            for (int q = 0; q < 4; ++q) stats4[q] = v[q];
    }
}

// max |v| per block (non-finite -> +inf)
__global__ __launch_bounds__(RB) void k_absmax(const float *__restrict__ v, size_t npix, size_t chunk,
                                               double *__restrict__ part) {
    __shared__ double sh[RB];
    const size_t lo = (size_t)blockIdx.x * chunk;
    const size_t hi = min(npix, lo + chunk);
    float m = 0.f;
    for (size_t p = lo + threadIdx.x; p < hi; p += RB) {
        const float x = v[p];
        m = (x != x) ? INFINITY : fmaxf(m, fabsf(x));
    }
    const double r = block_max((double)m, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// CFL time step (Sec. III-C): dt = eta / max|v|, capped at dt_max; or fixed.
__global__ __launch_bounds__(RB) void k_finish_dt(const double *__restrict__ part, int nblk, int dt_mode,
                                                  float eta, float dt_max, double *__restrict__ scal) {
    __shared__ double sh[RB];
    double m = 0.0;
    for (int b = threadIdx.x; b < nblk; b += RB) m = fmax(m, part[b]);
    m = block_max(m, sh);
    if (threadIdx.x == 0) {
        const float mv = (float)m;
        float dt;
        if (dt_mode == 1) {
            dt = eta;
        } else if (mv > 0.f && isfinite(mv)) {
            dt = eta / mv;
            if (dt_max > 0.f) dt = fminf(dt, dt_max);
        } else {
            dt = dt_max > 0.f && mv == 0.f ? dt_max : 0.f;
        }
        scal[SC_MV] = m;
        scal[SC_DT] = (double)dt;
        if (!isfinite(mv)) scal[SC_NONFIN] += 1.0;
    }
}

// --------------------------------------------------------------------------
// Level-set step (Sec. II-A, III-A "Numerical settings", Sec. III-C).
// 32 x 32 output tile per block, staged in LDS with a replicated 1-pixel halo.
// phi' = phi + dt (v |grad phi| + lambda m K).
// --------------------------------------------------------------------------
// --------------------------------------------------------------------------
// Conjugate gradient (Sec. III-C): Polak-Ribiere with non-negative restart.
//   k_cg_dots:   block partials of <g,g>, <g,g_prev>, <g_prev,g_prev> (FP64)
//   k_cg_beta:   beta = max(0, (<g,g> - <g,g_prev>) / <g_prev,g_prev>), 0 when first
//   k_cg_update: d = g + beta d (d = g when first), g_prev = g, block max |d|
// --------------------------------------------------------------------------
__global__ __launch_bounds__(RB) void k_cg_dots(const float *__restrict__ g, const float *__restrict__ gp,
                                                size_t npix, size_t chunk, double *__restrict__ part) {
    __shared__ double sh[RB];
    const size_t lo = (size_t)blockIdx.x * chunk;
    const size_t hi = min(npix, lo + chunk);
    double gg = 0.0, ggp = 0.0, gpgp = 0.0;
    for (size_t p = lo + threadIdx.x; p < hi; p += RB) {
        const double a = g[p], b = gp[p];
        gg += a * a;
        ggp += a * b;
        gpgp += b * b;
    }
    gg = block_sum(gg, sh);
    ggp = block_sum(ggp, sh);
    gpgp = block_sum(gpgp, sh);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = gg;
        part[3 * blockIdx.x + 1] = ggp;
        part[3 * blockIdx.x + 2] = gpgp;
    }
}

__global__ __launch_bounds__(RB) void k_cg_beta(const double *__restrict__ part, int nblk, int first,
                                                double *__restrict__ scal) {
    __shared__ double sh[RB];
    double v[3] = {0.0, 0.0, 0.0};
    thread_partial_sums<3, 8>(part, nblk, v);
    for (int q = 0; q < 3; ++q) v[q] = block_sum(v[q], sh);
    if (threadIdx.x == 0) scal[SC_BETA] = (first || !(v[2] > 0.0)) ? 0.0 : fmax(0.0, (v[0] - v[1]) / v[2]);
}

__global__ __launch_bounds__(RB) void k_cg_update(const float *__restrict__ g, float *__restrict__ gp,
                                                  float *__restrict__ d, size_t npix, size_t chunk, int first,
                                                  const double *__restrict__ scal, double *__restrict__ maxpart) {
    __shared__ double sh[RB];
    const float beta = (float)scal[SC_BETA];
    const size_t lo = (size_t)blockIdx.x * chunk;
    const size_t hi = min(npix, lo + chunk);
    float m = 0.f;
    for (size_t p = lo + threadIdx.x; p < hi; p += RB) {
        const float gv = g[p];
        const float dv = first ? gv : fmaf(beta, d[p], gv);
        d[p] = dv;
        gp[p] = gv;
        m = (dv != dv) ? INFINITY : fmaxf(m, fabsf(dv));
    }
    const double r = block_max((double)m, sh);
    if (threadIdx.x == 0) maxpart[blockIdx.x] = r;
}

__global__ __launch_bounds__(256) void k_levelset(const float *__restrict__ phi, const float *__restrict__ vel,
                                                  const float *__restrict__ mod, float lam, float eps_kappa,
                                                  const double *__restrict__ scal, int N,
                                                  float *__restrict__ out, double *__restrict__ part) {
    __shared__ float t[34][35];
    __shared__ int wsum[4];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    // the time step, and the velocity (and modulation) of this thread's
    // pixels, requested before the tile so that all loads are in flight
    // together
    const float dt = (float)scal[SC_DT];
    float vv[4], mv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int y = by + ty + 8 * j, x = bx + tx;
        const bool ok = y < N && x < N;
        const size_t p = ok ? (size_t)y * N + x : 0;
        vv[j] = ok ? vel[p] : 0.f;
        mv[j] = (ok && mod) ? mod[p] : 1.f;
    }
    // the tile with its 1-pixel halo (clamped at the image edge): all of a
    // thread's loads are issued before any is stored
    constexpr int TE = 34 * 34, TU = (TE + 255) / 256;
    float tv[TU];
#pragma unroll
    for (int u = 0; u < TU; ++u) {
        const int e = threadIdx.x + 256 * u;
        if (e < TE) {
            const int yy = e / 34, xx = e - (e / 34) * 34;
            const int gy = min(max(by + yy - 1, 0), N - 1);
            const int gx = min(max(bx + xx - 1, 0), N - 1);
            tv[u] = phi[(size_t)gy * N + gx];
        }
    }
#pragma unroll
    for (int u = 0; u < TU; ++u) {
        const int e = threadIdx.x + 256 * u;
        if (e < TE) t[e / 34][e - (e / 34) * 34] = tv[u];
    }
    __syncthreads();
    int flips = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int ly = ty + 8 * j + 1, lx = tx + 1;
        const int y = by + ly - 1, x = bx + lx - 1;
        if (y < N && x < N) {
            const float c = t[ly][lx];
            const float xp = t[ly][lx + 1], xm = t[ly][lx - 1];
            const float yp = t[ly + 1][lx], ym = t[ly - 1][lx];
            const float pp = t[ly + 1][lx + 1], pm = t[ly + 1][lx - 1];
            const float mp = t[ly - 1][lx + 1], mm = t[ly - 1][lx - 1];
            const float px = 0.5f * (xp - xm);
            const float py = 0.5f * (yp - ym);
            const float pxx = (xp + xm) - 2.f * c;
            const float pyy = (yp + ym) - 2.f * c;
            const float pxy = 0.25f * ((pp - pm) - (mp - mm));
            const float g2 = px * px + py * py;
            const float num = pxx * py * py - 2.f * px * py * pxy + pyy * px * px;
            const float kap = num * __builtin_amdgcn_rcpf(g2 + eps_kappa);
            const size_t p = (size_t)y * N + x;
            const float nv = c + dt * (vv[j] * sqrtf(g2) + lam * mv[j] * kap);
            out[p] = nv;
            flips += ((nv <= 0.f) != (c <= 0.f)) ? 1 : 0;
        }
    }
    // integer count: wave sums, then the four waves in order
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) flips += __shfl_xor(flips, o);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = flips;
    __syncthreads();
    if (threadIdx.x == 0)
        part[blockIdx.y * gridDim.x + blockIdx.x] = (double)(wsum[0] + wsum[1] + wsum[2] + wsum[3]);
}

__global__ __launch_bounds__(RB) void k_finish_step(const double *__restrict__ part, int nblk,
                                                    double *__restrict__ scal, double *__restrict__ stats4,
                                                    double *__restrict__ trace_row, int iter, double ns_per_tick) {
    __shared__ double sh[RB];
    double fs[1] = {0.0};
    thread_partial_sums<1, 16>(part, nblk, fs);
    const double f = block_sum(fs[0], sh);
    if (threadIdx.x == 0) {
        scal[SC_FLIPS] = f;
        if (stats4) {
            stats4[0] = scal[SC_MV];
            stats4[1] = scal[SC_DT];
            stats4[2] = f;
            stats4[3] = 0.0;
        }
        if (trace_row) {
            trace_row[0] = (double)iter;
            trace_row[1] = scal[SC_LOSS];
            trace_row[2] = scal[SC_L2];
            trace_row[3] = scal[SC_PVB];
            trace_row[4] = f;
            trace_row[5] = scal[SC_MV];
            trace_row[6] = scal[SC_DT];
            trace_row[7] = (double)wall_clock64() * ns_per_tick;
        }
    }
}

// --------------------------------------------------------------------------
// Exact squared EDT (Sec. II-A SDF, Sec. III-A TSDF, Alg. 1 CUDA_TSDF).
//
// Column pass, step 1: pack the class bits of every column, 32 rows per word:
// colbits[w][x] bit b = [pixel (32w + b, x) is inside].
// --------------------------------------------------------------------------
constexpr uint32_t NONE16 = 0xFFFFu;

__global__ __launch_bounds__(256) void k_edt_pack(const float *__restrict__ phi, const uint8_t *__restrict__ mask,
                                                  int N, uint32_t *__restrict__ colbits) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int w = blockIdx.y;
    if (x >= N) return;
    uint32_t bits = 0u;
#pragma unroll 8
    for (int b = 0; b < 32; ++b) {
        const int y = 32 * w + b;
        if (y < N) {
            const bool in = phi ? (phi[(size_t)y * N + x] <= 0.f) : (mask[(size_t)y * N + x] != 0);
            bits |= (in ? 1u : 0u) << b;
        }
    }
    colbits[(size_t)w * N + x] = bits;
}

// Column pass, step 2: for each pixel, the distance along its column to the
// nearest pixel of each class (0 = outside, 1 = inside), packed as two 16-bit
// fields (0xFFFF = none).  One thread per (column, 32-row word): the nearest
// class pixels above and below the word come from a scan over whole words,
// the rest from clz / ctz of the word itself.
__device__ __forceinline__ uint32_t valid_bits(int w, int N) {
    const int rows = N - 32 * w;
    return rows >= 32 ? 0xFFFFFFFFu : ((1u << rows) - 1u);
}

__global__ __launch_bounds__(256) void k_edt_coldist(const uint32_t *__restrict__ colbits, int N,
                                                     uint32_t *__restrict__ gout) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int w = blockIdx.y;
    if (x >= N) return;
    const int W = (N + 31) / 32;
    const uint32_t vm = valid_bits(w, N);
    const uint32_t w1 = colbits[(size_t)w * N + x];
    const uint32_t w0 = ~w1 & vm;
    // nearest rows of each class strictly above this word / strictly below it
    int up1 = -1, up0 = -1, dn1 = -1, dn0 = -1;
    for (int v = w - 1; v >= 0 && (up1 < 0 || up0 < 0); --v) {
        const uint32_t b1 = colbits[(size_t)v * N + x];
        const uint32_t b0 = ~b1;                      // words above are full
        if (up1 < 0 && b1) up1 = 32 * v + 31 - __clz(b1);
        if (up0 < 0 && b0) up0 = 32 * v + 31 - __clz(b0);
    }
    for (int v = w + 1; v < W && (dn1 < 0 || dn0 < 0); ++v) {
        const uint32_t b1 = colbits[(size_t)v * N + x];
        const uint32_t b0 = ~b1 & valid_bits(v, N);
        if (dn1 < 0 && b1) dn1 = 32 * v + __ffs(b1) - 1;
        if (dn0 < 0 && b0) dn0 = 32 * v + __ffs(b0) - 1;
    }
#pragma unroll 4
    for (int b = 0; b < 32; ++b) {
        const int y = 32 * w + b;
        if (y >= N) break;
        const uint32_t le = (b == 31) ? 0xFFFFFFFFu : ((2u << b) - 1u);   // bits <= b
        uint32_t d[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const uint32_t word = c ? w1 : w0;
            const int up = c ? up1 : up0, dn = c ? dn1 : dn0;
            const uint32_t a = word & le;
            const uint32_t bl = word & ~le;
            int best = 0x7FFFFFFF;
            if (a) best = min(best, b - (31 - __clz(a)));
            else if (up >= 0) best = min(best, y - up);
            if (bl) best = min(best, (__ffs(bl) - 1) - b);
            else if (dn >= 0) best = min(best, dn - y);
            d[c] = best == 0x7FFFFFFF ? NONE16 : (uint32_t)best;
        }
        gout[(size_t)y * N + x] = d[0] | (d[1] << 16);
    }
}

// Correctly rounded FP32 value of sqrt(D) - 1/2 for an integer D >= 1.
// Start from the FP64 estimate and move to the neighbour while the exact
// midpoint tests (signs of fma(u, u, -D), which are exact) say the true value
// lies outside the rounding interval.
__device__ float sqrt_minus_half(int D) {
    const double dd = (double)D;
    float t = (float)(sqrt(dd) - 0.5);
    for (int it = 0; it < 4; ++it) {
        const double lo = 0.5 * ((double)t + (double)nextafterf(t, -INFINITY)) + 0.5;
        const double hi = 0.5 * ((double)t + (double)nextafterf(t, INFINITY)) + 0.5;
        if (fma(lo, lo, -dd) > 0.0) t = nextafterf(t, -INFINITY);
        else if (fma(hi, hi, -dd) < 0.0) t = nextafterf(t, INFINITY);
        else break;
    }
    return t;
}

// Row pass: for each row and class c, D_c(x) = min_x' f(x') + (x - x')^2,
// f = g_c^2 (2^30 stand-in where the column has no class-c pixel).  The cost
// matrix is Monge, so the leftmost minimiser is non-decreasing in x; the
// minimisers are found level by level over x (stride halving), each query
// searching only between its neighbours' minimisers.  The candidates of all
// queries of a level are laid end to end and split evenly over the 64 lanes
// of the row's wave; partial minima meet in LDS through a 64-bit atomic
// minimum of (value, index), which keeps the leftmost minimiser.
constexpr int FBIG = 1 << 30;

struct RowLevel {
    int s;      // stride (0: the two end points)
    int N;
    int nq;     // queries per class
};

// Query q of a level covers class q / nq; returns its pixel, candidate range
// and the class arrays it reads.
// arg and f hold both classes back to back: class c at [c * N, (c + 1) * N).
__device__ __forceinline__ void query_of(const RowLevel &L, const int16_t *arg, int q, int &cls, int &xq,
                                         int &lo, int &hi) {
    cls = q >= L.nq;
    const int qq = q - cls * L.nq;
    if (L.s == 0) {
        xq = qq ? L.N - 1 : 0;
        lo = 0;
        hi = L.N - 1;
    } else {
        xq = L.s * (2 * qq + 1);
        lo = arg[cls * L.N + xq - L.s];
        hi = arg[cls * L.N + min(xq + L.s, L.N - 1)];
    }
}

__device__ __forceinline__ void row_level(const RowLevel &L, const int *f, int16_t *arg, int *off,
                                          unsigned long long *key, int lane) {
    const int nq = 2 * L.nq;                  // both classes
    const int qb = (nq + 63) / 64;
    const int qlo = min(nq, lane * qb), qhi = min(nq, qlo + qb);
    int sum = 0;
    for (int q = qlo; q < qhi; ++q) {
        int cls, xq, lo, hi;
        query_of(L, arg, q, cls, xq, lo, hi);
        sum += hi - lo + 1;
    }
    int incl = sum;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    const int T = __shfl(incl, 63);
    int run = incl - sum;
    for (int q = qlo; q < qhi; ++q) {
        int cls, xq, lo, hi;
        query_of(L, arg, q, cls, xq, lo, hi);
        off[q] = run;
        run += hi - lo + 1;
        key[q] = ~0ull;
    }
    __syncthreads();
    const int C = (T + 63) / 64;
    const int i0 = lane * C, i1 = min(T, i0 + C);
    if (i0 < i1) {
        int a = 0, b = nq - 1;                  // largest q with off[q] <= i0
        while (a < b) {
            const int m = (a + b + 1) >> 1;
            if (off[m] <= i0) a = m; else b = m - 1;
        }
        int q = a, i = i0;
        while (i < i1) {
            int cls, xq, lo, hi;
            query_of(L, arg, q, cls, xq, lo, hi);
            const int *fc = f + cls * L.N;
            const int cs = lo + (i - off[q]);
            const int ce = min(hi, lo + (i1 - off[q]) - 1);
            int bv = 0x7FFFFFFF, bi = 0;
            int cnd = cs;
            for (; cnd + 3 <= ce; cnd += 4) {
                const int f0 = fc[cnd], f1 = fc[cnd + 1], f2 = fc[cnd + 2], f3 = fc[cnd + 3];
                const int d0 = xq - cnd;
                const int v0 = f0 + d0 * d0;
                const int v1 = f1 + (d0 - 1) * (d0 - 1);
                const int v2 = f2 + (d0 - 2) * (d0 - 2);
                const int v3 = f3 + (d0 - 3) * (d0 - 3);
                if (v0 < bv) { bv = v0; bi = cnd; }
                if (v1 < bv) { bv = v1; bi = cnd + 1; }
                if (v2 < bv) { bv = v2; bi = cnd + 2; }
                if (v3 < bv) { bv = v3; bi = cnd + 3; }
            }
            for (; cnd <= ce; ++cnd) {
                const int v = fc[cnd] + (xq - cnd) * (xq - cnd);
                if (v < bv) { bv = v; bi = cnd; }
            }
            atomicMin(&key[q], ((unsigned long long)(unsigned)bv << 32) | (unsigned)bi);
            i = off[q] + (hi - lo + 1);
            ++q;
        }
    }
    __syncthreads();
    for (int q = lane; q < nq; q += 64) {
        int cls, xq, lo, hi;
        query_of(L, arg, q, cls, xq, lo, hi);
        arg[cls * L.N + xq] = (int16_t)(key[q] & 0xFFFFFFFFull);
    }
    __syncthreads();
}

__device__ __forceinline__ void row_transform(const int *f, int16_t *arg, int *off, unsigned long long *key,
                                              int N, int lane) {
    row_level(RowLevel{0, N, N > 1 ? 2 : 1}, f, arg, off, key, lane);
    int Lp = 1;
    while (Lp < N - 1) Lp <<= 1;
    for (int s = Lp >> 1; s >= 1; s >>= 1) {
        const int nq = (N - 1 > s) ? ((N - 1 - s + 2 * s - 1) / (2 * s)) : 0;
        if (nq > 0) row_level(RowLevel{s, N, nq}, f, arg, off, key, lane);
    }
}

// Both classes of one row per 64-lane block.  LDS: packed column distances,
// f and minimisers for each class, and the level's query offsets and keys.
__global__ __launch_bounds__(64) void k_edt_rows(const uint32_t *__restrict__ gin, int N, float d_lower,
                                                 float d_upper, float *__restrict__ phi_out,
                                                 int *__restrict__ sqdist) {
    extern __shared__ unsigned long long smem_u64[];
    const int nqmax = 2 * (N / 2 + 2);
    unsigned long long *key = smem_u64;                           // [nqmax]
    uint32_t *gr = reinterpret_cast<uint32_t *>(key + nqmax);     // [N]
    int *f0 = reinterpret_cast<int *>(gr + N);                    // [N]
    int *f1 = f0 + N;                                             // [N]
    int *off = f1 + N;                                            // [nqmax]
    int16_t *a0 = reinterpret_cast<int16_t *>(off + nqmax);       // [N]
    int16_t *a1 = a0 + N;                                         // [N]
    const int y = blockIdx.x, lane = threadIdx.x;
    const uint32_t *grow = gin + (size_t)y * N;
    for (int x = lane; x < N; x += 64) {
        const uint32_t g = grow[x];
        gr[x] = g;
        const uint32_t g0 = g & 0xFFFFu, g1 = g >> 16;
        f0[x] = (g0 == NONE16) ? FBIG : (int)(g0 * g0);
        f1[x] = (g1 == NONE16) ? FBIG : (int)(g1 * g1);
    }
    __syncthreads();
    row_transform(f0, a0, off, key, N, lane);
    for (int x = lane; x < N; x += 64) {
        const bool inside = (gr[x] >> 16) == 0;        // distance 0 to class 1
        // inside pixels need the distance to class 0 (D_out), outside to class 1 (D_in)
        const int c0 = a0[x], c1 = a1[x];
        const int D0 = f0[c0] + (x - c0) * (x - c0);
        const int D1 = f1[c1] + (x - c1) * (x - c1);
        if (sqdist) {
            sqdist[(size_t)y * N + x] = D1 >= FBIG ? 0x7FFFFFFF : D1;
            sqdist[(size_t)N * N + (size_t)y * N + x] = D0 >= FBIG ? 0x7FFFFFFF : D0;
        }
        float v;
        if (inside) v = D0 >= FBIG ? d_lower : -sqrt_minus_half(D0);
        else v = D1 >= FBIG ? d_upper : sqrt_minus_half(D1);
        phi_out[(size_t)y * N + x] = fminf(fmaxf(v, d_lower), d_upper);
    }
}

// Row pass for a clipped TSDF only (no squared-distance output).  A pixel
// needs its exact D only while sqrt(D) - 1/2 stays inside the clip bound B,
// i.e. D <= Rb^2 with Rb = bound + 1/2.  Each pixel scans candidate columns
// outward from its own, x' = x +- d: every scanned candidate is an upper
// bound of D, and the scan stops once d^2 >= best (nothing farther can beat
// it) or d passes floor(Rb) (a minimiser with D <= Rb^2 lies within that
// window).  So the result is exact whenever it is at most Rb^2, and above
// Rb^2 only when D is; such pixels take the clip value.  One block per row.
__global__ __launch_bounds__(256) void k_edt_rows_clip(const uint32_t *__restrict__ gin, int N, int pad,
                                                       float d_lower, float d_upper, float *__restrict__ phi_out) {
    // each class row is stored with `pad` sentinel entries on both sides, so
    // the scan needs no bounds checks (sentinels never win: FBIG >= any bound)
    extern __shared__ int fsh[];
    const int W = N + 2 * pad;
    int *f0 = fsh + pad;          // squared column distance to class 0 (FBIG: none)
    int *f1 = fsh + W + pad;      // ... to class 1
    const int y = blockIdx.x;
    const uint32_t *grow = gin + (size_t)y * N;
    for (int i = threadIdx.x; i < 2 * W; i += 256) fsh[i] = FBIG;
    __syncthreads();
    for (int x = threadIdx.x; x < N; x += 256) {
        const uint32_t g = grow[x];
        const uint32_t g0 = g & 0xFFFFu, g1 = g >> 16;
        f0[x] = (g0 == NONE16) ? FBIG : (int)(g0 * g0);
        f1[x] = (g1 == NONE16) ? FBIG : (int)(g1 * g1);
    }
    __syncthreads();
    const int r_out = (int)floorf(d_upper + 0.5f);     // outside pixels: bound d_upper
    const int r_in = (int)floorf(-d_lower + 0.5f);     // inside pixels: bound |d_lower|
    for (int x = threadIdx.x; x < N; x += 256) {
        const bool inside = f1[x] == 0;
        const int *fc = inside ? f0 : f1;
        const int R = min(inside ? r_in : r_out, pad - 8);
        int best = fc[x];
        int d = 1, q = 1;                               // q = d^2
        while (d <= R && q < best) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                best = min(best, min(fc[x - d], fc[x + d]) + q);
                q += 2 * d + 1;
                ++d;
            }
        }
        const float rb = inside ? (-d_lower + 0.5f) : (d_upper + 0.5f);
        float v;
        if ((double)best > (double)rb * (double)rb) {
            v = inside ? d_lower : d_upper;
        } else {
            const float t = sqrt_minus_half(best);
            v = inside ? -t : t;
        }
        phi_out[(size_t)y * N + x] = fminf(fmaxf(v, d_lower), d_upper);
    }
}

__global__ void k_copy(float *__restrict__ dst, const float *__restrict__ src, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_fill(float *__restrict__ dst, float v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = v;
}

size_t chunk_of(size_t npix, int nblk) { return (npix + nblk - 1) / nblk; }

}  // namespace

int resist_blocks(const ilt_ctx *c) {
    const size_t npix = (size_t)c->N * c->N;
    return (int)std::min<size_t>(MAX_RBLK, (npix + 2047) / 2048);
}

hipError_t launch_resist(ilt_ctx *c, const float *I, const uint8_t *target, const resist_args &ra, float *G,
                         double *part) {
    const size_t npix = (size_t)c->N * c->N;
    const int nblk = resist_blocks(c);
    if (npix % 4 == 0 && reinterpret_cast<uintptr_t>(I) % 16 == 0 && reinterpret_cast<uintptr_t>(G) % 16 == 0 &&
        reinterpret_cast<uintptr_t>(target) % 4 == 0)
    {
        // the corner layouts of the fixed-layout kernels (set_used must agree)
        const bool one = ra.n_corners == 1 && ra.cset[0] == 0 && ra.set_used[0] && !ra.set_used[1] &&
                         !ra.set_used[2] && !ra.set_used[3];
        const bool three = ra.n_corners == 3 && ra.cset[0] == 0 && ra.cset[1] == 0 && ra.cset[2] == 1 &&
                           ra.set_used[0] && ra.set_used[1] && !ra.set_used[2] && !ra.set_used[3];
        const size_t ch = chunk_of(npix / 4, nblk);
        if (one) k_resist4<1><<<nblk, RB, 0, c->stream>>>(I, npix, target, ra, npix, ch, G, part);
        else if (three) k_resist4<2><<<nblk, RB, 0, c->stream>>>(I, npix, target, ra, npix, ch, G, part);
        else k_resist4<0><<<nblk, RB, 0, c->stream>>>(I, npix, target, ra, npix, ch, G, part);
    }
    else
        k_resist1<<<nblk, RB, 0, c->stream>>>(I, npix, target, ra, npix, chunk_of(npix, nblk), G, part);
    return hipGetLastError();
}

hipError_t launch_finish_resist(ilt_ctx *c, const double *part, int nblk, double *scal, double *stats4) {
    k_finish_resist<<<1, RB, 0, c->stream>>>(part, nblk, scal, stats4);
    return hipGetLastError();
}

int gradmax_blocks(const ilt_ctx *c) { return resist_blocks(c); }

int launch_cg(ilt_ctx *c, int first, double *part, double *maxpart, hipError_t *err) {
    const size_t npix = (size_t)c->N * c->N;
    const int nblk = gradmax_blocks(c);
    const size_t chunk = chunk_of(npix, nblk);
    k_cg_dots<<<nblk, RB, 0, c->stream>>>(c->g, c->g_prev, npix, chunk, part);
    k_cg_beta<<<1, RB, 0, c->stream>>>(part, nblk, first, c->scal);
    k_cg_update<<<nblk, RB, 0, c->stream>>>(c->g, c->g_prev, c->dcg, npix, chunk, first, c->scal, maxpart);
    *err = hipGetLastError();
    return nblk;
}

hipError_t launch_absmax(ilt_ctx *c, const float *v, double *part) {
    const size_t npix = (size_t)c->N * c->N;
    const int nblk = gradmax_blocks(c);
    k_absmax<<<nblk, RB, 0, c->stream>>>(v, npix, chunk_of(npix, nblk), part);
    return hipGetLastError();
}

hipError_t launch_finish_dt(ilt_ctx *c, const double *part, int nblk, int dt_mode, float eta, float dt_max,
                            double *scal) {
    k_finish_dt<<<1, RB, 0, c->stream>>>(part, nblk, dt_mode, eta, dt_max, scal);
    return hipGetLastError();
}

int step_blocks(const ilt_ctx *c) {
    const int nb = (c->N + 31) / 32;
    return nb * nb;
}

hipError_t launch_levelset(ilt_ctx *c, const float *phi, const float *vel, const float *mod, float lam,
                           float eps_kappa, const double *scal, float *phi_out, double *part) {
    const int nb = (c->N + 31) / 32;
    k_levelset<<<dim3(nb, nb), 256, 0, c->stream>>>(phi, vel, mod, lam, eps_kappa, scal, c->N, phi_out, part);
    return hipGetLastError();
}

static double g_ns_per_tick = 10.0;
void set_ns_per_tick(double v) { g_ns_per_tick = v; }

hipError_t launch_finish_step(ilt_ctx *c, const double *part, int nblk, double *scal, double *stats4,
                              double *trace_row, int iter) {
    k_finish_step<<<1, RB, 0, c->stream>>>(part, nblk, scal, stats4, trace_row, iter, g_ns_per_tick);
    return hipGetLastError();
}

hipError_t launch_edt(ilt_ctx *c, const float *phi, const uint8_t *mask, float *phi_out, int *sqdist,
                      float d_lower, float d_upper) {
    const int N = c->N;
    const dim3 grid((N + 255) / 256, (N + 31) / 32);
    k_edt_pack<<<grid, 256, 0, c->stream>>>(phi, mask, N, c->colbits);
    k_edt_coldist<<<grid, 256, 0, c->stream>>>(c->colbits, N, c->edtg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!sqdist) {
        // sentinel padding covers the largest clip radius plus one unrolled step
        const int r = (int)std::ceil(std::max(d_upper, -d_lower) + 0.5f);
        const int pad = std::min(r, N) + 8;
        const size_t sm = (size_t)(N + 2 * pad) * 2 * sizeof(int);
        if (sm <= 160 * 1024) {
            k_edt_rows_clip<<<N, 256, sm, c->stream>>>(c->edtg, N, pad, d_lower, d_upper, phi_out);
            return hipGetLastError();
        }
    }
    const int nqmax = 2 * (N / 2 + 2);
    const size_t sm = (size_t)nqmax * 8 + (size_t)N * 4 * 3 + (size_t)nqmax * 4 + (size_t)N * 2 * 2;
    k_edt_rows<<<N, 64, sm, c->stream>>>(c->edtg, N, d_lower, d_upper, phi_out, sqdist);
    return hipGetLastError();
}

hipError_t launch_copy(ilt_ctx *c, float *dst, const float *src, size_t n) {
    k_copy<<<1024, 256, 0, c->stream>>>(dst, src, n);
    return hipGetLastError();
}

hipError_t launch_fill(ilt_ctx *c, float *dst, float v, size_t n) {
    k_fill<<<1024, 256, 0, c->stream>>>(dst, v, n);
    return hipGetLastError();
}
