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
                                               double *__restrict__ part, size_t i_cs, size_t t_cs, size_t p_cs) {
    __shared__ double sh[RB];
    // grid.y: clips, each with its own images, target, G and partials
    I += blockIdx.y * i_cs;
    G += blockIdx.y * i_cs;
    target += blockIdx.y * t_cs;
    part += blockIdx.y * p_cs;
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
                                                double *__restrict__ part, size_t i_cs, size_t t_cs, size_t p_cs) {
    __shared__ double sh[RB];
    I += blockIdx.y * i_cs;
    G += blockIdx.y * i_cs;
    target += blockIdx.y * t_cs;
    part += blockIdx.y * p_cs;
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
                                                      double *__restrict__ scal, double *__restrict__ stats4,
                                                      size_t p_cs) {
    __shared__ double sh[RB];
    // block = clip
    part += blockIdx.x * p_cs;
    scal += blockIdx.x * SC_COUNT;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    thread_partial_sums<4, 8>(part, nblk, v);
    for (int q = 0; q < 4; ++q) v[q] = block_sum(v[q], sh);
    if (threadIdx.x == 0) {
        scal[SC_LOSS] = v[0];
        scal[SC_L2] = v[1];
        scal[SC_PVB] = v[2];
        scal[SC_NONFIN] = v[3];
        scal[SC_BAD] += v[3];
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
                                                  float eta, float dt_max, double *__restrict__ scal, size_t p_cs) {
    __shared__ double sh[RB];
    // block = clip
    part += blockIdx.x * p_cs;
    scal += blockIdx.x * SC_COUNT;
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
        if (!isfinite(mv)) {
            scal[SC_NONFIN] += 1.0;
            scal[SC_BAD] += 1.0;
        }
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
                                                  float *__restrict__ out, double *__restrict__ part, size_t p_cs) {
    __shared__ float t[34][35];
    __shared__ int wsum[4], wbad[4];
    // grid.z: clips, each with its own phi, velocity, output, scalars and partials
    {
        const size_t o = (size_t)blockIdx.z * N * N;
        phi += o;
        vel += o;
        out += o;
        scal += blockIdx.z * SC_COUNT;
        part += blockIdx.z * p_cs;
    }
    // tiles in dispatch order go round the eight XCDs; give each XCD a
    // contiguous range of tiles (whole tile rows) instead, so that the
    // sectors of a tile's halo that its neighbours also read are fetched
    // into that XCD's L2 once
    int tile;
    {
        const int nblk = gridDim.x * gridDim.y, b = blockIdx.y * gridDim.x + blockIdx.x;
        const int q = nblk >> 3, r = nblk & 7, xcd = b & 7, k = b >> 3;
        tile = (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + k;
    }
    const int bx = (tile % gridDim.x) * 32, by = (tile / gridDim.x) * 32;
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
    // the tile with its 1-pixel halo (clamped at the image edge): the 32
    // interior columns of each of the 34 rows as aligned 16-byte loads, the
    // two halo columns as single words; all of a thread's loads are issued
    // before any is stored
    const bool vec = (N & 3) == 0;
    float4 iv[2];
    float hv = 0.f;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int e = threadIdx.x + 256 * u;
        if (e < 34 * 8) {
            const int row = e >> 3, q = e & 7;
            const size_t rb = (size_t)min(max(by + row - 1, 0), N - 1) * N;
            const int gx = bx + 4 * q;
            if (vec && gx + 3 < N) {
                iv[u] = *reinterpret_cast<const float4 *>(phi + rb + gx);
            } else {
                iv[u].x = phi[rb + min(gx, N - 1)];
                iv[u].y = phi[rb + min(gx + 1, N - 1)];
                iv[u].z = phi[rb + min(gx + 2, N - 1)];
                iv[u].w = phi[rb + min(gx + 3, N - 1)];
            }
        }
    }
    if (threadIdx.x < 68) {
        const int row = threadIdx.x >> 1, side = threadIdx.x & 1;
        const size_t rb = (size_t)min(max(by + row - 1, 0), N - 1) * N;
        hv = phi[rb + (side ? min(bx + 32, N - 1) : max(bx - 1, 0))];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int e = threadIdx.x + 256 * u;
        if (e < 34 * 8) {
            const int row = e >> 3, q = e & 7;
            t[row][1 + 4 * q] = iv[u].x;
            t[row][2 + 4 * q] = iv[u].y;
            t[row][3 + 4 * q] = iv[u].z;
            t[row][4 + 4 * q] = iv[u].w;
        }
    }
    if (threadIdx.x < 68) t[threadIdx.x >> 1][(threadIdx.x & 1) ? 33 : 0] = hv;
    __syncthreads();
    int flips = 0, bad = 0;
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
            bad += isfinite(nv) ? 0 : 1;
        }
    }
    // integer counts: wave sums, then the four waves in order
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        flips += __shfl_xor(flips, o);
        bad += __shfl_xor(bad, o);
    }
    if ((threadIdx.x & 63) == 0) {
        wsum[threadIdx.x >> 6] = flips;
        wbad[threadIdx.x >> 6] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const size_t b = (size_t)tile;
        part[2 * b] = (double)(wsum[0] + wsum[1] + wsum[2] + wsum[3]);
        part[2 * b + 1] = (double)(wbad[0] + wbad[1] + wbad[2] + wbad[3]);
    }
}

__global__ __launch_bounds__(RB) void k_finish_step(const double *__restrict__ part, int nblk,
                                                    double *__restrict__ scal, double *__restrict__ stats4,
                                                    double *__restrict__ trace_row, int iter, double ns_per_tick,
                                                    size_t p_cs, double *const *__restrict__ trace_tab, int row) {
    __shared__ double sh[RB];
    // block = clip; with a table, clip b's row goes to trace_tab[b] (if set)
    part += blockIdx.x * p_cs;
    scal += blockIdx.x * SC_COUNT;
    if (trace_tab) trace_row = trace_tab[blockIdx.x] ? trace_tab[blockIdx.x] + (size_t)row * ILT_TRACE_W : nullptr;
    double fs[2] = {0.0, 0.0};
    thread_partial_sums<2, 8>(part, nblk, fs);
    const double f = block_sum(fs[0], sh);
    const double bad = block_sum(fs[1], sh);
    if (threadIdx.x == 0) {
        scal[SC_FLIPS] = f;
        scal[SC_BAD] += bad;
        if (stats4) {
            stats4[0] = scal[SC_MV];
            stats4[1] = scal[SC_DT];
            stats4[2] = f;
            stats4[3] = bad;
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
// Separable: a column pass gives, for every pixel and class c, the distance
// g_c along its column to the nearest class-c pixel; a row pass then takes
// D_c(x) = min_x' g_c(x')^2 + (x - x')^2, the lower envelope of one
// parabola per column, which is exact integer arithmetic throughout.
//
// Column pass, step 1: pack the class bits of every column, 32 rows per word:
// colbits[w][x] bit b = [pixel (32w + b, x) is inside].  Block = 32 rows x
// 256 columns; each lane reads four adjacent columns (one 16-byte load per
// row when the rows allow it), each wave eight of the 32 rows; the four
// waves' bits meet in LDS.
// --------------------------------------------------------------------------
__device__ __forceinline__ uint32_t valid_bits(int w, int N) {
    const int rows = N - 32 * w;
    return rows >= 32 ? 0xFFFFFFFFu : ((1u << rows) - 1u);
}

template <bool PHI, typename TP>
__global__ __launch_bounds__(256) void k_edt_bits(const TP *__restrict__ phi, const uint8_t *__restrict__ mask,
                                                  int N, int vec, uint32_t *__restrict__ colbits, size_t scr_words) {
    __shared__ uint32_t part[4][256];
    // grid.z: clips, each with its own image and scratch
    if (PHI) phi += (size_t)blockIdx.z * N * N;
    else mask += (size_t)blockIdx.z * N * N;
    colbits += blockIdx.z * scr_words;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int w = blockIdx.y;
    const int x0 = blockIdx.x * 256 + 4 * lane;
    bool in[8][4];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int y = 32 * w + wave + 4 * i;
#pragma unroll
        for (int e = 0; e < 4; ++e) in[i][e] = false;
        if (y >= N) continue;
        const size_t row = (size_t)y * N;
        if (sizeof(TP) == 4 && vec && x0 + 3 < N) {
            if (PHI) {
                const float4 v = *reinterpret_cast<const float4 *>(phi + row + x0);
                in[i][0] = v.x <= 0.f; in[i][1] = v.y <= 0.f; in[i][2] = v.z <= 0.f; in[i][3] = v.w <= 0.f;
            } else {
                const uchar4 v = *reinterpret_cast<const uchar4 *>(mask + row + x0);
                in[i][0] = v.x != 0; in[i][1] = v.y != 0; in[i][2] = v.z != 0; in[i][3] = v.w != 0;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (x0 + e < N) in[i][e] = PHI ? (phi[row + x0 + e] <= (TP)0) : (mask[row + x0 + e] != 0);
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        uint32_t b = 0u;
#pragma unroll
        for (int i = 0; i < 8; ++i) b |= (in[i][e] ? 1u : 0u) << (wave + 4 * i);
        part[wave][4 * lane + e] = b;
    }
    __syncthreads();
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x < N)
        colbits[(size_t)w * N + x] = ((part[0][threadIdx.x] | part[1][threadIdx.x]) | part[2][threadIdx.x]) |
                                     part[3][threadIdx.x];
}

constexpr int EDT_CB = 16;        // columns per block of the column pass

// Column pass, step 2: for every column x and word w, the nearest rows of
// each class strictly above the word and strictly below it:
// info[0][w][x] = class 1 above, [1] class 0 above, [2] class 1 below,
// [3] class 0 below (-1: none).  Block = EDT_CB columns x every word: the
// words sit in LDS, and per column a bit mask of the words holding each
// class turns "nearest word above / below" into one bit scan.
// Up to 128 words (N <= 4096).
__device__ __forceinline__ int word_below(const unsigned long long (&m)[2], int v) {   // largest u < v, or -1
    if (v > 64) {
        const unsigned long long t = m[1] & (v == 128 ? ~0ull : ((1ull << (v - 64)) - 1ull));
        if (t) return 64 + 63 - __clzll((long long)t);
        v = 64;
    }
    const unsigned long long t = m[0] & (v == 64 ? ~0ull : ((1ull << v) - 1ull));
    return t ? 63 - __clzll((long long)t) : -1;
}

__device__ __forceinline__ int word_above(const unsigned long long (&m)[2], int v) {   // smallest u > v, or -1
    int u = v + 1;
    if (u < 64) {
        const unsigned long long t = m[0] & (~0ull << u);
        if (t) return __ffsll((long long)t) - 1;
        u = 64;
    }
    if (u < 128) {
        const unsigned long long t = m[1] & (~0ull << (u - 64));
        if (t) return 64 + __ffsll((long long)t) - 1;
    }
    return -1;
}

__global__ __launch_bounds__(256) void k_edt_colinfo(const uint32_t *__restrict__ colbits, int N,
                                                     int16_t *__restrict__ info, size_t scr_words) {
    // grid.y: clips, each with its own scratch
    colbits += blockIdx.y * scr_words;
    info += blockIdx.y * 2 * scr_words;
    // block = EDT_CB columns; the 256 / EDT_CB thread rows step over the words
    constexpr int WL = 256 / EDT_CB;
    extern __shared__ uint32_t wsh[];                       // [W][EDT_CB]
    __shared__ unsigned long long any1[EDT_CB][2], any0[EDT_CB][2];
    const int W = (N + 31) / 32;
    const int c = threadIdx.x % EDT_CB, v0 = threadIdx.x / EDT_CB;
    const int x = blockIdx.x * EDT_CB + c;
    if (threadIdx.x < 2 * EDT_CB) {
        any1[threadIdx.x >> 1][threadIdx.x & 1] = 0ull;
        any0[threadIdx.x >> 1][threadIdx.x & 1] = 0ull;
    }
    __syncthreads();
    for (int v = v0; v < W; v += WL) {
        const uint32_t wd = x < N ? colbits[(size_t)v * N + x] : 0u;
        wsh[v * EDT_CB + c] = wd;
        if (x < N) {
            if (wd) atomicOr(&any1[c][v >> 6], 1ull << (v & 63));
            if (~wd & valid_bits(v, N)) atomicOr(&any0[c][v >> 6], 1ull << (v & 63));
        }
    }
    __syncthreads();
    if (x >= N) return;
    const unsigned long long m1[2] = {any1[c][0], any1[c][1]}, m0[2] = {any0[c][0], any0[c][1]};
    const size_t plane = (size_t)W * N;
    for (int v = v0; v < W; v += WL) {
        int r[4];
        int u = word_below(m1, v);
        r[0] = u < 0 ? -1 : 32 * u + 31 - __clz(wsh[u * EDT_CB + c]);
        u = word_below(m0, v);
        r[1] = u < 0 ? -1 : 32 * u + 31 - __clz(~wsh[u * EDT_CB + c] & valid_bits(u, N));
        u = word_above(m1, v);
        r[2] = u < 0 ? -1 : 32 * u + __ffs(wsh[u * EDT_CB + c]) - 1;
        u = word_above(m0, v);
        r[3] = u < 0 ? -1 : 32 * u + __ffs(~wsh[u * EDT_CB + c] & valid_bits(u, N)) - 1;
        const size_t o = (size_t)v * N + x;
#pragma unroll
        for (int q = 0; q < 4; ++q) info[q * plane + o] = (int16_t)r[q];
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

// Row pass.  One block per row, one wave per class c (0 = outside, 1 =
// inside): D_c(x) = min over columns x' holding a class-c pixel of
// g_c(x')^2 + (x - x')^2.  In the dual, column x' is the point
// (x', x'^2 + g^2) and D_c(x) - x^2 is the minimum of c' - 2 x x' over the
// points, attained on their lower convex hull; hull vertices are the
// columns whose parabola is lowest somewhere.  Lane l owns the band of M
// columns [l M, l M + M) (64 M >= N).
//   1. each lane builds the hull of its band as a stack (the top vertex is
//      dropped while it lies on or above the chord from the one below it to
//      the new column; exact in 64-bit integers) and keeps it as a chain in
//      LDS; a range [r0, r1) of the chain stays alive;
//   2. six rounds merge adjacent groups of bands pairwise.  The merged
//      hull is the left group's chain up to a vertex a and the right
//      group's from a vertex b on (the bridge).  From a = the left group's
//      last vertex, b = the right group's first one, alternately b becomes
//      the tangent point from a on the right group (least slope, the
//      farthest on ties) and a the tangent point from b on the left group
//      (greatest slope, the nearest on ties) until neither moves: each lane
//      finds its own chain's tangent point by bisection and the pair's lanes
//      reduce over their group; a only moves left and b only right, so the
//      iteration ends, at the bridge.  Lanes then trim their ranges;
//   3. each surviving vertex s marks, at the first pixel where it is at
//      least as low as its predecessor p on the hull (the exact integer
//      ceiling of (c_s - c_p) / 2 (s - p)), itself; along the hull these
//      pixels do not decrease, so the owner of pixel x is the marked vertex
//      of largest column at or before x: a prefix maximum over the row.
// Every value is an exact integer, so the result is unique.  A class that
// is absent from the whole image leaves D = FBIG.
constexpr int FBIG = 1 << 30;
constexpr int GNONE = 0xFFFF;

// a vertex as one word: column << 16 | g (so that comparing words compares
// columns); -1: none
__device__ __forceinline__ int vx(int e) { return e >> 16; }
__device__ __forceinline__ int vg(int e) { return e & 0xFFFF; }
__device__ __forceinline__ int vc(int e) { return vx(e) * vx(e) + vg(e) * vg(e); }

// is the point (b, cb) on or above the chord from (a, ca) to (q, cq), a < b < q?
__device__ __forceinline__ bool hull_above(int a, int ca, int b, int cb, int q, int cq) {
    return (long long)(cb - ca) * (q - b) >= (long long)(cq - cb) * (b - a);
}
// slope(P, U) <= slope(P, V) for U, V right of P
__device__ __forceinline__ bool slope_le_from(int xp, int cp, int u, int v) {
    return (long long)(vc(u) - cp) * (vx(v) - xp) <= (long long)(vc(v) - cp) * (vx(u) - xp);
}
// slope(U, Q) >= slope(V, Q) for U, V left of Q
__device__ __forceinline__ bool slope_ge_to(int u, int v, int xq, int cq) {
    return (long long)(cq - vc(u)) * (xq - vx(v)) >= (long long)(cq - vc(v)) * (xq - vx(u));
}
// tangent candidates: from P on the right (least slope, larger column on
// ties) and to Q on the left (greatest slope, smaller column on ties)
__device__ __forceinline__ bool better_from(int xp, int cp, int u, int v) {
    if (u < 0) return false;
    if (v < 0) return true;
    const long long l = (long long)(vc(u) - cp) * (vx(v) - xp), r = (long long)(vc(v) - cp) * (vx(u) - xp);
    return l < r || (l == r && vx(u) > vx(v));
}
__device__ __forceinline__ bool better_to(int xq, int cq, int u, int v) {
    if (u < 0) return false;
    if (v < 0) return true;
    const long long l = (long long)(cq - vc(u)) * (xq - vx(v)), r = (long long)(cq - vc(v)) * (xq - vx(u));
    return l > r || (l == r && vx(u) < vx(v));
}

// exclusive prefix maximum over the 64 lanes of a wave (lane 0 gets -1)
__device__ __forceinline__ int wave_excl_max(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d *= 2) {
        const int u = __shfl_up(v, d, 64);
        if (lane >= d) v = max(v, u);
    }
    const int ex = __shfl_up(v, 1, 64);
    return lane == 0 ? -1 : ex;
}

template <int M, typename TP>
__global__ __launch_bounds__(128) void k_edt_rows_env(const uint32_t *__restrict__ colbits,
                                                      const int16_t *__restrict__ info, int N, float d_lower,
                                                      float d_upper, TP *__restrict__ phi_out,
                                                      int *__restrict__ sqdist, size_t scr_words) {
    // per class: g of every column, then (in place: a band's chain never
    // gets ahead of the column it has read) the band chains, later the hull
    // marks and then D, M + 1 words per band; the pad puts the 64 lanes'
    // equal band offsets in different banks.  Plus the row's inside bits.
    // About 17 KB, so that 8 blocks of 2 waves share a CU.
    constexpr int S32 = 64 * (M + 1);
    __shared__ int chn[2][S32];
    __shared__ uint32_t insb[2 * M];
    __shared__ int need[2];
    // grid.y: clips, each with its own scratch and output
    colbits += blockIdx.y * scr_words;
    info += blockIdx.y * 2 * scr_words;
    phi_out += (size_t)blockIdx.y * N * N;
    const int y = blockIdx.x;
    const int lane = threadIdx.x & 63, cls = threadIdx.x >> 6;
    const int W = (N + 31) / 32;
    const int w = y >> 5, b = y & 31;
    const uint32_t le = (b == 31) ? 0xFFFFFFFFu : ((2u << b) - 1u);
    const uint32_t vm = valid_bits(w, N);
    const size_t plane = (size_t)W * N;
    // (positions are never negative)
    constexpr int LM = M >= 64 ? 6 : M >= 32 ? 5 : M >= 16 ? 4 : M >= 8 ? 3 : M >= 4 ? 2 : M >= 2 ? 1 : 0;
    auto a32 = [](int p) { return p + (p >> LM); };
    // 0. g_c of every column of this row from the column bits and the
    // nearest class rows above and below this row's word (all loads issued
    // first).  Class c is needed where pixels of the other class lie (or
    // everywhere when squared distances are written).
    if (threadIdx.x < 2) need[threadIdx.x] = sqdist != nullptr;
    __syncthreads();
    {
        bool any_in = false, any_out = false;
        constexpr int R = (64 * M + 127) / 128;
        uint32_t wv[R];
        int16_t iv[R][4];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int x = threadIdx.x + 128 * r;
            if (x < N) {
                const size_t o = (size_t)w * N + x;
                wv[r] = colbits[o];
#pragma unroll
                for (int q = 0; q < 4; ++q) iv[r][q] = info[q * plane + o];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int x = threadIdx.x + 128 * r;
            // inside bits of columns 128 r + 64 cls .. + 63, one ballot per wave
            const unsigned long long ib = __ballot(x < N && ((wv[r] >> b) & 1u));
            if (lane == 0 && 128 * r + 64 * cls < 64 * M) {
                insb[(128 * r + 64 * cls) / 32] = (uint32_t)ib;
                insb[(128 * r + 64 * cls) / 32 + 1] = (uint32_t)(ib >> 32);
            }
            if (x >= N) continue;
            const uint32_t w1 = wv[r], w0 = ~w1 & vm;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const uint32_t word = c ? w1 : w0;
                const int up = iv[r][c ? 0 : 1], dn = iv[r][c ? 2 : 3];
                const uint32_t a = word & le, bl = word & ~le;
                int best = 0x7FFFFFFF;
                if (a) best = b - (31 - __clz(a));
                else if (up >= 0) best = y - up;
                if (bl) best = min(best, (__ffs(bl) - 1) - b);
                else if (dn >= 0) best = min(best, dn - y);
                chn[c][a32(x)] = best == 0x7FFFFFFF ? GNONE : best;
                if (c == 1) {
                    any_in |= best == 0;
                    any_out |= best != 0;
                }
            }
        }
        if (any_in) need[0] = 1;
        if (any_out) need[1] = 1;
    }
    __syncthreads();
    const bool work = need[cls] != 0;      // uniform over the wave
    const int lo = lane * M;
    int *ch = chn[cls];
    int r0 = 0, r1 = 0;
    // 1. the hull of this lane's band, as a chain at ch[a32(lo + k)]
    if (work) {
        // one event per step (skip an empty column, drop the top, or push),
        // so that a wave runs at most 2 M steps however its lanes' drops fall
        const int hi = min(N, lo + M);
        int k = 0, s1 = 0, s2 = 0, c1 = 0, c2 = 0;
        int q = lo, gq = q < hi ? ch[a32(q)] : GNONE;
        while (q < hi) {
            const int cq = q * q + gq * gq;
            if (gq != GNONE && k >= 2 && hull_above(s2, c2, s1, c1, q, cq)) {
                s1 = s2;
                c1 = c2;
                --k;
                if (k >= 2) {
                    const int e = ch[a32(lo + k - 2)];
                    s2 = vx(e);
                    c2 = vc(e);
                }
                continue;
            }
            if (gq != GNONE) {
                ch[a32(lo + k)] = (q << 16) | gq;
                s2 = s1;
                c2 = c1;
                s1 = q;
                c1 = cq;
                ++k;
            }
            ++q;
            gq = q < hi ? ch[a32(q)] : GNONE;
        }
        r1 = k;
    }
    __syncthreads();
    // 2. pairwise merges; chains are read-only from here and every lane's
    // range lives in its registers, so no barrier is needed between rounds
    for (int gs = 1; gs < 64 && work; gs *= 2) {
        const bool left = (lane & gs) == 0;
        const bool ne = r1 > r0;
        int a = (left && ne) ? ch[a32(lo + r1 - 1)] : -1;
        int bb = (!left && ne) ? ch[a32(lo + r0)] : 0x7FFFFFFF;
#pragma unroll
        for (int d = 1; d < 64; d *= 2) {
            if (d < 2 * gs) {
                a = max(a, __shfl_xor(a, d, 64));
                bb = min(bb, __shfl_xor(bb, d, 64));
            }
        }
        if (a < 0 || bb == 0x7FFFFFFF) continue;      // uniform over the pair's lanes
        for (int it = 0; it < 4096; ++it) {
            // b: tangent point from a on the right group
            const int xa = vx(a), ca = vc(a);
            int cand = -1;
            if (!left && ne) {
                int l = r0, h = r1 - 1;
                while (l < h) {
                    const int mid = (l + h + 1) >> 1;
                    if (slope_le_from(xa, ca, ch[a32(lo + mid)], ch[a32(lo + mid - 1)])) l = mid;
                    else h = mid - 1;
                }
                cand = ch[a32(lo + l)];
            }
#pragma unroll
            for (int d = 1; d < 64; d *= 2) {
                if (d < 2 * gs) {
                    const int o = __shfl_xor(cand, d, 64);
                    if (better_from(xa, ca, o, cand)) cand = o;
                }
            }
            const int nb = cand;
            // a: tangent point from b on the left group
            const int xb = vx(nb), cb = vc(nb);
            cand = -1;
            if (left && ne) {
                int l = r0, h = r1 - 1;
                while (l < h) {
                    const int mid = (l + h) >> 1;
                    if (slope_ge_to(ch[a32(lo + mid)], ch[a32(lo + mid + 1)], xb, cb)) h = mid;
                    else l = mid + 1;
                }
                cand = ch[a32(lo + l)];
            }
#pragma unroll
            for (int d = 1; d < 64; d *= 2) {
                if (d < 2 * gs) {
                    const int o = __shfl_xor(cand, d, 64);
                    if (better_to(xb, cb, o, cand)) cand = o;
                }
            }
            const int na = cand;
            const bool done = na == a && nb == bb;
            a = na;
            bb = nb;
            if (done) break;
        }
        // trim: the left group keeps columns <= a, the right one >= b
        if (ne) {
            if (left) {
                const int xa = vx(a);
                if (vx(ch[a32(lo + r0)]) > xa) {
                    r1 = r0;
                } else if (vx(ch[a32(lo + r1 - 1)]) > xa) {
                    int l = r0, h = r1 - 1;                  // last entry <= xa
                    while (l < h) {
                        const int mid = (l + h + 1) >> 1;
                        if (vx(ch[a32(lo + mid)]) <= xa) l = mid;
                        else h = mid - 1;
                    }
                    r1 = l + 1;
                }
            } else {
                const int xb = vx(bb);
                if (vx(ch[a32(lo + r1 - 1)]) < xb) {
                    r0 = r1;
                } else if (vx(ch[a32(lo + r0)]) < xb) {
                    int l = r0, h = r1 - 1;                  // first entry >= xb
                    while (l < h) {
                        const int mid = (l + h) >> 1;
                        if (vx(ch[a32(lo + mid)]) >= xb) h = mid;
                        else l = mid + 1;
                    }
                    r0 = l;
                }
            }
        }
    }
    // 3. marks, then the owner of every pixel and its D, in the chain
    // storage once every lane holds its surviving vertices in registers
    int alive[M];
#pragma unroll
    for (int i = 0; i < M; ++i) alive[i] = (work && r0 + i < r1) ? ch[a32(lo + r0 + i)] : -1;
    const int pred = wave_excl_max(r1 > r0 ? ch[a32(lo + r1 - 1)] : -1);
    __syncthreads();
    if (work) {
#pragma unroll
        for (int i = 0; i < M; ++i) ch[a32(lo + i)] = -1;
    }
    __syncthreads();
    if (work) {
        int p = pred;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const int e = alive[i];
            if (e < 0) break;
            int start = 0;
            if (p >= 0) {
                const int num = vc(e) - vc(p), den = 2 * (vx(e) - vx(p));
                start = num >= 0 ? (num + den - 1) / den : -((-num) / den);
                start = max(start, 0);
            }
            if (start < N) atomicMax(&ch[a32(start)], e);
            p = e;
        }
    }
    __syncthreads();
    if (work) {
        int pre[M];
        int r = -1;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            r = max(r, ch[a32(lo + i)]);
            pre[i] = r;
        }
        const int base = wave_excl_max(r);
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const int x = lo + i, o = max(base, pre[i]);
            int D = FBIG;
            if (o >= 0) D = vg(o) * vg(o) + (x - vx(o)) * (x - vx(o));
            ch[a32(x)] = D;
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < N; x += 128) {
        // inside pixels (g_1 = 0) take D_0, outside ones D_1
        const bool inside = (insb[x >> 5] >> (x & 31)) & 1u;
        const int D = chn[inside ? 0 : 1][a32(x)];
        if (sqdist) {
            const int d1 = chn[1][a32(x)], d0 = chn[0][a32(x)];
            sqdist[(size_t)y * N + x] = d1 >= FBIG ? 0x7FFFFFFF : d1;
            sqdist[(size_t)N * N + (size_t)y * N + x] = d0 >= FBIG ? 0x7FFFFFFF : d0;
        }
        if (sizeof(TP) == 4) {
            float v;
            if (inside) v = D >= FBIG ? d_lower : -sqrt_minus_half(D);
            else v = D >= FBIG ? d_upper : sqrt_minus_half(D);
            phi_out[(size_t)y * N + x] = fminf(fmaxf(v, d_lower), d_upper);
        } else {
            // FP64: the correctly rounded square root less 1/2, which is exact
            // (sqrt(D) >= 1 has an ulp that divides 1/2)
            double v;
            if (inside) v = D >= FBIG ? (double)d_lower : 0.5 - sqrt((double)D);
            else v = D >= FBIG ? (double)d_upper : sqrt((double)D) - 0.5;
            phi_out[(size_t)y * N + x] = (TP)fmin(fmax(v, (double)d_lower), (double)d_upper);
        }
    }
}

__global__ void k_copy(float *__restrict__ dst, const float *__restrict__ src, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// H(phi + dh) as 0/1 (H(z) = 1 for z >= 0): the shifted Heaviside maps that
// are the modulation branch's candidate targets (Sec. III-B).  The FP32 sum
// has the sign of the exact one (rounding never crosses zero).
__global__ void k_heaviside_shift(const float *__restrict__ phi, float dh, size_t n, float *__restrict__ out) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = (phi[i] + dh >= 0.f) ? 1.f : 0.f;
}

__global__ void k_set_scal(double *__restrict__ scal, int slot, double v) {
    scal += blockIdx.x * SC_COUNT;      // block = clip
    if (threadIdx.x == 0) scal[slot] = v;
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
    // clips (c->ncur) step by n_sets images, one target and their partials
    const size_t ics = (size_t)c->n_sets * npix, pcs = (size_t)c->n_part;
    if (npix % 4 == 0 && reinterpret_cast<uintptr_t>(I) % 16 == 0 && reinterpret_cast<uintptr_t>(G) % 16 == 0 &&
        reinterpret_cast<uintptr_t>(target) % 4 == 0)
    {
        // the corner layouts of the fixed-layout kernels (set_used must agree)
        const bool one = ra.n_corners == 1 && ra.cset[0] == 0 && ra.set_used[0] && !ra.set_used[1] &&
                         !ra.set_used[2] && !ra.set_used[3];
        const bool three = ra.n_corners == 3 && ra.cset[0] == 0 && ra.cset[1] == 0 && ra.cset[2] == 1 &&
                           ra.set_used[0] && ra.set_used[1] && !ra.set_used[2] && !ra.set_used[3];
        const size_t ch = chunk_of(npix / 4, nblk);
        if (one) k_resist4<1><<<dim3(nblk, c->ncur), RB, 0, c->stream>>>(I, npix, target, ra, npix, ch, G, part, ics, npix, pcs);
        else if (three) k_resist4<2><<<dim3(nblk, c->ncur), RB, 0, c->stream>>>(I, npix, target, ra, npix, ch, G, part, ics, npix, pcs);
        else k_resist4<0><<<dim3(nblk, c->ncur), RB, 0, c->stream>>>(I, npix, target, ra, npix, ch, G, part, ics, npix, pcs);
    }
    else
        k_resist1<<<dim3(nblk, c->ncur), RB, 0, c->stream>>>(I, npix, target, ra, npix, chunk_of(npix, nblk), G, part,
                                                              ics, npix, pcs);
    return hipGetLastError();
}

hipError_t launch_finish_resist(ilt_ctx *c, const double *part, int nblk, double *scal, double *stats4) {
    k_finish_resist<<<c->ncur, RB, 0, c->stream>>>(part, nblk, scal, stats4, (size_t)c->n_part);
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
    k_finish_dt<<<c->ncur, RB, 0, c->stream>>>(part, nblk, dt_mode, eta, dt_max, scal, (size_t)c->n_part);
    return hipGetLastError();
}

int step_blocks(const ilt_ctx *c) {
    const int nb = (c->N + 31) / 32;
    return nb * nb;
}

hipError_t launch_levelset(ilt_ctx *c, const float *phi, const float *vel, const float *mod, float lam,
                           float eps_kappa, const double *scal, float *phi_out, double *part) {
    const int nb = (c->N + 31) / 32;
    k_levelset<<<dim3(nb, nb, c->ncur), 256, 0, c->stream>>>(phi, vel, mod, lam, eps_kappa, scal, c->N, phi_out, part,
                                                             (size_t)c->n_part);
    return hipGetLastError();
}

static double g_ns_per_tick = 10.0;
void set_ns_per_tick(double v) { g_ns_per_tick = v; }

hipError_t launch_finish_step(ilt_ctx *c, const double *part, int nblk, double *scal, double *stats4,
                              double *trace_row, int iter, double *const *trace_tab, int row) {
    k_finish_step<<<c->ncur, RB, 0, c->stream>>>(part, nblk, scal, stats4, trace_row, iter, g_ns_per_tick,
                                                 (size_t)c->n_part, trace_tab, row);
    return hipGetLastError();
}

// columns per lane of the row pass: the smallest power of two M with 64 M >= N
static int edt_band(int N) {
    int M = 1;
    while (64 * M < N) M *= 2;
    return M;
}

size_t edt_scratch_bytes(int N) {
    const size_t W = (size_t)(N + 31) / 32;
    return W * N * sizeof(uint32_t) + 4 * W * N * sizeof(int16_t);
}

template <typename TP>
hipError_t edt_any(hipStream_t st, int N, const TP *phi, const uint8_t *mask, TP *phi_out, int *sqdist,
                   float d_lower, float d_upper, void *scratch, int nclip = 1) {
    // nclip images one after another (and as many scratch areas); squared
    // distances only for one
    if (nclip > 1 && sqdist) return hipErrorInvalidValue;
    const int W = (N + 31) / 32;
    const size_t scr_words = edt_scratch_bytes(N) / sizeof(uint32_t);
    uint32_t *colbits = static_cast<uint32_t *>(scratch);
    int16_t *info = reinterpret_cast<int16_t *>(colbits + (size_t)W * N);
    const int vec = (N % 4) == 0 && (phi ? reinterpret_cast<uintptr_t>(phi) % 16 == 0
                                         : reinterpret_cast<uintptr_t>(mask) % 4 == 0);
    const dim3 g1((N + 255) / 256, W, nclip);
    if (phi) k_edt_bits<true, TP><<<g1, 256, 0, st>>>(phi, nullptr, N, vec, colbits, scr_words);
    else k_edt_bits<false, TP><<<g1, 256, 0, st>>>(nullptr, mask, N, vec, colbits, scr_words);
    k_edt_colinfo<<<dim3((N + EDT_CB - 1) / EDT_CB, nclip), 256, (size_t)W * EDT_CB * sizeof(uint32_t), st>>>(
        colbits, N, info, scr_words);
    // row pass: bands of M >= N / 64 columns per lane (a power of two)
    const dim3 gr(N, nclip);
    switch (edt_band(N)) {
    case 1: k_edt_rows_env<1, TP><<<gr, 128, 0, st>>>(colbits, info, N, d_lower, d_upper, phi_out, sqdist, scr_words); break;
    case 2: k_edt_rows_env<2, TP><<<gr, 128, 0, st>>>(colbits, info, N, d_lower, d_upper, phi_out, sqdist, scr_words); break;
    case 4: k_edt_rows_env<4, TP><<<gr, 128, 0, st>>>(colbits, info, N, d_lower, d_upper, phi_out, sqdist, scr_words); break;
    case 8: k_edt_rows_env<8, TP><<<gr, 128, 0, st>>>(colbits, info, N, d_lower, d_upper, phi_out, sqdist, scr_words); break;
    case 16: k_edt_rows_env<16, TP><<<gr, 128, 0, st>>>(colbits, info, N, d_lower, d_upper, phi_out, sqdist, scr_words); break;
    case 32: k_edt_rows_env<32, TP><<<gr, 128, 0, st>>>(colbits, info, N, d_lower, d_upper, phi_out, sqdist, scr_words); break;
    default: k_edt_rows_env<64, TP><<<gr, 128, 0, st>>>(colbits, info, N, d_lower, d_upper, phi_out, sqdist, scr_words); break;
    }
    return hipGetLastError();
}

hipError_t launch_edt_raw(hipStream_t st, int N, const float *phi, const uint8_t *mask, float *phi_out, int *sqdist,
                          float d_lower, float d_upper, void *scratch) {
    return edt_any<float>(st, N, phi, mask, phi_out, sqdist, d_lower, d_upper, scratch);
}

hipError_t launch_edt64(ilt_ctx *c, const double *phi, const uint8_t *mask, double *phi_out, int *sqdist,
                        float d_lower, float d_upper) {
    return edt_any<double>(c->stream, c->N, phi, mask, phi_out, sqdist, d_lower, d_upper, c->edt_scratch);
}

hipError_t launch_edt(ilt_ctx *c, const float *phi, const uint8_t *mask, float *phi_out, int *sqdist,
                      float d_lower, float d_upper) {
    return edt_any<float>(c->stream, c->N, phi, mask, phi_out, sqdist, d_lower, d_upper, c->edt_scratch, c->ncur);
}

hipError_t launch_copy(ilt_ctx *c, float *dst, const float *src, size_t n) {
    k_copy<<<1024, 256, 0, c->stream>>>(dst, src, n);
    return hipGetLastError();
}

hipError_t launch_heaviside_shift(const float *phi, float dh, size_t n, float *out, hipStream_t st) {
    const int nb = (int)std::min<size_t>(4096, (n + 255) / 256);
    k_heaviside_shift<<<std::max(nb, 1), 256, 0, st>>>(phi, dh, n, out);
    return hipGetLastError();
}

hipError_t launch_set_scal(ilt_ctx *c, int slot, double v) {
    k_set_scal<<<c->ncur, 64, 0, c->stream>>>(c->scal, slot, v);
    return hipGetLastError();
}

hipError_t launch_fill(ilt_ctx *c, float *dst, float v, size_t n) {
    k_fill<<<1024, 256, 0, c->stream>>>(dst, v, n);
    return hipGetLastError();
}
