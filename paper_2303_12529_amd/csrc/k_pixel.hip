// Pixel-wise kernels: resist and loss, reductions, the level-set step and the
// exact squared EDT.  All reductions are two-stage with a fixed order (block
// partials, then one block), so results are bitwise reproducible.
#include <algorithm>

#include "ilt_internal.h"

namespace {

constexpr int RB = 256;           // threads per reduction block
constexpr int MAX_RBLK = 1024;    // cap on reduction blocks

__device__ __forceinline__ double block_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = RB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = RB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// --------------------------------------------------------------------------
// Resist (Sec. III-A): per corner Z = 1/(1+exp(-sigma_z (d I_s - I_th))),
// loss += omega (Z - Zt)^2, G_s += omega 2 sigma_z d (Z - Zt) Z (1 - Z);
// binary print (Sec. II-B) for L2 (corner 0) and PVBand (corners 1, 2).
// Block b covers a contiguous pixel range; partials {loss, l2, pvb, nonfinite}.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(RB) void k_resist(const float *__restrict__ I, size_t set_stride,
                                               const uint8_t *__restrict__ target, resist_args ra,
                                               size_t npix, size_t chunk, float *__restrict__ G,
                                               double *__restrict__ part) {
    __shared__ double sh[RB];
    const size_t lo = (size_t)blockIdx.x * chunk;
    const size_t hi = min(npix, lo + chunk);
    double loss = 0.0, l2 = 0.0, pvb = 0.0, bad = 0.0;
    for (size_t p = lo + threadIdx.x; p < hi; p += RB) {
        const float zt = target[p] ? 1.f : 0.f;
        float gs[ILT_MAX_SETS] = {0.f, 0.f, 0.f, 0.f};
        float lp = 0.f;
        bool print[4] = {false, false, false, false};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (c < ra.n_corners) {
                const int s = ra.cset[c];
                const float d = ra.dose[c];
                const float di = d * I[(size_t)s * set_stride + p];
                const float z = 1.f / (1.f + expf(-ra.sigma_z * (di - ra.i_th)));
                const float r = z - zt;
                lp = fmaf(ra.omega[c] * r, r, lp);
                const float gv = ra.omega[c] * 2.f * ra.sigma_z * d * r * (z * (1.f - z));
#pragma unroll
                for (int q = 0; q < ILT_MAX_SETS; ++q)
                    if (q == s) gs[q] += gv;
                print[c] = di >= ra.i_th;
            }
        }
        loss += (double)lp;
        if (!isfinite(lp)) bad += 1.0;
        l2 += (print[0] != (zt != 0.f)) ? 1.0 : 0.0;
        if (ra.n_corners >= 3) pvb += (print[1] != print[2]) ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < ILT_MAX_SETS; ++q)
            if (ra.set_used[q]) G[(size_t)q * set_stride + p] = gs[q];
    }
    loss = block_sum(loss, sh);
    l2 = block_sum(l2, sh);
    pvb = block_sum(pvb, sh);
    bad = block_sum(bad, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 4 + 0] = loss;
        part[blockIdx.x * 4 + 1] = l2;
        part[blockIdx.x * 4 + 2] = pvb;
        part[blockIdx.x * 4 + 3] = bad;
    }
}

__global__ __launch_bounds__(RB) void k_finish_resist(const double *__restrict__ part, int nblk,
                                                      double *__restrict__ scal, double *__restrict__ stats4) {
    __shared__ double sh[RB];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += RB)
        for (int q = 0; q < 4; ++q) v[q] += part[b * 4 + q];
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
__global__ __launch_bounds__(256) void k_levelset(const float *__restrict__ phi, const float *__restrict__ vel,
                                                  const float *__restrict__ mod, float lam, float eps_kappa,
                                                  const double *__restrict__ scal, int N,
                                                  float *__restrict__ out, double *__restrict__ part) {
    __shared__ float t[34][35];
    __shared__ double sh[RB];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    for (int e = threadIdx.x; e < 34 * 34; e += 256) {
        const int yy = e / 34, xx = e % 34;
        const int gy = min(max(by + yy - 1, 0), N - 1);
        const int gx = min(max(bx + xx - 1, 0), N - 1);
        t[yy][xx] = phi[(size_t)gy * N + gx];
    }
    __syncthreads();
    const float dt = (float)scal[SC_DT];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    double flips = 0.0;
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
            const float kap = num / (g2 + eps_kappa);
            const size_t p = (size_t)y * N + x;
            const float m = mod ? mod[p] : 1.f;
            const float nv = c + dt * (vel[p] * sqrtf(g2) + lam * m * kap);
            out[p] = nv;
            flips += ((nv <= 0.f) != (c <= 0.f)) ? 1.0 : 0.0;
        }
    }
    flips = block_sum(flips, sh);
    if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = flips;
}

__global__ __launch_bounds__(RB) void k_finish_step(const double *__restrict__ part, int nblk,
                                                    double *__restrict__ scal, double *__restrict__ stats4,
                                                    double *__restrict__ trace_row, int iter, double ns_per_tick) {
    __shared__ double sh[RB];
    double f = 0.0;
    for (int b = threadIdx.x; b < nblk; b += RB) f += part[b];
    f = block_sum(f, sh);
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
// Column pass: for every pixel, the distance along its column to the nearest
// pixel of each class (0 = outside, 1 = inside), packed as two 16-bit fields
// (0xFFFF = none).  One block per 64-column strip; its 16 waves split the
// rows; class bits live in LDS.
// --------------------------------------------------------------------------
constexpr uint32_t NONE16 = 0xFFFFu;

__global__ __launch_bounds__(1024) void k_edt_cols(const float *__restrict__ phi, const uint8_t *__restrict__ mask,
                                                   int N, uint32_t *__restrict__ gout) {
    __shared__ uint32_t bits[ILT_MAX_N / 32][64];
    __shared__ int fl[16][64][4];   // first0, last0, first1, last1 per segment
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x = blockIdx.x * 64 + lane;
    const bool xok = x < N;
    const int seg = (N + 15) / 16;
    const int ylo = w * seg, yhi = min(N, ylo + seg);
    // class bits, 32 rows per word; each wave owns whole words when seg % 32 == 0,
    // otherwise words are assembled after a barrier from per-row bytes below.
    for (int e = threadIdx.x; e < (ILT_MAX_N / 32) * 64; e += 1024) (&bits[0][0])[e] = 0u;
    __syncthreads();
    int f0 = -1, l0 = -1, f1 = -1, l1 = -1;
    for (int y = ylo; y < yhi; ++y) {
        int cls = 0;
        if (xok) cls = phi ? (phi[(size_t)y * N + x] <= 0.f) : (mask[(size_t)y * N + x] != 0);
        if (cls) { if (f1 < 0) f1 = y; l1 = y; }
        else { if (f0 < 0) f0 = y; l0 = y; }
        // set bit y of this lane's column (atomics on LDS keep words shared by
        // two segments correct)
        if (cls) atomicOr(&bits[y >> 5][lane], 1u << (y & 31));
    }
    fl[w][lane][0] = f0; fl[w][lane][1] = l0; fl[w][lane][2] = f1; fl[w][lane][3] = l1;
    __syncthreads();
    if (!xok || ylo >= yhi) return;
    // nearest pixel of each class above / below this segment
    int up0 = -1, up1 = -1, dn0 = -1, dn1 = -1;
    for (int v = w - 1; v >= 0 && (up0 < 0 || up1 < 0); --v) {
        if (up0 < 0 && fl[v][lane][1] >= 0) up0 = fl[v][lane][1];
        if (up1 < 0 && fl[v][lane][3] >= 0) up1 = fl[v][lane][3];
    }
    for (int v = w + 1; v < 16 && (dn0 < 0 || dn1 < 0); ++v) {
        if (dn0 < 0 && fl[v][lane][0] >= 0) dn0 = fl[v][lane][0];
        if (dn1 < 0 && fl[v][lane][2] >= 0) dn1 = fl[v][lane][2];
    }
    // downward sweep: distance to the nearest pixel above (or at) y
    int p0 = up0, p1 = up1;
    for (int y = ylo; y < yhi; ++y) {
        const int cls = (bits[y >> 5][lane] >> (y & 31)) & 1;
        if (cls) p1 = y; else p0 = y;
        const uint32_t d0 = p0 >= 0 ? (uint32_t)(y - p0) : NONE16;
        const uint32_t d1 = p1 >= 0 ? (uint32_t)(y - p1) : NONE16;
        gout[(size_t)y * N + x] = d0 | (d1 << 16);
    }
    // upward sweep: merge with the nearest pixel below
    int n0 = dn0, n1 = dn1;
    for (int y = yhi - 1; y >= ylo; --y) {
        const int cls = (bits[y >> 5][lane] >> (y & 31)) & 1;
        if (cls) n1 = y; else n0 = y;
        uint32_t v = gout[(size_t)y * N + x];
        uint32_t d0 = v & 0xFFFFu, d1 = v >> 16;
        if (n0 >= 0) d0 = min(d0, (uint32_t)(n0 - y));
        if (n1 >= 0) d1 = min(d1, (uint32_t)(n1 - y));
        gout[(size_t)y * N + x] = d0 | (d1 << 16);
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
// f = g_c^2 (2^30 stand-in where the column has no class-c pixel).  The
// cost matrix is Monge, so the leftmost minimiser is non-decreasing in x;
// minimisers are found by bisection levels over x, each query scanning only
// the candidate range between its neighbours' minimisers.  One wave per row.
constexpr int FBIG = 1 << 30;

__device__ __forceinline__ void argmin_combine(int &bv, int &bi, int ov, int oi) {
    if (ov < bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
}

__device__ void row_transform(const int *f, int16_t *arg, int N, int lane) {
    // full scans for x = 0 and x = N-1
    for (int q = 0; q < 2; ++q) {
        const int x = q ? N - 1 : 0;
        int bv = 0x7FFFFFFF, bi = 0x7FFFFFFF;
        for (int c = lane; c < N; c += 64) {
            const int v = f[c] + (x - c) * (x - c);
            argmin_combine(bv, bi, v, c);
        }
        for (int o = 32; o > 0; o >>= 1) {
            const int ov = __shfl_xor(bv, o), oi = __shfl_xor(bi, o);
            argmin_combine(bv, bi, ov, oi);
        }
        if (lane == 0) arg[x] = (int16_t)bi;
        __syncthreads();
    }
    int L = 1;
    while (L < N - 1) L <<= 1;
    for (int s = L >> 1; s >= 1; s >>= 1) {
        // queries x = s, 3s, 5s, ... < N-1
        const int nq = (N - 1 > s) ? ((N - 1 - s + 2 * s - 1) / (2 * s)) : 0;
        if (nq <= 0) continue;
        int gq = 1;                       // lanes per query (power of two)
        while (gq * 2 * nq <= 64 && gq < 64) gq <<= 1;
        const int per_pass = 64 / gq;
        for (int q0 = 0; q0 < nq; q0 += per_pass) {
            const int qi = q0 + lane / gq;
            const int sub = lane % gq;
            int bv = 0x7FFFFFFF, bi = 0x7FFFFFFF;
            int x = -1;
            if (qi < nq) {
                x = s * (2 * qi + 1);
                const int lo = arg[x - s];
                const int hi = arg[min(x + s, N - 1)];
                for (int c = lo + sub; c <= hi; c += gq) {
                    const int v = f[c] + (x - c) * (x - c);
                    argmin_combine(bv, bi, v, c);
                }
            }
            for (int o = gq >> 1; o > 0; o >>= 1) {
                const int ov = __shfl_xor(bv, o), oi = __shfl_xor(bi, o);
                argmin_combine(bv, bi, ov, oi);
            }
            if (qi < nq && sub == 0) arg[x] = (int16_t)bi;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void k_edt_rows(const uint32_t *__restrict__ gin, int N, float d_lower,
                                                 float d_upper, float *__restrict__ phi_out,
                                                 int *__restrict__ sqdist) {
    extern __shared__ unsigned char smem[];
    uint32_t *gr = reinterpret_cast<uint32_t *>(smem);            // [N]
    int *f = reinterpret_cast<int *>(gr + N);                     // [N]
    int16_t *arg = reinterpret_cast<int16_t *>(f + N);            // [N]
    const int y = blockIdx.x, lane = threadIdx.x;
    for (int x = lane; x < N; x += 64) gr[x] = gin[(size_t)y * N + x];
    __syncthreads();
    for (int c = 0; c < 2; ++c) {
        for (int x = lane; x < N; x += 64) {
            const uint32_t g = c ? (gr[x] >> 16) : (gr[x] & 0xFFFFu);
            f[x] = (g == NONE16) ? FBIG : (int)(g * g);
        }
        __syncthreads();
        row_transform(f, arg, N, lane);
        for (int x = lane; x < N; x += 64) {
            const int a = arg[x];
            const int D = f[a] + (x - a) * (x - a);
            const bool none = D >= FBIG;
            const bool inside = (gr[x] >> 16) == 0;        // distance 0 to class 1
            if (sqdist) {
                // c = 1: distance to inside pixels (D_in); c = 0: to outside (D_out)
                int *dst = sqdist + (size_t)(1 - c) * N * N;
                dst[(size_t)y * N + x] = none ? 0x7FFFFFFF : D;
            }
            if (c == 0 && inside) {          // inside pixel: 1/2 - sqrt(D_out)
                const float v = none ? d_lower : -sqrt_minus_half(D);
                phi_out[(size_t)y * N + x] = fminf(fmaxf(v, d_lower), d_upper);
            }
            if (c == 1 && !inside) {         // outside pixel: sqrt(D_in) - 1/2
                const float v = none ? d_upper : sqrt_minus_half(D);
                phi_out[(size_t)y * N + x] = fminf(fmaxf(v, d_lower), d_upper);
            }
        }
        __syncthreads();
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
    return (int)std::min<size_t>(MAX_RBLK, (npix + 4095) / 4096);
}

hipError_t launch_resist(ilt_ctx *c, const float *I, const uint8_t *target, const resist_args &ra, float *G,
                         double *part) {
    const size_t npix = (size_t)c->N * c->N;
    const int nblk = resist_blocks(c);
    k_resist<<<nblk, RB, 0, c->stream>>>(I, npix, target, ra, npix, chunk_of(npix, nblk), G, part);
    return hipGetLastError();
}

hipError_t launch_finish_resist(ilt_ctx *c, const double *part, int nblk, double *scal, double *stats4) {
    k_finish_resist<<<1, RB, 0, c->stream>>>(part, nblk, scal, stats4);
    return hipGetLastError();
}

int gradmax_blocks(const ilt_ctx *c) { return resist_blocks(c); }

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
    k_edt_cols<<<(N + 63) / 64, 1024, 0, c->stream>>>(phi, mask, N, c->edtg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t sm = (size_t)N * (4 + 4 + 2);
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
