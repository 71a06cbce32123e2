// The DSO loop in FP64 (ILT_FP64): every step of an iteration in double
// precision on the vector units (this part runs FP64 vector and matrix
// arithmetic at the same rate, so the pruned transforms are plain FMA loops
// with their operands staged in LDS), for an exact-trajectory comparison of
// the whole loop with an FP64 reference.
//
//   spectrum   S = A M A^T              (Sec. II-B; M = [phi <= 0], Sec. II-A)
//   fields     E_k = N^-2 A^H (H_k . S) conj(A),  I_s = sum_k w_k |E_k|^2
//   resist     Z_c, L_DSO, G_s, L2 / PVB (Sec. III-A, Sec. II-C)
//   adjoint    W = sum_k w_k conj(H_k) . N^-2 A (G_s . E_k) A^T,
//              g = 2 Re(A^H W conj(A))  (Sec. III-A, ILT gradient)
//   step       phi += dt (g |grad phi| + lambda K), dt = eta / max|g|
//              (Sec. II-A, III-A numerics, III-C CFL)
//   TSDF       re-initialisation through the exact EDT (Alg. 1)
//
// Reductions are two-stage in a fixed order, so results are reproducible
// bit for bit.
#include <algorithm>
#include <cmath>

#include "ilt_internal.h"

namespace {

constexpr int FB64 = 256;                   // threads per block

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// fixed-order block sum of 256 threads: a shuffle tree per wave, then the
// four waves in order; every thread receives the result
__device__ __forceinline__ double bsum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double bmax(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    __syncthreads();
    return r;
}

// Row transform: out[r][b] = sum_x v(r, x) A[b][x] for rows r of a real
// image (PHI: v = [src <= 0], else v = src).  Block = one row; the b loop
// runs in groups of 4 window columns, each a fixed-order block sum.
template <bool PHI>
__global__ __launch_bounds__(FB64) void k64_rows_real(const double *__restrict__ src, int N, int P,
                                                      const double2 *__restrict__ A, double2 *__restrict__ out) {
    __shared__ double sh[4];
    const int r = blockIdx.x;
    const double *row = src + (size_t)r * N;
    for (int b0 = 0; b0 < P; b0 += 4) {
        double2 acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = make_double2(0.0, 0.0);
        for (int x = threadIdx.x; x < N; x += FB64) {
            const double v = PHI ? (row[x] <= 0.0 ? 1.0 : 0.0) : row[x];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (b0 + j < P) {
                    const double2 a = A[(size_t)(b0 + j) * N + x];
                    acc[j].x = fma(v, a.x, acc[j].x);
                    acc[j].y = fma(v, a.y, acc[j].y);
                }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double re = bsum(acc[j].x, sh), im = bsum(acc[j].y, sh);
            if (threadIdx.x == 0 && b0 + j < P) out[(size_t)r * P + b0 + j] = make_double2(re, im);
        }
    }
}

// Column transform of a [N][P] complex array: out[a][b] = scale * sum_y
// A[a][y] T[y][b].  Block = one (a, b).
__global__ __launch_bounds__(FB64) void k64_cols(const double2 *__restrict__ T, int N, int P,
                                                 const double2 *__restrict__ A, double scale,
                                                 double2 *__restrict__ out) {
    __shared__ double sh[4];
    const int a = blockIdx.x / P, b = blockIdx.x % P;
    double re = 0.0, im = 0.0;
    for (int y = threadIdx.x; y < N; y += FB64) {
        const double2 p = cmul(A[(size_t)a * N + y], T[(size_t)y * P + b]);
        re += p.x;
        im += p.y;
    }
    re = bsum(re, sh);
    im = bsum(im, sh);
    if (threadIdx.x == 0) out[(size_t)a * P + b] = make_double2(scale * re, scale * im);
}

// Window -> rows: Y[s][k][a][x] = N^-2 sum_b (H[s][k][a][b] S[a][b]) conj(A[b][x])
// for the sets [s0, s1).  Thread = one x of one (s, k, a).
__global__ __launch_bounds__(FB64) void k64_make_Y(const double2 *__restrict__ S, const double2 *__restrict__ H,
                                                   int s0, int K, int P, int N, const double2 *__restrict__ A,
                                                   double inv_n2, double2 *__restrict__ Y) {
    __shared__ double2 u[64];
    const int s = s0 + blockIdx.z, k = blockIdx.y / P, a = blockIdx.y % P;
    const double2 *h = H + ((size_t)s * K + k) * P * P + (size_t)a * P;
    if (threadIdx.x < P) u[threadIdx.x] = cmul(h[threadIdx.x], S[(size_t)a * P + threadIdx.x]);
    __syncthreads();
    const int x = blockIdx.x * FB64 + threadIdx.x;
    if (x >= N) return;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < P; ++b) {
        const double2 p = cmulc(u[b], A[(size_t)b * N + x]);
        re += p.x;
        im += p.y;
    }
    Y[(((size_t)s * K + k) * P + a) * N + x] = make_double2(inv_n2 * re, inv_n2 * im);
}

// Field of kernel k at pixel (y, x): E = sum_a conj(A[a][y]) Y[a][x]
__device__ __forceinline__ double2 field_at(const double2 *__restrict__ Yk, const double2 *ay, int P, int N, int x) {
    double re = 0.0, im = 0.0;
    for (int a = 0; a < P; ++a) {
        const double2 p = cmulc(Yk[(size_t)a * N + x], ay[a]);
        re += p.x;
        im += p.y;
    }
    return make_double2(re, im);
}

// I[s - s0][y][x] = sum_k w[s][k] |E_k(y, x)|^2.  Block = 256 pixels of one
// row of one set; conj(A[.][y]) of the row staged in LDS.
__global__ __launch_bounds__(FB64) void k64_image(const double2 *__restrict__ Y, const double *__restrict__ w,
                                                  int s0, int K, int P, int N, const double2 *__restrict__ A,
                                                  double *__restrict__ I) {
    __shared__ double2 ay[64];
    const int s = s0 + blockIdx.z, y = blockIdx.y;
    if (threadIdx.x < P) ay[threadIdx.x] = A[(size_t)threadIdx.x * N + y];
    __syncthreads();
    const int x = blockIdx.x * FB64 + threadIdx.x;
    if (x >= N) return;
    double acc = 0.0;
    for (int k = 0; k < K; ++k) {
        const double2 e = field_at(Y + ((size_t)s * K + k) * P * N, ay, P, N, x);
        acc += w[(size_t)s * K + k] * (e.x * e.x + e.y * e.y);
    }
    I[((size_t)blockIdx.z * N + y) * N + x] = acc;
}

// Resist in FP64 (Sec. III-A): per corner Z = 1/(1 + exp(-sigma_z (d I - I_th))),
// loss += omega (Z - Zt)^2, G_s += omega 2 sigma_z d (Z - Zt) Z (1 - Z); the
// binary prints for L2 (corner 0) and PVBand (corners 1, 2).  Block partials
// {loss, l2, pvb, non-finite}.
struct resist64_args {
    int n_corners;
    int cset[4];
    double dose[4], omega[4];
    double sigma_z, i_th;
    int set_used[ILT_MAX_SETS];
};

__global__ __launch_bounds__(FB64) void k64_resist(const double *__restrict__ I, const uint8_t *__restrict__ target,
                                                   resist64_args ra, size_t npix, size_t chunk,
                                                   double *__restrict__ G, double *__restrict__ part) {
    __shared__ double sh[4];
    const size_t lo = (size_t)blockIdx.x * chunk, hi = min(npix, lo + chunk);
    double loss = 0.0, l2 = 0.0, pvb = 0.0, bad = 0.0;
    for (size_t p = lo + threadIdx.x; p < hi; p += FB64) {
        const double zt = target[p] ? 1.0 : 0.0;
        double gs[ILT_MAX_SETS] = {0.0, 0.0, 0.0, 0.0};
        bool pr[4] = {false, false, false, false};
        double lp = 0.0;
        for (int c = 0; c < ra.n_corners; ++c) {
            const int s = ra.cset[c];
            const double di = ra.dose[c] * I[(size_t)s * npix + p];
            const double z = 1.0 / (1.0 + exp(-ra.sigma_z * (di - ra.i_th)));
            const double r = z - zt;
            lp += ra.omega[c] * r * r;
            gs[s] += ra.omega[c] * 2.0 * ra.sigma_z * ra.dose[c] * r * z * (1.0 - z);
            pr[c] = di >= ra.i_th;
        }
        loss += lp;
        bad += isfinite(lp) ? 0.0 : 1.0;
        l2 += (pr[0] != (zt != 0.0)) ? 1.0 : 0.0;
        if (ra.n_corners >= 3) pvb += (pr[1] != pr[2]) ? 1.0 : 0.0;
        for (int s = 0; s < ILT_MAX_SETS; ++s)
            if (ra.set_used[s]) G[(size_t)s * npix + p] = gs[s];
    }
    loss = bsum(loss, sh);
    l2 = bsum(l2, sh);
    pvb = bsum(pvb, sh);
    bad = bsum(bad, sh);
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x + 0] = loss;
        part[4 * blockIdx.x + 1] = l2;
        part[4 * blockIdx.x + 2] = pvb;
        part[4 * blockIdx.x + 3] = bad;
    }
}

// Adjoint, rows: Q[s][k][y][b] = sum_x (G_s . E_k)[y][x] A[b][x] (G holds
// the sets from s0 on), the field recomputed from Y.  Block = one (y, k, s): X = G . E for the row in LDS,
// then the window columns in groups of 4 with fixed-order block sums.
__global__ __launch_bounds__(FB64) void k64_adj_rows(const double2 *__restrict__ Y, const double *__restrict__ G,
                                                     int s0, int K, int P, int N, const double2 *__restrict__ A,
                                                     double2 *__restrict__ Q) {
    extern __shared__ double2 xrow[];          // [N]
    __shared__ double2 ay[64];
    __shared__ double sh[4];
    const int y = blockIdx.x, k = blockIdx.y, s = s0 + blockIdx.z;
    if (threadIdx.x < P) ay[threadIdx.x] = A[(size_t)threadIdx.x * N + y];
    __syncthreads();
    const double2 *Yk = Y + ((size_t)s * K + k) * P * N;
    const double *Gr = G + ((size_t)blockIdx.z * N + y) * N;
    for (int x = threadIdx.x; x < N; x += FB64) {
        const double2 e = field_at(Yk, ay, P, N, x);
        const double gv = Gr[x];
        xrow[x] = make_double2(gv * e.x, gv * e.y);
    }
    __syncthreads();
    double2 *q = Q + (((size_t)s * K + k) * N + y) * P;
    for (int b0 = 0; b0 < P; b0 += 4) {
        double2 acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = make_double2(0.0, 0.0);
        for (int x = threadIdx.x; x < N; x += FB64) {
            const double2 v = xrow[x];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (b0 + j < P) {
                    const double2 p = cmul(v, A[(size_t)(b0 + j) * N + x]);
                    acc[j].x += p.x;
                    acc[j].y += p.y;
                }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double re = bsum(acc[j].x, sh), im = bsum(acc[j].y, sh);
            if (threadIdx.x == 0 && b0 + j < P) q[b0 + j] = make_double2(re, im);
        }
    }
}

// Adjoint, columns and the window sum: W[a][b] = sum over sets s in
// [s0, s1) and kernels k of w[s][k] conj(H[s][k][a][b]) N^-2 sum_y A[a][y]
// Q[s][k][y][b].  Block = one (a, b); sets and kernels in a fixed order.
__global__ __launch_bounds__(FB64) void k64_adj_cols(const double2 *__restrict__ Q, const double2 *__restrict__ H,
                                                     const double *__restrict__ w, int s0, int s1, int K, int P,
                                                     int N, const double2 *__restrict__ A, double inv_n2,
                                                     double2 *__restrict__ W) {
    __shared__ double sh[4];
    const int a = blockIdx.x / P, b = blockIdx.x % P;
    double wre = 0.0, wim = 0.0;
    for (int s = s0; s < s1; ++s)
        for (int k = 0; k < K; ++k) {
            const double2 *q = Q + ((size_t)s * K + k) * N * P;
            double re = 0.0, im = 0.0;
            for (int y = threadIdx.x; y < N; y += FB64) {
                const double2 p = cmul(A[(size_t)a * N + y], q[(size_t)y * P + b]);
                re += p.x;
                im += p.y;
            }
            re = bsum(re, sh) * inv_n2;
            im = bsum(im, sh) * inv_n2;
            // w conj(H) V
            const double2 h = H[((size_t)s * K + k) * P * P + (size_t)a * P + b];
            const double2 t = cmulc(make_double2(re, im), h);
            wre += w[(size_t)s * K + k] * t.x;
            wim += w[(size_t)s * K + k] * t.y;
        }
    if (threadIdx.x == 0) W[(size_t)a * P + b] = make_double2(wre, wim);
}

// Z[a][x] = sum_b W[a][b] conj(A[b][x])
__global__ __launch_bounds__(FB64) void k64_window_rows(const double2 *__restrict__ W, int P, int N,
                                                        const double2 *__restrict__ A, double2 *__restrict__ Z) {
    const int a = blockIdx.y, x = blockIdx.x * FB64 + threadIdx.x;
    if (x >= N) return;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < P; ++b) {
        const double2 p = cmulc(W[(size_t)a * P + b], A[(size_t)b * N + x]);
        re += p.x;
        im += p.y;
    }
    Z[(size_t)a * N + x] = make_double2(re, im);
}

// g[y][x] = 2 Re sum_a conj(A[a][y]) Z[a][x], and per-block max |g|
// (non-finite -> +inf).  Block = 256 pixels of one row.
__global__ __launch_bounds__(FB64) void k64_gradient(const double2 *__restrict__ Z, int P, int N,
                                                     const double2 *__restrict__ A, double *__restrict__ g,
                                                     double *__restrict__ maxpart) {
    __shared__ double2 ay[64];
    __shared__ double sh[4];
    const int y = blockIdx.y;
    if (threadIdx.x < P) ay[threadIdx.x] = A[(size_t)threadIdx.x * N + y];
    __syncthreads();
    const int x = blockIdx.x * FB64 + threadIdx.x;
    double m = 0.0;
    if (x < N) {
        double re = 0.0;
        for (int a = 0; a < P; ++a) {
            const double2 z = Z[(size_t)a * N + x];
            re += z.x * ay[a].x + z.y * ay[a].y;        // Re(conj(A) Z)
        }
        const double gv = 2.0 * re;
        g[(size_t)y * N + x] = gv;
        m = isfinite(gv) ? fabs(gv) : INFINITY;
    }
    m = bmax(m, sh);
    if (threadIdx.x == 0) maxpart[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = m;
}

// CFL step in FP64 (Sec. III-C): dt = eta / max|g|, capped at dt_max; or fixed.
__global__ __launch_bounds__(FB64) void k64_finish_dt(const double *__restrict__ part, int nblk, int dt_mode,
                                                      double eta, double dt_max, double *__restrict__ scal) {
    __shared__ double sh[4];
    double m = 0.0;
    for (int b = threadIdx.x; b < nblk; b += FB64) m = fmax(m, part[b]);
    m = bmax(m, sh);
    if (threadIdx.x == 0) {
        double dt;
        if (dt_mode == 1) {
            dt = eta;
        } else if (m > 0.0 && isfinite(m)) {
            dt = eta / m;
            if (dt_max > 0.0) dt = fmin(dt, dt_max);
        } else {
            dt = dt_max > 0.0 && m == 0.0 ? dt_max : 0.0;
        }
        scal[SC_MV] = m;
        scal[SC_DT] = dt;
        if (!isfinite(m)) {
            scal[SC_NONFIN] += 1.0;
            scal[SC_BAD] += 1.0;
        }
    }
}

// Level-set step in FP64: phi' = phi + dt (g |grad phi| + lambda K), central
// differences with replicated borders (Sec. III-A numerics).  Block = 256
// pixels of one row; part[2 b] = flips, part[2 b + 1] = non-finite outputs.
__global__ __launch_bounds__(FB64) void k64_levelset(const double *__restrict__ phi, const double *__restrict__ vel,
                                                     double lam, double eps_kappa, const double *__restrict__ scal,
                                                     int N, double *__restrict__ out, double *__restrict__ part) {
    __shared__ double sh[4];
    const int y = blockIdx.y, x = blockIdx.x * FB64 + threadIdx.x;
    double flips = 0.0, bad = 0.0;
    if (x < N) {
        const double dt = scal[SC_DT];
        const int ym = max(y - 1, 0), yp = min(y + 1, N - 1), xm = max(x - 1, 0), xp = min(x + 1, N - 1);
        const double c = phi[(size_t)y * N + x];
        const double vxp = phi[(size_t)y * N + xp], vxm = phi[(size_t)y * N + xm];
        const double vyp = phi[(size_t)yp * N + x], vym = phi[(size_t)ym * N + x];
        const double vpp = phi[(size_t)yp * N + xp], vpm = phi[(size_t)yp * N + xm];
        const double vmp = phi[(size_t)ym * N + xp], vmm = phi[(size_t)ym * N + xm];
        const double px = 0.5 * (vxp - vxm);
        const double py = 0.5 * (vyp - vym);
        const double pxx = vxp + vxm - 2.0 * c;
        const double pyy = vyp + vym - 2.0 * c;
        const double pxy = 0.25 * ((vpp - vpm) - (vmp - vmm));
        const double g2 = px * px + py * py;
        const double num = pxx * py * py - 2.0 * px * py * pxy + pyy * px * px;
        const double K = num / (g2 + eps_kappa);
        const double nv = c + dt * (vel[(size_t)y * N + x] * sqrt(g2) + lam * K);
        out[(size_t)y * N + x] = nv;
        flips = ((nv <= 0.0) != (c <= 0.0)) ? 1.0 : 0.0;
        bad = isfinite(nv) ? 0.0 : 1.0;
    }
    flips = bsum(flips, sh);
    bad = bsum(bad, sh);
    if (threadIdx.x == 0) {
        const size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        part[2 * b] = flips;
        part[2 * b + 1] = bad;
    }
}

__global__ void k64_copy(double *__restrict__ dst, const double *__restrict__ src, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

size_t chunk64(size_t npix, int nblk) { return (npix + nblk - 1) / nblk; }

}  // namespace

int resist64_blocks(const ilt_ctx *c) {
    const size_t npix = (size_t)c->N * c->N;
    return (int)std::min<size_t>(2048, (npix + 2047) / 2048);
}

int rowblk64(const ilt_ctx *c) { return (c->N + FB64 - 1) / FB64; }

hipError_t launch64_spectrum(ilt_ctx *c, const double *src, int src_is_phi) {
    const int N = c->N, P = c->P;
    if (src_is_phi) k64_rows_real<true><<<N, FB64, 0, c->stream>>>(src, N, P, c->A64, c->T64);
    else k64_rows_real<false><<<N, FB64, 0, c->stream>>>(src, N, P, c->A64, c->T64);
    k64_cols<<<P * P, FB64, 0, c->stream>>>(c->T64, N, P, c->A64, 1.0, c->S64);
    return hipGetLastError();
}

hipError_t launch64_make_Y(ilt_ctx *c, int s0, int s1) {
    const int N = c->N, P = c->P, K = c->K;
    const double inv = 1.0 / ((double)N * (double)N);
    k64_make_Y<<<dim3(rowblk64(c), K * P, s1 - s0), FB64, 0, c->stream>>>(c->S64, c->H64, s0, K, P, N, c->A64, inv,
                                                                          c->Y64);
    return hipGetLastError();
}

// I: the images of sets [s0, s1), [s1 - s0][N][N]
hipError_t launch64_image(ilt_ctx *c, int s0, int s1, double *I) {
    const int N = c->N, P = c->P, K = c->K;
    hipError_t e = launch64_make_Y(c, s0, s1);
    if (e != hipSuccess) return e;
    k64_image<<<dim3(rowblk64(c), N, s1 - s0), FB64, 0, c->stream>>>(c->Y64, c->w64, s0, K, P, N, c->A64, I);
    return hipGetLastError();
}

hipError_t launch64_resist(ilt_ctx *c, const double *I, const uint8_t *target, const ilt_params *p, double *G,
                           double *part) {
    resist64_args ra{};
    ra.n_corners = p->n_corners;
    for (int i = 0; i < 4; ++i) {
        ra.cset[i] = i < p->n_corners ? p->corners[i].set : 0;
        ra.dose[i] = i < p->n_corners ? (double)p->corners[i].dose : 1.0;
        ra.omega[i] = i < p->n_corners ? (double)p->corners[i].omega : 0.0;
    }
    for (int i = 0; i < p->n_corners; ++i) ra.set_used[p->corners[i].set] = 1;
    ra.sigma_z = p->sigma_z;
    ra.i_th = p->i_th;
    const size_t npix = (size_t)c->N * c->N;
    const int nblk = resist64_blocks(c);
    k64_resist<<<nblk, FB64, 0, c->stream>>>(I, target, ra, npix, chunk64(npix, nblk), G, part);
    return hipGetLastError();
}

// G: dL/dI of sets [s0, s1), [s1 - s0][N][N]; needs Y of those sets
hipError_t launch64_adjoint(ilt_ctx *c, const double *G, int s0, int s1) {
    const int N = c->N, P = c->P, K = c->K;
    k64_adj_rows<<<dim3(N, K, s1 - s0), FB64, (size_t)N * sizeof(double2), c->stream>>>(c->Y64, G, s0, K, P, N,
                                                                                       c->A64, c->Q64);
    k64_adj_cols<<<P * P, FB64, 0, c->stream>>>(c->Q64, c->H64, c->w64, s0, s1, K, P, N, c->A64,
                                                1.0 / ((double)N * (double)N), c->W64);
    return hipGetLastError();
}

int launch64_gradient(ilt_ctx *c, double *g, double *maxpart, hipError_t *err) {
    const int N = c->N, P = c->P;
    k64_window_rows<<<dim3(rowblk64(c), P), FB64, 0, c->stream>>>(c->W64, P, N, c->A64, c->Z64);
    k64_gradient<<<dim3(rowblk64(c), N), FB64, 0, c->stream>>>(c->Z64, P, N, c->A64, g, maxpart);
    *err = hipGetLastError();
    return rowblk64(c) * N;
}

hipError_t launch64_finish_dt(ilt_ctx *c, const double *part, int nblk, const ilt_params *p) {
    k64_finish_dt<<<1, FB64, 0, c->stream>>>(part, nblk, p->dt_mode, (double)p->eta, (double)p->dt_max, c->scal);
    return hipGetLastError();
}

int launch64_levelset(ilt_ctx *c, const double *phi, const double *vel, const ilt_params *p, double *out,
                      double *part, hipError_t *err) {
    const int N = c->N;
    k64_levelset<<<dim3(rowblk64(c), N), FB64, 0, c->stream>>>(phi, vel, (double)p->lambda, (double)p->eps_kappa,
                                                               c->scal, N, out, part);
    *err = hipGetLastError();
    return rowblk64(c) * N;
}

hipError_t launch64_copy(ilt_ctx *c, double *dst, const double *src, size_t n) {
    k64_copy<<<1024, 256, 0, c->stream>>>(dst, src, n);
    return hipGetLastError();
}
