// Edge placement error of a printed pattern against its target (a metric of
// the results; the paper scores masks by L2 and PVBand, Sec. II-C, and names
// no EPE, so this reading is the library's own).
//
// Sample points lie every step_nm along each straight edge of the Manhattan
// target, starting end_nm from the edge's ends.  At each, the signed number
// of pixels from the target edge to the boundary of the print, along the
// edge's outward normal, is found on the pixel grid (positive: the print
// extends beyond the target), searched within ceil(search_nm / pitch)
// pixels and clipped to +-search_nm.  The print is [I >= I_th] (the hard
// threshold of Sec. II-C).
//
// One block: each thread takes whole boundary lines (rows, then columns),
// walks the edge runs of its lines and keeps its own sums; the block then
// adds them in a fixed order, so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cmath>

#include "ilt_internal.h"

namespace {

constexpr int EB = 1024;

struct epe_acc {
    double n, sum_abs, max_abs, over;
};

// the printed pixel at (row r, column t) of a horizontal boundary, or at
// (t, r) of a vertical one; outside the image nothing is printed
__device__ __forceinline__ bool printed(const float *I, float i_th, int N, bool horiz, int r, int t) {
    if (r < 0 || r >= N) return false;
    const size_t p = horiz ? (size_t)r * N + t : (size_t)t * N + r;
    return I[p] >= i_th;
}

__device__ __forceinline__ bool target_at(const unsigned char *Z, int N, bool horiz, int r, int t) {
    if (r < 0 || r >= N) return false;
    const size_t p = horiz ? (size_t)r * N + t : (size_t)t * N + r;
    return Z[p] != 0;
}

__global__ __launch_bounds__(EB) void k_epe(const unsigned char *__restrict__ Z, const float *__restrict__ I,
                                            float i_th, int N, double pitch, double step_nm, double end_nm,
                                            double search_nm, double limit_nm, double *__restrict__ out) {
    __shared__ double red[EB];
    const int reach = (int)ceil(search_nm / pitch);
    epe_acc a{0.0, 0.0, 0.0, 0.0};
    // boundary lines: L in [0, N] between rows (or columns) L - 1 and L; two
    // orientations
    for (int id = threadIdx.x; id < 2 * (N + 1); id += EB) {
        const bool horiz = id <= N;
        const int L = horiz ? id : id - (N + 1);
        // runs of each sign along the line: +1 where the target lies on the
        // lower-index side only, -1 where it lies on the higher-index side only
        for (int sign = 1; sign >= -1; sign -= 2) {
            int t = 0;
            while (t < N) {
                const bool above = target_at(Z, N, horiz, L - 1, t), below = target_at(Z, N, horiz, L, t);
                const bool on = sign > 0 ? (above && !below) : (!above && below);
                if (!on) {
                    ++t;
                    continue;
                }
                const int a0 = t;
                while (t < N) {
                    const bool ab = target_at(Z, N, horiz, L - 1, t), be = target_at(Z, N, horiz, L, t);
                    if (!(sign > 0 ? (ab && !be) : (!ab && be))) break;
                    ++t;
                }
                const int b0 = t;                           // run [a0, b0)
                const double length = (b0 - a0) * pitch;
                for (double pos = end_nm; pos <= length - end_nm + 1e-9; pos += step_nm) {
                    const int tt = a0 + (int)(pos / pitch);
                    // k-th pixel outward (k >= 0) or inward (k < 0) across the line
                    auto pix = [&](int k) {
                        const int r = sign > 0 ? L + k : L - 1 - k;
                        return printed(I, i_th, N, horiz, r, tt);
                    };
                    int d;
                    if (pix(0)) {
                        int k = 0;
                        while (k < reach && pix(k)) ++k;
                        d = k;
                    } else if (!pix(-1)) {
                        int k = -1;
                        while (k >= -reach && !pix(k)) --k;
                        d = k < -reach ? -reach : k + 1;
                    } else {
                        d = 0;
                    }
                    const double v = fmin(fmax(d * pitch, -search_nm), search_nm);
                    const double av = fabs(v);
                    a.n += 1.0;
                    a.sum_abs += av;
                    a.max_abs = fmax(a.max_abs, av);
                    a.over += av > limit_nm ? 1.0 : 0.0;
                }
            }
        }
    }
    // fixed-order block reductions
    double r4[4] = {a.n, a.sum_abs, a.max_abs, a.over};
    for (int q = 0; q < 4; ++q) {
        red[threadIdx.x] = r4[q];
        __syncthreads();
        for (int o = EB / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o)
                red[threadIdx.x] = q == 2 ? fmax(red[threadIdx.x], red[threadIdx.x + o])
                                          : red[threadIdx.x] + red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) r4[q] = red[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = r4[0];
        out[1] = r4[0] > 0.0 ? r4[1] / r4[0] : 0.0;
        out[2] = r4[2];
        out[3] = r4[3];
    }
}

}  // namespace

hipError_t launch_epe(const unsigned char *Z, const float *I, float i_th, int N, double pitch, double step_nm,
                      double end_nm, double search_nm, double limit_nm, double *out, hipStream_t st) {
    k_epe<<<1, EB, 0, st>>>(Z, I, i_th, N, pitch, step_nm, end_nm, search_nm, limit_nm, out);
    return hipGetLastError();
}
