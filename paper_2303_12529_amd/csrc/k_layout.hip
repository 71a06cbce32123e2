// Full-layout tiling and the mask-fracturing shot count.
//
// Tiling: N x N tiles whose cores (C = N - 2 halo pixels square) cover the
// layout at stride C; tile (i, j) starts at layout (i C - halo, j C - halo)
// and reads zero outside the layout.  Extraction and stitching are plain
// gathers, one thread per output pixel (row-major, coalesced).
//
// Shot count (Sec. II-C, the number of rectangles of an exact fracturing of
// the mask): a maximal run of ones in a row continues the rectangle of the
// identical run (same first and last column) in the row above, otherwise it
// starts a new rectangle.  Per row the count is a left-to-right scan over
// (this row, row above) with two bits of state; the same scan down each
// column (against the column to its left) gives the fracturing with rows
// and columns exchanged.  Counts are summed exactly in 64-bit integers.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ilt_internal.h"

namespace {

// ---------------------------------------------------------------- tiling

__global__ void k_layout_extract(const unsigned char *__restrict__ layout, int H, int W, int N, int halo, int cols,
                                 long long total, unsigned char *__restrict__ tiles) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= total) return;
    const long long NN = (long long)N * N;
    const int t = (int)(id / NN);
    const int rem = (int)(id - (long long)t * NN);
    const int r = rem / N, c = rem - (rem / N) * N;
    const int C = N - 2 * halo;
    const int y = (t / cols) * C - halo + r;
    const int x = (t % cols) * C - halo + c;
    tiles[id] = (y >= 0 && y < H && x >= 0 && x < W) ? layout[(size_t)y * W + x] : (unsigned char)0;
}

__global__ void k_layout_stitch(const float *__restrict__ tiles, int H, int W, int N, int halo, int cols,
                                float *__restrict__ out) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)H * W) return;
    const int y = (int)(id / W), x = (int)(id - (long long)(id / W) * W);
    const int C = N - 2 * halo;
    const int i = y / C, j = x / C;
    const int r = y - i * C + halo, c = x - j * C + halo;
    out[id] = tiles[((size_t)(i * cols + j) * N + r) * N + c];
}

// ---------------------------------------------------------------- shot count

template <bool PHI>
__device__ __forceinline__ unsigned pix(const void *m, size_t i) {
    if (PHI) return static_cast<const float *>(m)[i] <= 0.f;
    return static_cast<const unsigned char *>(m)[i] != 0;
}

// One step of the run scan: c = this line's pixel, p = the neighbouring
// line's pixel at the same position, pl = the neighbour's previous pixel.
// A run that ends continues the neighbour's identical run iff the neighbour
// started a run where this one started, had ones all along, and ends here.
struct RunScan {
    unsigned in_run = 0, ok = 0, pl = 0;
    int count = 0;
    __device__ __forceinline__ void step(unsigned c, unsigned p) {
        if (c) {
            if (!in_run) {
                in_run = 1;
                ok = p & (pl ^ 1u);
            } else {
                ok &= p;
            }
        } else if (in_run) {
            count += (ok & (p ^ 1u)) ^ 1u;
            in_run = 0;
        }
        pl = p;
    }
};

__device__ __forceinline__ int block_sum(int v) {
    __shared__ int red[4];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int s = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    return s;
}

// Rows: one thread per row, scanning 16 pixels per load when rows are
// 16-byte aligned (vec), else pixel by pixel.
template <bool PHI>
__global__ __launch_bounds__(256) void k_shots_rows(const void *__restrict__ m, int H, int W, int vec,
                                                    unsigned long long *__restrict__ counts) {
    const int y = blockIdx.x * 256 + threadIdx.x;
    RunScan s;
    if (y < H) {
        const size_t row = (size_t)y * W, up = (size_t)(y - 1) * W;
        int x = 0;
        if (vec) {
            for (; x + 16 <= W; x += 16) {
                unsigned cb = 0, pb = 0;
                if (PHI) {
                    const float4 *cr = reinterpret_cast<const float4 *>(static_cast<const float *>(m) + row + x);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float4 v = cr[q];
                        cb |= ((v.x <= 0.f) | (v.y <= 0.f) << 1 | (v.z <= 0.f) << 2 | (v.w <= 0.f) << 3) << (4 * q);
                    }
                    if (y > 0) {
                        const float4 *pr = reinterpret_cast<const float4 *>(static_cast<const float *>(m) + up + x);
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const float4 v = pr[q];
                            pb |= ((v.x <= 0.f) | (v.y <= 0.f) << 1 | (v.z <= 0.f) << 2 | (v.w <= 0.f) << 3)
                                  << (4 * q);
                        }
                    }
                } else {
                    const uint4 v = *reinterpret_cast<const uint4 *>(static_cast<const unsigned char *>(m) + row + x);
                    const unsigned w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int q = 0; q < 16; ++q) cb |= (((w4[q >> 2] >> (8 * (q & 3))) & 0xffu) != 0) << q;
                    if (y > 0) {
                        const uint4 u = *reinterpret_cast<const uint4 *>(static_cast<const unsigned char *>(m) + up + x);
                        const unsigned u4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                        for (int q = 0; q < 16; ++q) pb |= (((u4[q >> 2] >> (8 * (q & 3))) & 0xffu) != 0) << q;
                    }
                }
#pragma unroll
                for (int b = 0; b < 16; ++b) s.step((cb >> b) & 1u, (pb >> b) & 1u);
            }
        }
        for (; x < W; ++x) s.step(pix<PHI>(m, row + x), y > 0 ? pix<PHI>(m, up + x) : 0u);
        s.step(0u, 0u);                       // past the last column
    }
    const int total = block_sum(s.count);
    if (threadIdx.x == 0) atomicAdd(counts, (unsigned long long)total);
}

// Columns: one thread per column, scanning down against the column to its
// left (loads coalesced across the wave).
template <bool PHI>
__global__ __launch_bounds__(256) void k_shots_cols(const void *__restrict__ m, int H, int W,
                                                    unsigned long long *__restrict__ counts) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    RunScan s;
    if (x < W) {
        for (int y = 0; y < H; ++y) {
            const size_t i = (size_t)y * W + x;
            s.step(pix<PHI>(m, i), x > 0 ? pix<PHI>(m, i - 1) : 0u);
        }
        s.step(0u, 0u);                       // past the last row
    }
    const int total = block_sum(s.count);
    if (threadIdx.x == 0) atomicAdd(counts + 1, (unsigned long long)total);
}

__global__ void k_shots_zero(unsigned long long *counts) {
    if (threadIdx.x < 3) counts[threadIdx.x] = 0ull;
}

__global__ void k_shots_min(unsigned long long *counts) {
    if (threadIdx.x == 0) counts[2] = counts[0] < counts[1] ? counts[0] : counts[1];
}

inline unsigned blocks_of(long long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_layout_extract(const unsigned char *d_layout, int H, int W, int N, int halo,
                                 unsigned char *d_tiles, hipStream_t st) {
    int rows, cols;
    layout_grid_dims(H, W, N, halo, &rows, &cols);
    const long long total = (long long)rows * cols * N * N;
    k_layout_extract<<<blocks_of(total), 256, 0, st>>>(d_layout, H, W, N, halo, cols, total, d_tiles);
    return hipGetLastError();
}

hipError_t launch_layout_stitch(const float *d_tiles, int H, int W, int N, int halo, float *d_out, hipStream_t st) {
    int rows, cols;
    layout_grid_dims(H, W, N, halo, &rows, &cols);
    k_layout_stitch<<<blocks_of((long long)H * W), 256, 0, st>>>(d_tiles, H, W, N, halo, cols, d_out);
    return hipGetLastError();
}

hipError_t launch_shot_count(const float *d_phi, const unsigned char *d_mask, int H, int W,
                             unsigned long long *d_counts, hipStream_t st) {
    k_shots_zero<<<1, 64, 0, st>>>(d_counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const void *m = d_phi ? static_cast<const void *>(d_phi) : static_cast<const void *>(d_mask);
    const size_t esz = d_phi ? 4 : 1;
    const int vec = (reinterpret_cast<uintptr_t>(m) % 16 == 0) && ((size_t)W * esz) % 16 == 0;
    if (d_phi) {
        k_shots_rows<true><<<blocks_of(H), 256, 0, st>>>(m, H, W, vec, d_counts);
        k_shots_cols<true><<<blocks_of(W), 256, 0, st>>>(m, H, W, d_counts);
    } else {
        k_shots_rows<false><<<blocks_of(H), 256, 0, st>>>(m, H, W, vec, d_counts);
        k_shots_cols<false><<<blocks_of(W), 256, 0, st>>>(m, H, W, d_counts);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_shots_min<<<1, 64, 0, st>>>(d_counts);
    return hipGetLastError();
}
