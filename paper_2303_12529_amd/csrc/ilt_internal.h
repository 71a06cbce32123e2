// Internal declarations of the gfx950 level-set ILT library.
//
// Device data layout (all FP32 unless noted; Np = N rounded up to 128, and
// every padded row/column of a table is zero so that GEMMs over padded
// indices add nothing):
//
//   KP  = 2P rounded up to a multiple of 8 (real inner dimension of the
//         window transforms: rows [0,P) real parts, [P,2P) imaginary parts)
//   window columns of the row transform (spectrum and adjoint), NZ of them:
//         FB = P / 16 full 16-column blocks of real parts followed by FB
//         blocks of imaginary parts; when 0 < P % 16 <= 8 the leftover real
//         and imaginary columns share one more block (real at lanes 0..7,
//         imaginary at lanes 8..15: MIX = 1); when P % 16 > 8 they get a
//         padded pair of blocks (FB rounded up, MIX = 0).
//         NZ = 32 FB + 16 MIX; column of (b, real) = win_re(b), (b, imag) = win_im(b).
//   AP  = P rounded up to 16
//
//   tl   [2][KP][Np]   L1^T, L2^T: rows r of the image-side transform
//                      L1[y][r] = Ar[r][y] (r<P), Ai[r-P][y] (P<=r<2P)
//                      L2[y][r] = -Ai[r][y] (r<P), Ar[r-P][y] (P<=r<2P)
//                      so that for a window array Y (rows r as above)
//                      Re(A^H Y) = L1 Y and Im(A^H Y) = L2 Y.
//   tb   [2][Np][NZ]   image -> window row transform for a real (part 0)
//                      or imaginary (part 1) input column
//   ta4  [2][Np][AP]   Ar[a][y], Ai[a][y] stored [y][a]
//   ar, ai [P][Np]     A = exp(-2 pi i ((f_a x) mod N) / N)
//   Y    [n_sets][K][KP][Np]  window -> image operands, scaled sqrt(w_k)/N^2
//   Est  [n_sets][K][Np/16][Np/16][2][64][4]  fields E_k in the matrix-core
//        accumulator layout (real fragment, then imaginary), one 2 KB record
//        per 16 x 16 block
//
// A is computed on the host in FP64 from the integer-reduced phase and
// rounded once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ilt.h"

#define ILT_MAX_N 4096
#define ILT_MAX_P 35
#define ILT_MAX_K 64
#define ILT_MAX_SETS 4
#define ILT_TRACE_W 8
// clips of one size that a context runs in one launch per phase
#define ILT_MAX_BATCH 64

typedef float f4 __attribute__((ext_vector_type(4)));

__host__ __device__ __forceinline__ int win_re(int b, int FB) { return b < 16 * FB ? b : 32 * FB + (b - 16 * FB); }
__host__ __device__ __forceinline__ int win_im(int b, int FB) {
    return b < 16 * FB ? 16 * FB + b : 32 * FB + 8 + (b - 16 * FB);
}

// 16x16x4 FP32 matrix-core step.  Lane l supplies A[m = l%16][k = l/16] and
// B[k = l/16][n = l%16]; accumulator register i of lane l is
// C[m = 4*(l/16) + i][n = l%16].
__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

struct ilt_ctx {
    int N, P, K, n_sets, precision;
    int Np, KP, FB, MIX, NZ, AP;
    int device;
    hipStream_t stream;
    // clips: a context created for nb > 1 clips holds every per-clip
    // workspace nb times, one after another (strides cs_*), and runs the
    // ncur clips of the current sequence in one launch per phase (the clip
    // index is a grid dimension); ncur = 1 outside such a sequence
    int nb, ncur;
    float *phib;            // [nb][N][N] the clips' phi (nb > 1 only)
    unsigned char *tgtb;    // [nb][N][N] the clips' targets (nb > 1 only)
    double **trace_tab;     // [nb] device pointers of the clips' traces (or NULL)

    // tables
    float *tl;         // [2][KP][Np]
    float *tb;         // [2][Np][NZ]
    float *tbs;        // part 0 of tb in the spectrum's fragment order [Np/16][NZ/16][64][4]
    float *tba;        // tb in the stored-field adjoint's fragment order [Np/32][2][NZ/16][2][64][4]
    float *ta4;        // [2][Np][AP]
    float *ar, *ai;    // [P][Np]
    float2 *H;         // [n_sets][K][P][P]   kernels (FP32)
    float *sw;         // [n_sets][K]         sqrt(w_k) / N^2
    float2 *coef;      // [n_sets][K][P][P]   sqrt(w_k)/N^2 conj(H)
    __bf16 *tlhl;      // split-BF16 form: L operands [2][Np][hi|lo][KP]
    __bf16 *tbhl;      // split-BF16 form: B3 in fragment order [Np/32][2][NZ/16][hi|lo][64][8]
    __bf16 *Yhl;       // split-BF16 form: window rows [n_sets][K][Np][hi|lo][KP]
    // G-window adjoint (ILT_FLAG_GWINDOW_ADJOINT): difference window Q = 2P - 1
    int gwin, Q;
    float *tbQ;        // columns f >= 0 of the difference window (layout of P), fragment order [Np/16][NZ/16][64][4]
    float *arQ, *aiQ;  // [Q][Np]
    float2 *Ghat;      // [n_sets][Q][Q]
    float2 *Ghalf;     // [n_sets][Q][P]: the columns f >= 0 of Ghat
    float *Ugw;        // [n_sets][Fpad][NC] U_k = H_k . S as real columns (Fpad = P^2 rounded up to 4, NC = 2K rounded up to 16)
    double2 *Vpart;    // [gw_groups][n_sets][P][P] partial sums of W over ranges of window rows
    int hop;           // ILT_FLAG_HOPKINS_FORWARD: the image through its difference-window spectrum
    float *tlQ;        // [KP][Np] image-side table of the rows Da >= 0 of the difference window
    float *Tq;         // [n_sets][KP][Np] window rows of each set's image (rows >= 2P stay zero)
    double2 *Ipart;    // [n_sets][K][P][Q] image spectra per kernel, rows Da >= 0
    float2 *Ihat;      // [n_sets][P][Q] image spectra, rows Da >= 0 of the difference window
    int gw_groups;     // ranges the window sum is split into (grid.y of the correlation GEMM)

    // FP64 form (ILT_FP64 contexts only)
    double2 *A64;      // [P][N]      A in FP64
    double2 *H64;      // [n_sets][K][P][P]
    double *w64;       // [n_sets][K]
    double2 *T64;      // [N][P]      rows of the spectrum (and scratch of the column transform)
    double2 *S64;      // [P][P]
    double2 *Y64;      // [n_sets][K][P][N]  N^-2 (H . S) conj(A)
    double *I64, *G64; // [n_sets][N][N]
    double2 *Q64;      // [n_sets][K][N][P]  adjoint row transforms
    double2 *W64;      // [P][P]
    double2 *Z64;      // [P][N]
    double *g64, *phi64; // [N][N] gradient, the step's output
    double *part64;    // partials: resist [4 x 2048], max |g| and the step [3 x rows x row blocks]

    // workspaces
    float2 *Spart;     // spectrum band partials [Np/16][column ranges][P][P] (G-window: [set][Np/16][ranges][Q][Q])
    float2 *S;         // [P][P]
    float *Est;        // stored fields [n_sets][K][Np/16][Np/16][2][64][4] (null: recompute)
    float *Y;          // [n_sets][K][KP][Np]
    float *Tg;         // [KP][Np]
    float *I;          // [n_sets][N][N]
    float *G;          // [n_sets][N][N]
    float *g;          // [N][N]
    float *g_prev;     // [N][N] conjugate gradient: previous gradient
    float *dcg;        // [N][N] conjugate gradient: direction
    float *phi2;       // [N][N]
    float *Wpart;      // adjoint partials
    float2 *W;         // [P][P]
    // EDT scratch (edt_scratch_bytes): class bits [W][N] u32 (W = ceil(N/32),
    // 32 rows per word), then the nearest class rows above / below each
    // word, [4][W][N] int16
    void *edt_scratch;
    double *part;      // reduction partials (doubles)
    double *scal;      // device scalars (see SC_* below)
    int n_part;        // capacity of part (doubles)
    int n_wpart;       // capacity of Wpart (floats)

    // whole-solve hipGraph, captured on an internal stream and replayed on
    // `stream`; reused while the solve's arguments are unchanged
    int use_graph;
    // tuning (ilt_set_tuning / ilt_autotune); none changes what is computed
    // beyond rounding order
    int store_fields;  // FP32: 1 = forward stores the fields, the adjoint streams them
    int b3_xsplit;     // BF16x3 adjoint: column chunks split over this many blocks (0 = by size)
    int st_xsplit;     // FP32 stored-field adjoint: the same split (0 = by size)
    hipStream_t cap_stream;
    hipGraph_t graph;
    hipGraphExec_t graph_exec;
    unsigned char graph_key[160];
    int graph_key_len;

    // measurement hook: event pairs per recorded launch
    int profiling;
    int xcd_remap;     // BF16x3 image: XCD-aware tile order
    int n_ev;                 // events recorded in the current solve
    int ev_cap;
    hipEvent_t *ev;           // [ev_cap][2]
    int *ev_phase;            // [ev_cap]
};

// per-clip strides (elements) of the workspaces of a context with nb > 1
inline size_t cs_npix(const ilt_ctx *c) { return (size_t)c->N * c->N; }
inline size_t cs_y(const ilt_ctx *c) { return (size_t)c->n_sets * c->K * c->KP * c->Np; }
inline size_t cs_est(const ilt_ctx *c) { return (size_t)c->n_sets * c->K * (c->Np / 16) * (c->Np / 16) * 512; }
inline size_t cs_tg(const ilt_ctx *c) { return (size_t)c->KP * c->Np; }
inline size_t cs_spart(const ilt_ctx *c) { return (size_t)(c->Np / 16) * 4 * c->P * c->P; }

// device scalar slots
enum {
    SC_LOSS = 0, SC_L2 = 1, SC_PVB = 2, SC_NONFIN = 3,
    SC_MV = 4, SC_DT = 5, SC_FLIPS = 6, SC_ITER = 7, SC_BETA = 8,
    // non-finite values met anywhere in the current solve (loss, gradient,
    // phi after a step); zeroed when a solve starts, never reset inside it
    SC_BAD = 9,
    SC_COUNT = 16
};

struct resist_args {
    int n_corners;
    int cset[4];
    float dose[4];
    float omega[4];
    float sigma_z, i_th;
    int set_used[ILT_MAX_SETS];
};

// ---- launchers (k_litho.hip) ----
hipError_t launch_spectrum(ilt_ctx *c, const float *src, int src_is_phi);
hipError_t launch_make_Y(ilt_ctx *c, int set_lo, int set_hi);
hipError_t launch_image_to(ilt_ctx *c, int set_lo, int set_hi, float *out, int store_fields);
hipError_t launch_adjoint(ilt_ctx *c, const float *G, size_t g_set_stride, int set_lo, int set_hi,
                          int fields_stored);
hipError_t launch_window_sum(ilt_ctx *c, int set_lo, int set_hi);  // partial count follows c->precision
hipError_t launch_gradient(ilt_ctx *c, float *g_out, double *maxpart);

// ---- launchers (k_bf16.hip) ----
hipError_t launch_image_b3(ilt_ctx *c, int set_lo, int set_hi, float *out);
hipError_t launch_adjoint_b3(ilt_ctx *c, const float *G, size_t g_set_stride, int set_lo, int set_hi);
// G-window adjoint: W for sets [set_lo, set_hi) directly (no window_sum)
hipError_t launch_adjoint_gwindow(ilt_ctx *c, const float *G, size_t g_set_stride, int set_lo, int set_hi);
hipError_t launch_hopkins_spectrum(ilt_ctx *c, int set_lo, int set_hi);
hipError_t launch_hopkins_image(ilt_ctx *c, int set_lo, int set_hi, float *out);
// conjugate gradient: d = g + beta d, g_prev = g (beta = 0 when first), and the
// block maxima of |d| into maxpart for the CFL step; returns that block count
int launch_cg(ilt_ctx *c, int first, double *part, double *maxpart, hipError_t *err);
int adjoint_b3_parts(const ilt_ctx *c, int nsets);
// column ranges per 16-row band of the spectrum: every range writes a whole
// window partial that is summed afterwards, so fewer ranges once the launch
// has enough blocks (several images fill the device with one range); each
// wave's share, Np / (8 ranges), must stay a multiple of 16, so Np (a
// multiple of 128) is split only where 128 x ranges divides it
inline int spectrum_xsplit(const ilt_ctx *c, int nimg) {
    if (c->Np < 512) return c->Np / 128;
    return (nimg >= 2 || c->Np % 256 != 0) ? 1 : 2;
}
int adjoint_b3_max_parts(const ilt_ctx *c, int nsets);
#define ILT_B3_MAX_XSPLIT 4
#define ILT_ST_MAX_XSPLIT 2
// G-window correlation GEMM: column tiles of 16 over [Re U | Im U] and row
// tiles of 16 over the window frequencies.
inline int gwin_ntiles(int K) { return (2 * K + 15) / 16; }
inline int gwin_ftiles(int P) { return (P * P + 15) / 16; }
// LDS of one correlation block (floats): Ghat, then the block's rows of U
#define GWIN_LDS_FLOATS 16384
// by size: split the columns in two when the row tiles x kernel groups x sets
// would leave compute units without a block
inline int adjoint_st_xsplit(const ilt_ctx *c) {
    if (c->st_xsplit > 0) return c->st_xsplit;
    return ((c->N + 31) / 32) * ((c->K + 3) / 4) * c->n_sets < 256 ? 2 : 1;
}
// partial W count of the FP32 adjoint for nsets sets: row tiles x kernel
// groups, times the column split when the fields are stored
inline int adjoint_fp32_parts(const ilt_ctx *c, int nsets) {
    const int base = nsets * ((c->N + 31) / 32) * ((c->K + 3) / 4);
    return (c->Est && c->store_fields) ? base * adjoint_st_xsplit(c) : base;
}

// ---- launchers (k_pixel.hip) ----
int resist_blocks(const ilt_ctx *c);
hipError_t launch_resist(ilt_ctx *c, const float *I, const uint8_t *target, const resist_args &ra,
                         float *G, double *part);
hipError_t launch_finish_resist(ilt_ctx *c, const double *part, int nblk, double *scal, double *stats4);
int gradmax_blocks(const ilt_ctx *c);
hipError_t launch_absmax(ilt_ctx *c, const float *v, double *part);
hipError_t launch_finish_dt(ilt_ctx *c, const double *part, int nblk, int dt_mode, float eta,
                            float dt_max, double *scal);
int step_blocks(const ilt_ctx *c);
hipError_t launch_levelset(ilt_ctx *c, const float *phi, const float *vel, const float *mod,
                           float lam, float eps_kappa, const double *scal, float *phi_out,
                           double *part);
// trace rows: trace_row (one clip), or with trace_tab row `row` of each
// clip's trace trace_tab[clip] (NULL entries skipped)
hipError_t launch_finish_step(ilt_ctx *c, const double *part, int nblk, double *scal, double *stats4,
                              double *trace_row, int iter, double *const *trace_tab = nullptr, int row = 0);
hipError_t launch_edt(ilt_ctx *c, const float *phi, const uint8_t *mask, float *phi_out, int *sqdist,
                      float d_lower, float d_upper);
// the EDT on any stream with a caller-given scratch of edt_scratch_bytes(N)
size_t edt_scratch_bytes(int N);
hipError_t launch_edt_raw(hipStream_t st, int N, const float *phi, const uint8_t *mask, float *phi_out, int *sqdist,
                          float d_lower, float d_upper, void *scratch);
hipError_t launch_copy(ilt_ctx *c, float *dst, const float *src, size_t n);
// out = H(phi + dh) (0/1) over n values, on stream st
hipError_t launch_heaviside_shift(const float *phi, float dh, size_t n, float *out, hipStream_t st);
// scal[slot] = v on the context's stream (a kernel, so that it may be captured)
hipError_t launch_set_scal(ilt_ctx *c, int slot, double v);
hipError_t launch_fill(ilt_ctx *c, float *dst, float v, size_t n);

// ---- FP64 form (k_fp64.hip) ----
int resist64_blocks(const ilt_ctx *c);
int rowblk64(const ilt_ctx *c);
hipError_t launch64_spectrum(ilt_ctx *c, const double *src, int src_is_phi);
hipError_t launch64_make_Y(ilt_ctx *c, int s0, int s1);
hipError_t launch64_image(ilt_ctx *c, int s0, int s1, double *I);
hipError_t launch64_resist(ilt_ctx *c, const double *I, const uint8_t *target, const ilt_params *p, double *G,
                           double *part);
hipError_t launch64_adjoint(ilt_ctx *c, const double *G, int s0, int s1);
int launch64_gradient(ilt_ctx *c, double *g, double *maxpart, hipError_t *err);
hipError_t launch64_finish_dt(ilt_ctx *c, const double *part, int nblk, const ilt_params *p);
int launch64_levelset(ilt_ctx *c, const double *phi, const double *vel, const ilt_params *p, double *out,
                      double *part, hipError_t *err);
hipError_t launch64_copy(ilt_ctx *c, double *dst, const double *src, size_t n);
hipError_t launch_edt64(ilt_ctx *c, const double *phi, const uint8_t *mask, double *phi_out, int *sqdist,
                        float d_lower, float d_upper);
#define ILT_FP64_MAX_N 2048

// ---- edge placement error (k_metrics.hip): out[4] = samples, mean |EPE| (nm),
// max |EPE| (nm), samples with |EPE| > limit ----
hipError_t launch_epe(const unsigned char *Z, const float *I, float i_th, int N, double pitch, double step_nm,
                      double end_nm, double search_nm, double limit_nm, double *out, hipStream_t st);

// ---- full-layout tiling and shot count (k_layout.hip) ----
// tiles per column / row of the layout grid (cores of C = N - 2 halo pixels)
inline void layout_grid_dims(int H, int W, int N, int halo, int *rows, int *cols) {
    const int C = N - 2 * halo;
    *rows = (H + C - 1) / C;
    *cols = (W + C - 1) / C;
}
hipError_t launch_layout_extract(const unsigned char *d_layout, int H, int W, int N, int halo,
                                 unsigned char *d_tiles, hipStream_t st);
hipError_t launch_layout_stitch(const float *d_tiles, int H, int W, int N, int halo, float *d_out, hipStream_t st);
// d_counts [3]: row fracturing, column fracturing, their minimum
hipError_t launch_shot_count(const float *d_phi, const unsigned char *d_mask, int H, int W,
                             unsigned long long *d_counts, hipStream_t st);
