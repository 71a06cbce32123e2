/*
 * ilt.h -- C ABI of the MI355X (gfx950) level-set ILT hot path.
 *
 * The operations follow DevelSet (Chen et al., arXiv 2303.12529):
 *   forward lithography   Sec. II-B (Hopkins / truncated SOCS sum
 *                         I = sum_k w_k |M (*) h_k|^2, N_k = 24 kernels);
 *   resist and loss       Sec. III-A (sigmoid resist, L_ilt, L_pvb, L_DSO)
 *                         and Sec. II-C (binary print, squared L2, PVBand);
 *   adjoint gradient      Sec. III-A (dL_ilt/dM through the rotated and
 *                         conjugated kernels; dL_pvb/dM likewise);
 *   level-set step        Sec. II-A (explicit update of phi), Sec. III-A
 *                         (velocity = the ILT gradient, curvature term,
 *                         central differences and numeric curvature),
 *                         Sec. III-C (CFL time step eta / max|v|);
 *   re-initialisation     Sec. II-A (signed distance function), Sec. III-A
 *                         (TSDF clip to [D_l, D_u]) and Alg. 1 (CUDA_TSDF);
 *   the loop              Sec. III-A/B (DSO) and Fig. "DevelSet flow".
 *
 * Conventions shared by every call
 *   - Images are N x N, row-major [y][x], contiguous, 4-byte floats unless
 *     stated; every device pointer must be 16-byte aligned (torch tensors are).
 *   - "d_" pointers are device memory on the context's device; "h_" pointers
 *     are host memory.  The caller owns all of them; the library never frees
 *     or retains them beyond the call.
 *   - Work is enqueued on the context's stream and is asynchronous unless a
 *     call says otherwise.  One context must not be used from two host
 *     threads at once; calls on one context are ordered by its stream.
 *   - Frequency convention: forward DFT unnormalised, inverse with 1/N^2.
 *     A kernel is given by its frequency samples Hhat[a][b] on a P x P
 *     window, P odd, with (f_y, f_x) = (a - c, b - c), c = (P-1)/2, in units
 *     of 1/(N pitch).  The clear-field intensity is sum_k w_k |Hhat_k[c][c]|^2.
 *   - Return value: ILT_OK or a negative ILT_E* code; arguments are checked
 *     before anything is launched.  ilt_last_error() gives a message.
 */
#ifndef ILT_H
#define ILT_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ilt_ctx ilt_ctx;

enum {
    ILT_OK = 0,
    ILT_EINVAL = -1,       /* bad argument (null, size, range, alignment)     */
    ILT_ENOMEM = -2,       /* device allocation at create time failed         */
    ILT_EDEVICE = -3,      /* a HIP runtime call failed                       */
    ILT_ENUMERIC = -4,     /* non-finite loss, gradient or phi detected       */
    ILT_EUNSUPPORTED = -5  /* valid but not built for (e.g. P too large)      */
};

/* Arithmetic of the two dense contractions (forward image, adjoint).
 * ILT_BF16X3: each FP32 operand is split into BF16 hi + lo and products are
 * taken as hi*hi + hi*lo + lo*hi with FP32 accumulation on the BF16 matrix
 * cores; the adjoint then recomputes the fields (no field store).  Every
 * other step is FP32/FP64 as in ILT_FP32.
 * ILT_FP64: the context also holds FP64 tables and workspaces for the _f64
 * entry points below (N <= 2048), which run every step of the loop in FP64;
 * the FP32 entry points work on it as on an ILT_FP32 context (without the
 * field store). */
enum { ILT_FP32 = 0, ILT_BF16X3 = 1, ILT_FP64 = 2 };

/* ilt_optics.flags */
enum {
    /* Recompute the K coherent fields in the adjoint instead of storing them
     * during the forward pass.  Storing needs n_sets * K * N^2 * 8 bytes of
     * device memory (1.6 GB at N = 2048, K = 24, two sets) and halves the
     * adjoint's matrix-core work; recomputing needs no such workspace. */
    ILT_FLAG_RECOMPUTE_FIELDS = 1,
    /* Compute the adjoint through the G-window identity (the same W, exact
     * up to rounding): the DFT of G at the (2P-1)^2 difference frequencies,
     * then V_k(f') = N^-4 sum_f U_k(f) Ghat(f' - f) over the window and
     * W = sum_k w_k conj(H_k) V_k.  One pruned transform of G per kernel set
     * replaces the K adjoint field transforms, and no fields are stored or
     * recomputed.  Implies no field store (ILT_FLAG_RECOMPUTE_FIELDS is
     * then irrelevant). */
    ILT_FLAG_GWINDOW_ADJOINT = 2,
    /* Compute the aerial image through its spectrum on the (2P-1)^2
     * difference window (the TCC form of the SOCS sum, Sec. II-B; exact up to
     * rounding): Ihat(D) = sum_k w_k N^-4 sum_f U_k(f + D) conj(U_k(f)) with
     * U_k = H_k . S, then I(r) = sum_D Ihat(D) exp(+2 pi i D.r / N).  One
     * pruned inverse transform per kernel set replaces the K field
     * transforms.  Requires ILT_FLAG_GWINDOW_ADJOINT (no fields are formed)
     * and ILT_FP32; ILT_EINVAL otherwise. */
    ILT_FLAG_HOPKINS_FORWARD = 4
};

/* Optical model, read at create time and copied to the device. */
typedef struct {
    int N;                  /* grid side, 16 <= N <= 4096                     */
    int P;                  /* odd window side, 1 <= P <= 35, 2P-1 <= N       */
    int K;                  /* kernels per set, 1 <= K <= 64                  */
    int n_sets;             /* focus conditions (kernel sets), 1 <= n <= 4    */
    int precision;          /* ILT_FP32 or ILT_BF16X3                         */
    int flags;              /* ILT_FLAG_*                                     */
    const double *h_kernels;/* host [n_sets][K][P][P][2] (re, im)             */
    const double *h_weights;/* host [n_sets][K], each >= 0                    */
} ilt_optics;

/* A process corner: resist sees dose * I_set; loss weight omega. */
typedef struct { int set; float dose; float omega; } ilt_corner;

typedef struct {
    int iters;              /* DSO iterations T                               */
    int reinit_every;       /* R: TSDF re-initialisation after steps i with
                               (i+1) % R == 0; 0 = never                      */
    int dt_mode;            /* 0: dt = eta / max|g| (CFL), 1: dt = eta        */
    int init_mode;          /* ilt_solve: 0 = phi0 = TSDF(target), 1 = use the
                               caller's phi as phi0                           */
    float eta;              /* CFL number (dt_mode 0) or fixed dt (1)         */
    float dt_max;           /* cap on dt in CFL mode; <= 0: no cap            */
    float lambda;           /* curvature weight                               */
    float sigma_z;          /* sigmoid steepness                              */
    float i_th;             /* resist threshold                               */
    float eps_kappa;        /* added to |grad phi|^2 in the curvature ratio   */
    float d_lower;          /* TSDF clip bounds, pixels (D_l < 0 < D_u)       */
    float d_upper;
    int n_corners;          /* 1..4; corner 0 = nominal (L2 metric); with 3
                               corners, 1 and 2 are the PVBand extremes       */
    ilt_corner corners[4];
    int optimizer;          /* ilt_solve: 0 = move along the gradient g; 1 =
                               conjugate gradient (Sec. III-C): Polak-Ribiere
                               with non-negative restart, d = g + beta d_prev,
                               beta = max(0, <g, g - g_prev>/<g_prev, g_prev>)
                               (FP64 inner products, beta = 0 on the first
                               step of a call), CFL step on max|d|            */
    int iter0;              /* ilt_solve: index of the first iteration (>= 0).
                               The loop's state is phi and this index: a solve
                               of T1 iterations followed by one from its phi
                               with init_mode 1 and iter0 = T1 takes the same
                               steps as one solve of T1 + T2 iterations (the
                               re-initialisation schedule and the trace's i
                               column count from iter0); the conjugate
                               directions restart at a call's first step     */
} ilt_params;

typedef struct {
    int iters_done;
    int status;
    double loss;            /* L_DSO of the final mask                        */
    long long l2;           /* squared L2 (pixels) of the final nominal print */
    long long pvb;          /* PVBand (pixels) of the final mask              */
    long long flips;        /* mask pixels flipped by the last step           */
} ilt_report;

/* Create a context on the current HIP device.  Copies the kernels, builds
 * the DFT tables (FP64 on the host, rounded once to FP32) and allocates all
 * workspaces; nothing is allocated after this.  stream: a hipStream_t
 * (NULL = the default stream).  max_batch in [1, 64]: the clips of one size
 * that the batched form (ilt_solve_batch) runs together in one launch per
 * phase; the per-clip workspaces are allocated that many times.  Above 1
 * only for ILT_FP32 without ILT_FLAG_GWINDOW_ADJOINT (else ILT_EUNSUPPORTED).
 * The single-clip entry points below use the first clip's workspaces. */
int ilt_create(ilt_ctx **out, const ilt_optics *optics, int max_batch, void *stream);
int ilt_destroy(ilt_ctx *ctx);
/* Thread-local message for the last non-OK status of this thread. */
const char *ilt_last_error(void);
/* Grid side and window of a context (for bindings). */
int ilt_get_dims(const ilt_ctx *ctx, int *N, int *P, int *K, int *n_sets);

/* Sec. II-B: aerial image of kernel set `set` for a real-valued mask.
 * d_mask [N][N] (any real values), d_aerial [N][N] out.  Async. */
int litho_forward(ilt_ctx *ctx, const float *d_mask, int set, float *d_aerial);

/* Sec. II-A (mask of a level-set function, M = 1 where phi <= 0) and
 * Sec. II-B: the aerial image of kernel set `set` for the binary mask
 * [d_phi <= 0], formed as the spectrum's operand is loaded (no mask array is
 * written).  d_phi, d_aerial [N][N].  Async. */
int litho_forward_phi(ilt_ctx *ctx, const float *d_phi, int set, float *d_aerial);

/* Sec. III-B (modulation branch target): the Heaviside map of a shifted
 * level-set function, d_out[i] = 1 if d_phi[i] + dh >= 0 else 0, for n
 * values (FP32 in and out; the sign of the FP32 sum is that of the exact
 * one).  n >= 0, dh finite.  No context: async on `stream` (a hipStream_t,
 * NULL = default). */
int ilt_shifted_heaviside(const float *d_phi, float dh, long long n, float *d_out, void *stream);

/* Sec. III-A (ILT gradient): dL/dM = 2 sum_k w_k Re T_k^H (G . T_k M) for a
 * loss with dL/dI = G on kernel set `set` (T_k M = field of kernel k).
 * d_mask, d_dL_dI [N][N] in; d_dL_dM [N][N] out (overwritten).  Async. */
int litho_adjoint(ilt_ctx *ctx, const float *d_mask, const float *d_dL_dI, int set,
                  float *d_dL_dM);

/* Sec. III-A: sigmoid resist per corner, L_DSO = sum_c omega_c sum (Z_c - Z_t)^2,
 * G_s = dL/dI_s, and the binary-print L2 / PVBand counts.
 * d_aerial [n_sets][N][N] in (only sets used by a corner are read);
 * d_target [N][N] bytes (0/1); d_G [n_sets][N][N] out (sets not used by any
 * corner are zero-filled); d_stats: NULL or device double[4] =
 * {loss, l2, pvb, non-finite count}.  Async. */
int resist_loss(ilt_ctx *ctx, const float *d_aerial, const unsigned char *d_target,
                const ilt_params *params, float *d_G, double *d_stats);

/* Sec. II-A / III-A / III-C: one DSO evolution step, in place on d_phi:
 *   phi += dt * (v |grad phi| + lambda * m * K),
 * K = (phi_xx phi_y^2 - 2 phi_x phi_y phi_xy + phi_yy phi_x^2)/(phi_x^2+phi_y^2+eps),
 * central differences with replicated borders, v = d_vel = dL/dM (descent
 * sign), m = d_mod or 1 if NULL, dt from params (CFL uses max|v|, computed on
 * the device).  d_stats: NULL or device double[4] = {max|v|, dt, flips, non-finite
 * phi values after the step}.
 * Async. */
int levelset_step(ilt_ctx *ctx, float *d_phi, const float *d_vel, const float *d_mod,
                  const ilt_params *params, double *d_stats);

/* Sec. II-A, III-A (TSDF), Alg. 1: truncated signed distance of a mask.
 * Exactly one of d_phi (mask = [phi <= 0]) and d_mask (bytes, nonzero = 1)
 * is non-NULL.  Squared distances between pixel centres are exact integers:
 * phi = sqrt(D_in) - 1/2 outside, 1/2 - sqrt(D_out) inside, correctly rounded
 * to FP32, clipped to [d_lower, d_upper] from params.  d_phi_out [N][N] out
 * (may equal d_phi).  d_sqdist: NULL or device int32 [2][N][N] = {D_in, D_out}
 * (squared distance to the nearest inside / outside pixel; INT32_MAX when
 * that class is absent).  Async. */
int edt_reinit(ilt_ctx *ctx, const float *d_phi, const unsigned char *d_mask,
               float *d_phi_out, int *d_sqdist, const ilt_params *params);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * TSDF as edt_reinit, bit for bit, with no context.  N x N (1 <= N <= 4096;
 * larger N -> ILT_EINVAL), exactly one of d_phi (device fp32 [N][N], 4-byte
 * aligned; mask = [phi <= 0]) and d_mask (device bytes [N][N], nonzero =
 * inside), d_lower < 0 < d_upper (pixels), d_phi_out and d_sqdist as for
 * edt_reinit.  stream: a HIP stream of the current device (NULL = its null
 * stream).  Nothing is allocated: the EDT's scratch is a static 6 MiB device
 * array (one per device, held until the process ends), whose address is
 * looked up on the first call on each device.  Calls that overlap on one
 * device share that array and race; order them on one stream.  Async. */
int edt_reinit_noalloc(int N, const float *d_phi, const unsigned char *d_mask, float d_lower, float d_upper,
                       float *d_phi_out, int *d_sqdist, void *stream);

/* Sec. III-A/B: the plain DSO loop, params->iters iterations, entirely on the
 * device.  d_target [N][N] bytes; d_phi [N][N] in (used when init_mode = 1)
 * and out (final phi).  h_report: final loss / L2 / PVB of [phi_T <= 0].
 * d_trace: NULL or device double [iters][8] rows
 *   {i, loss, l2, pvb, flips, max|g|, dt, device time (ns)}.
 * Synchronous: waits for the stream once at the end.  Returns ILT_ENUMERIC
 * (h_report->status likewise) when a non-finite loss, gradient maximum or
 * phi value after a step occurred at any iteration of the call. */
int ilt_solve(ilt_ctx *ctx, const unsigned char *d_target, float *d_phi,
              const ilt_params *params, ilt_report *h_report, double *d_trace);

/* Edge placement error of the print [I >= I_th] (the hard threshold of
 * Sec. II-C) against the target; the paper scores masks by L2 and PVBand
 * and defines no EPE, so this is the library's own reading: sample points
 * every step along each straight edge of the (Manhattan) target, from
 * `end` after its ends; at each, the signed pixel distance along the
 * edge's outward normal from the target edge to the print's boundary
 * (positive: the print extends beyond the target), searched within
 * ceil(search / pitch) pixels and clipped to +-search.  d_target [N][N]
 * bytes, d_aerial [N][N] FP32 on the device; pitch_nm > 0; h_sampling: NULL
 * (10, 5, 40, 15 nm) or host float[4] {step, end, search, limit} in nm.
 * d_out: device double[4] = {samples, mean |EPE| nm, max |EPE| nm, samples
 * with |EPE| > limit}.  Async on stream (NULL = default); no context. */
int ilt_epe(const unsigned char *d_target, const float *d_aerial, float i_th, int N, float pitch_nm,
            const float *h_sampling, double *d_out, void *stream);

/* The loop and its two transforms in FP64, on an ILT_FP64 context: the
 * same steps and arguments as litho_forward, litho_adjoint and ilt_solve
 * with FP64 images (d_mask, d_aerial, d_dL_dI, d_dL_dM, d_phi: double
 * [N][N], 8-byte aligned) and every operation in double precision: the
 * pruned transforms, fields and image (Sec. II-B), the resist, L_DSO, G and
 * the print counts (Sec. III-A, II-C; corner doses and weights, sigma_z and
 * I_th taken as the FP64 values of the FP32 parameters), the adjoint
 * (Sec. III-A), the CFL step (Sec. III-C, dt = eta / max|g| in FP64), the
 * level-set update (Sec. II-A, III-A) and the TSDF (phi = sqrt(D) - 1/2
 * correctly rounded in FP64).  ilt_solve_f64 supports optimizer 0 only and
 * no modulation map; its trace rows and report are those of ilt_solve.
 * ILT_EINVAL on a context that is not ILT_FP64. */
int litho_forward_f64(ilt_ctx *ctx, const double *d_mask, int set, double *d_aerial);
int litho_adjoint_f64(ilt_ctx *ctx, const double *d_mask, const double *d_dL_dI, int set, double *d_dL_dM);
int ilt_solve_f64(ilt_ctx *ctx, const unsigned char *d_target, double *d_phi, const ilt_params *params,
                  ilt_report *h_report, double *d_trace);

/* Sec. III-C (DevelSet): ilt_solve with the curvature term of every step
 * weighted by a modulation map, phi += dt * (v |grad phi| + lambda * m * K)
 * with m = d_mod [N][N] FP32 (the DSN's modulation branch output upsampled
 * to the clip, values in [0, 1]; ilt_solve is the case m = 1).  d_mod is
 * read by every iteration and must stay valid and unchanged for the call;
 * a replayed graph keys on its address, not its contents.  Same arguments,
 * errors and synchronisation as ilt_solve. */
int ilt_solve_modulated(ilt_ctx *ctx, const unsigned char *d_target, float *d_phi, const float *d_mod,
                        const ilt_params *params, ilt_report *h_report, double *d_trace);

/* Sec. III-A/B, device-resident loop: by default ilt_solve captures its
 * whole launch sequence (init, iterations, final metrics) into a hipGraph on
 * an internal stream the first time it sees a set of arguments, and replays
 * the graph on the context's stream while the arguments (pointers and
 * params) stay the same.  enable = 0 launches every kernel directly
 * instead; solves with the measurement hook on always launch directly. */
int ilt_set_graph(ilt_ctx *ctx, int enable);

/* Measurement hook.  ilt_profile(ctx, 1) makes later ilt_solve calls record
 * a HIP event pair on the context's stream around every launch of each
 * phase of the loop; ilt_profile_read() then returns, per phase, the summed
 * device time in ms and the launch count of the most recent ilt_solve:
 * h_out[2*p] = ms, h_out[2*p+1] = launches, for p in
 *   0 spectrum, 1 window->rows, 2 image (forward), 3 resist, 4 adjoint,
 *   5 window sum + gradient, 6 level-set step, 7 re-initialisation.
 * n = number of doubles available at h_out (>= 16).  Synchronous. */
#define ILT_N_PHASES 8
int ilt_profile(ilt_ctx *ctx, int enable);
int ilt_profile_read(ilt_ctx *ctx, double *h_out, int n);

/* ------------------------------------------------------------------------
 * Tuning (not in the paper: launch-level choices of this implementation).
 * None changes what is computed beyond the order of rounding.
 *   store_fields  FP32: the forward pass stores the coherent fields and the
 *                 adjoint streams them (1), or the adjoint recomputes them
 *                 (0).  1 needs a context created without
 *                 ILT_FLAG_RECOMPUTE_FIELDS.
 *   b3_xsplit     BF16x3 adjoint: column chunks split over this many blocks
 *                 per row tile, 1..4 (0 = chosen by size).
 *   xcd_remap     BF16x3 image: XCD-aware tile order (1) or plain (0).
 *   st_xsplit     FP32 adjoint from stored fields: column chunks split over
 *                 this many blocks per row tile, 1..2 (0 = chosen by size:
 *                 2 when the grid would hold fewer than 256 blocks; the
 *                 autotuner leaves it there).
 * ilt_set_tuning drops a captured solve graph (it is re-captured).
 * ilt_autotune: with cache_path non-NULL and a line for this device
 * architecture and problem (N, P, K, n_sets, precision, field buffer) in that
 * text file (one JSON object per line, written by this function), applies
 * it and returns 1.  Otherwise times every candidate with HIP events on a
 * synthetic clip (the fastest of three 4-iteration solves after a warm-up,
 * on the context's stream; allocates and
 * frees two N x N scratch buffers), applies the fastest, appends it to
 * cache_path (if given) and returns 0.  h_best, h_ms_per_iter: NULL or out.
 * Synchronous. */
typedef struct {
    int store_fields;
    int b3_xsplit;
    int xcd_remap;
    int st_xsplit;
} ilt_tuning;

int ilt_get_tuning(const ilt_ctx *ctx, ilt_tuning *h_tuning);
int ilt_set_tuning(ilt_ctx *ctx, const ilt_tuning *h_tuning);
int ilt_autotune(ilt_ctx *ctx, const char *cache_path, ilt_tuning *h_best, double *h_ms_per_iter);

/* ------------------------------------------------------------------------
 * Batched form (many clips per call).  The paper solves one clip at a time
 * (Sec. IV reports per-clip turnaround); this form runs the same DSO loop of
 * ilt_solve on a list of clips, possibly of different sizes, in one call.
 * Every clip's result is bitwise identical to ilt_solve on that clip alone.
 *
 * ilt_batch_create: one batch object on the current device.  optics->N is
 * ignored; sizes[0..n_sizes) lists the clip sides the batch accepts (each in
 * [16, 4096], distinct).  The same kernels are used at every size, so the
 * caller passes kernels whose frequency samples suit all of them (clips of
 * one physical field width at different pixel pitches).  n_lanes in
 * [1, ILT_BATCH_MAX_LANES]: clips are spread over that many internal streams
 * and run side by side; device memory grows with n_sizes x n_lanes contexts, each
 * holding the workspaces of one chunk of clips (below).
 * max_clips: largest n accepted by ilt_solve_batch.  stream: the caller's
 * stream (NULL = default); ilt_solve_batch orders its work after what is
 * already queued there and returns when every clip is done.
 *
 * The clips of one size and identical parameters (compared byte for byte)
 * are run in chunks of up to (2048 / N)^2 clips (at most 16; one for
 * conjugate-gradient solves and in the split-BF16 and G-window forms): one
 * launch per phase covers every clip of a chunk, whose targets and phi are
 * copied into the context's clip buffers and phi back at the end.  Chunks
 * are spread over the lanes, longest first.
 *
 * ilt_solve_batch: clips[i] names a listed size N, its device target
 * [N][N] bytes, its phi [N][N] (in when params.init_mode = 1, out always;
 * no two clips may share phi), an optional device trace [iters][8] (rows as
 * for ilt_solve) and its own parameters (the TSDF bounds depend on the
 * pixel pitch).  h_reports: NULL or host [n].  The first call with a given
 * clip list captures each lane's sequence of solves into a hipGraph; later
 * calls with an identical list (byte for byte, including struct padding)
 * replay it.  Returns ILT_ENUMERIC if any clip's loss or gradient went
 * non-finite (its report says which). */
#define ILT_BATCH_MAX_SIZES 8
#define ILT_BATCH_MAX_LANES 4
#define ILT_BATCH_MAX_CLIPS 1024

typedef struct ilt_batch ilt_batch;

typedef struct {
    int N;                            /* clip side: one of the listed sizes  */
    const unsigned char *d_target;    /* device [N][N], nonzero = metal      */
    float *d_phi;                     /* device [N][N], in/out               */
    double *d_trace;                  /* NULL or device [params.iters][8]    */
    ilt_params params;                /* this clip's loop parameters         */
} ilt_clip;

int ilt_batch_create(ilt_batch **out, const ilt_optics *optics, const int *sizes, int n_sizes,
                     int max_clips, int n_lanes, void *stream);
int ilt_batch_destroy(ilt_batch *batch);
/* Capture and replay hipGraphs (1, default) or launch directly (0). */
int ilt_batch_set_graph(ilt_batch *batch, int enable);
int ilt_solve_batch(ilt_batch *batch, int n, const ilt_clip *clips, ilt_report *h_reports);

/* Project autotuner of the batched form.  For every listed size, times
 * (HIP events, best of three after a warm-up, per clip and iteration, on
 * chunks of a synthetic clip) the clips per chunk (the contexts' whole
 * capacity, half of it, a quarter) crossed with the FP32 adjoint's field
 * store and column split, and applies the fastest to every lane of that
 * size; sizes run one clip per chunk get ilt_autotune's choice.  cache_path:
 * NULL or a JSON-lines file; a line keyed by (arch, N, P, K, n_sets,
 * precision, field buffer, chunk capacity) is reused, a new choice
 * appended.  Outputs (each NULL or host [n_sizes]): the clips per chunk,
 * the tuning and its time per clip and iteration (us).  Results of every
 * clip stay those of ilt_solve with the same tuning.  Synchronous. */
int ilt_batch_autotune(ilt_batch *batch, const char *cache_path, int *h_chunk, ilt_tuning *h_tuning,
                       double *h_us_per_clip_iter);

/* ------------------------------------------------------------------------
 * Full layouts (beyond one clip).  The paper optimises clips of a fixed
 * size (Sec. IV: 2048 x 2048); a larger layout is covered by N x N tiles
 * whose cores, C = N - 2 halo pixels square, tile the layout at stride C.
 * Tile (i, j), i < rows, j < cols, spans layout rows [i C - halo,
 * i C - halo + N) and columns [j C - halo, j C - halo + N); tile pixels
 * outside the layout are empty.  The halo is optical context: the imaging
 * kernels reach beyond a core, so each core is solved with its surroundings
 * and only the core is kept.  Tiles are stored [rows][cols][N][N].
 *
 * Layout sides in [1, ILT_LAYOUT_MAX_SIDE], N in [16, 4096], 0 <= halo,
 * N - 2 halo >= 1, rows x cols <= ILT_LAYOUT_MAX_TILES; ILT_EINVAL otherwise.
 * ilt_layout_grid: rows and cols of the tiling (host only).
 * ilt_layout_extract: d_tiles [rows][cols][N][N] bytes from d_layout [H][W]
 *   bytes.  Async on `stream` (a hipStream_t, NULL = default).
 * ilt_layout_stitch: d_layout [H][W] FP32, each pixel from the core of the
 *   tile holding it in d_tiles [rows][cols][N][N] FP32.  Async.
 * ilt_solve_layout: extract, then the DSO loop of ilt_solve on every tile
 *   through the batch (N must be one of its sizes; chunks of max_clips),
 *   then stitch phi.  d_tile_targets [rows][cols][N][N] bytes and
 *   d_tile_phi [rows][cols][N][N] FP32 are the caller's workspaces (tile
 *   results stay there); d_layout_phi [H][W] out.  params->init_mode must be
 *   0 (each tile starts from the TSDF of its own target).  h_reports: NULL
 *   or host [rows x cols], per tile.  Synchronous; ILT_ENUMERIC if any tile
 *   went non-finite (the stitched result is still written). */
#define ILT_LAYOUT_MAX_SIDE (1 << 20)
#define ILT_LAYOUT_MAX_TILES (1 << 20)

int ilt_layout_grid(int H, int W, int N, int halo, int *rows, int *cols);
int ilt_layout_extract(const unsigned char *d_layout, int H, int W, int N, int halo, unsigned char *d_tiles,
                       void *stream);
int ilt_layout_stitch(const float *d_tiles, int H, int W, int N, int halo, float *d_layout, void *stream);
int ilt_solve_layout(ilt_batch *batch, const unsigned char *d_layout, int H, int W, int N, int halo,
                     const ilt_params *params, unsigned char *d_tile_targets, float *d_tile_phi,
                     float *d_layout_phi, ilt_report *h_reports);

/* Sec. II-C, mask fracturing shot count: the number of rectangles of an
 * exact fracturing of the mask (the paper's scripts are not given).  The
 * estimate: every maximal run of ones in a row continues the rectangle of
 * the identical run (same first and last column) in the row above, or
 * starts a rectangle; the same with rows and columns exchanged; the smaller
 * of the two counts.  Exactly one of d_phi (mask [phi <= 0], FP32) and
 * d_mask (bytes, nonzero = 1) is given, [H][W], sides in
 * [1, ILT_LAYOUT_MAX_SIDE].  d_counts: device int64 [3] = {row fracturing,
 * column fracturing, minimum}.  Exact integers.  Async on `stream`. */
int ilt_shot_count(const float *d_phi, const unsigned char *d_mask, int H, int W, long long *d_counts,
                   void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ILT_H */
