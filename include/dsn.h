/* C ABI of DevelSet-Net on one AMD MI355X (gfx950).
 *
 * Sec. III-B of Chen et al., "DevelSet: Deep Neural Level Set for Instant
 * Mask Optimization" (arXiv 2303.12529): a UNet backbone predicts the initial
 * level-set function phi_0 of DSO from the target image and is trained with
 * the squared error L_0 = sum (phi_0,theta - phi_gt)^2 against level-set
 * functions produced by DSO.  Its second branch predicts the modulation map
 * m_theta = H_eps(phi_m), H_eps(z) = 1/2 (1 + (2/pi) atan(z / eps)) the
 * approximated Heaviside function with the paper's eps = DSN_EPS_AHF (Sec.
 * III-B, Sec. IV), trained with L_m = sum (m_theta - m_gt)^2 and m_gt a
 * binary map that the caller derives from phi_gt by a shift search.  The paper leaves the layer sizes, resampling and
 * optimiser open; this library fixes them as follows:
 *   - network grid H x W (the 2048 clip's 4 x 4 means: 512 x 512); four
 *     levels of width C, 2C, 4C, 8C (C = base, a multiple of 32); per level
 *     two 3x3 convolutions (zero padding 1, bias, ReLU); 2x2 max-pooling
 *     down; up: nearest 2x upsampling, a 3x3 convolution (bias, ReLU) to the
 *     level's width, concatenation [up | skip], the level's two
 *     convolutions; a 1x1 head (bias, no ReLU) giving phi / 100, and with
 *     the modulation branch a second 1x1 head on the same features giving
 *     phi_m (the two branches share the backbone);
 *   - input = 4 x 4 mean of the binary target; target = 4 x 4 mean of phi_gt
 *     (pixels of the fine grid) / 100; phi_0 = clip(100 x bilinear 4x
 *     upsample of the output) with half-pixel centres and clamped borders;
 *     the modulation target t_m = 4 x 4 mean of m_gt, and the fine-grid
 *     modulation map m_0 = bilinear 4x upsample of H_eps(phi_m);
 *   - losses L_0 and L_m per sample (sums over pixels of the network grid)
 *     averaged over the batch; the trained objective is L_0 + L_m;
 *     Adam on FP32 master weights; BF16 activations, weights and activation
 *     gradients with FP32 accumulation; FP32 weight gradients.
 * Parameters are one flat FP32 vector: for each layer in the order enc0_a,
 * enc0_b, ..., enc3_a, enc3_b, dec2_up, dec2_a, dec2_b, dec1_*, dec0_*, head
 * and, with the modulation branch, head_m: the weights [C_out][3][3][C_in]
 * (heads: [1][1][1][C]) then the bias [C_out].
 *
 * Buffers are device pointers owned by the caller unless stated; every call
 * is enqueued on the context's stream and returns without waiting.  Errors:
 * DSN_EINVAL (bad argument, checked before any launch), DSN_EDEVICE (a HIP
 * call failed; the message says which), DSN_ENOMEM.  No exception crosses
 * the ABI.  One context per stream. */
#ifndef DSN_H
#define DSN_H

#ifdef __cplusplus
extern "C" {
#endif

enum { DSN_OK = 0, DSN_EINVAL = -1, DSN_ENOMEM = -2, DSN_EDEVICE = -3 };
#define DSN_LEVELS 4
#define DSN_SCALE 100.0f
#define DSN_EPS_AHF 0.03f

typedef struct dsn_ctx dsn_ctx;

/* H, W: network grid, multiples of 8 (three poolings), at most 2048;
 * base: level-0 width, 32 or 64; max_batch >= 1 with max_batch H W below
 * 2^31; modulation: 1 adds the modulation head, 0 leaves it out.  Allocates
 * the parameters (zero), Adam moments, and activations/gradients for
 * max_batch samples.
 * stream: a hipStream_t (NULL = default stream). */
int dsn_create(dsn_ctx **out, int H, int W, int base, int max_batch, int modulation, void *stream);
int dsn_destroy(dsn_ctx *ctx);
const char *dsn_last_error(void);
/* Number of FP32 entries of the flat parameter vector. */
long long dsn_num_params(const dsn_ctx *ctx);
/* Load / read the flat FP32 parameters (device [num_params]).  Loading also
 * refreshes the BF16 working copies and zeroes the Adam moments and step. */
int dsn_set_params(dsn_ctx *ctx, const float *d_params);
int dsn_get_params(const dsn_ctx *ctx, float *d_params);

/* Forward pass.  d_x: [B][H][W] FP32 network input; d_out: [B][H][W] FP32
 * network output (target scale, i.e. phi / 100); d_out_m: NULL, or (only
 * with the modulation head) [B][H][W] FP32 receiving phi_m before H_eps.
 * Keeps every activation for dsn_backward, which also reads d_x, d_out and
 * d_out_m again: they must stay valid until then.  1 <= B <= max_batch. */
int dsn_forward(dsn_ctx *ctx, const float *d_x, int B, float *d_out, float *d_out_m);
/* Backward pass for the last forward (same B).  d_target [B][H][W];
 * d_target_m: NULL (L_m is left out; the modulation head's gradient is
 * zero) or [B][H][W] modulation targets in [0, 1], which needs a forward
 * with d_out_m; the gradient is that of L_0 + L_m.  d_loss: device
 * double[2], set to L_0 and L_m (0 without d_target_m) averaged over the
 * batch; d_grad: NULL or device FP32 [num_params] receiving the gradient
 * (it is always kept internally for dsn_adam_step). */
int dsn_backward(dsn_ctx *ctx, const float *d_target, const float *d_target_m, int B, double *d_loss,
                 float *d_grad);
/* One Adam step with the gradient of the last backward (step count kept in
 * the context, starting at 1). */
int dsn_adam_step(dsn_ctx *ctx, float lr, float beta1, float beta2, float eps);

/* Resampling between the fine grid (4H x 4W) and the network grid.
 * dsn_prepare: d_target bytes [B][4H][4W] (nonzero = metal) -> d_x
 * [B][H][W] 4 x 4 means; if d_phi_gt (FP32 [B][4H][4W]) is non-NULL, also
 * d_t [B][H][W] = 4 x 4 means of phi_gt / 100; if d_m_gt (FP32
 * [B][4H][4W]) is non-NULL, also d_t_m [B][H][W] = its 4 x 4 means.
 * dsn_predict: forward pass of the targets' means, then
 * d_phi0 [B][4H][4W] = clip(100 x bilinear 4x upsample, d_lower, d_upper)
 * and, if d_m0 is non-NULL (modulation head only), d_m0 [B][4H][4W] =
 * bilinear 4x upsample of H_eps(phi_m), values in [0, 1]. */
int dsn_prepare(dsn_ctx *ctx, const unsigned char *d_target, const float *d_phi_gt, const float *d_m_gt, int B,
                float *d_x, float *d_t, float *d_t_m);
int dsn_predict(dsn_ctx *ctx, const unsigned char *d_target, int B, float d_lower, float d_upper,
                float *d_phi0, float *d_m0);

/* Single operations of the network, for callers composing their own layers
 * (and for testing each kernel alone).  BF16 tensors channels-last; N images
 * of H x W output pixels; zero padding 1.  Synchronous; the gradient
 * operations allocate and free a temporary buffer.
 * dsn_op_conv3x3: d_y [N][H][W][Cout] = act(d_b + conv(d_x, d_w)), with
 *   d_x [N][H'][W'][Cin] read through a nearest 2x upsampling when up != 0
 *   (H' = H/2, W' = W/2; else H' = H, W' = W); d_w [Cout][3][3][Cin]; d_b
 *   FP32 [Cout] or NULL; relu != 0 applies max(., 0).
 * dsn_op_conv3x3_dgrad: d_dx [N][H][W][Cin] = gradient of sum(d_dy . conv(x))
 *   with respect to x (no upsampling), d_dy [N][H][W][Cout]; with d_mask
 *   (BF16 [N][H][W][Cin], or NULL) d_dx is zeroed where d_mask <= 0: the
 *   backward of the ReLU whose output is d_mask, fused.
 * dsn_op_conv3x3_wgrad: FP32 d_dw [Cout][3][3][Cin] and d_db [Cout], the
 *   gradients of sum(d_dz . conv(x)) with d_dz [N][H][W][Cout] and x as in
 *   dsn_op_conv3x3: per split of whole 8 x 32 pixel tiles FP32 partials of
 *   all nine taps (the bias from the same staged d_dz), the splits added in
 *   FP64 in a fixed order.
 * Channel counts: multiples of 32 in [32, 1024]. */
int dsn_op_conv3x3(const void *d_x, int N, int H, int W, int Cin, int up, const void *d_w, const float *d_b,
                   int Cout, int relu, void *d_y, void *stream);
int dsn_op_conv3x3_dgrad(const void *d_dy, int N, int H, int W, int Cout, const void *d_w, int Cin,
                         const void *d_mask, void *d_dx, void *stream);
int dsn_op_conv3x3_wgrad(const void *d_dz, const void *d_x, int N, int H, int W, int Cin, int up, int Cout,
                         float *d_dw, float *d_db, void *stream);

/* The network's other layers, one call each (Sec. III-B; the same kernels as
 * dsn_forward / dsn_backward, with the same work split).  Every pointer
 * 16-byte aligned; C (channels) as stated per call.
 * dsn_op_conv_first: the first layer (one input channel, VALU): d_y BF16
 *   [N][H][W][Cout] = max(0, d_b + conv3x3(d_x)), d_x FP32 [N][H][W], d_w
 *   BF16 [Cout][3][3][1], d_b FP32 [Cout]; Cout a multiple of 8 in
 *   [8, 1024].  Async on `stream`.
 * dsn_op_wgrad_first: its weight and bias gradients, FP32 d_dw [C][3][3][1]
 *   and d_db [C], for the output gradient d_dz BF16 [N][H][W][C] and input
 *   d_x FP32 [N][H][W]: sums over pixel ranges (4096 pixels each, at most
 *   2048 ranges; a range may cross image boundaries) in FP32, the ranges
 *   added in FP64 in a fixed order.  C in {8, 16, 32, 64}.  Synchronous;
 *   allocates and frees the range partials.
 * dsn_op_head_bwd: backward of the 1x1 head(s) and the losses for npix
 *   pixels of features d_x BF16 [npix][C] (C a multiple of 8 in [8, 64]),
 *   level-set head weights d_w BF16 [C], outputs d_out and targets d_t FP32
 *   [npix], batch size B (the losses are sums over pixels averaged over B).
 *   With the modulation head, d_wm BF16 [C], d_out_m (phi_m before H_eps)
 *   and d_t_m FP32 [npix] (all three or none).  Out: d_dx BF16 [npix][C]
 *   = g w + g_m w_m with g = (2/B)(out - t), g_m = (2/B)(H_eps(out_m) - t_m)
 *   H_eps'(out_m); d_loss double[2] = {L_0, L_m (0 without the head)};
 *   d_gw FP32 [heads][C + 1] = per head the weight gradient sum_p g x[p]
 *   then the bias gradient sum_p g.  relu_mask != 0 also zeroes d_dx where
 *   d_x <= 0 (the backward of the ReLU that produced the features).
 *   Synchronous; allocates and frees the block partials.
 * dsn_op_maxpool2_bwd: d_dx BF16 [N][H][W][C] += each gradient of d_dy BF16
 *   [N][H/2][W/2][C] routed to the first maximum (row-major) of its 2x2
 *   window of d_x BF16 [N][H][W][C]; the sum in FP32, rounded once to BF16.
 *   relu_mask != 0 then zeroes every element of the windows where d_x <= 0
 *   (d_x a ReLU output: the ReLU's backward, fused).
 * dsn_op_upsample2_bwd: d_dx BF16 [N][H/2][W/2][C] = the FP32 sum of the
 *   four children in d_dy BF16 [N][H][W][C] (nearest 2x upsampling's
 *   gradient), rounded once to BF16; with d_mask (BF16 [N][H/2][W/2][C], or
 *   NULL) zeroed where d_mask <= 0.
 * dsn_op_relu_bwd: d_d BF16 [npix][C] *= [d_y > 0] in place (d_y BF16, the
 *   layer's output).
 * The last three: H, W even, C a multiple of 8 in [8, 2048]; async. */
int dsn_op_conv_first(const float *d_x, int N, int H, int W, const void *d_w, const float *d_b, int Cout, void *d_y,
                      void *stream);
int dsn_op_wgrad_first(const void *d_dz, const float *d_x, int N, int H, int W, int C, float *d_dw, float *d_db,
                       void *stream);
int dsn_op_head_bwd(const void *d_x, long long npix, int C, int B, const void *d_w, const void *d_wm,
                    const float *d_out, const float *d_out_m, const float *d_t, const float *d_t_m, int relu_mask,
                    void *d_dx, double *d_loss, float *d_gw, void *stream);
int dsn_op_maxpool2_bwd(const void *d_x, int N, int H, int W, int C, const void *d_dy, int relu_mask, void *d_dx,
                        void *stream);
int dsn_op_upsample2_bwd(const void *d_dy, int N, int H, int W, int C, const void *d_mask, void *d_dx,
                         void *stream);
int dsn_op_relu_bwd(void *d_d, const void *d_y, long long npix, int C, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DSN_H */
