/*
 * darc.h -- C ABI of libdarc, the gfx950 hot path of DARC (Diffeomorphic
 * Atlas Registration via Coordinate descent), the groupwise atlas
 * construction method of "An Efficient Model-Driven Groupwise Approach for
 * Atlas Construction" (arXiv 2508.10743).
 *
 * What the library computes (Section 3 of the paper):
 *   - the group objective of Eq. (1)-(2): for every subject i a dissimilarity
 *     between the warped image I_i o phi_i and the atlas A, plus a diffusion
 *     regulariser lambda ||grad phi_i||^2, under the centrality constraint
 *     sum_i phi_i = 0;
 *   - phi_i = Exp(v_i) for a stationary velocity field v_i, by scaling and
 *     squaring (Section 3, "Diffeomorphisms": seven squarings);
 *   - one coordinate-descent sweep of Eq. (3) / Algorithm 1: per-subject
 *     gradient steps against a fixed atlas, the centrality activation
 *     phi_i - (1/n) sum_j phi_j (fourth line of Eq. (3)), then the atlas
 *     update, which for MSE is the mean of the warped subjects (first equation
 *     of Section 3, "Dissimilarity metrics"), for L1 their voxelwise median
 *     (second equation there) and for NCC a minibatch stochastic descent
 *     (last paragraph there; Algorithm 1 `SGD_for_atlas`);
 *   - one-shot segmentation (Section 4, Eq. (oneshot)): atlas labels carried
 *     to each subject by Exp(-v_i), with the Dice counts of Section 5;
 *   - factor-2 resampling for a coarse-to-fine schedule of the sweeps (not in
 *     the paper; provided for large cohorts).
 *
 * Conventions shared by every call
 *   - A volume has dims (d0, d1, d2) with d2 fastest: voxel (x0, x1, x2) sits
 *     at linear index (x0 * d1 + x1) * d2 + x2.  V = d0 * d1 * d2.  Each dim is
 *     at least 2 and V is at most 2^29.
 *   - A field (velocity v, displacement u, their gradients) is [3][V] per
 *     subject; component c displaces axis c, in voxel units.  phi is handled as
 *     the displacement u = phi - id (the reading under which sum_i phi_i = 0
 *     is meaningful).  A batch of n subjects is [n][3][V] (fields) or [n][V]
 *     (images), contiguous.
 *   - Positions are voxel coordinates with voxel centres at integers.
 *     Sampling is trilinear.  Images are sampled with zero padding (a corner
 *     outside the volume contributes 0); fields are sampled with border
 *     clamping (the position is clamped into [0, D-1] per axis).
 *   - All float arrays are FP32 device memory owned by the caller, at least
 *     4-byte aligned; double arrays are FP64 device memory.  The library never
 *     frees or retains a caller pointer beyond the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call only enqueues work on that stream and returns without
 *     synchronising; results are ready once the stream has reached that point.
 *   - Scratch memory is passed in by the caller: `ws`/`ws_bytes` must hold at
 *     least what the matching *_ws_bytes query returns (256-byte aligned).
 *     The library allocates no device memory.
 *   - Every call returns DARC_OK (0) or a negative status; on error nothing is
 *     enqueued (argument errors) or the HIP error is reported (DARC_EHIP), and
 *     darc_last_error() returns a message for the calling thread.
 *   - Calls on different streams that write the same memory race; calls on
 *     one stream are ordered.
 */
#ifndef DARC_H
#define DARC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DARC_ABI_VERSION 4

/* status codes */
#define DARC_OK 0
#define DARC_EINVAL (-1)       /* null pointer, bad dims or parameter */
#define DARC_EHIP (-2)         /* a HIP launch or runtime call failed */
#define DARC_EWORKSPACE (-3)   /* ws is null, misaligned or too small */
#define DARC_EUNSUPPORTED (-4) /* valid but not built (e.g. window size) */

/* dissimilarity metrics (Section 3, "Dissimilarity metrics") */
#define DARC_MSE 0   /* (1/V) sum_x (Iw - A)^2 */
#define DARC_LNCC 1  /* -(1/V) sum_x cc(x), squared local NCC over a win^3 window */
#define DARC_L1 2    /* (1/V) sum_x |Iw - A| */

/* atlas updates (step 3 of a sweep) */
#define DARC_ATLAS_MEAN 0   /* MSE closed form: mean of the warped subjects */
#define DARC_ATLAS_MEDIAN 1 /* L1 closed form: voxelwise median of the warped subjects */
#define DARC_ATLAS_SGD 2    /* minibatch Adam on the LNCC of the warped subjects */

/* Start of the stochastic atlas update (Algorithm 1, SGD_for_atlas, opens
 * with A = initialize(), which the paper leaves unspecified). */
#define DARC_SGD_INIT_WARM 0    /* from the current atlas A^k */
#define DARC_SGD_INIT_INITIAL 1 /* from A^0 of main: the mean of the unwarped subjects */

/* Inner iterations in one launch each (persistent, grid-synchronised; MSE
 * and L1 without smoothing of v) instead of ~20 launches each.  The launch is
 * sized to be resident on the whole device at once: a fused sweep must not
 * overlap other work on the device (another stream's launches could keep
 * some of its blocks waiting; its barrier waits then give up, see
 * darc_fused_barrier_ticks). */
#define DARC_FUSED_AUTO 0 /* the autotuner's choice for the shape; separate otherwise */
#define DARC_FUSED_OFF 1  /* separate launches */
#define DARC_FUSED_ON 2   /* fused; DARC_EUNSUPPORTED for LNCC or smoothing */

/* smoothing modes */
#define DARC_GAUSS 0     /* separable Gaussian, replicated border */
#define DARC_DIFFUSION 1 /* gradient of the diffusion regulariser of Eq. (2) */

/* what the centrality activation acts on */
#define DARC_CENTER_DISPLACEMENT 0 /* u_i <- u_i - mean_j u_j (Eq. (3), line 4) */
#define DARC_CENTER_VELOCITY 1     /* v_i <- v_i - mean_j v_j, then u_i = Exp(v_i) */

/* Version of this header's ABI (DARC_ABI_VERSION). */
int darc_abi_version(void);

/* Message describing the last error on the calling thread ("" if none).
 * The pointer stays valid until the next call on that thread. */
const char* darc_last_error(void);

/* ------------------------------------------------------------------------
 * darc_exp_svf -- phi = Exp(v) by scaling and squaring (Section 3,
 * "Diffeomorphisms").
 *
 *   u_0 = v / 2^n_sq;  u_{t+1}(x) = u_t(x) + u_t(x + u_t(x))  (t = 0..n_sq-1)
 *   u   = u_{n_sq}, the displacement of Exp(v).
 *
 * The inner u_t(.) is sampled trilinearly with border clamping.
 *   v     [n][3][V] in.
 *   u     [n][3][V] out; must not alias v or ckpt.
 *   ckpt  [n_sq-1][n][3][V] out, or NULL: the intermediate u_1..u_{n_sq-1}
 *         (step-major: slot j holds u_{j+1} of all n subjects), which
 *         darc_exp_svf_bwd needs.  Unused when n_sq < 2.
 *   ws    scratch of darc_exp_svf_ws_bytes(); only needed when ckpt is NULL.
 *   n_sq  0..16 (n_sq = 0 gives u = v).
 * ---------------------------------------------------------------------- */
size_t darc_exp_svf_ws_bytes(int n, int d0, int d1, int d2, int n_sq, int has_ckpt);
int darc_exp_svf(const float* v, float* u, float* ckpt, int n, int d0, int d1, int d2,
                 int n_sq, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * darc_exp_svf_bwd -- adjoint of darc_exp_svf (the gradient that automatic
 * differentiation of the squaring steps gives, Algorithm 1 `loss.backward()`).
 *
 * Given g_u = dL/du, returns g_v = dL/dv = (du/dv)^T g_u.  One squaring step
 * u_{t+1}(x) = u_t(x) + S(u_t, x + u_t(x)) has the adjoint
 *   g_t(y) = g_{t+1}(y) + J_t(y)^T g_{t+1}(y) + sum_x sum_k [corner_k(x) = y] w_k(x) g_{t+1}(x)
 * where J_t is the position derivative of the sampled field at x + u_t(x)
 * (zero along an axis whose coordinate was clamped) and w_k the trilinear
 * weights; dL/dv = g_0 / 2^n_sq.
 *   v     [n][3][V] in (u_0 is recomputed from it).
 *   ckpt  [n_sq-1][n][3][V] in: the checkpoints written by darc_exp_svf, or
 *         NULL: each u_t is then recomputed from v (n_sq (n_sq-1)/2 extra
 *         squaring steps, two fields of scratch instead of n_sq-1 stored).
 *   g_u   [n][3][V] in.   g_v [n][3][V] out (overwritten, not accumulated).
 *   ws    scratch of darc_exp_svf_bwd_ws_bytes(..., has_ckpt = ckpt != NULL).
 * The scatter term is summed in an order that varies between runs (sources
 * take their cell's LDS slots by integer atomics, and sources beyond a
 * cell's slots are added by LDS float atomics): results are reproducible
 * only up to FP32 summation order, and so are sweeps built on them.
 * ---------------------------------------------------------------------- */
size_t darc_exp_svf_bwd_ws_bytes(int n, int d0, int d1, int d2, int n_sq, int has_ckpt);
int darc_exp_svf_bwd(const float* v, const float* ckpt, const float* g_u, float* g_v, int n,
                     int d0, int d1, int d2, int n_sq, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * darc_warp3d -- I o phi (the warping operator of Eq. (2)):
 *   out_i(x) = I_i(x + u_i(x)), trilinear, zero outside the volume.
 *   img [n][V] in, u [n][3][V] in, out [n][V] out (must not alias img).
 *
 * darc_warp3d_bwd -- its adjoint with respect to u:
 *   g_u_i(x) += g_out_i(x) * grad_p I_i(p) at p = x + u_i(x),
 * the derivative of the trilinear interpolant inside the cell
 * [floor p, floor p + 1] (right-sided at integer positions).
 *   g_u [n][3][V] in/out, accumulated.
 * ---------------------------------------------------------------------- */
int darc_warp3d(const float* img, const float* u, float* out, int n, int d0, int d1, int d2,
                void* stream);
int darc_warp3d_bwd(const float* img, const float* u, const float* g_out, float* g_u, int n,
                    int d0, int d1, int d2, void* stream);

/* ------------------------------------------------------------------------
 * darc_sim_grad -- dissimilarity between each warped subject and the atlas
 * (Section 3, "Dissimilarity metrics") and its gradient.
 *
 *   DARC_MSE : D_i = (1/V) sum_x (W_i - A)^2;   dD_i/dW_i = (2/V)(W_i - A).
 *   DARC_L1  : D_i = (1/V) sum_x |W_i - A|;     dD_i/dW_i = sign(W_i - A) / V
 *              (0 where W_i = A; the difference is formed in FP64).
 *   DARC_LNCC: window sums over the win^3 cube centred at x, zero outside the
 *              volume, with the fixed count N = win^3:
 *              cross = S_IJ - S_I S_J / N, Ivar = S_II - S_I^2 / N,
 *              Jvar = S_JJ - S_J^2 / N, cc = cross^2 / (Ivar Jvar + eps),
 *              D_i = -(1/V) sum_x cc(x)  (I = W_i, J = A).
 *              Window sums are accumulated in FP64.
 *   warped   [n][V] in, atlas [V] in (shared by the n subjects).
 *   loss     [n] FP64 in/out: loss[i] += D_i.
 *   g_warped [n][V] out (overwritten), or NULL for the loss only.
 *   win      LNCC window, odd, 3..11 (ignored for MSE).  eps > 0 (LNCC).
 *   ws       scratch of darc_sim_grad_ws_bytes() (LNCC with gradient only).
 * ---------------------------------------------------------------------- */
size_t darc_sim_grad_ws_bytes(int metric, int n, int d0, int d1, int d2);
int darc_sim_grad(const float* warped, const float* atlas, int metric, int win, float eps,
                  double* loss, float* g_warped, int n, int d0, int d1, int d2, void* ws,
                  size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * darc_sim_grad_noalloc -- darc_sim_grad without a workspace argument, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * results and errors as darc_sim_grad minus ws/ws_bytes.
 *
 * The LNCC gradient's scratch (darc_sim_grad_ws_bytes: 16 bytes per
 * subject-voxel) lives in a file-scope device array of
 * darc_sim_grad_noalloc_max_bytes() = 128 MiB that every GPU the library runs
 * on holds until the process ends; its address is looked up once per device
 * (hipGetSymbolAddress) on the first call there.  The call itself allocates
 * nothing.  A call that would need more scratch (more than 8 388 608
 * subject-voxels, e.g. one 160 x 192 x 224 subject fits, two do not) fails
 * with DARC_EWORKSPACE and enqueues nothing.  Every call on one GPU shares
 * that GPU's array and overwrites it completely before reading it (nothing
 * needs to start at zero); calls that overlap on one GPU (different streams,
 * or threads) race on it and must be ordered by the caller.
 * ---------------------------------------------------------------------- */
size_t darc_sim_grad_noalloc_max_bytes(void);
int darc_sim_grad_noalloc(const float* warped, const float* atlas, int metric, int win, float eps,
                          double* loss, float* g_warped, int n, int d0, int d1, int d2,
                          void* stream);

/* ------------------------------------------------------------------------
 * darc_smooth3d -- smoothing of ncomp-component volumes [n][ncomp][V].
 *
 *   DARC_GAUSS (param = sigma > 0): out = G_sigma * in per component,
 *     separable 1-D weights proportional to exp(-k^2 / (2 sigma^2)) for
 *     |k| <= r = int(3 sigma + 0.5) (r <= 8), normalised to sum 1, replicated
 *     border.  out must not alias in.  loss is ignored.
 *   DARC_DIFFUSION (param = lambda): the diffusion regulariser of Eq. (2) on a
 *     displacement u,
 *       R(u) = (1/3) sum_d mean_{c, x: x_d < D_d - 1} (u_c(x + e_d) - u_c(x))^2,
 *     out += lambda dR/din and, if loss is not NULL, loss[i] += lambda R(in_i).
 *     out must not alias in.
 *   ws  unused (pass NULL, 0).
 * ---------------------------------------------------------------------- */
int darc_smooth3d(const float* in, float* out, int n, int ncomp, int d0, int d1, int d2,
                  int mode, float param, double* loss, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * darc_adam_step -- one Adam step (the paper's optimiser, Section 5: Adam
 * with learning rate 1e-2; Kingma & Ba's bias-corrected update):
 *   m <- b1 m + (1 - b1) g;  s <- b2 s + (1 - b2) g^2;
 *   v <- v - lr (m / (1 - b1^t)) / (sqrt(s / (1 - b2^t)) + eps)
 * over `count` floats.  t >= 1 is the step number after this update.  The
 * betas are doubles because 1 - beta2 magnifies the rounding of beta2 to FP32
 * (0.999f is 1.3e-5 off in 1 - beta2).
 * v, m, s in/out; g in.
 * ---------------------------------------------------------------------- */
int darc_adam_step(float* v, float* m, float* s, const float* g, long long count, long long t,
                   float lr, double beta1, double beta2, float eps, void* stream);

/* ------------------------------------------------------------------------
 * darc_center -- the centrality activation (fourth line of Eq. (3)):
 *   mean = (1/n) sum_j u_j;  u_i <- u_i - mean  for every i.
 *   u [n][3][V] in/out.  mean_out [3][V] out, or NULL.
 * The mean is accumulated in FP64.
 * ---------------------------------------------------------------------- */
int darc_center(float* u, float* mean_out, int n, int d0, int d1, int d2, void* stream);

/* ------------------------------------------------------------------------
 * darc_atlas_update -- the MSE atlas closed form (Section 3, "Dissimilarity
 * metrics"): A = (1/n) sum_i I_i o phi_hat_i, i.e.
 *   A(x) = (1/n) sum_i I_i(x + u_i(x) - mean(x)),  trilinear, zero padding.
 *   images [n][V] in, u [n][3][V] in, or NULL for zero displacements (A is
 *          then the mean of the unwarped images, the A^0 of Algorithm 1).
 *   mean   [3][V] in, or NULL (u is then taken as already centred).
 *   atlas  [V] out.  Accumulated in FP64.
 * ---------------------------------------------------------------------- */
int darc_atlas_update(const float* images, const float* u, const float* mean, float* atlas,
                      int n, int d0, int d1, int d2, void* stream);

/* ------------------------------------------------------------------------
 * darc_atlas_median -- the L1 atlas closed form (Section 3, "Dissimilarity
 * metrics", second equation): A(x) = median_i I_i(x + u_i(x) - mean(x)).
 * For even n every value between the two middle samples minimises the L1
 * sum; their average is returned.  Arguments as darc_atlas_update; n <= 512
 * (DARC_EUNSUPPORTED above).  Each voxel's n samples are staged in LDS.
 * ---------------------------------------------------------------------- */
int darc_atlas_median(const float* images, const float* u, const float* mean, float* atlas,
                      int n, int d0, int d1, int d2, void* stream);

/* ------------------------------------------------------------------------
 * darc_atlas_sgd -- the atlas update for NCC by minibatch stochastic descent
 * (Section 3, last paragraph of "Dissimilarity metrics"; Algorithm 1
 * `SGD_for_atlas`): `epochs` passes over the n warped subjects in minibatches
 * of `batch` consecutive subjects (the last one may be smaller); each
 * minibatch takes one Adam step on A along the gradient of
 *   (1/|B|) sum_{i in B} D_LNCC(W_i, A)
 * (cc is symmetric in its two images, so dD/dA is the LNCC adjoint with the
 * roles exchanged).  The Adam moments start at zero and the step count at 1
 * on every call; A starts from its value on entry.
 *   warped [n][V] in; atlas [V] in/out.
 *   losses [epochs * ceil(n / batch)] FP64 out (overwritten), or NULL: the
 *          minibatch loss before each step.
 *   ws     scratch of darc_atlas_sgd_ws_bytes().
 * ---------------------------------------------------------------------- */
size_t darc_atlas_sgd_ws_bytes(int n, int d0, int d1, int d2, int batch);
int darc_atlas_sgd(const float* warped, float* atlas, int n, int d0, int d1, int d2, int batch,
                   int epochs, int win, float eps, float lr, double beta1, double beta2,
                   float adam_eps, double* losses, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * darc_warp_labels -- a label map carried by displacements (nearest voxel,
 * which keeps labels integral):
 *   out_i(x) = labels(round(x + u_i(x))),  round(p) = floor(p + 1/2) per axis,
 * with the addition and the rounding in FP32; label 0 outside the volume.
 *   labels [V] uint8 in (shared); u [n][3][V] in; out [n][V] uint8 out.
 *
 * darc_segment -- one-shot segmentation (Section 4, Eq. (oneshot)):
 *   out_i = labels o Exp(-v_i), the atlas labels carried to subject i by the
 *   inverse deformation, Exp(-v_i) computed by scaling and squaring as in
 *   darc_exp_svf (n_sq 1..16) into the workspace.
 *   ws  scratch of darc_segment_ws_bytes().
 * ---------------------------------------------------------------------- */
int darc_warp_labels(const unsigned char* labels, const float* u, unsigned char* out, int n,
                     int d0, int d1, int d2, void* stream);
size_t darc_segment_ws_bytes(int n, int d0, int d1, int d2, int n_sq);
int darc_segment(const unsigned char* labels, const float* v, unsigned char* out, int n, int d0,
                 int d1, int d2, int n_sq, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * darc_dice_counts -- overlap counts for the Dice score of Section 5: for
 * each subject i and label l < num_labels (<= 256),
 *   counts[i][l] += { |a_i = l and b_i = l|, |a_i = l|, |b_i = l| }
 * (uint64); Dice = 2 c0 / (c1 + c2).  Labels >= num_labels are not counted.
 *   a, b [n][V] uint8 in (V = voxels per subject, up to 2^40); counts
 *   [n][num_labels][3] in/out, accumulated.
 * ---------------------------------------------------------------------- */
int darc_dice_counts(const unsigned char* a, const unsigned char* b, int n, long long V,
                     int num_labels, unsigned long long* counts, void* stream);

/* ------------------------------------------------------------------------
 * Learned warm start: a 3-D U-Net mapping an (atlas, subject) pair to an
 * initial velocity field, from which DARC's per-subject registration then
 * starts instead of v = 0.  Its convolutions run on the BF16 matrix cores
 * (FP32 accumulation).
 *
 * darc_conv3d -- one convolution, zero padding (ksize - 1) / 2, bias,
 * optional leaky ReLU (slope) -- as deep-learning frameworks define it
 * (cross-correlation):
 *   y[o][co] = bias[co] + sum_{tap, ci} w[co][tap][ci] x[o * stride + tap - pad][ci].
 *   Input x = concat(x0, x1) along channels, channels-last BF16 (raw bits):
 *     x0 [n][h0][h1][h2][c0], at (d0, d1, d2) or, when up0, at half of each
 *        dim and doubled by nearest neighbour; x1 [n][d0][d1][d2][c1] or NULL
 *        with c1 = 0.  c0 >= 8 and c1 multiples of 8.
 *   w   [cout][kpad] BF16, kpad = darc_conv3d_kpad(c0 + c1, ksize):
 *       entry k = (tap * (cin / 8) + v) * 8 + j holds the weight of channel
 *       8 v + j at tap = (a * 3 + b) * 3 + c, offset (a-1, b-1, c-1) along
 *       (d0, d1, d2) (tap 0 only for ksize 1); entries past the taps are 0.
 *   bias [cout] FP32 or NULL.  stride 1 or 2; output dims (d - 1) / stride + 1.
 *   Exactly one output: y_bf16 channels-last [n][o][cout] (rounded to nearest
 *   even) or y_f32 planar [n][cout][o] (the field layout when cout = 3).
 *
 * darc_unet_forward -- v = UNet(A, I_i) for n subjects:
 *   e0 = act(conv(cat(A, I), 2 -> 16)); e1, e2, e3 = act(conv stride 2)
 *   to 32, 64, 128 channels at 1/2, 1/4, 1/8 of the dims; d2, d1, d0 =
 *   act(conv(cat(up(deeper), skip))) to 64, 32, 16 channels; v = conv(d0, 16
 *   -> 3), FP32 [n][3][V].  act: leaky ReLU 0.2; activations BF16.
 *   Parameters: layer l (0..7 in that order) has weights [cout][kpad] at
 *   w + w_offset and biases at b + b_offset (darc_unet_layout); the input
 *   layer's 2 channels are padded to 8 with zero weights.  dims multiples
 *   of 8.  ws: scratch of darc_unet_ws_bytes().
 * ---------------------------------------------------------------------- */
int darc_conv3d_kpad(int cin, int ksize);
int darc_conv3d(const unsigned short* x0, int c0, int up0, const unsigned short* x1, int c1,
                int n, int d0, int d1, int d2, int ksize, int stride, const unsigned short* w,
                const float* bias, int cout, int act, float slope, unsigned short* y_bf16,
                float* y_f32, void* stream);
/* darc_conv3d_grad -- adjoint of darc_conv3d (ksize 3, no activation) given
 * the output gradient dz, channels-last BF16 [n][o][cz] (cz >= cout, a
 * multiple of 8, zero beyond cout):
 *   dw [cout][kpad] += sum_o dz[o][co] x(o, k)   (FP32; x read as darc_conv3d reads it)
 *   db [cout] += sum_o dz[o][co]                 (or NULL)
 *   dx [n][d0][d1][d2][c0 + c1] FP32 channels-last = the gradient with respect
 *      to the concatenated (full-resolution) input, or NULL: the stride-1
 *      convolution of dz (on the zero-dilated grid for stride 2) with the
 *      taps flipped and the channels exchanged, from the BF16 rounding of the
 *      FP32 weights w [cout][kpad].
 *   wt scratch BF16 [c0 + c1][darc_conv3d_kpad(cz, 3)] (needed with dx). */
int darc_conv3d_grad(const unsigned short* dz, int cz, const unsigned short* x0, int c0, int up0,
                     const unsigned short* x1, int c1, int n, int d0, int d1, int d2, int stride,
                     const float* w, int cout, float* dw, float* db, float* dx,
                     unsigned short* wt, void* stream);
int darc_unet_layout(int layer, int* cin, int* cout, int* kpad, size_t* w_offset,
                     size_t* b_offset);
size_t darc_unet_num_weights(void); /* packed weights of all 8 layers */
int darc_unet_num_biases(void);
size_t darc_unet_ws_bytes(int n, int d0, int d1, int d2);
int darc_unet_forward(const unsigned short* w, const float* b, const float* atlas,
                      const float* images, float* v, int n, int d0, int d1, int d2, void* ws,
                      size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Training of the warm start on (atlas, subject, DARC velocity) triples:
 * loss = mean over n*3*V entries of (UNet(A, I_i) - v_target_i)^2.
 *
 * darc_unet_backward -- the loss (loss[0] += ...) and its gradient with
 * respect to the FP32 weights and biases (dw [num_weights], db [num_biases],
 * overwritten; zero at the padded entries).  The forward pass uses the BF16
 * weights wq; the backward pass reads the output gradient of every layer as
 * BF16 (rounded to nearest even) and accumulates in FP32; the input gradient
 * of a layer is the convolution of its output gradient with flipped,
 * channel-exchanged BF16 weights (on the zero-dilated grid for stride 2).
 * v_pred [n][3][V] receives the prediction, or NULL.
 * ws: scratch of darc_unet_train_ws_bytes().
 *
 * darc_unet_train_step -- darc_unet_backward, then one Adam step on the FP32
 * weights and biases (the paper's optimiser and constants, step count
 * t->step + 1), refreshing t->wq; t->step is advanced on the host.
 * ---------------------------------------------------------------------- */
typedef struct darc_unet_train {
  float* w;            /* [num_weights] FP32 master weights (packed layout), in/out */
  float* b;            /* [num_biases] FP32 biases, in/out */
  float* mw;           /* Adam moments of w and b, in/out */
  float* sw;
  float* mb;
  float* sb;
  unsigned short* wq;  /* [num_weights] BF16 copy of w used by the convolutions, out */
  float* dw;           /* [num_weights] gradient scratch */
  float* db;           /* [num_biases] gradient scratch */
  long long step;      /* Adam steps taken, in/out */
} darc_unet_train;

size_t darc_unet_train_ws_bytes(int n, int d0, int d1, int d2);
int darc_unet_backward(const unsigned short* wq, const float* w, const float* b,
                       const float* atlas, const float* images, const float* v_target,
                       float* dw, float* db, double* loss, float* v_pred, int n, int d0, int d1,
                       int d2, void* ws, size_t ws_bytes, void* stream);
int darc_unet_train_step(darc_unet_train* t, const float* atlas, const float* images,
                         const float* v_target, float lr, double beta1, double beta2, float eps,
                         double* loss, int n, int d0, int d1, int d2, void* ws, size_t ws_bytes,
                         void* stream);

/* ------------------------------------------------------------------------
 * darc_down2 / darc_up2 -- factor-2 resampling between the levels of a
 * coarse-to-fine schedule.  Coarse voxel k averages the fine voxels 2k and
 * 2k+1 of every axis, so fine voxel x sits at coarse coordinate (x - 1/2)/2.
 *   darc_down2: out = 2x2x2 block means of `nchan` fine volumes
 *               [nchan][d0][d1][d2] (even dims) into [nchan][d0/2][d1/2][d2/2].
 *   darc_up2:   out(x) = scale * S_B(in, (x - 1/2) / 2), trilinear with border
 *               clamping, from [nchan][d0/2][d1/2][d2/2] onto [nchan][d0][d1][d2]
 *               (even dims); scale = 2 turns a coarse displacement or velocity
 *               (coarse voxels) into fine voxels.
 *   (d0, d1, d2) are the fine dims in both; in and out must not alias.
 * ---------------------------------------------------------------------- */
int darc_down2(const float* in, float* out, int nchan, int d0, int d1, int d2, void* stream);
int darc_up2(const float* in, float* out, int nchan, int d0, int d1, int d2, float scale,
             void* stream);

/* ------------------------------------------------------------------------
 * darc_sweep -- one coordinate-descent sweep (Eq. (3), Algorithm 1 `main`).
 *
 *   step 1: for every subject i (independent given the atlas, Section 3 after
 *           Eq. (3)), k2 times: u = Exp(v_i); L = D(I_i o phi, A) + lam R(u);
 *           g = dL/dv_i; Adam step on v_i; if smooth_sigma > 0, v_i <- G * v_i.
 *   step 2: u_i = Exp(v_i); centrality activation (center_mode).
 *   step 3: the atlas update of atlas_mode from the warped subjects
 *           I_i o phi_hat_i: their mean, their median, or k3 epochs of the
 *           minibatch update of darc_atlas_sgd starting from A^k.
 *   then the group loss F = (1/n) sum_i [D(I_i o phi_hat_i, A) + lam R(u_hat_i)].
 *
 * k2 = 0 runs steps 2 and 3 only: the start of a level of a coarse-to-fine
 * schedule, from velocities carried over from the coarser level.
 * ---------------------------------------------------------------------- */
typedef struct darc_state {
  const float* images; /* [n][V] subject images I_i, in */
  float* v;            /* [n][3][V] stationary velocity fields, in/out */
  float* m;            /* [n][3][V] Adam first moments, in/out */
  float* s;            /* [n][3][V] Adam second moments, in/out */
  float* atlas;        /* [V] atlas: A^k in, A^{k+1} out */
  float* u_hat;        /* [n][3][V] centred displacements out, or NULL */
  long long step;      /* Adam step count shared by all subjects, in/out (host) */
  long long* step_dev; /* the same count in device memory (int64), or NULL.  When
                          given, the bias corrections are formed on the device
                          from it (and it is advanced by k2), so that a sweep
                          captured in a graph can be replayed; `step` is then
                          only advanced on the host for information */
  int n, d0, d1, d2;
} darc_state;

typedef struct darc_params {
  int metric;         /* DARC_MSE, DARC_LNCC or DARC_L1 */
  int win;            /* LNCC window (odd, 3..11) */
  float ncc_eps;      /* LNCC epsilon (> 0) */
  float lam;          /* diffusion regulariser weight (>= 0) */
  float smooth_sigma; /* Gaussian sigma applied to v after every step; 0 = off */
  int n_sq;           /* squaring steps, 1..16 (7 in the paper) */
  int k2;             /* inner iterations per subject per sweep (>= 0) */
  float lr;           /* Adam learning rate */
  double beta1, beta2; /* Adam moment decay rates, in [0, 1) */
  float adam_eps;     /* Adam epsilon (> 0) */
  int center_mode;    /* DARC_CENTER_DISPLACEMENT or DARC_CENTER_VELOCITY */
  int reinit_v;       /* 1: v, m, s and step reset to zero before step 1 */
  int batch;          /* subjects per launch in step 1: 1 = per subject, n = all */
  int atlas_mode;     /* DARC_ATLAS_MEAN, DARC_ATLAS_MEDIAN or DARC_ATLAS_SGD */
  int k3;             /* SGD atlas: epochs (>= 1) */
  int atlas_batch;    /* SGD atlas: subjects per minibatch (>= 1) */
  float atlas_lr;     /* SGD atlas: Adam learning rate (betas and eps as above) */
  int sgd_init;       /* SGD atlas start: DARC_SGD_INIT_WARM or DARC_SGD_INIT_INITIAL */
  int fused;          /* DARC_FUSED_AUTO, DARC_FUSED_OFF or DARC_FUSED_ON */
} darc_params;

/* sizeof(darc_state) and sizeof(darc_params) as compiled into the library,
 * for bindings that mirror the two structs. */
size_t darc_sizeof_state(void);
size_t darc_sizeof_params(void);

/* Scratch needed by darc_sweep for this state shape and parameters (0 when
 * the state or parameters are invalid). */
size_t darc_sweep_ws_bytes(const darc_state* st, const darc_params* p);

/* losses: FP64 device array [n * k2 + 1], overwritten: losses[i * k2 + k] is
 * subject i's loss before its (k+1)-th step, losses[n * k2] the group loss F
 * after the sweep.  st->step is advanced by k2 on the host. */
int darc_sweep(darc_state* st, const darc_params* p, double* losses, void* ws, size_t ws_bytes,
               void* stream);

/* ------------------------------------------------------------------------
 * darc_autotune -- picks launch shapes for this state's volume shape and
 * batch size by timing candidates on the sweep's workspace: for the squaring
 * steps and their adjoint, marching tiles 8, 16, 32 or 64 planes deep or one
 * plane per block without marching (-1); the tile depth of the window
 * kernels (when the metric is LNCC or v is smoothed); and, for MSE / L1
 * without smoothing, whether an inner iteration runs as one fused launch or
 * as separate launches (decides DARC_FUSED_AUTO).  v, m, s and the atlas are only read.  The choices are
 * kept for every later call with the same shape and batch in this process.
 * Blocks until `stream` is idle; must not run while a stream is being
 * captured.  chosen (nullable, 3 ints) receives {squaring tz (-1: planes),
 * window tz, fused: 1 fused, 2 separate} (0 = not tuned).  darc_autotune_clear forgets
 * all choices.
 * ---------------------------------------------------------------------- */
int darc_autotune(darc_state* st, const darc_params* p, void* ws, size_t ws_bytes, void* stream,
                  int* chosen);
int darc_autotune_clear(void);

/* ------------------------------------------------------------------------
 * darc_set_launch_shape -- sets one entry of the table darc_autotune fills,
 * for volumes d0 x d1 x d2 and n subjects per launch (all four zero: the
 * entry every shape without its own falls back to): kind
 * DARC_SHAPE_SQUARING (value 8, 16, 32, 64: marching tile depth; 1:
 * marching, depth by the built-in heuristic; -1: one plane per block without
 * marching), DARC_SHAPE_WINDOW (8, 16, 32, 64, 96) or DARC_SHAPE_FUSED (1
 * fused, 2 separate launches under DARC_FUSED_AUTO).  value 0 returns the
 * entry to the built-in heuristic.  Launch shapes change how the same
 * arithmetic is scheduled, never what it computes.
 * ---------------------------------------------------------------------- */
#define DARC_SHAPE_SQUARING 0
#define DARC_SHAPE_WINDOW 1
#define DARC_SHAPE_FUSED 2
int darc_set_launch_shape(int kind, int d0, int d1, int d2, int n, int value);

/* ------------------------------------------------------------------------
 * darc_fused_barrier_ticks -- bound of one grid-barrier wait of the fused
 * inner iteration (DARC_FUSED_*), in ticks of the GPU's 100 MHz real-time
 * counter (default 100 000 000, one second; a negative value restores it).
 * A wait that reaches the bound gives up: every wave still finishes, and the
 * sweep reports NaN as its group loss (losses[n * k2]).  Small bounds exist
 * to exercise that path from the host; process-wide, not thread-safe.
 * ---------------------------------------------------------------------- */
int darc_fused_barrier_ticks(long long ticks);

/* ------------------------------------------------------------------------
 * Kernel timing for measurement.  When enabled, every kernel launched by the
 * library records HIP events on its stream; darc_profile_collect()
 * synchronises those events and returns, per kernel class, the number of
 * launches and their summed duration in milliseconds since the last reset.
 * Class names come from darc_profile_name().  Not thread-safe; meant for a
 * benchmark driving one stream.
 * ---------------------------------------------------------------------- */
int darc_profile_enable(int on);
int darc_profile_reset(void);
int darc_profile_num_classes(void);
const char* darc_profile_name(int cls);
int darc_profile_collect(long long* counts, double* ms, int max_classes);

/* ------------------------------------------------------------------------
 * Attainable HBM bandwidth (measurement helpers, not part of the method):
 * plain streams over caller buffers that read the path's kernels against what
 * this GPU reaches, beside the vendor's peak.  `bytes` is a multiple of 16 and
 * every pointer 16-byte aligned; blocks = 0 gives each thread of 256-thread
 * blocks a single 16-byte vector (bytes / 4096 blocks), otherwise `blocks`
 * blocks walk the buffers in grid-stride loops (four vectors per trip).
 *   darc_bw_copy : dst = src (reads and writes `bytes`).
 *   darc_bw_read : reads `bytes` of non-negative floats from src; sink [1]
 *                  is written only for a negative sum (never, in effect).
 *   darc_bw_write: fills dst with a per-thread pattern (writes `bytes`).
 * Return DARC_EINVAL on a bad argument (nothing enqueued), DARC_EHIP on a
 * launch failure; darc_last_error() is not set by these three.
 * ---------------------------------------------------------------------- */
int darc_bw_copy(const void* src, void* dst, size_t bytes, int blocks, void* stream);
int darc_bw_read(const void* src, size_t bytes, float* sink, int blocks, void* stream);
int darc_bw_write(void* dst, size_t bytes, int blocks, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DARC_H */
