// Internal launchers of libdarc.  Every launcher enqueues on `st` and checks
// nothing: argument validation happens in the C ABI layer.  `n` is the number
// of subjects handled by one launch; array strides between subjects are 3V
// (fields) and V (images) unless stated.
#pragma once

#include "darc_common.hpp"

namespace darc {

RegW make_regw(const Geom& g, int ncomp, float lam);

// --- scaling and squaring -------------------------------------------------
// The squaring kernels work on 32 x 8 x 8 tiles (d2 x d1 x d0).  The forward
// step can record, per tile, the box of trilinear cells its sample positions
// fall in, and per subject how far those boxes reach past their own tile;
// the adjoint uses them to gather every contribution to an output tile
// without global atomics.  `aux` holds [n_sq][n][ntiles][8] boxes followed by
// [n_sq][n][8] reaches (ints).
size_t exp_aux_bytes(const Geom& g, int n, int n_sq);
// Full Exp(v) (Exp(-v) when negate, n_sq >= 1): ckpt ([n_sq-1][n][3][V]) or
// tmp ([n][3][V]) must be given when n_sq >= 2; aux (nullable) receives the
// boxes the adjoint needs.
void run_exp_fwd(const float* v, float* u, float* ckpt, float* tmp, int* aux, const Geom& g, int n,
                 int n_sq, hipStream_t st, bool negate = false);
// Full adjoint; tmp_a, tmp_b are [n][3][V]; g_v must not alias g_u.  When
// aux_ready is false the boxes in aux are recomputed from v and ckpt first.
void run_exp_bwd(const float* v, const float* ckpt, const float* g_u, float* g_v, float* tmp_a,
                 float* tmp_b, int* aux, bool aux_ready, const Geom& g, int n, int n_sq,
                 hipStream_t st);
// The same adjoint without checkpoints: each u_t is recomputed from v into
// rec_a / rec_b ([n][3][V] each); n_sq >= 2.
void run_exp_bwd_recompute(const float* v, const float* g_u, float* g_v, float* tmp_a,
                           float* tmp_b, float* rec_a, float* rec_b, int* aux, const Geom& g,
                           int n, int n_sq, hipStream_t st);

// One inner iteration of n subjects (Exp, warp + MSE or L1 + regulariser,
// both adjoints, Adam on v in place) in one persistent launch of at most as
// many blocks as the device holds at once, its phases separated by grid
// barriers; for small cohorts.  ckpt [n_sq-1][n][3][V], aux (records), uN,
// gU, gA, gB, gV [n][3][V] are scratch; bar and err are two device words (err
// zeroed once; raised if a barrier wait timed out).  The Adam step count is
// *step_dev + k + 1 when step_dev is given, else step_host + k + 1; Adam's
// results go to v_out, m_out, s_out when given (timing runs), else to v, m,
// s.  Returns false (nothing enqueued) when the launch cannot be made
// resident.
bool run_iter_fused(const float* img, const float* atlas, float* v, float* m, float* s,
                    float* ckpt, int* aux, float* uN, float* gU, float* gA, float* gB, float* gV,
                    double* loss, int loss_stride, const RegW& rw, const Geom& g, int n, int n_sq,
                    const long long* step_dev, long long step_host, int k, float lr, double b1,
                    double b2, float eps, bool l1, unsigned* bar, int* err, hipStream_t st,
                    float* v_out = nullptr, float* m_out = nullptr, float* s_out = nullptr);
// out[0] = NaN when err[0] is raised.
void flag_fused_error(const int* err, double* out, hipStream_t st);
// Blocks of the fused kernel the current device holds at once.
int fused_resident_blocks(bool l1);
// Bound of one grid-barrier wait of the fused kernel, in ticks of the 100 MHz
// real-time counter; negative restores the default (1 s).
constexpr long long kDefaultBarrierTicks = 100000000;
void set_barrier_ticks(long long ticks);

// --- warp -----------------------------------------------------------------
void launch_warp(const float* img, const float* u, float* out, const Geom& g, int n,
                 hipStream_t st);
void launch_warp_bwd(const float* img, const float* u, const float* gout, float* gu, const Geom& g,
                     int n, hipStream_t st);

// --- dissimilarities and regulariser --------------------------------------
// MSE (or L1 when l1) on given warped images: loss[i * loss_stride] += D_i;
// gw may be null.
void launch_mse(const float* w, const float* atlas, double* loss, int loss_stride, float* gw,
                const Geom& g, int n, bool l1, hipStream_t st);
// Warp + MSE or L1 + (optional) diffusion regulariser, fused.  With gu
// non-null it also writes gu = dL/du (overwrite); loss[i * loss_stride] +=
// D_i + lam R(u_i).
void launch_mse_fused(const float* img, const float* atlas, const float* u, float* gu,
                      double* loss, int loss_stride, const RegW& rw, const Geom& g, int n, bool l1,
                      hipStream_t st);
// Diffusion regulariser of an ncomp-component field: out += lam dR/din
// (when out is non-null) and loss[i * loss_stride] += lam R (when non-null).
void launch_diffusion(const float* in, float* out, double* loss, int loss_stride, const RegW& rw,
                      const Geom& g, int n, int ncomp, hipStream_t st);

// LNCC forward.  fields ([n][4][V], may be null) receives alpha, alpha*Jbar,
// beta, beta*Ibar; loss[i * loss_stride] += -(1/V) sum cc.  Returns false when
// the window size is not built.
bool launch_lncc_fwd(const float* w, const float* atlas, float* fields, double* loss,
                     int loss_stride, int win, double eps, const Geom& g, int n, hipStream_t st);
// LNCC adjoint: gw = dD/dw from the fields (gw [n][V]).
bool launch_lncc_bwd(const float* fields, const float* w, const float* atlas, float* gw, int win,
                     const Geom& g, int n, hipStream_t st);
// LNCC adjoint fused with the warp adjoint and the regulariser: gu = dL/du
// (overwrite); loss[i * loss_stride] += lam R(u_i).
bool launch_lncc_bwd_fused(const float* fields, const float* w, const float* atlas,
                           const float* img, const float* u, float* gu, double* loss,
                           int loss_stride, const RegW& rw, int win, const Geom& g, int n,
                           hipStream_t st);

// dD(warped_i, A)/dA for each of n warped subjects (the LNCC of one atlas
// against n images; cc is symmetric in its two images): ga [n][V] (overwrite),
// fields [n][4][V] scratch, loss[i * loss_stride] += D_i.
bool launch_lncc_atlas_grad(const float* warped, const float* atlas, float* fields, float* ga,
                            double* loss, int loss_stride, int win, double eps, const Geom& g,
                            int n, hipStream_t st);

bool lncc_window_supported(int win);
int gauss_radius(float sigma);

// Separable Gaussian of `nchan` volumes (out != in).  Returns false when the
// radius int(3 sigma + 0.5) is outside 1..8.
bool launch_gauss(const float* in, float* out, float sigma, const Geom& g, int nchan,
                  hipStream_t st);

// --- optimiser, centring, atlas -------------------------------------------
void launch_adam(const float* v_in, float* v_out, float* m, float* s, const float* g,
                 long long count, long long t, float lr, double b1, double b2, float eps,
                 hipStream_t st);
void launch_center(float* u, float* mean_out, const Geom& g, int n, hipStream_t st);
void launch_atlas(const float* images, const float* u, const float* mean, float* atlas,
                  const Geom& g, int n, hipStream_t st);

// --- chunk lengths of the marching kernels ---------------------------------
// Planes per block along d0.  0 = not tuned (the launchers then use their own
// heuristic); set by darc_autotune for one volume shape and batch size.
enum TuneKind : int { TUNE_EXP = 0, TUNE_WINDOW = 1, TUNE_FUSED = 2, TUNE_NUM };
int tuned_tz(int kind, const Geom& g, int n);
void set_tuned_tz(int kind, const Geom& g, int n, int tz);
void clear_tuned();

// --- Adam with a device-side step count (graph-capturable) ------------------
// The update of inner iteration k uses t = *step_dev + k + 1: bc[0] = 1 - b1^t
// and bc[1] = 1 - b2^t are formed on the device first.  launch_step_add then
// advances *step_dev once all subjects have taken their steps.
void launch_adam_dev(const float* v_in, float* v_out, float* m, float* s, const float* g,
                     long long count, const long long* step_dev, int k, float* bc, float lr,
                     double b1, double b2, float eps, hipStream_t st);
void launch_step_add(long long* step_dev, long long k, hipStream_t st);

// --- other branches: L1 atlas, stochastic NCC atlas, labels, resampling ----
// Threads per block of the median atlas for n subjects (0: n > 512 is not
// supported); each thread keeps n samples in LDS.
int median_threads(int n);
void launch_atlas_median(const float* images, const float* u, const float* mean, float* atlas,
                         const Geom& g, int n, hipStream_t st);
// a <- Adam(a, (1/nb) sum_j ga[j]) with step count t; ga is [nb][V].
void launch_adam_batch_mean(float* a, float* m, float* s, const float* ga, int nb, long long V,
                            long long t, float lr, double b1, double b2, float eps,
                            hipStream_t st);
// out [n][V] = labels [V] carried by u [n][3][V] (nearest voxel, 0 outside).
void launch_warp_labels(const uint8_t* labels, const float* u, uint8_t* out, const Geom& g, int n,
                        hipStream_t st);
// counts [n][L][3] += per-label (intersection, |a = l|, |b = l|); L <= 256.
void launch_dice_counts(const uint8_t* a, const uint8_t* b, int n, long long V, int L,
                        unsigned long long* counts, hipStream_t st);
// 2x2x2 averaging of nchan volumes of the (even) fine geometry, and trilinear
// upsampling of nchan coarse volumes onto the fine geometry, times scale.
void launch_down2(const float* in, float* out, const Geom& fine, int nchan, hipStream_t st);
void launch_up2(const float* in, float* out, const Geom& fine, int nchan, float scale,
                hipStream_t st);

// --- warm-start network ----------------------------------------------------
// One 3x3x3 (ntaps 27) or 1x1x1 (ntaps 1) convolution, zero padding, as an
// implicit GEMM on the BF16 matrix cores (see unet_kernels.hip for layouts).
struct ConvGeom {
  long long nvox;     // n * o0 * o1 * o2 (GEMM rows)
  int i0, i1, i2;     // input dims (full resolution)
  int o0, o1, o2;     // output dims, (i - 1) / stride + 1
  int stride, ntaps;  // 1 or 2; 27 or 1
  int c0, c1;         // channels of x0 and x1 (multiples of 8; c1 may be 0)
  int up0;            // x0 is at half resolution, doubled by nearest neighbour
  int dil0;           // x0 is at half resolution on the even positions only (zeros between)
  int kpad, cout, act;
  float slope;
  int ycl32, accum;   // y32 channels-last [nvox][cout] instead of planar; add to y32
  int csplit;         // > 0 (with ycl32): y32 takes channels [0, csplit) as [nvox][csplit]
  float* y32b;        //   and y32b channels [csplit, cout) as [nvox][cout - csplit]
  // non-null (with ycl32, csplit 0): the adjoint of the next layer's leaky
  // ReLU fused, dz16 [nvox][cout] = BF16(g * (acty > 0 ? 1 : slope)), g the
  // value (+ y32 when accum; y32 is then only read), acty that layer's
  // forward output [nvox][cout]
  uint16_t* dz16;
  const uint16_t* acty;
  // non-zero (with csplit, stride 1, 27 taps, even output dims; LDS-staged
  // kernel only): channels [0, csplit) are summed over the 2 x 2 x 2
  // children of each half-resolution voxel and written with the adjoint
  // fused, dz16 [n][o/2][csplit] = BF16(sum * (acty > 0 ? 1 : slope)), acty
  // [n][o/2][csplit] (the adjoint of nearest upsampling, then of the leaky
  // ReLU that made the half-resolution tensor); y32 is then unused
  int hpool;
};
// Weight row length for cin input channels: ntaps * ceil(cin/8) * 8 rounded up to 32.
int conv_kpad(int cin, int ntaps);
// y16 (channels-last BF16 [nvox][cout]) or y32 (planar FP32 [n][cout][O]).
void launch_conv3d(const uint16_t* x0, const uint16_t* x1, const uint16_t* w, const float* bias,
                   uint16_t* y16, float* y32, const ConvGeom& cg, hipStream_t st);
// x [n][V][cpad] BF16 = (atlas, image_i, 0 ...)
void launch_pack_pair(const float* atlas, const float* images, uint16_t* x, long long V, int n,
                      int cpad, hipStream_t st);

// --- training of the warm-start network ------------------------------------
// dw [cout][kpad] += sum over the forward conv cg's output voxels of
// dz[v][co] * X(v, k) (X the conv's input patch, as the forward loader reads
// it); dz channels-last BF16 [nvox][cz].  db [cout] += sum_v dz[v][co].
void launch_conv_wgrad(const uint16_t* dz, int cz, const uint16_t* x0, const uint16_t* x1,
                       const ConvGeom& cg, float* dw, float* db, hipStream_t st);
// Weights of the input-gradient convolution: wt[ci][k'] for k' = tap' * cz + co,
// = w[co][(26 - tap') * cin + ci] (flipped taps, exchanged channels), from the
// FP32 master weights w [cout][kpad_f]; zero for co >= cout, tap' >= 27.
void launch_pack_wt(const float* w, int cin, int cout, int cz, int kpad_f, int kpad_t,
                    uint16_t* wt, hipStream_t st);
// out = BF16(in), count values
void launch_to_bf16(const float* in, uint16_t* out, long long count, hipStream_t st);
// p, t [n][c][V]: loss += sum (p - t)^2 / count (FP64, count = n c V) and
// dz [n V][cz] channels-last BF16 = 2 (p - t) / count below channel c, zero
// from c to cz (c <= cz, cz a multiple of 8)
void launch_mse_dz(const float* p, const float* t, int n, long long V, int c, int cz,
                   double* loss, uint16_t* dz, hipStream_t st);

// --- small helpers --------------------------------------------------------
void launch_fill_f32(float* p, long long count, float value, hipStream_t st);
void launch_fill_f64(double* p, long long count, double value, hipStream_t st);
// out[0] = scale * sum_{i < n} in[i]
void launch_sum_f64(const double* in, int n, double scale, double* out, hipStream_t st);

}  // namespace darc
