// Voxel-parallel kernels of libdarc: warping and its adjoint, MSE, the
// diffusion regulariser, Adam, the centrality activation and the mean atlas.  One thread per voxel, 256-thread
// blocks, blocks remapped so that each XCD walks a contiguous range of voxels
// (the gathers of neighbouring voxels then share that XCD's L2).
#include "darc_kernels.hpp"
#include "voxel_bodies.hpp"

namespace darc {

namespace {

struct VoxelBlock {
  uint32_t s;  // subject within the launch
  int lin;     // voxel index, may be >= V in the last block
};

__device__ __forceinline__ VoxelBlock voxel_block(uint32_t nbx, uint32_t total) {
  const uint32_t b = xcd_remap(blockIdx.x, total);
  const uint32_t s = b / nbx;
  VoxelBlock r;
  r.s = s;
  r.lin = static_cast<int>((b - s * nbx) * kBlock + threadIdx.x);
  return r;
}

// -------------------------------------------------------------------- warp

__global__ __launch_bounds__(kBlock) void k_warp(const float* __restrict__ img,
                                                 const float* __restrict__ u,
                                                 float* __restrict__ out, Geom g, uint32_t nbx,
                                                 uint32_t total) {
  const VoxelBlock vb = voxel_block(nbx, total);
  if (vb.lin >= g.V) return;
  const int lin = vb.lin;
  const float* I = img + static_cast<size_t>(vb.s) * g.V;
  const float* f = u + static_cast<size_t>(vb.s) * 3 * g.V;
  int x0, x1, x2;
  voxel_coords(g, lin, x0, x1, x2);
  out[static_cast<size_t>(vb.s) * g.V + lin] =
      sample_zero_value(I, g, x0, x1, x2, f[lin], f[g.V + lin], f[2 * g.V + lin]);
}

__global__ __launch_bounds__(kBlock) void k_warp_bwd(const float* __restrict__ img,
                                                     const float* __restrict__ u,
                                                     const float* __restrict__ gout,
                                                     float* __restrict__ gu, Geom g, uint32_t nbx,
                                                     uint32_t total) {
  const VoxelBlock vb = voxel_block(nbx, total);
  if (vb.lin >= g.V) return;
  const int lin = vb.lin;
  const float* I = img + static_cast<size_t>(vb.s) * g.V;
  const size_t off = static_cast<size_t>(vb.s) * 3 * g.V;
  const float* f = u + off;
  float* o = gu + off;
  int x0, x1, x2;
  voxel_coords(g, lin, x0, x1, x2);
  const Tri t = sample_zero(I, g, x0, x1, x2, f[lin], f[g.V + lin], f[2 * g.V + lin]);
  const float go = gout[static_cast<size_t>(vb.s) * g.V + lin];
  o[lin] += go * t.d0;
  o[g.V + lin] += go * t.d1;
  o[2 * g.V + lin] += go * t.d2;
}

// -------------------------------------------------------------------- MSE

template <bool L1>
__global__ __launch_bounds__(kBlock) void k_mse(const float* __restrict__ w,
                                                const float* __restrict__ atlas,
                                                double* __restrict__ loss, int loss_stride,
                                                float* __restrict__ gw, Geom g, double inv_v,
                                                uint32_t nbx, uint32_t total) {
  __shared__ double red[kBlock / 64];
  const VoxelBlock vb = voxel_block(nbx, total);
  double acc = 0.0;
  if (vb.lin < g.V) {
    const size_t idx = static_cast<size_t>(vb.s) * g.V + vb.lin;
    const double diff = static_cast<double>(w[idx]) - static_cast<double>(atlas[vb.lin]);
    acc = point_loss<L1>(diff);
    if (gw) gw[idx] = point_grad<L1>(diff, inv_v);
  }
  const double tot = block_sum<kBlock>(acc, red);
  if (threadIdx.x == 0) atomicAdd(loss + static_cast<size_t>(vb.s) * loss_stride, tot * inv_v);
}

// Warp + MSE or L1 + diffusion regulariser (+ their adjoints when GRAD).
template <bool L1, bool GRAD>
__global__ __launch_bounds__(kBlock) void k_mse_fused(const float* __restrict__ img,
                                                      const float* __restrict__ atlas,
                                                      const float* __restrict__ u,
                                                      float* __restrict__ gu,
                                                      double* __restrict__ loss, int loss_stride,
                                                      RegW rw, Geom g, double inv_v, uint32_t nbx,
                                                      uint32_t total) {
  __shared__ double red[kBlock / 64];
  mse_fused_block<L1, GRAD>(xcd_remap(blockIdx.x, total), red, img, atlas, u, gu, loss,
                            loss_stride, rw, g, inv_v, nbx);
}

// Diffusion regulariser of an ncomp-component field (one launch covers the
// ncomp components of each subject, blocks over voxels).
__global__ __launch_bounds__(kBlock) void k_diffusion(const float* __restrict__ in,
                                                      float* __restrict__ out,
                                                      double* __restrict__ loss, int loss_stride,
                                                      RegW rw, Geom g, int ncomp, uint32_t nbx,
                                                      uint32_t total) {
  __shared__ double red[kBlock / 64];
  const VoxelBlock vb = voxel_block(nbx, total);
  double racc = 0.0;
  if (vb.lin < g.V) {
    const int lin = vb.lin;
    int x0, x1, x2;
    voxel_coords(g, lin, x0, x1, x2);
    const size_t off = static_cast<size_t>(vb.s) * ncomp * g.V;
    for (int c = 0; c < ncomp; ++c) {
      const float gr = reg_at(in + off + static_cast<size_t>(c) * g.V, g, lin, x0, x1, x2, rw, racc);
      if (out) out[off + static_cast<size_t>(c) * g.V + lin] += gr;
    }
  }
  if (loss) {
    const double tot = block_sum<kBlock>(racc, red);
    if (threadIdx.x == 0) atomicAdd(loss + static_cast<size_t>(vb.s) * loss_stride, rw.lam * tot);
  }
}

// ------------------------------------------------------------------- Adam

__global__ __launch_bounds__(kBlock) void k_adam(const float* __restrict__ v_in,
                                                 float* __restrict__ v_out, float* __restrict__ m,
                                                 float* __restrict__ s,
                                                 const float* __restrict__ g, long long count,
                                                 float lr, float b1, float omb1, float b2,
                                                 float omb2, float bc1, float bc2, float eps) {
  const long long stride = static_cast<long long>(gridDim.x) * kBlock;
  for (long long i = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x; i < count;
       i += stride)
    adam_update(v_in, v_out, m, s, g, i, lr, b1, omb1, b2, omb2, bc1, bc2, eps);
}

// The step count lives on the device so that a captured sweep can be
// replayed: one thread advances it and forms the bias corrections in FP64.
__global__ void k_adam_prep(const long long* __restrict__ step, int k, float* __restrict__ bc,
                            double b1, double b2) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double t = static_cast<double>(step[0] + k + 1);
    bc[0] = static_cast<float>(1.0 - pow(b1, t));
    bc[1] = static_cast<float>(1.0 - pow(b2, t));
  }
}

__global__ void k_step_add(long long* __restrict__ step, long long k) {
  if (threadIdx.x == 0 && blockIdx.x == 0) step[0] += k;
}

__global__ __launch_bounds__(kBlock) void k_adam_dev(const float* __restrict__ v_in,
                                                     float* __restrict__ v_out,
                                                     float* __restrict__ m, float* __restrict__ s,
                                                     const float* __restrict__ g, long long count,
                                                     float lr, float b1, float omb1, float b2,
                                                     float omb2, const float* __restrict__ bc,
                                                     float eps) {
  const float bc1 = bc[0], bc2 = bc[1];
  const long long stride = static_cast<long long>(gridDim.x) * kBlock;
  for (long long i = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x; i < count;
       i += stride)
    adam_update(v_in, v_out, m, s, g, i, lr, b1, omb1, b2, omb2, bc1, bc2, eps);
}

// ---------------------------------------------------------------- centring

// mean(e) = (1/n) sum_i u_i(e) over the 3V entries e; u_i <- u_i - mean.
// REGS (n <= kCenterRegs): the n values stay in registers between the sum
// and the update, so each entry is read once; the sum runs in the same order
// (unused slots add exact zeros).
constexpr int kCenterRegs = 16;

template <bool REGS>
__global__ __launch_bounds__(kBlock) void k_center(float* __restrict__ u,
                                                   float* __restrict__ mean_out, int n,
                                                   long long fs) {
  const long long e = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= fs) return;
  if (REGS) {
    // every slot loads (slots past n repeat subject n - 1, then count zero):
    // a load under a branch would be waited for at once
    float x[kCenterRegs];
#pragma unroll
    for (int i = 0; i < kCenterRegs; ++i) x[i] = u[min(i, n - 1) * fs + e];
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < kCenterRegs; ++i) acc += i < n ? static_cast<double>(x[i]) : 0.0;
    const double mean = acc / n;
    if (mean_out) mean_out[e] = static_cast<float>(mean);
#pragma unroll
    for (int i = 0; i < kCenterRegs; ++i)
      if (i < n) u[i * fs + e] = static_cast<float>(static_cast<double>(x[i]) - mean);
  } else {
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += static_cast<double>(u[i * fs + e]);
    const double mean = acc / n;
    if (mean_out) mean_out[e] = static_cast<float>(mean);
    for (int i = 0; i < n; ++i)
      u[i * fs + e] = static_cast<float>(static_cast<double>(u[i * fs + e]) - mean);
  }
}

// ------------------------------------------------------------------- atlas

__global__ __launch_bounds__(kBlock) void k_atlas(const float* __restrict__ images,
                                                  const float* __restrict__ u,
                                                  const float* __restrict__ mean,
                                                  float* __restrict__ atlas, Geom g, int n,
                                                  uint32_t nbx, uint32_t total) {
  const VoxelBlock vb = voxel_block(nbx, total);
  if (vb.lin >= g.V) return;
  const int lin = vb.lin;
  int x0, x1, x2;
  voxel_coords(g, lin, x0, x1, x2);
  float m0 = 0.0f, m1 = 0.0f, m2 = 0.0f;
  if (mean) {
    m0 = mean[lin];
    m1 = mean[g.V + lin];
    m2 = mean[2 * g.V + lin];
  }
  double acc = 0.0;
  if (!u) {
    // zero displacements: the sample at x is the voxel itself
    for (int i = 0; i < n; ++i) acc += static_cast<double>(images[static_cast<size_t>(i) * g.V + lin]);
  } else {
    for (int i = 0; i < n; ++i) {
      const float* f = u + static_cast<size_t>(i) * 3 * g.V;
      const float* I = images + static_cast<size_t>(i) * g.V;
      acc += static_cast<double>(sample_zero_value(I, g, x0, x1, x2, f[lin] - m0,
                                                   f[g.V + lin] - m1, f[2 * g.V + lin] - m2));
    }
  }
  atlas[lin] = static_cast<float>(acc / n);
}

// ---------------------------------------------------------------- helpers

__global__ __launch_bounds__(kBlock) void k_fill_f32(float* __restrict__ p, long long count,
                                                     float value) {
  const long long stride = static_cast<long long>(gridDim.x) * kBlock;
  for (long long i = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x; i < count;
       i += stride)
    p[i] = value;
}

__global__ __launch_bounds__(kBlock) void k_fill_f64(double* __restrict__ p, long long count,
                                                     double value) {
  const long long stride = static_cast<long long>(gridDim.x) * kBlock;
  for (long long i = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x; i < count;
       i += stride)
    p[i] = value;
}

__global__ __launch_bounds__(kBlock) void k_sum_f64(const double* __restrict__ in, int n,
                                                    double scale, double* __restrict__ out) {
  __shared__ double red[kBlock / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) acc += in[i];
  const double tot = block_sum<kBlock>(acc, red);
  if (threadIdx.x == 0) out[0] = scale * tot;
}

inline uint32_t grid_stride_blocks(long long count) {
  const long long b = (count + kBlock - 1) / kBlock;
  return static_cast<uint32_t>(b < 65536 ? (b < 1 ? 1 : b) : 65536);
}

}  // namespace

// ==========================================================================
// launchers

RegW make_regw(const Geom& g, int ncomp, float lam) {
  RegW r;
  const int ds[3] = {g.d0, g.d1, g.d2};
  for (int d = 0; d < 3; ++d) {
    const double cnt = static_cast<double>(ncomp) * (ds[d] - 1) * (static_cast<double>(g.V) / ds[d]);
    r.w[d] = 1.0 / (3.0 * cnt);
    r.g[d] = static_cast<float>(static_cast<double>(lam) * 2.0 * r.w[d]);
  }
  r.lam = lam;
  r.on = lam != 0.0f;
  return r;
}

void launch_warp(const float* img, const float* u, float* out, const Geom& g, int n,
                 hipStream_t st) {
  const uint32_t nbx = blocks_for(g.V, kBlock), total = nbx * n;
  prof_begin(st, KC_WARP);
  hipLaunchKernelGGL(k_warp, dim3(total), dim3(kBlock), 0, st, img, u, out, g, nbx, total);
  prof_end(st, KC_WARP);
}

void launch_warp_bwd(const float* img, const float* u, const float* gout, float* gu, const Geom& g,
                     int n, hipStream_t st) {
  const uint32_t nbx = blocks_for(g.V, kBlock), total = nbx * n;
  prof_begin(st, KC_WARP_BWD);
  hipLaunchKernelGGL(k_warp_bwd, dim3(total), dim3(kBlock), 0, st, img, u, gout, gu, g, nbx,
                     total);
  prof_end(st, KC_WARP_BWD);
}

void launch_mse(const float* w, const float* atlas, double* loss, int loss_stride, float* gw,
                const Geom& g, int n, bool l1, hipStream_t st) {
  const uint32_t nbx = blocks_for(g.V, kBlock), total = nbx * n;
  prof_begin(st, KC_MSE);
  if (l1)
    hipLaunchKernelGGL(k_mse<true>, dim3(total), dim3(kBlock), 0, st, w, atlas, loss, loss_stride,
                       gw, g, 1.0 / g.V, nbx, total);
  else
    hipLaunchKernelGGL(k_mse<false>, dim3(total), dim3(kBlock), 0, st, w, atlas, loss, loss_stride,
                       gw, g, 1.0 / g.V, nbx, total);
  prof_end(st, KC_MSE);
}

template <bool L1>
void mse_fused_l(const float* img, const float* atlas, const float* u, float* gu, double* loss,
                 int loss_stride, const RegW& rw, const Geom& g, int n, hipStream_t st) {
  const uint32_t nbx = blocks_for(g.V, kBlock), total = nbx * n;
  if (gu)
    hipLaunchKernelGGL((k_mse_fused<L1, true>), dim3(total), dim3(kBlock), 0, st, img, atlas, u,
                       gu, loss, loss_stride, rw, g, 1.0 / g.V, nbx, total);
  else
    hipLaunchKernelGGL((k_mse_fused<L1, false>), dim3(total), dim3(kBlock), 0, st, img, atlas, u,
                       gu, loss, loss_stride, rw, g, 1.0 / g.V, nbx, total);
}

void launch_mse_fused(const float* img, const float* atlas, const float* u, float* gu,
                      double* loss, int loss_stride, const RegW& rw, const Geom& g, int n, bool l1,
                      hipStream_t st) {
  prof_begin(st, KC_MSE);
  if (l1)
    mse_fused_l<true>(img, atlas, u, gu, loss, loss_stride, rw, g, n, st);
  else
    mse_fused_l<false>(img, atlas, u, gu, loss, loss_stride, rw, g, n, st);
  prof_end(st, KC_MSE);
}

void launch_diffusion(const float* in, float* out, double* loss, int loss_stride, const RegW& rw,
                      const Geom& g, int n, int ncomp, hipStream_t st) {
  const uint32_t nbx = blocks_for(g.V, kBlock), total = nbx * n;
  prof_begin(st, KC_DIFFUSION);
  hipLaunchKernelGGL(k_diffusion, dim3(total), dim3(kBlock), 0, st, in, out, loss, loss_stride, rw,
                     g, ncomp, nbx, total);
  prof_end(st, KC_DIFFUSION);
}

void launch_adam(const float* v_in, float* v_out, float* m, float* s, const float* g,
                 long long count, long long t, float lr, double b1, double b2, float eps,
                 hipStream_t st) {
  // coefficients formed in FP64 and rounded once
  const double bc1 = 1.0 - std::pow(b1, static_cast<double>(t));
  const double bc2 = 1.0 - std::pow(b2, static_cast<double>(t));
  prof_begin(st, KC_ADAM);
  hipLaunchKernelGGL(k_adam, dim3(grid_stride_blocks(count)), dim3(kBlock), 0, st, v_in, v_out, m,
                     s, g, count, lr, static_cast<float>(b1), static_cast<float>(1.0 - b1),
                     static_cast<float>(b2), static_cast<float>(1.0 - b2), static_cast<float>(bc1),
                     static_cast<float>(bc2), eps);
  prof_end(st, KC_ADAM);
}

void launch_adam_dev(const float* v_in, float* v_out, float* m, float* s, const float* g,
                     long long count, const long long* step_dev, int k, float* bc, float lr,
                     double b1, double b2, float eps, hipStream_t st) {
  prof_begin(st, KC_ADAM);
  hipLaunchKernelGGL(k_adam_prep, dim3(1), dim3(64), 0, st, step_dev, k, bc, b1, b2);
  hipLaunchKernelGGL(k_adam_dev, dim3(grid_stride_blocks(count)), dim3(kBlock), 0, st, v_in, v_out,
                     m, s, g, count, lr, static_cast<float>(b1), static_cast<float>(1.0 - b1),
                     static_cast<float>(b2), static_cast<float>(1.0 - b2), bc, eps);
  prof_end(st, KC_ADAM);
}

void launch_step_add(long long* step_dev, long long k, hipStream_t st) {
  prof_begin(st, KC_MISC);
  hipLaunchKernelGGL(k_step_add, dim3(1), dim3(64), 0, st, step_dev, k);
  prof_end(st, KC_MISC);
}

void launch_center(float* u, float* mean_out, const Geom& g, int n, hipStream_t st) {
  const long long fs = 3ll * g.V;
  prof_begin(st, KC_CENTER);
  if (n <= kCenterRegs)
    hipLaunchKernelGGL(k_center<true>, dim3(blocks_for(fs, kBlock)), dim3(kBlock), 0, st, u,
                       mean_out, n, fs);
  else
    hipLaunchKernelGGL(k_center<false>, dim3(blocks_for(fs, kBlock)), dim3(kBlock), 0, st, u,
                       mean_out, n, fs);
  prof_end(st, KC_CENTER);
}

void launch_atlas(const float* images, const float* u, const float* mean, float* atlas,
                  const Geom& g, int n, hipStream_t st) {
  const uint32_t nbx = blocks_for(g.V, kBlock);
  prof_begin(st, KC_ATLAS);
  hipLaunchKernelGGL(k_atlas, dim3(nbx), dim3(kBlock), 0, st, images, u, mean, atlas, g, n, nbx,
                     nbx);
  prof_end(st, KC_ATLAS);
}

void launch_fill_f32(float* p, long long count, float value, hipStream_t st) {
  if (count <= 0) return;
  prof_begin(st, KC_FILL);
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_stride_blocks(count)), dim3(kBlock), 0, st, p, count,
                     value);
  prof_end(st, KC_FILL);
}

void launch_fill_f64(double* p, long long count, double value, hipStream_t st) {
  if (count <= 0) return;
  prof_begin(st, KC_FILL);
  hipLaunchKernelGGL(k_fill_f64, dim3(grid_stride_blocks(count)), dim3(kBlock), 0, st, p, count,
                     value);
  prof_end(st, KC_FILL);
}

void launch_sum_f64(const double* in, int n, double scale, double* out, hipStream_t st) {
  prof_begin(st, KC_MISC);
  hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(kBlock), 0, st, in, n, scale, out);
  prof_end(st, KC_MISC);
}

}  // namespace darc
