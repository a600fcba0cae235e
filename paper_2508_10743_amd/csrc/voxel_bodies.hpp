// Bodies of voxel-parallel kernels shared by their own launches and by the
// fused per-iteration kernel: one block of warp + MSE/L1 + regulariser with
// their adjoints, and the Adam update of one entry.
#pragma once

#include "darc_common.hpp"

namespace darc {

// Pointwise dissimilarity of d = Iw - A: MSE (d^2, gradient 2d/V) or L1
// (|d|, subgradient sign(d)/V with sign(0) = 0).  The difference is formed in
// FP64 from the FP32 inputs, so the sign is exact.
template <bool L1>
__device__ __forceinline__ double point_loss(double d) {
  return L1 ? fabs(d) : d * d;
}
template <bool L1>
__device__ __forceinline__ float point_grad(double d, double inv_v) {
  return L1 ? static_cast<float>(((d > 0.0) - (d < 0.0)) * inv_v)
            : static_cast<float>(2.0 * inv_v * d);
}

// One block of kBlock voxels of one subject (blk = subject * nbx + block
// within the subject, after the caller's XCD remap): warp + MSE or L1 +
// diffusion regulariser, loss[s * loss_stride] += D_s + lam R over the block
// (one FP64 atomic per block), and with GRAD gu = dL/du (overwritten).  `red`
// is kBlock / 64 doubles of LDS; every thread of the block must call it.
template <bool L1, bool GRAD>
__device__ __forceinline__ void mse_fused_block(uint32_t blk, double* red,
                                                const float* __restrict__ img,
                                                const float* __restrict__ atlas,
                                                const float* __restrict__ u,
                                                float* __restrict__ gu, double* __restrict__ loss,
                                                int loss_stride, const RegW& rw, const Geom& g,
                                                double inv_v, uint32_t nbx) {
  const uint32_t sub = blk / nbx;
  const int lin = static_cast<int>((blk - sub * nbx) * kBlock + threadIdx.x);
  double acc = 0.0;
  if (lin < g.V) {
    const float* I = img + static_cast<size_t>(sub) * g.V;
    const size_t off = static_cast<size_t>(sub) * 3 * g.V;
    const float* f = u + off;
    int x0, x1, x2;
    voxel_coords(g, lin, x0, x1, x2);
    const Tri t = sample_zero(I, g, x0, x1, x2, f[lin], f[g.V + lin], f[2 * g.V + lin]);
    const double diff = static_cast<double>(t.v) - static_cast<double>(atlas[lin]);
    acc = point_loss<L1>(diff) * inv_v;
    float r0 = 0.0f, r1 = 0.0f, r2 = 0.0f;
    if (rw.on) {
      double racc = 0.0;
      r0 = reg_at(f, g, lin, x0, x1, x2, rw, racc);
      r1 = reg_at(f + g.V, g, lin, x0, x1, x2, rw, racc);
      r2 = reg_at(f + 2 * g.V, g, lin, x0, x1, x2, rw, racc);
      acc += rw.lam * racc;
    }
    if (GRAD) {
      const float gw = point_grad<L1>(diff, inv_v);
      float* o = gu + off;
      o[lin] = gw * t.d0 + r0;
      o[g.V + lin] = gw * t.d1 + r1;
      o[2 * g.V + lin] = gw * t.d2 + r2;
    }
  }
  const double tot = block_sum<kBlock>(acc, red);
  if (threadIdx.x == 0) atomicAdd(loss + static_cast<size_t>(sub) * loss_stride, tot);
}

// Adam (Kingma & Ba) on entry i: m <- b1 m + (1 - b1) g, s <- b2 s + (1 - b2) g^2,
// v_out = v_in - lr (m / bc1) / (sqrt(s / bc2) + eps), bc = 1 - beta^t.
__device__ __forceinline__ void adam_update(const float* __restrict__ v_in,
                                            float* __restrict__ v_out, float* __restrict__ m,
                                            float* __restrict__ s, const float* __restrict__ g,
                                            long long i, float lr, float b1, float omb1, float b2,
                                            float omb2, float bc1, float bc2, float eps) {
  const float gi = g[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float si = b2 * s[i] + omb2 * gi * gi;
  m[i] = mi;
  s[i] = si;
  v_out[i] = v_in[i] - lr * (mi / bc1) / (sqrtf(si / bc2) + eps);
}

// The same step with the new moments written elsewhere (v_out, m_out, s_out
// may be v, m, s themselves).
__device__ __forceinline__ void adam_step_to(const float* v, const float* m, const float* s,
                                             const float* __restrict__ g, float* v_out,
                                             float* m_out, float* s_out, long long i, float lr,
                                             float b1, float omb1, float b2, float omb2, float bc1,
                                             float bc2, float eps) {
  const float gi = g[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float si = b2 * s[i] + omb2 * gi * gi;
  const float vi = v[i];
  m_out[i] = mi;
  s_out[i] = si;
  v_out[i] = vi - lr * (mi / bc1) / (sqrtf(si / bc2) + eps);
}

}  // namespace darc
