// Kernels of the method's other branches: the L1 (median) atlas, the Adam
// step of the stochastic NCC atlas update, label propagation for one-shot
// segmentation with its Dice counts, and factor-2 resampling between the
// levels of a coarse-to-fine schedule.
#include "darc_kernels.hpp"

namespace darc {

namespace {

// ------------------------------------------------------------ median atlas
//
// A(x) = median_i I_i(x + u_i(x) - mean(x)) (Section 3, "Dissimilarity
// metrics", second closed form).  Each thread owns one voxel and keeps its n
// warped samples in an LDS column (stride T, so a wave's accesses hit
// distinct banks), then selects the middle order statistic in place with
// Hoare's partition-based selection.  For even n the two middle values are
// averaged.
template <int T>
__global__ __launch_bounds__(T) void k_atlas_median(const float* __restrict__ images,
                                                    const float* __restrict__ u,
                                                    const float* __restrict__ mean,
                                                    float* __restrict__ atlas, Geom g, int n,
                                                    uint32_t nblocks) {
  extern __shared__ float col_all[];
  const uint32_t b = xcd_remap(blockIdx.x, nblocks);
  const int lin = static_cast<int>(b * T + threadIdx.x);
  if (lin >= g.V) return;  // no barrier below
  float* col = col_all + threadIdx.x;
  int x0, x1, x2;
  voxel_coords(g, lin, x0, x1, x2);
  float m0 = 0.0f, m1 = 0.0f, m2 = 0.0f;
  if (mean) {
    m0 = mean[lin];
    m1 = mean[g.V + lin];
    m2 = mean[2 * g.V + lin];
  }
  for (int i = 0; i < n; ++i) {
    const float* f = u + static_cast<size_t>(i) * 3 * g.V;
    const float* I = images + static_cast<size_t>(i) * g.V;
    col[i * T] = sample_zero_value(I, g, x0, x1, x2, f[lin] - m0, f[g.V + lin] - m1,
                                   f[2 * g.V + lin] - m2);
  }
  const int k = (n - 1) / 2;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const float x = col[((lo + hi) >> 1) * T];
    int i = lo, j = hi;
    while (i <= j) {
      while (i <= hi && col[i * T] < x) ++i;
      while (j >= lo && x < col[j * T]) --j;
      if (i <= j) {
        const float t = col[i * T];
        col[i * T] = col[j * T];
        col[j * T] = t;
        ++i;
        --j;
      }
    }
    // [lo, j] <= x <= [i, hi], and every entry strictly between equals x
    if (k <= j)
      hi = j;
    else if (k >= i)
      lo = i;
    else
      break;
  }
  float med = col[k * T];
  if ((n & 1) == 0) {
    // the next order statistic is the smallest entry above position k
    float nxt = col[(k + 1) * T];
    for (int i = k + 2; i < n; ++i) nxt = fminf(nxt, col[i * T]);
    med = 0.5f * (med + nxt);
  }
  atlas[lin] = med;
}

// ------------------------------------------------- stochastic atlas update
//
// One Adam step on the atlas along the minibatch mean of the per-subject
// gradients ga [nb][V]: g = (1/nb) sum_i ga_i (Algorithm 1, SGD_for_atlas).
__global__ __launch_bounds__(kBlock) void k_adam_batch_mean(
    float* __restrict__ a, float* __restrict__ m, float* __restrict__ s,
    const float* __restrict__ ga, int nb, long long V, float inv_nb, float lr, float b1,
    float omb1, float b2, float omb2, float bc1, float bc2, float eps) {
  const long long stride = static_cast<long long>(gridDim.x) * kBlock;
  for (long long i = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x; i < V;
       i += stride) {
    float gi = 0.0f;
    for (int j = 0; j < nb; ++j) gi += ga[j * V + i];
    gi *= inv_nb;
    const float mi = b1 * m[i] + omb1 * gi;
    const float si = b2 * s[i] + omb2 * gi * gi;
    m[i] = mi;
    s[i] = si;
    a[i] = a[i] - lr * (mi / bc1) / (sqrtf(si / bc2) + eps);
  }
}

// ----------------------------------------------------- label propagation
//
// out_i(x) = L(round(x + u_i(x))) with round(p) = floor(p + 1/2) taken in
// FP32, label 0 outside the volume (one-shot segmentation, Section 4).
__global__ __launch_bounds__(kBlock) void k_warp_labels(const uint8_t* __restrict__ labels,
                                                        const float* __restrict__ u,
                                                        uint8_t* __restrict__ out, Geom g,
                                                        uint32_t nbx, uint32_t total) {
  const uint32_t b = xcd_remap(blockIdx.x, total);
  const uint32_t s = b / nbx;
  const int lin = static_cast<int>((b - s * nbx) * kBlock + threadIdx.x);
  if (lin >= g.V) return;
  const float* f = u + static_cast<size_t>(s) * 3 * g.V;
  int x0, x1, x2;
  voxel_coords(g, lin, x0, x1, x2);
  const float k0 = floorf(__fadd_rn(__fadd_rn(static_cast<float>(x0), f[lin]), 0.5f));
  const float k1 = floorf(__fadd_rn(__fadd_rn(static_cast<float>(x1), f[g.V + lin]), 0.5f));
  const float k2 = floorf(__fadd_rn(__fadd_rn(static_cast<float>(x2), f[2 * g.V + lin]), 0.5f));
  uint8_t lab = 0;
  // comparisons in float first: NaN and huge positions fall outside
  if (k0 >= 0.0f && k0 < static_cast<float>(g.d0) && k1 >= 0.0f &&
      k1 < static_cast<float>(g.d1) && k2 >= 0.0f && k2 < static_cast<float>(g.d2)) {
    const int i0 = static_cast<int>(k0), i1 = static_cast<int>(k1), i2 = static_cast<int>(k2);
    lab = labels[(i0 * g.d1 + i1) * g.d2 + i2];
  }
  out[static_cast<size_t>(s) * g.V + lin] = lab;
}

// Per label l < L: (|a = l and b = l|, |a = l|, |b = l|), counted in LDS per
// block and added to counts [n][L][3] with 64-bit atomics.
constexpr int kMaxLabels = 256;
__global__ __launch_bounds__(kBlock) void k_dice_counts(const uint8_t* __restrict__ a,
                                                        const uint8_t* __restrict__ bl,
                                                        long long V, int L,
                                                        unsigned long long* __restrict__ counts) {
  __shared__ unsigned int h[3 * kMaxLabels];
  for (int i = threadIdx.x; i < 3 * L; i += kBlock) h[i] = 0u;
  __syncthreads();
  const int s = blockIdx.y;
  const uint8_t* A = a + static_cast<size_t>(s) * V;
  const uint8_t* B = bl + static_cast<size_t>(s) * V;
  const long long stride = static_cast<long long>(gridDim.x) * kBlock;
  for (long long i = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x; i < V;
       i += stride) {
    const int la = A[i], lb = B[i];
    if (la < L) atomicAdd(&h[3 * la + 1], 1u);
    if (lb < L) atomicAdd(&h[3 * lb + 2], 1u);
    if (la == lb && la < L) atomicAdd(&h[3 * la], 1u);
  }
  __syncthreads();
  unsigned long long* c = counts + static_cast<size_t>(s) * 3 * L;
  for (int i = threadIdx.x; i < 3 * L; i += kBlock)
    if (h[i]) atomicAdd(&c[i], static_cast<unsigned long long>(h[i]));
}

// --------------------------------------------------------------- resampling
//
// Coarse voxel k averages fine voxels 2k, 2k+1 per axis; fine voxel x sits at
// coarse coordinate (x - 1/2) / 2.
__global__ __launch_bounds__(kBlock) void k_down2(const float* __restrict__ in,
                                                  float* __restrict__ out, Geom fine, Geom coarse,
                                                  uint32_t nbx, uint32_t total) {
  const uint32_t b = xcd_remap(blockIdx.x, total);
  const uint32_t c = b / nbx;
  const int lin = static_cast<int>((b - c * nbx) * kBlock + threadIdx.x);
  if (lin >= coarse.V) return;
  int k0, k1, k2;
  voxel_coords(coarse, lin, k0, k1, k2);
  const float* f = in + static_cast<size_t>(c) * fine.V;
  const int base = ((2 * k0) * fine.d1 + 2 * k1) * fine.d2 + 2 * k2;
  float acc = 0.0f;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int e = 0; e < 2; ++e) acc += f[base + a * fine.plane + bb * fine.d2 + e];
  out[static_cast<size_t>(c) * coarse.V + lin] = 0.125f * acc;
}

__global__ __launch_bounds__(kBlock) void k_up2(const float* __restrict__ in,
                                                float* __restrict__ out, Geom fine, Geom coarse,
                                                float scale, uint32_t nbx, uint32_t total) {
  const uint32_t b = xcd_remap(blockIdx.x, total);
  const uint32_t c = b / nbx;
  const int lin = static_cast<int>((b - c * nbx) * kBlock + threadIdx.x);
  if (lin >= fine.V) return;
  int x0, x1, x2;
  voxel_coords(fine, lin, x0, x1, x2);
  // (x - 1/2) / 2 is exact in FP32 for these sizes
  const BorderCell bc = border_cell(coarse, 0, 0, 0, (static_cast<float>(x0) - 0.5f) * 0.5f,
                                    (static_cast<float>(x1) - 0.5f) * 0.5f,
                                    (static_cast<float>(x2) - 0.5f) * 0.5f);
  float cv[8];
  corners_border(in + static_cast<size_t>(c) * coarse.V, coarse, bc.base, cv);
  out[static_cast<size_t>(c) * fine.V + lin] = scale * tri_value(cv, bc.t0, bc.t1, bc.t2);
}

}  // namespace

int median_threads(int n) { return n <= 256 ? 64 : (n <= 512 ? 32 : 0); }

void launch_atlas_median(const float* images, const float* u, const float* mean, float* atlas,
                         const Geom& g, int n, hipStream_t st) {
  const int T = median_threads(n);
  const uint32_t nb = blocks_for(g.V, T);
  const size_t lds = static_cast<size_t>(n) * T * sizeof(float);
  prof_begin(st, KC_ATLAS);
  if (T == 64)
    hipLaunchKernelGGL(k_atlas_median<64>, dim3(nb), dim3(64), lds, st, images, u, mean, atlas, g,
                       n, nb);
  else
    hipLaunchKernelGGL(k_atlas_median<32>, dim3(nb), dim3(32), lds, st, images, u, mean, atlas, g,
                       n, nb);
  prof_end(st, KC_ATLAS);
}

void launch_adam_batch_mean(float* a, float* m, float* s, const float* ga, int nb, long long V,
                            long long t, float lr, double b1, double b2, float eps,
                            hipStream_t st) {
  const double bc1 = 1.0 - std::pow(b1, static_cast<double>(t));
  const double bc2 = 1.0 - std::pow(b2, static_cast<double>(t));
  const long long blocks = (V + kBlock - 1) / kBlock;
  const uint32_t grid = static_cast<uint32_t>(blocks < 65536 ? blocks : 65536);
  prof_begin(st, KC_ADAM);
  hipLaunchKernelGGL(k_adam_batch_mean, dim3(grid), dim3(kBlock), 0, st, a, m, s, ga, nb, V,
                     static_cast<float>(1.0 / nb), lr, static_cast<float>(b1),
                     static_cast<float>(1.0 - b1), static_cast<float>(b2),
                     static_cast<float>(1.0 - b2), static_cast<float>(bc1),
                     static_cast<float>(bc2), eps);
  prof_end(st, KC_ADAM);
}

void launch_warp_labels(const uint8_t* labels, const float* u, uint8_t* out, const Geom& g, int n,
                        hipStream_t st) {
  const uint32_t nbx = blocks_for(g.V, kBlock), total = nbx * n;
  prof_begin(st, KC_WARP);
  hipLaunchKernelGGL(k_warp_labels, dim3(total), dim3(kBlock), 0, st, labels, u, out, g, nbx,
                     total);
  prof_end(st, KC_WARP);
}

void launch_dice_counts(const uint8_t* a, const uint8_t* b, int n, long long V, int L,
                        unsigned long long* counts, hipStream_t st) {
  const long long blocks = (V + kBlock - 1) / kBlock;
  const uint32_t gx = static_cast<uint32_t>(blocks < 1024 ? blocks : 1024);
  prof_begin(st, KC_MISC);
  hipLaunchKernelGGL(k_dice_counts, dim3(gx, n), dim3(kBlock), 0, st, a, b, V, L, counts);
  prof_end(st, KC_MISC);
}

void launch_down2(const float* in, float* out, const Geom& fine, int nchan, hipStream_t st) {
  const Geom coarse = make_geom(fine.d0 / 2, fine.d1 / 2, fine.d2 / 2);
  const uint32_t nbx = blocks_for(coarse.V, kBlock), total = nbx * nchan;
  prof_begin(st, KC_MISC);
  hipLaunchKernelGGL(k_down2, dim3(total), dim3(kBlock), 0, st, in, out, fine, coarse, nbx, total);
  prof_end(st, KC_MISC);
}

void launch_up2(const float* in, float* out, const Geom& fine, int nchan, float scale,
                hipStream_t st) {
  const Geom coarse = make_geom(fine.d0 / 2, fine.d1 / 2, fine.d2 / 2);
  const uint32_t nbx = blocks_for(fine.V, kBlock), total = nbx * nchan;
  prof_begin(st, KC_MISC);
  hipLaunchKernelGGL(k_up2, dim3(total), dim3(kBlock), 0, st, in, out, fine, coarse, scale, nbx,
                     total);
  prof_end(st, KC_MISC);
}

}  // namespace darc
