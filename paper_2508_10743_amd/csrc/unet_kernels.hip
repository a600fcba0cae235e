// The convolutions of the warm-start network: 3x3x3 (or 1x1x1) convolutions
// as implicit GEMMs on the BF16 matrix cores of gfx950.
//
// GEMM view of one convolution: rows M = output voxels (all subjects of the
// launch), columns N = output channels, reduction K = taps x input channels.
// Activations are channels-last BF16 ([n][voxel][C], C a multiple of 8), so
// one reduction step of 8 consecutive K entries is 8 channels of one tap: a
// single 16-byte load.  Weights are [Cout][Kpad] BF16 with
//   k = (tap * (Cin / 8) + v) * 8 + j,  tap = (a * 3 + b) * 3 + c,
// channel 8 v + j of tap offset (a - 1, b - 1, c - 1) (zero beyond 27 taps,
// Kpad a multiple of 32).  The input may be the concatenation of x0 (first
// c0 channels, optionally at half resolution and doubled by nearest
// neighbour) and x1 (next c1 channels), which is how the decoder reads its
// upsampled and skip tensors without materialising either.
//
// One wave computes a 16-voxel x (16 * NT16) tile with
// v_mfma_f32_16x16x32_bf16: per 32-wide K step, lane l supplies the A row
// l % 16 (its voxel) and B column l % 16 at K entries 8 (l / 16) .. + 7, and
// holds output rows 4 (l / 16) .. + 3 of column l % 16.  FP32 accumulation;
// bias, leaky ReLU and the BF16 rounding (to nearest even) in the epilogue.
#include "darc_kernels.hpp"

namespace darc {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int CWAVES = 4;              // waves per block
constexpr int CNT = 64 * CWAVES;       // threads per block
constexpr int CROWS = 16 * CWAVES;     // output voxels per block

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);  // NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

template <int NT16>
__global__ __launch_bounds__(CNT) void k_conv3d(const uint16_t* __restrict__ x0,
                                                const uint16_t* __restrict__ x1,
                                                const uint16_t* __restrict__ w,
                                                const float* __restrict__ bias,
                                                uint16_t* __restrict__ y16,
                                                float* __restrict__ y32, ConvGeom cg) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kg = lane >> 4;
  const long long m = static_cast<long long>(blockIdx.x) * CROWS + wave * 16 + r;
  const bool mv = m < cg.nvox;
  // output coordinates of this lane's A row
  int s = 0, o0 = 0, o1 = 0, o2 = 0;
  if (mv) {
    const long long ov = static_cast<long long>(cg.o0) * cg.o1 * cg.o2;
    s = static_cast<int>(m / ov);
    int rem = static_cast<int>(m - static_cast<long long>(s) * ov);
    o2 = rem % cg.o2;
    rem /= cg.o2;
    o1 = rem % cg.o1;
    o0 = rem / cg.o1;
  }
  const int nco0 = blockIdx.y * 16 * NT16;
  f32x4 acc[NT16];
#pragma unroll
  for (int t = 0; t < NT16; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const int cvec = (cg.c0 + cg.c1) >> 3;
  const int h0 = cg.up0 ? cg.i0 / 2 : cg.i0, h1 = cg.up0 ? cg.i1 / 2 : cg.i1,
            h2 = cg.up0 ? cg.i2 / 2 : cg.i2;
  for (int kc = 0; kc < cg.kpad; kc += 32) {
    // A fragment: 8 channels of one tap at this lane's voxel
    const int kv = (kc >> 3) + kg;
    const int tap = kv / cvec, v = kv - tap * cvec;
    uint4 araw = make_uint4(0u, 0u, 0u, 0u);
    if (mv && tap < cg.ntaps) {
      int a = 1, b = 1, c = 1;
      if (cg.ntaps == 27) {
        a = tap / 9;
        b = (tap / 3) % 3;
        c = tap % 3;
      }
      const int p0 = o0 * cg.stride + a - 1, p1 = o1 * cg.stride + b - 1,
                p2 = o2 * cg.stride + c - 1;
      if (p0 >= 0 && p0 < cg.i0 && p1 >= 0 && p1 < cg.i1 && p2 >= 0 && p2 < cg.i2) {
        const int ch = v * 8;
        const uint16_t* src;
        if (ch < cg.c0) {
          const int q0 = cg.up0 ? p0 >> 1 : p0, q1 = cg.up0 ? p1 >> 1 : p1,
                    q2 = cg.up0 ? p2 >> 1 : p2;
          src = x0 + ((((static_cast<long long>(s) * h0 + q0) * h1 + q1) * h2 + q2) * cg.c0 + ch);
        } else {
          src = x1 + ((((static_cast<long long>(s) * cg.i0 + p0) * cg.i1 + p1) * cg.i2 + p2) *
                          cg.c1 + (ch - cg.c0));
        }
        araw = *reinterpret_cast<const uint4*>(src);
      }
    }
    const bf16x8 afrag = __builtin_bit_cast(bf16x8, araw);
#pragma unroll
    for (int t = 0; t < NT16; ++t) {
      const int co = nco0 + t * 16 + r;
      uint4 braw = make_uint4(0u, 0u, 0u, 0u);
      if (co < cg.cout)
        braw = *reinterpret_cast<const uint4*>(w + static_cast<long long>(co) * cg.kpad + kc + kg * 8);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag, __builtin_bit_cast(bf16x8, braw),
                                                       acc[t], 0, 0, 0);
    }
  }
  // epilogue: lane holds rows 4 kg .. 4 kg + 3 of column r of each N sub-tile
  const long long ov = static_cast<long long>(cg.o0) * cg.o1 * cg.o2;
#pragma unroll
  for (int t = 0; t < NT16; ++t) {
    const int co = nco0 + t * 16 + r;
    if (co >= cg.cout) continue;
    const float bb = bias ? bias[co] : 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long long mo = static_cast<long long>(blockIdx.x) * CROWS + wave * 16 + kg * 4 + i;
      if (mo >= cg.nvox) continue;
      float val = acc[t][i] + bb;
      if (cg.act) val = val > 0.0f ? val : cg.slope * val;
      if (y16) {
        y16[mo * cg.cout + co] = to_bf16(val);
      } else {
        const long long so = mo / ov;
        y32[(so * cg.cout + co) * ov + (mo - so * ov)] = val;
      }
    }
  }
}

// x [n][V][cpad] BF16 = (A, I_i, 0, ...): the network's input pair.
__global__ __launch_bounds__(kBlock) void k_pack_pair(const float* __restrict__ atlas,
                                                      const float* __restrict__ images,
                                                      uint16_t* __restrict__ x, long long V,
                                                      int n, int cpad) {
  const long long i = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= V * n) return;
  const long long s = i / V, vx = i - s * V;
  uint16_t* o = x + i * cpad;
  o[0] = to_bf16(atlas[vx]);
  o[1] = to_bf16(images[s * V + vx]);
  for (int c = 2; c < cpad; ++c) o[c] = 0;
}

}  // namespace

int conv_kpad(int cin, int ntaps) {
  const int cv = (cin + 7) / 8;
  return (ntaps * cv * 8 + 31) / 32 * 32;
}

void launch_conv3d(const uint16_t* x0, const uint16_t* x1, const uint16_t* w, const float* bias,
                   uint16_t* y16, float* y32, const ConvGeom& cg, hipStream_t st) {
  const uint32_t gx = static_cast<uint32_t>((cg.nvox + CROWS - 1) / CROWS);
  prof_begin(st, KC_MISC);
  if (cg.cout <= 16) {
    hipLaunchKernelGGL(k_conv3d<1>, dim3(gx, 1), dim3(CNT), 0, st, x0, x1, w, bias, y16, y32, cg);
  } else if (cg.cout <= 32) {
    hipLaunchKernelGGL(k_conv3d<2>, dim3(gx, 1), dim3(CNT), 0, st, x0, x1, w, bias, y16, y32, cg);
  } else {
    const uint32_t gy = static_cast<uint32_t>((cg.cout + 63) / 64);
    hipLaunchKernelGGL(k_conv3d<4>, dim3(gx, gy), dim3(CNT), 0, st, x0, x1, w, bias, y16, y32,
                       cg);
  }
  prof_end(st, KC_MISC);
}

void launch_pack_pair(const float* atlas, const float* images, uint16_t* x, long long V, int n,
                      int cpad, hipStream_t st) {
  const long long tot = V * n;
  prof_begin(st, KC_MISC);
  hipLaunchKernelGGL(k_pack_pair, dim3(static_cast<uint32_t>((tot + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, st, atlas, images, x, V, n, cpad);
  prof_end(st, KC_MISC);
}

}  // namespace darc
