// Shared device helpers and launch plumbing of libdarc (gfx950).
//
// Layout: a volume is [d0][d1][d2] with d2 fastest, a field [3][V] per
// subject (component c displaces axis c), subjects contiguous.  Within one
// subject every offset fits in 32 bits (V <= 2^29); subject offsets are 64-bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <cmath>

namespace darc {

constexpr int kBlock = 256;  // threads per block of the voxel-parallel kernels

// ---------------------------------------------------------------------------
// Division by a divisor fixed at launch time, by a multiply-high and a shift
// (Granlund & Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, the round-up variant).  Exact for dividends
// below 2^31.
struct FastDiv {
  uint32_t d;
  uint32_t mul;
  uint32_t shift;
};

inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  const uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
  return FastDiv{d, static_cast<uint32_t>(m), l};
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return (__umulhi(n, f.mul) + n) >> f.shift;
}

// Voxel geometry passed by value to every kernel.
struct Geom {
  int d0, d1, d2;
  int V;          // d0 * d1 * d2
  int plane;      // d1 * d2
  FastDiv div_d2; // x / d2
  FastDiv div_d1; // (x / d2) / d1
};

inline Geom make_geom(int d0, int d1, int d2) {
  Geom g;
  g.d0 = d0;
  g.d1 = d1;
  g.d2 = d2;
  g.plane = d1 * d2;
  g.V = d0 * g.plane;
  g.div_d2 = make_fastdiv(static_cast<uint32_t>(d2));
  g.div_d1 = make_fastdiv(static_cast<uint32_t>(d1));
  return g;
}

__device__ __forceinline__ void voxel_coords(const Geom& g, int lin, int& x0, int& x1, int& x2) {
  const uint32_t q = fdiv(static_cast<uint32_t>(lin), g.div_d2);
  x2 = lin - static_cast<int>(q) * g.d2;
  const uint32_t r = fdiv(q, g.div_d1);
  x1 = static_cast<int>(q) - static_cast<int>(r) * g.d1;
  x0 = static_cast<int>(r);
}

// ---------------------------------------------------------------------------
// The hardware hands consecutive workgroups of a dispatch to the 8 XCDs in
// turn, and each XCD has its own L2.  Neighbouring voxel tiles share their
// gathers and halos, so the dispatch order is remapped such that every XCD
// walks one contiguous range of tiles.  The map is a bijection on [0, total).
constexpr uint32_t kNumXcd = 8;

__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t total) {
  const uint32_t per = total / kNumXcd;
  const uint32_t rem = total % kNumXcd;
  const uint32_t xcd = b % kNumXcd;
  const uint32_t j = b / kNumXcd;
  return xcd < rem ? xcd * (per + 1) + j : rem * (per + 1) + (xcd - rem) * per + j;
}

// ---------------------------------------------------------------------------
// Trilinear sampling in voxel coordinates.
//
// The position x + u is never formed in FP32 (its ulp grows with x): the cell
// index is x + floor(u), exact, and the fraction u - floor(u), exact except
// for -1 < u < 0 where it is rounded by at most 2^-25 voxel.

// Keeps the displacement finite and small enough for the integer cell index;
// any |u| beyond every volume extent samples the same clamped or zero value.
__device__ __forceinline__ float sane(float u) {
  return fminf(fmaxf(u, -4194304.0f), 4194304.0f);
}

// Cell [i, i+1] and fraction t of the position x + u, for zero padding.
__device__ __forceinline__ void cell_zero(int x, float u, int& i, float& t) {
  const float f = floorf(u);
  i = x + static_cast<int>(f);
  t = u - f;
}

// Cell and fraction for border sampling: the position is clamped into
// [0, D-1] and the cell is [min(floor p, D-2), +1], so p = D-1 lies in the last
// cell at fraction 1.  `clamped` is true when the position was outside
// [0, D-1] (the sample then does not move with the position).
__device__ __forceinline__ void cell_border(int x, float u, int D, int& i, float& t,
                                            bool& clamped) {
  // selects rather than branches: the same result without divergent control
  // flow in the callers' loops
  const float f = floorf(u);
  const int ii = x + static_cast<int>(f);
  const float tt = u - f;
  const bool lo = ii < 0;
  const bool hi = ii >= D - 1;
  clamped = lo || (hi && (ii > D - 1 || tt > 0.0f));
  i = lo ? 0 : (hi ? D - 2 : ii);
  t = lo ? 0.0f : (hi ? 1.0f : tt);
}

__device__ __forceinline__ float lerp(float a, float b, float t) { return a + t * (b - a); }

// Value and position derivatives of the trilinear interpolant of the 8 cell
// corners c[a][b][c] (a along axis 0, b axis 1, c axis 2), nested along axis
// 2, then 1, then 0 (so that a constant is reproduced exactly).
struct Tri {
  float v, d0, d1, d2;
};

__device__ __forceinline__ Tri tri_eval(const float (&c)[8], float t0, float t1, float t2) {
  // c index = a * 4 + b * 2 + c
  const float c00 = lerp(c[0], c[1], t2);
  const float c01 = lerp(c[2], c[3], t2);
  const float c10 = lerp(c[4], c[5], t2);
  const float c11 = lerp(c[6], c[7], t2);
  const float c0 = lerp(c00, c01, t1);
  const float c1 = lerp(c10, c11, t1);
  Tri r;
  r.v = lerp(c0, c1, t0);
  r.d0 = c1 - c0;
  r.d1 = lerp(c01 - c00, c11 - c10, t0);
  const float e00 = c[1] - c[0];
  const float e01 = c[3] - c[2];
  const float e10 = c[5] - c[4];
  const float e11 = c[7] - c[6];
  r.d2 = lerp(lerp(e00, e01, t1), lerp(e10, e11, t1), t0);
  return r;
}

__device__ __forceinline__ float tri_value(const float (&c)[8], float t0, float t1, float t2) {
  const float c00 = lerp(c[0], c[1], t2);
  const float c01 = lerp(c[2], c[3], t2);
  const float c10 = lerp(c[4], c[5], t2);
  const float c11 = lerp(c[6], c[7], t2);
  return lerp(lerp(c00, c01, t1), lerp(c10, c11, t1), t0);
}

// Two consecutive elements from a 4-byte aligned address (one 8-byte load;
// gfx9 global loads need only dword alignment).
__device__ __forceinline__ float2 ld_pair(const float* __restrict__ p) {
  float2 v;
  __builtin_memcpy(&v, p, sizeof(v));
  return v;
}

// The 8 corners of the cell at (i0, i1, i2) of an image, zero outside.
// Along d2 each corner row is one 8-byte load of the in-range pair
// (jj, jj + 1), jj = clamp(i2, 0, D2 - 2), which holds both corners when
// they are inside (i2 = -1 and i2 = D2 - 1 select its other half); rows and
// planes use clamped (always valid) positions, and masks apply the padding.
__device__ __forceinline__ void corners_zero(const float* __restrict__ img, const Geom& g, int i0,
                                             int i1, int i2, float (&c)[8]) {
  const bool a0 = (i0 >= 0) & (i0 < g.d0), a1 = (i0 + 1 >= 0) & (i0 + 1 < g.d0);
  const bool b0 = (i1 >= 0) & (i1 < g.d1), b1 = (i1 + 1 >= 0) & (i1 + 1 < g.d1);
  const bool e0 = (i2 >= 0) & (i2 < g.d2), e1 = (i2 + 1 >= 0) & (i2 + 1 < g.d2);
  const int j0 = min(max(i0, 0), g.d0 - 1), j0n = min(max(i0 + 1, 0), g.d0 - 1);
  const int j1 = min(max(i1, 0), g.d1 - 1), j1n = min(max(i1 + 1, 0), g.d1 - 1);
  const int jj = min(max(i2, 0), g.d2 - 2);
  const bool s0 = i2 == jj, s1 = i2 + 1 == jj;  // which half holds corner e = 0 / e = 1
  const float2 p00 = ld_pair(img + (j0 * g.d1 + j1) * g.d2 + jj);
  const float2 p01 = ld_pair(img + (j0 * g.d1 + j1n) * g.d2 + jj);
  const float2 p10 = ld_pair(img + (j0n * g.d1 + j1) * g.d2 + jj);
  const float2 p11 = ld_pair(img + (j0n * g.d1 + j1n) * g.d2 + jj);
  c[0] = (a0 & b0 & e0) ? (s0 ? p00.x : p00.y) : 0.0f;
  c[1] = (a0 & b0 & e1) ? (s1 ? p00.x : p00.y) : 0.0f;
  c[2] = (a0 & b1 & e0) ? (s0 ? p01.x : p01.y) : 0.0f;
  c[3] = (a0 & b1 & e1) ? (s1 ? p01.x : p01.y) : 0.0f;
  c[4] = (a1 & b0 & e0) ? (s0 ? p10.x : p10.y) : 0.0f;
  c[5] = (a1 & b0 & e1) ? (s1 ? p10.x : p10.y) : 0.0f;
  c[6] = (a1 & b1 & e0) ? (s0 ? p11.x : p11.y) : 0.0f;
  c[7] = (a1 & b1 & e1) ? (s1 ? p11.x : p11.y) : 0.0f;
}

// Zero-padded trilinear sample of an image at x + u (value and gradient).
__device__ __forceinline__ Tri sample_zero(const float* __restrict__ img, const Geom& g, int x0,
                                           int x1, int x2, float u0, float u1, float u2) {
  int i0, i1, i2;
  float t0, t1, t2;
  cell_zero(x0, sane(u0), i0, t0);
  cell_zero(x1, sane(u1), i1, t1);
  cell_zero(x2, sane(u2), i2, t2);
  float c[8];
  corners_zero(img, g, i0, i1, i2, c);
  return tri_eval(c, t0, t1, t2);
}

__device__ __forceinline__ float sample_zero_value(const float* __restrict__ img, const Geom& g,
                                                   int x0, int x1, int x2, float u0, float u1,
                                                   float u2) {
  int i0, i1, i2;
  float t0, t1, t2;
  cell_zero(x0, sane(u0), i0, t0);
  cell_zero(x1, sane(u1), i1, t1);
  cell_zero(x2, sane(u2), i2, t2);
  float c[8];
  corners_zero(img, g, i0, i1, i2, c);
  return tri_value(c, t0, t1, t2);
}

// Trilinear weight of corner (a, b, e) of a cell at fractions (t0, t1, t2).
// Each further factor (1 - t) is applied as w - w t in one fused
// multiply-add instead of a subtraction and a product; with the corner
// indices constant after unrolling, the selects fold away.
__device__ __forceinline__ float corner_weight(int a, int b, int e, float t0, float t1, float t2) {
  const float w0 = a ? t0 : 1.0f - t0;
  const float w1 = b ? w0 * t1 : fmaf(-w0, t1, w0);
  return e ? w1 * t2 : fmaf(-w1, t2, w1);
}

// Border cell of the position x + u in all three axes.
struct BorderCell {
  int base;        // linear index of corner (0, 0, 0)
  int i0, i1, i2;  // cell index (corner (0, 0, 0)) per axis, i_d in [0, D_d - 2]
  float t0, t1, t2;
  bool k0, k1, k2; // clamped along axis d
};

__device__ __forceinline__ BorderCell border_cell(const Geom& g, int x0, int x1, int x2, float u0,
                                                  float u1, float u2) {
  BorderCell b;
  cell_border(x0, sane(u0), g.d0, b.i0, b.t0, b.k0);
  cell_border(x1, sane(u1), g.d1, b.i1, b.t1, b.k1);
  cell_border(x2, sane(u2), g.d2, b.i2, b.t2, b.k2);
  b.base = (b.i0 * g.d1 + b.i1) * g.d2 + b.i2;
  return b;
}

// Element access at a 32-bit index from a wave-uniform base pointer: volumes
// are capped at 2^29 voxels, so the byte offset of one component fits in 32
// bits and the access needs no per-lane 64-bit address arithmetic.
__device__ __forceinline__ float ld_at(const float* __restrict__ base, uint32_t i) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + (i << 2));
}
__device__ __forceinline__ void st_at(float* __restrict__ base, uint32_t i, float v) {
  *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + (i << 2)) = v;
}

// Stores that a lane may skip without a branch: a raw buffer resource over
// one array of at most 2^31 bytes (one component of a capped volume), and a
// lane that must not write passes a byte offset of 2^31 or more, which the
// buffer range check discards.  Every lane then issues the same store
// instructions, so the in-order memory counter of the wave stays exact at
// later waits.
struct MaskedOut {
  __amdgpu_buffer_rsrc_t r;
};
__device__ __forceinline__ MaskedOut masked_out(float* base, uint32_t count) {
  constexpr int kRawWord3 = 0x00020000;  // untyped 32-bit access (gfx9 family)
  MaskedOut m;
  m.r = __builtin_amdgcn_make_buffer_rsrc(base, 0, static_cast<int>(count << 2), kRawWord3);
  return m;
}
__device__ __forceinline__ void store_masked(const MaskedOut& m, uint32_t i, float v, bool on) {
  const uint32_t off = on ? (i << 2) : 0x80000000u;
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), m.r, off, 0, 0);
}

// The 8 corners of one field component at a border cell (always in range).
__device__ __forceinline__ void corners_border(const float* __restrict__ f, const Geom& g,
                                               int base, float (&c)[8]) {
  const int s0 = g.plane, s1 = g.d2;
  c[0] = f[base];
  c[1] = f[base + 1];
  c[2] = f[base + s1];
  c[3] = f[base + s1 + 1];
  c[4] = f[base + s0];
  c[5] = f[base + s0 + 1];
  c[6] = f[base + s0 + s1];
  c[7] = f[base + s0 + s1 + 1];
}

// ---------------------------------------------------------------------------
// Diffusion regulariser R(u) = (1/3) sum_d mean_{c, x: x_d < D_d - 1}
// (u_c(x + e_d) - u_c(x))^2 of an ncomp-component field (Eq. (2) read on the
// displacement), and its gradient.
struct RegW {
  double w[3];  // 1 / (3 cnt_d), cnt_d = ncomp (D_d - 1) V / D_d
  float g[3];   // lam * 2 * w[d]
  double lam;   // weight of R in the loss
  bool on;      // lam != 0
};

// At voxel x of one component: adds w_d (u(x + e_d) - u(x))^2 over the forward
// neighbours to `racc` and returns lam dR/du(x).
__device__ __forceinline__ float reg_at(const float* __restrict__ f, const Geom& g, int lin, int x0,
                                        int x1, int x2, const RegW& rw, double& racc) {
  const float c = f[lin];
  float grad = 0.0f;
  const int strides[3] = {g.plane, g.d2, 1};
  const int xs[3] = {x0, x1, x2};
  const int ds[3] = {g.d0, g.d1, g.d2};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (xs[d] + 1 < ds[d]) {
      const float df = f[lin + strides[d]] - c;
      racc += rw.w[d] * static_cast<double>(df) * static_cast<double>(df);
      grad -= rw.g[d] * df;
    }
    if (xs[d] > 0) {
      const float db = c - f[lin - strides[d]];
      grad += rw.g[d] * db;
    }
  }
  return grad;
}

// ---------------------------------------------------------------------------
// Reductions: 64-lane wavefronts, then across the waves of the block.
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

// Sum of x over the block; the result is valid in thread 0.  Every thread of
// the block must call it.  `scratch` holds one double per wave.
template <int NT>
__device__ __forceinline__ double block_sum(double x, double* scratch) {
  constexpr int NW = NT / 64;
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) scratch[w] = x;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NW; ++i) r += scratch[i];
  }
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// Host side: kernel classes for timing, launch checks.

enum KernelClass : int {
  KC_EXP_FWD = 0,
  KC_EXP_BWD,
  KC_WARP,
  KC_WARP_BWD,
  KC_MSE,
  KC_LNCC_FWD,
  KC_LNCC_BWD,
  KC_GAUSS,
  KC_DIFFUSION,
  KC_ADAM,
  KC_CENTER,
  KC_ATLAS,
  KC_FILL,
  KC_MISC,
  KC_ITER,
  KC_NUM
};

void prof_begin(hipStream_t s, int cls);
void prof_end(hipStream_t s, int cls);

// Grid of `total` blocks of the 1-D voxel kernels (one thread per voxel).
inline uint32_t blocks_for(long long items, int per_block) {
  return static_cast<uint32_t>((items + per_block - 1) / per_block);
}

}  // namespace darc
