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
// One wave computes MT 16-voxel row tiles x (16 * NT16) channels with
// v_mfma_f32_16x16x32_bf16: per 32-wide K step, lane l supplies the A row
// l % 16 (its voxel of each row tile) and B column l % 16 at K entries
// 8 (l / 16) .. + 7 (loaded once and used by every row tile), and holds
// output rows 4 (l / 16) .. + 3 of column l % 16.  FP32 accumulation;
// bias, leaky ReLU and the BF16 rounding (to nearest even) in the epilogue.
#include <type_traits>

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

__device__ __forceinline__ float from_bf16(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

// One channels-last FP32 output element (ConvGeom: split channels, the skip
// channels of a pooled split, or the
// next layer's activation adjoint fused into a BF16 output).
__device__ __forceinline__ void store_cl32(const ConvGeom& cg, float* __restrict__ y32,
                                           long long mo, int co, float val) {
  if (cg.dz16 && !cg.hpool) {
    const long long i = mo * cg.cout + co;
    float tot = cg.accum ? y32[i] + val : val;
    if (!(from_bf16(cg.acty[i]) > 0.0f)) tot *= cg.slope;
    cg.dz16[i] = to_bf16(tot);
    return;
  }
  float* d = cg.csplit == 0 ? y32 + mo * cg.cout + co
             : co < cg.csplit ? y32 + mo * cg.csplit + co
                              : cg.y32b + mo * (cg.cout - cg.csplit) + (co - cg.csplit);
  *d = cg.accum ? *d + val : val;
}

// X0: how x0 is read (0: full resolution; 1: half resolution, nearest
// upsampled; 2: half resolution, zero-dilated), fixed per launch.
template <int NT16, int MT, int X0>
__global__ __launch_bounds__(CNT) void k_conv3d(const uint16_t* __restrict__ x0,
                                                const uint16_t* __restrict__ x1,
                                                const uint16_t* __restrict__ w,
                                                const float* __restrict__ bias,
                                                uint16_t* __restrict__ y16,
                                                float* __restrict__ y32, ConvGeom cg) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kg = lane >> 4;
  // this wave's MT consecutive 16-voxel row tiles
  const long long mbase = static_cast<long long>(blockIdx.x) * CROWS * MT + wave * 16 * MT;
  const long long ov = static_cast<long long>(cg.o0) * cg.o1 * cg.o2;
  constexpr bool half = X0 != 0;  // x0 is stored at half resolution
  const int h0 = half ? cg.i0 / 2 : cg.i0, h1 = half ? cg.i1 / 2 : cg.i1;
  const int h2 = half ? cg.i2 / 2 : cg.i2;
  // per row tile: this lane's voxel as input position of tap (0, 0, 0)
  // (output position * stride - 1), the subject's base pointers, and the
  // x1 voxel offset of that position within the subject
  int q0[MT], q1[MT], q2[MT], lb1[MT];
  const uint16_t* t0[MT];
  const uint16_t* t1[MT];
  bool mv[MT];
  const long long vin0 = static_cast<long long>(h0) * h1 * h2;
  const long long vin1 = static_cast<long long>(cg.i0) * cg.i1 * cg.i2;
#pragma unroll
  for (int q = 0; q < MT; ++q) {
    const long long m = mbase + q * 16 + r;
    mv[q] = m < cg.nvox;
    int ss = 0, a0 = 0, a1 = 0, a2 = 0;
    if (mv[q]) {
      ss = static_cast<int>(m / ov);
      int rem = static_cast<int>(m - static_cast<long long>(ss) * ov);
      a2 = rem % cg.o2;
      rem /= cg.o2;
      a1 = rem % cg.o1;
      a0 = rem / cg.o1;
    }
    q0[q] = a0 * cg.stride - 1;
    q1[q] = a1 * cg.stride - 1;
    q2[q] = a2 * cg.stride - 1;
    lb1[q] = (q0[q] * cg.i1 + q1[q]) * cg.i2 + q2[q];
    t0[q] = x0 + ss * vin0 * cg.c0;
    t1[q] = x1 + ss * vin1 * cg.c1 - cg.c0;  // x1 channels follow the c0 of x0
  }
  const int nco0 = blockIdx.y * 16 * NT16;
  f32x4 acc[MT][NT16];
#pragma unroll
  for (int q = 0; q < MT; ++q)
#pragma unroll
    for (int t = 0; t < NT16; ++t) acc[q][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const int cvec = (cg.c0 + cg.c1) >> 3;
  // this lane's 8-wide K group: tap and channel group, advanced by 4 groups
  // per K step without divisions; (ta, tb, tc) is the tap's offset + 1
  int tap = kg / cvec, v = kg - tap * cvec;
  int ta = 1, tb = 1, tc = 1;
  if (cg.ntaps == 27) {
    ta = tap / 9;
    tb = (tap / 3) % 3;
    tc = tap % 3;
  }
  for (int kc = 0; kc < cg.kpad; kc += 32) {
    // B fragments (weights) of this K step, shared by the wave's row tiles
    bf16x8 bfrag[NT16];
#pragma unroll
    for (int t = 0; t < NT16; ++t) {
      const int co = nco0 + t * 16 + r;
      uint4 braw = make_uint4(0u, 0u, 0u, 0u);
      if (co < cg.cout)
        braw = *reinterpret_cast<const uint4*>(w + static_cast<long long>(co) * cg.kpad + kc + kg * 8);
      bfrag[t] = __builtin_bit_cast(bf16x8, braw);
    }
    // A fragments: 8 channels of this lane's tap at its voxel of each tile.
    // Every load is issued (from x0 itself where the input is zero) before
    // the products; the zero padding is applied to the loaded values.
    const int ch = v * 8;
    const bool from0 = ch < cg.c0;
    const bool tap_ok = tap < cg.ntaps;
    const int toff1 = (ta * cg.i1 + tb) * cg.i2 + tc;
    uint4 araw[MT];
    bool in[MT];
#pragma unroll
    for (int q = 0; q < MT; ++q) {
      const int p0 = q0[q] + ta, p1 = q1[q] + tb, p2 = q2[q] + tc;
      bool ok = tap_ok && mv[q] && static_cast<unsigned>(p0) < static_cast<unsigned>(cg.i0) &&
                static_cast<unsigned>(p1) < static_cast<unsigned>(cg.i1) &&
                static_cast<unsigned>(p2) < static_cast<unsigned>(cg.i2);
      const uint16_t* src;
      if (!half) {
        // both inputs at full resolution: same voxel offset, own base and stride
        src = (from0 ? t0[q] : t1[q]) +
              static_cast<long long>(lb1[q] + toff1) * (from0 ? cg.c0 : cg.c1) + ch;
      } else if (from0) {
        if (X0 == 2) ok = ok && !((p0 | p1 | p2) & 1);
        src = t0[q] + static_cast<long long>(((p0 >> 1) * h1 + (p1 >> 1)) * h2 + (p2 >> 1)) * cg.c0 +
              ch;
      } else {
        src = t1[q] + static_cast<long long>(lb1[q] + toff1) * cg.c1 + ch;
      }
      in[q] = ok;
      araw[q] = *reinterpret_cast<const uint4*>(ok ? src : x0);
    }
#pragma unroll
    for (int q = 0; q < MT; ++q) {
      const uint4 z = make_uint4(0u, 0u, 0u, 0u);
      const bf16x8 afrag = __builtin_bit_cast(bf16x8, in[q] ? araw[q] : z);
#pragma unroll
      for (int t = 0; t < NT16; ++t)
        acc[q][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag, bfrag[t], acc[q][t], 0, 0, 0);
    }
    // next K step: 4 groups further
    v += 4;
    while (v >= cvec) {
      v -= cvec;
      ++tap;
      if (cg.ntaps == 27 && ++tc == 3) {
        tc = 0;
        if (++tb == 3) {
          tb = 0;
          ++ta;
        }
      }
    }
  }
  // epilogue: lane holds rows 4 kg .. 4 kg + 3 of column r of each N sub-tile
#pragma unroll
  for (int t = 0; t < NT16; ++t) {
    const int co = nco0 + t * 16 + r;
    if (co >= cg.cout) continue;
    const float bb = bias ? bias[co] : 0.0f;
#pragma unroll
    for (int q = 0; q < MT; ++q) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long long mo = mbase + q * 16 + kg * 4 + i;
        if (mo >= cg.nvox) continue;
        float val = acc[q][t][i] + bb;
        if (cg.act) val = val > 0.0f ? val : cg.slope * val;
        if (y16) {
          y16[mo * cg.cout + co] = to_bf16(val);
        } else if (cg.ycl32) {
          store_cl32(cg, y32, mo, co, val);
        } else {
          const long long so = mo / ov;
          y32[(so * cg.cout + co) * ov + (mo - so * ov)] = val;
        }
      }
    }
  }
}

// Stride-1 3x3x3 convolutions with the input staged in LDS.
//
// A block computes a brick of 4 (d0, one plane per wave) x MT (d1, the
// wave's row tiles) x 16 (d2, the rows of an MFMA tile) output voxels for
// 16 NT16 output channels.  Its input brick with the one-voxel halo,
// 6 x (MT + 2) x 18 voxels, is staged in LDS in chunks of CG channel groups
// (8 channels each): every input value is fetched from memory once per
// block instead of once per tap, and the 27 taps read their A fragments from
// LDS.  A voxel's CG groups sit at a stride of an odd number of 16-byte
// units, so the 8 lanes of a 16-byte LDS read phase (consecutive d2) hit
// distinct banks.  Within a chunk the reduction runs over (tap, group)
// pairs, four per 32-wide K step (one per 16-lane group), with the weights
// read at their place in the [cout][kpad] layout.
//
// The index arithmetic is hoisted out of the loops: each thread decodes its
// staging units (input voxel, inside flags) once and reuses them for every
// chunk, whose loads it issues one chunk ahead, and a table in LDS gives each (K step, lane group) its A byte
// offset and weight offset (the row tiles add compile-time immediates).
// The pairs past a chunk's 27 CG read their own tap-0 input with zero
// weights.  X0 selects how x0 is read, as in k_conv3d.
constexpr int LBZ = CWAVES;  // output planes per block (one per wave)
constexpr int LBX = 16;      // output voxels per MFMA row tile (d2)

template <int MT>
struct LdsBrick {
  static constexpr int NY = MT + 2, NX = LBX + 2;
  static constexpr int NVOX = (LBZ + 2) * NY * NX;
};

template <int NT16, int MT, int X0, int CG>
__global__ __launch_bounds__(CNT) void k_conv3d_lds(const uint16_t* __restrict__ x0,
                                                    const uint16_t* __restrict__ x1,
                                                    const uint16_t* __restrict__ w,
                                                    const float* __restrict__ bias,
                                                    uint16_t* __restrict__ y16,
                                                    float* __restrict__ y32, ConvGeom cg,
                                                    int nbz, int nby, int nbx) {
  using B = LdsBrick<MT>;
  constexpr int SU = CG % 2 ? CG : CG + 1;  // voxel stride in 16-byte units (odd)
  constexpr int NPAIR = 27 * CG;
  constexpr int NSTEP = (NPAIR + 3) / 4;
  constexpr int NUNIT = B::NVOX * CG;          // 16-byte units staged per chunk
  constexpr int NU = (NUNIT + CNT - 1) / CNT;  // per thread
  static_assert(CNT % CG == 0, "a thread's staging units share one channel group");
  static_assert(NU <= 16, "staging flags fit one word");
  __shared__ uint4 brick[B::NVOX * SU];
  __shared__ int2 ktab[NSTEP * 4];  // (A byte offset at row tile 0, weight offset) per pair
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kg = lane >> 4;
  // block -> (subject, brick); consecutive bricks of a subject share an XCD
  const long long per = static_cast<long long>(cg.o0) * cg.o1 * cg.o2;
  const uint32_t nblk = static_cast<uint32_t>(static_cast<long long>(nbz) * nby * nbx * (cg.nvox / per));
  uint32_t b = xcd_remap(blockIdx.x, nblk);
  const int bx = static_cast<int>(b % nbx);
  b /= nbx;
  const int by = static_cast<int>(b % nby);
  b /= nby;
  const int bz = static_cast<int>(b % nbz);
  const int s = static_cast<int>(b / nbz);
  const int oz = bz * LBZ, oy = by * MT, ox = bx * LBX;
  constexpr bool half = X0 != 0;  // x0 is stored at half resolution
  const int h1 = half ? cg.i1 / 2 : cg.i1, h2 = half ? cg.i2 / 2 : cg.i2;
  const long long vin0 = static_cast<long long>(half ? cg.i0 / 2 : cg.i0) * h1 * h2;
  const long long vin1 = static_cast<long long>(cg.i0) * cg.i1 * cg.i2;
  const uint16_t* sx0 = x0 + s * vin0 * cg.c0;
  const uint16_t* sx1 = x1 ? x1 + s * vin1 * cg.c1 - cg.c0 : nullptr;  // x1 channels follow c0
  const int cvec = (cg.c0 + cg.c1) >> 3;
  const int nco0 = blockIdx.y * 16 * NT16;

  // the K-step table: pair q = 4 st + lane group, tap q / CG, group q % CG
  if (threadIdx.x < NSTEP * 4) {
    const int q = threadIdx.x;
    const int tap = q < NPAIR ? q / CG : 0, g = q % CG;
    const int toff = ((tap / 9) * B::NY + (tap / 3) % 3) * B::NX + tap % 3;
    ktab[q] = make_int2(toff * SU * 16 + g * 16, q < NPAIR ? (tap * cvec + g) * 8 : -1);
  }
  // staging units of this thread: input voxel (full and, for x0 at half
  // resolution, half resolution); bit j of ubits: unit j inside the volume,
  // bit 16 + j: on the even grid (zero-dilated x0)
  const int sg = threadIdx.x % CG;  // its channel group within a chunk
  int uvf[NU], uvh[NU];
  unsigned ubits = 0u;
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    const int i = threadIdx.x + j * CNT;
    const int vb = (i < NUNIT ? i : 0) / CG;
    const int ex = vb % B::NX, rest = vb / B::NX;
    const int ey = rest % B::NY, ez = rest / B::NY;
    const int p0 = oz - 1 + ez, p1 = oy - 1 + ey, p2 = ox - 1 + ex;
    const bool in = i < NUNIT && static_cast<unsigned>(p0) < static_cast<unsigned>(cg.i0) &&
                    static_cast<unsigned>(p1) < static_cast<unsigned>(cg.i1) &&
                    static_cast<unsigned>(p2) < static_cast<unsigned>(cg.i2);
    uvf[j] = in ? (p0 * cg.i1 + p1) * cg.i2 + p2 : 0;
    uvh[j] = in ? ((p0 >> 1) * h1 + (p1 >> 1)) * h2 + (p2 >> 1) : 0;
    ubits |= (in ? 1u : 0u) << j;
    ubits |= (X0 != 2 || !((p0 | p1 | p2) & 1) ? 1u : 0u) << (16 + j);
  }
  // brick slot of unit j: (threadIdx.x + j CNT) / CG voxels in, group sg
  const int slot0 = (threadIdx.x / CG) * SU + sg;
  constexpr int SLOTJ = (CNT / CG) * SU;

  f32x4 acc[MT][NT16];
#pragma unroll
  for (int q = 0; q < MT; ++q)
#pragma unroll
    for (int t = 0; t < NT16; ++t) acc[q][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  // this lane's A fragment of tap (0, 0, 0), row tile 0
  const char* abase = reinterpret_cast<const char*>(brick) + ((wave * B::NY) * B::NX + r) * SU * 16;
  const uint16_t* wrow[NT16];
  bool cok[NT16];
#pragma unroll
  for (int t = 0; t < NT16; ++t) {
    const int co = nco0 + t * 16 + r;
    cok[t] = co < cg.cout;
    wrow[t] = w + static_cast<long long>(cok[t] ? co : 0) * cg.kpad;
  }

  // staging loads of one chunk into registers (units past the brick and
  // outside the volume give zeros)
  const bool lastu = NU * CNT > NUNIT && threadIdx.x + (NU - 1) * CNT >= NUNIT;
  uint4 pre[NU];
  auto load_chunk = [&](int cb) {
    const int ch = (cb + sg) * 8;
    const bool from0 = ch < cg.c0;
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      const uint16_t* src = from0 ? sx0 + static_cast<long long>(half ? uvh[j] : uvf[j]) * cg.c0 + ch
                                  : sx1 + static_cast<long long>(uvf[j]) * cg.c1 + ch;
      pre[j] = make_uint4(0u, 0u, 0u, 0u);
      if (((ubits >> j) & 1u) && (!from0 || ((ubits >> (16 + j)) & 1u)))
        pre[j] = *reinterpret_cast<const uint4*>(src);
    }
  };
  load_chunk(0);
  for (int cb = 0; cb < cvec; cb += CG) {
    // stage channel groups cb .. cb + CG - 1 of the input brick, then load
    // the next chunk's while this one is multiplied
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      if (j == NU - 1 && lastu) break;
      brick[slot0 + j * SLOTJ] = pre[j];
    }
    __syncthreads();
    if (cb + CG < cvec) load_chunk(cb + CG);
#pragma unroll 2
    for (int st = 0; st < NSTEP; ++st) {
      const int2 kt = ktab[4 * st + kg];
      bf16x8 bfrag[NT16];
#pragma unroll
      for (int t = 0; t < NT16; ++t) {
        uint4 braw = make_uint4(0u, 0u, 0u, 0u);
        if (cok[t] && kt.y >= 0) braw = *reinterpret_cast<const uint4*>(wrow[t] + cb * 8 + kt.y);
        bfrag[t] = __builtin_bit_cast(bf16x8, braw);
      }
      const char* ap = abase + kt.x;
#pragma unroll
      for (int q2 = 0; q2 < MT; ++q2) {
        // row tile q2 is B::NX voxels further: an immediate offset
        const uint4 araw = *reinterpret_cast<const uint4*>(ap + q2 * B::NX * SU * 16);
        const bf16x8 afrag = __builtin_bit_cast(bf16x8, araw);
#pragma unroll
        for (int t = 0; t < NT16; ++t)
          acc[q2][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag, bfrag[t], acc[q2][t], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // epilogue: lane holds d2 offsets 4 kg .. 4 kg + 3 of channel column r
  const int z = oz + wave;
  constexpr bool kVecOut = NT16 <= 2 && CWAVES * MT * 16 * 16 * sizeof(float) <= sizeof(brick);
  if (kVecOut && y16 && cg.cout % 8 == 0) {
    // BF16 outputs through the LDS brick (free since the loop's last
    // barrier), one column tile at a time: each wave writes its MT x 16
    // voxels x 16 channels as FP32 (bias and activation applied), then each
    // lane converts 8 channels of one voxel and stores them with one 16-byte
    // write
    float* tb = reinterpret_cast<float*>(brick) + wave * (MT * 16 * 16);
#pragma unroll
    for (int t = 0; t < NT16; ++t) {
      const int co = nco0 + t * 16 + r;
      const float bb = bias && co < cg.cout ? bias[co] : 0.0f;
#pragma unroll
      for (int q2 = 0; q2 < MT; ++q2)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float val = acc[q2][t][i] + bb;
          if (cg.act) val = val > 0.0f ? val : cg.slope * val;
          tb[(q2 * 16 + 4 * kg + i) * 16 + r] = val;
        }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < MT / 2; ++k) {
        const int c = lane + 64 * k;  // voxel c / 2 of the wave, channels 8 (c % 2) ..
        const int v = c >> 1, hh = c & 1;
        const int y = oy + v / 16, x = ox + v % 16, co8 = nco0 + t * 16 + 8 * hh;
        if (z < cg.o0 && y < cg.o1 && x < cg.o2 && co8 < cg.cout) {
          const float4 lo = *reinterpret_cast<const float4*>(tb + v * 16 + 8 * hh);
          const float4 hi = *reinterpret_cast<const float4*>(tb + v * 16 + 8 * hh + 4);
          const uint4 pk = make_uint4(
              static_cast<uint32_t>(to_bf16(lo.x)) | (static_cast<uint32_t>(to_bf16(lo.y)) << 16),
              static_cast<uint32_t>(to_bf16(lo.z)) | (static_cast<uint32_t>(to_bf16(lo.w)) << 16),
              static_cast<uint32_t>(to_bf16(hi.x)) | (static_cast<uint32_t>(to_bf16(hi.y)) << 16),
              static_cast<uint32_t>(to_bf16(hi.z)) | (static_cast<uint32_t>(to_bf16(hi.w)) << 16));
          const long long mo = s * per + (static_cast<long long>(z) * cg.o1 + y) * cg.o2 + x;
          *reinterpret_cast<uint4*>(y16 + mo * cg.cout + co8) = pk;
        }
      }
      __syncthreads();
    }
    return;
  }
  // rows of a wave's column tile that fit the brick at once as FP32
  constexpr int kRP = static_cast<int>(sizeof(brick) / (CWAVES * 16 * 16 * sizeof(float))) >= MT
                          ? MT
                          : (sizeof(brick) >= CWAVES * 2 * 16 * 16 * sizeof(float) ? 2 : 0);
  if (NT16 <= 2 && kRP > 0 && !y16 && cg.ycl32 && cg.dz16 && !cg.hpool && cg.csplit == 0 &&
      cg.cout % 8 == 0) {
    // the fused BF16 output gradient (the output layer's input gradient)
    // through the LDS brick, kRP rows of one column tile at a time: each lane
    // takes 8 channels of one voxel with 16-byte accesses (the FP32 sum it
    // adds to, the activation it differentiates, the BF16 result)
    float* tb = reinterpret_cast<float*>(brick) + wave * (kRP * 16 * 16);
#pragma unroll
    for (int t = 0; t < NT16; ++t) {
#pragma unroll
      for (int qb = 0; qb < MT; qb += kRP) {
#pragma unroll
        for (int q2 = 0; q2 < kRP; ++q2)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float val = acc[qb + q2][t][i];
            if (cg.act) val = val > 0.0f ? val : cg.slope * val;
            tb[(q2 * 16 + 4 * kg + i) * 16 + r] = val;
          }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kRP / 2; ++k) {
          const int c = lane + 64 * k;  // voxel c / 2 of the rows, channels 8 (c % 2) ..
          const int v = c >> 1, hh = c & 1;
          const int y = oy + qb + v / 16, x = ox + v % 16, co8 = nco0 + t * 16 + 8 * hh;
          if (z < cg.o0 && y < cg.o1 && x < cg.o2 && co8 < cg.cout) {
            const long long i0 =
                (s * per + (static_cast<long long>(z) * cg.o1 + y) * cg.o2 + x) * cg.cout + co8;
            const float4 lo = *reinterpret_cast<const float4*>(tb + v * 16 + 8 * hh);
            const float4 hi = *reinterpret_cast<const float4*>(tb + v * 16 + 8 * hh + 4);
            float tv[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
            if (cg.accum) {
              const float4 a0 = *reinterpret_cast<const float4*>(y32 + i0);
              const float4 a1 = *reinterpret_cast<const float4*>(y32 + i0 + 4);
              const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
              for (int j = 0; j < 8; ++j) tv[j] = av[j] + tv[j];
            }
            const uint4 ay = *reinterpret_cast<const uint4*>(cg.acty + i0);
            const uint32_t aw[4] = {ay.x, ay.y, ay.z, ay.w};
            uint32_t ow[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              float e0 = tv[2 * j], e1 = tv[2 * j + 1];
              if (!(__uint_as_float(aw[j] << 16) > 0.0f)) e0 *= cg.slope;
              if (!(__uint_as_float(aw[j] & 0xFFFF0000u) > 0.0f)) e1 *= cg.slope;
              ow[j] = static_cast<uint32_t>(to_bf16(e0)) | (static_cast<uint32_t>(to_bf16(e1)) << 16);
            }
            *reinterpret_cast<uint4*>(cg.dz16 + i0) = make_uint4(ow[0], ow[1], ow[2], ow[3]);
          }
        }
        __syncthreads();
      }
    }
    return;
  }
  if (cg.hpool) {
    // channels below csplit to half resolution: the lane's 2 (d1) x 2 (d2)
    // children of each pair of its row tiles and d2 offsets summed in
    // registers, then the odd wave's sums (plane z + 1) passed to the even
    // wave through the LDS brick, free since the loop's last barrier; the
    // brick origin is even on every axis, so no pair spans two blocks
    static_assert(2 * NT16 * MT * 64 * sizeof(float) <= sizeof(brick), "pair sums fit the brick");
    static_assert(MT % 2 == 0 && LBZ % 2 == 0, "row tiles and planes pair up");
    float hp[NT16][MT / 2][2];
#pragma unroll
    for (int t = 0; t < NT16; ++t)
#pragma unroll
      for (int yp = 0; yp < MT / 2; ++yp)
#pragma unroll
        for (int xp = 0; xp < 2; ++xp)
          hp[t][yp][xp] = (acc[2 * yp][t][2 * xp] + acc[2 * yp][t][2 * xp + 1]) +
                          (acc[2 * yp + 1][t][2 * xp] + acc[2 * yp + 1][t][2 * xp + 1]);
    float* xch = reinterpret_cast<float*>(brick) + (wave >> 1) * (NT16 * MT * 64);
    if (wave & 1) {
#pragma unroll
      for (int t = 0; t < NT16; ++t)
#pragma unroll
        for (int j = 0; j < MT; ++j) xch[(t * MT + j) * 64 + lane] = hp[t][j >> 1][j & 1];
    }
    __syncthreads();
    if (!(wave & 1) && z < cg.o0) {
      const int H0 = cg.o0 / 2, H1 = cg.o1 / 2, H2 = cg.o2 / 2;
#pragma unroll
      for (int t = 0; t < NT16; ++t) {
        const int co = nco0 + t * 16 + r;
        if (co >= cg.csplit) continue;
#pragma unroll
        for (int j = 0; j < MT; ++j) {
          const int y = oy + 2 * (j >> 1), x = ox + 4 * kg + 2 * (j & 1);
          if (y >= cg.o1 || x >= cg.o2) continue;
          const long long q = ((static_cast<long long>(s) * H0 + (z >> 1)) * H1 + (y >> 1)) * H2 + (x >> 1);
          float tot = hp[t][j >> 1][j & 1] + xch[(t * MT + j) * 64 + lane];
          if (!(from_bf16(cg.acty[q * cg.csplit + co]) > 0.0f)) tot *= cg.slope;
          cg.dz16[q * cg.csplit + co] = to_bf16(tot);
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT16; ++t) {
    const int co = nco0 + t * 16 + r;
    if (co >= cg.cout || (cg.hpool && co < cg.csplit)) continue;
    const float bb = bias ? bias[co] : 0.0f;
#pragma unroll
    for (int q2 = 0; q2 < MT; ++q2) {
      const int y = oy + q2;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int x = ox + 4 * kg + i;
        if (z >= cg.o0 || y >= cg.o1 || x >= cg.o2) continue;
        const long long vo = (static_cast<long long>(z) * cg.o1 + y) * cg.o2 + x;
        const long long mo = s * per + vo;
        float val = acc[q2][t][i] + bb;
        if (cg.act) val = val > 0.0f ? val : cg.slope * val;
        if (y16) {
          y16[mo * cg.cout + co] = to_bf16(val);
        } else if (cg.ycl32) {
          store_cl32(cg, y32, mo, co, val);
        } else {
          y32[(s * cg.cout + co) * per + vo] = val;
        }
      }
    }
  }
}

// Input gradients of the stride-2 layers: a stride-1 convolution over dz
// placed on the even positions of the full grid, zeros between.  Split by
// the parity of the output voxel p = 2q + par: along an axis with par 0 only
// the centre tap meets an even position (dz at q), with par 1 the two outer
// taps (dz at q and q + 1).  A block owns one parity class and a brick of
// 4 x MT x 16 half-resolution positions q; it stages the 5 x (MT + 1) x 17
// voxels of dz those outputs read (no zeros) and reduces over the class's
// 1 to 8 valid taps only, an eighth of the products on average.
template <int NT16, int MT, int CG>
__global__ __launch_bounds__(CNT) void k_conv3d_sub(const uint16_t* __restrict__ dz,
                                                    const uint16_t* __restrict__ w,
                                                    uint16_t* __restrict__ y16,
                                                    float* __restrict__ y32, ConvGeom cg,
                                                    int nbz, int nby, int nbx) {
  constexpr int NY = MT + 1, NX = LBX + 1;
  constexpr int NVOX = (LBZ + 1) * NY * NX;
  constexpr int SU = CG % 2 ? CG : CG + 1;  // voxel stride in 16-byte units (odd)
  constexpr int MAXQ = 8 * CG;             // pairs of the largest class
  constexpr int NUNIT = NVOX * CG;
  constexpr int NU = (NUNIT + CNT - 1) / CNT;
  static_assert(CNT % CG == 0, "a thread's staging units share one channel group");
  __shared__ uint4 brick[NVOX * SU];
  __shared__ int2 ktab[MAXQ + 3];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kg = lane >> 4;
  const int h0 = cg.i0 / 2, h1 = cg.i1 / 2, h2 = cg.i2 / 2;  // dz grid (even dims)
  const long long hv = static_cast<long long>(h0) * h1 * h2;
  const long long per = static_cast<long long>(cg.o0) * cg.o1 * cg.o2;
  const long long nsub = cg.nvox / per;
  const uint32_t nblk = static_cast<uint32_t>(8LL * nbz * nby * nbx * nsub);
  // the eight parity classes of a brick are neighbouring blocks (one XCD)
  uint32_t b = xcd_remap(blockIdx.x, nblk);
  const int par = static_cast<int>(b % 8);
  b /= 8;
  const int bx = static_cast<int>(b % nbx);
  b /= nbx;
  const int by = static_cast<int>(b % nby);
  b /= nby;
  const int bz = static_cast<int>(b % nbz);
  const int s = static_cast<int>(b / nbz);
  const int pz = par >> 2, py = (par >> 1) & 1, px = par & 1;
  const int oz = bz * LBZ, oy = by * MT, ox = bx * LBX;  // half-resolution origin
  const uint16_t* sdz = dz + s * hv * cg.c0;
  const int cvec = cg.c0 >> 3;
  const int nco0 = blockIdx.y * 16 * NT16;
  // valid taps of this class: per axis 1 (par 0: tap 1, dz at q) or 2
  // (par 1: taps 0 and 2, dz at q and q + 1)
  const int n0 = 1 + pz, n1 = 1 + py, n2 = 1 + px;
  const int ntap = n0 * n1 * n2;
  const int npair = ntap * CG, nstep = (npair + 3) / 4;
  if (static_cast<int>(threadIdx.x) < 4 * nstep) {
    const int q = threadIdx.x;
    int2 e = make_int2(0, -1);  // past the class's pairs: weight 0
    if (q < npair) {
      const int t = q / CG, g = q - t * CG;
      const int t2 = t % n2, t1 = (t / n2) % n1, t0 = t / (n2 * n1);
      // tap index per axis and its dz offset
      const int a = pz ? 2 * t0 : 1, bb = py ? 2 * t1 : 1, c = px ? 2 * t2 : 1;
      const int s0 = pz ? t0 : 0, s1 = py ? t1 : 0, s2 = px ? t2 : 0;
      e = make_int2((((s0 * NY + s1) * NX + s2) * SU + g) * 16, (((a * 3 + bb) * 3 + c) * cvec + g) * 8);
    }
    ktab[q] = e;
  }
  // staging units: dz voxel (half resolution) and whether it exists
  const int sg = threadIdx.x % CG;
  int uv[NU];
  unsigned ubits = 0u;
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    const int i = threadIdx.x + j * CNT;
    const int vb = (i < NUNIT ? i : 0) / CG;
    const int ex = vb % NX, rest = vb / NX;
    const int ey = rest % NY, ez = rest / NY;
    const int q0 = oz + ez, q1 = oy + ey, q2 = ox + ex;
    const bool in = i < NUNIT && q0 < h0 && q1 < h1 && q2 < h2;
    uv[j] = in ? (q0 * h1 + q1) * h2 + q2 : 0;
    ubits |= (in ? 1u : 0u) << j;
  }
  const int slot0 = (threadIdx.x / CG) * SU + sg;
  constexpr int SLOTJ = (CNT / CG) * SU;
  const bool lastu = NU * CNT > NUNIT && threadIdx.x + (NU - 1) * CNT >= NUNIT;

  f32x4 acc[MT][NT16];
#pragma unroll
  for (int q = 0; q < MT; ++q)
#pragma unroll
    for (int t = 0; t < NT16; ++t) acc[q][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const char* abase = reinterpret_cast<const char*>(brick) + ((wave * NY) * NX + r) * SU * 16;
  const uint16_t* wrow[NT16];
  bool cok[NT16];
#pragma unroll
  for (int t = 0; t < NT16; ++t) {
    const int co = nco0 + t * 16 + r;
    cok[t] = co < cg.cout;
    wrow[t] = w + static_cast<long long>(cok[t] ? co : 0) * cg.kpad;
  }
  uint4 pre[NU];
  auto load_chunk = [&](int cb) {
    const int ch = (cb + sg) * 8;
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      pre[j] = make_uint4(0u, 0u, 0u, 0u);
      if ((ubits >> j) & 1u)
        pre[j] = *reinterpret_cast<const uint4*>(sdz + static_cast<long long>(uv[j]) * cg.c0 + ch);
    }
  };
  load_chunk(0);
  for (int cb = 0; cb < cvec; cb += CG) {
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      if (j == NU - 1 && lastu) break;
      brick[slot0 + j * SLOTJ] = pre[j];
    }
    __syncthreads();
    if (cb + CG < cvec) load_chunk(cb + CG);
    for (int st = 0; st < nstep; ++st) {
      const int2 kt = ktab[4 * st + kg];
      bf16x8 bfrag[NT16];
#pragma unroll
      for (int t = 0; t < NT16; ++t) {
        uint4 braw = make_uint4(0u, 0u, 0u, 0u);
        if (cok[t] && kt.y >= 0) braw = *reinterpret_cast<const uint4*>(wrow[t] + cb * 8 + kt.y);
        bfrag[t] = __builtin_bit_cast(bf16x8, braw);
      }
      const char* ap = abase + kt.x;
#pragma unroll
      for (int q2 = 0; q2 < MT; ++q2) {
        const uint4 araw = *reinterpret_cast<const uint4*>(ap + q2 * NX * SU * 16);
        const bf16x8 afrag = __builtin_bit_cast(bf16x8, araw);
#pragma unroll
        for (int t = 0; t < NT16; ++t)
          acc[q2][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag, bfrag[t], acc[q2][t], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // epilogue: lane holds half-resolution d2 offsets 4 kg .. 4 kg + 3 of
  // channel column r; output voxel p = 2 q + par
  const int qz = oz + wave;
  constexpr bool kVecOut = CWAVES * MT * 16 * 16 * sizeof(float) <= sizeof(brick);
  if (kVecOut && !y16 && cg.ycl32 && cg.dz16 && !cg.hpool && cg.csplit == 0 &&
      cg.cout % 8 == 0) {
    // the fused BF16 output gradient through the LDS brick (free since the
    // loop's last barrier), one column tile at a time: each wave writes its
    // MT x 16 positions x 16 channels as FP32, then each lane takes 8
    // channels of one output voxel with 16-byte accesses (the FP32 sum it
    // adds to, the activation it differentiates, the BF16 result)
    float* tb = reinterpret_cast<float*>(brick) + wave * (MT * 16 * 16);
#pragma unroll
    for (int t = 0; t < NT16; ++t) {
#pragma unroll
      for (int q2 = 0; q2 < MT; ++q2)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float val = acc[q2][t][i];
          if (cg.act) val = val > 0.0f ? val : cg.slope * val;
          tb[(q2 * 16 + 4 * kg + i) * 16 + r] = val;
        }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < MT / 2; ++k) {
        const int c = lane + 64 * k;  // position c / 2 of the wave, channels 8 (c % 2) ..
        const int v = c >> 1, hh = c & 1;
        const int qy = oy + v / 16, qx = ox + v % 16, co8 = nco0 + t * 16 + 8 * hh;
        if (qz < h0 && qy < h1 && qx < h2 && co8 < cg.cout) {
          const long long vo =
              (static_cast<long long>(2 * qz + pz) * cg.o1 + 2 * qy + py) * cg.o2 + 2 * qx + px;
          const long long i0 = (s * per + vo) * cg.cout + co8;
          const float4 lo = *reinterpret_cast<const float4*>(tb + v * 16 + 8 * hh);
          const float4 hi = *reinterpret_cast<const float4*>(tb + v * 16 + 8 * hh + 4);
          float tv[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
          if (cg.accum) {
            const float4 a0 = *reinterpret_cast<const float4*>(y32 + i0);
            const float4 a1 = *reinterpret_cast<const float4*>(y32 + i0 + 4);
            const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) tv[j] = av[j] + tv[j];
          }
          const uint4 ay = *reinterpret_cast<const uint4*>(cg.acty + i0);
          const uint32_t aw[4] = {ay.x, ay.y, ay.z, ay.w};
          uint32_t ow[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            float e0 = tv[2 * j], e1 = tv[2 * j + 1];
            if (!(__uint_as_float(aw[j] << 16) > 0.0f)) e0 *= cg.slope;
            if (!(__uint_as_float(aw[j] & 0xFFFF0000u) > 0.0f)) e1 *= cg.slope;
            ow[j] = static_cast<uint32_t>(to_bf16(e0)) | (static_cast<uint32_t>(to_bf16(e1)) << 16);
          }
          *reinterpret_cast<uint4*>(cg.dz16 + i0) = make_uint4(ow[0], ow[1], ow[2], ow[3]);
        }
      }
      __syncthreads();
    }
    return;
  }
#pragma unroll
  for (int t = 0; t < NT16; ++t) {
    const int co = nco0 + t * 16 + r;
    if (co >= cg.cout) continue;
#pragma unroll
    for (int q2 = 0; q2 < MT; ++q2) {
      const int qy = oy + q2;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int qx = ox + 4 * kg + i;
        if (qz >= h0 || qy >= h1 || qx >= h2) continue;
        const long long vo =
            (static_cast<long long>(2 * qz + pz) * cg.o1 + 2 * qy + py) * cg.o2 + 2 * qx + px;
        const long long mo = s * per + vo;
        float val = acc[q2][t][i];
        if (cg.act) val = val > 0.0f ? val : cg.slope * val;
        if (y16) {
          y16[mo * cg.cout + co] = to_bf16(val);
        } else if (cg.ycl32) {
          store_cl32(cg, y32, mo, co, val);
        } else {
          y32[(s * cg.cout + co) * per + vo] = val;
        }
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

// ------------------------------------------------------------- training

// dW tiles 16 (co) x 16 NK (k) of one wave over a chunk of output voxels:
// C[co][k] = sum_v dz[v][co] X(v, k) with the 32 voxels of a K step as the
// MFMA reduction.  Both operands are stored channels-last, while each lane's
// MFMA fragment holds 8 consecutive voxels of one row or column.  A K step
// stages them channels-last in LDS, lane l writing the 8 channels of voxel
// l % 32 it loaded (one 16-byte write; for X, a group of 8 consecutive k is
// one tap and 8 channels), and reads its fragments with the transposing LDS
// read: within each 16-lane group, lane j points at the 4 channels
// 4 (j % 4).. of voxel base + j / 4, and lane i receives channel i of the
// voxels base.. base + 3, so two reads give a lane its 8 voxels.
// A wave reduces wch voxels (a multiple of 32) before its atomics into the
// gradient: longer chunks mean fewer atomics on the same gradient entries,
// shorter ones more waves for small layers (chosen at launch).
constexpr int WNK = 4;  // 16-column k tiles per wave
// MFMA fragment of lane (g, r) from a [32 voxel][16] BF16 LDS tile: element
// m of the result is tile[8 g + m][r] (two transposing reads of 4 voxels).
typedef short v4i16 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ bf16x8 tr_frag(const uint16_t* tile, int g, int r) {
  typedef __attribute__((address_space(3))) v4i16* lds_v4;
  const uint16_t* p = tile + (8 * g + (r >> 2)) * 16 + 4 * (r & 3);
  const v4i16 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4)(p));
  const v4i16 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4)(p + 4 * 16));
  return __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

template <int X0>
__global__ __launch_bounds__(64) void k_conv_wgrad(int wch, const uint16_t* __restrict__ dz, int cz,
                                                   const uint16_t* __restrict__ x0,
                                                   const uint16_t* __restrict__ x1, ConvGeom cg,
                                                   float* __restrict__ dw,
                                                   float* __restrict__ db) {
  __shared__ __align__(16) uint16_t at[32 * 16];       // dz: [voxel][co]
  __shared__ __align__(16) uint16_t bt[WNK][32 * 16];  // X:  [voxel][k]
  constexpr bool half = X0 != 0;  // x0 is stored at half resolution
  const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
  const int vl = lane & 31, h = lane >> 5;  // staged voxel, channel half
  const int cvec = (cg.c0 + cg.c1) >> 3;
  // the waves of one voxel chunk (every k group and co tile) are
  // consecutive on one XCD, so that its dz and input rows are read there
  // from L2 after the first of them
  const uint32_t ngk = (cg.kpad + 16 * WNK - 1) / (16 * WNK);
  const uint32_t wid = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t kgrp = wid % ngk, wrest = wid / ngk;
  const uint32_t ntz = (cg.cout + 15) / 16;
  const int co0 = static_cast<int>(wrest % ntz) * 16;
  const uint32_t chunk = wrest / ntz;
  const int kb = static_cast<int>(kgrp) * 16 * WNK;  // first k column of the wave
  const int h0 = half ? cg.i0 / 2 : cg.i0, h1 = half ? cg.i1 / 2 : cg.i1;
  const int h2 = half ? cg.i2 / 2 : cg.i2;
  const long long vin0 = static_cast<long long>(h0) * h1 * h2;
  const long long vin1 = static_cast<long long>(cg.i0) * cg.i1 * cg.i2;
  // column groups this lane stages: (tap, channel) of k = kb + 16 t + 8 h,
  // as tap offset + 1 per axis and, for full-resolution reads, the tap's
  // voxel offset
  int gta[WNK], gtb[WNK], gtc[WNK], gch[WNK], gto[WNK];
  bool gok[WNK];
#pragma unroll
  for (int t = 0; t < WNK; ++t) {
    const int kv = (kb + 16 * t) / 8 + h;
    const int tap = kv / cvec;
    gch[t] = (kv - tap * cvec) * 8;
    gok[t] = tap < cg.ntaps;
    gta[t] = gtb[t] = gtc[t] = 1;
    if (cg.ntaps == 27) {
      gta[t] = tap / 9;
      gtb[t] = (tap / 3) % 3;
      gtc[t] = tap % 3;
    }
    gto[t] = (gta[t] * cg.i1 + gtb[t]) * cg.i2 + gtc[t];
  }
  // coordinates of the staged voxel, advanced by 32 voxels per K step
  const long long vstart = static_cast<long long>(chunk) * wch + vl;
  const long long ov = static_cast<long long>(cg.o0) * cg.o1 * cg.o2;
  int s = 0, o0 = 0, o1 = 0, o2 = 0;
  if (vstart < cg.nvox) {
    s = static_cast<int>(vstart / ov);
    int rem = static_cast<int>(vstart - s * ov);
    o2 = rem % cg.o2;
    rem /= cg.o2;
    o1 = rem % cg.o1;
    o0 = rem / cg.o1;
  }
  f32x4 acc[WNK];
#pragma unroll
  for (int t = 0; t < WNK; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  // the bias gradient sum_v dz[v][co], from the staged dz of the first k tile
  const bool bias = db != nullptr && kgrp == 0;
  float bacc[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  // The loads of one K step (every load issued, from x0 or dz itself where
  // the value is zero; the padding is applied when staged), then the staged
  // voxel's coordinates advanced by 32.  A step's loads are issued before
  // the previous step's products, so they arrive while those run.
  auto issue = [&](int step, uint4& araw, bool& ain, uint4 (&braw)[WNK], bool (&bin)[WNK]) {
    const long long v = static_cast<long long>(chunk) * wch + step + vl;
    const bool live = v < cg.nvox;
    ain = live && co0 + 8 * h < cz;
    araw = *reinterpret_cast<const uint4*>(ain ? dz + v * cz + co0 + 8 * h : dz);
    const int q0 = o0 * cg.stride - 1, q1 = o1 * cg.stride - 1, q2 = o2 * cg.stride - 1;
    const int lb = (q0 * cg.i1 + q1) * cg.i2 + q2;
    const uint16_t* t0 = x0 + s * vin0 * cg.c0;
    const uint16_t* t1 = x1 + s * vin1 * cg.c1 - cg.c0;  // x1 channels follow the c0 of x0
#pragma unroll
    for (int t = 0; t < WNK; ++t) {
      const int p0 = q0 + gta[t], p1 = q1 + gtb[t], p2 = q2 + gtc[t];
      bool ok = live && gok[t] && static_cast<unsigned>(p0) < static_cast<unsigned>(cg.i0) &&
                static_cast<unsigned>(p1) < static_cast<unsigned>(cg.i1) &&
                static_cast<unsigned>(p2) < static_cast<unsigned>(cg.i2);
      const bool from0 = gch[t] < cg.c0;
      const uint16_t* src;
      if (!half) {
        src = (from0 ? t0 : t1) + static_cast<long long>(lb + gto[t]) * (from0 ? cg.c0 : cg.c1) +
              gch[t];
      } else if (from0) {
        if (X0 == 2) ok = ok && !((p0 | p1 | p2) & 1);
        src = t0 + static_cast<long long>(((p0 >> 1) * h1 + (p1 >> 1)) * h2 + (p2 >> 1)) * cg.c0 +
              gch[t];
      } else {
        src = t1 + static_cast<long long>(lb + gto[t]) * cg.c1 + gch[t];
      }
      bin[t] = ok;
      braw[t] = *reinterpret_cast<const uint4*>(ok ? src : x0);
    }
    o2 += 32;
    while (o2 >= cg.o2) {
      o2 -= cg.o2;
      if (++o1 == cg.o1) {
        o1 = 0;
        if (++o0 == cg.o0) {
          o0 = 0;
          ++s;
        }
      }
    }
  };
  uint4 ca, cb[WNK], na, nb[WNK];
  bool cain, cbin[WNK], nain, nbin[WNK];
  issue(0, ca, cain, cb, cbin);
  for (int step = 0; step < wch; step += 32) {
    const long long vb = static_cast<long long>(chunk) * wch + step;
    if (vb >= cg.nvox) break;  // uniform across the wave
    // zero padding by selects (a branch would wait for every load in flight)
    auto keep = [](uint4 q, bool k) {
      return make_uint4(k ? q.x : 0u, k ? q.y : 0u, k ? q.z : 0u, k ? q.w : 0u);
    };
    ca = keep(ca, cain);
#pragma unroll
    for (int t = 0; t < WNK; ++t) cb[t] = keep(cb[t], cbin[t]);
    *reinterpret_cast<uint4*>(&at[vl * 16 + 8 * h]) = ca;
    if (bias) {
      const uint32_t aw[4] = {ca.x, ca.y, ca.z, ca.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        bacc[2 * j] += __uint_as_float(aw[j] << 16);
        bacc[2 * j + 1] += __uint_as_float(aw[j] & 0xFFFF0000u);
      }
    }
#pragma unroll
    for (int t = 0; t < WNK; ++t) *reinterpret_cast<uint4*>(&bt[t][vl * 16 + 8 * h]) = cb[t];
    // the next step's loads (past the chunk or the volume: from clamped
    // addresses, never staged)
    issue(step + 32, na, nain, nb, nbin);
    // one wave: its LDS operations complete in order, so the reads below
    // see the writes above, and the next step's writes follow these reads
    const bf16x8 afrag = tr_frag(at, g, r);
#pragma unroll
    for (int t = 0; t < WNK; ++t)
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag, tr_frag(bt[t], g, r), acc[t], 0, 0,
                                                         0);
    ca = na;
    cain = nain;
#pragma unroll
    for (int t = 0; t < WNK; ++t) {
      cb[t] = nb[t];
      cbin[t] = nbin[t];
    }
  }
#pragma unroll
  for (int t = 0; t < WNK; ++t) {
    const int kcol = kb + 16 * t + r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = co0 + 4 * g + i;
      if (co < cg.cout && kcol < cg.kpad)
        atomicAdd(dw + static_cast<long long>(co) * cg.kpad + kcol, acc[t][i]);
    }
  }
  if (bias) {
    // sum over the 32 staged voxels of each channel half, one atomic per channel
#pragma unroll
    for (int j = 0; j < 8; ++j) {
#pragma unroll
      for (int m = 16; m >= 1; m >>= 1) bacc[j] += __shfl_xor(bacc[j], m, 64);
    }
    if (vl == 0) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int co = co0 + 8 * h + j;
        if (co < cg.cout) atomicAdd(db + co, bacc[j]);
      }
    }
  }
}

// Weight gradients of a stride-1, 27-tap layer, all taps of one input
// channel group at once: a wave takes a co tile of 16, one group of 8 input
// channels and a run of K steps, a K step being 32 output voxels, R rows
// (d1) of W = 32 / R along d2.  The input positions that the 27 taps read
// for them (3 x (R + 2) rows of W + 2 positions, 8 channels each) are staged
// in LDS once per step; each of the 14 column tiles (taps 2t and 2t + 1,
// 8 channels each) then reads its B fragment there through the transposing
// LDS read, lane j of a 16-lane group pointing at the 4 channels 4 (j % 4)..
// of tile column group j % 4 at voxel base + j / 4.  A step stages 9.6
// (R = 1), 6.8 (R = 2) or 5.6 (R = 4) input positions per output voxel
// where the tap-by-tap kernel above loads 27.
template <int X0, int R>
__global__ __launch_bounds__(64) void k_conv_wgrad_rows(int wsteps,
                                                        const uint16_t* __restrict__ dz, int cz,
                                                        const uint16_t* __restrict__ x0,
                                                        const uint16_t* __restrict__ x1,
                                                        ConvGeom cg, float* __restrict__ dw,
                                                        float* __restrict__ db) {
  constexpr int W = 32 / R;    // output voxels per row of a step
  constexpr int NXP = W + 2;   // input positions along d2
  constexpr int NYP = R + 2;   // input rows along d1
  constexpr int NPOS = 3 * NYP * NXP;
  constexpr int NLD = (NPOS + 63) / 64;  // staged positions per lane
  constexpr int NTT = 14;                // column tiles: 27 taps (and one empty) x 8 channels
  __shared__ __align__(16) uint16_t xs[NPOS * 8];  // [position][8 channels]
  __shared__ __align__(16) uint16_t at[32 * 16];   // dz: [voxel][co]
  const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
  const int vl = lane & 31, h = lane >> 5;  // staged voxel of dz, channel half
  // The waves of one run of K steps (every channel group and co tile) are
  // consecutive on one XCD, so that its dz and input rows are read there
  // from L2 after the first of them.
  const int cin = cg.c0 + cg.c1;
  const uint32_t wid = xcd_remap(blockIdx.x, gridDim.x);
  const int ngrp = cin / 8;
  const int grp = static_cast<int>(wid % ngrp);  // input channels 8 grp .. 8 grp + 7
  const uint32_t wrest = wid / ngrp;
  const int ntz = (cg.cout + 15) / 16;
  const int co0 = static_cast<int>(wrest % ntz) * 16;
  const uint32_t chunk = wrest / ntz;
  const bool from0 = grp * 8 < cg.c0;
  const uint16_t* src = from0 ? x0 : x1;
  const int cstr = from0 ? cg.c0 : cg.c1;  // channels per voxel of that tensor
  const int coff = from0 ? grp * 8 : grp * 8 - cg.c0;
  const bool half = X0 == 1 && from0;  // x0 at half resolution, nearest upsampled
  const int hi0 = half ? cg.i0 / 2 : cg.i0, hi1 = half ? cg.i1 / 2 : cg.i1;
  const int hi2 = half ? cg.i2 / 2 : cg.i2;
  const long long vin = static_cast<long long>(hi0) * hi1 * hi2;
  // per lane: the B row (position, channel half) of each column tile, as an
  // LDS element offset from its voxel's first position
  int toff[NTT];
#pragma unroll
  for (int t = 0; t < NTT; ++t) {
    const int tap = min(2 * t + ((r & 3) >> 1), 26);  // tap 27 (empty columns): any valid row
    toff[t] = (((tap / 9) * NYP + (tap / 3) % 3) * NXP + tap % 3) * 8 + (r & 1) * 4;
  }
  // voxel m = 8 g + j / 4 of the step (row m / W) and m + 4 (the same row)
  const int mv = 8 * g + (r >> 2);
  const int vrow = ((mv / W) * NXP + mv % W) * 8;
  const int nseg = (cg.o2 + W - 1) / W;
  const int nrg = (cg.o1 + R - 1) / R;  // groups of R rows per plane
  const long long nsteps = static_cast<long long>(cg.nvox / (static_cast<long long>(cg.o1) * cg.o2)) * nrg * nseg;
  f32x4 acc[NTT];
#pragma unroll
  for (int t = 0; t < NTT; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const bool bias = db != nullptr && grp == 0;
  float bacc[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  const long long s0 = static_cast<long long>(chunk) * wsteps;
  const long long s1 = min(s0 + wsteps, nsteps);
  // The loads of one K step (every load issued, from dz or the subject's
  // first input voxel where the value is zero; the padding is applied when
  // staged).  A step's loads are issued before the previous step's
  // products; past the run the last step is loaded again and never staged.
  // The step's rows (subject sj, output plane oz, first row oy) and segment
  // are kept as counters (wave-uniform, advanced once per step: no division
  // in the loop), and the per-lane offsets are 32-bit (the launch checks
  // that every input tensor's subject holds fewer than 2^31 elements).
  const long long rg0 = s0 / nseg;  // row group of the first step
  int seg = static_cast<int>(s0 - rg0 * nseg);
  int oy = static_cast<int>(rg0 % nrg) * R;
  int oz = static_cast<int>((rg0 / nrg) % cg.o0);
  int sj = static_cast<int>(rg0 / nrg / cg.o0);
  auto advance = [&]() {
    if (++seg == nseg) {
      seg = 0;
      oy += R;
      if (oy >= cg.o1) {
        oy = 0;
        if (++oz == cg.o0) {
          oz = 0;
          ++sj;
        }
      }
    }
  };
  const int vy = vl / W, vx = vl % W;  // the dz voxel this lane stages
  auto issue = [&](uint4& a, bool& aok, uint4 (&xv)[NLD], bool (&xin)[NLD]) {
    const int x0v = seg * W;
    aok = oy + vy < cg.o1 && x0v + vx < cg.o2 && co0 + 8 * h < cz;
    const uint16_t* dplane = dz + (static_cast<long long>(sj) * cg.o0 + oz) * cg.o1 * cg.o2 * cz;
    a = *reinterpret_cast<const uint4*>(
        dplane + (aok ? ((oy + vy) * cg.o2 + x0v + vx) * cz + co0 + 8 * h : 0));
    const int qz = oz - 1, qy = oy - 1, qx = x0v - 1;
    const uint16_t* base = src + static_cast<long long>(sj) * vin * cstr + coff;
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int i = lane + 64 * k;
      const int pa = i / (NYP * NXP), pb = (i / NXP) % NYP, xi = i % NXP;
      const int pz = qz + pa, py = qy + pb, px = qx + xi;
      xin[k] = i < NPOS && static_cast<unsigned>(pz) < static_cast<unsigned>(cg.i0) &&
               static_cast<unsigned>(py) < static_cast<unsigned>(cg.i1) &&
               static_cast<unsigned>(px) < static_cast<unsigned>(cg.i2);
      const int pv = half ? ((pz >> 1) * hi1 + (py >> 1)) * hi2 + (px >> 1) : (pz * hi1 + py) * hi2 + px;
      xv[k] = *reinterpret_cast<const uint4*>(base + static_cast<uint32_t>(xin[k] ? pv * cstr : 0));
    }
  };
  auto keep = [](uint4 q, bool kp) {
    return make_uint4(kp ? q.x : 0u, kp ? q.y : 0u, kp ? q.z : 0u, kp ? q.w : 0u);
  };
  uint4 ca, na, cx[NLD], nx[NLD];
  bool caok, naok, cxin[NLD], nxin[NLD];
  if (s0 < s1) issue(ca, caok, cx, cxin);
  for (long long step = s0; step < s1; ++step) {
    // stage dz of the segment's 32 voxels (zero past the row end) and the
    // input positions every tap reads (zero padding outside the volume)
    ca = keep(ca, caok);
    *reinterpret_cast<uint4*>(&at[vl * 16 + 8 * h]) = ca;
    if (bias) {
      const uint32_t aw[4] = {ca.x, ca.y, ca.z, ca.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        bacc[2 * j] += __uint_as_float(aw[j] << 16);
        bacc[2 * j + 1] += __uint_as_float(aw[j] & 0xFFFF0000u);
      }
    }
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int i = lane + 64 * k;
      if (i < NPOS) *reinterpret_cast<uint4*>(&xs[i * 8]) = keep(cx[k], cxin[k]);
    }
    if (step + 1 < s1) advance();
    issue(na, naok, nx, nxin);
    // one wave: its LDS operations complete in order
    const bf16x8 afrag = tr_frag(at, g, r);
    typedef __attribute__((address_space(3))) v4i16* lds_v4;
#pragma unroll
    for (int t = 0; t < NTT; ++t) {
      const uint16_t* p = xs + vrow + toff[t];
      const v4i16 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4)(p));
      const v4i16 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4)(p + 4 * 8));
      const bf16x8 bfrag =
          __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag, bfrag, acc[t], 0, 0, 0);
    }
    ca = na;
    caok = naok;
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      cx[q] = nx[q];
      cxin[q] = nxin[q];
    }
  }
#pragma unroll
  for (int t = 0; t < NTT; ++t) {
    const int tap = 2 * t + (r >> 3);
    if (tap > 26) continue;
    const int kcol = tap * cin + grp * 8 + (r & 7);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = co0 + 4 * g + i;
      if (co < cg.cout) atomicAdd(dw + static_cast<long long>(co) * cg.kpad + kcol, acc[t][i]);
    }
  }
  if (bias) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
#pragma unroll
      for (int m = 16; m >= 1; m >>= 1) bacc[j] += __shfl_xor(bacc[j], m, 64);
    }
    if (vl == 0) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int co = co0 + 8 * h + j;
        if (co < cg.cout) atomicAdd(db + co, bacc[j]);
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_pack_wt(const float* __restrict__ w, int cin, int cout,
                                                    int cz, int kpad_f, int kpad_t,
                                                    uint16_t* __restrict__ wt) {
  const long long i = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= static_cast<long long>(cin) * kpad_t) return;
  const int ci = static_cast<int>(i / kpad_t), k = static_cast<int>(i - static_cast<long long>(ci) * kpad_t);
  const int tp = k / cz, co = k - tp * cz;
  float val = 0.0f;
  if (tp < 27 && co < cout) val = w[static_cast<long long>(co) * kpad_f + (26 - tp) * cin + ci];
  wt[i] = to_bf16(val);
}

__global__ __launch_bounds__(kBlock) void k_to_bf16(const float* __restrict__ in,
                                                    uint16_t* __restrict__ out, long long count) {
  const long long i = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < count) out[i] = to_bf16(in[i]);
}

// The loss of the prediction p [n][c][V] against t (same layout) and its
// gradient as the output layer's BF16 output gradient: loss += sum (p - t)^2
// / count (FP64, count = n c V), dz [n V][cz] channels-last = BF16(2 (p - t)
// / count) for channels below c, zero above (the output layer has no
// activation).  One thread per voxel, grid-stride within subject
// blockIdx.y; one loss atomic per block.
__global__ __launch_bounds__(kBlock) void k_mse_dz(const float* __restrict__ p,
                                                   const float* __restrict__ t, long long V,
                                                   int c, int cz, double inv,
                                                   double* __restrict__ loss,
                                                   uint16_t* __restrict__ dz) {
  __shared__ double red[kBlock / 64];
  const long long sub = blockIdx.y;
  const float* ps = p + sub * c * V;
  const float* ts = t + sub * c * V;
  uint16_t* ds = dz + sub * V * cz;
  double acc = 0.0;
  const long long stride = static_cast<long long>(gridDim.x) * kBlock;
  for (long long v = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x; v < V; v += stride) {
    for (int c8 = 0; c8 < cz; c8 += 8) {
      uint32_t wd[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (c8 + j >= c) break;
        const double d = static_cast<double>(ps[(c8 + j) * V + v]) - static_cast<double>(ts[(c8 + j) * V + v]);
        acc += d * d * inv;
        wd[j >> 1] |= static_cast<uint32_t>(to_bf16(static_cast<float>(2.0 * d * inv))) << (16 * (j & 1));
      }
      *reinterpret_cast<uint4*>(ds + v * cz + c8) = make_uint4(wd[0], wd[1], wd[2], wd[3]);
    }
  }
  const double tot = block_sum<kBlock>(acc, red);
  if (threadIdx.x == 0) atomicAdd(loss, tot);
}


}  // namespace

uint32_t grid_1d(long long count) { return static_cast<uint32_t>((count + kBlock - 1) / kBlock); }

void launch_conv_wgrad(const uint16_t* dz, int cz, const uint16_t* x0, const uint16_t* x1,
                       const ConvGeom& cg, float* dw, float* db, hipStream_t st) {
  prof_begin(st, KC_MISC);
  const uint32_t gy = static_cast<uint32_t>((cg.kpad + 16 * WNK - 1) / (16 * WNK));
  const uint32_t gz = static_cast<uint32_t>((cg.cout + 15) / 16);
  // voxels per wave: doubled from 1024 up to 4096 while at least 2048
  // waves (two per SIMD) remain (measured on the warm-start network at
  // 96 x 112 x 96: longer chunks starve the low-resolution layers)
  const long long vfull = static_cast<long long>(cg.i0) * cg.i1 * cg.i2;
  if (cg.ntaps == 27 && cg.stride == 1 && !cg.dil0 && cg.c0 + cg.c1 >= 16 &&
      vfull * std::max(cg.c0, cg.c1) < (1LL << 31)) {
    // all taps of a channel group per wave (measured on the warm-start
    // network at 96 x 112 x 96: faster than the tap-by-tap kernel on its
    // decoder layers, six or more channel groups, and slightly on its output
    // layer, two groups; slower on its first layer, one group of 8 channels
    // of which two are used); K steps per wave doubled from 8 up to 256
    // while at least 2048 waves remain (longer runs mean fewer atomics on
    // the same gradient entries)
    // Rows per K step: 4 (8 voxels each) where d2 is a multiple of 8, so
    // that no lane of a step falls past the row, else one row of 32
    const int rr = cg.o2 % 8 == 0 ? 4 : 1;
    const uint32_t ngrp = static_cast<uint32_t>((cg.c0 + cg.c1) / 8);
    const int wv = 32 / rr;
    const long long nsteps = cg.nvox / (static_cast<long long>(cg.o1) * cg.o2) *
                             ((cg.o1 + rr - 1) / rr) * ((cg.o2 + wv - 1) / wv);
    long long ws = 8;
    while (ws < 256 && (nsteps + 2 * ws - 1) / (2 * ws) * ngrp * gz >= 2048) ws *= 2;
    const dim3 grid(static_cast<uint32_t>((nsteps + ws - 1) / ws * ngrp * gz));
    const int w = static_cast<int>(ws);
    auto go = [&](auto xm, auto rm) {
      constexpr int XM = decltype(xm)::value, RM = decltype(rm)::value;
      hipLaunchKernelGGL((k_conv_wgrad_rows<XM, RM>), grid, dim3(64), 0, st, w, dz, cz, x0, x1, cg,
                         dw, db);
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I4 = std::integral_constant<int, 4>;
    if (cg.up0) {
      if (rr == 4) go(I1{}, I4{}); else go(I1{}, I1{});
    } else {
      if (rr == 4) go(I0{}, I4{}); else go(I0{}, I1{});
    }
    prof_end(st, KC_MISC);
    return;
  }
  long long wch = 1024;
  while (wch < 4096 && (cg.nvox + 2 * wch - 1) / (2 * wch) * gy * gz >= 2048) wch *= 2;
  const dim3 grid(static_cast<uint32_t>((cg.nvox + wch - 1) / wch * gy * gz));
  const int w = static_cast<int>(wch);
  if (cg.dil0)
    hipLaunchKernelGGL((k_conv_wgrad<2>), grid, dim3(64), 0, st, w, dz, cz, x0, x1, cg, dw, db);
  else if (cg.up0)
    hipLaunchKernelGGL((k_conv_wgrad<1>), grid, dim3(64), 0, st, w, dz, cz, x0, x1, cg, dw, db);
  else
    hipLaunchKernelGGL((k_conv_wgrad<0>), grid, dim3(64), 0, st, w, dz, cz, x0, x1, cg, dw, db);
  prof_end(st, KC_MISC);
}

void launch_pack_wt(const float* w, int cin, int cout, int cz, int kpad_f, int kpad_t,
                    uint16_t* wt, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_wt, dim3(grid_1d(static_cast<long long>(cin) * kpad_t)), dim3(kBlock),
                     0, st, w, cin, cout, cz, kpad_f, kpad_t, wt);
}

void launch_to_bf16(const float* in, uint16_t* out, long long count, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_1d(count)), dim3(kBlock), 0, st, in, out, count);
}

void launch_mse_dz(const float* p, const float* t, int n, long long V, int c, int cz,
                   double* loss, uint16_t* dz, hipStream_t st) {
  const uint32_t bx = std::max(1u, std::min(grid_1d(V), 2048u / static_cast<uint32_t>(n)));
  hipLaunchKernelGGL(k_mse_dz, dim3(bx, static_cast<uint32_t>(n)), dim3(kBlock), 0, st, p, t, V, c,
                     cz, 1.0 / (static_cast<double>(n) * c * V), loss, dz);
}

int conv_kpad(int cin, int ntaps) {
  const int cv = (cin + 7) / 8;
  return (ntaps * cv * 8 + 31) / 32 * 32;
}

namespace {
template <int NT16, int MT>
void conv3d_x0(int mode, dim3 grid, const uint16_t* x0, const uint16_t* x1, const uint16_t* w,
               const float* bias, uint16_t* y16, float* y32, const ConvGeom& cg, hipStream_t st) {
  if (mode == 0)
    hipLaunchKernelGGL((k_conv3d<NT16, MT, 0>), grid, dim3(CNT), 0, st, x0, x1, w, bias, y16, y32,
                       cg);
  else if (mode == 1)
    hipLaunchKernelGGL((k_conv3d<NT16, MT, 1>), grid, dim3(CNT), 0, st, x0, x1, w, bias, y16, y32,
                       cg);
  else
    hipLaunchKernelGGL((k_conv3d<NT16, MT, 2>), grid, dim3(CNT), 0, st, x0, x1, w, bias, y16, y32,
                       cg);
}
}  // namespace

namespace {
constexpr int kLdsMT = 4;

template <int NT16, int CG>
void conv3d_lds_x0(int mode, dim3 grid, const uint16_t* x0, const uint16_t* x1, const uint16_t* w,
                   const float* bias, uint16_t* y16, float* y32, const ConvGeom& cg, int nbz,
                   int nby, int nbx, hipStream_t st) {
  if (mode == 0)
    hipLaunchKernelGGL((k_conv3d_lds<NT16, kLdsMT, 0, CG>), grid, dim3(CNT), 0, st, x0, x1, w,
                       bias, y16, y32, cg, nbz, nby, nbx);
  else if (mode == 1)
    hipLaunchKernelGGL((k_conv3d_lds<NT16, kLdsMT, 1, CG>), grid, dim3(CNT), 0, st, x0, x1, w,
                       bias, y16, y32, cg, nbz, nby, nbx);
  else
    hipLaunchKernelGGL((k_conv3d_lds<NT16, kLdsMT, 2, CG>), grid, dim3(CNT), 0, st, x0, x1, w,
                       bias, y16, y32, cg, nbz, nby, nbx);
}

template <int NT16>
void conv3d_lds_cg(int mode, dim3 grid, const uint16_t* x0, const uint16_t* x1, const uint16_t* w,
                   const float* bias, uint16_t* y16, float* y32, const ConvGeom& cg, int nbz,
                   int nby, int nbx, hipStream_t st) {
  // two channel groups per chunk when they pair up exactly
  if (((cg.c0 + cg.c1) / 8) % 2)
    conv3d_lds_x0<NT16, 1>(mode, grid, x0, x1, w, bias, y16, y32, cg, nbz, nby, nbx, st);
  else
    conv3d_lds_x0<NT16, 2>(mode, grid, x0, x1, w, bias, y16, y32, cg, nbz, nby, nbx, st);
}
}  // namespace

void launch_conv3d(const uint16_t* x0, const uint16_t* x1, const uint16_t* w, const float* bias,
                   uint16_t* y16, float* y32, const ConvGeom& cg, hipStream_t st) {
  // row tiles per wave (MT) share each K step's weight fragments
  auto gx = [&](int mt) {
    return static_cast<uint32_t>((cg.nvox + static_cast<long long>(CROWS) * mt - 1) /
                                 (static_cast<long long>(CROWS) * mt));
  };
  prof_begin(st, KC_MISC);
  const int mode = cg.dil0 ? 2 : (cg.up0 ? 1 : 0);
  if (cg.stride == 1 && cg.ntaps == 27 && cg.dil0 && cg.c1 == 0 && !bias) {
    // zero-dilated input (input gradients of stride-2 layers): one launch
    // over the eight parity classes, valid taps only
    const int nbz = (cg.o0 / 2 + LBZ - 1) / LBZ, nby = (cg.o1 / 2 + kLdsMT - 1) / kLdsMT;
    const int nbx = (cg.o2 / 2 + LBX - 1) / LBX;
    const long long per = static_cast<long long>(cg.o0) * cg.o1 * cg.o2;
    const uint32_t gx =
        static_cast<uint32_t>(8LL * nbz * nby * nbx * (cg.nvox / per));
    const bool cg2 = (cg.c0 / 8) % 2 == 0;
    auto go = [&](auto nt, uint32_t gy) {
      constexpr int NT = decltype(nt)::value;
      if (cg2)
        hipLaunchKernelGGL((k_conv3d_sub<NT, kLdsMT, 2>), dim3(gx, gy), dim3(CNT), 0, st, x0, w,
                           y16, y32, cg, nbz, nby, nbx);
      else
        hipLaunchKernelGGL((k_conv3d_sub<NT, kLdsMT, 1>), dim3(gx, gy), dim3(CNT), 0, st, x0, w,
                           y16, y32, cg, nbz, nby, nbx);
    };
    if (cg.cout <= 16)
      go(std::integral_constant<int, 1>{}, 1);
    else if (cg.cout <= 32)
      go(std::integral_constant<int, 2>{}, 1);
    else
      go(std::integral_constant<int, 4>{}, static_cast<uint32_t>((cg.cout + 63) / 64));
  } else if (cg.stride == 1 && cg.ntaps == 27) {
    // input bricks staged in LDS
    const int nbz = (cg.o0 + LBZ - 1) / LBZ, nby = (cg.o1 + kLdsMT - 1) / kLdsMT;
    const int nbx = (cg.o2 + LBX - 1) / LBX;
    const long long per = static_cast<long long>(cg.o0) * cg.o1 * cg.o2;
    const uint32_t gx = static_cast<uint32_t>(static_cast<long long>(nbz) * nby * nbx * (cg.nvox / per));
    // column tiles per wave: 48 channels where they divide cout and 64 do
    // not (the input gradients of concatenated layers: 48, 96), so that no
    // tile is computed for channels past cout
    if (cg.cout <= 16)
      conv3d_lds_cg<1>(mode, dim3(gx, 1), x0, x1, w, bias, y16, y32, cg, nbz, nby, nbx, st);
    else if (cg.cout <= 32)
      conv3d_lds_cg<2>(mode, dim3(gx, 1), x0, x1, w, bias, y16, y32, cg, nbz, nby, nbx, st);
    else if (cg.cout % 64 != 0 && cg.cout % 48 == 0)
      conv3d_lds_cg<3>(mode, dim3(gx, static_cast<uint32_t>(cg.cout / 48)), x0, x1, w, bias, y16,
                       y32, cg, nbz, nby, nbx, st);
    else
      conv3d_lds_cg<4>(mode, dim3(gx, static_cast<uint32_t>((cg.cout + 63) / 64)), x0, x1, w,
                       bias, y16, y32, cg, nbz, nby, nbx, st);
  } else if (cg.cout <= 16) {
    conv3d_x0<1, 4>(mode, dim3(gx(4), 1), x0, x1, w, bias, y16, y32, cg, st);
  } else if (cg.cout <= 32) {
    conv3d_x0<2, 2>(mode, dim3(gx(2), 1), x0, x1, w, bias, y16, y32, cg, st);
  } else {
    const uint32_t gy = static_cast<uint32_t>((cg.cout + 63) / 64);
    conv3d_x0<4, 2>(mode, dim3(gx(2), gy), x0, x1, w, bias, y16, y32, cg, st);
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
