// Scaling and squaring (Section 3, "Diffeomorphisms") and its adjoint.
//
// Forward step: u_{t+1}(x) = u_t(x) + u_t(x + u_t(x)), trilinear with border
// clamping; the first step reads v and scales it by 2^-N on the fly.
//
// Adjoint step: g_t(y) = g(y) + J_t(y)^T g(y) + sum_x sum_k [corner_k(x) = y] w_k(x) g(x)
// with g = g_{t+1}.  The scatter term is computed owner-side, as a gather: a
// block owns one output tile, bins the source voxels whose trilinear cells
// touch it by cell (one LDS integer atomic per source), and then every output
// voxel sums over the sources binned in its 8 neighbouring cells.  Which
// source voxels to look at follows from the offsets (cell index - voxel
// index) the forward step recorded per tile, so no global atomics and no
// zero-fill pass are needed, and each output value is written once.  (Float
// atomics in LDS are serialised lane by lane on this hardware: scattering the
// 24 weighted corner values of every source with them costs an order of
// magnitude more than this binning.)  Forward tiles are 32 (d2) x 8 (d1) x 8
// (d0) voxels, adjoint tiles 32 x 4 x 4.
#include <climits>

#include "darc_kernels.hpp"

namespace darc {

namespace {

constexpr int ETX = 32, ETY = 8, ETZ = 8;
constexpr int ENT = ETX * ETY;             // threads per block

struct TileGeom {
  Geom g;
  int ntx, nty, ntz, ntiles;
  uint32_t total;  // ntiles * subjects
};

TileGeom make_tiles(const Geom& g, int n) {
  TileGeom t;
  t.g = g;
  t.ntx = (g.d2 + ETX - 1) / ETX;
  t.nty = (g.d1 + ETY - 1) / ETY;
  t.ntz = (g.d0 + ETZ - 1) / ETZ;
  t.ntiles = t.ntx * t.nty * t.ntz;
  t.total = static_cast<uint32_t>(t.ntiles) * n;
  return t;
}

struct TileId {
  int s, tile, oz, oy, ox;
};

__device__ __forceinline__ TileId tile_id(const TileGeom& tg) {
  const uint32_t b = xcd_remap(blockIdx.x, tg.total);
  TileId id;
  id.s = static_cast<int>(b / tg.ntiles);
  id.tile = static_cast<int>(b - static_cast<uint32_t>(id.s) * tg.ntiles);
  const int tx = id.tile % tg.ntx;
  const int r = id.tile / tg.ntx;
  const int ty = r % tg.nty;
  const int tz = r / tg.nty;
  id.ox = tx * ETX;
  id.oy = ty * ETY;
  id.oz = tz * ETZ;
  return id;
}

__device__ __forceinline__ int wave_min(int x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x = min(x, __shfl_xor(x, m, 64));
  return x;
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x = max(x, __shfl_xor(x, m, 64));
  return x;
}

// MODE 0: squaring step only; 1: step and cell offsets; 2: cell offsets only.
// boxes[(s * ntiles + tile) * 8 + {0,1,2}] = min over the tile's voxels x of
// i_d(x) - x_d along d0, d1, d2 (i = cell index of x + u(x)), [.. + {3,4,5}] =
// the max; so the corners a voxel x touches lie in x + [min, max + 1].
// reach[s * 8 + d] = max(0, -min over tiles of the min offset) and
// reach[s * 8 + 3 + d] = max(0, max over tiles of the max offset + 1): how far
// below / above itself any voxel of the subject can scatter (zeroed before).
template <bool FIRST, int MODE>
__global__ __launch_bounds__(ENT) void k_exp_fwd(const float* __restrict__ src,
                                                 float* __restrict__ dst, TileGeom tg, float scale,
                                                 int* __restrict__ boxes, int* __restrict__ reach) {
  __shared__ int red[6][ENT / 64];
  const Geom& g = tg.g;
  const TileId id = tile_id(tg);
  const int lx = threadIdx.x % ETX, ly = threadIdx.x / ETX;
  const int x2 = id.ox + lx, x1 = id.oy + ly;
  const bool colv = (x2 < g.d2) && (x1 < g.d1);
  const size_t off = static_cast<size_t>(id.s) * 3 * g.V;
  const float* f = src + off;
  int mn0 = INT_MAX, mn1 = INT_MAX, mn2 = INT_MAX, mx0 = INT_MIN, mx1 = INT_MIN, mx2 = INT_MIN;
#pragma unroll 2
  for (int k = 0; k < ETZ; ++k) {
    const int x0 = id.oz + k;
    if (colv && x0 < g.d0) {
      const int lin = (x0 * g.d1 + x1) * g.d2 + x2;
      float u0 = f[lin], u1 = f[g.V + lin], u2 = f[2 * g.V + lin];
      if (FIRST) {
        u0 *= scale;
        u1 *= scale;
        u2 *= scale;
      }
      const BorderCell bc = border_cell(g, x0, x1, x2, u0, u1, u2);
      if (MODE != 2) {
        float c[8];
        corners_border(f, g, bc.base, c);
        float s0 = tri_value(c, bc.t0, bc.t1, bc.t2);
        corners_border(f + g.V, g, bc.base, c);
        float s1 = tri_value(c, bc.t0, bc.t1, bc.t2);
        corners_border(f + 2 * g.V, g, bc.base, c);
        float s2 = tri_value(c, bc.t0, bc.t1, bc.t2);
        if (FIRST) {
          s0 *= scale;
          s1 *= scale;
          s2 *= scale;
        }
        float* o = dst + off;
        o[lin] = u0 + s0;
        o[g.V + lin] = u1 + s1;
        o[2 * g.V + lin] = u2 + s2;
      }
      if (MODE != 0) {
        mn0 = min(mn0, bc.i0 - x0);
        mn1 = min(mn1, bc.i1 - x1);
        mn2 = min(mn2, bc.i2 - x2);
        mx0 = max(mx0, bc.i0 - x0);
        mx1 = max(mx1, bc.i1 - x1);
        mx2 = max(mx2, bc.i2 - x2);
      }
    }
  }
  if (MODE != 0) {
    mn0 = wave_min(mn0);
    mn1 = wave_min(mn1);
    mn2 = wave_min(mn2);
    mx0 = wave_max(mx0);
    mx1 = wave_max(mx1);
    mx2 = wave_max(mx2);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
      red[0][w] = mn0;
      red[1][w] = mn1;
      red[2][w] = mn2;
      red[3][w] = mx0;
      red[4][w] = mx1;
      red[5][w] = mx2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int i = 1; i < ENT / 64; ++i) {
        red[0][0] = min(red[0][0], red[0][i]);
        red[1][0] = min(red[1][0], red[1][i]);
        red[2][0] = min(red[2][0], red[2][i]);
        red[3][0] = max(red[3][0], red[3][i]);
        red[4][0] = max(red[4][0], red[4][i]);
        red[5][0] = max(red[5][0], red[5][i]);
      }
      int* bx = boxes + (static_cast<size_t>(id.s) * tg.ntiles + id.tile) * 8;
      int* rc = reach + id.s * 8;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        bx[d] = red[d][0];
        bx[3 + d] = red[3 + d][0];
        atomicMax(rc + d, max(0, -red[d][0]));
        atomicMax(rc + 3 + d, max(0, red[3 + d][0] + 1));
      }
    }
  }
}

// Adjoint tiles: 4 (d0) x 4 (d1) x 32 (d2) output voxels, two per thread.
constexpr int BTX = 32, BTY = 4, BTZ = 4;
constexpr int BNT = 256;
constexpr int BTILE = BTX * BTY * BTZ;
// cells whose trilinear corners can land in the tile: base index in [O-1, L]
constexpr int CX = BTX + 1, CY = BTY + 1, CZ = BTZ + 1;
constexpr int NCELL = CX * CY * CZ;
constexpr int KSLOT = 2;  // sources kept per cell; further ones take the atomic path

struct BwdGeom {
  TileGeom src;    // tiling of the forward step (its per-tile offsets)
  int ntx, nty, ntz, ntiles;
  uint32_t total;  // adjoint tiles * subjects
};

// Adjoint of one squaring step for one output tile; gout is overwritten.
//
// 1. Each thread keeps the direct term g + J^T g of its two voxels in registers.
// 2. Every source voxel whose cell lies in the tile's cell region takes a slot
//    of that cell (one LDS integer atomic) and stores its fractions and g
//    there; sources beyond KSLOT per cell add their corner contributions to an
//    overflow accumulator with LDS float atomics instead (strong compression
//    only).
// 3. Each thread gathers, for each of its voxels y and each corner offset k,
//    the sources stored in cell y - k with weight w_k.
template <bool FIRST>
__global__ __launch_bounds__(BNT) void k_exp_bwd(const float* __restrict__ ut,
                                                 const float* __restrict__ gin,
                                                 float* __restrict__ gout, BwdGeom bg,
                                                 float scale, float oscale,
                                                 const int* __restrict__ boxes,
                                                 const int* __restrict__ reach) {
  __shared__ int cnt[NCELL];
  __shared__ float sdat[KSLOT][6][NCELL];
  __shared__ float ovf[3][BTILE];
  const TileGeom& tg = bg.src;
  const Geom& g = tg.g;
  const uint32_t bid = xcd_remap(blockIdx.x, bg.total);
  const int s = static_cast<int>(bid / bg.ntiles);
  const int tile = static_cast<int>(bid - static_cast<uint32_t>(s) * bg.ntiles);
  const int ox = (tile % bg.ntx) * BTX;
  const int oy = ((tile / bg.ntx) % bg.nty) * BTY;
  const int oz = (tile / (bg.ntx * bg.nty)) * BTZ;
  const int L0 = min(oz + BTZ, g.d0) - 1;
  const int L1 = min(oy + BTY, g.d1) - 1;
  const int L2 = min(ox + BTX, g.d2) - 1;
  const int lx = threadIdx.x % BTX, ly = (threadIdx.x / BTX) % BTY, lz = threadIdx.x / (BTX * BTY);
  const size_t off = static_cast<size_t>(s) * 3 * g.V;
  const float* f = ut + off;
  const float* gi = gin + off;
  const float js = FIRST ? scale : 1.0f;

  for (int i = threadIdx.x; i < NCELL; i += BNT) cnt[i] = 0;
  for (int i = threadIdx.x; i < 3 * BTILE; i += BNT) (&ovf[0][0])[i] = 0.0f;

  // 1. direct term of the two voxels (z = 2 lz, 2 lz + 1) this thread owns
  float acc[2][3];
  const int y1 = oy + ly, y2 = ox + lx;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int y0 = oz + 2 * lz + k;
    acc[k][0] = acc[k][1] = acc[k][2] = 0.0f;
    if (y0 < g.d0 && y1 < g.d1 && y2 < g.d2) {
      const int lin = (y0 * g.d1 + y1) * g.d2 + y2;
      float u0 = f[lin], u1 = f[g.V + lin], u2 = f[2 * g.V + lin];
      if (FIRST) {
        u0 *= scale;
        u1 *= scale;
        u2 *= scale;
      }
      const BorderCell bc = border_cell(g, y0, y1, y2, u0, u1, u2);
      const float gc[3] = {gi[lin], gi[g.V + lin], gi[2 * g.V + lin]};
      float jt0 = 0.0f, jt1 = 0.0f, jt2 = 0.0f;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float cv[8];
        corners_border(f + c * g.V, g, bc.base, cv);
        const Tri t = tri_eval(cv, bc.t0, bc.t1, bc.t2);
        jt0 += t.d0 * gc[c];
        jt1 += t.d1 * gc[c];
        jt2 += t.d2 * gc[c];
      }
      acc[k][0] = gc[0] + (bc.k0 ? 0.0f : jt0 * js);
      acc[k][1] = gc[1] + (bc.k1 ? 0.0f : jt1 * js);
      acc[k][2] = gc[2] + (bc.k2 ? 0.0f : jt2 * js);
    }
  }
  __syncthreads();

  // 2. bin the source voxels whose cell base lies in [O - 1, L]: a source x of
  //    forward tile s has cell base in x + [min, max] (recorded offsets), so
  //    only x_d in [O_d - 1 - max_d, L_d - min_d] qualify.  Candidate forward
  //    tiles come from the subject-wide reach.
  const int* rc = reach + s * 8;
  const int lo0 = max(0, oz - rc[3]) / ETZ, hi0 = min(tg.ntz - 1, (L0 + rc[0]) / ETZ);
  const int lo1 = max(0, oy - rc[4]) / ETY, hi1 = min(tg.nty - 1, (L1 + rc[1]) / ETY);
  const int lo2 = max(0, ox - rc[5]) / ETX, hi2 = min(tg.ntx - 1, (L2 + rc[2]) / ETX);
  const int* sbox = boxes + static_cast<size_t>(s) * tg.ntiles * 8;
  for (int sz = lo0; sz <= hi0; ++sz) {
    for (int sy = lo1; sy <= hi1; ++sy) {
      for (int sx = lo2; sx <= hi2; ++sx) {
        const int* bx = sbox + ((sz * tg.nty + sy) * tg.ntx + sx) * 8;
        const int a0 = max(sz * ETZ, oz - 1 - bx[3]);
        const int b0 = min(min(sz * ETZ + ETZ, g.d0) - 1, L0 - bx[0]);
        const int a1 = max(sy * ETY, oy - 1 - bx[4]);
        const int b1 = min(min(sy * ETY + ETY, g.d1) - 1, L1 - bx[1]);
        const int a2 = max(sx * ETX, ox - 1 - bx[5]);
        const int b2 = min(min(sx * ETX + ETX, g.d2) - 1, L2 - bx[2]);
        if (a0 > b0 || a1 > b1 || a2 > b2) continue;
        const int e2 = b2 - a2 + 1, e1 = b1 - a1 + 1;
        const int nvox = (b0 - a0 + 1) * e1 * e2;
        for (int q = threadIdx.x; q < nvox; q += BNT) {
          const int r = q / e2;
          const int x2 = a2 + (q - r * e2);
          const int r1 = r / e1;
          const int x1 = a1 + (r - r1 * e1);
          const int x0 = a0 + r1;
          const int lin = (x0 * g.d1 + x1) * g.d2 + x2;
          float u0 = f[lin], u1 = f[g.V + lin], u2 = f[2 * g.V + lin];
          if (FIRST) {
            u0 *= scale;
            u1 *= scale;
            u2 *= scale;
          }
          const BorderCell bc = border_cell(g, x0, x1, x2, u0, u1, u2);
          // local cell index: base - (O - 1), in [0, C)
          const int c0 = bc.i0 - oz + 1, c1 = bc.i1 - oy + 1, c2 = bc.i2 - ox + 1;
          if (c0 < 0 || c0 >= CZ || c1 < 0 || c1 >= CY || c2 < 0 || c2 >= CX) continue;
          const int ci = (c0 * CY + c1) * CX + c2;
          const float g0 = gi[lin], g1 = gi[g.V + lin], g2 = gi[2 * g.V + lin];
          const int slot = atomicAdd(&cnt[ci], 1);
          if (slot < KSLOT) {
            sdat[slot][0][ci] = bc.t0;
            sdat[slot][1][ci] = bc.t1;
            sdat[slot][2][ci] = bc.t2;
            sdat[slot][3][ci] = g0;
            sdat[slot][4][ci] = g1;
            sdat[slot][5][ci] = g2;
          } else {
            const float w0[2] = {1.0f - bc.t0, bc.t0};
            const float w1[2] = {1.0f - bc.t1, bc.t1};
            const float w2[2] = {1.0f - bc.t2, bc.t2};
#pragma unroll
            for (int a = 0; a < 2; ++a) {
#pragma unroll
              for (int b = 0; b < 2; ++b) {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                  // corner (c + k) - 1 in tile-local coordinates
                  const int q0 = c0 + a - 1, q1 = c1 + b - 1, q2 = c2 + e - 1;
                  if (q0 >= 0 && q0 < BTZ && q1 >= 0 && q1 < BTY && q2 >= 0 && q2 < BTX) {
                    const float w = w0[a] * w1[b] * w2[e];
                    const int li = (q0 * BTY + q1) * BTX + q2;
                    atomicAdd(&ovf[0][li], w * g0);
                    atomicAdd(&ovf[1][li], w * g1);
                    atomicAdd(&ovf[2][li], w * g2);
                  }
                }
              }
            }
          }
        }
      }
    }
  }
  __syncthreads();

  // 3. gather: voxel y receives w_k(x) g(x) from every source x binned in
  //    cell y - k, k in {0,1}^3
  float* go = gout + off;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int z = 2 * lz + k;
    const int y0 = oz + z;
    if (!(y0 < g.d0 && y1 < g.d1 && y2 < g.d2)) continue;
    float r0 = acc[k][0], r1 = acc[k][1], r2 = acc[k][2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int ci = ((z + 1 - a) * CY + (ly + 1 - b)) * CX + (lx + 1 - e);
          const int nsrc = min(cnt[ci], KSLOT);
#pragma unroll
          for (int j = 0; j < KSLOT; ++j) {
            if (j < nsrc) {
              const float t0 = sdat[j][0][ci], t1 = sdat[j][1][ci], t2 = sdat[j][2][ci];
              const float w = (a ? t0 : 1.0f - t0) * (b ? t1 : 1.0f - t1) * (e ? t2 : 1.0f - t2);
              r0 += w * sdat[j][3][ci];
              r1 += w * sdat[j][4][ci];
              r2 += w * sdat[j][5][ci];
            }
          }
        }
      }
    }
    const int li = (z * BTY + ly) * BTX + lx;
    r0 += ovf[0][li];
    r1 += ovf[1][li];
    r2 += ovf[2][li];
    const int lin = (y0 * g.d1 + y1) * g.d2 + y2;
    go[lin] = r0 * oscale;
    go[g.V + lin] = r1 * oscale;
    go[2 * g.V + lin] = r2 * oscale;
  }
}

BwdGeom make_bwd(const TileGeom& tg, int n) {
  BwdGeom b;
  b.src = tg;
  b.ntx = (tg.g.d2 + BTX - 1) / BTX;
  b.nty = (tg.g.d1 + BTY - 1) / BTY;
  b.ntz = (tg.g.d0 + BTZ - 1) / BTZ;
  b.ntiles = b.ntx * b.nty * b.ntz;
  b.total = static_cast<uint32_t>(b.ntiles) * n;
  return b;
}

template <bool FIRST>
void launch_fwd(int mode, const float* src, float* dst, const TileGeom& tg, float scale, int* boxes,
                int* reach, hipStream_t st) {
  switch (mode) {
    case 0:
      hipLaunchKernelGGL((k_exp_fwd<FIRST, 0>), dim3(tg.total), dim3(ENT), 0, st, src, dst, tg,
                         scale, boxes, reach);
      break;
    case 1:
      hipLaunchKernelGGL((k_exp_fwd<FIRST, 1>), dim3(tg.total), dim3(ENT), 0, st, src, dst, tg,
                         scale, boxes, reach);
      break;
    default:
      hipLaunchKernelGGL((k_exp_fwd<FIRST, 2>), dim3(tg.total), dim3(ENT), 0, st, src, dst, tg,
                         scale, boxes, reach);
      break;
  }
}

struct AuxPtrs {
  int* boxes;  // [n_sq][n][ntiles][8]
  int* reach;  // [n_sq][n][8]
  size_t box_stride, reach_stride;
};

AuxPtrs aux_ptrs(int* aux, const TileGeom& tg, int n, int n_sq) {
  AuxPtrs a;
  a.box_stride = static_cast<size_t>(n) * tg.ntiles * 8;
  a.reach_stride = static_cast<size_t>(n) * 8;
  a.boxes = aux;
  a.reach = aux ? aux + a.box_stride * n_sq : nullptr;
  return a;
}

}  // namespace

size_t exp_aux_bytes(const Geom& g, int n, int n_sq) {
  const TileGeom tg = make_tiles(g, n);
  return (static_cast<size_t>(n) * tg.ntiles * 8 + static_cast<size_t>(n) * 8) * n_sq *
         sizeof(int);
}

void run_exp_fwd(const float* v, float* u, float* ckpt, float* tmp, int* aux, const Geom& g, int n,
                 int n_sq, hipStream_t st) {
  const size_t fs = static_cast<size_t>(n) * 3 * g.V;
  if (n_sq == 0) {
    prof_begin(st, KC_MISC);
    (void)hipMemcpyAsync(u, v, fs * sizeof(float), hipMemcpyDeviceToDevice, st);
    prof_end(st, KC_MISC);
    return;
  }
  const TileGeom tg = make_tiles(g, n);
  const AuxPtrs ap = aux_ptrs(aux, tg, n, n_sq);
  // the reaches are running maxima: start them at zero (all-zero bits)
  if (aux) launch_fill_f32(reinterpret_cast<float*>(ap.reach), static_cast<long long>(ap.reach_stride) * n_sq, 0.0f, st);
  const float scale = ldexpf(1.0f, -n_sq);
  const float* src = v;
  for (int t = 0; t < n_sq; ++t) {
    float* dst;
    if (t == n_sq - 1)
      dst = u;
    else if (ckpt)
      dst = ckpt + static_cast<size_t>(t) * fs;  // slot t holds u_{t+1}
    else
      dst = ((n_sq - 1 - t) % 2 == 0) ? u : tmp;  // ping-pong ending in u
    int* bx = aux ? ap.boxes + ap.box_stride * t : nullptr;
    int* rc = aux ? ap.reach + ap.reach_stride * t : nullptr;
    prof_begin(st, KC_EXP_FWD);
    if (t == 0)
      launch_fwd<true>(aux ? 1 : 0, src, dst, tg, scale, bx, rc, st);
    else
      launch_fwd<false>(aux ? 1 : 0, src, dst, tg, scale, bx, rc, st);
    prof_end(st, KC_EXP_FWD);
    src = dst;
  }
}

void run_exp_bwd(const float* v, const float* ckpt, const float* g_u, float* g_v, float* tmp_a,
                 float* tmp_b, int* aux, bool aux_ready, const Geom& g, int n, int n_sq,
                 hipStream_t st) {
  const size_t fs = static_cast<size_t>(n) * 3 * g.V;
  if (n_sq == 0) {
    prof_begin(st, KC_MISC);
    (void)hipMemcpyAsync(g_v, g_u, fs * sizeof(float), hipMemcpyDeviceToDevice, st);
    prof_end(st, KC_MISC);
    return;
  }
  const TileGeom tg = make_tiles(g, n);
  const BwdGeom bg = make_bwd(tg, n);
  const AuxPtrs ap = aux_ptrs(aux, tg, n, n_sq);
  const float scale = ldexpf(1.0f, -n_sq);
  if (!aux_ready) {
    launch_fill_f32(reinterpret_cast<float*>(ap.reach), static_cast<long long>(ap.reach_stride) * n_sq, 0.0f, st);
    for (int t = 0; t < n_sq; ++t) {
      const float* ut = (t == 0) ? v : ckpt + static_cast<size_t>(t - 1) * fs;
      prof_begin(st, KC_MISC);
      if (t == 0)
        launch_fwd<true>(2, ut, nullptr, tg, scale, ap.boxes, ap.reach, st);
      else
        launch_fwd<false>(2, ut, nullptr, tg, scale, ap.boxes + ap.box_stride * t,
                          ap.reach + ap.reach_stride * t, st);
      prof_end(st, KC_MISC);
    }
  }
  const float* gin = g_u;
  for (int t = n_sq - 1; t >= 0; --t) {
    float* gout = (t == 0) ? g_v : (((n_sq - 1 - t) % 2 == 0) ? tmp_a : tmp_b);
    const float* ut = (t == 0) ? v : ckpt + static_cast<size_t>(t - 1) * fs;
    const int* bx = ap.boxes + ap.box_stride * t;
    const int* rc = ap.reach + ap.reach_stride * t;
    prof_begin(st, KC_EXP_BWD);
    if (t == 0)
      hipLaunchKernelGGL((k_exp_bwd<true>), dim3(bg.total), dim3(BNT), 0, st, ut, gin, gout, bg,
                         scale, scale, bx, rc);
    else
      hipLaunchKernelGGL((k_exp_bwd<false>), dim3(bg.total), dim3(BNT), 0, st, ut, gin, gout, bg,
                         1.0f, 1.0f, bx, rc);
    prof_end(st, KC_EXP_BWD);
    gin = gout;
  }
}

}  // namespace darc
