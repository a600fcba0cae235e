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
#include "voxel_bodies.hpp"

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

// Minimum or maximum over the 64 lanes of a wave (every lane active), by DPP
// lane moves that need no LDS: shifts by 1, 2, 4 and 8 lanes within each
// 16-lane row (a lane with no source lane takes the identity) leave each
// row's extreme in its lane 15; broadcasting lane 15 into the next row and
// lane 31 into rows 2 and 3 folds the four rows into lane 63.
template <bool MAX>
__device__ __forceinline__ int wave_extreme(int x) {
  constexpr int kRowShr = 0x110, kBcast15 = 0x142, kBcast31 = 0x143;
  constexpr int id = MAX ? INT_MIN : INT_MAX;
  auto op = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
  x = op(x, __builtin_amdgcn_update_dpp(id, x, kRowShr + 1, 0xf, 0xf, false));
  x = op(x, __builtin_amdgcn_update_dpp(id, x, kRowShr + 2, 0xf, 0xf, false));
  x = op(x, __builtin_amdgcn_update_dpp(id, x, kRowShr + 4, 0xf, 0xf, false));
  x = op(x, __builtin_amdgcn_update_dpp(id, x, kRowShr + 8, 0xf, 0xf, false));
  x = op(x, __builtin_amdgcn_update_dpp(id, x, kBcast15, 0xa, 0xf, false));
  x = op(x, __builtin_amdgcn_update_dpp(id, x, kBcast31, 0xc, 0xf, false));
  return __builtin_amdgcn_readlane(x, 63);
}
__device__ __forceinline__ int wave_min(int x) { return wave_extreme<false>(x); }
__device__ __forceinline__ int wave_max(int x) { return wave_extreme<true>(x); }

// Per-tile records used by the adjoint: boxes[(s * ntiles + tile) * 8 + {0,1,2}]
// = min over the tile's voxels x of i_d(x) - x_d along d0, d1, d2 (i = cell
// index of x + u(x)), [.. + {3,4,5}] = the max; so the corners a voxel x
// touches lie in x + [min, max + 1].  reach[s * 8 + d] = max(0, -min over tiles
// of the min offset) and reach[s * 8 + 3 + d] = max(0, max over tiles of the
// max offset + 1): how far below / above itself any voxel of the subject can
// scatter (zeroed before).  Tiles are 32 (d2) x 8 (d1) x 8 (d0).
__device__ __forceinline__ void write_record(int mn0, int mn1, int mn2, int mx0, int mx1, int mx2,
                                             int (*red)[ENT / 64], int* __restrict__ boxes,
                                             int s, int tile, int ntiles, int& rmax) {
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
  // thread q < 6 writes entry q of the box and folds its reach into a running
  // maximum (flush_reach issues it once per block): nothing here waits for
  // memory, and no barrier follows, since `red` is rewritten only after the
  // caller's next barrier
  if (threadIdx.x < 6) {
    const int q = threadIdx.x;
    int r = red[q][0];
#pragma unroll
    for (int i = 1; i < ENT / 64; ++i) r = q < 3 ? min(r, red[q][i]) : max(r, red[q][i]);
    boxes[(static_cast<size_t>(s) * ntiles + tile) * 8 + q] = r;
    rmax = max(rmax, q < 3 ? -r : r + 1);
  }
}

// The block's reaches into the subject's (atomics only where they can raise
// it): thread q < 6 holds entry q.
__device__ __forceinline__ void flush_reach(int rmax, int* __restrict__ reach, int s) {
  if (threadIdx.x < 6 && rmax > 0) atomicMax(reach + s * 8 + threadIdx.x, rmax);
}

// Records only (for an adjoint whose forward pass did not record them).
template <bool FIRST>
__global__ __launch_bounds__(ENT) void k_exp_rec(const float* __restrict__ src, TileGeom tg,
                                                 float scale, int* __restrict__ boxes,
                                                 int* __restrict__ reach) {
  __shared__ int red[6][ENT / 64];
  const Geom& g = tg.g;
  const TileId id = tile_id(tg);
  const int lx = threadIdx.x % ETX, ly = threadIdx.x / ETX;
  const int x2 = id.ox + lx, x1 = id.oy + ly;
  const bool colv = (x2 < g.d2) && (x1 < g.d1);
  const float* f = src + static_cast<size_t>(id.s) * 3 * g.V;
  int mn0 = INT_MAX, mn1 = INT_MAX, mn2 = INT_MAX, mx0 = INT_MIN, mx1 = INT_MIN, mx2 = INT_MIN;
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
      mn0 = min(mn0, bc.i0 - x0);
      mn1 = min(mn1, bc.i1 - x1);
      mn2 = min(mn2, bc.i2 - x2);
      mx0 = max(mx0, bc.i0 - x0);
      mx1 = max(mx1, bc.i1 - x1);
      mx2 = max(mx2, bc.i2 - x2);
    }
  }
  int rmax = 0;
  write_record(mn0, mn1, mn2, mx0, mx1, mx2, red, boxes, id.s, id.tile, tg.ntiles, rmax);
  flush_reach(rmax, reach, id.s);
}

// ---------------------------------------------------------------------------
// Marching kernels: a block owns a 32 x 8 column of the (d1, d2) plane and
// walks a chunk of planes along d0.  A ring of the last planes of u (and g)
// with a one-voxel halo in d1 and d2 lives in LDS; the next plane is loaded
// into registers while the current one is computed, so every value is read
// from memory once and loads overlap compute.
constexpr int MHX = ETX + 2, MHY = ETY + 2;  // staged plane with halo
constexpr int MHP = MHX * MHY;               // 340 positions
constexpr int MNJ = (MHP + ENT - 1) / ENT;   // positions per thread (2)

struct MarchGeom {
  TileGeom rec;  // record tiling (same 32 x 8 columns, 8 planes per record)
  int nzc, tz;   // chunks along d0 and their length (a multiple of ETZ)
  uint32_t total;
};

MarchGeom make_march(const TileGeom& tg, int n, int tz) {
  MarchGeom m;
  m.rec = tg;
  m.tz = tz;
  m.nzc = (tg.g.d0 + tz - 1) / tz;
  m.total = static_cast<uint32_t>(tg.ntx) * tg.nty * m.nzc * n;
  return m;
}

struct MarchId {
  int s, tx, ty, ox, oy, z0, z1;
};

__device__ __forceinline__ MarchId march_id_at(const MarchGeom& m, uint32_t b) {
  MarchId id;
  id.tx = static_cast<int>(b % m.rec.ntx);
  b /= m.rec.ntx;
  id.ty = static_cast<int>(b % m.rec.nty);
  b /= m.rec.nty;
  const int zc = static_cast<int>(b % m.nzc);
  id.s = static_cast<int>(b / m.nzc);
  id.ox = id.tx * ETX;
  id.oy = id.ty * ETY;
  id.z0 = zc * m.tz;
  id.z1 = min(id.z0 + m.tz, m.rec.g.d0);
  return id;
}

__device__ __forceinline__ MarchId march_id(const MarchGeom& m) {
  return march_id_at(m, xcd_remap(blockIdx.x, m.total));
}

// Halo positions of one plane handled by this thread: in-plane offset of the
// (clamped) voxel, and whether the unclamped voxel exists.
struct HaloPos {
  int off[MNJ];
  bool use[MNJ];     // position index < MHP
  bool inside[MNJ];  // the voxel is inside the volume (d1, d2)
  int y[MNJ], x[MNJ];
};

__device__ __forceinline__ HaloPos halo_pos(const Geom& g, int oy, int ox) {
  HaloPos h;
#pragma unroll
  for (int j = 0; j < MNJ; ++j) {
    const int e = threadIdx.x + j * ENT;
    h.use[j] = e < MHP;
    const int hy = e / MHX, hx = e - hy * MHX;
    const int y = oy - 1 + hy, x = ox - 1 + hx;
    h.y[j] = y;
    h.x[j] = x;
    h.inside[j] = y >= 0 && y < g.d1 && x >= 0 && x < g.d2;
    h.off[j] = min(max(y, 0), g.d1 - 1) * g.d2 + min(max(x, 0), g.d2 - 1);
  }
  return h;
}

// Forward squaring step, marching.  REC: also write the per-tile records.
template <bool FIRST, bool REC>
__global__ __launch_bounds__(ENT) void k_exp_fwd(const float* __restrict__ src,
                                                 float* __restrict__ dst, MarchGeom m,
                                                 float scale, int* __restrict__ boxes,
                                                 int* __restrict__ reach) {
  __shared__ float ring[3][3][MHP];  // [plane slot][component][position]
  __shared__ int red[6][ENT / 64];
  const Geom& g = m.rec.g;
  const MarchId id = march_id(m);
  const size_t off = static_cast<size_t>(id.s) * 3 * g.V;
  const float* f = src + off;
  float* o = dst + off;
  const int lx = threadIdx.x % ETX, ly = threadIdx.x / ETX;
  const HaloPos hp = halo_pos(g, id.oy, id.ox);
  // the next plane in registers (planes past the chunk are loaded clamped)
  const float* fc[3] = {f, f + g.V, f + 2 * static_cast<size_t>(g.V)};
  float pre[MNJ][3];
  auto load_plane = [&](int z) {
    const int zc = min(max(z, 0), g.d0 - 1);
#pragma unroll
    for (int j = 0; j < MNJ; ++j)
      if (hp.use[j]) {
        const uint32_t lin = static_cast<uint32_t>(zc * g.plane + hp.off[j]);
#pragma unroll
        for (int c = 0; c < 3; ++c) pre[j][c] = ld_at(fc[c], lin);
      }
  };
  auto store_plane = [&](int z) {
    const int sl = (z + 3) % 3;
#pragma unroll
    for (int j = 0; j < MNJ; ++j)
      if (hp.use[j]) {
        const int e = threadIdx.x + j * ENT;
        ring[sl][0][e] = pre[j][0];
        ring[sl][1][e] = pre[j][1];
        ring[sl][2][e] = pre[j][2];
      }
  };
  load_plane(id.z0 - 1);
  store_plane(id.z0 - 1);
  load_plane(id.z0);
  store_plane(id.z0);
  load_plane(id.z0 + 1);
  const int x2 = id.ox + lx, x1 = id.oy + ly;
  const bool colv = (x2 < g.d2) && (x1 < g.d1);
  const int own = (ly + 1) * MHX + lx + 1;
  int mn0 = INT_MAX, mn1 = INT_MAX, mn2 = INT_MAX, mx0 = INT_MIN, mx1 = INT_MIN, mx2 = INT_MIN;
  int rmax = 0;
  for (int z = id.z0; z < id.z1; ++z) {
    store_plane(z + 1);
    __syncthreads();
    load_plane(z + 2);
    if (colv) {
      const int sz = z % 3;
      float u0 = ring[sz][0][own], u1 = ring[sz][1][own], u2 = ring[sz][2][own];
      if (FIRST) {
        u0 *= scale;
        u1 *= scale;
        u2 *= scale;
      }
      const BorderCell bc = border_cell(g, z, x1, x2, u0, u1, u2);
      const int c0 = bc.i0 - z + 1, c1 = bc.i1 - id.oy + 1, c2 = bc.i2 - id.ox + 1;
      float r[3];
      if (c0 >= 0 && c0 <= 1 && c1 >= 0 && c1 + 1 < MHY && c2 >= 0 && c2 + 1 < MHX) {
        // ring slots of planes i0 and i0 + 1, i0 in {z - 1, z}: uniform choices
        const int sa = c0 ? sz : (z + 2) % 3, sb = c0 ? (z + 1) % 3 : sz;
        const int pb = c1 * MHX + c2;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          float cv[8];
          cv[0] = ring[sa][c][pb];
          cv[1] = ring[sa][c][pb + 1];
          cv[2] = ring[sa][c][pb + MHX];
          cv[3] = ring[sa][c][pb + MHX + 1];
          cv[4] = ring[sb][c][pb];
          cv[5] = ring[sb][c][pb + 1];
          cv[6] = ring[sb][c][pb + MHX];
          cv[7] = ring[sb][c][pb + MHX + 1];
          r[c] = tri_value(cv, bc.t0, bc.t1, bc.t2);
        }
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          float cv[8];
          corners_border(fc[c], g, bc.base, cv);
          r[c] = tri_value(cv, bc.t0, bc.t1, bc.t2);
        }
      }
      if (FIRST) {
        r[0] *= scale;
        r[1] *= scale;
        r[2] *= scale;
      }
      const uint32_t lin = static_cast<uint32_t>(z * g.plane + x1 * g.d2 + x2);
      st_at(o, lin, u0 + r[0]);
      st_at(o + g.V, lin, u1 + r[1]);
      st_at(o + 2 * static_cast<size_t>(g.V), lin, u2 + r[2]);
      if (REC) {
        mn0 = min(mn0, bc.i0 - z);
        mn1 = min(mn1, bc.i1 - x1);
        mn2 = min(mn2, bc.i2 - x2);
        mx0 = max(mx0, bc.i0 - z);
        mx1 = max(mx1, bc.i1 - x1);
        mx2 = max(mx2, bc.i2 - x2);
      }
    }
    if (REC && ((z + 1) % ETZ == 0 || z + 1 == id.z1)) {
      const int tile = ((z / ETZ) * m.rec.nty + id.ty) * m.rec.ntx + id.tx;
      write_record(mn0, mn1, mn2, mx0, mx1, mx2, red, boxes, id.s, tile, m.rec.ntiles, rmax);
      mn0 = mn1 = mn2 = INT_MAX;
      mx0 = mx1 = mx2 = INT_MIN;
    } else {
      __syncthreads();
    }
  }
  if (REC) flush_reach(rmax, reach, id.s);
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
// LDS of the tiled adjoint.
struct TiledBwdLds {
  int cnt[NCELL];
  float4 sdat4[KSLOT][NCELL];  // t0, t1, t2, g0 of a binned source
  float2 sdat2[KSLOT][NCELL];  // g1, g2
  float ovf[3][BTILE];
  int ubox[6];  // union of the candidate source sub-boxes
};

// Blocks blk of nblk walk the adjoint tiles; ALL: every subject, otherwise
// only those with a reach beyond 1 (the marching kernel takes the others).
template <bool FIRST, bool ALL>
__device__ __forceinline__ void exp_bwd_tiled_body(TiledBwdLds& L, uint32_t blk, uint32_t nblk,
                                                   const float* __restrict__ ut,
                                                   const float* __restrict__ gin,
                                                   float* __restrict__ gout, const BwdGeom& bg,
                                                   float scale, float oscale,
                                                   const int* __restrict__ boxes,
                                                   const int* __restrict__ reach) {
  const TileGeom& tg = bg.src;
  const Geom& g = tg.g;
  // persistent: each block walks a contiguous run of tiles (runs of
  // neighbouring blocks sit on the same XCD)
  const uint32_t run = (bg.total + nblk - 1) / nblk;
  const uint32_t first = xcd_remap(blk, nblk) * run;
  for (uint32_t bid = first; bid < min(first + run, bg.total); ++bid) {
  const int s = static_cast<int>(bid / bg.ntiles);
  const int tile = static_cast<int>(bid - static_cast<uint32_t>(s) * bg.ntiles);
  const int ox = (tile % bg.ntx) * BTX;
  const int oy = ((tile / bg.ntx) % bg.nty) * BTY;
  const int oz = (tile / (bg.ntx * bg.nty)) * BTZ;
  const int L0 = min(oz + BTZ, g.d0) - 1;
  const int L1 = min(oy + BTY, g.d1) - 1;
  const int L2 = min(ox + BTX, g.d2) - 1;
  const int lx = threadIdx.x % BTX, ly = (threadIdx.x / BTX) % BTY, lz = threadIdx.x / (BTX * BTY);
  {
    // subjects with reach 2 or less everywhere are handled by the marching
    // kernels: skip the rest of this subject's tiles
    const int* rc = reach + s * 8;
    if (!ALL && rc[0] <= 2 && rc[1] <= 2 && rc[2] <= 2 && rc[3] <= 2 && rc[4] <= 2 &&
        rc[5] <= 2) {
      bid = static_cast<uint32_t>(s + 1) * bg.ntiles - 1;
      continue;
    }
  }
  const size_t off = static_cast<size_t>(s) * 3 * g.V;
  const float* f = ut + off;
  const float* gi = gin + off;
  const float js = FIRST ? scale : 1.0f;

  for (int i = threadIdx.x; i < NCELL; i += BNT) L.cnt[i] = 0;
  for (int i = threadIdx.x; i < 3 * BTILE; i += BNT) (&L.ovf[0][0])[i] = 0.0f;
  if (threadIdx.x < 6) L.ubox[threadIdx.x] = threadIdx.x < 3 ? INT_MAX : INT_MIN;

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

  // 2. bin the source voxels whose cell base lies in [O - 1, L].  A source x
  //    of forward tile s has its cell base in x + [min, max] (the recorded
  //    offsets), so only x_d in [O_d - 1 - max_d, L_d - min_d] can qualify;
  //    candidate forward tiles come from the subject-wide reach.  The union
  //    box of those sub-boxes is swept as one flattened range, four sources
  //    per thread at a time with all their loads issued before any is used.
  const int* rc = reach + s * 8;
  const int lo0 = max(0, oz - rc[3]) / ETZ, hi0 = min(tg.ntz - 1, (L0 + rc[0]) / ETZ);
  const int lo1 = max(0, oy - rc[4]) / ETY, hi1 = min(tg.nty - 1, (L1 + rc[1]) / ETY);
  const int lo2 = max(0, ox - rc[5]) / ETX, hi2 = min(tg.ntx - 1, (L2 + rc[2]) / ETX);
  const int* sbox = boxes + static_cast<size_t>(s) * tg.ntiles * 8;
  {
    const int nc2 = hi2 - lo2 + 1, nc1 = hi1 - lo1 + 1;
    const int ncand = (hi0 - lo0 + 1) * nc1 * nc2;
    for (int ic = threadIdx.x; ic < ncand; ic += BNT) {
      const int sx = lo2 + ic % nc2;
      const int rr = ic / nc2;
      const int sy = lo1 + rr % nc1;
      const int sz = lo0 + rr / nc1;
      const int* bx = sbox + ((sz * tg.nty + sy) * tg.ntx + sx) * 8;
      const int a0 = max(sz * ETZ, oz - 1 - bx[3]);
      const int b0 = min(min(sz * ETZ + ETZ, g.d0) - 1, L0 - bx[0]);
      const int a1 = max(sy * ETY, oy - 1 - bx[4]);
      const int b1 = min(min(sy * ETY + ETY, g.d1) - 1, L1 - bx[1]);
      const int a2 = max(sx * ETX, ox - 1 - bx[5]);
      const int b2 = min(min(sx * ETX + ETX, g.d2) - 1, L2 - bx[2]);
      if (a0 <= b0 && a1 <= b1 && a2 <= b2) {
        atomicMin(&L.ubox[0], a0);
        atomicMin(&L.ubox[1], a1);
        atomicMin(&L.ubox[2], a2);
        atomicMax(&L.ubox[3], b0);
        atomicMax(&L.ubox[4], b1);
        atomicMax(&L.ubox[5], b2);
      }
    }
  }
  __syncthreads();
  const int ua0 = L.ubox[0], ua1 = L.ubox[1], ua2 = L.ubox[2];
  const int ub0 = L.ubox[3], ub1 = L.ubox[4], ub2 = L.ubox[5];
  if (ua0 <= ub0 && ua1 <= ub1 && ua2 <= ub2) {
    const int e2 = ub2 - ua2 + 1, e1 = ub1 - ua1 + 1;
    const int nvox = (ub0 - ua0 + 1) * e1 * e2;
    // q -> (x0, x1, x2) by reciprocal multiplication: for q < 2^23 the FP32
    // product is within one of the exact quotient and is corrected to it;
    // larger boxes use integer division
    const float inv2 = 1.0f / static_cast<float>(e2), inv1 = 1.0f / static_cast<float>(e1);
    const bool small = nvox < (1 << 23);
    for (int qb = 0; qb < nvox; qb += 4 * BNT) {
      float uu[4][3], gg[4][3];
      int xs[4][3];
      bool ok[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = qb + j * BNT + static_cast<int>(threadIdx.x);
        ok[j] = q < nvox;
        const int qq = ok[j] ? q : 0;
        int r, r1;
        if (small) {
          r = static_cast<int>((static_cast<float>(qq) + 0.5f) * inv2);
          r -= (r * e2 > qq);
          r += ((r + 1) * e2 <= qq);
          r1 = static_cast<int>((static_cast<float>(r) + 0.5f) * inv1);
          r1 -= (r1 * e1 > r);
          r1 += ((r1 + 1) * e1 <= r);
        } else {
          r = qq / e2;
          r1 = r / e1;
        }
        xs[j][2] = ua2 + (qq - r * e2);
        xs[j][1] = ua1 + (r - r1 * e1);
        xs[j][0] = ua0 + r1;
        const int lin = (xs[j][0] * g.d1 + xs[j][1]) * g.d2 + xs[j][2];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          uu[j][c] = f[c * g.V + lin];
          gg[j][c] = gi[c * g.V + lin];
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!ok[j]) continue;
        float u0 = uu[j][0], u1 = uu[j][1], u2 = uu[j][2];
        if (FIRST) {
          u0 *= scale;
          u1 *= scale;
          u2 *= scale;
        }
        const BorderCell bc = border_cell(g, xs[j][0], xs[j][1], xs[j][2], u0, u1, u2);
        // local cell index: base - (O - 1), in [0, C)
        const int c0 = bc.i0 - oz + 1, c1 = bc.i1 - oy + 1, c2 = bc.i2 - ox + 1;
        if (c0 < 0 || c0 >= CZ || c1 < 0 || c1 >= CY || c2 < 0 || c2 >= CX) continue;
        const int ci = (c0 * CY + c1) * CX + c2;
        const float g0 = gg[j][0], g1 = gg[j][1], g2 = gg[j][2];
        const int slot = atomicAdd(&L.cnt[ci], 1);
        if (slot < KSLOT) {
          L.sdat4[slot][ci] = make_float4(bc.t0, bc.t1, bc.t2, g0);
          L.sdat2[slot][ci] = make_float2(g1, g2);
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
                  atomicAdd(&L.ovf[0][li], w * g0);
                  atomicAdd(&L.ovf[1][li], w * g1);
                  atomicAdd(&L.ovf[2][li], w * g2);
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
          const int nsrc = min(L.cnt[ci], KSLOT);
#pragma unroll
          for (int j = 0; j < KSLOT; ++j) {
            if (j < nsrc) {
              const float4 p = L.sdat4[j][ci];
              const float2 q = L.sdat2[j][ci];
              const float w = corner_weight(a, b, e, p.x, p.y, p.z);
              r0 += w * p.w;
              r1 += w * q.x;
              r2 += w * q.y;
            }
          }
        }
      }
    }
    const int li = (z * BTY + ly) * BTX + lx;
    r0 += L.ovf[0][li];
    r1 += L.ovf[1][li];
    r2 += L.ovf[2][li];
    const int lin = (y0 * g.d1 + y1) * g.d2 + y2;
    go[lin] = r0 * oscale;
    go[g.V + lin] = r1 * oscale;
    go[2 * g.V + lin] = r2 * oscale;
  }
  __syncthreads();  // the next tile reuses the LDS bins
  }
}

template <bool FIRST, bool ALL>
__global__ __launch_bounds__(BNT) void k_exp_bwd(const float* __restrict__ ut,
                                                 const float* __restrict__ gin,
                                                 float* __restrict__ gout, BwdGeom bg,
                                                 float scale, float oscale,
                                                 const int* __restrict__ boxes,
                                                 const int* __restrict__ reach) {
  __shared__ TiledBwdLds L;
  exp_bwd_tiled_body<FIRST, ALL>(L, blockIdx.x, gridDim.x, ut, gin, gout, bg, scale, oscale,
                                 boxes, reach);
}

// Adjoint of one squaring step, marching, for a subject whose every cell
// offset lies in [-1, 0] (reach 1 in every direction: all |u_t| < 1, the
// case of the early sweeps and of the first squaring steps).  A source in
// plane p then falls in cell plane p-1 or p, and cell plane c feeds exactly
// target planes c (as corner a = 0 of its cells) and c + 1 (corner a = 1).
// So one cell plane is live at a time: iteration z fills cell plane z and one
// pass over it completes the targets of plane z (their a = 1 part came from
// cell plane z - 1 in the previous iteration) and starts those of plane
// z + 1, kept in registers.  Each slot read serves both targets, which share
// the in-plane weight; the block's LDS (one cell plane, two overflow planes,
// the u ring) stays near a quarter of the CU's.  Iteration z: (i) clear the
// cell plane and target plane z+1's overflow, stage u_t of plane z+1; (ii)
// cells of the plane-(z+1) sources; (iii) fill cell plane z with the plane-z
// sources whose cell is in it (cells kept from the last iteration) and the
// plane-(z+1) sources whose cell is in it (one LDS integer atomic each, two
// zero-initialised slots per cell, further sources into the overflow
// accumulator); (iv) the direct term g + J^T g of the plane-z targets; (v)
// the gather over the four cells around each column.  Thread (ly, lx) stages
// and bins its own voxel, so a voxel's cell and g stay in its registers from
// staging to its direct term; threads below 84 also stage one voxel of the
// one-voxel halo ring.  Blocks of subjects with a larger reach return at
// once: the tiled kernel handles those.
constexpr int MCX = ETX + 1, MCY = ETY + 1;  // cells per cell plane: 33 x 9
constexpr int MCP = MCX * MCY;
constexpr int MRING = MHP - ENT;             // halo ring positions (84)

template <bool FIRST>
__global__ __launch_bounds__(ENT, 4) void k_exp_bwd_march(const float* __restrict__ ut,
                                                          const float* __restrict__ gin,
                                                          float* __restrict__ gout, MarchGeom m,
                                                          float scale, float oscale,
                                                          const int* __restrict__ reach) {
  __shared__ float uring[3][3][MHP];  // u_t of planes z-1, z, z+1 (slot p % 3)
  __shared__ int bcnt[MCP];           // the live cell plane
  __shared__ float4 bd4[KSLOT][MCP];  // t0, t1, t2, g0 per binned source (0 if empty)
  __shared__ float2 bd2[KSLOT][MCP];  // g1, g2
  __shared__ float ovf[2][3][ENT];    // overflow into target planes, by parity
  const Geom& g = m.rec.g;
  const MarchId id = march_id(m);
  {
    const int* rc = reach + id.s * 8;
    if (rc[0] > 1 || rc[1] > 1 || rc[2] > 1 || rc[3] > 1 || rc[4] > 1 || rc[5] > 1) return;
  }
  const size_t off = static_cast<size_t>(id.s) * 3 * g.V;
  const float* f = ut + off;
  const float* gi = gin + off;
  float* go = gout + off;
  const int lx = threadIdx.x % ETX, ly = threadIdx.x / ETX;
  const float js = FIRST ? scale : 1.0f;

  // staged positions: j = 0 the thread's own voxel, j = 1 a halo-ring voxel
  int pe[2], py[2], px[2], poff[2];
  bool puse[2], pin[2];
  pe[0] = (ly + 1) * MHX + lx + 1;
  py[0] = id.oy + ly;
  px[0] = id.ox + lx;
  puse[0] = true;
  {
    const int r = threadIdx.x;
    int hy, hx;
    if (r < MHX) {
      hy = 0;
      hx = r;
    } else if (r < 2 * MHX) {
      hy = MHY - 1;
      hx = r - MHX;
    } else if (r < 2 * MHX + ETY) {
      hy = 1 + r - 2 * MHX;
      hx = 0;
    } else {
      hy = 1 + min(r - 2 * MHX - ETY, ETY - 1);
      hx = MHX - 1;
    }
    puse[1] = r < MRING;
    pe[1] = hy * MHX + hx;
    py[1] = id.oy - 1 + hy;
    px[1] = id.ox - 1 + hx;
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    pin[j] = py[j] >= 0 && py[j] < g.d1 && px[j] >= 0 && px[j] < g.d2;
    poff[j] = min(max(py[j], 0), g.d1 - 1) * g.d2 + min(max(px[j], 0), g.d2 - 1);
  }
  // lanes without a halo voxel load their own voxel again (a cache line the
  // wave reads anyway) rather than fetching rows of other tiles
  if (!puse[1]) poff[1] = poff[0];

  // component base pointers (uniform across the block)
  const float* fc[3] = {f, f + g.V, f + 2 * static_cast<size_t>(g.V)};
  const float* gc[3] = {gi, gi + g.V, gi + 2 * static_cast<size_t>(g.V)};
  // Planes in flight: two register buffers, loaded two planes ahead of use.
  // Every lane loads (lanes without a halo voxel from a clamped, valid
  // position) and planes past the chunk are loaded clamped too: a
  // conditional load would make the compiler merge register values right
  // after it and so wait for it at once.
  float pu[2][3], pg[2][3], pu2[2][3], pg2[2][3];
  auto load_plane = [&](int z, float (&lu)[2][3], float (&lg)[2][3]) {
    const int zc = min(max(z, 0), g.d0 - 1);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const uint32_t lin = static_cast<uint32_t>(zc * g.plane + poff[j]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        lu[j][c] = ld_at(fc[c], lin);
        lg[j][c] = ld_at(gc[c], lin);
      }
    }
  };
  auto store_u = [&](int z, const float (&su_)[2][3]) {
    const int su = (z + 3) % 3;
#pragma unroll
    for (int j = 0; j < 2; ++j)
      if (puse[j]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) uring[su][c][pe[j]] = su_[j][c];
      }
  };
  auto clear_cells = [&]() {
    const float4 z4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const float2 z2 = make_float2(0.0f, 0.0f);
    // threads in reverse order: the cells past ENT fall to the last wave,
    // which stages no halo voxels
    for (int i = ENT - 1 - static_cast<int>(threadIdx.x); i < MCP; i += ENT) {
      bcnt[i] = 0;
#pragma unroll
      for (int k = 0; k < KSLOT; ++k) {
        bd4[k][i] = z4;
        bd2[k][i] = z2;
      }
    }
  };
  auto clear_ovf = [&](int tplane) {
    float* o = &ovf[tplane & 1][0][0];
    for (int i = threadIdx.x; i < 3 * ENT; i += ENT) o[i] = 0.0f;
  };
  // cells of the staged sources of plane p (ok = a source inside the volume)
  auto cells_of = [&](int p, const float (&vu)[2][3], BorderCell (&bc)[2], bool (&ok)[2]) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      ok[j] = puse[j] && pin[j] && p >= 0 && p < g.d0;
      bc[j] = BorderCell{};
      // lanes without a halo voxel (all of waves 2 and 3) skip the halo cell
      if (puse[j]) {
        float u0 = vu[j][0], u1 = vu[j][1], u2 = vu[j][2];
        if (FIRST) {
          u0 *= scale;
          u1 *= scale;
          u2 *= scale;
        }
        bc[j] = border_cell(g, min(max(p, 0), g.d0 - 1), py[j], px[j], u0, u1, u2);
      }
    }
  };
  // Bin one source into the live cell plane (its plane bc.i0 is the one
  // being filled).  The cell of a tile voxel (halo = false) always lies in the
  // tile's cell region (offsets in [-1, 0], and border clamping keeps a cell
  // inside the volume); a halo voxel's cell may not.
  auto bin_one = [&](const BorderCell& bc, float g0, float g1, float g2, bool halo) {
    const int c1 = bc.i1 - id.oy + 1, c2 = bc.i2 - id.ox + 1;
    if (halo && (c1 < 0 || c1 >= MCY || c2 < 0 || c2 >= MCX)) return;
    const int ci = c1 * MCX + c2;
    const int slot = atomicAdd(&bcnt[ci], 1);
    if (slot < KSLOT) {
      bd4[slot][ci] = make_float4(bc.t0, bc.t1, bc.t2, g0);
      bd2[slot][ci] = make_float2(g1, g2);
    } else {
      const float w0[2] = {1.0f - bc.t0, bc.t0};
      const float w1[2] = {1.0f - bc.t1, bc.t1};
      const float w2[2] = {1.0f - bc.t2, bc.t2};
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int tz = bc.i0 + a;  // target plane
        if (tz < id.z0 || tz >= id.z1) continue;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
          for (int ee = 0; ee < 2; ++ee) {
            const int ty = c1 + b - 1, tx = c2 + ee - 1;
            if (ty >= 0 && ty < ETY && tx >= 0 && tx < ETX) {
              const float w = w0[a] * w1[b] * w2[ee];
              float* ov = &ovf[tz & 1][0][0] + ty * ETX + tx;
              atomicAdd(ov, w * g0);
              atomicAdd(ov + ENT, w * g1);
              atomicAdd(ov + 2 * ENT, w * g2);
            }
          }
        }
      }
    }
  };
  // One pass over the live cell plane: for each of the four cells around the
  // thread's column and each slot, w12 = the in-plane weight of the corner
  // (b, e); the target of the cell's lower plane (a = 0) takes w12 (1 - t0),
  // the one of its upper plane (a = 1) w12 t0.  Empty slots hold zeros.
  auto gather = [&](float (&lo)[3], float (&up)[3], bool upper) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int ci = (ly + 1 - b) * MCX + (lx + 1 - e);
#pragma unroll
        for (int j = 0; j < KSLOT; ++j) {
          const float4 p = bd4[j][ci];
          const float2 q = bd2[j][ci];
          const float w1 = b ? p.y : 1.0f - p.y;
          const float w12 = e ? w1 * p.z : fmaf(-w1, p.z, w1);
          const float wl = fmaf(-w12, p.x, w12);
          lo[0] += wl * p.w;
          lo[1] += wl * q.x;
          lo[2] += wl * q.y;
          if (upper) {
            const float wu = w12 * p.x;
            up[0] += wu * p.w;
            up[1] += wu * q.x;
            up[2] += wu * q.y;
          }
        }
      }
    }
  };

  const bool colv = pin[0];
  BorderCell cb[2], nb[2];  // cells of the plane-z and plane-(z+1) sources
  bool cok[2], nok[2];
  float cg[2][3], qu[2][3], qg[2][3];
  // targets of the next plane, partly gathered (their a = 1 part)
  float accA[3] = {0.0f, 0.0f, 0.0f}, accB[3] = {0.0f, 0.0f, 0.0f};

  // prologue: cell plane z0-1 from the sources of planes z0-1 and z0, and
  // its a = 1 part of the plane-z0 targets; planes z0+1 and z0+2 in flight
  clear_cells();
  clear_ovf(id.z0);
  load_plane(id.z0 - 1, pu, pg);
  store_u(id.z0 - 1, pu);
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      qu[j][c] = pu[j][c];
      qg[j][c] = pg[j][c];
    }
  load_plane(id.z0, pu, pg);
  store_u(id.z0, pu);
  __syncthreads();
  cells_of(id.z0 - 1, qu, nb, nok);
#pragma unroll
  for (int j = 0; j < 2; ++j)
    if (nok[j] && nb[j].i0 == id.z0 - 1) bin_one(nb[j], qg[j][0], qg[j][1], qg[j][2], j == 1);
  cells_of(id.z0, pu, cb, cok);
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (cok[j] && cb[j].i0 == id.z0 - 1) bin_one(cb[j], pg[j][0], pg[j][1], pg[j][2], j == 1);
#pragma unroll
    for (int c = 0; c < 3; ++c) cg[j][c] = pg[j][c];
  }
  load_plane(id.z0 + 1, pu, pg);
  load_plane(id.z0 + 2, pu2, pg2);
  __syncthreads();
  {
    float none[3] = {0.0f, 0.0f, 0.0f};
    if (colv) gather(none, accA, true);
  }
  __syncthreads();

  // one plane; (xu, xg) holds plane z+1 on entry and takes plane z+3; acc
  // holds the plane-z targets' a = 1 part and receives plane z+1's
  auto step = [&](int z, float (&xu)[2][3], float (&xg)[2][3], float (&acc)[3],
                  float (&nacc)[3]) {
    // (i) clear the cell plane (held z-1) and target plane z+1 (held z-1);
    //     stage u of plane z+1
    clear_cells();
    clear_ovf(z + 1);
    store_u(z + 1, xu);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        qu[j][c] = xu[j][c];
        qg[j][c] = xg[j][c];
      }
    __syncthreads();
    load_plane(z + 3, xu, xg);
    // (ii) cells of the plane-(z+1) sources
    cells_of(z + 1, qu, nb, nok);
    // (iii) fill cell plane z
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (cok[j] && cb[j].i0 == z) bin_one(cb[j], cg[j][0], cg[j][1], cg[j][2], j == 1);
      if (nok[j] && nb[j].i0 == z) bin_one(nb[j], qg[j][0], qg[j][1], qg[j][2], j == 1);
    }
    // (iv) direct term of the plane-z targets
    float r[3] = {acc[0], acc[1], acc[2]};
    const int szm = (z + 2) % 3, szc = z % 3, szp = (z + 1) % 3;  // slots of z-1, z, z+1
    if (colv) {
      const BorderCell& bc = cb[0];
      const int c0 = bc.i0 - z + 1, c1 = bc.i1 - id.oy + 1, c2 = bc.i2 - id.ox + 1;
      const bool in_ring =
          c0 >= 0 && c0 <= 1 && c1 >= 0 && c1 + 1 < MHY && c2 >= 0 && c2 + 1 < MHX;
      // J^T g = grad of the trilinear interpolant of g . u at the sample.
      // Corners come from the staged ring; a cell outside it (not reached
      // while every offset lies in [-1, 0]) reads them from memory.  The
      // memory path combines three derivative evaluations instead of forming
      // g . u at the corners first: its arithmetic then cannot be merged with
      // the ring path's after the branch, which would make the ring path
      // wait for memory loads (and with them for the planes in flight).
      Tri t;
      if (in_ring) {
        // ring slots of planes i0 and i0 + 1, i0 in {z - 1, z}: uniform choices
        const int sa = c0 ? szc : szm, sb = c0 ? szp : szc;
        const int pb = c1 * MHX + c2;
        float h[8];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float cv[8] = {uring[sa][c][pb],       uring[sa][c][pb + 1],
                               uring[sa][c][pb + MHX], uring[sa][c][pb + MHX + 1],
                               uring[sb][c][pb],       uring[sb][c][pb + 1],
                               uring[sb][c][pb + MHX], uring[sb][c][pb + MHX + 1]};
#pragma unroll
          for (int k = 0; k < 8; ++k) h[k] = c == 0 ? cg[0][0] * cv[k] : h[k] + cg[0][c] * cv[k];
        }
        t = tri_eval(h, bc.t0, bc.t1, bc.t2);
      } else {
        t.v = 0.0f;
        t.d0 = t.d1 = t.d2 = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          float cv[8];
          corners_border(fc[c], g, bc.base, cv);
          const Tri tc = tri_eval(cv, bc.t0, bc.t1, bc.t2);
          t.d0 += tc.d0 * cg[0][c];
          t.d1 += tc.d1 * cg[0][c];
          t.d2 += tc.d2 * cg[0][c];
        }
      }
      r[0] += cg[0][0] + (bc.k0 ? 0.0f : t.d0 * js);
      r[1] += cg[0][1] + (bc.k1 ? 0.0f : t.d1 * js);
      r[2] += cg[0][2] + (bc.k2 ? 0.0f : t.d2 * js);
    }
    __syncthreads();
    // (v) gather: finish the plane-z targets, start the plane-(z+1) ones
#pragma unroll
    for (int c = 0; c < 3; ++c) nacc[c] = 0.0f;
    if (colv) {
      gather(r, nacc, z + 1 < id.z1);
      const float* ov = &ovf[z & 1][0][0];
      r[0] += ov[threadIdx.x];
      r[1] += ov[ENT + threadIdx.x];
      r[2] += ov[2 * ENT + threadIdx.x];
      const uint32_t lin = static_cast<uint32_t>(z * g.plane + py[0] * g.d2 + px[0]);
      st_at(go, lin, r[0] * oscale);
      st_at(go + g.V, lin, r[1] * oscale);
      st_at(go + 2 * static_cast<size_t>(g.V), lin, r[2] * oscale);
    }
    // (vi) the plane-(z+1) sources become the next iteration's plane-z sources
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cb[j] = nb[j];
      cok[j] = nok[j];
#pragma unroll
      for (int c = 0; c < 3; ++c) cg[j][c] = qg[j][c];
    }
    __syncthreads();
  };
  // unrolled by two so that each prefetch buffer and partial keeps its registers
  for (int z = id.z0; z < id.z1; z += 2) {
    step(z, pu, pg, accA, accB);
    if (z + 1 < id.z1) step(z + 1, pu2, pg2, accB, accA);
  }
}

// Adjoint of one squaring step, marching, for a subject whose cell offsets
// lie in [-2, 1] on every axis and reach beyond [-1, 0] somewhere (reach 2:
// roughly 1 <= max |u_t| < 2, the later squaring steps of moderate
// deformations).  The reach-1 kernel's scheme with wider windows: a source
// of plane p falls in cell planes p-2 .. p+1, so cell plane z is filled from
// the sources of planes z-1 .. z+2, whose cells are computed once, when their
// plane is staged, and kept in registers for four iterations; sources up to
// two voxels outside the column can land in its cell region (a two-voxel halo
// ring of 176 positions, one for each of the first 176 threads); the direct
// term's corners lie in planes z-2 .. z+2 of the u ring.  Iteration z:
// (i) clear the cell plane and target plane z+1's overflow, stage u of plane
// z+2 and compute its sources' cells; (ii) bin the sources of planes
// z-1 .. z+2 whose cell lies in plane z; (iii) the direct term of the plane-z
// targets; (iv) the gather, finishing plane z and starting plane z+1.
// Blocks of subjects with reach 1 everywhere (the reach-1 kernel's) or
// beyond 2 (the tiled kernel's) return at once.
constexpr int H2X = ETX + 4, H2Y = ETY + 4;  // staged plane with a two-voxel halo: 36 x 12
constexpr int H2P = H2X * H2Y;               // 432 positions
constexpr int H2RING = H2P - ENT;            // 176 halo positions

// One source: its cell packed as r2 (6 bits: corner column in the staged
// plane), r1 (4 bits: corner row), o0 + 2 (2 bits: cell plane - source
// plane + 2), the three clamped flags and a valid bit (the source exists and
// its cell's corners lie in the staged plane); fractions and g.
struct Src2 {
  int key;
  float t0, t1, t2, g0, g1, g2;
};
constexpr int kSrcValid = 1 << 15;

template <bool FIRST>
__global__ __launch_bounds__(ENT, 3) void k_exp_bwd_march2(const float* __restrict__ ut,
                                                            const float* __restrict__ gin,
                                                            float* __restrict__ gout,
                                                            MarchGeom m, float scale,
                                                            float oscale,
                                                            const int* __restrict__ reach) {
  __shared__ float uring[5][3][H2P];  // u_t of planes z-2 .. z+2 (slot p % 5)
  __shared__ int bcnt[MCP];           // the live cell plane
  __shared__ float4 bd4[KSLOT][MCP];  // t0, t1, t2, g0 per binned source (0 if empty)
  __shared__ float2 bd2[KSLOT][MCP];  // g1, g2
  __shared__ float ovf[2][3][ENT];    // overflow into target planes, by parity
  const Geom& g = m.rec.g;
  {
    // nothing to do unless some subject of the launch has reach 2
    const int nsub = static_cast<int>(m.total / (static_cast<uint32_t>(m.rec.ntx) * m.rec.nty *
                                                  m.nzc));
    int mine = 0;
    for (int q = threadIdx.x; q < nsub; q += ENT) {
      const int* rc = reach + q * 8;
      mine |= max(max(max(rc[0], rc[1]), max(rc[2], rc[3])), max(rc[4], rc[5])) == 2;
    }
    if (!__syncthreads_or(mine)) return;
  }
  // persistent: the blocks (all resident) step through the column chunks
  // together, block v taking chunks v, v + grid, ..., so that the chunks in
  // flight at once are neighbours (and those of one XCD a contiguous range);
  // chunks of subjects that are not this kernel's are passed over
  for (uint32_t bid = xcd_remap(blockIdx.x, gridDim.x); bid < m.total; bid += gridDim.x) {
  const MarchId id = march_id_at(m, bid);
  {
    const int* rc = reach + id.s * 8;
    const int mr = max(max(max(rc[0], rc[1]), max(rc[2], rc[3])), max(rc[4], rc[5]));
    if (mr != 2) continue;
  }
  const size_t off = static_cast<size_t>(id.s) * 3 * g.V;
  const float* f = ut + off;
  const float* gi = gin + off;
  float* go = gout + off;
  const int lx = threadIdx.x % ETX, ly = threadIdx.x / ETX;
  const float js = FIRST ? scale : 1.0f;

  // staged positions: j = 0 the thread's own voxel, j = 1 a halo-ring voxel
  int pe[2], py[2], px[2], poff[2];
  bool puse[2], pin[2];
  pe[0] = (ly + 2) * H2X + lx + 2;
  py[0] = id.oy + ly;
  px[0] = id.ox + lx;
  puse[0] = true;
  {
    const int r = threadIdx.x;
    int hy, hx;
    if (r < 2 * H2X) {  // rows 0 and 1
      hy = r / H2X;
      hx = r - hy * H2X;
    } else if (r < 4 * H2X) {  // rows H2Y - 2 and H2Y - 1
      const int q = r - 2 * H2X;
      hy = H2Y - 2 + q / H2X;
      hx = q - (q / H2X) * H2X;
    } else {  // columns 0, 1, H2X - 2, H2X - 1 of rows 2 .. H2Y - 3
      const int q = min(r - 4 * H2X, 4 * ETY - 1);
      hy = 2 + q / 4;
      const int col = q % 4;
      hx = col < 2 ? col : H2X - 4 + col;
    }
    puse[1] = r < H2RING;
    pe[1] = hy * H2X + hx;
    py[1] = id.oy - 2 + hy;
    px[1] = id.ox - 2 + hx;
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    pin[j] = py[j] >= 0 && py[j] < g.d1 && px[j] >= 0 && px[j] < g.d2;
    poff[j] = min(max(py[j], 0), g.d1 - 1) * g.d2 + min(max(px[j], 0), g.d2 - 1);
  }
  if (!puse[1]) poff[1] = poff[0];

  const float* fc[3] = {f, f + g.V, f + 2 * static_cast<size_t>(g.V)};
  const float* gc[3] = {gi, gi + g.V, gi + 2 * static_cast<size_t>(g.V)};
  // the next plane to stage in flight (every lane loads, planes past the
  // volume clamped; a second buffer measured slower at this register count)
  float pu[2][3], pg[2][3];
  auto load_plane = [&](int z, float (&lu)[2][3], float (&lg)[2][3]) {
    const int zc = min(max(z, 0), g.d0 - 1);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const uint32_t lin = static_cast<uint32_t>(zc * g.plane + poff[j]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        lu[j][c] = ld_at(fc[c], lin);
        lg[j][c] = ld_at(gc[c], lin);
      }
    }
  };
  auto store_u = [&](int z, const float (&su_)[2][3]) {
    const int sl = (z + 10) % 5;
#pragma unroll
    for (int j = 0; j < 2; ++j)
      if (puse[j]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) uring[sl][c][pe[j]] = su_[j][c];
      }
  };
  auto clear_cells = [&]() {
    const float4 z4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const float2 z2 = make_float2(0.0f, 0.0f);
    for (int i = threadIdx.x; i < MCP; i += ENT) {
      bcnt[i] = 0;
#pragma unroll
      for (int k = 0; k < KSLOT; ++k) {
        bd4[k][i] = z4;
        bd2[k][i] = z2;
      }
    }
  };
  auto clear_ovf = [&](int tplane) {
    float* o = &ovf[tplane & 1][0][0];
    for (int i = threadIdx.x; i < 3 * ENT; i += ENT) o[i] = 0.0f;
  };
  // cells of the staged sources of plane p
  auto cells_of = [&](int p, const float (&vu)[2][3], const float (&vg)[2][3], Src2 (&S)[2]) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      S[j].key = 0;
      S[j].t0 = S[j].t1 = S[j].t2 = 0.0f;
      S[j].g0 = vg[j][0];
      S[j].g1 = vg[j][1];
      S[j].g2 = vg[j][2];
      if (puse[j]) {
        float u0 = vu[j][0], u1 = vu[j][1], u2 = vu[j][2];
        if (FIRST) {
          u0 *= scale;
          u1 *= scale;
          u2 *= scale;
        }
        const int pc = min(max(p, 0), g.d0 - 1);
        const BorderCell bc = border_cell(g, pc, py[j], px[j], u0, u1, u2);
        const int o0 = bc.i0 - pc, r1 = bc.i1 - id.oy + 2, r2 = bc.i2 - id.ox + 2;
        const bool ok = pin[j] && p >= 0 && p < g.d0 && o0 >= -2 && o0 <= 1 && r1 >= 0 &&
                        r1 + 1 < H2Y && r2 >= 0 && r2 + 1 < H2X;
        S[j].key = ok ? (r2 | (r1 << 6) | ((o0 + 2) << 10) | (static_cast<int>(bc.k0) << 12) |
                         (static_cast<int>(bc.k1) << 13) | (static_cast<int>(bc.k2) << 14) |
                         kSrcValid)
                      : 0;
        S[j].t0 = bc.t0;
        S[j].t1 = bc.t1;
        S[j].t2 = bc.t2;
      }
    }
  };
  // bin source s of plane p if its cell lies in cell plane cz and in the
  // column's cell region
  auto bin_one = [&](int cz, int p, const Src2& sv) {
    if (!(sv.key & kSrcValid)) return;
    if (p + ((sv.key >> 10) & 3) - 2 != cz) return;
    const int cy = ((sv.key >> 6) & 15) - 1, cx = (sv.key & 63) - 1;
    if (cy < 0 || cy >= MCY || cx < 0 || cx >= MCX) return;
    const int ci = cy * MCX + cx;
    const int slot = atomicAdd(&bcnt[ci], 1);
    if (slot < KSLOT) {
      bd4[slot][ci] = make_float4(sv.t0, sv.t1, sv.t2, sv.g0);
      bd2[slot][ci] = make_float2(sv.g1, sv.g2);
    } else {
      const float w0[2] = {1.0f - sv.t0, sv.t0};
      const float w1[2] = {1.0f - sv.t1, sv.t1};
      const float w2[2] = {1.0f - sv.t2, sv.t2};
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int tz = cz + a;  // target plane
        if (tz < id.z0 || tz >= id.z1) continue;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
          for (int ee = 0; ee < 2; ++ee) {
            const int ty = cy + b - 1, tx = cx + ee - 1;
            if (ty >= 0 && ty < ETY && tx >= 0 && tx < ETX) {
              const float w = w0[a] * w1[b] * w2[ee];
              float* ov = &ovf[tz & 1][0][0] + ty * ETX + tx;
              atomicAdd(ov, w * sv.g0);
              atomicAdd(ov + ENT, w * sv.g1);
              atomicAdd(ov + 2 * ENT, w * sv.g2);
            }
          }
        }
      }
    }
  };
  // one pass over the live cell plane (as in the reach-1 kernel)
  auto gather = [&](float (&lo)[3], float (&up)[3], bool upper) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int ci = (ly + 1 - b) * MCX + (lx + 1 - e);
#pragma unroll
        for (int j = 0; j < KSLOT; ++j) {
          const float4 q4 = bd4[j][ci];
          const float2 q2 = bd2[j][ci];
          const float w1 = b ? q4.y : 1.0f - q4.y;
          const float w12 = e ? w1 * q4.z : fmaf(-w1, q4.z, w1);
          const float wl = fmaf(-w12, q4.x, w12);
          lo[0] += wl * q4.w;
          lo[1] += wl * q2.x;
          lo[2] += wl * q2.y;
          if (upper) {
            const float wu = w12 * q4.x;
            up[0] += wu * q4.w;
            up[1] += wu * q2.x;
            up[2] += wu * q2.y;
          }
        }
      }
    }
  };

  const bool colv = pin[0];
  Src2 R0[2], R1[2], R2[2], R3[2];  // sources of four consecutive planes
  float accA[3] = {0.0f, 0.0f, 0.0f}, accB[3] = {0.0f, 0.0f, 0.0f};

  // prologue: planes z0-2 .. z0+1 staged with their cells (in R3, R0, R1,
  // R2), cell plane z0-1 filled, its a = 1 part of the plane-z0 targets;
  // plane z0+2 in flight
  clear_cells();
  clear_ovf(id.z0);
  load_plane(id.z0 - 2, pu, pg);
  store_u(id.z0 - 2, pu);
  cells_of(id.z0 - 2, pu, pg, R3);
  load_plane(id.z0 - 1, pu, pg);
  store_u(id.z0 - 1, pu);
  cells_of(id.z0 - 1, pu, pg, R0);
  load_plane(id.z0, pu, pg);
  store_u(id.z0, pu);
  cells_of(id.z0, pu, pg, R1);
  load_plane(id.z0 + 1, pu, pg);
  store_u(id.z0 + 1, pu);
  cells_of(id.z0 + 1, pu, pg, R2);
  load_plane(id.z0 + 2, pu, pg);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    bin_one(id.z0 - 1, id.z0 - 2, R3[j]);
    bin_one(id.z0 - 1, id.z0 - 1, R0[j]);
    bin_one(id.z0 - 1, id.z0, R1[j]);
    bin_one(id.z0 - 1, id.z0 + 1, R2[j]);
  }
  __syncthreads();
  {
    float none[3] = {0.0f, 0.0f, 0.0f};
    if (colv) gather(none, accA, true);
  }
  __syncthreads();

  // one plane: Sm (plane z-1), S0 (z), S1 (z+1) hold their sources, Sn
  // receives plane z+2's; (xu, xg) holds plane z+2 on entry and takes z+3;
  // acc holds the plane-z targets' a = 1 part and nacc receives plane z+1's
  auto step = [&](int z, Src2 (&Sm)[2], Src2 (&S0)[2], Src2 (&S1)[2], Src2 (&Sn)[2],
                  float (&xu)[2][3], float (&xg)[2][3], float (&acc)[3], float (&nacc)[3]) {
    // (i)
    clear_cells();
    clear_ovf(z + 1);
    store_u(z + 2, xu);
    cells_of(z + 2, xu, xg, Sn);
    load_plane(z + 3, xu, xg);
    __syncthreads();
    // (ii)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      bin_one(z, z - 1, Sm[j]);
      bin_one(z, z, S0[j]);
      bin_one(z, z + 1, S1[j]);
      bin_one(z, z + 2, Sn[j]);
    }
    // (iii) direct term of the plane-z targets: the own source's cell
    float r[3] = {acc[0], acc[1], acc[2]};
    if (colv) {
      const Src2& sv = S0[0];
      Tri t;
      bool k0, k1, k2;
      if (sv.key & kSrcValid) {
        const int i0 = z + ((sv.key >> 10) & 3) - 2;
        const int sa = (i0 + 10) % 5, sb = (i0 + 11) % 5;
        const int pb = ((sv.key >> 6) & 15) * H2X + (sv.key & 63);
        float h[8];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float gcv = c == 0 ? sv.g0 : (c == 1 ? sv.g1 : sv.g2);
          const float cv[8] = {uring[sa][c][pb],       uring[sa][c][pb + 1],
                               uring[sa][c][pb + H2X], uring[sa][c][pb + H2X + 1],
                               uring[sb][c][pb],       uring[sb][c][pb + 1],
                               uring[sb][c][pb + H2X], uring[sb][c][pb + H2X + 1]};
#pragma unroll
          for (int k = 0; k < 8; ++k) h[k] = c == 0 ? gcv * cv[k] : h[k] + gcv * cv[k];
        }
        t = tri_eval(h, sv.t0, sv.t1, sv.t2);
        k0 = (sv.key >> 12) & 1;
        k1 = (sv.key >> 13) & 1;
        k2 = (sv.key >> 14) & 1;
      } else {
        // a cell outside the staged planes (not reached while every offset
        // lies in [-2, 1]): corners from memory
        float u0 = uring[(z + 10) % 5][0][pe[0]], u1 = uring[(z + 10) % 5][1][pe[0]],
              u2 = uring[(z + 10) % 5][2][pe[0]];
        if (FIRST) {
          u0 *= scale;
          u1 *= scale;
          u2 *= scale;
        }
        const BorderCell bc = border_cell(g, z, py[0], px[0], u0, u1, u2);
        t.v = 0.0f;
        t.d0 = t.d1 = t.d2 = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float gcv = c == 0 ? sv.g0 : (c == 1 ? sv.g1 : sv.g2);
          float cv[8];
          corners_border(fc[c], g, bc.base, cv);
          const Tri tc = tri_eval(cv, bc.t0, bc.t1, bc.t2);
          t.d0 += tc.d0 * gcv;
          t.d1 += tc.d1 * gcv;
          t.d2 += tc.d2 * gcv;
        }
        k0 = bc.k0;
        k1 = bc.k1;
        k2 = bc.k2;
      }
      r[0] += sv.g0 + (k0 ? 0.0f : t.d0 * js);
      r[1] += sv.g1 + (k1 ? 0.0f : t.d1 * js);
      r[2] += sv.g2 + (k2 ? 0.0f : t.d2 * js);
    }
    __syncthreads();
    // (iv)
#pragma unroll
    for (int c = 0; c < 3; ++c) nacc[c] = 0.0f;
    if (colv) {
      gather(r, nacc, z + 1 < id.z1);
      const float* ov = &ovf[z & 1][0][0];
      r[0] += ov[threadIdx.x];
      r[1] += ov[ENT + threadIdx.x];
      r[2] += ov[2 * ENT + threadIdx.x];
      const uint32_t lin = static_cast<uint32_t>(z * g.plane + py[0] * g.d2 + px[0]);
      st_at(go, lin, r[0] * oscale);
      st_at(go + g.V, lin, r[1] * oscale);
      st_at(go + 2 * static_cast<size_t>(g.V), lin, r[2] * oscale);
    }
    __syncthreads();
  };
  // unrolled by four so that the source sets and partials keep their
  // registers
  for (int z = id.z0; z < id.z1; z += 4) {
    step(z, R0, R1, R2, R3, pu, pg, accA, accB);
    if (z + 1 < id.z1) step(z + 1, R1, R2, R3, R0, pu, pg, accB, accA);
    if (z + 2 < id.z1) step(z + 2, R2, R3, R0, R1, pu, pg, accA, accB);
    if (z + 3 < id.z1) step(z + 3, R3, R0, R1, R2, pu, pg, accB, accA);
  }
  }  // the last step's barrier lets the next chunk reuse the LDS
}

// Blocks of the persistent reach-2 marching adjoint: as many as are resident
// at once on the current device (so that no block waits for a second round),
// each taking every grid-th column chunk.
uint32_t march2_grid(const MarchGeom& m) {
  static int cap[64] = {};
  int dev = 0;
  uint32_t grid = 2048u;  // when the occupancy query fails
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) {
    int& c = cap[dev];
    if (c == 0) {
      int per_cu = 0, cus = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_exp_bwd_march2<false>, ENT,
                                                       0) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
        c = per_cu * cus;
    }
    if (c > 0) grid = static_cast<uint32_t>(c);
  }
  return m.total < grid ? m.total : grid;
}

// Blocks of the persistent tiled adjoint: enough to fill the chip several
// times over; each walks total / grid tiles.
uint32_t bwd_grid(const BwdGeom& bg) { return bg.total < 4096u ? bg.total : 4096u; }

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


// ---------------------------------------------------------------------------
// One inner iteration in one launch (small cohorts).
//
// For small volumes the marching kernels are bound by their serial planes
// (a 32^3 subject gives a squaring launch only 64 blocks of 8+ planes each)
// and by the ~20 launches of an iteration, not by memory.  This persistent
// kernel runs the whole iteration -- the squaring steps, warp + MSE/L1 +
// regulariser with their adjoints, the squaring adjoint and Adam -- as
// phases of tile-parallel work separated by grid barriers.  Its squaring
// steps gather directly (no plane ring) and write the same per-tile records
// as the marching forward; its adjoint is the tiled adjoint for every
// subject; the loss and the Adam update are the bodies of the separate
// kernels.

// One plane of a record tile (32 x 8 voxels, one per thread) of a squaring
// step: the arithmetic of k_exp_fwd<FIRST, REC> with the corners read from
// memory.  With REC the block merges its cell offsets into the tile's record
// (global atomics on boxes initialised by k_box_init) and raises the
// subject's reaches.  Blocks are (subject, tile, plane), so a small volume
// gets eight times the blocks of the marching kernel and no serial planes.
template <bool FIRST, bool REC>
__device__ __forceinline__ void exp_fwd_plane_body(int (*red)[ENT / 64], uint32_t blk,
                                                   const float* __restrict__ src,
                                                   float* __restrict__ dst, const TileGeom& tg,
                                                   float scale, int* __restrict__ boxes,
                                                   int* __restrict__ reach) {
  const Geom& g = tg.g;
  const uint32_t b = xcd_remap(blk, tg.total * ETZ);
  const uint32_t bt = b / ETZ;
  const int k = static_cast<int>(b - bt * ETZ);
  const int s = static_cast<int>(bt / tg.ntiles);
  const int tile = static_cast<int>(bt - static_cast<uint32_t>(s) * tg.ntiles);
  const int ox = (tile % tg.ntx) * ETX;
  const int oy = ((tile / tg.ntx) % tg.nty) * ETY;
  const int x0 = (tile / (tg.ntx * tg.nty)) * ETZ + k;
  const size_t off = static_cast<size_t>(s) * 3 * g.V;
  const float* f = src + off;
  float* o = dst + off;
  const float* fc[3] = {f, f + g.V, f + 2 * static_cast<size_t>(g.V)};
  const int lx = threadIdx.x % ETX, ly = threadIdx.x / ETX;
  const int x2 = ox + lx, x1 = oy + ly;
  int mn0 = INT_MAX, mn1 = INT_MAX, mn2 = INT_MAX, mx0 = INT_MIN, mx1 = INT_MIN, mx2 = INT_MIN;
  if (x2 < g.d2 && x1 < g.d1 && x0 < g.d0) {
    const uint32_t lin = static_cast<uint32_t>(x0 * g.plane + x1 * g.d2 + x2);
    float u0 = ld_at(fc[0], lin), u1 = ld_at(fc[1], lin), u2 = ld_at(fc[2], lin);
    if (FIRST) {
      u0 *= scale;
      u1 *= scale;
      u2 *= scale;
    }
    const BorderCell bc = border_cell(g, x0, x1, x2, u0, u1, u2);
    float cv[3][8];
#pragma unroll
    for (int c = 0; c < 3; ++c) corners_border(fc[c], g, bc.base, cv[c]);
    float r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[c] = tri_value(cv[c], bc.t0, bc.t1, bc.t2);
      if (FIRST) r[c] *= scale;
    }
    st_at(o, lin, u0 + r[0]);
    st_at(o + g.V, lin, u1 + r[1]);
    st_at(o + 2 * static_cast<size_t>(g.V), lin, u2 + r[2]);
    mn0 = mx0 = bc.i0 - x0;
    mn1 = mx1 = bc.i1 - x1;
    mn2 = mx2 = bc.i2 - x2;
  }
  if (REC) {
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
    if (threadIdx.x < 6) {
      const int q = threadIdx.x;
      int r = red[q][0];
      for (int i = 1; i < ENT / 64; ++i) r = q < 3 ? min(r, red[q][i]) : max(r, red[q][i]);
      int* bx = boxes + (static_cast<size_t>(s) * tg.ntiles + tile) * 8;
      if (q < 3) {
        atomicMin(bx + q, r);
        if (-r > 0) atomicMax(reach + s * 8 + q, -r);
      } else {
        atomicMax(bx + q, r);
        if (r + 1 > 0) atomicMax(reach + s * 8 + q, r + 1);
      }
    }
    __syncthreads();  // `red` is rewritten by the block's next plane
  }
}

// Record boxes of `count` tiles set to the empty box (min INT_MAX, max
// INT_MIN), before planes merge into them.
__global__ __launch_bounds__(ENT) void k_box_init(int* __restrict__ boxes, long long count) {
  const long long stride = static_cast<long long>(gridDim.x) * ENT;
  for (long long i = static_cast<long long>(blockIdx.x) * ENT + threadIdx.x; i < count * 8;
       i += stride) {
    const int e = static_cast<int>(i & 7);
    boxes[i] = e < 3 ? INT_MAX : (e < 6 ? INT_MIN : 0);
  }
}

template <bool FIRST, bool REC>
__global__ __launch_bounds__(ENT) void k_exp_fwd_planes(const float* __restrict__ src,
                                                        float* __restrict__ dst, TileGeom tg,
                                                        float scale, int* __restrict__ boxes,
                                                        int* __restrict__ reach) {
  __shared__ int red[6][ENT / 64];
  exp_fwd_plane_body<FIRST, REC>(red, blockIdx.x, src, dst, tg, scale, boxes, reach);
}

// Grid-wide barrier of a launch whose blocks are all resident.  bar[0]
// counts arrivals over the launch (zeroed before it); the k-th barrier
// returns once k * gridDim.x blocks have arrived.  The wait is bounded by the
// real-time counter: a block that has waited `ticks` raises err[0] and goes
// on, so every wave reaches the end of the kernel even if some block never
// ran.
__device__ __forceinline__ void grid_barrier(unsigned* bar, int* err, unsigned k,
                                             long long ticks) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(bar, 1u);
    const unsigned target = k * gridDim.x;
    const long long t0 = wall_clock64();
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (wall_clock64() - t0 > ticks) {
        atomicOr(err, 1);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
  }
  __syncthreads();
}

struct IterArgs {
  const float* img;    // [B][V]
  const float* atlas;  // [V]
  float* v;            // [B][3][V], updated in place (no smoothing on this path)
  float* m;
  float* s;
  float* v_out;        // Adam's outputs: v, m, s themselves, or scratch when timing
  float* m_out;
  float* s_out;
  float* ckpt;         // [n_sq - 1][B][3][V]
  float* uN;
  float* gU;
  float* gA;
  float* gB;
  float* gV;
  int* boxes;          // [n_sq][B][ntiles][8]
  int* reach;          // [n_sq][B][8]
  size_t box_stride, reach_stride;
  double* loss;        // loss[b * loss_stride] += L_b
  int loss_stride;
  RegW rw;
  TileGeom tg;
  BwdGeom bg;
  int n_sq;
  float scale;         // 2^-n_sq
  double inv_v;
  uint32_t nbx;        // voxel blocks per subject
  long long count;     // B * 3V
  const long long* step_dev;  // device step count, or NULL: step_host
  long long step_host;
  int k;               // inner iteration within the sweep
  float lr;
  double b1, b2;
  float eps;
  unsigned* bar;
  int* err;
  long long ticks;     // bound of a barrier wait (real-time counter ticks)
};

constexpr size_t kIterLds = sizeof(TiledBwdLds);

template <bool L1>
__global__ __launch_bounds__(ENT) void k_iter_fused(IterArgs a) {
  __shared__ __align__(16) unsigned char lds[kIterLds];
  const Geom& g = a.tg.g;
  const uint32_t G = gridDim.x;
  const size_t fs = static_cast<size_t>(a.tg.total / a.tg.ntiles) * 3 * g.V;
  unsigned nbar = 0;
  // the records are running minima / maxima: start the reaches at zero and
  // the boxes empty
  {
    const long long cnt = static_cast<long long>(a.reach_stride) * a.n_sq;
    for (long long i = static_cast<long long>(blockIdx.x) * ENT + threadIdx.x; i < cnt;
         i += static_cast<long long>(G) * ENT)
      a.reach[i] = 0;
    const long long nb = static_cast<long long>(a.box_stride) * a.n_sq;
    for (long long i = static_cast<long long>(blockIdx.x) * ENT + threadIdx.x; i < nb;
         i += static_cast<long long>(G) * ENT) {
      const int e = static_cast<int>(i & 7);
      a.boxes[i] = e < 3 ? INT_MAX : (e < 6 ? INT_MIN : 0);
    }
  }
  grid_barrier(a.bar, a.err, ++nbar, a.ticks);
  // squaring steps (u_0 = v / 2^N scaled on the fly), records for the adjoint
  int (*red)[ENT / 64] = reinterpret_cast<int(*)[ENT / 64]>(lds);
  const float* src = a.v;
  for (int t = 0; t < a.n_sq; ++t) {
    float* dst = (t == a.n_sq - 1) ? a.uN : a.ckpt + static_cast<size_t>(t) * fs;
    int* bx = a.boxes + a.box_stride * t;
    int* rc = a.reach + a.reach_stride * t;
    for (uint32_t b = blockIdx.x; b < a.tg.total * ETZ; b += G) {
      if (t == 0)
        exp_fwd_plane_body<true, true>(red, b, src, dst, a.tg, a.scale, bx, rc);
      else
        exp_fwd_plane_body<false, true>(red, b, src, dst, a.tg, 1.0f, bx, rc);
    }
    grid_barrier(a.bar, a.err, ++nbar, a.ticks);
    src = dst;
  }
  // dissimilarity + regulariser, and dL/du_N
  {
    const uint32_t total = a.nbx * (a.tg.total / a.tg.ntiles);
    double* rd = reinterpret_cast<double*>(lds);
    for (uint32_t b = blockIdx.x; b < total; b += G)
      mse_fused_block<L1, true>(xcd_remap(b, total), rd, a.img, a.atlas, a.uN, a.gU, a.loss,
                                a.loss_stride, a.rw, g, a.inv_v, a.nbx);
  }
  grid_barrier(a.bar, a.err, ++nbar, a.ticks);
  // squaring adjoint, every subject on the tiled path
  TiledBwdLds& L = *reinterpret_cast<TiledBwdLds*>(lds);
  const float* gin = a.gU;
  for (int t = a.n_sq - 1; t >= 0; --t) {
    float* gout = (t == 0) ? a.gV : (((a.n_sq - 1 - t) % 2 == 0) ? a.gA : a.gB);
    const float* ut = (t == 0) ? a.v : a.ckpt + static_cast<size_t>(t - 1) * fs;
    const int* bx = a.boxes + a.box_stride * t;
    const int* rc = a.reach + a.reach_stride * t;
    if (t == 0)
      exp_bwd_tiled_body<true, true>(L, blockIdx.x, G, ut, gin, gout, a.bg, a.scale, a.scale, bx,
                                     rc);
    else
      exp_bwd_tiled_body<false, true>(L, blockIdx.x, G, ut, gin, gout, a.bg, 1.0f, 1.0f, bx, rc);
    grid_barrier(a.bar, a.err, ++nbar, a.ticks);
    gin = gout;
  }
  // Adam; bias corrections formed in FP64 and rounded once, as the separate
  // kernels do
  const double tt = static_cast<double>((a.step_dev ? a.step_dev[0] : a.step_host) + a.k + 1);
  const float bc1 = static_cast<float>(1.0 - pow(a.b1, tt));
  const float bc2 = static_cast<float>(1.0 - pow(a.b2, tt));
  const float b1f = static_cast<float>(a.b1), b2f = static_cast<float>(a.b2);
  const float omb1 = static_cast<float>(1.0 - a.b1), omb2 = static_cast<float>(1.0 - a.b2);
  for (long long i = static_cast<long long>(blockIdx.x) * ENT + threadIdx.x; i < a.count;
       i += static_cast<long long>(G) * ENT)
    adam_step_to(a.v, a.m, a.s, a.gV, a.v_out, a.m_out, a.s_out, i, a.lr, b1f, omb1, b2f, omb2,
                 bc1, bc2, a.eps);
}

// A barrier that timed out leaves NaN as the group loss.
__global__ void k_flag_loss(const int* __restrict__ err, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && err[0]) out[0] = __builtin_nan("");
}
}  // namespace

size_t exp_aux_bytes(const Geom& g, int n, int n_sq) {
  const TileGeom tg = make_tiles(g, n);
  return (static_cast<size_t>(n) * tg.ntiles * 8 + static_cast<size_t>(n) * 8) * n_sq *
         sizeof(int);
}

// Chunk length along d0 of the marching kernels: long chunks amortise the two
// planes of ramp-up; shorter ones give small cohorts enough blocks.
int march_tz(const TileGeom& tg, int n) {
  const int tuned = tuned_tz(TUNE_EXP, tg.g, n);
  if (tuned > 1) return tuned;
  if (tuned < 0) return ETZ;  // plane-parallel kernels; the chunk is not used
  // long chunks amortise the ramp-up planes, short ones keep each block's
  // planes in flight within L2 (64 planes measured no faster than 32 and
  // fetched more from HBM); shorter still for small cohorts
  int tz = 32;
  while (tz > ETZ && static_cast<long long>(tg.ntx) * tg.nty * ((tg.g.d0 + tz - 1) / tz) * n < 4096)
    tz /= 2;
  return tz;
}

// The other shape of the squaring steps and their adjoint: one plane of a
// tile per block (k_exp_fwd_planes) and the tiled adjoint for every subject,
// no marching.  It wins on small volumes, where the marching kernels' serial
// planes are the whole cost (4 x 32^3: 0.78 ms per sweep against 1.60).
// Untuned, it is taken when the marching grid would hold fewer than four
// blocks per CU even with 8-plane chunks.
bool plane_mode(const Geom& g, int n) {
  const int tuned = tuned_tz(TUNE_EXP, g, n);
  if (tuned != 0) return tuned < 0;
  const long long march_blocks = static_cast<long long>((g.d2 + ETX - 1) / ETX) *
                                 ((g.d1 + ETY - 1) / ETY) * ((g.d0 + ETZ - 1) / ETZ) * n;
  return march_blocks < 1024;
}

void run_exp_fwd(const float* v, float* u, float* ckpt, float* tmp, int* aux, const Geom& g, int n,
                 int n_sq, hipStream_t st, bool negate) {
  const size_t fs = static_cast<size_t>(n) * 3 * g.V;
  if (n_sq == 0) {
    prof_begin(st, KC_MISC);
    (void)hipMemcpyAsync(u, v, fs * sizeof(float), hipMemcpyDeviceToDevice, st);
    prof_end(st, KC_MISC);
    return;
  }
  const TileGeom tg = make_tiles(g, n);
  const MarchGeom m = make_march(tg, n, march_tz(tg, n));
  const AuxPtrs ap = aux_ptrs(aux, tg, n, n_sq);
  const bool planes = plane_mode(g, n);
  // the reaches are running maxima: start them at zero (all-zero bits); the
  // planes kernel merges into its boxes, which start empty
  if (aux) {
    launch_fill_f32(reinterpret_cast<float*>(ap.reach),
                    static_cast<long long>(ap.reach_stride) * n_sq, 0.0f, st);
    if (planes) {
      const long long nbox = static_cast<long long>(ap.box_stride / 8) * n_sq;
      prof_begin(st, KC_FILL);
      hipLaunchKernelGGL(k_box_init, dim3(static_cast<uint32_t>(
                                         nbox * 8 / ENT + 1 < 65536 ? nbox * 8 / ENT + 1 : 65536)),
                         dim3(ENT), 0, st, ap.boxes, nbox);
      prof_end(st, KC_FILL);
    }
  }
  // Exp(-v) negates the scaled field of the first step (exact)
  const float scale = negate ? -ldexpf(1.0f, -n_sq) : ldexpf(1.0f, -n_sq);
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
    if (planes) {
      const dim3 grid(tg.total * ETZ);
      if (t == 0 && aux)
        hipLaunchKernelGGL((k_exp_fwd_planes<true, true>), grid, dim3(ENT), 0, st, src, dst, tg,
                           scale, bx, rc);
      else if (t == 0)
        hipLaunchKernelGGL((k_exp_fwd_planes<true, false>), grid, dim3(ENT), 0, st, src, dst, tg,
                           scale, bx, rc);
      else if (aux)
        hipLaunchKernelGGL((k_exp_fwd_planes<false, true>), grid, dim3(ENT), 0, st, src, dst, tg,
                           1.0f, bx, rc);
      else
        hipLaunchKernelGGL((k_exp_fwd_planes<false, false>), grid, dim3(ENT), 0, st, src, dst,
                           tg, 1.0f, bx, rc);
    } else if (t == 0) {
      if (aux)
        hipLaunchKernelGGL((k_exp_fwd<true, true>), dim3(m.total), dim3(ENT), 0, st, src, dst, m,
                           scale, bx, rc);
      else
        hipLaunchKernelGGL((k_exp_fwd<true, false>), dim3(m.total), dim3(ENT), 0, st, src, dst, m,
                           scale, bx, rc);
    } else {
      if (aux)
        hipLaunchKernelGGL((k_exp_fwd<false, true>), dim3(m.total), dim3(ENT), 0, st, src, dst, m,
                           1.0f, bx, rc);
      else
        hipLaunchKernelGGL((k_exp_fwd<false, false>), dim3(m.total), dim3(ENT), 0, st, src, dst,
                           m, 1.0f, bx, rc);
    }
    prof_end(st, KC_EXP_FWD);
    src = dst;
  }
}

namespace {

// Records of one step (positions x + u_t) and the adjoint of that step.
void launch_rec(const float* ut, bool first, const TileGeom& tg, float scale, int* bx, int* rc,
                hipStream_t st) {
  prof_begin(st, KC_MISC);
  if (first)
    hipLaunchKernelGGL((k_exp_rec<true>), dim3(tg.total), dim3(ENT), 0, st, ut, tg, scale, bx, rc);
  else
    hipLaunchKernelGGL((k_exp_rec<false>), dim3(tg.total), dim3(ENT), 0, st, ut, tg, 1.0f, bx, rc);
  prof_end(st, KC_MISC);
}

void launch_bwd_step(const float* ut, const float* gin, float* gout, bool first, const MarchGeom& m,
                     const BwdGeom& bg, float scale, const int* bx, const int* rc, bool planes,
                     hipStream_t st) {
  prof_begin(st, KC_EXP_BWD);
  if (planes) {
    // every subject on the tiled adjoint
    if (first)
      hipLaunchKernelGGL((k_exp_bwd<true, true>), dim3(bwd_grid(bg)), dim3(BNT), 0, st, ut, gin,
                         gout, bg, scale, scale, bx, rc);
    else
      hipLaunchKernelGGL((k_exp_bwd<false, true>), dim3(bwd_grid(bg)), dim3(BNT), 0, st, ut, gin,
                         gout, bg, 1.0f, 1.0f, bx, rc);
    prof_end(st, KC_EXP_BWD);
    return;
  }
  // each subject is handled by exactly one of the three kernels (decided on
  // the device from its reach: 1, 2, beyond); the others' blocks return at once
  if (first) {
    hipLaunchKernelGGL((k_exp_bwd_march<true>), dim3(m.total), dim3(ENT), 0, st, ut, gin, gout, m,
                       scale, scale, rc);
    hipLaunchKernelGGL((k_exp_bwd_march2<true>), dim3(march2_grid(m)), dim3(ENT), 0, st, ut, gin,
                       gout, m, scale, scale, rc);
    hipLaunchKernelGGL((k_exp_bwd<true, false>), dim3(bwd_grid(bg)), dim3(BNT), 0, st, ut, gin,
                       gout, bg, scale, scale, bx, rc);
  } else {
    hipLaunchKernelGGL((k_exp_bwd_march<false>), dim3(m.total), dim3(ENT), 0, st, ut, gin, gout, m,
                       1.0f, 1.0f, rc);
    hipLaunchKernelGGL((k_exp_bwd_march2<false>), dim3(march2_grid(m)), dim3(ENT), 0, st, ut, gin,
                       gout, m, 1.0f, 1.0f, rc);
    hipLaunchKernelGGL((k_exp_bwd<false, false>), dim3(bwd_grid(bg)), dim3(BNT), 0, st, ut, gin,
                       gout, bg, 1.0f, 1.0f, bx, rc);
  }
  prof_end(st, KC_EXP_BWD);
}

}  // namespace

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
  const MarchGeom m = make_march(tg, n, march_tz(tg, n));
  const AuxPtrs ap = aux_ptrs(aux, tg, n, n_sq);
  const float scale = ldexpf(1.0f, -n_sq);
  if (!aux_ready) {
    launch_fill_f32(reinterpret_cast<float*>(ap.reach),
                    static_cast<long long>(ap.reach_stride) * n_sq, 0.0f, st);
    for (int t = 0; t < n_sq; ++t) {
      const float* ut = (t == 0) ? v : ckpt + static_cast<size_t>(t - 1) * fs;
      launch_rec(ut, t == 0, tg, scale, ap.boxes + ap.box_stride * t,
                 ap.reach + ap.reach_stride * t, st);
    }
  }
  const float* gin = g_u;
  for (int t = n_sq - 1; t >= 0; --t) {
    float* gout = (t == 0) ? g_v : (((n_sq - 1 - t) % 2 == 0) ? tmp_a : tmp_b);
    const float* ut = (t == 0) ? v : ckpt + static_cast<size_t>(t - 1) * fs;
    launch_bwd_step(ut, gin, gout, t == 0, m, bg, scale, ap.boxes + ap.box_stride * t,
                    ap.reach + ap.reach_stride * t, plane_mode(g, n), st);
    gin = gout;
  }
}

void run_exp_bwd_recompute(const float* v, const float* g_u, float* g_v, float* tmp_a,
                           float* tmp_b, float* rec_a, float* rec_b, int* aux, const Geom& g,
                           int n, int n_sq, hipStream_t st) {
  const TileGeom tg = make_tiles(g, n);
  const BwdGeom bg = make_bwd(tg, n);
  const MarchGeom m = make_march(tg, n, march_tz(tg, n));
  const AuxPtrs ap = aux_ptrs(aux, tg, n, n_sq);
  const float scale = ldexpf(1.0f, -n_sq);
  launch_fill_f32(reinterpret_cast<float*>(ap.reach),
                  static_cast<long long>(ap.reach_stride) * n_sq, 0.0f, st);
  const float* gin = g_u;
  for (int t = n_sq - 1; t >= 0; --t) {
    // u_t = t squaring steps of v / 2^N, ping-ponging so that it ends in rec_a
    const float* ut = v;
    for (int k = 0; k < t; ++k) {
      float* dst = ((t - 1 - k) % 2 == 0) ? rec_a : rec_b;
      prof_begin(st, KC_EXP_FWD);
      if (k == 0)
        hipLaunchKernelGGL((k_exp_fwd<true, false>), dim3(m.total), dim3(ENT), 0, st, ut, dst, m,
                           scale, nullptr, nullptr);
      else
        hipLaunchKernelGGL((k_exp_fwd<false, false>), dim3(m.total), dim3(ENT), 0, st, ut, dst, m,
                           1.0f, nullptr, nullptr);
      prof_end(st, KC_EXP_FWD);
      ut = dst;
    }
    int* bx = ap.boxes + ap.box_stride * t;
    int* rc = ap.reach + ap.reach_stride * t;
    launch_rec(ut, t == 0, tg, scale, bx, rc, st);
    float* gout = (t == 0) ? g_v : (((n_sq - 1 - t) % 2 == 0) ? tmp_a : tmp_b);
    launch_bwd_step(ut, gin, gout, t == 0, m, bg, scale, bx, rc, plane_mode(g, n), st);
    gin = gout;
  }
}

namespace {

long long g_barrier_ticks = kDefaultBarrierTicks;

// Resident blocks of the fused kernel on the current device (0 when the
// query fails).
template <bool L1>
int fused_capacity() {
  static int cap[2][64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  int& c = cap[L1 ? 1 : 0][dev];
  if (c == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_iter_fused<L1>, ENT, 0) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    c = per_cu * cus;
  }
  return c;
}

template <bool L1>
bool launch_iter(const IterArgs& a, uint32_t needed, hipStream_t st) {
  const int cap = fused_capacity<L1>();
  if (cap < 8) return false;
  uint32_t grid = needed < static_cast<uint32_t>(cap) ? needed : static_cast<uint32_t>(cap);
  // a multiple of the 8 XCDs, so that the XCD of a virtual block index is
  // that of the hardware block running it
  // at most 128 blocks: every block's agent-scope fence in a grid barrier
  // writes back its XCD's L2, and the fences serialise (measured 4.6 us per
  // barrier at 64 blocks, 8.1 at 128, 37 at 512)
  grid = grid < 128u ? grid : 128u;
  grid = grid >= 8 ? grid / 8 * 8 : 8;
  if (grid > static_cast<uint32_t>(cap)) return false;
  hipLaunchKernelGGL((k_iter_fused<L1>), dim3(grid), dim3(ENT), 0, st, a);
  return true;
}

}  // namespace

bool run_iter_fused(const float* img, const float* atlas, float* v, float* m, float* s,
                    float* ckpt, int* aux, float* uN, float* gU, float* gA, float* gB, float* gV,
                    double* loss, int loss_stride, const RegW& rw, const Geom& g, int n, int n_sq,
                    const long long* step_dev, long long step_host, int k, float lr, double b1,
                    double b2, float eps, bool l1, unsigned* bar, int* err, hipStream_t st,
                    float* v_out, float* m_out, float* s_out) {
  if (n_sq < 1 || (!ckpt && n_sq >= 2)) return false;
  const TileGeom tg = make_tiles(g, n);
  const AuxPtrs ap = aux_ptrs(aux, tg, n, n_sq);
  IterArgs a;
  a.img = img;
  a.atlas = atlas;
  a.v = v;
  a.m = m;
  a.s = s;
  a.v_out = v_out ? v_out : v;
  a.m_out = m_out ? m_out : m;
  a.s_out = s_out ? s_out : s;
  a.ckpt = ckpt;
  a.uN = uN;
  a.gU = gU;
  a.gA = gA;
  a.gB = gB;
  a.gV = gV;
  a.boxes = ap.boxes;
  a.reach = ap.reach;
  a.box_stride = ap.box_stride;
  a.reach_stride = ap.reach_stride;
  a.loss = loss;
  a.loss_stride = loss_stride;
  a.rw = rw;
  a.tg = tg;
  a.bg = make_bwd(tg, n);
  a.n_sq = n_sq;
  a.scale = ldexpf(1.0f, -n_sq);
  a.inv_v = 1.0 / g.V;
  a.nbx = blocks_for(g.V, kBlock);
  a.count = static_cast<long long>(n) * 3 * g.V;
  a.step_dev = step_dev;
  a.step_host = step_host;
  a.k = k;
  a.lr = lr;
  a.b1 = b1;
  a.b2 = b2;
  a.eps = eps;
  a.bar = bar;
  a.err = err;
  a.ticks = g_barrier_ticks;
  const uint32_t nv = a.nbx * static_cast<uint32_t>(n);
  uint32_t needed = tg.total * ETZ > nv ? tg.total * ETZ : nv;
  needed = needed > a.bg.total ? needed : a.bg.total;
  // the arrival counter starts every launch at zero (a fill kernel, so that
  // the sequence can be captured)
  launch_fill_f32(reinterpret_cast<float*>(bar), 1, 0.0f, st);
  prof_begin(st, KC_ITER);
  const bool ok = l1 ? launch_iter<true>(a, needed, st) : launch_iter<false>(a, needed, st);
  prof_end(st, KC_ITER);
  return ok;
}

void flag_fused_error(const int* err, double* out, hipStream_t st) {
  prof_begin(st, KC_MISC);
  hipLaunchKernelGGL(k_flag_loss, dim3(1), dim3(64), 0, st, err, out);
  prof_end(st, KC_MISC);
}

void set_barrier_ticks(long long ticks) {
  g_barrier_ticks = ticks < 0 ? kDefaultBarrierTicks : ticks;
}

int fused_resident_blocks(bool l1) { return l1 ? fused_capacity<true>() : fused_capacity<false>(); }

}  // namespace darc
