// Window kernels of libdarc: the local NCC statistics and their adjoint
// (win^3 box sums, FP64) and the separable Gaussian smoother.
//
// Each block owns a TX x TY tile of a (d1, d2) plane and marches along d0 over
// a chunk of TZ planes.  For every plane it stages the tile plus its halo in
// LDS, sums along d2 and then d1 in LDS, and keeps the last W plane sums in a
// register ring from which the d0-direction window sum follows (running sum
// for the box, weighted sum for the Gaussian).  The plane loop is unrolled by
// W so that every ring slot is a compile-time register.
#include "darc_kernels.hpp"

namespace darc {

namespace {

constexpr int kTX = 32;  // tile width along d2
constexpr int kTY = 8;   // tile height along d1
constexpr int kNT = kTX * kTY;

struct MarchGeom {
  Geom g;
  int ntx, nty, nz, tz;
  uint32_t total;  // ntx * nty * nz * nchan blocks
};

struct Tile {
  int xb, yb, z0, z1, chan;
};

template <int TX = kTX, int TY = kTY>
__device__ __forceinline__ Tile march_tile(const MarchGeom& mg) {
  uint32_t b = xcd_remap(blockIdx.x, mg.total);
  Tile t;
  const int tx = static_cast<int>(b % mg.ntx);
  b /= mg.ntx;
  const int ty = static_cast<int>(b % mg.nty);
  b /= mg.nty;
  const int zc = static_cast<int>(b % mg.nz);
  t.chan = static_cast<int>(b / mg.nz);
  t.xb = tx * TX;
  t.yb = ty * TY;
  t.z0 = zc * mg.tz;
  t.z1 = min(t.z0 + mg.tz, mg.g.d0);
  return t;
}

MarchGeom make_march(const Geom& g, int nchan, int halo, int tx = kTX, int ty = kTY) {
  MarchGeom mg;
  mg.g = g;
  mg.ntx = (g.d2 + tx - 1) / tx;
  mg.nty = (g.d1 + ty - 1) / ty;
  // long chunks amortise the 2*halo planes of ramp-up (d0 split into equal
  // chunks of at most 96 planes); shorter ones give enough blocks for small
  // cohorts
  int tz = tuned_tz(TUNE_WINDOW, g, nchan);
  if (tz <= 0) {
    const int nzc = (g.d0 + 95) / 96;
    tz = (g.d0 + nzc - 1) / nzc;
    while (tz > 8 && tz > 2 * halo &&
           static_cast<long long>(mg.ntx) * mg.nty * ((g.d0 + tz - 1) / tz) * nchan < 2048)
      tz = (tz + 1) / 2;
  }
  mg.tz = tz;
  mg.nz = (g.d0 + tz - 1) / tz;
  mg.total = static_cast<uint32_t>(mg.ntx) * mg.nty * mg.nz * nchan;
  return mg;
}

// Window sums along y of NQ row-sum planes sr [NQ][HY][kTX] into
// sc [NQ][kTY][kTX]: one thread per (quantity, column) slides down the
// column (add the entering row, drop the leaving one).
template <int W, int NQ>
__device__ __forceinline__ void column_sums(const double* __restrict__ sr, double* __restrict__ sc,
                                            int tid) {
  constexpr int HY = kTY + W - 1;
  if (tid < NQ * kTX) {
    const int c = tid / kTX, cx = tid - c * kTX;
    const double* col = sr + c * HY * kTX + cx;
    double* out = sc + c * kTY * kTX + cx;
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) a += col[k * kTX];
    out[0] = a;
#pragma unroll
    for (int r = 1; r < kTY; ++r) {
      a += col[(r + W - 1) * kTX] - col[(r - 1) * kTX];
      out[r * kTX] = a;
    }
  }
}

// -------------------------------------------------------------- LNCC forward
//
// Window sums S_I, S_J, S_II, S_JJ, S_IJ over the W^3 cube centred at each
// voxel (zero outside the volume, N = W^3), then
//   cross = S_IJ - S_I S_J / N, Ivar = S_II - S_I^2 / N, Jvar = S_JJ - S_J^2 / N,
//   den = Ivar Jvar + eps, cc = cross^2 / den,
// loss += -(1/V) sum cc and, when FIELDS, the four per-voxel factors of the
// adjoint: alpha = 2 cross / den, alpha * Jbar, beta = 2 cross^2 Jvar / den^2,
// beta * Ibar.
template <int W, bool FIELDS>
__global__ __launch_bounds__(kNT) void k_lncc_fwd(const float* __restrict__ wimg,
                                                  const float* __restrict__ atlas,
                                                  float* __restrict__ fields,
                                                  double* __restrict__ loss, int loss_stride,
                                                  MarchGeom mg, double eps, double neg_inv_v,
                                                  long long wstr, long long astr) {
  constexpr int R = W / 2, HX = kTX + 2 * R, HY = kTY + 2 * R;
  constexpr double kInvN = 1.0 / (W * W * W);
  // staged planes in FP32 (the inputs' own precision), widened at the taps
  __shared__ __attribute__((aligned(16))) float sI[HY * HX];
  __shared__ __attribute__((aligned(16))) float sJ[HY * HX];
  __shared__ double sr[5][HY * kTX];
  __shared__ double sc[5][kTY * kTX];
  __shared__ double red[kNT / 64];
  const Geom& g = mg.g;
  const Tile tl = march_tile(mg);
  const int tid = threadIdx.x, lx = tid % kTX, ly = tid / kTX;
  const float* I = wimg + tl.chan * wstr;
  const float* Jm = atlas + tl.chan * astr;
  double ring[W][5];
  double S[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    S[c] = 0.0;
#pragma unroll
    for (int j = 0; j < W; ++j) ring[j][c] = 0.0;
  }
  double acc = 0.0;
  // planes walked: the chunk and R on either side, padded to a multiple of W
  // so that the unrolled body has no branch around its loads and stores
  // (padding planes stage clamped values and store nothing)
  const int nplanes = (tl.z1 - tl.z0) + 2 * R;
  const int npad = (nplanes + W - 1) / W * W;
  // Staged positions of this thread (NPRE per plane): the next plane is
  // loaded into registers while the current one is summed.  Loads are
  // unconditional from clamped positions; out-of-volume values become zeros
  // when staged.
  constexpr int NPRE = (HY * HX + kNT - 1) / kNT;
  uint32_t poff[NPRE];
  bool pin[NPRE];
#pragma unroll
  for (int j = 0; j < NPRE; ++j) {
    const int e = min(tid + j * kNT, HY * HX - 1);
    const int hy = e / HX, hx = e - hy * HX;
    const int y = tl.yb - R + hy, x = tl.xb - R + hx;
    pin[j] = y >= 0 && y < g.d1 && x >= 0 && x < g.d2;
    poff[j] = static_cast<uint32_t>(min(max(y, 0), g.d1 - 1) * g.d2 + min(max(x, 0), g.d2 - 1));
  }
  float pI[NPRE], pJ[NPRE];
  auto load_plane = [&](int p) {
    const int zc = min(max(tl.z0 - R + p, 0), g.d0 - 1);
#pragma unroll
    for (int j = 0; j < NPRE; ++j) {
      const uint32_t lin = static_cast<uint32_t>(zc) * static_cast<uint32_t>(g.plane) + poff[j];
      pI[j] = ld_at(I, lin);
      pJ[j] = ld_at(Jm, lin);
    }
  };
  // the four factor fields of this subject (stores masked per lane)
  MaskedOut fo[4];
  if (FIELDS) {
    float* F = fields + static_cast<size_t>(tl.chan) * 4 * g.V;
#pragma unroll
    for (int k = 0; k < 4; ++k) fo[k] = masked_out(F + static_cast<size_t>(k) * g.V, g.V);
  }
  load_plane(0);
  for (int base = 0; base < npad; base += W) {
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const int p = base + j;
      {
        const int zz = tl.z0 - R + p;
        const bool zin = (zz >= 0) && (zz < g.d0);
#pragma unroll
        for (int k = 0; k < NPRE; ++k) {
          const int e = tid + k * kNT;
          if (k + 1 < NPRE || e < HY * HX) {
            const bool in = zin && pin[k];
            sI[e] = in ? pI[k] : 0.0f;
            sJ[e] = in ? pJ[k] : 0.0f;
          }
        }
        load_plane(p + 1);
        __syncthreads();
        // row sums along x, two neighbouring outputs per thread: the second
        // slides the first by one (add the entering tap, drop the leaving one)
        for (int e = tid; e < HY * (kTX / 2); e += kNT) {
          const int hy = e / (kTX / 2), cx = 2 * (e - hy * (kTX / 2));
          // (scalar loads: staging the W + 1 taps in registers would push
          // the kernel past the register budget of three waves per SIMD)
          const float* rI = sI + hy * HX + cx;
          const float* rJ = sJ + hy * HX + cx;
          double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0;
#pragma unroll
          for (int k = 0; k < W; ++k) {
            const double vi = rI[k], vj = rJ[k];  // exact widening
            a0 += vi;
            a1 += vj;
            a2 += vi * vi;
            a3 += vj * vj;
            a4 += vi * vj;
          }
          const double io = rI[0], jo = rJ[0], in = rI[W], jn = rJ[W];
          const int o = hy * kTX + cx;
          sr[0][o] = a0;
          sr[1][o] = a1;
          sr[2][o] = a2;
          sr[3][o] = a3;
          sr[4][o] = a4;
          sr[0][o + 1] = a0 + (in - io);
          sr[1][o + 1] = a1 + (jn - jo);
          sr[2][o + 1] = a2 + (in * in - io * io);
          sr[3][o + 1] = a3 + (jn * jn - jo * jo);
          sr[4][o + 1] = a4 + (in * jn - io * jo);
        }
        __syncthreads();
        column_sums<W, 5>(&sr[0][0], &sc[0][0], tid);
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          const double P = sc[c][ly * kTX + lx];
          S[c] += P - ring[j][c];
          ring[j][c] = P;
        }
        const int zo = zz - R;
        const int y = tl.yb + ly, x = tl.xb + lx;
        const bool out = zo >= tl.z0 && zo < tl.z1 && y < g.d1 && x < g.d2;
        float fv[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (out) {
          const double cross = S[4] - S[0] * S[1] * kInvN;
          const double ivar = S[2] - S[0] * S[0] * kInvN;
          const double jvar = S[3] - S[1] * S[1] * kInvN;
          const double den = ivar * jvar + eps;
          const double rden = 1.0 / den;  // one division for the three quotients
          const double cc = cross * cross * rden;
          acc += cc;
          if (FIELDS) {
            const double alpha = 2.0 * cross * rden;
            const double beta = alpha * cross * jvar * rden;
            fv[0] = static_cast<float>(alpha);
            fv[1] = static_cast<float>(alpha * S[1] * kInvN);
            fv[2] = static_cast<float>(beta);
            fv[3] = static_cast<float>(beta * S[0] * kInvN);
          }
        }
        if (FIELDS) {
          const uint32_t idx = static_cast<uint32_t>((zo * g.d1 + y) * g.d2 + x);
#pragma unroll
          for (int k = 0; k < 4; ++k) store_masked(fo[k], idx, fv[k], out);
        }
        __syncthreads();
      }
    }
  }
  const double tot = block_sum<kNT>(acc, red);
  if (tid == 0) atomicAdd(loss + static_cast<size_t>(tl.chan) * loss_stride, tot * neg_inv_v);
}

// -------------------------------------------------------------- LNCC adjoint
//
// Box sums (same zero-padded W^3 window) of the four factor fields, then
//   dD/dI(y) = -(1/V) [J(y) Box(alpha) - Box(alpha Jbar) - I(y) Box(beta) + Box(beta Ibar)].
// FUSED: continues through the warp adjoint, gu = dD/dI * grad I_orig(x + u)
// + lam dR/du, and adds lam R(u) to the loss; otherwise writes dD/dI.
template <int W, bool FUSED>
__global__ __launch_bounds__(kNT, W <= 9 ? 3 : 2) void k_lncc_bwd(
    const float* __restrict__ fields, const float* __restrict__ wimg,
    const float* __restrict__ atlas, float* __restrict__ gw, const float* __restrict__ img,
    const float* __restrict__ u, float* __restrict__ gu, double* __restrict__ loss,
    int loss_stride, RegW rw, MarchGeom mg, double neg_inv_v, long long wstr, long long astr) {
  constexpr int R = W / 2, HX = kTX + 2 * R, HY = kTY + 2 * R;
  // staged factor planes in FP32 (their stored precision), widened at the taps
  __shared__ __attribute__((aligned(16))) float sIn[4][HY * HX];
  __shared__ double sr[4][HY * kTX];
  __shared__ double sc[4][kTY * kTX];
  __shared__ double red[kNT / 64];
  const Geom& g = mg.g;
  const Tile tl = march_tile(mg);
  const int tid = threadIdx.x, lx = tid % kTX, ly = tid / kTX;
  const float* F = fields + static_cast<size_t>(tl.chan) * 4 * g.V;
  double ring[W][4];
  double S[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    S[c] = 0.0;
#pragma unroll
    for (int j = 0; j < W; ++j) ring[j][c] = 0.0;
  }
  double racc = 0.0;
  const int nplanes = (tl.z1 - tl.z0) + 2 * R;
  // The next plane's four factors are loaded into registers while the
  // current plane is summed.  Every load is unconditional, from a clamped
  // (valid) position, and the zero padding outside the volume is applied
  // when the values are staged: a load under a branch, or a select right
  // after it, would make the compiler wait for it at once.
  constexpr int NE = (HY * HX + kNT - 1) / kNT;
  int eoff[NE];
  bool ein[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = tid + k * kNT;
    const int hy = e / HX, hx = e - hy * HX;
    const int y = tl.yb - R + hy, x = tl.xb - R + hx;
    ein[k] = e < HY * HX && y >= 0 && y < g.d1 && x >= 0 && x < g.d2;
    eoff[k] = min(max(y, 0), g.d1 - 1) * g.d2 + min(max(x, 0), g.d2 - 1);
  }
  float pre[NE][4];
  bool pzin = false;  // the prefetched plane lies inside the volume
  auto load_plane = [&](int p) {
    const int zz = tl.z0 - R + p;
    pzin = (zz >= 0) && (zz < g.d0);
    const int zc = min(max(zz, 0), g.d0 - 1);
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int idx = zc * g.plane + eoff[k];
      pre[k][0] = F[idx];
      pre[k][1] = F[g.V + idx];
      pre[k][2] = F[2 * g.V + idx];
      pre[k][3] = F[3 * g.V + idx];
    }
  };
  load_plane(0);
  // Output voxel (clamped: always valid, used only for live outputs; the
  // ramp-up planes before the chunk read its first output plane).  With the
  // warp adjoint fused, u at the output voxel is loaded one plane ahead, so
  // that the image corners around x + u go out before the next plane's
  // factors and arrive while the plane is summed.
  const int oy = min(tl.yb + ly, g.d1 - 1), ox = min(tl.xb + lx, g.d2 - 1);
  auto out_idx = [&](int zo) { return (min(max(zo, tl.z0), g.d0 - 1) * g.d1 + oy) * g.d2 + ox; };
  const float* uf = u + static_cast<size_t>(tl.chan) * 3 * g.V;
  const float* Io = img + static_cast<size_t>(tl.chan) * g.V;
  float nu[3] = {0.0f, 0.0f, 0.0f};
  if (FUSED) {
    const int i = out_idx(tl.z0 - 2 * R);
#pragma unroll
    for (int c = 0; c < 3; ++c) nu[c] = uf[static_cast<size_t>(c) * g.V + i];
  }
  for (int base = 0; base < nplanes; base += W) {
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const int p = base + j;
      if (p < nplanes) {
        const int zz = tl.z0 - R + p;
#pragma unroll
        for (int k = 0; k < NE; ++k) {
          const int e = tid + k * kNT;
          if (e < HY * HX) {
            const bool ok = pzin && ein[k];
            sIn[0][e] = ok ? pre[k][0] : 0.0f;
            sIn[1][e] = ok ? pre[k][1] : 0.0f;
            sIn[2][e] = ok ? pre[k][2] : 0.0f;
            sIn[3][e] = ok ? pre[k][3] : 0.0f;
          }
        }
        // the output voxel's own values, issued before the next plane's
        // factors so that waiting for them does not wait for those too
        const int zo = zz - R;
        const int y = tl.yb + ly, x = tl.xb + lx;
        const int idx = out_idx(zo);
        const float eJ = atlas[tl.chan * astr + idx];
        const float eI = wimg[tl.chan * wstr + idx];
        // fused: the image corners around x + u (zero padding applied when
        // they are used), then u of the next plane's output voxel
        float2 cr[4];  // corner rows (a, b): the pair (jj, jj + 1) along d2
        float ct[3];
        unsigned cmask = 0u, chalf = 0u;
        if (FUSED) {
          const int zc = min(max(zo, tl.z0), g.d0 - 1);
          int ci[3];
          cell_zero(zc, sane(nu[0]), ci[0], ct[0]);
          cell_zero(oy, sane(nu[1]), ci[1], ct[1]);
          cell_zero(ox, sane(nu[2]), ci[2], ct[2]);
          const int dims[3] = {g.d0, g.d1, g.d2};
          int lo[3], hi[3];
          unsigned inl = 0u, inh = 0u;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            lo[d] = min(max(ci[d], 0), dims[d] - 1);
            hi[d] = min(max(ci[d] + 1, 0), dims[d] - 1);
            inl |= static_cast<unsigned>(ci[d] >= 0 && ci[d] < dims[d]) << d;
            inh |= static_cast<unsigned>(ci[d] + 1 >= 0 && ci[d] + 1 < dims[d]) << d;
          }
          // one 8-byte load per corner row: jj = clamp(i2, 0, D2 - 2) holds
          // both in-range corners; bit e of chalf picks the half of corner e
          const int jj = min(max(ci[2], 0), g.d2 - 2);
          chalf = static_cast<unsigned>(ci[2] != jj) | (static_cast<unsigned>(ci[2] + 1 != jj) << 1);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int j0 = (r >> 1) ? hi[0] : lo[0], j1 = (r & 1) ? hi[1] : lo[1];
            cr[r] = ld_pair(Io + (j0 * g.d1 + j1) * g.d2 + jj);
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int ka = k >> 2, kb = (k >> 1) & 1, kc = k & 1;
            const bool ok = ((ka ? inh : inl) & 1u) && ((kb ? inh : inl) & 2u) &&
                            ((kc ? inh : inl) & 4u);
            cmask |= static_cast<unsigned>(ok) << k;
          }
          const int in = out_idx(zo + 1);
#pragma unroll
          for (int c = 0; c < 3; ++c) nu[c] = uf[static_cast<size_t>(c) * g.V + in];
        }
        load_plane(p + 1);  // past the chunk: clamped, never staged
        __syncthreads();
        // row sums along x, two neighbouring outputs per thread (sliding)
        for (int e = tid; e < HY * (kTX / 2); e += kNT) {
          const int hy = e / (kTX / 2), cx = 2 * (e - hy * (kTX / 2));
          const int o = hy * kTX + cx;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            // aligned 8-byte pairs
            const float2* pr = reinterpret_cast<const float2*>(&sIn[c][hy * HX + cx]);
            double t[W + 1];
#pragma unroll
            for (int q = 0; q < (W + 1) / 2; ++q) {
              const float2 a = pr[q];
              t[2 * q] = a.x;
              t[2 * q + 1] = a.y;
            }
            double a = 0.0;
#pragma unroll
            for (int k = 0; k < W; ++k) a += t[k];
            sr[c][o] = a;
            sr[c][o + 1] = a + (t[W] - t[0]);
          }
        }
        __syncthreads();
        column_sums<W, 4>(&sr[0][0], &sc[0][0], tid);
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double P = sc[c][ly * kTX + lx];
          S[c] += P - ring[j][c];
          ring[j][c] = P;
        }
        if (zo >= tl.z0 && y < g.d1 && x < g.d2) {
          const size_t vidx = static_cast<size_t>(tl.chan) * g.V + idx;
          const double Jc = eJ;
          const double Ic = eI;
          const double gI = neg_inv_v * (Jc * S[0] - S[1] - Ic * S[2] + S[3]);
          if (!FUSED) {
            gw[vidx] = static_cast<float>(gI);
          } else {
            const size_t off = static_cast<size_t>(tl.chan) * 3 * g.V;
            const float* f = uf;
            float cv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const float2 pr = cr[k >> 1];
              const float vk = ((chalf >> (k & 1)) & 1u) ? pr.y : pr.x;
              cv[k] = ((cmask >> k) & 1u) ? vk : 0.0f;
            }
            const Tri t = tri_eval(cv, ct[0], ct[1], ct[2]);
            float r0 = 0.0f, r1 = 0.0f, r2 = 0.0f;
            if (rw.on) {
              r0 = reg_at(f, g, idx, zo, y, x, rw, racc);
              r1 = reg_at(f + g.V, g, idx, zo, y, x, rw, racc);
              r2 = reg_at(f + 2 * g.V, g, idx, zo, y, x, rw, racc);
            }
            const float gf = static_cast<float>(gI);
            float* o = gu + off;
            o[idx] = gf * t.d0 + r0;
            o[g.V + idx] = gf * t.d1 + r1;
            o[2 * g.V + idx] = gf * t.d2 + r2;
          }
        }
        __syncthreads();
      }
    }
  }
  if (FUSED && rw.on) {
    const double tot = block_sum<kNT>(racc, red);
    if (tid == 0) atomicAdd(loss + static_cast<size_t>(tl.chan) * loss_stride, rw.lam * tot);
  }
}

// ------------------------------------------------------------ Gaussian smoother
//
// out = G_sigma * in, separable, weights w[0..2R], replicated border.
struct GaussW {
  float w[17];
};

// A Gaussian block owns 32 x (8 GR) outputs of a plane: thread (lx, r) holds
// the GR consecutive rows r*GR.. of column lx, so each staged value is reused
// by GR outputs along d1 from registers, and the pass along d2 produces four
// adjacent outputs from one run of 16-byte LDS reads.  GR = 4 (32 x 32
// tiles); 2 for the widest radii, whose ring of (2R + 1) x GR plane sums
// would not stay in registers.
constexpr int kGX = 32;
constexpr int gauss_rows(int R) { return R <= 6 ? 4 : 2; }

template <int R>
__global__ __launch_bounds__(kNT) void k_gauss(const float* __restrict__ in,
                                               float* __restrict__ out, MarchGeom mg, GaussW gw) {
  constexpr int kGR = gauss_rows(R), kGY = kNT * kGR / kGX;
  constexpr int W2 = 2 * R + 1, HX = kGX + 2 * R, HY = kGY + 2 * R;
  constexpr int NV = (4 + 2 * R + 3) / 4;  // 16-byte reads per four d2-outputs
  constexpr int SX = kGX - 4 + 4 * NV;     // LDS row stride: >= HX, a multiple of 4
  constexpr int GPR = kGX / 4;             // groups of four outputs per row
  constexpr int NE = (HY * HX + kNT - 1) / kNT;
  __shared__ __align__(16) float sIn[HY * SX];
  __shared__ __align__(16) float sr[HY * kGX];
  const Geom& g = mg.g;
  const Tile tl = march_tile<kGX, kGY>(mg);
  const int tid = threadIdx.x, lx = tid % kGX, y0 = (tid / kGX) * kGR;
  const float* src = in + static_cast<size_t>(tl.chan) * g.V;
  // outputs written by range-checked stores issued on every plane
  const MaskedOut dst = masked_out(out + static_cast<size_t>(tl.chan) * g.V, g.V);
  float ring[W2][kGR];
#pragma unroll
  for (int j = 0; j < W2; ++j)
#pragma unroll
    for (int r = 0; r < kGR; ++r) ring[j][r] = 0.0f;
  // planes walked: the chunk and R on either side, padded to a multiple of
  // W2 so that the unrolled body has no branch around its loads and stores
  const int nplanes = (tl.z1 - tl.z0) + 2 * R;
  const int npad = (nplanes + W2 - 1) / W2 * W2;
  // staged positions: volume offset (replicated border; positions past the
  // staged plane load a clamped voxel that is never staged) and LDS slot
  int eoff[NE], eslot[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = tid + k * kNT;
    const int hy = e / HX, hx = e - hy * HX;
    const int y = min(max(tl.yb - R + hy, 0), g.d1 - 1);
    const int x = min(max(tl.xb - R + hx, 0), g.d2 - 1);
    eoff[k] = y * g.d2 + x;
    eslot[k] = hy * SX + hx;
  }
  // the next plane is loaded into registers while the current one is
  // filtered; every lane loads (a conditional load would be waited for at
  // once)
  float pre[NE];
  auto load_plane = [&](int p) {
    const int zc = min(max(tl.z0 - R + p, 0), g.d0 - 1);
#pragma unroll
    for (int k = 0; k < NE; ++k)
      pre[k] = ld_at(src, static_cast<uint32_t>(zc * g.plane + eoff[k]));
  };
  load_plane(0);
  const int x = tl.xb + lx;
  for (int base = 0; base < npad; base += W2) {
#pragma unroll
    for (int j = 0; j < W2; ++j) {
      const int p = base + j;
      {
#pragma unroll
        for (int k = 0; k < NE; ++k)
          if (tid + k * kNT < HY * HX) sIn[eslot[k]] = pre[k];
        load_plane(p + 1);
        __syncthreads();
        // along d2: four adjacent outputs per work item
        for (int e = tid; e < HY * GPR; e += kNT) {
          const int hy = e / GPR, x0 = (e - hy * GPR) * 4;
          const float4* row = reinterpret_cast<const float4*>(sIn + hy * SX + x0);
          float t[4 * NV];
#pragma unroll
          for (int q = 0; q < NV; ++q) {
            const float4 a = row[q];
            t[4 * q] = a.x;
            t[4 * q + 1] = a.y;
            t[4 * q + 2] = a.z;
            t[4 * q + 3] = a.w;
          }
          float o[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float a = 0.0f;
#pragma unroll
            for (int k = 0; k < W2; ++k) a += gw.w[k] * t[i + k];
            o[i] = a;
          }
          *reinterpret_cast<float4*>(sr + hy * kGX + x0) = make_float4(o[0], o[1], o[2], o[3]);
        }
        __syncthreads();
        // along d1 from one column run in registers, then along d0 from the ring
        float c[kGR + 2 * R];
#pragma unroll
        for (int i = 0; i < kGR + 2 * R; ++i) c[i] = sr[(y0 + i) * kGX + lx];
#pragma unroll
        for (int r = 0; r < kGR; ++r) {
          float a = 0.0f;
#pragma unroll
          for (int k = 0; k < W2; ++k) a += gw.w[k] * c[r + k];
          ring[j][r] = a;
        }
        const int zo = tl.z0 - 2 * R + p;
        const bool zout = p >= 2 * R && zo < tl.z1 && x < g.d2;
#pragma unroll
        for (int r = 0; r < kGR; ++r) {
          const int y = tl.yb + y0 + r;
          float o = 0.0f;
#pragma unroll
          for (int k = 0; k < W2; ++k) o += gw.w[k] * ring[(j + 1 + k) % W2][r];
          store_masked(dst, static_cast<uint32_t>((zo * g.d1 + y) * g.d2 + x), o,
                       zout && y < g.d1);
        }
      }
    }
  }
}

// Operand strides between channels: the image operand advances by wstr
// and the reference by astr elements (V and 0 for warped subjects against one
// atlas; 0 and V for the atlas against each warped subject).
struct Strides {
  long long w, a;
};

template <int W>
void lncc_fwd_w(const float* w, const float* atlas, float* fields, double* loss, int loss_stride,
                double eps, const Geom& g, int n, Strides sd, hipStream_t st) {
  const MarchGeom mg = make_march(g, n, W / 2);
  const double neg_inv_v = -1.0 / g.V;
  if (fields)
    hipLaunchKernelGGL((k_lncc_fwd<W, true>), dim3(mg.total), dim3(kNT), 0, st, w, atlas, fields,
                       loss, loss_stride, mg, eps, neg_inv_v, sd.w, sd.a);
  else
    hipLaunchKernelGGL((k_lncc_fwd<W, false>), dim3(mg.total), dim3(kNT), 0, st, w, atlas, fields,
                       loss, loss_stride, mg, eps, neg_inv_v, sd.w, sd.a);
}

template <int W, bool FUSED>
void lncc_bwd_w(const float* fields, const float* w, const float* atlas, float* gw,
                const float* img, const float* u, float* gu, double* loss, int loss_stride,
                const RegW& rw, const Geom& g, int n, Strides sd, hipStream_t st) {
  const MarchGeom mg = make_march(g, n, W / 2);
  hipLaunchKernelGGL((k_lncc_bwd<W, FUSED>), dim3(mg.total), dim3(kNT), 0, st, fields, w, atlas,
                     gw, img, u, gu, loss, loss_stride, rw, mg, -1.0 / g.V, sd.w, sd.a);
}

bool lncc_fwd_dispatch(const float* w, const float* atlas, float* fields, double* loss,
                       int loss_stride, int win, double eps, const Geom& g, int n, Strides sd,
                       hipStream_t st) {
  switch (win) {
    case 3: lncc_fwd_w<3>(w, atlas, fields, loss, loss_stride, eps, g, n, sd, st); return true;
    case 5: lncc_fwd_w<5>(w, atlas, fields, loss, loss_stride, eps, g, n, sd, st); return true;
    case 7: lncc_fwd_w<7>(w, atlas, fields, loss, loss_stride, eps, g, n, sd, st); return true;
    case 9: lncc_fwd_w<9>(w, atlas, fields, loss, loss_stride, eps, g, n, sd, st); return true;
    case 11: lncc_fwd_w<11>(w, atlas, fields, loss, loss_stride, eps, g, n, sd, st); return true;
    default: return false;
  }
}

template <bool FUSED>
bool lncc_bwd_dispatch(const float* fields, const float* w, const float* atlas, float* gw,
                       const float* img, const float* u, float* gu, double* loss, int loss_stride,
                       const RegW& rw, int win, const Geom& g, int n, Strides sd, hipStream_t st) {
  switch (win) {
    case 3: lncc_bwd_w<3, FUSED>(fields, w, atlas, gw, img, u, gu, loss, loss_stride, rw, g, n, sd, st); return true;
    case 5: lncc_bwd_w<5, FUSED>(fields, w, atlas, gw, img, u, gu, loss, loss_stride, rw, g, n, sd, st); return true;
    case 7: lncc_bwd_w<7, FUSED>(fields, w, atlas, gw, img, u, gu, loss, loss_stride, rw, g, n, sd, st); return true;
    case 9: lncc_bwd_w<9, FUSED>(fields, w, atlas, gw, img, u, gu, loss, loss_stride, rw, g, n, sd, st); return true;
    case 11: lncc_bwd_w<11, FUSED>(fields, w, atlas, gw, img, u, gu, loss, loss_stride, rw, g, n, sd, st); return true;
    default: return false;
  }
}

template <int R>
void gauss_r(const float* in, float* out, const GaussW& gw, const Geom& g, int nchan,
             hipStream_t st) {
  const MarchGeom mg = make_march(g, nchan, R, kGX, kNT * gauss_rows(R) / kGX);
  hipLaunchKernelGGL((k_gauss<R>), dim3(mg.total), dim3(kNT), 0, st, in, out, mg, gw);
}

}  // namespace

bool lncc_window_supported(int win) {
  return win == 3 || win == 5 || win == 7 || win == 9 || win == 11;
}

bool launch_lncc_fwd(const float* w, const float* atlas, float* fields, double* loss,
                     int loss_stride, int win, double eps, const Geom& g, int n, hipStream_t st) {
  if (!lncc_window_supported(win)) return false;
  prof_begin(st, KC_LNCC_FWD);
  lncc_fwd_dispatch(w, atlas, fields, loss, loss_stride, win, eps, g, n, Strides{g.V, 0}, st);
  prof_end(st, KC_LNCC_FWD);
  return true;
}

bool launch_lncc_atlas_grad(const float* warped, const float* atlas, float* fields, float* ga,
                            double* loss, int loss_stride, int win, double eps, const Geom& g,
                            int n, hipStream_t st) {
  if (!lncc_window_supported(win)) return false;
  RegW none{};
  const Strides sd{0, g.V};
  prof_begin(st, KC_LNCC_FWD);
  lncc_fwd_dispatch(atlas, warped, fields, loss, loss_stride, win, eps, g, n, sd, st);
  prof_end(st, KC_LNCC_FWD);
  prof_begin(st, KC_LNCC_BWD);
  lncc_bwd_dispatch<false>(fields, atlas, warped, ga, nullptr, nullptr, nullptr, nullptr, 0, none,
                           win, g, n, sd, st);
  prof_end(st, KC_LNCC_BWD);
  return true;
}

bool launch_lncc_bwd(const float* fields, const float* w, const float* atlas, float* gw, int win,
                     const Geom& g, int n, hipStream_t st) {
  if (!lncc_window_supported(win)) return false;
  RegW none{};
  prof_begin(st, KC_LNCC_BWD);
  lncc_bwd_dispatch<false>(fields, w, atlas, gw, nullptr, nullptr, nullptr, nullptr, 0, none, win,
                           g, n, Strides{g.V, 0}, st);
  prof_end(st, KC_LNCC_BWD);
  return true;
}

bool launch_lncc_bwd_fused(const float* fields, const float* w, const float* atlas,
                           const float* img, const float* u, float* gu, double* loss,
                           int loss_stride, const RegW& rw, int win, const Geom& g, int n,
                           hipStream_t st) {
  if (!lncc_window_supported(win)) return false;
  prof_begin(st, KC_LNCC_BWD);
  lncc_bwd_dispatch<true>(fields, w, atlas, nullptr, img, u, gu, loss, loss_stride, rw, win, g, n,
                          Strides{g.V, 0}, st);
  prof_end(st, KC_LNCC_BWD);
  return true;
}

int gauss_radius(float sigma) { return static_cast<int>(3.0f * sigma + 0.5f); }

bool launch_gauss(const float* in, float* out, float sigma, const Geom& g, int nchan,
                  hipStream_t st) {
  const int r = gauss_radius(sigma);
  if (r < 1 || r > 8) return false;
  GaussW gw{};
  double w[17];
  double sum = 0.0;
  for (int k = -r; k <= r; ++k) {
    w[k + r] = std::exp(-0.5 * k * k / (static_cast<double>(sigma) * sigma));
    sum += w[k + r];
  }
  for (int k = 0; k < 2 * r + 1; ++k) gw.w[k] = static_cast<float>(w[k] / sum);
  prof_begin(st, KC_GAUSS);
  switch (r) {
    case 1: gauss_r<1>(in, out, gw, g, nchan, st); break;
    case 2: gauss_r<2>(in, out, gw, g, nchan, st); break;
    case 3: gauss_r<3>(in, out, gw, g, nchan, st); break;
    case 4: gauss_r<4>(in, out, gw, g, nchan, st); break;
    case 5: gauss_r<5>(in, out, gw, g, nchan, st); break;
    case 6: gauss_r<6>(in, out, gw, g, nchan, st); break;
    case 7: gauss_r<7>(in, out, gw, g, nchan, st); break;
    default: gauss_r<8>(in, out, gw, g, nchan, st); break;
  }
  prof_end(st, KC_GAUSS);
  return true;
}

}  // namespace darc
