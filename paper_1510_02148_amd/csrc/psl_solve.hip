// libpsl solve path: deflated Jacobi-PCG (DEF1 form) on P1 A xhat = P1 b inside a float64
// refinement loop, plus the stand-alone operator entry points (A p, P1 r).
//
// One CG iteration is four launches on the caller's stream:
//   stencil   q = A p (flux form), partial (p, q) and Z^T q per tile
//             [last workgroup: s = Z^T q, (p, q) in a fixed order]
//   coarse    e = E^-1 s (dense float64 GEMV), partial s^T e
//             [last workgroup: alpha = rho / ((p, q) - s^T e)]
//   update    rhat = rhat - alpha (q - A Z e) [- A Z E^-1 Z^T rhat when re-projecting],
//             xhat += alpha p, partial (rhat, M^-1 rhat), ||rhat||^2 (and Z^T rhat)
//             [last workgroup: beta, rho, convergence / failure flags, iteration count]
// A Z v is evaluated only on cells with a cut face, in flux form sum T (v_l(i) - v_l(j)).
//   direction p = M^-1 rhat + beta p
// Every reduction is a fixed-order tree, so reruns with the same tiling are bit-identical.
// A finished solve raises a device flag that makes every later launch return at once, so
// the host enqueues several iterations between convergence checks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "psl_internal.hpp"

using psl::kBlock;
using psl::kMaxSlots;
using psl::Scalars;
using psl::Tile;

namespace {

constexpr int kTileMax = 2048;       // cells per tile (LDS correction buffer size)
constexpr int kCoarseRows = 16;      // GEMV rows per workgroup
constexpr int kSChunk = 4096;        // s entries staged in LDS per pass

struct Geo {
  int nx, ny, nz;
  int ntiles;
  const Tile* tiles;
};

// Workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous run of tiles
// (a slab of the grid) so that neighbouring tiles share an L2.
__device__ inline int tile_of_block(int b, int ntiles) {
  const int per = ntiles / 8, rem = ntiles % 8;
  const int x = b % 8, k = b / 8;
  return x * per + min(x, rem) + k;
}

__device__ inline void cell_coords(const Tile& T, int j, float inv_sx, float inv_sxy, int& ix,
                                   int& iy, int& iz) {
  const int sxy = T.sx * T.sy;
  const int lz = psl::div_small(j, sxy, inv_sxy);
  const int rem = j - lz * sxy;
  const int ly = psl::div_small(rem, T.sx, inv_sx);
  ix = T.x0 + rem - ly * T.sx;
  iy = T.y0 + ly;
  iz = T.z0 + lz;
}

// Last-workgroup election: every block calls this once after publishing its partials
// (thread 0 wrote them). Returns true in all threads of the last block to arrive, which
// then sees every other block's partials. The counter is reset by that last block.
__device__ inline bool last_block(uint32_t* counter) {
  __shared__ int am_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t prev = atomicAdd(counter, 1u);
    am_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (am_last) {
    __threadfence();
    if (threadIdx.x == 0) *counter = 0;
  }
  return am_last;
}

// Fixed-order sum of v[i*stride + off] over i < count by one workgroup.
__device__ inline double block_reduce_strided(const double* v, int count, int stride, int off,
                                              double* lds) {
  double acc[1] = {0.0};
  for (int i = threadIdx.x; i < count; i += kBlock) acc[0] += v[int64_t(i) * stride + off];
  psl::block_sum<1>(acc, lds);
  return acc[0];
}

// s[l] = sum of the (tile, slot) partials of label l, in list order.
__device__ inline void reduce_labels(const double* part, const int32_t* lab_ptr,
                                     const int32_t* lab_part, double* s, int d) {
  for (int l = threadIdx.x; l < d; l += kBlock) {
    double acc = 0.0;
    for (int i = lab_ptr[l]; i < lab_ptr[l + 1]; ++i) acc += part[lab_part[i]];
    s[l] = acc;
  }
}

// ---------------------------------------------------------------------------------------
// stencil pass. MODE 0: out = A in (inner CG, R = float or double), reductions (in, out)
// and Z^T out. MODE 1: out = b - A in (float64 outer residual), reductions ||out||^2 and
// Z^T out.
// ---------------------------------------------------------------------------------------
template <typename R, int MODE, int NS, int RP>
__global__ void __launch_bounds__(kBlock)
    k_stencil(Geo g, const R* __restrict__ Tx, const R* __restrict__ Ty, const R* __restrict__ Tz,
              const R* __restrict__ in, const double* __restrict__ b, R* __restrict__ out,
              const uint8_t* __restrict__ slot, double* zq_part, const double* zr_part,
              double* red_part, const int32_t* lab_ptr, const int32_t* lab_part, double* s,
              double* sr, int d, Scalars* sc, int check_done) {
  __shared__ double lds[(NS + 1) * (kBlock / psl::kWave)];
  if (check_done && sc->done) return;
  const int t = tile_of_block(blockIdx.x, g.ntiles);
  const Tile T = g.tiles[t];
  const float inv_sx = 1.0f / T.sx, inv_sxy = 1.0f / (T.sx * T.sy);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int sxy = nx * ny;
  double acc[NS + 1];
#pragma unroll
  for (int k = 0; k <= NS; ++k) acc[k] = 0.0;
  for (int j = threadIdx.x; j < T.ncell; j += kBlock) {
    int ix, iy, iz;
    cell_coords(T, j, inv_sx, inv_sxy, ix, iy, iz);
    const int c = ix + nx * (iy + ny * iz);
    const int fx = ix + (nx + 1) * (iy + ny * iz);
    const int fy = ix + nx * (iy + (ny + 1) * iz);
    const R pc = in[c];
    const R pw = ix > 0 ? in[c - 1] : R(0);
    const R pe = ix < nx - 1 ? in[c + 1] : R(0);
    const R ps = iy > 0 ? in[c - nx] : R(0);
    const R pn = iy < ny - 1 ? in[c + nx] : R(0);
    const R pb = iz > 0 ? in[c - sxy] : R(0);
    const R pt = iz < nz - 1 ? in[c + sxy] : R(0);
    R ap = Tx[fx] * (pc - pw);
    ap += Tx[fx + 1] * (pc - pe);
    ap += Ty[fy] * (pc - ps);
    ap += Ty[fy + nx] * (pc - pn);
    ap += Tz[c] * (pc - pb);
    ap += Tz[c + sxy] * (pc - pt);
    double v;
    if (MODE == 0) {
      out[c] = ap;
      v = double(ap);
      acc[NS] += double(pc) * v;
    } else {
      const double r = b[c] - double(ap);
      out[c] = R(r);
      v = r;
      acc[NS] += r * r;
    }
    const int sl = slot[c];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] += (sl == k) ? v : 0.0;
  }
  psl::block_sum<NS + 1>(acc, lds);
  if (threadIdx.x == 0) {
    for (int k = 0; k < T.nslot; ++k) zq_part[t * kMaxSlots + k] = acc[k];
    red_part[t * 4 + MODE] = acc[NS];
  }
  if (!last_block(&sc->cnt_a)) return;
  __shared__ double lds2[kBlock / psl::kWave];
  reduce_labels(zq_part, lab_ptr, lab_part, s, d);
  if (RP) reduce_labels(zr_part, lab_ptr, lab_part, sr, d);  // Z^T rhat from the update pass
  const double tot = block_reduce_strided(red_part, g.ntiles, 4, MODE, lds2);
  if (threadIdx.x == 0) {
    if (MODE == 0)
      sc->pq = tot;
    else
      sc->rr = tot;
  }
}

// ---------------------------------------------------------------------------------------
// coarse solve e = E^-1 s. MODE 0 (inner): alpha = rho / ((p, q) - s^T e) by the last
// block, with breakdown / non-finite detection. MODE 1: e only.
// ---------------------------------------------------------------------------------------
template <int MODE, int RP>
__global__ void __launch_bounds__(kBlock)
    k_coarse(const double* __restrict__ Einv, const double* __restrict__ s,
             const double* __restrict__ sr, double* e, double* er, double* se_part, int d,
             Scalars* sc, int check_done) {
  __shared__ double ss[(RP ? 2 : 1) * kSChunk];
  __shared__ double lds[kBlock / psl::kWave];
  if (check_done && sc->done) return;
  const int lane = threadIdx.x & (psl::kWave - 1), w = threadIdx.x / psl::kWave;
  constexpr int kRowsPerWave = kCoarseRows / (kBlock / psl::kWave);
  const int row0 = blockIdx.x * kCoarseRows + w * kRowsPerWave;
  double racc[kRowsPerWave], racc2[kRowsPerWave];
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) racc[r] = racc2[r] = 0.0;
  for (int c0 = 0; c0 < d; c0 += kSChunk) {
    const int c1 = min(d, c0 + kSChunk);
    __syncthreads();
    for (int c = c0 + threadIdx.x; c < c1; c += kBlock) {
      ss[c - c0] = s[c];
      if (RP) ss[kSChunk + c - c0] = sr[c];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
      const int row = row0 + r;
      if (row < d) {
        const double* erow = Einv + int64_t(row) * d;
        double a = 0.0, a2 = 0.0;
        for (int c = c0 + lane; c < c1; c += psl::kWave) {
          const double m = erow[c];
          a += m * ss[c - c0];
          if (RP) a2 += m * ss[kSChunk + c - c0];
        }
        racc[r] += a;
        racc2[r] += a2;
      }
    }
  }
  double se[1] = {0.0};
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    const double v = psl::wave_sum(racc[r]);
    const double v2 = RP ? psl::wave_sum(racc2[r]) : 0.0;
    const int row = row0 + r;
    if (row < d) {
      if (lane == 0) {
        e[row] = v;
        if (RP) er[row] = v2;
      }
      se[0] += (lane == 0) ? v * s[row] : 0.0;
    }
  }
  psl::block_sum<1>(se, lds);
  if (threadIdx.x == 0) se_part[blockIdx.x] = se[0];
  if (!last_block(&sc->cnt_b)) return;
  const double tot = block_reduce_strided(se_part, gridDim.x, 1, 0, lds);
  if (MODE == 0 && threadIdx.x == 0) {
    sc->se = tot;
    const double pw = sc->pq - tot;
    if (!(pw > 0.0)) {
      sc->status = (pw == pw && fabs(pw) < INFINITY) ? PSL_EBREAKDOWN : PSL_ENONFINITE;
      sc->done = 1;
      sc->alpha = 0.0;
    } else {
      sc->alpha = sc->rho / pw;
    }
  }
}

// Per tile: corr[local cell] = (A Z v)_cell = sum over its cut faces of T (v_l - v_other),
// v = ca * e + cb * e2 (e2 may be null), v_other = 0 across an outer face; 0 elsewhere.
template <typename CT>
__device__ inline void tile_correction(const Tile& T, int t, const int32_t* az_ptr,
                                       const int32_t* az_cell, const int32_t* az_lab,
                                       const int32_t* az_oth, const CT* az_t, const double* e,
                                       double ca, const double* e2, double cb, double* corr) {
  for (int j = threadIdx.x; j < T.ncell; j += kBlock) corr[j] = 0.0;
  __syncthreads();
  const int a = az_ptr[t], b = az_ptr[t + 1];
  for (int k = a + threadIdx.x; k < b; k += kBlock) {
    const int32_t cw = az_cell[k];
    if (cw >= 0) continue;  // not the first face of its cell
    const int ls = az_lab[k];
    const double vs = ca * e[ls] + (e2 ? cb * e2[ls] : 0.0);
    double acc = 0.0;
    int m = k;
    do {
      const int lo = az_oth[m];
      const double vo = lo < 0 ? 0.0 : ca * e[lo] + (e2 ? cb * e2[lo] : 0.0);
      acc += double(az_t[m]) * (vs - vo);
      ++m;
    } while (m < b && az_cell[m] >= 0);
    corr[cw & 0x7fffffff] = acc;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------------
// CG update pass: rhat = rhat - alpha q + A Z (alpha e - er) (er = E^-1 Z^T rhat when
// re-projecting, else 0), i.e. rhat <- P1 rhat - alpha P1 A p; xhat += alpha p;
// y = M^-1 rhat; reductions (rhat, y), ||rhat||^2 and, when re-projecting, Z^T rhat.
// The last block closes the iteration.
// ---------------------------------------------------------------------------------------
template <typename R, int NS, int RP>
__global__ void __launch_bounds__(kBlock)
    k_update(Geo g, const R* __restrict__ q, const R* __restrict__ p, R* __restrict__ rh,
             R* __restrict__ xh, const R* __restrict__ invd, const uint8_t* __restrict__ slot,
             const int32_t* az_ptr, const int32_t* az_cell, const int32_t* az_lab,
             const int32_t* az_oth, const R* az_t, const double* __restrict__ e,
             const double* __restrict__ er, double* zr_part, double* red_part, Scalars* sc) {
  __shared__ double corr[kTileMax];
  __shared__ double lds[(NS + 2) * (kBlock / psl::kWave)];
  if (sc->done) return;
  const int t = tile_of_block(blockIdx.x, g.ntiles);
  const Tile T = g.tiles[t];
  const double alpha_d = sc->alpha;
  tile_correction(T, t, az_ptr, az_cell, az_lab, az_oth, az_t, e, alpha_d, RP ? er : nullptr,
                  -1.0, corr);
  const float inv_sx = 1.0f / T.sx, inv_sxy = 1.0f / (T.sx * T.sy);
  const R alpha = R(alpha_d);
  double acc[NS + 2];
#pragma unroll
  for (int k = 0; k < NS + 2; ++k) acc[k] = 0.0;
  for (int j = threadIdx.x; j < T.ncell; j += kBlock) {
    int ix, iy, iz;
    cell_coords(T, j, inv_sx, inv_sxy, ix, iy, iz);
    const int c = ix + g.nx * (iy + g.ny * iz);
    const R r = rh[c] - alpha * q[c] + R(corr[j]);
    rh[c] = r;
    xh[c] += alpha * p[c];
    const double rd = double(r);
    acc[NS] += rd * double(r * invd[c]);
    acc[NS + 1] += rd * rd;
    if (RP) {
      const int sl = slot[c];
#pragma unroll
      for (int k = 0; k < NS; ++k) acc[k] += (sl == k) ? rd : 0.0;
    }
  }
  psl::block_sum<NS + 2>(acc, lds);
  if (threadIdx.x == 0) {
    red_part[t * 4 + 2] = acc[NS];
    red_part[t * 4 + 3] = acc[NS + 1];
    if (RP)
      for (int k = 0; k < T.nslot; ++k) zr_part[t * kMaxSlots + k] = acc[k];
  }
  if (!last_block(&sc->cnt_c)) return;
  const double ry = block_reduce_strided(red_part, g.ntiles, 4, 2, lds);
  const double rr = block_reduce_strided(red_part, g.ntiles, 4, 3, lds);
  if (threadIdx.x == 0) {
    sc->iters += 1;
    sc->rr = rr;
    if (!(fabs(ry) < INFINITY) || !(rr < INFINITY)) {
      sc->status = PSL_ENONFINITE;
      sc->done = 1;
    } else {
      sc->beta = ry / sc->rho;
      sc->rho = ry;
      if (rr <= sc->goal2 || sc->iters >= sc->maxit) sc->done = 1;
    }
  }
}

// p = M^-1 rhat + beta p
template <typename R>
__global__ void k_direction(int n, const R* __restrict__ rh, const R* __restrict__ invd,
                            R* __restrict__ p, const Scalars* sc) {
  if (sc->done) return;
  const R beta = R(sc->beta);
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
    p[c] = rh[c] * invd[c] + beta * p[c];
}

// Inner start: rhat = sigma r (cast to R), xhat = 0, p = M^-1 rhat; rho = (rhat, p),
// ||rhat||^2 (and Z^T rhat partials when re-projecting); done if already below the goal.
template <typename R, int NS, int RP>
__global__ void __launch_bounds__(kBlock)
    k_inner_init(Geo g, const double* __restrict__ r, R* __restrict__ rh, R* __restrict__ xh,
                 R* __restrict__ p, const R* __restrict__ invd,
                 const uint8_t* __restrict__ slot, double* zr_part, double* red_part,
                 Scalars* sc) {
  __shared__ double lds[(NS + 2) * (kBlock / psl::kWave)];
  const int t = tile_of_block(blockIdx.x, g.ntiles);
  const Tile T = g.tiles[t];
  const float inv_sx = 1.0f / T.sx, inv_sxy = 1.0f / (T.sx * T.sy);
  const double sigma = sc->sigma;
  double acc[NS + 2];
#pragma unroll
  for (int k = 0; k < NS + 2; ++k) acc[k] = 0.0;
  for (int j = threadIdx.x; j < T.ncell; j += kBlock) {
    int ix, iy, iz;
    cell_coords(T, j, inv_sx, inv_sxy, ix, iy, iz);
    const int c = ix + g.nx * (iy + g.ny * iz);
    const R rv = R(sigma * r[c]);
    const R y = rv * invd[c];
    rh[c] = rv;
    xh[c] = R(0);
    p[c] = y;
    const double rd = double(rv);
    acc[NS] += rd * double(y);
    acc[NS + 1] += rd * rd;
    if (RP) {
      const int sl = slot[c];
#pragma unroll
      for (int k = 0; k < NS; ++k) acc[k] += (sl == k) ? rd : 0.0;
    }
  }
  psl::block_sum<NS + 2>(acc, lds);
  if (threadIdx.x == 0) {
    red_part[t * 4 + 2] = acc[NS];
    red_part[t * 4 + 3] = acc[NS + 1];
    if (RP)
      for (int k = 0; k < T.nslot; ++k) zr_part[t * kMaxSlots + k] = acc[k];
  }
  if (!last_block(&sc->cnt_c)) return;
  const double ry = block_reduce_strided(red_part, g.ntiles, 4, 2, lds);
  const double rr = block_reduce_strided(red_part, g.ntiles, 4, 3, lds);
  if (threadIdx.x == 0) {
    sc->rho = ry;
    sc->rr = rr;
    sc->iters = 0;
    if (!(rr < INFINITY)) {
      sc->status = PSL_ENONFINITE;
      sc->done = 1;
    } else if (rr <= sc->goal2 || sc->maxit <= 0) {
      sc->done = 1;
    }
  }
}

// Outer deflation: x += Z e (if x != null), rout = rin - A Z e, ||rout||^2 -> sc->rr.
__global__ void __launch_bounds__(kBlock)
    k_outer_deflate(Geo g, double* __restrict__ x, const double* rin, double* rout,
                    const int32_t* __restrict__ labels, const int32_t* az_ptr,
                    const int32_t* az_cell, const int32_t* az_lab, const int32_t* az_oth,
                    const double* az_t, const double* __restrict__ e, double* red_part,
                    Scalars* sc) {
  __shared__ double corr[kTileMax];
  __shared__ double lds[kBlock / psl::kWave];
  const int t = tile_of_block(blockIdx.x, g.ntiles);
  const Tile T = g.tiles[t];
  tile_correction(T, t, az_ptr, az_cell, az_lab, az_oth, az_t, e, 1.0,
                  static_cast<const double*>(nullptr), 0.0, corr);
  const float inv_sx = 1.0f / T.sx, inv_sxy = 1.0f / (T.sx * T.sy);
  double acc[1] = {0.0};
  for (int j = threadIdx.x; j < T.ncell; j += kBlock) {
    int ix, iy, iz;
    cell_coords(T, j, inv_sx, inv_sxy, ix, iy, iz);
    const int c = ix + g.nx * (iy + g.ny * iz);
    if (x) x[c] += e[labels[c]];
    const double r = rin[c] - corr[j];
    rout[c] = r;
    acc[0] += r * r;
  }
  psl::block_sum<1>(acc, lds);
  if (threadIdx.x == 0) red_part[t * 4 + 1] = acc[0];
  if (!last_block(&sc->cnt_c)) return;
  const double rr = block_reduce_strided(red_part, g.ntiles, 4, 1, lds);
  if (threadIdx.x == 0) sc->rr = rr;
}

// Z^T v partials only (for psl_deflate), last block -> s.
template <int NS>
__global__ void __launch_bounds__(kBlock)
    k_zt(Geo g, const double* __restrict__ v, const uint8_t* __restrict__ slot, double* zq_part,
         const int32_t* lab_ptr, const int32_t* lab_part, double* s, int d, Scalars* sc) {
  __shared__ double lds[NS * (kBlock / psl::kWave)];
  const int t = tile_of_block(blockIdx.x, g.ntiles);
  const Tile T = g.tiles[t];
  const float inv_sx = 1.0f / T.sx, inv_sxy = 1.0f / (T.sx * T.sy);
  double acc[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc[k] = 0.0;
  for (int j = threadIdx.x; j < T.ncell; j += kBlock) {
    int ix, iy, iz;
    cell_coords(T, j, inv_sx, inv_sxy, ix, iy, iz);
    const int c = ix + g.nx * (iy + g.ny * iz);
    const double val = v[c];
    const int sl = slot[c];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] += (sl == k) ? val : 0.0;
  }
  psl::block_sum<NS>(acc, lds);
  if (threadIdx.x == 0)
    for (int k = 0; k < T.nslot; ++k) zq_part[t * kMaxSlots + k] = acc[k];
  if (!last_block(&sc->cnt_a)) return;
  reduce_labels(zq_part, lab_ptr, lab_part, s, d);
}

// x += scale * xhat (float64 accumulation of an inner correction)
template <typename R>
__global__ void k_accumulate(int n, double* __restrict__ x, const R* __restrict__ xh,
                             const Scalars* sc) {
  const double scale = sc->rnorm;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
    x[c] += scale * double(xh[c]);
}

__global__ void k_set_inner(Scalars* sc, double goal2, int maxit) {
  sc->rnorm = sqrt(sc->rr);
  sc->sigma = sc->rnorm > 0.0 ? 1.0 / sc->rnorm : 0.0;
  sc->goal2 = goal2;
  sc->maxit = maxit;
  sc->done = 0;
  sc->iters = 0;
  sc->status = 0;
}

__global__ void k_reset(Scalars* sc) {
  sc->done = 0;
  sc->iters = 0;
  sc->status = 0;
  sc->cnt_a = sc->cnt_b = sc->cnt_c = 0;
}

// ||v||^2 -> sc->bnorm2 and finiteness (tiles; used for b and x0)
__global__ void __launch_bounds__(kBlock)
    k_norm2(Geo g, const double* __restrict__ v, double* red_part, Scalars* sc, int into_b) {
  __shared__ double lds[kBlock / psl::kWave];
  const int t = tile_of_block(blockIdx.x, g.ntiles);
  const Tile T = g.tiles[t];
  const float inv_sx = 1.0f / T.sx, inv_sxy = 1.0f / (T.sx * T.sy);
  double acc[1] = {0.0};
  for (int j = threadIdx.x; j < T.ncell; j += kBlock) {
    int ix, iy, iz;
    cell_coords(T, j, inv_sx, inv_sxy, ix, iy, iz);
    const double val = v[ix + g.nx * (iy + g.ny * iz)];
    acc[0] += val * val;
  }
  psl::block_sum<1>(acc, lds);
  if (threadIdx.x == 0) red_part[t * 4 + 0] = acc[0];
  if (!last_block(&sc->cnt_a)) return;
  const double tot = block_reduce_strided(red_part, g.ntiles, 4, 0, lds);
  if (threadIdx.x == 0) {
    if (into_b)
      sc->bnorm2 = tot;
    else
      sc->rr = tot;
  }
}

__global__ void k_zero(double* x, int n) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
    x[c] = 0.0;
}

// ---------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------
inline Geo geo(const psl_ctx* c) { return Geo{c->nx, c->ny, c->nz, c->ntiles, c->tiles}; }

inline unsigned elem_grid(int64_t n) {
  return static_cast<unsigned>(std::min<int64_t>((n + kBlock - 1) / kBlock, 256 * 64));
}

template <typename R>
struct Prec;
template <>
struct Prec<double> {
  static const double* face(const psl_ctx* c, int a) { return a == 0 ? c->Tx : (a == 1 ? c->Ty : c->Tz); }
  static const double* invd(const psl_ctx* c) { return c->invdiag; }
  static const double* azt(const psl_ctx* c) { return c->az_t; }
  static psl::VecSet<double>& vecs(psl_ctx* c) { return c->v64; }
  static hipGraphExec_t& graph(psl_ctx* c) { return c->graph64; }
  static int& graph_key(psl_ctx* c) { return c->graph_chunk64; }
};
template <>
struct Prec<float> {
  static const float* face(const psl_ctx* c, int a) { return a == 0 ? c->Tx32 : (a == 1 ? c->Ty32 : c->Tz32); }
  static const float* invd(const psl_ctx* c) { return c->invdiag32; }
  static const float* azt(const psl_ctx* c) { return c->az_t32; }
  static psl::VecSet<float>& vecs(psl_ctx* c) { return c->v32; }
  static hipGraphExec_t& graph(psl_ctx* c) { return c->graph32; }
  static int& graph_key(psl_ctx* c) { return c->graph_chunk32; }
};

template <typename R>
int ensure_vecs(psl_ctx* c) {
  psl::VecSet<R>& v = Prec<R>::vecs(c);
  if (v.xh) return PSL_OK;
  const size_t bytes = sizeof(R) * size_t(c->n);
  R** ptrs[4] = {&v.xh, &v.rh, &v.p, &v.q};
  for (R** p : ptrs)
    if (psl_internal_alloc(reinterpret_cast<void**>(p), bytes) != PSL_OK) return PSL_ENOMEM;
  return PSL_OK;
}

// Dispatch on the number of label slots per tile (compile-time width of the segmented sums).
template <template <int> class F, typename... A>
void with_ns(int ns, A&&... args) {
  if (ns <= 1)
    F<1>::run(args...);
  else if (ns <= 2)
    F<2>::run(args...);
  else if (ns <= 4)
    F<4>::run(args...);
  else if (ns <= 8)
    F<8>::run(args...);
  else
    F<16>::run(args...);
}

template <typename R, int MODE, int RP>
struct StencilL {
  template <int NS>
  struct F {
    static void run(psl_ctx* c, const R* in, const double* b, R* out, int check_done,
                    hipStream_t st) {
      hipLaunchKernelGGL((k_stencil<R, MODE, NS, RP>), dim3(c->ntiles), dim3(kBlock), 0, st,
                         geo(c), Prec<R>::face(c, 0), Prec<R>::face(c, 1), Prec<R>::face(c, 2),
                         in, b, out, c->slot, c->zq_part, c->zr_part, c->red_part, c->lab_ptr,
                         c->lab_part, c->s, c->sr, c->d, c->sc, check_done);
    }
  };
};

template <typename R, int MODE, int RP = 0>
void launch_stencil(psl_ctx* c, const R* in, const double* b, R* out, int check_done,
                    hipStream_t st) {
  with_ns<StencilL<R, MODE, RP>::template F>(c->nslot_max, c, in, b, out, check_done, st);
}

template <typename R, int RP>
struct UpdateL {
  template <int NS>
  struct F {
    static void run(psl_ctx* c, hipStream_t st) {
      psl::VecSet<R>& v = Prec<R>::vecs(c);
      hipLaunchKernelGGL((k_update<R, NS, RP>), dim3(c->ntiles), dim3(kBlock), 0, st, geo(c),
                         v.q, v.p, v.rh, v.xh, Prec<R>::invd(c), c->slot, c->az_ptr, c->az_cell,
                         c->az_lab, c->az_oth, Prec<R>::azt(c), c->e, c->er, c->zr_part,
                         c->red_part, c->sc);
    }
  };
};

template <typename R, int RP>
struct InitL {
  template <int NS>
  struct F {
    static void run(psl_ctx* c, hipStream_t st) {
      psl::VecSet<R>& v = Prec<R>::vecs(c);
      hipLaunchKernelGGL((k_inner_init<R, NS, RP>), dim3(c->ntiles), dim3(kBlock), 0, st,
                         geo(c), c->r64, v.rh, v.xh, v.p, Prec<R>::invd(c), c->slot,
                         c->zr_part, c->red_part, c->sc);
    }
  };
};

template <int NS>
struct ZtL {
  static void run(psl_ctx* c, const double* r, hipStream_t st) {
    hipLaunchKernelGGL(k_zt<NS>, dim3(c->ntiles), dim3(kBlock), 0, st, geo(c), r, c->slot,
                       c->zq_part, c->lab_ptr, c->lab_part, c->s, c->d, c->sc);
  }
};

template <int MODE, int RP = 0>
void launch_coarse(psl_ctx* c, int check_done, hipStream_t st) {
  const int nbk = (c->d + kCoarseRows - 1) / kCoarseRows;
  hipLaunchKernelGGL((k_coarse<MODE, RP>), dim3(nbk), dim3(kBlock), 0, st, c->Einv, c->s, c->sr,
                     c->e, c->er, c->se_part, c->d, c->sc, check_done);
}

void launch_outer_deflate(psl_ctx* c, double* x, const double* rin, double* rout,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_outer_deflate, dim3(c->ntiles), dim3(kBlock), 0, st, geo(c), x, rin,
                     rout, c->labels, c->az_ptr, c->az_cell, c->az_lab, c->az_oth, c->az_t,
                     c->e, c->red_part, c->sc);
}

// r = b - A x ; then twice: x += Z E^-1 Z^T r, r = P1 r  (||r||^2 -> sc->rr).
// E^-1 is applied as an explicit inverse, whose coarse residual is about kappa(E) u
// ||Z^T r||; when ||Z^T r|| is much larger than ||P1 r|| (a rough start vector, or a
// float32 correction) one projection leaves a Z^T component in r that derails the
// deflated CG. The second projection removes it (its own error is kappa(E) u times an
// already tiny Z^T r).
void enqueue_outer_step(psl_ctx* c, const double* b, double* x, hipStream_t st) {
  launch_stencil<double, 1>(c, x, b, c->r64, 0, st);
  launch_coarse<1>(c, 0, st);
  launch_outer_deflate(c, x, c->r64, c->r64, st);
  with_ns<ZtL>(c->nslot_max, c, c->r64, st);
  launch_coarse<1>(c, 0, st);
  launch_outer_deflate(c, x, c->r64, c->r64, st);
}

// one CG iteration (four launches)
template <typename R, int RP>
void enqueue_iteration(psl_ctx* c, hipStream_t st) {
  psl::VecSet<R>& v = Prec<R>::vecs(c);
  launch_stencil<R, 0, RP>(c, v.p, nullptr, v.q, 1, st);
  launch_coarse<0, RP>(c, 1, st);
  with_ns<UpdateL<R, RP>::template F>(c->nslot_max, c, st);
  hipLaunchKernelGGL(k_direction<R>, dim3(elem_grid(c->n)), dim3(kBlock), 0, st, int(c->n),
                     v.rh, Prec<R>::invd(c), v.p, c->sc);
}

template <typename R>
void enqueue_iterations(psl_ctx* c, int count, int rp, hipStream_t st) {
  for (int i = 0; i < count; ++i) {
    if (rp)
      enqueue_iteration<R, 1>(c, st);
    else
      enqueue_iteration<R, 0>(c, st);
  }
}

// Capture `chunk` iterations into a graph once per (precision, chunk, re-projection);
// replay it afterwards.
template <typename R>
int run_chunk(psl_ctx* c, int chunk, int rp, hipStream_t st) {
  hipGraphExec_t& ge = Prec<R>::graph(c);
  int& key = Prec<R>::graph_key(c);
  const int want = chunk * 2 + (rp ? 1 : 0);
  if (!ge || key != want) {
    if (ge) {
      (void)hipGraphExecDestroy(ge);
      ge = nullptr;
    }
    hipStream_t cap;
    PSL_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t graph;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipStreamDestroy(cap);
      return PSL_EHIP;
    }
    enqueue_iterations<R>(c, chunk, rp, cap);
    hipError_t e1 = hipStreamEndCapture(cap, &graph);
    (void)hipStreamDestroy(cap);
    if (e1 != hipSuccess) return PSL_EHIP;
    hipError_t e2 = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
      ge = nullptr;
      return PSL_EHIP;
    }
    key = want;
  }
  PSL_HIP(hipGraphLaunch(ge, st));
  return PSL_OK;
}

int read_scalars(psl_ctx* c, hipStream_t st) {
  PSL_HIP(hipMemcpyAsync(c->h_sc, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
  PSL_HIP(hipStreamSynchronize(st));
  return PSL_OK;
}

constexpr int kStallWindow = 512;   // inner iterations without halving ||rhat|| -> stop

// Inner deflated PCG on the current outer residual (c->r64, ||r||^2 in sc->rr); adds
// ||r|| xhat to x. *status: PSL_OK (goal reached or stalled), PSL_EBREAKDOWN, PSL_ENONFINITE.
template <typename R>
int inner_solve(psl_ctx* c, double* x, double goal, int maxit, int check_every, int rp,
                int use_graph, hipStream_t st, int* iters, int* status, int* stalled) {
  int rc = ensure_vecs<R>(c);
  if (rc != PSL_OK) return rc;
  psl::VecSet<R>& v = Prec<R>::vecs(c);
  hipLaunchKernelGGL(k_set_inner, dim3(1), dim3(1), 0, st, c->sc, goal * goal, maxit);
  if (rp)
    with_ns<InitL<R, 1>::template F>(c->nslot_max, c, st);
  else
    with_ns<InitL<R, 0>::template F>(c->nslot_max, c, st);
  double best = INFINITY;
  int best_it = 0;
  *stalled = 0;
  for (;;) {
    if (use_graph) {
      rc = run_chunk<R>(c, check_every, rp, st);
      if (rc != PSL_OK) return rc;
    } else {
      enqueue_iterations<R>(c, check_every, rp, st);
      PSL_HIP(hipGetLastError());
    }
    rc = read_scalars(c, st);
    if (rc != PSL_OK) return rc;
    if (c->h_sc->done) break;
    const double rr = c->h_sc->rr;
    if (rr < 0.25 * best) {
      best = rr;
      best_it = c->h_sc->iters;
    } else if (c->h_sc->iters - best_it >= kStallWindow) {
      *stalled = 1;
      break;
    }
  }
  *iters = c->h_sc->iters;
  *status = c->h_sc->status;
  // x += ||r|| xhat
  hipLaunchKernelGGL(k_accumulate<R>, dim3(elem_grid(c->n)), dim3(kBlock), 0, st, int(c->n), x,
                     v.xh, c->sc);
  return PSL_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------------------
extern "C" int psl_apply_A(psl_ctx* c, const double* p, double* q, void* stream) {
  if (!c || !p || !q || p == q) return PSL_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, st, c->sc);
  launch_stencil<double, 0>(c, p, nullptr, q, 0, st);
  PSL_HIP(hipGetLastError());
  return PSL_OK;
}

extern "C" int psl_deflate(psl_ctx* c, const double* r, double* out, double* cvec,
                           void* stream) {
  if (!c || !r || !out) return PSL_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, st, c->sc);
  with_ns<ZtL>(c->nslot_max, c, r, st);
  launch_coarse<1>(c, 0, st);
  // out may alias r: each cell reads r before writing out
  launch_outer_deflate(c, nullptr, r, out, st);
  if (cvec)
    PSL_HIP(hipMemcpyAsync(cvec, c->e, sizeof(double) * c->d, hipMemcpyDeviceToDevice, st));
  PSL_HIP(hipGetLastError());
  return PSL_OK;
}

extern "C" int psl_solve(psl_ctx* c, const double* b, double* x, const psl_solve_opts* o_in,
                         psl_solve_stats* st_out, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!c || !b || !x) return PSL_EINVAL;
  psl_solve_opts o;
  psl_default_opts(&o);
  if (o_in) o = *o_in;
  if (!(o.tol > 0.0) || o.maxit < 0 || o.max_outer < 1 ||
      (o.mode != PSL_FP64 && o.mode != PSL_MIXED) || o.check_every < 1 ||
      o.check_every > 4096 || !(o.tau_inner > 0.0 && o.tau_inner < 1.0) || o.reproject < -1 ||
      o.reproject > 1)
    return PSL_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int n = int(c->n);
  psl_solve_stats stats;
  std::memset(&stats, 0, sizeof(stats));
  auto finish = [&](int status) {
    stats.status = status;
    stats.t_solve_s =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st_out) *st_out = stats;
    return status;
  };
  int rc;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, st, c->sc);
  hipLaunchKernelGGL(k_norm2, dim3(c->ntiles), dim3(kBlock), 0, st, geo(c), b, c->red_part,
                     c->sc, 1);
  if (o.use_x0)
    hipLaunchKernelGGL(k_norm2, dim3(c->ntiles), dim3(kBlock), 0, st, geo(c), x, c->red_part,
                       c->sc, 0);
  if ((rc = read_scalars(c, st)) != PSL_OK) return finish(rc);
  const double bnorm = std::sqrt(c->h_sc->bnorm2);
  stats.bnorm = bnorm;
  if (!std::isfinite(bnorm) || (o.use_x0 && !std::isfinite(c->h_sc->rr)))
    return finish(PSL_ENONFINITE);
  if (bnorm == 0.0) {
    hipLaunchKernelGGL(k_zero, dim3(elem_grid(n)), dim3(kBlock), 0, st, x, n);
    PSL_HIP(hipStreamSynchronize(st));
    return finish(PSL_OK);
  }
  if (!o.use_x0) hipLaunchKernelGGL(k_zero, dim3(elem_grid(n)), dim3(kBlock), 0, st, x, n);

  const int use_graph = 1;
  const char* verbose_env = std::getenv("PSL_VERBOSE");
  const bool verbose = verbose_env && verbose_env[0] == '1';
  int mode = o.mode;
  int total_iters = 0;
  int status = PSL_EMAXIT;
  double prev_rnorm = INFINITY;
  int last_inner_broke = 0;
  for (int outer = 0;; ++outer) {
    // projects the previous inner correction and forms x* for the next inner solve
    enqueue_outer_step(c, b, x, st);
    if ((rc = read_scalars(c, st)) != PSL_OK) return finish(rc);
    const double rnorm = std::sqrt(c->h_sc->rr);
    stats.outer = outer;
    if (verbose)
      std::fprintf(stderr, "libpsl: outer %d  ||P1 r||/||b|| = %.3e  mode %s  iters %d\n", outer,
                   rnorm / bnorm, mode == PSL_MIXED ? "mixed" : "fp64", total_iters);
    if (!std::isfinite(rnorm)) {
      status = PSL_ENONFINITE;
      break;
    }
    if (rnorm <= o.tol * bnorm) {
      status = PSL_OK;
      break;
    }
    if (total_iters >= o.maxit || outer >= o.max_outer) {
      status = PSL_EMAXIT;
      break;
    }
    if (outer > 0 && rnorm > 0.5 * prev_rnorm) {
      if (mode == PSL_MIXED) {
        mode = PSL_FP64;  // float32 CG stopped reducing the float64 residual
        stats.fell_back = 1;
      } else if (rnorm > 0.9 * prev_rnorm) {
        status = last_inner_broke ? PSL_EBREAKDOWN : PSL_ESTAGNATION;
        break;
      }
    }
    prev_rnorm = std::min(prev_rnorm, rnorm);
    const double target = o.tol * bnorm / rnorm;  // relative to ||rhat_0|| = 1
    int it = 0, ist = 0, stalled = 0;
    if (mode == PSL_MIXED) {
      const int rp = o.reproject != 0;
      rc = inner_solve<float>(c, x, std::max(o.tau_inner, target), o.maxit - total_iters,
                              o.check_every, rp, use_graph, st, &it, &ist, &stalled);
    } else {
      const int rp = o.reproject == 1;
      rc = inner_solve<double>(c, x, target, o.maxit - total_iters, o.check_every, rp,
                               use_graph, st, &it, &ist, &stalled);
    }
    if (rc != PSL_OK) return finish(rc);
    if (verbose)
      std::fprintf(stderr, "libpsl:   inner %d iterations, status %d, stalled %d, ||rhat||/||rhat0|| = %.3e\n",
                   it, ist, stalled, std::sqrt(c->h_sc->rr));
    total_iters += it;
    stats.iters = total_iters;
    if (ist == PSL_ENONFINITE) {
      status = ist;
      enqueue_outer_step(c, b, x, st);  // leave x projected
      break;
    }
    // a breakdown or stall ends this inner solve; the refinement loop decides what next
    last_inner_broke = (ist == PSL_EBREAKDOWN && it == 0);
  }
  // fresh float64 residual of the returned x
  launch_stencil<double, 1>(c, x, b, c->t64, 0, st);
  if ((rc = read_scalars(c, st)) != PSL_OK) return finish(rc);
  stats.relres_true = std::sqrt(c->h_sc->rr) / bnorm;
  stats.iters = total_iters;
  return finish(status);
}
