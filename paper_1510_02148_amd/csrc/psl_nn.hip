// libpsl start-vector network kernels: bf16 matrix-core convolutions (implicit GEMM on
// v_mfma_f32_16x16x32_bf16, float32 accumulation) and the small passes around them.
//
// Operand layout of the 16x16x32 bf16 product, one wave: lane l supplies 8 consecutive
// k-values of row (l % 16) of A and of column (l % 16) of B from k-slice (l / 16), and
// receives D rows 4 (l / 16) + r, r = 0..3, of column (l % 16). For the convolution,
// A = weights (rows = output channels), B = shifted inputs (columns = cells), k = tap *
// Cin + ci, so a lane's 8 values are 8 consecutive channels of one cell: one 16-byte load.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/psl_nn.h"

namespace {

constexpr int kBlock = 256;
constexpr int kWgradChunk = 4096;   // cells per weight-gradient workgroup (multiple of 32)
constexpr int kRedBlocks = 1024;    // partial sums of the row reductions

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t to_bf16(float f) {   // round to nearest, ties to even
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40);   // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

__device__ inline float from_bf16(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

__device__ inline bf16x8 load8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

__device__ inline bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

__device__ inline void tap_offsets(int t, int& dz, int& dy, int& dx) {
  dz = t / 9 - 1;
  dy = (t / 3) % 3 - 1;
  dx = t % 3 - 1;
}

// ---------------------------------------------------------------------------------------
// 3x3x3 convolution, forward (and input gradient with the flipped weights).
// Workgroup: 4 waves x 16 cells; each wave accumulates all MT output-channel tiles.
// ---------------------------------------------------------------------------------------
template <int MT>
__global__ void __launch_bounds__(kBlock)
    k_conv3(const uint16_t* __restrict__ x, int cin, const uint16_t* __restrict__ w, int kp,
            const float* __restrict__ bias, int nx, int ny, int nz, int relu,
            uint16_t* __restrict__ y, float* __restrict__ yf) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = nx * ny * nz;
  const int col = lane & 15, ks = lane >> 4;
  const int v = (blockIdx.x * 4 + wave) * 16 + col;
  const bool vin = v < n;
  int ix = 0, iy = 0, iz = 0;
  if (vin) {
    ix = v % nx;
    const int r = v / nx;
    iy = r % ny;
    iz = r / ny;
  }
  f32x4 acc[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* wrow = w + size_t(col) * kp;
  for (int k0 = 0; k0 < kp; k0 += 32) {
    const int k = k0 + ks * 8;
    const int t = k / cin, ci = k - t * cin;
    bf16x8 b = zero8();
    if (vin && t < 27) {
      int dz, dy, dx;
      tap_offsets(t, dz, dy, dx);
      const int jx = ix + dx, jy = iy + dy, jz = iz + dz;
      if (jx >= 0 && jx < nx && jy >= 0 && jy < ny && jz >= 0 && jz < nz)
        b = load8(x + size_t(v + dx + nx * (dy + ny * dz)) * cin + ci);
    }
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const bf16x8 a = load8(wrow + size_t(m) * 16 * kp + k);
      acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[m], 0, 0, 0);
    }
  }
  if (!vin) return;
  const int cout = MT * 16;
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int co0 = m * 16 + 4 * ks;
    float o[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float val = acc[m][r] + (bias ? bias[co0 + r] : 0.f);
      if (relu) val = val > 0.f ? val : 0.f;
      o[r] = val;
    }
    if (y) {
      const uint32_t lo = uint32_t(to_bf16(o[0])) | (uint32_t(to_bf16(o[1])) << 16);
      const uint32_t hi = uint32_t(to_bf16(o[2])) | (uint32_t(to_bf16(o[3])) << 16);
      *reinterpret_cast<uint2*>(y + size_t(v) * cout + co0) = make_uint2(lo, hi);
    }
    if (yf)
      *reinterpret_cast<float4*>(yf + size_t(v) * cout + co0) = make_float4(o[0], o[1], o[2], o[3]);
  }
}

// ---------------------------------------------------------------------------------------
// Weight gradient: D[co][col] = sum over cells of gy(c, co) * B(c, col), B = x(c + tap,
// ci) for col = t cin + ci < 27 cin, 1 for col = kp (bias), 0 otherwise. K = cells, split
// into chunks of kWgradChunk (one per blockIdx.y); each wave owns a 16-column tile.
// Cell slices of 8 stay inside one row (nx % 8 == 0, chunk starts multiple of 8).
// ---------------------------------------------------------------------------------------
template <int MT>
__global__ void __launch_bounds__(kBlock)
    k_conv3_wgrad(const uint16_t* __restrict__ gy, const uint16_t* __restrict__ x, int cin,
                  int kp, int nx, int ny, int nz, float* __restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cout = MT * 16;
  const int ncol = kp + 16;
  const int c0 = (blockIdx.x * 4 + wave) * 16;
  if (c0 >= ncol) return;   // whole wave (no barriers in this kernel)
  const int n = nx * ny * nz;
  const int colid = c0 + (lane & 15), ks = lane >> 4;
  int kind = 2, ci = 0, dz = 0, dy = 0, dx = 0;
  if (colid < 27 * cin) {
    kind = 0;
    const int t = colid / cin;
    ci = colid - t * cin;
    tap_offsets(t, dz, dy, dx);
  } else if (colid == kp) {
    kind = 1;
  }
  const int vb = blockIdx.y * kWgradChunk;
  const int ve = min(n, vb + kWgradChunk);
  f32x4 acc[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int v0 = vb; v0 < ve; v0 += 32) {
    const int s0 = v0 + ks * 8;   // first cell of this lane's k-slice
    uint16_t bv[8];
    int ix = 0, iy = 0, iz = 0;
    if (s0 < ve) {
      ix = s0 % nx;
      const int r = s0 / nx;
      iy = r % ny;
      iz = r / ny;
    }
    const bool rowok = (iy + dy >= 0) && (iy + dy < ny) && (iz + dz >= 0) && (iz + dz < nz);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = s0 + j;
      uint16_t val = 0;
      if (c < ve) {
        if (kind == 0) {
          const int jx = ix + j + dx;
          if (rowok && jx >= 0 && jx < nx) val = x[size_t(c + dx + nx * (dy + ny * dz)) * cin + ci];
        } else if (kind == 1) {
          val = 0x3f80;   // 1.0
        }
      }
      bv[j] = val;
    }
    const bf16x8 b = __builtin_bit_cast(bf16x8, make_uint4(uint32_t(bv[0]) | (uint32_t(bv[1]) << 16),
                                                           uint32_t(bv[2]) | (uint32_t(bv[3]) << 16),
                                                           uint32_t(bv[4]) | (uint32_t(bv[5]) << 16),
                                                           uint32_t(bv[6]) | (uint32_t(bv[7]) << 16)));
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int co = m * 16 + (lane & 15);
      uint16_t av[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) av[j] = (s0 + j < ve) ? gy[size_t(s0 + j) * cout + co] : 0;
      const bf16x8 a = __builtin_bit_cast(bf16x8, make_uint4(uint32_t(av[0]) | (uint32_t(av[1]) << 16),
                                                             uint32_t(av[2]) | (uint32_t(av[3]) << 16),
                                                             uint32_t(av[4]) | (uint32_t(av[5]) << 16),
                                                             uint32_t(av[6]) | (uint32_t(av[7]) << 16)));
      acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[m], 0, 0, 0);
    }
  }
  float* out = part + size_t(blockIdx.y) * cout * ncol;
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) out[size_t(m * 16 + 4 * ks + r) * ncol + colid] = acc[m][r];
}

// out[i] = sum over chunks q of part[q * len + i], in chunk order
__global__ void k_sum_chunks(const float* __restrict__ part, int64_t len, int nchunk,
                             float* __restrict__ out) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < len;
       i += int64_t(gridDim.x) * blockDim.x) {
    float s = 0.f;
    for (int q = 0; q < nchunk; ++q) s += part[q * len + i];
    out[i] = s;
  }
}

// ---------------------------------------------------------------------------------------
// elementwise and resampling passes
// ---------------------------------------------------------------------------------------
__global__ void k_relu_grad(int64_t count, const float* __restrict__ gy,
                            const uint16_t* __restrict__ y, int relu, uint16_t* __restrict__ gq) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x) {
    const float g = (!relu || from_bf16(y[i]) > 0.f) ? gy[i] : 0.f;
    gq[i] = to_bf16(g);
  }
}

__device__ inline int child(int px, int py, int pz, int o, int nx, int ny) {
  return (2 * px + (o & 1)) + nx * ((2 * py + ((o >> 1) & 1)) + ny * (2 * pz + (o >> 2)));
}

__global__ void k_pool2(int nx, int ny, int nz, const uint16_t* __restrict__ x, int c,
                        uint16_t* __restrict__ y) {
  const int mx = nx / 2, my = ny / 2, mz = nz / 2;
  const int64_t total = int64_t(mx) * my * mz * c;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int ch = int(i % c);
    const int p = int(i / c);
    const int px = p % mx, py = (p / mx) % my, pz = p / (mx * my);
    float s = 0.f;
#pragma unroll
    for (int o = 0; o < 8; ++o) s += from_bf16(x[size_t(child(px, py, pz, o, nx, ny)) * c + ch]);
    y[i] = to_bf16(s * 0.125f);
  }
}

__global__ void k_pool2_grad_add(int nx, int ny, int nz, const float* __restrict__ gy, int c,
                                 float* __restrict__ gx) {
  const int64_t total = int64_t(nx) * ny * nz * c;
  const int mx = nx / 2, my = ny / 2;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int ch = int(i % c);
    const int v = int(i / c);
    const int ix = v % nx, iy = (v / nx) % ny, iz = v / (nx * ny);
    const int p = ix / 2 + mx * (iy / 2 + my * (iz / 2));
    gx[i] += gy[size_t(p) * c + ch] * 0.125f;
  }
}

__global__ void k_upcat(int nx, int ny, int nz, const uint16_t* __restrict__ h, int ca,
                        const uint16_t* __restrict__ s, int cb, uint16_t* __restrict__ y) {
  const int cc = ca + cb;
  const int64_t total = int64_t(nx) * ny * nz * cc;
  const int mx = nx / 2, my = ny / 2;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int ch = int(i % cc);
    const int v = int(i / cc);
    if (ch < ca) {
      const int ix = v % nx, iy = (v / nx) % ny, iz = v / (nx * ny);
      const int p = ix / 2 + mx * (iy / 2 + my * (iz / 2));
      y[i] = h[size_t(p) * ca + ch];
    } else {
      y[i] = s[size_t(v) * cb + (ch - ca)];
    }
  }
}

__global__ void k_upcat_grad(int nx, int ny, int nz, const float* __restrict__ gy, int ca,
                             int cb, float* __restrict__ gh, float* __restrict__ gs) {
  const int cc = ca + cb;
  const int mx = nx / 2, my = ny / 2, mz = nz / 2;
  const int64_t nh = int64_t(mx) * my * mz * ca;
  const int64_t ns = int64_t(nx) * ny * nz * cb;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < nh + ns;
       i += int64_t(gridDim.x) * blockDim.x) {
    if (i < nh) {
      const int ch = int(i % ca);
      const int p = int(i / ca);
      const int px = p % mx, py = (p / mx) % my, pz = p / (mx * my);
      float acc = 0.f;
#pragma unroll
      for (int o = 0; o < 8; ++o) acc += gy[size_t(child(px, py, pz, o, nx, ny)) * cc + ch];
      gh[i] = acc;
    } else {
      const int64_t j = i - nh;
      const int ch = int(j % cb);
      const int64_t v = j / cb;
      gs[j] = gy[v * cc + ca + ch];
    }
  }
}

// ---------------------------------------------------------------------------------------
// 1x1x1 output layer
// ---------------------------------------------------------------------------------------
__global__ void k_conv1(int64_t n, const uint16_t* __restrict__ h, int cin,
                        const uint16_t* __restrict__ w, const float* __restrict__ bias,
                        float* __restrict__ y) {
  const float b = bias[0];
  for (int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; v < n;
       v += int64_t(gridDim.x) * blockDim.x) {
    float s = 0.f;
    for (int ci = 0; ci < cin; ++ci) s += from_bf16(w[ci]) * from_bf16(h[v * cin + ci]);
    y[v] = b + s;
  }
}

// gh = gq w; per-workgroup partials of sum gq h (cin columns) and sum gq (column cin)
__global__ void __launch_bounds__(kBlock)
    k_conv1_grad(int64_t n, const float* __restrict__ gy, const uint16_t* __restrict__ h,
                 int cin, const uint16_t* __restrict__ w, float* __restrict__ gh,
                 float* __restrict__ part) {
  extern __shared__ float sm[];   // [kBlock / 64][cin + 1]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float acc[33];
  const int nc = cin + 1;
  for (int j = 0; j < nc; ++j) acc[j] = 0.f;
  for (int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; v < n;
       v += int64_t(gridDim.x) * blockDim.x) {
    const float g = from_bf16(to_bf16(gy[v]));
    for (int ci = 0; ci < cin; ++ci) {
      gh[v * cin + ci] = g * from_bf16(w[ci]);
      acc[ci] += g * from_bf16(h[v * cin + ci]);
    }
    acc[cin] += g;
  }
  for (int j = 0; j < nc; ++j) {
    float s = acc[j];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) sm[wave * nc + j] = s;
  }
  __syncthreads();
  if (threadIdx.x < nc) {
    float s = 0.f;
    for (int q = 0; q < kBlock / 64; ++q) s += sm[q * nc + threadIdx.x];
    part[size_t(blockIdx.x) * nc + threadIdx.x] = s;
  }
}

// out[j] = sum over rows q < nrow of part[q * len + j] (fixed order), one thread per j
__global__ void k_sum_rows(const float* __restrict__ part, int nrow, int len, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= len) return;
  float s = 0.f;
  for (int q = 0; q < nrow; ++q) s += part[size_t(q) * len + j];
  out[j] = s;
}

// ---------------------------------------------------------------------------------------
// network input: log10 K standardised, b / max|b|
// ---------------------------------------------------------------------------------------
__device__ inline void block_sum3(double (&v)[3], double* sm) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = 0; k < 3; ++k) {
    double s = v[k];
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(s, off, 64);
      s = (k == 2) ? fmax(s, o) : s + o;
    }
    v[k] = s;
  }
  __syncthreads();
  if (lane == 0)
    for (int k = 0; k < 3; ++k) sm[k * 4 + wave] = v[k];
  __syncthreads();
  for (int k = 0; k < 3; ++k) {
    double s = sm[k * 4];
    for (int q = 1; q < kBlock / 64; ++q) s = (k == 2) ? fmax(s, sm[k * 4 + q]) : s + sm[k * 4 + q];
    v[k] = s;
  }
  __syncthreads();
}

// partials: sum log10 K, sum (log10 K)^2, max |b|
__global__ void __launch_bounds__(kBlock)
    k_input_stats(int64_t n, const double* __restrict__ K, const double* __restrict__ b,
                  double* __restrict__ part) {
  __shared__ double sm[12];
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double l = log10(K[i]);
    v[0] += l;
    v[1] += l * l;
    v[2] = fmax(v[2], fabs(b[i]));
  }
  block_sum3(v, sm);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = v[0];
    part[3 * blockIdx.x + 1] = v[1];
    part[3 * blockIdx.x + 2] = v[2];
  }
}

__global__ void __launch_bounds__(kBlock)
    k_input_fin(int64_t n, int nblk, const double* __restrict__ part, double* __restrict__ st) {
  __shared__ double sm[12];
  double v[3] = {0.0, 0.0, 0.0};
  for (int q = threadIdx.x; q < nblk; q += kBlock) {
    v[0] += part[3 * q];
    v[1] += part[3 * q + 1];
    v[2] = fmax(v[2], part[3 * q + 2]);
  }
  block_sum3(v, sm);
  if (threadIdx.x == 0) {
    const double mean = v[0] / double(n);
    const double var = fmax(v[1] / double(n) - mean * mean, 0.0);
    st[0] = mean;
    st[1] = fmax(sqrt(var), 1e-12);
    st[2] = v[2];
  }
}

__global__ void k_input_fill(int64_t n, const double* __restrict__ K, const double* __restrict__ b,
                             const double* __restrict__ st, uint16_t* __restrict__ x) {
  const double mean = st[0], sd = st[1], bm = st[2];
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const float c0 = float((log10(K[i]) - mean) / sd);
    const float c1 = bm > 0.0 ? float(b[i] / bm) : 0.f;
    const uint32_t lo = uint32_t(to_bf16(c0)) | (uint32_t(to_bf16(c1)) << 16);
    *reinterpret_cast<uint4*>(x + i * 8) = make_uint4(lo, 0u, 0u, 0u);
  }
}

// ---------------------------------------------------------------------------------------
// energy loss of alpha y
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
    k_energy_part(int64_t n, const float* __restrict__ y, const double* __restrict__ P1b,
                  const double* __restrict__ P1Ay, double* __restrict__ part) {
  __shared__ double sm[12];
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double yi = y[i];
    v[0] += yi * P1b[i];
    v[1] += yi * P1Ay[i];
  }
  block_sum3(v, sm);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = v[0];
    part[2 * blockIdx.x + 1] = v[1];
  }
}

__global__ void __launch_bounds__(kBlock)
    k_energy_fin(int nblk, const double* __restrict__ part, double c, double sigma,
                 double* __restrict__ out) {
  __shared__ double sm[12];
  double v[3] = {0.0, 0.0, 0.0};
  for (int q = threadIdx.x; q < nblk; q += kBlock) {
    v[0] += part[2 * q];
    v[1] += part[2 * q + 1];
  }
  block_sum3(v, sm);
  if (threadIdx.x == 0) {
    const double u = v[0], w = v[1];
    const bool ok = w > 0.0;
    if (sigma > 0.0)
      out[0] = c > 0.0 ? (sigma * sigma * w - 2.0 * sigma * u + c) / c : 1.0;
    else
      out[0] = (ok && c > 0.0) ? 1.0 - u * u / (w * c) : 1.0;
    out[1] = ok ? u / w : 0.0;   // no usable direction: alpha = 0 (the zero start)
    out[2] = u;
    out[3] = w;
  }
}

__global__ void k_energy_apply(int64_t n, const float* __restrict__ y, const double* __restrict__ P1b,
                               const double* __restrict__ P1Ay, double c, double sigma,
                               const double* __restrict__ out, float* __restrict__ gy,
                               double* __restrict__ x0) {
  const double alpha = out[1], u = out[2], w = out[3];
  // gy = fa P1 A y - fb P1 b
  double fa = 0.0, fb = 0.0;
  if (sigma > 0.0) {
    fa = 2.0 * sigma * sigma / c;
    fb = 2.0 * sigma / c;
  } else if (w > 0.0) {
    fb = 2.0 * u / (w * c);
    fa = fb * alpha;
  }
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    if (gy) gy[i] = float(fa * P1Ay[i] - fb * P1b[i]);
    if (x0) x0[i] = alpha * double(y[i]);
  }
}

__global__ void __launch_bounds__(kBlock)
    k_wl2_part(int64_t n, const float* __restrict__ y, const float* __restrict__ t,
               const float* __restrict__ d, double* __restrict__ part) {
  __shared__ double sm[12];
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double e = double(y[i]) - double(t[i]);
    v[0] += double(d[i]) * e * e;
    v[1] += double(d[i]) * double(t[i]) * double(t[i]);
  }
  block_sum3(v, sm);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = v[0];
    part[2 * blockIdx.x + 1] = v[1];
  }
}

__global__ void __launch_bounds__(kBlock)
    k_wl2_fin(int nblk, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sm[12];
  double v[3] = {0.0, 0.0, 0.0};
  for (int q = threadIdx.x; q < nblk; q += kBlock) {
    v[0] += part[2 * q];
    v[1] += part[2 * q + 1];
  }
  block_sum3(v, sm);
  if (threadIdx.x == 0) {
    out[0] = v[1] > 0.0 ? v[0] / v[1] : 0.0;
    out[1] = v[1];
  }
}

__global__ void k_wl2_grad(int64_t n, const float* __restrict__ y, const float* __restrict__ t,
                           const float* __restrict__ d, const double* __restrict__ out,
                           float* __restrict__ gy) {
  const double f = out[1] > 0.0 ? 2.0 / out[1] : 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    gy[i] = float(f * double(d[i]) * (double(y[i]) - double(t[i])));
}

__global__ void k_cell_diag(int nx, int ny, int nz, const double* __restrict__ Tx,
                            const double* __restrict__ Ty, const double* __restrict__ Tz,
                            float* __restrict__ d) {
  const int64_t n = int64_t(nx) * ny * nz;
  for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < n;
       c += int64_t(gridDim.x) * blockDim.x) {
    const int64_t ix = c % nx, r = c / nx, iy = r % ny, iz = r / ny;
    const int64_t fx = c + (iy + int64_t(ny) * iz), fy = c + int64_t(nx) * iz;
    d[c] = float(Tx[fx] + Tx[fx + 1] + Ty[fy] + Ty[fy + nx] + Tz[c] + Tz[c + int64_t(nx) * ny]);
    (void)ix;
  }
}

__global__ void k_widen(int64_t n, const float* __restrict__ y, double* __restrict__ y64) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    y64[i] = y[i];
}

// ---------------------------------------------------------------------------------------
// Adam and operand packing
// ---------------------------------------------------------------------------------------
__device__ inline float adam(float& p, float& m, float& v, float g, int t, float lr, float b1,
                             float b2, float eps) {
  if (t > 0) {
    m = b1 * m + (1.f - b1) * g;
    v = b2 * v + (1.f - b2) * g * g;
    const float mh = m / (1.f - powf(b1, float(t)));
    const float vh = v / (1.f - powf(b2, float(t)));
    p -= lr * mh / (sqrtf(vh) + eps);
  }
  return p;
}

__global__ void k_adam_conv(int cout, int cin, int kp, int kpt, float* __restrict__ p,
                            float* __restrict__ m, float* __restrict__ v, float* __restrict__ pb,
                            float* __restrict__ mb, float* __restrict__ vb,
                            const float* __restrict__ dw, int t, float lr, float b1, float b2,
                            float eps, uint16_t* __restrict__ w, uint16_t* __restrict__ wt) {
  const int kk = 27 * cin;
  const int64_t total = int64_t(cout) * kk;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total + cout;
       i += int64_t(gridDim.x) * blockDim.x) {
    if (i >= total) {
      const int co = int(i - total);
      adam(pb[co], mb[co], vb[co], t > 0 ? dw[size_t(co) * (kp + 16) + kp] : 0.f, t, lr, b1, b2, eps);
      continue;
    }
    const int co = int(i / kk), k = int(i % kk);
    const float g = t > 0 ? dw[size_t(co) * (kp + 16) + k] : 0.f;
    const float val = adam(p[i], m[i], v[i], g, t, lr, b1, b2, eps);
    const uint16_t h = to_bf16(val);
    w[size_t(co) * kp + k] = h;
    if (wt) {
      const int tap = k / cin, ci = k - tap * cin;
      wt[size_t(ci) * kpt + (26 - tap) * cout + co] = h;
    }
  }
}

__global__ void k_adam_vec(int count, float* __restrict__ p, float* __restrict__ m,
                           float* __restrict__ v, const float* __restrict__ dw, int t, float lr,
                           float b1, float b2, float eps, uint16_t* __restrict__ w) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const float val = adam(p[i], m[i], v[i], t > 0 ? dw[i] : 0.f, t, lr, b1, b2, eps);
    if (i < count - 1) w[i] = to_bf16(val);   // the last entry is the bias (kept in float)
  }
}

inline unsigned grid_for(int64_t work, int64_t per = kBlock, int64_t cap = 256 * 64) {
  return unsigned(std::max<int64_t>(1, std::min<int64_t>((work + per - 1) / per, cap)));
}

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

inline bool grid_ok(const psl_grid* g) { return g && g->nx > 0 && g->ny > 0 && g->nz > 0; }

template <int MT>
void launch_conv3(const psl_grid* g, const uint16_t* x, int cin, const uint16_t* w, int kp,
                  const float* bias, int relu, uint16_t* y, float* yf, hipStream_t st) {
  const int64_t n = int64_t(g->nx) * g->ny * g->nz;
  hipLaunchKernelGGL(k_conv3<MT>, dim3(unsigned((n + 63) / 64)), dim3(kBlock), 0, st, x, cin, w,
                     kp, bias, g->nx, g->ny, g->nz, relu, y, yf);
}

template <int MT>
void launch_wgrad(const psl_grid* g, const uint16_t* gy, const uint16_t* x, int cin, int kp,
                  float* part, int nchunk, hipStream_t st) {
  const int ncol = kp + 16;
  hipLaunchKernelGGL(k_conv3_wgrad<MT>, dim3(unsigned((ncol + 63) / 64), unsigned(nchunk)),
                     dim3(kBlock), 0, st, gy, x, cin, kp, g->nx, g->ny, g->nz, part);
}

}  // namespace

extern "C" int32_t psl_nn_kp(int32_t cin) { return (27 * cin + 31) / 32 * 32; }

extern "C" int psl_nn_conv3(const psl_grid* g, const uint16_t* x, int32_t cin, const uint16_t* w,
                            int32_t cout, const float* bias, int32_t relu, uint16_t* y, float* yf,
                            void* stream) {
  if (!grid_ok(g) || !x || !w || (!y && !yf) || cin < 8 || cin % 8 || cout < 16 || cout % 16 ||
      cout > 128 || !aligned16(x) || !aligned16(w) || (y && (reinterpret_cast<uintptr_t>(y) & 7u)) ||
      (yf && !aligned16(yf)) || int64_t(g->nx) * g->ny * g->nz > (int64_t(1) << 31) / 128)
    return PSL_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int kp = psl_nn_kp(cin);
  switch (cout / 16) {
    case 1: launch_conv3<1>(g, x, cin, w, kp, bias, relu, y, yf, st); break;
    case 2: launch_conv3<2>(g, x, cin, w, kp, bias, relu, y, yf, st); break;
    case 3: launch_conv3<3>(g, x, cin, w, kp, bias, relu, y, yf, st); break;
    case 4: launch_conv3<4>(g, x, cin, w, kp, bias, relu, y, yf, st); break;
    case 5: launch_conv3<5>(g, x, cin, w, kp, bias, relu, y, yf, st); break;
    case 6: launch_conv3<6>(g, x, cin, w, kp, bias, relu, y, yf, st); break;
    case 7: launch_conv3<7>(g, x, cin, w, kp, bias, relu, y, yf, st); break;
    default: launch_conv3<8>(g, x, cin, w, kp, bias, relu, y, yf, st); break;
  }
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}

extern "C" int64_t psl_nn_wgrad_work(const psl_grid* g, int32_t cin, int32_t cout) {
  if (!grid_ok(g)) return 0;
  const int64_t n = int64_t(g->nx) * g->ny * g->nz;
  const int64_t nchunk = (n + kWgradChunk - 1) / kWgradChunk;
  return nchunk * cout * (psl_nn_kp(cin) + 16);
}

extern "C" int psl_nn_conv3_wgrad(const psl_grid* g, const uint16_t* gy, int32_t cout,
                                  const uint16_t* x, int32_t cin, float* dw, float* work,
                                  void* stream) {
  if (!grid_ok(g) || !gy || !x || !dw || !work || cin < 8 || cin % 8 || cout < 16 ||
      cout % 16 || cout > 64 || g->nx % 8)
    return PSL_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t n = int64_t(g->nx) * g->ny * g->nz;
  const int nchunk = int((n + kWgradChunk - 1) / kWgradChunk);
  const int kp = psl_nn_kp(cin);
  switch (cout / 16) {
    case 1: launch_wgrad<1>(g, gy, x, cin, kp, work, nchunk, st); break;
    case 2: launch_wgrad<2>(g, gy, x, cin, kp, work, nchunk, st); break;
    case 3: launch_wgrad<3>(g, gy, x, cin, kp, work, nchunk, st); break;
    default: launch_wgrad<4>(g, gy, x, cin, kp, work, nchunk, st); break;
  }
  const int64_t len = int64_t(cout) * (kp + 16);
  hipLaunchKernelGGL(k_sum_chunks, dim3(grid_for(len)), dim3(kBlock), 0, st, work, len, nchunk, dw);
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}

extern "C" int psl_nn_relu_grad(int64_t count, const float* gy, const uint16_t* y, int32_t relu,
                                uint16_t* gq, void* stream) {
  if (count < 0 || !gy || !gq || (relu && !y)) return PSL_EINVAL;
  hipLaunchKernelGGL(k_relu_grad, dim3(grid_for(count)), dim3(kBlock), 0,
                     static_cast<hipStream_t>(stream), count, gy, y, relu, gq);
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}

extern "C" int psl_nn_pool2(const psl_grid* g, const uint16_t* x, int32_t c, uint16_t* y,
                            void* stream) {
  if (!grid_ok(g) || !x || !y || c < 1 || g->nx % 2 || g->ny % 2 || g->nz % 2) return PSL_EINVAL;
  const int64_t total = int64_t(g->nx / 2) * (g->ny / 2) * (g->nz / 2) * c;
  hipLaunchKernelGGL(k_pool2, dim3(grid_for(total)), dim3(kBlock), 0,
                     static_cast<hipStream_t>(stream), g->nx, g->ny, g->nz, x, c, y);
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}

extern "C" int psl_nn_pool2_grad_add(const psl_grid* g, const float* gy, int32_t c, float* gx,
                                     void* stream) {
  if (!grid_ok(g) || !gy || !gx || c < 1 || g->nx % 2 || g->ny % 2 || g->nz % 2) return PSL_EINVAL;
  const int64_t total = int64_t(g->nx) * g->ny * g->nz * c;
  hipLaunchKernelGGL(k_pool2_grad_add, dim3(grid_for(total)), dim3(kBlock), 0,
                     static_cast<hipStream_t>(stream), g->nx, g->ny, g->nz, gy, c, gx);
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}

extern "C" int psl_nn_upcat(const psl_grid* g, const uint16_t* h, int32_t ca, const uint16_t* s,
                            int32_t cb, uint16_t* y, void* stream) {
  if (!grid_ok(g) || !h || !s || !y || ca < 1 || cb < 1 || g->nx % 2 || g->ny % 2 || g->nz % 2)
    return PSL_EINVAL;
  const int64_t total = int64_t(g->nx) * g->ny * g->nz * (ca + cb);
  hipLaunchKernelGGL(k_upcat, dim3(grid_for(total)), dim3(kBlock), 0,
                     static_cast<hipStream_t>(stream), g->nx, g->ny, g->nz, h, ca, s, cb, y);
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}

extern "C" int psl_nn_upcat_grad(const psl_grid* g, const float* gy, int32_t ca, int32_t cb,
                                 float* gh, float* gs, void* stream) {
  if (!grid_ok(g) || !gy || !gh || !gs || ca < 1 || cb < 1 || g->nx % 2 || g->ny % 2 || g->nz % 2)
    return PSL_EINVAL;
  const int64_t total = int64_t(g->nx / 2) * (g->ny / 2) * (g->nz / 2) * ca +
                        int64_t(g->nx) * g->ny * g->nz * cb;
  hipLaunchKernelGGL(k_upcat_grad, dim3(grid_for(total)), dim3(kBlock), 0,
                     static_cast<hipStream_t>(stream), g->nx, g->ny, g->nz, gy, ca, cb, gh, gs);
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}

extern "C" int psl_nn_conv1(int64_t n, const uint16_t* h, int32_t cin, const uint16_t* w,
                            const float* bias, float* y, void* stream) {
  if (n < 1 || !h || !w || !bias || !y || cin < 1 || cin > 32) return PSL_EINVAL;
  hipLaunchKernelGGL(k_conv1, dim3(grid_for(n)), dim3(kBlock), 0, static_cast<hipStream_t>(stream),
                     n, h, cin, w, bias, y);
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}

extern "C" int64_t psl_nn_conv1_work(int64_t n, int32_t cin) {
  return int64_t(grid_for(n, kBlock, kRedBlocks)) * (cin + 1);
}

extern "C" int psl_nn_conv1_grad(int64_t n, const float* gy, const uint16_t* h, int32_t cin,
                                 const uint16_t* w, float* gh, float* dw, float* work,
                                 void* stream) {
  if (n < 1 || !gy || !h || !w || !gh || !dw || !work || cin < 1 || cin > 32) return PSL_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const unsigned nb = grid_for(n, kBlock, kRedBlocks);
  hipLaunchKernelGGL(k_conv1_grad, dim3(nb), dim3(kBlock), sizeof(float) * 4 * (cin + 1), st, n,
                     gy, h, cin, w, gh, work);
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(64), 0, st, work, int(nb), cin + 1, dw);
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}

extern "C" int64_t psl_nn_input_work(int64_t n) {
  return int64_t(grid_for(n, kBlock, kRedBlocks)) * 3 + 4;
}

extern "C" int psl_nn_make_input(int64_t n, const double* K, const double* b, uint16_t* x,
                                 double* work, void* stream) {
  if (n < 1 || !K || !b || !x || !work || !aligned16(x)) return PSL_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const unsigned nb = grid_for(n, kBlock, kRedBlocks);
  double* stats = work + int64_t(nb) * 3;
  hipLaunchKernelGGL(k_input_stats, dim3(nb), dim3(kBlock), 0, st, n, K, b, work);
  hipLaunchKernelGGL(k_input_fin, dim3(1), dim3(kBlock), 0, st, n, int(nb), work, stats);
  hipLaunchKernelGGL(k_input_fill, dim3(grid_for(n)), dim3(kBlock), 0, st, n, K, b, stats, x);
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}

extern "C" int64_t psl_nn_energy_work(int64_t n) {
  return int64_t(grid_for(n, kBlock, kRedBlocks)) * 2;
}

extern "C" int psl_nn_energy(int64_t n, const float* y, const double* P1b, const double* P1Ay,
                             double c, double sigma, double* out, float* gy, double* x0,
                             double* work, void* stream) {
  if (n < 1 || !y || !P1b || !P1Ay || !out || !work || !(c >= 0.0) || !(sigma >= 0.0))
    return PSL_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const unsigned nb = grid_for(n, kBlock, kRedBlocks);
  hipLaunchKernelGGL(k_energy_part, dim3(nb), dim3(kBlock), 0, st, n, y, P1b, P1Ay, work);
  hipLaunchKernelGGL(k_energy_fin, dim3(1), dim3(kBlock), 0, st, int(nb), work, c, sigma, out);
  if (gy || x0)
    hipLaunchKernelGGL(k_energy_apply, dim3(grid_for(n)), dim3(kBlock), 0, st, n, y, P1b, P1Ay,
                       c, sigma, out, c > 0.0 ? gy : nullptr, x0);
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}

extern "C" int psl_nn_widen(int64_t n, const float* y, double* y64, void* stream) {
  if (n < 0 || !y || !y64) return PSL_EINVAL;
  hipLaunchKernelGGL(k_widen, dim3(grid_for(n)), dim3(kBlock), 0, static_cast<hipStream_t>(stream),
                     n, y, y64);
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}

extern "C" int psl_nn_adam_conv(int32_t cout, int32_t cin, float* p, float* m, float* v,
                                float* pb, float* mb, float* vb, const float* dw, int32_t t,
                                float lr, float b1, float b2, float eps, uint16_t* w,
                                uint16_t* wt, void* stream) {
  if (cout < 1 || cin < 1 || !p || !m || !v || !pb || !mb || !vb || !w || t < 0 || (t > 0 && !dw))
    return PSL_EINVAL;
  const int kp = psl_nn_kp(cin), kpt = psl_nn_kp(cout);
  const int64_t total = int64_t(cout) * 27 * cin + cout;
  hipLaunchKernelGGL(k_adam_conv, dim3(grid_for(total)), dim3(kBlock), 0,
                     static_cast<hipStream_t>(stream), cout, cin, kp, kpt, p, m, v, pb, mb, vb,
                     dw, t, lr, b1, b2, eps, w, wt);
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}

extern "C" int psl_nn_adam_vec(int32_t count, float* p, float* m, float* v, const float* dw,
                               int32_t t, float lr, float b1, float b2, float eps, uint16_t* w,
                               void* stream) {
  if (count < 2 || !p || !m || !v || !w || t < 0 || (t > 0 && !dw)) return PSL_EINVAL;
  hipLaunchKernelGGL(k_adam_vec, dim3(grid_for(count)), dim3(kBlock), 0,
                     static_cast<hipStream_t>(stream), count, p, m, v, dw, t, lr, b1, b2, eps, w);
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}

extern "C" int64_t psl_nn_wl2_work(int64_t n) { return int64_t(grid_for(n, kBlock, kRedBlocks)) * 2; }

extern "C" int psl_nn_wl2(int64_t n, const float* y, const float* t, const float* d, double* out,
                          float* gy, double* work, void* stream) {
  if (n < 1 || !y || !t || !d || !out || !work) return PSL_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const unsigned nb = grid_for(n, kBlock, kRedBlocks);
  hipLaunchKernelGGL(k_wl2_part, dim3(nb), dim3(kBlock), 0, st, n, y, t, d, work);
  hipLaunchKernelGGL(k_wl2_fin, dim3(1), dim3(kBlock), 0, st, int(nb), work, out);
  if (gy)
    hipLaunchKernelGGL(k_wl2_grad, dim3(grid_for(n)), dim3(kBlock), 0, st, n, y, t, d, out, gy);
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}

extern "C" int psl_nn_cell_diag(const psl_grid* g, const double* Tx, const double* Ty,
                                const double* Tz, float* d, void* stream) {
  if (!grid_ok(g) || !Tx || !Ty || !Tz || !d) return PSL_EINVAL;
  const int64_t n = int64_t(g->nx) * g->ny * g->nz;
  hipLaunchKernelGGL(k_cell_diag, dim3(grid_for(n)), dim3(kBlock), 0,
                     static_cast<hipStream_t>(stream), g->nx, g->ny, g->nz, Tx, Ty, Tz, d);
  return hipGetLastError() == hipSuccess ? PSL_OK : PSL_EHIP;
}
