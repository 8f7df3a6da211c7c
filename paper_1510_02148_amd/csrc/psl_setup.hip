// libpsl set-up path: transmissibilities, subdomain-levelset labels, the work tiling,
// the interface rows of A Z, E = Z^T A Z and its float64 Cholesky factor and inverse.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "psl_internal.hpp"

using psl::kBlock;
using psl::kMaxSlots;
using psl::Tile;

// ---------------------------------------------------------------------------------------
// status strings and defaults
// ---------------------------------------------------------------------------------------
extern "C" const char* psl_status_str(int s) {
  switch (s) {
    case PSL_OK: return "ok";
    case PSL_EINVAL: return "invalid argument";
    case PSL_ENOMEM: return "device allocation failed";
    case PSL_EHIP: return "HIP runtime error";
    case PSL_ENOTSPD: return "matrix not positive definite";
    case PSL_EMAXIT: return "iteration cap reached";
    case PSL_EBREAKDOWN: return "CG breakdown (p^T P1 A p <= 0)";
    case PSL_ENONFINITE: return "non-finite value in input or iterate";
    case PSL_ESTAGNATION: return "refinement stagnated";
    case PSL_ENOTSUP: return "not supported by the library";
    default: return "unknown status";
  }
}

extern "C" void psl_default_opts(psl_solve_opts* o) {
  if (!o) return;
  o->tol = 1e-8;
  o->maxit = 10000;
  o->mode = PSL_FP64;
  o->use_x0 = 0;
  o->max_outer = 30;
  o->tau_inner = 0.01;
  o->check_every = 16;
  o->reproject = -1;
  o->mixed_floor = 1e-7;
}

// Device memory comes from the device's stream-ordered pool, which keeps freed blocks
// (release threshold raised once per device), so building and destroying contexts
// repeatedly does not return memory to the HIP runtime. Blocks are ordered on the stream of the
// entry point that asks for them; psl_destroy waits for the device before freeing.
thread_local hipStream_t psl_alloc_stream = nullptr;

static void keep_pool_memory() {
  static bool done[64] = {false};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64 || done[dev]) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  done[dev] = true;
}

int psl_internal_alloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  keep_pool_memory();
  if (hipMallocAsync(p, bytes, psl_alloc_stream) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return PSL_ENOMEM;
  }
  return PSL_OK;
}

void psl_internal_free(void* p) {
  if (p) (void)hipFreeAsync(p, psl_alloc_stream);
}

hipStream_t psl_internal_capture_stream() {
  static std::mutex mu;
  static hipStream_t streams[64] = {nullptr};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
    streams[dev] = nullptr;
  return streams[dev];
}

int psl_ctx_alloc(psl_ctx* c, void** p, size_t bytes, size_t reserve) {
  *p = nullptr;
  bytes = (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
  if (bytes > c->arena_left) {
    void* blk = nullptr;
    const size_t sz = std::max(bytes, reserve);
    if (psl_internal_alloc(&blk, sz) != PSL_OK) return PSL_ENOMEM;
    c->blocks.push_back(blk);
    c->arena = static_cast<char*>(blk);
    c->arena_left = sz;
  }
  *p = c->arena;
  c->arena += bytes;
  c->arena_left -= bytes;
  return PSL_OK;
}

// Pinned host mirrors of the solve scalars are recycled process-wide: pinning and
// unpinning host memory costs milliseconds, a context's whole set-up a few.
static std::mutex g_pinned_mu;
static std::vector<void*> g_pinned_free;

void* psl_internal_pinned_get(size_t bytes) {
  {
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    if (!g_pinned_free.empty()) {
      void* p = g_pinned_free.back();
      g_pinned_free.pop_back();
      return p;
    }
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes < 1024 ? 1024 : bytes) != hipSuccess) return nullptr;
  return p;
}

void psl_internal_pinned_put(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pinned_mu);
  g_pinned_free.push_back(p);
}

// PSL_OK, PSL_EINVAL (missing grid or a non-positive extent) or PSL_ENOTSUP (more than
// PSL_MAX_CELLS cells or entries in a face array: the solve kernels form byte offsets of
// float64 cell and face arrays in 32 bits, which stay exact below 2^29 elements)
static int grid_check(const psl_grid* g) {
  if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1) return PSL_EINVAL;
  const int64_t lim = PSL_MAX_CELLS;
  const int64_t nx = g->nx, ny = g->ny, nz = g->nz;
  if (nx * ny * nz > lim || (nx + 1) * ny * nz > lim || nx * (ny + 1) * nz > lim ||
      nx * ny * (nz + 1) > lim)
    return PSL_ENOTSUP;
  return PSL_OK;
}

static inline unsigned nblocks(int64_t work, int per = kBlock) {
  return static_cast<unsigned>((work + per - 1) / per);
}

template <typename T>
__global__ void k_fill(T* a, T v, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// ---------------------------------------------------------------------------------------
// transmissibilities (two-point flux, harmonic mean)
// ---------------------------------------------------------------------------------------
__device__ inline double harmonic_face(double a, double b) {
  const double s = a + b;
  return s > 0.0 ? 2.0 * a * b / s : 0.0;
}

// axis 0: faces (nx+1) x ny x nz ; axis 1: nx x (ny+1) x nz ; axis 2: nx x ny x (nz+1)
__global__ void k_tpfa(const double* __restrict__ K, double* __restrict__ T, int axis,
                       int nx, int ny, int nz, int lo_dirichlet, int hi_dirichlet) {
  const int fx = nx + (axis == 0), fy = ny + (axis == 1), fz = nz + (axis == 2);
  const int nf = fx * fy * fz;
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int ix = f % fx;
  const int iy = (f / fx) % fy;
  const int iz = f / (fx * fy);
  const int m = axis == 0 ? ix : (axis == 1 ? iy : iz);          // face coordinate
  const int ext = axis == 0 ? nx : (axis == 1 ? ny : nz);
  const int stride = axis == 0 ? 1 : (axis == 1 ? nx : nx * ny);
  // cell on the high side of the face (coordinate m), and on the low side (m-1)
  const int cx = axis == 0 ? 0 : ix, cy = axis == 1 ? 0 : iy, cz = axis == 2 ? 0 : iz;
  const int base = cx + nx * (cy + ny * cz);
  double t;
  if (m == 0) {
    t = lo_dirichlet ? 2.0 * K[base] : 0.0;
  } else if (m == ext) {
    t = hi_dirichlet ? 2.0 * K[base + (ext - 1) * stride] : 0.0;
  } else {
    t = harmonic_face(K[base + (m - 1) * stride], K[base + m * stride]);
  }
  T[f] = t;
}

extern "C" int psl_assemble_tpfa(const psl_grid* g, const double* K, uint32_t mask,
                                 double* Tx, double* Ty, double* Tz, void* stream) {
  if (const int grc = grid_check(g)) return grc;
  if (!K || !Tx || !Ty || !Tz || (mask & ~63u)) return PSL_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  double* T[3] = {Tx, Ty, Tz};
  for (int a = 0; a < 3; ++a) {
    const int64_t nf = int64_t(nx + (a == 0)) * (ny + (a == 1)) * (nz + (a == 2));
    hipLaunchKernelGGL(k_tpfa, dim3(nblocks(nf)), dim3(kBlock), 0, st, K, T[a], a, nx, ny,
                       nz, int((mask >> (2 * a)) & 1u), int((mask >> (2 * a + 1)) & 1u));
  }
  PSL_HIP(hipGetLastError());
  return PSL_OK;
}

// ---------------------------------------------------------------------------------------
// subdomain-levelset labels
// ---------------------------------------------------------------------------------------
struct ThrPack {
  double t[PSL_MAX_THRESHOLDS];
  int nthr;
};

__device__ inline int cell_key(int c, int nx, int ny, int nz, int sx, int sy, int sz, int ncls,
                               const double* K, const int32_t* cls, const ThrPack& thr) {
  const int ix = c % nx, iy = (c / nx) % ny, iz = c / (nx * ny);
  const int bx = int((int64_t(ix) * sx) / nx);
  const int by = int((int64_t(iy) * sy) / ny);
  const int bz = int((int64_t(iz) * sz) / nz);
  const int s = bx + sx * (by + sy * bz);
  int k;
  if (cls) {
    k = cls[c];
    if (k < 0 || k >= ncls) return -1;   // reported as an invalid class by the caller
  } else {
    const double v = K[c];
    k = 0;
    for (int t = 0; t < thr.nthr; ++t) k += (v >= thr.t[t]) ? 1 : 0;
  }
  return s * ncls + k;
}

__global__ void k_key_present(int n, int nx, int ny, int nz, int sx, int sy, int sz, int ncls,
                              const double* K, const int32_t* cls, ThrPack thr,
                              int32_t* present, int nkeys, int32_t* bad) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int key = cell_key(c, nx, ny, nz, sx, sy, sz, ncls, K, cls, thr);
  if (key < 0 || key >= nkeys) {
    bad[0] = 1;
    return;
  }
  present[key] = 1;
}

__global__ void k_key_rank(int n, int nx, int ny, int nz, int sx, int sy, int sz, int ncls,
                           const double* K, const int32_t* cls, ThrPack thr,
                           const int32_t* rank, int nkeys, int32_t* labels) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int key = cell_key(c, nx, ny, nz, sx, sy, sz, ncls, K, cls, thr);
  labels[c] = (key >= 0 && key < nkeys) ? rank[key] : -1;
}

// argument checks shared by psl_build_Z, psl_build_Z_noalloc and psl_build_Z_cc
static int build_z_args(const psl_grid* g, const double* K, const int32_t nsub[3],
                        const double* thr, int32_t nthr, const int32_t* cls, int32_t& ncls,
                        int32_t* labels, int32_t* d, ThrPack& tp, int& nkeys);

// Exclusive prefix sum of int32 counts in one workgroup of 1024 threads (set-up sizes).
// out[m] = total.
__global__ void __launch_bounds__(1024) k_scan_small(const int32_t* in, int32_t* out, int m) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x;
  const int chunk = (m + 1023) / 1024;
  const int a = min(m, t * chunk), b = min(m, a + chunk);
  int32_t s = 0;
  for (int i = a; i < b; ++i) s += in[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int32_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t run = part[t] - s;
  for (int i = a; i < b; ++i) {
    const int32_t v = in[i];
    out[i] = run;
    run += v;
  }
  if (t == 1023) out[m] = part[1023];
}

// The labelling proper: key presence flags, their exclusive scan (the rank of each key
// among the present ones) and the labels, on scratch the caller provides: present[nkeys],
// rank[nkeys + 1], bad[1]. present and bad are cleared here (fill kernels).
static int build_z_on(int nx, int ny, int nz, const int32_t nsub[3], int ncls, const double* K,
                      const int32_t* cls, const ThrPack& tp, int nkeys, int32_t* present,
                      int32_t* rank, int32_t* bad, int32_t* labels, int32_t* d, hipStream_t st) {
  const int n = nx * ny * nz;
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(nblocks(nkeys)), dim3(kBlock), 0, st, present, 0,
                     int64_t(nkeys));
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(kBlock), 0, st, bad, 0, int64_t(1));
  hipLaunchKernelGGL(k_key_present, dim3(nblocks(n)), dim3(kBlock), 0, st, n, nx, ny, nz,
                     nsub[0], nsub[1], nsub[2], ncls, K, cls, tp, present, nkeys, bad);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, present, rank, nkeys);
  hipLaunchKernelGGL(k_key_rank, dim3(nblocks(n)), dim3(kBlock), 0, st, n, nx, ny, nz, nsub[0],
                     nsub[1], nsub[2], ncls, K, cls, tp, rank, nkeys, labels);
  int32_t h[2] = {0, 0};
  hipError_t e1 = hipMemcpyAsync(&h[0], rank + nkeys, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  hipError_t e2 = hipMemcpyAsync(&h[1], bad, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  hipError_t e3 = hipStreamSynchronize(st);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return PSL_EHIP;
  if (h[1]) return PSL_EINVAL;  // a manual class outside [0, ncls)
  *d = h[0];
  return PSL_OK;
}

extern "C" int psl_build_Z(const psl_grid* g, const double* K, const int32_t nsub[3],
                           const double* thr, int32_t nthr, const int32_t* cls, int32_t ncls,
                           int32_t* labels, int32_t* d, void* stream) {
  psl_alloc_stream = static_cast<hipStream_t>(stream);
  ThrPack tp;
  int nkeys = 0;
  int rc = build_z_args(g, K, nsub, thr, nthr, cls, ncls, labels, d, tp, nkeys);
  if (rc != PSL_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t *present = nullptr, *rank = nullptr, *bad = nullptr;
  rc = psl_internal_alloc((void**)&present, sizeof(int32_t) * nkeys);
  if (rc == PSL_OK) rc = psl_internal_alloc((void**)&rank, sizeof(int32_t) * (nkeys + 1));
  if (rc == PSL_OK) rc = psl_internal_alloc((void**)&bad, sizeof(int32_t));
  if (rc == PSL_OK)
    rc = build_z_on(g->nx, g->ny, g->nz, nsub, ncls, K, cls, tp, nkeys, present, rank, bad, labels,
                    d, st);
  psl_internal_free(present);
  psl_internal_free(rank);
  psl_internal_free(bad);
  return rc;
}

// Scratch of psl_build_Z_noalloc: present[max keys], rank[max keys + 1], bad[1], in a
// file-scope device array that every call on a device shares. Host code reaches it only
// through the address hipGetSymbolAddress returns for the current device (kept per
// device): the array's name in host code is a host-side stand-in, not a device address.
constexpr int kNoAllocWords = 2 * PSL_NOALLOC_MAX_KEYS + 2;
static __device__ __align__(256) int32_t scratch[kNoAllocWords];

static std::mutex g_scratch_mu;
static int32_t* g_scratch_ptr[64] = {nullptr};

static int noalloc_scratch(int32_t** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return PSL_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PSL_EHIP;
    g_scratch_ptr[dev] = static_cast<int32_t*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return PSL_OK;
}

extern "C" int psl_build_Z_noalloc(const psl_grid* g, const double* K, const int32_t nsub[3],
                                   const double* thr, int32_t nthr, const int32_t* cls,
                                   int32_t ncls, int32_t* labels, int32_t* d, void* stream) {
  ThrPack tp;
  int nkeys = 0;
  int rc = build_z_args(g, K, nsub, thr, nthr, cls, ncls, labels, d, tp, nkeys);
  if (rc != PSL_OK) return rc;
  if (nkeys > PSL_NOALLOC_MAX_KEYS) return PSL_ENOTSUP;
  int32_t* base = nullptr;
  if ((rc = noalloc_scratch(&base)) != PSL_OK) return rc;
  int32_t* present = base;
  int32_t* rank = base + PSL_NOALLOC_MAX_KEYS;
  int32_t* bad = base + 2 * PSL_NOALLOC_MAX_KEYS + 1;
  return build_z_on(g->nx, g->ny, g->nz, nsub, ncls, K, cls, tp, nkeys, present, rank, bad,
                    labels, d, static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------------------------------
// psl_build_Z_cc: connected components of the (subdomain, class) regions
// ---------------------------------------------------------------------------------------
// Union-find over face neighbours with equal key. A union always hangs the larger root
// under the smaller one, so whatever order the atomics land in, the final root of every
// component is its smallest cell index; parent[c] <= c at all times, so every search
// ends. The parent array is read and written with device-scope atomics (coherent across
// the XCDs' L2 caches).
__device__ inline int cc_load(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int cc_find(int32_t* parent, int x) {
  int cur = x;
  int next = cc_load(parent + cur);
  while (next != cur) {
    const int up = cc_load(parent + next);
    if (up != next)   // path halving: cur is not a root, so no union targets it
      __hip_atomic_store(parent + cur, up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    cur = next;
    next = up;
  }
  return cur;
}

__device__ inline void cc_union(int32_t* parent, int a, int b) {
  a = cc_find(parent, a);
  b = cc_find(parent, b);
  while (a != b) {
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    int expected = a;   // a must still be a root
    if (__hip_atomic_compare_exchange_strong(parent + a, &expected, b, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return;
    a = cc_find(parent, expected);   // a was hung under a smaller root meanwhile
    b = cc_find(parent, b);
  }
}

__global__ void k_cc_init(int n, int nx, int ny, int nz, int sx, int sy, int sz, int ncls,
                          const double* K, const int32_t* cls, ThrPack thr, int nkeys,
                          int32_t* key, int32_t* parent, int32_t* bad) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int k = cell_key(c, nx, ny, nz, sx, sy, sz, ncls, K, cls, thr);
  if (k < 0 || k >= nkeys) bad[0] = 1;
  key[c] = k;
  parent[c] = c;
}

__global__ void k_cc_hook(int n, int nx, int ny, int nz, const int32_t* __restrict__ key,
                          int32_t* parent) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int ix = c % nx, iy = (c / nx) % ny, iz = c / (nx * ny);
  const int k = key[c];
  if (ix + 1 < nx && key[c + 1] == k) cc_union(parent, c, c + 1);
  if (iy + 1 < ny && key[c + nx] == k) cc_union(parent, c, c + nx);
  if (iz + 1 < nz && key[c + nx * ny] == k) cc_union(parent, c, c + nx * ny);
}

// The same union-find inside one subdomain box, in LDS. A component never crosses a
// subdomain boundary (the key holds the subdomain), so each box is labelled on its own:
// one workgroup per box loads its cells' keys, unites equal-key neighbours with LDS
// compare-and-swap (larger root under smaller, as above), and writes every cell's root as
// a global cell index. Local order within a box is global order, so the root of each
// component is again its smallest cell and the result equals the global kernels'.
constexpr int kCcLocalMax = 8192;   // cells of the largest box held in LDS

__device__ inline int lcc_load(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ inline int lcc_find(int32_t* par, int x) {
  int cur = x;
  int next = lcc_load(par + cur);
  while (next != cur) {
    const int up = lcc_load(par + next);
    if (up != next)   // path halving: cur is not a root, so no union targets it
      __hip_atomic_store(par + cur, up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    cur = next;
    next = up;
  }
  return cur;
}

__device__ inline void lcc_union(int32_t* par, int a, int b) {
  a = lcc_find(par, a);
  b = lcc_find(par, b);
  while (a != b) {
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    int expected = a;   // a must still be a root
    if (__hip_atomic_compare_exchange_strong(par + a, &expected, b, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
      return;
    a = lcc_find(par, expected);
    b = lcc_find(par, b);
  }
}

__global__ void __launch_bounds__(kBlock) k_cc_local(int nx, int ny, int nz, int sx, int sy,
                                                     int sz, int ncls, const double* K,
                                                     const int32_t* cls, ThrPack thr,
                                                     int nkeys, int32_t* parent, int32_t* bad) {
  __shared__ int32_t lpar[kCcLocalMax];
  __shared__ int32_t lkey[kCcLocalMax];
  const int b = blockIdx.x, bx = b % sx, by = (b / sx) % sy, bz = b / (sx * sy);
  // the box: cells whose floor-partition index is (bx, by, bz)
  const int x0 = int((int64_t(bx) * nx + sx - 1) / sx), x1 = int((int64_t(bx + 1) * nx + sx - 1) / sx);
  const int y0 = int((int64_t(by) * ny + sy - 1) / sy), y1 = int((int64_t(by + 1) * ny + sy - 1) / sy);
  const int z0 = int((int64_t(bz) * nz + sz - 1) / sz), z1 = int((int64_t(bz + 1) * nz + sz - 1) / sz);
  const int ex = x1 - x0, ey = y1 - y0, m = ex * ey * (z1 - z0);
  for (int li = threadIdx.x; li < m; li += kBlock) {
    const int lx = li % ex, ly = (li / ex) % ey, lz = li / (ex * ey);
    const int c = (x0 + lx) + nx * ((y0 + ly) + ny * (z0 + lz));
    const int k = cell_key(c, nx, ny, nz, sx, sy, sz, ncls, K, cls, thr);
    if (k < 0 || k >= nkeys) bad[0] = 1;
    lkey[li] = k;
    lpar[li] = li;
  }
  __syncthreads();
  for (int li = threadIdx.x; li < m; li += kBlock) {
    const int lx = li % ex, ly = (li / ex) % ey, lz = li / (ex * ey);
    const int k = lkey[li];
    if (lx + 1 < ex && lkey[li + 1] == k) lcc_union(lpar, li, li + 1);
    if (ly + 1 < ey && lkey[li + ex] == k) lcc_union(lpar, li, li + ex);
    if (lz + 1 < z1 - z0 && lkey[li + ex * ey] == k) lcc_union(lpar, li, li + ex * ey);
  }
  __syncthreads();
  for (int li = threadIdx.x; li < m; li += kBlock) {
    int r = li;
    while (lpar[r] != r) r = lpar[r];
    const int lx = li % ex, ly = (li / ex) % ey, lz = li / (ex * ey);
    const int rx = r % ex, ry = (r / ex) % ey, rz = r / (ex * ey);
    parent[(x0 + lx) + nx * ((y0 + ly) + ny * (z0 + lz))] =
        (x0 + rx) + nx * ((y0 + ry) + ny * (z0 + rz));
  }
}

// Every cell points straight at its root. The walk does not halve paths: a halving
// store from one thread could land after another thread has written the root to that
// cell and leave it pointing at an intermediate node. Here each thread writes only its
// own cell, and only the root, so every pointer a walk reads is an ancestor or the root.
__global__ void k_cc_compress(int n, int32_t* parent) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int r = c;
  int next = cc_load(parent + r);
  while (next != r) {
    r = next;
    next = cc_load(parent + r);
  }
  __hip_atomic_store(parent + c, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kCcBlock = 4 * kBlock;   // cells per counting block (4 consecutive per thread)

// roots (parent[c] == c) per block of kCcBlock cells
__global__ void __launch_bounds__(kBlock) k_cc_count(int n, const int32_t* parent,
                                                     int32_t* bsum) {
  __shared__ int32_t red[kBlock / psl::kWave];
  const int base = blockIdx.x * kCcBlock + 4 * threadIdx.x;
  int cnt = 0;
  for (int u = 0; u < 4; ++u)
    if (base + u < n && parent[base + u] == base + u) ++cnt;
  for (int off = psl::kWave / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
  if ((threadIdx.x & (psl::kWave - 1)) == 0) red[threadIdx.x / psl::kWave] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < kBlock / psl::kWave; ++w) s += red[w];
    bsum[blockIdx.x] = s;
  }
}

// column of each root = number of roots before it (block offset + exclusive scan in the
// block, in cell order)
__global__ void __launch_bounds__(kBlock) k_cc_rank(int n, const int32_t* parent,
                                                    const int32_t* boff, int32_t* rank) {
  __shared__ int32_t part[kBlock];
  const int base = blockIdx.x * kCcBlock + 4 * threadIdx.x;
  int is_root[4];
  int cnt = 0;
  for (int u = 0; u < 4; ++u) {
    is_root[u] = base + u < n && parent[base + u] == base + u;
    cnt += is_root[u];
  }
  part[threadIdx.x] = cnt;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = boff[blockIdx.x] + part[threadIdx.x] - cnt;
  for (int u = 0; u < 4; ++u)
    if (is_root[u]) rank[base + u] = run++;
}

// labels[c] = column of c's root (labels may hold the parent array: each cell reads its
// own entry before writing it)
__global__ void k_cc_label(int n, const int32_t* parent, const int32_t* rank, int32_t* labels) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  labels[c] = rank[parent[c]];
}

// argument checks shared by the label builders
static int build_z_args(const psl_grid* g, const double* K, const int32_t nsub[3],
                        const double* thr, int32_t nthr, const int32_t* cls, int32_t& ncls,
                        int32_t* labels, int32_t* d, ThrPack& tp, int& nkeys) {
  if (const int grc = grid_check(g)) return grc;
  if (!nsub || !labels || !d) return PSL_EINVAL;
  if (!cls && !K) return PSL_EINVAL;
  const int ext[3] = {g->nx, g->ny, g->nz};
  for (int a = 0; a < 3; ++a)
    if (nsub[a] < 1 || nsub[a] > ext[a]) return PSL_EINVAL;
  tp = ThrPack{};
  if (cls) {
    if (ncls < 1 || ncls > PSL_MAX_THRESHOLDS + 1) return PSL_EINVAL;
    tp.nthr = 0;
  } else {
    if (nthr < 0 || nthr > PSL_MAX_THRESHOLDS || (nthr > 0 && !thr)) return PSL_EINVAL;
    for (int t = 0; t < nthr; ++t) {
      if (!std::isfinite(thr[t])) return PSL_EINVAL;
      if (t > 0 && !(thr[t] > thr[t - 1])) return PSL_EINVAL;
      tp.t[t] = thr[t];
    }
    tp.nthr = nthr;
    ncls = nthr + 1;
  }
  const int64_t nkeys64 = int64_t(nsub[0]) * nsub[1] * nsub[2] * ncls;
  if (nkeys64 > (int64_t(1) << 26)) return PSL_ENOTSUP;
  nkeys = int(nkeys64);
  return PSL_OK;
}

extern "C" int psl_build_Z_cc(const psl_grid* g, const double* K, const int32_t nsub[3],
                              const double* thr, int32_t nthr, const int32_t* cls, int32_t ncls,
                              int32_t* labels, int32_t* d, void* stream) {
  psl_alloc_stream = static_cast<hipStream_t>(stream);
  ThrPack tp;
  int nkeys = 0;
  int rc = build_z_args(g, K, nsub, thr, nthr, cls, ncls, labels, d, tp, nkeys);
  if (rc != PSL_OK) return rc;
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  const int n = nx * ny * nz;
  const int nblk = (n + kCcBlock - 1) / kCcBlock;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t *key = nullptr, *bsum = nullptr, *boff = nullptr, *bad = nullptr;
  rc = psl_internal_alloc((void**)&key, sizeof(int32_t) * n);
  if (rc == PSL_OK) rc = psl_internal_alloc((void**)&bsum, sizeof(int32_t) * nblk);
  if (rc == PSL_OK) rc = psl_internal_alloc((void**)&boff, sizeof(int32_t) * (nblk + 1));
  if (rc == PSL_OK) rc = psl_internal_alloc((void**)&bad, sizeof(int32_t));
  auto release = [&]() {
    psl_internal_free(key);
    psl_internal_free(bsum);
    psl_internal_free(boff);
    psl_internal_free(bad);
  };
  if (rc != PSL_OK) {
    release();
    return rc;
  }
  int32_t* parent = labels;   // the output array holds the union-find forest until the end
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(kBlock), 0, st, bad, 0, int64_t(1));
  // the largest subdomain box of the floor partition
  const int64_t box_max = int64_t((nx + nsub[0] - 1) / nsub[0]) * ((ny + nsub[1] - 1) / nsub[1]) *
                          ((nz + nsub[2] - 1) / nsub[2]);
  if (box_max <= kCcLocalMax) {   // every box in LDS: one workgroup per box
    hipLaunchKernelGGL(k_cc_local, dim3(nsub[0] * nsub[1] * nsub[2]), dim3(kBlock), 0, st, nx, ny,
                       nz, nsub[0], nsub[1], nsub[2], ncls, K, cls, tp, nkeys, parent, bad);
  } else {
    hipLaunchKernelGGL(k_cc_init, dim3(nblocks(n)), dim3(kBlock), 0, st, n, nx, ny, nz,
                       nsub[0], nsub[1], nsub[2], ncls, K, cls, tp, nkeys, key, parent, bad);
    hipLaunchKernelGGL(k_cc_hook, dim3(nblocks(n)), dim3(kBlock), 0, st, n, nx, ny, nz, key,
                       parent);
    hipLaunchKernelGGL(k_cc_compress, dim3(nblocks(n)), dim3(kBlock), 0, st, n, parent);
  }
  hipLaunchKernelGGL(k_cc_count, dim3(nblk), dim3(kBlock), 0, st, n, parent, bsum);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, bsum, boff, nblk);
  hipLaunchKernelGGL(k_cc_rank, dim3(nblk), dim3(kBlock), 0, st, n, parent, boff, key);
  hipLaunchKernelGGL(k_cc_label, dim3(nblocks(n)), dim3(kBlock), 0, st, n, parent, key, labels);
  int32_t h[2] = {0, 0};
  hipError_t e1 = hipMemcpyAsync(&h[0], boff + nblk, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  hipError_t e2 = hipMemcpyAsync(&h[1], bad, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  hipError_t e3 = hipStreamSynchronize(st);
  release();
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return PSL_EHIP;
  if (h[1]) return PSL_EINVAL;  // a manual class outside [0, ncls)
  *d = h[0];
  return PSL_OK;
}

// ---------------------------------------------------------------------------------------
// psl_setup_E kernels
// ---------------------------------------------------------------------------------------
struct GridDev {
  int nx, ny, nz;
};

// diag(A) = sum of the six face transmissibilities of the cell; its inverse in both
// precisions; flags a cell whose diagonal is not a positive finite number.
__global__ void k_diag(GridDev g, const double* __restrict__ Tx, const double* __restrict__ Ty,
                       const double* __restrict__ Tz, double* invd, float* invd32,
                       int32_t* bad) {
  const int n = g.nx * g.ny * g.nz;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int ix = c % g.nx, iy = (c / g.nx) % g.ny, iz = c / (g.nx * g.ny);
  const int fx = ix + (g.nx + 1) * (iy + g.ny * iz);
  const int fy = ix + g.nx * (iy + (g.ny + 1) * iz);
  const int fz = c;
  const int sz = g.nx * g.ny;
  const double dg = Tx[fx] + Tx[fx + 1] + Ty[fy] + Ty[fy + g.nx] + Tz[fz] + Tz[fz + sz];
  if (!(dg > 0.0) || !(dg < INFINITY)) bad[0] = 1;
  const double inv = 1.0 / dg;
  invd[c] = inv;
  invd32[c] = static_cast<float>(inv);
}

__global__ void k_check_labels(const int32_t* __restrict__ labels, int n, int d, int32_t* bad) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n && (labels[c] < 0 || labels[c] >= d)) bad[0] = 1;
}

__global__ void k_cast_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = static_cast<float>(a[i]);
}

// Per tile: sorted distinct labels (up to kMaxSlots; more is flagged), and for every
// cell the index of its label in that list.
__global__ void __launch_bounds__(kBlock) k_tile_labels(GridDev g, const Tile* tiles,
                                                        const int32_t* __restrict__ labels,
                                                        int32_t* tile_lab, Tile* tiles_out,
                                                        uint8_t* slot, int32_t* overflow) {
  __shared__ int32_t red[kBlock / psl::kWave];
  __shared__ int32_t list[kMaxSlots];
  __shared__ int32_t cnt_s;
  const Tile T = tiles[blockIdx.x];
  const float inv_sx = 1.0f / T.sx, inv_sxy = 1.0f / (T.sx * T.sy);
  int prev = -1;
  int cnt = 0;
  for (;;) {
    int best = 0x7fffffff;
    for (int j = threadIdx.x; j < T.ncell; j += kBlock) {
      const int lz = psl::div_small(j, T.sx * T.sy, inv_sxy);
      const int rem = j - lz * T.sx * T.sy;
      const int ly = psl::div_small(rem, T.sx, inv_sx);
      const int lx = rem - ly * T.sx;
      const int c = (T.x0 + lx) + g.nx * ((T.y0 + ly) + g.ny * (T.z0 + lz));
      const int l = labels[c];
      if (l > prev && l < best) best = l;
    }
    for (int off = psl::kWave / 2; off > 0; off >>= 1) best = min(best, __shfl_xor(best, off));
    if ((threadIdx.x & (psl::kWave - 1)) == 0) red[threadIdx.x / psl::kWave] = best;
    __syncthreads();
    int m = red[0];
    for (int w = 1; w < kBlock / psl::kWave; ++w) m = min(m, red[w]);
    __syncthreads();
    if (m == 0x7fffffff) break;
    if (cnt == kMaxSlots) {
      cnt = kMaxSlots + 1;
      break;
    }
    if (threadIdx.x == 0) list[cnt] = m;
    ++cnt;
    prev = m;
  }
  if (threadIdx.x == 0) {
    cnt_s = cnt;
    if (cnt > kMaxSlots) overflow[0] = 1;
  }
  __syncthreads();
  cnt = min(cnt_s, kMaxSlots);
  if (threadIdx.x < kMaxSlots)
    tile_lab[blockIdx.x * kMaxSlots + threadIdx.x] = threadIdx.x < cnt ? list[threadIdx.x] : -1;
  if (threadIdx.x == 0) {
    Tile o = T;
    o.nslot = cnt;
    tiles_out[blockIdx.x] = o;
  }
  for (int j = threadIdx.x; j < T.ncell; j += kBlock) {
    const int lz = psl::div_small(j, T.sx * T.sy, inv_sxy);
    const int rem = j - lz * T.sx * T.sy;
    const int ly = psl::div_small(rem, T.sx, inv_sx);
    const int lx = rem - ly * T.sx;
    const int c = (T.x0 + lx) + g.nx * ((T.y0 + ly) + g.ny * (T.z0 + lz));
    const int l = labels[c];
    int k = 0;
    for (int s = 0; s < cnt; ++s)
      if (list[s] == l) k = s;
    slot[c] = static_cast<uint8_t>(k);
  }
}

// label -> (tile, slot) lists: count, fill at atomic cursors, then sort each list.
__global__ void k_lab_count(const int32_t* tile_lab, int nparts, int32_t* cnt, int d,
                            int32_t* bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nparts) return;
  const int l = tile_lab[i];
  if (l < 0) return;
  if (l >= d) {
    bad[0] = 1;
    return;
  }
  atomicAdd(&cnt[l], 1);
}

__global__ void k_lab_fill(const int32_t* tile_lab, int nparts, const int32_t* ptr,
                           int32_t* cursor, int32_t* part, int d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nparts) return;
  const int l = tile_lab[i];
  if (l < 0 || l >= d) return;
  const int pos = atomicAdd(&cursor[l], 1);
  part[ptr[l] + pos] = i;
}

// slot_pos[(tile, slot)] = its index in the label-major list
__global__ void k_slot_pos(const int32_t* ptr, const int32_t* part, int d, int32_t* slot_pos) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ptr[d]) return;
  slot_pos[part[i]] = i;
}

__global__ void k_lab_sort(const int32_t* ptr, int32_t* part, int d, int32_t* empty) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= d) return;
  const int a = ptr[l], b = ptr[l + 1];
  if (a == b) empty[0] = 1;  // a column of Z without cells
  for (int i = a + 1; i < b; ++i) {
    const int v = part[i];
    int j = i - 1;
    while (j >= a && part[j] > v) {
      part[j + 1] = part[j];
      --j;
    }
    part[j + 1] = v;
  }
}

// Cut faces of A Z. A face f of cell i with T_f > 0 is "cut" when it is an outer face or
// its neighbour j carries another label. Then
//   (A Z e)_i = sum over the cut faces of i of T_f (e_l(i) - e_l(j))   (e_l(j) = 0 outside),
// the flux form of A (Z e), which keeps the cancellation between neighbouring coarse
// values exact instead of summing rounded per-label coefficients. Cells with no cut face
// have (A Z)_i = 0 and no entry. Entries of one cell are contiguous, in face order
// (-x, +x, -y, +y, -z, +z); the first carries bit 31 in az_cell.
struct CutFaces {
  int n;
  int oth[6];
  double t[6];
};

__device__ inline void cut_faces(GridDev g, const double* __restrict__ Tx,
                                 const double* __restrict__ Ty, const double* __restrict__ Tz,
                                 const int32_t* __restrict__ labels, int c, CutFaces& cf) {
  const int ix = c % g.nx, iy = (c / g.nx) % g.ny, iz = c / (g.nx * g.ny);
  const int fx = ix + (g.nx + 1) * (iy + g.ny * iz);
  const int fy = ix + g.nx * (iy + (g.ny + 1) * iz);
  const int sxy = g.nx * g.ny;
  const int li = labels[c];
  const double tf[6] = {Tx[fx], Tx[fx + 1], Ty[fy], Ty[fy + g.nx], Tz[c], Tz[c + sxy]};
  const int nb[6] = {ix > 0 ? c - 1 : -1,       ix < g.nx - 1 ? c + 1 : -1,
                     iy > 0 ? c - g.nx : -1,    iy < g.ny - 1 ? c + g.nx : -1,
                     iz > 0 ? c - sxy : -1,     iz < g.nz - 1 ? c + sxy : -1};
  cf.n = 0;
  for (int f = 0; f < 6; ++f) {
    if (tf[f] == 0.0) continue;
    const int lj = nb[f] < 0 ? -1 : labels[nb[f]];
    if (lj == li) continue;
    cf.oth[cf.n] = lj;
    cf.t[cf.n] = tf[f];
    ++cf.n;
  }
}

__device__ inline int tile_cell(GridDev g, const Tile& T, int j, float inv_sx, float inv_sxy) {
  const int lz = psl::div_small(j, T.sx * T.sy, inv_sxy);
  const int rem = j - lz * T.sx * T.sy;
  const int ly = psl::div_small(rem, T.sx, inv_sx);
  const int lx = rem - ly * T.sx;
  return (T.x0 + lx) + g.nx * ((T.y0 + ly) + g.ny * (T.z0 + lz));
}

__global__ void __launch_bounds__(kBlock) k_az_count(GridDev g, const Tile* tiles,
                                                     const double* Tx, const double* Ty,
                                                     const double* Tz, const int32_t* labels,
                                                     int32_t* tile_cnt) {
  __shared__ double red[kBlock / psl::kWave];
  const Tile T = tiles[blockIdx.x];
  const float inv_sx = 1.0f / T.sx, inv_sxy = 1.0f / (T.sx * T.sy);
  double cnt = 0;
  for (int j = threadIdx.x; j < T.ncell; j += kBlock) {
    CutFaces cf;
    cut_faces(g, Tx, Ty, Tz, labels, tile_cell(g, T, j, inv_sx, inv_sxy), cf);
    cnt += cf.n;
  }
  double v[1] = {cnt};
  psl::block_sum<1>(v, red);
  if (threadIdx.x == 0) tile_cnt[blockIdx.x] = static_cast<int32_t>(v[0]);
}

__global__ void __launch_bounds__(kBlock) k_az_fill(GridDev g, const Tile* tiles,
                                                    const double* Tx, const double* Ty,
                                                    const double* Tz, const int32_t* labels,
                                                    const int32_t* az_ptr, int32_t* az_cell,
                                                    int32_t* az_lab, int32_t* az_oth,
                                                    double* az_t, float* az_t32) {
  __shared__ int32_t wsum[kBlock / psl::kWave];
  __shared__ int32_t base_s;
  const Tile T = tiles[blockIdx.x];
  const float inv_sx = 1.0f / T.sx, inv_sxy = 1.0f / (T.sx * T.sy);
  const int lane = threadIdx.x & (psl::kWave - 1), w = threadIdx.x / psl::kWave;
  if (threadIdx.x == 0) base_s = az_ptr[blockIdx.x];
  __syncthreads();
  for (int j0 = 0; j0 < T.ncell; j0 += kBlock) {
    const int j = j0 + threadIdx.x;
    CutFaces cf;
    cf.n = 0;
    int c = 0;
    if (j < T.ncell) {
      c = tile_cell(g, T, j, inv_sx, inv_sxy);
      cut_faces(g, Tx, Ty, Tz, labels, c, cf);
    }
    // block-exclusive prefix of cf.n in thread order
    int incl = cf.n;
    for (int off = 1; off < psl::kWave; off <<= 1) {
      const int v = __shfl_up(incl, off);
      if (lane >= off) incl += v;
    }
    if (lane == psl::kWave - 1) wsum[w] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int k = 0; k < kBlock / psl::kWave; ++k) {
      if (k < w) before += wsum[k];
      total += wsum[k];
    }
    const int pos = base_s + before + incl - cf.n;
    const int li = cf.n ? labels[c] : 0;
    for (int k = 0; k < cf.n; ++k) {
      az_cell[pos + k] = j | (k == 0 ? int32_t(0x80000000u) : 0);
      az_lab[pos + k] = li;
      az_oth[pos + k] = cf.oth[k];
      az_t[pos + k] = cf.t[k];
      az_t32[pos + k] = static_cast<float>(cf.t[k]);
    }
    __syncthreads();
    if (threadIdx.x == 0) base_s += total;
    __syncthreads();
  }
}

// E row l = sum over the cells of label l of their A Z rows: each cut face adds T to
// E[l][l] and -T to E[l][other]. One workgroup per row. The faces are summed in 64-bit
// fixed point scaled to the row (2^-60 of an upper bound of the diagonal), so the LDS
// atomics that let all threads work at once give an order-independent, deterministic row
// whose absolute error is below 2^-50 of the diagonal.
constexpr int kEChunk = 4096;
__global__ void __launch_bounds__(kBlock) k_E_rows(const int32_t* lab_ptr,
                                                   const int32_t* lab_part,
                                                   const int32_t* az_ptr,
                                                   const int32_t* az_lab,
                                                   const int32_t* az_oth,
                                                   const double* az_t, double* E, int d) {
  __shared__ unsigned long long rowbuf[kEChunk];
  __shared__ double red[kBlock / psl::kWave];
  const int l = blockIdx.x;
  // pass 1: an upper bound of the diagonal (sum of the row's cut-face T), fixed order
  double acc[1] = {0.0};
  for (int pi = lab_ptr[l]; pi < lab_ptr[l + 1]; ++pi) {
    const int tile = lab_part[pi] / kMaxSlots;
    for (int k = az_ptr[tile] + threadIdx.x; k < az_ptr[tile + 1]; k += kBlock)
      if (az_lab[k] == l) acc[0] += az_t[k];
  }
  psl::block_sum<1>(acc, red);
  const double diag_bound = acc[0] > 0.0 ? acc[0] * 1.0000001 : 1.0;
  int ex;
  frexp(diag_bound, &ex);                 // diag_bound < 2^ex
  const double scale = ldexp(1.0, 60 - ex), inv_scale = ldexp(1.0, ex - 60);
  for (int c0 = 0; c0 < d; c0 += kEChunk) {
    const int c1 = min(d, c0 + kEChunk);
    for (int c = c0 + threadIdx.x; c < c1; c += kBlock) rowbuf[c - c0] = 0ull;
    __syncthreads();
    for (int pi = lab_ptr[l]; pi < lab_ptr[l + 1]; ++pi) {
      const int tile = lab_part[pi] / kMaxSlots;
      for (int k = az_ptr[tile] + threadIdx.x; k < az_ptr[tile + 1]; k += kBlock) {
        if (az_lab[k] != l) continue;
        const long long v = llrint(az_t[k] * scale);
        if (l >= c0 && l < c1) atomicAdd(&rowbuf[l - c0], static_cast<unsigned long long>(v));
        const int o = az_oth[k];
        if (o >= c0 && o < c1)
          atomicAdd(&rowbuf[o - c0], static_cast<unsigned long long>(-v));
      }
    }
    __syncthreads();
    for (int c = c0 + threadIdx.x; c < c1; c += kBlock)
      E[int64_t(l) * d + c] = static_cast<double>(static_cast<long long>(rowbuf[c - c0])) * inv_scale;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// dense float64 Cholesky E = L L^T (lower, in place) and E^-1 = L^-T L^-1
// ---------------------------------------------------------------------------------------
constexpr int kNB = 64;

// The nb x nb block at src (leading dimension ld) into l[0:nb][0:nb] (zeros beyond nb),
// for a workgroup of NT threads: thread t covers column t % 64 of every (NT / 64)-th row,
// and issues all its global loads before its first LDS store.
template <int NT>
__device__ inline void stage_block(double (*l)[kNB + 1], const double* src, int64_t ld, int nb) {
  constexpr int kRows = NT / psl::kWave, kLoads = kNB / kRows;
  const int c = threadIdx.x % psl::kWave, r0 = threadIdx.x / psl::kWave;
  double v[kLoads];
#pragma unroll
  for (int u = 0; u < kLoads; ++u) {
    const int r = r0 + kRows * u;
    v[u] = (r < nb && c < nb) ? src[int64_t(r) * ld + c] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kLoads; ++u) l[r0 + kRows * u][c] = v[u];
}

__device__ inline double readlane_f64(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// Factor the kb diagonal block by columns (left-looking, one wave): lane i owns row i;
// column j needs s_i = sum_{k<j} L[i][k] L[j][k], then L[j][j] = sqrt(A[j][j] - s_j) and
// L[i][j] = (A[i][j] - s_i) / L[j][j]. Columns go in groups of eight. The terms of the
// finished columns k < jb are summed for the whole group in one pass over row i in LDS
// (with a transposed copy lt[k][j] = L[j][k], so the eight multipliers of a k are one
// contiguous read); inside the group each lane keeps its new entries in registers and
// row j's come by lane reads, so a column costs no LDS round trip or barrier. Every s_i
// is the plain sequential sum in k order. A non-positive pivot raises *bad.
__global__ void __launch_bounds__(psl::kWave) k_potrf_diag(double* A, int d, int kb, int32_t* bad) {
  constexpr int kG = 8;
  __shared__ double l[kNB][kNB + 1];
  __shared__ __align__(16) double lt[kNB][kNB + 2];  // rows of 528 bytes keep 16-byte reads aligned
  const int i = threadIdx.x;
  const int nb = min(kNB, d - kb);
  const bool own = i < nb;
  stage_block<psl::kWave>(l, A + int64_t(kb) * d + kb, d, nb);
  __syncthreads();
  for (int jb = 0; jb < nb; jb += kG) {
    double t[kG] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (own && i >= jb) {
      for (int k = 0; k < jb; ++k) {
        const double x = l[i][k];
        const double2* q = reinterpret_cast<const double2*>(&lt[k][jb]);
#pragma unroll
        for (int u = 0; u < kG / 2; ++u) {
          const double2 w = q[u];
          t[2 * u] += x * w.x;
          t[2 * u + 1] += x * w.y;
        }
      }
    }
    double g[kG];
#pragma unroll
    for (int c = 0; c < kG; ++c) {
      const int j = jb + c;
      g[c] = 0.0;
      if (j < nb) {  // uniform
        double s = t[c];
#pragma unroll
        for (int u = 0; u < c; ++u) s += g[u] * readlane_f64(g[u], j);
        const double r = l[i][j] - s;
        const double p = readlane_f64(r, j);
        if (i == 0 && (!(p > 0.0) || !(p < INFINITY))) bad[0] = 1;
        const double piv = sqrt(p > 0.0 ? p : 1.0);
        g[c] = (i == j) ? piv : r / piv;  // entries above the diagonal are never used
      }
    }
#pragma unroll
    for (int c = 0; c < kG; ++c) {
      if (jb + c < nb) {
        l[i][jb + c] = g[c];
        lt[jb + c][i] = g[c];
      }
    }
    __syncthreads();
  }
  double* o = A + int64_t(kb) * d + kb + i;
  if (own)
    for (int r = 0; r < nb; ++r) o[int64_t(r) * d] = (i <= r) ? l[r][i] : 0.0;
}

// Wave-parallel substitution with the nb x nb lower block l (in LDS): lane j holds x_j.
// forward (trans = 0): solves l x = x_in; backward (trans = 1): solves l^T x = x_in.
// Each solved entry is divided once (uniformly) and broadcast with a lane read.
__device__ inline double wave_trsv(const double (*l)[kNB + 1], int nb, double x, int trans) {
  const int lane = threadIdx.x & (psl::kWave - 1);
  if (!trans) {
    for (int m = 0; m < nb; ++m) {
      const double xm = readlane_f64(x, m) / l[m][m];
      if (lane == m) x = xm;
      else if (lane > m && lane < nb) x -= l[lane][m] * xm;
    }
  } else {
    for (int m = nb - 1; m >= 0; --m) {
      const double xm = readlane_f64(x, m) / l[m][m];
      if (lane == m) x = xm;
      else if (lane < m) x -= l[m][lane] * xm;
    }
  }
  return x;
}

// rows below the diagonal block: L[i, kb:kb+nb] = A[i, kb:kb+nb] L_kk^-T, i.e. solve
// L_kk y = a^T for every row i; one wave per row.
__global__ void __launch_bounds__(kBlock) k_trsm_panel(double* A, int d, int kb) {
  __shared__ double l[kNB][kNB + 1];
  const int nb = min(kNB, d - kb);
  stage_block<kBlock>(l, A + int64_t(kb) * d + kb, d, nb);
  __syncthreads();
  const int lane = threadIdx.x & (psl::kWave - 1);
  const int i = kb + nb + blockIdx.x * (kBlock / psl::kWave) + threadIdx.x / psl::kWave;
  if (i >= d) return;
  double* row = A + int64_t(i) * d + kb;
  double x = lane < nb ? row[lane] : 0.0;
  x = wave_trsv(l, nb, x, 0);
  if (lane < nb) row[lane] = x;
}

// C[i][j] -= sum_k A(i,k) B(k,j) for a 64x64 output tile per workgroup, K <= kNB.
// AM = 0: A(i,k) = A[i*lda + k]; AM = 1: A(i,k) = A[k*lda + i].
// BM = 0: B(k,j) = B[k*ldb + j]; BM = 1: B(k,j) = B[j*ldb + k].
// LOWER: only entries with j <= i are updated (tiles wholly above the diagonal exit).
// C += A B for 64 x 64 blocks staged in LDS as sa[k][row] = A(row, k) and sb[k][col] =
// B(k, col), on the float64 matrix cores (v_mfma_f64_16x16x4f64): wave w forms rows
// 16w .. 16w + 15 as four 16 x 16 tiles, four k per instruction. Lane l feeds A(16w +
// l % 16, k + l / 16) and B(k + l / 16, 16u + l % 16), and holds C(mac_row(r),
// mac_col(u)) in acc[u][r] (the result layout of the instruction, checked on gfx950 with
// a one-wave probe: register r of lane l is row l / 16 + 4 r, column l % 16 of the tile). An instruction reads two operands per lane from LDS where
// the vector form read 32 bytes per multiply-add pair: the products stop being bound by
// LDS bandwidth. The summation order inside an instruction is the hardware's, fixed.
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline int mac_row(int r) {
  const int l = threadIdx.x & (psl::kWave - 1), w = threadIdx.x / psl::kWave;
  return 16 * w + (l / 16) + 4 * r;
}
__device__ inline int mac_col(int u) { return 16 * u + (threadIdx.x & 15); }

__device__ inline void block_mac(const double (*sa)[kNB + 2], const double (*sb)[kNB + 2],
                                 double (&acc)[4][4]) {
  const int l = threadIdx.x & (psl::kWave - 1), w = threadIdx.x / psl::kWave;
  const int lr = l & 15, lk = l >> 4;
  v4d c[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) c[u] = v4d{acc[u][0], acc[u][1], acc[u][2], acc[u][3]};
#pragma unroll 4
  for (int k = 0; k < kNB; k += 4) {
    const double a = sa[k + lk][16 * w + lr];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      c[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sb[k + lk][16 * u + lr], c[u], 0, 0, 0);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[u][r] = c[u][r];
}

template <int AM, int BM, int LOWER>
__global__ void __launch_bounds__(kBlock) k_gemm_sub(double* C, int ldc, const double* A,
                                                     int lda, const double* B, int ldb, int M,
                                                     int N, int K) {
  // K = kNB here (a trailing update follows only a full 64-column panel)
  __shared__ __align__(16) double sa[kNB][kNB + 2];  // sa[k][i]
  __shared__ __align__(16) double sb[kNB][kNB + 2];  // sb[k][j]
  const int ti = blockIdx.y * 64, tj = blockIdx.x * 64;
  if (LOWER && tj > ti + 63) return;
  // K * 64 <= 4096 entries per operand: 16 per thread, all loads issued before the stores;
  // each operand is walked along its contiguous dimension
  constexpr int kLoads = kNB * 64 / kBlock;
  double va[kLoads], vb[kLoads];
#pragma unroll
  for (int u = 0; u < kLoads; ++u) {
    const int t = threadIdx.x + u * kBlock;
    const int ka = AM ? t / 64 : t % K, ra = AM ? t % 64 : t / K;
    const int kb = BM ? t % K : t / 64, rb = BM ? t / K : t % 64;
    const int i = ti + ra, j = tj + rb;
    const bool in = t < K * 64;
    va[u] = in && i < M ? (AM ? A[int64_t(ka) * lda + i] : A[int64_t(i) * lda + ka]) : 0.0;
    vb[u] = in && j < N ? (BM ? B[int64_t(j) * ldb + kb] : B[int64_t(kb) * ldb + j]) : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kLoads; ++u) {
    const int t = threadIdx.x + u * kBlock;
    if (t < K * 64) {
      const int ka = AM ? t / 64 : t % K, ra = AM ? t % 64 : t / K;
      const int kb = BM ? t % K : t / 64, rb = BM ? t / K : t % 64;
      sa[ka][ra] = va[u];
      sb[kb][rb] = vb[u];
    }
  }
  __syncthreads();
  double acc[4][4] = {};
  block_mac(sa, sb, acc);
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ti + mac_row(v), j = tj + mac_col(u);
      if (i < M && j < N && (!LOWER || j <= i)) C[int64_t(i) * ldc + j] -= acc[u][v];
    }
}

// A rows x cols block at src (leading dimension ld) on its way into LDS, zero beyond rows /
// cols: dst[r][c] (TRANS = 0) or dst[c][r] (TRANS = 1). A workgroup of kBlock threads; each
// thread holds 16 entries of one column (loads along a row are coalesced). Loading and
// storing are separate steps so the next block's loads can be in flight during a product.
struct RectRegs {
  double v[kNB / (kBlock / psl::kWave)];
  __device__ void load(const double* src, int64_t ld, int rows, int cols) {
    constexpr int kRows = kBlock / psl::kWave;
    const int c = threadIdx.x % psl::kWave, r0 = threadIdx.x / psl::kWave;
#pragma unroll
    for (int u = 0; u < kNB / kRows; ++u) {
      const int r = r0 + kRows * u;
      v[u] = (r < rows && c < cols) ? src[int64_t(r) * ld + c] : 0.0;
    }
  }
  template <int TRANS>
  __device__ void store(double (*dst)[kNB + 2]) const {
    constexpr int kRows = kBlock / psl::kWave;
    const int c = threadIdx.x % psl::kWave, r0 = threadIdx.x / psl::kWave;
#pragma unroll
    for (int u = 0; u < kNB / kRows; ++u) {
      const int r = r0 + kRows * u;
      if (TRANS)
        dst[c][r] = v[u];
      else
        dst[r][c] = v[u];
    }
  }
};

template <int TRANS>
__device__ inline void stage_rect(double (*dst)[kNB + 2], const double* src, int64_t ld,
                                  int rows, int cols) {
  RectRegs g;
  g.load(src, ld, rows, cols);
  g.template store<TRANS>(dst);
}

// acc[u][v] += sum_m sa[m][4 ty + u] sb[m][4 tx + v] over m < 64 (a 64x64 block product,
// 4x4 outputs per thread, tx = thread % 16, ty = thread / 16). A thread's four rows and
// four columns are contiguous, so each k step is two 16-byte reads per operand (the rows
// are shared by the 16 threads of a row group, i.e. broadcast).

// Inverse of each diagonal block of the lower factor, all blocks at once (one wave per
// block): lane j forms column j of L_kk^-1 by forward substitution,
// X_kk[i][j] = (delta_ij - sum_{k<i} L_kk[i][k] X_kk[k][j]) / L_kk[i][i]; entries above
// the diagonal are written as 0.
__global__ void __launch_bounds__(psl::kWave) k_trtri_diag(const double* L, double* X, int d) {
  __shared__ double l[kNB][kNB + 1];
  __shared__ double xs[kNB][kNB + 1];
  const int kb = blockIdx.x * kNB, nb = min(kNB, d - kb), j = threadIdx.x;
  stage_block<psl::kWave>(l, L + int64_t(kb) * d + kb, d, nb);
  __syncthreads();
  for (int i = 0; i < nb; ++i) {
    double s4[4] = {0.0, 0.0, 0.0, 0.0};   // independent partial sums: the LDS reads overlap
    int k = 0;
    for (; k + 4 <= i; k += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) s4[u] += l[i][k + u] * xs[k + u][j];   // xs[k][j] = 0, k < j
    }
    for (; k < i; ++k) s4[0] += l[i][k] * xs[k][j];
    const double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    xs[i][j] = (i >= j) ? ((i == j ? 1.0 : 0.0) - s) / l[i][i] : 0.0;
  }
  __syncthreads();
  if (j < nb)
    for (int r = 0; r < nb; ++r) X[int64_t(kb + r) * d + kb + j] = xs[r][j];
}

// Off-diagonal blocks of L^-1 on block diagonal s (block row i, column j = i - s), all in
// one launch: X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj, which needs only blocks of lower
// diagonals (formed by earlier launches).
__global__ void __launch_bounds__(kBlock) k_trtri_off(const double* L, double* X, int d, int s) {
  __shared__ __align__(16) double sa[kNB][kNB + 2];   // rows of 528 bytes: 16-byte reads stay aligned
  __shared__ __align__(16) double sb[kNB][kNB + 2];
  const int i = blockIdx.x + s, j = i - s;
  const int ri = i * kNB, cj = j * kNB, mi = min(kNB, d - ri);
  double acc[4][4] = {};
  RectRegs ga, gb;   // blocks k < i are full
  ga.load(L + int64_t(ri) * d + j * kNB, d, mi, kNB);
  gb.load(X + int64_t(j * kNB) * d + cj, d, kNB, kNB);
  for (int k = j; k < i; ++k) {
    ga.store<1>(sa);   // sa[m][r] = L_ik(r, m)
    gb.store<0>(sb);   // sb[m][c] = X_kj(m, c)
    __syncthreads();
    if (k + 1 < i) {
      ga.load(L + int64_t(ri) * d + (k + 1) * kNB, d, mi, kNB);
      gb.load(X + int64_t((k + 1) * kNB) * d + cj, d, kNB, kNB);
    }
    block_mac(sa, sb, acc);
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) sb[mac_row(v)][mac_col(u)] = acc[u][v];   // T(m, c)
  stage_rect<1>(sa, X + int64_t(ri) * d + ri, d, mi, mi);                  // sa[m][r] = X_ii(r, m)
  __syncthreads();
  double y[4][4] = {};
  block_mac(sa, sb, y);
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (mac_row(v) < mi) X[int64_t(ri + mac_row(v)) * d + cj + mac_col(u)] = -y[u][v];
}

// Long block diagonals (s > kTrtriChunk products per block) are split: workgroup (ii, ch)
// sums the products L_ik X_kj of its chunk of k into a partial block of P, and a second
// launch adds the chunks in order and applies -X_ii. A workgroup's chain of dependent
// block products stays at most kTrtriChunk long (on d = 4141 the unsplit form spent up
// to 65 products in one workgroup).
constexpr int kTrtriChunk = 4;

__global__ void __launch_bounds__(kBlock) k_trtri_part(const double* L, const double* X, int d,
                                                       int s, int nchunk, double* P) {
  __shared__ __align__(16) double sa[kNB][kNB + 2];
  __shared__ __align__(16) double sb[kNB][kNB + 2];
  const int ii = blockIdx.x / nchunk, ch = blockIdx.x % nchunk;
  const int i = ii + s, j = i - s;
  const int ri = i * kNB, cj = j * kNB, mi = min(kNB, d - ri);
  const int k0 = j + ch * kTrtriChunk, k1 = min(i, k0 + kTrtriChunk);
  double acc[4][4] = {};
  RectRegs ga, gb;   // blocks k < i are full
  ga.load(L + int64_t(ri) * d + k0 * kNB, d, mi, kNB);
  gb.load(X + int64_t(k0 * kNB) * d + cj, d, kNB, kNB);
  for (int k = k0; k < k1; ++k) {
    ga.store<1>(sa);   // sa[m][r] = L_ik(r, m)
    gb.store<0>(sb);   // sb[m][c] = X_kj(m, c)
    __syncthreads();
    if (k + 1 < k1) {
      ga.load(L + int64_t(ri) * d + (k + 1) * kNB, d, mi, kNB);
      gb.load(X + int64_t((k + 1) * kNB) * d + cj, d, kNB, kNB);
    }
    block_mac(sa, sb, acc);
    __syncthreads();
  }
  double* out = P + int64_t(blockIdx.x) * kNB * kNB;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) out[mac_row(v) * kNB + mac_col(u)] = acc[u][v];
}

__global__ void __launch_bounds__(kBlock) k_trtri_fin(double* X, int d, int s, int nchunk,
                                                      const double* P) {
  __shared__ __align__(16) double sa[kNB][kNB + 2];
  __shared__ __align__(16) double sb[kNB][kNB + 2];
  const int ii = blockIdx.x, i = ii + s, j = i - s;
  const int ri = i * kNB, cj = j * kNB, mi = min(kNB, d - ri);
  double t[4][4] = {};
  for (int ch = 0; ch < nchunk; ++ch) {   // fixed order
    const double* part = P + int64_t(ii * nchunk + ch) * kNB * kNB;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) t[u][v] += part[mac_row(v) * kNB + mac_col(u)];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) sb[mac_row(v)][mac_col(u)] = t[u][v];   // T(m, c)
  stage_rect<1>(sa, X + int64_t(ri) * d + ri, d, mi, mi);                // sa[m][r] = X_ii(r, m)
  __syncthreads();
  double y[4][4] = {};
  block_mac(sa, sb, y);
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (mac_row(v) < mi) X[int64_t(ri + mac_row(v)) * d + cj + mac_col(u)] = -y[u][v];
}

// doubles of scratch the split diagonals of cholesky_inverse need (0 when none is split)
static int64_t trtri_scratch(int d) {
  const int nblk = (d + kNB - 1) / kNB;
  int64_t most = 0;
  for (int s = kTrtriChunk + 1; s < nblk; ++s)
    most = std::max<int64_t>(most, int64_t(nblk - s) * ((s + kTrtriChunk - 1) / kTrtriChunk));
  return most * kNB * kNB;
}

// out = Li^T Li for lower-block-triangular Li (= L^-1), one 64x64 block (I >= J) per
// workgroup: out_IJ = sum_{k >= I} Li_kI^T Li_kJ, written to (I, J) and mirrored to (J, I).
__global__ void __launch_bounds__(kBlock) k_lower_gram(const double* Li, double* out, int d,
                                                       int nblk) {
  __shared__ __align__(16) double sa[kNB][kNB + 2];
  __shared__ __align__(16) double sb[kNB][kNB + 2];
  int I = 0;
  while ((I + 1) * (I + 2) / 2 <= int(blockIdx.x)) ++I;
  const int J = int(blockIdx.x) - I * (I + 1) / 2;
  const int mI = min(kNB, d - I * kNB), mJ = min(kNB, d - J * kNB);
  double acc[4][4] = {};
  RectRegs ga, gb;
  {
    const int mk = min(kNB, d - I * kNB);
    ga.load(Li + int64_t(I * kNB) * d + I * kNB, d, mk, mI);
    gb.load(Li + int64_t(I * kNB) * d + J * kNB, d, mk, mJ);
  }
  for (int k = I; k < nblk; ++k) {
    ga.store<0>(sa);   // sa[m][r] = Li_kI(m, r)
    gb.store<0>(sb);   // sb[m][c] = Li_kJ(m, c)
    __syncthreads();
    if (k + 1 < nblk) {
      const int mk = min(kNB, d - (k + 1) * kNB);
      ga.load(Li + int64_t((k + 1) * kNB) * d + I * kNB, d, mk, mI);
      gb.load(Li + int64_t((k + 1) * kNB) * d + J * kNB, d, mk, mJ);
    }
    block_mac(sa, sb, acc);
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = mac_row(v), c = mac_col(u);
      if (r < mI && c < mJ) {
        out[int64_t(I * kNB + r) * d + J * kNB + c] = acc[u][v];
        if (I != J) out[int64_t(J * kNB + c) * d + I * kNB + r] = acc[u][v];
      }
    }
}

// E (in L, overwritten by its lower Cholesky factor and then by scratch) -> X = E^-1 =
// L^-T L^-1. A non-positive pivot raises *bad.
static int cholesky_inverse(double* L, double* X, int d, int32_t* bad, double* scratch,
                            hipStream_t st) {
  for (int kb = 0; kb < d; kb += kNB) {
    const int nb = std::min(kNB, d - kb);
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(psl::kWave), 0, st, L, d, kb, bad);
    const int rest = d - kb - nb;
    if (rest > 0) {
      hipLaunchKernelGGL(k_trsm_panel, dim3(nblocks(rest, kBlock / psl::kWave)), dim3(kBlock), 0,
                         st, L, d, kb);
      // rest > 0 implies nb = kNB: the trailing update's block product always has K = kNB
      const double* P = L + int64_t(kb + nb) * d + kb;   // rest x nb panel
      double* C = L + int64_t(kb + nb) * d + kb + nb;    // trailing block
      dim3 grid(nblocks(rest, 64), nblocks(rest, 64));
      hipLaunchKernelGGL((k_gemm_sub<0, 1, 1>), grid, dim3(kBlock), 0, st, C, d, P, d, P, d,
                         rest, rest, nb);
    }
  }
  // L^-1: diagonal blocks, then one block diagonal per launch (into X); E^-1 = L^-T L^-1
  // as a block Gram product into L's storage (the factor is no longer needed), copied to X
  const int nblk = (d + kNB - 1) / kNB;
  hipLaunchKernelGGL(k_trtri_diag, dim3(nblk), dim3(psl::kWave), 0, st, L, X, d);
  for (int s = 1; s < nblk; ++s) {
    const int nchunk = (s + kTrtriChunk - 1) / kTrtriChunk;
    if (nchunk == 1) {
      hipLaunchKernelGGL(k_trtri_off, dim3(nblk - s), dim3(kBlock), 0, st, L, X, d, s);
    } else {
      hipLaunchKernelGGL(k_trtri_part, dim3((nblk - s) * nchunk), dim3(kBlock), 0, st, L, X, d,
                         s, nchunk, scratch);
      hipLaunchKernelGGL(k_trtri_fin, dim3(nblk - s), dim3(kBlock), 0, st, X, d, s, nchunk,
                         scratch);
    }
  }
  hipLaunchKernelGGL(k_lower_gram, dim3(nblk * (nblk + 1) / 2), dim3(kBlock), 0, st, X, L, d,
                     nblk);
  PSL_HIP(hipMemcpyAsync(X, L, sizeof(double) * size_t(d) * size_t(d), hipMemcpyDeviceToDevice,
                         st));
  PSL_HIP(hipGetLastError());
  return PSL_OK;
}

// ---------------------------------------------------------------------------------------
// work tiling: subdomain boxes of the floor partition, split to at most tile_max cells
// ---------------------------------------------------------------------------------------
static inline int part_lo(int b, int n, int s) {  // first index of part b in a floor partition
  return int((int64_t(b) * n + s - 1) / s);
}

static std::vector<Tile> make_tiles(int nx, int ny, int nz, const int nsub[3], int tile_max,
                                    bool span) {
  std::vector<Tile> out;
  const int bstep = span ? 2 : 1;
  for (int bz = 0; bz < nsub[2]; ++bz)
    for (int by = 0; by < nsub[1]; ++by)
      for (int bx = 0; bx < nsub[0]; bx += bstep) {
        const int x0 = part_lo(bx, nx, nsub[0]);
        const int x1 = part_lo(std::min(bx + bstep, nsub[0]), nx, nsub[0]);
        const int y0 = part_lo(by, ny, nsub[1]), y1 = part_lo(by + 1, ny, nsub[1]);
        const int z0 = part_lo(bz, nz, nsub[2]), z1 = part_lo(bz + 1, nz, nsub[2]);
        const int ex = x1 - x0, ey = y1 - y0, ez = z1 - z0;
        if (ex <= 0 || ey <= 0 || ez <= 0) continue;
        // fewest z chunks whose largest part fits, else whole planes cut into the fewest
        // y chunks that fit, else rows cut in x
        int cz = 1, cy = 1, cx = 1;
        const int64_t vol = int64_t(ex) * ey * ez;
        const int64_t plane = int64_t(ex) * ey;
        if (vol > tile_max) {
          cz = int(std::min<int64_t>(ez, (vol + tile_max - 1) / tile_max));
          while (cz < ez && plane * ((ez + cz - 1) / cz) > tile_max) ++cz;
          if (plane * ((ez + cz - 1) / cz) > tile_max) {
            cz = ez;
            cy = int(std::min<int64_t>(ey, (plane + tile_max - 1) / tile_max));
            while (cy < ey && int64_t(ex) * ((ey + cy - 1) / cy) > tile_max) ++cy;
            if (int64_t(ex) * ((ey + cy - 1) / cy) > tile_max) {
              cy = ey;
              cx = (ex + tile_max - 1) / tile_max;
            }
          }
        }
        for (int kz = 0; kz < cz; ++kz)
          for (int ky = 0; ky < cy; ++ky)
            for (int kx = 0; kx < cx; ++kx) {
              Tile t;
              t.x0 = x0 + part_lo(kx, ex, cx);
              t.sx = part_lo(kx + 1, ex, cx) - part_lo(kx, ex, cx);
              t.y0 = y0 + part_lo(ky, ey, cy);
              t.sy = part_lo(ky + 1, ey, cy) - part_lo(ky, ey, cy);
              t.z0 = z0 + part_lo(kz, ez, cz);
              t.sz = part_lo(kz + 1, ez, cz) - part_lo(kz, ez, cz);
              t.ncell = t.sx * t.sy * t.sz;
              t.nslot = 0;
              if (t.ncell > 0) out.push_back(t);
            }
      }
  return out;
}

// ---------------------------------------------------------------------------------------
// context life cycle
// ---------------------------------------------------------------------------------------
extern "C" void psl_destroy(psl_ctx* c) {
  if (!c) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(c->dev);
  (void)hipDeviceSynchronize();
  psl_alloc_stream = nullptr;   // the caller's stream may be gone; the device is idle
  psl::destroy_batch_plan(c->plan);
  for (int i = 0; i < psl::kGraphSlots; ++i) {
    if (c->graphs64[i].exec) (void)hipGraphExecDestroy(c->graphs64[i].exec);
    if (c->graphs32[i].exec) (void)hipGraphExecDestroy(c->graphs32[i].exec);
  }
  for (void* blk : c->blocks) psl_internal_free(blk);
  psl_internal_pinned_put(c->h_sc);
  psl_internal_pinned_put(c->pc_h);
  if (c->gm_host) (void)hipHostFree(c->gm_host);
  for (hipEvent_t ev : c->gm_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (c->prof_ev) {
    for (int i = 0; i < 2 * c->prof_cap; ++i) (void)hipEventDestroy(c->prof_ev[i]);
    delete[] c->prof_ev;
  }
  (void)hipSetDevice(cur);
  delete c;
}

#define PSL_TRY(expr)            \
  do {                           \
    int _rc = (expr);            \
    if (_rc != PSL_OK) {         \
      psl_destroy(c);            \
      return _rc;                \
    }                            \
  } while (0)

#define PSL_TRYHIP(call)                                                          \
  do {                                                                            \
    hipError_t _e = (call);                                                       \
    if (_e != hipSuccess) {                                                       \
      std::fprintf(stderr, "libpsl: %s failed: %s\n", #call, hipGetErrorString(_e)); \
      psl_destroy(c);                                                             \
      return PSL_EHIP;                                                            \
    }                                                                             \
  } while (0)

template <typename T>
static int dalloc(psl_ctx* c, T** p, int64_t count) {
  return psl_ctx_alloc(c, reinterpret_cast<void**>(p), sizeof(T) * size_t(count));
}

extern "C" int psl_setup_E(psl_ctx** out, const psl_grid* g, const double* Tx,
                           const double* Ty, const double* Tz, const int32_t* labels,
                           int32_t d, const int32_t nsub[3], void* stream) {
  return psl_setup_E_ex(out, g, Tx, Ty, Tz, labels, d, nsub, nullptr, stream);
}

extern "C" void psl_default_setup_opts(psl_setup_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
}

// the lower 64 x 64 blocks of E^-1, packed block after block (row-major inside a block,
// zero past d) for the symmetric coarse product: workgroup t copies block t
__global__ void __launch_bounds__(kBlock) k_pack_sym(const double* __restrict__ Einv,
                                                     double* __restrict__ Esym, int d) {
  constexpr int B = psl::kSymBlock;
  int I, J;
  psl::sym_block_of(blockIdx.x, I, J);
  double* dst = Esym + int64_t(blockIdx.x) * B * B;
  for (int i = threadIdx.x; i < B * B; i += kBlock) {
    const int row = I * B + i / B, col = J * B + i % B;
    dst[i] = (row < d && col < d) ? Einv[int64_t(row) * d + col] : 0.0;
  }
}

// Per-tile coarse tables of the float32 update (one workgroup per tile): the labels the
// tile's cut faces reference are marked in an LDS bitmap over [0, d) (d <= 8192: 256
// words, one per thread); a label's local index is its rank among the marked ones, so the
// table is in ascending label order. Each face is packed into one word: local cell (bits
// 0..10, tiles hold at most 2048 cells), the first-face bit 31, the local index of its own
// label << 11 and of the other label << 18 (127 for an outer face). A tile with more than
// 126 labels raises *overflow (the context then keeps the unpacked faces).
__global__ void __launch_bounds__(kBlock) k_az_pack(const int32_t* az_ptr, const int32_t* az_cell,
                                                    const int32_t* az_lab, const int32_t* az_oth,
                                                    int d, int32_t* az_pk, int32_t* tlab,
                                                    int32_t* tlab_n, int32_t* overflow) {
  constexpr int NW = PSL_MAX_DENSE_D / 32;
  static_assert(NW <= kBlock, "one bitmap word per thread");
  __shared__ uint32_t bits[NW];
  __shared__ int32_t wrank[NW];
  __shared__ int32_t wtot[kBlock / psl::kWave];
  const int t = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & (psl::kWave - 1), w = tid / psl::kWave;
  const int a = az_ptr[t], b = az_ptr[t + 1], nw = (d + 31) / 32;
  if (tid < NW) bits[tid] = 0u;
  __syncthreads();
  for (int k = a + tid; k < b; k += kBlock) {
    const int ls = az_lab[k], lo = az_oth[k];
    atomicOr(&bits[ls >> 5], 1u << (ls & 31));
    if (lo >= 0) atomicOr(&bits[lo >> 5], 1u << (lo & 31));
  }
  __syncthreads();
  // exclusive prefix of the words' popcounts
  const int cnt = tid < nw ? __popc(bits[tid]) : 0;
  int incl = cnt;
  for (int off = 1; off < psl::kWave; off <<= 1) {
    const int v = __shfl_up(incl, off);
    if (lane >= off) incl += v;
  }
  if (lane == psl::kWave - 1) wtot[w] = incl;
  __syncthreads();
  int before = 0, total = 0;
  for (int k = 0; k < kBlock / psl::kWave; ++k) {
    if (k < w) before += wtot[k];
    total += wtot[k];
  }
  if (tid < NW) wrank[tid] = before + incl - cnt;
  if (total > psl::kTileLabels - 1) {   // uniform
    if (tid == 0) overflow[0] = 1;
    return;
  }
  __syncthreads();
  if (tid == 0) tlab_n[t] = total;
  if (tid < nw) {
    uint32_t m = bits[tid];
    int r = wrank[tid];
    while (m) {
      tlab[int64_t(t) * psl::kTileLabels + r++] = tid * 32 + (__ffs(m) - 1);
      m &= m - 1u;
    }
  }
  for (int k = a + tid; k < b; k += kBlock) {
    const int ls = az_lab[k], lo = az_oth[k], cw = az_cell[k];
    const int il = wrank[ls >> 5] + __popc(bits[ls >> 5] & ((1u << (ls & 31)) - 1u));
    const int io = lo < 0 ? psl::kTileLabels - 1
                          : wrank[lo >> 5] + __popc(bits[lo >> 5] & ((1u << (lo & 31)) - 1u));
    az_pk[k] = int32_t((uint32_t(cw) & 0x80000000u) | (uint32_t(cw) & 0x7FFu) |
                       (uint32_t(il) << 11) | (uint32_t(io) << 18));
  }
}

extern "C" int psl_setup_E_ex(psl_ctx** out, const psl_grid* g, const double* Tx,
                              const double* Ty, const double* Tz, const int32_t* labels,
                              int32_t d, const int32_t nsub[3], const psl_setup_opts* so,
                              void* stream) {
  psl_alloc_stream = static_cast<hipStream_t>(stream);
  if (so) {
    if (so->tile_cells != 0 && (so->tile_cells < 64 || so->tile_cells > 2048)) return PSL_EINVAL;
    if (so->finish_kernels < -1 || so->finish_kernels > 1) return PSL_EINVAL;
    if (so->coarse_sym < -1 || so->coarse_sym > 1) return PSL_EINVAL;
    if (so->stencil_split < -1 || so->stencil_split > 1) return PSL_EINVAL;
    if (so->face_tables < -1 || so->face_tables > 1) return PSL_EINVAL;
    if (so->wide_tiles < -1 || so->wide_tiles > 1) return PSL_EINVAL;
    for (int32_t r : so->reserved)
      if (r != 0) return PSL_EINVAL;
  }
  if (!out) return PSL_EINVAL;
  *out = nullptr;
  if (const int grc = grid_check(g)) return grc;
  if (!Tx || !Ty || !Tz || !labels || d < 1) return PSL_EINVAL;
  if (d > PSL_MAX_DENSE_D) return PSL_ENOTSUP;
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  int ns[3];
  if (nsub) {
    const int ext[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
      if (nsub[a] < 1 || nsub[a] > ext[a]) return PSL_EINVAL;
      ns[a] = nsub[a];
    }
  } else {
    ns[0] = (nx + 15) / 16;
    ns[1] = (ny + 15) / 16;
    ns[2] = (nz + 7) / 8;
  }
  if (int64_t(d) > int64_t(nx) * ny * nz) return PSL_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  static std::atomic<uint64_t> next_id{1};
  psl_ctx* c = new psl_ctx();
  c->id = next_id.fetch_add(1);
  (void)hipGetDevice(&c->dev);
  c->nx = nx;
  c->ny = ny;
  c->nz = nz;
  c->n = int64_t(nx) * ny * nz;
  c->d = d;
  for (int a = 0; a < 3; ++a) c->nsub[a] = ns[a];
  const int n = int(c->n);
  const int64_t nfx = int64_t(nx + 1) * ny * nz, nfy = int64_t(nx) * (ny + 1) * nz,
                nfz = int64_t(nx) * ny * (nz + 1);
  GridDev gd{nx, ny, nz};

  // one block for what the context and both solve precisions need (further blocks only
  // if the tiling or the cut faces outgrow the estimate)
  {
    const size_t nn = size_t(n), nf = size_t(nfx + nfy + nfz);
    const size_t est = nf * 12 + nn * (8 + 4 + 4 + 1 + 16) + nn * (7 * 8 + 7 * 4) +
                       size_t(d) * d * 8 * 3 + nn * 3 * 28 / 4 + (size_t(16) << 20);
    void* first = nullptr;
    PSL_TRY(psl_ctx_alloc(c, &first, 256, est));
  }
  PSL_TRY(dalloc(c, &c->Tx, nfx));
  PSL_TRY(dalloc(c, &c->Ty, nfy));
  PSL_TRY(dalloc(c, &c->Tz, nfz));
  PSL_TRY(dalloc(c, &c->Tx32, nfx));
  PSL_TRY(dalloc(c, &c->Ty32, nfy));
  PSL_TRY(dalloc(c, &c->Tz32, nfz));
  PSL_TRY(dalloc(c, &c->invdiag, n));
  PSL_TRY(dalloc(c, &c->invdiag32, n));
  PSL_TRY(dalloc(c, &c->labels, n));
  PSL_TRY(dalloc(c, &c->slot, n));
  int32_t* flags = nullptr;  // 0 diag, 1 tile overflow, 2 empty column, 3 label range, 4 E pivot,
                             // 5 tile label table overflow
  PSL_TRY(dalloc(c, &flags, 8));
  auto free_flags = [&]() { flags = nullptr; };   // arena memory, freed with the context
  int32_t hflags[8] = {0};
  auto read_flags = [&]() -> int {
    if (hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, st) != hipSuccess)
      return PSL_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return PSL_EHIP;
    return PSL_OK;
  };
#define PSL_FAIL(rc)   \
  do {                 \
    free_flags();      \
    psl_destroy(c);    \
    return (rc);       \
  } while (0)

  hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(kBlock), 0, st, flags, 0, int64_t(8));
  if (hipMemcpyAsync(c->Tx, Tx, sizeof(double) * nfx, hipMemcpyDeviceToDevice, st) ||
      hipMemcpyAsync(c->Ty, Ty, sizeof(double) * nfy, hipMemcpyDeviceToDevice, st) ||
      hipMemcpyAsync(c->Tz, Tz, sizeof(double) * nfz, hipMemcpyDeviceToDevice, st) ||
      hipMemcpyAsync(c->labels, labels, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st))
    PSL_FAIL(PSL_EHIP);
  hipLaunchKernelGGL(k_check_labels, dim3(nblocks(n)), dim3(kBlock), 0, st, c->labels, n, d,
                     flags + 3);
  hipLaunchKernelGGL(k_diag, dim3(nblocks(n)), dim3(kBlock), 0, st, gd, c->Tx, c->Ty, c->Tz,
                     c->invdiag, c->invdiag32, flags);
  hipLaunchKernelGGL(k_cast_f32, dim3(nblocks(nfx)), dim3(kBlock), 0, st, c->Tx, c->Tx32, nfx);
  hipLaunchKernelGGL(k_cast_f32, dim3(nblocks(nfy)), dim3(kBlock), 0, st, c->Ty, c->Ty32, nfy);
  hipLaunchKernelGGL(k_cast_f32, dim3(nblocks(nfz)), dim3(kBlock), 0, st, c->Tz, c->Tz32, nfz);

  // tiles: enough workgroups to fill the chip (>= 8 per CU when the grid allows) unless
  // the caller fixes the size; then shrink until no tile holds more than kMaxSlots labels
  int tile_max = 1024;
  while (tile_max > 256 && int64_t(n) / tile_max < 2048) tile_max /= 2;
  if (so && so->tile_cells) tile_max = so->tile_cells;
  // step decisions in finish kernels on large grids (the pass kernels then skip the
  // repeated partial sums; below this size the extra launches cost more)
  c->pre = (so && so->finish_kernels) ? (so->finish_kernels > 0) : (int64_t(n) >= (int64_t(1) << 21));
  // tiles two subdomain boxes wide when a box is under 32 cells wide: rows of at least 128
  // bytes in the float32 passes (whole cache lines) instead of half lines; by default not
  // on grids under 2^15 cells, whose vectors stay in cache
  bool span = ns[0] >= 2 && nx / ns[0] < 32 &&
              (so && so->wide_tiles ? so->wide_tiles > 0 : int64_t(n) >= (int64_t(1) << 15));
  for (;;) {
    c->h_tiles = make_tiles(nx, ny, nz, ns, tile_max, span);
    c->ntiles = int(c->h_tiles.size());
    c->tiles = nullptr;
    c->tile_lab = nullptr;
    if (dalloc(c, &c->tiles, c->ntiles) || dalloc(c, &c->tile_lab, int64_t(c->ntiles) * kMaxSlots))
      PSL_FAIL(PSL_ENOMEM);
    if (hipMemcpyAsync(c->tiles, c->h_tiles.data(), sizeof(Tile) * c->ntiles,
                       hipMemcpyHostToDevice, st))
      PSL_FAIL(PSL_EHIP);
    hipLaunchKernelGGL(k_tile_labels, dim3(c->ntiles), dim3(kBlock), 0, st, gd, c->tiles,
                       c->labels, c->tile_lab, c->tiles, c->slot, flags + 1);
    // the first read also reports the label-range and diagonal checks above (the tile
    // pass only compares labels, so it is safe on out-of-range values)
    if (read_flags()) PSL_FAIL(PSL_EHIP);
    if (hflags[3]) PSL_FAIL(PSL_EINVAL);  // a label outside [0, d)
    if (hflags[0]) PSL_FAIL(PSL_ENOTSPD);
    if (!hflags[1]) {
      c->wide_tiles = span;
      break;
    }
    if (span) {
      span = false;   // too many labels in a tile: first give up the wide tiles
    } else {
      if (tile_max == 1) PSL_FAIL(PSL_EINVAL);
      tile_max = std::max(1, tile_max / 2);
    }
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(kBlock), 0, st, flags, 0, int64_t(8));
  }
  // label -> partial lists
  const int nparts = c->ntiles * kMaxSlots;
  int32_t* cnt = nullptr;
  if (dalloc(c, &cnt, d + 1) || dalloc(c, &c->lab_ptr, d + 1) || dalloc(c, &c->lab_part, nparts))
    PSL_FAIL(PSL_ENOMEM);
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(nblocks(d + 1)), dim3(kBlock), 0, st, cnt, 0,
                     int64_t(d + 1));
  hipLaunchKernelGGL(k_lab_count, dim3(nblocks(nparts)), dim3(kBlock), 0, st, c->tile_lab,
                     nparts, cnt, d, flags + 3);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, cnt, c->lab_ptr, d);
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(nblocks(d + 1)), dim3(kBlock), 0, st, cnt, 0,
                     int64_t(d + 1));
  hipLaunchKernelGGL(k_lab_fill, dim3(nblocks(nparts)), dim3(kBlock), 0, st, c->tile_lab,
                     nparts, c->lab_ptr, cnt, c->lab_part, d);
  hipLaunchKernelGGL(k_lab_sort, dim3(nblocks(d)), dim3(kBlock), 0, st, c->lab_ptr,
                     c->lab_part, d, flags + 2);
  if (dalloc(c, &c->slot_pos, nparts)) PSL_FAIL(PSL_ENOMEM);
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(nblocks(nparts)), dim3(kBlock), 0, st, c->slot_pos, 0,
                     int64_t(nparts));
  hipLaunchKernelGGL(k_slot_pos, dim3(nblocks(nparts)), dim3(kBlock), 0, st, c->lab_ptr,
                     c->lab_part, d, c->slot_pos);

  // interface rows of A Z
  int32_t* tile_cnt = nullptr;
  if (dalloc(c, &tile_cnt, c->ntiles + 1) || dalloc(c, &c->az_ptr, c->ntiles + 1))
    PSL_FAIL(PSL_ENOMEM);
  hipLaunchKernelGGL(k_az_count, dim3(c->ntiles), dim3(kBlock), 0, st, gd, c->tiles, c->Tx,
                     c->Ty, c->Tz, c->labels, tile_cnt);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, tile_cnt, c->az_ptr, c->ntiles);

  // one round trip for every size the host needs: the tiles with their label counts, the
  // number of cut faces and of label partials
  int32_t m = 0;
  if (hipMemcpyAsync(c->h_tiles.data(), c->tiles, sizeof(Tile) * c->ntiles,
                     hipMemcpyDeviceToHost, st) ||
      hipMemcpyAsync(&m, c->az_ptr + c->ntiles, sizeof(int32_t), hipMemcpyDeviceToHost, st) ||
      hipMemcpyAsync(&c->npart, c->lab_ptr + d, sizeof(int32_t), hipMemcpyDeviceToHost, st) ||
      hipStreamSynchronize(st))
    PSL_FAIL(PSL_EHIP);
  c->nslot_max = 1;
  int max_cells = 1;
  for (const Tile& t : c->h_tiles) {
    c->nslot_max = std::max(c->nslot_max, t.nslot);
    max_cells = std::max(max_cells, t.ncell);
  }
  c->tile_max = max_cells;
  c->cpt = (max_cells + kBlock - 1) / kBlock;
  c->m_az = m;
  if (dalloc(c, &c->az_cell, m) || dalloc(c, &c->az_lab, m) || dalloc(c, &c->az_oth, m) ||
      dalloc(c, &c->az_t, m) || dalloc(c, &c->az_t32, m))
    PSL_FAIL(PSL_ENOMEM);
  hipLaunchKernelGGL(k_az_fill, dim3(c->ntiles), dim3(kBlock), 0, st, gd, c->tiles, c->Tx,
                     c->Ty, c->Tz, c->labels, c->az_ptr, c->az_cell, c->az_lab, c->az_oth,
                     c->az_t, c->az_t32);
  c->face_tab = !(so && so->face_tables < 0);
  if (c->face_tab) {
    if (dalloc(c, &c->az_pk, std::max(m, 1)) ||
        dalloc(c, &c->tlab, int64_t(c->ntiles) * psl::kTileLabels) ||
        dalloc(c, &c->tlab_n, c->ntiles))
      PSL_FAIL(PSL_ENOMEM);
    hipLaunchKernelGGL(k_az_pack, dim3(c->ntiles), dim3(kBlock), 0, st, c->az_ptr, c->az_cell,
                       c->az_lab, c->az_oth, d, c->az_pk, c->tlab, c->tlab_n, flags + 5);
  }

  // coarse GEMV layout and solve work space
  c->coarse_blocks = (d + psl::kCoarseRows - 1) / psl::kCoarseRows;
  // coarse workgroups stage all of s (d <= 4096 doubles of LDS) and each re-sums the
  // label partials; beyond ~4M partial reads a separate reduction kernel is cheaper
  c->coarse_fused = (d <= 4096) && (int64_t(c->npart) * c->coarse_blocks <= (int64_t(1) << 22));
  // large d: the coarse product reads only the lower block triangle of E^-1
  c->coarse_sym = (so && so->coarse_sym) ? (so->coarse_sym > 0) : (d >= psl::kSymMinD);
  c->sym_parts = (d + psl::kBlock / 4 - 1) / (psl::kBlock / 4);
  c->sd_split = !(so && so->stencil_split < 0);
  // grids up to 4096 cells with up to 32 vectors: float64 inner solves in one workgroup
  // (the iteration's vectors in LDS, no launch per iteration)
  c->small = (n <= 4096) && (d <= 32);
  const int64_t dd = int64_t(d) * d;
  double* Lw = nullptr;
  if (dalloc(c, &c->E, dd) || dalloc(c, &c->Einv, dd) || dalloc(c, &Lw, dd) ||
      dalloc(c, &c->zq, std::max(1, c->npart)) || dalloc(c, &c->zr, std::max(1, c->npart)) ||
      dalloc(c, &c->red, int64_t(c->ntiles) * 4) || dalloc(c, &c->s, d) || dalloc(c, &c->e, d) ||
      dalloc(c, &c->sr, d) || dalloc(c, &c->er, d) ||
      dalloc(c, &c->cpart, 4 * std::max(c->coarse_blocks, c->sym_parts)) ||
      dalloc(c, &c->r64, n) || dalloc(c, &c->t64, n) || dalloc(c, &c->sc, 1))
    PSL_FAIL(PSL_ENOMEM);
  if (c->coarse_sym) {
    const int64_t nb = (d + psl::kSymBlock - 1) / psl::kSymBlock;
    if (dalloc(c, &c->spart, nb * nb * psl::kSymBlock) ||
        dalloc(c, &c->spart2, nb * nb * psl::kSymBlock) ||
        dalloc(c, &c->Esym, nb * (nb + 1) / 2 * psl::kSymBlock * psl::kSymBlock))
      PSL_FAIL(PSL_ENOMEM);
  }
  static_assert(sizeof(psl::Scalars) <= 1024, "pinned mirror slot size");
  c->h_sc = static_cast<psl::Scalars*>(psl_internal_pinned_get(sizeof(psl::Scalars)));
  if (!c->h_sc) PSL_FAIL(PSL_ENOMEM);
  std::memset(c->h_sc, 0, sizeof(psl::Scalars));
  if (hipMemcpyAsync(c->sc, c->h_sc, sizeof(psl::Scalars), hipMemcpyHostToDevice, st))
    PSL_FAIL(PSL_EHIP);

  // E = Z^T A Z, then Cholesky and inverse; the flags read waits for all of the set-up
  hipLaunchKernelGGL(k_E_rows, dim3(d), dim3(kBlock), 0, st, c->lab_ptr, c->lab_part, c->az_ptr,
                     c->az_lab, c->az_oth, c->az_t, c->E, d);
  if (hipMemcpyAsync(Lw, c->E, sizeof(double) * dd, hipMemcpyDeviceToDevice, st))
    PSL_FAIL(PSL_EHIP);
  double* tri_scratch = nullptr;
  const int64_t ntri = trtri_scratch(d);
  if (ntri > 0 && dalloc(c, &tri_scratch, ntri)) PSL_FAIL(PSL_ENOMEM);
  int rc = cholesky_inverse(Lw, c->Einv, d, flags + 4, tri_scratch, st);
  if (rc == PSL_OK && c->coarse_sym) {
    const int nb = (d + psl::kSymBlock - 1) / psl::kSymBlock;
    hipLaunchKernelGGL(k_pack_sym, dim3(nb * (nb + 1) / 2), dim3(kBlock), 0, st, c->Einv,
                       c->Esym, d);
  }
  if (rc == PSL_OK) rc = read_flags();
  if (rc != PSL_OK) PSL_FAIL(rc);
  if (hflags[2] || hflags[3]) PSL_FAIL(PSL_EINVAL);  // empty column / label out of range
  if (hflags[4]) PSL_FAIL(PSL_ENOTSPD);
  if (hflags[5]) c->face_tab = 0;   // a tile references more labels than a table holds
  free_flags();
#undef PSL_FAIL
  *out = c;
  return PSL_OK;
}

extern "C" int psl_get_coarse(psl_ctx* c, double* E, double* Einv, int32_t* d, void* stream) {
  if (!c) return PSL_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t bytes = sizeof(double) * size_t(c->d) * c->d;
  if (E) PSL_HIP(hipMemcpyAsync(E, c->E, bytes, hipMemcpyDeviceToDevice, st));
  if (Einv) PSL_HIP(hipMemcpyAsync(Einv, c->Einv, bytes, hipMemcpyDeviceToDevice, st));
  if (d) *d = c->d;
  return PSL_OK;
}

extern "C" int psl_get_info(const psl_ctx* c, psl_ctx_info* info) {
  if (!c || !info) return PSL_EINVAL;
  info->n = c->n;
  info->d = c->d;
  info->ntiles = c->ntiles;
  info->m_faces = c->m_az;
  info->nslot_max = c->nslot_max;
  info->coarse_sym = c->coarse_sym;
  info->small_solve = c->small;
  info->face_tables = c->face_tab;
  info->wide_tiles = c->wide_tiles;
  return PSL_OK;
}
