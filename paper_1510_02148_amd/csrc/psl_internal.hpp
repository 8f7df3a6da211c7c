// Internal declarations shared by the libpsl translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <vector>

#include "../../include/psl.h"

namespace psl {

constexpr int kBlock = 256;          // threads per workgroup for every cell kernel
constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kMaxSlots = PSL_MAX_TILE_LABELS;
constexpr int kCoarseRows = 8;       // coarse GEMV rows per workgroup (two per wave)
constexpr int kSymBlock = 64;        // block size of the symmetric coarse product
constexpr int kSymMinD = 1024;       // d from which the coarse product is the symmetric one
constexpr int kTileLabels = 128;     // per-tile coarse table of the float32 update: local
                                     // indices 0..126, 127 marks an outer face

// Work tile: a box of cells inside one subdomain; one workgroup per tile.
struct Tile {
  int32_t x0, y0, z0;   // first cell
  int32_t sx, sy, sz;   // extent
  int32_t ncell;        // sx*sy*sz
  int32_t nslot;        // distinct labels in the tile
};

// Device-resident scalars of one solve; read and written only by kernels. Quantities
// carried from one CG iteration to the next are double-buffered by iteration parity, so a
// kernel reads slot (i+1)&1 while its workgroup 0 writes slot i&1.
struct Scalars {
  double gamma[2];   // (r, M^-1 r); in the two-reduction form rho = (r, M^-1 r)
  double alpha[2];   // step length (single-reduction form)
  double rr;         // ||r||^2 at the last check
  double goal2;      // inner stop: ||r||^2 <= goal2
  double rnorm;      // float64 refinement residual norm
  double sigma;      // inner scale: r0 = sigma * r
  double bnorm2;
  double delta;      // (p, P1 A p) of the last step (diagnostic)
  double ztr2;       // ||Z^T r||^2 of the final float64 residual (diagnostic)
  double beta[2];    // direction coefficient of the step (finish kernels)
  int32_t cnt[2];    // iterations done
  int32_t done;      // inner loop finished (converged or failed)
  int32_t iters;     // inner iterations done in this inner solve
  int32_t status;    // PSL_OK or failure code raised on device
  int32_t maxit;     // iteration budget for this inner solve
  int32_t stop_par;  // parity of the launch that ended the last two-reduction inner solve
  int32_t stalled;   // the one-workgroup inner solve stopped without halving ||r|| in a window
};

template <typename R>
struct VecSet {       // inner CG vectors in precision R
  R* xh = nullptr;      // iterate of the deflated system
  R* rh = nullptr;      // residual
  R* p = nullptr;       // search direction
  R* q = nullptr;       // P1 A p, by recurrence
  R* v = nullptr;       // A M^-1 r
  R* u = nullptr;       // M^-1 r
  R* p2 = nullptr;      // second search-direction buffer (two-reduction form)
};

constexpr int kGraphSlots = 4;      // captured iteration chunks kept per precision

struct GraphSlot {
  int key = -1;                      // chunk, CG form and re-projection it was captured for
  hipGraphExec_t exec = nullptr;
};

}  // namespace psl

namespace psl {
struct BatchPlan;   // batched-solve launch plan (psl_solve.hip)
void destroy_batch_plan(BatchPlan* p);
}  // namespace psl

struct psl_ctx {
  int dev = 0;
  uint64_t id = 0;                    // unique per context in the process (never reused)
  psl::BatchPlan* plan = nullptr;     // batched-solve plan cached on the batch's first context
  int nx = 0, ny = 0, nz = 0;
  int64_t n = 0;
  int d = 0;
  int ntiles = 0;
  int nslot_max = 0;
  int tile_max = 0;                   // cells per tile (<= 2048)
  int cpt = 1;                        // cells per thread = ceil(tile_max / kBlock)
  int wide_tiles = 0;                 // tiles span two x-adjacent subdomain boxes
  int small = 0;                      // float64 inner solves in one workgroup (small grids)
  int16_t* small_lptr = nullptr;      // its label-major cell lists: [d + 1] offsets
  uint16_t* small_lcell = nullptr;    // [n] cells
  int pre = 0;                        // CG step decisions in one-workgroup finish kernels
                                      // (the pass kernels read the coefficients)
  int nsub[3] = {1, 1, 1};
  // operator data (owned copies)
  double *Tx = nullptr, *Ty = nullptr, *Tz = nullptr;
  float *Tx32 = nullptr, *Ty32 = nullptr, *Tz32 = nullptr;
  double* invdiag = nullptr;
  float* invdiag32 = nullptr;
  int32_t* labels = nullptr;
  // tiling
  psl::Tile* tiles = nullptr;
  std::vector<psl::Tile> h_tiles;
  uint8_t* slot = nullptr;            // [n] slot of the cell's label within its tile
  int32_t* tile_lab = nullptr;        // [ntiles*kMaxSlots] label of each slot, -1 unused
  int32_t* lab_ptr = nullptr;         // [d+1] CSR over the (tile, slot) pairs of each label
  int32_t* lab_part = nullptr;        // [npart] tile*kMaxSlots+slot, sorted within a label
  int32_t* slot_pos = nullptr;        // [ntiles*kMaxSlots] position of (tile, slot) in lab_part
  int npart = 0;                      // lab_ptr[d]
  // cut faces of A Z (faces between labels, and Dirichlet faces), grouped by tile and cell
  int32_t* az_ptr = nullptr;          // [ntiles+1]
  int32_t* az_cell = nullptr;         // [m] local cell index in the tile; bit 31 = first face of its cell
  int32_t* az_lab = nullptr;          // [m] label of the cell
  int32_t* az_oth = nullptr;          // [m] label across the face, -1 for an outer face
  double* az_t = nullptr;             // [m] face transmissibility
  float* az_t32 = nullptr;            // [m]
  // per-tile coarse tables (float32 update): the labels a tile's cut faces reference, in
  // ascending order, and each face packed as local cell | first-face bit 31 | local index
  // of its own label << 11 | of the other label << 18 (127: outer face)
  int face_tab = 0;
  int32_t* az_pk = nullptr;           // [m]
  int32_t* tlab = nullptr;            // [ntiles * kTileLabels]
  int32_t* tlab_n = nullptr;          // [ntiles]
  int64_t m_az = 0;
  // coarse operator
  double* E = nullptr;                // [d*d] row-major
  double* Einv = nullptr;             // [d*d]
  int coarse_blocks = 1;              // ceil(d / kCoarseRows) GEMV workgroups
  int coarse_fused = 1;               // coarse workgroups sum s themselves (small d)
  int coarse_sym = 0;                 // coarse product over the lower block triangle of E^-1
  int sd_split = 1;                   // two-reduction stencil split in two (with finish kernels)
  int sym_parts = 0;                  // its summing workgroups: ceil(d / (kBlock / 4))
  double* Esym = nullptr;             // its lower blocks of E^-1, packed [nb (nb + 1) / 2 * 64 * 64]
  double* spart = nullptr;            // its block shares [nb * nb * 64] (nb = ceil(d / 64))
  double* spart2 = nullptr;           // the same for the second right-hand side
  // work
  double* zq = nullptr;               // [npart] label-major partials of Z^T q (or Z^T r)
  double* zr = nullptr;               // [npart] label-major partials of Z^T rhat
  double* red = nullptr;              // [4*ntiles] per-tile scalar partials, quantity-major
  double* cpart = nullptr;            // [4*coarse_blocks] s^T e and slices of the CG partials
  double* upart = nullptr;            // [2*upd_blocks] (r, M^-1 r), (r, r) per update workgroup
  int upd_blocks = 1;                 // workgroups of the two-reduction update pass
  double* s = nullptr;                // [d]
  double* e = nullptr;                // [d]
  double* sr = nullptr;               // [d] Z^T rhat
  double* er = nullptr;               // [d] E^-1 Z^T rhat
  double* r64 = nullptr;              // [n] FP64 outer residual
  double* t64 = nullptr;              // [n] FP64 scratch
  double* xbest = nullptr;            // [n] best projected iterate of the current solve
  double* gm_v = nullptr;             // deflated GMRES: gm_cap basis vectors of n doubles
  int gm_cap = 0;
  double* gm_part = nullptr;          // [(gm_cap + 1) * ceil(n / kBlock)] workgroup partials
  double* gm_dev = nullptr;           // [3 * gm_cap + 4] dots, norm and step coefficients
  double* gm_host = nullptr;          // pinned: two slots of one Arnoldi column each
  hipEvent_t gm_ev[2] = {nullptr, nullptr};  // marks each slot's copy
  double* pc_v = nullptr;             // polynomial-preconditioned CG: p, w, y, y2, d [5 n]
  float* pc_v32 = nullptr;            // its float32 inner solve: p, w, y, y2, d, r, xi [7 n]
  double* pc_part = nullptr;          // workgroup / tile partials of its two dot pairs
  void* pc_sc = nullptr;              // its device scalars
  void* pc_h = nullptr;               // pinned host mirror of them
  psl::Scalars* sc = nullptr;
  psl::Scalars* h_sc = nullptr;       // pinned host mirror
  psl::VecSet<double> v64;
  psl::VecSet<float> v32;
  // captured iteration chunks per precision
  psl::GraphSlot graphs64[psl::kGraphSlots], graphs32[psl::kGraphSlots];
  // device memory arena: every buffer of the context is carved from a few large blocks,
  // released together by psl_destroy
  std::vector<void*> blocks;
  char* arena = nullptr;
  size_t arena_left = 0;
  int last_iters64[8] = {0}, last_iters32[8] = {0};  // inner iterations per refinement step
  // per-launch timing of one CG kernel inside the solves (psl_profile_kernel): events
  // recorded on the solve's stream before and after each launch of that kernel in that
  // precision, up to prof_cap launches
  int prof_kernel = -1;               // PSL_KERNEL_* id, -1 when off
  int prof_mode = 0;                  // PSL_FP64 or PSL_MIXED (float32 launches)
  int prof_cap = 0, prof_count = 0;
  hipEvent_t* prof_ev = nullptr;      // [2 * prof_cap]
};

#define PSL_HIP(call)                                                              \
  do {                                                                             \
    hipError_t _e = (call);                                                        \
    if (_e != hipSuccess) {                                                        \
      std::fprintf(stderr, "libpsl: %s failed: %s (%s:%d)\n", #call,              \
                   hipGetErrorString(_e), __FILE__, __LINE__);                     \
      return PSL_EHIP;                                                             \
    }                                                                              \
  } while (0)

namespace psl {

// ---- reductions ----------------------------------------------------------------------
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// a float64 value moved across lanes by a DPP control (both 32-bit halves; every control
// used here is a permutation within a row of 16 lanes, so every source lane is active
// whenever the whole wave is)
template <int CTRL>
__device__ inline double dpp_double(double v) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  // the move form (no "old" operand to preset; no source lane is ever out of range)
  const int lo = __builtin_amdgcn_mov_dpp(int(unsigned(b)), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(int(unsigned(b >> 32)), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(static_cast<long long>(
      (static_cast<unsigned long long>(unsigned(hi)) << 32) | unsigned(lo)));
}

__device__ inline double read_lane(double v, int lane) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(unsigned(b)), lane));
  const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(unsigned(b >> 32)), lane));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// Sum of a float64 over each row of 16 lanes (every lane active), in a fixed order: a
// butterfly of lane pairs (lane xor 1, xor 2 by quad permutes, then the mirrored quad of
// each 8 and the mirrored 8 of each 16; a + b and b + a round alike, so every lane of a
// row ends holding the same row sum). DPP moves run on the vector ALU; the generic
// version's cross-lane permutes go through the LDS unit.
__device__ inline double row_sum(double v) {
  v += dpp_double<0xB1>(v);    // quad_perm [1, 0, 3, 2]: lane xor 1
  v += dpp_double<0x4E>(v);    // quad_perm [2, 3, 0, 1]: lane xor 2
  v += dpp_double<0x141>(v);   // row_half_mirror: the other quad of each 8
  v += dpp_double<0x140>(v);   // row_mirror: the other 8 of each 16
  return v;
}

// Sum of a float64 over the 64 lanes of a wave, the same value in every lane: the row
// sums, then the four rows added in row order by lane reads.
__device__ inline double wave_sum(double v) {
  v = row_sum(v);
  return ((read_lane(v, 0) + read_lane(v, 16)) + read_lane(v, 32)) + read_lane(v, 48);
}

constexpr int kSumRows = kBlock / 16;   // rows of 16 lanes in a workgroup

// doubles of LDS that block_sum_active<NV> needs
constexpr int block_sum_lds(int nv) { return nv * (kSumRows + 1); }

// Workgroup sums of the entries of v whose bit is set in `active` (the same mask in every
// thread, so the skips are uniform branches), in a fixed order: each row of 16 lanes sums
// by the DPP butterfly, then the 16 row sums of an entry are added in row order by one
// thread, and every thread reads the results back. The other entries are left unreduced
// and must not be read. Each wave moves only its row sums, so an entry costs a wave four
// DPP steps rather than the four steps plus eight lane reads of a whole-wave sum, and the
// row sums of all entries are added by different threads side by side. lds must hold
// block_sum_lds(NV) doubles.
template <int NV>
__device__ inline void block_sum_active(double (&v)[NV], double* lds, unsigned long long active) {
  static_assert(NV <= 64, "active mask");
  static_assert(NV <= kBlock, "one thread per entry");
  const int row = threadIdx.x >> 4;
  double* tot = lds + NV * kSumRows;
#pragma unroll
  for (int k = 0; k < NV; ++k)
    if ((active >> k) & 1ull) v[k] = row_sum(v[k]);
  __syncthreads();
  if ((threadIdx.x & 15) == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if ((active >> k) & 1ull) lds[k * kSumRows + row] = v[k];
  }
  __syncthreads();
  const int e = threadIdx.x;
  if (e < NV && ((active >> e) & 1ull)) {
    const double* r = lds + e * kSumRows;
    double acc = r[0];
#pragma unroll
    for (int j = 1; j < kSumRows; ++j) acc += r[j];
    tot[e] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k)
    if ((active >> k) & 1ull) v[k] = tot[k];
  __syncthreads();
}

// lower-triangle block t = I (I + 1) / 2 + J (J <= I) of the symmetric coarse product
__device__ inline void sym_block_of(int t, int& I, int& J) {
  int i = int((sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  I = i;
  J = t - i * (i + 1) / 2;
}

// bits 0 .. n-1
__device__ inline unsigned long long low_bits(int n) {
  return n >= 64 ? ~0ull : ((1ull << n) - 1ull);
}

template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* lds) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  constexpr int NW = kBlock / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[k * NW + w] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < NW; ++j) acc += lds[k * NW + j];
    v[k] = acc;
  }
  __syncthreads();
}

// Element load/store with a 32-bit element index: the byte offset is formed in 32 bits
// and added to the (wave-uniform) base, which lets the compiler use the scalar-base plus
// 32-bit vector-offset addressing form instead of 64-bit vector address arithmetic.
// Valid for arrays below 4 GiB.
template <typename T>
__device__ inline T ld(const T* base, uint32_t i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * uint32_t(sizeof(T)));
}
template <typename T>
__device__ inline void st(T* base, uint32_t i, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * uint32_t(sizeof(T))) = v;
}

// j / d for 0 <= j < 2^22, 1 <= d <= 2^11, via a float reciprocal with exact fix-up.
__device__ inline int div_small(int j, int d, float inv) {
  int q = static_cast<int>(static_cast<float>(j) * inv);
  if ((q + 1) * d <= j) ++q;
  if (q * d > j) --q;
  return q;
}

}  // namespace psl

// host-side helpers implemented in psl_setup.hip: device memory from the stream-ordered
// pool, ordered on psl_alloc_stream (set by each entry point to the caller's stream)
extern thread_local hipStream_t psl_alloc_stream;
int psl_internal_alloc(void** p, size_t bytes);
void psl_internal_free(void* p);
// bytes from the context's arena (256-byte aligned); a new block when the current one is
// exhausted (at least `reserve` bytes)
int psl_ctx_alloc(psl_ctx* c, void** p, size_t bytes, size_t reserve = size_t(32) << 20);
// pinned host blocks (<= 1024 bytes), recycled across contexts
void* psl_internal_pinned_get(size_t bytes);
void psl_internal_pinned_put(void* p);
// per-device non-blocking stream used only to capture graphs (created once, kept)
hipStream_t psl_internal_capture_stream();
