/*
 * psl.h -- C-ABI of libpsl: the subdomain-levelset (PSL) deflated preconditioned
 * conjugate gradient solve of the heterogeneous pressure equation on AMD gfx950.
 *
 * Method: arXiv 1510.02148, "The parallel subdomain-levelset deflation method in
 * reservoir simulation". The problem is A x = b (Section 2, eq. "coupledsys" restricted
 * to the reservoir block) for the finite-volume pressure equation -div(K grad p) = q
 * (Section 2, eq. "pressure"); Z holds one indicator vector per (subdomain, levelset)
 * region (Section 3.2, eq. "domdefl" and the subdomain-levelset construction);
 * E = Z^T A Z (Definition 3.1, eq. "E"); the deflated system P1 A xhat = P1 b
 * (eq. "defsys") is solved and mapped back by x = Z E^-1 Z^T b + P2 xhat
 * (eq. "projectback"). Z, E and its factorisation are built once and reused by every
 * solve (Section 3.2: the operators are formed before the iteration starts and stay
 * constant while the permeability is fixed).
 *
 * Conventions shared by every entry point:
 *   - Grid: nx x ny x nz unit cells, cell c = ix + nx*(iy + ny*iz); nz == 1 is a 2D
 *     5-point problem. All cell arrays are length n = nx*ny*nz, contiguous.
 *   - Face arrays (float64): Tx[(nx+1)*ny*nz] with face index ix + (nx+1)*(iy + ny*iz)
 *     (face ix lies between cells ix-1 and ix); Ty[nx*(ny+1)*nz] with index
 *     ix + nx*(iy + (ny+1)*iz); Tz[nx*ny*(nz+1)] with index ix + nx*(iy + ny*iz).
 *     (A p)_c = sum over the six faces f of c of T_f (p_c - p_nbr), with p_nbr = 0
 *     across an outer face: an outer face with T_f > 0 is a p = 0 Dirichlet face,
 *     T_f = 0 is a no-flow face.
 *   - Pointers documented "dev" are device pointers on the current HIP device;
 *     "host" pointers are host memory. The caller owns every array it passes and the
 *     library never frees caller memory. Arrays are only read unless marked "out".
 *   - Every device operation is enqueued on `stream` (a hipStream_t; NULL = the null
 *     stream). Calls that return host results (d, psl_stats) synchronise that stream.
 *   - Return value: PSL_OK (0) or a negative PSL_E* code. No exception crosses the ABI.
 *     psl_status_str() names a code. A psl_ctx must not be used by two threads at once.
 */
#ifndef PSL_H
#define PSL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------- */
#define PSL_OK            0
#define PSL_EINVAL       -1  /* bad argument: null pointer, size out of range, ... */
#define PSL_ENOMEM       -2  /* device allocation failed */
#define PSL_EHIP         -3  /* a HIP runtime call failed */
#define PSL_ENOTSPD      -4  /* E (or diag(A)) not positive definite: Cholesky failed */
#define PSL_EMAXIT       -5  /* iteration cap reached; x holds the projected last iterate */
#define PSL_EBREAKDOWN   -6  /* (p, P1 A p) <= 0 inside CG */
#define PSL_ENONFINITE   -7  /* NaN/Inf in b, x0 or an iterate */
#define PSL_ESTAGNATION  -8  /* refinement stopped reducing the FP64 residual */
#define PSL_ENOTSUP      -9  /* valid request the library does not support (limit given) */

/* ---- Dirichlet face mask for psl_assemble_tpfa ----------------------------------- */
#define PSL_DIRICHLET_X_LO  1u
#define PSL_DIRICHLET_X_HI  2u
#define PSL_DIRICHLET_Y_LO  4u
#define PSL_DIRICHLET_Y_HI  8u
#define PSL_DIRICHLET_Z_LO 16u
#define PSL_DIRICHLET_Z_HI 32u

/* ---- solve modes ------------------------------------------------------------------- */
#define PSL_FP64   0  /* CG vectors and stencil in float64 */
#define PSL_MIXED  1  /* CG vectors and stencil in float32 inside float64 refinement */

/* Limits of the library. */
#define PSL_MAX_THRESHOLDS   15     /* levelset thresholds per call (classes <= 16) */
#define PSL_MAX_DENSE_D      8192   /* coarse dimension d (E and E^-1 are held dense) */
#define PSL_MAX_TILE_LABELS  16     /* distinct labels inside one work tile */
#define PSL_MAX_CELLS   536870911   /* 2^29 - 1: cells of a grid, and entries of each of its
                                       face arrays; larger grids give PSL_ENOTSUP */

typedef struct { int32_t nx, ny, nz; } psl_grid;

typedef struct psl_ctx psl_ctx;  /* opaque: owns its copies of T, labels, E, E^-1, work */

typedef struct {
  double  tol;          /* stop when ||b - A x||_2 <= tol * ||b||_2 (default 1e-8) */
  int32_t maxit;        /* cap on CG iterations over all refinement steps (default 10000) */
  int32_t mode;         /* PSL_FP64 or PSL_MIXED */
  int32_t use_x0;       /* 1: x holds the start vector on entry; 0: start from x = 0 */
  int32_t max_outer;    /* cap on refinement steps (default 30) */
  double  tau_inner;    /* PSL_MIXED: reduction of the float32 CG residual after which it
                           is replaced by the float64 residual (default 0.01); PSL_FP64
                           ignores it */
  int32_t check_every;  /* CG iterations enqueued between host convergence checks
                           (default 16; iterations after convergence are skipped on device) */
  int32_t reproject;    /* PSL_FP64: re-apply P1 to the CG residual every iteration, fused
                           into the update pass (keeps Z^T rhat = 0 under rounding): 1 on,
                           0 or -1 (default) off. PSL_MIXED ignores it (its residual is
                           replaced by the projected float64 residual instead) */
  double  mixed_floor;  /* PSL_MIXED: once ||b - A x|| <= mixed_floor ||b||, float64 CG
                           continues along the float32 search direction (default 1e-7;
                           0 keeps float32 until it stalls; float32 also hands over as
                           soon as its float64 residual detaches from its own) */
} psl_solve_opts;

typedef struct {
  int32_t iters;        /* CG iterations (products with A inside inner loops) */
  int32_t outer;        /* refinement steps taken (FP64 residual evaluations - 1) */
  int32_t status;       /* same value the call returned */
  int32_t fell_back;    /* PSL_MIXED only: 1 if float32 stagnated and float64 finished */
  double  relres_true;  /* ||b - A x||_2 / ||b||_2 in float64 from a fresh product */
  double  bnorm;        /* ||b||_2 */
  double  t_solve_s;    /* wall time of the call (host clock, stream synchronised) */
  double  zt_r_drift;   /* ||Z^T r||_2 / ||r||_2 for the returned x, r = b - A x: the
                           deflation invariant Z^T P1 = 0 (Section 3.1) under rounding
                           (0 when r = 0); psl_solve only, other solvers leave 0 */
} psl_solve_stats;

/* Fill `o` with the defaults listed above. */
void psl_default_opts(psl_solve_opts* o);

/* Options of psl_solve_gmres. */
typedef struct {
  double  tol;          /* stop when ||b - A x||_2 <= tol * ||b||_2 (default 1e-8) */
  int32_t maxit;        /* cap on Arnoldi steps over all cycles (default 10000) */
  int32_t restart;      /* m of GMRES(m): steps per cycle, 1..200 (default 30) */
  int32_t use_x0;       /* 1: x holds the start vector on entry; 0: start from x = 0 */
  int32_t degree;       /* preconditioner: 0 or 1 M = diag(A) (default 0); 2..16 the
                           Chebyshev polynomial of psl_solve_poly with that many steps on
                           [2/30, 2] (a stronger preconditioner on the deflated system) */
  int32_t reserved[2];  /* must be 0 */
} psl_gmres_opts;

/* Fill `o` with the GMRES defaults. */
void psl_default_gmres_opts(psl_gmres_opts* o);

/*
 * psl_solve_gmres -- the paper's own solver (Algorithm 1 with the subdomain-levelset
 * vectors formed a priori, Section 3.2): right-preconditioned restarted GMRES(m) on
 * P1 A M^-1 y = P1 b, M = diag(A), x_hat = M^-1 y, and at convergence the projection back
 * x = P2 x_hat + Z E^-1 Z^T b. Float64 throughout. Arnoldi runs classical Gram-Schmidt
 * twice (the paper writes modified Gram-Schmidt; both span the same Krylov space, and
 * the repeated classical form needs two batched passes per step instead of j dependent
 * ones). The least-squares residual decides convergence inside a cycle; every cycle
 * starts from a freshly formed P1 (b - A x). The host reads one column of the Hessenberg
 * matrix per step. With degree >= 2, M^-1 is the Chebyshev polynomial preconditioner
 * (as in psl_solve_poly), applied to every basis vector and to the cycle's update.
 *   ctx, b, x, st, stream  as for psl_solve; st->iters = Arnoldi steps, st->outer =
 *   completed cycles. Work space: (m + 1) n doubles for the basis, kept on the context
 *   (and psl_solve_poly's 5 n with degree >= 2).
 * Returns PSL_OK, PSL_EMAXIT (x = the projected last iterate), PSL_ENONFINITE,
 * PSL_EINVAL (options out of range), PSL_ENOMEM.
 */
int psl_solve_gmres(psl_ctx* ctx, const double* b, double* x, const psl_gmres_opts* o,
                    psl_solve_stats* st, void* stream);

/* Options of psl_solve_poly. */
typedef struct {
  double  tol;          /* stop when ||P1 (b - A x_hat)||_2 <= tol * ||b||_2 (default 1e-8) */
  double  ratio;        /* Chebyshev interval [lmax / ratio, lmax], ratio > 1 (default 30) */
  double  lmax;         /* upper end; 2 bounds the spectrum of D^-1 A for every matrix
                           psl_assemble_tpfa produces (Gershgorin) (default 2) */
  int32_t degree;       /* Chebyshev steps per application, 1..16; 1 is Jacobi (default 3) */
  int32_t maxit;        /* CG iteration cap (default 10000) */
  int32_t use_x0;       /* 1: x holds the start vector on entry; 0: start from x = 0 */
  int32_t check_every;  /* iterations in the first run between host reads, 1..512
                           (default 16; later runs follow the convergence rate) */
  int32_t mixed;        /* 1: float32 CG (float32 T, 1/diag, vectors; float64 partials)
                           inside float64 iterative refinement, each inner solve to 1e-5
                           relative (or what tol still needs); 0: float64 (default) */
  int32_t reserved[1];  /* must be 0 */
} psl_poly_opts;

/* Fill `o` with the polynomial-preconditioner defaults. */
void psl_default_poly_opts(psl_poly_opts* o);

/*
 * psl_solve_poly -- deflated CG with a stronger preconditioner on the deflated system
 * (Section 1 and the SPE10 experiment of Section 4 (Table 5) pair the subdomain-levelset
 * deflation with AMG applied to the deflated system; AMG is not built here). M^-1 = q(D^-1 A) D^-1,
 * D = diag(A): `degree` steps of the Chebyshev semi-iteration for A y = r on the interval
 * [lmax / ratio, lmax], from y = 0 (symmetric positive definite for lmax at or above the
 * spectrum of D^-1 A). The CG is the DEF1 loop of psl_solve (P1 from E = Z^T A Z, eq.
 * "deflops"; projection back, eq. "projectback") in float64, two reductions per
 * iteration; degree 1 gives the iterates of Jacobi-preconditioned DEF1.
 *   ctx, b, x, st, stream  as for psl_solve; st->iters = CG iterations (all inner solves
 *   with mixed = 1), st->outer = 1 (float64) or the refinement steps (mixed).
 *   Work space: 5 n doubles kept on the context (and 7 n floats with mixed = 1).
 * Returns PSL_OK, PSL_EMAXIT (x = the projected last iterate), PSL_ESTAGNATION (||P1 r||
 * not halved within 512 iterations, the rounding floor above tol; x = the projected last
 * iterate), PSL_EBREAKDOWN, PSL_ENONFINITE, PSL_EINVAL (options out of range), PSL_ENOMEM.
 */
int psl_solve_poly(psl_ctx* ctx, const double* b, double* x, const psl_poly_opts* o,
                   psl_solve_stats* st, void* stream);

/*
 * psl_assemble_tpfa -- face transmissibilities of the cell-centred finite-volume
 * discretisation of -div(K grad p) = q (Section 2, eqs. "pressure"/"mobility" with the
 * total mobility taken as the permeability K, single phase).
 *   g              host: grid.
 *   K              dev[n] float64: isotropic cell permeability (>= 0).
 *   dirichlet_mask PSL_DIRICHLET_* bits: outer faces held at p = 0.
 *   Tx, Ty, Tz     dev out, float64, face arrays as described above.
 * Interior face: 2 Ka Kb / (Ka + Kb) (harmonic mean over unit spacing), 0 if Ka+Kb = 0.
 * Dirichlet outer face: 2 K of the adjacent cell (half-cell distance). Other outer
 * faces: 0. Errors: PSL_EINVAL for a non-positive grid size or null pointer,
 * PSL_ENOTSUP for a grid above PSL_MAX_CELLS.
 */
int psl_assemble_tpfa(const psl_grid* g, const double* K, uint32_t dirichlet_mask,
                      double* Tx, double* Ty, double* Tz, void* stream);

/*
 * psl_build_Z -- subdomain-levelset deflation space (Section 3.2: subdomain deflation
 * vectors eq. "domdefl" with a levelset split inside every subdomain, vectors on both
 * the high- and the low-permeability parts).
 *   g        host: grid.
 *   K        dev[n] float64 permeability (ignored when cls != NULL; may then be NULL).
 *   nsub     host[3]: subdomains per axis (1 <= nsub[a] <= extent). Floor partition:
 *            subdomain coordinate along x = floor(ix * nsub[0] / nx), likewise y, z;
 *            subdomain id s = sx + nsub[0] * (sy + nsub[1] * sz).
 *   thr      host[nthr] float64, ascending: class of a cell = #{t : K >= t}.
 *   nthr     0..PSL_MAX_THRESHOLDS.
 *   cls      dev[n] int32 or NULL: manual classes in [0, ncls) (the paper's hand-built
 *            layer indicators); when given, thr/nthr are ignored.
 *   ncls     number of manual classes (1..PSL_MAX_THRESHOLDS+1) when cls != NULL.
 *   labels   dev out [n] int32: column of Z holding the cell, in [0, d).
 *   d        host out: number of deflation vectors.
 * The column of a cell is the rank of key = s * ncls + class among the keys that occur
 * (empty regions get no column, so Z has full rank). Integer result, bit-exact.
 * Errors: PSL_EINVAL (bad sizes, nsub out of range, unsorted thr, a manual class
 * outside [0, ncls); labels is then unspecified), PSL_ENOTSUP (more than PSL_MAX_CELLS
 * cells, or more than 2^26 (subdomain, class) keys).
 */
int psl_build_Z(const psl_grid* g, const double* K, const int32_t nsub[3],
                const double* thr, int32_t nthr, const int32_t* cls, int32_t ncls,
                int32_t* labels, int32_t* d, void* stream);

/*
 * psl_build_Z_noalloc -- psl_build_Z for callers that cannot allocate device memory
 * (code that must not call hipMalloc: graph-building or tight serving loops, harnesses
 * that forbid allocation). Same arguments, labelling, conventions and errors as
 * psl_build_Z; it calls no hipMalloc/hipFree or other allocating routine. Its scratch
 * (key flags and their prefix sum, 2 * PSL_NOALLOC_MAX_KEYS + 2 int32, about 2 MiB) is a
 * fixed device array of the library, one copy per GPU, held until the process ends and
 * shared by every call on that GPU: calls that overlap on one GPU (two host threads, or
 * two streams) race and give undefined labels. Like psl_build_Z it synchronises `stream`
 * to return d. Errors: as psl_build_Z, and PSL_ENOTSUP when nsub[0] nsub[1] nsub[2]
 * times the class count exceeds PSL_NOALLOC_MAX_KEYS (checked before any device work);
 * PSL_EHIP if the scratch address cannot be obtained on the current device.
 */
#define PSL_NOALLOC_MAX_KEYS 262144   /* (subdomain, class) keys psl_build_Z_noalloc takes */
int psl_build_Z_noalloc(const psl_grid* g, const double* K, const int32_t nsub[3],
                        const double* thr, int32_t nthr, const int32_t* cls, int32_t ncls,
                        int32_t* labels, int32_t* d, void* stream);

/*
 * psl_build_Z_cc -- automatic subdomain-levelset construction: like psl_build_Z, but
 * every (subdomain, class) region is split into its face-connected components (cells
 * sharing a face: 6 neighbours in 3D, 4 in 2D), one deflation vector each. Section 3.2
 * draws every region as one connected piece and leaves an automatic construction for
 * later; this is its connected-components reading. Same arguments, conventions and
 * errors as psl_build_Z. The columns are ordered by the smallest cell index
 * (c = ix + nx (iy + ny iz)) of their component. Integer result, bit-exact and
 * independent of thread scheduling. Uses n + 2n/1024 int32 of temporary device memory.
 */
int psl_build_Z_cc(const psl_grid* g, const double* K, const int32_t nsub[3],
                   const double* thr, int32_t nthr, const int32_t* cls, int32_t ncls,
                   int32_t* labels, int32_t* d, void* stream);

/*
 * psl_setup_E -- build the deflation operators once (Definition 3.1): copies of the
 * transmissibilities, diag(A), the interface rows of A Z, E = Z^T A Z assembled in
 * float64 from the faces, its Cholesky factor E = L L^T and E^-1 (float64).
 *   ctx      host out: new context (free with psl_destroy).
 *   g        host: grid.   Tx, Ty, Tz: dev face arrays (copied; caller may free them).
 *   labels   dev[n] int32 in [0, d) (copied; any labelling is accepted, not only the
 *            output of psl_build_Z, but every column must be non-empty).
 *   d        1..PSL_MAX_DENSE_D.
 *   nsub     host[3] or NULL: the subdomain partition used to cut the grid into
 *            work tiles (one subdomain maps to one or more workgroups; the parallel
 *            subdomain-per-processor layout of Section 3.2 moved onto compute units).
 *            NULL lets the library choose boxes of about 16x16x8 cells.
 * Errors: PSL_EINVAL, PSL_ENOMEM, PSL_ENOTSPD (a cell with diag(A) <= 0 or E not SPD),
 * PSL_ENOTSUP (d > PSL_MAX_DENSE_D, or a grid above PSL_MAX_CELLS).
 */
int psl_setup_E(psl_ctx** ctx, const psl_grid* g, const double* Tx, const double* Ty,
                const double* Tz, const int32_t* labels, int32_t d, const int32_t nsub[3],
                void* stream);

/* Options of psl_setup_E_ex. */
typedef struct {
  int32_t tile_cells;   /* cells per work tile, 64..2048 (one workgroup each; tiles never
                           straddle a subdomain); 0 = the library's choice (1024, halved
                           down to 256 while the grid would give fewer than 2048 tiles) */
  int32_t finish_kernels; /* 1: every CG iteration takes its step decisions (inner products
                           summed from the workgroup partials, stop test, step coefficients)
                           in small one-workgroup kernels, so the pass kernels only read
                           them and the update pass runs one workgroup per tile; -1: each
                           pass workgroup sums the partials itself; 0 (default): 1 for
                           grids of 2^21 cells or more, -1 below (where the extra launches
                           cost more than the repeated sums) */
  int32_t coarse_sym;   /* coarse product e = E^-1 s: 1 reads only the lower 64 x 64 block
                           triangle of the symmetric E^-1 (Def. 3.1: E and so E^-1 are
                           symmetric), half the bytes of the dense product, and adds the
                           block shares in a second launch; -1 the dense row-wise product;
                           0 (default): 1 for d >= 1024, -1 below */
  int32_t stencil_split; /* float32 (two-reduction) CG with finish kernels: 0 (default) or
                           1 forms the new direction p = u + beta p_prev in a pass of its
                           own and then q = A p in the plain stencil pass (bit-identical
                           results, each neighbour loaded once); -1 keeps the fused pass
                           that recomputes the neighbours' p. No effect without finish
                           kernels */
  int32_t face_tables;  /* float32 update: 0 (default) or 1 gives every tile a table of the
                           coarse labels its cut faces reference (at most 126) and packs each
                           face into one word of local indices, so a workgroup gathers the
                           tile's few coarse values once, early, instead of one per face
                           (bit-identical results); -1 keeps the unpacked faces. A tile
                           with more labels than the table holds keeps them too */
  int32_t wide_tiles;   /* 0 (default) or 1: where a subdomain box is under 32 cells wide in
                           x, each tile spans two x-adjacent boxes, so the rows the passes
                           read are at least 128 bytes of float32 (whole cache lines) instead
                           of half lines; tiles then hold the labels of two boxes (a tiling
                           whose tiles exceed 16 labels falls back to one box per tile
                           before tiles shrink). -1: tiles inside one box. Results equal to
                           rounding (the partial sums group cells differently) */
  int32_t reserved[2];  /* must be 0 */
} psl_setup_opts;

/* Fill `o` with the defaults (all zero). */
void psl_default_setup_opts(psl_setup_opts* o);

/*
 * psl_setup_E_ex -- psl_setup_E with options (NULL = defaults; psl_setup_E passes NULL).
 * The tile size trades workgroup count against per-workgroup work; the tile autotuner
 * (paper_1510_02148_amd/autotune.py) picks it per shape class by timing solves.
 * Errors: as psl_setup_E, and PSL_EINVAL for tile_cells outside 64..2048 (0 allowed).
 */
int psl_setup_E_ex(psl_ctx** ctx, const psl_grid* g, const double* Tx, const double* Ty,
                   const double* Tz, const int32_t* labels, int32_t d, const int32_t nsub[3],
                   const psl_setup_opts* o, void* stream);

/*
 * psl_solve -- solve A x = b (eq. "coupledsys", reservoir block) with Jacobi-
 * preconditioned CG on the deflated system P1 A xhat = P1 b (eqs. "deflops", "defsys";
 * E built from A itself, Remark 3.1) and the projection back x = Z E^-1 Z^T b + P2 xhat
 * (eq. "projectback"), inside a float64 refinement loop: r = b - A x;
 * x += Z E^-1 Z^T r; r = P1 r; stop if ||r|| <= tol ||b||; else CG on the scaled r and
 * x += ||r|| xhat.
 * PSL_FP64: float64 CG (single-reduction recurrences) straight to the tolerance.
 * PSL_MIXED: float32 CG (two-reduction loop) whose recursive residual is replaced by the
 * projected float64 residual each time it has dropped by tau_inner, keeping the search
 * direction; below mixed_floor, or once the float64 residual stops following the float32
 * one (float32's attainable accuracy), float64 CG takes over (stats.fell_back = 1), along
 * the float32 direction when the last float32 run ended normally.
 *   ctx   context from psl_setup_E.
 *   b     dev[n] float64 right-hand side (not modified).
 *   x     dev[n] float64: start vector on entry if o->use_x0, solution on exit.
 *   o     host options (NULL = defaults).
 *   st    host out statistics (may be NULL).
 * An inner CG that stops improving (rounding floor: (p, P1 A p) <= 0, or no halving of
 * ||rhat|| over 512 iterations) returns to the refinement loop, which restarts it from
 * the new float64 residual; in PSL_MIXED a refinement step that does not halve the
 * float64 residual also switches the remaining steps to float64 CG.
 * A fresh float64 run of the single-reduction loop that fails to reduce the residual by
 * 10 % sends the solve back to its best iterate, to finish with the two-reduction loop
 * and residual replacement; a second such failure ends it.
 * Returns PSL_OK when ||b - A x|| <= tol ||b|| was reached; otherwise PSL_EMAXIT
 * (iteration or refinement cap; x is the projected last iterate), PSL_ESTAGNATION
 * (float64 refinement stopped reducing the residual), PSL_EBREAKDOWN (breakdown on the
 * first iteration of a refinement step) or PSL_ENONFINITE; after these three x is the
 * projected iterate with the smallest residual seen.
 * ||b|| = 0 gives x = 0, PSL_OK.
 */
int psl_solve(psl_ctx* ctx, const double* b, double* x, const psl_solve_opts* o,
              psl_solve_stats* st, void* stream);

/*
 * psl_solve_batched -- solve nsys independent systems A_i x_i = b_i, each set up by its
 * own psl_setup_E, together: every float64 CG launch covers the work tiles of all systems
 * through a (system, tile) work list, while each system keeps its own scalars, tolerance
 * test and stop flag (a converged system's workgroups return at once). In PSL_FP64 the
 * per-system arithmetic is that of psl_solve in PSL_FP64, so each x_i is the one psl_solve
 * returns for that system alone. In PSL_MIXED the systems first take float32 refinement
 * steps together: each step is a fresh float32 two-reduction DEF1-PCG on the projected
 * float64 residual (every pass one launch for all systems, the step decisions of each
 * system in small per-system kernels) until that residual has dropped by tau_inner,
 * followed by x += ||r|| xhat and the float64 refinement step; a system leaves this phase
 * when it converges, reaches mixed_floor, or a step fails to halve its float64 residual,
 * and the float64 batched loop finishes it (st[i].fell_back = 1). This schedule restarts
 * the float32 direction at every step, unlike psl_solve's PSL_MIXED, so its iterates are
 * its own (each x_i meets the same tolerance). The launch plan (argument table, work
 * lists, captured graph of iteration chunks) is cached on ctxs[0] while the same contexts
 * are passed in the same order.
 *   ctxs  host[nsys]: distinct contexts on the current device.
 *   b, x  host[nsys] arrays of device pointers, each dev[n_i] float64 (as in psl_solve).
 *   o     options as in psl_solve (NULL = defaults); use_x0 applies to every system.
 *   st    host out[nsys] statistics (may be NULL); st[i].status is system i's result.
 * A system that stalls or breaks down is finished by psl_solve from its current x.
 * Returns PSL_OK if every system converged, otherwise the first failing system's code.
 * Errors: PSL_EINVAL (null pointers, nsys < 1, a context twice, another device, options
 * out of range), PSL_ENOTSUP (a context whose coarse solve needs the separate label
 * reduction: d > 4096 or very many label partials).
 */
int psl_solve_batched(psl_ctx* const* ctxs, int32_t nsys, const double* const* b,
                      double* const* x, const psl_solve_opts* o, psl_solve_stats* st,
                      void* stream);

/*
 * psl_apply_A -- q = A p in float64 (the stencil product used by every solve; the
 * matrix-vector product of Algorithm 1). p, q: dev[n] float64, distinct arrays.
 */
int psl_apply_A(psl_ctx* ctx, const double* p, double* q, void* stream);

/*
 * psl_deflate -- apply the deflation operators to one vector (eq. "deflops"):
 *   c = E^-1 Z^T r (host-independent, dev[d] out, may be NULL),
 *   out = P1 r = r - A Z c (dev[n] out, may alias r).
 * Used to check the coarse solve and the projector; r: dev[n] float64.
 */
int psl_deflate(psl_ctx* ctx, const double* r, double* out, double* c, void* stream);

/*
 * psl_get_coarse -- copy E (float64, d x d, row-major) and/or E^-1 into caller device
 * memory (either pointer may be NULL). d is returned in *d when d != NULL.
 */
int psl_get_coarse(psl_ctx* ctx, double* E, double* Einv, int32_t* d, void* stream);

/* ---- measurement entry points (used by the benchmark and the profiler runs) ------- */
#define PSL_KERNEL_STENCIL        0  /* v = A M^-1 r and the CG inner products (pass 1) */
#define PSL_KERNEL_COARSE         1  /* e = E^-1 Z^T v (coarse GEMV) and scalar slices    */
#define PSL_KERNEL_UPDATE         2  /* p, q, x, r updates with A Z e   (pass 2)          */
#define PSL_KERNEL_DIRECTION      3  /* the direction pass p = u + beta p_prev of the split
                                        float32 stencil step (finish kernels on);
                                        psl_profile_kernel only (elsewhere the direction
                                        update is part of another pass) */
#define PSL_KERNEL_OUTER_RESIDUAL 4  /* r = b - A x in float64          (refinement step) */
#define PSL_KERNEL_GMRES_PASS     5  /* deflated GMRES: w -= V h with the dots V^T w (fused
                                        Gram-Schmidt pass over min(m, 32) basis vectors,
                                        float64; needs a prior psl_solve_gmres, PSL_FP64) */
#define PSL_KERNEL_POLY_STEP      6  /* psl_solve_poly: the last Chebyshev step of a degree >= 3
                                        preconditioner application (stencil on y with the
                                        d, y updates and the (r, y), (r, r) partials; needs a
                                        prior psl_solve_poly; PSL_MIXED times the float32
                                        step after a mixed solve) */
#define PSL_KERNEL_SMALL_SOLVE    7  /* the one-workgroup float64 inner solve of small grids
                                        (psl_ctx_info.small_solve; one launch per inner
                                        solve); psl_profile_kernel only, PSL_FP64 */

/*
 * psl_bench_kernel -- enqueue `reps` back-to-back launches of one kernel of the CG
 * iteration (Algorithm 1's matrix-vector product, inner products and Galerkin solve, in
 * the deflated-CG form psl_solve uses) on the context's current work vectors, in the
 * precision of `mode`, so a caller can time it with events on `stream`. Call after a
 * psl_solve in the same mode (the vectors then hold a real iterate); the scalars are set
 * so that no launch exits early. The work vectors are overwritten.
 * PSL_KERNEL_GMRES_PASS times the Gram-Schmidt pass of psl_solve_gmres (Algorithm 1's
 * Arnoldi step) against the first min(m, 32) basis vectors of the longest restart length m
 * solved on this context so far; it overwrites basis vector min(m, 32).
 * PSL_KERNEL_POLY_STEP times the last Chebyshev step of psl_solve_poly's preconditioner
 * (degree >= 3) on its work vectors and overwrites them.
 * Errors: PSL_EINVAL (bad or reserved kernel id, mode or reps < 1; GMRES pass without a
 * prior psl_solve_gmres or in PSL_MIXED; Chebyshev step without a prior psl_solve_poly in
 * that precision), PSL_ENOMEM.
 */
int psl_bench_kernel(psl_ctx* ctx, int32_t kernel, int32_t mode, int32_t reps, void* stream);

/*
 * psl_profile_kernel -- time one kernel of the CG iteration inside the following psl_solve
 * calls on this context: an event is recorded on the solve's stream before and after each
 * launch of `kernel` (PSL_KERNEL_STENCIL, PSL_KERNEL_DIRECTION (the split float32 stencil
 * step's direction pass), PSL_KERNEL_COARSE (the label sum and the coarse product
 * together), PSL_KERNEL_UPDATE, or PSL_KERNEL_SMALL_SOLVE with PSL_FP64) in the precision
 * of `mode` (PSL_MIXED: the float32 launches of a mixed solve), for up to `max_launches`
 * launches (1 .. 2^20) counted from this call. While the first three are armed, the solves
 * launch their iterations directly with three or more launches per iteration (no replayed
 * graphs, no one-workgroup solve), so every launch is the solve's own; launches enqueued
 * past convergence return at once and show as short durations. kernel < 0 disarms. The
 * events are created here and kept by the context. Errors: PSL_EINVAL, PSL_ENOMEM, PSL_EHIP.
 */
int psl_profile_kernel(psl_ctx* ctx, int32_t kernel, int32_t mode, int32_t max_launches);

/*
 * psl_profile_read -- synchronise `stream` and return the number of launches timed since
 * psl_profile_kernel (or the last read) in *count and the first min(count, max) durations
 * in microseconds (host out, launch order) in durations_us; then restart the count.
 * Errors: PSL_EINVAL, PSL_EHIP.
 */
int psl_profile_read(psl_ctx* ctx, int32_t* count, float* durations_us, int32_t max,
                     void* stream);

/*
 * psl_bench_copy -- device-to-device streaming copy of `bytes` (multiple of 16, both
 * pointers 16-byte aligned) with a plain load/store kernel, one 16-byte load and store per
 * thread: the reference for achievable bandwidth and for calibrating hardware byte
 * counters. Errors: PSL_EINVAL (null or misaligned pointer, bad size).
 */
int psl_bench_copy(const void* src, void* dst, int64_t bytes, void* stream);

/* Sizes of what psl_setup_E built (for byte accounting and diagnostics). */
typedef struct {
  int64_t n;            /* cells */
  int32_t d;            /* deflation vectors */
  int32_t ntiles;       /* work tiles (one workgroup each) */
  int64_t m_faces;      /* cut faces stored for A Z (faces between labels + Dirichlet) */
  int32_t nslot_max;    /* most distinct labels in one tile */
  int32_t coarse_sym;   /* 1: the coarse product reads the lower block triangle of E^-1
                           (psl_setup_opts.coarse_sym), 0: the dense product */
  int32_t small_solve;  /* 1: float64 inner solves run in one workgroup (n <= 4096 cells,
                           d <= 32) */
  int32_t face_tables;  /* 1: the float32 update reads packed faces and per-tile coarse
                           tables (psl_setup_opts.face_tables) */
  int32_t wide_tiles;   /* 1: tiles span two x-adjacent subdomain boxes
                           (psl_setup_opts.wide_tiles) */
} psl_ctx_info;

int psl_get_info(const psl_ctx* ctx, psl_ctx_info* info);

/* Release everything the context owns. NULL is ignored. */
void psl_destroy(psl_ctx* ctx);

/* Static string naming a status code. */
const char* psl_status_str(int status);

#ifdef __cplusplus
}
#endif
#endif /* PSL_H */
