/*
 * h2ulv.h -- C-ABI of the MI355X H^2-ULV dense direct solver.
 *
 * The method is the H^2-matrix ULV factorization without trailing sub-matrix
 * dependencies of Ma, Deshmukh and Yokota (arXiv 2208.10907):
 *   - a binary cluster tree over the points with strong admissibility
 *     (Sec. I; Sec. III-D), dense blocks only for inadmissible pairs (Sec. II-D);
 *   - fill-ins pre-computed per block row from one LU per diagonal block and one
 *     triangular solve per dense block (Sec. III-B);
 *   - one shared basis per box from the concatenated fill-in and low-rank
 *     blocks (Sec. III-C, Eq. fillu/fillv), skeleton/redundant split (Sec. II-A);
 *   - the USV rotation of every block (Sec. II-B, Eq. rs and Eq. ss), LU of the
 *     redundant-redundant diagonal block, triangular solves and the Schur
 *     update of the skeleton block (Sec. II-B, Eq. lu and following), all boxes
 *     of a level independent of each other;
 *   - merge of the skeleton blocks into the parent level (Sec. II-C) and a
 *     dense LU at the root (Eq. BLR2final);
 *   - the three-step solve L z = U^T b, U y = z, x = V^T y (Sec. II-B).
 *
 * Conventions shared by every call:
 *   - Pointers documented as "device" point to memory on the GPU that is current
 *     when the call is made; "host" pointers are ordinary CPU memory.
 *   - All vectors/matrices are float64 and column-major; vector entries are in
 *     the caller's original point order (the tree permutation is internal).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *     ordered on that stream.  Calls that return host values synchronise it.
 *   - No exception crosses the ABI.  Every call returns an h2ulv_status;
 *     h2ulv_last_error() gives a thread-local message for the last failure.
 *   - Argument errors are detected before any device work is issued.
 *   - A factor is used by one stream at a time; distinct factors are
 *     independent.  The factor owns all of its device memory.
 */
#ifndef H2ULV_H
#define H2ULV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  H2ULV_OK = 0,
  H2ULV_ERR_INVALID_ARG = -1,      /* bad size, pointer, parameter or NaN input */
  H2ULV_ERR_OOM = -2,              /* device or host allocation failed */
  H2ULV_ERR_HIP = -3,              /* a HIP runtime call failed */
  H2ULV_ERR_SINGULAR = -4,         /* zero or non-finite pivot in a block LU */
  H2ULV_ERR_DUPLICATE_POINTS = -5, /* two distinct points coincide (r = 0) */
  H2ULV_ERR_NOT_CONVERGED = -6,    /* refinement did not reach the tolerance */
  H2ULV_ERR_RANK_CHECK = -7        /* a predicted-rank basis failed its randomized
                                      check and params.sketch_fallback is 0 */
} h2ulv_status;

enum { H2ULV_LAPLACE = 0, H2ULV_YUKAWA = 1, H2ULV_ADVECTION = 2 };
enum { H2ULV_FP64 = 0, H2ULV_MIXED = 1 };

/*
 * Problem and accuracy parameters (the paper's problem statement: points and a
 * kernel, Sec. IV and V; admissibility, Sec. I; leaf size, Sec. IV-C; rank /
 * tolerance of the shared bases, Sec. II-A).
 */
typedef struct h2ulv_params {
  int32_t struct_size; /* sizeof(h2ulv_params); set by h2ulv_params_default */
  int32_t kernel;      /* H2ULV_LAPLACE: 1/r; H2ULV_YUKAWA: exp(-alpha r)/r;
                          H2ULV_ADVECTION: exp(b.(x_i - x_j) - alpha r)/r with
                          b = drift, the steady advection-diffusion Green's
                          function (not symmetric for b != 0)                   */
  double alpha;        /* Yukawa decay constant                                 */
  double diag;         /* A_ii                                                  */
  double eta;          /* admissible iff |c_i - c_j| > eta (r_i + r_j); >= 0    */
  int32_t leaf_size;   /* max points per leaf; >= 2                             */
  int32_t rank_cap;    /* 0 = no cap, else k <= rank_cap                        */
  double tol;          /* basis tolerance: keep pivots with |R_tt| > tol |R_00| */
  int32_t far_sample;  /* 0 = exact far field; s > 0 = s samples per ancestor
                          far box (own-level far boxes use all candidate rows) */
  int32_t precision;   /* H2ULV_FP64 or H2ULV_MIXED (fp32 products, fp64 QR/LU) */
  int32_t verbose;     /* 0 = silent; 1 = per-level timing on stderr            */
  int32_t oversample;  /* learned ranks: sketch columns beyond 1.25 k-hat; >= 0 */
  const struct h2ulv_rankmodel* rank_model; /* NULL: every basis from the full
                          column-pivoted QR.  Else the model's predicted rank
                          k-hat of each box sizes a Gaussian sketch of M' whose
                          row ID replaces the full one when a randomized probe
                          accepts it (see h2ulv_rankmodel_create)              */
  uint64_t sketch_seed; /* key of the Gaussian sketch matrices                 */
  int32_t fill_in;      /* 1 (default): shared bases from [F_i+ A_i+], the
                          fill-ins included (Sec. III-C Eq. fillu).  0: ablation,
                          bases from the low-rank blocks A_i+ alone (F = 0), as
                          without the pre-computed fill-ins of Sec. III-B; not
                          combinable with a rank model                          */
  int32_t partition;    /* cluster tree: 0 (default) k-d split at the median of
                          the widest bounding-box axis; 1 balanced 2-means
                          bisection (the k-means partition of Sec. V: every
                          box splits into two clusters of floor(n/2) and
                          ceil(n/2) points, so leaves stay a power of two)      */
  int32_t structure;    /* 0 (default): the H^2 hierarchy, skeletons merged level
                          by level into the parent (Sec. III).  1: flat BLR^2
                          (Sec. II-B): the leaves are the only level, every
                          leaf pair is classified by the admissibility rule,
                          and after the leaf sweep all skeletons form one dense
                          root block (Eq. BLR2final); levels above the leaves
                          hold nothing (their accessors return INVALID_ARG)    */
  int32_t bases;        /* 0 (default): one shared basis per box (V = U) for the
                          symmetric kernels, separate row and column bases for
                          H2ULV_ADVECTION.  1: separate bases for any kernel.
                          Separate bases (Sec. III-C: U from [F_i+ A_i+], V from
                          [F_+j^T A_+j^T], Eq. fillu/fillv) need structure 0,
                          precision FP64 and no rank model                     */
  int32_t sketch_fallback; /* rank model only.  1 (default): a box whose sketched
                          row ID fails the randomized check (at its first width
                          and, when that was narrower than m - 8, again at the
                          full width m - 8) takes the full column-pivoted QR.
                          0: the factorization stops with H2ULV_ERR_RANK_CHECK
                          instead (for callers that want to know when the model
                          under-predicts)                                      */
  int32_t sketch_min_level; /* rank model only: the levels above this one (level
                          l < sketch_min_level, the root's children at l = 1)
                          take the full column-pivoted QR; the others use the
                          predicted-rank sketches.  0 (default): every level.
                          The few boxes of the top levels cost little in full,
                          and their bases decide much of the preconditioner's
                          quality                                             */
  double drift[3];      /* b of H2ULV_ADVECTION (ignored by the other kernels)  */
} h2ulv_params;

typedef struct h2ulv_factor h2ulv_factor; /* opaque */
typedef struct h2ulv_rankmodel h2ulv_rankmodel; /* opaque */

/* Per-factor statistics (host).  Flops are the algorithmic count of the
 * paper's steps from the actual ranks (LU 2/3 n^3, GEMM 2mnk, QR 2mn^2-2/3n^3),
 * not the instructions the GPU issued. */
typedef struct h2ulv_stats {
  int32_t levels;          /* L: leaves are at level L, root at 0          */
  int32_t max_rank;        /* max k over all boxes and levels              */
  int32_t root_size;       /* size of the dense root block                 */
  int32_t reserved;
  int64_t n;               /* number of points                             */
  double flops_fill;       /* fill-in LU, solves and products              */
  double flops_basis;      /* QR / ID / orthogonal complement              */
  double flops_couple;     /* low-rank couplings T K T^T                   */
  double flops_rotate;     /* U^T D U                                      */
  double flops_elim;       /* RR LU, triangular solves, Schur update       */
  double flops_root;       /* root LU                                      */
  double kernel_evals;     /* kernel entries generated                     */
  double time_setup_s;     /* host tree/list construction                  */
  double time_factor_s;    /* wall time of h2ulv_factorize                 */
  double device_bytes;     /* peak device memory held by the factor        */
  double logabsdet;        /* log|det A~| = sum log|diag U^RR| + log|det D_root| */
} h2ulv_stats;

/* Fill *p with the defaults: Laplace, diag 1e3, eta 1, leaf 256, tol 1e-8, no
 * cap, far_sample 32, FP64, no rank model (oversample 8, sketch_seed 0).
 * Returns INVALID_ARG if p is NULL. */
h2ulv_status h2ulv_params_default(h2ulv_params* p);

/*
 * Device memory from the caller (the torch caching allocator from Python, a
 * memory pool, ...).  alloc returns `bytes` bytes of device memory usable by work
 * on `stream`, or NULL when it has none (the call then fails with OOM); free takes
 * back a block from alloc.  free may be called while work queued on `stream`
 * still reads the block: the allocator must not hand it to work on other
 * streams before that work is done (stream-ordered reuse, as hipFreeAsync and
 * torch's caching allocator give).  The struct is copied; ctx and the two
 * functions must stay valid until every factor made with them is destroyed.
 */
typedef struct h2ulv_allocator {
  void* ctx;
  void* (*alloc)(void* ctx, size_t bytes, void* stream);
  void (*free)(void* ctx, void* ptr, void* stream);
} h2ulv_allocator;

/*
 * Factorize A = [K(x_i, x_j)] (A_ii = diag) for n points.
 *   pts     device, n x 3 row-major (x0 y0 z0 x1 ...); read only; caller owns.
 *   n       number of points, >= 1.
 *   params  host; copied.
 *   alloc   host, may be NULL: where all device memory of the call and of the
 *           factor comes from (the factor keeps its blocks until
 *           h2ulv_destroy; later calls on the factor draw their temporaries
 *           from it too).  NULL: the library's own caching allocator.
 *   stream  hipStream_t.
 *   out     host; receives a new factor (free with h2ulv_destroy).
 * The call copies the points to the host to build the cluster tree and the
 * near/far lists (Sec. III-D), then runs every level of the sweep on the GPU.
 * It synchronises the stream once per level to read back the ranks.
 * Errors: INVALID_ARG (n < 1, NULL pointer, bad params, non-finite point, an
 * allocator with a NULL function), DUPLICATE_POINTS, SINGULAR, OOM (also when
 * the allocator returns NULL: the first device allocation precedes every
 * launch), RANK_CHECK (a rank model with sketch_fallback 0 and a sketch that
 * failed its check), HIP.  On error *out is NULL.
 */
h2ulv_status h2ulv_factorize(const double* pts, int64_t n, const h2ulv_params* params,
                             const h2ulv_allocator* alloc, void* stream, h2ulv_factor** out);

/*
 * Factorize several independent problems with one launch per kernel and level:
 * levels are aligned by height above the leaves, so the boxes of every problem
 * at the same height share the same batched launches (the box independence of
 * Sec. II-B / III-D, extended across problems).
 *   nprob   number of problems, >= 1.
 *   pts     host array of nprob device pointers (n[p] x 3 row-major each).
 *   n       host array of nprob sizes.
 *   params  host; one set shared by all problems.
 *   alloc   as for h2ulv_factorize (shared by all problems).
 *   out     host array of nprob factor handles.
 * Results are identical to nprob separate h2ulv_factorize calls.
 * Errors: as h2ulv_factorize, and INVALID_ARG for nprob < 1 or a NULL array;
 * on any error every out[p] is NULL (no partial batch is returned).
 */
h2ulv_status h2ulv_factorize_batch(int32_t nprob, const double* const* pts, const int64_t* n,
                                   const h2ulv_params* params, const h2ulv_allocator* alloc,
                                   void* stream, h2ulv_factor** out);

/*
 * Solve A~ x = b in place (Sec. II-B three-step solve, level by level).
 *   b     device, n x nrhs column-major with leading dimension ldb >= n;
 *         on entry the right-hand sides, on exit the solutions.
 * Errors: INVALID_ARG (NULL, nrhs < 1, ldb < n), HIP.
 */
h2ulv_status h2ulv_solve(const h2ulv_factor* f, double* b, int32_t nrhs, int64_t ldb,
                         void* stream);

/*
 * h2ulv_solve for callers that apply one factor many times (iterative
 * methods; the library's refinement calls use it): the first call for a given
 * nrhs records the solve's launches in a HIP graph on buffers the factor
 * keeps (an n x nrhs staging block, scratch and descriptors) and takes longer;
 * later calls copy b in, replay the graph and copy the result back.  Results
 * are identical to h2ulv_solve.  Replays on one factor are ordered through an
 * event, whatever their streams.  The recorded graphs live until
 * h2ulv_destroy.  Errors as h2ulv_solve.
 */
h2ulv_status h2ulv_solve_repeated(const h2ulv_factor* f, double* b, int32_t nrhs, int64_t ldb,
                                  void* stream);

/*
 * y = A x with the exact kernel matrix generated on the fly in float64
 * (A_ii = diag; used for residuals).  x, y device, n x nrhs column-major.
 * For n >= 65536 the sources are split over several workgroups whose partial
 * sums are added in a fixed order (deterministic); the call then waits for
 * its stream before returning.
 */
h2ulv_status h2ulv_matvec_exact(const h2ulv_factor* f, const double* x, int64_t ldx,
                                double* y, int64_t ldy, int32_t nrhs, void* stream);

/*
 * h2ulv_matvec_exact without any device allocation, for callers that cannot
 * allocate: code under stream capture, tight serving loops, harnesses that
 * forbid allocation.  Same arguments, launches, split and summation order as
 * h2ulv_matvec_exact (the results are identical); it neither allocates nor
 * synchronises the stream.  The partial sums live in a file-scope device
 * array of 16 Mi doubles (128 MiB) that each GPU the library runs on holds
 * until the process ends.  A request needs the largest of: n * min(nrhs, 8) *
 * splits doubles for the split sources (splits = min(8, 4096 / ceil(n / 512))
 * from n >= 65536 on, none below) and, for the Laplace and Yukawa kernels from
 * n > 261632 on (the pair forms), 72 n when nrhs >= 8 and 9 n when nrhs is
 * not a multiple of 4.  So every n <= 261632 fits, one column fits up to
 * n = 1864135, and larger requests return INVALID_ARG before any launch.  All calls on
 * one GPU share that array: calls whose executions overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller.
 * Errors: INVALID_ARG (as h2ulv_matvec_exact, or too large), HIP.
 */
h2ulv_status h2ulv_matvec_exact_noalloc(const h2ulv_factor* f, const double* x, int64_t ldx,
                                        double* y, int64_t ldy, int32_t nrhs, void* stream);

/*
 * Iterative refinement with the exact float64 matvec:
 *   x = solve(b); repeat r = b - A x; stop when max_c |r_c| / |b_c| <= rtol,
 *   else x += solve(r); at most max_iter corrections.
 *   b     device, read only; x device, receives the solution.
 *   iters host (may be NULL): number of corrections applied.
 *   relres host (may be NULL): final max relative residual.
 * Synchronises the stream once per iteration.
 * Errors: INVALID_ARG, NOT_CONVERGED (x holds the last iterate), HIP, OOM.
 */
h2ulv_status h2ulv_refine(const h2ulv_factor* f, const double* b, int64_t ldb, double* x,
                          int64_t ldx, int32_t nrhs, double rtol, int32_t max_iter,
                          int32_t* iters, double* relres, void* stream);

/*
 * The refinement's correction equation solved by restarted GMRES, right-
 * preconditioned by the ULV solve: x0 = solve(b); each step applies one solve
 * and one exact matvec (as a classical refinement step does) and keeps the best
 * correction in the Krylov space; after at most `restart` (1..128) steps the
 * correction is added and the true residual is recomputed with the exact
 * matvec; stop when max_c |r_c| / |b_c| <= rtol.  Right-hand sides are solved
 * one after another.
 *   iters  host (may be NULL): Krylov steps taken (largest over the columns).
 *   relres host (may be NULL): final max relative residual.
 * Synchronises the stream once per step.  Device scratch: (2 restart + 3) n nrhs
 * doubles (the right-hand sides advance together).
 * Errors: INVALID_ARG, NOT_CONVERGED (after max_iter steps; x holds the last
 * iterate), HIP, OOM.
 */
h2ulv_status h2ulv_refine_gmres(const h2ulv_factor* f, const double* b, int64_t ldb, double* x,
                                int64_t ldx, int32_t nrhs, double rtol, int32_t max_iter,
                                int32_t restart, int32_t* iters, double* relres, void* stream);

/*
 * Block GMRES for several right-hand sides: the refinement's correction
 * equations of all nrhs columns share one Krylov space of the operator A M^-1
 * (M the ULV solve), restarted after `restart` (1..128) block steps.  Each step
 * applies one solve and one exact matvec to a block of up to nrhs vectors, so
 * the outlying eigenvalues of the preconditioned operator, the same for every
 * column, are found once for all columns.  Columns are scaled by 1/|b_c|;
 * directions of a block below 1e-12 of its largest (or, in a restart's first
 * block, below 1e-3 rtol) are dropped.  Stops when every column's relative
 * residual (exact matvec) is <= rtol.  iters: block steps taken; relres: the
 * largest relative residual.  Device scratch about (2 restart + 3) n nrhs
 * doubles.  Same arguments and errors as h2ulv_refine_gmres.
 */
h2ulv_status h2ulv_refine_block_gmres(const h2ulv_factor* f, const double* b, int64_t ldb,
                                      double* x, int64_t ldx, int32_t nrhs, double rtol,
                                      int32_t max_iter, int32_t restart, int32_t* iters,
                                      double* relres, void* stream);

/* Statistics of a factor (host).  Synchronises nothing. */
h2ulv_status h2ulv_get_stats(const h2ulv_factor* f, h2ulv_stats* s);

/*
 * Inspection of a factor, for checking it against an independent
 * implementation.  All arrays are host memory provided by the caller.
 *   h2ulv_get_levels: *L = number of levels (leaves at level L).
 *   h2ulv_get_perm:   perm[n]: tree position -> original point index.
 *   h2ulv_get_ranks:  for level `lev` (1..L): m[2^lev], k[2^lev] (either may be NULL).
 *   h2ulv_get_skeleton: for box `box` of level `lev`: the k skeleton point
 *                       indices (original numbering) in pivot order.
 *   h2ulv_get_basis:  U (m x m column-major, [U^S U^R]) of a box; copies from
 *                     the device and synchronises the stream.
 *   h2ulv_get_column_skeleton, h2ulv_get_column_basis: the same for the
 *                     column side, V (m x m, [V^S V^R]) and the column
 *                     skeletons (Sec. III-C, Eq. fillv); with shared bases
 *                     (V = U) they return the row side's.
 */
h2ulv_status h2ulv_get_levels(const h2ulv_factor* f, int32_t* L);
h2ulv_status h2ulv_get_perm(const h2ulv_factor* f, int64_t* perm);
h2ulv_status h2ulv_get_ranks(const h2ulv_factor* f, int32_t lev, int32_t* m, int32_t* k);
h2ulv_status h2ulv_get_skeleton(const h2ulv_factor* f, int32_t lev, int32_t box, int64_t* sk);
h2ulv_status h2ulv_get_basis(const h2ulv_factor* f, int32_t lev, int32_t box, double* U);
h2ulv_status h2ulv_get_column_skeleton(const h2ulv_factor* f, int32_t lev, int32_t box,
                                        int64_t* sk);
h2ulv_status h2ulv_get_column_basis(const h2ulv_factor* f, int32_t lev, int32_t box, double* V);

void h2ulv_destroy(h2ulv_factor* f);

/*
 * Host-only structure (no GPU needed): cluster tree and near/far lists
 * (Sec. I strong admissibility; Sec. III-D binary tree) built from host points.
 *   h2ulv_structure_create: pts host n x 3 row-major.
 *   h2ulv_structure_perm:   perm[n].
 *   h2ulv_structure_lists:  for level lev, CSR arrays of the near and far lists:
 *       near_ptr[2^lev + 1], near_idx[near_ptr[2^lev]] (sorted per row), same
 *       for far.  Pass NULL index arrays to query only the row pointers.
 *   h2ulv_structure_geometry: centre[2^lev * 3], radius[2^lev] of level lev.
 */
typedef struct h2ulv_structure h2ulv_structure;
h2ulv_status h2ulv_structure_create(const double* pts, int64_t n, const h2ulv_params* params,
                                    h2ulv_structure** out);
h2ulv_status h2ulv_structure_levels(const h2ulv_structure* s, int32_t* L);
h2ulv_status h2ulv_structure_perm(const h2ulv_structure* s, int64_t* perm);
h2ulv_status h2ulv_structure_lists(const h2ulv_structure* s, int32_t lev, int64_t* near_ptr,
                                   int32_t* near_idx, int64_t* far_ptr, int32_t* far_idx);
h2ulv_status h2ulv_structure_geometry(const h2ulv_structure* s, int32_t lev, double* centre,
                                      double* radius);
void h2ulv_structure_destroy(h2ulv_structure* s);

/*
 * Kernel timing (the measurement behind the reported roofline fractions).
 * h2ulv_profile_enable(1) clears earlier records, creates a pool of events and
 * starts recording a pair of HIP events around every batched launch of the main
 * kernels, on the stream the launch uses; h2ulv_profile_enable(0) stops
 * recording.
 * h2ulv_profile_read waits for the recorded events, aggregates them per kernel
 * (launch count, summed duration, summed algorithmic flops and operand bytes:
 * GEMM 2MNK flops and (MK + KN + MN) element bytes; kernel generation counts
 * entries in `flops`) into out[0 .. min(max, count) - 1] and clears the
 * records.  *count receives the number of distinct kernels.  Host memory.
 */
typedef struct h2ulv_kernel_profile {
  char name[32];
  int64_t launches;
  double time_ms;
  double flops;
  double bytes;
} h2ulv_kernel_profile;
h2ulv_status h2ulv_profile_enable(int32_t on);
h2ulv_status h2ulv_profile_read(h2ulv_kernel_profile* out, int32_t max, int32_t* count);

/*
 * The grouped GEMM's tile shapes are chosen per batch from their full-tile
 * rates on the device, measured (autotuned) the first time a precision is used
 * on a device and kept for the process.  out (host, 6 doubles) receives the
 * measured rates in TFLOP/s: FP64 tiles 64x64, 64x128, 128x64, 128x128, then FP32
 * tiles 64x64, 128x128; 0 where not measured yet on the current device.
 * Errors: INVALID_ARG (NULL).
 */
h2ulv_status h2ulv_gemm_tile_rates(double* out);

/*
 * Learned rank prediction for the shared-basis step (the row ID of Sec. II-A /
 * III-C, computed differently; the method is unchanged).
 *
 * Features.  Every factorization records 16 features per box and level (float32):
 *   0 log2(1+m)/12 (candidate rows)        1 log2(1+points of the box)/20
 *   2 level/L                              3 log2(1+|Near|)/6
 *   4 log2(1+|Far|)/6                      5 log2(1+|fill targets|)/8
 *   6 log2(1+columns of M')/20             7 -log10(tol)/16 (1 if tol = 0)
 *   8 alpha r (Yukawa) else 0              9-11 sqrt(covariance eigenvalues of the
 *                                               box's points, descending) / r
 *   12 log2(max(r/r_root, 2^-30))/16       13 (k_c1+k_c2)/(m_c1+m_c2) of the
 *                                              children (1 at the leaves)
 *   14 1 at the leaves else 0              15 eta/2
 * with r the box radius (half its bounding-box diagonal).  The training target
 * is log2(1 + k).
 *
 * Model.  16 -> 64 -> 64 -> 64 (ReLU) -> 1, float32, one flat parameter array
 * of H2ULV_MLP_NPARAM floats: W1 (64 x 16 row-major), b1, W2 (64 x 64), b2, W3,
 * b3, w4 (64), b4.  Prediction k-hat = max(0, round(2^y - 1)).
 *
 * Use in the factorization (params.rank_model != NULL).  For each box the
 * sketch size is l = min(ceil(1.25 k-hat) + oversample, m - 8).  When
 * 0 < l < columns of M' and (rank_cap == 0 or l < rank_cap), the row ID comes from
 * the column-pivoted QR of (M' Omega)^T for a Gaussian matrix Omega (columns
 * of M' x l) whose rows are keyed by point: entry (p, c) is Box-Muller deviate
 * number c N + p (N points) of the SplitMix64 stream at position
 * (level << 40) | (2^39 + s) of the stream seeded by sketch_seed, s = 0 for the
 * far-field columns and s = 1 for the fill-in columns.  M' is never formed for
 * a sketched box: its fill part is applied as sum_k Z'_ik Q_k with
 * Q_k = sum_j D_kj Omega_j shared by the boxes next to k.  8 further columns G
 * of the same rows probe the error, and the sketch is
 * accepted iff it was not exhausted (k < l) and
 *   ||Z[piv[k:]] - E^T Z[piv[:k]]||_F <= 10 sqrt(m - k) tol max_j ||Z[j]||,
 * Z = M' G, E = R11^-1 R12.  A rejected sketch narrower than m - 8 is retried
 * once at l = m - 8; if that is rejected too, the box uses the full pivoted QR.
 */
#define H2ULV_NFEAT 16
#define H2ULV_MLP_NPARAM 9473

/* New model with He-normal weights from the Gaussian generator keyed by seed
 * (biases 0); parameters live on the current device.  Free with
 * h2ulv_rankmodel_destroy (after every factorization that uses it). */
h2ulv_status h2ulv_rankmodel_create(uint64_t seed, h2ulv_rankmodel** out);
void h2ulv_rankmodel_destroy(h2ulv_rankmodel* m);
/* Copy the H2ULV_MLP_NPARAM parameters from / to host memory (synchronous). */
h2ulv_status h2ulv_rankmodel_set_params(h2ulv_rankmodel* m, const float* host);
h2ulv_status h2ulv_rankmodel_get_params(const h2ulv_rankmodel* m, float* host);
/* Write the model (parameters, both Adam moments and the Adam step count) to
 * the file at path, in the library's versioned binary format ("H2RM", format
 * version 1, H2ULV_MLP_NPARAM float32 values per array, host byte order), so a
 * model trained in one process can size the sketches of another.  Synchronous.
 * Errors: INVALID_ARG (NULL argument, a file that cannot be written), HIP. */
h2ulv_status h2ulv_rankmodel_save(const h2ulv_rankmodel* m, const char* path);
/* New model read from a file that h2ulv_rankmodel_save wrote, with its Adam
 * state, so training can continue.  The file is checked (magic, version,
 * parameter count, exact size) before any device work.  Free with
 * h2ulv_rankmodel_destroy.  Errors: INVALID_ARG (NULL argument, missing,
 * foreign, truncated or oversized file; *out is then NULL), OOM, HIP. */
h2ulv_status h2ulv_rankmodel_load(const char* path, h2ulv_rankmodel** out);
/* y[s] = model(feat[s, :]) for n samples; feat device n x 16 row-major, y device. */
h2ulv_status h2ulv_rankmodel_forward(const h2ulv_rankmodel* m, const float* feat, int64_t n,
                                     float* y, void* stream);
/* grad (device, H2ULV_MLP_NPARAM) = d/dparams of mean_s (y_s - target_s)^2;
 * *loss (host, may be NULL) = that mean.  Synchronises the stream. */
h2ulv_status h2ulv_rankmodel_gradient(const h2ulv_rankmodel* m, const float* feat,
                                      const float* target, int64_t n, float* grad, float* loss,
                                      void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the given gradient. */
h2ulv_status h2ulv_rankmodel_adam_step(h2ulv_rankmodel* m, const float* grad, float lr,
                                       void* stream);
/* `steps` full-batch Adam steps on (feat, target); *loss (host, may be NULL)
 * receives the loss before the last step.  Synchronises the stream. */
h2ulv_status h2ulv_rankmodel_train(h2ulv_rankmodel* m, const float* feat, const float* target,
                                   int64_t n, int32_t steps, float lr, float* loss, void* stream);

/* Features of level lev (1..L) of a factor: feat host 2^lev x 16 row-major,
 * target host 2^lev (log2(1 + k)); either may be NULL. */
h2ulv_status h2ulv_get_features(const h2ulv_factor* f, int32_t lev, float* feat, float* target);
/* Per box of level lev: predicted rank (-1 without a model; predicted also on
 * the levels above params.sketch_min_level, which are not sketched), sketch
 * columns of the last attempt (0: not sketched) and outcome (0 not sketched,
 * 1 accepted, 2 fell back to the full pivoted QR, 3 accepted on the full-width
 * retry). */
h2ulv_status h2ulv_get_sketch_info(const h2ulv_factor* f, int32_t lev, int32_t* khat,
                                   int32_t* ell, int32_t* state);

/*
 * Device memory the library freed is kept in a cache and reused by later
 * calls (hipMalloc/hipFree stall behind queued work).  The cache gives memory
 * back by itself before free device memory would fall below
 * max(16 GiB, 1/16 of the device); h2ulv_release_cache waits for the device and
 * hands every cached block back to the runtime now.
 */
h2ulv_status h2ulv_release_cache(void);

const char* h2ulv_status_string(h2ulv_status s);
const char* h2ulv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* H2ULV_H */
