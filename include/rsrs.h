/*
 * rsrs.h -- C ABI of the MI355X (gfx950) implementation of randomized strong
 * recursive skeletonization (RSRS): compression and LU factorization of a
 * strongly admissible H2 matrix from one set of sketches
 *     Y = A Omega,   Z = A^T Psi,   Omega, Psi ~ N(0, 1)   (N x s each),
 * where A (N x N, rows and columns tagged with points in R^2 or R^3) is known
 * only through products with A and A^T (Yesypenko & Martinsson, Sec. 1 and
 * Sec. 4, eq. rand_sample_setting).  The factorization produced is the one of
 * Sec. 3 (eq. Afact, Ainvfact) reconstructed by Algorithm 1.
 *
 * Conventions (all entry points)
 *  - Every function returns rsrs_status; RSRS_OK is 0.  On error nothing is
 *    allocated for the caller and rsrs_last_error() (thread-local) describes
 *    the failure.
 *  - "device" pointers are HIP device allocations on the current device;
 *    "host" pointers are ordinary process memory.
 *  - Dense blocks of points are ROW-MAJOR: entry (point i, column j) of an
 *    N x w block X with leading dimension ldx is X[i*ldx + j], ldx >= w.
 *    Points are in the caller's ("user") order unless stated otherwise.
 *  - stream: a hipStream_t passed as void*; NULL means the default stream.
 *    Work is stream-ordered; functions that must read results on the host
 *    (tree building, factor bookkeeping) synchronise the stream themselves.
 *  - Handles are not thread-safe; distinct handles may be used from
 *    distinct threads.  The library owns everything it returns through an
 *    out-pointer until the matching *_destroy call.
 */
#ifndef RSRS_H
#define RSRS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RSRS_OK = 0,
  RSRS_E_INVALID = 1,      /* bad argument (null pointer, size, layout)          */
  RSRS_E_SAMPLES = 2,      /* s below the requirement; see rsrs_last_required_s   */
  RSRS_E_SINGULAR = 3,     /* a pivot block or the root block is singular        */
  RSRS_E_CALLBACK = 4,     /* the user matvec returned nonzero                    */
  RSRS_E_NUMERIC = 5,      /* NaN or Inf met in samples or residuals              */
  RSRS_E_NOMEM = 6,        /* device allocation failed                            */
  RSRS_E_HIP = 7,          /* HIP runtime error                                   */
  RSRS_E_UNSUPPORTED = 8,  /* option not implemented                              */
  RSRS_E_TIMEOUT = 9       /* a server wait ran out of time (request still pending) */
} rsrs_status;

typedef struct rsrs_tree_s rsrs_tree_t;
typedef struct rsrs_samples_s rsrs_samples_t;
typedef struct rsrs_factor_s rsrs_factor_t;
typedef struct rsrs_operator_s rsrs_operator_t;
typedef struct rsrs_server_s rsrs_server_t;

const char* rsrs_status_string(rsrs_status st);
const char* rsrs_last_error(void);
/* After RSRS_E_SAMPLES: the number of samples that would have been enough. */
int64_t rsrs_last_required_s(void);

/* ------------------------------------------------------------------------
 * Tree (Sec. 3, opening paragraphs; eq. active, BNactive).  Pure host code,
 * deterministic and bit-identical for identical input bits.
 *  - Root box: the cube [root_lo, root_lo + root_side)^dim.
 *  - Coordinates are quantized to qbits (<= 20; 0 selects 20) bits per axis:
 *    q = clamp(floor(((x - lo) / side) * 2^qbits), 0, 2^qbits - 1) in FP64;
 *    a point on a split plane belongs to the upper child.
 *  - A box holding more than leaf_size points is split into its non-empty
 *    children; leaves are then split until the tree is 2:1 balanced
 *    (no leaf's closed box meets a leaf two or more levels finer).
 *  - Box ids: sorted by (level, Morton code), axis 0 in the lowest bit.
 *  - Tree order of points: leaves in Morton order of their first finest cell,
 *    ascending user index inside a leaf; each box owns a contiguous range.
 * pts: host, n x dim row-major FP64.  *out is owned by the caller and freed
 * with rsrs_tree_destroy.
 * ---------------------------------------------------------------------- */
typedef struct {
  int dim;             /* 2 or 3 */
  int leaf_size;       /* m >= 1 */
  int qbits;           /* 0 -> 20 */
  double root_lo[3];
  double root_side;    /* > 0 */
} rsrs_tree_opts;

rsrs_status rsrs_build_tree(const double* pts, int64_t n, const rsrs_tree_opts* opts,
                            rsrs_tree_t** out);
void rsrs_tree_destroy(rsrs_tree_t* t);

/* Read-only views of the tree arrays (host memory owned by the tree, valid
 * until rsrs_tree_destroy).  coords is nbox x dim; perm maps tree position to
 * user index. */
typedef struct {
  int dim, nlevels, qbits;
  int64_t n, nbox;
  const int32_t* level;
  const int32_t* coords;
  const int64_t* parent;     /* -1 for the root */
  const uint8_t* is_leaf;
  const int64_t* pt_begin;
  const int64_t* pt_end;
  const int64_t* perm;
} rsrs_tree_info;
rsrs_status rsrs_tree_get_info(const rsrs_tree_t* t, rsrs_tree_info* out);

/* Neighbour lists while level `level` (1..nlevels) is processed: for each
 * level-`level` box (ascending id, *nb of them, ids in *boxes), the
 * representatives (level-`level` boxes and coarser leaves) whose closed box
 * meets it, self excluded, ascending by id, in CSR form (offsets has *nb+1
 * entries).  Pointers are owned by the tree. */
rsrs_status rsrs_tree_neighbours(const rsrs_tree_t* t, int level, int64_t* nb,
                                 const int64_t** boxes, const int64_t** offsets,
                                 const int64_t** nbrs);

/* Box order for fixed rank k (Algorithm 1 with the order the paper leaves
 * open fixed as follows): levels nlevels..1; a level-l box is processed when
 * its active count b exceeds k.  Processed boxes of a level are coloured
 * greedily in order (sum_a (coord_a mod 3) 3^a, id): each takes the smallest
 * colour not held by a box whose closed neighbourhood {B} u N(B) meets its
 * own; colours run ascending, boxes inside a colour by id.  Host outputs of
 * nbox entries (caller-allocated): colour (-1 = not processed), b_count
 * (active count when its level runs), l_count (b + active neighbour count
 * when processed, else 0).  *root_count = |B_t|. */
rsrs_status rsrs_tree_schedule(const rsrs_tree_t* t, int k, int32_t* colour, int64_t* b_count,
                               int64_t* l_count, int64_t* root_count);

/* Smallest s with s >= |B_a| + |N_a| + k + p for every processed box
 * (eq. s_L, s_B; count of Sec. 4.5 under the order above) and s >= |B_t|.
 * Returns -1 on invalid arguments. */
int64_t rsrs_samples_required(const rsrs_tree_t* t, int k, int p);

/* Tile autotuning of the batched MFMA GEMM behind every factorization and
 * solve product (not a step of the paper: a property of this implementation).
 * The candidates are 64 x 64 tiles on 4 waves, 128 x 64 on 4 waves and
 * 128 x 128 on 8 waves; the triangular (SYRK) form takes only the square
 * ones.  Launch classes: element type (FP32, FP64), product form, the
 * launch's count of 64 x 64 output tiles (4^1 .. 4^7, nearest in log scale)
 * and its contraction length (128 or 1024, nearest in log scale): 196
 * classes.  Each class is timed on synthetic operands (one warm-up and the
 * best of three launches per candidate), and a challenger replaces the
 * built-in rule only when it is 3% faster.  The fastest shape then serves
 * every later automatic launch of its class in this process.  Without a
 * table the built-in rule applies: 128 x 128 when the launch has >= 256 such
 * tiles, else 64 x 64.
 * cache_path (may be NULL): a table that an earlier call wrote there is
 * loaded and nothing is timed; otherwise the table is measured on the current
 * device (about 3 GB of scratch, freed again) and written there.
 * *entries receives the number of classes and *changed how many of them
 * differ from the built-in rule (either may be NULL).  The shape never
 * changes a result: every candidate accumulates each output entry over the
 * same K slices in the same order.  Call it while no factorization or solve
 * is running.  Errors: RSRS_E_HIP, RSRS_E_NOMEM. */
rsrs_status rsrs_gemm_autotune(const char* cache_path, int64_t* entries, int64_t* changed);
/* Forces one tile shape for every automatic launch: 0 = 64 x 64,
 * 1 = 128 x 64 (64 x 64 for the triangular form), 2 = 128 x 128.  -1 goes
 * back to the tables (or the built-in rule).  -2 also forgets both tables.  For
 * tests and measurements.  Other values -> RSRS_E_INVALID. */
rsrs_status rsrs_gemm_tile_override(int shape);

/* ------------------------------------------------------------------------
 * Black-box operator access (Sec. 4, eq. rand_sample_setting).
 * The callback computes Y = A X (transpose = 0) or Y = A^T X (transpose = 1)
 * for an N x ncols device block X (row-major, user order, leading dimension
 * ldx) into the device block Y (leading dimension ldy), stream-ordered on
 * `stream`.  It returns 0 on success; any other value aborts the caller with
 * RSRS_E_CALLBACK.
 * ---------------------------------------------------------------------- */
/* Element type of a device block: RSRS_F64 (double) or RSRS_F32 (float).
 * RSRS_BF16 names float blocks whose values are BF16 numbers: a product
 * requested with it may round the operator to BF16 and accumulate in FP32. */
enum { RSRS_F64 = 0, RSRS_F32 = 1, RSRS_BF16 = 2 };
/* X and Y have element type `dtype` (float for RSRS_BF16).  The library asks
 * for RSRS_F32 / RSRS_BF16 products only while sampling FP32 sketches
 * (rsrs_sample with that dtype); residuals of rsrs_solve_refine are always
 * requested in RSRS_F64.  A callback that does not provide the requested
 * type returns nonzero. */
typedef int (*rsrs_matvec_fn)(void* user, int transpose, int dtype, int64_t ncols, const void* X,
                              int64_t ldx, void* Y, int64_t ldy, void* stream);

/* Built-in synthetic operators (HIP kernels; the handle is the `user` of
 * rsrs_op_matvec, which has the rsrs_matvec_fn signature):
 *  RSRS_OP_LOG2D  A_ij = delta_ij + h^2 (-log|x_i - x_j| / (2 pi)), i != j,
 *                 A_ii = 1 + h^2 / 2      (param = h; dim 2)
 *  RSRS_OP_INVR3D A_ij = delta_ij + (1/N) / (4 pi |x_i - x_j|), A_ii = 1
 *                 (param unused; dim 3)
 *  RSRS_OP_LOG2D_SKEW  LOG2D plus param2 * (x_i - x_j)_0 / |x_i - x_j|^2
 *                 (non-symmetric)
 *  RSRS_OP_LOG2D_FIRST  the first-kind log kernel (no identity term):
 *                 A_ij = h^2 (-log|x_i - x_j| / (2 pi)), i != j, and
 *                 A_ii = h^2 (-log h - c) / (2 pi), the kernel's mean over a
 *                 cell of side h, c = (log 2 - 3 + pi/2) / 2 - log 2 the
 *                 mean of log|u| over the unit square (param = h; dim 2)
 * pts: host n x dim (user order); copied to the device.  The kernel matrix is
 * materialised on the device in FP64 at creation (n^2 doubles); an FP32 copy
 * (n^2 floats) is added at the first RSRS_F32 product, whose product is then
 * an FP32 MFMA GEMM with FP32 accumulation, and a BF16 copy (n^2 x 2 bytes) at
 * the first RSRS_BF16 product (BF16 MFMA, FP32 accumulation; n a multiple of
 * 8; transposed products of the skewed kernel use the FP32 product). */
enum { RSRS_OP_LOG2D = 1, RSRS_OP_INVR3D = 2, RSRS_OP_LOG2D_SKEW = 3, RSRS_OP_LOG2D_FIRST = 4 };
rsrs_status rsrs_op_create_kernel(int kind, const double* pts, int64_t n, int dim,
                                  double param, double param2, rsrs_operator_t** out);
/* Explicit matrix: A is a device n x n row-major array (leading dimension
 * lda), borrowed (must outlive the operator).  RSRS_F64 products only. */
rsrs_status rsrs_op_create_dense(const double* A, int64_t n, int64_t lda, rsrs_operator_t** out);
/* 7-point -div(a grad u) on the n^3 interior nodes of the grid h = 1/(n+1)
 * (x fastest), face coefficient = mean of the two node values, Dirichlet
 * nodes eliminated; coef: host (n+2)^3 node values indexed [z][y][x].
 * RSRS_F32 products read and write float and accumulate in FP64. */
rsrs_status rsrs_op_create_poisson7(int n, const double* coef, rsrs_operator_t** out);
int rsrs_op_matvec(void* op, int transpose, int dtype, int64_t ncols, const void* X, int64_t ldx,
                   void* Y, int64_t ldy, void* stream);
void rsrs_op_destroy(rsrs_operator_t* op);
/* Products of the built-in dense operators (kernel matrices and explicit
 * matrices, the stand-ins for a user's black box) with blocks wider than 16
 * columns are plain GEMMs: they go to rocBLAS (FP64, FP32) and hipBLASLt
 * (BF16) when those take the shape.  enable = 0 sends them to the library's
 * own MFMA GEMM kernels instead, process-wide; 1 restores the default.  The
 * results agree to rounding either way.  For tests and comparisons; call it
 * while no product is running.  Returns RSRS_OK. */
rsrs_status rsrs_op_library_gemm(int enable);

/* ------------------------------------------------------------------------
 * Samples {Y, Z, Omega, Psi} (Algorithm 1, Require).  Stored by the library
 * in tree order, row-major N x s on the device, element type dtype
 * (RSRS_F64, or RSRS_F32 for the mixed-precision factorization).
 * ---------------------------------------------------------------------- */
/* Copy caller-provided device sketches (user order, row-major, leading
 * dimension ld >= s, element type dtype) into library-owned tree-ordered
 * storage.  The caller's arrays are not modified. */
rsrs_status rsrs_samples_wrap(const rsrs_tree_t* t, int dtype, const void* Y, const void* Z,
                              const void* Omega, const void* Psi, int64_t ld, int64_t s,
                              void* stream, rsrs_samples_t** out);
/* Draw Omega, Psi on the device with Philox-4x32-10 (Salmon et al., SC'11)
 * and Box-Muller, then Y = A Omega and Z = A^T Psi through `mv`.  Element
 * (user row i, column j) of Omega uses counter (i, j, 0, seed_hi) and key
 * (seed_lo, 0x2311); Psi uses stream word 1 in place of 0.  With dtype
 * RSRS_F32 the FP64 normal is rounded to float and `mv` is asked for FP32
 * products of the rounded test matrices; with RSRS_BF16 it is rounded
 * further to BF16 (kept in float) and `mv` is asked for RSRS_BF16 products.
 * Both give FP32 samples for RSRS_PREC_F32_MIXED. */
rsrs_status rsrs_sample(const rsrs_tree_t* t, rsrs_matvec_fn mv, void* user, int64_t s,
                        uint64_t seed, int dtype, void* stream, rsrs_samples_t** out);
/* Symmetric operators (A = A^T): only Omega and Y = A Omega are drawn /
 * taken (Z = Y and Psi = Omega implicitly); for opts.symmetric = 1. */
rsrs_status rsrs_sample_symmetric(const rsrs_tree_t* t, rsrs_matvec_fn mv, void* user, int64_t s,
                                  uint64_t seed, int dtype, void* stream, rsrs_samples_t** out);
rsrs_status rsrs_samples_wrap_symmetric(const rsrs_tree_t* t, int dtype, const void* Y,
                                        const void* Omega, int64_t ld, int64_t s, void* stream,
                                        rsrs_samples_t** out);
void rsrs_samples_destroy(rsrs_samples_t* smp);

/* Fill a device array with standard normals from the generator above:
 * out[i*ld + j] for i < nrows, j < ncols uses counter (i, j, word, seed_hi). */
rsrs_status rsrs_gaussian(double* out, int64_t nrows, int64_t ncols, int64_t ld, uint64_t seed,
                          uint32_t word, void* stream);

/* ------------------------------------------------------------------------
 * Factorization (Algorithm 1).  The samples are consumed: Algorithm 1
 * updates them in place, so they cannot be reused afterwards.
 *  s < rsrs_samples_required(t, k, p)  -> RSRS_E_SAMPLES
 *  singular pivot block / root block   -> RSRS_E_SINGULAR
 *  non-finite value in the samples     -> RSRS_E_NUMERIC
 *  precision / sample dtype mismatch   -> RSRS_E_INVALID
 * The factor is device-resident and owned by the caller.
 *
 * Precision.  RSRS_PREC_F64: FP64 samples, FP64 arithmetic and factor.
 * RSRS_PREC_F32_MIXED: FP32 samples and an FP32 stored factor; every product
 * of sketch-sized operands (Gram matrices, projections, extraction,
 * multipliers, sparsification and elimination updates) runs on FP32 MFMA with
 * FP32 accumulation, and the Gram matrices are Cholesky-factored in FP32,
 * while the rank decisions stay FP64: the column-pivoted QR of the ID keeps
 * the projected sketch's rows in FP32 but takes its dot products, norms and
 * coefficients in FP64, and X_RR and the root block are inverted by FP64
 * Gauss-Jordan with partial pivoting.  Solves with such a
 * factor take and return FP64 blocks and compute in FP32; accuracy is
 * recovered by rsrs_solve_refine with the FP64 black-box residual.
 *
 * Symmetric variant (opts.symmetric = 1, for A = A^T; U = L^T as noted in
 * Sec. 2.2 and after eq. Ainvfact): with Psi = Omega the two sketches
 * coincide, so only Y and Omega are used (samples from
 * rsrs_sample_symmetric / rsrs_samples_wrap_symmetric, or the Y / Omega half
 * of general samples).  Each box runs the Y / Omega side of the general step;
 * X_RR and the root block are replaced by their symmetric parts and
 * K_L = K_U^T, so the approximate inverse is exactly symmetric.  Symmetric
 * samples with opts.symmetric = 0 -> RSRS_E_INVALID.
 * ---------------------------------------------------------------------- */
enum { RSRS_PREC_F64 = 0, RSRS_PREC_F32_MIXED = 1 };
/* Sketch the ID is taken of (Algorithm 1 writes the sum of the projected
 * sketches; Sec. 3.1 skeletonizes rows and columns with one index set, the
 * concatenated form).  The symmetric variant takes the ID of M_Y either way. */
enum { RSRS_ID_SUM = 0, RSRS_ID_CONCAT = 1 };
typedef struct {
  int k;            /* rank (k_B = min(k, b)); with rank_tol > 0 the cap on k_B */
  int p;            /* oversampling used in the sample check; < 0 -> p = k */
  int precision;    /* RSRS_PREC_F64 (FP64 samples) or RSRS_PREC_F32_MIXED (FP32 samples) */
  int reproject;    /* extra projection passes in the nullification (0 or 1; default 1) */
  int symmetric;    /* 1: symmetric variant for A = A^T (see below); 0: general */
  int id_mode;      /* RSRS_ID_SUM (0): ID of M = M_Y + M_Z; RSRS_ID_CONCAT: of [M_Y, M_Z] */
  double rank_tol;  /* 0: fixed rank.  > 0: k_B = the number of leading pivots of the
                       column-pivoted QR whose |R_jj| exceeds rank_tol ||[Y_B Z_B]||_F
                       (at most min(k, b)); boxes and their order stay those of the
                       fixed-rank schedule, whose active counts bound the actual ones */
  int col_subset;   /* 0: every box reads all s sample columns.  1: a box with l active
                       columns reads only the first s_B = min(s, l + k + p) in its
                       nullification, ID and extraction (the leading columns of a sample
                       pair are a sample pair, Sec. 1.1; s_B - l = k + p is the null-space
                       dimension the count of Sec. 4.5 gives every box); its
                       sparsification and elimination still update all s columns.  Less
                       oversampling for boxes with small l: a variant, not the default */
} rsrs_factor_opts;

/* Algorithmic work of a fixed-rank factorization with s samples and the
 * options opts (k, p, symmetric, col_subset are read), as the cost analysis
 * of Sec. 4.5 prices the steps of Algorithm 1 (the method's own operations,
 * not the kernels that carry them out): per processed box with b active
 * points, n active neighbour points, l = b + n, k_B = min(k, b), r = b - k_B,
 * and c = s (c = s_B = min(s, l + k + p) with col_subset) columns read,
 *   2(4 c l^2 - 4/3 l^3) + 8 b c l + 4 c b k_B + 8 r k_B s + 4 r c l
 *   + 2/3 r^3 + 4 r^2 (k_B + n) + 8 r (k_B + n) s  flops,
 * esize (c (2l + 2b) + 2 s n + s (4b + 2n) + stored) bytes with
 * r k_B + r^2 + 2 r (k_B + n) stored entries; symmetric != 0 halves the
 * two-sided terms (all but the pivoted QR and the LU) and stores one
 * multiplier.  The root adds (4 s t^2 - 4/3 t^3) + 2 s t^2 + t^3 + 2/3 t^3
 * flops and t^2 stored entries, t = |B_t|.  A solve costs 2 flops per stored
 * entry and right-hand side.  Outputs may be NULL.  esize is 4 or 8. */
rsrs_status rsrs_work_model(const rsrs_tree_t* t, const rsrs_factor_opts* opts, int64_t s, int esize,
                            double* flops, double* bytes, int64_t* stored_entries);
/* Workload tuning of the GEMM tile choice (see rsrs_gemm_autotune below): the factorization of (t, opts, s)
 * -- the fixed-rank launch sequence; opts.rank_tol is ignored -- is run on
 * Gaussian samples (Philox, drawn here) once per candidate: the current
 * choice, then each of the three shapes forced.  Every automatic GEMM launch
 * is timed with HIP events under its product's shape signature (element
 * type, form and the list of (M, N, K) of its descriptors).  Each signature
 * then keeps its fastest candidate; a challenger must be 2% faster.  From
 * then on an exact signature match overrides the class table and the
 * built-in rule, so later factorizations and solves with those shapes take
 * the measured choice.  Results never change.  Cost: five factorizations of
 * the workload, including one warm-up.  *signatures receives the number of
 * signatures measured and *changed how many moved from the current choice
 * (either may be NULL).  Call it while no other factorization or solve is
 * running.  Errors: RSRS_E_INVALID and those of rsrs_factor. */
rsrs_status rsrs_gemm_autotune_workload(const rsrs_tree_t* t, const rsrs_factor_opts* opts, int64_t s,
                                        int64_t* signatures, int64_t* changed);

rsrs_status rsrs_factor(const rsrs_tree_t* t, rsrs_samples_t* smp, const rsrs_factor_opts* opts,
                        void* stream, rsrs_factor_t** out);
/* Sampling and factorization with the samples redrawn at the start of every
 * processed level after the first (Sec. 4.4: the approximation errors of a
 * fixed set of sketches accumulate from level to level).  The first samples
 * are those of rsrs_sample / rsrs_sample_symmetric (mv, user, s, seed,
 * dtype; opts.symmetric selects which).  The boxes processed so far have
 * turned A into V^{-1} A W^{-1} (eq. tildeA_diag), and the updated sketches
 * are a sample pair of it (Sec. 1.1).  A redraw replaces them by a fresh
 * pair of the same operator: Omega' Gaussian (Philox as in rsrs_sample, rows
 * in tree order, word 2r for the r-th redraw) and Y' = V^{-1} A W^{-1} Omega'.
 * For the general variant also Psi' (word 2r + 1) and
 * Z' = W^{-T} A^T V^{-T} Psi'. W^{-1} and V^{-1} are the downward and upward
 * sweeps of eq. Ainvfact over the processed boxes, and mv gets and returns
 * blocks in user point order (FP64 for the FP64 factorization, FP32 for the
 * mixed one, whatever the first samples' dtype).  Each redraw costs one
 * product with A (and one with A^T) of s columns.  Fixed rank or rank_tol
 * as in opts.  Errors: those of rsrs_sample and rsrs_factor; RSRS_E_CALLBACK
 * when mv fails during a redraw. */
rsrs_status rsrs_factor_redraw(const rsrs_tree_t* t, rsrs_matvec_fn mv, void* user, int64_t s, uint64_t seed,
                               int dtype, const rsrs_factor_opts* opts, void* stream, rsrs_factor_t** out);
/* Many independent problems factored together (Algorithm 1 on each): trees,
 * samples and opts are arrays of nprob entries (each problem its own N, tree,
 * s and k; all of one precision); out receives nprob factors.  The problems
 * advance through their colour classes in lock step, class t of every
 * problem that has one running in the same batched launches, so the whole
 * batch takes as many host synchronisations as its longest member has colour
 * classes.  Each factor equals the one rsrs_factor computes for that problem
 * alone.  On any error no factor is returned (out[i] = NULL), the error
 * message names the problem, and every sample set that had passed validation
 * counts as consumed. */
rsrs_status rsrs_factor_batched(int64_t nprob, const rsrs_tree_t* const* trees,
                                rsrs_samples_t* const* samples, const rsrs_factor_opts* opts,
                                void* stream, rsrs_factor_t** out);
void rsrs_factor_destroy(rsrs_factor_t* f);
/* A factorization's scratch (device workspace, pinned staging of its
 * uploads) is kept when it returns and reused by the next factorization of
 * a similar size on the same device, which saves milliseconds of allocation
 * and release per call; at most 16 buffers and 32 GiB are kept, the oldest
 * released first.  rsrs_release_cached frees every kept buffer (call it with
 * no factorization running). */
void rsrs_release_cached(void);

typedef struct {
  int64_t n, s, k;
  int64_t nboxes;          /* processed boxes */
  int64_t root_size;       /* |B_t| */
  int64_t stored_values;   /* T, X_RR, X_RR^{-1}, K_U, K_L, root (elements) */
  int64_t stored_bytes;    /* stored_values times the element size */
  int precision;           /* RSRS_PREC_* of the factorization */
  double flops;            /* algorithmic flop count of this factorization */
  double factor_ms;        /* wall time of rsrs_factor (stream synchronised) */
} rsrs_factor_info;
rsrs_status rsrs_factor_get_info(const rsrs_factor_t* f, rsrs_factor_info* out);

/* Per-box export for verification (box i in processing order).  Sizes first,
 * then copies into caller host buffers (any pointer may be NULL to skip):
 * Ba (b), Na (n), S (k), R (r) as tree positions; T r x k, XRR r x r,
 * KU r x (k+n), KL (k+n) x r, row-major FP64 (converted from FP32 for a
 * mixed-precision factor). */
rsrs_status rsrs_factor_box_sizes(const rsrs_factor_t* f, int64_t i, int64_t* box, int32_t* level,
                                  int32_t* colour, int64_t* b, int64_t* n, int64_t* r,
                                  int64_t* k);
rsrs_status rsrs_factor_box_copy(const rsrs_factor_t* f, int64_t i, int64_t* Ba, int64_t* Na,
                                 int64_t* S, int64_t* R, double* T, double* XRR, double* KU,
                                 double* KL);
/* Root block: *nt = |B_t|; Bt (nt tree positions) and At (nt x nt row-major). */
rsrs_status rsrs_factor_root_copy(const rsrs_factor_t* f, int64_t* nt, int64_t* Bt, double* At);

/* ------------------------------------------------------------------------
 * Using the factorization (eq. Afact and eq. Ainvfact).
 *  rsrs_solve: U = A_approx^{-1} F (transpose = 0) or A_approx^{-T} F.
 *  rsrs_apply: Y = A_approx X      (transpose = 0) or A_approx^T X.
 * F, U, X, Y: device N x nrhs row-major blocks in user order; F == U (and
 * X == Y) is allowed.  Stream-ordered, no host synchronisation.
 * ---------------------------------------------------------------------- */
rsrs_status rsrs_solve(const rsrs_factor_t* f, int transpose, int64_t nrhs, const double* F,
                       int64_t ldf, double* U, int64_t ldu, void* stream);
/* Solves and applies of up to 1024 columns replay a HIP graph of the
 * factor's launch sequence, assembled at the first call for each operation
 * and width bucket (16, 32, ..., 1024; narrower blocks are padded with zero
 * columns, which leave the others unchanged); the factor then keeps the
 * graph, its descriptors and work blocks of n x bucket elements (twice)
 * until it is destroyed.  rsrs_solve_graphs(0) switches to direct launches
 * (process-wide; results are identical). */
void rsrs_solve_graphs(int on);
rsrs_status rsrs_apply(const rsrs_factor_t* f, int transpose, int64_t nrhs, const double* X,
                       int64_t ldx, double* Y, int64_t ldy, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rsrs_solve
 * with the same arguments and results, but no allocation of any kind on the
 * device.  Its two tree-ordered work blocks (n x nrhs elements of the
 * factor's type each, rounded up to 256 bytes) and the launch descriptors
 * live in one fixed library array of 96 MiB per device, which every GPU the
 * library runs on holds until the process ends; a call that needs more
 * (e.g. more than ~6 M FP64 elements n x nrhs) fails with RSRS_E_INVALID
 * and a message giving the bytes needed.  Every call on one GPU shares that
 * array: calls that overlap on a GPU (different streams or threads) race and
 * must be serialised by the caller.  Launches are direct (no graph); the
 * descriptors are copied from pageable host memory on `stream`. */
rsrs_status rsrs_solve_noalloc(const rsrs_factor_t* f, int transpose, int64_t nrhs, const double* F,
                               int64_t ldf, double* U, int64_t ldu, void* stream);

/* Iterative refinement u_{j+1} = u_j + A_approx^{-1} (f - A u_j) with the
 * residual from the black-box product mv (FP64), until
 * max_col ||f - A u||_2 / ||f||_2 <= tol or maxit corrections.  Returns
 * RSRS_OK with *relres = the achieved value and *iters = corrections done
 * (also when maxit is reached; compare *relres with tol).  Synchronises the
 * stream once per step to read the residual norm. */
rsrs_status rsrs_solve_refine(const rsrs_factor_t* f, rsrs_matvec_fn mv, void* user, int64_t nrhs,
                              const double* F, int64_t ldf, double* U, int64_t ldu, double tol,
                              int maxit, double* relres, int* iters, void* stream);

/* GMRES preconditioned by the factorization (Sec. 5, where the factorization
 * is the preconditioner of GMRES and the iteration counts are reported):
 * right preconditioning, GMRES on A M^{-1} y = f with M^{-1} = A_approx^{-1}
 * (rsrs_solve) and u = M^{-1} y, so the residual minimised is the true one,
 * through the black-box product mv (FP64).  Restarted every `restart`
 * (1..64) steps from the true residual; each column is an independent run
 * (columns advance in lock step, 64 at a time, sharing every solve and
 * product); a column stops once its residual estimate is <= tol.  Returns
 * RSRS_OK with *relres = max_col ||f - A u|| / ||f|| (true residual) and
 * *iters = GMRES steps of the longest run, also when maxit is reached
 * (compare *relres with tol).  For operators where the plain refinement of
 * rsrs_solve_refine does not converge (||I - A_approx^{-1} A|| >= 1).
 * Synchronises the stream once per step. */
rsrs_status rsrs_solve_gmres(const rsrs_factor_t* f, rsrs_matvec_fn mv, void* user, int64_t nrhs,
                             const double* F, int64_t ldf, double* U, int64_t ldu, double tol,
                             int restart, int maxit, double* relres, int* iters, void* stream);

/* ------------------------------------------------------------------------
 * Serving (continuous batching).  The method factors once from one set of
 * sketches and then solves many right-hand sides (Sec. 1, Sec. 4.4); the
 * server keeps factorizations resident on the device and serves a stream of
 * requests with two worker threads, each on its own HIP stream:
 *  - solve requests for a resident factor are batched: the oldest pending
 *    request and every other pending request for the same factor, in arrival
 *    order, while the batch has at most max_batch_cols columns, are solved by
 *    one apply of the factor; requests arriving meanwhile join the next
 *    batch.  Each result equals the solve of that request alone (the columns
 *    of a batch are computed independently by the same kernels).
 *  - factor requests (tree, black-box operator, s, seed, options) are
 *    admitted in arrival order when the device bytes they need (estimated
 *    from the schedule: samples, sampling buffers, workspace, stored factor)
 *    fit in hbm_budget next to the resident factors and the factorizations in
 *    flight; they run on the second stream, overlapping with solve batches,
 *    and the factor becomes resident (result id of the ticket).  Requests
 *    admitted together (up to 64, same precision) are factored as one
 *    rsrs_factor_batched batch; if that batch fails, each of its requests is
 *    sampled and factored again alone, so only the faulty one fails.
 * Budget 0 means unlimited.  A resident factor is charged its stored bytes,
 * its permutation and the solve buffers a batch of up to max_batch_cols
 * columns makes it hold (the per-width solve graphs' blocks in the factor's
 * element type); the server's FP64 batch blocks are charged at their size;
 * device memory the library keeps from finished factorizations for reuse
 * counts against the budget when a factor request is admitted and is freed
 * (oldest first) when the request would not fit otherwise.  Device blocks passed to a
 * request must stay valid until its ticket completes; a tree or operator
 * passed to a factor request must outlive it and must not be used by the
 * caller while the request runs.  All functions are thread-safe.
 * ---------------------------------------------------------------------- */
typedef struct {
  int64_t hbm_budget;      /* bytes; 0 = unlimited */
  int64_t max_batch_cols;  /* columns per batched solve (>= 1) */
} rsrs_server_opts;
rsrs_status rsrs_server_create(const rsrs_server_opts* opts, rsrs_server_t** out);
/* Finishes every pending request, then frees the resident factors. */
void rsrs_server_destroy(rsrs_server_t* sv);
/* Makes a factor resident (the server takes ownership); RSRS_E_NOMEM if it
 * does not fit in the budget (ownership stays with the caller then). */
rsrs_status rsrs_server_add_factor(rsrs_server_t* sv, rsrs_factor_t* f, int64_t* id);
/* Served solves of resident factor id are refined (rsrs_solve_refine with
 * the black-box product mv, user) until the batch's max_col relative
 * residual is <= tol or maxit corrections are made; mv = NULL switches back
 * to one-shot solves.  The latency of a request then includes its batch's
 * refinement; the stats report the largest residual a batch ended with.
 * mv and user must outlive the factor's residency. */
rsrs_status rsrs_server_set_refine(rsrs_server_t* sv, int64_t id, rsrs_matvec_fn mv, void* user,
                                   double tol, int maxit);
/* Frees a resident factor once its in-flight batch is done; later requests
 * for it fail with RSRS_E_INVALID. */
rsrs_status rsrs_server_release_factor(rsrs_server_t* sv, int64_t id);
/* Queues U = A_approx^{-1} F for resident factor id (device N x nrhs blocks,
 * user order, FP64); *ticket identifies the request. */
rsrs_status rsrs_server_submit_solve(rsrs_server_t* sv, int64_t id, int64_t nrhs, const double* F,
                                     int64_t ldf, double* U, int64_t ldu, int64_t* ticket);
/* Queues sampling (rsrs_sample with dtype) and factorization (opts); fails at
 * once with RSRS_E_SAMPLES if s is too small and RSRS_E_NOMEM if the request
 * alone exceeds the budget. */
rsrs_status rsrs_server_submit_factor(rsrs_server_t* sv, const rsrs_tree_t* t, rsrs_matvec_fn mv,
                                      void* user, int64_t s, uint64_t seed, int dtype,
                                      const rsrs_factor_opts* opts, int64_t* ticket);
/* Waits for a ticket (timeout_ms < 0: no limit; RSRS_E_TIMEOUT leaves it
 * pending) and returns the request's status; *result receives the resident
 * id of a factor request, *latency_ms submit-to-completion time.  A ticket
 * can be waited for once. */
rsrs_status rsrs_server_wait(rsrs_server_t* sv, int64_t ticket, double timeout_ms, int64_t* result,
                             double* latency_ms);
typedef struct {
  int64_t solves_done, factors_done, batches, cols_done;
  int64_t hbm_in_use, hbm_peak;          /* bytes charged to the budget */
  int64_t resident_factors, queued_solves, queued_factors;
  double solve_p50_ms, solve_p99_ms;     /* submit-to-completion latency */
  double factor_p50_ms, factor_p99_ms;
  int64_t refined_batches, refine_steps; /* batches served with refinement, corrections made */
  double max_relres;                     /* largest residual a refined batch ended with */
} rsrs_server_stats;
/* Counters since creation or the last reset (reset != 0 clears them). */
rsrs_status rsrs_server_get_stats(rsrs_server_t* sv, int reset, rsrs_server_stats* out);
/* ------------------------------------------------------------------------
 * Measurement.  While enabled (process-wide), every kernel launch of the
 * library is bracketed by HIP events recorded on the launch's own stream and
 * accounted under a tag naming the kernel and its form (e.g.
 * "gemm_nt_syrk_64x64").  Each record carries the algorithmic flops and bytes
 * of the launch: 2MNK flops for a full product (half for triangle-restricted
 * forms) and 8(MK + KN + MN [+ MN read when accumulating]) bytes.
 * rsrs_profile_read synchronises the device, fills up to `max` entries and
 * returns the number of tags (or -1 on error); rsrs_profile_reset clears.
 * rsrs_profile_filter restricts recording to tags beginning with `prefix`
 * (NULL or "" records every launch), so that a single kernel can be timed
 * without bracketing every other launch; the string is copied.
 * ---------------------------------------------------------------------- */
typedef struct {
  char tag[48];
  int64_t launches;
  double ms;       /* summed event time of the launches */
  double flops;    /* summed algorithmic flops */
  double bytes;    /* summed algorithmic bytes */
} rsrs_profile_entry;
void rsrs_profile_enable(int on);
void rsrs_profile_reset(void);
void rsrs_profile_filter(const char* prefix);
int rsrs_profile_read(rsrs_profile_entry* out, int max);

#ifdef __cplusplus
}
#endif

#endif /* RSRS_H */
