/*
 * slm.h -- C ABI of libslm.so, the MI355X (gfx950) per-node split search of
 * the accelerated Subspace Learning Machine (Fu et al., "Acceleration of
 * Subspace Learning Machine via Particle Swarm Optimization and Parallel
 * Processing", arXiv 2208.07023).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array arguments are DEVICE pointers owned by the caller, unless marked
 *   [host].  The library never frees, retains or reallocates caller memory.
 * - Matrices are row-major and densely packed.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *   are asynchronous on that stream unless documented as synchronous.
 * - Every call validates its arguments on the host before launching anything;
 *   on failure it returns a non-zero slm_status, launches nothing and leaves a
 *   message for slm_last_error().  Nothing throws across the ABI.
 * - Segments: node j owns rows row_off[j] .. row_off[j+1]-1 of X / Z / target
 *   and particles j*P .. j*P+P-1 of W / x / v / pbest.  Offsets are int64
 *   device arrays; kernels clamp every offset to [0, N] and treat an inverted
 *   range as empty, so bad offsets cannot cause out-of-bounds accesses.
 * - Sizes: N < 2^31 rows, 1 <= D <= 4096, 1 <= P <= 4096, n_nodes >= 0.
 */
#ifndef SLM_H
#define SLM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SLM_OK = 0,
  SLM_E_INVALID = 1,     /* null pointer, negative size, bad enum value     */
  SLM_E_SHAPE = 2,       /* inconsistent or out-of-range sizes              */
  SLM_E_DTYPE = 3,       /* unsupported dtype or dtype combination          */
  SLM_E_NOMEM = 4,       /* workspace too small / device allocation failed  */
  SLM_E_HIP = 5,         /* a HIP runtime call failed (message has details) */
  SLM_E_UNSUPPORTED = 6  /* valid request this build does not implement     */
} slm_status;

typedef enum { SLM_F32 = 0, SLM_BF16 = 1, SLM_F64 = 2, SLM_I32 = 3 } slm_dtype;

/* Split criteria (the loss of the best threshold of a projected feature,
 * Sec. III-B): weighted Gini impurity, weighted base-2 entropy, weighted
 * squared error.  The loss of a split is the children's impurity weighted by
 * their sample counts and divided by the node's count. */
typedef enum { SLM_GINI = 0, SLM_ENTROPY = 1, SLM_MSE = 2 } slm_criterion;

/* Layout of a projected-feature matrix Z (N rows, P particles per node):
 *   SLM_Z_ROWS   : row-major [N, P]; Z[i, p] at i * P + p.
 *   SLM_Z_TILED  : particle-tiled [ceil(P/32), N, 32]; Z[i, p] at
 *                  ((p / 32) * N + i) * 32 + p % 32.  Each 32-particle tile
 *                  is one contiguous [N, 32] block, and the buffer holds
 *                  ceil(P/32) * 32 * N floats; columns p >= P of the last
 *                  tile are not written.
 *   SLM_Z_TILED8 : the same with 8-particle tiles, [ceil(P/8), N, 8]; Z[i, p]
 *                  at ((p / 8) * N + i) * 8 + p % 8 (ceil(P/8) * 8 * N floats).
 *                  A scan work-group of 8 particles streams whole 32-byte
 *                  rows of one tile instead of a quarter of each 128-byte
 *                  row.  The kernels address the four tiles of a
 *                  32-particle block over a chunk of up to 65536 rows with
 *                  32-bit offsets, so 96 N + 32 * 65600 + 124 < 2^31 bytes
 *                  is required (N up to 22347753); larger N is refused with
 *                  SLM_E_INVALID.
 *   SLM_Z_TILED8_BF16 : SLM_Z_TILED8 with bfloat16 elements (2 bytes each:
 *                  ceil(P/8) * 8 * N of them; N up to 44717374 by the same
 *                  rule in 2-byte elements), each the float32 projection
 *                  rounded to the nearest bfloat16 (ties to even), and zmin /
 *                  zmax the min / max of the stored values; columns p >= P
 *                  of the last tile may be written (with zeros).  The storage of
 *                  a screening pass: slm_project writes it with the
 *                  streaming kernel (X BF16 with D <= 256, or X and W F32
 *                  with 64 < D <= 128; other shapes return
 *                  SLM_E_UNSUPPORTED), slm_split_scan reads it
 *                  for classification histogram scans (bins > 0, Gini or
 *                  entropy; otherwise SLM_E_UNSUPPORTED). */
typedef enum {
  SLM_Z_ROWS = 0,
  SLM_Z_TILED = 1,
  SLM_Z_TILED8 = 2,
  SLM_Z_TILED8_BF16 = 3
} slm_z_layout;

/* Library version string (static storage). */
const char *slm_version(void);

/* Message of the last failed call on this thread ("" if none).  Valid until
 * the next slm_* call on the same thread. */
const char *slm_last_error(void);

/* ------------------------------------------------------------------------
 * slm_project -- projected features Z = X W^T per node (Sec. II-A, Eq. (1)).
 *
 *   Z[i, p] = sum_d X[i, d] * W[j*P + p, d]   for every row i of node j,
 *   zmin[j*P + p] = min over node j's rows of Z[i, p], zmax likewise.
 *
 * (x_dtype, w_dtype) is (F32, F32), (BF16, BF16) or (BF16, F32).  Products
 * are accumulated in FP32 on the matrix cores: FP32 MFMA when W is F32 (a
 * BF16 X is widened exactly), BF16 MFMA when both are BF16 (the screening
 * projection; each 16-term block of the dot product is summed inside one
 * MFMA, so the rounding order differs from a sequential FP32 sum).  For F32
 * W every element of Z is the same sequence of MFMA steps whatever P and the
 * node layout, so a column recomputed alone is bit-identical.  Z is FP32 in
 * z_layout (slm_z_layout; [N, P] for SLM_Z_ROWS).  Rows outside every
 * segment are not written.  For an empty node zmin = +inf, zmax = -inf.
 * A -0.0 projection is recorded in zmin/zmax as +0.0 (the two compare equal
 * and give identical bin edges).  Asynchronous.
 * ------------------------------------------------------------------------ */
slm_status slm_project(const void *X, int32_t x_dtype, int64_t N, int32_t D,
                       const void *W, int32_t w_dtype,
                       const int64_t *row_off, int32_t n_nodes, int32_t P,
                       float *Z, int32_t z_layout, float *zmin, float *zmax, void *stream);

/* ------------------------------------------------------------------------
 * slm_split_scan -- best threshold of every projected feature (Sec. II-A,
 * Eqs. (3)-(4): samples with z >= t go right, z < t go left; Sec. III-B: the
 * loss of a direction is the loss of its best threshold).
 *
 * Z is read in z_layout (slm_z_layout), as written by slm_project.
 * bins = 0: exact scan.  Candidates are the boundaries between consecutive
 *   distinct sorted values of a node's column; the threshold is the smallest
 *   value sent right and best_split is the number of samples sent left.
 *   Synchronous (reads row_off back); nodes must hold <= 8192 rows.
 * bins in [2, 256]: histogram scan.  With r = zmax - zmin and
 *   delta = r / bins (float32, each operation rounded once), the edges are
 *   e_j = zmin + j * delta for j = 1..bins-1 and a sample's bin is the number
 *   of edges <= z.  Split b (1..bins-1) sends bins < b left; threshold = e_b;
 *   best_split = b.  zmin/zmax are those written by slm_project.
 *   Asynchronous.
 * Ties between candidates go to the smallest split; a candidate needs a
 * sample on each side.  Without one: best_split = -1, best_loss = +inf,
 * threshold = +inf.
 *
 * target: I32 labels in [0, K) for SLM_GINI / SLM_ENTROPY (rows with labels
 *   outside [0, K) are ignored), 2 <= K <= 16; F64 y with K = 0 for SLM_MSE.
 * Outputs [n_nodes*P]: best_split (i32), best_loss (f64), threshold (f32).
 * hist_out (optional, histogram mode): per (node, particle) the bin counts,
 *   [n_nodes*P, bins, K] u32 for classification or [n_nodes*P, bins] for MSE.
 * sums_out (optional, MSE histogram mode): [n_nodes*P, bins, 2] f64
 *   (sum y, sum y^2 per bin; FP64 atomics, last bits order-dependent).
 * workspace: device scratch of at least slm_split_scan_workspace(...) bytes.
 *   It must be zero-filled before its first use and not modified by the
 *   caller between calls: every call leaves it zero-filled again, so one
 *   workspace can be reused by consecutive calls on one stream.
 * ------------------------------------------------------------------------ */
size_t slm_split_scan_workspace(int64_t N, int32_t n_nodes, int32_t P, int32_t bins,
                                int32_t K, int32_t crit);
slm_status slm_split_scan(const float *Z, int32_t z_layout, const float *zmin, const float *zmax,
                          const void *target, int32_t t_dtype, int32_t K, int64_t N,
                          const int64_t *row_off, int32_t n_nodes, int32_t P,
                          int32_t bins, int32_t crit,
                          int32_t *best_split, double *best_loss, float *threshold,
                          uint32_t *hist_out, double *sums_out,
                          void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * slm_split_scan_noalloc -- slm_split_scan's histogram scan for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the same kernels and outputs, with the
 * accumulator in the library's own per-GPU scratch array instead of a caller
 * workspace.  It allocates nothing and calls no allocating routine.
 *
 * Arguments as slm_split_scan without workspace / ws_bytes; bins in 2..256
 * (the exact scan needs no scratch: bins = 0 returns SLM_E_UNSUPPORTED).
 * The scratch holds slm_split_scan_noalloc_max_bytes() bytes (128 MiB) per
 * GPU, kept until the process ends; a scan whose slm_split_scan_workspace
 * exceeds it returns SLM_E_NOMEM before any launch.  The array is cleared on
 * the call's stream at the first call on a device (and after a failed call);
 * every completed scan leaves it zero.  All calls on one GPU share the array:
 * calls that overlap in time on one GPU (different streams, threads or
 * processes' graphs replayed concurrently) race and give wrong results.
 * Asynchronous.
 * ------------------------------------------------------------------------ */
size_t slm_split_scan_noalloc_max_bytes(void);
slm_status slm_split_scan_noalloc(const float *Z, int32_t z_layout, const float *zmin,
                                  const float *zmax, const void *target, int32_t t_dtype,
                                  int32_t K, int64_t N, const int64_t *row_off, int32_t n_nodes,
                                  int32_t P, int32_t bins, int32_t crit, int32_t *best_split,
                                  double *best_loss, float *threshold, uint32_t *hist_out,
                                  double *sums_out, void *stream);

/* ------------------------------------------------------------------------
 * slm_evaluate -- one swarm evaluation fused: the projected features of
 * slm_project (Sec. II-A, Eq. (1)) binned and scanned as by slm_split_scan
 * (histogram mode, Sec. II-A Eqs. (3)-(4), Sec. III-B) without ever storing Z.
 * A first pass computes zmin / zmax (written to the caller's arrays); the
 * second recomputes each projection on the matrix cores and bins it from the
 * registers.  Every z is the float32 number slm_project(..., SLM_Z_TILED)
 * would store, so zmin / zmax, best_split, best_loss and threshold are
 * identical to slm_project followed by slm_split_scan.
 * X [N, D] and W [n_nodes*P, D] F32 with D <= 64; labels I32 with
 * 2 <= K <= 4; crit SLM_GINI or SLM_ENTROPY; 2 <= bins <= 256.  Other
 * combinations return SLM_E_UNSUPPORTED (use the two calls).  workspace as
 * for slm_split_scan (slm_split_scan_workspace bytes, zero-filled before
 * first use, left zero-filled).  Asynchronous.
 * ------------------------------------------------------------------------ */
slm_status slm_evaluate(const float *X, int64_t N, int32_t D, const float *W,
                        const int64_t *row_off, int32_t n_nodes, int32_t P,
                        const int32_t *labels, int32_t K, int32_t bins, int32_t crit, float *zmin,
                        float *zmax, int32_t *best_split, double *best_loss, float *threshold,
                        void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * slm_pso_init -- initial swarm of every node (Sec. III-A: particles start
 * at random positions; this build draws N(0, I) directions and scales them to
 * unit norm, Eq. (2), with zero velocity).
 *
 * For particle p of node j, dimension pair m = d/2 uses one Philox4x32-10
 * call (key = seed; counter = (p*ceil(D/2) + m, 0xFFFFFFFF, node_id[j],
 * tree)); u1 = (w0 + 1/2) 2^-32, u2 = w1 2^-32 and the pair is
 * sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2).  Rows are then divided by their
 * norm (squared norm summed in dimension order).
 * Writes x, v = 0, pbest = x, pbest_loss = +inf, gbest = x of particle 0,
 * gbest_loss = +inf, gbest_p = -1, and W_out = x rounded to w_dtype (F32 or
 * BF16, round to nearest even).  Asynchronous.
 * ------------------------------------------------------------------------ */
slm_status slm_pso_init(double *x, double *v, double *pbest, double *pbest_loss,
                        double *gbest, double *gbest_loss, int32_t *gbest_p,
                        const int32_t *node_id, int32_t n_nodes, int32_t P, int32_t D,
                        uint64_t seed, uint32_t tree, void *W_out, int32_t w_dtype,
                        void *stream);

/* ------------------------------------------------------------------------
 * slm_pso_init_subspace -- slm_pso_init with each node's swarm started in
 * the span of n_sel of its input dimensions (Alg. 2: the swarm runs in the
 * node's top n channels).  sel [n_nodes, n_sel] ([device] int32) lists the
 * dimensions of node j in row j; the same normals as slm_pso_init are drawn,
 * those of unlisted dimensions are replaced by zero before each row is
 * divided by its norm.  The swarm steps keep the unlisted coordinates at zero
 * (x, v and the bests are zero there).  1 <= n_sel <= D; indices outside
 * [0, D) are ignored.  Other arguments and outputs as slm_pso_init.
 * ------------------------------------------------------------------------ */
slm_status slm_pso_init_subspace(double *x, double *v, double *pbest, double *pbest_loss,
                                 double *gbest, double *gbest_loss, int32_t *gbest_p,
                                 const int32_t *node_id, int32_t n_nodes, int32_t P, int32_t D,
                                 uint64_t seed, uint32_t tree, void *W_out, int32_t w_dtype,
                                 const int32_t *sel, int32_t n_sel, void *stream);

/* ------------------------------------------------------------------------
 * slm_dft_select -- discriminant feature test of every node and its top n
 * channels (Sec. II-A: the DFT selects the threshold of a 1-D subspace;
 * Alg. 2: run the DFT for the node, select the top n channels).
 *
 * The DFT loss of input feature d of node j is the loss of the best
 * threshold of x_d over the node's rows: x_d is the projection on the unit
 * vector e_d, so it is binned and scanned exactly as slm_split_scan treats a
 * projected feature (histogram edges over the node's [min, max] of x_d, or
 * the exact scan with bins = 0; +inf when no threshold splits the node).
 * X [N, D] F32 row-major, row_off [n_nodes + 1] (int64, non-decreasing),
 * target: I32 labels (K classes, Gini / entropy) or F64 y (SLM_MSE, K = 0);
 * all [device].  Outputs [device]: dft_loss [n_nodes, D]; sel [n_nodes, n]:
 * the n features of smallest loss of each node, ascending by (loss, index).
 * workspace: slm_dft_select_workspace bytes ([device], zero-filled before
 * first use and left zero-filled; it holds the scan's accumulators and the
 * per-node column min / max).  1 <= n <= D <= 4096; the exact scan needs
 * nodes of at most 8192 rows.  Asynchronous.
 * ------------------------------------------------------------------------ */
size_t slm_dft_select_workspace(int64_t N, int32_t D, int32_t n_nodes, int32_t bins, int32_t K,
                                int32_t crit);
slm_status slm_dft_select(const float *X, int64_t N, int32_t D, const int64_t *row_off,
                          int32_t n_nodes, const void *target, int32_t t_dtype, int32_t K,
                          int32_t bins, int32_t crit, int32_t n, double *dft_loss, int32_t *sel,
                          void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * slm_ps_candidates -- candidate directions of the probabilistic search
 * (Sec. II-B, Eqs. (5)-(8)), iteration t, for every node.
 *
 * Particle p of node j combines the R features ranks[j R .. j R + R) (most
 * discriminant first, e.g. sel of slm_dft_select) with integer
 * coefficients.  One Philox4x32-10 call per (p, rank d), key = seed,
 * counter = (p R + d, 0x40000000 + t, node_id[j], tree); u24(w) = (w >> 8)
 * 2^-24.  Rank d is used iff u24(w0) < pd[d]; its coefficient is k + 1 if
 * k < m, else -(k - m + 1), with k = floor(u24(w1) 2m), m = amax[d] >= 1.  A
 * particle that uses no rank takes +1 on rank 1.  x[j P + p] = c / ||c||
 * (FP64, every coordinate written, zeros outside the used ranks) and W_out =
 * x rounded to w_dtype (F32 or BF16).  ranks [n_nodes, R] int32, pd [R]
 * float64, amax [R] int32, node_id [n_nodes], x [n_nodes P, D]: all
 * [device].  1 <= R <= min(D, 64).  Asynchronous.
 * ------------------------------------------------------------------------ */
slm_status slm_ps_candidates(double *x, void *W_out, int32_t w_dtype, const int32_t *node_id,
                             int32_t n_nodes, int32_t P, int32_t D, const int32_t *ranks,
                             int32_t R, const double *pd, const int32_t *amax, uint64_t seed,
                             uint32_t tree, uint32_t t, void *stream);

/* ------------------------------------------------------------------------
 * slm_ps_tables -- the tables slm_ps_candidates draws from (Sec. II-B,
 * Eq. (8): the coefficient range falls exponentially with the rank):
 *   A_d = alpha0 exp(-alpha d), alpha = ln(alpha0) / (R - 1)  (0 if R = 1),
 * for ranks d = 0 .. R-1, so A falls from alpha0 at the first rank to 1 at
 * the last; pd[d] = A_d / alpha0 (selection probability), amax[d] =
 * max(1, floor(A_d + 1e-9)) (coefficient range).  FP64 on the device.
 * pd [device] f64 [R], amax [device] int32 [R]; 1 <= R <= 64; alpha0
 * finite, >= 1.  Asynchronous.
 * ------------------------------------------------------------------------ */
slm_status slm_ps_tables(int32_t R, double alpha0, double *pd, int32_t *amax, void *stream);

/* ------------------------------------------------------------------------
 * slm_pso_step -- one synchronous swarm step for every node (Sec. III-A,
 * Eqs. (11)-(12), Alg. 1).
 *
 * (1) Bests from `loss` (the losses of the current positions): pbest_p <- x_p
 *     iff loss_p < pbest_loss_p; then p* = argmin_p g_p (lowest p on ties)
 *     replaces the global best iff g_p* < gbest_loss, where g = gloss if
 *     given (the losses eligible for the global best, see slm_screen_merge)
 *     and g = loss otherwise.  When split/thr are
 *     given, the winner's split and threshold are copied to gbest_split /
 *     gbest_thr.
 * (2) If move != 0: for every particle, with r1, r2 drawn per dimension from
 *     Philox4x32-10 (key = seed, counter = (p*ceil(D/2) + d/2, iter,
 *     node_id[j], tree); words 0,1 -> r1,r2 of dimension 2m, words 2,3 -> of
 *     2m+1; r = (w >> 8) 2^-24):
 *       v <- ((omega v) + ((c1 r1)(pbest - x))) + ((c2 r2)(gbest - x))
 *       x <- (x + v) / ||x + v||   (x kept if the norm is 0)
 *     each operation rounded once in FP64; W_out <- x rounded to w_dtype.
 * Shapes: x, v, pbest [n_nodes*P, D]; pbest_loss, loss, gloss [n_nodes*P];
 * gbest [n_nodes, D]; gbest_loss, gbest_p, node_id [n_nodes].
 * split, thr, gbest_split, gbest_thr: optional ([n_nodes*P] / [n_nodes]).
 * Asynchronous.
 * ------------------------------------------------------------------------ */
slm_status slm_pso_step(double *x, double *v, double *pbest, double *pbest_loss,
                        double *gbest, double *gbest_loss, int32_t *gbest_p,
                        const double *loss, const double *gloss,
                        const int32_t *split, const float *thr,
                        int32_t *gbest_split, float *gbest_thr,
                        const int32_t *node_id, int32_t n_nodes, int32_t P, int32_t D,
                        double omega, double c1, double c2, uint64_t seed, uint32_t tree,
                        uint32_t iter, int32_t move, void *W_out, int32_t w_dtype,
                        void *stream);

/* ------------------------------------------------------------------------
 * slm_apso_step -- one step of the adaptive swarm (APSO, Sec. III-B) for a
 * batch of nodes: the bests exactly as slm_pso_step, then per node the
 * evolutionary state estimation and parameter change, then the move of
 * Eqs. (11)-(12) with the node's own omega, c1, c2.
 *   dist [n_nodes * P] (out): d_i, the mean distance of particle i to the
 *     other particles of its node;
 *   f [n_nodes] (out): (d_g - d_min) / (d_max - d_min), g = gbest_p (0 if
 *     negative); 0 when d_max = d_min;
 *   state [n_nodes] (in/out): 1 exploration, 2 exploitation, 3 convergence,
 *     4 jumping-out (1 before the first move); the previous state is kept
 *     while its fuzzy membership of f stays positive, else the state of
 *     largest membership (lower state on ties);
 *   par [n_nodes * 3] (in/out): omega, c1, c2 (c1 = c2 = 2 before the first
 *     move); omega = 1 / (1 + 1.5 exp(-2.6 f)); c1, c2 move by delta ~
 *     U[0.05, 0.1] (half of it in states 2 and 3) in the state's directions,
 *     are clamped to [1.5, 2.5] and scaled to sum 4 when above it;
 *   worst [n_nodes] (out): the particle of highest loss (NaN as +inf, lowest
 *     index on ties);
 *   elite [n_nodes * D] (out, state 3 only): one coordinate (uniform) of the
 *     global best moved by 2 sigma N(0, 1), sigma = 1 - 0.9 iter / T, scaled
 *     to unit norm; it replaces the worst particle after the move, with zero
 *     velocity;
 *   sel [device, n_nodes * n_sel] or NULL (n_sel 0): the coordinates each
 *     node's swarm lives in (its top DFT channels, Alg. 2); the elite step
 *     then perturbs sel[j n_sel + floor(w n_sel / 2^32)] instead of
 *     coordinate floor(w D / 2^32).
 * The draws of move iter use Philox counters (0 | 1, 0x20000000 + iter, node
 * id, tree).  P in 2..4096.  workspace [device] >= slm_apso_workspace(n_nodes,
 * P) bytes (partial distance sums).  Other arguments as slm_pso_step (with
 * move = 1 and no screening).  Asynchronous.
 * ------------------------------------------------------------------------ */
size_t slm_apso_workspace(int32_t n_nodes, int32_t P);
slm_status slm_apso_step(double *x, double *v, double *pbest, double *pbest_loss, double *gbest,
                         double *gbest_loss, int32_t *gbest_p, const double *loss,
                         const int32_t *node_id, int32_t n_nodes, int32_t P, int32_t D,
                         uint64_t seed, uint32_t tree, uint32_t iter, uint32_t T, int32_t *state,
                         double *par, double *dist, double *f, int32_t *worst, double *elite,
                         const int32_t *sel, int32_t n_sel, void *workspace, size_t ws_bytes,
                         void *W_out, int32_t w_dtype, void *stream);

/* ------------------------------------------------------------------------
 * Mixed-precision screening of one swarm evaluation.  The paper scores a
 * direction by the loss of its best threshold (Sec. III-B) and names faster
 * projection search on high-dimensional data as open (Sec. VI); screening
 * scores every particle on the BF16 projection (slm_project with BF16 X and
 * W, slm_split_scan), re-scores the k best of each node on the FP32
 * projection of the same BF16 X, and merges:
 *
 * slm_screen_select: sel[j*k + s] = index of the particle of node j with the
 *   s-th smallest loss (ascending by (loss, index); -0.0 equals +0.0).
 *   loss [n_nodes*P] f64, sel [n_nodes*k] i32, 1 <= k <= P.  Asynchronous.
 * slm_screen_gather: W32[j*k + s, :] = float32(x[j*P + sel[j*k + s], :]),
 *   the FP32 directions of the re-projection ([n_nodes*k, D]).  Asynchronous.
 * slm_screen_merge: for the selected particles p = sel[j*k + s]:
 *   loss/split/thr[j*P + p] <- loss_r/split_r/thr_r[j*k + s] (the re-scored
 *   results, computed with P = k on W32) and gloss[j*P + p] <- loss_r; every
 *   other particle keeps its screened loss/split/thr and gets
 *   gloss = +inf.  gloss is the eligibility input of slm_pso_step: only
 *   re-scored particles can become the global best.  Asynchronous.
 * ------------------------------------------------------------------------ */
slm_status slm_screen_select(const double *loss, int32_t n_nodes, int32_t P, int32_t k,
                             int32_t *sel, void *stream);
slm_status slm_screen_gather(const double *x, const int32_t *sel, int32_t n_nodes, int32_t P,
                             int32_t k, int32_t D, float *W32, void *stream);
slm_status slm_screen_merge(const int32_t *sel, const double *loss_r, const int32_t *split_r,
                            const float *thr_r, int32_t n_nodes, int32_t P, int32_t k,
                            double *loss, int32_t *split, float *thr, double *gloss,
                            void *stream);

/* ------------------------------------------------------------------------
 * slm_grow_tree -- one binary SLM tree (Sec. III-B, Alg. 2) grown breadth
 * first, all frontier nodes of a depth searched together.
 *
 * A node is split when depth < max_depth, it holds >= min_node rows and it is
 * impure (classification: impurity > 0; regression: targets not all equal).
 * Its swarm (P particles, T moves, T+1 evaluations; keyed by the node's heap
 * id: root 0, children 2j+1 / 2j+2) searches directions; the split is kept
 * iff the global-best loss is strictly below the node's impurity.  Rows with
 * a^T x >= t go to the right child.  Leaves hold class counts or the mean.
 *
 * X [N, D] F32 (BF16 with precision = 1); target as in slm_split_scan.
 * precision = 1 runs every evaluation as a screened one (BF16 projection of
 * all P particles, FP32 re-scoring of the best rescore_k, see
 * slm_screen_select); the partition projects on the FP32 split direction,
 * exactly as the re-scoring does, so the stored threshold splits the rows
 * the way the re-scored loss was computed.
 * Output arrays are [host], sized for max_nodes nodes; nodes are numbered in
 * breadth-first order (left child before right).  Synchronous: the host
 * reads a few bytes of frontier state back once per depth.
 * workspace: device scratch >= slm_grow_tree_workspace(prm, N, D) bytes; its
 * contents on entry are ignored.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t crit;        /* slm_criterion                                 */
  int32_t K;           /* classes (0 for SLM_MSE)                       */
  int32_t max_depth;
  int32_t min_node;
  int32_t P;           /* particles per node                            */
  int32_t T;           /* moves (T+1 evaluations)                       */
  int32_t bins;        /* 2..256 (histogram scan); 0 = exact scan, which
                          takes nodes of at most 8192 rows: slm_grow_tree,
                          slm_grow_forest and slm_boost with N > 8192
                          return SLM_E_UNSUPPORTED (their workspace
                          queries 0) before any launch                  */
  int32_t precision;   /* 0 = FP32 projection; 1 = BF16 screen + FP32
                          re-scoring of the best rescore_k per node      */
  int32_t rescore_k;   /* 1..P, used with precision = 1                 */
  double omega, c1, c2;
  uint64_t seed;
  uint32_t tree;
  int32_t use_graph;   /* 1 = replay each depth's swarm loop as a HIP graph */
  int32_t profile;     /* 1 = time every projection / scan / step launch with
                          HIP events (fills timing[3..7]; no graph replay)    */
  int32_t proposal;    /* 0 = random start (Sec. III-A); 1 = learned start:
                          the first min(n_seeds, P) particles of every node
                          start at the network's seeds (slm_node_stats,
                          slm_mlp_forward with BF16 inference,
                          slm_proposal_seeds); classification only;
                          2 = probabilistic search instead of the swarm
                          (Sec. II-B): every searched node ranks its
                          features by DFT loss (slm_dft_select), and each of
                          the T + 1 iterations evaluates P new candidates
                          (slm_ps_candidates) and keeps the best; float32
                          data only                                        */
  int32_t n_seeds;     /* M seeds per node (network output M * D)        */
  int32_t mlp_hidden;  /* hidden width H (network input (K + 1) * D)     */
  const float *mlp;    /* [device] packed parameters, slm_mlp_param_count */
  int32_t dft_top_n;   /* 0 or D: the swarm searches all D dimensions;
                          1..D-1: every searched node first runs the DFT
                          (slm_dft_select) and its swarm starts in the span
                          of its top dft_top_n channels (Alg. 2);
                          float32 data (precision 0) only                  */
  const double *ps_pd;     /* proposal 2: [device] selection probability per
                              rank (slm_ps_candidates)                      */
  const int32_t *ps_amax;  /* proposal 2: [device] coefficient range per rank */
  int32_t ps_R;            /* proposal 2: ranks combined, 1..min(D, 64)     */
  int32_t apso;            /* 1 = adaptive swarm (slm_apso_step) in place of
                              the plain one (Sec. III-B); P >= 2, not with
                              proposal 2                                    */
} slm_tree_params;

#define SLM_TIMING_SLOTS 12

typedef struct {
  int32_t max_nodes;   /* capacity of every array below                 */
  int32_t n_nodes;     /* [out] nodes written                           */
  float *w;            /* [max_nodes, D] split direction (FP32 image)   */
  float *thr;          /* [max_nodes] threshold (+inf for leaves)       */
  int32_t *left, *right;     /* child indices, -1 for leaves           */
  double *leaf;        /* [max_nodes, max(K,1)] class counts or mean    */
  int64_t *n;          /* rows per node                                 */
  double *impurity;    /* node impurity                                 */
  double *split_loss;  /* global-best loss (+inf if not searched)       */
  int32_t *depth, *heap;
  double *timing;      /* optional [SLM_TIMING_SLOTS = 12]: [0] whole
                          call, [1] swarm loops, [2] partitions (ms); with
                          profile = 1 also the summed kernel times of
                          [3] projections, [4] scans, [5] swarm steps (ms),
                          [6] projection launches, [7] scan launches, and
                          for screened evaluations (precision = 1) of the
                          FP32 re-scoring: [8] projections, [9] scans (ms),
                          [10] / [11] their launches ([3] / [4] then hold
                          the screening launches only)                   */
  int64_t *sample_splits;    /* optional [2]: [0] sum over evaluations of
                                n_j * P (screened ones with precision = 1),
                                [1] re-scored n_j * rescore_k (else 0)      */
  float *stats;        /* optional [max_nodes, (K + 1) D]: node statistics
                          (slm_node_stats) of every searched node          */
  float *sigma;        /* optional [max_nodes, D], with stats               */
} slm_tree_out;

size_t slm_grow_tree_workspace(const slm_tree_params *prm, int64_t N, int32_t D);
slm_status slm_grow_tree(const void *X, int32_t x_dtype, int64_t N, int32_t D,
                         const void *target, int32_t t_dtype,
                         const slm_tree_params *prm, void *workspace, size_t ws_bytes,
                         slm_tree_out *out, void *stream);

/* ------------------------------------------------------------------------
 * slm_autotune_set -- launch plans of the tree builds (Alg. 2's per-depth
 * batches): which particle tile and chunk length the histogram scan uses,
 * and how many particle blocks per wave and which work-group order the
 * projection uses, per shape class (kernel, rows, nodes, P, D, bins,
 * classes, criterion; keyed by the GPU architecture).  A plan changes no
 * result of a classification tree (integer counts, the same MFMA sequence
 * per element); a regression scan's FP64 bin sums may change in the last
 * bits with the chunking.
 *   mode 0: the kernels' fitted rules only;
 *   mode 1 (the default): measured plans where the cache holds one, else the
 *     rules; the cache is read from `path`, or (NULL) from
 *     plans_<arch>.json beside the library;
 *   mode 2: as 1, and every depth of a tree build whose launch shapes have no
 *     plan first times each shape's candidate plans with HIP events on the
 *     build's stream (one eager evaluation, not captured) and keeps the
 *     fastest; the cache is then written to `path` (required).
 * Changing the plans makes the next tree builds capture new graphs.  Not
 * thread-safe with concurrent tree builds.  slm_autotune_plans returns the
 * number of cached plans.
 * ------------------------------------------------------------------------ */
slm_status slm_autotune_set(int32_t mode, const char *path);
int32_t slm_autotune_plans(void);

/* ------------------------------------------------------------------------
 * slm_predict -- route rows through a tree (Sec. II-A, Eqs. (3)-(4)):
 * right iff float32(w . x) >= thr, the dot product accumulated in FP32 in
 * dimension order.  Tree arrays are device copies of slm_tree_out's w, thr,
 * left, right (n_tree nodes).  leaf_out [N] receives the index of the leaf
 * reached.  Asynchronous.
 * ------------------------------------------------------------------------ */
slm_status slm_predict(const float *w, const float *thr, const int32_t *left,
                       const int32_t *right, int32_t n_tree, int32_t D,
                       const float *X, int64_t N, int32_t *leaf_out, void *stream);

/* ------------------------------------------------------------------------
 * slm_grow_forest -- SLM/SLR Forest (Sec. V; bagging after random forests):
 * n_trees trees, tree b grown as slm_grow_tree grows one, with tree id
 * prm->tree + b, on a bootstrap sample of the N rows (bootstrap = 1) or on all
 * N rows (bootstrap = 0).
 *
 * Bootstrap draw i of tree b (i = 0 .. N-1) is word (i mod 4) of Philox4x32-10
 * with counter (i div 4, 0x80000000, 0xFFFFFFFF, prm->tree + b) and the seed
 * as key, mapped to row floor(w * N / 2^32); the sample keeps draw order.
 * All trees grow together: each depth's frontier nodes of every tree are
 * searched in one swarm loop (rows of tree b sit at b*N .. (b+1)*N - 1 of a
 * gathered copy of X in the workspace).
 *
 * X, target, prm: as slm_grow_tree.  n_trees in 1..65535, n_trees * N < 2^31.
 * out ([host], max_nodes for the whole forest): nodes of all trees, numbered
 * breadth first over the forest (roots are nodes 0 .. n_trees-1; each depth's
 * nodes follow tree order); child indices are global.  tree_of ([host]
 * [max_nodes] or NULL) receives every node's tree b.  sample_idx ([device]
 * int32 [n_trees, N] or NULL) receives the drawn rows (bootstrap = 1).
 * workspace: device scratch >= slm_grow_forest_workspace(prm, N, D, n_trees)
 * bytes (about n_trees times a tree's).  Synchronous.
 * ------------------------------------------------------------------------ */
size_t slm_grow_forest_workspace(const slm_tree_params *prm, int64_t N, int32_t D,
                                 int32_t n_trees);
slm_status slm_grow_forest(const void *X, int32_t x_dtype, int64_t N, int32_t D,
                           const void *target, int32_t t_dtype, const slm_tree_params *prm,
                           int32_t n_trees, int32_t bootstrap, void *workspace, size_t ws_bytes,
                           int32_t *sample_idx, slm_tree_out *out, int32_t *tree_of,
                           void *stream);

/* ------------------------------------------------------------------------
 * slm_forest_predict -- the forest's output for rows X [device, N, D] F32
 * (Sec. V): every tree routes each row from its root as slm_predict does
 * (right iff float32(w . x) >= thr, FP32 accumulation in dimension order).
 * Classification (K in 2..16): each tree votes for its leaf's majority class
 * (first maximum of the leaf's class counts) and out (int32 [N]) receives the
 * class with most votes, the smallest on ties.  Regression (K = 0): out (f64
 * [N]) receives the mean of the trees' leaf values, summed in tree order.
 * Tree arrays are device copies of a forest's w [n_nodes, D], thr, left,
 * right, leaf [n_nodes, max(K, 1)]; roots [device, n_trees] index the roots
 * (a root outside 0 .. n_nodes-1 gives leaf -1: no vote, or a NaN mean).
 * leaf_ids [device] int32 [n_trees, N] receives the leaf of every (tree, row).
 * Asynchronous.
 * ------------------------------------------------------------------------ */
slm_status slm_forest_predict(const float *w, const float *thr, const int32_t *left,
                              const int32_t *right, const double *leaf, int32_t n_nodes,
                              const int32_t *roots, int32_t n_trees, int32_t D, int32_t K,
                              const float *X, int64_t N, int32_t *leaf_ids, void *out,
                              void *stream);

/* ------------------------------------------------------------------------
 * slm_boost -- SLM/SLR Boost (Sec. V; gradient boosting after XGBoost):
 * n_rounds rounds of SLR trees (prm: crit SLM_MSE, K 0, precision 0) fitted
 * to negative gradients, each added with shrinkage lr.
 *   regression (n_classes = 0, target F64 [N]): F0 = mean(y); round m grows
 *     one tree (tree id prm->tree + m) on r = y - F and sets F += lr * h(x);
 *   classification (n_classes = K in 2..16, target I32 labels): F0 = 0;
 *     round m computes p = softmax(F) (FP64, maximum subtracted) and grows K
 *     trees together (tree k: id prm->tree + m*K + k, on the K-fold copy of
 *     X with targets 1{y = k} - p_k), then F_k += lr * h_k(x).
 * h(x) is the leaf mean each training row reaches under the prediction rule
 * (right iff float32(w . x) >= thr, FP32 accumulation in dimension order).
 * X [device, N, D] F32.  F [device] f64 [N, max(K, 1)] receives the final
 * training scores; F0 [host] f64 [max(K, 1)] the initial ones.  out ([host],
 * max_nodes for all rounds): the trees in round order (round m's K trees
 * together, roots first), child indices global; tree_of ([host] or NULL)
 * receives m * max(K, 1) + k per node.  workspace: device scratch >=
 * slm_boost_workspace(prm, N, D, n_classes) bytes.  Synchronous.
 * ------------------------------------------------------------------------ */
size_t slm_boost_workspace(const slm_tree_params *prm, int64_t N, int32_t D, int32_t n_classes);
slm_status slm_boost(const float *X, int64_t N, int32_t D, const void *target, int32_t t_dtype,
                     int32_t n_classes, const slm_tree_params *prm, int32_t n_rounds, double lr,
                     void *workspace, size_t ws_bytes, double *F, double *F0, slm_tree_out *out,
                     int32_t *tree_of, void *stream);

/* ------------------------------------------------------------------------
 * slm_boost_scores -- the scores of a boosted model for rows X (Sec. V):
 * F(x) = F0 + lr * sum over rounds m of h_m(x), added round by round in the
 * order slm_boost accumulated its training scores (so the training rows get
 * slm_boost's F bit for bit).  h_m,k(x) is the leaf mean that row x reaches
 * in tree m * max(K, 1) + k (right iff float32(w . x) >= thr, FP32
 * accumulation in dimension order).
 * Tree arrays: device copies of slm_boost's output (w [n_nodes, D], thr,
 * left, right, leaf [n_nodes]); roots [device, n_rounds * max(K, 1)] the
 * root of every tree in tree order.  F0 [host] f64 [max(K, 1)]; X [device]
 * F32 [N, D]; leaf_ids [device] int32 [n_rounds * max(K, 1), N] scratch
 * (receives every tree's leaf); F [device] f64 [N, max(K, 1)] receives the
 * scores.  n_classes: 0 (regression) or K in 2..16.  n_rounds = 0 gives F0.
 * Asynchronous.
 * ------------------------------------------------------------------------ */
slm_status slm_boost_scores(const float *w, const float *thr, const int32_t *left,
                            const int32_t *right, const double *leaf, int32_t n_nodes,
                            const int32_t *roots, int32_t n_rounds, int32_t n_classes, int32_t D,
                            const double *F0, double lr, const float *X, int64_t N,
                            int32_t *leaf_ids, double *F, void *stream);

/* ------------------------------------------------------------------------
 * slm_search_nodes -- the swarm search of a batch of nodes (Alg. 1 for every
 * node, all evaluated together), without partitioning: the per-depth step of
 * slm_grow_tree on caller-given node row sets.
 *
 * Node j owns rows row_off[j] .. row_off[j+1]-1 of X / target ([device]
 * int64, non-decreasing); node_id[j] ([device]) keys its random numbers as
 * the heap id does in slm_grow_tree.  prm supplies the criterion, P, T,
 * bins, precision, proposal and seed (max_depth and min_node are ignored).
 * target_loss ([device] [n_nodes] or NULL): a node stops after the first
 * evaluation whose global-best loss is <= target_loss[j] (its rows are
 * skipped from then on); the search ends when every node has stopped or
 * after T moves.  Outputs ([device]): gbest [n_nodes, D], gbest_loss,
 * gbest_split, gbest_thr [n_nodes] and evals [n_nodes] (evaluations run for
 * the node: the one that reached its target, else T + 1).  Synchronous (one
 * host read per evaluation when target_loss is given).
 * ------------------------------------------------------------------------ */
size_t slm_search_nodes_workspace(const slm_tree_params *prm, int64_t N, int32_t D,
                                  int32_t n_nodes);
slm_status slm_search_nodes(const void *X, int32_t x_dtype, int64_t N, int32_t D,
                            const void *target, int32_t t_dtype, const int64_t *row_off,
                            const int32_t *node_id, int32_t n_nodes, const slm_tree_params *prm,
                            const double *target_loss, double *gbest, double *gbest_loss,
                            int32_t *gbest_split, float *gbest_thr, int32_t *evals,
                            void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Learned proposal of initial swarm positions.  The paper starts every swarm
 * at random (Sec. III-A); these calls only replace that start, so the swarm
 * and its loss stay the judge of every direction and random starts remain the
 * fallback.  Not in the paper: the definitions below are this library's.
 *
 * slm_node_stats: per node j (rows as in slm_split_scan, labels in [0, K),
 *   1 <= K <= 16, K * D <= 4096), with feature mean mu, population standard
 *   deviation sigma, class proportions pi_k and class means m_k, classes
 *   ordered by count (largest first, ties to the lower id):
 *     stats[j, c*D + d] = pi_k (m_k,d - mu_d) / sigma_d  (c-th class k),
 *     stats[j, K*D + d] = sum_k pi_k Var_k(x_d) / sigma_d^2,
 *   0 where sigma_d = 0; sigma[j, d] = sigma_d.  Sums in FP64 (atomics: the
 *   last bits depend on the order), outputs FP32.  workspace: >=
 *   slm_node_stats_workspace bytes, zero-filled before first use, left
 *   zero-filled.  Asynchronous.
 * slm_mlp_forward: o = W3 GELU(W2 GELU(W1 s + b1) + b2) + b3 for a batch of
 *   inputs s [batch, n_in]; GELU(x) = x Phi(x).  params packed as W1
 *   [hidden, n_in], b1 [hidden], W2 [hidden, hidden], b2, W3 [n_out, hidden],
 *   b3 (FP32, slm_mlp_param_count floats).  bf16 = 1 rounds both operands
 *   of every product to BF16 (BF16 inference; FP32 accumulation).  cache
 *   (4 batch hidden floats) receives four consecutive [batch, hidden]
 *   blocks z1, h1, z2, h2 (pre- and post-GELU of both hidden layers; the
 *   backward reads them).
 *   out [batch, n_out].  Asynchronous.
 * slm_mlp_backward: gradient of sum(d_out * o) with respect to the packed
 *   parameters (grads, same layout), from the forward's cache; work [batch,
 *   2 hidden] scratch.  Asynchronous.
 * slm_wta_loss: per sample b, with M seeds of D values o[b] (unit seeds
 *   u_i = o_i / |o_i|) and a unit target t[b]: q_i = (u_i . t)^2, winner =
 *   first argmax, loss[b] = sum_i w_i (1 - q_i) with w = 1 - eps for the
 *   winner and eps / (M - 1) otherwise; d_out = scale * d loss[b] / d o[b]
 *   (scale = 1 / batch gives the gradient of the batch mean).  Asynchronous.
 * slm_proposal_targets: training target of a raw unit direction g (a swarm's
 *   global best) with the node's sigma: t = g sigma / |g sigma|, the
 *   standardised-space direction the seeds are compared with.  [n, D] each.
 *   Asynchronous.
 * slm_adam_step: Adam (Kingma and Ba) on n floats, step counted from 1.
 * slm_proposal_seeds: seed i of node j (o [n_nodes, M * D], standardised
 *   space) -> raw direction a_d = u_d / sigma_d scaled to unit norm, written
 *   as position, personal best and projection copy (w_dtype F32 or BF16) of
 *   particle i < min(M, P) of node j; a seed of zero norm leaves the particle
 *   as it was.  Asynchronous.
 * ------------------------------------------------------------------------ */
size_t slm_node_stats_workspace(int32_t n_nodes, int32_t D, int32_t K);
slm_status slm_node_stats(const void *X, int32_t x_dtype, int64_t N, int32_t D,
                          const int32_t *labels, int32_t K, const int64_t *row_off,
                          int32_t n_nodes, float *stats, float *sigma, void *workspace,
                          size_t ws_bytes, void *stream);
int64_t slm_mlp_param_count(int32_t n_in, int32_t hidden, int32_t n_out);
slm_status slm_mlp_forward(const float *params, int32_t n_in, int32_t hidden, int32_t n_out,
                           const float *in, int32_t batch, int32_t bf16, float *out, float *cache,
                           void *stream);
slm_status slm_mlp_backward(const float *params, int32_t n_in, int32_t hidden, int32_t n_out,
                            const float *in, int32_t batch, const float *cache,
                            const float *d_out, float *grads, float *work, void *stream);
slm_status slm_wta_loss(const float *out, const float *target, int32_t batch, int32_t M,
                        int32_t D, float eps, float scale, float *loss, float *d_out,
                        void *stream);
slm_status slm_proposal_targets(const float *g, const float *sigma, int32_t n, int32_t D,
                                float *t, void *stream);
slm_status slm_adam_step(float *params, const float *grads, float *m, float *v, int64_t n,
                         float lr, float b1, float b2, float eps, int32_t step, void *stream);
slm_status slm_proposal_seeds(const float *out, const float *sigma, int32_t n_nodes, int32_t M,
                              int32_t D, int32_t P, double *x, double *pbest, void *W_out,
                              int32_t w_dtype, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SLM_H */
