// Internal declarations shared by the HIP translation units of libslm.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/slm.h"

namespace slm {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
void clear_error();

#define SLM_HIP(expr)                                                          \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ::slm::set_error("%s failed: %s", #expr, hipGetErrorString(e_));         \
      return SLM_E_HIP;                                                        \
    }                                                                          \
  } while (0)

// Launch errors are read with hipGetLastError, which is not allowed while the
// stream is being captured into a graph; during capture they surface at
// instantiation instead.
bool capturing();
void set_capturing(bool on);
#define SLM_LAUNCHED()                                                         \
  do {                                                                         \
    if (!::slm::capturing()) SLM_HIP(hipGetLastError());                       \
  } while (0)

#define SLM_CHECK(cond, code, ...)                                             \
  do {                                                                         \
    if (!(cond)) {                                                             \
      ::slm::set_error(__VA_ARGS__);                                           \
      return code;                                                             \
    }                                                                          \
  } while (0)

// ---------------------------------------------------------------- segments
// Node j owns rows [beg[j], end[j]).  Offsets are clamped into [0, N] and an
// inverted range is empty, so kernels stay in bounds for any offset values.
struct Range {
  int64_t lo, hi;
};

__device__ __forceinline__ Range load_range(const int64_t *beg, const int64_t *end, int j,
                                            int64_t N) {
  int64_t b = beg[j], e = end[j];
  b = b < 0 ? 0 : (b > N ? N : b);
  e = e < b ? b : (e > N ? N : e);
  return {b, e};
}

// Work items are "chunk of CH global rows  x  node": node j's items start at
// TS(j) = floor(beg_j / CH) + j and cover the global chunks its rows touch.
// TS is strictly increasing for non-decreasing offsets; the total number of
// items is at most n_nodes + floor((N - 1) / CH) + 1.
struct Item {
  int node;       // -1: no work
  int64_t lo, hi; // rows of this item
  int chunk;      // index of this item within its node
  int nchunks;    // items of this node
};

__device__ __forceinline__ int64_t item_start(const int64_t *beg, int j, int64_t N, int64_t CH) {
  int64_t b = beg[j];
  b = b < 0 ? 0 : (b > N ? N : b);
  return b / CH + j;
}

__device__ __forceinline__ Item find_item(const int64_t *beg, const int64_t *end, int n_nodes,
                                          int64_t N, int64_t CH, int64_t v) {
  Item it{-1, 0, 0, 0, 0};
  if (n_nodes <= 0) return it;
  // largest j with TS(j) <= v
  int lo = 0, hi = n_nodes - 1;
  if (item_start(beg, 0, N, CH) > v) return it;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (item_start(beg, mid, N, CH) <= v) lo = mid; else hi = mid - 1;
  }
  Range r = load_range(beg, end, lo, N);
  if (r.hi <= r.lo) return it;
  int64_t g0 = r.lo / CH, g1 = (r.hi - 1) / CH;
  int64_t c = v - (g0 + lo);
  if (c < 0 || g0 + c > g1) return it;
  int64_t g = g0 + c;
  it.node = lo;
  it.lo = r.lo > g * CH ? r.lo : g * CH;
  it.hi = r.hi < (g + 1) * CH ? r.hi : (g + 1) * CH;
  it.chunk = (int)c;
  it.nchunks = (int)(g1 - g0 + 1);
  return it;
}

__host__ __device__ __forceinline__ int64_t num_items(int n_nodes, int64_t N, int64_t CH) {
  return N > 0 ? (int64_t)n_nodes + (N - 1) / CH + 1 : 0;
}

// Work-group barrier that orders LDS only.  __syncthreads() also waits for
// the group's outstanding global stores, which stalls loops that stream
// results out while staging the next tile in LDS.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------- float atomics
// Order-preserving min/max on float via integer atomics.  -0.0 is folded to
// +0.0 first (they compare equal), NaN is not expected.
__device__ __forceinline__ void atomic_min_f32(float *a, float v) {
  v = v + 0.0f;
  if (v >= 0.0f) atomicMin(reinterpret_cast<int *>(a), __float_as_int(v));
  else atomicMax(reinterpret_cast<unsigned *>(a), __float_as_uint(v));
}
__device__ __forceinline__ void atomic_max_f32(float *a, float v) {
  v = v + 0.0f;
  if (v >= 0.0f) atomicMax(reinterpret_cast<int *>(a), __float_as_int(v));
  else atomicMin(reinterpret_cast<unsigned *>(a), __float_as_uint(v));
}

// bfloat16 (bit pattern in uint16) <-> float
__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
// The BF16 image of an FP64 position is the RNE bfloat16 of its RNE float32.
__device__ __forceinline__ uint16_t f64_to_bf16(double d) {
  return f32_to_bf16_rne(static_cast<float>(d));
}

// ---------------------------------------------------------------- launchers
// Placement of Z[i, p] (row i, particle p), in elements: (p >> sh) * ts +
// i * rs + (p & (2^sh - 1)).  Row-major [N, P]: sh = 5, ts = 32, rs = P (the
// sum is i P + p).  Particle-tiled with tiles of w = 2^sh particles (w = 32
// or 8) [ceil(P/w), N, w]: ts = w N, rs = w, each tile a contiguous [N, w]
// block.  Elements are float32 (eb = 4) or, for the screening pass's 8-wide
// tiles, bfloat16 (eb = 2: the float32 projection rounded to nearest even).
// Word 3 of a gfx9 raw buffer resource (32-bit data format, no swizzle).
constexpr int BUF_DW3 = 0x00020000;
// Cache policy of the projection stream Z (the aux operand of the buffer
// builtins; bit 1 = non-temporal).  Z is written once by the projection and
// read once by the histogram scan.  The streaming projection's 8-wide Z
// tiles are stored non-temporally, and the scan's Z loads are non-temporal
// when the whole array is larger than the MALL (256 MiB).  Measured on the
// graph-replayed screening tree (N = 4e6, D = 256, P = 1024, 8 GB of Z):
// 1.9 % faster (stores alone 1.7 % faster, loads alone 0.4 % slower); timed
// one launch at a time (no graph) the projection then takes about 5 % longer
// and the scans 5-12 % less, so with the default policy part of the
// projection's writing is still under way when it is reported done.  A Z
// that fits the MALL (the plain tree's 102 MB) is loaded with the default
// policy: non-temporal loads made that tree about 6 % slower.  The store
// policy is not chosen at run time: a uniform branch around each store made
// the projection about 10 % slower.
constexpr int Z_CPOL_NT = 2;
__host__ __device__ inline bool z_streams(int64_t N, int P, int eb) {
  return N * (int64_t)P * eb > (256ll << 20);
}

struct ZLayout {
  int64_t ts, rs;
  int sh;
  int eb;   // bytes per element
};
__host__ __device__ __forceinline__ int64_t z_col(const ZLayout &l, int p) {
  return (int64_t)(p >> l.sh) * l.ts + (p & ((1 << l.sh) - 1));
}
// layout: SLM_Z_ROWS, SLM_Z_TILED (32-particle tiles), SLM_Z_TILED8 or
// SLM_Z_TILED8_BF16
__host__ __device__ __forceinline__ ZLayout zlayout_of(int layout, int64_t N, int P) {
  if (layout == 1) return ZLayout{32 * N, 32, 5, 4};
  if (layout == 2) return ZLayout{8 * N, 8, 3, 4};
  if (layout == 3) return ZLayout{8 * N, 8, 3, 2};
  return ZLayout{32, P, 5, 4};
}
// Tiles narrower than 32 put the 32 particles of a matrix-core block (and of
// a scan tile of up to 32 particles) up to 3 tiles apart: kernels address
// them through one buffer resource, whose offsets must stay below 2^31 bytes.
__host__ __device__ __forceinline__ bool zlayout_fits(const ZLayout &l, int64_t rows) {
  const int64_t span = ((int64_t)(31 >> l.sh) * l.ts + 31 + (rows + 64) * l.rs) * l.eb;
  return span < ((int64_t)1 << 31);
}
// Layout of a tree search's Z: 8-particle tiles (a scan work-group of 8
// particles streams whole rows of one tile), 32-particle tiles past the
// offset limit above (chunks of at most 65536 rows).  bf16: the screening
// pass of a classification histogram search stores bfloat16.
inline int grow_z_layout(int64_t N, bool bf16 = false) {
  if (bf16 && zlayout_fits(zlayout_of(3, N, 0), 65536)) return 3;
  return zlayout_fits(zlayout_of(2, N, 0), 65536) ? 2 : 1;
}

struct ProjectArgs {
  const void *X;
  int x_bf16;        // X stored as bfloat16 (else float32)
  int w_bf16;        // W stored as bfloat16 (else float32); both bfloat16 runs
                     // the bfloat16 matrix cores, otherwise float32 ones
  int64_t N;
  int D;
  const void *W;
  const int64_t *beg, *end;
  int n_nodes, P;
  float *Z;
  float *zmin, *zmax;
  ZLayout zl;
  // Optional: vpre[j] = rows of nodes 0 .. j-1 (n_nodes + 1 entries, on the
  // device).  Work is then split over the nodes' rows alone, as if they
  // were contiguous, instead of over [0, N).
  const int64_t *vpre;
  // with vpre: a host-side bound on those rows (the shape class of the
  // launch in the plan cache); 0 otherwise
  int64_t rows;
};
slm_status launch_project(const ProjectArgs &a, hipStream_t s);
// the launch's kernel can write bfloat16 Z (the streaming projection)
bool project_writes_bf16(const ProjectArgs &a);
slm_status launch_fill_minmax(float *zmin, float *zmax, int64_t n, hipStream_t s);
// zeroes n 32-bit words with a fill kernel (no memset node in captured graphs)
slm_status launch_zero_words(uint32_t *p, int64_t n, hipStream_t s);
// raises the dynamic-LDS limit of the streaming projection kernels
void prepare_project_kernels(int lds_max);

struct ScanArgs {
  const float *Z;
  ZLayout zl;
  const float *zmin, *zmax;
  const int32_t *labels;
  const double *y;
  int K;
  int64_t N;
  const int64_t *beg, *end;
  int n_nodes, P, bins, crit;
  int32_t *best_split;
  double *best_loss;
  float *threshold;
  uint32_t *hist_out;
  double *sums_out;
  void *ws;
  size_t ws_bytes;
  // Optional (histogram scan only): vpre[j] = rows of nodes 0 .. j-1
  // (n_nodes + 1 entries, on the device) and rows >= vpre[n_nodes], rows <=
  // N.  Work items and accumulator slots then follow the nodes' rows alone,
  // as if the nodes were contiguous, and the chunk plan is made for rows.
  const int64_t *vpre;
  int64_t rows;
};
size_t scan_workspace_bytes(int64_t N, int n_nodes, int P, int bins, int K, int crit);
slm_status launch_scan_hist(const ScanArgs &a, hipStream_t s);
// "no split" outputs for nodes without rows (the histogram scan skips them)
slm_status launch_scan_empty_nodes(const ScanArgs &a, hipStream_t s);
// The exact scan sorts one node's rows in one work-group's LDS: nodes of at
// most EXACT_ROWS rows.
constexpr int EXACT_ROWS = 8192;
slm_status launch_scan_exact(const ScanArgs &a, int max_rows, hipStream_t s);
// fused projection + histogram scan (float32, D <= 64, 2 <= K <= 4, Gini /
// entropy, particle-tiled layout of the scan arguments)
bool fused_eligible(const ScanArgs &a, int D, bool x_bf16, bool w_bf16);
slm_status launch_fused_eval(const ProjectArgs &pr, const ScanArgs &a, hipStream_t s);
slm_status launch_fused_hist(const ProjectArgs &pr, const ScanArgs &a, hipStream_t s);

struct PsoArgs {
  double *x, *v, *pbest, *pbest_loss, *gbest, *gbest_loss;
  int32_t *gbest_p;
  const double *loss;
  const double *gloss;   // optional: losses eligible for the global best (else loss)
  const int32_t *split;
  const float *thr;
  int32_t *gbest_split;
  float *gbest_thr;
  const int32_t *node_id;
  int n_nodes, P, D;
  double omega, c1, c2;
  uint64_t seed;
  uint32_t tree, iter;
  int move;
  void *W_out;
  int w_bf16;
  // optional: reset zmin/zmax of every (node, particle) for the next projection
  float *zmin_reset, *zmax_reset;
  // optional device copy of (seed, tree): lets one captured graph serve every tree
  const uint64_t *seed_tree_dev;
  // internal: only the global best (a final evaluation whose personal bests
  // are never read again)
  int bests_only;
  // optional [n_nodes, n_sel]: the start draws only these dimensions of each
  // node (the others are zero; the top-n DFT channels)
  const int32_t *dim_sel;
  int n_sel;
  // optional [n_nodes]: added to the tree id of node j's draws (the trees of
  // a forest grown together)
  const uint32_t *tree_off;
  // adaptive swarm (APSO): state estimation and parameter change between the
  // bests and the move; apso_state null = plain swarm
  int32_t *apso_state;   // [n_nodes] 1 exploration .. 4 jumping-out
  double *apso_par;      // [n_nodes * 3] omega, c1, c2
  double *apso_dist;     // [n_nodes * P] mean distances
  double *apso_f;        // [n_nodes] evolutionary factor
  int32_t *apso_worst;   // [n_nodes] particle replaced by the elite candidate
  double *apso_elite;    // [n_nodes * D] elite candidate (convergence)
  double *apso_part;     // [n_nodes * P * ceil(P / 64)] partial distance sums
  uint32_t apso_T;       // moves of the run (the elite step's sigma schedule)
  // optional [n_nodes, apso_n_sel]: the coordinates the swarm lives in (the
  // top DFT channels); the elite step perturbs one of them
  const int32_t *apso_sel;
  int apso_n_sel;
  // fused step (bests and move in one launch): positions and the global-best
  // record are read from these buffers and written to x / gbest / gbest_loss
  // (ping-pong; the other work-groups of a node still read the old record).
  // Also, for a bests-only step, the record to compare with and to carry
  // over when not improved.
  const double *x_in, *gbest_in, *gbest_loss_in;
};
// bests and move in one launch (plain swarm, no screening): every work-group
// finds its node's argmin itself; the record and positions ping-pong
slm_status launch_pso_fused(const PsoArgs &a, hipStream_t s);
// bytes of apso_part for n_nodes swarms of P particles
size_t apso_part_bytes(int n_nodes, int P);
slm_status launch_pso_init(const PsoArgs &a, hipStream_t s);
void prepare_pso_kernels(int lds_max);
slm_status launch_pso_step(const PsoArgs &a, hipStream_t s);
// probabilistic search candidates (ranks [n_nodes, R], pd / amax [R], device)
constexpr int PS_RMAX = 64;
slm_status launch_ps_tables(int R, double alpha0, double *pd, int32_t *amax, hipStream_t s);
slm_status launch_ps_candidates(const PsoArgs &a, const int32_t *ranks, int R, const double *pd,
                                const int32_t *amax, uint32_t t, hipStream_t s);

// discriminant feature test of every node and its top n channels
constexpr int DFT_DMAX = 4096;
struct DftArgs {
  const float *X;            // [N, D] float32, node rows contiguous
  int64_t N;
  int D;
  const int64_t *beg, *end;  // node row ranges
  int n_nodes;
  const int32_t *labels;     // classification
  const double *y;           // regression
  int K, bins, crit;
  int n;                     // channels kept per node
  double *loss;              // [n_nodes, D] DFT losses
  int32_t *sel;              // [n_nodes, n]
  void *ws;                  // dft_workspace_bytes, zero-filled, left zero-filled
  size_t ws_bytes;
};
size_t dft_workspace_bytes(int64_t N, int n_nodes, int D, int bins, int K, int crit);
slm_status launch_dft_select(const DftArgs &d, hipStream_t s);

// mixed-precision screening (bfloat16 screen, float32 re-score)
slm_status launch_screen_select(const double *loss, int n_nodes, int P, int k, int32_t *sel,
                                hipStream_t s);
slm_status launch_screen_gather(const double *x, const int32_t *sel, int n_nodes, int P, int k,
                                int D, float *W32, hipStream_t s);
slm_status launch_screen_merge(const int32_t *sel, const double *loss_r, const int32_t *split_r,
                               const float *thr_r, int n_nodes, int P, int k, double *loss,
                               int32_t *split, float *thr, double *gloss, hipStream_t s);

// learned proposal
struct StatsArgs {
  const void *X;
  int x_bf16;
  int64_t N;
  int D;
  const int32_t *labels;
  int K;
  const int64_t *beg, *end;
  int n_nodes;
  double *sums;          // accumulator [n_nodes][K][D][2]: zero on entry, zero on exit
  uint32_t *counts;      // [n_nodes][K]: zero on entry, zero on exit
  float *stats;          // [n_nodes][(K + 1) D]
  float *sigma;          // [n_nodes][D]
};
size_t stats_workspace_bytes(int n_nodes, int D, int K);
slm_status launch_node_stats_full(const StatsArgs &a, hipStream_t s);
int64_t mlp_param_count(int I, int H, int O);
slm_status launch_mlp_forward(const float *params, int I, int H, int O, const float *in, int B,
                              int bf16, float *out, float *cache, hipStream_t s);
slm_status launch_mlp_backward(const float *params, int I, int H, int O, const float *in, int B,
                               const float *cache, const float *d_out, float *grads, float *work,
                               hipStream_t s);
slm_status launch_wta(const float *o, const float *t, int B, int M, int D, float eps, float scale,
                      float *loss, float *d_o, hipStream_t s);
slm_status launch_targets(const float *g, const float *sigma, int n, int D, float *t,
                          hipStream_t s);
slm_status launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s);
slm_status launch_seeds(const float *o, const float *sigma, int n_nodes, int M, int D, int P,
                        double *x, double *pbest, void *W_out, int w_bf16, hipStream_t s);

slm_status launch_predict(const float *w, const float *thr, const int32_t *left,
                          const int32_t *right, int n_tree, int D, const float *X, int64_t N,
                          int32_t *leaf_out, hipStream_t s);

// ensembles (k_forest.hip)
slm_status launch_boot_draw(uint64_t seed, uint32_t tree0, int n_trees, int64_t N, int32_t *idx,
                            hipStream_t s);
slm_status launch_gather_rows(const void *src, size_t row_bytes, int64_t N, int64_t n_out,
                              const int32_t *idx, void *dst, const void *tsrc, int tb, void *tdst,
                              hipStream_t s);
slm_status launch_forest_leaves(const float *w, const float *thr, const int32_t *left,
                                const int32_t *right, int n_nodes, const int32_t *roots,
                                int n_trees, int D, const float *X, int64_t N, int32_t *leaf_out,
                                hipStream_t s);
slm_status launch_forest_combine(const int32_t *leaf_ids, const double *leaf, int n_nodes,
                                 int n_trees, int K, int64_t N, void *out, hipStream_t s);
slm_status launch_boost_residual(const int32_t *labels, const double *y, const double *F,
                                 int64_t N, int K, double *r, hipStream_t s);
slm_status launch_boost_init(double *F, int64_t N, int Kc, const double *F0, hipStream_t s);
slm_status launch_boost_update(double *F, const int32_t *leaf_ids, const double *leaf,
                               int n_nodes, int64_t N, int Kc, double lr, hipStream_t s);

struct TreeStats {
  uint32_t *counts;   // [n * K] classification
  uint32_t *cnt;      // [n] regression
  double *s1, *s2;    // [n]
  unsigned long long *ymin, *ymax;  // [n] order-preserving encodings of double
};

struct PartArgs {
  const void *X;        // current rows [N, D] (float32, or bfloat16 with x_bf16)
  void *Xn;             // destination rows
  int x_bf16;
  const int32_t *lab;   // labels (classification) or null
  int32_t *labn;
  const double *y;      // targets (regression) or null
  double *yn;
  const float *zsel;    // projection of each row on its node's split direction
  const float *thr;     // [n] threshold per node
  const int32_t *do_split;  // [n] 1 = split this node
  const int64_t *beg, *end;
  int n_nodes, D, K;
  int64_t N, CH;
  uint32_t *cnt_left;   // [items]
  int64_t *off_left, *off_right;  // [items]
  int64_t *n_left;      // [n]
  TreeStats child;      // children stats at index 2*j + side
};

slm_status launch_node_stats(const int64_t *beg, const int64_t *end, int n_nodes, int64_t N,
                             const int32_t *lab, const double *y, int K, TreeStats st,
                             hipStream_t s);
slm_status launch_partition(const PartArgs &a, hipStream_t s);
slm_status launch_search_stop(const double *gbest_loss, const double *target, const int64_t *beg,
                              int64_t *end_act, int32_t *done, int32_t *evals, int n,
                              int evals_now, bool last, uint32_t *remaining, hipStream_t s);
int64_t partition_items(int n_nodes, int64_t N);
// sets kernel attributes once per process (call outside stream capture)
slm_status prepare_kernels();

// ---------------------------------------------------------------- launch plans
// The autotuner's plan cache (autotune.cpp): mode 0 = fitted rules only,
// 1 = measured plans where cached, 2 = also measure the missing ones.
std::string device_arch();
int autotune_mode();
uint64_t autotune_generation();   // changes whenever the plans in use change
bool plan_lookup(const std::string &key, int64_t *a, int64_t *b);
bool plan_known(const std::string &key);
void plan_store(const std::string &key, int64_t a, int64_t b);
// measure the candidate plans of one launch's shape (not under capture) and
// cache the fastest; a shape already cached is left alone
slm_status tune_scan_hist(const ScanArgs &a, hipStream_t s);
slm_status tune_project(const ProjectArgs &a, hipStream_t s);

}  // namespace slm
