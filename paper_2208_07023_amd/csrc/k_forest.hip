// Ensembles of SLM trees on the device (Sec. V: SLM/SLR Forest, bagging, and
// SLM/SLR Boost, boosting):
//   k_boot_draw       bootstrap rows of every tree (N draws with replacement)
//   k_gather_rows     row gather / replication of X and the targets: the
//                     trees of a forest, or the K copies a softmax boosting
//                     round grows its per-class trees on, sit in consecutive
//                     row ranges of one matrix, so one breadth-first pass
//                     grows all of them together
//   k_forest_leaves   the leaf every (tree, row) reaches
//   k_forest_vote     majority vote of the trees' leaf classes
//   k_forest_mean     mean of the trees' leaf values (regression)
//   k_boost_residual  negative gradients: y - F, or 1{y = k} - softmax(F)_k
//   k_boost_update    F += lr * (leaf value reached)
#include "slm_internal.hpp"
#include "philox.hpp"

#include <algorithm>

namespace slm {
namespace {

constexpr int FWG = 256;
constexpr int VOTE_KMAX = 16;

// Draw i of tree b is word (i mod 4) of the Philox counter
// (i div 4, BOOT_STREAM, NO_NODE, tree0 + b), mapped to row floor(w N / 2^32).
__global__ __launch_bounds__(FWG) void k_boot_draw(uint64_t seed, uint32_t tree0, int64_t N,
                                                   int64_t groups, int32_t *idx) {
  const int64_t g = (int64_t)blockIdx.x * FWG + threadIdx.x;
  const uint32_t b = blockIdx.y;
  if (g >= groups) return;
  const uint4 w = philox4x32_10(make_uint4((uint32_t)g, BOOT_STREAM, NO_NODE, tree0 + b),
                                make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
  int32_t *o = idx + (int64_t)b * N;
  const int64_t i = 4 * g;
  const uint64_t n = (uint64_t)N;
  o[i] = (int32_t)(((uint64_t)w.x * n) >> 32);
  if (i + 1 < N) o[i + 1] = (int32_t)(((uint64_t)w.y * n) >> 32);
  if (i + 2 < N) o[i + 2] = (int32_t)(((uint64_t)w.z * n) >> 32);
  if (i + 3 < N) o[i + 3] = (int32_t)(((uint64_t)w.w * n) >> 32);
}

// dst row r = src row idx[r] (idx null: src row r mod N), upr units of U per
// row; the target of the row (tb = 4 or 8 bytes, or 0) moves with it.
template <typename U>
__global__ __launch_bounds__(FWG) void k_gather_rows(const U *src, int upr, int64_t N,
                                                     int64_t n_out, const int32_t *idx, U *dst,
                                                     const void *tsrc, int tb, void *tdst) {
  const int tid = threadIdx.x;
  auto move_target = [&](int64_t r, int64_t s) {
    if (tb == 8) static_cast<uint64_t *>(tdst)[r] = static_cast<const uint64_t *>(tsrc)[s];
    else if (tb == 4) static_cast<uint32_t *>(tdst)[r] = static_cast<const uint32_t *>(tsrc)[s];
  };
  if (upr <= FWG) {
    const int rpp = FWG / upr, lr = tid / upr, c = tid - lr * upr;
    if (lr >= rpp) return;
    for (int64_t r = (int64_t)blockIdx.x * rpp + lr; r < n_out; r += (int64_t)gridDim.x * rpp) {
      const int64_t s = idx ? (int64_t)idx[r] : r % N;
      dst[r * upr + c] = src[s * upr + c];
      if (c == 0) move_target(r, s);
    }
  } else {
    for (int64_t r = blockIdx.x; r < n_out; r += gridDim.x) {
      const int64_t s = idx ? (int64_t)idx[r] : r % N;
      for (int c = tid; c < upr; c += FWG) dst[r * upr + c] = src[s * upr + c];
      if (tid == 0) move_target(r, s);
    }
  }
}

// leaf reached by row i of X from root roots[b]: right iff
// float32(w . x) >= thr, the dot product accumulated in FP32 in dimension
// order (as slm_predict); -1 for a root index outside [0, n_nodes)
__global__ __launch_bounds__(FWG) void k_forest_leaves(const float *w, const float *thr,
                                                       const int32_t *left, const int32_t *right,
                                                       int n_nodes, const int32_t *roots, int D,
                                                       const float *X, int64_t N,
                                                       int32_t *leaf_out) {
  const int64_t i = (int64_t)blockIdx.x * FWG + threadIdx.x;
  if (i >= N) return;
  const int b = blockIdx.y;
  int node = roots[b];
  if (node < 0 || node >= n_nodes) {
    leaf_out[(int64_t)b * N + i] = -1;
    return;
  }
  const float *xr = X + i * D;
  for (int steps = 0; steps < n_nodes; ++steps) {
    const int l = left[node], r = right[node];
    if (l < 0 || l >= n_nodes || r < 0 || r >= n_nodes) break;
    const float *wr = w + (int64_t)node * D;
    float z = 0.0f;
    for (int d = 0; d < D; ++d) z = __fadd_rn(z, __fmul_rn(wr[d], xr[d]));
    node = z >= thr[node] ? r : l;
  }
  leaf_out[(int64_t)b * N + i] = node;
}

// every tree votes for its leaf's majority class (first maximum of the class
// counts); the row takes the class with most votes (smallest on ties); a -1
// leaf casts no vote
__global__ __launch_bounds__(FWG) void k_forest_vote(const int32_t *leaf_ids, const double *leaf,
                                                     int n_nodes, int n_trees, int K, int64_t N,
                                                     int32_t *out) {
  const int64_t i = (int64_t)blockIdx.x * FWG + threadIdx.x;
  if (i >= N) return;
  int votes[VOTE_KMAX];
#pragma unroll
  for (int k = 0; k < VOTE_KMAX; ++k) votes[k] = 0;
  for (int b = 0; b < n_trees; ++b) {
    const int node = leaf_ids[(int64_t)b * N + i];
    if (node < 0 || node >= n_nodes) continue;
    const double *lv = leaf + (int64_t)node * K;
    int c = 0;
    double best = lv[0];
    for (int k = 1; k < K; ++k)
      if (lv[k] > best) {
        best = lv[k];
        c = k;
      }
#pragma unroll
    for (int k = 0; k < VOTE_KMAX; ++k) votes[k] += c == k;
  }
  int c = 0, best = votes[0];
#pragma unroll
  for (int k = 1; k < VOTE_KMAX; ++k)
    if (k < K && votes[k] > best) {
      best = votes[k];
      c = k;
    }
  out[i] = c;
}

// mean of the trees' leaf values, summed in tree order (NaN if a leaf is -1)
__global__ __launch_bounds__(FWG) void k_forest_mean(const int32_t *leaf_ids, const double *leaf,
                                                     int n_nodes, int n_trees, int64_t N,
                                                     double *out) {
  const int64_t i = (int64_t)blockIdx.x * FWG + threadIdx.x;
  if (i >= N) return;
  double acc = 0.0;
  for (int b = 0; b < n_trees; ++b) {
    const int node = leaf_ids[(int64_t)b * N + i];
    acc = __dadd_rn(acc, node >= 0 && node < n_nodes ? leaf[node] : __builtin_nan(""));
  }
  out[i] = __ddiv_rn(acc, (double)n_trees);
}

// regression (labels null): r[i] = y[i] - F[i];
// classification: p = softmax(F[i, :]) (max subtracted, exponentials summed
// in class order), r[k N + i] = 1{y_i = k} - p_k
__global__ __launch_bounds__(FWG) void k_boost_residual(const int32_t *labels, const double *y,
                                                        const double *F, int64_t N, int K,
                                                        double *r) {
  const int64_t i = (int64_t)blockIdx.x * FWG + threadIdx.x;
  if (i >= N) return;
  if (!labels) {
    r[i] = __dsub_rn(y[i], F[i]);
    return;
  }
  const double *f = F + i * K;
  double m = f[0];
  for (int k = 1; k < K; ++k) m = fmax(m, f[k]);
  double s = 0.0;
  for (int k = 0; k < K; ++k) s = __dadd_rn(s, exp(__dsub_rn(f[k], m)));
  const int yi = labels[i];
  for (int k = 0; k < K; ++k) {
    const double p = __ddiv_rn(exp(__dsub_rn(f[k], m)), s);
    r[(int64_t)k * N + i] = __dsub_rn(yi == k ? 1.0 : 0.0, p);
  }
}

// F[i * Kc + k] += lr * leaf[leaf_ids[k N + i]] (leaf values of regression
// trees, one column)
__global__ __launch_bounds__(FWG) void k_boost_update(double *F, const int32_t *leaf_ids,
                                                      const double *leaf, int n_nodes, int64_t N,
                                                      int Kc, double lr) {
  const int64_t i = (int64_t)blockIdx.x * FWG + threadIdx.x;
  if (i >= N) return;
  for (int k = 0; k < Kc; ++k) {
    const int node = leaf_ids[(int64_t)k * N + i];
    const double h = node >= 0 && node < n_nodes ? leaf[node] : __builtin_nan("");
    F[i * Kc + k] = __dadd_rn(F[i * Kc + k], __dmul_rn(lr, h));
  }
}

// F[i * Kc + k] = F0[k] (the boosted model's initial scores)
struct F0Vals {
  double v[16];
};
__global__ __launch_bounds__(FWG) void k_boost_init(double *F, int64_t N, int Kc, F0Vals f0) {
  const int64_t i = (int64_t)blockIdx.x * FWG + threadIdx.x;
  if (i >= N) return;
  for (int k = 0; k < Kc; ++k) F[i * Kc + k] = f0.v[k];
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + FWG - 1) / FWG); }

}  // namespace

slm_status launch_boot_draw(uint64_t seed, uint32_t tree0, int n_trees, int64_t N, int32_t *idx,
                            hipStream_t s) {
  SLM_CHECK(n_trees >= 0 && n_trees <= 65535 && N >= 0 && N < (1ll << 31), SLM_E_SHAPE,
            "bootstrap: n_trees = %d, N = %lld out of range", n_trees, (long long)N);
  if (n_trees == 0 || N == 0) return SLM_OK;
  const int64_t groups = (N + 3) / 4;
  hipLaunchKernelGGL(k_boot_draw, dim3(blocks_for(groups), (unsigned)n_trees), dim3(FWG), 0, s,
                     seed, tree0, N, groups, idx);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_gather_rows(const void *src, size_t row_bytes, int64_t N, int64_t n_out,
                              const int32_t *idx, void *dst, const void *tsrc, int tb, void *tdst,
                              hipStream_t s) {
  SLM_CHECK(row_bytes >= 2 && row_bytes % 2 == 0 && (tb == 0 || tb == 4 || tb == 8), SLM_E_SHAPE,
            "gather: row of %zu bytes, target of %d bytes", row_bytes, tb);
  if (n_out == 0) return SLM_OK;
  SLM_CHECK(N >= 1, SLM_E_SHAPE, "gather: no source rows");
  const auto a16 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  const auto a4 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 3) == 0; };
  const unsigned grid = 2048;
  if (row_bytes % 16 == 0 && a16(src) && a16(dst)) {
    const int upr = (int)(row_bytes / 16);
    hipLaunchKernelGGL(k_gather_rows<uint4>, dim3(grid), dim3(FWG), 0, s,
                       static_cast<const uint4 *>(src), upr, N, n_out, idx,
                       static_cast<uint4 *>(dst), tsrc, tb, tdst);
  } else if (row_bytes % 4 == 0 && a4(src) && a4(dst)) {
    const int upr = (int)(row_bytes / 4);
    hipLaunchKernelGGL(k_gather_rows<uint32_t>, dim3(grid), dim3(FWG), 0, s,
                       static_cast<const uint32_t *>(src), upr, N, n_out, idx,
                       static_cast<uint32_t *>(dst), tsrc, tb, tdst);
  } else {
    const int upr = (int)(row_bytes / 2);
    hipLaunchKernelGGL(k_gather_rows<uint16_t>, dim3(grid), dim3(FWG), 0, s,
                       static_cast<const uint16_t *>(src), upr, N, n_out, idx,
                       static_cast<uint16_t *>(dst), tsrc, tb, tdst);
  }
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_forest_leaves(const float *w, const float *thr, const int32_t *left,
                                const int32_t *right, int n_nodes, const int32_t *roots,
                                int n_trees, int D, const float *X, int64_t N, int32_t *leaf_out,
                                hipStream_t s) {
  SLM_CHECK(n_trees >= 0 && n_trees <= 65535, SLM_E_SHAPE, "forest: n_trees = %d out of range",
            n_trees);
  if (N == 0 || n_trees == 0) return SLM_OK;
  hipLaunchKernelGGL(k_forest_leaves, dim3(blocks_for(N), (unsigned)n_trees), dim3(FWG), 0, s, w,
                     thr, left, right, n_nodes, roots, D, X, N, leaf_out);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_forest_combine(const int32_t *leaf_ids, const double *leaf, int n_nodes,
                                 int n_trees, int K, int64_t N, void *out, hipStream_t s) {
  SLM_CHECK(K == 0 || (K >= 2 && K <= VOTE_KMAX), SLM_E_SHAPE, "forest: K = %d (0 or 2..%d)", K,
            VOTE_KMAX);
  if (N == 0) return SLM_OK;
  if (K > 0)
    hipLaunchKernelGGL(k_forest_vote, dim3(blocks_for(N)), dim3(FWG), 0, s, leaf_ids, leaf,
                       n_nodes, n_trees, K, N, static_cast<int32_t *>(out));
  else
    hipLaunchKernelGGL(k_forest_mean, dim3(blocks_for(N)), dim3(FWG), 0, s, leaf_ids, leaf,
                       n_nodes, n_trees, N, static_cast<double *>(out));
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_boost_residual(const int32_t *labels, const double *y, const double *F,
                                 int64_t N, int K, double *r, hipStream_t s) {
  if (N == 0) return SLM_OK;
  hipLaunchKernelGGL(k_boost_residual, dim3(blocks_for(N)), dim3(FWG), 0, s, labels, y, F, N, K,
                     r);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_boost_update(double *F, const int32_t *leaf_ids, const double *leaf,
                               int n_nodes, int64_t N, int Kc, double lr, hipStream_t s) {
  if (N == 0) return SLM_OK;
  hipLaunchKernelGGL(k_boost_update, dim3(blocks_for(N)), dim3(FWG), 0, s, F, leaf_ids, leaf,
                     n_nodes, N, Kc, lr);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_boost_init(double *F, int64_t N, int Kc, const double *F0, hipStream_t s) {
  SLM_CHECK(Kc >= 1 && Kc <= 16, SLM_E_SHAPE, "boost: %d score columns (1..16)", Kc);
  if (N == 0) return SLM_OK;
  F0Vals f0{};
  for (int k = 0; k < Kc; ++k) f0.v[k] = F0[k];
  hipLaunchKernelGGL(k_boost_init, dim3(blocks_for(N)), dim3(FWG), 0, s, F, N, Kc, f0);
  SLM_LAUNCHED();
  return SLM_OK;
}

}  // namespace slm
