// Discriminant feature test of every node and its top n channels (Alg. 2:
// run the DFT for the node, select the top n channels, run the swarm in
// those n dimensions).
//
// The DFT loss of input feature d is the loss of the best threshold of x_d
// over the node's rows.  x_d is the projection on the unit vector e_d, so X
// itself, read as a row-major Z with D "particles", goes through the same
// histogram (or exact) scan as any projected feature: edges over the node's
// [min, max] of x_d, the criterion at every bin boundary.
//   k_col_minmax   per-(node, feature) min and max of X's columns: work items
//                  of at most MM_CH rows of one node, 64 columns per
//                  work-group (lanes = consecutive columns of a row).
// The n channels of smallest loss (ties to the lower index) are then picked
// by the screening selection (k_screen_select), and k_pso_init starts the
// swarm in their span.
#include "slm_internal.hpp"

#include <algorithm>

namespace slm {
namespace {

constexpr int MM_CH = 2048;   // rows per work item
constexpr int MM_WG = 256;    // 4 row groups x 64 columns

__global__ __launch_bounds__(MM_WG) void k_col_minmax(const float *X, int64_t N, int D,
                                                      const int64_t *beg, const int64_t *end,
                                                      int n_nodes, int n_cb, float *zmin,
                                                      float *zmax) {
  __shared__ float smn[MM_WG], smx[MM_WG];
  const int64_t v = blockIdx.x / n_cb;
  const int cb = (int)(blockIdx.x % n_cb);
  const Item it = find_item(beg, end, n_nodes, N, MM_CH, v);
  if (it.node < 0) return;
  const int tid = threadIdx.x;
  const int c = cb * 64 + (tid & 63), rg = tid >> 6;
  float mn = __builtin_huge_valf(), mx = -__builtin_huge_valf();
  if (c < D)
    for (int64_t r = it.lo + rg; r < it.hi; r += MM_WG / 64) {
      const float z = X[r * D + c];
      mn = fminf(mn, z);
      mx = fmaxf(mx, z);
    }
  smn[tid] = mn;
  smx[tid] = mx;
  __syncthreads();
  if (rg == 0 && c < D) {
#pragma unroll
    for (int g = 1; g < MM_WG / 64; ++g) {
      mn = fminf(mn, smn[tid + 64 * g]);
      mx = fmaxf(mx, smx[tid + 64 * g]);
    }
    if (mn <= mx) {
      const int64_t o = (int64_t)it.node * D + c;
      atomic_min_f32(&zmin[o], mn);
      atomic_max_f32(&zmax[o], mx);
    }
  }
}

// Zeroes n 32-bit words (a kernel, not a memset: it may sit in a captured
// graph).
__global__ void k_zero_words(uint32_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

}  // namespace

slm_status launch_zero_words(uint32_t *p, int64_t n, hipStream_t s) {
  if (n <= 0) return SLM_OK;
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  SLM_LAUNCHED();
  return SLM_OK;
}

size_t dft_workspace_bytes(int64_t N, int n_nodes, int D, int bins, int K, int crit) {
  const size_t nd = (size_t)std::max(0, n_nodes) * std::max(0, D);
  const size_t scan = bins ? scan_workspace_bytes(N, n_nodes, D, bins, K, crit) : 0;
  auto r = [](size_t b) { return (b + 255) / 256 * 256; };
  return r(scan) + 3 * r(nd * 4) + r(nd * 4) + 256;
}

slm_status launch_dft_select(const DftArgs &d, hipStream_t s) {
  SLM_CHECK(d.D >= 1 && d.D <= DFT_DMAX && d.n >= 1 && d.n <= d.D, SLM_E_SHAPE,
            "dft: D = %d, n = %d (1 <= n <= D <= %d)", d.D, d.n, DFT_DMAX);
  if (d.n_nodes <= 0 || d.N <= 0) return SLM_OK;
  const size_t nd = (size_t)d.n_nodes * d.D;
  SLM_CHECK(d.ws_bytes >= dft_workspace_bytes(d.N, d.n_nodes, d.D, d.bins, d.K, d.crit),
            SLM_E_NOMEM, "dft: workspace of %zu bytes too small", d.ws_bytes);
  auto r = [](size_t b) { return (b + 255) / 256 * 256; };
  char *p = static_cast<char *>(d.ws);
  const size_t scan_b = d.bins ? scan_workspace_bytes(d.N, d.n_nodes, d.D, d.bins, d.K, d.crit) : 0;
  void *scan_ws = p;
  p += r(scan_b);
  float *zmin = reinterpret_cast<float *>(p);
  p += r(nd * 4);
  float *zmax = reinterpret_cast<float *>(p);
  p += r(nd * 4);
  int32_t *split = reinterpret_cast<int32_t *>(p);
  p += r(nd * 4);
  float *thr = reinterpret_cast<float *>(p);

  slm_status st = launch_fill_minmax(zmin, zmax, (int64_t)nd, s);
  if (st) return st;
  const int n_cb = (d.D + 63) / 64;
  const int64_t grid = num_items(d.n_nodes, d.N, MM_CH) * n_cb;
  SLM_CHECK(grid < (1ll << 31), SLM_E_SHAPE, "dft: grid too large");
  hipLaunchKernelGGL(k_col_minmax, dim3((unsigned)grid), dim3(MM_WG), 0, s, d.X, d.N, d.D, d.beg,
                     d.end, d.n_nodes, n_cb, zmin, zmax);
  SLM_LAUNCHED();

  ScanArgs sa{};
  sa.Z = d.X;
  sa.zl = zlayout_of(0, d.N, d.D);   // row-major [N, D]: column d is x_d
  sa.zmin = zmin;
  sa.zmax = zmax;
  sa.labels = d.labels;
  sa.y = d.y;
  sa.K = d.K;
  sa.N = d.N;
  sa.beg = d.beg;
  sa.end = d.end;
  sa.n_nodes = d.n_nodes;
  sa.P = d.D;
  sa.bins = d.bins;
  sa.crit = d.crit;
  sa.best_split = split;
  sa.best_loss = d.loss;
  sa.threshold = thr;
  sa.ws = scan_ws;
  sa.ws_bytes = scan_b;
  if ((st = d.bins ? launch_scan_hist(sa, s) : launch_scan_exact(sa, EXACT_ROWS, s))) return st;
  if ((st = launch_scan_empty_nodes(sa, s))) return st;
  if ((st = launch_screen_select(d.loss, d.n_nodes, d.D, d.n, d.sel, s))) return st;
  // leave the whole workspace zero-filled (the scan part already is)
  const int64_t words = (int64_t)(4 * r(nd * 4)) / 4;
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<uint32_t *>(zmin), words);
  SLM_LAUNCHED();
  return SLM_OK;
}

}  // namespace slm
