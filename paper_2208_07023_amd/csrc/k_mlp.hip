// Learned proposal of initial swarm positions: node statistics, a three-layer
// GELU network (forward and backward), its relaxed winner-take-all loss,
// Adam, and the map from network seeds to unit directions.  The paper starts
// every swarm at random positions (Sec. III-A); these kernels only replace
// that start -- the swarm, its loss and its acceptance rule are unchanged.
//
// Definitions (one node, K classes, D features):
//   mu, sigma       feature mean and population standard deviation;
//   pi_k, m_k       class proportion and class mean; classes ordered by count
//                   (largest first, ties to the lower id);
//   block c         pi_k (m_k - mu) / sigma for the c-th class in that order;
//   last block      v = sum_k pi_k Var_k / sigma^2;  0 where sigma = 0.
//   network         o = W3 GELU(W2 GELU(W1 s + b1) + b2) + b3, GELU(x) = x Phi(x)
//   seeds           o holds M seeds of D values in the standardised space; a
//                   seed u maps to the raw direction u / sigma, unit norm.
#include "slm_internal.hpp"

namespace slm {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int STATS_WG = 256;
constexpr int64_t STATS_CH = 2048;

// ---------------------------------------------------------------- statistics
// Per (chunk x node) item: per-class sums of x and x^2 of every feature in
// FP64 (a thread owns a feature and keeps KT >= K class sums in registers),
// added into the node's accumulator [K][D][2] with FP64 atomics, and
// per-class counts.
template <int KT>
__global__ __launch_bounds__(STATS_WG) void k_stats_sums(StatsArgs a) {
  __shared__ uint32_t cnt[16];
  const Item it = find_item(a.beg, a.end, a.n_nodes, a.N, STATS_CH, blockIdx.x);
  if (it.node < 0) return;
  const int tid = threadIdx.x, D = a.D, K = a.K;
  if (tid < 16) cnt[tid] = 0;
  __syncthreads();
  double *g = a.sums + (size_t)it.node * K * D * 2;
  for (int d = tid; d < D; d += STATS_WG) {
    double s1[KT], s2[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) s1[k] = s2[k] = 0.0;
    constexpr int U = 8;
    int64_t r = it.lo;
    for (; r + U <= it.hi; r += U) {
      float xv[U];
      int lb[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        lb[u] = a.labels[r + u];
        xv[u] = a.x_bf16 ? bf16_to_f32(static_cast<const uint16_t *>(a.X)[(r + u) * D + d])
                         : static_cast<const float *>(a.X)[(r + u) * D + d];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double x = (double)xv[u];
#pragma unroll
        for (int k = 0; k < KT; ++k) {
          const double m = lb[u] == k ? x : 0.0;
          s1[k] += m;
          s2[k] += m * m;
        }
      }
    }
    for (; r < it.hi; ++r) {
      const int l = a.labels[r];
      const double x = (double)(a.x_bf16 ? bf16_to_f32(static_cast<const uint16_t *>(a.X)[r * D + d])
                                         : static_cast<const float *>(a.X)[r * D + d]);
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        const double m = l == k ? x : 0.0;
        s1[k] += m;
        s2[k] += m * m;
      }
    }
#pragma unroll
    for (int k = 0; k < KT; ++k)
      if (k < K) {
        if (s1[k] != 0.0) unsafeAtomicAdd(&g[(k * D + d) * 2], s1[k]);
        if (s2[k] != 0.0) unsafeAtomicAdd(&g[(k * D + d) * 2 + 1], s2[k]);
      }
  }
  for (int64_t r = it.lo + tid; r < it.hi; r += STATS_WG) {
    const int k = a.labels[r];
    if ((unsigned)k < (unsigned)K) atomicAdd(&cnt[k], 1u);
  }
  __syncthreads();
  if (tid < K && cnt[tid]) atomicAdd(&a.counts[(size_t)it.node * K + tid], cnt[tid]);
}

// Per node: mean, deviation, class order, blocks; clears the accumulators.
__global__ __launch_bounds__(STATS_WG) void k_stats_finish(StatsArgs a) {
  __shared__ int order[16];
  __shared__ uint32_t cs[16];
  const int j = blockIdx.x, tid = threadIdx.x, D = a.D, K = a.K;
  if (tid < K) cs[tid] = a.counts[(size_t)j * K + tid];
  __syncthreads();
  if (tid == 0) {
    // counts descending, ties to the lower class id (insertion sort, K <= 16)
    for (int k = 0; k < K; ++k) order[k] = k;
    for (int i = 1; i < K; ++i) {
      const int v = order[i];
      int p = i - 1;
      while (p >= 0 && (cs[order[p]] < cs[v] || (cs[order[p]] == cs[v] && order[p] > v))) {
        order[p + 1] = order[p];
        --p;
      }
      order[p + 1] = v;
    }
  }
  __syncthreads();
  uint64_t n = 0;
  for (int k = 0; k < K; ++k) n += cs[k];
  const double dn = (double)n;
  double *g = a.sums + (size_t)j * K * D * 2;
  float *s = a.stats + (size_t)j * (K + 1) * D;
  for (int d = tid; d < D; d += STATS_WG) {
    double S1 = 0.0, S2 = 0.0;
    for (int k = 0; k < K; ++k) {
      S1 += g[(k * D + d) * 2];
      S2 += g[(k * D + d) * 2 + 1];
    }
    double mu = 0.0, var = 0.0;
    if (n) {
      mu = S1 / dn;
      var = S2 / dn - mu * mu;
      var = var > 0.0 ? var : 0.0;
    }
    const double sg = sqrt(var);
    const bool ok = sg > 0.0;
    double within = 0.0;
    for (int c = 0; c < K; ++c) {
      const int k = order[c];
      const double nk = (double)cs[k];
      double blk = 0.0;
      if (cs[k] && ok) {
        const double s1 = g[(k * D + d) * 2], s2 = g[(k * D + d) * 2 + 1];
        const double mk = s1 / nk;
        const double vk = s2 / nk - mk * mk;
        const double pk = nk / dn;
        blk = pk * (mk - mu) / sg;
        within += pk * (vk > 0.0 ? vk : 0.0);
      }
      s[c * D + d] = (float)blk;
    }
    s[K * D + d] = ok ? (float)(within / var) : 0.0f;
    a.sigma[(size_t)j * D + d] = (float)sg;
  }
  __syncthreads();
  for (int i = tid; i < K * D * 2; i += STATS_WG) g[i] = 0.0;
  if (tid < K) a.counts[(size_t)j * K + tid] = 0;
}

// ---------------------------------------------------------------- GEMM
// C[m, n] = sum_k A(m, k) B(k, n) (+ bias[n]), A(m, k) = A[m sam + k sak],
// B(k, n) = B[k sbk + n sbn], C row-major [M, N].  64 x 64 tiles, k in steps
// of 16 staged in LDS, four waves of v_mfma_f32_32x32x2_f32.  RB: operands are
// rounded to bfloat16 on load (products stay exact in FP32).  EPI: 0 = store
// z; 1 = store z and GELU(z) (second output C2).
struct GemmArgs {
  const float *A, *B, *bias;
  float *C, *C2;
  int M, N, K;
  int64_t sam, sak, sbk, sbn;
};

__device__ __forceinline__ float round_bf16(float x) {
  return __uint_as_float((uint32_t)f32_to_bf16_rne(x) << 16);
}

__device__ __forceinline__ float gelu_f(float x) {
  return x * (0.5f * erfcf(-x * 0.70710678118654752f));
}

template <bool RB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  constexpr int TM = 64, TN = 64, TK = 16;
  __shared__ float As[TM][TK + 1];
  __shared__ float Bs[TK][TN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int li = lane & 31, kh = lane >> 5;
  f32x16 acc = f32x16{};
  for (int k0 = 0; k0 < g.K; k0 += TK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + u * 256;          // 1024 = 64 x 16
      const int m = e / TK, k = e % TK;
      const int gm = m0 + m, gk = k0 + k;
      float v = (gm < g.M && gk < g.K) ? g.A[gm * g.sam + gk * g.sak] : 0.f;
      As[m][k] = RB ? round_bf16(v) : v;
      const int kb = e / TN, n = e % TN;
      const int gn = n0 + n, gkb = k0 + kb;
      float w = (gn < g.N && gkb < g.K) ? g.B[gkb * g.sbk + gn * g.sbn] : 0.f;
      Bs[kb][n] = RB ? round_bf16(w) : w;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < TK / 2; ++ks) {
      const float av = As[wm * 32 + li][2 * ks + kh];
      const float bv = Bs[2 * ks + kh][wn * 32 + li];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int n = n0 + wn * 32 + li;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + wm * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
    if (m < g.M && n < g.N) {
      float z = acc[r];
      if (g.bias) z = z + g.bias[n];
      g.C[(int64_t)m * g.N + n] = z;
      if constexpr (EPI == 1) g.C2[(int64_t)m * g.N + n] = gelu_f(z);
    }
  }
}

template <bool RB, int EPI>
slm_status gemm(const GemmArgs &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return SLM_OK;
  const dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64));
  hipLaunchKernelGGL((k_gemm<RB, EPI>), grid, dim3(256), 0, s, g);
  SLM_LAUNCHED();
  return SLM_OK;
}

// d_z = d_h * GELU'(z) (in place on d_h), n elements
__global__ void k_gelu_bwd(const float *z, float *dh, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = z[i];
  const float cdf = 0.5f * erfcf(-x * 0.70710678118654752f);
  const float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
  dh[i] = dh[i] * (cdf + x * pdf);
}

// out[n] = sum over rows of d [rows, cols]
__global__ void k_colsum(const float *d, int rows, int cols, float *out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += d[(int64_t)r * cols + c];
  out[c] = s;
}

// ---------------------------------------------------------------- loss
// One work-group per sample: q_i = (u_i . t)^2 for the unit seeds u_i, winner
// b = first argmax, L = sum_i w_i (1 - q_i), d o_i = -2 w_i c_i (t - c_i u_i) / r_i.
constexpr int WTA_WG = 256;
__global__ __launch_bounds__(WTA_WG) void k_wta(const float *o, const float *t, int M, int D,
                                                float eps, float scale, float *loss, float *d_o) {
  __shared__ float sr[256], sc[256];
  __shared__ int s_best;
  const int b = blockIdx.x, tid = threadIdx.x;
  const float *ob = o + (int64_t)b * M * D;
  const float *tb = t + (int64_t)b * D;
  for (int i = tid; i < M; i += WTA_WG) {
    float rr = 0.f, dc = 0.f;
    for (int d = 0; d < D; ++d) {
      const float v = ob[i * D + d];
      rr += v * v;
      dc += v * tb[d];
    }
    const float r = sqrtf(rr);
    sr[i] = r;
    sc[i] = r > 0.f ? dc / r : 0.f;
  }
  __syncthreads();
  if (tid == 0) {
    int best = 0;
    float bq = -1.f;
    for (int i = 0; i < M; ++i) {
      const float q = sc[i] * sc[i];
      if (q > bq) {
        bq = q;
        best = i;
      }
    }
    s_best = best;
    const float wo = M > 1 ? eps / (float)(M - 1) : 0.f;
    const float wb = M > 1 ? 1.f - eps : 1.f;
    float L = 0.f;
    for (int i = 0; i < M; ++i) L += (i == best ? wb : wo) * (1.f - sc[i] * sc[i]);
    loss[b] = L;
  }
  __syncthreads();
  const float wo = M > 1 ? eps / (float)(M - 1) : 0.f;
  const float wb = M > 1 ? 1.f - eps : 1.f;
  for (int e = tid; e < M * D; e += WTA_WG) {
    const int i = e / D, d = e - i * D;
    const float r = sr[i];
    float gv = 0.f;
    if (r > 0.f) {
      const float c = sc[i], w = i == s_best ? wb : wo;
      const float u = ob[e] / r;
      gv = -2.f * w * c * (tb[d] - c * u) / r * scale;
    }
    d_o[(int64_t)b * M * D + e] = gv;
  }
}

// ---------------------------------------------------------------- Adam
__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- seeds
// Seed i of node j -> raw unit direction u / sigma written as the FP64 position
// (and personal best, and projection copy) of particle i (< min(M, P)).  A
// seed whose direction has zero norm leaves the particle's random start.
__global__ __launch_bounds__(64) void k_seeds(const float *o, const float *sigma, int n_nodes,
                                              int M, int D, int P, double *x, double *pbest,
                                              void *W_out, int w_bf16) {
  const int64_t row = blockIdx.x;          // node j, seed i
  const int j = (int)(row / M), i = (int)(row % M);
  if (j >= n_nodes || i >= P) return;
  const int lane = threadIdx.x;
  const float *u = o + row * D;
  const float *sg = sigma + (int64_t)j * D;
  double ss = 0.0;
  for (int d = lane; d < D; d += 64) {
    const double a = sg[d] > 0.f ? (double)u[d] / (double)sg[d] : 0.0;
    ss += a * a;
  }
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
  if (!(ss > 0.0)) return;
  const double inv = 1.0 / sqrt(ss);
  const int64_t base = ((int64_t)j * P + i) * D;
  for (int d = lane; d < D; d += 64) {
    const double a = sg[d] > 0.f ? (double)u[d] / (double)sg[d] : 0.0;
    const double xv = a * inv;
    x[base + d] = xv;
    pbest[base + d] = xv;
    if (w_bf16) static_cast<uint16_t *>(W_out)[base + d] = f64_to_bf16(xv);
    else static_cast<float *>(W_out)[base + d] = (float)xv;
  }
}

// Raw unit direction g -> standardised unit target t = g sigma / |g sigma|
// (zero where the product has zero norm).  One wave per row.
__global__ __launch_bounds__(64) void k_targets(const float *g, const float *sigma, int D,
                                                float *t) {
  const int64_t row = blockIdx.x;
  const int lane = threadIdx.x;
  double ss = 0.0;
  for (int d = lane; d < D; d += 64) {
    const double v = (double)g[row * D + d] * (double)sigma[row * D + d];
    ss += v * v;
  }
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
  const double inv = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
  for (int d = lane; d < D; d += 64)
    t[row * D + d] = (float)((double)g[row * D + d] * (double)sigma[row * D + d] * inv);
}

}  // namespace

// ---------------------------------------------------------------- launchers
slm_status launch_targets(const float *g, const float *sigma, int n, int D, float *t,
                          hipStream_t s) {
  if (n <= 0) return SLM_OK;
  hipLaunchKernelGGL(k_targets, dim3((unsigned)n), dim3(64), 0, s, g, sigma, D, t);
  SLM_LAUNCHED();
  return SLM_OK;
}

size_t stats_workspace_bytes(int n_nodes, int D, int K) {
  return ((size_t)n_nodes * K * D * 2 * 8 + 255) / 256 * 256 + (size_t)n_nodes * K * 4 + 256;
}

slm_status launch_node_stats_full(const StatsArgs &a, hipStream_t s) {
  if (a.n_nodes <= 0) return SLM_OK;
  const int64_t items = num_items(a.n_nodes, a.N, STATS_CH);
  SLM_CHECK(a.K >= 1 && a.K <= 16, SLM_E_SHAPE, "slm_node_stats: K = %d not in [1, 16]", a.K);
  if (items > 0) {
    const dim3 grid((unsigned)items);
    if (a.K <= 2) hipLaunchKernelGGL(k_stats_sums<2>, grid, dim3(STATS_WG), 0, s, a);
    else if (a.K <= 4) hipLaunchKernelGGL(k_stats_sums<4>, grid, dim3(STATS_WG), 0, s, a);
    else if (a.K <= 8) hipLaunchKernelGGL(k_stats_sums<8>, grid, dim3(STATS_WG), 0, s, a);
    else hipLaunchKernelGGL(k_stats_sums<16>, grid, dim3(STATS_WG), 0, s, a);
    SLM_LAUNCHED();
  }
  hipLaunchKernelGGL(k_stats_finish, dim3((unsigned)a.n_nodes), dim3(STATS_WG), 0, s, a);
  SLM_LAUNCHED();
  return SLM_OK;
}

// params packed (W1 [H, I], b1 [H], W2 [H, H], b2 [H], W3 [O, H], b3 [O])
struct MlpView {
  const float *W1, *b1, *W2, *b2, *W3, *b3;
};
static MlpView view(const float *p, int I, int H, int O) {
  MlpView v;
  v.W1 = p;
  v.b1 = v.W1 + (size_t)H * I;
  v.W2 = v.b1 + H;
  v.b2 = v.W2 + (size_t)H * H;
  v.W3 = v.b2 + H;
  v.b3 = v.W3 + (size_t)O * H;
  return v;
}

int64_t mlp_param_count(int I, int H, int O) {
  return (int64_t)H * I + H + (int64_t)H * H + H + (int64_t)O * H + O;
}

// cache [B, 4H]: z1 | h1 | z2 | h2 (row-major blocks of [B, H])
slm_status launch_mlp_forward(const float *params, int I, int H, int O, const float *in, int B,
                              int bf16, float *out, float *cache, hipStream_t s) {
  const MlpView w = view(params, I, H, O);
  float *z1 = cache, *h1 = cache + (size_t)B * H, *z2 = cache + (size_t)2 * B * H,
        *h2 = cache + (size_t)3 * B * H;
  GemmArgs g{};
  // layer 1: z1 = in W1^T + b1
  g = GemmArgs{in, w.W1, w.b1, z1, h1, B, H, I, I, 1, 1, I};
  slm_status st = bf16 ? gemm<true, 1>(g, s) : gemm<false, 1>(g, s);
  if (st) return st;
  g = GemmArgs{h1, w.W2, w.b2, z2, h2, B, H, H, H, 1, 1, H};
  st = bf16 ? gemm<true, 1>(g, s) : gemm<false, 1>(g, s);
  if (st) return st;
  g = GemmArgs{h2, w.W3, w.b3, out, nullptr, B, O, H, H, 1, 1, H};
  return bf16 ? gemm<true, 0>(g, s) : gemm<false, 0>(g, s);
}

// grads packed like params; work [B, 2H]
slm_status launch_mlp_backward(const float *params, int I, int H, int O, const float *in, int B,
                               const float *cache, const float *d_out, float *grads, float *work,
                               hipStream_t s) {
  const MlpView w = view(params, I, H, O);
  float *gW1 = grads, *gb1 = gW1 + (size_t)H * I, *gW2 = gb1 + H, *gb2 = gW2 + (size_t)H * H,
        *gW3 = gb2 + H, *gb3 = gW3 + (size_t)O * H;
  const float *z1 = cache, *h1 = cache + (size_t)B * H, *z2 = cache + (size_t)2 * B * H,
              *h2 = cache + (size_t)3 * B * H;
  float *d2 = work, *d1 = work + (size_t)B * H;
  slm_status st;
  // gW3 [O, H] = d_out^T h2: A(m=o, k=b) = d_out[b O + o], B(k=b, n=h) = h2[b H + h]
  if ((st = gemm<false, 0>(GemmArgs{d_out, h2, nullptr, gW3, nullptr, O, H, B, 1, O, H, 1}, s)))
    return st;
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)((O + 255) / 256)), dim3(256), 0, s, d_out, B, O,
                     gb3);
  SLM_LAUNCHED();
  // d2 [B, H] = d_out W3: B(k=o, n=h) = W3[o H + h]
  if ((st = gemm<false, 0>(GemmArgs{d_out, w.W3, nullptr, d2, nullptr, B, H, O, O, 1, H, 1}, s)))
    return st;
  const int64_t bh = (int64_t)B * H;
  hipLaunchKernelGGL(k_gelu_bwd, dim3((unsigned)((bh + 255) / 256)), dim3(256), 0, s, z2, d2, bh);
  SLM_LAUNCHED();
  if ((st = gemm<false, 0>(GemmArgs{d2, h1, nullptr, gW2, nullptr, H, H, B, 1, H, H, 1}, s)))
    return st;
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)((H + 255) / 256)), dim3(256), 0, s, d2, B, H, gb2);
  SLM_LAUNCHED();
  if ((st = gemm<false, 0>(GemmArgs{d2, w.W2, nullptr, d1, nullptr, B, H, H, H, 1, H, 1}, s)))
    return st;
  hipLaunchKernelGGL(k_gelu_bwd, dim3((unsigned)((bh + 255) / 256)), dim3(256), 0, s, z1, d1, bh);
  SLM_LAUNCHED();
  if ((st = gemm<false, 0>(GemmArgs{d1, in, nullptr, gW1, nullptr, H, I, B, 1, H, I, 1}, s)))
    return st;
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)((H + 255) / 256)), dim3(256), 0, s, d1, B, H, gb1);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_wta(const float *o, const float *t, int B, int M, int D, float eps, float scale,
                      float *loss, float *d_o, hipStream_t s) {
  if (B <= 0) return SLM_OK;
  hipLaunchKernelGGL(k_wta, dim3((unsigned)B), dim3(WTA_WG), 0, s, o, t, M, D, eps, scale, loss,
                     d_o);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s) {
  if (n <= 0) return SLM_OK;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, lr,
                     b1, b2, eps, c1, c2);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_seeds(const float *o, const float *sigma, int n_nodes, int M, int D, int P,
                        double *x, double *pbest, void *W_out, int w_bf16, hipStream_t s) {
  if (n_nodes <= 0 || M <= 0) return SLM_OK;
  hipLaunchKernelGGL(k_seeds, dim3((unsigned)((int64_t)n_nodes * M)), dim3(64), 0, s, o, sigma,
                     n_nodes, M, D, P, x, pbest, W_out, w_bf16);
  SLM_LAUNCHED();
  return SLM_OK;
}

}  // namespace slm
