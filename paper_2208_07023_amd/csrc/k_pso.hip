// Particle swarm state on the device (Sec. III-A, Eqs. (11)-(12), Alg. 1).
//
// Positions, velocities and bests are FP64 [n_nodes * P, D]; the projection
// reads an FP32 (or BF16) image W of the positions, refreshed by every move.
// r1, r2 and the initial directions come from Philox4x32-10 (Salmon et al.,
// SC'11) with counter (p * ceil(D/2) + d/2, iteration, node id, tree) and the
// 64-bit seed as key, so any (tree, node, iteration, particle, dimension)
// draw can be reproduced independently.
#include "slm_internal.hpp"

namespace slm {
namespace {

constexpr uint32_t PH_M0 = 0xD2511F53u, PH_M1 = 0xCD9E8D57u;
constexpr uint32_t PH_W0 = 0x9E3779B9u, PH_W1 = 0xBB67AE85u;
constexpr uint32_t INIT_STREAM = 0xFFFFFFFFu;
constexpr int DMAX = 4096;
constexpr int STEP_WG = 256;

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k.x += PH_W0;
      k.y += PH_W1;
    }
    const uint32_t lo0 = PH_M0 * c.x, hi0 = __umulhi(PH_M0, c.x);
    const uint32_t lo1 = PH_M1 * c.z, hi1 = __umulhi(PH_M1, c.z);
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
  }
  return c;
}

__device__ __forceinline__ double u24(uint32_t w) { return (double)(w >> 8) * 0x1p-24; }

__device__ __forceinline__ void rng_key(const PsoArgs &a, uint2 *key, uint32_t *tree) {
  const uint64_t seed = a.seed_tree_dev ? a.seed_tree_dev[0] : a.seed;
  *tree = a.seed_tree_dev ? (uint32_t)a.seed_tree_dev[1] : a.tree;
  *key = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ __forceinline__ void store_w(void *W, int bf16, int64_t i, double x) {
  if (bf16) static_cast<uint16_t *>(W)[i] = f64_to_bf16(x);
  else static_cast<float *>(W)[i] = static_cast<float>(x);
}

__global__ void k_pso_init(PsoArgs a) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)a.n_nodes * a.P;
  if (gid >= total) return;
  const int j = (int)(gid / a.P), p = (int)(gid % a.P);
  const int D = a.D, dh = (D + 1) / 2;
  uint2 key;
  uint32_t tree;
  rng_key(a, &key, &tree);
  const uint32_t node = (uint32_t)a.node_id[j];
  double *x = a.x + gid * D;
  double s = 0.0;
  for (int m = 0; m < dh; ++m) {
    const uint4 w = philox4x32_10(make_uint4((uint32_t)(p * dh + m), INIT_STREAM, node, tree), key);
    const double u1 = ((double)w.x + 0.5) * 0x1p-32;
    const double u2 = (double)w.y * 0x1p-32;
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 6.283185307179586 * u2;
    const double g0 = rad * cos(ang);
    x[2 * m] = g0;
    s = s + g0 * g0;
    if (2 * m + 1 < D) {
      const double g1 = rad * sin(ang);
      x[2 * m + 1] = g1;
      s = s + g1 * g1;
    }
  }
  const double nrm = sqrt(s);
  for (int d = 0; d < D; ++d) {
    const double xv = nrm > 0.0 ? x[d] / nrm : x[d];
    x[d] = xv;
    a.v[gid * D + d] = 0.0;
    a.pbest[gid * D + d] = xv;
    store_w(a.W_out, a.w_bf16, gid * D + d, xv);
    if (p == 0) a.gbest[(int64_t)j * D + d] = xv;
  }
  a.pbest_loss[gid] = __builtin_huge_val();
  if (p == 0) {
    a.gbest_loss[j] = __builtin_huge_val();
    a.gbest_p[j] = -1;
    if (a.gbest_split) a.gbest_split[j] = -1;
    if (a.gbest_thr) a.gbest_thr[j] = __builtin_huge_valf();
  }
  if (a.zmin_reset) {
    a.zmin_reset[gid] = __builtin_huge_valf();
    a.zmax_reset[gid] = -__builtin_huge_valf();
  }
}

// One work-group per node; threads stride over the node's particles.
__global__ __launch_bounds__(STEP_WG) void k_pso_step(PsoArgs a) {
  __shared__ double gb[DMAX];
  __shared__ double red_l[STEP_WG];
  __shared__ int red_p[STEP_WG];
  __shared__ int s_improved, s_pstar;

  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  const int P = a.P, D = a.D;
  const int64_t base = (int64_t)j * P;

  // (1) personal bests; argmin of the current losses (lowest p on ties)
  double bl = __builtin_huge_val();
  int bp = 0x7fffffff;
  for (int p = tid; p < P; p += STEP_WG) {
    const double l = a.loss[base + p];
    if (l < a.pbest_loss[base + p]) {
      a.pbest_loss[base + p] = l;
      const double *xs = a.x + (base + p) * D;
      double *pb = a.pbest + (base + p) * D;
      for (int d = 0; d < D; ++d) pb[d] = xs[d];
    }
    if (l < bl) {
      bl = l;
      bp = p;
    }
  }
  red_l[tid] = bl;
  red_p[tid] = bp;
  __syncthreads();
  for (int o = STEP_WG / 2; o > 0; o >>= 1) {
    if (tid < o) {
      const double l2 = red_l[tid + o];
      const int p2 = red_p[tid + o];
      if (l2 < red_l[tid] || (l2 == red_l[tid] && p2 < red_p[tid])) {
        red_l[tid] = l2;
        red_p[tid] = p2;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int ps = red_p[0];
    const bool imp = ps != 0x7fffffff && red_l[0] < a.gbest_loss[j];
    s_improved = imp;
    s_pstar = ps;
    if (imp) {
      a.gbest_loss[j] = red_l[0];
      a.gbest_p[j] = ps;
      if (a.gbest_split && a.split) a.gbest_split[j] = a.split[base + ps];
      if (a.gbest_thr && a.thr) a.gbest_thr[j] = a.thr[base + ps];
    }
  }
  __syncthreads();
  const bool improved = s_improved;
  const int pstar = s_pstar;
  for (int d = tid; d < D; d += STEP_WG) {
    const double g = improved ? a.x[(base + pstar) * D + d] : a.gbest[(int64_t)j * D + d];
    gb[d] = g;
    if (improved) a.gbest[(int64_t)j * D + d] = g;
  }
  __syncthreads();
  if (a.zmin_reset) {
    for (int p = tid; p < P; p += STEP_WG) {
      a.zmin_reset[base + p] = __builtin_huge_valf();
      a.zmax_reset[base + p] = -__builtin_huge_valf();
    }
  }
  if (!a.move) return;

  // (2) move: Eq. (11), Eq. (12), unit-norm rescale
  const int dh = (D + 1) / 2;
  uint2 key;
  uint32_t tree;
  rng_key(a, &key, &tree);
  const uint32_t node = (uint32_t)a.node_id[j];
  for (int p = tid; p < P; p += STEP_WG) {
    double *xs = a.x + (base + p) * D;
    double *vs = a.v + (base + p) * D;
    const double *pb = a.pbest + (base + p) * D;
    double s = 0.0;
    for (int m = 0; m < dh; ++m) {
      const uint4 w = philox4x32_10(make_uint4((uint32_t)(p * dh + m), a.iter, node, tree), key);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int d = 2 * m + h;
        if (d >= D) break;
        const double r1 = u24(h ? w.z : w.x);
        const double r2 = u24(h ? w.w : w.y);
        const double xv = xs[d];
        const double t0 = a.omega * vs[d];
        const double t1 = (a.c1 * r1) * (pb[d] - xv);
        const double t2 = (a.c2 * r2) * (gb[d] - xv);
        const double vn = (t0 + t1) + t2;
        const double xn = xv + vn;
        vs[d] = vn;
        xs[d] = xn;
        s = s + xn * xn;
      }
    }
    const double nrm = sqrt(s);
    for (int d = 0; d < D; ++d) {
      // x + v == 0 exactly means x == -v: restore the previous position
      const double xv = nrm > 0.0 ? xs[d] / nrm : -vs[d];
      xs[d] = xv;
      store_w(a.W_out, a.w_bf16, (base + p) * D + d, xv);
    }
  }
}

__global__ void k_predict(const float *w, const float *thr, const int32_t *left,
                          const int32_t *right, int n_tree, int D, const float *X, int64_t N,
                          int32_t *leaf_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int node = 0;
  for (int steps = 0; steps < n_tree; ++steps) {
    const int l = left[node], r = right[node];
    if (l < 0 || l >= n_tree || r < 0 || r >= n_tree) break;
    const float *wr = w + (int64_t)node * D;
    const float *xr = X + i * D;
    float z = 0.0f;
    for (int d = 0; d < D; ++d) z = __fadd_rn(z, __fmul_rn(wr[d], xr[d]));
    node = z >= thr[node] ? r : l;
  }
  leaf_out[i] = node;
}

}  // namespace

slm_status launch_pso_init(const PsoArgs &a, hipStream_t s) {
  const int64_t total = (int64_t)a.n_nodes * a.P;
  if (total == 0) return SLM_OK;
  hipLaunchKernelGGL(k_pso_init, dim3((unsigned)((total + 127) / 128)), dim3(128), 0, s, a);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_pso_step(const PsoArgs &a, hipStream_t s) {
  SLM_CHECK(a.D <= DMAX, SLM_E_SHAPE, "slm_pso_step: D = %d exceeds %d", a.D, DMAX);
  if (a.n_nodes == 0) return SLM_OK;
  hipLaunchKernelGGL(k_pso_step, dim3((unsigned)a.n_nodes), dim3(STEP_WG), 0, s, a);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_predict(const float *w, const float *thr, const int32_t *left,
                          const int32_t *right, int n_tree, int D, const float *X, int64_t N,
                          int32_t *leaf_out, hipStream_t s) {
  if (N == 0) return SLM_OK;
  hipLaunchKernelGGL(k_predict, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, w, thr, left,
                     right, n_tree, D, X, N, leaf_out);
  SLM_LAUNCHED();
  return SLM_OK;
}

}  // namespace slm
