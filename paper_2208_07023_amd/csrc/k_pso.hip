// Particle swarm state on the device (Sec. III-A, Eqs. (11)-(12), Alg. 1).
//
// Positions, velocities and bests are FP64 [n_nodes * P, D]; the projection
// reads an FP32 (or BF16) image W of the positions, refreshed by every move.
// r1, r2 and the initial directions come from Philox4x32-10 (Salmon et al.,
// SC'11) with counter (p * ceil(D/2) + d/2, iteration, node id, tree) and the
// 64-bit seed as key, so any (tree, node, iteration, particle, dimension)
// draw can be reproduced independently.
#include "slm_internal.hpp"
#include "philox.hpp"

namespace slm {
namespace {

constexpr int DMAX = 4096;

// key and tree word of node j's draws (trees of a forest add their index to
// the base tree id)
__device__ __forceinline__ void rng_key(const PsoArgs &a, int j, uint2 *key, uint32_t *tree) {
  const uint64_t seed = a.seed_tree_dev ? a.seed_tree_dev[0] : a.seed;
  *tree = (a.seed_tree_dev ? (uint32_t)a.seed_tree_dev[1] : a.tree) +
          (a.tree_off ? a.tree_off[j] : 0u);
  *key = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ __forceinline__ void store_w(void *W, int bf16, int64_t i, double x) {
  if (bf16) static_cast<uint16_t *>(W)[i] = f64_to_bf16(x);
  else static_cast<float *>(W)[i] = static_cast<float>(x);
}

// Work-group of 256 threads covering PPB = 256 / Dp particles of one node,
// Dp = D rounded up to a power of two (<= 256); thread (pl, d) owns dimension
// d (and d + 256k for D > 256) of particle pl.  Norms are summed in
// dimension order by one thread per particle from LDS, so every operation
// happens in the same order as the sequential definition.
constexpr int MOVE_WG = 256;

// Squared norm of row r[0..D) summed in dimension order (s + r_d * r_d, each
// operation rounded, as the sequential definition); the loads of eight
// dimensions are issued before their adds so their latencies overlap.
__device__ __forceinline__ double sq_norm_ordered(const double *r, int D) {
  double s = 0.0;
  int d = 0;
  for (; d + 8 <= D; d += 8) {
    double t[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) t[k] = r[d + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) s = s + t[k] * t[k];
  }
  for (; d < D; ++d) s = s + r[d] * r[d];
  return s;
}

struct MoveGeom {
  int Dp, PPB;
};
__host__ __device__ __forceinline__ MoveGeom move_geom(int D) {
  int Dp = 1;
  while (Dp < D && Dp < MOVE_WG) Dp <<= 1;
  return {Dp, MOVE_WG / Dp};
}

__global__ __launch_bounds__(MOVE_WG) void k_pso_init(PsoArgs a) {
  extern __shared__ double buf[];          // [PPB][D]
  __shared__ double nrm_s[MOVE_WG];
  __shared__ unsigned char keep[DMAX];     // with dim_sel: dimensions drawn
  const MoveGeom g = move_geom(a.D);
  const int bpn = (a.P + g.PPB - 1) / g.PPB; // blocks per node
  const int j = blockIdx.x / bpn;
  const int pl = threadIdx.x / g.Dp, dl = threadIdx.x % g.Dp;
  const int p = (blockIdx.x % bpn) * g.PPB + pl;
  const bool pv = p < a.P;
  const int D = a.D, dh = (D + 1) / 2;
  uint2 key;
  uint32_t tree;
  rng_key(a, j, &key, &tree);
  const uint32_t node = (uint32_t)a.node_id[j];
  const int64_t gid = (int64_t)j * a.P + p;
  const bool masked = a.dim_sel != nullptr;
  if (masked) {
    for (int d = threadIdx.x; d < D; d += MOVE_WG) keep[d] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < a.n_sel; i += MOVE_WG) {
      const int d = a.dim_sel[(int64_t)j * a.n_sel + i];
      if (d >= 0 && d < D) keep[d] = 1;
    }
    __syncthreads();
  }
  if (pv) {
    for (int d = dl; d < D; d += g.Dp) {
      const int m = d >> 1;
      const uint4 w = philox4x32_10(make_uint4((uint32_t)(p * dh + m), INIT_STREAM, node, tree), key);
      const double u1 = ((double)w.x + 0.5) * 0x1p-32;
      const double u2 = (double)w.y * 0x1p-32;
      const double rad = sqrt(-2.0 * log(u1));
      const double ang = 6.283185307179586 * u2;
      const double gv = (d & 1) ? rad * sin(ang) : rad * cos(ang);
      // outside the selected channels the normal is replaced by zero
      buf[pl * D + d] = masked && !keep[d] ? 0.0 : gv;
    }
  }
  __syncthreads();
  if (pv && dl == 0) nrm_s[pl] = sqrt(sq_norm_ordered(buf + pl * D, D));
  __syncthreads();
  if (!pv) return;
  const double nrm = nrm_s[pl];
  for (int d = dl; d < D; d += g.Dp) {
    const double xv = nrm > 0.0 ? buf[pl * D + d] / nrm : buf[pl * D + d];
    a.x[gid * D + d] = xv;
    a.v[gid * D + d] = 0.0;
    a.pbest[gid * D + d] = xv;
    store_w(a.W_out, a.w_bf16, gid * D + d, xv);
    if (p == 0) a.gbest[(int64_t)j * D + d] = xv;
  }
  if (dl == 0) {
    a.pbest_loss[gid] = __builtin_huge_val();
    if (a.zmin_reset) {
      a.zmin_reset[gid] = __builtin_huge_valf();
      a.zmax_reset[gid] = -__builtin_huge_valf();
    }
    if (p == 0) {
      a.gbest_loss[j] = __builtin_huge_val();
      a.gbest_p[j] = -1;
      if (a.gbest_split) a.gbest_split[j] = -1;
      if (a.gbest_thr) a.gbest_thr[j] = __builtin_huge_valf();
    }
  }
}

// (1) of the step: one work-group per node.  The argmin of the current losses
// (or of the losses eligible for the global best, gloss, when a screened
// evaluation gives them; lowest p on ties) replaces the global best iff
// strictly better; the position is copied before the move kernel changes x.  The personal bests
// are updated by the move kernel, where every particle's threads are.
constexpr int BEST_WG = 256;
constexpr int PMAX_STEP = 4096;

__global__ __launch_bounds__(BEST_WG) void k_pso_bests(PsoArgs a) {
  __shared__ double red_l[BEST_WG];
  __shared__ int red_p[BEST_WG];
  __shared__ int s_pstar, s_improved;
  const int j = blockIdx.x, tid = threadIdx.x;
  const int P = a.P, D = a.D;
  const int64_t base = (int64_t)j * P;
  double bl = __builtin_huge_val();
  int bp = 0x7fffffff;
  const double *gl = a.gloss ? a.gloss : a.loss;
  const double gold = tid == 0 ? a.gbest_loss[j] : 0.0;   // prefetched with the losses
  for (int p = tid; p < P; p += BEST_WG) {
    const double l = gl[base + p];
    if (l < bl) {
      bl = l;
      bp = p;
    }
  }
  // smallest loss, ties to the lower p: over the wave by shuffles, then over
  // the waves
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double l2 = __shfl_xor(bl, o);
    const int p2 = __shfl_xor(bp, o);
    if (l2 < bl || (l2 == bl && p2 < bp)) {
      bl = l2;
      bp = p2;
    }
  }
  if ((tid & 63) == 0) {
    red_l[tid >> 6] = bl;
    red_p[tid >> 6] = bp;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < BEST_WG / 64; ++w)
      if (red_l[w] < red_l[0] || (red_l[w] == red_l[0] && red_p[w] < red_p[0])) {
        red_l[0] = red_l[w];
        red_p[0] = red_p[w];
      }
    const int ps = red_p[0];
    const bool g = ps != 0x7fffffff && red_l[0] < gold;
    s_pstar = ps;
    s_improved = g;
    if (g) {
      a.gbest_loss[j] = red_l[0];
      a.gbest_p[j] = ps;
      if (a.gbest_split && a.split) a.gbest_split[j] = a.split[base + ps];
      if (a.gbest_thr && a.thr) a.gbest_thr[j] = a.thr[base + ps];
    }
  }
  __syncthreads();
  if (s_improved) {
    const int ps = s_pstar;
    for (int d = tid; d < D; d += BEST_WG) a.gbest[(int64_t)j * D + d] = a.x[(base + ps) * D + d];
  }
  if (a.zmin_reset) {
    for (int p = tid; p < P; p += BEST_WG) {
      a.zmin_reset[base + p] = __builtin_huge_valf();
      a.zmax_reset[base + p] = -__builtin_huge_valf();
    }
  }
}

// (2) of the step: personal bests (strict <), then with move != 0 Eq. (11),
// Eq. (12) and the unit-norm rescale.
__global__ __launch_bounds__(MOVE_WG) void k_pso_move(PsoArgs a) {
  extern __shared__ double buf[];          // [PPB][D]
  __shared__ double nrm_s[MOVE_WG];
  const MoveGeom g = move_geom(a.D);
  const int bpn = (a.P + g.PPB - 1) / g.PPB;
  const int j = blockIdx.x / bpn;
  const int pl = threadIdx.x / g.Dp, dl = threadIdx.x % g.Dp;
  const int p = (blockIdx.x % bpn) * g.PPB + pl;
  const bool pv = p < a.P;
  const int D = a.D, dh = (D + 1) / 2;
  const bool move = a.move != 0;
  // each thread reads the global-best coordinates of its own dimensions, so
  // every load of the step is independent of the others
  const double *gb = a.gbest + (int64_t)j * D;
  uint2 key;
  uint32_t tree;
  rng_key(a, j, &key, &tree);
  const uint32_t node = (uint32_t)a.node_id[j];
  const int64_t gid = (int64_t)j * a.P + p;
  const double lp = pv ? a.loss[gid] : 0.0;
  const bool imp = pv && lp < a.pbest_loss[gid];
  if (pv) {
    for (int d = dl; d < D; d += g.Dp) {
      const int64_t e = gid * D + d;
      const double xv = a.x[e];
      const double pold = a.pbest[e];   // loaded with x, before imp is known
      double pb;
      if (imp) {
        a.pbest[e] = xv;
        pb = xv;
      } else {
        pb = pold;
      }
      if (!move) continue;
      const int m = d >> 1, h = d & 1;
      const uint4 w = philox4x32_10(make_uint4((uint32_t)(p * dh + m), a.iter, node, tree), key);
      const double r1 = u24(h ? w.z : w.x);
      const double r2 = u24(h ? w.w : w.y);
      const double t0 = a.omega * a.v[e];
      const double t1 = (a.c1 * r1) * (pb - xv);
      const double t2 = (a.c2 * r2) * (gb[d] - xv);
      const double vn = (t0 + t1) + t2;
      a.v[e] = vn;
      buf[pl * D + d] = xv + vn;
    }
  }
  lds_barrier();   // every thread of the particle has read pbest_loss
  if (imp && dl == 0) a.pbest_loss[gid] = lp;
  if (!move) return;
  if (pv && dl == 0) nrm_s[pl] = sqrt(sq_norm_ordered(buf + pl * D, D));
  lds_barrier();
  if (!pv) return;
  const double nrm = nrm_s[pl];
  for (int d = dl; d < D; d += g.Dp) {
    const int64_t e = gid * D + d;
    // x + v == 0 exactly means x == -v: keep the previous position
    const double xv = nrm > 0.0 ? buf[pl * D + d] / nrm : -a.v[e];
    a.x[e] = xv;
    store_w(a.W_out, a.w_bf16, e, xv);
  }
}

// Candidates of the probabilistic search (Sec. II-B, Eqs. (5)-(8)): particle
// p of node j combines the node's R first-ranked features (ranks[j R + d],
// most discriminant first) with integer coefficients.  One Philox4x32-10 call
// per (p, rank d), counter (p R + d, 0x40000000 + t, node id, tree): rank d is
// used iff u24(w0) < pd[d], with coefficient k + 1 (k < m) or -(k - m + 1),
// k = floor(u24(w1) 2m), m = amax[d]; a draw that uses no rank takes +1 on
// rank 1.  x = c / sqrt(sum c^2): the squared norm of the integers is exact,
// so every coordinate is one correctly rounded division.  One thread per
// (node, particle); x and its image W_out are written in full (zeros
// elsewhere).

__global__ void k_ps_candidates(PsoArgs a, const int32_t *ranks, int R, const double *pd,
                                const int32_t *amax, uint32_t t) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)a.n_nodes * a.P) return;
  const int j = (int)(gid / a.P), p = (int)(gid % a.P);
  const int D = a.D;
  uint2 key;
  uint32_t tree;
  rng_key(a, j, &key, &tree);
  const uint32_t node = (uint32_t)a.node_id[j];
  // coefficient of rank d (recomputed in the second pass: no private array)
  auto coef = [&](int d) {
    const uint4 w = philox4x32_10(make_uint4((uint32_t)(p * R + d), PS_STREAM + t, node, tree), key);
    const int m = amax[d];
    const int k = (int)floor(u24(w.y) * (2.0 * m));
    return u24(w.x) < pd[d] ? (k < m ? k + 1 : -(k - m + 1)) : 0;
  };
  int64_t s = 0;
  for (int d = 0; d < R; ++d) {
    const int64_t v = coef(d);
    s += v * v;
  }
  const bool none = s == 0;   // no rank used: +1 on rank 1
  const double nrm = none ? 1.0 : sqrt((double)s);
  double *xr = a.x + gid * D;
  for (int dd = 0; dd < D; ++dd) {
    xr[dd] = 0.0;
    store_w(a.W_out, a.w_bf16, gid * D + dd, 0.0);
  }
  for (int d = 0; d < R; ++d) {
    const int col = ranks[(int64_t)j * R + d];
    const int v = none ? (d == 0 ? 1 : 0) : coef(d);
    if (col < 0 || col >= D || v == 0) continue;
    const double xv = (double)v / nrm;
    xr[col] = xv;
    store_w(a.W_out, a.w_bf16, gid * D + col, xv);
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

void prepare_pso_kernels(int lds_max) {
  const int dyn = lds_max - 4096;
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_pso_move),
                          hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess)
    (void)hipGetLastError();
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_pso_init),
                          hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess)
    (void)hipGetLastError();
}

slm_status launch_pso_init(const PsoArgs &a, hipStream_t s) {
  SLM_CHECK(a.D <= DMAX, SLM_E_SHAPE, "slm_pso_init: D = %d exceeds %d", a.D, DMAX);
  if ((int64_t)a.n_nodes * a.P == 0) return SLM_OK;
  const MoveGeom g = move_geom(a.D);
  const int64_t grid = (int64_t)a.n_nodes * ((a.P + g.PPB - 1) / g.PPB);
  const size_t lds = (size_t)g.PPB * a.D * sizeof(double);
  hipLaunchKernelGGL(k_pso_init, dim3((unsigned)grid), dim3(MOVE_WG), lds, s, a);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_pso_step(const PsoArgs &a, hipStream_t s) {
  SLM_CHECK(a.D <= DMAX, SLM_E_SHAPE, "slm_pso_step: D = %d exceeds %d", a.D, DMAX);
  SLM_CHECK(a.P <= PMAX_STEP, SLM_E_SHAPE, "slm_pso_step: P = %d exceeds %d", a.P, PMAX_STEP);
  if (a.n_nodes == 0) return SLM_OK;
  hipLaunchKernelGGL(k_pso_bests, dim3((unsigned)a.n_nodes), dim3(BEST_WG), 0, s, a);
  SLM_LAUNCHED();
  if (a.bests_only) return SLM_OK;
  const MoveGeom g = move_geom(a.D);
  const int64_t grid = (int64_t)a.n_nodes * ((a.P + g.PPB - 1) / g.PPB);
  const size_t lds = (size_t)g.PPB * a.D * sizeof(double);
  hipLaunchKernelGGL(k_pso_move, dim3((unsigned)grid), dim3(MOVE_WG), lds, s, a);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_ps_candidates(const PsoArgs &a, const int32_t *ranks, int R, const double *pd,
                                const int32_t *amax, uint32_t t, hipStream_t s) {
  SLM_CHECK(R >= 1 && R <= PS_RMAX && R <= a.D, SLM_E_SHAPE,
            "probabilistic search: R = %d not in [1, min(D, %d)]", R, PS_RMAX);
  const int64_t n = (int64_t)a.n_nodes * a.P;
  if (n == 0) return SLM_OK;
  hipLaunchKernelGGL(k_ps_candidates, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, a,
                     ranks, R, pd, amax, t);
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
