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

#include <algorithm>

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
      if (a.apso_state) {   // the adaptive swarm starts exploring with c1 = c2 = 2
        a.apso_state[j] = 1;
        a.apso_par[(int64_t)j * 3 + 0] = 0.9;
        a.apso_par[(int64_t)j * 3 + 1] = 2.0;
        a.apso_par[(int64_t)j * 3 + 2] = 2.0;
      }
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
  const double *gl_in = a.gbest_loss_in ? a.gbest_loss_in : a.gbest_loss;
  const double gold = tid == 0 ? gl_in[j] : 0.0;   // prefetched with the losses
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
    } else if (a.gbest_loss_in) {
      a.gbest_loss[j] = gold;   // carried over from the input record
    }
  }
  __syncthreads();
  if (s_improved) {
    const int ps = s_pstar;
    for (int d = tid; d < D; d += BEST_WG) a.gbest[(int64_t)j * D + d] = a.x[(base + ps) * D + d];
  } else if (a.gbest_in) {
    for (int d = tid; d < D; d += BEST_WG)
      a.gbest[(int64_t)j * D + d] = a.gbest_in[(int64_t)j * D + d];
  }
  if (a.zmin_reset) {
    for (int p = tid; p < P; p += BEST_WG) {
      a.zmin_reset[base + p] = __builtin_huge_valf();
      a.zmax_reset[base + p] = -__builtin_huge_valf();
    }
  }
}

// ---------------------------------------------------------------- adaptive swarm
// APSO (Sec. III-B; the state estimation and the changes as in the APSO
// reference): between the bests and the move, every node estimates its
// evolutionary state from the particles' mean distances, changes c1, c2 and
// the inertia weight with the state, and in the convergence state prepares an
// elitist-learning candidate that replaces its worst particle after the move.
constexpr int AD_KC = 16;         // dimensions per LDS chunk
constexpr uint32_t APSO_STREAM = 0x20000000u;

// Partial sums of ||x_i - x_j|| over the j of one particle tile, for the i of
// another: work-group (node, i tile, j tile) of 256 threads (16 x 16), each an
// MT x MT block of pairs (tiles of 16 MT particles); dimensions staged through
// LDS 16 at a time.  part[(node P + i) * ceil(P / 16) + j tile].  Few nodes
// take small tiles (enough work-groups to fill the chip), many nodes large
// ones (fewer LDS reads per pair).
template <int MT>
__global__ __launch_bounds__(256) void k_apso_dist(PsoArgs a) {
  constexpr int TL = 16 * MT;
  __shared__ double xi[TL][AD_KC + 1], xj[TL][AD_KC + 1];
  const int P = a.P, D = a.D, nb = (P + TL - 1) / TL, stride = (P + 15) / 16;
  const int blk = blockIdx.x;
  const int j = blk / (nb * nb), bi = (blk / nb) % nb, bj = blk % nb;
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  const int64_t base = (int64_t)j * P;
  double acc[MT][MT];
#pragma unroll
  for (int r = 0; r < MT; ++r)
#pragma unroll
    for (int c = 0; c < MT; ++c) acc[r][c] = 0.0;
  for (int d0 = 0; d0 < D; d0 += AD_KC) {
#pragma unroll
    for (int k = 0; k < MT; ++k) {
      const int e = tid + 256 * k, row = e / AD_KC, col = e % AD_KC;
      const int i = bi * TL + row, jj = bj * TL + row, d = d0 + col;
      xi[row][col] = i < P && d < D ? a.x[(base + i) * D + d] : 0.0;
      xj[row][col] = jj < P && d < D ? a.x[(base + jj) * D + d] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < AD_KC; ++k) {
      double u[MT], w[MT];
#pragma unroll
      for (int r = 0; r < MT; ++r) u[r] = xi[ti * MT + r][k];
#pragma unroll
      for (int c = 0; c < MT; ++c) w[c] = xj[tj * MT + c][k];
#pragma unroll
      for (int r = 0; r < MT; ++r)
#pragma unroll
        for (int c = 0; c < MT; ++c) {
          const double df = u[r] - w[c];
          acc[r][c] = acc[r][c] + df * df;
        }
    }
    __syncthreads();
  }
  // row sums over this thread's MT columns, then over the 16 column groups in
  // a fixed order (the LDS of the staging is reused)
  double *red = &xi[0][0];   // [TL rows][16 groups] fits in xi
#pragma unroll
  for (int r = 0; r < MT; ++r) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < MT; ++c)
      if (bj * TL + tj * MT + c < P) s = s + sqrt(acc[r][c]);
    red[(ti * MT + r) * 16 + tj] = s;
  }
  __syncthreads();
  if (tid < TL) {
    const int i = bi * TL + tid;
    if (i < P) {
      double s = 0.0;
      for (int g = 0; g < 16; ++g) s = s + red[tid * 16 + g];
      a.apso_part[(base + i) * stride + bj] = s;
    }
  }
}

// micro-tile of the distance kernel: the largest whose grid still has 512
// work-groups (1 when none has)
__host__ __device__ __forceinline__ int apso_mt(int n_nodes, int P) {
  for (int mt = 4; mt > 1; mt >>= 1) {
    const int64_t nb = (P + 16 * mt - 1) / (16 * mt);
    if ((int64_t)n_nodes * nb * nb >= 512) return mt;
  }
  return 1;
}

__device__ __forceinline__ double apso_mu(int s, double f) {
  switch (s) {
    case 1:   // exploration
      return f <= 0.4 ? 0.0 : f <= 0.6 ? 5.0 * f - 2.0 : f <= 0.7 ? 1.0 : f <= 0.8 ? -10.0 * f + 8.0 : 0.0;
    case 2:   // exploitation
      return f <= 0.2 ? 0.0 : f <= 0.3 ? 10.0 * f - 2.0 : f <= 0.4 ? 1.0 : f <= 0.6 ? -5.0 * f + 3.0 : 0.0;
    case 3:   // convergence
      return f <= 0.1 ? 1.0 : f <= 0.3 ? -5.0 * f + 1.5 : 0.0;
    default:  // jumping-out
      return f <= 0.7 ? 0.0 : f <= 0.9 ? 5.0 * f - 3.5 : 1.0;
  }
}

// One work-group per node: mean distances d_i, f = (d_g - d_min) / (d_max -
// d_min) (g = the global best's particle; f = 0 if d_max = d_min), the state
// (kept while its membership is positive, else the largest membership, lower
// state on ties), inertia 1 / (1 + 1.5 exp(-2.6 f)), c1 / c2 changed by
// delta ~ U[0.05, 0.1] (half in exploitation and convergence), clamped to
// [1.5, 2.5] and scaled to sum 4; the worst particle (highest loss, NaN as
// +inf, lowest index on ties); in convergence the elite candidate: one
// coordinate of the global best moved by 2 sigma N(0, 1), sigma = 1 - 0.9 t/T,
// scaled to unit norm (with apso_sel, the coordinate is one of the node's
// listed channels).  Draws: Philox counters (0 | 1, APSO_STREAM + t, node,
// tree).
__global__ __launch_bounds__(256) void k_apso_adapt(PsoArgs a) {
  __shared__ double s_mn[4], s_mx[4], s_wl[4], s_dg, s_nrm;
  __shared__ int s_wp[4], s_dim, s_state;
  __shared__ double e[DMAX];
  const int j = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int P = a.P, D = a.D, stride = (P + 15) / 16;
  const int nb = (P + 16 * apso_mt(a.n_nodes, P) - 1) / (16 * apso_mt(a.n_nodes, P));
  const int64_t base = (int64_t)j * P;
  const int g = max(0, a.gbest_p[j]);
  double mn = __builtin_huge_val(), mx = -__builtin_huge_val(), wl = -__builtin_huge_val();
  int wp = 0x7fffffff;
  for (int i = tid; i < P; i += 256) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s = s + a.apso_part[(base + i) * stride + b];
    const double di = s / (double)(P - 1);
    a.apso_dist[base + i] = di;
    mn = fmin(mn, di);
    mx = fmax(mx, di);
    if (i == g) s_dg = di;
    double l = a.loss[base + i];
    if (l != l) l = __builtin_huge_val();
    if (l > wl || (l == wl && i < wp)) {
      wl = l;
      wp = i;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o));
    mx = fmax(mx, __shfl_xor(mx, o));
    const double l2 = __shfl_xor(wl, o);
    const int p2 = __shfl_xor(wp, o);
    if (l2 > wl || (l2 == wl && p2 < wp)) {
      wl = l2;
      wp = p2;
    }
  }
  if (lane == 0) {
    s_mn[wv] = mn;
    s_mx[wv] = mx;
    s_wl[wv] = wl;
    s_wp[wv] = wp;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 4; ++w) {
      mn = fmin(mn, s_mn[w]);
      mx = fmax(mx, s_mx[w]);
      if (s_wl[w] > wl || (s_wl[w] == wl && s_wp[w] < wp)) {
        wl = s_wl[w];
        wp = s_wp[w];
      }
    }
    const double f = mx > mn ? (s_dg - mn) / (mx - mn) : 0.0;
    const int prev = a.apso_state[j];
    int st = prev;
    if (!(prev >= 1 && prev <= 4 && apso_mu(prev, f) > 0.0)) {
      st = 1;
      for (int q = 2; q <= 4; ++q)
        if (apso_mu(q, f) > apso_mu(st, f)) st = q;
    }
    uint2 key;
    uint32_t tree;
    rng_key(a, j, &key, &tree);
    const uint32_t node = (uint32_t)a.node_id[j];
    const uint4 w0 = philox4x32_10(make_uint4(0u, APSO_STREAM + a.iter, node, tree), key);
    const double d1 = 0.05 + 0.05 * u24(w0.x), d2 = 0.05 + 0.05 * u24(w0.y);
    double c1 = a.apso_par[(int64_t)j * 3 + 1], c2 = a.apso_par[(int64_t)j * 3 + 2];
    if (st == 1) {
      c1 = c1 + d1;
      c2 = c2 - d2;
    } else if (st == 2) {
      c1 = c1 + 0.5 * d1;
      c2 = c2 - 0.5 * d2;
    } else if (st == 3) {
      c1 = c1 + 0.5 * d1;
      c2 = c2 + 0.5 * d2;
    } else {
      c1 = c1 - d1;
      c2 = c2 + d2;
    }
    c1 = fmin(fmax(c1, 1.5), 2.5);
    c2 = fmin(fmax(c2, 1.5), 2.5);
    if (c1 + c2 > 4.0) {
      const double sc = 4.0 / (c1 + c2);
      c1 = c1 * sc;
      c2 = c2 * sc;
    }
    a.apso_par[(int64_t)j * 3 + 0] = 1.0 / (1.0 + 1.5 * exp(-2.6 * f));
    a.apso_par[(int64_t)j * 3 + 1] = c1;
    a.apso_par[(int64_t)j * 3 + 2] = c2;
    a.apso_state[j] = st;
    a.apso_f[j] = f;
    a.apso_worst[j] = wp == 0x7fffffff ? 0 : wp;
    s_state = st;
    if (a.apso_sel && a.apso_n_sel > 0) {
      const int k = (int)(((uint64_t)w0.z * (uint64_t)a.apso_n_sel) >> 32);
      const int dsel = a.apso_sel[(int64_t)j * a.apso_n_sel + k];
      s_dim = dsel >= 0 && dsel < D ? dsel : 0;
    } else {
      s_dim = (int)(((uint64_t)w0.z * (uint64_t)D) >> 32);
    }
    if (st == 3) {
      const uint4 w1 = philox4x32_10(make_uint4(1u, APSO_STREAM + a.iter, node, tree), key);
      const double u1 = ((double)w1.x + 0.5) * 0x1p-32;
      const double u2 = (double)w1.y * 0x1p-32;
      const double gv = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
      const double sig = 1.0 - (1.0 - 0.1) * ((double)a.iter / (double)max(1u, a.apso_T));
      s_nrm = (2.0 * sig) * gv;   // the step, until the norm is known
    }
  }
  __syncthreads();
  if (s_state != 3) return;
  const double *gb = a.gbest + (int64_t)j * D;
  for (int d = tid; d < D; d += 256) e[d] = d == s_dim ? gb[d] + s_nrm : gb[d];
  __syncthreads();
  if (tid == 0) s_nrm = sqrt(sq_norm_ordered(e, D));
  __syncthreads();
  const double nrm = s_nrm;
  for (int d = tid; d < D; d += 256)
    a.apso_elite[(int64_t)j * D + d] = nrm > 0.0 ? e[d] / nrm : gb[d];
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
  // the adaptive swarm's parameters of this node, and the particle its elite
  // candidate replaces (convergence state)
  const bool ap = a.apso_state != nullptr;
  const double omega = ap ? a.apso_par[(int64_t)j * 3 + 0] : a.omega;
  const double c1 = ap ? a.apso_par[(int64_t)j * 3 + 1] : a.c1;
  const double c2 = ap ? a.apso_par[(int64_t)j * 3 + 2] : a.c2;
  const bool el = ap && a.apso_state[j] == 3 && p == a.apso_worst[j];
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
      const double t0 = omega * a.v[e];
      const double t1 = (c1 * r1) * (pb - xv);
      const double t2 = (c2 * r2) * (gb[d] - xv);
      const double vn = (t0 + t1) + t2;
      a.v[e] = el ? 0.0 : vn;
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
    const double xv = el ? a.apso_elite[(int64_t)j * D + d]
                         : (nrm > 0.0 ? buf[pl * D + d] / nrm : -a.v[e]);
    a.x[e] = xv;
    store_w(a.W_out, a.w_bf16, e, xv);
  }
}

// Bests and move in one launch (the plain swarm): every work-group of node j
// finds the node's argmin over the P losses itself (lowest p on ties), so the
// global best it moves towards is x_in[p*] when that improves on the input
// record, else the input record; work-group 0 of the node writes the new
// record to gbest / gbest_loss (other buffers than the ones read), the
// positions move from x_in to x.  Same arithmetic as k_pso_bests followed by
// k_pso_move.
__global__ __launch_bounds__(MOVE_WG) void k_pso_fused(PsoArgs a) {
  extern __shared__ double buf[];          // [PPB][D]
  __shared__ double nrm_s[MOVE_WG];
  __shared__ double red_l[MOVE_WG / 64];
  __shared__ int red_p[MOVE_WG / 64];
  const MoveGeom g = move_geom(a.D);
  const int bpn = (a.P + g.PPB - 1) / g.PPB;
  const int j = blockIdx.x / bpn, blk = blockIdx.x % bpn;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int pl = tid / g.Dp, dl = tid % g.Dp;
  const int p = blk * g.PPB + pl;
  const bool pv = p < a.P;
  const int D = a.D, dh = (D + 1) / 2, P = a.P;
  const int64_t base = (int64_t)j * P;
  // the node's argmin
  double bl = __builtin_huge_val();
  int bp = 0x7fffffff;
  for (int q = tid; q < P; q += MOVE_WG) {
    const double l = a.loss[base + q];
    if (l < bl) {
      bl = l;
      bp = q;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double l2 = __shfl_xor(bl, o);
    const int p2 = __shfl_xor(bp, o);
    if (l2 < bl || (l2 == bl && p2 < bp)) {
      bl = l2;
      bp = p2;
    }
  }
  if (lane == 0) {
    red_l[wv] = bl;
    red_p[wv] = bp;
  }
  const double gold = a.gbest_loss_in[j];
  lds_barrier();
  bl = red_l[0];
  bp = red_p[0];
#pragma unroll
  for (int w = 1; w < MOVE_WG / 64; ++w)
    if (red_l[w] < bl || (red_l[w] == bl && red_p[w] < bp)) {
      bl = red_l[w];
      bp = red_p[w];
    }
  const bool improved = bp != 0x7fffffff && bl < gold;
  const double *gsrc = improved ? a.x_in + (base + bp) * D : a.gbest_in + (int64_t)j * D;
  if (blk == 0) {
    for (int d = tid; d < D; d += MOVE_WG) a.gbest[(int64_t)j * D + d] = gsrc[d];
    if (tid == 0) {
      a.gbest_loss[j] = improved ? bl : gold;
      if (improved) {
        a.gbest_p[j] = bp;
        if (a.gbest_split && a.split) a.gbest_split[j] = a.split[base + bp];
        if (a.gbest_thr && a.thr) a.gbest_thr[j] = a.thr[base + bp];
      }
    }
  }
  if (a.zmin_reset && pv && dl == 0) {
    a.zmin_reset[base + p] = __builtin_huge_valf();
    a.zmax_reset[base + p] = -__builtin_huge_valf();
  }
  uint2 key;
  uint32_t tree;
  rng_key(a, j, &key, &tree);
  const uint32_t node = (uint32_t)a.node_id[j];
  const int64_t gid = base + p;
  const double lp = pv ? a.loss[gid] : 0.0;
  const bool imp = pv && lp < a.pbest_loss[gid];
  if (pv) {
    for (int d = dl; d < D; d += g.Dp) {
      const int64_t e = gid * D + d;
      const double xv = a.x_in[e];
      const double pold = a.pbest[e];
      double pb;
      if (imp) {
        a.pbest[e] = xv;
        pb = xv;
      } else {
        pb = pold;
      }
      const int m = d >> 1, h = d & 1;
      const uint4 w = philox4x32_10(make_uint4((uint32_t)(p * dh + m), a.iter, node, tree), key);
      const double r1 = u24(h ? w.z : w.x);
      const double r2 = u24(h ? w.w : w.y);
      const double t0 = a.omega * a.v[e];
      const double t1 = (a.c1 * r1) * (pb - xv);
      const double t2 = (a.c2 * r2) * (gsrc[d] - xv);
      const double vn = (t0 + t1) + t2;
      a.v[e] = vn;
      buf[pl * D + d] = xv + vn;
    }
  }
  lds_barrier();
  if (imp && dl == 0) a.pbest_loss[gid] = lp;
  if (pv && dl == 0) nrm_s[pl] = sqrt(sq_norm_ordered(buf + pl * D, D));
  lds_barrier();
  if (!pv) return;
  const double nrm = nrm_s[pl];
  for (int d = dl; d < D; d += g.Dp) {
    const int64_t e = gid * D + d;
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

// Tables of the probabilistic search over R ranks (Eq. (8), reading of this
// build): A_d = alpha0 exp(-alpha d), alpha = ln(alpha0) / (R - 1), so A falls
// from alpha0 at the first rank (d = 0) to 1 at the last; the selection
// probability is A_d / alpha0 and the coefficient range floor(A_d) (at least 1;
// the 1e-9 keeps a rounded A just below an integer on it).
__global__ void k_ps_tables(int R, double alpha0, double *pd, int32_t *amax) {
  const int d = threadIdx.x;
  if (d >= R) return;
  const double alpha = R > 1 ? log(alpha0) / (double)(R - 1) : 0.0;
  const double A = alpha0 * exp(-(alpha * (double)d));
  pd[d] = A / alpha0;
  const double f = floor(A + 1e-9);
  amax[d] = f < 1.0 ? 1 : (int32_t)f;
}

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
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_pso_fused),
                          hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess)
    (void)hipGetLastError();
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_pso_move),
                          hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess)
    (void)hipGetLastError();
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_pso_init),
                          hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess)
    (void)hipGetLastError();
}

slm_status launch_pso_fused(const PsoArgs &a, hipStream_t s) {
  SLM_CHECK(a.D <= DMAX, SLM_E_SHAPE, "pso step: D = %d exceeds %d", a.D, DMAX);
  SLM_CHECK(a.x_in && a.gbest_in && a.gbest_loss_in && !a.gloss && !a.apso_state && a.move,
            SLM_E_INVALID, "pso step: fused step needs its input buffers");
  if (a.n_nodes == 0) return SLM_OK;
  const MoveGeom g = move_geom(a.D);
  const int64_t grid = (int64_t)a.n_nodes * ((a.P + g.PPB - 1) / g.PPB);
  const size_t lds = (size_t)g.PPB * a.D * sizeof(double);
  hipLaunchKernelGGL(k_pso_fused, dim3((unsigned)grid), dim3(MOVE_WG), lds, s, a);
  SLM_LAUNCHED();
  return SLM_OK;
}

size_t apso_part_bytes(int n_nodes, int P) {
  return (size_t)std::max(0, n_nodes) * std::max(0, P) * ((std::max(0, P) + 15) / 16) *
         sizeof(double);
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
  if (a.apso_state && a.move) {
    SLM_CHECK(a.P >= 2, SLM_E_SHAPE, "apso: P = %d (at least 2 particles)", a.P);
    const int mt = apso_mt(a.n_nodes, a.P), nb = (a.P + 16 * mt - 1) / (16 * mt);
    const dim3 grid((unsigned)((int64_t)a.n_nodes * nb * nb));
    if (mt == 4) hipLaunchKernelGGL(k_apso_dist<4>, grid, dim3(256), 0, s, a);
    else if (mt == 2) hipLaunchKernelGGL(k_apso_dist<2>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_apso_dist<1>, grid, dim3(256), 0, s, a);
    SLM_LAUNCHED();
    hipLaunchKernelGGL(k_apso_adapt, dim3((unsigned)a.n_nodes), dim3(256), 0, s, a);
    SLM_LAUNCHED();
  }
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

slm_status launch_ps_tables(int R, double alpha0, double *pd, int32_t *amax, hipStream_t s) {
  hipLaunchKernelGGL(k_ps_tables, dim3(1), dim3(PS_RMAX), 0, s, R, alpha0, pd, amax);
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
