// Best threshold of every projected feature (Sec. II-A, Eqs. (3)-(4);
// Sec. III-B: a direction's loss is the loss of its best threshold).
//
// Histogram scan.  A work-group owns (item, particle tile): the rows of one
// node inside one global chunk of CH rows, and PT particles of that node.
// Lanes map to (row, particle): lane = rsub * PT + pl, so a wave reads
// 64 / PT row segments of PT consecutive floats of Z (row-major [N, P]) and
// each lane bins its own particle's value.  Counts go to LDS histograms laid
// out [bin][class][PT], so lanes of one row touch PT consecutive words.
//   * A node inside one chunk is finished by the same work-group: it scans
//     the histogram in LDS and writes (split, loss, threshold) per particle.
//   * A node spanning several chunks adds its histogram into a global
//     accumulator slot (the node's first chunk index identifies the slot),
//     and the last work-group to arrive (atomic ticket) loads the total,
//     zeroes the slot and ticket for the next call, and finishes the scan.
// Finishing one particle is one wave: each lane holds 4 consecutive bins,
// class prefixes come from wave shuffles, each lane evaluates the criterion
// at its 4 candidate splits in FP64 and a butterfly argmin (smallest split on
// ties) picks the best.
//
// Exact scan.  One work-group per (node, particle): bitonic sort of the
// node's (z, row) pairs in LDS (stable through the row tie-break), then a
// block scan of class counts (or FP64 sums of y, y^2) and the criterion at
// every boundary between distinct values.
#include "slm_internal.hpp"

#include <algorithm>
#include <mutex>

namespace slm {
namespace {

constexpr int WG = 256;

// ---------------------------------------------------------------- binning
struct BinRule {
  float zmin, delta, inv;
  int B;
  bool flat;   // delta == 0 (zmax == zmin or underflow): every edge equals zmin
};

__device__ __forceinline__ BinRule make_rule(float zmin, float zmax, int B) {
  BinRule r;
  const float range = __fsub_rn(zmax, zmin);
  r.zmin = zmin;
  r.delta = __fdiv_rn(range, (float)B);
  r.inv = (float)B / range;
  r.B = B;
  r.flat = !(r.delta > 0.0f);
  return r;
}

__device__ __forceinline__ float edge(const BinRule &r, int j) {
  return __fadd_rn(r.zmin, __fmul_rn((float)j, r.delta));
}

// bin(z) = #{ j in 1..B-1 : e_j <= z }.  A guess from (z - zmin) / delta is
// corrected against the exact float32 edges; the edges are non-decreasing,
// so the loops stop at the exact count.
__device__ __forceinline__ int bin_of(const BinRule &r, float z) {
  if (r.flat) return r.B - 1;
  int g = (int)((z - r.zmin) * r.inv);
  g = g < 0 ? 0 : (g > r.B - 1 ? r.B - 1 : g);
  while (g >= 1 && edge(r, g) > z) --g;
  while (g + 1 <= r.B - 1 && edge(r, g + 1) <= z) ++g;
  return g;
}

// ---------------------------------------------------------------- wave helpers
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  return x;
}

__device__ __forceinline__ void wave_argmin(double &l, int &b) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double l2 = __shfl_xor(l, o);
    const int b2 = __shfl_xor(b, o);
    if (l2 < l || (l2 == l && b2 < b)) {
      l = l2;
      b = b2;
    }
  }
}

__device__ __forceinline__ double nlog2n(double x) { return x > 0.0 ? x * log2(x) : 0.0; }

// ---------------------------------------------------------------- plan
struct Plan {
  int PT;       // particles per work-group
  int64_t CH;   // rows per global chunk
  int G;        // particle tiles sharing one 128-byte line of a Z row
};

int64_t chunk_min(int64_t N) {
  int64_t c = std::max<int64_t>(2048, (N + 255) / 256);
  return (c + 63) / 64 * 64;
}

Plan make_plan(int64_t N, int n_nodes, int P, int B, int K, int crit) {
  const int64_t per_particle = crit == SLM_MSE ? (int64_t)B * 20 : (int64_t)B * K * 4;
  int PT = 32;
  while (PT > 4 && PT * per_particle > 96 * 1024) PT >>= 1;
  while (PT > 4 && PT / 2 >= P) PT >>= 1;
  // few, large nodes: narrower particle tiles give more work-groups
  const int64_t n_pt = (P + PT - 1) / PT;
  const int64_t cmin = chunk_min(N);
  int64_t CH = cmin;
  const int64_t blocks = (num_items(n_nodes, N, CH)) * n_pt;
  if (blocks > 4096) {
    // plenty of parallelism: larger chunks cut accumulator traffic
    CH = std::min<int64_t>(65536, cmin * std::max<int64_t>(1, blocks / 4096));
    CH = (CH + 63) / 64 * 64;
  }
  Plan pl{PT, CH, std::max(1, 32 / PT)};
  return pl;
}

size_t lds_bytes(int PT, int B, int K, bool mse) {
  if (mse) return (size_t)B * PT * 4 + (size_t)B * PT * 16 + 16;
  return (size_t)B * K * PT * 4;
}

size_t slot_bytes(int PT, int B, int K, bool mse) {
  size_t b = mse ? (size_t)B * PT * 4 : (size_t)B * K * PT * 4;
  b = (b + 255) / 256 * 256;
  if (mse) b += (size_t)B * PT * 16;
  return (b + 255) / 256 * 256;
}

// ---------------------------------------------------------------- histogram kernel
template <int PT, bool MSE>
__global__ __launch_bounds__(WG) void k_scan_hist(ScanArgs a, int64_t CH, int n_pt, int G,
                                                  int64_t total_blocks, size_t slot_sz,
                                                  int64_t n_slots) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_last;
  const int B = a.bins;
  const int K = MSE ? 1 : a.K;
  const int HB = B * K;
  uint32_t *hc = reinterpret_cast<uint32_t *>(smem);
  double *hs1 = nullptr, *hs2 = nullptr;
  if constexpr (MSE) {
    hs1 = reinterpret_cast<double *>(smem + (((size_t)B * PT * 4 + 15) / 16) * 16);
    hs2 = hs1 + (size_t)B * PT;
  }

  // XCD-aware order: the G particle tiles that share a Z cache line get
  // block ids congruent modulo 8, dispatched close together.
  const int64_t b = blockIdx.x;
  const int64_t hi8 = b / (8 * G), rem = b % (8 * G);
  const int64_t L = ((hi8 * 8 + rem % 8) * G) + rem / 8;
  if (L >= total_blocks) return;
  const int64_t v = L / n_pt;
  const int pt = (int)(L % n_pt);
  const Item it = find_item(a.beg, a.end, a.n_nodes, a.N, CH, v);
  if (it.node < 0) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < HB * PT; i += WG) hc[i] = 0u;
  if constexpr (MSE) {
    for (int i = tid; i < B * PT; i += WG) {
      hs1[i] = 0.0;
      hs2[i] = 0.0;
    }
  }

  constexpr int RPW = 64 / PT;                 // rows per wave step
  const int pl = lane % PT, rsub = lane / PT;
  const int P = a.P;
  const int p = pt * PT + pl;
  const bool pv = p < P;
  const int64_t np = (int64_t)it.node * P;
  BinRule rule = make_rule(pv ? a.zmin[np + p] : 0.f, pv ? a.zmax[np + p] : 0.f, B);
  __syncthreads();

  // ---- accumulate
  const int64_t step = (int64_t)(WG / 64) * RPW;
  int64_t row = it.lo + wave * RPW + rsub;
  constexpr int U = 4;
  for (; row + (U - 1) * step < it.hi; row += U * step) {
    float z[U];
    int lab[U];
    double yv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t rr = row + u * step;
      z[u] = pv ? a.Z[rr * P + p] : 0.f;
      if constexpr (MSE) yv[u] = a.y[rr];
      else lab[u] = a.labels[rr];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!pv) continue;
      const int bn = bin_of(rule, z[u]);
      if constexpr (MSE) {
        atomicAdd(&hc[bn * PT + pl], 1u);
        unsafeAtomicAdd(&hs1[bn * PT + pl], yv[u]);
        unsafeAtomicAdd(&hs2[bn * PT + pl], yv[u] * yv[u]);
      } else {
        if ((unsigned)lab[u] < (unsigned)K) atomicAdd(&hc[(bn * K + lab[u]) * PT + pl], 1u);
      }
    }
  }
  for (; row < it.hi; row += step) {
    if (!pv) continue;
    const float z = a.Z[row * P + p];
    const int bn = bin_of(rule, z);
    if constexpr (MSE) {
      const double yv = a.y[row];
      atomicAdd(&hc[bn * PT + pl], 1u);
      unsafeAtomicAdd(&hs1[bn * PT + pl], yv);
      unsafeAtomicAdd(&hs2[bn * PT + pl], yv * yv);
    } else {
      const int lab = a.labels[row];
      if ((unsigned)lab < (unsigned)K) atomicAdd(&hc[(bn * K + lab) * PT + pl], 1u);
    }
  }
  __syncthreads();

  // ---- merge chunks of a node spanning several of them
  if (it.nchunks > 1) {
    const Range nr = load_range(a.beg, a.end, it.node, a.N);
    const int64_t slot = nr.lo / CH;
    if (slot >= n_slots) return;   // cannot happen with a workspace sized by the plan
    unsigned char *base = static_cast<unsigned char *>(a.ws) + (size_t)(slot * n_pt + pt) * slot_sz;
    uint32_t *gc = reinterpret_cast<uint32_t *>(base);
    const size_t cnt_bytes = ((MSE ? (size_t)B * PT * 4 : (size_t)HB * PT * 4) + 255) / 256 * 256;
    double *gs = reinterpret_cast<double *>(base + cnt_bytes);
    uint32_t *tickets = reinterpret_cast<uint32_t *>(static_cast<unsigned char *>(a.ws) +
                                                     (size_t)n_slots * n_pt * slot_sz);
    const int ncnt = MSE ? B * PT : HB * PT;
    for (int i = tid; i < ncnt; i += WG) {
      const uint32_t c = hc[i];
      if (c) {
        atomicAdd(&gc[i], c);
        if constexpr (MSE) {
          unsafeAtomicAdd(&gs[i], hs1[i]);
          unsafeAtomicAdd(&gs[(size_t)B * PT + i], hs2[i]);
        }
      }
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) {
      const unsigned t = atomicAdd(&tickets[slot * n_pt + pt], 1u);
      s_last = (t == (unsigned)(it.nchunks - 1));
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    for (int i = tid; i < ncnt; i += WG) {
      hc[i] = __hip_atomic_load(&gc[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      gc[i] = 0u;
      if constexpr (MSE) {
        hs1[i] = __hip_atomic_load(&gs[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        hs2[i] = __hip_atomic_load(&gs[(size_t)B * PT + i], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        gs[i] = 0.0;
        gs[(size_t)B * PT + i] = 0.0;
      }
    }
    if (tid == 0) tickets[slot * n_pt + pt] = 0u;
    __syncthreads();
  }

  // ---- finish: one wave per particle
  for (int q = wave; q < PT; q += WG / 64) {
    const int pp = pt * PT + q;
    const bool active = pp < P;
    const int64_t out = np + pp;
    const BinRule rr = make_rule(active ? a.zmin[out] : 0.f, active ? a.zmax[out] : 0.f, B);
    const int b0 = lane * 4;
    if (active && a.hist_out) {
      for (int bb = b0; bb < b0 + 4 && bb < B; ++bb)
        for (int k = 0; k < K; ++k)
          a.hist_out[(out * B + bb) * K + k] = hc[(bb * K + k) * PT + q];
    }
    if constexpr (MSE) {
      if (active && a.sums_out) {
        for (int bb = b0; bb < b0 + 4 && bb < B; ++bb) {
          a.sums_out[(out * B + bb) * 2] = hs1[bb * PT + q];
          a.sums_out[(out * B + bb) * 2 + 1] = hs2[bb * PT + q];
        }
      }
    }
    // inclusive prefixes over bins, in place
    for (int k = 0; k < K; ++k) {
      uint32_t c[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) c[u] = (b0 + u < B) ? hc[((b0 + u) * K + k) * PT + q] : 0u;
      c[1] += c[0];
      c[2] += c[1];
      c[3] += c[2];
      const uint32_t excl = wave_incl_scan(c[3], lane) - c[3];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (b0 + u < B) hc[((b0 + u) * K + k) * PT + q] = c[u] + excl;
    }
    if constexpr (MSE) {
      double s1[4], s2[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        s1[u] = (b0 + u < B) ? hs1[(b0 + u) * PT + q] : 0.0;
        s2[u] = (b0 + u < B) ? hs2[(b0 + u) * PT + q] : 0.0;
      }
      s1[1] += s1[0]; s1[2] += s1[1]; s1[3] += s1[2];
      s2[1] += s2[0]; s2[2] += s2[1]; s2[3] += s2[2];
      const double e1 = wave_incl_scan(s1[3], lane) - s1[3];
      const double e2 = wave_incl_scan(s2[3], lane) - s2[3];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (b0 + u < B) {
          hs1[(b0 + u) * PT + q] = s1[u] + e1;
          hs2[(b0 + u) * PT + q] = s2[u] + e2;
        }
    }
    __syncthreads();
    double best = __builtin_huge_val();
    int bestb = 0x7fffffff;
    if (active) {
      for (int u = 0; u < 4; ++u) {
        const int cand = b0 + u;          // split: bins < cand go left
        if (cand < 1 || cand > B - 1) continue;
        double loss;
        if constexpr (MSE) {
          const uint32_t nL = hc[(cand - 1) * PT + q];
          const uint32_t n = hc[(B - 1) * PT + q];
          const uint32_t nR = n - nL;
          if (nL == 0 || nR == 0) continue;
          const double S1L = hs1[(cand - 1) * PT + q], S2L = hs2[(cand - 1) * PT + q];
          const double S1 = hs1[(B - 1) * PT + q], S2 = hs2[(B - 1) * PT + q];
          const double S1R = S1 - S1L, S2R = S2 - S2L;
          const double dL = (double)nL, dR = (double)nR;
          const double sseL = S2L - (S1L * S1L) / dL;
          const double sseR = S2R - (S1R * S1R) / dR;
          loss = (sseL + sseR) / (dL + dR);
        } else {
          uint64_t AL = 0, AR = 0;
          int64_t nL = 0, n = 0;
          double sL = 0.0, sR = 0.0;
          for (int k = 0; k < K; ++k) {
            const uint32_t l = hc[((cand - 1) * K + k) * PT + q];
            const uint32_t t = hc[((B - 1) * K + k) * PT + q];
            const uint32_t r = t - l;
            nL += l;
            n += t;
            if (a.crit == SLM_GINI) {
              AL += (uint64_t)l * l;
              AR += (uint64_t)r * r;
            } else {
              sL += nlog2n((double)l);
              sR += nlog2n((double)r);
            }
          }
          const int64_t nR = n - nL;
          if (nL == 0 || nR == 0) continue;
          const double dn = (double)n;
          if (a.crit == SLM_GINI) {
            const double s = (double)AL / (double)nL + (double)AR / (double)nR;
            loss = (dn - s) / dn;
          } else {
            const double TL = nlog2n((double)nL) - sL;
            const double TR = nlog2n((double)nR) - sR;
            loss = (TL + TR) / dn;
          }
        }
        if (loss < best) {
          best = loss;
          bestb = cand;
        }
      }
    }
    wave_argmin(best, bestb);
    if (active && lane == 0) {
      if (bestb == 0x7fffffff) {
        a.best_split[out] = -1;
        a.best_loss[out] = __builtin_huge_val();
        a.threshold[out] = __builtin_huge_valf();
      } else {
        a.best_split[out] = bestb;
        a.best_loss[out] = best;
        a.threshold[out] = edge(rr, bestb);
      }
    }
    __syncthreads();
  }
}

// Nodes without rows get no work item in the histogram scan: report "no
// split" and empty histograms for them here.
__global__ void k_scan_empty_nodes(ScanArgs a, int Kc) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)a.n_nodes * a.P) return;
  const int j = (int)(gid / a.P);
  const Range r = load_range(a.beg, a.end, j, a.N);
  if (r.hi > r.lo) return;
  a.best_split[gid] = -1;
  a.best_loss[gid] = __builtin_huge_val();
  a.threshold[gid] = __builtin_huge_valf();
  if (a.hist_out)
    for (int i = 0; i < a.bins * Kc; ++i) a.hist_out[gid * a.bins * Kc + i] = 0u;
  if (a.sums_out)
    for (int i = 0; i < a.bins * 2; ++i) a.sums_out[gid * a.bins * 2 + i] = 0.0;
}

// ---------------------------------------------------------------- exact kernel
constexpr int EXACT_MAX = 8192;
constexpr int EXACT_KMAX = 16;

template <bool MSE>
__global__ __launch_bounds__(WG) void k_scan_exact(ScanArgs a) {
  __shared__ float key[EXACT_MAX];
  __shared__ int idx[EXACT_MAX];
  __shared__ double red_l[WG];
  __shared__ int red_b[WG];
  // per-thread class counts (classification) or sums (MSE) for the block scan
  __shared__ double part[WG * 2];
  __shared__ int cnt[WG * EXACT_KMAX];

  const int j = blockIdx.x / a.P;
  const int p = blockIdx.x % a.P;
  const Range rg = load_range(a.beg, a.end, j, a.N);
  const int64_t n64 = rg.hi - rg.lo;
  const int tid = threadIdx.x;
  const int64_t out = (int64_t)j * a.P + p;
  if (n64 > EXACT_MAX) {
    if (tid == 0) {
      a.best_split[out] = -2;
      a.best_loss[out] = __builtin_nan("");
      a.threshold[out] = __builtin_nanf("");
    }
    return;
  }
  const int n = (int)n64;
  int np2 = 1;
  while (np2 < n) np2 <<= 1;
  for (int i = tid; i < np2; i += WG) {
    if (i < n) {
      key[i] = a.Z[(rg.lo + i) * a.P + p];
      idx[i] = i;
    } else {
      key[i] = __builtin_huge_valf();
      idx[i] = 0x7fffffff;
    }
  }
  __syncthreads();
  // bitonic sort on (key, idx): equal keys keep row order
  for (int k = 2; k <= np2; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int i = tid; i < np2; i += WG) {
        const int ixj = i ^ jj;
        if (ixj > i) {
          const bool up = (i & k) == 0;
          const float ka = key[i], kb = key[ixj];
          const int ia = idx[i], ib = idx[ixj];
          const bool a_gt_b = (ka > kb) || (ka == kb && ia > ib);
          if (a_gt_b == up) {
            key[i] = kb; key[ixj] = ka;
            idx[i] = ib; idx[ixj] = ia;
          }
        }
      }
      __syncthreads();
    }
  }
  const int K = MSE ? 0 : a.K;
  const int C = (n + WG - 1) / WG;          // sorted positions per thread
  const int s0 = tid * C, s1 = min(n, s0 + C);
  // local totals
  double ly = 0.0, ly2 = 0.0;
  if constexpr (MSE) {
    for (int s = s0; s < s1; ++s) {
      const double yv = a.y[rg.lo + idx[s]];
      ly += yv;
      ly2 += yv * yv;
    }
    part[tid] = ly;
    part[WG + tid] = ly2;
  } else {
    for (int k = 0; k < K; ++k) cnt[tid * EXACT_KMAX + k] = 0;
    for (int s = s0; s < s1; ++s) {
      const int lab = a.labels[rg.lo + idx[s]];
      if ((unsigned)lab < (unsigned)K) cnt[tid * EXACT_KMAX + lab] += 1;
    }
  }
  __syncthreads();
  // exclusive scans over threads (sequential per class: tiny)
  if constexpr (MSE) {
    if (tid < 2) {
      double run = 0.0;
      for (int t = 0; t < WG; ++t) {
        const double vv = part[tid * WG + t];
        part[tid * WG + t] = run;
        run += vv;
      }
      red_l[tid] = run;   // totals
    }
  } else {
    if (tid < K) {
      int run = 0;
      for (int t = 0; t < WG; ++t) {
        const int vv = cnt[t * EXACT_KMAX + tid];
        cnt[t * EXACT_KMAX + tid] = run;
        run += vv;
      }
      red_b[tid] = run;   // totals
    }
  }
  __syncthreads();
  double tot1 = 0.0, tot2 = 0.0;
  int tot[EXACT_KMAX];
  int left[EXACT_KMAX];
  int ntot = 0;
  if constexpr (MSE) {
    tot1 = red_l[0];
    tot2 = red_l[1];
    ntot = n;
  } else {
#pragma unroll
    for (int k = 0; k < EXACT_KMAX; ++k) {
      tot[k] = k < K ? red_b[k] : 0;
      left[k] = k < K ? cnt[tid * EXACT_KMAX + k] : 0;
      ntot += tot[k];
    }
  }
  double run1 = MSE ? part[tid] : 0.0, run2 = MSE ? part[WG + tid] : 0.0;
  int nl_lab = 0;
  if constexpr (!MSE) {
#pragma unroll
    for (int k = 0; k < EXACT_KMAX; ++k) nl_lab += left[k];
  }
  __syncthreads();
  double best = __builtin_huge_val();
  int bestn = 0x7fffffff;
  for (int s = s0; s < s1; ++s) {
    int nL;
    if constexpr (MSE) {
      const double yv = a.y[rg.lo + idx[s]];
      run1 += yv;
      run2 += yv * yv;
      nL = s + 1;
    } else {
      const int lab = a.labels[rg.lo + idx[s]];
#pragma unroll
      for (int k = 0; k < EXACT_KMAX; ++k)
        if (k == lab) left[k] += 1;
      if ((unsigned)lab < (unsigned)K) nl_lab += 1;
      nL = nl_lab;
    }
    if (s + 1 >= n || !(key[s] < key[s + 1])) continue;
    double loss;
    if constexpr (MSE) {
      const int nR = n - nL;
      const double dL = (double)nL, dR = (double)nR;
      const double S1R = tot1 - run1, S2R = tot2 - run2;
      const double sseL = run2 - (run1 * run1) / dL;
      const double sseR = S2R - (S1R * S1R) / dR;
      loss = (sseL + sseR) / (dL + dR);
    } else {
      const int nR = ntot - nL;
      if (nL == 0 || nR == 0) continue;
      const double dn = (double)ntot;
      if (a.crit == SLM_GINI) {
        uint64_t AL = 0, AR = 0;
#pragma unroll
        for (int k = 0; k < EXACT_KMAX; ++k) {
          const uint64_t l = (uint64_t)left[k], r = (uint64_t)(tot[k] - left[k]);
          AL += l * l;
          AR += r * r;
        }
        const double sv = (double)AL / (double)nL + (double)AR / (double)nR;
        loss = (dn - sv) / dn;
      } else {
        double sL = 0.0, sR = 0.0;
        for (int k = 0; k < K; ++k) {
          sL += nlog2n((double)left[k]);
          sR += nlog2n((double)(tot[k] - left[k]));
        }
        loss = ((nlog2n((double)nL) - sL) + (nlog2n((double)nR) - sR)) / dn;
      }
    }
    // split index = number sent left = s + 1 (all rows; labels out of range are
    // ignored by the criterion but still move with their value)
    if (loss < best) {
      best = loss;
      bestn = s + 1;
    }
  }
  red_l[tid] = best;
  red_b[tid] = bestn;
  __syncthreads();
  for (int o = WG / 2; o > 0; o >>= 1) {
    if (tid < o) {
      const double l2 = red_l[tid + o];
      const int b2 = red_b[tid + o];
      if (l2 < red_l[tid] || (l2 == red_l[tid] && b2 < red_b[tid])) {
        red_l[tid] = l2;
        red_b[tid] = b2;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (red_b[0] == 0x7fffffff) {
      a.best_split[out] = -1;
      a.best_loss[out] = __builtin_huge_val();
      a.threshold[out] = __builtin_huge_valf();
    } else {
      a.best_split[out] = red_b[0];
      a.best_loss[out] = red_l[0];
      a.threshold[out] = key[red_b[0]];
    }
  }
}

template <int PT, bool MSE>
slm_status launch_hist_pt(const ScanArgs &a, const Plan &pl, hipStream_t s) {
  const int n_pt = (a.P + PT - 1) / PT;
  const int64_t items = num_items(a.n_nodes, a.N, pl.CH);
  const int64_t total = items * n_pt;
  if (total == 0) return SLM_OK;
  const int64_t grid = (total + 8 * pl.G - 1) / (8 * pl.G) * (8 * pl.G);
  SLM_CHECK(grid < (1ll << 31), SLM_E_SHAPE, "slm_split_scan: grid too large");
  const size_t lds = lds_bytes(PT, a.bins, a.K, MSE);
  const size_t slot = slot_bytes(PT, a.bins, MSE ? 1 : a.K, MSE);
  const int64_t n_slots = (a.N - 1) / chunk_min(a.N) + 1;
  auto kern = k_scan_hist<PT, MSE>;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(WG), lds, s, a, pl.CH, n_pt, pl.G, total,
                     slot, n_slots);
  SLM_LAUNCHED();
  return SLM_OK;
}

template <bool MSE>
slm_status launch_hist(const ScanArgs &a, const Plan &pl, hipStream_t s) {
  switch (pl.PT) {
    case 32: return launch_hist_pt<32, MSE>(a, pl, s);
    case 16: return launch_hist_pt<16, MSE>(a, pl, s);
    case 8: return launch_hist_pt<8, MSE>(a, pl, s);
    default: return launch_hist_pt<4, MSE>(a, pl, s);
  }
}

template <int PT, bool MSE>
void set_lds_attr(int bytes) {
  // Best effort: raise the dynamic-LDS limit for the large-histogram tiles.
  // A refusal is cleared and left to the launch, which then reports it.
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_scan_hist<PT, MSE>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess)
    (void)hipGetLastError();
}

}  // namespace

slm_status prepare_kernels() {
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0, lds = 65536;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
      (void)hipGetLastError();
      return;
    }
    const int dyn = lds - 1024;   // room for the kernels' static LDS
    set_lds_attr<32, false>(dyn);
    set_lds_attr<16, false>(dyn);
    set_lds_attr<8, false>(dyn);
    set_lds_attr<4, false>(dyn);
    set_lds_attr<32, true>(dyn);
    set_lds_attr<16, true>(dyn);
    set_lds_attr<8, true>(dyn);
    set_lds_attr<4, true>(dyn);
  });
  return SLM_OK;
}

size_t scan_workspace_bytes(int64_t N, int n_nodes, int P, int bins, int K, int crit) {
  (void)n_nodes;
  if (bins == 0 || N <= 0) return 256;
  const bool mse = crit == SLM_MSE;
  const int Kc = mse ? 1 : K;
  // the plan may pick any PT in {4, 8, 16, 32}; size for the largest footprint
  size_t worst = 0;
  for (int PT = 4; PT <= 32; PT <<= 1) {
    const int64_t n_pt = (P + PT - 1) / PT;
    worst = std::max(worst, (size_t)n_pt * slot_bytes(PT, bins, Kc, mse) +
                                (size_t)n_pt * 4);
  }
  const int64_t n_slots = (N - 1) / chunk_min(N) + 1;
  return (size_t)n_slots * worst + 256;
}

slm_status launch_scan_empty_nodes(const ScanArgs &a, hipStream_t s) {
  const int64_t total = (int64_t)a.n_nodes * a.P;
  if (total == 0) return SLM_OK;
  hipLaunchKernelGGL(k_scan_empty_nodes, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a,
                     a.crit == SLM_MSE ? 1 : a.K);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_scan_hist(const ScanArgs &a, hipStream_t s) {
  if (a.N <= 0 || a.n_nodes <= 0) return SLM_OK;
  const Plan pl = make_plan(a.N, a.n_nodes, a.P, a.bins, a.crit == SLM_MSE ? 1 : a.K, a.crit);
  if (a.crit == SLM_MSE) return launch_hist<true>(a, pl, s);
  return launch_hist<false>(a, pl, s);
}

slm_status launch_scan_exact(const ScanArgs &a, int max_rows, hipStream_t s) {
  SLM_CHECK(max_rows <= EXACT_MAX, SLM_E_UNSUPPORTED,
            "slm_split_scan: exact scan supports nodes of at most %d rows (got %d)", EXACT_MAX,
            max_rows);
  SLM_CHECK(a.crit == SLM_MSE || a.K <= EXACT_KMAX, SLM_E_UNSUPPORTED,
            "slm_split_scan: exact scan supports K <= %d", EXACT_KMAX);
  const int64_t grid = (int64_t)a.n_nodes * a.P;
  if (grid == 0) return SLM_OK;
  if (a.crit == SLM_MSE)
    hipLaunchKernelGGL(k_scan_exact<true>, dim3((unsigned)grid), dim3(WG), 0, s, a);
  else
    hipLaunchKernelGGL(k_scan_exact<false>, dim3((unsigned)grid), dim3(WG), 0, s, a);
  SLM_LAUNCHED();
  return SLM_OK;
}

}  // namespace slm
