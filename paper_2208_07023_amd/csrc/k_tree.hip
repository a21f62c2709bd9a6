// Frontier bookkeeping of the tree build (Sec. III-B, Alg. 2): node
// statistics (class counts, or count / sum y / sum y^2 / min y / max y for
// regression) and the stable partition of a node's rows by its split
// (Sec. II-A, Eqs. (3)-(4): rows with a^T x >= t go right).
//
// Rows of every frontier node are contiguous.  A split node's children take
// the same row range, left rows first, each side in the parent's order, so
// the next depth's nodes are again contiguous ranges.  The partition runs in
// three passes over "chunk x node" items: count the left rows of each item,
// turn the counts into per-item offsets inside each node (one thread per
// node), then scatter rows, targets and the children's statistics.
#include "slm_internal.hpp"

namespace slm {

namespace {

constexpr int WG = 256;
constexpr int64_t PART_CH = 1024;

__device__ __forceinline__ unsigned long long enc_f64(double d) {
  unsigned long long u = (unsigned long long)__double_as_longlong(d);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__global__ __launch_bounds__(WG) void k_node_stats(const int64_t *beg, const int64_t *end,
                                                   int n_nodes, int64_t N, const int32_t *lab,
                                                   const double *y, int K, TreeStats st,
                                                   int64_t CH) {
  __shared__ uint32_t sc[64];
  __shared__ double ss1, ss2;
  __shared__ unsigned long long smin, smax;
  const Item it = find_item(beg, end, n_nodes, N, CH, blockIdx.x);
  if (it.node < 0) return;
  const int tid = threadIdx.x;
  if (tid < 64) sc[tid] = 0;
  if (tid == 0) {
    ss1 = 0.0;
    ss2 = 0.0;
    smin = ~0ull;
    smax = 0ull;
  }
  __syncthreads();
  for (int64_t r = it.lo + tid; r < it.hi; r += WG) {
    if (lab) {
      const int k = lab[r];
      if ((unsigned)k < (unsigned)K) atomicAdd(&sc[k], 1u);
    } else {
      const double v = y[r];
      atomicAdd(&sc[0], 1u);
      unsafeAtomicAdd(&ss1, v);
      unsafeAtomicAdd(&ss2, v * v);
      atomicMin(&smin, enc_f64(v));
      atomicMax(&smax, enc_f64(v));
    }
  }
  __syncthreads();
  const int j = it.node;
  if (lab) {
    if (tid < K && sc[tid]) atomicAdd(&st.counts[(int64_t)j * K + tid], sc[tid]);
  } else if (tid == 0) {
    atomicAdd(&st.cnt[j], sc[0]);
    unsafeAtomicAdd(&st.s1[j], ss1);
    unsafeAtomicAdd(&st.s2[j], ss2);
    atomicMin(&st.ymin[j], smin);
    atomicMax(&st.ymax[j], smax);
  }
}

__global__ __launch_bounds__(WG) void k_part_count(PartArgs a) {
  __shared__ uint32_t s;
  const int64_t v = blockIdx.x;
  const Item it = find_item(a.beg, a.end, a.n_nodes, a.N, a.CH, v);
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  if (it.node < 0 || !a.do_split[it.node]) {
    if (threadIdx.x == 0) a.cnt_left[v] = 0;
    return;
  }
  const float t = a.thr[it.node];
  uint32_t c = 0;
  for (int64_t r = it.lo + threadIdx.x; r < it.hi; r += WG) c += (a.zsel[r] >= t) ? 0u : 1u;
  atomicAdd(&s, c);
  __syncthreads();
  if (threadIdx.x == 0) a.cnt_left[v] = s;
}

__global__ void k_part_offsets(PartArgs a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_nodes) return;
  const Range r = load_range(a.beg, a.end, j, a.N);
  if (r.hi <= r.lo) {
    a.n_left[j] = 0;
    return;
  }
  const int64_t g0 = r.lo / a.CH, g1 = (r.hi - 1) / a.CH;
  const int64_t v0 = item_start(a.beg, j, a.N, a.CH);
  int64_t L = 0, R = 0;
  for (int64_t g = g0; g <= g1; ++g) {
    const int64_t v = v0 + (g - g0);
    const int64_t lo = r.lo > g * a.CH ? r.lo : g * a.CH;
    const int64_t hi = r.hi < (g + 1) * a.CH ? r.hi : (g + 1) * a.CH;
    const int64_t cl = a.cnt_left[v];
    a.off_left[v] = L;
    a.off_right[v] = R;
    L += cl;
    R += (hi - lo) - cl;
  }
  a.n_left[j] = a.do_split[j] ? L : (r.hi - r.lo);
}

// Rows r0 .. r0+nin-1 of X to rows dest[0 .. nin-1] of Xn, element by element
// in row-major order: 8 loads in flight per thread, then the stores.
template <typename T>
__device__ __forceinline__ void copy_rows(const T *X, T *Xn, int64_t r0, int64_t nin, int D,
                                          const int64_t *dest, int tid) {
  const int ne = (int)nin * D;
  for (int e0 = tid; e0 < ne; e0 += 8 * WG) {
    T vals[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * WG;
      vals[u] = e < ne ? X[r0 * D + e] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * WG;
      if (e < ne) {
        const int q = e / D, c = e - q * D;
        Xn[dest[q] * D + c] = vals[u];
      }
    }
  }
}

__global__ __launch_bounds__(WG) void k_part_scatter(PartArgs a) {
  __shared__ int64_t dest[WG];
  __shared__ uint32_t wl[WG / 64];
  __shared__ uint32_t sc[2 * 32];
  __shared__ double ss1[2], ss2[2];
  __shared__ unsigned long long smin[2], smax[2];
  const int64_t v = blockIdx.x;
  const Item it = find_item(a.beg, a.end, a.n_nodes, a.N, a.CH, v);
  if (it.node < 0 || !a.do_split[it.node]) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < 64) sc[tid] = 0;
  if (tid < 2) {
    ss1[tid] = 0.0;
    ss2[tid] = 0.0;
    smin[tid] = ~0ull;
    smax[tid] = 0ull;
  }
  const int j = it.node;
  const Range nr = load_range(a.beg, a.end, j, a.N);
  const int64_t nL = a.n_left[j];
  const float t = a.thr[j];
  int64_t base_l = nr.lo + a.off_left[v];
  int64_t base_r = nr.lo + nL + a.off_right[v];
  __syncthreads();
  for (int64_t r0 = it.lo; r0 < it.hi; r0 += WG) {
    const int64_t r = r0 + tid;
    const bool in = r < it.hi;
    const bool right = in && a.zsel[r] >= t;
    const bool left = in && !right;
    // stable ranks: ballots within each wave, wave totals across the group
    const unsigned long long bl = __ballot(left);
    const unsigned long long br = __ballot(right);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t rl = __popcll(bl & below), rr = __popcll(br & below);
    if (lane == 0) wl[wave] = __popcll(bl);
    __syncthreads();
    uint32_t pre_l = 0, tot_l = 0;
    for (int w = 0; w < WG / 64; ++w) {
      if (w < wave) pre_l += wl[w];
      tot_l += wl[w];
    }
    const int64_t nin = (it.hi - r0) < WG ? (it.hi - r0) : WG;
    // rows before this wave in this round: wave * 64 (all valid except in the last round)
    const int64_t before = (int64_t)wave * 64 < nin ? (int64_t)wave * 64 : nin;
    const uint32_t pre_r = (uint32_t)before - pre_l;
    if (left) dest[tid] = base_l + pre_l + rl;
    else if (right) dest[tid] = base_r + pre_r + rr;
    if (in) {
      const int side = right ? 1 : 0;
      if (a.lab) {
        const int k = a.lab[r];
        if ((unsigned)k < (unsigned)a.K) atomicAdd(&sc[side * 32 + k], 1u);
      } else {
        const double yv = a.y[r];
        atomicAdd(&sc[side * 32], 1u);
        unsafeAtomicAdd(&ss1[side], yv);
        unsafeAtomicAdd(&ss2[side], yv * yv);
        atomicMin(&smin[side], enc_f64(yv));
        atomicMax(&smax[side], enc_f64(yv));
      }
    }
    __syncthreads();
    // coalesced copy of the round's rows to their destinations
    if (a.x_bf16)
      copy_rows(static_cast<const uint16_t *>(a.X), static_cast<uint16_t *>(a.Xn), r0, nin, a.D,
                dest, tid);
    else
      copy_rows(static_cast<const float *>(a.X), static_cast<float *>(a.Xn), r0, nin, a.D, dest,
                tid);
    if (in) {
      if (a.lab) a.labn[dest[tid]] = a.lab[r];
      else a.yn[dest[tid]] = a.y[r];
    }
    base_l += tot_l;
    base_r += (uint32_t)nin - tot_l;
    lds_barrier();
  }
  // children statistics: index 2*j (left), 2*j+1 (right)
  for (int side = 0; side < 2; ++side) {
    const int64_t c = 2 * (int64_t)j + side;
    if (a.lab) {
      if (tid < a.K && sc[side * 32 + tid])
        atomicAdd(&a.child.counts[c * a.K + tid], sc[side * 32 + tid]);
    } else if (tid == 0 && sc[side * 32]) {
      atomicAdd(&a.child.cnt[c], sc[side * 32]);
      unsafeAtomicAdd(&a.child.s1[c], ss1[side]);
      unsafeAtomicAdd(&a.child.s2[c], ss2[side]);
      atomicMin(&a.child.ymin[c], smin[side]);
      atomicMax(&a.child.ymax[c], smax[side]);
    }
  }
}

}  // namespace

int64_t partition_items(int n_nodes, int64_t N) { return num_items(n_nodes, N, PART_CH); }

slm_status launch_node_stats(const int64_t *beg, const int64_t *end, int n_nodes, int64_t N,
                             const int32_t *lab, const double *y, int K, TreeStats st,
                             hipStream_t s) {
  SLM_CHECK(K <= 32, SLM_E_SHAPE, "node stats: K = %d > 32", K);
  const int64_t items = num_items(n_nodes, N, PART_CH);
  if (items == 0) return SLM_OK;
  hipLaunchKernelGGL(k_node_stats, dim3((unsigned)items), dim3(WG), 0, s, beg, end, n_nodes, N,
                     lab, y, K, st, PART_CH);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_partition(const PartArgs &a0, hipStream_t s) {
  PartArgs a = a0;
  a.CH = PART_CH;
  SLM_CHECK(a.K <= 32, SLM_E_SHAPE, "partition: K = %d > 32", a.K);
  const int64_t items = num_items(a.n_nodes, a.N, a.CH);
  if (items == 0) return SLM_OK;
  hipLaunchKernelGGL(k_part_count, dim3((unsigned)items), dim3(WG), 0, s, a);
  SLM_LAUNCHED();
  hipLaunchKernelGGL(k_part_offsets, dim3((unsigned)((a.n_nodes + 63) / 64)), dim3(64), 0, s, a);
  SLM_LAUNCHED();
  hipLaunchKernelGGL(k_part_scatter, dim3((unsigned)items), dim3(WG), 0, s, a);
  SLM_LAUNCHED();
  return SLM_OK;
}

// ---------------------------------------------------------------- node-batch search
namespace {
// Stop state after evaluation number evals_now: a node whose global-best
// loss reached its target stops (its active row range collapses to empty and
// evals = evals_now); on the last evaluation every node still searching gets
// evals = evals_now.  remaining = nodes still searching.  One work-group.
__global__ __launch_bounds__(1024) void k_search_stop(const double *gbest_loss,
                                                      const double *target, const int64_t *beg,
                                                      int64_t *end_act, int32_t *done,
                                                      int32_t *evals, int n, int evals_now,
                                                      int last, uint32_t *remaining) {
  __shared__ uint32_t cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  uint32_t c = 0;
  for (int j = threadIdx.x; j < n; j += 1024) {
    if (done[j]) continue;
    if (target && gbest_loss[j] <= target[j]) {
      done[j] = 1;
      evals[j] = evals_now;
      end_act[j] = beg[j];
    } else if (last) {
      done[j] = 1;
      evals[j] = evals_now;
    } else {
      ++c;
    }
  }
  atomicAdd(&cnt, c);
  __syncthreads();
  if (threadIdx.x == 0) *remaining = cnt;
}
}  // namespace

slm_status launch_search_stop(const double *gbest_loss, const double *target, const int64_t *beg,
                              int64_t *end_act, int32_t *done, int32_t *evals, int n,
                              int evals_now, bool last, uint32_t *remaining, hipStream_t s) {
  if (n <= 0) return SLM_OK;
  hipLaunchKernelGGL(k_search_stop, dim3(1), dim3(1024), 0, s, gbest_loss, target, beg, end_act,
                     done, evals, n, evals_now, (int)last, remaining);
  SLM_LAUNCHED();
  return SLM_OK;
}

}  // namespace slm
