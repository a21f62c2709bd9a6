// Mixed-precision screening of a swarm evaluation: every particle is scored
// on the bfloat16 projection, the k best of each node are projected again in
// float32 and re-scored, and the two sets of results are merged for the
// swarm step (Sec. III-B: a direction is scored by the loss of its best
// threshold; Sec. VI names faster projection search on high-dimensional data
// as the open problem this step addresses).
//
//   k_screen_select  per node, the k particles with the smallest screened
//                    losses, ascending by (loss, index): a bitonic sort of
//                    (loss, index) keys in LDS.
//   k_screen_gather  float32 images of the selected positions (the
//                    directions of the float32 re-projection).
//   k_screen_merge   re-scored loss / split / threshold written over the
//                    screened ones of the selected particles; the losses
//                    eligible for the global best are the re-scored ones
//                    (+inf for every other particle).
#include "slm_internal.hpp"

namespace slm {
namespace {

constexpr int SEL_WG = 1024;

// Order-preserving image of a double (total order for non-NaN values; -0.0 is
// folded into +0.0 first so the two compare equal as in IEEE).
__device__ __forceinline__ unsigned long long ord_f64(double d) {
  d = d + 0.0;
  const unsigned long long u = (unsigned long long)__double_as_longlong(d);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__global__ __launch_bounds__(SEL_WG) void k_screen_select(const double *loss, int n_nodes, int P,
                                                          int P2, int k, int32_t *sel) {
  extern __shared__ __align__(8) unsigned char smem[];
  unsigned long long *key = reinterpret_cast<unsigned long long *>(smem);
  int *idx = reinterpret_cast<int *>(key + P2);
  const int j = blockIdx.x;
  if (j >= n_nodes) return;
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)j * P;
  for (int i = tid; i < P2; i += SEL_WG) {
    key[i] = i < P ? ord_f64(loss[base + i]) : ~0ull;
    idx[i] = i;                       // padding sorts after every particle
  }
  __syncthreads();
  // bitonic sort ascending by (key, idx)
  for (int size = 2; size <= P2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = tid; t < P2 / 2; t += SEL_WG) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const unsigned long long ka = key[lo], kb = key[hi];
        const int ia = idx[lo], ib = idx[hi];
        const bool gt = ka > kb || (ka == kb && ia > ib);
        if (gt == up) {
          key[lo] = kb;
          key[hi] = ka;
          idx[lo] = ib;
          idx[hi] = ia;
        }
      }
      __syncthreads();
    }
  }
  for (int s = tid; s < k; s += SEL_WG) sel[(int64_t)j * k + s] = idx[s];
}

__global__ void k_screen_gather(const double *x, const int32_t *sel, int n_nodes, int P, int k,
                                int D, float *W32) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)n_nodes * k * D;
  if (e >= tot) return;
  const int64_t r = e / D;
  const int d = (int)(e - r * D);
  const int j = (int)(r / k);
  int p = sel[r];
  p = p < 0 ? 0 : (p >= P ? P - 1 : p);
  W32[e] = (float)x[((int64_t)j * P + p) * D + d];
}

__global__ __launch_bounds__(256) void k_screen_merge(const int32_t *sel, const double *loss_r,
                                                      const int32_t *split_r, const float *thr_r,
                                                      int n_nodes, int P, int k, double *loss,
                                                      int32_t *split, float *thr, double *gloss) {
  extern __shared__ int pos[];        // [P]: slot of each particle in the selection, or -1
  const int j = blockIdx.x;
  if (j >= n_nodes) return;
  const int tid = threadIdx.x;
  for (int p = tid; p < P; p += 256) pos[p] = -1;
  __syncthreads();
  for (int s = tid; s < k; s += 256) {
    const int p = sel[(int64_t)j * k + s];
    if (p >= 0 && p < P) pos[p] = s;
  }
  __syncthreads();
  for (int p = tid; p < P; p += 256) {
    const int64_t g = (int64_t)j * P + p;
    const int s = pos[p];
    if (s >= 0) {
      const int64_t r = (int64_t)j * k + s;
      const double l = loss_r[r];
      loss[g] = l;
      split[g] = split_r[r];
      thr[g] = thr_r[r];
      gloss[g] = l;
    } else {
      gloss[g] = __builtin_huge_val();
    }
  }
}

}  // namespace

slm_status launch_screen_select(const double *loss, int n_nodes, int P, int k, int32_t *sel,
                                hipStream_t s) {
  if (n_nodes <= 0 || k <= 0) return SLM_OK;
  int P2 = 1;
  while (P2 < P) P2 <<= 1;
  const size_t lds = (size_t)P2 * (8 + 4);
  hipLaunchKernelGGL(k_screen_select, dim3((unsigned)n_nodes), dim3(SEL_WG), lds, s, loss,
                     n_nodes, P, P2, k, sel);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_screen_gather(const double *x, const int32_t *sel, int n_nodes, int P, int k,
                                int D, float *W32, hipStream_t s) {
  const int64_t tot = (int64_t)n_nodes * k * D;
  if (tot <= 0) return SLM_OK;
  hipLaunchKernelGGL(k_screen_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, x,
                     sel, n_nodes, P, k, D, W32);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_screen_merge(const int32_t *sel, const double *loss_r, const int32_t *split_r,
                               const float *thr_r, int n_nodes, int P, int k, double *loss,
                               int32_t *split, float *thr, double *gloss, hipStream_t s) {
  if (n_nodes <= 0) return SLM_OK;
  hipLaunchKernelGGL(k_screen_merge, dim3((unsigned)n_nodes), dim3(256), (size_t)P * 4, s, sel,
                     loss_r, split_r, thr_r, n_nodes, P, k, loss, split, thr, gloss);
  SLM_LAUNCHED();
  return SLM_OK;
}

}  // namespace slm
