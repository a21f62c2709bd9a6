// Projection of a node's rows onto its particles' directions on the matrix
// cores (Sec. II-A, Eq. (1)):  Z[i, p] = sum_d X[i, d] * W[j*P + p, d]  for
// every row i of node j, with per-(node, particle) min and max of Z.
//
// One work-group computes a BM x BN tile of Z: BM consecutive global rows
// (aligned to BM, rows outside the item's node masked) against BN particles
// of that node.  X and W tiles of KC dimensions are staged in LDS with an odd
// row stride and fed to v_mfma_f32_32x32x2_f32; each output element is the
// same sequence of MFMA accumulations over k whatever the tile shape, so a
// column recomputed alone (P = 1) is bit-identical to the same column
// computed among many particles.
#include "slm_internal.hpp"

namespace slm {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int KC = 64;          // dimensions staged per LDS round
constexpr int LDSTR = KC + 1;   // odd stride: the 32 rows a fragment reads hit 32 banks

template <bool BF16>
__device__ __forceinline__ float load_x(const void *p, int64_t idx) {
  if constexpr (BF16) return bf16_to_f32(static_cast<const uint16_t *>(p)[idx]);
  else return static_cast<const float *>(p)[idx];
}

template <int BM, int BN, int WM, int WN, bool BF16>
__global__ __launch_bounds__(256) void k_project(ProjectArgs a) {
  static_assert(WM * WN == 4, "4 waves per work-group");
  constexpr int TM = BM / WM, TN = BN / WN, FM = TM / 32, FN = TN / 32;
  static_assert(FM >= 1 && FN >= 1, "wave tile must hold whole 32x32 blocks");

  __shared__ float Xs[BM * LDSTR];
  __shared__ float Ws[BN * LDSTR];

  const int n_pt = (a.P + BN - 1) / BN;
  const int64_t v = blockIdx.x / n_pt;
  const int pt = blockIdx.x % n_pt;
  const Item it = find_item(a.beg, a.end, a.n_nodes, a.N, BM, v);
  if (it.node < 0) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t r0 = (it.lo / BM) * BM;      // tile origin (global chunk start)
  const int p0 = pt * BN;
  const int D = a.D, P = a.P;
  const int64_t wbase = (int64_t)it.node * P;

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int k = 0; k < FN; ++k) acc[i][k] = f32x16{};

  for (int k0 = 0; k0 < D; k0 += KC) {
    const int kc = min(KC, D - k0);
    for (int e = tid; e < BM * KC; e += 256) {
      const int r = e / KC, c = e - r * KC;
      const int64_t row = r0 + r;
      float val = 0.f;
      if (c < kc && row >= it.lo && row < it.hi) val = load_x<BF16>(a.X, row * D + k0 + c);
      Xs[r * LDSTR + c] = val;
    }
    for (int e = tid; e < BN * KC; e += 256) {
      const int r = e / KC, c = e - r * KC;
      const int p = p0 + r;
      float val = 0.f;
      if (c < kc && p < P) val = load_x<BF16>(a.W, (wbase + p) * D + k0 + c);
      Ws[r * LDSTR + c] = val;
    }
    __syncthreads();
    const int ksteps = (kc + 1) >> 1;
    const int kh = lane >> 5, li = lane & 31;
    for (int ks = 0; ks < ksteps; ++ks) {
      const int kk = 2 * ks + kh;
      float af[FM], bf[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) af[i] = Xs[(wm * TM + i * 32 + li) * LDSTR + kk];
#pragma unroll
      for (int k = 0; k < FN; ++k) bf[k] = Ws[(wn * TN + k * 32 + li) * LDSTR + kk];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int k = 0; k < FN; ++k)
          acc[i][k] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i], bf[k], acc[i][k], 0, 0, 0);
    }
    __syncthreads();
  }

  // Epilogue.  32x32 f32 accumulator layout: lane l, register r holds
  // row 8*(r/4) + 4*(l/32) + r%4, column l%32 of the block.
  const bool do_mm = a.zmin != nullptr;
#pragma unroll
  for (int k = 0; k < FN; ++k) {
    const int p = p0 + wn * TN + k * 32 + (lane & 31);
    float mn = __builtin_huge_valf(), mx = -__builtin_huge_valf();
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rr = wm * TM + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t row = r0 + rr;
        if (p < P && row >= it.lo && row < it.hi) {
          const float z = acc[i][k][r];
          a.Z[row * P + p] = z;
          mn = fminf(mn, z);
          mx = fmaxf(mx, z);
        }
      }
    }
    if (do_mm) {
      mn = fminf(mn, __shfl_xor(mn, 32));
      mx = fmaxf(mx, __shfl_xor(mx, 32));
      if (lane < 32 && p < P && mn <= mx) {
        atomic_min_f32(&a.zmin[wbase + p], mn);
        atomic_max_f32(&a.zmax[wbase + p], mx);
      }
    }
  }
}

__global__ void k_fill_minmax(float *zmin, float *zmax, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    zmin[i] = __builtin_huge_valf();
    zmax[i] = -__builtin_huge_valf();
  }
}

template <int BM, int BN, int WM, int WN>
slm_status launch_cfg(const ProjectArgs &a, hipStream_t s) {
  const int64_t items = num_items(a.n_nodes, a.N, BM);
  const int64_t n_pt = (a.P + BN - 1) / BN;
  const int64_t grid = items * n_pt;
  if (grid == 0) return SLM_OK;
  SLM_CHECK(grid < (1ll << 31), SLM_E_SHAPE, "slm_project: grid of %lld blocks too large",
            (long long)grid);
  if (a.bf16)
    hipLaunchKernelGGL((k_project<BM, BN, WM, WN, true>), dim3((unsigned)grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_project<BM, BN, WM, WN, false>), dim3((unsigned)grid), dim3(256), 0, s, a);
  SLM_LAUNCHED();
  return SLM_OK;
}

}  // namespace

slm_status launch_fill_minmax(float *zmin, float *zmax, int64_t n, hipStream_t s) {
  if (n <= 0) return SLM_OK;
  hipLaunchKernelGGL(k_fill_minmax, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, zmin,
                     zmax, n);
  SLM_LAUNCHED();
  return SLM_OK;
}

slm_status launch_project(const ProjectArgs &a, hipStream_t s) {
  // Tile shape by particle count: wide tiles for large swarms, a single
  // 32-particle column block for small ones (and for P = 1 recomputation).
  if (a.P >= 128) return launch_cfg<128, 128, 2, 2>(a, s);
  if (a.P > 32) return launch_cfg<128, 64, 2, 2>(a, s);
  return launch_cfg<128, 32, 4, 1>(a, s);
}

}  // namespace slm
