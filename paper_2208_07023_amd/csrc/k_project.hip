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

#include <algorithm>
#include <cstdlib>

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
    // staging in batches of 8 independent loads per thread
    for (int e0 = tid; e0 < BM * KC; e0 += 8 * 256) {
      float val[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256;
        const int r = e / KC, c = e - r * KC;
        const int64_t row = r0 + r;
        val[u] = (e < BM * KC && c < kc && row >= it.lo && row < it.hi)
                     ? load_x<BF16>(a.X, row * D + k0 + c) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256;
        if (e < BM * KC) Xs[(e / KC) * LDSTR + (e % KC)] = val[u];
      }
    }
    for (int e0 = tid; e0 < BN * KC; e0 += 8 * 256) {
      float val[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256;
        const int r = e / KC, c = e - r * KC;
        const int p = p0 + r;
        val[u] = (e < BN * KC && c < kc && p < P) ? load_x<BF16>(a.W, (wbase + p) * D + k0 + c) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256;
        if (e < BN * KC) Ws[(e / KC) * LDSTR + (e % KC)] = val[u];
      }
    }
    lds_barrier();
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
    lds_barrier();
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
          a.Z[z_col(a.zl, p) + row * a.zl.rs] = z;
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

// Short projections (D <= 64): each wave keeps the B fragments of its 32*FN
// particles for all KSP k-steps in registers for the whole work item, and
// 32-row sub-tiles of X stream through a double-buffered LDS tile.  A work
// item is (node, chunk of RT global rows) x (particle tile of 32*FN*WAVES).
// D is padded with zeros to 2*KSP; the extra steps add exact zeros, so each
// output element is the same MFMA sequence whatever FN / WAVES / KSP.
constexpr int SR = 32;             // rows per sub-tile
constexpr int XS = 64 + 1;         // LDS row stride of a sub-tile (odd)

template <int FN, int WAVES, int KSP, bool BF16>
__global__ __launch_bounds__(64 * WAVES) void k_project_short(ProjectArgs a, int64_t RT) {
  __shared__ float Xs[2][SR * XS];
  constexpr int PTILE = 32 * FN * WAVES;
  constexpr int NT = 64 * WAVES;
  constexpr int DP = 2 * KSP;              // padded dimensions staged per row
  constexpr int PER = SR * DP / NT;        // floats per thread per sub-tile
  static_assert(PER >= 1 && SR * DP % NT == 0, "sub-tile must divide evenly");
  const int n_pt = (a.P + PTILE - 1) / PTILE;
  const int64_t v = blockIdx.x / n_pt;
  const int pt = blockIdx.x % n_pt;
  const Item it = find_item(a.beg, a.end, a.n_nodes, a.N, RT, v);
  if (it.node < 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int D = a.D, P = a.P;
  const int li = lane & 31, kh = lane >> 5;
  const int64_t wbase = (int64_t)it.node * P;
  const int pw = pt * PTILE + wave * 32 * FN;   // first particle of this wave
  const bool wave_full = pw + 32 * FN <= P;     // every column of the wave exists

  // B fragments: lane holds W[p = pw + f*32 + li][k = 2 ks + kh]
  float bfrag[FN][KSP];
#pragma unroll
  for (int f = 0; f < FN; ++f) {
    const int p = pw + f * 32 + li;
#pragma unroll
    for (int ks = 0; ks < KSP; ++ks) {
      const int k = 2 * ks + kh;
      bfrag[f][ks] = (k < D && p < P) ? load_x<BF16>(a.W, (wbase + p) * D + k) : 0.f;
    }
  }
  float mn[FN], mx[FN];
#pragma unroll
  for (int f = 0; f < FN; ++f) {
    mn[f] = __builtin_huge_valf();
    mx[f] = -__builtin_huge_valf();
  }
  const int64_t r_first = (it.lo / SR) * SR;
  const int nsub = (int)((it.hi - r_first + SR - 1) / SR);
  // X sub-tile staging: every thread prefetches its share into registers
  // before the current sub-tile's MFMAs and writes it to LDS after them, so
  // global latency overlaps the matrix work.
  float pre[PER];
  // Branch-free: rows and columns outside the item read a clamped in-bounds
  // address and are replaced by zero.
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * NT;
      const int r = e / DP, c = e % DP;
      const int64_t row = r0 + r;
      const bool ok = c < D && row >= it.lo && row < it.hi;
      const int64_t rc = row < it.lo ? it.lo : (row >= it.hi ? it.hi - 1 : row);
      const float x = load_x<BF16>(a.X, rc * D + (c < D ? c : D - 1));
      pre[u] = ok ? x : 0.f;
    }
  };
  auto commit = [&](int buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * NT;
      Xs[buf][(e / DP) * XS + (e % DP)] = pre[u];
    }
  };
  fetch(r_first);
  commit(0);
  lds_barrier();
  for (int sidx = 0; sidx < nsub; ++sidx) {
    const int cur = sidx & 1;
    const int64_t r0 = r_first + (int64_t)sidx * SR;
    const bool more = sidx + 1 < nsub;
    if (more) fetch(r0 + SR);
    f32x16 acc[FN];
#pragma unroll
    for (int f = 0; f < FN; ++f) acc[f] = f32x16{};
#pragma unroll
    for (int ks = 0; ks < KSP; ++ks) {
      const float af = Xs[cur][li * XS + 2 * ks + kh];
#pragma unroll
      for (int f = 0; f < FN; ++f)
        acc[f] = __builtin_amdgcn_mfma_f32_32x32x2f32(af, bfrag[f][ks], acc[f], 0, 0, 0);
    }
    if (more) commit(cur ^ 1);
    // Epilogue.  Lane l, register r holds row 8*(r/4) + 4*(l/32) + r%4 of the
    // sub-tile and particle column l%32 of block f.
    const bool interior = wave_full && r0 >= it.lo && r0 + SR <= it.hi;
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      const int p = pw + f * 32 + li;
      const int64_t rs = a.zl.rs;
      float *zc = a.Z + z_col(a.zl, p) + (r0 + 4 * kh) * rs;
      if (interior) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float z = acc[f][r];
          zc[(int64_t)(8 * (r >> 2) + (r & 3)) * rs] = z;
          mn[f] = fminf(mn[f], z);
          mx[f] = fmaxf(mx[f], z);
        }
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t row = r0 + 8 * (r >> 2) + 4 * kh + (r & 3);
          if (p < P && row >= it.lo && row < it.hi) {
            const float z = acc[f][r];
            zc[(int64_t)(8 * (r >> 2) + (r & 3)) * rs] = z;
            mn[f] = fminf(mn[f], z);
            mx[f] = fmaxf(mx[f], z);
          }
        }
      }
    }
    lds_barrier();
  }
  if (a.zmin != nullptr) {
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      const int p = pw + f * 32 + li;
      const float m0 = fminf(mn[f], __shfl_xor(mn[f], 32));
      const float m1 = fmaxf(mx[f], __shfl_xor(mx[f], 32));
      if (lane < 32 && p < P && m0 <= m1) {
        atomic_min_f32(&a.zmin[wbase + p], m0);
        atomic_max_f32(&a.zmax[wbase + p], m1);
      }
    }
  }
}

template <int FN, int WAVES, int KSP>
slm_status launch_short_k(const ProjectArgs &a, int64_t RT, int64_t grid, hipStream_t s) {
  if (a.bf16)
    hipLaunchKernelGGL((k_project_short<FN, WAVES, KSP, true>), dim3((unsigned)grid),
                       dim3(64 * WAVES), 0, s, a, RT);
  else
    hipLaunchKernelGGL((k_project_short<FN, WAVES, KSP, false>), dim3((unsigned)grid),
                       dim3(64 * WAVES), 0, s, a, RT);
  SLM_LAUNCHED();
  return SLM_OK;
}

template <int FN, int WAVES>
slm_status launch_short(const ProjectArgs &a, hipStream_t s) {
  constexpr int PTILE = 32 * FN * WAVES;
  const int64_t n_pt = (a.P + PTILE - 1) / PTILE;
  // rows per work item: about 4 work-groups per CU over the whole matrix
  // (SLM_PROJ_RT overrides it for tuning sweeps)
  int64_t RT = (a.N * n_pt + 1023) / 1024;
  RT = std::max<int64_t>(256, std::min<int64_t>(4096, (RT + SR - 1) / SR * SR));
  if (const char *env = getenv("SLM_PROJ_RT")) {
    const long long v = atoll(env);
    if (v >= SR && v <= 65536) RT = (v + SR - 1) / SR * SR;
  }
  const int64_t grid = num_items(a.n_nodes, a.N, RT) * n_pt;
  if (grid == 0) return SLM_OK;
  SLM_CHECK(grid < (1ll << 31), SLM_E_SHAPE, "slm_project: grid too large");
  if (a.D <= 8) return launch_short_k<FN, WAVES, 4>(a, RT, grid, s);
  if (a.D <= 16) return launch_short_k<FN, WAVES, 8>(a, RT, grid, s);
  if (a.D <= 32) return launch_short_k<FN, WAVES, 16>(a, RT, grid, s);
  return launch_short_k<FN, WAVES, 32>(a, RT, grid, s);
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
  // D <= 64: register-resident directions, 256 / 128 / 32 particles per work-group.
  if (a.D <= 64) {
    if (a.P > 128) return launch_short<2, 4>(a, s);
    if (a.P > 32) return launch_short<2, 2>(a, s);
    return launch_short<1, 1>(a, s);
  }
  // Tile shape by particle count: wide tiles for large swarms, a single
  // 32-particle column block for small ones (and for P = 1 recomputation).
  if (a.P >= 128) return launch_cfg<128, 128, 2, 2>(a, s);
  if (a.P > 32) return launch_cfg<128, 64, 2, 2>(a, s);
  return launch_cfg<128, 32, 4, 1>(a, s);
}

}  // namespace slm
