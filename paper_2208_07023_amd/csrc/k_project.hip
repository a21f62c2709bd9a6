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
#include <string>
#include <vector>

namespace slm {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

int num_cus_proj() {
  static int n = 0;
  if (!n) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) {
      (void)hipGetLastError();
      n = 256;
    }
  }
  return n;
}

constexpr int KC = 64;          // dimensions staged per LDS round
constexpr int LDSTR = KC + 1;   // odd stride: the 32 rows a fragment reads hit 32 banks

template <bool BF16>
__device__ __forceinline__ float load_x(const void *p, int64_t idx) {
  if constexpr (BF16) return bf16_to_f32(static_cast<const uint16_t *>(p)[idx]);
  else return static_cast<const float *>(p)[idx];
}

template <int BM, int BN, int WM, int WN, bool XB, bool WB>
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
                     ? load_x<XB>(a.X, row * D + k0 + c) : 0.f;
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
        val[u] = (e < BN * KC && c < kc && p < P) ? load_x<WB>(a.W, (wbase + p) * D + k0 + c) : 0.f;
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

// Short projections (D <= 64), without LDS.  Lane (i, h) of a wave supplies
// row i of a 32-row sub-tile and k = h KSP + s at MFMA step s (s < KSP), so a
// lane's A operand is a contiguous run of its X row and its B operand a
// contiguous run of its W row, both read with 16-byte loads straight from
// global memory (scalar loads when D is not a multiple of 4).  Each wave
// keeps the B fragments of its 32 FN particles in registers while the node
// stays the same and double-buffers the A operand in registers: the next
// sub-tile is loaded while the current one's MFMAs run.  A work-group walks a
// contiguous range of rows across node boundaries (rows of no node are
// skipped); its waves take different particle blocks of the same rows.  D is
// padded with zeros to 2 KSP; the accumulation order over k depends on KSP
// alone, so every output element is the same MFMA sequence whatever FN,
// WAVES and the split of the rows.
constexpr int SR = 32;             // rows per sub-tile

struct SubTile {
  int j;                           // node (-1: none left)
  int64_t lo, hi;                  // rows lo .. hi-1 of node j, hi - lo <= SR
  int64_t end;                     // end of node j's rows inside the run
};

// First sub-tile of rows >= r inside [.., r_end), starting the search at node j.
// With a.vpre, r and r_end count the nodes' rows alone (node j's rows are
// vpre[j] .. vpre[j+1]-1 of that count) and the sub-tile is in data rows.
__device__ __forceinline__ SubTile next_subtile(const ProjectArgs &a, int j, int64_t r,
                                                int64_t r_end) {
  if (a.vpre) {
    for (; j < a.n_nodes; ++j) {
      const int64_t v0 = a.vpre[j], v1 = a.vpre[j + 1];
      if (v0 >= r_end) break;
      const int64_t vl = r > v0 ? r : v0;
      if (vl < v1) {
        const Range nr = load_range(a.beg, a.end, j, a.N);
        const int64_t lo = nr.lo + (vl - v0);
        int64_t hi = nr.lo + ((v1 < r_end ? v1 : r_end) - v0);
        hi = hi < nr.hi ? hi : nr.hi;
        if (lo >= hi) continue;
        return {j, lo, hi < lo + SR ? hi : lo + SR, hi};
      }
    }
    return {-1, 0, 0, 0};
  }
  for (; j < a.n_nodes; ++j) {
    const Range nr = load_range(a.beg, a.end, j, a.N);
    const int64_t lo = r > nr.lo ? r : nr.lo;
    if (lo >= r_end) break;
    if (lo < nr.hi) {
      const int64_t hi = nr.hi < r_end ? nr.hi : r_end;
      return {j, lo, hi < lo + SR ? hi : lo + SR, hi};
    }
  }
  return {-1, 0, 0, 0};
}


// MASK = false leaves rows and dimensions outside the data as loaded (from a
// clamped address) instead of zeroing them, so nothing consumes the loads
// before the MFMAs do and they stay in flight: used for the A operand (X),
// whose out-of-range rows are never stored and whose dimensions past D meet
// zeros in the (masked) B operand.
template <int KSP, bool BF16, bool VEC, bool MASK = true>
__device__ __forceinline__ void load_run(const void *base, int64_t row, int D, int k0, bool ok,
                                         float (&v)[KSP]) {
  if constexpr (VEC) {
#pragma unroll
    for (int q = 0; q < KSP / 4; ++q) {
      const int kk = k0 + 4 * q;
      const bool in = !MASK || (ok && kk < D);
      const int64_t idx = row * D + (kk < D ? kk : 0);
      float t[4];
      if constexpr (BF16) {
        const uint2 u = *reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(base) + idx);
        t[0] = bf16_to_f32((uint16_t)(u.x & 0xFFFFu));
        t[1] = bf16_to_f32((uint16_t)(u.x >> 16));
        t[2] = bf16_to_f32((uint16_t)(u.y & 0xFFFFu));
        t[3] = bf16_to_f32((uint16_t)(u.y >> 16));
      } else {
        const float4 f = *reinterpret_cast<const float4 *>(static_cast<const float *>(base) + idx);
        t[0] = f.x;
        t[1] = f.y;
        t[2] = f.z;
        t[3] = f.w;
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) v[4 * q + e] = in ? t[e] : 0.f;
    }
  } else {
#pragma unroll
    for (int s = 0; s < KSP; ++s) {
      const int kk = k0 + s;
      const float t = load_x<BF16>(base, row * D + (kk < D ? kk : D - 1));
      v[s] = (!MASK || (ok && kk < D)) ? t : 0.f;
    }
  }
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// The nearest bfloat16 of x (ties to even), as a float.
__device__ __forceinline__ float round_bf16(float x) {
  const bf16x2_t v = {(__bf16)x, (__bf16)x};
  return __uint_as_float(__builtin_bit_cast(uint32_t, v) << 16);
}

// Two floats as a packed pair of bfloat16 (a low, b high), each rounded to
// nearest even (one v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  const bf16x2_t v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}

// 4 x 4 transpose of 8-lane groups within each 32-lane half of the wave:
// register i, lane group u (lanes 8u .. 8u+7 of the half) <-> register u,
// lane group i.  From the matrix-core layout (register 4g + i holds row
// 8g + i (+4 in the upper half), lane l%32 particle l%32 of the block) this
// gives register t: row 8g + (l%32)/8 (+4), particle 8t + l%8, so one store
// per register writes rows 8g .. 8g+7 of the 8-particle tile t, 256
// contiguous bytes of an 8-wide particle-tiled Z.  Two steps: swap of 8-lane
// groups inside 16-lane rows (row rotation by 8 and a select), then of
// 16-lane rows between register pairs (v_permlane16_swap).
__device__ __forceinline__ void transpose_lane_groups(uint32_t (&a)[4], int lane) {
  const bool u0 = (lane >> 3) & 1;
  uint32_t c[4];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const uint32_t e = a[2 * k], o = a[2 * k + 1];
    const uint32_t ro = __builtin_amdgcn_update_dpp(0u, o, 0x128, 0xf, 0xf, false);   // row_ror:8
    const uint32_t re = __builtin_amdgcn_update_dpp(0u, e, 0x128, 0xf, 0xf, false);
    c[2 * k] = u0 ? ro : e;
    c[2 * k + 1] = u0 ? o : re;
  }
#pragma unroll
  for (int i0 = 0; i0 < 2; ++i0) {
    const auto r = __builtin_amdgcn_permlane16_swap(c[i0], c[2 + i0], false, false);
    a[i0] = r[0];
    a[2 + i0] = r[1];
  }
}

// STORE = false: only the per-column min / max (a.Z is not written), the
// first pass of the fused evaluation.  ZT: the tile width of a particle-tiled
// Z (32 or 8) as a constant, or 0 (row-major: the stride is read from the
// layout).  With 32-wide tiles the 16 stores of an accumulator block use
// immediate offsets from one address; with 8-wide tiles the block is first
// transposed in registers (transpose_lane_groups) so that every store writes
// 256 contiguous bytes.
// The row loop is unrolled twice over two A buffers: the loads of the next
// sub-tile go to the buffer the current MFMAs do not read.  A node change
// (flush of the min / max, B fragments of the new node) happens before the
// next sub-tile's loads are issued, so the MFMAs only wait for the B loads.
// Full sub-tiles take a straight-line epilogue; sub-tiles cut by a node end or
// columns past P take a masked one.
template <int FN, int WAVES, int KSP, bool XB, bool VEC, bool STORE, int ZT>
__global__ __launch_bounds__(64 * WAVES) void k_project_short(ProjectArgs a, int64_t RB,
                                                              int blocks_per_pt) {
  constexpr int PTILE = 32 * FN * WAVES;
  const int pt = blockIdx.x / blocks_per_pt;
  if (a.n_nodes <= 0) return;
  // rows of the run: data rows, or (a.vpre) rows of the nodes alone, whose
  // count is read here so that a captured launch serves any node sizes
  const int64_t n_rows = a.vpre ? a.vpre[a.n_nodes] : a.N;
  if (a.vpre) RB = ((n_rows + blocks_per_pt - 1) / blocks_per_pt + SR - 1) / SR * SR;
  const int64_t r_begin = (int64_t)(blockIdx.x % blocks_per_pt) * RB;
  const int64_t r_end = r_begin + RB < n_rows ? r_begin + RB : n_rows;
  if (r_begin >= r_end) return;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int D = a.D, P = a.P;
  const int li = lane & 31, kh = lane >> 5, k0 = kh * KSP;
  const int pw = pt * PTILE + wave * 32 * FN;   // first particle of this wave
  const bool wave_full = pw + 32 * FN <= P;     // every column of the wave exists
  const int64_t rs = ZT ? (int64_t)ZT : a.zl.rs;
  const bool do_mm = a.zmin != nullptr;

  // first node whose rows reach past r_begin (ends are non-decreasing)
  int j0 = 0;
  {
    int lo = 0, hi = a.n_nodes;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const int64_t e = a.vpre ? a.vpre[mid + 1] : load_range(a.beg, a.end, mid, a.N).hi;
      if (e <= r_begin) lo = mid + 1; else hi = mid;
    }
    j0 = lo;
  }
  SubTile cur = next_subtile(a, j0, r_begin, r_end);
  if (cur.j < 0) return;

  float bfrag[FN][KSP];
  float mn[FN], mx[FN];
  int node_c = -1;
  auto flush = [&]() {
    if (node_c < 0 || !do_mm) return;
    const int64_t wb = (int64_t)node_c * P;
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      const int p = pw + f * 32 + li;
      const float m0 = fminf(mn[f], __shfl_xor(mn[f], 32));
      const float m1 = fmaxf(mx[f], __shfl_xor(mx[f], 32));
      if (lane < 32 && p < P && m0 <= m1) {
        atomic_min_f32(&a.zmin[wb + p], m0);
        atomic_max_f32(&a.zmax[wb + p], m1);
      }
    }
  };
  // node change: publish the finished node's min / max, load the new node's
  // directions
  auto prep = [&](const SubTile &c) {
    if (c.j == node_c) return;
    flush();
    node_c = c.j;
    const int64_t wb = (int64_t)node_c * P;
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      const int p = pw + f * 32 + li;
      load_run<KSP, false, VEC>(a.W, wb + (p < P ? p : P - 1), D, k0, p < P, bfrag[f]);
      mn[f] = __builtin_huge_valf();
      mx[f] = -__builtin_huge_valf();
    }
    // Wait for the B loads here, on this rare path: a wait placed after the
    // paths merge would also hold the common path until its stores drain
    // (the vector memory counter counts stores too).
#pragma unroll
    for (int f = 0; f < FN; ++f)
#pragma unroll
      for (int k = 0; k < KSP; ++k) asm volatile("" ::"v"(bfrag[f][k]));
  };
  auto load_a = [&](const SubTile &c, float (&A)[KSP]) {
    const bool ok = c.lo + li < c.hi;
    load_run<KSP, XB, VEC, false>(a.X, ok ? c.lo + li : c.hi - 1, D, k0, ok, A);
  };
  auto mma = [&](const float (&A)[KSP], f32x16 (&acc)[FN]) {
#pragma unroll
    for (int f = 0; f < FN; ++f) acc[f] = f32x16{};
#pragma unroll
    for (int ks = 0; ks < KSP; ++ks)
#pragma unroll
      for (int f = 0; f < FN; ++f)
        acc[f] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[ks], bfrag[f][ks], acc[f], 0, 0, 0);
  };
  // Lane l, register r holds row 8*(r/4) + 4*(l/32) + r%4 of the sub-tile and
  // particle column l%32 of block f.
  // Full sub-tile (32 rows, every column of the wave real): 16 stores per
  // block from one address with immediate offsets.
  auto compute_full = [&](int64_t lo, const float (&A)[KSP]) {
    f32x16 acc[FN];
    mma(A, acc);
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      if constexpr (STORE && ZT == 8) {
        // register t of group g after the transpose: row 8g + lane/8,
        // particle 8t + lane%8 of the block
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          uint32_t v[4] = {__float_as_uint(acc[f][4 * g]), __float_as_uint(acc[f][4 * g + 1]),
                           __float_as_uint(acc[f][4 * g + 2]), __float_as_uint(acc[f][4 * g + 3])};
          transpose_lane_groups(v, lane);
#pragma unroll
          for (int t = 0; t < 4; ++t)
            a.Z[z_col(a.zl, pw + f * 32 + 8 * t) + (lo + 8 * g) * 8 + lane] = __uint_as_float(v[t]);
        }
      } else if constexpr (STORE) {
        float *zc = a.Z + z_col(a.zl, pw + f * 32 + li) + (lo + 4 * kh) * rs;
#pragma unroll
        for (int r = 0; r < 16; ++r) zc[(int64_t)(8 * (r >> 2) + (r & 3)) * rs] = acc[f][r];
      }
      float l = acc[f][0], h = acc[f][0];
#pragma unroll
      for (int r = 1; r < 16; ++r) {
        l = fminf(l, acc[f][r]);
        h = fmaxf(h, acc[f][r]);
      }
      mn[f] = fminf(mn[f], l);
      mx[f] = fmaxf(mx[f], h);
    }
  };
  // Sub-tile cut by the node's end, or a wave with columns past P: buffer
  // stores whose offset is set out of range (rows past the sub-tile, columns
  // past P) are dropped by the hardware.
  auto compute_masked = [&](const SubTile &c, const float (&A)[KSP]) {
    f32x16 acc[FN];
    mma(A, acc);
    const int nrow = (int)(c.hi - c.lo);
    // lane column offset within the block's 32 particles (tiles of 8 put
    // them in 4 tiles), and the block's span; both < 2^31 bytes (the
    // layout is checked on the host)
    const int lcol = (int)z_col(a.zl, li);
    const uint32_t nb = (uint32_t)((z_col(a.zl, 31) + nrow * rs) * 4);
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      const bool pin = pw + f * 32 + li < P;
      if constexpr (STORE) {
        const __amdgpu_buffer_rsrc_t zr = __builtin_amdgcn_make_buffer_rsrc(
            a.Z + z_col(a.zl, pw + f * 32) + c.lo * rs, 0, nb, BUF_DW3);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 4 * kh + 8 * (r >> 2) + (r & 3);
          const uint32_t off =
              pin && row < nrow ? (uint32_t)((row * (int)rs + lcol) * 4) : 0x80000000u;
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(acc[f][r]), zr, (int)off, 0, 0);
        }
      }
      float l = __builtin_nanf(""), h = __builtin_nanf("");
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 4 * kh + 8 * (r >> 2) + (r & 3);
        const float z = pin && row < nrow ? acc[f][r] : __builtin_nanf("");
        l = fminf(l, z);
        h = fmaxf(h, z);
      }
      mn[f] = fminf(mn[f], l);
      mx[f] = fmaxf(mx[f], h);
    }
  };
  auto load_full = [&](int64_t lo, float (&A)[KSP]) {
    load_run<KSP, XB, VEC, false>(a.X, lo + li, D, k0, true, A);
  };

  // Node by node: the node's directions (prep), its full sub-tiles in a
  // ping-pong loop whose only branches are its exits -- so the waits before
  // each MFMA chain are for that chain's A operand alone, never for the
  // previous sub-tile's stores (the vector memory counter counts both, in
  // order) -- then its ragged last sub-tile.
  float A0[KSP], A1[KSP];
  // (the next node's rows all lie past r_begin, in either count)
  for (SubTile c = cur; c.j >= 0; c = next_subtile(a, c.j + 1, r_begin, r_end)) {
    const int64_t end = c.end;
    const int64_t nfull = wave_full ? (end - c.lo) / SR : 0;
    int64_t r = c.lo;
    // the first A tile is loaded together with the node's B fragments
    // (prep waits for both)
    if (nfull > 0) load_full(r, A0);
    prep(c);
    if (nfull > 0) {
#pragma unroll
      for (int k = 0; k < KSP; ++k) asm volatile("" ::"v"(A0[k]));
      int64_t s = 0;
      while (true) {
        load_full(s + 1 < nfull ? r + SR : r, A1);
        compute_full(r, A0);
        if (++s == nfull) break;
        r += SR;
        load_full(s + 1 < nfull ? r + SR : r, A0);
        compute_full(r, A1);
        if (++s == nfull) break;
        r += SR;
      }
      r += SR;
    }
    while (r < end) {   // rows not in a full sub-tile of a full wave
      const SubTile t{c.j, r, r + SR < end ? r + SR : end, end};
      load_a(t, A0);
      compute_masked(t, A0);
      r = t.hi;
    }
  }
  flush();
}

// X float32 or bfloat16, W float32 (both widened exactly to float32)
template <int FN, int WAVES, int KSP, bool VEC, int ZT>
slm_status launch_short_g(const ProjectArgs &a, int64_t RB, int bpp, int64_t grid, hipStream_t s) {
  const dim3 blk(64 * WAVES);
  if (a.Z == nullptr)   // min / max only (X float32)
    hipLaunchKernelGGL((k_project_short<FN, WAVES, KSP, false, VEC, false, 0>),
                       dim3((unsigned)grid), blk, 0, s, a, RB, bpp);
  else if (a.x_bf16)
    hipLaunchKernelGGL((k_project_short<FN, WAVES, KSP, true, VEC, true, ZT>),
                       dim3((unsigned)grid), blk, 0, s, a, RB, bpp);
  else
    hipLaunchKernelGGL((k_project_short<FN, WAVES, KSP, false, VEC, true, ZT>),
                       dim3((unsigned)grid), blk, 0, s, a, RB, bpp);
  SLM_LAUNCHED();
  return SLM_OK;
}

// the tile width of a particle-tiled Z, 0 for row-major
inline int z_tile_width(const ZLayout &l) {
  if (l.rs == 32 && l.sh == 5) return 32;   // (also row-major with P = 32: the same placement)
  if (l.rs == 8 && l.sh == 3) return 8;
  return 0;
}

template <int FN, int WAVES, int KSP, bool VEC>
slm_status launch_short_k(const ProjectArgs &a, int64_t RB, int bpp, int64_t grid, hipStream_t s) {
  const int zt = z_tile_width(a.zl);
  if (zt == 32) return launch_short_g<FN, WAVES, KSP, VEC, 32>(a, RB, bpp, grid, s);
  if (zt == 8) return launch_short_g<FN, WAVES, KSP, VEC, 8>(a, RB, bpp, grid, s);
  return launch_short_g<FN, WAVES, KSP, VEC, 0>(a, RB, bpp, grid, s);
}

template <int FN, int WAVES, bool VEC>
slm_status launch_short_v(const ProjectArgs &a, int64_t RB, int bpp, int64_t grid, hipStream_t s) {
  if (a.D <= 8) return launch_short_k<FN, WAVES, 4, VEC>(a, RB, bpp, grid, s);
  if (a.D <= 16) return launch_short_k<FN, WAVES, 8, VEC>(a, RB, bpp, grid, s);
  if (a.D <= 32) return launch_short_k<FN, WAVES, 16, VEC>(a, RB, bpp, grid, s);
  return launch_short_k<FN, WAVES, 32, VEC>(a, RB, bpp, grid, s);
}

template <int FN, int WAVES>
slm_status launch_short(const ProjectArgs &a, hipStream_t s) {
  constexpr int PTILE = 32 * FN * WAVES;
  const int64_t n_pt = (a.P + PTILE - 1) / PTILE;
  // One wave per SIMD over the whole launch (measured faster than two: a
  // wave keeps its SIMD's matrix core busy on its own, and longer runs
  // amortise its prologue); each work-group takes a contiguous run of whole
  // 32-row sub-tiles (SLM_PROJ_RT overrides the run length).
  //
  // With a.vpre the runs split the nodes' rows alone (the kernel reads their
  // count), so a depth whose nodes hold a small part of the data (the last
  // levels of trees grown together) still spreads over the whole chip.
  const int64_t cap = std::max<int64_t>(1, (int64_t)num_cus_proj() * 4 / WAVES);
  int64_t bpp = std::max<int64_t>(1, std::min<int64_t>((a.N + SR - 1) / SR, cap / n_pt));
  int64_t RB = ((a.N + bpp - 1) / bpp + SR - 1) / SR * SR;
  if (!a.vpre) bpp = (a.N + RB - 1) / RB;
  if (const char *env = a.vpre ? nullptr : getenv("SLM_PROJ_RT")) {
    const long long v = atoll(env);
    if (v >= 1 && v <= (1 << 24)) {
      RB = v;
      bpp = (a.N + RB - 1) / RB;
    }
  }
  const int64_t grid = bpp * n_pt;
  if (grid == 0) return SLM_OK;
  SLM_CHECK(grid < (1ll << 31), SLM_E_SHAPE, "slm_project: grid too large");
  const size_t es = a.x_bf16 ? 8 : 16;   // bytes of one vector load of X (W is float32)
  const bool vec = a.D % 4 == 0 && reinterpret_cast<uintptr_t>(a.X) % es == 0 &&
                   reinterpret_cast<uintptr_t>(a.W) % 16 == 0;
  if (vec) return launch_short_v<FN, WAVES, true>(a, RB, (int)bpp, grid, s);
  return launch_short_v<FN, WAVES, false>(a, RB, (int)bpp, grid, s);
}

// bfloat16 projection on the bfloat16 matrix cores (v_mfma_f32_32x32x16_bf16,
// float32 accumulation): X [N, D] and W [n_nodes P, D] both bfloat16.
// A work-group computes a BM x BN tile of Z (4 waves of 64 x 64); tiles of BKC
// dimensions of X and W are staged in LDS as bfloat16 (rows padded to 144
// bytes, 16-byte aligned) and each lane feeds the MFMA 8 consecutive
// dimensions of its row straight from one 16-byte LDS read.  Work-groups are
// ordered so that the particle tiles of one row tile run on one XCD (its L2
// serves the X tile to all of them).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int BKC = 64;          // dimensions staged per LDS round
constexpr int BST = BKC + 8;     // LDS row stride in bfloat16 elements

// 8 consecutive bfloat16 of one row starting at dimension k (k % 8 == 0),
// zeros past D.  VEC: D % 8 == 0 and 16-byte aligned rows.
template <bool VEC>
__device__ __forceinline__ uint4 load8_bf16(const uint16_t *row, int k, int D) {
  if constexpr (VEC) {
    return *reinterpret_cast<const uint4 *>(row + k);
  } else {
    uint32_t w[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int k0 = k + 2 * h, k1 = k0 + 1;
      const uint32_t lo = k0 < D ? row[k0] : 0u;
      const uint32_t hi = k1 < D ? row[k1] : 0u;
      w[h] = lo | (hi << 16);
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
  }
}

template <int BM, int BN, bool VEC>
__global__ __launch_bounds__(256) void k_project_bf16(ProjectArgs a, int n_pt, int64_t n_items) {
  constexpr int WM = 2, WN = 2, TM = BM / WM, TN = BN / WN, FM = TM / 32, FN = TN / 32;
  constexpr int CPR = BKC / 8;                       // 16-byte chunks per staged row
  constexpr int XPT = BM * CPR / 256, WPT = BN * CPR / 256;
  static_assert(FM >= 1 && FN >= 1 && XPT >= 1 && WPT >= 1, "tile shape");
  __shared__ __align__(16) uint16_t Xs[BM * BST];
  __shared__ __align__(16) uint16_t Ws[BN * BST];

  const int64_t bid = blockIdx.x;
  const int64_t local = bid >> 3;
  const int64_t v = (local / n_pt) * 8 + (bid & 7);
  const int pt = (int)(local % n_pt);
  if (v >= n_items) return;
  const Item it = find_item(a.beg, a.end, a.n_nodes, a.N, BM, v);
  if (it.node < 0) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int li = lane & 31, kh = lane >> 5;
  const int64_t r0 = (it.lo / BM) * BM;
  const int p0 = pt * BN;
  const int D = a.D, P = a.P;
  const int64_t wbase = (int64_t)it.node * P;
  const uint16_t *X = static_cast<const uint16_t *>(a.X);
  const uint16_t *W = static_cast<const uint16_t *>(a.W);

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int f = 0; f < FN; ++f) acc[i][f] = f32x16{};

  for (int k0 = 0; k0 < D; k0 += BKC) {
    uint4 xv[XPT], wv[WPT];
#pragma unroll
    for (int u = 0; u < XPT; ++u) {
      const int e = tid + u * 256, r = e / CPR, c = (e % CPR) * 8;
      const int64_t row = r0 + r;
      const bool in = row >= it.lo && row < it.hi && k0 + c < D;
      xv[u] = in ? load8_bf16<VEC>(X + row * D, k0 + c, D) : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
      const int e = tid + u * 256, r = e / CPR, c = (e % CPR) * 8;
      const int p = p0 + r;
      const bool in = p < P && k0 + c < D;
      wv[u] = in ? load8_bf16<VEC>(W + (wbase + p) * D, k0 + c, D) : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int u = 0; u < XPT; ++u) {
      const int e = tid + u * 256;
      *reinterpret_cast<uint4 *>(&Xs[(e / CPR) * BST + (e % CPR) * 8]) = xv[u];
    }
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
      const int e = tid + u * 256;
      *reinterpret_cast<uint4 *>(&Ws[(e / CPR) * BST + (e % CPR) * 8]) = wv[u];
    }
    lds_barrier();
    const int ksteps = min(BKC, D - k0 + 15) / 16;
    for (int ks = 0; ks < ksteps; ++ks) {
      const int kk = ks * 16 + kh * 8;
      bf16x8 af[FM], bfr[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        af[i] = __builtin_bit_cast(bf16x8,
                                   *reinterpret_cast<const uint4 *>(&Xs[(wm * TM + i * 32 + li) * BST + kk]));
#pragma unroll
      for (int f = 0; f < FN; ++f)
        bfr[f] = __builtin_bit_cast(bf16x8,
                                    *reinterpret_cast<const uint4 *>(&Ws[(wn * TN + f * 32 + li) * BST + kk]));
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int f = 0; f < FN; ++f)
          acc[i][f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bfr[f], acc[i][f], 0, 0, 0);
    }
    lds_barrier();
  }

  // Epilogue: lane l, register r holds row 8*(r/4) + 4*(l/32) + r%4 and
  // column l%32 of each 32x32 block.
  const bool do_mm = a.zmin != nullptr;
#pragma unroll
  for (int f = 0; f < FN; ++f) {
    const int p = p0 + wn * TN + f * 32 + li;
    float mn = __builtin_huge_valf(), mx = -__builtin_huge_valf();
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rr = wm * TM + i * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
        const int64_t row = r0 + rr;
        if (p < P && row >= it.lo && row < it.hi) {
          const float z = acc[i][f][r];
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

template <int BM, int BN>
slm_status launch_bf16(const ProjectArgs &a, hipStream_t s) {
  const int64_t items = num_items(a.n_nodes, a.N, BM);
  const int64_t n_pt = (a.P + BN - 1) / BN;
  const int64_t grid = (items + 7) / 8 * 8 * n_pt;
  if (items == 0) return SLM_OK;
  SLM_CHECK(grid < (1ll << 31), SLM_E_SHAPE, "slm_project: grid of %lld blocks too large",
            (long long)grid);
  const bool vec = a.D % 8 == 0 && reinterpret_cast<uintptr_t>(a.X) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(a.W) % 16 == 0;
  if (vec)
    hipLaunchKernelGGL((k_project_bf16<BM, BN, true>), dim3((unsigned)grid), dim3(256), 0, s, a,
                       (int)n_pt, items);
  else
    hipLaunchKernelGGL((k_project_bf16<BM, BN, false>), dim3((unsigned)grid), dim3(256), 0, s, a,
                       (int)n_pt, items);
  SLM_LAUNCHED();
  return SLM_OK;
}

// ---------------------------------------------------------------- streaming projection
// W-stationary projection for D > 64 (float32 data) and for bfloat16 data.
// A work-group of SW = 4 waves owns PT = 32 FN particles of the current
// node: their directions sit in LDS in MFMA fragment order (each lane's
// operand of one step is one 16-byte LDS read, 64 lanes read 1 KB
// contiguously, no bank conflicts), loaded once per node.  Each wave takes
// its own 32-row sub-tiles (the work-group steps over the node's rows 128 at
// a time) and reads its A operand straight from global memory into
// registers, double-buffered across sub-tiles; every wave computes all PT
// particles of its rows, so each X row is read once per particle tile.
//
// The kernel takes D <= KCH dimensions (zero-padded to KCH).  Group q of the
// A operand is the row's q-th 32-byte piece: lanes 0-31 supply its first 16
// bytes and lanes 32-63 its second, so one A load touches a single 32-byte
// piece (one cache line) of each of the sub-tile's rows, and consecutive
// loads walk the rows' lines in order.  Larger D take the tile kernels.
// Three operand kinds:
//   MK_BB  X and W bfloat16: v_mfma_f32_32x32x16_bf16, KCH = 256 (16 steps
//          of 8 dimensions per half);
//   MK_XB  X bfloat16, W float32: each direction is split into three
//          bfloat16 parts, w = w1 + w2 + w3 (w1 = bf16(w), w2 = bf16(w - w1),
//          w3 = bf16(w - w1 - w2), each remainder exact in float32), kept
//          as three fragment planes in LDS; v_mfma_f32_32x32x16_bf16 over
//          the three planes into three accumulators (every product exact,
//          float32 accumulation), added as acc1 + (acc2 + acc3) at the end,
//          KCH = 256;
//   MK_FF  X and W float32: v_mfma_f32_32x32x2f32, KCH = 128 (64 steps).
// Dimensions past D are zero in W (the A operand there holds whatever
// finite X values the clamped loads read).  Each output element is the same
// MFMA sequence whatever FN, the grid and the row split, so a column
// recomputed alone (P = 1, the partition) is bit-identical to the column
// computed among many particles.
constexpr int MK_BB = 0, MK_XB = 1, MK_FF = 2;
constexpr int SW = 4;   // waves per work-group, one per SIMD

template <int MK>
struct StreamOps {
  static constexpr int KCH = MK == MK_FF ? 128 : 256;   // dimensions per chunk
  static constexpr int XBYTES = MK == MK_FF ? 4 : 2;     // bytes per X element
  static constexpr int WBYTES = MK == MK_FF ? 4 : 2;     // bytes per LDS W element
  static constexpr int PLANES = MK == MK_XB ? 3 : 1;     // W planes (bfloat16 parts)
  // 16-byte W groups per lane and chunk: the lane's half-chunk of W, per plane
  static constexpr int GP = KCH / 2 * WBYTES / 16;
  static constexpr int G = GP * PLANES;
};

// LDS of a work-group's W tile: FN blocks of G 1-KB fragment groups.
__host__ __device__ constexpr size_t stream_lds_bytes(int MK, int FN) {
  return (size_t)FN * (MK == MK_XB ? 48 : 16) * 1024;
}
// bfloat16 Z goes out through a per-wave LDS staging area: the
// eight-particle tiles of one 32-particle block (FN odd) or of one pair of
// blocks (64 particles, FN even) of a sub-tile, 32 rows of 16 bytes each
// plus one row of padding (so the lanes of one row write distinct banks),
// reused block after block (a wave's LDS accesses complete in order).
constexpr int STAGE_TILE = 33 * 16;
__host__ __device__ constexpr size_t stream_stage_bytes(int FN) {
  return (size_t)SW * (FN % 2 == 0 ? 8 : 4) * STAGE_TILE;
}
// The particle in MFMA column c (0..31) of accumulator block f, counted from
// the work-group's first particle.  With bfloat16 Z and an even FN, blocks
// 2m and 2m + 1 interleave the 64 particles 64 m .. 64 m + 63 (even ones in
// block 2m), so a lane holds two neighbouring particles of each row and
// rounds and stages them as one packed pair; otherwise block f holds
// particles 32 f .. 32 f + 31 in order.  Only the particle's MFMA column
// changes, not the sequence of operations that computes its projections.
template <bool ZB, int FN>
__device__ __forceinline__ int stream_particle(int f, int c) {
  if constexpr (ZB && FN % 2 == 0) return 64 * (f >> 1) + 2 * c + (f & 1);
  else return 32 * f + c;
}
// The dimensions one chunk covers: the kernel takes D <= KCH (one chunk).
__host__ __device__ constexpr int stream_kch(int MK) { return MK == MK_FF ? 128 : 256; }

// one 16-byte group of a row: elements e0 .. e0 + 16/EB - 1 (EB bytes each)
// of row `row` of a [*, D] matrix; elements past D read as zero when MASK,
// else from element 0 of the row (finite data, met by zeros in W).
template <int EB, bool VEC, bool MASK>
__device__ __forceinline__ uint4 load_group(const void *base, int64_t row, int D, int e0) {
  constexpr int NE = 16 / EB;
  if constexpr (VEC) {
    const bool in = e0 < D;
    const char *p = static_cast<const char *>(base) + (row * D + (in ? e0 : 0)) * EB;
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    if (MASK && !in) return make_uint4(0u, 0u, 0u, 0u);
    return v;
  } else {
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if constexpr (EB == 4) {
      const float *r = static_cast<const float *>(base) + row * D;
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int k = e0 + e;
        const float v = r[k < D ? k : 0];
        w[e] = (!MASK || k < D) ? __float_as_uint(v) : 0u;
      }
    } else {
      const uint16_t *r = static_cast<const uint16_t *>(base) + row * D;
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int k = e0 + e;
        const uint32_t v = r[k < D ? k : 0];
        w[e >> 1] |= ((!MASK || k < D) ? v : 0u) << (16 * (e & 1));
      }
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
  }
}

template <int MK, int FN, bool VEC, int ZT, bool ZB = false>
__global__ __launch_bounds__(64 * SW) void k_project_stream(ProjectArgs a, int64_t RB,
                                                            int blocks_per_pt, int n_pt,
                                                            int xcd_map) {
  using O = StreamOps<MK>;
  constexpr int KCH = O::KCH, G = O::G, XB = O::XBYTES;
  constexpr int PT = 32 * FN;
  extern __shared__ __align__(16) uint4 wl[];   // [f][g][lane]
  if (a.n_nodes <= 0) return;
  // work-group -> (particle tile, row run).  xcd_map: work-groups are dealt
  // to the 8 XCDs round robin; the particle tiles of one row run are kept on
  // one XCD so that its L2 serves the run's X rows to all of them.
  int pt, run;
  {
    const int b = blockIdx.x;
    if (xcd_map) {
      const int x = b & 7, q = b >> 3;
      pt = q % n_pt;
      run = x * (blocks_per_pt >> 3) + q / n_pt;
    } else {
      pt = b / blocks_per_pt;
      run = b % blocks_per_pt;
    }
  }
  const int64_t n_rows = a.vpre ? a.vpre[a.n_nodes] : a.N;
  if (a.vpre) RB = ((n_rows + blocks_per_pt - 1) / blocks_per_pt + SR - 1) / SR * SR;
  const int64_t r_begin = (int64_t)run * RB;
  const int64_t r_end = r_begin + RB < n_rows ? r_begin + RB : n_rows;
  if (r_begin >= r_end) return;
  const int D = a.D, P = a.P;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 31, kh = lane >> 5;
  const int p0 = pt * PT;
  const bool tile_full = p0 + PT <= P;
  const int64_t rs = ZT ? (int64_t)ZT : a.zl.rs;
  const bool do_mm = a.zmin != nullptr;
  const int64_t row_bytes = (int64_t)D * XB;

  int j0 = 0;
  {
    int lo = 0, hi = a.n_nodes;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const int64_t e = a.vpre ? a.vpre[mid + 1] : load_range(a.beg, a.end, mid, a.N).hi;
      if (e <= r_begin) lo = mid + 1; else hi = mid;
    }
    j0 = lo;
  }

  float mn[FN], mx[FN];
  // the node's W tile into LDS, fragment order: group g of lane (li, h) in
  // block f holds W elements g (32 / WBYTES) + h (16 / WBYTES) ..., the
  // dimensions of A's group g on that lane
  auto fill_w = [&](int j) {
    const int64_t wb = (int64_t)j * P;
    if constexpr (MK == MK_XB) {
      // unit (f, g, lane): 8 float32 of the lane's row, split into the three
      // bfloat16 planes at groups g, GP + g, 2 GP + g of block f
      constexpr int GP = O::GP;
      constexpr int units = FN * GP * 64;
      constexpr int UB = 4;
      for (int u0 = threadIdx.x; u0 < units; u0 += UB * 64 * SW) {
        uint4 v[UB][2];
#pragma unroll
        for (int e = 0; e < UB; ++e) {
          const int u = u0 + e * 64 * SW;
          const int l = u & 63, g = (u >> 6) % GP, f = u / (64 * GP);
          const int p = p0 + stream_particle<ZB, FN>(f, l & 31);
          const int e0 = g * 16 + (l >> 5) * 8;
          v[e][0] = v[e][1] = make_uint4(0u, 0u, 0u, 0u);
          if (u < units && p < P) {
            v[e][0] = load_group<4, VEC, true>(a.W, wb + p, D, e0);
            v[e][1] = load_group<4, VEC, true>(a.W, wb + p, D, e0 + 4);
          }
        }
#pragma unroll
        for (int e = 0; e < UB; ++e) {
          const int u = u0 + e * 64 * SW;
          if (u >= units) continue;
          const int l = u & 63, g = (u >> 6) % GP, f = u / (64 * GP);
          const uint32_t w[8] = {v[e][0].x, v[e][0].y, v[e][0].z, v[e][0].w,
                                 v[e][1].x, v[e][1].y, v[e][1].z, v[e][1].w};
          uint32_t h[3][4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float r0 = __uint_as_float(w[2 * i]), r1 = __uint_as_float(w[2 * i + 1]);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              const float b0 = round_bf16(r0), b1 = round_bf16(r1);
              h[q][i] = pack_bf16(b0, b1);
              r0 = __fsub_rn(r0, b0);
              r1 = __fsub_rn(r1, b1);
            }
          }
#pragma unroll
          for (int q = 0; q < 3; ++q)
            wl[((f * 3 + q) * GP + g) * 64 + l] = make_uint4(h[q][0], h[q][1], h[q][2], h[q][3]);
        }
      }
      return;
    }
    constexpr int units = FN * G * 64;
    constexpr int UB = 8;   // loads in flight per thread
    for (int u0 = threadIdx.x; u0 < units; u0 += UB * 64 * SW) {
      uint4 v[UB];
#pragma unroll
      for (int e = 0; e < UB; ++e) {
        const int u = u0 + e * 64 * SW;
        const int l = u & 63;
        const int g = (u >> 6) % G;
        const int f = u / (64 * G);
        const int p = p0 + stream_particle<ZB, FN>(f, l & 31);
        const int e0 = g * (32 / O::WBYTES) + (l >> 5) * (16 / O::WBYTES);
        v[e] = make_uint4(0u, 0u, 0u, 0u);
        if (u < units && p < P) v[e] = load_group<O::WBYTES, VEC, true>(a.W, wb + p, D, e0);
      }
#pragma unroll
      for (int e = 0; e < UB; ++e) {
        const int u = u0 + e * 64 * SW;
        if (u < units) wl[u] = v[e];
      }
    }
  };
  auto flush = [&](int j) {
    if (!do_mm) return;
    const int64_t wb = (int64_t)j * P;
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      const int p = p0 + stream_particle<ZB, FN>(f, li);
      float m0 = fminf(mn[f], __shfl_xor(mn[f], 32));
      float m1 = fmaxf(mx[f], __shfl_xor(mx[f], 32));
      if constexpr (ZB) {
        // the min / max of the stored (rounded) values: rounding is monotonic
        m0 = round_bf16(m0);
        m1 = round_bf16(m1);
      }
      if (lane < 32 && p < P && m0 <= m1) {
        atomic_min_f32(&a.zmin[wb + p], m0);
        atomic_max_f32(&a.zmax[wb + p], m1);
      }
    }
  };
  // A operand: 16 groups of 16 bytes, the lane's half of each 32-byte piece
  // of row lo + li (the sub-tile's last row for lanes past its n rows).  VEC: buffer loads from a resource at the sub-tile's first row,
  // so the per-load offsets are immediates and the row base is scalar.
  auto load_a = [&](int64_t lo, int n, uint4 (&A)[16]) {
    const int lr = li < n ? li : n - 1;
    if constexpr (VEC) {
      const char *base = static_cast<const char *>(a.X) + lo * row_bytes;
      const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<char *>(base), 0, (int)(n * row_bytes), BUF_DW3);
      const int vo = (int)(lr * row_bytes) + kh * 16;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(xr, vo + q * 32, 0, 0);
        A[q] = make_uint4(v[0], v[1], v[2], v[3]);
      }
    } else {
      const int e0 = kh * (16 / XB);
#pragma unroll
      for (int q = 0; q < 16; ++q)
        A[q] = load_group<XB, false, false>(a.X, lo + lr, D, e0 + q * (32 / XB));
    }
  };
  // The W fragments of step group q + 1 are read from LDS while the MFMAs of
  // group q run (two register sets).
  auto mma = [&](const uint4 (&A)[16], f32x16 (&acc)[FN]) {
    const uint4 *wc = wl + lane;
    if constexpr (MK == MK_BB) {
      uint4 b[2][FN];
#pragma unroll
      for (int f = 0; f < FN; ++f) b[0][f] = wc[(f * G) * 64];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        if (q + 1 < 16) {
#pragma unroll
          for (int f = 0; f < FN; ++f) b[(q + 1) & 1][f] = wc[(f * G + q + 1) * 64];
        }
#pragma unroll
        for (int f = 0; f < FN; ++f)
          acc[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, A[q]),
                                                           __builtin_bit_cast(bf16x8, b[q & 1][f]),
                                                           acc[f], 0, 0, 0);
      }
    } else if constexpr (MK == MK_XB) {
      // the three bfloat16 planes of W (groups q, GP + q, 2 GP + q of each
      // block) into three accumulators; W of step q + 1 is read while the
      // MFMAs of step q run
      constexpr int GP = O::GP;
      f32x16 a2[FN], a3[FN];
#pragma unroll
      for (int f = 0; f < FN; ++f) a2[f] = a3[f] = f32x16{};
      uint4 b[2][FN][3];
#pragma unroll
      for (int f = 0; f < FN; ++f)
#pragma unroll
        for (int q3 = 0; q3 < 3; ++q3) b[0][f][q3] = wc[((f * 3 + q3) * GP) * 64];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        if (q + 1 < 16) {
#pragma unroll
          for (int f = 0; f < FN; ++f)
#pragma unroll
            for (int q3 = 0; q3 < 3; ++q3)
              b[(q + 1) & 1][f][q3] = wc[((f * 3 + q3) * GP + q + 1) * 64];
        }
        const bf16x8 av = __builtin_bit_cast(bf16x8, A[q]);
#pragma unroll
        for (int f = 0; f < FN; ++f) {
          acc[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              av, __builtin_bit_cast(bf16x8, b[q & 1][f][0]), acc[f], 0, 0, 0);
          a2[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              av, __builtin_bit_cast(bf16x8, b[q & 1][f][1]), a2[f], 0, 0, 0);
          a3[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              av, __builtin_bit_cast(bf16x8, b[q & 1][f][2]), a3[f], 0, 0, 0);
        }
      }
#pragma unroll
      for (int f = 0; f < FN; ++f)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[f][r] = __fadd_rn(acc[f][r], __fadd_rn(a2[f][r], a3[f][r]));
    } else {
      uint4 b[2][FN];
#pragma unroll
      for (int f = 0; f < FN; ++f) b[0][f] = wc[(f * G) * 64];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        if (q + 1 < 16) {
#pragma unroll
          for (int f = 0; f < FN; ++f) b[(q + 1) & 1][f] = wc[(f * G + q + 1) * 64];
        }
        const uint32_t w4[4] = {A[q].x, A[q].y, A[q].z, A[q].w};
#pragma unroll
        for (int f = 0; f < FN; ++f) {
          const uint4 bq = b[q & 1][f];
          const uint32_t bw[4] = {bq.x, bq.y, bq.z, bq.w};
#pragma unroll
          for (int e = 0; e < 4; ++e)
            acc[f] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(w4[e]),
                                                          __uint_as_float(bw[e]), acc[f], 0, 0, 0);
        }
      }
    }
  };
  // Lane l, register r of block f holds row 8 (r/4) + 4 (l/32) + r%4 of the
  // sub-tile and particle p0 + 32 f + l%32.  Stores go through a buffer
  // resource at (block f, row lo): the lane's offset is fixed, each
  // register's row offset an immediate; rows past the sub-tile's n (and
  // columns past P) take an out-of-range offset, which the hardware drops.
  auto epilogue = [&](int64_t lo, int n, const f32x16 (&acc)[FN]) {
    const bool full = n == SR && tile_full;
    constexpr int EB = ZB ? 2 : 4;   // bytes per element of Z
    if constexpr (ZB && FN % 2 == 0) {
      // bfloat16, 8-wide tiles, blocks in interleaved pairs: lane (li, kh)
      // holds particles pb + 2 li (block f) and pb + 2 li + 1 (block f + 1)
      // of each of its rows, rounded to nearest even as one packed pair and
      // written as one 32-bit word of the staging area's tile row; each lane
      // then reads one 16-byte tile row and the wave writes two tiles' 32
      // rows per 16-byte store.  The pair's 8 tiles go out through two
      // resources of 4 tiles each, so the 32-bit offsets span what they do
      // for a single block.  Rows past the sub-tile's n and tiles past P are
      // dropped (an out-of-range offset); the columns past P of the last
      // tile take the zeros their padded directions project to.
      unsigned char *stg = reinterpret_cast<unsigned char *>(wl) + stream_lds_bytes(MK, FN) +
                           (size_t)wave * (8 * STAGE_TILE);
      unsigned char *wp = stg + (li >> 2) * STAGE_TILE + 4 * kh * 16 + (li & 3) * 4;
#pragma unroll
      for (int f = 0; f < FN; f += 2) {
        const int pb = p0 + 32 * f;
        float le = __builtin_huge_valf(), he = -__builtin_huge_valf();
        float lo_ = __builtin_huge_valf(), ho = -__builtin_huge_valf();
        // No masks: the A rows past the sub-tile's n repeat its last row
        // (load_a clamps them), so their projections equal that row's bit
        // for bit and leave the min / max unchanged; a particle past P is
        // never flushed.
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          le = fminf(le, acc[f][r]);
          he = fmaxf(he, acc[f][r]);
          lo_ = fminf(lo_, acc[f + 1][r]);
          ho = fmaxf(ho, acc[f + 1][r]);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r)
          *reinterpret_cast<uint32_t *>(wp + (8 * (r >> 2) + (r & 3)) * 16) =
              pack_bf16(acc[f][r], acc[f + 1][r]);
        // (the wave's own LDS writes and reads complete in order)
        const int64_t zb0 = z_col(a.zl, pb) + lo * rs, zb1 = z_col(a.zl, pb + 32) + lo * rs;
        const int nrec = (int)((z_col(a.zl, 31) + n * rs) * EB);
        const __amdgpu_buffer_rsrc_t zr0 = __builtin_amdgcn_make_buffer_rsrc(
            reinterpret_cast<char *>(a.Z) + zb0 * EB, 0, nrec, BUF_DW3);
        const __amdgpu_buffer_rsrc_t zr1 = __builtin_amdgcn_make_buffer_rsrc(
            reinterpret_cast<char *>(a.Z) + zb1 * EB, 0, nrec, BUF_DW3);
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
          const int t = 2 * s2 + (lane >> 5), row = lane & 31;
          const uint4 v = *reinterpret_cast<const uint4 *>(stg + t * STAGE_TILE + row * 16);
          const bool ok = row < n && pb + 8 * t < P;
          __builtin_amdgcn_raw_buffer_store_b128(
              __builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned int, v),
              s2 < 2 ? zr0 : zr1,
              ok ? (int)((lane >> 5) * a.zl.ts * 2) + row * 16 : (int)0x80000000,
              (int)(2 * (s2 & 1) * a.zl.ts * 2), Z_CPOL_NT);
        }
        mn[f] = fminf(mn[f], le);
        mx[f] = fmaxf(mx[f], he);
        mn[f + 1] = fminf(mn[f + 1], lo_);
        mx[f + 1] = fmaxf(mx[f + 1], ho);
      }
      return;
    }
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      const bool pin = p0 + f * 32 + li < P;
      const __amdgpu_buffer_rsrc_t zr = __builtin_amdgcn_make_buffer_rsrc(
          reinterpret_cast<char *>(a.Z) + (z_col(a.zl, p0 + f * 32) + lo * rs) * EB, 0,
          (int)((z_col(a.zl, 31) + n * rs) * EB), BUF_DW3);
      const int vo = (int)((4 * kh * rs + z_col(a.zl, li)) * EB);
      float l = __builtin_huge_valf(), h = -__builtin_huge_valf();
      if constexpr (ZB) {
        // bfloat16, 8-wide tiles, through this wave's LDS staging area:
        // every element goes in as a bfloat16 (nearest even) at (tile, row,
        // column), then each lane reads one 16-byte tile row and the wave
        // writes two tiles' 32 rows (two 512-byte runs) per 16-byte store.
        // Rows past the sub-tile's n and tiles past P are dropped (an
        // out-of-range offset); the columns past P of the last tile take
        // the zeros their padded directions project to.
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 4 * kh + 8 * (r >> 2) + (r & 3);
          const bool ok = full || (pin && row < n);
          l = fminf(l, ok ? acc[f][r] : __builtin_huge_valf());
          h = fmaxf(h, ok ? acc[f][r] : -__builtin_huge_valf());
        }
        unsigned char *stg = reinterpret_cast<unsigned char *>(wl) + stream_lds_bytes(MK, FN) +
                             (size_t)wave * (4 * STAGE_TILE);
        unsigned char *wp = stg + (li >> 3) * STAGE_TILE + 4 * kh * 16 + (li & 7) * 2;
#pragma unroll
        for (int r = 0; r < 16; ++r)
          *reinterpret_cast<unsigned short *>(wp + (8 * (r >> 2) + (r & 3)) * 16) =
              (unsigned short)pack_bf16(acc[f][r], acc[f][r]);
        // (the wave's own LDS writes and reads complete in order)
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
          const int t = 2 * s2 + (lane >> 5), row = lane & 31;
          const uint4 v = *reinterpret_cast<const uint4 *>(stg + t * STAGE_TILE + row * 16);
          const bool ok = row < n && p0 + f * 32 + 8 * t < P;
          __builtin_amdgcn_raw_buffer_store_b128(
              __builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned int, v), zr,
              ok ? (int)((lane >> 5) * a.zl.ts * 2) + row * 16 : (int)0x80000000,
              (int)(2 * s2 * a.zl.ts * 2), Z_CPOL_NT);
        }
      } else if (full && ZT == 8) {
        // 8-wide tiles: after the transpose, register t of group g holds
        // rows 8g + lane/8 of tile t (at t * ts), lane%8 its particle
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          l = fminf(l, acc[f][r]);
          h = fmaxf(h, acc[f][r]);
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          uint32_t v[4] = {__float_as_uint(acc[f][4 * g]), __float_as_uint(acc[f][4 * g + 1]),
                           __float_as_uint(acc[f][4 * g + 2]), __float_as_uint(acc[f][4 * g + 3])};
          transpose_lane_groups(v, lane);
#pragma unroll
          for (int t = 0; t < 4; ++t)
            __builtin_amdgcn_raw_buffer_store_b32(v[t], zr, lane * 4 + 256 * g,
                                                  (int)(t * a.zl.ts * 4), Z_CPOL_NT);
        }
      } else if (full) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int ro = (int)((8 * (r >> 2) + (r & 3)) * rs * 4);
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(acc[f][r]), zr, vo + ro, 0, 0);
          l = fminf(l, acc[f][r]);
          h = fmaxf(h, acc[f][r]);
        }
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 4 * kh + 8 * (r >> 2) + (r & 3);
          const bool ok = pin && row < n;
          const int off = ok ? vo + (int)((8 * (r >> 2) + (r & 3)) * rs * 4) : (int)0x80000000;
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(acc[f][r]), zr, off, 0, 0);
          l = fminf(l, ok ? acc[f][r] : __builtin_huge_valf());
          h = fmaxf(h, ok ? acc[f][r] : -__builtin_huge_valf());
        }
      }
      mn[f] = fminf(mn[f], l);
      mx[f] = fmaxf(mx[f], h);
    }
  };
  auto subtile = [&](int64_t lo, int n, const uint4 (&A)[16]) {
    f32x16 acc[FN];
#pragma unroll
    for (int f = 0; f < FN; ++f) acc[f] = f32x16{};
    mma(A, acc);
    epilogue(lo, n, acc);
  };

  uint4 A0[16], A1[16];
  bool first = true;
  for (SubTile c = next_subtile(a, j0, r_begin, r_end); c.j >= 0;
       c = next_subtile(a, c.j + 1, r_begin, r_end)) {
    const int64_t end = c.end;
    int64_t my = c.lo + SR * wave;   // this wave's first sub-tile
    auto rows_at = [&](int64_t lo) { return (int)(end - lo < SR ? end - lo : SR); };
    if (my < end) load_a(my, rows_at(my), A0);
    // the previous node's LDS reads are done before its tile is replaced
    // (an LDS-only barrier: the A loads just issued stay in flight)
    if (!first) lds_barrier();
    first = false;
    fill_w(c.j);
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      mn[f] = __builtin_huge_valf();
      mx[f] = -__builtin_huge_valf();
    }
    lds_barrier();
    // the first tile's loads have landed before the loop is entered, so the
    // waits inside it count only what the loop itself issues (vmcnt(0))
    __builtin_amdgcn_s_waitcnt(0x0F70);
    // ping-pong over this wave's sub-tiles of the node, SW SR rows apart
    while (my < end) {
      const int64_t nx = my + SW * SR;
      if (nx < end) load_a(nx, rows_at(nx), A1);
      // the next sub-tile's loads stay ahead of this one's matrix-core chain
      // (left to itself the scheduler sinks them next to their use)
      __builtin_amdgcn_sched_barrier(0);
      subtile(my, rows_at(my), A0);
      if (nx >= end) break;
      const int64_t nx2 = nx + SW * SR;
      if (nx2 < end) load_a(nx2, rows_at(nx2), A0);
      __builtin_amdgcn_sched_barrier(0);
      subtile(nx, rows_at(nx), A1);
      my = nx2;
    }
    flush(c.j);
  }
}

// want_xcd: 1 = keep a row run's particle tiles on one XCD when the grid
// allows (the rule), 0 = plain order (an autotuned alternative)
template <int MK, int FN, bool VEC>
slm_status launch_stream_f(const ProjectArgs &a, hipStream_t s, int want_xcd = 1) {
  constexpr int PT = 32 * FN;
  const int n_pt = (a.P + PT - 1) / PT;
  const int cus = num_cus_proj();
  // one work-group per CU (LDS and registers allow one): the particle tiles
  // share the CUs, each tile's rows split into runs of whole sub-tiles
  int64_t bpp = std::max<int64_t>(1, std::min<int64_t>((a.N + SR - 1) / SR, cus / n_pt));
  int xcd = 0;
  if (want_xcd && bpp >= 8 && n_pt * bpp >= 64) {
    bpp = bpp / 8 * 8;
    xcd = 1;
  }
  int64_t RB = ((a.N + bpp - 1) / bpp + SR - 1) / SR * SR;
  if (!a.vpre && !xcd) bpp = (a.N + RB - 1) / RB;
  const int64_t grid = bpp * n_pt;
  if (grid == 0) return SLM_OK;
  SLM_CHECK(grid < (1ll << 31), SLM_E_SHAPE, "slm_project: grid too large");
  const size_t lds = stream_lds_bytes(MK, FN) + (a.zl.eb == 2 ? stream_stage_bytes(FN) : 0);
  const int zt = z_tile_width(a.zl);
  if (a.zl.eb == 2)
    hipLaunchKernelGGL((k_project_stream<MK, FN, VEC, 8, true>), dim3((unsigned)grid), dim3(64 * SW),
                       lds, s, a, RB, (int)bpp, n_pt, xcd);
  else if (zt == 32)
    hipLaunchKernelGGL((k_project_stream<MK, FN, VEC, 32>), dim3((unsigned)grid), dim3(64 * SW),
                       lds, s, a, RB, (int)bpp, n_pt, xcd);
  else if (zt == 8)
    hipLaunchKernelGGL((k_project_stream<MK, FN, VEC, 8>), dim3((unsigned)grid), dim3(64 * SW),
                       lds, s, a, RB, (int)bpp, n_pt, xcd);
  else
    hipLaunchKernelGGL((k_project_stream<MK, FN, VEC, 0>), dim3((unsigned)grid), dim3(64 * SW),
                       lds, s, a, RB, (int)bpp, n_pt, xcd);
  SLM_LAUNCHED();
  return SLM_OK;
}

constexpr size_t STREAM_LDS_MAX = 159 * 1024;

// Shape class of a projection launch in the plan cache: the kernel (the
// streaming kernel's operand kind 0..2, or 3 for the short kernel), D, P and
// the data rows.
std::string proj_key(int kind, const ProjectArgs &a) {
  char buf[160];
  const int64_t n = a.vpre && a.rows > 0 ? a.rows : a.N;
  snprintf(buf, sizeof buf, "proj/%s/k%d/D%d/P%d/N%lld", device_arch().c_str(), kind, a.D, a.P,
           (long long)n);
  return buf;
}

// the autotuner's candidate in flight: (variant, option)
thread_local const int64_t *g_forced_proj = nullptr;

bool stream_fn_fits(int MK, int FN, const ProjectArgs &a) {
  const size_t stage = a.zl.eb == 2 ? stream_stage_bytes(FN) : 0;
  return (FN == 1 || (a.P + 31) / 32 >= FN) &&
         stream_lds_bytes(MK, FN) + stage <= STREAM_LDS_MAX;
}

// Particle blocks per wave FN (the widest that fits: 8 for bfloat16 data
// and directions, else 4, 2 or 1; or the cached / forced plan's) and the
// work-group order.
template <int MK>
slm_status launch_stream(const ProjectArgs &a, hipStream_t s) {
  const size_t xe = MK == MK_FF ? 4 : 2, we = MK == MK_BB ? 2 : 4;
  // 16-byte groups need rows that are whole groups in both matrices
  const bool vec = (a.D * xe) % 16 == 0 && (a.D * we) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(a.X) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(a.W) % 16 == 0;
  int fn = stream_fn_fits(MK, 4, a) ? 4 : stream_fn_fits(MK, 2, a) ? 2 : 1;
  // 256 particles per work-group (bfloat16 data and directions): half the
  // X reads per matrix-core operation
  if (MK == MK_BB && stream_fn_fits(MK, 8, a)) fn = 8;
  int xcd = 1;
  int64_t v0 = 0, v1 = 0;
  if (g_forced_proj) {
    v0 = g_forced_proj[0];
    v1 = g_forced_proj[1];
  }
  if ((g_forced_proj || plan_lookup(proj_key(MK, a), &v0, &v1)) &&
      (v0 == 1 || v0 == 2 || v0 == 4 || (MK == MK_BB && v0 == 8)) &&
      stream_fn_fits(MK, (int)v0, a)) {
    fn = (int)v0;
    xcd = v1 != 0;
  }
  if constexpr (MK == MK_BB)
    if (fn == 8)
      return vec ? launch_stream_f<MK, 8, true>(a, s, xcd) : launch_stream_f<MK, 8, false>(a, s, xcd);
  if (fn == 4)
    return vec ? launch_stream_f<MK, 4, true>(a, s, xcd) : launch_stream_f<MK, 4, false>(a, s, xcd);
  if (fn == 2)
    return vec ? launch_stream_f<MK, 2, true>(a, s, xcd) : launch_stream_f<MK, 2, false>(a, s, xcd);
  return vec ? launch_stream_f<MK, 1, true>(a, s, xcd) : launch_stream_f<MK, 1, false>(a, s, xcd);
}

// The streaming kernel serves every launch of a given (D, data types) or
// none, so a column recomputed alone always runs the kernel the swarm ran.
bool stream_eligible(const ProjectArgs &a) {
  if (a.Z == nullptr) return false;
  const int mk = a.x_bf16 && a.w_bf16 ? MK_BB : a.x_bf16 ? MK_XB : MK_FF;
  if (mk == MK_FF && a.D <= 64) return false;      // k_project_short
  if (a.w_bf16 && !a.x_bf16) return false;
  return a.D <= stream_kch(mk);
}

template <int MK, int FN, bool VEC, int ZT, bool ZB = false>
void set_stream_attr(int bytes) {
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_project_stream<MK, FN, VEC, ZT, ZB>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess)
    (void)hipGetLastError();
}
template <int MK, int FN>
void set_stream_attr_fn(int bytes) {
  set_stream_attr<MK, FN, true, 32>(bytes);
  set_stream_attr<MK, FN, true, 8>(bytes);
  set_stream_attr<MK, FN, true, 8, true>(bytes);
  set_stream_attr<MK, FN, true, 0>(bytes);
  set_stream_attr<MK, FN, false, 32>(bytes);
  set_stream_attr<MK, FN, false, 8>(bytes);
  set_stream_attr<MK, FN, false, 8, true>(bytes);
  set_stream_attr<MK, FN, false, 0>(bytes);
}
template <int MK>
void set_stream_attr_mk(int bytes) {
  set_stream_attr_fn<MK, 1>(bytes);
  set_stream_attr_fn<MK, 2>(bytes);
  set_stream_attr_fn<MK, 4>(bytes);
  if constexpr (MK == MK_BB) set_stream_attr_fn<MK, 8>(bytes);
}

// SLM_PROJ_STREAM=0 keeps the tile kernels for every shape (timing
// comparisons; read once per process)
bool stream_enabled() {
  static const int on = [] {
    const char *e = getenv("SLM_PROJ_STREAM");
    return e && e[0] == '0' ? 0 : 1;
  }();
  return on != 0;
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
  if (a.x_bf16)
    hipLaunchKernelGGL((k_project<BM, BN, WM, WN, true, false>), dim3((unsigned)grid), dim3(256), 0,
                       s, a);
  else
    hipLaunchKernelGGL((k_project<BM, BN, WM, WN, false, false>), dim3((unsigned)grid), dim3(256),
                       0, s, a);
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

void prepare_project_kernels(int lds_max) {
  const int dyn = (int)std::min<size_t>((size_t)lds_max, STREAM_LDS_MAX);
  set_stream_attr_mk<MK_BB>(dyn);
  set_stream_attr_mk<MK_XB>(dyn);
  set_stream_attr_mk<MK_FF>(dyn);
}

bool project_writes_bf16(const ProjectArgs &a) {
  return a.Z != nullptr && stream_enabled() && stream_eligible(a);
}

slm_status launch_project(const ProjectArgs &a, hipStream_t s) {
  SLM_CHECK(a.Z != nullptr || (a.D <= 64 && !a.x_bf16 && !a.w_bf16 && a.zmin), SLM_E_INVALID,
            "slm_project: a min/max-only pass needs float32 data, D <= 64 and zmin/zmax");
  SLM_CHECK(a.zl.eb == 4 || project_writes_bf16(a), SLM_E_UNSUPPORTED,
            "slm_project: bfloat16 Z is written by the streaming kernel only (D = %d, X %s, W %s)",
            a.D, a.x_bf16 ? "BF16" : "F32", a.w_bf16 ? "BF16" : "F32");
  if (stream_enabled() && stream_eligible(a)) {
    if (a.x_bf16 && a.w_bf16) return launch_stream<MK_BB>(a, s);
    if (a.x_bf16) return launch_stream<MK_XB>(a, s);
    return launch_stream<MK_FF>(a, s);
  }
  // both bfloat16: bfloat16 matrix cores
  if (a.x_bf16 && a.w_bf16) {
    if (a.P > 64) return launch_bf16<128, 128>(a, s);
    return launch_bf16<128, 64>(a, s);
  }
  // D <= 64: register-resident directions, 256 / 128 / 32 particles per
  // work-group (or the cached / forced plan's choice).
  if (a.D <= 64) {
    int variant = a.P > 128 ? 0 : a.P > 32 ? 1 : 2;
    int64_t v0 = 0, v1 = 0;
    if (g_forced_proj) v0 = g_forced_proj[0];
    if ((g_forced_proj || plan_lookup(proj_key(3, a), &v0, &v1)) && v0 >= 0 && v0 <= 2)
      variant = (int)v0;
    if (variant == 0) return launch_short<2, 4>(a, s);
    if (variant == 1) return launch_short<2, 2>(a, s);
    return launch_short<1, 1>(a, s);
  }
  // Tile shape by particle count: wide tiles for large swarms, a single
  // 32-particle column block for small ones (and for P = 1 recomputation).
  if (a.P >= 128) return launch_cfg<128, 128, 2, 2>(a, s);
  if (a.P > 32) return launch_cfg<128, 64, 2, 2>(a, s);
  return launch_cfg<128, 32, 4, 1>(a, s);
}

slm_status tune_project(const ProjectArgs &a, hipStream_t s) {
  if (a.Z == nullptr || a.N <= 0 || a.n_nodes <= 0) return SLM_OK;
  const bool stream = stream_enabled() && stream_eligible(a);
  int kind = -1;
  if (stream) kind = a.x_bf16 && a.w_bf16 ? MK_BB : a.x_bf16 ? MK_XB : MK_FF;
  else if (a.D <= 64 && !a.x_bf16 && !a.w_bf16) kind = 3;
  if (kind < 0) return SLM_OK;
  const std::string key = proj_key(kind, a);
  if (plan_known(key)) return SLM_OK;
  std::vector<std::pair<int64_t, int64_t>> cand;
  if (kind == 3) {
    for (int v = 0; v <= 2; ++v) cand.push_back({v, 0});
  } else {
    for (int fn : {8, 4, 2, 1})
      if ((fn < 8 || kind == MK_BB) && stream_fn_fits(kind, fn, a))
        for (int x : {1, 0}) cand.push_back({fn, x});
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SLM_HIP(hipEventCreate(&e0));
  SLM_HIP(hipEventCreate(&e1));
  float best_ms = 0.f;
  std::pair<int64_t, int64_t> best = cand[0];
  slm_status st = SLM_OK;
  for (size_t c = 0; c < cand.size() && !st; ++c) {
    const int64_t v[2] = {cand[c].first, cand[c].second};
    g_forced_proj = v;
    st = launch_project(a, s);                   // warm-up
    // the faster of two runs of four launches
    float ms = 0.f;
    for (int trial = 0; trial < 2 && !st; ++trial) {
      if (hipEventRecord(e0, s) != hipSuccess) st = SLM_E_HIP;
      for (int r = 0; r < 4 && !st; ++r) st = launch_project(a, s);
      float t = 0.f;
      if (!st && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        st = SLM_E_HIP;
      if (!st) ms = trial == 0 ? t : std::min(ms, t);
    }
    g_forced_proj = nullptr;
    if (st) break;
    if (c == 0 || ms < best_ms) {
      best_ms = ms;
      best = cand[c];
    }
  }
  g_forced_proj = nullptr;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) {
    (void)hipGetLastError();
    set_error("slm autotune: projection candidate failed");
    return st;
  }
  plan_store(key, best.first, best.second);
  return SLM_OK;
}

}  // namespace slm
