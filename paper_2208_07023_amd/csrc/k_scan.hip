// Best threshold of every projected feature (Sec. II-A, Eqs. (3)-(4);
// Sec. III-B: a direction's loss is the loss of its best threshold).
//
// Histogram scan.  k_scan_hist: a work-group owns (item, particle tile): the
// rows of one node inside one global chunk of CH rows, and PT particles of
// that node.  Lanes map to (row, particle): lane = rsub * PT + pl, so a wave
// reads 64 / PT row segments of PT consecutive floats of Z (with the
// particle-tiled layout, consecutive rows of a tile are contiguous) and each
// lane bins its own particle's value.  Counts go to LDS histograms laid out
// [bin][class][PT], so lanes of one row touch PT consecutive words.
//   * A node inside one chunk is finished by the same work-group from the
//     LDS histogram (finish_scan below).
//   * A node spanning several chunks adds its histogram into a global
//     accumulator slot (the node's first chunk index identifies the slot);
//     k_scan_finish_bins (classification: one work-group per particle, one
//     thread per bin) or k_scan_finish (regression: groups of particles),
//     launched next on the same stream, finishes each such node and clears
//     the slot for the next call.
//
// Exact scan.  One work-group per (node, particle): bitonic sort of the
// node's (z, row) pairs in LDS (stable through the row tie-break), then a
// block scan of class counts (or FP64 sums of y, y^2) and the criterion at
// every boundary between distinct values.
#include "slm_internal.hpp"

#include <algorithm>
#include <type_traits>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

namespace slm {
namespace {

constexpr int WG = 256;

// a word of the LDS, addressed with a 32-bit LDS pointer
typedef __attribute__((address_space(3))) uint32_t lds_u32;

// ---------------------------------------------------------------- binning
struct BinRule {
  float zmin, delta, inv;
  int B;
  bool flat;   // delta == 0 (zmax == zmin or underflow): every edge equals zmin
  bool fast;   // the guess below is provably within one bin of the count
};

// The guess floor((z - zmin) * B / r) differs from the exact count by less
// than 1 + eps bins, with eps <= B u (6 + |zmin| / r) (u = 2^-24: rounding of
// z - zmin, j * delta, zmin + j * delta, delta and the product); for
// |zmin| <= 64 r and B <= 256 that is below 1.1e-3, so one step down or up
// against the exact edges always lands on the count.  Otherwise (a range
// tiny next to its offset) the exact edges are searched step by step.
__device__ __forceinline__ BinRule make_rule(float zmin, float zmax, int B) {
  BinRule r;
  const float range = __fsub_rn(zmax, zmin);
  r.zmin = zmin;
  r.delta = __fdiv_rn(range, (float)B);
  r.inv = (float)B / range;
  r.B = B;
  r.flat = !(r.delta > 0.0f);
  r.fast = !r.flat && range < __builtin_huge_valf() && fabsf(zmin) <= 64.0f * range;
  return r;
}

__device__ __forceinline__ float edge(const BinRule &r, int j) {
  return __fadd_rn(r.zmin, __fmul_rn((float)j, r.delta));
}

// bin(z) = #{ j in 1..B-1 : e_j <= z } (the edges are non-decreasing).
__device__ __forceinline__ int bin_of(const BinRule &r, float z) {
  int g = (int)((z - r.zmin) * r.inv);
  g = g < 0 ? 0 : (g > r.B - 1 ? r.B - 1 : g);
  if (r.fast) {
    g -= (g >= 1 && edge(r, g) > z) ? 1 : 0;
    g += (g + 1 <= r.B - 1 && edge(r, g + 1) <= z) ? 1 : 0;
    return g;
  }
  if (r.flat) return r.B - 1;
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

// n log2 n of an integer count without a library call (the finish evaluates
// it 2K + 2 times per candidate split, inside fully unrolled code where a
// call would spill the register-resident histogram).  With n = m 2^e,
// m in [1, 2), and c = 1 + j/128 the largest grid point <= m:
//   log2 n = e + log2 c + log1p(r) / ln 2,   r = (m - c) / c in [0, 2^-7),
// m - c is exact, 1/c and log2 c come from a 128-entry table (lg[j], rc[j])
// filled by the work-group with the device log2, and log1p(r) is its Taylor
// series to r^8 (truncation < 2^-63 / 9).  Relative error is a few ulp.
constexpr int LG_TBL = 128;
__device__ __forceinline__ double nlog2n_cnt(uint32_t n, const double *lg, const double *rc) {
  const double x = (double)n;
  int e;
  const double m = 2.0 * frexp(x, &e);            // x = m 2^(e - 1), m in [1, 2)
  const int j = (int)((m - 1.0) * 128.0) & (LG_TBL - 1);   // n = 0 gives m = 0: any j
  const double r = (m - (1.0 + (double)j * (1.0 / 128.0))) * rc[j];
  double q = -1.0 / 8.0;
  q = fma(q, r, 1.0 / 7.0);
  q = fma(q, r, -1.0 / 6.0);
  q = fma(q, r, 1.0 / 5.0);
  q = fma(q, r, -1.0 / 4.0);
  q = fma(q, r, 1.0 / 3.0);
  q = fma(q, r, -1.0 / 2.0);
  q = fma(q, r, 1.0);
  const double l2 = (double)(e - 1) + fma(q * r, 1.4426950408889634, lg[j]);
  return n ? x * l2 : 0.0;
}

__device__ __forceinline__ void fill_log_table(double *lg, double *rc, int tid) {
  if (tid < LG_TBL) {
    const double c = 1.0 + (double)tid * (1.0 / 128.0);
    lg[tid] = log2(c);
    rc[tid] = 1.0 / c;
  }
}

// ---------------------------------------------------------------- plan
struct Plan {
  int PT;       // particles per work-group
  int64_t CH;   // rows per global chunk (<= 65472: 16-bit LDS counters)
  int G;        // particle tiles sharing one 128-byte line of a Z row
  int KT;       // class register tile: K for K <= 4, else 8 or 16; 1 for regression
};

constexpr int64_t CH_MAX = 65472;

// Shortest chunk of a plan for N rows: about N / 256 (the accumulator holds
// one slot per possible first chunk), at most the counter limit CH_MAX, so
// above 256 CH_MAX rows the slots grow with N instead.
int64_t chunk_min(int64_t N) {
  int64_t c = std::max<int64_t>(1024, (N + 255) / 256);
  return std::min<int64_t>((c + 63) / 64 * 64, CH_MAX);
}

// Histogram layout.  LDS holds 16-bit counters packed in pairs in 32-bit
// words, so a work-group's counts must stay below 2^16 (chunks of at most
// CH_MAX rows).  The global accumulator of a multi-chunk node mirrors the LDS
// words with 64-bit words holding two 32-bit counters (the low half's count
// low), so one 64-bit atomic merges both halves of an LDS word.
//   classification: particles 2j and 2j + 1 of a (bin, class) share a word:
//                   count(b, k, q) in the (q & 1) half of word
//                   b SB + k PT / 2 + q / 2, SB = K PT / 2 + 1.  A lane
//                   holding particles of one parity adds a constant (1 or
//                   2^16) at an address that is one multiply-add of the bin.
//                   K PT / 2 is even, so the odd stride spreads random bins
//                   over all the banks.
//   regression:     bins b and b + 128 share a word: count(b, q) in the
//                   (b >> 7) half of word (b & 127) SB + q, SB = PT; sum y and
//                   sum y^2 at b * PT + q in two double arrays
struct HistLayout {
  int SB;            // words per bin row
  int nwords;        // packed count words (LDS u32, accumulator u64)
  size_t lds_cnt;    // packed count region in LDS, 16-byte aligned
  size_t glob_cnt;   // count region of an accumulator slot, 256-byte aligned
  size_t sums;       // regression sums (both arrays)
};

__host__ __device__ __forceinline__ HistLayout hist_layout(int PT, int B, int K, bool mse) {
  HistLayout h;
  h.SB = mse ? PT : K * (PT / 2) + 1;
  h.nwords = mse ? (B < 128 ? B : 128) * h.SB : B * h.SB;
  h.lds_cnt = ((size_t)h.nwords * 4 + 15) / 16 * 16;
  h.glob_cnt = ((size_t)h.nwords * 8 + 255) / 256 * 256;
  h.sums = mse ? (size_t)2 * B * PT * 8 : 0;
  return h;
}

// Word and half (0 low, 1 high) of count (bin b, class k, particle q of the
// tile) in the layout above.
__host__ __device__ __forceinline__ int cnt_word(bool mse, int b, int k, int q, int SB, int PT) {
  return mse ? (b & 127) * SB + q : b * SB + k * (PT >> 1) + (q >> 1);
}
__host__ __device__ __forceinline__ int cnt_half(bool mse, int b, int q) {
  return mse ? b >> 7 : q & 1;
}

// Work-groups are 512 threads; the finish gives thread t particle t % PT and
// bin segment t / PT, so there are 512 / PT segments of at most PT / 2 bins.
constexpr int HIST_WG = 512;

// Class counts rounded up to the register tile of the finish.
__host__ __device__ __forceinline__ int class_tile(int K, bool mse) {
  return mse ? 1 : (K <= 4 ? K : (K <= 8 ? 8 : 16));
}

// Finish scratch (aliases the histogram once it is in registers): segment
// totals [NSEG][KT][PT] u32 (regression: counts, then sum y and sum y^2 as
// [NSEG][PT] doubles) and segment bests [NSEG][PT] (double, then int).
__host__ __device__ __forceinline__ size_t finish_tot_bytes(int KT, bool mse) {
  return mse ? (size_t)HIST_WG * (4 + 16) : (size_t)HIST_WG * KT * 4;
}
__host__ __device__ __forceinline__ size_t finish_bytes(int KT, bool mse) {
  return (finish_tot_bytes(KT, mse) + 15) / 16 * 16 + (size_t)HIST_WG * 12;
}
// Offset of the n log2 n table: after the histogram or the finish scratch.
__host__ __device__ __forceinline__ size_t table_offset(int PT, int B, int K, bool mse) {
  const HistLayout h = hist_layout(PT, B, K, mse);
  const size_t a = h.lds_cnt + h.sums, f = finish_bytes(class_tile(K, mse), mse);
  return ((a > f ? a : f) + 15) / 16 * 16;
}

size_t lds_bytes(int PT, int B, int K, bool mse, bool table) {
  return table_offset(PT, B, K, mse) + (table ? (size_t)2 * LG_TBL * 8 : 0);
}
size_t slot_bytes(int PT, int B, int K, bool mse) {
  const HistLayout h = hist_layout(PT, B, K, mse);
  return (h.glob_cnt + h.sums + 255) / 256 * 256;
}
// Accumulator slots of one replica: one per possible first chunk of a
// multi-chunk node, sized for the largest footprint of any tile width.
size_t slot_set_bytes(int64_t N, int P, int B, int K, bool mse) {
  size_t worst = 0;
  for (int PT = 4; PT <= 32; PT <<= 1) {
    const int64_t n_pt = (P + PT - 1) / PT;
    worst = std::max(worst, (size_t)n_pt * slot_bytes(PT, B, K, mse));
  }
  const int64_t n_slots = (N - 1) / chunk_min(N) + 1;
  return (size_t)n_slots * worst;
}
// Replicas of every slot: the work-groups of a node can spread their atomic
// merges over R copies (chunk % R), which k_scan_finish adds up.  Measured on
// MI355X (plain-tree shapes, N = 1e5, P = 256), every extra replica costs the
// finish more than it saves the merges (root scan 72 / 80 / 97 us for R = 1 /
// 2 / 4), so one copy is used.
int slot_replicas(int64_t, int, int, int, bool) { return 1; }

// Largest particle tile whose histograms fit in 80 KB of LDS (two
// work-groups per CU) and whose finish registers (PT / 2 bins x KT classes)
// stay at 64 per thread.
int pick_pt(int P, int B, int K, int crit) {
  const bool mse = crit == SLM_MSE;
  const int KT = class_tile(K, mse);
  int PT = 32;
  while (PT > 4 && (lds_bytes(PT, B, mse ? 1 : K, mse, crit == SLM_ENTROPY) > 80 * 1024 ||
                    PT * (mse ? 5 : KT) > 128))
    PT >>= 1;
  while (PT > 4 && PT / 2 >= P) PT >>= 1;
  return PT;
}

int num_cus() {
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

// Plan: the largest particle tile that fits (a 32-particle Z row segment is
// one 128-byte line) and a chunk length that makes the number of work-groups
// a whole number of rounds over the CUs (two resident per CU).
// SLM_SCAN_PLAN="PT:CH" overrides it (tuning sweeps).
// A (PT, CH) pair any launch of the shape may use: a tile whose register
// finish and LDS histogram fit, a chunk within the 16-bit counters whose
// slots the workspace (counted for chunk_min(N)) covers.
bool plan_fits(int64_t N, int B, int K, int crit, int pt, int64_t ch) {
  const bool mse = crit == SLM_MSE;
  return (pt == 4 || pt == 8 || pt == 16 || pt == 32) &&
         pt * (mse ? 5 : class_tile(K, mse)) <= 128 &&
         lds_bytes(pt, B, mse ? 1 : K, mse, crit == SLM_ENTROPY) <= 160 * 1024 - 1024 &&
         ch >= chunk_min(N) && ch <= CH_MAX && ch % 64 == 0;
}

// Shape class of a scan launch in the plan cache: the plan's row count, the
// node count rounded up to a power of two, P, bins, classes and criterion.
std::string scan_key(int64_t N, int n_nodes, int P, int B, int K, int crit) {
  int nb = 1;
  while (nb < n_nodes) nb <<= 1;
  char buf[192];
  snprintf(buf, sizeof buf, "scan/%s/N%lld/n%d/P%d/B%d/K%d/c%d", device_arch().c_str(),
           (long long)N, nb, P, B, K, crit);
  return buf;
}

// the autotuner's candidate in flight (one thread tunes at a time per launch)
thread_local const Plan *g_forced_scan = nullptr;

Plan make_plan(int64_t N, int n_nodes, int P, int B, int K, int crit, bool cached = true) {
  const bool mse = crit == SLM_MSE;
  Plan pl{pick_pt(P, B, K, crit), chunk_min(N), 1, class_tile(K, mse)};
  if (g_forced_scan) {
    pl.PT = g_forced_scan->PT;
    pl.CH = g_forced_scan->CH;
    pl.G = std::max(1, 32 / pl.PT);
    return pl;
  }
  const char *env = getenv("SLM_SCAN_PLAN");
  int pt = 0;
  long long ch = 0;
  int64_t tpt = 0, tch = 0;
  if (env && sscanf(env, "%d:%lld", &pt, &ch) == 2 &&
      plan_fits(N, B, K, crit, pt, (ch + 63) / 64 * 64)) {
    pl.PT = pt;
    pl.CH = (ch + 63) / 64 * 64;
  } else if (cached && plan_lookup(scan_key(N, n_nodes, P, B, K, crit), &tpt, &tch) &&
             plan_fits(N, B, K, crit, (int)tpt, tch)) {
    // measured by the autotuner for this shape class
    pl.PT = (int)tpt;
    pl.CH = tch;
  } else {
    const int64_t n_pt = (P + pl.PT - 1) / pl.PT;
    const int64_t slots = 2 * (int64_t)num_cus();
    // Small problems (one round of work-groups even at 4096-row chunks) take
    // the longer chunks: fewer work-groups per node means fewer accumulator
    // merges and less finish work (measured: N = 1e5, P = 256 root 70 -> 64
    // us, 128 nodes of 781 rows 181 -> 156 us); large ones keep >= 2048.
    const int64_t cmin = std::max<int64_t>(chunk_min(N), N * n_pt <= slots * 4096 ? 4096 : 2048);
    int64_t CH = cmin;
    for (int64_t m = 1; m <= 64; ++m) {
      const int64_t c = (N * n_pt + slots * m - 1) / (slots * m);
      if (c < cmin) break;
      CH = c;
      if (num_items(n_nodes, N, c) * n_pt >= slots * m) break;
    }
    pl.CH = std::min<int64_t>(CH_MAX, (CH + 63) / 64 * 64);
    // Few large nodes in one round of work-groups: 8-particle tiles with
    // chunks long enough for about one work-group per CU.  The atomic merges
    // of multi-chunk nodes scale with (work-groups x tile words), so narrower
    // tiles over more rows merge less for the same parallelism (measured,
    // N = 1e5, P = 256 root: 52 -> 39-44 us; tiles of 4 lose to the extra
    // loads of narrow row segments).
    //
    // The chunk length is the one with the fewest rows on the busiest CU.
    // Items (chunk pieces of n_nodes equal nodes, a chunk cut by a node
    // boundary being two) go out in order, CUs / ceil(P / 8) per round of
    // work-groups: each round costs its longest item, and every extra round
    // a fixed 3072 rows (its start latency).  Chunks are whole multiples of
    // 1024 rows, so every wave's rows of a full chunk go through the
    // 16-row unrolled loop (12544-row chunks: 42.2 us, 13312: 35.5 us, both 8
    // items).  Measured on MI355X (N = 1e5,
    // P = 256, standalone scan), the time follows this cost: one node 35.6 us
    // at 8 items of 13312 rows against 46.9 us at 10 items of 10240 (a
    // second round of 10240 rows); four nodes of 25 000 rows 50.7 us at 16
    // items of 8192 against 68.1 us at one item per node (25 000 rows).
    if (N * n_pt <= slots * 4096 && N / std::max(1, n_nodes) >= 16384 && P >= 8) {
      const int64_t n_pt8 = (P + 7) / 8;
      const int64_t per = std::max<int64_t>(1, (int64_t)num_cus() / n_pt8);
      const int nn = std::max(1, n_nodes);
      // the last answer is kept: one search per shape, not per launch
      static thread_local int64_t memo[4] = {-1, -1, -1, -1};
      if (memo[0] == N && memo[1] == nn && memo[2] == per) {
        pl.PT = 8;
        pl.CH = memo[3];
        pl.G = std::max(1, 32 / pl.PT);
        return pl;
      }
      int64_t best = -1, best_cost = 0;
      for (int64_t c = std::max<int64_t>(4096, (chunk_min(N) + 1023) / 1024 * 1024); c <= CH_MAX;
           c += 1024) {
        int64_t cost = 0, rmax = 0, idx = 0;
        for (int j = 0; j < nn; ++j) {
          const int64_t b = N * j / nn, e = N * (j + 1) / nn;
          for (int64_t k = b / c; k * c < e; ++k) {
            rmax = std::max(rmax, std::min(e, (k + 1) * c) - std::max(b, k * c));
            if (++idx % per == 0) {
              cost += rmax;
              rmax = 0;
            }
          }
        }
        cost += rmax + 3072 * ((idx + per - 1) / per - 1);
        if (best < 0 || cost < best_cost) {
          best = c;
          best_cost = cost;
        }
      }
      memo[0] = N;
      memo[1] = nn;
      memo[2] = per;
      memo[3] = best;
      pl.PT = 8;
      pl.CH = best;
    }
  }
  pl.G = std::max(1, 32 / pl.PT);
  return pl;
}

// ---------------------------------------------------------------- finish
// Particles per work-group of k_scan_finish: 4 (2 with 16 class slots), so a
// large node's finish spreads over 8 (16) work-groups per 32-particle tile.
__host__ __device__ constexpr int fin_nq(int PT, int KT) {
  return PT < (KT <= 8 ? 4 : 2) ? PT : (KT <= 8 ? 4 : 2);
}

// Best split of NQ particles (q0 .. q0 + NQ - 1 of a PT-particle tile) of one
// node from its complete histogram, by NT threads.  Thread t takes particle
// q = t % NQ and the segment s = t / NQ of SEGB consecutive bins (NSEG =
// NT / NQ segments).  The segment's counts are loaded into registers (all
// loads in flight together: clamped addresses, out-of-range values discarded
// afterwards); pass 1 stores the segment's class totals in LDS; pass 2 forms
// the left counts at the segment start from the totals of the segments before
// it and evaluates every candidate split of the segment in bin order,
// keeping the first minimum; pass 3 takes the minimum over segments in
// segment order (ties keep the smaller split).
// Source: the work-group's packed 16-bit LDS histogram (GSRC = false) or a
// multi-chunk accumulator slot (GSRC = true: 64-bit words holding bins b and
// b + 128, zeroed here after reading).
template <int NT, int KT, bool MSE>
__host__ __device__ constexpr size_t finish_tot_bytes() {
  return MSE ? (size_t)NT * (4 + 16) : (size_t)NT * KT * 4;
}
template <int NT, int KT, bool MSE>
__host__ __device__ constexpr size_t finish_scratch_bytes() {
  return (finish_tot_bytes<NT, KT, MSE>() + 15) / 16 * 16 + (size_t)NT * 12;
}

struct FinishSrc {
  const void *cnt;               // u32 LDS words or u64 slot words
  const double *s1, *s2;         // regression sums [B][PT]
  unsigned long long *gzero;     // slot words to clear after reading (GSRC)
  double *gz1, *gz2;
  int R;                         // GSRC: replicas of the slot, rstride bytes apart
  size_t rstride;
};

// ntab / tn: when tn > 0, ntab[n] = nlog2n_cnt(n) for n < tn is filled here
// (entropy), and counts below tn are looked up instead of evaluated.
template <int NQ, int NT, int KT, bool MSE, bool GSRC>
__device__ __forceinline__ void finish_scan(const ScanArgs &a, const FinishSrc &src, int PT,
                                            int pt, int q0, int64_t np, unsigned char *fin,
                                            const double *lg, const double *rc, int tid,
                                            double *ntab = nullptr, int tn = 0) {
  constexpr int NSEG = NT / NQ;
  constexpr int SEGMAX = (256 + NSEG - 1) / NSEG;
  const int B = a.bins;
  const int K = MSE ? 1 : a.K;
  const int SB = hist_layout(PT, B, K, MSE).SB;
  const int P = a.P;
  const int SEGB = (B + NSEG - 1) / NSEG;
  const int seg = tid / NQ, q = tid % NQ, qt = q0 + q;   // qt: particle within the tile
  const int b_lo = seg * SEGB;
  const int nb = max(0, min(SEGB, B - b_lo));
  const bool qv = pt * PT + qt < P;
  const int64_t out = np + (int64_t)pt * PT + qt;

  uint32_t c[SEGMAX][KT];
  double s1[MSE ? SEGMAX : 1], s2[MSE ? SEGMAX : 1];
#pragma unroll
  for (int i = 0; i < SEGMAX; ++i) {
#pragma unroll
    for (int k = 0; k < KT; ++k) c[i][k] = 0u;
    if constexpr (MSE) s1[i] = s2[i] = 0.0;
  }
  for (int r = 0; r < (GSRC ? src.R : 1); ++r) {
    const unsigned char *rb = static_cast<const unsigned char *>(src.cnt) + (size_t)r * src.rstride;
    const double *r1 = reinterpret_cast<const double *>(
        reinterpret_cast<const unsigned char *>(src.s1) + (size_t)r * src.rstride);
    const double *r2 = reinterpret_cast<const double *>(
        reinterpret_cast<const unsigned char *>(src.s2) + (size_t)r * src.rstride);
#pragma unroll
    for (int i = 0; i < SEGMAX; ++i) {
      const int b = min(b_lo + i, B - 1);
      const int h = cnt_half(MSE, b, qt);
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        const int w = cnt_word(MSE, b, min(k, K - 1), qt, SB, PT);
        uint32_t x;
        if constexpr (GSRC)
          x = (uint32_t)(reinterpret_cast<const unsigned long long *>(rb)[w] >> (h << 5));
        else
          x = (reinterpret_cast<const uint32_t *>(rb)[w] >> (h << 4)) & 0xFFFFu;
        c[i][k] += (i < nb && k < K) ? x : 0u;
      }
      if constexpr (MSE) {
        const double x1 = r1[b * PT + qt], x2 = r2[b * PT + qt];
        s1[i] += i < nb ? x1 : 0.0;
        s2[i] += i < nb ? x2 : 0.0;
      }
    }
  }
  if constexpr (!GSRC) lds_barrier();   // the histogram region becomes finish scratch

  uint32_t *stot = reinterpret_cast<uint32_t *>(fin);                       // [NSEG][KT][NQ]
  double *stot1 = reinterpret_cast<double *>(fin + (size_t)NT * 4);        // regression
  double *stot2 = stot1 + NT;
  double *sbl = reinterpret_cast<double *>(fin + (finish_tot_bytes<NT, KT, MSE>() + 15) / 16 * 16);
  int *sbb = reinterpret_cast<int *>(sbl + NT);

  // pass 1: segment totals
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    uint32_t t = 0;
#pragma unroll
    for (int i = 0; i < SEGMAX; ++i) t += c[i][k];
    stot[(seg * KT + k) * NQ + q] = t;
  }
  if constexpr (MSE) {
    double t1 = 0.0, t2 = 0.0;
#pragma unroll
    for (int i = 0; i < SEGMAX; ++i) {
      t1 += s1[i];
      t2 += s2[i];
    }
    stot1[seg * NQ + q] = t1;
    stot2[seg * NQ + q] = t2;
  }
  for (int i = tid; i < tn; i += NT) ntab[i] = nlog2n_cnt((uint32_t)i, lg, rc);
  lds_barrier();
  if constexpr (GSRC) {
    // every thread's loads completed before the barrier: clear what was read
    for (int r = 0; r < src.R; ++r) {
      unsigned long long *zc = reinterpret_cast<unsigned long long *>(
          reinterpret_cast<unsigned char *>(src.gzero) + (size_t)r * src.rstride);
      double *z1 = reinterpret_cast<double *>(reinterpret_cast<unsigned char *>(src.gz1) +
                                              (size_t)r * src.rstride);
      double *z2 = reinterpret_cast<double *>(reinterpret_cast<unsigned char *>(src.gz2) +
                                              (size_t)r * src.rstride);
#pragma unroll
      for (int i = 0; i < SEGMAX; ++i) {
        if (i < nb) {
          const int b = b_lo + i;
          // classification: only this particle's 32-bit half (its pair
          // partner may be read by another work-group)
#pragma unroll
          for (int k = 0; k < KT; ++k)
            if (k < K) {
              const int w = cnt_word(MSE, b, k, qt, SB, PT);
              if constexpr (MSE) zc[w] = 0ull;
              else reinterpret_cast<uint32_t *>(zc + w)[qt & 1] = 0u;
            }
          if constexpr (MSE) {
            z1[b * PT + qt] = 0.0;
            z2[b * PT + qt] = 0.0;
          }
        }
      }
    }
  }

  // pass 2: left totals at the segment start, then the segment's candidates
  uint32_t left[KT], tot[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) left[k] = tot[k] = 0;
  double l1 = 0.0, l2 = 0.0, T1 = 0.0, T2 = 0.0;
#pragma unroll 16
  for (int s2i = 0; s2i < NSEG; ++s2i) {
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      const uint32_t x = stot[(s2i * KT + k) * NQ + q];
      tot[k] += x;
      left[k] += s2i < seg ? x : 0u;
    }
    if constexpr (MSE) {
      const double x1 = stot1[s2i * NQ + q], x2 = stot2[s2i * NQ + q];
      if (s2i < seg) {
        l1 += x1;
        l2 += x2;
      }
      T1 += x1;
      T2 += x2;
    }
  }
  int64_t n = 0;
#pragma unroll
  for (int k = 0; k < KT; ++k) n += tot[k];
  const double dn = (double)n;
  double best = __builtin_huge_val();
  int bestb = 0x7fffffff;
#pragma unroll
  for (int i = 0; i < SEGMAX; ++i) {
    const int b = b_lo + i;
    if (i < nb) {
      if (b >= 1) {                                  // split b: bins < b go left
        double loss = __builtin_huge_val();
        bool valid;
        if constexpr (MSE) {
          const uint32_t nL = left[0], nR = tot[0] - left[0];
          valid = nL != 0 && nR != 0;
          if (valid) {
            const double dL = (double)nL, dR = (double)nR;
            const double S1R = T1 - l1, S2R = T2 - l2;
            const double sseL = l2 - (l1 * l1) / dL;
            const double sseR = S2R - (S1R * S1R) / dR;
            loss = (sseL + sseR) / (dL + dR);
          }
        } else {
          int64_t nL = 0;
#pragma unroll
          for (int k = 0; k < KT; ++k) nL += left[k];
          const int64_t nR = n - nL;
          valid = nL != 0 && nR != 0;
          if (valid) {
            if (a.crit == SLM_GINI) {
              uint64_t AL = 0, AR = 0;
#pragma unroll
              for (int k = 0; k < KT; ++k) {
                const uint64_t l = left[k], r = tot[k] - left[k];
                AL += l * l;
                AR += r * r;
              }
              const double sv = (double)AL / (double)nL + (double)AR / (double)nR;
              loss = (dn - sv) / dn;
            } else {
              auto nl = [&](uint32_t v) {
                return v < (uint32_t)tn ? ntab[v] : nlog2n_cnt(v, lg, rc);
              };
              double sL = 0.0, sR = 0.0;
#pragma unroll
              for (int k = 0; k < KT; ++k)
                if (k < K) {
                  sL += nl(left[k]);
                  sR += nl(tot[k] - left[k]);
                }
              const double TL = nl((uint32_t)nL) - sL;
              const double TR = nl((uint32_t)nR) - sR;
              loss = (TL + TR) / dn;
            }
          }
        }
        if (valid && loss < best) {
          best = loss;
          bestb = b;
        }
      }
#pragma unroll
      for (int k = 0; k < KT; ++k) left[k] += c[i][k];
      if constexpr (MSE) {
        l1 += s1[i];
        l2 += s2[i];
      }
    }
  }
  sbl[seg * NQ + q] = best;
  sbb[seg * NQ + q] = bestb;

  // optional raw histogram / sums output
  if (qv && a.hist_out) {
#pragma unroll
    for (int i = 0; i < SEGMAX; ++i)
      if (i < nb)
#pragma unroll
        for (int k = 0; k < KT; ++k)
          if (k < K) a.hist_out[(out * B + b_lo + i) * K + k] = c[i][k];
  }
  if constexpr (MSE) {
    if (qv && a.sums_out) {
#pragma unroll
      for (int i = 0; i < SEGMAX; ++i)
        if (i < nb) {
          a.sums_out[(out * B + b_lo + i) * 2] = s1[i];
          a.sums_out[(out * B + b_lo + i) * 2 + 1] = s2[i];
        }
    }
  }
  lds_barrier();

  // pass 3: minimum over segments in bin order
  if (tid < NQ && pt * PT + q0 + tid < P) {
    double bl = __builtin_huge_val();
    int bb = 0x7fffffff;
#pragma unroll 16
    for (int s2i = 0; s2i < NSEG; ++s2i) {
      const double l = sbl[s2i * NQ + tid];
      if (l < bl) {
        bl = l;
        bb = sbb[s2i * NQ + tid];
      }
    }
    const int64_t o = np + (int64_t)pt * PT + q0 + tid;
    if (bb == 0x7fffffff) {
      a.best_split[o] = -1;
      a.best_loss[o] = __builtin_huge_val();
      a.threshold[o] = __builtin_huge_valf();
    } else {
      const BinRule rr = make_rule(a.zmin[o], a.zmax[o], B);
      a.best_split[o] = bb;
      a.best_loss[o] = bl;
      a.threshold[o] = edge(rr, bb);
    }
  }
}

// ---------------------------------------------------------------- histogram kernel
// Two 512-thread work-groups per CU: at most 128 VGPRs per thread.
// Row coordinates of the histogram's work items and slots: data rows, or
// (a.vpre) the rows of the nodes alone, node j holding vpre[j] .. vpre[j+1]-1.
struct Coords {
  const int64_t *beg, *end;
  int64_t N;
};
__device__ __forceinline__ Coords coords_of(const ScanArgs &a) {
  if (a.vpre) return {a.vpre, a.vpre + 1, a.vpre[a.n_nodes]};
  return {a.beg, a.end, a.N};
}

// One particle per lane (pl = lane % PT, rows rsub, rsub + 64/PT, ... of the
// wave's steps): regression, row-major Z, and every tile width.
// Straight-line code for the common case: every lane's particle exists and
// its edges are well conditioned (the guess is within one bin), so the bin is
// computed without branches; 16 rows are in flight per lane.  Classification
// adds the lane's constant (1 or 2^16 by the particle's parity) to the word
// of hist_layout; regression adds 1 << 16 (b >> 7) to word (b & 127).  A lane
// without a particle, or a row whose label is out of range, adds 0.
template <int PT, int WGS, bool MSE>
__device__ __forceinline__ void accumulate_rows1(const ScanArgs &a, const Item &it, int p, bool pv,
                                                 int pl, int rsub, int wave, const BinRule &rule,
                                                 uint32_t *hc, double *hs1, double *hs2, int SB,
                                                 int SD) {
  constexpr int RPW = 64 / PT;                 // rows per wave step
  const int B = a.bins;
  const int K = MSE ? 1 : a.K;
  const int P = a.P;
  const int pt = (p - pl) / PT;
  const int64_t step = (int64_t)(WGS / 64) * RPW;
  const int64_t row0 = it.lo + wave * RPW + rsub;
  const int pcl = pv ? p : P - 1;                        // always a valid column
  const float *zp = a.Z + z_col(a.zl, pcl) + row0 * a.zl.rs;
  const int64_t zstep = step * a.zl.rs;
  const bool wave_fast = __all(rule.fast || !pv);
  uint32_t *hrow = hc + pl;
  auto add_cls = [&](int bn, int lab) {
    const bool ok = pv && (unsigned)lab < (unsigned)K;
    const uint32_t inc = ok ? (1u << ((pl & 1) << 4)) : 0u;
    const int lb = ok ? lab : 0;
    atomicAdd(&hc[cnt_word(false, bn, lb, pl, SB, PT)], inc);
  };
  auto add_mse = [&](int bn, double yv) {
    if (!pv) return;
    atomicAdd(&hrow[(bn & 127) * SB], 1u << ((bn >> 7) << 4));
    unsafeAtomicAdd(&hs1[bn * SD + pl], yv);
    unsafeAtomicAdd(&hs2[bn * SD + pl], yv * yv);
  };
  const int nrows = (int)((it.hi - row0 + step - 1) / step);   // rows of this lane (may be <= 0)
  constexpr int U = 16;
  int i = 0;
  if (wave_fast) {
    // Binning without branches.  The guess t = z B / r - (zmin B / r + 0.005)
    // (one fused multiply-add) is within B u (6 + 3 |zmin| / r) <= 3.1e-3
    // bins of the count of edges <= z when |zmin| <= 64 r and B <= 256 (the
    // rounding of the edges, of B / r, of the constant and of the result), so
    // g = trunc(t) is the bin or the one below it, never negative: one
    // comparison with the exact edge e_{g+1} settles it.  The unsigned clamp
    // keeps any input in range.  Classification adds the lane's parity
    // constant at b SB + class PT / 2 + pl / 2; a lane without a particle, or
    // a label outside [0, K), adds 0.
    const float zmin = rule.zmin, delta = rule.delta, inv = rule.inv;
    const float off0 = -fmaf(zmin, inv, 0.005f);
    const unsigned bmax = (unsigned)B - 1u;
    const unsigned labk = pv ? (unsigned)K : 0u;
    const uint32_t ph4 = PT * 2u, sb4 = (uint32_t)SB * 4u, pl4 = (uint32_t)(pl >> 1) * 4u;
    const uint32_t pinc = 1u << ((pl & 1) << 4);
    unsigned char *hb = reinterpret_cast<unsigned char *>(hc);
    auto bin_fast = [&](float zu) -> unsigned {
      const int g0 = (int)fmaf(zu, inv, off0);
      const float e1 = __fadd_rn(zmin, __fmul_rn((float)(g0 + 1), delta));
      return min((unsigned)(g0 + (e1 <= zu ? 1 : 0)), bmax);
    };
    // Z and labels through buffer loads: each lane's offset is fixed and the
    // offset of step (i + u) is a uniform scalar, so the loads need no
    // vector address arithmetic.  Ranges: rows below it.hi, at most CH_MAX
    // rows of at most 4096 floats from the base (< 2^31 bytes).
    const int64_t rbase = it.lo + (int64_t)wave * RPW;     // this wave's first row
    const int rs = (int)a.zl.rs;
    // base: the Z tile holding the work-group's first particle (tiles of 8
    // put a work-group's particles into up to 4 tiles, at lane offsets)
    const int t0p = (pt * PT) & ~((1 << a.zl.sh) - 1);
    const int64_t c0 = z_col(a.zl, t0p);
    const int plast = min(pt * PT + PT, P) - 1;
    const int64_t zspan = (z_col(a.zl, plast) - c0 + 1 + (it.hi - rbase) * rs) * 4;
    const __amdgpu_buffer_rsrc_t zr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float *>(a.Z + c0 + rbase * rs), 0,
        (int)(zspan < 0x7FFFFFFF ? zspan : 0x7FFFFFFF), BUF_DW3);
    const int zvo = (int)((z_col(a.zl, pcl) - c0 + rsub * rs) * 4), zso = (int)(step * rs * 4);
    const __amdgpu_buffer_rsrc_t lr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int32_t *>(a.labels ? a.labels + rbase : nullptr), 0,
        MSE ? 0 : (int)((it.hi - rbase) * 4), BUF_DW3);
    const int lvo = rsub * 4, lso = (int)(step * 4);
    for (; i + U <= nrows; i += U) {
      float z[U];
      int lab[U];
      double yv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        z[u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(zr, zvo, (i + u) * zso, 0));
        if constexpr (MSE) yv[u] = a.y[row0 + (int64_t)(i + u) * step];
        else lab[u] = (int)__builtin_amdgcn_raw_buffer_load_b32(lr, lvo, (i + u) * lso, 0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const unsigned g = bin_fast(z[u]);
        if constexpr (MSE) {
          add_mse((int)g, yv[u]);
        } else {
          const unsigned lb = min((unsigned)lab[u], (unsigned)K - 1u);
          const uint32_t inc = (unsigned)lab[u] < labk ? pinc : 0u;
          const uint32_t off = __umul24(g, sb4) + lb * ph4 + pl4;
          atomicAdd(reinterpret_cast<uint32_t *>(hb + off), inc);
        }
      }
    }
  }
  for (; i < nrows; ++i) {
    const float z = zp[(int64_t)i * zstep];
    const int bn = bin_of(rule, z);
    if constexpr (MSE) add_mse(bn, a.y[row0 + (int64_t)i * step]);
    else add_cls(bn, a.labels[row0 + (int64_t)i * step]);
  }
}

// Four consecutive particles per lane (classification, particle-tiled Z with
// tiles of 8 or 32): lane (q, r) takes particles 4q .. 4q+3 of the tile and
// rows r, r + 64/(PT/4), ... of the wave's steps.  Per row: one 16-byte
// buffer load of the four projections, one label load, and the label's part
// of the LDS address; per sample-split: the branch-free bin and one LDS
// atomic, whose address is one multiply-add.
//
// In the classification layout of hist_layout a lane's particles 4q, 4q+1
// share word 2q of a (bin, class) and 4q+2, 4q+3 word 2q+1, so the increment
// of particle e is 1 or 2^16 by the parity of e alone.
//
// Fast path (every particle of the tile exists and every edge rule is well
// conditioned): the guess is taken one bin up, g1 = trunc(z B / r -
// (zmin B / r + 0.005) + 1) in one fused multiply-add with the constant
// rounded once, and the bin is g1 - 1 + [e_{g1} <= z], clamped to B - 1.
// Against the guess of accumulate_rows1 the constant's rounding and the
// larger result add at most B u (1 + |zmin| / r) + u bins, so the guess stays
// within B u (7 + 4 |zmin| / r) <= 4.0e-3 < 0.005 bins of the count of edges
// <= z (u = 2^-24, |zmin| <= 64 r, B <= 256): g1 - 1 is the bin or the one
// below, g1 >= 0, and e_0 = zmin <= z keeps g1 = 0 at bin 0.  The test is
// written !(e_{g1} > z), so a NaN projection lands in bin 0 as in bin_of;
// the clamp keeps every address inside the histogram whatever zmin / zmax
// the caller passed.  Rows are taken U4 at a time: loads, then every bin,
// then the addresses and atomics.  When every label of the wave's U4 rows is
// a class (the usual case, one vote per step) the increments are constants;
// otherwise a label outside [0, K) keeps its row's address in range and
// adds 0.  ZCP: the cache policy of the Z loads (0, or Z_CPOL_NT for a Z
// larger than the MALL).
template <int PT, int WGS, bool ZB, int ZCP>
__device__ __forceinline__ void accumulate_rows4(const ScanArgs &a, const Item &it, int pt,
                                                 int64_t np, int wave, int lane,
                                                 unsigned char *hb, int SB) {
  constexpr int QG = PT / 4, RPW4 = 64 / QG;   // lanes per row, rows per wave step
  static_assert(PT % 4 == 0 && QG >= 1, "four particles per lane");
  const int B = a.bins, K = a.K, P = a.P;
  const int q4 = lane % QG, r4 = lane / QG;
  const int64_t step4 = (int64_t)(WGS / 64) * RPW4;
  const int64_t rb4 = it.lo + (int64_t)wave * RPW4;   // the wave's first row
  const int64_t row4 = rb4 + r4;
  const int n4 = (int)((it.hi - row4 + step4 - 1) / step4);   // rows of this lane (may be <= 0)
  BinRule rl[4];
  float zm[4], dl[4], iv[4], o1[4];
  bool pv4[4];
  bool lane_fast = true;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int pe = pt * PT + 4 * q4 + e;
    pv4[e] = pe < P;
    rl[e] = make_rule(pv4[e] ? a.zmin[np + pe] : 0.f, pv4[e] ? a.zmax[np + pe] : 0.f, B);
    lane_fast = lane_fast && rl[e].fast;
    zm[e] = rl[e].zmin;
    dl[e] = rl[e].delta;
    iv[e] = rl[e].inv;
    o1[e] = __fadd_rn(-fmaf(zm[e], iv[e], 0.005f), 1.0f);
  }
  // uniform: the tile is full and every lane's rules are fast
  const bool wave_fast = __all(lane_fast) && (pt + 1) * PT <= P;
  const unsigned bmax = (unsigned)B - 1u;
  // bytes: per bin, per class, and the lane's first pair word
  const uint32_t sb4 = (uint32_t)SB * 4u, ph4 = (uint32_t)PT * 2u, q8 = 8u * (uint32_t)q4;
  // Z from the tile holding the work-group's first particle, at the wave's
  // first row; each lane adds its four particles' tile and column offset (a
  // lane past P reads the last existing group of four, whose counts it never
  // adds).  Offsets stay below 2^31 bytes: the layout is checked on the host.
  // ZB: bfloat16 elements, four of them in one 8-byte load, widened exactly.
  constexpr int EB = ZB ? 2 : 4;
  const int rs = (int)a.zl.rs;
  const int t0p = (pt * PT) & ~((1 << a.zl.sh) - 1);
  const int64_t c0 = z_col(a.zl, t0p);
  const int pa = min(pt * PT + 4 * q4, (P - 1) & ~3);
  const int plast = min(pt * PT + PT, P) - 1;
  const int64_t zspan = (z_col(a.zl, plast) - c0 + 1 + (it.hi - rb4) * rs) * EB;
  const __amdgpu_buffer_rsrc_t zr = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<char *>(reinterpret_cast<const char *>(a.Z) + (c0 + rb4 * rs) * EB), 0,
      (int)(zspan < 0x7FFFFFFF ? zspan : 0x7FFFFFFF), BUF_DW3);
  const int zvo = (int)((z_col(a.zl, pa) - c0 + (int64_t)r4 * rs) * EB);
  const int zso = (int)(step4 * rs * EB);
  // Z of row step j as loaded (RW words: four bfloat16 in two, or four
  // float32), and its four projections as float32 bit patterns
  constexpr int RW = ZB ? 2 : 4;
  auto load_raw = [&](int j, uint32_t (&r)[RW]) {
    if constexpr (ZB) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(zr, zvo, j * zso, ZCP);
      r[0] = v[0];
      r[1] = v[1];
    } else {
      const auto v = __builtin_amdgcn_raw_buffer_load_b128(zr, zvo, j * zso, ZCP);
      r[0] = v[0];
      r[1] = v[1];
      r[2] = v[2];
      r[3] = v[3];
    }
  };
  auto widen = [&](const uint32_t (&r)[RW], uint32_t (&zw)[4]) {
    if constexpr (ZB) {
      zw[0] = r[0] << 16;
      zw[1] = r[0] & 0xFFFF0000u;
      zw[2] = r[1] << 16;
      zw[3] = r[1] & 0xFFFF0000u;
    } else {
      zw[0] = r[0];
      zw[1] = r[1];
      zw[2] = r[2];
      zw[3] = r[3];
    }
  };
  auto load_z = [&](int j, uint32_t (&zw)[4]) {
    uint32_t r[RW];
    load_raw(j, r);
    widen(r, zw);
  };
  const __amdgpu_buffer_rsrc_t lr = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<int32_t *>(a.labels + rb4), 0, (int)((it.hi - rb4) * 4), BUF_DW3);
  const int lvo = r4 * 4, lso = (int)(step4 * 4);
  // LDS byte address of the histogram (32-bit LDS pointers: the address of
  // a sample-split is one 24-bit multiply-add)
  const uint32_t hbase = (uint32_t)(uintptr_t)(lds_u32 *)hb + q8;
  constexpr int U4 = 4;
  // the loads of U4 row steps from step j
  auto issue = [&](int j, uint32_t (&r)[U4][RW], int (&lab)[U4]) {
#pragma unroll
    for (int u = 0; u < U4; ++u) {
      load_raw(j + u, r[u]);
      lab[u] = (int)__builtin_amdgcn_raw_buffer_load_b32(lr, lvo, (j + u) * lso, 0);
    }
  };
  // bins and LDS atomics of U4 loaded row steps
  auto process = [&](const uint32_t (&r)[U4][RW], const int (&lab)[U4]) {
    uint32_t g[U4][4];
    bool ok = true;
#pragma unroll
    for (int u = 0; u < U4; ++u) {
      ok = ok && (unsigned)lab[u] < (unsigned)K;
      uint32_t zw[4];
      widen(r[u], zw);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float z = __uint_as_float(zw[e]);
        const int g1 = (int)fmaf(z, iv[e], o1[e]);
        const float eg = __fadd_rn(zm[e], __fmul_rn((float)g1, dl[e]));
        g[u][e] = min((uint32_t)(g1 - 1 + (eg > z ? 0 : 1)), bmax);
      }
    }
    if (__all(ok)) {
      // every label of the wave's rows is a class: constant increments
#pragma unroll
      for (int u = 0; u < U4; ++u) {
        const uint32_t base = (uint32_t)lab[u] * ph4 + hbase;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          __hip_atomic_fetch_add((lds_u32 *)(uintptr_t)(__umul24(g[u][e], sb4) + base) + (e >> 1),
                                 (e & 1) ? 0x10000u : 1u, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    } else {
#pragma unroll
      for (int u = 0; u < U4; ++u) {
        const bool lok = (unsigned)lab[u] < (unsigned)K;
        const uint32_t base = (lok ? (uint32_t)lab[u] : 0u) * ph4 + hbase;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          __hip_atomic_fetch_add((lds_u32 *)(uintptr_t)(__umul24(g[u][e], sb4) + base) + (e >> 1),
                                 lok ? ((e & 1) ? 0x10000u : 1u) : 0u, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  };
  // Full groups of U4 row steps that every lane of the wave has: lanes hold
  // n4 or n4 - 1 steps, the last lane the fewest, so its count is the
  // wave's (a uniform trip count keeps the load offsets scalar).  A lane's
  // steps past them (at most U4) take the exact loop below.
  const int ngw = __builtin_amdgcn_readfirstlane(max(0, __shfl(n4, 63)) / U4);
  int i = 0;
  if (wave_fast && ngw > 0) {
    // two register sets: the next U4 row steps are loaded before the
    // current ones are binned.  Inside the loop every pass loads (so each
    // waits for the current group alone); the last one or two groups are
    // peeled off.
    uint32_t ra[U4][RW], rb[U4][RW];
    int la[U4], lb[U4];
    issue(0, ra, la);
    int t = 0;
    for (; t + 2 < ngw; t += 2) {
      issue((t + 1) * U4, rb, lb);
      __builtin_amdgcn_sched_barrier(0);
      process(ra, la);
      issue((t + 2) * U4, ra, la);
      __builtin_amdgcn_sched_barrier(0);
      process(rb, lb);
    }
    if (t + 1 < ngw) {
      issue((t + 1) * U4, rb, lb);
      __builtin_amdgcn_sched_barrier(0);
      process(ra, la);
      process(rb, lb);
    } else {
      process(ra, la);
    }
    i = ngw * U4;
  }
  // remaining rows (all rows when a rule is ill conditioned or the tile is
  // partial): the fast bin when the wave is on the fast path, else the exact
  // search; nothing added for particles past P
  for (; i < n4; ++i) {
    uint32_t v[4];
    load_z(i, v);
    const int lab = (int)__builtin_amdgcn_raw_buffer_load_b32(lr, lvo, i * lso, 0);
    const bool lok = (unsigned)lab < (unsigned)K;
    const uint32_t base = (uint32_t)(lok ? lab : 0) * ph4 + q8;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float z = __uint_as_float(v[e]);
      unsigned g;
      if (wave_fast) {
        const int g1 = (int)fmaf(z, iv[e], o1[e]);
        const float eg = __fadd_rn(zm[e], __fmul_rn((float)g1, dl[e]));
        g = min((uint32_t)(g1 - 1 + (eg > z ? 0 : 1)), bmax);
      } else {
        g = (unsigned)bin_of(rl[e], z);
      }
      const uint32_t inc = lok && pv4[e] ? ((e & 1) ? 0x10000u : 1u) : 0u;
      atomicAdd(reinterpret_cast<uint32_t *>(hb + g * sb4 + base + 4u * (e >> 1)), inc);
    }
  }
}

template <int PT, int KT, bool MSE>
__global__ __launch_bounds__(HIST_WG) __attribute__((amdgpu_waves_per_eu(4)))
void k_scan_hist(ScanArgs a, int64_t CH, int n_pt, int G, int64_t total_blocks, size_t slot_sz,
                 int64_t n_slots, int R) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int WGS = HIST_WG;
  const int B = a.bins;
  const int K = MSE ? 1 : a.K;
  const HistLayout hl = hist_layout(PT, B, K, MSE);
  const int SB = hl.SB, SD = PT;
  uint32_t *hc = reinterpret_cast<uint32_t *>(smem);
  double *hs1 = reinterpret_cast<double *>(smem + hl.lds_cnt);
  double *hs2 = hs1 + (size_t)B * SD;
  double *lg = reinterpret_cast<double *>(smem + table_offset(PT, B, K, MSE));
  double *rc = lg + LG_TBL;
  const bool use_tbl = !MSE && a.crit == SLM_ENTROPY;

  // XCD-aware order: the G particle tiles that share a Z cache line get
  // block ids congruent modulo 8, dispatched close together.
  const int64_t bid = blockIdx.x;
  const int64_t hi8 = bid / (8 * G), rem = bid % (8 * G);
  const int64_t L = ((hi8 * 8 + rem % 8) * G) + rem / 8;
  if (L >= total_blocks) return;
  const int64_t v = L / n_pt;
  const int pt = (int)(L % n_pt);
  const Coords co = coords_of(a);
  Item it = find_item(co.beg, co.end, a.n_nodes, co.N, CH, v);
  if (it.node < 0) return;
  if (a.vpre) {   // back to data rows
    const Range nr = load_range(a.beg, a.end, it.node, a.N);
    const int64_t off = nr.lo - co.beg[it.node];
    it.lo += off;
    it.hi += off;
    if (it.hi > nr.hi) it.hi = nr.hi;
    if (it.lo >= it.hi) return;   // cannot happen with vpre matching the ranges
  }

  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int i = tid; i < hl.nwords; i += WGS) hc[i] = 0u;
  if constexpr (MSE) {
    for (int i = tid; i < B * SD; i += WGS) {
      hs1[i] = 0.0;
      hs2[i] = 0.0;
    }
  }
  if (use_tbl) fill_log_table(lg, rc, tid);

  constexpr int RPW = 64 / PT;                 // rows per wave step
  const int pl = lane % PT, rsub = lane / PT;
  const int P = a.P;
  const int p = pt * PT + pl;
  const bool pv = p < P;
  const int64_t np = (int64_t)it.node * P;
  const BinRule rule = make_rule(pv ? a.zmin[np + p] : 0.f, pv ? a.zmax[np + p] : 0.f, B);
  lds_barrier();

  // ---- accumulate, classification with particle-tiled Z: every lane takes
  // four consecutive particles of one row, so one 16-byte load of the row's
  // Z segment and one label load serve four sample-splits, and the label's
  // part of the LDS address is formed once per row.
  unsigned char *const hb = reinterpret_cast<unsigned char *>(hc);
  const bool znt = z_streams(a.N, P, a.zl.eb);
  if (!MSE && a.zl.eb == 2) {
    if (znt)
      accumulate_rows4<PT, WGS, true, Z_CPOL_NT>(a, it, pt, np, wave, lane, hb, SB);
    else
      accumulate_rows4<PT, WGS, true, 0>(a, it, pt, np, wave, lane, hb, SB);
  } else if (!MSE && a.zl.rs == (1 << a.zl.sh) && a.zl.rs >= 8) {
    if (znt)
      accumulate_rows4<PT, WGS, false, Z_CPOL_NT>(a, it, pt, np, wave, lane, hb, SB);
    else
      accumulate_rows4<PT, WGS, false, 0>(a, it, pt, np, wave, lane, hb, SB);
  } else {
    accumulate_rows1<PT, WGS, MSE>(a, it, p, pv, pl, rsub, wave, rule, hc, hs1, hs2, SB, SD);
  }
  lds_barrier();

  // ---- a node spanning several chunks: add into its accumulator slot (the
  // node's first chunk index); k_scan_finish completes it
  if (it.nchunks > 1) {
    const Range nr = load_range(co.beg, co.end, it.node, co.N);
    const int64_t slot = nr.lo / CH;
    if (slot >= n_slots) return;   // cannot happen with a workspace sized by the plan
    // replica it.chunk % R of the slot: fewer atomics on each address
    unsigned char *base = static_cast<unsigned char *>(a.ws) +
                          ((size_t)(slot * R + it.chunk % R) * n_pt + pt) * slot_sz;
    unsigned long long *gc = reinterpret_cast<unsigned long long *>(base);
    for (int i = tid; i < hl.nwords; i += WGS) {
      const uint32_t w = hc[i];
      if (w)
        atomicAdd(&gc[i], (unsigned long long)(w & 0xFFFFu) | ((unsigned long long)(w >> 16) << 32));
    }
    if constexpr (MSE) {
      double *g1 = reinterpret_cast<double *>(base + hl.glob_cnt);
      double *g2 = g1 + (size_t)B * SD;
      for (int i = tid; i < B * SD; i += WGS) {
        if (hs1[i] != 0.0) unsafeAtomicAdd(&g1[i], hs1[i]);
        if (hs2[i] != 0.0) unsafeAtomicAdd(&g2[i], hs2[i]);
      }
    }
    return;
  }

  // ---- a node inside one chunk: finish from the LDS histogram
  // n log2 n table for the node's counts (at most its row count) in the LDS
  // between the finish scratch and the end of the histogram region
  const FinishSrc src{hc, hs1, hs2, nullptr, nullptr, nullptr, 1, 0};
  const size_t t0 = (finish_scratch_bytes<WGS, KT, MSE>() + 15) / 16 * 16;
  const size_t t1 = table_offset(PT, B, K, MSE);
  const int64_t tcap = t1 > t0 ? (int64_t)((t1 - t0) / 8) : 0;
  const int64_t rows1 = it.hi - it.lo + 1;
  const int tn = use_tbl ? (int)(rows1 < tcap ? rows1 : tcap) : 0;
  finish_scan<PT, WGS, KT, MSE, false>(a, src, PT, pt, 0, np, smem, lg, rc, tid,
                                       reinterpret_cast<double *>(smem + t0), tn);
}

// Completes the nodes that span several chunks, once every chunk's histogram
// is in the node's accumulator slot.  Work-group (slot s, particle tile,
// group of NQ particles); slots without such a node exit at once.
template <int PT, int KT, bool MSE>
__global__ __launch_bounds__(256) void k_scan_finish(ScanArgs a, int64_t CH, int n_pt,
                                                     size_t slot_sz, int64_t n_slots, int R) {
  constexpr int NQ = fin_nq(PT, KT);
  constexpr int NGRP = PT / NQ;
  __shared__ __align__(16) unsigned char fin[finish_scratch_bytes<256, KT, MSE>()];
  __shared__ double lgt[2 * LG_TBL];
  const int64_t bid = blockIdx.x;
  const int grp = (int)(bid % NGRP);
  const int pt = (int)((bid / NGRP) % n_pt);
  const int64_t slot = bid / ((int64_t)NGRP * n_pt);
  if (slot >= n_slots) return;
  // the node whose rows start in chunk `slot` and continue past it
  const int64_t lim = (slot + 1) * CH;
  if (a.n_nodes <= 0) return;
  const Coords co = coords_of(a);
  auto beg_of = [&](int j) {
    const int64_t x = co.beg[j];
    return x < 0 ? (int64_t)0 : (x > co.N ? co.N : x);
  };
  if (beg_of(0) >= lim) return;
  int lo = 0, hi = a.n_nodes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (beg_of(mid) < lim) lo = mid; else hi = mid - 1;
  }
  const Range r = load_range(co.beg, co.end, lo, co.N);
  if (r.hi <= r.lo || r.lo / CH != slot || (r.hi - 1) / CH == slot) return;
  const int B = a.bins;
  const int K = MSE ? 1 : a.K;
  const HistLayout hl = hist_layout(PT, B, K, MSE);
  unsigned char *base =
      static_cast<unsigned char *>(a.ws) + ((size_t)slot * R * n_pt + pt) * slot_sz;
  unsigned long long *gc = reinterpret_cast<unsigned long long *>(base);
  double *g1 = reinterpret_cast<double *>(base + hl.glob_cnt);
  double *g2 = g1 + (size_t)B * PT;
  const int tid = threadIdx.x;
  double *lg = lgt, *rc = lgt + LG_TBL;
  if (!MSE && a.crit == SLM_ENTROPY) fill_log_table(lg, rc, tid);
  lds_barrier();
  const FinishSrc src{gc, g1, g2, gc, g1, g2, R, (size_t)n_pt * slot_sz};
  finish_scan<NQ, 256, KT, MSE, true>(a, src, PT, pt, grp * NQ, (int64_t)lo * a.P, fin, lg, rc,
                                      tid);
}


// Classification nodes spanning several chunks, finished one bin per thread:
// work-group (slot s, particle tile, particle pair j) of 256 threads, thread
// b holding bin b of the node's accumulated histogram for particles 2j and
// 2j + 1 (the two halves of each 64-bit slot word, so every word is read
// once).  Class counts are summed over the bins by wave scans (then across
// the 4 waves); thread b evaluates, for each of the two particles, the split
// "bins < b go left" with the same arithmetic as finish_scan, and the
// work-group keeps each particle's smallest loss, ties to the smaller bin
// (the first minimum in bin order), so the outputs equal finish_scan's.  The
// slot words of the pair are cleared for the next call.
template <int KT>
__global__ __launch_bounds__(256) void k_scan_finish_bins(ScanArgs a, int PT, int64_t CH,
                                                          int n_pt, size_t slot_sz,
                                                          int64_t n_slots, int R) {
  __shared__ uint32_t wtot[2][4][KT];
  __shared__ double wbl[2][4];
  __shared__ int wbb[2][4];
  __shared__ double lgt[2 * LG_TBL];
  const int PH = PT / 2;
  const int64_t bid = blockIdx.x;
  const int jp = (int)(bid % PH);
  const int pt = (int)((bid / PH) % n_pt);
  const int64_t slot = bid / ((int64_t)PH * n_pt);
  if (slot >= n_slots || pt * PT + 2 * jp >= a.P) return;
  // the node whose rows start in chunk `slot` and continue past it
  const int64_t lim = (slot + 1) * CH;
  if (a.n_nodes <= 0) return;
  const Coords co = coords_of(a);
  auto beg_of = [&](int j) {
    const int64_t x = co.beg[j];
    return x < 0 ? (int64_t)0 : (x > co.N ? co.N : x);
  };
  if (beg_of(0) >= lim) return;
  int lo = 0, hi = a.n_nodes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (beg_of(mid) < lim) lo = mid; else hi = mid - 1;
  }
  const Range r = load_range(co.beg, co.end, lo, co.N);
  if (r.hi <= r.lo || r.lo / CH != slot || (r.hi - 1) / CH == slot) return;
  const int B = a.bins, K = a.K, SB = hist_layout(PT, B, K, false).SB;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const bool ent = a.crit == SLM_ENTROPY;
  if (ent) fill_log_table(lgt, lgt + LG_TBL, tid);
  unsigned char *base =
      static_cast<unsigned char *>(a.ws) + ((size_t)slot * R * n_pt + pt) * slot_sz;
  const int b = tid;
  const bool bv = b < B;
  const int w = cnt_word(false, b, 0, 2 * jp, SB, PT);
  uint32_t c[2][KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) c[0][k] = c[1][k] = 0u;
  for (int rr = 0; rr < R; ++rr) {
    const unsigned long long *gc =
        reinterpret_cast<const unsigned long long *>(base + (size_t)rr * n_pt * slot_sz);
#pragma unroll
    for (int k = 0; k < KT; ++k)
      if (bv && k < K) {
        const unsigned long long v = gc[w + k * PH];
        c[0][k] += (uint32_t)v;
        c[1][k] += (uint32_t)(v >> 32);
      }
  }
  // inclusive scans of the counts over the lanes of the wave
  uint32_t inc[2][KT];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int k = 0; k < KT; ++k) inc[h][k] = c[h][k];
#pragma unroll
  for (int d = 1; d < 64; d <<= 1)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        const uint32_t t = __shfl_up(inc[h][k], d);
        inc[h][k] += lane >= d ? t : 0u;
      }
  if (lane == 63)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < KT; ++k) wtot[h][wv][k] = inc[h][k];
  lds_barrier();   // also: every thread's slot reads are complete
  // this work-group alone reads the pair's words: clear them whole
  if (bv)
    for (int rr = 0; rr < R; ++rr) {
      unsigned long long *gz =
          reinterpret_cast<unsigned long long *>(base + (size_t)rr * n_pt * slot_sz);
#pragma unroll
      for (int k = 0; k < KT; ++k)
        if (k < K) gz[w + k * PH] = 0ull;
    }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    uint32_t left[KT], tot[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      uint32_t before = 0u, all = 0u;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const uint32_t t = wtot[h][v][k];
        all += t;
        before += v < wv ? t : 0u;
      }
      left[k] = before + inc[h][k] - c[h][k];   // bins < b
      tot[k] = all;
    }
    int64_t n = 0;
#pragma unroll
    for (int k = 0; k < KT; ++k) n += tot[k];
    const double dn = (double)n;
    double bl = __builtin_huge_val();
    int bb = 0x7fffffff;
    if (bv && b >= 1) {
      int64_t nL = 0;
#pragma unroll
      for (int k = 0; k < KT; ++k) nL += left[k];
      const int64_t nR = n - nL;
      if (nL != 0 && nR != 0) {
        double loss;
        if (!ent) {
          uint64_t AL = 0, AR = 0;
#pragma unroll
          for (int k = 0; k < KT; ++k) {
            const uint64_t l = left[k], rt = tot[k] - left[k];
            AL += l * l;
            AR += rt * rt;
          }
          const double sv = (double)AL / (double)nL + (double)AR / (double)nR;
          loss = (dn - sv) / dn;
        } else {
          double sL = 0.0, sR = 0.0;
#pragma unroll
          for (int k = 0; k < KT; ++k)
            if (k < K) {
              sL += nlog2n_cnt(left[k], lgt, lgt + LG_TBL);
              sR += nlog2n_cnt(tot[k] - left[k], lgt, lgt + LG_TBL);
            }
          const double TL = nlog2n_cnt((uint32_t)nL, lgt, lgt + LG_TBL) - sL;
          const double TR = nlog2n_cnt((uint32_t)nR, lgt, lgt + LG_TBL) - sR;
          loss = (TL + TR) / dn;
        }
        bl = loss;
        bb = b;
      }
    }
    // smallest loss, ties to the smaller bin: over the wave, then the 4 waves
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const double ol = __shfl_xor(bl, d);
      const int ob = __shfl_xor(bb, d);
      if (ol < bl || (ol == bl && ob < bb)) {
        bl = ol;
        bb = ob;
      }
    }
    if (lane == 0) {
      wbl[h][wv] = bl;
      wbb[h][wv] = bb;
    }
  }
  const int64_t o0 = (int64_t)lo * a.P + (int64_t)pt * PT + 2 * jp;
  const bool v1 = pt * PT + 2 * jp + 1 < a.P;
  if (a.hist_out && bv)
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (h == 0 || v1)
#pragma unroll
        for (int k = 0; k < KT; ++k)
          if (k < K) a.hist_out[((o0 + h) * B + b) * K + k] = c[h][k];
  lds_barrier();
  if (tid < 2 && (tid == 0 || v1)) {
    const int h = tid;
    const int64_t o = o0 + h;
    double l = wbl[h][0];
    int bw = wbb[h][0];
#pragma unroll
    for (int v = 1; v < 4; ++v)
      if (wbl[h][v] < l || (wbl[h][v] == l && wbb[h][v] < bw)) {
        l = wbl[h][v];
        bw = wbb[h][v];
      }
    if (bw == 0x7fffffff) {
      a.best_split[o] = -1;
      a.best_loss[o] = __builtin_huge_val();
      a.threshold[o] = __builtin_huge_valf();
    } else {
      const BinRule rr = make_rule(a.zmin[o], a.zmax[o], B);
      a.best_split[o] = bw;
      a.best_loss[o] = l;
      a.threshold[o] = edge(rr, bw);
    }
  }
}

// ---------------------------------------------------------------- fused evaluation
// Projection and histogram scan in one pass (classification, float32 X and W,
// D <= 64): the per-column min / max come from a first, store-free projection
// pass; here every wave recomputes its 32-row sub-tiles of Z on the matrix
// cores and bins them straight from the accumulator registers, so Z never
// reaches memory.  A work-group is (chunk-of-node item, 32-particle tile) with
// eight waves taking the item's sub-tiles in turn; lane (i, h) feeds row i
// and dimensions h KSP + s at MFMA step s, exactly as the short projection
// does, so every z is the float32 number the unfused path would store and the
// histograms, splits and losses are identical.  Accumulator layout, merge of
// multi-chunk nodes and finish are those of k_scan_hist (PT = 32).
typedef float f32x16s __attribute__((ext_vector_type(16)));

// MASK = false: values outside the data are left as loaded (see the
// short projection: X rows out of range are never used, X dimensions past D
// meet zeros in the masked W operand), so the loads stay in flight.
template <int KSP, bool VEC, bool MASK = true>
__device__ __forceinline__ void load_run_f32(const float *base, int64_t row, int D, int k0,
                                             bool ok, float (&v)[KSP]) {
  if constexpr (VEC) {
#pragma unroll
    for (int q = 0; q < KSP / 4; ++q) {
      const int kk = k0 + 4 * q;
      const bool in = !MASK || (ok && kk < D);
      const float4 f = *reinterpret_cast<const float4 *>(base + row * D + (kk < D ? kk : 0));
      v[4 * q + 0] = in ? f.x : 0.f;
      v[4 * q + 1] = in ? f.y : 0.f;
      v[4 * q + 2] = in ? f.z : 0.f;
      v[4 * q + 3] = in ? f.w : 0.f;
    }
  } else {
#pragma unroll
    for (int q = 0; q < KSP; ++q) {
      const int kk = k0 + q;
      const float t = base[row * D + (kk < D ? kk : D - 1)];
      v[q] = (!MASK || (ok && kk < D)) ? t : 0.f;
    }
  }
}

template <int KSP, int KT, bool VEC>
__global__ __launch_bounds__(HIST_WG) __attribute__((amdgpu_waves_per_eu(4)))
void k_fused_hist(ScanArgs a, const float *X, const float *W, int D, int64_t CH, int n_pt,
                  int64_t n_items, size_t slot_sz, int64_t n_slots) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int PT = 32, WGS = HIST_WG;
  const int B = a.bins, K = a.K;
  const HistLayout hl = hist_layout(PT, B, K, false);
  uint32_t *hc = reinterpret_cast<uint32_t *>(smem);
  double *lg = reinterpret_cast<double *>(smem + table_offset(PT, B, K, false));
  double *rc = lg + LG_TBL;
  const bool use_tbl = a.crit == SLM_ENTROPY;

  // the particle tiles of one item run on one XCD (its L2 serves their X rows)
  const int64_t bid = blockIdx.x;
  const int64_t local = bid >> 3;
  const int64_t v = (local / n_pt) * 8 + (bid & 7);
  const int pt = (int)(local % n_pt);
  if (v >= n_items) return;
  const Coords co = coords_of(a);
  Item it = find_item(co.beg, co.end, a.n_nodes, co.N, CH, v);
  if (it.node < 0) return;
  if (a.vpre) {   // back to data rows
    const Range nr = load_range(a.beg, a.end, it.node, a.N);
    const int64_t off = nr.lo - co.beg[it.node];
    it.lo += off;
    it.hi += off;
    if (it.hi > nr.hi) it.hi = nr.hi;
    if (it.lo >= it.hi) return;   // cannot happen with vpre matching the ranges
  }

  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int i = tid; i < hl.nwords; i += WGS) hc[i] = 0u;
  if (use_tbl) fill_log_table(lg, rc, tid);
  const int li = lane & 31, kh = lane >> 5;
  const int P = a.P;
  const int p = pt * PT + li;
  const bool pv = p < P;
  const int64_t np = (int64_t)it.node * P;
  const BinRule rule = make_rule(pv ? a.zmin[np + p] : 0.f, pv ? a.zmax[np + p] : 0.f, B);
  float bfrag[KSP];
  load_run_f32<KSP, VEC>(W, np + (pv ? p : P - 1), D, kh * KSP, pv, bfrag);
  lds_barrier();

  const bool wave_fast = __all(rule.fast || !pv);
  const float zmin = rule.zmin, delta = rule.delta, inv = rule.inv;
  const float off0 = -fmaf(zmin, inv, 0.005f);
  const unsigned bmax = (unsigned)B - 1u;
  const unsigned labk = pv ? (unsigned)K : 0u;
  const uint32_t ph4 = PT * 2u, sb4 = (uint32_t)hl.SB * 4u, pl4 = (uint32_t)(li >> 1) * 4u;
  const uint32_t pinc = 1u << ((li & 1) << 4);
  unsigned char *hb = reinterpret_cast<unsigned char *>(hc);
  const int nsub = (int)((it.hi - it.lo + 31) / 32);

  // A operands are single-buffered (the eight waves of two resident
  // work-groups per CU hide the load latency); B stays in registers
  float acur[KSP];
  for (int t = wave; t < nsub; t += WGS / 64) {
    const int64_t r0 = it.lo + 32 * (int64_t)t;
    const int64_t rl = r0 + li;
    load_run_f32<KSP, VEC, false>(X, rl < it.hi ? rl : it.hi - 1, D, kh * KSP, rl < it.hi, acur);
    const int labv = a.labels[rl < it.hi ? rl : it.hi - 1];
    f32x16s acc = f32x16s{};
#pragma unroll
    for (int ks = 0; ks < KSP; ++ks)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(acur[ks], bfrag[ks], acc, 0, 0, 0);
    // lane (li, kh), register r: row 8 (r / 4) + 4 kh + r % 4 of the sub-tile, particle li
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int rs = 8 * (r >> 2) + 4 * kh + (r & 3);
      const int lab = __shfl(labv, rs);
      const bool rin = r0 + rs < it.hi;
      const float z = acc[r];
      unsigned g;
      if (wave_fast) {
        const int g0 = (int)fmaf(z, inv, off0);
        const float e1 = __fadd_rn(zmin, __fmul_rn((float)(g0 + 1), delta));
        g = min((unsigned)(g0 + (e1 <= z ? 1 : 0)), bmax);
      } else {
        g = (unsigned)bin_of(rule, z);
      }
      const unsigned lb = min((unsigned)lab, (unsigned)K - 1u);
      const uint32_t inc = (rin && (unsigned)lab < labk) ? pinc : 0u;
      const uint32_t off = __umul24(g, sb4) + lb * ph4 + pl4;
      atomicAdd(reinterpret_cast<uint32_t *>(hb + off), inc);
    }
  }
  lds_barrier();

  // ---- a node spanning several chunks: add into its accumulator slot
  if (it.nchunks > 1) {
    const Range nr = load_range(co.beg, co.end, it.node, co.N);
    const int64_t slot = nr.lo / CH;
    if (slot >= n_slots) return;   // cannot happen with a workspace sized by the plan
    unsigned long long *gc = reinterpret_cast<unsigned long long *>(
        static_cast<unsigned char *>(a.ws) + ((size_t)slot * n_pt + pt) * slot_sz);
    for (int i = tid; i < hl.nwords; i += WGS) {
      const uint32_t w = hc[i];
      if (w)
        atomicAdd(&gc[i], (unsigned long long)(w & 0xFFFFu) | ((unsigned long long)(w >> 16) << 32));
    }
    return;
  }
  const FinishSrc src{hc, nullptr, nullptr, nullptr, nullptr, nullptr, 1, 0};
  finish_scan<PT, WGS, KT, false, false>(a, src, PT, pt, 0, np, smem, lg, rc, tid);
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
constexpr int EXACT_MAX = EXACT_ROWS;
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
      key[i] = a.Z[z_col(a.zl, p) + (rg.lo + i) * a.zl.rs];
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

// Finish of multi-chunk classification nodes: one work-group per particle
// and bin-parallel (k_scan_finish_bins) when the nodes average at least 16384
// rows (few large nodes: root-like levels), else groups of particles per
// work-group (k_scan_finish), whose fewer work-groups suit many small nodes
// that merely straddle a chunk boundary.  Measured (N = 1e5, P = 256): root
// 58.8 -> 51.9 us by bins; two nodes of 50000 rows 15.6 -> 8.6 us by bins;
// 128 nodes of 781 rows 128 us by groups, 154 us by bins.
// With a row prefix the nodes hold a.rows rows between them, not a.N.
bool finish_by_bins(const ScanArgs &a, int64_t) {
  return (a.vpre ? a.rows : a.N) / std::max(1, a.n_nodes) >= 16384;
}

template <int PT, int KT, bool MSE>
slm_status launch_hist_cfg(const ScanArgs &a, const Plan &pl, hipStream_t s) {
  const int n_pt = (a.P + PT - 1) / PT;
  const int64_t NW = a.vpre ? a.rows : a.N;   // extent of the item coordinates
  const int64_t items = num_items(a.n_nodes, NW, pl.CH);
  const int64_t total = items * n_pt;
  if (total == 0) return SLM_OK;
  const int64_t grid = (total + 8 * pl.G - 1) / (8 * pl.G) * (8 * pl.G);
  SLM_CHECK(grid < (1ll << 31), SLM_E_SHAPE, "slm_split_scan: grid too large");
  const int Kc = MSE ? 1 : a.K;
  const bool table = !MSE && a.crit == SLM_ENTROPY;
  const size_t lds = lds_bytes(PT, a.bins, Kc, MSE, table);
  const size_t slot = slot_bytes(PT, a.bins, Kc, MSE);
  const int64_t n_slots = (a.N - 1) / chunk_min(a.N) + 1;
  const int R = slot_replicas(a.N, a.P, a.bins, Kc, MSE);
  SLM_CHECK(slot_set_bytes(a.N, a.P, a.bins, Kc, MSE) * R <= a.ws_bytes, SLM_E_NOMEM,
            "slm_split_scan: workspace of %zu bytes too small for this launch", a.ws_bytes);
  hipLaunchKernelGGL((k_scan_hist<PT, KT, MSE>), dim3((unsigned)grid), dim3(HIST_WG), lds, s, a, pl.CH,
                     n_pt, pl.G, total, slot, n_slots, R);
  SLM_LAUNCHED();
  if (NW > pl.CH) {   // some node may span several chunks
    const int64_t used = (NW - 1) / pl.CH + 1;
    if (MSE || !finish_by_bins(a, pl.CH)) {
      constexpr int NQ = fin_nq(PT, KT);
      const int64_t grid_f = used * n_pt * (PT / NQ);
      SLM_CHECK(used <= n_slots && grid_f < (1ll << 31), SLM_E_SHAPE,
                "slm_split_scan: finish grid too large");
      hipLaunchKernelGGL((k_scan_finish<PT, KT, MSE>), dim3((unsigned)grid_f), dim3(256), 0, s, a,
                         pl.CH, n_pt, slot, n_slots, R);
    } else {
      const int64_t grid_f = used * n_pt * (PT / 2);
      SLM_CHECK(used <= n_slots && grid_f < (1ll << 31) && a.bins <= 256, SLM_E_SHAPE,
                "slm_split_scan: finish grid too large");
      hipLaunchKernelGGL((k_scan_finish_bins<KT>), dim3((unsigned)grid_f), dim3(256), 0, s, a, PT,
                         pl.CH, n_pt, slot, n_slots, R);
    }
    SLM_LAUNCHED();
  }
  return SLM_OK;
}

// Only tiles whose finish registers fit (PT x KT <= 128; regression
// PT <= 16) are instantiated; the plan never picks another.
template <int PT>
slm_status launch_hist_pt(const ScanArgs &a, const Plan &pl, hipStream_t s) {
  if (a.crit == SLM_MSE) {
    if constexpr (PT <= 16) return launch_hist_cfg<PT, 1, true>(a, pl, s);
  } else if (pl.KT == 2) {
    return launch_hist_cfg<PT, 2, false>(a, pl, s);
  } else if (pl.KT == 3) {
    return launch_hist_cfg<PT, 3, false>(a, pl, s);
  } else if (pl.KT == 4) {
    return launch_hist_cfg<PT, 4, false>(a, pl, s);
  } else if (pl.KT == 8) {
    if constexpr (PT <= 16) return launch_hist_cfg<PT, 8, false>(a, pl, s);
  } else {
    if constexpr (PT <= 8) return launch_hist_cfg<PT, 16, false>(a, pl, s);
  }
  SLM_CHECK(false, SLM_E_UNSUPPORTED, "slm_split_scan: no histogram kernel for PT=%d KT=%d", PT, pl.KT);
}

slm_status launch_hist(const ScanArgs &a, const Plan &pl, hipStream_t s) {
  switch (pl.PT) {
    case 32: return launch_hist_pt<32>(a, pl, s);
    case 16: return launch_hist_pt<16>(a, pl, s);
    case 8: return launch_hist_pt<8>(a, pl, s);
    default: return launch_hist_pt<4>(a, pl, s);
  }
}

template <int PT, int KT, bool MSE>
void set_lds_attr(int bytes) {
  // Best effort: raise the dynamic-LDS limit for the large-histogram tiles.
  // A refusal is cleared and left to the launch, which then reports it.
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_scan_hist<PT, KT, MSE>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess)
    (void)hipGetLastError();
}

template <int PT>
void set_lds_attr_pt(int bytes) {
  if constexpr (PT <= 16) set_lds_attr<PT, 1, true>(bytes);
  set_lds_attr<PT, 2, false>(bytes);
  set_lds_attr<PT, 3, false>(bytes);
  set_lds_attr<PT, 4, false>(bytes);
  if constexpr (PT <= 16) set_lds_attr<PT, 8, false>(bytes);
  if constexpr (PT <= 8) set_lds_attr<PT, 16, false>(bytes);
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
    set_lds_attr_pt<32>(dyn);
    set_lds_attr_pt<16>(dyn);
    set_lds_attr_pt<8>(dyn);
    set_lds_attr_pt<4>(dyn);
    prepare_pso_kernels(lds);
    prepare_project_kernels(lds);
  });
  return SLM_OK;
}

size_t scan_workspace_bytes(int64_t N, int n_nodes, int P, int bins, int K, int crit) {
  (void)n_nodes;
  if (bins == 0 || N <= 0) return 256;
  const bool mse = crit == SLM_MSE;
  const int Kc = mse ? 1 : K;
  return slot_set_bytes(N, P, bins, Kc, mse) * slot_replicas(N, P, bins, Kc, mse) + 256;
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
  SLM_CHECK(a.zl.eb == 4 || a.crit != SLM_MSE, SLM_E_UNSUPPORTED,
            "slm_split_scan: bfloat16 Z is read by the classification histogram scan only");
  if (a.N <= 0 || a.n_nodes <= 0) return SLM_OK;
  SLM_CHECK(!a.vpre || (a.rows >= 1 && a.rows <= a.N), SLM_E_INVALID,
            "slm_split_scan: row-prefix bound %lld outside [1, N]", (long long)a.rows);
  // With a row prefix the plan is made for the nodes' rows; its chunks stay
  // at least chunk_min(rows) long, so the slots, counted for N, still cover
  // every first chunk.
  const int64_t NW = a.vpre ? a.rows : a.N;
  const Plan pl = make_plan(NW, a.n_nodes, a.P, a.bins, a.crit == SLM_MSE ? 1 : a.K, a.crit);
  return launch_hist(a, pl, s);
}

slm_status tune_scan_hist(const ScanArgs &a, hipStream_t s) {
  if (a.N <= 0 || a.n_nodes <= 0 || a.bins == 0) return SLM_OK;
  const int64_t NW = a.vpre ? a.rows : a.N;
  const bool mse = a.crit == SLM_MSE;
  const int K = mse ? 1 : a.K;
  const std::string key = scan_key(NW, a.n_nodes, a.P, a.bins, K, a.crit);
  if (plan_known(key)) return SLM_OK;
  // candidates: the rule's plan, then every tile width with chunks from
  // chunk_min to the counter limit
  std::vector<Plan> cand;
  const Plan rule = make_plan(NW, a.n_nodes, a.P, a.bins, K, a.crit, false);
  cand.push_back(rule);
  const int64_t chs[] = {2048, 3072, 4096, 6144, 8192, 12288, 16384, 24576, 32768, 49152, CH_MAX};
  for (int pt = 4; pt <= 32; pt <<= 1) {
    if (pt / 2 >= a.P && pt > 4) continue;
    for (int64_t c : chs) {
      const int64_t ch = std::max<int64_t>(c, chunk_min(NW));
      if (!plan_fits(NW, a.bins, K, a.crit, pt, ch)) continue;
      Plan pl = rule;
      pl.PT = pt;
      pl.CH = ch;
      pl.G = std::max(1, 32 / pt);
      bool dup = false;
      for (const Plan &q : cand) dup = dup || (q.PT == pl.PT && q.CH == pl.CH);
      if (!dup) cand.push_back(pl);
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SLM_HIP(hipEventCreate(&e0));
  SLM_HIP(hipEventCreate(&e1));
  float best_ms = 0.f;
  Plan best = rule;
  slm_status st = SLM_OK;
  for (const Plan &pl : cand) {
    g_forced_scan = &pl;
    st = launch_hist(a, pl, s);                  // warm-up
    // the faster of two runs of four launches
    float ms = 0.f;
    for (int trial = 0; trial < 2 && !st; ++trial) {
      if (hipEventRecord(e0, s) != hipSuccess) st = SLM_E_HIP;
      for (int r = 0; r < 4 && !st; ++r) st = launch_hist(a, pl, s);
      float t = 0.f;
      if (!st && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        st = SLM_E_HIP;
      if (!st) ms = trial == 0 ? t : std::min(ms, t);
    }
    g_forced_scan = nullptr;
    if (st) break;
    if (&pl == &cand[0] || ms < best_ms) {
      best_ms = ms;
      best = pl;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) {
    (void)hipGetLastError();
    set_error("slm autotune: scan candidate failed");
    return st;
  }
  plan_store(key, best.PT, best.CH);
  return SLM_OK;
}

bool fused_eligible(const ScanArgs &a, int D, bool x_bf16, bool w_bf16) {
  return D >= 1 && D <= 64 && !x_bf16 && !w_bf16 && a.crit != SLM_MSE && a.bins >= 2 &&
         a.K >= 2 && a.K <= 4;
}

template <int KSP, int KT, bool VEC>
static slm_status launch_fused_k(const ScanArgs &a, const float *X, const float *W, int D,
                                 int64_t CH, hipStream_t s) {
  constexpr int PT = 32;
  const int n_pt = (a.P + PT - 1) / PT;
  const int64_t items = num_items(a.n_nodes, a.N, CH);
  if (items == 0) return SLM_OK;
  const int64_t grid = (items + 7) / 8 * 8 * n_pt;
  SLM_CHECK(grid < (1ll << 31), SLM_E_SHAPE, "slm_evaluate: grid too large");
  const bool table = a.crit == SLM_ENTROPY;
  const size_t lds = lds_bytes(PT, a.bins, a.K, false, table);
  const size_t slot = slot_bytes(PT, a.bins, a.K, false);
  const int64_t n_slots = (a.N - 1) / chunk_min(a.N) + 1;
  SLM_CHECK(slot_set_bytes(a.N, a.P, a.bins, a.K, false) <= a.ws_bytes, SLM_E_NOMEM,
            "slm_evaluate: workspace of %zu bytes too small", a.ws_bytes);
  hipLaunchKernelGGL((k_fused_hist<KSP, KT, VEC>), dim3((unsigned)grid), dim3(HIST_WG), lds, s, a,
                     X, W, D, CH, n_pt, items, slot, n_slots);
  SLM_LAUNCHED();
  if (a.N > CH) {
    const int64_t used = (a.N - 1) / CH + 1;
    if (finish_by_bins(a, CH)) {
      const int64_t grid_f = used * n_pt * (PT / 2);
      SLM_CHECK(used <= n_slots && grid_f < (1ll << 31) && a.bins <= 256, SLM_E_SHAPE,
                "slm_evaluate: finish grid too large");
      hipLaunchKernelGGL((k_scan_finish_bins<KT>), dim3((unsigned)grid_f), dim3(256), 0, s, a, PT,
                         CH, n_pt, slot, n_slots, 1);
    } else {
      constexpr int NQ = fin_nq(PT, KT);
      const int64_t grid_f = used * n_pt * (PT / NQ);
      SLM_CHECK(used <= n_slots && grid_f < (1ll << 31), SLM_E_SHAPE,
                "slm_evaluate: finish grid too large");
      hipLaunchKernelGGL((k_scan_finish<PT, KT, false>), dim3((unsigned)grid_f), dim3(256), 0, s,
                         a, CH, n_pt, slot, n_slots, 1);
    }
    SLM_LAUNCHED();
  }
  return SLM_OK;
}

template <int KSP, bool VEC>
static slm_status launch_fused_v(const ScanArgs &a, const float *X, const float *W, int D,
                                 int64_t CH, hipStream_t s) {
  if (a.K == 2) return launch_fused_k<KSP, 2, VEC>(a, X, W, D, CH, s);
  if (a.K == 3) return launch_fused_k<KSP, 3, VEC>(a, X, W, D, CH, s);
  return launch_fused_k<KSP, 4, VEC>(a, X, W, D, CH, s);
}

// Second pass of the fused evaluation (zmin / zmax already computed by the
// store-free projection pass).  Requires fused_eligible().
slm_status launch_fused_hist(const ProjectArgs &pr, const ScanArgs &a, hipStream_t s) {
  SLM_CHECK(fused_eligible(a, pr.D, pr.x_bf16, pr.w_bf16), SLM_E_UNSUPPORTED,
            "slm_evaluate: the fused evaluation needs float32 data, D <= 64, 2 <= K <= 4 and "
            "Gini or entropy");
  if (a.N <= 0 || a.n_nodes <= 0) return SLM_OK;
  const Plan pl = make_plan(a.N, a.n_nodes, a.P, a.bins, a.K, a.crit);
  const int64_t CH = pl.CH;
  const float *X = static_cast<const float *>(pr.X);
  const float *W = static_cast<const float *>(pr.W);
  const int D = pr.D;
  const bool vec = D % 4 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(W) % 16 == 0;
  auto go = [&](auto ksp) -> slm_status {
    constexpr int KSP = decltype(ksp)::value;
    return vec ? launch_fused_v<KSP, true>(a, X, W, D, CH, s)
               : launch_fused_v<KSP, false>(a, X, W, D, CH, s);
  };
  if (D <= 8) return go(std::integral_constant<int, 4>{});
  if (D <= 16) return go(std::integral_constant<int, 8>{});
  if (D <= 32) return go(std::integral_constant<int, 16>{});
  return go(std::integral_constant<int, 32>{});
}

// Fused evaluation: the min / max pass (the short projection without Z
// stores) then the fused projection-histogram pass.
slm_status launch_fused_eval(const ProjectArgs &pr, const ScanArgs &a, hipStream_t s) {
  SLM_CHECK(fused_eligible(a, pr.D, pr.x_bf16, pr.w_bf16), SLM_E_UNSUPPORTED,
            "slm_evaluate: the fused evaluation needs float32 data, D <= 64, 2 <= K <= 4 and "
            "Gini or entropy");
  if (a.N <= 0 || a.n_nodes <= 0) return SLM_OK;
  ProjectArgs p1 = pr;
  p1.Z = nullptr;
  slm_status st = launch_project(p1, s);
  if (st) return st;
  return launch_fused_hist(pr, a, s);
}

slm_status launch_scan_exact(const ScanArgs &a, int max_rows, hipStream_t s) {
  SLM_CHECK(a.zl.eb == 4, SLM_E_UNSUPPORTED,
            "slm_split_scan: bfloat16 Z is read by the classification histogram scan only");
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
