// C ABI of libslm.so: argument validation, workspace carving and the
// breadth-first tree driver (Sec. III-B, Alg. 2).  Every numeric step runs in
// the HIP kernels of this library; the host only sequences launches and reads
// a few bytes of frontier state back per depth.
#include "slm_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

namespace slm {

static thread_local char g_err[512] = "";
static thread_local bool g_capturing = false;
bool capturing() { return g_capturing; }
void set_capturing(bool on) { g_capturing = on; }

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}
void clear_error() { g_err[0] = 0; }

namespace {

constexpr int DMAX = 4096;
constexpr int PMAX = 4096;

inline hipStream_t S(void *s) { return static_cast<hipStream_t>(s); }

// ---------------------------------------------------------------- workspace carving
struct Carver {
  char *base;
  size_t off = 0;
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) / 256 * 256;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Most nodes one depth searches: per tree 2^(max_depth - 1), and at most
// N / min_node over all trees (their row sets are disjoint).  At least one
// slot per root (the roots' statistics).
int64_t max_active(const slm_tree_params &p, int64_t N, int64_t n_roots = 1) {
  if (p.max_depth <= 0) return n_roots;
  const int64_t by_depth = p.max_depth - 1 >= 30 ? (1ll << 30) : (1ll << (p.max_depth - 1));
  const int64_t by_size = std::max<int64_t>(1, N / std::max(1, p.min_node));
  return std::max<int64_t>(n_roots, std::min(by_depth * n_roots, by_size));
}

struct TreeWS {
  void *Xa, *Xb;
  void *ta, *tb;
  float *Z, *zsel, *zmin, *zmax;
  double *x, *v, *pbest, *pbest_loss, *loss, *gbest, *gbest_loss;
  void *W, *gW;
  int32_t *split, *gbest_p, *gbest_split, *node_id, *do_split;
  uint32_t *tree_off;   // tree of every searched node (several roots)
  int64_t *vpre;        // rows of the searched nodes before each one (F + 1)
  // adaptive swarm: per-node state, parameters, distances, worst particle,
  // elite candidate, partial distance sums
  int32_t *ap_state, *ap_worst;
  double *ap_par, *ap_dist, *ap_f, *ap_elite, *ap_part;
  // fused swarm steps: the second position buffer and global-best record
  double *x2, *gbest2, *gbest_loss2;
  float *thr, *gbest_thr;
  int64_t *beg, *end, *n_left, *off_left, *off_right;
  uint64_t *seed_tree;
  uint32_t *cnt_left;
  // screening (precision = 1): selection, float32 re-projection and its scan
  int32_t *sel, *split_r;
  float *W32, *Zr, *zmin_r, *zmax_r, *thr_r;
  double *loss_r, *gloss;
  // node statistics and learned proposal
  double *stat_sums;
  uint32_t *stat_counts;
  float *stats, *sigma, *mlp_cache, *mlp_out;
  // top-n DFT channels (dft_top_n): losses, selection, scan scratch
  double *dft_loss;
  int32_t *dft_sel;
  void *dft_ws;
  size_t dft_ws_bytes;
  // node-batch search: active row ends, stop state
  int64_t *end_act;
  int32_t *done;
  uint32_t *remaining;
  TreeStats st;
  void *scan_ws;
  size_t scan_ws_bytes;
  size_t total;
};

// The plain swarm's bests and move run as one launch (k_pso_fused) in tree
// builds; SLM_PSO_FUSED=0 keeps the two launches (timing comparisons).
bool fused_step_enabled() {
  static const int on = [] {
    const char *e = getenv("SLM_PSO_FUSED");
    return e && e[0] == '0' ? 0 : 1;
  }();
  return on != 0;
}
bool fused_step_possible(const slm_tree_params &p) {
  return fused_step_enabled() && p.apso == 0 && p.precision == 0 && p.proposal != 2;
}

// Workspace of a tree build (search_nodes = 0) or of one node-batch search of
// search_nodes nodes (no partition buffers).  stats: node statistics wanted.
TreeWS carve(const slm_tree_params &p, int64_t N, int32_t D, void *base, int search_nodes = 0,
             bool stats = false, int64_t n_roots = 1) {
  Carver c{static_cast<char *>(base)};
  TreeWS w{};
  const bool search = search_nodes > 0;
  const int64_t F = search ? search_nodes : max_active(p, N, n_roots);
  const bool mse = p.crit == SLM_MSE;
  const size_t xb = p.precision == 1 ? 2 : 4;
  const int Kc = mse ? 1 : p.K;
  if (!search) {
    w.Xa = c.take<char>((size_t)N * D * xb);
    w.Xb = c.take<char>((size_t)N * D * xb);
    w.ta = c.take<char>((size_t)N * (mse ? 8 : 4));
    w.tb = c.take<char>((size_t)N * (mse ? 8 : 4));
  }
  w.Z = c.take<float>((size_t)N * ((p.P + 31) / 32 * 32));   // particle-tiled
  if (!search) w.zsel = c.take<float>((size_t)N);
  w.zmin = c.take<float>((size_t)F * p.P);
  w.zmax = c.take<float>((size_t)F * p.P);
  w.x = c.take<double>((size_t)F * p.P * D);
  w.v = c.take<double>((size_t)F * p.P * D);
  w.pbest = c.take<double>((size_t)F * p.P * D);
  w.W = c.take<char>((size_t)F * p.P * D * xb);
  w.pbest_loss = c.take<double>((size_t)F * p.P);
  w.loss = c.take<double>((size_t)F * p.P);
  w.split = c.take<int32_t>((size_t)F * p.P);
  w.thr = c.take<float>((size_t)F * p.P);
  w.gbest = c.take<double>((size_t)F * D);
  w.gbest_loss = c.take<double>((size_t)F);
  w.gbest_p = c.take<int32_t>((size_t)F);
  w.gbest_split = c.take<int32_t>((size_t)F);
  w.gbest_thr = c.take<float>((size_t)F);
  w.gW = c.take<float>((size_t)F * D);     // float32 split directions of the partition
  w.beg = c.take<int64_t>((size_t)F);
  w.end = c.take<int64_t>((size_t)F);
  w.node_id = c.take<int32_t>((size_t)F);
  if (n_roots > 1) w.tree_off = c.take<uint32_t>((size_t)F);
  w.vpre = c.take<int64_t>((size_t)F + 1);
  if (!search && fused_step_possible(p)) {
    w.x2 = c.take<double>((size_t)F * p.P * D);
    w.gbest2 = c.take<double>((size_t)F * D);
    w.gbest_loss2 = c.take<double>((size_t)F);
  }
  if (p.apso) {
    w.ap_state = c.take<int32_t>((size_t)F);
    w.ap_worst = c.take<int32_t>((size_t)F);
    w.ap_par = c.take<double>((size_t)F * 3);
    w.ap_dist = c.take<double>((size_t)F * p.P);
    w.ap_f = c.take<double>((size_t)F);
    w.ap_elite = c.take<double>((size_t)F * D);
    w.ap_part = reinterpret_cast<double *>(c.take<char>(apso_part_bytes((int)F, p.P)));
  }
  w.do_split = c.take<int32_t>((size_t)F);
  w.n_left = c.take<int64_t>((size_t)F);
  w.seed_tree = c.take<uint64_t>(2);
  if (!search) {
    const int64_t items = partition_items((int)F, N);
    w.cnt_left = c.take<uint32_t>((size_t)items);
    w.off_left = c.take<int64_t>((size_t)items);
    w.off_right = c.take<int64_t>((size_t)items);
  } else {
    w.end_act = c.take<int64_t>((size_t)F);
    w.done = c.take<int32_t>((size_t)F);
    w.remaining = c.take<uint32_t>(1);
  }
  if (stats || p.proposal == 1) {
    const size_t sws = stats_workspace_bytes((int)F, D, Kc);
    char *sb = c.take<char>(sws);
    w.stat_sums = reinterpret_cast<double *>(sb);
    w.stat_counts = sb ? reinterpret_cast<uint32_t *>(sb + ((size_t)F * Kc * D * 2 * 8 + 255) / 256 * 256)
                       : nullptr;
    w.stats = c.take<float>((size_t)F * (Kc + 1) * D);
    w.sigma = c.take<float>((size_t)F * D);
  }
  if (p.proposal == 1) {
    w.mlp_cache = c.take<float>((size_t)F * 4 * p.mlp_hidden);
    w.mlp_out = c.take<float>((size_t)F * p.n_seeds * D);
  }
  if (p.precision == 1) {
    const int k = p.rescore_k;
    w.sel = c.take<int32_t>((size_t)F * k);
    w.W32 = c.take<float>((size_t)F * k * D);
    w.Zr = c.take<float>((size_t)N * ((k + 31) / 32 * 32));   // particle-tiled
    w.zmin_r = c.take<float>((size_t)F * k);
    w.zmax_r = c.take<float>((size_t)F * k);
    w.loss_r = c.take<double>((size_t)F * k);
    w.split_r = c.take<int32_t>((size_t)F * k);
    w.thr_r = c.take<float>((size_t)F * k);
    w.gloss = c.take<double>((size_t)F * p.P);
  }
  const int n_sel = p.proposal == 2 ? p.ps_R : (p.dft_top_n > 0 && p.dft_top_n < D ? p.dft_top_n : 0);
  if (n_sel > 0) {
    w.dft_loss = c.take<double>((size_t)F * D);
    w.dft_sel = c.take<int32_t>((size_t)F * n_sel);
    w.dft_ws_bytes = dft_workspace_bytes(N, (int)F, D, p.bins, p.K, p.crit);
    w.dft_ws = c.take<char>(w.dft_ws_bytes);
  }
  w.st.counts = c.take<uint32_t>((size_t)2 * F * Kc);
  w.st.cnt = c.take<uint32_t>((size_t)2 * F);
  w.st.s1 = c.take<double>((size_t)2 * F);
  w.st.s2 = c.take<double>((size_t)2 * F);
  w.st.ymin = c.take<unsigned long long>((size_t)2 * F);
  w.st.ymax = c.take<unsigned long long>((size_t)2 * F);
  w.scan_ws_bytes = p.bins ? scan_workspace_bytes(N, (int)F, p.P, p.bins, p.K, p.crit) : 256;
  if (p.bins && p.precision == 1)   // the re-scoring scan runs with rescore_k particles
    w.scan_ws_bytes = std::max(w.scan_ws_bytes,
                               scan_workspace_bytes(N, (int)F, p.rescore_k, p.bins, p.K, p.crit));
  w.scan_ws = c.take<char>(w.scan_ws_bytes);
  w.total = c.off + 256;
  return w;
}

slm_status check_tree_params(const slm_tree_params *p, int64_t N, int32_t D) {
  SLM_CHECK(p != nullptr, SLM_E_INVALID, "slm_grow_tree: params is NULL");
  SLM_CHECK(N >= 1 && N < (1ll << 31), SLM_E_SHAPE, "slm_grow_tree: N = %lld out of range",
            (long long)N);
  SLM_CHECK(D >= 1 && D <= DMAX, SLM_E_SHAPE, "slm_grow_tree: D = %d out of range", D);
  SLM_CHECK(p->crit >= 0 && p->crit <= 2, SLM_E_INVALID, "slm_grow_tree: bad criterion %d",
            p->crit);
  if (p->crit == SLM_MSE)
    SLM_CHECK(p->K == 0, SLM_E_SHAPE, "slm_grow_tree: K must be 0 for SLM_MSE");
  else
    SLM_CHECK(p->K >= 2 && p->K <= 16, SLM_E_SHAPE, "slm_grow_tree: K = %d not in [2,16]", p->K);
  SLM_CHECK(p->P >= 1 && p->P <= PMAX, SLM_E_SHAPE, "slm_grow_tree: P = %d out of range", p->P);
  SLM_CHECK(p->T >= 0 && p->T <= 100000, SLM_E_SHAPE, "slm_grow_tree: T = %d out of range", p->T);
  SLM_CHECK(p->bins == 0 || (p->bins >= 2 && p->bins <= 256), SLM_E_SHAPE,
            "slm_grow_tree: bins = %d (0 or 2..256)", p->bins);
  SLM_CHECK(p->max_depth >= 0 && p->max_depth <= 30, SLM_E_SHAPE,
            "slm_grow_tree: max_depth = %d out of range", p->max_depth);
  SLM_CHECK(p->min_node >= 1, SLM_E_SHAPE, "slm_grow_tree: min_node must be >= 1");
  SLM_CHECK(p->precision == 0 || p->precision == 1, SLM_E_INVALID,
            "slm_grow_tree: precision %d (0 = float32, 1 = bfloat16 screen)", p->precision);
  if (p->precision == 1)
    SLM_CHECK(p->rescore_k >= 1 && p->rescore_k <= p->P, SLM_E_SHAPE,
              "slm_grow_tree: rescore_k = %d not in [1, P]", p->rescore_k);
  SLM_CHECK(p->dft_top_n >= 0 && p->dft_top_n <= D, SLM_E_SHAPE,
            "slm_grow_tree: dft_top_n = %d not in [0, D]", p->dft_top_n);
  if (p->dft_top_n > 0 && p->dft_top_n < D)
    SLM_CHECK(p->precision == 0, SLM_E_UNSUPPORTED,
              "slm_grow_tree: dft_top_n needs float32 data (precision 0)");
  SLM_CHECK(p->proposal >= 0 && p->proposal <= 2, SLM_E_INVALID,
            "slm_grow_tree: proposal %d (0 = random, 1 = learned, 2 = probabilistic search)",
            p->proposal);
  if (p->proposal == 2) {
    SLM_CHECK(p->ps_R >= 1 && p->ps_R <= std::min(D, PS_RMAX), SLM_E_SHAPE,
              "slm_grow_tree: ps_R = %d not in [1, min(D, %d)]", p->ps_R, PS_RMAX);
    SLM_CHECK(p->ps_pd != nullptr && p->ps_amax != nullptr, SLM_E_INVALID,
              "slm_grow_tree: proposal 2 needs ps_pd and ps_amax");
    SLM_CHECK(p->precision == 0 && (p->dft_top_n == 0 || p->dft_top_n == D), SLM_E_UNSUPPORTED,
              "slm_grow_tree: proposal 2 needs float32 data and no dft_top_n");
  }
  SLM_CHECK(p->apso == 0 || p->apso == 1, SLM_E_INVALID, "slm_grow_tree: apso %d (0 or 1)",
            p->apso);
  if (p->apso)
    SLM_CHECK(p->P >= 2 && p->proposal != 2, SLM_E_UNSUPPORTED,
              "slm_grow_tree: the adaptive swarm needs P >= 2 and a swarm (not proposal 2)");
  if (p->proposal == 1) {
    SLM_CHECK(p->crit != SLM_MSE, SLM_E_UNSUPPORTED,
              "slm_grow_tree: the learned proposal needs class labels");
    SLM_CHECK(p->mlp != nullptr, SLM_E_INVALID, "slm_grow_tree: proposal 1 needs mlp parameters");
    SLM_CHECK(p->n_seeds >= 1 && p->n_seeds <= 4096 && p->mlp_hidden >= 1 &&
                  p->mlp_hidden <= 4096,
              SLM_E_SHAPE, "slm_grow_tree: n_seeds = %d / mlp_hidden = %d out of range",
              p->n_seeds, p->mlp_hidden);
    SLM_CHECK(p->K * D <= 4096, SLM_E_SHAPE, "slm_grow_tree: K * D = %d too large for the proposal",
              p->K * D);
  }
  return SLM_OK;
}

double nlog2n(double x) { return x > 0 ? x * std::log2(x) : 0.0; }

// ---------------------------------------------------------------- host tree state
struct HNode {
  int idx;
  int64_t beg, end;
  int depth, heap;
  double impurity;
  bool impure;
  uint32_t tree;   // root index (trees grown together)
};

// ---------------------------------------------------------------- pinned staging
// The tree driver's per-depth host <-> device transfers go through
// page-locked host memory: one arena per thread, grown at the start of a
// build (when no transfer of an earlier build is in flight) and then reused,
// so every transfer is a direct DMA copy instead of a staged pageable one.
struct PinnedArena {
  char *base = nullptr;
  size_t cap = 0, off = 0;
};
thread_local PinnedArena g_pin;

slm_status pinned_begin(size_t bytes) {
  if (g_pin.cap < bytes) {
    if (g_pin.base) (void)hipHostFree(g_pin.base);
    g_pin.base = nullptr;
    g_pin.cap = 0;
    SLM_HIP(hipHostMalloc(reinterpret_cast<void **>(&g_pin.base), bytes, hipHostMallocDefault));
    g_pin.cap = bytes;
  }
  g_pin.off = 0;
  return SLM_OK;
}

template <typename T>
T *pinned_take(size_t n) {
  const size_t o = (g_pin.off + 63) / 64 * 64;
  g_pin.off = o + n * sizeof(T);
  return reinterpret_cast<T *>(g_pin.base + o);
}

size_t pinned_bytes(size_t n, size_t elem) { return (n * elem + 63) / 64 * 64; }

// host copies of the node statistics (capacity 2F entries, pinned)
struct StatsHost {
  uint32_t *counts, *cnt;
  double *s1, *s2;
  unsigned long long *ymin, *ymax;
};

double dec_f64(unsigned long long e) {
  const unsigned long long u = (e >> 63) ? (e & 0x7FFFFFFFFFFFFFFFull) : ~e;
  double d;
  std::memcpy(&d, &u, 8);
  return d;
}

// impurity, purity flag and leaf value of stats entry i (same formulas as the
// criteria: Gini (n - A/n)/n, entropy (n log2 n - sum n_k log2 n_k)/n,
// squared error (S2 - S1^2/n)/n)
void summarize(const StatsHost &h, int i, int crit, int K, double *imp, bool *impure,
               double *leaf, int64_t *n) {
  if (crit == SLM_MSE) {
    const double cnt = h.cnt[i];
    *n = h.cnt[i];
    if (cnt == 0) {
      *imp = 0;
      *impure = false;
      leaf[0] = 0;
      return;
    }
    *imp = (h.s2[i] - h.s1[i] * h.s1[i] / cnt) / cnt;
    *impure = dec_f64(h.ymax[i]) > dec_f64(h.ymin[i]);
    leaf[0] = h.s1[i] / cnt;
    return;
  }
  int64_t tot = 0;
  uint64_t A = 0;
  double sl = 0;
  for (int k = 0; k < K; ++k) {
    const uint64_t c = h.counts[(size_t)i * K + k];
    tot += c;
    A += c * c;
    sl += nlog2n((double)c);
    leaf[k] = (double)c;
  }
  *n = tot;
  if (tot == 0) {
    *imp = 0;
    *impure = false;
    return;
  }
  const double dn = (double)tot;
  *imp = crit == SLM_GINI ? (dn - (double)A / dn) / dn : (nlog2n(dn) - sl) / dn;
  *impure = *imp > 0;
}

slm_status read_stats(const TreeWS &w, int n, int crit, int K, StatsHost &h, hipStream_t s) {
  if (crit == SLM_MSE) {
    SLM_HIP(hipMemcpyAsync(h.cnt, w.st.cnt, n * 4, hipMemcpyDeviceToHost, s));
    SLM_HIP(hipMemcpyAsync(h.s1, w.st.s1, n * 8, hipMemcpyDeviceToHost, s));
    SLM_HIP(hipMemcpyAsync(h.s2, w.st.s2, n * 8, hipMemcpyDeviceToHost, s));
    SLM_HIP(hipMemcpyAsync(h.ymin, w.st.ymin, n * 8, hipMemcpyDeviceToHost, s));
    SLM_HIP(hipMemcpyAsync(h.ymax, w.st.ymax, n * 8, hipMemcpyDeviceToHost, s));
  } else {
    SLM_HIP(hipMemcpyAsync(h.counts, w.st.counts, (size_t)n * K * 4, hipMemcpyDeviceToHost, s));
  }
  return SLM_OK;
}

slm_status clear_stats(const TreeWS &w, int n, int crit, int K, hipStream_t s) {
  if (crit == SLM_MSE) {
    SLM_HIP(hipMemsetAsync(w.st.cnt, 0, (size_t)n * 4, s));
    SLM_HIP(hipMemsetAsync(w.st.s1, 0, (size_t)n * 8, s));
    SLM_HIP(hipMemsetAsync(w.st.s2, 0, (size_t)n * 8, s));
    SLM_HIP(hipMemsetAsync(w.st.ymin, 0xFF, (size_t)n * 8, s));
    SLM_HIP(hipMemsetAsync(w.st.ymax, 0, (size_t)n * 8, s));
  } else {
    SLM_HIP(hipMemsetAsync(w.st.counts, 0, (size_t)n * K * 4, s));
  }
  return SLM_OK;
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  bool on = false;
  double *acc = nullptr;
  slm_status start(double *target, hipStream_t s) {
    acc = target;
    on = target != nullptr;
    if (!on) return SLM_OK;
    if (!a) {
      SLM_HIP(hipEventCreate(&a));
      SLM_HIP(hipEventCreate(&b));
    }
    SLM_HIP(hipEventRecord(a, s));
    return SLM_OK;
  }
  slm_status stop(hipStream_t s) {
    if (!on) return SLM_OK;
    SLM_HIP(hipEventRecord(b, s));
    SLM_HIP(hipEventSynchronize(b));
    float ms = 0;
    SLM_HIP(hipEventElapsedTime(&ms, a, b));
    *acc += ms;
    return SLM_OK;
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// ---------------------------------------------------------------- graph cache
// One captured swarm loop (T+1 evaluations) per distinct launch signature.
struct GraphKey {
  std::vector<uint64_t> k;
  bool operator<(const GraphKey &o) const { return k < o.k; }
};
std::mutex g_graph_mu;
std::map<GraphKey, hipGraphExec_t> g_graphs;

}  // namespace

// Optional per-launch timing: event pairs recorded around launches on the
// launch stream, read after the depth's synchronisation.  The events skip the
// system-scope fence a recorded event otherwise issues (a write-back of the
// dirty L2 lines, e.g. of the Z a projection has just written): they order
// nothing, the stream synchronisation does, and the fence would add several
// microseconds to every measured span.
struct LaunchTimes {
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, size_t>> marks;   // (kind, index of the start event)
  size_t used = 0;
  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  slm_status begin(int kind, hipStream_t s) {
    hipEvent_t e = next();
    SLM_CHECK(e != nullptr, SLM_E_HIP, "hipEventCreate failed");
    marks.push_back({kind, used - 1});
    SLM_HIP(hipEventRecord(e, s));
    return SLM_OK;
  }
  slm_status end(hipStream_t s) {
    hipEvent_t e = next();
    SLM_CHECK(e != nullptr, SLM_E_HIP, "hipEventCreate failed");
    SLM_HIP(hipEventRecord(e, s));
    return SLM_OK;
  }
  // after a stream sync: add each kind's elapsed time to acc[kind], counts to cnt[kind]
  slm_status collect(double *acc, double *cnt) {
    for (auto &m : marks) {
      float ms = 0;
      SLM_HIP(hipEventElapsedTime(&ms, pool[m.second], pool[m.second + 1]));
      acc[m.first] += ms;
      if (cnt) cnt[m.first] += 1;
    }
    marks.clear();
    used = 0;
    return SLM_OK;
  }
  ~LaunchTimes() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// Stop control of a node-batch search: per-node loss targets, evaluation
// counts, and the host copy of the number of nodes still searching.
struct SearchCtl {
  const double *target;   // [device] per-node targets or null (run all T + 1)
  int32_t *evals;         // [device] evaluations per node
  uint32_t *h_remaining;  // [host]
};

// Learned start: node statistics, BF16 network inference, seeds written over
// the first min(n_seeds, P) particles of every node (after the random start).
static slm_status learned_start(const slm_tree_params &p, const TreeWS &w, const void *Xc,
                                const void *tc, int64_t N, int32_t D, int na, hipStream_t s) {
  StatsArgs sa{};
  sa.X = Xc; sa.x_bf16 = p.precision == 1; sa.N = N; sa.D = D;
  sa.labels = static_cast<const int32_t *>(tc); sa.K = p.K; sa.beg = w.beg; sa.end = w.end;
  sa.n_nodes = na; sa.sums = w.stat_sums; sa.counts = w.stat_counts; sa.stats = w.stats;
  sa.sigma = w.sigma;
  slm_status st = launch_node_stats_full(sa, s);
  if (st) return st;
  const int I = (p.K + 1) * D, O = p.n_seeds * D;
  if ((st = launch_mlp_forward(p.mlp, I, p.mlp_hidden, O, w.stats, na, 1, w.mlp_out, w.mlp_cache,
                               s)))
    return st;
  return launch_seeds(w.mlp_out, w.sigma, na, p.n_seeds, D, p.P, w.x, w.pbest, w.W,
                      p.precision == 1, s);
}

// swarm loop of one depth: T+1 evaluations (project, scan, step)
// tune: the autotuner's pass (plan cache mode 2, never under capture): the
// first evaluation only, each projection and scan launch preceded by the
// measurement of its shape's candidate plans (shapes already cached are
// skipped); the swarm loop that follows takes the measured plans.
static slm_status swarm_loop(const slm_tree_params &p, const TreeWS &w, const void *Xc,
                             const void *tc, int64_t N, int32_t D, int na, int64_t vrows,
                             hipStream_t s,
                             LaunchTimes *lt = nullptr, const SearchCtl *sc = nullptr,
                             bool tune = false) {
  const bool mse = p.crit == SLM_MSE;
  PsoArgs pa{};
  pa.x = w.x; pa.v = w.v; pa.pbest = w.pbest; pa.pbest_loss = w.pbest_loss;
  pa.gbest = w.gbest; pa.gbest_loss = w.gbest_loss; pa.gbest_p = w.gbest_p;
  pa.loss = w.loss; pa.split = w.split; pa.thr = w.thr;
  pa.gbest_split = w.gbest_split; pa.gbest_thr = w.gbest_thr;
  pa.node_id = w.node_id; pa.n_nodes = na; pa.P = p.P; pa.D = D;
  pa.omega = p.omega; pa.c1 = p.c1; pa.c2 = p.c2; pa.seed = p.seed; pa.tree = p.tree;
  const bool scr = p.precision == 1;
  pa.W_out = w.W; pa.w_bf16 = scr;
  pa.gloss = scr ? w.gloss : nullptr;
  pa.zmin_reset = w.zmin; pa.zmax_reset = w.zmax;
  pa.seed_tree_dev = w.seed_tree;
  pa.tree_off = w.tree_off;
  if (p.apso) {
    pa.apso_state = w.ap_state; pa.apso_par = w.ap_par; pa.apso_dist = w.ap_dist;
    pa.apso_f = w.ap_f; pa.apso_worst = w.ap_worst; pa.apso_elite = w.ap_elite;
    pa.apso_part = w.ap_part; pa.apso_T = (uint32_t)std::max(1, p.T);
  }
  slm_status st;
  const bool psearch = p.proposal == 2;
  if (psearch || (p.dft_top_n > 0 && p.dft_top_n < D)) {
    // Alg. 2: the DFT of every node, then the swarm starts in the span of
    // its top dft_top_n channels; the probabilistic search (proposal 2)
    // combines the node's ps_R best-ranked features instead
    DftArgs da{};
    da.X = static_cast<const float *>(Xc); da.N = N; da.D = D; da.beg = w.beg;
    da.end = sc ? w.end_act : w.end; da.n_nodes = na;
    da.labels = mse ? nullptr : static_cast<const int32_t *>(tc);
    da.y = mse ? static_cast<const double *>(tc) : nullptr;
    da.K = p.K; da.bins = p.bins; da.crit = p.crit; da.n = psearch ? p.ps_R : p.dft_top_n;
    da.loss = w.dft_loss; da.sel = w.dft_sel; da.ws = w.dft_ws; da.ws_bytes = w.dft_ws_bytes;
    if ((st = launch_dft_select(da, s))) return st;
    if (!psearch) {
      pa.dim_sel = w.dft_sel;
      pa.n_sel = p.dft_top_n;
      if (p.apso) {   // the elitist step stays in the node's channels
        pa.apso_sel = w.dft_sel;
        pa.apso_n_sel = p.dft_top_n;
      }
    }
  }
  st = launch_pso_init(pa, s);
  if (st) return st;
  pa.dim_sel = nullptr;
  pa.n_sel = 0;
  if (p.proposal == 1 && (st = learned_start(p, w, Xc, tc, N, D, na, s))) return st;
  // a search skips the rows of stopped nodes: their active end collapses to
  // their start, and their scan results read "no split"
  const int64_t *ends = sc ? w.end_act : w.end;
  ProjectArgs pr{};
  pr.X = Xc; pr.x_bf16 = scr; pr.w_bf16 = scr; pr.N = N; pr.D = D; pr.W = w.W; pr.beg = w.beg;
  pr.end = ends;
  pr.n_nodes = na; pr.P = p.P; pr.Z = w.Z; pr.zmin = w.zmin; pr.zmax = w.zmax;
  // the screening pass of a classification histogram search stores its Z in
  // bfloat16 (it only ranks the directions; the re-scoring is float32)
  const bool zbf = scr && !mse && p.bins > 0 && project_writes_bf16(pr);
  pr.zl = zlayout_of(grow_z_layout(N, zbf), N, p.P);
  pr.vpre = vrows > 0 ? w.vpre : nullptr;
  pr.rows = vrows > 0 ? vrows : 0;
  ScanArgs sa{};
  sa.Z = w.Z; sa.zl = pr.zl; sa.zmin = w.zmin; sa.zmax = w.zmax;
  sa.labels = mse ? nullptr : static_cast<const int32_t *>(tc);
  sa.y = mse ? static_cast<const double *>(tc) : nullptr;
  sa.K = p.K; sa.N = N; sa.beg = w.beg; sa.end = ends; sa.n_nodes = na; sa.P = p.P;
  sa.bins = p.bins; sa.crit = p.crit; sa.best_split = w.split; sa.best_loss = w.loss;
  sa.threshold = w.thr; sa.ws = w.scan_ws; sa.ws_bytes = w.scan_ws_bytes;
  // row prefix for the histogram scan (vrows: a bound on the nodes' rows)
  sa.vpre = vrows > 0 && p.bins ? w.vpre : nullptr;
  sa.rows = vrows;
  // float32 re-scoring of the screened evaluation's best rescore_k particles
  const int k = p.rescore_k;
  ProjectArgs prr = pr;
  ScanArgs sar = sa;
  if (scr) {
    prr.x_bf16 = 1; prr.w_bf16 = 0; prr.W = w.W32; prr.P = k; prr.Z = w.Zr;
    prr.zmin = w.zmin_r; prr.zmax = w.zmax_r; prr.zl = zlayout_of(grow_z_layout(N), N, k);
    sar.Z = w.Zr; sar.zl = prr.zl; sar.zmin = w.zmin_r; sar.zmax = w.zmax_r; sar.P = k;
    sar.best_split = w.split_r; sar.best_loss = w.loss_r; sar.threshold = w.thr_r;
  }
  auto scan = [&](const ScanArgs &x) {
    slm_status r = p.bins ? launch_scan_hist(x, s) : launch_scan_exact(x, EXACT_ROWS, s);
    if (!r && sc && p.bins) r = launch_scan_empty_nodes(x, s);
    return r;
  };
  // The fused projection + histogram scan (slm_evaluate) is opt-in
  // (SLM_FUSED=1): on MI355X at D = 64 the second MFMA projection it needs
  // costs more than the round trip of Z through memory (plain-tree root: 191
  // vs 135 us per evaluation).
  const char *fz = getenv("SLM_FUSED");
  const bool fused = !scr && fz && fz[0] == '1' && fused_eligible(sa, D, false, false);
  if (fused) sa.vpre = nullptr;   // the fused kernels count data rows
  ProjectArgs pmm = pr;
  pmm.Z = nullptr;
  // bests and move in one launch (plain swarm in a tree build)
  const bool fused_steps = w.x2 != nullptr && !sc && !psearch && !scr && !p.apso;
  for (int t = 0; t <= p.T; ++t) {
    if (psearch &&
        (st = launch_ps_candidates(pa, w.dft_sel, p.ps_R, p.ps_pd, p.ps_amax, (uint32_t)t, s)))
      return st;
    if (tune && !fused && (st = tune_project(pr, s))) return st;
    if (lt && (st = lt->begin(0, s))) return st;
    if ((st = launch_project(fused ? pmm : pr, s))) return st;
    if (lt && (st = lt->end(s))) return st;
    if (tune && !fused && p.bins && (st = tune_scan_hist(sa, s))) return st;
    if (lt && (st = lt->begin(1, s))) return st;
    if (fused) {
      if ((st = launch_fused_hist(pr, sa, s))) return st;
      if (sc && (st = launch_scan_empty_nodes(sa, s))) return st;
    } else if ((st = scan(sa))) {
      return st;
    }
    if (lt && (st = lt->end(s))) return st;
    if (scr) {
      if ((st = launch_screen_select(w.loss, na, p.P, k, w.sel, s))) return st;
      if ((st = launch_screen_gather(w.x, w.sel, na, p.P, k, D, w.W32, s))) return st;
      if ((st = launch_fill_minmax(w.zmin_r, w.zmax_r, (int64_t)na * k, s))) return st;
      if (tune && (st = tune_project(prr, s))) return st;
      if (lt && (st = lt->begin(3, s))) return st;
      if ((st = launch_project(prr, s))) return st;
      if (lt && (st = lt->end(s))) return st;
      if (tune && p.bins && (st = tune_scan_hist(sar, s))) return st;
      if (lt && (st = lt->begin(4, s))) return st;
      if ((st = scan(sar))) return st;
      if (lt && (st = lt->end(s))) return st;
      if ((st = launch_screen_merge(w.sel, w.loss_r, w.split_r, w.thr_r, na, p.P, k, w.loss,
                                    w.split, w.thr, w.gloss, s)))
        return st;
    }
    if (tune) return SLM_OK;
    pa.move = t < p.T;
    // the swarm ends (or the search draws new candidates): only the global
    // best is kept
    pa.bests_only = t == p.T || psearch;
    pa.iter = (uint32_t)(t + 1);
    if (lt && (st = lt->begin(2, s))) return st;
    if (fused_steps) {
      // ping-pong: step t reads buffer t % 2 and writes the other; the last
      // (bests-only) step writes the primary record
      double *X[2] = {w.x, w.x2}, *G[2] = {w.gbest, w.gbest2}, *L[2] = {w.gbest_loss, w.gbest_loss2};
      const int cur = t & 1;
      PsoArgs pf = pa;
      pf.x_in = X[cur];
      pf.gbest_in = G[cur];
      pf.gbest_loss_in = L[cur];
      if (t < p.T) {
        pf.x = X[cur ^ 1];
        pf.gbest = G[cur ^ 1];
        pf.gbest_loss = L[cur ^ 1];
        st = launch_pso_fused(pf, s);
      } else {
        pf.x = X[cur];
        pf.gbest = w.gbest;
        pf.gbest_loss = w.gbest_loss;
        if (cur == 0) {
          pf.gbest_in = nullptr;
          pf.gbest_loss_in = nullptr;
        }
        st = launch_pso_step(pf, s);
      }
      if (st) return st;
    } else if ((st = launch_pso_step(pa, s))) {
      return st;
    }
    if (lt && (st = lt->end(s))) return st;
    if (sc) {
      if ((st = launch_search_stop(w.gbest_loss, sc->target, w.beg, w.end_act, w.done, sc->evals,
                                   na, t + 1, t == p.T, w.remaining, s)))
        return st;
      if (sc->target) {
        SLM_HIP(hipMemcpyAsync(sc->h_remaining, w.remaining, 4, hipMemcpyDeviceToHost, s));
        SLM_HIP(hipStreamSynchronize(s));
        if (*sc->h_remaining == 0) break;
      }
    }
  }
  return SLM_OK;
}

static slm_status swarm_loop_graph(const slm_tree_params &p, const TreeWS &w, const void *Xc,
                                   const void *tc, int64_t N, int32_t D, int na, int64_t vrows,
                                   hipStream_t s) {
  GraphKey key;
  key.k = {(uint64_t)(uintptr_t)Xc, (uint64_t)(uintptr_t)tc, (uint64_t)(uintptr_t)w.Z,
           (uint64_t)N, (uint64_t)D, (uint64_t)na, (uint64_t)p.P, (uint64_t)p.T,
           (uint64_t)p.bins, (uint64_t)p.crit, (uint64_t)p.K,
           (uint64_t)(uintptr_t)w.scan_ws, (uint64_t)p.precision,
           (uint64_t)(p.precision == 1 ? p.rescore_k : 0), (uint64_t)p.proposal,
           (uint64_t)(uintptr_t)(p.proposal == 1 ? p.mlp : nullptr),
           (uint64_t)(p.proposal == 1 ? p.n_seeds : 0),
           (uint64_t)(p.proposal == 1 ? p.mlp_hidden : 0),
           (uint64_t)(getenv("SLM_FUSED") && getenv("SLM_FUSED")[0] == '1'),
           (uint64_t)p.dft_top_n, (uint64_t)(uintptr_t)w.dft_ws,
           (uint64_t)(p.proposal == 2 ? p.ps_R : 0),
           (uint64_t)(uintptr_t)(p.proposal == 2 ? p.ps_pd : nullptr),
           (uint64_t)(uintptr_t)(p.proposal == 2 ? p.ps_amax : nullptr),
           (uint64_t)(uintptr_t)w.tree_off, (uint64_t)p.apso, (uint64_t)(uintptr_t)w.x2,
           (uint64_t)vrows, autotune_generation()};
  uint64_t om, c1, c2;
  std::memcpy(&om, &p.omega, 8);
  std::memcpy(&c1, &p.c1, 8);
  std::memcpy(&c2, &p.c2, 8);
  key.k.push_back(om);
  key.k.push_back(c1);
  key.k.push_back(c2);
  hipGraphExec_t exec = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) exec = it->second;
  }
  if (!exec) {
    // Capture on a private stream (the null stream cannot be captured); the
    // graph is then launched on the caller's stream.
    static thread_local hipStream_t cs = nullptr;
    if (!cs) SLM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    SLM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    set_capturing(true);
    slm_status st = swarm_loop(p, w, Xc, tc, N, D, na, vrows, cs);
    set_capturing(false);
    hipGraph_t gcap = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &gcap);
    if (st || e != hipSuccess) {
      if (gcap) (void)hipGraphDestroy(gcap);
      (void)hipGetLastError();
      if (!st) set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e));
      return st ? st : SLM_E_HIP;
    }
    const hipError_t ei = hipGraphInstantiate(&exec, gcap, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gcap);
    if (ei != hipSuccess) {
      (void)hipGetLastError();
      set_error("hipGraphInstantiate failed: %s", hipGetErrorString(ei));
      return SLM_E_HIP;
    }
    std::lock_guard<std::mutex> lk(g_graph_mu);
    g_graphs[key] = exec;
  }
  SLM_HIP(hipGraphLaunch(exec, s));
  return SLM_OK;
}

}  // namespace slm

using namespace slm;

extern "C" {

const char *slm_version(void) { return "slm-mi355x 0.1 (gfx950)"; }

const char *slm_last_error(void) { return g_err; }

slm_status slm_project(const void *X, int32_t x_dtype, int64_t N, int32_t D, const void *W,
                       int32_t w_dtype, const int64_t *row_off, int32_t n_nodes, int32_t P,
                       float *Z, int32_t z_layout, float *zmin, float *zmax, void *stream) {
  clear_error();
  SLM_CHECK(N >= 0 && N < (1ll << 31), SLM_E_SHAPE, "slm_project: N = %lld out of range",
            (long long)N);
  SLM_CHECK(D >= 1 && D <= DMAX, SLM_E_SHAPE, "slm_project: D = %d out of range", D);
  SLM_CHECK(P >= 1 && P <= PMAX, SLM_E_SHAPE, "slm_project: P = %d out of range", P);
  SLM_CHECK(n_nodes >= 0, SLM_E_SHAPE, "slm_project: n_nodes < 0");
  SLM_CHECK((x_dtype == SLM_F32 || x_dtype == SLM_BF16) &&
                (w_dtype == SLM_F32 || w_dtype == SLM_BF16) &&
                !(x_dtype == SLM_F32 && w_dtype == SLM_BF16),
            SLM_E_DTYPE, "slm_project: (X, W) must be (F32, F32), (BF16, BF16) or (BF16, F32)");
  SLM_CHECK(z_layout >= SLM_Z_ROWS && z_layout <= SLM_Z_TILED8_BF16, SLM_E_INVALID,
            "slm_project: bad Z layout %d", z_layout);
  SLM_CHECK(z_layout < SLM_Z_TILED8 || zlayout_fits(zlayout_of(z_layout, N, P), 65536),
            SLM_E_INVALID, "slm_project: N = %lld too large for SLM_Z_TILED8", (long long)N);
  if (N == 0 || n_nodes == 0) return SLM_OK;
  SLM_CHECK(X && W && row_off && Z && zmin && zmax, SLM_E_INVALID, "slm_project: NULL pointer");
  slm_status st = prepare_kernels();
  if (st) return st;
  if ((st = launch_fill_minmax(zmin, zmax, (int64_t)n_nodes * P, S(stream)))) return st;
  ProjectArgs a{};
  a.X = X; a.x_bf16 = x_dtype == SLM_BF16; a.w_bf16 = w_dtype == SLM_BF16; a.N = N; a.D = D;
  a.W = W;
  a.beg = row_off; a.end = row_off + 1; a.n_nodes = n_nodes; a.P = P;
  a.Z = Z; a.zl = zlayout_of(z_layout, N, P); a.zmin = zmin; a.zmax = zmax;
  return launch_project(a, S(stream));
}

size_t slm_split_scan_workspace(int64_t N, int32_t n_nodes, int32_t P, int32_t bins, int32_t K,
                                int32_t crit) {
  if (N <= 0 || P <= 0 || bins < 0 || bins > 256) return 256;
  return scan_workspace_bytes(N, n_nodes, P, bins, crit == SLM_MSE ? 0 : K, crit);
}

slm_status slm_split_scan(const float *Z, int32_t z_layout, const float *zmin, const float *zmax,
                          const void *target, int32_t t_dtype, int32_t K, int64_t N,
                          const int64_t *row_off, int32_t n_nodes, int32_t P, int32_t bins,
                          int32_t crit, int32_t *best_split, double *best_loss, float *threshold,
                          uint32_t *hist_out, double *sums_out, void *workspace, size_t ws_bytes,
                          void *stream) {
  clear_error();
  SLM_CHECK(N >= 0 && N < (1ll << 31), SLM_E_SHAPE, "slm_split_scan: N out of range");
  SLM_CHECK(P >= 1 && P <= PMAX, SLM_E_SHAPE, "slm_split_scan: P = %d out of range", P);
  SLM_CHECK(n_nodes >= 0, SLM_E_SHAPE, "slm_split_scan: n_nodes < 0");
  SLM_CHECK(bins == 0 || (bins >= 2 && bins <= 256), SLM_E_SHAPE,
            "slm_split_scan: bins = %d (0 or 2..256)", bins);
  SLM_CHECK(crit >= 0 && crit <= 2, SLM_E_INVALID, "slm_split_scan: bad criterion %d", crit);
  SLM_CHECK(z_layout >= SLM_Z_ROWS && z_layout <= SLM_Z_TILED8_BF16, SLM_E_INVALID,
            "slm_split_scan: bad Z layout %d", z_layout);
  SLM_CHECK(z_layout < SLM_Z_TILED8 || zlayout_fits(zlayout_of(z_layout, N, P), 65536),
            SLM_E_INVALID, "slm_split_scan: N = %lld too large for SLM_Z_TILED8", (long long)N);
  SLM_CHECK(z_layout != SLM_Z_TILED8_BF16 || (bins > 0 && crit != SLM_MSE), SLM_E_UNSUPPORTED,
            "slm_split_scan: bfloat16 Z is read by the classification histogram scan only");
  if (crit == SLM_MSE) {
    SLM_CHECK(t_dtype == SLM_F64, SLM_E_DTYPE, "slm_split_scan: SLM_MSE needs an F64 target");
    SLM_CHECK(K == 0, SLM_E_SHAPE, "slm_split_scan: K must be 0 for SLM_MSE");
  } else {
    SLM_CHECK(t_dtype == SLM_I32, SLM_E_DTYPE, "slm_split_scan: classification needs I32 labels");
    SLM_CHECK(K >= 2 && K <= 16, SLM_E_SHAPE, "slm_split_scan: K = %d not in [2, 16]", K);
  }
  if (n_nodes == 0) return SLM_OK;
  SLM_CHECK(row_off && best_split && best_loss && threshold, SLM_E_INVALID,
            "slm_split_scan: NULL pointer");
  SLM_CHECK(N == 0 || (Z && target), SLM_E_INVALID, "slm_split_scan: NULL pointer");
  if (bins) {
    SLM_CHECK(zmin && zmax, SLM_E_INVALID, "slm_split_scan: zmin/zmax required for bins > 0");
    const size_t need = scan_workspace_bytes(N, n_nodes, P, bins, K, crit);
    SLM_CHECK(workspace && ws_bytes >= need, SLM_E_NOMEM,
              "slm_split_scan: workspace of %zu bytes, %zu needed", ws_bytes, need);
    SLM_CHECK(crit == SLM_MSE || sums_out == nullptr, SLM_E_INVALID,
              "slm_split_scan: sums_out is only for SLM_MSE");
  } else {
    SLM_CHECK(hist_out == nullptr && sums_out == nullptr, SLM_E_INVALID,
              "slm_split_scan: hist_out/sums_out need histogram mode");
  }
  slm_status pst = prepare_kernels();
  if (pst) return pst;
  ScanArgs a{};
  a.Z = Z; a.zl = zlayout_of(z_layout, N, P); a.zmin = zmin; a.zmax = zmax;
  a.labels = crit == SLM_MSE ? nullptr : static_cast<const int32_t *>(target);
  a.y = crit == SLM_MSE ? static_cast<const double *>(target) : nullptr;
  a.K = K; a.N = N; a.beg = row_off; a.end = row_off + 1; a.n_nodes = n_nodes; a.P = P;
  a.bins = bins; a.crit = crit; a.best_split = best_split; a.best_loss = best_loss;
  a.threshold = threshold; a.hist_out = hist_out; a.sums_out = sums_out;
  a.ws = workspace; a.ws_bytes = ws_bytes;
  if (bins) {
    if ((pst = launch_scan_empty_nodes(a, S(stream)))) return pst;
    if (N == 0) return SLM_OK;
    return launch_scan_hist(a, S(stream));
  }
  // exact scan: node sizes decide whether the LDS sort applies
  std::vector<int64_t> off(n_nodes + 1);
  SLM_HIP(hipMemcpyAsync(off.data(), row_off, (n_nodes + 1) * 8, hipMemcpyDeviceToHost, S(stream)));
  SLM_HIP(hipStreamSynchronize(S(stream)));
  int64_t mx = 0;
  for (int j = 0; j < n_nodes; ++j) {
    int64_t b = std::min<int64_t>(std::max<int64_t>(off[j], 0), N);
    int64_t e = std::min<int64_t>(std::max<int64_t>(off[j + 1], b), N);
    mx = std::max(mx, e - b);
  }
  return launch_scan_exact(a, (int)std::min<int64_t>(mx, 1 << 30), S(stream));
}

static slm_status pso_init_impl(double *x, double *v, double *pbest, double *pbest_loss,
                                double *gbest, double *gbest_loss, int32_t *gbest_p,
                                const int32_t *node_id, int32_t n_nodes, int32_t P, int32_t D,
                                uint64_t seed, uint32_t tree, void *W_out, int32_t w_dtype,
                                const int32_t *sel, int32_t n_sel, void *stream) {
  clear_error();
  SLM_CHECK(n_nodes >= 0 && P >= 1 && P <= PMAX && D >= 1 && D <= DMAX, SLM_E_SHAPE,
            "slm_pso_init: bad sizes");
  SLM_CHECK(w_dtype == SLM_F32 || w_dtype == SLM_BF16, SLM_E_DTYPE,
            "slm_pso_init: W_out must be F32 or BF16");
  SLM_CHECK(sel == nullptr || (n_sel >= 1 && n_sel <= D), SLM_E_SHAPE,
            "slm_pso_init_subspace: n_sel = %d not in [1, D]", n_sel);
  if (n_nodes == 0) return SLM_OK;
  SLM_CHECK(x && v && pbest && pbest_loss && gbest && gbest_loss && gbest_p && node_id && W_out,
            SLM_E_INVALID, "slm_pso_init: NULL pointer");
  slm_status pst = prepare_kernels();
  if (pst) return pst;
  PsoArgs a{};
  a.x = x; a.v = v; a.pbest = pbest; a.pbest_loss = pbest_loss; a.gbest = gbest;
  a.gbest_loss = gbest_loss; a.gbest_p = gbest_p; a.node_id = node_id;
  a.n_nodes = n_nodes; a.P = P; a.D = D; a.seed = seed; a.tree = tree;
  a.W_out = W_out; a.w_bf16 = w_dtype == SLM_BF16;
  a.dim_sel = sel; a.n_sel = sel ? n_sel : 0;
  return launch_pso_init(a, S(stream));
}

slm_status slm_pso_init(double *x, double *v, double *pbest, double *pbest_loss, double *gbest,
                        double *gbest_loss, int32_t *gbest_p, const int32_t *node_id,
                        int32_t n_nodes, int32_t P, int32_t D, uint64_t seed, uint32_t tree,
                        void *W_out, int32_t w_dtype, void *stream) {
  return pso_init_impl(x, v, pbest, pbest_loss, gbest, gbest_loss, gbest_p, node_id, n_nodes, P,
                       D, seed, tree, W_out, w_dtype, nullptr, 0, stream);
}

slm_status slm_pso_init_subspace(double *x, double *v, double *pbest, double *pbest_loss,
                                 double *gbest, double *gbest_loss, int32_t *gbest_p,
                                 const int32_t *node_id, int32_t n_nodes, int32_t P, int32_t D,
                                 uint64_t seed, uint32_t tree, void *W_out, int32_t w_dtype,
                                 const int32_t *sel, int32_t n_sel, void *stream) {
  if (!sel) {
    clear_error();
    SLM_CHECK(false, SLM_E_INVALID, "slm_pso_init_subspace: sel is NULL");
  }
  return pso_init_impl(x, v, pbest, pbest_loss, gbest, gbest_loss, gbest_p, node_id, n_nodes, P,
                       D, seed, tree, W_out, w_dtype, sel, n_sel, stream);
}

size_t slm_dft_select_workspace(int64_t N, int32_t D, int32_t n_nodes, int32_t bins, int32_t K,
                                int32_t crit) {
  if (N <= 0 || D <= 0 || n_nodes < 0 || bins < 0 || bins > 256) return 256;
  return dft_workspace_bytes(N, n_nodes, D, bins, K, crit);
}

slm_status slm_dft_select(const float *X, int64_t N, int32_t D, const int64_t *row_off,
                          int32_t n_nodes, const void *target, int32_t t_dtype, int32_t K,
                          int32_t bins, int32_t crit, int32_t n, double *dft_loss, int32_t *sel,
                          void *workspace, size_t ws_bytes, void *stream) {
  clear_error();
  SLM_CHECK(N >= 0 && N < (1ll << 31) && n_nodes >= 0 && D >= 1 && D <= DFT_DMAX && n >= 1 &&
                n <= D,
            SLM_E_SHAPE, "slm_dft_select: N = %lld, D = %d, n = %d", (long long)N, D, n);
  SLM_CHECK(crit >= 0 && crit <= 2, SLM_E_INVALID, "slm_dft_select: bad criterion %d", crit);
  SLM_CHECK(bins == 0 || (bins >= 2 && bins <= 256), SLM_E_SHAPE,
            "slm_dft_select: bins = %d (0 or 2..256)", bins);
  const bool mse = crit == SLM_MSE;
  if (mse)
    SLM_CHECK(t_dtype == SLM_F64 && K == 0, SLM_E_DTYPE, "slm_dft_select: MSE needs F64 y, K = 0");
  else
    SLM_CHECK(t_dtype == SLM_I32 && K >= 2 && K <= 16, SLM_E_DTYPE,
              "slm_dft_select: classification needs I32 labels and 2 <= K <= 16");
  if (n_nodes == 0 || N == 0) return SLM_OK;
  SLM_CHECK(X && row_off && target && dft_loss && sel && workspace, SLM_E_INVALID,
            "slm_dft_select: NULL pointer");
  slm_status pst = prepare_kernels();
  if (pst) return pst;
  DftArgs da{};
  da.X = X; da.N = N; da.D = D; da.beg = row_off; da.end = row_off + 1; da.n_nodes = n_nodes;
  da.labels = mse ? nullptr : static_cast<const int32_t *>(target);
  da.y = mse ? static_cast<const double *>(target) : nullptr;
  da.K = K; da.bins = bins; da.crit = crit; da.n = n; da.loss = dft_loss; da.sel = sel;
  da.ws = workspace; da.ws_bytes = ws_bytes;
  return launch_dft_select(da, S(stream));
}

slm_status slm_ps_candidates(double *x, void *W_out, int32_t w_dtype, const int32_t *node_id,
                             int32_t n_nodes, int32_t P, int32_t D, const int32_t *ranks,
                             int32_t R, const double *pd, const int32_t *amax, uint64_t seed,
                             uint32_t tree, uint32_t t, void *stream) {
  clear_error();
  SLM_CHECK(n_nodes >= 0 && P >= 1 && P <= PMAX && D >= 1 && D <= DMAX, SLM_E_SHAPE,
            "slm_ps_candidates: bad sizes");
  SLM_CHECK(R >= 1 && R <= std::min(D, PS_RMAX), SLM_E_SHAPE,
            "slm_ps_candidates: R = %d not in [1, min(D, %d)]", R, PS_RMAX);
  SLM_CHECK(w_dtype == SLM_F32 || w_dtype == SLM_BF16, SLM_E_DTYPE,
            "slm_ps_candidates: W_out must be F32 or BF16");
  if (n_nodes == 0) return SLM_OK;
  SLM_CHECK(x && W_out && node_id && ranks && pd && amax, SLM_E_INVALID,
            "slm_ps_candidates: NULL pointer");
  slm_status pst = prepare_kernels();
  if (pst) return pst;
  PsoArgs a{};
  a.x = x; a.node_id = node_id; a.n_nodes = n_nodes; a.P = P; a.D = D; a.seed = seed;
  a.tree = tree; a.W_out = W_out; a.w_bf16 = w_dtype == SLM_BF16;
  return launch_ps_candidates(a, ranks, R, pd, amax, t, S(stream));
}

slm_status slm_ps_tables(int32_t R, double alpha0, double *pd, int32_t *amax, void *stream) {
  clear_error();
  SLM_CHECK(R >= 1 && R <= PS_RMAX, SLM_E_SHAPE, "slm_ps_tables: R = %d not in [1, %d]", R,
            PS_RMAX);
  SLM_CHECK(std::isfinite(alpha0) && alpha0 >= 1.0, SLM_E_INVALID,
            "slm_ps_tables: alpha0 must be finite and >= 1");
  SLM_CHECK(pd && amax, SLM_E_INVALID, "slm_ps_tables: NULL pointer");
  return launch_ps_tables(R, alpha0, pd, amax, S(stream));
}

slm_status slm_pso_step(double *x, double *v, double *pbest, double *pbest_loss, double *gbest,
                        double *gbest_loss, int32_t *gbest_p, const double *loss,
                        const double *gloss, const int32_t *split, const float *thr, int32_t *gbest_split,
                        float *gbest_thr, const int32_t *node_id, int32_t n_nodes, int32_t P,
                        int32_t D, double omega, double c1, double c2, uint64_t seed,
                        uint32_t tree, uint32_t iter, int32_t move, void *W_out, int32_t w_dtype,
                        void *stream) {
  clear_error();
  SLM_CHECK(n_nodes >= 0 && P >= 1 && P <= PMAX && D >= 1 && D <= DMAX, SLM_E_SHAPE,
            "slm_pso_step: bad sizes");
  SLM_CHECK(w_dtype == SLM_F32 || w_dtype == SLM_BF16, SLM_E_DTYPE,
            "slm_pso_step: W_out must be F32 or BF16");
  SLM_CHECK(std::isfinite(omega) && std::isfinite(c1) && std::isfinite(c2), SLM_E_INVALID,
            "slm_pso_step: non-finite coefficient");
  if (n_nodes == 0) return SLM_OK;
  SLM_CHECK(x && v && pbest && pbest_loss && gbest && gbest_loss && gbest_p && loss && node_id,
            SLM_E_INVALID, "slm_pso_step: NULL pointer");
  SLM_CHECK(!move || W_out, SLM_E_INVALID, "slm_pso_step: W_out required when moving");
  SLM_CHECK((split == nullptr) == (gbest_split == nullptr) &&
                (thr == nullptr) == (gbest_thr == nullptr),
            SLM_E_INVALID, "slm_pso_step: split/gbest_split and thr/gbest_thr go in pairs");
  slm_status pst = prepare_kernels();
  if (pst) return pst;
  PsoArgs a{};
  a.x = x; a.v = v; a.pbest = pbest; a.pbest_loss = pbest_loss; a.gbest = gbest;
  a.gbest_loss = gbest_loss; a.gbest_p = gbest_p; a.loss = loss; a.gloss = gloss;
  a.split = split; a.thr = thr;
  a.gbest_split = gbest_split; a.gbest_thr = gbest_thr; a.node_id = node_id;
  a.n_nodes = n_nodes; a.P = P; a.D = D; a.omega = omega; a.c1 = c1; a.c2 = c2;
  a.seed = seed; a.tree = tree; a.iter = iter; a.move = move;
  a.W_out = W_out; a.w_bf16 = w_dtype == SLM_BF16;
  return launch_pso_step(a, S(stream));
}

size_t slm_apso_workspace(int32_t n_nodes, int32_t P) {
  return std::max<size_t>(256, apso_part_bytes(n_nodes, P));
}

slm_status slm_apso_step(double *x, double *v, double *pbest, double *pbest_loss, double *gbest,
                         double *gbest_loss, int32_t *gbest_p, const double *loss,
                         const int32_t *node_id, int32_t n_nodes, int32_t P, int32_t D,
                         uint64_t seed, uint32_t tree, uint32_t iter, uint32_t T, int32_t *state,
                         double *par, double *dist, double *f, int32_t *worst, double *elite,
                         const int32_t *sel, int32_t n_sel, void *workspace, size_t ws_bytes,
                         void *W_out, int32_t w_dtype, void *stream) {
  clear_error();
  SLM_CHECK((sel == nullptr) == (n_sel == 0) && n_sel >= 0 && n_sel <= D, SLM_E_INVALID,
            "slm_apso_step: sel and n_sel (1..D) go together");
  SLM_CHECK(n_nodes >= 0 && P >= 2 && P <= PMAX && D >= 1 && D <= DMAX, SLM_E_SHAPE,
            "slm_apso_step: bad sizes (2 <= P <= %d, 1 <= D <= %d)", PMAX, DMAX);
  SLM_CHECK(w_dtype == SLM_F32 || w_dtype == SLM_BF16, SLM_E_DTYPE,
            "slm_apso_step: W_out must be F32 or BF16");
  SLM_CHECK(iter >= 1 && T >= 1, SLM_E_INVALID, "slm_apso_step: iter and T must be >= 1");
  if (n_nodes == 0) return SLM_OK;
  SLM_CHECK(x && v && pbest && pbest_loss && gbest && gbest_loss && gbest_p && loss && node_id &&
                state && par && dist && f && worst && elite && workspace && W_out,
            SLM_E_INVALID, "slm_apso_step: NULL pointer");
  SLM_CHECK(ws_bytes >= apso_part_bytes(n_nodes, P), SLM_E_NOMEM,
            "slm_apso_step: workspace of %zu bytes too small", ws_bytes);
  slm_status pst = prepare_kernels();
  if (pst) return pst;
  PsoArgs a{};
  a.x = x; a.v = v; a.pbest = pbest; a.pbest_loss = pbest_loss; a.gbest = gbest;
  a.gbest_loss = gbest_loss; a.gbest_p = gbest_p; a.loss = loss; a.node_id = node_id;
  a.n_nodes = n_nodes; a.P = P; a.D = D; a.seed = seed; a.tree = tree; a.iter = iter;
  a.move = 1; a.W_out = W_out; a.w_bf16 = w_dtype == SLM_BF16;
  a.apso_state = state; a.apso_par = par; a.apso_dist = dist; a.apso_f = f;
  a.apso_worst = worst; a.apso_elite = elite;
  a.apso_part = static_cast<double *>(workspace); a.apso_T = T;
  a.apso_sel = sel; a.apso_n_sel = n_sel;
  return launch_pso_step(a, S(stream));
}

slm_status slm_screen_select(const double *loss, int32_t n_nodes, int32_t P, int32_t k,
                             int32_t *sel, void *stream) {
  clear_error();
  SLM_CHECK(n_nodes >= 0 && P >= 1 && P <= PMAX && k >= 1 && k <= P, SLM_E_SHAPE,
            "slm_screen_select: need n_nodes >= 0 and 1 <= k <= P <= %d", PMAX);
  if (n_nodes == 0) return SLM_OK;
  SLM_CHECK(loss && sel, SLM_E_INVALID, "slm_screen_select: NULL pointer");
  return launch_screen_select(loss, n_nodes, P, k, sel, S(stream));
}

slm_status slm_screen_gather(const double *x, const int32_t *sel, int32_t n_nodes, int32_t P,
                             int32_t k, int32_t D, float *W32, void *stream) {
  clear_error();
  SLM_CHECK(n_nodes >= 0 && P >= 1 && P <= PMAX && k >= 1 && k <= P && D >= 1 && D <= DMAX,
            SLM_E_SHAPE, "slm_screen_gather: bad sizes");
  if (n_nodes == 0) return SLM_OK;
  SLM_CHECK(x && sel && W32, SLM_E_INVALID, "slm_screen_gather: NULL pointer");
  return launch_screen_gather(x, sel, n_nodes, P, k, D, W32, S(stream));
}

slm_status slm_screen_merge(const int32_t *sel, const double *loss_r, const int32_t *split_r,
                            const float *thr_r, int32_t n_nodes, int32_t P, int32_t k,
                            double *loss, int32_t *split, float *thr, double *gloss,
                            void *stream) {
  clear_error();
  SLM_CHECK(n_nodes >= 0 && P >= 1 && P <= PMAX && k >= 1 && k <= P, SLM_E_SHAPE,
            "slm_screen_merge: bad sizes");
  if (n_nodes == 0) return SLM_OK;
  SLM_CHECK(sel && loss_r && split_r && thr_r && loss && split && thr && gloss, SLM_E_INVALID,
            "slm_screen_merge: NULL pointer");
  return launch_screen_merge(sel, loss_r, split_r, thr_r, n_nodes, P, k, loss, split, thr, gloss,
                             S(stream));
}

// ---------------------------------------------------------------- fused evaluation
slm_status slm_evaluate(const float *X, int64_t N, int32_t D, const float *W,
                        const int64_t *row_off, int32_t n_nodes, int32_t P,
                        const int32_t *labels, int32_t K, int32_t bins, int32_t crit, float *zmin,
                        float *zmax, int32_t *best_split, double *best_loss, float *threshold,
                        void *workspace, size_t ws_bytes, void *stream) {
  clear_error();
  SLM_CHECK(N >= 0 && N < (1ll << 31), SLM_E_SHAPE, "slm_evaluate: N out of range");
  SLM_CHECK(P >= 1 && P <= PMAX && n_nodes >= 0 && D >= 1 && D <= DMAX, SLM_E_SHAPE,
            "slm_evaluate: bad sizes");
  SLM_CHECK(bins >= 2 && bins <= 256, SLM_E_SHAPE, "slm_evaluate: bins = %d not in [2, 256]", bins);
  SLM_CHECK(crit == SLM_GINI || crit == SLM_ENTROPY, SLM_E_UNSUPPORTED,
            "slm_evaluate: Gini or entropy only");
  SLM_CHECK(D <= 64 && K >= 2 && K <= 4, SLM_E_UNSUPPORTED,
            "slm_evaluate: the fused evaluation takes D <= 64 and 2 <= K <= 4 (D = %d, K = %d)",
            D, K);
  if (N == 0 || n_nodes == 0) return SLM_OK;
  SLM_CHECK(X && W && row_off && labels && zmin && zmax && best_split && best_loss && threshold &&
                workspace,
            SLM_E_INVALID, "slm_evaluate: NULL pointer");
  const size_t need = scan_workspace_bytes(N, n_nodes, P, bins, K, crit);
  SLM_CHECK(ws_bytes >= need, SLM_E_NOMEM, "slm_evaluate: workspace of %zu bytes, %zu needed",
            ws_bytes, need);
  hipStream_t s = S(stream);
  slm_status st = launch_fill_minmax(zmin, zmax, (int64_t)n_nodes * P, s);
  if (st) return st;
  ProjectArgs pr{};
  pr.X = X; pr.x_bf16 = 0; pr.w_bf16 = 0; pr.N = N; pr.D = D; pr.W = W; pr.beg = row_off;
  pr.end = row_off + 1; pr.n_nodes = n_nodes; pr.P = P; pr.Z = nullptr; pr.zmin = zmin;
  pr.zmax = zmax; pr.zl = zlayout_of(1, N, P);
  ScanArgs sa{};
  sa.Z = nullptr; sa.zl = pr.zl; sa.zmin = zmin; sa.zmax = zmax; sa.labels = labels; sa.y = nullptr;
  sa.K = K; sa.N = N; sa.beg = row_off; sa.end = row_off + 1; sa.n_nodes = n_nodes; sa.P = P;
  sa.bins = bins; sa.crit = crit; sa.best_split = best_split; sa.best_loss = best_loss;
  sa.threshold = threshold; sa.ws = workspace; sa.ws_bytes = ws_bytes;
  if ((st = launch_fused_eval(pr, sa, s))) return st;
  return launch_scan_empty_nodes(sa, s);
}

// ---------------------------------------------------------------- node-batch search
size_t slm_search_nodes_workspace(const slm_tree_params *prm, int64_t N, int32_t D,
                                  int32_t n_nodes) {
  if (check_tree_params(prm, N, D) != SLM_OK || n_nodes < 1) return 0;
  return carve(*prm, N, D, nullptr, n_nodes, prm->proposal == 1).total;
}

slm_status slm_search_nodes(const void *X, int32_t x_dtype, int64_t N, int32_t D,
                            const void *target, int32_t t_dtype, const int64_t *row_off,
                            const int32_t *node_id, int32_t n_nodes, const slm_tree_params *prm,
                            const double *target_loss, double *gbest, double *gbest_loss,
                            int32_t *gbest_split, float *gbest_thr, int32_t *evals,
                            void *workspace, size_t ws_bytes, void *stream) {
  clear_error();
  slm_status st = check_tree_params(prm, N, D);
  if (st) return st;
  const slm_tree_params &p = *prm;
  const bool mse = p.crit == SLM_MSE;
  SLM_CHECK(n_nodes >= 1 && n_nodes <= (1 << 24), SLM_E_SHAPE,
            "slm_search_nodes: n_nodes = %d out of range", n_nodes);
  SLM_CHECK(x_dtype == (p.precision == 1 ? SLM_BF16 : SLM_F32), SLM_E_DTYPE,
            "slm_search_nodes: X must be F32 (precision 0) or BF16 (precision 1)");
  SLM_CHECK(t_dtype == (mse ? SLM_F64 : SLM_I32), SLM_E_DTYPE,
            "slm_search_nodes: target dtype does not match the criterion");
  SLM_CHECK(X && target && row_off && node_id && gbest && gbest_loss && gbest_split && gbest_thr &&
                evals && workspace,
            SLM_E_INVALID, "slm_search_nodes: NULL pointer");
  const TreeWS w = carve(p, N, D, workspace, n_nodes, p.proposal == 1);
  SLM_CHECK(ws_bytes >= w.total, SLM_E_NOMEM,
            "slm_search_nodes: workspace of %zu bytes, %zu needed", ws_bytes, w.total);
  if (p.bins == 0) {
    std::vector<int64_t> ho((size_t)n_nodes + 1);
    SLM_HIP(hipMemcpy(ho.data(), row_off, ho.size() * 8, hipMemcpyDeviceToHost));
    for (int j = 0; j < n_nodes; ++j)
      SLM_CHECK(ho[j + 1] - ho[j] <= EXACT_ROWS, SLM_E_UNSUPPORTED,
                "slm_search_nodes: the exact scan takes nodes of at most %d rows", EXACT_ROWS);
  }
  if ((st = prepare_kernels())) return st;
  hipStream_t s = S(stream);
  const int Kc = mse ? 1 : p.K;
  SLM_HIP(hipMemsetAsync(w.scan_ws, 0, w.scan_ws_bytes, s));
  if (w.dft_ws) SLM_HIP(hipMemsetAsync(w.dft_ws, 0, w.dft_ws_bytes, s));
  if (w.stat_sums)
    SLM_HIP(hipMemsetAsync(w.stat_sums, 0, stats_workspace_bytes(n_nodes, D, Kc), s));
  const uint64_t seed_tree[2] = {p.seed, (uint64_t)p.tree};
  SLM_HIP(hipMemcpyAsync(w.seed_tree, seed_tree, 16, hipMemcpyHostToDevice, s));
  SLM_HIP(hipMemcpyAsync(w.beg, row_off, (size_t)n_nodes * 8, hipMemcpyDeviceToDevice, s));
  SLM_HIP(hipMemcpyAsync(w.end, row_off + 1, (size_t)n_nodes * 8, hipMemcpyDeviceToDevice, s));
  SLM_HIP(hipMemcpyAsync(w.end_act, row_off + 1, (size_t)n_nodes * 8, hipMemcpyDeviceToDevice, s));
  SLM_HIP(hipMemcpyAsync(w.node_id, node_id, (size_t)n_nodes * 4, hipMemcpyDeviceToDevice, s));
  SLM_HIP(hipMemsetAsync(w.done, 0, (size_t)n_nodes * 4, s));
  uint32_t h_remaining = 0;
  const SearchCtl sc{target_loss, evals, &h_remaining};
  if ((st = swarm_loop(p, w, X, target, N, D, n_nodes, 0, s, nullptr, &sc))) return st;
  SLM_HIP(hipMemcpyAsync(gbest, w.gbest, (size_t)n_nodes * D * 8, hipMemcpyDeviceToDevice, s));
  SLM_HIP(hipMemcpyAsync(gbest_loss, w.gbest_loss, (size_t)n_nodes * 8, hipMemcpyDeviceToDevice, s));
  SLM_HIP(hipMemcpyAsync(gbest_split, w.gbest_split, (size_t)n_nodes * 4, hipMemcpyDeviceToDevice,
                         s));
  SLM_HIP(hipMemcpyAsync(gbest_thr, w.gbest_thr, (size_t)n_nodes * 4, hipMemcpyDeviceToDevice, s));
  SLM_HIP(hipStreamSynchronize(s));
  return SLM_OK;
}

// ---------------------------------------------------------------- learned proposal
size_t slm_node_stats_workspace(int32_t n_nodes, int32_t D, int32_t K) {
  if (n_nodes < 0 || D < 1 || K < 1) return 256;
  return stats_workspace_bytes(n_nodes, D, K);
}

slm_status slm_node_stats(const void *X, int32_t x_dtype, int64_t N, int32_t D,
                          const int32_t *labels, int32_t K, const int64_t *row_off,
                          int32_t n_nodes, float *stats, float *sigma, void *workspace,
                          size_t ws_bytes, void *stream) {
  clear_error();
  SLM_CHECK(N >= 0 && N < (1ll << 31) && D >= 1 && D <= DMAX && n_nodes >= 0, SLM_E_SHAPE,
            "slm_node_stats: bad sizes");
  SLM_CHECK(K >= 1 && K <= 16 && K * D <= 4096, SLM_E_SHAPE,
            "slm_node_stats: need 1 <= K <= 16 and K * D <= 4096");
  SLM_CHECK(x_dtype == SLM_F32 || x_dtype == SLM_BF16, SLM_E_DTYPE,
            "slm_node_stats: X must be F32 or BF16");
  if (n_nodes == 0) return SLM_OK;
  SLM_CHECK(row_off && stats && sigma && workspace && (N == 0 || (X && labels)), SLM_E_INVALID,
            "slm_node_stats: NULL pointer");
  const size_t need = stats_workspace_bytes(n_nodes, D, K);
  SLM_CHECK(ws_bytes >= need, SLM_E_NOMEM, "slm_node_stats: workspace of %zu bytes, %zu needed",
            ws_bytes, need);
  StatsArgs a{};
  a.X = X; a.x_bf16 = x_dtype == SLM_BF16; a.N = N; a.D = D; a.labels = labels; a.K = K;
  a.beg = row_off; a.end = row_off + 1; a.n_nodes = n_nodes;
  a.sums = static_cast<double *>(workspace);
  a.counts = reinterpret_cast<uint32_t *>(static_cast<char *>(workspace) +
                                          ((size_t)n_nodes * K * D * 2 * 8 + 255) / 256 * 256);
  a.stats = stats; a.sigma = sigma;
  return launch_node_stats_full(a, S(stream));
}

int64_t slm_mlp_param_count(int32_t n_in, int32_t hidden, int32_t n_out) {
  if (n_in < 1 || hidden < 1 || n_out < 1) return 0;
  return mlp_param_count(n_in, hidden, n_out);
}

static slm_status check_mlp(int32_t n_in, int32_t hidden, int32_t n_out, int32_t batch,
                            const char *who) {
  SLM_CHECK(n_in >= 1 && n_in <= (1 << 20) && hidden >= 1 && hidden <= 4096 && n_out >= 1 &&
                n_out <= (1 << 20) && batch >= 0 && batch <= (1 << 21),
            SLM_E_SHAPE, "%s: bad sizes", who);
  SLM_CHECK((int64_t)batch * n_out < (1ll << 40), SLM_E_SHAPE, "%s: batch too large", who);
  return SLM_OK;
}

slm_status slm_mlp_forward(const float *params, int32_t n_in, int32_t hidden, int32_t n_out,
                           const float *in, int32_t batch, int32_t bf16, float *out, float *cache,
                           void *stream) {
  clear_error();
  slm_status st = check_mlp(n_in, hidden, n_out, batch, "slm_mlp_forward");
  if (st) return st;
  if (batch == 0) return SLM_OK;
  SLM_CHECK(params && in && out && cache, SLM_E_INVALID, "slm_mlp_forward: NULL pointer");
  return launch_mlp_forward(params, n_in, hidden, n_out, in, batch, bf16 != 0, out, cache,
                            S(stream));
}

slm_status slm_mlp_backward(const float *params, int32_t n_in, int32_t hidden, int32_t n_out,
                            const float *in, int32_t batch, const float *cache,
                            const float *d_out, float *grads, float *work, void *stream) {
  clear_error();
  slm_status st = check_mlp(n_in, hidden, n_out, batch, "slm_mlp_backward");
  if (st) return st;
  SLM_CHECK(batch >= 1, SLM_E_SHAPE, "slm_mlp_backward: empty batch");
  SLM_CHECK(params && in && cache && d_out && grads && work, SLM_E_INVALID,
            "slm_mlp_backward: NULL pointer");
  return launch_mlp_backward(params, n_in, hidden, n_out, in, batch, cache, d_out, grads, work,
                             S(stream));
}

slm_status slm_wta_loss(const float *out, const float *target, int32_t batch, int32_t M,
                        int32_t D, float eps, float scale, float *loss, float *d_out,
                        void *stream) {
  clear_error();
  SLM_CHECK(batch >= 0 && M >= 1 && M <= 256 && D >= 1 && D <= DMAX, SLM_E_SHAPE,
            "slm_wta_loss: need 1 <= M <= 256, 1 <= D <= %d", DMAX);
  SLM_CHECK(eps >= 0.f && eps <= 1.f, SLM_E_INVALID, "slm_wta_loss: eps not in [0, 1]");
  if (batch == 0) return SLM_OK;
  SLM_CHECK(out && target && loss && d_out, SLM_E_INVALID, "slm_wta_loss: NULL pointer");
  return launch_wta(out, target, batch, M, D, eps, scale, loss, d_out, S(stream));
}

slm_status slm_proposal_targets(const float *g, const float *sigma, int32_t n, int32_t D,
                                float *t, void *stream) {
  clear_error();
  SLM_CHECK(n >= 0 && D >= 1 && D <= DMAX, SLM_E_SHAPE, "slm_proposal_targets: bad sizes");
  if (n == 0) return SLM_OK;
  SLM_CHECK(g && sigma && t, SLM_E_INVALID, "slm_proposal_targets: NULL pointer");
  return launch_targets(g, sigma, n, D, t, S(stream));
}

slm_status slm_adam_step(float *params, const float *grads, float *m, float *v, int64_t n,
                         float lr, float b1, float b2, float eps, int32_t step, void *stream) {
  clear_error();
  SLM_CHECK(n >= 0 && step >= 1, SLM_E_SHAPE, "slm_adam_step: need n >= 0 and step >= 1");
  SLM_CHECK(b1 >= 0.f && b1 < 1.f && b2 >= 0.f && b2 < 1.f && eps >= 0.f, SLM_E_INVALID,
            "slm_adam_step: bad coefficients");
  if (n == 0) return SLM_OK;
  SLM_CHECK(params && grads && m && v, SLM_E_INVALID, "slm_adam_step: NULL pointer");
  return launch_adam(params, grads, m, v, n, lr, b1, b2, eps, step, S(stream));
}

slm_status slm_proposal_seeds(const float *out, const float *sigma, int32_t n_nodes, int32_t M,
                              int32_t D, int32_t P, double *x, double *pbest, void *W_out,
                              int32_t w_dtype, void *stream) {
  clear_error();
  SLM_CHECK(n_nodes >= 0 && M >= 1 && M <= 4096 && D >= 1 && D <= DMAX && P >= 1 && P <= PMAX,
            SLM_E_SHAPE, "slm_proposal_seeds: bad sizes");
  SLM_CHECK(w_dtype == SLM_F32 || w_dtype == SLM_BF16, SLM_E_DTYPE,
            "slm_proposal_seeds: W_out must be F32 or BF16");
  if (n_nodes == 0) return SLM_OK;
  SLM_CHECK(out && sigma && x && pbest && W_out, SLM_E_INVALID, "slm_proposal_seeds: NULL pointer");
  return launch_seeds(out, sigma, n_nodes, M, D, P, x, pbest, W_out, w_dtype == SLM_BF16,
                      S(stream));
}

slm_status slm_predict(const float *w, const float *thr, const int32_t *left,
                       const int32_t *right, int32_t n_tree, int32_t D, const float *X, int64_t N,
                       int32_t *leaf_out, void *stream) {
  clear_error();
  SLM_CHECK(n_tree >= 1 && D >= 1 && D <= DMAX && N >= 0 && N < (1ll << 31), SLM_E_SHAPE,
            "slm_predict: bad sizes");
  if (N == 0) return SLM_OK;
  SLM_CHECK(w && thr && left && right && X && leaf_out, SLM_E_INVALID, "slm_predict: NULL pointer");
  return launch_predict(w, thr, left, right, n_tree, D, X, N, leaf_out, S(stream));
}

// node statistics are kept for classification trees (the learned start, and
// the optional per-node statistics output)
static bool tree_stats(const slm_tree_params &p, int32_t D) {
  return p.crit != SLM_MSE && p.K * D <= 4096;
}

// Breadth-first growth of one tree per root: root r owns rows
// roots[r].first .. roots[r].second - 1 of X / target and its draws use tree
// id p.tree + r.  Every depth searches the frontier nodes of all trees in one
// swarm loop.  Nodes are written to out from index base on (children indices
// are global); tree_of (optional) receives each node's root index.  ss[0..1]
// accumulate the sample-split counts.
static slm_status grow_impl(const void *X, int64_t N, int32_t D, const void *target,
                            const slm_tree_params &p, const TreeWS &w,
                            const std::vector<std::pair<int64_t, int64_t>> &roots, int base,
                            slm_tree_out *out, int32_t *tree_of, int64_t *ss, hipStream_t s) {
  slm_status st;
  const bool mse = p.crit == SLM_MSE;
  const bool want_stats = out->stats != nullptr;
  const int KD1 = (p.K + 1) * D;
  const int n_roots = (int)roots.size();
  std::vector<float> hst, hsg;
  const int Kc = mse ? 1 : p.K;
  const int64_t F = max_active(p, N, n_roots);
  double *timing = out->timing;
  Timer tm_swarm, tm_part;
  const bool prof = p.profile && timing;
  LaunchTimes lt;

  // scan accumulators start (and stay) zero; RNG key and tree id on the
  // device; root statistics
  SLM_HIP(hipMemsetAsync(w.scan_ws, 0, w.scan_ws_bytes, s));
  if (w.dft_ws) SLM_HIP(hipMemsetAsync(w.dft_ws, 0, w.dft_ws_bytes, s));
  if (w.stat_sums)
    SLM_HIP(hipMemsetAsync(w.stat_sums, 0, stats_workspace_bytes((int)F, D, Kc), s));
  const uint64_t seed_tree[2] = {p.seed, (uint64_t)p.tree};
  SLM_HIP(hipMemcpyAsync(w.seed_tree, seed_tree, 16, hipMemcpyHostToDevice, s));
  // pinned host arrays of the per-depth transfers (the previous build's
  // transfers have completed: every build ends with a synchronisation)
  // The depth's upload (row ranges, heap ids, tree indices) and the swarm's
  // results (global bests, losses, thresholds) are each one contiguous span
  // of the workspace; their host images mirror the spans, so each moves in
  // one copy (the results span only while it is small).
  char *const up0 = reinterpret_cast<char *>(w.beg);
  const size_t up_span = reinterpret_cast<char *>(w.vpre + F + 1) - up0;
  char *const dn0 = reinterpret_cast<char *>(w.gbest);
  const size_t dn_span = reinterpret_cast<char *>(w.gbest_thr + F) - dn0;
  {
    const size_t F2 = (size_t)2 * F;
    const size_t need = pinned_bytes(up_span, 1) + pinned_bytes(dn_span, 1) + pinned_bytes(F, 8) +
                        pinned_bytes(F, 4) + pinned_bytes((size_t)F * D, 4) +
                        pinned_bytes(F2 * Kc, 4) + pinned_bytes(F2, 4) + 4 * pinned_bytes(F2, 8) +
                        64;
    if ((st = pinned_begin(need))) return st;
  }
  char *const hup = pinned_take<char>(up_span), *const hdn = pinned_take<char>(dn_span);
  int64_t *hb = reinterpret_cast<int64_t *>(hup);
  int64_t *he = reinterpret_cast<int64_t *>(hup + (reinterpret_cast<char *>(w.end) - up0));
  int32_t *hid = reinterpret_cast<int32_t *>(hup + (reinterpret_cast<char *>(w.node_id) - up0));
  uint32_t *htr =
      w.tree_off ? reinterpret_cast<uint32_t *>(hup + (reinterpret_cast<char *>(w.tree_off) - up0))
                 : nullptr;
  int64_t *hvp = reinterpret_cast<int64_t *>(hup + (reinterpret_cast<char *>(w.vpre) - up0));
  double *hgb = reinterpret_cast<double *>(hdn);
  double *hgl = reinterpret_cast<double *>(hdn + (reinterpret_cast<char *>(w.gbest_loss) - dn0));
  float *hgt = reinterpret_cast<float *>(hdn + (reinterpret_cast<char *>(w.gbest_thr) - dn0));
  int64_t *hnl = pinned_take<int64_t>(F);
  int32_t *hsplit = pinned_take<int32_t>(F);
  float *hgw = pinned_take<float>((size_t)F * D);
  StatsHost sh;
  sh.counts = pinned_take<uint32_t>((size_t)2 * F * Kc);
  sh.cnt = pinned_take<uint32_t>((size_t)2 * F);
  sh.s1 = pinned_take<double>((size_t)2 * F);
  sh.s2 = pinned_take<double>((size_t)2 * F);
  sh.ymin = pinned_take<unsigned long long>((size_t)2 * F);
  sh.ymax = pinned_take<unsigned long long>((size_t)2 * F);
  for (int r = 0; r < n_roots; ++r) {
    hb[r] = roots[r].first;
    he[r] = roots[r].second;
  }
  SLM_HIP(hipMemcpyAsync(w.beg, hb, n_roots * 8, hipMemcpyHostToDevice, s));
  SLM_HIP(hipMemcpyAsync(w.end, he, n_roots * 8, hipMemcpyHostToDevice, s));
  if ((st = clear_stats(w, n_roots, p.crit, Kc, s))) return st;
  if ((st = launch_node_stats(w.beg, w.end, n_roots, N, mse ? nullptr : (const int32_t *)target,
                              mse ? (const double *)target : nullptr, Kc, w.st, s)))
    return st;
  if ((st = read_stats(w, n_roots, p.crit, Kc, sh, s))) return st;
  SLM_HIP(hipStreamSynchronize(s));

  int nn = base;
  auto new_node = [&](int depth, int heap, int stat_i, int64_t b, int64_t e, uint32_t tree,
                      HNode *hn) -> bool {
    if (nn >= out->max_nodes) return false;
    const int i = nn++;
    double imp;
    bool impure;
    int64_t cnt;
    summarize(sh, stat_i, p.crit, Kc, &imp, &impure, out->leaf + (size_t)i * Kc, &cnt);
    out->n[i] = e - b;
    out->impurity[i] = imp;
    out->split_loss[i] = INFINITY;
    out->thr[i] = INFINITY;
    out->left[i] = -1;
    out->right[i] = -1;
    out->depth[i] = depth;
    out->heap[i] = heap;
    if (tree_of) tree_of[i] = (int32_t)tree;
    std::fill(out->w + (size_t)i * D, out->w + (size_t)(i + 1) * D, 0.0f);
    if (out->stats)
      std::fill(out->stats + (size_t)i * KD1, out->stats + (size_t)(i + 1) * KD1, 0.0f);
    if (out->stats && out->sigma)
      std::fill(out->sigma + (size_t)i * D, out->sigma + (size_t)(i + 1) * D, 0.0f);
    *hn = HNode{i, b, e, depth, heap, imp, impure, tree};
    return true;
  };
  std::vector<HNode> frontier(n_roots);
  for (int r = 0; r < n_roots; ++r)
    SLM_CHECK(new_node(0, 0, r, roots[r].first, roots[r].second, (uint32_t)r, &frontier[r]),
              SLM_E_SHAPE, "grow: max_nodes = %d holds fewer than the %d roots", out->max_nodes,
              n_roots);

  const void *Xc = X;
  const void *tc = target;
  void *Xbuf[2] = {w.Xa, w.Xb};
  void *tbuf[2] = {w.ta, w.tb};
  int nb = 0;

  while (!frontier.empty()) {
    std::vector<HNode> active;
    for (const HNode &f : frontier)
      if (f.depth < p.max_depth && f.end - f.beg >= p.min_node && f.impure) active.push_back(f);
    if (active.empty()) break;
    const int na = (int)active.size();
    SLM_CHECK(na <= F, SLM_E_SHAPE, "grow: frontier of %d nodes exceeds %lld", na,
              (long long)F);
    hvp[0] = 0;
    for (int j = 0; j < na; ++j) {
      hvp[j + 1] = hvp[j] + (active[j].end - active[j].beg);
      hb[j] = active[j].beg;
      he[j] = active[j].end;
      hid[j] = active[j].heap;
      if (htr) htr[j] = active[j].tree;
      ss[0] += (active[j].end - active[j].beg) * (int64_t)p.P * (p.T + 1);
      if (p.precision == 1)
        ss[1] += (active[j].end - active[j].beg) * (int64_t)p.rescore_k * (p.T + 1);
    }
    // The histogram's chunk plan is made for the depth's rows rounded up to
    // a multiple of an eighth of N / 2^k (the smallest such power at or
    // above them): captured swarm loops are keyed by it, and the rounding
    // keeps trees of one shape on a few graphs (measured against N / 2^k
    // alone: 2.45 -> 2.47e11 sample-splits/s, 30-tree forest 217 -> 214 ms).
    int64_t rows_q = N;
    while (rows_q > 1 && (rows_q >> 1) >= hvp[na]) rows_q >>= 1;
    if (rows_q >= 8) {
      const int64_t step = rows_q / 8;
      rows_q = std::min(rows_q, (hvp[na] + step - 1) / step * step);
    }
    {
      // one copy: beg, end, node_id (and tree_off) up to entry na, and the
      // row prefix up to entry na + 1
      char *last = reinterpret_cast<char *>(w.vpre + na + 1);
      SLM_HIP(hipMemcpyAsync(up0, hup, (size_t)(last - up0), hipMemcpyHostToDevice, s));
    }
    if (want_stats && p.proposal != 1) {
      StatsArgs sa{};
      sa.X = Xc; sa.x_bf16 = p.precision == 1; sa.N = N; sa.D = D;
      sa.labels = static_cast<const int32_t *>(tc); sa.K = p.K; sa.beg = w.beg; sa.end = w.end;
      sa.n_nodes = na; sa.sums = w.stat_sums; sa.counts = w.stat_counts; sa.stats = w.stats;
      sa.sigma = w.sigma;
      if ((st = launch_node_stats_full(sa, s))) return st;
    }
    if (autotune_mode() == 2 && !prof) {
      // measure the plans of this depth's launch shapes that have none yet
      if ((st = swarm_loop(p, w, Xc, tc, N, D, na, rows_q, s, nullptr, nullptr, true))) return st;
      SLM_HIP(hipStreamSynchronize(s));
    }
    if ((st = tm_swarm.start(timing ? &timing[1] : nullptr, s))) return st;
    if (prof)
      st = swarm_loop(p, w, Xc, tc, N, D, na, rows_q, s, &lt);
    else
      st = p.use_graph ? swarm_loop_graph(p, w, Xc, tc, N, D, na, rows_q, s)
                       : swarm_loop(p, w, Xc, tc, N, D, na, rows_q, s);
    if (st) return st;
    if ((st = tm_swarm.stop(s))) return st;
    if (prof) {
      SLM_HIP(hipStreamSynchronize(s));
      // kinds: 0 projection, 1 scan, 2 swarm step, 3 re-scoring
      // projection, 4 re-scoring scan (screened evaluations)
      double acc[5] = {0, 0, 0, 0, 0}, cnt[5] = {0, 0, 0, 0, 0};
      if ((st = lt.collect(acc, cnt))) return st;
      timing[3] += acc[0];
      timing[4] += acc[1];
      timing[5] += acc[2];
      timing[6] += cnt[0];
      timing[7] += cnt[1];
      timing[8] += acc[3];
      timing[9] += acc[4];
      timing[10] += cnt[3];
      timing[11] += cnt[4];
    }
    if (dn_span <= ((size_t)512 << 10)) {
      const size_t n_dn = reinterpret_cast<char *>(w.gbest_thr + na) - dn0;
      SLM_HIP(hipMemcpyAsync(hdn, dn0, n_dn, hipMemcpyDeviceToHost, s));
    } else {
      SLM_HIP(hipMemcpyAsync(hgl, w.gbest_loss, na * 8, hipMemcpyDeviceToHost, s));
      SLM_HIP(hipMemcpyAsync(hgt, w.gbest_thr, na * 4, hipMemcpyDeviceToHost, s));
      SLM_HIP(hipMemcpyAsync(hgb, w.gbest, (size_t)na * D * 8, hipMemcpyDeviceToHost, s));
    }
    if (want_stats) {
      hst.resize((size_t)na * KD1);
      hsg.resize((size_t)na * D);
      SLM_HIP(hipMemcpyAsync(hst.data(), w.stats, hst.size() * 4, hipMemcpyDeviceToHost, s));
      SLM_HIP(hipMemcpyAsync(hsg.data(), w.sigma, hsg.size() * 4, hipMemcpyDeviceToHost, s));
    }
    SLM_HIP(hipStreamSynchronize(s));
    if (want_stats) {
      for (int j = 0; j < na; ++j) {
        const int i = active[j].idx;
        std::copy(hst.begin() + (size_t)j * KD1, hst.begin() + (size_t)(j + 1) * KD1,
                  out->stats + (size_t)i * KD1);
        if (out->sigma)
          std::copy(hsg.begin() + (size_t)j * D, hsg.begin() + (size_t)(j + 1) * D,
                    out->sigma + (size_t)i * D);
      }
    }
    int nsplit = 0;
    for (int j = 0; j < na; ++j) {
      out->split_loss[active[j].idx] = hgl[j];
      hsplit[j] = hgl[j] < active[j].impurity ? 1 : 0;
      nsplit += hsplit[j];
      for (int d = 0; d < D; ++d) hgw[(size_t)j * D + d] = (float)hgb[(size_t)j * D + d];
    }
    if (nsplit == 0) break;
    if ((st = tm_part.start(timing ? &timing[2] : nullptr, s))) return st;
    SLM_HIP(hipMemcpyAsync(w.do_split, hsplit, na * 4, hipMemcpyHostToDevice, s));
    SLM_HIP(hipMemcpyAsync(w.gW, hgw, (size_t)na * D * 4, hipMemcpyHostToDevice, s));
    ProjectArgs pr{};
    pr.X = Xc; pr.x_bf16 = p.precision == 1; pr.w_bf16 = 0; pr.N = N; pr.D = D; pr.W = w.gW;
    pr.beg = w.beg; pr.end = w.end;
    pr.n_nodes = na; pr.P = 1; pr.Z = w.zsel; pr.zmin = nullptr; pr.zmax = nullptr;
    pr.zl = zlayout_of(0, N, 1);
    if ((st = launch_project(pr, s))) return st;
    if ((st = clear_stats(w, 2 * na, p.crit, Kc, s))) return st;
    PartArgs pa{};
    pa.X = Xc; pa.Xn = Xbuf[nb]; pa.x_bf16 = p.precision == 1;
    pa.lab = mse ? nullptr : static_cast<const int32_t *>(tc);
    pa.labn = mse ? nullptr : static_cast<int32_t *>(tbuf[nb]);
    pa.y = mse ? static_cast<const double *>(tc) : nullptr;
    pa.yn = mse ? static_cast<double *>(tbuf[nb]) : nullptr;
    pa.zsel = w.zsel; pa.thr = w.gbest_thr; pa.do_split = w.do_split;
    pa.beg = w.beg; pa.end = w.end; pa.n_nodes = na; pa.D = D; pa.K = Kc; pa.N = N;
    pa.cnt_left = w.cnt_left; pa.off_left = w.off_left; pa.off_right = w.off_right;
    pa.n_left = w.n_left; pa.child = w.st;
    if ((st = launch_partition(pa, s))) return st;
    SLM_HIP(hipMemcpyAsync(hnl, w.n_left, na * 8, hipMemcpyDeviceToHost, s));
    if ((st = read_stats(w, 2 * na, p.crit, Kc, sh, s))) return st;
    SLM_HIP(hipStreamSynchronize(s));
    if ((st = tm_part.stop(s))) return st;
    std::vector<HNode> next;
    for (int j = 0; j < na; ++j) {
      if (!hsplit[j]) continue;
      const HNode &a = active[j];
      const int i = a.idx;
      std::copy(hgw + (size_t)j * D, hgw + (size_t)(j + 1) * D,
                out->w + (size_t)i * D);
      out->thr[i] = hgt[j];
      HNode l, r;
      const int64_t mid = a.beg + hnl[j];
      SLM_CHECK(new_node(a.depth + 1, 2 * a.heap + 1, 2 * j, a.beg, mid, a.tree, &l),
                SLM_E_SHAPE, "grow: more than max_nodes = %d nodes", out->max_nodes);
      SLM_CHECK(new_node(a.depth + 1, 2 * a.heap + 2, 2 * j + 1, mid, a.end, a.tree, &r),
                SLM_E_SHAPE, "grow: more than max_nodes = %d nodes", out->max_nodes);
      out->left[i] = l.idx;
      out->right[i] = r.idx;
      next.push_back(l);
      next.push_back(r);
    }
    Xc = Xbuf[nb];
    tc = tbuf[nb];
    nb ^= 1;
    frontier.swap(next);
  }
  out->n_nodes = nn;
  return SLM_OK;
}

// common argument checks of the tree, forest and boosting entry points
static slm_status check_grow_args(const char *who, const void *X, int32_t x_dtype,
                                  const void *target, int32_t t_dtype, const slm_tree_params &p,
                                  int32_t D, const slm_tree_out *out) {
  const bool mse = p.crit == SLM_MSE;
  SLM_CHECK(x_dtype == (p.precision == 1 ? SLM_BF16 : SLM_F32), SLM_E_DTYPE,
            "%s: X must be F32 (precision 0) or BF16 (precision 1)", who);
  SLM_CHECK(t_dtype == (mse ? SLM_F64 : SLM_I32), SLM_E_DTYPE,
            "%s: target dtype does not match the criterion", who);
  SLM_CHECK(X && target && out, SLM_E_INVALID, "%s: NULL pointer", who);
  SLM_CHECK(out->w && out->thr && out->left && out->right && out->leaf && out->n &&
                out->impurity && out->split_loss && out->depth && out->heap,
            SLM_E_INVALID, "%s: NULL output array", who);
  SLM_CHECK(out->max_nodes >= 1, SLM_E_SHAPE, "%s: max_nodes < 1", who);
  SLM_CHECK(!out->stats || tree_stats(p, D), SLM_E_UNSUPPORTED,
            "%s: node statistics need class labels and K * D <= 4096", who);
  return SLM_OK;
}

// A grown tree's root holds all of its N rows, and the exact scan (bins = 0)
// takes nodes of at most EXACT_ROWS rows: larger trees are refused before any
// launch rather than left unsplit.
static slm_status check_exact_rows(const char *who, const slm_tree_params *p, int64_t N) {
  SLM_CHECK(p->bins != 0 || N <= EXACT_ROWS, SLM_E_UNSUPPORTED,
            "%s: the exact scan (bins = 0) takes nodes of at most %d rows; the root holds %lld",
            who, EXACT_ROWS, (long long)N);
  return SLM_OK;
}

size_t slm_grow_tree_workspace(const slm_tree_params *prm, int64_t N, int32_t D) {
  if (check_tree_params(prm, N, D) != SLM_OK) return 0;
  if (check_exact_rows("slm_grow_tree_workspace", prm, N) != SLM_OK) return 0;
  return carve(*prm, N, D, nullptr, 0, tree_stats(*prm, D)).total;
}

slm_status slm_grow_tree(const void *X, int32_t x_dtype, int64_t N, int32_t D, const void *target,
                         int32_t t_dtype, const slm_tree_params *prm, void *workspace,
                         size_t ws_bytes, slm_tree_out *out, void *stream) {
  clear_error();
  slm_status st = check_tree_params(prm, N, D);
  if (st) return st;
  if ((st = check_exact_rows("slm_grow_tree", prm, N))) return st;
  const slm_tree_params &p = *prm;
  if ((st = check_grow_args("slm_grow_tree", X, x_dtype, target, t_dtype, p, D, out))) return st;
  SLM_CHECK(workspace, SLM_E_INVALID, "slm_grow_tree: NULL workspace");
  const TreeWS w = carve(p, N, D, workspace, 0, tree_stats(p, D));
  SLM_CHECK(ws_bytes >= w.total, SLM_E_NOMEM, "slm_grow_tree: workspace of %zu bytes, %zu needed",
            ws_bytes, w.total);
  if ((st = prepare_kernels())) return st;
  hipStream_t s = S(stream);
  if (out->timing) std::fill(out->timing, out->timing + SLM_TIMING_SLOTS, 0.0);
  Timer tm_all;
  if ((st = tm_all.start(out->timing ? &out->timing[0] : nullptr, s))) return st;
  int64_t ss[2] = {0, 0};
  if ((st = grow_impl(X, N, D, target, p, w, {{0, N}}, 0, out, nullptr, ss, s))) return st;
  SLM_HIP(hipStreamSynchronize(s));
  if ((st = tm_all.stop(s))) return st;
  if (out->sample_splits) {
    out->sample_splits[0] = ss[0];
    out->sample_splits[1] = ss[1];
  }
  return SLM_OK;
}

// ---------------------------------------------------------------- forest
// Workspace of a forest: the gathered rows of every tree (X, targets, draws)
// ahead of the tree workspace of n_trees * N rows.
struct ForestWS {
  void *X, *t;
  int32_t *idx;
  TreeWS tree;
  size_t total;
};

static ForestWS carve_forest(const slm_tree_params &p, int64_t N, int32_t D, int32_t n_trees,
                             void *base) {
  Carver c{static_cast<char *>(base)};
  ForestWS f{};
  const int64_t NT = N * n_trees;
  const size_t xb = p.precision == 1 ? 2 : 4;
  f.X = c.take<char>((size_t)NT * D * xb);
  f.t = c.take<char>((size_t)NT * (p.crit == SLM_MSE ? 8 : 4));
  f.idx = c.take<int32_t>((size_t)NT);
  c.off = (c.off + 255) / 256 * 256;
  f.tree = carve(p, NT, D, base ? static_cast<char *>(base) + c.off : nullptr, 0, tree_stats(p, D),
                 n_trees);
  f.total = c.off + f.tree.total;
  return f;
}

static slm_status check_forest(const slm_tree_params *prm, int64_t N, int32_t D, int32_t n_trees) {
  slm_status st = check_tree_params(prm, N, D);
  if (st) return st;
  SLM_CHECK(n_trees >= 1 && n_trees <= 65535 && N * n_trees < (1ll << 31), SLM_E_SHAPE,
            "slm_grow_forest: n_trees = %d (1..65535, n_trees * N < 2^31)", n_trees);
  return check_exact_rows("slm_grow_forest", prm, N);
}

size_t slm_grow_forest_workspace(const slm_tree_params *prm, int64_t N, int32_t D,
                                 int32_t n_trees) {
  if (check_forest(prm, N, D, n_trees) != SLM_OK) return 0;
  return carve_forest(*prm, N, D, n_trees, nullptr).total;
}

slm_status slm_grow_forest(const void *X, int32_t x_dtype, int64_t N, int32_t D,
                           const void *target, int32_t t_dtype, const slm_tree_params *prm,
                           int32_t n_trees, int32_t bootstrap, void *workspace, size_t ws_bytes,
                           int32_t *sample_idx, slm_tree_out *out, int32_t *tree_of,
                           void *stream) {
  clear_error();
  slm_status st = check_forest(prm, N, D, n_trees);
  if (st) return st;
  const slm_tree_params &p = *prm;
  if ((st = check_grow_args("slm_grow_forest", X, x_dtype, target, t_dtype, p, D, out))) return st;
  SLM_CHECK(bootstrap == 0 || bootstrap == 1, SLM_E_INVALID, "slm_grow_forest: bootstrap %d",
            bootstrap);
  SLM_CHECK(workspace, SLM_E_INVALID, "slm_grow_forest: NULL workspace");
  const ForestWS f = carve_forest(p, N, D, n_trees, workspace);
  SLM_CHECK(ws_bytes >= f.total, SLM_E_NOMEM,
            "slm_grow_forest: workspace of %zu bytes, %zu needed", ws_bytes, f.total);
  if ((st = prepare_kernels())) return st;
  hipStream_t s = S(stream);
  if (out->timing) std::fill(out->timing, out->timing + SLM_TIMING_SLOTS, 0.0);
  Timer tm_all;
  if ((st = tm_all.start(out->timing ? &out->timing[0] : nullptr, s))) return st;
  const int64_t NT = N * n_trees;
  const size_t xb = p.precision == 1 ? 2 : 4;
  const int tb = p.crit == SLM_MSE ? 8 : 4;
  if (bootstrap && (st = launch_boot_draw(p.seed, p.tree, n_trees, N, f.idx, s))) return st;
  if ((st = launch_gather_rows(X, (size_t)D * xb, N, NT, bootstrap ? f.idx : nullptr, f.X, target,
                               tb, f.t, s)))
    return st;
  if (sample_idx && bootstrap)
    SLM_HIP(hipMemcpyAsync(sample_idx, f.idx, (size_t)NT * 4, hipMemcpyDeviceToDevice, s));
  std::vector<std::pair<int64_t, int64_t>> roots(n_trees);
  for (int b = 0; b < n_trees; ++b) roots[b] = {(int64_t)b * N, (int64_t)(b + 1) * N};
  int64_t ss[2] = {0, 0};
  if ((st = grow_impl(f.X, NT, D, f.t, p, f.tree, roots, 0, out, tree_of, ss, s))) return st;
  SLM_HIP(hipStreamSynchronize(s));
  if ((st = tm_all.stop(s))) return st;
  if (out->sample_splits) {
    out->sample_splits[0] = ss[0];
    out->sample_splits[1] = ss[1];
  }
  return SLM_OK;
}

slm_status slm_forest_predict(const float *w, const float *thr, const int32_t *left,
                              const int32_t *right, const double *leaf, int32_t n_nodes,
                              const int32_t *roots, int32_t n_trees, int32_t D, int32_t K,
                              const float *X, int64_t N, int32_t *leaf_ids, void *out,
                              void *stream) {
  clear_error();
  SLM_CHECK(n_nodes >= 1 && n_trees >= 1 && n_trees <= 65535 && D >= 1 && D <= DMAX && N >= 0 &&
                N < (1ll << 31) && N * n_trees < (1ll << 31),
            SLM_E_SHAPE, "slm_forest_predict: bad sizes");
  SLM_CHECK(K == 0 || (K >= 2 && K <= 16), SLM_E_SHAPE, "slm_forest_predict: K = %d (0 or 2..16)",
            K);
  if (N == 0) return SLM_OK;
  SLM_CHECK(w && thr && left && right && leaf && roots && X && leaf_ids && out, SLM_E_INVALID,
            "slm_forest_predict: NULL pointer");
  hipStream_t s = S(stream);
  slm_status st = launch_forest_leaves(w, thr, left, right, n_nodes, roots, n_trees, D, X, N,
                                       leaf_ids, s);
  if (st) return st;
  return launch_forest_combine(leaf_ids, leaf, n_nodes, n_trees, K, N, out, s);
}

slm_status slm_boost_scores(const float *w, const float *thr, const int32_t *left,
                            const int32_t *right, const double *leaf, int32_t n_nodes,
                            const int32_t *roots, int32_t n_rounds, int32_t n_classes, int32_t D,
                            const double *F0, double lr, const float *X, int64_t N,
                            int32_t *leaf_ids, double *F, void *stream) {
  clear_error();
  const int Kc = std::max(1, (int)n_classes);
  SLM_CHECK(n_classes == 0 || (n_classes >= 2 && n_classes <= 16), SLM_E_SHAPE,
            "slm_boost_scores: n_classes = %d (0 or 2..16)", n_classes);
  SLM_CHECK(n_rounds >= 0 && n_nodes >= 0 && D >= 1 && D <= DMAX && N >= 0 && N < (1ll << 31) &&
                (int64_t)n_rounds * Kc <= 65535 && N * n_rounds * Kc < (1ll << 31),
            SLM_E_SHAPE, "slm_boost_scores: bad sizes");
  SLM_CHECK(std::isfinite(lr), SLM_E_INVALID, "slm_boost_scores: lr must be finite");
  SLM_CHECK(F0 && F, SLM_E_INVALID, "slm_boost_scores: NULL pointer");
  if (N == 0) return SLM_OK;
  hipStream_t s = S(stream);
  slm_status st = launch_boost_init(F, N, Kc, F0, s);
  if (st || n_rounds == 0) return st;
  SLM_CHECK(n_nodes >= 1 && w && thr && left && right && leaf && roots && X && leaf_ids,
            SLM_E_INVALID, "slm_boost_scores: NULL pointer");
  const int nt = n_rounds * Kc;
  if ((st = launch_forest_leaves(w, thr, left, right, n_nodes, roots, nt, D, X, N, leaf_ids, s)))
    return st;
  // round by round, as the training scores were accumulated
  for (int m = 0; m < n_rounds; ++m)
    if ((st = launch_boost_update(F, leaf_ids + (size_t)m * Kc * N, leaf, n_nodes, N, Kc, lr, s)))
      return st;
  return SLM_OK;
}

// ---------------------------------------------------------------- boosting
// Workspace of boosting: the per-class copies of X (n_classes > 1), the
// residual targets, leaf ids, one round's tree arrays and the tree workspace
// of Kc * N rows.
struct BoostWS {
  float *Xrep;
  double *r;
  int32_t *leaf_ids, *roots;
  float *dw, *dthr;
  int32_t *dl, *dr;
  double *dleaf;
  int64_t round_nodes;
  TreeWS tree;
  size_t total;
};

static int64_t boost_round_nodes(const slm_tree_params &p, int64_t N, int Kc) {
  const int64_t by_depth = p.max_depth >= 29 ? (1ll << 30) : (2ll << p.max_depth) - 1;
  return Kc * std::min(by_depth, 2 * N - 1);
}

static BoostWS carve_boost(const slm_tree_params &p, int64_t N, int32_t D, int32_t n_classes,
                           void *base) {
  Carver c{static_cast<char *>(base)};
  BoostWS b{};
  const int Kc = std::max(1, (int)n_classes);
  if (Kc > 1) b.Xrep = c.take<float>((size_t)Kc * N * D);
  b.r = c.take<double>((size_t)Kc * N);
  b.leaf_ids = c.take<int32_t>((size_t)Kc * N);
  b.roots = c.take<int32_t>((size_t)Kc);
  b.round_nodes = boost_round_nodes(p, N, Kc);
  b.dw = c.take<float>((size_t)b.round_nodes * D);
  b.dthr = c.take<float>((size_t)b.round_nodes);
  b.dl = c.take<int32_t>((size_t)b.round_nodes);
  b.dr = c.take<int32_t>((size_t)b.round_nodes);
  b.dleaf = c.take<double>((size_t)b.round_nodes);
  c.off = (c.off + 255) / 256 * 256;
  b.tree = carve(p, (int64_t)Kc * N, D, base ? static_cast<char *>(base) + c.off : nullptr, 0,
                 false, Kc);
  b.total = c.off + b.tree.total;
  return b;
}

static slm_status check_boost(const slm_tree_params *prm, int64_t N, int32_t D, int32_t n_classes,
                              int32_t n_rounds) {
  slm_status st = check_tree_params(prm, N, D);
  if (st) return st;
  if ((st = check_exact_rows("slm_boost", prm, N))) return st;
  SLM_CHECK(prm->crit == SLM_MSE && prm->precision == 0, SLM_E_INVALID,
            "slm_boost: the trees are SLR trees (crit SLM_MSE, precision 0)");
  SLM_CHECK(prm->proposal != 1, SLM_E_UNSUPPORTED, "slm_boost: no learned proposal");
  SLM_CHECK(n_classes == 0 || (n_classes >= 2 && n_classes <= 16), SLM_E_SHAPE,
            "slm_boost: n_classes = %d (0 = regression, 2..16)", n_classes);
  SLM_CHECK(n_rounds >= 0 && N * std::max(1, (int)n_classes) < (1ll << 31), SLM_E_SHAPE,
            "slm_boost: n_rounds = %d, N = %lld out of range", n_rounds, (long long)N);
  SLM_CHECK(boost_round_nodes(*prm, N, std::max(1, (int)n_classes)) < (1ll << 31), SLM_E_SHAPE,
            "slm_boost: too many nodes per round");
  return SLM_OK;
}

size_t slm_boost_workspace(const slm_tree_params *prm, int64_t N, int32_t D, int32_t n_classes) {
  if (check_boost(prm, N, D, n_classes, 0) != SLM_OK) return 0;
  return carve_boost(*prm, N, D, n_classes, nullptr).total;
}

slm_status slm_boost(const float *X, int64_t N, int32_t D, const void *target, int32_t t_dtype,
                     int32_t n_classes, const slm_tree_params *prm, int32_t n_rounds, double lr,
                     void *workspace, size_t ws_bytes, double *F, double *F0, slm_tree_out *out,
                     int32_t *tree_of, void *stream) {
  clear_error();
  slm_status st = check_boost(prm, N, D, n_classes, n_rounds);
  if (st) return st;
  const slm_tree_params &p = *prm;
  const int Kc = std::max(1, (int)n_classes);
  SLM_CHECK(t_dtype == (n_classes ? SLM_I32 : SLM_F64), SLM_E_DTYPE,
            "slm_boost: target must be I32 labels (n_classes > 0) or F64 (regression)");
  SLM_CHECK(std::isfinite(lr), SLM_E_INVALID, "slm_boost: lr must be finite");
  SLM_CHECK(X && target && F && F0 && out && workspace, SLM_E_INVALID, "slm_boost: NULL pointer");
  SLM_CHECK(!out->stats, SLM_E_UNSUPPORTED, "slm_boost: no node statistics output");
  slm_tree_params q = p;
  if ((st = check_grow_args("slm_boost", X, SLM_F32, F, SLM_F64, q, D, out))) return st;
  const BoostWS b = carve_boost(p, N, D, n_classes, workspace);
  SLM_CHECK(ws_bytes >= b.total, SLM_E_NOMEM, "slm_boost: workspace of %zu bytes, %zu needed",
            ws_bytes, b.total);
  if ((st = prepare_kernels())) return st;
  hipStream_t s = S(stream);
  if (out->timing) std::fill(out->timing, out->timing + SLM_TIMING_SLOTS, 0.0);
  Timer tm_all;
  if ((st = tm_all.start(out->timing ? &out->timing[0] : nullptr, s))) return st;
  const int64_t NT = (int64_t)Kc * N;
  const int32_t *labels = n_classes ? static_cast<const int32_t *>(target) : nullptr;
  const double *y = n_classes ? nullptr : static_cast<const double *>(target);
  // initial scores: the mean target (regression, from the root statistics
  // kernel) or zero; every row starts at F0
  std::vector<double> f0(Kc, 0.0);
  if (!n_classes) {
    const TreeWS &w = b.tree;
    const int64_t be[2] = {0, N};
    SLM_HIP(hipMemcpyAsync(w.beg, &be[0], 8, hipMemcpyHostToDevice, s));
    SLM_HIP(hipMemcpyAsync(w.end, &be[1], 8, hipMemcpyHostToDevice, s));
    if ((st = clear_stats(w, 1, SLM_MSE, 1, s))) return st;
    if ((st = launch_node_stats(w.beg, w.end, 1, N, nullptr, y, 1, w.st, s))) return st;
    double s1 = 0;
    uint32_t cnt = 0;
    SLM_HIP(hipMemcpyAsync(&s1, w.st.s1, 8, hipMemcpyDeviceToHost, s));
    SLM_HIP(hipMemcpyAsync(&cnt, w.st.cnt, 4, hipMemcpyDeviceToHost, s));
    SLM_HIP(hipStreamSynchronize(s));
    f0[0] = s1 / (double)cnt;
  }
  for (int k = 0; k < Kc; ++k) F0[k] = f0[k];
  // F [N, Kc] = F0 in every row: the one row replicated by a gather
  SLM_HIP(hipMemcpyAsync(b.r, f0.data(), Kc * 8, hipMemcpyHostToDevice, s));
  if ((st = launch_gather_rows(b.r, (size_t)Kc * 8, 1, N, nullptr, F, nullptr, 0, nullptr, s)))
    return st;
  if (Kc > 1 &&
      (st = launch_gather_rows(X, (size_t)D * 4, N, NT, nullptr, b.Xrep, nullptr, 0, nullptr, s)))
    return st;
  const float *Xg = Kc > 1 ? b.Xrep : X;
  std::vector<std::pair<int64_t, int64_t>> roots(Kc);
  for (int k = 0; k < Kc; ++k) roots[k] = {(int64_t)k * N, (int64_t)(k + 1) * N};
  int64_t ss[2] = {0, 0};
  int base = 0;
  std::vector<int32_t> hl, hr, rts(Kc), rtree;
  std::vector<double> hlv;
  for (int m = 0; m < n_rounds; ++m) {
    if ((st = launch_boost_residual(labels, y, F, N, n_classes, b.r, s))) return st;
    q.tree = p.tree + (uint32_t)(m * Kc);
    rtree.assign(out->max_nodes, 0);
    if ((st = grow_impl(Xg, NT, D, b.r, q, b.tree, roots, base, out,
                        tree_of ? rtree.data() : nullptr, ss, s)))
      return st;
    const int cnt = out->n_nodes - base;
    SLM_CHECK(cnt <= b.round_nodes, SLM_E_SHAPE, "slm_boost: round of %d nodes", cnt);
    if (tree_of)
      for (int i = base; i < out->n_nodes; ++i) tree_of[i] = m * Kc + rtree[i];
    // this round's trees on the device, indices relative to the round
    hl.resize(cnt);
    hr.resize(cnt);
    hlv.resize(cnt);
    for (int i = 0; i < cnt; ++i) {
      const int l = out->left[base + i], r = out->right[base + i];
      hl[i] = l < 0 ? -1 : l - base;
      hr[i] = r < 0 ? -1 : r - base;
      hlv[i] = out->leaf[base + i];
    }
    for (int k = 0; k < Kc; ++k) rts[k] = k;   // the roots come first
    SLM_HIP(hipMemcpyAsync(b.dw, out->w + (size_t)base * D, (size_t)cnt * D * 4,
                           hipMemcpyHostToDevice, s));
    SLM_HIP(hipMemcpyAsync(b.dthr, out->thr + base, (size_t)cnt * 4, hipMemcpyHostToDevice, s));
    SLM_HIP(hipMemcpyAsync(b.dl, hl.data(), (size_t)cnt * 4, hipMemcpyHostToDevice, s));
    SLM_HIP(hipMemcpyAsync(b.dr, hr.data(), (size_t)cnt * 4, hipMemcpyHostToDevice, s));
    SLM_HIP(hipMemcpyAsync(b.dleaf, hlv.data(), (size_t)cnt * 8, hipMemcpyHostToDevice, s));
    SLM_HIP(hipMemcpyAsync(b.roots, rts.data(), (size_t)Kc * 4, hipMemcpyHostToDevice, s));
    if ((st = launch_forest_leaves(b.dw, b.dthr, b.dl, b.dr, cnt, b.roots, Kc, D, X, N,
                                   b.leaf_ids, s)))
      return st;
    if ((st = launch_boost_update(F, b.leaf_ids, b.dleaf, cnt, N, Kc, lr, s))) return st;
    // the host arrays above are reused next round
    SLM_HIP(hipStreamSynchronize(s));
    base = out->n_nodes;
  }
  out->n_nodes = base;
  SLM_HIP(hipStreamSynchronize(s));
  if ((st = tm_all.stop(s))) return st;
  if (out->sample_splits) {
    out->sample_splits[0] = ss[0];
    out->sample_splits[1] = ss[1];
  }
  return SLM_OK;
}

}  // extern "C"
