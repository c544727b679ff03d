// C ABI of the selected-inversion library: context, device plan construction
// and upload, and the entry points declared in include/selinv.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <queue>
#include <string>
#include <utility>
#include <vector>

#include "internal.hpp"
#include "plan.hpp"

namespace selinv {
hipError_t launch_normalize(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, bool cplx_, const void *src,
                            void *panels, void *dt, hipStream_t st, int part, int steps);
hipError_t launch_run(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, bool cplx_, int sched,
                      const void *panels, void *x, int64_t budget_ticks, int grid, hipStream_t st, int q0, int q1);
hipError_t launch_level_range(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, bool cplx_, const void *panels,
                              void *x, hipStream_t st, int q, int32_t b, int32_t e);
hipError_t launch_extract(const DevPlan &pl, const DevPlan *dpl, bool cplx_, const void *x, void *out, hipStream_t st);
int persistent_blocks_per_cu(bool cplx_);
hipError_t launch_backward(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, bool cplx, const void *panels,
                           const void *x, const void *dt, void *xbar, const void *wlogdet, void *abar, hipStream_t st);
hipError_t launch_scatter(const DevPlan &pl, const DevPlan *dpl, bool cplx_, const void *vals, void *panel,
                          hipStream_t st);
hipError_t launch_factor(const DevPlan &pl, const DevPlan *dpl, const FactorAux &fa, bool cplx_, const void *values,
                         void *panels, hipStream_t st);
}  // namespace selinv

using namespace selinv;

// Work area of selinv_normalize_run_noalloc, for callers that cannot allocate
// device memory: one fixed array per GPU, created with the code object and
// held until the process ends.  Host code never takes the symbol itself for
// an address; each device's address comes from hipGetSymbolAddress.
static constexpr int64_t kNoAllocBytes = int64_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int64_t kAlign = 256;
inline int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Host image of every device table plus its byte offset in the work buffer.
struct HostPlan {
  std::vector<int32_t> node_s, node_c;
  std::vector<int64_t> node_off, node_rowptr, node_sq, node_first, node_poff;
  std::vector<int64_t> kcol, kpos;
  std::vector<Item> items;
  std::vector<int32_t> item_ptr, nph, node_parent, node_ldg, node_split, node_kchunk;  // nph: [kPhases][ns]
  std::vector<int64_t> node_yoff;
  int64_t y_elems = 0;
  int64_t ns = 0;
  std::vector<int64_t> node_goff;
  int64_t g_elems = 0;
  int64_t dense_min_c = 0;  // threshold in use (INT64_MAX: no dense buffers)
  std::vector<int32_t> order;  // ticket order of the persistent schedule (all matrices)
  std::vector<Item> bitems;    // adjoint items in (sweep, depth, phase) order
  std::vector<int4> blaunch;   // adjoint launches in order (see LaunchAux)
  std::vector<int32_t> tiny_dptr;  // [depth + 1] small-node records of each etree depth
  std::vector<int32_t> tiny_dadj;  // [depth] end of each depth's c <= kTinyC prefix (the adjoint's)
  bool adjoint = false;        // adjoint scratch allocated (opts.adjoint >= 0)
  bool lu = false;             // LU plan: two panel sets (L, U^T), gathered GEMM-1 tiles only
  std::vector<int32_t> lvl_items, lvl_ptr, lvl_tiny, lvl_kind;
  std::vector<int32_t> lvl_tsplit;  // [nlvl]: a single-wavefront launch's first forward-only position (else -1)
  std::vector<int32_t> node_defer;  // GEMM-2 of the node in ITEM_P items (push schedule; level schedule: unsplit 128 x 128 tiles)
  std::vector<int32_t> node_ykern;  // GEMM-1 tiles in k_ydense (level schedule, dense buffer)
  std::vector<int8_t> node_y128;    // ... on 128 x 128 tiles in k_ydense128 (FP64, tune table)
  std::vector<Item> y128;           // the k_ydense128 records, in launch order
  std::vector<int8_t> node_tuned;   // a tune-table entry applied to the node
  int32_t lvl_top = 0;        // level launches of the top depths (see LaunchAux)
  std::vector<int32_t> lvl_depth_first;  // [depth + 1] first level launch of each etree depth (level schedule)
  // normalization chunks (see LaunchAux): level launch and list boundaries
  std::vector<int32_t> lvl_cut, norm_cut;
  // single-matrix level plans: the subtrees under the top chain of the tree
  // in two groups that run on two streams (see subtree_groups)
  std::vector<int8_t> node_grp;   // 0: a node of the top chain (or no split); 1, 2: its subtree's group
  int32_t grp_q = -1;             // first level launch below the chain (-1: no split)
  std::vector<int32_t> grp_rptr;  // [nlvl + 1]: the group ranges of launch q
  std::vector<int4> grp_ranges;   // {group, launch, first position, end position}
  std::vector<LRec> lvl_recs;  // the items of lvl_items with their nodes, in level order
  std::vector<TinyRec> tiny;  // single-wavefront nodes, in launch order
  std::vector<PushRec> push;  // push-form tiles (SELINV_SCHED_PUSH), in launch order
  std::vector<uint32_t> toff;  // their X_{C,C} tables (byte offsets into the panel array)
  std::vector<int2> chunks, chunks_narrow, rblocks;
  std::vector<int32_t> small_nodes;  // normalized by the single-wavefront kernel
  std::vector<int4> sq_tiles;
  std::vector<int64_t> apos;
  std::vector<uint8_t> adiag;
  std::vector<uint8_t> aflip;
  // device factorization: per-depth launch lists (deepest first) and pivot positions
  std::vector<int32_t> fac_nodes;
  std::vector<int2> fac_cn, fac_cw, fac_rb;
  std::vector<int4> fac_tiles;
  std::vector<FacLevel> fac_lev;
  std::vector<int64_t> dpos;
  int64_t sq_elems = 0;
  int64_t part_elems = 0;
  // byte offsets inside the work buffer
  struct Off {
    int64_t node_s, node_c, node_off, node_rowptr, node_sq, node_first, node_poff, kcol, kpos, posarr, items, item_ptr,
        nph, node_split, node_kchunk, node_yoff, node_goff, node_ldg, node_parent, order, lvl_items, lvl_recs, chunks, chunks_narrow, rblocks, small_nodes,
        sq_tiles, tiny, toff,
        apos, adiag, aflip, bitems, pushrecs, y128recs, fac_nodes, fac_cn, fac_cw, fac_rb, fac_tiles, dpos, plan, plan2, linv, dinv, part, gbuf, ypart,
        cnt, ctrl, fwd_end, adj_z, adj_l, adj_s, adj_t, adj_f, adj_d, ferr, fldet, end;
  } off{};
  int64_t tables_bytes = 0;  // [0, tables_bytes) is uploaded once
};

template <typename V>
void put(std::vector<unsigned char> &img, int64_t off, const std::vector<V> &v) {
  if (!v.empty()) std::memcpy(img.data() + off, v.data(), sizeof(V) * v.size());
}

// Ticket order of the persistent schedule.  The dependency graph of every
// matrix of the batch is list-scheduled on kSimWorkers identical workers
// under a simple cost model (flops at a fixed per-workgroup rate plus a fixed
// per-item overhead), always starting the ready item with the longest
// remaining path to the end of the traversal; tickets follow the simulated
// start order.  An item starts only after its dependencies have finished, so
// every dependency of an item holds a smaller ticket: the kernel, which hands
// tickets out in order and lets each workgroup wait for its own item's
// dependencies, can never deadlock.
constexpr int kSimWorkers = 256;
constexpr int64_t kDefaultDenseMinC = 256;
constexpr int64_t kSplitTarget = 512;  // GEMM-1 tiles that keep every CU busy (2 per CU)
constexpr int64_t kSplitMax = 8;
constexpr int64_t kSplitMinK = 320;    // default shortest contraction part
constexpr int64_t kSplitAlign = 32;    // parts start on a contraction-stage boundary
constexpr int64_t kDefaultDenseMaxBytes = int64_t(32) << 30;
constexpr double kNormChunkMin = 2e10;  // smallest normalization chunk (c s^2 + s^3 units, x4 complex)

double item_cost_ns(const HostPlan &H, const Item &it) {
  const double s = H.node_s[it.K], c = H.node_c[it.K];
  const bool dense = H.node_goff[it.K] >= 0;
  switch (it.type) {
    case ITEM_G:
      return 2500.0 + (double)kTileM * kTileM * 24.0 / 60.0;
    case ITEM_Y:
    case ITEM_YU: {
      const double m = std::min<double>(kTileM, c - (double)kTileM * it.a);
      const double nn = std::min<double>(kTileN, s - (double)kTileN * (it.b & 0xffff));
      const double kk = H.node_kchunk[it.K];
      const double gemm2 = H.node_yoff[it.K] >= 0 ? 0.0 : (2.0 * s * m * nn) / 150.0;
      return 1500.0 + (2.0 * m * nn * kk) / (dense ? 150.0 : 40.0) + gemm2;
    }
    case ITEM_R: {
      const double m = std::min<double>(kTileM, c - (double)kTileM * it.a);
      const double nn = std::min<double>(kTileN, s - (double)kTileN * (it.b & 0xffff));
      const double rq = std::max(1, it.b >> 24);
      return 1500.0 + H.node_split[it.K] * m * nn * 8.0 / 60.0 + (2.0 * s * m * nn) / 150.0 / rq;
    }
    case ITEM_D: {
      const double nr = std::ceil(c / kTileM);
      const double w = (it.b >> 16) ? kDSlabW : kTileN;
      return 1000.0 + nr * (double)kTileN * w * 8.0 / 60.0;
    }
    default:
      return 1500.0 + (2.0 * c * c * s + 2.0 * c * s * s) / 40.0;
  }
}

// Items of phase ph of node K: [phase_begin, phase_begin + phase_count).
int32_t phase_count(const HostPlan &H, int64_t K, int ph) { return H.nph[(size_t)ph * H.ns + K]; }
int32_t phase_begin(const HostPlan &H, int64_t K, int ph) {
  int32_t b = H.item_ptr[K];
  for (int q = 0; q < ph; ++q) b += phase_count(H, K, q);
  return b;
}
int first_phase(const HostPlan &H, int64_t K) {
  int ph = 0;
  while (ph < kPhases - 1 && phase_count(H, K, ph) == 0) ++ph;
  return ph;
}
int item_phase(const Item &it) { return selinv::item_phase(it.type); }

void ticket_order(const Symbolic &S, HostPlan &H, int64_t batch) {
  const int64_t ns = S.nsuper(), nit = (int64_t)H.items.size();
  std::vector<double> cost(nit), height(nit);
  for (int64_t i = 0; i < nit; ++i) cost[i] = item_cost_ns(H, H.items[i]);
  // remaining path: supernodes are numbered children first
  std::vector<double> tail(ns, 0.0);
  for (int64_t K = 0; K < ns; ++K) {
    double next = tail[K];  // longest path after the current phase
    for (int ph = kPhases - 1; ph >= 0; --ph) {
      const int32_t b = phase_begin(H, K, ph), n = phase_count(H, K, ph);
      if (n == 0) continue;
      double hmax = 0.0;
      for (int32_t i = b; i < b + n; ++i) {
        height[i] = cost[i] + next;
        hmax = std::max(hmax, height[i]);
      }
      next = hmax;
    }
    if (S.sparent[K] >= 0) tail[S.sparent[K]] = std::max(tail[S.sparent[K]], next);
  }
  std::vector<std::vector<int32_t>> kids(ns);
  for (int64_t K = 0; K < ns; ++K)
    if (S.sparent[K] >= 0) kids[S.sparent[K]].push_back((int32_t)K);
  // ready set: largest remaining path first, then the lowest id
  using RItem = std::pair<double, int64_t>;
  auto rcmp = [](const RItem &x, const RItem &y) { return x.first < y.first || (x.first == y.first && x.second > y.second); };
  std::priority_queue<RItem, std::vector<RItem>, decltype(rcmp)> ready(rcmp);
  using Ev = std::pair<double, int64_t>;
  std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> running;
  std::vector<int32_t> left((size_t)(batch * ns * kPhases));
  auto release = [&](int64_t l, int64_t K, int ph) {
    const int32_t b = phase_begin(H, K, ph), n = phase_count(H, K, ph);
    for (int32_t i = b; i < b + n; ++i) ready.push({height[i], l * nit + i});
  };
  for (int64_t l = 0; l < batch; ++l)
    for (int64_t K = 0; K < ns; ++K) {
      for (int ph = 0; ph < kPhases; ++ph) left[(l * ns + K) * kPhases + ph] = phase_count(H, K, ph);
      if (S.sparent[K] < 0) release(l, K, first_phase(H, K));
    }
  H.order.clear();
  H.order.reserve((size_t)(batch * nit));
  double now = 0.0;
  int64_t busy = 0;
  while (!ready.empty() || !running.empty()) {
    while (busy < kSimWorkers && !ready.empty()) {
      const int64_t id = ready.top().second;
      ready.pop();
      H.order.push_back((int32_t)id);
      running.push({now + cost[id % nit], id});
      ++busy;
    }
    if (running.empty()) break;
    now = running.top().first;
    while (!running.empty() && running.top().first <= now) {
      const int64_t id = running.top().second;
      running.pop();
      --busy;
      const int64_t l = id / nit, i = id % nit, K = H.items[i].K;
      int ph = item_phase(H.items[i]);
      if (--left[(l * ns + K) * kPhases + ph] != 0) continue;
      // phase done: release the next non-empty phase, or the children
      int nx = ph + 1;
      while (nx < kPhases && phase_count(H, K, nx) == 0) ++nx;
      if (nx < kPhases) {
        release(l, K, nx);
      } else {
        for (int32_t ch : kids[K]) release(l, ch, first_phase(H, ch));
      }
    }
  }
}

// Nodes with |C(K)| >= the threshold get a dense X_{C,C} buffer; the
// threshold is the requested one, raised in powers of two until the buffers of
// the whole batch fit in max_bytes.
// Dense X_{C,C} buffers for the nodes with c >= threshold.  Under the level
// schedule a buffer is live only while its own depth runs (the G items fill
// it, the Y items of the same depth read it; the adjoint sweeps also fill and
// read it within one depth), so the nodes of each depth are packed from
// offset 0 of one shared pool and only the largest depth counts against
// max_bytes.  The persistent schedule overlaps depths: every node gets its own
// buffer.  The threshold doubles until the footprint fits.
// pref[K] (from a tune table): -1 = by the threshold, 0 = never, 1 = from
// c >= 65 on; the forced ones are thinned by their own doubling threshold
// when the buffers do not fit.
// Dense X_{C,C} buffers.  Under the level schedule the buffers of one
// depth share a region with those of every other depth (a depth's gathers
// start after the previous depth is done); with subtree groups (node_grp),
// group 2 gets a region of its own, since the groups run on two streams and
// reach their depths at different times (the top chain runs before both).
void choose_dense(const Symbolic &S, int64_t batch, int64_t scalar_bytes, int64_t min_c, int64_t max_bytes,
                  bool per_level, const std::vector<int8_t> &pref, HostPlan &H) {
  const bool two = per_level && !H.node_grp.empty();
  auto key = [&](int64_t K) { return per_level ? 2 * S.sdepth[K] + (two && H.node_grp[K] == 2 ? 1 : 0) : int64_t(0); };
  const int64_t nkeys = per_level ? 2 * S.depth : 1;
  const int64_t ns = S.nsuper();
  H.node_goff.assign(ns, -1);
  H.node_ldg.assign(ns, 0);
  H.g_elems = 0;
  H.dense_min_c = INT64_MAX;
  auto ldg_of = [](int64_t c) { return (c + kPanelAlign - 1) / kPanelAlign * kPanelAlign; };
  const int64_t t0 = min_c < 0 ? INT64_MAX / 4 : std::max<int64_t>(min_c, kTileM + 1);
  auto wants = [&](int64_t K, int64_t t, int64_t tf) {
    const int64_t c = S.nrows(K);
    return pref[K] == 0 ? false : pref[K] == 1 ? c >= tf : c >= t;
  };
  // the largest depth of each region (even keys: the first, odd: group 2's)
  auto regions = [&](int64_t t, int64_t tf) {
    std::vector<int64_t> per(nkeys, 0);
    for (int64_t K = 0; K < ns; ++K)
      if (wants(K, t, tf)) per[key(K)] += ldg_of(S.nrows(K)) * S.nrows(K);
    std::pair<int64_t, int64_t> m{0, 0};
    for (int64_t k = 0; k < nkeys; ++k) (k & 1 ? m.second : m.first) = std::max(k & 1 ? m.second : m.first, per[k]);
    return m;
  };
  auto footprint = [&](int64_t t, int64_t tf) {
    const auto m = regions(t, tf);
    return m.first + m.second;
  };
  int64_t t = t0, tf = kTileM + 1;
  while (true) {
    const int64_t tot = footprint(t, tf);
    if (tot == 0) return;
    if (tot * batch * scalar_bytes <= max_bytes) break;
    t = std::min<int64_t>(t, INT64_MAX / 4) * 2;
    tf *= 2;
  }
  H.dense_min_c = t;
  const int64_t base2 = regions(t, tf).first;  // group 2's region starts after the first
  std::vector<int64_t> next(nkeys, 0);
  for (int64_t k = 1; k < nkeys; k += 2) next[k] = base2;
  for (int64_t K = 0; K < ns; ++K) {
    const int64_t c = S.nrows(K);
    if (!wants(K, t, tf)) continue;
    int64_t &o = next[key(K)];
    H.node_goff[K] = o;
    H.node_ldg[K] = (int32_t)ldg_of(c);
    o += ldg_of(c) * c;
    H.g_elems = std::max(H.g_elems, o);
  }
}

// Subtree groups of a single-matrix level plan: from the roots down, the
// nodes with exactly one child form the top chain (group 0); the subtrees
// under it are independent (a node's X needs only its ancestors' X), so they
// are dealt, largest first by the work of GEMM-1 and GEMM-2, to two groups of
// about equal work, which run on two streams after the chain (the launches of
// one fill the other's launch tails).  Returns the depth of the subtree roots,
// or -1 (a chain only, or fewer than two subtrees).
int64_t subtree_groups(const Symbolic &S, HostPlan &H) {
  const int64_t ns = S.nsuper();
  H.node_grp.assign(ns, 0);
  std::vector<std::vector<int64_t>> kids(ns);
  std::vector<int64_t> front;
  for (int64_t K = 0; K < ns; ++K)
    if (S.sparent[K] < 0)
      front.push_back(K);
    else
      kids[S.sparent[K]].push_back(K);
  while (front.size() == 1) front = kids[front[0]];
  if (front.size() < 2) {
    H.node_grp.clear();
    return -1;
  }
  std::vector<int64_t> byd(ns);  // nodes by depth, root first
  for (int64_t K = 0; K < ns; ++K) byd[K] = K;
  std::stable_sort(byd.begin(), byd.end(), [&](int64_t a, int64_t b) { return S.sdepth[a] < S.sdepth[b]; });
  std::vector<double> work(ns, 0.0);  // subtree work, leaves up
  for (int64_t i = ns - 1; i >= 0; --i) {
    const int64_t K = byd[i];
    const double c = (double)S.nrows(K), s = (double)S.width(K);
    work[K] += c * c * s + c * s * s;
    if (S.sparent[K] >= 0) work[S.sparent[K]] += work[K];
  }
  std::stable_sort(front.begin(), front.end(), [&](int64_t a, int64_t b) { return work[a] > work[b]; });
  double w1 = 0, w2 = 0;
  for (int64_t K : front) {
    H.node_grp[K] = w1 <= w2 ? 1 : 2;
    (w1 <= w2 ? w1 : w2) += work[K];
  }
  for (int64_t K : byd)  // top down
    if (H.node_grp[K] == 0 && S.sparent[K] >= 0) H.node_grp[K] = H.node_grp[S.sparent[K]];
  return S.sdepth[front[0]];
}

void build_plan(const Symbolic &S, int64_t batch, int64_t scalar_bytes, int64_t dense_min_c, int64_t dense_max_bytes,
                int64_t split_min_k, int sched, const TuneTable *tt, bool adjoint, bool herm, bool lu, HostPlan &H) {
  const int64_t ns = S.nsuper();
  H.lu = lu;
  // the push form (Alg. 2) runs one launch per depth and step like the level
  // schedule; its GEMM-1 work is done by push tiles, so no node gets a dense
  // buffer, a split contraction, a single-item or a single-wavefront path
  const bool push = sched == SELINV_SCHED_PUSH;
  const bool per_level = sched != SELINV_SCHED_PERSISTENT;
  // The LU form of Alg. 1 (Section 2.1) runs the level schedule with
  // gathered or dense-buffer GEMM-1 tiles (the buffer holds all of
  // X_{C,C}, its upper part from the X^T panel set): no split contraction,
  // R phase, tune table, single-item or single-wavefront node and no
  // single-wavefront normalization.
  if (push) dense_min_c = -1;
  if (push || lu) {
    split_min_k = -1;
    tt = nullptr;
  }
  // per-node choices from the tune table (bucket of (s, c)), else the defaults
  std::vector<int8_t> dense_pref(ns, -1), ykern_pref(ns, -1), tile128(ns, 0);
  std::vector<int64_t> node_mink(ns, split_min_k);
  H.node_tuned.assign(ns, 0);
  if (tt)
    for (int64_t K = 0; K < ns; ++K)
      if (const TuneEntry *e = tt->find(S.width(K), S.nrows(K))) {
        H.node_tuned[K] = 1;
        if (e->dense >= 0) dense_pref[K] = (int8_t)(e->dense != 0);
        if (e->ydense >= 0) ykern_pref[K] = (int8_t)(e->ydense != 0);
        if (e->split_min_k != 0) node_mink[K] = e->split_min_k;
        if (e->tile == 128 && scalar_bytes == 8) tile128[K] = 1;
      }
  H.node_s.resize(ns);
  H.node_c.resize(ns);
  H.node_off = S.panel_off;
  H.node_rowptr.assign(S.rowptr.begin(), S.rowptr.end() - 1);
  H.node_sq.resize(ns);
  H.node_first.assign(S.xsuper.begin(), S.xsuper.end() - 1);
  int64_t sq = 0;
  for (int64_t K = 0; K < ns; ++K) {
    H.node_s[K] = (int32_t)S.width(K);
    H.node_c[K] = (int32_t)S.nrows(K);
    H.node_sq[K] = sq;
    sq += S.width(K) * S.width(K);
  }
  H.sq_elems = sq;
  // Contraction split of the GEMM-1 tiles: a node whose tiles (over the whole
  // batch) cannot fill the GPU splits its contraction into parts of at least
  // kSplitMinK indices; the parts write partial tiles that phase-2 items sum.
  H.ns = ns;
  H.node_split.assign(ns, 1);
  H.node_kchunk.assign(ns, 0);
  H.node_yoff.assign(ns, -1);
  H.y_elems = 0;
  // GEMM-1 tiles of each depth (over the batch)
  std::vector<int64_t> dtiles(S.depth, 0);
  for (int64_t K = 0; K < ns; ++K)
    if (!(S.nrows(K) <= kSmallC && S.width(K) <= kSmallS))
      dtiles[S.sdepth[K]] += batch * ((S.nrows(K) + kTileM - 1) / kTileM) * ((S.width(K) + kTileN - 1) / kTileN);
  // the top depths: every depth down to here fills at most a quarter of the GPU
  int64_t top_depth = -1;
  while (top_depth + 1 < S.depth && dtiles[top_depth + 1] * 4 <= kSplitTarget) ++top_depth;
  for (int64_t K = 0; K < ns; ++K) {
    const int64_t s = S.width(K), c = S.nrows(K);
    H.node_kchunk[K] = (int32_t)c;
    if (c <= kSmallC && s <= kSmallS) continue;  // single-item node
    if (c == 0) continue;
    const int64_t tiles = batch * ((c + kTileM - 1) / kTileM) * ((s + kTileN - 1) / kTileN);
    const int64_t nq = (s + kTileN - 1) / kTileN;
    int64_t parts = 1;
    if (tiles < kSplitTarget) parts = std::min<int64_t>(kSplitMax, (kSplitTarget + tiles - 1) / tiles);
    if (node_mink[K] < 0) parts = 1;
    // at a depth that fills at most a quarter of the GPU, the parts may be a
    // quarter as long (as many as one round of items over the GPU allows):
    // there the GEMM-1 tiles wait on memory latency, and the R items that sum
    // the extra parts run on otherwise idle CUs
    const bool sparse = dtiles[S.sdepth[K]] * 4 <= kSplitTarget;
    const int64_t mink = sparse ? std::max<int64_t>(2 * kSplitAlign, node_mink[K] / 4) : node_mink[K];
    if (sparse) parts = std::min<int64_t>(parts, kSplitTarget / dtiles[S.sdepth[K]]);  // one round of items
    parts = std::max<int64_t>(1, std::min<int64_t>(parts, c / std::max<int64_t>(mink, kSplitAlign)));
    int64_t chunk = c;
    if (parts > 1) {
      chunk = (c + parts - 1) / parts;
      chunk = (chunk + kSplitAlign - 1) / kSplitAlign * kSplitAlign;
      parts = (c + chunk - 1) / chunk;
    }
    // An unsplit node whose GEMM-2 share spans several 64-row blocks of P,
    // at a depth with few tiles, also takes the R phase (one part): its
    // tiles' GEMM-2 shares are then cut into R items instead of running
    // block after block at the end of each GEMM-1 tile.
    if (parts <= 1 && (push || lu || !(nq > 1 && dtiles[S.sdepth[K]] * nq <= kSplitTarget))) continue;
    H.node_split[K] = (int32_t)parts;
    H.node_kchunk[K] = (int32_t)chunk;
    H.node_yoff[K] = H.y_elems;
    H.y_elems += (parts * c * s + kPanelAlign - 1) / kPanelAlign * kPanelAlign;
  }
  // GEMM-2 partial products: one s x s block per 64-row tile of C(K)
  H.node_poff.resize(ns);
  int64_t pe = 0;
  for (int64_t K = 0; K < ns; ++K) {
    H.node_poff[K] = pe;
    const int64_t nr = (S.nrows(K) + kTileM - 1) / kTileM;
    pe += (nr * S.width(K) * S.width(K) + kPanelAlign - 1) / kPanelAlign * kPanelAlign;
  }
  H.part_elems = pe;
  // per-row gather tables
  H.kcol.resize(S.rowind_L.size());
  H.kpos.resize(S.rowind_L.size());
  for (int64_t K = 0; K < ns; ++K) {
    const int64_t c = S.nrows(K), rp = S.rowptr[K];
    for (int64_t g = S.seg_ptr[K]; g < S.seg_ptr[K + 1]; ++g) {
      const int64_t J = S.seg_super[g], st = S.seg_start[g];
      const int64_t en = (g + 1 < S.seg_ptr[K + 1]) ? S.seg_start[g + 1] : c;
      const int64_t ldJ = S.width(J) + S.nrows(J);
      for (int64_t k = st; k < en; ++k) {
        H.kcol[rp + k] = S.panel_off[J] + (S.rowind_L[rp + k] - S.xsuper[J]) * ldJ;
        H.kpos[rp + k] = S.seg_posoff[g] - st;
      }
    }
  }
  // work items, phase by phase (see plan.hpp)
  H.node_grp.clear();
  H.grp_q = -1;
  const int64_t grp_depth = sched == SELINV_SCHED_LEVELS && batch == 1 ? subtree_groups(S, H) : -1;
  choose_dense(S, batch, scalar_bytes, dense_min_c, dense_max_bytes, per_level, dense_pref, H);
  // GEMM-2 shares of the R items: a depth whose R tiles (over the batch)
  // cannot fill the GPU cuts each tile's share into rq items by 64-row blocks
  // of P (the R phase of the top separator chain is otherwise one long item
  // per tile).
  // Under the level schedule, the GEMM-1 tiles of nodes with a dense buffer
  // run in their own kernel, which also runs the GEMM-2 shares of unsplit 64 x
  // 64 tiles; those of 128 x 128 tiles move to ITEM_P items of phase 2.
  H.node_defer.assign(ns, 0);
  H.node_ykern.assign(ns, 0);
  H.node_y128.assign(ns, 0);
  if (push)
    for (int64_t K = 0; K < ns; ++K) H.node_defer[K] = S.nrows(K) > 0;
  if (per_level && !push)
    for (int64_t K = 0; K < ns; ++K)
      if (H.node_goff[K] >= 0 && ykern_pref[K] != 0 && !(S.nrows(K) <= kSmallC && S.width(K) <= kSmallS)) {
        H.node_ykern[K] = 1;
        H.node_y128[K] = tile128[K];
        // GEMM-2 fused into k_ydense's tiles; the 128 x 128 tiles leave it to ITEM_P items
        if (H.node_yoff[K] < 0 && H.node_y128[K]) H.node_defer[K] = 1;
      }
  std::vector<int64_t> rtiles(S.depth, 0);
  for (int64_t K = 0; K < ns; ++K)
    if (H.node_yoff[K] >= 0 || H.node_defer[K])
      rtiles[S.sdepth[K]] += batch * ((S.nrows(K) + kTileM - 1) / kTileM) * ((S.width(K) + kTileN - 1) / kTileN);
  H.item_ptr.assign(ns + 1, 0);
  H.nph.assign((size_t)kPhases * ns, 0);
  auto nph = [&](int ph, int64_t K) -> int32_t & { return H.nph[(size_t)ph * ns + K]; };
  H.items.clear();
  for (int64_t K = 0; K < ns; ++K) {
    const int32_t s = H.node_s[K], c = H.node_c[K];
    H.item_ptr[K] = (int32_t)H.items.size();
    const int32_t nb = (s + kTileN - 1) / kTileN;
    const int32_t nr = (c + kTileM - 1) / kTileM;
    const int32_t parts = H.node_split[K];
    if (H.node_goff[K] >= 0) {
      for (int32_t a = 0; a < nr; ++a)
        for (int32_t b = 0; b <= a; ++b) H.items.push_back(Item{(int32_t)K, ITEM_G, a, b});
      nph(0, K) = nr * (nr + 1) / 2;
    }
    if (c <= kSmallC && s <= kSmallS && !push && !lu) {
      H.items.push_back(Item{(int32_t)K, ITEM_S, 0, 0});
      nph(3, K) = 1;
      continue;
    }
    if (c > 0) {
      if (!push) {
        for (int32_t p = 0; p < parts; ++p)
          for (int32_t b = 0; b < nb; ++b)
            for (int32_t a = 0; a < nr; ++a) H.items.push_back(Item{(int32_t)K, ITEM_Y, a, b | (p << 16)});
        nph(1, K) = nr * nb * parts;
        if (lu) {  // the upper part's GEMM-1 tiles, in the same phase
          for (int32_t b = 0; b < nb; ++b)
            for (int32_t a = 0; a < nr; ++a) H.items.push_back(Item{(int32_t)K, ITEM_YU, a, b});
          nph(1, K) += nr * nb;
        }
      }
      if (H.node_yoff[K] >= 0 || H.node_defer[K]) {  // partial tiles summed by R items, or GEMM-2 by P items
        const int32_t type = H.node_defer[K] ? ITEM_P : ITEM_R;
        const int64_t nq = (s + kTileN - 1) / kTileN;
        const int32_t rq = (int32_t)std::max<int64_t>(1, std::min<int64_t>(nq, kSplitTarget / rtiles[S.sdepth[K]]));
        for (int32_t r = 0; r < rq; ++r)
          for (int32_t b = 0; b < nb; ++b)
            for (int32_t a = 0; a < nr; ++a)
              H.items.push_back(Item{(int32_t)K, type, a, rq > 1 ? b | (r << 16) | (rq << 24) : b});
        nph(2, K) = nr * nb * rq;
      }
    }
    const int32_t nsl = nr >= kDSlabRows && !lu ? 64 / kDSlabW : 1;
    for (int32_t a = 0; a < nb; ++a)
      for (int32_t b = 0; b <= a; ++b)
        for (int32_t q = 0; q < nsl; ++q) H.items.push_back(Item{(int32_t)K, ITEM_D, a, nsl > 1 ? b | ((q + 1) << 16) : b});
    nph(3, K) = nb * (nb + 1) / 2 * nsl;
  }
  H.item_ptr[ns] = (int32_t)H.items.size();
  // item ids of the whole batch are int32 (and the ticket order holds one per
  // item and matrix): refuse before anything of that size is allocated
  if ((int64_t)H.items.size() * batch >= (int64_t)INT32_MAX) {
    Failure f;
    f.status = SELINV_ENOMEM;
    f.msg = "too many work items for int32 item ids (batch x items)";
    f.info0 = (int64_t)H.items.size();
    f.info1 = batch;
    throw f;
  }
  H.node_parent.resize(ns);
  for (int64_t K = 0; K < ns; ++K) H.node_parent[K] = (int32_t)S.sparent[K];
  ticket_order(S, H, batch);
  // level lists (every phase of every etree depth); at phase 3 the
  // single-wavefront nodes of a depth form a range of their own
  H.lvl_items.clear();
  H.lvl_ptr.assign(1, 0);
  H.lvl_top = 0;
  H.lvl_tiny.clear();
  H.lvl_kind.clear();
  H.lvl_tsplit.clear();
  H.tiny.clear();
  H.toff.clear();
  H.tiny_dptr.assign(S.depth + 1, 0);
  H.tiny_dadj.assign(S.depth, 0);
  // small nodes address X through 32-bit byte offsets
  const bool tiny_ok = !lu && S.panel_elems * scalar_bytes < (int64_t(1) << 32);
  // the forward sweep's single-wavefront nodes: c <= kTinyCF (complex plans
  // run the ones beyond kTinyC in a kernel of their own)
  const int64_t tiny_cf = kTinyCF;
  auto adj_tiny = [&](int64_t K) { return !push && tiny_ok && H.node_c[K] <= kTinyC && H.node_s[K] <= kTinyS; };
  H.push.clear();
  H.y128.clear();
  if (push) {
    // per depth, root first: the D step of the depth's nodes (P items, then
    // D items), then every tile its nodes push into their descendants
    std::vector<std::vector<int64_t>> bydepth(S.depth);
    for (int64_t K = 0; K < ns; ++K) bydepth[S.sdepth[K]].push_back(K);
    std::vector<std::vector<int64_t>> segs_of(ns);  // segments (of descendants) owned by K
    for (int64_t I = 0; I < ns; ++I)
      for (int64_t g = S.seg_ptr[I]; g < S.seg_ptr[I + 1]; ++g) segs_of[S.seg_super[g]].push_back(g);
    std::vector<int64_t> seg_node(S.seg_super.size());
    for (int64_t I = 0; I < ns; ++I)
      for (int64_t g = S.seg_ptr[I]; g < S.seg_ptr[I + 1]; ++g) seg_node[g] = I;
    auto close_items = [&]() {
      if ((int32_t)H.lvl_items.size() > H.lvl_ptr.back()) {
        H.lvl_ptr.push_back((int32_t)H.lvl_items.size());
        H.lvl_tiny.push_back(-1);
        H.lvl_kind.push_back(LVL_ITEMS);
        H.lvl_tsplit.push_back(-1);
      }
    };
    for (int64_t d = 0; d < S.depth; ++d) {
      for (int ph = 2; ph <= 3; ++ph) {
        for (int64_t K : bydepth[d]) {
          const int32_t b = phase_begin(H, K, ph), n = phase_count(H, K, ph);
          for (int32_t q = 0; q < n; ++q) H.lvl_items.push_back(b + q);
        }
        close_items();
      }
      const int32_t first = (int32_t)H.push.size();
      for (int64_t K : bydepth[d])
        for (int64_t g : segs_of[K]) {
          const int64_t I = seg_node[g];
          const int32_t cI = H.node_c[I], sI = H.node_s[I];
          const int32_t st = (int32_t)S.seg_start[g];
          const int32_t en = (g + 1 < S.seg_ptr[I + 1]) ? (int32_t)S.seg_start[g + 1] : cI;
          for (int32_t i0 = st; i0 < cI; i0 += kTileM)
            for (int32_t x0 = 0; x0 < sI; x0 += kTileN)
              H.push.push_back(PushRec{(int32_t)I, i0, x0, st, en, i0 >= en ? en : cI, 0, 0});
        }
      for (int32_t q = first; q < (int32_t)H.push.size(); ++q) H.lvl_items.push_back(q);
      if ((int32_t)H.push.size() > first) {
        H.lvl_ptr.push_back((int32_t)H.lvl_items.size());
        H.lvl_tiny.push_back(first);
        H.lvl_kind.push_back(LVL_PUSH);
        H.lvl_tsplit.push_back(-1);
      }
    }
  } else {
    auto is_tiny = [&](int64_t K) { return tiny_ok && H.node_c[K] <= tiny_cf && H.node_s[K] <= kTinyS; };
    int32_t tsplit = -1;  // of the single-wavefront launch being built
    auto close = [&](int32_t tiny_base, int32_t kind) {
      if ((int32_t)H.lvl_items.size() > H.lvl_ptr.back()) {
        H.lvl_ptr.push_back((int32_t)H.lvl_items.size());
        H.lvl_tiny.push_back(tiny_base);
        H.lvl_kind.push_back(kind);
        H.lvl_tsplit.push_back(kind == LVL_TINY ? tsplit : -1);
      }
    };
    std::vector<std::vector<int64_t>> bydepth(S.depth);
    for (int64_t K = 0; K < ns; ++K) bydepth[S.sdepth[K]].push_back(K);
    if (!H.node_grp.empty())  // group 1's nodes before group 2's at every depth: each launch is two ranges
      for (auto &v : bydepth)
        std::stable_sort(v.begin(), v.end(), [&](int64_t a, int64_t b) { return H.node_grp[a] < H.node_grp[b]; });
    H.lvl_depth_first.assign(S.depth + 1, 0);
    for (int64_t d = 0; d < S.depth; ++d) {
      H.lvl_depth_first[d] = (int32_t)H.lvl_ptr.size() - 1;
      for (int ph = 0; ph < kPhases; ++ph) {
        // phase 1: the GEMM-1 tiles of nodes with a dense buffer form a launch of their own
        for (int pass = 0; pass < (ph == 1 && per_level ? 2 : 1); ++pass) {
          for (int64_t K : bydepth[d]) {
            if (ph == 3 && is_tiny(K)) continue;
            if (ph == 1 && per_level && (H.node_ykern[K] != 0) != (pass == 1)) continue;
            if (ph == 1 && H.node_y128[K]) continue;  // launched on 128 x 128 tiles below
            const int32_t b = phase_begin(H, K, ph), n = phase_count(H, K, ph);
            for (int32_t q = 0; q < n; ++q) H.lvl_items.push_back(b + q);
          }
          close(-1, pass == 1 ? LVL_YDENSE : ph == 0 ? LVL_GATHER : ph == 2 ? LVL_GEMM2 : LVL_ITEMS);
        }
        if (ph == 1) {
          // 128 x 128 GEMM-1 tiles of the depth's FP64 dense-buffer nodes the tune table marks
          const int32_t first = (int32_t)H.y128.size();
          for (int64_t K : bydepth[d]) {
            if (!H.node_y128[K]) continue;
            const int32_t nr = (H.node_c[K] + 127) / 128, nb = (H.node_s[K] + 127) / 128;
            for (int32_t part = 0; part < H.node_split[K]; ++part)
              for (int32_t a = 0; a < nr; ++a)
                for (int32_t bb = 0; bb < nb; ++bb)
                  H.y128.push_back(Item{(int32_t)K, ITEM_Y, a, bb | (part << 16)});
          }
          for (int32_t q = first; q < (int32_t)H.y128.size(); ++q) H.lvl_items.push_back(q);
          close(first, LVL_Y128);
        }
      }
      const int32_t tiny_base = (int32_t)H.tiny.size();
      H.tiny_dptr[d] = tiny_base;
      // the adjoint's nodes (c <= kTinyC) first, then the forward-only ones
      for (int pass = 0; pass < 2; ++pass) {
        for (int64_t K : bydepth[d]) {
          if (!is_tiny(K) || adj_tiny(K) != (pass == 0)) continue;
          const int32_t it = phase_begin(H, K, 3);
          const int64_t c = H.node_c[K], rp = S.rowptr[K];
          H.lvl_items.push_back(it);
          H.tiny.push_back(TinyRec{(int32_t)K, it, H.node_s[K], (int32_t)c, S.panel_off[K], (int64_t)H.toff.size()});
          // X(row i, row k), i >= k, lives in the panel of row k's supernode;
          // the table is c x c (both triangles), then one padding row of
          // offset 0 so that the loads of columns k < 64 of any row stay in it
          const size_t t0 = H.toff.size();
          H.toff.resize(t0 + c * c + kTinyCF, 0u);
          for (int64_t i = 0; i < c; ++i)
            for (int64_t k = 0; k <= i; ++k) {
              const uint32_t v = (uint32_t)((H.kcol[rp + k] + S.posarr[H.kpos[rp + k] + i]) * scalar_bytes);
              H.toff[t0 + i * c + k] = v;
              // entry (k, i), k < i, is X(i, k) transposed: conjugated in a Hermitian plan
              H.toff[t0 + k * c + i] = v | (herm && k < i ? 1u : 0u);
            }
        }
        if (pass == 0) {
          H.tiny_dadj[d] = (int32_t)H.tiny.size();
          tsplit = (int32_t)H.lvl_items.size();
        }
      }
      close(tiny_base, LVL_TINY);
      if (d == top_depth && d + 1 < S.depth) H.lvl_top = (int32_t)H.lvl_ptr.size() - 1;
    }
    H.lvl_depth_first[S.depth] = (int32_t)H.lvl_ptr.size() - 1;
    H.tiny_dptr[S.depth] = (int32_t)H.tiny.size();
    // the group ranges of every launch below the chain (maximal runs of one
    // group; a single-wavefront launch lists its adjoint nodes first, so it
    // can hold two runs of each group)
    const int32_t nl = (int32_t)H.lvl_ptr.size() - 1;
    H.grp_rptr.assign(nl + 1, 0);
    H.grp_ranges.clear();
    if (grp_depth >= 0) {
      H.grp_q = H.lvl_depth_first[grp_depth];
      for (int32_t q = 0; q < nl; ++q) {
        H.grp_rptr[q] = (int32_t)H.grp_ranges.size();
        if (q < H.grp_q) continue;
        const int32_t b = H.lvl_ptr[q], e = H.lvl_ptr[q + 1];
        auto grp_at = [&](int32_t pos) {
          const int32_t K = H.lvl_kind[q] == LVL_Y128 ? H.y128[H.lvl_items[pos]].K : H.items[H.lvl_items[pos]].K;
          return (int32_t)H.node_grp[K];
        };
        for (int32_t p0 = b; p0 < e;) {
          const int32_t g = grp_at(p0);
          int32_t p1 = p0 + 1;
          while (p1 < e && grp_at(p1) == g) ++p1;
          H.grp_ranges.push_back(int4{g, q, p0, p1});
          p0 = p1;
        }
      }
      H.grp_rptr[nl] = (int32_t)H.grp_ranges.size();
    }
  }
  H.lvl_recs.resize(H.lvl_items.size());
  for (size_t q = 0; q < H.lvl_items.size(); ++q) {
    const int32_t kind =
        H.lvl_kind[std::upper_bound(H.lvl_ptr.begin(), H.lvl_ptr.end(), (int32_t)q) - H.lvl_ptr.begin() - 1];
    if (kind == LVL_PUSH || kind == LVL_Y128) {
      H.lvl_recs[q] = LRec{};  // push tiles and 128-tile records carry their own records
      continue;
    }
    const Item &it = H.items[H.lvl_items[q]];
    const int64_t K = it.K;
    NodeInfo n{};
    n.K = it.K;
    n.s = H.node_s[K];
    n.c = H.node_c[K];
    n.ldg = H.node_ldg[K];
    n.split = H.node_split[K];
    n.kchunk = H.node_kchunk[K];
    n.defer2 = H.node_defer[K];
    // the dense buffer of a node whose GEMM-1 runs in k_ydense holds the
    // lower triangle only (k_ydense reads the rest mirrored)
    n.glow = H.node_ykern[K] && !H.node_y128[K] && !lu;
    n.off = H.node_off[K];
    n.rp = H.node_rowptr[K];
    n.goff = H.node_goff[K];
    n.poff = H.node_poff[K];
    n.yoff = H.node_yoff[K];
    H.lvl_recs[q] = LRec{it, n};
  }
  // adjoint items: R1 leaves -> root (deepest level first), then R3 root -> leaves
  H.bitems.clear();
  H.blaunch.clear();
  {
    auto is_tiny = adj_tiny;
    int32_t bstart = 0;
    std::vector<std::vector<int64_t>> bydepth(S.depth);
    for (int64_t K = 0; K < ns; ++K) bydepth[S.sdepth[K]].push_back(K);
    auto emit = [&](int64_t K, int32_t type) {
      const int32_t s = H.node_s[K], c = H.node_c[K];
      const int32_t nb = (s + kTileN - 1) / kTileN, nr = (c + kTileM - 1) / kTileM;
      const bool dense = H.node_goff[K] >= 0;
      switch (type) {
        case BI_T: case BI_F: case BI_D0:
          for (int32_t a = 0; a < nb; ++a)
            for (int32_t b = 0; b < nb; ++b) H.bitems.push_back(Item{(int32_t)K, type, a, b});
          break;
        case BI_DF:
          for (int32_t a = 0; a < nb; ++a)
            for (int32_t b = 0; b <= a; ++b) H.bitems.push_back(Item{(int32_t)K, type, a, b});
          break;
        case BI_G: case BI_SG:
          if (dense)
            for (int32_t a = 0; a < nr; ++a)
              for (int32_t b = 0; b <= a; ++b) H.bitems.push_back(Item{(int32_t)K, type, a, b});
          break;
        case BI_SC:
          for (int32_t a = 0; a < nr; ++a)
            for (int32_t b = 0; b <= a; ++b) H.bitems.push_back(Item{(int32_t)K, type, a, b});
          break;
        default:  // c x s tiles
          for (int32_t b = 0; b < nb; ++b)
            for (int32_t a = 0; a < nr; ++a) H.bitems.push_back(Item{(int32_t)K, type, a, b});
      }
    };
    auto close = [&]() {
      const int32_t n = (int32_t)H.bitems.size() - bstart;
      if (n > 0) H.blaunch.push_back(int4{0, bstart, n, 0});
      bstart = (int32_t)H.bitems.size();
    };
    auto tiny_launch = [&](int64_t d, int32_t kind) {
      const int32_t n = H.tiny_dadj[d] - H.tiny_dptr[d];
      if (n > 0) H.blaunch.push_back(int4{kind, H.tiny_dptr[d], n, 0});
    };
    static const int32_t r1[kBackR1Phases][3] = {{BI_T, BI_G, -1}, {BI_Z, -1, -1}, {BI_L, BI_SC, BI_F}, {BI_D0, -1, -1}};
    static const int32_t r3[kBackR3Phases][3] = {{BI_SG, -1, -1}, {BI_M, -1, -1}, {BI_LB, -1, -1}, {BI_N, -1, -1},
                                                 {BI_DF, -1, -1}};
    for (int64_t d = S.depth - 1; d >= 0; --d) {
      for (int ph = 0; ph < kBackR1Phases; ++ph) {
        for (int64_t K : bydepth[d])
          if (!is_tiny(K))
            for (int q = 0; q < 3 && r1[ph][q] >= 0; ++q) emit(K, r1[ph][q]);
        close();
      }
      tiny_launch(d, 1);
    }
    for (int64_t d = 0; d < S.depth; ++d) {
      for (int ph = 0; ph < kBackR3Phases; ++ph) {
        for (int64_t K : bydepth[d])
          if (!is_tiny(K))
            for (int q = 0; q < 3 && r3[ph][q] >= 0; ++q) emit(K, r3[ph][q]);
        close();
      }
      tiny_launch(d, 2);
    }
  }
  // normalization work lists
  H.chunks.clear();
  H.chunks_narrow.clear();
  H.rblocks.clear();
  H.sq_tiles.clear();
  H.small_nodes.clear();
  H.lvl_cut.clear();
  H.norm_cut.clear();
  {
    // Chunks for selinv_normalize_run (level schedule): the top depths, then
    // depth ranges whose normalization (estimated as sum c s^2 + s^3 per
    // node) starts at 1/32 of the rest, or kNormChunkMin, and doubles from
    // chunk to chunk up to a quarter of the rest.  The traversal of a chunk's
    // depths needs only that chunk's normalization, so the next chunks are
    // normalized while it runs.
    std::vector<uint8_t> cut(S.depth + 1, 0);
    if (H.lvl_top > 0 && !push && sched == SELINV_SCHED_LEVELS) {
      cut[top_depth + 1] = 1;
      std::vector<double> wd(S.depth, 0.0);
      for (int64_t K = 0; K < ns; ++K) {
        const double s = H.node_s[K], c = H.node_c[K];
        wd[S.sdepth[K]] += (c * s * s + s * s * s) * (double)batch * (scalar_bytes == 16 ? 4.0 : 1.0);
      }
      double rest = 0.0;
      for (int64_t d = top_depth + 1; d < S.depth; ++d) rest += wd[d];
      double target = std::max(rest / 32.0, kNormChunkMin), acc = 0.0;
      if (rest >= 4.0 * kNormChunkMin)
        for (int64_t d = top_depth + 1; d + 1 < S.depth; ++d) {
          acc += wd[d];
          if (acc >= target) {
            cut[d + 1] = 1;
            acc = 0.0;
            target = std::min(2.0 * target, std::max(rest / 4.0, kNormChunkMin));
          }
        }
    }
    auto mark = [&]() {
      H.norm_cut.push_back((int32_t)H.small_nodes.size());
      H.norm_cut.push_back((int32_t)H.chunks_narrow.size());
      H.norm_cut.push_back((int32_t)H.chunks.size());
      H.norm_cut.push_back((int32_t)H.rblocks.size());
      H.norm_cut.push_back((int32_t)H.sq_tiles.size());
    };
    mark();
    H.lvl_cut.push_back(0);
    // root first: the workgroups of the large top nodes, which take longest,
    // are dispatched first (measured: C2 normalization 0.55 -> 0.45 ms)
    std::vector<std::vector<int64_t>> bydepth(S.depth);
    for (int64_t K = 0; K < ns; ++K) bydepth[S.sdepth[K]].push_back(K);
    for (int64_t d = 0; d < S.depth; ++d) {
      if (cut[d]) {
        mark();
        H.lvl_cut.push_back(H.lvl_depth_first[d]);
      }
      for (int64_t K : bydepth[d]) {
        const int32_t s = H.node_s[K], c = H.node_c[K];
        if (s <= kSmallNormS && !lu) {
          H.small_nodes.push_back((int32_t)K);
          continue;
        }
        const int32_t nch = (s + 15) / 16;  // 16-column blocks of L_KK^{-1} (s <= 256)
        for (int32_t q = 0; q < nch; ++q) (s <= 64 ? H.chunks_narrow : H.chunks).push_back(int2{(int32_t)K, q});
        for (int32_t a = 0; a < (c + kTileM - 1) / kTileM; ++a) H.rblocks.push_back(int2{(int32_t)K, a});
        const int32_t nt = (s + 31) / 32;
        for (int32_t a = 0; a < nt; ++a)
          for (int32_t b = 0; b < nt; ++b) H.sq_tiles.push_back(int4{(int32_t)K, a, b, 0});
      }
    }
    mark();
    H.lvl_cut.push_back((int32_t)H.lvl_ptr.size() - 1);
  }
  H.apos = S.apos;
  H.adiag = S.apos_diag;
  H.aflip = S.aflip;
  // device factorization lists, deepest depth first
  H.fac_nodes.clear();
  H.fac_cn.clear();
  H.fac_cw.clear();
  H.fac_rb.clear();
  H.fac_tiles.clear();
  H.fac_lev.clear();
  {
    std::vector<std::vector<int64_t>> bydepth(S.depth);
    for (int64_t K = 0; K < ns; ++K) bydepth[S.sdepth[K]].push_back(K);
    for (int64_t d = S.depth - 1; d >= 0; --d) {
      FacLevel lv{};
      lv.nodes_b = (int32_t)H.fac_nodes.size();
      lv.narrow_b = (int32_t)H.fac_cn.size();
      lv.wide_b = (int32_t)H.fac_cw.size();
      lv.rb_b = (int32_t)H.fac_rb.size();
      lv.tiles_b = (int32_t)H.fac_tiles.size();
      for (int64_t K : bydepth[d]) {
        const int32_t s = H.node_s[K], c = H.node_c[K];
        H.fac_nodes.push_back((int32_t)K);
        for (int32_t q = 0; q < (s + 15) / 16; ++q) (s <= 64 ? H.fac_cn : H.fac_cw).push_back(int2{(int32_t)K, q});
        const int32_t nr = (c + kTileM - 1) / kTileM;
        for (int32_t a = 0; a < nr; ++a) {
          H.fac_rb.push_back(int2{(int32_t)K, a});
          for (int32_t b = 0; b <= a; ++b) H.fac_tiles.push_back(int4{(int32_t)K, a, b, 0});
        }
      }
      lv.nodes_n = (int32_t)H.fac_nodes.size() - lv.nodes_b;
      lv.narrow_n = (int32_t)H.fac_cn.size() - lv.narrow_b;
      lv.wide_n = (int32_t)H.fac_cw.size() - lv.wide_b;
      lv.rb_n = (int32_t)H.fac_rb.size() - lv.rb_b;
      lv.tiles_n = (int32_t)H.fac_tiles.size() - lv.tiles_b;
      H.fac_lev.push_back(lv);
    }
  }
  H.dpos.assign(S.n, 0);
  for (int64_t K = 0; K < ns; ++K) {
    const int64_t s = S.width(K), ld = s + S.nrows(K);
    for (int64_t j = 0; j < s; ++j) H.dpos[S.xsuper[K] + j] = S.panel_off[K] + j * ld + j;
  }

  // layout
  auto &o = H.off;
  int64_t p = 0;
  auto take = [&](int64_t bytes) {
    int64_t r = p;
    p = align_up(p + std::max<int64_t>(bytes, 1));
    return r;
  };
  o.node_s = take(4 * ns);
  o.node_c = take(4 * ns);
  o.node_off = take(8 * ns);
  o.node_rowptr = take(8 * ns);
  o.node_sq = take(8 * ns);
  o.node_first = take(8 * ns);
  o.node_poff = take(8 * ns);
  o.kcol = take(8 * (int64_t)H.kcol.size());
  o.kpos = take(8 * (int64_t)H.kpos.size());
  o.posarr = take(4 * (int64_t)S.posarr.size());
  o.items = take(16 * (int64_t)H.items.size());
  o.item_ptr = take(4 * (ns + 1));
  o.nph = take(4 * kPhases * ns);
  o.node_split = take(4 * ns);
  o.node_kchunk = take(4 * ns);
  o.node_yoff = take(8 * ns);
  o.node_goff = take(8 * ns);
  o.node_ldg = take(4 * ns);
  o.node_parent = take(4 * ns);
  o.order = take(4 * (int64_t)H.order.size());
  o.lvl_items = take(4 * (int64_t)H.lvl_items.size());
  o.lvl_recs = take((int64_t)sizeof(LRec) * (int64_t)H.lvl_items.size());
  o.tiny = take((int64_t)sizeof(TinyRec) * (int64_t)H.tiny.size());
  o.toff = take(4 * (int64_t)H.toff.size());
  o.chunks = take(8 * (int64_t)H.chunks.size());
  o.chunks_narrow = take(8 * (int64_t)H.chunks_narrow.size());
  o.small_nodes = take(4 * (int64_t)H.small_nodes.size());
  o.rblocks = take(8 * (int64_t)H.rblocks.size());
  o.sq_tiles = take(16 * (int64_t)H.sq_tiles.size());
  o.apos = take(8 * (int64_t)H.apos.size());
  o.adiag = take((int64_t)H.adiag.size());
  o.aflip = take((int64_t)H.aflip.size());
  o.bitems = take(16 * (int64_t)H.bitems.size());
  o.pushrecs = take((int64_t)sizeof(PushRec) * (int64_t)H.push.size());
  o.y128recs = take((int64_t)sizeof(Item) * (int64_t)H.y128.size());
  o.fac_nodes = take(4 * (int64_t)H.fac_nodes.size());
  o.fac_cn = take(8 * (int64_t)H.fac_cn.size());
  o.fac_cw = take(8 * (int64_t)H.fac_cw.size());
  o.fac_rb = take(8 * (int64_t)H.fac_rb.size());
  o.fac_tiles = take(16 * (int64_t)H.fac_tiles.size());
  o.dpos = take(8 * (int64_t)H.dpos.size());
  H.tables_bytes = p;
  o.plan = take((int64_t)sizeof(DevPlan));
  o.plan2 = take((int64_t)sizeof(DevPlan));  // the plan of the second half of the batch (see batch_half)
  o.linv = take(scalar_bytes * batch * H.sq_elems * (H.lu ? 2 : 1));  // LU: L_KK^{-1}, then U_KK^{-T}
  o.dinv = take(scalar_bytes * batch * S.n);
  o.part = take(scalar_bytes * batch * H.part_elems);
  o.gbuf = take(scalar_bytes * batch * H.g_elems);
  o.ypart = take(scalar_bytes * batch * H.y_elems);
  o.cnt = take(4 * kPhases * batch * ns);
  o.ctrl = take(4 * CTRL_WORDS);
  o.fwd_end = p;  // the forward path (normalize, run) touches [0, fwd_end) only
  H.adjoint = adjoint;
  const int64_t pan = H.adjoint ? scalar_bytes * batch * S.panel_elems : 0;
  const int64_t sqb = H.adjoint ? scalar_bytes * batch * H.sq_elems : 0;
  o.adj_z = take(pan);
  o.adj_l = take(pan);
  o.adj_s = take(pan);
  o.adj_t = take(sqb);
  o.adj_f = take(sqb);
  o.adj_d = take(sqb);
  o.ferr = take(8 * batch);
  o.fldet = take(16 * batch);
  o.end = p;
}

}  // namespace

struct selinv_ctx {
  Symbolic S;
  selinv_opts opts{};
  HostPlan H;
  std::vector<unsigned char> image;  // tables image (host)
  std::string err;
  int64_t info[2] = {-1, -1};
  std::vector<double> logdet;        // 2 per matrix
  bool factored = false;
  bool have_logdet = false;
  // What the buffers hold, for selinv_backward's state checks: `gen` counts
  // successful normalizations (selinv_factor / selinv_normalize /
  // selinv_normalize_run); the others record the generation and the buffer
  // of the last Dt output and of the last traversal.
  uint64_t gen = 0, dtilde_gen = 0, run_gen = 0;
  const void *panels_at = nullptr, *dtilde_at = nullptr, *x_at = nullptr;
  std::vector<Item> bseq;            // adjoint launch sequence for selinv_items (built on demand)
  std::vector<Item> lseq;            // forward level launches for selinv_items (built on demand)
  std::vector<Item> nseq;            // normalization chunks for selinv_items (built on demand)
  const void *ctrl_at = nullptr;     // control words of the last persistent launch (for selinv_sync)
  void *devfac_work = nullptr;       // work buffer of a device factorization not yet checked by selinv_sync
  uint64_t serial = 0;               // unique per context (owner tag of the no-alloc work area)
  std::string tune_path;             // copy of opts.tune_cache
  DevPlan plan_noalloc{};            // staging of the plan copy in the no-alloc work area
  void *uploaded_to = nullptr;       // work buffer holding the tables
  int device = -1;
  double *pinned = nullptr;          // host staging of the factor panels
  size_t pinned_bytes = 0;
  int64_t wall_khz = 0;
  DevPlan plan_host{};  // staging of the plan copy in the work buffer
  DevPlan plan2_host{};  // and of the second half's plan
  void *trace = nullptr;  // optional device trace buffer for the persistent schedule
  int grid = 0;
  // cached strings for views
  std::vector<int64_t> panel_off_view;

  hipStream_t side = nullptr, side2 = nullptr;  // side streams of selinv_normalize_run, and its events
  hipEvent_t ev_fork = nullptr, ev_inv = nullptr, ev_sq = nullptr;
  std::vector<hipEvent_t> ev_chunk;  // one per normalization chunk after the top one
  int side_device = -1;
  // the second half of the batch's traversal under the level schedule, and its events
  hipStream_t tst = nullptr;
  hipEvent_t ev_tfork = nullptr, ev_tjoin = nullptr;
  int tst_device = -1;

  ~selinv_ctx() {
    if (pinned) (void)hipHostFree(pinned);
    for (hipEvent_t ev : {ev_fork, ev_inv, ev_sq, ev_tfork, ev_tjoin})
      if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : ev_chunk)
      if (ev) (void)hipEventDestroy(ev);
    if (side) (void)hipStreamDestroy(side);
    if (side2) (void)hipStreamDestroy(side2);
    if (tst) (void)hipStreamDestroy(tst);
  }
  bool is_complex() const { return opts.dtype == SELINV_C128 || opts.dtype == SELINV_H128; }
  bool is_herm() const { return opts.dtype == SELINV_H128; }
  bool is_lu() const { return opts.dtype == SELINV_LU64; }
  int64_t sbytes() const { return is_complex() ? 16 : 8; }
  // elements of one matrix's panels (an LU context holds the L and the U^T
  // panel sets, one after the other) and doubles of one matrix's values
  int64_t pelems() const { return is_lu() ? 2 * S.panel_elems : S.panel_elems; }
  int64_t vdoubles() const { return (is_complex() || is_lu() ? 2 : 1) * S.nnzA; }
};

namespace {

selinv_status set_err(selinv_ctx *h, selinv_status st, const std::string &m, int64_t i0 = -1, int64_t i1 = -1) {
  if (h) {
    h->err = m;
    h->info[0] = i0;
    h->info[1] = i1;
  }
  return st;
}

// A normalization into panels_dev (with Dt into dtilde_dev when non-null) was enqueued.
void note_normalized(selinv_ctx *h, const void *panels_dev, const void *dtilde_dev) {
  h->factored = true;
  h->gen++;
  h->panels_at = panels_dev;
  if (dtilde_dev) {
    h->dtilde_gen = h->gen;
    h->dtilde_at = dtilde_dev;
  }
}

selinv_status hip_err(selinv_ctx *h, hipError_t e, const char *where) {
  return set_err(h, SELINV_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

DevPlan make_devplan(const selinv_ctx *h, void *work) {
  const auto &H = h->H;
  const auto &o = H.off;
  unsigned char *b = static_cast<unsigned char *>(work);
  DevPlan d{};
  d.n = h->S.n;
  d.ns = h->S.nsuper();
  d.nitems = (int64_t)H.items.size();
  d.batch = h->opts.batch;
  d.panel_elems = h->pelems();
  d.half = h->is_lu() ? h->S.panel_elems : 0;
  d.sq_elems = H.sq_elems;
  d.part_elems = H.part_elems;
  d.nnzA = h->S.nnzA;
  d.total_rows = (int64_t)H.kcol.size();
  d.node_s = (int32_t *)(b + o.node_s);
  d.node_c = (int32_t *)(b + o.node_c);
  d.node_off = (int64_t *)(b + o.node_off);
  d.node_rowptr = (int64_t *)(b + o.node_rowptr);
  d.node_sq = (int64_t *)(b + o.node_sq);
  d.node_first = (int64_t *)(b + o.node_first);
  d.node_poff = (int64_t *)(b + o.node_poff);
  d.kcol = (int64_t *)(b + o.kcol);
  d.kpos = (int64_t *)(b + o.kpos);
  d.posarr = (int32_t *)(b + o.posarr);
  d.items = (Item *)(b + o.items);
  d.item_ptr = (int32_t *)(b + o.item_ptr);
  d.nph = (int32_t *)(b + o.nph);
  d.node_split = (int32_t *)(b + o.node_split);
  d.node_kchunk = (int32_t *)(b + o.node_kchunk);
  d.node_yoff = (int64_t *)(b + o.node_yoff);
  d.node_goff = (int64_t *)(b + o.node_goff);
  d.node_ldg = (int32_t *)(b + o.node_ldg);
  d.g_elems = H.g_elems;
  d.node_parent = (int32_t *)(b + o.node_parent);
  d.order = (int32_t *)(b + o.order);
  d.lvl_items = (int32_t *)(b + o.lvl_items);
  d.toff = (uint32_t *)(b + o.toff);
  d.apos = (int64_t *)(b + o.apos);
  d.adiag = (uint8_t *)(b + o.adiag);
  d.aflip = (uint8_t *)(b + o.aflip);
  d.csign = h->is_herm() ? -1.0 : 1.0;
  d.linv = (void *)(b + o.linv);
  d.dinv = (void *)(b + o.dinv);
  d.part = (void *)(b + o.part);
  d.gbuf = (void *)(b + o.gbuf);
  d.ypart = (void *)(b + o.ypart);
  d.y_elems = H.y_elems;
  d.cnt = (int32_t *)(b + o.cnt);
  d.adj_z = H.adjoint ? (void *)(b + o.adj_z) : nullptr;
  d.adj_l = H.adjoint ? (void *)(b + o.adj_l) : nullptr;
  d.adj_s = H.adjoint ? (void *)(b + o.adj_s) : nullptr;
  d.adj_t = H.adjoint ? (void *)(b + o.adj_t) : nullptr;
  d.adj_f = H.adjoint ? (void *)(b + o.adj_f) : nullptr;
  d.adj_d = H.adjoint ? (void *)(b + o.adj_d) : nullptr;
  d.bitems = (Item *)(b + o.bitems);
  d.dpos = (int64_t *)(b + o.dpos);
  d.ferr = (unsigned long long *)(b + o.ferr);
  d.fldet = (double *)(b + o.fldet);
  d.ctrl = (int32_t *)(b + o.ctrl);
  d.trace = (int64_t *)h->trace;
  return d;
}

const DevPlan *dev_plan(const selinv_ctx *h, void *work) {
  return reinterpret_cast<const DevPlan *>(static_cast<unsigned char *>(work) + h->H.off.plan);
}

// The plan of matrices [bh, batch) seen as a batch of their own: the
// per-matrix work arrays the traversal kernels reach through the plan start
// at matrix bh (the panels, X and the GEMM-2 partials are kernel arguments).
DevPlan half_plan(const DevPlan &pl, int64_t bh, int64_t sbytes) {
  DevPlan b = pl;
  b.batch = pl.batch - bh;
  b.part = static_cast<unsigned char *>(pl.part) + bh * pl.part_elems * sbytes;
  b.gbuf = static_cast<unsigned char *>(pl.gbuf) + bh * pl.g_elems * sbytes;
  b.ypart = static_cast<unsigned char *>(pl.ypart) + bh * pl.y_elems * sbytes;
  return b;
}

// Under the level schedule a batch runs as two halves, matrices [0, bh) on
// the caller's stream and [bh, batch) on a second stream: the halves share
// no data, and the launches of each fill the other's launch tails.  0: one
// stream (other schedules, a single matrix, or a traced run, whose trace rows
// are laid out for one launch over the whole batch).
int64_t batch_half(const selinv_ctx *h) {
  const int64_t B = h->opts.batch;
  return h->opts.sched == SELINV_SCHED_LEVELS && B >= 2 && !h->trace ? (B + 1) / 2 : 0;
}

// The second traversal stream and its fork and join events (all or nothing).
selinv_status ensure_tstream(selinv_ctx *h) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_err(h, e, "hipGetDevice");
  if (h->tst) return h->tst_device == dev ? SELINV_OK : set_err(h, SELINV_ESTATE, "context used on another device");
  hipStream_t s = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&a, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (s) (void)hipStreamDestroy(s);
    return hip_err(h, e, "traversal stream and events");
  }
  h->tst = s;
  h->ev_tfork = a;
  h->ev_tjoin = b;
  h->tst_device = dev;
  return SELINV_OK;
}

// A single-matrix level plan with subtree groups runs them on two streams:
// the launches above the groups on st, then (after a fork event) group 1's
// ranges on st and group 2's on the traversal stream.  No split for a traced
// run (its trace rows are laid out for one stream).
bool use_groups(const selinv_ctx *h) { return h->H.grp_q >= 0 && !h->trace; }

// Level launches [q0, q1) of a plan with subtree groups; `forked` records
// whether the traversal stream has been forked off st (once, at the first
// launch below the chain).
hipError_t launch_groups(selinv_ctx *h, const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, const void *panels,
                         void *x, hipStream_t st, int q0, int q1, bool &forked) {
  const HostPlan &H = h->H;
  const int qs = std::min(q1, std::max(q0, H.grp_q));
  hipError_t e = hipSuccess;
  if (qs > q0) e = launch_run(pl, dpl, aux, h->is_complex(), h->opts.sched, panels, x, 0, h->grid, st, q0, qs);
  for (int q = qs; q < q1 && e == hipSuccess; ++q) {
    if (!forked) {
      e = hipEventRecord(h->ev_tfork, st);
      if (e == hipSuccess) e = hipStreamWaitEvent(h->tst, h->ev_tfork, 0);
      if (e != hipSuccess) break;
      forked = true;
    }
    for (int32_t r = H.grp_rptr[q]; r < H.grp_rptr[q + 1] && e == hipSuccess; ++r) {
      const int4 g = H.grp_ranges[r];
      e = launch_level_range(pl, dpl, aux, h->is_complex(), panels, x, g.x == 2 ? h->tst : st, q, g.z, g.w);
    }
  }
  return e;
}

// Level launches [q0, q1) of both halves of the batch (bh > 0): the first
// half on st, the second on the traversal stream with the second half's plan.
hipError_t launch_halves(const selinv_ctx *h, const DevPlan &pl, const LaunchAux &aux, void *work, const void *panels,
                         void *x, hipStream_t st, int q0, int q1, int64_t bh) {
  DevPlan a = pl;
  a.batch = bh;
  hipError_t e = launch_run(a, dev_plan(h, work), aux, h->is_complex(), h->opts.sched, panels, x, 0, h->grid, st, q0, q1);
  if (e != hipSuccess) return e;
  const DevPlan b = half_plan(pl, bh, h->sbytes());
  const int64_t off = bh * pl.panel_elems * h->sbytes();
  const DevPlan *db = reinterpret_cast<const DevPlan *>(static_cast<unsigned char *>(work) + h->H.off.plan2);
  return launch_run(b, db, aux, h->is_complex(), h->opts.sched, static_cast<const unsigned char *>(panels) + off,
                    static_cast<unsigned char *>(x) + off, 0, h->grid, h->tst, q0, q1);
}

FactorAux make_fac_aux(const selinv_ctx *h, void *work) {
  const auto &H = h->H;
  unsigned char *b = static_cast<unsigned char *>(work);
  FactorAux a{};
  a.nodes = (const int32_t *)(b + H.off.fac_nodes);
  a.chunks_narrow = (const int2 *)(b + H.off.fac_cn);
  a.chunks_wide = (const int2 *)(b + H.off.fac_cw);
  a.rblocks = (const int2 *)(b + H.off.fac_rb);
  a.tiles = (const int4 *)(b + H.off.fac_tiles);
  a.lev = H.fac_lev.data();
  a.nlev = (int32_t)H.fac_lev.size();
  return a;
}

LaunchAux make_aux(const selinv_ctx *h, void *work) {
  const auto &H = h->H;
  unsigned char *b = static_cast<unsigned char *>(work);
  LaunchAux a{};
  a.small_nodes = (const int32_t *)(b + H.off.small_nodes);
  a.nsmall = (int32_t)H.small_nodes.size();
  a.chunks = (const int2 *)(b + H.off.chunks);
  a.nchunks = (int32_t)H.chunks.size();
  a.chunks_narrow = (const int2 *)(b + H.off.chunks_narrow);
  a.nchunks_narrow = (int32_t)H.chunks_narrow.size();
  a.rblocks = (const int2 *)(b + H.off.rblocks);
  a.nrblocks = (int32_t)H.rblocks.size();
  a.sq_tiles = (const int4 *)(b + H.off.sq_tiles);
  a.nsq_tiles = (int32_t)H.sq_tiles.size();
  a.lvl_items = (const int32_t *)(b + H.off.lvl_items);
  a.lvl_recs = (const LRec *)(b + H.off.lvl_recs);
  a.lvl_ptr = H.lvl_ptr.data();
  a.lvl_tiny = H.lvl_tiny.data();
  a.lvl_tsplit = H.lvl_tsplit.data();
  a.lvl_kind = H.lvl_kind.data();
  a.push = (const PushRec *)(b + H.off.pushrecs);
  a.y128 = (const Item *)(b + H.off.y128recs);
  a.tiny = (const TinyRec *)(b + H.off.tiny);
  a.nlvl = (int32_t)H.lvl_ptr.size() - 1;
  a.blaunch = H.blaunch.data();
  a.nblaunch = (int32_t)H.blaunch.size();
  a.lvl_top = H.lvl_top;
  a.nnorm_chunks = (int32_t)H.lvl_cut.size() - 1;
  a.lvl_cut = H.lvl_cut.data();
  a.norm_cut = H.norm_cut.data();
  return a;
}

void build_image(selinv_ctx *h) {
  auto &H = h->H;
  const auto &o = H.off;
  h->image.assign((size_t)H.tables_bytes, 0);
  auto &img = h->image;
  put(img, o.node_s, H.node_s);
  put(img, o.node_c, H.node_c);
  put(img, o.node_off, H.node_off);
  put(img, o.node_rowptr, H.node_rowptr);
  put(img, o.node_sq, H.node_sq);
  put(img, o.node_first, H.node_first);
  put(img, o.node_poff, H.node_poff);
  put(img, o.kcol, H.kcol);
  put(img, o.kpos, H.kpos);
  put(img, o.posarr, h->S.posarr);
  put(img, o.items, H.items);
  put(img, o.item_ptr, H.item_ptr);
  put(img, o.nph, H.nph);
  put(img, o.node_split, H.node_split);
  put(img, o.node_kchunk, H.node_kchunk);
  put(img, o.node_yoff, H.node_yoff);
  put(img, o.node_goff, H.node_goff);
  put(img, o.node_ldg, H.node_ldg);
  put(img, o.node_parent, H.node_parent);
  put(img, o.order, H.order);
  put(img, o.lvl_items, H.lvl_items);
  put(img, o.lvl_recs, H.lvl_recs);
  put(img, o.tiny, H.tiny);
  put(img, o.toff, H.toff);
  put(img, o.chunks, H.chunks);
  put(img, o.chunks_narrow, H.chunks_narrow);
  put(img, o.small_nodes, H.small_nodes);
  put(img, o.rblocks, H.rblocks);
  put(img, o.sq_tiles, H.sq_tiles);
  put(img, o.apos, H.apos);
  put(img, o.adiag, H.adiag);
  put(img, o.aflip, H.aflip);
  put(img, o.bitems, H.bitems);
  put(img, o.pushrecs, H.push);
  put(img, o.y128recs, H.y128);
  put(img, o.fac_nodes, H.fac_nodes);
  put(img, o.fac_cn, H.fac_cn);
  put(img, o.fac_cw, H.fac_cw);
  put(img, o.fac_rb, H.fac_rb);
  put(img, o.fac_tiles, H.fac_tiles);
  put(img, o.dpos, H.dpos);
}

selinv_status ensure_uploaded(selinv_ctx *h, void *work, hipStream_t st) {
  if (h->uploaded_to == work) return SELINV_OK;
  hipError_t e = hipMemcpyAsync(work, h->image.data(), h->image.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_err(h, e, "table upload");
  h->plan_host = make_devplan(h, work);
  e = hipMemcpyAsync(static_cast<unsigned char *>(work) + h->H.off.plan, &h->plan_host, sizeof(DevPlan),
                     hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_err(h, e, "plan upload");
  h->plan2_host = half_plan(h->plan_host, (h->plan_host.batch + 1) / 2, h->sbytes());
  e = hipMemcpyAsync(static_cast<unsigned char *>(work) + h->H.off.plan2, &h->plan2_host, sizeof(DevPlan),
                     hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_err(h, e, "plan upload");
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_err(h, e, "table upload sync");
  h->uploaded_to = work;
  return SELINV_OK;
}

// Launch geometry of the persistent schedule (once per context) and the
// per-wait budget in device clock ticks: watchdog_ms milliseconds, 0 = 10 s,
// < 0 = -watchdog_ms ticks.
selinv_status run_setup(selinv_ctx *h, int64_t *budget) {
  hipError_t e;
  if (h->grid == 0) {
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_err(h, e, "hipGetDevice");
    int ncu = 0, khz = 0;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_err(h, e, "device attribute");
    e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return hip_err(h, e, "device attribute");
    // One persistent workgroup per CU by default: with two, items at the
    // narrow top of the tree can land on the same CU while others idle.
    int per = persistent_blocks_per_cu(h->is_complex());
    int want = 1;
    if (const char *v = std::getenv("SELINV_PERSISTENT_WG_PER_CU")) want = std::atoi(v);
    if (want < 1) want = 1;
    if (per < 1) per = 1;
    h->grid = ncu * std::min(per, want);
    h->wall_khz = khz > 0 ? khz : 100000;
  }
  const int64_t wd = h->opts.watchdog_ms;
  *budget = wd < 0 ? -wd : (wd > 0 ? wd : 10000) * h->wall_khz;
  return SELINV_OK;
}

// Device address of this GPU's no-alloc work area, looked up once per device
// (with that device current) and kept; and which context's tables it holds.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
uint64_t g_scratch_owner[kMaxDevices] = {};
std::atomic<uint64_t> g_ctx_serial{0};

selinv_status scratch_for_device(selinv_ctx *h, int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return set_err(h, SELINV_EUNSUPPORTED, "device index beyond the no-alloc table");
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_err(h, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SELINV_OK;
}

}  // namespace

extern "C" {

void selinv_default_opts(selinv_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_super = 256;
  o->dtype = SELINV_R64;
  o->batch = 1;
  o->sched = SELINV_SCHED_LEVELS;
  o->relax = 0.05;
  o->nthreads = 0;
  o->dense_min_c = 0;
  o->watchdog_ms = 0;
  o->dense_max_bytes = 0;
  o->split_min_k = 0;
  o->adjoint = 0;
}

const char *selinv_version(void) { return "selinv-mi355x 0.2"; }

const char *selinv_tune_key(void) {
  static const std::string key = std::string("arch=") + tune_arch() + " rocm=" + tune_rocm();
  return key.c_str();
}

selinv_status selinv_analyze(int64_t n, const int64_t *colptr, const int64_t *rowind, const int64_t *perm,
                             const selinv_opts *opts, selinv_ctx **out) {
  if (!out) return SELINV_EINVAL;
  *out = nullptr;
  selinv_ctx *h = new (std::nothrow) selinv_ctx();
  if (!h) return SELINV_ENOMEM;
  h->serial = ++g_ctx_serial;
  if (opts)
    h->opts = *opts;
  else
    selinv_default_opts(&h->opts);
  if (h->opts.tune_cache) {  // keep a copy: the caller's string is borrowed for the call only
    h->tune_path = h->opts.tune_cache;
    h->opts.tune_cache = h->tune_path.c_str();
  }
  *out = h;
  const selinv_opts &o = h->opts;
  if (o.dtype != SELINV_R64 && o.dtype != SELINV_C128 && o.dtype != SELINV_H128 && o.dtype != SELINV_LU64)
    return set_err(h, SELINV_EUNSUPPORTED, "unknown dtype");
  if (o.dtype == SELINV_LU64 && o.sched != SELINV_SCHED_LEVELS)
    return set_err(h, SELINV_EUNSUPPORTED, "the LU form runs on the level schedule only");
  if (o.batch < 1) return set_err(h, SELINV_EINVAL, "batch must be >= 1");
  if (o.max_super < 1 || o.max_super > 256) return set_err(h, SELINV_EINVAL, "max_super must be in [1, 256]");
  if (o.sched != SELINV_SCHED_PERSISTENT && o.sched != SELINV_SCHED_LEVELS && o.sched != SELINV_SCHED_PUSH)
    return set_err(h, SELINV_EINVAL, "unknown schedule");
  try {
    analyze(h->S, n, colptr, rowind, perm, o.max_super, o.relax);
    const int64_t min_c = o.dense_min_c == 0 ? kDefaultDenseMinC : o.dense_min_c;
    const int64_t max_b = o.dense_max_bytes > 0 ? o.dense_max_bytes : kDefaultDenseMaxBytes;
    const int64_t split_k = o.split_min_k == 0 ? kSplitMinK : o.split_min_k;
    TuneTable tt;
    if (o.tune_cache && o.tune_cache[0]) tt = load_tune_table(o.tune_cache, h->is_complex() ? "c128" : "f64");
    build_plan(h->S, o.batch, h->sbytes(), min_c, max_b, split_k, o.sched,
               (o.tune_cache && o.tune_cache[0]) ? &tt : nullptr,
               o.adjoint >= 0 && o.dtype != SELINV_H128 && o.dtype != SELINV_LU64, o.dtype == SELINV_H128,
               o.dtype == SELINV_LU64, h->H);
    if ((int64_t)h->H.items.size() * (int64_t)o.batch >= (int64_t)INT32_MAX)
      return set_err(h, SELINV_ENOMEM, "too many work items for int32 item ids");
    build_image(h);
  } catch (const Failure &f) {
    return set_err(h, f.status, f.msg, f.info0, f.info1);
  } catch (const std::bad_alloc &) {
    return set_err(h, SELINV_ENOMEM, "host allocation failed in analyze");
  } catch (...) {
    return set_err(h, SELINV_EINVAL, "unexpected failure in analyze");
  }
  h->logdet.assign(2 * (size_t)o.batch, 0.0);
  return SELINV_OK;
}

selinv_status selinv_symbolic(const selinv_ctx *h, selinv_symbolic_view *v) {
  if (!h || !v) return SELINV_EINVAL;
  const Symbolic &S = h->S;
  if (S.n == 0) return SELINV_ESTATE;
  std::memset(v, 0, sizeof(*v));
  v->n = S.n;
  v->nsuper = S.nsuper();
  v->nnzL = S.nnzL;
  v->panel_elems = h->pelems();
  v->batch = h->opts.batch;
  v->dtype = h->opts.dtype;
  v->perm = S.perm.data();
  v->parent = S.parent.data();
  v->colcount = S.colcount.data();
  v->xsuper = S.xsuper.data();
  v->sparent = S.sparent.data();
  v->rowptr = S.rowptr.data();
  v->rowind_L = S.rowind_L.data();
  v->panel_off = S.panel_off.data();
  v->seg_ptr = S.seg_ptr.data();
  v->seg_super = S.seg_super.data();
  v->seg_start = S.seg_start.data();
  v->seg_posoff = S.seg_posoff.data();
  v->posarr = S.posarr.data();
  v->nseg = (int64_t)S.seg_super.size();
  v->nposarr = (int64_t)S.posarr.size();
  const double mul = h->is_complex() ? 4.0 : 1.0;
  v->flops = S.flops * mul;
  v->flops_exact = S.flops_exact * mul;
  v->depth = S.depth;
  int64_t tuned = 0;
  for (int8_t t : h->H.node_tuned) tuned += t;
  v->tuned_nodes = tuned;
  return SELINV_OK;
}

selinv_status selinv_sizes(const selinv_ctx *h, selinv_sizes_t *s) {
  if (!h || !s) return SELINV_EINVAL;
  if (h->S.n == 0) return SELINV_ESTATE;
  const int64_t B = h->opts.batch, sb = h->sbytes();
  s->panels_bytes = align_up(B * h->pelems() * sb);
  s->x_bytes = s->panels_bytes;
  s->work_bytes = h->H.off.end;
  s->dtilde_bytes = align_up(B * h->H.sq_elems * sb);
  s->abar_bytes = align_up(B * h->vdoubles() * 8);
  s->trace_bytes = align_up(64 * B * (int64_t)std::max(h->H.items.size(), h->H.lvl_items.size()));
  s->tables_bytes = h->H.tables_bytes;
  return SELINV_OK;
}

selinv_status selinv_factor(selinv_ctx *h, const void *values, void *panels_dev, void *work_dev, void *dtilde_dev,
                            void *stream) {
  if (!h) return SELINV_EINVAL;
  if (h->S.n == 0) return set_err(h, SELINV_ESTATE, "analyze did not succeed");
  if (!values || !panels_dev || !work_dev) return set_err(h, SELINV_EINVAL, "null buffer");
  hipStream_t st = (hipStream_t)stream;
  h->factored = false;
  h->have_logdet = false;
  if (dtilde_dev && h->is_lu()) return set_err(h, SELINV_EUNSUPPORTED, "no Dt output for the LU form");
  const int64_t B = h->opts.batch, sb = h->sbytes(), pe = h->pelems();
  const size_t need = (size_t)(B * pe * sb);
  hipError_t e;
  if (h->pinned_bytes < need) {
    if (h->pinned) (void)hipHostFree(h->pinned);
    h->pinned = nullptr;
    h->pinned_bytes = 0;
    e = hipHostMalloc((void **)&h->pinned, need, 0);
    if (e != hipSuccess) return hip_err(h, e, "pinned staging allocation");
    h->pinned_bytes = need;
  }
  const int64_t scal = h->is_complex() ? 2 : 1;
  const double *vals = static_cast<const double *>(values);
  try {
    for (int64_t l = 0; l < B; ++l) {
      double ld[2] = {0.0, 0.0};
      int64_t bad = factor_host(h->S, h->opts.dtype, vals + l * h->vdoubles(), h->pinned + l * pe * scal,
                                h->opts.nthreads, ld);
      if (bad >= 0) return set_err(h, SELINV_ESINGULAR, "zero or non-finite pivot", bad, l);
      h->logdet[2 * l] = ld[0];
      h->logdet[2 * l + 1] = ld[1];
    }
  } catch (const std::bad_alloc &) {
    return set_err(h, SELINV_ENOMEM, "host allocation failed in factor");
  }
  h->have_logdet = true;
  selinv_status ss = ensure_uploaded(h, work_dev, st);
  if (ss != SELINV_OK) return ss;
  e = hipMemcpyAsync(panels_dev, h->pinned, need, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_err(h, e, "panel upload");
  DevPlan pl = make_devplan(h, work_dev);
  LaunchAux aux = make_aux(h, work_dev);
  e = launch_normalize(pl, dev_plan(h, work_dev), aux, h->is_complex(), panels_dev, panels_dev, dtilde_dev, st, -1,
                       NORM_ALL);
  if (e != hipSuccess) return hip_err(h, e, "normalize launch");
  // the staging buffer is reused by the next call: wait for the copy
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_err(h, e, "factor sync");
  note_normalized(h, panels_dev, dtilde_dev);
  return SELINV_OK;
}

selinv_status selinv_normalize(selinv_ctx *h, const void *ldlt_dev, void *panels_dev, void *work_dev,
                               void *dtilde_dev, void *stream) {
  if (!h) return SELINV_EINVAL;
  if (h->S.n == 0) return set_err(h, SELINV_ESTATE, "analyze did not succeed");
  if (!ldlt_dev || !panels_dev || !work_dev) return set_err(h, SELINV_EINVAL, "null buffer");
  if (dtilde_dev && h->is_lu()) return set_err(h, SELINV_EUNSUPPORTED, "no Dt output for the LU form");
  hipStream_t st = (hipStream_t)stream;
  selinv_status ss = ensure_uploaded(h, work_dev, st);
  if (ss != SELINV_OK) return ss;
  DevPlan pl = make_devplan(h, work_dev);
  LaunchAux aux = make_aux(h, work_dev);
  hipError_t e =
      launch_normalize(pl, dev_plan(h, work_dev), aux, h->is_complex(), ldlt_dev, panels_dev, dtilde_dev, st, -1,
                       NORM_ALL);
  if (e != hipSuccess) return hip_err(h, e, "normalize launch");
  note_normalized(h, panels_dev, dtilde_dev);
  return SELINV_OK;
}

selinv_status selinv_factor_host(selinv_ctx *h, const void *values, void *panels_host) {
  if (!h) return SELINV_EINVAL;
  if (h->S.n == 0) return set_err(h, SELINV_ESTATE, "analyze did not succeed");
  if (!values || !panels_host) return set_err(h, SELINV_EINVAL, "null buffer");
  h->have_logdet = false;
  const int64_t B = h->opts.batch, pe = h->pelems();
  const int64_t scal = h->is_complex() ? 2 : 1;
  const double *vals = static_cast<const double *>(values);
  double *out = static_cast<double *>(panels_host);
  try {
    for (int64_t l = 0; l < B; ++l) {
      double ld[2] = {0.0, 0.0};
      int64_t bad = factor_host(h->S, h->opts.dtype, vals + l * h->vdoubles(), out + l * pe * scal,
                                h->opts.nthreads, ld);
      if (bad >= 0) return set_err(h, SELINV_ESINGULAR, "zero or non-finite pivot", bad, l);
      h->logdet[2 * l] = ld[0];
      h->logdet[2 * l + 1] = ld[1];
    }
  } catch (const std::bad_alloc &) {
    return set_err(h, SELINV_ENOMEM, "host allocation failed in factor");
  }
  h->have_logdet = true;
  return SELINV_OK;
}

selinv_status selinv_factor_device(selinv_ctx *h, const void *values_dev, void *ldlt_dev, void *work_dev,
                                   void *stream) {
  if (!h) return SELINV_EINVAL;
  if (h->S.n == 0) return set_err(h, SELINV_ESTATE, "analyze did not succeed");
  if (!values_dev || !ldlt_dev || !work_dev) return set_err(h, SELINV_EINVAL, "null buffer");
  if (h->is_lu()) return set_err(h, SELINV_EUNSUPPORTED, "selinv_factor_device: no device LU factorization");
  hipStream_t st = (hipStream_t)stream;
  selinv_status ss = ensure_uploaded(h, work_dev, st);
  if (ss != SELINV_OK) return ss;
  h->have_logdet = false;
  DevPlan pl = make_devplan(h, work_dev);
  FactorAux fa = make_fac_aux(h, work_dev);
  hipError_t e = launch_factor(pl, dev_plan(h, work_dev), fa, h->is_complex(), values_dev, ldlt_dev, st);
  if (e != hipSuccess) return hip_err(h, e, "factor launch");
  h->devfac_work = work_dev;
  return SELINV_OK;
}

selinv_status selinv_run(selinv_ctx *h, const void *panels_dev, void *x_dev, void *work_dev, void *stream) {
  if (!h) return SELINV_EINVAL;
  if (!h->factored) return set_err(h, SELINV_ESTATE, "selinv_run before a successful selinv_factor");
  if (!panels_dev || !x_dev || !work_dev) return set_err(h, SELINV_EINVAL, "null buffer");
  hipStream_t st = (hipStream_t)stream;
  selinv_status ss = ensure_uploaded(h, work_dev, st);
  if (ss != SELINV_OK) return ss;
  int64_t budget = 0;
  ss = run_setup(h, &budget);
  if (ss != SELINV_OK) return ss;
  hipError_t e;
  DevPlan pl = make_devplan(h, work_dev);
  LaunchAux aux = make_aux(h, work_dev);
  const int64_t bh = batch_half(h);
  if (bh > 0) {
    ss = ensure_tstream(h);
    if (ss != SELINV_OK) return ss;
    e = hipEventRecord(h->ev_tfork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(h->tst, h->ev_tfork, 0);
    if (e == hipSuccess) e = launch_halves(h, pl, aux, work_dev, panels_dev, x_dev, st, 0, aux.nlvl, bh);
    if (e == hipSuccess) e = hipEventRecord(h->ev_tjoin, h->tst);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, h->ev_tjoin, 0);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(h->tst);
      return hip_err(h, e, "selinv launch");
    }
  } else if (use_groups(h)) {
    ss = ensure_tstream(h);
    if (ss != SELINV_OK) return ss;
    bool forked = false;
    e = launch_groups(h, pl, dev_plan(h, work_dev), aux, panels_dev, x_dev, st, 0, aux.nlvl, forked);
    if (e == hipSuccess && forked) e = hipEventRecord(h->ev_tjoin, h->tst);
    if (e == hipSuccess && forked) e = hipStreamWaitEvent(st, h->ev_tjoin, 0);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(h->tst);
      return hip_err(h, e, "selinv launch");
    }
  } else {
    e = launch_run(pl, dev_plan(h, work_dev), aux, h->is_complex(), h->opts.sched, panels_dev, x_dev, budget, h->grid,
                   st, 0, aux.nlvl);
    if (e != hipSuccess) return hip_err(h, e, "selinv launch");
  }
  h->run_gen = h->gen;
  h->x_at = x_dev;
  h->ctrl_at = static_cast<unsigned char *>(work_dev) + h->H.off.ctrl;
  return SELINV_OK;
}

selinv_status selinv_normalize_run(selinv_ctx *h, const void *ldlt_dev, void *panels_dev, void *x_dev, void *work_dev,
                                   void *dtilde_dev, void *stream) {
  if (!h) return SELINV_EINVAL;
  if (h->S.n == 0) return set_err(h, SELINV_ESTATE, "analyze did not succeed");
  if (!ldlt_dev || !panels_dev || !x_dev || !work_dev) return set_err(h, SELINV_EINVAL, "null buffer");
  if (dtilde_dev && h->is_lu()) return set_err(h, SELINV_EUNSUPPORTED, "no Dt output for the LU form");
  hipStream_t st = (hipStream_t)stream;
  selinv_status ss = ensure_uploaded(h, work_dev, st);
  if (ss != SELINV_OK) return ss;
  LaunchAux aux = make_aux(h, work_dev);
  if (h->opts.sched != SELINV_SCHED_LEVELS || aux.lvl_top == 0) {
    ss = selinv_normalize(h, ldlt_dev, panels_dev, work_dev, dtilde_dev, stream);
    return ss != SELINV_OK ? ss : selinv_run(h, panels_dev, x_dev, work_dev, stream);
  }
  hipError_t e;
  int dev = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_err(h, e, "hipGetDevice");
  if (h->side && h->side_device != dev) return set_err(h, SELINV_ESTATE, "context used on another device");
  const int nq = aux.nnorm_chunks;  // >= 2: the top depths, then the rest in chunks
  if (!h->side) {  // all or nothing: the context keeps them only if every one was created
    hipStream_t s1 = nullptr, s2 = nullptr;
    std::vector<hipEvent_t> ev((size_t)(3 + nq - 1), nullptr);
    e = hipStreamCreateWithFlags(&s1, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking);
    for (hipEvent_t &v : ev)
      if (e == hipSuccess) e = hipEventCreateWithFlags(&v, hipEventDisableTiming);
    if (e != hipSuccess) {
      for (hipEvent_t v : ev)
        if (v) (void)hipEventDestroy(v);
      if (s1) (void)hipStreamDestroy(s1);
      if (s2) (void)hipStreamDestroy(s2);
      return hip_err(h, e, "side streams and events");
    }
    h->side = s1;
    h->side2 = s2;
    h->ev_fork = ev[0];
    h->ev_inv = ev[1];
    h->ev_sq = ev[2];
    h->ev_chunk.assign(ev.begin() + 3, ev.end());
    h->side_device = dev;
  }
  const int64_t bh = batch_half(h);
  const bool groups = bh == 0 && use_groups(h);
  if (bh > 0 || groups) {
    ss = ensure_tstream(h);
    if (ss != SELINV_OK) return ss;
  }
  bool forked = false;  // the traversal stream has been forked off `stream`
  // on a failure after the fork, the side streams are drained before
  // returning, so that no work of this call still writes the caller's buffers
  auto fail = [&](hipError_t err, const char *what) {
    (void)hipStreamSynchronize(h->side);
    (void)hipStreamSynchronize(h->side2);
    if (bh > 0 || groups) (void)hipStreamSynchronize(h->tst);
    return hip_err(h, err, what);
  };
  DevPlan pl = make_devplan(h, work_dev);
  const DevPlan *dpl = dev_plan(h, work_dev);
  const bool cx = h->is_complex();
  // fork: the deeper nodes' normalization on the first side stream, after
  // the caller's earlier work, chunk by chunk root first, an event after each
  e = hipEventRecord(h->ev_fork, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(h->side, h->ev_fork, 0);
  for (int q = 1; q < nq && e == hipSuccess; ++q) {
    e = launch_normalize(pl, dpl, aux, cx, ldlt_dev, panels_dev, dtilde_dev, h->side, q, NORM_ALL);
    if (e == hipSuccess) e = hipEventRecord(h->ev_chunk[q - 1], h->side);
  }
  if (e != hipSuccess) return fail(e, "normalize (side stream)");
  // the top nodes: L_KK^{-1} on the caller's stream, then Lhat there and
  // Dt^{-1} on the second side stream at the same time (both need only
  // L_KK^{-1}; they write different parts of the panels)
  e = launch_normalize(pl, dpl, aux, cx, ldlt_dev, panels_dev, dtilde_dev, st, 0, NORM_INV);
  if (e == hipSuccess) e = hipEventRecord(h->ev_inv, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(h->side2, h->ev_inv, 0);
  if (e == hipSuccess) e = launch_normalize(pl, dpl, aux, cx, ldlt_dev, panels_dev, dtilde_dev, h->side2, 0, NORM_SQ);
  if (e == hipSuccess) e = hipEventRecord(h->ev_sq, h->side2);
  if (e == hipSuccess) e = launch_normalize(pl, dpl, aux, cx, ldlt_dev, panels_dev, dtilde_dev, st, 0, NORM_GEMM);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, h->ev_sq, 0);
  if (e != hipSuccess) return fail(e, "normalize launch");
  note_normalized(h, panels_dev, dtilde_dev);
  // the traversal of a chunk's depths (Alg. 1 steps 3-4 of its nodes need only
  // their own normalization and the ancestors' X) waits for that chunk alone;
  // the second half of the batch follows the top nodes' normalization on the
  // traversal stream and waits for the same chunk events
  auto trav = [&](int q0, int q1) {
    if (bh > 0) return launch_halves(h, pl, aux, work_dev, panels_dev, x_dev, st, q0, q1, bh);
    if (groups) return launch_groups(h, pl, dpl, aux, panels_dev, x_dev, st, q0, q1, forked);
    return launch_run(pl, dpl, aux, h->is_complex(), h->opts.sched, panels_dev, x_dev, 0, h->grid, st, q0, q1);
  };
  if (bh > 0) {
    e = hipEventRecord(h->ev_tfork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(h->tst, h->ev_tfork, 0);
    if (e != hipSuccess) return fail(e, "traversal fork");
    forked = true;
  }
  e = trav(aux.lvl_cut[0], aux.lvl_cut[1]);
  for (int q = 1; q < nq && e == hipSuccess; ++q) {
    e = hipStreamWaitEvent(st, h->ev_chunk[q - 1], 0);
    if (e == hipSuccess && forked) e = hipStreamWaitEvent(h->tst, h->ev_chunk[q - 1], 0);
    if (e == hipSuccess) e = trav(aux.lvl_cut[q], aux.lvl_cut[q + 1]);
  }
  if (e == hipSuccess && forked) e = hipEventRecord(h->ev_tjoin, h->tst);
  if (e == hipSuccess && forked) e = hipStreamWaitEvent(st, h->ev_tjoin, 0);
  if (e != hipSuccess) return fail(e, "selinv launch");
  h->run_gen = h->gen;
  h->x_at = x_dev;
  return SELINV_OK;
}

selinv_status selinv_normalize_run_noalloc(selinv_ctx *h, const void *ldlt_dev, void *panels_dev, void *x_dev,
                                           void *dtilde_dev, void *stream) {
  if (!h) return SELINV_EINVAL;
  if (h->S.n == 0) return set_err(h, SELINV_ESTATE, "analyze did not succeed");
  if (!ldlt_dev || !panels_dev || !x_dev) return set_err(h, SELINV_EINVAL, "null buffer");
  if (dtilde_dev && h->is_lu()) return set_err(h, SELINV_EUNSUPPORTED, "no Dt output for the LU form");
  const int64_t need = h->H.off.fwd_end;
  if (need > kNoAllocBytes)
    return set_err(h, SELINV_ENOMEM,
                   "selinv_normalize_run_noalloc: this plan needs " + std::to_string(need) +
                       " bytes of work area, more than the fixed " + std::to_string(kNoAllocBytes) +
                       " (use selinv_normalize_run with a caller-allocated work buffer)",
                   need, kNoAllocBytes);
  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_err(h, e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  void *work = nullptr;
  selinv_status ss = scratch_for_device(h, dev, &work);
  if (ss != SELINV_OK) return ss;
  // this context's tables and plan into the work area, unless they are still
  // there from this context's previous call on this device
  if (g_scratch_owner[dev] != h->serial) {
    g_scratch_owner[dev] = 0;
    e = hipMemcpyAsync(work, h->image.data(), h->image.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_err(h, e, "table upload (no-alloc)");
    h->plan_noalloc = make_devplan(h, work);
    e = hipMemcpyAsync(static_cast<unsigned char *>(work) + h->H.off.plan, &h->plan_noalloc, sizeof(DevPlan),
                       hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_err(h, e, "plan upload (no-alloc)");
    e = hipStreamSynchronize(st);  // the host staging is reused
    if (e != hipSuccess) return hip_err(h, e, "table upload sync (no-alloc)");
    g_scratch_owner[dev] = h->serial;
  }
  int64_t budget = 0;
  ss = run_setup(h, &budget);
  if (ss != SELINV_OK) return ss;
  DevPlan pl = make_devplan(h, work);
  const DevPlan *dpl = dev_plan(h, work);
  LaunchAux aux = make_aux(h, work);
  e = launch_normalize(pl, dpl, aux, h->is_complex(), ldlt_dev, panels_dev, dtilde_dev, st, -1, NORM_ALL);
  if (e != hipSuccess) return hip_err(h, e, "normalize launch (no-alloc)");
  note_normalized(h, panels_dev, dtilde_dev);
  e = launch_run(pl, dpl, aux, h->is_complex(), h->opts.sched, panels_dev, x_dev, budget, h->grid, st, 0, aux.nlvl);
  if (e != hipSuccess) return hip_err(h, e, "selinv launch (no-alloc)");
  h->run_gen = h->gen;
  h->x_at = x_dev;
  h->ctrl_at = static_cast<unsigned char *>(work) + h->H.off.ctrl;
  return SELINV_OK;
}

selinv_status selinv_extract(const selinv_ctx *hc, const void *x_dev, void *work_dev, void *out_dev, void *stream) {
  selinv_ctx *h = const_cast<selinv_ctx *>(hc);
  if (!h) return SELINV_EINVAL;
  if (!x_dev || !out_dev || !work_dev) return set_err(h, SELINV_EINVAL, "null buffer");
  hipStream_t st = (hipStream_t)stream;
  selinv_status ss = ensure_uploaded(h, work_dev, st);
  if (ss != SELINV_OK) return ss;
  DevPlan pl = make_devplan(h, work_dev);
  hipError_t e = launch_extract(pl, dev_plan(h, work_dev), h->is_complex(), x_dev, out_dev, st);
  if (e != hipSuccess) return hip_err(h, e, "extract launch");
  return SELINV_OK;
}

selinv_status selinv_scatter(const selinv_ctx *hc, const void *vals_dev, void *work_dev, void *panel_dev,
                             void *stream) {
  selinv_ctx *h = const_cast<selinv_ctx *>(hc);
  if (!h) return SELINV_EINVAL;
  if (h->S.n == 0) return set_err(h, SELINV_ESTATE, "analyze did not succeed");
  if (!vals_dev || !panel_dev || !work_dev) return set_err(h, SELINV_EINVAL, "null buffer");
  if (h->is_lu()) return set_err(h, SELINV_EUNSUPPORTED, "selinv_scatter: not defined for the LU form");
  hipStream_t st = (hipStream_t)stream;
  selinv_status ss = ensure_uploaded(h, work_dev, st);
  if (ss != SELINV_OK) return ss;
  DevPlan pl = make_devplan(h, work_dev);
  hipError_t e = launch_scatter(pl, dev_plan(h, work_dev), h->is_complex(), vals_dev, panel_dev, st);
  if (e != hipSuccess) return hip_err(h, e, "scatter launch");
  return SELINV_OK;
}

selinv_status selinv_backward(selinv_ctx *h, const void *panels_dev, const void *x_dev, const void *dtilde_dev,
                              void *xbar_dev, const void *wlogdet_dev, void *work_dev, void *abar_dev,
                              void *stream) {
  if (!h) return SELINV_EINVAL;
  if (!h->factored) return set_err(h, SELINV_ESTATE, "selinv_backward before a successful selinv_factor");
  if (h->is_herm()) return set_err(h, SELINV_EUNSUPPORTED, "selinv_backward: no adjoint for Hermitian matrices");
  if (h->is_lu()) return set_err(h, SELINV_EUNSUPPORTED, "selinv_backward: no adjoint for the LU form");
  if (!h->H.adjoint)
    return set_err(h, SELINV_EUNSUPPORTED, "selinv_backward: the work area was sized without the adjoint's scratch "
                                           "(opts.adjoint < 0)");
  if (!panels_dev || !x_dev || !dtilde_dev || !xbar_dev || !work_dev || !abar_dev)
    return set_err(h, SELINV_EINVAL, "null buffer");
  if (h->dtilde_gen != h->gen || dtilde_dev != h->dtilde_at)
    return set_err(h, SELINV_ESTATE, "selinv_backward: dtilde_dev does not hold the Dt blocks of the last "
                                     "factorization (pass dtilde_dev to selinv_factor / selinv_normalize)");
  if (panels_dev != h->panels_at)
    return set_err(h, SELINV_ESTATE, "selinv_backward: panels_dev is not the buffer of the last factorization");
  if (h->run_gen != h->gen || x_dev != h->x_at)
    return set_err(h, SELINV_ESTATE, "selinv_backward: x_dev does not hold the selected inverse of the last "
                                     "factorization (call selinv_run after selinv_factor)");
  hipStream_t st = (hipStream_t)stream;
  selinv_status ss = ensure_uploaded(h, work_dev, st);
  if (ss != SELINV_OK) return ss;
  DevPlan pl = make_devplan(h, work_dev);
  LaunchAux aux = make_aux(h, work_dev);
  hipError_t e = launch_backward(pl, dev_plan(h, work_dev), aux, h->is_complex(), panels_dev, x_dev, dtilde_dev,
                                 xbar_dev, wlogdet_dev, abar_dev, st);
  if (e != hipSuccess) return hip_err(h, e, "backward launch");
  return SELINV_OK;
}

selinv_status selinv_logdet(const selinv_ctx *hc, double *out_host) {
  selinv_ctx *h = const_cast<selinv_ctx *>(hc);
  if (!h || !out_host) return SELINV_EINVAL;
  if (!h->have_logdet) return set_err(h, SELINV_ESTATE, "selinv_logdet before a successful factorization");
  for (int64_t l = 0; l < h->opts.batch; ++l) {
    if (h->is_complex()) {
      out_host[2 * l] = h->logdet[2 * l];
      out_host[2 * l + 1] = h->logdet[2 * l + 1];
    } else {
      out_host[l] = h->logdet[2 * l];
    }
  }
  return SELINV_OK;
}

selinv_status selinv_check_plan(const selinv_ctx *hc) {
  selinv_ctx *h = const_cast<selinv_ctx *>(hc);
  if (!h) return SELINV_EINVAL;
  if (h->S.n == 0) return set_err(h, SELINV_ESTATE, "analyze did not succeed");
  const HostPlan &H = h->H;
  const Symbolic &S = h->S;
  const int64_t ns = S.nsuper(), nit = (int64_t)H.items.size(), B = h->opts.batch;
  // Replay of the ticket protocol: running the tickets one at a time in
  // order, each item's dependencies must already be done when its turn comes.
  if ((int64_t)H.order.size() != B * nit)
    return set_err(h, SELINV_EINVAL, "plan check: ticket order has the wrong length", (int64_t)H.order.size(), B * nit);
  std::vector<int32_t> left((size_t)(B * ns * kPhases));
  std::vector<uint8_t> seen((size_t)(B * nit), 0);
  for (int64_t l = 0; l < B; ++l)
    for (int64_t K = 0; K < ns; ++K)
      for (int ph = 0; ph < kPhases; ++ph) left[(l * ns + K) * kPhases + ph] = phase_count(H, K, ph);
  for (int64_t t = 0; t < B * nit; ++t) {
    const int64_t id = H.order[t];
    if (id < 0 || id >= B * nit) return set_err(h, SELINV_EINVAL, "plan check: ticket names no item", t, id);
    const int64_t l = id / nit, itn = id % nit;
    if (seen[id]) return set_err(h, SELINV_EINVAL, "plan check: item holds two tickets", itn, l);
    seen[id] = 1;
    const Item it = H.items[itn];
    const int64_t K = it.K;
    const int ph = item_phase(it);
    const int32_t b = phase_begin(H, K, ph);
    if (itn < b || itn >= b + phase_count(H, K, ph))
      return set_err(h, SELINV_EINVAL, "plan check: item outside its phase range", K, itn);
    if (ph == 1 && (H.node_goff[K] >= 0) != (phase_count(H, K, 0) > 0))
      return set_err(h, SELINV_EINVAL, "plan check: dense buffer without gather items", K, l);
    // the kernel's wait rule: the previous non-empty phase, else the parent
    int pv = ph - 1;
    while (pv >= 0 && phase_count(H, K, pv) == 0) --pv;
    if (pv >= 0) {
      if (left[(l * ns + K) * kPhases + pv] != 0)
        return set_err(h, SELINV_EINVAL, "plan check: phase started before the previous one finished", K, l);
    } else {
      const int64_t P = H.node_parent[K];
      if (P != S.sparent[K]) return set_err(h, SELINV_EINVAL, "plan check: wrong parent table", K, P);
      if (P >= 0 && left[(l * ns + P) * kPhases + kPhases - 1] != 0)
        return set_err(h, SELINV_EINVAL, "plan check: node started before its parent finished", K, l);
    }
    --left[(l * ns + K) * kPhases + ph];
  }
  for (size_t q = 0; q < left.size(); ++q)
    if (left[q] != 0) return set_err(h, SELINV_EINVAL, "plan check: node never finished", (int64_t)(q / kPhases) % ns, (int64_t)(q / kPhases) / ns);
  // Normalization chunks of selinv_normalize_run: the level launches and each
  // normalization list are cut into consecutive ranges, and every level launch
  // touches only nodes normalized in its own chunk or an earlier one.
  const int64_t nlvl = (int64_t)H.lvl_ptr.size() - 1, nq = (int64_t)H.lvl_cut.size() - 1;
  if (nq < 1 || H.lvl_cut.front() != 0 || H.lvl_cut.back() != nlvl || (int64_t)H.norm_cut.size() != 5 * (nq + 1))
    return set_err(h, SELINV_EINVAL, "plan check: malformed normalization chunks", nq, nlvl);
  const int64_t sizes[5] = {(int64_t)H.small_nodes.size(), (int64_t)H.chunks_narrow.size(), (int64_t)H.chunks.size(),
                            (int64_t)H.rblocks.size(), (int64_t)H.sq_tiles.size()};
  for (int j = 0; j < 5; ++j) {
    if (H.norm_cut[j] != 0 || H.norm_cut[5 * nq + j] != sizes[j])
      return set_err(h, SELINV_EINVAL, "plan check: normalization chunks do not cover a list", j, nq);
    for (int64_t q = 0; q < nq; ++q)
      if (H.norm_cut[5 * q + j] > H.norm_cut[5 * (q + 1) + j] || H.lvl_cut[q] > H.lvl_cut[q + 1])
        return set_err(h, SELINV_EINVAL, "plan check: normalization chunks out of order", j, q);
  }
  std::vector<int64_t> nchunk(ns, -1);  // chunk of each node's normalization (its last entry)
  auto note = [&](int j, int64_t idx, int64_t K) {
    int64_t q = 0;
    while (idx >= H.norm_cut[5 * (q + 1) + j]) ++q;
    nchunk[K] = std::max(nchunk[K], q);
  };
  for (size_t i = 0; i < H.small_nodes.size(); ++i) note(0, (int64_t)i, H.small_nodes[i]);
  for (size_t i = 0; i < H.chunks_narrow.size(); ++i) note(1, (int64_t)i, H.chunks_narrow[i].x);
  for (size_t i = 0; i < H.chunks.size(); ++i) note(2, (int64_t)i, H.chunks[i].x);
  for (size_t i = 0; i < H.rblocks.size(); ++i) note(3, (int64_t)i, H.rblocks[i].x);
  for (size_t i = 0; i < H.sq_tiles.size(); ++i) note(4, (int64_t)i, H.sq_tiles[i].x);
  for (int64_t q = 0; q < nq; ++q)
    for (int64_t lv = H.lvl_cut[q]; lv < H.lvl_cut[q + 1]; ++lv)
      for (int32_t r = H.lvl_ptr[lv]; r < H.lvl_ptr[lv + 1]; ++r) {
        const int32_t kind = H.lvl_kind[lv];
        int64_t K;
        if (kind == LVL_PUSH)
          K = H.push[H.lvl_items[r]].I;
        else if (kind == LVL_Y128)
          K = H.y128[H.lvl_items[r]].K;
        else
          K = H.items[H.lvl_items[r]].K;
        if (nchunk[K] > q)
          return set_err(h, SELINV_EINVAL, "plan check: a level launch runs before its node is normalized", K, q);
      }
  // Subtree groups: the launches above the groups hold chain nodes only; the
  // ranges of every later launch cover it in order, each range one group
  // (1 or 2) that all its items belong to; and no node has an ancestor in
  // the other group, so the two streams share no X.
  if (H.grp_q >= 0) {
    const int32_t nl = (int32_t)H.lvl_ptr.size() - 1;
    auto node_at = [&](int32_t lv, int32_t r) -> int64_t {
      return H.lvl_kind[lv] == LVL_Y128 ? H.y128[H.lvl_items[r]].K : H.items[H.lvl_items[r]].K;
    };
    for (int32_t lv = 0; lv < nl; ++lv) {
      if (lv < H.grp_q) {
        for (int32_t r = H.lvl_ptr[lv]; r < H.lvl_ptr[lv + 1]; ++r)
          if (H.node_grp[node_at(lv, r)] != 0)
            return set_err(h, SELINV_EINVAL, "plan check: a launch above the subtree groups runs a group's node", lv, r);
        continue;
      }
      int32_t pos = H.lvl_ptr[lv];
      for (int32_t i = H.grp_rptr[lv]; i < H.grp_rptr[lv + 1]; ++i) {
        const int4 g = H.grp_ranges[i];
        if (g.y != lv || g.z != pos || g.w <= g.z || (g.x != 1 && g.x != 2))
          return set_err(h, SELINV_EINVAL, "plan check: subtree group ranges do not tile their launch", lv, i);
        for (int32_t r = g.z; r < g.w; ++r)
          if (H.node_grp[node_at(lv, r)] != g.x)
            return set_err(h, SELINV_EINVAL, "plan check: an item outside its range's group", lv, r);
        pos = g.w;
      }
      if (pos != H.lvl_ptr[lv + 1])
        return set_err(h, SELINV_EINVAL, "plan check: subtree group ranges do not cover their launch", lv, pos);
    }
    for (int64_t K = 0; K < ns; ++K)
      for (int64_t J = S.sparent[K]; J >= 0; J = S.sparent[J])
        if (H.node_grp[J] != 0 && H.node_grp[J] != H.node_grp[K])
          return set_err(h, SELINV_EINVAL, "plan check: a node with an ancestor in the other subtree group", K, J);
  }
  return SELINV_OK;
}

selinv_status selinv_items(const selinv_ctx *hc, int32_t which, const int32_t **items, int64_t *n) {
  selinv_ctx *h = const_cast<selinv_ctx *>(hc);
  if (!h || !items || !n) return SELINV_EINVAL;
  if (h->S.n == 0) return set_err(h, SELINV_ESTATE, "analyze did not succeed");
  if (which == 0) {
    *items = reinterpret_cast<const int32_t *>(h->H.items.data());
    *n = (int64_t)h->H.items.size();
    return SELINV_OK;
  }
  if (which == 2) {
    // the forward traversal's level launches in order (what the level and
    // push schedules launch): {kind, items per matrix, type of the first
    // item (-1 for a push launch), etree depth}
    if (h->lseq.empty()) {
      const HostPlan &H = h->H;
      int32_t depth = -1;  // a push launch follows the D step of its depth
      for (size_t q = 0; q + 1 < H.lvl_ptr.size(); ++q) {
        const int32_t first = H.lvl_ptr[q], cnt = H.lvl_ptr[q + 1] - first;
        int32_t type = -1;
        if (H.lvl_kind[q] == LVL_Y128) {
          const Item &it = H.y128[H.lvl_items[first]];
          type = it.type;
          depth = (int32_t)h->S.sdepth[it.K];
        } else if (H.lvl_kind[q] != LVL_PUSH) {
          const Item &it = H.items[H.lvl_items[first]];
          type = it.type;
          depth = (int32_t)h->S.sdepth[it.K];
        }
        h->lseq.push_back(Item{H.lvl_kind[q], cnt, type, depth});
      }
    }
    *items = reinterpret_cast<const int32_t *>(h->lseq.data());
    *n = (int64_t)h->lseq.size();
    return SELINV_OK;
  }
  if (which == 3) {
    // the normalization chunks of selinv_normalize_run: {first level launch,
    // etree depth of that launch, normalization work-list entries, 0}
    if (h->nseq.empty()) {
      const HostPlan &H = h->H;
      const int64_t nq = (int64_t)H.lvl_cut.size() - 1;
      for (int64_t q = 0; q < nq; ++q) {
        int32_t depth = 0;
        while (depth + 1 < (int32_t)H.lvl_depth_first.size() && H.lvl_depth_first[depth + 1] <= H.lvl_cut[q]) ++depth;
        int32_t entries = 0;
        for (int j = 0; j < 5; ++j) entries += H.norm_cut[5 * (q + 1) + j] - H.norm_cut[5 * q + j];
        h->nseq.push_back(Item{H.lvl_cut[q], depth, entries, 0});
      }
    }
    *items = reinterpret_cast<const int32_t *>(h->nseq.data());
    *n = (int64_t)h->nseq.size();
    return SELINV_OK;
  }
  if (which == 4) {
    // the subtree group ranges of a single-matrix level plan: {group, level
    // launch, first position, end position} (none without groups)
    *items = reinterpret_cast<const int32_t *>(h->H.grp_ranges.data());
    *n = (int64_t)h->H.grp_ranges.size();
    return SELINV_OK;
  }
  if (which != 1)
    return set_err(h, SELINV_EINVAL,
                   "selinv_items: which must be 0 (forward), 1 (adjoint), 2 (level launches), 3 (normalization "
                   "chunks) or 4 (subtree group ranges)");
  // the adjoint's launches in order, a small-node launch expanded into one
  // row per node
  if (h->bseq.empty()) {
    const HostPlan &H = h->H;
    for (const int4 &bl : H.blaunch) {
      if (bl.x == 0) {
        for (int32_t q = bl.y; q < bl.y + bl.z; ++q) h->bseq.push_back(H.bitems[q]);
      } else {
        for (int32_t q = bl.y; q < bl.y + bl.z; ++q)
          h->bseq.push_back(Item{H.tiny[q].K, bl.x == 1 ? BI_TINY_R1 : BI_TINY_R3, 0, 0});
      }
    }
  }
  *items = reinterpret_cast<const int32_t *>(h->bseq.data());
  *n = (int64_t)h->bseq.size();
  return SELINV_OK;
}

selinv_status selinv_trace(selinv_ctx *h, void *trace_dev) {
  if (!h) return SELINV_EINVAL;
  h->trace = trace_dev;
  h->uploaded_to = nullptr;  // the device copies of the plan carry the pointer
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  for (uint64_t &o : g_scratch_owner)
    if (o == h->serial) o = 0;
  return SELINV_OK;
}

selinv_status selinv_sync(selinv_ctx *h, void *stream) {
  if (!h) return SELINV_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_err(h, e, "stream synchronize");
  if (h->devfac_work) {  // pivots and log det of the last device factorization
    const int64_t B = h->opts.batch;
    const unsigned char *b = static_cast<const unsigned char *>(h->devfac_work);
    std::vector<unsigned long long> ferr((size_t)B);
    std::vector<double> ld((size_t)(2 * B));
    e = hipMemcpy(ferr.data(), b + h->H.off.ferr, sizeof(unsigned long long) * B, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(ld.data(), b + h->H.off.fldet, sizeof(double) * 2 * B, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_err(h, e, "factor status readback");
    h->devfac_work = nullptr;
    for (int64_t l = 0; l < B; ++l)
      if (ferr[l] != ~0ull) return set_err(h, SELINV_ESINGULAR, "zero or non-finite pivot", (int64_t)ferr[l], l);
    h->logdet = ld;
    h->have_logdet = true;
  }
  if (h->ctrl_at && h->opts.sched == SELINV_SCHED_PERSISTENT) {
    int32_t ctrl[4] = {0, 0, 0, 0};
    e = hipMemcpy(ctrl, h->ctrl_at, sizeof(ctrl), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_err(h, e, "control readback");
    if (ctrl[CTRL_ERR] == 2)
      return set_err(h, SELINV_EDEVICE, "persistent scheduler: a workgroup drew more tickets than there are items");
    if (ctrl[CTRL_ERR] != 0)
      return set_err(h, SELINV_EDEVICE, "persistent scheduler watchdog expired (an item waited too long for its dependencies)");
  }
  return SELINV_OK;
}

const char *selinv_last_error(const selinv_ctx *h) { return h ? h->err.c_str() : "null context"; }

int64_t selinv_error_info(const selinv_ctx *h, int which) {
  if (!h || which < 0 || which > 1) return -1;
  return h->info[which];
}

void selinv_destroy(selinv_ctx *h) { delete h; }

}  // extern "C"
