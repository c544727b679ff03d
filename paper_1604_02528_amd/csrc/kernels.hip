// HIP kernels of the selected-inversion library for gfx950 (CDNA4).
//
//  normalize  Alg. 1 steps 1-2 in LDL^T form (LU form: both panel sets):
//             L_KK^{-1} into scratch (strip-wise forward substitution),
//             Lhat_{C,K} = L_{C,K} L_KK^{-1} (MFMA, in place),
//             Dt_K = L_KK D_K L_KK^T (optional, for the adjoint) and
//             Dt_K^{-1} = L_KK^{-T} D_K^{-1} L_KK^{-1} into the panel's top block.
//  selinv     Alg. 1 second loop (root first): per supernode K the gather of
//             X_{C,C} through the ancestor maps (on the fly, or once into a
//             dense buffer), GEMM-1 X_{C,K} = -X_{C,C} Lhat_{C,K} and GEMM-2
//             X_KK = Dt^{-1} - Lhat^T X_{C,K} on FP64 MFMA
//             (v_mfma_f64_16x16x4f64; complex128 by four real products, or
//             three in the dense GEMM-1, GEMM-2 and normalization kernels),
//             the diagonal-block symmetrization of Section 2.3, coalesced
//             stores.  Scheduled level by level (one launch per etree depth
//             and phase, each phase in a kernel sized for it), by one
//             persistent launch whose workgroups draw tickets and wait on
//             per-node dependency counters (the device counterpart of the
//             task dependencies of Section 3), or in the push form of Alg. 2.
//  extract    X on A's pattern.
//
// MFMA f64 16x16x4 operand layout (measured on gfx950): lane l holds
// A[l % 16][l / 16], B[l / 16][l % 16] and D[4 v + l / 16][l % 16] in its v-th
// accumulator register.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"
#include "scalar.hpp"
#include "items.hpp"
#include "tile.hpp"

namespace selinv {

// ---------------------------------------------------------------------------
// Schedules
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(NT, Planes<T>::P == 1 ? 2 : 1) k_items_list(const DevPlan *__restrict__ plp, const T *Lp, T *Xp, T *Pp, const LRec *recs,
                                                   const int32_t *list, int32_t count, int32_t list_pos) {
  const DevPlan &pl = *plp;
  __shared__ double smem[smem_doubles<T>()];
  __shared__ int64_t rt[128];
  const int64_t g = blockIdx.x;
  const int64_t l = g / count;
  const int64_t q = g - l * count;
  const int64_t t_start = pl.trace ? wall_clock64() : 0;
  Ctx<T> cx{&pl, Lp + l * pl.panel_elems, Xp + l * pl.panel_elems, Pp + l * pl.part_elems,
            static_cast<T *>(pl.gbuf) + l * pl.g_elems, static_cast<T *>(pl.ypart) + l * pl.y_elems};
  // the record carries the item and its node: one dependent load before the operands
  const LRec rec = recs[q];
  do_item<T, false>(cx, rec.it, uniform(rec.nd), smem, rt);
  if (pl.trace) {
    __syncthreads();
    if (threadIdx.x == 0) {  // row of this item in the trace: levels in order, matrices inside a level
      int64_t *tr = pl.trace + 8 * ((int64_t)list_pos * pl.batch + g);
      tr[0] = l * pl.nitems + list[q];
      tr[1] = blockIdx.x;
      tr[2] = t_start;
      tr[3] = t_start;
      tr[4] = wall_clock64();
    }
  }
}

// Gathers of X_{C,C} into the dense buffers (the G items of a depth, Alg. 1
// step 3): three dependent rounds of loads per 64 x 64 block and no MFMA,
// so the kernel takes one tile of LDS and few registers, and twice as many
// workgroups share a CU as in k_items_list (more loads in flight).
template <typename T, bool LU>
__global__ void __launch_bounds__(NT, Planes<T>::P == 1 && !LU ? 4 : 2) k_gather_list(const DevPlan *__restrict__ plp, T *Xp,
                                                                              const LRec *recs, const int32_t *list,
                                                                              int32_t count, int32_t list_pos) {
  const DevPlan &pl = *plp;
  __shared__ double smem[tile_doubles<T>()];
  __shared__ int64_t rt[128];
  const int64_t g = blockIdx.x;
  const int64_t l = g / count;
  const int64_t q = g - l * count;
  const int64_t t_start = pl.trace ? wall_clock64() : 0;
  Ctx<T> cx{&pl, nullptr, Xp + l * pl.panel_elems, nullptr, static_cast<T *>(pl.gbuf) + l * pl.g_elems, nullptr};
  const LRec rec = recs[q];
  const Item it = uniform(rec.it);
  do_gtile<T, LU>(cx, uniform(rec.nd), it.a, it.b, smem, rt, cx.Xp);
  if (pl.trace) {
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t *tr = pl.trace + 8 * ((int64_t)list_pos * pl.batch + g);
      tr[0] = l * pl.nitems + list[q];
      tr[1] = blockIdx.x;
      tr[2] = t_start;
      tr[3] = t_start;
      tr[4] = wall_clock64();
    }
  }
}

// GEMM-2 shares of a depth (the R and P items, Alg. 1 step 4): one tile of
// LDS and no GEMM-1 operand stages (and, for complex, no Lhat prefetch), so
// that two workgroups share a CU also for complex (one in k_items_list).
template <typename T>
__global__ void __launch_bounds__(NT, 2) k_gemm2_list(const DevPlan *__restrict__ plp, const T *Lp,
                                                                             T *Xp, T *Pp, const LRec *recs,
                                                                             const int32_t *list, int32_t count,
                                                                             int32_t list_pos) {
  const DevPlan &pl = *plp;
  __shared__ double smem[tile_doubles<T>()];
  const int64_t g = blockIdx.x;
  const int64_t l = g / count;
  const int64_t q = g - l * count;
  const int64_t t_start = pl.trace ? wall_clock64() : 0;
  Ctx<T> cx{&pl, Lp + l * pl.panel_elems, Xp + l * pl.panel_elems, Pp + l * pl.part_elems, nullptr,
            static_cast<T *>(pl.ypart) + l * pl.y_elems};
  const LRec rec = recs[q];
  const Item it = uniform(rec.it);
  constexpr bool PF = Planes<T>::P == 1;  // FP64 keeps the prefetch within two workgroups per CU
  if (it.type == ITEM_R)
    do_rtile<T, false, PF>(cx, uniform(rec.nd), it.a, it.b, smem);
  else
    do_ptile<T, false, PF>(cx, uniform(rec.nd), it.a, it.b, smem);
  if (pl.trace) {
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t *tr = pl.trace + 8 * ((int64_t)list_pos * pl.batch + g);
      tr[0] = l * pl.nitems + list[q];
      tr[1] = blockIdx.x;
      tr[2] = t_start;
      tr[3] = t_start;
      tr[4] = wall_clock64();
    }
  }
}

// GEMM-1 tiles of nodes with a dense X_{C,C} buffer (see do_ytile_dense),
// each followed by its GEMM-2 share when unsplit: dense loaders only, so it
// fits two workgroups per CU also for complex.
template <typename T>
__global__ void __launch_bounds__(NT, 2) k_ydense(const DevPlan *__restrict__ plp, const T *Lp, T *Xp, T *Pp,
                                                  const LRec *recs, const int32_t *list, int32_t count,
                                                  int32_t list_pos) {
  const DevPlan &pl = *plp;
  constexpr int kStages = 2 * dense_stage_doubles<T, DenseTK<T>::TK>();
  __shared__ double smem[kStages > tile_doubles<T>() ? kStages : tile_doubles<T>()];
  const int64_t g = blockIdx.x;
  const int64_t l = g / count;
  const int64_t q = g - l * count;
  const int64_t t_start = pl.trace ? wall_clock64() : 0;
  Ctx<T> cx{&pl, Lp + l * pl.panel_elems, Xp + l * pl.panel_elems, Pp + l * pl.part_elems,
            static_cast<T *>(pl.gbuf) + l * pl.g_elems, static_cast<T *>(pl.ypart) + l * pl.y_elems};
  const LRec rec = recs[q];
  const Item it = uniform(rec.it);
  do_ytile_dense<T>(cx, uniform(rec.nd), it.a, it.b, it.type == ITEM_YU, smem);
  if (pl.trace) {
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t *tr = pl.trace + 8 * ((int64_t)list_pos * pl.batch + g);
      tr[0] = l * pl.nitems + list[q];
      tr[1] = blockIdx.x;
      tr[2] = t_start;
      tr[3] = t_start;
      tr[4] = wall_clock64();
    }
  }
}

// Push-form tiles of one etree depth (see PushRec): a gathered GEMM-1 tile
// over the ancestor's share of X_{C(I),C(I)}, subtracted from X_{C(I),I}.
// No two tiles of a launch touch the same entries: the ancestors of I form a
// chain, so one depth holds at most one of them, and its tiles of I cover
// distinct rows and columns.
template <typename T>
__global__ void __launch_bounds__(NT, Planes<T>::P == 1 ? 2 : 1)
    k_push(const DevPlan *__restrict__ plp, const T *Lp, T *Xp, const PushRec *recs, int32_t count, int32_t list_pos) {
  const DevPlan &pl = *plp;
  __shared__ double smem[smem_doubles<T>()];
  __shared__ int64_t rt[128];
  const int64_t g = blockIdx.x;
  const int64_t l = g / count;
  const int64_t q = g - l * count;
  const int64_t t_start = pl.trace ? wall_clock64() : 0;
  const PushRec r = recs[q];
  const int I = uniform(r.I), i0 = uniform(r.i0), x0 = uniform(r.x0), st = uniform(r.st);
  const int en = uniform(r.en), kend = uniform(r.kend);
  const NodeInfo nd = node_info(pl, I);
  const int s = nd.s, c = nd.c, ld = s + c;
  const T *L = Lp + l * pl.panel_elems;
  T *X = Xp + l * pl.panel_elems;
  if (threadIdx.x < 64) {
    const int ig = i0 + threadIdx.x;
    rt[threadIdx.x] = gp(pl.kcol)[nd.rp + (ig < c ? ig : 0)];
    rt[64 + threadIdx.x] = gp(pl.kpos)[nd.rp + (ig < c ? ig : 0)];
  }
  lds_barrier();
  LoadGatherSeg<T, false> la;
  la.X = X;
  la.kcol = pl.kcol + nd.rp;
  la.kpos = pl.kpos + nd.rp;
  la.posarr = pl.posarr;
  la.rt_col = rt;
  la.rt_pos = rt + 64;
  la.c = c;
  la.kend = kend;
  la.i0 = i0;
  la.en = en;
  la.cs = pl.csign;
  LoadPanelK<T, false> lb{L, nd.off, ld, s, 0, kend, x0, s};
  Acc<T> acc;
  gemm_tile<T>(st, kend, la, lb, smem, acc);
  acc_to_lds<T>(acc, smem);
  lds_barrier();
  T *Y = X + nd.off + s;
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = e & 63, j = e >> 6;
    if (i0 + i < c && x0 + j < s) {
      T *p = Y + (int64_t)(x0 + j) * ld + i0 + i;
      gstore(p, gload(p) - lds_get<T>(smem, i, j));
    }
  }
  if (pl.trace) {
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t *tr = pl.trace + 8 * ((int64_t)list_pos * pl.batch + g);
      tr[0] = -1 - q;  // push tiles are not items: the row names the record
      tr[1] = blockIdx.x;
      tr[2] = t_start;
      tr[3] = t_start;
      tr[4] = wall_clock64();
    }
  }
}

// GEMM-1 of FP64 dense-buffer nodes on 128 x 128 tiles (the tune table's
// tile choice): record {K, type, a, b} names the node, 128-row tile a of C(K)
// and, in b, the 128-column tile of K (low 16 bits) and the contraction part
// (high bits).  No GEMM-2 here (ITEM_P items run it); the tile goes to X (-acc) or
// to the split contraction's partial tiles.  Each lane stores its
// accumulator elements directly: per store, the four lanes of a block column
// write four consecutive rows (32 bytes).
__global__ void __launch_bounds__(NT, 2) k_ydense128(const DevPlan *__restrict__ plp, const double *Lp, double *Xp,
                                                     const Item *recs, int32_t count, int32_t list_pos) {
  const DevPlan &pl = *plp;
  __shared__ double smem[2 * stage128_doubles()];
  const int64_t g = blockIdx.x;
  const int64_t l = g / count;
  const int64_t q = g - l * count;
  const int64_t t_start = pl.trace ? wall_clock64() : 0;
  const Item it = uniform(gload(recs + q));
  const NodeInfo nd = node_info(pl, it.K);
  const int s = nd.s, c = nd.c, ld = s + c;
  const int part = it.b >> 16;
  const int kb = part * nd.kchunk, ke = min(c, kb + nd.kchunk);
  const int i0 = it.a * 128, j0 = (it.b & 0xffff) * 128;
  const double *G = static_cast<const double *>(pl.gbuf) + l * pl.g_elems + nd.goff;
  LoadDenseA128 la{G, nd.ldg, c, ke, i0};
  LoadDenseB128 lb{Lp + l * pl.panel_elems, nd.off, ld, s, ke, j0, s};
  Acc128 acc;
  gemm_dense128(kb, ke, la, lb, smem, acc);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w & 1, wj = w >> 1;
  const bool to_x = nd.yoff < 0;
  double *dst = to_x ? Xp + l * pl.panel_elems + nd.off + s
                     : static_cast<double *>(pl.ypart) + l * pl.y_elems + nd.yoff + (int64_t)part * c * s;
  const int64_t ldd = to_x ? ld : c;
  const double sg = to_x ? -1.0 : 1.0;
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      // accumulator element v of a lane: row 4 v + lane / 16, column lane % 16 of the block
      const int j = j0 + 64 * wj + 16 * bj + (lane & 15);
      const int ib = i0 + 64 * wi + 16 * bi + (lane >> 4);
      if (j < s) {
        double *col = dst + (int64_t)j * ldd;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (ib + 4 * v < c) gstore(col + ib + 4 * v, sg * acc.v[bi][bj][v]);
      }
    }
  if (pl.trace) {
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t *tr = pl.trace + 8 * ((int64_t)list_pos * pl.batch + g);
      tr[0] = -1 - q;  // 128-tile records are not items: the row names the record
      tr[1] = blockIdx.x;
      tr[2] = t_start;
      tr[3] = t_start;
      tr[4] = wall_clock64();
    }
  }
}

// Small nodes of one level, one wavefront each (see do_tiny).
template <typename T, bool HERM>
__global__ void __launch_bounds__(64) k_tiny(const DevPlan *__restrict__ plp, const T *Lp, T *Xp,
                                             const TinyRec *__restrict__ recs, int32_t count, int32_t list_pos) {
  const DevPlan &pl = *plp;
  __shared__ T ls[kTinyS * tiny_ldc<T>()], ys[kTinyS * tiny_ldc<T>()];
  const int64_t g = blockIdx.x;
  const int64_t l = g / count;
  const TinyRec r = recs[g - l * count];
  const int64_t t_start = pl.trace ? wall_clock64() : 0;
  const T *L = Lp + l * pl.panel_elems;
  T *X = Xp + l * pl.panel_elems;
  if (r.c <= 8)
    do_tiny<T, 8, HERM>(r, pl.toff, L, X, ls, ys);
  else if (r.c <= 16)
    do_tiny<T, 16, HERM>(r, pl.toff, L, X, ls, ys);
  else if constexpr (sizeof(T) == 16)  // complex launches send c > kTinyC to k_tiny64
    do_tiny<T, 32, HERM>(r, pl.toff, L, X, ls, ys);
  else if (r.c <= 32)
    do_tiny<T, 32, HERM>(r, pl.toff, L, X, ls, ys);
  else
    do_tiny64<T>(r, pl.toff, L, X, ls, ys);
  if (pl.trace) {
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t *tr = pl.trace + 8 * ((int64_t)list_pos * pl.batch + g);
      tr[0] = l * pl.nitems + r.it;
      tr[1] = blockIdx.x;
      tr[2] = t_start;
      tr[3] = t_start;
      tr[4] = wall_clock64();
    }
  }
}

// Complex single-wavefront nodes with kTinyC < c <= kTinyCF (the
// forward-only part of a depth's list): do_tiny64, in a kernel of its own so
// that the narrower nodes keep k_tiny's registers and LDS.
template <typename T, bool HERM>
__global__ void __launch_bounds__(64) k_tiny64(const DevPlan *__restrict__ plp, const T *Lp, T *Xp,
                                               const TinyRec *__restrict__ recs, int32_t count, int32_t list_pos) {
  const DevPlan &pl = *plp;
  __shared__ T ls[kTinyS * kTinyCF], ys[kTinyS * kTinyCF];
  const int64_t g = blockIdx.x;
  const int64_t l = g / count;
  const TinyRec r = recs[g - l * count];
  const int64_t t_start = pl.trace ? wall_clock64() : 0;
  do_tiny64<T, HERM>(r, pl.toff, Lp + l * pl.panel_elems, Xp + l * pl.panel_elems, ls, ys);
  if (pl.trace) {
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t *tr = pl.trace + 8 * ((int64_t)list_pos * pl.batch + g);
      tr[0] = l * pl.nitems + r.it;
      tr[1] = blockIdx.x;
      tr[2] = t_start;
      tr[3] = t_start;
      tr[4] = wall_clock64();
    }
  }
}

// Scheduler atomics (agent scope, relaxed).  Producers order their data
// stores before a counter update with a release fence; consumers spin on the
// counter with relaxed loads and then read the data with plain loads (the
// coherence argument is given at the release fence below).
__device__ __forceinline__ int32_t ld_relaxed(const int32_t *p) {
  return __hip_atomic_load(gp(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(int32_t *p, int32_t v) {
  __hip_atomic_store(gw(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t add_relaxed(int32_t *p, int32_t v) {
  return __hip_atomic_fetch_add(gw(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reset the dependency counters and the control words.
__global__ void k_sched_init(const DevPlan *__restrict__ plp) {
  const DevPlan &pl = *plp;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t nsb = pl.batch * pl.ns;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nsb; i += stride) {
    const int64_t K = i % pl.ns;
#pragma unroll
    for (int ph = 0; ph < kPhases; ++ph) gw(pl.cnt)[ph * nsb + i] = gp(pl.nph)[ph * pl.ns + K];
  }
  if (blockIdx.x == 0 && threadIdx.x < CTRL_WORDS) gw(pl.ctrl)[threadIdx.x] = 0;
}

// Wait (executed by one whole wave, with wave-uniform control flow) until
// item `it` of matrix l may run: an item waits for the previous non-empty
// phase of its node; an item of the node's first phase waits for the node's
// parent to finish (a root's first items are ready at once).  Returns false
// when another workgroup raised the error flag or when this wait alone has
// spun for more than budget_ticks device clock ticks (then it raises the
// flag): a long traversal is never cut short, only a dependency that does
// not arrive.
__device__ bool wait_ready(const DevPlan &pl, int64_t l, const Item &it, int64_t budget_ticks) {
  const int64_t nsb = pl.batch * pl.ns;
  int pv = item_phase(it.type) - 1;
  while (pv >= 0 && uniform(gp(pl.nph)[pv * pl.ns + it.K]) == 0) --pv;
  const int32_t *ctr;
  if (pv >= 0) {
    ctr = pl.cnt + pv * nsb + l * pl.ns + it.K;
  } else {
    const int32_t P = uniform(gp(pl.node_parent)[it.K]);
    if (P < 0) return true;
    ctr = pl.cnt + (kPhases - 1) * nsb + l * pl.ns + P;
  }
  int backoff = 1;
  const int64_t t_begin = wall_clock64();
  while (uniform(ld_relaxed(ctr)) != 0) {
    if (uniform(ld_relaxed(pl.ctrl + CTRL_ERR)) != 0) return false;
    if (wall_clock64() - t_begin > budget_ticks) {
      if ((threadIdx.x & 63) == 0) st_relaxed(pl.ctrl + CTRL_ERR, 1);
      return false;
    }
    for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(1);
    backoff = backoff < 8 ? 2 * backoff : 8;
  }
  return true;
}

// Persistent traversal: every workgroup draws tickets from one counter and
// runs the items of the ticket order (a topological order of the dependency
// graph), each after its own dependencies are done.  The ticket draw, the
// wait and the counter update are done by wave 0 as a whole; every branch
// around a barrier is wave-uniform.  Exits: the tickets run out, the error
// flag is up (checked at every draw), a wait expires, or a workgroup has
// drawn more tickets than there are items (impossible unless the loop
// misbehaves; it then raises the flag instead of spinning on).
template <typename T>
__global__ void __launch_bounds__(NT, 1)
    k_persistent(const DevPlan *__restrict__ plp, const T *Lp, T *Xp, T *Pp, int64_t budget_ticks) {
  const DevPlan &pl = *plp;
  __shared__ double smem[smem_doubles<T>()];
  __shared__ int64_t rt[128];
  __shared__ int32_t s_id, s_ticket;
  __shared__ int64_t s_tpop;
  const int64_t total = pl.batch * pl.nitems;
  const bool wave0 = uniform((int32_t)threadIdx.x) < 64;
  const bool lane0 = threadIdx.x == 0;
  int64_t draws = 0;
  while (true) {
    if (wave0) {
      int32_t id = -1;
      int32_t t = 0;
      int64_t t_draw = 0;
      if (uniform(ld_relaxed(pl.ctrl + CTRL_ERR)) != 0) {
        id = -2;
      } else if (++draws > total + 1) {
        if (lane0) st_relaxed(pl.ctrl + CTRL_ERR, 2);
        id = -2;
      } else {
        if (lane0) t = add_relaxed(pl.ctrl + CTRL_TICKET, 1);
        t = uniform(t);
        t_draw = pl.trace ? wall_clock64() : 0;
        if (t < total) {
          id = uniform(gp(pl.order)[t]);
          const int64_t l = id / pl.nitems;
          if (!wait_ready(pl, l, uniform(gload(pl.items + (id - l * pl.nitems))), budget_ticks)) id = -2;
        }
      }
      if (lane0) {
        s_id = id;
        s_ticket = t;
        s_tpop = t_draw;
      }
    }
    __syncthreads();
    const int32_t id = uniform(s_id);
    if (id < 0) break;
    const int64_t t_start = pl.trace ? wall_clock64() : 0;
    const int64_t l = id / pl.nitems;
    const int32_t itn = (int32_t)(id - l * pl.nitems);
    const Item it = uniform(gload(pl.items + itn));
    Ctx<T> cx{&pl, Lp + l * pl.panel_elems, Xp + l * pl.panel_elems, Pp + l * pl.part_elems,
            static_cast<T *>(pl.gbuf) + l * pl.g_elems, static_cast<T *>(pl.ypart) + l * pl.y_elems};
    do_item<T, false>(cx, it, node_info(pl, it.K), smem, rt);
    // Publishing protocol: write back this item's stores (agent-scope release)
    // before the counter update.  Readers use plain cached loads: every panel
    // and partial block starts on its own cache line, and a node's data is
    // read only after the node has completed, so no cache can hold a line of
    // it from before it was written (caches start clean at kernel launch).
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (wave0 && lane0) {
      if (pl.trace) {
        int64_t *tr = pl.trace + 8 * (int64_t)s_ticket;
        tr[0] = id;
        tr[1] = blockIdx.x;
        tr[2] = s_tpop;
        tr[3] = t_start;
        tr[4] = wall_clock64();
      }
      add_relaxed(pl.cnt + item_phase(it.type) * pl.batch * pl.ns + l * pl.ns + it.K, -1);
    }
  }
}

// ---------------------------------------------------------------------------
// Normalization (Alg. 1 steps 1-2)
// ---------------------------------------------------------------------------

// L_KK^{-1} and D_K^{-1} (Alg. 1 step 1, with the LDL^T factor of Section
// 2.3: L_KK is unit lower triangular, its diagonal slot holds D).  The
// columns of X = L_KK^{-1} are independent: one workgroup per 16-column block
// [j0, j0 + 16) of one node solves L_KK X(:, J) = I(:, J) by forward
// substitution down 16-row strips, with X(:, J) held in LDS.  Strip I:
//   X(I, J) = I(I, J) - L(I, j0:I0) X(j0:I0, J)   (one 16 x 16 MFMA product:
//   the four waves take interleaved 4-deep slices of the contraction and sum
//   their partials through LDS; complex in the 3M form)
// then the 16 x 16 unit triangular solve with L(I, I) (one thread per column).
// The L strip of the next row block is loaded while the current one is used.
// MAXS bounds s for the nodes of the launch (256, or 64 for a launch of narrow
// nodes with a quarter of the LDS, so that more workgroups share a CU).
// LU plans launch nsets = 2 grids' worth of workgroups: the second half
// works on the second panel set, U^T, whose unit lower diagonal block gives
// U_KK^{-T} (into the second half of the linv buffer); D_K^{-1} is written by
// the first half only.
template <typename T, int MAXS>
__global__ void __launch_bounds__(NT) k_normalize_inv(const DevPlan *__restrict__ plp, const T *Src_all, const int2 *chunks,
                                                      int32_t nchunks, int nsets) {
  constexpr int P = Planes<T>::P, XP = 17, LPI = MAXS + 1, U = MAXS / 16;
  const DevPlan &pl = *plp;
  __shared__ double xs[P][MAXS * XP];  // X(j0 + r, j0 + q) at [r * XP + q]
  __shared__ double lsd[P][16 * LPI];  // L(I0 + i, j0 + k) at [i * LPI + k]
  __shared__ double red[P][4 * 256];   // the waves' 16 x 16 partial products, [w * 256 + i * 16 + q]
  const int64_t per = (int64_t)nchunks * pl.batch;  // workgroups per panel set
  const int hs = nsets > 1 ? (int)(blockIdx.x / per) : 0;
  const int64_t g = blockIdx.x - hs * per;
  const int64_t l = g / nchunks;
  const int2 ck = chunks[g - l * nchunks];
  const int K = uniform(ck.x), j0 = uniform(ck.y) * 16;
  const int s = uniform(gp(pl.node_s)[K]), c = gp(pl.node_c)[K], ld = s + c;
  const T *Q = Src_all + l * pl.panel_elems + hs * pl.half + gp(pl.node_off)[K];  // LDL^T panel (read only)
  T *Linv = reinterpret_cast<T *>(pl.linv) + (hs * pl.batch + l) * pl.sq_elems + gp(pl.node_sq)[K];
  T *dinv = reinterpret_cast<T *>(pl.dinv) + l * pl.n + gp(pl.node_first)[K];
  const int w = min(16, s - j0);
  const int t = threadIdx.x;
  if (t < w && hs == 0) gstore(dinv + j0 + t, SOps<T>::div(SOps<T>::one(), Q[(int64_t)(j0 + t) * ld + j0 + t]));
  // strip element u of thread t: i = e & 15, k = e >> 4 with e = t + NT u (k < MAXS)
  auto strip_ok = [&](int I0, int u) {
    const int e = t + NT * u, i = e & 15, k = e >> 4;
    return k < min(I0 + 16, s) - j0 && I0 + i < s;
  };
  T pre[U];
  auto load_strip = [&](int I0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = t + NT * u, i = e & 15, k = e >> 4;
      pre[u] = gload(Q + (((int64_t)(j0 + k) * ld + I0 + i) & opaque_mask(strip_ok(I0, u))));
    }
  };
  load_strip(j0);
  const int ti = t & 15, tq = t >> 4;
  for (int I0 = j0; I0 < s; I0 += 16) {
    const int h = min(16, s - I0), r0 = I0 - j0;
    lds_barrier();
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = t + NT * u, i = e & 15, k = e >> 4;
      const T v = masked(pre[u], opaque_mask(strip_ok(I0, u)));
#pragma unroll
      for (int p = 0; p < P; ++p) lsd[p][i * LPI + k] = Planes<T>::get(v, p);
    }
    if (I0 + 16 < s) load_strip(I0 + 16);
    lds_barrier();
    // X(I0 + ti, j0 + tq) before the diagonal block: identity minus the
    // earlier strips, L(I, j0:I0) X(j0:I0, J) on MFMA (lane l of a wave
    // holds A(l % 16, l / 16), B(l / 16, l % 16) and the result rows
    // 4 v + l / 16 of column l % 16)
    {
      constexpr int C = P == 1 ? 1 : 3;  // product chains (3M for complex)
      const int lane = t & 63, wv = t >> 6, m = lane & 15;
      d4 pc[C];
#pragma unroll
      for (int q = 0; q < C; ++q) pc[q] = d4{0.0, 0.0, 0.0, 0.0};
      for (int k0 = 4 * wv; k0 < r0; k0 += 16) {
        const int ka = k0 + (lane >> 4);
        if constexpr (P == 1) {
          pc[0] = mfma16(lsd[0][m * LPI + ka], xs[0][ka * XP + m], pc[0]);
        } else {
          const double a0 = lsd[0][m * LPI + ka], a1 = lsd[1][m * LPI + ka];
          const double b0 = xs[0][ka * XP + m], b1 = xs[1][ka * XP + m];
          pc[0] = mfma16(a0, b0, pc[0]);
          pc[1] = mfma16(a1, b1, pc[1]);
          pc[2] = mfma16(a0 + a1, b0 + b1, pc[2]);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int o = wv * 256 + (4 * v + (lane >> 4)) * 16 + m;
        if constexpr (P == 1) {
          red[0][o] = pc[0][v];
        } else {
          red[0][o] = pc[0][v] - pc[1][v];
          red[1][o] = pc[2][v] - pc[0][v] - pc[1][v];
        }
      }
    }
    lds_barrier();
    if (ti < h) {
      T acc = (I0 + ti == j0 + tq) ? SOps<T>::one() : zero_of<T>();
#pragma unroll
      for (int wq = 0; wq < 4; ++wq) acc -= Planes<T>::from(&red[0][wq * 256 + ti * 16 + tq], 4 * 256);
#pragma unroll
      for (int p = 0; p < P; ++p) xs[p][(r0 + ti) * XP + tq] = Planes<T>::get(acc, p);
    }
    lds_barrier();
    // unit lower triangular solve with L(I, I), one thread per column
    if (t < 16) {
      T xv[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        if (i < h) {
          T v = Planes<T>::from(&xs[0][(r0 + i) * XP + t], MAXS * XP);
#pragma unroll
          for (int k = 0; k < i; ++k) v -= Planes<T>::from(&lsd[0][i * LPI + r0 + k], 16 * LPI) * xv[k];
          xv[i] = v;
#pragma unroll
          for (int p = 0; p < P; ++p) xs[p][(r0 + i) * XP + t] = Planes<T>::get(v, p);
        }
      }
    }
  }
  lds_barrier();
  // whole columns j0 .. j0 + w - 1 of L_KK^{-1} (column-major, ld s), zeros above the diagonal
  for (int q = 0; q < w; ++q)
    for (int r = t; r < s; r += NT)
      gstore(Linv + (int64_t)(j0 + q) * s + r,
             r < j0 ? zero_of<T>() : Planes<T>::from(&xs[0][(r - j0) * XP + q], MAXS * XP));
}

// All of the normalization (Alg. 1 steps 1-2, LDL^T form of Section 2.3) of
// a node with s <= kSmallNormS in one wavefront: L_KK^{-1} by forward
// substitution (lane q owns column q), D^{-1}, Dt^{-1} = L_KK^{-T} D^{-1}
// L_KK^{-1} into the top block, Dt = L_KK D L_KK^T when dt is given (^H for
// ^T in a Hermitian plan), and
// Lhat_{C,K} = L_{C,K} L_KK^{-1} one row per lane.  L_KK is read into LDS
// before anything is written, and each row of L_{C,K} is read by the lane that
// overwrites it, so Src may alias Lp.
template <typename T>
__global__ void __launch_bounds__(64) k_normalize_small(const DevPlan *__restrict__ plp, const T *Src_all, T *Lp_all,
                                                        T *dt_all, const int32_t *__restrict__ nodes, int32_t count) {
  constexpr int S = kSmallNormS, SP = S + 1;
  const DevPlan &pl = *plp;
  __shared__ T lk[S * SP], xs[S * SP], dv[S];
  const int64_t g = blockIdx.x;
  const int64_t l = g / count;
  const int K = nodes[g - l * count];
  const int s = gp(pl.node_s)[K], c = gp(pl.node_c)[K], ld = s + c;
  const int64_t off = gp(pl.node_off)[K];
  const T *Q = Src_all + l * pl.panel_elems + off;
  T *P = Lp_all + l * pl.panel_elems + off;
  T *dinv = reinterpret_cast<T *>(pl.dinv) + l * pl.n + gp(pl.node_first)[K];
  const int t = threadIdx.x;
#pragma unroll
  for (int u = 0; u < S * S / 64; ++u) {
    const int e = t + 64 * u, i = e % S, k = e / S;
    lk[i * SP + k] = (i < s && k < s) ? Q[(int64_t)k * ld + i] : zero_of<T>();
    xs[i * SP + k] = zero_of<T>();  // the rows k >= s are read (times zero) by the Lhat loop below
  }
  __syncthreads();
  if (t < s) {  // column t of L_KK^{-1}, kept in LDS (only this lane touches it)
    const T d = SOps<T>::div(SOps<T>::one(), lk[t * SP + t]);
    dv[t] = d;
    gstore(dinv + t, d);
    for (int i = 0; i < s; ++i) {
      T v = (i == t) ? SOps<T>::one() : zero_of<T>();
      for (int k = t; k < i; ++k) v -= lk[i * SP + k] * xs[k * SP + t];
      xs[i * SP + t] = v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < S * S / 64; ++u) {
    const int e = t + 64 * u, a = e % S, b = e / S;
    if (a < s && b < s) {
      const double cs = pl.csign;
      T acc = zero_of<T>();
      for (int k = a > b ? a : b; k < s; ++k) acc += (cj(xs[k * SP + a], cs) * dv[k]) * xs[k * SP + b];
      P[(int64_t)b * ld + a] = acc;
      if (dt_all) {
        T dd = zero_of<T>();
        for (int k = 0; k <= (a < b ? a : b); ++k) {
          const T la = (a == k) ? SOps<T>::one() : lk[a * SP + k], lb = (b == k) ? SOps<T>::one() : lk[b * SP + k];
          dd += (la * lk[k * SP + k]) * cj(lb, cs);
        }
        dt_all[l * pl.sq_elems + gp(pl.node_sq)[K] + (int64_t)b * s + a] = dd;
      }
    }
  }
  for (int i0 = 0; i0 < c; i0 += 64) {
    const int i = i0 + t;
    if (i < c) {
      T lr[S];
#pragma unroll
      for (int k = 0; k < S; ++k) lr[k] = k < s ? Q[(int64_t)k * ld + s + i] : zero_of<T>();
#pragma unroll 1
      for (int q = 0; q < s; ++q) {
        T v = zero_of<T>();
#pragma unroll
        for (int k = 0; k < S; ++k)
          if (k >= q && k < s) v += lr[k] * xs[k * SP + q];
        P[(int64_t)q * ld + s + i] = v;
      }
    }
  }
}

// Lhat_{C,K} = L_{C,K} L_KK^{-1} (Alg. 1 steps 1-2) for one 64-row block a of
// C(K), column tiles left to right on MFMA (hs = 1, LU plans: Uhat_{K,C}^T =
// U_{K,C}^T U_KK^{-T} in the second panel set).  Column x of Lhat needs only
// columns k >= x of L (L_KK^{-1} is lower triangular), so a workgroup that
// owns its row block and writes tile b after finishing it never reads a
// column it has already overwritten: Q may alias P.
template <typename T>
__global__ void __launch_bounds__(NT, 2)
    k_normalize_gemm(const DevPlan *__restrict__ plp, const T *Src_all, T *Lp_all, const int2 *rblocks, int32_t nrb,
                     int nsets) {
  const DevPlan &pl = *plp;
  // two GEMM stages or one 64 x 64 result tile, whichever is larger (complex:
  // half of smem_doubles, so that two workgroups share a CU)
  constexpr int kStages = 2 * dense_stage_doubles<T, DenseTK<T>::TK>();
  __shared__ double smem[kStages > tile_doubles<T>() ? kStages : tile_doubles<T>()];
  constexpr int TK = DenseTK<T>::TK;
  const int64_t per = (int64_t)nrb * pl.batch;  // workgroups per panel set (LU: two sets)
  const int hs = nsets > 1 ? (int)(blockIdx.x / per) : 0;
  const int64_t g = blockIdx.x - hs * per;
  const int64_t l = g / nrb;
  const int2 rb = rblocks[g - l * nrb];
  const int K = uniform(rb.x), i0 = uniform(rb.y) * 64;
  const int s = uniform(gp(pl.node_s)[K]), c = uniform(gp(pl.node_c)[K]), ld = s + c;
  const int64_t off = gp(pl.node_off)[K] + hs * pl.half;
  const T *Q = Src_all + l * pl.panel_elems + off;
  T *P = Lp_all + l * pl.panel_elems + off;
  const T *Linv = reinterpret_cast<const T *>(pl.linv) + (hs * pl.batch + l) * pl.sq_elems + gp(pl.node_sq)[K];
  for (int x0 = 0; x0 < s; x0 += 64) {
    LoadDenseA<T, TK> la{Q + s, ld, c, s, i0};      // L_{C,K}(i, k)
    LoadDenseB<T, TK> lb{Linv, 0, s, 0, s, x0, s};  // L_KK^{-1}(k, x)
    Acc<T> acc;
    gemm_dense<T, true>(x0, s, la, lb, smem, acc);  // complex: three real product chains
    acc_to_lds<T>(acc, smem);
    lds_barrier();
    for (int e = threadIdx.x; e < 64 * 64; e += NT) {
      const int i = e & 63, x = e >> 6;
      if (i0 + i < c && x0 + x < s) P[(int64_t)(x0 + x) * ld + s + i0 + i] = lds_get<T>(smem, i, x);
    }
    lds_barrier();
  }
}

// 32 x 32 output tiles of the s x s blocks (^H for ^T in a Hermitian plan):
//   mode 0: Dt = L_KK D L_KK^T              -> dt buffer (reads the LDL^T top block)
//   mode 1: Dt^{-1} = Linv^T D^{-1} Linv    -> panel top block
//           (LU plans: U_KK^{-1} D^{-1} L_KK^{-1}, the left factor from the
//           second half of the linv buffer; no mode 0)
// The contraction runs in 32-deep stages through LDS, the diagonal factor
// folded into the left operand as it is stored; wave w computes the 16 x 16
// block (w & 1, w >> 1) of the tile on MFMA (complex in the 3M form), and the
// tile leaves through LDS so that the stores coalesce.
template <typename T>
__global__ void __launch_bounds__(NT) k_normalize_sq(const DevPlan *__restrict__ plp, const T *Src_all, T *Lp_all, T *dt_all,
                                                     const int4 *tiles, int32_t ntiles, int mode) {
  constexpr int P = Planes<T>::P, C = P == 1 ? 1 : 3;  // product chains (3M for complex)
  const DevPlan &pl = *plp;
  __shared__ double la[P][32 * 33], lb[P][32 * 33];
  const int64_t g = blockIdx.x;
  const int64_t l = g / ntiles;
  const int4 tk = tiles[g - l * ntiles];
  const int K = tk.x, i0 = tk.y * 32, j0 = tk.z * 32;
  const int s = gp(pl.node_s)[K], c = gp(pl.node_c)[K], ld = s + c;
  const T *Q = Src_all + l * pl.panel_elems + gp(pl.node_off)[K];  // LDL^T panel (mode 0 reads it)
  T *P_ = Lp_all + l * pl.panel_elems + gp(pl.node_off)[K];        // normalized panel (mode 1 writes it)
  const T *Linv = reinterpret_cast<const T *>(pl.linv) + l * pl.sq_elems + gp(pl.node_sq)[K];
  const T *Uinv = pl.half > 0 ? Linv + pl.batch * pl.sq_elems : Linv;  // U_KK^{-T} in LU plans
  const T *dinv = reinterpret_cast<const T *>(pl.dinv) + l * pl.n + gp(pl.node_first)[K];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, m = lane & 15;
  const int bi = wv & 1, bj = wv >> 1;
  d4 pc[C];
#pragma unroll
  for (int q = 0; q < C; ++q) pc[q] = d4{0.0, 0.0, 0.0, 0.0};
  int kb, ke;
  if (mode == 0) {
    kb = 0;
    ke = min(s, min(i0, j0) + 32);
  } else {
    kb = max(i0, j0);
    ke = s;
  }
  for (int k0 = kb; k0 < ke; k0 += 32) {
    lds_barrier();
    for (int e = threadIdx.x; e < 32 * 32; e += NT) {
      const int kk = e & 31, x = e >> 5;
      const int k = k0 + kk;
      T va = zero_of<T>(), vb = zero_of<T>();
      if (k < ke) {
        const int ia = i0 + x, jb = j0 + x;
        T d;
        if (mode == 0) {  // L[i][k] with unit diagonal, D_k
          if (ia < s) va = (ia == k) ? SOps<T>::one() : (ia > k ? Q[(int64_t)k * ld + ia] : zero_of<T>());
          if (jb < s) vb = (jb == k) ? SOps<T>::one() : (jb > k ? Q[(int64_t)k * ld + jb] : zero_of<T>());
          d = Q[(int64_t)k * ld + k];
        } else {  // Linv[k][i] (column-major, ld s), lower triangular; D_k^{-1}
          if (ia < s) va = gload(Uinv + (int64_t)ia * s + k);
          if (jb < s) vb = gload(Linv + (int64_t)jb * s + k);
          d = gload(dinv + k);
        }
        // the transposed factor: L_KK^T (mode 0, right) or Linv^T (mode 1, left)
        if (mode == 0)
          vb = cj(vb, pl.csign);
        else
          va = cj(va, pl.csign);
        va = va * d;
      }
#pragma unroll
      for (int p = 0; p < P; ++p) {
        la[p][x * 33 + kk] = Planes<T>::get(va, p);
        lb[p][x * 33 + kk] = Planes<T>::get(vb, p);
      }
    }
    lds_barrier();
    // lane l: A(i = 16 bi + l % 16, k = 4 k4 + l / 16), B(k, j = 16 bj + l % 16)
#pragma unroll
    for (int k4 = 0; k4 < 8; ++k4) {
      const int ka = 4 * k4 + (lane >> 4);
      if constexpr (P == 1) {
        pc[0] = mfma16(la[0][(16 * bi + m) * 33 + ka], lb[0][(16 * bj + m) * 33 + ka], pc[0]);
      } else {
        const double a0 = la[0][(16 * bi + m) * 33 + ka], a1 = la[1][(16 * bi + m) * 33 + ka];
        const double b0 = lb[0][(16 * bj + m) * 33 + ka], b1 = lb[1][(16 * bj + m) * 33 + ka];
        pc[0] = mfma16(a0, b0, pc[0]);
        pc[1] = mfma16(a1, b1, pc[1]);
        pc[2] = mfma16(a0 + a1, b0 + b1, pc[2]);
      }
    }
  }
  lds_barrier();
  // the tile into la as [j][i] (result row 4 v + l / 16 of column l % 16 of
  // the wave's block), then stores with lanes along i
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 16 * bi + 4 * v + (lane >> 4), j = 16 * bj + m;
    if constexpr (P == 1) {
      la[0][j * 33 + i] = pc[0][v];
    } else {
      la[0][j * 33 + i] = pc[0][v] - pc[1][v];
      la[1][j * 33 + i] = pc[2][v] - pc[0][v] - pc[1][v];
    }
  }
  lds_barrier();
  for (int e = threadIdx.x; e < 32 * 32; e += NT) {
    const int i = e & 31, jj = e >> 5;
    const int gi = i0 + i, gj = j0 + jj;
    if (gi < s && gj < s) {
      const T v = Planes<T>::from(&la[0][jj * 33 + i], 32 * 33);
      if (mode == 0)
        dt_all[l * pl.sq_elems + gp(pl.node_sq)[K] + (int64_t)gj * s + gi] = v;
      else
        P_[(int64_t)gj * ld + gi] = v;
    }
  }
}

template <typename T>
__global__ void k_extract(const DevPlan *__restrict__ plp, const T *Xp, T *out) {
  const DevPlan &pl = *plp;
  const int64_t total = pl.batch * pl.nnzA;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = q / pl.nnzA, e = q - l * pl.nnzA;
    // an entry the permutation moved into B's upper triangle is the transpose
    // of the stored one (conjugated in a Hermitian plan)
    out[q] = cj(Xp[l * pl.panel_elems + gp(pl.apos)[e]], gp(pl.aflip)[e] ? pl.csign : 1.0);
  }
}

// LU plans: out[l][e] = A^{-1}(rowind[e], col e) and out[l][nnz + e] =
// A^{-1}(col e, rowind[e]); entry e sits at the same position in both panel
// sets, the X set holding B^{-1} there and the X^T set its transpose, which
// trade places where the permutation moved the entry into B's upper triangle.
template <typename T>
__global__ void k_extract_lu(const DevPlan *__restrict__ plp, const T *Xp, T *out) {
  const DevPlan &pl = *plp;
  const int64_t total = pl.batch * pl.nnzA;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = q / pl.nnzA, e = q - l * pl.nnzA;
    const T *X = Xp + l * pl.panel_elems + gp(pl.apos)[e];
    const T xl = X[0], xu = X[pl.half];
    const bool f = gp(pl.aflip)[e] != 0;
    out[2 * l * pl.nnzA + e] = f ? xu : xl;
    out[2 * l * pl.nnzA + pl.nnzA + e] = f ? xl : xu;
  }
}

// Zero a [batch][panel_elems] array (a kernel rather than a memset, so that
// the call can sit in a captured graph).
template <typename T>
__global__ void k_zero(const DevPlan *__restrict__ plp, T *P) {
  const DevPlan &pl = *plp;
  const int64_t total = pl.batch * pl.panel_elems;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x)
    P[q] = zero_of<T>();
}

// P[l][position of A entry e] = vals[l][e], conjugated where k_extract
// conjugates (the transpose of k_extract).
template <typename T>
__global__ void k_scatter(const DevPlan *__restrict__ plp, const T *vals, T *P) {
  const DevPlan &pl = *plp;
  const int64_t total = pl.batch * pl.nnzA;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = q / pl.nnzA, e = q - l * pl.nnzA;
    P[l * pl.panel_elems + gp(pl.apos)[e]] = cj(vals[q], gp(pl.aflip)[e] ? pl.csign : 1.0);
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from the C ABI translation unit)
// ---------------------------------------------------------------------------
// part < 0: every node; q >= 0: normalization chunk q (see LaunchAux).
// steps: a mask of NORM_INV (the small nodes' whole normalization and
// L_KK^{-1}), NORM_GEMM (Lhat) and NORM_SQ (Dt^{-1}, and Dt when dt is
// given); NORM_GEMM and NORM_SQ need NORM_INV done.
template <typename T>
static hipError_t normalize_impl(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, const void *src,
                                 void *panels, void *dt, hipStream_t st, int part, int steps) {
  const T *Q = reinterpret_cast<const T *>(src);
  T *Lp = reinterpret_cast<T *>(panels);
  // [b, b + n) of list j, which has nall entries
  auto range = [&](int j, int32_t nall, int32_t &b) {
    if (part < 0) {
      b = 0;
      return nall;
    }
    b = aux.norm_cut[5 * part + j];
    return aux.norm_cut[5 * (part + 1) + j] - b;
  };
  int32_t b;
  // LU plans (no single-wavefront nodes) normalize both panel sets
  const int nsets = pl.half > 0 ? 2 : 1;
  const int32_t nsm = (steps & NORM_INV) ? range(0, aux.nsmall, b) : 0;
  if (nsm > 0)
    hipLaunchKernelGGL(k_normalize_small<T>, dim3((unsigned)(nsm * pl.batch)), dim3(64), 0, st, dpl, Q, Lp,
                       reinterpret_cast<T *>(dt), aux.small_nodes + b, nsm);
  const int32_t nna = (steps & NORM_INV) ? range(1, aux.nchunks_narrow, b) : 0;
  if (nna > 0)
    hipLaunchKernelGGL((k_normalize_inv<T, 64>), dim3((unsigned)(nna * pl.batch * nsets)), dim3(NT), 0, st, dpl, Q,
                       aux.chunks_narrow + b, nna, nsets);
  const int32_t nch = (steps & NORM_INV) ? range(2, aux.nchunks, b) : 0;
  if (nch > 0)
    hipLaunchKernelGGL((k_normalize_inv<T, 256>), dim3((unsigned)(nch * pl.batch * nsets)), dim3(NT), 0, st, dpl, Q,
                       aux.chunks + b, nch, nsets);
  const int32_t nrb = (steps & NORM_GEMM) ? range(3, aux.nrblocks, b) : 0;
  if (nrb > 0)
    hipLaunchKernelGGL(k_normalize_gemm<T>, dim3((unsigned)(nrb * pl.batch * nsets)), dim3(NT), 0, st, dpl, Q, Lp,
                       aux.rblocks + b, nrb, nsets);
  const int32_t nsq = (steps & NORM_SQ) ? range(4, aux.nsq_tiles, b) : 0;
  if (nsq > 0) {
    if (dt)
      hipLaunchKernelGGL(k_normalize_sq<T>, dim3((unsigned)(nsq * pl.batch)), dim3(NT), 0, st, dpl, Q, Lp,
                         reinterpret_cast<T *>(dt), aux.sq_tiles + b, nsq, 0);
    hipLaunchKernelGGL(k_normalize_sq<T>, dim3((unsigned)(nsq * pl.batch)), dim3(NT), 0, st, dpl, Q, Lp,
                       (T *)nullptr, aux.sq_tiles + b, nsq, 1);
  }
  return hipGetLastError();
}

// L_KK^{-1} and D_K^{-1} of the nodes of a chunk list (the device factorization).
hipError_t launch_linv(const DevPlan &pl, const DevPlan *dpl, bool cplx_, const void *src, const int2 *chunks,
                       int32_t n, bool narrow, hipStream_t st) {
  const dim3 grid((unsigned)(n * pl.batch));
  if (cplx_) {
    if (narrow)
      hipLaunchKernelGGL((k_normalize_inv<cplx, 64>), grid, dim3(NT), 0, st, dpl, reinterpret_cast<const cplx *>(src),
                         chunks, n, 1);
    else
      hipLaunchKernelGGL((k_normalize_inv<cplx, 256>), grid, dim3(NT), 0, st, dpl, reinterpret_cast<const cplx *>(src),
                         chunks, n, 1);
  } else {
    if (narrow)
      hipLaunchKernelGGL((k_normalize_inv<double, 64>), grid, dim3(NT), 0, st, dpl,
                         reinterpret_cast<const double *>(src), chunks, n, 1);
    else
      hipLaunchKernelGGL((k_normalize_inv<double, 256>), grid, dim3(NT), 0, st, dpl,
                         reinterpret_cast<const double *>(src), chunks, n, 1);
  }
  return hipGetLastError();
}

hipError_t launch_normalize(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, bool cplx_, const void *src,
                            void *panels, void *dt, hipStream_t st, int part, int steps) {
  return cplx_ ? normalize_impl<cplx>(pl, dpl, aux, src, panels, dt, st, part, steps)
               : normalize_impl<double>(pl, dpl, aux, src, panels, dt, st, part, steps);
}

// Positions [b, e) of level launch q (a sub-range of [lvl_ptr[q],
// lvl_ptr[q + 1]): the records of a single-wavefront, push or 128-tile launch
// are laid out in the launch's order, so a sub-range starts b - lvl_ptr[q]
// records in).
template <typename T>
static void launch_level(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, const T *Lp, T *Xp, T *Pp,
                         hipStream_t st, int q, int32_t b, int32_t e) {
  if (e <= b) return;
  if (aux.lvl_kind[q] == LVL_TINY) {
    // complex plans: the forward-only nodes (from lvl_tsplit[q]) in k_tiny64
    const int32_t ts = sizeof(T) == 16 && aux.lvl_tsplit[q] >= 0 ? aux.lvl_tsplit[q] : aux.lvl_ptr[q + 1];
    const int32_t m0 = std::min(e, std::max(b, ts));
    if (m0 > b)
      hipLaunchKernelGGL((pl.csign < 0 ? k_tiny<T, true> : k_tiny<T, false>), dim3((unsigned)((m0 - b) * pl.batch)),
                         dim3(64), 0, st, dpl, Lp, Xp, aux.tiny + aux.lvl_tiny[q] + (b - aux.lvl_ptr[q]), m0 - b, b);
    if (e > m0)
      hipLaunchKernelGGL((pl.csign < 0 ? k_tiny64<T, true> : k_tiny64<T, false>), dim3((unsigned)((e - m0) * pl.batch)),
                         dim3(64), 0, st, dpl, Lp, Xp,
                         aux.tiny + aux.lvl_tiny[q] + (m0 - aux.lvl_ptr[q]), e - m0, m0);
  } else if (aux.lvl_kind[q] == LVL_PUSH)
    hipLaunchKernelGGL(k_push<T>, dim3((unsigned)((e - b) * pl.batch)), dim3(NT), 0, st, dpl, Lp, Xp,
                       aux.push + aux.lvl_tiny[q] + (b - aux.lvl_ptr[q]), e - b, b);
  else if (aux.lvl_kind[q] == LVL_Y128) {
    if constexpr (sizeof(T) == 8)
      hipLaunchKernelGGL(k_ydense128, dim3((unsigned)((e - b) * pl.batch)), dim3(NT), 0, st, dpl,
                         reinterpret_cast<const double *>(Lp), reinterpret_cast<double *>(Xp),
                         aux.y128 + aux.lvl_tiny[q] + (b - aux.lvl_ptr[q]), e - b, b);
  } else if (aux.lvl_kind[q] == LVL_YDENSE)
    hipLaunchKernelGGL(k_ydense<T>, dim3((unsigned)((e - b) * pl.batch)), dim3(NT), 0, st, dpl, Lp, Xp, Pp,
                       aux.lvl_recs + b, aux.lvl_items + b, e - b, b);
  else if (aux.lvl_kind[q] == LVL_GATHER)
    hipLaunchKernelGGL((pl.half > 0 ? k_gather_list<T, true> : k_gather_list<T, false>),
                       dim3((unsigned)((e - b) * pl.batch)), dim3(NT), 0, st, dpl, Xp, aux.lvl_recs + b,
                       aux.lvl_items + b, e - b, b);
  else if (aux.lvl_kind[q] == LVL_GEMM2)
    hipLaunchKernelGGL(k_gemm2_list<T>, dim3((unsigned)((e - b) * pl.batch)), dim3(NT), 0, st, dpl, Lp, Xp, Pp,
                       aux.lvl_recs + b, aux.lvl_items + b, e - b, b);
  else
    hipLaunchKernelGGL(k_items_list<T>, dim3((unsigned)((e - b) * pl.batch)), dim3(NT), 0, st, dpl, Lp, Xp, Pp,
                       aux.lvl_recs + b, aux.lvl_items + b, e - b, b);
}

// Level launches [q0, q1) under the level schedule (the whole traversal
// is [0, aux.nlvl)); the persistent schedule ignores the range.
template <typename T>
static hipError_t run_impl(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, int sched, const void *panels, void *x,
                           int64_t budget_ticks, int grid, hipStream_t st, int q0, int q1) {
  const T *Lp = reinterpret_cast<const T *>(panels);
  T *Xp = reinterpret_cast<T *>(x);
  T *Pp = reinterpret_cast<T *>(pl.part);
  if (sched == 2 && q0 == 0) {  // the push form accumulates into X: start from zero
    const int64_t total = pl.batch * pl.panel_elems;
    unsigned gz = (unsigned)((total + 255) / 256);
    if (gz > 65536u) gz = 65536u;
    hipLaunchKernelGGL(k_zero<T>, dim3(gz ? gz : 1), dim3(256), 0, st, dpl, Xp);
  }
  if (sched == 1 || sched == 2) {
    for (int q = q0; q < q1; ++q) launch_level<T>(pl, dpl, aux, Lp, Xp, Pp, st, q, aux.lvl_ptr[q], aux.lvl_ptr[q + 1]);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_sched_init, dim3(256), dim3(256), 0, st, dpl);
  hipLaunchKernelGGL(k_persistent<T>, dim3((unsigned)grid), dim3(NT), 0, st, dpl, Lp, Xp, Pp, budget_ticks);
  return hipGetLastError();
}

// Positions [b, e) of level launch q alone, on st (level schedule).
hipError_t launch_level_range(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, bool cplx_, const void *panels,
                              void *x, hipStream_t st, int q, int32_t b, int32_t e) {
  if (cplx_)
    launch_level<cplx>(pl, dpl, aux, reinterpret_cast<const cplx *>(panels), reinterpret_cast<cplx *>(x),
                       reinterpret_cast<cplx *>(pl.part), st, q, b, e);
  else
    launch_level<double>(pl, dpl, aux, reinterpret_cast<const double *>(panels), reinterpret_cast<double *>(x),
                         reinterpret_cast<double *>(pl.part), st, q, b, e);
  return hipGetLastError();
}

hipError_t launch_run(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, bool cplx_, int sched, const void *panels,
                      void *x, int64_t budget_ticks, int grid, hipStream_t st, int q0, int q1) {
  return cplx_ ? run_impl<cplx>(pl, dpl, aux, sched, panels, x, budget_ticks, grid, st, q0, q1)
               : run_impl<double>(pl, dpl, aux, sched, panels, x, budget_ticks, grid, st, q0, q1);
}

int persistent_blocks_per_cu(bool cplx_) {
  int nb = 0;
  if (cplx_)
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<cplx>, NT, 0);
  else
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<double>, NT, 0);
  return nb;
}

hipError_t launch_extract(const DevPlan &pl, const DevPlan *dpl, bool cplx_, const void *x, void *out, hipStream_t st) {
  const int64_t total = pl.batch * pl.nnzA;
  unsigned grid = (unsigned)((total + 255) / 256);
  if (grid > 65536u) grid = 65536u;
  if (grid == 0) grid = 1;
  if (pl.half > 0)
    hipLaunchKernelGGL(k_extract_lu<double>, dim3(grid), dim3(256), 0, st, dpl, reinterpret_cast<const double *>(x),
                       reinterpret_cast<double *>(out));
  else if (cplx_)
    hipLaunchKernelGGL(k_extract<cplx>, dim3(grid), dim3(256), 0, st, dpl, reinterpret_cast<const cplx *>(x),
                       reinterpret_cast<cplx *>(out));
  else
    hipLaunchKernelGGL(k_extract<double>, dim3(grid), dim3(256), 0, st, dpl, reinterpret_cast<const double *>(x),
                       reinterpret_cast<double *>(out));
  return hipGetLastError();
}

hipError_t launch_scatter(const DevPlan &pl, const DevPlan *dpl, bool cplx_, const void *vals, void *panel,
                          hipStream_t st) {
  auto grid_for = [](int64_t total) {
    unsigned g = (unsigned)((total + 255) / 256);
    return g > 65536u ? 65536u : (g == 0 ? 1u : g);
  };
  const unsigned gz = grid_for(pl.batch * pl.panel_elems), gs = grid_for(pl.batch * pl.nnzA);
  if (cplx_) {
    hipLaunchKernelGGL(k_zero<cplx>, dim3(gz), dim3(256), 0, st, dpl, reinterpret_cast<cplx *>(panel));
    hipLaunchKernelGGL(k_scatter<cplx>, dim3(gs), dim3(256), 0, st, dpl, reinterpret_cast<const cplx *>(vals),
                       reinterpret_cast<cplx *>(panel));
  } else {
    hipLaunchKernelGGL(k_zero<double>, dim3(gz), dim3(256), 0, st, dpl, reinterpret_cast<double *>(panel));
    hipLaunchKernelGGL(k_scatter<double>, dim3(gs), dim3(256), 0, st, dpl, reinterpret_cast<const double *>(vals),
                       reinterpret_cast<double *>(panel));
  }
  return hipGetLastError();
}

}  // namespace selinv
