// HIP kernels of the selected-inversion library for gfx950 (CDNA4).
//
//  normalize  Alg. 1 steps 1-2 in LDL^T form: Lhat_{C,K} = L_{C,K} L_KK^{-1}
//             (row-wise back substitution, in place), L_KK^{-1} into scratch,
//             Dt_K = L_KK D_K L_KK^T (optional, for the adjoint) and
//             Dt_K^{-1} = L_KK^{-T} D_K^{-1} L_KK^{-1} into the panel's top block.
//  selinv     Alg. 1 second loop (root first): per supernode K the gather of
//             X_{C,C} through the ancestor maps into LDS, GEMM-1
//             X_{C,K} = -X_{C,C} Lhat_{C,K} and GEMM-2
//             X_KK = Dt^{-1} - Lhat^T X_{C,K} on FP64 MFMA
//             (v_mfma_f64_16x16x4f64; complex128 by four real products), the
//             diagonal-block symmetrization of Section 2.3, coalesced stores.
//             Scheduled either level by level or by one persistent launch
//             whose workgroups pop items from a device ready queue fed by
//             per-node dependency counters (the device counterpart of the
//             task dependencies of Section 3).
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
__global__ void __launch_bounds__(NT, Planes<T>::P == 1 ? 2 : 1) k_items_list(const DevPlan *__restrict__ plp, const T *Lp, T *Xp, T *Pp, const int32_t *list,
                                                   int32_t count, int32_t list_pos) {
  const DevPlan &pl = *plp;
  __shared__ double smem[smem_doubles<T>()];
  __shared__ int64_t rt[128];
  const int64_t g = blockIdx.x;
  const int64_t l = g / count;
  const int32_t it = list[g - l * count];
  const int64_t t_start = pl.trace ? wall_clock64() : 0;
  Ctx<T> cx{&pl, Lp + l * pl.panel_elems, Xp + l * pl.panel_elems, Pp + l * pl.part_elems,
            static_cast<T *>(pl.gbuf) + l * pl.g_elems, static_cast<T *>(pl.ypart) + l * pl.y_elems};
  do_item<T, false>(cx, gload(pl.items + it), smem, rt);
  if (pl.trace) {
    __syncthreads();
    if (threadIdx.x == 0) {  // row of this item in the trace: levels in order, matrices inside a level
      int64_t *tr = pl.trace + 8 * ((int64_t)list_pos * pl.batch + g);
      tr[0] = l * pl.nitems + it;
      tr[1] = blockIdx.x;
      tr[2] = t_start;
      tr[3] = t_start;
      tr[4] = wall_clock64();
    }
  }
}

// Small nodes of one level, one wavefront each (see do_tiny).
template <typename T>
__global__ void __launch_bounds__(64) k_tiny(const DevPlan *__restrict__ plp, const T *Lp, T *Xp,
                                             const TinyRec *__restrict__ recs, int32_t count, int32_t list_pos) {
  const DevPlan &pl = *plp;
  __shared__ T ls[kTinyS * kTinyC], ys[kTinyS * kTinyC];
  const int64_t g = blockIdx.x;
  const int64_t l = g / count;
  const TinyRec r = recs[g - l * count];
  const int64_t t_start = pl.trace ? wall_clock64() : 0;
  const T *L = Lp + l * pl.panel_elems;
  T *X = Xp + l * pl.panel_elems;
  if (r.c <= 8)
    do_tiny<T, 8>(r, pl.toff, L, X, ls, ys);
  else if (r.c <= 16)
    do_tiny<T, 16>(r, pl.toff, L, X, ls, ys);
  else
    do_tiny<T, 32>(r, pl.toff, L, X, ls, ys);
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
// when another workgroup raised the error flag or when the watchdog, counted
// from kernel start, expires (then it raises the flag).
__device__ bool wait_ready(const DevPlan &pl, int64_t l, const Item &it, int64_t t_begin, int64_t budget_ticks) {
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
// around a barrier is wave-uniform.
template <typename T>
__global__ void __launch_bounds__(NT, 1)
    k_persistent(const DevPlan *__restrict__ plp, const T *Lp, T *Xp, T *Pp, int64_t budget_ticks) {
  const DevPlan &pl = *plp;
  __shared__ double smem[smem_doubles<T>()];
  __shared__ int64_t rt[128];
  __shared__ int32_t s_id, s_ticket;
  __shared__ int64_t s_tpop;
  const int64_t total = pl.batch * pl.nitems;
  const int64_t t_begin = wall_clock64();
  const bool wave0 = uniform((int32_t)threadIdx.x) < 64;
  const bool lane0 = threadIdx.x == 0;
  while (true) {
    if (wave0) {
      int32_t t = 0;
      if (lane0) t = add_relaxed(pl.ctrl + CTRL_TICKET, 1);
      t = uniform(t);
      const int64_t t_draw = pl.trace ? wall_clock64() : 0;
      int32_t id = -1;
      if (t < total) {
        id = uniform(gp(pl.order)[t]);
        const int64_t l = id / pl.nitems;
        if (!wait_ready(pl, l, uniform(gload(pl.items + (id - l * pl.nitems))), t_begin, budget_ticks)) id = -2;
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
    do_item<T, false>(cx, it, smem, rt);
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

// One thread per row r < s of I_s solving x L_KK = e_r (L_KK unit lower): row r
// of L_KK^{-1} (scratch, column-major ld s), and D_K^{-1}.  Back substitution
// in 16-column chunks, L_KK chunks staged in LDS.
template <typename T>
__global__ void __launch_bounds__(NT) k_normalize_rows(const DevPlan *__restrict__ plp, const T *Src_all, T *Lp_all, const int2 *chunks,
                                                       int32_t nchunks) {
  const DevPlan &pl = *plp;
  __shared__ double ls[Planes<T>::P][16 * 257];
  const int64_t g = blockIdx.x;
  const int64_t l = g / nchunks;
  const int2 ck = chunks[g - l * nchunks];
  const int K = ck.x;
  const int s = gp(pl.node_s)[K], c = gp(pl.node_c)[K], ld = s + c;
  const int64_t off = gp(pl.node_off)[K];
  const T *Q = Src_all + l * pl.panel_elems + off;  // LDL^T panel (read only)
  T *P = Lp_all + l * pl.panel_elems + off;         // normalized panel (may alias Q)
  T *Linv = reinterpret_cast<T *>(pl.linv) + l * pl.sq_elems + gp(pl.node_sq)[K];
  T *dinv = reinterpret_cast<T *>(pl.dinv) + l * pl.n + gp(pl.node_first)[K];
  const int r = ck.y * NT + threadIdx.x;
  const bool active = r < s;
  if (ck.y == 0 && threadIdx.x < s) gstore(dinv + threadIdx.x, SOps<T>::div(SOps<T>::one(), Q[(int64_t)threadIdx.x * ld + threadIdx.x]));
  for (int jb = ((s - 1) / 16) * 16; jb >= 0; jb -= 16) {
    const int w = (s - jb < 16) ? s - jb : 16;
    const int nrow = s - jb;  // rows jb .. s-1 of L_KK, columns jb .. jb+w-1
    lds_barrier();
    for (int e = threadIdx.x; e < 16 * nrow; e += NT) {
      const int q = e / nrow, i = e - q * nrow;
      T v = zero_of<T>();
      if (q < w) v = Q[(int64_t)(jb + q) * ld + jb + i];
#pragma unroll
      for (int p = 0; p < Planes<T>::P; ++p) ls[p][q * 257 + i] = Planes<T>::get(v, p);
    }
    lds_barrier();
    if (active) {
      T x[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) x[q] = (q < w && r == jb + q) ? SOps<T>::one() : zero_of<T>();
      // x_i for i beyond the chunk: this thread's own earlier results, read
      // 16 at a time so the loads overlap (indices past s are clamped and
      // their values zeroed)
      for (int ib = jb + w; ib < s; ib += 16) {
        T xi[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) xi[u] = gload(Linv + (int64_t)min(ib + u, s - 1) * s + r);
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int ii = min(ib + u, s - 1) - jb;
          const T xu = masked(xi[u], opaque_mask(ib + u < s));  // zeroed where it is used, not at the load
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            T lv;
            if constexpr (Planes<T>::P == 1) lv = ls[0][q * 257 + ii];
            else lv = T{ls[0][q * 257 + ii], ls[1][q * 257 + ii]};
            x[q] -= xu * lv;
          }
        }
      }
#pragma unroll
      for (int q = 15; q >= 0; --q) {
        if (q < w) {
#pragma unroll
          for (int q2 = q + 1; q2 < 16; ++q2) {
            if (q2 < w) {
              T lv;
              if constexpr (Planes<T>::P == 1) lv = ls[0][q * 257 + q2];
              else lv = T{ls[0][q * 257 + q2], ls[1][q * 257 + q2]};
              x[q] -= x[q2] * lv;
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (q < w) gstore(Linv + (int64_t)(jb + q) * s + r, x[q]);
    }
  }
}

// Lhat_{C,K} = L_{C,K} L_KK^{-1} (Alg. 1 steps 1-2) for one 64-row block a of
// C(K), column tiles left to right on MFMA.  Column x of Lhat needs only
// columns k >= x of L (L_KK^{-1} is lower triangular), so a workgroup that
// owns its row block and writes tile b after finishing it never reads a
// column it has already overwritten: Q may alias P.
template <typename T>
__global__ void __launch_bounds__(NT, Planes<T>::P == 1 ? 2 : 1)
    k_normalize_gemm(const DevPlan *__restrict__ plp, const T *Src_all, T *Lp_all, const int2 *rblocks, int32_t nrb) {
  const DevPlan &pl = *plp;
  __shared__ double smem[smem_doubles<T>()];
  constexpr int TK = DenseTK<T>::TK;
  const int64_t g = blockIdx.x;
  const int64_t l = g / nrb;
  const int2 rb = rblocks[g - l * nrb];
  const int K = uniform(rb.x), i0 = uniform(rb.y) * 64;
  const int s = uniform(gp(pl.node_s)[K]), c = uniform(gp(pl.node_c)[K]), ld = s + c;
  const int64_t off = gp(pl.node_off)[K];
  const T *Q = Src_all + l * pl.panel_elems + off;
  T *P = Lp_all + l * pl.panel_elems + off;
  const T *Linv = reinterpret_cast<const T *>(pl.linv) + l * pl.sq_elems + gp(pl.node_sq)[K];
  for (int x0 = 0; x0 < s; x0 += 64) {
    LoadDenseA<T, TK> la{Q + s, ld, c, s, i0};      // L_{C,K}(i, k)
    LoadDenseB<T, TK> lb{Linv, 0, s, 0, s, x0, s};  // L_KK^{-1}(k, x)
    Acc<T> acc;
    gemm_dense<T>(x0, s, la, lb, smem, acc);
    acc_to_lds<T>(acc, smem);
    lds_barrier();
    for (int e = threadIdx.x; e < 64 * 64; e += NT) {
      const int i = e & 63, x = e >> 6;
      if (i0 + i < c && x0 + x < s) P[(int64_t)(x0 + x) * ld + s + i0 + i] = lds_get<T>(smem, i, x);
    }
    lds_barrier();
  }
}

// 32 x 32 output tiles of the s x s blocks:
//   mode 0: Dt = L_KK D L_KK^T              -> dt buffer (reads the LDL^T top block)
//   mode 1: Dt^{-1} = Linv^T D^{-1} Linv    -> panel top block
template <typename T>
__global__ void __launch_bounds__(NT) k_normalize_sq(const DevPlan *__restrict__ plp, const T *Src_all, T *Lp_all, T *dt_all,
                                                     const int4 *tiles, int32_t ntiles, int mode) {
  const DevPlan &pl = *plp;
  __shared__ double la[Planes<T>::P][32 * 33], lb[Planes<T>::P][32 * 33], dv[Planes<T>::P][32];
  const int64_t g = blockIdx.x;
  const int64_t l = g / ntiles;
  const int4 tk = tiles[g - l * ntiles];
  const int K = tk.x, i0 = tk.y * 32, j0 = tk.z * 32;
  const int s = gp(pl.node_s)[K], c = gp(pl.node_c)[K], ld = s + c;
  const T *Q = Src_all + l * pl.panel_elems + gp(pl.node_off)[K];  // LDL^T panel (mode 0 reads it)
  T *P = Lp_all + l * pl.panel_elems + gp(pl.node_off)[K];         // normalized panel (mode 1 writes it)
  const T *Linv = reinterpret_cast<const T *>(pl.linv) + l * pl.sq_elems + gp(pl.node_sq)[K];
  const T *dinv = reinterpret_cast<const T *>(pl.dinv) + l * pl.n + gp(pl.node_first)[K];
  T acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = zero_of<T>();
  const int ti = threadIdx.x & 31, tj = threadIdx.x >> 5;  // tj 0..7, 4 columns each
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
        if (mode == 0) {  // L[i][k] with unit diagonal
          if (ia < s) va = (ia == k) ? SOps<T>::one() : (ia > k ? Q[(int64_t)k * ld + ia] : zero_of<T>());
          if (jb < s) vb = (jb == k) ? SOps<T>::one() : (jb > k ? Q[(int64_t)k * ld + jb] : zero_of<T>());
        } else {  // Linv[k][i] (column-major, ld s), lower triangular
          if (ia < s) va = gload(Linv + (int64_t)ia * s + k);
          if (jb < s) vb = gload(Linv + (int64_t)jb * s + k);
        }
      }
#pragma unroll
      for (int p = 0; p < Planes<T>::P; ++p) {
        la[p][x * 33 + kk] = Planes<T>::get(va, p);
        lb[p][x * 33 + kk] = Planes<T>::get(vb, p);
      }
    }
    if (threadIdx.x < 32) {
      const int k = k0 + threadIdx.x;
      T d = zero_of<T>();
      if (k < ke) d = (mode == 0) ? Q[(int64_t)k * ld + k] : gload(dinv + k);
#pragma unroll
      for (int p = 0; p < Planes<T>::P; ++p) dv[p][threadIdx.x] = Planes<T>::get(d, p);
    }
    lds_barrier();
    for (int kk = 0; kk < 32; ++kk) {
      T a, d;
      if constexpr (Planes<T>::P == 1) {
        a = la[0][ti * 33 + kk];
        d = dv[0][kk];
      } else {
        a = T{la[0][ti * 33 + kk], la[1][ti * 33 + kk]};
        d = T{dv[0][kk], dv[1][kk]};
      }
      const T ad = a * d;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int jj = tj * 4 + q;
        T b;
        if constexpr (Planes<T>::P == 1) b = lb[0][jj * 33 + kk];
        else b = T{lb[0][jj * 33 + kk], lb[1][jj * 33 + kk]};
        acc[q] += ad * b;
      }
    }
  }
  const int i = i0 + ti;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = j0 + tj * 4 + q;
    if (i < s && j < s) {
      if (mode == 0)
        dt_all[l * pl.sq_elems + gp(pl.node_sq)[K] + (int64_t)j * s + i] = acc[q];
      else
        P[(int64_t)j * ld + i] = acc[q];
    }
  }
}

template <typename T>
__global__ void k_extract(const DevPlan *__restrict__ plp, const T *Xp, T *out) {
  const DevPlan &pl = *plp;
  const int64_t total = pl.batch * pl.nnzA;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = q / pl.nnzA, e = q - l * pl.nnzA;
    out[q] = Xp[l * pl.panel_elems + gp(pl.apos)[e]];
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

// P[l][position of A entry e] = vals[l][e] (the transpose of k_extract).
template <typename T>
__global__ void k_scatter(const DevPlan *__restrict__ plp, const T *vals, T *P) {
  const DevPlan &pl = *plp;
  const int64_t total = pl.batch * pl.nnzA;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = q / pl.nnzA, e = q - l * pl.nnzA;
    P[l * pl.panel_elems + gp(pl.apos)[e]] = vals[q];
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from the C ABI translation unit)
// ---------------------------------------------------------------------------
template <typename T>
static hipError_t normalize_impl(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, const void *src,
                                 void *panels, void *dt, hipStream_t st) {
  const T *Q = reinterpret_cast<const T *>(src);
  T *Lp = reinterpret_cast<T *>(panels);
  if (aux.nchunks > 0) {
    hipLaunchKernelGGL(k_normalize_rows<T>, dim3((unsigned)(aux.nchunks * pl.batch)), dim3(NT), 0, st, dpl, Q, Lp,
                       aux.chunks, aux.nchunks);
  }
  if (aux.nrblocks > 0) {
    hipLaunchKernelGGL(k_normalize_gemm<T>, dim3((unsigned)(aux.nrblocks * pl.batch)), dim3(NT), 0, st, dpl, Q, Lp,
                       aux.rblocks, aux.nrblocks);
  }
  if (aux.nsq_tiles > 0) {
    if (dt)
      hipLaunchKernelGGL(k_normalize_sq<T>, dim3((unsigned)(aux.nsq_tiles * pl.batch)), dim3(NT), 0, st, dpl, Q, Lp,
                         reinterpret_cast<T *>(dt), aux.sq_tiles, aux.nsq_tiles, 0);
    hipLaunchKernelGGL(k_normalize_sq<T>, dim3((unsigned)(aux.nsq_tiles * pl.batch)), dim3(NT), 0, st, dpl, Q, Lp,
                       (T *)nullptr, aux.sq_tiles, aux.nsq_tiles, 1);
  }
  return hipGetLastError();
}

hipError_t launch_normalize(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, bool cplx_, const void *src,
                            void *panels, void *dt, hipStream_t st) {
  return cplx_ ? normalize_impl<cplx>(pl, dpl, aux, src, panels, dt, st)
               : normalize_impl<double>(pl, dpl, aux, src, panels, dt, st);
}

template <typename T>
static hipError_t run_impl(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, int sched, const void *panels, void *x,
                           int64_t budget_ticks, int grid, hipStream_t st) {
  const T *Lp = reinterpret_cast<const T *>(panels);
  T *Xp = reinterpret_cast<T *>(x);
  T *Pp = reinterpret_cast<T *>(pl.part);
  if (sched == 1) {
    for (int q = 0; q < aux.nlvl; ++q) {
      const int32_t b = aux.lvl_ptr[q], e = aux.lvl_ptr[q + 1];
      if (e <= b) continue;
      if (aux.lvl_tiny[q] >= 0)
        hipLaunchKernelGGL(k_tiny<T>, dim3((unsigned)((e - b) * pl.batch)), dim3(64), 0, st, dpl, Lp, Xp,
                           aux.tiny + aux.lvl_tiny[q], e - b, b);
      else
        hipLaunchKernelGGL(k_items_list<T>, dim3((unsigned)((e - b) * pl.batch)), dim3(NT), 0, st, dpl, Lp, Xp, Pp,
                           aux.lvl_items + b, e - b, b);
    }
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_sched_init, dim3(256), dim3(256), 0, st, dpl);
  hipLaunchKernelGGL(k_persistent<T>, dim3((unsigned)grid), dim3(NT), 0, st, dpl, Lp, Xp, Pp, budget_ticks);
  return hipGetLastError();
}

hipError_t launch_run(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, bool cplx_, int sched, const void *panels,
                      void *x, int64_t budget_ticks, int grid, hipStream_t st) {
  return cplx_ ? run_impl<cplx>(pl, dpl, aux, sched, panels, x, budget_ticks, grid, st)
               : run_impl<double>(pl, dpl, aux, sched, panels, x, budget_ticks, grid, st);
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
  if (cplx_)
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
