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

namespace selinv {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int NT = 256;     // threads per workgroup (4 waves)
constexpr int TK = 16;      // contraction step
constexpr int PITCH = 65;   // LDS row pitch in doubles

template <typename T> struct Planes;
template <> struct Planes<double> {
  static constexpr int P = 1;
  static __device__ __forceinline__ double get(double v, int) { return v; }
};
template <> struct Planes<cplx> {
  static constexpr int P = 2;
  static __device__ __forceinline__ double get(cplx v, int p) { return p ? v.im : v.re; }
};

template <typename T> __device__ __forceinline__ T zero_of() { return SOps<T>::zero(); }

// ---------------------------------------------------------------------------
// 64 x 64 MFMA tile: acc += A (64 x kc) * B (kc x 64), operands staged
// through LDS by loader functors (double buffered, one-step register prefetch).
// LDS layout of one stage: A planes [P][TK][PITCH] (k-major), then B planes.
// ---------------------------------------------------------------------------
template <typename T> struct Acc {
  d4 v[Planes<T>::P][2][2];
};

template <typename T> __device__ __forceinline__ constexpr int stage_doubles() {
  return 2 * Planes<T>::P * TK * PITCH;
}
template <typename T> __device__ __forceinline__ constexpr int smem_doubles() {
  return 2 * stage_doubles<T>();  // two stages == one 64 x PITCH tile per plane
}

template <typename T>
__device__ __forceinline__ void stage_store(double *stg, const T va[4], const int ia[4], const T vb[4],
                                            const int ib[4]) {
  constexpr int P = Planes<T>::P;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int p = 0; p < P; ++p) {
      stg[p * TK * PITCH + ia[m]] = Planes<T>::get(va[m], p);
      stg[(P + p) * TK * PITCH + ib[m]] = Planes<T>::get(vb[m], p);
    }
}

template <typename T>
__device__ __forceinline__ void stage_compute(const double *stg, Acc<T> &acc) {
  constexpr int P = Planes<T>::P;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w & 1, wj = w >> 1;
#pragma unroll
  for (int k4 = 0; k4 < 4; ++k4) {
    const int r = (4 * k4 + (lane >> 4)) * PITCH + (lane & 15);
    double a[2][P], b[2][P];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int p = 0; p < P; ++p) {
        a[x][p] = stg[p * TK * PITCH + r + 32 * wi + 16 * x];
        b[x][p] = stg[(P + p) * TK * PITCH + r + 32 * wj + 16 * x];
      }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        if constexpr (P == 1) {
          acc.v[0][bi][bj] = mfma16(a[bi][0], b[bj][0], acc.v[0][bi][bj]);
        } else {
          acc.v[0][bi][bj] = mfma16(a[bi][0], b[bj][0], acc.v[0][bi][bj]);
          acc.v[0][bi][bj] = mfma16(-a[bi][1], b[bj][1], acc.v[0][bi][bj]);
          acc.v[1][bi][bj] = mfma16(a[bi][0], b[bj][1], acc.v[1][bi][bj]);
          acc.v[1][bi][bj] = mfma16(a[bi][1], b[bj][0], acc.v[1][bi][bj]);
        }
      }
  }
}

template <typename T, class LA, class LB>
__device__ __forceinline__ void gemm_tile(int kc, const LA &la, const LB &lb, double *smem, Acc<T> &acc) {
  constexpr int P = Planes<T>::P;
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc.v[p][bi][bj] = d4{0.0, 0.0, 0.0, 0.0};
  const int nk = (kc + TK - 1) / TK;
  if (nk == 0) return;
  T va[4], vb[4];
  int ia[4], ib[4];
  la(0, va, ia);
  lb(0, vb, ib);
  stage_store<T>(smem, va, ia, vb, ib);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    double *cur = smem + (kt & 1) * stage_doubles<T>();
    double *nxt = smem + ((kt + 1) & 1) * stage_doubles<T>();
    const bool more = kt + 1 < nk;
    if (more) {
      la((kt + 1) * TK, va, ia);
      lb((kt + 1) * TK, vb, ib);
    }
    stage_compute<T>(cur, acc);
    if (more) stage_store<T>(nxt, va, ia, vb, ib);
    __syncthreads();
  }
}

// Scatter the accumulators into an LDS tile C[j * PITCH + i] (per plane),
// i = row 0..63, j = column 0..63.  Caller syncs before and after.
template <typename T>
__device__ __forceinline__ void acc_to_lds(const Acc<T> &acc, double *ct) {
  constexpr int P = Planes<T>::P;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w & 1, wj = w >> 1;
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 32 * wi + 16 * bi + 4 * v + (lane >> 4);
          const int j = 32 * wj + 16 * bj + (lane & 15);
          ct[p * 64 * PITCH + j * PITCH + i] = acc.v[p][bi][bj][v];
        }
}

template <typename T> __device__ __forceinline__ T lds_get(const double *ct, int i, int j);
template <> __device__ __forceinline__ double lds_get<double>(const double *ct, int i, int j) {
  return ct[j * PITCH + i];
}
template <> __device__ __forceinline__ cplx lds_get<cplx>(const double *ct, int i, int j) {
  return cplx{ct[j * PITCH + i], ct[64 * PITCH + j * PITCH + i]};
}

// ---------------------------------------------------------------------------
// Loaders.  Each fills 4 values per thread for the k-block starting at k0,
// together with their LDS slot kk * PITCH + (row or column).
// ---------------------------------------------------------------------------

// A = X_{C,C} (rows i0.., cols k0..), gathered from the ancestors' X panels:
// lower (i >= k): X[kcol[k] + posarr[kpos[k] + i]]; upper: the transpose.
template <typename T> struct LoadGather {
  const T *X;
  const int64_t *kcol, *kpos;
  const int32_t *posarr;
  int c, i0;
  __device__ __forceinline__ void operator()(int k0, T v[4], int idx[4]) const {
    const bool upper = (i0 + 63 < k0);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int e = threadIdx.x + NT * m;
      int i, kk;
      if (!upper) {
        i = e & 63;
        kk = e >> 6;
      } else {
        kk = e & 15;
        i = e >> 4;
      }
      const int ig = i0 + i, kg = k0 + kk;
      T val = zero_of<T>();
      if (ig < c && kg < c) {
        if (ig >= kg)
          val = X[kcol[kg] + posarr[kpos[kg] + ig]];
        else
          val = X[kcol[ig] + posarr[kpos[ig] + kg]];
      }
      v[m] = val;
      idx[m] = kk * PITCH + i;
    }
  }
};

// Column block of a panel's bottom part read k-major: value(kk, x) =
// P[off + (x0 + x) * ld + s + k0 + kk], x = 0..63 (rows of A^T or columns of B).
template <typename T> struct LoadPanelK {
  const T *Pn;
  int64_t off;
  int ld, s, c, x0, xmax;
  __device__ __forceinline__ void operator()(int k0, T v[4], int idx[4]) const {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int e = threadIdx.x + NT * m;
      const int kk = e & 15, x = e >> 4;
      const int kg = k0 + kk, xg = x0 + x;
      T val = zero_of<T>();
      if (kg < c && xg < xmax) val = Pn[off + (int64_t)xg * ld + s + kg];
      v[m] = val;
      idx[m] = kk * PITCH + x;
    }
  }
};

// ---------------------------------------------------------------------------
// Work items
// ---------------------------------------------------------------------------
template <typename T> struct Ctx {
  const DevPlan *pl;
  const T *Lp;  // normalized panels of this matrix
  T *Xp;        // selected inverse of this matrix
};

// GEMM-1 tile: X_{C,K}[64a.., 64b..] = -(X_{C,C} Lhat_{C,K})[...]
template <typename T>
__device__ void do_ytile(const Ctx<T> &cx, int K, int a, int b, double *smem) {
  const DevPlan &pl = *cx.pl;
  const int s = pl.node_s[K], c = pl.node_c[K], ld = s + c;
  const int64_t off = pl.node_off[K], rp = pl.node_rowptr[K];
  LoadGather<T> la{cx.Xp, pl.kcol + rp, pl.kpos + rp, pl.posarr, c, a * 64};
  LoadPanelK<T> lb{cx.Lp, off, ld, s, c, b * 64, s};
  Acc<T> acc;
  gemm_tile<T>(c, la, lb, smem, acc);
  acc_to_lds<T>(acc, smem);
  __syncthreads();
  const int i0 = a * 64, j0 = b * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = e & 63, j = e >> 6;
    if (i0 + i < c && j0 + j < s) {
      T val = lds_get<T>(smem, i, j);
      cx.Xp[off + (int64_t)(j0 + j) * ld + s + i0 + i] = SOps<T>::scale(-1.0, val);
    }
  }
  __syncthreads();
}

// GEMM-2 + symmetrization for the block pair (a, b), a >= b, of X_KK.
template <typename T>
__device__ void do_dtile(const Ctx<T> &cx, int K, int a, int b, double *smem) {
  const DevPlan &pl = *cx.pl;
  const int s = pl.node_s[K], c = pl.node_c[K], ld = s + c;
  const int64_t off = pl.node_off[K];
  const T *Dti = cx.Lp + off;  // top block of the normalized panel = Dt^{-1}
  T *Xkk = cx.Xp + off;        // top block of the X panel
  const int a0 = a * 64, b0 = b * 64;
  Acc<T> acc;
  // T_ab = Dt^{-1}[a, b] - Lhat_a^T Y_b
  {
    LoadPanelK<T> la{cx.Lp, off, ld, s, c, a0, s};
    LoadPanelK<T> lb{cx.Xp, off, ld, s, c, b0, s};
    gemm_tile<T>(c, la, lb, smem, acc);
  }
  acc_to_lds<T>(acc, smem);
  __syncthreads();
  if (a == b) {
    for (int e = threadIdx.x; e < 64 * 64; e += NT) {
      const int i = e & 63, j = e >> 6;
      if (a0 + i < s && a0 + j < s) {
        T tij = Dti[(int64_t)(a0 + j) * ld + a0 + i] - lds_get<T>(smem, i, j);
        T tji = Dti[(int64_t)(a0 + i) * ld + a0 + j] - lds_get<T>(smem, j, i);
        Xkk[(int64_t)(a0 + j) * ld + a0 + i] = SOps<T>::scale(0.5, tij + tji);
      }
    }
    __syncthreads();
    return;
  }
  // stash T_ab (unsymmetrized) in X_KK[a, b]
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = e & 63, j = e >> 6;
    if (a0 + i < s && b0 + j < s)
      Xkk[(int64_t)(b0 + j) * ld + a0 + i] = Dti[(int64_t)(b0 + j) * ld + a0 + i] - lds_get<T>(smem, i, j);
  }
  __threadfence_block();
  __syncthreads();
  // T_ba = Dt^{-1}[b, a] - Lhat_b^T Y_a
  {
    LoadPanelK<T> la{cx.Lp, off, ld, s, c, b0, s};
    LoadPanelK<T> lb{cx.Xp, off, ld, s, c, a0, s};
    gemm_tile<T>(c, la, lb, smem, acc);
  }
  acc_to_lds<T>(acc, smem);
  __syncthreads();
  // X[a, b] = X[b, a]^T = (T_ab + T_ba^T) / 2
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = e & 63, j = e >> 6;  // element (a0 + i, b0 + j)
    if (a0 + i < s && b0 + j < s) {
      T tab = Xkk[(int64_t)(b0 + j) * ld + a0 + i];
      T tba = Dti[(int64_t)(a0 + i) * ld + b0 + j] - lds_get<T>(smem, j, i);
      T x = SOps<T>::scale(0.5, tab + tba);
      Xkk[(int64_t)(b0 + j) * ld + a0 + i] = x;
      Xkk[(int64_t)(a0 + i) * ld + b0 + j] = x;
    }
  }
  __syncthreads();
}

template <typename T>
__device__ void do_item(const Ctx<T> &cx, const Item &it, double *smem) {
  if (it.type == ITEM_Y) {
    do_ytile<T>(cx, it.K, it.a, it.b, smem);
  } else if (it.type == ITEM_D) {
    do_dtile<T>(cx, it.K, it.a, it.b, smem);
  } else {  // ITEM_S: the whole node (c <= 64, s <= 64) in this workgroup
    if (cx.pl->node_c[it.K] > 0) {
      do_ytile<T>(cx, it.K, 0, 0, smem);
      __threadfence_block();
      __syncthreads();
    }
    do_dtile<T>(cx, it.K, 0, 0, smem);
  }
}

// ---------------------------------------------------------------------------
// Schedules
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(NT) k_items_list(DevPlan pl, const T *Lp, T *Xp, const int32_t *list,
                                                   int32_t count) {
  __shared__ double smem[smem_doubles<T>()];
  const int64_t g = blockIdx.x;
  const int64_t l = g / count;
  const int32_t it = list[g - l * count];
  Ctx<T> cx{&pl, Lp + l * pl.panel_elems, Xp + l * pl.panel_elems};
  do_item<T>(cx, pl.items[it], smem);
}

__device__ __forceinline__ int32_t ld_acquire(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_relaxed(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t fetch_add(int32_t *p, int32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}

// Reset the dependency counters and the control words.
__global__ void k_sched_init(DevPlan pl) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t nsb = pl.batch * pl.ns;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nsb; i += stride) {
    const int64_t K = i % pl.ns;
    pl.cnt1[i] = pl.n_phase1[K];
    pl.cnt2[i] = pl.n_phase2[K];
  }
  if (blockIdx.x == 0 && threadIdx.x < CTRL_WORDS) pl.ctrl[threadIdx.x] = 0;
}

// Seed the ready queue with the first-phase items of every root of every matrix.
__global__ void k_sched_seed(DevPlan pl) {
  // queue[0 .. batch*nroot) = roots of every matrix; the rest stays -1.
  const int64_t nseed = pl.batch * pl.nroot_items;
  const int64_t total = pl.batch * pl.nitems;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    int32_t v = -1;
    if (i < nseed) {
      const int64_t l = i / pl.nroot_items;
      v = (int32_t)(l * pl.nitems + pl.root_list[i - l * pl.nroot_items]);
    }
    pl.queue[i] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) pl.ctrl[CTRL_TAIL] = (int32_t)nseed;
}

template <typename T>
__global__ void __launch_bounds__(NT) k_persistent(DevPlan pl, const T *Lp, T *Xp, int64_t budget_ticks) {
  __shared__ double smem[smem_doubles<T>()];
  __shared__ int32_t s_id, s_push_beg, s_push_cnt, s_push_base, s_push_l, s_push_kind;
  const int64_t total = pl.batch * pl.nitems;
  while (true) {
    if (threadIdx.x == 0) {
      int32_t id = -3;
      const int32_t idx = fetch_add(pl.ctrl + CTRL_HEAD, 1);
      if (idx < total) {
        const int64_t t0 = wall_clock64();
        while (true) {
          id = ld_acquire(pl.queue + idx);
          if (id >= 0) break;
          if (ld_relaxed(pl.ctrl + CTRL_ERR) != 0) {
            id = -2;
            break;
          }
          if (wall_clock64() - t0 > budget_ticks) {
            __hip_atomic_store(pl.ctrl + CTRL_ERR, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            id = -2;
            break;
          }
          __builtin_amdgcn_s_sleep(4);
        }
      }
      s_id = id;
    }
    __syncthreads();
    const int32_t id = s_id;
    if (id < 0) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // agent-scope acquire for every wave
    const int64_t l = id / pl.nitems;
    const int32_t itn = (int32_t)(id - l * pl.nitems);
    const Item it = pl.items[itn];
    Ctx<T> cx{&pl, Lp + l * pl.panel_elems, Xp + l * pl.panel_elems};
    do_item<T>(cx, it, smem);
    __threadfence();  // release this workgroup's stores at agent scope
    __syncthreads();
    if (threadIdx.x == 0) {
      const int64_t nk = l * pl.ns + it.K;
      int32_t cnt = 0, beg = 0;
      if (it.type == ITEM_Y) {
        if (fetch_add(pl.cnt1 + nk, -1) == 1) {  // phase 1 done: release phase 2
          beg = pl.item_ptr[it.K] + pl.n_phase1[it.K];
          cnt = pl.n_phase2[it.K];
          s_push_kind = 0;
        }
      } else {
        if (fetch_add(pl.cnt2 + nk, -1) == 1) {  // node done: release the children
          beg = pl.push_ptr[it.K];
          cnt = pl.push_ptr[it.K + 1] - beg;
          s_push_kind = 1;
        }
      }
      s_push_cnt = cnt;
      s_push_beg = beg;
      s_push_l = (int32_t)l;
      s_push_base = cnt > 0 ? fetch_add(pl.ctrl + CTRL_TAIL, cnt) : 0;
    }
    __syncthreads();
    const int32_t cnt = s_push_cnt;
    if (cnt > 0) {
      const int32_t beg = s_push_beg, base = s_push_base, kind = s_push_kind;
      const int64_t loff = (int64_t)s_push_l * pl.nitems;
      for (int32_t q = threadIdx.x; q < cnt; q += NT) {
        const int32_t item = kind == 0 ? beg + q : pl.push_list[beg + q];
        if ((int64_t)base + q < total)
          st_release(pl.queue + base + q, (int32_t)(loff + item));
        else  // more pushes than items: a broken dependency table; stop everyone
          __hip_atomic_store(pl.ctrl + CTRL_ERR, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Normalization (Alg. 1 steps 1-2)
// ---------------------------------------------------------------------------

// One thread per row r of [I_s; L_{C,K}] solving x L_KK = rhs (L_KK unit lower):
// rows r < s give row r of L_KK^{-1} (scratch, column-major ld s); rows r >= s
// give Lhat in place (panel row r).  Back substitution in 16-column chunks,
// L_KK chunks staged in LDS.
template <typename T>
__global__ void __launch_bounds__(NT) k_normalize_rows(DevPlan pl, T *Lp_all, const int2 *chunks, int32_t nchunks) {
  __shared__ double ls[Planes<T>::P][16 * 257];
  const int64_t g = blockIdx.x;
  const int64_t l = g / nchunks;
  const int2 ck = chunks[g - l * nchunks];
  const int K = ck.x;
  const int s = pl.node_s[K], c = pl.node_c[K], ld = s + c;
  const int64_t off = pl.node_off[K];
  T *P = Lp_all + l * pl.panel_elems + off;
  T *Linv = reinterpret_cast<T *>(pl.linv) + l * pl.sq_elems + pl.node_sq[K];
  T *dinv = reinterpret_cast<T *>(pl.dinv) + l * pl.n + pl.node_first[K];
  const int r = ck.y * NT + threadIdx.x;
  const bool active = r < s + c;
  if (ck.y == 0 && threadIdx.x < s) dinv[threadIdx.x] = SOps<T>::div(SOps<T>::one(), P[(int64_t)threadIdx.x * ld + threadIdx.x]);
  for (int jb = ((s - 1) / 16) * 16; jb >= 0; jb -= 16) {
    const int w = (s - jb < 16) ? s - jb : 16;
    const int nrow = s - jb;  // rows jb .. s-1 of L_KK, columns jb .. jb+w-1
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * nrow; e += NT) {
      const int q = e / nrow, i = e - q * nrow;
      T v = zero_of<T>();
      if (q < w) v = P[(int64_t)(jb + q) * ld + jb + i];
#pragma unroll
      for (int p = 0; p < Planes<T>::P; ++p) ls[p][q * 257 + i] = Planes<T>::get(v, p);
    }
    __syncthreads();
    if (active) {
      T x[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        T v = zero_of<T>();
        if (q < w) {
          if (r < s)
            v = (r == jb + q) ? SOps<T>::one() : zero_of<T>();
          else
            v = P[(int64_t)(jb + q) * ld + r];
        }
        x[q] = v;
      }
      for (int i = jb + w; i < s; ++i) {
        const T xi = (r < s) ? Linv[(int64_t)i * s + r] : P[(int64_t)i * ld + r];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          T lv;
          if constexpr (Planes<T>::P == 1) lv = ls[0][q * 257 + (i - jb)];
          else lv = T{ls[0][q * 257 + (i - jb)], ls[1][q * 257 + (i - jb)]};
          x[q] -= xi * lv;
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
      for (int q = 0; q < 16; ++q) {
        if (q < w) {
          if (r < s)
            Linv[(int64_t)(jb + q) * s + r] = x[q];
          else
            P[(int64_t)(jb + q) * ld + r] = x[q];
        }
      }
    }
  }
}

// 32 x 32 output tiles of the s x s blocks:
//   mode 0: Dt = L_KK D L_KK^T              -> dt buffer (reads the LDL^T top block)
//   mode 1: Dt^{-1} = Linv^T D^{-1} Linv    -> panel top block
template <typename T>
__global__ void __launch_bounds__(NT) k_normalize_sq(DevPlan pl, T *Lp_all, T *dt_all, const int4 *tiles,
                                                     int32_t ntiles, int mode) {
  __shared__ double la[Planes<T>::P][32 * 33], lb[Planes<T>::P][32 * 33], dv[Planes<T>::P][32];
  const int64_t g = blockIdx.x;
  const int64_t l = g / ntiles;
  const int4 tk = tiles[g - l * ntiles];
  const int K = tk.x, i0 = tk.y * 32, j0 = tk.z * 32;
  const int s = pl.node_s[K], c = pl.node_c[K], ld = s + c;
  T *P = Lp_all + l * pl.panel_elems + pl.node_off[K];
  const T *Linv = reinterpret_cast<const T *>(pl.linv) + l * pl.sq_elems + pl.node_sq[K];
  const T *dinv = reinterpret_cast<const T *>(pl.dinv) + l * pl.n + pl.node_first[K];
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
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * 32; e += NT) {
      const int kk = e & 31, x = e >> 5;
      const int k = k0 + kk;
      T va = zero_of<T>(), vb = zero_of<T>();
      if (k < ke) {
        const int ia = i0 + x, jb = j0 + x;
        if (mode == 0) {  // L[i][k] with unit diagonal
          if (ia < s) va = (ia == k) ? SOps<T>::one() : (ia > k ? P[(int64_t)k * ld + ia] : zero_of<T>());
          if (jb < s) vb = (jb == k) ? SOps<T>::one() : (jb > k ? P[(int64_t)k * ld + jb] : zero_of<T>());
        } else {  // Linv[k][i] (column-major, ld s), lower triangular
          if (ia < s) va = Linv[(int64_t)ia * s + k];
          if (jb < s) vb = Linv[(int64_t)jb * s + k];
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
      if (k < ke) d = (mode == 0) ? P[(int64_t)k * ld + k] : dinv[k];
#pragma unroll
      for (int p = 0; p < Planes<T>::P; ++p) dv[p][threadIdx.x] = Planes<T>::get(d, p);
    }
    __syncthreads();
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
        dt_all[l * pl.sq_elems + pl.node_sq[K] + (int64_t)j * s + i] = acc[q];
      else
        P[(int64_t)j * ld + i] = acc[q];
    }
  }
}

template <typename T>
__global__ void k_extract(DevPlan pl, const T *Xp, T *out) {
  const int64_t total = pl.batch * pl.nnzA;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = q / pl.nnzA, e = q - l * pl.nnzA;
    out[q] = Xp[l * pl.panel_elems + pl.apos[e]];
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from the C ABI translation unit)
// ---------------------------------------------------------------------------
template <typename T>
static hipError_t normalize_impl(const DevPlan &pl, const LaunchAux &aux, void *panels, void *dt, hipStream_t st) {
  T *Lp = reinterpret_cast<T *>(panels);
  if (aux.nchunks > 0) {
    hipLaunchKernelGGL(k_normalize_rows<T>, dim3((unsigned)(aux.nchunks * pl.batch)), dim3(NT), 0, st, pl, Lp,
                       aux.chunks, aux.nchunks);
  }
  if (aux.nsq_tiles > 0) {
    if (dt)
      hipLaunchKernelGGL(k_normalize_sq<T>, dim3((unsigned)(aux.nsq_tiles * pl.batch)), dim3(NT), 0, st, pl, Lp,
                         reinterpret_cast<T *>(dt), aux.sq_tiles, aux.nsq_tiles, 0);
    hipLaunchKernelGGL(k_normalize_sq<T>, dim3((unsigned)(aux.nsq_tiles * pl.batch)), dim3(NT), 0, st, pl, Lp,
                       (T *)nullptr, aux.sq_tiles, aux.nsq_tiles, 1);
  }
  return hipGetLastError();
}

hipError_t launch_normalize(const DevPlan &pl, const LaunchAux &aux, bool cplx_, void *panels, void *dt,
                            hipStream_t st) {
  return cplx_ ? normalize_impl<cplx>(pl, aux, panels, dt, st) : normalize_impl<double>(pl, aux, panels, dt, st);
}

template <typename T>
static hipError_t run_impl(const DevPlan &pl, const LaunchAux &aux, int sched, const void *panels, void *x,
                           int64_t budget_ticks, int grid, hipStream_t st) {
  const T *Lp = reinterpret_cast<const T *>(panels);
  T *Xp = reinterpret_cast<T *>(x);
  if (sched == 1) {
    for (int q = 0; q < aux.nlvl; ++q) {
      const int32_t b = aux.lvl_ptr[q], e = aux.lvl_ptr[q + 1];
      if (e > b)
        hipLaunchKernelGGL(k_items_list<T>, dim3((unsigned)((e - b) * pl.batch)), dim3(NT), 0, st, pl, Lp, Xp,
                           aux.lvl_items + b, e - b);
    }
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_sched_init, dim3(256), dim3(256), 0, st, pl);
  hipLaunchKernelGGL(k_sched_seed, dim3(256), dim3(256), 0, st, pl);
  hipLaunchKernelGGL(k_persistent<T>, dim3((unsigned)grid), dim3(NT), 0, st, pl, Lp, Xp, budget_ticks);
  return hipGetLastError();
}

hipError_t launch_run(const DevPlan &pl, const LaunchAux &aux, bool cplx_, int sched, const void *panels, void *x,
                      int64_t budget_ticks, int grid, hipStream_t st) {
  return cplx_ ? run_impl<cplx>(pl, aux, sched, panels, x, budget_ticks, grid, st)
               : run_impl<double>(pl, aux, sched, panels, x, budget_ticks, grid, st);
}

int persistent_blocks_per_cu(bool cplx_) {
  int nb = 0;
  if (cplx_)
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<cplx>, NT, 0);
  else
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<double>, NT, 0);
  return nb;
}

hipError_t launch_extract(const DevPlan &pl, bool cplx_, const void *x, void *out, hipStream_t st) {
  const int64_t total = pl.batch * pl.nnzA;
  unsigned grid = (unsigned)((total + 255) / 256);
  if (grid > 65536u) grid = 65536u;
  if (grid == 0) grid = 1;
  if (cplx_)
    hipLaunchKernelGGL(k_extract<cplx>, dim3(grid), dim3(256), 0, st, pl, reinterpret_cast<const cplx *>(x),
                       reinterpret_cast<cplx *>(out));
  else
    hipLaunchKernelGGL(k_extract<double>, dim3(grid), dim3(256), 0, st, pl, reinterpret_cast<const double *>(x),
                       reinterpret_cast<double *>(out));
  return hipGetLastError();
}

}  // namespace selinv
