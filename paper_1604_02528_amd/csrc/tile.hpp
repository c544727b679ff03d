// Device building blocks shared by the forward and adjoint kernels:
// a 64 x 64 FP64 MFMA tile with a three-level software-pipelined operand
// loader (index tables -> positions -> data), LDS staging, and memory
// access policies for data produced by other workgroups of the same launch.
//
// MFMA f64 16x16x4 operand layout (measured on gfx950): lane l holds
// A[l % 16][l / 16], B[l / 16][l % 16] and D[4 v + l / 16][l % 16] in its v-th
// accumulator register.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "plan.hpp"
#include "scalar.hpp"

namespace selinv {

typedef double d4 __attribute__((ext_vector_type(4)));

// Global-address-space views of pointers.  Table and data pointers live in the
// device-resident plan, so the compiler sees them as generic pointers and
// would emit flat loads, which count against the LDS wait counter too and
// make every LDS wait drain the operand prefetch.
#define SELINV_GAS __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ const SELINV_GAS T *gp(const T *p) { return (const SELINV_GAS T *)p; }
template <typename T> __device__ __forceinline__ SELINV_GAS T *gw(T *p) { return (SELINV_GAS T *)p; }

// An all-ones / all-zero mask the optimizer cannot see through: selecting
// loaded values with it keeps every load unconditional (a plain select lets
// the compiler sink a load into a branch, which then waits on it).
__device__ __forceinline__ uint32_t opaque_mask32(bool keep) {
  uint32_t m = keep ? ~0u : 0u;
  asm("" : "+v"(m));
  return m;
}
__device__ __forceinline__ int64_t opaque_mask(bool keep) {
  int64_t m = keep ? -1 : 0;
  asm("" : "+v"(m));
  return m;
}
__device__ __forceinline__ double masked(double v, int64_t m) {
  return __builtin_bit_cast(double, __builtin_bit_cast(int64_t, v) & m);
}

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int NT = 256;    // threads per workgroup (4 waves)


// Workgroup barrier that orders LDS only.  __syncthreads() also waits for
// every outstanding global load (vmcnt(0)), which would drain the operand
// prefetch pipeline at each stage; global-memory ordering inside a workgroup
// uses __syncthreads() explicitly where it is needed.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
constexpr int PITCH = 65;  // LDS row pitch in doubles

template <typename T> struct Planes;
template <> struct Planes<double> {
  static constexpr int P = 1;
  static constexpr int TK = 16;  // contraction step per LDS stage
  static __device__ __forceinline__ double get(double v, int) { return v; }
  // the value whose planes are q[0], q[stride], ...
  static __device__ __forceinline__ double from(const double *q, int) { return q[0]; }
};
template <> struct Planes<cplx> {
  static constexpr int P = 2;
  static constexpr int TK = 16;
  static __device__ __forceinline__ double get(cplx v, int p) { return p ? v.im : v.re; }
  static __device__ __forceinline__ cplx from(const double *q, int stride) { return cplx{q[0], q[stride]}; }
};

template <typename T> __device__ __forceinline__ T zero_of() { return SOps<T>::zero(); }

// Elements of one operand stage loaded by each thread.
template <typename T> __device__ __forceinline__ constexpr int ept() { return 64 * Planes<T>::TK / NT; }
template <typename T> __device__ __forceinline__ constexpr int stage_doubles() {
  return 2 * Planes<T>::P * Planes<T>::TK * PITCH;
}
// One 64 x PITCH tile (all planes).  Two stages fit in one tile.
template <typename T> __device__ __forceinline__ constexpr int tile_doubles() { return Planes<T>::P * 64 * PITCH; }
// Workgroup LDS: two tiles (the GEMM stages live in the first).
template <typename T> __device__ __forceinline__ constexpr int smem_doubles() { return 2 * tile_doubles<T>(); }

// ---------------------------------------------------------------------------
// Memory policy for the selected inverse X (and partial products), which
// other workgroups of the same launch write.  Coherent accesses are
// agent-scope relaxed atomics: they bypass the non-coherent per-XCD caches,
// so no cache-wide invalidation is ever needed to read a producer's data.
// ---------------------------------------------------------------------------
template <bool COH> struct Mem;
template <> struct Mem<false> {
  static __device__ __forceinline__ double ld(const double *p) { return *gp(p); }
  static __device__ __forceinline__ cplx ld(const cplx *p) {
    const double *q = reinterpret_cast<const double *>(p);
    return cplx{*gp(q), *gp(q + 1)};
  }
  static __device__ __forceinline__ void st(double *p, double v) { *gw(p) = v; }
  static __device__ __forceinline__ void st(cplx *p, cplx v) {
    double *q = reinterpret_cast<double *>(p);
    *gw(q) = v.re;
    *gw(q + 1) = v.im;
  }
};
template <> struct Mem<true> {
  static __device__ __forceinline__ double ld(const double *p) {
    return __hip_atomic_load(gp(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  static __device__ __forceinline__ cplx ld(const cplx *p) {
    const double *q = reinterpret_cast<const double *>(p);
    return cplx{__hip_atomic_load(gp(q), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                __hip_atomic_load(gp(q + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)};
  }
  static __device__ __forceinline__ void st(double *p, double v) {
    __hip_atomic_store(gw(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  static __device__ __forceinline__ void st(cplx *p, cplx v) {
    double *q = reinterpret_cast<double *>(p);
    __hip_atomic_store(gw(q), v.re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(gw(q + 1), v.im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};

__device__ __forceinline__ cplx masked(cplx v, int64_t m) { return cplx{masked(v.re, m), masked(v.im, m)}; }
__device__ __forceinline__ double shfl_xor_t(double v, int m) { return __shfl_xor(v, m); }
__device__ __forceinline__ cplx shfl_xor_t(cplx v, int m) { return cplx{__shfl_xor(v.re, m), __shfl_xor(v.im, m)}; }

// Plain global loads / stores of scalars through generic pointers.
template <typename T> __device__ __forceinline__ T gload(const T *p) { return Mem<false>::ld(p); }
template <typename T> __device__ __forceinline__ void gstore(T *p, T v) { Mem<false>::st(p, v); }
__device__ __forceinline__ Item gload(const Item *p) {
  const int32_t *q = reinterpret_cast<const int32_t *>(p);
  return Item{gp(q)[0], gp(q)[1], gp(q)[2], gp(q)[3]};
}

// Value of the first active lane, held in a scalar register.  Every branch
// and loop bound that a workgroup barrier depends on is made wave-uniform this
// way: a condition the compiler takes for divergent lets it restructure the
// loop so that some lanes of a wave reach the next barrier ahead of others
// (the barrier counts waves, not lanes).
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ Item uniform(const Item &it) {
  return Item{uniform(it.K), uniform(it.type), uniform(it.a), uniform(it.b)};
}

// ---------------------------------------------------------------------------
// MFMA tile
// ---------------------------------------------------------------------------
template <typename T> struct Acc {
  d4 v[Planes<T>::P][2][2];
};

template <typename T> __device__ __forceinline__ void acc_zero(Acc<T> &acc) {
#pragma unroll
  for (int p = 0; p < Planes<T>::P; ++p)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc.v[p][bi][bj] = d4{0.0, 0.0, 0.0, 0.0};
}

template <typename T, int TK = Planes<T>::TK>
__device__ __forceinline__ void stage_compute(const double *stg, Acc<T> &acc) {
  constexpr int P = Planes<T>::P;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w & 1, wj = w >> 1;
#pragma unroll
  for (int k4 = 0; k4 < TK / 4; ++k4) {
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

// Operand loaders run a three-level pipeline per stage of TK contraction
// indices: lev1 (index tables), lev2 (positions), lev3 (values).  Each loader
// defines its own per-stage state types S1, S2 (empty when a level has
// nothing to load) and the LDS slot of its m-th element for a stage.
template <typename T> struct Vals {
  T v[64 * Planes<T>::TK / NT];
};

// Loaders return raw loaded values; out-of-range elements (which were read
// from a clamped, valid address) are zeroed here, where the values are
// consumed.  Masking at the load would make the compiler wait for every load
// in the iteration that issued it, which serializes the pipeline.
// A loader whose elements may be stored transposed (the upper triangle of a
// Hermitian X_{C,C}) declares kConj and gives, per element, the factor of the
// imaginary plane: -1 where the element is conjugated, else +1.
template <class L, class = void> struct LoaderConj {
  static constexpr bool value = false;
};
template <class L> struct LoaderConj<L, std::void_t<decltype(L::kConj)>> {
  static constexpr bool value = L::kConj;
};

template <typename T, class L, class V, int TK = Planes<T>::TK>
__device__ __forceinline__ void stage_store(double *stg, int plane_off, int k0, const L &ld, const V &v) {
  constexpr int P = Planes<T>::P;
  constexpr int E = sizeof(v.v) / sizeof(v.v[0]);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int slot = ld.slot(k0, m);
    const T x = masked(v.v[m], ld.mask(k0, m));
#pragma unroll
    for (int p = 0; p < P; ++p) {
      double y = Planes<T>::get(x, p);
      if constexpr (LoaderConj<L>::value && P == 2) {
        if (p == 1) y *= ld.imsign(k0, m);
      }
      stg[(plane_off + p) * TK * PITCH + slot] = y;
    }
  }
}

// acc = A (64 x [kb, ke)) * B ([kb, ke) x 64).  LA fills the A planes, LB the
// B planes.  Pipeline: while stage kt is multiplied, the values of stage kt+2,
// the positions of stage kt+3 and the index entries of stage kt+4 are in
// flight.  The loop body has no branches: prefetch stage indices are clamped
// to the last stage (the redundant reloads at the end are harmless), so the
// waits the compiler inserts are counted waits on the oldest loads only.
// kb and ke must be wave-uniform.
template <typename T, class LA, class LB>
__device__ __forceinline__ void gemm_tile(int kb, int ke, const LA &la, const LB &lb, double *smem, Acc<T> &acc) {
  constexpr int P = Planes<T>::P, TK = Planes<T>::TK;
  acc_zero<T>(acc);
  const int nk = (ke - kb + TK - 1) / TK;
  if (nk <= 0) return;
  const int klast = kb + (nk - 1) * TK;
  auto kat = [&](int j) { return min(kb + j * TK, klast); };
  typename LA::S1 a1;
  typename LB::S1 b1;
  typename LA::S2 a2;
  typename LB::S2 b2;
  Vals<T> av, bv;
  la.lev1(kb, a1);
  lb.lev1(kb, b1);
  la.lev2(kb, a1, a2);
  lb.lev2(kb, b1, b2);
  la.lev3(kb, a2, av);
  lb.lev3(kb, b2, bv);
  stage_store<T>(smem, 0, kb, la, av);
  stage_store<T>(smem, P, kb, lb, bv);
  la.lev1(kat(1), a1);
  lb.lev1(kat(1), b1);
  la.lev2(kat(1), a1, a2);
  lb.lev2(kat(1), b1, b2);
  la.lev3(kat(1), a2, av);
  lb.lev3(kat(1), b2, bv);
  la.lev1(kat(2), a1);
  lb.lev1(kat(2), b1);
  la.lev2(kat(2), a1, a2);
  lb.lev2(kat(2), b1, b2);
  la.lev1(kat(3), a1);
  lb.lev1(kat(3), b1);
  lds_barrier();
  for (int kt = 0; kt < nk; ++kt) {
    stage_compute<T>(smem + (kt & 1) * stage_doubles<T>(), acc);
    double *nxt = smem + ((kt + 1) & 1) * stage_doubles<T>();
    stage_store<T>(nxt, 0, kat(kt + 1), la, av);
    stage_store<T>(nxt, P, kat(kt + 1), lb, bv);
    lds_barrier();
    la.lev3(kat(kt + 2), a2, av);
    lb.lev3(kat(kt + 2), b2, bv);
    la.lev2(kat(kt + 3), a1, a2);
    lb.lev2(kat(kt + 3), b1, b2);
    la.lev1(kat(kt + 4), a1);
    lb.lev1(kat(kt + 4), b1);
    __builtin_amdgcn_sched_barrier(0);  // issue the loads before the next MFMA block
  }
}

// Scatter the accumulators into an LDS tile C[p][j * PITCH + i]; caller syncs.
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
template <typename T> __device__ __forceinline__ void lds_put(double *ct, int i, int j, T v);
template <> __device__ __forceinline__ void lds_put<double>(double *ct, int i, int j, double v) {
  ct[j * PITCH + i] = v;
}
template <> __device__ __forceinline__ void lds_put<cplx>(double *ct, int i, int j, cplx v) {
  ct[j * PITCH + i] = v.re;
  ct[64 * PITCH + j * PITCH + i] = v.im;
}

// ---------------------------------------------------------------------------
// Loaders
// ---------------------------------------------------------------------------

struct Empty {};

// Column block of a panel's bottom part, k-major: value(kk, x) =
// P[off + (x0 + x) * ld + s + kbase + k0 + kk] for kbase + k0 + kk < kend and
// x0 + x < xmax (x = 0..63: a row of A^T or a column of B).
template <typename T, bool COH> struct LoadPanelK {
  using S1 = Empty;
  using S2 = Empty;
  const T *Pn;
  int64_t off;
  int ld, s, kbase, kend, x0, xmax;
  __device__ __forceinline__ int slot(int, int m) const {
    constexpr int TK = Planes<T>::TK;
    const int e = threadIdx.x + NT * m;
    return (e & (TK - 1)) * PITCH + e / TK;
  }
  __device__ __forceinline__ void lev1(int, S1 &) const {}
  __device__ __forceinline__ void lev2(int, const S1 &, S2 &) const {}
  __device__ __forceinline__ int64_t mask(int k0, int m) const {
    constexpr int TK = Planes<T>::TK;
    const int e = threadIdx.x + NT * m;
    return opaque_mask(kbase + k0 + (e & (TK - 1)) < kend && x0 + e / TK < xmax);
  }
  // Branch-free: out-of-range elements read the panel's first element (zeroed
  // when stored), so all loads of a stage issue together.
  __device__ __forceinline__ void lev3(int k0, const S2 &, Vals<T> &v) const {
    constexpr int TK = Planes<T>::TK;
#pragma unroll
    for (int m = 0; m < ept<T>(); ++m) {
      const int e = threadIdx.x + NT * m;
      const int kg = kbase + k0 + (e & (TK - 1)), xg = x0 + e / TK;
      const int64_t msk = mask(k0, m);
      v.v[m] = Mem<COH>::ld(Pn + ((((int64_t)xg * ld + s + kg) & msk) + off));
    }
  }
};

// A = X_{C,C} of node K (rows i0.., all columns), gathered from the
// ancestors' X panels through the canonical maps:
//   lower (i >= k): X[kcol[k] + posarr[kpos[k] + i]],  upper: X[kcol[i] + posarr[kpos[i] + k]].
// kcol/kpos of the 64 tile rows are staged in LDS (rt_col, rt_pos).  Lower
// blocks map lanes along i, upper blocks along k, so both read panel columns
// contiguously.
template <typename T, bool COH> struct LoadGather {
  static constexpr int E = 64 * Planes<T>::TK / NT;
  struct S1 {  // raw kcol / kpos entries of the stage's lower-part columns
    int64_t bl[E];
    int64_t plo[E];
  };
  struct S2 {  // panel column base and raw posarr entry
    int64_t base[E];
    int32_t pos[E];
  };
  static constexpr bool kConj = true;
  const T *X;
  const int64_t *kcol, *kpos;  // node-local per-row tables (global)
  const int32_t *posarr;
  const int64_t *rt_col, *rt_pos;  // LDS copies for rows i0 .. i0+63
  int c, kend, i0;  // rows and columns of X_{C,C} < c; contraction indices < kend
  double cs = 1.0;  // -1 in a Hermitian plan: the upper part is the conjugate of the stored lower part
  int64_t du = 0;   // LU plans: the upper part is read from X + du (the other panel set) at the
                    // transposed position
  __device__ __forceinline__ void coords(int k0, int m, int &i, int &kk) const {
    constexpr int TK = Planes<T>::TK;
    const int e = threadIdx.x + NT * m;
    if (i0 + 63 < k0) {  // strictly upper block
      kk = e & (TK - 1);
      i = e / TK;
    } else {
      i = e & 63;
      kk = e >> 6;
    }
  }
  __device__ __forceinline__ int slot(int k0, int m) const {
    int i, kk;
    coords(k0, m, i, kk);
    return kk * PITCH + i;
  }
  __device__ __forceinline__ int64_t mask(int k0, int m) const {
    int i, kk;
    coords(k0, m, i, kk);
    return opaque_mask(i0 + i < c && k0 + kk < kend);
  }
  __device__ __forceinline__ double imsign(int k0, int m) const {
    int i, kk;
    coords(k0, m, i, kk);
    return i0 + i < k0 + kk ? cs : 1.0;
  }
  // Each level loads unconditionally (clamped indices, opaque masks) and
  // keeps the raw results; they are combined one level later.
  __device__ __forceinline__ void lev1(int k0, S1 &r) const {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      int i, kk;
      coords(k0, m, i, kk);
      const int ig = i0 + i, kg = k0 + kk;
      const int64_t kq = (int64_t)kg & opaque_mask(ig < c && kg < c && ig >= kg);
      r.bl[m] = gp(kcol)[kq];
      r.plo[m] = gp(kpos)[kq];
    }
  }
  __device__ __forceinline__ void lev2(int k0, const S1 &r, S2 &q) const {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      int i, kk;
      coords(k0, m, i, kk);
      const int ig = i0 + i, kg = k0 + kk;
      const int64_t okm = opaque_mask(ig < c && kg < c);
      const int64_t lm = opaque_mask(ig >= kg);
      const int64_t bu = rt_col[i] + du, pu = rt_pos[i];
      q.base[m] = (r.bl[m] & lm) | (bu & ~lm);
      const int64_t pidx = (((r.plo[m] + ig) & lm) | ((pu + kg) & ~lm)) & okm;
      q.pos[m] = gp(posarr)[pidx];
    }
  }
  __device__ __forceinline__ void lev3(int k0, const S2 &q, Vals<T> &v) const {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      v.v[m] = Mem<COH>::ld(X + ((q.base[m] + (int64_t)q.pos[m]) & mask(k0, m)));
    }
  }
};

// LoadGather restricted to the terms one ancestor owns (the push form of
// Alg. 2): X_{C,C}(i, k) counts only when min(i, k) < en, i.e. when column
// min(i, k) of X_{C,C} lies in the owner's columns (rows and contraction
// indices start at the owner's first row st).  Loads stay at the base
// loader's (valid) addresses; the extra terms are zeroed where the stage is
// stored to LDS.
template <typename T, bool COH> struct LoadGatherSeg : LoadGather<T, COH> {
  int en;
  __device__ __forceinline__ int64_t mask(int k0, int m) const {
    int i, kk;
    this->coords(k0, m, i, kk);
    const int ig = this->i0 + i, kg = k0 + kk;
    return opaque_mask(ig < this->c && kg < this->kend && min(ig, kg) < en);
  }
};

// ---------------------------------------------------------------------------
// Dense operands (no index chain): the node's X_{C,C} buffer and the panel.
// ---------------------------------------------------------------------------
template <typename T> struct DenseTK;
template <> struct DenseTK<double> { static constexpr int TK = 32; };
template <> struct DenseTK<cplx> { static constexpr int TK = 16; };

template <typename T, int TK> struct DVals {
  T v[64 * TK / NT];
};

// Dense operand loaders.  Each thread owns fixed positions of the stage
// (slot m of thread t is element e = t + NT m); everything that does not move
// with the stage is computed once, so a full stage costs 64 TK / NT plain
// loads addressed as (wave-uniform base pointer) + (fixed 32-bit per-thread
// byte offset) and no per-load arithmetic.  Positions outside the operand are
// clamped onto valid memory and zeroed when the stage is stored to LDS; a
// stage that reaches past kend (the last one) clamps its contraction index.

// Load at a (wave-uniform) base plus a 32-bit byte offset, with the addition
// done on global-space pointers so that it maps onto the scalar-base +
// vector-offset addressing of the global loads.
__device__ __forceinline__ double ld_off(const double *base, uint32_t b) {
  return *reinterpret_cast<const SELINV_GAS double *>(reinterpret_cast<const SELINV_GAS char *>(gp(base)) + b);
}
__device__ __forceinline__ uint32_t ld_off(const uint32_t *base, uint32_t b) {
  return *reinterpret_cast<const SELINV_GAS uint32_t *>(reinterpret_cast<const SELINV_GAS char *>(gp(base)) + b);
}
__device__ __forceinline__ cplx ld_off(const cplx *base, uint32_t b) {
  const SELINV_GAS char *q = reinterpret_cast<const SELINV_GAS char *>(gp(base)) + b;
  return cplx{*reinterpret_cast<const SELINV_GAS double *>(q), *reinterpret_cast<const SELINV_GAS double *>(q + 8)};
}

// A(i, k) = G[k * ldg + i0 + i] for i0 + i < rows, k < kend (column-major);
// lanes run along i, so each column of the stage is one contiguous read.  The
// contraction index of a slot, k0 + (t >> 6) + 4 m, is uniform in a wave.
template <typename T, int TK> struct LoadDenseA {
  static constexpr int E = 64 * TK / NT;
  const T *G;
  int64_t ldg;
  int kend, kq;
  uint32_t vrow;  // byte offset of this thread's row (row 0 when outside)
  int64_t rmask;
  bool rows_full;
  __device__ __forceinline__ LoadDenseA(const T *G_, int ldg_, int rows, int kend_, int i0)
      : G(G_), ldg(ldg_), kend(kend_) {
    const int i = i0 + (threadIdx.x & 63);
    kq = uniform((int)(threadIdx.x >> 6));
    vrow = (uint32_t)(i < rows ? i : 0) * (uint32_t)sizeof(T);
    rmask = opaque_mask(i < rows);
    rows_full = i0 + 64 <= rows;
  }
  __device__ __forceinline__ int slot(int, int m) const {
    const int e = threadIdx.x + NT * m;
    return (e >> 6) * PITCH + (e & 63);
  }
  __device__ __forceinline__ bool all_valid(int k0) const { return rows_full && k0 + TK <= kend; }
  __device__ __forceinline__ int64_t mask(int k0, int m) const {
    return rmask & opaque_mask(k0 + kq + (NT / 64) * m < kend);
  }
  __device__ __forceinline__ void load(int k0, DVals<T, TK> &v) const {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int k = min(k0 + kq + (NT / 64) * m, kend - 1);
      v.v[m] = ld_off(G + (int64_t)k * ldg, vrow);
    }
  }
};

// A(i, k) = G(i0 + i, k) of a dense column-major buffer (leading dimension
// ldg), where the stages k0 >= kmir read the mirrored entries
// G[(i0 + i) * ldg + k] (conjugated in a Hermitian plan) with lanes along k,
// so that the loads stay contiguous, and the other stages read as
// LoadDenseA.  kmir = i0 + 64: X_{C,C} from a buffer that holds only its
// lower triangle and the full diagonal 64 x 64 blocks (X_{C,C} symmetric or
// Hermitian); kmir = 0: the transpose of the whole buffer; kmir past the
// contraction: the buffer itself.  Slot m of a thread in a mirrored stage is
// kk = t % TK, i = t / TK + (NT / TK) m.
template <typename T, int TK> struct LoadDenseASym : LoadDenseA<T, TK> {
  using Base = LoadDenseA<T, TK>;
  static constexpr int E = Base::E;
  static constexpr bool kConj = true;
  double cs = 1.0;       // -1 in a Hermitian plan
  int i0, kmir, kkt;     // row tile start; first mirrored stage; this thread's k in a mirrored stage
  uint32_t uoff[E];      // byte offsets of (row i0 + i, k0 + kkt) relative to G + i0 * ldg + k0 (rows clamped)
  uint32_t urow_ok = 0;  // bit m: the row of slot m is inside the operand
  __device__ __forceinline__ LoadDenseASym(const T *G_, int ldg_, int rows, int kend_, int i0_, int kmir_)
      : Base(G_, ldg_, rows, kend_, i0_), i0(i0_), kmir(kmir_) {
    kkt = threadIdx.x % TK;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int i = threadIdx.x / TK + (NT / TK) * m;
      const bool ok = i0 + i < rows;
      urow_ok |= ok ? (1u << m) : 0u;
      uoff[m] = (uint32_t)((int64_t)(ok ? i : 0) * ldg_ + kkt) * (uint32_t)sizeof(T);
    }
  }
  __device__ __forceinline__ bool upper(int k0) const { return k0 >= kmir; }
  __device__ __forceinline__ int slot(int k0, int m) const {
    const int e = threadIdx.x + NT * m;
    return upper(k0) ? (e % TK) * PITCH + e / TK : Base::slot(k0, m);
  }
  __device__ __forceinline__ int64_t mask(int k0, int m) const {
    return upper(k0) ? opaque_mask(((urow_ok >> m) & 1u) != 0 && k0 + kkt < this->kend) : Base::mask(k0, m);
  }
  __device__ __forceinline__ double imsign(int k0, int) const { return upper(k0) ? cs : 1.0; }
  // Branch-free forms of load and of the stage store (masks always applied;
  // the mirrored or direct form picked by wave-uniform selects), so that a
  // stage's loads and stores can share a basic block with the MFMAs of the
  // previous stage.
  __device__ __forceinline__ void load_bf(int k0, DVals<T, TK> &v) const {
    const bool up = upper(k0);
    const int over = k0 + kkt - (this->kend - 1);
    const uint32_t back = (uint32_t)(over > 0 ? over : 0) * (uint32_t)sizeof(T);
    // the element offset of the slot's base blended with an opaque uniform
    // mask, so that the compiler keeps one straight-line block (a select of
    // the two offsets becomes a branch)
    int su32 = uniform(up ? -1 : 0);
    asm("" : "+s"(su32));
    const int64_t su = su32;
    const int64_t eu = (int64_t)i0 * this->ldg + k0;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int k = min(k0 + this->kq + (NT / 64) * m, this->kend - 1);
      const int64_t eo = (eu & su) | (((int64_t)k * this->ldg) & ~su);
      v.v[m] = ld_off(this->G + eo, up ? uoff[m] - back : this->vrow);
    }
  }
  __device__ __forceinline__ void store_bf(double *stg, int plane_off, int k0, const DVals<T, TK> &v) const {
    constexpr int P = Planes<T>::P;
    const bool up = upper(k0);
    const double sg = up ? cs : 1.0;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int e = threadIdx.x + NT * m;
      const int slot = up ? (e % TK) * PITCH + e / TK : (e >> 6) * PITCH + (e & 63);
      const bool oku = ((urow_ok >> m) & 1u) != 0 && k0 + kkt < this->kend;
      const bool okl = this->rmask != 0 && k0 + this->kq + (NT / 64) * m < this->kend;
      const T x = masked(v.v[m], opaque_mask(up ? oku : okl));
#pragma unroll
      for (int p = 0; p < P; ++p) stg[(plane_off + p) * TK * PITCH + slot] = p == 1 ? Planes<T>::get(x, p) * sg : Planes<T>::get(x, p);
    }
  }
  __device__ __forceinline__ void load(int k0, DVals<T, TK> &v) const {
    if (upper(k0)) {
      const int over = k0 + kkt - (this->kend - 1);  // the last stage clamps k onto kend - 1
      const uint32_t back = (uint32_t)(over > 0 ? over : 0) * (uint32_t)sizeof(T);
      const T *base = this->G + (int64_t)i0 * this->ldg + k0;
#pragma unroll
      for (int m = 0; m < E; ++m) v.v[m] = ld_off(base, uoff[m] - back);
    } else {
      Base::load(k0, v);
    }
  }
};

// B(kk, x) = P[off + (x0 + x) * ld + s + k0 + kk] for k0 + kk < kend,
// x0 + x < xmax: a column block of a panel's bottom part, k-major.  Slot m of
// a thread is kk = t % TK, x = t / TK + (NT / TK) m.
template <typename T, int TK> struct LoadDenseB {
  static constexpr int E = 64 * TK / NT;
  const T *Pn;  // + off
  int kend, kk, xq, x0, xmax;
  uint32_t voff[E];  // byte offsets of (x, kk) relative to Pn + k0 (columns clamped)
  bool cols_full;
  __device__ __forceinline__ LoadDenseB(const T *Pn_, int64_t off, int ld, int s, int kend_, int x0_, int xmax_)
      : Pn(Pn_ + off), kend(kend_), x0(x0_), xmax(xmax_) {
    kk = threadIdx.x % TK;
    xq = threadIdx.x / TK;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int x = min(x0 + xq + (NT / TK) * m, xmax - 1);
      voff[m] = (uint32_t)((int64_t)x * ld + s + kk) * (uint32_t)sizeof(T);
    }
    cols_full = x0 + 64 <= xmax;
  }
  __device__ __forceinline__ int slot(int, int m) const {
    const int e = threadIdx.x + NT * m;
    return (e & (TK - 1)) * PITCH + e / TK;
  }
  __device__ __forceinline__ bool all_valid(int k0) const { return cols_full && k0 + TK <= kend; }
  __device__ __forceinline__ int64_t mask(int k0, int m) const {
    return opaque_mask(k0 + kk < kend && x0 + xq + (NT / TK) * m < xmax);
  }
  // branch-free forms (see LoadDenseASym::load_bf)
  __device__ __forceinline__ void load_bf(int k0, DVals<T, TK> &v) const {
    const int over = k0 + kk - (kend - 1);
    const uint32_t back = (uint32_t)(over > 0 ? over : 0) * (uint32_t)sizeof(T);
    const T *base = Pn + k0;
#pragma unroll
    for (int m = 0; m < E; ++m) v.v[m] = ld_off(base, voff[m] - back);
  }
  __device__ __forceinline__ void store_bf(double *stg, int plane_off, int k0, const DVals<T, TK> &v) const {
    constexpr int P = Planes<T>::P;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const T x = masked(v.v[m], mask(k0, m));
#pragma unroll
      for (int p = 0; p < P; ++p) stg[(plane_off + p) * TK * PITCH + slot(k0, m)] = Planes<T>::get(x, p);
    }
  }
  __device__ __forceinline__ void load(int k0, DVals<T, TK> &v) const {
    if (k0 + TK <= kend) {
      const T *base = Pn + k0;
#pragma unroll
      for (int m = 0; m < E; ++m) v.v[m] = ld_off(base, voff[m]);
    } else {  // last stage: clamp kk onto kend - 1
      const int over = k0 + kk - (kend - 1);
      const uint32_t back = (uint32_t)(over > 0 ? over : 0) * (uint32_t)sizeof(T);
      const T *base = Pn + k0;
#pragma unroll
      for (int m = 0; m < E; ++m) v.v[m] = ld_off(base, voff[m] - back);
    }
  }
};

// B(k, x) = M[k * ld + x0 + x] for k < kend, x0 + x < xmax: a row-major view
// (the transpose of a column-major block); lanes run along x, and the row of a
// slot, k0 + (t >> 6) + 4 m, is uniform in a wave.
template <typename T, int TK> struct LoadDenseBT {
  static constexpr int E = 64 * TK / NT;
  static constexpr bool kConj = true;  // the transposed operand: conjugated in a Hermitian plan
  const T *M;
  int64_t ld;
  int kend, kq;
  uint32_t vcol;
  int64_t cmask;
  bool cols_full;
  double cs = 1.0;  // -1: conjugate every element
  __device__ __forceinline__ double imsign(int, int) const { return cs; }
  __device__ __forceinline__ LoadDenseBT(const T *M_, int ld_, int kend_, int x0, int xmax)
      : M(M_), ld(ld_), kend(kend_) {
    const int x = x0 + (threadIdx.x & 63);
    kq = uniform((int)(threadIdx.x >> 6));
    vcol = (uint32_t)(x < xmax ? x : x0) * (uint32_t)sizeof(T);
    cmask = opaque_mask(x < xmax);
    cols_full = x0 + 64 <= xmax;
  }
  __device__ __forceinline__ int slot(int, int m) const {
    const int e = threadIdx.x + NT * m;
    return (e >> 6) * PITCH + (e & 63);
  }
  __device__ __forceinline__ bool all_valid(int k0) const { return cols_full && k0 + TK <= kend; }
  __device__ __forceinline__ int64_t mask(int k0, int m) const {
    return cmask & opaque_mask(k0 + kq + (NT / 64) * m < kend);
  }
  __device__ __forceinline__ void load(int k0, DVals<T, TK> &v) const {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int k = min(k0 + kq + (NT / 64) * m, kend - 1);
      v.v[m] = ld_off(M + (int64_t)k * ld, vcol);
    }
  }
};

// Stage store of the dense loaders: a stage wholly inside the operand (the
// common case) is stored without masks.
template <typename T, class L, class V, int TK>
__device__ __forceinline__ void stage_store_dense(double *stg, int plane_off, int k0, const L &ld, const V &v) {
  constexpr int P = Planes<T>::P;
  constexpr int E = sizeof(v.v) / sizeof(v.v[0]);
  // the imaginary plane's factor of a conjugating loader (see LoaderConj)
  auto plane = [&](const T &x, int p, int m) {
    double y = Planes<T>::get(x, p);
    if constexpr (LoaderConj<L>::value && P == 2) {
      if (p == 1) y *= ld.imsign(k0, m);
    }
    return y;
  };
  if (uniform(ld.all_valid(k0) ? 1 : 0)) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int slot = ld.slot(k0, m);
#pragma unroll
      for (int p = 0; p < P; ++p) stg[(plane_off + p) * TK * PITCH + slot] = plane(v.v[m], p, m);
    }
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int slot = ld.slot(k0, m);
      const T x = masked(v.v[m], ld.mask(k0, m));
#pragma unroll
      for (int p = 0; p < P; ++p) stg[(plane_off + p) * TK * PITCH + slot] = plane(x, p, m);
    }
  }
}

template <typename T, int TK> __device__ __forceinline__ constexpr int dense_stage_doubles() {
  return 2 * Planes<T>::P * TK * PITCH;
}

// Complex products with three real MFMA chains instead of four (the 3M or
// Gauss form): P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi), then
// Re = P1 - P2 and Im = P3 - P1 - P2.  The operand sums are formed from the
// two LDS planes as they are read, so the stages keep their layout.  Its
// rounding error bound is that of the four-product form with |Ar| + |Ai| and
// |Br| + |Bi| in place of the moduli (the same order).
struct Acc3M {
  d4 v[3][2][2];
};

template <int TK>
__device__ __forceinline__ void stage_compute_3m(const double *stg, Acc3M &acc) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w & 1, wj = w >> 1;
#pragma unroll
  for (int k4 = 0; k4 < TK / 4; ++k4) {
    const int r = (4 * k4 + (lane >> 4)) * PITCH + (lane & 15);
    double a[2][2], b[2][2], as[2], bs[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        a[x][p] = stg[p * TK * PITCH + r + 32 * wi + 16 * x];
        b[x][p] = stg[(2 + p) * TK * PITCH + r + 32 * wj + 16 * x];
      }
      as[x] = a[x][0] + a[x][1];
      bs[x] = b[x][0] + b[x][1];
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        acc.v[0][bi][bj] = mfma16(a[bi][0], b[bj][0], acc.v[0][bi][bj]);
        acc.v[1][bi][bj] = mfma16(a[bi][1], b[bj][1], acc.v[1][bi][bj]);
        acc.v[2][bi][bj] = mfma16(as[bi], bs[bj], acc.v[2][bi][bj]);
      }
  }
}

// acc (+)= A (64 x [kb, ke)) * B ([kb, ke) x 64) from dense operands.  Two
// register sets alternate, so the loads of a stage are issued two
// stage-computations before they are stored to LDS; waits are counted waits
// on the older set only.  kb, ke and accumulate must be wave-uniform.
// G3: complex products in the three-chain form (Acc3M) instead of four.
template <typename T, bool G3 = false, class LA, class LB>
__device__ __forceinline__ void gemm_dense(int kb, int ke, const LA &la, const LB &lb, double *smem, Acc<T> &acc,
                                           bool accumulate = false) {
  constexpr int TK = DenseTK<T>::TK, P = Planes<T>::P;
  constexpr bool M3 = G3 && P == 2;
  constexpr int SD = dense_stage_doubles<T, TK>();
  using V = DVals<T, TK>;
  if (!accumulate) acc_zero<T>(acc);
  const int nk = (ke - kb + TK - 1) / TK;
  if (nk <= 0) return;
  Acc3M a3;
  if constexpr (M3) {
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) a3.v[q][bi][bj] = d4{0.0, 0.0, 0.0, 0.0};
  }
  auto compute = [&](const double *stg) {
    if constexpr (M3)
      stage_compute_3m<TK>(stg, a3);
    else
      stage_compute<T, TK>(stg, acc);
  };
  const int klast = kb + (nk - 1) * TK;
  auto kat = [&](int j) { return min(kb + j * TK, klast); };
  V a0, b0, a1, b1;
  la.load(kb, a0);
  lb.load(kb, b0);
  la.load(kat(1), a1);
  lb.load(kat(1), b1);
  stage_store_dense<T, LA, V, TK>(smem, 0, kb, la, a0);
  stage_store_dense<T, LB, V, TK>(smem, P, kb, lb, b0);
  la.load(kat(2), a0);
  lb.load(kat(2), b0);
  lds_barrier();
  for (int kt = 0;; kt += 2) {
    // LDS stage 0 holds kt; set 1 holds kt + 1, set 0 holds kt + 2
    compute(smem);
    if (kt + 1 >= nk) break;
    stage_store_dense<T, LA, V, TK>(smem + SD, 0, kat(kt + 1), la, a1);
    stage_store_dense<T, LB, V, TK>(smem + SD, P, kat(kt + 1), lb, b1);
    lds_barrier();
    la.load(kat(kt + 3), a1);
    lb.load(kat(kt + 3), b1);
    __builtin_amdgcn_sched_barrier(0);  // issue the loads before the MFMA block
    compute(smem + SD);
    if (kt + 2 >= nk) break;
    stage_store_dense<T, LA, V, TK>(smem, 0, kat(kt + 2), la, a0);
    stage_store_dense<T, LB, V, TK>(smem, P, kat(kt + 2), lb, b0);
    lds_barrier();
    la.load(kat(kt + 4), a0);
    lb.load(kat(kt + 4), b0);
    __builtin_amdgcn_sched_barrier(0);
  }
  if constexpr (M3) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const d4 re = a3.v[0][bi][bj] - a3.v[1][bi][bj];
        const d4 im = a3.v[2][bi][bj] - a3.v[0][bi][bj] - a3.v[1][bi][bj];
        acc.v[0][bi][bj] += re;
        acc.v[1][bi][bj] += im;
      }
  }
  lds_barrier();  // the caller reuses the stage buffers
}


// Issue order inside one step of gemm_dense_il: each of its NM MFMAs is
// followed by one of the NW LDS stores of the next stage, then by one of the
// NL global loads of the stage after it (the stage's own LDS reads are left
// to the scheduler).
template <int NM, int NW, int NL>
__device__ __forceinline__ void interleave_stage() {
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
    if (i < NW)
      __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // DS write
    else if (i < NW + NL)
      __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // VMEM read
  }
}

// gemm_dense with the branch-free loaders (load_bf / store_bf): each loop
// step is one basic block holding a stage's MFMAs, the LDS stores of the next
// stage (into the other buffer) and the global loads of the stage after
// that, so the stores and loads can issue in the shadow of the MFMAs instead
// of between them; one barrier per stage.  Same operands and results as
// gemm_dense (accumulate = false).
template <typename T, bool G3, class LA, class LB>
__device__ __forceinline__ void gemm_dense_il(int kb, int ke, const LA &la, const LB &lb, double *smem, Acc<T> &acc) {
  constexpr int TK = DenseTK<T>::TK, P = Planes<T>::P;
  constexpr bool M3 = G3 && P == 2;
  constexpr int SD = dense_stage_doubles<T, TK>();
  using V = DVals<T, TK>;
  acc_zero<T>(acc);
  const int nk = (ke - kb + TK - 1) / TK;
  if (nk <= 0) return;
  Acc3M a3;
  if constexpr (M3) {
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) a3.v[q][bi][bj] = d4{0.0, 0.0, 0.0, 0.0};
  }
  auto compute = [&](const double *stg) {
    if constexpr (M3)
      stage_compute_3m<TK>(stg, a3);
    else
      stage_compute<T, TK>(stg, acc);
  };
  const int klast = kb + (nk - 1) * TK;
  auto kat = [&](int j) { return min(kb + j * TK, klast); };
  // one register set: the loads of stage kt + 2 are issued with the MFMAs of
  // stage kt and stored with those of stage kt + 1
  V a, b;
  la.load_bf(kb, a);
  lb.load_bf(kb, b);
  la.store_bf(smem, 0, kb, a);
  lb.store_bf(smem, P, kb, b);
  la.load_bf(kat(1), a);
  lb.load_bf(kat(1), b);
  lds_barrier();
  for (int kt = 0; kt + 1 < nk; ++kt) {
    double *nxt = smem + ((kt + 1) & 1) * SD;
    compute(smem + (kt & 1) * SD);
    la.store_bf(nxt, 0, kat(kt + 1), a);
    lb.store_bf(nxt, P, kat(kt + 1), b);
    la.load_bf(kat(kt + 2), a);
    lb.load_bf(kat(kt + 2), b);
    // MFMAs per stage: (TK / 4) steps of 2 x 2 blocks (x 3 chains in the 3M form)
    interleave_stage<(TK / 4) * 4 * (M3 ? 3 : 1), 2 * LA::E * P, 2 * LA::E>();
    lds_barrier();
  }
  compute(smem + ((nk - 1) & 1) * SD);
  if constexpr (M3) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const d4 re = a3.v[0][bi][bj] - a3.v[1][bi][bj];
        const d4 im = a3.v[2][bi][bj] - a3.v[0][bi][bj] - a3.v[1][bi][bj];
        acc.v[0][bi][bj] += re;
        acc.v[1][bi][bj] += im;
      }
  }
  lds_barrier();  // the caller reuses the stage buffers
}

// ---------------------------------------------------------------------------
// 128 x 128 FP64 tile (GEMM-1 of large dense-buffer nodes, a tune-table
// choice).  Each wave owns a 64 x 64 quadrant (4 x 4 blocks of 16 x 16), so a
// 16-deep stage carries 64 MFMAs per wave for the same 32 KB of operands as a
// 32-deep stage of the 64 x 64 tile (which carries 32): twice the flops per
// byte read through L2, for the FP64 case where the 64 x 64 tile is bound by
// the operand traffic rather than by the matrix cores.
// ---------------------------------------------------------------------------
constexpr int kT128K = 16;      // contraction indices per stage
constexpr int PITCH128 = 129;   // LDS row pitch (doubles) of a 128-wide operand plane

struct Acc128 {
  d4 v[4][4];
};

__device__ __forceinline__ constexpr int stage128_doubles() { return 2 * kT128K * PITCH128; }

// A(i, k) = G[k * ldg + i0 + i], i < 128 (column-major): lanes along i, the
// contraction index of a slot (k0 + (t >> 7) + 2 m) is uniform in a wave.
struct LoadDenseA128 {
  static constexpr int E = 128 * kT128K / NT;
  const double *G;
  int64_t ldg;
  int kend, kq;
  uint32_t vrow;
  int64_t rmask;
  bool rows_full;
  __device__ __forceinline__ LoadDenseA128(const double *G_, int ldg_, int rows, int kend_, int i0)
      : G(G_), ldg(ldg_), kend(kend_) {
    const int i = i0 + (threadIdx.x & 127);
    kq = uniform((int)(threadIdx.x >> 7));
    vrow = (uint32_t)(i < rows ? i : 0) * 8u;
    rmask = opaque_mask(i < rows);
    rows_full = i0 + 128 <= rows;
  }
  __device__ __forceinline__ int slot(int m) const {
    const int e = threadIdx.x + NT * m;
    return (e >> 7) * PITCH128 + (e & 127);
  }
  __device__ __forceinline__ bool all_valid(int k0) const { return rows_full && k0 + kT128K <= kend; }
  __device__ __forceinline__ int64_t mask(int k0, int m) const {
    return rmask & opaque_mask(k0 + kq + (NT / 128) * m < kend);
  }
  __device__ __forceinline__ void load(int k0, double (&v)[E]) const {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int k = min(k0 + kq + (NT / 128) * m, kend - 1);
      v[m] = ld_off(G + (int64_t)k * ldg, vrow);
    }
  }
};

// B(kk, x) = P[off + (x0 + x) * ld + s + k0 + kk], x < 128: a column block of
// a panel's bottom part, k-major.  Slot m of a thread: kk = t % 16,
// x = t / 16 + 16 m.
struct LoadDenseB128 {
  static constexpr int E = 128 * kT128K / NT;
  const double *Pn;
  int kend, kk, xq, x0, xmax;
  uint32_t voff[E];
  bool cols_full;
  __device__ __forceinline__ LoadDenseB128(const double *Pn_, int64_t off, int ld, int s, int kend_, int x0_, int xmax_)
      : Pn(Pn_ + off), kend(kend_), x0(x0_), xmax(xmax_) {
    kk = threadIdx.x % kT128K;
    xq = threadIdx.x / kT128K;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int x = min(x0 + xq + (NT / kT128K) * m, xmax - 1);
      voff[m] = (uint32_t)((int64_t)x * ld + s + kk) * 8u;
    }
    cols_full = x0 + 128 <= xmax;
  }
  __device__ __forceinline__ int slot(int m) const {
    const int e = threadIdx.x + NT * m;
    return (e % kT128K) * PITCH128 + e / kT128K;
  }
  __device__ __forceinline__ bool all_valid(int k0) const { return cols_full && k0 + kT128K <= kend; }
  __device__ __forceinline__ int64_t mask(int k0, int m) const {
    return opaque_mask(k0 + kk < kend && x0 + xq + (NT / kT128K) * m < xmax);
  }
  __device__ __forceinline__ void load(int k0, double (&v)[E]) const {
    const int over = k0 + kk - (kend - 1);  // the last stage clamps kk onto kend - 1
    const uint32_t back = (uint32_t)(over > 0 ? over : 0) * 8u;
    const double *base = Pn + k0;
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = ld_off(base, voff[m] - back);
  }
};

template <class L>
__device__ __forceinline__ void stage128_store(double *plane, int k0, const L &ld, const double (&v)[L::E]) {
  if (uniform(ld.all_valid(k0) ? 1 : 0)) {
#pragma unroll
    for (int m = 0; m < L::E; ++m) plane[ld.slot(m)] = v[m];
  } else {
#pragma unroll
    for (int m = 0; m < L::E; ++m) plane[ld.slot(m)] = masked(v[m], ld.mask(k0, m));
  }
}

// One stage: A plane [k][i] then B plane [k][x], both kT128K x PITCH128.
__device__ __forceinline__ void stage128_compute(const double *stg, Acc128 &acc) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w & 1, wj = w >> 1;
#pragma unroll
  for (int k4 = 0; k4 < kT128K / 4; ++k4) {
    const int r = (4 * k4 + (lane >> 4)) * PITCH128 + (lane & 15);
    double a[4], b[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      a[x] = stg[r + 64 * wi + 16 * x];
      b[x] = stg[kT128K * PITCH128 + r + 64 * wj + 16 * x];
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) acc.v[bi][bj] = mfma16(a[bi], b[bj], acc.v[bi][bj]);
  }
}

// acc = A (128 x [kb, ke)) * B ([kb, ke) x 128), the two-register-set
// pipeline of gemm_dense.  kb and ke must be wave-uniform.
__device__ __forceinline__ void gemm_dense128(int kb, int ke, const LoadDenseA128 &la, const LoadDenseB128 &lb,
                                              double *smem, Acc128 &acc) {
  constexpr int TK = kT128K, SD = stage128_doubles();
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc.v[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};
  const int nk = (ke - kb + TK - 1) / TK;
  if (nk <= 0) return;
  const int klast = kb + (nk - 1) * TK;
  auto kat = [&](int j) { return min(kb + j * TK, klast); };
  double a0[LoadDenseA128::E], b0[LoadDenseB128::E], a1[LoadDenseA128::E], b1[LoadDenseB128::E];
  la.load(kb, a0);
  lb.load(kb, b0);
  la.load(kat(1), a1);
  lb.load(kat(1), b1);
  stage128_store(smem, kb, la, a0);
  stage128_store(smem + TK * PITCH128, kb, lb, b0);
  la.load(kat(2), a0);
  lb.load(kat(2), b0);
  lds_barrier();
  for (int kt = 0;; kt += 2) {
    stage128_compute(smem, acc);
    if (kt + 1 >= nk) break;
    stage128_store(smem + SD, kat(kt + 1), la, a1);
    stage128_store(smem + SD + TK * PITCH128, kat(kt + 1), lb, b1);
    lds_barrier();
    la.load(kat(kt + 3), a1);
    lb.load(kat(kt + 3), b1);
    __builtin_amdgcn_sched_barrier(0);
    stage128_compute(smem + SD, acc);
    if (kt + 2 >= nk) break;
    stage128_store(smem, kat(kt + 2), la, a0);
    stage128_store(smem + TK * PITCH128, kat(kt + 2), lb, b0);
    lds_barrier();
    la.load(kat(kt + 4), a0);
    lb.load(kat(kt + 4), b0);
    __builtin_amdgcn_sched_barrier(0);
  }
  lds_barrier();
}

}  // namespace selinv
