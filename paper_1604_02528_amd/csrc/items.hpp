// Work items of the selected-inversion traversal (device code shared by the
// forward and adjoint kernels): the dense X_{C,C} gather, the GEMM-1 tile with
// its fused share of GEMM-2, the split-tile reduction and the diagonal-block
// tile.  See plan.hpp for the item vocabulary.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"
#include "scalar.hpp"
#include "tile.hpp"

namespace selinv {

// ---------------------------------------------------------------------------
// Work items
// ---------------------------------------------------------------------------
template <typename T> struct Ctx {
  const DevPlan *pl;
  const T *Lp;  // normalized panels of this matrix
  T *Xp;        // selected inverse of this matrix
  T *Pp;        // GEMM-2 partial products of this matrix
  T *Gp;        // dense X_{C,C} buffers of this matrix
  T *Yp;        // partial GEMM-1 tiles of this matrix (split nodes)
};

// The same from a record (wave-uniform values, kept in scalar registers).
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = uniform((int32_t)(uint32_t)v), hi = uniform((int32_t)(v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ NodeInfo uniform(const NodeInfo &a) {
  NodeInfo n = a;
  n.K = uniform(a.K);
  n.s = uniform(a.s);
  n.c = uniform(a.c);
  n.ldg = uniform(a.ldg);
  n.split = uniform(a.split);
  n.kchunk = uniform(a.kchunk);
  n.defer2 = uniform(a.defer2);
  n.glow = uniform(a.glow);
  n.off = uniform64(a.off);
  n.rp = uniform64(a.rp);
  n.goff = uniform64(a.goff);
  n.poff = uniform64(a.poff);
  n.yoff = uniform64(a.yoff);
  return n;
}

// NodeInfo from the plan's node tables (the persistent schedule and the
// adjoint, whose items carry only the node index).
__device__ __forceinline__ NodeInfo node_info(const DevPlan &pl, int K) {
  NodeInfo n;
  n.K = K;
  n.s = uniform(gp(pl.node_s)[K]);
  n.c = uniform(gp(pl.node_c)[K]);
  n.ldg = uniform(gp(pl.node_ldg)[K]);
  n.split = uniform(gp(pl.node_split)[K]);
  n.kchunk = uniform(gp(pl.node_kchunk)[K]);
  n.defer2 = n.glow = 0;
  n.off = uniform64(gp(pl.node_off)[K]);
  n.rp = uniform64(gp(pl.node_rowptr)[K]);
  n.goff = uniform64(gp(pl.node_goff)[K]);
  n.poff = uniform64(gp(pl.node_poff)[K]);
  n.yoff = uniform64(gp(pl.node_yoff)[K]);
  n.pad2 = 0;
  return n;
}

// Block (a, b), a >= b, of X_{C,C} for a node with a dense buffer G (column
// major, leading dimension ldg): element (i, k), i >= k, is the lower-part
// entry Src[kcol[k] + posarr[kpos[k] + i]] of the ancestor owning column k
// (Src: the X panels, or any array in the same panel layout); it is written
// to G(i, k) and G(k, i) (conjugated in a Hermitian plan; in an LU plan G(k, i)
// is the entry at the same position of the second panel set, X^T).  Lanes run
// along i (one column k per wave and step) for the gather and the G(i, k)
// stores; the mirror stores go through an LDS transpose so that they are
// contiguous too.
// MAYBE_LU = false compiles the LU branch out (a kernel that never runs an LU plan).
template <typename T, bool MAYBE_LU = true>
__device__ void do_gtile(const Ctx<T> &cx, const NodeInfo &nd, int a, int b, double *smem, int64_t *rt, const T *Src) {
  const DevPlan &pl = *cx.pl;
  const int c = uniform(nd.c);
  const int64_t rp = nd.rp;
  const int ldg = nd.ldg;
  T *G = cx.Gp + nd.goff;
  const int i0 = a * 64, k0 = b * 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int Q = 64 * 64 / NT;
  // three dependent rounds: the gather tables of the block's 64 columns (into
  // LDS), the positions of all of a thread's elements, then their values.
  // Element q of a thread: row i = i0 + lane, column k = k0 + w + 4 q.
  if (threadIdx.x < 64) {
    const int k = k0 + threadIdx.x;
    const int64_t kq = k < c ? k : 0;
    rt[threadIdx.x] = gp(pl.kcol)[rp + kq];
    rt[64 + threadIdx.x] = gp(pl.kpos)[rp + kq];
  }
  lds_barrier();
  const int i = i0 + lane;
  int32_t pos[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int kl = w + 4 * q, k = k0 + kl;
    pos[q] = gp(pl.posarr)[(rt[64 + kl] + i) & opaque_mask(i < c && k < c && i >= k)];
  }
  T v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int kl = w + 4 * q, k = k0 + kl;
    v[q] = Mem<false>::ld(Src + ((rt[kl] + (int64_t)pos[q]) & opaque_mask(i < c && k < c && i >= k)));
  }
  const bool lu = MAYBE_LU && uniform(pl.half > 0 ? 1 : 0) != 0;
  if (lu) {  // the mirror values: the same positions of the X^T set
    T u[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int kl = w + 4 * q, k = k0 + kl;
      u[q] = Mem<false>::ld(Src + pl.half + ((rt[kl] + (int64_t)pos[q]) & opaque_mask(i < c && k < c && i >= k)));
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int kl = w + 4 * q, k = k0 + kl;
      const bool ok = i < c && k < c && i >= k;
      lds_put<T>(smem, lane, kl, masked(u[q], opaque_mask(ok)));
      if (ok) Mem<false>::st(G + (int64_t)k * ldg + i, masked(v[q], opaque_mask(ok)));
    }
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int kl = w + 4 * q, k = k0 + kl;
      const bool ok = i < c && k < c && i >= k;
      const T x = masked(v[q], opaque_mask(ok));
      lds_put<T>(smem, lane, kl, x);  // tile[i][k] at smem[k * PITCH + i]
      if (ok) Mem<false>::st(G + (int64_t)k * ldg + i, x);
    }
  }
  lds_barrier();
  // mirror: G(k, i) = tile[i][k] (its conjugate if Hermitian; the X^T entry
  // in an LU plan), lanes along k; a lower-only buffer keeps the mirrors of
  // diagonal blocks alone
  const double cs = lu ? 1.0 : pl.csign;
  if (uniform(nd.glow != 0 && a != b ? 0 : 1)) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + NT * q;
      const int kl = e & 63, il = e >> 6, i = i0 + il, k = k0 + kl;
      if (i < c && k < c && i > k) Mem<false>::st(G + (int64_t)i * ldg + k, cj(lds_get<T>(smem, il, kl), cs));
    }
  }
  lds_barrier();
}

// Store -acc (a 64 x 64 tile of X_{C,K} = -X_{C,C} Lhat) into X, rows 64a..
// of C(K) and columns 64b.. of K, through LDS so that the stores coalesce.
template <typename T, bool COH>
__device__ void store_xtile(const Ctx<T> &cx, const NodeInfo &nd, int a, int b, const Acc<T> &acc, double *smem) {
  const DevPlan &pl = *cx.pl;
  const int s = nd.s, c = nd.c, ld = s + c;
  const int64_t off = nd.off;
  const int i0 = a * 64, j0 = b * 64;
  acc_to_lds<T>(acc, smem);
  lds_barrier();
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = e & 63, j = e >> 6;
    if (i0 + i < c && j0 + j < s)
      Mem<COH>::st(cx.Xp + off + (int64_t)(j0 + j) * ld + s + i0 + i, SOps<T>::scale(-1.0, lds_get<T>(smem, i, j)));
  }
  lds_barrier();
}

// R[p][j * PITCH + x] = (Ls^T acc)(x, j) for a 64 x 64 block: Ls holds
// Lhat[tile rows i, 64 columns x] as Ls[p][i * PITCH + x] (already in LDS,
// barrier done); acc is a 64 x 64 GEMM-1 tile in the accumulator layout,
// which is the MFMA B-operand layout for a contraction over the tile rows
// (register v of a 16 x 16 block holds rows 4v..4v+3 of lanes l / 16).  R
// overwrites Ls; ends with a barrier.  The 64 columns x run in parts of
// 16 XB (all 64 for FP64, 16 for complex, whose three product chains per
// block take more registers): R's columns of a part overwrite Ls's, which
// only that part reads.  Complex products take three real chains (see
// Acc3M).
template <typename T>
__device__ void gemm2_block(const Acc<T> &acc, double *Ls) {
  constexpr int P = Planes<T>::P, C = P == 1 ? 1 : 3;  // product chains
  constexpr int XB = P == 1 ? 4 : 1;                   // 16-column blocks per part
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w & 1, wj = w >> 1;
#pragma unroll 1
  for (int h = 0; h < 4 / XB; ++h) {
    d4 pacc[C][XB][2];
#pragma unroll
    for (int q = 0; q < C; ++q)
#pragma unroll
      for (int xb = 0; xb < XB; ++xb)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) pacc[q][xb][bj] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4) {
        const int row = 32 * wi + 16 * bi + 4 * k4 + (lane >> 4);
#pragma unroll
        for (int xb = 0; xb < XB; ++xb) {
          const int x = 16 * (XB * h + xb) + (lane & 15);
          if constexpr (P == 1) {
            const double af = Ls[row * PITCH + x];
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) pacc[0][xb][bj] = mfma16(af, acc.v[0][bi][bj][k4], pacc[0][xb][bj]);
          } else {
            const double a0 = Ls[row * PITCH + x], a1 = Ls[64 * PITCH + row * PITCH + x];
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
              const double b0 = acc.v[0][bi][bj][k4], b1 = acc.v[1][bi][bj][k4];
              pacc[0][xb][bj] = mfma16(a0, b0, pacc[0][xb][bj]);
              pacc[1][xb][bj] = mfma16(a1, b1, pacc[1][xb][bj]);
              pacc[2][xb][bj] = mfma16(a0 + a1, b0 + b1, pacc[2][xb][bj]);
            }
          }
        }
      }
    lds_barrier();
    // sum the two row halves (wi = 0, 1) into R's columns of this part
    double *R = Ls;
    for (int part = 0; part < 2; ++part) {
      if (wi == part) {
#pragma unroll
        for (int xb = 0; xb < XB; ++xb)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) {
            d4 out[P];
            if constexpr (P == 1) {
              out[0] = pacc[0][xb][bj];
            } else {
              out[0] = pacc[0][xb][bj] - pacc[1][xb][bj];
              out[1] = pacc[2][xb][bj] - pacc[0][xb][bj] - pacc[1][xb][bj];
            }
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int x = 16 * (XB * h + xb) + 4 * v + (lane >> 4);
                const int j = 32 * wj + 16 * bj + (lane & 15);
                double &r = R[p * 64 * PITCH + j * PITCH + x];
                r = part == 0 ? out[p][v] : r + out[p][v];
              }
          }
      }
      lds_barrier();
    }
  }
}

// Row tile a's share of GEMM-2 (Alg. 1 step 4): P_a[:, 64b..] = Lhat[rows of
// tile a, :]^T Y[tile a, 64b..] = -(Lhat_a^T acc) (^H in a Hermitian plan;
// Uhat_{K,C} of the U^T panel set in place of Lhat^T in an LU plan),
// written to the partial buffer (column-major s x s per row tile); rows
// 64qb .. 64qe - 1 of P_a only.  PF: load the next 64 columns of Lhat while
// the current block is multiplied (off in kernels that rely on occupancy
// instead, so that the prefetch registers do not cost a workgroup per CU).
template <typename T, bool COH, bool PF = true>
__device__ void gemm2_partial(const Ctx<T> &cx, const NodeInfo &nd, int a, int b, const Acc<T> &acc, double *smem,
                              int qb = 0, int qe = 1 << 20) {
  constexpr int P = Planes<T>::P;
  const DevPlan &pl = *cx.pl;
  const int s = nd.s, c = nd.c, ld = s + c;
  const int64_t off = nd.off;
  const int i0 = a * 64, j0 = b * 64;
  const int64_t pbase = nd.poff + (int64_t)a * s * s;
  double *Ls = smem;  // Lhat[i0 .. i0+63, q0 .. q0+63] as Ls[p][i * PITCH + x]
  // the next 64 columns of Lhat are loaded while the current block is multiplied
  T lv[64 * 64 / NT];
  auto load_l = [&](int q0) {
#pragma unroll
    for (int q = 0; q < 64 * 64 / NT; ++q) {
      const int e = threadIdx.x + NT * q;
      const int i = e & 63, x = e >> 6;
      lv[q] = gload(cx.Lp + pl.half + off + (((int64_t)(q0 + x) * ld + s + i0 + i) & opaque_mask(i0 + i < c && q0 + x < s)));
    }
  };
  const int qend = min(s, qe * 64);
  const double cs = pl.csign;
  if (PF) load_l(qb * 64);
  for (int q0 = qb * 64; q0 < qend; q0 += 64) {
    if (!PF) load_l(q0);
#pragma unroll
    for (int q = 0; q < 64 * 64 / NT; ++q) {
      const int e = threadIdx.x + NT * q;
      const int i = e & 63, x = e >> 6;
      const T v = cj(masked(lv[q], opaque_mask(i0 + i < c && q0 + x < s)), cs);
#pragma unroll
      for (int p = 0; p < P; ++p) Ls[p * 64 * PITCH + i * PITCH + x] = Planes<T>::get(v, p);
    }
    lds_barrier();
    if (PF && q0 + 64 < qend) load_l(q0 + 64);
    gemm2_block<T>(acc, Ls);
    // P = Lhat^T Y = -(Lhat^T acc)
    const double *R = Ls;
    for (int e = threadIdx.x; e < 64 * 64; e += NT) {
      const int x = e & 63, j = e >> 6;
      if (q0 + x < s && j0 + j < s)
        Mem<COH>::st(cx.Pp + pbase + (int64_t)(j0 + j) * s + q0 + x, SOps<T>::scale(-1.0, lds_get<T>(R, x, j)));
    }
    lds_barrier();
  }
}

// GEMM-1 tile, rows 64a.. and columns 64b.. of X_{C,K} (Alg. 1 step 3):
//   acc = X_{C,C}[tile rows, k] Lhat_{C,K}[k, tile columns], k in this part's
// share of [0, c).  A node without an R phase stores Y = -acc into X and its
// row tile's share of GEMM-2 (step 4); otherwise acc is stored as a partial
// tile (a split node's parts, or the one part of a node whose GEMM-2 shares
// are cut into R items).
template <typename T, bool COH>
__device__ void do_ytile(const Ctx<T> &cx, const NodeInfo &nd, int a, int bp, double *smem, int64_t *rt) {
  const DevPlan &pl = *cx.pl;
  const int s = uniform(nd.s), c = uniform(nd.c), ld = s + c;
  const int64_t off = nd.off, rp = nd.rp;
  const int64_t goff = nd.goff;
  const int b = bp & 0xffff, part = bp >> 16;
  const int parts = uniform(nd.split), kchunk = uniform(nd.kchunk);
  const int kb = part * kchunk, ke = min(c, kb + kchunk);
  const int i0 = a * 64, j0 = b * 64;
  Acc<T> acc;
  if (uniform(goff >= 0 ? 1 : 0)) {  // X_{C,C} already gathered into the dense buffer
    constexpr int TK = DenseTK<T>::TK;
    const T *G = static_cast<const T *>(cx.Gp) + goff;
    LoadDenseA<T, TK> la{G, nd.ldg, c, ke, i0};
    LoadDenseB<T, TK> lb{cx.Lp, off, ld, s, ke, j0, s};
    gemm_dense<T>(kb, ke, la, lb, smem, acc);
  } else {
    if (threadIdx.x < 64) {
      const int ig = i0 + threadIdx.x;
      rt[threadIdx.x] = gp(pl.kcol)[rp + (ig < c ? ig : 0)];
      rt[64 + threadIdx.x] = gp(pl.kpos)[rp + (ig < c ? ig : 0)];
    }
    lds_barrier();
    LoadGather<T, COH> la{cx.Xp, pl.kcol + rp, pl.kpos + rp, pl.posarr, rt, rt + 64, c, ke, i0};
    la.cs = pl.csign;
    la.du = pl.half;  // LU plans: X_{C,C}'s upper part from the X^T panel set
    LoadPanelK<T, false> lb{cx.Lp, off, ld, s, 0, ke, j0, s};
    gemm_tile<T>(kb, ke, la, lb, smem, acc);
  }
  if (nd.yoff < 0) {
    store_xtile<T, COH>(cx, nd, a, b, acc, smem);
    if (!uniform(nd.defer2)) gemm2_partial<T, COH>(cx, nd, a, b, acc, smem);
    return;
  }
  // partial tile of a node with an R phase: Ypart[part] (column-major c x s)
  T *Y = static_cast<T *>(cx.Yp) + nd.yoff + (int64_t)part * c * s;
  acc_to_lds<T>(acc, smem);
  lds_barrier();
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = e & 63, j = e >> 6;
    if (i0 + i < c && j0 + j < s) Mem<COH>::st(Y + (int64_t)(j0 + j) * c + i0 + i, lds_get<T>(smem, i, j));
  }
  lds_barrier();
}

// Sum of a split node's partial tiles (a, b) into X, then the row tile's share
// of GEMM-2 (the step-3 and step-4 work that an unsplit tile does itself).
// With br = b | r << 16 | rq << 24 and rq > 1, the tile's GEMM-2 share is cut
// into rq items by rows of P_a: item r computes 64-row blocks [r nq / rq,
// (r + 1) nq / rq) of the nq = ceil(s / 64), and item 0 alone stores the tile.
// Every item sums the parts in the same order, so the result is the same.
template <typename T, bool COH, bool PF = true>
__device__ void do_rtile(const Ctx<T> &cx, const NodeInfo &nd, int a, int br, double *smem) {
  const DevPlan &pl = *cx.pl;
  const int s = uniform(nd.s), c = uniform(nd.c);
  const int b = br & 0xffff, r = (br >> 16) & 0xff, rq = max(1, br >> 24);
  const int nq = (s + 63) / 64, qb = uniform(r * nq / rq), qe = uniform((r + 1) * nq / rq);
  const int parts = uniform(nd.split);
  const T *Y = static_cast<const T *>(cx.Yp) + nd.yoff;
  const int i0 = a * 64, j0 = b * 64;
  constexpr int Q = 64 * 64 / NT;
  T sum[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) sum[q] = zero_of<T>();
  // the loads of PB parts are issued together; the sum runs over p in order
  constexpr int PB = 2 / Planes<T>::P;
  for (int p0 = 0; p0 < parts; p0 += PB) {
    T v[PB][Q];
#pragma unroll
    for (int pp = 0; pp < PB; ++pp) {
      const int64_t pbase = (int64_t)min(p0 + pp, parts - 1) * c * s;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int e = threadIdx.x + NT * q;
        const int i = e & 63, j = e >> 6;
        v[pp][q] = Mem<COH>::ld(Y + pbase + (((int64_t)(j0 + j) * c + i0 + i) & opaque_mask(i0 + i < c && j0 + j < s)));
      }
    }
#pragma unroll
    for (int pp = 0; pp < PB; ++pp) {
      const int64_t m = opaque_mask(p0 + pp < parts);
#pragma unroll
      for (int q = 0; q < Q; ++q) sum[q] += masked(v[pp][q], m);
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = threadIdx.x + NT * q;
    const int i = e & 63, j = e >> 6;
    lds_put<T>(smem, i, j, masked(sum[q], opaque_mask(i0 + i < c && j0 + j < s)));
  }
  lds_barrier();
  // into the accumulator layout of the MFMA tile
  constexpr int P = Planes<T>::P;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w & 1, wj = w >> 1;
  Acc<T> acc;
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
          acc.v[p][bi][bj][v] = smem[p * 64 * PITCH + j * PITCH + i];
        }
  lds_barrier();
  if (r == 0) store_xtile<T, COH>(cx, nd, a, b, acc, smem);
  gemm2_partial<T, COH, PF>(cx, nd, a, b, acc, smem, qb, qe);
}

// The GEMM-2 share of a tile whose GEMM-1 item stored Y = X_{C,K} (rows 64a..,
// columns 64b..) without it: the tile is read back from X into the
// accumulator layout (acc = -Y) and gemm2_partial computes 64-row blocks
// [qb, qe) of P_a, with br = b | r << 16 | rq << 24 as for do_rtile.
template <typename T, bool COH, bool PF = true>
__device__ void do_ptile(const Ctx<T> &cx, const NodeInfo &nd, int a, int br, double *smem) {
  const int s = uniform(nd.s), c = uniform(nd.c), ld = s + c;
  const int b = br & 0xffff, r = (br >> 16) & 0xff, rq = max(1, br >> 24);
  const int nq = (s + 63) / 64, qb = uniform(r * nq / rq), qe = uniform((r + 1) * nq / rq);
  const int i0 = a * 64, j0 = b * 64;
  const T *Y = cx.Xp + nd.off + s;
  constexpr int Q = 64 * 64 / NT;
  T v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = threadIdx.x + NT * q;
    const int i = e & 63, j = e >> 6;
    v[q] = Mem<COH>::ld(Y + (((int64_t)(j0 + j) * ld + i0 + i) & opaque_mask(i0 + i < c && j0 + j < s)));
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = threadIdx.x + NT * q;
    const int i = e & 63, j = e >> 6;
    lds_put<T>(smem, i, j, SOps<T>::scale(-1.0, masked(v[q], opaque_mask(i0 + i < c && j0 + j < s))));
  }
  lds_barrier();
  constexpr int P = Planes<T>::P;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w & 1, wj = w >> 1;
  Acc<T> acc;
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
          const int i = 32 * wi + 16 * bi + 4 * vv + (lane >> 4);
          const int j = 32 * wj + 16 * bj + (lane & 15);
          acc.v[p][bi][bj][vv] = smem[p * 64 * PITCH + j * PITCH + i];
        }
  lds_barrier();
  gemm2_partial<T, COH, PF>(cx, nd, a, b, acc, smem, qb, qe);
}

// GEMM-1 tile of a node with a dense X_{C,C} buffer: the level schedule runs
// these in k_ydense (dense loaders only, so fewer registers than the general
// item kernel: two workgroups per CU).  An unsplit tile goes to X and then
// adds its GEMM-2 share from the registers; a 128 x 128 tile leaves that
// share to ITEM_P items, and a split contraction writes partial tiles that
// ITEM_R items sum.
// LU plans: up (an ITEM_YU tile) takes X_{K,C}^T = -(X_{C,C})^T Uhat^T from
// the transposed full buffer and the second panel sets.
template <typename T>
__device__ __forceinline__ void do_ytile_dense(const Ctx<T> &cx, const NodeInfo &nd, int a, int bp, bool up,
                                               double *smem) {
  const int s = uniform(nd.s), c = uniform(nd.c), ld = s + c;
  const int b = bp & 0xffff, part = bp >> 16;
  const int kchunk = uniform(nd.kchunk);
  const int kb = part * kchunk, ke = min(c, kb + kchunk);
  const int i0 = a * 64, j0 = b * 64;
  constexpr int TK = DenseTK<T>::TK;
  const int64_t hs = up ? cx.pl->half : 0;
  const T *G = static_cast<const T *>(cx.Gp) + nd.goff;
  // a lower-only buffer (see the plan) mirrors the stages right of the
  // diagonal block; a full one (LU) reads as is, or transposed for up
  const int kmir = nd.glow ? i0 + 64 : up ? 0 : 1 << 30;
  LoadDenseASym<T, TK> la{G, nd.ldg, c, ke, i0, uniform(kmir)};
  la.cs = cx.pl->csign;
  LoadDenseB<T, TK> lb{cx.Lp + hs, nd.off, ld, s, ke, j0, s};
  Acc<T> acc;
  gemm_dense_il<T, true>(kb, ke, la, lb, smem, acc);  // complex: three real product chains
  acc_to_lds<T>(acc, smem);
  lds_barrier();
  if (nd.yoff < 0) {  // Y = -acc into X_{C,K} (LU up: the second set)
    T *X = cx.Xp + hs + nd.off + s;
    for (int e = threadIdx.x; e < 64 * 64; e += NT) {
      const int i = e & 63, j = e >> 6;
      if (i0 + i < c && j0 + j < s) gstore(X + (int64_t)(j0 + j) * ld + i0 + i, SOps<T>::scale(-1.0, lds_get<T>(smem, i, j)));
    }
    // the row tile's GEMM-2 share (Alg. 1 step 4) from the tile still in
    // registers, unless the plan runs it in ITEM_P items (the LU upper part
    // has none)
    if (!up && !uniform(nd.defer2)) {
      lds_barrier();
      gemm2_partial<T, false, Planes<T>::P == 1>(cx, nd, a, b, acc, smem);
    }
  } else {  // partial tile Ypart[part] (column-major c x s)
    T *Y = static_cast<T *>(cx.Yp) + nd.yoff + (int64_t)part * c * s;
    for (int e = threadIdx.x; e < 64 * 64; e += NT) {
      const int i = e & 63, j = e >> 6;
      if (i0 + i < c && j0 + j < s) gstore(Y + (int64_t)(j0 + j) * c + i0 + i, lds_get<T>(smem, i, j));
    }
  }
}

// Blocks (a, b) and (b, a), a >= b, of sym(Src - sum_r P_r) into Dst, where
// Src and Dst are s x s column-major with leading dimensions sld and dld and
// P_r are the node's row-tile partial products.
template <typename T, bool COH>
__device__ void dtile_core(const Ctx<T> &cx, const NodeInfo &nd, int a, int b, double *smem, const T *Dti, int sld, T *Xkk,
                           int dld) {
  const DevPlan &pl = *cx.pl;
  const int s = nd.s, c = nd.c;
  const int nr = (c + 63) / 64;
  const int64_t pb = nd.poff;
  const int64_t ss = (int64_t)s * s;
  const int a0 = a * 64, b0 = b * 64;
  double *Sab = smem, *Sba = smem + tile_doubles<T>();
  // T[a0 + i, b0 + j] into Sab[i][j] and T[b0 + i, a0 + j] into Sba[i][j].
  // Each thread owns 16 elements of each block, taken in two halves of 8;
  // for every row tile the 16 loads of a half are issued together.
  constexpr int Q = 64 * 64 / NT, QH = Q / 2;
  const int ie = threadIdx.x & 63, jb = threadIdx.x >> 6;  // element (ie, jb + 4 q)
  for (int h = 0; h < 2; ++h) {
    T sab[QH], sba[QH];
    int64_t mab[QH], mba[QH];
#pragma unroll
    for (int q = 0; q < QH; ++q) {
      const int j = jb + 4 * (QH * h + q);
      sab[q] = zero_of<T>();
      sba[q] = zero_of<T>();
      mab[q] = opaque_mask(a0 + ie < s && b0 + j < s);
      mba[q] = opaque_mask(b0 + ie < s && a0 + j < s);
    }
    // two row tiles per round trip: their 32 loads are issued together
    for (int r = 0; r < nr; r += 2) {
      const T *pr0 = cx.Pp + pb + r * ss;
      const T *pr1 = cx.Pp + pb + min(r + 1, nr - 1) * ss;
      const int64_t m1 = opaque_mask(r + 1 < nr);
      T la0[QH], lb0[QH], la1[QH], lb1[QH];
#pragma unroll
      for (int q = 0; q < QH; ++q) {
        const int j = jb + 4 * (QH * h + q);
        la0[q] = Mem<COH>::ld(pr0 + (((int64_t)(b0 + j) * s + a0 + ie) & mab[q]));
        lb0[q] = Mem<COH>::ld(pr0 + (((int64_t)(a0 + j) * s + b0 + ie) & mba[q]));
        la1[q] = Mem<COH>::ld(pr1 + (((int64_t)(b0 + j) * s + a0 + ie) & mab[q]));
        lb1[q] = Mem<COH>::ld(pr1 + (((int64_t)(a0 + j) * s + b0 + ie) & mba[q]));
      }
#pragma unroll
      for (int q = 0; q < QH; ++q) {
        sab[q] += la0[q] + masked(la1[q], m1);
        sba[q] += lb0[q] + masked(lb1[q], m1);
      }
    }
#pragma unroll
    for (int q = 0; q < QH; ++q) {
      const int j = jb + 4 * (QH * h + q);
      const T dab = gload(Dti + (((int64_t)(b0 + j) * sld + a0 + ie) & mab[q]));
      const T dba = gload(Dti + (((int64_t)(a0 + j) * sld + b0 + ie) & mba[q]));
      lds_put<T>(Sab, ie, j, masked(dab - sab[q], mab[q]));
      lds_put<T>(Sba, ie, j, masked(dba - sba[q], mba[q]));
    }
  }
  lds_barrier();
  if (uniform(pl.half > 0 ? 1 : 0)) {
    // LU plan: no symmetrization.  X_KK's blocks (a, b) and (b, a) into the
    // L half, their transposes into the U^T half (entry (r, q) = X(q, r)).
    T *Xu = Xkk + pl.half;
    for (int e = threadIdx.x; e < 64 * 64; e += NT) {
      const int i = e & 63, j = e >> 6;
      if (a0 + i < s && b0 + j < s) {
        Mem<COH>::st(Xkk + (int64_t)(b0 + j) * dld + a0 + i, lds_get<T>(Sab, i, j));
        Mem<COH>::st(Xu + (int64_t)(b0 + j) * dld + a0 + i, lds_get<T>(Sba, j, i));
      }
      if (a != b && b0 + i < s && a0 + j < s) {
        Mem<COH>::st(Xkk + (int64_t)(a0 + j) * dld + b0 + i, lds_get<T>(Sba, i, j));
        Mem<COH>::st(Xu + (int64_t)(a0 + j) * dld + b0 + i, lds_get<T>(Sab, j, i));
      }
    }
    lds_barrier();
    return;
  }
  // x(i, j) = (T[a0+i, b0+j] + T[b0+j, a0+i]) / 2 (the second term conjugated
  // in a Hermitian plan); keep it in Sab
  const double cs = cx.pl->csign;
  T xv[64 * 64 / NT];
#pragma unroll
  for (int q = 0; q < 64 * 64 / NT; ++q) {
    const int e = threadIdx.x + NT * q;
    const int i = e & 63, j = e >> 6;
    xv[q] = SOps<T>::scale(0.5, lds_get<T>(Sab, i, j) + cj(lds_get<T>(Sba, j, i), cs));
  }
  lds_barrier();
#pragma unroll
  for (int q = 0; q < 64 * 64 / NT; ++q) {
    const int e = threadIdx.x + NT * q;
    lds_put<T>(Sab, e & 63, e >> 6, xv[q]);
  }
  lds_barrier();
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = e & 63, j = e >> 6;
    if (a0 + i < s && b0 + j < s) Mem<COH>::st(Xkk + (int64_t)(b0 + j) * dld + a0 + i, lds_get<T>(Sab, i, j));
    if (a != b && b0 + i < s && a0 + j < s)
      Mem<COH>::st(Xkk + (int64_t)(a0 + j) * dld + b0 + i, cj(lds_get<T>(Sab, j, i), cs));
  }
  lds_barrier();
}

// Blocks (a, b) and (b, a), a >= b, of X_KK = sym(Dt^{-1} - sum_r P_r)
// (Alg. 1 step 4 and the symmetrization of Section 2.3).
// The same as dtile_core for the column slab [b0 + kDSlabW sl, b0 +
// kDSlabW (sl + 1)) of block (a, b) only (and the matching row slab of block
// (b, a)), for nodes with many row tiles: with a quarter of the elements per
// thread, the loads of several row tiles' partials are in flight together.
template <typename T, bool COH>
__device__ void dtile_slab(const Ctx<T> &cx, const NodeInfo &nd, int a, int b, int sl, double *smem, const T *Dti, int sld, T *Xkk,
                           int dld) {
  constexpr int W = kDSlabW, QE = 64 * W / NT;
  constexpr int R = Planes<T>::P == 1 ? 4 : 2;  // row tiles per round trip
  const DevPlan &pl = *cx.pl;
  const int s = nd.s, c = nd.c;
  const int nr = uniform((c + 63) / 64);
  const int64_t pb = nd.poff;
  const int64_t ss = (int64_t)s * s;
  const int a0 = a * 64, b0 = b * 64 + sl * W;
  // element q of a thread: (i, j) = (e % 64, e / 64) of the (a, b) slab, and
  // (j', i') = (e % W, e / W) of the (b, a) slab, e = threadIdx.x + NT q
  int64_t oab[QE], oba[QE];
  T sab[QE], sba[QE];
#pragma unroll
  for (int q = 0; q < QE; ++q) {
    const int e = threadIdx.x + NT * q;
    const int ia = e % 64, ja = e / 64, jb = e % W, ib = e / W;
    oab[q] = ((int64_t)(b0 + ja) * s + a0 + ia) & opaque_mask(a0 + ia < s && b0 + ja < s);
    oba[q] = ((int64_t)(a0 + ib) * s + b0 + jb) & opaque_mask(b0 + jb < s && a0 + ib < s);
    sab[q] = zero_of<T>();
    sba[q] = zero_of<T>();
  }
  for (int r = 0; r < nr; r += R) {
    T la[R][QE], lb[R][QE];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const T *pr = cx.Pp + pb + min(r + rr, nr - 1) * ss;
#pragma unroll
      for (int q = 0; q < QE; ++q) {
        la[rr][q] = Mem<COH>::ld(pr + oab[q]);
        lb[rr][q] = Mem<COH>::ld(pr + oba[q]);
      }
    }
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int64_t m = opaque_mask(r + rr < nr);
#pragma unroll
      for (int q = 0; q < QE; ++q) {
        sab[q] += masked(la[rr][q], m);
        sba[q] += masked(lb[rr][q], m);
      }
    }
  }
  T *Sab = reinterpret_cast<T *>(smem);  // [i + 64 j]
  T *Sba = Sab + 64 * W;                  // [j' + W i']
  T *Xs = Sba + 64 * W;                   // [i + 64 j]
#pragma unroll
  for (int q = 0; q < QE; ++q) {
    const int e = threadIdx.x + NT * q;
    const int ia = e % 64, ja = e / 64, jb = e % W, ib = e / W;
    const int64_t mab = opaque_mask(a0 + ia < s && b0 + ja < s), mba = opaque_mask(b0 + jb < s && a0 + ib < s);
    const T dab = gload(Dti + (((int64_t)(b0 + ja) * sld + a0 + ia) & mab));
    const T dba = gload(Dti + (((int64_t)(a0 + ib) * sld + b0 + jb) & mba));
    Sab[e] = masked(dab - sab[q], mab);
    Sba[e] = masked(dba - sba[q], mba);
  }
  lds_barrier();
  // x(i, j) = (T[a0 + i, b0 + j] + T[b0 + j, a0 + i]) / 2 (the second term
  // conjugated in a Hermitian plan)
  const double cs = pl.csign;
#pragma unroll
  for (int q = 0; q < QE; ++q) {
    const int e = threadIdx.x + NT * q;
    const int ia = e % 64, ja = e / 64;
    const T x = SOps<T>::scale(0.5, Sab[e] + cj(Sba[ja + W * ia], cs));
    Xs[e] = x;
    if (a0 + ia < s && b0 + ja < s) Mem<COH>::st(Xkk + (int64_t)(b0 + ja) * dld + a0 + ia, x);
  }
  lds_barrier();
  if (a != b) {
#pragma unroll
    for (int q = 0; q < QE; ++q) {
      const int e = threadIdx.x + NT * q;
      const int jb = e % W, ib = e / W;
      if (b0 + jb < s && a0 + ib < s) Mem<COH>::st(Xkk + (int64_t)(a0 + ib) * dld + b0 + jb, cj(Xs[ib + 64 * jb], cs));
    }
  }
  lds_barrier();
}

template <typename T, bool COH>
__device__ void do_dtile(const Ctx<T> &cx, const NodeInfo &nd, int a, int b, double *smem) {
  const DevPlan &pl = *cx.pl;
  const int ld = nd.s + nd.c;
  const int64_t off = nd.off;
  // top block of the normalized panel = Dt^{-1}; top block of the X panel.
  // b carries the slab number + 1 in its high half for slab items.
  if (b >> 16)
    dtile_slab<T, COH>(cx, nd, a, b & 0xffff, (b >> 16) - 1, smem, cx.Lp + off, ld, cx.Xp + off, ld);
  else
    dtile_core<T, COH>(cx, nd, a, b, smem, cx.Lp + off, ld, cx.Xp + off, ld);
}

// A whole node with c <= 64 and s <= 64 in one workgroup (Alg. 1 steps 3-4
// and the symmetrization of Section 2.3), in three dependent rounds of
// memory reads (and Dt^{-1} at the end): (1) the row tables of C(K) and Lhat; (2) the panel
// positions of X_{C,C} (the column tables of X_{C,C} are the row tables:
// both index C(K)); (3) the values of X_{C,C}.  GEMM-1, GEMM-2 and the
// diagonal block then run from LDS; nothing goes through the partial buffer.
template <typename T, bool COH>
__device__ void do_stile(const Ctx<T> &cx, const NodeInfo &nd, double *smem, int64_t *rt) {
  constexpr int P = Planes<T>::P, TK = Planes<T>::TK;
  constexpr int Q = 64 * 64 / NT;
  const DevPlan &pl = *cx.pl;
  const int s = uniform(nd.s), c = uniform(nd.c), ld = s + c;
  const int64_t off = nd.off, rp = nd.rp;
  // round 1: row tables into LDS; Lhat (c x s) straight into the B planes of
  // the four GEMM-1 stages (B(k, x) = Lhat(k, x): plane [kk][x] of stage k / TK)
  if (threadIdx.x < 64) {
    const int ig = threadIdx.x < c ? threadIdx.x : 0;
    rt[threadIdx.x] = gp(pl.kcol)[rp + ig];
    rt[64 + threadIdx.x] = gp(pl.kpos)[rp + ig];
  }
  {
    T lv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + NT * q;
      const int i = e & 63, j = e >> 6;
      lv[q] = gload(cx.Lp + off + ((((int64_t)j * ld + s + i) & opaque_mask(i < c && j < s))));
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + NT * q;
      const int i = e & 63, j = e >> 6;
      const T l = masked(lv[q], opaque_mask(i < c && j < s));
      double *stgb = smem + (i / TK) * stage_doubles<T>() + P * TK * PITCH + (i % TK) * PITCH + j;
#pragma unroll
      for (int p = 0; p < P; ++p) stgb[p * TK * PITCH] = Planes<T>::get(l, p);
    }
  }
  lds_barrier();
  Acc<T> acc;
  acc_zero<T>(acc);
  if (c > 0) {
    // round 2: positions of X_{C,C}(i, k): lower part (i >= k) through column
    // k's table, upper part through row i's table; element e -> (i = e & 63, k = e >> 6)
    int32_t pos[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + NT * q;
      const int i = e & 63, k = e >> 6;
      const int64_t okm = opaque_mask(i < c && k < c);
      const int64_t lm = opaque_mask(i >= k);
      const int64_t pidx = (((rt[64 + k] + i) & lm) | ((rt[64 + i] + k) & ~lm)) & okm;
      pos[q] = gp(pl.posarr)[pidx];
    }
    // round 3: the values (panel column bases read again from LDS)
    T gv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + NT * q;
      const int i = e & 63, k = e >> 6;
      const int64_t lm = opaque_mask(i >= k);
      const int64_t base = (rt[k] & lm) | (rt[i] & ~lm);
      gv[q] = Mem<COH>::ld(cx.Xp + ((base + (int64_t)pos[q]) & opaque_mask(i < c && k < c)));
    }
    // GEMM-1 from LDS: four stages of TK contraction indices, A = X_{C,C}
    // (upper part conjugated in a Hermitian plan), B = Lhat
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + NT * q;
      const int i = e & 63, k = e >> 6;
      const T g = cj(masked(gv[q], opaque_mask(i < c && k < c)), i < k ? pl.csign : 1.0);
      double *stg = smem + (k / TK) * stage_doubles<T>() + (k % TK) * PITCH + i;
#pragma unroll
      for (int p = 0; p < P; ++p) stg[p * TK * PITCH] = Planes<T>::get(g, p);  // A plane [kk][i]
    }
    lds_barrier();
#pragma unroll
    for (int st = 0; st < 64 / TK; ++st) stage_compute<T>(smem + st * stage_doubles<T>(), acc);
    // Lhat back out of the B planes before store_xtile reuses the stages
    T lv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + NT * q;
      const int i = e & 63, x = e >> 6;
      lv[q] = Planes<T>::from(smem + (i / TK) * stage_doubles<T>() + P * TK * PITCH + (i % TK) * PITCH + x,
                              TK * PITCH);
    }
    lds_barrier();
    // Y = -acc into X_{C,K}
    store_xtile<T, COH>(cx, nd, 0, 0, acc, smem);
    // Lhat (conjugated if Hermitian) into LDS as Ls[p][i * PITCH + x], then R = Lhat^T acc
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + NT * q;
      const int i = e & 63, x = e >> 6;
      const T l = cj(lv[q], pl.csign);
#pragma unroll
      for (int p = 0; p < P; ++p) smem[p * 64 * PITCH + i * PITCH + x] = Planes<T>::get(l, p);
    }
    lds_barrier();
    gemm2_block<T>(acc, smem);  // R[p][j * PITCH + x] = (Lhat^T acc)(x, j) = -(Lhat^T Y)(x, j)
  } else {
#pragma unroll
    for (int e = threadIdx.x; e < 64 * 64; e += NT) lds_put<T>(smem, e >> 6, e & 63, zero_of<T>());
    lds_barrier();
  }
  // T = Dt^{-1} - Lhat^T Y = Dt^{-1} + R; X_KK = (T + T^T) / 2.  Dt^{-1} is
  // read only now: holding it through both products costs registers.
  double *Tt = smem + tile_doubles<T>();
  T dv[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = threadIdx.x + NT * q;
    const int i = e & 63, j = e >> 6;
    dv[q] = gload(cx.Lp + off + ((((int64_t)j * ld + i) & opaque_mask(i < s && j < s))));
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = threadIdx.x + NT * q;
    const int i = e & 63, j = e >> 6;
    const T d = masked(dv[q], opaque_mask(i < s && j < s));
    lds_put<T>(Tt, i, j, d + lds_get<T>(smem, i, j));
  }
  lds_barrier();
  const double cs = pl.csign;
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = e & 63, j = e >> 6;
    if (i < s && j < s)
      Mem<COH>::st(cx.Xp + off + (int64_t)j * ld + i,
                   SOps<T>::scale(0.5, lds_get<T>(Tt, i, j) + cj(lds_get<T>(Tt, j, i), cs)));
  }
  lds_barrier();
}

// A whole small node (c <= CM <= kTinyCF, s <= kTinyS) of one matrix in one
// wavefront, for the level schedule.  Three dependent memory rounds: the
// record, then the byte offsets of X_{C,C} in the panel array (host table:
// c x c row-major, then padding), Lhat and Dt^{-1}, then the X_{C,C} values.
// Lane (i, grp) holds X_{C,C}(i, k) for k = grp + G u; the partial sums of
// X_{C,C} Lhat over the G lane groups are combined with a fixed butterfly, so
// the result does not depend on timing.  LDS blocks are c x s with leading
// dimension tiny_ldc<T>().  HERM: a Hermitian plan (conjugate transposes).
//   Y = -X_{C,C} Lhat (stored into X_{C,K});  T = Dt^{-1} - Lhat^T Y;
//   X_{K,K} = (T + T^T) / 2                      (Alg. 1, Eqs. (2.9)-(2.10))
template <typename T, int CM, bool HERM>
__device__ __forceinline__ void do_tiny(const TinyRec &r, const uint32_t *toff, const T *L, T *X, T *ls, T *ys) {
  constexpr double cs = HERM ? -1.0 : 1.0;
  constexpr int G = 64 / CM, U = CM / G, LDC = tiny_ldc<T>();
  const int lane = threadIdx.x, i = lane % CM, grp = lane / CM;
  const int s = r.s, c = r.c;
  const int64_t ld = s + c;
  const uint32_t *tb = toff + r.tbl;
  // round 2: the offsets of this lane's X_{C,C}(i, k); Lhat as ls[j * LDC + k]; Dt^{-1}(x, y), (y, x)
  const uint32_t rowb = 4u * ((uint32_t)(i * c + grp) & opaque_mask32(i < c));
  uint32_t o[U];
#pragma unroll
  for (int u = 0; u < U; ++u) o[u] = ld_off(tb, rowb + 4u * (G * u));
  constexpr int QL = CM * kTinyS / 64;
  T lv[QL];
#pragma unroll
  for (int q = 0; q < QL; ++q) {
    const int e = lane + 64 * q, k = e % CM, j = e / CM;
    lv[q] = gload(L + r.off + ((j * ld + s + k) & opaque_mask(k < c && j < s)));
  }
  const int x = lane % kTinyS, y = lane / kTinyS;
  const int64_t dm = opaque_mask(x < s && y < s);
  const T dxy = gload(L + r.off + ((y * ld + x) & dm)), dyx = gload(L + r.off + ((x * ld + y) & dm));
  // round 3: the values (bit 0 of an offset: the entry is read conjugated,
  // Hermitian plans only; the bits are kept packed so that the offsets die here)
  T xv[U];
  uint32_t cbits = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if constexpr (HERM) {
      xv[u] = ld_off(X, o[u] & ~1u);
      cbits |= (o[u] & 1u) << u;
    } else {
      xv[u] = ld_off(X, o[u]);
    }
  }
#pragma unroll
  for (int q = 0; q < QL; ++q) {
    const int e = lane + 64 * q, k = e % CM, j = e / CM;
    ls[j * LDC + k] = masked(lv[q], opaque_mask(k < c && j < s));
  }
  __syncthreads();
  T acc[kTinyS];
#pragma unroll
  for (int j = 0; j < kTinyS; ++j) acc[j] = zero_of<T>();
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = grp + G * u;
    T g = masked(xv[u], opaque_mask(i < c && k < c));
    if constexpr (HERM) g = cj(g, ((cbits >> u) & 1u) ? -1.0 : 1.0);
#pragma unroll
    for (int j = 0; j < kTinyS; ++j)
      if (j < s) acc[j] += g * ls[j * LDC + k];
  }
#pragma unroll
  for (int m = CM; m < 64; m <<= 1)
#pragma unroll
    for (int j = 0; j < kTinyS; ++j)
      if (j < s) acc[j] += shfl_xor_t(acc[j], m);
  if (grp == 0 && i < c) {
#pragma unroll
    for (int j = 0; j < kTinyS; ++j)
      if (j < s) {
        X[r.off + j * ld + s + i] = SOps<T>::scale(-1.0, acc[j]);
        ys[j * LDC + i] = acc[j];
      }
  }
  __syncthreads();
  // T = Dt^{-1} + Lhat^T (X_{C,C} Lhat); X_KK = (T + T^T) / 2 (^H and
  // conjugated Lhat in a Hermitian plan)
  if (x < s && y < s) {
    T rxy = zero_of<T>(), ryx = zero_of<T>();
    for (int q = 0; q < c; ++q) {
      rxy += cj(ls[x * LDC + q], cs) * ys[y * LDC + q];
      ryx += cj(ls[y * LDC + q], cs) * ys[x * LDC + q];
    }
    X[r.off + y * ld + x] = SOps<T>::scale(0.5, (dxy + rxy) + cj(dyx + ryx, cs));
  }
}

// The same for 32 < c <= kTinyCF (FP64): lane i holds row i of X_{C,C}, and
// the contraction runs in two halves of 32 columns so that one half's
// offsets and one half's values are in registers at a time; Y(i, j) is
// accumulated in LDS (each lane owns its row), one column j at a time.  Four
// dependent rounds: the record; Lhat, Dt^{-1} and the first half's offsets;
// the first half's values with the second half's offsets; the second half's
// values.  HERM: a Hermitian plan (bit 0 of an offset marks an entry read
// conjugated; the diagonal block takes Lhat^H and the conjugate transpose).
template <typename T, bool HERM = false>
__device__ __forceinline__ void do_tiny64(const TinyRec &r, const uint32_t *toff, const T *L, T *X, T *ls, T *ys) {
  constexpr int H = kTinyCF / 2, LDC = kTinyCF;
  constexpr double cs = HERM ? -1.0 : 1.0;
  const int i = threadIdx.x;
  const int s = r.s, c = r.c;
  const int64_t ld = s + c;
  const uint32_t *tb = toff + r.tbl;
  constexpr int QL = kTinyCF * kTinyS / 64;
  T lv[QL];
#pragma unroll
  for (int q = 0; q < QL; ++q) {
    const int e = i + 64 * q, k = e % kTinyCF, j = e / kTinyCF;
    lv[q] = gload(L + r.off + ((j * ld + s + k) & opaque_mask(k < c && j < s)));
  }
  const int x = i % kTinyS, y = i / kTinyS;
  const int64_t dm = opaque_mask(x < s && y < s);
  const T dxy = gload(L + r.off + ((y * ld + x) & dm)), dyx = gload(L + r.off + ((x * ld + y) & dm));
  const uint32_t rowb = 4u * ((uint32_t)(i * c) & opaque_mask32(i < c));
  uint32_t o[H];
  T xv[H];
#pragma unroll
  for (int u = 0; u < H; ++u) o[u] = ld_off(tb, rowb + 4u * u);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    uint32_t cbits = 0;
#pragma unroll
    for (int u = 0; u < H; ++u) {
      if constexpr (HERM) {
        xv[u] = ld_off(X, o[u] & ~1u);
        cbits |= (o[u] & 1u) << u;
      } else {
        xv[u] = ld_off(X, o[u]);
      }
    }
    if (h == 0) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < H; ++u) o[u] = ld_off(tb, rowb + 4u * (H + u));
#pragma unroll
      for (int q = 0; q < QL; ++q) {
        const int e = i + 64 * q, k = e % kTinyCF, j = e / kTinyCF;
        ls[j * LDC + k] = masked(lv[q], opaque_mask(k < c && j < s));
      }
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < H; ++u) {
      xv[u] = masked(xv[u], opaque_mask(i < c && H * h + u < c));
      if constexpr (HERM) xv[u] = cj(xv[u], ((cbits >> u) & 1u) ? -1.0 : 1.0);
    }
#pragma unroll 1
    for (int j = 0; j < s; ++j) {
      T a = h ? ys[j * LDC + i] : zero_of<T>();
#pragma unroll
      for (int u = 0; u < H; ++u) {
        a += xv[u] * ls[j * LDC + H * h + u];
        if (u % 8 == 7) __builtin_amdgcn_sched_barrier(0);  // bounds the Lhat reads in flight
      }
      ys[j * LDC + i] = a;
    }
  }
  if (i < c)
    for (int j = 0; j < s; ++j) X[r.off + j * ld + s + i] = SOps<T>::scale(-1.0, ys[j * LDC + i]);
  __syncthreads();
  if (x < s && y < s) {
    T rxy = zero_of<T>(), ryx = zero_of<T>();
    for (int q = 0; q < c; ++q) {
      rxy += cj(ls[x * LDC + q], cs) * ys[y * LDC + q];
      ryx += cj(ls[y * LDC + q], cs) * ys[x * LDC + q];
    }
    X[r.off + y * ld + x] = SOps<T>::scale(0.5, (dxy + rxy) + cj(dyx + ryx, cs));
  }
}

// LU plans (gathered X_{C,C}, unsplit nodes): the GEMM-1 tile of the upper
// part, rows 64a.. and columns 64b.. of X_{K,C}^T = -(X_{C,C})^T Uhat^T, where
// Uhat^T is the normalized U^T panel set and (X_{C,C})^T is gathered with the
// two X panel sets exchanged; stored into the U half of X.  The upper part
// takes no GEMM-2 share (A^{-1}_{K,K} needs only X_{C,K}).
template <typename T, bool COH>
__device__ void do_yutile(const Ctx<T> &cx, const NodeInfo &nd, int a, int b, double *smem, int64_t *rt) {
  const DevPlan &pl = *cx.pl;
  const int s = uniform(nd.s), c = uniform(nd.c), ld = s + c;
  const int64_t off = nd.off, rp = nd.rp;
  const int i0 = a * 64, j0 = b * 64;
  if (threadIdx.x < 64) {
    const int ig = i0 + threadIdx.x;
    rt[threadIdx.x] = gp(pl.kcol)[rp + (ig < c ? ig : 0)];
    rt[64 + threadIdx.x] = gp(pl.kpos)[rp + (ig < c ? ig : 0)];
  }
  lds_barrier();
  Ctx<T> cu = cx;
  cu.Xp = cx.Xp + pl.half;
  LoadGather<T, COH> la{cu.Xp, pl.kcol + rp, pl.kpos + rp, pl.posarr, rt, rt + 64, c, c, i0};
  la.du = -pl.half;
  LoadPanelK<T, false> lb{cx.Lp + pl.half, off, ld, s, 0, c, j0, s};
  Acc<T> acc;
  gemm_tile<T>(0, c, la, lb, smem, acc);
  store_xtile<T, COH>(cu, nd, a, b, acc, smem);
}

// Inlined into the kernels, so that the node record stays in scalar registers
// (a call would pass it through the stack).
template <typename T, bool COH>
__device__ __forceinline__ void do_item(const Ctx<T> &cx, const Item &item, const NodeInfo &nd, double *smem,
                                        int64_t *rt) {
  const Item it = uniform(item);
  if (it.type == ITEM_G) {
    do_gtile<T>(cx, nd, it.a, it.b, smem, rt, cx.Xp);
  } else if (it.type == ITEM_Y) {
    do_ytile<T, COH>(cx, nd, it.a, it.b, smem, rt);
  } else if (it.type == ITEM_YU) {
    do_yutile<T, COH>(cx, nd, it.a, it.b, smem, rt);
  } else if (it.type == ITEM_R) {
    do_rtile<T, COH>(cx, nd, it.a, it.b, smem);
  } else if (it.type == ITEM_P) {
    do_ptile<T, COH>(cx, nd, it.a, it.b, smem);
  } else if (it.type == ITEM_D) {
    do_dtile<T, COH>(cx, nd, it.a, it.b, smem);
  } else {  // ITEM_S: the whole node (c <= 64, s <= 64) in this workgroup
    do_stile<T, COH>(cx, nd, smem, rt);
  }
}

}  // namespace selinv
