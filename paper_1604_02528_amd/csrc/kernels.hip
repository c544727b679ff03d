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

// Block (a, b), a >= b, of X_{C,C} for a node with a dense buffer G (column
// major, leading dimension ldg): element (i, k), i >= k, is the lower-part
// entry X[kcol[k] + posarr[kpos[k] + i]] of the ancestor owning column k; it
// is written to G(i, k) and G(k, i).  Lanes run along i (one column k per
// wave and step) for the gather and the G(i, k) stores; the mirror stores go
// through an LDS transpose so that they are contiguous too.
template <typename T>
__device__ void do_gtile(const Ctx<T> &cx, int K, int a, int b, double *smem) {
  const DevPlan &pl = *cx.pl;
  const int c = uniform(gp(pl.node_c)[K]);
  const int64_t rp = gp(pl.node_rowptr)[K];
  const int ldg = gp(pl.node_ldg)[K];
  T *G = cx.Gp + gp(pl.node_goff)[K];
  const int i0 = a * 64, k0 = b * 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int Q = 64 * 64 / NT, QH = Q / 2;
  for (int h = 0; h < 2; ++h) {
    int64_t pidx[QH], base[QH], msk[QH];
#pragma unroll
    for (int q = 0; q < QH; ++q) {
      const int kl = w + 4 * (QH * h + q), i = i0 + lane, k = k0 + kl;
      msk[q] = opaque_mask(i < c && k < c && i >= k);
      const int64_t kq = (int64_t)(k < c ? k : 0);
      base[q] = gp(pl.kcol)[rp + kq];
      pidx[q] = (gp(pl.kpos)[rp + kq] + i) & msk[q];
    }
    int64_t addr[QH];
#pragma unroll
    for (int q = 0; q < QH; ++q) addr[q] = (base[q] + (int64_t)gp(pl.posarr)[pidx[q]]) & msk[q];
    T v[QH];
#pragma unroll
    for (int q = 0; q < QH; ++q) v[q] = masked(Mem<false>::ld(cx.Xp + addr[q]), msk[q]);
#pragma unroll
    for (int q = 0; q < QH; ++q) {
      const int kl = w + 4 * (QH * h + q), i = i0 + lane, k = k0 + kl;
      lds_put<T>(smem, lane, kl, v[q]);  // tile[i][k] at smem[k * PITCH + i]
      if (i < c && k < c && i >= k) Mem<false>::st(G + (int64_t)k * ldg + i, v[q]);
    }
  }
  lds_barrier();
  // mirror: G(k, i) = tile[i][k], lanes along k
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = threadIdx.x + NT * q;
    const int kl = e & 63, il = e >> 6, i = i0 + il, k = k0 + kl;
    if (i < c && k < c && i > k) Mem<false>::st(G + (int64_t)i * ldg + k, lds_get<T>(smem, il, kl));
  }
  lds_barrier();
}

// Store -acc (a 64 x 64 tile of X_{C,K} = -X_{C,C} Lhat) into X, rows 64a..
// of C(K) and columns 64b.. of K, through LDS so that the stores coalesce.
template <typename T, bool COH>
__device__ void store_xtile(const Ctx<T> &cx, int K, int a, int b, const Acc<T> &acc, double *smem) {
  const DevPlan &pl = *cx.pl;
  const int s = gp(pl.node_s)[K], c = gp(pl.node_c)[K], ld = s + c;
  const int64_t off = gp(pl.node_off)[K];
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

// Row tile a's share of GEMM-2 (Alg. 1 step 4): P_a[:, 64b..] = Lhat[rows of
// tile a, :]^T Y[tile a, 64b..] = -(Lhat_a^T acc), written to the partial
// buffer (column-major s x s per row tile).  The accumulators already sit in
// the MFMA B-operand layout for a contraction over the tile rows (register v
// of a 16 x 16 block holds rows 4v..4v+3 of lanes l / 16).
template <typename T, bool COH>
__device__ void gemm2_partial(const Ctx<T> &cx, int K, int a, int b, const Acc<T> &acc, double *smem) {
  constexpr int P = Planes<T>::P;
  const DevPlan &pl = *cx.pl;
  const int s = gp(pl.node_s)[K], c = gp(pl.node_c)[K], ld = s + c;
  const int64_t off = gp(pl.node_off)[K];
  const int i0 = a * 64, j0 = b * 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w & 1, wj = w >> 1;
  const int64_t pbase = gp(pl.node_poff)[K] + (int64_t)a * s * s;
  double *Ls = smem;  // Lhat[i0 .. i0+63, q0 .. q0+63] as Ls[p][i * PITCH + x]
  for (int q0 = 0; q0 < s; q0 += 64) {
    T lv[64 * 64 / NT];
#pragma unroll
    for (int q = 0; q < 64 * 64 / NT; ++q) {
      const int e = threadIdx.x + NT * q;
      const int i = e & 63, x = e >> 6;
      lv[q] = gload(cx.Lp + off + (((int64_t)(q0 + x) * ld + s + i0 + i) & opaque_mask(i0 + i < c && q0 + x < s)));
    }
#pragma unroll
    for (int q = 0; q < 64 * 64 / NT; ++q) {
      const int e = threadIdx.x + NT * q;
      const int i = e & 63, x = e >> 6;
      const T v = masked(lv[q], opaque_mask(i0 + i < c && q0 + x < s));
#pragma unroll
      for (int p = 0; p < P; ++p) Ls[p * 64 * PITCH + i * PITCH + x] = Planes<T>::get(v, p);
    }
    lds_barrier();
    d4 pacc[P][4][2];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int xb = 0; xb < 4; ++xb)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) pacc[p][xb][bj] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4) {
        const int row = 32 * wi + 16 * bi + 4 * k4 + (lane >> 4);
#pragma unroll
        for (int xb = 0; xb < 4; ++xb) {
          double af[P];
#pragma unroll
          for (int p = 0; p < P; ++p) af[p] = Ls[p * 64 * PITCH + row * PITCH + 16 * xb + (lane & 15)];
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) {
            if constexpr (P == 1) {
              pacc[0][xb][bj] = mfma16(af[0], acc.v[0][bi][bj][k4], pacc[0][xb][bj]);
            } else {
              pacc[0][xb][bj] = mfma16(af[0], acc.v[0][bi][bj][k4], pacc[0][xb][bj]);
              pacc[0][xb][bj] = mfma16(-af[1], acc.v[1][bi][bj][k4], pacc[0][xb][bj]);
              pacc[1][xb][bj] = mfma16(af[0], acc.v[1][bi][bj][k4], pacc[1][xb][bj]);
              pacc[1][xb][bj] = mfma16(af[1], acc.v[0][bi][bj][k4], pacc[1][xb][bj]);
            }
          }
        }
      }
    lds_barrier();
    // sum the two row halves (wi = 0, 1) in LDS: R[p][j * PITCH + x]
    double *R = smem;
    for (int half = 0; half < 2; ++half) {
      if (wi == half) {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
          for (int xb = 0; xb < 4; ++xb)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int x = 16 * xb + 4 * v + (lane >> 4);
                const int j = 32 * wj + 16 * bj + (lane & 15);
                double &r = R[p * 64 * PITCH + j * PITCH + x];
                r = half == 0 ? pacc[p][xb][bj][v] : r + pacc[p][xb][bj][v];
              }
      }
      lds_barrier();
    }
    // P = Lhat^T Y = -(Lhat^T acc)
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
// share of [0, c).  An unsplit node stores Y = -acc into X and its row tile's
// share of GEMM-2 (step 4); a split node stores acc as a partial tile.
template <typename T, bool COH>
__device__ void do_ytile(const Ctx<T> &cx, int K, int a, int bp, double *smem, int64_t *rt) {
  const DevPlan &pl = *cx.pl;
  const int s = uniform(gp(pl.node_s)[K]), c = uniform(gp(pl.node_c)[K]), ld = s + c;
  const int64_t off = gp(pl.node_off)[K], rp = gp(pl.node_rowptr)[K];
  const int64_t goff = gp(pl.node_goff)[K];
  const int b = bp & 0xffff, part = bp >> 16;
  const int parts = uniform(gp(pl.node_split)[K]), kchunk = uniform(gp(pl.node_kchunk)[K]);
  const int kb = part * kchunk, ke = min(c, kb + kchunk);
  const int i0 = a * 64, j0 = b * 64;
  Acc<T> acc;
  if (uniform(goff >= 0 ? 1 : 0)) {  // X_{C,C} already gathered into the dense buffer
    constexpr int TK = DenseTK<T>::TK;
    const T *G = static_cast<const T *>(cx.Gp) + goff;
    LoadDenseA<T, TK> la{G, gp(pl.node_ldg)[K], c, ke, i0};
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
    LoadPanelK<T, false> lb{cx.Lp, off, ld, s, 0, ke, j0, s};
    gemm_tile<T>(kb, ke, la, lb, smem, acc);
  }
  if (parts == 1) {
    store_xtile<T, COH>(cx, K, a, b, acc, smem);
    gemm2_partial<T, COH>(cx, K, a, b, acc, smem);
    return;
  }
  // partial tile of a split node: Ypart[part] (column-major c x s)
  T *Y = static_cast<T *>(cx.Yp) + gp(pl.node_yoff)[K] + (int64_t)part * c * s;
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
template <typename T, bool COH>
__device__ void do_rtile(const Ctx<T> &cx, int K, int a, int b, double *smem) {
  const DevPlan &pl = *cx.pl;
  const int s = uniform(gp(pl.node_s)[K]), c = uniform(gp(pl.node_c)[K]);
  const int parts = uniform(gp(pl.node_split)[K]);
  const T *Y = static_cast<const T *>(cx.Yp) + gp(pl.node_yoff)[K];
  const int i0 = a * 64, j0 = b * 64;
  constexpr int Q = 64 * 64 / NT;
  T sum[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) sum[q] = zero_of<T>();
  for (int p = 0; p < parts; ++p) {
    T v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = threadIdx.x + NT * q;
      const int i = e & 63, j = e >> 6;
      v[q] = Mem<COH>::ld(Y + (int64_t)p * c * s + (((int64_t)(j0 + j) * c + i0 + i) & opaque_mask(i0 + i < c && j0 + j < s)));
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) sum[q] += v[q];
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
  store_xtile<T, COH>(cx, K, a, b, acc, smem);
  gemm2_partial<T, COH>(cx, K, a, b, acc, smem);
}

// Blocks (a, b) and (b, a), a >= b, of X_KK = sym(Dt^{-1} - sum_r P_r)
// (Alg. 1 step 4 and the symmetrization of Section 2.3).
template <typename T, bool COH>
__device__ void do_dtile(const Ctx<T> &cx, int K, int a, int b, double *smem) {
  const DevPlan &pl = *cx.pl;
  const int s = gp(pl.node_s)[K], c = gp(pl.node_c)[K], ld = s + c;
  const int64_t off = gp(pl.node_off)[K];
  const int nr = (c + 63) / 64;
  const int64_t pb = gp(pl.node_poff)[K];
  const int64_t ss = (int64_t)s * s;
  const T *Dti = cx.Lp + off;  // top block of the normalized panel = Dt^{-1}
  T *Xkk = cx.Xp + off;        // top block of the X panel
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
    for (int r = 0; r < nr; ++r) {
      const T *pr = cx.Pp + pb + r * ss;
      T la[QH], lb[QH];
#pragma unroll
      for (int q = 0; q < QH; ++q) {
        const int j = jb + 4 * (QH * h + q);
        la[q] = Mem<COH>::ld(pr + (((int64_t)(b0 + j) * s + a0 + ie) & mab[q]));
        lb[q] = Mem<COH>::ld(pr + (((int64_t)(a0 + j) * s + b0 + ie) & mba[q]));
      }
#pragma unroll
      for (int q = 0; q < QH; ++q) {
        sab[q] += la[q];
        sba[q] += lb[q];
      }
    }
#pragma unroll
    for (int q = 0; q < QH; ++q) {
      const int j = jb + 4 * (QH * h + q);
      const T dab = gload(Dti + (((int64_t)(b0 + j) * ld + a0 + ie) & mab[q]));
      const T dba = gload(Dti + (((int64_t)(a0 + j) * ld + b0 + ie) & mba[q]));
      lds_put<T>(Sab, ie, j, masked(dab - sab[q], mab[q]));
      lds_put<T>(Sba, ie, j, masked(dba - sba[q], mba[q]));
    }
  }
  lds_barrier();
  // x(i, j) = (T[a0+i, b0+j] + T[b0+j, a0+i]) / 2 ; keep it in Sab
  T xv[64 * 64 / NT];
#pragma unroll
  for (int q = 0; q < 64 * 64 / NT; ++q) {
    const int e = threadIdx.x + NT * q;
    const int i = e & 63, j = e >> 6;
    xv[q] = SOps<T>::scale(0.5, lds_get<T>(Sab, i, j) + lds_get<T>(Sba, j, i));
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
    if (a0 + i < s && b0 + j < s) Mem<COH>::st(Xkk + (int64_t)(b0 + j) * ld + a0 + i, lds_get<T>(Sab, i, j));
    if (a != b && b0 + i < s && a0 + j < s) Mem<COH>::st(Xkk + (int64_t)(a0 + j) * ld + b0 + i, lds_get<T>(Sab, j, i));
  }
  lds_barrier();
}

template <typename T, bool COH>
__device__ void do_item(const Ctx<T> &cx, const Item &item, double *smem, int64_t *rt) {
  const Item it = uniform(item);
  if (it.type == ITEM_G) {
    do_gtile<T>(cx, it.K, it.a, it.b, smem);
  } else if (it.type == ITEM_Y) {
    do_ytile<T, COH>(cx, it.K, it.a, it.b, smem, rt);
  } else if (it.type == ITEM_R) {
    do_rtile<T, COH>(cx, it.K, it.a, it.b, smem);
  } else if (it.type == ITEM_D) {
    do_dtile<T, COH>(cx, it.K, it.a, it.b, smem);
  } else {  // ITEM_S: the whole node (c <= 64, s <= 64) in this workgroup
    if (uniform(gp(cx.pl->node_c)[it.K]) > 0) {
      do_ytile<T, COH>(cx, it.K, 0, 0, smem, rt);
      __threadfence_block();
      __syncthreads();
    }
    do_dtile<T, COH>(cx, it.K, 0, 0, smem);
  }
}

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
      if (e > b)
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

}  // namespace selinv
