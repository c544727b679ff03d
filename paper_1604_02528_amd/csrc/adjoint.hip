// Adjoint of the selected inversion (reverse mode), FP64 and complex128 on
// gfx950.  For a complex-symmetric A the same formulas hold with plain
// transposes: they give the holomorphic derivative dloss/da of a loss that is
// a holomorphic function of the selected entries.
//
// Not in the paper.  A loss depends on the stored lower selected entries
// x_pq = (A^{-1})_pq on the pattern F of L; the caller passes W_pq =
// dloss/dx_pq in the panel layout (stored-value convention: an off-diagonal
// value stands for (p, q) and (q, p)).  The gradient with respect to the
// stored values of A is G_ij (i = j) or 2 G_ij (i != j), G = -X W_s X,
// W_s = (W + W^T)/2.  It is computed node by node by reversing the forward
// traversal (Alg. 1 with the LDL^T normalization of Section 2.3) and the
// block LDL^T factorization, re-reading X instead of storing per-node
// intermediates.  In stored-value units (E = Dt^{-1}, Lhat, X_{C,K} = Y):
//
//  R1, leaves -> root (a node starts once every descendant has pushed into W):
//    Tbar = sym(W_KK) (diagonal kept, off-diagonal halved and mirrored)
//    Zbar = W_{C,K} - Lhat Tbar
//    Lhatbar = -(X_{C,C} Zbar + Y Tbar)
//    W[ancestors] += -(Zbar Lhat^T + Lhat Zbar^T) on the lower part of C(K) x C(K)
//                    (halved on the diagonal), through the ancestor index maps
//  R2: Dtbar0 = -E Tbar E
//  R3, root -> leaves, Sbar the adjoint of the trailing Schur complements:
//    M = Sbar_{C,C} Lhat,  Lb = Lhatbar - 2 M Dt,  N = Lb E
//    Sbar_{C,K} = N / 2,  Sbar_KK = sym(Dtbar0 - Lhat^T (M + N))
//  Output: Abar = Sbar on A's pattern, doubled off the diagonal.
//
// Every step is a 64 x 64 tile on the MFMA machinery of the forward sweep;
// the scatter-add uses hardware FP64 atomics (one per real plane; summation
// order, and hence the last bits, may differ between runs).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "items.hpp"
#include "plan.hpp"
#include "tile.hpp"

namespace selinv {
namespace {

template <typename T> struct BCtx {
  Ctx<T> cx;        // Lp normalized panels, Xp the forward X, Pp partials, Gp dense buffers
  T *W;             // stored-value gradient on F, accumulated in place
  T *Z, *L, *S;     // panel-layout scratch: Zbar then M; Lhatbar then Lb; Sbar
  T *TB, *FB, *DB;  // s x s scratch: Tbar; F = Tbar E; Dtbar0
  const T *DT;      // Dt = L_KK D_K L_KK^T
};

__device__ __forceinline__ void atomic_add_t(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_t(cplx *p, cplx v) {
  double *q = reinterpret_cast<double *>(p);
  unsafeAtomicAdd(q, v.re);
  unsafeAtomicAdd(q + 1, v.im);
}

struct Geo {
  int s, c, ld;
  int64_t off, sq, rp, goff;
  int ldg;
};

__device__ __forceinline__ Geo geo(const DevPlan &pl, int K) {
  Geo g;
  g.s = uniform(gp(pl.node_s)[K]);
  g.c = uniform(gp(pl.node_c)[K]);
  g.ld = g.s + g.c;
  g.off = gp(pl.node_off)[K];
  g.sq = gp(pl.node_sq)[K];
  g.rp = gp(pl.node_rowptr)[K];
  g.goff = gp(pl.node_goff)[K];
  g.ldg = gp(pl.node_ldg)[K];
  return g;
}

// dst[(j0 + j) * ld + i0 + i] = f(i0 + i, j0 + j, acc(i, j)) for i0 + i < rows,
// j0 + j < cols, through LDS so that the stores coalesce.
template <typename T, class F>
__device__ void store_tile(const Acc<T> &acc, double *smem, T *dst, int64_t ld, int i0, int j0, int rows, int cols,
                           F f) {
  acc_to_lds<T>(acc, smem);
  lds_barrier();
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = e & 63, j = e >> 6;
    if (i0 + i < rows && j0 + j < cols) {
      const int64_t q = (int64_t)(j0 + j) * ld + i0 + i;
      dst[q] = f(q, lds_get<T>(smem, i, j));
    }
  }
  lds_barrier();
}

template <typename T> using DA = LoadDenseA<T, DenseTK<T>::TK>;
template <typename T> using DB = LoadDenseB<T, DenseTK<T>::TK>;
template <typename T> using DBT = LoadDenseBT<T, DenseTK<T>::TK>;

// acc = X_{C,C}[tile rows, :] B[:, tile cols] with X_{C,C} gathered from Src (panel
// layout) or read from the node's dense buffer; B = the c x s bottom block of a
// panel-layout array Bp.
template <typename T>
__device__ void gemm_cc(const BCtx<T> &bx, const Geo &g, const T *Src, const T *Bp, int i0, int j0, double *smem,
                        int64_t *rt, Acc<T> &acc) {
  const DevPlan &pl = *bx.cx.pl;
  if (uniform(g.goff >= 0 ? 1 : 0)) {
    DA<T> la{bx.cx.Gp + g.goff, g.ldg, g.c, g.c, i0};
    DB<T> lb{Bp, g.off, g.ld, g.s, g.c, j0, g.s};
    gemm_dense<T>(0, g.c, la, lb, smem, acc);
  } else {
    if (threadIdx.x < 64) {
      const int ig = i0 + threadIdx.x;
      rt[threadIdx.x] = gp(pl.kcol)[g.rp + (ig < g.c ? ig : 0)];
      rt[64 + threadIdx.x] = gp(pl.kpos)[g.rp + (ig < g.c ? ig : 0)];
    }
    lds_barrier();
    LoadGather<T, false> la{Src, pl.kcol + g.rp, pl.kpos + g.rp, pl.posarr, rt, rt + 64, g.c, g.c, i0};
    LoadPanelK<T, false> lb{Bp, g.off, g.ld, g.s, 0, g.c, j0, g.s};
    gemm_tile<T>(0, g.c, la, lb, smem, acc);
  }
}

template <typename T>
__device__ void bi_t(const BCtx<T> &bx, const Geo &g, int a, int b) {
  const int i0 = a * 64, j0 = b * 64;
  const T *Wk = bx.W + g.off;
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = i0 + (e & 63), j = j0 + (e >> 6);
    if (i < g.s && j < g.s) {
      const T w = i >= j ? Wk[(int64_t)j * g.ld + i] : Wk[(int64_t)i * g.ld + j];
      bx.TB[g.sq + (int64_t)j * g.s + i] = i == j ? w : SOps<T>::scale(0.5, w);
    }
  }
}

template <typename T>
__device__ void bi_z(const BCtx<T> &bx, const Geo &g, int a, int b, double *smem) {
  const int i0 = a * 64, j0 = b * 64;
  Acc<T> acc;
  gemm_dense<T>(0, g.s, DA<T>{bx.cx.Lp + g.off + g.s, g.ld, g.c, g.s, i0},
                DB<T>{bx.TB + g.sq, 0, g.s, 0, g.s, j0, g.s}, smem, acc);
  const T *Wb = bx.W + g.off + g.s;
  store_tile<T>(acc, smem, bx.Z + g.off + g.s, g.ld, i0, j0, g.c, g.s, [&](int64_t q, T v) { return Wb[q] - v; });
}

template <typename T>
__device__ void bi_l(const BCtx<T> &bx, const Geo &g, int a, int b, double *smem, int64_t *rt) {
  const int i0 = a * 64, j0 = b * 64;
  Acc<T> acc;
  gemm_cc<T>(bx, g, bx.cx.Xp, bx.Z, i0, j0, smem, rt, acc);  // X_{C,C} Zbar
  gemm_dense<T>(0, g.s, DA<T>{bx.cx.Xp + g.off + g.s, g.ld, g.c, g.s, i0},
                DB<T>{bx.TB + g.sq, 0, g.s, 0, g.s, j0, g.s}, smem, acc, true);  // + Y Tbar
  store_tile<T>(acc, smem, bx.L + g.off + g.s, g.ld, i0, j0, g.c, g.s,
                [](int64_t, T v) { return SOps<T>::scale(-1.0, v); });
}

// Rows 64a.., columns 64a2.. (a >= a2) of Zbar Lhat^T + Lhat Zbar^T, subtracted
// from the stored-value gradient of the ancestors' entries of X_{C,C}.
template <typename T>
__device__ void bi_sc(const BCtx<T> &bx, const Geo &g, int a, int a2, double *smem) {
  const DevPlan &pl = *bx.cx.pl;
  const int i0 = a * 64, k0 = a2 * 64;
  const T *Zb = bx.Z + g.off + g.s, *Lh = bx.cx.Lp + g.off + g.s;
  Acc<T> acc;
  gemm_dense<T>(0, g.s, DA<T>{Zb, g.ld, g.c, g.s, i0}, DBT<T>{Lh, g.ld, g.s, k0, g.c}, smem, acc);
  gemm_dense<T>(0, g.s, DA<T>{Lh, g.ld, g.c, g.s, i0}, DBT<T>{Zb, g.ld, g.s, k0, g.c}, smem, acc, true);
  acc_to_lds<T>(acc, smem);
  lds_barrier();
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = e & 63, k = e >> 6;
    const int ig = i0 + i, kg = k0 + k;
    if (ig < g.c && kg < g.c && ig >= kg) {
      const T v = lds_get<T>(smem, i, k);
      const int64_t addr = gp(pl.kcol)[g.rp + kg] + gp(pl.posarr)[gp(pl.kpos)[g.rp + kg] + ig];
      atomic_add_t(bx.W + addr, SOps<T>::scale(ig == kg ? -0.5 : -1.0, v));
    }
  }
  lds_barrier();
}

template <typename T>
__device__ void bi_f(const BCtx<T> &bx, const Geo &g, int a, int b, double *smem) {
  const int i0 = a * 64, j0 = b * 64;
  Acc<T> acc;
  gemm_dense<T>(0, g.s, DA<T>{bx.TB + g.sq, g.s, g.s, g.s, i0}, DB<T>{bx.cx.Lp, g.off, g.ld, 0, g.s, j0, g.s}, smem,
                acc);
  store_tile<T>(acc, smem, bx.FB + g.sq, g.s, i0, j0, g.s, g.s, [](int64_t, T v) { return v; });
}

template <typename T>
__device__ void bi_d0(const BCtx<T> &bx, const Geo &g, int a, int b, double *smem) {
  const int i0 = a * 64, j0 = b * 64;
  Acc<T> acc;
  gemm_dense<T>(0, g.s, DA<T>{bx.cx.Lp + g.off, g.ld, g.s, g.s, i0}, DB<T>{bx.FB + g.sq, 0, g.s, 0, g.s, j0, g.s},
                smem, acc);
  store_tile<T>(acc, smem, bx.DB + g.sq, g.s, i0, j0, g.s, g.s, [](int64_t, T v) { return SOps<T>::scale(-1.0, v); });
}

template <typename T>
__device__ void bi_m(const BCtx<T> &bx, const Geo &g, int a, int b, double *smem, int64_t *rt) {
  const int i0 = a * 64, j0 = b * 64;
  Acc<T> acc;
  gemm_cc<T>(bx, g, bx.S, bx.cx.Lp, i0, j0, smem, rt, acc);  // Sbar_{C,C} Lhat
  store_tile<T>(acc, smem, bx.Z + g.off + g.s, g.ld, i0, j0, g.c, g.s, [](int64_t, T v) { return v; });
}

template <typename T>
__device__ void bi_lb(const BCtx<T> &bx, const Geo &g, int a, int b, double *smem) {
  const int i0 = a * 64, j0 = b * 64;
  Acc<T> acc;
  gemm_dense<T>(0, g.s, DA<T>{bx.Z + g.off + g.s, g.ld, g.c, g.s, i0}, DB<T>{bx.DT + g.sq, 0, g.s, 0, g.s, j0, g.s},
                smem, acc);
  T *Lb = bx.L + g.off + g.s;
  store_tile<T>(acc, smem, Lb, g.ld, i0, j0, g.c, g.s,
                [&](int64_t q, T v) { return Lb[q] - SOps<T>::scale(2.0, v); });
}

template <typename T>
__device__ void bi_n(const BCtx<T> &bx, const Geo &g, int K, int a, int b, double *smem) {
  constexpr int P = Planes<T>::P;
  const int i0 = a * 64, j0 = b * 64;
  Acc<T> acc;
  gemm_dense<T>(0, g.s, DA<T>{bx.L + g.off + g.s, g.ld, g.c, g.s, i0}, DB<T>{bx.cx.Lp, g.off, g.ld, 0, g.s, j0, g.s},
                smem, acc);  // N = Lb E
  store_tile<T>(acc, smem, bx.S + g.off + g.s, g.ld, i0, j0, g.c, g.s,
                [](int64_t, T v) { return SOps<T>::scale(0.5, v); });
  // acc <- -(M + N) in the accumulator layout, then the row tile's share of
  // Lhat^T (M + N) into the partial products
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w & 1, wj = w >> 1;
  const T *M = bx.Z + g.off + g.s;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 32 * wi + 16 * bi + 4 * v + (lane >> 4);
        const int j = j0 + 32 * wj + 16 * bj + (lane & 15);
        const int64_t m = opaque_mask(i < g.c && j < g.s);
        const T mv = masked(M[((int64_t)j * g.ld + i) & m], m);
#pragma unroll
        for (int p = 0; p < P; ++p)
          acc.v[p][bi][bj][v] = -(Planes<T>::get(mv, p) + masked(acc.v[p][bi][bj][v], m));
      }
  gemm2_partial<T, false>(bx.cx, node_info(*bx.cx.pl, K), a, b, acc, smem);
}

template <typename T>
__global__ void __launch_bounds__(NT, Planes<T>::P == 1 ? 2 : 1)
    k_back_items(const DevPlan *__restrict__ plp, const T *panels, const T *x, const T *dt, T *xbar, int32_t first,
                 int32_t count) {
  const DevPlan &pl = *plp;
  __shared__ double smem[smem_doubles<T>()];
  __shared__ int64_t rt[128];
  const int64_t g0 = blockIdx.x;
  const int64_t l = g0 / count;
  const Item it = uniform(gload(pl.bitems + first + (g0 - l * count)));
  const int64_t pe = pl.panel_elems, sq = pl.sq_elems;
  BCtx<T> bx;
  bx.cx = Ctx<T>{&pl, panels + l * pe, const_cast<T *>(x) + l * pe, static_cast<T *>(pl.part) + l * pl.part_elems,
                 static_cast<T *>(pl.gbuf) + l * pl.g_elems, nullptr};
  bx.W = xbar + l * pe;
  bx.Z = static_cast<T *>(pl.adj_z) + l * pe;
  bx.L = static_cast<T *>(pl.adj_l) + l * pe;
  bx.S = static_cast<T *>(pl.adj_s) + l * pe;
  bx.TB = static_cast<T *>(pl.adj_t) + l * sq;
  bx.FB = static_cast<T *>(pl.adj_f) + l * sq;
  bx.DB = static_cast<T *>(pl.adj_d) + l * sq;
  bx.DT = dt + l * sq;
  const Geo g = geo(pl, it.K);
  switch (it.type) {
    case BI_T: bi_t<T>(bx, g, it.a, it.b); break;
    case BI_G: do_gtile<T>(bx.cx, node_info(pl, it.K), it.a, it.b, smem, rt, bx.cx.Xp); break;
    case BI_Z: bi_z<T>(bx, g, it.a, it.b, smem); break;
    case BI_L: bi_l<T>(bx, g, it.a, it.b, smem, rt); break;
    case BI_SC: bi_sc<T>(bx, g, it.a, it.b, smem); break;
    case BI_F: bi_f<T>(bx, g, it.a, it.b, smem); break;
    case BI_D0: bi_d0<T>(bx, g, it.a, it.b, smem); break;
    case BI_SG: do_gtile<T>(bx.cx, node_info(pl, it.K), it.a, it.b, smem, rt, bx.S); break;
    case BI_M: bi_m<T>(bx, g, it.a, it.b, smem, rt); break;
    case BI_LB: bi_lb<T>(bx, g, it.a, it.b, smem); break;
    case BI_N: bi_n<T>(bx, g, it.K, it.a, it.b, smem); break;
    case BI_DF:
      dtile_core<T, false>(bx.cx, node_info(pl, it.K), it.a, it.b, smem, bx.DB + g.sq, g.s, bx.S + g.off, g.ld);
      break;
    default: break;
  }
}

// Small nodes (c <= kTinyC, s <= kTinyS): all of R1 (mode 1) or all of R3
// (mode 2) of one node in one wavefront, with the same algebra as the tile
// items above.  X_{C,C} (R1) and Sbar_{C,C} (R3) are read through the node's
// offset table (c x c row-major byte offsets), and the R1 scatter goes through
// the same table.  LDS blocks are [j * kTinyC + i] (c x s) and [j * 8 + i]
// (s x s).

// acc[j] = (Src_{C,C} B)(i, j), i = lane % CM, for B in LDS; lane groups
// over the contraction index are combined by a fixed butterfly.
template <int CM, typename T>
__device__ __forceinline__ void tiny_cc(const TinyRec &r, const uint32_t *toff, const T *Src, const T *bs,
                                        T (&acc)[kTinyS]) {
  constexpr int G = 64 / CM, U = CM / G;
  const int lane = threadIdx.x, i = lane % CM, grp = lane / CM;
  const int s = r.s, c = r.c;
  const uint32_t *tb = toff + r.tbl;
  const uint32_t rowb = 4u * ((uint32_t)(i * c + grp) & opaque_mask32(i < c));
  uint32_t o[U];
#pragma unroll
  for (int u = 0; u < U; ++u) o[u] = ld_off(tb, rowb + 4u * (G * u));
  T xv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) xv[u] = ld_off(Src, o[u]);
#pragma unroll
  for (int j = 0; j < kTinyS; ++j) acc[j] = zero_of<T>();
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = grp + G * u;
    const T g = masked(xv[u], opaque_mask(i < c && k < c));
#pragma unroll
    for (int j = 0; j < kTinyS; ++j)
      if (j < s) acc[j] += g * bs[j * kTinyC + k];
  }
#pragma unroll
  for (int m = CM; m < 64; m <<= 1)
#pragma unroll
    for (int j = 0; j < kTinyS; ++j)
      if (j < s) acc[j] += shfl_xor_t(acc[j], m);
}

template <typename T>
__device__ __forceinline__ void tiny_cc_any(const TinyRec &r, const uint32_t *toff, const T *Src, const T *bs,
                                            T (&acc)[kTinyS]) {
  if (r.c <= 8)
    tiny_cc<8, T>(r, toff, Src, bs, acc);
  else if (r.c <= 16)
    tiny_cc<16, T>(r, toff, Src, bs, acc);
  else
    tiny_cc<32, T>(r, toff, Src, bs, acc);
}

template <int MODE, typename T>
__global__ void __launch_bounds__(64) k_back_tiny(const DevPlan *__restrict__ plp, const T *panels, const T *x,
                                                  const T *dt, T *xbar, const TinyRec *__restrict__ recs,
                                                  int32_t count) {
  constexpr int TC = kTinyC, TS = kTinyS;
  const DevPlan &pl = *plp;
  __shared__ T lh[TS * TC], cb[TS * TC], yb[TS * TC];  // Lhat; Zbar (R1) / M + N (R3); Y Tbar (R1)
  __shared__ T tb[64], eb[64], fb[64];                  // Tbar (R1) / Dt (R3); E = Dt^{-1}; F (R1) / Dtbar0 (R3)
  const int64_t g0 = blockIdx.x;
  const int64_t l = g0 / count;
  const TinyRec r = recs[g0 - l * count];
  const int64_t pe = pl.panel_elems, sqe = pl.sq_elems;
  const T *Lp = panels + l * pe, *Xp = x + l * pe;
  T *W = xbar + l * pe;
  T *Lbar = static_cast<T *>(pl.adj_l) + l * pe;
  T *Sb = static_cast<T *>(pl.adj_s) + l * pe;
  T *DB = static_cast<T *>(pl.adj_d) + l * sqe;
  const T *DT = dt + l * sqe;
  const T zero = zero_of<T>();
  const int s = r.s, c = r.c, lane = threadIdx.x;
  const int64_t ld = s + c, off = r.off, sq = gp(pl.node_sq)[r.K];
  const int x8 = lane % 8, y8 = lane / 8;  // (x, y) of an s x s block
  const bool in_sq = x8 < s && y8 < s;
#pragma unroll
  for (int u = 0; u < TS * TC / 64; ++u) {
    const int e = lane + 64 * u, k = e % TC, j = e / TC;
    lh[e] = (k < c && j < s) ? Lp[off + j * ld + s + k] : zero;
  }
  eb[lane] = in_sq ? Lp[off + (int64_t)y8 * ld + x8] : zero;
  if (MODE == 1) {
    // Tbar = sym(W_KK)
    T t = zero;
    if (in_sq) {
      const T w = x8 >= y8 ? W[off + (int64_t)y8 * ld + x8] : W[off + (int64_t)x8 * ld + y8];
      t = x8 == y8 ? w : SOps<T>::scale(0.5, w);
    }
    tb[lane] = t;
    __syncthreads();
    // Zbar = W_{C,K} - Lhat Tbar;  Y Tbar (Y = X_{C,K}).  Every entry of the
    // Zbar block is written (zeros outside c x s): it is the B operand below.
    if (lane < TC) {
      const bool row = lane < c;
      T yr[TS];
#pragma unroll
      for (int k = 0; k < TS; ++k) yr[k] = (row && k < s) ? Xp[off + k * ld + s + lane] : zero;
#pragma unroll
      for (int j = 0; j < TS; ++j) {
        T z = zero, yt = zero;
        if (row && j < s) {
          z = W[off + j * ld + s + lane];
#pragma unroll
          for (int k = 0; k < TS; ++k) {
            z -= lh[k * TC + lane] * tb[j * 8 + k];
            yt += yr[k] * tb[j * 8 + k];
          }
        }
        cb[j * TC + lane] = z;
        yb[j * TC + lane] = yt;
      }
    }
    __syncthreads();
    // Lhatbar = -(X_{C,C} Zbar + Y Tbar)
    T acc[TS];
    tiny_cc_any<T>(r, pl.toff, Xp, cb, acc);
    if (lane < c && lane < (c <= 8 ? 8 : c <= 16 ? 16 : 32)) {
#pragma unroll
      for (int j = 0; j < TS; ++j)
        if (j < s) Lbar[off + j * ld + s + lane] = SOps<T>::scale(-1.0, acc[j] + yb[j * TC + lane]);
    }
    // W[ancestors] -= Zbar Lhat^T + Lhat Zbar^T on the lower part (halved on the diagonal)
    const int ne = c * (c + 1) / 2;
    for (int e = lane; e < ne; e += 64) {
      int i = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
      while (i * (i + 1) / 2 > e) --i;
      while ((i + 1) * (i + 2) / 2 <= e) ++i;
      const int k = e - i * (i + 1) / 2;
      T v = zero;
#pragma unroll
      for (int j = 0; j < TS; ++j)
        if (j < s) v += cb[j * TC + i] * lh[j * TC + k] + lh[j * TC + i] * cb[j * TC + k];
      atomic_add_t(reinterpret_cast<T *>(reinterpret_cast<char *>(W) + gp(pl.toff)[r.tbl + i * c + k]),
                   SOps<T>::scale(i == k ? -0.5 : -1.0, v));
    }
    // F = Tbar E;  Dtbar0 = -E F
    if (in_sq) {
      T f = zero;
      for (int k = 0; k < s; ++k) f += tb[k * 8 + x8] * eb[y8 * 8 + k];
      fb[lane] = f;
    }
    __syncthreads();
    if (in_sq) {
      T d = zero;
      for (int k = 0; k < s; ++k) d += eb[k * 8 + x8] * fb[y8 * 8 + k];
      DB[sq + (int64_t)y8 * s + x8] = SOps<T>::scale(-1.0, d);
    }
  } else {
    // Dt, Dtbar0
    tb[lane] = in_sq ? DT[sq + (int64_t)y8 * s + x8] : zero;
    fb[lane] = in_sq ? DB[sq + (int64_t)y8 * s + x8] : zero;
    __syncthreads();
    // M = Sbar_{C,C} Lhat;  Lb = Lhatbar - 2 M Dt;  N = Lb E;  Sbar_{C,K} = N / 2
    T m[TS];
    tiny_cc_any<T>(r, pl.toff, Sb, lh, m);
    if (lane < c && lane < (c <= 8 ? 8 : c <= 16 ? 16 : 32)) {
      T lb[TS];
#pragma unroll
      for (int j = 0; j < TS; ++j) {
        T v = zero;
        if (j < s) {
          T md = zero;
#pragma unroll
          for (int k = 0; k < TS; ++k)
            if (k < s) md += m[k] * tb[j * 8 + k];
          v = Lbar[off + j * ld + s + lane] - SOps<T>::scale(2.0, md);
        }
        lb[j] = v;
      }
#pragma unroll
      for (int j = 0; j < TS; ++j) {
        if (j < s) {
          T nv = zero;
#pragma unroll
          for (int k = 0; k < TS; ++k)
            if (k < s) nv += lb[k] * eb[j * 8 + k];
          Sb[off + j * ld + s + lane] = SOps<T>::scale(0.5, nv);
          cb[j * TC + lane] = m[j] + nv;
        }
      }
    }
    __syncthreads();
    // Sbar_KK = sym(Dtbar0 - Lhat^T (M + N))
    if (in_sq) {
      T rxy = zero, ryx = zero;
      for (int i = 0; i < c; ++i) {
        rxy += lh[x8 * TC + i] * cb[y8 * TC + i];
        ryx += lh[y8 * TC + i] * cb[x8 * TC + i];
      }
      Sb[off + (int64_t)y8 * ld + x8] = SOps<T>::scale(0.5, (fb[y8 * 8 + x8] - rxy) + (fb[x8 * 8 + y8] - ryx));
    }
  }
}

// Abar on A's pattern (stored-value convention: doubled off the diagonal),
// plus wlogdet[l] X (d log det A / dA = A^{-1}) when the loss has log-det terms.
template <typename T>
__global__ void k_abar(const DevPlan *__restrict__ plp, const T *x, const T *wlogdet, T *abar) {
  const DevPlan &pl = *plp;
  const int64_t total = pl.batch * pl.nnzA;
  const T *S = static_cast<const T *>(pl.adj_s);
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = q / pl.nnzA, e = q - l * pl.nnzA;
    const int64_t p = l * pl.panel_elems + gp(pl.apos)[e];
    T v = S[p];
    if (wlogdet) v += wlogdet[l] * x[p];
    abar[q] = gp(pl.adiag)[e] ? v : SOps<T>::scale(2.0, v);
  }
}

template <typename T>
hipError_t backward_impl(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, const void *panels,
                         const void *x, const void *dt, void *xbar, const void *wlogdet, void *abar, hipStream_t st) {
  const T *P = static_cast<const T *>(panels), *X = static_cast<const T *>(x), *D = static_cast<const T *>(dt);
  T *Wb = static_cast<T *>(xbar);
  for (int q = 0; q < aux.nblaunch; ++q) {
    const int4 bl = aux.blaunch[q];  // {kind, first, count}: 0 items, 1 small-node R1, 2 small-node R3
    if (bl.z <= 0) continue;
    const dim3 grid((unsigned)(bl.z * pl.batch));
    if (bl.x == 0)
      hipLaunchKernelGGL(k_back_items<T>, grid, dim3(NT), 0, st, dpl, P, X, D, Wb, bl.y, bl.z);
    else if (bl.x == 1)
      hipLaunchKernelGGL((k_back_tiny<1, T>), grid, dim3(64), 0, st, dpl, P, X, D, Wb, aux.tiny + bl.y, bl.z);
    else
      hipLaunchKernelGGL((k_back_tiny<2, T>), grid, dim3(64), 0, st, dpl, P, X, D, Wb, aux.tiny + bl.y, bl.z);
  }
  const int64_t total = pl.batch * pl.nnzA;
  unsigned grid = (unsigned)((total + 255) / 256);
  if (grid > 65536u) grid = 65536u;
  if (grid == 0) grid = 1;
  hipLaunchKernelGGL(k_abar<T>, dim3(grid), dim3(256), 0, st, dpl, X, static_cast<const T *>(wlogdet),
                     static_cast<T *>(abar));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_backward(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, bool cplx_, const void *panels,
                           const void *x, const void *dt, void *xbar, const void *wlogdet, void *abar, hipStream_t st) {
  if (!pl.adj_s) return hipErrorNotSupported;
  return cplx_ ? backward_impl<cplx>(pl, dpl, aux, panels, x, dt, xbar, wlogdet, abar, st)
               : backward_impl<double>(pl, dpl, aux, panels, x, dt, xbar, wlogdet, abar, st);
}

}  // namespace selinv
