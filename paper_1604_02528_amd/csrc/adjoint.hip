// Adjoint of the selected inversion (reverse mode), FP64 on gfx950.
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
// the scatter-add uses hardware FP64 atomics (summation order, and hence the
// last bits, may differ between runs).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "items.hpp"
#include "plan.hpp"
#include "tile.hpp"

namespace selinv {
namespace {

struct BCtx {
  Ctx<double> cx;        // Lp normalized panels, Xp the forward X, Pp partials, Gp dense buffers
  double *W;             // stored-value gradient on F, accumulated in place
  double *Z, *L, *S;     // panel-layout scratch: Zbar then M; Lhatbar then Lb; Sbar
  double *TB, *FB, *DB;  // s x s scratch: Tbar; F = Tbar E; Dtbar0
  const double *DT;      // Dt = L_KK D_K L_KK^T
};

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
template <class F>
__device__ void store_tile(const Acc<double> &acc, double *smem, double *dst, int64_t ld, int i0, int j0, int rows,
                           int cols, F f) {
  acc_to_lds<double>(acc, smem);
  lds_barrier();
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = e & 63, j = e >> 6;
    if (i0 + i < rows && j0 + j < cols) {
      const int64_t q = (int64_t)(j0 + j) * ld + i0 + i;
      dst[q] = f(q, smem[j * PITCH + i]);
    }
  }
  lds_barrier();
}

using DA = LoadDenseA<double, DenseTK<double>::TK>;
using DB = LoadDenseB<double, DenseTK<double>::TK>;
using DBT = LoadDenseBT<double, DenseTK<double>::TK>;

// acc = X_{C,C}[tile rows, :] B[:, tile cols] with X_{C,C} gathered from Src (panel
// layout) or read from the node's dense buffer; B = the c x s bottom block of a
// panel-layout array Bp.
__device__ void gemm_cc(const BCtx &bx, const Geo &g, const double *Src, const double *Bp, int i0, int j0,
                        double *smem, int64_t *rt, Acc<double> &acc) {
  const DevPlan &pl = *bx.cx.pl;
  if (uniform(g.goff >= 0 ? 1 : 0)) {
    DA la{bx.cx.Gp + g.goff, g.ldg, g.c, g.c, i0};
    DB lb{Bp, g.off, g.ld, g.s, g.c, j0, g.s};
    gemm_dense<double>(0, g.c, la, lb, smem, acc);
  } else {
    if (threadIdx.x < 64) {
      const int ig = i0 + threadIdx.x;
      rt[threadIdx.x] = gp(pl.kcol)[g.rp + (ig < g.c ? ig : 0)];
      rt[64 + threadIdx.x] = gp(pl.kpos)[g.rp + (ig < g.c ? ig : 0)];
    }
    lds_barrier();
    LoadGather<double, false> la{Src, pl.kcol + g.rp, pl.kpos + g.rp, pl.posarr, rt, rt + 64, g.c, g.c, i0};
    LoadPanelK<double, false> lb{Bp, g.off, g.ld, g.s, 0, g.c, j0, g.s};
    gemm_tile<double>(0, g.c, la, lb, smem, acc);
  }
}

__device__ void bi_t(const BCtx &bx, const Geo &g, int a, int b) {
  const int i0 = a * 64, j0 = b * 64;
  const double *Wk = bx.W + g.off;
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = i0 + (e & 63), j = j0 + (e >> 6);
    if (i < g.s && j < g.s) {
      const double w = i >= j ? Wk[(int64_t)j * g.ld + i] : Wk[(int64_t)i * g.ld + j];
      bx.TB[g.sq + (int64_t)j * g.s + i] = i == j ? w : 0.5 * w;
    }
  }
}

__device__ void bi_z(const BCtx &bx, const Geo &g, int a, int b, double *smem) {
  const int i0 = a * 64, j0 = b * 64;
  Acc<double> acc;
  gemm_dense<double>(0, g.s, DA{bx.cx.Lp + g.off + g.s, g.ld, g.c, g.s, i0}, DB{bx.TB + g.sq, 0, g.s, 0, g.s, j0, g.s},
                     smem, acc);
  const double *Wb = bx.W + g.off + g.s;
  store_tile(acc, smem, bx.Z + g.off + g.s, g.ld, i0, j0, g.c, g.s,
             [&](int64_t q, double v) { return Wb[q] - v; });
}

__device__ void bi_l(const BCtx &bx, const Geo &g, int a, int b, double *smem, int64_t *rt) {
  const int i0 = a * 64, j0 = b * 64;
  Acc<double> acc;
  gemm_cc(bx, g, bx.cx.Xp, bx.Z, i0, j0, smem, rt, acc);  // X_{C,C} Zbar
  gemm_dense<double>(0, g.s, DA{bx.cx.Xp + g.off + g.s, g.ld, g.c, g.s, i0}, DB{bx.TB + g.sq, 0, g.s, 0, g.s, j0, g.s},
                     smem, acc, true);  // + Y Tbar
  store_tile(acc, smem, bx.L + g.off + g.s, g.ld, i0, j0, g.c, g.s, [](int64_t, double v) { return -v; });
}

// Rows 64a.., columns 64a2.. (a >= a2) of Zbar Lhat^T + Lhat Zbar^T, subtracted
// from the stored-value gradient of the ancestors' entries of X_{C,C}.
__device__ void bi_sc(const BCtx &bx, const Geo &g, int a, int a2, double *smem) {
  const DevPlan &pl = *bx.cx.pl;
  const int i0 = a * 64, k0 = a2 * 64;
  const double *Zb = bx.Z + g.off + g.s, *Lh = bx.cx.Lp + g.off + g.s;
  Acc<double> acc;
  gemm_dense<double>(0, g.s, DA{Zb, g.ld, g.c, g.s, i0}, DBT{Lh, g.ld, g.s, k0, g.c}, smem, acc);
  gemm_dense<double>(0, g.s, DA{Lh, g.ld, g.c, g.s, i0}, DBT{Zb, g.ld, g.s, k0, g.c}, smem, acc, true);
  acc_to_lds<double>(acc, smem);
  lds_barrier();
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = e & 63, k = e >> 6;
    const int ig = i0 + i, kg = k0 + k;
    if (ig < g.c && kg < g.c && ig >= kg) {
      const double v = smem[k * PITCH + i];
      const int64_t addr = gp(pl.kcol)[g.rp + kg] + gp(pl.posarr)[gp(pl.kpos)[g.rp + kg] + ig];
      unsafeAtomicAdd(bx.W + addr, ig == kg ? -0.5 * v : -v);
    }
  }
  lds_barrier();
}

__device__ void bi_f(const BCtx &bx, const Geo &g, int a, int b, double *smem) {
  const int i0 = a * 64, j0 = b * 64;
  Acc<double> acc;
  gemm_dense<double>(0, g.s, DA{bx.TB + g.sq, g.s, g.s, g.s, i0}, DB{bx.cx.Lp, g.off, g.ld, 0, g.s, j0, g.s}, smem,
                     acc);
  store_tile(acc, smem, bx.FB + g.sq, g.s, i0, j0, g.s, g.s, [](int64_t, double v) { return v; });
}

__device__ void bi_d0(const BCtx &bx, const Geo &g, int a, int b, double *smem) {
  const int i0 = a * 64, j0 = b * 64;
  Acc<double> acc;
  gemm_dense<double>(0, g.s, DA{bx.cx.Lp + g.off, g.ld, g.s, g.s, i0}, DB{bx.FB + g.sq, 0, g.s, 0, g.s, j0, g.s},
                     smem, acc);
  store_tile(acc, smem, bx.DB + g.sq, g.s, i0, j0, g.s, g.s, [](int64_t, double v) { return -v; });
}

__device__ void bi_m(const BCtx &bx, const Geo &g, int a, int b, double *smem, int64_t *rt) {
  const int i0 = a * 64, j0 = b * 64;
  Acc<double> acc;
  gemm_cc(bx, g, bx.S, bx.cx.Lp, i0, j0, smem, rt, acc);  // Sbar_{C,C} Lhat
  store_tile(acc, smem, bx.Z + g.off + g.s, g.ld, i0, j0, g.c, g.s, [](int64_t, double v) { return v; });
}

__device__ void bi_lb(const BCtx &bx, const Geo &g, int a, int b, double *smem) {
  const int i0 = a * 64, j0 = b * 64;
  Acc<double> acc;
  gemm_dense<double>(0, g.s, DA{bx.Z + g.off + g.s, g.ld, g.c, g.s, i0}, DB{bx.DT + g.sq, 0, g.s, 0, g.s, j0, g.s},
                     smem, acc);
  double *Lb = bx.L + g.off + g.s;
  store_tile(acc, smem, Lb, g.ld, i0, j0, g.c, g.s, [&](int64_t q, double v) { return Lb[q] - 2.0 * v; });
}

__device__ void bi_n(const BCtx &bx, const Geo &g, int K, int a, int b, double *smem) {
  const int i0 = a * 64, j0 = b * 64;
  Acc<double> acc;
  gemm_dense<double>(0, g.s, DA{bx.L + g.off + g.s, g.ld, g.c, g.s, i0}, DB{bx.cx.Lp, g.off, g.ld, 0, g.s, j0, g.s},
                     smem, acc);  // N = Lb E
  store_tile(acc, smem, bx.S + g.off + g.s, g.ld, i0, j0, g.c, g.s, [](int64_t, double v) { return 0.5 * v; });
  // acc <- -(M + N) in the accumulator layout, then the row tile's share of
  // Lhat^T (M + N) into the partial products
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w & 1, wj = w >> 1;
  const double *M = bx.Z + g.off + g.s;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 32 * wi + 16 * bi + 4 * v + (lane >> 4);
        const int j = j0 + 32 * wj + 16 * bj + (lane & 15);
        const int64_t m = opaque_mask(i < g.c && j < g.s);
        const double mv = masked(M[((int64_t)j * g.ld + i) & m], m);
        acc.v[0][bi][bj][v] = -(mv + masked(acc.v[0][bi][bj][v], m));
      }
  gemm2_partial<double, false>(bx.cx, node_info(*bx.cx.pl, K), a, b, acc, smem);
}

__global__ void __launch_bounds__(NT, 2)
    k_back_items(const DevPlan *__restrict__ plp, const double *panels, const double *x, const double *dt,
                 double *xbar, int32_t first, int32_t count) {
  const DevPlan &pl = *plp;
  __shared__ double smem[smem_doubles<double>()];
  __shared__ int64_t rt[128];
  const int64_t g0 = blockIdx.x;
  const int64_t l = g0 / count;
  const Item it = uniform(gload(pl.bitems + first + (g0 - l * count)));
  const int64_t pe = pl.panel_elems, sq = pl.sq_elems;
  BCtx bx;
  bx.cx = Ctx<double>{&pl, panels + l * pe, const_cast<double *>(x) + l * pe,
                      static_cast<double *>(pl.part) + l * pl.part_elems,
                      static_cast<double *>(pl.gbuf) + l * pl.g_elems, nullptr};
  bx.W = xbar + l * pe;
  bx.Z = static_cast<double *>(pl.adj_z) + l * pe;
  bx.L = static_cast<double *>(pl.adj_l) + l * pe;
  bx.S = static_cast<double *>(pl.adj_s) + l * pe;
  bx.TB = static_cast<double *>(pl.adj_t) + l * sq;
  bx.FB = static_cast<double *>(pl.adj_f) + l * sq;
  bx.DB = static_cast<double *>(pl.adj_d) + l * sq;
  bx.DT = dt + l * sq;
  const Geo g = geo(pl, it.K);
  switch (it.type) {
    case BI_T: bi_t(bx, g, it.a, it.b); break;
    case BI_G: do_gtile<double>(bx.cx, node_info(pl, it.K), it.a, it.b, smem, rt, bx.cx.Xp); break;
    case BI_Z: bi_z(bx, g, it.a, it.b, smem); break;
    case BI_L: bi_l(bx, g, it.a, it.b, smem, rt); break;
    case BI_SC: bi_sc(bx, g, it.a, it.b, smem); break;
    case BI_F: bi_f(bx, g, it.a, it.b, smem); break;
    case BI_D0: bi_d0(bx, g, it.a, it.b, smem); break;
    case BI_SG: do_gtile<double>(bx.cx, node_info(pl, it.K), it.a, it.b, smem, rt, bx.S); break;
    case BI_M: bi_m(bx, g, it.a, it.b, smem, rt); break;
    case BI_LB: bi_lb(bx, g, it.a, it.b, smem); break;
    case BI_N: bi_n(bx, g, it.K, it.a, it.b, smem); break;
    case BI_DF:
      dtile_core<double, false>(bx.cx, node_info(pl, it.K), it.a, it.b, smem, bx.DB + g.sq, g.s, bx.S + g.off, g.ld);
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
template <int CM>
__device__ __forceinline__ void tiny_cc(const TinyRec &r, const uint32_t *toff, const double *Src, const double *bs,
                                        double (&acc)[kTinyS]) {
  constexpr int G = 64 / CM, U = CM / G;
  const int lane = threadIdx.x, i = lane % CM, grp = lane / CM;
  const int s = r.s, c = r.c;
  const uint32_t *tb = toff + r.tbl;
  const uint32_t rowb = 4u * ((uint32_t)(i * c + grp) & opaque_mask32(i < c));
  uint32_t o[U];
#pragma unroll
  for (int u = 0; u < U; ++u) o[u] = ld_off(tb, rowb + 4u * (G * u));
  double xv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) xv[u] = ld_off(Src, o[u]);
#pragma unroll
  for (int j = 0; j < kTinyS; ++j) acc[j] = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = grp + G * u;
    const double g = masked(xv[u], opaque_mask(i < c && k < c));
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

__device__ __forceinline__ void tiny_cc_any(const TinyRec &r, const uint32_t *toff, const double *Src, const double *bs,
                                            double (&acc)[kTinyS]) {
  if (r.c <= 8)
    tiny_cc<8>(r, toff, Src, bs, acc);
  else if (r.c <= 16)
    tiny_cc<16>(r, toff, Src, bs, acc);
  else
    tiny_cc<32>(r, toff, Src, bs, acc);
}

template <int MODE>
__global__ void __launch_bounds__(64) k_back_tiny(const DevPlan *__restrict__ plp, const double *panels,
                                                  const double *x, const double *dt, double *xbar,
                                                  const TinyRec *__restrict__ recs, int32_t count) {
  constexpr int TC = kTinyC, TS = kTinyS;
  const DevPlan &pl = *plp;
  __shared__ double lh[TS * TC], cb[TS * TC], yb[TS * TC];  // Lhat; Zbar (R1) / M + N (R3); Y Tbar (R1)
  __shared__ double tb[64], eb[64], fb[64];                   // Tbar (R1) / Dt (R3); E = Dt^{-1}; F (R1) / Dtbar0 (R3)
  const int64_t g0 = blockIdx.x;
  const int64_t l = g0 / count;
  const TinyRec r = recs[g0 - l * count];
  const int64_t pe = pl.panel_elems, sqe = pl.sq_elems;
  const double *Lp = panels + l * pe, *Xp = x + l * pe;
  double *W = xbar + l * pe;
  double *Lbar = static_cast<double *>(pl.adj_l) + l * pe;
  double *Sb = static_cast<double *>(pl.adj_s) + l * pe;
  double *DB = static_cast<double *>(pl.adj_d) + l * sqe;
  const double *DT = dt + l * sqe;
  const int s = r.s, c = r.c, lane = threadIdx.x;
  const int64_t ld = s + c, off = r.off, sq = gp(pl.node_sq)[r.K];
  const int x8 = lane % 8, y8 = lane / 8;  // (x, y) of an s x s block
  const bool in_sq = x8 < s && y8 < s;
#pragma unroll
  for (int u = 0; u < TS * TC / 64; ++u) {
    const int e = lane + 64 * u, k = e % TC, j = e / TC;
    lh[e] = (k < c && j < s) ? Lp[off + j * ld + s + k] : 0.0;
  }
  eb[lane] = in_sq ? Lp[off + (int64_t)y8 * ld + x8] : 0.0;
  if (MODE == 1) {
    // Tbar = sym(W_KK)
    double t = 0.0;
    if (in_sq) {
      const double w = x8 >= y8 ? W[off + (int64_t)y8 * ld + x8] : W[off + (int64_t)x8 * ld + y8];
      t = x8 == y8 ? w : 0.5 * w;
    }
    tb[lane] = t;
    __syncthreads();
    // Zbar = W_{C,K} - Lhat Tbar;  Y Tbar (Y = X_{C,K}).  Every entry of the
    // Zbar block is written (zeros outside c x s): it is the B operand below.
    if (lane < TC) {
      const bool row = lane < c;
      double yr[TS];
#pragma unroll
      for (int k = 0; k < TS; ++k) yr[k] = (row && k < s) ? Xp[off + k * ld + s + lane] : 0.0;
#pragma unroll
      for (int j = 0; j < TS; ++j) {
        double z = 0.0, yt = 0.0;
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
    double acc[TS];
    tiny_cc_any(r, pl.toff, Xp, cb, acc);
    if (lane < c && lane < (c <= 8 ? 8 : c <= 16 ? 16 : 32)) {
#pragma unroll
      for (int j = 0; j < TS; ++j)
        if (j < s) Lbar[off + j * ld + s + lane] = -(acc[j] + yb[j * TC + lane]);
    }
    // W[ancestors] -= Zbar Lhat^T + Lhat Zbar^T on the lower part (halved on the diagonal)
    const int ne = c * (c + 1) / 2;
    for (int e = lane; e < ne; e += 64) {
      int i = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
      while (i * (i + 1) / 2 > e) --i;
      while ((i + 1) * (i + 2) / 2 <= e) ++i;
      const int k = e - i * (i + 1) / 2;
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < TS; ++j)
        if (j < s) v += cb[j * TC + i] * lh[j * TC + k] + lh[j * TC + i] * cb[j * TC + k];
      unsafeAtomicAdd(reinterpret_cast<double *>(reinterpret_cast<char *>(W) + gp(pl.toff)[r.tbl + i * c + k]),
                      i == k ? -0.5 * v : -v);
    }
    // F = Tbar E;  Dtbar0 = -E F
    if (in_sq) {
      double f = 0.0;
      for (int k = 0; k < s; ++k) f += tb[k * 8 + x8] * eb[y8 * 8 + k];
      fb[lane] = f;
    }
    __syncthreads();
    if (in_sq) {
      double d = 0.0;
      for (int k = 0; k < s; ++k) d += eb[k * 8 + x8] * fb[y8 * 8 + k];
      DB[sq + (int64_t)y8 * s + x8] = -d;
    }
  } else {
    // Dt, Dtbar0
    tb[lane] = in_sq ? DT[sq + (int64_t)y8 * s + x8] : 0.0;
    fb[lane] = in_sq ? DB[sq + (int64_t)y8 * s + x8] : 0.0;
    __syncthreads();
    // M = Sbar_{C,C} Lhat;  Lb = Lhatbar - 2 M Dt;  N = Lb E;  Sbar_{C,K} = N / 2
    double m[TS];
    tiny_cc_any(r, pl.toff, Sb, lh, m);
    if (lane < c && lane < (c <= 8 ? 8 : c <= 16 ? 16 : 32)) {
      double lb[TS];
#pragma unroll
      for (int j = 0; j < TS; ++j) {
        double v = 0.0;
        if (j < s) {
          double md = 0.0;
#pragma unroll
          for (int k = 0; k < TS; ++k)
            if (k < s) md += m[k] * tb[j * 8 + k];
          v = Lbar[off + j * ld + s + lane] - 2.0 * md;
        }
        lb[j] = v;
      }
#pragma unroll
      for (int j = 0; j < TS; ++j) {
        if (j < s) {
          double nv = 0.0;
#pragma unroll
          for (int k = 0; k < TS; ++k)
            if (k < s) nv += lb[k] * eb[j * 8 + k];
          Sb[off + j * ld + s + lane] = 0.5 * nv;
          cb[j * TC + lane] = m[j] + nv;
        }
      }
    }
    __syncthreads();
    // Sbar_KK = sym(Dtbar0 - Lhat^T (M + N))
    if (in_sq) {
      double rxy = 0.0, ryx = 0.0;
      for (int i = 0; i < c; ++i) {
        rxy += lh[x8 * TC + i] * cb[y8 * TC + i];
        ryx += lh[y8 * TC + i] * cb[x8 * TC + i];
      }
      Sb[off + (int64_t)y8 * ld + x8] = 0.5 * ((fb[y8 * 8 + x8] - rxy) + (fb[x8 * 8 + y8] - ryx));
    }
  }
}

// Abar on A's pattern (stored-value convention: doubled off the diagonal),
// plus wlogdet[l] X (d log det A / dA = A^{-1}) when the loss has log-det terms.
__global__ void k_abar(const DevPlan *__restrict__ plp, const double *x, const double *wlogdet, double *abar) {
  const DevPlan &pl = *plp;
  const int64_t total = pl.batch * pl.nnzA;
  const double *S = static_cast<const double *>(pl.adj_s);
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = q / pl.nnzA, e = q - l * pl.nnzA;
    const int64_t p = l * pl.panel_elems + gp(pl.apos)[e];
    double v = S[p];
    if (wlogdet) v += wlogdet[l] * x[p];
    abar[q] = gp(pl.adiag)[e] ? v : 2.0 * v;
  }
}

}  // namespace

hipError_t launch_backward(const DevPlan &pl, const DevPlan *dpl, const LaunchAux &aux, const void *panels,
                           const void *x, const void *dt, void *xbar, const void *wlogdet, void *abar, hipStream_t st) {
  if (!pl.adj_s) return hipErrorNotSupported;
  const double *P = static_cast<const double *>(panels), *X = static_cast<const double *>(x),
               *D = static_cast<const double *>(dt);
  double *Wb = static_cast<double *>(xbar);
  for (int q = 0; q < aux.nblaunch; ++q) {
    const int4 bl = aux.blaunch[q];  // {kind, first, count}: 0 items, 1 small-node R1, 2 small-node R3
    if (bl.z <= 0) continue;
    const dim3 grid((unsigned)(bl.z * pl.batch));
    if (bl.x == 0)
      hipLaunchKernelGGL(k_back_items, grid, dim3(NT), 0, st, dpl, P, X, D, Wb, bl.y, bl.z);
    else if (bl.x == 1)
      hipLaunchKernelGGL(k_back_tiny<1>, grid, dim3(64), 0, st, dpl, P, X, D, Wb, aux.tiny + bl.y, bl.z);
    else
      hipLaunchKernelGGL(k_back_tiny<2>, grid, dim3(64), 0, st, dpl, P, X, D, Wb, aux.tiny + bl.y, bl.z);
  }
  const int64_t total = pl.batch * pl.nnzA;
  unsigned grid = (unsigned)((total + 255) / 256);
  if (grid > 65536u) grid = 65536u;
  if (grid == 0) grid = 1;
  hipLaunchKernelGGL(k_abar, dim3(grid), dim3(256), 0, st, dpl, X, static_cast<const double *>(wlogdet),
                     static_cast<double *>(abar));
  return hipGetLastError();
}

}  // namespace selinv
