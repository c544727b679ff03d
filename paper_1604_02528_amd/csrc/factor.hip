// Numeric factorization on the GPU: unpivoted supernodal LDL^T of B = P A P^T
// (LDL^H for a Hermitian A: the transposed factor of every product below is
// conjugated, Section 2.3).
//
// The paper takes its factors from an external solver that permutes
// symmetrically and does no dynamic pivoting (Section 4); this is the
// library's device producer of that input, in the panel layout the rest of
// the path reads (strict lower L_KK, D_K on the diagonal, L_{C,K} below).
// Right-looking supernodal form, one launch per etree depth and step, the
// deepest depth first (every descendant of K is complete before K starts):
//
//   diag   S_KK = L_KK D_K L_KK^T, unblocked in LDS on 32-column blocks with
//          the trailing update of the rest of the block (one workgroup per
//          node; zero or non-finite pivots are recorded, not fixed)
//   inv    L_KK^{-1} and D_K^{-1} (the normalization's inverse kernel)
//   lc     L_{C,K} = S_{C,K} L_KK^{-T} D_K^{-1}, one workgroup per 64-row block
//          of C(K), column tiles right to left on FP64 MFMA (in place)
//   schur  S_{C,C} -= L_{C,K} D_K L_{C,K}^T on the lower block pairs of C(K),
//          scattered into the ancestors' panels through the same index maps
//          the selected inversion gathers through (Eq. (newset)), with FP64
//          atomic adds: siblings of one depth update shared ancestors, so the
//          summation order (and the last bits) may vary from run to run.
//
// A last kernel sums log D_jj per matrix (log det B, Section 2.3) in a fixed
// order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "items.hpp"
#include "plan.hpp"
#include "scalar.hpp"
#include "tile.hpp"

namespace selinv {

hipError_t launch_linv(const DevPlan &pl, const DevPlan *dpl, bool cplx_, const void *src, const int2 *chunks,
                       int32_t n, bool narrow, hipStream_t st);
hipError_t launch_scatter(const DevPlan &pl, const DevPlan *dpl, bool cplx_, const void *vals, void *panel,
                          hipStream_t st);

namespace {

__device__ __forceinline__ bool finite_nonzero(double d) { return d != 0.0 && isfinite(d); }
__device__ __forceinline__ bool finite_nonzero(cplx d) {
  return (d.re != 0.0 || d.im != 0.0) && isfinite(d.re) && isfinite(d.im);
}

__device__ __forceinline__ void atomic_sub(double *p, double v) { unsafeAtomicAdd(p, -v); }
__device__ __forceinline__ void atomic_sub(cplx *p, cplx v) {
  double *q = reinterpret_cast<double *>(p);
  unsafeAtomicAdd(q, -v.re);
  unsafeAtomicAdd(q + 1, -v.im);
}

// B(k, x) = D(k) M[k ld + x0 + x] with D(k) = Dg[k dld]: the transposed view
// of LoadDenseBT with row k scaled by the pivot D_k (the row of a slot is
// uniform in a wave, so the pivot is one scalar load per slot).
template <typename T, int TK> struct LoadDenseBTScaled : LoadDenseBT<T, TK> {
  const T *Dg;
  int64_t dld;
  __device__ __forceinline__ LoadDenseBTScaled(const T *M_, int ld_, int kend_, int x0, int xmax, const T *Dg_,
                                               int64_t dld_)
      : LoadDenseBT<T, TK>(M_, ld_, kend_, x0, xmax), Dg(Dg_), dld(dld_) {}
  __device__ __forceinline__ void load(int k0, DVals<T, TK> &v) const {
#pragma unroll
    for (int m = 0; m < LoadDenseBT<T, TK>::E; ++m) {
      const int k = min(k0 + this->kq + (NT / 64) * m, this->kend - 1);
      v.v[m] = ld_off(this->M + (int64_t)k * this->ld, this->vcol) * gload(Dg + (int64_t)k * dld);
    }
  }
};

constexpr int kFacBW = 32;             // column block of the diagonal factorization
constexpr int kFacRows = 256 - kFacBW; // rows below a block inside a diagonal block (s <= 256)

// Unpivoted LDL^T of the diagonal block S_KK of one node (one workgroup).
// For each block of BW columns: the block's own LDL^T in LDS (column by
// column, each step a rank-one update of the rest of the block), then the
// rows of S_KK below the block by forward substitution (one row per
// thread), then the trailing update of S_KK below the block.  Only the lower
// triangle is read and written.
template <typename T>
__global__ void __launch_bounds__(NT) k_fac_diag(const DevPlan *__restrict__ plp, T *Pall, const int32_t *nodes,
                                                 int32_t count, unsigned long long *ferr) {
  constexpr int BW = kFacBW, BP = BW + 1;
  const DevPlan &pl = *plp;
  __shared__ T ajj[BW * BP];
  __shared__ T lb[kFacRows * BW];
  __shared__ T dv[BW];
  const int64_t g = blockIdx.x;
  const int64_t l = g / count;
  const int K = uniform(nodes[g - l * count]);
  const int s = uniform(gp(pl.node_s)[K]), c = uniform(gp(pl.node_c)[K]), ld = s + c;
  T *P = Pall + l * pl.panel_elems + gp(pl.node_off)[K];
  const int64_t first = gp(pl.node_first)[K];
  const int t = threadIdx.x;
  const double cs = pl.csign;  // LDL^H in a Hermitian plan: the right factor conjugated
  for (int jb = 0; jb < s; jb += BW) {
    const int w = min(BW, s - jb);
    for (int e = t; e < BW * BW; e += NT) {
      const int i = e % BW, k = e / BW;
      if (i < w && k <= i) ajj[i * BP + k] = P[(int64_t)(jb + k) * ld + jb + i];
    }
    __syncthreads();
    for (int j = 0; j < w; ++j) {
      const T d = ajj[j * BP + j];
      if (t == 0 && !finite_nonzero(d)) atomicMin(ferr + l, (unsigned long long)(first + jb + j));
      if (t > j && t < w) ajj[t * BP + j] = SOps<T>::div(ajj[t * BP + j], d);
      __syncthreads();
      for (int e = t; e < BW * BW; e += NT) {
        const int i = e % BW, k = e / BW;
        if (k > j && k <= i && i < w) ajj[i * BP + k] -= ajj[i * BP + j] * d * cj(ajj[k * BP + j], cs);
      }
      __syncthreads();
    }
    for (int e = t; e < BW * BW; e += NT) {
      const int i = e % BW, k = e / BW;
      if (i < w && k <= i) P[(int64_t)(jb + k) * ld + jb + i] = ajj[i * BP + k];
    }
    if (t < w) dv[t] = ajj[t * BP + t];
    __syncthreads();
    // rows r = jb + w + rr of S_KK: L(r, jb + j) = (S(r, jb + j) - sum_{k<j} L(r, jb + k) D_k L(jb + j, jb + k)) / D_j
    const int m = s - jb - w;
    for (int rr = t; rr < m; rr += NT) {
      const int r = jb + w + rr;
      T a[BW];
#pragma unroll
      for (int j = 0; j < BW; ++j) a[j] = j < w ? P[(int64_t)(jb + j) * ld + r] : zero_of<T>();
#pragma unroll
      for (int j = 0; j < BW; ++j) {
        if (j < w) {
          T v = a[j];
#pragma unroll
          for (int k = 0; k < j; ++k) v -= a[k] * dv[k] * cj(ajj[j * BP + k], cs);
          a[j] = SOps<T>::div(v, dv[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < BW; ++j)
        if (j < w) {
          P[(int64_t)(jb + j) * ld + r] = a[j];
          lb[rr * BW + j] = a[j];
        }
    }
    __syncthreads();
    // trailing update: S(r, q) -= sum_j L(r, j) D_j L(q, j), jb + w <= q <= r < s
    const int npair = m * (m + 1) / 2;
    for (int e = t; e < npair; e += NT) {
      int rr = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
      while (rr * (rr + 1) / 2 > e) --rr;
      while ((rr + 1) * (rr + 2) / 2 <= e) ++rr;
      const int qq = e - rr * (rr + 1) / 2;
      T acc = zero_of<T>();
      for (int j = 0; j < w; ++j) acc += lb[rr * BW + j] * dv[j] * cj(lb[qq * BW + j], cs);
      P[(int64_t)(jb + w + qq) * ld + jb + w + rr] -= acc;
    }
    __syncthreads();
  }
}

// L_{C,K} = S_{C,K} L_KK^{-T} D_K^{-1} (L_KK^{-H} if Hermitian) for one 64-row
// block of C(K), in place.
// Column tile x of the result needs columns k <= x of S_{C,K} only (L_KK^{-1}
// is lower triangular), so tiles run right to left and each is stored after
// its own product has read everything it needs.
template <typename T>
__global__ void __launch_bounds__(NT, Planes<T>::P == 1 ? 2 : 1)
    k_fac_lc(const DevPlan *__restrict__ plp, T *Pall, const int2 *rblocks, int32_t nrb) {
  const DevPlan &pl = *plp;
  constexpr int TK = DenseTK<T>::TK;
  constexpr int kStages = 2 * dense_stage_doubles<T, TK>();
  __shared__ double smem[kStages > tile_doubles<T>() ? kStages : tile_doubles<T>()];
  const int64_t g = blockIdx.x;
  const int64_t l = g / nrb;
  const int2 rb = rblocks[g - l * nrb];
  const int K = uniform(rb.x), i0 = uniform(rb.y) * 64;
  const int s = uniform(gp(pl.node_s)[K]), c = uniform(gp(pl.node_c)[K]), ld = s + c;
  T *P = Pall + l * pl.panel_elems + gp(pl.node_off)[K];
  const T *Linv = reinterpret_cast<const T *>(pl.linv) + l * pl.sq_elems + gp(pl.node_sq)[K];
  const T *dinv = reinterpret_cast<const T *>(pl.dinv) + l * pl.n + gp(pl.node_first)[K];
  for (int x0 = uniform(((s - 1) / 64) * 64); x0 >= 0; x0 -= 64) {
    const int kend = min(s, x0 + 64);
    LoadDenseA<T, TK> la{P + s, ld, c, kend, i0};     // S_{C,K}(i, k)
    LoadDenseBT<T, TK> lb{Linv, s, kend, x0, s};       // L_KK^{-1}(x, k), conjugated if Hermitian
    lb.cs = pl.csign;
    Acc<T> acc;
    gemm_dense<T>(0, kend, la, lb, smem, acc);
    acc_to_lds<T>(acc, smem);
    lds_barrier();
    for (int e = threadIdx.x; e < 64 * 64; e += NT) {
      const int i = e & 63, x = e >> 6;
      if (i0 + i < c && x0 + x < s)
        P[(int64_t)(x0 + x) * ld + s + i0 + i] = lds_get<T>(smem, i, x) * gload(dinv + x0 + x);
    }
    __syncthreads();  // the next tile reads columns this one did not write; LDS reuse
  }
}

// Block (a, b), a >= b, of the update L_{C,K} D_K L_{C,K}^T (^H if Hermitian), subtracted from
// the ancestors' entries of S_{C,C} (lower part: C-local rows i >= k).
template <typename T>
__global__ void __launch_bounds__(NT, Planes<T>::P == 1 ? 2 : 1)
    k_fac_schur(const DevPlan *__restrict__ plp, T *Pall, const int4 *tiles, int32_t ntiles) {
  const DevPlan &pl = *plp;
  constexpr int TK = DenseTK<T>::TK;
  constexpr int kStages = 2 * dense_stage_doubles<T, TK>();
  __shared__ double smem[kStages > tile_doubles<T>() ? kStages : tile_doubles<T>()];
  const int64_t g = blockIdx.x;
  const int64_t l = g / ntiles;
  const int4 tl = tiles[g - l * ntiles];
  const int K = uniform(tl.x), i0 = uniform(tl.y) * 64, k0 = uniform(tl.z) * 64;
  const int s = uniform(gp(pl.node_s)[K]), c = uniform(gp(pl.node_c)[K]), ld = s + c;
  T *Pl = Pall + l * pl.panel_elems;
  const int64_t off = gp(pl.node_off)[K], rp = gp(pl.node_rowptr)[K];
  const T *P = Pl + off;
  LoadDenseA<T, TK> la{P + s, ld, c, s, i0};                           // L_C(i, j)
  LoadDenseBTScaled<T, TK> lb{P + s, ld, s, k0, c, P, (int64_t)ld + 1};  // D_j L_C(k, j) (conjugated if Hermitian)
  lb.cs = pl.csign;
  Acc<T> acc;
  gemm_dense<T>(0, s, la, lb, smem, acc);
  acc_to_lds<T>(acc, smem);
  lds_barrier();
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = e & 63, k = e >> 6;
    const int ig = i0 + i, kg = k0 + k;
    if (ig < c && kg < c && ig >= kg) {
      const int64_t addr = gp(pl.kcol)[rp + kg] + gp(pl.posarr)[gp(pl.kpos)[rp + kg] + ig];
      atomic_sub(Pl + addr, lds_get<T>(smem, i, k));
    }
  }
}

__global__ void k_fac_init(unsigned long long *ferr, int64_t batch) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < batch) ferr[i] = ~0ull;
}

// log det B = sum_j log D_jj per matrix: the sum of the principal logarithms
// of the pivots (real part log |d|, imaginary part arg d; pi per negative
// pivot of a real matrix), reduced in a fixed order.
template <typename T>
__global__ void __launch_bounds__(NT) k_fac_logdet(const DevPlan *__restrict__ plp, const T *Pall, double *out) {
  const DevPlan &pl = *plp;
  __shared__ double sr[NT], si[NT];
  const int64_t l = blockIdx.x;
  const T *P = Pall + l * pl.panel_elems;
  double re = 0.0, im = 0.0;
  for (int64_t j = threadIdx.x; j < pl.n; j += NT) {
    const T d = P[gp(pl.dpos)[j]];
    if constexpr (Planes<T>::P == 1) {
      re += log(fabs(d));
      if (d < 0) im += M_PI;
    } else {
      re += log(hypot(d.re, d.im));
      im += atan2(d.im, d.re);
    }
  }
  sr[threadIdx.x] = re;
  si[threadIdx.x] = im;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sr[threadIdx.x] += sr[threadIdx.x + h];
      si[threadIdx.x] += si[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * l] = sr[0];
    out[2 * l + 1] = si[0];
  }
}

template <typename T>
hipError_t factor_impl(const DevPlan &pl, const DevPlan *dpl, const FactorAux &fa, const void *values, void *panels,
                       hipStream_t st) {
  T *P = reinterpret_cast<T *>(panels);
  hipError_t e = launch_scatter(pl, dpl, sizeof(T) == 16, values, panels, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fac_init, dim3((unsigned)((pl.batch + 255) / 256)), dim3(256), 0, st, pl.ferr, pl.batch);
  const unsigned B = (unsigned)pl.batch;
  for (int q = 0; q < fa.nlev; ++q) {
    const FacLevel &lv = fa.lev[q];
    if (lv.nodes_n > 0)
      hipLaunchKernelGGL(k_fac_diag<T>, dim3(lv.nodes_n * B), dim3(NT), 0, st, dpl, P, fa.nodes + lv.nodes_b,
                         lv.nodes_n, pl.ferr);
    if (lv.narrow_n > 0) {
      e = launch_linv(pl, dpl, sizeof(T) == 16, panels, fa.chunks_narrow + lv.narrow_b, lv.narrow_n, true, st);
      if (e != hipSuccess) return e;
    }
    if (lv.wide_n > 0) {
      e = launch_linv(pl, dpl, sizeof(T) == 16, panels, fa.chunks_wide + lv.wide_b, lv.wide_n, false, st);
      if (e != hipSuccess) return e;
    }
    if (lv.rb_n > 0)
      hipLaunchKernelGGL(k_fac_lc<T>, dim3(lv.rb_n * B), dim3(NT), 0, st, dpl, P, fa.rblocks + lv.rb_b, lv.rb_n);
    if (lv.tiles_n > 0)
      hipLaunchKernelGGL(k_fac_schur<T>, dim3(lv.tiles_n * B), dim3(NT), 0, st, dpl, P, fa.tiles + lv.tiles_b,
                         lv.tiles_n);
  }
  hipLaunchKernelGGL(k_fac_logdet<T>, dim3(B), dim3(NT), 0, st, dpl, P, pl.fldet);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_factor(const DevPlan &pl, const DevPlan *dpl, const FactorAux &fa, bool cplx_, const void *values,
                         void *panels, hipStream_t st) {
  return cplx_ ? factor_impl<cplx>(pl, dpl, fa, values, panels, st)
               : factor_impl<double>(pl, dpl, fa, values, panels, st);
}

}  // namespace selinv
