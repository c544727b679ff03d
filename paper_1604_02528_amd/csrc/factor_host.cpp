// Host numeric factorization: unpivoted supernodal LDL^T of B = P A P^T
// (LDL^H for a Hermitian A: every transpose below is then a conjugate
// transpose, Section 2.3), or L D U of an unsymmetric real B with a
// symmetric pattern (the factors of Alg. 1's LU form, Section 2.1): L and
// U^T then fill two panel sets of the same layout, and every update of one
// set takes its other factor from the other set.
//
// The paper takes its factors from an external package that does no dynamic
// pivoting (Section 4); this is the library's own producer of that input.
// Right-looking supernodal form: a supernode is factored once all of its
// children are done; its update L_{C,K} D_K L_{C,K}^T is subtracted from the
// ancestors' panels (positions from the canonical ancestor maps; every target
// lies in the pattern of L by the fill property).  Independent subtrees run
// on separate threads; an ancestor panel is updated under its own mutex.
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "scalar.hpp"

namespace selinv {

namespace {

inline bool finite_nonzero(double d) { return d != 0.0 && std::isfinite(d); }
inline bool finite_nonzero(cplx d) {
  return (d.re != 0.0 || d.im != 0.0) && std::isfinite(d.re) && std::isfinite(d.im);
}

template <typename T>
struct Factorizer {
  const Symbolic &S;
  T *P;  // panels of one matrix
  double cs;  // -1: Hermitian (conjugate transposes), +1 otherwise
  T *PU = nullptr;  // L D U: the U^T panel set (P holds L); null for LDL^T
  std::vector<std::mutex> locks;
  std::atomic<int64_t> bad_col{-1};
  std::atomic<bool> abort{false};

  Factorizer(const Symbolic &s, T *p, double csign) : S(s), P(p), cs(csign), locks(s.nsuper()) {}

  void record_bad(int64_t col) {
    int64_t cur = bad_col.load();
    while ((cur < 0 || col < cur) && !bad_col.compare_exchange_weak(cur, col)) {
    }
    abort.store(true);
  }

  // Dense right-looking L D U of the (s + c) x s panels of both sets in
  // place: B(i, k) -= L(i, j) d_j U(j, k) into the L set and, transposed,
  // B(k, i) into the U^T set, for i >= k.
  bool factor_panel_lu(int64_t K) {
    const int64_t s = S.width(K), c = S.nrows(K), ld = s + c;
    T *A = P + S.panel_off[K], *B = PU + S.panel_off[K];
    for (int64_t jj = 0; jj < s; ++jj) {
      const T d = A[jj + jj * ld];
      if (!finite_nonzero(d)) {
        record_bad(S.xsuper[K] + jj);
        return false;
      }
      T *lj = A + jj * ld, *uj = B + jj * ld;
      for (int64_t k = jj + 1; k < s; ++k) {
        const T fl = SOps<T>::div(uj[k], d), fu = SOps<T>::div(lj[k], d);
        T *lk = A + k * ld, *uk = B + k * ld;
        for (int64_t i = k; i < ld; ++i) {
          lk[i] -= lj[i] * fl;
          uk[i] -= uj[i] * fu;
        }
      }
      for (int64_t i = jj + 1; i < ld; ++i) {
        lj[i] = SOps<T>::div(lj[i], d);
        uj[i] = SOps<T>::div(uj[i], d);
      }
      uj[jj] = d;
    }
    return true;
  }

  // Dense right-looking LDL^T of the (s + c) x s panel in place.
  bool factor_panel(int64_t K) {
    if (PU) return factor_panel_lu(K);
    const int64_t s = S.width(K), c = S.nrows(K), ld = s + c;
    T *A = P + S.panel_off[K];
    for (int64_t jj = 0; jj < s; ++jj) {
      T d = A[jj + jj * ld];
      if (!finite_nonzero(d)) {
        record_bad(S.xsuper[K] + jj);
        return false;
      }
      T *colj = A + jj * ld;
      // trailing update: A[i, k] -= A[i, jj] * tr(A[k, jj] / d) for k in (jj, s),
      // i > k-1 (tr = conj for a Hermitian matrix, where d is real)
      for (int64_t k = jj + 1; k < s; ++k) {
        T f = cj(SOps<T>::div(colj[k], d), cs);
        T *colk = A + k * ld;
        for (int64_t i = k; i < ld; ++i) colk[i] -= colj[i] * f;
      }
      for (int64_t i = jj + 1; i < ld; ++i) colj[i] = SOps<T>::div(colj[i], d);
    }
    return true;
  }

  // Subtract L_{C,K} D_K L_{C,K}^T (^H if Hermitian) from the ancestors (lower
  // triangle only); L D U: L_{C,K} D_K U_{K,C} from the L set and its
  // transpose U_{K,C}^T D_K L_{C,K}^T from the U^T set.
  void update_ancestors(int64_t K, std::vector<T> &W, std::vector<T> &U) {
    if (!PU) {
      update_from(K, P, P, P, W, U);
    } else {
      update_from(K, P, PU, P, W, U);
      update_from(K, PU, P, PU, W, U);
    }
  }

  // Target(a, b) -= sum_k Left_C(a, k) D_k tr(Right_C(b, k)), a >= b, for the
  // rows a, b of C(K), scattered into the ancestors' panels of the set
  // Target; D from the L set's diagonal.
  void update_from(int64_t K, const T *Lset, const T *Rset, T *Tset, std::vector<T> &W, std::vector<T> &U) {
    const int64_t s = S.width(K), c = S.nrows(K), ld = s + c;
    if (c == 0) return;
    const T *A = Rset + S.panel_off[K];
    const T *Al = Lset + S.panel_off[K], *Ad = P + S.panel_off[K];
    const int64_t *C = S.rowind_L.data() + S.rowptr[K];
    // W = Left_C D (c x s, column-major, ld c)
    W.resize((size_t)(c * s));
    for (int64_t k = 0; k < s; ++k) {
      T d = Ad[k + k * ld];
      for (int64_t a = 0; a < c; ++a) W[a + k * c] = Al[s + a + k * ld] * d;
    }
    for (int64_t g = S.seg_ptr[K]; g < S.seg_ptr[K + 1]; ++g) {
      const int64_t J = S.seg_super[g], st = S.seg_start[g];
      const int64_t en = (g + 1 < S.seg_ptr[K + 1]) ? S.seg_start[g + 1] : c;
      const int64_t m = c - st, w = en - st;
      U.assign((size_t)(m * w), SOps<T>::zero());
      // U[a - st, b - st] = sum_k W[a, k] L_C[b, k], a >= b; four columns at a time
      int64_t b = st;
      for (; b + 4 <= en; b += 4) {
        T *u0 = U.data() + (b - st) * m, *u1 = u0 + m, *u2 = u1 + m, *u3 = u2 + m;
        for (int64_t k = 0; k < s; ++k) {
          const T *wk = W.data() + k * c;
          const T *lk = A + s + k * ld;
          T l0 = cj(lk[b], cs), l1 = cj(lk[b + 1], cs), l2 = cj(lk[b + 2], cs), l3 = cj(lk[b + 3], cs);
          for (int64_t a = b; a < c; ++a) {
            T wv = wk[a];
            u0[a - st] += wv * l0;
            u1[a - st] += wv * l1;
            u2[a - st] += wv * l2;
            u3[a - st] += wv * l3;
          }
        }
      }
      for (; b < en; ++b) {
        T *u0 = U.data() + (b - st) * m;
        for (int64_t k = 0; k < s; ++k) {
          const T *wk = W.data() + k * c;
          T l0 = cj(A[s + b + k * ld], cs);
          for (int64_t a = b; a < c; ++a) u0[a - st] += wk[a] * l0;
        }
      }
      // scatter-subtract into J's panel
      const int64_t fJ = S.xsuper[J], sJ = S.width(J), ldJ = sJ + S.nrows(J);
      const int32_t *pos = S.posarr.data() + S.seg_posoff[g];
      T *PJ = Tset + S.panel_off[J];
      std::lock_guard<std::mutex> lk(locks[J]);
      for (int64_t bb = st; bb < en; ++bb) {
        T *col = PJ + (C[bb] - fJ) * ldJ;
        const T *u = U.data() + (bb - st) * m;
        for (int64_t a = bb; a < c; ++a) col[pos[a - st]] -= u[a - st];
      }
    }
  }

  void run(int nthreads) {
    const int64_t ns = S.nsuper();
    std::vector<int64_t> pending(ns, 0);
    for (int64_t K = 0; K < ns; ++K)
      if (S.sparent[K] >= 0) pending[S.sparent[K]]++;
    std::deque<int64_t> ready;
    for (int64_t K = 0; K < ns; ++K)
      if (pending[K] == 0) ready.push_back(K);
    std::mutex qm;
    std::condition_variable cv;
    int64_t ndone = 0;
    auto worker = [&]() {
      std::vector<T> W, U;
      while (true) {
        int64_t K;
        {
          std::unique_lock<std::mutex> lk(qm);
          cv.wait(lk, [&] { return !ready.empty() || ndone == ns || abort.load(); });
          if (abort.load() || (ready.empty() && ndone == ns)) return;
          K = ready.front();
          ready.pop_front();
        }
        if (factor_panel(K)) update_ancestors(K, W, U);
        {
          std::lock_guard<std::mutex> lk(qm);
          ndone++;
          int64_t Pn = S.sparent[K];
          if (Pn >= 0 && --pending[Pn] == 0) ready.push_back(Pn);
        }
        cv.notify_all();
      }
    };
    int nt = nthreads > 0 ? nthreads : (int)std::thread::hardware_concurrency();
    if (nt < 1) nt = 1;
    if (nt > 64) nt = 64;
    std::vector<std::thread> th;
    for (int i = 0; i < nt; ++i) th.emplace_back(worker);
    for (auto &t : th) t.join();
  }
};

template <typename T>
int64_t factor_impl(const Symbolic &S, const double *vals, double *panels_raw, int nthreads, double logdet[2],
                    double cs, bool lu) {
  T *P = reinterpret_cast<T *>(panels_raw);
  const T *v = reinterpret_cast<const T *>(vals);
  T *PU = lu ? P + S.panel_elems : nullptr;
  std::memset((void *)P, 0, sizeof(T) * (size_t)S.panel_elems * (lu ? 2 : 1));
  if (lu) {
    // v[e] = A(row, col), v[nnz + e] = A(col, row); an entry that the
    // permutation moves into B's upper triangle swaps the two roles
    for (int64_t e = 0; e < S.nnzA; ++e) {
      const T lo = v[e], up = v[S.nnzA + e];
      P[S.apos[e]] = S.aflip[e] ? up : lo;
      PU[S.apos[e]] = S.aflip[e] ? lo : up;
    }
  } else {
    // an entry that the permutation moves into B's upper triangle is B's lower
    // entry transposed (conjugated if Hermitian)
    for (int64_t e = 0; e < S.nnzA; ++e) P[S.apos[e]] = S.aflip[e] ? cj(v[e], cs) : v[e];
  }
  Factorizer<T> F(S, P, cs);
  F.PU = PU;
  F.run(nthreads);
  if (F.abort.load()) return F.bad_col.load();
  // log det = sum log D_jj
  double lr = 0.0, li = 0.0;
  for (int64_t K = 0; K < S.nsuper(); ++K) {
    const int64_t s = S.width(K), ld = s + S.nrows(K);
    const T *A = P + S.panel_off[K];
    for (int64_t j = 0; j < s; ++j) {
      if constexpr (std::is_same<T, double>::value) {
        double d = A[j + j * ld];
        lr += std::log(std::fabs(d));
        if (d < 0) li += M_PI;
      } else {
        cplx d = A[j + j * ld];
        lr += std::log(std::hypot(d.re, d.im));
        li += std::atan2(d.im, d.re);
      }
    }
  }
  logdet[0] = lr;
  logdet[1] = li;
  return -1;
}

}  // namespace

int64_t factor_host(const Symbolic &S, int kind, const double *vals, double *panels, int nthreads,
                    double logdet[2]) {
  if (kind == SELINV_R64 || kind == SELINV_LU64)
    return factor_impl<double>(S, vals, panels, nthreads, logdet, 1.0, kind == SELINV_LU64);
  return factor_impl<cplx>(S, vals, panels, nthreads, logdet, kind == SELINV_H128 ? -1.0 : 1.0, false);
}

}  // namespace selinv
