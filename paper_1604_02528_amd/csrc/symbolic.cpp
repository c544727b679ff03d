// Symbolic analysis (Section 2.1 of the paper; Eq. (newset) for the row sets).
//
// Pipeline: validate A's lower CSC -> lower CSC of B = P A P^T -> column
// elimination tree (Liu's algorithm with path compression) -> column counts
// (row-subtree traversal) -> supernode partition (greedy from the lowest
// column, capped, optional chain relaxation) -> supernodal row sets C(K) (union
// over the supernode's columns of B and over child supernodes) -> panel
// offsets -> canonical ancestor index maps -> maps from A's entries to panel
// positions -> work counts.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>

#include "internal.hpp"

namespace selinv {

namespace {

[[noreturn]] void fail(selinv_status st, const std::string &m, int64_t info0 = -1) {
  Failure f;
  f.status = st;
  f.msg = m;
  f.info0 = info0;
  throw f;
}

}  // namespace

void analyze(Symbolic &S, int64_t n, const int64_t *colptr, const int64_t *rowind, const int64_t *perm,
             int64_t cap, double relax) {
  if (n <= 0) fail(SELINV_EINVAL, "n must be positive");
  if (!colptr || !rowind) fail(SELINV_EINVAL, "null pattern pointer");
  if (cap < 1) fail(SELINV_EINVAL, "max_super must be >= 1");
  if (!(relax >= 0.0) || !(relax < 1.0)) fail(SELINV_EINVAL, "relax must be in [0, 1)");
  S.n = n;
  S.cap = cap;
  S.relax = relax;

  // ---- validate A's lower CSC ------------------------------------------
  if (colptr[0] != 0) fail(SELINV_EPATTERN, "colptr[0] != 0", 0);
  for (int64_t j = 0; j < n; ++j) {
    int64_t lo = colptr[j], hi = colptr[j + 1];
    if (hi <= lo) fail(SELINV_EPATTERN, "empty column (diagonal missing)", j);
    if (rowind[lo] != j) fail(SELINV_EPATTERN, "column does not start with its diagonal entry", j);
    for (int64_t p = lo + 1; p < hi; ++p) {
      if (rowind[p] <= rowind[p - 1]) fail(SELINV_EPATTERN, "rows not strictly increasing", j);
      if (rowind[p] >= n) fail(SELINV_EPATTERN, "row index out of range", j);
    }
  }
  const int64_t nnz = colptr[n];
  S.nnzA = nnz;

  S.perm.resize(n);
  S.iperm.assign(n, -1);
  for (int64_t i = 0; i < n; ++i) {
    int64_t p = perm ? perm[i] : i;
    if (p < 0 || p >= n || S.iperm[p] != -1) fail(SELINV_EPATTERN, "perm is not a permutation", i);
    S.perm[i] = p;
    S.iperm[p] = i;
  }

  // ---- B = P A P^T, lower CSC with rows ascending --------------------------
  std::vector<int64_t> ehi(nnz), elo(nnz);
  S.aflip.assign(nnz, 0);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
      int64_t a = S.iperm[rowind[p]], b = S.iperm[j];
      ehi[p] = std::max(a, b);
      elo[p] = std::min(a, b);
      S.aflip[p] = a < b ? 1 : 0;  // the stored lower entry lands in B's upper triangle
    }
  // bucket by row, then stable placement by column -> rows ascending per column
  std::vector<int64_t> rptr(n + 1, 0), byrow(nnz);
  for (int64_t p = 0; p < nnz; ++p) rptr[ehi[p] + 1]++;
  for (int64_t i = 0; i < n; ++i) rptr[i + 1] += rptr[i];
  {
    std::vector<int64_t> nxt(rptr.begin(), rptr.end() - 1);
    for (int64_t p = 0; p < nnz; ++p) byrow[nxt[ehi[p]]++] = p;
  }
  S.Bcolptr.assign(n + 1, 0);
  for (int64_t p = 0; p < nnz; ++p) S.Bcolptr[elo[p] + 1]++;
  for (int64_t j = 0; j < n; ++j) S.Bcolptr[j + 1] += S.Bcolptr[j];
  S.Browind.resize(nnz);
  S.amap.resize(nnz);
  {
    std::vector<int64_t> nxt(S.Bcolptr.begin(), S.Bcolptr.end() - 1);
    for (int64_t q = 0; q < nnz; ++q) {
      int64_t p = byrow[q];
      int64_t pos = nxt[elo[p]]++;
      S.Browind[pos] = ehi[p];
      S.amap[p] = pos;
    }
  }
  // B's rows: for each row i, the columns j < i with B_ij != 0 (transpose access)
  std::vector<int64_t> &Rptr = rptr;  // rows of B: entries with ehi == i (includes the diagonal)
  std::vector<int64_t> Rcol(nnz);
  for (int64_t q = 0; q < nnz; ++q) Rcol[q] = elo[byrow[q]];

  // ---- column elimination tree (Liu 1990, path compression) --------------
  S.parent.assign(n, -1);
  {
    std::vector<int64_t> anc(n, -1);
    for (int64_t k = 0; k < n; ++k) {
      for (int64_t q = Rptr[k]; q < Rptr[k + 1]; ++q) {
        int64_t i = Rcol[q];
        if (i >= k) continue;
        while (true) {
          int64_t a = anc[i];
          if (a == k) break;
          anc[i] = k;
          if (a == -1) {
            S.parent[i] = k;
            break;
          }
          i = a;
        }
      }
    }
  }

  // ---- column counts: row k of L is the row subtree reached from the
  // nonzeros of row k of B by walking up the etree, stopping at k ------------
  S.colcount.assign(n, 1);
  {
    std::vector<int64_t> mark(n, -1);
    for (int64_t k = 0; k < n; ++k) {
      mark[k] = k;
      for (int64_t q = Rptr[k]; q < Rptr[k + 1]; ++q) {
        int64_t i = Rcol[q];
        while (i < k && mark[i] != k) {
          mark[i] = k;
          S.colcount[i]++;
          i = S.parent[i];
          if (i < 0) fail(SELINV_EPATTERN, "internal: etree walk escaped", k);
        }
      }
    }
  }
  S.nnzL = 0;
  for (int64_t j = 0; j < n; ++j) S.nnzL += S.colcount[j];

  // ---- supernode partition -------------------------------------------------
  // Column j joins the open supernode [f, j-1] iff parent(j-1) = j, the merged
  // supernode has at most `cap` columns, and the merged block holds at most
  // relax * (its entries) structural zeros; relax = 0 is the maximal (capped)
  // supernode of the definition (struct(L_{j-1}) = {j-1} U struct(L_j)).
  auto partition = [&](double rl, std::vector<int64_t> &xs) {
    xs.clear();
    xs.push_back(0);
    int64_t run_cc = S.colcount[0];
    for (int64_t j = 1; j < n; ++j) {
      int64_t f = xs.back();
      int64_t size = j - f + 1;
      bool joins = S.parent[j - 1] == j && size <= cap;
      if (joins) {
        int64_t entries = size * (size + 1) / 2 + size * (S.colcount[j] - 1);
        int64_t zeros = entries - (run_cc + S.colcount[j]);
        joins = (double)zeros <= rl * (double)entries;
      }
      if (!joins) {
        xs.push_back(j);
        run_cc = 0;
      }
      run_cc += S.colcount[j];
    }
    xs.push_back(n);
  };
  partition(relax, S.xsuper);
  const int64_t ns = S.nsuper();
  S.col2super.resize(n);
  for (int64_t K = 0; K < ns; ++K)
    for (int64_t j = S.xsuper[K]; j < S.xsuper[K + 1]; ++j) S.col2super[j] = K;

  // exact-partition work count (the algorithmic flops of the maximal supernodes)
  {
    std::vector<int64_t> xe;
    if (relax == 0.0) xe = S.xsuper; else partition(0.0, xe);
    double fe = 0.0;
    for (size_t K = 0; K + 1 < xe.size(); ++K) {
      double s = (double)(xe[K + 1] - xe[K]);
      double c = (double)(S.colcount[xe[K + 1] - 1] - 1);
      fe += 2.0 * c * c * s + 2.0 * c * s * s;
    }
    S.flops_exact = fe;
  }

  // ---- supernodal row sets C(K) --------------------------------------------
  // rows(K) = (U_{j in K} {i > last(K) : B_ij != 0}) U (U_{children K'} {r in C(K') : r > last(K)})
  S.rowptr.assign(ns + 1, 0);
  S.sparent.assign(ns, -1);
  std::vector<std::vector<int64_t>> kids(ns);
  {
    std::vector<int64_t> mark(n, -1), buf;
    std::vector<std::vector<int64_t>> rows(ns);
    for (int64_t K = 0; K < ns; ++K) {
      const int64_t f = S.xsuper[K], l = S.xsuper[K + 1] - 1;
      buf.clear();
      for (int64_t j = f; j <= l; ++j)
        for (int64_t p = S.Bcolptr[j]; p < S.Bcolptr[j + 1]; ++p) {
          int64_t r = S.Browind[p];
          if (r > l && mark[r] != K) {
            mark[r] = K;
            buf.push_back(r);
          }
        }
      for (int64_t ch : kids[K])
        for (int64_t r : rows[ch])
          if (r > l && mark[r] != K) {
            mark[r] = K;
            buf.push_back(r);
          }
      std::sort(buf.begin(), buf.end());
      if ((int64_t)buf.size() != S.colcount[l] - 1)
        fail(SELINV_EPATTERN, "internal: supernodal structure disagrees with column count", l);
      rows[K] = buf;
      if (!buf.empty()) {
        int64_t P = S.col2super[buf[0]];
        S.sparent[K] = P;
        kids[P].push_back(K);
      }
    }
    for (int64_t K = 0; K < ns; ++K) S.rowptr[K + 1] = (int64_t)rows[K].size();
    for (int64_t K = 0; K < ns; ++K) S.rowptr[K + 1] += S.rowptr[K];
    S.rowind_L.resize(S.rowptr[ns]);
    for (int64_t K = 0; K < ns; ++K)
      std::copy(rows[K].begin(), rows[K].end(), S.rowind_L.begin() + S.rowptr[K]);
  }

  // ---- panel offsets, depth, work ------------------------------------------
  S.panel_off.resize(ns);
  int64_t off = 0;
  double fl = 0.0;
  for (int64_t K = 0; K < ns; ++K) {
    int64_t s = S.width(K), c = S.nrows(K);
    S.panel_off[K] = off;
    // each panel starts on a 16-element (>= 128-byte) boundary, so no cache
    // line is shared by two nodes' panels
    off += ((s + c) * s + kPanelAlign - 1) / kPanelAlign * kPanelAlign;
    fl += 2.0 * (double)c * (double)c * (double)s + 2.0 * (double)c * (double)s * (double)s;
  }
  S.panel_elems = off;
  S.flops = fl;
  S.sdepth.assign(ns, 0);
  S.depth = 0;
  for (int64_t K = ns - 1; K >= 0; --K) {
    int64_t P = S.sparent[K];
    S.sdepth[K] = P < 0 ? 0 : S.sdepth[P] + 1;
    S.depth = std::max(S.depth, S.sdepth[K] + 1);
  }

  // ---- canonical ancestor index maps ---------------------------------------
  // Segment t of K: owner J_t and the positions, inside J_t's panel, of the
  // rows C(K)[start_t:] (rows inside J_t's columns map to r - first(J_t),
  // rows above map to s_J + their index in C(J_t), found by a merge walk).
  S.seg_ptr.assign(ns + 1, 0);
  S.seg_super.clear();
  S.seg_start.clear();
  S.seg_posoff.clear();
  S.posarr.clear();
  for (int64_t K = 0; K < ns; ++K) {
    const int64_t *C = S.rowind_L.data() + S.rowptr[K];
    const int64_t c = S.nrows(K);
    int64_t st = 0;
    while (st < c) {
      const int64_t J = S.col2super[C[st]];
      const int64_t fJ = S.xsuper[J], lJ = S.xsuper[J + 1] - 1, sJ = lJ - fJ + 1;
      const int64_t *CJ = S.rowind_L.data() + S.rowptr[J];
      const int64_t cJ = S.nrows(J);
      S.seg_super.push_back(J);
      S.seg_start.push_back(st);
      S.seg_posoff.push_back((int64_t)S.posarr.size());
      int64_t q = 0;  // merge cursor into C(J)
      for (int64_t i = st; i < c; ++i) {
        int64_t r = C[i];
        if (r <= lJ) {
          S.posarr.push_back((int32_t)(r - fJ));
        } else {
          while (q < cJ && CJ[q] < r) ++q;
          if (q >= cJ || CJ[q] != r) fail(SELINV_EPATTERN, "internal: fill property violated", K);
          S.posarr.push_back((int32_t)(sJ + q));
        }
      }
      int64_t en = st;
      while (en < c && S.col2super[C[en]] == J) ++en;
      st = en;
    }
    S.seg_ptr[K + 1] = (int64_t)S.seg_super.size();
  }
  if (S.posarr.size() > (size_t)INT32_MAX) fail(SELINV_ENOMEM, "ancestor maps exceed int32 indexing");

  // ---- A entry -> panel element ---------------------------------------------
  S.apos.resize(nnz);
  S.apos_diag.resize(nnz);
  for (int64_t p = 0; p < nnz; ++p) {
    int64_t r = ehi[p], cc = elo[p];
    int64_t K = S.col2super[cc];
    int64_t f = S.xsuper[K], l = S.xsuper[K + 1] - 1, s = l - f + 1, c = S.nrows(K);
    int64_t pr;
    if (r <= l) {
      pr = r - f;
    } else {
      const int64_t *C = S.rowind_L.data() + S.rowptr[K];
      const int64_t *it = std::lower_bound(C, C + c, r);
      if (it == C + c || *it != r) fail(SELINV_EPATTERN, "internal: A entry outside the pattern of L", cc);
      pr = s + (it - C);
    }
    S.apos[p] = S.panel_off[K] + (cc - f) * (s + c) + pr;
    S.apos_diag[p] = (r == cc) ? 1 : 0;
  }
}

}  // namespace selinv
