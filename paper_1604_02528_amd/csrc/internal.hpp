// Internal declarations shared by the host-side translation units of the
// selected-inversion library (symbolic analysis, host factorization, device
// plan and the C ABI).  Nothing here is exported.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "selinv.h"

namespace selinv {

// Alignment (in elements) of every panel and partial-product block.
constexpr int64_t kPanelAlign = 16;

struct Failure {
  selinv_status status;
  std::string msg;
  int64_t info0 = -1;
  int64_t info1 = -1;
};

// Symbolic data of B = P A P^T (Section 2.1; Eq. (newset) for C(K)).
struct Symbolic {
  int64_t n = 0;
  int64_t nnzA = 0;
  int64_t cap = 256;
  double relax = 0.0;
  std::vector<int64_t> perm, iperm;          // new -> old, old -> new
  std::vector<int64_t> Bcolptr, Browind;      // lower CSC of B
  std::vector<int64_t> amap;                  // A entry -> B entry
  std::vector<int64_t> parent, colcount;      // column etree, nnz per column of L
  std::vector<int64_t> xsuper, col2super, sparent;
  std::vector<int64_t> rowptr, rowind_L;      // C(K)
  std::vector<int64_t> panel_off;             // element offset of K's panel
  int64_t panel_elems = 0;
  std::vector<int64_t> seg_ptr, seg_super, seg_start, seg_posoff;
  std::vector<int32_t> posarr;
  std::vector<int64_t> apos;                  // A entry -> element offset inside one matrix's panels
  std::vector<uint8_t> apos_diag;             // A entry is a diagonal entry
  std::vector<uint8_t> aflip;                 // A entry (r, c) has iperm[r] < iperm[c]: B's lower entry is its
                                              // transpose (conjugated for a Hermitian A)
  std::vector<int64_t> sdepth;                // depth of each supernode (root = 0)
  int64_t depth = 0;
  int64_t nnzL = 0;
  double flops = 0.0, flops_exact = 0.0;      // real-arithmetic counts (x4 applied by the caller for C128)

  int64_t nsuper() const { return (int64_t)xsuper.size() - 1; }
  int64_t width(int64_t K) const { return xsuper[K + 1] - xsuper[K]; }
  int64_t nrows(int64_t K) const { return rowptr[K + 1] - rowptr[K]; }
};

// Tune table (tune.cpp): per node-size bucket, how a supernode's GEMM-1 runs.
struct TuneEntry {
  std::string arch, rocm, dtype;
  int64_t s_max = 0, c_max = 0;
  int dense = -1, ydense = -1, split_min_k = 0;  // -1: not given
  int tile = 0;                                   // 0: not given; 64 or 128
};
struct TuneTable {
  std::vector<TuneEntry> entries;  // those of this target, ROCm version and dtype
  const TuneEntry *find(int64_t s, int64_t c) const;  // smallest bucket holding (s, c), or null
};
const char *tune_arch();
std::string tune_rocm();
TuneTable load_tune_table(const std::string &path, const std::string &dtype);  // throws Failure

// Throws Failure on malformed input.
void analyze(Symbolic &S, int64_t n, const int64_t *colptr, const int64_t *rowind, const int64_t *perm,
             int64_t cap, double relax);

// Host numeric factorization into LDL^T panels (strict lower L_KK, D_K on the
// diagonal, L_{C,K} below).  `vals` points at one matrix's values in A order;
// `panels` receives panel_elems scalars.  Real or complex (interleaved).
// Returns the failing column (>= 0) on a zero / non-finite pivot, else -1.
// logdet receives sum log D_jj (re, im).
// kind: SELINV_R64, SELINV_C128, SELINV_H128 or SELINV_LU64 (2 nnz values:
// the lower ones, then their mirrors; 2 panel_elems panels: L with D on the
// diagonal, then U^T with D on the diagonal)
int64_t factor_host(const Symbolic &S, int kind, const double *vals, double *panels, int nthreads,
                    double logdet[2]);

}  // namespace selinv
