// Host-side driver for the sanitizer build of the library's host code
// (symbolic analysis, host factorization, plan construction, tune tables,
// the C ABI's host entry points).  Built by tests/test_host_sanitizers.py with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host code only; the
// device launchers are replaced by stubs below, and no HIP runtime call is
// reached.  Exits non-zero on a wrong status; the sanitizers abort on their
// own findings.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include <hip/hip_runtime.h>

#include "plan.hpp"
#include "selinv.h"

namespace selinv {
// stubs of the device launchers (kernels.hip, adjoint.hip, factor.hip)
hipError_t launch_normalize(const DevPlan &, const DevPlan *, const LaunchAux &, bool, const void *, void *, void *,
                            hipStream_t, int, int) { return hipErrorNotSupported; }
hipError_t launch_run(const DevPlan &, const DevPlan *, const LaunchAux &, bool, int, const void *, void *, int64_t, int,
                      hipStream_t, int, int) { return hipErrorNotSupported; }
hipError_t launch_level_range(const DevPlan &, const DevPlan *, const LaunchAux &, bool, const void *, void *,
                              hipStream_t, int, int32_t, int32_t) {
  return hipErrorNotSupported;
}
hipError_t launch_extract(const DevPlan &, const DevPlan *, bool, const void *, void *, hipStream_t) {
  return hipErrorNotSupported;
}
int persistent_blocks_per_cu(bool) { return 1; }
hipError_t launch_backward(const DevPlan &, const DevPlan *, const LaunchAux &, bool, const void *, const void *,
                           const void *, void *, const void *, void *, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_scatter(const DevPlan &, const DevPlan *, bool, const void *, void *, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_factor(const DevPlan &, const DevPlan *, const FactorAux &, bool, const void *, void *, hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace selinv

static int failures = 0;
#define CHECK(cond)                                                           \
  do {                                                                        \
    if (!(cond)) {                                                            \
      std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                             \
    }                                                                         \
  } while (0)

struct Csc {
  int64_t n;
  std::vector<int64_t> colptr, rowind;
  std::vector<double> vals;
};

// random structurally symmetric pattern, strictly diagonally dominant values
static Csc random_matrix(int64_t n, double dens, std::mt19937_64 &rng) {
  std::uniform_real_distribution<double> u(0.0, 1.0);
  Csc a;
  a.n = n;
  a.colptr.assign(n + 1, 0);
  std::vector<std::vector<int64_t>> rows(n);
  std::vector<std::vector<double>> vv(n);
  std::vector<double> absum(n, 0.0);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = j + 1; i < n; ++i)
      if (u(rng) < dens) {
        const double v = u(rng) * 2.0 - 1.0;
        rows[j].push_back(i);
        vv[j].push_back(v);
        absum[i] += std::fabs(v);
        absum[j] += std::fabs(v);
      }
  for (int64_t j = 0; j < n; ++j) {
    a.rowind.push_back(j);
    a.vals.push_back(absum[j] + 1.0);
    for (size_t q = 0; q < rows[j].size(); ++q) {
      a.rowind.push_back(rows[j][q]);
      a.vals.push_back(vv[j][q]);
    }
    a.colptr[j + 1] = (int64_t)a.rowind.size();
  }
  return a;
}

static void exercise(const Csc &a, const std::vector<int64_t> &perm, int cap, double relax, int dtype, int batch,
                     int sched, const char *tune) {
  selinv_opts o;
  selinv_default_opts(&o);
  o.max_super = cap;
  o.relax = relax;
  o.dtype = dtype;
  o.batch = batch;
  o.sched = sched;
  o.nthreads = 2;
  o.tune_cache = tune;
  selinv_ctx *h = nullptr;
  selinv_status st = selinv_analyze(a.n, a.colptr.data(), a.rowind.data(), perm.data(), &o, &h);
  CHECK(st == SELINV_OK);
  if (st != SELINV_OK) {
    std::fprintf(stderr, "analyze: %s\n", selinv_last_error(h));
    selinv_destroy(h);
    return;
  }
  selinv_symbolic_view v;
  CHECK(selinv_symbolic(h, &v) == SELINV_OK);
  selinv_sizes_t sz;
  CHECK(selinv_sizes(h, &sz) == SELINV_OK);
  CHECK(sz.work_bytes > 0 && sz.tables_bytes <= sz.work_bytes);
  const int32_t *it = nullptr;
  int64_t nit = 0;
  CHECK(selinv_items(h, 0, &it, &nit) == SELINV_OK);
  CHECK(selinv_items(h, 1, &it, &nit) == SELINV_OK);
  CHECK(selinv_items(h, 7, &it, &nit) == SELINV_EINVAL);
  CHECK(selinv_check_plan(h) == SELINV_OK);
  const int scal = dtype == SELINV_C128 ? 2 : 1;
  std::vector<double> vals((size_t)batch * a.vals.size() * scal);
  for (int l = 0; l < batch; ++l)
    for (size_t e = 0; e < a.vals.size(); ++e) {
      vals[((size_t)l * a.vals.size() + e) * scal] = a.vals[e] * (1.0 + 0.01 * l);
      if (scal == 2) vals[((size_t)l * a.vals.size() + e) * scal + 1] = 0.05 * a.vals[e];
    }
  std::vector<double> panels((size_t)batch * v.panel_elems * scal);
  CHECK(selinv_factor_host(h, vals.data(), panels.data()) == SELINV_OK);
  std::vector<double> ld((size_t)batch * scal);
  CHECK(selinv_logdet(h, ld.data()) == SELINV_OK);
  for (double x : ld) CHECK(std::isfinite(x));
  // out-of-order and null-argument calls are reported, not dereferenced
  CHECK(selinv_run(h, nullptr, nullptr, nullptr, nullptr) == SELINV_ESTATE);
  CHECK(selinv_backward(h, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == SELINV_ESTATE);
  CHECK(selinv_normalize_run_noalloc(h, nullptr, nullptr, nullptr, nullptr, nullptr) == SELINV_EINVAL);
  // a zero pivot
  vals[0] = 0.0;
  if (perm.empty() || perm[0] == 0) {
    CHECK(selinv_factor_host(h, vals.data(), panels.data()) == SELINV_ESINGULAR);
    CHECK(selinv_error_info(h, 0) == 0 && selinv_error_info(h, 1) == 0);
  }
  selinv_destroy(h);
}

int main(int argc, char **argv) {
  const char *tune = argc > 1 ? argv[1] : nullptr;
  std::mt19937_64 rng(12345);
  for (int t = 0; t < 24; ++t) {
    const int64_t n = 2 + (int64_t)(rng() % 150);
    Csc a = random_matrix(n, 0.02 + 0.2 * (double)(rng() % 100) / 100.0, rng);
    std::vector<int64_t> perm(n);
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    if (t % 2) std::shuffle(perm.begin(), perm.end(), rng);
    exercise(a, perm, 1 + (int)(rng() % 40), (t % 3) * 0.1, t % 4 == 3 ? SELINV_C128 : SELINV_R64, 1 + t % 3,
             t % 2 ? SELINV_SCHED_PERSISTENT : SELINV_SCHED_LEVELS, (t % 5 == 0) ? tune : nullptr);
  }
  // malformed patterns: every one is an error status, never a crash
  Csc a = random_matrix(30, 0.2, rng);
  auto expect_pattern = [&](std::vector<int64_t> cp, std::vector<int64_t> ri, selinv_status want) {
    selinv_ctx *h = nullptr;
    const selinv_status st = selinv_analyze(30, cp.data(), ri.data(), nullptr, nullptr, &h);
    CHECK(st == want);
    selinv_destroy(h);
  };
  {
    auto ri = a.rowind;
    ri[a.colptr[5] + 1] = 30;  // out of range (rows after it then fail ordering or range)
    expect_pattern(a.colptr, ri, SELINV_EPATTERN);
  }
  {
    auto ri = a.rowind;
    ri[a.colptr[7]] = 8;  // diagonal missing
    expect_pattern(a.colptr, ri, SELINV_EPATTERN);
  }
  {
    auto cp = a.colptr;
    cp[0] = 1;
    expect_pattern(cp, a.rowind, SELINV_EPATTERN);
  }
  {
    selinv_ctx *h = nullptr;
    std::vector<int64_t> bad(30, 0);
    CHECK(selinv_analyze(30, a.colptr.data(), a.rowind.data(), bad.data(), nullptr, &h) == SELINV_EPATTERN);
    selinv_destroy(h);
  }
  {
    selinv_ctx *h = nullptr;
    CHECK(selinv_analyze(0, a.colptr.data(), a.rowind.data(), nullptr, nullptr, &h) == SELINV_EINVAL);
    selinv_destroy(h);
  }
  CHECK(selinv_analyze(30, a.colptr.data(), a.rowind.data(), nullptr, nullptr, nullptr) == SELINV_EINVAL);
  std::printf("host sanitizer driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
