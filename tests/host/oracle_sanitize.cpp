// Sanitizer driver for the oracle (test harness only): built together with
// oracle.cpp under -fsanitize=address,undefined, it runs every entry point on
// small inputs (theta, error-bound, periodic and background-subtracted lists,
// both softening kernels, the VJPs, the bad-argument paths) so that an
// out-of-bounds access, a leak or undefined behaviour ends the run with a
// sanitizer report.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
int oracle_tree_build(int64_t n, const double* pos, int n_leaf, int n_group, const double* box,
                      void** out);
void oracle_tree_destroy(void* h);
int oracle_tree_counts(void* h, int64_t* out);
int oracle_build_lists(void* h, double theta, int direct_max, int64_t n_sel, const int64_t* sel);
int oracle_build_lists_err(void* h, const double* mass, double tol, int pmax, int direct_max,
                           int64_t n_sel, const int64_t* sel);
int oracle_build_lists_periodic(void* h, double theta, int direct_max, int64_t n_sel,
                                const int64_t* sel);
int oracle_build_lists_periodic_bs(void* h, double theta, int direct_max, int width,
                                   int64_t n_sel, const int64_t* sel);
int oracle_build_lists_periodic_err(void* h, const double* mass, double tol, int pmax,
                                    int direct_max, int64_t n_sel, const int64_t* sel);
int oracle_compute_moments(void* h, const double* pos, const double* mass, int p, int64_t n_sel,
                           const int64_t* sel);
int oracle_eval_tree(void* h, const double* pos, const double* mass, int kernel, double eps,
                     int64_t n_sinks, const int64_t* sinks, double* acc, double* pot,
                     int64_t* counts, double* absum, double* condsum);
int oracle_tree_vjp(void* h, const double* pos, const double* mass, int kernel, double eps,
                    const double* abar, double* xbar, double* mbar);
int oracle_direct(int64_t n, const double* pos, const double* mass, int kernel, double eps,
                  int64_t n_sinks, const int64_t* sinks, double* acc, double* pot);
int oracle_direct_vjp(int64_t n, const double* pos, const double* mass, int kernel, double eps,
                      const double* abar, int64_t n_rows, const int64_t* rows, double* xbar,
                      double* mbar);
int oracle_ewald_direct(int64_t n, const double* pos, const double* mass, double L, double eps,
                        int64_t n_sinks, const int64_t* sinks, double* acc, double* pot);
}

static int failures = 0;
#define EXPECT(c)                                                  \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "expectation failed line %d: %s\n", __LINE__, #c); \
      ++failures;                                                  \
    }                                                              \
  } while (0)

int main() {
  const int64_t n = 256;
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  std::vector<double> pos(3 * n), mass(n), abar(3 * n);
  for (auto& x : pos) x = U(rng);
  for (int64_t i = 0; i < 20; ++i)  // coincident points
    for (int d = 0; d < 3; ++d) pos[3 * (n - 1 - i) + d] = pos[3 * i + d];
  for (auto& m : mass) m = 1.0 / n;
  for (auto& a : abar) a = U(rng) - 0.5;
  const double box[4] = {0.0, 0.0, 0.0, 1.0};
  std::vector<double> acc(3 * n), pot(n), ab(n), cs(n), xbar(3 * n), mbar(n);
  int64_t counts[16];
  for (int kernel = 0; kernel < 2; ++kernel) {
    for (int mode = 0; mode < 5; ++mode) {
      void* t = nullptr;
      EXPECT(oracle_tree_build(n, pos.data(), 8, 32, box, &t) == 0);
      int rc = -1;
      switch (mode) {
        case 0: rc = oracle_build_lists(t, 0.5, 4, 0, nullptr); break;
        case 1: rc = oracle_build_lists_err(t, mass.data(), 1e-3, 3, 0, 0, nullptr); break;
        case 2: rc = oracle_build_lists_periodic(t, 0.5, 4, 0, nullptr); break;
        case 3: rc = oracle_build_lists_periodic_bs(t, 0.5, 0, 3, 0, nullptr); break;
        case 4: rc = oracle_build_lists_periodic_err(t, mass.data(), 1e-3, 3, 0, 0, nullptr); break;
      }
      EXPECT(rc == 0);
      EXPECT(oracle_compute_moments(t, pos.data(), mass.data(), 3, 0, nullptr) == 0);
      EXPECT(oracle_tree_counts(t, counts) == 0);
      const double eps = 0.01;
      EXPECT(oracle_eval_tree(t, pos.data(), mass.data(), kernel, eps, 0, nullptr, acc.data(),
                              mode == 3 ? nullptr : pot.data(), counts, ab.data(),
                              cs.data()) == 0);
      for (int64_t i = 0; i < 3 * n; ++i) EXPECT(std::isfinite(acc[i]));
      EXPECT(oracle_tree_vjp(t, pos.data(), mass.data(), kernel, eps, abar.data(), xbar.data(),
                             mbar.data()) == 0);
      for (int64_t i = 0; i < 3 * n; ++i) EXPECT(std::isfinite(xbar[i]));
      // moments of a lower order than the error-bound lists need: refused
      if (mode == 1) {
        EXPECT(oracle_compute_moments(t, pos.data(), mass.data(), 2, 0, nullptr) == 0);
        EXPECT(oracle_eval_tree(t, pos.data(), mass.data(), kernel, eps, 0, nullptr, acc.data(),
                                nullptr, counts, nullptr, nullptr) != 0);
      }
      // bad arguments are refused, not read out of bounds
      EXPECT(oracle_eval_tree(t, pos.data(), mass.data(), 7, eps, 0, nullptr, acc.data(), nullptr,
                              counts, nullptr, nullptr) != 0);
      EXPECT(oracle_eval_tree(t, pos.data(), mass.data(), kernel, -1.0, 0, nullptr, acc.data(),
                              nullptr, counts, nullptr, nullptr) != 0);
      oracle_tree_destroy(t);
    }
    const int64_t sinks[3] = {0, 17, n - 1};
    EXPECT(oracle_direct(n, pos.data(), mass.data(), kernel, 0.0, 3, sinks, acc.data(),
                         pot.data()) == 0);
    EXPECT(oracle_direct_vjp(n, pos.data(), mass.data(), kernel, 0.01, abar.data(), 3, sinks,
                             xbar.data(), mbar.data()) == 0);
  }
  EXPECT(oracle_ewald_direct(64, pos.data(), mass.data(), 1.0, 0.01, 0, nullptr, acc.data(),
                             pot.data()) == 0);
  void* t = nullptr;
  EXPECT(oracle_tree_build(0, pos.data(), 8, 32, nullptr, &t) != 0);
  EXPECT(oracle_tree_build(n, pos.data(), 64, 32, nullptr, &t) != 0);
  std::vector<double> bad(pos);
  bad[5] = NAN;
  EXPECT(oracle_tree_build(n, bad.data(), 8, 32, nullptr, &t) != 0);
  const double small_box[4] = {0.0, 0.0, 0.0, 0.5};
  EXPECT(oracle_tree_build(n, pos.data(), 8, 32, small_box, &t) != 0);
  std::printf("sanitized oracle run: %d failed expectations\n", failures);
  return failures ? 1 : 0;
}
