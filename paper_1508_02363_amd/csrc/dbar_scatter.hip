// DS II scattering transforms (Section 6) on top of the iterated solver (Section 5.3).
//
// Reflection coefficient (equation rviah, in the Section 6 convention where k is replaced by k/2 so that k lies on
// the xi grid): r(k) = i h(i conj k), with h the solution of the iterated equation for the potential q at spectral
// parameter k/2.  The shift of that solve is 2i conj(k/2) = i conj k, so h(i conj k) is h at the shift offset and is
// gathered on the device; S and m are not formed.
//
// Reconstruction (equations dbarrecA, dbarrecB, qRec): the same D-bar problem with z and k interchanged and q
// replaced by conj(r).  The xi grid of the forward problem (spacing 1/L) is read as the x grid of a dual problem with
// L' = N/(2 pi L); the dual xi grid (spacing 2 pi L / N) contains every point of the forward x grid, so
// q(z) = i h'(i conj z) with h' solved at spectral parameter z/2 on the dual grid.  Time dependence enters through
// r(k, t) = r(k, 0) exp(-i t Re(k^2)/2) (equation rt in the Section 6 convention).
#include <cmath>
#include <complex>
#include <vector>

#include "dbar_solver.h"

namespace dbar {
namespace {

bool finite_all(const double* p, size_t cnt) {
  for (size_t i = 0; i < cnt; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

bool on_grid(double v, double L) {
  const double m = v * L;
  return std::fabs(m - std::nearbyint(m)) <= 1e-9 * std::max(1.0, std::fabs(m));
}

int reflection_impl(const dbar_grid* grid, const double* q, int64_t nk, const double* k, double tol,
                    const dbar_opts* opts, double* r_out, dbar_info* info) {
  int rc = validate_grid(grid);
  if (rc) return rc;
  if (nk < 1) return fail(DBAR_EINVAL, "nk must be >= 1");
  if (!q || !k || !r_out) return fail(DBAR_EINVAL, "q, k and r_out must not be NULL");
  if (!finite_all(k, 2 * (size_t)nk)) return fail(DBAR_EINVAL, "k contains NaN or Inf");
  for (int64_t j = 0; j < 2 * nk; ++j)
    if (!on_grid(k[j], grid->L))
      return fail(DBAR_EINVAL, "the reflection coefficient is computed on the xi grid: L Re k and L Im k integers");
  dbar_opts o;
  dbar_default_opts(&o);
  if (opts) o = *opts;
  o.method = DBAR_METHOD_ITERATED;
  std::vector<double> kh(2 * (size_t)nk);
  for (size_t j = 0; j < kh.size(); ++j) kh[j] = 0.5 * k[j];
  return solve_impl(grid, q, false, nk, kh.data(), tol, &o, nullptr, nullptr, false, info, nullptr, r_out);
}

}  // namespace
}  // namespace dbar

using namespace dbar;

extern "C" {

int dbar_reflection(const dbar_grid* grid, const double* q, int64_t nk, const double* k, double tol,
                    const dbar_opts* opts, double* r_out, dbar_info* info) {
  return reflection_impl(grid, q, nk, k, tol, opts, r_out, info);
}

int dbar_reconstruct(const dbar_grid* grid, const double* r, double t, double tol, const dbar_opts* opts,
                     double* q_out, dbar_info* info) {
  int rc = validate_grid(grid);
  if (rc) return rc;
  if (!r || !q_out) return fail(DBAR_EINVAL, "r and q_out must not be NULL");
  if (!std::isfinite(t)) return fail(DBAR_EINVAL, "t must be finite");
  const int N = grid->n;
  const size_t n = (size_t)N * N;
  if (!finite_all(r, 2 * n)) return fail(DBAR_EINVAL, "r contains NaN or Inf");
  const double L = grid->L;
  dbar_grid dual{N, grid->M, (double)N / (2.0 * M_PI * L)};
  // potential of the dual problem: conj(r(k, t)) moved from FFT order to the dual x grid (index p -> p + N/2 mod N)
  std::vector<std::complex<double>> P(n);
  auto wave = [N](int p) { return p <= N / 2 ? p : p - N; };
  for (int p2 = 0; p2 < N; ++p2) {
    for (int p1 = 0; p1 < N; ++p1) {
      const double k1 = wave(p1) / L, k2 = wave(p2) / L;
      const double ph = -0.5 * t * (k1 * k1 - k2 * k2);
      const std::complex<double> rv(r[2 * ((size_t)p2 * N + p1)], r[2 * ((size_t)p2 * N + p1) + 1]);
      const int j1 = (p1 + N / 2) % N, j2 = (p2 + N / 2) % N;
      P[(size_t)j2 * N + j1] = std::conj(rv * std::polar(1.0, ph));
    }
  }
  // one solve per point z of the forward x grid, row-major like q_out: z = x_{j1} + i x_{j2}, z L' = j - N/2
  std::vector<double> z(2 * n);
  for (int j2 = 0; j2 < N; ++j2) {
    for (int j1 = 0; j1 < N; ++j1) {
      z[2 * ((size_t)j2 * N + j1)] = (j1 - N / 2) / dual.L;
      z[2 * ((size_t)j2 * N + j1) + 1] = (j2 - N / 2) / dual.L;
    }
  }
  return reflection_impl(&dual, reinterpret_cast<const double*>(P.data()), (int64_t)n, z.data(), tol, opts, q_out,
                         info);
}

}  // extern "C"
