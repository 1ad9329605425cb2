// The optimal window of image domain gridding (§4.3, Appendix A) and the rms
// window the master-grid image is divided by (Algorithms 1 and 2, "inverse rms
// taper").  Host code, float64.
//
// Index units: subgrid pixel k at x = k, the imaged field [0, L), side lobes
// x < 0 and x >= L.  A sample shifted by s uv pixels from its subgrid centre
// sees the window f(x, s) = sum_k a_k sinc(x - k) exp(2 pi i (k - x) s / L);
// the cost is its side-lobe energy averaged over |s| <= h:
//   eps^2 = a^T (Qbar o Sbar) a,
//   Qbar_kl = (int_{-inf}^0 + int_L^inf) sinc(x - k) sinc(x - l) dx,
//   Sbar_kl = sinc(2 h (k - l) / L).
// Table 1 is computed with h = (L - beta + 1)/2; the plans of idg_plan keep
// every sample within (L - 1 - beta)/2 of its subgrid centre.
// Qbar in closed form: for k != l the partial fractions of
// sin^2(pi x) / ((x - k)(x - l)) integrate to G(y) = (ln|y| - Ci(2 pi |y|))/2
// (G(0) = -(gamma + ln 2 pi)/2); for k == l the tails of sinc^2 give
// 1 - (Si(2 pi k) + Si(2 pi (L - k)))/pi.  Si and Ci are needed only at
// x = 2 pi m, m = 1 .. L, where the continued fraction of the exponential
// integral E1(i x) converges in a few dozen terms: E1(ix) = -Ci(x) + i (Si(x) - pi/2).
// The smallest eigenpair of the L x L symmetric matrix comes from cyclic
// Jacobi rotations.
#include "taper.h"

#include <cmath>
#include <complex>
#include <vector>

namespace idg {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;

// E1(z) for Re z >= 0, |z| >= 2: e^{-z} / (z + 1 - 1/(z + 3 - 4/(z + 5 - 9/(z + 7 - ...)))),
// evaluated front to back with the modified Lentz scheme.
std::complex<double> expint_e1_cf(std::complex<double> z) {
  const double tiny = 1e-300;
  std::complex<double> f = z + 1.0, C = f, D = 0.0;
  for (int n = 1; n < 100000; ++n) {
    const double an = -double(n) * double(n);
    const std::complex<double> bn = z + double(2 * n + 1);
    D = bn + an * D;
    if (std::abs(D) == 0.0) D = tiny;
    C = bn + an / C;
    if (std::abs(C) == 0.0) C = tiny;
    D = 1.0 / D;
    const std::complex<double> delta = C * D;
    f *= delta;
    if (std::abs(delta - 1.0) < 1e-16) break;
  }
  return std::exp(-z) / f;
}

// (Si(x), Ci(x)) for x >= 2
void sine_cosine_integrals(double x, double &si, double &ci) {
  const std::complex<double> e = expint_e1_cf(std::complex<double>(0.0, x));
  ci = -e.real();
  si = 0.5 * kPi + e.imag();
}

double sinc(double y) {
  if (y == 0.0) return 1.0;
  const double t = kPi * y;
  return std::sin(t) / t;
}

// Cyclic Jacobi: eigenvalues of the symmetric n x n matrix a (row-major,
// destroyed) into w, eigenvectors into the columns of v.
void jacobi_eigen(std::vector<double> &a, int n, std::vector<double> &w, std::vector<double> &v) {
  v.assign(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) v[size_t(i) * n + i] = 1.0;
  auto A = [&](int i, int j) -> double & { return a[size_t(i) * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += A(i, i) * A(i, i);
      for (int j = i + 1; j < n; ++j) off += A(i, j) * A(i, j);
    }
    if (off <= 1e-34 * diag || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = A(p, q);
        if (apq == 0.0) continue;
        // rotation zeroing a_pq: t = tan(phi) is the smaller root of t^2 + 2 theta t - 1 = 0
        const double theta = (A(q, q) - A(p, p)) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp - s * akq;
          A(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk - s * aqk;
          A(q, k) = s * apk + c * aqk;
        }
        A(p, q) = A(q, p) = 0.0;
        for (int k = 0; k < n; ++k) {
          const double vkp = v[size_t(k) * n + p], vkq = v[size_t(k) * n + q];
          v[size_t(k) * n + p] = c * vkp - s * vkq;
          v[size_t(k) * n + q] = s * vkp + c * vkq;
        }
      }
    }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A(i, i);
}

}  // namespace

std::vector<double> taper_error_matrix(int L, double max_shift) {
  std::vector<double> si(L + 1, 0.0), ci(L + 1, 0.0);
  for (int m = 1; m <= L; ++m) sine_cosine_integrals(2.0 * kPi * m, si[m], ci[m]);
  const double g0 = -0.5 * (kEulerGamma + std::log(2.0 * kPi));
  auto G = [&](int y) { return y == 0 ? g0 : 0.5 * (std::log(double(y)) - ci[y]); };
  const double width = 2.0 * max_shift / double(L);
  std::vector<double> R(size_t(L) * L);
  for (int k = 0; k < L; ++k) {
    for (int l = 0; l < L; ++l) {
      double q;
      if (k == l) {
        q = 1.0 - (si[k] + si[L - k]) / kPi;
      } else {
        const double sgn = ((k + l) & 1) ? -1.0 : 1.0;
        q = sgn / (kPi * kPi * double(k - l)) * ((G(k) - G(l)) - (G(L - k) - G(L - l)));
      }
      R[size_t(k) * L + l] = q * sinc(double(k - l) * width);
    }
  }
  return R;
}

int optimal_taper(int L, double max_shift, double *taper, double *epsilon) {
  std::vector<double> R = taper_error_matrix(L, max_shift), w, V;
  jacobi_eigen(R, L, w, V);
  int i0 = 0;
  double wmax = w[0];
  for (int i = 1; i < L; ++i) {
    if (w[i] < w[i0]) i0 = i;
    wmax = std::fmax(wmax, w[i]);
  }
  const double pivot = V[size_t(L / 2) * L + i0];
  for (int k = 0; k < L; ++k) taper[k] = V[size_t(k) * L + i0] / pivot;
  *epsilon = std::sqrt(std::fmax(w[i0], 0.0));
  // float64 entries carry ~1e-16 absolute error: below this the eigenpair is not resolved
  return w[i0] < kTaperMinEps2 * wmax ? IDG_ERANGE : IDG_OK;
}

void taper_correction(int L, double max_shift, const double *taper, int N, float *corr) {
  const double width = 2.0 * max_shift / double(L);
  std::vector<double> sbar(size_t(L) * L), v(L);
  for (int k = 0; k < L; ++k)
    for (int l = 0; l < L; ++l) sbar[size_t(k) * L + l] = sinc(double(k - l) * width);
  for (int X = 0; X < N; ++X) {
    const double x = double(L) * double(X) / double(N);  // image pixel X in subgrid index units
    for (int k = 0; k < L; ++k) v[k] = taper[k] * sinc(x - double(k));
    double acc = 0.0;
    for (int k = 0; k < L; ++k) {
      double row = 0.0;
      for (int l = 0; l < L; ++l) row += sbar[size_t(k) * L + l] * v[l];
      acc += v[k] * row;
    }
    corr[X] = float(double(L) * std::sqrt(std::fmax(acc, 0.0)));
  }
}

}  // namespace idg
