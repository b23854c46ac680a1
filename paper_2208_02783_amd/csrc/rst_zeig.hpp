// rst_zeig.hpp -- eigenvalues and right eigenvectors of a small dense complex
// matrix (host code), for the Rayleigh-Ritz step of the eigen route.
//
// Standard dense algorithm (Golub and Van Loan, Matrix Computations, 4th ed.,
// Sec. 7.4-7.6): Householder reduction to upper Hessenberg form, single-shift QR
// iteration with Wilkinson shifts and deflation to the Schur form B = Z T Z^H,
// eigenvectors of the triangular T by back substitution, back-transformed by Z.
// Column-major n x n storage, a[i + j*n].  Sizes of a few hundred at most.
#pragma once
#include <cmath>
#include <complex>
#include <vector>

namespace rst {
namespace zeig {

using cd = std::complex<double>;

// Householder reduction of a (n x n) to upper Hessenberg form; Z accumulates the
// unitary transformations (a_in = Z H Z^H).
inline void hessenberg(int n, std::vector<cd>& a, std::vector<cd>& z) {
  z.assign((size_t)n * n, cd(0.0));
  for (int i = 0; i < n; ++i) z[i + (size_t)i * n] = 1.0;
  std::vector<cd> v(n);
  for (int k = 0; k < n - 2; ++k) {
    double alpha2 = 0.0;
    for (int i = k + 1; i < n; ++i) alpha2 += std::norm(a[i + (size_t)k * n]);
    const double alpha = std::sqrt(alpha2);
    if (alpha == 0.0) continue;
    const cd x0 = a[k + 1 + (size_t)k * n];
    const cd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1.0);
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    v[k + 1] = x0 + ph * alpha;
    for (int i = k + 2; i < n; ++i) v[i] = a[i + (size_t)k * n];
    double vn2 = 0.0;
    for (int i = k + 1; i < n; ++i) vn2 += std::norm(v[i]);
    if (vn2 == 0.0) continue;
    // a = P a P with P = I - 2 v v^H / (v^H v)
    for (int j = 0; j < n; ++j) {  // left: rows k+1..n-1
      cd s = 0.0;
      for (int i = k + 1; i < n; ++i) s += std::conj(v[i]) * a[i + (size_t)j * n];
      s *= 2.0 / vn2;
      for (int i = k + 1; i < n; ++i) a[i + (size_t)j * n] -= v[i] * s;
    }
    for (int i = 0; i < n; ++i) {  // right: columns k+1..n-1
      cd s = 0.0;
      for (int j = k + 1; j < n; ++j) s += a[i + (size_t)j * n] * v[j];
      s *= 2.0 / vn2;
      for (int j = k + 1; j < n; ++j) a[i + (size_t)j * n] -= s * std::conj(v[j]);
    }
    for (int i = 0; i < n; ++i) {  // z = z P
      cd s = 0.0;
      for (int j = k + 1; j < n; ++j) s += z[i + (size_t)j * n] * v[j];
      s *= 2.0 / vn2;
      for (int j = k + 1; j < n; ++j) z[i + (size_t)j * n] -= s * std::conj(v[j]);
    }
    for (int i = k + 2; i < n; ++i) a[i + (size_t)k * n] = 0.0;
  }
}

// Givens rotation (c real, s complex) with [c s; -conj(s) c] [x; y] = [r; 0].
inline void givens(cd x, cd y, double& c, cd& s) {
  const double ax = std::abs(x), ay = std::abs(y);
  if (ay == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  if (ax == 0.0) {
    c = 0.0;
    s = std::conj(y) / ay;
    return;
  }
  const double r = std::hypot(ax, ay);
  c = ax / r;
  s = (x / ax) * std::conj(y) / r;
}

// Schur form of an upper Hessenberg h by shifted QR (Wilkinson shift, deflation
// when a subdiagonal falls below eps times its neighbours); z accumulates.
// Returns false if an eigenvalue needed more than 60 iterations.
inline bool schur(int n, std::vector<cd>& h, std::vector<cd>& z) {
  const double eps = 2.2e-16;
  int hi = n - 1, iter = 0;
  while (hi > 0) {
    // find the active block [lo, hi]
    int lo = hi;
    while (lo > 0) {
      const double sub = std::abs(h[lo + (size_t)(lo - 1) * n]);
      const double dia = std::abs(h[lo - 1 + (size_t)(lo - 1) * n]) + std::abs(h[lo + (size_t)lo * n]);
      if (sub <= eps * (dia > 0 ? dia : 1.0)) {
        h[lo + (size_t)(lo - 1) * n] = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (++iter > 60) return false;
    // Wilkinson shift from the trailing 2 x 2 block (exceptional shift every 10 iterations)
    const cd a = h[hi - 1 + (size_t)(hi - 1) * n], b = h[hi - 1 + (size_t)hi * n];
    const cd cc = h[hi + (size_t)(hi - 1) * n], d = h[hi + (size_t)hi * n];
    const cd tr = a + d, det = a * d - b * cc;
    const cd disc = std::sqrt(tr * tr * 0.25 - det);
    const cd l1 = tr * 0.5 + disc, l2 = tr * 0.5 - disc;
    cd mu = std::abs(l1 - d) < std::abs(l2 - d) ? l1 : l2;
    if (iter % 10 == 0) mu = d + cd(std::abs(h[hi + (size_t)(hi - 1) * n]), 0.0);
    // QR step on the block [lo, hi] with shift mu, as a chase of Givens rotations
    cd x = h[lo + (size_t)lo * n] - mu, y = h[lo + 1 + (size_t)lo * n];
    for (int k = lo; k < hi; ++k) {
      double c;
      cd s;
      givens(x, y, c, s);
      // rows k, k+1 of h (columns from max(lo, k-1) to n-1)
      for (int j = (k > lo ? k - 1 : lo); j < n; ++j) {
        const cd u = h[k + (size_t)j * n], w = h[k + 1 + (size_t)j * n];
        h[k + (size_t)j * n] = c * u + s * w;
        h[k + 1 + (size_t)j * n] = -std::conj(s) * u + c * w;
      }
      // columns k, k+1 of h (rows 0..min(k+2, hi))
      const int imax = k + 2 < hi ? k + 2 : hi;
      for (int i = 0; i <= imax; ++i) {
        const cd u = h[i + (size_t)k * n], w = h[i + (size_t)(k + 1) * n];
        h[i + (size_t)k * n] = c * u + std::conj(s) * w;
        h[i + (size_t)(k + 1) * n] = -s * u + c * w;
      }
      for (int i = 0; i < n; ++i) {
        const cd u = z[i + (size_t)k * n], w = z[i + (size_t)(k + 1) * n];
        z[i + (size_t)k * n] = c * u + std::conj(s) * w;
        z[i + (size_t)(k + 1) * n] = -s * u + c * w;
      }
      if (k < hi - 1) {
        x = h[k + 1 + (size_t)k * n];
        y = h[k + 2 + (size_t)k * n];
      }
    }
  }
  return true;
}

// Eigenvalues w (n) and right eigenvectors v (n x n, unit 2-norm columns) of a
// general complex a (column-major, destroyed).  Returns false on QR failure.
inline bool eig(int n, std::vector<cd> a, std::vector<cd>& w, std::vector<cd>& v) {
  std::vector<cd> z;
  hessenberg(n, a, z);
  if (!schur(n, a, z)) return false;
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = a[i + (size_t)i * n];
  // eigenvectors of the triangular T: (T - t_ii) y = 0 with y_i = 1, y_j = 0 (j > i)
  double tnorm = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= j; ++i) tnorm = std::max(tnorm, std::abs(a[i + (size_t)j * n]));
  const double small = 1e-14 * (tnorm > 0 ? tnorm : 1.0);
  std::vector<cd> y(n);
  v.assign((size_t)n * n, cd(0.0));
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) y[j] = 0.0;
    y[i] = 1.0;
    for (int r = i - 1; r >= 0; --r) {
      cd s = 0.0;
      for (int j = r + 1; j <= i; ++j) s += a[r + (size_t)j * n] * y[j];
      cd d = a[r + (size_t)r * n] - w[i];
      if (std::abs(d) < small) d = small;
      y[r] = -s / d;
    }
    double nrm = 0.0;
    for (int r = 0; r < n; ++r) {
      cd s = 0.0;
      for (int j = 0; j <= i; ++j) s += z[r + (size_t)j * n] * y[j];
      v[r + (size_t)i * n] = s;
      nrm += std::norm(s);
    }
    nrm = std::sqrt(nrm);
    for (int r = 0; r < n; ++r) v[r + (size_t)i * n] /= nrm;
  }
  return true;
}

}  // namespace zeig
}  // namespace rst
