// Dense host-side linear algebra of the surrogate's fits (binary64): the
// symmetric eigen-decomposition of the basis Gram matrices and the Cholesky
// solves of the least-squares normal equations.  Plain C++ with no device
// code, so that it can also be built and checked on its own on the host.
#pragma once

#include <cmath>
#include <cstddef>
#include <vector>

namespace gw {
namespace linalg {

// Symmetric eigen-decomposition in two stages (Golub & Van Loan, Matrix
// Computations, 4th ed., chapter 8): Householder reduction to tridiagonal
// form (section 8.3.1), then the symmetric QR algorithm with implicit
// Wilkinson shifts (section 8.3.3-8.3.5): the trailing unreduced block is
// swept by a chain of Givens rotations that chases the bulge the shift
// introduces down the band, and negligible off-diagonal entries split the
// problem.  a: n x n row-major, overwritten with the eigenvectors as ROWS;
// w: eigenvalues (unsorted).  The accumulated orthogonal factor is kept
// transposed so that every update runs along rows.
inline void sym_eig(std::vector<double>& a, int n, std::vector<double>& w) {
  std::vector<double> d(n), e(n, 0.0), v(n), p(n);
  std::vector<double> Q(size_t(n) * n, 0.0), acc(n);  // Q holds Q^T
  for (int i = 0; i < n; ++i) Q[size_t(i) * n + i] = 1.0;
  auto A = [&](int i, int j) -> double& { return a[size_t(i) * n + j]; };
  for (int k = 0; k < n - 2; ++k) {
    const int m = n - k - 1;
    double nx = 0.0;
    for (int i = 0; i < m; ++i) nx += A(k + 1 + i, k) * A(k + 1 + i, k);
    nx = std::sqrt(nx);
    if (nx == 0.0) { e[k + 1] = 0.0; continue; }
    const double x0 = A(k + 1, k);
    const double alpha = x0 > 0 ? -nx : nx;
    for (int i = 0; i < m; ++i) v[i] = A(k + 1 + i, k);
    v[0] -= alpha;
    double nv = 0.0;
    for (int i = 0; i < m; ++i) nv += v[i] * v[i];
    nv = std::sqrt(nv);
    for (int i = 0; i < m; ++i) v[i] /= nv;
    // p = A22 v ; K = v^T p ; q = p - K v ; A22 -= 2 (v q^T + q v^T)
    for (int i = 0; i < m; ++i) {
      double s = 0.0;
      const double* row = &a[size_t(k + 1 + i) * n + k + 1];
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      p[i] = s;
    }
    double K = 0.0;
    for (int i = 0; i < m; ++i) K += v[i] * p[i];
    for (int i = 0; i < m; ++i) p[i] -= K * v[i];
    for (int i = 0; i < m; ++i) {
      double* row = &a[size_t(k + 1 + i) * n + k + 1];
      const double vi = v[i], pi = p[i];
      for (int j = 0; j < m; ++j) row[j] -= 2.0 * (vi * p[j] + pi * v[j]);
    }
    for (int i = 1; i < m; ++i) { A(k + 1 + i, k) = 0.0; A(k, k + 1 + i) = 0.0; }
    A(k + 1, k) = alpha;
    A(k, k + 1) = alpha;
    // Q^T[k+1:, :] -= 2 v (v^T Q^T[k+1:, :])
    std::fill(acc.begin(), acc.end(), 0.0);
    for (int j = 0; j < m; ++j) {
      const double* qj = &Q[size_t(k + 1 + j) * n];
      const double vj = v[j];
      for (int c = 0; c < n; ++c) acc[c] += vj * qj[c];
    }
    for (int j = 0; j < m; ++j) {
      double* qj = &Q[size_t(k + 1 + j) * n];
      const double vj2 = 2.0 * v[j];
      for (int c = 0; c < n; ++c) qj[c] -= vj2 * acc[c];
    }
  }
  // T = tridiag(dg, od): diagonal dg[0..n-1], off-diagonal od[i] = T(i+1, i)
  std::vector<double>& dg = d;
  std::vector<double>& od = e;
  for (int i = 0; i < n; ++i) dg[i] = A(i, i);
  for (int i = 0; i + 1 < n; ++i) od[i] = A(i + 1, i);
  od[n - 1] = 0.0;
  // Plane rotation of rows/columns (k, k+1) of T, row k' = c row_k + s row_k+1,
  // row k+1' = -s row_k + c row_k+1, and the same on the columns; Q^T's rows
  // k, k+1 take the same combination, so that A = Q T Q^T is kept.
  auto rotate_q = [&](int k, double c, double sn) {
    double* qa = &Q[size_t(k) * n];
    double* qb = &Q[size_t(k + 1) * n];
    for (int j = 0; j < n; ++j) {
      const double x = qa[j], y = qb[j];
      qa[j] = c * x + sn * y;
      qb[j] = c * y - sn * x;
    }
  };
  const double tiny = 1e-15;
  int hi = n - 1;  // T(hi+1.., hi+1..) is already diagonal
  int sweeps = 0;
  while (hi > 0) {
    // deflate: drop negligible couplings, then find the unreduced block [lo, hi]
    for (int i = 0; i < hi; ++i)
      if (std::fabs(od[i]) <= tiny * (std::fabs(dg[i]) + std::fabs(dg[i + 1]))) od[i] = 0.0;
    while (hi > 0 && od[hi - 1] == 0.0) --hi;
    if (hi == 0) break;
    int lo = hi - 1;
    while (lo > 0 && od[lo - 1] != 0.0) --lo;
    if (++sweeps > 60 * n) break;  // no convergence: keep what there is
    // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block nearer its
    // last diagonal entry
    const double half = 0.5 * (dg[hi - 1] - dg[hi]);
    const double b2 = od[hi - 1] * od[hi - 1];
    const double mu = dg[hi] - b2 / (half + std::copysign(std::hypot(half, od[hi - 1]), half));
    // first rotation from the shifted first column, then chase the bulge
    double x = dg[lo] - mu, z = od[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, z);
      const double c = r == 0.0 ? 1.0 : x / r, sn = r == 0.0 ? 0.0 : z / r;
      if (k > lo) od[k - 1] = r;  // the bulge T(k+1, k-1) is annihilated into T(k, k-1)
      const double a0 = dg[k], a1 = dg[k + 1], b = od[k];
      dg[k] = c * c * a0 + 2.0 * c * sn * b + sn * sn * a1;
      dg[k + 1] = sn * sn * a0 - 2.0 * c * sn * b + c * c * a1;
      od[k] = c * sn * (a1 - a0) + (c * c - sn * sn) * b;
      if (k + 1 < hi) {
        // the column rotation moves T(k+2, k+1) partly into T(k+2, k): the new bulge
        x = od[k];
        z = sn * od[k + 1];
        od[k + 1] *= c;
      }
      rotate_q(k, c, sn);
    }
  }
  w = dg;
  a = Q;
}

// Cholesky solve of the SPD system P x = rhs (P n x n, rhs n x ncol), in place.
inline bool chol_solve(std::vector<double>& P, int n, std::vector<double>& rhs, int ncol) {
  for (int j = 0; j < n; ++j) {
    double s = P[j * n + j];
    for (int k = 0; k < j; ++k) s -= P[j * n + k] * P[j * n + k];
    if (s <= 0.0) return false;
    P[j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = P[i * n + j];
      for (int k = 0; k < j; ++k) t -= P[i * n + k] * P[j * n + k];
      P[i * n + j] = t / P[j * n + j];
    }
  }
  for (int c = 0; c < ncol; ++c) {
    for (int i = 0; i < n; ++i) {
      double t = rhs[i * ncol + c];
      for (int k = 0; k < i; ++k) t -= P[i * n + k] * rhs[k * ncol + c];
      rhs[i * ncol + c] = t / P[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = rhs[i * ncol + c];
      for (int k = i + 1; k < n; ++k) t -= P[k * n + i] * rhs[k * ncol + c];
      rhs[i * ncol + c] = t / P[i * n + i];
    }
  }
  return true;
}

}  // namespace linalg
}  // namespace gw
