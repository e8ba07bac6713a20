// Eigenvalues and eigenvectors of small complex upper Hessenberg matrices
// (host code): the m x m matrices that Arnoldi builds.  Eigenvalues by the
// shifted QR iteration -- each step factors H - s I = Q R with Givens
// rotations and forms R Q + s I, the shift s being the eigenvalue of the
// trailing 2x2 block nearer its last diagonal entry (Wilkinson), with an
// exceptional shift every 11 steps without deflation; a subdiagonal entry
// below eps (|h_kk| + |h_k+1,k+1|) splits the matrix.  Eigenvectors of the
// original matrix by inverse iteration on H - mu I (two solves of the
// Hessenberg system with partial pivoting, from a fixed start).
#pragma once

#include <cmath>
#include <complex>
#include <stdexcept>
#include <vector>

namespace lq {

using cplx = std::complex<double>;

// H: n x n row-major (only the upper Hessenberg part is used); returns the n
// eigenvalues in the order they deflate.
inline std::vector<cplx> hessenberg_eigenvalues(std::vector<cplx> H, int n) {
  auto at = [&](int i, int j) -> cplx& { return H[(size_t)i * n + j]; };
  const double eps = 1e-15;
  std::vector<cplx> eig;
  std::vector<double> cs(n);
  std::vector<cplx> sn(n);
  int hi = n - 1, iter = 0, total = 0;
  while (hi >= 0) {
    if (hi == 0) { eig.push_back(at(0, 0)); break; }
    int l = hi;
    while (l > 0 && std::abs(at(l, l - 1)) > eps * (std::abs(at(l, l)) + std::abs(at(l - 1, l - 1))))
      --l;
    if (l > 0) at(l, l - 1) = 0.0;
    if (l == hi) { eig.push_back(at(hi, hi)); --hi; iter = 0; continue; }
    if (++total > 200 * n) throw std::runtime_error("Hessenberg QR did not converge");
    // shift: the eigenvalue of the trailing 2x2 block nearer h_hi,hi
    const cplx a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
    const cplx half = 0.5 * (a + d);
    const cplx disc = std::sqrt(half * half - (a * d - b * c));
    const cplx m1 = half + disc, m2 = half - disc;
    cplx s = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    if (++iter % 11 == 0) s = d + std::abs(c);   // exceptional shift
    for (int k = l; k <= hi; ++k) at(k, k) -= s;
    // H - s I = Q R: rotation k zeroes (k+1, k) from rows k, k+1
    for (int k = l; k < hi; ++k) {
      const cplx x = at(k, k), y = at(k + 1, k);
      const double ax = std::abs(x), r = std::hypot(ax, std::abs(y));
      double cc;
      cplx ss;
      if (r == 0.0) { cc = 1.0; ss = 0.0; }
      else if (ax == 0.0) { cc = 0.0; ss = std::conj(y) / r; }
      else { cc = ax / r; ss = (x / ax) * std::conj(y) / r; }
      cs[k] = cc;
      sn[k] = ss;
      for (int j = k; j <= hi; ++j) {
        const cplx u = at(k, j), v = at(k + 1, j);
        at(k, j) = cc * u + ss * v;
        at(k + 1, j) = -std::conj(ss) * u + cc * v;
      }
    }
    // R Q: the adjoint rotations from the right, on columns k, k+1
    for (int k = l; k < hi; ++k) {
      const double cc = cs[k];
      const cplx ss = sn[k];
      const int top = k + 2 < hi ? k + 2 : hi;
      for (int i = l; i <= top; ++i) {
        const cplx u = at(i, k), v = at(i, k + 1);
        at(i, k) = cc * u + std::conj(ss) * v;
        at(i, k + 1) = -ss * u + cc * v;
      }
    }
    for (int k = l; k <= hi; ++k) at(k, k) += s;
  }
  return eig;
}

// Solve (H - mu I) y = b for upper Hessenberg H (row-major n x n) by
// Gaussian elimination with partial pivoting between neighbouring rows;
// a vanishing pivot is replaced by eps |H| (inverse iteration wants the
// near-singular solve).
inline std::vector<cplx> hessenberg_solve(const std::vector<cplx>& H, int n, cplx mu,
                                          std::vector<cplx> b) {
  std::vector<cplx> A(H);
  double norm = 0.0;
  for (const cplx& z : A) norm = std::fmax(norm, std::abs(z));
  const double tiny = 1e-14 * (norm > 0.0 ? norm : 1.0);
  auto at = [&](int i, int j) -> cplx& { return A[(size_t)i * n + j]; };
  for (int i = 0; i < n; ++i) at(i, i) -= mu;
  for (int k = 0; k < n - 1; ++k) {
    if (std::abs(at(k + 1, k)) > std::abs(at(k, k))) {
      for (int j = k; j < n; ++j) std::swap(at(k, j), at(k + 1, j));
      std::swap(b[k], b[k + 1]);
    }
    if (std::abs(at(k, k)) < tiny) at(k, k) = tiny;
    const cplx f = at(k + 1, k) / at(k, k);
    for (int j = k; j < n; ++j) at(k + 1, j) -= f * at(k, j);
    b[k + 1] -= f * b[k];
  }
  if (std::abs(at(n - 1, n - 1)) < tiny) at(n - 1, n - 1) = tiny;
  for (int i = n - 1; i >= 0; --i) {
    cplx acc = b[i];
    for (int j = i + 1; j < n; ++j) acc -= at(i, j) * b[j];
    b[i] = acc / at(i, i);
  }
  return b;
}

// Unit eigenvector of H for the eigenvalue mu by two steps of inverse iteration.
inline std::vector<cplx> hessenberg_eigenvector(const std::vector<cplx>& H, int n, cplx mu) {
  std::vector<cplx> y(n, cplx(1.0, 0.0));
  for (int it = 0; it < 2; ++it) {
    y = hessenberg_solve(H, n, mu, y);
    double s = 0.0;
    for (const cplx& z : y) s += std::norm(z);
    s = std::sqrt(s);
    for (cplx& z : y) z /= s;
  }
  return y;
}

}  // namespace lq
