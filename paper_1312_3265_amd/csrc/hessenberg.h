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

namespace lq {

// Complex Schur decomposition A = Q T Q^H of a general n x n matrix
// (row-major, in place: A becomes T, upper triangular; Q unitary, row-major):
// Householder reduction to Hessenberg form, then the shifted QR iteration of
// hessenberg_eigenvalues with every rotation applied to whole rows and
// columns and accumulated into Q.
inline void schur_decompose(std::vector<cplx>& A, std::vector<cplx>& Q, int n) {
  auto a = [&](int i, int j) -> cplx& { return A[(size_t)i * n + j]; };
  auto q = [&](int i, int j) -> cplx& { return Q[(size_t)i * n + j]; };
  Q.assign((size_t)n * n, cplx(0.0, 0.0));
  for (int i = 0; i < n; ++i) q(i, i) = 1.0;
  // Householder: column k below the subdiagonal
  std::vector<cplx> v(n);
  for (int k = 0; k < n - 2; ++k) {
    double norm2 = 0.0;
    for (int i = k + 1; i < n; ++i) norm2 += std::norm(a(i, k));
    const double alpha = std::sqrt(norm2);
    if (alpha == 0.0) continue;
    const cplx x0 = a(k + 1, k);
    const cplx ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cplx(1.0, 0.0);
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    for (int i = k + 1; i < n; ++i) v[i] = a(i, k);
    v[k + 1] += ph * alpha;
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
    if (vn == 0.0) continue;
    // P = I - 2 v v^H / (v^H v); A <- P A P, Q <- Q P
    for (int j = 0; j < n; ++j) {
      cplx s = 0.0;
      for (int i = k + 1; i < n; ++i) s += std::conj(v[i]) * a(i, j);
      s *= 2.0 / vn;
      for (int i = k + 1; i < n; ++i) a(i, j) -= v[i] * s;
    }
    for (int i = 0; i < n; ++i) {
      cplx s = 0.0;
      for (int j = k + 1; j < n; ++j) s += a(i, j) * v[j];
      s *= 2.0 / vn;
      for (int j = k + 1; j < n; ++j) a(i, j) -= s * std::conj(v[j]);
      cplx t = 0.0;
      for (int j = k + 1; j < n; ++j) t += q(i, j) * v[j];
      t *= 2.0 / vn;
      for (int j = k + 1; j < n; ++j) q(i, j) -= t * std::conj(v[j]);
    }
    for (int i = k + 2; i < n; ++i) a(i, k) = 0.0;
  }
  // shifted QR on the Hessenberg matrix, rotations applied to whole rows and
  // columns and accumulated into Q
  const double eps = 1e-15;
  std::vector<double> cs(n);
  std::vector<cplx> sn(n);
  int hi = n - 1, iter = 0, total = 0;
  while (hi > 0) {
    int l = hi;
    while (l > 0 && std::abs(a(l, l - 1)) > eps * (std::abs(a(l, l)) + std::abs(a(l - 1, l - 1))))
      --l;
    if (l > 0) a(l, l - 1) = 0.0;
    if (l == hi) { --hi; iter = 0; continue; }
    if (++total > 200 * n) throw std::runtime_error("Schur QR did not converge");
    const cplx aa = a(hi - 1, hi - 1), b = a(hi - 1, hi), c = a(hi, hi - 1), d = a(hi, hi);
    const cplx half = 0.5 * (aa + d);
    const cplx disc = std::sqrt(half * half - (aa * d - b * c));
    const cplx m1 = half + disc, m2 = half - disc;
    cplx s = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    if (++iter % 11 == 0) s = d + std::abs(c);
    for (int k = l; k <= hi; ++k) a(k, k) -= s;
    for (int k = l; k < hi; ++k) {
      const cplx x = a(k, k), y = a(k + 1, k);
      const double ax = std::abs(x), r = std::hypot(ax, std::abs(y));
      double cc;
      cplx ss;
      if (r == 0.0) { cc = 1.0; ss = 0.0; }
      else if (ax == 0.0) { cc = 0.0; ss = std::conj(y) / r; }
      else { cc = ax / r; ss = (x / ax) * std::conj(y) / r; }
      cs[k] = cc;
      sn[k] = ss;
      for (int j = k; j < n; ++j) {
        const cplx u = a(k, j), w = a(k + 1, j);
        a(k, j) = cc * u + ss * w;
        a(k + 1, j) = -std::conj(ss) * u + cc * w;
      }
    }
    for (int k = l; k < hi; ++k) {
      const double cc = cs[k];
      const cplx ss = sn[k];
      const int top = k + 2 < hi ? k + 2 : hi;
      for (int i = 0; i <= top; ++i) {
        const cplx u = a(i, k), w = a(i, k + 1);
        a(i, k) = cc * u + std::conj(ss) * w;
        a(i, k + 1) = -ss * u + cc * w;
      }
      for (int i = 0; i < n; ++i) {
        const cplx u = q(i, k), w = q(i, k + 1);
        q(i, k) = cc * u + std::conj(ss) * w;
        q(i, k + 1) = -ss * u + cc * w;
      }
    }
    for (int k = l; k <= hi; ++k) a(k, k) += s;
  }
  for (int i = 1; i < n; ++i)
    for (int j = 0; j < i; ++j) a(i, j) = 0.0;
}

// Reorder a complex Schur form T (row-major, with its Q) so that the
// diagonal entries for which wanted[i] holds come first (their order kept):
// adjacent entries are exchanged by a rotation that maps the second one's
// eigenvector onto the first coordinate (Givens swap).
inline void schur_reorder(std::vector<cplx>& T, std::vector<cplx>& Q, int n,
                          std::vector<char> wanted) {
  auto t = [&](int i, int j) -> cplx& { return T[(size_t)i * n + j]; };
  auto q = [&](int i, int j) -> cplx& { return Q[(size_t)i * n + j]; };
  int next = 0;
  for (int i = 0; i < n; ++i) {
    if (!wanted[i]) continue;
    for (int j = i; j > next; --j) {
      // swap diagonal entries j-1 and j
      const cplx a = t(j - 1, j - 1), b = t(j - 1, j), c = t(j, j);
      // eigenvector of [[a, b], [0, c]] for c: (b, c - a)
      cplx x = b, y = c - a;
      const double r = std::hypot(std::abs(x), std::abs(y));
      if (r == 0.0) { std::swap(wanted[j - 1], wanted[j]); continue; }
      x /= r;
      y /= r;
      // G = [[x, -conj(y)], [y, conj(x)]] (unitary), T <- G^H T G, Q <- Q G
      for (int k = 0; k < n; ++k) {   // rows j-1, j: G^H from the left
        const cplx u = t(j - 1, k), w = t(j, k);
        t(j - 1, k) = std::conj(x) * u + std::conj(y) * w;
        t(j, k) = -y * u + x * w;
      }
      for (int k = 0; k < n; ++k) {   // columns j-1, j: G from the right
        const cplx u = t(k, j - 1), w = t(k, j);
        t(k, j - 1) = u * x + w * y;
        t(k, j) = -u * std::conj(y) + w * std::conj(x);
        const cplx qu = q(k, j - 1), qw = q(k, j);
        q(k, j - 1) = qu * x + qw * y;
        q(k, j) = -qu * std::conj(y) + qw * std::conj(x);
      }
      t(j, j - 1) = 0.0;
      std::swap(wanted[j - 1], wanted[j]);
    }
    ++next;
  }
}

// Unit eigenvector of Q T Q^H for the diagonal entry i of the upper
// triangular T: back substitution in (T - t_ii I) z = 0 with z_i = 1 and
// z_j = 0 beyond i, then y = Q z.
inline std::vector<cplx> schur_eigenvector(const std::vector<cplx>& T, const std::vector<cplx>& Q,
                                           int n, int i) {
  std::vector<cplx> z(n, cplx(0.0, 0.0));
  z[i] = 1.0;
  const cplx lam = T[(size_t)i * n + i];
  double norm = 0.0;
  for (const cplx& v : T) norm = std::fmax(norm, std::abs(v));
  const double tiny = 1e-14 * (norm > 0.0 ? norm : 1.0);
  for (int r = i - 1; r >= 0; --r) {
    cplx acc = 0.0;
    for (int c = r + 1; c <= i; ++c) acc += T[(size_t)r * n + c] * z[c];
    cplx den = T[(size_t)r * n + r] - lam;
    if (std::abs(den) < tiny) den = tiny;
    z[r] = -acc / den;
  }
  std::vector<cplx> y(n, cplx(0.0, 0.0));
  double s = 0.0;
  for (int r = 0; r < n; ++r) {
    for (int c = 0; c <= i; ++c) y[r] += Q[(size_t)r * n + c] * z[c];
    s += std::norm(y[r]);
  }
  s = std::sqrt(s);
  for (cplx& v : y) v /= s;
  return y;
}

}  // namespace lq
