// Reads n, an n x n complex matrix (row-major re im pairs) and n flags; prints
// max |A - Q T Q^H|, max |Q^H Q - I|, max |T below the diagonal| after the
// Schur decomposition, the diagonal (re im per line), the same three after
// reordering the flagged diagonal entries to the front, then that diagonal.
#include <cstdio>
#include "../paper_1312_3265_amd/csrc/hessenberg.h"

using lq::cplx;

static void checks(const std::vector<cplx>& A, const std::vector<cplx>& T,
                   const std::vector<cplx>& Q, int n) {
  double e1 = 0, e2 = 0, e3 = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      cplx s = 0.0, u = 0.0;
      for (int k = 0; k < n; ++k)
        for (int l = 0; l < n; ++l) s += Q[i * n + k] * T[k * n + l] * std::conj(Q[j * n + l]);
      for (int k = 0; k < n; ++k) u += std::conj(Q[k * n + i]) * Q[k * n + j];
      e1 = std::fmax(e1, std::abs(s - A[i * n + j]));
      e2 = std::fmax(e2, std::abs(u - (i == j ? 1.0 : 0.0)));
      if (i > j) e3 = std::fmax(e3, std::abs(T[i * n + j]));
    }
  std::printf("%.3e %.3e %.3e\n", e1, e2, e3);
}

int main() {
  int n;
  if (std::scanf("%d", &n) != 1) return 2;
  std::vector<cplx> A((size_t)n * n);
  for (auto& z : A) {
    double re, im;
    if (std::scanf("%lf %lf", &re, &im) != 2) return 2;
    z = cplx(re, im);
  }
  std::vector<char> w(n);
  for (int i = 0; i < n; ++i) {
    int f;
    if (std::scanf("%d", &f) != 1) return 2;
    w[i] = (char)f;
  }
  std::vector<cplx> T = A, Q;
  lq::schur_decompose(T, Q, n);
  checks(A, T, Q, n);
  // flags refer to the diagonal order after the decomposition
  for (int i = 0; i < n; ++i) std::printf("%.17g %.17g\n", T[i * n + i].real(), T[i * n + i].imag());
  lq::schur_reorder(T, Q, n, w);
  checks(A, T, Q, n);
  for (int i = 0; i < n; ++i) std::printf("%.17g %.17g\n", T[i * n + i].real(), T[i * n + i].imag());
  return 0;
}
