// Reads n and an n x n complex upper Hessenberg matrix (row-major, re im
// pairs) from stdin; prints its eigenvalues (re im per line), then for each
// eigenvalue the residual ||H y - mu y|| of the inverse-iteration eigenvector.
#include <cstdio>
#include "../paper_1312_3265_amd/csrc/hessenberg.h"

int main() {
  int n;
  if (std::scanf("%d", &n) != 1) return 2;
  std::vector<lq::cplx> H((size_t)n * n);
  for (auto& z : H) {
    double re, im;
    if (std::scanf("%lf %lf", &re, &im) != 2) return 2;
    z = lq::cplx(re, im);
  }
  const auto ev = lq::hessenberg_eigenvalues(H, n);
  for (const auto& z : ev) std::printf("%.17g %.17g\n", z.real(), z.imag());
  for (const auto& mu : ev) {
    const auto y = lq::hessenberg_eigenvector(H, n, mu);
    double r = 0.0;
    for (int i = 0; i < n; ++i) {
      lq::cplx acc = -mu * y[i];
      for (int j = 0; j < n; ++j) acc += H[(size_t)i * n + j] * y[j];
      r += std::norm(acc);
    }
    std::printf("%.17g\n", std::sqrt(r));
  }
  return 0;
}
