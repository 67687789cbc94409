// Host-side checks of the library's 1D tables (tables.cpp), built by
// tests/test_host_tables.py with AddressSanitizer and UndefinedBehaviorSanitizer.
// Every check compares with a closed form or a printed constant; the process
// prints "OK" and exits 0 when all hold, else names the failing check and exits 1.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "tables.hpp"

static int fails = 0;

static void check(bool ok, const char* what, int p, double got, double want) {
  if (!ok) {
    std::printf("FAIL %s (p=%d): got %.17g want %.17g\n", what, p, got, want);
    ++fails;
  }
}

int main() {
  // Gauss rules on [0,1]: q points integrate x^k exactly for k <= 2q - 1.
  for (int q = 1; q <= CDG2_MAXQ; ++q) {
    double x[CDG2_MAXQ], w[CDG2_MAXQ];
    gauss_rule01(q, x, w);
    for (int k = 0; k <= 2 * q - 1; ++k) {
      double s = 0.0;
      for (int i = 0; i < q; ++i) s += w[i] * std::pow(x[i], k);
      check(std::fabs(s - 1.0 / (k + 1)) < 1e-15, "gauss exactness", q, s, 1.0 / (k + 1));
    }
    for (int i = 0; i < q; ++i) check(x[i] > 0.0 && x[i] < 1.0 && w[i] > 0.0, "gauss points inside", q, x[i], 0.5);
  }
  for (int p = 1; p + 1 <= CDG2_MAXQ; ++p) {
    const int q = p + 1;
    Tables t;
    build_tables(p, &t);
    // orthonormal basis under the rule; phi_0 = 1
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) {
        double s = 0.0;
        for (int k = 0; k < q; ++k) s += t.w[k] * t.B[k][i] * t.B[k][j];
        check(std::fabs(s - (i == j ? 1.0 : 0.0)) < 1e-14, "orthonormality", p, s, i == j);
      }
    // end values: phi_i(1) = sqrt(2i+1), phi_i(0) = (-1)^i sqrt(2i+1); liftc = (p+1)^2
    for (int i = 0; i < q; ++i) {
      const double r = std::sqrt(2.0 * i + 1.0);
      check(std::fabs(t.E[1][i] - r) < 1e-14, "phi(1)", p, t.E[1][i], r);
      check(std::fabs(t.E[0][i] - (i % 2 ? -r : r)) < 1e-14, "phi(0)", p, t.E[0][i], i % 2 ? -r : r);
    }
    check(std::fabs(t.liftc - q * q) < 1e-12, "liftc", p, t.liftc, q * q);
    // stiffness: symmetric, S_00 = 0, S_11 = int (2 sqrt 3)^2 = 12
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) check(std::fabs(t.S[i][j] - t.S[j][i]) < 1e-12, "S symmetric", p, t.S[i][j], t.S[j][i]);
    check(std::fabs(t.S[0][0]) < 1e-14, "S00", p, t.S[0][0], 0.0);
    check(std::fabs(t.S[1][1] - 12.0) < 1e-12, "S11", p, t.S[1][1], 12.0);
    // Lagrange functions of the Gauss points: l_i(x_q) = delta_iq through the
    // modal expansion l_i = w_i sum_k phi_k(x_i) phi_k
    for (int i = 0; i < q; ++i)
      for (int r = 0; r < q; ++r) {
        double s = 0.0;
        for (int k = 0; k < q; ++k) s += t.w[i] * t.B[i][k] * t.B[r][k];
        check(std::fabs(s - (i == r ? 1.0 : 0.0)) < 1e-13, "Lagrange property", p, s, i == r);
      }
    // sum of the Lagrange end values is 1 (partition of unity), derivatives sum to 0
    for (int e = 0; e < 2; ++e) {
      double s = 0.0, d = 0.0;
      for (int i = 0; i < q; ++i) {
        s += t.Le[e][i];
        d += t.dLe[e][i];
      }
      check(std::fabs(s - 1.0) < 1e-13, "sum l_i(end)", p, s, 1.0);
      check(std::fabs(d) < 1e-11, "sum l_i'(end)", p, d, 0.0);
    }
  }
  // spectral constants of the 1D CDG2 form (chi_e = 2: quadrilaterals, 3:
  // hexahedra), to the digits they are printed with
  const double quads[4] = {84.00, 362.06, 1058.74, 2470.93}, hexes[3] = {132.00, 578.04, 1698.46};
  for (int p = 1; p <= 4; ++p) {
    const double r = spectral_constant_1d(p, 2.0);
    check(std::fabs(r - quads[p - 1]) <= 0.005, "rho_hat quads", p, r, quads[p - 1]);
  }
  for (int p = 1; p <= 3; ++p) {
    const double r = spectral_constant_1d(p, 3.0);
    check(std::fabs(r - hexes[p - 1]) <= 0.005, "rho_hat hexes", p, r, hexes[p - 1]);
  }
  if (fails) return 1;
  std::printf("OK\n");
  return 0;
}
