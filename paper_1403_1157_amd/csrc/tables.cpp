// Host-side 1D tables (see tables.hpp).
#include "tables.hpp"

#include <cmath>
#include <cstring>
#include <vector>

namespace {

// Cyclic Jacobi eigenvalue iteration for a small dense symmetric matrix A (n x n,
// row-major, overwritten).  Eigenvalues end up on the diagonal; V holds the
// eigenvectors as columns.
void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double v = A[i * n + j] * A[i * n + j];
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double app = A[p * n + p], aqq = A[q * n + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

// Legendre P_n(t) and P_n'(t) on [-1,1].
void legendre_pm1(int n, double t, double* P, double* dP) {
  P[0] = 1.0;
  dP[0] = 0.0;
  if (n >= 1) {
    P[1] = t;
    dP[1] = 1.0;
  }
  for (int k = 1; k < n; ++k) {
    P[k + 1] = ((2 * k + 1) * t * P[k] - k * P[k - 1]) / (k + 1);
    // differentiate the recurrence
    dP[k + 1] = ((2 * k + 1) * (P[k] + t * dP[k]) - k * dP[k - 1]) / (k + 1);
  }
}

}  // namespace

void gauss_rule01(int q, double* x, double* w) {
  // Jacobi matrix of monic Legendre polynomials: zero diagonal, off-diagonal
  // k / sqrt(4k^2 - 1).  Nodes = eigenvalues, weights = 2 v_0^2.
  std::vector<double> A(q * q, 0.0), V;
  for (int k = 1; k < q; ++k) {
    double b = k / std::sqrt(4.0 * k * k - 1.0);
    A[(k - 1) * q + k] = b;
    A[k * q + k - 1] = b;
  }
  jacobi_eigen(q, A, V);
  std::vector<std::pair<double, double>> nw(q);
  for (int j = 0; j < q; ++j) nw[j] = {A[j * q + j], 2.0 * V[0 * q + j] * V[0 * q + j]};
  for (int a = 0; a < q; ++a)
    for (int b = a + 1; b < q; ++b)
      if (nw[b].first < nw[a].first) std::swap(nw[a], nw[b]);
  double P[16], dP[16];
  for (int j = 0; j < q; ++j) {
    double t = nw[j].first;
    for (int it = 0; it < 3; ++it) {  // Newton polishing on P_q
      legendre_pm1(q, t, P, dP);
      t -= P[q] / dP[q];
    }
    legendre_pm1(q, t, P, dP);
    x[j] = 0.5 * (t + 1.0);
    w[j] = 0.5 * 2.0 / ((1.0 - t * t) * dP[q] * dP[q]);
  }
}

void legendre01(int p, double xi, double* val, double* der) {
  double P[16], dP[16];
  legendre_pm1(p, 2.0 * xi - 1.0, P, dP);
  for (int i = 0; i <= p; ++i) {
    double s = std::sqrt(2.0 * i + 1.0);
    val[i] = s * P[i];
    der[i] = s * 2.0 * dP[i];
  }
}

void build_tables(int p, Tables* t) {
  std::memset(t, 0, sizeof(Tables));
  int q = p + 1;
  gauss_rule01(q, t->x, t->w);
  double v[16], d[16];
  for (int k = 0; k < q; ++k) {
    legendre01(p, t->x[k], v, d);
    for (int i = 0; i < q; ++i) {
      t->B[k][i] = v[i];
      t->Bd[k][i] = d[i];
    }
  }
  for (int s = 0; s < 2; ++s) {
    legendre01(p, (double)s, v, d);
    for (int i = 0; i < q; ++i) {
      t->E[s][i] = v[i];
      t->dE[s][i] = d[i];
    }
  }
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) {
      double acc = 0.0;
      for (int k = 0; k < q; ++k) acc += t->w[k] * t->Bd[k][i] * t->Bd[k][j];
      t->S[i][j] = acc;
    }
  // Lifting on K^-: projecting the jump onto the modes of K^- and taking the trace
  // back on the face multiplies it by sum_i phi_i(1)^2 (orthonormal basis).
  double l = 0.0;
  for (int i = 0; i < q; ++i) l += t->E[1][i] * t->E[1][i];
  t->liftc = l;
  for (int i = 0; i < q; ++i) {
    for (int r = 0; r < q; ++r) {
      double acc = 0.0;
      for (int k = 0; k < q; ++k) acc += t->B[i][k] * t->Bd[r][k];
      t->Dn[r][i] = t->w[i] * acc;
    }
    for (int s = 0; s < 2; ++s) {
      double a0 = 0.0, a1 = 0.0;
      for (int k = 0; k < q; ++k) {
        a0 += t->B[i][k] * t->E[s][k];
        a1 += t->B[i][k] * t->dE[s][k];
      }
      t->Le[s][i] = t->w[i] * a0;
      t->dLe[s][i] = t->w[i] * a1;
    }
  }
}

double spectral_constant_1d(int p, double pen_c, double sym, double wm, double wp) {
  // Bilinear form of the 1D periodic diffusion operator on N = 8 unit cells:
  // sum_K int u'v' - sum_e ({u'}[v] + sym {v'}[u]) + pen [u][v], with the average
  // {w'} = wm w'^- + wp w'^+; its largest singular value (the largest eigenvalue
  // when the form is symmetric).
  Tables t;
  build_tables(p, &t);
  const int q = p + 1, N = 8, n = N * q;
  const double pen = pen_c * t.liftc;
  std::vector<double> K(n * n, 0.0), V;
  for (int c = 0; c < N; ++c)
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) K[(c * q + i) * n + c * q + j] += t.S[i][j];
  for (int c = 0; c < N; ++c) {
    int L = c, R = (c + 1) % N;  // face between cell L (minus side) and R (plus side)
    // jump vector [[phi]] = phi^- (1) - phi^+ (0), average of derivatives
    double jv[2 * CDG2_MAXQ], av[2 * CDG2_MAXQ];
    int idx[2 * CDG2_MAXQ];
    for (int i = 0; i < q; ++i) {
      idx[i] = L * q + i;
      jv[i] = t.E[1][i];
      av[i] = wm * t.dE[1][i];
      idx[q + i] = R * q + i;
      jv[q + i] = -t.E[0][i];
      av[q + i] = wp * t.dE[0][i];
    }
    for (int a = 0; a < 2 * q; ++a)
      for (int b = 0; b < 2 * q; ++b)
        K[idx[a] * n + idx[b]] += -av[b] * jv[a] - sym * jv[b] * av[a] + pen * jv[a] * jv[b];
  }
  if (sym != 1.0) {   // K^T K
    std::vector<double> KK((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += K[k * n + i] * K[k * n + j];
        KK[i * n + j] = acc;
      }
    jacobi_eigen(n, KK, V);
    double mx = 0.0;
    for (int i = 0; i < n; ++i) mx = std::fmax(mx, KK[i * n + i]);
    return std::sqrt(mx);
  }
  jacobi_eigen(n, K, V);
  double mx = 0.0;
  for (int i = 0; i < n; ++i) mx = std::fmax(mx, K[i * n + i]);
  return mx;
}
