// Host side of the tetrahedral-mesh operator (cdg2_tet_*): reference tables,
// mesh validation and geometry, launches.  Included at the end of cdg2.hip (it
// uses that file's error helpers).
#pragma once

struct cdg2_tet {
  int k = 1, E = 0, nb = 4;
  size_t ndof = 0;
  TetParams hp{};
  TetParams* dprm = nullptr;
  double* geo = nullptr;   // jit, vol, area, nrm, xv (one allocation)
  int* topo = nullptr;     // nbr, nbe, minus, ori
  double* stage[2] = {nullptr, nullptr};
  int* flags = nullptr;
  hipStream_t stream = nullptr;
};

namespace {

constexpr int TET_FACE_VERTS[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
constexpr int TET_PERMS[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

double fact(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

// Fully symmetric rule on the triangle exact for degree 2k (barycentric points,
// weights for the mean): orbits (a, a, 1-2a) of three points and (b, c, 1-b-c) of
// six; k = 1: one 3-orbit; k = 2: two 3-orbits; k = 3: two 3-orbits and one
// 6-orbit.  The orbit parameters and all but the last weight solve the moment
// equations of the monomials l1^i l2^j (i + j <= 2k, mean 2 i! j! / (i+j+2)!)
// by Gauss-Newton from rough starting values; returns the number of points, or
// -1 if the iteration does not reach the equations to rounding level.
int tet_face_rule(int k, double (*bary)[3], double* wts) {
  int norb = k == 1 ? 1 : k == 2 ? 2 : 3;
  const bool six[3] = {false, false, k == 3};
  double x[8];
  int nx;
  if (k == 1) {
    x[0] = 0.17;
    nx = 1;
  } else if (k == 2) {
    x[0] = 0.45;   // a1
    x[1] = 0.22;   // w1
    x[2] = 0.09;   // a2 (w2 closes the sum)
    nx = 3;
  } else {
    x[0] = 0.25;   // a1
    x[1] = 0.12;   // w1
    x[2] = 0.06;   // a2
    x[3] = 0.05;   // w2
    x[4] = 0.05;   // b
    x[5] = 0.31;   // c (w3 closes the sum)
    nx = 6;
  }
  auto build = [&](const double* y, double (*P)[3], double* W) {
    int n = 0, i = 0;
    double used = 0.0;
    for (int o = 0; o < norb; ++o) {
      double pts[6][3];
      int m;
      if (!six[o]) {
        const double a = y[i++];
        const double t[3][3] = {{a, a, 1 - 2 * a}, {a, 1 - 2 * a, a}, {1 - 2 * a, a, a}};
        for (int r = 0; r < 3; ++r)
          for (int cc = 0; cc < 3; ++cc) pts[r][cc] = t[r][cc];
        m = 3;
      } else {
        const double b = y[i], cv = y[i + 1];
        i += 2;
        const double v3[3] = {b, cv, 1 - b - cv};
        for (int r = 0; r < 6; ++r)
          for (int cc = 0; cc < 3; ++cc) pts[r][cc] = v3[TET_PERMS[r][cc]];
        m = 6;
      }
      double w;
      if (o < norb - 1) {
        w = y[i++];
        used += m * w;
      } else {
        w = (1.0 - used) / m;
      }
      for (int r = 0; r < m; ++r) {
        for (int cc = 0; cc < 3; ++cc) P[n][cc] = pts[r][cc];
        W[n++] = w;
      }
    }
    return n;
  };
  std::vector<std::pair<int, int>> mons;
  for (int d = 0; d <= 2 * k; ++d)
    for (int i = 0; i <= d; ++i) mons.push_back({i, d - i});
  const int ne = (int)mons.size();
  auto resid = [&](const double* y, double* r) {
    double P[TET_MAXF][3], W[TET_MAXF];
    const int n = build(y, P, W);
    for (int q = 0; q < ne; ++q) {
      double acc = 0.0;
      for (int p = 0; p < n; ++p) acc += W[p] * std::pow(P[p][0], mons[q].first) * std::pow(P[p][1], mons[q].second);
      r[q] = acc - 2.0 * fact(mons[q].first) * fact(mons[q].second) / fact(mons[q].first + mons[q].second + 2);
    }
  };
  std::vector<double> r(ne), rp(ne), rm(ne), Jm(ne * nx);
  bool ok = false;
  for (int it = 0; it < 80; ++it) {
    resid(x, r.data());
    double mx = 0.0;
    for (double v : r) mx = std::fmax(mx, std::fabs(v));
    if (mx < 1e-15) {
      ok = true;
      break;
    }
    for (int j = 0; j < nx; ++j) {
      double xp[8], xm[8];
      std::memcpy(xp, x, sizeof x);
      std::memcpy(xm, x, sizeof x);
      xp[j] += 1e-7;
      xm[j] -= 1e-7;
      resid(xp, rp.data());
      resid(xm, rm.data());
      for (int q = 0; q < ne; ++q) Jm[q * nx + j] = (rp[q] - rm[q]) / 2e-7;
    }
    // normal equations (J^T J) dx = J^T r, Gaussian elimination with pivoting
    double A[8][9] = {};
    for (int a = 0; a < nx; ++a) {
      for (int b = 0; b < nx; ++b)
        for (int q = 0; q < ne; ++q) A[a][b] += Jm[q * nx + a] * Jm[q * nx + b];
      for (int q = 0; q < ne; ++q) A[a][nx] += Jm[q * nx + a] * r[q];
    }
    for (int col = 0; col < nx; ++col) {
      int piv = col;
      for (int row = col + 1; row < nx; ++row)
        if (std::fabs(A[row][col]) > std::fabs(A[piv][col])) piv = row;
      for (int cc = 0; cc <= nx; ++cc) std::swap(A[col][cc], A[piv][cc]);
      for (int row = 0; row < nx; ++row) {
        if (row == col) continue;
        const double fct = A[row][col] / A[col][col];
        for (int cc = col; cc <= nx; ++cc) A[row][cc] -= fct * A[col][cc];
      }
    }
    for (int j = 0; j < nx; ++j) x[j] -= A[j][nx] / A[j][j];
  }
  if (!ok) {
    resid(x, r.data());
    double mx = 0.0;
    for (double v : r) mx = std::fmax(mx, std::fabs(v));
    if (mx > 1e-14) return -1;
  }
  return build(x, bary, wts);
}

// Fully symmetric rule on the tetrahedron exact for degree D = 2k, but D = 5 for
// k = 2 (barycentric points, weights for the mean): orbits of the vertex
// permutations (a, a, a, 1-3a) of 4 points, (b, b, 1/2-b, 1/2-b) of 6,
// (b, b, c, 1-2b-c) of 12; k = 1: one 4-orbit; k = 2: two 4-orbits and a 6-orbit;
// k = 3: three 4-orbits and a 12-orbit.  The orbit parameters and all but the
// last weight solve the moment equations of the monomials l1^a l2^b l3^c
// (a + b + c <= D, mean 6 a! b! c! / (a+b+c+3)!) by Gauss-Newton from rough
// starting values.  Degree 4 leaves the 14-point layout a one-parameter family
// of rules; degree 5 isolates one, so the rule does not depend on the solver.
// Returns the number of points, or -1 if the equations are not met to rounding
// level.
int tet_volume_rule(int k, double (*bary)[4], double* wts) {
  enum { S31, S22, S211 };
  int kinds[4], norb;
  double x[10];
  int nx;
  if (k == 1) {
    norb = 1;
    kinds[0] = S31;
    x[0] = 0.14;
    nx = 1;
  } else if (k == 2) {
    norb = 3;
    kinds[0] = S31;
    kinds[1] = S31;
    kinds[2] = S22;
    const double g[5] = {0.093, 0.073, 0.311, 0.113, 0.045};   // a1, w1, a2, w2, b
    std::memcpy(x, g, sizeof g);
    nx = 5;
  } else {
    norb = 4;
    kinds[0] = S31;
    kinds[1] = S31;
    kinds[2] = S31;
    kinds[3] = S211;
    const double g[8] = {0.215, 0.24, 0.041, 0.06, 0.322, 0.33, 0.064, 0.27};   // a_i, w_i; b, c
    std::memcpy(x, g, sizeof g);
    nx = 8;
  }
  auto build = [&](const double* y, double (*P)[4], double* W) {
    int n = 0, i = 0;
    double used = 0.0;
    for (int o = 0; o < norb; ++o) {
      double base[4];
      if (kinds[o] == S31) {
        const double a = y[i++];
        base[0] = base[1] = base[2] = a;
        base[3] = 1 - 3 * a;
      } else if (kinds[o] == S22) {
        const double b = y[i++];
        base[0] = base[1] = b;
        base[2] = base[3] = 0.5 - b;
      } else {
        const double b = y[i], c = y[i + 1];
        i += 2;
        base[0] = base[1] = b;
        base[2] = c;
        base[3] = 1 - 2 * b - c;
      }
      // the distinct permutations of base
      double pts[24][4];
      int m = 0;
      std::sort(base, base + 4);
      do {
        for (int q = 0; q < 4; ++q) pts[m][q] = base[q];
        ++m;
      } while (std::next_permutation(base, base + 4));
      double w;
      if (o < norb - 1) {
        w = y[i++];
        used += m * w;
      } else {
        w = (1.0 - used) / m;
      }
      for (int r = 0; r < m; ++r) {
        for (int q = 0; q < 4; ++q) P[n][q] = pts[r][q];
        W[n++] = w;
      }
    }
    return n;
  };
  std::vector<std::array<int, 3>> mons;
  const int deg = k == 2 ? 5 : 2 * k;
  for (int d = 0; d <= deg; ++d)
    for (int a = 0; a <= d; ++a)
      for (int b = 0; b <= d - a; ++b) mons.push_back({a, b, d - a - b});
  const int ne = (int)mons.size();
  auto resid = [&](const double* y, double* r) {
    double P[24][4], W[24];
    const int n = build(y, P, W);
    for (int q = 0; q < ne; ++q) {
      double acc = 0.0;
      for (int p = 0; p < n; ++p)
        acc += W[p] * std::pow(P[p][1], mons[q][0]) * std::pow(P[p][2], mons[q][1]) * std::pow(P[p][3], mons[q][2]);
      r[q] = acc - 6.0 * fact(mons[q][0]) * fact(mons[q][1]) * fact(mons[q][2]) /
                       fact(mons[q][0] + mons[q][1] + mons[q][2] + 3);
    }
  };
  std::vector<double> r(ne), rp(ne), rm(ne), Jm((size_t)ne * nx);
  bool ok = false;
  for (int it = 0; it < 100; ++it) {
    resid(x, r.data());
    double mx = 0.0;
    for (double v : r) mx = std::fmax(mx, std::fabs(v));
    if (mx < 1e-15) {
      ok = true;
      break;
    }
    for (int j = 0; j < nx; ++j) {
      double xp[10], xm[10];
      std::memcpy(xp, x, sizeof x);
      std::memcpy(xm, x, sizeof x);
      xp[j] += 1e-7;
      xm[j] -= 1e-7;
      resid(xp, rp.data());
      resid(xm, rm.data());
      for (int q = 0; q < ne; ++q) Jm[(size_t)q * nx + j] = (rp[q] - rm[q]) / 2e-7;
    }
    double A[10][11] = {};
    for (int a = 0; a < nx; ++a) {
      for (int b = 0; b < nx; ++b)
        for (int q = 0; q < ne; ++q) A[a][b] += Jm[(size_t)q * nx + a] * Jm[(size_t)q * nx + b];
      for (int q = 0; q < ne; ++q) A[a][nx] += Jm[(size_t)q * nx + a] * r[q];
    }
    for (int col = 0; col < nx; ++col) {
      int piv = col;
      for (int row = col + 1; row < nx; ++row)
        if (std::fabs(A[row][col]) > std::fabs(A[piv][col])) piv = row;
      for (int cc = 0; cc <= nx; ++cc) std::swap(A[col][cc], A[piv][cc]);
      for (int row = 0; row < nx; ++row) {
        if (row == col) continue;
        const double fct = A[row][col] / A[col][col];
        for (int cc = col; cc <= nx; ++cc) A[row][cc] -= fct * A[col][cc];
      }
    }
    for (int j = 0; j < nx; ++j) x[j] -= A[j][nx] / A[j][j];
  }
  if (!ok) {
    resid(x, r.data());
    double mx = 0.0;
    for (double v : r) mx = std::fmax(mx, std::fabs(v));
    if (mx > 1e-14) return -1;
  }
  return build(x, bary, wts);
}

// Orthonormal basis of P_k on the reference tetrahedron for the mean: modified
// Gram-Schmidt of the monomials xi^a eta^b zeta^c (total degree, then power of
// zeta, then of eta), taken about the centroid (1/4, 1/4, 1/4) -- every prefix
// spans the same space as the plain monomials, with far less cancellation --
// under a collapsed Gauss rule exact for the products; then the values and
// gradients at the points of the symmetric volume rule and of the symmetric face
// rule on each local face.
int build_tet_tables(int k, TetTables* t) {
  std::memset(t, 0, sizeof(TetTables));
  int pw[TET_MAXB][3], nb = 0;
  for (int d = 0; d <= k; ++d)
    for (int cz = 0; cz <= d; ++cz)
      for (int by = 0; by <= d - cz; ++by) {
        pw[nb][0] = d - by - cz;
        pw[nb][1] = by;
        pw[nb][2] = cz;
        ++nb;
      }
  auto ipow = [](double x, int n) {
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
  };
  auto mono = [&](const double* X, double* v, double (*gd)[3]) {
    const double x = X[0] - 0.25, y = X[1] - 0.25, z = X[2] - 0.25;
    for (int m = 0; m < nb; ++m) {
      const int a = pw[m][0], b = pw[m][1], c = pw[m][2];
      v[m] = ipow(x, a) * ipow(y, b) * ipow(z, c);
      gd[m][0] = a ? a * ipow(x, a - 1) * ipow(y, b) * ipow(z, c) : 0.0;
      gd[m][1] = b ? b * ipow(x, a) * ipow(y, b - 1) * ipow(z, c) : 0.0;
      gd[m][2] = c ? c * ipow(x, a) * ipow(y, b) * ipow(z, c - 1) : 0.0;
    }
  };
  // collapsed rule with qu points in u and qv in v, w; weights for the mean (sum 1)
  auto collapsed = [](int qu, int qv, std::vector<std::array<double, 3>>& P, std::vector<double>& W) {
    double xu[CDG2_MAXQ + 8], wu[CDG2_MAXQ + 8], xv[CDG2_MAXQ + 8], wv[CDG2_MAXQ + 8];
    gauss_rule01(qu, xu, wu);
    gauss_rule01(qv, xv, wv);
    P.clear();
    W.clear();
    for (int i = 0; i < qu; ++i)
      for (int j = 0; j < qv; ++j)
        for (int l = 0; l < qv; ++l) {
          P.push_back({xu[i], xv[j] * (1 - xu[i]), xv[l] * (1 - xu[i]) * (1 - xv[j])});
          W.push_back(6.0 * wu[i] * wv[j] * wv[l] * (1 - xu[i]) * (1 - xu[i]) * (1 - xv[j]));
        }
  };
  std::vector<std::array<double, 3>> P;
  std::vector<double> W;
  collapsed(k + 4, k + 3, P, W);
  double G[TET_MAXB][TET_MAXB] = {};
  for (size_t n = 0; n < P.size(); ++n) {
    double v[TET_MAXB], gd[TET_MAXB][3];
    mono(P[n].data(), v, gd);
    for (int a = 0; a < nb; ++a)
      for (int b = 0; b < nb; ++b) G[a][b] += W[n] * v[a] * v[b];
  }
  auto ip = [&](const double* x, const double* y) {
    double r = 0.0;
    for (int a = 0; a < nb; ++a)
      for (int b = 0; b < nb; ++b) r += x[a] * G[a][b] * y[b];
    return r;
  };
  double C[TET_MAXB][TET_MAXB] = {};
  for (int j = 0; j < nb; ++j) {
    double c[TET_MAXB] = {};
    c[j] = 1.0;
    for (int i = 0; i < j; ++i) {
      const double r = ip(C[i], c);
      for (int m = 0; m < nb; ++m) c[m] -= r * C[i][m];
    }
    const double nrm = std::sqrt(ip(c, c));
    for (int m = 0; m < nb; ++m) C[j][m] = c[m] / nrm;
  }
  auto basis = [&](const double* X, double* v, double (*gd)[3]) {
    double mv[TET_MAXB], mg[TET_MAXB][3];
    mono(X, mv, mg);
    for (int j = 0; j < nb; ++j) {
      double a = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0;
      for (int m = 0; m < nb; ++m) {
        a += C[j][m] * mv[m];
        b0 += C[j][m] * mg[m][0];
        b1 += C[j][m] * mg[m][1];
        b2 += C[j][m] * mg[m][2];
      }
      v[j] = a;
      gd[j][0] = b0;
      gd[j][1] = b1;
      gd[j][2] = b2;
    }
  };
  double vb[24][4], vw[24];
  const int nq = tet_volume_rule(k, vb, vw);
  if (nq != TetSz<3>::NQ && nq != TetSz<2>::NQ && nq != TetSz<1>::NQ) return -1;
  for (int q = 0; q < nq; ++q) {
    const double X[3] = {vb[q][1], vb[q][2], vb[q][3]};   // (xi, eta, zeta): coordinates of vertices 1, 2, 3
    double v[TET_MAXB], gd[TET_MAXB][3];
    basis(X, v, gd);
    for (int j = 0; j < nb; ++j) {
      t->Bv[q][j] = v[j];
      for (int a = 0; a < 3; ++a) t->Bg[q][j][a] = gd[j][a];
    }
    t->wv[q] = vw[q];
  }
  double bary[TET_MAXF][3], fw[TET_MAXF];
  const int nf = tet_face_rule(k, bary, fw);
  if (nf != tet_face_points(k)) return -1;
  const double RV[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int p = 0; p < nf; ++p) {
    t->wf[p] = fw[p];
    for (int c3 = 0; c3 < 3; ++c3) t->fbary[p][c3] = bary[p][c3];
  }
  for (int f = 0; f < 4; ++f)
    for (int p = 0; p < nf; ++p) {
      double X[3] = {0, 0, 0};
      for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 3; ++a) X[a] += bary[p][i] * RV[TET_FACE_VERTS[f][i]][a];
      double v[TET_MAXB], gd[TET_MAXB][3];
      basis(X, v, gd);
      for (int j = 0; j < nb; ++j) {
        t->Bf[f][p][j] = v[j];
        t->ftab[f][p][j][0] = v[j];
        for (int a = 0; a < 3; ++a) t->Bgf[f][p][j][a] = t->ftab[f][p][j][a + 1] = gd[j][a];
      }
    }
  // point permutations: under orientation o the neighbour's barycentric coordinates
  // are (l[s0], l[s1], l[s2]) with s = TET_PERMS[o]
  for (int o = 0; o < 6; ++o)
    for (int p = 0; p < nf; ++p) {
      const double want[3] = {bary[p][TET_PERMS[o][0]], bary[p][TET_PERMS[o][1]], bary[p][TET_PERMS[o][2]]};
      int found = -1;
      for (int q = 0; q < nf; ++q)
        if (std::fabs(bary[q][0] - want[0]) + std::fabs(bary[q][1] - want[1]) + std::fabs(bary[q][2] - want[2]) <
            1e-13)
          found = q;
      if (found < 0) return -1;
      t->perm[o][p] = found;
    }
  return 0;
}

void tet_free(cdg2_tet* t) {
  if (t->dprm) (void)hipFree(t->dprm);
  if (t->geo) (void)hipFree(t->geo);
  if (t->topo) (void)hipFree(t->topo);
  for (int i = 0; i < 2; ++i)
    if (t->stage[i]) (void)hipFree(t->stage[i]);
  if (t->flags) (void)hipFree(t->flags);
}

hipError_t tet_launch(cdg2_tet* t, const double* U, const double* U0, double* out, double dt, double ca, double cb,
                      int stage) {
  auto nblk = [&](int eb) { return (t->E + eb - 1) / eb; };
  if (t->k == 1)
    hipLaunchKernelGGL((tet_kernel<1>), dim3(nblk(tet_eb<1>())), dim3(6 * tet_eb<1>()), 0, t->stream, t->dprm, U, U0,
                       out, dt, ca, cb, stage, t->flags);
  else if (t->k == 2)
    hipLaunchKernelGGL((tet_kernel<2>), dim3(nblk(tet_eb<2>())), dim3(6 * tet_eb<2>()), 0, t->stream, t->dprm, U, U0,
                       out, dt, ca, cb, stage, t->flags);
  else
    hipLaunchKernelGGL((tet_kernel<3>), dim3(nblk(tet_eb<3>())), dim3(6 * tet_eb<3>()), 0, t->stream, t->dprm, U, U0,
                       out, dt, ca, cb, stage, t->flags);
  return hipGetLastError();
}

}  // namespace

extern "C" {

int cdg2_tet_create(int order, int n_elements, const double* xyz, const int* vid, const int* nbr, const int* nbe,
                    const cdg2_coeffs* coeffs, double gamma1_in_lo, double gamma1_in_hi, cdg2_tet** out) {
  if (!out || !xyz || !vid || !nbr || !nbe || !coeffs) return fail(CDG2_EINVAL, "NULL argument");
  *out = nullptr;
  if (order < 1 || order > 3) return fail(CDG2_EINVAL, "tetrahedron order must be 1, 2 or 3");
  if (n_elements < 1) return fail(CDG2_EINVAL, "n_elements < 1");
  const int E = n_elements;
  std::vector<int> ori((size_t)E * 4, 0);
  for (int e = 0; e < E; ++e)
    for (int f = 0; f < 4; ++f) {
      const int g = nbr[4 * e + f];
      if (g >= 0) {
        const int gf = nbe[4 * e + f];
        if (g >= E || gf < 0 || gf > 3) return fail(CDG2_EINVAL, "neighbour of element %d face %d out of range", e, f);
        if (nbr[4 * g + gf] != e || nbe[4 * g + gf] != f)
          return fail(CDG2_EINVAL, "neighbour tables not reciprocal at element %d face %d", e, f);
        // orientation: the own face vertex matching each of the neighbour's
        int s[3];
        for (int i2 = 0; i2 < 3; ++i2) {
          const int id = vid[4 * g + TET_FACE_VERTS[gf][i2]];
          s[i2] = -1;
          for (int i = 0; i < 3; ++i)
            if (vid[4 * e + TET_FACE_VERTS[f][i]] == id) s[i2] = i;
          if (s[i2] < 0) return fail(CDG2_EINVAL, "element %d face %d and its neighbour share no such face", e, f);
        }
        int o = -1;
        for (int q = 0; q < 6; ++q)
          if (TET_PERMS[q][0] == s[0] && TET_PERMS[q][1] == s[1] && TET_PERMS[q][2] == s[2]) o = q;
        if (o < 0) return fail(CDG2_EINVAL, "face vertices of element %d face %d repeat", e, f);
        ori[4 * (size_t)e + f] = o;
      } else if (g != -1 && g != -2) {
        return fail(CDG2_EINVAL, "boundary code %d at element %d face %d (allowed: -1, -2)", g, e, f);
      }
    }
  auto* t = new (std::nothrow) cdg2_tet;
  if (!t) return fail(CDG2_ENOMEM, "out of host memory");
  t->k = order;
  t->E = E;
  t->nb = (order + 1) * (order + 2) * (order + 3) / 6;
  t->ndof = (size_t)6 * E * t->nb;
  if (build_tet_tables(order, &t->hp.tb) != 0) {
    delete t;
    return fail(CDG2_EINVAL, "tetrahedron tables could not be built");
  }
  std::vector<double> geo((size_t)E * (9 + 1 + 4 + 12 + 4));
  double* jit = geo.data();
  double* volv = jit + 9 * (size_t)E;
  double* area = volv + E;
  double* nrm = area + 4 * (size_t)E;
  double* xv = nrm + 12 * (size_t)E;
  std::vector<int> topo((size_t)E * 16);
  for (int e = 0; e < E; ++e) {
    const double* v = xyz + 12 * (size_t)e;
    double J[3][3];   // columns v1 - v0, v2 - v0, v3 - v0
    for (int a = 0; a < 3; ++a)
      for (int cidx = 0; cidx < 3; ++cidx) J[a][cidx] = v[3 * (cidx + 1) + a] - v[a];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(det > 0.0)) {
      delete t;
      return fail(CDG2_EINVAL, "element %d is not positively oriented (or degenerate)", e);
    }
    // J^-1 by cofactors; J^-T row-major is jit[3a + b] = (J^-1)[b][a]
    double inv[3][3];
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) jit[9 * (size_t)e + 3 * a + b] = inv[b][a];
    volv[e] = det / 6.0;
    for (int f = 0; f < 4; ++f) {
      const double* A = v + 3 * TET_FACE_VERTS[f][0];
      const double* B = v + 3 * TET_FACE_VERTS[f][1];
      const double* Cc = v + 3 * TET_FACE_VERTS[f][2];
      const double u1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
      const double u2[3] = {Cc[0] - A[0], Cc[1] - A[1], Cc[2] - A[2]};
      double cr[3] = {u1[1] * u2[2] - u1[2] * u2[1], u1[2] * u2[0] - u1[0] * u2[2], u1[0] * u2[1] - u1[1] * u2[0]};
      const double len = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      const double* O = v + 3 * f;   // the opposite vertex
      const double away = (A[0] - O[0]) * cr[0] + (A[1] - O[1]) * cr[1] + (A[2] - O[2]) * cr[2];
      const double sg = away > 0 ? 1.0 : -1.0;
      area[4 * (size_t)e + f] = 0.5 * len;
      for (int a = 0; a < 3; ++a) nrm[12 * (size_t)e + 3 * f + a] = sg * cr[a] / len;
    }
    for (int i = 0; i < 4; ++i) xv[4 * (size_t)e + i] = v[3 * i];
  }
  for (int e = 0; e < E; ++e)
    for (int f = 0; f < 4; ++f) {
      const int g = nbr[4 * e + f];
      topo[4 * (size_t)e + f] = g;
      topo[4 * (size_t)E + 4 * e + f] = g >= 0 ? nbe[4 * e + f] : 0;
      // K^-: the smaller tetrahedron, ties to the lower element index
      topo[8 * (size_t)E + 4 * e + f] = g >= 0 && (volv[e] < volv[g] || (volv[e] == volv[g] && e < g)) ? 1 : 0;
      topo[12 * (size_t)E + 4 * e + f] = ori[4 * (size_t)e + f];
    }
  if (hipMalloc((void**)&t->dprm, sizeof(TetParams)) != hipSuccess ||
      hipMalloc((void**)&t->geo, geo.size() * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&t->topo, topo.size() * sizeof(int)) != hipSuccess ||
      hipMalloc((void**)&t->stage[0], t->ndof * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&t->stage[1], t->ndof * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&t->flags, 64) != hipSuccess) {
    tet_free(t);
    delete t;
    return fail(CDG2_ENOMEM, "hipMalloc for the tetrahedral mesh failed");
  }
  TetGeo& g = t->hp.g;
  g.E = E;
  g.jit = t->geo;
  g.vol = t->geo + 9 * (size_t)E;
  g.area = g.vol + E;
  g.nrm = g.area + 4 * (size_t)E;
  g.xv = g.nrm + 12 * (size_t)E;
  g.nbr = t->topo;
  g.nbe = t->topo + 4 * (size_t)E;
  g.minus = t->topo + 8 * (size_t)E;
  g.ori = t->topo + 12 * (size_t)E;
  g.g1in[0] = gamma1_in_lo;
  g.g1in[1] = gamma1_in_hi;
  std::memcpy(t->hp.cf.c, coeffs, sizeof(double) * K_NCOEFF);
  if (hipMemcpy(t->geo, geo.data(), geo.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t->topo, topo.data(), topo.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t->dprm, &t->hp, sizeof(TetParams), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(t->flags, 0, 64) != hipSuccess) {
    tet_free(t);
    delete t;
    return fail(CDG2_EHIP, "tetrahedral mesh upload failed");
  }
  *out = t;
  return CDG2_OK;
}

int cdg2_tet_destroy(cdg2_tet* t) {
  if (!t) return CDG2_OK;
  tet_free(t);
  delete t;
  return CDG2_OK;
}

int cdg2_tet_set_stream(cdg2_tet* t, void* stream) {
  if (!t) return fail(CDG2_EINVAL, "handle is NULL");
  t->stream = (hipStream_t)stream;
  return CDG2_OK;
}

size_t cdg2_tet_num_dofs(const cdg2_tet* t) { return t ? t->ndof : 0; }

int cdg2_tet_apply_operator(cdg2_tet* t, const double* U, double* F) {
  if (!t || !U || !F) return fail(CDG2_EINVAL, "NULL argument");
  if (overlap(U, F, t->ndof * sizeof(double))) return fail(CDG2_EINVAL, "U and F overlap");
  HIP_TRY(tet_launch(t, U, nullptr, F, 0.0, 0.0, 1.0, 0));
  return CDG2_OK;
}

int cdg2_tet_rk_step(cdg2_tet* t, double* U, double dt, int nsteps) {
  if (!t || !U) return fail(CDG2_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(CDG2_EINVAL, "nsteps < 0");
  if (!std::isfinite(dt)) return fail(CDG2_EINVAL, "dt is not finite");
  const size_t bytes = t->ndof * sizeof(double);
  if (overlap(U, t->stage[0], bytes) || overlap(U, t->stage[1], bytes))
    return fail(CDG2_EINVAL, "U overlaps a stage buffer");
  for (int n = 0; n < nsteps; ++n) {
    HIP_TRY(tet_launch(t, U, nullptr, t->stage[0], dt, 0.0, 1.0, 1));
    HIP_TRY(tet_launch(t, t->stage[0], U, t->stage[1], dt, 0.75, 0.25, 2));
    HIP_TRY(tet_launch(t, t->stage[1], U, U, dt, 1.0 / 3.0, 2.0 / 3.0, 3));
  }
  return CDG2_OK;
}

int cdg2_tet_sync(cdg2_tet* t) {
  if (!t) return fail(CDG2_EINVAL, "handle is NULL");
  HIP_TRY(hipStreamSynchronize(t->stream));
  int f = 0;
  HIP_TRY(hipMemcpy(&f, t->flags, sizeof f, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(t->flags, 0, sizeof(int)));
  if (f & FLAG_NONFINITE) return fail(CDG2_ENONFINITE, "non-finite value written to a state buffer");
  if (f & FLAG_DOMAIN) return fail(CDG2_EDOMAIN, "c + chi^th <= 0 in a chemotactic sensitivity");
  return CDG2_OK;
}

}  // extern "C"
