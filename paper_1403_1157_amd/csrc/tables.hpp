// Host-side 1D tables for the tensor Legendre DG basis on [0,1] and the
// spectral constant of the 1D CDG2 diffusion operator.
#pragma once

#define CDG2_MAXQ 5

// Everything a kernel needs about the 1D basis, passed by value as a kernel
// argument.  Row index q is a Gauss point, column index i a Legendre mode.
struct Tables {
  double B[CDG2_MAXQ][CDG2_MAXQ];   // phi_i(x_q)
  double Bd[CDG2_MAXQ][CDG2_MAXQ];  // d phi_i / d xi (x_q)
  double w[CDG2_MAXQ];              // Gauss weights on [0,1] (sum 1)
  double x[CDG2_MAXQ];              // Gauss points on [0,1]
  double E[2][CDG2_MAXQ];           // phi_i(0), phi_i(1)
  double dE[2][CDG2_MAXQ];          // phi_i'(0), phi_i'(1)
  double S[CDG2_MAXQ][CDG2_MAXQ];   // int_0^1 phi_i' phi_j' (exact)
  double liftc;                     // sum_i phi_i(1)^2
  // Lagrange basis l_i of the Gauss points (nodal form of the same space):
  // l_i = w_i sum_k phi_k(x_i) phi_k, exact because the rule integrates Q_p x Q_p.
  double Dn[CDG2_MAXQ][CDG2_MAXQ];  // l_i'(x_q) (row q, column i)
  double Le[2][CDG2_MAXQ];          // l_i(0), l_i(1)
  double dLe[2][CDG2_MAXQ];         // l_i'(0), l_i'(1)
};

// q-point Gauss-Legendre rule on [0,1] (Golub-Welsch: eigen-decomposition of the
// Jacobi matrix of the Legendre recurrence, then Newton polishing).
void gauss_rule01(int q, double* x, double* w);

// Orthonormal Legendre basis sqrt(2i+1) P_i(2 xi - 1) and its xi-derivative.
void legendre01(int p, double xi, double* val, double* der);

// Build the tables for order p (p+1 <= CDG2_MAXQ).
void build_tables(int p, Tables* t);

// Spectral radius of the 1D periodic CDG2 diffusion operator with a = h = 1 and
// lift factor chi_e (its penalty reduces to chi_e * liftc on Cartesian cells).
double spectral_constant_1d(int p, double pen_c, double sym = 1.0, double wm = 0.5, double wp = 0.5);
