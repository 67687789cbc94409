// Device-side building blocks shared by the CDG2 kernels: parameter structs,
// compile-time sizes and sum-factorised tensor contractions on gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include "tables.hpp"

namespace cdg2 {

// Species order of the state vector U = (n1, n2, n3, c1, c2, c3).
enum { S_N1 = 0, S_N2 = 1, S_N3 = 2, S_C1 = 3, S_C2 = 4, S_C3 = 5 };

// Coefficient vector (26 entries, order of cdg2_coeffs).
enum {
  K_MU1 = 0, K_MU2, K_MU3, K_NU1, K_NU2, K_NU3,
  K_X011, K_X013, K_X021, K_X022, K_XT11, K_XT13, K_XT21, K_XT22,
  K_D1, K_D2, K_GAM, K_AL1, K_AL2, K_F1, K_K,
  K_BE1, K_BE2, K_SIG, K_C1S, K_C1SS, K_NCOEFF
};

struct Coef {
  double c[K_NCOEFF];
};

// Grid geometry of one instance.
struct Geo {
  int n[3];          // cells per axis
  int E;             // number of cells
  int wall;          // wall axis (-1: fully periodic)
  int llf_cells;     // 1: LLF dissipation on n1, n2 only
  int tz;            // z-planes per slab of the processing order (<= 1: lexicographic)
  double h[3], ih[3];
  double vol;        // |K|
  double area[3];    // |e| of a face normal to each axis
  double g1in[2];    // Gamma_{1,in} on the first tangential axis
  double pen_c;      // penalty factor: stabilisation pen_c (p+1)^2 a / h [[u]] (CDG2: chi_e = N/2)
  double sym;        // sign of the symmetry term {A grad phi}:[[U]] (-1: Baumann-Oden)
  double wm, wp;     // weights of K^- and K^+ in the face average of A grad u.n (and of
                     // the symmetry term): 1/2, 1/2 (central); 1, 0 (CDG: one-sided on K^-)
};

__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

template <int D, int P>
struct Sz {
  static constexpr int Q = P + 1;
  static constexpr int NM = ipow(Q, D);      // modes per species per cell
  static constexpr int NQ = NM;              // volume quadrature points
  static constexpr int NF = ipow(Q, D - 1);  // face points / tangential modes
  static constexpr int NFACE = 2 * D;
};

// Matrix entry M[r][c] (or its transpose) of a CDG2_MAXQ-strided table.
template <bool TR, typename T>
__device__ __forceinline__ T mat(const double (*M)[CDG2_MAXQ], int r, int c) {
  return TR ? T(M[c][r]) : T(M[r][c]);
}

// out[q] = sum_i (Mx (x) My (x) Mz)[q][i] in[i] over Q^D entries, x index fastest;
// TR = true uses the transposed matrices (test integration).  Sum-factorised:
// one 1D contraction per axis, all in registers.
template <int D, int Q, bool TR, typename T>
__device__ __forceinline__ void tapply(const T* in, T* out, const double (*Mx)[CDG2_MAXQ],
                                       const double (*My)[CDG2_MAXQ],
                                       const double (*Mz)[CDG2_MAXQ]) {
  if constexpr (D == 2) {
    T t[Q * Q];
#pragma unroll
    for (int j = 0; j < Q; ++j)
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        T s = T(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) s += mat<TR, T>(Mx, a, i) * in[i + Q * j];
        t[a + Q * j] = s;
      }
#pragma unroll
    for (int b = 0; b < Q; ++b)
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        T s = T(0);
#pragma unroll
        for (int j = 0; j < Q; ++j) s += mat<TR, T>(My, b, j) * t[a + Q * j];
        out[a + Q * b] = s;
      }
  } else {
    T t[Q * Q * Q], u[Q * Q * Q];
#pragma unroll
    for (int k = 0; k < Q; ++k)
#pragma unroll
      for (int j = 0; j < Q; ++j)
#pragma unroll
        for (int a = 0; a < Q; ++a) {
          T s = T(0);
#pragma unroll
          for (int i = 0; i < Q; ++i) s += mat<TR, T>(Mx, a, i) * in[i + Q * (j + Q * k)];
          t[a + Q * (j + Q * k)] = s;
        }
#pragma unroll
    for (int k = 0; k < Q; ++k)
#pragma unroll
      for (int b = 0; b < Q; ++b)
#pragma unroll
        for (int a = 0; a < Q; ++a) {
          T s = T(0);
#pragma unroll
          for (int j = 0; j < Q; ++j) s += mat<TR, T>(My, b, j) * t[a + Q * (j + Q * k)];
          u[a + Q * (b + Q * k)] = s;
        }
#pragma unroll
    for (int c = 0; c < Q; ++c)
#pragma unroll
      for (int b = 0; b < Q; ++b)
#pragma unroll
        for (int a = 0; a < Q; ++a) {
          T s = T(0);
#pragma unroll
          for (int k = 0; k < Q; ++k) s += mat<TR, T>(Mz, c, k) * u[a + Q * (b + Q * k)];
          out[a + Q * (b + Q * c)] = s;
        }
  }
}

// Mode index of (normal index i along axis a, tangential index J); the
// tangential axes are the remaining axes in increasing order, first fastest.
template <int D, int Q>
__device__ __forceinline__ int face_mode(int a, int i, int J) {
  if constexpr (D == 2) {
    return a == 0 ? i + Q * J : J + Q * i;
  } else {
    int j0 = J % Q, j1 = J / Q;
    if (a == 0) return i + Q * (j0 + Q * j1);
    if (a == 1) return j0 + Q * (i + Q * j1);
    return j0 + Q * (j1 + Q * i);
  }
}

// Tangential basis value Phi_J at tangential Gauss point t (both multi-indices
// over the D-1 tangential axes, first fastest).
template <int D, int Q, typename T>
__device__ __forceinline__ T tang_basis(const Tables& tb, int J, int t) {
  if constexpr (D == 2) {
    return T(tb.B[t][J]);
  } else {
    return T(tb.B[t % Q][J % Q]) * T(tb.B[t / Q][J / Q]);
  }
}

template <int D, int Q, typename T>
__device__ __forceinline__ T tang_weight(const Tables& tb, int t) {
  if constexpr (D == 2) {
    return T(tb.w[t]);
  } else {
    return T(tb.w[t % Q]) * T(tb.w[t / Q]);
  }
}

template <int D, int Q, typename T>
__device__ __forceinline__ T vol_weight(const Tables& tb, int qp) {
  if constexpr (D == 2) {
    return T(tb.w[qp % Q]) * T(tb.w[qp / Q]);
  } else {
    return T(tb.w[qp % Q]) * T(tb.w[(qp / Q) % Q]) * T(tb.w[qp / (Q * Q)]);
  }
}

// Index of the neighbour across face f = 2a + sigma (sigma = 1: high side) of
// cell e, or -1 (Gamma1: low end of the wall axis) / -2 (Gamma2: high end).
template <int D>
__device__ __forceinline__ int neighbour(const Geo& g, int e, int f) {
  int c[3];
  c[0] = e % g.n[0];
  c[1] = (e / g.n[0]) % g.n[1];
  c[2] = D == 3 ? e / (g.n[0] * g.n[1]) : 0;
  int a = f >> 1, sg = f & 1;
  int v = c[a] + (sg ? 1 : -1);
  if (v < 0 || v >= g.n[a]) {
    if (a == g.wall) return sg ? -2 : -1;
    v = v < 0 ? g.n[a] - 1 : 0;
  }
  c[a] = v;
  return c[0] + g.n[0] * (c[1] + g.n[1] * c[2]);
}

// Cell at position i of the processing order.  The x index runs fastest, so
// EB consecutive positions are (mostly) EB consecutive cells of one row; the rows
// (y, z) are visited in slabs of tz z-planes, y outer and z inner within a slab.
// The y- and z-neighbours of a row were then read at most 2 tz rows earlier,
// while the state is still in the L2 cache of the XCD, instead of one whole
// z-plane earlier as in the lexicographic order.
template <int D>
__device__ __forceinline__ int cell_of(const Geo& g, int i) {
  if (D == 2 || g.tz <= 1) return i;
  const int nx = g.n[0], ny = g.n[1];
  const int x = i % nx, r = i / nx;
  const int slab = g.tz * ny;
  const int z0 = (r / slab) * g.tz, w = r % slab;
  const int tz = min(g.tz, g.n[2] - z0);
  return x + nx * (w / tz + ny * (z0 + w % tz));
}

// Cell coordinate along axis a.
template <int D>
__device__ __forceinline__ int cell_coord(const Geo& g, int e, int a) {
  if (a == 0) return e % g.n[0];
  if (a == 1) return (e / g.n[0]) % g.n[1];
  return e / (g.n[0] * g.n[1]);
}

// Logical block index with blocks of each XCD kept contiguous: hardware places
// block b on XCD b % 8, so the XCD's L2 sees a contiguous run of cells.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int nx = 8;
  int x = b % nx, per = nb / nx, rem = nb % nx;
  return x * per + (x < rem ? x : rem) + b / nx;
}

// Everything a kernel reads besides the state: kept in device memory (one copy
// per handle) so that kernels index it freely without private copies.
struct Params {
  Tables tb;
  Geo g;
  Coef cf;
};

// Flag bits reported by cdg2_sync.
enum { FLAG_NONFINITE = 1, FLAG_DOMAIN = 2 };

}  // namespace cdg2
