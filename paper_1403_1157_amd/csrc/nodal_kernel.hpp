// CDG2 operator kernel for 3D grids of order p <= 2 in nodal form, one thread per
// (cell, species).
//
// The discrete operator is the one of es_kernel.hpp (Section 3.1: volume terms,
// LLF and CDG2 face fluxes, the lifting on K^- reduced to a penalty on Cartesian
// cells).  What changes is the basis the thread works in: the Q = p + 1 point
// Gauss rule per axis integrates every product of two Q_p functions exactly, so
// the Lagrange basis l_q of the Gauss points spans the same space with the same
// (diagonal) mass matrix, and every integral of the operator — the stiffness
// (degree 2p - 2 along the derivative, 2p across), the nonlinear volume and face
// fluxes (evaluated at the Gauss points in both forms) — takes the same value.
// In that basis
//   * point values are the coefficients themselves, gradients one 1D
//     derivative matrix per axis (Dn[q][i] = l_i'(x_q));
//   * a face's tangential Gauss points are the tangential nodes, so traces need
//     only the end values l_i(0 or 1) along the normal, and face integrals
//     against the tangential test functions are pointwise with the face weights;
//   * the linear reactions are pointwise.
// The modes u (orthonormal Legendre, as stored) enter through one transform
// v = (B x B x B) u at the start and leave through one transposed transform:
// R_m = sum_q phi_m(x_q) R~_q for the residual R~ tested against l_q, and
// u_m = sum_q W_q phi_m(x_q) v_q, so the stage combination
//   cb (u + dt R / |K|) = cb B^T (W v + dt R~ / |K|)
// is formed before the one transform back.  The neighbour across a face is
// read as modes (global memory / L2) and evaluated at the face points by the
// modal route: normal contraction with phi_i(end), then the tangential basis.
//
// Compared with the modal kernel this removes the modal-to-point transforms of
// every face and of the volume layers (the FP64 instructions per wavefront drop
// by about a third); the exchange through LDS (volume layers and faces, point
// items for the nonlinear fluxes) and the staged coalesced loads and stores are
// the same.  The cell mean is kept apart from the point values (of the
// fluctuation), so that face jumps of a nearly continuous field keep their
// digits.
#pragma once

#include "es_kernel.hpp"

namespace cdg2 {

// The 1D tables of the nodal form for Q = p + 1 <= 3 Gauss points on [0,1], as
// compile-time constants (the compiler folds the zeros and ones and keeps no
// table in registers): Gauss rule, orthonormal Legendre basis
// phi_i = sqrt(2i+1) P_i(2 xi - 1) at the points and ends, and the Lagrange
// functions of the points l_i = w_i sum_k phi_k(x_i) phi_k.
constexpr double nd_sqrt(double a) {
  double r = a > 1.0 ? a : 1.0;
  for (int it = 0; it < 64; ++it) r = 0.5 * (r + a / r);
  return r;
}

template <int Q>
struct NdTab {
  double x[Q], w[Q];
  double B[Q][Q];      // phi_i(x_q)
  double E[2][Q];      // phi_i(0), phi_i(1)
  double dE[2][Q];     // phi_i'(0), phi_i'(1)
  double Dn[Q][Q];     // l_i'(x_q)
  double Le[2][Q];     // l_i(0), l_i(1)
  double dLe[2][Q];    // l_i'(0), l_i'(1)
};

// phi_i and phi_i' at xi for i < Q (Legendre recurrence on t = 2 xi - 1).
template <int Q>
constexpr void nd_legendre(double xi, double* val, double* der) {
  const double t = 2.0 * xi - 1.0;
  double P[Q + 1] = {}, dP[Q + 1] = {};
  P[0] = 1.0;
  if (Q > 1) {
    P[1] = t;
    dP[1] = 1.0;
  }
  for (int k = 1; k + 1 < Q; ++k) {
    P[k + 1] = ((2 * k + 1) * t * P[k] - k * P[k - 1]) / (k + 1);
    dP[k + 1] = ((2 * k + 1) * (P[k] + t * dP[k]) - k * dP[k - 1]) / (k + 1);
  }
  for (int i = 0; i < Q; ++i) {
    const double sc = nd_sqrt(2.0 * i + 1.0);
    val[i] = sc * P[i];
    der[i] = 2.0 * sc * dP[i];
  }
}

template <int Q>
constexpr NdTab<Q> nd_tab() {
  static_assert(Q == 2 || Q == 3, "nodal tables for p = 1, 2");
  NdTab<Q> tb{};
  if (Q == 2) {
    const double d = 0.5 / nd_sqrt(3.0);
    tb.x[0] = 0.5 - d;
    tb.x[Q - 1] = 0.5 + d;
    tb.w[0] = 0.5;
    tb.w[Q - 1] = 0.5;
  } else {
    const double d = 0.5 * nd_sqrt(0.6);
    tb.x[0] = 0.5 - d;
    tb.x[1] = 0.5;
    tb.x[Q - 1] = 0.5 + d;
    tb.w[0] = 5.0 / 18.0;
    tb.w[1] = 8.0 / 18.0;
    tb.w[Q - 1] = 5.0 / 18.0;
  }
  double Bd[Q][Q] = {};
  for (int q = 0; q < Q; ++q) nd_legendre<Q>(tb.x[q], tb.B[q], Bd[q]);
  for (int s = 0; s < 2; ++s) nd_legendre<Q>((double)s, tb.E[s], tb.dE[s]);
  for (int i = 0; i < Q; ++i) {
    for (int r = 0; r < Q; ++r) {
      double acc = 0.0;
      for (int k = 0; k < Q; ++k) acc += tb.B[i][k] * Bd[r][k];
      tb.Dn[r][i] = tb.w[i] * acc;
    }
    for (int s = 0; s < 2; ++s) {
      double a0 = 0.0, a1 = 0.0;
      for (int k = 0; k < Q; ++k) {
        a0 += tb.B[i][k] * tb.E[s][k];
        a1 += tb.B[i][k] * tb.dE[s][k];
      }
      tb.Le[s][i] = tb.w[i] * a0;
      tb.dLe[s][i] = tb.w[i] * a1;
    }
  }
  return tb;
}

// s += c x for a compile-time constant c (nothing for c = 0).
template <typename T>
__device__ __forceinline__ void nd_acc(T& s, double c, T x) {
  if (c != 0.0) s += T(c) * x;
}

// out = (B (x) B) in over the Q^2 tangential entries (TR: transposed), first
// index fastest.
template <int Q, bool TR, typename T>
__device__ __forceinline__ void nd_tapply2(const T* in, T* out) {
  constexpr NdTab<Q> ct = nd_tab<Q>();
  T t[Q * Q];
#pragma unroll
  for (int j = 0; j < Q; ++j)
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      T s = T(0);
#pragma unroll
      for (int i = 0; i < Q; ++i) nd_acc(s, TR ? ct.B[i][a] : ct.B[a][i], in[i + Q * j]);
      t[a + Q * j] = s;
    }
#pragma unroll
  for (int b = 0; b < Q; ++b)
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      T s = T(0);
#pragma unroll
      for (int j = 0; j < Q; ++j) nd_acc(s, TR ? ct.B[j][b] : ct.B[b][j], t[a + Q * j]);
      out[a + Q * b] = s;
    }
}

// out = (B (x) B (x) B) in over Q^3 entries (TR: transposed), x fastest.
template <int Q, bool TR, typename T>
__device__ __forceinline__ void nd_tapply3(const T* in, T* out) {
  constexpr NdTab<Q> ct = nd_tab<Q>();
  constexpr int F = Q * Q;
  T t[Q * F];
#pragma unroll
  for (int k = 0; k < Q; ++k) nd_tapply2<Q, TR, T>(in + F * k, t + F * k);
#pragma unroll
  for (int q = 0; q < F; ++q)
#pragma unroll
    for (int c = 0; c < Q; ++c) {
      T s = T(0);
#pragma unroll
      for (int k = 0; k < Q; ++k) nd_acc(s, TR ? ct.B[k][c] : ct.B[c][k], t[q + F * k]);
      out[q + F * c] = s;
    }
}

// u <- (B (x) B (x) B) u in place, one line of Q entries at a time along each
// axis (only Q temporaries live).
template <int Q, typename T>
__device__ __forceinline__ void nd_tapply3_inplace(T* u) {
  constexpr NdTab<Q> ct = nd_tab<Q>();
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const int st = ax == 0 ? 1 : ax == 1 ? Q : Q * Q;
#pragma unroll
    for (int b = 0; b < Q; ++b)
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        // the line through (a, b) of the two other axes
        const int o = ax == 0 ? Q * a + Q * Q * b : ax == 1 ? a + Q * Q * b : a + Q * b;
        T t[Q];
#pragma unroll
        for (int c = 0; c < Q; ++c) {
          T acc = T(0);
#pragma unroll
          for (int i = 0; i < Q; ++i) nd_acc(acc, ct.B[c][i], u[o + st * i]);
          t[c] = acc;
        }
#pragma unroll
        for (int c = 0; c < Q; ++c) u[o + st * c] = t[c];
      }
  }
}

// Volume exchange slots per point: 0 n1, 1 n2, 2 c1, 3 c3, 4..6 grad n1,
// 7..9 grad c1, 10..12 grad c3, 13 n3, 14 c2.  The point items overwrite
// 4..6 with F1 (weighted, / h_a), 7..9 with F2 and 10 with the alpha term.
constexpr int ND_NVQ = 15;

// After the face slots: each thread's face jump and derivative sum (2 x NF
// values), parked there through the face point pass.  The per-thread stride
// stays 2 NF (16-byte aligned, so two values move in one LDS access): an odd
// stride, free of bank conflicts, measured slower.
template <int P>
constexpr int nd_park_stride() { return 2 * (P + 1) * (P + 1); }
template <int P, typename T, int EB>
using NdSmem = EsSmem<3, P, T, EB, ND_NVQ, 6 * EB * nd_park_stride<P>() + 4>;
// Start of the parked values: after the face slots, rounded up to 4 elements.
template <int P, typename T, int EB>
constexpr int nd_park_base() { return (NdSmem<P, T, EB>::FAC + 3) & ~3; }

// Workgroup barrier that is also a scheduling fence: no instruction moves across
// it, so the compiler cannot start a later layer's or face's arithmetic early and
// hold its registers through the current one.
__device__ __forceinline__ void nd_sync() {
  __syncthreads();
  __builtin_amdgcn_sched_barrier(0);
}

// KIND: 0 an operator application (out = f(U)); 1 an SSP-RK3 stage without the
// u0 term (out = cb (U + dt f(U))); 2 a stage with it (out = ca U0 + cb (U + dt f(U))).
// Kinds 0 to 2 read and write modes.  Kinds 3 to 5 are the stages of an SSP-RK3
// step whose two intermediate states are kept as point values (the coefficients
// of the Lagrange basis of the Gauss points, same layout as the modes: point
// i + Q (j + Q k) where mode i + Q (j + Q k) would be):
//   3  stage 1, modes in, point values out, out = cb (U + dt f(U));
//   4  stage 2, point values in and out, out = ca U0 + cb (U + dt f(U)) with U0
//      given as modes and taken to the points in the kernel;
//   5  stage 3, point values in, modes out, out = ca U0 + cb (U + dt f(U)).
// The point values of an intermediate state are what the kernel computes first
// anyway, and a neighbour's traces from them cost one contraction along the
// normal (three terms per face point) instead of that and two tangential
// transforms; the three stages make the same discrete step up to rounding.
// Each kind is its own kernel (the profiles tell them apart, and the branches of
// the other kinds are not compiled in).
template <int P, typename T, int EB, int KIND>
__device__ __forceinline__ void nd_block(const Params& prm, const T* __restrict__ U, const T* U0, T* out, T dt,
                                         T ca, T cb, int* __restrict__ flags, int e0, NdSmem<P, T, EB>& sm) {
  constexpr int D = 3;
  using S = EsSz<D, P>;
  constexpr int Q = S::Q, NM = S::NM, NF = S::NF, NFACE = S::NFACE, PC = S::PC;
  constexpr int NVQ = ND_NVQ, NT = 6 * EB;
  static_assert(NdSmem<P, T, EB>::STAGED, "3D staging");
  constexpr int FST = NdSmem<P, T, EB>::FST;
  static_assert(EB * NVQ * PC <= NdSmem<P, T, EB>::N && nd_park_base<P, T, EB>() + NT * nd_park_stride<P>() <= NdSmem<P, T, EB>::N &&
                    NT * NM <= NdSmem<P, T, EB>::N,
                "LDS union");
  const Tables& tb = prm.tb;
  constexpr NdTab<Q> ct = nd_tab<Q>();
  const Geo& g = prm.g;
  const double* c = prm.cf.c;
  const int tid = threadIdx.x;
  const int s = tid / EB, el = tid % EB;
  const int E = g.E;
  const bool live = e0 + el < E;
  const size_t SE = (size_t)E * NM;
  const T vol = T(g.vol);
  int flag = 0;

  constexpr bool nodal_in = KIND == 4 || KIND == 5;
  constexpr bool nodal_out = KIND == 3 || KIND == 4;

  // ---- own modes -> nodal values --------------------------------------------------
  T v[NM], R[NM], m0;
  if (tid < EB) sm.cell[tid] = e0 + tid < E ? cell_of<D>(g, e0 + tid) : -1;
  nd_sync();
  stage_modes<D, P, T, EB>(U, SE, E, sm, tid);
  // the neighbour table is built while the modes are in flight
  for (int it = tid; it < EB * NFACE; it += NT) {
    int l = it / NFACE, f = it % NFACE;
    sm.nb[l][f] = e0 + l < E ? neighbour<D>(g, cell_of<D>(g, e0 + l), f) : -3;
  }
  wait_staged();
  nd_sync();
  if constexpr (nodal_in) {
    // point values as stored (their rounding is already that of the full values,
    // so no mean is kept apart)
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      const T x = staged<D, P, T, EB>(sm, tid, m);
      v[m] = live ? x : T(0);
    }
    m0 = T(0);
  } else {
    T u[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      const T x = staged<D, P, T, EB>(sm, tid, m);   // in range for every thread
      u[m] = live ? x : T(0);
    }
    // v holds the fluctuation u - mean (mode 0 kept apart in m0): its point
    // values are small for a smooth field, so face jumps formed from them keep
    // the accuracy that the difference of two full traces would lose
    m0 = u[0];
    u[0] = T(0);
    nd_tapply3<Q, false, T>(u, v);
  }
#pragma unroll
  for (int m = 0; m < NM; ++m) R[m] = T(0);

  // ---- volume, one layer of Gauss points (along z) at a time --------------------------
  const T as = T(c[K_MU1 + s]);
  const int vslot = s == S_N1 ? 0 : s == S_N2 ? 1 : s == S_C1 ? 2 : s == S_C3 ? 3 : s == S_N3 ? 13 : 14;
  const int gslot = s == S_N1 ? 4 : s == S_C1 ? 7 : s == S_C3 ? 10 : -1;
  // linear reactions: n1 -d1 n1; n2 -d2 n2; n3 (d1 - gamma) n1 + d2 n2; c1 f1 n3;
  // c2 -k c2; c3 k c2 (the own value, or up to two other species' values)
  const T kown = T(s == S_N1 ? -c[K_D1] : s == S_N2 ? -c[K_D2] : s == S_C2 ? -c[K_K] : 0.0);
  const int r0 = s == S_N3 ? 0 : s == S_C1 ? 13 : s == S_C3 ? 14 : 0;   // k0 = 0 selects nothing
  const T k0 = T(s == S_N3 ? c[K_D1] - c[K_GAM] : s == S_C1 ? c[K_F1] : s == S_C3 ? c[K_K] : 0.0);
  const T k1 = T(s == S_N3 ? c[K_D2] : 0.0);
  // nonlinear volume fluxes: F1 (slots 4..6) on n1, F2 (7..9) on n2; alpha term
  // (slot 10) on c1
  const int fs = s == S_N2 ? 7 : 4;
  const T fw = T(s == S_N1 || s == S_N2 ? 1 : 0), rw = T(s == S_C1 ? 1 : 0);
  T* V = sm.buf;   // [EB][NVQ][PC]
  // The layer loop is not unrolled (an unrolled one let the compiler hold several
  // layers' temporaries at once).  So that registers are still indexed statically,
  // v and R are rotated by one layer per iteration: position k holds layer
  // (lc + k) mod Q, the current layer is always at position 0, and after Q
  // iterations the order is the original one.
#pragma unroll 1
  for (int lc = 0; lc < Q; ++lc) {
    T dz[Q];   // l'_{(lc + k) mod Q}(x_lc): z-derivative weights of position k
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int r = lc + k < Q ? lc + k : lc + k - Q;
      dz[k] = T(tb.Dn[lc][r]);
    }
    const T wl = vol * T(tb.w[lc]);
    // own gradient at the layer's points (physical)
    T gr[3][NF];
#pragma unroll
    for (int j = 0; j < Q; ++j)
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        T ax = T(0), ay = T(0), az = T(0);
#pragma unroll
        for (int r = 0; r < Q; ++r) {
          nd_acc(ax, ct.Dn[i][r], v[r + Q * j]);
          nd_acc(ay, ct.Dn[j][r], v[i + Q * r]);
          az += dz[r] * v[i + Q * j + PC * r];
        }
        gr[0][i + Q * j] = ax * T(g.ih[0]);
        gr[1][i + Q * j] = ay * T(g.ih[1]);
        gr[2][i + Q * j] = az * T(g.ih[2]);
      }
    nd_sync();
    {
      T* o = V + el * NVQ * PC;
#pragma unroll
      for (int q = 0; q < PC; ++q) o[vslot * PC + q] = m0 + v[q];
      if (gslot >= 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int q = 0; q < PC; ++q) o[(gslot + a) * PC + q] = gr[a][q];
      }
    }
    nd_sync();
    // point items: chemotactic fluxes and the alpha reaction term, weighted
    for (int it = tid; it < EB * PC; it += NT) {
      const int l = it / PC, q = it % PC;
      T* x = V + l * NVQ * PC + q;
      const T n1 = x[0], n2 = x[PC], c1 = x[2 * PC], c3 = x[3 * PC];
      const T d11 = c1 + T(c[K_XT11]), d13 = c3 + T(c[K_XT13]), d21 = c1 + T(c[K_XT21]),
              d22 = n1 + T(c[K_XT22]);
      if (e0 + l < E && !(d11 > T(0) && d13 > T(0) && d21 > T(0) && d22 > T(0))) flag |= FLAG_DOMAIN;
      T r11, r13, r21, r22;
      recip4(d11, d13, d21, d22, r11, r13, r21, r22);
      const T k11 = T(c[K_X011]) * r11, k13 = T(c[K_X013]) * r13, k21 = T(c[K_X021]) * r21,
              k22 = T(c[K_X022]) * r22;
      const T wt = wl * T(ct.w[q % Q] * ct.w[q / Q]);
      T F1[3], F2[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const T gn1 = x[(4 + a) * PC], gc1 = x[(7 + a) * PC], gc3 = x[(10 + a) * PC];
        F1[a] = n1 * (k11 * gc1 + k13 * gc3) * wt * T(g.ih[a]);
        F2[a] = n2 * (k21 * gc1 - k22 * gn1) * wt * T(g.ih[a]);
      }
      const T rc = -(T(c[K_AL1]) * n1 + T(c[K_AL2]) * n2) * c1 * wt;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        x[(4 + a) * PC] = F1[a];
        x[(7 + a) * PC] = F2[a];
      }
      x[10 * PC] = rc;
    }
    nd_sync();
    // test integration of the layer against the Lagrange functions (branch-free:
    // species-dependent terms enter with 0/1 factors, every read is in range)
    {
      const T* x = V + el * NVQ * PC;
      // the gradient registers become the weighted fluxes (F - a_s grad u) / h_a
#pragma unroll
      for (int q = 0; q < PC; ++q) {
        const T wt = wl * T(ct.w[q % Q] * ct.w[q / Q]);
#pragma unroll
        for (int a = 0; a < 3; ++a) gr[a][q] = fw * x[(fs + a) * PC + q] - as * gr[a][q] * (wt * T(g.ih[a]));
        const T re = kown * (m0 + v[q]) + k0 * x[r0 * PC + q] + k1 * x[PC + q];
        R[q] += wt * re + rw * x[10 * PC + q];
      }
#pragma unroll
      for (int j = 0; j < Q; ++j)
#pragma unroll
        for (int r = 0; r < Q; ++r) {
          T ax = T(0), ay = T(0);
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            nd_acc(ax, ct.Dn[i][r], gr[0][i + Q * j]);
            nd_acc(ay, ct.Dn[i][r], gr[1][j + Q * i]);
          }
          R[r + Q * j] += ax;
          R[j + Q * r] += ay;
        }
#pragma unroll
      for (int r = 0; r < Q; ++r) {
#pragma unroll
        for (int q = 0; q < PC; ++q) R[q + PC * r] += dz[r] * gr[2][q];
      }
    }
    // rotate: the next layer to position 0
#pragma unroll
    for (int q = 0; q < PC; ++q) {
      const T v0 = v[q], r0v = R[q];
#pragma unroll
      for (int k = 0; k + 1 < Q; ++k) {
        v[q + PC * k] = v[q + PC * (k + 1)];
        R[q + PC * k] = R[q + PC * (k + 1)];
      }
      v[q + PC * (Q - 1)] = v0;
      R[q + PC * (Q - 1)] = r0v;
    }
  }

  // ---- faces ------------------------------------------------------------------------
  const bool diss = !(g.llf_cells && s > S_N2);
  // face exchange slots (x NF): 0..3 values n1 n2 c1 c3 own, 4..7 same neighbour,
  // 8..10 d_a n1 c1 c3 own, 11..13 neighbour.  After the point pass: 0 lambda/2,
  // 1 -F1.n_o/2 sum, 2 -F2.n_o/2 sum, 3..5 inflow fluxes n1, n2, c2 (boundary).
  T* Fx = sm.buf;
  const int fvslot = s == S_N1 ? 0 : s == S_N2 ? 1 : s == S_C1 ? 2 : s == S_C3 ? 3 : -1;
  const int dslot = s == S_N1 ? 8 : s == S_C1 ? 9 : s == S_C3 ? 10 : -1;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll 1
  for (int sg = 0; sg < 2; ++sg) {
    const int f = 2 * a + sg;
    nd_sync();
    const int nb = sm.nb[el][f];
    // traces at the face points: own from the nodal values (end values of the
    // Lagrange functions along the normal), neighbour from its values in global
    // memory.  The side's end values come from the run-time tables: selected
    // among compile-time constants, the compiler formed both sides' products and
    // kept them live.
    T uo[NF], duo[NF], un[NF], dun[NF];
    T w0;   // neighbour mean (mode 0); un, dun are its fluctuation's traces
    {
      // a boundary face reads the own cell (in range) and weighs it by zero
      const T inner = T(nb >= 0 ? 1 : 0);
      const T* un_src = U + s * SE + (size_t)(nb >= 0 ? nb : sm.cell[el] >= 0 ? sm.cell[el] : 0) * NM;
      if constexpr (nodal_in) {
        // the neighbour's point values on the normal lines through the face points
#pragma unroll
        for (int t = 0; t < NF; ++t) {
          T a0 = T(0), a1 = T(0);
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const T x = un_src[face_mode<D, Q>(a, i, t)];
            a0 += T(tb.Le[1 - sg][i]) * x;
            a1 += T(tb.dLe[1 - sg][i]) * x;
          }
          un[t] = a0 * inner;
          dun[t] = a1 * (inner * T(g.ih[a]));
        }
        w0 = T(0);
      } else {
        T mv[NF], md[NF];
#pragma unroll
        for (int J = 0; J < NF; ++J) {
          T a0 = T(0), a1 = T(0);
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const int m = face_mode<D, Q>(a, i, J);
            const T x = un_src[m];
            if (m != 0) a0 += T(tb.E[1 - sg][i]) * x;   // the mean apart
            if (i != 0) a1 += T(tb.dE[1 - sg][i]) * x;  // phi_0' = 0
          }
          mv[J] = a0 * inner;
          md[J] = a1 * (inner * T(g.ih[a]));
        }
        nd_tapply2<Q, false, T>(mv, un);
        nd_tapply2<Q, false, T>(md, dun);
        w0 = un_src[0] * inner;
      }
    }
#pragma unroll
    for (int t = 0; t < NF; ++t) {
      T a0 = T(0), a1 = T(0);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const T x = v[face_mode<D, Q>(a, i, t)];
        a0 += T(tb.Le[sg][i]) * x;
        a1 += T(tb.dLe[sg][i]) * x;
      }
      uo[t] = a0;
      duo[t] = a1 * T(g.ih[a]);
    }
    // publish the point values of the face point pass (the exchange slots overlay
    // the volume slots: everyone has finished reading them)
    if (fvslot >= 0) {
#pragma unroll
      for (int t = 0; t < NF; ++t) {
        Fx[el * FST + (fvslot) * NF + t] = m0 + uo[t];
        Fx[el * FST + (4 + fvslot) * NF + t] = w0 + un[t];
      }
    }
    if (dslot >= 0) {
#pragma unroll
      for (int t = 0; t < NF; ++t) {
        Fx[el * FST + (dslot) * NF + t] = duo[t];
        Fx[el * FST + (dslot + 3) * NF + t] = dun[t];
      }
    }
    // the jump and the derivative sum wait in LDS during the point pass (no
    // registers held through it)
    T* park = sm.buf + nd_park_base<P, T, EB>() + tid * nd_park_stride<P>();
    // weights of the own side and the neighbour in the average (own is K^- on the
    // high face, sg = 1)
    const T wo = T(sg ? g.wm : g.wp), wn = T(sg ? g.wp : g.wm);
#pragma unroll
    for (int t = 0; t < NF; ++t) {
      park[t] = (m0 - w0) + (uo[t] - un[t]);
      park[NF + t] = wo * duo[t] + wn * dun[t];
    }
    nd_sync();
    // face point pass (kind 4 keeps one point per thread: with the split points its
    // register allocation spilled 8 VGPRs, and the launch took 11% longer)
    const int b0 = a == 0 ? 1 : 0;   // first tangential axis
    face_points<D, Q, NF, EB, FST, KIND != 4, T>(Fx, sm.nb, f, sg, b0, c, g, tb, e0, E, tid, flag);
    nd_sync();
    // species pass: all face terms at the face points, weighted, spread onto the
    // Lagrange functions of the normal line through each point
    {
      const T* x = Fx + el * FST;
      const T ar = T(g.area[a]);
      const T so = sg ? T(1) : T(-1);
      const T pen = T(g.pen_c * tb.liftc * g.ih[a]) * as;
      const T hs = T((sg ? g.wm : g.wp) * g.sym) * as * so * T(g.ih[a]);
      const bool in = nb >= 0;
      const T dw = T(diss ? 1 : 0);
      // the one flux slot this species adds: interior n1 F1 (1), n2 F2 (2);
      // boundary inflow n1 (3), n2 (4), c2 (5); weight 0 for the others
      const int ksl = in ? (s == S_N2 ? 2 : 1) : (s == S_N2 ? 4 : s == S_C2 ? 5 : 3);
      const T kw = T(in ? (s == S_N1 || s == S_N2 ? 1 : 0) : (s == S_N1 || s == S_N2 || s == S_C2 ? 1 : 0));
      const T li = T(in ? 1 : 0);   // linear face terms on interior faces only
      const T le0 = T(tb.Le[sg][0]), le1 = T(tb.Le[sg][1]), dle0 = T(tb.dLe[sg][0]), dle1 = T(tb.dLe[sg][1]);
      const T le2 = T(tb.Le[sg][Q - 1]), dle2 = T(tb.dLe[sg][Q - 1]);
      const T* park = sm.buf + nd_park_base<P, T, EB>() + tid * nd_park_stride<P>();
      // the per-face factors (area, the 0/1 weights) folded once
      const T fa = li * ar, cs = fa * so * as, cp = fa * pen, cd = fa * dw, ck = kw * ar, ch = fa * hs;
#pragma unroll
      for (int t = 0; t < NF; ++t) {
        const T jm = park[t], sd = park[NF + t];
        const T wq = T(ct.w[t % Q] * ct.w[t / Q]);
        const T G = wq * (cs * sd - (cp + cd * x[t]) * jm + ck * x[ksl * NF + t]);
        const T H = (wq * ch) * jm;
        // spread at once onto the normal line through the point
        R[face_mode<D, Q>(a, 0, t)] += le0 * G + dle0 * H;
        if (Q == 3) R[face_mode<D, Q>(a, 1, t)] += le1 * G + dle1 * H;
        R[face_mode<D, Q>(a, Q - 1, t)] += le2 * G + dle2 * H;
      }
    }
  }

  // ---- back to modes: M^{-1}, stage combination, coalesced store ------------------------
  // (+ ca U0 in the store, whose U0 loads come in chunks: all of them in flight
  // through the transform back would not fit the register budget)
  // Kinds 2, 4 and 5 take the workgroup's U0 modes through the staging area: the
  // loads are issued before the last transform and occupy no registers while in
  // flight (the faces are done with the shared LDS area after the first sync).
  // Loaded at the store instead, their latency was exposed (stage 3: 635 ->
  // 591 us per 64^3 Q2 launch).
  constexpr bool u0_staged = KIND == 2 || KIND == 4 || KIND == 5;
  if constexpr (u0_staged) {
    nd_sync();
    stage_modes<D, P, T, EB>(U0, SE, E, sm, tid);
  }
  if constexpr (nodal_out) {
    // point values: M = |K| W_q is diagonal in the Lagrange basis of the points
    const T dti = dt * T(1.0 / g.vol);
    T y[NM];
#pragma unroll
    for (int k = 0; k < Q; ++k)
#pragma unroll
      for (int j = 0; j < Q; ++j)
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const int m = i + Q * (j + Q * k);
          y[m] = cb * ((m0 + v[m]) + dti * R[m] * T(1.0 / (ct.w[i] * ct.w[j] * ct.w[k])));
        }
    if constexpr (KIND == 4) {
      // + ca U0 at the points
      wait_staged();
      nd_sync();
      T u[NM];
      staged_all<D, P, T, EB>(sm, tid, u);
      nd_tapply3_inplace<Q, T>(u);
#pragma unroll
      for (int m = 0; m < NM; ++m) y[m] += ca * u[m];
    }
    nd_sync();
#pragma unroll
    for (int m = 0; m < NM; ++m) sm.buf[tid * NM + m] = y[m];
  } else {
    const T ivol = T(1.0 / g.vol);
    T z[NM], y[NM];
    if constexpr (KIND == 0) {
#pragma unroll
      for (int m = 0; m < NM; ++m) z[m] = R[m] * ivol;
    } else {
      const T dti = dt * ivol;
#pragma unroll
      for (int k = 0; k < Q; ++k)
#pragma unroll
        for (int j = 0; j < Q; ++j)
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const int m = i + Q * (j + Q * k);
            // one fused operation that needs R: the compiler cannot form W v
            // early and hold it through the faces
            z[m] = __builtin_fma(T(ct.w[i] * ct.w[j] * ct.w[k]), v[m], dti * R[m]);
          }
    }
    nd_tapply3<Q, true, T>(z, y);
    if constexpr (KIND != 0) y[0] += m0;
    if constexpr (KIND == 2 || KIND == 5) {
      // + ca U0 (modes, the thread's own cell and species)
      wait_staged();
      nd_sync();
      T u[NM];
      staged_all<D, P, T, EB>(sm, tid, u);
#pragma unroll
      for (int m = 0; m < NM; ++m) y[m] = cb * y[m] + ca * u[m];
    }
    nd_sync();
#pragma unroll
    for (int m = 0; m < NM; ++m) sm.buf[tid * NM + m] = KIND == 1 ? cb * y[m] : y[m];
  }
  nd_sync();
  store_results<T, EB, NM>(sm.cell, sm.buf, U0, out, SE, ca, false, tid, flag);
  if (flag) atomicOr(flags, flag);
}

template <int P, typename T, int EB, int KIND>
__global__ void __launch_bounds__(6 * EB, 2)
nd_kernel(const Params* __restrict__ prm, const T* __restrict__ U, const T* U0, T* out, T dt, T ca, T cb,
          int* __restrict__ flags) {
  __shared__ NdSmem<P, T, EB> sm;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  nd_block<P, T, EB, KIND>(*prm, U, U0, out, dt, ca, cb, flags, blk * EB, sm);
}

}  // namespace cdg2
