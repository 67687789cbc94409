// Transposed Jacobian of the CDG2 operator, one thread per (cell, species).
//
// For f(U) = M^{-1} L_h(U) and an adjoint vector w, the kernel forms
//   out = cw w + cj J(U)^T w + c2 X2 + c3 X3        (X2, X3 optional, own cell)
// and, on request, the parameter derivatives d(w . f(U))/d theta_j of the 21
// differentiable coefficients, scaled by cj, as per-workgroup partial sums.
//
// With v = w / |K| (M = |K| I) and Lambda = sum v . R(U):
//   * linear diffusion (volume stiffness, face consistency / symmetry / CDG2
//     lifting terms): the bilinear form is symmetric, so its transpose applied to
//     v is the same modal operator applied to v;
//   * linear reactions: the transposed 6x6 mode-wise coupling;
//   * volume nonlinear terms: pointwise derivatives of F1 . grad psi_n1 +
//     F2 . grad psi_n2 - (alpha1 n1 + alpha2 n2) c1 psi_c1, with psi_s = sum v phi,
//     integrated against phi and grad phi;
//   * face nonlinear terms: each face contributes int_e sum_s g_s (psi_s^own -
//     psi_s^nb) with g_s = -1/2 (F_o + F_n).n_o - 1/2 lam (u_o - u_n); a cell
//     differentiates it with respect to its own traces.  |x| has derivative
//     sign(x) (0 at 0), the max in lam picks the first maximiser in the order
//     (w1_o, w2_o, w1_n, w2_n), the Heaviside of the inflow has derivative 0.
// Parameter derivatives of a face are added by the cell for which it is the high
// face (interior) or by its only cell (boundary), so that each face counts once.
#pragma once

#include "es_kernel.hpp"

namespace cdg2 {

template <int D, int P>
struct AdjSz {
  using Z = Sz<D, P>;
  static constexpr int Q = Z::Q, NM = Z::NM, NF = Z::NF, PC = NF;
  // volume slots: 13 forward (n1 n2 c1 c3 | grad n1 | grad c1 | grad c3), then
  // grad psi_n1 (D), grad psi_n2 (D), psi_c1
  static constexpr int NVQ = 4 + 3 * D + 2 * D + 1;
  // face slots: 14 forward (as in the forward kernel), 6 adjoint jumps dpsi,
  // 6 forward jumps
  static constexpr int NFQ = 26;
};

template <int D, int P, typename T, int EB>
struct AdjSmem {
  using S = AdjSz<D, P>;
  // per-cell strides, odd in elements of T so that the cells of the workgroup
  // start on different LDS banks (the plain ones are multiples of 32 dwords in 3D)
  static constexpr int VST = (S::NVQ * S::PC) | 1, FST = (S::NFQ * S::NF) | 1;
  static constexpr int VOL = EB * VST;
  static constexpr int FAC = EB * FST;
  static constexpr int N = VOL > FAC ? VOL : FAC;
  alignas(16) T buf[N];  // also holds the doubles of the final reduction
  int nb[EB][2 * D];
};

// Parameter-derivative slots (indices into the 21 differentiable coefficients).
template <int D, int P, typename T, int EB>
__device__ __forceinline__ void adj_block(const Params& prm, const T* __restrict__ U, const T* __restrict__ W,
                                          T* out, T cw, T cj, const T* X2, T c2, const T* X3, T c3,
                                          double* __restrict__ part, int want_theta,
                                          int* __restrict__ flags, int e0, int blk,
                                          AdjSmem<D, P, T, EB>& sm) {
  using S = AdjSz<D, P>;
  constexpr int Q = S::Q, NM = S::NM, NF = S::NF, NFACE = 2 * D, PC = S::PC, NVQ = S::NVQ;
  constexpr int VST = AdjSmem<D, P, T, EB>::VST, FST = AdjSmem<D, P, T, EB>::FST;
  constexpr int NT = 6 * EB;
  const Tables& tb = prm.tb;
  const Geo& g = prm.g;
  const double* c = prm.cf.c;
  const int tid = threadIdx.x;
  const int s = tid / EB, el = tid % EB;
  const int E = g.E;
  const int e = e0 + el;
  const bool live = e < E;
  const size_t SE = (size_t)E * NM;
  const T vol = T(g.vol), ivol = T(1.0 / g.vol);
  int flag = 0;
  double th[CDG2_NDIFF];
#pragma unroll
  for (int j = 0; j < CDG2_NDIFF; ++j) th[j] = 0.0;

  T u[NM], v[NM], R[NM];
  {
    const size_t off = s * SE + (size_t)(live ? e : 0) * NM;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      u[m] = live ? U[off + m] : T(0);
      v[m] = live ? W[off + m] * ivol : T(0);
    }
  }
  for (int it = tid; it < EB * NFACE; it += NT) {
    int l = it / NFACE, f = it % NFACE;
    sm.nb[l][f] = e0 + l < E ? neighbour<D>(g, e0 + l, f) : -3;
  }

  // ---- linear diffusion (symmetric: applied to v), parameter derivative via a = 1 -----
  // d/d a_s of the diffusion part is the a_s = 1 form of u against v; it is
  // accumulated as the scalar thd term by term (volume here, faces below) rather
  // than through a second residual array, which would not fit the registers at
  // 3D p = 3.  The form is symmetric, so the volume part is S(v) . u.
  const T as = T(c[K_MU1 + s]);
  double thd = 0.0;
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    T accv = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int st = ipow(Q, a);
      const int ia = (m / st) % Q;
      const int base = m - ia * st;
      T sv = T(0);
#pragma unroll
      for (int j = 0; j < Q; ++j) sv += T(tb.S[ia][j]) * v[base + j * st];
      accv += T(g.ih[a] * g.ih[a]) * sv;
    }
    R[m] = -as * vol * accv;
    if (want_theta) thd += (double)(-vol * accv) * (double)u[m];
  }
  // transposed linear reactions: (J^T w)_{s'} += sum_s L[s][s'] w_s = vol sum_s L[s][s'] v_s
  {
    const T* wc = W + (size_t)(live ? e : 0) * NM;
    if (live) {
      auto addw = [&](int sp, double k) {
        const T* src = wc + sp * SE;
        const T kk = T(k);
#pragma unroll
        for (int m = 0; m < NM; ++m) R[m] += kk * src[m];
      };
      switch (s) {
        case S_N1: addw(S_N1, -c[K_D1]); addw(S_N3, c[K_D1] - c[K_GAM]); break;
        case S_N2: addw(S_N2, -c[K_D2]); addw(S_N3, c[K_D2]); break;
        case S_N3: addw(S_C1, c[K_F1]); break;
        case S_C2: addw(S_C2, -c[K_K]); addw(S_C3, c[K_K]); break;
        default: break;
      }
      if (want_theta) {
        // d/d{d1, d2, gamma, f1, k} of sum w . (L U) (mode-wise, this cell)
        const T* Uc = U + (size_t)e * NM;
        const T* Wc = wc;
        if (s == S_N1) {
          double a1 = 0, a2 = 0;
#pragma unroll
          for (int m = 0; m < NM; ++m) {
            const double un1 = Uc[S_N1 * SE + m];
            a1 += (-(double)Wc[S_N1 * SE + m] + (double)Wc[S_N3 * SE + m]) * un1;
            a2 += -(double)Wc[S_N3 * SE + m] * un1;
          }
          th[K_D1] += a1;
          th[K_GAM] += a2;
        } else if (s == S_N2) {
          double a1 = 0;
#pragma unroll
          for (int m = 0; m < NM; ++m)
            a1 += (-(double)Wc[S_N2 * SE + m] + (double)Wc[S_N3 * SE + m]) * (double)Uc[S_N2 * SE + m];
          th[K_D2] += a1;
        } else if (s == S_N3) {
          double a1 = 0;
#pragma unroll
          for (int m = 0; m < NM; ++m) a1 += (double)Wc[S_C1 * SE + m] * (double)Uc[S_N3 * SE + m];
          th[K_F1] += a1;
        } else if (s == S_C2) {
          double a1 = 0;
#pragma unroll
          for (int m = 0; m < NM; ++m)
            a1 += (-(double)Wc[S_C2 * SE + m] + (double)Wc[S_C3 * SE + m]) * (double)Uc[S_C2 * SE + m];
          th[K_K] += a1;
        }
      }
    }
  }

  // ---- volume nonlinear terms, one layer of Gauss points at a time ------------------
  const int prod = s == S_N1 ? 0 : s == S_N2 ? 1 : s == S_C1 ? 2 : s == S_C3 ? 3 : -1;
  const bool grads = s == S_N1 || s == S_C1 || s == S_C3;
  const int gslot = s == S_N1 ? 4 : s == S_C1 ? 4 + D : 4 + 2 * D;
  constexpr int AG1 = 4 + 3 * D, AG2 = AG1 + D, AL3 = AG2 + D;   // adjoint slots
  T* V = sm.buf;   // [EB][VST]: NVQ slots of PC points, then the pad
  constexpr int LA = D - 1;
  constexpr int LST = ipow(Q, D - 1);
  const double(*Bt0)[CDG2_MAXQ] = tb.B;
  for (int lc = 0; lc < Q; ++lc) {
    __syncthreads();
    if (prod >= 0) {
      T tv[NF], td[NF], o[NF];
#pragma unroll
      for (int r = 0; r < NF; ++r) {
        T a0 = T(0), a1 = T(0);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          a0 += T(tb.B[lc][k]) * u[r + LST * k];
          a1 += T(tb.Bd[lc][k]) * u[r + LST * k];
        }
        tv[r] = a0;
        td[r] = a1;
      }
      tapply_lo<D, Q, false, T>(tv, o, Bt0, Bt0);
#pragma unroll
      for (int q = 0; q < PC; ++q) V[el * VST + (prod) * PC + q] = o[q];
      if (grads) {
#pragma unroll
        for (int a = 0; a < D - 1; ++a) {
          tapply_lo<D, Q, false, T>(tv, o, a == 0 ? tb.Bd : tb.B, a == 1 ? tb.Bd : tb.B);
#pragma unroll
          for (int q = 0; q < PC; ++q) V[el * VST + (gslot + a) * PC + q] = o[q] * T(g.ih[a]);
        }
        tapply_lo<D, Q, false, T>(td, o, Bt0, Bt0);
#pragma unroll
        for (int q = 0; q < PC; ++q) V[el * VST + (gslot + LA) * PC + q] = o[q] * T(g.ih[LA]);
      }
    }
    // adjoint fields: grad psi_n1, grad psi_n2, psi_c1
    if (s == S_N1 || s == S_N2 || s == S_C1) {
      T tv[NF], td[NF], o[NF];
#pragma unroll
      for (int r = 0; r < NF; ++r) {
        T a0 = T(0), a1 = T(0);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          a0 += T(tb.B[lc][k]) * v[r + LST * k];
          a1 += T(tb.Bd[lc][k]) * v[r + LST * k];
        }
        tv[r] = a0;
        td[r] = a1;
      }
      if (s == S_C1) {
        tapply_lo<D, Q, false, T>(tv, o, Bt0, Bt0);
#pragma unroll
        for (int q = 0; q < PC; ++q) V[el * VST + (AL3) * PC + q] = o[q];
      } else {
        const int base = s == S_N1 ? AG1 : AG2;
#pragma unroll
        for (int a = 0; a < D - 1; ++a) {
          tapply_lo<D, Q, false, T>(tv, o, a == 0 ? tb.Bd : tb.B, a == 1 ? tb.Bd : tb.B);
#pragma unroll
          for (int q = 0; q < PC; ++q) V[el * VST + (base + a) * PC + q] = o[q] * T(g.ih[a]);
        }
        tapply_lo<D, Q, false, T>(td, o, Bt0, Bt0);
#pragma unroll
        for (int q = 0; q < PC; ++q) V[el * VST + (base + LA) * PC + q] = o[q] * T(g.ih[LA]);
      }
    }
    __syncthreads();
    // point pass: derivatives of the pointwise integrand, weighted; slots after:
    // 0 d/dn1, 1 d/dn2, 2 d/dc1, 3 d/dc3 (value tests), 4+a d/d grad n1,
    // 4+D+a d/d grad c1, 4+2D+a d/d grad c3 (gradient tests, scaled by 1/h_a)
    for (int it = tid; it < EB * PC; it += NT) {
      const int l = it / PC, q = it % PC;
      T* x = V + l * VST + q;
      const T n1 = x[0], n2 = x[PC], c1 = x[2 * PC], c3 = x[3 * PC];
      const T d11 = c1 + T(c[K_XT11]), d13 = c3 + T(c[K_XT13]), d21 = c1 + T(c[K_XT21]),
              d22 = n1 + T(c[K_XT22]);
      const bool ok = e0 + l < E;
      if (ok && !(d11 > T(0) && d13 > T(0) && d21 > T(0) && d22 > T(0))) flag |= FLAG_DOMAIN;
      const T i11 = T(1) / d11, i13 = T(1) / d13, i21 = T(1) / d21, i22 = T(1) / d22;
      const T k11 = T(c[K_X011]) * i11, k13 = T(c[K_X013]) * i13, k21 = T(c[K_X021]) * i21,
              k22 = T(c[K_X022]) * i22;
      T wt = vol * T(tb.w[lc]);
      if constexpr (D == 2) {
        wt *= T(tb.w[q]);
      } else {
        wt *= T(tb.w[q % Q]) * T(tb.w[q / Q]);
      }
      T gn1[D], gc1[D], gc3[D], g1[D], g2[D];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        gn1[a] = x[(4 + a) * PC];
        gc1[a] = x[(4 + D + a) * PC];
        gc3[a] = x[(4 + 2 * D + a) * PC];
        g1[a] = x[(AG1 + a) * PC];
        g2[a] = x[(AG2 + a) * PC];
      }
      const T l3 = x[AL3 * PC];
      T w1g1 = T(0), w2g2 = T(0), gc1g1 = T(0), gc1g2 = T(0), gc3g1 = T(0), gn1g2 = T(0);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        w1g1 += (k11 * gc1[a] + k13 * gc3[a]) * g1[a];
        w2g2 += (k21 * gc1[a] - k22 * gn1[a]) * g2[a];
        gc1g1 += gc1[a] * g1[a];
        gc1g2 += gc1[a] * g2[a];
        gc3g1 += gc3[a] * g1[a];
        gn1g2 += gn1[a] * g2[a];
      }
      const T al1 = T(c[K_AL1]), al2 = T(c[K_AL2]);
      const T dn1 = w1g1 + n2 * k22 * i22 * gn1g2 - al1 * c1 * l3;
      const T dn2 = w2g2 - al2 * c1 * l3;
      const T dc1 = -n1 * k11 * i11 * gc1g1 - n2 * k21 * i21 * gc1g2 - (al1 * n1 + al2 * n2) * l3;
      const T dc3 = -n1 * k13 * i13 * gc3g1;
      x[0] = dn1 * wt;
      x[PC] = dn2 * wt;
      x[2 * PC] = dc1 * wt;
      x[3 * PC] = dc3 * wt;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const T sa = wt * T(g.ih[a]);
        x[(4 + a) * PC] = -n2 * k22 * g2[a] * sa;
        x[(4 + D + a) * PC] = (n1 * k11 * g1[a] + n2 * k21 * g2[a]) * sa;
        x[(4 + 2 * D + a) * PC] = n1 * k13 * g1[a] * sa;
      }
      if (want_theta && ok) {
        th[K_X011] += (double)(wt * n1 * gc1g1 * i11);
        th[K_XT11] += (double)(-wt * n1 * k11 * gc1g1 * i11);
        th[K_X013] += (double)(wt * n1 * gc3g1 * i13);
        th[K_XT13] += (double)(-wt * n1 * k13 * gc3g1 * i13);
        th[K_X021] += (double)(wt * n2 * gc1g2 * i21);
        th[K_XT21] += (double)(-wt * n2 * k21 * gc1g2 * i21);
        th[K_X022] += (double)(-wt * n2 * gn1g2 * i22);
        th[K_XT22] += (double)(wt * n2 * k22 * gn1g2 * i22);
        th[K_AL1] += (double)(-wt * n1 * c1 * l3);
        th[K_AL2] += (double)(-wt * n2 * c1 * l3);
      }
    }
    __syncthreads();
    // test integration of this layer for n1, n2, c1, c3: value part and gradient part
    if (prod >= 0) {
      T r[NF], acc[NF], sum[NF];
#pragma unroll
      for (int q = 0; q < PC; ++q) r[q] = V[el * VST + (prod) * PC + q];
      tapply_lo<D, Q, true, T>(r, sum, Bt0, Bt0);    // value test, layer factor B[lc][k]
      T dz[NF];
#pragma unroll
      for (int m = 0; m < NF; ++m) dz[m] = T(0);
      if (grads) {
#pragma unroll
        for (int a = 0; a < D - 1; ++a) {
#pragma unroll
          for (int q = 0; q < PC; ++q) r[q] = V[el * VST + (gslot + a) * PC + q];
          tapply_lo<D, Q, true, T>(r, acc, a == 0 ? tb.Bd : tb.B, a == 1 ? tb.Bd : tb.B);
#pragma unroll
          for (int m = 0; m < NF; ++m) sum[m] += acc[m];
        }
#pragma unroll
        for (int q = 0; q < PC; ++q) r[q] = V[el * VST + (gslot + LA) * PC + q];
        tapply_lo<D, Q, true, T>(r, dz, Bt0, Bt0);
      }
#pragma unroll
      for (int k = 0; k < Q; ++k)
#pragma unroll
        for (int m = 0; m < NF; ++m) R[m + LST * k] += T(tb.B[lc][k]) * sum[m] + T(tb.Bd[lc][k]) * dz[m];
    }
  }

  // ---- faces ------------------------------------------------------------------------
  const bool diss = !(g.llf_cells && s > S_N2);
  T* Fx = sm.buf;   // [EB][FST]: 26 slots of NF points, then the pad
  const int vslot = prod;
  const int dslot = s == S_N1 ? 8 : s == S_C1 ? 9 : s == S_C3 ? 10 : -1;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll 1
  for (int sg = 0; sg < 2; ++sg) {
    const int f = 2 * a + sg;
    __syncthreads();
    const int nb = sm.nb[el][f];
    const double(*Tb0)[CDG2_MAXQ] = tb.B;
    // The traces are formed and published one group at a time, and only what the
    // species pass needs is kept: the normal-derivative averages and the jumps
    // of u and of v.  At 3D p = 3 a scheduling fence separates the groups (all
    // ten trace arrays at once did not fit the registers); elsewhere the
    // compiler may interleave them, which measured faster.
    constexpr bool FENCE = D == 3 && P == 3;
    T sdu[NF], jm[NF], sdv[NF], jv[NF];
    const bool inner = nb >= 0;
    const T* us = U + s * SE + (size_t)(inner ? nb : (live ? e : 0)) * NM;   // in range; unused on boundaries
    const T* ws = W + s * SE + (size_t)(inner ? nb : (live ? e : 0)) * NM;
    // trace of the modes x at end `side` along axis a (d: derivative, scaled by 1/h_a)
    auto own_tr = [&](const T* x, int side, bool d, T* o) {
#pragma unroll
      for (int J = 0; J < NF; ++J) {
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) acc += T(d ? tb.dE[side][i] : tb.E[side][i]) * x[face_mode<D, Q>(a, i, J)];
        o[J] = d ? acc * T(g.ih[a]) : acc;
      }
    };
    auto nb_tr = [&](const T* src, T scale, bool d, T* o) {
#pragma unroll
      for (int J = 0; J < NF; ++J) {
        T acc = T(0);
        if (inner) {
#pragma unroll
          for (int i = 0; i < Q; ++i)
            acc += T(d ? tb.dE[1 - sg][i] : tb.E[1 - sg][i]) * (src[face_mode<D, Q>(a, i, J)] * scale);
        }
        o[J] = d ? acc * T(g.ih[a]) : acc;
      }
    };
    // jump own - neighbour of modes x (own, registers) and src (neighbour), with
    // the mean terms differenced first
    auto jump = [&](const T* x, const T* src, T scale, T* o) {
#pragma unroll
      for (int J = 0; J < NF; ++J) {
        T acc = T(0);
        if (inner) {
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const int m = face_mode<D, Q>(a, i, J);
            const T y = src[m] * scale;
            acc += i == 0 ? x[m] - y : T(tb.E[sg][i]) * x[m] - T(tb.E[1 - sg][i]) * y;
          }
        }
        o[J] = acc;
      }
    };
    // the neighbour's modes: read where they are used at 3D p = 3, else loaded
    // once into registers (three reads per face measured slower there)
    T nbu[FENCE ? 1 : NM], nbw[FENCE ? 1 : NM];
    if constexpr (!FENCE) {
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        nbu[m] = us[m];
        nbw[m] = ws[m];
      }
    }
    const T* su = FENCE ? us : nbu;
    const T* sw = FENCE ? ws : nbw;
    {
      T o[NF];
      if (vslot >= 0) {
        T tr[NF];
        own_tr(u, sg, false, tr);
        tapply_lo<D, Q, false, T>(tr, o, Tb0, Tb0);
#pragma unroll
        for (int t = 0; t < NF; ++t) Fx[el * FST + (vslot) * NF + t] = o[t];
        nb_tr(su, T(1), false, tr);
        tapply_lo<D, Q, false, T>(tr, o, Tb0, Tb0);
#pragma unroll
        for (int t = 0; t < NF; ++t) Fx[el * FST + (4 + vslot) * NF + t] = o[t];
      }
      if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
      {
        T d0[NF], d1[NF];
        own_tr(u, sg, true, d0);
        nb_tr(su, T(1), true, d1);
        if (dslot >= 0) {
          tapply_lo<D, Q, false, T>(d0, o, Tb0, Tb0);
#pragma unroll
          for (int t = 0; t < NF; ++t) Fx[el * FST + (dslot) * NF + t] = o[t];
          tapply_lo<D, Q, false, T>(d1, o, Tb0, Tb0);
#pragma unroll
          for (int t = 0; t < NF; ++t) Fx[el * FST + (dslot + 3) * NF + t] = o[t];
        }
#pragma unroll
        for (int J = 0; J < NF; ++J) sdu[J] = d0[J] + d1[J];
      }
      if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
      // forward jump at the points (boundary: 0)
      jump(u, su, T(1), jm);
      tapply_lo<D, Q, false, T>(jm, o, Tb0, Tb0);
#pragma unroll
      for (int t = 0; t < NF; ++t) Fx[el * FST + (20 + s) * NF + t] = o[t];
      if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
      {
        T d0[NF], d1[NF];
        own_tr(v, sg, true, d0);
        nb_tr(sw, ivol, true, d1);
#pragma unroll
        for (int J = 0; J < NF; ++J) sdv[J] = d0[J] + d1[J];
      }
      if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
      // adjoint jump psi_own - psi_nb (boundary: psi_own)
      if (inner) {
        jump(v, sw, ivol, jv);
      } else {
        own_tr(v, sg, false, jv);
      }
      tapply_lo<D, Q, false, T>(jv, o, Tb0, Tb0);
#pragma unroll
      for (int t = 0; t < NF; ++t) Fx[el * FST + (14 + s) * NF + t] = o[t];
    }
    __syncthreads();
    // face point pass: derivatives of sum_s g_s dpsi_s with respect to the own
    // traces; slots after: 0..5 d/du_o,s (all species), 6 d/d(d_a n1_o),
    // 7 d/d(d_a c1_o), 8 d/d(d_a c3_o); weighted by the tangential weights
    for (int it = tid; it < EB * NF; it += NT) {
      const int l = it / NF, t = it % NF;
      T* x = Fx + l * FST + t;
      const int nbl = sm.nb[l][f];
      const bool ok = e0 + l < E;
      T wt;
      if constexpr (D == 2) {
        wt = T(tb.w[t]);
      } else {
        wt = T(tb.w[t % Q]) * T(tb.w[t / Q]);
      }
      T dps[6], jj[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        dps[q] = x[(14 + q) * NF];
        jj[q] = x[(20 + q) * NF];
      }
      T out_v[6], odn1 = T(0), odc1 = T(0), odc3 = T(0);
#pragma unroll
      for (int q = 0; q < 6; ++q) out_v[q] = T(0);
      if (nbl >= 0) {
        const T so = sg ? T(1) : T(-1);
        const T n1o = x[0], n2o = x[NF], c1o = x[2 * NF], c3o = x[3 * NF];
        const T n1n = x[4 * NF], n2n = x[5 * NF], c1n = x[6 * NF], c3n = x[7 * NF];
        const T dn1o = x[8 * NF], dc1o = x[9 * NF], dc3o = x[10 * NF];
        const T dn1n = x[11 * NF], dc1n = x[12 * NF], dc3n = x[13 * NF];
        const T i11o = T(1) / (c1o + T(c[K_XT11])), i13o = T(1) / (c3o + T(c[K_XT13]));
        const T i21o = T(1) / (c1o + T(c[K_XT21])), i22o = T(1) / (n1o + T(c[K_XT22]));
        const T i11n = T(1) / (c1n + T(c[K_XT11])), i13n = T(1) / (c3n + T(c[K_XT13]));
        const T i21n = T(1) / (c1n + T(c[K_XT21])), i22n = T(1) / (n1n + T(c[K_XT22]));
        const T x11 = T(c[K_X011]), x13 = T(c[K_X013]), x21 = T(c[K_X021]), x22 = T(c[K_X022]);
        const T w1o = so * (x11 * dc1o * i11o + x13 * dc3o * i13o);
        const T w2o = so * (x21 * dc1o * i21o - x22 * dn1o * i22o);
        const T w1n = so * (x11 * dc1n * i11n + x13 * dc3n * i13n);
        const T w2n = so * (x21 * dc1n * i21n - x22 * dn1n * i22n);
        // lam = max(|w1o|, |w2o|, |w1n|, |w2n|), first maximiser
        T lam = fabs(w1o);
        int am = 0;
        if (fabs(w2o) > lam) { lam = fabs(w2o); am = 1; }
        if (fabs(w1n) > lam) { lam = fabs(w1n); am = 2; }
        if (fabs(w2n) > lam) { lam = fabs(w2n); am = 3; }
        T Ll = T(0);   // d Lambda / d lam
#pragma unroll
        for (int q = 0; q < 6; ++q)
          if (!(g.llf_cells && q > S_N2)) {
            out_v[q] = -T(0.5) * lam * dps[q];
            Ll += -T(0.5) * jj[q] * dps[q];
          }
        const T sgn = am == 0 ? (w1o > T(0) ? T(1) : w1o < T(0) ? T(-1) : T(0))
                    : am == 1 ? (w2o > T(0) ? T(1) : w2o < T(0) ? T(-1) : T(0))
                    : am == 2 ? (w1n > T(0) ? T(1) : w1n < T(0) ? T(-1) : T(0))
                              : (w2n > T(0) ? T(1) : w2n < T(0) ? T(-1) : T(0));
        // d Lambda / d w1o, d w2o (own) and d w1n, d w2n (neighbour, parameters only)
        const T A1o = -T(0.5) * n1o * dps[S_N1] + (am == 0 ? Ll * sgn : T(0));
        const T A2o = -T(0.5) * n2o * dps[S_N2] + (am == 1 ? Ll * sgn : T(0));
        const T A1n = -T(0.5) * n1n * dps[S_N1] + (am == 2 ? Ll * sgn : T(0));
        const T A2n = -T(0.5) * n2n * dps[S_N2] + (am == 3 ? Ll * sgn : T(0));
        out_v[S_N1] += -T(0.5) * w1o * dps[S_N1];
        out_v[S_N2] += -T(0.5) * w2o * dps[S_N2];
        // w1o = so (x11 dc1o i11o + x13 dc3o i13o); w2o = so (x21 dc1o i21o - x22 dn1o i22o)
        out_v[S_C1] += A1o * (-so * x11 * dc1o * i11o * i11o) + A2o * (-so * x21 * dc1o * i21o * i21o);
        out_v[S_C3] += A1o * (-so * x13 * dc3o * i13o * i13o);
        out_v[S_N1] += A2o * (so * x22 * dn1o * i22o * i22o);
        odc1 = A1o * so * x11 * i11o + A2o * so * x21 * i21o;
        odc3 = A1o * so * x13 * i13o;
        odn1 = -A2o * so * x22 * i22o;
        if (want_theta && sg == 1 && ok) {
          const T ar = T(g.area[a]) * wt;
          th[K_X011] += (double)(ar * (A1o * so * dc1o * i11o + A1n * so * dc1n * i11n));
          th[K_XT11] += (double)(ar * (-A1o * so * x11 * dc1o * i11o * i11o - A1n * so * x11 * dc1n * i11n * i11n));
          th[K_X013] += (double)(ar * (A1o * so * dc3o * i13o + A1n * so * dc3n * i13n));
          th[K_XT13] += (double)(ar * (-A1o * so * x13 * dc3o * i13o * i13o - A1n * so * x13 * dc3n * i13n * i13n));
          th[K_X021] += (double)(ar * (A2o * so * dc1o * i21o + A2n * so * dc1n * i21n));
          th[K_XT21] += (double)(ar * (-A2o * so * x21 * dc1o * i21o * i21o - A2n * so * x21 * dc1n * i21n * i21n));
          th[K_X022] += (double)(ar * (-A2o * so * dn1o * i22o - A2n * so * dn1n * i22n));
          th[K_XT22] += (double)(ar * (A2o * so * x22 * dn1o * i22o * i22o + A2n * so * x22 * dn1n * i22n * i22n));
        }
      } else if (nbl == -1 || nbl == -2) {
        // inflow fluxes depend on U only through H (derivative 0); parameters:
        // mu1 (Gamma1, n1), mu2 (Gamma2, n2), nu2 (Gamma_{1,in}, c2)
        if (want_theta && ok) {
          const T ar = T(g.area[a]) * wt;
          const T c1o = x[2 * NF];
          if (nbl == -1) {
            if (c1o - T(c[K_C1S]) > T(0)) th[K_MU1] += (double)(ar * T(c[K_BE1]) * dps[S_N1]);
            const int b0 = a == 0 ? 1 : 0;
            const double xc = (cell_coord<D>(g, e0 + l, b0) + tb.x[t % Q]) * g.h[b0];
            if (xc >= g.g1in[0] && xc <= g.g1in[1]) th[K_NU2] += (double)(ar * T(c[K_SIG]) * dps[S_C2]);
          } else {
            if (c1o - T(c[K_C1SS]) > T(0)) th[K_MU2] += (double)(ar * T(c[K_BE2]) * dps[S_N2]);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) x[q * NF] = out_v[q] * wt;
      x[6 * NF] = odn1 * wt;
      x[7 * NF] = odc1 * wt;
      x[8 * NF] = odc3 * wt;
    }
    __syncthreads();
    // species pass: linear face terms applied to v, nonlinear derivatives spread
    {
      const T* x = Fx + el * FST;
      T gp[NF], gh[NF], dp[NF], dh[NF];
#pragma unroll
      for (int t = 0; t < NF; ++t) gp[t] = x[s * NF + t];
      tapply_lo<D, Q, true, T>(gp, gh, Tb0, Tb0);
      const int ds = s == S_N1 ? 6 : s == S_C1 ? 7 : s == S_C3 ? 8 : -1;
      if (ds >= 0) {
#pragma unroll
        for (int t = 0; t < NF; ++t) dp[t] = x[ds * NF + t];
        tapply_lo<D, Q, true, T>(dp, dh, Tb0, Tb0);
      } else {
#pragma unroll
        for (int J = 0; J < NF; ++J) dh[J] = T(0);
      }
      const T ar = T(g.area[a]);
      const T so = sg ? T(1) : T(-1);
      const T pen = T(g.pen_c * tb.liftc * g.ih[a]);   // symmetric fluxes only (host check)
      T G[NF], H[NF], Gu[NF], Hu[NF];
#pragma unroll
      for (int J = 0; J < NF; ++J) {
        T lin = T(0), hh = T(0), linu = T(0), hhu = T(0);
        if (nb >= 0) {
          lin = as * (so * T(0.5) * sdv[J] - pen * jv[J]);
          hh = as * T(0.5) * jv[J] * so * T(g.ih[a]);
          linu = so * T(0.5) * sdu[J] - pen * jm[J];
          hhu = T(0.5) * jm[J] * so * T(g.ih[a]);
        }
        G[J] = ar * (lin + gh[J]);
        H[J] = ar * (hh + dh[J] * T(g.ih[a]));
        Gu[J] = ar * linu;
        Hu[J] = ar * hhu;
      }
#pragma unroll
      for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int J = 0; J < NF; ++J) {
          const int m = face_mode<D, Q>(a, i, J);
          R[m] += T(tb.E[sg][i]) * G[J] + T(tb.dE[sg][i]) * H[J];
          if (want_theta)
            thd += (double)(T(tb.E[sg][i]) * Gu[J] + T(tb.dE[sg][i]) * Hu[J]) * (double)v[m];
        }
    }
  }

  // ---- output, parameter derivatives of the diffusivities ---------------------------
  if (live) {
    const size_t off = s * SE + (size_t)e * NM;
    const T* w0 = W + off;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      T val = cw * w0[m] + cj * R[m];
      if (X2) val += c2 * X2[off + m];
      if (X3) val += c3 * X3[off + m];
      if (!isfinite(val)) flag |= FLAG_NONFINITE;
      out[off + m] = val;
    }
  }
  if (!live) thd = 0.0;
  if (flag) atomicOr(flags, flag);

  // ---- deterministic per-workgroup reduction of the parameter derivatives -----------
  // Through the exchange buffer (free now), JB derivatives per pass: every thread
  // writes its values, then thread j sums derivative j over the threads in a
  // fixed order.  Any workgroup size works (no whole wavefronts needed).
  if (want_theta) {
    constexpr int JB0 = AdjSmem<D, P, T, EB>::N * (int)sizeof(T) / (8 * NT);
    constexpr int JB = JB0 < CDG2_NDIFF ? JB0 : CDG2_NDIFF;
    static_assert(JB >= 1, "exchange buffer holds one derivative per thread");
    double* red = reinterpret_cast<double*>(sm.buf);
#pragma unroll
    for (int j0 = 0; j0 < CDG2_NDIFF; j0 += JB) {
      __syncthreads();
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) {
        const int j = j0 + jj;
        if (j < CDG2_NDIFF) red[jj * NT + tid] = th[j] + (j < 6 && j == s ? thd : 0.0);
      }
      __syncthreads();
      if (tid < JB && j0 + tid < CDG2_NDIFF) {
        double acc = 0.0;
        for (int k = 0; k < NT; ++k) acc += red[tid * NT + k];
        double* dst = part + (size_t)blk * CDG2_NDIFF + j0 + tid;
        *dst = want_theta == 2 ? *dst + acc * (double)cj : acc * (double)cj;
      }
    }
  }
}

template <int D, int P, typename T, int EB>
__global__ void __launch_bounds__(6 * EB)
adj_kernel(const Params* __restrict__ prm, const T* __restrict__ U, const T* __restrict__ W, T* out, T cw, T cj,
           const T* X2, T c2, const T* X3, T c3, double* __restrict__ part, int want_theta,
           int* __restrict__ flags) {
  __shared__ AdjSmem<D, P, T, EB> sm;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  adj_block<D, P, T, EB>(*prm, U, W, out, cw, cj, X2, c2, X3, c3, part, want_theta, flags, blk * EB, blk, sm);
}

// Sum the per-workgroup partials in a fixed order and add them to acc[21].
__global__ void theta_reduce_kernel(const double* __restrict__ part, int nblk, double* __restrict__ acc) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += part[(size_t)b * CDG2_NDIFF + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[j] += red[0];
}

}  // namespace cdg2
