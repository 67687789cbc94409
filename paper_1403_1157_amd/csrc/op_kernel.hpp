// Fused CDG2 operator kernel: f = M^{-1} L_h(U) for EPW cells per workgroup,
// optionally combined with an SSP-RK3 stage in the epilogue so that f never
// reaches HBM.
//
// Per cell (Section 3.1):
//   volume:   int_K (F(U) - A grad U) : grad phi + S(U) phi
//   faces:    int_e {A grad phi}:[[U]] + {A grad U}:[[phi]] - (F^ - A^):[[phi]]
// with the local Lax-Friedrichs flux F^ and the CDG2 flux
// A^ = 2 chi_e (A r_e([[U]]))|_{K^-_e}.  On Cartesian cells with the orthonormal
// Legendre basis, the lifting of a face jump on K^- (the low-side cell) has the
// trace -(liftc / (2h)) [[U]], liftc = sum_i phi_i(1)^2, so A^ . n^- is
// -chi_e a liftc / h (u^- - u^+); it is formed from K^-'s end values only.
//
// Each cell evaluates all of its faces from its own side, written in the cell's
// outward normal n_o (the expression is symmetric in the two sides):
//   R_j += int_e 1/2 a (u_o - u_n) d_{n_o} phi_j
//        + [ 1/2 a (d_{n_o} u_o + d_{n_o} u_n) - pen (u_o - u_n)
//            - 1/2 (F_o + F_n).n_o - 1/2 lam (u_o - u_n) ] phi_j.
// All terms linear in U (volume diffusion, linear reactions, consistency,
// symmetry and lifting terms) are applied exactly in modal form; the nonlinear
// ones (chemotactic fluxes, alpha n c reactions, LLF flux) are evaluated at the
// Gauss points.  Work is organised in LDS phases separated by barriers; every
// thread loops over an item space of the phase.
#pragma once

#include "op_common.hpp"

namespace cdg2 {

template <int D, int P, typename T, int EPW, int NT>
struct OpKernel {
  using Z = Sz<D, P>;
  static constexpr int Q = Z::Q, NM = Z::NM, NQ = Z::NQ, NF = Z::NF, NFACE = Z::NFACE;
  static constexpr int NPV = 4 + 3 * D;   // n1, n2, c1, c3 values; grad n1, c1, c3

  struct Smem {
    T U[EPW][6][NM];
    T R[EPW][6][NM];
    T V[EPW][NPV][NQ];
    T Tr[EPW][NFACE][6][5][NF];      // own u, own d_a u, neighbour u, neighbour d_a u, u_o - u_n
    T Fp[EPW][NFACE][6][NF];         // weighted nonlinear face flux at face points
    T G[EPW][NFACE][6][2][NF];       // modal face coefficients (value / normal-derivative tests)
    int nb[EPW][NFACE];
    int cell[EPW];
  };
};

// stage == 0: out = f(U).  stage != 0: out = ca * U0 + cb * (U + dt f(U)) (U0 may
// alias out; each cell reads its own U0 entries before writing them).
template <int D, int P, typename T, int EPW, int NT>
__global__ void __launch_bounds__(NT)
op_kernel(const Params* __restrict__ prm, const T* __restrict__ U, const T* U0,
          T* out, T dt, T ca, T cb, int stage, int* __restrict__ flags) {
  const Tables& tb = prm->tb;
  const Geo& g = prm->g;
  const Coef& cf = prm->cf;
  using K = OpKernel<D, P, T, EPW, NT>;
  constexpr int Q = K::Q, NM = K::NM, NQ = K::NQ, NF = K::NF, NFACE = K::NFACE, NPV = K::NPV;
  __shared__ typename K::Smem sm;
  const int tid = threadIdx.x;
  const int nblk = gridDim.x;
  const int blk = xcd_block(blockIdx.x, nblk);
  const int e0 = blk * EPW;
  const int E = g.E;
  const size_t SE = (size_t)E * NM;   // species stride
  const double* c = cf.c;
  int flag = 0;

  // ---- phase 0: load own modes, neighbour table -------------------------------
  for (int it = tid; it < 6 * EPW * NM; it += NT) {
    int s = it / (EPW * NM), off = it % (EPW * NM);
    int el = off / NM, m = off % NM;
    int e = e0 + el;
    sm.U[el][s][m] = e < E ? U[s * SE + (size_t)e0 * NM + off] : T(0);
  }
  for (int it = tid; it < EPW * NFACE; it += NT) {
    int el = it / NFACE, f = it % NFACE;
    int e = e0 + el;
    sm.nb[el][f] = e < E ? neighbour<D>(g, e, f) : -3;
  }
  __syncthreads();

  // ---- phase 1: linear modal residual | point values | face traces -------------
  {
    constexpr int nB = EPW * NPV, nA = EPW * 6, nC = EPW * NFACE * 6 * NF;
    for (int it = tid; it < nB + nA + nC; it += NT) {
      if (it < nB) {
        // point values / physical gradients at the volume Gauss points
        int el = it / NPV, qty = it % NPV;
        T in[NM], o[NM];
        int sp;
        const double(*Mx)[CDG2_MAXQ] = tb.B;
        const double(*My)[CDG2_MAXQ] = tb.B;
        const double(*Mz)[CDG2_MAXQ] = tb.B;
        T scale = T(1);
        if (qty < 4) {
          sp = qty == 0 ? S_N1 : qty == 1 ? S_N2 : qty == 2 ? S_C1 : S_C3;
        } else {
          int k = qty - 4, gsp = k / D, a = k % D;
          sp = gsp == 0 ? S_N1 : gsp == 1 ? S_C1 : S_C3;
          if (a == 0) Mx = tb.Bd;
          if (a == 1) My = tb.Bd;
          if (a == 2) Mz = tb.Bd;
          scale = T(g.ih[a]);
        }
#pragma unroll
        for (int m = 0; m < NM; ++m) in[m] = sm.U[el][sp][m];
        tapply<D, Q, false, T>(in, o, Mx, My, Mz);
#pragma unroll
        for (int m = 0; m < NQ; ++m) sm.V[el][qty][m] = o[m] * scale;
      } else if (it < nB + nA) {
        // linear part of the residual, exact in modal form:
        //   -a_s int grad u . grad phi  = -a_s |K| sum_a h_a^-2 (S along a) U
        //   linear reactions (mode-wise, M = |K| I)
        int k = it - nB, el = k / 6, s = k % 6;
        T u[NM], r[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m) u[m] = sm.U[el][s][m];
        const T as = T(c[K_MU1 + s]);
        const T vol = T(g.vol);
#pragma unroll
        for (int m = 0; m < NM; ++m) {
          T acc = T(0);
#pragma unroll
          for (int a = 0; a < D; ++a) {
            const int st = ipow(Q, a);
            const int ia = (m / st) % Q;
            const int base = m - ia * st;
            T sa = T(0);
#pragma unroll
            for (int j = 0; j < Q; ++j) sa += T(tb.S[ia][j]) * u[base + j * st];
            acc += T(g.ih[a] * g.ih[a]) * sa;
          }
          r[m] = -as * vol * acc;
        }
        // S_lin: n1: -d1 n1; n2: -d2 n2; n3: (d1 - gamma) n1 + d2 n2; c1: f1 n3;
        //        c2: -k c2; c3: k c2   (alpha n c terms are at the points)
#pragma unroll
        for (int m = 0; m < NM; ++m) {
          T src;
          switch (s) {
            case S_N1: src = -T(c[K_D1]) * sm.U[el][S_N1][m]; break;
            case S_N2: src = -T(c[K_D2]) * sm.U[el][S_N2][m]; break;
            case S_N3:
              src = T(c[K_D1] - c[K_GAM]) * sm.U[el][S_N1][m] + T(c[K_D2]) * sm.U[el][S_N2][m];
              break;
            case S_C1: src = T(c[K_F1]) * sm.U[el][S_N3][m]; break;
            case S_C2: src = -T(c[K_K]) * sm.U[el][S_C2][m]; break;
            default: src = T(c[K_K]) * sm.U[el][S_C2][m]; break;
          }
          sm.R[el][s][m] = r[m] + vol * src;
        }
      } else {
        // tangential-modal traces on face f: value and d/dx_a, own and neighbour
        int k = it - nB - nA;
        int J = k % NF;
        int s = (k / NF) % 6;
        int f = (k / (NF * 6)) % NFACE;
        int el = k / (NF * 6 * NFACE);
        int a = f >> 1, sg = f & 1;
        T uo = T(0), duo = T(0), un = T(0), dun = T(0), jmp = T(0);
        T vo[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          T v = sm.U[el][s][face_mode<D, Q>(a, i, J)];
          vo[i] = v;
          uo += T(tb.E[sg][i]) * v;
          duo += T(tb.dE[sg][i]) * v;
        }
        int nb = sm.nb[el][f];
        if (nb >= 0) {
          const T* Un = U + s * SE + (size_t)nb * NM;
          // the jump u_o - u_n is formed mode by mode: the i = 0 terms (value 1 at
          // both ends) cancel exactly instead of leaving the rounding of O(1) traces
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            T v = Un[face_mode<D, Q>(a, i, J)];
            un += T(tb.E[1 - sg][i]) * v;
            dun += T(tb.dE[1 - sg][i]) * v;
            jmp += i == 0 ? vo[0] - v : T(tb.E[sg][i]) * vo[i] - T(tb.E[1 - sg][i]) * v;
          }
        }
        const T ih = T(g.ih[a]);
        sm.Tr[el][f][s][0][J] = uo;
        sm.Tr[el][f][s][1][J] = duo * ih;
        sm.Tr[el][f][s][2][J] = un;
        sm.Tr[el][f][s][3][J] = dun * ih;
        sm.Tr[el][f][s][4][J] = jmp;
      }
    }
  }
  __syncthreads();

  // ---- phase 2: pointwise physics at volume and face points ---------------------
  {
    constexpr int nA = EPW * NQ, nB = EPW * NFACE * NF;
    const T x11 = T(c[K_X011]), x13 = T(c[K_X013]), x21 = T(c[K_X021]), x22 = T(c[K_X022]);
    const T t11 = T(c[K_XT11]), t13 = T(c[K_XT13]), t21 = T(c[K_XT21]), t22 = T(c[K_XT22]);
    for (int it = tid; it < nA + nB; it += NT) {
      if (it < nA) {
        int el = it / NQ, qp = it % NQ;
        T n1 = sm.V[el][0][qp], n2 = sm.V[el][1][qp], c1 = sm.V[el][2][qp], c3 = sm.V[el][3][qp];
        T gn1[D], gc1[D], gc3[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          gn1[a] = sm.V[el][4 + a][qp];
          gc1[a] = sm.V[el][4 + D + a][qp];
          gc3[a] = sm.V[el][4 + 2 * D + a][qp];
        }
        T d11 = c1 + t11, d13 = c3 + t13, d21 = c1 + t21, d22 = n1 + t22;
        if (!(d11 > T(0) && d13 > T(0) && d21 > T(0) && d22 > T(0))) flag |= FLAG_DOMAIN;
        T k11 = x11 / d11, k13 = x13 / d13, k21 = x21 / d21, k22 = x22 / d22;
        T wt = T(g.vol) * vol_weight<D, Q, T>(tb, qp);
#pragma unroll
        for (int a = 0; a < D; ++a) {
          T w1 = k11 * gc1[a] + k13 * gc3[a];
          T w2 = k21 * gc1[a] - k22 * gn1[a];
          sm.V[el][a][qp] = n1 * w1 * wt * T(g.ih[a]);
          sm.V[el][D + a][qp] = n2 * w2 * wt * T(g.ih[a]);
        }
        sm.V[el][2 * D][qp] = -(T(c[K_AL1]) * n1 + T(c[K_AL2]) * n2) * c1 * wt;
      } else {
        int k = it - nA;
        int t = k % NF, f = (k / NF) % NFACE, el = k / (NF * NFACE);
        int a = f >> 1, sg = f & 1;
        int nb = sm.nb[el][f];
        T phi[NF];
#pragma unroll
        for (int J = 0; J < NF; ++J) phi[J] = tang_basis<D, Q, T>(tb, J, t);
        T wt = tang_weight<D, Q, T>(tb, t);
        T uo[6], un[6], jp[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) {
          T a0 = T(0), a1 = T(0), a2 = T(0);
#pragma unroll
          for (int J = 0; J < NF; ++J) {
            a0 += phi[J] * sm.Tr[el][f][s][0][J];
            a1 += phi[J] * sm.Tr[el][f][s][2][J];
            a2 += phi[J] * sm.Tr[el][f][s][4][J];
          }
          uo[s] = a0;
          un[s] = a1;
          jp[s] = a2;
        }
        T gflux[6];
        if (nb >= 0) {
          T dn1o = T(0), dc1o = T(0), dc3o = T(0), dn1n = T(0), dc1n = T(0), dc3n = T(0);
#pragma unroll
          for (int J = 0; J < NF; ++J) {
            dn1o += phi[J] * sm.Tr[el][f][S_N1][1][J];
            dc1o += phi[J] * sm.Tr[el][f][S_C1][1][J];
            dc3o += phi[J] * sm.Tr[el][f][S_C3][1][J];
            dn1n += phi[J] * sm.Tr[el][f][S_N1][3][J];
            dc1n += phi[J] * sm.Tr[el][f][S_C1][3][J];
            dc3n += phi[J] * sm.Tr[el][f][S_C3][3][J];
          }
          const T so = sg ? T(1) : T(-1);
          T d11o = uo[S_C1] + t11, d13o = uo[S_C3] + t13, d21o = uo[S_C1] + t21, d22o = uo[S_N1] + t22;
          T d11n = un[S_C1] + t11, d13n = un[S_C3] + t13, d21n = un[S_C1] + t21, d22n = un[S_N1] + t22;
          if (!(d11o > T(0) && d13o > T(0) && d21o > T(0) && d22o > T(0) && d11n > T(0) &&
                d13n > T(0) && d21n > T(0) && d22n > T(0)))
            flag |= FLAG_DOMAIN;
          T w1o = so * (x11 * dc1o / d11o + x13 * dc3o / d13o);
          T w2o = so * (x21 * dc1o / d21o - x22 * dn1o / d22o);
          T w1n = so * (x11 * dc1n / d11n + x13 * dc3n / d13n);
          T w2n = so * (x21 * dc1n / d21n - x22 * dn1n / d22n);
          T lam = fmax(fmax(fabs(w1o), fabs(w2o)), fmax(fabs(w1n), fabs(w2n)));
          T hl = T(0.5) * lam;
#pragma unroll
          for (int s = 0; s < 6; ++s) {
            T diss = (g.llf_cells && s > S_N2) ? T(0) : hl * jp[s];
            gflux[s] = -diss;
          }
          gflux[S_N1] -= T(0.5) * (uo[S_N1] * w1o + un[S_N1] * w1n);
          gflux[S_N2] -= T(0.5) * (uo[S_N2] * w2o + un[S_N2] * w2n);
        } else {
          // inflow boundary fluxes (eqs. (7)-(9)), into the domain
#pragma unroll
          for (int s = 0; s < 6; ++s) gflux[s] = T(0);
          if (nb == -1) {
            if (uo[S_C1] - T(c[K_C1S]) > T(0)) gflux[S_N1] = T(c[K_MU1] * c[K_BE1]);
            // first tangential coordinate of the face point
            int b0 = a == 0 ? 1 : 0;
            int tb0 = t % Q;
            int e = e0 + el;
            double x = (cell_coord<D>(g, e, b0) + tb.x[tb0]) * g.h[b0];
            if (x >= g.g1in[0] && x <= g.g1in[1]) gflux[S_C2] = T(c[K_NU2] * c[K_SIG]);
          } else if (nb == -2) {
            if (uo[S_C1] - T(c[K_C1SS]) > T(0)) gflux[S_N2] = T(c[K_MU2] * c[K_BE2]);
          }
        }
#pragma unroll
        for (int s = 0; s < 6; ++s) sm.Fp[el][f][s][t] = gflux[s] * wt;
      }
    }
  }
  __syncthreads();

  // ---- phase 3: volume test integration (n1, n2, c1) | face modal coefficients ---
  {
    constexpr int nA = EPW * 3, nB = EPW * NFACE * 6 * NF;
    for (int it = tid; it < nA + nB; it += NT) {
      if (it < nA) {
        int el = it / 3, w = it % 3;
        T r[NM], acc[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m) acc[m] = T(0);
        if (w < 2) {
          // int F . grad phi, F already weighted and scaled by h_a^-1
#pragma unroll
          for (int a = 0; a < D; ++a) {
            T in[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) in[q] = sm.V[el][w * D + a][q];
            tapply<D, Q, true, T>(in, r, a == 0 ? tb.Bd : tb.B, a == 1 ? tb.Bd : tb.B,
                                  a == 2 ? tb.Bd : tb.B);
#pragma unroll
            for (int m = 0; m < NM; ++m) acc[m] += r[m];
          }
        } else {
          T in[NQ];
#pragma unroll
          for (int q = 0; q < NQ; ++q) in[q] = sm.V[el][2 * D][q];
          tapply<D, Q, true, T>(in, acc, tb.B, tb.B, tb.B);
        }
        int sp = w == 0 ? S_N1 : w == 1 ? S_N2 : S_C1;
#pragma unroll
        for (int m = 0; m < NM; ++m) sm.R[el][sp][m] += acc[m];
      } else {
        int k = it - nA;
        int J = k % NF, s = (k / NF) % 6, f = (k / (NF * 6)) % NFACE, el = k / (NF * 6 * NFACE);
        int a = f >> 1, sg = f & 1;
        int nb = sm.nb[el][f];
        T gh = T(0);
#pragma unroll
        for (int t = 0; t < NF; ++t) gh += tang_basis<D, Q, T>(tb, J, t) * sm.Fp[el][f][s][t];
        T G = T(0), H = T(0);
        if (nb >= 0) {
          const T as = T(c[K_MU1 + s]);
          const T so = sg ? T(1) : T(-1);
          T duo = sm.Tr[el][f][s][1][J], dun = sm.Tr[el][f][s][3][J];
          T jmp = sm.Tr[el][f][s][4][J];
          T pen = T(g.chi_e * tb.liftc * g.ih[a]) * as;
          G = so * T(0.5) * as * (duo + dun) - pen * jmp;
          H = T(0.5) * as * jmp * so * T(g.ih[a]);
        }
        const T ar = T(g.area[a]);
        sm.G[el][f][s][0][J] = ar * (G + gh);
        sm.G[el][f][s][1][J] = ar * H;
      }
    }
  }
  __syncthreads();

  // ---- phase 4: spread face terms, M^{-1}, RK stage combination, store ----------
  {
    const T ivol = T(1.0 / g.vol);
    for (int it = tid; it < 6 * EPW * NM; it += NT) {
      int s = it / (EPW * NM), off = it % (EPW * NM);
      int el = off / NM, m = off % NM;
      int e = e0 + el;
      if (e >= E) continue;
      T R = sm.R[el][s][m];
#pragma unroll
      for (int f = 0; f < NFACE; ++f) {
        int a = f >> 1, sg = f & 1;
        int st = ipow(Q, a);
        int ia = (m / st) % Q;
        int J;
        if constexpr (D == 2) {
          J = a == 0 ? m / Q : m % Q;
        } else {
          int i0 = m % Q, i1 = (m / Q) % Q, i2 = m / (Q * Q);
          J = a == 0 ? i1 + Q * i2 : a == 1 ? i0 + Q * i2 : i0 + Q * i1;
        }
        R += T(tb.E[sg][ia]) * sm.G[el][f][s][0][J] + T(tb.dE[sg][ia]) * sm.G[el][f][s][1][J];
      }
      T fv = R * ivol;
      size_t gi = s * SE + (size_t)e0 * NM + off;
      T v;
      if (stage == 0) {
        v = fv;
      } else {
        v = cb * (sm.U[el][s][m] + dt * fv);
        if (ca != T(0)) v += ca * U0[gi];
      }
      if (!isfinite(v)) flag |= FLAG_NONFINITE;
      out[gi] = v;
    }
  }
  if (flag) atomicOr(flags, flag);
}

}  // namespace cdg2
