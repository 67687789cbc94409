// CDG2 operator on unstructured triangle meshes (P_k, k = 1, 2, 3), FP64, one thread
// per (element, species).
//
// The discrete operator (Section 3.1 on simplices): basis phi_j = phi^_j o F_K^-1
// with phi^_j orthonormal on the reference triangle for the mean (phi_0 = 1,
// M_K = |K| I); volume integrals with the collapsed Gauss rule of k + 1 points
// per direction; edge integrals with the (k + 1)-point Gauss rule; per interior
// edge the consistency term {a grad u}.n, the symmetry term
// 1/2 a (u_o - u_n) d_n phi, the LLF flux of the chemotactic fluxes, and the
// CDG2 flux A^ = 2 chi_e a r_e|_{K^-}: the lifting of the jump is formed on K^-
// only (the smaller triangle, ties to the lower index; chi_e = 3/2), which for an
// orthonormal basis gives at an edge point x
//   A^.n_o (x) = -(chi_e a / |K^-|) (n^-.n_o) sum_j phi_j^-(x) int_e (u^- - u^+) phi_j^-;
// on Gamma1 / Gamma2 the inflow fluxes of eqs. (7)-(9).  Then f = R / |K|,
// optionally combined with an SSP-RK3 stage in the epilogue.
//
// Mapping: a workgroup owns tri_eb<K>() elements; thread (s, el) keeps the modes and
// the residual of species s of element el in registers.  The nonlinear terms
// go through LDS: the volume points of the workgroup's elements at once, then the
// edges one local edge index at a time.  Point items evaluate the chemotactic
// velocities, fluxes and lambda; species threads integrate them back.
#pragma once

#include <hip/hip_runtime.h>

#include "es_kernel.hpp"   // recip4, shared point-pass helpers

namespace cdg2 {

constexpr int TRI_MAXB = 10;   // P_3
constexpr int TRI_MAXQ = 16;   // (k + 1)^2 volume points
constexpr int TRI_MAXE = 4;    // k + 1 edge points
// Elements per workgroup (6 threads each): 32 (three waves), and 21 for P3 (two
// waves of 63 lanes): P3 runs at 2 waves per SIMD, whose 8 wave slots per CU
// hold two three-wave workgroups (6 slots) but four two-wave ones.
template <int K>
constexpr int tri_eb() { return K == 3 ? 21 : 32; }

// Reference tables (host-built).
struct TriTables {
  double Bv[TRI_MAXQ][TRI_MAXB];             // phi^_j at the volume points
  double Bg[TRI_MAXQ][TRI_MAXB][2];          // reference gradients
  double wv[TRI_MAXQ];                       // weights for the mean (sum 1)
  double Be[3][TRI_MAXE][TRI_MAXB];          // phi^_j at the points of each local edge
  double Bge[3][TRI_MAXE][TRI_MAXB][2];      // reference gradients there
  double ws[TRI_MAXE];                       // edge weights (sum 1)
  double s[TRI_MAXE];                        // edge parameters in [0, 1]
};

// Per-element geometry (device arrays, host-built from the mesh).
struct TriGeo {
  int E;
  const double* jit;     // [E][4]: J^-T row-major (grad = J^-T grad^)
  const double* area;    // [E]
  const double* len;     // [E][3]
  const double* nrm;     // [E][3][2] outward unit normals
  const double* xv;      // [E][3] vertex x coordinates (for Gamma1,in)
  const int* nbr;        // [E][3] neighbour element, -1 Gamma1, -2 Gamma2
  const int* nbe;        // [E][3] the neighbour's local edge
  const int* minus;      // [E][3] 1 if this element is K^- of the edge
  double g1in[2];
};

struct TriParams {
  TriTables tb;
  TriGeo g;
  Coef cf;
};

template <int K>
struct TriSz {
  static constexpr int NB = (K + 1) * (K + 2) / 2, NQ = (K + 1) * (K + 1), NE = K + 1;
  static constexpr int NVQ = 12;   // volume slots: 0 n1 1 n2 2 c1 3 c3 | 4,5 grad n1 | 6,7 grad c1 | 8,9 grad c3 | 10 n3 11 c2
  static constexpr int NFQ = 14;   // edge slots as in the Cartesian kernel
};

// Per-element strides of the exchange slots, odd in doubles: with an even stride
// that is a multiple of 16 doubles (P1 and P3 volume slots) every element of a
// species hits the same LDS bank, a 32-way conflict; odd strides spread the 32
// elements over all banks.
template <int K>
struct TriStride {
  using S = TriSz<K>;
  static constexpr int VS = S::NVQ * S::NQ + 1, FS = S::NFQ * S::NE + 1;
};

template <int K>
struct TriSmem {
  using S = TriSz<K>;
  static constexpr int VOL = tri_eb<K>() * TriStride<K>::VS, FAC = tri_eb<K>() * TriStride<K>::FS;
  static constexpr int N = VOL > FAC ? VOL : FAC;
  double buf[N];
  double etab[3 * S::NE * S::NB * 3];   // edge tables: [edge][point][mode][value, d/dxi, d/deta]
};

// At least 3 waves per SIMD for P1, P2: P2 then fits 152 VGPRs (1.4x faster than
// the 2 waves its free allocation of 172 VGPRs allowed).  P3 at 2 waves: its
// 52 KB of LDS holds a CU to three workgroups anyway, and under the 3-wave
// bound it spilled.
template <int K>
__global__ void __launch_bounds__(6 * tri_eb<K>(), K == 3 ? 2 : 3)
tri_kernel(const TriParams* __restrict__ prm, const double* __restrict__ U, const double* U0, double* out,
           double dt, double ca, double cb, int stage, int* __restrict__ flags) {
  using S = TriSz<K>;
  constexpr int TRI_EB = tri_eb<K>();
  constexpr int NB = S::NB, NQ = S::NQ, NE = S::NE, NT = 6 * TRI_EB;
  constexpr int VS = TriStride<K>::VS, FS = TriStride<K>::FS;
  __shared__ TriSmem<K> sm;
  const TriTables& tb = prm->tb;
  const TriGeo& g = prm->g;
  const double* c = prm->cf.c;
  const int tid = threadIdx.x;
  const int s = tid / TRI_EB, el = tid % TRI_EB;
  const int e0 = blockIdx.x * TRI_EB;
  const int E = g.E;
  const bool live = e0 + el < E;
  const int e = live ? e0 + el : 0;
  const size_t SE = (size_t)E * NB;
  int flag = 0;

  double u[NB], R[NB];
  {
    const double* src = U + s * SE + (size_t)e * NB;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      u[j] = live ? src[j] : 0.0;
      R[j] = 0.0;
    }
  }
  // the edge tables into LDS: the neighbour's local edge index differs from lane
  // to lane, and LDS serves such reads without a memory round trip
  for (int i = tid; i < 3 * NE * NB * 3; i += NT) {
    const int c3 = i % 3, j = (i / 3) % NB, p = (i / (3 * NB)) % NE, k = i / (3 * NB * NE);
    sm.etab[i] = c3 == 0 ? tb.Be[k][p][j] : tb.Bge[k][p][j][c3 - 1];
  }
  const double* et = sm.etab;
  const double jt[4] = {g.jit[4 * e], g.jit[4 * e + 1], g.jit[4 * e + 2], g.jit[4 * e + 3]};
  const double area = g.area[e];
  const double as = c[K_MU1 + s];

  // ---- volume ---------------------------------------------------------------------
  double* V = sm.buf;   // [EB][VS]: NVQ slots of NQ points, then one pad
  const int vslot = s == S_N1 ? 0 : s == S_N2 ? 1 : s == S_C1 ? 2 : s == S_C3 ? 3 : s == S_N3 ? 10 : 11;
  const int gslot = s == S_N1 ? 4 : s == S_C1 ? 6 : s == S_C3 ? 8 : -1;
  double gq[NQ][2];
  {
    double* o = V + el * VS;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double v = 0.0, r0 = 0.0, r1 = 0.0;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        v += tb.Bv[q][j] * u[j];
        r0 += tb.Bg[q][j][0] * u[j];
        r1 += tb.Bg[q][j][1] * u[j];
      }
      gq[q][0] = jt[0] * r0 + jt[1] * r1;
      gq[q][1] = jt[2] * r0 + jt[3] * r1;
      o[vslot * NQ + q] = v;
      if (gslot >= 0) {
        o[gslot * NQ + q] = gq[q][0];
        o[(gslot + 1) * NQ + q] = gq[q][1];
      }
    }
  }
  __syncthreads();
  // point items: chemotactic fluxes F1 (slots 4, 5), F2 (6, 7), alpha term (8)
  for (int it = tid; it < TRI_EB * NQ; it += NT) {
    const int l = it / NQ, q = it % NQ;
    double* x = V + l * VS + q;
    const double n1 = x[0], n2 = x[NQ], c1 = x[2 * NQ], c3 = x[3 * NQ];
    const double d11 = c1 + c[K_XT11], d13 = c3 + c[K_XT13], d21 = c1 + c[K_XT21], d22 = n1 + c[K_XT22];
    if (e0 + l < E && !(d11 > 0.0 && d13 > 0.0 && d21 > 0.0 && d22 > 0.0)) flag |= FLAG_DOMAIN;
    double r11, r13, r21, r22;
    recip4(d11, d13, d21, d22, r11, r13, r21, r22);   // one division for the four
    const double k11 = c[K_X011] * r11, k13 = c[K_X013] * r13, k21 = c[K_X021] * r21, k22 = c[K_X022] * r22;
    double F1[2], F2[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const double gn1 = x[(4 + a) * NQ], gc1 = x[(6 + a) * NQ], gc3 = x[(8 + a) * NQ];
      F1[a] = n1 * (k11 * gc1 + k13 * gc3);
      F2[a] = n2 * (k21 * gc1 - k22 * gn1);
    }
    const double rc = -(c[K_AL1] * n1 + c[K_AL2] * n2) * c1;
    x[4 * NQ] = F1[0];
    x[5 * NQ] = F1[1];
    x[6 * NQ] = F2[0];
    x[7 * NQ] = F2[1];
    x[8 * NQ] = rc;
  }
  __syncthreads();
  {
    // linear reactions: n1 -d1 n1; n2 -d2 n2; n3 (d1 - gamma) n1 + d2 n2; c1 f1 n3 (+ alpha
    // term); c2 -k c2; c3 k c2
    const double kown = s == S_N1 ? -c[K_D1] : s == S_N2 ? -c[K_D2] : s == S_C2 ? -c[K_K] : 0.0;
    const int r0 = s == S_N3 ? 0 : s == S_C1 ? 10 : s == S_C3 ? 11 : 0;
    const double k0 = s == S_N3 ? c[K_D1] - c[K_GAM] : s == S_C1 ? c[K_F1] : s == S_C3 ? c[K_K] : 0.0;
    const double k1 = s == S_N3 ? c[K_D2] : 0.0;
    const int fs = s == S_N2 ? 6 : 4;
    const double fw = s == S_N1 || s == S_N2 ? 1.0 : 0.0, rw = s == S_C1 ? 1.0 : 0.0;
    const double* x = V + el * VS;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double wt = area * tb.wv[q];
      const double f0 = fw * x[fs * NQ + q] - as * gq[q][0];
      const double f1 = fw * x[(fs + 1) * NQ + q] - as * gq[q][1];
      // (J^-T g^) . f = g^ . (J^-1 f): the flux in reference coordinates
      const double h0 = jt[0] * f0 + jt[2] * f1, h1 = jt[1] * f0 + jt[3] * f1;
      const double sv = kown * x[vslot * NQ + q] + k0 * x[r0 * NQ + q] + k1 * x[NQ + q] + rw * x[8 * NQ + q];
#pragma unroll
      for (int j = 0; j < NB; ++j) R[j] += wt * (h0 * tb.Bg[q][j][0] + h1 * tb.Bg[q][j][1] + sv * tb.Bv[q][j]);
    }
  }

  // ---- edges ----------------------------------------------------------------------
  double* Fx = sm.buf;   // [EB][FS]: NFQ slots of NE points, then one pad
  const int fvslot = s == S_N1 ? 0 : s == S_N2 ? 1 : s == S_C1 ? 2 : s == S_C3 ? 3 : -1;
  const int dslot = s == S_N1 ? 8 : s == S_C1 ? 9 : s == S_C3 ? 10 : -1;
#pragma unroll 1
  for (int k = 0; k < 3; ++k) {
    __syncthreads();
    const int nb = live ? g.nbr[3 * e + k] : -3;
    const int kk = nb >= 0 ? g.nbe[3 * e + k] : 0;
    const double nx = g.nrm[6 * e + 2 * k], ny = g.nrm[6 * e + 2 * k + 1];
    double uo[NE], dno[NE], un[NE], dnn[NE];
#pragma unroll
    for (int p = 0; p < NE; ++p) {
      double v = 0.0, r0 = 0.0, r1 = 0.0;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        v += tb.Be[k][p][j] * u[j];
        r0 += tb.Bge[k][p][j][0] * u[j];
        r1 += tb.Bge[k][p][j][1] * u[j];
      }
      uo[p] = v;
      dno[p] = nx * (jt[0] * r0 + jt[1] * r1) + ny * (jt[2] * r0 + jt[3] * r1);
      un[p] = 0.0;
      dnn[p] = 0.0;
    }
    double jn[4] = {0.0, 0.0, 0.0, 0.0};
    if (nb >= 0) {
      const double* src = U + s * SE + (size_t)nb * NB;
      double w[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) w[j] = src[j];
#pragma unroll
      for (int i = 0; i < 4; ++i) jn[i] = g.jit[4 * nb + i];
#pragma unroll
      for (int p = 0; p < NE; ++p) {
        const double* t = et + (kk * NE + (NE - 1 - p)) * NB * 3;   // the neighbour's edge runs the other way
        double v = 0.0, r0 = 0.0, r1 = 0.0;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          v += t[3 * j] * w[j];
          r0 += t[3 * j + 1] * w[j];
          r1 += t[3 * j + 2] * w[j];
        }
        un[p] = v;
        dnn[p] = nx * (jn[0] * r0 + jn[1] * r1) + ny * (jn[2] * r0 + jn[3] * r1);
      }
    }
    if (fvslot >= 0) {
#pragma unroll
      for (int p = 0; p < NE; ++p) {
        Fx[el * FS + fvslot * NE + p] = uo[p];
        Fx[el * FS + (4 + fvslot) * NE + p] = un[p];
      }
    }
    if (dslot >= 0) {
#pragma unroll
      for (int p = 0; p < NE; ++p) {
        Fx[el * FS + dslot * NE + p] = dno[p];
        Fx[el * FS + (dslot + 3) * NE + p] = dnn[p];
      }
    }
    __syncthreads();
    // edge point items: lambda / 2, -(F1 + F1').n / 2, -(F2 + F2').n / 2, or inflow
    for (int it = tid; it < TRI_EB * NE; it += NT) {
      const int l = it / NE, p = it % NE;
      double* x = Fx + l * FS + p;
      const int el2 = e0 + l;
      const int nbl = el2 < E ? g.nbr[3 * el2 + k] : -3;
      const double c1o = x[2 * NE];
      if (nbl >= 0) {
        const double n1o = x[0], n2o = x[NE], c3o = x[3 * NE];
        const double n1n = x[4 * NE], n2n = x[5 * NE], c1n = x[6 * NE], c3n = x[7 * NE];
        const double dn1o = x[8 * NE], dc1o = x[9 * NE], dc3o = x[10 * NE];
        const double dn1n = x[11 * NE], dc1n = x[12 * NE], dc3n = x[13 * NE];
        const double d11o = c1o + c[K_XT11], d13o = c3o + c[K_XT13], d21o = c1o + c[K_XT21], d22o = n1o + c[K_XT22];
        const double d11n = c1n + c[K_XT11], d13n = c3n + c[K_XT13], d21n = c1n + c[K_XT21], d22n = n1n + c[K_XT22];
        if (!(d11o > 0.0 && d13o > 0.0 && d21o > 0.0 && d22o > 0.0 && d11n > 0.0 && d13n > 0.0 && d21n > 0.0 &&
              d22n > 0.0))
          flag |= FLAG_DOMAIN;
        double r11o, r13o, r21o, r22o, r11n, r13n, r21n, r22n;
        recip4(d11o, d13o, d21o, d22o, r11o, r13o, r21o, r22o);
        recip4(d11n, d13n, d21n, d22n, r11n, r13n, r21n, r22n);
        const double w1o = c[K_X011] * dc1o * r11o + c[K_X013] * dc3o * r13o;
        const double w2o = c[K_X021] * dc1o * r21o - c[K_X022] * dn1o * r22o;
        const double w1n = c[K_X011] * dc1n * r11n + c[K_X013] * dc3n * r13n;
        const double w2n = c[K_X021] * dc1n * r21n - c[K_X022] * dn1n * r22n;
        const double lam = fmax(fmax(fabs(w1o), fabs(w2o)), fmax(fabs(w1n), fabs(w2n)));
        x[0] = 0.5 * lam;
        x[NE] = -0.5 * (n1o * w1o + n1n * w1n);
        x[2 * NE] = -0.5 * (n2o * w2o + n2n * w2n);
      } else {
        double q1 = 0.0, q2 = 0.0, q5 = 0.0;
        if (nbl == -1) {
          if (c1o - c[K_C1S] > 0.0) q1 = c[K_MU1] * c[K_BE1];
          const double xa = g.xv[3 * el2 + k], xb = g.xv[3 * el2 + (k + 1) % 3];
          const double xc = xa + tb.s[p] * (xb - xa);
          if (xc >= g.g1in[0] && xc <= g.g1in[1]) q5 = c[K_NU2] * c[K_SIG];
        } else if (nbl == -2) {
          if (c1o - c[K_C1SS] > 0.0) q2 = c[K_MU2] * c[K_BE2];
        }
        x[0] = 0.0;
        x[NE] = 0.0;
        x[2 * NE] = 0.0;
        x[3 * NE] = q1;
        x[4 * NE] = q2;
        x[5 * NE] = q5;
      }
    }
    __syncthreads();
    // species pass
    if (live) {
      const double* x = Fx + el * FS;
      const double len = g.len[3 * e + k];
      double G[NE], H[NE];
      if (nb >= 0) {
        const bool mine = g.minus[3 * e + k] != 0;
        const double am = mine ? area : g.area[nb];
        const double sgn = mine ? 1.0 : -1.0;   // n^- . n_o
        // K^-'s basis at the edge points (in this element's point order)
        double Bm[NE][NB];
#pragma unroll
        for (int p = 0; p < NE; ++p)
#pragma unroll
          for (int j = 0; j < NB; ++j) Bm[p][j] = et[(((mine ? k : kk) * NE + (mine ? p : NE - 1 - p)) * NB + j) * 3];
        double gm[NE], proj[NB];
#pragma unroll
        for (int p = 0; p < NE; ++p) gm[p] = sgn * (uo[p] - un[p]) * (len * tb.ws[p]);   // (u^- - u^+) w L
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          double a = 0.0;
#pragma unroll
          for (int p = 0; p < NE; ++p) a += gm[p] * Bm[p][j];
          proj[j] = a;
        }
        const double fa = -(1.5 * as / am) * sgn;
#pragma unroll
        for (int p = 0; p < NE; ++p) {
          double rt = 0.0;
#pragma unroll
          for (int j = 0; j < NB; ++j) rt += Bm[p][j] * proj[j];
          const double jm = uo[p] - un[p];
          double gv = 0.5 * as * (dno[p] + dnn[p]) + fa * rt - x[p] * jm;
          if (s == S_N1) gv += x[NE + p];
          if (s == S_N2) gv += x[2 * NE + p];
          G[p] = len * tb.ws[p] * gv;
          H[p] = len * tb.ws[p] * 0.5 * as * jm;
        }
      } else {
#pragma unroll
        for (int p = 0; p < NE; ++p) {
          const double q = s == S_N1 ? x[3 * NE + p] : s == S_N2 ? x[4 * NE + p] : s == S_C2 ? x[5 * NE + p] : 0.0;
          G[p] = len * tb.ws[p] * q;
          H[p] = 0.0;
        }
      }
#pragma unroll
      for (int p = 0; p < NE; ++p)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const double r0 = tb.Bge[k][p][j][0], r1 = tb.Bge[k][p][j][1];
          const double dphi = nx * (jt[0] * r0 + jt[1] * r1) + ny * (jt[2] * r0 + jt[3] * r1);
          R[j] += G[p] * tb.Be[k][p][j] + H[p] * dphi;
        }
    }
  }

  // ---- M^{-1}, stage combination, store -------------------------------------------------
  if (live) {
    double* dst = out + s * SE + (size_t)e * NB;
    const double ia = 1.0 / area;
    const bool combine = stage != 0 && ca != 0.0;   // U0 is read (and non-null) only then
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      double v = R[j] * ia;
      if (stage != 0) v = cb * (u[j] + dt * v);
      if (combine) v += ca * U0[s * SE + (size_t)e * NB + j];
      if (!isfinite(v)) flag |= FLAG_NONFINITE;
      dst[j] = v;
    }
  }
  if (flag) atomicOr(flags, flag);
}

}  // namespace cdg2
