// CDG2 operator on unstructured tetrahedral meshes (P_k, k = 1, 2, 3), FP64, one
// thread per (element, species).
//
// The discrete operator (Section 3.1 on tetrahedra, the element of the paper's 3D
// runs): basis phi_j = phi^_j o F_K^-1 with phi^_j orthonormal on the reference
// tetrahedron for the mean (phi_0 = 1, M_K = |K| I); volume integrals with a
// fully symmetric rule of 4, 14, 24 points (exact for degree 2k); face
// integrals with a fully symmetric triangle rule of degree 2k, so both elements
// of a face evaluate at the same physical points: the neighbour's point index is
// the own index under one of the six vertex permutations (orientation, host
// computed from the shared vertex ids).  Per interior face: the consistency term
// {a grad u}.n, the symmetry term 1/2 a (u_o - u_n) d_n phi, the LLF flux of the
// chemotactic fluxes and the CDG2 flux A^ = 2 chi_e a r_e|_{K^-} with the lifting
// formed on K^- only (the smaller tetrahedron, ties to the lower index;
// chi_e = 2), which for an orthonormal basis gives at a face point x
//   A^.n_o (x) = -(chi_e a / |K^-|) (n^-.n_o) sum_j phi_j^-(x) int_e (u^- - u^+) phi_j^-;
// on Gamma1 / Gamma2 the inflow fluxes of eqs. (7)-(9).  Then f = R / |K|,
// optionally combined with an SSP-RK3 stage in the epilogue.
//
// Mapping: a workgroup owns tet_eb<K>() elements; thread (s, el) keeps the modes and
// the residual of species s of element el in registers.  The nonlinear terms go
// through LDS: the volume points in chunks of TetSz::QC, then the faces one
// local face index at a time (all its points at once).  The neighbour's local
// face and orientation differ from lane to lane, so its face tables are read per
// lane (from LDS for P1 and P2).  Point loops are not unrolled (the mode loops
// are): unrolled, the table reads of P3 exhaust the scalar registers.
#pragma once

#include <hip/hip_runtime.h>

#include "es_kernel.hpp"   // recip4, coefficient indices, flags

namespace cdg2 {

constexpr int TET_MAXB = 20;   // P_3
constexpr int TET_MAXQ = 24;   // points of the symmetric volume rule (degree 2k)
constexpr int TET_MAXF = 12;   // points of the symmetric face rule (degree 2k)
// Elements per workgroup (6 threads each): 32 for P1 (three waves at 3 waves
// per SIMD); 21 for P2 (two waves of 63 lanes: at 2 waves per SIMD four such
// workgroups fill a CU's 8 wave slots, where three-wave ones left two idle);
// 19 for P3, whose face table then fits in LDS beside the exchange slots (two
// workgroups per CU).
template <int K>
constexpr int tet_eb() { return K == 3 ? 19 : K == 2 ? 21 : 32; }

// Reference tables (host-built).
struct TetTables {
  double Bv[TET_MAXQ][TET_MAXB];              // phi^_j at the volume points
  double Bg[TET_MAXQ][TET_MAXB][3];           // reference gradients
  double wv[TET_MAXQ];                        // weights for the mean (sum 1)
  double Bf[4][TET_MAXF][TET_MAXB];           // phi^_j at the points of each local face
  double Bgf[4][TET_MAXF][TET_MAXB][3];       // reference gradients there
  double wf[TET_MAXF];                        // face weights for the mean (sum 1)
  double fbary[TET_MAXF][3];                  // barycentric coordinates of the face points
  int perm[6][TET_MAXF];                      // point index under each vertex permutation
  double ftab[4][TET_MAXF][TET_MAXB][4];      // Bf and Bgf interleaved: [value, d/dxi, d/deta, d/dzeta]
};

// Per-element geometry and topology (device arrays, host-built from the mesh).
struct TetGeo {
  int E;
  const double* jit;     // [E][9]: J^-T row-major (grad = J^-T grad^)
  const double* vol;     // [E]
  const double* area;    // [E][4]
  const double* nrm;     // [E][4][3] outward unit normals
  const double* xv;      // [E][4] vertex x coordinates (for Gamma1,in)
  const int* nbr;        // [E][4] neighbour element, -1 Gamma1, -2 Gamma2
  const int* nbe;        // [E][4] the neighbour's local face
  const int* minus;      // [E][4] 1 if this element is K^- of the face
  const int* ori;        // [E][4] orientation: own point p is the neighbour's point perm[ori][p]
  double g1in[2];
};

struct TetParams {
  TetTables tb;
  TetGeo g;
  Coef cf;
};

constexpr int tet_face_points(int K) { return K == 1 ? 3 : K == 2 ? 6 : 12; }

template <int K>
struct TetSz {
  static constexpr int NB = (K + 1) * (K + 2) * (K + 3) / 6, NQ = K == 1 ? 4 : K == 2 ? 14 : 24;
  static constexpr int NF = tet_face_points(K);
  static constexpr int QC = K == 1 ? 4 : K == 2 ? 7 : 8;   // volume points per LDS chunk
  static_assert(NQ % QC == 0, "volume chunks");
  // volume slots: 0 n1 1 n2 2 c1 3 c3 | 4..6 grad n1 | 7..9 grad c1 | 10..12 grad c3 | 13 n3 14 c2
  static constexpr int NVQ = 15;
  static constexpr int NFQ = 14;   // face slots as in the other kernels
};

// The interleaved face table lives in LDS (1.7, 7.9 and 30.8 KB for P1, P2, P3):
// the neighbour's local face and orientation differ from lane to lane, and read
// through the cache the P3 table kept the vector-memory return path busy (each
// lane reads the whole table once per application).  Each (face, point) row of
// NB x 4 values is padded by two doubles: unpadded, the rows of P3 (160 dwords)
// and P2 (80) start on one or two LDS banks, and lanes reading the same mode of
// different rows collide (a 4.5-fold conflict measured at P3).
template <int K>
constexpr int tet_frow() { return TetSz<K>::NB * 4 + 2; }

// Per-element (and per-thread) strides of the LDS slots, odd in doubles: the
// plain even strides (15 QC at P1 and P3, 14 NF, 2 NF doubles) put the elements
// of a species on 2 to 16 banks (up to a 16-way conflict); odd strides spread
// them over all.  (15 QC is odd at P2 and stays as it is.)
template <int K>
struct TetStride {
  using S = TetSz<K>;
  static constexpr int VS = (S::NVQ * S::QC) | 1, FS = (S::NFQ * S::NF) | 1, PS = 2 * S::NF + 1;
};

template <int K>
struct TetSmem {
  using S = TetSz<K>;
  static constexpr int VOL = tet_eb<K>() * TetStride<K>::VS, FAC = tet_eb<K>() * TetStride<K>::FS;
  static constexpr int N = VOL > FAC ? VOL : FAC;
  double buf[N];
  double park[6 * tet_eb<K>() * TetStride<K>::PS];   // each thread's face jump and normal-derivative sum
  double ftab[4 * S::NF * tet_frow<K>()];   // [face][point] rows of [mode][4], padded
};

// Two waves per SIMD (the registers of P2 and P3 and the LDS of P3 allow no more).
template <int K>
__global__ void __launch_bounds__(6 * tet_eb<K>(), 2)
tet_kernel(const TetParams* __restrict__ prm, const double* __restrict__ U, const double* U0, double* out,
           double dt, double ca, double cb, int stage, int* __restrict__ flags) {
  using S = TetSz<K>;
  constexpr int TET_EB = tet_eb<K>();
  constexpr int NB = S::NB, NQ = S::NQ, NF = S::NF, QC = S::QC, NT = 6 * TET_EB;
  constexpr int VS = TetStride<K>::VS, FS = TetStride<K>::FS, PS = TetStride<K>::PS;
  __shared__ TetSmem<K> sm;
  const TetTables& tb = prm->tb;
  const TetGeo& g = prm->g;
  const double* c = prm->cf.c;
  const int tid = threadIdx.x;
  const int s = tid / TET_EB, el = tid % TET_EB;
  const int e0 = blockIdx.x * TET_EB;
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
  constexpr int FR = tet_frow<K>();
  for (int i = tid; i < 4 * NF * NB * 4; i += NT) {
    const int c4 = i % 4, j = (i / 4) % NB, p = (i / (4 * NB)) % NF, f = i / (4 * NB * NF);
    sm.ftab[(f * NF + p) * FR + 4 * j + c4] = tb.ftab[f][p][j][c4];
  }
  double jt[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) jt[i] = g.jit[9 * (size_t)e + i];
  const double vol = g.vol[e];
  const double as = c[K_MU1 + s];

  // ---- volume, QC points at a time ---------------------------------------------------
  double* V = sm.buf;   // [EB][VS]: NVQ slots of QC points (VS odd)
  const int vslot = s == S_N1 ? 0 : s == S_N2 ? 1 : s == S_C1 ? 2 : s == S_C3 ? 3 : s == S_N3 ? 13 : 14;
  const int gslot = s == S_N1 ? 4 : s == S_C1 ? 7 : s == S_C3 ? 10 : -1;
  // linear reactions: n1 -d1 n1; n2 -d2 n2; n3 (d1 - gamma) n1 + d2 n2; c1 f1 n3 (+ alpha
  // term); c2 -k c2; c3 k c2
  const double kown = s == S_N1 ? -c[K_D1] : s == S_N2 ? -c[K_D2] : s == S_C2 ? -c[K_K] : 0.0;
  const int r0 = s == S_N3 ? 0 : s == S_C1 ? 13 : s == S_C3 ? 14 : 0;
  const double k0 = s == S_N3 ? c[K_D1] - c[K_GAM] : s == S_C1 ? c[K_F1] : s == S_C3 ? c[K_K] : 0.0;
  const double k1 = s == S_N3 ? c[K_D2] : 0.0;
  const int fs = s == S_N2 ? 7 : 4;
  const double fw = s == S_N1 || s == S_N2 ? 1.0 : 0.0, rw = s == S_C1 ? 1.0 : 0.0;
#pragma unroll 1
  for (int q0 = 0; q0 < NQ; q0 += QC) {
    __syncthreads();
    {
      double* o = V + el * VS;
#pragma unroll 1
      for (int qq = 0; qq < QC; ++qq) {
        const int q = q0 + qq;
        double v = 0.0, a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          v += tb.Bv[q][j] * u[j];
          a0 += tb.Bg[q][j][0] * u[j];
          a1 += tb.Bg[q][j][1] * u[j];
          a2 += tb.Bg[q][j][2] * u[j];
        }
        o[vslot * QC + qq] = v;
        if (gslot >= 0) {
#pragma unroll
          for (int a = 0; a < 3; ++a) o[(gslot + a) * QC + qq] = jt[3 * a] * a0 + jt[3 * a + 1] * a1 + jt[3 * a + 2] * a2;
        }
      }
    }
    __syncthreads();
    // point items: chemotactic fluxes F1 (slots 4..6), F2 (7..9), alpha term (10)
    for (int it = tid; it < TET_EB * QC; it += NT) {
      const int l = it / QC, qq = it % QC;
      double* x = V + l * VS + qq;
      const double n1 = x[0], n2 = x[QC], c1 = x[2 * QC], c3 = x[3 * QC];
      const double d11 = c1 + c[K_XT11], d13 = c3 + c[K_XT13], d21 = c1 + c[K_XT21], d22 = n1 + c[K_XT22];
      if (e0 + l < E && !(d11 > 0.0 && d13 > 0.0 && d21 > 0.0 && d22 > 0.0)) flag |= FLAG_DOMAIN;
      double r11, r13, r21, r22;
      recip4(d11, d13, d21, d22, r11, r13, r21, r22);
      const double k11 = c[K_X011] * r11, k13 = c[K_X013] * r13, k21 = c[K_X021] * r21, k22 = c[K_X022] * r22;
      double F1[3], F2[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double gn1 = x[(4 + a) * QC], gc1 = x[(7 + a) * QC], gc3 = x[(10 + a) * QC];
        F1[a] = n1 * (k11 * gc1 + k13 * gc3);
        F2[a] = n2 * (k21 * gc1 - k22 * gn1);
      }
      const double rc = -(c[K_AL1] * n1 + c[K_AL2] * n2) * c1;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        x[(4 + a) * QC] = F1[a];
        x[(7 + a) * QC] = F2[a];
      }
      x[10 * QC] = rc;
    }
    __syncthreads();
    {
      // test integration; the own gradient is formed again here rather than held
      // in registers through the exchange
      const double* x = V + el * VS;
#pragma unroll 1
      for (int qq = 0; qq < QC; ++qq) {
        const int q = q0 + qq;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          a0 += tb.Bg[q][j][0] * u[j];
          a1 += tb.Bg[q][j][1] * u[j];
          a2 += tb.Bg[q][j][2] * u[j];
        }
        const double wt = vol * tb.wv[q];
        double f[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
          f[a] = fw * x[(fs + a) * QC + qq] - as * (jt[3 * a] * a0 + jt[3 * a + 1] * a1 + jt[3 * a + 2] * a2);
        // (J^-T g^) . f = g^ . (J^-1 f): the flux in reference coordinates
        double h[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) h[b] = jt[b] * f[0] + jt[3 + b] * f[1] + jt[6 + b] * f[2];
        const double sv = kown * x[vslot * QC + qq] + k0 * x[r0 * QC + qq] + k1 * x[QC + qq] + rw * x[10 * QC + qq];
#pragma unroll
        for (int j = 0; j < NB; ++j)
          R[j] += wt * (h[0] * tb.Bg[q][j][0] + h[1] * tb.Bg[q][j][1] + h[2] * tb.Bg[q][j][2] + sv * tb.Bv[q][j]);
      }
    }
  }

  // ---- faces ----------------------------------------------------------------------
  double* Fx = sm.buf;   // [EB][FS]: NFQ slots of NF points, then one pad
  const double* ft = sm.ftab;
  double* park = sm.park + tid * PS;
  const int fvslot = s == S_N1 ? 0 : s == S_N2 ? 1 : s == S_C1 ? 2 : s == S_C3 ? 3 : -1;
  const int dslot = s == S_N1 ? 8 : s == S_C1 ? 9 : s == S_C3 ? 10 : -1;
#pragma unroll 1
  for (int f = 0; f < 4; ++f) {
    __syncthreads();
    const int nb = live ? g.nbr[4 * e + f] : -3;
    const int gf = nb >= 0 ? g.nbe[4 * e + f] : 0;
    const int ori = nb >= 0 ? g.ori[4 * e + f] : 0;
    const double n0 = g.nrm[12 * e + 3 * f], n1v = g.nrm[12 * e + 3 * f + 1], n2v = g.nrm[12 * e + 3 * f + 2];
    // normal derivative weights of this element: d_n = sum_b (n . J^-T e_b) d/dxi_b
    const double dw0 = n0 * jt[0] + n1v * jt[3] + n2v * jt[6];
    const double dw1 = n0 * jt[1] + n1v * jt[4] + n2v * jt[7];
    const double dw2 = n0 * jt[2] + n1v * jt[5] + n2v * jt[8];
    // traces at the face points: own from the own modes, neighbour from its modes
    // at the permuted points; the point values go to the exchange, the thread's
    // jump and sum of normal derivatives wait in LDS through the point pass
    const bool inner = nb >= 0;
    const double* src = U + s * SE + (size_t)(inner ? nb : e) * NB;
    double w[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) w[j] = inner ? src[j] : 0.0;
    double jn[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) jn[i] = g.jit[9 * (size_t)(inner ? nb : e) + i];
    const double ew0 = n0 * jn[0] + n1v * jn[3] + n2v * jn[6];
    const double ew1 = n0 * jn[1] + n1v * jn[4] + n2v * jn[7];
    const double ew2 = n0 * jn[2] + n1v * jn[5] + n2v * jn[8];
#pragma unroll 1
    for (int p = 0; p < NF; ++p) {
      double v = 0.0, a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        v += tb.Bf[f][p][j] * u[j];
        a0 += tb.Bgf[f][p][j][0] * u[j];
        a1 += tb.Bgf[f][p][j][1] * u[j];
        a2 += tb.Bgf[f][p][j][2] * u[j];
      }
      const double uo = v, dno = dw0 * a0 + dw1 * a1 + dw2 * a2;
      const double* t = ft + (gf * NF + tb.perm[ori][p]) * FR;
      double vn = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        vn += t[4 * j] * w[j];
        b0 += t[4 * j + 1] * w[j];
        b1 += t[4 * j + 2] * w[j];
        b2 += t[4 * j + 3] * w[j];
      }
      const double un = vn, dnn = ew0 * b0 + ew1 * b1 + ew2 * b2;   // zero on boundary faces (w = 0)
      park[p] = uo - un;
      park[NF + p] = dno + dnn;
      if (fvslot >= 0) {
        Fx[el * FS + fvslot * NF + p] = uo;
        Fx[el * FS + (4 + fvslot) * NF + p] = un;
      }
      if (dslot >= 0) {
        Fx[el * FS + dslot * NF + p] = dno;
        Fx[el * FS + (dslot + 3) * NF + p] = dnn;
      }
    }
    __syncthreads();
    // face point items: lambda / 2, -(F1 + F1').n / 2, -(F2 + F2').n / 2, or inflow
    for (int it = tid; it < TET_EB * NF; it += NT) {
      const int l = it / NF, p = it % NF;
      double* x = Fx + l * FS + p;
      const int el2 = e0 + l;
      const int nbl = el2 < E ? g.nbr[4 * el2 + f] : -3;
      const double c1o = x[2 * NF];
      if (nbl >= 0) {
        const double n1o = x[0], n2o = x[NF], c3o = x[3 * NF];
        const double n1n = x[4 * NF], n2n = x[5 * NF], c1n = x[6 * NF], c3n = x[7 * NF];
        const double dn1o = x[8 * NF], dc1o = x[9 * NF], dc3o = x[10 * NF];
        const double dn1n = x[11 * NF], dc1n = x[12 * NF], dc3n = x[13 * NF];
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
        x[NF] = -0.5 * (n1o * w1o + n1n * w1n);
        x[2 * NF] = -0.5 * (n2o * w2o + n2n * w2n);
      } else {
        double q1 = 0.0, q2 = 0.0, q5 = 0.0;
        if (nbl == -1) {
          if (c1o - c[K_C1S] > 0.0) q1 = c[K_MU1] * c[K_BE1];
          // the face's vertices are the element's local vertices other than f
          const int va = f == 0 ? 1 : 0, vb = f <= 1 ? 2 : 1, vc = f <= 2 ? 3 : 2;
          const double xc = tb.fbary[p][0] * g.xv[4 * el2 + va] + tb.fbary[p][1] * g.xv[4 * el2 + vb] +
                            tb.fbary[p][2] * g.xv[4 * el2 + vc];
          if (xc >= g.g1in[0] && xc <= g.g1in[1]) q5 = c[K_NU2] * c[K_SIG];
        } else if (nbl == -2) {
          if (c1o - c[K_C1SS] > 0.0) q2 = c[K_MU2] * c[K_BE2];
        }
        x[0] = 0.0;
        x[NF] = 0.0;
        x[2 * NF] = 0.0;
        x[3 * NF] = q1;
        x[4 * NF] = q2;
        x[5 * NF] = q5;
      }
    }
    __syncthreads();
    // species pass: every face term at the face points, weighted, spread onto the
    // own basis at once
    if (live) {
      const double* x = Fx + el * FS;
      const double ar = g.area[4 * e + f];
      const bool mine = g.minus[4 * e + f] != 0;
      const double vm = mine ? vol : inner ? g.vol[nb] : vol;
      const double sgn = mine ? 1.0 : -1.0;   // n^- . n_o
      // int_e (u^- - u^+) phi_j^- with K^-'s basis at the face points (own order)
      double proj[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) proj[j] = 0.0;
      if (inner) {
#pragma unroll 1
        for (int p = 0; p < NF; ++p) {
          const double gm = sgn * park[p] * (ar * tb.wf[p]);
          const double* t = mine ? ft + (f * NF + p) * FR : ft + (gf * NF + tb.perm[ori][p]) * FR;
#pragma unroll
          for (int j = 0; j < NB; ++j) proj[j] += gm * t[4 * j];
        }
      }
      const double fa = -(2.0 * as / vm) * sgn;
      const double lw = inner ? 1.0 : 0.0;   // linear face terms on interior faces only
      // the one flux slot this species adds: interior n1 F1 (1), n2 F2 (2); boundary
      // inflow n1 (3), n2 (4), c2 (5); weight 0 for the others
      const int ksl = inner ? (s == S_N2 ? 2 : 1) : (s == S_N2 ? 4 : s == S_C2 ? 5 : 3);
      const double kw = inner ? (s == S_N1 || s == S_N2 ? 1.0 : 0.0) : (s == S_N1 || s == S_N2 || s == S_C2 ? 1.0 : 0.0);
#pragma unroll 1
      for (int p = 0; p < NF; ++p) {
        const double* t = mine ? ft + (f * NF + p) * FR : ft + (gf * NF + tb.perm[ori][p]) * FR;
        const double jm = park[p], sd = park[NF + p];
        double rt = 0.0;
#pragma unroll
        for (int j = 0; j < NB; ++j) rt += t[4 * j] * proj[j];
        const double gv = lw * (0.5 * as * sd + fa * rt - x[p] * jm) + kw * x[ksl * NF + p];
        const double G = ar * tb.wf[p] * gv, H = lw * ar * tb.wf[p] * 0.5 * as * jm;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const double dphi = dw0 * tb.Bgf[f][p][j][0] + dw1 * tb.Bgf[f][p][j][1] + dw2 * tb.Bgf[f][p][j][2];
          R[j] += G * tb.Bf[f][p][j] + H * dphi;
        }
      }
    }
  }

  // ---- M^{-1}, stage combination, store -------------------------------------------------
  if (live) {
    double* dst = out + s * SE + (size_t)e * NB;
    const double iv = 1.0 / vol;
    const bool combine = stage != 0 && ca != 0.0;   // U0 is read (and non-null) only then
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      double v = R[j] * iv;
      if (stage != 0) v = cb * (u[j] + dt * v);
      if (combine) v += ca * U0[s * SE + (size_t)e * NB + j];
      if (!isfinite(v)) flag |= FLAG_NONFINITE;
      dst[j] = v;
    }
  }
  if (flag) atomicOr(flags, flag);
}

}  // namespace cdg2
