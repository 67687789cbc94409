// CFL reduction: over all volume Gauss points, the largest chemotactic velocity
// component |w1_a|, |w2_a| and the largest n1, n2 values (clamped at 0).  Each
// workgroup reduces its cells in LDS and issues one 64-bit atomicMax per value on
// the bit patterns (non-negative doubles order like their bit patterns), so the
// result does not depend on the order of the blocks.
#pragma once

#include "op_common.hpp"

namespace cdg2 {

template <int D, int P, typename T, int EPW, int NT>
__global__ void __launch_bounds__(NT)
cfl_kernel(const Params* __restrict__ prm, const T* __restrict__ U,
           unsigned long long* __restrict__ out3, int* __restrict__ flags) {
  const Tables& tb = prm->tb;
  const Geo& g = prm->g;
  const Coef& cf = prm->cf;
  using Z = Sz<D, P>;
  constexpr int Q = Z::Q, NM = Z::NM, NQ = Z::NQ;
  constexpr int NPV = 4 + 3 * D;
  __shared__ T sU[EPW][6][NM];
  __shared__ T sV[EPW][NPV][NQ];
  __shared__ double red[3][NT];
  const int tid = threadIdx.x;
  const int e0 = blockIdx.x * EPW;
  const int E = g.E;
  const size_t SE = (size_t)E * NM;
  const double* c = cf.c;
  for (int it = tid; it < 6 * EPW * NM; it += NT) {
    int s = it / (EPW * NM), off = it % (EPW * NM);
    int e = e0 + off / NM;
    sU[off / NM][s][off % NM] = e < E ? U[s * SE + (size_t)e0 * NM + off] : T(0);
  }
  __syncthreads();
  for (int it = tid; it < EPW * NPV; it += NT) {
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
    for (int m = 0; m < NM; ++m) in[m] = sU[el][sp][m];
    tapply<D, Q, false, T>(in, o, Mx, My, Mz);
#pragma unroll
    for (int m = 0; m < NQ; ++m) sV[el][qty][m] = o[m] * scale;
  }
  __syncthreads();
  double lam = 0.0, mn1 = 0.0, mn2 = 0.0;
  int flag = 0;
  for (int it = tid; it < EPW * NQ; it += NT) {
    int el = it / NQ, qp = it % NQ;
    if (e0 + el >= E) continue;
    T n1 = sV[el][0][qp], n2 = sV[el][1][qp], c1 = sV[el][2][qp], c3 = sV[el][3][qp];
    T d11 = c1 + T(c[K_XT11]), d13 = c3 + T(c[K_XT13]), d21 = c1 + T(c[K_XT21]), d22 = n1 + T(c[K_XT22]);
    if (!(d11 > T(0) && d13 > T(0) && d21 > T(0) && d22 > T(0))) flag |= FLAG_DOMAIN;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T w1 = T(c[K_X011]) * sV[el][4 + D + a][qp] / d11 + T(c[K_X013]) * sV[el][4 + 2 * D + a][qp] / d13;
      T w2 = T(c[K_X021]) * sV[el][4 + D + a][qp] / d21 - T(c[K_X022]) * sV[el][4 + a][qp] / d22;
      lam = fmax(lam, fmax(fabs((double)w1), fabs((double)w2)));
    }
    mn1 = fmax(mn1, (double)n1);
    mn2 = fmax(mn2, (double)n2);
  }
  red[0][tid] = lam;
  red[1][tid] = mn1;
  red[2][tid] = mn2;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w)
      for (int k = 0; k < 3; ++k) red[k][tid] = fmax(red[k][tid], red[k][tid + w]);
    __syncthreads();
  }
  if (tid < 3) {
    double v = red[tid][0];
    if (!(v >= 0.0)) {  // NaN
      v = 0.0;
      atomicOr(flags, FLAG_NONFINITE);
    }
    atomicMax(out3 + tid, (unsigned long long)__double_as_longlong(v));
  }
  if (flag) atomicOr(flags, flag);
}

}  // namespace cdg2
