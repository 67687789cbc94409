// CFL reduction: over all volume Gauss points, the largest chemotactic velocity
// component |w1_a|, |w2_a| and the largest n1, n2 values (clamped at 0).
//
// Same mapping as the operator kernel: one thread per (cell, species) holds the
// species' modes; n1, n2, c1, c3 threads produce values / gradients one layer of
// Gauss points at a time into LDS, point items evaluate w1, w2.  Each workgroup
// reduces in LDS and issues one 64-bit atomicMax per value on the bit patterns
// (non-negative doubles order like their bit patterns), so the result does not
// depend on the order of the blocks.
#pragma once

#include "es_kernel.hpp"

namespace cdg2 {

template <int D, int P, typename T, int EB>
__global__ void __launch_bounds__(6 * EB)
cfl_kernel(const Params* __restrict__ prm, const T* __restrict__ U, unsigned long long* __restrict__ out3,
           int* __restrict__ flags) {
  using S = EsSz<D, P>;
  constexpr int Q = S::Q, NM = S::NM, NF = S::NF, PC = S::PC, NVQ = S::NVQ;
  constexpr int NT = 6 * EB;
  __shared__ T V[EB * NVQ * PC];
  __shared__ double red[3][NT];
  const Tables& tb = prm->tb;
  const Geo& g = prm->g;
  const double* c = prm->cf.c;
  const int tid = threadIdx.x;
  const int s = tid / EB, el = tid % EB;
  const int e0 = xcd_block(blockIdx.x, gridDim.x) * EB;
  const int E = g.E;
  const bool live = e0 + el < E;
  const size_t SE = (size_t)E * NM;
  const int prod = s == S_N1 ? 0 : s == S_N2 ? 1 : s == S_C1 ? 2 : s == S_C3 ? 3 : -1;
  T u[NM];
  {
    // only n1, n2, c1, c3 enter the velocities and bounds: n3, c2 read nothing
    const bool need = live && prod >= 0;
    const T* src = U + s * SE + (size_t)(live ? e0 + el : 0) * NM;
#pragma unroll
    for (int m = 0; m < NM; ++m) u[m] = need ? src[m] : T(0);
  }
  const bool grads = s == S_N1 || s == S_C1 || s == S_C3;
  const int gslot = s == S_N1 ? 4 : s == S_C1 ? 4 + D : 4 + 2 * D;
  double lam = 0.0, mn1 = 0.0, mn2 = 0.0;
  int flag = 0;
  for (int lc = 0; lc < Q; ++lc) {
    __syncthreads();
    if (prod >= 0) produce_layer<D, Q, T>(tb, g, u, lc, V + el * NVQ * PC, prod, grads ? gslot : -1);
    __syncthreads();
    for (int it = tid; it < EB * PC; it += NT) {
      const int l = it / PC, q = it % PC;
      if (e0 + l >= E) continue;
      const T* v = V + l * NVQ * PC + q;
      const T n1 = v[0], n2 = v[PC], c1 = v[2 * PC], c3 = v[3 * PC];
      const T d11 = c1 + T(c[K_XT11]), d13 = c3 + T(c[K_XT13]), d21 = c1 + T(c[K_XT21]),
              d22 = n1 + T(c[K_XT22]);
      if (!(d11 > T(0) && d13 > T(0) && d21 > T(0) && d22 > T(0))) flag |= FLAG_DOMAIN;
      T r11, r13, r21, r22;
      recip4(d11, d13, d21, d22, r11, r13, r21, r22);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const T gn1 = v[(4 + a) * PC], gc1 = v[(4 + D + a) * PC], gc3 = v[(4 + 2 * D + a) * PC];
        const T w1 = T(c[K_X011]) * gc1 * r11 + T(c[K_X013]) * gc3 * r13;
        const T w2 = T(c[K_X021]) * gc1 * r21 - T(c[K_X022]) * gn1 * r22;
        lam = fmax(lam, fmax(fabs((double)w1), fabs((double)w2)));
        if (!(w1 == w1 && w2 == w2)) flag |= FLAG_NONFINITE;
      }
      mn1 = fmax(mn1, (double)n1);
      mn2 = fmax(mn2, (double)n2);
    }
  }
  red[0][tid] = lam;
  red[1][tid] = mn1;
  red[2][tid] = mn2;
  __syncthreads();
  if (tid < 3) {
    double v = 0.0;
    for (int k = 0; k < NT; ++k) v = fmax(v, red[tid][k]);
    atomicMax(out3 + tid, (unsigned long long)__double_as_longlong(v));
  }
  if (flag) atomicOr(flags, flag);
}

}  // namespace cdg2
