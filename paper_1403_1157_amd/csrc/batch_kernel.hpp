// Batched SSP-RK3 stage kernel: many independent 2D instances with different
// grids, orders and coefficient sets in one launch per stage (or one per order).
//
// The work list holds one item per (instance, block of EB cells), sorted by the
// host (by default by decreasing cost).  The grid is either one workgroup per
// item, or a fixed number of persistent workgroups that walk the list with a
// static stride (item = blockIdx.x + k * gridDim.x: no dynamic queue, so the
// schedule is reproducible); the autotuner picks.  Each item
// runs the same per-block code as the single-instance kernel (es_block), chosen
// by the instance's order p (uniform within a workgroup), on the LDS buffer sized
// for the largest order.
#pragma once

#include "es_kernel.hpp"

namespace cdg2 {

struct BatchInst {
  Params prm;
  size_t off;     // element offset of the instance in the packed state
  double dt;      // time step of this instance
  int p;          // order (1..3)
  int pad;
};

struct WorkItem {
  int inst;
  int e0;         // first cell of the block
};

template <typename T, int EB>
struct BatchSmem {
  static constexpr size_t S1 = sizeof(EsSmem<2, 1, T, EB>);
  static constexpr size_t S2 = sizeof(EsSmem<2, 2, T, EB>);
  static constexpr size_t S3 = sizeof(EsSmem<2, 3, T, EB>);
  static constexpr size_t S12 = S1 > S2 ? S1 : S2;
  static constexpr size_t N = S12 > S3 ? S12 : S3;
};

// stage 1: S0 = U + dt f(U); stage 2: S1 = 3/4 U + 1/4 (S0 + dt f(S0));
// stage 3: U = 1/3 U + 2/3 (S1 + dt f(S1))  (per instance, packed buffers)
template <typename T, int EB>
__global__ void __launch_bounds__(6 * EB, 3)
batch_stage_kernel(const BatchInst* __restrict__ insts, const WorkItem* __restrict__ items, int nitems,
                   T* U, T* S0, T* S1, int stage, int* __restrict__ flags) {
  __shared__ __align__(16) unsigned char smem[BatchSmem<T, EB>::N];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[it];
    const BatchInst& in = insts[wi.inst];
    const size_t off = in.off;
    const T dt = T(in.dt);
    const T* src;
    const T* u0;
    T* dst;
    T ca, cb;
    if (stage == 1) {
      src = U + off; u0 = nullptr; dst = S0 + off; ca = T(0); cb = T(1);
    } else if (stage == 2) {
      src = S0 + off; u0 = U + off; dst = S1 + off; ca = T(0.75); cb = T(0.25);
    } else {
      src = S1 + off; u0 = U + off; dst = U + off; ca = T(1.0 / 3.0); cb = T(2.0 / 3.0);
    }
    switch (in.p) {
      case 1:
        es_block<2, 1, T, EB>(in.prm, src, u0, dst, dt, ca, cb, stage, flags, wi.e0,
                              *reinterpret_cast<EsSmem<2, 1, T, EB>*>(smem));
        break;
      case 2:
        es_block<2, 2, T, EB>(in.prm, src, u0, dst, dt, ca, cb, stage, flags, wi.e0,
                              *reinterpret_cast<EsSmem<2, 2, T, EB>*>(smem));
        break;
      default:
        es_block<2, 3, T, EB>(in.prm, src, u0, dst, dt, ca, cb, stage, flags, wi.e0,
                              *reinterpret_cast<EsSmem<2, 3, T, EB>*>(smem));
        break;
    }
    __syncthreads();   // the next item reuses the LDS buffer
  }
}

// The same stage for work items of one order P only (one launch per order):
// each launch gets the occupancy of its own order's registers and LDS.  At P = 3
// at least 3 waves per SIMD (168 VGPRs with a few spills; 6% faster than the 2
// waves its free allocation of 219 VGPRs allowed).
template <typename T, int EB, int P>
__global__ void __launch_bounds__(6 * EB, P == 3 ? 3 : 1)
batch_stage_kernel_p(const BatchInst* __restrict__ insts, const WorkItem* __restrict__ items, int nitems,
                     T* U, T* S0, T* S1, int stage, int* __restrict__ flags) {
  __shared__ EsSmem<2, P, T, EB> sm;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[it];
    const BatchInst& in = insts[wi.inst];
    const size_t off = in.off;
    const T dt = T(in.dt);
    const T* src;
    const T* u0;
    T* dst;
    T ca, cb;
    if (stage == 1) {
      src = U + off; u0 = nullptr; dst = S0 + off; ca = T(0); cb = T(1);
    } else if (stage == 2) {
      src = S0 + off; u0 = U + off; dst = S1 + off; ca = T(0.75); cb = T(0.25);
    } else {
      src = S1 + off; u0 = U + off; dst = U + off; ca = T(1.0 / 3.0); cb = T(2.0 / 3.0);
    }
    es_block<2, P, T, EB>(in.prm, src, u0, dst, dt, ca, cb, stage, flags, wi.e0, sm);
    __syncthreads();   // the next item reuses the LDS buffer
  }
}

// Fill a buffer with a constant (autotuning inputs).
template <typename T>
__global__ void fill_kernel(T* x, size_t n, T v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (size_t)gridDim.x * blockDim.x) x[i] = v;
}

}  // namespace cdg2
