// CDG2 operator kernel, one thread per (cell, species), in the modal basis (2D
// and 3D p = 3; 3D p <= 2 runs the nodal form of nodal_kernel.hpp).
//
// Per cell (Section 3.1) the residual is
//   volume:   int_K (F(U) - A grad U) : grad phi + S(U) phi
//   faces:    int_e {A grad phi}:[[U]] + {A grad U}:[[phi]] - (F^ - A^):[[phi]]
// with the local Lax-Friedrichs flux F^ and the CDG2 flux
// A^ = 2 chi_e (A r_e([[U]]))|_{K^-_e}.  On Cartesian cells with the orthonormal
// Legendre basis the lifting of a face jump on K^- (the low-side cell) has the
// trace -(liftc / (2h)) [[U]], liftc = sum_i phi_i(1)^2, so A^ . n^- is
// -chi_e a liftc / h (u^- - u^+): it is formed from K^-'s end values only.
// Each cell evaluates all of its faces from its own side, in its outward normal
// n_o (the expression is symmetric in the two sides):
//   R_j += int_e 1/2 a (u_o - u_n) d_{n_o} phi_j
//        + [ 1/2 a (d_{n_o} u_o + d_{n_o} u_n) - pen (u_o - u_n)
//            - 1/2 (F_o + F_n).n_o - 1/2 lam (u_o - u_n) ] phi_j,
// then f = R / |K| (M = |K| I), optionally combined with an SSP-RK3 stage in the
// epilogue so that f never reaches HBM.
//
// Mapping:
//   * a workgroup owns EB consecutive cells; thread (s, el) keeps the modes and
//     the modal residual of species s of cell el in registers (in 3D the
//     workgroup first moves all its cells' modes into LDS with coalesced
//     load-to-LDS instructions, and its results leave through LDS with coalesced
//     stores);
//   * everything linear in U is applied by that thread alone, exactly, in modal
//     form: -a_s int grad u . grad phi (1D stiffness per axis), the face
//     consistency / symmetry / lifting terms (tangential-modal traces of the
//     cell and of its neighbour, whose modes the thread reads from global
//     memory), and the linear reactions (other species' modes of the same cell);
//   * the nonlinear terms need several species at one point; they are
//     exchanged through LDS: the volume one layer of Gauss points (along the
//     last axis) at a time, the faces one face direction at a time.  Point items
//     (cell, point) evaluate w1, w2, F1, F2, alpha n c, lambda and the inflow
//     fluxes; species threads integrate them back against their test functions.
#pragma once

#include "op_common.hpp"

namespace cdg2 {

// Sizes for D, P with chunks of Gauss points = layers along the last axis.
template <int D, int P>
struct EsSz {
  using Z = Sz<D, P>;
  static constexpr int Q = Z::Q, NM = Z::NM, NQ = Z::NQ, NF = Z::NF, NFACE = Z::NFACE;
  static constexpr int PC = NF;            // points per layer
  static constexpr int NVQ = 4 + 3 * D;    // n1 n2 c1 c3 | grad n1 | grad c1 | grad c3
  static constexpr int NFQ = 14;           // face exchange: 4 values x 2 sides, 3 d_n x 2 sides
};

// LDS: one union buffer, reused by the volume layers and by the faces, and (3D)
// also as the staging area of the coalesced load of the workgroup's own cells'
// modes (all six species) and of the coalesced store of the results.
// Staged loads move chunks of CB bytes (16; 12 when a cell's modes are not a
// multiple of 16 bytes; else 4), NCH per (cell, species).  The load-to-LDS
// instruction places lane t's chunk at LS t bytes, LS = 16 for 12- and 16-byte
// chunks and 4 for 4-byte ones, so chunk k of thread g = (s, l) sits at byte
// LS (g NCH + k) (a 12-byte chunk leaves 4 bytes unused).
template <int D, int P, typename T, int EB, int NV = EsSz<D, P>::NVQ, int XTRA = 0>
struct EsSmem {
  using S = EsSz<D, P>;
  // 3D only: in 2D (72 to 200 bytes per (cell, species)) the staging measured no
  // gain and its LDS lowered the occupancy of the batched kernel
  static constexpr bool STAGED = D == 3;
  static constexpr int BYTES = S::NM * (int)sizeof(T);
  static constexpr int CB = BYTES % 16 == 0 ? 16 : BYTES % 12 == 0 ? 12 : 4;
  static constexpr int LS = CB == 4 ? 4 : 16;
  static constexpr int NCH = BYTES / CB;
  // Per-cell strides of the exchange slots, odd in elements of T: with the plain
  // strides (3D Q3: 13 x 16 and 14 x 16 doubles) every cell of the workgroup
  // starts on the same LDS bank, and lanes reading the same slot of different
  // cells collide; odd strides spread the cells over the banks.
  static constexpr int VST = (NV * S::PC) | 1;   // NV exchange slots per volume point
  static constexpr int FST = (S::NFQ * S::NF) | 1;
  static constexpr int VOL = EB * VST;
  static constexpr int FAC = EB * FST;
  static constexpr int STG = STAGED ? 6 * EB * NCH * LS / (int)sizeof(T) : 0;
  static constexpr int N0 = VOL > FAC + XTRA ? VOL : FAC + XTRA;   // XTRA values after the face slots
  static constexpr int N = N0 > STG ? N0 : STG;
  int nb[EB][2 * D];
  int cell[EB];
  __align__(16) T buf[N];
};

// Rotation of the chunks of the cell in workgroup slot l, and the position (in
// units of LS bytes) of chunk j of thread g = (species, cell l = g mod EB): the
// thread's NCH chunks are contiguous, rotated by (l / 2) mod NCH.  Unrotated, the
// threads' chunk j would sit NCH positions apart, which maps most lanes of a
// wavefront onto a few LDS banks; with the rotation and whole-chunk reads the
// banks are hit at most 1.5 times as often as without conflicts, for the chunk
// sizes used here.  The rotation depends on the cell only, so the loads need one
// rotated chunk index per lane and round, not one per species.
template <int NCH>
__device__ __forceinline__ int stage_rot(int l) {
  return (l >> 1) % NCH;
}

template <int NCH, int EB>
__device__ __forceinline__ int stage_pos(int g, int j) {
  int c = j + stage_rot<NCH>(g % EB);
  if (c >= NCH) c -= NCH;
  return g * NCH + c;
}

// Element m of thread g's staged values.
template <int D, int P, typename T, int EB, int NV, int XT>
__device__ __forceinline__ T staged(const EsSmem<D, P, T, EB, NV, XT>& sm, int g, int m) {
  using SM = EsSmem<D, P, T, EB, NV, XT>;
  constexpr int CB = SM::CB, NCH = SM::NCH, LS = SM::LS;
  const unsigned char* base = reinterpret_cast<const unsigned char*>(sm.buf);
  const int b = m * (int)sizeof(T), j = b / CB, r = b % CB;
  if (r + (int)sizeof(T) <= CB) {
    return *reinterpret_cast<const T*>(base + stage_pos<NCH, EB>(g, j) * LS + r);
  } else {   // a double split over two chunks, 4 + 4 bytes
    const int lo = *reinterpret_cast<const int*>(base + stage_pos<NCH, EB>(g, j) * LS + r);
    const int hi = *reinterpret_cast<const int*>(base + stage_pos<NCH, EB>(g, j + 1) * LS);
    return T(__hiloint2double(hi, lo));
  }
}

// All NM staged values of thread g, read chunk by chunk (one 16-, 12- or 4-byte
// LDS read per chunk) and reassembled in registers.
template <int D, int P, typename T, int EB, int NV, int XT>
__device__ __forceinline__ void staged_all(const EsSmem<D, P, T, EB, NV, XT>& sm, int g, T* u) {
  using SM = EsSmem<D, P, T, EB, NV, XT>;
  constexpr int CB = SM::CB, NCH = SM::NCH, LS = SM::LS, NW = SM::BYTES / 4, NM = EsSz<D, P>::NM;
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
  const unsigned char* base = reinterpret_cast<const unsigned char*>(sm.buf);
  unsigned int w[NW];
#pragma unroll
  for (int j = 0; j < NCH; ++j) {
    const unsigned char* src = base + stage_pos<NCH, EB>(g, j) * LS;
    if constexpr (CB == 16) {
      const u32x4 x = *reinterpret_cast<const u32x4*>(src);
      w[4 * j] = x.x;
      w[4 * j + 1] = x.y;
      w[4 * j + 2] = x.z;
      w[4 * j + 3] = x.w;
    } else if constexpr (CB == 12) {
      const u32x3 x = *reinterpret_cast<const u32x3*>(src);
      w[3 * j] = x.x;
      w[3 * j + 1] = x.y;
      w[3 * j + 2] = x.z;
    } else {
      w[j] = *reinterpret_cast<const unsigned int*>(src);
    }
  }
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    if constexpr (sizeof(T) == 8)
      u[m] = T(__hiloint2double((int)w[2 * m + 1], (int)w[2 * m]));
    else
      u[m] = T(__uint_as_float(w[m]));
  }
}

// Start loading the values of the cells cells[l * cstride] (l < EB; outside
// [0, E): none, cell 0 is loaded and not used) of all six species straight into
// the staging area, without registers in flight: consecutive lanes take
// consecutive chunks of one cell, so each load instruction reads whole cache
// lines of consecutive cells (one lane per cell and 216-byte modes would put
// every lane on its own line).  The caller waits (vmcnt) and synchronises before
// reading.
template <int D, int P, typename T, int EB, int NV, int XT>
__device__ __forceinline__ void stage_cells(const T* U, size_t SE, int E, const int* cells, int cstride,
                                            EsSmem<D, P, T, EB, NV, XT>& sm, int tid) {
  using SM = EsSmem<D, P, T, EB, NV, XT>;
  constexpr int NM = EsSz<D, P>::NM, NT = 6 * EB, CB = SM::CB, NCH = SM::NCH;
  static_assert(SM::BYTES % CB == 0, "chunking");
  constexpr int PER = EB * NCH;                 // chunks per species
  constexpr int RR = (PER + NT - 1) / NT;
  unsigned char* base = reinterpret_cast<unsigned char*>(sm.buf);
  // the instruction's LDS address is per wavefront (lane t of the wavefront at
  // LS t): offset each wavefront by its first thread
  const int wbase = __builtin_amdgcn_readfirstlane((tid / 64) * 64);
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    const int ch = r * NT + tid;   // position within the species block
    if (ch < PER) {
      const int l = ch / NCH, c = ch % NCH;
      const int n = cells[l * cstride];
      // the chunk that belongs at this position (inverse of stage_pos)
      int k = c - stage_rot<NCH>(l);
      if (k < 0) k += NCH;
      const char* src = reinterpret_cast<const char*>(U + (size_t)(n >= 0 && n < E ? n : 0) * NM) + k * CB;
#pragma unroll
      for (int sp = 0; sp < 6; ++sp) {
        auto* dst = (__attribute__((address_space(3))) void*)(base + (sp * PER + r * NT + wbase) * SM::LS);
        const char* sps = src + (size_t)sp * SE * sizeof(T);
        if constexpr (CB == 16) {
          __builtin_amdgcn_global_load_lds(sps, dst, 16, 0, 0);
        } else if constexpr (CB == 12) {
          __builtin_amdgcn_global_load_lds(sps, dst, 12, 0, 0);
        } else {
          __builtin_amdgcn_global_load_lds(sps, dst, 4, 0, 0);
        }
      }
    }
  }
}

// The workgroup's own cells sm.cell[l].
template <int D, int P, typename T, int EB, int NV, int XT>
__device__ __forceinline__ void stage_modes(const T* U, size_t SE, int E, EsSmem<D, P, T, EB, NV, XT>& sm, int tid) {
  stage_cells<D, P, T, EB>(U, SE, E, sm.cell, 1, sm, tid);
}

__device__ __forceinline__ void wait_staged() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Coalesced store of the workgroup's results, which sit in buf as
// [species][cell][mode] (6 EB NM values): thread tid stores slots
// i = tid + k 6EB, out = buf (+ ca U0 for the stage combination).  The U0 values
// of a chunk of CH slots are all loaded before the first one is used, so the
// loads overlap instead of each costing a full memory latency.
template <int EB, int NM>
__device__ __forceinline__ size_t slot_index(const int* cell, size_t SE, int i, bool& ok) {
  constexpr int TOT = 6 * EB * NM, PERS = EB * NM;
  const int ii = i < TOT ? i : 0;
  const int sp = ii / PERS, rem = ii - sp * PERS;
  const int l = rem / NM, m = rem - l * NM;
  const int cl = cell[l];
  ok = i < TOT && cl >= 0;
  return sp * SE + (size_t)(cl >= 0 ? cl : 0) * NM + m;   // in range in every case
}

template <int EB, int NM>
constexpr int store_slots() { return (6 * EB * NM + 6 * EB - 1) / (6 * EB); }

template <typename T, int EB, int NM, int CH>
__device__ __forceinline__ void load_u0_chunk(const int* cell, const T* U0, size_t SE, int tid, int k0, T* u0) {
  constexpr int NT = 6 * EB, IT = store_slots<EB, NM>();
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    bool ok;
    const size_t gi = slot_index<EB, NM>(cell, SE, tid + (k0 + k) * NT, ok);
    u0[k] = ok && k0 + k < IT ? U0[gi] : T(0);
  }
}

template <typename T, int EB, int NM, int CH>
__device__ __forceinline__ void store_chunk(const int* cell, const T* buf, const T* u0, T* out, size_t SE, T ca,
                                            bool combine, int tid, int k0, int& flag) {
  constexpr int NT = 6 * EB, IT = store_slots<EB, NM>();
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    if (k0 + k >= IT) break;
    const int i = tid + (k0 + k) * NT;
    bool ok;
    const size_t gi = slot_index<EB, NM>(cell, SE, i, ok);
    if (!ok) continue;
    T val = buf[i];
    if (combine) val += ca * u0[k];
    if (!isfinite(val)) flag |= FLAG_NONFINITE;
    out[gi] = val;
  }
}

template <typename T, int EB, int NM>
__device__ __forceinline__ void store_results(const int* cell, const T* buf, const T* U0, T* out, size_t SE,
                                              T ca, bool combine, int tid, int& flag) {
  constexpr int IT = store_slots<EB, NM>(), CH = IT < 16 ? IT : 16;
#pragma unroll
  for (int k0 = 0; k0 < IT; k0 += CH) {
    T u0[CH];
    if (combine) load_u0_chunk<T, EB, NM, CH>(cell, U0, SE, tid, k0, u0);
    store_chunk<T, EB, NM, CH>(cell, buf, u0, out, SE, ca, combine, tid, k0, flag);
  }
}

// (D-1)-dimensional tensor contraction of NF values (tangential / layer axes).
template <int D, int Q, bool TR, typename T>
__device__ __forceinline__ void tapply_lo(const T* in, T* out, const double (*M0)[CDG2_MAXQ],
                                          const double (*M1)[CDG2_MAXQ]) {
  if constexpr (D == 2) {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      T s = T(0);
#pragma unroll
      for (int i = 0; i < Q; ++i) s += mat<TR, T>(M0, a, i) * in[i];
      out[a] = s;
    }
  } else {
    tapply<2, Q, TR, T>(in, out, M0, M1, nullptr);
  }
}

// Values (slot vslot) and, if gslot >= 0, physical gradients (slots gslot..+D-1)
// of one species at the Gauss points of layer lc (along the last axis) of a cell,
// from its modes u; out is the cell's [NVQ][NF] slot array.
template <int D, int Q, typename T>
__device__ __forceinline__ void produce_layer(const Tables& tb, const Geo& g, const T* u, int lc, T* out,
                                              int vslot, int gslot) {
  constexpr int NF = ipow(Q, D - 1), LST = NF, LA = D - 1;
  const double(*Bt0)[CDG2_MAXQ] = tb.B;
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
  for (int q = 0; q < NF; ++q) out[vslot * NF + q] = o[q];
  if (gslot >= 0) {
#pragma unroll
    for (int a = 0; a < D - 1; ++a) {
      tapply_lo<D, Q, false, T>(tv, o, a == 0 ? tb.Bd : tb.B, a == 1 ? tb.Bd : tb.B);
#pragma unroll
      for (int q = 0; q < NF; ++q) out[(gslot + a) * NF + q] = o[q] * T(g.ih[a]);
    }
    tapply_lo<D, Q, false, T>(td, o, Bt0, Bt0);
#pragma unroll
    for (int q = 0; q < NF; ++q) out[(gslot + LA) * NF + q] = o[q] * T(g.ih[LA]);
  }
}

// Reciprocals of four positive numbers with one division: 1/a = (b c d) / (a b c d).
template <typename T>
__device__ __forceinline__ void recip4(T a, T b, T c, T d, T& ra, T& rb, T& rc, T& rd) {
  const T ab = a * b, cd = c * d;
  const T r = T(1) / (ab * cd);
  const T rab = r * cd, rcd = r * ab;
  ra = rab * b;
  rb = rab * a;
  rc = rcd * d;
  rd = rcd * c;
}

// Face point pass of the Cartesian kernels, face f = 2 a + sg of every cell of the
// workgroup.  Exchange slots of point t of cell l, x = Fx + l FST + t (stride NF):
// 0..3 own n1 n2 c1 c3, 4..7 the neighbour's, 8..10 own normal derivatives of n1
// c1 c3, 11..13 the neighbour's.  Written: on an interior face lambda / 2 (0) and
// the averaged chemotactic normal fluxes -(F1 . n) / 2, -(F2 . n) / 2 (1, 2); on a
// boundary face zeros there and the inflow fluxes of n1, n2, c2 (3..5).
// The EB NF points go to the threads in whole rounds of one point per thread.
// With HALVES, the remaining points, when twice their number fits the workgroup,
// are split in two halves (own side, neighbour side) on a pair of adjacent lanes
// joined by two-lane shuffles: 3D Q2 has 90 points for 60 threads, one round and
// 30 points on 60 lanes instead of a second round at half occupancy.
template <int D, int Q, int NF, int EB, int FST, bool HALVES_OK, typename T>
__device__ __forceinline__ void face_points(T* Fx, const int (*nbt)[2 * D], int f, int sg, int b0,
                                            const double* c, const Geo& g, const Tables& tb, int e0, int E,
                                            int tid, int& flag) {
  constexpr int NT = 6 * EB, NPT = EB * NF, NFULL = NPT / NT * NT, REM = NPT - NFULL;
  constexpr bool HALVES = HALVES_OK && REM > 0 && 2 * REM <= NT;
  // boundary point: no LLF terms, the inflow fluxes.  (Used by the split points;
  // the whole-point loop keeps the same statements inline, which left the
  // register allocation of the configurations without split points (2D Q3,
  // Q4, 3D Q3) as it was: through the shared helper they ran 2% slower.)
  auto inflow = [&](T* x, int l, int t, int nbl, T c1o) {
    T q1 = T(0), q2 = T(0), q5 = T(0);
    if (nbl == -1) {
      if (c1o - T(c[K_C1S]) > T(0)) q1 = T(c[K_MU1] * c[K_BE1]);
      const double xc = (cell_coord<D>(g, cell_of<D>(g, e0 + l), b0) + tb.x[t % Q]) * g.h[b0];
      if (xc >= g.g1in[0] && xc <= g.g1in[1]) q5 = T(c[K_NU2] * c[K_SIG]);
    } else if (nbl == -2) {
      if (c1o - T(c[K_C1SS]) > T(0)) q2 = T(c[K_MU2] * c[K_BE2]);
    }
    x[0] = T(0);
    x[NF] = T(0);
    x[2 * NF] = T(0);
    x[3 * NF] = q1;
    x[4 * NF] = q2;
    x[5 * NF] = q5;
  };
  for (int it = tid; it < (HALVES ? NFULL : NPT); it += NT) {
    const int l = it / NF, t = it % NF;
    T* x = Fx + l * FST + t;
    const int nbl = nbt[l][f];
    const T c1o = x[2 * NF];
    if (nbl >= 0) {
      const T so = sg ? T(1) : T(-1);
      const T n1o = x[0], n2o = x[NF], c3o = x[3 * NF];
      const T n1n = x[4 * NF], n2n = x[5 * NF], c1n = x[6 * NF], c3n = x[7 * NF];
      const T dn1o = x[8 * NF], dc1o = x[9 * NF], dc3o = x[10 * NF];
      const T dn1n = x[11 * NF], dc1n = x[12 * NF], dc3n = x[13 * NF];
      const T t11 = T(c[K_XT11]), t13 = T(c[K_XT13]), t21 = T(c[K_XT21]), t22 = T(c[K_XT22]);
      const T d11o = c1o + t11, d13o = c3o + t13, d21o = c1o + t21, d22o = n1o + t22;
      const T d11n = c1n + t11, d13n = c3n + t13, d21n = c1n + t21, d22n = n1n + t22;
      if (e0 + l < E && !(d11o > T(0) && d13o > T(0) && d21o > T(0) && d22o > T(0) &&
                          d11n > T(0) && d13n > T(0) && d21n > T(0) && d22n > T(0)))
        flag |= FLAG_DOMAIN;
      T r11o, r13o, r21o, r22o, r11n, r13n, r21n, r22n;
      recip4(d11o, d13o, d21o, d22o, r11o, r13o, r21o, r22o);
      recip4(d11n, d13n, d21n, d22n, r11n, r13n, r21n, r22n);
      const T w1o = so * (T(c[K_X011]) * dc1o * r11o + T(c[K_X013]) * dc3o * r13o);
      const T w2o = so * (T(c[K_X021]) * dc1o * r21o - T(c[K_X022]) * dn1o * r22o);
      const T w1n = so * (T(c[K_X011]) * dc1n * r11n + T(c[K_X013]) * dc3n * r13n);
      const T w2n = so * (T(c[K_X021]) * dc1n * r21n - T(c[K_X022]) * dn1n * r22n);
      const T lam = fmax(fmax(fabs(w1o), fabs(w2o)), fmax(fabs(w1n), fabs(w2n)));
      x[0] = T(0.5) * lam;
      x[NF] = -T(0.5) * (n1o * w1o + n1n * w1n);
      x[2 * NF] = -T(0.5) * (n2o * w2o + n2n * w2n);
    } else {
      T q1 = T(0), q2 = T(0), q5 = T(0);
      if (nbl == -1) {
        if (c1o - T(c[K_C1S]) > T(0)) q1 = T(c[K_MU1] * c[K_BE1]);
        const double xc = (cell_coord<D>(g, cell_of<D>(g, e0 + l), b0) + tb.x[t % Q]) * g.h[b0];
        if (xc >= g.g1in[0] && xc <= g.g1in[1]) q5 = T(c[K_NU2] * c[K_SIG]);
      } else if (nbl == -2) {
        if (c1o - T(c[K_C1SS]) > T(0)) q2 = T(c[K_MU2] * c[K_BE2]);
      }
      x[0] = T(0);
      x[NF] = T(0);
      x[2 * NF] = T(0);
      x[3 * NF] = q1;
      x[4 * NF] = q2;
      x[5 * NF] = q5;
    }
  }
  if constexpr (HALVES) {
    static_assert(NT % 2 == 0, "lane pairs");
    const int hi = tid >> 1, side = tid & 1;   // side 0 own, 1 neighbour
    const bool act = hi < REM;
    const int it = NFULL + (act ? hi : 0);
    const int l = it / NF, t = it % NF;
    T* x = Fx + l * FST + t;
    const int nbl = nbt[l][f];
    T m = T(0), p1 = T(0), p2 = T(0);
    if (act && nbl >= 0) {
      const T so = sg ? T(1) : T(-1);
      const T t11 = T(c[K_XT11]), t13 = T(c[K_XT13]), t21 = T(c[K_XT21]), t22 = T(c[K_XT22]);
      const int vb = side ? 4 : 0, db = side ? 11 : 8;
      const T n1 = x[vb * NF], n2 = x[(vb + 1) * NF], c1 = x[(vb + 2) * NF], c3 = x[(vb + 3) * NF];
      const T dn1 = x[db * NF], dc1 = x[(db + 1) * NF], dc3 = x[(db + 2) * NF];
      const T d11 = c1 + t11, d13 = c3 + t13, d21 = c1 + t21, d22 = n1 + t22;
      if (e0 + l < E && !(d11 > T(0) && d13 > T(0) && d21 > T(0) && d22 > T(0))) flag |= FLAG_DOMAIN;
      T r11, r13, r21, r22;
      recip4(d11, d13, d21, d22, r11, r13, r21, r22);
      const T w1 = so * (T(c[K_X011]) * dc1 * r11 + T(c[K_X013]) * dc3 * r13);
      const T w2 = so * (T(c[K_X021]) * dc1 * r21 - T(c[K_X022]) * dn1 * r22);
      m = fmax(fabs(w1), fabs(w2));
      p1 = n1 * w1;
      p2 = n2 * w2;
    }
    // every lane takes part in the shuffles; the lanes of a point are 2k, 2k + 1
    const T m2 = __shfl_xor(m, 1, 64), q1 = __shfl_xor(p1, 1, 64), q2 = __shfl_xor(p2, 1, 64);
    if (act && side == 0) {
      if (nbl >= 0) {
        x[0] = T(0.5) * fmax(m, m2);
        x[NF] = -T(0.5) * (p1 + q1);
        x[2 * NF] = -T(0.5) * (p2 + q2);
      } else {
        inflow(x, l, t, nbl, x[2 * NF]);
      }
    }
  }
}

template <int D, int P, typename T, int EB>
__device__ __forceinline__ void es_block(const Params& prm, const T* __restrict__ U, const T* U0, T* out,
                                         T dt, T ca, T cb, int stage, int* __restrict__ flags, int e0,
                                         EsSmem<D, P, T, EB>& sm) {
  using S = EsSz<D, P>;
  constexpr int Q = S::Q, NM = S::NM, NF = S::NF, NFACE = S::NFACE, PC = S::PC, NVQ = S::NVQ;
  constexpr int NT = 6 * EB;
  const Tables& tb = prm.tb;
  const Geo& g = prm.g;
  const double* c = prm.cf.c;
  const int tid = threadIdx.x;
  const int s = tid / EB, el = tid % EB;
  const int E = g.E;
  const bool live = e0 + el < E;
  const int e = live ? cell_of<D>(g, e0 + el) : 0;
  const size_t SE = (size_t)E * NM;
  const T vol = T(g.vol);
  int flag = 0;

  // ---- own modes, neighbour table ------------------------------------------------
  constexpr bool STAGED = EsSmem<D, P, T, EB>::STAGED;
  constexpr int VST = EsSmem<D, P, T, EB>::VST, FST = EsSmem<D, P, T, EB>::FST;
  T u[NM], R[NM];
  for (int it = tid; it < EB * NFACE; it += NT) {
    int l = it / NFACE, f = it % NFACE;
    sm.nb[l][f] = e0 + l < E ? neighbour<D>(g, cell_of<D>(g, e0 + l), f) : -3;
  }
  if constexpr (STAGED) {
    if (tid < EB) sm.cell[tid] = e0 + tid < E ? cell_of<D>(g, e0 + tid) : -1;
    __syncthreads();
    stage_modes<D, P, T, EB>(U, SE, E, sm, tid);
    wait_staged();
    __syncthreads();
    staged_all<D, P, T, EB>(sm, tid, u);
#pragma unroll
    for (int m = 0; m < NM; ++m) u[m] = live ? u[m] : T(0);
  } else {
    const T* src = U + s * SE + (size_t)e * NM;
#pragma unroll
    for (int m = 0; m < NM; ++m) u[m] = live ? src[m] : T(0);
  }

  // ---- linear volume terms: -a_s |K| sum_a h_a^-2 (S along a) u + linear reactions --
  {
    const T as = T(c[K_MU1 + s]);
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
      R[m] = -as * vol * acc;
    }
    // S_lin: n1: -d1 n1; n2: -d2 n2; n3: (d1 - gamma) n1 + d2 n2; c1: f1 n3;
    //        c2: -k c2; c3: k c2.  Other species' modes of the same cell come from
    //        the staging area (3D) or global memory (the workgroup has just read them).
    const T* cell = U + (size_t)e * NM;
    if (s == S_N1 || s == S_N2 || s == S_C2) {
      const T k = -T(s == S_N1 ? c[K_D1] : s == S_N2 ? c[K_D2] : c[K_K]) * vol;
#pragma unroll
      for (int m = 0; m < NM; ++m) R[m] += k * u[m];
    } else if (live) {
      const int s0 = s == S_N3 ? S_N1 : s == S_C1 ? S_N3 : S_C2;
      const T* a0 = cell + s0 * SE;
      const T k0 = T(s == S_N3 ? c[K_D1] - c[K_GAM] : s == S_C1 ? c[K_F1] : c[K_K]) * vol;
#pragma unroll
      for (int m = 0; m < NM; ++m) R[m] += k0 * (STAGED ? staged<D, P, T, EB>(sm, s0 * EB + el, m) : a0[m]);
      if (s == S_N3) {
        const T* a1 = cell + S_N2 * SE;
        const T k1 = T(c[K_D2]) * vol;
#pragma unroll
        for (int m = 0; m < NM; ++m) R[m] += k1 * (STAGED ? staged<D, P, T, EB>(sm, S_N2 * EB + el, m) : a1[m]);
      }
    }
  }

  // ---- nonlinear volume terms, one layer of Gauss points at a time ------------------
  // producer quantity slots: 0 n1, 1 n2, 2 c1, 3 c3, 4+a grad n1, 4+D+a grad c1,
  // 4+2D+a grad c3.  After the point pass: slots 0..D-1 F1 (weighted, /h_a),
  // D..2D-1 F2, 2D alpha-term.
  const int prod = s == S_N1 ? 0 : s == S_N2 ? 1 : s == S_C1 ? 2 : s == S_C3 ? 3 : -1;
  const bool grads = s == S_N1 || s == S_C1 || s == S_C3;
  const int gslot = s == S_N1 ? 4 : s == S_C1 ? 4 + D : 4 + 2 * D;
  T* V = sm.buf;   // [EB][VST]: NVQ slots of PC points, then the pad
  constexpr int LA = D - 1;   // layer axis
  constexpr int LST = ipow(Q, D - 1);
  const double(*Bt0)[CDG2_MAXQ] = tb.B;
  for (int lc = 0; lc < Q; ++lc) {
    __syncthreads();
    if (prod >= 0) produce_layer<D, Q, T>(tb, g, u, lc, V + el * VST, prod, grads ? gslot : -1);
    __syncthreads();
    // point pass: chemotactic fluxes and the alpha reaction term, weighted
    for (int it = tid; it < EB * PC; it += NT) {
      const int l = it / PC, q = it % PC;
      T* v = V + l * VST + q;
      const T n1 = v[0], n2 = v[PC], c1 = v[2 * PC], c3 = v[3 * PC];
      const T d11 = c1 + T(c[K_XT11]), d13 = c3 + T(c[K_XT13]), d21 = c1 + T(c[K_XT21]),
              d22 = n1 + T(c[K_XT22]);
      if (e0 + l < E && !(d11 > T(0) && d13 > T(0) && d21 > T(0) && d22 > T(0))) flag |= FLAG_DOMAIN;
      T r11, r13, r21, r22;
      recip4(d11, d13, d21, d22, r11, r13, r21, r22);
      const T k11 = T(c[K_X011]) * r11, k13 = T(c[K_X013]) * r13, k21 = T(c[K_X021]) * r21,
              k22 = T(c[K_X022]) * r22;
      // weight of the point: |K| w_q (layer index lc along the last axis)
      T wt = vol * T(tb.w[lc]);
      if constexpr (D == 2) {
        wt *= T(tb.w[q]);
      } else {
        wt *= T(tb.w[q % Q]) * T(tb.w[q / Q]);
      }
      T F1[D], F2[D];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const T gn1 = v[(4 + a) * PC], gc1 = v[(4 + D + a) * PC], gc3 = v[(4 + 2 * D + a) * PC];
        F1[a] = n1 * (k11 * gc1 + k13 * gc3) * wt * T(g.ih[a]);
        F2[a] = n2 * (k21 * gc1 - k22 * gn1) * wt * T(g.ih[a]);
      }
      const T rc = -(T(c[K_AL1]) * n1 + T(c[K_AL2]) * n2) * c1 * wt;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        v[a * PC] = F1[a];
        v[(D + a) * PC] = F2[a];
      }
      v[2 * D * PC] = rc;
    }
    __syncthreads();
    // test integration of this layer: n1, n2 (F . grad phi), c1 (alpha term phi)
    if (s == S_N1 || s == S_N2 || s == S_C1) {
      const int base = s == S_N2 ? D : 0;
      T r[NF], acc[NF];
      if (s == S_C1) {
#pragma unroll
        for (int q = 0; q < PC; ++q) r[q] = V[el * VST + 2 * D * PC + q];
        tapply_lo<D, Q, true, T>(r, acc, Bt0, Bt0);
#pragma unroll
        for (int k = 0; k < Q; ++k)
#pragma unroll
          for (int m = 0; m < NF; ++m) R[m + LST * k] += T(tb.B[lc][k]) * acc[m];
      } else {
        // in-layer derivative directions: phi along the layer axis is B[lc][k]
        T sum[NF];
#pragma unroll
        for (int m = 0; m < NF; ++m) sum[m] = T(0);
#pragma unroll
        for (int a = 0; a < D - 1; ++a) {
#pragma unroll
          for (int q = 0; q < PC; ++q) r[q] = V[el * VST + (base + a) * PC + q];
          tapply_lo<D, Q, true, T>(r, acc, a == 0 ? tb.Bd : tb.B, a == 1 ? tb.Bd : tb.B);
#pragma unroll
          for (int m = 0; m < NF; ++m) sum[m] += acc[m];
        }
#pragma unroll
        for (int q = 0; q < PC; ++q) r[q] = V[el * VST + (base + LA) * PC + q];
        tapply_lo<D, Q, true, T>(r, acc, Bt0, Bt0);
#pragma unroll
        for (int k = 0; k < Q; ++k)
#pragma unroll
          for (int m = 0; m < NF; ++m)
            R[m + LST * k] += T(tb.B[lc][k]) * sum[m] + T(tb.Bd[lc][k]) * acc[m];
      }
    }
  }

  // ---- faces ------------------------------------------------------------------------
  const T as = T(c[K_MU1 + s]);
  const bool diss = !(g.llf_cells && s > S_N2);
  // face exchange slots (x NF): 0..3 values n1 n2 c1 c3 own, 4..7 same neighbour,
  // 8..10 d_a n1 c1 c3 own, 11..13 neighbour.  After the point pass: 0 lambda/2,
  // 1 -F1.n_o/2 sum, 2 -F2.n_o/2 sum, 3..5 inflow fluxes n1, n2, c2 (boundary).
  T* Fx = sm.buf;   // [EB][FST]: 14 slots of NF points, then the pad
  const int vslot = prod;   // value slot of this species (or -1)
  const int dslot = s == S_N1 ? 8 : s == S_C1 ? 9 : s == S_C3 ? 10 : -1;
  // the face axis is unrolled (a compile-time constant, so that the register
  // arrays u and R are indexed statically); the two sides of an axis are not
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll 1
  for (int sg = 0; sg < 2; ++sg) {
    const int f = 2 * a + sg;
    __syncthreads();
    // 3D: the neighbours' modes arrive in the staging area while the own traces
    // are formed

    const int nb = sm.nb[el][f];
    // tangential-modal traces: value / d_a of own and neighbour, accurate jump
    T uo[NF], duo[NF], un[NF], dun[NF], jm[NF];
#pragma unroll
    for (int J = 0; J < NF; ++J) {
      T a0 = T(0), a1 = T(0);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const T v = u[face_mode<D, Q>(a, i, J)];
        a0 += T(tb.E[sg][i]) * v;
        a1 += T(tb.dE[sg][i]) * v;
      }
      uo[J] = a0;
      duo[J] = a1 * T(g.ih[a]);
      un[J] = T(0);
      dun[J] = T(0);
      jm[J] = T(0);
    }
    if (nb >= 0) {
      const T* un_src = U + s * SE + (size_t)nb * NM;
#pragma unroll
      for (int J = 0; J < NF; ++J) {
        T a0 = T(0), a1 = T(0), a2 = T(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const int m = face_mode<D, Q>(a, i, J);
          const T v = un_src[m];
          a0 += T(tb.E[1 - sg][i]) * v;
          a1 += T(tb.dE[1 - sg][i]) * v;
          // u_o - u_n formed mode by mode: the i = 0 terms (value 1 at both ends)
          // cancel exactly
          a2 += i == 0 ? u[m] - v : T(tb.E[sg][i]) * u[m] - T(tb.E[1 - sg][i]) * v;
        }
        un[J] = a0;
        dun[J] = a1 * T(g.ih[a]);
        jm[J] = a2;
      }
    }
    // publish point values needed by the face point pass (the exchange slots
    // overlay the staging area: everyone has finished reading it)
    const int b0 = a == 0 ? 1 : 0, b1 = a == 2 ? 1 : 2;   // tangential axes
    const double(*Tb0)[CDG2_MAXQ] = tb.B;
    if (vslot >= 0) {
      T o[NF];
      tapply_lo<D, Q, false, T>(uo, o, Tb0, Tb0);
#pragma unroll
      for (int t = 0; t < NF; ++t) Fx[el * FST + vslot * NF + t] = o[t];
      tapply_lo<D, Q, false, T>(un, o, Tb0, Tb0);
#pragma unroll
      for (int t = 0; t < NF; ++t) Fx[el * FST + (4 + vslot) * NF + t] = o[t];
    }
    if (dslot >= 0) {
      T o[NF];
      tapply_lo<D, Q, false, T>(duo, o, Tb0, Tb0);
#pragma unroll
      for (int t = 0; t < NF; ++t) Fx[el * FST + dslot * NF + t] = o[t];
      tapply_lo<D, Q, false, T>(dun, o, Tb0, Tb0);
#pragma unroll
      for (int t = 0; t < NF; ++t) Fx[el * FST + (dslot + 3) * NF + t] = o[t];
    }
    // the species pass needs only the weighted derivative sum (own is K^- on the
    // high face, sg = 1) and the jump: formed now, so that the four trace arrays
    // are not live through the point pass
    const T wo = T(sg ? g.wm : g.wp), wn = T(sg ? g.wp : g.wm);
    T sd[NF];
#pragma unroll
    for (int J = 0; J < NF; ++J) sd[J] = wo * duo[J] + wn * dun[J];
    __syncthreads();
    // face point pass
    face_points<D, Q, NF, EB, FST, true, T>(Fx, sm.nb, f, sg, b0, c, g, tb, e0, E, tid, flag);
    __syncthreads();
    // species pass: nonlinear flux at the points, projected on the tangential modes,
    // plus the linear face terms; spread onto the normal modes
    {
      T gp[NF], gh[NF];
      const T* x = Fx + el * FST;
      if (nb >= 0) {
        T jp[NF];
        tapply_lo<D, Q, false, T>(jm, jp, Tb0, Tb0);
#pragma unroll
        for (int t = 0; t < NF; ++t) {
          T v = diss ? -x[t] * jp[t] : T(0);
          if (s == S_N1) v += x[NF + t];
          if (s == S_N2) v += x[2 * NF + t];
          gp[t] = v;
        }
      } else {
#pragma unroll
        for (int t = 0; t < NF; ++t) {
          gp[t] = s == S_N1 ? x[3 * NF + t] : s == S_N2 ? x[4 * NF + t] : s == S_C2 ? x[5 * NF + t] : T(0);
        }
      }
      // weights of the tangential Gauss points
#pragma unroll
      for (int t = 0; t < NF; ++t) {
        if constexpr (D == 2) {
          gp[t] *= T(tb.w[t]);
        } else {
          gp[t] *= T(tb.w[t % Q]) * T(tb.w[t / Q]);
        }
      }
      tapply_lo<D, Q, true, T>(gp, gh, Tb0, Tb0);
      const T ar = T(g.area[a]);
      const T so = sg ? T(1) : T(-1);
      const T pen = T(g.pen_c * tb.liftc * g.ih[a]) * as;
      T G[NF], H[NF];
#pragma unroll
      for (int J = 0; J < NF; ++J) {
        T lin = T(0), hh = T(0);
        if (nb >= 0) {
          lin = so * as * sd[J] - pen * jm[J];
          hh = wo * T(g.sym) * as * jm[J] * so * T(g.ih[a]);
        }
        G[J] = ar * (lin + gh[J]);
        H[J] = ar * hh;
      }
#pragma unroll
      for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int J = 0; J < NF; ++J)
          R[face_mode<D, Q>(a, i, J)] += T(tb.E[sg][i]) * G[J] + T(tb.dE[sg][i]) * H[J];
    }
  }

  // ---- M^{-1}, stage combination, store ---------------------------------------------
  if constexpr (STAGED) {
    // values into the staging area, then coalesced stores (and u0 loads) by
    // consecutive lanes over consecutive modes of consecutive cells
    const T ivol = T(1.0 / g.vol);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NM; ++m) sm.buf[tid * NM + m] = stage == 0 ? R[m] * ivol : cb * (u[m] + dt * (R[m] * ivol));
    __syncthreads();
    store_results<T, EB, NM>(sm.cell, sm.buf, U0, out, SE, ca, stage != 0 && ca != T(0), tid, flag);
  } else if (live) {
    const T ivol = T(1.0 / g.vol);
    T* dst = out + s * SE + (size_t)e * NM;
    if (stage == 0) {
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        const T v = R[m] * ivol;
        if (!isfinite(v)) flag |= FLAG_NONFINITE;
        dst[m] = v;
      }
    } else {
      const bool combine = ca != T(0);   // U0 is read (and non-null) only then
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        T v = cb * (u[m] + dt * (R[m] * ivol));
        if (combine) v += ca * U0[s * SE + (size_t)e * NM + m];
        if (!isfinite(v)) flag |= FLAG_NONFINITE;
        dst[m] = v;
      }
    }
  }
  if (flag) atomicOr(flags, flag);
}

template <int D, int P, typename T, int EB>
__global__ void __launch_bounds__(6 * EB)
es_kernel(const Params* __restrict__ prm, const T* __restrict__ U, const T* U0, T* out, T dt, T ca, T cb,
          int stage, int* __restrict__ flags) {
  __shared__ EsSmem<D, P, T, EB> sm;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  es_block<D, P, T, EB>(*prm, U, U0, out, dt, ca, cb, stage, flags, blk * EB, sm);
}

}  // namespace cdg2
