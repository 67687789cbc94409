// C-ABI implementation of libcdg2 (declarations and contract in include/cdg2.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>
#include <algorithm>
#include <array>
#include <mutex>

#include "../../include/cdg2.h"
#include "cfl_kernel.hpp"
#include "adj_kernel.hpp"
#include "batch_kernel.hpp"
#include "es_kernel.hpp"
#include "nodal_kernel.hpp"
#include "tri_kernel.hpp"
#include "tet_kernel.hpp"
#include "vec_kernel.hpp"
#include "tables.cpp"

using namespace cdg2;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess) return fail(CDG2_EHIP, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

}  // namespace

struct cdg2_handle {
  cdg2_config cfg;
  Tables tb;
  Geo geo;
  Coef coef;
  Params* dprm = nullptr;   // device copy of tb, geo, coef
  int dim, p, fp32;
  size_t ndof;
  void* stage[2] = {nullptr, nullptr};
  int* flags = nullptr;
  unsigned long long* red = nullptr;
  void* adj[2] = {nullptr, nullptr};   // adjoint stage buffers (allocated on first use)
  double* part = nullptr;              // per-workgroup parameter partials
  double* dth = nullptr;               // device accumulator of parameter derivatives
  int nblk_adj = 0;
  void* seg = nullptr;                 // adjoint segment workspace (3 states per step)
  size_t seg_cap = 0;                  // its capacity in states
  double* imp = nullptr;               // implicit integrator workspace (imp_nvec states)
  int imp_nvec = 0;
  double* imp_part = nullptr;          // dot-product partials
  double* imp_dres = nullptr;          // dot-product results (device)
  double* imp_dcoef = nullptr;         // combination coefficients (device)
  double* imp_hres = nullptr;          // pinned host copies
  double* imp_hcoef = nullptr;
  hipStream_t stream = nullptr;
  double rho_hat = 0.0;
  int device = 0;                      // device current at create
};

namespace {

void coef_from(const cdg2_coeffs& c, Coef* o) {
  const double v[K_NCOEFF] = {c.mu[0], c.mu[1], c.mu[2], c.nu[0], c.nu[1], c.nu[2],
                              c.chi0[0], c.chi0[1], c.chi0[2], c.chi0[3],
                              c.chith[0], c.chith[1], c.chith[2], c.chith[3],
                              c.d1, c.d2, c.gamma, c.alpha1, c.alpha2, c.f1, c.k,
                              c.beta1, c.beta2, c.sigma, c.c1_star, c.c1_sstar};
  std::memcpy(o->c, v, sizeof v);
}

int validate(const cdg2_config* c) {
  if (!c) return fail(CDG2_EINVAL, "config is NULL");
  if (c->dim != 2 && c->dim != 3) return fail(CDG2_EINVAL, "dim must be 2 or 3 (got %d)", c->dim);
  int pmax = c->dim == 2 ? 4 : 3;
  if (c->order < 1 || c->order > pmax)
    return fail(CDG2_EINVAL, "order must be in 1..%d for dim %d (got %d)", pmax, c->dim, c->order);
  for (int a = 0; a < c->dim; ++a)
    if (c->n[a] < 2 || c->n[a] > (1 << 16)) return fail(CDG2_EINVAL, "n[%d] must be in 2..65536", a);
  if (c->precision != CDG2_FP64 && c->precision != CDG2_FP32)
    return fail(CDG2_EINVAL, "precision must be CDG2_FP64 or CDG2_FP32");
  if (c->wall_axis < -1 || c->wall_axis >= c->dim) return fail(CDG2_EINVAL, "wall_axis out of range");
  if (c->llf_mode != CDG2_LLF_ALL && c->llf_mode != CDG2_LLF_CELLS) return fail(CDG2_EINVAL, "bad llf_mode");
  if (c->diff_flux < CDG2_FLUX_CDG2 || c->diff_flux > CDG2_FLUX_CDG) return fail(CDG2_EINVAL, "bad diff_flux");
  if (!(c->flux_eta >= 0) || !std::isfinite(c->flux_eta)) return fail(CDG2_EINVAL, "flux_eta must be finite and >= 0");
  if (!(c->gamma1_in[0] <= c->gamma1_in[1])) return fail(CDG2_EINVAL, "gamma1_in must be an interval");
  const double* v = &c->coeffs.mu[0];
  for (int i = 0; i < CDG2_NCOEFF; ++i)
    if (!std::isfinite(v[i])) return fail(CDG2_EINVAL, "coefficient %d is not finite", i);
  for (int i = 0; i < 6; ++i)
    if (v[i] < 0) return fail(CDG2_EINVAL, "diffusivities must be >= 0");
  size_t E = (size_t)c->n[0] * c->n[1] * (c->dim == 3 ? c->n[2] : 1);
  size_t nm = 1;
  for (int a = 0; a < c->dim; ++a) nm *= (size_t)(c->order + 1);
  if (6 * E * nm > (size_t)1 << 34) return fail(CDG2_EINVAL, "problem too large");
  return CDG2_OK;
}

void build_geo(const cdg2_config& c, Geo* g) {
  std::memset(g, 0, sizeof(Geo));
  g->E = 1;
  for (int a = 0; a < 3; ++a) {
    g->n[a] = a < c.dim ? c.n[a] : 1;
    g->h[a] = 1.0 / g->n[a];
    g->ih[a] = (double)g->n[a];
    g->E *= g->n[a];
  }
  g->wall = c.wall_axis;
  g->llf_cells = c.llf_mode == CDG2_LLF_CELLS;
  g->vol = 1.0;
  for (int a = 0; a < c.dim; ++a) g->vol *= g->h[a];
  for (int a = 0; a < c.dim; ++a) g->area[a] = g->vol / g->h[a];
  g->g1in[0] = c.gamma1_in[0];
  g->g1in[1] = c.gamma1_in[1];
  // stabilisation factor of the diffusion flux (times (p+1)^2 a / h [[u]] on
  // Cartesian cells) and the sign of its symmetry term
  const double nf = 2.0 * c.dim, eta = c.flux_eta > 0 ? c.flux_eta : 2.0 * c.dim;
  g->sym = 1.0;
  g->wm = g->wp = 0.5;
  switch (c.diff_flux) {
    case CDG2_FLUX_BR2: g->pen_c = 0.5 * eta; break;       // eta {r_e}: trace (p+1)^2/(2h) per side
    case CDG2_FLUX_IP: g->pen_c = eta; break;
    case CDG2_FLUX_BO: g->pen_c = 0.0; g->sym = -1.0; break;
    case CDG2_FLUX_CDG:   // one-sided on K^-: gradient plus the lifting of the whole jump there
      g->pen_c = 1.0;
      g->wm = 1.0;
      g->wp = 0.0;
      break;
    default: g->pen_c = 0.5 * nf; break;                    // CDG2: 2 chi_e r_e|K-, chi_e = N/2
  }
  g->tz = c.dim == 3 ? 8 : 0;   // slabs of 8 z-planes (processing order of the 3D kernel)
}

// ---- launch dispatch ----------------------------------------------------------

// Launch codes of run_op: 0 an operator application; 1, 2, 3 the SSP-RK3 stages
// (modes in and out); STAGE_POINTS1 + 0, 1, 2 the stages of a step whose
// intermediate states are point values (3D p <= 2 only: modes -> points,
// points -> points, points -> modes).
constexpr int STAGE_POINTS1 = 11;

// The SSP-RK3 step of rk_steps keeps its intermediate states as point values.
bool point_stages(const cdg2_handle* h) { return h->dim == 3 && h->p <= 2; }

// cells per workgroup of the (cell, species) kernel: 6 * EB threads.  3D: 10
// (one wavefront).  2D: 21 (two wavefronts of 63 lanes): at p = 4, whose
// registers allow 2 waves per SIMD, the CU's 8 wave slots hold four such
// workgroups but only two three-wave ones (Q4 apply 138 -> 128 us at 256^2);
// p <= 2 gained a little (Q2 apply 42.7 -> 42.0 us).  p = 3 keeps 32, the cells
// per work item of the batched default: with 21 the compiler contracted a few
// terms differently and p = 3 results differed from the batched kernel's in the
// last bits (5e-19 relative), where they are otherwise equal bit for bit.
template <int D, int P>
struct EsCfg {
  static constexpr int EB = D == 3 ? 10 : P == 3 ? 32 : 21;
};

template <int D, int P, typename T>
hipError_t launch_op(cdg2_handle* h, const void* U, const void* U0, void* out, double dt, double ca,
                     double cb, int stage) {
  constexpr int EB = EsCfg<D, P>::EB;
  int nb = (h->geo.E + EB - 1) / EB;
  // nodal form for 3D p <= 2; 3D p = 3 keeps the modal kernel (register budget)
  if constexpr (D == 3 && P <= 2) {
    // one kernel per launch kind: apply, stage without u0, stage with u0 (modes
    // in and out); the three stages of a step with point-value intermediates
    const int kind = stage == 0 ? 0 : stage >= STAGE_POINTS1 ? 3 + stage - STAGE_POINTS1 : ca == 0.0 ? 1 : 2;
    switch (kind) {
#define CDG2_ND_LAUNCH(KD)                                                                                  \
  case KD:                                                                                                   \
    hipLaunchKernelGGL((nd_kernel<P, T, EB, KD>), dim3(nb), dim3(6 * EB), 0, h->stream, h->dprm, (const T*)U, \
                       (const T*)U0, (T*)out, (T)dt, (T)ca, (T)cb, h->flags);                                \
    break;
      CDG2_ND_LAUNCH(0)
      CDG2_ND_LAUNCH(1)
      CDG2_ND_LAUNCH(2)
      CDG2_ND_LAUNCH(3)
      CDG2_ND_LAUNCH(4)
      CDG2_ND_LAUNCH(5)
#undef CDG2_ND_LAUNCH
      default: return hipErrorInvalidValue;
    }
  } else {
    if (stage >= STAGE_POINTS1) return hipErrorInvalidValue;   // the modal kernel has no point-value stages
    hipLaunchKernelGGL((es_kernel<D, P, T, EB>), dim3(nb), dim3(6 * EB), 0, h->stream, h->dprm,
                       (const T*)U, (const T*)U0, (T*)out, (T)dt, (T)ca, (T)cb, stage, h->flags);
  }
  return hipGetLastError();
}

template <int D, int P, typename T>
hipError_t launch_cfl(cdg2_handle* h, const void* U) {
  constexpr int EB = EsCfg<D, P>::EB;
  int nb = (h->geo.E + EB - 1) / EB;
  hipLaunchKernelGGL((cfl_kernel<D, P, T, EB>), dim3(nb), dim3(6 * EB), 0, h->stream, h->dprm, (const T*)U,
                     h->red, h->flags);
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_op(cdg2_handle* h, const void* U, const void* U0, void* out, double dt, double ca,
                       double cb, int stage) {
  switch (h->dim * 10 + h->p) {
    case 21: return launch_op<2, 1, T>(h, U, U0, out, dt, ca, cb, stage);
    case 22: return launch_op<2, 2, T>(h, U, U0, out, dt, ca, cb, stage);
    case 23: return launch_op<2, 3, T>(h, U, U0, out, dt, ca, cb, stage);
    case 24: return launch_op<2, 4, T>(h, U, U0, out, dt, ca, cb, stage);
    case 31: return launch_op<3, 1, T>(h, U, U0, out, dt, ca, cb, stage);
    case 32: return launch_op<3, 2, T>(h, U, U0, out, dt, ca, cb, stage);
    case 33: return launch_op<3, 3, T>(h, U, U0, out, dt, ca, cb, stage);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch_cfl(cdg2_handle* h, const void* U) {
  switch (h->dim * 10 + h->p) {
    case 21: return launch_cfl<2, 1, T>(h, U);
    case 22: return launch_cfl<2, 2, T>(h, U);
    case 23: return launch_cfl<2, 3, T>(h, U);
    case 24: return launch_cfl<2, 4, T>(h, U);
    case 31: return launch_cfl<3, 1, T>(h, U);
    case 32: return launch_cfl<3, 2, T>(h, U);
    case 33: return launch_cfl<3, 3, T>(h, U);
  }
  return hipErrorInvalidValue;
}

// Cells per adjoint workgroup: 21 cells = 126 threads = two wavefronts.  The
// adjoint's registers allow two waves per SIMD (2D p <= 2, 3D p = 1) or one:
// two-wave workgroups fill all eight (or four) wave slots of a CU, where
// three-wave ones left two (or one) idle.
constexpr int ADJ_EB = 21;

template <int D, int P>
struct AdjCfg {
  static constexpr int EB = ADJ_EB;
};

template <int D, int P, typename T>
hipError_t launch_adj(cdg2_handle* h, const void* U, const void* W, void* out, double cw, double cj,
                      const void* X2, double c2, const void* X3, double c3, int want_theta, bool reduce) {
  constexpr int EB = AdjCfg<D, P>::EB;
  int nb = (h->geo.E + EB - 1) / EB;
  hipLaunchKernelGGL((adj_kernel<D, P, T, EB>), dim3(nb), dim3(6 * EB), 0, h->stream, h->dprm, (const T*)U,
                     (const T*)W, (T*)out, (T)cw, (T)cj, (const T*)X2, (T)c2, (const T*)X3, (T)c3, h->part,
                     want_theta, h->flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !reduce) return e;
  hipLaunchKernelGGL(theta_reduce_kernel, dim3(CDG2_NDIFF), dim3(256), 0, h->stream, (const double*)h->part, nb,
                     h->dth);
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_adj(cdg2_handle* h, const void* U, const void* W, void* out, double cw, double cj,
                        const void* X2, double c2, const void* X3, double c3, int want_theta, bool reduce) {
  switch (h->dim * 10 + h->p) {
    case 21: return launch_adj<2, 1, T>(h, U, W, out, cw, cj, X2, c2, X3, c3, want_theta, reduce);
    case 22: return launch_adj<2, 2, T>(h, U, W, out, cw, cj, X2, c2, X3, c3, want_theta, reduce);
    case 23: return launch_adj<2, 3, T>(h, U, W, out, cw, cj, X2, c2, X3, c3, want_theta, reduce);
    case 24: return launch_adj<2, 4, T>(h, U, W, out, cw, cj, X2, c2, X3, c3, want_theta, reduce);
    case 31: return launch_adj<3, 1, T>(h, U, W, out, cw, cj, X2, c2, X3, c3, want_theta, reduce);
    case 32: return launch_adj<3, 2, T>(h, U, W, out, cw, cj, X2, c2, X3, c3, want_theta, reduce);
    case 33: return launch_adj<3, 3, T>(h, U, W, out, cw, cj, X2, c2, X3, c3, want_theta, reduce);
  }
  return hipErrorInvalidValue;
}

// want_theta: 0 no parameter derivatives, 1 per-workgroup partials written,
// 2 added to the partials of the previous call; reduce: sum the partials into
// h->dth after the launch.
hipError_t run_adj(cdg2_handle* h, const void* U, const void* W, void* out, double cw, double cj,
                   const void* X2, double c2, const void* X3, double c3, int want_theta, bool reduce) {
  return h->fp32 ? dispatch_adj<float>(h, U, W, out, cw, cj, X2, c2, X3, c3, want_theta, reduce)
                 : dispatch_adj<double>(h, U, W, out, cw, cj, X2, c2, X3, c3, want_theta, reduce);
}

// Adjoint buffers, allocated on the first adjoint call.
int ensure_adjoint(cdg2_handle* h) {
  // the adjoint applies the diffusion form to the adjoint state unchanged, which
  // needs the form to be symmetric
  if (h->geo.sym < 0 || h->geo.wm != 0.5)
    return fail(CDG2_EINVAL, "the adjoint needs a central symmetric diffusion flux (CDG2, BR2 or IP)");
  if (h->part) return CDG2_OK;
  size_t bytes = h->ndof * (h->fp32 ? 4 : 8);
  int nb = (h->geo.E + ADJ_EB - 1) / ADJ_EB;
  for (int k = 0; k < 2; ++k)
    if (hipMalloc(&h->adj[k], bytes) != hipSuccess) return fail(CDG2_ENOMEM, "hipMalloc of adjoint buffers failed");
  if (hipMalloc((void**)&h->dth, 64 * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->part, (size_t)nb * CDG2_NDIFF * sizeof(double)) != hipSuccess)
    return fail(CDG2_ENOMEM, "hipMalloc of parameter buffers failed");
  h->nblk_adj = nb;
  return CDG2_OK;
}

hipError_t run_op(cdg2_handle* h, const void* U, const void* U0, void* out, double dt, double ca, double cb,
                  int stage) {
  return h->fp32 ? dispatch_op<float>(h, U, U0, out, dt, ca, cb, stage)
                 : dispatch_op<double>(h, U, U0, out, dt, ca, cb, stage);
}

hipError_t upload_params(cdg2_handle* h) {
  Params p;
  p.tb = h->tb;
  p.g = h->geo;
  p.cf = h->coef;
  // pageable source: the copy is staged before the call returns, in stream order
  return hipMemcpyAsync(h->dprm, &p, sizeof(Params), hipMemcpyHostToDevice, h->stream);
}

bool overlap(const void* a, const void* b, size_t bytes) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + bytes && y < x + bytes;
}

// 3D launches move whole cells with 16-byte load-to-LDS chunks: their state
// buffers must be 16-byte aligned (device allocations are)
bool misaligned(const cdg2_handle* h, const void* p) {
  return h->dim == 3 && ((uintptr_t)p & 15) != 0;
}

// [a, a + na) and [b, b + nb) intersect
bool overlap2(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + nb && y < x + na;
}


// ---- scratch memory of the allocation-free entry point ------------------------------

// The two intermediate SSP-RK3 states of cdg2_rk_step_noalloc.  A file-scope
// device array: every GPU the library runs on holds its own copy from module load
// until the process ends.  In host code its name is only a host-side stand-in, so
// the kernels get the device address that hipGetSymbolAddress returns for the
// current device (looked up once per device at cdg2_create, kept in scratch_dev).
static __device__ __align__(256) unsigned char scratch[CDG2_SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[SCRATCH_MAX_DEVICES] = {};

// Look up (once) the device address of the scratch array on the current device.
int scratch_setup(int device) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) return fail(CDG2_EINVAL, "device index %d out of range", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return CDG2_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(CDG2_EHIP, "hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
  g_scratch_dev[device] = ptr;
  return CDG2_OK;
}

void* scratch_device(int device) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_dev[device];
}

// nsteps fused SSP-RK3 steps on U with the intermediate states in st0, st1.
// On the nodal 3D path the two intermediate states are point values (the
// stage kernels of kinds 3 to 5); the states the adjoint recomputes stay modes.
int rk_steps(cdg2_handle* h, void* U, double dt, int nsteps, void* st0, void* st1) {
  const int k0 = point_stages(h) ? STAGE_POINTS1 : 1;
  for (int n = 0; n < nsteps; ++n) {
    HIP_TRY(run_op(h, U, nullptr, st0, dt, 0.0, 1.0, k0));
    HIP_TRY(run_op(h, st0, U, st1, dt, 0.75, 0.25, k0 + 1));
    HIP_TRY(run_op(h, st1, U, U, dt, 1.0 / 3.0, 2.0 / 3.0, k0 + 2));
  }
  return CDG2_OK;
}

// ---- implicit SDIRK integrator: Jacobian-free Newton-Krylov (GMRES) ---------------

constexpr int IMP_KMAX = 64;   // largest Krylov dimension
constexpr int IMP_FIXED = 13;  // 5 stage derivatives + rhs, X, F, G, T, Fe, W, out

// Butcher tableau of the L-stable, stiffly accurate SDIRK scheme of an order.
struct Sdirk {
  int s = 0;
  double A[5][5] = {};
  double b[5] = {};
};

bool sdirk(int order, Sdirk* t) {
  *t = Sdirk();
  if (order == 2) {
    const double g = 1.0 - 1.0 / std::sqrt(2.0);
    t->s = 2;
    t->A[0][0] = g;
    t->A[1][0] = 1.0 - g;
    t->A[1][1] = g;
  } else if (order == 3) {
    // gamma: root in (1/6, 1/2) of x^3 - 3x^2 + 3x/2 - 1/6 (Newton from 0.44)
    double g = 0.44;
    for (int it = 0; it < 60; ++it) g -= (((g - 3.0) * g + 1.5) * g - 1.0 / 6.0) / ((3.0 * g - 6.0) * g + 1.5);
    t->s = 3;
    t->A[0][0] = g;
    t->A[1][0] = 0.5 * (1.0 - g);
    t->A[1][1] = g;
    t->A[2][0] = -(6.0 * g * g - 16.0 * g + 1.0) / 4.0;
    t->A[2][1] = (6.0 * g * g - 20.0 * g + 5.0) / 4.0;
    t->A[2][2] = g;
  } else if (order == 4) {
    const double A[5][5] = {{1.0 / 4, 0, 0, 0, 0},
                            {1.0 / 2, 1.0 / 4, 0, 0, 0},
                            {17.0 / 50, -1.0 / 25, 1.0 / 4, 0, 0},
                            {371.0 / 1360, -137.0 / 2720, 15.0 / 544, 1.0 / 4, 0},
                            {25.0 / 24, -49.0 / 48, 125.0 / 16, -85.0 / 12, 1.0 / 4}};
    t->s = 5;
    std::memcpy(t->A, A, sizeof A);
  } else {
    return false;
  }
  for (int i = 0; i < t->s; ++i) t->b[i] = t->A[t->s - 1][i];   // stiffly accurate
  return true;
}

int ensure_implicit(cdg2_handle* h, int kdim) {
  const int nvec = IMP_FIXED + kdim + 1;
  if (h->imp && h->imp_nvec >= nvec) return CDG2_OK;
  if (h->imp) {
    HIP_TRY(hipStreamSynchronize(h->stream));
    (void)hipFree(h->imp);
    h->imp = nullptr;
    h->imp_nvec = 0;
  }
  if (hipMalloc((void**)&h->imp, (size_t)nvec * h->ndof * sizeof(double)) != hipSuccess)
    return fail(CDG2_ENOMEM, "hipMalloc of the implicit workspace (%d states) failed", nvec);
  h->imp_nvec = nvec;
  if (!h->imp_part) {
    if (hipMalloc((void**)&h->imp_part, (size_t)DOT_NB * (IMP_KMAX + 2) * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&h->imp_dres, 2 * (IMP_KMAX + 2) * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&h->imp_dcoef, (IMP_KMAX + 2) * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void**)&h->imp_hres, 2 * (IMP_KMAX + 2) * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h->imp_hcoef, (IMP_KMAX + 2) * sizeof(double), hipHostMallocDefault) != hipSuccess)
      return fail(CDG2_ENOMEM, "allocation of the implicit reduction buffers failed");
  }
  return CDG2_OK;
}

struct Vec {
  cdg2_handle* h;
  size_t n;
  int grid() const {
    size_t g = (n + VEC_NT - 1) / VEC_NT;
    return (int)(g < 4096 ? g : 4096);
  }
  hipError_t lc(double* out, const double* x0, double a0, const double* x1 = nullptr, double a1 = 0.0,
                const double* x2 = nullptr, double a2 = 0.0, const double* x3 = nullptr, double a3 = 0.0) const {
    hipLaunchKernelGGL(lincomb_kernel, dim3(grid()), dim3(VEC_NT), 0, h->stream, n, out, x0, a0, x1, a1, x2, a2,
                       x3, a3);
    return hipGetLastError();
  }
  // dots of w with V_0..V_{k-1} (stride n) and, if self, with itself -> out[0..k(+1))
  hipError_t dots(const double* w, const double* V, int k, int self, double* out) const {
    const int kk = k + (self ? 1 : 0);
    hipLaunchKernelGGL(dots_kernel, dim3(DOT_NB, (kk + DOT_W - 1) / DOT_W), dim3(VEC_NT), 0, h->stream, n, w, V, n,
                       k, self, h->imp_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dots_reduce_kernel, dim3(kk), dim3(VEC_NT), 0, h->stream, (const double*)h->imp_part,
                       h->imp_dres);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(h->imp_hres, h->imp_dres, kk * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return e;
    std::memcpy(out, h->imp_hres, kk * sizeof(double));
    return hipSuccess;
  }
  // the same dots left on the device at h->imp_dres + off (no host wait)
  hipError_t dots_dev(const double* w, const double* V, int k, int self, int off) const {
    const int kk = k + (self ? 1 : 0);
    hipLaunchKernelGGL(dots_kernel, dim3(DOT_NB, (kk + DOT_W - 1) / DOT_W), dim3(VEC_NT), 0, h->stream, n, w, V, n,
                       k, self, h->imp_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dots_reduce_kernel, dim3(kk), dim3(VEC_NT), 0, h->stream, (const double*)h->imp_part,
                       h->imp_dres + off);
    return hipGetLastError();
  }
  // w -= scale sum_j c[j] V_j with c on the device
  hipError_t maxpy_dev(double* w, const double* V, int k, const double* c, double scale) const {
    hipLaunchKernelGGL(multi_axpy_kernel, dim3(grid()), dim3(VEC_NT), 0, h->stream, n, w, V, n, k, c, scale);
    return hipGetLastError();
  }
  // copy cnt device results from offset 0 to the host (waits for the stream)
  hipError_t fetch(int cnt, double* out) const {
    hipError_t e = hipMemcpyAsync(h->imp_hres, h->imp_dres, cnt * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return e;
    std::memcpy(out, h->imp_hres, cnt * sizeof(double));
    return hipSuccess;
  }
  double norm_of(const double* x, hipError_t* e) const {
    double r = 0.0;
    *e = dots(x, nullptr, 0, 1, &r);
    return std::sqrt(r);
  }
  // w -= scale sum_j c[j] V_j   (c: host values, copied through the pinned buffer;
  // the previous copy has completed: every dots() waits for the stream)
  hipError_t maxpy(double* w, const double* V, int k, const double* c, double scale) const {
    std::memcpy(h->imp_hcoef, c, k * sizeof(double));
    hipError_t e = hipMemcpyAsync(h->imp_dcoef, h->imp_hcoef, k * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(multi_axpy_kernel, dim3(grid()), dim3(VEC_NT), 0, h->stream, n, w, V, n, k,
                       (const double*)h->imp_dcoef, scale);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // keep the pinned coefficients alive until the copy has run
    return hipStreamSynchronize(h->stream);
  }
};

}  // namespace

extern "C" {

int cdg2_create(const cdg2_config* cfg, cdg2_handle** out) {
  if (!out) return fail(CDG2_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(cfg);
  if (rc) return rc;
  cdg2_handle* h = new (std::nothrow) cdg2_handle();
  if (!h) return fail(CDG2_ENOMEM, "host allocation failed");
  h->cfg = *cfg;
  h->dim = cfg->dim;
  h->p = cfg->order;
  h->fp32 = cfg->precision == CDG2_FP32;
  build_tables(h->p, &h->tb);
  build_geo(*cfg, &h->geo);
  coef_from(cfg->coeffs, &h->coef);
  size_t nm = 1;
  for (int a = 0; a < h->dim; ++a) nm *= (size_t)(h->p + 1);
  h->ndof = 6 * (size_t)h->geo.E * nm;
  h->rho_hat = spectral_constant_1d(h->p, h->geo.pen_c, h->geo.sym, h->geo.wm, h->geo.wp);
  size_t bytes = h->ndof * (h->fp32 ? 4 : 8);
  for (int k = 0; k < 2; ++k) {
    if (hipMalloc(&h->stage[k], bytes) != hipSuccess) {
      cdg2_destroy(h);
      return fail(CDG2_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
  }
  if (hipMalloc((void**)&h->flags, 64) != hipSuccess || hipMalloc((void**)&h->red, 64) != hipSuccess ||
      hipMalloc((void**)&h->dprm, sizeof(Params)) != hipSuccess) {
    cdg2_destroy(h);
    return fail(CDG2_ENOMEM, "hipMalloc of flag buffers failed");
  }
  if (hipMemset(h->flags, 0, 64) != hipSuccess || upload_params(h) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    cdg2_destroy(h);
    return fail(CDG2_EHIP, "device initialisation failed");
  }
  if (hipGetDevice(&h->device) != hipSuccess) {
    cdg2_destroy(h);
    return fail(CDG2_EHIP, "hipGetDevice failed");
  }
  rc = scratch_setup(h->device);
  if (rc) {
    cdg2_destroy(h);
    return rc;
  }
  *out = h;
  return CDG2_OK;
}

int cdg2_destroy(cdg2_handle* h) {
  if (!h) return CDG2_OK;
  for (int k = 0; k < 2; ++k)
    if (h->stage[k]) (void)hipFree(h->stage[k]);
  if (h->flags) (void)hipFree(h->flags);
  if (h->red) (void)hipFree(h->red);
  if (h->dprm) (void)hipFree(h->dprm);
  for (int k = 0; k < 2; ++k)
    if (h->adj[k]) (void)hipFree(h->adj[k]);
  if (h->part) (void)hipFree(h->part);
  if (h->dth) (void)hipFree(h->dth);
  if (h->seg) (void)hipFree(h->seg);
  if (h->imp) (void)hipFree(h->imp);
  if (h->imp_part) (void)hipFree(h->imp_part);
  if (h->imp_dres) (void)hipFree(h->imp_dres);
  if (h->imp_dcoef) (void)hipFree(h->imp_dcoef);
  if (h->imp_hres) (void)hipHostFree(h->imp_hres);
  if (h->imp_hcoef) (void)hipHostFree(h->imp_hcoef);
  delete h;
  return CDG2_OK;
}

int cdg2_set_stream(cdg2_handle* h, void* s) {
  if (!h) return fail(CDG2_EINVAL, "handle is NULL");
  h->stream = (hipStream_t)s;
  return CDG2_OK;
}

int cdg2_set_coeffs(cdg2_handle* h, const cdg2_coeffs* c) {
  if (!h || !c) return fail(CDG2_EINVAL, "NULL argument");
  cdg2_config tmp = h->cfg;
  tmp.coeffs = *c;
  int rc = validate(&tmp);
  if (rc) return rc;
  h->cfg.coeffs = *c;
  coef_from(*c, &h->coef);
  HIP_TRY(upload_params(h));
  return CDG2_OK;
}

size_t cdg2_num_dofs(const cdg2_handle* h) { return h ? h->ndof : 0; }

double cdg2_rho_hat(const cdg2_handle* h) { return h ? h->rho_hat : 0.0; }

int cdg2_apply_operator(cdg2_handle* h, const void* U, void* dUdt) {
  if (!h || !U || !dUdt) return fail(CDG2_EINVAL, "NULL argument");
  size_t bytes = h->ndof * (h->fp32 ? 4 : 8);
  if (overlap(U, dUdt, bytes)) return fail(CDG2_EINVAL, "U and dUdt overlap");
  if (misaligned(h, U) || misaligned(h, dUdt)) return fail(CDG2_EINVAL, "3D state buffers must be 16-byte aligned");
  HIP_TRY(run_op(h, U, nullptr, dUdt, 0.0, 0.0, 1.0, 0));
  return CDG2_OK;
}

int cdg2_rk_step(cdg2_handle* h, void* U, double dt, int nsteps) {
  if (!h || !U) return fail(CDG2_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(CDG2_EINVAL, "nsteps < 0");
  if (!std::isfinite(dt)) return fail(CDG2_EINVAL, "dt is not finite");
  size_t bytes = h->ndof * (h->fp32 ? 4 : 8);
  if (overlap(U, h->stage[0], bytes) || overlap(U, h->stage[1], bytes))
    return fail(CDG2_EINVAL, "U overlaps a stage buffer");
  if (misaligned(h, U)) return fail(CDG2_EINVAL, "3D state buffers must be 16-byte aligned");
  return rk_steps(h, U, dt, nsteps, h->stage[0], h->stage[1]);
}

int cdg2_rk_step_noalloc(cdg2_handle* h, void* U, double dt, int nsteps) {
  if (!h || !U) return fail(CDG2_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(CDG2_EINVAL, "nsteps < 0");
  if (!std::isfinite(dt)) return fail(CDG2_EINVAL, "dt is not finite");
  const size_t bytes = h->ndof * (h->fp32 ? 4 : 8);
  const size_t slot = (bytes + 255) / 256 * 256;   // second state 256-byte aligned
  if (slot > CDG2_SCRATCH_BYTES / 2)
    return fail(CDG2_EINVAL, "state of %zu bytes exceeds the scratch limit of %zu bytes per state", bytes,
                (size_t)CDG2_SCRATCH_BYTES / 2);
  char* base = (char*)scratch_device(h->device);
  if (!base) return fail(CDG2_EINVAL, "scratch memory not set up on device %d", h->device);
  if (overlap2(U, bytes, base, CDG2_SCRATCH_BYTES)) return fail(CDG2_EINVAL, "U overlaps the scratch memory");
  if (misaligned(h, U)) return fail(CDG2_EINVAL, "3D state buffers must be 16-byte aligned");
  return rk_steps(h, U, dt, nsteps, base, base + slot);
}

int cdg2_apply_adjoint(cdg2_handle* h, const void* U, const void* w, void* JTw, double* dtheta) {
  if (!h || !U || !w || !JTw) return fail(CDG2_EINVAL, "NULL argument");
  size_t bytes = h->ndof * (h->fp32 ? 4 : 8);
  if (overlap(JTw, U, bytes) || overlap(JTw, w, bytes)) return fail(CDG2_EINVAL, "JTw overlaps U or w");
  int rc = ensure_adjoint(h);
  if (rc) return rc;
  if (dtheta) HIP_TRY(hipMemsetAsync(h->dth, 0, CDG2_NDIFF * sizeof(double), h->stream));
  HIP_TRY(run_adj(h, U, w, JTw, 0.0, 1.0, nullptr, 0.0, nullptr, 0.0, dtheta != nullptr, dtheta != nullptr));
  if (dtheta) {
    HIP_TRY(hipMemcpyAsync(dtheta, h->dth, CDG2_NDIFF * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
  }
  return CDG2_OK;
}

int cdg2_rk_step_adjoint(cdg2_handle* h, const void* U_n, const void* lam_np1, void* lam_n, double dt,
                         double* dtheta_acc) {
  if (!h || !U_n || !lam_np1 || !lam_n) return fail(CDG2_EINVAL, "NULL argument");
  if (!std::isfinite(dt)) return fail(CDG2_EINVAL, "dt is not finite");
  size_t bytes = h->ndof * (h->fp32 ? 4 : 8);
  if (overlap(lam_n, U_n, bytes)) return fail(CDG2_EINVAL, "lam_n overlaps U_n");
  if (misaligned(h, U_n)) return fail(CDG2_EINVAL, "3D state buffers must be 16-byte aligned");
  int rc = ensure_adjoint(h);
  if (rc) return rc;
  const int th = dtheta_acc != nullptr;
  double* acc_save = h->dth;
  if (th) h->dth = dtheta_acc;   // the reductions add straight into the caller's buffer
  // forward stages of the step, recomputed from U_n
  hipError_t e = run_op(h, U_n, nullptr, h->stage[0], dt, 0.0, 1.0, 1);
  if (e == hipSuccess) e = run_op(h, h->stage[0], U_n, h->stage[1], dt, 0.75, 0.25, 2);
  // reverse sweep of the Shu-Osher stages
  //   lam2 = 2/3 lam3 + 2/3 dt J(U2)^T lam3
  //   lam1 = 1/4 lam2 + 1/4 dt J(U1)^T lam2
  //   lam_n = 1/3 lam3 + 3/4 lam2 + lam1 + dt J(U_n)^T lam1
  if (e == hipSuccess)
    e = run_adj(h, h->stage[1], lam_np1, h->adj[0], 2.0 / 3.0, 2.0 / 3.0 * dt, nullptr, 0.0, nullptr, 0.0, th,
                false);
  if (e == hipSuccess)
    e = run_adj(h, h->stage[0], h->adj[0], h->adj[1], 0.25, 0.25 * dt, nullptr, 0.0, nullptr, 0.0, th ? 2 : 0,
                false);
  // the three stages' partials are summed per workgroup, then reduced once
  if (e == hipSuccess)
    e = run_adj(h, U_n, h->adj[1], lam_n, 1.0, dt, lam_np1, 1.0 / 3.0, h->adj[0], 0.75, th ? 2 : 0, th);
  h->dth = acc_save;
  if (e != hipSuccess) return fail(CDG2_EHIP, "adjoint step launch: %s", hipGetErrorString(e));
  return CDG2_OK;
}

int cdg2_rk_adjoint_segment(cdg2_handle* h, const void* U_start, int nsteps, double dt, void* lam,
                            double* dtheta_acc) {
  if (!h || !U_start || !lam) return fail(CDG2_EINVAL, "NULL argument");
  if (nsteps < 1) return fail(CDG2_EINVAL, "nsteps must be >= 1 (got %d)", nsteps);
  if (!std::isfinite(dt)) return fail(CDG2_EINVAL, "dt is not finite");
  const size_t esz = h->fp32 ? 4 : 8;
  const size_t bytes = h->ndof * esz;
  if (overlap(lam, U_start, bytes)) return fail(CDG2_EINVAL, "lam overlaps U_start");
  int rc = ensure_adjoint(h);
  if (rc) return rc;
  const size_t need = 3 * (size_t)nsteps;
  if (need > h->seg_cap) {
    // the stream may still use the old workspace
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (h->seg) (void)hipFree(h->seg);
    h->seg = nullptr;
    h->seg_cap = 0;
    if (hipMalloc(&h->seg, need * bytes) != hipSuccess)
      return fail(CDG2_ENOMEM, "hipMalloc of the adjoint segment workspace (%zu states) failed", need);
    h->seg_cap = need;
  }
  auto st = [&](size_t k) { return (void*)((char*)h->seg + k * bytes); };
  // forward: X^n at 3n, U1 at 3n+1, U2 at 3n+2; stage 3 writes X^{n+1} at 3n+3
  // (not needed after the last step)
  hipError_t e = hipMemcpyAsync(st(0), U_start, bytes, hipMemcpyDeviceToDevice, h->stream);
  for (int n = 0; n < nsteps && e == hipSuccess; ++n) {
    e = run_op(h, st(3 * n), nullptr, st(3 * n + 1), dt, 0.0, 1.0, 1);
    if (e == hipSuccess) e = run_op(h, st(3 * n + 1), st(3 * n), st(3 * n + 2), dt, 0.75, 0.25, 2);
    if (e == hipSuccess && n + 1 < nsteps)
      e = run_op(h, st(3 * n + 2), st(3 * n), st(3 * n + 3), dt, 1.0 / 3.0, 2.0 / 3.0, 3);
  }
  // reverse sweep (recurrences of cdg2_rk_step_adjoint), lam in place
  const int th = dtheta_acc != nullptr;
  double* acc_save = h->dth;
  if (th) h->dth = dtheta_acc;
  for (int n = nsteps - 1; n >= 0 && e == hipSuccess; --n) {
    const int first = th && n == nsteps - 1 ? 1 : th ? 2 : 0;
    e = run_adj(h, st(3 * n + 2), lam, h->adj[0], 2.0 / 3.0, 2.0 / 3.0 * dt, nullptr, 0.0, nullptr, 0.0, first,
                false);
    if (e == hipSuccess)
      e = run_adj(h, st(3 * n + 1), h->adj[0], h->adj[1], 0.25, 0.25 * dt, nullptr, 0.0, nullptr, 0.0,
                  th ? 2 : 0, false);
    if (e == hipSuccess)
      e = run_adj(h, st(3 * n), h->adj[1], lam, 1.0, dt, lam, 1.0 / 3.0, h->adj[0], 0.75, th ? 2 : 0,
                  th && n == 0);
  }
  h->dth = acc_save;
  if (e != hipSuccess) return fail(CDG2_EHIP, "adjoint segment launch: %s", hipGetErrorString(e));
  return CDG2_OK;
}


int cdg2_dirk_step(cdg2_handle* h, void* U, double dt, const cdg2_implicit_opts* opts,
                   cdg2_implicit_stats* stats) {
  if (!h || !U) return fail(CDG2_EINVAL, "NULL argument");
  if (h->fp32) return fail(CDG2_EINVAL, "the implicit integrator needs a CDG2_FP64 handle");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(CDG2_EINVAL, "dt must be finite and > 0");
  cdg2_implicit_opts o = {3, 10, 30, 1e-10, 1e-3};
  if (opts) o = *opts;
  Sdirk tab;
  if (!sdirk(o.order, &tab)) return fail(CDG2_EINVAL, "order must be 2, 3 or 4 (got %d)", o.order);
  if (o.max_newton < 1) return fail(CDG2_EINVAL, "max_newton must be >= 1");
  if (o.krylov_dim < 1 || o.krylov_dim > IMP_KMAX) return fail(CDG2_EINVAL, "krylov_dim must be in 1..%d", IMP_KMAX);
  if (!(o.newton_rtol > 0) || !(o.krylov_rtol > 0)) return fail(CDG2_EINVAL, "tolerances must be > 0");
  int rc = ensure_implicit(h, o.krylov_dim);
  if (rc) return rc;
  const size_t n = h->ndof;
  if (overlap2(U, n * sizeof(double), h->imp, (size_t)h->imp_nvec * n * sizeof(double)))
    return fail(CDG2_EINVAL, "U overlaps the implicit workspace");
  double* W0 = h->imp;
  auto vec = [&](int k) { return W0 + (size_t)k * n; };
  double* K[5] = {vec(0), vec(1), vec(2), vec(3), vec(4)};
  double *rhs = vec(5), *X = vec(6), *F = vec(7), *G = vec(8), *T = vec(9), *Fe = vec(10), *Wv = vec(11),
         *out = vec(12);
  double* V = vec(IMP_FIXED);
  const double* Un = (const double*)U;
  const Vec v{h, n};
  const int m = o.krylov_dim;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), h1(m + 2), h2(m + 2);
  auto Hij = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  cdg2_implicit_stats st = {0, 0, 1, 0, 0.0};
  hipError_t e = hipSuccess;
#define IMP_TRY(expr)                                                       \
  do {                                                                      \
    e = (expr);                                                             \
    if (e != hipSuccess) return fail(CDG2_EHIP, "implicit step: %s", hipGetErrorString(e)); \
  } while (0)
  for (int i = 0; i < tab.s; ++i) {
    // rhs_i = U^n + dt sum_{j<i} a_ij K_j (in groups of three terms)
    IMP_TRY(v.lc(rhs, Un, 1.0));
    for (int j0 = 0; j0 < i; j0 += 3) {
      const int j1 = j0 + 1 < i ? j0 + 1 : -1, j2 = j0 + 2 < i ? j0 + 2 : -1;
      IMP_TRY(v.lc(rhs, rhs, 1.0, K[j0], dt * tab.A[i][j0], j1 >= 0 ? K[j1] : nullptr,
                   j1 >= 0 ? dt * tab.A[i][j1] : 0.0, j2 >= 0 ? K[j2] : nullptr, j2 >= 0 ? dt * tab.A[i][j2] : 0.0));
    }
    const double dg = dt * tab.A[i][i];
    IMP_TRY(v.lc(X, rhs, 1.0));
    bool ok = false;
    double rel = 0.0;
    for (int it = 0; it <= o.max_newton; ++it) {
      IMP_TRY(run_op(h, X, nullptr, F, 0.0, 0.0, 1.0, 0));
      IMP_TRY(v.lc(G, X, 1.0, F, -dg, rhs, -1.0));
      const double nG = v.norm_of(G, &e);
      if (e != hipSuccess) return fail(CDG2_EHIP, "implicit step: %s", hipGetErrorString(e));
      const double nX = v.norm_of(X, &e);
      if (e != hipSuccess) return fail(CDG2_EHIP, "implicit step: %s", hipGetErrorString(e));
      const double nF = v.norm_of(F, &e);
      if (e != hipSuccess) return fail(CDG2_EHIP, "implicit step: %s", hipGetErrorString(e));
      if (!std::isfinite(nG) || !std::isfinite(nX) || !std::isfinite(nF))
        return fail(CDG2_ENONFINITE, "non-finite value in the implicit stage iteration");
      const double scale = nX + dg * nF;
      rel = scale > 0 ? nG / scale : nG;
      if (nG <= o.newton_rtol * scale) {
        ok = true;
        break;
      }
      if (it == o.max_newton) break;
      ++st.newton_iters;
      // GMRES on (I - dg J(X)) d = -G from d = 0: V_0 = -G / ||G||
      const double beta = nG;
      IMP_TRY(v.lc(V, G, -1.0 / beta));
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      const double eps = std::sqrt(2.220446049250313e-16) * (1.0 + nX);
      int jend = 0;
      for (int j = 0; j < m; ++j) {
        double* Vj = V + (size_t)j * n;
        double* Vn = V + (size_t)(j + 1) * n;
        // W = V_j - dg (f(X + eps V_j) - f(X)) / eps
        IMP_TRY(v.lc(T, X, 1.0, Vj, eps));
        IMP_TRY(run_op(h, T, nullptr, Fe, 0.0, 0.0, 1.0, 0));
        IMP_TRY(v.lc(Wv, Vj, 1.0, Fe, -dg / eps, F, dg / eps));
        // classical Gram-Schmidt with the coefficients kept on the device; a
        // second pass only when the first removed most of W (the "twice is
        // enough" test ||W'|| < 0.7 ||W||); norms by Pythagoras from the dots
        const int o2 = IMP_KMAX + 2;
        IMP_TRY(v.dots_dev(Wv, V, j + 1, 1, 0));
        IMP_TRY(v.maxpy_dev(Wv, V, j + 1, h->imp_dres, 1.0));
        IMP_TRY(v.fetch(j + 2, h1.data()));
        double w2 = h1[j + 1], hn2 = w2;
        for (int q = 0; q <= j; ++q) {
          hn2 -= h1[q] * h1[q];
          Hij(q, j) = h1[q];
        }
        if (!(hn2 >= 0.49 * w2)) {
          IMP_TRY(v.dots_dev(Wv, V, j + 1, 1, o2));
          IMP_TRY(v.maxpy_dev(Wv, V, j + 1, h->imp_dres + o2, 1.0));
          std::vector<double> both(2 * o2);
          IMP_TRY(v.fetch(2 * o2, both.data()));
          for (int q = 0; q <= j + 1; ++q) h2[q] = both[o2 + q];
          hn2 = h2[j + 1];
          for (int q = 0; q <= j; ++q) {
            hn2 -= h2[q] * h2[q];
            Hij(q, j) += h2[q];
          }
        }
        const double hn = hn2 > 0 ? std::sqrt(hn2) : 0.0;
        Hij(j + 1, j) = hn;
        if (hn > 0) IMP_TRY(v.lc(Vn, Wv, 1.0 / hn));
        // Givens rotations: previous ones on column j, then a new one
        for (int q = 0; q < j; ++q) {
          const double a = Hij(q, j), b = Hij(q + 1, j);
          Hij(q, j) = cs[q] * a + sn[q] * b;
          Hij(q + 1, j) = -sn[q] * a + cs[q] * b;
        }
        const double r = std::hypot(Hij(j, j), Hij(j + 1, j));
        cs[j] = r > 0 ? Hij(j, j) / r : 1.0;
        sn[j] = r > 0 ? Hij(j + 1, j) / r : 0.0;
        Hij(j, j) = r;
        Hij(j + 1, j) = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        ++st.krylov_iters;
        jend = j + 1;
        if (std::fabs(g[j + 1]) <= o.krylov_rtol * beta || hn == 0) break;
      }
      // y = H^{-1} g (upper triangular), X += sum y_q V_q
      for (int q = jend - 1; q >= 0; --q) {
        double sacc = g[q];
        for (int c2 = q + 1; c2 < jend; ++c2) sacc -= Hij(q, c2) * y[c2];
        y[q] = Hij(q, q) != 0 ? sacc / Hij(q, q) : 0.0;
      }
      IMP_TRY(v.maxpy(X, V, jend, y.data(), -1.0));
    }
    st.max_residual = std::fmax(st.max_residual, rel);
    if (!ok) {
      st.converged = 0;
      if (stats) *stats = st;
      return fail(CDG2_ENOCONV, "implicit stage %d: Newton residual %.3e > %.3e after %d steps", i, rel,
                  o.newton_rtol, o.max_newton);
    }
    // K_i = (X - rhs_i) / (dt a_ii)
    IMP_TRY(v.lc(K[i], X, 1.0 / dg, rhs, -1.0 / dg));
  }
  // U^{n+1} = U^n + dt sum b_i K_i
  IMP_TRY(v.lc(out, Un, 1.0));
  for (int j0 = 0; j0 < tab.s; j0 += 3) {
    const int j1 = j0 + 1 < tab.s ? j0 + 1 : -1, j2 = j0 + 2 < tab.s ? j0 + 2 : -1;
    IMP_TRY(v.lc(out, out, 1.0, K[j0], dt * tab.b[j0], j1 >= 0 ? K[j1] : nullptr, j1 >= 0 ? dt * tab.b[j1] : 0.0,
                 j2 >= 0 ? K[j2] : nullptr, j2 >= 0 ? dt * tab.b[j2] : 0.0));
  }
  IMP_TRY(hipMemcpyAsync(U, out, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  IMP_TRY(hipStreamSynchronize(h->stream));
#undef IMP_TRY
  if (stats) *stats = st;
  return CDG2_OK;
}

int cdg2_max_dt(cdg2_handle* h, const void* U, double cfl, double* dt) {
  if (!h || !U || !dt) return fail(CDG2_EINVAL, "NULL argument");
  if (!(cfl > 0)) return fail(CDG2_EINVAL, "cfl must be > 0");
  HIP_TRY(hipMemsetAsync(h->red, 0, 3 * sizeof(unsigned long long), h->stream));
  HIP_TRY(h->fp32 ? dispatch_cfl<float>(h, U) : dispatch_cfl<double>(h, U));
  unsigned long long r[3];
  HIP_TRY(hipMemcpyAsync(r, h->red, sizeof r, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  double v[3];
  std::memcpy(v, r, sizeof v);
  const double* c = h->coef.c;
  double amax = 0.0;
  for (int s = 0; s < 6; ++s) amax = std::fmax(amax, std::fabs(c[s]));
  double sih2 = 0.0, sih = 0.0;
  for (int a = 0; a < h->dim; ++a) {
    sih2 += h->geo.ih[a] * h->geo.ih[a];
    sih += h->geo.ih[a];
  }
  double rmax = c[K_D1] + c[K_D2] + std::fabs(c[K_GAM]) + c[K_K] + c[K_AL1] * v[1] + c[K_AL2] * v[2];
  double inv = h->rho_hat * amax * sih2 / 2.51 + (2 * h->p + 1) * v[0] * sih + rmax / 2.51;
  *dt = inv > 0 ? cfl / inv : INFINITY;
  return CDG2_OK;
}

int cdg2_sync(cdg2_handle* h) {
  if (!h) return fail(CDG2_EINVAL, "handle is NULL");
  HIP_TRY(hipStreamSynchronize(h->stream));
  int f = 0;
  HIP_TRY(hipMemcpy(&f, h->flags, sizeof f, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(h->flags, 0, sizeof(int)));
  if (f & FLAG_NONFINITE) return fail(CDG2_ENONFINITE, "non-finite value written to a state buffer");
  if (f & FLAG_DOMAIN) return fail(CDG2_EDOMAIN, "c + chi^th <= 0 in a chemotactic sensitivity");
  return CDG2_OK;
}

const char* cdg2_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---- batched instances ------------------------------------------------------------

extern "C" int cdg2_batch_destroy(cdg2_batch* b);

struct cdg2_batch {
  int count = 0;
  std::vector<BatchInst> insts;
  std::vector<size_t> ndof;
  size_t total = 0;
  BatchInst* d_insts = nullptr;
  WorkItem* d_items = nullptr;
  int nitems = 0;
  double* S0 = nullptr;
  double* S1 = nullptr;
  int* flags = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  hipStream_t aux[2] = {nullptr, nullptr};     // order 2: the p = 2 and p = 1 launches of a stage
  hipEvent_t ev_fork = nullptr, ev_join[2] = {nullptr, nullptr};
  int eb = 32, nwg = 0, order = 0;
  int pstart[4] = {0, 0, 0, 0}, pcount[4] = {0, 0, 0, 0};   // order 2: item range per p
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  void* g_U = nullptr;
  int g_nsteps = -1;
  int use_graph = 1;
  std::vector<size_t> packing;   // the library's offsets
};

namespace {

void batch_free_graph(cdg2_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->g_U = nullptr;
  b->g_nsteps = -1;
}

int batch_build_items(cdg2_batch* b) {
  std::vector<WorkItem> items;
  std::vector<double> cost;
  for (int i = 0; i < b->count; ++i) {
    const int E = b->insts[i].prm.g.E;
    const int q = b->insts[i].p + 1;
    for (int e0 = 0; e0 < E; e0 += b->eb) {
      items.push_back({i, e0});
      cost.push_back((double)q * q * q);
    }
  }
  if (b->order == 0 || b->order == 2) {
    std::vector<int> idx(items.size());
    for (size_t k = 0; k < idx.size(); ++k) idx[k] = (int)k;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<WorkItem> sorted(items.size());
    for (size_t k = 0; k < idx.size(); ++k) sorted[k] = items[idx[k]];
    items.swap(sorted);
  }
  for (int p = 0; p < 4; ++p) b->pstart[p] = b->pcount[p] = 0;
  if (b->order == 2) {
    // cost-sorted is order-sorted (cost = (p+1)^3): record each order's range
    for (size_t k = 0; k < items.size(); ++k) {
      const int p = b->insts[items[k].inst].p;
      if (b->pcount[p] == 0) b->pstart[p] = (int)k;
      ++b->pcount[p];
    }
  }
  if (b->d_items) (void)hipFree(b->d_items);
  b->d_items = nullptr;
  if (hipMalloc((void**)&b->d_items, items.size() * sizeof(WorkItem)) != hipSuccess)
    return fail(CDG2_ENOMEM, "hipMalloc of the work list failed");
  if (hipMemcpy(b->d_items, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice) != hipSuccess)
    return fail(CDG2_EHIP, "work list upload failed");
  b->nitems = (int)items.size();
  batch_free_graph(b);
  return CDG2_OK;
}

template <int EB>
hipError_t batch_launch_eb(cdg2_batch* b, hipStream_t st, double* U, int stage) {
  int grid = b->nwg > 0 ? std::min(b->nwg, b->nitems) : b->nitems;
  hipLaunchKernelGGL((batch_stage_kernel<double, EB>), dim3(grid), dim3(6 * EB), 0, st, b->d_insts, b->d_items,
                     b->nitems, U, b->S0, b->S1, stage, b->flags);
  return hipGetLastError();
}

template <int EB, int P>
hipError_t batch_launch_p(cdg2_batch* b, hipStream_t st, double* U, int stage) {
  const int cnt = b->pcount[P];
  if (cnt == 0) return hipSuccess;
  int grid = b->nwg > 0 ? std::min(b->nwg, cnt) : cnt;
  hipLaunchKernelGGL((batch_stage_kernel_p<double, EB, P>), dim3(grid), dim3(6 * EB), 0, st, b->d_insts,
                     b->d_items + b->pstart[P], cnt, U, b->S0, b->S1, stage, b->flags);
  return hipGetLastError();
}

template <int EB>
hipError_t batch_launch_split(cdg2_batch* b, hipStream_t st, double* U, int stage) {
  // The three orders touch disjoint instances, so their launches run side by side
  // on forked streams and join back into st before the next stage.
  hipError_t e = hipEventRecord(b->ev_fork, st);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->aux[k], b->ev_fork, 0);
  if (e == hipSuccess) e = batch_launch_p<EB, 3>(b, st, U, stage);
  if (e == hipSuccess) e = batch_launch_p<EB, 2>(b, b->aux[0], U, stage);
  if (e == hipSuccess) e = batch_launch_p<EB, 1>(b, b->aux[1], U, stage);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventRecord(b->ev_join[k], b->aux[k]);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipStreamWaitEvent(st, b->ev_join[k], 0);
  return e;
}

hipError_t batch_launch(cdg2_batch* b, hipStream_t st, double* U, int stage) {
  if (b->order == 2) {
    switch (b->eb) {
      case 16: return batch_launch_split<16>(b, st, U, stage);
      case 64: return batch_launch_split<64>(b, st, U, stage);
      default: return batch_launch_split<32>(b, st, U, stage);
    }
  }
  switch (b->eb) {
    case 16: return batch_launch_eb<16>(b, st, U, stage);
    case 64: return batch_launch_eb<64>(b, st, U, stage);
    default: return batch_launch_eb<32>(b, st, U, stage);
  }
}

}  // namespace

extern "C" {

int cdg2_batch_create(const cdg2_config* cfgs, int count, int autotune, cdg2_batch** out) {
  if (!out || !cfgs || count <= 0) return fail(CDG2_EINVAL, "bad arguments");
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    int rc = validate(&cfgs[i]);
    if (rc) return rc;
    if (cfgs[i].dim != 2 || cfgs[i].order > 3 || cfgs[i].precision != CDG2_FP64)
      return fail(CDG2_EINVAL, "batched instances must be 2D, FP64, order 1..3 (instance %d)", i);
  }
  cdg2_batch* b = new (std::nothrow) cdg2_batch();
  if (!b) return fail(CDG2_ENOMEM, "host allocation failed");
  b->count = count;
  b->insts.resize(count);
  b->ndof.resize(count);
  size_t off = 0;
  for (int i = 0; i < count; ++i) {
    BatchInst& in = b->insts[i];
    std::memset(&in, 0, sizeof(in));
    build_tables(cfgs[i].order, &in.prm.tb);
    build_geo(cfgs[i], &in.prm.g);
    coef_from(cfgs[i].coeffs, &in.prm.cf);
    in.p = cfgs[i].order;
    in.off = off;
    b->packing.push_back(off);
    const size_t nd = 6 * (size_t)in.prm.g.E * (size_t)((in.p + 1) * (in.p + 1));
    b->ndof[i] = nd;
    off += nd;
  }
  b->total = off;
  if (hipMalloc((void**)&b->d_insts, count * sizeof(BatchInst)) != hipSuccess ||
      hipMalloc((void**)&b->S0, off * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&b->S1, off * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&b->flags, 64) != hipSuccess) {
    cdg2_batch_destroy(b);
    return fail(CDG2_ENOMEM, "hipMalloc for the batch failed");
  }
  if (hipMemset(b->flags, 0, 64) != hipSuccess ||
      hipMemcpy(b->d_insts, b->insts.data(), count * sizeof(BatchInst), hipMemcpyHostToDevice) != hipSuccess ||
      hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&b->aux[0], hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&b->aux[1], hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_join[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_join[1], hipEventDisableTiming) != hipSuccess) {
    cdg2_batch_destroy(b);
    return fail(CDG2_EHIP, "batch initialisation failed");
  }
  int rc = batch_build_items(b);
  if (!rc && autotune) rc = cdg2_batch_autotune(b, nullptr);
  if (rc) {
    cdg2_batch_destroy(b);
    return rc;
  }
  *out = b;
  return CDG2_OK;
}

int cdg2_batch_autotune(cdg2_batch* b, double* best) {
  if (!b) return fail(CDG2_EINVAL, "batch is NULL");
  int dev = 0, ncu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  double* W = nullptr;
  if (hipMalloc((void**)&W, b->total * sizeof(double)) != hipSuccess)
    return fail(CDG2_ENOMEM, "hipMalloc of the autotuning state failed");
  std::vector<BatchInst> saved = b->insts;
  for (auto& in : b->insts) {
    in.dt = 0.0;
    in.off = b->packing[&in - b->insts.data()];
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMemsetAsync(W, 0, b->total * sizeof(double), b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_insts, b->insts.data(), b->count * sizeof(BatchInst), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const int ebs[3] = {16, 32, 64}, wpc[4] = {0, 1, 2, 4};
  double tbest = 1e300;
  int bb[3] = {32, 0, 0};
  for (int ie = 0; ie < 3 && e == hipSuccess; ++ie)
    for (int iw = 0; iw < 4 && e == hipSuccess; ++iw)
      for (int order = 0; order < 3 && e == hipSuccess; ++order) {
        b->eb = ebs[ie];
        b->nwg = wpc[iw] * ncu;
        b->order = order;
        int rc = batch_build_items(b);
        if (rc) {
          e = hipErrorUnknown;
          break;
        }
        for (int st = 1; st <= 3 && e == hipSuccess; ++st) e = batch_launch(b, b->stream, W, st);   // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep)
          for (int st = 1; st <= 3 && e == hipSuccess; ++st) e = batch_launch(b, b->stream, W, st);
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms / 3.0 < tbest) {
          tbest = ms / 3.0;
          bb[0] = b->eb;
          bb[1] = b->nwg;
          bb[2] = b->order;
        }
      }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(b->stream);
  (void)hipFree(W);
  // restore the caller's time steps and placement, clear what the zero state raised
  b->insts = saved;
  hipError_t e2 = hipMemcpy(b->d_insts, b->insts.data(), b->count * sizeof(BatchInst), hipMemcpyHostToDevice);
  if (e2 == hipSuccess) e2 = hipMemset(b->flags, 0, sizeof(int));
  if (e != hipSuccess || e2 != hipSuccess)
    return fail(CDG2_EHIP, "autotuning failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  b->eb = bb[0];
  b->nwg = bb[1];
  b->order = bb[2];
  int rc = batch_build_items(b);
  if (rc) return rc;
  if (best) {
    best[0] = bb[0];
    best[1] = bb[1];
    best[2] = bb[2];
    best[3] = tbest;
  }
  return CDG2_OK;
}

int cdg2_batch_set_graph(cdg2_batch* b, int on) {
  if (!b) return fail(CDG2_EINVAL, "batch is NULL");
  b->use_graph = on != 0;
  return CDG2_OK;
}

int cdg2_batch_destroy(cdg2_batch* b) {
  if (!b) return CDG2_OK;
  batch_free_graph(b);
  if (b->d_insts) (void)hipFree(b->d_insts);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->S0) (void)hipFree(b->S0);
  if (b->S1) (void)hipFree(b->S1);
  if (b->flags) (void)hipFree(b->flags);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (int k = 0; k < 2; ++k) {
    if (b->aux[k]) (void)hipStreamDestroy(b->aux[k]);
    if (b->ev_join[k]) (void)hipEventDestroy(b->ev_join[k]);
  }
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  delete b;
  return CDG2_OK;
}

int cdg2_batch_set_stream(cdg2_batch* b, void* s) {
  if (!b) return fail(CDG2_EINVAL, "batch is NULL");
  b->stream = (hipStream_t)s;
  return CDG2_OK;
}

size_t cdg2_batch_num_dofs(const cdg2_batch* b) { return b ? b->total : 0; }

size_t cdg2_batch_offset(const cdg2_batch* b, int i) {
  if (!b || i < 0 || i >= b->count) return (size_t)-1;
  return b->insts[i].off;
}

int cdg2_batch_set_schedule(cdg2_batch* b, int eb, int nwg, int order) {
  if (!b) return fail(CDG2_EINVAL, "batch is NULL");
  if (eb != 16 && eb != 32 && eb != 64) return fail(CDG2_EINVAL, "eb must be 16, 32 or 64");
  if (nwg < 0 || order < 0 || order > 2) return fail(CDG2_EINVAL, "bad schedule");
  b->eb = eb;
  b->nwg = nwg;
  b->order = order;
  return batch_build_items(b);
}

int cdg2_batch_rk(cdg2_batch* b, void* U_packed, const size_t* offsets, const double* dts, int nsteps) {
  if (!b || !U_packed || !dts) return fail(CDG2_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(CDG2_EINVAL, "nsteps < 0");
  if (overlap(U_packed, b->S0, b->total * 8) || overlap(U_packed, b->S1, b->total * 8))
    return fail(CDG2_EINVAL, "U_packed overlaps a stage buffer");
  const size_t* off = offsets ? offsets : b->packing.data();
  if (offsets) {
    // any non-overlapping placement inside the packed size (the stage buffers
    // use the same offsets)
    std::vector<int> idx(b->count);
    for (int i = 0; i < b->count; ++i) {
      idx[i] = i;
      if (off[i] > b->total || b->ndof[i] > b->total - off[i])
        return fail(CDG2_EINVAL, "offset of instance %d leaves the packed size", i);
    }
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return off[x] < off[y]; });
    for (int k = 1; k < b->count; ++k)
      if (off[idx[k - 1]] + b->ndof[idx[k - 1]] > off[idx[k]])
        return fail(CDG2_EINVAL, "instances %d and %d overlap", idx[k - 1], idx[k]);
  }
  bool changed = false;
  for (int i = 0; i < b->count; ++i) {
    if (!std::isfinite(dts[i])) return fail(CDG2_EINVAL, "dt of instance %d is not finite", i);
    if (b->insts[i].dt != dts[i] || b->insts[i].off != off[i]) changed = true;
    b->insts[i].dt = dts[i];
    b->insts[i].off = off[i];
  }
  if (changed)
    HIP_TRY(hipMemcpyAsync(b->d_insts, b->insts.data(), b->count * sizeof(BatchInst), hipMemcpyHostToDevice,
                           b->stream));
  double* U = (double*)U_packed;
  if (!b->use_graph || nsteps == 0) {
    for (int n = 0; n < nsteps; ++n)
      for (int st = 1; st <= 3; ++st) HIP_TRY(batch_launch(b, b->stream, U, st));
    return CDG2_OK;
  }
  if (!b->gexec || b->g_U != U_packed || b->g_nsteps != nsteps) {
    batch_free_graph(b);
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int n = 0; n < nsteps && e == hipSuccess; ++n)
      for (int st = 1; st <= 3 && e == hipSuccess; ++st) e = batch_launch(b, b->cap, U, st);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(CDG2_EHIP, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
    b->g_U = U_packed;
    b->g_nsteps = nsteps;
  }
  HIP_TRY(hipGraphLaunch(b->gexec, b->stream));
  return CDG2_OK;
}

int cdg2_batch_sync(cdg2_batch* b) {
  if (!b) return fail(CDG2_EINVAL, "batch is NULL");
  HIP_TRY(hipStreamSynchronize(b->stream));
  int f = 0;
  HIP_TRY(hipMemcpy(&f, b->flags, sizeof f, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(b->flags, 0, sizeof(int)));
  if (f & FLAG_NONFINITE) return fail(CDG2_ENONFINITE, "non-finite value written to a state buffer");
  if (f & FLAG_DOMAIN) return fail(CDG2_EDOMAIN, "c + chi^th <= 0 in a chemotactic sensitivity");
  return CDG2_OK;
}

}  // extern "C"

// ---- unstructured triangle meshes (P_k) -------------------------------------------

struct cdg2_tri {
  int k = 1, E = 0, nb = 3;
  size_t ndof = 0;
  TriParams hp{};
  TriParams* dprm = nullptr;
  double* geo = nullptr;   // jit, area, len, nrm, xv (one allocation)
  int* topo = nullptr;     // nbr, nbe, minus
  double* stage[2] = {nullptr, nullptr};
  int* flags = nullptr;
  hipStream_t stream = nullptr;
};

namespace {

// Orthonormal basis of P_k on the reference triangle for the mean, by modified
// Gram-Schmidt of the monomials xi^a eta^b (total degree, then power of eta;
// taken about the centroid),
// with a collapsed Gauss rule exact for the products; then its values and
// gradients at the volume and edge points of the operator's rules.
void build_tri_tables(int k, TriTables* t) {
  std::memset(t, 0, sizeof(TriTables));
  int pw[TRI_MAXB][2], nb = 0;
  for (int d = 0; d <= k; ++d)
    for (int b = 0; b <= d; ++b) {
      pw[nb][0] = d - b;
      pw[nb][1] = b;
      ++nb;
    }
  // monomials about the centroid (1/3, 1/3): every prefix of the order spans the
  // same space as the plain monomials (the same Gram-Schmidt basis), with far less
  // cancellation when the basis is evaluated (P3 stays orthonormal to ~1e-14)
  auto mono = [&](double x0, double y0, double* v, double* gx, double* gy) {
    const double x = x0 - 1.0 / 3.0, y = y0 - 1.0 / 3.0;
    for (int m = 0; m < nb; ++m) {
      const int a = pw[m][0], b = pw[m][1];
      v[m] = std::pow(x, a) * std::pow(y, b);
      gx[m] = a > 0 ? a * std::pow(x, a - 1) * std::pow(y, b) : 0.0;
      gy[m] = b > 0 ? b * std::pow(x, a) * std::pow(y, b - 1) : 0.0;
    }
  };
  auto duffy = [](int q, std::vector<double>& px, std::vector<double>& py, std::vector<double>& pw2) {
    double x[CDG2_MAXQ + 4], w[CDG2_MAXQ + 4];
    gauss_rule01(q, x, w);
    px.clear(); py.clear(); pw2.clear();
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) {
        px.push_back(x[i]);
        py.push_back(x[j] * (1.0 - x[i]));
        pw2.push_back(2.0 * w[i] * w[j] * (1.0 - x[i]));   // for the mean (sum 1)
      }
  };
  // Gram matrix of the monomials
  std::vector<double> px, py, pwt;
  duffy(k + 3, px, py, pwt);
  double G[TRI_MAXB][TRI_MAXB] = {};
  for (size_t n = 0; n < px.size(); ++n) {
    double v[TRI_MAXB], gx[TRI_MAXB], gy[TRI_MAXB];
    mono(px[n], py[n], v, gx, gy);
    for (int a = 0; a < nb; ++a)
      for (int b = 0; b < nb; ++b) G[a][b] += pwt[n] * v[a] * v[b];
  }
  auto ip = [&](const double* x, const double* y) {
    double r = 0.0;
    for (int a = 0; a < nb; ++a)
      for (int b = 0; b < nb; ++b) r += x[a] * G[a][b] * y[b];
    return r;
  };
  double C[TRI_MAXB][TRI_MAXB] = {};
  for (int j = 0; j < nb; ++j) {
    double c[TRI_MAXB] = {};
    c[j] = 1.0;
    for (int i = 0; i < j; ++i) {
      const double r = ip(C[i], c);
      for (int m = 0; m < nb; ++m) c[m] -= r * C[i][m];
    }
    const double nrm = std::sqrt(ip(c, c));
    for (int m = 0; m < nb; ++m) C[j][m] = c[m] / nrm;
  }
  auto basis = [&](double x, double y, double* v, double* g0, double* g1) {
    double mv[TRI_MAXB], mx[TRI_MAXB], my[TRI_MAXB];
    mono(x, y, mv, mx, my);
    for (int j = 0; j < nb; ++j) {
      double a = 0.0, b = 0.0, c2 = 0.0;
      for (int m = 0; m < nb; ++m) {
        a += C[j][m] * mv[m];
        b += C[j][m] * mx[m];
        c2 += C[j][m] * my[m];
      }
      v[j] = a;
      g0[j] = b;
      g1[j] = c2;
    }
  };
  duffy(k + 1, px, py, pwt);
  for (size_t q = 0; q < px.size(); ++q) {
    double v[TRI_MAXB], g0[TRI_MAXB], g1[TRI_MAXB];
    basis(px[q], py[q], v, g0, g1);
    for (int j = 0; j < nb; ++j) {
      t->Bv[q][j] = v[j];
      t->Bg[q][j][0] = g0[j];
      t->Bg[q][j][1] = g1[j];
    }
    t->wv[q] = pwt[q];
  }
  double es[CDG2_MAXQ], ew[CDG2_MAXQ];
  gauss_rule01(k + 1, es, ew);
  const double VX[3] = {0.0, 1.0, 0.0}, VY[3] = {0.0, 0.0, 1.0};
  for (int p = 0; p <= k; ++p) {
    t->s[p] = es[p];
    t->ws[p] = ew[p];
  }
  for (int e = 0; e < 3; ++e)
    for (int p = 0; p <= k; ++p) {
      const double x = VX[e] + es[p] * (VX[(e + 1) % 3] - VX[e]);
      const double y = VY[e] + es[p] * (VY[(e + 1) % 3] - VY[e]);
      double v[TRI_MAXB], g0[TRI_MAXB], g1[TRI_MAXB];
      basis(x, y, v, g0, g1);
      for (int j = 0; j < nb; ++j) {
        t->Be[e][p][j] = v[j];
        t->Bge[e][p][j][0] = g0[j];
        t->Bge[e][p][j][1] = g1[j];
      }
    }
}

void tri_free(cdg2_tri* t) {
  if (t->dprm) (void)hipFree(t->dprm);
  if (t->geo) (void)hipFree(t->geo);
  if (t->topo) (void)hipFree(t->topo);
  for (int i = 0; i < 2; ++i)
    if (t->stage[i]) (void)hipFree(t->stage[i]);
  if (t->flags) (void)hipFree(t->flags);
}

hipError_t tri_launch(cdg2_tri* t, const double* U, const double* U0, double* out, double dt, double ca, double cb,
                      int stage) {
  auto nblk = [&](int eb) { return (t->E + eb - 1) / eb; };
  if (t->k == 1)
    hipLaunchKernelGGL((tri_kernel<1>), dim3(nblk(tri_eb<1>())), dim3(6 * tri_eb<1>()), 0, t->stream, t->dprm, U, U0,
                       out, dt, ca, cb, stage, t->flags);
  else if (t->k == 2)
    hipLaunchKernelGGL((tri_kernel<2>), dim3(nblk(tri_eb<2>())), dim3(6 * tri_eb<2>()), 0, t->stream, t->dprm, U, U0,
                       out, dt, ca, cb, stage, t->flags);
  else
    hipLaunchKernelGGL((tri_kernel<3>), dim3(nblk(tri_eb<3>())), dim3(6 * tri_eb<3>()), 0, t->stream, t->dprm, U, U0,
                       out, dt, ca, cb, stage, t->flags);
  return hipGetLastError();
}

}  // namespace

extern "C" {

int cdg2_tri_create(int order, int n_elements, const double* xy, const int* nbr, const int* nbe,
                    const cdg2_coeffs* coeffs, double gamma1_in_lo, double gamma1_in_hi, cdg2_tri** out) {
  if (!out || !xy || !nbr || !nbe || !coeffs) return fail(CDG2_EINVAL, "NULL argument");
  *out = nullptr;
  if (order < 1 || order > 3) return fail(CDG2_EINVAL, "triangle order must be 1, 2 or 3");
  if (n_elements < 1) return fail(CDG2_EINVAL, "n_elements < 1");
  const int E = n_elements;
  // topology checks: codes, ranges, reciprocity
  for (int e = 0; e < E; ++e)
    for (int j = 0; j < 3; ++j) {
      const int f = nbr[3 * e + j];
      if (f >= 0) {
        const int jj = nbe[3 * e + j];
        if (f >= E || jj < 0 || jj > 2) return fail(CDG2_EINVAL, "neighbour of element %d edge %d out of range", e, j);
        if (nbr[3 * f + jj] != e || nbe[3 * f + jj] != j)
          return fail(CDG2_EINVAL, "neighbour tables not reciprocal at element %d edge %d", e, j);
      } else if (f != -1 && f != -2) {
        return fail(CDG2_EINVAL, "boundary code %d at element %d edge %d (allowed: -1, -2)", f, e, j);
      }
    }
  auto* t = new (std::nothrow) cdg2_tri;
  if (!t) return fail(CDG2_ENOMEM, "out of host memory");
  t->k = order;
  t->E = E;
  t->nb = (order + 1) * (order + 2) / 2;
  t->ndof = (size_t)6 * E * t->nb;
  build_tri_tables(order, &t->hp.tb);
  std::vector<double> geo((size_t)E * (4 + 1 + 3 + 6 + 3));
  double* jit = geo.data();
  double* area = jit + 4 * (size_t)E;
  double* len = area + E;
  double* nrm = len + 3 * (size_t)E;
  double* xv = nrm + 6 * (size_t)E;
  std::vector<int> topo((size_t)E * 9);
  for (int e = 0; e < E; ++e) {
    const double* v = xy + 6 * (size_t)e;
    const double j00 = v[2] - v[0], j10 = v[3] - v[1], j01 = v[4] - v[0], j11 = v[5] - v[1];
    const double det = j00 * j11 - j01 * j10;
    if (!(det > 0.0)) {
      delete t;
      return fail(CDG2_EINVAL, "element %d is not counter-clockwise (or degenerate)", e);
    }
    jit[4 * e + 0] = j11 / det;
    jit[4 * e + 1] = -j10 / det;
    jit[4 * e + 2] = -j01 / det;
    jit[4 * e + 3] = j00 / det;
    area[e] = 0.5 * det;
    for (int j = 0; j < 3; ++j) {
      const int a = j, b = (j + 1) % 3;
      const double tx = v[2 * b] - v[2 * a], ty = v[2 * b + 1] - v[2 * a + 1];
      const double L = std::hypot(tx, ty);
      len[3 * e + j] = L;
      nrm[6 * e + 2 * j] = ty / L;
      nrm[6 * e + 2 * j + 1] = -tx / L;
      xv[3 * e + j] = v[2 * j];
    }
  }
  for (int e = 0; e < E; ++e)
    for (int j = 0; j < 3; ++j) {
      const int f = nbr[3 * e + j];
      topo[3 * e + j] = f;
      topo[3 * (size_t)E + 3 * e + j] = f >= 0 ? nbe[3 * e + j] : 0;
      // K^-: the smaller triangle, ties to the lower element index
      topo[6 * (size_t)E + 3 * e + j] = f >= 0 && (area[e] < area[f] || (area[e] == area[f] && e < f)) ? 1 : 0;
    }
  if (hipMalloc((void**)&t->dprm, sizeof(TriParams)) != hipSuccess ||
      hipMalloc((void**)&t->geo, geo.size() * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&t->topo, topo.size() * sizeof(int)) != hipSuccess ||
      hipMalloc((void**)&t->stage[0], t->ndof * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&t->stage[1], t->ndof * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&t->flags, 64) != hipSuccess) {
    tri_free(t);
    delete t;
    return fail(CDG2_ENOMEM, "hipMalloc for the triangle mesh failed");
  }
  TriGeo& g = t->hp.g;
  g.E = E;
  g.jit = t->geo;
  g.area = t->geo + 4 * (size_t)E;
  g.len = g.area + E;
  g.nrm = g.len + 3 * (size_t)E;
  g.xv = g.nrm + 6 * (size_t)E;
  g.nbr = t->topo;
  g.nbe = t->topo + 3 * (size_t)E;
  g.minus = t->topo + 6 * (size_t)E;
  g.g1in[0] = gamma1_in_lo;
  g.g1in[1] = gamma1_in_hi;
  static_assert(sizeof(cdg2_coeffs) == sizeof(double) * K_NCOEFF, "coefficient order");
  std::memcpy(t->hp.cf.c, coeffs, sizeof(double) * K_NCOEFF);
  if (hipMemcpy(t->geo, geo.data(), geo.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t->topo, topo.data(), topo.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t->dprm, &t->hp, sizeof(TriParams), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(t->flags, 0, 64) != hipSuccess) {
    tri_free(t);
    delete t;
    return fail(CDG2_EHIP, "triangle mesh upload failed");
  }
  *out = t;
  return CDG2_OK;
}

int cdg2_tri_destroy(cdg2_tri* t) {
  if (!t) return CDG2_OK;
  tri_free(t);
  delete t;
  return CDG2_OK;
}

int cdg2_tri_set_stream(cdg2_tri* t, void* stream) {
  if (!t) return fail(CDG2_EINVAL, "handle is NULL");
  t->stream = (hipStream_t)stream;
  return CDG2_OK;
}

size_t cdg2_tri_num_dofs(const cdg2_tri* t) { return t ? t->ndof : 0; }

int cdg2_tri_apply_operator(cdg2_tri* t, const double* U, double* F) {
  if (!t || !U || !F) return fail(CDG2_EINVAL, "NULL argument");
  if (overlap(U, F, t->ndof * sizeof(double))) return fail(CDG2_EINVAL, "U and F overlap");
  HIP_TRY(tri_launch(t, U, nullptr, F, 0.0, 0.0, 1.0, 0));
  return CDG2_OK;
}

int cdg2_tri_rk_step(cdg2_tri* t, double* U, double dt, int nsteps) {
  if (!t || !U) return fail(CDG2_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(CDG2_EINVAL, "nsteps < 0");
  if (!std::isfinite(dt)) return fail(CDG2_EINVAL, "dt is not finite");
  const size_t bytes = t->ndof * sizeof(double);
  if (overlap(U, t->stage[0], bytes) || overlap(U, t->stage[1], bytes))
    return fail(CDG2_EINVAL, "U overlaps a stage buffer");
  for (int n = 0; n < nsteps; ++n) {
    HIP_TRY(tri_launch(t, U, nullptr, t->stage[0], dt, 0.0, 1.0, 1));
    HIP_TRY(tri_launch(t, t->stage[0], U, t->stage[1], dt, 0.75, 0.25, 2));
    HIP_TRY(tri_launch(t, t->stage[1], U, U, dt, 1.0 / 3.0, 2.0 / 3.0, 3));
  }
  return CDG2_OK;
}

int cdg2_tri_sync(cdg2_tri* t) {
  if (!t) return fail(CDG2_EINVAL, "handle is NULL");
  HIP_TRY(hipStreamSynchronize(t->stream));
  int f = 0;
  HIP_TRY(hipMemcpy(&f, t->flags, sizeof f, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(t->flags, 0, sizeof(int)));
  if (f & FLAG_NONFINITE) return fail(CDG2_ENONFINITE, "non-finite value written to a state buffer");
  if (f & FLAG_DOMAIN) return fail(CDG2_EDOMAIN, "c + chi^th <= 0 in a chemotactic sensitivity");
  return CDG2_OK;
}

}  // extern "C"

// ---- unstructured tetrahedral meshes (P_k) ----------------------------------------

#include "tet_api.hpp"
