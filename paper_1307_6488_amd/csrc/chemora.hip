// chemora.hip -- gfx950 kernels and host ABI of the BSSN right-hand side and
// RK4 step (see include/chemora.h for the contract).
//
// Stage kernel: one work-item per interior point.  It evaluates every
// stencil the point needs straight from the stage input (the paper's
// "RHS derivatives" step), the pointwise BSSN algebra ("RHS evaluations"),
// the upwinded advection ("RHS advection") and Kreiss-Oliger dissipation,
// and applies the RK4 stage combination in the same pass, so derivatives
// never travel through HBM (section "Binary Black Hole Simulations", timer
// table; the paper's derivative/RHS split costs bandwidth, section
// "Automated Code Generation with Kranc", "Optimization").
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "chemora.h"
#include "stage_common.hpp"

namespace chemora {

// Ghost shells, one work-group per stored row (j, k) of the full extent.
// STATIC: copy the ghosts of `src` into dst0 and dst1.  PERIODIC: fill the
// ghosts of dst0 with periodic images of its own interior.
template <bool PERIODIC>
__global__ __launch_bounds__(64) void ghost_kernel(const double* __restrict__ src, double* dst0,
                                                   double* dst1, Geo G) {
  const int j = blockIdx.x, k = blockIdx.y;
  const int ex = G.nx + 2 * G.g;
  const bool ghost_row = j < G.g || j >= G.ny + G.g || k < G.g || k >= G.nz + G.g;
  int jj = j, kk = k;
  if (PERIODIC) {
    jj = ((j - G.g) % G.ny + G.ny) % G.ny + G.g;
    kk = ((k - G.g) % G.nz + G.nz) % G.nz + G.g;
  }
  const int64_t row = (int64_t)k * G.sz + (int64_t)j * G.sy;
  const int64_t srow = (int64_t)kk * G.sz + (int64_t)jj * G.sy;
  for (int i = threadIdx.x; i < ex; i += blockDim.x) {
    if (!ghost_row && i >= G.g && i < G.nx + G.g) continue;
    if (PERIODIC) {
      const int ii = ((i - G.g) % G.nx + G.nx) % G.nx + G.g;
      for (int f = 0; f < 24; ++f) dst0[f * G.sf + row + i] = dst0[f * G.sf + srow + ii];
    } else {
      for (int f = 0; f < 24; ++f) {
        const double v = src[f * G.sf + row + i];
        dst0[f * G.sf + row + i] = v;
        dst1[f * G.sf + row + i] = v;
      }
    }
  }
}

__global__ __launch_bounds__(256) void finite_kernel(const double* __restrict__ u, Geo G,
                                                     unsigned long long* count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int k = blockIdx.z;
  if (i >= G.nx) return;
  const int64_t idx = (int64_t)(k + G.g) * G.sz + (int64_t)(j + G.g) * G.sy + (i + G.g);
  unsigned int bad = 0;
  for (int f = 0; f < 24; ++f) bad += isfinite(u[f * G.sf + idx]) ? 0u : 1u;
  if (bad) atomicAdd(count, (unsigned long long)bad);
}

}  // namespace chemora

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

thread_local std::string g_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

int required_ghost(int order, int upwind, int ko) {
  if (order != 4 && order != 8) return -1;
  int g = order / 2;
  if (upwind) g = order / 2 + 1;
  return ko > g ? ko : g;
}

int validate(const chemora_params* P, const chemora_patch* X) {
  if (!P) return fail(CHEMORA_EINVAL, "params is NULL");
  if (!X) return fail(CHEMORA_EINVAL, "patch is NULL");
  if (P->fd_order != 4 && P->fd_order != 8)
    return fail(CHEMORA_EINVAL, "fd_order %d not in {4, 8}", P->fd_order);
  if (P->upwind != 0 && P->upwind != 1) return fail(CHEMORA_EINVAL, "upwind must be 0 or 1");
  if (P->ko_radius != 0 && P->ko_radius != 2 && P->ko_radius != 3 && P->ko_radius != 5)
    return fail(CHEMORA_EUNSUPPORTED, "ko_radius %d not in {0, 2, 3, 5}", P->ko_radius);
  const int need = required_ghost(P->fd_order, P->upwind, P->ko_radius);
  if (P->ghost < need)
    return fail(CHEMORA_EINVAL, "ghost %d < %d required by order %d, upwind %d, ko_radius %d", P->ghost,
                need, P->fd_order, P->upwind, P->ko_radius);
  if (!(P->eps_diss >= 0.0) || !std::isfinite(P->eps_diss))
    return fail(CHEMORA_EINVAL, "eps_diss must be finite and >= 0");
  if (P->lapse < 0 || P->lapse > 2) return fail(CHEMORA_EINVAL, "lapse %d unknown", P->lapse);
  if (P->shift < 0 || P->shift > 1) return fail(CHEMORA_EINVAL, "shift %d unknown", P->shift);
  if (!std::isfinite(P->eta)) return fail(CHEMORA_EINVAL, "eta must be finite");
  if (P->bc != 0 && P->bc != 1) return fail(CHEMORA_EINVAL, "bc %d unknown", P->bc);
  if (P->precision != CHEMORA_PREC_FP64)
    return fail(CHEMORA_EUNSUPPORTED, "precision %d not built", P->precision);
  for (int a = 0; a < 3; ++a) {
    if (X->n[a] < 1) return fail(CHEMORA_EINVAL, "n[%d] = %d < 1", a, X->n[a]);
    if (P->bc == CHEMORA_BC_PERIODIC && X->n[a] < P->ghost)
      return fail(CHEMORA_EINVAL, "periodic boundary needs n[%d] = %d >= ghost %d", a, X->n[a], P->ghost);
  }
  if (X->reserved != 0) return fail(CHEMORA_EINVAL, "patch.reserved must be 0");
  const int64_t g2 = 2 * (int64_t)P->ghost;
  if (X->sy < X->n[0] + g2) return fail(CHEMORA_EINVAL, "sy %lld < nx + 2g", (long long)X->sy);
  if ((X->n[0] & 1) && X->sy < X->n[0] + g2 + 1)
    return fail(CHEMORA_EINVAL, "sy %lld: odd nx needs one element of row padding (sy >= nx + 2g + 1)",
                (long long)X->sy);
  if (X->sz < X->sy * (X->n[1] + g2)) return fail(CHEMORA_EINVAL, "sz %lld < sy*(ny + 2g)", (long long)X->sz);
  if (X->sf < X->sz * (X->n[2] + g2)) return fail(CHEMORA_EINVAL, "sf %lld < sz*(nz + 2g)", (long long)X->sf);
  const int64_t tiles = (int64_t)((X->n[0] + 63) / 64) * ((X->n[1] + 3) / 4) * X->n[2];
  if (X->sz > INT32_MAX || tiles > INT32_MAX || X->n[1] + g2 > 65535 || X->n[2] + g2 > 65535)
    return fail(CHEMORA_EINVAL, "patch too large for the launch geometry");
  if (((uint64_t)CHEMORA_NGF * (uint64_t)X->sf + 8) * 8 > 0xFFFFFFFFull)
    return fail(CHEMORA_EUNSUPPORTED, "patch state of %lld bytes exceeds 4 GiB; split it into patches",
                (long long)((uint64_t)CHEMORA_NGF * X->sf * 8));
  if (P->fd_order == 4 && P->ko_radius > 3)
    return fail(CHEMORA_EUNSUPPORTED, "order 4 supports ko_radius <= 3");
  if (!(X->h > 0.0) || !std::isfinite(X->h)) return fail(CHEMORA_EINVAL, "h must be finite and > 0");
  if (!X->u) return fail(CHEMORA_EINVAL, "patch.u is NULL");
  if (((uintptr_t)X->u) % 8) return fail(CHEMORA_EINVAL, "patch.u not 8-byte aligned");
  return CHEMORA_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
  return pa < pb + nb && pb < pa + na;
}

chemora::Geo make_geo(const chemora_params* P, const chemora_patch* X) {
  chemora::Geo G;
  G.nx = X->n[0]; G.ny = X->n[1]; G.nz = X->n[2]; G.g = P->ghost;
  G.sy = X->sy; G.sz = X->sz; G.sf = X->sf;
  return G;
}

chemora::Scales make_scales(const chemora_params* P, double h) {
  chemora::Scales s;
  const bool o8 = P->fd_order == 8;
  const double D1 = o8 ? 840.0 : 12.0, D2 = o8 ? 5040.0 : 12.0;
  s.d1 = 1.0 / (D1 * h);
  s.d2 = 1.0 / (D2 * h * h);
  s.d11 = s.d1 * s.d1;
  s.up = 1.0 / (D1 * h);
  s.ko_r = P->ko_radius;
  s.ko = P->ko_radius > 0 ? std::ldexp(P->eps_diss / h, -2 * P->ko_radius) : 0.0;
  return s;
}

// single-patch form: one work-group per tile
void dispatch_stage(const chemora_params* P, const chemora::StageArgs& a, hipStream_t s) {
  chemora::BatchTable none;
  std::memset(&none, 0, sizeof none);
  const int tiles = a.tiles_x * a.tiles_y * a.geo.nz;
  if (P->fd_order == 4)
    chemora::launch_stage_o4(P->upwind != 0, P->ko_radius, a, none, tiles, s);
  else
    chemora::launch_stage_o8(P->upwind != 0, P->ko_radius, a, none, tiles, s);
}

// batched form: one work-group per tile of the plan's tile list
void dispatch_batch(const chemora_params* P, const chemora::BatchTable& bt, int grid, hipStream_t s) {
  chemora::StageArgs none;
  std::memset(&none, 0, sizeof none);
  if (P->fd_order == 4)
    chemora::launch_stage_o4(P->upwind != 0, P->ko_radius, none, bt, grid, s);
  else
    chemora::launch_stage_o8(P->upwind != 0, P->ko_radius, none, bt, grid, s);
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CHEMORA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return CHEMORA_OK;
}

chemora::StageArgs base_args(const chemora_params* P, const chemora_patch* X) {
  chemora::StageArgs a;
  std::memset(&a, 0, sizeof a);
  a.geo = make_geo(P, X);
  a.sc = make_scales(P, X->h);
  a.gauge.lapse = P->lapse;
  a.gauge.shift = P->shift;
  a.gauge.eta = P->eta;
  a.tiles_x = (X->n[0] + chemora::TILE_X - 1) / chemora::TILE_X;
  a.tiles_y = (X->n[1] + chemora::TILE_Y - 1) / chemora::TILE_Y;
  return a;
}

void launch_ghosts(bool periodic, const chemora::Geo& G, const double* src, double* d0, double* d1,
                   hipStream_t s) {
  dim3 grid(G.ny + 2 * G.g, G.nz + 2 * G.g, 1);
  if (periodic)
    hipLaunchKernelGGL((chemora::ghost_kernel<true>), grid, dim3(64), 0, s, src, d0, d1, G);
  else
    hipLaunchKernelGGL((chemora::ghost_kernel<false>), grid, dim3(64), 0, s, src, d0, d1, G);
}

}  // namespace

extern "C" {

int chemora_abi_version(void) { return 100; }

const char* chemora_last_error(void) { return g_error.c_str(); }

int chemora_required_ghost(int fd_order, int upwind, int ko_radius) {
  return required_ghost(fd_order, upwind, ko_radius);
}

size_t chemora_rk4_scratch_elems(const chemora_patch* patch) {
  if (!patch || patch->sf <= 0) return 0;
  return (size_t)3 * CHEMORA_NGF * (size_t)patch->sf;
}

int chemora_bssn_rhs(const chemora_params* params, const chemora_patch* patch, double* rhs, void* stream) {
  g_error.clear();
  int rc = validate(params, patch);
  if (rc) return rc;
  if (!rhs) return fail(CHEMORA_EINVAL, "rhs is NULL");
  if (((uintptr_t)rhs) % 8) return fail(CHEMORA_EINVAL, "rhs not 8-byte aligned");
  const size_t bytes = (size_t)CHEMORA_NGF * patch->sf * sizeof(double);
  if (overlap(rhs, bytes, patch->u, bytes)) return fail(CHEMORA_EINVAL, "rhs overlaps patch.u");
  chemora::StageArgs a = base_args(params, patch);
  a.in = a.un = a.yin = patch->u;
  a.out = rhs;
  a.mode = chemora::MODE_RHS;
  dispatch_stage(params, a, (hipStream_t)stream);
  return check_launch("bssn_rhs");
}

}  // extern "C"

namespace {

int rk4_checks(const chemora_params* params, const chemora_patch* patch, double dt, double* scratch) {
  int rc = validate(params, patch);
  if (rc) return rc;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CHEMORA_EINVAL, "dt must be finite and > 0");
  if (!scratch) return fail(CHEMORA_EINVAL, "scratch is NULL");
  if (((uintptr_t)scratch) % 8) return fail(CHEMORA_EINVAL, "scratch not 8-byte aligned");
  const size_t state = (size_t)CHEMORA_NGF * patch->sf;
  if (overlap(scratch, 3 * state * sizeof(double), patch->u, state * sizeof(double)))
    return fail(CHEMORA_EINVAL, "scratch overlaps patch.u");
  return CHEMORA_OK;
}

// Arguments of RK4 stage `stage` (1-4).  Buffers: u = u_n (overwritten by
// stage 4), SA/SB stage inputs, Y accumulator.
//   1: Y = u + dt/6 k1(u),  SA = u + dt/2 k1      3: Y += dt/3 k3(SB), SA = u + dt k3
//   2: Y += dt/3 k2(SA),    SB = u + dt/2 k2      4: u = Y + dt/6 k4(SA)
// Returns the buffer the stage writes.
double* stage_args(chemora::StageArgs& a, int stage, double dt, double* u, double* SA, double* SB, double* Y) {
  a.y = Y;
  switch (stage) {
    case 1:
      a.in = u; a.un = u; a.yin = u; a.out = SA; a.cy = dt / 6.0; a.cs = 0.5 * dt;
      a.mode = chemora::MODE_STAGE1;
      return SA;
    case 2:
      a.in = SA; a.un = u; a.yin = Y; a.out = SB; a.cy = dt / 3.0; a.cs = 0.5 * dt;
      a.mode = chemora::MODE_STAGE23;
      return SB;
    case 3:
      a.in = SB; a.un = u; a.yin = Y; a.out = SA; a.cy = dt / 3.0; a.cs = dt;
      a.mode = chemora::MODE_STAGE23;
      return SA;
    default:
      a.in = SA; a.un = Y; a.yin = Y; a.out = u; a.cy = dt / 6.0; a.cs = 0.0;
      a.mode = chemora::MODE_STAGE4;
      return u;
  }
}

int rk4_stage(const chemora_params* params, const chemora_patch* patch, int stage, double dt, double* scratch,
              hipStream_t s) {
  if (stage < 1 || stage > 4) return fail(CHEMORA_EINVAL, "stage %d not in 1..4", stage);
  const size_t state = (size_t)CHEMORA_NGF * patch->sf;
  double* u = patch->u;
  double* SA = scratch;
  double* SB = scratch + state;
  double* Y = scratch + 2 * state;
  const bool periodic = params->bc == CHEMORA_BC_PERIODIC;
  chemora::StageArgs a = base_args(params, patch);
  if (stage == 1 && !periodic) launch_ghosts(false, a.geo, u, SA, SB, s);
  double* written = stage_args(a, stage, dt, u, SA, SB, Y);
  dispatch_stage(params, a, s);
  if (periodic) launch_ghosts(true, a.geo, nullptr, written, nullptr, s);
  return check_launch("rk4 stage");
}

}  // namespace

extern "C" {

int chemora_rk4_step(const chemora_params* params, const chemora_patch* patch, double dt, double* scratch,
                     void* stream) {
  g_error.clear();
  int rc = rk4_checks(params, patch, dt, scratch);
  if (rc) return rc;
  for (int st = 1; st <= 4; ++st)
    if ((rc = rk4_stage(params, patch, st, dt, scratch, (hipStream_t)stream))) return rc;
  return CHEMORA_OK;
}

int chemora_rk4_stage(const chemora_params* params, const chemora_patch* patch, int stage, double dt,
                      double* scratch, void* stream) {
  g_error.clear();
  int rc = rk4_checks(params, patch, dt, scratch);
  if (rc) return rc;
  if (stage < 1 || stage > 4) return fail(CHEMORA_EINVAL, "stage %d not in 1..4", stage);
  return rk4_stage(params, patch, stage, dt, scratch, (hipStream_t)stream);
}

int chemora_check_finite(const chemora_params* params, const chemora_patch* patch, int64_t* bad_count,
                         void* stream) {
  g_error.clear();
  int rc = validate(params, patch);
  if (rc) return rc;
  if (!bad_count) return fail(CHEMORA_EINVAL, "bad_count is NULL");
  const chemora::Geo G = make_geo(params, patch);
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* d = nullptr;
  if (hipMallocAsync((void**)&d, sizeof *d, s) != hipSuccess) return fail(CHEMORA_EDEVICE, "hipMallocAsync failed");
  hipError_t e = hipMemsetAsync(d, 0, sizeof *d, s);
  dim3 grid((G.nx + 255) / 256, G.ny, G.nz);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(chemora::finite_kernel, grid, dim3(256), 0, s, patch->u, G, d);
    e = hipGetLastError();
  }
  unsigned long long h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof h, hipMemcpyDeviceToHost, s);
  const hipError_t ef = hipFreeAsync(d, s);
  if (e == hipSuccess) e = ef;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(CHEMORA_EDEVICE, "check_finite: %s", hipGetErrorString(e));
  *bad_count = (int64_t)h;
  return h ? fail(CHEMORA_ENOTFINITE, "%llu non-finite interior values", h) : CHEMORA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// plans (batched form)
// ---------------------------------------------------------------------------
struct chemora_plan {
  chemora_params params;
  int npatch = 0;
  int64_t points = 0;
  int ntiles = 0;
  int grid = 0;                                   // work-groups per launch (one per tile)
  chemora::StageArgs* d_args = nullptr;           // 4 stage tables of npatch entries
  int* d_tile_start = nullptr;
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void plan_free(chemora_plan* pl) {
  if (!pl) return;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->capture) {
    (void)hipStreamSynchronize(pl->capture);
    (void)hipStreamDestroy(pl->capture);
  }
  if (pl->d_args) (void)hipFree(pl->d_args);
  if (pl->d_tile_start) (void)hipFree(pl->d_tile_start);
  delete pl;
}

}  // namespace

extern "C" {

int chemora_plan_create(const chemora_params* params, const chemora_patch* patches, double* const* scratch,
                        int32_t npatch, double courant, const char* tune_cache_path, void* stream,
                        chemora_plan** out) {
  (void)tune_cache_path;
  g_error.clear();
  if (!out) return fail(CHEMORA_EINVAL, "out is NULL");
  *out = nullptr;
  if (!patches || !scratch) return fail(CHEMORA_EINVAL, "patches or scratch is NULL");
  if (npatch < 1) return fail(CHEMORA_EINVAL, "npatch %d < 1", npatch);
  if (!(courant > 0.0) || !std::isfinite(courant)) return fail(CHEMORA_EINVAL, "courant must be finite and > 0");
  int rc;
  int64_t tiles = 0, points = 0;
  for (int p = 0; p < npatch; ++p) {
    if ((rc = rk4_checks(params, &patches[p], courant * patches[p].h, scratch[p]))) {
      const std::string m = g_error;
      return fail(rc, "patch %d: %s", p, m.c_str());
    }
    const chemora::StageArgs a = base_args(params, &patches[p]);
    tiles += (int64_t)a.tiles_x * a.tiles_y * a.geo.nz;
    points += (int64_t)patches[p].n[0] * patches[p].n[1] * patches[p].n[2];
  }
  if (tiles > INT32_MAX) return fail(CHEMORA_EINVAL, "too many tiles in the plan");

  chemora_plan* pl = new (std::nothrow) chemora_plan;
  if (!pl) return fail(CHEMORA_ENOMEM, "host allocation failed");
  pl->params = *params;
  pl->npatch = npatch;
  pl->points = points;
  pl->ntiles = (int)tiles;

  // per-stage argument tables and tile offsets (host side first)
  std::vector<chemora::StageArgs> args(4 * (size_t)npatch);
  std::vector<int> start(npatch + 1, 0);
  for (int p = 0; p < npatch; ++p) {
    const chemora_patch* X = &patches[p];
    const double dt = courant * X->h;
    const size_t state = (size_t)CHEMORA_NGF * X->sf;
    double* u = X->u;
    double* SA = scratch[p];
    double* SB = scratch[p] + state;
    double* Y = scratch[p] + 2 * state;
    chemora::StageArgs a = base_args(params, X);
    start[p + 1] = start[p] + a.tiles_x * a.tiles_y * a.geo.nz;
    for (int st = 0; st < 4; ++st) {
      chemora::StageArgs sa = a;
      stage_args(sa, st + 1, dt, u, SA, SB, Y);
      args[st * npatch + p] = sa;
    }
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMalloc((void**)&pl->d_args, args.size() * sizeof(chemora::StageArgs));
  if (e == hipSuccess) e = hipMalloc((void**)&pl->d_tile_start, start.size() * sizeof(int));
  if (e != hipSuccess) {
    plan_free(pl);
    (void)hipGetLastError();
    return fail(CHEMORA_ENOMEM, "device allocation of plan tables failed");
  }
  e = hipMemcpyAsync(pl->d_args, args.data(), args.size() * sizeof(chemora::StageArgs), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(pl->d_tile_start, start.data(), start.size() * sizeof(int), hipMemcpyHostToDevice, s);
  // static ghosts of the stage buffers, once
  if (e == hipSuccess && params->bc == CHEMORA_BC_STATIC) {
    for (int p = 0; p < npatch && e == hipSuccess; ++p) {
      const size_t state = (size_t)CHEMORA_NGF * patches[p].sf;
      launch_ghosts(false, make_geo(params, &patches[p]), patches[p].u, scratch[p], scratch[p] + state, s);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // tables and ghosts in place before capture
  if (e != hipSuccess) {
    plan_free(pl);
    return fail(CHEMORA_EDEVICE, "plan setup: %s", hipGetErrorString(e));
  }

  // one work-group per tile of the concatenated tile list
  pl->grid = pl->ntiles;

  // capture one RK4 step
  e = hipStreamCreateWithFlags(&pl->capture, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(pl->capture, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    plan_free(pl);
    return fail(CHEMORA_EDEVICE, "graph capture start: %s", hipGetErrorString(e));
  }
  const bool periodic = params->bc == CHEMORA_BC_PERIODIC;
  for (int st = 0; st < 4; ++st) {
    chemora::BatchTable bt;
    bt.args = pl->d_args + st * npatch;
    bt.tile_start = pl->d_tile_start;
    bt.npatch = npatch;
    bt.ntiles = pl->ntiles;
    dispatch_batch(params, bt, pl->grid, pl->capture);
    if (periodic)
      for (int p = 0; p < npatch; ++p) {
        const double* wr = args[st * npatch + p].out;
        launch_ghosts(true, make_geo(params, &patches[p]), nullptr, const_cast<double*>(wr), nullptr, pl->capture);
      }
  }
  hipError_t le = hipGetLastError();
  e = hipStreamEndCapture(pl->capture, &pl->graph);
  if (le != hipSuccess || e != hipSuccess) {
    plan_free(pl);
    return fail(CHEMORA_EDEVICE, "graph capture: %s", hipGetErrorString(le != hipSuccess ? le : e));
  }
  e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    plan_free(pl);
    return fail(CHEMORA_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
  }
  *out = pl;
  return CHEMORA_OK;
}

int chemora_batch_step(chemora_plan* plan, int32_t nsteps, void* stream) {
  g_error.clear();
  if (!plan) return fail(CHEMORA_EINVAL, "plan is NULL");
  if (nsteps < 0) return fail(CHEMORA_EINVAL, "nsteps %d < 0", nsteps);
  for (int n = 0; n < nsteps; ++n) {
    hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    if (e != hipSuccess) return fail(CHEMORA_EDEVICE, "graph launch: %s", hipGetErrorString(e));
  }
  return CHEMORA_OK;
}

int64_t chemora_plan_points(const chemora_plan* plan) { return plan ? plan->points : 0; }

int chemora_plan_destroy(chemora_plan* plan) {
  g_error.clear();
  if (!plan) return CHEMORA_OK;
  const hipError_t e = hipDeviceSynchronize();
  plan_free(plan);
  return e == hipSuccess ? CHEMORA_OK : fail(CHEMORA_EDEVICE, "plan destroy: %s", hipGetErrorString(e));
}

}  // extern "C"
