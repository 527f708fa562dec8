// olb_runtime.hip -- host runtime behind the C-ABI of include/olb.h.
//
// A context owns no device memory: it carves the caller's workspace into
//   A, B, C   three distribution arrays (25 planes of (ny + 6) x nx values:
//             f^n and the two RK-3 intermediates)
//   carry[2]  the carried (n, Delta p) of the current and the next stage
//   nw        wall densities of the last stage
//   flag      non-finite flag
// and enqueues all device work on the caller's stream.  B and C double as a
// staging area for host transfers (they hold no state between steps).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/olb.h"
#include "olb_consts.hpp"
#include "olb_device.hpp"

struct olb_ctx {
  olb_params p;
  hipStream_t stream;
  unsigned char* ws;
  size_t ws_bytes;
  int rb;             // bytes per stored distribution value (8 or 4)
  size_t buf_bytes;   // bytes of one distribution array
  void* f[3];
  double* carry[2];
  double* nw;
  int* flag;
  int cur;            // carry index of the current f
  bool have_f;
  int by;             // stage-kernel block height (8 or 16)
  olbk::Geometry g;
  std::string err;
};

namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
  size_t buf, carry, nw, flag, total;
};

Layout layout_of(const olb_params& p) {
  Layout L;
  const size_t rb = p.precision == OLB_FP32_MIXED ? 4 : 8;
  const size_t N = (size_t)p.nx * (size_t)p.ny;
  L.buf = align_up(25 * (size_t)(p.ny + 6) * (size_t)p.nx * rb);
  L.carry = align_up(2 * N * sizeof(double));
  L.nw = align_up(2 * (size_t)p.nx * sizeof(double));
  L.flag = ALIGN;
  L.total = 3 * L.buf + 2 * L.carry + L.nw + L.flag;
  return L;
}

olb_status set_err(olb_ctx* c, olb_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

olb_status hip_check(olb_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return OLB_OK;
  return set_err(c, OLB_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

olb_status validate(const olb_params* p, std::string& why) {
  if (!p) { why = "null params"; return OLB_E_ARG; }
  if (p->nx < 1 || p->ny < 1) { why = "nx, ny must be >= 1"; return OLB_E_ARG; }
  if ((int64_t)(p->ny + 6) * p->nx >= (int64_t)1 << 31) { why = "lattice too large"; return OLB_E_ARG; }
  if (p->bc_x != OLB_BC_PERIODIC) { why = "walls are supported across y only (bc_x must be periodic)"; return OLB_E_ARG; }
  if (p->bc_y != OLB_BC_PERIODIC && p->bc_y != OLB_BC_DIFFUSE) { why = "bad bc_y"; return OLB_E_ARG; }
  if (p->bc_y == OLB_BC_DIFFUSE && p->ny < 3) { why = "diffuse walls need ny >= 3"; return OLB_E_ARG; }
  if (p->precision != OLB_FP64 && p->precision != OLB_FP32_MIXED) { why = "bad precision"; return OLB_E_ARG; }
  if (!(p->ds > 0.0) || !(p->dt > 0.0) || !std::isfinite(p->ds) || !std::isfinite(p->dt)) {
    why = "ds, dt must be positive and finite"; return OLB_E_ARG;
  }
  if (!(p->a >= 0.0) || !(p->b >= 0.0) || !(p->sigma >= 0.0) || !std::isfinite(p->a) ||
      !std::isfinite(p->b) || !std::isfinite(p->sigma)) {
    why = "a, b, sigma must be finite and >= 0"; return OLB_E_ARG;
  }
  if (p->precision == OLB_FP32_MIXED && !(p->rho_ref > 0.0 && std::isfinite(p->rho_ref))) {
    why = "rho_ref must be positive for FP32 storage"; return OLB_E_ARG;
  }
  if (!(p->tau > 0.0) || !std::isfinite(p->tau)) { why = "tau must be positive"; return OLB_E_DOMAIN; }
  if (p->bc_y == OLB_BC_DIFFUSE &&
      (!(p->tw_lo > 0.0) || !(p->tw_hi > 0.0) || !std::isfinite(p->uw_lo) || !std::isfinite(p->uw_hi))) {
    why = "wall temperatures must be positive"; return OLB_E_DOMAIN;
  }
  // CFL condition (Sec. 4.1): p_max dt / (m ds) < 1 with p_max = sqrt(5 + sqrt 10)
  if (!(olbc::R4 * p->dt / p->ds < 1.0)) { why = "CFL: p_max dt / ds >= 1"; return OLB_E_CFL; }
  return OLB_OK;
}

olb_status check_fields(olb_ctx* c, const double* n, const double* ux, const double* uy,
                        const double* T) {
  const size_t N = (size_t)c->p.nx * c->p.ny;
  const double nmax = c->p.b > 0.0 ? 1.0 / c->p.b : INFINITY;
  for (size_t i = 0; i < N; ++i) {
    if (!std::isfinite(ux[i]) || !std::isfinite(uy[i]))
      return set_err(c, OLB_E_DOMAIN, "non-finite velocity");
    if (!(n[i] > 0.0) || !(n[i] < nmax) || !std::isfinite(n[i]))
      return set_err(c, OLB_E_DOMAIN, "density outside (0, 1/b)");
    if (!(T[i] > 0.0) || !std::isfinite(T[i])) return set_err(c, OLB_E_DOMAIN, "temperature <= 0");
  }
  return OLB_OK;
}

double rho0_of(const olb_ctx* c) { return c->p.precision == OLB_FP32_MIXED ? c->p.rho_ref : 0.0; }

olb_status read_flag(olb_ctx* c) {
  int h = 0;
  olb_status s = hip_check(c, hipMemcpyAsync(&h, c->flag, sizeof h, hipMemcpyDeviceToHost, c->stream),
                           "flag copy");
  if (s) return s;
  s = hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
  if (s) return s;
  if (h) return set_err(c, OLB_E_NONFINITE, "a non-finite density was produced");
  return OLB_OK;
}

}  // namespace

extern "C" {

olb_status olb_workspace_bytes(const olb_params* p, size_t* bytes) {
  std::string why;
  if (!bytes) return OLB_E_ARG;
  olb_status s = validate(p, why);
  if (s) return s;
  *bytes = layout_of(*p).total;
  return OLB_OK;
}

olb_status olb_init(const olb_params* p, void* dev_workspace, size_t bytes, void* hip_stream,
                    olb_ctx** out) {
  if (!out) return OLB_E_ARG;
  *out = nullptr;
  std::string why;
  olb_status s = validate(p, why);
  if (s) return s;
  const Layout L = layout_of(*p);
  if (!dev_workspace || bytes < L.total || ((uintptr_t)dev_workspace % ALIGN) != 0)
    return OLB_E_WORKSPACE;
  olb_ctx* c = new (std::nothrow) olb_ctx();
  if (!c) return OLB_E_WORKSPACE;
  c->p = *p;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (unsigned char*)dev_workspace;
  c->ws_bytes = bytes;
  c->rb = p->precision == OLB_FP32_MIXED ? 4 : 8;
  c->buf_bytes = L.buf;
  for (int i = 0; i < 3; ++i) c->f[i] = c->ws + i * L.buf;
  c->carry[0] = (double*)(c->ws + 3 * L.buf);
  c->carry[1] = (double*)(c->ws + 3 * L.buf + L.carry);
  c->nw = (double*)(c->ws + 3 * L.buf + 2 * L.carry);
  c->flag = (int*)(c->ws + 3 * L.buf + 2 * L.carry + L.nw);
  c->cur = 0;
  c->have_f = false;
  c->by = 8;
  c->g.nx = p->nx;
  c->g.ny = p->ny;
  c->g.ps = (int64_t)(p->ny + 6) * p->nx;
  c->g.walls = p->bc_y == OLB_BC_DIFFUSE;
  // zero everything once: ghost rows of periodic lattices are never written
  s = hip_check(c, hipMemsetAsync(c->ws, 0, L.total, c->stream), "workspace clear");
  if (!s) s = hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
  if (s) {
    delete c;
    return s;
  }
  *out = c;
  return OLB_OK;
}

olb_status olb_set_fields(olb_ctx* c, const double* n, const double* ux, const double* uy,
                          const double* T) {
  if (!c || !n || !ux || !uy || !T) return OLB_E_ARG;
  olb_status s = check_fields(c, n, ux, uy, T);
  if (s) return s;
  const size_t N = (size_t)c->p.nx * c->p.ny;
  double* stage = (double*)c->f[1];
  const double* src[4] = {n, ux, uy, T};
  for (int i = 0; i < 4; ++i) {
    s = hip_check(c, hipMemcpyAsync(stage + i * N, src[i], N * sizeof(double), hipMemcpyHostToDevice,
                                    c->stream), "field upload");
    if (s) return s;
  }
  s = hip_check(c, olbk::launch_init(c->g, stage, c->f[0], c->carry[0], rho0_of(c), c->p.a, c->p.b,
                                     c->rb, c->stream), "init kernel");
  if (s) return s;
  s = hip_check(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream), "flag clear");
  if (s) return s;
  c->cur = 0;
  c->have_f = true;
  return hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
}

olb_status olb_step(olb_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return OLB_E_ARG;
  if (!c->have_f) return set_err(c, OLB_E_STATE, "olb_step before olb_set_fields / olb_set_f");
  const olb_params& p = c->p;
  olbk::StageArgs a;
  a.g = c->g;
  a.flag = c->flag;
  a.inv_ds = 1.0 / p.ds;
  a.inv_ds3 = 1.0 / (p.ds * p.ds * p.ds);
  a.dt = p.dt;
  a.inv_tau = 1.0 / p.tau;
  a.a = p.a;
  a.b = p.b;
  a.sigma = p.sigma;
  a.rho0 = rho0_of(c);
  a.tiles_x = (p.nx + olbk::TILE_X - 1) / olbk::TILE_X;
  const int tiles_y = (p.ny + (c->by - 1) - 1) / (c->by - 1);
  a.ntiles = a.tiles_x * tiles_y;
  olbk::WallArgs w;
  w.g = c->g;
  w.nw = c->nw;
  w.tw[0] = p.tw_lo;
  w.tw[1] = p.tw_hi;
  w.uw[0] = p.uw_lo;
  w.uw[1] = p.uw_hi;
  w.rho0 = a.rho0;
  for (int32_t st = 0; st < nsteps; ++st) {
    for (int s = 0; s < 3; ++s) {
      void* src = c->f[s];                 // A, B, C
      void* dst = c->f[(s + 1) % 3];       // B, C, A
      if (c->g.walls) {
        w.f = src;
        olb_status e = hip_check(c, olbk::launch_walls(w, c->rb, c->stream), "wall kernel");
        if (e) return e;
      }
      a.fsrc = src;
      a.fn = c->f[0];
      a.fdst = dst;
      a.cin = c->carry[c->cur];
      a.cout = c->carry[c->cur ^ 1];
      a.A = olbc::RK_A[s];
      a.B = olbc::RK_B[s];
      olb_status e = hip_check(c, olbk::launch_stage(a, c->rb, c->by, c->stream), "stage kernel");
      if (e) return e;
      c->cur ^= 1;
    }
  }
  return OLB_OK;
}

olb_status olb_sync(olb_ctx* c) {
  if (!c) return OLB_E_ARG;
  return read_flag(c);
}

olb_status olb_moments_device(olb_ctx* c, double* dev_out) {
  if (!c || !dev_out) return OLB_E_ARG;
  if (!c->have_f) return set_err(c, OLB_E_STATE, "no distribution set");
  return hip_check(c, olbk::launch_moments(c->g, c->f[0], dev_out, rho0_of(c), c->rb, c->stream),
                   "moments kernel");
}

olb_status olb_moments(olb_ctx* c, double* n, double* ux, double* uy, double* T) {
  if (!c || !n || !ux || !uy || !T) return OLB_E_ARG;
  if (!c->have_f) return set_err(c, OLB_E_STATE, "no distribution set");
  const size_t N = (size_t)c->p.nx * c->p.ny;
  double* stage = (double*)c->f[1];
  olb_status s = olb_moments_device(c, stage);
  if (s) return s;
  double* dst[4] = {n, ux, uy, T};
  for (int i = 0; i < 4; ++i) {
    s = hip_check(c, hipMemcpyAsync(dst[i], stage + i * N, N * sizeof(double), hipMemcpyDeviceToHost,
                                    c->stream), "moments download");
    if (s) return s;
  }
  return read_flag(c);
}

olb_status olb_get_f(olb_ctx* c, double* f) {
  if (!c || !f) return OLB_E_ARG;
  if (!c->have_f) return set_err(c, OLB_E_STATE, "no distribution set");
  const size_t N = (size_t)c->p.nx * c->p.ny;
  double* stage = (double*)c->f[1];
  olb_status s = hip_check(c, olbk::launch_pack(c->g, c->f[0], stage, rho0_of(c), c->rb, c->stream),
                           "pack kernel");
  if (s) return s;
  s = hip_check(c, hipMemcpyAsync(f, stage, 25 * N * sizeof(double), hipMemcpyDeviceToHost, c->stream),
                "f download");
  if (s) return s;
  return read_flag(c);
}

olb_status olb_set_f(olb_ctx* c, const double* f) {
  if (!c || !f) return OLB_E_ARG;
  const size_t N = (size_t)c->p.nx * c->p.ny;
  double* stage = (double*)c->f[1];
  olb_status s = hip_check(c, hipMemcpyAsync(stage, f, 25 * N * sizeof(double), hipMemcpyHostToDevice,
                                             c->stream), "f upload");
  if (s) return s;
  s = hip_check(c, olbk::launch_unpack(c->g, stage, c->f[0], rho0_of(c), c->rb, c->stream),
                "unpack kernel");
  if (s) return s;
  s = hip_check(c, olbk::launch_carry(c->g, c->f[0], c->carry[0], rho0_of(c), c->p.a, c->p.b, c->rb,
                                      c->stream), "carry kernel");
  if (s) return s;
  s = hip_check(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream), "flag clear");
  if (s) return s;
  c->cur = 0;
  c->have_f = true;
  return hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
}

olb_status olb_wall_density(olb_ctx* c, double* nw_lo, double* nw_hi) {
  if (!c || !nw_lo || !nw_hi) return OLB_E_ARG;
  if (!c->g.walls) return set_err(c, OLB_E_STATE, "no walls");
  const size_t nx = (size_t)c->p.nx;
  olb_status s = hip_check(c, hipMemcpyAsync(nw_lo, c->nw, nx * sizeof(double), hipMemcpyDeviceToHost,
                                             c->stream), "nw download");
  if (s) return s;
  s = hip_check(c, hipMemcpyAsync(nw_hi, c->nw + nx, nx * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream), "nw download");
  if (s) return s;
  return hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
}

olb_status olb_set_tile(olb_ctx* c, int32_t by) {
  if (!c || (by != 8 && by != 16)) return OLB_E_ARG;
  c->by = by;
  return OLB_OK;
}

olb_status olb_launch_counts(const olb_ctx* c, int32_t* stage, int32_t* walls) {
  if (!c || !stage || !walls) return OLB_E_ARG;
  *stage = 3;
  *walls = c->g.walls ? 3 : 0;
  return OLB_OK;
}

const char* olb_last_error(const olb_ctx* c) { return c ? c->err.c_str() : "null context"; }

const char* olb_strerror(olb_status s) {
  switch (s) {
    case OLB_OK: return "ok";
    case OLB_E_ARG: return "bad argument";
    case OLB_E_CFL: return "CFL condition violated (p_max dt / ds >= 1)";
    case OLB_E_DOMAIN: return "value outside the model's domain";
    case OLB_E_NONFINITE: return "non-finite distribution";
    case OLB_E_WORKSPACE: return "workspace too small or misaligned";
    case OLB_E_DEVICE: return "HIP runtime error";
    case OLB_E_STATE: return "call out of order";
  }
  return "unknown status";
}

void olb_free(olb_ctx* c) { delete c; }

}  // extern "C"
