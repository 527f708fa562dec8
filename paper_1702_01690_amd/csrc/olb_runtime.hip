// olb_runtime.hip -- host runtime behind the C-ABI of include/olb.h.
//
// An engine holds one or more lattice instances that advance in lockstep.
// It owns no device memory: it carves the caller's workspace into
//   desc      the device table of instances (InstDesc)
//   flag      non-finite flag
//   per instance: A, B, C (f^n and the two RK-3 intermediates, 25 planes of
//             (ny + 6) x nx values), carry[2] (carried n and Delta p,
//             ping-pong) and nw (wall densities)
// and enqueues all device work on the caller's stream.  Every stage is one
// launch over the tile queue of all instances (plus one wall-ghost launch
// with walls).  B and C double as staging for host transfers.  A single
// context (olb_ctx) is an engine with one instance; olb_batch exposes N.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/olb.h"
#include "olb_consts.hpp"
#include "olb_device.hpp"

namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct InstLayout {
  size_t buf, carry, nw, total;
};

InstLayout inst_layout(const olb_params& p) {
  InstLayout L;
  const size_t rb = p.precision == OLB_FP32_MIXED ? 4 : 8;
  const size_t N = (size_t)p.nx * (size_t)p.ny;
  L.buf = align_up(25 * (size_t)(p.ny + 6) * (size_t)p.nx * rb);
  L.carry = align_up(2 * N * sizeof(double));
  L.nw = align_up(2 * (size_t)p.nx * sizeof(double));
  L.total = 3 * L.buf + 2 * L.carry + L.nw;
  return L;
}

size_t head_bytes(int count) { return align_up((size_t)count * sizeof(olbk::InstDesc)) + ALIGN; }

olb_status validate(const olb_params* p, std::string& why) {
  if (!p) { why = "null params"; return OLB_E_ARG; }
  if (p->nx < 1 || p->ny < 1) { why = "nx, ny must be >= 1"; return OLB_E_ARG; }
  // plane and carried-field offsets are 32-bit byte offsets (buffer resources):
  // an FP64 plane of (ny + 6) x nx values must stay below 2^31 bytes
  if ((int64_t)(p->ny + 6) * p->nx * 8 >= (int64_t)1 << 31) {
    why = "lattice too large: (ny + 6) * nx * 8 bytes must stay below 2^31";
    return OLB_E_ARG;
  }
  if (p->bc_x != OLB_BC_PERIODIC && p->bc_x != OLB_BC_SPECULAR) {
    why = "bc_x must be periodic or specular (walls are supported across y only)"; return OLB_E_ARG;
  }
  if (p->bc_x == OLB_BC_SPECULAR && p->nx < 3) { why = "specular x planes need nx >= 3"; return OLB_E_ARG; }
  if (p->bc_y != OLB_BC_PERIODIC && p->bc_y != OLB_BC_DIFFUSE && p->bc_y != OLB_BC_SPECULAR_DIFFUSE) {
    why = "bad bc_y"; return OLB_E_ARG;
  }
  if (p->bc_y != OLB_BC_PERIODIC && p->ny < 3) { why = "walls need ny >= 3"; return OLB_E_ARG; }
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
  if (p->bc_y != OLB_BC_PERIODIC &&
      (!(p->tw_lo > 0.0) || !(p->tw_hi > 0.0) || !std::isfinite(p->tw_lo) ||
       !std::isfinite(p->tw_hi) || !std::isfinite(p->uw_lo) || !std::isfinite(p->uw_hi))) {
    why = "wall temperatures must be positive"; return OLB_E_DOMAIN;
  }
  // CFL condition (Sec. 4.1): p_max dt / (m ds) < 1 with p_max = sqrt(5 + sqrt 10)
  if (!(olbc::R4 * p->dt / p->ds < 1.0)) { why = "CFL: p_max dt / ds >= 1"; return OLB_E_CFL; }
  return OLB_OK;
}

olb_status validate_batch(const olb_params* p, int32_t count, std::string& why) {
  if (!p || count < 1) { why = "need at least one instance"; return OLB_E_ARG; }
  for (int32_t i = 0; i < count; ++i) {
    olb_status s = validate(p + i, why);
    if (s) {
      why = "instance " + std::to_string(i) + ": " + why;
      return s;
    }
    if (p[i].precision != p[0].precision || p[i].bc_y != p[0].bc_y || p[i].bc_x != p[0].bc_x) {
      why = "all instances of a batch share precision and boundary kind";
      return OLB_E_ARG;
    }
  }
  return OLB_OK;
}

}  // namespace

struct Engine {
  std::vector<olb_params> p;
  std::vector<olbk::InstDesc> desc;  // host copy of the device table
  std::vector<bool> have_f;
  hipStream_t stream = nullptr;
  unsigned char* ws = nullptr;
  size_t ws_bytes = 0;
  olbk::InstDesc* d_desc = nullptr;
  int* flag = nullptr;
  int rb = 8;
  bool walls = false;
  bool xspec = false;              // specular planes at both ends of x
  int by = 8;
  int strip = 8;                   // tile order (BatchArgs::strip)
  int cur = 0;                     // carry index of the current f^n
  int total_tiles = 0, wall_blocks = 0;
  int graph_steps = 0;             // 0: direct launches
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::string err;

  int count() const { return (int)p.size(); }

  olb_status fail(olb_status s, const std::string& msg) {
    err = msg;
    return s;
  }
  olb_status hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return OLB_OK;
    return fail(OLB_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
  double rho0(int i) const { return p[i].precision == OLB_FP32_MIXED ? p[i].rho_ref : 0.0; }

  void drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
  }

  // FP32 departure base per population, rho0 b_kx b_ky with
  // b = w (1 + (theta / 2) He2 + (theta^2 / 8) He4), theta = tref - 1
  static void fill_base(olbk::InstDesc& d) {
    const double c2 = 0.5 * (d.tref - 1.0), c4 = 0.5 * c2 * c2;
    double bw[5];
    for (int i = 0; i < 5; ++i) bw[i] = olbc::Wk[i] * (1.0 + c2 * olbc::HE.v[2][i] + c4 * olbc::HE.v[4][i]);
    for (int k = 0; k < 25; ++k) d.base[k] = (float)(d.rho0 * bw[k % 5] * bw[k / 5]);
  }

  // tile counts for the current block height, and the device table
  olb_status upload_desc() {
    int tiles = 0, blocks = 0;
    for (int i = 0; i < count(); ++i) {
      olbk::InstDesc& d = desc[i];
      d.tiles_x = (p[i].nx + olbk::TILE_X - 1) / olbk::TILE_X;
      d.tiles_y = (p[i].ny + by - 1) / by;
      d.tile_base = tiles;
      d.wall_block_base = blocks;
      tiles += d.tiles_x * d.tiles_y;
      blocks += (p[i].nx + 63) / 64;
    }
    total_tiles = tiles;
    wall_blocks = blocks;
    drop_graph();
    olb_status s = hip(hipMemcpyAsync(d_desc, desc.data(), desc.size() * sizeof(olbk::InstDesc),
                                      hipMemcpyHostToDevice, stream), "descriptor upload");
    if (s) return s;
    return hip(hipStreamSynchronize(stream), "stream sync");
  }

  olb_status init(const olb_params* params, int32_t n, void* workspace, size_t bytes, void* strm) {
    p.assign(params, params + n);
    have_f.assign(n, false);
    stream = (hipStream_t)strm;
    ws = (unsigned char*)workspace;
    ws_bytes = bytes;
    rb = p[0].precision == OLB_FP32_MIXED ? 4 : 8;
    // default tile order: whole rows of tiles with FP64 storage (on the 2048^2
    // lattice 0.9 % ahead of strips of 8 tile columns), strips of 8 with FP32
    // storage (0.4 % ahead of whole rows on 4096^2)
    strip = rb == 8 ? 0 : 8;
    walls = p[0].bc_y != OLB_BC_PERIODIC;
    xspec = p[0].bc_x == OLB_BC_SPECULAR;
    d_desc = (olbk::InstDesc*)ws;
    flag = (int*)(ws + align_up((size_t)n * sizeof(olbk::InstDesc)));
    size_t off = head_bytes(n);
    desc.resize(n);
    for (int i = 0; i < n; ++i) {
      const InstLayout L = inst_layout(p[i]);
      olbk::InstDesc& d = desc[i];
      std::memset(&d, 0, sizeof d);
      d.g.nx = p[i].nx;
      d.g.ny = p[i].ny;
      // storage order: the rows of the 25 populations interleaved (element
      // (k, row, x) at (row * 25 + k) * nx + x) when every byte offset into the
      // array fits the 32-bit offsets of the buffer accesses, so that a tile's
      // reads of one row of all populations are one run of addresses; one
      // plane per population ((k * (ny + 6) + row) * nx + x) for larger arrays
      if (25 * (int64_t)(p[i].ny + 6) * p[i].nx * rb < ((int64_t)1 << 31)) {
        d.g.ps = p[i].nx;
        d.g.rs = 25 * (int64_t)p[i].nx;
      } else {
        d.g.ps = (int64_t)(p[i].ny + 6) * p[i].nx;
        d.g.rs = p[i].nx;
      }
      d.g.walls = p[i].bc_y;  // 0 periodic, 1 diffuse walls, 2 specular low end + diffuse high wall
      for (int k = 0; k < 3; ++k) d.f[k] = ws + off + k * L.buf;
      d.carry[0] = (double*)(ws + off + 3 * L.buf);
      d.carry[1] = (double*)(ws + off + 3 * L.buf + L.carry);
      d.nw = (double*)(ws + off + 3 * L.buf + 2 * L.carry);
      d.inv_ds = 1.0 / p[i].ds;
      d.inv_ds3 = 1.0 / (p[i].ds * p[i].ds * p[i].ds);
      d.dt = p[i].dt;
      d.inv_tau = 1.0 / p[i].tau;
      d.a = p[i].a;
      d.b = p[i].b;
      d.sigma = p[i].sigma;
      d.rho0 = rho0(i);
      d.tref = 1.0;
      fill_base(d);
      d.tw[0] = p[i].tw_lo;
      d.tw[1] = p[i].tw_hi;
      d.uw[0] = p[i].uw_lo;
      d.uw[1] = p[i].uw_hi;
      off += L.total;
    }
    // zero everything once (ghost rows of periodic lattices are never written)
    olb_status s = hip(hipMemsetAsync(ws, 0, off, stream), "workspace clear");
    if (s) return s;
    return upload_desc();
  }

  olb_status check_index(int i) {
    if (i < 0 || i >= count()) return fail(OLB_E_ARG, "instance index out of range");
    return OLB_OK;
  }

  olb_status check_fields(int i, const double* n, const double* ux, const double* uy, const double* T) {
    const size_t N = (size_t)p[i].nx * p[i].ny;
    const double nmax = p[i].b > 0.0 ? 1.0 / p[i].b : INFINITY;
    for (size_t k = 0; k < N; ++k) {
      if (!std::isfinite(ux[k]) || !std::isfinite(uy[k])) return fail(OLB_E_DOMAIN, "non-finite velocity");
      if (!(n[k] > 0.0) || !(n[k] < nmax) || !std::isfinite(n[k]))
        return fail(OLB_E_DOMAIN, "density outside (0, 1/b)");
      if (!(T[k] > 0.0) || !std::isfinite(T[k])) return fail(OLB_E_DOMAIN, "temperature <= 0");
    }
    return OLB_OK;
  }

  // f = f^eq of device fields [4][ny][nx] already in instance i's staging area
  olb_status init_from_staging(int i) {
    const olbk::InstDesc& d = desc[i];
    olb_status s = hip(olbk::launch_init(d.g, (const double*)d.f[1], d.f[0], d.carry[cur], d.rho0,
                                         d.tref, d.a, d.b, rb, stream), "init kernel");
    if (s) return s;
    have_f[i] = true;
    return OLB_OK;
  }

  olb_status set_fields(int i, const double* n, const double* ux, const double* uy, const double* T) {
    olb_status s = check_index(i);
    if (s) return s;
    if (!n || !ux || !uy || !T) return fail(OLB_E_ARG, "null field");
    s = check_fields(i, n, ux, uy, T);
    if (s) return s;
    const size_t N = (size_t)p[i].nx * p[i].ny;
    double* stage = (double*)desc[i].f[1];
    const double* src[4] = {n, ux, uy, T};
    for (int k = 0; k < 4; ++k) {
      s = hip(hipMemcpyAsync(stage + k * N, src[k], N * sizeof(double), hipMemcpyHostToDevice, stream),
              "field upload");
      if (s) return s;
    }
    s = init_from_staging(i);
    if (s) return s;
    s = hip(hipMemsetAsync(flag, 0, sizeof(int), stream), "flag clear");
    if (s) return s;
    return hip(hipStreamSynchronize(stream), "stream sync");
  }

  // the same from device fields [4][ny][nx], checked on the device first
  olb_status set_fields_device(int i, const double* fields) {
    olb_status s = check_index(i);
    if (s) return s;
    if (!fields) return fail(OLB_E_ARG, "null fields");
    const olbk::InstDesc& d = desc[i];
    int* bad = flag + 1;
    int h = 0;
    s = hip(hipMemsetAsync(bad, 0, sizeof(int), stream), "flag clear");
    if (s) return s;
    s = hip(olbk::launch_check_fields(d.g, fields, d.b, bad, stream), "field check");
    if (s) return s;
    s = hip(hipMemcpyAsync(&h, bad, sizeof h, hipMemcpyDeviceToHost, stream), "flag copy");
    if (s) return s;
    s = hip(hipStreamSynchronize(stream), "stream sync");
    if (s) return s;
    if (h) return fail(OLB_E_DOMAIN, "field outside the domain (n in (0, 1/b), T > 0, finite)");
    const size_t N = (size_t)p[i].nx * p[i].ny;
    s = hip(hipMemcpyAsync(d.f[1], fields, 4 * N * sizeof(double), hipMemcpyDeviceToDevice, stream),
            "field copy");
    if (s) return s;
    s = init_from_staging(i);
    if (s) return s;
    s = hip(hipMemsetAsync(flag, 0, sizeof(int), stream), "flag clear");
    if (s) return s;
    return hip(hipStreamSynchronize(stream), "stream sync");
  }

  olb_status set_f(int i, const double* f) {
    olb_status s = check_index(i);
    if (s) return s;
    if (!f) return fail(OLB_E_ARG, "null f");
    const olbk::InstDesc& d = desc[i];
    const size_t N = (size_t)p[i].nx * p[i].ny;
    s = hip(hipMemcpyAsync(d.f[1], f, 25 * N * sizeof(double), hipMemcpyHostToDevice, stream), "f upload");
    if (s) return s;
    s = hip(olbk::launch_unpack(d.g, (const double*)d.f[1], d.f[0], d.rho0, d.tref, rb, stream), "unpack kernel");
    if (s) return s;
    s = hip(olbk::launch_carry(d.g, d.f[0], d.carry[cur], d.rho0, d.tref, d.a, d.b, rb, stream), "carry kernel");
    if (s) return s;
    s = hip(hipMemsetAsync(flag, 0, sizeof(int), stream), "flag clear");
    if (s) return s;
    have_f[i] = true;
    return hip(hipStreamSynchronize(stream), "stream sync");
  }

  // FP32 departure base at rest and temperature T (FP64 storage ignores it).
  // A stored state is re-based in place: packed with the old base, unpacked
  // with the new one, its carry recomputed.
  olb_status set_base_temperature(int i, double T) {
    olb_status s = check_index(i);
    if (s) return s;
    if (!(T > 0.0) || !std::isfinite(T)) return fail(OLB_E_ARG, "base temperature must be positive and finite");
    olbk::InstDesc& d = desc[i];
    if (have_f[i] && rb == 4) {
      s = hip(olbk::launch_pack(d.g, d.f[0], (double*)d.f[1], d.rho0, d.tref, rb, stream), "pack kernel");
      if (s) return s;
      s = hip(olbk::launch_unpack(d.g, (const double*)d.f[1], d.f[0], d.rho0, T, rb, stream), "unpack kernel");
      if (s) return s;
      s = hip(olbk::launch_carry(d.g, d.f[0], d.carry[cur], d.rho0, T, d.a, d.b, rb, stream), "carry kernel");
      if (s) return s;
    }
    d.tref = T;
    fill_base(d);
    s = upload_desc();
    if (s) return s;
    return hip(hipStreamSynchronize(stream), "stream sync");
  }

  olb_status read_flag() {
    int h = 0;
    olb_status s = hip(hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, stream), "flag copy");
    if (s) return s;
    s = hip(hipStreamSynchronize(stream), "stream sync");
    if (s) return s;
    if (h) return fail(OLB_E_NONFINITE, "a non-finite density was produced");
    return OLB_OK;
  }

  olb_status get_f(int i, double* f) {
    olb_status s = check_index(i);
    if (s) return s;
    if (!f) return fail(OLB_E_ARG, "null f");
    if (!have_f[i]) return fail(OLB_E_STATE, "no distribution set");
    const olbk::InstDesc& d = desc[i];
    const size_t N = (size_t)p[i].nx * p[i].ny;
    s = hip(olbk::launch_pack(d.g, d.f[0], (double*)d.f[1], d.rho0, d.tref, rb, stream), "pack kernel");
    if (s) return s;
    s = hip(hipMemcpyAsync(f, d.f[1], 25 * N * sizeof(double), hipMemcpyDeviceToHost, stream), "f download");
    if (s) return s;
    return read_flag();
  }

  olb_status moments_device(int i, double* out) {
    olb_status s = check_index(i);
    if (s) return s;
    if (!out) return fail(OLB_E_ARG, "null output");
    if (!have_f[i]) return fail(OLB_E_STATE, "no distribution set");
    const olbk::InstDesc& d = desc[i];
    return hip(olbk::launch_moments(d.g, d.f[0], out, d.rho0, d.tref, rb, stream), "moments kernel");
  }

  olb_status moments(int i, double* n, double* ux, double* uy, double* T) {
    olb_status s = check_index(i);
    if (s) return s;
    if (!n || !ux || !uy || !T) return fail(OLB_E_ARG, "null output");
    const size_t N = (size_t)p[i].nx * p[i].ny;
    double* stage = (double*)desc[i].f[1];
    s = moments_device(i, stage);
    if (s) return s;
    double* dst[4] = {n, ux, uy, T};
    for (int k = 0; k < 4; ++k) {
      s = hip(hipMemcpyAsync(dst[k], stage + k * N, N * sizeof(double), hipMemcpyDeviceToHost, stream),
              "moments download");
      if (s) return s;
    }
    return read_flag();
  }

  olb_status wall_density(int i, double* lo, double* hi) {
    olb_status s = check_index(i);
    if (s) return s;
    if (!lo || !hi) return fail(OLB_E_ARG, "null output");
    if (!walls) return fail(OLB_E_STATE, "no walls");
    const size_t nx = (size_t)p[i].nx;
    s = hip(hipMemcpyAsync(lo, desc[i].nw, nx * sizeof(double), hipMemcpyDeviceToHost, stream), "nw download");
    if (s) return s;
    s = hip(hipMemcpyAsync(hi, desc[i].nw + nx, nx * sizeof(double), hipMemcpyDeviceToHost, stream),
            "nw download");
    if (s) return s;
    return hip(hipStreamSynchronize(stream), "stream sync");
  }

  // one RK-3 step: per stage, wall ghosts of f_src (with walls), then the
  // stage launch over every instance's tiles
  olb_status enqueue_step() {
    for (int s = 0; s < 3; ++s) {
      if (walls) {
        olbk::WallBatchArgs wa{d_desc, count(), s};
        olb_status e = hip(olbk::launch_walls(wa, rb, wall_blocks, stream), "wall kernel");
        if (e) return e;
      }
      olbk::BatchArgs ba;
      ba.inst = d_desc;
      ba.ninst = count();
      ba.total_tiles = total_tiles;
      ba.stage = s;
      ba.cur = cur;
      ba.flag = flag;
      ba.strip = strip;
      ba.A = olbc::RK_A[s];
      ba.B = olbc::RK_B[s];
      ba.wguard = 0x1p-1000;
      olb_status e = hip(olbk::launch_stage(ba, rb, by, walls, xspec, stream), "stage kernel");
      if (e) return e;
      cur ^= 1;
    }
    return OLB_OK;
  }

  olb_status step(int32_t nsteps) {
    if (nsteps < 0) return fail(OLB_E_ARG, "negative step count");
    for (int i = 0; i < count(); ++i)
      if (!have_f[i]) return fail(OLB_E_STATE, "step before every instance has f (set_fields / set_f)");
    int32_t left = nsteps;
    // graph replays: graph_steps is even, so the carry index returns to 0
    while (graph_steps > 0 && left >= graph_steps && cur == 0) {
      if (!graph_exec) {
        olb_status s = hip(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal), "graph capture");
        if (s) return fail(OLB_E_STATE, err + " (graphs need a non-default stream)");
        for (int k = 0; k < graph_steps; ++k) {
          s = enqueue_step();
          if (s) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(stream, &g);
            if (g) (void)hipGraphDestroy(g);
            cur = 0;
            return s;
          }
        }
        s = hip(hipStreamEndCapture(stream, &graph), "graph capture end");
        if (s) return s;
        s = hip(hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0), "graph instantiate");
        if (s) return s;
        cur = 0;  // capture enqueued nothing on the device
      }
      olb_status s = hip(hipGraphLaunch(graph_exec, stream), "graph launch");
      if (s) return s;
      left -= graph_steps;
    }
    for (int32_t k = 0; k < left; ++k) {
      olb_status s = enqueue_step();
      if (s) return s;
    }
    return OLB_OK;
  }

  olb_status set_tile_order(int32_t w) {
    if (w < 0 || w > 1024) return fail(OLB_E_ARG, "strip width must be in 0..1024 tiles");
    if (w == strip) return OLB_OK;
    strip = w;
    drop_graph();
    return OLB_OK;
  }

  olb_status set_tile(int32_t b) {
    // 12 only with FP32 storage: two 12-wave workgroups per CU fit its
    // 80-register budget, while FP64 (128 registers) would run one
    if (b != 8 && b != 16 && !(b == 12 && rb == 4))
      return fail(OLB_E_ARG, "tile height must be 8 or 16 (or 12 with FP32 storage)");
    if (b == by) return OLB_OK;
    by = b;
    return upload_desc();
  }

  // uniform rest state (n = rho_ref or 1, T = wall temperature or 1) in every
  // instance, for timing trials
  olb_status fill_rest_state() {
    for (int i = 0; i < count(); ++i) {
      const size_t N = (size_t)p[i].nx * p[i].ny;
      std::vector<double> h(4 * N);
      const double n0 = p[i].precision == OLB_FP32_MIXED ? p[i].rho_ref : 1.0;
      const double T0 = walls ? p[i].tw_lo : 1.0;
      for (size_t k = 0; k < N; ++k) {
        h[k] = n0;
        h[N + k] = 0.0;
        h[2 * N + k] = 0.0;
        h[3 * N + k] = T0;
      }
      olb_status s = hip(hipMemcpyAsync(desc[i].f[1], h.data(), 4 * N * sizeof(double),
                                        hipMemcpyHostToDevice, stream), "trial upload");
      if (s) return s;
      s = init_from_staging(i);
      if (s) return s;
      s = hip(hipStreamSynchronize(stream), "stream sync");
      if (s) return s;
    }
    return OLB_OK;
  }

  std::string tune_key() const {
    long long nodes = 0;
    for (const auto& q : p) nodes += (long long)q.nx * q.ny;
    std::ostringstream k;
    k << (rb == 8 ? "fp64" : "fp32") << (walls ? "-walls" : "-periodic") << (xspec ? "-xspec" : "") << "-n" << count()
      << "-nodes" << nodes << (graph_steps > 0 ? "-graphs" : "-direct");
    return k.str();
  }

  // A tuned launch configuration: tile height, tile order (strip width) and
  // RK-3 steps per graph (0 when the batch launches directly).
  struct Tuning {
    int by = 8, strip = 8, graph = 0;
  };

  static bool read_int(const std::string& text, size_t from, const char* field, int& v) {
    const size_t at = text.find(std::string("\"") + field + "\":", from);
    if (at == std::string::npos) return false;
    v = std::atoi(text.c_str() + at + std::strlen(field) + 3);
    return true;
  }

  bool read_cache(const char* path, const std::string& key, Tuning& t) const {
    if (!path) return false;
    std::ifstream in(path);
    if (!in) return false;
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string text = ss.str();
    const size_t at = text.find("\"" + key + "\"");
    if (at == std::string::npos) return false;
    Tuning c;
    if (!read_int(text, at, "by", c.by) || !read_int(text, at, "strip", c.strip) ||
        !read_int(text, at, "graph", c.graph))
      return false;
    const bool by_ok = c.by == 8 || c.by == 16 || (c.by == 12 && rb == 4);
    if (!by_ok || c.strip < 0 || c.strip > 1024 || c.graph < 0 || (c.graph > 0) != (graph_steps > 0)) return false;
    t = c;
    return true;
  }

  static void write_cache(const char* path, const std::string& key, const Tuning& t, const std::string& trials) {
    if (!path) return;
    // keep other keys: naive merge by rewriting the object
    std::string body;
    {
      std::ifstream in(path);
      if (in) {
        std::stringstream ss;
        ss << in.rdbuf();
        body = ss.str();
      }
    }
    std::ostringstream entry;
    entry << "\"" << key << "\": {\"by\": " << t.by << ", \"strip\": " << t.strip << ", \"graph\": " << t.graph
          << ", \"ms_per_step\": {" << trials << "}}";
    std::string out;
    const size_t open = body.find('{'), close = body.rfind('}');
    if (open == std::string::npos || close == std::string::npos || body.find("\"" + key + "\"") != std::string::npos) {
      out = "{\n " + entry.str() + "\n}\n";
    } else {
      std::string inner = body.substr(open + 1, close - open - 1);
      while (!inner.empty() && (inner.back() == '\n' || inner.back() == ' ')) inner.pop_back();
      out = "{" + inner + (inner.find_first_not_of(" \n") == std::string::npos ? "\n " : ",\n ") +
            entry.str() + "\n}\n";
    }
    std::ofstream o(path);
    o << out;
  }

  olb_status apply_tuning(const Tuning& t) {
    olb_status s = set_tile(t.by);
    if (!s) s = set_tile_order(t.strip);
    if (s) return s;
    if (t.graph != graph_steps) {
      drop_graph();
      graph_steps = t.graph;
    }
    return OLB_OK;
  }

  // ms per RK-3 step of the current configuration, continuing from the
  // uniform rest state autotune set up (a fixed point of the update): two
  // untimed steps (or one graph, captured), then trial_steps rounded up to an
  // even count (or to whole graphs) timed.  Even counts keep the carry index
  // at 0, where graph replays start.
  olb_status trial(int32_t trial_steps, hipEvent_t e0, hipEvent_t e1, double& ms) {
    const int32_t warm = graph_steps > 0 ? graph_steps : 2;
    const int32_t timed = graph_steps > 0 ? graph_steps * ((trial_steps + graph_steps - 1) / graph_steps)
                                          : 2 * ((trial_steps + 1) / 2);
    olb_status s = step(warm);
    if (!s) s = hip(hipEventRecord(e0, stream), "event record");
    if (!s) s = step(timed);
    if (!s) s = hip(hipEventRecord(e1, stream), "event record");
    if (!s) s = hip(hipEventSynchronize(e1), "event sync");
    float t = 0.0f;
    if (!s) s = hip(hipEventElapsedTime(&t, e0, e1), "event time");
    ms = (double)t / timed;
    return s;
  }

  // Search, one parameter at a time: the tile height (8, 16, and 12 with FP32
  // storage) in the default order, then the tile order (rows, strips of 4, 8
  // and 16 tiles) at the best height, then, when the batch replays graphs,
  // the steps per graph (2, 10, 30).  Results do not depend on any of them.
  olb_status autotune(int32_t trial_steps, const char* cache_path, int32_t* chosen) {
    if (trial_steps < 1) return fail(OLB_E_ARG, "trial_steps must be >= 1");
    const std::string key = tune_key();
    Tuning best;
    if (read_cache(cache_path, key, best)) {
      olb_status s = apply_tuning(best);
      if (s) return s;
      if (chosen) *chosen = best.by;
      return OLB_OK;
    }
    const bool graphs = graph_steps > 0;
    best.graph = graph_steps;
    hipEvent_t e0, e1;
    olb_status s = hip(hipEventCreate(&e0), "event");
    if (s) return s;
    s = hip(hipEventCreate(&e1), "event");
    if (s) {
      (void)hipEventDestroy(e0);
      return s;
    }
    // one rest state for all trials (every instance re-initialised, into
    // carry 0)
    cur = 0;
    s = fill_rest_state();
    std::ostringstream trials;
    auto run = [&](const Tuning& t, const char* label, double& ms) {
      olb_status r = apply_tuning(t);
      if (!r) r = trial(trial_steps, e0, e1, ms);
      if (!r) {
        if (trials.tellp() > 0) trials << ", ";
        trials << "\"" << label << "\": " << ms;
      }
      return r;
    };
    // direct launches while the height and order are chosen
    Tuning t = best;
    t.graph = 0;
    double best_ms = 1e300;
    const int heights[3] = {8, 16, 12};
    for (int h = 0; h < (rb == 4 ? 3 : 2) && !s; ++h) {
      t.by = heights[h];
      t.strip = 8;
      double ms = 0.0;
      const std::string label = "by" + std::to_string(t.by);
      s = run(t, label.c_str(), ms);
      if (!s && ms < best_ms) {
        best_ms = ms;
        best.by = t.by;
      }
    }
    t.by = best.by;
    best_ms = 1e300;
    const int strips[4] = {8, 0, 4, 16};
    for (int w = 0; w < 4 && !s; ++w) {
      t.strip = strips[w];
      double ms = 0.0;
      const std::string label = "by" + std::to_string(t.by) + "-strip" + std::to_string(t.strip);
      s = run(t, label.c_str(), ms);
      if (!s && ms < best_ms) {
        best_ms = ms;
        best.strip = t.strip;
      }
    }
    if (graphs) {
      t.strip = best.strip;
      best_ms = 1e300;
      const int lengths[3] = {10, 2, 30};
      for (int g = 0; g < 3 && !s; ++g) {
        t.graph = lengths[g];
        double ms = 0.0;
        const std::string label = "graph" + std::to_string(t.graph);
        s = run(t, label.c_str(), ms);
        if (!s && ms < best_ms) {
          best_ms = ms;
          best.graph = t.graph;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int i = 0; i < count(); ++i) have_f[i] = false;  // trial states are discarded
    cur = 0;
    if (s) {
      Tuning keep;
      keep.graph = graphs ? best.graph : 0;
      (void)apply_tuning(keep);
      return s;
    }
    s = apply_tuning(best);
    if (s) return s;
    write_cache(cache_path, key, best, trials.str());
    if (chosen) *chosen = best.by;
    return OLB_OK;
  }

  ~Engine() { drop_graph(); }
};

struct olb_ctx {
  Engine e;
};
struct olb_batch {
  Engine e;
};

namespace olbk {
olb_status instance_view(olb_ctx* c, InstanceView* v) {
  if (!c || !v) return OLB_E_ARG;
  Engine& e = c->e;
  if (!e.have_f[0]) return e.fail(OLB_E_STATE, "no distribution set");
  v->g = e.desc[0].g;
  v->f = e.desc[0].f[0];
  v->real_bytes = e.rb;
  v->rho0 = e.desc[0].rho0;
  v->b = e.desc[0].b;
  v->stream = e.stream;
  return OLB_OK;
}

olb_status refresh_carry(olb_ctx* c, hipStream_t s) {
  if (!c) return OLB_E_ARG;
  Engine& e = c->e;
  const InstDesc& d = e.desc[0];
  return e.hip(launch_carry(d.g, d.f[0], d.carry[e.cur], d.rho0, d.tref, d.a, d.b, e.rb, s), "carry kernel");
}
}  // namespace olbk

static size_t engine_bytes(const olb_params* p, int32_t n) {
  size_t total = head_bytes(n);
  for (int32_t i = 0; i < n; ++i) total += inst_layout(p[i]).total;
  return total;
}

template <typename H>
static olb_status make_engine(const olb_params* p, int32_t n, void* ws, size_t bytes, void* stream,
                              H** out) {
  if (!out) return OLB_E_ARG;
  *out = nullptr;
  std::string why;
  olb_status s = validate_batch(p, n, why);
  if (s) return s;
  if (!ws || bytes < engine_bytes(p, n) || ((uintptr_t)ws % ALIGN) != 0) return OLB_E_WORKSPACE;
  H* h = new (std::nothrow) H();
  if (!h) return OLB_E_WORKSPACE;
  s = h->e.init(p, n, ws, bytes, stream);
  if (s) {
    delete h;
    return s;
  }
  *out = h;
  return OLB_OK;
}

extern "C" {

// ------------------------------------------------------------ one instance --

olb_status olb_workspace_bytes(const olb_params* p, size_t* bytes) {
  std::string why;
  if (!bytes) return OLB_E_ARG;
  olb_status s = validate(p, why);
  if (s) return s;
  *bytes = engine_bytes(p, 1);
  return OLB_OK;
}

olb_status olb_init(const olb_params* p, void* dev_workspace, size_t bytes, void* hip_stream,
                    olb_ctx** out) {
  return make_engine(p, 1, dev_workspace, bytes, hip_stream, out);
}

olb_status olb_set_fields(olb_ctx* c, const double* n, const double* ux, const double* uy,
                          const double* T) {
  return c ? c->e.set_fields(0, n, ux, uy, T) : OLB_E_ARG;
}
olb_status olb_set_fields_device(olb_ctx* c, const double* dev_fields) {
  return c ? c->e.set_fields_device(0, dev_fields) : OLB_E_ARG;
}
olb_status olb_step(olb_ctx* c, int32_t nsteps) { return c ? c->e.step(nsteps) : OLB_E_ARG; }
olb_status olb_sync(olb_ctx* c) { return c ? c->e.read_flag() : OLB_E_ARG; }
olb_status olb_moments(olb_ctx* c, double* n, double* ux, double* uy, double* T) {
  return c ? c->e.moments(0, n, ux, uy, T) : OLB_E_ARG;
}
olb_status olb_moments_device(olb_ctx* c, double* dev_out) {
  return c ? c->e.moments_device(0, dev_out) : OLB_E_ARG;
}
olb_status olb_get_f(olb_ctx* c, double* f) { return c ? c->e.get_f(0, f) : OLB_E_ARG; }
olb_status olb_set_f(olb_ctx* c, const double* f) { return c ? c->e.set_f(0, f) : OLB_E_ARG; }
olb_status olb_wall_density(olb_ctx* c, double* lo, double* hi) {
  return c ? c->e.wall_density(0, lo, hi) : OLB_E_ARG;
}
olb_status olb_set_tile(olb_ctx* c, int32_t by) { return c ? c->e.set_tile(by) : OLB_E_ARG; }
olb_status olb_set_base_temperature(olb_ctx* c, double T) { return c ? c->e.set_base_temperature(0, T) : OLB_E_ARG; }
olb_status olb_set_tile_order(olb_ctx* c, int32_t strip) { return c ? c->e.set_tile_order(strip) : OLB_E_ARG; }
olb_status olb_launch_counts(const olb_ctx* c, int32_t* stage, int32_t* walls) {
  if (!c || !stage || !walls) return OLB_E_ARG;
  *stage = 3;
  *walls = c->e.walls ? 3 : 0;
  return OLB_OK;
}
const char* olb_last_error(const olb_ctx* c) { return c ? c->e.err.c_str() : "null context"; }
void olb_free(olb_ctx* c) { delete c; }

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

// ----------------------------------------------------------------- batches --

olb_status olb_batch_workspace_bytes(const olb_params* p, int32_t count, size_t* bytes) {
  std::string why;
  if (!bytes) return OLB_E_ARG;
  olb_status s = validate_batch(p, count, why);
  if (s) return s;
  *bytes = engine_bytes(p, count);
  return OLB_OK;
}

olb_status olb_batch_init(const olb_params* p, int32_t count, void* dev_workspace, size_t bytes,
                          void* hip_stream, olb_batch** out) {
  return make_engine(p, count, dev_workspace, bytes, hip_stream, out);
}

olb_status olb_batch_set_fields(olb_batch* b, int32_t i, const double* n, const double* ux,
                                const double* uy, const double* T) {
  return b ? b->e.set_fields(i, n, ux, uy, T) : OLB_E_ARG;
}
olb_status olb_batch_set_fields_device(olb_batch* b, int32_t i, const double* dev_fields) {
  return b ? b->e.set_fields_device(i, dev_fields) : OLB_E_ARG;
}
olb_status olb_batch_set_f(olb_batch* b, int32_t i, const double* f) {
  return b ? b->e.set_f(i, f) : OLB_E_ARG;
}
olb_status olb_batch_get_f(olb_batch* b, int32_t i, double* f) { return b ? b->e.get_f(i, f) : OLB_E_ARG; }
olb_status olb_batch_step(olb_batch* b, int32_t nsteps) { return b ? b->e.step(nsteps) : OLB_E_ARG; }
olb_status olb_batch_sync(olb_batch* b) { return b ? b->e.read_flag() : OLB_E_ARG; }
olb_status olb_batch_moments(olb_batch* b, int32_t i, double* n, double* ux, double* uy, double* T) {
  return b ? b->e.moments(i, n, ux, uy, T) : OLB_E_ARG;
}
olb_status olb_batch_moments_device(olb_batch* b, int32_t i, double* dev_out) {
  return b ? b->e.moments_device(i, dev_out) : OLB_E_ARG;
}
olb_status olb_batch_wall_density(olb_batch* b, int32_t i, double* lo, double* hi) {
  return b ? b->e.wall_density(i, lo, hi) : OLB_E_ARG;
}
olb_status olb_batch_use_graph(olb_batch* b, int32_t steps_per_graph) {
  if (!b || steps_per_graph < 0) return OLB_E_ARG;
  b->e.drop_graph();
  b->e.graph_steps = steps_per_graph == 0 ? 0 : 2 * ((steps_per_graph + 1) / 2);
  return OLB_OK;
}
olb_status olb_batch_set_tile(olb_batch* b, int32_t by) { return b ? b->e.set_tile(by) : OLB_E_ARG; }
olb_status olb_batch_set_base_temperature(olb_batch* b, int32_t i, double T) {
  return b ? b->e.set_base_temperature(i, T) : OLB_E_ARG;
}
olb_status olb_batch_set_tile_order(olb_batch* b, int32_t strip) {
  return b ? b->e.set_tile_order(strip) : OLB_E_ARG;
}
olb_status olb_batch_autotune(olb_batch* b, int32_t trial_steps, const char* cache_path,
                              int32_t* chosen_by) {
  return b ? b->e.autotune(trial_steps, cache_path, chosen_by) : OLB_E_ARG;
}
olb_status olb_batch_launch_config(const olb_batch* b, int32_t* by, int32_t* strip, int32_t* steps_per_graph) {
  if (!b || !by || !strip || !steps_per_graph) return OLB_E_ARG;
  *by = b->e.by;
  *strip = b->e.strip;
  *steps_per_graph = b->e.graph_steps;
  return OLB_OK;
}
olb_status olb_batch_tiles(const olb_batch* b, int32_t* tiles, int32_t* by) {
  if (!b || !tiles || !by) return OLB_E_ARG;
  *tiles = b->e.total_tiles;
  *by = b->e.by;
  return OLB_OK;
}
const char* olb_batch_last_error(const olb_batch* b) { return b ? b->e.err.c_str() : "null batch"; }
void olb_batch_free(olb_batch* b) { delete b; }

}  // extern "C"
