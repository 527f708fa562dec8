// olb_device.hpp -- launch interface between the host runtime and the gfx950
// kernels of the D2Q25 stage update.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/olb.h"

namespace olbk {

// Storage of one distribution array: 25 planes, each (ny + 6) rows of nx
// values (3 ghost rows below and above the lattice for diffuse walls), x
// fastest.  Interior row y lives at plane row y + 3.
struct Geometry {
  int nx, ny;
  // element (k, storage row, x) of a distribution array is at
  // k * ps + row * rs + x: planes (ps = (ny + 6) nx, rs = nx) or rows of the
  // 25 populations interleaved (ps = nx, rs = 25 nx)
  int64_t ps;      // population stride in elements
  int64_t rs;      // storage-row stride in elements
  int walls;       // 0: periodic y; 1: diffuse walls across y; 2: specular
                   // symmetry plane at the low end, diffuse wall at the high end
};

// One RK stage of one instance, as the tile function sees it.
struct StageArgs {
  Geometry g;
  const void* fsrc;     // f^(s-1)
  const void* fn;       // f^n (RK base); unused when A == 0
  void* fdst;           // f^(s)
  const double* cin;    // carried n and Delta p of fsrc: [2][ny][nx]
  double* cout;         // carried n and Delta p of fdst
  int* flag;            // set to 1 when a non-finite density is produced
  double inv_ds, inv_ds3, dt, inv_tau, a, b, sigma;
  double A, B;          // f_dst = A f^n + B (f_src + dt L[f_src])
  double rho0;          // FP32 departure base: f = rho0 b_kx b_ky + stored value,
  double tref;          // b = w (1 + h(0, tref - 1)) per axis (tref = 1: b = w)
  const float* base;    // [25] rho0 b_kx b_ky (FP32 storage), in the instance descriptor
  double wguard;        // BatchArgs::wguard
};

// One lattice instance of a batch (device table, ascending tile_base).
struct InstDesc {
  Geometry g;
  void* f[3];           // f^n, f^(1), f^(2)
  double* carry[2];     // carried (n, Delta p), ping-pong
  double* nw;           // [2][nx] wall densities (lower, upper)
  double inv_ds, inv_ds3, dt, inv_tau, a, b, sigma, rho0, tref;
  float base[25];       // FP32 departure base per population: rho0 b_kx b_ky
  double tw[2], uw[2];  // lower / upper wall temperature and tangential velocity
  int tiles_x, tiles_y; // stage tiles of 63 x BY nodes
  int tile_base;        // first tile of this instance in the batch's tile queue
  int wall_block_base;  // first 64-column block of this instance (walls)
};

struct BatchArgs {
  const InstDesc* inst;
  int ninst, total_tiles;
  int stage;            // 0, 1, 2: f_src = f[stage], f_dst = f[(stage + 1) % 3]
  int cur;              // carry[cur] belongs to f_src
  int* flag;            // set to 1 when a non-finite density is produced
  int strip;            // tile order: 0 = rows of the tile grid; W > 0 = strips
                        // W tiles wide, rows within a strip, strips left to right
  double A, B;          // f_dst = A f^n + B (f_src + dt L[f_src])
  double wguard;        // 2^-1000: keeps the FP64 WENO denominator positive (an
                        // argument, so that it stays in scalar registers)
};

struct WallBatchArgs {
  const InstDesc* inst;
  int ninst;
  int stage;            // ghost rows are written into f[stage]
};

// Tile geometry of the stage kernel: 64 lanes across x produce 63 cells, BY
// waves across y produce BY rows.
constexpr int TILE_X = 63;

// One workgroup per tile of the batch's tile queue.
hipError_t launch_stage(const BatchArgs& a, int real_bytes, int by, bool walls, bool xspec, hipStream_t s);
// wall_blocks: sum over instances of ceil(nx / 64).
hipError_t launch_walls(const WallBatchArgs& a, int real_bytes, int wall_blocks, hipStream_t s);
// f = f^eq(n, u, T) from device fields [4][ny][nx]; also writes the carry.
hipError_t launch_init(const Geometry& g, const double* fields, void* f, double* carry,
                       double rho0, double tref, double a, double b, int real_bytes, hipStream_t s);
// *bad = 1 if a node of device fields [4][ny][nx] is outside the domain.
hipError_t launch_check_fields(const Geometry& g, const double* fields, double b, int* bad, hipStream_t s);
// n, u_x, u_y, T planes [4][ny][nx] of f.
hipError_t launch_moments(const Geometry& g, const void* f, double* out, double rho0, double tref,
                          int real_bytes, hipStream_t s);
// carried n and Delta p of f.
hipError_t launch_carry(const Geometry& g, const void* f, double* carry, double rho0, double tref,
                        double a, double b, int real_bytes, hipStream_t s);
// packed double [25][ny][nx] <-> stored array.
hipError_t launch_pack(const Geometry& g, const void* f, double* out, double rho0, double tref,
                       int real_bytes, hipStream_t s);
hipError_t launch_unpack(const Geometry& g, const double* in, void* f, double rho0, double tref,
                         int real_bytes, hipStream_t s);

// The stored f^n of a single-instance context, for kernels outside the stage
// update (the learned closure) that modify it in place.
struct InstanceView {
  Geometry g;
  void* f;           // stored f^n (25 planes)
  int real_bytes;    // 8: double, 4: float departure from w_k rho0
  double rho0, b;
  hipStream_t stream;
};
olb_status instance_view(olb_ctx* c, InstanceView* v);
// Recompute the carried (n, Delta p) of f^n after f^n changed, on stream s.
olb_status refresh_carry(olb_ctx* c, hipStream_t s);

}  // namespace olbk
