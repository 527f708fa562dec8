// olb_closure.hip -- learned coarse-grid closure on gfx950.
//
// A 3-layer convolutional network (3x3 kernels, periodic padding, 4 -> 32 ->
// 32 -> 4 channels, ReLU between layers) maps the moments (n, u_x, u_y, T) of
// a coarse lattice to a correction of those moments.  Every convolution is an
// implicit GEMM on the bf16 matrix cores with FP32 accumulation: forward
// (v_mfma_f32_16x16x32_bf16, K steps of 32), backward-data (fused with the
// ReLU mask) and backward-weight (pixel reduction) on
// v_mfma_f32_16x16x16_bf16.  Master weights, Adam
// moments and gradients are FP32; activations and gradients entering the
// matrix cores are rounded to bf16 (round to nearest even).
//
// Every sum over pixels (weight and bias gradients, the loss, the channel
// sums of the conservative projection) is formed from per-workgroup partial
// sums added in a fixed order, never with atomics: for a given lattice size
// and device, a computation gives the same bits on every run.
//
// Layouts: activations [pixel][channel], pixel = y * nx + x; parameters are
// one FP32 vector [W1 | b1 | W2 | b2 | W3 | b3] with W[co][ci][ky][kx];
// bf16 weight matrices Wt[co][k] with k = tap * Cin + ci, tap = 3 ky + kx,
// rows padded to 16 and k padded to a multiple of 32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/olb.h"
#include "olb_consts.hpp"
#include "olb_device.hpp"
#include "olb_feq.hpp"

namespace olbk {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8s __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16;

// FP32 -> bf16, rounded to nearest even: gfx950's conversion instruction
// (v_cvt_pk_bf16_f32, two values at a time)
typedef __bf16 bf16x2h __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned to_bf16x2(float lo, float hi) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{lo, hi}, bf16x2h));
}
__device__ __forceinline__ bf16 to_bf16(float f) { return __builtin_bit_cast(bf16, (__bf16)f); }
// The same rounding in integer arithmetic, for values converted from an FP64
// expression: given (__bf16)(float)x the compiler may merge the two
// conversions into one rounding from FP64 (in some code paths and not in
// others), which differs where rounding twice does; the network input is
// defined as rounded to FP32, then to bf16.
__device__ __forceinline__ bf16 to_bf16_int(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16)(u >> 16);
}
__device__ __forceinline__ float from_bf16(bf16 h) { return __uint_as_float(((unsigned)h) << 16); }

// pixel coordinates (one division per lane and kernel, not per tap)
struct Pix {
  int x, y;
};
__device__ __forceinline__ Pix pix_of(int p, int nx) {
  const int y = p / nx;
  return {p - y * nx, y};
}
// neighbour of q for tap = 3 ky + kx: (x + kx - 1, y + ky - 1), periodic
__device__ __forceinline__ int nbr(Pix q, int tap, int nx, int ny) {
  const int ky = tap / 3, kx = tap - 3 * ky;
  int yy = q.y + ky - 1, xx = q.x + kx - 1;
  yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
  xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
  return yy * nx + xx;
}

// bf16 weight matrices Wt[co][k] have their rows padded to a multiple of 32
// (the K step of the forward convolutions' matrix instruction)
constexpr int kp_of(int cin) { return (9 * cin + 31) / 32 * 32; }

// One forward K step (32 values of k = tap * CIN + ci) of the A operand of
// v_mfma_f32_16x16x32_bf16: lane (i, g) holds A[i][8g .. 8g + 7], i.e. the
// 8 consecutive k from k0 = 32 ks + 8g of its pixel.  With CIN a multiple of
// 8 they share a tap (one 16-byte load); with CIN = 4 they span two taps.
// at(tap, ci) is the address of channel ci of the tap's neighbour; k >= K
// reads nothing and gives zeros.
template <int CIN, typename At>
__device__ __forceinline__ bf16x8 a_frag(int k0, int K, At at) {
  bf16x8s v;
  if constexpr (CIN % 8 == 0) {
    if (k0 < K) {
      const int tap = k0 / CIN, ci = k0 - tap * CIN;
      const bf16* p = at(tap, ci);
      const bf16x4 lo = *reinterpret_cast<const bf16x4*>(p), hi = *reinterpret_cast<const bf16x4*>(p + 4);
      v = bf16x8s{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    } else {
      v = bf16x8s{0, 0, 0, 0, 0, 0, 0, 0};
    }
  } else {
    static_assert(CIN == 4, "CIN: a multiple of 8, or 4");
    bf16x4 h[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int k = k0 + 4 * j;
      h[j] = k < K ? *reinterpret_cast<const bf16x4*>(at(k / 4, 0)) : bf16x4{0, 0, 0, 0};
    }
    v = bf16x8s{h[0][0], h[0][1], h[0][2], h[0][3], h[1][0], h[1][1], h[1][2], h[1][3]};
  }
  return __builtin_bit_cast(bf16x8, v);
}
// The same fragment without branches, for LDS operands: with CIN a multiple
// of 8 and K a multiple of 32 every k0 is below K; with CIN = 4 the reads
// past K use tap 0 and are replaced by zeros.
template <int CIN, typename At>
__device__ __forceinline__ bf16x8 a_frag_sel(int k0, int K, At at) {
  bf16x8s v;
  if constexpr (CIN % 8 == 0) {
    static_assert((9 * CIN) % 32 == 0, "K a multiple of the K step");
    const int tap = k0 / CIN, ci = k0 - tap * CIN;
    const bf16* p = at(tap, ci);
    const bf16x4 lo = *reinterpret_cast<const bf16x4*>(p), hi = *reinterpret_cast<const bf16x4*>(p + 4);
    v = bf16x8s{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  } else {
    static_assert(CIN == 4, "CIN: a multiple of 8, or 4");
    bf16x4 h[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int k = k0 + 4 * j;
      const bf16x4 r = *reinterpret_cast<const bf16x4*>(at(k < K ? k / 4 : 0, 0));
      h[j] = k < K ? r : bf16x4{0, 0, 0, 0};
    }
    v = bf16x8s{h[0][0], h[0][1], h[0][2], h[0][3], h[1][0], h[1][1], h[1][2], h[1][3]};
  }
  return __builtin_bit_cast(bf16x8, v);
}
// B operand of the same step: lane (i, g) holds B[8g .. 8g + 7][i] = row i
// of the weight block, 8 consecutive k (16-byte aligned)
__device__ __forceinline__ bf16x8 b_frag(const bf16* row_k0) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const bf16x8s*>(row_k0));
}

// ---------------------------------------------------------------- forward --
// Z[p][co] = b[co] + sum_k Wt[co][k] X[p + off(tap)][ci];  A = bf16(relu(Z)).
// The bf16 weight matrix is staged in LDS once per workgroup (rows padded by 8
// elements, so that every row starts 16-byte aligned for the fragments'
// 16-byte reads).  A wave
// computes FWD_MT tiles of 16 pixels x all output channels; for each tile all
// activation loads are issued before its MFMAs (FWD_MT at most; fewer on small
// lattices so that the grid still fills the chip).  STORE_Z keeps the FP32
// pre-activation (the ReLU mask of the backward pass); STORE_A writes the bf16
// activation (the next layer's input).
constexpr int FWD_MT = 4;
template <int CIN, int COUT, bool RELU, bool STORE_Z, bool STORE_A>
__global__ void __launch_bounds__(256) conv_fwd(const bf16* __restrict__ X, const bf16* __restrict__ Wt,
                                                const float* __restrict__ bias, float* __restrict__ Z,
                                                bf16* __restrict__ A, int nx, int ny, int mtw) {
  constexpr int K = 9 * CIN, KP = kp_of(CIN), KS = KP / 32, NT = (COUT + 15) / 16, ROWS = 16 * NT;
  constexpr int KL = KP + 8;  // LDS row stride (elements): 16-byte aligned rows
  __shared__ __attribute__((aligned(16))) bf16 wl[ROWS * KL];
  for (int e = threadIdx.x; e < ROWS * (KP / 8); e += 256) {
    const int r = e / (KP / 8), c = e - r * (KP / 8);
    *reinterpret_cast<bf16x8s*>(wl + r * KL + 8 * c) = *reinterpret_cast<const bf16x8s*>(Wt + (size_t)r * KP + 8 * c);
  }
  __syncthreads();
  const int P = nx * ny;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  for (int m = 0; m < mtw; ++m) {
    const int p0 = ((blockIdx.x * 4 + wave) * mtw + m) * 16;
    if (p0 >= P) break;  // wave-uniform; no barrier follows
    const Pix qa = pix_of(min(p0 + i, P - 1), nx);  // A-operand row (pixel)
    auto at = [&](int tap, int ci) { return X + (size_t)nbr(qa, tap, nx, ny) * CIN + ci; };
    bf16x8 a[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) a[ks] = a_frag<CIN>(ks * 32 + 8 * g, K, at);
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k0 = ks * 32 + 8 * g;
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ks], b_frag(wl + (t * 16 + i) * KL + k0), acc[t], 0, 0, 0);
    }
    // lane holds D[4g + v][i]: pixel p0 + 4g + v, channel t * 16 + i
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int co = t * 16 + i;
      if (co >= COUT) continue;
      const float bc = bias[co];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = p0 + 4 * g + v;
        if (p >= P) continue;
        const float z = acc[t][v] + bc;
        if (STORE_Z) Z[(size_t)p * COUT + co] = z;
        if (STORE_A) A[(size_t)p * COUT + co] = to_bf16(RELU ? fmaxf(z, 0.f) : z);
      }
    }
  }
}

// ----------------------------------------------------------- backward data --
// dX[q][ci] = sum_{tap, co} G[q - off(tap)][co] Wt[co][tap * CIN + ci]; the
// result is multiplied by the ReLU mask (Zprev > 0) of the layer below and
// rounded to bf16: the gradient with respect to that layer's pre-activation.
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) conv_bwd_data(const bf16* __restrict__ G, const bf16* __restrict__ Wt,
                                                     const float* __restrict__ Zprev,
                                                     bf16* __restrict__ Gprev, int nx, int ny) {
  constexpr int K = 9 * COUT, KP = (K + 15) / 16 * 16, NT = (CIN + 15) / 16;
  constexpr int WKP = kp_of(CIN);
  const int P = nx * ny;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q0 = (blockIdx.x * 4 + wave) * 16;
  if (q0 >= P) return;
  const int i = lane & 15, g = lane >> 4;
  const Pix qa = pix_of(min(q0 + i, P - 1), nx);
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KP / 16; ++ks) {
    const int k0 = ks * 16 + 4 * g;  // k = tap * COUT + co
    bf16x4 a;
    if (k0 < K) {
      const int tap = k0 / COUT, co = k0 - tap * COUT;
      // neighbour q - off(tap): the tap mirrored through the centre (8-byte load)
      a = *reinterpret_cast<const bf16x4*>(G + (size_t)nbr(qa, 8 - tap, nx, ny) * COUT + co);
    } else {
      a = bf16x4{0, 0, 0, 0};
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      bf16x4 b;
      const int ci = t * 16 + i;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = k0 + v;
        if (k < K && ci < CIN) {
          const int tap = k / COUT, co = k - tap * COUT;
          b[v] = (short)Wt[(size_t)co * WKP + tap * CIN + ci];
        } else {
          b[v] = 0;
        }
      }
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int ci = t * 16 + i;
    if (ci >= CIN) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = q0 + 4 * g + v;
      if (q >= P) continue;
      const size_t o = (size_t)q * CIN + ci;
      Gprev[o] = to_bf16(Zprev[o] > 0.f ? acc[t][v] : 0.f);
    }
  }
}

// --------------------------------------------------------- backward weight --
// dW[co][ci][tap] = sum_p G[p][co] X[p + off(tap)][ci]  (GEMM M = COUT,
// N = 9 CIN, reduction over pixels).  Each wave owns one 16 x 16 output tile
// (blockIdx.x picks 4 tiles) and reduces it over one pixel chunk
// (blockIdx.y), whose partial sums it writes to row blockIdx.y of
// dWp[chunk][COUT * CIN * 9]; sum_segments adds the rows in order.
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) conv_bwd_weight(const bf16* __restrict__ G, const bf16* __restrict__ X,
                                                       float* __restrict__ dWp, int nx, int ny, int chunk) {
  constexpr int K = 9 * CIN, KP = (K + 15) / 16 * 16, MT = (COUT + 15) / 16, NTK = KP / 16;
  constexpr int TILES = MT * NTK;
  const int P = nx * ny;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tile = blockIdx.x * 4 + wave;
  if (tile >= TILES) return;
  const int i = lane & 15, g = lane >> 4;
  const int mt = tile / NTK, nt = tile - mt * NTK;
  const int co = mt * 16 + i;             // A-operand row: output channel
  const int k = nt * 16 + i;              // B-operand column: tap * CIN + ci
  const int tap = k / CIN, ci = k - tap * CIN;
  const bool co_ok = co < COUT, k_ok = k < K;
  const int pbeg = blockIdx.y * chunk, pend = min(pbeg + chunk, P);
  // two accumulators over alternate 16-pixel steps keep more loads in flight
  f32x4 acc0 = f32x4{0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
  // coordinates of this lane's 4 pixels in the current and the next step
  Pix q[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int v = 0; v < 4; ++v) q[h][v] = pix_of(min(pbeg + 16 * h + 4 * g + v, P - 1), nx);
  for (int p0 = pbeg; p0 < pend; p0 += 32) {
    bf16x4 a[2], b[2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = p0 + 16 * h + 4 * g + v;
        const bool ok = p < pend;
        a[h][v] = (ok && co_ok) ? (short)G[(size_t)p * COUT + co] : (short)0;
        b[h][v] = (ok && k_ok) ? (short)X[(size_t)nbr(q[h][v], tap, nx, ny) * CIN + ci] : (short)0;
      }
    acc0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[0], acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[1], b[1], acc1, 0, 0, 0);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        q[h][v].x += 32;
        while (q[h][v].x >= nx) {  // at most ceil(32 / nx) passes
          q[h][v].x -= nx;
          ++q[h][v].y;
        }
      }
  }
  const f32x4 acc = acc0 + acc1;
  // lane holds D[4g + v][i]: output channel mt*16 + 4g + v, k = nt*16 + i
  if (!k_ok) return;
  float* row = dWp + (size_t)blockIdx.y * (COUT * CIN * 9);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int c = mt * 16 + 4 * g + v;
    if (c < COUT) row[(c * CIN + ci) * 9 + tap] = acc[v];
  }
}

// Partial bias gradients dbp[block][c] = sum over the block's pixels of
// G[p][c]: thread (row r, channel c) sums channel c over rows r, r + R, ...
// (coalesced rows of C values), then one LDS reduction
template <int C>
__global__ void __launch_bounds__(256) bias_grad(const bf16* __restrict__ G, float* __restrict__ dbp, int P) {
  constexpr int R = 256 / C;
  __shared__ float part[256];
  const int c = threadIdx.x % C, r = threadIdx.x / C;
  float s = 0.f;
  for (int p = blockIdx.x * R + r; p < P; p += gridDim.x * R) s += from_bf16(G[(size_t)p * C + c]);
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < C) {
    float t = 0.f;
#pragma unroll
    for (int j = 0; j < R; ++j) t += part[j * C + threadIdx.x];
    dbp[(size_t)blockIdx.x * C + threadIdx.x] = t;
  }
}

// Fixed-order sums of row-major partial sums: dst[j] = sum over rows r of
// src[r * n + j], for up to 8 segments (blockIdx.y).  A block takes C columns
// (the smallest power of two >= n, at most 256) and R = 256 / C row phases:
// thread (r, c) adds rows r, r + R, ... in order, then a tree over the phases.
// The order depends only on (rows, n), so every run gives the same bits.  The
// rows are loaded 16 at a time before they are added, so that a thread waits
// for one load latency per 16 rows rather than per row.
struct SumSeg {
  const float* src;
  float* dst;
  int rows, n;
};
struct SumSegs {
  SumSeg s[8];
};
__global__ void __launch_bounds__(256) sum_segments(SumSegs segs) {
  const SumSeg sg = segs.s[blockIdx.y];
  int C = 256;
  while (C > 1 && C / 2 >= sg.n) C >>= 1;
  if ((int)blockIdx.x * C >= sg.n) return;  // the whole block: no column here
  const int R = 256 / C, c = threadIdx.x % C, r = threadIdx.x / C;
  const int col = blockIdx.x * C + c;
  __shared__ float red[256];
  constexpr int U = 16;
  float acc = 0.f;
  if (col < sg.n) {
    const float* src = sg.src + col;
    int row = r;
    for (; row + (U - 1) * R < sg.rows; row += U * R) {
      float v[U];
#pragma unroll
      for (int j = 0; j < U; ++j) v[j] = src[(size_t)(row + j * R) * sg.n];
#pragma unroll
      for (int j = 0; j < U; ++j) acc += v[j];
    }
    for (; row < sg.rows; row += R) acc += src[(size_t)row * sg.n];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = R / 2; h > 0; h >>= 1) {
    if (r < h) red[r * C + c] += red[(r + h) * C + c];
    __syncthreads();
  }
  if (r == 0 && col < sg.n) sg.dst[col] = red[c];
}

// Most partial sums of the projection (workgroups of output_sums and of
// infer_kernel)
constexpr int MAX_PARTS = 256;

// Fixed-order total of nparts <= MAX_PARTS rows of four FP64 partial sums,
// for a block of 256 threads: thread t loads row t, then a tree over the
// threads.  Every block (and every run) gets the same bits; red[c][0] holds
// channel c's total on return.  All threads of the block must call it.
__device__ __forceinline__ void block_total4(const double* __restrict__ part, int nparts, double (*red)[256]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int c = 0; c < 4; ++c) red[c][t] = t < nparts ? part[(size_t)t * 4 + c] : 0.0;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h)
#pragma unroll
      for (int c = 0; c < 4; ++c) red[c][t] += red[c][t + h];
    __syncthreads();
  }
}

// ------------------------------------------------------------ glue kernels --

// Conservative restriction r x r: density, momentum and energy densities are
// averaged, then (n, u, T) recovered (m = 1, D = 2).
__global__ void restrict_kernel(const double* __restrict__ fine, int fnx, int fny, int r,
                                double* __restrict__ coarse) {
  const int cnx = fnx / r, cny = fny / r;
  const int X = blockIdx.x * blockDim.x + threadIdx.x, Y = blockIdx.y;
  if (X >= cnx || Y >= cny) return;
  const size_t FN = (size_t)fnx * fny, CN = (size_t)cnx * cny;
  double n = 0.0, jx = 0.0, jy = 0.0, e = 0.0;
  for (int dy = 0; dy < r; ++dy)
    for (int dx = 0; dx < r; ++dx) {
      const size_t m = (size_t)(Y * r + dy) * fnx + (X * r + dx);
      const double nn = fine[m], ux = fine[FN + m], uy = fine[2 * FN + m], T = fine[3 * FN + m];
      n += nn;
      jx += nn * ux;
      jy += nn * uy;
      e += nn * (ux * ux + uy * uy + 2.0 * T);
    }
  const double inv = 1.0 / (r * r);
  n *= inv;
  jx *= inv;
  jy *= inv;
  e *= inv;
  const size_t c = (size_t)Y * cnx + X;
  const double ux = jx / n, uy = jy / n;
  coarse[c] = n;
  coarse[CN + c] = ux;
  coarse[2 * CN + c] = uy;
  coarse[3 * CN + c] = 0.5 * (e / n - ux * ux - uy * uy);
}

struct Norm {
  float in_mean[4], in_inv_scale[4], out_scale[4];
};

// n 32-bit words of p set to zero (the correction's skip counter), as a
// kernel rather than a memset node, so that callers may capture the
// correction in a HIP graph
__global__ void zero_words(unsigned* __restrict__ p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// moment planes (FP64) -> normalised bf16 input [p][4]
__global__ void prep_kernel(const double* __restrict__ m, int P, Norm nm, bf16* __restrict__ x) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
#pragma unroll
  for (int c = 0; c < 4; ++c)
    x[(size_t)p * 4 + c] = to_bf16_int((float)((m[(size_t)c * P + p] - nm.in_mean[c]) * nm.in_inv_scale[c]));
}

// MSE loss on the normalised correction, whose target is (reference - m) /
// out_scale; G3 = dL/dZ3 (bf16); lossp[block] = the block's share of the loss
// (pixels blockIdx.x * 256 + threadIdx.x, stepping by the grid)
__global__ void __launch_bounds__(256) loss_kernel(const float* __restrict__ Z3, const double* __restrict__ m,
                                                   const double* __restrict__ ref, int P, Norm nm,
                                                   bf16* __restrict__ G3, float* __restrict__ lossp) {
  __shared__ float part[256];
  const float scale = 2.0f / (4.0f * (float)P);
  float l = 0.f;
  for (int p = blockIdx.x * 256 + threadIdx.x; p < P; p += gridDim.x * 256) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const size_t o = (size_t)c * P + p;
      const float t = (float)((ref[o] - m[o]) / nm.out_scale[c]);
      const float d = Z3[(size_t)p * 4 + c] - t;
      l += d * d;
      G3[(size_t)p * 4 + c] = to_bf16(scale * d);
    }
  }
  part[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) lossp[blockIdx.x] = part[0] / (4.0f * (float)P);
}

// FP32 master parameters -> bf16 weight matrices (padded) of the three layers
__global__ void pack_weights(const float* __restrict__ w, bf16* __restrict__ W1, bf16* __restrict__ W2,
                             bf16* __restrict__ W3) {
  // layer l: Cin, Cout, offset of W in the flat vector
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  constexpr int KP1 = kp_of(4), KP2 = kp_of(32), KP3 = kp_of(32);
  constexpr int N1 = 32 * KP1, N2 = 32 * KP2, N3 = 16 * KP3;
  constexpr int O1 = 0, O2 = 32 * 4 * 9 + 32, O3 = O2 + 32 * 32 * 9 + 32;
  if (idx < N1) {
    const int co = idx / KP1, k = idx - co * KP1;
    float v = 0.f;
    if (k < 9 * 4) v = w[O1 + (co * 4 + k % 4) * 9 + k / 4];
    W1[idx] = to_bf16(v);
  } else if (idx < N1 + N2) {
    const int j = idx - N1, co = j / KP2, k = j - co * KP2;
    float v = 0.f;
    if (k < 9 * 32) v = w[O2 + (co * 32 + k % 32) * 9 + k / 32];
    W2[j] = to_bf16(v);
  } else if (idx < N1 + N2 + N3) {
    const int j = idx - N1 - N2, co = j / KP3, k = j - co * KP3;
    float v = 0.f;
    if (co < 4 && k < 9 * 32) v = w[O3 + (co * 32 + k % 32) * 9 + k / 32];
    W3[j] = to_bf16(v);
  }
}

__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// partial channel sums of the network output (double), for the conservative
// projection: part[block][c] over pixels blockIdx.x * 256 + threadIdx.x,
// stepping by the grid (at most MAX_PARTS blocks)
__global__ void __launch_bounds__(256) output_sums(const float* __restrict__ Z3, int P, double* __restrict__ part4) {
  __shared__ double part[4][256];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int p = blockIdx.x * 256 + threadIdx.x; p < P; p += gridDim.x * 256)
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c] += (double)Z3[(size_t)p * 4 + c];
#pragma unroll
  for (int c = 0; c < 4; ++c) part[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int c = 0; c < 4; ++c) part[c][threadIdx.x] += part[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) part4[blockIdx.x * 4 + threadIdx.x] = part[threadIdx.x][0];
}

// network output (normalised) -> correction planes (FP64); channels in
// conserve_mask lose their lattice mean (the nparts partial sums of
// output_sums, totalled in a fixed order); 256 threads per block
__global__ void __launch_bounds__(256) delta_kernel(const float* __restrict__ Z3, int P, Norm nm,
                                                    const double* __restrict__ part4, int nparts,
                                                    int conserve_mask, double* __restrict__ delta) {
  __shared__ double red[4][256];
  if (conserve_mask) block_total4(part4, nparts, red);
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double mean = ((conserve_mask >> c) & 1) ? red[c][0] / (double)P : 0.0;
    delta[(size_t)c * P + p] = ((double)Z3[(size_t)p * 4 + c] - mean) * (double)nm.out_scale[c];
  }
}

// ------------------------------------------------------- fused inference --
// The whole network for 16 x 16 output tiles in one persistent workgroup of
// IW waves per CU: the three bf16 weight matrices are staged in LDS once, then
// the workgroup takes tiles blockIdx.x, blockIdx.x + gridDim.x, ...  For each,
// the normalised input on the 22 x 22 region around the tile, layer 1 on
// 20 x 20, layer 2 on 18 x 18 and layer 3 on the tile itself, every
// intermediate in LDS (the halo rows are recomputed by neighbouring tiles).
// The next tile's input is loaded into registers while layer 2 runs and
// written to LDS before its end (the input region is free once layer 1 is
// done), so only two barriers separate the layers of a tile.  Same operands,
// instruction and k order as the layer-by-layer kernels, so the network
// output is the same to the bit; only the moment planes and the corrections
// touch HBM.  Channel sums of the output (for the conservative projection)
// are added to sums[4] when sums != nullptr.
constexpr int FT = 16;            // output tile edge
constexpr int R0 = FT + 6, R1 = FT + 4, R2 = FT + 2;
// weight matrices, rows padded by 8 (16-byte aligned rows)
constexpr int WL = kp_of(32) + 8;
// hidden activations: 32 channels per pixel padded to 36, so that the 16
// pixels one fragment reads start in 16 different bank pairs.  Region rows
// are stored with a stride of (output width of the layer reading them) + 16
// pixels: an m-tile of 16 pixels that wraps to the next output row then
// still falls on 16 different bank pairs (with the natural stride, output
// width + 2, the pixels before and after the wrap collide two by two).
constexpr int HS = 36;
constexpr int S0 = R1 + 16, S1 = R2 + 16, S2 = FT + 2;  // row strides of x0, a1, a2 (a2: no wrap, FT = 16)
// waves per inference workgroup
constexpr int IW = 8;
// K steps whose fragments are read ahead in layers 1, 2, 3 (a step of
// layer 3 is two matrix instructions, of layer 2 six)
constexpr int PD1 = 1, PD2 = 1, PD3 = 3;
struct InferLds {
  __attribute__((aligned(16))) bf16 w2[32 * WL];
  bf16 x0[R0 * S0 * 4];
  bf16 a1[R1 * S1 * HS];
  bf16 a2[R2 * S2 * HS];
  double part[IW][4];
};
static_assert(R0 * R0 <= 64 * IW, "one input pixel per thread");

// copy a bf16 weight matrix (rows x KP) into LDS with row stride KP + 8
template <int ROWS, int KP>
__device__ __forceinline__ void stage_weights(bf16* w, const bf16* __restrict__ Wt, int tid) {
  for (int e = tid; e < ROWS * (KP / 8); e += 64 * IW) {
    const int r = e / (KP / 8), c = e - r * (KP / 8);
    *reinterpret_cast<bf16x8s*>(w + r * (KP + 8) + 8 * c) = *reinterpret_cast<const bf16x8s*>(Wt + (size_t)r * KP + 8 * c);
  }
}

// MFMA layer on an R x R output region from an (R + 2) x (R + 2) input
// region in LDS (rows RI pixels apart): m-tiles of 16 region pixels (row-major), wave w of the IW
// waves taking tiles w, w + IW, ...  The product is taken transposed, weights as the A
// operand and activations as the B operand, so that a lane receives four
// consecutive output channels of one pixel (one 8-byte LDS store instead of
// four 2-byte ones); each output is the same sum of the same exact bf16
// products in the same K steps as in conv_fwd.  The K steps run outermost:
// each weight fragment is read from LDS once per wave and used for all of
// the wave's m-tiles (every accumulator still sees its K steps in ascending
// order).  All fragments of a K step are read before its MFMAs, and a wave
// with one m-tile fewer than the others computes its last one on a clamped
// (valid) region pixel and discards it, so that a K step is one branch-free
// block whose reads the compiler can move ahead of the previous step's
// MFMAs.  `wave` must be uniform (readfirstlane).  The epilogue functor gets
// (pixel, first channel co, the four values of channels co .. co + 3), for
// co < COUT.
// A lane's bias values of one layer: channels t*16 + 4g .. + 3 of each
// n-tile t (zeros past COUT), read once per workgroup so that no global
// read waits in the layers' epilogues.
template <int COUT>
struct BiasRegs {
  static constexpr int NT = (COUT + 15) / 16;
  f32x4 b[NT];
  __device__ __forceinline__ void load(const float* __restrict__ bias, int lane) {
    const int g = lane >> 4;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int co = t * 16 + 4 * g;
      b[t] = co < COUT ? f32x4{bias[co], bias[co + 1], bias[co + 2], bias[co + 3]} : f32x4{0.f, 0.f, 0.f, 0.f};
    }
  }
};

// A wave's weight fragments of one layer for all K steps, held in registers:
// lane (i, g) holds rows t*16 + i, columns ks*32 + 8g .. + 7 of the bf16
// matrix Wt[co][k] (rows padded to 16, row length KP), read from global
// memory once per workgroup: the values the LDS-staged rows give.
template <int CIN, int COUT>
struct WeightFrags {
  static constexpr int KP = kp_of(CIN), KS = KP / 32, NT = (COUT + 15) / 16;
  bf16x8 f[KS][NT];
  __device__ __forceinline__ void load(const bf16* __restrict__ Wt, int lane) {
    const int i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int t = 0; t < NT; ++t) f[ks][t] = b_frag(Wt + (size_t)(t * 16 + i) * KP + ks * 32 + 8 * g);
  }
};
// Weight fragments read from an LDS copy of the matrix (row stride KP + 8).
template <int CIN, int COUT>
struct WeightLds {
  static constexpr int KP = kp_of(CIN);
  const bf16* w;
  __device__ __forceinline__ bf16x8 frag(int ks, int t, int lane) const {
    return b_frag(w + (t * 16 + (lane & 15)) * (KP + 8) + ks * 32 + 8 * (lane >> 4));
  }
};
template <int CIN, int COUT>
__device__ __forceinline__ bf16x8 wfrag(const WeightFrags<CIN, COUT>& w, int ks, int t, int) { return w.f[ks][t]; }
template <int CIN, int COUT>
__device__ __forceinline__ bf16x8 wfrag(const WeightLds<CIN, COUT>& w, int ks, int t, int lane) { return w.frag(ks, t, lane); }

template <int CIN, int COUT, int R, int IS, int RI, int PD, typename Wts, typename Epi>
__device__ __forceinline__ void lds_layer(const bf16* in, const Wts& w, const BiasRegs<COUT>& bias,
                                          int wave, int lane, Epi epi) {
  constexpr int K = 9 * CIN, KP = kp_of(CIN), KS = KP / 32, NT = (COUT + 15) / 16;
  constexpr int NPIX = R * R, MTILES = (NPIX + 15) / 16, MW = (MTILES + IW - 1) / IW;
  static_assert(RI >= R + 2, "input rows hold the output row and its two halo columns");
  static_assert(COUT % 4 == 0, "four channels per lane");
  const int i = lane & 15, g = lane >> 4;
  int base[MW];  // this lane's activation row (region pixel) of each m-tile
#pragma unroll
  for (int m = 0; m < MW; ++m) {
    const int j = min((wave + IW * m) * 16 + i, NPIX - 1);
    const int r = j / R, c = j - r * R;
    base[m] = (r * RI + c) * IS;
  }
  f32x4 acc[MW][NT];
#pragma unroll
  for (int m = 0; m < MW; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  // the fragments of K step ks + PD are read before the MFMAs of step ks
  // (a ring of PD + 1 fragment sets; the scheduling barriers keep that
  // order), so each step waits for reads issued PD steps earlier
  auto read_step = [&](int ks, bf16x8* b, bf16x8* a) {
    const int k0 = ks * 32 + 8 * g;
#pragma unroll
    for (int t = 0; t < NT; ++t) b[t] = wfrag(w, ks, t, lane);
#pragma unroll
    for (int m = 0; m < MW; ++m) {
      auto at = [&](int tap, int ci) {
        const int ky = tap / 3, kx = tap - 3 * ky;
        return in + base[m] + (ky * RI + kx) * IS + ci;
      };
      a[m] = a_frag_sel<CIN>(k0, K, at);
    }
  };
  static_assert(PD >= 1, "prefetch depth");
  bf16x8 b[PD + 1][NT], a[PD + 1][MW];
#pragma unroll
  for (int p = 0; p < PD && p < KS; ++p) read_step(p, b[p], a[p]);
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int cur = ks % (PD + 1);
    if (ks + PD < KS) read_step(ks + PD, b[(ks + PD) % (PD + 1)], a[(ks + PD) % (PD + 1)]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = 0; m < MW; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[cur][t], a[cur][m], acc[m][t], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
  // lane (i, g) holds the transposed D[4g + v][i]: channel t*16 + 4g + v of
  // region pixel mt*16 + i
#pragma unroll
  for (int m = 0; m < MW; ++m) {
    const int mt = wave + IW * m;
    if (mt >= MTILES) continue;
    const int q = mt * 16 + i;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int co = t * 16 + 4 * g;
      if (co >= COUT || q >= NPIX) continue;
      epi(q, co, f32x4{acc[m][t][0] + bias.b[t][0], acc[m][t][1] + bias.b[t][1], acc[m][t][2] + bias.b[t][2],
                       acc[m][t][3] + bias.b[t][3]});
    }
  }
}

// four bf16 values of ReLU(z) as one 8-byte LDS store (dst 8-byte aligned)
__device__ __forceinline__ void store_relu4(bf16* dst, f32x4 z) {
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  *reinterpret_cast<u32x2*>(dst) = u32x2{to_bf16x2(fmaxf(z[0], 0.f), fmaxf(z[1], 0.f)),
                                         to_bf16x2(fmaxf(z[2], 0.f), fmaxf(z[3], 0.f))};
}

__global__ void __launch_bounds__(64 * IW) infer_kernel(const double* __restrict__ m, Norm nm,
                                                    const bf16* __restrict__ W1, const bf16* __restrict__ W2,
                                                    const bf16* __restrict__ W3, const float* __restrict__ b1,
                                                    const float* __restrict__ b2, const float* __restrict__ b3,
                                                    int nx, int ny, int tiles_x, int ntiles,
                                                    double* __restrict__ delta, double* __restrict__ part4) {
  __shared__ InferLds sm;
  const int P = nx * ny;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // thread tid < 22 * 22 carries input pixel tid of the region: its four
  // moments, loaded (periodic wrap) and then written normalised to LDS
  double in[4];
  auto load_input = [&](int tile) {
    if (tid >= R0 * R0) return;
    const int ty0 = (tile / tiles_x) * FT, tx0 = (tile % tiles_x) * FT;
    const int r = tid / R0, c = tid - r * R0;
    int gy = (ty0 - 3 + r) % ny, gx = (tx0 - 3 + c) % nx;
    gy += gy < 0 ? ny : 0;
    gx += gx < 0 ? nx : 0;
    const size_t p = (size_t)gy * nx + gx;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) in[ch] = m[(size_t)ch * P + p];
  };
  auto store_input = [&]() {
    if (tid >= R0 * R0) return;
    const int r = tid / R0, c = tid - r * R0;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch)
      sm.x0[(r * S0 + c) * 4 + ch] = to_bf16_int((float)((in[ch] - nm.in_mean[ch]) * nm.in_inv_scale[ch]));
  };
  int tile = blockIdx.x;
  load_input(tile);
  // layer 2's weights in LDS; layers 1 and 3 (16 and 36 registers) in registers
  stage_weights<32, kp_of(32)>(sm.w2, W2, tid);
  WeightFrags<4, 32> wf1;
  WeightFrags<32, 4> wf3;
  wf1.load(W1, lane);
  wf3.load(W3, lane);
  const WeightLds<32, 32> wl2{sm.w2};
  store_input();
  BiasRegs<32> bias1, bias2;
  BiasRegs<4> bias3;
  bias1.load(b1, lane);
  bias2.load(b2, lane);
  bias3.load(b3, lane);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (; tile < ntiles; tile += gridDim.x) {
    const int ty0 = (tile / tiles_x) * FT, tx0 = (tile % tiles_x) * FT;
    // the input region (and, on the first tile, the weights) are in LDS; a1
    // was last read by the previous tile's layer 2, before its second barrier
    __syncthreads();
    lds_layer<4, 32, R1, 4, S0, PD1>(sm.x0, wf1, bias1, wave, lane, [&](int q, int co, f32x4 z) {
      const int r = q / R1, c = q - r * R1;
      store_relu4(sm.a1 + (r * S1 + c) * HS + co, z);
    });
    // a1 complete; the input region is free (layer 2 writes a2, which the
    // previous tile's layer 3 read before this tile's first barrier)
    __syncthreads();
    const int next = tile + gridDim.x;
    if (next < ntiles) load_input(next);
    lds_layer<32, 32, R2, HS, S1, PD2>(sm.a1, wl2, bias2, wave, lane, [&](int q, int co, f32x4 z) {
      const int r = q / R2, c = q - r * R2;
      store_relu4(sm.a2 + (r * S2 + c) * HS + co, z);
    });
    if (next < ntiles) store_input();
    __syncthreads();
    lds_layer<32, 4, FT, HS, S2, PD3>(sm.a2, wf3, bias3, wave, lane, [&](int q, int, f32x4 z) {
      const int r = q / FT, c = q - r * FT;
      const int gy = ty0 + r, gx = tx0 + c;
      if (gy < ny && gx < nx) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          delta[(size_t)k * P + (size_t)gy * nx + gx] = (double)z[k] * (double)nm.out_scale[k];
          s[k] += (double)z[k];
        }
      }
    });
  }
  if (part4) {
    // lanes 0..15 hold all four channels of their pixels (the others hold
    // zeros): fold the 64 lanes, then the waves, into this workgroup's row
    // of partial sums
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double v = s[k];
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o);
      s[k] = v;
    }
    if (lane < 4) sm.part[wave][lane] = s[lane];
    __syncthreads();
    if (tid < 4) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < IW; ++w) t += sm.part[w][tid];
      part4[blockIdx.x * 4 + tid] = t;
    }
  }
}

// Workgroups of infer_kernel: one per CU (its LDS holds all three weight
// matrices and the intermediates, about 93 KB), at most one per tile and at
// most MAX_PARTS (one row of projection partial sums each).
static int infer_grid(int ntiles) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  return std::min(std::min(ntiles, cus), MAX_PARTS);
}

// delta[c] -= mean_c * out_scale[c] for the channels in mask; the channel
// totals of the normalised output over P nodes are the nparts rows of
// partial sums of infer_kernel, totalled in a fixed order; 256 threads per
// block
__global__ void __launch_bounds__(256) project_kernel(double* __restrict__ delta, int P, Norm nm,
                                                      const double* __restrict__ part4, int nparts, int mask) {
  __shared__ double red[4][256];
  block_total4(part4, nparts, red);
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if ((mask >> c) & 1) delta[(size_t)c * P + p] -= red[c][0] / (double)P * (double)nm.out_scale[c];
}

// f <- f + f^eq(m') - f^eq(m) with m' = m + dm (absolute == 0) or m' = dm
// (absolute == 1) where m' is admissible (finite, 0 < n < 1/b, T > 0); other
// nodes keep f (counted in skipped).
template <typename Real>
__global__ void apply_kernel(const double* __restrict__ m, const double* __restrict__ dm, int absolute,
                             Geometry geo, Real* __restrict__ f, double b, int* __restrict__ skipped) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= geo.nx) return;
  const size_t N = (size_t)geo.nx * geo.ny, c = (size_t)y * geo.nx + x;
  const double n0 = m[c], ux0 = m[N + c], uy0 = m[2 * N + c], T0 = m[3 * N + c];
  const double base = absolute ? 0.0 : 1.0;
  const double n1 = base * n0 + dm[c], ux1 = base * ux0 + dm[N + c], uy1 = base * uy0 + dm[2 * N + c],
               T1 = base * T0 + dm[3 * N + c];
  const bool ok = isfinite(n1) && isfinite(ux1) && isfinite(uy1) && isfinite(T1) && n1 > 0.0 &&
                  (b <= 0.0 || n1 * b < 1.0) && T1 > 0.0;
  if (!ok) {
    atomicAdd(skipped, 1);
    return;
  }
  double h0x[5], h0y[5], h1x[5], h1y[5];
  hfac(ux0, T0 - 1.0, h0x);
  hfac(uy0, T0 - 1.0, h0y);
  hfac(ux1, T1 - 1.0, h1x);
  hfac(uy1, T1 - 1.0, h1y);
  const int own = (y + 3) * (int)geo.rs + x;
#pragma unroll
  for (int ky = 0; ky < 5; ++ky)
#pragma unroll
    for (int kx = 0; kx < 5; ++kx) {
      const double w = Wk[kx] * Wk[ky];
      const double d = w * (n1 * (1.0 + h1x[kx]) * (1.0 + h1y[ky]) - n0 * (1.0 + h0x[kx]) * (1.0 + h0y[ky]));
      Real* q = f + (5 * ky + kx) * geo.ps + own;
      *q = (Real)((double)*q + d);
    }
}

}  // namespace olbk

// --------------------------------------------------------------------------
// device scratch of the allocation-free inference entry point
// --------------------------------------------------------------------------
// The bf16 weight matrices of the three layers and the projection's partial
// channel sums (one row of four per inference workgroup).  One copy per GPU,
// held until the process ends; every call on a GPU overwrites it.  In host code the name stands for a host-side
// stand-in: kernels and copies get its device address from
// hipGetSymbolAddress (noalloc_scratch below), never the name itself.
namespace {
constexpr size_t NA_W1 = 0;
constexpr size_t NA_W2 = NA_W1 + 32 * olbk::kp_of(4) * sizeof(olbk::bf16);
constexpr size_t NA_W3 = NA_W2 + 32 * olbk::kp_of(32) * sizeof(olbk::bf16);
constexpr size_t NA_PART = NA_W3 + 16 * olbk::kp_of(32) * sizeof(olbk::bf16);
constexpr size_t NA_USED = NA_PART + olbk::MAX_PARTS * 4 * sizeof(double);
constexpr size_t NA_BYTES = 40960;
static_assert(NA_USED <= NA_BYTES, "scratch layout");
static_assert(NA_PART % 8 == 0, "partial sums alignment");
}  // namespace
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

// --------------------------------------------------------------------------
// host side
// --------------------------------------------------------------------------


namespace {
constexpr int NPARAM = 32 * 4 * 9 + 32 + 32 * 32 * 9 + 32 + 4 * 32 * 9 + 4;
static_assert(NPARAM == OLB_CLOSURE_NPARAM, "parameter count");
constexpr size_t AL = 256;
size_t al(size_t v) { return (v + AL - 1) / AL * AL; }

// Pixel chunks of the weight-gradient kernel: about 512 workgroups (tile
// groups x chunks), chunks of a multiple of 16 pixels
template <int CIN, int COUT>
struct BwdWeightGrid {
  static constexpr int tiles = ((COUT + 15) / 16) * (olbk::kp_of(CIN) / 16);
  static constexpr int groups = (tiles + 3) / 4;
  int chunk, nchunks;
  explicit BwdWeightGrid(int P) {
    const int chunks = std::max(1, std::min((P + 63) / 64, 512 / groups));
    chunk = ((P + chunks - 1) / chunks + 15) / 16 * 16;
    nchunks = (P + chunk - 1) / chunk;
  }
};
int bias_blocks(int P) { return std::min(1024, std::max(1, P / 256)); }
int loss_blocks(int P) { return std::min(1024, (P + 255) / 256); }

// Rows of partial sums of the backward pass, in the order of the parameter
// vector's blocks: W1, b1, W2, b2, W3, b3, then the loss
struct GradParts {
  int rows[7], n[7];
  size_t off[7], floats;
  explicit GradParts(int P) {
    rows[0] = BwdWeightGrid<4, 32>(P).nchunks;
    rows[2] = BwdWeightGrid<32, 32>(P).nchunks;
    rows[4] = BwdWeightGrid<32, 4>(P).nchunks;
    rows[1] = rows[3] = rows[5] = bias_blocks(P);
    rows[6] = loss_blocks(P);
    const int ns[7] = {32 * 4 * 9, 32, 32 * 32 * 9, 32, 4 * 32 * 9, 4, 1};
    floats = 0;
    for (int k = 0; k < 7; ++k) {
      n[k] = ns[k];
      off[k] = floats;
      floats += (size_t)rows[k] * n[k];
    }
  }
};

struct CLayout {
  size_t x0, z1, a1, z2, a2, z3, g3, g2, g1, mom, delta, par, grad, am, av, w1, w2, w3, loss, skip, part4, gpart,
      total;
};

CLayout clayout(int nx, int ny) {
  const size_t P = (size_t)nx * ny;
  CLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += al(bytes); return r; };
  L.x0 = take(P * 4 * 2);
  L.z1 = take(P * 32 * 4);
  L.a1 = take(P * 32 * 2);
  L.z2 = take(P * 32 * 4);
  L.a2 = take(P * 32 * 2);
  L.z3 = take(P * 4 * 4);
  L.g3 = take(P * 4 * 2);
  L.g2 = take(P * 32 * 2);
  L.g1 = take(P * 32 * 2);
  L.mom = take(P * 4 * 8);
  L.delta = take(P * 4 * 8);
  L.par = take(NPARAM * 4);
  L.grad = take(NPARAM * 4);
  L.am = take(NPARAM * 4);
  L.av = take(NPARAM * 4);
  L.w1 = take(32 * olbk::kp_of(4) * 2);
  L.w2 = take(32 * olbk::kp_of(32) * 2);
  L.w3 = take(16 * olbk::kp_of(32) * 2);
  L.loss = take(4);
  L.skip = take(4);
  L.part4 = take(olbk::MAX_PARTS * 4 * 8);
  L.gpart = take(GradParts((int)P).floats * 4);
  L.total = o;
  return L;
}
}  // namespace

struct olb_closure {
  int nx, ny, P;
  hipStream_t stream;
  unsigned char* ws;
  CLayout L;
  olbk::Norm norm;
  int adam_t = 0;
  int conserve_mask = 7;  // n, u_x, u_y corrections are made mean-free
  bool have_params = false;
  std::string err;

  template <typename T>
  T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }

  olb_status hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return OLB_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return OLB_E_DEVICE;
  }

  int pix_blocks() const { return (P + 63) / 64; }  // 4 waves x 16 pixels
  // 16-pixel tiles per wave of the forward convolutions: up to FWD_MT while
  // at least 1024 workgroups remain
  int fwd_mtw() const { return std::max(1, std::min(olbk::FWD_MT, P / (64 * 1024))); }
  int fwd_blocks() const { return (P + 64 * fwd_mtw() - 1) / (64 * fwd_mtw()); }

  // keep_z: also store the pre-activations of the hidden layers (backward)
  olb_status forward(const double* dev_m, bool keep_z) {
    using namespace olbk;
    const float* par = at<float>(L.par);
    const float* b1 = par + 32 * 4 * 9;
    const float* b2 = par + (32 * 4 * 9 + 32) + 32 * 32 * 9;
    const float* b3 = par + (NPARAM - 4);
    hipLaunchKernelGGL(prep_kernel, dim3((P + 255) / 256), dim3(256), 0, stream, dev_m, P, norm, at<bf16>(L.x0));
    const dim3 fg(fwd_blocks());
    const int mtw = fwd_mtw();
    if (keep_z) {
      hipLaunchKernelGGL((conv_fwd<4, 32, true, true, true>), fg, dim3(256), 0, stream,
                         at<bf16>(L.x0), at<bf16>(L.w1), b1, at<float>(L.z1), at<bf16>(L.a1), nx, ny, mtw);
      hipLaunchKernelGGL((conv_fwd<32, 32, true, true, true>), fg, dim3(256), 0, stream,
                         at<bf16>(L.a1), at<bf16>(L.w2), b2, at<float>(L.z2), at<bf16>(L.a2), nx, ny, mtw);
    } else {
      hipLaunchKernelGGL((conv_fwd<4, 32, true, false, true>), fg, dim3(256), 0, stream,
                         at<bf16>(L.x0), at<bf16>(L.w1), b1, at<float>(L.z1), at<bf16>(L.a1), nx, ny, mtw);
      hipLaunchKernelGGL((conv_fwd<32, 32, true, false, true>), fg, dim3(256), 0, stream,
                         at<bf16>(L.a1), at<bf16>(L.w2), b2, at<float>(L.z2), at<bf16>(L.a2), nx, ny, mtw);
    }
    // layer 3: no activation, only the FP32 output
    hipLaunchKernelGGL((conv_fwd<32, 4, false, true, false>), fg, dim3(256), 0, stream,
                       at<bf16>(L.a2), at<bf16>(L.w3), b3, at<float>(L.z3), at<bf16>(L.g3), nx, ny, mtw);
    return hip(hipGetLastError(), "closure forward");
  }

  // corrections for device moments through the fused kernel, projected
  olb_status infer(const double* dev_m, double* dev_delta) {
    using namespace olbk;
    const float* par = at<float>(L.par);
    double* part4 = conserve_mask ? at<double>(L.part4) : nullptr;
    const int tiles_x = (nx + FT - 1) / FT, tiles_y = (ny + FT - 1) / FT, ntiles = tiles_x * tiles_y;
    const int grid = infer_grid(ntiles);
    hipLaunchKernelGGL(infer_kernel, dim3(grid), dim3(64 * IW), 0, stream, dev_m, norm, at<bf16>(L.w1),
                       at<bf16>(L.w2), at<bf16>(L.w3), par + 32 * 4 * 9, par + (32 * 4 * 9 + 32) + 32 * 32 * 9,
                       par + (NPARAM - 4), nx, ny, tiles_x, ntiles, dev_delta, part4);
    if (part4)
      hipLaunchKernelGGL(project_kernel, dim3((P + 255) / 256), dim3(256), 0, stream, dev_delta, P, norm, part4,
                         grid, conserve_mask);
    return hip(hipGetLastError(), "closure inference");
  }

  // layer-by-layer forward (the reference for the fused kernel; training)
  olb_status forward_layers(const double* dev_m, double* dev_delta) {
    using namespace olbk;
    olb_status s = forward(dev_m, false);
    if (s) return s;
    double* part4 = at<double>(L.part4);
    const int nparts = std::min(MAX_PARTS, (P + 255) / 256);
    if (conserve_mask)
      hipLaunchKernelGGL(output_sums, dim3(nparts), dim3(256), 0, stream, at<float>(L.z3), P, part4);
    hipLaunchKernelGGL(delta_kernel, dim3((P + 255) / 256), dim3(256), 0, stream, at<float>(L.z3), P, norm, part4,
                       nparts, conserve_mask, dev_delta);
    return hip(hipGetLastError(), "delta kernel");
  }

  // Gradient of the loss for every parameter, and the loss: each kernel
  // writes partial sums (per pixel chunk or block) to its rows of L.gpart,
  // which sum_segments then adds in a fixed order into L.grad and L.loss.
  olb_status backward(const double* dev_m, const double* dev_ref) {
    using namespace olbk;
    const GradParts gp(P);
    float* part = at<float>(L.gpart);
    hipLaunchKernelGGL(loss_kernel, dim3(gp.rows[6]), dim3(256), 0, stream, at<float>(L.z3), dev_m, dev_ref, P,
                       norm, at<bf16>(L.g3), part + gp.off[6]);
    // layer 3
    launch_bwd_weight<32, 4>(at<bf16>(L.g3), at<bf16>(L.a2), part + gp.off[4]);
    hipLaunchKernelGGL((bias_grad<4>), dim3(gp.rows[5]), dim3(256), 0, stream, at<bf16>(L.g3), part + gp.off[5], P);
    hipLaunchKernelGGL((conv_bwd_data<32, 4>), dim3(pix_blocks()), dim3(256), 0, stream, at<bf16>(L.g3),
                       at<bf16>(L.w3), at<float>(L.z2), at<bf16>(L.g2), nx, ny);
    // layer 2
    launch_bwd_weight<32, 32>(at<bf16>(L.g2), at<bf16>(L.a1), part + gp.off[2]);
    hipLaunchKernelGGL((bias_grad<32>), dim3(gp.rows[3]), dim3(256), 0, stream, at<bf16>(L.g2), part + gp.off[3],
                       P);
    hipLaunchKernelGGL((conv_bwd_data<32, 32>), dim3(pix_blocks()), dim3(256), 0, stream, at<bf16>(L.g2),
                       at<bf16>(L.w2), at<float>(L.z1), at<bf16>(L.g1), nx, ny);
    // layer 1 (the input needs no gradient)
    launch_bwd_weight<4, 32>(at<bf16>(L.g1), at<bf16>(L.x0), part + gp.off[0]);
    hipLaunchKernelGGL((bias_grad<32>), dim3(gp.rows[1]), dim3(256), 0, stream, at<bf16>(L.g1), part + gp.off[1],
                       P);
    // the parameter vector's blocks follow each other in gp's order
    SumSegs segs{};
    float* dst = at<float>(L.grad);
    int bx = 1;
    for (int k = 0; k < 7; ++k) {
      segs.s[k] = SumSeg{part + gp.off[k], k < 6 ? dst : at<float>(L.loss), gp.rows[k], gp.n[k]};
      if (k < 6) dst += gp.n[k];
      bx = std::max(bx, (gp.n[k] + 255) / 256);
    }
    hipLaunchKernelGGL(sum_segments, dim3(bx, 7), dim3(256), 0, stream, segs);
    return hip(hipGetLastError(), "closure backward");
  }

  // about 512 workgroups per weight gradient: tile groups x pixel chunks;
  // dWp receives one row of partial sums per chunk
  template <int CIN, int COUT>
  void launch_bwd_weight(const olbk::bf16* G, const olbk::bf16* X, float* dWp) {
    const BwdWeightGrid<CIN, COUT> g(P);
    hipLaunchKernelGGL((olbk::conv_bwd_weight<CIN, COUT>), dim3(BwdWeightGrid<CIN, COUT>::groups, g.nchunks),
                       dim3(256), 0, stream, G, X, dWp, nx, ny, g.chunk);
  }

  olb_status pack() {
    using namespace olbk;
    const int n = 32 * kp_of(4) + 32 * kp_of(32) + 16 * kp_of(32);
    hipLaunchKernelGGL(pack_weights, dim3((n + 255) / 256), dim3(256), 0, stream, at<float>(L.par),
                       at<bf16>(L.w1), at<bf16>(L.w2), at<bf16>(L.w3));
    return hip(hipGetLastError(), "weight pack");
  }
};

namespace {
bool valid_size(int32_t nx, int32_t ny) { return nx >= 1 && ny >= 1 && (int64_t)nx * ny < (1 << 30); }
}  // namespace

extern "C" {

olb_status olb_closure_workspace_bytes(int32_t nx, int32_t ny, size_t* bytes) {
  if (!bytes || !valid_size(nx, ny)) return OLB_E_ARG;
  *bytes = clayout(nx, ny).total;
  return OLB_OK;
}

olb_status olb_closure_init(int32_t nx, int32_t ny, void* dev_workspace, size_t bytes, void* hip_stream,
                            olb_closure** out) {
  if (!out || !valid_size(nx, ny)) return OLB_E_ARG;
  *out = nullptr;
  const CLayout L = clayout(nx, ny);
  if (!dev_workspace || bytes < L.total || ((uintptr_t)dev_workspace % AL) != 0) return OLB_E_WORKSPACE;
  olb_closure* c = new (std::nothrow) olb_closure();
  if (!c) return OLB_E_WORKSPACE;
  c->nx = nx;
  c->ny = ny;
  c->P = nx * ny;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (unsigned char*)dev_workspace;
  c->L = L;
  for (int k = 0; k < 4; ++k) {
    c->norm.in_mean[k] = 0.f;
    c->norm.in_inv_scale[k] = 1.f;
    c->norm.out_scale[k] = 1.f;
  }
  olb_status s = c->hip(hipMemsetAsync(c->ws, 0, L.total, c->stream), "workspace clear");
  if (!s) s = c->hip(hipStreamSynchronize(c->stream), "stream sync");
  if (s) {
    delete c;
    return s;
  }
  *out = c;
  return OLB_OK;
}

olb_status olb_closure_set_norm(olb_closure* c, const double in_mean[4], const double in_scale[4],
                                const double out_scale[4]) {
  if (!c || !in_mean || !in_scale || !out_scale) return OLB_E_ARG;
  for (int k = 0; k < 4; ++k) {
    if (!(in_scale[k] > 0.0) || !(out_scale[k] > 0.0) || !std::isfinite(in_mean[k])) return OLB_E_ARG;
    c->norm.in_mean[k] = (float)in_mean[k];
    c->norm.in_inv_scale[k] = (float)(1.0 / in_scale[k]);
    c->norm.out_scale[k] = (float)out_scale[k];
  }
  return OLB_OK;
}

olb_status olb_closure_set_params(olb_closure* c, const float* params) {
  if (!c || !params) return OLB_E_ARG;
  for (int k = 0; k < NPARAM; ++k)
    if (!std::isfinite(params[k])) return OLB_E_ARG;
  olb_status s = c->hip(hipMemcpyAsync(c->at<float>(c->L.par), params, NPARAM * 4, hipMemcpyHostToDevice,
                                       c->stream), "param upload");
  if (s) return s;
  s = c->hip(hipMemsetAsync(c->at<float>(c->L.am), 0, NPARAM * 4, c->stream), "adam clear");
  if (!s) s = c->hip(hipMemsetAsync(c->at<float>(c->L.av), 0, NPARAM * 4, c->stream), "adam clear");
  if (!s) s = c->pack();
  if (!s) s = c->hip(hipStreamSynchronize(c->stream), "stream sync");
  if (s) return s;
  c->adam_t = 0;
  c->have_params = true;
  return OLB_OK;
}

olb_status olb_closure_get_params(olb_closure* c, float* params) {
  if (!c || !params) return OLB_E_ARG;
  olb_status s = c->hip(hipMemcpyAsync(params, c->at<float>(c->L.par), NPARAM * 4, hipMemcpyDeviceToHost,
                                       c->stream), "param download");
  if (s) return s;
  return c->hip(hipStreamSynchronize(c->stream), "stream sync");
}

olb_status olb_closure_forward(olb_closure* c, const double* dev_moments, double* dev_delta) {
  if (!c || !dev_moments || !dev_delta) return OLB_E_ARG;
  if (!c->have_params) return OLB_E_STATE;
  return c->infer(dev_moments, dev_delta);
}

olb_status olb_closure_forward_layers(olb_closure* c, const double* dev_moments, double* dev_delta) {
  if (!c || !dev_moments || !dev_delta) return OLB_E_ARG;
  if (!c->have_params) return OLB_E_STATE;
  return c->forward_layers(dev_moments, dev_delta);
}
olb_status olb_closure_set_conserve(olb_closure* c, int32_t mask) {
  if (!c || mask < 0 || mask > 15) return OLB_E_ARG;
  c->conserve_mask = mask;
  return OLB_OK;
}

olb_status olb_closure_gradients(olb_closure* c, const double* dev_moments, const double* dev_reference,
                                 float* grad, float* loss) {
  if (!c || !dev_moments || !dev_reference || !grad) return OLB_E_ARG;
  if (!c->have_params) return OLB_E_STATE;
  olb_status s = c->forward(dev_moments, true);
  if (!s) s = c->backward(dev_moments, dev_reference);
  if (!s) s = c->hip(hipMemcpyAsync(grad, c->at<float>(c->L.grad), NPARAM * 4, hipMemcpyDeviceToHost,
                                    c->stream), "grad download");
  if (!s && loss)
    s = c->hip(hipMemcpyAsync(loss, c->at<float>(c->L.loss), 4, hipMemcpyDeviceToHost, c->stream), "loss");
  if (!s) s = c->hip(hipStreamSynchronize(c->stream), "stream sync");
  return s;
}

olb_status olb_closure_train_step(olb_closure* c, const double* dev_moments, const double* dev_reference,
                                  float lr, float* loss) {
  if (!c || !dev_moments || !dev_reference || !(lr > 0.f)) return OLB_E_ARG;
  if (!c->have_params) return OLB_E_STATE;
  olb_status s = c->forward(dev_moments, true);
  if (!s) s = c->backward(dev_moments, dev_reference);
  if (s) return s;
  c->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.0f / (1.0f - std::pow(b1, (float)c->adam_t));
  const float c2 = 1.0f / (1.0f - std::pow(b2, (float)c->adam_t));
  hipLaunchKernelGGL(olbk::adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, c->stream,
                     c->at<float>(c->L.par), c->at<float>(c->L.grad), c->at<float>(c->L.am),
                     c->at<float>(c->L.av), NPARAM, lr, b1, b2, eps, c1, c2);
  s = c->hip(hipGetLastError(), "adam kernel");
  if (!s) s = c->pack();
  if (!s && loss) {
    s = c->hip(hipMemcpyAsync(loss, c->at<float>(c->L.loss), 4, hipMemcpyDeviceToHost, c->stream), "loss");
    if (!s) s = c->hip(hipStreamSynchronize(c->stream), "stream sync");
  }
  return s;
}

}  // extern "C"

namespace {
// moments of the coarse lattice into m_buf, then f <- f + f^eq(m') - f^eq(m)
// with m' = m + network(m) (target == nullptr) or m' = target
olb_status correct(olb_closure* c, olb_ctx* coarse, const double* target, double* m_buf, int32_t* skipped) {
  if (!c || !coarse) return OLB_E_ARG;
  if (!target && !c->have_params) return OLB_E_STATE;
  olbk::InstanceView v;
  olb_status s = olbk::instance_view(coarse, &v);
  if (s) return s;
  if (v.g.nx != c->nx || v.g.ny != c->ny) return OLB_E_ARG;
  if (v.stream != c->stream) {
    // order the two streams: the closure waits for the solver's queued steps
    s = c->hip(hipStreamSynchronize(v.stream), "solver sync");
    if (s) return s;
  }
  if (!m_buf) m_buf = c->at<double>(c->L.mom);
  s = olb_moments_device(coarse, m_buf);
  if (s) return s;
  if (v.stream != c->stream) {
    s = c->hip(hipStreamSynchronize(v.stream), "solver sync");
    if (s) return s;
  }
  const int absolute = target != nullptr;
  if (!target) {
    s = olb_closure_forward(c, m_buf, c->at<double>(c->L.delta));
    if (s) return s;
    target = c->at<double>(c->L.delta);
  }
  hipLaunchKernelGGL(olbk::zero_words, dim3(1), dim3(64), 0, c->stream, reinterpret_cast<unsigned*>(c->at<int>(c->L.skip)),
                     1);
  dim3 grid((c->nx + 63) / 64, c->ny);
  if (v.real_bytes == 8)
    hipLaunchKernelGGL(olbk::apply_kernel<double>, grid, dim3(64), 0, c->stream, m_buf, target, absolute, v.g,
                       (double*)v.f, v.b, c->at<int>(c->L.skip));
  else
    hipLaunchKernelGGL(olbk::apply_kernel<float>, grid, dim3(64), 0, c->stream, m_buf, target, absolute, v.g,
                       (float*)v.f, v.b, c->at<int>(c->L.skip));
  s = c->hip(hipGetLastError(), "apply kernel");
  if (s) return s;
  // the carried (n, Delta p) of the solver must follow the corrected f
  s = olbk::refresh_carry(coarse, c->stream);
  if (s) return s;
  if (skipped) {
    s = c->hip(hipMemcpyAsync(skipped, c->at<int>(c->L.skip), 4, hipMemcpyDeviceToHost, c->stream), "skip");
    if (s) return s;
  }
  // the solver's next steps on its own stream must see the corrected f
  if (skipped || v.stream != c->stream) s = c->hip(hipStreamSynchronize(c->stream), "stream sync");
  return s;
}
}  // namespace

extern "C" {

olb_status olb_closure_apply(olb_closure* c, olb_ctx* coarse, int32_t* skipped) {
  return correct(c, coarse, nullptr, nullptr, skipped);
}

olb_status olb_closure_nudge(olb_closure* c, olb_ctx* coarse, const double* dev_target, double* dev_moments,
                             int32_t* skipped) {
  if (!dev_target) return OLB_E_ARG;
  return correct(c, coarse, dev_target, dev_moments, skipped);
}

olb_status olb_restrict(const double* dev_fine, int32_t fnx, int32_t fny, int32_t factor, double* dev_coarse,
                        void* hip_stream) {
  if (!dev_fine || !dev_coarse || factor < 1 || fnx < factor || fny < factor || fnx % factor ||
      fny % factor)
    return OLB_E_ARG;
  const int cnx = fnx / factor, cny = fny / factor;
  hipLaunchKernelGGL(olbk::restrict_kernel, dim3((cnx + 63) / 64, cny), dim3(64), 0, (hipStream_t)hip_stream,
                     dev_fine, fnx, fny, factor, dev_coarse);
  return hipGetLastError() == hipSuccess ? OLB_OK : OLB_E_DEVICE;
}

}  // extern "C"

namespace {
// Device address of `scratch` on the current device, looked up once per
// device (each GPU holds its own copy at its own address).
constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mutex;
void* na_ptr[NA_MAX_DEVICES] = {};

olb_status noalloc_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NA_MAX_DEVICES) return OLB_E_DEVICE;
  std::lock_guard<std::mutex> lock(na_mutex);
  if (!na_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return OLB_E_DEVICE;
    na_ptr[dev] = p;
  }
  *out = na_ptr[dev];
  return OLB_OK;
}
}  // namespace

extern "C" {

olb_status olb_closure_forward_noalloc(int32_t nx, int32_t ny, const float* dev_params, const double in_mean[4],
                                       const double in_scale[4], const double out_scale[4], int32_t conserve_mask,
                                       const double* dev_moments, double* dev_delta, void* hip_stream) {
  using namespace olbk;
  if (!dev_params || !in_mean || !in_scale || !out_scale || !dev_moments || !dev_delta) return OLB_E_ARG;
  if (!valid_size(nx, ny) || conserve_mask < 0 || conserve_mask > 15) return OLB_E_ARG;
  Norm nm;
  for (int k = 0; k < 4; ++k) {
    if (!(in_scale[k] > 0.0) || !(out_scale[k] > 0.0) || !std::isfinite(in_mean[k])) return OLB_E_ARG;
    nm.in_mean[k] = (float)in_mean[k];
    nm.in_inv_scale[k] = (float)(1.0 / in_scale[k]);
    nm.out_scale[k] = (float)out_scale[k];
  }
  void* base = nullptr;
  olb_status s = noalloc_scratch(&base);
  if (s) return s;
  unsigned char* sc = static_cast<unsigned char*>(base);
  bf16* W1 = reinterpret_cast<bf16*>(sc + NA_W1);
  bf16* W2 = reinterpret_cast<bf16*>(sc + NA_W2);
  bf16* W3 = reinterpret_cast<bf16*>(sc + NA_W3);
  double* part4 = conserve_mask ? reinterpret_cast<double*>(sc + NA_PART) : nullptr;
  hipStream_t st = (hipStream_t)hip_stream;
  const int n = 32 * kp_of(4) + 32 * kp_of(32) + 16 * kp_of(32);
  hipLaunchKernelGGL(pack_weights, dim3((n + 255) / 256), dim3(256), 0, st, dev_params, W1, W2, W3);
  const int tiles_x = (nx + FT - 1) / FT, tiles_y = (ny + FT - 1) / FT, ntiles = tiles_x * tiles_y;
  const int P = nx * ny;
  const int grid = infer_grid(ntiles);
  hipLaunchKernelGGL(infer_kernel, dim3(grid), dim3(64 * IW), 0, st, dev_moments, nm, W1, W2, W3,
                     dev_params + 32 * 4 * 9, dev_params + (32 * 4 * 9 + 32) + 32 * 32 * 9, dev_params + (NPARAM - 4),
                     nx, ny, tiles_x, ntiles, dev_delta, part4);
  if (part4)
    hipLaunchKernelGGL(project_kernel, dim3((P + 255) / 256), dim3(256), 0, st, dev_delta, P, nm, part4, grid,
                       conserve_mask);
  return hipGetLastError() == hipSuccess ? OLB_OK : OLB_E_DEVICE;
}

const char* olb_closure_last_error(const olb_closure* c) { return c ? c->err.c_str() : "null closure"; }
void olb_closure_free(olb_closure* c) { delete c; }

}  // extern "C"
