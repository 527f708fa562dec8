// olb_kernels.hip -- gfx950 kernels of the D2Q25 off-lattice thermal Boltzmann
// stage update (arXiv:1702.01690, Secs. 2-3).
//
// stage_kernel  one RK-3 stage, fused: moments, EOS, 49-point force, Hermite
//               equilibrium, force term, BGK, WENO-5 fluxes in x and y and the
//               RK combine, plus the carried (n, Delta p) of the result for the
//               next stage's stencils.
// walls_kernel  ghost rows of the stage's source array across y: diffuse-
//               reflection walls, or a specular plane at the low end.
// init / moments / carry / pack / unpack  set-up and read-out.
//
// Data layout: element (k, y + 3, x) of f at k * ps + (y + 3) * rs + x (see
// Geometry: planes, or rows of the 25 populations interleaved), one cell per
// thread.  A 64 x BY
// thread block covers 64 x BY nodes; lane 63 only provides the left face of
// its neighbour, so each block writes 63 x BY cells.  Per population, the
// tile plus a 3-node halo (69 x (BY + 6) values) is staged in LDS; each
// thread reconstructs the WENO value on its left (x) and lower (y) face only,
// the right face arrives from lane + 1 by a DPP wavefront shift and the upper
// face from the next wave through LDS.  The tile's top face is reconstructed
// by one wave per population, in turn.  Specular planes across x are folded
// into the halo's load addresses.
#include <type_traits>

#include "olb_consts.hpp"
#include "olb_device.hpp"
#include "olb_feq.hpp"

namespace olbk {
using namespace olbc;

// Global-memory views of pointers that reach a kernel through a descriptor
// in memory (the compiler cannot prove their address space and would emit
// flat accesses, which share the LDS wait counter: every wait for an LDS read
// would then also wait for all loads in flight).
template <typename T>
using gmem = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ gmem<T>* as_global(T* p) {
  return (gmem<T>*)p;
}

// Buffer resource starting at population k of an array whose populations are
// pop_bytes apart, with rec_bytes of records (the plane, or everything from
// population k's first element to the end of the array when the rows of the
// populations are interleaved), and loads / stores through it.  A lane's byte
// offset from the population's start is the same for every population, and
// the base sits in scalar registers, so these accesses cost the vector ALUs no
// address arithmetic.  Offsets at or past rec_bytes read 0 and write nothing.
// (Word 3 of the descriptor: raw 32-bit data, the gfx9 buffer format.)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, int k, uint32_t pop_bytes,
                                                            uint32_t rec_bytes) {
  const char* p = static_cast<const char*>(base) + (int64_t)k * pop_bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(p), (short)0, (int)rec_bytes, 0x00020000);
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, int k, uint32_t plane_bytes) {
  return plane_rsrc(base, k, plane_bytes, plane_bytes);
}
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
template <typename Real>
__device__ __forceinline__ Real bload(__amdgpu_buffer_rsrc_t r, int byte_off) {
  if constexpr (sizeof(Real) == 4)
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
  else
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
}
template <typename Real>
__device__ __forceinline__ void bstore(Real v, __amdgpu_buffer_rsrc_t r, int byte_off) {
  if constexpr (sizeof(Real) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, byte_off, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, byte_off, 0, 0);
}

// Value held by lane + 1 of the wavefront (lane 63 receives 0): a DPP
// wavefront shift by one lane, a VALU move rather than an LDS round trip.
__device__ __forceinline__ float lane_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_next(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ int wrapi(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

// Reciprocal: the hardware estimate (about 2^-23 relative) refined by one
// Newton step (about 2^-46, far below what the weight normalisation below
// needs), or the single-precision estimate (FP32).
__device__ __forceinline__ double frcp(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  return __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
}
__device__ __forceinline__ float frcp(float d) { return __builtin_amdgcn_rcpf(d); }

// WENO-5 reconstruction at i + 1/2 for a positive speed from
// (f_{i-2}, f_{i-1}, f_i, f_{i+1}, f_{i+2}) (Eqs. weno5_flux..weno5_sigma).
// No epsilon: when indicators vanish, the weights follow Tab. weno, i.e. the
// ideal weights restricted to the vanishing candidates.  Indicators are formed
// from first differences d, so a vanishing indicator is exactly "three equal
// values".  The weights are scale free, so each indicator is used times 4:
// s_q = (13/3) a_q^2 + b_q^2.  The normalised weights need one reciprocal:
//   w_q ~ delta_q prod_{r != q} s_r^2,  delta_q ~ (1, 6, 3),
// which already gives Tab. weno when one indicator vanishes (that candidate
// alone keeps a non-zero weight).  When two or more vanish, every candidate
// that keeps a weight equals f_i (its values are all f_i), so the result is
// f_i.  The candidates enter through their offsets from f_i, times 6:
//   e1 = 5 d2 - 2 d1,  e2 = d2 + 2 d3,  e3 = 4 d3 - d4,
// and the ideal weights and the 1/6 are folded into them: with
// W1 = (s2 s3)^2, W2 = (s1 s3)^2, W3 = (s1 s2)^2 the face value is
//   f_i + [W1 e1/6 + W2 e2 + W3 e3/2] / [W1 + 6 W2 + 3 W3].
__device__ __forceinline__ double weno_rec(double v0, double v1, double v2, double v3, double v4,
                                           double guard = 0x1p-1000) {
  const double d1 = v1 - v0, d2 = v2 - v1, d3 = v3 - v2, d4 = v4 - v3;
  const double a1 = d2 - d1, b1 = __builtin_fma(3.0, d2, -d1);
  const double a2 = d3 - d2, b2 = d2 + d3;
  const double a3 = d4 - d3, b3 = __builtin_fma(3.0, d3, -d4);
  const double s1 = __builtin_fma(a1 * (13.0 / 3.0), a1, b1 * b1);
  const double s2 = __builtin_fma(a2 * (13.0 / 3.0), a2, b2 * b2);
  const double s3 = __builtin_fma(a3 * (13.0 / 3.0), a3, b3 * b3);
  const double q1 = s1 * s1, q2 = s2 * s2, q3 = s3 * s3;
  // guard = 2^-1000 in the second weight keeps den > 0 without a branch (the
  // FP32 form below explains why the result is then f_i when two indicators
  // vanish); a weight it could disturb would need differences of 1e-36, far
  // below the rounding of any population value.  The stage kernel passes it
  // from a kernel argument: FP64 constants have no literal form in the
  // three-operand FMA, and a constant addend is otherwise rebuilt in vector
  // registers (two moves) for every face.
  const double w1 = q2 * q3, w2 = __builtin_fma(q1, q3, guard), w3 = q1 * q2;
  const double g1 = __builtin_fma(5.0 / 6.0, d2, d1 * (-1.0 / 3.0));
  const double g2 = __builtin_fma(2.0, d3, d2);
  const double g3 = __builtin_fma(2.0, d3, d4 * -0.5);
  const double num = __builtin_fma(w1, g1, __builtin_fma(w2, g2, w3 * g3));
  const double den = __builtin_fma(3.0, w3, __builtin_fma(6.0, w2, w1));
  return __builtin_fma(num, frcp(den), v2);
}

// FP32: the weights are products of squared indicators (eighth powers of the
// differences), which would leave the FP32 range, so the three indicators are
// multiplied by one factor c close to 1/m, m the largest of them: the scaled
// indicators lie in [0, 1) and the largest in [1/2, 9/16].  A common factor
// cancels in the weights (it only adds a rounding to each scaled indicator);
// the candidate offsets stay unscaled.  An indicator that underflows acts as a
// vanishing one, which changes the result by far less than FP32 rounding (its
// three values then agree to far below the rounding of f_i).
//
// Instruction forms (gfx950 issues two FP32 add / mul / FMA instructions per
// SIMD quad-cycle when no operand sits in a scalar register, and one
// ldexp / frexp / scalar-operand instruction): the outer differences are
// formed with the opposite sign (e1 = -d1, e4 = -d4), so that 3 d2 - d1 and
// 3 d3 - d4 are FMAs with a literal and no negated operand (3.0 is not an
// inline constant, and the negated form would take it from a scalar
// register); a3 enters squared only, so its sign is free.  The factor c is
// one integer subtraction from the bits of m: for a normal m = (1 + u) 2^(E-127)
// (biased exponent E, mantissa fraction u), the bits 0x7e800000 - bits(m)
// encode c = (2 - u) 2^(125-E), so that c m = (2 - u)(1 + u) / 4 lies in
// [1/2, 9/16]; no frexp / ldexp, and no mask of the exponent field.  This
// holds for m < 2^125, i.e. for differences below about 1e18, far beyond any
// population value (from 2^125 on, c falls below the normal range).
// (m below the normal range, i.e. differences of order 1e-19, gets c close to
// 2^126; the weights are then those of values that agree far below FP32
// rounding.  m = 0 happens only with d2 = d3 = 0 and e1 = e4 = 0, when every
// candidate offset vanishes.)
__device__ __forceinline__ float weno_rec(float v0, float v1, float v2, float v3, float v4) {
  const float e1 = v0 - v1, d2 = v2 - v1, d3 = v3 - v2, e4 = v3 - v4;
  const float a1 = d2 + e1, b1 = __builtin_fmaf(3.0f, d2, e1);
  const float a2 = d3 - d2, b2 = d2 + d3;
  const float a3 = d3 + e4, b3 = __builtin_fmaf(3.0f, d3, e4);
  const float t1 = __builtin_fmaf(a1 * (13.0f / 3.0f), a1, b1 * b1);
  const float t2 = __builtin_fmaf(a2 * (13.0f / 3.0f), a2, b2 * b2);
  const float t3 = __builtin_fmaf(a3 * (13.0f / 3.0f), a3, b3 * b3);
  const float m = fmaxf(fmaxf(t1, t2), t3);
  const float sc = __uint_as_float(0x7e800000u - __float_as_uint(m));
  const float s1 = t1 * sc, s2 = t2 * sc, s3 = t3 * sc;
  const float q1 = s1 * s1, q2 = s2 * s2, q3 = s3 * s3;
  // 2^-126 in the second weight keeps den > 0 without a branch: den would
  // vanish only with two indicators zero, and then d2 = d3 = 0 (s1 = s2 = 0,
  // s1 = s3 = 0) or d2 = d3 = d4 = 0 (s2 = s3 = 0), so g2 = 0 and the other
  // two weights vanish: num = 0 and the result is f_i, as the rule above
  // requires.  Elsewhere it moves den by 1e-37 at most.
  const float w1 = q2 * q3, w2 = __builtin_fmaf(q1, q3, 0x1p-126f), w3 = q1 * q2;
  const float g1 = __builtin_fmaf(5.0f / 6.0f, d2, e1 * (1.0f / 3.0f));
  const float g2 = __builtin_fmaf(2.0f, d3, d2);
  const float g3 = __builtin_fmaf(2.0f, d3, e4 * 0.5f);
  const float num = __builtin_fmaf(w1, g1, __builtin_fmaf(w2, g2, w3 * g3));
  const float den = __builtin_fmaf(3.0f, w3, __builtin_fmaf(6.0f, w2, w1));
  return __builtin_fmaf(num, frcp(den), v2);
}

// FP32 departure base: f = rho0 b_kx b_ky + stored value, with per-axis
// factors b = w (1 + h0) of the equilibrium at rest and temperature tref,
// h0 = h(0, tref - 1) (tref = 1: b = w).  Its moments: sum b = 1,
// sum b p = 0, sum b p^2 = tref.
__device__ __forceinline__ void base_h0(double tref, double h0[5]) { hfac(0.0, tref - 1.0, h0); }

// Moment sums of one node: n = sum f, j = sum p f, e = sum |p|^2 f, with the
// FP32 departure base added back (n: rho0, e: 2 rho0 tref).
template <typename Real>
__device__ __forceinline__ void sums25(const Real* f, double rho0, double tref, double& n, double& jx,
                                       double& jy, double& e) {
  double cs[5], rs[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    cs[i] = 0.0;
    rs[i] = 0.0;
  }
#pragma unroll
  for (int ky = 0; ky < 5; ++ky)
#pragma unroll
    for (int kx = 0; kx < 5; ++kx) {
      const double v = (double)f[5 * ky + kx];
      cs[kx] += v;
      rs[ky] += v;
    }
  n = (cs[0] + cs[4]) + (cs[1] + cs[3]) + cs[2];
  jx = R4 * (cs[4] - cs[0]) + R3 * (cs[3] - cs[1]);
  jy = R4 * (rs[4] - rs[0]) + R3 * (rs[3] - rs[1]);
  e = (R4 * R4) * ((cs[0] + cs[4]) + (rs[0] + rs[4])) + (R3 * R3) * ((cs[1] + cs[3]) + (rs[1] + rs[3]));
  if (std::is_same<Real, float>::value) {
    n += rho0;
    e += 2.0 * rho0 * tref;
  }
}

// f^eq of one node, stored form (FP64: f^eq; FP32: f^eq minus the base, as
//   w_x w_y [dn (1 + hx)(1 + hy) + rho0 ((hx - h0x)(1 + hy) + (1 + h0x)(hy - h0y))],
// every term small near the base state).
template <typename Real>
__device__ __forceinline__ void feq25(double n, double ux, double uy, double T, double rho0, double tref,
                                      Real out[25]) {
  double hx[5], hy[5], h0[5];
  hfac(ux, T - 1.0, hx);
  hfac(uy, T - 1.0, hy);
  base_h0(tref, h0);
#pragma unroll
  for (int ky = 0; ky < 5; ++ky)
#pragma unroll
    for (int kx = 0; kx < 5; ++kx) {
      const double w = Wk[kx] * Wk[ky];
      if (std::is_same<Real, float>::value) {
        const double dn = n - rho0;
        out[5 * ky + kx] = (Real)(w * (dn * (1.0 + hx[kx]) * (1.0 + hy[ky]) +
                                      rho0 * ((hx[kx] - h0[kx]) * (1.0 + hy[ky]) +
                                              (1.0 + h0[kx]) * (hy[ky] - h0[ky]))));
      } else {
        out[5 * ky + kx] = (Real)(n * (Wk[kx] * (1.0 + hx[kx])) * (Wk[ky] * (1.0 + hy[ky])));
      }
    }
}

__device__ __forceinline__ double delta_p(double n, double T, double a, double b) {
  // Delta p = p^i - p^w = nT - [nT/(1 - bn) - a n^2]
  const double nT = n * T;
  return nT - nT / (1.0 - b * n) + a * n * n;
}

// Running moment sums n = sum f, j = sum p f, e = sum |p|^2 f of a node's
// populations, which must arrive in population order (k = 0..24, row by row
// of the 5 x 5 set).  The velocity rows share p_y, so a row's values are
// first added up (r) and n, j_y and the p_y^2 part of e take r once per row;
// j_x and the p_x^2 part of e take each value with p_x != 0.  That is 72 FP64
// operations per node instead of 100.  The stage kernel accumulates the sums
// as it produces each population, and the set-up kernels use the same sequence
// so that a restart is bitwise identical.
struct MomSum {
  double n = 0.0, jx = 0.0, jy = 0.0, e = 0.0, r = 0.0;
  __device__ __forceinline__ void add(int k, double v) {
    const int kx = k % 5, ky = k / 5;
    const double px = Rk[kx], py = Rk[ky];
    r = kx == 0 ? v : r + v;
    if (kx != 2) {
      jx += px * v;
      e += (px * px) * v;
    }
    if (kx == 4) {
      n += r;
      if (ky != 2) {
        jy += py * r;
        e += (py * py) * r;
      }
    }
  }
};

// (n, Delta p) of the carry from the running sums.
template <bool F32>
__device__ __forceinline__ void carry_finish(const MomSum& s, double rho0, double tref, double va,
                                             double vb, double& n_out, double& dp_out) {
  double n = s.n, jx = s.jx, jy = s.jy, e = s.e;
  if (F32) {
    n += rho0;
    e += 2.0 * rho0 * tref;
  }
  const double in = 1.0 / n;
  const double vx = jx * in, vy = jy * in;
  n_out = n;
  dp_out = delta_p(n, 0.5 * (e * in - vx * vx - vy * vy), va, vb);
}

// --------------------------------------------------------------------------
// stage kernel
// --------------------------------------------------------------------------

// LDS of one stage workgroup.
#ifndef OLB_GROUP64
#define OLB_GROUP64 1
#endif
#ifndef OLB_GROUP32
#define OLB_GROUP32 1
#endif
// populations per LDS barrier in the stage loop: one for both (FP64: two
// cost 6 registers and 2 %; FP32: with the first group reconstructed before
// the force, two push the stage past 80 registers and spill, -4 %)
template <typename Real>
constexpr int pop_group() { return std::is_same<Real, float>::value ? OLB_GROUP32 : OLB_GROUP64; }

// Wide layout (FP32 stage, 63 x 8 and 63 x 16 tiles, no specular x planes):
// the population planes sit side by side in LDS rows whose pitch is a
// multiple of 64 values (planes 128 values apart), so that the reads six rows
// apart of a y-face reconstruction take the 64-value offset unit of the
// paired LDS reads, and every read of every plane takes its offset from one
// of two base registers as an immediate (no address arithmetic per read).
// Otherwise planes one after another, rows of 69 values: the FP64 stage has
// no registers to spare for the two bases, and the FP32 specular-x and
// 63 x 12 variants would spill with them.
template <typename Real, int BY, bool XSPEC>
constexpr bool wide_lds() { return std::is_same<Real, float>::value && !XSPEC && BY != 12; }

template <typename Real, int BY, bool WIDE_>
struct StageLds {
  static constexpr bool WIDE = WIDE_;
  static constexpr int TW = 69;          // tile columns x0-3 .. x0+65
  static constexpr int TH = BY + 6;      // tile rows    y0-3 .. y0+BY+2
  static constexpr int TN = TW * TH;     // values per plane
  static constexpr int G = pop_group<Real>();
  static constexpr int PR = WIDE ? 2 * G * 128 : TW;   // row pitch of the planes
  static constexpr int PO = WIDE ? 128 : TN;           // offset from one plane to the next
  // 2G population planes
  __attribute__((aligned(16))) Real buf[WIDE ? TH * PR : 2 * G * TN];
  // the carried (n, Delta p) tile, apart from the planes: the first group of
  // populations is reconstructed while it is still on its way
  __attribute__((aligned(16))) double cm[2 * TN];
  // double-buffered rows of lower-face reconstructions, one per plane buffer
  // (row BY: the tile's top face)
  Real fy[2 * G][BY + 1][64];
  // x advection of the first group, parked while the force is computed
  Real ga[G][BY][64];
};

// One 64 x BY tile (origin x0, y0) of one RK stage.
#ifndef OLB_PREFETCH64
#define OLB_PREFETCH64 4
#endif
#ifndef OLB_PREFETCH32
#define OLB_PREFETCH32 3
#endif
// population planes in flight: plane ti is in LDS, ti + 1 .. ti + PREFETCH - 1
// are being loaded into registers (deeper gains nothing measurable; the FP32
// stage, bound by its VALU issue rate, keeps one slot fewer, which frees the
// registers it would otherwise spill)
// FP32 stage: ask for 6 waves per SIMD (three 8-wave workgroups per CU), a
// budget of 80 registers, 8 % faster than 5 waves.  FP64 needs ~128 registers
// (four waves per SIMD).
#ifndef OLB_WAVES32
#define OLB_WAVES32 6
#endif
#ifndef OLB_WAVES64
#define OLB_WAVES64 1
#endif
template <typename Real>
constexpr int min_waves_per_simd() { return std::is_same<Real, float>::value ? OLB_WAVES32 : OLB_WAVES64; }
template <typename Real>
constexpr int prefetch_depth() { return std::is_same<Real, float>::value ? OLB_PREFETCH32 : OLB_PREFETCH64; }

template <typename Real, int BY, bool WALLS, bool FN, bool XSPEC>
__device__ __forceinline__ void stage_tile(const StageArgs& a, const int x0, const int y0,
                                           StageLds<Real, BY, wide_lds<Real, BY, XSPEC>()>& sm) {
  constexpr bool F32 = std::is_same<Real, float>::value;
  using SL = StageLds<Real, BY, wide_lds<Real, BY, XSPEC>()>;
  constexpr int TW = SL::TW;
  constexpr int TH = SL::TH;
  constexpr int TN = SL::TN;
  constexpr int PO = SL::PO;
  constexpr int PR = SL::PR;
  constexpr int NT = 64 * BY;
  constexpr int SLOTS = (TN + NT - 1) / NT;
  Real* const pl0 = sm.buf;
  double* const mn = sm.cm;
  double* const mp = mn + TN;
  auto& fy_sh = sm.fy;
  const __attribute__((address_space(4))) float* const fbase =
      (const __attribute__((address_space(4))) float*)a.base;

  // one wave per tile row: make the row index a scalar so that branches on
  // it are uniform
  const int tx = threadIdx.x, ty = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int tid = ty * 64 + tx;
  const int nx = a.g.nx, ny = a.g.ny;
  const int64_t ps = a.g.ps;
  const int x = x0 + tx, y = y0 + ty;
  const bool active = (tx < TILE_X) && (x < nx) && (y < ny);

  // storage offsets of this thread's tile slots (same for every population)
  // XSPEC: specular planes at both ends of x (Sec. 3.4.1 across x): a halo
  // column past a plane holds the mirror column of the population with the
  // reversed x velocity (xfl), and the carried fields of the mirror column.
  // In a wall's ghost rows this reflects the wall ghosts once more (corners).
  int soff[SLOTS], moff[SLOTS];
  // LDS places of the slots in a plane (add the plane's offset)
  int lpo[SLOTS];
  bool xfl[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int i = tid + s * NT;
    const int ii = i < TN ? i : TN - 1;
    const int rr = ii / TW, cc = ii - rr * TW;
    lpo[s] = SL::WIDE ? rr * PR + cc : i;
    int gx;
    xfl[s] = false;
    if (XSPEC) {
      const int gr = x0 - 3 + cc;
      xfl[s] = gr < 0 || gr >= nx;
      gx = gr < 0 ? -1 - gr : (gr >= nx ? 2 * nx - 1 - gr : gr);
      gx = min(max(gx, 0), nx - 1);   // columns beyond the mirror band feed inactive threads only
    } else {
      gx = wrapi(x0 - 3 + cc, nx);
    }
    const int gy = y0 - 3 + rr;
    int sy, my;
    if (WALLS) {
      sy = min(max(gy, -3), ny + 2);
      my = gy < 0 ? -1 - gy : (gy >= ny ? 2 * ny - 1 - gy : gy);
      my = min(max(my, 0), ny - 1);
    } else {
      sy = wrapi(gy, ny);
      my = sy;
    }
    soff[s] = (sy + 3) * (int)a.g.rs + gx;
    moff[s] = my * nx + gx;
  }
  const int oy = WALLS ? min(y, ny + 2) : wrapi(y, ny);
  const int own = (oy + 3) * (int)a.g.rs + wrapi(x, nx);
  // byte offsets from a population's first element, for the buffer accesses
  constexpr int RB = (int)sizeof(Real);
  const uint32_t pbytes = (uint32_t)ps * RB, rbytes = (uint32_t)((ny + 5) * a.g.rs + nx) * RB;
  const uint32_t cbytes = (uint32_t)nx * (uint32_t)ny * 8u;
  int soffb[SLOTS], moffb[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    soffb[s] = soff[s] * RB;
    moffb[s] = moff[s] * 8;
  }
  const int ownb = own * RB;

  // Pointer views of the source array and the carried fields, for the
  // specular-x loads (the other accesses go through buffer resources).  No
  // __restrict__ anywhere: in the last RK stage f^n and f_dst are the same
  // array (each node's f^n is read before its f_dst is written, by the same
  // thread).
  const gmem<const Real>* src = as_global(reinterpret_cast<const Real*>(a.fsrc));
  const gmem<const Real>* fnp = as_global(reinterpret_cast<const Real*>(a.fn));
  gmem<Real>* dst = as_global(reinterpret_cast<Real*>(a.fdst));
  const gmem<const double>* cin = as_global(a.cin);
  gmem<double>* cout = as_global(a.cout);

  constexpr int G = pop_group<Real>();
  static_assert(12 % G == 0, "population 12 must start a group: the moment sums take the populations in order");
  constexpr int NB = 2 * G;
  constexpr int PF = prefetch_depth<Real>() - 1;
  static_assert(PF >= G, "the register ring must hold the next group");
  auto tile_pop = [](int t) { return t < 12 ? t : t + 1; };
  // storage offset of population k at tile slot s (mirrored populations past
  // specular x planes)
  auto pl_off = [&](int k, int s) -> int64_t {
    const int64_t o = (int64_t)k * ps + soff[s];
    if (!XSPEC) return o;
    return xfl[s] ? (int64_t)(5 * (k / 5) + 4 - k % 5) * ps + soff[s] : o;
  };
  // value of population k at tile slot s of the source array (specular x
  // planes pick the plane per lane: pointer form)
  auto ld_src = [&](int k, int s) -> Real {
    if constexpr (XSPEC) return src[pl_off(k, s)];
    else return bload<Real>(plane_rsrc(a.fsrc, k, pbytes, rbytes), soffb[s]);
  };
  // FN: the stage has an RK base term A f^n (A != 0); a template parameter so
  // that the load counts the waits below rely on are known at compile time
  constexpr bool use_fn = FN;
  // Loads are issued before anything waits, in the order they are needed
  // (memory reads complete in issue order): the first group of planes, the
  // carried fields of the tile, the register ring of the next planes.  The
  // first group is reconstructed while the carried fields are in flight; the
  // force stencils then wait for those alone.  (Slots past the tile read a
  // clamped, valid address.)
  Real pre0[G][SLOTS], pre[PF][SLOTS];
#pragma unroll
  for (int j = 0; j < G; ++j)
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) pre0[j][s] = ld_src(tile_pop(j), s);
  __builtin_amdgcn_sched_barrier(0);
  double cn_in[SLOTS], cp_in[SLOTS];
  {
    const int64_t N = (int64_t)nx * ny;
    const __amdgpu_buffer_rsrc_t rn = plane_rsrc(a.cin, 0, cbytes), rp = plane_rsrc(a.cin, 1, cbytes);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if constexpr (XSPEC) {
        cn_in[s] = cin[moff[s]];
        cp_in[s] = cin[N + moff[s]];
      } else {
        cn_in[s] = bload<double>(rn, moffb[s]);
        cp_in[s] = bload<double>(rp, moffb[s]);
      }
    }
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int t = G; t < G + PF; ++t)
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) pre[t % PF][s] = ld_src(tile_pop(t), s);
  // population 12 (p = 0 on both axes) needs no halo: read its own value
  const Real f12 = XSPEC ? src[12 * ps + own] : bload<Real>(plane_rsrc(a.fsrc, 12, pbytes, rbytes), ownb);

  auto plane = [&](int t) { return pl0 + (t % NB) * PO; };
#pragma unroll
  for (int j = 0; j < G; ++j)
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int i = tid + s * NT;
      if (i < TN) plane(j)[lpo[s]] = pre0[j][s];
    }
  __syncthreads();

  // x-face row values and y-face column values start at these places (wide
  // layout: held in registers as they are, so that every read of a plane
  // takes its offset as an immediate)
  int rowc = (ty + 3) * PR + tx;
  int colc = ty * PR + tx + 3;
  if (SL::WIDE) asm volatile("" : "+v"(rowc), "+v"(colc));
  const int ownc = rowc + 3;

  // one WENO-5 face value (FP64: with the denominator guard from the arguments)
  auto wrec = [&](Real v0, Real v1, Real v2, Real v3, Real v4) -> Real {
    if constexpr (F32) return weno_rec(v0, v1, v2, v3, v4);
    else return weno_rec(v0, v1, v2, v3, v4, a.wguard);
  };

  // WENO face reconstructions of population slot t from its plane: the left
  // x face (its right neighbour's arrives by a lane shift) and the lower y
  // face (published in fy_sh for the wave below); returns the x advection
  // difference, the lower-face value and the node's own value
  auto faces = [&](int t, Real& advx, Real& ryl, Real& fk) {
    const int k = tile_pop(t);
    const int kx = k % 5, ky = k / 5;
    const double px = Rk[kx], py = Rk[ky];
    const Real* const P = plane(t);
    // the tile's top face (the lower face of the row above it): wave t mod BY
    // takes it, so the extra reconstruction is spread over the waves; first,
    // and fenced off, so that none of this node's face values are live yet.
    // The wave doing it runs at raised issue priority until its own faces are
    // published: the other waves of the tile wait for it at the barrier.
    if (ky != 2 && ty == t % BY) {
      __builtin_amdgcn_s_setprio(2);
      __builtin_amdgcn_sched_barrier(0);
      const int ct = BY * PR + tx + 3;
      const Real d0 = P[ct], d1 = P[ct + PR], d2 = P[ct + 2 * PR], d3 = P[ct + 3 * PR],
                 d4 = P[ct + 4 * PR], d5 = P[ct + 5 * PR];
      fy_sh[t % NB][BY][tx] = py > 0.0 ? wrec(d0, d1, d2, d3, d4) : wrec(d5, d4, d3, d2, d1);
      __builtin_amdgcn_sched_barrier(0);
    }
    fk = P[ownc];
    Real rxl = 0;
    ryl = 0;
    if (kx != 2) {
      const Real c0 = P[rowc], c1 = P[rowc + 1], c2 = P[rowc + 2], c3 = P[rowc + 3],
                 c4 = P[rowc + 4], c5 = P[rowc + 5];
      rxl = px > 0.0 ? wrec(c0, c1, c2, c3, c4) : wrec(c5, c4, c3, c2, c1);
    }
    if (ky != 2) {
      const Real c0 = P[colc], c1 = P[colc + PR], c2 = P[colc + 2 * PR], c3 = P[colc + 3 * PR],
                 c4 = P[colc + 4 * PR], c5 = P[colc + 5 * PR];
      ryl = py > 0.0 ? wrec(c0, c1, c2, c3, c4) : wrec(c5, c4, c3, c2, c1);
      fy_sh[t % NB][ty][tx] = ryl;
    }
    if (ky != 2 && ty == t % BY) __builtin_amdgcn_s_setprio(0);
    const Real rxr = (kx != 2) ? lane_next(rxl) : (Real)0;
    advx = (kx != 2) ? (Real)px * (rxr - rxl) : (Real)0;
  };

  // the first group, before the force is known; its x advection waits in
  // LDS and its lower faces in fy_sh (registers are short here)
  Real fk0[G];
#pragma unroll
  for (int j = 0; j < G; ++j) {
    Real advx, ryl;
    faces(j, advx, ryl, fk0[j]);
    sm.ga[j][ty][tx] = advx;
  }
  // this node's f^n now (it would crowd the registers of the reconstructions
  // above); its latency still hides behind the force stencils
  __builtin_amdgcn_sched_barrier(0);
  Real fnv[25];
#pragma unroll
  for (int k = 0; k < 25; ++k)
    fnv[k] = !use_fn ? (Real)0 : XSPEC ? fnp[k * ps + own] : bload<Real>(plane_rsrc(a.fn, k, pbytes, rbytes), ownb);

  // stage the second group and refill the ring behind it
#pragma unroll
  for (int j = 0; j < G; ++j) {
    const int t = G + j;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int i = tid + s * NT;
      if (i < TN) plane(t)[lpo[s]] = pre[t % PF][s];
    }
    if (t + PF < 24) {
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) pre[t % PF][s] = ld_src(tile_pop(t + PF), s);
    }
  }
  // carried n and Delta p of f_src, tile + halo, into LDS
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int i = tid + s * NT;
    if (i < TN) {
      mn[i] = cn_in[s];
      mp[i] = cp_in[s];
    }
  }
  __syncthreads();

  // force F = (1/n) grad Delta p + sigma grad lap n (Eq. F_def), 7x7 stencils
  // of the carried fields, one column offset at a time (scheduling barriers
  // keep the compiler from issuing all ~100 LDS reads at once).
  double Fx, Fy;
  {
    const int ctx = tx < TILE_X ? tx : TILE_X - 1;
    const int c = (ty + 3) * TW + (ctx + 3);
    double gxs = 0.0, gys = 0.0, lxs = 0.0, lys = 0.0;
#pragma unroll
    for (int l = 1; l <= 3; ++l) {
#pragma unroll
      for (int m = -3; m <= 3; ++m) {
        const int am = m < 0 ? -m : m;
        if (GW[l][am] != 0.0) gxs += (l * GW[l][am]) * (mp[c + m * TW + l] - mp[c + m * TW - l]);
        if (GL[l - 1][am] != 0.0) lxs += GL[l - 1][am] * (mn[c + m * TW + l] - mn[c + m * TW - l]);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int m = -3; m <= 3; ++m) {
        const int am = m < 0 ? -m : m;
        if (GW[l][am] != 0.0) gys += (l * GW[l][am]) * (mp[c + l * TW + m] - mp[c - l * TW + m]);
        if (GL[l - 1][am] != 0.0) lys += GL[l - 1][am] * (mn[c + l * TW + m] - mn[c - l * TW + m]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    const double inv_nc = 1.0 / mn[c];
    Fx = gxs * a.inv_ds * inv_nc + a.sigma * (lxs * a.inv_ds3);
    Fy = gys * a.inv_ds * inv_nc + a.sigma * (lys * a.inv_ds3);
  }
  // materialise the force here (left alone, the compiler interleaves the
  // stencils with the population stream and runs out of registers)
  asm volatile("" : "+v"(Fx));
  asm volatile("" : "+v"(Fy));

  // Every population is streamed through LDS once.  As population k arrives,
  // its contributions to
  //   f_dst = A f^n + B (f + dt L),  L = -adv - F.(grad_p f) + (f^eq - f)/tau
  // that do not need f^eq are accumulated: B (1 - dt/tau) f_k and
  // -B dt adv_k into acc[k], and the force term (Eq. derf folded into M) is
  // scattered into the accumulators of the populations sharing its velocity
  // row (x-derivative) or column (y-derivative).  f^eq needs all 25
  // populations (their moments) and is added at the end.
  const double Bdt = a.B * a.dt;
  const Real cx = (Real)(-Bdt * Fx), cy = (Real)(-Bdt * Fy);
  const Real cb = (Real)(a.B * (1.0 - a.dt * a.inv_tau));
  const Real cadv = (Real)(-Bdt * a.inv_ds);
  const Real rA = (Real)a.A;
  Real acc[25];
#pragma unroll
  for (int k = 0; k < 25; ++k) acc[k] = use_fn ? rA * fnv[k] : (Real)0;
  // The 24 planes with a halo (population 12 has none) stream through LDS in
  // groups of G: while group g is used from buffers (t mod 2G), group g + 1 is
  // written into the other G buffers and later planes are in flight into
  // registers (ring of PF slots); one barrier per group.  Per population, the
  // contributions that do not need the upper face are accumulated before the
  // barrier, the y-advection after it.
  MomSum fsum;   // moments of f_src
  const Real tfac = cb;

  // everything of population k except its y-advection
  auto local_terms = [&](int k, Real fk) {
    const int kx = k % 5, ky = k / 5;
    fsum.add(k, (double)fk);
    acc[k] += tfac * fk;
    // the force term acts on the whole population: with FP32 storage the
    // base rho0 b_kx b_ky (a uniform value, read through the scalar cache)
    // is added back for it
    const Real ff = F32 ? fk + (Real)fbase[k] : fk;
    const Real tfx = cx * ff, tfy = cy * ff;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      acc[5 * ky + i] += (Real)MT.v[i][kx] * tfx;
      acc[5 * i + kx] += (Real)MT.v[i][ky] * tfy;
    }
  };

  // y-advection of group tg once the upper faces (written by the next wave)
  // are visible
  auto finish_y = [&](int tg, const Real* advx, const Real* ryl) {
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int t = tg + j, k = tile_pop(t);
      const int ky = k / 5;
      Real adv = advx[j];
      if (ky != 2) {
        const Real ryt = fy_sh[t % NB][ty + 1][tx];
        adv += (Real)Rk[ky] * (ryt - ryl[j]);
      }
      acc[k] += cadv * adv;
    }
  };

  // the first group, now that the force is known (its upper faces became
  // visible at the barrier before the stencils)
  {
    Real advx[G], ryl[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
      local_terms(tile_pop(j), fk0[j]);
      advx[j] = sm.ga[j][ty][tx];
      ryl[j] = tile_pop(j) / 5 != 2 ? fy_sh[j % NB][ty][tx] : (Real)0;
    }
    finish_y(0, advx, ryl);
  }

#pragma unroll
  for (int t0 = G; t0 < 24; t0 += G) {
    if (t0 == 12) local_terms(12, f12);   // population 12 keeps its place in the sums
    // stage the next group and refill the ring
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int t = t0 + G + j;
      if (t < 24) {
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
          const int i = tid + s * NT;
          if (i < TN) plane(t)[lpo[s]] = pre[t % PF][s];
        }
        if (t + PF < 24) {
#pragma unroll
          for (int s = 0; s < SLOTS; ++s) pre[t % PF][s] = ld_src(tile_pop(t + PF), s);
        }
      }
    }
    Real advx[G], ryl[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
      Real fk;
      faces(t0 + j, advx[j], ryl[j], fk);
      local_terms(tile_pop(t0 + j), fk);
    }
    __syncthreads();
    finish_y(t0, advx, ryl);
    // do the updates now: left alone, the compiler sinks them to the end of
    // the kernel and keeps every population's inputs live until then
#pragma unroll
    for (int i = 0; i < 25; ++i) asm volatile("" : "+v"(acc[i]));
    asm volatile("" : "+v"(fsum.n), "+v"(fsum.jx), "+v"(fsum.jy), "+v"(fsum.e), "+v"(fsum.r));
  }

  // moments of f_src, equilibrium (Eqs. feq, g_alpha), RK combine
  double sn = fsum.n, se = fsum.e;
  if (F32) {
    sn += a.rho0;
    se += 2.0 * a.rho0 * a.tref;
  }
  const double inv_n = 1.0 / sn;
  const double ux = fsum.jx * inv_n, uy = fsum.jy * inv_n;
  const double T = 0.5 * (se * inv_n - ux * ux - uy * uy);
  double hx[5], hy[5];
  hfac(ux, T - 1.0, hx);
  hfac(uy, T - 1.0, hy);
  const double cfe = Bdt * a.inv_tau;
  const double dn0 = sn - a.rho0;
  // FP32 storage: the equilibrium's departure from w rho0 (collision
  // arithmetic, FP32 like the rest of it) from the FP64 moments, in per-axis
  // factors with w rho0 taken out exactly and every term small (nothing
  // cancels):
  //   cfe w_x w_y [dn0 (1 + hx)(1 + hy) + rho0 ((1 + hx)(1 + hy) - (1 + h0x)(1 + h0y))]
  //     = [cfe w_x (dn0 (1 + hx) + rho0 (hx - h0x))] [w_y (1 + hy)]
  //       + [cfe rho0 w_x (1 + h0x)] [w_y (hy - h0y)]
  // (h0 = 0 for tref = 1), so each population takes two FMAs on top of its
  // accumulator.
  float px[5], qx[5], by[5], hy_w[5];
  if (F32) {
    const float cfef = (float)cfe, dn0f = (float)dn0, rho0f = (float)a.rho0;
    const float crf = (float)(cfe * a.rho0);
    // h0 = (theta / 2) He2 + (theta^2 / 8) He4 of the base, per index
    const double c2 = 0.5 * (a.tref - 1.0), c4 = 0.5 * c2 * c2;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const double h0 = c2 * HE.v[2][i] + c4 * HE.v[4][i];
      const float w = (float)Wk[i];
      const float hxi = (float)hx[i], dxi = (float)(hx[i] - h0), dyi = (float)(hy[i] - h0);
      px[i] = (cfef * w) * __builtin_fmaf(dn0f, 1.0f + hxi, rho0f * dxi);
      qx[i] = crf * (float)(Wk[i] * (1.0 + h0));
      by[i] = __builtin_fmaf(w, (float)hy[i], w);
      hy_w[i] = w * dyi;
    }
  }
  MomSum dsum;
#pragma unroll
  for (int k = 0; k < 25; ++k) {
    const int kx = k % 5, ky = k / 5;
    Real out;
    if (F32)
      out = (Real)__builtin_fmaf(px[kx], by[ky], __builtin_fmaf(qx[kx], hy_w[ky], (float)acc[k]));
    else
      out = acc[k] + (Real)(cfe * (sn * (Wk[kx] * (1.0 + hx[kx])) * (Wk[ky] * (1.0 + hy[ky]))));
    if (active) {
      if constexpr (XSPEC) dst[k * ps + own] = out;
      else bstore<Real>(out, plane_rsrc(a.fdst, k, pbytes, rbytes), ownb);
    }
    dsum.add(k, (double)out);
  }

  if (active) {
    double cn, cdp;
    carry_finish<F32>(dsum, a.rho0, a.tref, a.a, a.b, cn, cdp);
    const int64_t N = (int64_t)nx * ny;
    const int m = y * nx + x;
    if constexpr (XSPEC) {
      cout[m] = cn;
      cout[N + m] = cdp;
    } else {
      bstore<double>(cn, plane_rsrc(a.cout, 0, cbytes), m * 8);
      bstore<double>(cdp, plane_rsrc(a.cout, 1, cbytes), m * 8);
    }
    if (!(fabs(cn) < INFINITY)) a.flag[0] = 1;
  }
}

// First instance whose tiles include tile t (tile_base is ascending).
__device__ __forceinline__ int find_instance(const InstDesc* inst, int ninst, int t) {
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (inst[mid].tile_base <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Stage kernel: one launch over the tile queue of every instance of a batch,
// one tile per workgroup.  Consecutive workgroups are dispatched to different
// XCDs, so workgroup b takes tile (b mod 8) * ceil(T/8) + b / 8 (each XCD
// works through a contiguous run of the queue).  Within an instance tiles are
// numbered row by row inside strips of ba.strip tile columns (whole rows when
// 0): an XCD then runs vertically adjacent tiles close together in time, so
// the halo rows they share are still in its L2 (in row order a tile's lower
// neighbour starts about half a tile lifetime later and misses them).
template <typename Real, int BY, bool WALLS, bool FN, bool XSPEC>
__global__ void __launch_bounds__(64 * BY, min_waves_per_simd<Real>()) stage_kernel(const BatchArgs ba) {
  __shared__ StageLds<Real, BY, wide_lds<Real, BY, XSPEC>()> sm;
  const int bid = blockIdx.x;
  const int q8 = ba.total_tiles >> 3, r8 = ba.total_tiles & 7, xcd = bid & 7;
  const int t = xcd * q8 + (xcd < r8 ? xcd : r8) + (bid >> 3);
  // the instance index is uniform: keep it (and so the descriptor loads) scalar
  const int i = __builtin_amdgcn_readfirstlane(find_instance(ba.inst, ba.ninst, t));
  const InstDesc& d = ba.inst[i];
  StageArgs a;
  a.g = d.g;
  a.fsrc = d.f[ba.stage];
  a.fn = d.f[0];
  a.fdst = d.f[ba.stage == 2 ? 0 : ba.stage + 1];
  a.cin = d.carry[ba.cur];
  a.cout = d.carry[ba.cur ^ 1];
  a.flag = ba.flag;
  a.inv_ds = d.inv_ds;
  a.inv_ds3 = d.inv_ds3;
  a.dt = d.dt;
  a.inv_tau = d.inv_tau;
  a.a = d.a;
  a.b = d.b;
  a.sigma = d.sigma;
  a.A = ba.A;
  a.B = ba.B;
  a.rho0 = d.rho0;
  a.tref = d.tref;
  a.base = d.base;
  a.wguard = ba.wguard;
  const int local = t - d.tile_base;
  int tile_x, tile_y;
  if (ba.strip > 0 && ba.strip < d.tiles_x) {
    // strips of ba.strip tile columns (the last one may be narrower), rows
    // within a strip: tiles that start together share their halo rows and
    // columns while those are still in L2
    const int per = ba.strip * d.tiles_y;
    const int s = local / per;
    const int w = min(ba.strip, d.tiles_x - s * ba.strip);
    const int r = local - s * per;
    tile_y = r / w;
    tile_x = s * ba.strip + (r - tile_y * w);
  } else {
    tile_y = local / d.tiles_x;
    tile_x = local - tile_y * d.tiles_x;
  }
  stage_tile<Real, BY, WALLS, FN, XSPEC>(a, tile_x * TILE_X, tile_y * BY, sm);
}

// --------------------------------------------------------------------------
// diffuse-reflection ghosts (Sec. 3.4.2, walls across y)
// --------------------------------------------------------------------------

template <typename Real>
__global__ void walls_kernel(const WallBatchArgs wa) {
  constexpr bool F32 = std::is_same<Real, float>::value;
  // instance of this 64-column block (wall_block_base is ascending)
  int lo = 0, hi = wa.ninst - 1;
  const int blk = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wa.inst[mid].wall_block_base <= blk) lo = mid; else hi = mid - 1;
  }
  const InstDesc& d = wa.inst[lo];
  const int x = (blk - d.wall_block_base) * 64 + threadIdx.x;
  const int wall = blockIdx.y;  // 0: lower wall (y = -1/2), 1: upper wall
  const int nx = d.g.nx, ny = d.g.ny;
  if (x >= nx) return;
  Real* __restrict__ f = reinterpret_cast<Real*>(d.f[wa.stage]);
  const int64_t ps = d.g.ps, rs = d.g.rs;
  // storage rows: interior y -> y + 3
  const int r0 = wall ? ny + 2 : 3, r1 = wall ? ny + 1 : 4, r2 = wall ? ny : 5;
  const int g1 = wall ? ny + 3 : 2, g2 = wall ? ny + 4 : 1, g3 = wall ? ny + 5 : 0;
  const double Tw = wall ? d.tw[1] : d.tw[0];
  const double uw = wall ? d.uw[1] : d.uw[0];
  const double rho0 = d.rho0;
  // per-axis factors of the FP32 departure base
  double bw[5];
  {
    double h0[5];
    base_h0(d.tref, h0);
#pragma unroll
    for (int i = 0; i < 5; ++i) bw[i] = Wk[i] * (1.0 + h0[i]);
  }
  if (wall == 0 && d.g.walls == 2) {
    // specular symmetry plane (Sec. 3.4.1): ghost row -1 - j of population
    // (kx, ky) is interior row j of (kx, 4 - ky); the FP32 departure base is
    // even in p_y, so the departure values mirror the same way
#pragma unroll
    for (int k = 0; k < 25; ++k) {
      const int km = 5 * (4 - k / 5) + k % 5;
      const Real* src = f + km * ps + x;
      Real* pk = f + k * ps + x;
      pk[g1 * rs] = src[r0 * rs];
      pk[g2 * rs] = src[r1 * rs];
      pk[g3 * rs] = src[r2 * rs];
    }
    d.nw[x] = 0.0;
    return;
  }

  // populations travelling towards the wall (and p_y = 0): quadratic
  // extrapolation; their WENO flux through the wall face
  double out = 0.0;
#pragma unroll
  for (int ky = 0; ky < 5; ++ky) {
    const bool towards = wall ? (ky >= 2) : (ky <= 2);
    if (!towards) continue;
#pragma unroll
    for (int kx = 0; kx < 5; ++kx) {
      const int k = 5 * ky + kx;
      Real* pk = f + k * ps + x;
      const Real v0 = pk[r0 * rs], v1 = pk[r1 * rs], v2 = pk[r2 * rs];
      const Real e1 = (Real)3 * v0 - (Real)3 * v1 + v2;
      const Real e2 = (Real)6 * v0 - (Real)8 * v1 + (Real)3 * v2;
      const Real e3 = (Real)10 * v0 - (Real)15 * v1 + (Real)6 * v2;
      pk[g1 * rs] = e1;
      pk[g2 * rs] = e2;
      pk[g3 * rs] = e3;
      if (ky != 2) {
        // face between the adjacent interior row and the first ghost row;
        // upwind order (far interior ... ghost) is the same at both walls
        double rec = (double)weno_rec(v2, v1, v0, e1, e2);
        if (F32) rec += bw[kx] * bw[ky] * rho0;
        out += Rk[ky] * rec;
      }
    }
  }
  // Eq. nw: the denominator sums g_kx(u_w, T_w) g_ky(0, T_w) p_ky over the
  // wall-emitted velocities; sum_kx g_kx = 1 leaves sum_ky g_ky(0, T_w) p_ky.
  double hx[5], hy[5];
  hfac(uw, Tw - 1.0, hx);
  hfac(0.0, Tw - 1.0, hy);
  double den = 0.0;
#pragma unroll
  for (int ky = 0; ky < 5; ++ky) {
    const bool emitted = wall ? (ky < 2) : (ky > 2);
    if (emitted) den += Wk[ky] * (1.0 + hy[ky]) * Rk[ky];
  }
  const double nw = -out / den;
  d.nw[wall * nx + x] = nw;
#pragma unroll
  for (int ky = 0; ky < 5; ++ky) {
    const bool emitted = wall ? (ky < 2) : (ky > 2);
    if (!emitted) continue;
#pragma unroll
    for (int kx = 0; kx < 5; ++kx) {
      const int k = 5 * ky + kx;
      double v = nw * (Wk[kx] * (1.0 + hx[kx])) * (Wk[ky] * (1.0 + hy[ky]));
      if (F32) v -= bw[kx] * bw[ky] * rho0;
      Real* pk = f + k * ps + x;
      pk[g1 * rs] = (Real)v;
      pk[g2 * rs] = (Real)v;
      pk[g3 * rs] = (Real)v;
    }
  }
}

// --------------------------------------------------------------------------
// set-up and read-out
// --------------------------------------------------------------------------

template <typename Real>
__global__ void init_kernel(Geometry g, const double* __restrict__ fld, Real* __restrict__ f,
                            double* __restrict__ carry, double rho0, double tref, double va, double vb) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= g.nx) return;
  const int64_t N = (int64_t)g.nx * g.ny;
  const int m = y * g.nx + x;
  Real fe[25];
  feq25<Real>(fld[m], fld[N + m], fld[2 * N + m], fld[3 * N + m], rho0, tref, fe);
  const int own = (y + 3) * (int)g.rs + x;
  MomSum sum;
#pragma unroll
  for (int k = 0; k < 25; ++k) {
    f[k * g.ps + own] = fe[k];
    sum.add(k, (double)fe[k]);
  }
  carry_finish<std::is_same<Real, float>::value>(sum, rho0, tref, va, vb, carry[m], carry[N + m]);
}

template <typename Real>
__device__ __forceinline__ void load_own(const Geometry& g, const Real* f, int x, int y, Real v[25]) {
  const int own = (y + 3) * (int)g.rs + x;
#pragma unroll
  for (int k = 0; k < 25; ++k) v[k] = f[k * g.ps + own];
}

template <typename Real>
__global__ void moments_kernel(Geometry g, const Real* __restrict__ f, double* __restrict__ out,
                               double rho0, double tref) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= g.nx) return;
  Real v[25];
  load_own(g, f, x, y, v);
  double n, jx, jy, e;
  sums25<Real>(v, rho0, tref, n, jx, jy, e);
  const double in = 1.0 / n, ux = jx * in, uy = jy * in;
  const int64_t N = (int64_t)g.nx * g.ny;
  const int m = y * g.nx + x;
  out[m] = n;
  out[N + m] = ux;
  out[2 * N + m] = uy;
  out[3 * N + m] = 0.5 * (e * in - ux * ux - uy * uy);
}

template <typename Real>
__global__ void carry_kernel(Geometry g, const Real* __restrict__ f, double* __restrict__ carry,
                             double rho0, double tref, double va, double vb) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= g.nx) return;
  Real v[25];
  load_own(g, f, x, y, v);
  MomSum sum;
#pragma unroll
  for (int k = 0; k < 25; ++k) sum.add(k, (double)v[k]);
  const int64_t N = (int64_t)g.nx * g.ny;
  const int m = y * g.nx + x;
  carry_finish<std::is_same<Real, float>::value>(sum, rho0, tref, va, vb, carry[m], carry[N + m]);
}

template <typename Real>
__global__ void pack_kernel(Geometry g, const Real* __restrict__ f, double* __restrict__ out,
                            double rho0, double tref) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= g.nx) return;
  const int64_t N = (int64_t)g.nx * g.ny;
  const int own = (y + 3) * (int)g.rs + x, m = y * g.nx + x;
  double h0[5];
  base_h0(tref, h0);
#pragma unroll
  for (int k = 0; k < 25; ++k) {
    double v = (double)f[k * g.ps + own];
    if (std::is_same<Real, float>::value)
      v += (Wk[k % 5] * (1.0 + h0[k % 5])) * (Wk[k / 5] * (1.0 + h0[k / 5])) * rho0;
    out[k * N + m] = v;
  }
}

template <typename Real>
__global__ void unpack_kernel(Geometry g, const double* __restrict__ in, Real* __restrict__ f,
                              double rho0, double tref) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= g.nx) return;
  const int64_t N = (int64_t)g.nx * g.ny;
  const int own = (y + 3) * (int)g.rs + x, m = y * g.nx + x;
  double h0[5];
  base_h0(tref, h0);
#pragma unroll
  for (int k = 0; k < 25; ++k) {
    double v = in[k * N + m];
    if (std::is_same<Real, float>::value)
      v -= (Wk[k % 5] * (1.0 + h0[k % 5])) * (Wk[k / 5] * (1.0 + h0[k / 5])) * rho0;
    f[k * g.ps + own] = (Real)v;
  }
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------

template <typename Real, int BY, bool XSPEC>
static hipError_t stage_by(const BatchArgs& a, bool walls, int grid, hipStream_t s) {
  dim3 block(64, BY);
  const bool fn = a.A != 0.0;
  if (walls && fn)
    hipLaunchKernelGGL((stage_kernel<Real, BY, true, true, XSPEC>), dim3(grid), block, 0, s, a);
  else if (walls)
    hipLaunchKernelGGL((stage_kernel<Real, BY, true, false, XSPEC>), dim3(grid), block, 0, s, a);
  else if (fn)
    hipLaunchKernelGGL((stage_kernel<Real, BY, false, true, XSPEC>), dim3(grid), block, 0, s, a);
  else
    hipLaunchKernelGGL((stage_kernel<Real, BY, false, false, XSPEC>), dim3(grid), block, 0, s, a);
  return hipGetLastError();
}

template <typename Real, int BY>
static hipError_t stage_x(const BatchArgs& a, bool walls, bool xspec, int grid, hipStream_t s) {
  return xspec ? stage_by<Real, BY, true>(a, walls, grid, s) : stage_by<Real, BY, false>(a, walls, grid, s);
}

hipError_t launch_stage(const BatchArgs& a, int real_bytes, int by, bool walls, bool xspec, hipStream_t s) {
  const int grid = a.total_tiles;
  if (grid < 1) return hipErrorInvalidValue;
  if (real_bytes == 8) {
    if (by == 16) return stage_x<double, 16>(a, walls, xspec, grid, s);
    if (by == 8) return stage_x<double, 8>(a, walls, xspec, grid, s);
  } else {
    if (by == 16) return stage_x<float, 16>(a, walls, xspec, grid, s);
    if (by == 12) return stage_x<float, 12>(a, walls, xspec, grid, s);
    if (by == 8) return stage_x<float, 8>(a, walls, xspec, grid, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_walls(const WallBatchArgs& a, int real_bytes, int wall_blocks, hipStream_t s) {
  dim3 block(64), grid(wall_blocks, 2);
  if (real_bytes == 8)
    hipLaunchKernelGGL(walls_kernel<double>, grid, block, 0, s, a);
  else
    hipLaunchKernelGGL(walls_kernel<float>, grid, block, 0, s, a);
  return hipGetLastError();
}

static dim3 cell_grid(const Geometry& g) { return dim3((g.nx + 63) / 64, g.ny); }

// bad = 1 if any node of device fields [4][ny][nx] is outside the model's
// domain (non-finite, n outside (0, 1/b), T <= 0)
__global__ void check_fields_kernel(Geometry g, const double* __restrict__ fld, double b, int* __restrict__ bad) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= g.nx) return;
  const size_t N = (size_t)g.nx * g.ny, m = (size_t)y * g.nx + x;
  const double n = fld[m], ux = fld[N + m], uy = fld[2 * N + m], T = fld[3 * N + m];
  const bool ok = isfinite(n) && isfinite(ux) && isfinite(uy) && isfinite(T) && n > 0.0 &&
                  (b <= 0.0 || n * b < 1.0) && T > 0.0;
  if (!ok) *bad = 1;
}

hipError_t launch_check_fields(const Geometry& g, const double* fields, double b, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(check_fields_kernel, cell_grid(g), dim3(64), 0, s, g, fields, b, bad);
  return hipGetLastError();
}

hipError_t launch_init(const Geometry& g, const double* fields, void* f, double* carry,
                       double rho0, double tref, double va, double vb, int real_bytes, hipStream_t s) {
  if (real_bytes == 8)
    hipLaunchKernelGGL(init_kernel<double>, cell_grid(g), dim3(64), 0, s, g, fields,
                       (double*)f, carry, rho0, tref, va, vb);
  else
    hipLaunchKernelGGL(init_kernel<float>, cell_grid(g), dim3(64), 0, s, g, fields,
                       (float*)f, carry, rho0, tref, va, vb);
  return hipGetLastError();
}

hipError_t launch_moments(const Geometry& g, const void* f, double* out, double rho0, double tref,
                          int real_bytes, hipStream_t s) {
  if (real_bytes == 8)
    hipLaunchKernelGGL(moments_kernel<double>, cell_grid(g), dim3(64), 0, s, g,
                       (const double*)f, out, rho0, tref);
  else
    hipLaunchKernelGGL(moments_kernel<float>, cell_grid(g), dim3(64), 0, s, g,
                       (const float*)f, out, rho0, tref);
  return hipGetLastError();
}

hipError_t launch_carry(const Geometry& g, const void* f, double* carry, double rho0, double tref,
                        double va, double vb, int real_bytes, hipStream_t s) {
  if (real_bytes == 8)
    hipLaunchKernelGGL(carry_kernel<double>, cell_grid(g), dim3(64), 0, s, g,
                       (const double*)f, carry, rho0, tref, va, vb);
  else
    hipLaunchKernelGGL(carry_kernel<float>, cell_grid(g), dim3(64), 0, s, g,
                       (const float*)f, carry, rho0, tref, va, vb);
  return hipGetLastError();
}

hipError_t launch_pack(const Geometry& g, const void* f, double* out, double rho0, double tref,
                       int real_bytes, hipStream_t s) {
  if (real_bytes == 8)
    hipLaunchKernelGGL(pack_kernel<double>, cell_grid(g), dim3(64), 0, s, g, (const double*)f,
                       out, rho0, tref);
  else
    hipLaunchKernelGGL(pack_kernel<float>, cell_grid(g), dim3(64), 0, s, g, (const float*)f,
                       out, rho0, tref);
  return hipGetLastError();
}

hipError_t launch_unpack(const Geometry& g, const double* in, void* f, double rho0, double tref,
                         int real_bytes, hipStream_t s) {
  if (real_bytes == 8)
    hipLaunchKernelGGL(unpack_kernel<double>, cell_grid(g), dim3(64), 0, s, g, in, (double*)f,
                       rho0, tref);
  else
    hipLaunchKernelGGL(unpack_kernel<float>, cell_grid(g), dim3(64), 0, s, g, in, (float*)f,
                       rho0, tref);
  return hipGetLastError();
}

}  // namespace olbk
