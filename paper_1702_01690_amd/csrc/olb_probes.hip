// olb_probes -- measurement probes for the roofline of the stage kernels on
// gfx950.  A standalone program (not part of the library); each mode prints
// one JSON line per measurement.
//
//   olb_probes issue     issue cost of single VALU instruction forms (wave64,
//                        register operands, 8 waves per SIMD, 8 independent
//                        chains per wave): which forms the SIMD dual-issues
//   olb_probes pattern   the stage kernel's memory traffic with its arithmetic
//                        removed, on the 2048 x 2048 FP64 lattice: 63 x 8
//                        tiles, the 69 x 14 region of every population through
//                        a double-buffered LDS plane with one barrier per
//                        population, the carried fields, f^n at the tile's own
//                        nodes, one store per node and population; in the
//                        library's storage order (25 planes) and tile order
//                        (XCD-contiguous runs, strips of 8 tile columns), in
//                        whole-row tile order, and with rows of the 25
//                        populations interleaved; workgroups that march up
//                        2, 4 or 8 tiles of a column and keep the 6 rows that
//                        consecutive tiles share in LDS; a plain device copy
//   olb_probes stream    the HBM ceilings a streaming kernel reaches: copy,
//                        read-only and write-only streams over 2 GiB buffers
//                        with 16-byte accesses, over several grid sizes; the
//                        last line gives the best of each
//   olb_probes all       issue and pattern
//
// Every access of the pattern kernels stays inside the arrays it addresses
// (periodic wrap of rows and columns; buffer resources sized to the array).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

#define CK(x)                                                                    \
  do {                                                                           \
    hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess) {                                                      \
      std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                              \
    }                                                                            \
  } while (0)

namespace {

// ---------------------------------------------------------------------------
// issue costs
// ---------------------------------------------------------------------------

constexpr int CHAINS = 8;

// One wave64 instruction per chain step; a step of chain j reads chains j+1
// (and j+2, j+3), so every chain depends on the others and nothing folds.
#define P_OP2(INS) asm volatile(INS " %0, %1, %2" : "=v"(a[j]) : "v"(a[(j + 1) & 7]), "v"(a[(j + 2) & 7]))
#define P_OP1(INS) asm volatile(INS " %0, %1" : "=v"(a[j]) : "v"(a[(j + 1) & 7]))

template <int FORM>
__global__ void __launch_bounds__(512) issue_kernel(float* out, int iters, float sv) {
  float a[CHAINS];
#pragma unroll
  for (int j = 0; j < CHAINS; ++j) a[j] = (float)(threadIdx.x + j) * 1e-3f + 1.0f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < CHAINS; ++j) {
        if constexpr (FORM == 0) P_OP2("v_mul_f32");
        if constexpr (FORM == 1) asm volatile("v_fma_f32 %0, %1, %2, -%3" : "=v"(a[j]) : "v"(a[(j + 1) & 7]), "v"(a[(j + 2) & 7]), "v"(a[(j + 3) & 7]));
        if constexpr (FORM == 2) asm volatile("v_fmamk_f32 %0, %1, 0x40400000, %2" : "=v"(a[j]) : "v"(a[(j + 1) & 7]), "v"(a[(j + 2) & 7]));
        if constexpr (FORM == 3) asm volatile("v_mul_f32 %0, %1, %2" : "=v"(a[j]) : "s"(sv), "v"(a[(j + 2) & 7]));
        if constexpr (FORM == 4) asm volatile("v_fma_f32 %0, %1, %2, -%3" : "=v"(a[j]) : "v"(a[(j + 1) & 7]), "s"(sv), "v"(a[(j + 3) & 7]));
        if constexpr (FORM == 5) P_OP2("v_add_u32");
        if constexpr (FORM == 6) asm volatile("v_and_b32 %0, 0x7f800000, %1" : "=v"(a[j]) : "v"(a[(j + 1) & 7]));
        if constexpr (FORM == 7) P_OP1("v_mov_b32");
        if constexpr (FORM == 8) P_OP2("v_ldexp_f32");
        if constexpr (FORM == 9) P_OP1("v_frexp_exp_i32_f32");
        if constexpr (FORM == 10) P_OP2("v_max_f32");
        if constexpr (FORM == 11) asm volatile("v_max3_f32 %0, %1, %2, %3" : "=v"(a[j]) : "v"(a[(j + 1) & 7]), "v"(a[(j + 2) & 7]), "v"(a[(j + 3) & 7]));
        if constexpr (FORM == 12) asm volatile("v_sub_f32_dpp %0, %1, %2 row_shr:1 row_mask:0xf bank_mask:0xf" : "=v"(a[j]) : "v"(a[(j + 1) & 7]), "v"(a[(j + 2) & 7]));
        if constexpr (FORM == 13) P_OP1("v_cvt_f32_i32");
        if constexpr (FORM == 14) P_OP1("v_rcp_f32");
      }
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < CHAINS; ++j) s += a[j];
  out[blockIdx.x * 512 + threadIdx.x] = s;
}

// FP64 chains (the FP64 forms take 64-bit register pairs)
template <int FORM>
__global__ void __launch_bounds__(512) issue_kernel64(double* out, int iters) {
  double a[CHAINS];
#pragma unroll
  for (int j = 0; j < CHAINS; ++j) a[j] = (double)(threadIdx.x + j) * 1e-3 + 1.0;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < CHAINS; ++j) {
        if constexpr (FORM == 0) asm volatile("v_fma_f64 %0, %1, %2, %3" : "=v"(a[j]) : "v"(a[(j + 1) & 7]), "v"(a[(j + 2) & 7]), "v"(a[(j + 3) & 7]));
        if constexpr (FORM == 1) asm volatile("v_add_f64 %0, %1, %2" : "=v"(a[j]) : "v"(a[(j + 1) & 7]), "v"(a[(j + 2) & 7]));
      }
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < CHAINS; ++j) s += a[j];
  out[blockIdx.x * 512 + threadIdx.x] = s;
}

template <typename L>
float time_ms(L launch, int reps) {
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  launch();
  CK(hipGetLastError());
  CK(hipDeviceSynchronize());
  CK(hipEventRecord(e0));
  for (int r = 0; r < reps; ++r) launch();
  CK(hipEventRecord(e1));
  CK(hipEventSynchronize(e1));
  float ms = 0.0f;
  CK(hipEventElapsedTime(&ms, e0, e1));
  CK(hipEventDestroy(e0));
  CK(hipEventDestroy(e1));
  return ms / reps;
}

void run_issue() {
  // 256 CUs x 4 SIMDs x 8 waves: one full round of 512-thread workgroups
  const int blocks = 256 * 4;
  const int iters = 2000;
  void* out = nullptr;
  CK(hipMalloc(&out, (size_t)blocks * 512 * 8));
  const double insts = blocks * 8.0 * iters * 4 * CHAINS;  // wave64 instructions
  auto rep = [&](const char* form, float ms) {
    // cycles per wave64 instruction per SIMD at the 2.4 GHz peak clock
    std::printf("{\"probe\":\"issue\",\"form\":\"%s\",\"ms\":%.4f,\"cycles_per_inst_at_2.4GHz\":%.3f}\n", form, ms,
                ms * 1e-3 * 1024 * 2.4e9 / insts);
    std::fflush(stdout);
  };
  float* f = static_cast<float*>(out);
  double* d = static_cast<double*>(out);
#define ISSUE(F, NAME) rep(NAME, time_ms([&] { issue_kernel<F><<<blocks, 512>>>(f, iters, 1.0001f); }, 5))
  ISSUE(0, "v_mul_f32 v, v");
  ISSUE(1, "v_fma_f32 v, v, -v");
  ISSUE(2, "v_fmamk_f32 v, literal, v");
  ISSUE(3, "v_mul_f32 s, v");
  ISSUE(4, "v_fma_f32 v, s, -v");
  ISSUE(5, "v_add_u32 v, v");
  ISSUE(6, "v_and_b32 literal, v");
  ISSUE(7, "v_mov_b32 v");
  ISSUE(8, "v_ldexp_f32 v, v");
  ISSUE(9, "v_frexp_exp_i32_f32 v");
  ISSUE(10, "v_max_f32 v, v");
  ISSUE(11, "v_max3_f32 v, v, v");
  ISSUE(12, "v_sub_f32_dpp row_shr:1");
  ISSUE(13, "v_cvt_f32_i32 v");
  ISSUE(14, "v_rcp_f32 v");
#undef ISSUE
  rep("v_fma_f64 v, v, v", time_ms([&] { issue_kernel64<0><<<blocks, 512>>>(d, iters); }, 5));
  rep("v_add_f64 v, v", time_ms([&] { issue_kernel64<1><<<blocks, 512>>>(d, iters); }, 5));
  CK(hipFree(out));
}

// ---------------------------------------------------------------------------
// memory pattern of the stage kernel
// ---------------------------------------------------------------------------

constexpr int NX = 2048, NY = 2048;
constexpr int TILE_X = 63, BY = 8;
constexpr int TW = 69, TH = BY + 6, TN = TW * TH, NT = 64 * BY;
constexpr int SLOTS = (TN + NT - 1) / NT;
constexpr int TILES_X = (NX + TILE_X - 1) / TILE_X;
constexpr int TILES_Y = NY / BY;
constexpr int TILES = TILES_X * TILES_Y;
constexpr long long ROWS = NY + 6;                 // 3 ghost rows each side
constexpr long long ARRAY = 25 * ROWS * NX;        // elements per distribution array
constexpr int PF = 3;                              // planes in flight

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void st(double v, __amdgpu_buffer_rsrc_t r, int off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}
__device__ __forceinline__ int wrap(int v, int n) {
  const int r = v % n;
  return r < 0 ? r + n : r;
}

// ROWS_INTERLEAVED: element (k, row, x) at (row * 25 + k) * NX + x instead of
// (k * ROWS + row) * NX + x.  strip: tile columns per strip (>= TILES_X: rows).
template <bool FN, bool ROWS_INTERLEAVED>
__global__ void __launch_bounds__(NT) pattern_kernel(const double* src, const double* fn, double* dst,
                                                     const double* cin, double* cout, int strip) {
  constexpr long long KS = ROWS_INTERLEAVED ? NX : ROWS * NX;   // population stride
  constexpr int RS = ROWS_INTERLEAVED ? 25 * NX : NX;          // row stride
  __shared__ double plane[2][TN];
  // XCD-contiguous runs of the tile queue, as the stage kernel
  const int b = blockIdx.x;
  const int t = (b & 7) * (TILES / 8) + (b >> 3);
  const int per = strip * TILES_Y;
  const int s = t / per;
  const int w = min(strip, TILES_X - s * strip);
  const int r = t - s * per;
  const int tile_y = r / w, tile_x = s * strip + (r - tile_y * w);
  const int x0 = tile_x * TILE_X, y0 = tile_y * BY;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 64 + tx;
  const bool active = tx < TILE_X && x0 + tx < NX;
  int foff[SLOTS], coff[SLOTS];
#pragma unroll
  for (int q = 0; q < SLOTS; ++q) {
    const int i = min(tid + q * NT, TN - 1);
    const int rr = i / TW, cc = i - rr * TW;
    const int gx = wrap(x0 - 3 + cc, NX), gy = wrap(y0 - 3 + rr, NY);
    foff[q] = ((gy + 3) * RS + gx) * 8;
    coff[q] = (gy * NX + gx) * 8;
  }
  const int xo = wrap(x0 + tx, NX), yo = y0 + ty;
  const int own = ((yo + 3) * RS + xo) * 8, ownc = (yo * NX + xo) * 8;
  // one resource per population: base at the population's first element,
  // records to the end of the array
  auto pop = [&](const double* a, int k) { return rsrc(a + k * KS, (unsigned)((ARRAY - k * KS) * 8)); };
  const unsigned cbytes = (unsigned)NX * NY * 8u;
  double acc = 0.0;
  {
    const auto rn = rsrc(cin, cbytes), rp = rsrc(cin + (long long)NX * NY, cbytes);
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) acc += ld(rn, coff[q]) + ld(rp, coff[q]);
  }
  double ring[PF][SLOTS];
#pragma unroll
  for (int k = 0; k < PF; ++k)
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) ring[k][q] = ld(pop(src, k), foff[q]);
  double fnv[25];
#pragma unroll
  for (int k = 0; k < 25; ++k) fnv[k] = FN ? ld(pop(fn, k), own) : 0.0;
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < 25; ++k) {
    double* pl = plane[k & 1];
#pragma unroll
    for (int q = 0; q < SLOTS; ++q)
      if (tid + q * NT < TN) pl[tid + q * NT] = ring[k % PF][q];
    if (k + PF < 25) {
#pragma unroll
      for (int q = 0; q < SLOTS; ++q) ring[k % PF][q] = ld(pop(src, k + PF), foff[q]);
    }
    __syncthreads();
    // the node, its left neighbour and the rows 3 below and 3 above
    const double v = pl[(ty + 3) * TW + tx + 3] + pl[(ty + 3) * TW + tx] + pl[ty * TW + tx + 3] +
                     pl[(ty + 6) * TW + tx + 3];
    sum += v;
    if (active) st(v + fnv[k] + (k == 0 ? acc : 0.0), pop(dst, k), own);
  }
  if (active) {
    st(sum, rsrc(cout, cbytes), ownc);
    st(0.5 * sum, rsrc(cout + (long long)NX * NY, cbytes), ownc);
  }
}

// Marching: a workgroup takes MT vertically adjacent tiles of one tile column
// in turn; per population it keeps the 6 rows the next tile shares (rows BY ..
// BY + 5 of the region) in LDS and loads only the other BY rows of the next
// region.  25 x 6 x 69 values of LDS (83 KB): one workgroup per CU.
template <bool FN, int MT>
__global__ void __launch_bounds__(NT) march_kernel(const double* src, const double* fn, double* dst,
                                                   const double* cin, double* cout) {
  constexpr int GY = TILES_Y / MT;                   // tile groups per column
  constexpr int GROUPS = TILES_X * GY;
  constexpr int NEW = TW * BY;                       // region values loaded after the first tile
  extern __shared__ double lds[];
  double* plane = lds;                               // [2][TN]
  double* keep = lds + 2 * TN;                       // [25][6 * TW]
  const int b = blockIdx.x;
  const int g = (b & 7) * (GROUPS / 8) + (b >> 3);
  const int per = 8 * GY;                            // strips of 8 tile columns, as the library
  const int s = g / per;
  const int w = min(8, TILES_X - s * 8);
  const int r = g - s * per;
  const int gy = r / w, tile_x = s * 8 + (r - gy * w);
  const int x0 = tile_x * TILE_X;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 64 + tx;
  const bool active = tx < TILE_X && x0 + tx < NX;
  const unsigned pbytes = (unsigned)(ROWS * NX * 8), cbytes = (unsigned)NX * NY * 8u;
  auto pop = [&](const double* a, int k) { return rsrc(a + k * ROWS * NX, pbytes); };
  for (int j = 0; j < MT; ++j) {
    const int y0 = (gy * MT + j) * BY;
    const int first = j == 0 ? 0 : 6 * TW;           // region index of the first value loaded
    const int count = j == 0 ? TN : NEW;
    int foff[SLOTS], coff[SLOTS], slot[SLOTS];
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
      const int i = tid + q * NT;
      const int ri = first + min(i, count - 1);
      const int rr = ri / TW, cc = ri - rr * TW;
      foff[q] = ((wrap(y0 - 3 + rr, NY) + 3) * NX + wrap(x0 - 3 + cc, NX)) * 8;
      slot[q] = i < count ? ri : -1;
      const int ci = min(i, TN - 1), cr = ci / TW, ccc = ci - cr * TW;
      coff[q] = (wrap(y0 - 3 + cr, NY) * NX + wrap(x0 - 3 + ccc, NX)) * 8;
    }
    const int xo = wrap(x0 + tx, NX), yo = y0 + ty;
    const int own = ((yo + 3) * NX + xo) * 8, ownc = (yo * NX + xo) * 8;
    double acc = 0.0;
    {
      const auto rn = rsrc(cin, cbytes), rp = rsrc(cin + (long long)NX * NY, cbytes);
#pragma unroll
      for (int q = 0; q < SLOTS; ++q) acc += ld(rn, coff[q]) + ld(rp, coff[q]);
    }
    double ring[PF][SLOTS];
#pragma unroll
    for (int k = 0; k < PF; ++k)
#pragma unroll
      for (int q = 0; q < SLOTS; ++q) ring[k][q] = ld(pop(src, k), foff[q]);
    double fnv[25];
#pragma unroll
    for (int k = 0; k < 25; ++k) fnv[k] = FN ? ld(pop(fn, k), own) : 0.0;
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < 25; ++k) {
      double* pl = plane + (k & 1) * TN;
      double* kp = keep + k * 6 * TW;
#pragma unroll
      for (int q = 0; q < SLOTS; ++q)
        if (slot[q] >= 0) pl[slot[q]] = ring[k % PF][q];
      if (j > 0)
        for (int i = tid; i < 6 * TW; i += NT) pl[i] = kp[i];
      if (k + PF < 25) {
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) ring[k % PF][q] = ld(pop(src, k + PF), foff[q]);
      }
      __syncthreads();
      const double v = pl[(ty + 3) * TW + tx + 3] + pl[(ty + 3) * TW + tx] + pl[ty * TW + tx + 3] +
                       pl[(ty + 6) * TW + tx + 3];
      // rows BY .. BY + 5 for the next tile: read after this barrier, and kp is
      // next read (for population k of the next tile) after further barriers
      if (j + 1 < MT)
        for (int i = tid; i < 6 * TW; i += NT) kp[i] = pl[BY * TW + i];
      sum += v;
      if (active) st(v + fnv[k] + (k == 0 ? acc : 0.0), pop(dst, k), own);
    }
    if (active) {
      st(sum, rsrc(cout, cbytes), ownc);
      st(0.5 * sum, rsrc(cout + (long long)NX * NY, cbytes), ownc);
    }
    __syncthreads();
  }
}

__global__ void copy_kernel(const double* __restrict__ a, double* __restrict__ b, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    b[i] = a[i];
}

void run_pattern() {
  const size_t bytes = (size_t)ARRAY * 8;
  double *f0, *f1, *f2, *c0, *c1;
  CK(hipMalloc(&f0, bytes));
  CK(hipMalloc(&f1, bytes));
  CK(hipMalloc(&f2, bytes));
  CK(hipMalloc(&c0, (size_t)2 * NX * NY * 8));
  CK(hipMalloc(&c1, (size_t)2 * NX * NY * 8));
  CK(hipMemset(f0, 0, bytes));
  CK(hipMemset(f1, 0, bytes));
  CK(hipMemset(c0, 0, (size_t)2 * NX * NY * 8));
  const int reps = 20;
  const double nodes = (double)NX * NY;
  {
    const float ms = time_ms([&] { copy_kernel<<<8192, 256>>>(f0, f2, ARRAY); }, reps);
    std::printf("{\"probe\":\"pattern\",\"kernel\":\"copy\",\"bytes\":%.6g,\"ms\":%.4f,\"GBps\":%.1f}\n", 2.0 * bytes, ms,
                2.0 * bytes / ms / 1e6);
    std::fflush(stdout);
  }
  auto rep = [&](const char* order, const char* layout, bool fn, float ms) {
    // algorithmic bytes of the stage launch this mirrors: 25 values read (and
    // 25 more of f^n in stages 2 and 3) and 25 written per node, 8 bytes each
    const double alg = nodes * (fn ? 600.0 : 400.0);
    std::printf("{\"probe\":\"pattern\",\"kernel\":\"%s\",\"order\":\"%s\",\"layout\":\"%s\",\"ms\":%.4f,"
                "\"alg_GBps\":%.1f,\"frac_of_8TBps\":%.4f}\n",
                fn ? "stage 2/3 (f^n)" : "stage 1", order, layout, ms, alg / ms / 1e6, alg / ms / 1e6 / 8000.0);
    std::fflush(stdout);
  };
  const dim3 blk(64, BY);
  for (int strip : {8, TILES_X}) {
    const char* order = strip == 8 ? "strips of 8 tile columns" : "rows of tiles";
    rep(order, "planes", false, time_ms([&] { pattern_kernel<false, false><<<TILES, blk>>>(f0, f1, f2, c0, c1, strip); }, reps));
    rep(order, "planes", true, time_ms([&] { pattern_kernel<true, false><<<TILES, blk>>>(f0, f1, f2, c0, c1, strip); }, reps));
    rep(order, "rows interleaved", false, time_ms([&] { pattern_kernel<false, true><<<TILES, blk>>>(f0, f1, f2, c0, c1, strip); }, reps));
    rep(order, "rows interleaved", true, time_ms([&] { pattern_kernel<true, true><<<TILES, blk>>>(f0, f1, f2, c0, c1, strip); }, reps));
  }
  const size_t lds = (size_t)(2 * TN + 25 * 6 * TW) * 8;
  auto marching = [&](auto kern, int mt, bool fn) {
    CK(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    char order[64];
    std::snprintf(order, sizeof order, "strips of 8, marching %d tiles", mt);
    rep(order, "planes", fn, time_ms([&] { kern<<<TILES / mt, blk, lds>>>(f0, f1, f2, c0, c1); }, reps));
  };
  marching(march_kernel<false, 2>, 2, false);
  marching(march_kernel<true, 2>, 2, true);
  marching(march_kernel<false, 4>, 4, false);
  marching(march_kernel<true, 4>, 4, true);
  marching(march_kernel<false, 8>, 8, false);
  marching(march_kernel<true, 8>, 8, true);
  CK(hipFree(f0));
  CK(hipFree(f1));
  CK(hipFree(f2));
  CK(hipFree(c0));
  CK(hipFree(c1));
}

// ---------------------------------------------------------------------------
// HBM streaming ceilings
// ---------------------------------------------------------------------------

typedef float f32x4 __attribute__((ext_vector_type(4)));

// grid-stride streams of 16-byte elements, U per thread and iteration (all
// loads of an iteration issued before its stores); NT: non-temporal hints
template <int U, bool NT>
__global__ void __launch_bounds__(256) stream_copy(const f32x4* __restrict__ a, f32x4* __restrict__ b, long long n) {
  const long long step = (long long)gridDim.x * 256 * U;
  for (long long i = (long long)blockIdx.x * 256 * U + threadIdx.x; i < n; i += step) {
    f32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long j = i + (long long)u * 256;
      if (j < n) v[u] = NT ? __builtin_nontemporal_load(a + j) : a[j];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long j = i + (long long)u * 256;
      if (j < n) {
        if (NT)
          __builtin_nontemporal_store(v[u], b + j);
        else
          b[j] = v[u];
      }
    }
  }
}
template <int U>
__global__ void __launch_bounds__(256) stream_read(const f32x4* __restrict__ a, float* __restrict__ out, long long n) {
  const long long step = (long long)gridDim.x * 256 * U;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (long long i = (long long)blockIdx.x * 256 * U + threadIdx.x; i < n; i += step) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long j = i + (long long)u * 256;
      if (j < n) acc += a[j];
    }
  }
  // the buffer holds zeros: the store never happens, but the loads are kept
  const float t = acc[0] + acc[1] + acc[2] + acc[3];
  if (t != 0.f) out[threadIdx.x] = t;
}
template <int U>
__global__ void __launch_bounds__(256) stream_write(f32x4* __restrict__ b, long long n) {
  const long long step = (long long)gridDim.x * 256 * U;
  for (long long i = (long long)blockIdx.x * 256 * U + threadIdx.x; i < n; i += step) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long j = i + (long long)u * 256;
      if (j < n) b[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  }
}

void run_stream() {
  const long long bytes = 1LL << 31;
  const long long n = bytes / 16;
  f32x4 *a, *b;
  float* out;
  CK(hipMalloc(&a, bytes));
  CK(hipMalloc(&b, bytes));
  CK(hipMalloc(&out, 256 * sizeof(float)));
  CK(hipMemset(a, 0, bytes));
  CK(hipMemset(b, 0, bytes));
  const int reps = 10;
  double best_copy = 0, best_read = 0, best_write = 0;
  auto rep = [&](const char* kind, int blocks, double moved, float ms, double& best) {
    const double gbps = moved / ms / 1e6;
    best = gbps > best ? gbps : best;
    std::printf("{\"probe\":\"stream\",\"kind\":\"%s\",\"blocks\":%d,\"GBps\":%.1f}\n", kind, blocks, gbps);
    std::fflush(stdout);
  };
  for (int blocks : {4096, 8192, 16384}) {
    rep("copy, non-temporal", blocks, 2.0 * bytes,
        time_ms([&] { stream_copy<4, true><<<blocks, 256>>>(a, b, n); }, reps), best_copy);
    rep("copy", blocks, 2.0 * bytes, time_ms([&] { stream_copy<4, false><<<blocks, 256>>>(a, b, n); }, reps),
        best_copy);
    rep("read", blocks, 1.0 * bytes, time_ms([&] { stream_read<8><<<blocks, 256>>>(a, out, n); }, reps), best_read);
    rep("write", blocks, 1.0 * bytes, time_ms([&] { stream_write<8><<<blocks, 256>>>(b, n); }, reps), best_write);
  }
  std::printf("{\"probe\":\"stream\",\"best\":{\"copy_GBps\":%.1f,\"read_GBps\":%.1f,\"write_GBps\":%.1f}}\n",
              best_copy, best_read, best_write);
  CK(hipFree(a));
  CK(hipFree(b));
  CK(hipFree(out));
}

}  // namespace

int main(int argc, char** argv) {
  const char* mode = argc > 1 ? argv[1] : "all";
  const bool all = std::strcmp(mode, "all") == 0;
  if (!all && std::strcmp(mode, "issue") != 0 && std::strcmp(mode, "pattern") != 0 &&
      std::strcmp(mode, "stream") != 0) {
    std::fprintf(stderr, "usage: olb_probes [issue|pattern|stream|all]\n");
    return 2;
  }
  if (all || std::strcmp(mode, "issue") == 0) run_issue();
  if (all || std::strcmp(mode, "pattern") == 0) run_pattern();
  if (std::strcmp(mode, "stream") == 0) run_stream();
  return 0;
}
