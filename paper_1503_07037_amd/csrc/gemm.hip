// Matrix-core (MFMA) products of the DMPT recursion on gfx950.
//
// Every product on the recursion path (Sec. II: D^2, the cross terms of the
// perturbation jets, the right-hand sides of Algorithm 1's per-step systems
// and the system-matrix products inside the linear solves) has the form
//
//     C = alpha * X * Y^T + beta1 * C1 + beta2 * C2,   Y symmetric in use,
//
// with X and Y stored row major, so both operands are read along contiguous
// rows (k is the fast index of both).  Solves are run on transposed
// unknowns (U = Y^T solves U T' = R^T with T' = T'^T), which keeps the
// non-symmetric iterate on the X side; every Y operand on the path (D, S^(k),
// T' factors) is symmetric, so X * Y^T = X * Y.
//
// Engines:
//   F64     v_mfma_f64_16x16x4f64, FP64 accumulation
//   F32     v_mfma_f32_32x32x2f32 on operands rounded to FP32; FP32 sums over
//           16-wide k slices, FP64 across slices
//   BF16S2  x = x_hi + x_lo (BF16 splits): x_hi y_hi + x_hi y_lo + x_lo y_hi
//   BF16S3  x = x_0 + x_1 + x_2: the six products x_p y_q with p + q <= 2
//           (both BF16 engines use v_mfma_f32_32x32x16_bf16, FP32 accumulation)
//   I8S4    x = q_x (d_0 + d_1 / 254 + d_2 / 254^2 + d_3 / 254^3), one q per
//           matrix, int8 digits (q8_off): the thirteen products d_p e_q
//           with p + q <= 4 on v_mfma_i32_32x32x32_i8, summed exactly in
//           int32 (one accumulator per weight p + q), combined in FP64 at the
//           end
//   I8S3    the same slices, digits 0-2 only: the six products with p + q <= 2
// Master copies (the operands of the FP64 and FP32 engines, C1, C2, W and C)
// are FP64 for every engine.
//
// FP64 and FP32: 128 x 128 output tile per 512-thread workgroup (eight waves,
// 64 x 32 each, two per SIMD), K staged through LDS in a two-stage ring.  Split BF16: 256 x
// 256 tiles (128 x 128 per wave) when Np allows, else 128 x 128; the BF16
// planes are stored in a blocked layout in the MFMA operand order (see
// plane_off), so operand tiles move as contiguous 1 KB blocks.  Operands are
// zero-padded to a multiple of 128 so no edge handling is needed.  The block
// index is remapped so that the tiles of one XCD form a contiguous,
// row-grouped range (better reuse of that XCD's L2).
#include "dmpt_internal.h"

namespace dmpt {
namespace {

typedef double d4v __attribute__((__vector_size__(4 * sizeof(double))));
typedef float f16v __attribute__((__vector_size__(16 * sizeof(float))));
typedef __bf16 bf8v __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef unsigned int u4v __attribute__((__vector_size__(4 * sizeof(unsigned int))));

constexpr int BM = 128, BN = 128;
constexpr int kWaves256 = 8;  // waves of the 256 x 256 split-BF16 kernel (two per SIMD)
constexpr int kGroupM = 8;   // tile rows per raster group
constexpr int kXcd = 8;      // XCDs of an MI355X
constexpr int kDiagParts = 4;  // row parts per diagonal tile in the summing kernel of split products

// Tile coordinates of a (possibly remapped) linear block index.
__device__ inline void raster(int b, int tiles_m, int tiles_n, int& tm, int& tn) {
  const int T = tiles_m * tiles_n;
  if (T % kXcd == 0) b = (b % kXcd) * (T / kXcd) + b / kXcd;
  const int per_group = kGroupM * tiles_n;
  const int g = b / per_group;
  const int first = g * kGroupM;
  const int gsz = min(tiles_m - first, kGroupM);
  const int r = b % per_group;
  tm = first + r % gsz;
  tn = r / gsz;
}

// With sym, only the tiles on and below the diagonal of the square T x T
// tile grid (T even): rows p and T - 1 - p hold p + 1 and T - p of them,
// T + 1 together, so the triangle is the (T / 2) x (T + 1) grid folded at
// q = p (gemm_launch_tiles gives the launch size).
__device__ inline void tile_coords(int b, int tiles_m, int tiles_n, int& tm, int& tn, int sym = 0) {
  if (!sym) {
    raster(b, tiles_m, tiles_n, tm, tn);
    return;
  }
  const int T = tiles_m;
  int p, q;
  raster(b, T / 2, T + 1, p, q);
  if (q <= p) {
    tm = p;
    tn = q;
  } else {
    tm = T - 1 - p;
    tn = q - p - 1;
  }
}

__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  }
  return s;
}

// Round-to-nearest-even FP32 -> BF16 bits.
__device__ inline uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Write the BF16 slices of v to planes[0..np-1] at offset idx: slice p is
// the BF16 rounding of what the slices before it left over (the remainder is
// exact in FP64, so three slices keep about 24 bits of v).
__device__ inline void write_split(double v, uint16_t* const* pl, int np, int64_t idx) {
  double r = v;
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    if (p < np) {
      const uint16_t h = bf16_rne((float)r);
      pl[p][idx] = h;
      r -= (double)bf16_to_f(h);
    }
  }
}

// Epilogue for output element (row, col): master at row * Np + col, BF16
// planes (when requested) in the plane layout.
template <class T>
__device__ inline double epi(const GemmArgs& a, int z, int64_t row, int64_t col, double acc,
                             double& dsum) {
  const int64_t off = row * a.Np + col;
  double v = a.alpha * acc;
  if (a.C1) v += a.beta1 * (double)((const T*)a.C1)[z * a.sC1 + off];
  if (a.C2) v += a.beta2 * (double)((const T*)a.C2)[z * a.sC2 + off];
  const T out = (T)v;
  ((T*)a.C)[z * a.sC + off] = out;
  if (a.Cpl[0]) {
    uint16_t* pl[3] = {a.Cpl[0] ? a.Cpl[0] + z * a.sC : nullptr,
                       a.Cpl[1] ? a.Cpl[1] + z * a.sC : nullptr,
                       a.Cpl[2] ? a.Cpl[2] + z * a.sC : nullptr};
    write_split((double)out, pl, a.Cpl[2] ? 3 : (a.Cpl[1] ? 2 : 1), plane_off(row, col, a.Np));
  }
  if (a.W) dsum += (double)((const T*)a.W)[z * a.sW + off] * (double)out;
  return (double)out;
}

__device__ inline double block_max(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s = fmax(s, red[i]);
  }
  return s;
}

// One thread per running member adds the member's work to the tally.
__device__ inline void count_member(const GemmArgs& a, int bx) {
  if (a.tally && bx == 0 && threadIdx.x == 0) {
    atomicAdd(a.tally, a.tally_m);
    atomicAdd(a.tally + 1, a.tally_u);
  }
}

// ------------------------------------------------------------------ FP64
// 128 x 128 output tile, NW waves (two along m, NW / 2 along n; wave (wm, wn)
// owns 64 x (256 / NW) as 16 x 16 MFMA tiles), k staged through a two-stage
// LDS ring of BK-wide slices.
#ifndef DMPT_F64_BK
#define DMPT_F64_BK 8
#endif
#ifndef DMPT_F64_NW
#define DMPT_F64_NW 8
#endif
constexpr int kF64BK = DMPT_F64_BK, kF64NW = DMPT_F64_NW;

template <int BK, int NW>
__device__ __forceinline__ void gemm_f64_tile(const GemmArgs& a, int z, int bx, int nbx) {
  constexpr int LD = BK + 1;
  constexpr int FN = 16 / NW;                  // 16-wide MFMA tiles per wave along n
  constexpr int THREADS = NW * 64;
  constexpr int Q = BK / 2;                    // double2 per row and stage
  constexpr int L = BM * Q / THREADS;          // double2 loads per thread, operand and stage
  static_assert(L >= 1 && FN >= 1, "tile split");
  if (a.active && !a.active[z]) return;
  count_member(a, bx);
  const int64_t Np = a.Np;
  int tm, tn;
  tile_coords(bx, (int)(Np / BM), (int)(Np / BN), tm, tn, a.sym);
  const double* X = (const double*)a.X.m + (z / a.X.div) * a.X.stride + (int64_t)tm * BM * Np;
  const double* Y = (const double*)a.Y.m + (z / a.Y.div) * a.Y.stride + (int64_t)tn * BN * Np;
  __shared__ double sX[2][BM][LD];
  __shared__ double sY[2][BN][LD];
  __shared__ double red[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / (NW / 2), wn = wave % (NW / 2);
  double2 rx[L], ry[L];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const int idx = tid + i * THREADS, row = idx / Q, q = idx % Q;
      rx[i] = *(const double2*)(X + (int64_t)row * Np + k0 + 2 * q);
      ry[i] = *(const double2*)(Y + (int64_t)row * Np + k0 + 2 * q);
    }
  };
  auto swrite = [&](int buf) {
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const int idx = tid + i * THREADS, row = idx / Q, q = idx % Q;
      sX[buf][row][2 * q] = rx[i].x;
      sX[buf][row][2 * q + 1] = rx[i].y;
      sY[buf][row][2 * q] = ry[i].x;
      sY[buf][row][2 * q + 1] = ry[i].y;
    }
  };
  d4v acc[4][FN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = (d4v){0.0, 0.0, 0.0, 0.0};
  gload(0);
  swrite(0);
  __syncthreads();
  const int nk = (int)(Np / BK);
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double av[4], bv[FN];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = sX[buf][wm * 64 + i * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < FN; ++j) bv[j] = sY[buf][wn * (16 * FN) + j * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) swrite(buf ^ 1);
    __syncthreads();
  }
  double dsum = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // v_mfma_f64_16x16x4f64 result: register r of lane l holds row 4r + l/16, column l%16
        const int64_t row = (int64_t)tm * BM + wm * 64 + i * 16 + 4 * r + (lane >> 4);
        const int64_t col = (int64_t)tn * BN + wn * (16 * FN) + j * 16 + (lane & 15);
        epi<double>(a, z, row, col, acc[i][j][r], dsum);
      }
  if (a.W) {
    const double s = block_sum(dsum, red);
    if (tid == 0) a.partials[(int64_t)z * nbx + bx] = s;
  }
}

template <int BK, int NW>
__global__ __launch_bounds__(NW * 64) void k_gemm_f64(GemmArgs a) {
  gemm_f64_tile<BK, NW>(a, blockIdx.z, blockIdx.x, gridDim.x);
}

// Grouped launch: the blocks of nprob products (members x tiles each, in
// order) in one grid; block b belongs to the problem p with start[p] <= b < start[p + 1].
template <int BK, int NW>
__global__ __launch_bounds__(NW * 64) void k_gemm_f64_grouped(const GemmArgs* __restrict__ list,
                                                               const int* __restrict__ start, int nprob) {
  int p = 0;
  const int b = blockIdx.x;
  while (p + 1 < nprob && b >= start[p + 1]) ++p;
  const GemmArgs& a = list[p];
  const int tiles = (int)((a.Np / BM) * (a.Np / BN));
  const int local = b - start[p];
  gemm_f64_tile<BK, NW>(a, local / tiles, local % tiles, tiles);
}

// ------------------------------------------------------------------ FP32
// Operands are the FP64 masters, rounded to FP32 as a stage is written to
// LDS (BK-wide k stages, two-stage ring).  The MFMAs of each 16-wide slice of
// k accumulate into a fresh FP32 tile which is then added into an FP64
// accumulator, so the FP32 rounding covers 16 products per output instead of
// all of k.  Two FP32 tiles alternate between slices: while the MFMAs of
// slice s fill one, the other (slice s - 1) is converted and added into
// FP64, four values after each of the slice's first MFMAs, so that VALU work
// runs beside the matrix core.  NW waves: two along m, NW / 2 along n; wave
// (wm, wn) owns 64 x (256 / NW).
#ifndef DMPT_F32_BK
#define DMPT_F32_BK 32
#endif
#ifndef DMPT_F32_NW
#define DMPT_F32_NW 8
#endif
constexpr int kF32BK = DMPT_F32_BK, kF32NW = DMPT_F32_NW;
constexpr int kF32Slice = 16;  // k extent of one FP32 partial sum

template <int BK, int NW>
__device__ __forceinline__ void gemm_f32_tile(const GemmArgs& a, int z, int bx, int nbx) {
  constexpr int LD = BK + 1;
  constexpr int FN = 8 / NW;                      // MFMA tiles per wave along n: 2 (NW 4), 1 (NW 8)
  constexpr int THREADS = NW * 64;
  constexpr int L = BM * BK / 2 / THREADS;        // double2 loads per thread, operand and stage
  constexpr int SL = BK / kF32Slice;              // FP32 slices per stage
  static_assert(FN >= 1 && L >= 1 && SL >= 1 && BK % kF32Slice == 0, "tile split");
  if (a.active && !a.active[z]) return;
  count_member(a, bx);
  const int64_t Np = a.Np;
  int tm, tn;
  tile_coords(bx, (int)(Np / BM), (int)(Np / BN), tm, tn, a.sym);
  const double* X = (const double*)a.X.m + (z / a.X.div) * a.X.stride + (int64_t)tm * BM * Np;
  const double* Y = (const double*)a.Y.m + (z / a.Y.div) * a.Y.stride + (int64_t)tn * BN * Np;
  __shared__ float sX[2][BM][LD];
  __shared__ float sY[2][BN][LD];
  __shared__ double red[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / (NW / 2), wn = wave % (NW / 2);
  constexpr int Q = BK / 2;  // double2 per row and stage
  double2 rx[L], ry[L];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const int idx = tid + i * THREADS, row = idx / Q, q = idx % Q;
      rx[i] = *(const double2*)(X + (int64_t)row * Np + k0 + 2 * q);
      ry[i] = *(const double2*)(Y + (int64_t)row * Np + k0 + 2 * q);
    }
  };
  auto swrite = [&](int buf) {
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const int idx = tid + i * THREADS, row = idx / Q, q = idx % Q;
      sX[buf][row][2 * q] = (float)rx[i].x;
      sX[buf][row][2 * q + 1] = (float)rx[i].y;
      sY[buf][row][2 * q] = (float)ry[i].x;
      sY[buf][row][2 * q + 1] = (float)ry[i].y;
    }
  };
  f16v acc[2][FN], acc2[2][FN];
  double accd[2][FN][16];
  f16v zero;
#pragma unroll
  for (int r = 0; r < 16; ++r) zero[r] = 0.0f;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      acc[i][j] = zero;
      acc2[i][j] = zero;
#pragma unroll
      for (int r = 0; r < 16; ++r) accd[i][j][r] = 0.0;
    }
  const int nk = (int)(Np / BK);
  gload(0);
  swrite(0);
  __syncthreads();
  constexpr int V = 2 * FN * 16;  // FP32 values per lane to fold
  static_assert(4 * (kF32Slice / 2) * 2 * FN >= V, "a slice must fold the whole previous tile");
  // One 16-wide slice of k from LDS buffer buf at column k0: MFMAs into a
  // fresh acur; when fold_prev, aprev (the previous slice) is added into FP64
  // meanwhile.
  auto slice = [&](int buf, int k0, f16v (&acur)[2][FN], f16v (&aprev)[2][FN], bool fold_prev) {
    int m = 0;  // MFMA index within the slice
#pragma unroll
    for (int kk = 0; kk < kF32Slice; kk += 2) {
      float av[2], bv[FN];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = sX[buf][wm * 64 + i * 32 + (lane & 31)][k0 + kk + (lane >> 5)];
#pragma unroll
      for (int j = 0; j < FN; ++j)
        bv[j] = sY[buf][wn * (32 * FN) + j * 32 + (lane & 31)][k0 + kk + (lane >> 5)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          acur[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], kk == 0 ? zero : acur[i][j], 0,
                                                            0, 0);
          if (fold_prev && 4 * m < V) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int v = 4 * m + q;
              accd[v / (16 * FN)][(v / 16) % FN][v % 16] += (double)aprev[v / (16 * FN)][(v / 16) % FN][v % 16];
            }
          }
          ++m;
        }
    }
  };
  // slices alternate between acc (even global slice index) and acc2 (odd)
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      const int gs = kt * SL + sl;  // global slice index
      if ((gs & 1) == 0) slice(buf, sl * kF32Slice, acc, acc2, gs > 0);
      else slice(buf, sl * kF32Slice, acc2, acc, true);
    }
    if (kt + 1 < nk) swrite(buf ^ 1);
    __syncthreads();
  }
  {
    // the last slice's tile
    f16v (&last)[2][FN] = ((nk * SL) & 1) ? acc : acc2;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) accd[i][j][r] += (double)last[i][j][r];
  }
  double dsum = 0.0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = (int64_t)tm * BM + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t col = (int64_t)tn * BN + wn * (32 * FN) + j * 32 + (lane & 31);
        epi<double>(a, z, row, col, accd[i][j][r], dsum);
      }
  if (a.W) {
    const double s = block_sum(dsum, red);
    if (tid == 0) a.partials[(int64_t)z * nbx + bx] = s;
  }
}

template <int BK, int NW>
__global__ __launch_bounds__(NW * 64) void k_gemm_f32(GemmArgs a) {
  gemm_f32_tile<BK, NW>(a, blockIdx.z, blockIdx.x, gridDim.x);
}

template <int BK, int NW>
__global__ __launch_bounds__(NW * 64) void k_gemm_f32_grouped(const GemmArgs* __restrict__ list,
                                                               const int* __restrict__ start, int nprob) {
  int p = 0;
  const int b = blockIdx.x;
  while (p + 1 < nprob && b >= start[p + 1]) ++p;
  const GemmArgs& a = list[p];
  const int tiles = (int)((a.Np / BM) * (a.Np / BN));
  const int local = b - start[p];
  gemm_f32_tile<BK, NW>(a, local / tiles, local % tiles, tiles);
}

// ------------------------------------------------------------------ split BF16
// One kernel for both split engines and both tile sizes:
//   S   planes per operand (2: three products, 3: six products)
//   TM  output tile edge of the workgroup (128 or 256)
//   BK  k extent of one pipeline stage (16 or 32)
//   NW  waves (4 or 8), two along m and NW/2 along n; wave (wm, wn) owns a
//       TM/2 x 2TM/NW block as MFMA tiles of 32 x 32.  With eight waves (two
//       per SIMD) one wave's MFMAs cover the other's LDS waits and barrier.
// Operands are read in the plane layout (1 KB blocks of 32 rows x 16 k, in
// the MFMA operand order): a stage of one operand plane is TM/32 x BK/16
// blocks, and lane l of a wave copies bytes 16 l .. 16 l + 15 of a block, so
// every global load instruction reads 1 KB contiguous and every LDS access
// of a wave is 1 KB contiguous (no bank conflicts, no swizzle).
// Pipeline over k: two LDS stages and one register stage.  While the MFMAs
// of stage k run, stage k + 1 (already in registers) is written to the other
// LDS buffer and the global loads of stage k + 2 are in flight.
// FL  1: the MFMAs of each stage accumulate into a fresh FP32 tile that is
//     then added to an FP64 accumulator (each FP32 sum covers BK of k, so
//     the FP32 rounding no longer grows with N).  Two FP32 tiles alternate
//     between stages: while the MFMAs of stage k fill one, the VALU adds the
//     other (stage k - 1) into FP64, a few values after each MFMA of the
//     first k block, so the conversions and FP64 adds run beside the matrix
//     core instead of after it.  0: one FP32 accumulator over all of k.
template <int S, int TM, int BK, int NW, int FL>
__device__ __forceinline__ void gemm_bf16_tile(const GemmArgs& a, int z, int bx, int nbx) {
  constexpr int WN = NW / 2;           // waves along n (two along m)
  constexpr int FM = TM / 64;          // MFMA tiles per wave along m
  constexpr int FN = TM / (32 * WN);   // MFMA tiles per wave along n
  constexpr int RB = TM / 32;          // 32-row blocks of an operand tile
  constexpr int KB = BK / 16;          // 16-wide k blocks of a stage
  constexpr int NBLK = RB * KB;        // blocks per operand plane and stage
  constexpr int SBLK = 2 * S * NBLK;   // blocks per stage: [operand][plane][row block][k block]
  constexpr int LOADS = SBLK / NW;     // blocks each wave copies per stage
  constexpr int SBYTES = SBLK * 1024;
  static_assert(SBLK % NW == 0, "a stage must split evenly over the waves");
  static_assert(FN >= 1, "at least one MFMA tile per wave along n");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ double red[NW];
  if (a.active && !a.active[z]) return;
  count_member(a, bx);
  const int64_t Np = a.Np;
  const int64_t kbr = Np >> 4;         // blocks per 32-row block row of a plane
  int tm, tn;
  tile_coords(bx, (int)(Np / TM), (int)(Np / TM), tm, tn, a.sym);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  // the blocks this wave copies: stage block q = wave + NW j
  const uint16_t* src[LOADS];
  int dst[LOADS];
#pragma unroll
  for (int j = 0; j < LOADS; ++j) {
    const int q = wave + NW * j;
    const int op = q / (S * NBLK), p = (q / NBLK) % S, b = q % NBLK;
    const int rb = b / KB, kb = b % KB;
    const uint16_t* base = op ? a.Y.pl[p] + (int64_t)(z / a.Y.div) * a.Y.stride
                              : a.X.pl[p] + (int64_t)(z / a.X.div) * a.X.stride;
    const int64_t brow = (int64_t)(op ? tn : tm) * RB + rb;
    src[j] = base + ((brow * kbr + kb) << 9) + lane * 8;
    dst[j] = q * 1024 + lane * 16;
  }
  u4v stg[LOADS];
  auto gload = [&](int kt) {
    const int64_t koff = (int64_t)kt * (KB << 9);
#pragma unroll
    for (int j = 0; j < LOADS; ++j) stg[j] = *(const u4v*)(src[j] + koff);
  };
  auto swrite = [&](int st) {
#pragma unroll
    for (int j = 0; j < LOADS; ++j) *(u4v*)(smem + st * SBYTES + dst[j]) = stg[j];
  };
  f16v acc[FM][FN], acc2[FM][FN];
  double accd[FL == 1 ? FM : 1][FL == 1 ? FN : 1][FL == 1 ? 16 : 1];
  f16v zero;
#pragma unroll
  for (int r = 0; r < 16; ++r) zero[r] = 0.0f;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
      acc[i][j] = zero;
  if constexpr (FL == 1) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) accd[i][j][r] = 0.0;
  }
  const int nk = (int)(Np / BK);
  gload(0);
  swrite(0);
  if (nk > 1) gload(1);
  __syncthreads();
  auto fold = [&](f16v (&ac)[FM][FN]) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) accd[i][j][r] += (double)ac[i][j][r];
  };
  // One stage: MFMAs into acur; with FL = 1 the other FP32 tile, filled by
  // the previous stage, is added into FP64 meanwhile (independent of the
  // MFMAs in flight, so the VALU work overlaps them).
  auto stage = [&](int kt, f16v (&acur)[FM][FN], f16v (&aprev)[FM][FN], bool fold_prev) {
    const unsigned char* sb = smem + (kt & 1) * SBYTES + lane * 16;
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
      // fragments in the order the MFMAs below consume them (X plane p with
      // Y plane S - 1 - p first), so the first products wait for two reads,
      // not for all of them
      bf8v xa[S][FM], yb[S][FN];
#pragma unroll
      for (int p = 0; p < S; ++p) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
          xa[p][i] = __builtin_bit_cast(
              bf8v, *(const u4v*)(sb + ((p * NBLK + (wm * FM + i) * KB + kk) << 10)));
        const int q = S - 1 - p;
#pragma unroll
        for (int j = 0; j < FN; ++j)
          yb[q][j] = __builtin_bit_cast(
              bf8v, *(const u4v*)(sb + (((S + q) * NBLK + (wn * FN + j) * KB + kk) << 10)));
        __builtin_amdgcn_sched_barrier(0);  // keep this order
      }
      if (kk == 0 && kt + 1 < nk) {
        swrite((kt + 1) & 1);
        if (kt + 2 < nk) gload(kt + 2);
      }
      // smallest terms first
      int m = 0;  // MFMA index within the k block
#pragma unroll
      for (int t = S - 1; t >= 0; --t)          // t = p + q
#pragma unroll
        for (int p = 0; p <= t; ++p)
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
              // FL: the stage's first product starts a fresh FP32 tile
              const bool fresh = FL == 1 && kk == 0 && t == S - 1 && p == 0;
              acur[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[p][i], yb[t - p][j],
                                                                   fresh ? zero : acur[i][j], 0, 0, 0);
              if constexpr (FL == 1) {
                // four values of the previous tile after each MFMA of the first k block
                constexpr int kFold = 4;
                static_assert(kFold * (S * (S + 1) / 2) >= 16, "the first k block must fold the whole tile");
                if (kk == 0 && fold_prev && m * kFold < FM * FN * 16) {
#pragma unroll
                  for (int q = 0; q < kFold; ++q) {
                    const int v = m * kFold + q;
                    const int fi = v / (16 * FN), fj = (v / 16) % FN, fr = v % 16;
                    accd[fi][fj][fr] += (double)aprev[fi][fj][fr];
                  }
                }
              }
              ++m;
            }
    }
    __syncthreads();
  };
  if constexpr (FL == 1) {
    for (int kt = 0; kt < nk; kt += 2) {
      stage(kt, acc, acc2, kt > 0);
      if (kt + 1 < nk) stage(kt + 1, acc2, acc, true);
    }
    fold((nk & 1) ? acc : acc2);  // the last stage's tile
  } else {
    for (int kt = 0; kt < nk; ++kt) stage(kt, acc, acc2, false);
  }
  double dsum = 0.0;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = (int64_t)tm * TM + wm * (TM / 2) + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t col = (int64_t)tn * TM + wn * (TM / WN) + j * 32 + (lane & 31);
        double v;
        if constexpr (FL == 1) v = accd[i][j][r];
        else v = (double)acc[i][j][r];
        epi<double>(a, z, row, col, v, dsum);
      }
  if (a.W) {
    const double s = block_sum(dsum, red);
    if (tid == 0) a.partials[(int64_t)z * nbx + bx] = s;
  }
}

template <int S, int TM, int BK, int NW, int FL>
__global__ __launch_bounds__(NW * 64) void k_gemm_bf16(GemmArgs a) {
  gemm_bf16_tile<S, TM, BK, NW, FL>(a, blockIdx.z, blockIdx.x, gridDim.x);
}

template <int S, int TM, int BK, int NW, int FL>
__global__ __launch_bounds__(NW * 64) void k_gemm_bf16_grouped(const GemmArgs* __restrict__ list,
                                                                const int* __restrict__ start, int nprob) {
  int p = 0;
  const int b = blockIdx.x;
  while (p + 1 < nprob && b >= start[p + 1]) ++p;
  const GemmArgs& a = list[p];
  const int tiles = (int)((a.Np / TM) * (a.Np / TM));
  const int local = b - start[p];
  gemm_bf16_tile<S, TM, BK, NW, FL>(a, local / tiles, local % tiles, tiles);
}

template <int S, int TM, int BK>
constexpr size_t bf16_lds() { return (size_t)2 * 2 * S * (TM / 32) * (BK / 16) * 1024; }

template <int S, int TM, int BK, int NW, int FL = 0>
hipError_t launch_bf16(const GemmArgs& a, dim3 grid, hipStream_t s) {
  const size_t lds = bf16_lds<S, TM, BK>();
  hipLaunchKernelGGL((k_gemm_bf16<S, TM, BK, NW, FL>), grid, dim3(NW * 64), lds, s, a);
  return hipGetLastError();
}

template <int S, int TM, int BK, int NW, int FL = 0>
hipError_t prepare_bf16() {
  hipError_t e = hipFuncSetAttribute((const void*)k_gemm_bf16<S, TM, BK, NW, FL>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bf16_lds<S, TM, BK>());
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_gemm_bf16_grouped<S, TM, BK, NW, FL>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bf16_lds<S, TM, BK>());
}

template <int S, int TM, int BK, int NW, int FL = 0>
hipError_t launch_bf16_grouped(const GemmArgs* list, const int* start, int nprob, int blocks, hipStream_t s) {
  const size_t lds = bf16_lds<S, TM, BK>();
  hipLaunchKernelGGL((k_gemm_bf16_grouped<S, TM, BK, NW, FL>), dim3(blocks), dim3(NW * 64), lds, s, list, start,
                     nprob);
  return hipGetLastError();
}

// ------------------------------------------------------------------ int8 slices
// 128 x 128 output tile, NW waves (WM along m, NW / WM along n; wave (wm, wn)
// owns (128 / WM) x (128 WM / NW) as 32 x 32 MFMA tiles), one int32
// accumulator tile per weight w = p + q of the digit products: SD = 4 digits
// read and weights 0 .. 4 (I8S4), or SD = 3 and weights 0 .. 2 (I8S3).  The operands move as 1 KB slice
// blocks in MFMA operand order (q8_off), through the same pipeline as the
// split-BF16 kernel: two LDS stages of BK of k and one register stage.  The
// int32 sums are exact over the whole inner dimension, so nothing is folded
// during the k loop; the epilogue evaluates
//   q_x q_y (A_0 + (A_1 + (A_2 + (A_3 + A_4 / 254) / 254) / 254) / 254)
// (or its first three terms) in FP64 (A_w: the weight-w accumulator).
typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i16v __attribute__((ext_vector_type(16)));

template <int BK, int NW, int WM, int SD>
__device__ __forceinline__ void gemm_i8_tile(const GemmArgs& a, int z, int bx, int nbx) {
  constexpr int TM = 128;
  constexpr int S = SD;               // digits read (of the kQ8Slices stored)
  constexpr int W = SD == 4 ? 5 : 3;  // weights kept: 0 .. 4 or 0 .. 2
  constexpr int WN = NW / WM;         // waves along n
  constexpr int FM = TM / (32 * WM);  // MFMA tiles per wave along m
  constexpr int FN = TM / (32 * WN);  // MFMA tiles per wave along n
  constexpr int RB = TM / 32;         // 32-row blocks of an operand tile
  constexpr int KB = BK / 32;         // 32-wide k blocks of a stage
  constexpr int NBLK = RB * KB;       // slice blocks per operand slice and stage
  constexpr int SBLK = 2 * S * NBLK;  // per stage: [operand][slice][row block][k block]
  constexpr int LOADS = SBLK / NW;
  constexpr int SBYTES = SBLK * 1024;
  static_assert(SBLK % NW == 0, "a stage must split evenly over the waves");
  static_assert(FN >= 1, "at least one MFMA tile per wave along n");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ double red[NW];
  if (a.active && !a.active[z]) return;
  count_member(a, bx);
  const int64_t Np = a.Np;
  const int64_t kbr = Np >> 5;  // 32-wide blocks per block row
  const int T = (int)(Np / TM);
  int nk = (int)(Np / BK);
  int tm, tn, split = -1, kfirst = 0, cslot = bx;
  if (a.sym == 2) {
    // the T dsplit blocks of the diagonal tiles first (diagonal tile tm,
    // k stages [split nk / dsplit, (split + 1) nk / dsplit)), then the strictly
    // lower triangle folded into (T / 2) x (T - 1); the maxima of the
    // diagonal tiles come from the summing kernel (kDiagParts per tile, slots
    // 0 .. T kDiagParts - 1)
    const int nd = T * a.dsplit;
    if (bx < nd) {
      tm = tn = bx / a.dsplit;
      split = bx % a.dsplit;
      kfirst = split * nk / a.dsplit;
      nk = (split + 1) * nk / a.dsplit - kfirst;
    } else {
      int p, q;
      raster(bx - nd, T / 2, T - 1, p, q);
      if (q < p) {
        tm = p;
        tn = q;
      } else {
        tm = T - 1 - p;
        tn = q - p;
      }
      cslot = T * kDiagParts + (bx - nd);
    }
  } else {
    tile_coords(bx, T, T, tm, tn, a.sym);
  }
  // all of these are the same for the whole block: keep them in scalar
  // registers (the vector registers hold the accumulators)
  tm = __builtin_amdgcn_readfirstlane(tm);
  tn = __builtin_amdgcn_readfirstlane(tn);
  split = __builtin_amdgcn_readfirstlane(split);
  kfirst = __builtin_amdgcn_readfirstlane(kfirst);
  nk = __builtin_amdgcn_readfirstlane(nk);
  cslot = __builtin_amdgcn_readfirstlane(cslot);
  // the wave index is uniform: block addresses live in scalar registers
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WN, wn = wave % WN;
  const int zx = z / a.X.div, zy = z / a.Y.div;
  const int8_t* xq = a.X.q8 + (int64_t)zx * a.X.stride * kQ8Slices;
  const int8_t* yq = a.Y.q8 + (int64_t)zy * a.Y.stride * kQ8Slices;
  const double scale = a.X.qs[a.X.stride ? zx : 0] * a.Y.qs[a.Y.stride ? zy : 0];
  const int8_t* src[LOADS];
  int dst[LOADS];
#pragma unroll
  for (int j = 0; j < LOADS; ++j) {
    const int q = wave + NW * j;
    const int op = q / (S * NBLK), sl = (q / NBLK) % S, b = q % NBLK;
    const int rb = b / KB, kb = b % KB;
    const int64_t brow = (int64_t)(op ? tn : tm) * RB + rb;
    src[j] = (op ? yq : xq) + (((brow * kbr + (int64_t)kfirst * KB + kb) * kQ8Slices + sl) << 10) + lane * 16;
    dst[j] = q * 1024 + lane * 16;
  }
  u4v stg[LOADS];
  auto gload = [&](int kt) {
    const int64_t koff = (int64_t)kt * KB * kQ8Slices * 1024;
#pragma unroll
    for (int j = 0; j < LOADS; ++j) stg[j] = *(const u4v*)(src[j] + koff);
  };
  auto swrite = [&](int st) {
#pragma unroll
    for (int j = 0; j < LOADS; ++j) *(u4v*)(smem + st * SBYTES + dst[j]) = stg[j];
  };
  i16v acc[W][FM][FN];
#pragma unroll
  for (int w = 0; w < W; ++w)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[w][i][j][r] = 0;
  gload(0);
  swrite(0);
  if (nk > 1) gload(1);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const unsigned char* sb = smem + (kt & 1) * SBYTES + lane * 16;
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
      // fragments in consumption order: X digit 0 and every Y digit first
      i4v xa[S][FM], yb[S][FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        xa[0][i] = __builtin_bit_cast(i4v, *(const u4v*)(sb + (((0 * NBLK) + (wm * FM + i) * KB + kk) << 10)));
#pragma unroll
      for (int q = 0; q < S; ++q)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          yb[q][j] = __builtin_bit_cast(
              i4v, *(const u4v*)(sb + ((((S + q) * NBLK) + (wn * FN + j) * KB + kk) << 10)));
#pragma unroll
      for (int p = 1; p < S; ++p)
#pragma unroll
        for (int i = 0; i < FM; ++i)
          xa[p][i] = __builtin_bit_cast(i4v, *(const u4v*)(sb + (((p * NBLK) + (wm * FM + i) * KB + kk) << 10)));
      if (kk == 0 && kt + 1 < nk) {
        swrite((kt + 1) & 1);
        if (kt + 2 < nk) gload(kt + 2);
      }
      // X digit p against Y digits q = 0 .. 4 - p: consecutive products go to
      // different accumulators
#pragma unroll
      for (int p = 0; p < S; ++p)
#pragma unroll
        for (int q = 0; q < S && p + q < W; ++q)
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[p + q][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[p][i], yb[q][j], acc[p + q][i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  const double rb = 1.0 / kQ8Base;
  // the epilogue's view of the arguments: a partial diagonal tile goes as it
  // is (alpha = 1, nothing added, no maxima) to rows 0 .. 127 of the strip
  // [member][split] of 128 x Np values in dpart, at its own columns
  GemmArgs e = a;
  if (split >= 0) {
    e.C = (void*)((uintptr_t)a.dpart + (uintptr_t)(((int64_t)split - (int64_t)tm) * TM * Np * (int64_t)sizeof(double)));
    e.sC = (int64_t)a.dsplit * TM * Np;
    e.alpha = 1.0;
    e.C1 = nullptr;
    e.C2 = nullptr;
    e.W = nullptr;
    e.cmax = nullptr;
    e.Cpl[0] = e.Cpl[1] = e.Cpl[2] = nullptr;
  }
  double dsum = 0.0;
  // largest |C| of the tile, rounded up to FP32: an upper bound, so the
  // digits of the slicing still fit (their scale is at most 2^-24 larger than
  // the exact maximum's), and one register instead of two keeps the epilogue
  // within the register budget
  float fmx = 0.0f;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = (int64_t)tm * TM + wm * (TM / WM) + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t col = (int64_t)tn * TM + wn * (TM / WN) + j * 32 + (lane & 31);
        double v = (double)acc[W - 1][i][j][r];
#pragma unroll
        for (int w = W - 2; w >= 0; --w) v = v * rb + (double)acc[w][i][j][r];
        {
          const double o = epi<double>(e, z, row, col, v * scale, dsum);
          fmx = o == o ? fmaxf(fmx, __double2float_ru(fabs(o))) : INFINITY;
        }
      }
  if (e.W) {
    const double s = block_sum(dsum, red);
    if (tid == 0) a.partials[(int64_t)z * nbx + bx] = s;
  }
  if (e.cmax) {
    const double m = block_max((double)fmx, red);
    if (tid == 0) a.cmax[(int64_t)z * a.cmax_stride + cslot] = m;
  }
}

// The same product with the operand stages copied by the LDS DMA path
// (global_load_lds_dwordx4: each lane's 16 bytes go straight to LDS at
// base + 16 lane, the 1 KB slice-block order): no staging registers and no
// LDS write instructions, so a stage can hold 64 of k (two k blocks) in two
// 64 KB LDS buffers, one barrier per 64 of k.  Per stage: wait for this
// wave's copies of the stage, barrier (everyone's copies landed, everyone is
// done with the other buffer), read the first k block's fragments, start the
// copies of the next stage into the other buffer, multiply.
template <int NW, int WM, int SD>
__device__ __forceinline__ void gemm_i8_dma_tile(const GemmArgs& a, int z, int bx, int nbx) {
  constexpr int TM = 128, BK = 64;
  constexpr int S = SD;
  constexpr int W = SD == 4 ? 5 : 3;
  constexpr int WN = NW / WM;
  constexpr int FM = TM / (32 * WM);
  constexpr int FN = TM / (32 * WN);
  constexpr int RB = TM / 32;
  constexpr int KB = BK / 32;
  constexpr int NBLK = RB * KB;
  constexpr int SBLK = 2 * S * NBLK;
  constexpr int LOADS = SBLK / NW;
  constexpr int SBYTES = SBLK * 1024;
  static_assert(SBLK % NW == 0, "a stage must split evenly over the waves");
  static_assert(FN >= 1 && FM >= 1, "at least one MFMA tile per wave");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ double red[NW];
  if (a.active && !a.active[z]) return;
  count_member(a, bx);
  const int64_t Np = a.Np;
  const int64_t kbr = Np >> 5;
  int tm, tn;
  tile_coords(bx, (int)(Np / TM), (int)(Np / TM), tm, tn, a.sym);
  // the wave index is uniform: block addresses live in scalar registers
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WN, wn = wave % WN;
  const int zx = z / a.X.div, zy = z / a.Y.div;
  const int8_t* xq = a.X.q8 + (int64_t)zx * a.X.stride * kQ8Slices;
  const int8_t* yq = a.Y.q8 + (int64_t)zy * a.Y.stride * kQ8Slices;
  const double scale = a.X.qs[a.X.stride ? zx : 0] * a.Y.qs[a.Y.stride ? zy : 0];
  const int8_t* src[LOADS];
  int dst[LOADS];
#pragma unroll
  for (int j = 0; j < LOADS; ++j) {
    const int q = wave + NW * j;
    const int op = q / (S * NBLK), sl = (q / NBLK) % S, b = q % NBLK;
    const int rb = b / KB, kb = b % KB;
    const int64_t brow = (int64_t)(op ? tn : tm) * RB + rb;
    src[j] = (op ? yq : xq) + (((brow * kbr + kb) * kQ8Slices + sl) << 10);  // uniform
    dst[j] = q * 1024;  // uniform: the DMA adds 16 lane itself
  }
  auto issue = [&](int kt) {
    const int64_t koff = (int64_t)kt * KB * kQ8Slices * 1024 + lane * 16;
    unsigned char* base = smem + (kt & 1) * SBYTES;
#pragma unroll
    for (int j = 0; j < LOADS; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(src[j] + koff),
                                       (__attribute__((address_space(3))) void*)(base + dst[j]), 16, 0, 0);
  };
  i16v acc[W][FM][FN];
#pragma unroll
  for (int w = 0; w < W; ++w)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[w][i][j][r] = 0;
  const int nk = (int)(Np / BK);
  issue(0);
  for (int kt = 0; kt < nk; ++kt) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's copies of stage kt
    __syncthreads();
    const unsigned char* sb = smem + (kt & 1) * SBYTES + lane * 16;
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
      i4v xa[S][FM], yb[S][FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        xa[0][i] = __builtin_bit_cast(i4v, *(const u4v*)(sb + (((0 * NBLK) + (wm * FM + i) * KB + kk) << 10)));
#pragma unroll
      for (int q = 0; q < S; ++q)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          yb[q][j] = __builtin_bit_cast(
              i4v, *(const u4v*)(sb + ((((S + q) * NBLK) + (wn * FN + j) * KB + kk) << 10)));
#pragma unroll
      for (int p = 1; p < S; ++p)
#pragma unroll
        for (int i = 0; i < FM; ++i)
          xa[p][i] = __builtin_bit_cast(i4v, *(const u4v*)(sb + (((p * NBLK) + (wm * FM + i) * KB + kk) << 10)));
      if (kk == 0 && kt + 1 < nk) issue(kt + 1);
#pragma unroll
      for (int p = 0; p < S; ++p)
#pragma unroll
        for (int q = 0; q < S && p + q < W; ++q)
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[p + q][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[p][i], yb[q][j], acc[p + q][i][j], 0, 0, 0);
    }
  }
  const double rb = 1.0 / kQ8Base;
  double dsum = 0.0;
  // largest |C| of the tile, rounded up to FP32: an upper bound, so the
  // digits of the slicing still fit (their scale is at most 2^-24 larger than
  // the exact maximum's), and one register instead of two keeps the epilogue
  // within the register budget
  float fmx = 0.0f;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = (int64_t)tm * TM + wm * (TM / WM) + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t col = (int64_t)tn * TM + wn * (TM / WN) + j * 32 + (lane & 31);
        double v = (double)acc[W - 1][i][j][r];
#pragma unroll
        for (int w = W - 2; w >= 0; --w) v = v * rb + (double)acc[w][i][j][r];
        {
          const double o = epi<double>(a, z, row, col, v * scale, dsum);
          fmx = o == o ? fmaxf(fmx, __double2float_ru(fabs(o))) : INFINITY;
        }
      }
  if (a.W) {
    const double s = block_sum(dsum, red);
    if (tid == 0) a.partials[(int64_t)z * nbx + bx] = s;
  }
  if (a.cmax) {
    const double m = block_max((double)fmx, red);
    if (tid == 0) a.cmax[(int64_t)z * a.cmax_stride + bx] = m;
  }
}

template <int NW, int WM, int SD>
__global__ __launch_bounds__(NW * 64) void k_gemm_i8_dma(GemmArgs a) {
  gemm_i8_dma_tile<NW, WM, SD>(a, blockIdx.z, blockIdx.x, gridDim.x);
}

template <int NW, int WM, int SD>
__global__ __launch_bounds__(NW * 64) void k_gemm_i8_dma_grouped(const GemmArgs* __restrict__ list,
                                                                  const int* __restrict__ start, int nprob) {
  int p = 0;
  const int b = blockIdx.x;
  while (p + 1 < nprob && b >= start[p + 1]) ++p;
  const GemmArgs& a = list[p];
  const int tiles = (int)((a.Np / 128) * (a.Np / 128));
  const int local = b - start[p];
  gemm_i8_dma_tile<NW, WM, SD>(a, local / tiles, local % tiles, tiles);
}

template <int BK, int NW, int WM, int SD>
__global__ __launch_bounds__(NW * 64) void k_gemm_i8(GemmArgs a) {
  gemm_i8_tile<BK, NW, WM, SD>(a, blockIdx.z, blockIdx.x, gridDim.x);
}

template <int BK, int NW, int WM, int SD>
__global__ __launch_bounds__(NW * 64) void k_gemm_i8_grouped(const GemmArgs* __restrict__ list,
                                                              const int* __restrict__ start, int nprob) {
  int p = 0;
  const int b = blockIdx.x;
  while (p + 1 < nprob && b >= start[p + 1]) ++p;
  const GemmArgs& a = list[p];
  const int tiles = (int)((a.Np / 128) * (a.Np / 128));
  const int local = b - start[p];
  gemm_i8_tile<BK, NW, WM, SD>(a, local / tiles, local % tiles, tiles);
}

template <int BK, int SD>
constexpr size_t i8_lds() { return (size_t)2 * 2 * SD * 4 * (BK / 32) * 1024; }

template <int BK, int NW, int WM, int SD>
hipError_t prepare_i8() {
  hipError_t e = hipFuncSetAttribute((const void*)k_gemm_i8<BK, NW, WM, SD>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)i8_lds<BK, SD>());
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_gemm_i8_grouped<BK, NW, WM, SD>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)i8_lds<BK, SD>());
}

template <int BK, int NW, int WM, int SD>
hipError_t launch_i8(const GemmArgs& a, dim3 grid, hipStream_t s) {
  hipLaunchKernelGGL((k_gemm_i8<BK, NW, WM, SD>), grid, dim3(NW * 64), (i8_lds<BK, SD>()), s, a);
  return hipGetLastError();
}

template <int BK, int NW, int WM, int SD>
hipError_t launch_i8_grouped(const GemmArgs* list, const int* start, int nprob, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((k_gemm_i8_grouped<BK, NW, WM, SD>), dim3(blocks), dim3(NW * 64), (i8_lds<BK, SD>()), s, list,
                     start, nprob);
  return hipGetLastError();
}

template <int SD>
constexpr size_t i8_dma_lds() { return (size_t)2 * 2 * SD * 4 * 2 * 1024; }

template <int NW, int WM, int SD>
hipError_t prepare_i8_dma() {
  hipError_t e = hipFuncSetAttribute((const void*)k_gemm_i8_dma<NW, WM, SD>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)i8_dma_lds<SD>());
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_gemm_i8_dma_grouped<NW, WM, SD>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)i8_dma_lds<SD>());
}

template <int NW, int WM, int SD>
hipError_t launch_i8_dma(const GemmArgs& a, dim3 grid, hipStream_t s) {
  hipLaunchKernelGGL((k_gemm_i8_dma<NW, WM, SD>), grid, dim3(NW * 64), (i8_dma_lds<SD>()), s, a);
  return hipGetLastError();
}

template <int NW, int WM, int SD>
hipError_t launch_i8_dma_grouped(const GemmArgs* list, const int* start, int nprob, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((k_gemm_i8_dma_grouped<NW, WM, SD>), dim3(blocks), dim3(NW * 64), (i8_dma_lds<SD>()), s, list,
                     start, nprob);
  return hipGetLastError();
}

// Int8 launch by variant: 0, 1 register-staged (32 x 64 / 64 x 32 wave tiles),
// 2, 3 LDS DMA with 64-deep stages (same wave tiles).
template <int SD>
hipError_t launch_i8_variant(const GemmArgs& a, dim3 grid, hipStream_t s) {
  switch (a.variant) {
    case 1: return launch_i8<32, 8, 2, SD>(a, grid, s);
    case 2: return launch_i8_dma<8, 4, SD>(a, grid, s);
    case 3: return launch_i8_dma<8, 2, SD>(a, grid, s);
    default: return launch_i8<32, 8, 4, SD>(a, grid, s);
  }
}

template <int SD>
hipError_t launch_i8_variant_grouped(int variant, const GemmArgs* list, const int* start, int nprob, int blocks,
                                     hipStream_t s) {
  switch (variant) {
    case 1: return launch_i8_grouped<32, 8, 2, SD>(list, start, nprob, blocks, s);
    case 2: return launch_i8_dma_grouped<8, 4, SD>(list, start, nprob, blocks, s);
    case 3: return launch_i8_dma_grouped<8, 2, SD>(list, start, nprob, blocks, s);
    default: return launch_i8_grouped<32, 8, 4, SD>(list, start, nprob, blocks, s);
  }
}

}  // namespace

// Kernel variants of each engine, chosen per padded size by the autotuner
// (0 is the default):
//   FP64  0: BK 8, 8 waves   1: BK 16, 8 waves   2: BK 8, 4 waves
//   FP32  0: BK 32, 8 waves  1: BK 16, 8 waves   2: BK 32, 4 waves
//   split BF16  0: 256 x 256 tiles where Np allows (else 128)   1: 128 x 128 tiles
//   (the 6-product kernel with FP64 slice sums has 128 x 128 tiles only)
//   int8 (both digit counts)  0: BK 32, 8 waves of 32 x 64   1: BK 32, 8 waves of 64 x 32
//                             2, 3: the same wave tiles, LDS DMA copies, BK 64
int gemm_variants(Engine eng, int acc64) {
  switch (eng) {
    case Engine::F64: return 3;
    case Engine::F32: return 3;
    case Engine::BF16S2: return 2;
    case Engine::BF16S3: return acc64 ? 1 : 2;
    case Engine::I8S4: return 4;
    case Engine::I8S3: return 4;
  }
  return 1;
}

const char* gemm_variant_name(Engine eng, int acc64, int v) {
  static const char* f64[3] = {"FP64 BK 8, 8 waves", "FP64 BK 16, 8 waves", "FP64 BK 8, 4 waves"};
  static const char* f32[3] = {"FP32 BK 32, 8 waves", "FP32 BK 16, 8 waves", "FP32 BK 32, 4 waves"};
  static const char* bf[2] = {"BF16 256 x 256 tiles", "BF16 128 x 128 tiles"};
  static const char* i8[4] = {"int8 BK 32, 8 waves of 32 x 64", "int8 BK 32, 8 waves of 64 x 32",
                              "int8 LDS DMA, BK 64, 8 waves of 32 x 64", "int8 LDS DMA, BK 64, 8 waves of 64 x 32"};
  if (v < 0 || v >= gemm_variants(eng, acc64)) return "invalid";
  if (eng == Engine::I8S4 || eng == Engine::I8S3) return i8[v];
  if (eng == Engine::F64) return f64[v];
  if (eng == Engine::F32) return f32[v];
  if (eng == Engine::BF16S3 && acc64) return "BF16 128 x 128 tiles, FP64 slice sums";
  return bf[v];
}

// Output tile edge of the kernel `gemm` uses for an engine, size and variant:
// the 256-wide split-BF16 kernel when Np and the variant allow it.
int gemm_tile_edge(Engine eng, int64_t Np, int variant, int acc64) {
  const bool bf = eng == Engine::BF16S2 || (eng == Engine::BF16S3 && !acc64);
  if (bf && variant == 0 && Np % 256 == 0) return 256;
  return BM;
}

// Raise the dynamic-LDS limit of every kernel that needs more than the
// default, once, before any launch (and so never inside a graph capture).
hipError_t gemm_prepare() {
  hipError_t e;
  if ((e = prepare_bf16<2, 128, 32, 4>())) return e;
  if ((e = prepare_bf16<3, 128, 32, 4>())) return e;
  if ((e = prepare_bf16<3, 128, 32, 8, 1>())) return e;
  if ((e = prepare_bf16<2, 256, 16, kWaves256>())) return e;
  if ((e = prepare_i8<32, 8, 2, 4>())) return e;
  if ((e = prepare_i8<32, 8, 4, 4>())) return e;
  if ((e = prepare_i8<32, 8, 2, 3>())) return e;
  if ((e = prepare_i8<32, 8, 4, 3>())) return e;
  if ((e = prepare_i8_dma<8, 4, 4>())) return e;
  if ((e = prepare_i8_dma<8, 2, 4>())) return e;
  if ((e = prepare_i8_dma<8, 4, 3>())) return e;
  if ((e = prepare_i8_dma<8, 2, 3>())) return e;
  return prepare_bf16<3, 256, 16, kWaves256>();
}

int gemm_tiles(Engine eng, int64_t Np, int variant, int acc64) {
  const int e = gemm_tile_edge(eng, Np, variant, acc64);
  return (int)((Np / e) * (Np / e));
}

int gemm_launch_tiles(const GemmArgs& a) {
  const int T = (int)(a.Np / gemm_tile_edge(a.eng, a.Np, a.variant, a.acc64));
  if (a.sym && !a.W && T % 2 == 0) return T / 2 * (T + 1);
  return T * T;
}

// Whether gemm() computes the diagonal tiles of a symmetric product in parts:
// int8 register-staged kernels with at least 8 tile rows (more, shorter
// blocks fill the last round of the launch).
static bool diag_split(const GemmArgs& a) {
  const int T = (int)(a.Np / 128);
  return (a.eng == Engine::I8S4 || a.eng == Engine::I8S3) && a.variant <= 1 && a.dpart && a.dsplit >= 2 &&
         a.dsplit <= 8 && a.batch <= a.dpart_members && T >= 8 && a.Np / 32 >= a.dsplit &&
         gemm_launch_tiles(a) < T * T;
}

int gemm_cmax_entries(const GemmArgs& a) {
  if (!diag_split(a)) return gemm_launch_tiles(a);
  const int T = (int)(a.Np / 128);
  return T * kDiagParts + T * (T - 1) / 2;
}

namespace {

struct Planes3 {
  uint16_t* p[3];
};

// Upper triangle of each symmetric product output from its lower triangle
// (master and, when requested, split planes): 32 x 32 blocks (bi, bj) with
// bi >= bj go through LDS and are written transposed at (bj, bi); diagonal
// blocks copy their strictly lower part only.
__global__ __launch_bounds__(256) void k_mirror(double* __restrict__ C, int64_t Np, int64_t sC, Planes3 pl, int np,
                                                const int* active) {
  const int z = blockIdx.z;
  if (active && !active[z]) return;
  const int64_t nb = Np / 32;
  const int64_t bi = blockIdx.x / nb, bj = blockIdx.x % nb;
  if (bi < bj) return;
  __shared__ double t[32][33];
  double* c = C + (int64_t)z * sC;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) t[r][tx] = c[(bi * 32 + r) * Np + bj * 32 + tx];
  __syncthreads();
  uint16_t* p[3] = {nullptr, nullptr, nullptr};
  for (int i = 0; i < np; ++i) p[i] = pl.p[i] + (int64_t)z * sC;
  // destination row bj*32 + r2 (source column), column bi*32 + tx (source row)
  for (int r2 = ty; r2 < 32; r2 += 8) {
    if (bi == bj && tx <= r2) continue;  // diagonal block: source (tx, r2) must lie below the diagonal
    const double v = t[tx][r2];
    const int64_t row = bj * 32 + r2, col = bi * 32 + tx;
    c[row * Np + col] = v;
    if (np) write_split(v, p, np, plane_off(row, col, Np));
  }
}

// The diagonal tiles of a split symmetric int8 product: block (d, part, z)
// sums the dsplit partial tiles of rows 32 part .. 32 part + 31 of diagonal
// tile d in order, applies the epilogue of the product kernels and leaves
// their max |C| in slot d kDiagParts + part.
__global__ __launch_bounds__(256) void k_diag_sum(GemmArgs a) {
  constexpr int TM = 128, RP = TM / kDiagParts, PER = RP * TM / 256;
  const int z = blockIdx.z, d = blockIdx.x, part = blockIdx.y;
  if (a.active && !a.active[z]) return;
  __shared__ double red[4];
  // partial s of member z: rows 0 .. 127 of the strip (z, s) of 128 x Np
  // values, diagonal tile d at columns 128 d ..
  const int64_t strip = (int64_t)TM * a.Np;
  const double* dp = a.dpart + (int64_t)z * a.dsplit * strip + (int64_t)d * TM;
  double dsum = 0.0, m = 0.0;
  bool bad = false;
  double v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int64_t lr = part * RP + e / TM, lc = e % TM;
    v[u] = dp[lr * a.Np + lc];
  }
  for (int sp = 1; sp < a.dsplit; ++sp)
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int64_t lr = part * RP + e / TM, lc = e % TM;
      v[u] += dp[sp * strip + lr * a.Np + lc];
    }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int64_t row = (int64_t)d * TM + part * RP + e / TM, col = (int64_t)d * TM + e % TM;
    const double o = epi<double>(a, z, row, col, v[u], dsum);
    const double ao = fabs(o);
    bad |= !(ao <= 1.0e308);
    m = fmax(m, ao);
  }
  if (a.cmax) {
    // an FP32 value rounded up, as the product kernels leave it
    const double bm = block_max(bad ? (double)INFINITY : (double)__double2float_ru(m), red);
    if (threadIdx.x == 0) a.cmax[(int64_t)z * a.cmax_stride + d * kDiagParts + part] = bm;
  }
}

}  // namespace

hipError_t gemm_launch(const GemmArgs& a, int tiles, hipStream_t s);

hipError_t gemm(const GemmArgs& a0, hipStream_t s) {
  if (a0.Np <= 0 || a0.Np % BM != 0 || a0.batch <= 0 || a0.X.div < 1 || a0.Y.div < 1 || a0.variant < 0 ||
      a0.variant >= gemm_variants(a0.eng, a0.acc64))
    return hipErrorInvalidValue;
  GemmArgs a = a0;
  const int full = gemm_tiles(a.eng, a.Np, a.variant, a.acc64);
  int tiles = gemm_launch_tiles(a);
  a.sym = tiles < full ? 1 : 0;
  const int T = (int)(a.Np / 128);
  if (a.sym && diag_split(a)) {
    a.sym = 2;
    tiles = T * a.dsplit + T * (T - 1) / 2;
  }
  hipError_t e = gemm_launch(a, tiles, s);
  if (e != hipSuccess || !a.sym) return e;
  if (a.sym == 2) {
    hipLaunchKernelGGL(k_diag_sum, dim3((unsigned)T, kDiagParts, (unsigned)a.batch), dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  Planes3 pl{{a.Cpl[0], a.Cpl[1], a.Cpl[2]}};
  const int np = a.Cpl[2] ? 3 : (a.Cpl[1] ? 2 : (a.Cpl[0] ? 1 : 0));
  const int64_t nb = a.Np / 32;
  hipLaunchKernelGGL(k_mirror, dim3((unsigned)(nb * nb), 1, (unsigned)a.batch), dim3(256), 0, s, (double*)a.C,
                     a.Np, a.sC, pl, np, a.active);
  return hipGetLastError();
}

hipError_t gemm_launch(const GemmArgs& a, int tiles, hipStream_t s) {
  const int edge = gemm_tile_edge(a.eng, a.Np, a.variant, a.acc64);
  const dim3 grid((unsigned)tiles, 1, (unsigned)a.batch);
  switch (a.eng) {
    case Engine::I8S4:
    case Engine::I8S3:
      if (a.Np > kQ8MaxK || !a.X.q8 || !a.Y.q8 || !a.X.qs || !a.Y.qs) return hipErrorInvalidValue;
      return a.eng == Engine::I8S3 ? launch_i8_variant<3>(a, grid, s) : launch_i8_variant<4>(a, grid, s);
    case Engine::F64:
      if (a.variant == 1) hipLaunchKernelGGL((k_gemm_f64<16, 8>), grid, dim3(8 * 64), 0, s, a);
      else if (a.variant == 2) hipLaunchKernelGGL((k_gemm_f64<8, 4>), grid, dim3(4 * 64), 0, s, a);
      else hipLaunchKernelGGL((k_gemm_f64<kF64BK, kF64NW>), grid, dim3(kF64NW * 64), 0, s, a);
      return hipGetLastError();
    case Engine::F32:
      if (a.variant == 1) hipLaunchKernelGGL((k_gemm_f32<16, 8>), grid, dim3(8 * 64), 0, s, a);
      else if (a.variant == 2) hipLaunchKernelGGL((k_gemm_f32<32, 4>), grid, dim3(4 * 64), 0, s, a);
      else hipLaunchKernelGGL((k_gemm_f32<kF32BK, kF32NW>), grid, dim3(kF32NW * 64), 0, s, a);
      return hipGetLastError();
    case Engine::BF16S2:
      return edge == 256 ? launch_bf16<2, 256, 16, kWaves256>(a, grid, s)
                         : launch_bf16<2, 128, 32, 4>(a, grid, s);
    case Engine::BF16S3:
      if (a.acc64) {
        if (edge != 128) return hipErrorInvalidValue;
        return launch_bf16<3, 128, 32, 8, 1>(a, grid, s);
      }
      return edge == 256 ? launch_bf16<3, 256, 16, kWaves256>(a, grid, s)
                         : launch_bf16<3, 128, 32, 4>(a, grid, s);
  }
  return hipErrorInvalidValue;
}

hipError_t gemm_grouped(Engine eng, int variant, int acc64, int edge, const GemmArgs* list, const int* start,
                        int nprob, int blocks, hipStream_t s) {
  if (nprob < 1 || blocks < 1 || variant < 0 || variant >= gemm_variants(eng, acc64)) return hipErrorInvalidValue;
  switch (eng) {
    case Engine::I8S4: return launch_i8_variant_grouped<4>(variant, list, start, nprob, blocks, s);
    case Engine::I8S3: return launch_i8_variant_grouped<3>(variant, list, start, nprob, blocks, s);
    case Engine::F64:
      if (variant == 1) hipLaunchKernelGGL((k_gemm_f64_grouped<16, 8>), dim3(blocks), dim3(8 * 64), 0, s, list, start, nprob);
      else if (variant == 2) hipLaunchKernelGGL((k_gemm_f64_grouped<8, 4>), dim3(blocks), dim3(4 * 64), 0, s, list, start, nprob);
      else hipLaunchKernelGGL((k_gemm_f64_grouped<kF64BK, kF64NW>), dim3(blocks), dim3(kF64NW * 64), 0, s, list, start, nprob);
      return hipGetLastError();
    case Engine::F32:
      if (variant == 1) hipLaunchKernelGGL((k_gemm_f32_grouped<16, 8>), dim3(blocks), dim3(8 * 64), 0, s, list, start, nprob);
      else if (variant == 2) hipLaunchKernelGGL((k_gemm_f32_grouped<32, 4>), dim3(blocks), dim3(4 * 64), 0, s, list, start, nprob);
      else hipLaunchKernelGGL((k_gemm_f32_grouped<kF32BK, kF32NW>), dim3(blocks), dim3(kF32NW * 64), 0, s, list, start, nprob);
      return hipGetLastError();
    case Engine::BF16S2:
      return edge == 256 ? launch_bf16_grouped<2, 256, 16, kWaves256>(list, start, nprob, blocks, s)
                         : launch_bf16_grouped<2, 128, 32, 4>(list, start, nprob, blocks, s);
    case Engine::BF16S3:
      if (acc64) return launch_bf16_grouped<3, 128, 32, 8, 1>(list, start, nprob, blocks, s);
      return edge == 256 ? launch_bf16_grouped<3, 256, 16, kWaves256>(list, start, nprob, blocks, s)
                         : launch_bf16_grouped<3, 128, 32, 4>(list, start, nprob, blocks, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace dmpt
