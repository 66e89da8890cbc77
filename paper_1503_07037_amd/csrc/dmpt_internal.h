// Internal declarations shared by the HIP kernels and the host drivers of
// the DMPT library.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <cmath>

#include "dmpt.h"

namespace dmpt {

// Padding granule of the workspace: every working matrix is stored Np x Np
// with Np = roundup(N, kPad) and zeros outside the leading N x N block, so
// product kernels never need edge masks.
constexpr int kPad = 128;

inline int64_t padded(int64_t n) { return (n + kPad - 1) / kPad * kPad; }

// Product engines (see gemm.hip).
enum class Engine : int { F64 = 0, F32 = 1, BF16S2 = 2, BF16S3 = 3, I8S4 = 4, I8S3 = 5 };
constexpr int kEngines = 6;
inline bool engine_int8(Engine e) { return e == Engine::I8S4 || e == Engine::I8S3; }

// BF16 planes per operand (the int8 engine keeps its slices apart, see q8_off).
inline int engine_planes(Engine e) {
  return e == Engine::BF16S2 ? 2 : (e == Engine::BF16S3 ? 3 : 0);
}
// Matrix-core products per logical product.
inline int engine_terms(Engine e) {
  switch (e) {
    case Engine::BF16S2: return 3;
    case Engine::BF16S3: return 6;
    case Engine::I8S4: return 13;
    case Engine::I8S3: return 6;
    default: return 1;
  }
}

// Int8 slices of the I8S4 engine.  A member x (Np x Np, FP64 master) with
// m = max |x| is stored as x = q (d0 + d1 / 254 + d2 / 254^2 + d3 / 254^3),
// q = m / 127, every digit a signed int8 in [-127, 127] (each digit rounds
// the scaled remainder of the ones before it to the nearest integer, so the
// remainder stays within 1/2 and 254 times it fits the next digit).  Slice
// s of the 32 x 32 block (row / 32, col / 32) is 1 KB at
// ((row / 32) * (Np / 32) + col / 32) * 4 + s KB; inside it element (r, c)
// sits at ((c / 16) * 32 + r) * 16 + c % 16: the operand order of
// v_mfma_i32_32x32x32_i8 (lane l holds row l % 32 and 16 consecutive k of
// half l / 32), so a wave moves a slice block as 64 consecutive 16-byte
// pieces.  A member takes 4 Np^2 bytes; its q sits in a separate FP64 array.
constexpr int kQ8Slices = 4;
constexpr double kQ8Base = 254.0;
__host__ __device__ inline int64_t q8_off(int64_t row, int64_t col, int64_t Np, int s) {
  return ((((row >> 5) * (Np >> 5) + (col >> 5)) * kQ8Slices + s) << 10) + ((((col >> 4) & 1) << 5) + (row & 31)) * 16 +
         (col & 15);
}
// Largest inner dimension whose int32 sums stay exact: four digit products
// of weight 3, each at most 127^2 per term.  The products kept are the
// thirteen of weight p + q <= 4: without (2, 2) the square of the third digit
// would be missing from every diagonal entry of a product of a matrix with
// itself (a one-signed error that traces add up), and (1, 3), (3, 1) bring the
// remaining truncation to 254^-5 of the operands' scales.
constexpr int64_t kQ8MaxK = 32768;

// BF16 plane layout of an Np x Np member (Np a multiple of 32): blocks of
// 32 rows x 16 columns, 512 elements (1 KB) each; block (row / 32, col / 16)
// starts at element ((row / 32) * (Np / 16) + col / 16) * 512, and inside a
// block element (r, c) sits at ((c / 8) * 32 + r) * 8 + c % 8.  That is the
// operand order of v_mfma_f32_32x32x16_bf16 (lane l holds row l % 32 and
// k = 8 (l / 32) .. 8 (l / 32) + 7), so one wave moves a block between HBM,
// LDS and registers as 64 consecutive 16-byte pieces: coalesced loads and
// bank-conflict-free LDS reads without any swizzle.
__host__ __device__ inline int64_t plane_off(int64_t row, int64_t col, int64_t Np) {
  return (((row >> 5) * (Np >> 4) + (col >> 4)) << 9) + ((((col >> 3) & 1) << 5) + (row & 31)) * 8 +
         (col & 7);
}

// Np of an n-element square member that carries planes, or 0 when n is not
// the square of a multiple of 32 below 2^16 (plane writers need both).
inline int64_t plane_np(int64_t n) {
  const int64_t r = (int64_t)(std::sqrt((double)n) + 0.5);
  return (r > 0 && r < 65536 && r % 32 == 0 && r * r == n) ? r : 0;
}

// Batched operand: base matrix and element stride between batch members
// (0 = the same matrix for every member).  Member z of the launch reads
// operand member z / div, so div = d lets d directions share one matrix.
struct BOp {
  const void* m = nullptr;
  const uint16_t* pl[3] = {nullptr, nullptr, nullptr};
  const int8_t* q8 = nullptr;  // I8S4: int8 slices of the member (4 stride bytes apart)
  const double* qs = nullptr;  // I8S4: q of the member (one double apart)
  int64_t stride = 0;
  int div = 1;
};

struct GemmArgs {
  Engine eng;
  int64_t Np;          // all operands are Np x Np, ld = Np
  int batch;           // gridDim.z
  BOp X, Y;            // C = alpha * X * Y^T (+ beta1 C1 + beta2 C2)
  void* C;             // master output
  uint16_t* Cpl[3];    // optional split planes of C (nullptr: not written)
  int64_t sC;
  double alpha;
  const void* C1; int64_t sC1; double beta1;
  const void* C2; int64_t sC2; double beta2;
  const void* W; int64_t sW;   // optional: per-tile partials of <W, C>
  double* partials;            // [batch][tiles]
  const int* active;           // optional per-batch mask; 0 = skip the member
  int variant;                 // kernel variant of the engine (gemm_variants; 0 = default)
  int acc64;                   // BF16S3 only: FP32 per stage, FP64 across stages (128-wide tiles)
  double* cmax;                // int8 kernels, optional: max |C| of every launched tile at
  int64_t cmax_stride;         //   cmax[z * cmax_stride + tile] (the int8 slicing of C then skips its scan)
  int sym;                     // C is symmetric: only the tiles on and below the diagonal are
                               // computed (when the tile count per side is even and W is unset),
                               // then the upper triangle is mirrored from the lower one
  // int8 kernels with sym, optional: each diagonal tile is computed as dsplit
  // blocks over consecutive ranges of the inner index that leave their FP64
  // partial tiles in dpart (room for dpart_members members), then summed in a
  // fixed order by a second kernel; the off-diagonal tiles keep one block each
  double* dpart;
  int dsplit;
  int dpart_members;
  // optional executed-work tally (graph replays, where the host cannot see
  // which members are skipped): every member that runs adds tally_m and
  // tally_u to tally[0] and tally[1]
  double* tally;
  double tally_m, tally_u;
};

// Kernel variants of an engine (gemm.hip), their names, and the output tile
// edge and number of output tiles per batch member of the kernel gemm()
// launches for an engine, size and variant.
int gemm_variants(Engine eng, int acc64);
const char* gemm_variant_name(Engine eng, int acc64, int variant);
int gemm_tile_edge(Engine eng, int64_t Np, int variant, int acc64);
int gemm_tiles(Engine eng, int64_t Np, int variant, int acc64);
// Output tiles per member that gemm() computes (fewer than gemm_tiles with sym).
int gemm_launch_tiles(const GemmArgs& a);
// Tile maxima per member that an int8 product with cmax leaves.
int gemm_cmax_entries(const GemmArgs& a);
hipError_t gemm(const GemmArgs& a, hipStream_t s);
// One grouped launch over nprob products of the same engine, variant and tile
// edge (list, start: device arrays; problem p owns the blocks start[p] ..
// start[p + 1] - 1, members x tiles in order; blocks = start[nprob]).
hipError_t gemm_grouped(Engine eng, int variant, int acc64, int edge, const GemmArgs* list, const int* start,
                        int nprob, int blocks, hipStream_t s);
// Set the launch attributes of the product kernels (once per process and device).
hipError_t gemm_prepare();

// ---------------------------------------------------------------- element-wise
// out = a (in + in^T) + a2 (in2 + in2^T) + dshift I on the leading N x N
// block, 0 elsewhere (in2 may be null).  When gate is not null the kernel
// does nothing while *gate == 0.
// in: Tin with leading dim ldi; out: Tout with leading dim ldo (+ split planes).
// Batched over `batch` members with element strides.
// The tile pair (i, j) / (j, i) is handled by one block, so in == out is allowed.
// With mx (and no gate), member z also leaves sym_pair_blocks(span) partial
// maxima of |out| at mx + z mstride (their max is the member's max |out|).
template <class Tin, class Tout>
hipError_t sym_combine(const Tin* in, int64_t ldi, int64_t si, int64_t N, int64_t Np, double a,
                       const double* dshift, int dstride, Tout* out, int64_t ldo, int64_t so,
                       uint16_t* const* planes, int nplanes, int batch, hipStream_t s,
                       const Tin* in2 = nullptr, double a2 = 0.0, const int* gate = nullptr,
                       double* mx = nullptr, int64_t mstride = 0);
// Blocks per member of sym_combine over span rows: one per 128 x 128 tile
// pair on and above the diagonal (with mx, the maxima each member leaves).
int64_t sym_pair_blocks(int64_t span);

// out = in^T (Np x Np members, batched, with planes); in != out.
template <class T>
hipError_t transpose(const T* in, int64_t Np, int64_t stride, T* out, uint16_t* const* planes,
                     int nplanes, int batch, hipStream_t s);

// Int8 slices (I8S4) of `batch` FP64 members x + z sx (Np x Np): block maxima
// of |x| into part[z * nb ..] (nb = q8_blocks(Np)), then every block of the
// slicing kernel reduces them to the member's max, writes q to qs[z] and its
// share of the slices to q8 + z sq (bytes).
int q8_blocks(int64_t Np);
hipError_t quantize_q8(const double* x, int64_t sx, int64_t Np, int batch, double* part, int8_t* q8, int64_t sq,
                       double* qs, const int* active, hipStream_t s);
// The same with the maxima already known: nb partial maxima per member at
// part[z * pstride ..] (e.g. the tile maxima a product kernel wrote).
hipError_t quantize_q8_known(const double* x, int64_t sx, int64_t Np, int batch, const double* part,
                             int64_t pstride, int nb, int8_t* q8, int64_t sq, double* qs, hipStream_t s);

// Split a master matrix into BF16 planes (batched).
hipError_t split_planes(const double* x, int64_t n_elems, int64_t sx, uint16_t* const* planes,
                        int64_t sp, int nplanes, int batch, hipStream_t s);

// Reductions; every result is FP64 and deterministic.
// Number of partial slots a streaming reduction over n elements uses.
int reduce_blocks(int64_t n_elems);
// partials[z*nb + b] of sum x*y over n elements (batched; strides in elements)
template <class T>
hipError_t dot_partials(const T* x, int64_t sx, const T* y, int64_t sy, int64_t n, int batch,
                        double* partials, hipStream_t s);
// out[z * ostride + oidx] = sum of partials[z*count .. z*count+count)
hipError_t sum_partials(const double* partials, int count, int batch, double* out,
                        int ostride, int oidx, hipStream_t s);
// out[z*ostride] = sum_i x[z][i*ld + i], i < N (trace, FP64 input);
// aout[z*ostride] = sum_i |x_ii| when aout is not null
template <class T>
hipError_t trace(const T* x, int64_t ld, int64_t sx, int64_t N, int batch, double* out,
                 int ostride, double* aout, hipStream_t s);

// CG updates (batched over right-hand sides z).
//   update_xr: alpha = rr[z]/pq[z]; U += alpha P; R -= alpha Q; partials of <R,R>
//   (and, when rmax is not null, block maxima of |R| at rmax[z * blocks + b])
template <class T>
hipError_t cg_update_xr(T* U, T* R, const T* P, const T* Q, int64_t n, int64_t stride, int batch,
                        const double* rr, const double* pq, int hstride, const int* active,
                        double* partials, hipStream_t s, double* rmax = nullptr);
//   update_p with int8 slices (FP64, Np x Np members): P = R + beta P, and the
//   slices of the new P (q8 + z sq bytes, q at qs[z]) from the scale bound
//   max |R| (rmax from update_xr) + |beta| pb_old[z hstride], written to
//   pb_new[z hstride]
hipError_t cg_update_p_q8(double* P, const double* R, int64_t Np, int64_t stride, int batch, const double* rr_new,
                          const double* rr_old, int hstride, const int* active, const double* rmax,
                          const double* pb_old, double* pb_new, int8_t* q8, int64_t sq, double* qs,
                          hipStream_t s);
//   pb[z hstride] = 127 qs[z] (the bound of the first sliced P)
hipError_t q8_bound_init(const double* qs, double* pb, int hstride, int batch, hipStream_t s);
//   update_p: beta = rr_new[z]/rr_old[z]; P = R + beta P (+ planes)
template <class T>
hipError_t cg_update_p(T* P, const T* R, int64_t n, int64_t stride, int batch,
                       const double* rr_new, const double* rr_old, int hstride, const int* active,
                       uint16_t* const* planes, int nplanes, hipStream_t s);
// convergence: active[z] stays 1 while rr > tol2 ref or rr > eta2 rr0 (rr0: the
// initial residual); iters[z] counts the checks.  Any batch size.
hipError_t cg_check(const double* rr, const double* rr0, const double* ref, int hstride, int batch,
                    double tol2, double eta2, int* active, int* iters, hipStream_t s);

// *status = DMPT_ERR_NONFINITE when *flag is set, DMPT_ERR_RANGE when
// beta max(|gersh[0] - mu|, |gersh[1] - mu|) >= 2^(n+1), else DMPT_OK (one thread).
hipError_t input_status(const double* gersh, const int* flag, double beta, double mu, int n, int* status,
                        hipStream_t s);

// Statistics of a fixed-count solve: stat[0] += sum of iterations, stat[1] =
// max(stat[1], iterations), stat[2] += members still active (unconverged).
hipError_t cg_account(const int* active, const int* iters, int batch, int* stat, hipStream_t s);

// Element-wise linear combination: y = a x + b y (batched, master only) + planes
template <class T>
hipError_t axpby(const T* x, int64_t sx, T* y, int64_t sy, int64_t n, int batch, double a,
                 double b, uint16_t* const* planes, int64_t sp, int nplanes, hipStream_t s);

// Element-wise linear combination into a third array: out = a x + b y
// (one member, master) + planes of out
template <class T>
hipError_t axpbyz(const T* x, const T* y, T* out, int64_t n, double a, double b, uint16_t* const* planes,
                  int nplanes, hipStream_t s, double* mx = nullptr, int64_t mblocks = 0);
// With mx, axpbyz, convert and scaled_plus_identity run mblocks blocks per
// member, and block b of member z leaves max |out| over its elements at
// mx[z * mstride + b] (their max is the member's max |out|).  The block
// count for n elements and at most cap maxima:
int64_t ew_sink_blocks(int64_t n, int64_t cap);

// out = (Tout) in for n elements per member (batched) + planes of out
template <class Tin, class Tout>
hipError_t convert(const Tin* in, int64_t si, Tout* out, int64_t so, int64_t n, int batch,
                   uint16_t* const* planes, int64_t sp, int nplanes, hipStream_t s, double* mx = nullptr,
                   int64_t mstride = 0, int64_t mblocks = 0);

// Fill identity-plus-scaled matrix: out = a I + b x (Np x Np, zero padding kept)
template <class T>
hipError_t scaled_plus_identity(const T* x, T* out, int64_t N, int64_t Np, double a, double b,
                                uint16_t* const* planes, int nplanes, hipStream_t s, double* mx = nullptr,
                                int64_t mblocks = 0);

// p[0..n) = v and q[0..nq) = qv; either pointer may be null with count 0
hipError_t set_values(int* p, int v, int n, double* q, double qv, int nq, hipStream_t s);
// dst[z] = src[z / div] for z < n (member masks from system masks)
hipError_t expand_mask(const int* src, int div, int* dst, int n, hipStream_t s);

// Hashed pattern in [-1, 1) (with planes), for timing runs.
template <class T>
hipError_t fill_pattern(T* x, int64_t n, uint32_t seed, uint16_t* const* planes, int nplanes,
                        hipStream_t s);

// Linear canonical correction of one system's order-k responses, k = order
// (1 or 2; batched solve): with t its trace record (Tr Pk_z at 1 + (k-1) d + z,
// Tr(H1_z Pk_z) at 2J + 1 + (k-1) d + z, Tr P_J at rs0, Tr(H1_z P_J) at
// rs0 + 2 + z), mu / shift its mu jet and shifts, c its scale:
// delta_z = Tr Pk_z / Tr P_J, muk_z += delta_z, Pk[z] -= delta_z PJ (N x N
// FP64), records updated.  Does nothing while *gate == 0.
hipError_t lin_correct(double* t, int d, int J, int rs0, double* mu, double* shift, double c,
                       double* delta, double* const* Pk, const double* PJ, int64_t N, const int* gate,
                       hipStream_t s, int order);

// First guess of mu1 for each of d directions from a converged P0 (N x N FP64):
// with w_i = (P0 - P0^2)_ii, mu1_z = sum_i w_i (H1_z)_ii / sum_i w_i (the
// Tr P1 = 0 condition with the response to H1 = I taken as beta P0 (I - P0)
// and only the diagonal of H1).  w: N doubles of scratch.  Entries z with
// want[z] == 0 are left as they are (want: device ints).
hipError_t mu1_guess(const double* P0, int64_t N, const double* const* H1, int d, double* w,
                     double* mu, double* shift, double c, const int* want, hipStream_t s);

// Device-side canonical Newton update of a batch of systems (see elementwise.hip).
hipError_t newton_update(const double* tr, int rs, const double* par, double* mu, double* shift,
                         int J, int nk, double tol, int final_stage, int* active, int* done,
                         double* prev_err, double* brk, double* occ, int* passes, int* status,
                         int nsys, hipStream_t s);

// Scan for non-finite values: flag |= any(!isfinite(x))
// out (Np x Np) = in (N x N, leading dimension ldi) or its transpose, zero
// outside the leading N x N block (no planes).
hipError_t pad_copy(const double* in, int64_t ldi, int64_t N, double* out, int64_t Np, bool trans,
                    hipStream_t s);
hipError_t nonfinite_scan(const double* x, int64_t ld, int64_t N, int* flag, hipStream_t s);
// Gershgorin interval of sym(H): out[0] = min_i (h_ii - r_i), out[1] = max_i (h_ii + r_i)
hipError_t gershgorin(const double* h, int64_t N, double* out, hipStream_t s);
// asymmetry max |x - x^T| and antisymmetric-part norm ||x - x^T||_F^2 partial
hipError_t asym_max(const double* x, int64_t N, double* out_max, hipStream_t s);
template <class T>
hipError_t antisym_sq_partials(const T* x, int64_t ld, int64_t N, double* partials, hipStream_t s);

// ---------------------------------------------------------------- block sparse (sparse.hip)
constexpr int kSparseBlock = 32;  // block edge of the thresholded block-sparse form

// Device view of a block-sparse matrix: rows[nb + 1] block-row pointers,
// cols[s] / ridx[s] block column / row of slot s (ascending columns within a
// row), val[s * 1024 ...] the 32 x 32 block, row major.
struct BSView {
  int* rows = nullptr;
  int* cols = nullptr;
  int* ridx = nullptr;
  double* val = nullptr;
};

// C = alpha[0] A[0] B[0] + alpha[1] A[1] B[1] + beta[0] C[0] + beta[1] C[1] + diag I
// (the first nterm products and nadd addends; I restricted to the n x n region).
struct BSExpr {
  int nterm = 0;
  BSView A[2], B[2];
  double alpha[2] = {1.0, 1.0};
  int nadd = 0;
  BSView C[2];
  double beta[2] = {1.0, 1.0};
  double diag = 0.0;
  int64_t n = 0;
};

int sparse_words(int nb);
// Candidate pattern of e: bit rows, block-row counts and their exclusive scan rows[0..nb].
hipError_t sparse_symbolic(const BSExpr& e, int nb, uint32_t* bits, int* counts, int* rows, hipStream_t s);
// cols / ridx of a pattern from its bit rows and scanned rows.
hipError_t sparse_fill(const uint32_t* bits, int nb, const int* rows, int* cols, int* ridx, hipStream_t s);
// Values of the candidate blocks of C (pattern given), their largest elements bmax, keep
// flags (bmax >= tau max(bmax); tau = 0: all), the number of 32 x 32 block products formed
// (per slot in nprods, summed into scal[0]) and the largest element in scal[1].
hipError_t sparse_numeric(const BSExpr& e, const BSView& C, int nslots, double tau, double* bmax, int* keep,
                          double* nprods, double* scal, hipStream_t s);
// Kept-block counts per row and their scan into out_rows[0..nb].
hipError_t sparse_keep_rows(const int* rows, const int* keep, int nb, int* counts, int* out_rows, hipStream_t s);
// The kept blocks of src into dst (dst.rows from sparse_keep_rows).
hipError_t sparse_compact(const BSView& src, const int* keep, int nb, const BSView& dst, hipStream_t s);
// Pattern of a sym(H) + shift I (H N x N dense FP64, may be null): the blocks whose largest
// element reaches tau times the largest element (tau = 0: non-zero blocks); bmax: nb^2
// doubles of scratch, gmax: one.
hipError_t sparse_dense_pattern(const double* H, int64_t N, int nb, double a, double shift, double tau,
                                double* bmax, double* gmax, uint32_t* bits, int* counts, int* rows,
                                hipStream_t s);
hipError_t sparse_dense_values(const double* H, int64_t N, double a, double shift, const BSView& m, int nslots,
                               hipStream_t s);
// out (N x N dense FP64) = a sym(m) + shift I.
hipError_t sparse_to_dense(const BSView& m, int nb, int64_t N, double a, double shift, double* out,
                           hipStream_t s);
// out[0] = trace over the n x n region, out[1] = sum of squares, out[2] = number of elements of
// shift I - m with magnitude >= thr, out[3] = sum of H .* m (H: n x n dense FP64, or null: 0);
// part: 4 nslots doubles of scratch.
hipError_t sparse_stats(const BSView& m, int nslots, int64_t n, double shift, double thr, const double* H,
                        double* part, double* out, hipStream_t s);

}  // namespace dmpt
