// Thresholded block-sparse algebra for the linear-scaling form of the
// recursion (Sec. V.B: for non-metallic systems the Hamiltonian, the density
// matrix and its responses are sparse above a numerical threshold, and every
// operation of Algorithm 1 is a matrix-matrix operation, so sparse algebra
// makes the cost grow linearly with the system size).
//
// A matrix is stored as 32 x 32 FP64 blocks in block-row order (CSR over
// blocks): rows[nb + 1] block-row pointers, cols[s] the block column and
// ridx[s] the block row of slot s, val[s] the block, row major.  Column
// indices are ascending within a block row, so a block is found by binary
// search and no dense index of the block grid is kept: memory grows with the
// number of stored blocks.  Blocks beyond the matrix edge are zero.
//
// Every product or combination
//     C = a1 A1 B1 + a2 A2 B2 + b1 C1 + b2 C2 + s I
// runs in three launches: a symbolic pass marks the candidate blocks of each
// block row in a bit row (union of the products' and addends' patterns), a
// fill pass turns the bit rows into the block list (after a scan of the row
// counts), and a numeric pass forms each candidate block with FP64 MFMA
// block products (v_mfma_f64_16x16x4f64, one wave per output block) and its
// largest element.  Truncation keeps the blocks whose largest element
// reaches tau times the largest element of the whole result (tau = 0 keeps
// every candidate), and a compaction packs them.
#include "dmpt_internal.h"

namespace dmpt {
namespace {

typedef double d4v __attribute__((__vector_size__(4 * sizeof(double))));

constexpr int kB = kSparseBlock;     // block edge
constexpr int kBB = kB * kB;         // elements per block
constexpr int kT = 256;

// Slot of block (i, j) of m, or -1 (binary search in block row i).
__device__ inline int find_block(const BSView& m, int i, int j) {
  int lo = m.rows[i], hi = m.rows[i + 1] - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int c = m.cols[mid];
    if (c == j) return mid;
    if (c < j) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

// ------------------------------------------------------------------ symbolic
// Block row i: bit j of bits[i * words + j / 32] is set when block (i, j) of C
// can be non-zero; counts[i] = number of set bits.  One workgroup per block
// row, the bit row built in LDS.
__global__ __launch_bounds__(kT) void k_symbolic(BSExpr e, int nb, int words, uint32_t* bits, int* counts) {
  extern __shared__ uint32_t row[];
  const int i = blockIdx.x;
  for (int w = threadIdx.x; w < words; w += kT) row[w] = 0u;
  __syncthreads();
  for (int t = 0; t < e.nterm; ++t) {
    const BSView& A = e.A[t];
    const BSView& B = e.B[t];
    const int a0 = A.rows[i], a1 = A.rows[i + 1];
    // (k slot, j slot) pairs spread over the threads
    for (int as = a0; as < a1; ++as) {
      const int k = A.cols[as];
      for (int bs = B.rows[k] + (int)threadIdx.x; bs < B.rows[k + 1]; bs += kT) {
        const int j = B.cols[bs];
        atomicOr(&row[j >> 5], 1u << (j & 31));
      }
    }
  }
  for (int t = 0; t < e.nadd; ++t) {
    const BSView& C = e.C[t];
    for (int cs = C.rows[i] + (int)threadIdx.x; cs < C.rows[i + 1]; cs += kT) {
      const int j = C.cols[cs];
      atomicOr(&row[j >> 5], 1u << (j & 31));
    }
  }
  __syncthreads();
  if (e.diag != 0.0 && threadIdx.x == 0) row[i >> 5] |= 1u << (i & 31);
  __syncthreads();
  int cnt = 0;
  for (int w = threadIdx.x; w < words; w += kT) {
    bits[(int64_t)i * words + w] = row[w];
    cnt += __popc(row[w]);
  }
  // block sum of the counts
  __shared__ int red[kT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int q = 0; q < kT / 64; ++q) s += red[q];
    counts[i] = s;
  }
}

// Exclusive scan of n ints into out[0..n] (out[n] = total), one workgroup.
__global__ __launch_bounds__(1024) void k_scan(const int* in, int n, int* out) {
  __shared__ int part[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024) {
    const int idx = base + (int)threadIdx.x;
    const int v = idx < n ? in[idx] : 0;
    part[threadIdx.x] = v;
    __syncthreads();
    // Hillis-Steele inclusive scan
    for (int off = 1; off < 1024; off <<= 1) {
      const int add = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
      __syncthreads();
      part[threadIdx.x] += add;
      __syncthreads();
    }
    if (idx < n) out[idx] = carry + part[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += part[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = carry;
}

// Block row i: the set bits of its bit row, ascending, become cols[rows[i] ..]
// (ridx = i).  One workgroup per block row; a scan of the word popcounts
// places each word's bits.
__global__ __launch_bounds__(kT) void k_fill(const uint32_t* bits, int words, const int* rows, int* cols,
                                             int* ridx) {
  __shared__ int pre[kT];
  __shared__ int carry;
  const int i = blockIdx.x;
  const uint32_t* row = bits + (int64_t)i * words;
  if (threadIdx.x == 0) carry = rows[i];
  __syncthreads();
  for (int base = 0; base < words; base += kT) {
    const int w = base + (int)threadIdx.x;
    const uint32_t v = w < words ? row[w] : 0u;
    const int pc = __popc(v);
    pre[threadIdx.x] = pc;
    __syncthreads();
    for (int off = 1; off < kT; off <<= 1) {
      const int add = threadIdx.x >= (unsigned)off ? pre[threadIdx.x - off] : 0;
      __syncthreads();
      pre[threadIdx.x] += add;
      __syncthreads();
    }
    int pos = carry + pre[threadIdx.x] - pc;
    uint32_t x = v;
    while (x) {
      const int b = __ffs(x) - 1;
      x &= x - 1;
      cols[pos] = w * 32 + b;
      ridx[pos] = i;
      ++pos;
    }
    __syncthreads();
    if (threadIdx.x == kT - 1) carry += pre[kT - 1];
    __syncthreads();
  }
}

// ------------------------------------------------------------------ numeric
// One wave per candidate block s of C: the block products of every term over
// the common inner blocks (FP64 MFMA, 2 x 2 tiles of 16 x 16, k in steps of
// 4), the addends and the diagonal; bmax[s] = max |C_s|, nprods[s] = block
// products formed.  Block products read their operand blocks straight from
// global memory (each is 8 KB contiguous).
__global__ __launch_bounds__(kT) void k_numeric(BSExpr e, BSView Cv, int nslots, double* bmax,
                                                double* nprods) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = blockIdx.x * (kT / 64) + wave;
  if (s >= nslots) return;
  const int i = Cv.ridx[s], j = Cv.cols[s];
  d4v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (d4v){0.0, 0.0, 0.0, 0.0};
  int nprod = 0;
  for (int t = 0; t < e.nterm; ++t) {
    const BSView& A = e.A[t];
    const BSView& B = e.B[t];
    const double alpha = e.alpha[t];
    for (int as = A.rows[i]; as < A.rows[i + 1]; ++as) {
      const int k = A.cols[as];
      const int bs = find_block(B, k, j);
      if (bs < 0) continue;
      ++nprod;
      const double* Ab = A.val + (int64_t)as * kBB;
      const double* Bb = B.val + (int64_t)bs * kBB;
#pragma unroll
      for (int kk = 0; kk < kB; kk += 4) {
        double av[2], bv[2];
        // A operand: lane l holds row (l % 16) and inner index kk + l / 16
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = alpha * Ab[(a * 16 + (lane & 15)) * kB + kk + (lane >> 4)];
        // B operand: lane l holds inner index kk + l / 16 and column (l % 16)
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = Bb[(kk + (lane >> 4)) * kB + b * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
  }
  // addends, diagonal, output and the block's largest element
  double* Cb = Cv.val + (int64_t)s * kBB;
  int cslot[2] = {-1, -1};
  for (int t = 0; t < e.nadd; ++t) cslot[t] = find_block(e.C[t], i, j);
  double mx = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // v_mfma_f64_16x16x4f64 result: register r of lane l holds row 4r + l/16, column l%16
        const int row = a * 16 + 4 * r + (lane >> 4), col = b * 16 + (lane & 15);
        double v = acc[a][b][r];
        for (int t = 0; t < e.nadd; ++t)
          if (cslot[t] >= 0) v += e.beta[t] * e.C[t].val[(int64_t)cslot[t] * kBB + row * kB + col];
        if (i == j && row == col && (int64_t)i * kB + row < e.n) v += e.diag;
        Cb[row * kB + col] = v;
        mx = fmax(mx, fabs(v));
      }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if (lane == 0) {
    bmax[s] = mx;
    nprods[s] = (double)nprod;
  }
}

// Largest of n values into out[0] (one workgroup, n = 0 gives 0).
__global__ __launch_bounds__(kT) void k_max(const double* p, int64_t n, double* out) {
  double m = 0.0;
  for (int64_t q = threadIdx.x; q < n; q += kT) m = fmax(m, p[q]);
  __shared__ double red[kT];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int off = kT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < (unsigned)off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// keep[s] = bmax[s] >= tau * gmax (tau > 0, relative to the matrix's largest
// element), else bmax[s] > 0 or always (tau = 0: every candidate block).
__global__ void k_keep(const double* bmax, int n, double tau, const double* gmax, int* keep) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  keep[s] = tau > 0.0 ? (bmax[s] >= tau * gmax[0] ? 1 : 0) : 1;
}

// Kept-block counts per block row.
__global__ void k_row_keep(const int* rows, const int* keep, int nb, int* counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  int c = 0;
  for (int s = rows[i]; s < rows[i + 1]; ++s) c += keep[s];
  counts[i] = c;
}

// Copy the kept blocks of src into dst (dst.rows already scanned), in order.
// One wave per block row walks its slots; the lanes copy each block.
__global__ __launch_bounds__(kT) void k_compact(BSView src, const int* keep, int nb, BSView dst) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * (kT / 64) + wave;
  if (i >= nb) return;
  int pos = dst.rows[i];
  for (int s = src.rows[i]; s < src.rows[i + 1]; ++s) {
    if (!keep[s]) continue;
    if (lane == 0) {
      dst.cols[pos] = src.cols[s];
      dst.ridx[pos] = i;
    }
    const double2* from = (const double2*)(src.val + (int64_t)s * kBB);
    double2* to = (double2*)(dst.val + (int64_t)pos * kBB);
    for (int q = lane; q < kBB / 2; q += 64) to[q] = from[q];
    ++pos;
  }
}

// ------------------------------------------------------------------ dense <-> blocks
// Block (i, j) of a * sym(H) + shift I (H: N x N FP64, leading dimension N,
// may be null) over the N x N region; max |.| of each block of the padded grid.
__global__ __launch_bounds__(kT) void k_dense_blockmax(const double* H, int64_t N, int nb, double a,
                                                       double shift, double* bmax) {
  const int64_t b = blockIdx.x;
  const int bi = (int)(b / nb), bj = (int)(b % nb);
  double mx = 0.0;
  for (int q = threadIdx.x; q < kBB; q += kT) {
    const int64_t r = (int64_t)bi * kB + q / kB, c = (int64_t)bj * kB + q % kB;
    if (r >= N || c >= N) continue;
    double v = H ? 0.5 * a * (H[r * N + c] + H[c * N + r]) : 0.0;
    if (r == c) v += shift;
    mx = fmax(mx, fabs(v));
  }
  __shared__ double red[kT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int q = 0; q < kT / 64; ++q) m = fmax(m, red[q]);
    bmax[b] = m;
  }
}

// Bit rows of the blocks whose max reaches tau * gmax (tau = 0: max > 0) and row counts.
__global__ __launch_bounds__(kT) void k_dense_bits(const double* bmax, int nb, int words, double tau,
                                                   const double* gmax, uint32_t* bits, int* counts) {
  const int i = blockIdx.x;
  int cnt = 0;
  for (int w = threadIdx.x; w < words; w += kT) {
    uint32_t v = 0u;
    for (int q = 0; q < 32; ++q) {
      const int j = w * 32 + q;
      if (j < nb) {
        const double m = bmax[(int64_t)i * nb + j];
        if (tau > 0.0 ? (m > 0.0 && m >= tau * gmax[0]) : m > 0.0) v |= 1u << q;
      }
    }
    bits[(int64_t)i * words + w] = v;
    cnt += __popc(v);
  }
  __shared__ int red[kT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int q = 0; q < kT / 64; ++q) s += red[q];
    counts[i] = s;
  }
}

// Values of the stored blocks from the dense matrix (one workgroup per slot).
__global__ __launch_bounds__(kT) void k_dense_vals(const double* H, int64_t N, double a, double shift,
                                                   BSView m) {
  const int s = blockIdx.x;
  const int bi = m.ridx[s], bj = m.cols[s];
  double* out = m.val + (int64_t)s * kBB;
  for (int q = threadIdx.x; q < kBB; q += kT) {
    const int64_t r = (int64_t)bi * kB + q / kB, c = (int64_t)bj * kB + q % kB;
    double v = 0.0;
    if (r < N && c < N) {
      v = H ? 0.5 * a * (H[r * N + c] + H[c * N + r]) : 0.0;
      if (r == c) v += shift;
    }
    out[q] = v;
  }
}

// out (N x N, leading dimension N) = a sym(M) + shift I, written in full:
// one workgroup per 32 x 32 tile of out; absent blocks give a zero tile.
__global__ __launch_bounds__(kT) void k_to_dense(BSView m, int nb, int64_t N, double a, double shift,
                                                 double* out) {
  const int bi = blockIdx.x / nb, bj = blockIdx.x % nb;
  const int s1 = find_block(m, bi, bj), s2 = find_block(m, bj, bi);
  for (int q = threadIdx.x; q < kBB; q += kT) {
    const int r = q / kB, c = q % kB;
    const int64_t R = (int64_t)bi * kB + r, C = (int64_t)bj * kB + c;
    if (R >= N || C >= N) continue;
    const double x = s1 >= 0 ? m.val[(int64_t)s1 * kBB + r * kB + c] : 0.0;
    const double y = s2 >= 0 ? m.val[(int64_t)s2 * kBB + c * kB + r] : 0.0;
    double v = 0.5 * a * (x + y);
    if (R == C) v += shift;
    out[R * N + C] = v;
  }
}

// ------------------------------------------------------------------ reductions
// Per slot: partial sums of the diagonal (i < n), of the squares and of
// H .* m (H: n x n dense, may be null), and the number of elements of
// shift I - m (a density matrix I/2 - D, or a response -D^(k) with shift 0)
// whose magnitude reaches thr.
__global__ __launch_bounds__(kT) void k_stats(BSView m, int nslots, int64_t n, double shift, double thr,
                                              const double* H, double* tr_part, double* sq_part,
                                              double* cnt_part, double* h_part) {
  const int s = blockIdx.x;
  if (s >= nslots) return;
  const int bi = m.ridx[s], bj = m.cols[s];
  const double* v = m.val + (int64_t)s * kBB;
  double tr = 0.0, sq = 0.0, c = 0.0, hd = 0.0;
  for (int q = threadIdx.x; q < kBB; q += kT) {
    const int r = q / kB, cc = q % kB;
    const int64_t R = (int64_t)bi * kB + r, C = (int64_t)bj * kB + cc;
    if (R >= n || C >= n) continue;
    const double x = v[q];
    sq += x * x;
    if (H) hd += H[R * n + C] * x;
    double y = -x;
    if (R == C) {
      tr += x;
      y += shift;
    }
    if (fabs(y) >= thr) c += 1.0;
  }
  __shared__ double rt[kT / 64], rs[kT / 64], rc[kT / 64], rh[kT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    tr += __shfl_xor(tr, o, 64);
    sq += __shfl_xor(sq, o, 64);
    c += __shfl_xor(c, o, 64);
    hd += __shfl_xor(hd, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    rt[threadIdx.x >> 6] = tr;
    rs[threadIdx.x >> 6] = sq;
    rc[threadIdx.x >> 6] = c;
    rh[threadIdx.x >> 6] = hd;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0, k = 0.0, h = 0.0;
    for (int q = 0; q < kT / 64; ++q) {
      a += rt[q];
      b += rs[q];
      k += rc[q];
      h += rh[q];
    }
    tr_part[s] = a;
    sq_part[s] = b;
    cnt_part[s] = k;
    h_part[s] = h;
  }
}

// Deterministic sum of n partials into out[0] (one workgroup, fixed order).
__global__ __launch_bounds__(kT) void k_sum(const double* p, int n, double* out) {
  double s = 0.0;
  for (int q = threadIdx.x; q < n; q += kT) s += p[q];
  __shared__ double red[kT];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = kT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < (unsigned)off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace

int sparse_words(int nb) { return (nb + 31) / 32; }

hipError_t sparse_symbolic(const BSExpr& e, int nb, uint32_t* bits, int* counts, int* rows,
                           hipStream_t s) {
  const int words = sparse_words(nb);
  const size_t lds = (size_t)words * sizeof(uint32_t);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_symbolic, dim3(nb), dim3(kT), lds, s, e, nb, words, bits, counts);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, nb, rows);
  return hipGetLastError();
}

hipError_t sparse_fill(const uint32_t* bits, int nb, const int* rows, int* cols, int* ridx, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(nb), dim3(kT), 0, s, bits, sparse_words(nb), rows, cols, ridx);
  return hipGetLastError();
}

hipError_t sparse_numeric(const BSExpr& e, const BSView& C, int nslots, double tau, double* bmax, int* keep,
                          double* nprods, double* scal, hipStream_t s) {
  if (nslots > 0)
    hipLaunchKernelGGL(k_numeric, dim3((nslots + kT / 64 - 1) / (kT / 64)), dim3(kT), 0, s, e, C, nslots, bmax,
                       nprods);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kT), 0, s, nprods, nslots, scal);
  hipLaunchKernelGGL(k_max, dim3(1), dim3(kT), 0, s, bmax, (int64_t)nslots, scal + 1);
  if (nslots > 0)
    hipLaunchKernelGGL(k_keep, dim3((nslots + 255) / 256), dim3(256), 0, s, bmax, nslots, tau, scal + 1, keep);
  return hipGetLastError();
}

hipError_t sparse_keep_rows(const int* rows, const int* keep, int nb, int* counts, int* out_rows,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_row_keep, dim3((nb + 255) / 256), dim3(256), 0, s, rows, keep, nb, counts);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, nb, out_rows);
  return hipGetLastError();
}

hipError_t sparse_compact(const BSView& src, const int* keep, int nb, const BSView& dst, hipStream_t s) {
  hipLaunchKernelGGL(k_compact, dim3((nb + kT / 64 - 1) / (kT / 64)), dim3(kT), 0, s, src, keep, nb, dst);
  return hipGetLastError();
}

hipError_t sparse_dense_pattern(const double* H, int64_t N, int nb, double a, double shift, double tau,
                                double* bmax, double* gmax, uint32_t* bits, int* counts, int* rows,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_dense_blockmax, dim3((unsigned)((int64_t)nb * nb)), dim3(kT), 0, s, H, N, nb, a, shift,
                     bmax);
  hipLaunchKernelGGL(k_max, dim3(1), dim3(kT), 0, s, bmax, (int64_t)nb * nb, gmax);
  hipLaunchKernelGGL(k_dense_bits, dim3(nb), dim3(kT), 0, s, bmax, nb, sparse_words(nb), tau, gmax, bits,
                     counts);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, nb, rows);
  return hipGetLastError();
}

hipError_t sparse_dense_values(const double* H, int64_t N, double a, double shift, const BSView& m, int nslots,
                               hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dense_vals, dim3(nslots), dim3(kT), 0, s, H, N, a, shift, m);
  return hipGetLastError();
}

hipError_t sparse_to_dense(const BSView& m, int nb, int64_t N, double a, double shift, double* out,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_to_dense, dim3((unsigned)((int64_t)nb * nb)), dim3(kT), 0, s, m, nb, N, a, shift, out);
  return hipGetLastError();
}

hipError_t sparse_stats(const BSView& m, int nslots, int64_t n, double shift, double thr, const double* H,
                        double* part, double* out, hipStream_t s) {
  if (nslots > 0)
    hipLaunchKernelGGL(k_stats, dim3(nslots), dim3(kT), 0, s, m, nslots, n, shift, thr, H, part, part + nslots,
                       part + 2 * (int64_t)nslots, part + 3 * (int64_t)nslots);
  for (int q = 0; q < 4; ++q)
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kT), 0, s, part + q * (int64_t)nslots, nslots > 0 ? nslots : 0,
                       out + q);
  return hipGetLastError();
}

}  // namespace dmpt
