// Bandwidth-bound kernels of the DMPT path: symmetrised initialisation and
// output, BF16 splitting, conjugate-gradient vector updates, and FP64
// reductions (traces, Frobenius products) for the Newton update of the mu
// jet (Algorithm 1) and the response observables (Eq. Resp_0).
//
// Reductions never use floating-point atomics: each block writes one FP64
// partial and a second kernel sums a fixed-size partial array in a fixed
// order, so every result is bitwise reproducible.
#include "dmpt_internal.h"

namespace dmpt {
namespace {

constexpr int kT = 256;
constexpr int kMaxRedBlocks = 1024;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the block; the result is valid in thread 0.
__device__ inline double block_sum(double v) {
  __shared__ double red[kT / 64];
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

__device__ inline uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// BF16 slices of v: slice p rounds what the earlier slices left (FP64
// remainder); off is the element's offset in the plane layout.
__device__ inline void split_store(double v, uint16_t* const* pl, int np, int64_t off) {
  double r = v;
  for (int p = 0; p < np; ++p) {
    const uint16_t h = bf16_rne((float)r);
    pl[p][off] = h;
    r -= (double)bf16_to_f(h);
  }
}

// Plane offset of linear element i of an Np x Np member (Np^2 < 2^32).
__device__ inline int64_t plane_off_lin(int64_t i, int64_t Np) {
  const uint32_t u = (uint32_t)i, n = (uint32_t)Np;
  const uint32_t r = u / n;
  return plane_off(r, u - r * n, Np);
}

struct Planes {
  uint16_t* p[3];
};

// Two consecutive elements per thread and load (the launchers take this path
// when every base and stride is 16-byte aligned and n is even): a wave's
// load instruction then covers one contiguous 1 KB (FP64) or 512 B (FP32)
// span, and the two BF16 slices of a plane go out as one 4-byte store (two
// consecutive columns are adjacent in the plane layout when the first is
// even).
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

// Largest |x| of a block; any NaN or infinity makes it infinite, so the
// member's q becomes infinite and its products non-finite.
__device__ inline double block_max(double v) {
  __shared__ double red[kT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) m = fmax(m, red[i]);
  return m;
}

template <class T>
__device__ inline void ld2(const T* __restrict__ p, T (&v)[2]) {
  if constexpr (sizeof(T) == 8) {
    const d2v t = *(const d2v*)p;
    v[0] = t[0];
    v[1] = t[1];
  } else {
    const f2v t = *(const f2v*)p;
    v[0] = t[0];
    v[1] = t[1];
  }
}

template <class T>
__device__ inline void st2(T* __restrict__ p, const T (&v)[2]) {
  if constexpr (sizeof(T) == 8) *(d2v*)p = d2v{v[0], v[1]};
  else *(f2v*)p = f2v{v[0], v[1]};
}

// split_store for two consecutive columns; off = plane offset of the first
template <class T>
__device__ inline void split_store2(const T (&v)[2], uint16_t* const* pl, int np, int64_t off) {
  double r0 = (double)v[0], r1 = (double)v[1];
  for (int p = 0; p < np; ++p) {
    const uint16_t h0 = bf16_rne((float)r0), h1 = bf16_rne((float)r1);
    r0 -= (double)bf16_to_f(h0);
    r1 -= (double)bf16_to_f(h1);
    *(uint32_t*)(pl[p] + off) = (uint32_t)h0 | ((uint32_t)h1 << 16);
  }
}

// The pair path's precondition for one batched operand: n even, and the
// base and member stride aligned to two elements.
template <class T>
inline bool pair_ok(const T* p, int64_t stride, int64_t n) {
  return n % 2 == 0 && stride % 2 == 0 && ((uintptr_t)p % (2 * sizeof(T))) == 0;
}

// ------------------------------------------------------------ symmetrise
// Block t owns the 32 g x 32 g tile pair (BI, BJ) and (BJ, BI), BI <= BJ,
// t = BJ (BJ + 1) / 2 + BI, and walks its 32 x 32 pairs (bi, bj), bi <= bj
// (g = 4 when the block leaves a maximum, else 1: one pair per block):
// both input tiles of a pair are read before either output tile is written,
// and the pairs are disjoint (reading the next pair while writing this one
// touches other elements), so the kernel may run in place.  Reads and writes
// stay row-contiguous.  With mx, the block leaves max |out| over its pair (an
// infinite one for a non-finite value) at mx[z * mstride + t].
template <class Tin, class Tout>
__global__ __launch_bounds__(kT) void k_sym(const Tin* in, int64_t ldi, int64_t si, int64_t N,
                                            int64_t Np, double a, const double* dshift,
                                            int dstride, Tout* out, int64_t ldo, int64_t so,
                                            Planes pl, int np, int64_t out_rows, const Tin* in2,
                                            double a2, const int* gate, int64_t nb, int g, double* mx,
                                            int64_t mstride) {
  __shared__ double ta[32][33], tb[32][33];
  if (gate && !*gate) return;  // a converged system of a batch keeps its outputs
  const int64_t t = blockIdx.x;
  int64_t BJ = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (BJ > 0 && BJ * (BJ + 1) / 2 > t) --BJ;
  while ((BJ + 1) * (BJ + 2) / 2 <= t) ++BJ;
  const int64_t BI = t - BJ * (BJ + 1) / 2;
  const int z = blockIdx.y;
  in += z * si;
  if (in2) in2 += z * si;
  out += z * so;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const double ds = dshift ? dshift[z * dstride] : 0.0;
  uint16_t* p3[3] = {pl.p[0] ? pl.p[0] + z * so : nullptr, pl.p[1] ? pl.p[1] + z * so : nullptr,
                     pl.p[2] ? pl.p[2] + z * so : nullptr};
  // the block's pairs (bi, bj) = (4 BI + q / 4, 4 BJ + q % 4), bi <= bj, in
  // order of q; the next pair's inputs are loaded into registers while the
  // current pair is written
  auto valid = [&](int q) {
    const int64_t bi = BI * g + q / g, bj = BJ * g + q % g;
    return bi <= bj && bj < nb;
  };
  auto next = [&](int q) {
    do ++q;
    while (q < g * g && !valid(q));
    return q;
  };
  auto load = [&](int q, double (&ra)[4], double (&rb)[4]) {
    const int64_t bi = BI * g + q / g, bj = BJ * g + q % g;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = ty + 8 * u;
      // ra = a in(bi,bj) + a2 in2(bi,bj), rb likewise for (bj,bi)
      int64_t gi = bi * 32 + r, gj = bj * 32 + tx;
      bool ok = gi < N && gj < N;
      ra[u] = ok ? a * (double)in[gi * ldi + gj] + (in2 ? a2 * (double)in2[gi * ldi + gj] : 0.0) : 0.0;
      gi = bj * 32 + r;
      gj = bi * 32 + tx;
      ok = gi < N && gj < N;
      rb[u] = ok ? a * (double)in[gi * ldi + gj] + (in2 ? a2 * (double)in2[gi * ldi + gj] : 0.0) : 0.0;
    }
  };
  double m = 0.0;
  bool bad = false;
  double ra[4], rb[4];
  int q = valid(0) ? 0 : next(0);
  if (q < g * g) load(q, ra, rb);
  while (q < g * g) {  // the same pairs for every thread of the block
    const int qn = next(q);
    const int64_t bi = BI * g + q / g, bj = BJ * g + q % g;
    __syncthreads();  // the previous pair is written: ta, tb are free
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ta[ty + 8 * u][tx] = ra[u];
      tb[ty + 8 * u][tx] = rb[u];
    }
    __syncthreads();
    if (qn < g * g) load(qn, ra, rb);
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 1 && bi == bj) break;
      const int64_t ti = pass ? bj : bi, tj = pass ? bi : bj;
      for (int r = ty; r < 32; r += 8) {
        const int64_t gi = ti * 32 + r, gj = tj * 32 + tx;
        if (gi >= out_rows || gj >= out_rows) continue;
        double v = 0.0;
        if (gi < N && gj < N) {
          // out(ti,tj)[r][tx] = ta(ti,tj)[r][tx] + ta(tj,ti)[tx][r] (scales already applied)
          v = pass ? (tb[r][tx] + ta[tx][r]) : (ta[r][tx] + tb[tx][r]);
          if (gi == gj) v += ds;
        }
        const Tout o = (Tout)v;
        out[gi * ldo + gj] = o;
        if (np) split_store((double)o, p3, np, plane_off(gi, gj, ldo));
        const double ao = fabs((double)o);
        bad |= !(ao <= 1.0e308);
        m = fmax(m, ao);
      }
    }
    q = qn;
  }
  if (mx) {
    const double bm = block_max(bad ? INFINITY : m);
    if (threadIdx.x == 0) mx[z * mstride + t] = bm;
  }
}

// out = in^T on Np x Np (batched, with planes); out and in must differ.
template <class T>
__global__ __launch_bounds__(kT) void k_transpose(const T* __restrict__ in, int64_t Np, int64_t s,
                                                  T* __restrict__ out, Planes pl, int np) {
  __shared__ T t[32][33];
  const int z = blockIdx.z;
  in += z * s;
  out += z * s;
  const int64_t bi = blockIdx.y, bj = blockIdx.x;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) t[r][tx] = in[(bi * 32 + r) * Np + bj * 32 + tx];
  __syncthreads();
  uint16_t* p3[3] = {pl.p[0] ? pl.p[0] + z * s : nullptr, pl.p[1] ? pl.p[1] + z * s : nullptr,
                     pl.p[2] ? pl.p[2] + z * s : nullptr};
  for (int r = ty; r < 32; r += 8) {
    const int64_t idx = (bj * 32 + r) * Np + bi * 32 + tx;
    const T v = t[tx][r];
    out[idx] = v;
    if (np) split_store((double)v, p3, np, plane_off(bj * 32 + r, bi * 32 + tx, Np));
  }
}

__global__ __launch_bounds__(kT) void k_split(const double* __restrict__ x, int64_t n, int64_t sx,
                                              Planes pl, int64_t sp, int np, int64_t Np) {
  const int z = blockIdx.y;
  x += z * sx;
  uint16_t* p3[3] = {pl.p[0] ? pl.p[0] + z * sp : nullptr, pl.p[1] ? pl.p[1] + z * sp : nullptr,
                     pl.p[2] ? pl.p[2] + z * sp : nullptr};
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    split_store(x[i], p3, np, plane_off_lin(i, Np));
}

// ------------------------------------------------------------ reductions
template <class T>
__global__ __launch_bounds__(kT) void k_dot(const T* __restrict__ x, int64_t sx,
                                            const T* __restrict__ y, int64_t sy, int64_t n,
                                            double* partials, int v2) {
  const int z = blockIdx.y;
  x += z * sx;
  y += z * sy;
  double s = 0.0;
  if (v2) {
    for (int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x; c < (n >> 1); c += (int64_t)gridDim.x * kT) {
      T a2[2], b2[2];
      ld2(x + (c << 1), a2);
      ld2(y + (c << 1), b2);
      s += (double)a2[0] * (double)b2[0];
      s += (double)a2[1] * (double)b2[1];
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
      s += (double)x[i] * (double)y[i];
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[(int64_t)z * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(kT) void k_sum_partials(const double* __restrict__ p, int count,
                                                     double* out, int ostride, int oidx) {
  const int z = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += kT) s += p[(int64_t)z * count + i];
  s = block_sum(s);
  if (threadIdx.x == 0) out[z * ostride + oidx] = s;
}

template <class T>
__global__ __launch_bounds__(kT) void k_trace(const T* __restrict__ x, int64_t ld, int64_t sx,
                                              int64_t N, double* out, int ostride, double* aout) {
  const int z = blockIdx.x;
  x += z * sx;
  double s = 0.0, sa = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += kT) {
    const double v = (double)x[i * ld + i];
    s += v;
    sa += fabs(v);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) out[z * ostride] = s;
  if (aout) {
    sa = block_sum(sa);
    if (threadIdx.x == 0) aout[z * ostride] = sa;
  }
}

// ------------------------------------------------------------ CG
template <class T>
__global__ __launch_bounds__(kT) void k_cg_xr(T* __restrict__ U, T* __restrict__ R,
                                              const T* __restrict__ P, const T* __restrict__ Q,
                                              int64_t n, int64_t stride, const double* rr,
                                              const double* pq, int hstride, const int* active,
                                              double* partials, double* rmax) {
  const int z = blockIdx.y;
  if (active && !active[z]) {
    if (threadIdx.x == 0) partials[(int64_t)z * gridDim.x + blockIdx.x] = 0.0;
    return;
  }
  const double den = pq[z * hstride];
  const double alpha = den != 0.0 ? rr[z * hstride] / den : 0.0;
  const T al = (T)alpha;
  U += z * stride;
  R += z * stride;
  P += z * stride;
  Q += z * stride;
  double s = 0.0, m = 0.0;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    U[i] += al * P[i];
    const T r = R[i] - al * Q[i];
    R[i] = r;
    s += (double)r * (double)r;
    const double ar = fabs((double)r);
    bad |= !(ar <= 1.0e308);  // NaN or infinity: the slicing scale becomes infinite
    m = fmax(m, ar);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[(int64_t)z * gridDim.x + blockIdx.x] = s;
  if (rmax) {
    m = block_max(bad ? INFINITY : m);
    if (threadIdx.x == 0) rmax[(int64_t)z * gridDim.x + blockIdx.x] = m;
  }
}

template <class T>
__global__ __launch_bounds__(kT) void k_cg_p(T* __restrict__ P, const T* __restrict__ R, int64_t n,
                                             int64_t stride, const double* rr_new,
                                             const double* rr_old, int hstride, const int* active,
                                             Planes pl, int np, int64_t Np, int v2) {
  const int z = blockIdx.y;
  if (active && !active[z]) return;
  const double ro = rr_old[z * hstride];
  const double beta = ro != 0.0 ? rr_new[z * hstride] / ro : 0.0;
  const T be = (T)beta;
  P += z * stride;
  R += z * stride;
  uint16_t* p3[3] = {pl.p[0] ? pl.p[0] + z * stride : nullptr,
                     pl.p[1] ? pl.p[1] + z * stride : nullptr,
                     pl.p[2] ? pl.p[2] + z * stride : nullptr};
  if (v2) {
    for (int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x; c < (n >> 1); c += (int64_t)gridDim.x * kT) {
      const int64_t i = c << 1;
      T r[2], p[2];
      ld2(R + i, r);
      ld2(P + i, p);
#pragma unroll
      for (int e = 0; e < 2; ++e) p[e] = r[e] + be * p[e];
      st2(P + i, p);
      if (np) split_store2(p, p3, np, plane_off_lin(i, Np));
    }
    return;
  }
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const T p = R[i] + be * P[i];
    P[i] = p;
    if (np) split_store((double)p, p3, np, plane_off_lin(i, Np));
  }
}

// A member stays active while ||r||^2 > tol2 ||rhs||^2 or ||r||^2 > eta2 ||r_0||^2:
// a warm-started solve must also shrink its own initial residual, so the
// solution follows small changes of the right-hand side (a mu update)
// instead of keeping the previous solution within the tolerance.
__global__ void k_cg_check(const double* rr, const double* rr0, const double* ref, int hstride,
                           int batch, double tol2, double eta2, int* active, int* iters) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= batch || !active[z]) return;
  iters[z] += 1;
  const double r = rr[z * hstride];
  if (!(r > tol2 * ref[z] || r > eta2 * rr0[z * hstride])) active[z] = 0;
}

// Device-side verdict on the inputs of a call that reads nothing back: a
// non-finite value (flag set) gives DMPT_ERR_NONFINITE, beta max|eps - mu| >=
// 2^(n+1) over the Gershgorin interval g[0..1] gives DMPT_ERR_RANGE, else 0.
__global__ void k_input_status(const double* g, const int* flag, double beta, double mu, int n,
                               int* status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double emax = fmax(fabs(g[0] - mu), fabs(g[1] - mu));
  int st = 0;
  if (*flag) st = DMPT_ERR_NONFINITE;
  else if (!(beta * emax < ldexp(1.0, n + 1))) st = DMPT_ERR_RANGE;
  *status = st;
}

// Statistics of a fixed-count (graph-replayed) solve: iterations summed and
// their maximum over the members that ran, and the members still above their
// tolerance at the end (iters counts the initial check as well).
__global__ void k_cg_account(const int* active, const int* iters, int batch, int* stat) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= batch) return;
  const int its = max(0, iters[z] - 1);
  if (its > 0) {
    atomicAdd(stat, its);
    atomicMax(stat + 1, its);
  }
  if (active[z]) atomicAdd(stat + 2, 1);
}

template <class T>
__global__ __launch_bounds__(kT) void k_axpby(const T* __restrict__ x, int64_t sx, T* __restrict__ y,
                                              int64_t sy, int64_t n, double a, double b, Planes pl,
                                              int64_t sp, int np, int64_t Np, int v2) {
  const int z = blockIdx.y;
  x += z * sx;
  y += z * sy;
  uint16_t* p3[3] = {pl.p[0] ? pl.p[0] + z * sp : nullptr, pl.p[1] ? pl.p[1] + z * sp : nullptr,
                     pl.p[2] ? pl.p[2] + z * sp : nullptr};
  const T ta = (T)a, tb = (T)b;
  if (v2) {
    for (int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x; c < (n >> 1); c += (int64_t)gridDim.x * kT) {
      const int64_t i = c << 1;
      T xv[2], yv[2];
      ld2(x + i, xv);
      if (b != 0.0) ld2(y + i, yv);  // b = 0: y is not read
#pragma unroll
      for (int e = 0; e < 2; ++e) yv[e] = (b != 0.0) ? ta * xv[e] + tb * yv[e] : ta * xv[e];
      st2(y + i, yv);
      if (np) split_store2(yv, p3, np, plane_off_lin(i, Np));
    }
    return;
  }
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const T v = (b != 0.0) ? ta * x[i] + tb * y[i] : ta * x[i];  // b = 0: y is not read
    y[i] = v;
    if (np) split_store((double)v, p3, np, plane_off_lin(i, Np));
  }
}

// out = a x + b y (one member), with planes of out: the same arithmetic as
// k_axpby with y read from a third array.  With mx, block b leaves max |out|
// over its elements (infinite for a non-finite one) at mx[b].
template <class T>
__global__ __launch_bounds__(kT) void k_axpbyz(const T* __restrict__ x, const T* __restrict__ y,
                                               T* __restrict__ out, int64_t n, double a, double b, Planes pl,
                                               int np, int64_t Np, int v2, double* __restrict__ mx) {
  uint16_t* p3[3] = {pl.p[0], pl.p[1], pl.p[2]};
  const T ta = (T)a, tb = (T)b;
  double m = 0.0;
  bool bad = false;
  if (v2) {
    for (int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x; c < (n >> 1); c += (int64_t)gridDim.x * kT) {
      const int64_t i = c << 1;
      T xv[2], yv[2];
      ld2(x + i, xv);
      ld2(y + i, yv);
#pragma unroll
      for (int e = 0; e < 2; ++e) yv[e] = ta * xv[e] + tb * yv[e];
      st2(out + i, yv);
      if (np) split_store2(yv, p3, np, plane_off_lin(i, Np));
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const double av = fabs((double)yv[e]);
        bad |= !(av <= 1.0e308);
        m = fmax(m, av);
      }
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
      const T v = ta * x[i] + tb * y[i];
      out[i] = v;
      if (np) split_store((double)v, p3, np, plane_off_lin(i, Np));
      const double av = fabs((double)v);
      bad |= !(av <= 1.0e308);
      m = fmax(m, av);
    }
  }
  if (mx) {
    const double bm = block_max(bad ? INFINITY : m);
    if (threadIdx.x == 0) mx[blockIdx.x] = bm;
  }
}

// out = (Tout) in, batched, with planes of out.  With mx, block b of member z
// leaves max |out| over its elements (infinite for a non-finite one) at
// mx[z * mstride + b].
template <class Tin, class Tout>
__global__ __launch_bounds__(kT) void k_convert(const Tin* __restrict__ in, int64_t si,
                                                Tout* __restrict__ out, int64_t so, int64_t n,
                                                Planes pl, int64_t sp, int np, int64_t Np, int v2,
                                                double* __restrict__ mx, int64_t mstride) {
  const int z = blockIdx.y;
  in += z * si;
  out += z * so;
  uint16_t* p3[3] = {pl.p[0] ? pl.p[0] + z * sp : nullptr, pl.p[1] ? pl.p[1] + z * sp : nullptr,
                     pl.p[2] ? pl.p[2] + z * sp : nullptr};
  double m = 0.0;
  bool bad = false;
  if (v2) {
    for (int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x; c < (n >> 1); c += (int64_t)gridDim.x * kT) {
      const int64_t i = c << 1;
      Tin a2[2];
      Tout o2[2];
      ld2(in + i, a2);
      o2[0] = (Tout)a2[0];
      o2[1] = (Tout)a2[1];
      st2(out + i, o2);
      if (np) split_store2(o2, p3, np, plane_off_lin(i, Np));
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const double av = fabs((double)o2[e]);
        bad |= !(av <= 1.0e308);
        m = fmax(m, av);
      }
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
      const Tout v = (Tout)in[i];
      out[i] = v;
      if (np) split_store((double)v, p3, np, plane_off_lin(i, Np));
      const double av = fabs((double)v);
      bad |= !(av <= 1.0e308);
      m = fmax(m, av);
    }
  }
  if (mx) {
    const double bm = block_max(bad ? INFINITY : m);
    if (threadIdx.x == 0) mx[z * mstride + blockIdx.x] = bm;
  }
}

template <class T>
__global__ __launch_bounds__(kT) void k_spi(const T* __restrict__ x, T* __restrict__ out, int64_t N,
                                            int64_t Np, double a, double b, Planes pl, int np,
                                            double* __restrict__ mx) {
  const int64_t n = Np * Np;
  double m = 0.0;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const int64_t r = i / Np, c = i % Np;
    double v = (b != 0.0) ? b * (double)x[i] : 0.0;
    if (r == c && r < N) v += a;
    const T o = (T)v;
    out[i] = o;
    if (np) split_store((double)o, pl.p, np, plane_off(r, c, Np));
    const double ao = fabs((double)o);
    bad |= !(ao <= 1.0e308);
    m = fmax(m, ao);
  }
  if (mx) {  // block b: max |out| over its elements at mx[b]
    const double bm = block_max(bad ? INFINITY : m);
    if (threadIdx.x == 0) mx[blockIdx.x] = bm;
  }
}

// out (Np x Np, ld Np) = in (N x N, ld ldi) or its transpose, zero outside
// the leading N x N block; 32 x 32 tiles staged in LDS so both sides stay
// row-contiguous.
__global__ __launch_bounds__(kT) void k_pad_copy(const double* __restrict__ in, int64_t ldi, int64_t N,
                                                 double* __restrict__ out, int64_t Np, int trans) {
  __shared__ double t[32][33];
  const int64_t bi = blockIdx.y, bj = blockIdx.x;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  // source tile: (bi, bj) or, transposed, (bj, bi)
  const int64_t si = trans ? bj : bi, sj = trans ? bi : bj;
  for (int r = ty; r < 32; r += 8) {
    const int64_t gi = si * 32 + r, gj = sj * 32 + tx;
    t[r][tx] = (gi < N && gj < N) ? in[gi * ldi + gj] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t gi = bi * 32 + r, gj = bj * 32 + tx;
    out[gi * Np + gj] = trans ? t[tx][r] : t[r][tx];
  }
}

__global__ __launch_bounds__(kT) void k_nonfinite(const double* __restrict__ x, int64_t ld, int64_t N,
                                                  int* flag) {
  int bad = 0;
  const int64_t n = N * N;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const double v = x[(i / N) * ld + (i % N)];
    if (!isfinite(v)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

// Gershgorin bounds of sym(H): per row i, c_i = h_ii, r_i = sum_{j != i} |h_ij + h_ji|/2.
__global__ __launch_bounds__(kT) void k_gersh_rows(const double* __restrict__ h, int64_t N,
                                                   double* lo, double* hi) {
  const int64_t i = blockIdx.x;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < N; j += kT)
    if (j != i) s += fabs(0.5 * (h[i * N + j] + h[j * N + i]));
  s = block_sum(s);
  if (threadIdx.x == 0) {
    const double c = h[i * N + i];
    lo[i] = c - s;
    hi[i] = c + s;
  }
}

__global__ __launch_bounds__(kT) void k_minmax(const double* lo, const double* hi, int64_t N,
                                               double* out) {
  __shared__ double smin[kT], smax[kT];
  double mn = 1e300, mx = -1e300;
  for (int64_t i = threadIdx.x; i < N; i += kT) {
    mn = fmin(mn, lo[i]);
    mx = fmax(mx, hi[i]);
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = smin[0];
    out[1] = smax[0];
  }
}

__global__ __launch_bounds__(kT) void k_asym_max(const double* __restrict__ x, int64_t N, double* out) {
  __shared__ double sm[kT];
  double m = 0.0;
  const int64_t n = N * N;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const int64_t r = i / N, c = i % N;
    m = fmax(m, fabs(x[r * N + c] - x[c * N + r]));
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

template <class T>
__global__ __launch_bounds__(kT) void k_antisym_sq(const T* __restrict__ x, int64_t ld, int64_t N,
                                                   double* partials) {
  double s = 0.0;
  const int64_t n = N * N;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const int64_t r = i / N, c = i % N;
    const double d = (double)x[r * ld + c] - (double)x[c * ld + r];
    s += d * d;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void k_set(int* p, int v, int n, double* q, double qv, int nq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
  if (i < nq) q[i] = qv;
}

__global__ void k_expand(const int* src, int div, int* dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i / div];
}

// Deterministic non-trivial fill (a hashed pattern in [-1, 1)) with planes.
template <class T>
__global__ __launch_bounds__(kT) void k_fill(T* x, int64_t n, uint32_t seed, Planes pl, int np,
                                             int64_t Np) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    uint32_t h = (uint32_t)i * 2654435761u ^ seed;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    const T v = (T)((double)(h & 0xffffff) / 8388608.0 - 1.0);
    x[i] = v;
    if (np) split_store((double)v, pl.p, np, plane_off_lin(i, Np));
  }
}

// Canonical Newton update of every system of a batch (Algorithm 1's mu
// update with Tr P_mu = beta (Tr P0 - ||P0||_F^2)), one thread per system.
// tr[s*rs + ...]: Tr P^(k) (J values), sum |P^(k)_ii| (J), ||P0||_F^2.
// par[s*6 + ...]: beta, Ne, c = 2^-(n+2) beta, mu0 lower bound, mu0 upper bound, N.
// brk[s*2 + ...]: the current bracket of mu0 (starts as the bounds);
// prev_err[s]: the previous pass's normalised error (starts at +inf).
__global__ void k_newton(const double* tr, int rs, const double* par, double* mu, double* shift,
                         int J, int nk, double tol, int final_stage, int* active, int* done,
                         double* prev_err, double* brk, double* occ, int* passes, int* status,
                         int nsys) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys || !active[s]) return;
  const double* t = tr + (int64_t)s * rs;
  const double beta = par[s * 6 + 0], Ne = par[s * 6 + 1], c = par[s * 6 + 2];
  const double lo = par[s * 6 + 3], hi = par[s * 6 + 4], N = par[s * 6 + 5];
  // occupation error (absolute) and its normalised form
  double err = fabs(t[0] - Ne);
  double rel = err / N;
  for (int i = 1; i <= nk; ++i) {
    const double a = fabs(t[i]);
    err += a;
    rel = fmax(rel, a / fmax(t[J + i], 1e-300));
  }
  passes[s] += 1;
  occ[s] = err;
  if (!isfinite(err) || !isfinite(t[2 * J])) {
    status[s] = -6;
    active[s] = 0;
    return;
  }
  bool ok = rel <= tol;
  // noise floor: stopped shrinking within 1000 tol (the traces carry the
  // products' rounding); status 1 records such an acceptance
  const bool floor_ok = !ok && rel > 0.5 * prev_err[s] && rel <= 1e3 * tol;
  prev_err[s] = rel;
  if (ok || floor_ok) {
    active[s] = 0;
    done[s] = final_stage;
    if (final_stage && floor_ok) status[s] = 1;
    return;
  }
  double* m = mu + (int64_t)s * J;
  double* sh = shift + (int64_t)s * J;
  // bracket of mu0 from the signs of Tr P0 - Ne (Tr P0 grows with mu0); a
  // Newton step outside it, or a vanishing Tr P_mu, becomes a bisection
  double* b = brk + 2 * (int64_t)s;
  if (t[0] < Ne) b[0] = fmax(b[0], m[0]);
  else b[1] = fmin(b[1], m[0]);
  const double trpmu = beta * (t[0] - t[2 * J]);
  const double mn = m[0] + (Ne - t[0]) / trpmu;
  // once Tr P0 meets its own tolerance the (tiny) step is always taken
  const bool occ_met = fabs(t[0] - Ne) <= tol * N;
  if (trpmu > 0.0 && (occ_met || (mn >= b[0] && mn <= b[1]))) {
    m[0] = mn;
    for (int i = 1; i <= nk; ++i) m[i] -= t[i] / trpmu;
  } else {
    m[0] = 0.5 * (b[0] + b[1]);
  }
  m[0] = fmin(fmax(m[0], lo), hi);
  for (int i = 0; i < J; ++i) sh[i] = -c * m[i];
}

// Linear canonical correction of one system's first-order responses (the
// order-1 response is affine in mu1 with slope -P_J, P_J the response to
// H1 = I, Sec. III's Tr P^(1) = 0 condition): thread z takes
// delta_z = Tr P1_z / Tr P_J, moves mu1_z by it, and updates the trace
// record (Tr P1_z and Tr(H1_z P1_z)) to the corrected response.
__global__ void k_lin_delta(double* t, int d, int J, int rs0, double* mu, double* shift, double c,
                            double* delta, const int* gate, int off) {
  const int z = threadIdx.x;
  if (z >= d || (gate && !*gate)) return;
  const int i = 1 + off + z;  // slot of the corrected order's trace and mu
  const double trj = t[rs0];
  const double dl = trj != 0.0 ? t[i] / trj : 0.0;
  delta[z] = dl;
  t[i] -= dl * trj;
  t[2 * J + i] -= dl * t[rs0 + 2 + z];
  mu[i] += dl;
  shift[i] = -c * mu[i];
}

// w_i = (P0 - P0^2)_ii for one row per block (P0 symmetric, FP64, N x N).
__global__ __launch_bounds__(kT) void k_row_w(const double* P0, int64_t N, double* w) {
  __shared__ double red[kT / 64];
  const int64_t i = blockIdx.x;
  const double* row = P0 + i * N;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < N; j += kT) s += row[j] * row[j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kT / 64; ++q) t += red[q];
    w[i] = row[i] - t;
  }
}

struct DiagPtrs {
  const double* h[8];
};

// mu1_z = sum_i w_i (H1_z)_ii / sum_i w_i (one block; fixed summation order),
// written with its shift -c mu1_z where the caller gave no value (want[z]).
__global__ __launch_bounds__(kT) void k_mu1_guess(const double* w, int64_t N, DiagPtrs h1, int d,
                                                  double* mu, double* shift, double c,
                                                  const int* want) {
  __shared__ double red[kT / 64][9];
  double acc[9];
  for (int z = 0; z <= 8; ++z) acc[z] = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += kT) {
    const double wi = w[i];
    acc[8] += wi;
    for (int z = 0; z < d; ++z) acc[z] += wi * h1.h[z][i * N + i];
  }
  for (int z = 0; z <= 8; ++z) {
    double v = acc[z];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][z] = v;
  }
  __syncthreads();
  if (threadIdx.x < d && want[threadIdx.x]) {
    const int z = threadIdx.x;
    double num = 0.0, den = 0.0;
    for (int q = 0; q < kT / 64; ++q) {
      num += red[q][z];
      den += red[q][8];
    }
    if (den > 1e-12 * (double)N) {
      mu[1 + z] = num / den;
      shift[1 + z] = -c * mu[1 + z];
    }
  }
}

// P1 -= delta * PJ over an N x N FP64 caller matrix.
__global__ __launch_bounds__(kT) void k_lin_axpy(double* P1, const double* PJ, int64_t n,
                                                 const double* delta, const int* gate) {
  if (gate && !*gate) return;
  const double dl = *delta;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    P1[i] -= dl * PJ[i];
}

// ---------------------------------------------------------------- int8 slices (I8S4)
__global__ __launch_bounds__(kT) void k_amax(const double* __restrict__ x, int64_t sx, int64_t n,
                                             double* __restrict__ part, int nb, const int* active) {
  const int z = blockIdx.y;
  if (active && !active[z]) return;
  const double* xm = x + (int64_t)z * sx;
  double m = 0.0;
  bool bad = false;
  for (int64_t i = ((int64_t)blockIdx.x * kT + threadIdx.x) * 2; i < n; i += (int64_t)gridDim.x * kT * 2) {
    const d2v v = *(const d2v*)(xm + i);
    const double a0 = fabs(v.x), a1 = fabs(v.y);
    bad |= !(a0 <= 1.0e308) || !(a1 <= 1.0e308);
    m = fmax(m, fmax(a0, a1));
  }
  m = block_max(bad ? INFINITY : m);
  if (threadIdx.x == 0) part[(int64_t)z * nb + blockIdx.x] = m;
}

// Pack the low byte of eight digits into two words (byte e of word e / 4).
__device__ inline uint32_t pack4(const int* d) {
  return (uint32_t)(d[0] & 0xff) | ((uint32_t)(d[1] & 0xff) << 8) | ((uint32_t)(d[2] & 0xff) << 16) |
         ((uint32_t)(d[3] & 0xff) << 24);
}

// One 16-element piece per thread and pass: piece u of a member is lane
// u % 64 of 32 x 32 block u / 64 (block row major), i.e. row
// 32 (block row) + l % 32, columns 32 (block col) + 16 (l / 32) .. + 15, and
// its four slices go to the four 1 KB slice blocks of that block at byte 16 l.
// qs[z] = (the largest of member z's nb partial maxima) / 127, one block per member.
__global__ __launch_bounds__(kT) void k_qscale(const double* __restrict__ part, int64_t pstride, int nb,
                                               double* __restrict__ qs, const int* active) {
  const int z = blockIdx.x;
  if (active && !active[z]) return;
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += kT) m = fmax(m, part[(int64_t)z * pstride + i]);
  m = block_max(m);
  if (threadIdx.x == 0) qs[z] = m / 127.0;
}

__global__ __launch_bounds__(kT) void k_quant(const double* __restrict__ x, int64_t sx, int64_t Np,
                                              int8_t* __restrict__ q8, int64_t sq, const double* __restrict__ qs,
                                              const int* active) {
  const int z = blockIdx.y;
  if (active && !active[z]) return;
  // one 32 x 32 block per wave and round, staged through LDS: read with whole
  // 256-byte rows, then each lane takes 16 consecutive elements of one row
  __shared__ double tile[kT / 64][32][33];
  // digits of x / q, q = qs[z] = max |x| / 127 (the scale the products apply)
  const double q = qs[z];
  const double inv = (q > 0.0 && q <= 1.0e306) ? 1.0 / q : 0.0;
  const double* xm = x + (int64_t)z * sx;
  int8_t* qm = q8 + (int64_t)z * sq;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  double(*t)[33] = tile[wave];
  const int64_t kbr = Np >> 5;
  const int64_t nblk = kbr * kbr;
  // every wave of the block takes the same number of rounds (the barriers)
  for (int64_t g = blockIdx.x; g * (kT / 64) < nblk; g += gridDim.x) {
    const int64_t blk = g * (kT / 64) + wave;
    const bool live = blk < nblk;
    const int64_t rb = live ? blk / kbr : 0, cb = live ? blk - rb * kbr : 0;
    if (live) {
      const double* base = xm + rb * 32 * Np + cb * 32;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int r = i * 4 + (l >> 4), c = (l & 15) * 2;
        const d2v v = *(const d2v*)(base + (int64_t)r * Np + c);
        t[r][c] = v.x;
        t[r][c + 1] = v.y;
      }
    }
    __syncthreads();
    if (live) {
      const int row = l & 31, c0 = (l >> 5) * 16;
      int d[kQ8Slices][16];
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        double r = t[row][c0 + e] * inv;
#pragma unroll
        for (int sl = 0; sl < kQ8Slices; ++sl) {
          const double q = rint(r);
          d[sl][e] = (int)q;
          r = (r - q) * kQ8Base;
        }
      }
#pragma unroll
      for (int sl = 0; sl < kQ8Slices; ++sl) {
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = pack4(&d[sl][4 * q]);
        uint32_t* dst = (uint32_t*)(qm + ((blk * kQ8Slices + sl) << 10) + l * 16);
        *(uint4*)dst = make_uint4(w[0], w[1], w[2], w[3]);
      }
    }
    __syncthreads();
  }
}

// CG direction update P = R + beta P with the int8 slices of the new P
// written in the same pass (I8S4 / I8S3 operands).  The slicing scale needs a
// bound on max |P| before P exists: max |R| (block maxima from the residual
// update) + |beta| times the previous bound, from the per-iteration bound
// history pb (pb_old read, pb_new and the member's q written by block 0, so
// no block reads what another block of this launch writes).  The bound is at
// least the true maximum, so every digit fits; it can exceed it by at most
// the previous bound's slack times beta (< 1 in practice), a fraction of a bit.
__global__ __launch_bounds__(kT) void k_cg_p_q8(double* __restrict__ P, const double* __restrict__ R, int64_t Np,
                                                int64_t stride, const double* rr_new, const double* rr_old,
                                                int hstride, const int* active, const double* __restrict__ rmax,
                                                int nb, const double* pb_old, double* pb_new, int8_t* __restrict__ q8,
                                                int64_t sq, double* __restrict__ qs) {
  const int z = blockIdx.y;
  if (active && !active[z]) return;
  __shared__ double sm;
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += kT) m = fmax(m, rmax[(int64_t)z * nb + i]);
  m = block_max(m);
  if (threadIdx.x == 0) sm = m;
  __syncthreads();
  const double ro = rr_old[z * hstride];
  const double beta = ro != 0.0 ? rr_new[z * hstride] / ro : 0.0;
  const double bound = (sm + fabs(beta) * pb_old[z * hstride]) * (1.0 + 1.0e-12);
  const double inv = (bound > 0.0 && bound <= 1.0e308) ? 127.0 / bound : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    pb_new[z * hstride] = bound;
    qs[z] = bound / 127.0;
  }
  double* pm = P + (int64_t)z * stride;
  const double* rm = R + (int64_t)z * stride;
  int8_t* qm = q8 + (int64_t)z * sq;
  const int64_t kbr = Np >> 5;
  const int64_t pieces = kbr * kbr * 64;
  for (int64_t u = (int64_t)blockIdx.x * kT + threadIdx.x; u < pieces; u += (int64_t)gridDim.x * kT) {
    const int64_t blk = u >> 6;
    const int l = (int)(u & 63);
    const int64_t rb = blk / kbr, cb = blk - rb * kbr;
    const int64_t off = (rb * 32 + (l & 31)) * Np + cb * 32 + (l >> 5) * 16;
    int d[kQ8Slices][16];
#pragma unroll
    for (int e = 0; e < 16; e += 2) {
      const d2v rv = *(const d2v*)(rm + off + e);
      d2v pv = *(const d2v*)(pm + off + e);
      pv.x = rv.x + beta * pv.x;
      pv.y = rv.y + beta * pv.y;
      *(d2v*)(pm + off + e) = pv;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double r = (h ? pv.y : pv.x) * inv;
#pragma unroll
        for (int sl = 0; sl < kQ8Slices; ++sl) {
          const double t = rint(r);
          d[sl][e + h] = (int)t;
          r = (r - t) * kQ8Base;
        }
      }
    }
#pragma unroll
    for (int sl = 0; sl < kQ8Slices; ++sl) {
      uint32_t w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) w[q] = pack4(&d[sl][4 * q]);
      *(uint4*)(qm + ((blk * kQ8Slices + sl) << 10) + l * 16) = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
}

// pb[z * hstride] = 127 q[z]: the bound history starts at the sliced maximum of the first P.
__global__ void k_q8_bound_init(const double* qs, double* pb, int hstride, int batch) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z < batch) pb[z * hstride] = 127.0 * qs[z];
}

inline unsigned red_grid(int64_t n) {
  int64_t b = (n + kT * 8 - 1) / (kT * 8);
  if (b < 1) b = 1;
  if (b > kMaxRedBlocks) b = kMaxRedBlocks;
  return (unsigned)b;
}

inline unsigned ew_grid(int64_t n) {
  int64_t b = (n + kT * 4 - 1) / (kT * 4);
  if (b < 1) b = 1;
  if (b > 65535) b = 65535;
  return (unsigned)b;
}

}  // namespace

int reduce_blocks(int64_t n) { return (int)red_grid(n); }

template <class T>
hipError_t transpose(const T* in, int64_t Np, int64_t stride, T* out, uint16_t* const* planes,
                     int nplanes, int batch, hipStream_t s) {
  Planes pl{{nullptr, nullptr, nullptr}};
  for (int p = 0; p < nplanes; ++p) pl.p[p] = planes[p];
  if (Np % 32 != 0) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)(Np / 32);
  hipLaunchKernelGGL(k_transpose<T>, dim3(nb, nb, batch), dim3(kT), 0, s, in, Np, stride, out, pl,
                     nplanes);
  return hipGetLastError();
}
template hipError_t transpose<double>(const double*, int64_t, int64_t, double*, uint16_t* const*,
                                      int, int, hipStream_t);
template hipError_t transpose<float>(const float*, int64_t, int64_t, float*, uint16_t* const*, int,
                                     int, hipStream_t);

template <class Tin, class Tout>
hipError_t sym_combine(const Tin* in, int64_t ldi, int64_t si, int64_t N, int64_t Np, double a,
                       const double* dshift, int dstride, Tout* out, int64_t ldo, int64_t so,
                       uint16_t* const* planes, int nplanes, int batch, hipStream_t s,
                       const Tin* in2, double a2, const int* gate, double* mx, int64_t mstride) {
  Planes pl{{nullptr, nullptr, nullptr}};
  for (int p = 0; p < nplanes; ++p) pl.p[p] = planes[p];
  // planes exist only for workspace members: Np x Np with ld = Np
  if (nplanes && (ldo != Np || Np % 32 != 0)) return hipErrorInvalidValue;
  const int64_t rows = (ldo == N && ldo != Np) ? N : ldo;  // caller buffer: only N x N
  const int64_t span = rows > N ? rows : N;
  const int64_t nb = (span + 31) / 32;
  // with maxima: one block per 128 x 128 pair (few maxima); else one per 32 x 32 pair
  const int g = mx ? 4 : 1;
  const int64_t nbg = (nb + g - 1) / g;
  const int64_t pairs = nbg * (nbg + 1) / 2;
  if (mx && (mstride < pairs || gate || pairs != sym_pair_blocks(span))) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sym<Tin, Tout>), dim3((unsigned)pairs, batch), dim3(kT), 0, s, in, ldi, si, N, Np, a,
                     dshift, dstride, out, ldo, so, pl, nplanes, rows, in2, a2, gate, nb, g, mx, mstride);
  return hipGetLastError();
}

int64_t sym_pair_blocks(int64_t span) {
  const int64_t nb128 = (span + 127) / 128;
  return nb128 * (nb128 + 1) / 2;
}

#define DMPT_SYM_INST(TI, TO)                                                                   \
  template hipError_t sym_combine<TI, TO>(const TI*, int64_t, int64_t, int64_t, int64_t, double,  \
                                          const double*, int, TO*, int64_t, int64_t,             \
                                          uint16_t* const*, int, int, hipStream_t, const TI*,    \
                                          double, const int*, double*, int64_t);
DMPT_SYM_INST(double, double)
DMPT_SYM_INST(double, float)
DMPT_SYM_INST(float, float)
DMPT_SYM_INST(float, double)
#undef DMPT_SYM_INST

int q8_blocks(int64_t Np) { return (int)red_grid(Np * Np); }

hipError_t quantize_q8(const double* x, int64_t sx, int64_t Np, int batch, double* part, int8_t* q8, int64_t sq,
                       double* qs, const int* active, hipStream_t s) {
  if (Np <= 0 || Np % 32 != 0 || batch < 1 || !x || !part || !q8 || !qs) return hipErrorInvalidValue;
  const int64_t n = Np * Np;
  const unsigned nb = red_grid(n);
  hipLaunchKernelGGL(k_amax, dim3(nb, batch), dim3(kT), 0, s, x, sx, n, part, (int)nb, active);
  hipLaunchKernelGGL(k_qscale, dim3(batch), dim3(kT), 0, s, part, (int64_t)nb, (int)nb, qs, active);
  const int64_t nblk = (Np / 32) * (Np / 32);
  int64_t g = (nblk + 2 * (kT / 64) - 1) / (2 * (kT / 64));
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k_quant, dim3((unsigned)g, batch), dim3(kT), 0, s, x, sx, Np, q8, sq, (const double*)qs,
                     active);
  return hipGetLastError();
}

hipError_t quantize_q8_known(const double* x, int64_t sx, int64_t Np, int batch, const double* part,
                             int64_t pstride, int nb, int8_t* q8, int64_t sq, double* qs, hipStream_t s) {
  if (Np <= 0 || Np % 32 != 0 || batch < 1 || !x || !part || nb < 1 || pstride < nb || !q8 || !qs)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_qscale, dim3(batch), dim3(kT), 0, s, part, pstride, nb, qs, (const int*)nullptr);
  const int64_t nblk = (Np / 32) * (Np / 32);
  int64_t g = (nblk + 2 * (kT / 64) - 1) / (2 * (kT / 64));
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k_quant, dim3((unsigned)g, batch), dim3(kT), 0, s, x, sx, Np, q8, sq, (const double*)qs,
                     (const int*)nullptr);
  return hipGetLastError();
}

hipError_t split_planes(const double* x, int64_t n, int64_t sx, uint16_t* const* planes, int64_t sp,
                        int nplanes, int batch, hipStream_t s) {
  Planes pl{{nullptr, nullptr, nullptr}};
  for (int p = 0; p < nplanes; ++p) pl.p[p] = planes[p];
  const int64_t Np = plane_np(n);
  if (!Np) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_split, dim3(ew_grid(n), batch), dim3(kT), 0, s, x, n, sx, pl, sp, nplanes, Np);
  return hipGetLastError();
}

template <class T>
hipError_t dot_partials(const T* x, int64_t sx, const T* y, int64_t sy, int64_t n, int batch,
                        double* partials, hipStream_t s) {
  const int v2 = pair_ok(x, sx, n) && pair_ok(y, sy, n);
  hipLaunchKernelGGL(k_dot<T>, dim3(red_grid(n), batch), dim3(kT), 0, s, x, sx, y, sy, n, partials, v2);
  return hipGetLastError();
}
template hipError_t dot_partials<double>(const double*, int64_t, const double*, int64_t, int64_t,
                                         int, double*, hipStream_t);
template hipError_t dot_partials<float>(const float*, int64_t, const float*, int64_t, int64_t, int,
                                        double*, hipStream_t);

hipError_t sum_partials(const double* partials, int count, int batch, double* out, int ostride,
                        int oidx, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(batch), dim3(kT), 0, s, partials, count, out, ostride,
                     oidx);
  return hipGetLastError();
}

template <class T>
hipError_t trace(const T* x, int64_t ld, int64_t sx, int64_t N, int batch, double* out, int ostride,
                 double* aout, hipStream_t s) {
  hipLaunchKernelGGL(k_trace<T>, dim3(batch), dim3(kT), 0, s, x, ld, sx, N, out, ostride, aout);
  return hipGetLastError();
}
template hipError_t trace<double>(const double*, int64_t, int64_t, int64_t, int, double*, int,
                                  double*, hipStream_t);
template hipError_t trace<float>(const float*, int64_t, int64_t, int64_t, int, double*, int, double*,
                                 hipStream_t);

template <class T>
hipError_t cg_update_xr(T* U, T* R, const T* P, const T* Q, int64_t n, int64_t stride, int batch,
                        const double* rr, const double* pq, int hstride, const int* active,
                        double* partials, hipStream_t s, double* rmax) {
  // (element pairs per thread measured 4 % slower here than one element)
  hipLaunchKernelGGL(k_cg_xr<T>, dim3(red_grid(n), batch), dim3(kT), 0, s, U, R, P, Q, n, stride,
                     rr, pq, hstride, active, partials, rmax);
  return hipGetLastError();
}
template hipError_t cg_update_xr<double>(double*, double*, const double*, const double*, int64_t,
                                         int64_t, int, const double*, const double*, int,
                                         const int*, double*, hipStream_t, double*);
template hipError_t cg_update_xr<float>(float*, float*, const float*, const float*, int64_t,
                                        int64_t, int, const double*, const double*, int, const int*,
                                        double*, hipStream_t, double*);

hipError_t cg_update_p_q8(double* P, const double* R, int64_t Np, int64_t stride, int batch, const double* rr_new,
                          const double* rr_old, int hstride, const int* active, const double* rmax,
                          const double* pb_old, double* pb_new, int8_t* q8, int64_t sq, double* qs,
                          hipStream_t s) {
  if (Np <= 0 || Np % 32 != 0 || batch < 1) return hipErrorInvalidValue;
  const int64_t n = Np * Np;
  const int64_t pieces = n / 16;
  int64_t g = (pieces + 2 * kT - 1) / (2 * kT);
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k_cg_p_q8, dim3((unsigned)g, batch), dim3(kT), 0, s, P, R, Np, stride, rr_new, rr_old, hstride,
                     active, rmax, (int)red_grid(n), pb_old, pb_new, q8, sq, qs);
  return hipGetLastError();
}

hipError_t q8_bound_init(const double* qs, double* pb, int hstride, int batch, hipStream_t s) {
  hipLaunchKernelGGL(k_q8_bound_init, dim3((batch + 63) / 64), dim3(64), 0, s, qs, pb, hstride, batch);
  return hipGetLastError();
}

template <class T>
hipError_t cg_update_p(T* P, const T* R, int64_t n, int64_t stride, int batch, const double* rr_new,
                       const double* rr_old, int hstride, const int* active,
                       uint16_t* const* planes, int nplanes, hipStream_t s) {
  Planes pl{{nullptr, nullptr, nullptr}};
  for (int p = 0; p < nplanes; ++p) pl.p[p] = planes[p];
  const int64_t Np = nplanes ? plane_np(n) : 0;
  if (nplanes && !Np) return hipErrorInvalidValue;
  bool ok = pair_ok(P, stride, n) && pair_ok(R, stride, n);
  for (int p = 0; p < nplanes; ++p) ok = ok && pair_ok(pl.p[p], stride, n);
  hipLaunchKernelGGL(k_cg_p<T>, dim3(ew_grid(n), batch), dim3(kT), 0, s, P, R, n, stride, rr_new,
                     rr_old, hstride, active, pl, nplanes, Np, ok ? 1 : 0);
  return hipGetLastError();
}
template hipError_t cg_update_p<double>(double*, const double*, int64_t, int64_t, int,
                                        const double*, const double*, int, const int*,
                                        uint16_t* const*, int, hipStream_t);
template hipError_t cg_update_p<float>(float*, const float*, int64_t, int64_t, int, const double*,
                                       const double*, int, const int*, uint16_t* const*, int,
                                       hipStream_t);

hipError_t cg_check(const double* rr, const double* rr0, const double* ref, int hstride, int batch,
                    double tol2, double eta2, int* active, int* iters, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_check, dim3((batch + 63) / 64), dim3(64), 0, s, rr, rr0, ref, hstride,
                     batch, tol2, eta2, active, iters);
  return hipGetLastError();
}

hipError_t input_status(const double* gersh, const int* flag, double beta, double mu, int n, int* status,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_input_status, dim3(1), dim3(64), 0, s, gersh, flag, beta, mu, n, status);
  return hipGetLastError();
}

hipError_t cg_account(const int* active, const int* iters, int batch, int* stat, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_account, dim3((batch + 63) / 64), dim3(64), 0, s, active, iters, batch, stat);
  return hipGetLastError();
}

template <class T>
hipError_t axpby(const T* x, int64_t sx, T* y, int64_t sy, int64_t n, int batch, double a, double b,
                 uint16_t* const* planes, int64_t sp, int nplanes, hipStream_t s) {
  Planes pl{{nullptr, nullptr, nullptr}};
  for (int p = 0; p < nplanes; ++p) pl.p[p] = planes[p];
  const int64_t Np = nplanes ? plane_np(n) : 0;
  if (nplanes && !Np) return hipErrorInvalidValue;
  bool ok = pair_ok(x, sx, n) && pair_ok(y, sy, n);
  for (int p = 0; p < nplanes; ++p) ok = ok && pair_ok(pl.p[p], sp, n);
  hipLaunchKernelGGL(k_axpby<T>, dim3(ew_grid(n), batch), dim3(kT), 0, s, x, sx, y, sy, n, a, b, pl,
                     sp, nplanes, Np, ok ? 1 : 0);
  return hipGetLastError();
}
template hipError_t axpby<double>(const double*, int64_t, double*, int64_t, int64_t, int, double,
                                  double, uint16_t* const*, int64_t, int, hipStream_t);
template hipError_t axpby<float>(const float*, int64_t, float*, int64_t, int64_t, int, double,
                                 double, uint16_t* const*, int64_t, int, hipStream_t);

template <class T>
hipError_t axpbyz(const T* x, const T* y, T* out, int64_t n, double a, double b, uint16_t* const* planes,
                  int nplanes, hipStream_t s, double* mx, int64_t mblocks) {
  Planes pl{{nullptr, nullptr, nullptr}};
  for (int p = 0; p < nplanes; ++p) pl.p[p] = planes[p];
  const int64_t Np = nplanes ? plane_np(n) : 0;
  if (nplanes && !Np) return hipErrorInvalidValue;
  if (mx && (mblocks < 1 || mblocks > 65535)) return hipErrorInvalidValue;
  bool ok = pair_ok(x, 0, n) && pair_ok(y, 0, n) && pair_ok(out, 0, n);
  for (int p = 0; p < nplanes; ++p) ok = ok && pair_ok(pl.p[p], 0, n);
  const unsigned g = mx ? (unsigned)mblocks : ew_grid(n);
  hipLaunchKernelGGL(k_axpbyz<T>, dim3(g), dim3(kT), 0, s, x, y, out, n, a, b, pl, nplanes, Np, ok ? 1 : 0, mx);
  return hipGetLastError();
}
template hipError_t axpbyz<double>(const double*, const double*, double*, int64_t, double, double,
                                   uint16_t* const*, int, hipStream_t, double*, int64_t);
template hipError_t axpbyz<float>(const float*, const float*, float*, int64_t, double, double,
                                  uint16_t* const*, int, hipStream_t, double*, int64_t);

int64_t ew_sink_blocks(int64_t n, int64_t cap) {
  const int64_t g = (int64_t)ew_grid(n);
  return g < cap ? g : cap;
}

template <class Tin, class Tout>
hipError_t convert(const Tin* in, int64_t si, Tout* out, int64_t so, int64_t n, int batch,
                   uint16_t* const* planes, int64_t sp, int nplanes, hipStream_t s, double* mx,
                   int64_t mstride, int64_t mblocks) {
  Planes pl{{nullptr, nullptr, nullptr}};
  for (int p = 0; p < nplanes; ++p) pl.p[p] = planes[p];
  const int64_t Np = nplanes ? plane_np(n) : 0;
  if (nplanes && !Np) return hipErrorInvalidValue;
  if (mx && (mblocks < 1 || mblocks > 65535 || (batch > 1 && mstride < mblocks))) return hipErrorInvalidValue;
  bool ok = pair_ok(in, si, n) && pair_ok(out, so, n);
  for (int p = 0; p < nplanes; ++p) ok = ok && pair_ok(pl.p[p], sp, n);
  const unsigned g = mx ? (unsigned)mblocks : ew_grid(n);
  hipLaunchKernelGGL((k_convert<Tin, Tout>), dim3(g, batch), dim3(kT), 0, s, in, si, out, so, n, pl, sp,
                     nplanes, Np, ok ? 1 : 0, mx, mstride);
  return hipGetLastError();
}
#define DMPT_CONV_INST(TI, TO)                                                                \
  template hipError_t convert<TI, TO>(const TI*, int64_t, TO*, int64_t, int64_t, int,         \
                                      uint16_t* const*, int64_t, int, hipStream_t, double*,   \
                                      int64_t, int64_t);
DMPT_CONV_INST(double, float)
DMPT_CONV_INST(float, double)
DMPT_CONV_INST(float, float)
DMPT_CONV_INST(double, double)
#undef DMPT_CONV_INST

template <class T>
hipError_t scaled_plus_identity(const T* x, T* out, int64_t N, int64_t Np, double a, double b,
                                uint16_t* const* planes, int nplanes, hipStream_t s, double* mx,
                                int64_t mblocks) {
  Planes pl{{nullptr, nullptr, nullptr}};
  for (int p = 0; p < nplanes; ++p) pl.p[p] = planes[p];
  if (mx && (mblocks < 1 || mblocks > 65535)) return hipErrorInvalidValue;
  const unsigned g = mx ? (unsigned)mblocks : ew_grid(Np * Np);
  hipLaunchKernelGGL(k_spi<T>, dim3(g), dim3(kT), 0, s, x, out, N, Np, a, b, pl, nplanes, mx);
  return hipGetLastError();
}
template hipError_t scaled_plus_identity<double>(const double*, double*, int64_t, int64_t, double,
                                                 double, uint16_t* const*, int, hipStream_t, double*,
                                                 int64_t);
template hipError_t scaled_plus_identity<float>(const float*, float*, int64_t, int64_t, double,
                                                double, uint16_t* const*, int, hipStream_t, double*,
                                                int64_t);

hipError_t set_values(int* p, int v, int n, double* q, double qv, int nq, hipStream_t s) {
  const int m = n > nq ? n : nq;
  hipLaunchKernelGGL(k_set, dim3((m + 63) / 64 > 0 ? (m + 63) / 64 : 1), dim3(64), 0, s, p, v, n, q,
                     qv, nq);
  return hipGetLastError();
}

hipError_t expand_mask(const int* src, int div, int* dst, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_expand, dim3((n + 63) / 64), dim3(64), 0, s, src, div, dst, n);
  return hipGetLastError();
}

template <class T>
hipError_t fill_pattern(T* x, int64_t n, uint32_t seed, uint16_t* const* planes, int nplanes,
                        hipStream_t s) {
  Planes pl{{nullptr, nullptr, nullptr}};
  for (int p = 0; p < nplanes; ++p) pl.p[p] = planes[p];
  const int64_t Np = nplanes ? plane_np(n) : 0;
  if (nplanes && !Np) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fill<T>, dim3(ew_grid(n)), dim3(kT), 0, s, x, n, seed, pl, nplanes, Np);
  return hipGetLastError();
}
template hipError_t fill_pattern<double>(double*, int64_t, uint32_t, uint16_t* const*, int, hipStream_t);
template hipError_t fill_pattern<float>(float*, int64_t, uint32_t, uint16_t* const*, int, hipStream_t);

hipError_t lin_correct(double* t, int d, int J, int rs0, double* mu, double* shift, double c,
                       double* delta, double* const* P1, const double* PJ, int64_t N, const int* gate,
                       hipStream_t s, int order) {
  if (d < 1 || d > 64 || order < 1 || order > 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lin_delta, dim3(1), dim3(64), 0, s, t, d, J, rs0, mu, shift, c, delta, gate,
                     (order - 1) * d);
  hipError_t e = hipGetLastError();
  for (int z = 0; z < d && e == hipSuccess; ++z) {
    hipLaunchKernelGGL(k_lin_axpy, dim3(ew_grid(N * N)), dim3(kT), 0, s, P1[z], PJ, N * N, delta + z,
                       gate);
    e = hipGetLastError();
  }
  return e;
}

hipError_t mu1_guess(const double* P0, int64_t N, const double* const* H1, int d, double* w,
                     double* mu, double* shift, double c, const int* want, hipStream_t s) {
  if (d < 1 || d > 8 || N < 1) return hipErrorInvalidValue;
  DiagPtrs h{};
  for (int z = 0; z < d; ++z) h.h[z] = H1[z];
  hipLaunchKernelGGL(k_row_w, dim3((unsigned)N), dim3(kT), 0, s, P0, N, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mu1_guess, dim3(1), dim3(kT), 0, s, w, N, h, d, mu, shift, c, want);
  return hipGetLastError();
}

hipError_t newton_update(const double* tr, int rs, const double* par, double* mu, double* shift,
                         int J, int nk, double tol, int final_stage, int* active, int* done,
                         double* prev_err, double* brk, double* occ, int* passes, int* status,
                         int nsys, hipStream_t s) {
  hipLaunchKernelGGL(k_newton, dim3((nsys + 63) / 64), dim3(64), 0, s, tr, rs, par, mu, shift, J, nk,
                     tol, final_stage, active, done, prev_err, brk, occ, passes, status, nsys);
  return hipGetLastError();
}

hipError_t pad_copy(const double* in, int64_t ldi, int64_t N, double* out, int64_t Np, bool trans,
                    hipStream_t s) {
  if (Np % 32 != 0 || N > Np) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)(Np / 32);
  hipLaunchKernelGGL(k_pad_copy, dim3(nb, nb), dim3(kT), 0, s, in, ldi, N, out, Np, trans ? 1 : 0);
  return hipGetLastError();
}

hipError_t nonfinite_scan(const double* x, int64_t ld, int64_t N, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_nonfinite, dim3(red_grid(N * N)), dim3(kT), 0, s, x, ld, N, flag);
  return hipGetLastError();
}

hipError_t gershgorin(const double* h, int64_t N, double* out, hipStream_t s) {
  // out[0..1]: bounds; out[2 .. 2+2N): per-row scratch
  double* lo = out + 2;
  double* hi = out + 2 + N;
  hipLaunchKernelGGL(k_gersh_rows, dim3((unsigned)N), dim3(kT), 0, s, h, N, lo, hi);
  hipLaunchKernelGGL(k_minmax, dim3(1), dim3(kT), 0, s, lo, hi, N, out);
  return hipGetLastError();
}

hipError_t asym_max(const double* x, int64_t N, double* out_max, hipStream_t s) {
  // out_max[0..nb): per-block maxima (host reduces)
  hipLaunchKernelGGL(k_asym_max, dim3(red_grid(N * N)), dim3(kT), 0, s, x, N, out_max);
  return hipGetLastError();
}

template <class T>
hipError_t antisym_sq_partials(const T* x, int64_t ld, int64_t N, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_antisym_sq<T>, dim3(red_grid(N * N)), dim3(kT), 0, s, x, ld, N, partials);
  return hipGetLastError();
}
template hipError_t antisym_sq_partials<double>(const double*, int64_t, int64_t, double*,
                                                hipStream_t);
template hipError_t antisym_sq_partials<float>(const float*, int64_t, int64_t, double*, hipStream_t);

}  // namespace dmpt
