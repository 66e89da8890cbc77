/*
 * dmpt.h -- C ABI of the MI355X (gfx950) canonical density-matrix
 * perturbation theory library.
 *
 * The method (Niklasson, Rubensson, Rudberg, Cawkwell, "Canonical density
 * matrix perturbation theory"):
 *   Sec. II, Eq. (Rec_F_2)   recursive Fermi-operator expansion
 *        X_0 = I/2 - 2^-(n+2) beta (H - mu I),  X_k = X^2 [X^2 + (I - X)^2]^-1,
 *        P = X_n  (n recursion steps; the paper calls it M);
 *   Sec. II, Eqs. (P_resp), (H_prt) and Algorithm 1
 *        perturbed recursions for P^(1), P^(2) under H = H0 + lambda H1 + lambda^2 H2,
 *        each step a linear solve with the same system matrix T = X^2 + (I - X)^2;
 *   Sec. II, Eq. (NewtRaphs) and Algorithm 1's while loop
 *        canonical Newton update of the mu jet with P_mu = beta P0 (I - P0) so
 *        that Tr P0 = Ne and Tr P1 = Tr P2 = 0;
 *   Sec. III, Eq. (Resp_0)   response traces Tr[H^(k) P^(m-k)].
 *
 * Internally the recursion runs in the shifted variable D = I/2 - X, for
 * which a step reads D_k = 2 D (I + 4 D^2)^-1 (algebraically identical; it
 * keeps the iterate away from the rounding grid of 1/2).
 *
 * Conventions shared by every entry point
 *   - Matrices are DEVICE pointers to dense, row-major, N x N FP64 arrays with
 *     leading dimension N, owned by the caller.  Inputs are read only and are
 *     used through their symmetric part (A + A^T)/2.  Outputs are written in
 *     full and are symmetric.  The library keeps no reference to caller
 *     buffers after a call returns.  A diagonal perturbation must still be
 *     passed as a full matrix.
 *   - Work is queued on the context's HIP stream, in order with the work the
 *     caller queued before the call on the stream given to dmpt_init (see
 *     there for NULL).  A call returns after the values it reports on the
 *     host (statistics, the mu jet) are final; output matrices are complete
 *     when the call returns.
 *   - Errors are status codes; nothing is thrown across the ABI.  Arguments
 *     are checked on the host before any device work; dmpt_last_error()
 *     describes the most recent failure of a context.
 *   - A context is not thread safe; use one context per host thread.
 */
#ifndef DMPT_H
#define DMPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dmpt_ctx_s* dmpt_ctx;

typedef enum {
  DMPT_OK = 0,
  DMPT_ERR_ARG = -1,        /* invalid argument (checked before any launch) */
  DMPT_ERR_HIP = -2,        /* a HIP runtime call failed */
  DMPT_ERR_NOMEM = -3,      /* device allocation failed or the problem exceeds the context */
  DMPT_ERR_NOCONV = -4,     /* Newton loop or a linear solve did not reach its tolerance */
  DMPT_ERR_RANGE = -5,      /* beta * spread(H0) >= 2^(n+1): X_0 leaves [0, 1] (Appendix A) */
  DMPT_ERR_NONFINITE = -6,  /* NaN or Inf in an input or in an iterate */
  DMPT_ERR_UNSUPPORTED = -7 /* feature not built for this configuration */
} dmpt_status;

/* Arithmetic of the matrix products.  Every mode keeps the iterates (the
 * D^(k) of every step, the solver vectors) in FP64 storage, and FP64 for
 * traces, norms, the mu jet and the reported outputs; the modes differ in
 * the products only. */
typedef enum {
  DMPT_FP64 = 0,    /* FP64 MFMA products */
  DMPT_FP32 = 1,    /* operands rounded to FP32, FP32 MFMA products; each 16-wide slice of the
                       inner index is summed in FP32 and the slices in FP64 */
  DMPT_BF16X3 = 2,  /* products as hi*hi + hi*lo + lo*hi of two-way BF16 splits, FP32 accumulation */
  DMPT_BF16X6 = 3,  /* three-way BF16 split, the six cross products with p + q <= 2; with
                       options.acc64 each 32-wide slice of the inner index is summed in FP32
                       and the slices in FP64 */
  DMPT_INT8X13 = 4, /* each operand as q (d0 + d1/254 + d2/254^2 + d3/254^3) with one FP64 q per
                       matrix (its largest |entry| / 127) and signed int8 digits; the thirteen
                       digit products with p + q <= 4 on int8 MFMA, summed exactly in int32 over
                       the whole inner index (N <= 32768) and combined in FP64 */
  DMPT_INT8X6 = 5   /* the same int8 digits, the first three only: the six products with p + q <= 2
                       (exact int32 sums, no accumulation bias in traces; ~1e-6) */
} dmpt_prec;

/* Per-step linear solver for T' Y = R, T' = I + 4 D^2 (2 T of Algorithm 1). */
typedef enum {
  DMPT_SOLVER_CG = 0,  /* conjugate gradients, one product per iteration and right-hand side (Sec. II) */
  DMPT_SOLVER_NS = 1,  /* shared inverse Z of T' by Newton-Schulz from the minimax linear start on
                          the step's spectral interval [1, 1 + 4 b^2], b = min(1/2, 2^step ||D_0||)
                          with ||D_0|| from the Gershgorin interval of H0, iterated to a residual
                          of 2^-60 (four steps once ||D|| ~ 1/2, none while ||D|| < ~1e-5; with
                          INT8X13 products 2^-34 2^-(n - step), in the INT8X6 first phase of
                          refine = 2 2^-26 2^-(n - step), never below 2^-60), reused for every order and
                          direction (Sec. II remark): one product per right-hand side, plus one
                          refinement step with FP32, BF16 and INT8X6 products; single-system paths
                          (the batched and adjoint paths keep CG).  Under the linear schedule the
                          order-1 pass starts each step from the final order-0 pass's inverse
                          where a bound on the mu0 shift allows fewer steps.  In the environment,
                          DMPT_NS_ITERS=k forces k steps everywhere, DMPT_NS_REFINE=0|1 the
                          refinement step off or on and DMPT_NS_COLD the fresh start (debugging) */
  DMPT_SOLVER_HYBRID = 2 /* the shared inverse in the passes whose products are FP64 or INT8X13 (no
                            refinement step needed) and in the first-phase passes of INT8X6 with
                            refine = 2 (loose tolerance: no refinement step; that phase then ends
                            at an occupation error of 5e-4), CG in the others (FP32, BF16 and
                            final INT8X6 products: the inverse's rounding biases the jets' traces);
                            under the linear schedule the order-1 pass keeps Z of every step
                            (n N^2 master elements, when the memory is there) and the later
                            passes reuse it */
} dmpt_solver;

/* Initial guess of the conjugate-gradient solve. */
typedef enum {
  DMPT_GUESS_PREV = 0,   /* the previous iterate X_{n-1}^(k) (Algorithm 1 remark) */
  DMPT_GUESS_TAYLOR = 1  /* 2D - 8D^3 for order 0 (one more product per step), previous iterate
                            for the others; a stored trajectory (warm_traj) takes precedence */
} dmpt_guess;

typedef struct {
  dmpt_prec prec;       /* arithmetic mode */
  dmpt_solver solver;   /* per-step solver */
  dmpt_guess guess;     /* CG initial guess */
  double tol_occ;       /* Newton stops when |Tr P0 - Ne| <= tol_occ * N and, for k >= 1,
                           |Tr P^(k)| <= tol_occ * sum_i |P^(k)_ii| (or when that normalised
                           error stopped shrinking within 1000 tol_occ); <= 0: default for prec */
  double tol_cg;        /* relative residual of each solve; <= 0: default for prec */
  int max_newton;       /* Newton passes (default 50) */
  int max_cg;           /* CG iterations per solve (default 60) */
  int refine;           /* BF16X3 and INT8X6: after convergence, redo the last passes in BF16X6 (1),
                           in INT8X13 (2) or not (0) */
  int ckpt_every;       /* adjoint: keep every ckpt_every-th iterate, recompute the rest (default 5) */
  int check;            /* 1: compute the commutator and idempotency checks at the end of a call */
  int staged;           /* 1: converge mu0 with order-0 passes first, then run full passes (same fixed point) */
  int warm_traj;        /* 1: keep every step's iterates (FP32 copies) and start each CG of the next
                           Newton pass from the same step's previous solution instead of the
                           previous recursion step's iterate; falls back when memory is short, and
                           is not allocated when every pass solves with the shared inverse */
  int schedule;         /* canonical loop for orders >= 1: 0 = Algorithm 1's Newton update of every
                           mu^(k) with Tr P_mu; 1 = after mu0 has converged, one pass per order with
                           the extra response J to H1 = I: P^(k) is affine in mu^(k) with slope -J,
                           so mu^(k) = Tr P^(k)(0) / Tr J and P^(k) = P^(k)(0) - mu^(k) J exactly;
                           the order-1 pass keeps its order-0/1 solutions of every step (memory:
                           n (d + 2) N^2 master elements) and the order-2 pass reuses them;
                           2 = as 1 but the order-2 pass solves orders 0 and 1 again */
  int acc64;            /* 6-product split-BF16 products: 1 = each 32-wide slice of k is summed in FP32
                           and the slices in FP64 (128 x 128 tiles; the FP32 rounding then no longer
                           grows with N), 0 = one FP32 accumulator over all of k (256 x 256 tiles) */
  int autotune;         /* 1: before the first products of a padded size, time every product-kernel
                           variant of the context's engines at that size and keep the fastest
                           (dmpt_autotune); the batched solve tunes every bucket size */
  int grouped;          /* batched solve: 1 (default) = the launches of every recursion step are
                           issued for all size buckets together, each product as one grouped launch
                           over every bucket's (member, tile) blocks; 0 = bucket by bucket */
} dmpt_options;

#define DMPT_MAX_DIRS 8

/* Bits of dmpt_stats.flags. */
#define DMPT_FLAG_NOISE_FLOOR 1  /* the Newton loop accepted a normalised occupation error that had
                                    stopped shrinking (between tol_occ and 1000 tol_occ: the traces
                                    carry the products' rounding) instead of one below tol_occ */
#define DMPT_FLAG_CG_FLOOR 2     /* a solve of a graph-replayed (batched) pass ended its fixed,
                                    a-priori iteration count above tol_cg; cg_unconverged counts them */

typedef struct {
  int newton_iters;                      /* Newton passes executed (batched: graph replays) */
  int cg_iters_total;                    /* CG iterations summed over steps, orders, directions (and
                                            systems) */
  int cg_iters_max;                      /* largest CG iteration count of a single solve */
  int flags;                             /* DMPT_FLAG_* */
  int cg_unconverged;                    /* solves that ended above tol_cg (graph-replayed passes) */
  double occ_err;                        /* |Tr P0 - Ne| + sum_k |Tr P^(k)| of the returned P */
  double mu[1 + 3 * DMPT_MAX_DIRS];      /* mu0, mu1[d], mu2[d], mu3[d] used for the returned P */
  double trP[1 + 3 * DMPT_MAX_DIRS];     /* Tr P0, Tr P1[d], Tr P2[d], Tr P3[d] */
  double tr_pmu;                         /* Tr P_mu = beta (Tr P0 - ||P0||_F^2) */
  /* Response traces Tr[H^(k) P^(j)] per direction (Sec. III, Eq. Resp_0), with
   * H^(k) used through its symmetric part and an absent H2 / H3 counting as 0;
   * computed on the returned matrices for k >= 1, j <= order, k + j <= order + 1 */
  double tr_h1p1[DMPT_MAX_DIRS];         /* Tr(H1 P1) */
  double tr_h1p2[DMPT_MAX_DIRS];         /* Tr(H1 P2) (order >= 2) */
  double tr_h2p0[DMPT_MAX_DIRS];         /* Tr(H2 P0) (order >= 2) */
  double tr_h1p3[DMPT_MAX_DIRS];         /* Tr(H1 P3) (order 3) */
  double tr_h1p0[DMPT_MAX_DIRS];         /* Tr(H1 P0) (order >= 1) */
  double tr_h2p1[DMPT_MAX_DIRS];         /* Tr(H2 P1) (order >= 2) */
  double tr_h2p2[DMPT_MAX_DIRS];         /* Tr(H2 P2) (order 3) */
  double tr_h3p0[DMPT_MAX_DIRS];         /* Tr(H3 P0) (order 3) */
  double tr_h3p1[DMPT_MAX_DIRS];         /* Tr(H3 P1) (order 3) */
  /* Free-energy responses by Eq. Resp_0, Omega^(m) = (1/m) sum_{k=1..m} k Tr[H^(k) P^(m-k)]
   * (H^(k) = 0 for k > order): Omega^(m) for m <= order + 1, 0 otherwise */
  double omega1[DMPT_MAX_DIRS];          /* Tr(H1 P0) */
  double omega2[DMPT_MAX_DIRS];          /* Tr(H1 P1) / 2 + Tr(H2 P0) */
  double omega3[DMPT_MAX_DIRS];          /* (Tr(H1 P2) + 2 Tr(H2 P1) + 3 Tr(H3 P0)) / 3 */
  double omega4[DMPT_MAX_DIRS];          /* (Tr(H1 P3) + 2 Tr(H2 P2) + 3 Tr(H3 P1)) / 4 */
  double idempotency;                    /* Tr[P0 (I - P0)] (check = 1) */
  double commutator;                     /* ||H0 P0 - P0 H0||_F (check = 1) */
  double asymmetry;                      /* max |P - P^T| over the outputs (check = 1) */
  double mfma_flops;                     /* matrix-core flops executed (every split product counted) */
  double useful_flops;                   /* 2 N^3 per logical matrix product */
  double seconds;                        /* wall time of the call */
} dmpt_stats;

/* Fill *opt with defaults: FP64, CG, previous-iterate guess, default tolerances. */
void dmpt_default_options(dmpt_options* opt);

/* Create a context on HIP device `device` able to handle N <= n_max
 * (1 <= n_max <= 65408) and up to dirs_max perturbation directions.  All device workspace is allocated
 * here (sized by n_max, dirs_max and opt->prec) and freed in
 * dmpt_finalize.  `hip_stream` is the caller's hipStream_t: the context
 * queues its work on it, in order with the caller's own work.  NULL stands
 * for the null (default) stream: the context then queues on a private
 * stream, and every entry point first makes that stream wait for the work
 * already queued on the null stream (an event recorded there) and at the
 * end makes the null stream wait for the context's work, so inputs written
 * by earlier kernels on the null stream are complete before they are read.
 * opt may be NULL (defaults). */
dmpt_status dmpt_init(dmpt_ctx* ctx, int device, int64_t n_max, int dirs_max,
                      const dmpt_options* opt, void* hip_stream);

/* Release a context and its workspace.  NULL is accepted. */
dmpt_status dmpt_finalize(dmpt_ctx ctx);

/* Text of the last error of ctx (a static string when ctx is NULL). */
const char* dmpt_last_error(dmpt_ctx ctx);

/* Replace the options of an existing context; the precision must not need
 * more workspace than the context was created with. */
dmpt_status dmpt_set_options(dmpt_ctx ctx, const dmpt_options* opt);

/* Grand-canonical density matrix at fixed mu: P0 = X_n of Eq. (Rec_F_2).
 * H0: N x N device FP64 (input); P0: N x N device FP64 (output). */
dmpt_status dmpt_fermi_recursion(dmpt_ctx ctx, int64_t N, const double* H0, double beta,
                                 double mu, int n, double* P0, dmpt_stats* st);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same P0 as
 * dmpt_fermi_recursion in FP64 (FP64 MFMA products, conjugate gradients from
 * the previous iterate), without a context and without any allocation.  The
 * workspace is a file-scope device array of the library (11 MiB per device,
 * held until the process ends), which limits N to 1 <= N <= 512 (larger N:
 * DMPT_ERR_ARG).  Work is queued on `hip_stream` (NULL: the null stream) of
 * the current device; the call returns without waiting and reads nothing
 * back, so every solve runs a fixed, a-priori number of CG iterations (the
 * Chebyshev bound for the system matrix's condition number of at most 2;
 * solves that converge earlier stop on the device).  Inputs are checked on the
 * device: `status` (device int, may be NULL) receives DMPT_OK,
 * DMPT_ERR_NONFINITE or DMPT_ERR_RANGE when the queued work runs; P0 is
 * meaningless unless it reads DMPT_OK.  Host-side argument errors return
 * DMPT_ERR_ARG before anything is queued (dmpt_last_error(NULL) explains).
 * Every call on a device shares that device's array: calls that overlap in
 * time on one device (two streams, two host threads) race and give wrong
 * results.  H0, P0: N x N device FP64, row major. */
dmpt_status dmpt_fermi_recursion_noalloc(int64_t N, const double* H0, double beta, double mu, int n,
                                         double* P0, int* status, void* hip_stream);

/* One pass of Algorithm 1's inner loop at a given mu jet (no Newton):
 * orders 0..order (order in {0, 1, 2, 3}: Algorithm 1's solve lines) for d
 * directions of H(lambda) = H0 + lambda H1 + lambda^2 H2 + lambda^3 H3.
 *   H1[d]  device pointers to the first-order perturbations (order >= 1)
 *   H2[d]  device pointers to second-order perturbations, or H2 == NULL / H2[i] == NULL for zero
 *   H3[d]  third-order perturbations, likewise (order 3)
 *   mu     host array: mu0, then mu1[0..d-1] (order >= 1), mu2[0..d-1] (order >= 2),
 *          mu3[0..d-1] (order 3)
 *   P0, P1[d], P2[d], P3[d]  device outputs (P1 / P2 / P3 may be NULL when order is lower). */
dmpt_status dmpt_response(dmpt_ctx ctx, int64_t N, const double* H0, int d,
                          const double* const* H1, const double* const* H2,
                          const double* const* H3, double beta, int n, int order, const double* mu,
                          double* P0, double* const* P1, double* const* P2, double* const* P3,
                          dmpt_stats* st);

/* Canonical response (Algorithm 1): Newton on the mu jet until the
 * occupation error is at most tol_occ (the mu0 step is safeguarded by a
 * bracket and bisection; options.schedule picks how mu^(k), k >= 1, are
 * found).  The context needs dirs_max >= d.  mu_inout (host, 1 + order*d
 * doubles): in, mu0 guess (NaN: Tr H0 / N) and mu^(k) guesses (NaN: 0); out,
 * the jet at which the returned P was computed.  On DMPT_ERR_NOCONV the
 * outputs and *st hold the last pass.  order in {0, 1, 2, 3}; arguments as
 * for dmpt_response. */
dmpt_status dmpt_mu_newton(dmpt_ctx ctx, int64_t N, const double* H0, int d,
                           const double* const* H1, const double* const* H2,
                           const double* const* H3, double beta, double Ne, int n, int order,
                           double* mu_inout, double* P0, double* const* P1, double* const* P2,
                           double* const* P3, dmpt_stats* st);

/* Batched canonical response: nsys independent systems of sizes Ns[s] (each
 * <= the context's n_max), with per-system beta and Ne, d directions each.
 * H0s[s], P0s[s]: N_s x N_s device FP64; H1s[s*d + i], P1s[s*d + i],
 * P2s[s*d + i] likewise (P1s / P2s may be NULL for lower orders).  mus
 * (host, nsys * (1 + 2d)): in, guesses (NaN: none); out, each system's jet.
 * st (may be NULL) receives the aggregate statistics; its mfma_flops and
 * useful_flops count the products of the members that actually ran (tallied
 * on the device; useful flops at each size bucket's padded size).  Systems
 * converge independently, one graph replay per Newton update of every
 * system still active.  order in {0, 1, 2}.  With options.schedule >= 1 and
 * order 1: mu0 first (order-0 replays, to 1e-2 tol_occ), then mu1 from a
 * guess out of the converged P0 and one order-1 replay that carries the
 * response to H1 = I and moves each P1 to Tr P1 = 0 exactly; otherwise (and
 * at order 2) Algorithm 1's joint Newton. */
dmpt_status dmpt_mu_newton_batched(dmpt_ctx ctx, int nsys, const int64_t* Ns,
                                   const double* const* H0s, int d, const double* const* H1s,
                                   const double* betas, const double* Nes, int n, int order,
                                   double* mus, double* const* P0s, double* const* P1s,
                                   double* const* P2s, dmpt_stats* st);

/* Adjoint of the canonical map: G = d Tr(Abar P0) / d H0 with mu0 following
 * H0 through Tr P0 = Ne.  mu0: host pointer to a converged mu0, or NULL to
 * solve for it first.  Abar, G: N x N device FP64 (G symmetric, so
 * dTr(Abar P0) = <G, dH> for symmetric dH).  The forward iterates are kept
 * every ckpt_every steps and recomputed in between. */
dmpt_status dmpt_backward(dmpt_ctx ctx, int64_t N, const double* H0, double beta, double Ne,
                          int n, const double* mu0, const double* Abar, double* G,
                          dmpt_stats* st);

/* Statistics of the thresholded block-sparse path (dmpt_sparse_response). */
typedef struct {
  int newton_iters;                      /* order-0 Newton passes plus the order-1 / order-2 passes */
  int block;                             /* block edge of the sparse form (32) */
  double mu[1 + 2 * DMPT_MAX_DIRS];      /* mu0, mu1[d], mu2[d] of the returned P */
  double trP[1 + 2 * DMPT_MAX_DIRS];     /* Tr P0, Tr P1[d], Tr P2[d] */
  double tr_h1p1[DMPT_MAX_DIRS];         /* Tr(H1 P1) */
  double tr_h1p2[DMPT_MAX_DIRS];         /* Tr(H1 P2) (order 2) */
  double nnz_p0;                         /* elements of P0 with |x| >= count_thr */
  double nnz_p1[DMPT_MAX_DIRS];          /* likewise for P1[d] */
  double nnz_p2[DMPT_MAX_DIRS];          /* likewise for P2[d] */
  double blocks_p0, blocks_p1[DMPT_MAX_DIRS], blocks_p2[DMPT_MAX_DIRS];  /* stored 32 x 32 blocks */
  double blocks_max;                     /* most candidate blocks of any intermediate result */
  double block_products;                 /* 32 x 32 block products formed (2 * 32^3 flop each) */
  double seconds;                        /* wall time of the call */
} dmpt_sparse_stats;

/* Thresholded block-sparse canonical response (Sec. V.B, linear scaling):
 * the recursion of Eq. Rec_F_2 and its perturbed forms to order 0, 1 or 2 in
 * 32 x 32 block-sparse FP64 storage.  After every product or combination the
 * blocks whose largest element is below tau times the largest element of the
 * result are dropped (tau = 0: no truncation, the result equals the dense
 * one up to rounding).  Each step's linear systems share T' = I + 4 D0^2 and
 * are solved with its Newton-Schulz inverse (four steps from the minimax
 * linear start), so every operation is a sparse product or combination; mu0
 * by safeguarded Newton passes, then mu1 and mu2 by the linear schedule (one
 * order-1 pass with the response J to H1 = I, one order-2 pass), as in
 * dmpt_mu_newton.  Work and memory grow with the number of stored blocks,
 * i.e. linearly in N for matrices whose significant elements lie within a
 * fixed distance of the diagonal.
 *   H0, H1[d]      N x N device FP64 inputs (dense, used through sym(.); no H2)
 *   tau            relative truncation threshold (>= 0)
 *   count_thr      elements of the returned P0, P1, P2 with |x| >= count_thr are
 *                  counted into st (e.g. 1e-5, the threshold of Fig. Fig_Scaling)
 *   blocks_per_row capacity of every sparse matrix: blocks_per_row * ceil(N / 32)
 *                  blocks (0: all); a result that does not fit gives DMPT_ERR_NOMEM
 *   mu_inout       host, 1 + order * d doubles, as for dmpt_mu_newton
 *   P0, P1[d], P2[d]  dense N x N device FP64 outputs, each may be NULL (then
 *                  only the statistics are produced)
 * N may exceed the context's n_max (the dense workspace is not used); the
 * sparse storage is allocated for the call and freed before it returns. */
dmpt_status dmpt_sparse_response(dmpt_ctx ctx, int64_t N, const double* H0, int d, const double* const* H1,
                                 double beta, double Ne, int n, int order, double tau, double count_thr,
                                 int blocks_per_row, double* mu_inout, double* P0, double* const* P1,
                                 double* const* P2, dmpt_sparse_stats* st);

/* Device-time accounting of the matrix-product kernels (the MFMA engine of
 * the context's precision).  dmpt_profile(ctx, 1) resets the totals and
 * starts recording a pair of HIP events on the context stream around every
 * product launch; dmpt_profile(ctx, 0) stops.  dmpt_profile_get
 * synchronises the context stream, resolves the pending events and reports
 * the totals since the last reset.  Intended for measurement; the events
 * add a few microseconds per launch. */
typedef struct {
  int64_t launches;      /* product kernel launches timed */
  double ms;             /* summed device time of those launches (ms) */
  double mfma_flops;     /* matrix-core flops of those launches (every split product counted) */
  double useful_flops;   /* 2 N^3 per logical product and batch member */
  /* the same, per product engine: [0] FP64, [1] FP32, [2] BF16 3-product, [3] BF16 6-product,
     [4] int8 13-product, [5] int8 6-product (their mfma_flops are int8 operations) */
  int64_t eng_launches[6];
  double eng_ms[6];
  double eng_mfma_flops[6];
  /* algorithmic HBM bytes of those launches: every operand member read once
     (BF16 planes or int8 slices for the split engines, masters otherwise; C1, C2 and W
     masters), C's master and planes written once */
  double eng_bytes[6];
  /* algorithmic flops of those launches: 2 N^3 per logical product and member */
  double eng_useful_flops[6];
} dmpt_profile_data;

dmpt_status dmpt_profile(dmpt_ctx ctx, int enable);
dmpt_status dmpt_profile_get(dmpt_ctx ctx, dmpt_profile_data* out);

/* Change of basis for a non-orthogonal basis set (Sec. II, self-consistent
 * free energy response: F_perp = Z^T F Z, D = Z D_perp Z^T, with Z the
 * inverse factor of the overlap, Z^T S Z = I).
 *   mode 0: B = Z^T A Z  (an operator into the orthogonalised basis)
 *   mode 1: B = Z A Z^T  (a density matrix or response back to the basis)
 * Z: N x N device FP64, row major, any inverse factor (need not be
 * triangular); A: N x N device FP64, used as sym(A); B: N x N device FP64
 * output, symmetrised; B must not alias A or Z.  Two FP64 MFMA products on
 * the context's workspace; not available in an FP32 context
 * (DMPT_ERR_UNSUPPORTED).  For a restricted (two electrons per state)
 * calculation with 2 Tr[D S] = Ne the orthogonalised problem has
 * Tr P_perp = Ne / 2. */
dmpt_status dmpt_congruence(dmpt_ctx ctx, int64_t N, const double* Z, const double* A, double* B,
                            int mode, dmpt_stats* st);

/* Product-kernel variants (per engine; 0 is the default):
 *   DMPT_FP64    0: 8-deep k stages, 8 waves   1: 16-deep, 8 waves   2: 8-deep, 4 waves
 *   DMPT_FP32    0: 32-deep k stages, 8 waves  1: 16-deep, 8 waves   2: 32-deep, 4 waves
 *   DMPT_BF16X3, DMPT_BF16X6 (options.acc64 = 0)
 *                0: 256 x 256 output tiles where the padded size allows   1: 128 x 128 tiles
 *   DMPT_BF16X6 with options.acc64 = 1: 0 only (128 x 128 tiles, FP64 slice sums)
 *   DMPT_INT8X13, DMPT_INT8X6  0: 128 x 128 tiles, 8 waves of 32 x 64   1: 8 waves of 64 x 32
 *                2, 3: the same with operand stages copied by LDS DMA, 64 deep
 * Every variant computes the same products; they differ in speed. */

/* Time the matrix-product kernel alone: `reps` products C = X Y^T of size N
 * (N <= n_max; X, Y, C are workspace matrices filled with a fixed pattern)
 * in precision `prec` with kernel variant `variant`.  *ms: mean device time
 * per product (HIP events on the context stream); *tflops: matrix-core
 * TFLOP/s (every split product counted).  prec must not need more workspace
 * than the context holds. */
dmpt_status dmpt_bench_product(dmpt_ctx ctx, int64_t N, dmpt_prec prec, int variant, int reps,
                               double* ms, double* tflops);

/* Product-kernel autotuner: times every variant of the context's engines
 * (its precision's, and the 6-product refinement's when enabled) at the
 * padded size of N and keeps the fastest for all later products of that
 * padded size on this context.  When the environment variable
 * DMPT_TUNE_CACHE names a file, choices are read from it (per GPU
 * architecture, engine and padded size) and new ones appended, so later
 * processes skip the timing.  *variant (may be NULL) receives the choice for
 * the context's precision. */
dmpt_status dmpt_autotune(dmpt_ctx ctx, int64_t N, int* variant);

/* Pin the product-kernel variant of precision prec's engine for the padded
 * size of N on this context (as the autotuner would). */
dmpt_status dmpt_set_variant(dmpt_ctx ctx, int64_t N, dmpt_prec prec, int variant);

/* The variant later products of precision prec at the padded size of N use:
 * *variant, *tuned (may be NULL) = 1 when it was tuned or pinned, 0 for the
 * default, and its name in name[0 .. name_len) (may be NULL). */
dmpt_status dmpt_get_variant(dmpt_ctx ctx, int64_t N, dmpt_prec prec, int* variant, int* tuned,
                             char* name, int name_len);

#ifdef __cplusplus
}
#endif

#endif /* DMPT_H */
