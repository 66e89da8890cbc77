// Host side of the DMPT library: context and workspace, argument checks,
// the per-step recursion driver (Algorithm 1's inner loop), the canonical
// Newton loop (Algorithm 1's while loop) and the C ABI of dmpt.h.
//
// The recursion runs on D = I/2 - X (Eq. Rec_F_2 with X_0 = I/2 - c(H - mu I),
// c = 2^-(n+2) beta):  D_0^(0) = c (H0 - mu0 I),  D_0^(k) = c (H^(k) - mu^(k) I),
// and each step solves, with T' = I + 4 D^2 (= 2 T of Algorithm 1),
//     T' Y^(0) = 2 D^(0)
//     T' Y^(1) = 2 D^(1) - 4 S^(1) Y^(0)
//     T' Y^(2) = 2 D^(2) - 4 S^(1) Y^(1) - 4 S^(2) Y^(0)
//     T' Y^(3) = 2 D^(3) - 4 S^(1) Y^(2) - 4 S^(2) Y^(1) - 4 S^(3) Y^(0)
// with S^(1) = D^(0) D^(1) + D^(1) D^(0), S^(2) = D^(0) D^(2) + D^(2) D^(0) + D^(1) D^(1),
// S^(3) = D^(0) D^(3) + D^(3) D^(0) + D^(1) D^(2) + D^(2) D^(1)
// (the lambda-expansion of T'(lambda) Y(lambda) = 2 D(lambda); these are the
// systems of Algorithm 1, up to its third order, written for D).  After n
// steps P^(0) = I/2 - D^(0), P^(k) = -D^(k).
#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "dmpt_internal.h"

using namespace dmpt;

namespace {

const char* kNoCtx = "invalid context (NULL)";

// Pinned host ints: CG active flags at [0, kIterSlot), iteration counts at
// [kIterSlot, 2 kIterSlot); one solve covers at most kIterSlot members.
constexpr int kIterSlot = 512;

struct Group {
  void* m = nullptr;             // master base, members at m + z * stride elements
  uint16_t* pl[3] = {nullptr, nullptr, nullptr};
  int8_t* q8 = nullptr;          // int8 slices (I8S4, I8S3), members 4 stride bytes apart
  double* qs = nullptr;          // their q, one per member
  int count = 0;
};

// Slicing state of a group with int8 slices: a member is re-sliced before a
// product reads it when a plane writer touched its group since (plane
// writers mark every member from the first they write to the end).
struct Q8Reg {
  const char* m = nullptr;
  int64_t stride = 0;            // member stride (elements)
  int count = 0;
  int8_t* q8 = nullptr;
  double* qs = nullptr;
  std::vector<char> dirty;
  // max |x| of the tiles of each member as the int8 product that last wrote
  // it left them (mx + z * mx_cap; mx_n[z] of them, 0: unknown, scan again)
  double* mx = nullptr;
  int64_t mx_cap = 0;
  std::vector<int> mx_n;
};
// Members sliced by one launch pair at most (the block maxima of a launch
// fill kQ8Chunk * 1024 doubles of the context's buffer).
constexpr int kQ8Chunk = 64;

// The matrices and solver scalars one recursion pass works on.  Members of
// the per-direction groups are laid out [system][direction]; the single
// system entry points use one system.
struct WS {
  Group D0, D1, D2, D3, S0, S1, S2, S3, R, P, Q;
  Group Zi;                      // T'^-1 of the current step (Newton-Schulz solver): two members,
                                 // the iteration alternates them (ctx zcur: the current one)
  double* rr = nullptr;          // CG <r,r> history [member][hstride]
  double* pq = nullptr;          // CG <p,Tp> history [member][hstride]
  double* pb = nullptr;          // CG bounds of max |P| for its int8 slices [member][hstride]
  double* ref = nullptr;         // ||rhs||^2 [member]
  int* active = nullptr;         // CG masks [member]
  int* iters = nullptr;          // CG iteration counters [member]
  int* mask0 = nullptr;          // system mask (order-0 members), batched passes only
  int* mask1 = nullptr;          // system mask expanded to [system][direction] members
};

}  // namespace

struct dmpt_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // private stream standing in for the null stream: every entry point
  // orders it after the null stream's queued work (ev_in) and the null
  // stream after it (ev_out)
  bool sync_null = false;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int64_t n_max = 0, np_max = 0;
  int dirs_max = 0;
  dmpt_options opt{};
  size_t esize = 8;              // master element size of the workspace
  int planes = 0;                // BF16 planes per operand allocated
  bool q8 = false;               // operand groups carry int8 slices (I8S4, I8S3)
  std::vector<Q8Reg> q8reg;
  double* d_qpart = nullptr;     // block maxima of the slicing launches
  double* d_dpart = nullptr;     // partial diagonal tiles of split symmetric int8 products
  int dpart_members = 0;
  int diag_split = 4;            // parts per diagonal tile (DMPT_DIAG_SPLIT; 0: no split)
  std::vector<void*> allocs;
  // matrix groups and solver scalars of the single-system entry points
  WS ws;
  // adjoint workspace, allocated by the first dmpt_backward that needs it:
  // seeds AY, CG unknowns AU, transposes AW, products AV, AG, the iterate
  // D_m (AD), checkpoints CK and the recomputed segment SG
  Group AY, AU, AW, AV, AG, AD, CK, SG;
  std::vector<void*> ad_allocs;
  // every device allocation of the context (base, bytes): launches are
  // checked against it on the host before they are queued
  std::vector<std::pair<const char*, size_t>> regions;
  double* d_tally = nullptr;     // [executed MFMA flops, useful flops] of graph-replayed products
  bool log = false;              // DMPT_LOG set: one line per Newton pass on stderr
  // DMPT_DEBUG_CHECKS set: every product's output is scanned for non-finite
  // values and, after every recursion step, every iterate for non-finite values
  // and exact symmetry (host-synchronising; passes recorded for a graph skip it)
  bool debug = false;
  double* d_dbg = nullptr;       // per-block maxima of the asymmetry scans
  // product-kernel variant per (engine, padded size): chosen by the autotuner or pinned
  struct Tuned {
    int eng;
    int64_t Np;
    int variant;
  };
  std::vector<Tuned> tuned;
  // iterates of the previous Newton pass (FP32 copies, warm starts):
  // [step][jet member] of tj_np^2 each; tj_valid = highest order stored
  float* tj = nullptr;
  size_t tj_bytes = 0;
  // master-precision chains of the linear schedule's order-1 pass: per step,
  // the order-0 solution and the order-1 solutions of its d + 1 jets
  void* st = nullptr;
  size_t st_bytes = 0;
  // square terms of the order-1 pass of every step (S0 and the d + 1 S1 jets),
  // loaded by the order-2 pass instead of forming them again (optional)
  void* ss = nullptr;
  size_t ss_bytes = 0;
  // per step the shared inverse Z of T' (Newton-Schulz passes of the linear
  // schedule: the order-1 pass saves it, the order-2 and -3 passes load it)
  void* zs = nullptr;
  size_t zs_bytes = 0;
  int zcur = 0;                  // member of ws.Zi that holds the current step's inverse
  bool zs_valid = false;         // zs holds this call's inverses of a pass at mu0 = zs_mu0
  double zs_mu0 = 0.0;
  int ns_iters_env = 0;          // DMPT_NS_ITERS (debugging): Newton-Schulz steps in every step
  int ns_refine_env = -1;        // DMPT_NS_REFINE (debugging): refinement step off (0) or on (1)
  bool full_tiles = false;       // DMPT_FULL_TILES set: symmetric products compute every tile
  bool ns_cold = false;          // DMPT_NS_COLD set: no Newton-Schulz start from stored inverses
  int64_t tj_np = 0;
  int tj_valid = -1;
  Group U0;                      // order-0 CG unknown when the guess comes from tj
  double* jout = nullptr;        // N x N FP64: response to H1 = I (linear schedule)
  // larger partial-sum blocks allocated by batched calls
  std::vector<void*> bt_allocs;
  // scalars
  int hstride = 0;               // CG history length per right-hand side
  int* d_flag = nullptr;         // non-finite flag
  double* d_res = nullptr;       // results block (traces etc.)
  double* d_part = nullptr;      // partials
  size_t part_count = 0;
  double* d_gersh = nullptr;     // 2 + 2 n_max
  double* h_res = nullptr;       // pinned mirror of d_res
  int* h_int = nullptr;          // pinned ints: CG active flags, then iteration counts at kIterSlot
  std::string err;
  // product-kernel timing (dmpt_profile)
  bool prof_on = false;
  struct Timed {
    hipEvent_t a, b;
    double mfma, useful, bytes;
    int eng;
  };
  std::vector<Timed> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  dmpt_profile_data prof{};
  // per-call statistics accumulators
  double mfma_flops = 0, useful_flops = 0;
  long cg_total = 0;
  int cg_max = 0;
  bool cg_capped = false;
  int flags = 0;                 // DMPT_FLAG_* of the call
  long cg_unconv = 0;            // graph-replayed solves that ended above tol_cg
  // graph-replayed solves: [0] iterations summed, [1] largest count, [2] unconverged solves
  int* d_cgstat = nullptr;
};

namespace {

// Layout of the results block d_res.
enum : int {
  RES_TR = 0,                          // Tr P0, Tr P1[d], Tr P2[d], Tr P3[d]
  RES_ATR = RES_TR + 1 + 3 * DMPT_MAX_DIRS,
  RES_FRO = RES_ATR + 1 + 3 * DMPT_MAX_DIRS,
  // response traces Tr[H^(k) P^(j)], k = 1..3, j = 0..3, per direction:
  // RES_HP + ((k - 1) * 4 + j) * DMPT_MAX_DIRS + z
  RES_HP = RES_FRO + 1,
  RES_MISC = RES_HP + 12 * DMPT_MAX_DIRS,  // scratch scalars
  RES_HALF = RES_MISC + 15,             // constant 1/2
  RES_COUNT = RES_MISC + 16
};

inline int res_hp(int k, int j, int z) { return RES_HP + ((k - 1) * 4 + j) * DMPT_MAX_DIRS + z; }

// DMPT_LOG lines: seconds on the host's steady clock (differences time the
// passes, each of which ends with a stream synchronisation) and the executed
// matrix-core work so far.
double log_clock() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

dmpt_status fail(dmpt_ctx c, dmpt_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(ctx, expr)                                                             \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail((ctx), DMPT_ERR_HIP,                                                \
                  std::string("HIP error: ") + hipGetErrorString(e_) + " in " #expr); \
  } while (0)

#define STCHK(expr)                    \
  do {                                 \
    dmpt_status s_ = (expr);           \
    if (s_ != DMPT_OK) return s_;      \
  } while (0)

// A context created without a caller stream works on a private stream that
// stands in for the null stream: order it after the work already queued on
// the null stream before any device work of a call ...
dmpt_status enter_call(dmpt_ctx c) {
  // the caller may have changed anything since the last call
  for (auto& r : c->q8reg) std::fill(r.dirty.begin(), r.dirty.end(), 1);
  if (c->sync_null) {
    HIPCHK(c, hipEventRecord(c->ev_in, nullptr));
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_in, 0));
  }
  return DMPT_OK;
}

// ... and the null stream after the call's work, on every return path.
struct CallScope {
  dmpt_ctx c = nullptr;
  ~CallScope() {
    if (c && c->sync_null && hipEventRecord(c->ev_out, c->stream) == hipSuccess)
      (void)hipStreamWaitEvent(nullptr, c->ev_out, 0);
  }
};

#define ENTER(ctx)             \
  CallScope scope_{};          \
  STCHK(enter_call(ctx));      \
  scope_.c = (ctx)

dmpt_status autotune_if_asked(dmpt_ctx c, int64_t N);

// A roctx range over a scope (Newton passes, recursion steps, graph replays):
// `rocprofv3 --marker-trace` shows them on the host timeline.
struct Range {
  explicit Range(const char* fmt, ...) __attribute__((format(printf, 2, 3))) {
    char buf[96];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    roctxRangePushA(buf);
  }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

Engine engine_of(dmpt_prec p) {
  switch (p) {
    case DMPT_FP64: return Engine::F64;
    case DMPT_FP32: return Engine::F32;
    case DMPT_BF16X3: return Engine::BF16S2;
    case DMPT_BF16X6: return Engine::BF16S3;
    case DMPT_INT8X13: return Engine::I8S4;
    case DMPT_INT8X6: return Engine::I8S3;
  }
  return Engine::F64;
}

// Modes whose converged passes options.refine can finish in a finer engine.
bool refinable(dmpt_prec p) { return p == DMPT_BF16X3 || p == DMPT_INT8X6; }
// The engine and precision of those final passes (options.refine 1 or 2).
Engine refine_engine(const dmpt_options& o) { return o.refine == 2 ? Engine::I8S4 : Engine::BF16S3; }
dmpt_prec final_prec(dmpt_prec p, int refine) {
  if (refinable(p) && refine) return refine == 2 ? DMPT_INT8X13 : DMPT_BF16X6;
  return p;
}

double default_tol_cg(dmpt_prec p, int refine) {
  p = final_prec(p, refine);
  switch (p) {
    case DMPT_FP64: return 1e-14;
    case DMPT_FP32: return 1e-9;
    case DMPT_BF16X3: return 1e-5;
    case DMPT_BF16X6: return 1e-9;
    case DMPT_INT8X13: return 1e-9;
    case DMPT_INT8X6: return 1e-7;
  }
  return 1e-14;
}

// Tolerances of the 3-product passes that precede the 6-product refinement
// (they only bring the mu jet close; the 3-product split's rounding sits
// near 1e-6 of the occupation).
constexpr double kPhaseATolCg = 1e-5;
constexpr double kPhaseATolOcc = 1e-5;
// With 6-product int8 products and the shared inverse the first phase's
// traces are within ~1e-8 of the final engine's, so its one Newton step from
// an occupation error below this lands in the final engine's quadratic
// regime (banded N = 8192: 3.6e-4 -> 2.2e-7) and one pass of the first phase
// suffices.
constexpr double kPhaseATolOccI8 = 5e-4;
// When the first phase meets its tolerance with an occupation error below
// this, its Newton step is not taken: the error is then within that phase's
// own trace bias (the 3-product split's rounding), and a step on it moves mu0
// away (banded N = 8192: from 1.3e-7 to 6e-6 of the occupation, measured by
// the int8 pass that follows).
constexpr double kPhaseABias = 3e-5;

double default_tol_occ(dmpt_prec p, int refine) {
  p = final_prec(p, refine);
  switch (p) {
    case DMPT_FP64: return 1e-12;
    case DMPT_FP32: return 1e-7;
    case DMPT_BF16X3: return 1e-6;
    case DMPT_BF16X6: return 1e-7;
    case DMPT_INT8X13: return 1e-7;
    case DMPT_INT8X6: return 1e-6;
  }
  return 1e-12;
}

int planes_needed(const dmpt_options& o) {
  int p = engine_planes(engine_of(o.prec));
  if (refinable(o.prec) && o.refine == 1) p = 3;
  return p;
}

bool q8_needed(const dmpt_options& o) {
  return o.prec == DMPT_INT8X13 || o.prec == DMPT_INT8X6 || (refinable(o.prec) && o.refine == 2);
}

// Master copies (iterates, solver vectors) are FP64 in every mode; the
// modes differ in the products only.
size_t esize_needed(const dmpt_options&) { return 8; }

// A launch of the recursion step code kept for a grouped replay: a product
// (its arguments) or any other launch (a closure that issues it).
struct Op {
  bool gemm = false;
  GemmArgs ga{};
  std::function<hipError_t()> fn;
};

// ------------------------------------------------------------------ views
struct Call {
  dmpt_ctx c;
  const WS* w;                   // matrices and scalars of this pass
  Engine eng;
  int np;                        // planes used by the engine
  int64_t N, Np, nn;             // nn = Np*Np
  int64_t stride;                // member stride of every group (elements)
  double tol_cg;                 // relative residual of every solve of this pass
  int m = 1;                     // systems in the pass (members of D0, S0)
  bool graph = false;            // no host synchronisation: fixed CG iteration counts
  int cg_iters = 0;              // iterations per solve when graph is set
  bool traj = false;             // single system: read / write the trajectory c->tj
  int jets = 1;                  // members per step in c->tj (1 + 2 d)
  int chain = 0;                 // kSave01 | kLoad01 | kSave2 | kLoad2 (c->st, see st_ptr), kSaveS | kLoadS
  int cs = 0;                    // members per step in c->st
  int cj = 0;                    // member of the J jet's solution in c->st (1 + d)
  const double* cmu = nullptr;   // chain loads: mu1[d], mu2[d]; D^(k) = D^(k)(mu = 0) - mu D_J
  double* part = nullptr;        // partial sums of this call's products and reductions
  size_t part_count = 0;         // ... and their capacity
  std::vector<Op>* rec = nullptr;  // when set, launches are recorded here instead of issued
  double glo = NAN, ghi = NAN;   // Gershgorin interval of sym(H0), when the caller scanned it
  double d0b = -1.0;             // this pass: a bound on ||D_0||_2 (< 0: none known)
  int jdir = -1;                 // order-1 member that is the response J to H1 = I (linear schedule)
  bool first_phase = false;      // a pass of the loose first phase before the final engine's passes
  double cscale = 0.0;           // this pass: c = beta 2^-(n+2)
  int nsteps = 0;                // this pass: recursion steps n
  double z_dmu = -1.0;           // |mu0 - mu0 of the stored inverses| (kWarmZ; < 0: none)
};

// Issue a launch of the recursion step code now, or record it (k.rec).
#define EMIT(k, expr)                                                          \
  do {                                                                         \
    if ((k).rec) {                                                             \
      Op op_;                                                                  \
      op_.fn = [=]() { return (expr); };                                      \
      (k).rec->push_back(op_);                                                 \
    } else {                                                                   \
      HIPCHK((k).c, (expr));                                                   \
    }                                                                          \
  } while (0)

// Chain flags of a pass (linear schedule): save or load the order-0/1
// solutions, save or load the order-2 solutions.
constexpr int kSave01 = 1, kLoad01 = 2, kSave2 = 4, kLoad2 = 8;
// ... and save or load the square terms S0, S1 of every step (c->ss, see ss_ptr)
constexpr int kSaveS = 16, kLoadS = 32;
// ... and save or load the shared inverse Z of every step (c->zs)
constexpr int kSaveZ = 64, kLoadZ = 128;
// ... or start each step's Newton-Schulz iteration from the stored Z of a
// pass at a nearby mu0 when that needs fewer steps (see ns_warm_iters)
constexpr int kWarmZ = 256;

// Member z of a group as an operand.
BOp op(const Call& k, const Group& g, int z, bool batched) {
  BOp o;
  const size_t es = k.c->esize;
  o.m = (const char*)g.m + (size_t)z * k.stride * es;
  for (int p = 0; p < 3; ++p) o.pl[p] = g.pl[p] ? g.pl[p] + (size_t)z * k.stride : nullptr;
  o.stride = batched ? k.stride : 0;
  return o;
}

// A writer is about to change members z.. of g: their int8 slices go stale.
void q8_touch(dmpt_ctx c, const Group& g, int z, int n = -1) {
  for (auto& r : c->q8reg)
    if (r.m == (const char*)g.m) {
      // n members from z (n < 0: every member from z on)
      const int e = n < 0 ? r.count : std::min(r.count, z + n);
      for (int i = std::max(z, 0); i < e; ++i) {
        r.dirty[i] = 1;
        r.mx_n[i] = 0;
      }
      return;
    }
}
// Maxima sink of an element-wise writer of members z0 .. z0 + batch - 1 of g
// (called after planes_of, which marks them stale): the writer leaves
// `entries` partial maxima of |x| per member at the returned address (member
// stride *stride), and the next slicing of these members reads them instead
// of scanning.  Null when g has no int8 slices or the maxima do not fit.
double* q8_sink(const Call& k, const Group& g, int z0, int batch, int64_t entries, int64_t* stride) {
  if (k.rec || !engine_int8(k.eng)) return nullptr;
  for (auto& r : k.c->q8reg)
    if (r.m == (const char*)g.m) {
      if (z0 < 0 || batch < 1 || z0 + batch > r.count || entries < 1 || entries > r.mx_cap ||
          r.stride != k.stride)
        return nullptr;
      for (int i = z0; i < z0 + batch; ++i) r.mx_n[i] = (int)entries;
      *stride = r.mx_cap;
      return r.mx + (size_t)z0 * r.mx_cap;
    }
  return nullptr;
}
// The maxima sink of a grid-stride element-wise writer of member z of g: the
// block count it must run with in *blocks (0 without a sink).
double* ew_sink(const Call& k, const Group& g, int z, int64_t* stride, int64_t* blocks) {
  *blocks = 0;
  for (auto& r : k.c->q8reg)
    if (r.m == (const char*)g.m) {
      const int64_t e = ew_sink_blocks(k.nn, r.mx_cap);
      double* mx = q8_sink(k, g, z, 1, e, stride);
      if (mx) *blocks = e;
      return mx;
    }
  return nullptr;
}
void* mptr(const Call& k, const Group& g, int z) {
  return (char*)g.m + (size_t)z * k.stride * k.c->esize;
}
// The planes of member z of g for a writer of n members from z (n < 0: the
// writer may cover every member from z on); their int8 slices go stale.
void planes_of(const Call& k, const Group& g, int z, uint16_t** out, int n = -1) {
  for (int p = 0; p < 3; ++p)
    out[p] = (g.pl[p] && p < k.np) ? g.pl[p] + (size_t)z * k.stride : nullptr;
  q8_touch(k.c, g, z, n);
}

// C(batch members z0..z0+batch) = alpha X Y^T + beta1 C1 + beta2 C2
struct G {
  BOp X, Y;
  void* C = nullptr;
  int64_t sC = 0;
  uint16_t* Cpl[3] = {nullptr, nullptr, nullptr};
  double alpha = 1.0;
  const void* C1 = nullptr; int64_t sC1 = 0; double beta1 = 0.0;
  const void* C2 = nullptr; int64_t sC2 = 0; double beta2 = 0.0;
  const void* W = nullptr; int64_t sW = 0;
  int batch = 1;
  const int* active = nullptr;
  int counted = -1;  // members whose flops are tallied (-1: all; the host knows the others are skipped)
  bool sym = false;  // C = X Y^T is symmetric (and so are C1, C2): compute the lower triangle, mirror it
};

// ------------------------------------------------------------------ host-side bounds
void reg_add(dmpt_ctx c, void* p, size_t bytes) { c->regions.push_back({(const char*)p, bytes}); }

void reg_del(dmpt_ctx c, void* p) {
  for (size_t i = 0; i < c->regions.size(); ++i)
    if (c->regions[i].first == (const char*)p) {
      c->regions.erase(c->regions.begin() + i);
      return;
    }
}

// True when [p, p + bytes) lies inside one device allocation of the context.
bool reg_ok(dmpt_ctx c, const void* p, size_t bytes) {
  const char* q = (const char*)p;
  for (auto& r : c->regions)
    if (q >= r.first && q + bytes <= r.first + r.second) return true;
  return false;
}

// hipMalloc that records the allocation.
void* dev_alloc(dmpt_ctx c, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  reg_add(c, p, std::max<size_t>(bytes, 256));
  return p;
}

void dev_free(dmpt_ctx c, void* p) {
  if (!p) return;
  reg_del(c, p);
  (void)hipFree(p);
}

dmpt_status prof_event(dmpt_ctx c, hipEvent_t* e) {
  if (!c->prof_pool.empty()) {
    *e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return DMPT_OK;
  }
  HIPCHK(c, hipEventCreateWithFlags(e, hipEventDefault));
  return DMPT_OK;
}

// Wait for the recorded product launches and add their durations.
dmpt_status prof_resolve(dmpt_ctx c) {
  if (c->prof_pending.empty()) return DMPT_OK;
  HIPCHK(c, hipEventSynchronize(c->prof_pending.back().b));
  for (auto& t : c->prof_pending) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, t.a, t.b));
    c->prof.launches += 1;
    c->prof.ms += ms;
    c->prof.mfma_flops += t.mfma;
    c->prof.useful_flops += t.useful;
    c->prof.eng_launches[t.eng] += 1;
    c->prof.eng_ms[t.eng] += ms;
    c->prof.eng_mfma_flops[t.eng] += t.mfma;
    c->prof.eng_bytes[t.eng] += t.bytes;
    c->prof.eng_useful_flops[t.eng] += t.useful;
    c->prof_pool.push_back(t.a);
    c->prof_pool.push_back(t.b);
  }
  c->prof_pending.clear();
  return DMPT_OK;
}

// Product-kernel variant for an engine and padded size: the autotuned (or
// pinned) one, else the default.
int variant_for(dmpt_ctx c, Engine eng, int64_t Np) {
  const int acc64 = eng == Engine::BF16S3 && c->opt.acc64;
  for (auto& t : c->tuned)
    if (t.eng == (int)eng && t.Np == Np && t.variant < gemm_variants(eng, acc64)) return t.variant;
  return 0;
}

int acc64_of(dmpt_ctx c, Engine eng) { return eng == Engine::BF16S3 && c->opt.acc64 ? 1 : 0; }

// Int8 slices of a product operand (I8S4): the members the launch reads are
// sliced again where a writer touched them since their last slicing.
// Host-side bounds of the int8 operands of a launch.
bool ok_q8_bounds(const Call& k, const GemmArgs& a, int batch) {
  if (!engine_int8(k.eng)) return true;
  auto span = [&](const BOp& o) -> size_t {
    return ((o.stride ? (size_t)((batch - 1) / o.div) * (size_t)o.stride : 0) + (size_t)k.nn) * kQ8Slices;
  };
  auto nq = [&](const BOp& o) -> size_t { return (o.stride ? (size_t)((batch - 1) / o.div) : 0) + 1; };
  return a.X.q8 && a.Y.q8 && reg_ok(k.c, a.X.q8, span(a.X)) && reg_ok(k.c, a.Y.q8, span(a.Y)) &&
         reg_ok(k.c, a.X.qs, nq(a.X) * sizeof(double)) && reg_ok(k.c, a.Y.qs, nq(a.Y) * sizeof(double));
}

dmpt_status q8_operand(const Call& k, BOp& o, int batch) {
  dmpt_ctx c = k.c;
  const char* p = (const char*)o.m;
  for (auto& r : c->q8reg) {
    const size_t mb = (size_t)r.stride * c->esize;
    if (p < r.m || p >= r.m + mb * r.count) continue;
    const size_t off = (size_t)(p - r.m);
    const int n = o.stride ? (batch - 1) / o.div + 1 : 1;
    const int z0 = (int)(off / mb);
    if (off % mb || r.stride != k.stride || z0 + n > r.count)
      return fail(c, DMPT_ERR_ARG, "internal: an int8 operand does not match its group's members");
    for (int z = z0; z < z0 + n;) {
      if (!r.dirty[z]) {
        ++z;
        continue;
      }
      // a run of dirty members with the same kind of maxima (known from the
      // product that wrote them, with the same tile count, or unknown)
      const int kn = r.mx_n[z];
      int e = z;
      while (e < z0 + n && r.dirty[e] && r.mx_n[e] == kn && e - z < kQ8Chunk) ++e;
      const double* src = (const double*)(r.m + (size_t)z * mb);
      int8_t* dst = r.q8 + (size_t)z * r.stride * kQ8Slices;
      double* qd = r.qs + z;
      const int cnt = e - z;
      const int64_t st = r.stride, Np = k.Np;
      double* part = c->d_qpart;
      hipStream_t s = c->stream;
      if (kn > 0) {
        const double* known = r.mx + (size_t)z * r.mx_cap;
        const int64_t cap = r.mx_cap;
        EMIT(k, quantize_q8_known(src, st, Np, cnt, known, cap, kn, dst, st * kQ8Slices, qd, s));
      } else {
        EMIT(k, quantize_q8(src, st, Np, cnt, part, dst, st * kQ8Slices, qd, nullptr, s));
      }
      for (int i = z; i < e; ++i) r.dirty[i] = 0;
      z = e;
    }
    o.q8 = r.q8 + (size_t)z0 * r.stride * kQ8Slices;
    o.qs = r.qs + z0;
    return DMPT_OK;
  }
  return fail(c, DMPT_ERR_ARG, "internal: an int8 product operand lies outside the sliced workspace");
}

dmpt_status run_gemm(const Call& k, const G& g) {
  GemmArgs a{};
  a.eng = k.eng;
  a.Np = k.Np;
  a.batch = g.batch;
  a.X = g.X;
  a.Y = g.Y;
  a.C = g.C;
  a.sC = g.sC;
  for (int p = 0; p < 3; ++p) a.Cpl[p] = (p < k.np) ? g.Cpl[p] : nullptr;
  a.alpha = g.alpha;
  a.C1 = g.C1; a.sC1 = g.sC1; a.beta1 = g.beta1;
  a.C2 = g.C2; a.sC2 = g.sC2; a.beta2 = g.beta2;
  a.W = g.W; a.sW = g.sW;
  a.partials = k.part;
  a.active = g.active;
  a.variant = variant_for(k.c, k.eng, k.Np);
  a.acc64 = acc64_of(k.c, k.eng);
  // recorded launches (graph replays, grouped launches) keep every tile
  a.sym = g.sym && !k.rec && !g.W && !k.c->full_tiles ? 1 : 0;
  if (a.sym && engine_int8(k.eng) && k.c->d_dpart) {
    a.dpart = k.c->d_dpart;
    a.dsplit = k.c->diag_split;
    a.dpart_members = k.c->dpart_members;
  }
  if (engine_int8(k.eng)) {
    if (k.Np > kQ8MaxK) return fail(k.c, DMPT_ERR_UNSUPPORTED, "int8 products need N <= 32768");
    STCHK(q8_operand(k, a.X, g.batch));
    STCHK(q8_operand(k, a.Y, g.batch));
    // the output's slices go stale too (C may be an operand group); when C
    // is whole members of a sliced group, the kernel leaves their tile
    // maxima for the next slicing
    for (auto& r : k.c->q8reg) {
      const size_t mb = (size_t)r.stride * k.c->esize;
      const char* p = (const char*)a.C;
      if (p >= r.m && p < r.m + mb * r.count) {
        const int z0 = (int)((size_t)(p - r.m) / mb);
        // C as whole members z0 .. z0 + batch - 1: exactly those go stale (an
        // operand member beside them keeps its slices), else every member from z0
        const bool whole = (size_t)(p - r.m) % mb == 0 && (g.batch == 1 || a.sC == r.stride) &&
                           z0 + g.batch <= r.count;
        for (int i = z0; i < (whole ? z0 + g.batch : r.count); ++i) {
          r.dirty[i] = 1;
          r.mx_n[i] = 0;
        }
        const int64_t tiles = gemm_cmax_entries(a);
        if (!k.rec && !g.active && whole && tiles <= r.mx_cap) {
          a.cmax = r.mx + (size_t)z0 * r.mx_cap;
          a.cmax_stride = r.mx_cap;
          for (int i = z0; i < z0 + g.batch; ++i) r.mx_n[i] = (int)tiles;
        }
      }
    }
  }
  // every member the launch touches must lie inside a workspace allocation
  {
    dmpt_ctx c = k.c;
    const size_t es = c->esize, nn = (size_t)k.nn;
    const int b = g.batch;
    auto span = [&](int64_t stride, int div) -> size_t {
      return (stride ? (size_t)((b - 1) / div) * (size_t)stride : 0) + nn;
    };
    bool ok = b >= 1 && reg_ok(c, a.X.m, span(a.X.stride, a.X.div) * es) &&
              reg_ok(c, a.Y.m, span(a.Y.stride, a.Y.div) * es) && reg_ok(c, a.C, span(a.sC, 1) * es);
    for (int p = 0; p < k.np && ok; ++p)
      ok = a.X.pl[p] && a.Y.pl[p] && reg_ok(c, a.X.pl[p], span(a.X.stride, a.X.div) * 2) &&
           reg_ok(c, a.Y.pl[p], span(a.Y.stride, a.Y.div) * 2);
    for (int p = 0; p < 3 && ok; ++p)
      if (a.Cpl[p]) ok = reg_ok(c, a.Cpl[p], span(a.sC, 1) * 2);
    if (ok && a.C1) ok = reg_ok(c, a.C1, span(a.sC1, 1) * es);
    if (ok && a.C2) ok = reg_ok(c, a.C2, span(a.sC2, 1) * es);
    if (ok && a.W) ok = reg_ok(c, a.W, span(a.sW, 1) * es) &&
                        (size_t)b * gemm_tiles(k.eng, k.Np, a.variant, a.acc64) <= k.part_count;
    if (ok && b > 1) ok = a.sC != 0;
    if (!ok) return fail(c, DMPT_ERR_ARG, "internal: a product would leave its workspace");
  }
  if (ok_q8_bounds(k, a, g.batch) == false)
    return fail(k.c, DMPT_ERR_ARG, "internal: an int8 operand would leave its workspace");
  // the share of the output tiles computed (below 1 for symmetric outputs)
  const double tf = (double)gemm_launch_tiles(a) / (double)gemm_tiles(k.eng, k.Np, a.variant, a.acc64);
  const double n3 = 2.0 * (double)k.Np * k.Np * k.Np * tf;
  if (k.graph) {
    // replays skip converged members on the device: count there
    a.tally = k.c->d_tally;
    a.tally_m = n3 * engine_terms(k.eng);
    a.tally_u = 2.0 * (double)k.N * k.N * k.N;
  }
  const int members = g.counted >= 0 ? g.counted : g.batch;
  const double mf = n3 * engine_terms(k.eng) * members;
  const double uf = 2.0 * (double)k.N * k.N * k.N * tf * members;
  dmpt_ctx c = k.c;
  // algorithmic bytes: distinct operand members read once, C written once
  double bytes = 0.0;
  {
    const double nn = (double)k.nn, es = (double)c->esize;
    // bytes per element of an operand as the kernel reads it
    const double opb = k.eng == Engine::I8S4 ? 4.0 : (k.eng == Engine::I8S3 ? 3.0 : (k.np ? 2.0 * k.np : es));
    auto distinct = [&](const BOp& o) { return o.stride ? (double)((members - 1) / o.div + 1) : 1.0; };
    bytes += (distinct(a.X) + distinct(a.Y)) * nn * opb;
    bytes += members * nn * es * (1.0 + (a.C1 ? 1.0 : 0.0) + (a.C2 ? 1.0 : 0.0) + (a.W ? 1.0 : 0.0));
    for (int p = 0; p < 3; ++p)
      if (a.Cpl[p]) bytes += members * nn * 2.0;
  }
  if (k.rec) {
    Op o;
    o.gemm = true;
    o.ga = a;
    k.rec->push_back(o);
    c->mfma_flops += mf;
    c->useful_flops += uf;
    return DMPT_OK;
  }
  hipEvent_t ea = nullptr, eb = nullptr;
  if (c->prof_on) {
    if (c->prof_pending.size() >= 2048) STCHK(prof_resolve(c));
    STCHK(prof_event(c, &ea));
    STCHK(prof_event(c, &eb));
    HIPCHK(c, hipEventRecord(ea, c->stream));
  }
  HIPCHK(c, gemm(a, c->stream));
  if (c->prof_on) {
    HIPCHK(c, hipEventRecord(eb, c->stream));
    c->prof_pending.push_back({ea, eb, mf, uf, bytes, (int)k.eng});
  }
  c->mfma_flops += mf;
  c->useful_flops += uf;
  if (c->debug && !k.graph) {
    HIPCHK(c, set_values(c->d_flag + 1, 0, 1, nullptr, 0.0, 0, c->stream));
    for (int z = 0; z < g.batch; ++z)
      HIPCHK(c, nonfinite_scan((const double*)((const char*)a.C + (size_t)z * a.sC * c->esize), k.Np, k.Np,
                               c->d_flag + 1, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->h_int, c->d_flag + 1, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->h_int[0]) {
      char msg[128];
      std::snprintf(msg, sizeof msg, "debug check: a product (engine %d, Np %lld) wrote a non-finite value",
                    (int)k.eng, (long long)k.Np);
      return fail(c, DMPT_ERR_NONFINITE, msg);
    }
  }
  return DMPT_OK;
}

// Sum the GEMM per-tile partials into out[z*ostride + oidx].
dmpt_status sum_gemm_partials(const Call& k, int batch, double* out, int ostride, int oidx) {
  const int tiles = gemm_tiles(k.eng, k.Np, variant_for(k.c, k.eng, k.Np), acc64_of(k.c, k.eng));
  hipStream_t s = k.c->stream;
  double* part = k.part;
  EMIT(k, sum_partials(part, tiles, batch, out, ostride, oidx, s));
  return DMPT_OK;
}

// ------------------------------------------------------------------ typed helpers
template <class T>
dmpt_status sym_inplace(const Call& k, const Group& g, int z0, int batch, double a) {
  if (z0 < 0 || z0 + batch > g.count) return fail(k.c, DMPT_ERR_ARG, "internal: sym batch too large");
  uint16_t* pl[3];
  planes_of(k, g, z0, pl);
  T* m = (T*)mptr(k, g, z0);
  hipStream_t s = k.c->stream;
  int64_t ms = 0;
  double* mx = q8_sink(k, g, z0, batch, sym_pair_blocks(k.Np), &ms);
  EMIT(k, (sym_combine<T, T>(m, k.Np, k.stride, k.N, k.Np, a, nullptr, 0, m, k.Np, k.stride, pl, k.np, batch,
                             s, nullptr, 0.0, nullptr, mx, ms)));
  return DMPT_OK;
}

// out group (members z0..) = a (in + in^T), in and out distinct groups.
template <class T>
dmpt_status sym_to(const Call& k, const Group& in, const Group& out, int batch, bool planes) {
  if (batch > in.count || batch > out.count) return fail(k.c, DMPT_ERR_ARG, "internal: sym batch too large");
  uint16_t* pl[3];
  planes_of(k, out, 0, pl);
  const T* src = (const T*)mptr(k, in, 0);
  T* dst = (T*)mptr(k, out, 0);
  const int npl = planes ? k.np : 0;
  hipStream_t s = k.c->stream;
  int64_t ms = 0;
  double* mx = q8_sink(k, out, 0, batch, sym_pair_blocks(k.Np), &ms);
  EMIT(k, (sym_combine<T, T>(src, k.Np, k.stride, k.N, k.Np, 1.0, nullptr, 0, dst, k.Np, k.stride, pl, npl,
                             batch, s, nullptr, 0.0, nullptr, mx, ms)));
  return DMPT_OK;
}

// Every solve also reduces its initial residual by this factor at least (see
// k_cg_check): warm starts must not freeze the iterate below the tolerance.
constexpr double kEta = 0.05;

// Conjugate gradients on the transposed unknowns U (U T' = R^T, see gemm.hip):
//   U (group `u`, members z = 0..batch-1) holds the initial guess and
//   receives the solution; R holds the initial residual, whose squared norm
//   is in rr[z][0]; ref[z] holds ||rhs||^2.  S0 member z / ydiv is the
//   system matrix factor of member z.  `mask` (or all ones) seeds the
//   per-member activity.  Without k.graph the host checks the masks after
//   every iteration and stops when all members converged; with k.graph a
//   fixed k.cg_iters iterations are queued and converged members skip their
//   work on the device.
template <class T>
dmpt_status cg_solve(const Call& k, const Group& u, int batch, int ydiv, const int* mask) {
  dmpt_ctx c = k.c;
  const WS* w = k.w;
  if (batch < 1 || ydiv < 1 || u.count < batch || w->R.count < batch || w->P.count < batch ||
      w->Q.count < batch || w->S0.count < (batch - 1) / ydiv + 1 || batch > kIterSlot ||
      (size_t)batch * reduce_blocks(k.nn) > k.part_count)
    return fail(c, DMPT_ERR_ARG, "internal: solve batch exceeds its workspace");
  if (k.rec && !k.graph) return fail(c, DMPT_ERR_ARG, "internal: recorded solves need fixed counts");
  hipStream_t s = c->stream;
  const int hs = c->hstride;
  const double tol = k.tol_cg;
  const int64_t n = k.nn;
  const int64_t st = k.stride;
  const int np = k.np;
  double* part = k.part;
  int* act = w->active;
  int* its = w->iters;
  double* rr = w->rr;
  double* pq = w->pq;
  const double* ref = w->ref;
  T* U = (T*)mptr(k, u, 0);
  T* R = (T*)mptr(k, w->R, 0);
  T* P = (T*)mptr(k, w->P, 0);
  const T* Q = (const T*)mptr(k, w->Q, 0);
  uint16_t* ppl[3];
  planes_of(k, w->P, 0, ppl);
  // P = R (with planes)
  EMIT(k, axpby<T>(R, st, P, st, n, batch, 1.0, 0.0, ppl, st, np, s));
  if (mask) EMIT(k, expand_mask(mask, 1, act, batch, s));
  else EMIT(k, set_values(act, 1, batch, nullptr, 0.0, 0, s));
  EMIT(k, set_values(its, 0, batch, nullptr, 0.0, 0, s));
  EMIT(k, cg_check(rr, rr, ref, hs, batch, tol * tol, kEta * kEta, act, its, s));
  const int red_nb = reduce_blocks(n);
  // int8 products: from the second iteration on, the direction update writes
  // P's slices itself (its scale from a bound on max |P|), so P is not sliced
  // again before the next product
  Q8Reg* preg = nullptr;
  if constexpr (std::is_same<T, double>::value) {
    if (engine_int8(k.eng) && !k.rec && w->pb && c->d_qpart && batch <= kQ8Chunk)
      for (auto& r : c->q8reg)
        if (r.m == (const char*)w->P.m && r.stride == k.stride && r.count >= batch) preg = &r;
  }
  const int cap = k.graph ? std::min(k.cg_iters, c->opt.max_cg) : c->opt.max_cg;
  for (int it = 0; it < cap && it + 1 < hs; ++it) {
    int live = -1;  // members still iterating (known on the host without a graph)
    if (!k.graph) {
      HIPCHK(c, hipMemcpyAsync(c->h_int, w->active, batch * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      live = 0;
      for (int z = 0; z < batch; ++z) live += c->h_int[z] != 0;
      if (!live) break;
    }
    // Q = P + 4 P S0  (T' applied on the right), partials of <P, Q>
    G g;
    g.X = op(k, w->P, 0, true);
    g.Y = op(k, w->S0, 0, true);
    g.Y.div = ydiv;
    g.C = mptr(k, w->Q, 0);
    g.sC = k.stride;
    g.alpha = 4.0;
    g.C1 = mptr(k, w->P, 0); g.sC1 = k.stride; g.beta1 = 1.0;
    g.W = mptr(k, w->P, 0); g.sW = k.stride;
    g.batch = batch;
    g.active = w->active;
    g.counted = live;
    STCHK(run_gemm(k, g));
    STCHK(sum_gemm_partials(k, batch, w->pq + it, hs, 0));
    if (preg && it == 0) EMIT(k, q8_bound_init(preg->qs, w->pb, hs, batch, s));  // P sliced exactly above
    EMIT(k, cg_update_xr<T>(U, R, P, Q, n, st, batch, rr + it, pq + it, hs, act, part, s,
                            preg ? c->d_qpart : nullptr));
    EMIT(k, sum_partials(part, red_nb, batch, rr + it + 1, hs, 0, s));
    if (preg) {
      if constexpr (std::is_same<T, double>::value) {
        EMIT(k, cg_update_p_q8(P, R, k.Np, st, batch, rr + it + 1, rr + it, hs, act, c->d_qpart, w->pb + it,
                               w->pb + it + 1, preg->q8, st * kQ8Slices, preg->qs, s));
      }
      for (int z = 0; z < batch; ++z) preg->dirty[z] = 0;
    } else {
      EMIT(k, cg_update_p<T>(P, R, n, st, batch, rr + it + 1, rr + it, hs, act, ppl, np, s));
      q8_touch(c, w->P, 0);  // ppl was fetched once: mark P's int8 slices stale on every write
    }
    EMIT(k, cg_check(rr + it + 1, rr, ref, hs, batch, tol * tol, kEta * kEta, act, its, s));
  }
  if (k.graph) {
    // fixed-count solve: its statistics accumulate on the device (read after the replays)
    int* stat = c->d_cgstat;
    EMIT(k, cg_account(act, its, batch, stat, s));
    return DMPT_OK;
  }
  HIPCHK(c, hipMemcpyAsync(c->h_int, w->active, batch * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(c->h_int + kIterSlot, w->iters, batch * sizeof(int),
                           hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  for (int z = 0; z < batch; ++z) {
    // iters counts the initial check too
    const int its = std::max(0, c->h_int[kIterSlot + z] - 1);
    c->cg_total += its;
    c->cg_max = std::max(c->cg_max, its);
    if (c->h_int[z]) c->cg_capped = true;
  }
  return DMPT_OK;
}

// Inputs of one recursion pass.
struct PassIn {
  const double* H0;
  int d;
  const double* const* H1;
  const double* const* H2;
  double beta;
  int n;
  int order;
  const double* mu;                    // mu0, mu1[d], mu2[d], mu3[d]
  const double* const* H3 = nullptr;   // third-order perturbations (NULL: zero)
};

// Group of the order-o jet (o = 1..3) and of its square term S^(o).
const Group& jet(const WS* w, int o) { return o == 1 ? w->D1 : (o == 2 ? w->D2 : w->D3); }
const Group& sqr(const WS* w, int o) { return o == 1 ? w->S1 : (o == 2 ? w->S2 : w->S3); }
// Slot of (order o >= 1, direction z) in the mu jet and in the trace results.
inline int slot_of(int o, int z, int d) { return 1 + (o - 1) * d + z; }

// Initialise D0^(k) = c (sym H^(k) - mu^(k) I) from the FP64 caller inputs.
template <class T>
dmpt_status init_d(const Call& k, const PassIn& in, double cscale) {
  dmpt_ctx c = k.c;
  const WS* w = k.w;
  hipStream_t s = c->stream;
  auto one = [&](const double* h, const Group& g, int z, double mu) -> dmpt_status {
    uint16_t* pl[3];
    planes_of(k, g, z, pl);
    T* out = (T*)mptr(k, g, z);
    if (h) {
      HIPCHK(c, (sym_combine<double, T>(h, k.N, 0, k.N, k.Np, 0.5 * cscale, nullptr, 0, out, k.Np, 0,
                                        pl, k.np, 1, s)));
      // diagonal shift -c mu applied by a scaled identity add
      HIPCHK(c, scaled_plus_identity<T>(out, out, k.N, k.Np, -cscale * mu, 1.0, pl, k.np, s));
    } else {
      HIPCHK(c, scaled_plus_identity<T>(out, out, k.N, k.Np, -cscale * mu, 0.0, pl, k.np, s));
    }
    return DMPT_OK;
  };
  STCHK(one(in.H0, w->D0, 0, in.mu[0]));
  if (in.order >= 1)
    for (int z = 0; z < in.d; ++z) STCHK(one(in.H1[z], w->D1, z, in.mu[1 + z]));
  if (in.order >= 2)
    for (int z = 0; z < in.d; ++z)
      STCHK(one(in.H2 ? in.H2[z] : nullptr, w->D2, z, in.mu[1 + in.d + z]));
  if (in.order >= 3)
    for (int z = 0; z < in.d; ++z)
      STCHK(one(in.H3 ? in.H3[z] : nullptr, w->D3, z, in.mu[1 + 2 * in.d + z]));
  return DMPT_OK;
}

// S0 = D0^2 for every system of the pass.
template <class T>
dmpt_status square0(const Call& k) {
  const WS* w = k.w;
  G g;
  g.X = op(k, w->D0, 0, true);
  g.Y = op(k, w->D0, 0, true);
  g.C = mptr(k, w->S0, 0);
  g.sC = k.stride;
  planes_of(k, w->S0, 0, g.Cpl);
  g.batch = k.m;
  g.active = w->mask0;
  g.sym = true;  // S0 = D0 D0
  return run_gemm(k, g);
}

// Pointer to the trajectory copy of jet member j at recursion step `step`.
float* tj_ptr(const Call& k, int step, int j) {
  return k.c->tj + ((size_t)step * k.jets + j) * (size_t)k.nn;
}

// Save member z of a group (its master) as trajectory entry (step, j).
bool tj_fits(const Call& k, int step, int j) {
  return step >= 0 && j >= 0 && j < k.jets &&
         ((size_t)step * k.jets + j + 1) * (size_t)k.nn * sizeof(float) <= k.c->tj_bytes;
}

template <class T>
dmpt_status tj_save(const Call& k, const Group& g, int z, int step, int j) {
  if (!tj_fits(k, step, j) || z >= g.count) return fail(k.c, DMPT_ERR_ARG, "internal: trajectory index");
  uint16_t* none[3] = {nullptr, nullptr, nullptr};
  HIPCHK(k.c, (convert<T, float>((const T*)mptr(k, g, z), 0, tj_ptr(k, step, j), 0, k.nn, 1, none, 0,
                                 0, k.c->stream)));
  return DMPT_OK;
}

// Load trajectory entry (step, j) into member z of a group (master + planes).
template <class T>
dmpt_status tj_load(const Call& k, const Group& g, int z, int step, int j) {
  if (!tj_fits(k, step, j) || z >= g.count) return fail(k.c, DMPT_ERR_ARG, "internal: trajectory index");
  uint16_t* pl[3];
  planes_of(k, g, z, pl);
  HIPCHK(k.c, (convert<float, T>(tj_ptr(k, step, j), 0, (T*)mptr(k, g, z), 0, k.nn, 1, pl, 0,
                                 g.pl[0] ? k.np : 0, k.c->stream)));
  return DMPT_OK;
}

// Chain store of the linear schedule (c->st, master precision), k.cs members
// per step: the order-0 solution (member 0), the order-1 solutions of the d
// directions and of J (members 1 .. d + 1) and, when a third-order pass
// follows, the order-2 solutions (members d + 2 .. 2d + 1).
template <class T>
T* st_ptr(const Call& k, int step, int j) {
  return (T*)k.c->st + ((size_t)step * k.cs + j) * (size_t)k.nn;
}

bool st_fits(const Call& k, int step, int j) {
  return step >= 0 && j >= 0 && j < k.cs &&
         ((size_t)step * k.cs + j + 1) * (size_t)k.nn * k.c->esize <= k.c->st_bytes;
}

// Save member z of a group (master only) as chain entry (step, j).
template <class T>
dmpt_status st_save(const Call& k, const Group& g, int z, int step, int j) {
  if (!st_fits(k, step, j) || z >= g.count) return fail(k.c, DMPT_ERR_ARG, "internal: chain index");
  uint16_t* none[3] = {nullptr, nullptr, nullptr};
  HIPCHK(k.c, (convert<T, T>((const T*)mptr(k, g, z), 0, st_ptr<T>(k, step, j), 0, k.nn, 1, none, 0,
                             0, k.c->stream)));
  return DMPT_OK;
}

// Member z of a group (with planes) = chain entry (step, j) - a * chain entry (step, jb).
template <class T>
dmpt_status st_load(const Call& k, const Group& g, int z, int step, int j, double a, int jb) {
  if (!st_fits(k, step, j) || (a != 0.0 && !st_fits(k, step, jb)) || z >= g.count)
    return fail(k.c, DMPT_ERR_ARG, "internal: chain index");
  uint16_t* pl[3];
  planes_of(k, g, z, pl);
  T* dst = (T*)mptr(k, g, z);
  int64_t ms = 0, mb = 0;
  double* mx = ew_sink(k, g, z, &ms, &mb);
  if (a == 0.0) {
    HIPCHK(k.c, (convert<T, T>(st_ptr<T>(k, step, j), 0, dst, 0, k.nn, 1, pl, 0,
                               g.pl[0] ? k.np : 0, k.c->stream, mx, ms, mb)));
  } else {
    HIPCHK(k.c, axpbyz<T>(st_ptr<T>(k, step, jb), st_ptr<T>(k, step, j), dst, k.nn, -a, 1.0, pl,
                          g.pl[0] ? k.np : 0, k.c->stream, mx, mb));
  }
  return DMPT_OK;
}

// Square-term store (c->ss, masters): per step, S0 (member 0) and the order-1
// square terms S1 of the d directions and of J (members 1 .. d + 1).
bool ss_fits(const Call& k, int step, int j) {
  return step >= 0 && j >= 0 && j < k.cj + 1 &&
         ((size_t)step * (k.cj + 1) + j + 1) * (size_t)k.nn * k.c->esize <= k.c->ss_bytes;
}

template <class T>
T* ss_ptr(const Call& k, int step, int j) {
  return (T*)k.c->ss + ((size_t)step * (k.cj + 1) + j) * (size_t)k.nn;
}

template <class T>
dmpt_status ss_save(const Call& k, const Group& g, int z, int step, int j) {
  if (!ss_fits(k, step, j) || z >= g.count) return fail(k.c, DMPT_ERR_ARG, "internal: square-term index");
  uint16_t* none[3] = {nullptr, nullptr, nullptr};
  HIPCHK(k.c, (convert<T, T>((const T*)mptr(k, g, z), 0, ss_ptr<T>(k, step, j), 0, k.nn, 1, none, 0, 0,
                             k.c->stream)));
  return DMPT_OK;
}

// Member z of a group (with planes) = stored (step, j) - a * stored (step, jb).
template <class T>
dmpt_status ss_load(const Call& k, const Group& g, int z, int step, int j, double a, int jb) {
  if (!ss_fits(k, step, j) || (a != 0.0 && !ss_fits(k, step, jb)) || z >= g.count)
    return fail(k.c, DMPT_ERR_ARG, "internal: square-term index");
  uint16_t* pl[3];
  planes_of(k, g, z, pl);
  T* dst = (T*)mptr(k, g, z);
  int64_t ms = 0, mb = 0;
  double* mx = ew_sink(k, g, z, &ms, &mb);
  if (a == 0.0) {
    HIPCHK(k.c, (convert<T, T>(ss_ptr<T>(k, step, j), 0, dst, 0, k.nn, 1, pl, 0, g.pl[0] ? k.np : 0,
                               k.c->stream, mx, ms, mb)));
  } else {
    HIPCHK(k.c, axpbyz<T>(ss_ptr<T>(k, step, jb), ss_ptr<T>(k, step, j), dst, k.nn, -a, 1.0, pl,
                          g.pl[0] ? k.np : 0, k.c->stream, mx, mb));
  }
  return DMPT_OK;
}

// Order 0 of one recursion step: T' Y0 = 2 D0 with S0 = D0^2 already formed;
// the previous iterate D0 is the initial guess and D0 is overwritten by the
// symmetrised solution.
template <class T>
dmpt_status solve_order0(const Call& k, int step) {
  dmpt_ctx c = k.c;
  const WS* w = k.w;
  hipStream_t s = c->stream;
  const int hs = c->hstride;
  uint16_t* pl[3] = {nullptr, nullptr, nullptr};
  // ||rhs||^2 = 4 ||D0||^2
  {
    const T* d0 = (const T*)mptr(k, w->D0, 0);
    double* part = k.part;
    double* ref = w->ref;
    EMIT(k, dot_partials<T>(d0, k.stride, d0, k.stride, k.nn, k.m, part, s));
    EMIT(k, sum_partials(part, reduce_blocks(k.nn), k.m, ref, 1, 0, s));
    EMIT(k, axpby<double>(ref, 0, ref, 0, k.m, 1, 0.0, 4.0, pl, 0, 0, s));
  }
  const bool guess_tj = k.traj && c->tj_valid >= 0 && step >= 0;
  if (guess_tj && k.rec) return fail(c, DMPT_ERR_ARG, "internal: recorded passes keep no trajectory");
  if (guess_tj) {
    // U = this step's solution of the previous pass; R = 2 D0 - U - 4 U S0
    STCHK(tj_load<T>(k, c->U0, 0, step, 0));
    G g;
    g.X = op(k, c->U0, 0, false);
    g.Y = op(k, w->S0, 0, false);
    g.C = mptr(k, w->R, 0);
    g.alpha = -4.0;
    g.C1 = mptr(k, w->D0, 0); g.beta1 = 2.0;
    g.C2 = mptr(k, c->U0, 0); g.beta2 = -1.0;
    g.W = mptr(k, w->R, 0);
    STCHK(run_gemm(k, g));
    STCHK(sum_gemm_partials(k, 1, w->rr, hs, 0));
    STCHK(cg_solve<T>(k, c->U0, 1, 1, w->mask0));
    uint16_t* pd[3];
    planes_of(k, w->D0, 0, pd);
    HIPCHK(c, (sym_combine<T, T>((const T*)mptr(k, c->U0, 0), k.Np, 0, k.N, k.Np, 0.5, nullptr, 0,
                                 (T*)mptr(k, w->D0, 0), k.Np, 0, pd, k.np, 1, s)));
  } else if (c->opt.guess == DMPT_GUESS_TAYLOR) {
    // guess U = 2 D0 - 8 D0^3 (the map's Taylor expansion); with Q = D0 S0
    // in P: U replaces D0, and R = 2 D0 - U - 4 U S0 = 8 Q - 4 U S0
    G q;
    q.X = op(k, w->D0, 0, true);
    q.Y = op(k, w->S0, 0, true);
    q.C = mptr(k, w->P, 0);
    q.sC = k.stride;
    q.batch = k.m;
    q.active = w->mask0;
    q.sym = true;  // D0 S0
    STCHK(run_gemm(k, q));
    uint16_t* pd[3];
    planes_of(k, w->D0, 0, pd);
    {
      const T* pp = (const T*)mptr(k, w->P, 0);
      T* d0 = (T*)mptr(k, w->D0, 0);
      EMIT(k, axpby<T>(pp, k.stride, d0, k.stride, k.nn, k.m, -8.0, 2.0, pd, k.stride, k.np, s));
    }
    G g;
    g.X = op(k, w->D0, 0, true);
    g.Y = op(k, w->S0, 0, true);
    g.C = mptr(k, w->R, 0);
    g.sC = k.stride;
    g.alpha = -4.0;
    g.C1 = mptr(k, w->P, 0); g.sC1 = k.stride; g.beta1 = 8.0;
    g.W = mptr(k, w->R, 0); g.sW = k.stride;
    g.batch = k.m;
    g.active = w->mask0;
    STCHK(run_gemm(k, g));
    STCHK(sum_gemm_partials(k, k.m, w->rr, hs, 0));
    STCHK(cg_solve<T>(k, w->D0, k.m, 1, w->mask0));
    STCHK(sym_inplace<T>(k, w->D0, 0, k.m, 0.5));
  } else {
    // R = 2 D0 - D0 - 4 D0 S0 = D0 - 4 D0 S0 (guess: the previous iterate), ||R||^2 -> rr[0]
    G g;
    g.X = op(k, w->D0, 0, true);
    g.Y = op(k, w->S0, 0, true);
    g.C = mptr(k, w->R, 0);
    g.sC = k.stride;
    g.alpha = -4.0;
    g.C1 = mptr(k, w->D0, 0); g.sC1 = k.stride; g.beta1 = 1.0;
    g.W = mptr(k, w->R, 0); g.sW = k.stride;
    g.batch = k.m;
    g.active = w->mask0;
    STCHK(run_gemm(k, g));
    STCHK(sum_gemm_partials(k, k.m, w->rr, hs, 0));
    STCHK(cg_solve<T>(k, w->D0, k.m, 1, w->mask0));
    STCHK(sym_inplace<T>(k, w->D0, 0, k.m, 0.5));
  }
  if (k.traj && step >= 0) STCHK(tj_save<T>(k, w->D0, 0, step, 0));
  return DMPT_OK;
}

// ---------------------------------------------------------------- Newton-Schulz
// Every system of a step has the same matrix T' = I + 4 S0 (Sec. II remark:
// one inverse serves all orders), whose eigenvalues lie in [1, 2].  The
// inverse Z is built from Z0 = (24 I - 8 T') / 17 = (16 I - 32 S0) / 17, the
// linear polynomial in T' with the smallest max |1 - y p(y)| on [1, 2] (it
// equioscillates at y = 1, 3/2, 2 with error 1/17), by
// Z <- Z (2 I - T' Z): the error squares each time, 17^-16 after four
// iterations.  Z is a polynomial in S0, so it commutes with T' and stays
// symmetric; it is re-symmetrised after every iteration.  Single system only.
//
// Early steps need far less: |f(d)| <= 2 |d| for the map f(d) = 2d / (1 + 4d^2),
// so ||D_s|| <= b_s = min(1/2, 2^s ||D_0||), with ||D_0|| <= c max|eps - mu0|
// from the Gershgorin interval of H0.  T' then has its eigenvalues in
// [1, 1 + delta], delta = 4 b_s^2, where the minimax linear start (the
// degree-2 Chebyshev residual on that interval) has error
// e0 = delta^2 / (8 + 8 delta + delta^2) -- 1/17 at delta = 1, ~ delta^2 / 8
// for small delta -- and the iteration count is the smallest k with
// e0^(2^k) <= the products' resolution (ns_target; FP64: 2^-60, four at
// delta = 1, none while ||D_s|| is below ~1e-5).
constexpr int kNsIters = 4;

struct NsStart {
  double a, b;  // Z0 = a I + b S0
  int iters;
};

bool ns_refines(const Call& k);

// Residual bound ||I - T' Z|| at which the iteration of step `step` stops:
// the resolution of the products, divided by the growth of an error from
// this step to the last one (|f'| <= 2 per step), so the inverse's share of
// the final error stays below that resolution, and never below 2^-60 (FP64
// and the forms with a refinement step stop there): 2^-34 for the
// 13-product int8 engine (its dropped digit products leave ~1e-10), 2^-26
// for the 6-product int8 first phase (three base-254 digits resolve 2^-24,
// and that phase only brackets mu0).  The growth factor matters: the
// start's error is the same polynomial for every element and does not
// average out in the traces (2^-44 in every step of the 13-product passes
// moved Tr(H1 P2) at N = 8192 from 6e-7 to 1.1e-6).
double ns_target(const Call& k, int step) {
  if (ns_refines(k) || k.nsteps <= 0 || step < 0 || step >= k.nsteps) return 0x1p-60;
  int res = 0;
  if (k.eng == Engine::I8S4) res = 34;
  else if (k.eng == Engine::I8S3 && k.first_phase) res = 26;
  if (!res) return 0x1p-60;
  return std::max(0x1p-60, std::ldexp(1.0, -res - (k.nsteps - step)));
}

NsStart ns_start(const Call& k, int step) {
  double delta = 1.0;
  if (k.d0b >= 0.0 && step >= 0) {
    const double bs = std::min(0.5, std::ldexp(k.d0b, std::min(step, 1000)) * (1.0 + 1e-3));
    delta = std::min(1.0, 4.0 * bs * bs);
  }
  const double den = 8.0 + 8.0 * delta + delta * delta;
  NsStart z{(8.0 + 8.0 * delta) / den, -32.0 / den, 0};
  const double e0 = delta * delta / den;
  const double target = ns_target(k, step);
  double e = e0;
  while (e > target && z.iters < kNsIters) {
    e = e * e;
    ++z.iters;
  }
  if (k.c->ns_iters_env > 0) z.iters = k.c->ns_iters_env;
  return z;
}

// Whether a solve with Z is followed by one refinement step: with FP32 and
// split-BF16 products Z and R Z carry the products' rounding (1e-7 .. 1e-5),
// and one residual correction recovers it.  FP64 products need none, and
// neither do the 13-product int8 ones: their only error is the dropped digit
// products (~1e-10 relative), the same as in a CG solve with those products
// (at N = 8192 the solve without the step matched or beat the CG form).
bool ns_refines(const Call& k) {
  if (k.c->ns_refine_env >= 0) return k.c->ns_refine_env != 0;
  if (k.first_phase && k.eng == Engine::I8S3) return false;  // its loose tolerance needs no refinement
  return k.eng != Engine::F64 && k.eng != Engine::I8S4;
}

// Whether the steps of a pass solve with the shared inverse: always with
// DMPT_SOLVER_NS; with DMPT_SOLVER_HYBRID when the products are FP64 or
// 13-product int8 (the inverse then needs no refinement step, and with the
// step-fitted start and symmetric products it costs fewer products than CG
// even for the single right-hand side of an order-0 pass; its traces are
// also cleaner: at N = 8192 the int8 occupation error after the Newton step
// fell from 6e-10 to 3e-11).  With FP32 and split-BF16 products the passes
// keep CG: the inverse's own rounding biases the traces of the jets
// (Tr(H1 P2) 1.8e-6 with BF16X6 at N = 8192, against 5e-7 with CG).
bool ns_pass(const Call& k, int order) {
  (void)order;
  const dmpt_solver sv = k.c->opt.solver;
  const bool hybrid_ns = sv == DMPT_SOLVER_HYBRID && (k.eng == Engine::F64 || k.eng == Engine::I8S4 ||
                                                      (k.eng == Engine::I8S3 && k.first_phase));
  return (sv == DMPT_SOLVER_NS || hybrid_ns) && k.m == 1 && !k.graph;
}

// Whether a product marked symmetric computes only the lower triangle of
// tiles (the tile count per side is even; DMPT_FULL_TILES unset; not recorded):
// then its output is exactly symmetric.
bool sym_tiles(const Call& k) {
  const int edge = gemm_tile_edge(k.eng, k.Np, variant_for(k.c, k.eng, k.Np), acc64_of(k.c, k.eng));
  return !k.rec && !k.c->full_tiles && (k.Np / edge) % 2 == 0;
}

// Steps of the iteration from a stored inverse Z_old of T'_old (a pass at
// mu0 - dmu): the perturbation enters D_0 = c (H - mu0 I) as c dmu I, which
// commutes with H, so ||D_s - D_s,old|| <= min(2^s c |dmu|, 2 b_s) (|f'| <= 2)
// and ||I - T' Z_old|| <= 4 ||D_s^2 - D_s,old^2|| <= 8 b_s ||D_s - D_s,old||,
// floored at the stored inverse's own rounding (1e-10).  Returns the step
// count to ns_target when it is below the count from the minimax start, else -1.
int ns_warm_iters(const Call& k, int step, int scratch) {
  if (!(k.z_dmu >= 0.0) || k.d0b < 0.0 || !(k.cscale > 0.0) || step < 0 || k.c->ns_iters_env > 0) return -1;
  const double bs = std::min(0.5, std::ldexp(k.d0b, std::min(step, 1000)) * (1.0 + 1e-3));
  const double dd = std::min(2.0 * bs, std::ldexp(k.cscale * k.z_dmu, std::min(step, 1000)) * (1.0 + 1e-3));
  double e = std::max(8.0 * bs * dd, 1e-10);
  if (!(e < 1.0)) return -1;
  const double target = ns_target(k, step);
  int it = 0;
  do {
    e = e * e;
    ++it;
  } while (e > target && it < kNsIters);
  return e <= target && it < scratch ? it : -1;
}

template <class T>
dmpt_status ns_iterate(const Call& k, int iters);
template <class T>
dmpt_status zs_load(const Call& k, int step);

template <class T>
dmpt_status ns_inverse(const Call& k, int step) {
  dmpt_ctx c = k.c;
  const WS* w = k.w;
  hipStream_t s = c->stream;
  if (k.m != 1) return fail(c, DMPT_ERR_ARG, "internal: Newton-Schulz runs on one system");
  const NsStart z0 = ns_start(k, step);
  if (k.chain & kWarmZ) {
    const int wi = ns_warm_iters(k, step, z0.iters);
    if (wi > 0) {
      STCHK(zs_load<T>(k, step));  // Z_old into member 0
      return ns_iterate<T>(k, wi);
    }
  }
  uint16_t* pz[3];
  planes_of(k, w->Zi, 0, pz);
  int64_t ms = 0, mb = 0;
  double* mx = ew_sink(k, w->Zi, 0, &ms, &mb);
  HIPCHK(c, scaled_plus_identity<T>((const T*)mptr(k, w->S0, 0), (T*)mptr(k, w->Zi, 0), k.N, k.Np, z0.a,
                                    z0.b, pz, k.np, s, mx, mb));
  return ns_iterate<T>(k, z0.iters);
}

// Newton-Schulz steps Z <- Z (2 I - T' Z) from the start in member 0 of Zi.
template <class T>
dmpt_status ns_iterate(const Call& k, int iters) {
  dmpt_ctx c = k.c;
  const WS* w = k.w;
  hipStream_t s = c->stream;
  int cur = 0;
  const bool exact = sym_tiles(k);  // symmetric products leave Z exactly symmetric
  for (int it = 0; it < iters; ++it) {
    const int nxt = 1 - cur;
    G g;  // M = T' Z = Z + 4 S0 Z  -> P[0] (with planes)
    g.X = op(k, w->S0, 0, false);
    g.Y = op(k, w->Zi, cur, false);
    g.C = mptr(k, w->P, 0);
    planes_of(k, w->P, 0, g.Cpl);
    g.alpha = 4.0;
    g.C1 = mptr(k, w->Zi, cur); g.beta1 = 1.0;
    g.sym = true;  // S0 and Z commute (Z is a polynomial in S0)
    STCHK(run_gemm(k, g));
    G h;  // Z' = 2 Z - Z M: straight into the other member, or via R[0] and a symmetrisation
    h.X = op(k, w->Zi, cur, false);
    h.Y = op(k, w->P, 0, false);
    h.C = exact ? mptr(k, w->Zi, nxt) : mptr(k, w->R, 0);
    if (exact) planes_of(k, w->Zi, nxt, h.Cpl, 1);  // Zi[cur], this product's X, keeps its slices
    h.alpha = -1.0;
    h.C1 = mptr(k, w->Zi, cur); h.beta1 = 2.0;
    h.sym = true;
    STCHK(run_gemm(k, h));
    if (!exact) {
      uint16_t* pn[3];
      planes_of(k, w->Zi, nxt, pn);
      HIPCHK(c, (sym_combine<T, T>((const T*)mptr(k, w->R, 0), k.Np, 0, k.N, k.Np, 0.5, nullptr, 0,
                                   (T*)mptr(k, w->Zi, nxt), k.Np, 0, pn, k.np, 1, s)));
    }
    cur = nxt;
  }
  c->zcur = cur;
  return DMPT_OK;
}

// Solve with the shared inverse: the unknowns U (transposed solutions) of the
// md members of group g from the right-hand sides rhs^T held in R:
// U = R Z; with products below FP64 one refinement U += (R - U T') Z follows.
template <class T>
dmpt_status ns_solve(const Call& k, const Group& g, int md) {
  const WS* w = k.w;
  if (k.np > 0) {
    // the products that formed R wrote its master only
    uint16_t* pr[3];
    planes_of(k, w->R, 0, pr);
    HIPCHK(k.c, split_planes((const double*)mptr(k, w->R, 0), k.nn, k.stride, pr, k.stride, k.np, md,
                             k.c->stream));
  }
  const int zc = k.c->zcur;
  G a;
  a.X = op(k, w->R, 0, true);
  a.Y = op(k, w->Zi, zc, true);
  a.Y.div = md;
  a.C = mptr(k, g, 0);
  a.sC = k.stride;
  planes_of(k, g, 0, a.Cpl);
  a.batch = md;
  a.sym = &g == &w->D0;  // order 0: R = 2 D0 commutes with Z
  STCHK(run_gemm(k, a));
  // an order-0 solution from symmetric tiles is symmetric already
  if (a.sym && sym_tiles(k) && !ns_refines(k)) return DMPT_OK;
  if (ns_refines(k)) {
    G r;  // R -= U + 4 U S0
    r.X = op(k, g, 0, true);
    r.Y = op(k, w->S0, 0, true);
    r.Y.div = md;
    r.C = mptr(k, w->R, 0);
    r.sC = k.stride;
    planes_of(k, w->R, 0, r.Cpl);
    r.alpha = -4.0;
    r.C1 = mptr(k, w->R, 0); r.sC1 = k.stride; r.beta1 = 1.0;
    r.C2 = mptr(k, g, 0); r.sC2 = k.stride; r.beta2 = -1.0;
    r.batch = md;
    STCHK(run_gemm(k, r));
    G u;  // U += R Z
    u.X = op(k, w->R, 0, true);
    u.Y = op(k, w->Zi, zc, true);
    u.Y.div = md;
    u.C = mptr(k, g, 0);
    u.sC = k.stride;
    planes_of(k, g, 0, u.Cpl);
    u.C1 = mptr(k, g, 0); u.sC1 = k.stride; u.beta1 = 1.0;
    u.batch = md;
    STCHK(run_gemm(k, u));
  }
  return sym_inplace<T>(k, g, 0, md, 0.5);
}

// Finish the solve of one jet order: R holds rhs^T (its norm in ref); with
// the guess U in group g (the previous iterate or a stored one) form the
// initial residual R -= U + 4 U S0, run CG and symmetrise the solution.
template <class T>
dmpt_status solve_jet(const Call& k, const Group& g, int md, int d) {
  const WS* w = k.w;
  G h;
  h.X = op(k, g, 0, true);
  h.Y = op(k, w->S0, 0, true);
  h.Y.div = d;
  h.C = mptr(k, w->R, 0);
  h.sC = k.stride;
  h.alpha = -4.0;
  h.C1 = mptr(k, w->R, 0); h.sC1 = k.stride; h.beta1 = 1.0;
  h.C2 = mptr(k, g, 0); h.sC2 = k.stride; h.beta2 = -1.0;
  h.W = mptr(k, w->R, 0); h.sW = k.stride;
  h.batch = md;
  h.active = w->mask1;
  STCHK(run_gemm(k, h));
  STCHK(sum_gemm_partials(k, md, w->rr, k.c->hstride, 0));
  STCHK(cg_solve<T>(k, g, md, d, w->mask1));
  STCHK(sym_inplace<T>(k, g, 0, md, 0.5));
  return DMPT_OK;
}

// Inverse store (c->zs, masters): per step the shared inverse Z of T'.
bool zs_fits(const Call& k, int step) {
  return step >= 0 && ((size_t)step + 1) * (size_t)k.nn * k.c->esize <= k.c->zs_bytes;
}

template <class T>
dmpt_status zs_save(const Call& k, int step) {
  if (!zs_fits(k, step)) return fail(k.c, DMPT_ERR_ARG, "internal: inverse-store index");
  uint16_t* none[3] = {nullptr, nullptr, nullptr};
  HIPCHK(k.c, (convert<T, T>((const T*)mptr(k, k.w->Zi, k.c->zcur), 0, (T*)k.c->zs + (size_t)step * k.nn, 0, k.nn,
                             1, none, 0, 0, k.c->stream)));
  return DMPT_OK;
}

template <class T>
dmpt_status zs_load(const Call& k, int step) {
  if (!zs_fits(k, step)) return fail(k.c, DMPT_ERR_ARG, "internal: inverse-store index");
  uint16_t* pl[3];
  planes_of(k, k.w->Zi, 0, pl);
  int64_t ms = 0, mb = 0;
  double* mx = ew_sink(k, k.w->Zi, 0, &ms, &mb);
  HIPCHK(k.c, (convert<T, T>((const T*)k.c->zs + (size_t)step * k.nn, 0, (T*)mptr(k, k.w->Zi, 0), 0, k.nn,
                             1, pl, 0, k.w->Zi.pl[0] ? k.np : 0, k.c->stream, mx, ms, mb)));
  k.c->zcur = 0;
  return DMPT_OK;
}

// One recursion step for orders 0..order, d directions per system, on the
// iterates held in k.w (Algorithm 1's inner loop body, in D form).
template <class T>
dmpt_status recursion_step(const Call& k, int order, int d, int step) {
  dmpt_ctx c = k.c;
  const WS* w = k.w;
  const int md = k.m * d;
  const bool ns = ns_pass(k, order);
  // S0 serves only the solves (T' in CG, the inverse's iteration and its
  // refinement): a pass that loads the order-0/1 chains and the inverse and
  // refines nothing does not read it
  const bool s0_unread = ns && (k.chain & kLoad01) && (k.chain & kLoadZ) && !ns_refines(k);
  if (k.chain & kLoadS) {
    if (!s0_unread) STCHK(ss_load<T>(k, w->S0, 0, step, 0, 0.0, 0));
  } else {
    STCHK(square0<T>(k));
  }
  // the pass that loads these chains then does not read S0 either
  const bool s0_unread_later = ns && (k.chain & kSave01) && (k.chain & kSaveZ) && !ns_refines(k);
  if ((k.chain & kSaveS) && !s0_unread_later) STCHK(ss_save<T>(k, w->S0, 0, step, 0));
  // the identity direction of an order-1 pass solved with the shared inverse:
  // with S1_J = 2 D0 D1_J, Y0 = 2 D0 Z and 4 S0 Z = I - Z, the order-1 step
  // (2 D1_J - 4 Y0 S1_J) Z is D1_J (4 Z^2 - 2 Z), two symmetric products
  // (used where Z is as accurate as the products: no refinement step)
  const bool jt = ns && !ns_refines(k) && order == 1 && k.m == 1 && k.jdir >= 0 && k.jdir == k.m * d - 1 &&
                  !(k.chain & kLoad01) && !(k.chain & kLoadS);
  if (ns) {
    if (k.chain & kLoadZ) STCHK(zs_load<T>(k, step));
    else STCHK(ns_inverse<T>(k, step));
    if (k.chain & kSaveZ) STCHK(zs_save<T>(k, step));
  }
  if (order >= 1 && (k.chain & kLoadS)) {
    // the order-1 pass stored S1 at mu1 = 0; S1 is linear in mu1: S1 = S1(0) - mu1 S1_J
    for (int z = 0; z < md; ++z) STCHK(ss_load<T>(k, w->S1, z, step, 1 + z, k.cmu[z], k.cj));
  } else if (order >= 1) {
    // Q = D1 D0 -> S1 = Q + Q^T (for J, a polynomial in D0 that commutes
    // with it, Q is symmetric: S1_J = 2 D1_J D0)
    const int mr = jt ? md - 1 : md;
    if (mr > 0) {
      G g;
      g.X = op(k, w->D1, 0, true);
      g.Y = op(k, w->D0, 0, true);
      g.Y.div = d;
      g.C = mptr(k, w->Q, 0);
      g.sC = k.stride;
      g.batch = mr;
      g.active = w->mask1;
      STCHK(run_gemm(k, g));
    }
    if (jt) {
      G g;
      g.X = op(k, w->D1, mr, false);
      g.Y = op(k, w->D0, 0, false);
      g.C = mptr(k, w->Q, mr);
      g.active = w->mask1 ? w->mask1 + mr : nullptr;
      g.sym = true;
      STCHK(run_gemm(k, g));
    }
    STCHK(sym_to<T>(k, w->Q, w->S1, md, true));
    if (k.chain & kSaveS)
      for (int z = 0; z < md; ++z) STCHK(ss_save<T>(k, w->S1, z, step, 1 + z));
  }
  if (order >= 2) {
    // Q = D2 D0 -> S2 = Q + Q^T; S2 += D1 D1
    G g;
    g.X = op(k, w->D2, 0, true);
    g.Y = op(k, w->D0, 0, true);
    g.Y.div = d;
    g.C = mptr(k, w->Q, 0);
    g.sC = k.stride;
    g.batch = md;
    g.active = w->mask1;
    STCHK(run_gemm(k, g));
    STCHK(sym_to<T>(k, w->Q, w->S2, md, false));
    G h;
    h.X = op(k, w->D1, 0, true);
    h.Y = op(k, w->D1, 0, true);
    h.C = mptr(k, w->S2, 0);
    h.sC = k.stride;
    planes_of(k, w->S2, 0, h.Cpl);
    h.C1 = mptr(k, w->S2, 0); h.sC1 = k.stride; h.beta1 = 1.0;
    h.batch = md;
    h.active = w->mask1;
    h.sym = true;  // D1 D1, added to the symmetric D2 D0 + D0 D2
    STCHK(run_gemm(k, h));
  }
  if (order >= 3) {
    // Q = D3 D0, R = D2 D1 -> S3 = Q + Q^T + R + R^T
    G g;
    g.X = op(k, w->D3, 0, true);
    g.Y = op(k, w->D0, 0, true);
    g.Y.div = d;
    g.C = mptr(k, w->Q, 0);
    g.sC = k.stride;
    g.batch = md;
    g.active = w->mask1;
    STCHK(run_gemm(k, g));
    G h;
    h.X = op(k, w->D2, 0, true);
    h.Y = op(k, w->D1, 0, true);
    h.C = mptr(k, w->R, 0);
    h.sC = k.stride;
    h.batch = md;
    h.active = w->mask1;
    STCHK(run_gemm(k, h));
    if (md > w->Q.count || md > w->R.count || md > w->S3.count)
      return fail(c, DMPT_ERR_ARG, "internal: sym batch too large");
    uint16_t* pl[3];
    planes_of(k, w->S3, 0, pl);
    HIPCHK(c, (sym_combine<T, T>((const T*)mptr(k, w->Q, 0), k.Np, k.stride, k.N, k.Np, 1.0, nullptr, 0,
                                 (T*)mptr(k, w->S3, 0), k.Np, k.stride, pl, k.np, md, c->stream,
                                 (const T*)mptr(k, w->R, 0), 1.0)));
  }
  // ---- order 0
  if (k.chain & kLoad01) {
    // the order-0 chain of this mu0 is stored: Y0 = its solution at this step
    STCHK(st_load<T>(k, w->D0, 0, step, 0, 0.0, 0));
  } else {
    if (ns && engine_int8(k.eng) && !ns_refines(k)) {
      // D0 = 2 D0 Z in place: the int8 product reads D0's slices (made before
      // it starts), never its master, and 2 D0 commutes with Z
      G a;
      a.X = op(k, w->D0, 0, false);
      a.Y = op(k, w->Zi, c->zcur, false);
      a.C = mptr(k, w->D0, 0);
      a.alpha = 2.0;
      a.sym = true;
      STCHK(run_gemm(k, a));
      if (!sym_tiles(k)) STCHK(sym_inplace<T>(k, w->D0, 0, 1, 0.5));
    } else if (ns) {
      // R = 2 D0 (with planes), D0 = R Z
      uint16_t* pr[3];
      planes_of(k, w->R, 0, pr);
      HIPCHK(c, axpby<T>((const T*)mptr(k, w->D0, 0), 0, (T*)mptr(k, w->R, 0), 0, k.nn, 1, 2.0, 0.0,
                         pr, 0, k.np, c->stream));
      STCHK(ns_solve<T>(k, w->D0, 1));
    } else {
      STCHK(solve_order0<T>(k, step));
    }
    if (k.chain & kSave01) STCHK(st_save<T>(k, w->D0, 0, step, 0));
  }
  // ---- order 1: T' Y1 = 2 D1 - 4 S1 Y0; transposed: rhs^T = 2 D1 - 4 Y0 S1
  if (order >= 1 && (k.chain & kLoad01)) {
    // the order-1 solutions are linear in mu1: Y1 = Y1(mu1 = 0) - mu1 Y_J
    for (int z = 0; z < md; ++z) STCHK(st_load<T>(k, w->D1, z, step, 1 + z, k.cmu[z], k.cj));
  } else if (order >= 1) {
    const int mr = jt ? md - 1 : md;
    if (mr > 0) {
      G g;  // R = 2 D1 - 4 Y0 S1   (Y0 = new D0), ||rhs||^2 -> ref
      g.X = op(k, w->D0, 0, true);
      g.X.div = d;
      g.Y = op(k, w->S1, 0, true);
      g.C = mptr(k, w->R, 0);
      g.sC = k.stride;
      g.alpha = -4.0;
      g.C1 = mptr(k, w->D1, 0); g.sC1 = k.stride; g.beta1 = 2.0;
      g.W = mptr(k, w->R, 0); g.sW = k.stride;
      g.batch = mr;
      g.active = w->mask1;
      STCHK(run_gemm(k, g));
      STCHK(sum_gemm_partials(k, mr, w->ref, 1, 0));
    }
    if (jt) {
      if (mr > 0) STCHK(ns_solve<T>(k, w->D1, mr));
      G m;  // M = 4 Z Z - 2 Z -> P[J]
      const int zc = c->zcur;
      m.X = op(k, w->Zi, zc, false);
      m.Y = op(k, w->Zi, zc, false);
      m.C = mptr(k, w->P, mr);
      planes_of(k, w->P, mr, m.Cpl);
      m.alpha = 4.0;
      m.C1 = mptr(k, w->Zi, zc); m.beta1 = -2.0;
      m.sym = true;
      STCHK(run_gemm(k, m));
      // D1_J = D1_J M: in place with int8 products (they read D1_J's slices,
      // not its master), else through R[J]
      const bool inplace = engine_int8(k.eng);
      G u;
      u.X = op(k, w->D1, mr, false);
      u.Y = op(k, w->P, mr, false);
      u.C = mptr(k, inplace ? w->D1 : w->R, mr);
      u.sym = true;
      STCHK(run_gemm(k, u));
      if (!inplace) {
        uint16_t* pj[3];
        planes_of(k, w->D1, mr, pj);
        HIPCHK(c, (convert<T, T>((const T*)mptr(k, w->R, mr), 0, (T*)mptr(k, w->D1, mr), 0, k.nn, 1, pj, 0,
                                 w->D1.pl[0] ? k.np : 0, c->stream)));
      }
    } else if (ns) {
      STCHK(ns_solve<T>(k, w->D1, md));
    } else {
      if (k.traj && c->tj_valid >= 1)  // guess: this step's solution of the previous pass
        for (int z = 0; z < md; ++z) STCHK(tj_load<T>(k, w->D1, z, step, 1 + z));
      STCHK(solve_jet<T>(k, w->D1, md, d));
    }
    if (k.traj && !ns)  // CG guesses only
      for (int z = 0; z < md; ++z) STCHK(tj_save<T>(k, w->D1, z, step, 1 + z));
    if (k.chain & kSave01)
      for (int z = 0; z < md; ++z) STCHK(st_save<T>(k, w->D1, z, step, 1 + z));
  }
  // ---- order 2: rhs^T = 2 D2 - 4 Y1 S1 - 4 Y0 S2
  if (order >= 2 && (k.chain & kLoad2)) {
    for (int z = 0; z < md; ++z)
      STCHK(st_load<T>(k, w->D2, z, step, 2 + d + z, k.cmu[d + z], k.cj));
  } else if (order >= 2) {
    G g;  // R = 2 D2 - 4 Y0 S2
    g.X = op(k, w->D0, 0, true);
    g.X.div = d;
    g.Y = op(k, w->S2, 0, true);
    g.C = mptr(k, w->R, 0);
    g.sC = k.stride;
    g.alpha = -4.0;
    g.C1 = mptr(k, w->D2, 0); g.sC1 = k.stride; g.beta1 = 2.0;
    g.batch = md;
    g.active = w->mask1;
    STCHK(run_gemm(k, g));
    G g2;  // R -= 4 Y1 S1, ||rhs||^2 -> ref
    g2.X = op(k, w->D1, 0, true);
    g2.Y = op(k, w->S1, 0, true);
    g2.C = mptr(k, w->R, 0);
    g2.sC = k.stride;
    g2.alpha = -4.0;
    g2.C1 = mptr(k, w->R, 0); g2.sC1 = k.stride; g2.beta1 = 1.0;
    g2.W = mptr(k, w->R, 0); g2.sW = k.stride;
    g2.batch = md;
    g2.active = w->mask1;
    STCHK(run_gemm(k, g2));
    STCHK(sum_gemm_partials(k, md, w->ref, 1, 0));
    if (ns) {
      STCHK(ns_solve<T>(k, w->D2, md));
    } else {
      if (k.traj && c->tj_valid >= 2)
        for (int z = 0; z < md; ++z) STCHK(tj_load<T>(k, w->D2, z, step, 1 + d + z));
      STCHK(solve_jet<T>(k, w->D2, md, d));
    }
    if (k.traj && !ns)  // CG guesses only
      for (int z = 0; z < md; ++z) STCHK(tj_save<T>(k, w->D2, z, step, 1 + d + z));
    if (k.chain & kSave2)
      for (int z = 0; z < md; ++z) STCHK(st_save<T>(k, w->D2, z, step, 2 + d + z));
  }
  // ---- order 3: rhs^T = 2 D3 - 4 Y0 S3 - 4 Y1 S2 - 4 Y2 S1
  if (order >= 3) {
    G g;  // R = 2 D3 - 4 Y0 S3
    g.X = op(k, w->D0, 0, true);
    g.X.div = d;
    g.Y = op(k, w->S3, 0, true);
    g.C = mptr(k, w->R, 0);
    g.sC = k.stride;
    g.alpha = -4.0;
    g.C1 = mptr(k, w->D3, 0); g.sC1 = k.stride; g.beta1 = 2.0;
    g.batch = md;
    g.active = w->mask1;
    STCHK(run_gemm(k, g));
    G g2;  // R -= 4 Y1 S2
    g2.X = op(k, w->D1, 0, true);
    g2.Y = op(k, w->S2, 0, true);
    g2.C = mptr(k, w->R, 0);
    g2.sC = k.stride;
    g2.alpha = -4.0;
    g2.C1 = mptr(k, w->R, 0); g2.sC1 = k.stride; g2.beta1 = 1.0;
    g2.batch = md;
    g2.active = w->mask1;
    STCHK(run_gemm(k, g2));
    G g3;  // R -= 4 Y2 S1, ||rhs||^2 -> ref
    g3.X = op(k, w->D2, 0, true);
    g3.Y = op(k, w->S1, 0, true);
    g3.C = mptr(k, w->R, 0);
    g3.sC = k.stride;
    g3.alpha = -4.0;
    g3.C1 = mptr(k, w->R, 0); g3.sC1 = k.stride; g3.beta1 = 1.0;
    g3.W = mptr(k, w->R, 0); g3.sW = k.stride;
    g3.batch = md;
    g3.active = w->mask1;
    STCHK(run_gemm(k, g3));
    STCHK(sum_gemm_partials(k, md, w->ref, 1, 0));
    if (ns) {
      STCHK(ns_solve<T>(k, w->D3, md));
    } else {
      if (k.traj && c->tj_valid >= 3)
        for (int z = 0; z < md; ++z) STCHK(tj_load<T>(k, w->D3, z, step, 1 + 2 * d + z));
      STCHK(solve_jet<T>(k, w->D3, md, d));
    }
    if (k.traj && !ns)  // CG guesses only
      for (int z = 0; z < md; ++z) STCHK(tj_save<T>(k, w->D3, z, step, 1 + 2 * d + z));
  }
  return DMPT_OK;
}

// DMPT_DEBUG_CHECKS, after recursion step `step`: S0 and the iterates of every
// order finite, and the iterates exactly symmetric (each is symmetrised after
// its solve).  The message names the step, the matrix and the member.
dmpt_status debug_step(const Call& k, int order, int d, int step) {
  dmpt_ctx c = k.c;
  if (!c->debug || k.rec) return DMPT_OK;
  hipStream_t s = c->stream;
  const WS* w = k.w;
  const int md = k.m * d;
  struct Item {
    const Group* g;
    int count;
    const char* name;
    bool sym;
  };
  const Item items[] = {{&w->D0, k.m, "D0", true},
                        {&w->S0, k.m, "S0", false},
                        {&w->D1, order >= 1 ? md : 0, "D1", true},
                        {&w->D2, order >= 2 ? md : 0, "D2", true},
                        {&w->D3, order >= 3 ? md : 0, "D3", true}};
  const int nb = reduce_blocks(k.Np * k.Np);
  std::vector<double> hm((size_t)nb);
  for (const Item& it : items)
    for (int z = 0; z < it.count; ++z) {
      const double* x = (const double*)mptr(k, *it.g, z);
      HIPCHK(c, set_values(c->d_flag + 1, 0, 1, nullptr, 0.0, 0, s));
      HIPCHK(c, nonfinite_scan(x, k.Np, k.Np, c->d_flag + 1, s));
      HIPCHK(c, hipMemcpyAsync(c->h_int, c->d_flag + 1, sizeof(int), hipMemcpyDeviceToHost, s));
      double asym = 0.0;
      if (it.sym) {
        HIPCHK(c, asym_max(x, k.Np, c->d_dbg, s));
        HIPCHK(c, hipMemcpyAsync(hm.data(), c->d_dbg, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
      }
      HIPCHK(c, hipStreamSynchronize(s));
      if (it.sym)
        for (double v : hm) asym = std::max(asym, v);
      if (c->h_int[0] || asym > 0.0) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "debug check after recursion step %d: %s member %d is %s", step, it.name, z,
                      c->h_int[0] ? "not finite" : "not symmetric");
        return fail(c, c->h_int[0] ? DMPT_ERR_NONFINITE : DMPT_ERR_ARG, msg);
      }
    }
  return DMPT_OK;
}

// One full pass of the recursion for orders 0..order (single system).
template <class T>
dmpt_status recursion_pass(const Call& k0, const PassIn& in) {
  const double cscale = std::ldexp(in.beta, -(in.n + 2));
  Call k = k0;
  k.cscale = cscale;
  k.nsteps = in.n;
  if (std::isfinite(k0.glo) && std::isfinite(k0.ghi) && in.mu)
    k.d0b = cscale * std::max(std::fabs(k0.glo - in.mu[0]), std::fabs(k0.ghi - in.mu[0]));
  STCHK(init_d<T>(k, in, cscale));
  for (int step = 0; step < in.n; ++step) {
    Range r("dmpt recursion step %d", step);
    STCHK(recursion_step<T>(k, in.order, in.d, step));
    STCHK(debug_step(k, in.order, in.d, step));
  }
  // passes with the shared inverse keep no trajectory (only CG reads it)
  if (k.traj) k.c->tj_valid = ns_pass(k, in.order) ? -1 : in.order;
  return DMPT_OK;
}

// Outputs and traces of a pass: P0 = I/2 - D0, P^(k) = -D^(k) (FP64,
// caller buffers), Tr P^(k), sum |P^(k)_ii| and ||P0||_F^2; then one
// synchronisation and the values land in c->h_res.
template <class T>
dmpt_status finish_pass(const Call& k, const PassIn& in, double* P0, double* const* P1,
                        double* const* P2, double* const* P3) {
  dmpt_ctx c = k.c;
  hipStream_t s = c->stream;
  double* shift = c->d_res + RES_HALF;  // device constant 1/2 for the P0 diagonal
  HIPCHK(c, (sym_combine<T, double>((const T*)mptr(k, c->ws.D0, 0), k.Np, 0, k.N, k.Np, -0.5, shift, 0,
                                    P0, k.N, 0, nullptr, 0, 1, s)));
  HIPCHK(c, trace(P0, k.N, 0, k.N, 1, c->d_res + RES_TR, 1, c->d_res + RES_ATR, s));
  HIPCHK(c, dot_partials<double>(P0, 0, P0, 0, k.N * k.N, 1, c->d_part, s));
  HIPCHK(c, sum_partials(c->d_part, reduce_blocks(k.N * k.N), 1, c->d_res + RES_FRO, 1, 0, s));
  const int d = in.d;
  for (int ord = 1; ord <= in.order; ++ord) {
    const Group& g = jet(&c->ws, ord);
    double* const* Pk = ord == 1 ? P1 : (ord == 2 ? P2 : P3);
    for (int z = 0; z < d; ++z) {
      const int slot = slot_of(ord, z, d);
      HIPCHK(c, (sym_combine<T, double>((const T*)mptr(k, g, z), k.Np, 0, k.N, k.Np, -0.5, nullptr,
                                        0, Pk[z], k.N, 0, nullptr, 0, 1, s)));
      HIPCHK(c, trace(Pk[z], k.N, 0, k.N, 1, c->d_res + RES_TR + slot, 1,
                      c->d_res + RES_ATR + slot, s));
    }
  }
  HIPCHK(c, hipMemcpyAsync(c->h_res, c->d_res, RES_MISC * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return DMPT_OK;
}

// Response traces Tr[H^(k) P^(j)] of the returned matrices (Sec. III, Eq.
// Resp_0) for k = 1..order, j = 0..order, k + j <= order + 1, every
// direction: <sym H^(k), P^(j)> = <H^(k), P^(j)> since P^(j) is symmetric; an
// absent H2 / H3 gives 0.  Lands in c->h_res after one synchronisation.
dmpt_status response_traces(dmpt_ctx c, int64_t N, const PassIn& in, const double* P0,
                            double* const* P1, double* const* P2, double* const* P3) {
  hipStream_t s = c->stream;
  const int64_t nn = N * N;
  for (int kk = 1; kk <= in.order; ++kk)
    for (int z = 0; z < in.d; ++z) {
      const double* h = kk == 1 ? in.H1[z]
                                : (kk == 2 ? (in.H2 ? in.H2[z] : nullptr) : (in.H3 ? in.H3[z] : nullptr));
      for (int j = 0; j <= in.order && kk + j <= in.order + 1; ++j) {
        double* out = c->d_res + res_hp(kk, j, z);
        const double* P = j == 0 ? P0 : (j == 1 ? P1[z] : (j == 2 ? P2[z] : P3[z]));
        if (!h) {
          HIPCHK(c, set_values(nullptr, 0, 0, out, 0.0, 1, s));
          continue;
        }
        HIPCHK(c, dot_partials<double>(h, 0, P, 0, nn, 1, c->d_part, s));
        HIPCHK(c, sum_partials(c->d_part, reduce_blocks(nn), 1, out, 1, 0, s));
      }
    }
  HIPCHK(c, hipMemcpyAsync(c->h_res + RES_HP, c->d_res + RES_HP, 12 * DMPT_MAX_DIRS * sizeof(double),
                           hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return DMPT_OK;
}

dmpt_status check_common(dmpt_ctx c, int64_t N, const double* H0, double beta, int n) {
  if (!c) return DMPT_ERR_ARG;
  if (N < 1) return fail(c, DMPT_ERR_ARG, "N must be >= 1");
  if (N > c->n_max) return fail(c, DMPT_ERR_NOMEM, "N exceeds the context's n_max");
  if (!H0) return fail(c, DMPT_ERR_ARG, "H0 is NULL");
  if (!(beta > 0.0) || !std::isfinite(beta)) return fail(c, DMPT_ERR_ARG, "beta must be finite and > 0");
  if (n < 1 || n > 62) return fail(c, DMPT_ERR_ARG, "recursion depth n must lie in [1, 62]");
  return DMPT_OK;
}

dmpt_status check_dirs(dmpt_ctx c, int d, int order, const double* const* H1, const double* const* P1v,
                       const double* const* P2v, const double* const* P3v) {
  if (order < 0 || order > 3) return fail(c, DMPT_ERR_ARG, "order must be 0, 1, 2 or 3");
  if (order == 0) return DMPT_OK;
  if (d < 1 || d > c->dirs_max || d > DMPT_MAX_DIRS)
    return fail(c, DMPT_ERR_ARG, "d must lie in [1, dirs_max]");
  if (!H1) return fail(c, DMPT_ERR_ARG, "H1 is NULL");
  for (int i = 0; i < d; ++i)
    if (!H1[i]) return fail(c, DMPT_ERR_ARG, "H1[i] is NULL");
  if (!P1v) return fail(c, DMPT_ERR_ARG, "P1 is NULL");
  for (int i = 0; i < d; ++i)
    if (!P1v[i]) return fail(c, DMPT_ERR_ARG, "P1[i] is NULL");
  if (order >= 2) {
    if (!P2v) return fail(c, DMPT_ERR_ARG, "P2 is NULL");
    for (int i = 0; i < d; ++i)
      if (!P2v[i]) return fail(c, DMPT_ERR_ARG, "P2[i] is NULL");
  }
  if (order >= 3) {
    if (!P3v) return fail(c, DMPT_ERR_ARG, "P3 is NULL");
    for (int i = 0; i < d; ++i)
      if (!P3v[i]) return fail(c, DMPT_ERR_ARG, "P3[i] is NULL");
  }
  return DMPT_OK;
}

// Non-finite scan of the inputs and the Gershgorin interval of sym(H0).
// gscratch: 2 + 2 N doubles for the Gershgorin row bounds (null: the
// context's, which holds n_max rows).
dmpt_status scan_inputs(dmpt_ctx c, int64_t N, const PassIn& in, double* glo, double* ghi,
                        double* gscratch = nullptr) {
  hipStream_t s = c->stream;
  double* gs = gscratch ? gscratch : c->d_gersh;
  if (!gscratch && N > c->n_max)
    return fail(c, DMPT_ERR_ARG, "internal: the context's Gershgorin scratch holds n_max rows");
  HIPCHK(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), s));
  HIPCHK(c, nonfinite_scan(in.H0, N, N, c->d_flag, s));
  for (int o = 1; o <= in.order; ++o)
    for (int z = 0; z < in.d; ++z) {
      const double* h = o == 1 ? in.H1[z]
                               : (o == 2 ? (in.H2 ? in.H2[z] : nullptr) : (in.H3 ? in.H3[z] : nullptr));
      if (h) HIPCHK(c, nonfinite_scan(h, N, N, c->d_flag, s));
    }
  HIPCHK(c, gershgorin(in.H0, N, gs, s));
  double g[2];
  HIPCHK(c, hipMemcpyAsync(g, gs, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(c->h_int, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (c->h_int[0]) return fail(c, DMPT_ERR_NONFINITE, "non-finite value in an input matrix");
  *glo = g[0];
  *ghi = g[1];
  return DMPT_OK;
}

// The engine of a single pass: BF16X3 with refinement runs a one-off pass
// (no Newton loop) directly in the refinement engine.
Call make_call(dmpt_ctx c, int64_t N, bool refined) {
  Call k;
  k.c = c;
  k.w = &c->ws;
  k.eng = engine_of(c->opt.prec);
  if (refined && refinable(c->opt.prec) && c->opt.refine) k.eng = refine_engine(c->opt);
  k.np = engine_planes(k.eng);
  k.N = N;
  k.Np = padded(N);
  k.nn = k.Np * k.Np;
  k.stride = c->np_max * c->np_max;
  k.tol_cg = c->opt.tol_cg;
  k.part = c->d_part;
  k.part_count = c->part_count;
  return k;
}

void reset_stats(dmpt_ctx c) {
  c->mfma_flops = c->useful_flops = 0;
  c->cg_total = 0;
  c->cg_max = 0;
  c->cg_capped = false;
  c->flags = 0;
  c->cg_unconv = 0;
}

void fill_stats(dmpt_ctx c, const PassIn& in, dmpt_stats* st, int newton, double occ_err, double secs) {
  if (!st) return;
  std::memset(st, 0, sizeof(*st));
  st->newton_iters = newton;
  st->cg_iters_total = (int)c->cg_total;
  st->cg_iters_max = c->cg_max;
  st->flags = c->flags;
  st->cg_unconverged = (int)c->cg_unconv;
  st->occ_err = occ_err;
  const int d = in.order >= 1 ? in.d : 0;
  const int nmu = 1 + in.order * d;
  for (int i = 0; i < nmu; ++i) st->mu[i] = in.mu[i];
  for (int i = 0; i < nmu; ++i) st->trP[i] = c->h_res[RES_TR + i];
  st->tr_pmu = in.beta * (c->h_res[RES_TR] - c->h_res[RES_FRO]);
  // response traces Tr[H^(k) P^(j)] (0 where not computed) and Eq. Resp_0
  auto hp = [&](int kk, int j, int z) -> double {
    return (kk <= in.order && j <= in.order && kk + j <= in.order + 1) ? c->h_res[res_hp(kk, j, z)] : 0.0;
  };
  for (int z = 0; z < d; ++z) {
    st->tr_h1p0[z] = hp(1, 0, z);
    st->tr_h1p1[z] = hp(1, 1, z);
    st->tr_h1p2[z] = hp(1, 2, z);
    st->tr_h1p3[z] = hp(1, 3, z);
    st->tr_h2p0[z] = hp(2, 0, z);
    st->tr_h2p1[z] = hp(2, 1, z);
    st->tr_h2p2[z] = hp(2, 2, z);
    st->tr_h3p0[z] = hp(3, 0, z);
    st->tr_h3p1[z] = hp(3, 1, z);
    double* om[4] = {st->omega1, st->omega2, st->omega3, st->omega4};
    for (int m = 1; m <= in.order + 1 && m <= 4; ++m) {
      double v = 0.0;
      for (int kk = 1; kk <= m; ++kk) v += kk * hp(kk, m - kk, z);
      om[m - 1][z] = v / m;
    }
  }
  st->idempotency = c->h_res[RES_TR] - c->h_res[RES_FRO];
  st->mfma_flops = c->mfma_flops;
  st->useful_flops = c->useful_flops;
  st->seconds = secs;
}

template <class T>
dmpt_status one_pass(const Call& k, const PassIn& in, double* P0, double* const* P1,
                     double* const* P2, double* const* P3) {
  STCHK(recursion_pass<T>(k, in));
  return finish_pass<T>(k, in, P0, P1, P2, P3);
}

dmpt_status pass_dispatch(const Call& k, const PassIn& in, double* P0, double* const* P1,
                          double* const* P2, double* const* P3 = nullptr) {
  if (in.order >= 3 && !P3) return fail(k.c, DMPT_ERR_ARG, "internal: P3 missing");
  Range r("dmpt pass: order %d, %d directions, engine %d", in.order, in.d, (int)k.eng);
  return one_pass<double>(k, in, P0, P1, P2, P3);
}

// Commutator ||H0 P0 - P0 H0||_F and output asymmetry (FP64 checks).
dmpt_status final_checks(dmpt_ctx c, int64_t N, const double* H0, const double* P0, dmpt_stats* st) {
  if (!st) return DMPT_OK;
  hipStream_t s = c->stream;
  // G = H0 P0 with the FP64 engine on workspace members
  {
    Call k = make_call(c, N, false);
    k.eng = Engine::F64;
    k.np = 0;
    // copy H0, P0 into padded FP64 members S1[0] (if present) / Q
    const Group& gh = c->ws.S0;
    const Group& gp = c->ws.Q;
    HIPCHK(c, (sym_combine<double, double>(H0, N, 0, N, k.Np, 0.5, nullptr, 0, (double*)mptr(k, gh, 0),
                                           k.Np, 0, nullptr, 0, 1, s)));
    HIPCHK(c, (sym_combine<double, double>(P0, N, 0, N, k.Np, 0.5, nullptr, 0, (double*)mptr(k, gp, 0),
                                           k.Np, 0, nullptr, 0, 1, s)));
    G g;
    g.X = op(k, gh, 0, false);
    g.Y = op(k, gp, 0, false);
    g.C = mptr(k, c->ws.R, 0);
    const double mf = c->mfma_flops, uf = c->useful_flops;
    STCHK(run_gemm(k, g));
    c->mfma_flops = mf;
    c->useful_flops = uf;
    // ||G - G^T||_F^2 = ||H P - P H||_F^2 (H, P symmetric)
    HIPCHK(c, antisym_sq_partials<double>((const double*)mptr(k, c->ws.R, 0), k.Np, N, c->d_part, s));
    HIPCHK(c, sum_partials(c->d_part, reduce_blocks(N * N), 1, c->d_res + RES_MISC + 1, 1, 0, s));
    HIPCHK(c, hipMemcpyAsync(c->h_res + RES_MISC + 1, c->d_res + RES_MISC + 1, sizeof(double),
                             hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    st->commutator = std::sqrt(std::max(0.0, c->h_res[RES_MISC + 1]));
  }
  HIPCHK(c, asym_max(P0, N, c->d_part, s));
  std::vector<double> mx(reduce_blocks(N * N));
  HIPCHK(c, hipMemcpyAsync(mx.data(), c->d_part, mx.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  double m = 0;
  for (double v : mx) m = std::max(m, v);
  st->asymmetry = m;
  return DMPT_OK;
}

// Allocate a group of `count` Np_max x Np_max members (master + planes).
bool alloc_group(dmpt_ctx c, Group& g, int count, bool planes, std::vector<void*>& owner) {
  const size_t nn = (size_t)c->np_max * c->np_max;
  g.count = count;
  void* p = dev_alloc(c, nn * c->esize * count);
  if (!p) return false;
  owner.push_back(p);
  g.m = p;
  if (hipMemsetAsync(p, 0, nn * c->esize * count, c->stream) != hipSuccess) return false;
  for (int q = 0; q < 3; ++q) g.pl[q] = nullptr;
  if (planes)
    for (int q = 0; q < c->planes; ++q) {
      p = dev_alloc(c, nn * 2 * count);
      if (!p) return false;
      owner.push_back(p);
      g.pl[q] = (uint16_t*)p;
      if (hipMemsetAsync(p, 0, nn * 2 * count, c->stream) != hipSuccess) return false;
    }
  return true;
}

dmpt_status ensure_adjoint(dmpt_ctx c, int n_ck, int n_seg) {
  if (c->CK.count >= n_ck && c->SG.count >= n_seg && c->AY.m) return DMPT_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (void* p : c->ad_allocs) dev_free(c, p);
  c->ad_allocs.clear();
  auto& o = c->ad_allocs;
  bool ok = alloc_group(c, c->AY, 2, true, o) && alloc_group(c, c->AU, 2, true, o) &&
            alloc_group(c, c->AW, 2, true, o) && alloc_group(c, c->AV, 2, true, o) &&
            alloc_group(c, c->AG, 2, false, o) && alloc_group(c, c->AD, 1, true, o) &&
            alloc_group(c, c->CK, n_ck, false, o) && alloc_group(c, c->SG, n_seg, false, o);
  if (!ok) {
    for (void* p : c->ad_allocs) dev_free(c, p);
    c->ad_allocs.clear();
    c->AY = c->AU = c->AW = c->AV = c->AG = c->AD = c->CK = c->SG = Group{};
    return fail(c, DMPT_ERR_NOMEM, "adjoint workspace allocation failed");
  }
  return DMPT_OK;
}

// dst member (with planes) = src member
template <class T>
dmpt_status copy_member(const Call& k, const Group& src, int zs, const Group& dst, int zd) {
  if (zs < 0 || zs >= src.count || zd < 0 || zd >= dst.count)
    return fail(k.c, DMPT_ERR_ARG, "internal: member index out of range");
  uint16_t* pl[3];
  planes_of(k, dst, zd, pl);
  HIPCHK(k.c, axpby<T>((const T*)mptr(k, src, zs), 0, (T*)mptr(k, dst, zd), 0, k.nn, 1, 1.0, 0.0,
                       pl, 0, dst.pl[0] ? k.np : 0, k.c->stream));
  return DMPT_OK;
}

// One order-0 recursion step on c->ws.D0 in place: S0 = D0^2, then T' Y = 2 D0.
template <class T>
dmpt_status forward_step0(const Call& k) {
  G g;
  g.X = op(k, k.c->ws.D0, 0, false);
  g.Y = op(k, k.c->ws.D0, 0, false);
  g.C = mptr(k, k.c->ws.S0, 0);
  planes_of(k, k.c->ws.S0, 0, g.Cpl);
  STCHK(run_gemm(k, g));
  return solve_order0<T>(k, -1);
}

// Reverse sweep of the order-0 recursion for the two seeds Abar and I:
// with Y = D_m = 2 D (I + 4 D^2)^-1, D = D_{m-1}, a cotangent Ybar of Y maps to
//   Dbar = 2 W - 4 (D V + V D),  W = T'^-1 Ybar,  V = W Y      (symmetrised),
// and D_0 = c (H - mu I) gives Hbar = c Dbar_0, mubar = -c Tr Dbar_0.  The
// canonical gradient eliminates mu through Tr P0 = Ne:
//   G = Hbar_A - (mubar_A / mubar_I) Hbar_I.
template <class T>
dmpt_status adjoint_impl(const Call& k, const double* H0, double beta, double mu0, int n,
                         const double* Abar, double* Gout, int ck) {
  dmpt_ctx c = k.c;
  hipStream_t s = c->stream;
  const int hs = c->hstride;
  const double cs = std::ldexp(beta, -(n + 2));
  const int nseg = (n + ck - 1) / ck;
  STCHK(ensure_adjoint(c, nseg, ck));
  // forward: D_0 and every ck-th iterate
  {
    PassIn in{H0, 0, nullptr, nullptr, beta, n, 0, &mu0};
    STCHK(init_d<T>(k, in, cs));
  }
  for (int m = 0; m < n; ++m) {
    if (m % ck == 0) STCHK(copy_member<T>(k, c->ws.D0, 0, c->CK, m / ck));
    STCHK(forward_step0<T>(k));
  }
  // seeds: Ybar_A = -sym(Abar), Ybar_I = -I
  {
    uint16_t* pl[3];
    planes_of(k, c->AY, 0, pl);
    HIPCHK(c, (sym_combine<double, T>(Abar, k.N, 0, k.N, k.Np, -0.5, nullptr, 0,
                                      (T*)mptr(k, c->AY, 0), k.Np, 0, pl, k.np, 1, s)));
    planes_of(k, c->AY, 1, pl);
    HIPCHK(c, scaled_plus_identity<T>((const T*)mptr(k, c->AY, 1), (T*)mptr(k, c->AY, 1), k.N, k.Np,
                                      -1.0, 0.0, pl, k.np, s));
  }
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int n0 = sg * ck, n1 = std::min(n0 + ck, n);
    // recompute D_{n0+1..n1} from the checkpoint D_{n0}
    STCHK(copy_member<T>(k, c->CK, sg, c->ws.D0, 0));
    for (int m = n0 + 1; m <= n1; ++m) {
      STCHK(forward_step0<T>(k));
      STCHK(copy_member<T>(k, c->ws.D0, 0, c->SG, m - n0 - 1));
    }
    for (int m = n1; m > n0; --m) {
      // D = D_{m-1} in c->ws.D0, Y = D_m in AD
      if (m - 1 == n0) STCHK(copy_member<T>(k, c->CK, sg, c->ws.D0, 0));
      else STCHK(copy_member<T>(k, c->SG, m - 2 - n0, c->ws.D0, 0));
      STCHK(copy_member<T>(k, c->SG, m - 1 - n0, c->AD, 0));
      {
        G g;  // S0 = D^2
        g.X = op(k, c->ws.D0, 0, false);
        g.Y = op(k, c->ws.D0, 0, false);
        g.C = mptr(k, c->ws.S0, 0);
        planes_of(k, c->ws.S0, 0, g.Cpl);
        STCHK(run_gemm(k, g));
      }
      // U T' = Ybar (Ybar symmetric), initial guess U = Ybar
      {
        uint16_t* pl[3];
        planes_of(k, c->AU, 0, pl);
        HIPCHK(c, axpby<T>((const T*)mptr(k, c->AY, 0), k.stride, (T*)mptr(k, c->AU, 0), k.stride,
                           k.nn, 2, 1.0, 0.0, pl, k.stride, k.np, s));
        HIPCHK(c, dot_partials<T>((const T*)mptr(k, c->AY, 0), k.stride, (const T*)mptr(k, c->AY, 0),
                                  k.stride, k.nn, 2, c->d_part, s));
        HIPCHK(c, sum_partials(c->d_part, reduce_blocks(k.nn), 2, c->ws.ref, 1, 0, s));
        G g;  // R = Ybar - U - 4 U S0 = -4 U S0
        g.X = op(k, c->AU, 0, true);
        g.Y = op(k, c->ws.S0, 0, false);
        g.C = mptr(k, c->ws.R, 0);
        g.sC = k.stride;
        g.alpha = -4.0;
        g.W = mptr(k, c->ws.R, 0);
        g.sW = k.stride;
        g.batch = 2;
        STCHK(run_gemm(k, g));
        STCHK(sum_gemm_partials(k, 2, c->ws.rr, hs, 0));
        STCHK(cg_solve<T>(k, c->AU, 2, 2, nullptr));  // both seeds share S0
      }
      // W = U^T;  V = W Y;  V <- sym(V);  AG = V D
      {
        uint16_t* pl[3];
        planes_of(k, c->AW, 0, pl);
        HIPCHK(c, transpose<T>((const T*)mptr(k, c->AU, 0), k.Np, k.stride, (T*)mptr(k, c->AW, 0), pl,
                               k.np, 2, s));
        G g;
        g.X = op(k, c->AW, 0, true);
        g.Y = op(k, c->AD, 0, false);
        g.C = mptr(k, c->AV, 0);
        g.sC = k.stride;
        g.batch = 2;
        STCHK(run_gemm(k, g));
        STCHK(sym_inplace<T>(k, c->AV, 0, 2, 0.5));
        G h;
        h.X = op(k, c->AV, 0, true);
        h.Y = op(k, c->ws.D0, 0, false);
        h.C = mptr(k, c->AG, 0);
        h.sC = k.stride;
        h.batch = 2;
        STCHK(run_gemm(k, h));
      }
      // Ybar <- 2 sym(W) - 4 (AG + AG^T) = (U + U^T) - 4 (AG + AG^T)
      {
        uint16_t* pl[3];
        planes_of(k, c->AY, 0, pl);
        HIPCHK(c, (sym_combine<T, T>((const T*)mptr(k, c->AU, 0), k.Np, k.stride, k.N, k.Np, 1.0,
                                     nullptr, 0, (T*)mptr(k, c->AY, 0), k.Np, k.stride, pl, k.np, 2,
                                     s, (const T*)mptr(k, c->AG, 0), -4.0)));
      }
    }
  }
  // G = c (Dbar_A - (Tr Dbar_A / Tr Dbar_I) Dbar_I)
  HIPCHK(c, trace<T>((const T*)mptr(k, c->AY, 0), k.Np, k.stride, k.N, 2, c->d_res + RES_MISC + 4, 1,
                     nullptr, s));
  HIPCHK(c, hipMemcpyAsync(c->h_res + RES_MISC + 4, c->d_res + RES_MISC + 4, 2 * sizeof(double),
                           hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  const double tA = c->h_res[RES_MISC + 4], tI = c->h_res[RES_MISC + 5];
  if (!(std::fabs(tI) > 0.0) || !std::isfinite(tA) || !std::isfinite(tI))
    return fail(c, DMPT_ERR_NONFINITE, "adjoint: d Tr P0 / d mu vanished or is not finite");
  const double r = tA / tI;
  HIPCHK(c, (sym_combine<T, double>((const T*)mptr(k, c->AY, 0), k.Np, 0, k.N, k.Np, 0.5 * cs, nullptr,
                                    0, Gout, k.N, 0, nullptr, 0, 1, s, (const T*)mptr(k, c->AY, 1),
                                    -0.5 * cs * r)));
  HIPCHK(c, hipStreamSynchronize(s));
  return DMPT_OK;
}

// ------------------------------------------------------------------ batched
// Systems of similar size share a bucket (same padded size Np); every
// product, solve and update of a bucket is one batched launch over its
// systems (and directions).  A whole Newton pass over all buckets is
// captured once into a HIP graph and replayed; the CG solves run a fixed,
// a-priori iteration count (members that converge earlier are masked off on
// the device) and the mu update runs on the device, so a pass needs no host
// synchronisation.
struct Bucket {
  int64_t Np = 0;
  int first = 0, m = 0;          // slots [first, first + m) of the bucketed order
  WS ws[3];                      // the same matrices with the system masks of each stage
  double xmax = 0.0;             // max_s c_s * spread_s (|D_0| bound)
};

// Smallest CG iteration count that the Chebyshev bound guarantees for
// kappa(T') <= kappa and relative residual tol, plus a small margin.
int cg_bound(double kappa, double tol, int cap) {
  if (kappa <= 1.0 + 1e-14) return std::min(cap, 2);
  const double sk = std::sqrt(kappa);
  const double rho = (sk - 1.0) / (sk + 1.0);
  const int kk = (int)std::ceil(std::log(tol / (2.0 * sk)) / std::log(rho)) + 2;
  return std::max(1, std::min(cap, kk));
}

// kappa(T'_step) = 1 + 4 max d^2 with |d| <= tanh(2^step artanh(2 x)) / 2, x >= |c (eps - mu)|.
double kappa_bound(double x, int step) {
  const double z = std::min(2.0 * x, 1.0 - 1e-15);
  const double t = std::tanh(std::ldexp(std::atanh(z), step));
  return 1.0 + t * t;
}

// The recursion steps of one batched pass, recorded before graph capture:
// every bucket runs the same sequence of launches (the same code path with a
// common CG count per step), so launch i of every bucket can be issued
// together.  Where launch i is a product in every bucket, one grouped launch
// covers all buckets' (member, tile) blocks; other launches are issued bucket
// by bucket.  Each bucket has its own slice of the partial-sum buffer.
struct BatchedPlan {
  std::vector<std::vector<Op>> ops;     // per bucket
  struct Group {
    int op;                             // launch index
    Engine eng;
    int variant, acc64, edge;
    int list_off, start_off, nprob, blocks;
  };
  std::vector<Group> groups;            // grouped products, in launch order
  std::vector<int> first_group;         // per launch index: first group, or -1 (issue per bucket)
  GemmArgs* d_list = nullptr;           // device copies of the grouped products' arguments
  int* d_start = nullptr;
};

// Per-bucket slices of the partial sums: the most a product's tiles or a
// reduction's blocks need over the bucket's members.
size_t bucket_part_need(const Bucket& b, int members, Engine eng, int variant, int acc64) {
  const size_t mem = (size_t)std::max(members, b.m);
  const size_t nn = (size_t)b.Np * b.Np;
  return std::max((size_t)gemm_tiles(eng, b.Np, variant, acc64), (size_t)reduce_blocks((int64_t)nn)) * mem;
}

// lin = 1: order 1 with the linear schedule; the response P_J to H1 = I runs
// as an extra direction (its D_0 is c I: no input, no mu shift), is written to
// PJs[slot], and each system's P1 is then corrected to Tr P1 = 0 exactly
// (lin_correct), so one pass settles mu1.  lin = 2: order 2 at the settled
// mu1 (no extra direction); each P2 is corrected to Tr P2 = 0 with the P_J
// the order-1 pass stored, so one pass settles mu2.  wsi: the stage's masks.
template <class T>
dmpt_status batched_pass(dmpt_ctx c, std::vector<Bucket>& bk, int wsi, int ord, int d, int n,
                         Engine eng, const std::vector<int>& slot_sys, const double* const* H0s,
                         const double* const* H1s, double* const* P0s, double* const* P1s,
                         double* const* P2s, const int64_t* Ns, const std::vector<double>& cs,
                         double* d_mu_shift, double* d_tr, int rs, double* d_half, int lin,
                         const double* d_par, double* d_mu, double* const* PJs, int rs0,
                         double* d_delta, BatchedPlan* plan, bool record) {
  hipStream_t s = c->stream;
  const int J = 1 + 2 * d;
  const int dd = d + (lin == 1 ? 1 : 0);  // directions the recursion carries
  std::vector<Call> ks(bk.size());
  size_t part_off = 0;
  for (size_t b = 0; b < bk.size(); ++b) {
    Call& k = ks[b];
    k = make_call(c, bk[b].Np, false);
    k.w = &bk[b].ws[wsi];
    k.eng = eng;
    k.np = engine_planes(eng);
    k.N = bk[b].Np;  // inside the workspace every member is treated as Np x Np
    k.Np = bk[b].Np;
    k.nn = k.Np * k.Np;
    k.stride = k.nn;
    k.m = bk[b].m;
    k.graph = true;
    if (plan) {
      // this bucket's slice of the partial sums
      const size_t need = bucket_part_need(bk[b], k.m * std::max(dd, 1), eng, variant_for(c, eng, k.Np),
                                           acc64_of(c, eng));
      k.part = c->d_part + part_off;
      k.part_count = need;
      part_off += need;
      if (part_off > c->part_count) return fail(c, DMPT_ERR_ARG, "internal: batched partials exceed their buffer");
    }
    if (record) continue;
    if (dd > 0) HIPCHK(c, expand_mask(k.w->mask0, dd, k.w->mask1, k.m * dd, s));
  }
  if (record) {
    // the steps only, every bucket with the same CG count per step
    plan->ops.assign(bk.size(), {});
    for (int step = 0; step < n; ++step) {
      int iters = 1;
      for (size_t b = 0; b < bk.size(); ++b)
        iters = std::max(iters, cg_bound(kappa_bound(bk[b].xmax, step), ks[b].tol_cg, c->opt.max_cg));
      for (size_t b = 0; b < bk.size(); ++b) {
        ks[b].cg_iters = iters;
        ks[b].rec = &plan->ops[b];
        STCHK(recursion_step<T>(ks[b], ord, dd, -1));
        ks[b].rec = nullptr;
      }
    }
    return DMPT_OK;
  }
  // D_0 of every system and direction from the caller inputs; the shifts
  // -c mu live on the device so the graph picks up each Newton update.
  for (size_t b = 0; b < bk.size(); ++b) {
    const Call& k = ks[b];
    for (int i = 0; i < k.m; ++i) {
      const int slot = bk[b].first + i, sys = slot_sys[slot];
      const int64_t N = Ns[sys];
      uint16_t* pl[3];
      planes_of(k, k.w->D0, i, pl);
      const int* gate = k.w->mask0 + i;  // this system's activity flag
      HIPCHK(c, (sym_combine<double, T>(H0s[sys], N, 0, N, k.Np, 0.5 * cs[sys],
                                        d_mu_shift + (int64_t)slot * J, 0, (T*)mptr(k, k.w->D0, i),
                                        k.Np, 0, pl, k.np, 1, s, nullptr, 0.0, gate)));
      if (lin == 1) {
        // D_0 of the J direction: c I (the input is not read with a = 0)
        planes_of(k, k.w->D1, i * dd + d, pl);
        HIPCHK(c, (sym_combine<double, T>(H0s[sys], N, 0, N, k.Np, 0.0, d_par + 6 * (int64_t)slot + 2, 0,
                                          (T*)mptr(k, k.w->D1, i * dd + d), k.Np, 0, pl, k.np, 1, s,
                                          nullptr, 0.0, gate)));
      }
      for (int z = 0; z < d && ord >= 1; ++z) {
        const int mem = i * dd + z;
        planes_of(k, k.w->D1, mem, pl);
        HIPCHK(c, (sym_combine<double, T>(H1s[sys * d + z], N, 0, N, k.Np, 0.5 * cs[sys],
                                          d_mu_shift + (int64_t)slot * J + 1 + z, 0,
                                          (T*)mptr(k, k.w->D1, mem), k.Np, 0, pl, k.np, 1, s,
                                          nullptr, 0.0, gate)));
        if (ord >= 2) {
          // H2 = 0: only the shift -c mu2 on the diagonal (a = 0 ignores the input)
          planes_of(k, k.w->D2, mem, pl);
          HIPCHK(c, (sym_combine<double, T>(H1s[sys * d + z], N, 0, N, k.Np, 0.0,
                                            d_mu_shift + (int64_t)slot * J + 1 + d + z, 0,
                                            (T*)mptr(k, k.w->D2, mem), k.Np, 0, pl, k.np, 1, s,
                                            nullptr, 0.0, gate)));
        }
      }
    }
  }
  if (plan) {
    // the recorded steps: launch i of every bucket together, products grouped
    const size_t nops = plan->ops.empty() ? 0 : plan->ops[0].size();
    for (size_t i = 0; i < nops; ++i) {
      const int g0 = plan->first_group[i];
      if (g0 >= 0) {
        for (size_t g = (size_t)g0; g < plan->groups.size() && plan->groups[g].op == (int)i; ++g) {
          const BatchedPlan::Group& G = plan->groups[g];
          HIPCHK(c, gemm_grouped(G.eng, G.variant, G.acc64, G.edge, plan->d_list + G.list_off,
                                 plan->d_start + G.start_off, G.nprob, G.blocks, s));
        }
      } else {
        for (size_t b = 0; b < bk.size(); ++b) {
          const Op& o = plan->ops[b][i];
          HIPCHK(c, o.gemm ? gemm(o.ga, s) : o.fn());
        }
      }
    }
  } else {
    for (int step = 0; step < n; ++step)
      for (size_t b = 0; b < bk.size(); ++b) {
        Call& k = ks[b];
        k.cg_iters = cg_bound(kappa_bound(bk[b].xmax, step), k.tol_cg, c->opt.max_cg);
        STCHK(recursion_step<T>(k, ord, dd, -1));
      }
  }
  // outputs and traces, per system
  for (size_t b = 0; b < bk.size(); ++b) {
    const Call& k = ks[b];
    for (int i = 0; i < k.m; ++i) {
      const int slot = bk[b].first + i, sys = slot_sys[slot];
      const int64_t N = Ns[sys];
      double* t = d_tr + (int64_t)slot * rs;
      const int* gate = k.w->mask0 + i;  // converged systems keep their outputs
      HIPCHK(c, (sym_combine<T, double>((const T*)mptr(k, k.w->D0, i), k.Np, 0, N, k.Np, -0.5, d_half,
                                        0, P0s[sys], N, 0, nullptr, 0, 1, s, nullptr, 0.0, gate)));
      HIPCHK(c, trace<double>(P0s[sys], N, 0, N, 1, t, 1, t + J, s));
      HIPCHK(c, dot_partials<double>(P0s[sys], 0, P0s[sys], 0, N * N, 1, c->d_part, s));
      HIPCHK(c, sum_partials(c->d_part, reduce_blocks(N * N), 1, t + 2 * J, 1, 0, s));
      for (int o = 1; o <= ord; ++o)
        for (int z = 0; z < d; ++z) {
          const int mem = i * dd + z;
          double* Pk = o == 1 ? P1s[sys * d + z] : P2s[sys * d + z];
          const Group& g = o == 1 ? k.w->D1 : k.w->D2;
          const int jt = (o == 1 ? 1 : 1 + d) + z;
          HIPCHK(c, (sym_combine<T, double>((const T*)mptr(k, g, mem), k.Np, 0, N, k.Np, -0.5, nullptr,
                                            0, Pk, N, 0, nullptr, 0, 1, s, nullptr, 0.0, gate)));
          HIPCHK(c, trace<double>(Pk, N, 0, N, 1, t + jt, 1, t + J + jt, s));
          HIPCHK(c, dot_partials<double>(H1s[sys * d + z], 0, Pk, 0, N * N, 1, c->d_part, s));
          HIPCHK(c, sum_partials(c->d_part, reduce_blocks(N * N), 1,
                                 t + 2 * J + 1 + (o == 1 ? 0 : d) + z, 1, 0, s));
        }
      if (lin == 1) {
        double* PJ = PJs[slot];
        HIPCHK(c, (sym_combine<T, double>((const T*)mptr(k, k.w->D1, i * dd + d), k.Np, 0, N, k.Np, -0.5,
                                          nullptr, 0, PJ, N, 0, nullptr, 0, 1, s, nullptr, 0.0, gate)));
        HIPCHK(c, trace<double>(PJ, N, 0, N, 1, t + rs0, 1, t + rs0 + 1, s));
        for (int z = 0; z < d; ++z) {
          HIPCHK(c, dot_partials<double>(H1s[sys * d + z], 0, PJ, 0, N * N, 1, c->d_part, s));
          HIPCHK(c, sum_partials(c->d_part, reduce_blocks(N * N), 1, t + rs0 + 2 + z, 1, 0, s));
        }
        HIPCHK(c, lin_correct(t, d, J, rs0, d_mu + (int64_t)slot * J, d_mu_shift + (int64_t)slot * J,
                              cs[sys], d_delta + (int64_t)slot * d, P1s + (size_t)sys * d, PJ, N, gate,
                              s, 1));
      }
      if (lin == 2) {
        // P2 -= (Tr P2 / Tr P_J) P_J with the P_J of the order-1 pass
        HIPCHK(c, lin_correct(t, d, J, rs0, d_mu + (int64_t)slot * J, d_mu_shift + (int64_t)slot * J,
                              cs[sys], d_delta + (int64_t)slot * d, P2s + (size_t)sys * d, PJs[slot], N,
                              gate, s, 2));
      }
    }
  }
  return DMPT_OK;
}

// Group the recorded launches: launch i is grouped when it is a product in
// every bucket; products with the same variant and tile edge share one
// grouped launch.  The arguments and block offsets are copied to the device
// (before capture; they stay there for every replay).
dmpt_status build_plan(dmpt_ctx c, BatchedPlan& plan, std::vector<void*>& owned) {
  const size_t nb = plan.ops.size();
  if (nb == 0) return DMPT_OK;
  const size_t nops = plan.ops[0].size();
  for (auto& o : plan.ops)
    if (o.size() != nops) return fail(c, DMPT_ERR_ARG, "internal: buckets recorded different launch sequences");
  std::vector<GemmArgs> list;
  std::vector<int> starts;
  plan.first_group.assign(nops, -1);
  for (size_t i = 0; i < nops; ++i) {
    bool all = true;
    for (size_t b = 0; b < nb && all; ++b) all = plan.ops[b][i].gemm;
    if (!all) continue;
    std::vector<bool> used(nb, false);
    for (size_t b0 = 0; b0 < nb; ++b0) {
      if (used[b0]) continue;
      const GemmArgs& a0 = plan.ops[b0][i].ga;
      const int edge = gemm_tile_edge(a0.eng, a0.Np, a0.variant, a0.acc64);
      BatchedPlan::Group G;
      G.op = (int)i;
      G.eng = a0.eng;
      G.variant = a0.variant;
      G.acc64 = a0.acc64;
      G.edge = edge;
      G.list_off = (int)list.size();
      G.start_off = (int)starts.size();
      G.nprob = 0;
      int blocks = 0;
      for (size_t b = b0; b < nb; ++b) {
        const GemmArgs& a = plan.ops[b][i].ga;
        if (used[b] || a.eng != a0.eng || a.variant != a0.variant || a.acc64 != a0.acc64 ||
            gemm_tile_edge(a.eng, a.Np, a.variant, a.acc64) != edge)
          continue;
        used[b] = true;
        list.push_back(a);
        starts.push_back(blocks);
        blocks += a.batch * gemm_tiles(a.eng, a.Np, a.variant, a.acc64);
        ++G.nprob;
      }
      starts.push_back(blocks);
      G.blocks = blocks;
      if (plan.first_group[i] < 0) plan.first_group[i] = (int)plan.groups.size();
      plan.groups.push_back(G);
    }
  }
  if (list.empty()) return DMPT_OK;
  plan.d_list = (GemmArgs*)dev_alloc(c, list.size() * sizeof(GemmArgs));
  plan.d_start = (int*)dev_alloc(c, starts.size() * sizeof(int));
  if (!plan.d_list || !plan.d_start) return fail(c, DMPT_ERR_NOMEM, "batched plan allocation failed");
  owned.push_back(plan.d_list);
  owned.push_back(plan.d_start);
  HIPCHK(c, hipMemcpy(plan.d_list, list.data(), list.size() * sizeof(GemmArgs), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(plan.d_start, starts.data(), starts.size() * sizeof(int), hipMemcpyHostToDevice));
  return DMPT_OK;
}

// Room for the trajectory of n steps x jets members of Np x Np FP32; false
// (and no warm starts) when the device cannot hold it.
bool ensure_traj(dmpt_ctx c, int n, int jets, int64_t Np) {
  const size_t need = (size_t)n * jets * (size_t)Np * Np * sizeof(float);
  c->tj_valid = -1;
  if (c->tj && c->tj_bytes >= need) {
    c->tj_np = Np;
    return true;
  }
  if (c->tj) {
    (void)hipStreamSynchronize(c->stream);
    dev_free(c, c->tj);
    c->tj = nullptr;
    c->tj_bytes = 0;
  }
  void* p = dev_alloc(c, need);
  if (!p) return false;
  c->tj = (float*)p;
  c->tj_bytes = need;
  c->tj_np = Np;
  return true;
}

// Chain store for n steps of 1 + jets1 members of Np x Np masters; false when
// the memory is not there (the order-2 pass then solves orders 0 and 1 again).
bool ensure_chain(dmpt_ctx c, int n, int jets1, int64_t Np) {
  const size_t need = (size_t)n * (1 + jets1) * (size_t)Np * Np * c->esize;
  if (c->st && c->st_bytes >= need) return true;
  if (c->st) {
    (void)hipStreamSynchronize(c->stream);
    dev_free(c, c->st);
    c->st = nullptr;
    c->st_bytes = 0;
  }
  void* p = dev_alloc(c, need);
  if (!p) return false;
  c->st = p;
  c->st_bytes = need;
  return true;
}

// Square-term store for n steps of `members` masters of Np x Np; false when
// the memory is not there (the order-2 pass then forms S0 and S1 again).
bool ensure_squares(dmpt_ctx c, int n, int members, int64_t Np) {
  const size_t need = (size_t)n * members * (size_t)Np * Np * c->esize;
  if (c->ss && c->ss_bytes >= need) return true;
  if (c->ss) {
    (void)hipStreamSynchronize(c->stream);
    dev_free(c, c->ss);
    c->ss = nullptr;
    c->ss_bytes = 0;
  }
  void* p = dev_alloc(c, need);
  if (!p) return false;
  c->ss = p;
  c->ss_bytes = need;
  return true;
}

// Inverse store for n steps of one Np x Np master; false when the memory is
// not there (the later passes then build Z again).
bool ensure_inverses(dmpt_ctx c, int n, int64_t Np) {
  const size_t need = (size_t)n * (size_t)Np * Np * c->esize;
  if (c->zs && c->zs_bytes >= need) return true;
  if (c->zs) {
    (void)hipStreamSynchronize(c->stream);
    dev_free(c, c->zs);
    c->zs = nullptr;
    c->zs_bytes = 0;
  }
  void* p = dev_alloc(c, need);
  if (!p) return false;
  c->zs = p;
  c->zs_bytes = need;
  return true;
}

// Occupation error of Algorithm 1 (*occ_err, absolute) and its normalised
// form (*rel): max(|Tr P0 - Ne| / N, max_k |Tr P^(k)| / sum_i |P^(k)_ii|).
void occupation_error(const double* res, int d, int order, double Ne, int64_t N, double* occ_err,
                      double* rel) {
  double e = std::fabs(res[RES_TR] - Ne);
  double r = e / (double)N;
  for (int i = 1; i < 1 + order * d; ++i) {
    const double t = std::fabs(res[RES_TR + i]);
    e += t;
    r = std::max(r, t / std::max(res[RES_ATR + i], 1e-300));
  }
  *occ_err = e;
  *rel = std::isfinite(e) ? r : INFINITY;
}

// The canonical conditions Tr P^(k) = 0 (k >= 1) are linear in mu^(k): with
// E^(k) = H^(k) - mu^(k) I, P^(k)(mu^(k)) = P^(k)(0) - mu^(k) J, where J is the
// first-order response to H1 = I (the k-th jet starts from c E^(k), and the
// recursion of every jet is linear in its start).  One pass for order 1 (the
// d directions plus J, mu1 = 0) gives mu1 = Tr P1(0) / Tr J; one pass for
// order 2 at that mu1 (mu2 = 0) gives mu2 = Tr P2(0) / Tr J.  This reaches
// the fixed point of Algorithm 1's Newton loop in one pass per order.
//
// The order-1 pass also settles mu0: Tr J = -d Tr P0 / d mu0 exactly (for
// the finite recursion), so while |Tr P0 - Ne| misses the tolerance the pass
// is repeated after the step mu0 += (Tr P0 - Ne) / Tr J.  Its order-0 and
// order-1 solutions of every step are kept (when memory allows) and the
// order-2 pass loads them instead of solving again, with
// Y1 = Y1(mu1 = 0) - mu1 Y_J.
// *settled: whether mu0 met the tolerance (or its noise floor).
dmpt_status linear_orders(Call& k, const PassIn& base, int64_t N, int order, double* mu,
                          double mu_lo, double mu_hi, double Ne, double tol, double prev_rel, double* P0,
                          double* const* P1, double* const* P2, double* const* P3, bool* settled,
                          int* passes) {
  dmpt_ctx c = k.c;
  hipStream_t s = c->stream;
  const int d = base.d;
  const int64_t nn = N * N;
  uint16_t* none[3] = {nullptr, nullptr, nullptr};
  *settled = false;
  c->flags &= ~DMPT_FLAG_NOISE_FLOOR;  // the order-1 pass measures the occupation again
  // ---- order 1 with the identity as direction d
  std::vector<const double*> h1x(base.H1, base.H1 + d);
  h1x.push_back(nullptr);
  std::vector<double*> p1x(P1, P1 + d);
  p1x.push_back(c->jout);
  std::vector<double> m1(2 + 2 * DMPT_MAX_DIRS, 0.0);
  m1[1 + d] = -1.0;  // D0^(1) = c (0 - (-1) I) = c I: the response to H1 = I
  PassIn in1{base.H0, d + 1, h1x.data(), nullptr, base.beta, base.n, 1, m1.data()};
  // chain store: order 0, order 1 (d + J), order 2 (d, when order 3 follows)
  const int cs = 2 + d + (order >= 3 ? d : 0);
  const bool keep = order >= 2 && c->opt.schedule == 1 && ensure_chain(c, base.n, cs, k.Np);
  // and the square terms S0, S1 (d directions and J) for the order-2 pass
  const bool keep_s = keep && ensure_squares(c, base.n, 2 + d, k.Np);
  // and, when these passes solve with the shared inverse, Z of every step
  const bool keep_z = keep_s && ns_pass(k, 1) && ns_pass(k, 2) && ensure_inverses(c, base.n, k.Np);
  k.cs = cs;
  k.cj = 1 + d;
  double trJ = 0.0, prev = INFINITY;
  constexpr int kMaxPasses = 4;
  for (int a = 0; a < kMaxPasses; ++a) {
    m1[0] = mu[0];
    k.chain = keep ? (kSave01 | (keep_s ? kSaveS : 0) | (keep_z ? kSaveZ : 0)) : 0;
    // the final order-0 pass (or the previous order-1 pass) left its inverses
    // at a nearby mu0: start from them where that saves steps
    const bool warm = keep_z && c->zs_valid && !c->ns_cold;
    if (warm) {
      k.chain |= kWarmZ;
      k.z_dmu = std::fabs(mu[0] - c->zs_mu0);
    }
    k.jdir = d;
    const dmpt_status e1 = pass_dispatch(k, in1, P0, p1x.data(), nullptr);
    k.jdir = -1;
    k.chain = 0;
    k.z_dmu = -1.0;
    STCHK(e1);
    c->zs_valid = keep_z;
    c->zs_mu0 = mu[0];
    *passes += 1;
    trJ = c->h_res[RES_TR + 1 + d];
    if (!(std::fabs(trJ) > 0.0) || !std::isfinite(trJ))
      return fail(c, DMPT_ERR_NOCONV, "Tr J vanished: the occupation does not respond to mu");
    const double rel = std::fabs(c->h_res[RES_TR] - Ne) / (double)N;
    if (c->log)
      std::fprintf(stderr,
                   "[dmpt] order-1 pass: mu0 %.15g TrP0-Ne %.3e rel %.3e TrJ %.6e cg_total %ld t %.4f "
                   "mfma %.4e\n",
                   mu[0], c->h_res[RES_TR] - Ne, rel, trJ, c->cg_total, log_clock(), c->mfma_flops);
    // noise floor: the error stopped shrinking (within 1000 tol), or, on the
    // first pass, the Newton step that set mu0 came from the quadratic regime
    // (100 prev_rel^2 <= tol: it should have left ~prev_rel^2) and the error
    // is still within 10 tol -- the floor of this engine's traces
    const bool quad_floor = a == 0 && 100.0 * prev_rel * prev_rel <= tol && rel <= 10.0 * tol;
    if (rel <= tol || quad_floor || (rel > 0.5 * prev && rel <= 1e3 * tol)) {
      if (rel > tol) c->flags |= DMPT_FLAG_NOISE_FLOOR;
      *settled = true;
      break;
    }
    prev = rel;
    mu[0] = std::min(std::max(mu[0] + (c->h_res[RES_TR] - Ne) / trJ, mu_lo), mu_hi);
  }
  if (!*settled) return DMPT_OK;
  for (int z = 0; z < d; ++z) {
    mu[1 + z] = c->h_res[RES_TR + 1 + z] / trJ;
    HIPCHK(c, axpby<double>(c->jout, 0, P1[z], 0, nn, 1, -mu[1 + z], 1.0, none, 0, 0, s));
  }
  if (order >= 2) {
    std::vector<double> m2(1 + 3 * DMPT_MAX_DIRS, 0.0);
    for (int i = 0; i <= d; ++i) m2[i] = mu[i];
    PassIn in2{base.H0, d, base.H1, base.H2, base.beta, base.n, 2, m2.data()};
    k.chain = keep ? (kLoad01 | (keep_s ? kLoadS : 0) | (keep_z ? kLoadZ : 0) | (order >= 3 ? kSave2 : 0)) : 0;
    k.cmu = mu + 1;
    STCHK(pass_dispatch(k, in2, P0, P1, P2));
    k.chain = 0;
    k.cmu = nullptr;
    *passes += 1;
    if (c->log)
      std::fprintf(stderr, "[dmpt] order-2 pass: cg_total %ld t %.4f mfma %.4e\n", c->cg_total, log_clock(),
                   c->mfma_flops);
    for (int z = 0; z < d; ++z) {
      mu[1 + d + z] = c->h_res[RES_TR + 1 + d + z] / trJ;
      HIPCHK(c, axpby<double>(c->jout, 0, P2[z], 0, nn, 1, -mu[1 + d + z], 1.0, none, 0, 0, s));
    }
  }
  if (order >= 3) {
    // order 3 at the exact mu1, mu2 (mu3 = 0); the stored order-2 chain is
    // affine in mu2 with the same slope: Y2 = Y2(mu2 = 0) - mu2 Y_J
    std::vector<double> m3(1 + 3 * DMPT_MAX_DIRS, 0.0);
    for (int i = 0; i <= 2 * d; ++i) m3[i] = mu[i];
    PassIn in3{base.H0, d, base.H1, base.H2, base.beta, base.n, 3, m3.data()};
    in3.H3 = base.H3;
    k.chain = keep ? (kLoad01 | kLoad2 | (keep_z ? kLoadZ : 0)) : 0;
    k.cmu = mu + 1;
    STCHK(pass_dispatch(k, in3, P0, P1, P2, P3));
    k.chain = 0;
    k.cmu = nullptr;
    *passes += 1;
    for (int z = 0; z < d; ++z) {
      mu[1 + 2 * d + z] = c->h_res[RES_TR + 1 + 2 * d + z] / trJ;
      HIPCHK(c, axpby<double>(c->jout, 0, P3[z], 0, nn, 1, -mu[1 + 2 * d + z], 1.0, none, 0, 0, s));
    }
  }
  // traces of the returned (corrected) matrices
  for (int o = 1; o <= order; ++o)
    for (int z = 0; z < d; ++z) {
      double* Pk = o == 1 ? P1[z] : (o == 2 ? P2[z] : P3[z]);
      const int slot = slot_of(o, z, d);
      HIPCHK(c, trace(Pk, N, 0, N, 1, c->d_res + RES_TR + slot, 1, c->d_res + RES_ATR + slot, s));
    }
  HIPCHK(c, hipMemcpyAsync(c->h_res, c->d_res, RES_MISC * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return DMPT_OK;
}

// ---------------------------------------------------------------- thresholded block-sparse path
// A block-sparse matrix (see sparse.hip) with its block count.
struct BSMat {
  BSView v;
  int nslots = 0;
};

// Storage and scratch of one sparse call; every matrix holds up to cap blocks.
struct Sparse {
  dmpt_ctx c = nullptr;
  hipStream_t s = nullptr;
  int64_t N = 0;
  int nb = 0;
  int cap = 0;
  double tau = 0.0;
  uint32_t* bits = nullptr;     // nb bit rows
  int* counts = nullptr;        // nb
  int* keep = nullptr;          // cap
  double* bmax = nullptr;       // max(cap, nb^2)
  double* part = nullptr;       // 4 cap
  double* nprods = nullptr;     // cap
  double* scal = nullptr;       // 8
  BSMat tmp;                    // candidate blocks of the current result
  std::vector<void*> allocs;
  double products = 0.0;
  double blocks_max = 0.0;
  ~Sparse() {
    if (s) (void)hipStreamSynchronize(s);
    for (void* p : allocs) dev_free(c, p);
  }
  void* alloc(size_t bytes) {
    void* p = dev_alloc(c, bytes);
    if (p) allocs.push_back(p);
    return p;
  }
  bool make(BSMat& m) {
    m.v.rows = (int*)alloc(sizeof(int) * (nb + 1));
    m.v.cols = (int*)alloc(sizeof(int) * (size_t)cap);
    m.v.ridx = (int*)alloc(sizeof(int) * (size_t)cap);
    m.v.val = (double*)alloc(sizeof(double) * (size_t)cap * kSparseBlock * kSparseBlock);
    m.nslots = 0;
    if (!m.v.rows || !m.v.cols || !m.v.ridx || !m.v.val) return false;
    return hipMemsetAsync(m.v.rows, 0, sizeof(int) * (nb + 1), s) == hipSuccess;
  }
};

dmpt_status sp_read_int(Sparse& w, const int* dev, int* out) {
  HIPCHK(w.c, hipMemcpyAsync(w.c->h_int, dev, sizeof(int), hipMemcpyDeviceToHost, w.s));
  HIPCHK(w.c, hipStreamSynchronize(w.s));
  *out = w.c->h_int[0];
  return DMPT_OK;
}

dmpt_status sp_capacity(Sparse& w, int need) {
  if (need > w.cap)
    return fail(w.c, DMPT_ERR_NOMEM,
                "sparse path: a result needs " + std::to_string(need) + " blocks, capacity " +
                    std::to_string(w.cap) + " (raise blocks_per_row)");
  return DMPT_OK;
}

// out = e, truncated (out must not be an operand of e).
dmpt_status sp_eval(Sparse& w, const BSExpr& e0, BSMat& out) {
  BSExpr e = e0;
  e.n = w.N;
  hipStream_t s = w.s;
  HIPCHK(w.c, sparse_symbolic(e, w.nb, w.bits, w.counts, w.tmp.v.rows, s));
  int cand = 0;
  STCHK(sp_read_int(w, w.tmp.v.rows + w.nb, &cand));
  STCHK(sp_capacity(w, cand));
  w.blocks_max = std::max(w.blocks_max, (double)cand);
  HIPCHK(w.c, sparse_fill(w.bits, w.nb, w.tmp.v.rows, w.tmp.v.cols, w.tmp.v.ridx, s));
  HIPCHK(w.c, sparse_numeric(e, w.tmp.v, cand, w.tau, w.bmax, w.keep, w.nprods, w.scal, s));
  HIPCHK(w.c, sparse_keep_rows(w.tmp.v.rows, w.keep, w.nb, w.counts, out.v.rows, s));
  HIPCHK(w.c, sparse_compact(w.tmp.v, w.keep, w.nb, out.v, s));
  HIPCHK(w.c, hipMemcpyAsync(w.c->h_int, out.v.rows + w.nb, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(w.c, hipMemcpyAsync(w.c->h_res + RES_MISC, w.scal, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(w.c, hipStreamSynchronize(s));
  out.nslots = w.c->h_int[0];
  w.products += w.c->h_res[RES_MISC];
  return DMPT_OK;
}

// out = a sym(H) + shift I from a dense N x N input (H may be null), truncated.
dmpt_status sp_from_dense(Sparse& w, const double* H, double a, double shift, BSMat& out) {
  HIPCHK(w.c, sparse_dense_pattern(H, w.N, w.nb, a, shift, w.tau, w.bmax, w.scal + 2, w.bits, w.counts,
                                   out.v.rows, w.s));
  int nsl = 0;
  STCHK(sp_read_int(w, out.v.rows + w.nb, &nsl));
  STCHK(sp_capacity(w, nsl));
  HIPCHK(w.c, sparse_fill(w.bits, w.nb, out.v.rows, out.v.cols, out.v.ridx, w.s));
  HIPCHK(w.c, sparse_dense_values(H, w.N, a, shift, out.v, nsl, w.s));
  out.nslots = nsl;
  return DMPT_OK;
}

// Trace, sum of squares, count of |shift I - m| >= thr, sum of H .* m.
dmpt_status sp_stats(Sparse& w, const BSMat& m, double shift, double thr, const double* H, double out[4]) {
  HIPCHK(w.c, sparse_stats(m.v, m.nslots, w.N, shift, thr, H, w.part, w.scal + 4, w.s));
  HIPCHK(w.c, hipMemcpyAsync(w.c->h_res + RES_MISC, w.scal + 4, 4 * sizeof(double), hipMemcpyDeviceToHost,
                             w.s));
  HIPCHK(w.c, hipStreamSynchronize(w.s));
  for (int q = 0; q < 4; ++q) out[q] = w.c->h_res[RES_MISC + q];
  return DMPT_OK;
}

BSExpr sp_prod(const BSMat& A, const BSMat& B, double alpha) {
  BSExpr e;
  e.nterm = 1;
  e.A[0] = A.v;
  e.B[0] = B.v;
  e.alpha[0] = alpha;
  return e;
}
void sp_term(BSExpr& e, const BSMat& A, const BSMat& B, double alpha) {
  e.A[e.nterm] = A.v;
  e.B[e.nterm] = B.v;
  e.alpha[e.nterm] = alpha;
  ++e.nterm;
}
void sp_add(BSExpr& e, const BSMat& C, double beta) {
  e.C[e.nadd] = C.v;
  e.beta[e.nadd] = beta;
  ++e.nadd;
}

// The matrices of one sparse pass: D^(k) jets and their per-step scratch.
struct SparseJets {
  BSMat D0, S0, Z, M, Zn, Y0;
  std::vector<BSMat> D1, S1, R, Y1;  // order-1 directions (+ J)
  std::vector<BSMat> D2, T2, S2, Y2; // order-2 directions
};

// One pass of the recursion (orders 0..order) at a fixed mu jet with the
// shared Newton-Schulz inverse Z of T' = I + 4 D0^2 per step:
//   T' Y0 = 2 D0, T' Y1 = 2 D1 - 4 S1 Y0, T' Y2 = 2 D2 - 4 S1 Y1 - 4 S2 Y0,
// each solved as Y = Z R (Z a polynomial in D0, so Y0 = 2 Z D0 as well).
// d1 order-1 jets start from c (sym H1[z] - mu1[z] I) (H1[z] null: c (-mu1[z]) I),
// d2 order-2 jets from -c mu2[z] I (no H2).
dmpt_status sparse_pass_impl(Sparse& w, SparseJets& J, const double* H0, int d1, const double* const* H1,
                        const double* mu1, int d2, const double* mu2, double mu0, double beta, int n) {
  const double cs = std::ldexp(beta, -(n + 2));
  STCHK(sp_from_dense(w, H0, cs, -cs * mu0, J.D0));
  for (int z = 0; z < d1; ++z) STCHK(sp_from_dense(w, H1[z], H1[z] ? cs : 0.0, -cs * mu1[z], J.D1[z]));
  for (int z = 0; z < d2; ++z) STCHK(sp_from_dense(w, nullptr, 0.0, -cs * mu2[z], J.D2[z]));
  for (int step = 0; step < n; ++step) {
    STCHK(sp_eval(w, sp_prod(J.D0, J.D0, 1.0), J.S0));
    {
      // minimax linear start on [1, 2]: Z = (16 I - 32 S0) / 17
      BSExpr e;
      sp_add(e, J.S0, -32.0 / 17.0);
      e.diag = 16.0 / 17.0;
      STCHK(sp_eval(w, e, J.Z));
    }
    for (int it = 0; it < kNsIters; ++it) {
      BSExpr m = sp_prod(J.S0, J.Z, 4.0);  // M = T' Z = Z + 4 S0 Z
      sp_add(m, J.Z, 1.0);
      STCHK(sp_eval(w, m, J.M));
      BSExpr z = sp_prod(J.Z, J.M, -1.0);  // Z <- 2 Z - Z M
      sp_add(z, J.Z, 2.0);
      STCHK(sp_eval(w, z, J.Zn));
      std::swap(J.Z, J.Zn);
    }
    STCHK(sp_eval(w, sp_prod(J.Z, J.D0, 2.0), J.Y0));
    for (int z = 0; z < d1; ++z) {
      BSExpr e = sp_prod(J.D1[z], J.D0, 1.0);  // S1 = D1 D0 + D0 D1
      sp_term(e, J.D0, J.D1[z], 1.0);
      STCHK(sp_eval(w, e, J.S1[z]));
      BSExpr r = sp_prod(J.S1[z], J.Y0, -4.0);  // R = 2 D1 - 4 S1 Y0
      sp_add(r, J.D1[z], 2.0);
      STCHK(sp_eval(w, r, J.R[z]));
      STCHK(sp_eval(w, sp_prod(J.Z, J.R[z], 1.0), J.Y1[z]));
    }
    for (int z = 0; z < d2; ++z) {
      STCHK(sp_eval(w, sp_prod(J.D1[z], J.D1[z], 1.0), J.T2[z]));
      BSExpr e = sp_prod(J.D2[z], J.D0, 1.0);  // S2 = D2 D0 + D0 D2 + D1 D1
      sp_term(e, J.D0, J.D2[z], 1.0);
      sp_add(e, J.T2[z], 1.0);
      STCHK(sp_eval(w, e, J.S2[z]));
      BSExpr r = sp_prod(J.S2[z], J.Y0, -4.0);  // R = 2 D2 - 4 S2 Y0 - 4 S1 Y1
      sp_term(r, J.S1[z], J.Y1[z], -4.0);
      sp_add(r, J.D2[z], 2.0);
      STCHK(sp_eval(w, r, J.R[z]));
      STCHK(sp_eval(w, sp_prod(J.Z, J.R[z], 1.0), J.Y2[z]));
    }
    std::swap(J.D0, J.Y0);
    for (int z = 0; z < d1; ++z) std::swap(J.D1[z], J.Y1[z]);
    for (int z = 0; z < d2; ++z) std::swap(J.D2[z], J.Y2[z]);
  }
  return DMPT_OK;
}

dmpt_status sparse_pass(Sparse& w, SparseJets& J, const double* H0, int d1, const double* const* H1,
                        const double* mu1, int d2, const double* mu2, double mu0, double beta, int n) {
  Range r("dmpt sparse pass: %d first-order and %d second-order jets", d1, d2);
  return sparse_pass_impl(w, J, H0, d1, H1, mu1, d2, mu2, mu0, beta, n);
}

// ---------------------------------------------------------------- no-allocation path
// dmpt_fermi_recursion_noalloc works in a file-scope device array instead of
// a context's workspace.  Each device holds its own copy of the array; its
// device address is looked up once per device (hipGetSymbolAddress, with the
// device current) and the host-side views of the workspace are built then.
// Nothing is allocated on the device afterwards.
constexpr int64_t kScratchNmax = 512;                     // largest N of the no-allocation path
constexpr size_t kScratchMember = (size_t)kScratchNmax * kScratchNmax * sizeof(double);
constexpr int kScratchMembers = 5;                        // D0, S0, R, P, Q
constexpr size_t kScratchBytes = kScratchMembers * kScratchMember + ((size_t)1 << 20);  // 11 MiB
constexpr int kScratchDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchDevice {
  std::once_flag once;
  dmpt_status st = DMPT_ERR_HIP;
  std::string err;
  dmpt_ctx c = nullptr;      // host-side views of this device's array (never freed)
  int* d_status = nullptr;   // in the array: status word when the caller passes none
};
ScratchDevice g_scratch[kScratchDevices];

// Carve the views once per device: five Np x Np FP64 members of the largest
// padded size, then the solver scalars, partial sums and results.
void scratch_setup(ScratchDevice& sd, int device) {
  char* base = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&base, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !base) {
    sd.err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
    sd.st = DMPT_ERR_HIP;
    return;
  }
  dmpt_ctx c = new dmpt_ctx_s();
  c->device = device;
  dmpt_default_options(&c->opt);
  c->opt.tol_occ = default_tol_occ(DMPT_FP64, 0);
  c->opt.tol_cg = default_tol_cg(DMPT_FP64, 0);
  c->n_max = kScratchNmax;
  c->np_max = padded(kScratchNmax);
  c->dirs_max = 0;
  c->esize = 8;
  c->planes = 0;
  c->hstride = c->opt.max_cg + 2;
  reg_add(c, base, kScratchBytes);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base + off;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  Group* gs[kScratchMembers] = {&c->ws.D0, &c->ws.S0, &c->ws.R, &c->ws.P, &c->ws.Q};
  for (Group* g : gs) {
    g->m = take(kScratchMember);
    g->count = 1;
  }
  c->ws.rr = (double*)take(sizeof(double) * c->hstride);
  c->ws.pq = (double*)take(sizeof(double) * c->hstride);
  c->ws.ref = (double*)take(sizeof(double));
  c->ws.active = (int*)take(sizeof(int));
  c->ws.iters = (int*)take(sizeof(int));
  c->part_count = std::max<size_t>((size_t)(c->np_max / 128) * (c->np_max / 128),
                                   (size_t)reduce_blocks((int64_t)c->np_max * c->np_max));
  c->d_part = (double*)take(sizeof(double) * c->part_count);
  c->d_res = (double*)take(sizeof(double) * RES_COUNT);
  c->d_flag = (int*)take(sizeof(int) * 4);
  c->d_gersh = (double*)take(sizeof(double) * (2 + 2 * (size_t)kScratchNmax));
  c->d_cgstat = (int*)take(sizeof(int) * 4);
  sd.d_status = (int*)take(sizeof(int));
  if (off > kScratchBytes) {
    sd.err = "internal: the no-allocation workspace does not fit its array";
    sd.st = DMPT_ERR_NOMEM;
    delete c;
    return;
  }
  sd.c = c;
  sd.st = DMPT_OK;
}

}  // namespace

// ======================================================================= C ABI
extern "C" {

void dmpt_default_options(dmpt_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->prec = DMPT_FP64;
  o->solver = DMPT_SOLVER_CG;
  o->guess = DMPT_GUESS_PREV;
  o->tol_occ = 0.0;
  o->tol_cg = 0.0;
  o->max_newton = 50;
  o->max_cg = 60;
  o->refine = 0;
  o->ckpt_every = 5;
  o->check = 0;
  o->staged = 1;
  o->warm_traj = 1;
  o->schedule = 1;
  o->acc64 = 1;
  o->autotune = 0;
  o->grouped = 1;
}

static dmpt_status normalise_options(dmpt_ctx c, const dmpt_options* in, dmpt_options* out) {
  dmpt_options o;
  if (in) o = *in; else dmpt_default_options(&o);
  if (o.prec < DMPT_FP64 || o.prec > DMPT_INT8X6) return fail(c, DMPT_ERR_ARG, "unknown precision");
  if (o.refine < 0 || o.refine > 2) return fail(c, DMPT_ERR_ARG, "refine must be 0, 1 or 2");
  if (o.solver != DMPT_SOLVER_CG && o.solver != DMPT_SOLVER_NS && o.solver != DMPT_SOLVER_HYBRID)
    return fail(c, DMPT_ERR_ARG, "unknown solver");
  if (o.guess != DMPT_GUESS_PREV && o.guess != DMPT_GUESS_TAYLOR)
    return fail(c, DMPT_ERR_ARG, "unknown initial guess");
  if (o.schedule < 0 || o.schedule > 2) return fail(c, DMPT_ERR_ARG, "schedule must be 0, 1 or 2");
  if (o.acc64 != 0 && o.acc64 != 1) return fail(c, DMPT_ERR_ARG, "acc64 must be 0 or 1");
  if (o.autotune != 0 && o.autotune != 1) return fail(c, DMPT_ERR_ARG, "autotune must be 0 or 1");
  if (o.grouped != 0 && o.grouped != 1) return fail(c, DMPT_ERR_ARG, "grouped must be 0 or 1");
  if (o.tol_occ <= 0) o.tol_occ = default_tol_occ(o.prec, o.refine);
  if (o.tol_cg <= 0) o.tol_cg = default_tol_cg(o.prec, o.refine);
  if (o.max_newton <= 0) o.max_newton = 50;
  if (o.max_cg <= 0) o.max_cg = 60;
  if (o.max_cg > 500) return fail(c, DMPT_ERR_ARG, "max_cg must be <= 500");
  if (o.ckpt_every <= 0) o.ckpt_every = 5;
  *out = o;
  return DMPT_OK;
}

static char g_noctx_err[256] = "";

dmpt_status dmpt_init(dmpt_ctx* out, int device, int64_t n_max, int dirs_max, const dmpt_options* opt,
                      void* hip_stream) {
  if (!out) return DMPT_ERR_ARG;
  *out = nullptr;
  // the BF16 plane layout indexes an Np x Np member with 32-bit offsets
  if (n_max < 1 || n_max > 65408) {
    std::snprintf(g_noctx_err, sizeof g_noctx_err, "n_max must lie in [1, 65408]");
    return DMPT_ERR_ARG;
  }
  if (dirs_max < 0 || dirs_max > DMPT_MAX_DIRS) {
    std::snprintf(g_noctx_err, sizeof g_noctx_err, "dirs_max must lie in [0, %d]", DMPT_MAX_DIRS);
    return DMPT_ERR_ARG;
  }
  dmpt_ctx c = new dmpt_ctx_s();
  dmpt_status st = normalise_options(c, opt, &c->opt);
  if (st != DMPT_OK) {
    std::snprintf(g_noctx_err, sizeof g_noctx_err, "%s", c->err.c_str());
    delete c;
    return st;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    std::snprintf(g_noctx_err, sizeof g_noctx_err, "no HIP device %d", device);
    delete c;
    return ndev == 0 ? DMPT_ERR_HIP : DMPT_ERR_ARG;
  }
  c->device = device;
  auto bail = [&](dmpt_status s, const char* what) {
    std::snprintf(g_noctx_err, sizeof g_noctx_err, "%s", what);
    dmpt_finalize(c);
    return s;
  };
  if (hipSetDevice(device) != hipSuccess) return bail(DMPT_ERR_HIP, "hipSetDevice failed");
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(DMPT_ERR_HIP, "hipStreamCreate failed");
    c->own_stream = true;
    c->sync_null = true;
    if (hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess)
      return bail(DMPT_ERR_HIP, "hipEventCreate failed");
  }
  if (gemm_prepare() != hipSuccess) return bail(DMPT_ERR_HIP, "product kernel attributes");
  c->log = std::getenv("DMPT_LOG") != nullptr;
  c->debug = std::getenv("DMPT_DEBUG_CHECKS") != nullptr;
  if (const char* e = std::getenv("DMPT_NS_ITERS")) c->ns_iters_env = std::atoi(e);
  if (const char* e = std::getenv("DMPT_NS_REFINE")) c->ns_refine_env = std::atoi(e);
  c->full_tiles = std::getenv("DMPT_FULL_TILES") != nullptr;
  if (const char* e = std::getenv("DMPT_DIAG_SPLIT")) c->diag_split = std::max(0, std::min(8, std::atoi(e)));
  c->ns_cold = std::getenv("DMPT_NS_COLD") != nullptr;


  c->n_max = n_max;
  c->np_max = padded(n_max);
  c->dirs_max = dirs_max;
  c->esize = esize_needed(c->opt);
  c->planes = planes_needed(c->opt);
  c->q8 = q8_needed(c->opt);
  // two members at least (the adjoint solves its two seeds together) and one
  // more than dirs_max (the response to the identity of the linear schedule)
  const int dm = std::max(2, dirs_max + 1);
  const size_t nn = (size_t)c->np_max * c->np_max;
  auto alloc = [&](size_t bytes) -> void* {
    void* p = dev_alloc(c, bytes);
    if (p) c->allocs.push_back(p);
    return p;
  };
  auto group = [&](Group& g, int count, bool planes) -> bool {
    g.count = count;
    g.m = alloc(nn * c->esize * count);
    if (!g.m) return false;
    if (planes)
      for (int p = 0; p < c->planes; ++p) {
        g.pl[p] = (uint16_t*)alloc(nn * 2 * count);
        if (!g.pl[p]) return false;
      }
    if (planes && c->q8 && count > 0) {
      g.q8 = (int8_t*)alloc(nn * kQ8Slices * count);
      g.qs = (double*)alloc(sizeof(double) * count);
      // room for one maximum per product tile, and for the blocks of the
      // element-wise writers (up to 16384 per member keeps them streaming)
      const int64_t cap = std::max<int64_t>((c->np_max / 128) * (c->np_max / 128), 16384);
      double* mx = (double*)alloc(sizeof(double) * (size_t)cap * count);
      if (!g.q8 || !g.qs || !mx) return false;
      Q8Reg r;
      r.m = (const char*)g.m;
      r.stride = (int64_t)nn;
      r.count = count;
      r.q8 = g.q8;
      r.qs = g.qs;
      r.dirty.assign(count, 1);
      r.mx = mx;
      r.mx_cap = cap;
      r.mx_n.assign(count, 0);
      c->q8reg.push_back(r);
    }
    return true;
  };
  const int dd = dirs_max > 0 ? dirs_max + 1 : 0;  // groups for perturbations may be empty
  // R carries planes: the Newton-Schulz solve reads the right-hand sides as an operand
  bool ok = group(c->ws.D0, 1, true) && group(c->ws.S0, 1, true) && group(c->ws.R, dm, true) &&
            group(c->ws.P, dm, true) && group(c->ws.Q, dm, false) && group(c->U0, 1, true) &&
            group(c->ws.Zi, 2, true);
  if (ok && dd > 0)
    ok = group(c->ws.D1, dd, true) && group(c->ws.D2, dd, true) && group(c->ws.D3, dd, true) &&
         group(c->ws.S1, dd, true) && group(c->ws.S2, dd, true) && group(c->ws.S3, dd, true);
  if (!ok) return bail(DMPT_ERR_NOMEM, "device workspace allocation failed");
  c->hstride = c->opt.max_cg + 2;
  c->ws.rr = (double*)alloc(sizeof(double) * dm * 512);
  c->ws.pq = (double*)alloc(sizeof(double) * dm * 512);
  if (c->q8) {
    c->ws.pb = (double*)alloc(sizeof(double) * dm * 512);
    if (!c->ws.pb) return bail(DMPT_ERR_NOMEM, "device scalar allocation failed");
  }
  c->ws.ref = (double*)alloc(sizeof(double) * dm);
  c->ws.active = (int*)alloc(sizeof(int) * dm);
  c->ws.iters = (int*)alloc(sizeof(int) * dm);
  c->d_flag = (int*)alloc(sizeof(int) * 4);
  c->d_res = (double*)alloc(sizeof(double) * RES_COUNT);
  c->d_tally = (double*)alloc(sizeof(double) * 2);
  c->d_cgstat = (int*)alloc(sizeof(int) * 4);
  const size_t tiles = (size_t)(c->np_max / 128) * (c->np_max / 128);
  c->part_count = std::max<size_t>(tiles, 1024) * dm;
  c->d_part = (double*)alloc(sizeof(double) * c->part_count);
  if (c->debug) {
    c->d_dbg = (double*)alloc(sizeof(double) * (size_t)reduce_blocks(c->np_max * c->np_max));
    if (!c->d_dbg) return bail(DMPT_ERR_NOMEM, "device scalar allocation failed");
  }
  if (c->q8) {
    c->d_qpart = (double*)alloc(sizeof(double) * (size_t)q8_blocks(c->np_max) * kQ8Chunk);
    if (!c->d_qpart) return bail(DMPT_ERR_NOMEM, "device scalar allocation failed");
    if (c->diag_split >= 2) {
      // the largest symmetric product batch: the order-2 square terms of every direction
      c->dpart_members = dm;
      c->d_dpart = (double*)alloc(sizeof(double) * (size_t)(c->np_max / 128) * c->diag_split * 128 * 128 * dm);
      if (!c->d_dpart) return bail(DMPT_ERR_NOMEM, "device workspace allocation failed");
    }
  }
  c->d_gersh = (double*)alloc(sizeof(double) * (2 + 2 * (size_t)n_max));
  if (dirs_max > 0) {
    c->jout = (double*)alloc(sizeof(double) * (size_t)n_max * n_max);
    if (!c->jout) return bail(DMPT_ERR_NOMEM, "device workspace allocation failed");
  }
  if (!c->ws.rr || !c->ws.pq || !c->ws.ref || !c->ws.active || !c->ws.iters || !c->d_flag || !c->d_res ||
      !c->d_tally || !c->d_cgstat || !c->d_part || !c->d_gersh)
    return bail(DMPT_ERR_NOMEM, "device scalar allocation failed");
  if (hipHostMalloc((void**)&c->h_res, sizeof(double) * RES_COUNT, hipHostMallocDefault) != hipSuccess)
    return bail(DMPT_ERR_NOMEM, "pinned allocation failed");
  if (hipHostMalloc((void**)&c->h_int, sizeof(int) * 2 * kIterSlot, hipHostMallocDefault) !=
      hipSuccess)
    return bail(DMPT_ERR_NOMEM, "pinned allocation failed");
  // zero the workspace once so the padding of every member starts at zero
  {
    auto zero = [&](const Group& g) -> bool {
      if (!g.m) return true;
      if (hipMemsetAsync(g.m, 0, nn * c->esize * g.count, c->stream) != hipSuccess) return false;
      for (int p = 0; p < 3; ++p)
        if (g.pl[p] && hipMemsetAsync(g.pl[p], 0, nn * 2 * g.count, c->stream) != hipSuccess)
          return false;
      return true;
    };
    if (!(zero(c->ws.D0) && zero(c->ws.S0) && zero(c->ws.R) && zero(c->ws.P) && zero(c->ws.Q) &&
          zero(c->U0) && zero(c->ws.D1) && zero(c->ws.D2) && zero(c->ws.D3) && zero(c->ws.S1) &&
          zero(c->ws.S2) && zero(c->ws.S3)))
      return bail(DMPT_ERR_HIP, "workspace clear failed");
    if (set_values(nullptr, 0, 0, c->d_res + RES_HALF, 0.5, 1, c->stream) != hipSuccess)
      return bail(DMPT_ERR_HIP, "constant init failed");
    if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(DMPT_ERR_HIP, "sync failed");
  }
  *out = c;
  return DMPT_OK;
}

dmpt_status dmpt_profile(dmpt_ctx c, int enable) {
  if (!c) return DMPT_ERR_ARG;
  if (enable) {
    if (c->stream) HIPCHK(c, hipStreamSynchronize(c->stream));
    STCHK(prof_resolve(c));
    c->prof = dmpt_profile_data{};
  }
  c->prof_on = enable != 0;
  return DMPT_OK;
}

dmpt_status dmpt_profile_get(dmpt_ctx c, dmpt_profile_data* out) {
  if (!c || !out) return DMPT_ERR_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  STCHK(prof_resolve(c));
  *out = c->prof;
  return DMPT_OK;
}

dmpt_status dmpt_congruence(dmpt_ctx c, int64_t N, const double* Z, const double* A, double* B,
                            int mode, dmpt_stats* st) {
  if (!c) return DMPT_ERR_ARG;
  if (N < 1 || N > c->n_max) return fail(c, DMPT_ERR_ARG, "N must lie in [1, n_max]");
  if (!Z || !A || !B) return fail(c, DMPT_ERR_ARG, "Z, A and B must be non-NULL");
  if (mode != 0 && mode != 1) return fail(c, DMPT_ERR_ARG, "mode must be 0 (Z^T A Z) or 1 (Z A Z^T)");
  if (B == A || B == Z) return fail(c, DMPT_ERR_ARG, "B must not alias A or Z");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, DMPT_ERR_HIP, "hipSetDevice failed");
  ENTER(c);
  const auto t0 = std::chrono::steady_clock::now();
  reset_stats(c);
  hipStream_t s = c->stream;
  HIPCHK(c, set_values(c->d_flag, 0, 1, nullptr, 0.0, 0, s));
  HIPCHK(c, nonfinite_scan(Z, N, N, c->d_flag, s));
  HIPCHK(c, nonfinite_scan(A, N, N, c->d_flag, s));
  HIPCHK(c, hipMemcpyAsync(c->h_int, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (c->h_int[0]) return fail(c, DMPT_ERR_NONFINITE, "non-finite value in Z or A");
  Call k = make_call(c, N, false);
  k.eng = Engine::F64;
  k.np = 0;
  const WS* w = k.w;
  if (w->R.count < 2) return fail(c, DMPT_ERR_ARG, "internal: workspace too small");
  double* zp = (double*)mptr(k, w->R, 0);  // Z^T (mode 0) or Z (mode 1), padded
  double* ap = (double*)mptr(k, w->R, 1);  // sym(A), padded
  HIPCHK(c, pad_copy(Z, N, N, zp, k.Np, mode == 0, s));
  HIPCHK(c, (sym_combine<double, double>(A, N, 0, N, k.Np, 0.5, nullptr, 0, ap, k.Np, 0, nullptr, 0, 1,
                                         s)));
  // C = X Y^T: mode 0: W = Z^T A, B = W Z; mode 1: V = Z A, B = V Z^T
  G g1;
  g1.X = op(k, w->R, 0, false);
  g1.Y = op(k, w->R, 1, false);
  g1.C = mptr(k, w->Q, 0);
  STCHK(run_gemm(k, g1));
  G g2;
  g2.X = op(k, w->Q, 0, false);
  g2.Y = op(k, w->R, 0, false);
  g2.C = mptr(k, w->P, 0);
  STCHK(run_gemm(k, g2));
  // B = its symmetric part (the exact result is symmetric)
  HIPCHK(c, (sym_combine<double, double>((const double*)mptr(k, w->P, 0), k.Np, 0, N, k.Np, 0.5, nullptr,
                                         0, B, N, 0, nullptr, 0, 1, s)));
  HIPCHK(c, hipStreamSynchronize(s));
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->mfma_flops = c->mfma_flops;
    st->useful_flops = c->useful_flops;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return DMPT_OK;
}

dmpt_status dmpt_bench_product(dmpt_ctx c, int64_t N, dmpt_prec prec, int variant, int reps, double* ms,
                               double* tflops) {
  if (!c || !ms) return DMPT_ERR_ARG;
  if (N < 1 || N > c->n_max) return fail(c, DMPT_ERR_ARG, "N must lie in [1, n_max]");
  if (reps < 1 || reps > 100000) return fail(c, DMPT_ERR_ARG, "reps must lie in [1, 100000]");
  if (prec < DMPT_FP64 || prec > DMPT_INT8X6) return fail(c, DMPT_ERR_ARG, "unknown precision");
  const Engine eng = engine_of(prec);
  if (variant < 0 || variant >= gemm_variants(eng, acc64_of(c, eng)))
    return fail(c, DMPT_ERR_ARG, "no such kernel variant for this precision");
  dmpt_options o = c->opt;
  o.prec = prec;
  o.refine = 0;
  if (esize_needed(o) != c->esize || planes_needed(o) > c->planes || (q8_needed(o) && !c->q8))
    return fail(c, DMPT_ERR_NOMEM, "precision needs a different workspace than the context holds");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, DMPT_ERR_HIP, "hipSetDevice failed");
  ENTER(c);
  Call k = make_call(c, N, false);
  k.eng = eng;
  k.np = engine_planes(k.eng);
  hipStream_t s = c->stream;
  uint16_t* px[3];
  uint16_t* py[3];
  planes_of(k, c->ws.D0, 0, px);
  planes_of(k, c->ws.S0, 0, py);
  HIPCHK(c, fill_pattern<double>((double*)mptr(k, c->ws.D0, 0), k.nn, 1u, px, k.np, s));
  HIPCHK(c, fill_pattern<double>((double*)mptr(k, c->ws.S0, 0), k.nn, 2u, py, k.np, s));
  GemmArgs a{};
  a.eng = k.eng;
  a.Np = k.Np;
  a.batch = 1;
  a.X = op(k, c->ws.D0, 0, false);
  a.Y = op(k, c->ws.S0, 0, false);
  a.C = mptr(k, c->ws.R, 0);
  a.alpha = 1.0;
  a.partials = c->d_part;
  a.acc64 = acc64_of(c, k.eng);
  a.variant = variant;
  if (engine_int8(k.eng)) {
    if (k.Np > kQ8MaxK) return fail(c, DMPT_ERR_UNSUPPORTED, "int8 products need N <= 32768");
    STCHK(q8_operand(k, a.X, 1));
    STCHK(q8_operand(k, a.Y, 1));
  }
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  HIPCHK(c, gemm(a, s));  // warm-up (and LDS attribute)
  HIPCHK(c, hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) HIPCHK(c, gemm(a, s));
  HIPCHK(c, hipEventRecord(e1, s));
  HIPCHK(c, hipEventSynchronize(e1));
  float t = 0.f;
  HIPCHK(c, hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t / reps;
  if (tflops)
    *tflops = 2.0 * (double)k.Np * k.Np * k.Np * engine_terms(k.eng) / (*ms * 1e-3) / 1e12;
  return DMPT_OK;
}

}  // extern "C"

namespace {

void set_variant(dmpt_ctx c, Engine eng, int64_t Np, int v) {
  for (auto& t : c->tuned)
    if (t.eng == (int)eng && t.Np == Np) {
      t.variant = v;
      return;
    }
  c->tuned.push_back({(int)eng, Np, v});
}

bool is_tuned(dmpt_ctx c, Engine eng, int64_t Np) {
  for (auto& t : c->tuned)
    if (t.eng == (int)eng && t.Np == Np) return true;
  return false;
}

dmpt_prec prec_of(Engine e) {
  switch (e) {
    case Engine::F64: return DMPT_FP64;
    case Engine::F32: return DMPT_FP32;
    case Engine::BF16S2: return DMPT_BF16X3;
    case Engine::BF16S3: return DMPT_BF16X6;
    case Engine::I8S4: return DMPT_INT8X13;
    case Engine::I8S3: return DMPT_INT8X6;
  }
  return DMPT_FP64;
}

// Variant from the tuning cache file (DMPT_TUNE_CACHE: lines "arch engine Np acc64 variant ms"),
// or -1.
int cache_lookup(const char* path, const std::string& arch, Engine eng, int64_t Np, int acc64) {
  FILE* f = std::fopen(path, "r");
  if (!f) return -1;
  char a[128];
  int e = 0, acc = 0, v = -1, found = -1;
  long long np = 0;
  double ms = 0.0;
  while (std::fscanf(f, "%127s %d %lld %d %d %lf", a, &e, &np, &acc, &v, &ms) == 6)
    if (arch == a && e == (int)eng && np == Np && acc == acc64) found = v;
  std::fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& arch, Engine eng, int64_t Np, int acc64, int v,
                 double ms) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %lld %d %d %.6f\n", arch.c_str(), (int)eng, (long long)Np, acc64, v, ms);
  std::fclose(f);
}

// Time every variant of one engine at padded size Np (a few products each) and
// keep the fastest; a cached choice for this architecture is taken as is.
dmpt_status tune_engine(dmpt_ctx c, Engine eng, int64_t N, int* chosen) {
  const int64_t Np = padded(N);
  const int acc64 = acc64_of(c, eng);
  const int nv = gemm_variants(eng, acc64);
  const char* path = std::getenv("DMPT_TUNE_CACHE");
  std::string arch;
  {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, c->device) == hipSuccess) arch = p.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    if (arch.empty()) arch = "unknown";
  }
  int best = path ? cache_lookup(path, arch, eng, Np, acc64) : -1;
  if (best < 0 || best >= nv) {
    best = 0;
    double best_ms = INFINITY;
    const int reps = Np >= 4096 ? 2 : (Np >= 1024 ? 5 : 20);
    for (int v = 0; v < nv; ++v) {
      double ms = 0.0;
      STCHK(dmpt_bench_product(c, N, prec_of(eng), v, reps, &ms, nullptr));
      if (ms < best_ms) {
        best_ms = ms;
        best = v;
      }
    }
    if (path) cache_store(path, arch, eng, Np, acc64, best, best_ms);
    if (c->log)
      std::fprintf(stderr, "[dmpt] autotune engine %d Np %lld: %s (%.3f ms)\n", (int)eng, (long long)Np,
                   gemm_variant_name(eng, acc64, best), best_ms);
  }
  set_variant(c, eng, Np, best);
  if (chosen) *chosen = best;
  return DMPT_OK;
}

// The engines a context's products use: its precision's, and the refinement's.
int context_engines(dmpt_ctx c, Engine* out) {
  int n = 0;
  out[n++] = engine_of(c->opt.prec);
  if (refinable(c->opt.prec) && c->opt.refine) out[n++] = refine_engine(c->opt);
  return n;
}

// options.autotune: tune every engine of the context at N unless done already.
dmpt_status autotune_if_asked(dmpt_ctx c, int64_t N) {
  if (!c->opt.autotune) return DMPT_OK;
  Engine e[2];
  const int ne = context_engines(c, e);
  for (int q = 0; q < ne; ++q)
    if (!is_tuned(c, e[q], padded(N))) STCHK(tune_engine(c, e[q], N, nullptr));
  return DMPT_OK;
}

}  // namespace

extern "C" {

dmpt_status dmpt_autotune(dmpt_ctx c, int64_t N, int* variant) {
  if (!c) return DMPT_ERR_ARG;
  if (N < 1 || N > c->n_max) return fail(c, DMPT_ERR_ARG, "N must lie in [1, n_max]");
  Engine e[2];
  const int ne = context_engines(c, e);
  int first = 0;
  for (int q = 0; q < ne; ++q) STCHK(tune_engine(c, e[q], N, q == 0 ? &first : nullptr));
  if (variant) *variant = first;
  return DMPT_OK;
}

dmpt_status dmpt_set_variant(dmpt_ctx c, int64_t N, dmpt_prec prec, int variant) {
  if (!c) return DMPT_ERR_ARG;
  if (N < 1 || N > c->n_max) return fail(c, DMPT_ERR_ARG, "N must lie in [1, n_max]");
  if (prec < DMPT_FP64 || prec > DMPT_INT8X6) return fail(c, DMPT_ERR_ARG, "unknown precision");
  const Engine eng = engine_of(prec);
  if (variant < 0 || variant >= gemm_variants(eng, acc64_of(c, eng)))
    return fail(c, DMPT_ERR_ARG, "no such kernel variant for this precision");
  set_variant(c, eng, padded(N), variant);
  return DMPT_OK;
}

dmpt_status dmpt_get_variant(dmpt_ctx c, int64_t N, dmpt_prec prec, int* variant, int* tuned, char* name,
                             int name_len) {
  if (!c || !variant) return DMPT_ERR_ARG;
  if (N < 1) return fail(c, DMPT_ERR_ARG, "N must be >= 1");
  if (prec < DMPT_FP64 || prec > DMPT_INT8X6) return fail(c, DMPT_ERR_ARG, "unknown precision");
  const Engine eng = engine_of(prec);
  *variant = variant_for(c, eng, padded(N));
  if (tuned) *tuned = is_tuned(c, eng, padded(N)) ? 1 : 0;
  if (name && name_len > 0)
    std::snprintf(name, (size_t)name_len, "%s", gemm_variant_name(eng, acc64_of(c, eng), *variant));
  return DMPT_OK;
}

dmpt_status dmpt_finalize(dmpt_ctx c) {
  if (!c) return DMPT_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto& t : c->prof_pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (auto e : c->prof_pool) (void)hipEventDestroy(e);
  for (void* p : c->allocs) dev_free(c, p);
  c->allocs.clear();
  for (void* p : c->ad_allocs) dev_free(c, p);
  c->ad_allocs.clear();
  for (void* p : c->bt_allocs) dev_free(c, p);
  c->bt_allocs.clear();
  if (c->h_res) (void)hipHostFree(c->h_res);
  if (c->h_int) (void)hipHostFree(c->h_int);
  if (c->tj) dev_free(c, c->tj);
  if (c->st) dev_free(c, c->st);
  if (c->ss) dev_free(c, c->ss);
  if (c->zs) dev_free(c, c->zs);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return DMPT_OK;
}

const char* dmpt_last_error(dmpt_ctx c) {
  if (!c) return g_noctx_err[0] ? g_noctx_err : kNoCtx;
  return c->err.c_str();
}

dmpt_status dmpt_set_options(dmpt_ctx c, const dmpt_options* opt) {
  if (!c) return DMPT_ERR_ARG;
  dmpt_options o;
  STCHK(normalise_options(c, opt, &o));
  if (esize_needed(o) > c->esize || planes_needed(o) > c->planes)
    return fail(c, DMPT_ERR_NOMEM, "options need more workspace than the context holds");
  if (o.max_cg + 2 > 512) return fail(c, DMPT_ERR_ARG, "max_cg too large");
  c->opt = o;
  c->hstride = o.max_cg + 2;
  return DMPT_OK;
}

dmpt_status dmpt_fermi_recursion(dmpt_ctx c, int64_t N, const double* H0, double beta, double mu, int n,
                                 double* P0, dmpt_stats* st) {
  STCHK(check_common(c, N, H0, beta, n));
  if (!P0) return fail(c, DMPT_ERR_ARG, "P0 is NULL");
  if (!std::isfinite(mu)) return fail(c, DMPT_ERR_ARG, "mu must be finite");
  double m[1] = {mu};
  return dmpt_response(c, N, H0, 0, nullptr, nullptr, nullptr, beta, n, 0, m, P0, nullptr, nullptr,
                       nullptr, st);
}

dmpt_status dmpt_sparse_response(dmpt_ctx c, int64_t N, const double* H0, int d, const double* const* H1,
                                 double beta, double Ne, int n, int order, double tau, double count_thr,
                                 int blocks_per_row, double* mu_inout, double* P0, double* const* P1,
                                 double* const* P2, dmpt_sparse_stats* st) {
  if (!c) return DMPT_ERR_ARG;
  if (N < 1 || N > (int64_t)kSparseBlock * 32768) return fail(c, DMPT_ERR_ARG, "sparse path: N must lie in [1, 2^20]");
  if (!H0) return fail(c, DMPT_ERR_ARG, "H0 is NULL");
  if (order < 0 || order > 2) return fail(c, DMPT_ERR_ARG, "sparse path: order must be 0, 1 or 2");
  if (order >= 1 && (d < 1 || d > DMPT_MAX_DIRS || !H1)) return fail(c, DMPT_ERR_ARG, "d must lie in [1, 8] with H1");
  for (int z = 0; order >= 1 && z < d; ++z)
    if (!H1[z]) return fail(c, DMPT_ERR_ARG, "H1[i] is NULL");
  if (!(beta > 0.0) || !std::isfinite(beta)) return fail(c, DMPT_ERR_ARG, "beta must be finite and > 0");
  if (n < 1 || n > 62) return fail(c, DMPT_ERR_ARG, "recursion depth n must lie in [1, 62]");
  if (!(Ne > 0.0 && Ne < (double)N)) return fail(c, DMPT_ERR_ARG, "Ne must lie in (0, N)");
  if (!(tau >= 0.0) || !(tau < 1.0)) return fail(c, DMPT_ERR_ARG, "tau must lie in [0, 1)");
  if (!(count_thr >= 0.0)) return fail(c, DMPT_ERR_ARG, "count_thr must be >= 0");
  if (blocks_per_row < 0) return fail(c, DMPT_ERR_ARG, "blocks_per_row must be >= 0");
  if (!mu_inout) return fail(c, DMPT_ERR_ARG, "mu_inout is NULL");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, DMPT_ERR_HIP, "hipSetDevice failed");
  ENTER(c);
  const auto t0 = std::chrono::steady_clock::now();
  const int dd = order >= 1 ? d : 0;
  // inputs: non-finite values, range of the recursion
  PassIn pin{H0, dd, H1, nullptr, beta, n, order >= 1 ? 1 : 0, nullptr};
  double glo, ghi;
  {
    // N is not bounded by the context's n_max here: a scratch of its own
    double* gs = (double*)dev_alloc(c, sizeof(double) * (2 + 2 * (size_t)N));
    if (!gs) return fail(c, DMPT_ERR_NOMEM, "sparse path: Gershgorin scratch allocation failed");
    const dmpt_status r = scan_inputs(c, N, pin, &glo, &ghi, gs);  // ends with a stream synchronisation
    dev_free(c, gs);
    STCHK(r);
  }
  if (beta * (ghi - glo) >= std::ldexp(1.0, n + 1))
    return fail(c, DMPT_ERR_RANGE, "beta * spread(H0) >= 2^(n+1): the recursion's start leaves [0, 1]");
  double mu0 = mu_inout[0];
  if (std::isnan(mu0)) {
    HIPCHK(c, trace(H0, N, 0, N, 1, c->d_res + RES_MISC + 2, 1, nullptr, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->h_res + RES_MISC + 2, c->d_res + RES_MISC + 2, sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    mu0 = c->h_res[RES_MISC + 2] / (double)N;
  }
  if (!std::isfinite(mu0)) return fail(c, DMPT_ERR_ARG, "mu0 guess must be finite");
  const double lrange = 0.999 * std::ldexp(1.0, n + 1) / beta;
  const double mu_lo = std::max(ghi - lrange, glo - 50.0 / beta);
  const double mu_hi = std::min(glo + lrange, ghi + 50.0 / beta);
  mu0 = std::min(std::max(mu0, mu_lo), mu_hi);
  // storage
  Sparse w;
  w.c = c;
  w.s = c->stream;
  w.N = N;
  w.nb = (int)((N + kSparseBlock - 1) / kSparseBlock);
  w.cap = blocks_per_row > 0 ? (int)std::min<int64_t>((int64_t)blocks_per_row * w.nb, (int64_t)w.nb * w.nb)
                             : (int)std::min<int64_t>((int64_t)w.nb * w.nb, INT32_MAX / 2);
  w.tau = tau;
  const int words = sparse_words(w.nb);
  w.bits = (uint32_t*)w.alloc(sizeof(uint32_t) * (size_t)w.nb * words);
  w.counts = (int*)w.alloc(sizeof(int) * (size_t)(w.nb + 1));
  w.keep = (int*)w.alloc(sizeof(int) * (size_t)w.cap);
  w.bmax = (double*)w.alloc(sizeof(double) * std::max<size_t>((size_t)w.cap, (size_t)w.nb * w.nb));
  w.part = (double*)w.alloc(sizeof(double) * 4 * (size_t)w.cap);
  w.nprods = (double*)w.alloc(sizeof(double) * (size_t)w.cap);
  w.scal = (double*)w.alloc(sizeof(double) * 8);
  const int d1max = dd + (order >= 1 ? 1 : 0);  // directions plus J
  SparseJets J;
  J.D1.resize(d1max); J.S1.resize(d1max); J.R.resize(d1max); J.Y1.resize(d1max);
  J.D2.resize(order >= 2 ? dd : 0); J.T2.resize(J.D2.size()); J.S2.resize(J.D2.size()); J.Y2.resize(J.D2.size());
  BSMat PJ, tmpJ;
  bool ok = w.bits && w.counts && w.keep && w.bmax && w.part && w.nprods && w.scal && w.make(w.tmp) &&
            w.make(J.D0) && w.make(J.S0) && w.make(J.Z) && w.make(J.M) && w.make(J.Zn) && w.make(J.Y0) &&
            w.make(PJ) && w.make(tmpJ);
  for (int z = 0; ok && z < d1max; ++z) ok = w.make(J.D1[z]) && w.make(J.S1[z]) && w.make(J.R[z]) && w.make(J.Y1[z]);
  for (size_t z = 0; ok && z < J.D2.size(); ++z)
    ok = w.make(J.D2[z]) && w.make(J.T2[z]) && w.make(J.S2[z]) && w.make(J.Y2[z]);
  if (!ok) return fail(c, DMPT_ERR_NOMEM, "sparse path: storage allocation failed (lower blocks_per_row)");
  const double tol = std::max(c->opt.tol_occ, tau);
  double st4[4];
  auto occupation = [&](double* trp0, double* frob) -> dmpt_status {
    STCHK(sp_stats(w, J.D0, 0.5, 0.0, nullptr, st4));
    *trp0 = 0.5 * (double)N - st4[0];                      // Tr (I/2 - D0)
    *frob = 0.25 * (double)N - st4[0] + st4[1];            // ||I/2 - D0||_F^2
    return DMPT_OK;
  };
  // ---- mu0: safeguarded Newton on order-0 passes
  int passes = 0;
  double br_lo = mu_lo, br_hi = mu_hi, prev = INFINITY, trp0 = 0.0, frob = 0.0;
  bool settled = false;
  std::vector<double> zero(DMPT_MAX_DIRS + 1, 0.0);
  for (int it = 0; it < c->opt.max_newton; ++it) {
    STCHK(sparse_pass(w, J, H0, 0, nullptr, nullptr, 0, nullptr, mu0, beta, n));
    ++passes;
    STCHK(occupation(&trp0, &frob));
    if (!std::isfinite(trp0)) return fail(c, DMPT_ERR_NONFINITE, "sparse path: non-finite trace");
    const double rel = std::fabs(trp0 - Ne) / (double)N;
    if (c->log)
      std::fprintf(stderr, "[dmpt] sparse pass %d mu0 %.15g TrP0-Ne %.3e blocks %d products %.3e\n", passes,
                   mu0, trp0 - Ne, J.D0.nslots, w.products);
    if (rel <= tol || (rel > 0.5 * prev && rel <= 1e3 * tol)) {
      settled = true;
      break;
    }
    prev = rel;
    if (trp0 < Ne) br_lo = std::max(br_lo, mu0);
    else br_hi = std::min(br_hi, mu0);
    const double trpmu = beta * (trp0 - frob);
    const double mn = mu0 + (Ne - trp0) / trpmu;
    const bool occ_met = std::fabs(trp0 - Ne) <= tol * (double)N;
    if (trpmu > 0.0 && (occ_met || (mn >= br_lo && mn <= br_hi))) mu0 = mn;
    else mu0 = 0.5 * (br_lo + br_hi);
  }
  if (!settled) return fail(c, DMPT_ERR_NOCONV, "sparse path: mu0 did not converge within max_newton passes");
  std::vector<double> mu1(DMPT_MAX_DIRS + 1, 0.0), mu2(DMPT_MAX_DIRS, 0.0);
  double trJ = 0.0;
  if (order >= 1) {
    // order 1 with J (the response to H1 = I: start c I, i.e. mu = -1 and no H1)
    std::vector<const double*> h1x(H1, H1 + dd);
    h1x.push_back(nullptr);
    std::vector<double> m1(dd + 1, 0.0);
    m1[dd] = -1.0;
    bool ok1 = false;
    for (int a = 0; a < 4 && !ok1; ++a) {
      STCHK(sparse_pass(w, J, H0, dd + 1, h1x.data(), m1.data(), 0, nullptr, mu0, beta, n));
      ++passes;
      STCHK(occupation(&trp0, &frob));
      STCHK(sp_stats(w, J.D1[dd], 0.0, 0.0, nullptr, st4));
      trJ = -st4[0];
      if (!(std::fabs(trJ) > 0.0) || !std::isfinite(trJ))
        return fail(c, DMPT_ERR_NOCONV, "sparse path: Tr J vanished");
      const double rel = std::fabs(trp0 - Ne) / (double)N;
      if (rel <= tol || rel <= 1e3 * tol) ok1 = rel <= tol || a > 0;
      if (!ok1) mu0 = std::min(std::max(mu0 + (trp0 - Ne) / trJ, mu_lo), mu_hi);
    }
    if (!ok1) return fail(c, DMPT_ERR_NOCONV, "sparse path: mu0 did not settle in the order-1 pass");
    // mu1 = Tr P1(0) / Tr J, P1 = P1(0) - mu1 J  (P = -D)
    for (int z = 0; z < dd; ++z) {
      STCHK(sp_stats(w, J.D1[z], 0.0, 0.0, nullptr, st4));
      mu1[z] = -st4[0] / trJ;
      BSExpr e;
      sp_add(e, J.D1[z], 1.0);
      sp_add(e, J.D1[dd], -mu1[z]);
      STCHK(sp_eval(w, e, J.Y1[z]));
      std::swap(J.D1[z], J.Y1[z]);
    }
    {
      BSExpr e;  // keep P_J's D for the order-2 correction
      sp_add(e, J.D1[dd], 1.0);
      STCHK(sp_eval(w, e, PJ));
    }
  }
  if (order >= 2) {
    // order 2 at the settled mu1 (mu2 = 0), then P2 = P2(0) - mu2 J
    STCHK(sparse_pass(w, J, H0, dd, H1, mu1.data(), dd, mu2.data(), mu0, beta, n));
    ++passes;
    STCHK(occupation(&trp0, &frob));
    for (int z = 0; z < dd; ++z) {
      STCHK(sp_stats(w, J.D2[z], 0.0, 0.0, nullptr, st4));
      mu2[z] = -st4[0] / trJ;
      BSExpr e;
      sp_add(e, J.D2[z], 1.0);
      sp_add(e, PJ, -mu2[z]);
      STCHK(sp_eval(w, e, J.Y2[z]));
      std::swap(J.D2[z], J.Y2[z]);
    }
  }
  // outputs and statistics
  if (P0) HIPCHK(c, sparse_to_dense(J.D0.v, w.nb, N, -1.0, 0.5, P0, c->stream));
  for (int z = 0; z < dd; ++z) {
    if (P1 && P1[z]) HIPCHK(c, sparse_to_dense(J.D1[z].v, w.nb, N, -1.0, 0.0, P1[z], c->stream));
    if (order >= 2 && P2 && P2[z]) HIPCHK(c, sparse_to_dense(J.D2[z].v, w.nb, N, -1.0, 0.0, P2[z], c->stream));
  }
  mu_inout[0] = mu0;
  for (int z = 0; z < dd; ++z) {
    mu_inout[1 + z] = mu1[z];
    if (order >= 2) mu_inout[1 + dd + z] = mu2[z];
  }
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->newton_iters = passes;
    st->block = kSparseBlock;
    st->mu[0] = mu0;
    STCHK(sp_stats(w, J.D0, 0.5, count_thr, nullptr, st4));
    st->trP[0] = 0.5 * (double)N - st4[0];
    st->nnz_p0 = st4[2];
    st->blocks_p0 = J.D0.nslots;
    for (int z = 0; z < dd; ++z) {
      st->mu[1 + z] = mu1[z];
      STCHK(sp_stats(w, J.D1[z], 0.0, count_thr, H1[z], st4));
      st->trP[1 + z] = -st4[0];
      st->nnz_p1[z] = st4[2];
      st->tr_h1p1[z] = -st4[3];
      st->blocks_p1[z] = J.D1[z].nslots;
      if (order >= 2) {
        st->mu[1 + dd + z] = mu2[z];
        STCHK(sp_stats(w, J.D2[z], 0.0, count_thr, H1[z], st4));
        st->trP[1 + dd + z] = -st4[0];
        st->nnz_p2[z] = st4[2];
        st->tr_h1p2[z] = -st4[3];
        st->blocks_p2[z] = J.D2[z].nslots;
      }
    }
    st->blocks_max = w.blocks_max;
    st->block_products = w.products;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (st) st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return DMPT_OK;
}

dmpt_status dmpt_fermi_recursion_noalloc(int64_t N, const double* H0, double beta, double mu, int n,
                                         double* P0, int* status, void* hip_stream) {
  auto arg = [](const char* msg) {
    std::snprintf(g_noctx_err, sizeof g_noctx_err, "%s", msg);
    return DMPT_ERR_ARG;
  };
  if (N < 1 || N > kScratchNmax) return arg("no-allocation path: N must lie in [1, 512]");
  if (!H0 || !P0) return arg("no-allocation path: H0 and P0 must be non-NULL");
  if (!(beta > 0.0) || !std::isfinite(beta)) return arg("no-allocation path: beta must be finite and > 0");
  if (!std::isfinite(mu)) return arg("no-allocation path: mu must be finite");
  if (n < 1 || n > 62) return arg("no-allocation path: n must lie in [1, 62]");
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess || device < 0 || device >= kScratchDevices) {
    std::snprintf(g_noctx_err, sizeof g_noctx_err, "no-allocation path: no usable current device");
    return DMPT_ERR_HIP;
  }
  ScratchDevice& sd = g_scratch[device];
  std::call_once(sd.once, [&]() { scratch_setup(sd, device); });
  if (sd.st != DMPT_OK) {
    std::snprintf(g_noctx_err, sizeof g_noctx_err, "%s", sd.err.c_str());
    return sd.st;
  }
  dmpt_ctx c = sd.c;
  c->stream = (hipStream_t)hip_stream;
  hipStream_t s = c->stream;
  int* st_word = status ? status : sd.d_status;
  auto hip = [&](hipError_t e) {
    if (e == hipSuccess) return DMPT_OK;
    std::snprintf(g_noctx_err, sizeof g_noctx_err, "no-allocation path: HIP error %s",
                  hipGetErrorString(e));
    return DMPT_ERR_HIP;
  };
  // inputs: non-finite values and the range of the recursion, decided on the device
  STCHK(hip(set_values(c->d_flag, 0, 1, c->d_res + RES_HALF, 0.5, 1, s)));
  STCHK(hip(set_values(c->d_cgstat, 0, 4, nullptr, 0.0, 0, s)));
  STCHK(hip(nonfinite_scan(H0, N, N, c->d_flag, s)));
  STCHK(hip(gershgorin(H0, N, c->d_gersh, s)));
  STCHK(hip(input_status(c->d_gersh, c->d_flag, beta, mu, n, st_word, s)));
  // the recursion with fixed-count solves (no host synchronisation): every
  // step's T' has eigenvalues in [1, 2], so the Chebyshev bound at kappa 2
  // covers every solve; converged solves stop early on the device
  Call k = make_call(c, N, false);
  k.graph = true;
  k.cg_iters = cg_bound(2.0, k.tol_cg, c->opt.max_cg);
  const double cs = std::ldexp(beta, -(n + 2));
  PassIn in{H0, 0, nullptr, nullptr, beta, n, 0, &mu};
  dmpt_status r = init_d<double>(k, in, cs);
  for (int step = 0; r == DMPT_OK && step < n; ++step) r = recursion_step<double>(k, 0, 0, -1);
  if (r == DMPT_OK) {
    // P0 = I/2 - sym(D_n)
    r = hip(sym_combine<double, double>((const double*)mptr(k, c->ws.D0, 0), k.Np, 0, k.N, k.Np, -0.5,
                                        c->d_res + RES_HALF, 0, P0, k.N, 0, nullptr, 0, 1, s));
  }
  if (r != DMPT_OK && r != DMPT_ERR_HIP) {
    std::snprintf(g_noctx_err, sizeof g_noctx_err, "%s", c->err.c_str());
  }
  return r;
}

dmpt_status dmpt_response(dmpt_ctx c, int64_t N, const double* H0, int d, const double* const* H1,
                          const double* const* H2, const double* const* H3, double beta, int n,
                          int order, const double* mu, double* P0, double* const* P1,
                          double* const* P2, double* const* P3, dmpt_stats* st) {
  STCHK(check_common(c, N, H0, beta, n));
  STCHK(check_dirs(c, d, order, H1, (const double* const*)P1, (const double* const*)P2,
                   (const double* const*)P3));
  if (!P0) return fail(c, DMPT_ERR_ARG, "P0 is NULL");
  if (!mu) return fail(c, DMPT_ERR_ARG, "mu is NULL");
  const int nmu = 1 + order * (order >= 1 ? d : 0);
  for (int i = 0; i < nmu; ++i)
    if (!std::isfinite(mu[i])) return fail(c, DMPT_ERR_ARG, "mu jet must be finite");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, DMPT_ERR_HIP, "hipSetDevice failed");
  ENTER(c);
  const auto t0 = std::chrono::steady_clock::now();
  reset_stats(c);
  PassIn in{H0, order >= 1 ? d : 0, H1, H2, beta, n, order, mu};
  in.H3 = H3;
  STCHK(autotune_if_asked(c, N));
  double glo, ghi;
  STCHK(scan_inputs(c, N, in, &glo, &ghi));
  const double emax = std::max(std::fabs(glo - mu[0]), std::fabs(ghi - mu[0]));
  if (beta * emax >= std::ldexp(1.0, n + 1))
    return fail(c, DMPT_ERR_RANGE, "beta * max|eps - mu| >= 2^(n+1): the recursion's start leaves [0, 1]");
  Call k = make_call(c, N, true);
  k.glo = glo;
  k.ghi = ghi;
  STCHK(pass_dispatch(k, in, P0, P1, P2, P3));
  double occ = 0;
  for (int i = 1; i < nmu; ++i) occ += std::fabs(c->h_res[RES_TR + i]);
  STCHK(response_traces(c, N, in, P0, P1, P2, P3));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  fill_stats(c, in, st, 1, occ, secs);
  if (c->opt.check) STCHK(final_checks(c, N, H0, P0, st));
  if (!std::isfinite(c->h_res[RES_TR])) return fail(c, DMPT_ERR_NONFINITE, "non-finite trace");
  if (c->cg_capped) return fail(c, DMPT_ERR_NOCONV, "a linear solve reached max_cg");
  return DMPT_OK;
}

dmpt_status dmpt_mu_newton(dmpt_ctx c, int64_t N, const double* H0, int d, const double* const* H1,
                           const double* const* H2, const double* const* H3, double beta, double Ne,
                           int n, int order, double* mu_inout, double* P0, double* const* P1,
                           double* const* P2, double* const* P3, dmpt_stats* st) {
  STCHK(check_common(c, N, H0, beta, n));
  STCHK(check_dirs(c, d, order, H1, (const double* const*)P1, (const double* const*)P2,
                   (const double* const*)P3));
  if (!P0) return fail(c, DMPT_ERR_ARG, "P0 is NULL");
  if (!mu_inout) return fail(c, DMPT_ERR_ARG, "mu_inout is NULL");
  if (!(Ne > 0.0 && Ne < (double)N)) return fail(c, DMPT_ERR_ARG, "Ne must lie in (0, N)");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, DMPT_ERR_HIP, "hipSetDevice failed");
  ENTER(c);
  const auto t0 = std::chrono::steady_clock::now();
  reset_stats(c);
  c->zs_valid = false;  // stored inverses belong to one call's Hamiltonian
  if (c->log) std::fprintf(stderr, "[dmpt] mu_newton N %lld d %d order %d t %.4f\n", (long long)N, d, order, log_clock());
  const int dd = order >= 1 ? d : 0;
  const int nmu = 1 + order * dd;
  std::vector<double> mu(1 + 3 * DMPT_MAX_DIRS, 0.0);
  for (int i = 0; i < nmu; ++i) mu[i] = mu_inout[i];
  for (int i = 1; i < nmu; ++i)
    if (std::isnan(mu[i])) mu[i] = 0.0;
  PassIn in{H0, dd, H1, H2, beta, n, order, mu.data()};
  in.H3 = H3;
  STCHK(autotune_if_asked(c, N));
  double glo, ghi;
  STCHK(scan_inputs(c, N, in, &glo, &ghi));
  if (beta * (ghi - glo) >= std::ldexp(1.0, n + 1))
    return fail(c, DMPT_ERR_RANGE, "beta * spread(H0) >= 2^(n+1): the recursion's start leaves [0, 1]");
  if (std::isnan(mu[0])) {
    // Tr H0 / N from the diagonal (trace kernel on the caller's H0)
    HIPCHK(c, trace(H0, N, 0, N, 1, c->d_res + RES_MISC + 2, 1, nullptr, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->h_res + RES_MISC + 2, c->d_res + RES_MISC + 2, sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    mu[0] = c->h_res[RES_MISC + 2] / (double)N;
  }
  if (!std::isfinite(mu[0])) return fail(c, DMPT_ERR_ARG, "mu0 guess must be finite");
  // mu0 stays where the recursion is defined (|eps - mu| < 2^(n+1)/beta for the
  // Gershgorin interval) and within a generous thermal margin of the spectrum
  const double lrange = 0.999 * std::ldexp(1.0, n + 1) / beta;
  const double mu_lo = std::max(ghi - lrange, glo - 50.0 / beta);
  const double mu_hi = std::min(glo + lrange, ghi + 50.0 / beta);
  mu[0] = std::min(std::max(mu[0], mu_lo), mu_hi);
  // Phases: with refinement, the cheaper engine of prec (3-product split
  // BF16 or 6-product int8; loose tolerances) brings mu0 close, then the
  // refinement engine (6-product split BF16 or 13-product int8) with the
  // final tolerances finishes; otherwise a single phase.
  Call k = make_call(c, N, false);
  k.glo = glo;
  k.ghi = ghi;
  const bool two_phase = refinable(c->opt.prec) && c->opt.refine;
  struct Phase {
    Engine eng;
    double tol_cg, tol_occ;
  };
  // linear schedule: the loop converges mu0 with order-0 passes, then one
  // pass per order (with the response J to H1 = I) fixes mu1, mu2, mu3 exactly
  const bool linear = c->opt.schedule >= 1 && order >= 1;
  const int loop_order = linear ? 0 : order;
  // trajectory members: order 0, order 1 (plus the identity direction of the
  // linear schedule), orders 2 and 3
  const int jets = linear ? std::max(2 + dd, 1 + order * dd) : 1 + order * dd;
  // only CG reads the trajectory: none when every pass solves with the shared inverse
  const Engine e_final = refinable(c->opt.prec) && c->opt.refine ? refine_engine(c->opt) : engine_of(c->opt.prec);
  const bool all_ns = c->opt.solver == DMPT_SOLVER_NS ||
                      (c->opt.solver == DMPT_SOLVER_HYBRID && (e_final == Engine::F64 || e_final == Engine::I8S4) &&
                       (!(refinable(c->opt.prec) && c->opt.refine) || engine_of(c->opt.prec) == Engine::I8S3));
  if (c->opt.warm_traj && !all_ns && ensure_traj(c, n, jets, k.Np)) {
    k.traj = true;
    k.jets = jets;
  }
  // the passes of the linear schedule run in the final engine.  An order-0
  // pass of the final engine always precedes them: its Newton step settles
  // mu0 far below the occupation tolerance, which P2 needs (its sensitivity
  // to mu0 is much larger than Tr P0's)
  const Phase lin_phase{two_phase ? refine_engine(c->opt) : k.eng, c->opt.tol_cg, c->opt.tol_occ};
  Phase phases[2];
  int nph = 0;
  if (two_phase) {
    const Engine ea = engine_of(c->opt.prec);
    const bool i8a = ea == Engine::I8S3 && c->opt.solver == DMPT_SOLVER_HYBRID;
    phases[nph++] = {ea, kPhaseATolCg, i8a ? kPhaseATolOccI8 : kPhaseATolOcc};
  }
  phases[nph++] = lin_phase;
  int ph = 0;
  double occ = 0;
  int it = 0;
  bool done = false;
  // staged: order-0 passes until mu0 is close, then passes of every order
  const bool staged = c->opt.staged && loop_order > 0;
  int stage_order = staged ? 0 : loop_order;
  double prev_err = INFINITY;
  // bracket of mu0 from the signs of Tr P0 - Ne seen so far (Tr P0 grows
  // with mu0); a Newton step that leaves it, or a vanishing Tr P_mu, is
  // replaced by bisection
  double br_lo = mu_lo, br_hi = mu_hi;
  double last_rel = INFINITY;  // normalised error of the last pass of the loop
  for (it = 1; it <= c->opt.max_newton; ++it) {
    const Phase& P = phases[ph];
    k.eng = P.eng;
    k.np = engine_planes(P.eng);
    k.tol_cg = P.tol_cg;
    k.first_phase = ph < nph - 1;
    in.order = stage_order;
    // the final engine's order-0 passes keep their inverses: the order-1
    // pass starts from them (one mu0 Newton step away)
    const bool save_z = linear && ph == nph - 1 && stage_order == 0 && ns_pass(k, 0) &&
                        ensure_inverses(c, n, k.Np);
    const double pass_mu0 = mu[0];
    k.chain = save_z ? kSaveZ : 0;
    const dmpt_status ep = pass_dispatch(k, in, P0, P1, P2, P3);
    k.chain = 0;
    STCHK(ep);
    if (save_z) {
      c->zs_valid = true;
      c->zs_mu0 = pass_mu0;
    }
    const double* r = c->h_res;
    if (!std::isfinite(r[RES_TR]) || !std::isfinite(r[RES_FRO]))
      return fail(c, DMPT_ERR_NONFINITE, "non-finite trace in the Newton loop");
    double rel = 0.0;
    occupation_error(r, dd, stage_order, Ne, N, &occ, &rel);
    last_rel = rel;
    bool ok = rel <= P.tol_occ;
    const bool last = ph == nph - 1 && stage_order == loop_order;
    if (c->log)
      std::fprintf(stderr,
                   "[dmpt] pass %d phase %d engine %d order %d mu0 %.15g TrP0-Ne %.3e occ_err %.3e "
                   "rel %.3e cg_total %ld t %.4f mfma %.4e\n",
                   it, ph, (int)P.eng, stage_order, mu[0], r[RES_TR] - Ne, occ, rel, c->cg_total, log_clock(),
                   c->mfma_flops);
    // noise floor: a normalised error that stopped shrinking and is within
    // 1000 tol_occ counts as converged (the traces carry the products'
    // rounding); before the final phase and stage this only moves on
    const bool floor_ok = !ok && rel > 0.5 * prev_err && rel <= 1e3 * P.tol_occ;
    if (floor_ok) ok = true;
    if (ok && last) {
      if (floor_ok) c->flags |= DMPT_FLAG_NOISE_FLOOR;
      // linear schedule: the order-1 pass recomputes every order at mu0 (and
      // checks it with the exact slope), so the Newton step from these traces
      // is free and takes mu0 from within tol_occ to its quadratic error; P2's
      // sensitivity to mu0 needs that (an occupation error of 1e-7 N moved P2
      // by a few 1e-6)
      const double trpmu_f = beta * (r[RES_TR] - r[RES_FRO]);
      if (linear && !floor_ok && trpmu_f > 0.0) {
        const double mu_n = mu[0] + (Ne - r[RES_TR]) / trpmu_f;
        if (mu_n >= br_lo && mu_n <= br_hi) mu[0] = mu_n;
      }
      done = true;
      break;
    }
    prev_err = rel;
    if (r[RES_TR] < Ne) br_lo = std::max(br_lo, mu[0]);
    else br_hi = std::min(br_hi, mu[0]);
    const double trpmu = beta * (r[RES_TR] - r[RES_FRO]);
    const double mu_n = mu[0] + (Ne - r[RES_TR]) / trpmu;
    // once Tr P0 meets its own tolerance the (tiny) Newton step is always
    // taken: the bracket's ends then carry the traces' rounding
    const bool occ_met = std::fabs(r[RES_TR] - Ne) <= P.tol_occ * (double)N;
    const bool newton_step = trpmu > 0.0 && (occ_met || (mu_n >= br_lo && mu_n <= br_hi));
    const bool switching = ok && stage_order == loop_order && ph < nph - 1;
    if (switching && rel <= kPhaseABias) {
      if (c->log) std::fprintf(stderr, "[dmpt] phase switch keeps mu0\n");
    } else if (newton_step) {
      mu[0] = mu_n;
      for (int i = 1; i < 1 + stage_order * dd; ++i) mu[i] -= r[RES_TR + i] / trpmu;
    } else {
      mu[0] = 0.5 * (br_lo + br_hi);
      if (c->log) std::fprintf(stderr, "[dmpt] bisection step to mu0 %.15g\n", mu[0]);
    }
    if (ok) {
      prev_err = INFINITY;
      if (stage_order < loop_order) {
        stage_order = loop_order;
      } else if (ph < nph - 1) {
        ++ph;  // the bracket came from a noisier engine: start over
        br_lo = mu_lo;
        br_hi = mu_hi;
      }
    }
    // linear schedule: in the final phase an error this small is settled by
    // the Newton step just taken (quadratic convergence); the order-1 pass
    // measures the result and corrects mu0 with the exact slope if needed
    if (linear && last && newton_step && 100.0 * rel * rel <= P.tol_occ) {
      done = true;
      break;
    }
  }
  if (it > c->opt.max_newton) it = c->opt.max_newton;
  if (done && linear) {
    const Phase& P = lin_phase;
    k.eng = P.eng;
    k.np = engine_planes(P.eng);
    k.tol_cg = P.tol_cg;
    k.first_phase = false;
    bool settled = false;
    int passes = 0;
    STCHK(linear_orders(k, in, N, order, mu.data(), mu_lo, mu_hi, Ne, P.tol_occ, last_rel, P0, P1, P2, P3,
                        &settled, &passes));
    it += passes;
    done = settled;
    occupation_error(c->h_res, dd, settled ? order : 1, Ne, N, &occ, &prev_err);
  }
  in.order = order;
  for (int i = 0; i < nmu; ++i) mu_inout[i] = mu[i];
  STCHK(response_traces(c, N, in, P0, P1, P2, P3));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  fill_stats(c, in, st, it, occ, secs);
  if (c->opt.check) STCHK(final_checks(c, N, H0, P0, st));
  if (!done) return fail(c, DMPT_ERR_NOCONV, "Newton loop did not reach tol_occ within max_newton passes");
  if (c->cg_capped) return fail(c, DMPT_ERR_NOCONV, "a linear solve reached max_cg");
  return DMPT_OK;
}

dmpt_status dmpt_mu_newton_batched(dmpt_ctx c, int nsys, const int64_t* Ns, const double* const* H0s,
                                   int d, const double* const* H1s, const double* betas,
                                   const double* Nes, int n, int order, double* mus,
                                   double* const* P0s, double* const* P1s, double* const* P2s,
                                   dmpt_stats* st) {
  if (!c) return DMPT_ERR_ARG;
  if (nsys < 1 || !Ns || !H0s || !betas || !Nes || !mus || !P0s)
    return fail(c, DMPT_ERR_ARG, "batched: nsys >= 1 and non-NULL Ns, H0s, betas, Nes, mus, P0s");
  if (order < 0 || order > 2) return fail(c, DMPT_ERR_ARG, "batched order must be 0, 1 or 2");
  if (order >= 1 && (d < 1 || d > DMPT_MAX_DIRS))
    return fail(c, DMPT_ERR_ARG, "d must lie in [1, DMPT_MAX_DIRS]");
  if (order == 0) d = 0;
  if (n < 1 || n > 62) return fail(c, DMPT_ERR_ARG, "recursion depth n must lie in [1, 62]");
  if (order >= 1 && (!H1s || !P1s)) return fail(c, DMPT_ERR_ARG, "H1s and P1s are required");
  if (order >= 2 && !P2s) return fail(c, DMPT_ERR_ARG, "P2s is required");
  for (int sy = 0; sy < nsys; ++sy) {
    if (Ns[sy] < 1 || Ns[sy] > c->n_max) return fail(c, DMPT_ERR_ARG, "each N must lie in [1, n_max]");
    if (!H0s[sy] || !P0s[sy]) return fail(c, DMPT_ERR_ARG, "NULL H0 or P0");
    if (!(betas[sy] > 0.0) || !std::isfinite(betas[sy])) return fail(c, DMPT_ERR_ARG, "beta must be > 0");
    if (!(Nes[sy] > 0.0 && Nes[sy] < (double)Ns[sy])) return fail(c, DMPT_ERR_ARG, "Ne must lie in (0, N)");
    for (int z = 0; z < d; ++z) {
      if (!H1s[sy * d + z] || !P1s[sy * d + z]) return fail(c, DMPT_ERR_ARG, "NULL H1 or P1");
      if (order >= 2 && !P2s[sy * d + z]) return fail(c, DMPT_ERR_ARG, "NULL P2");
    }
  }
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, DMPT_ERR_HIP, "hipSetDevice failed");
  ENTER(c);
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = c->stream;
  reset_stats(c);
  const int J = 1 + 2 * d;
  // linear schedule (orders 1 and 2): after the order-0 stage, one order-1
  // pass carries the J direction and settles mu1 (batched_pass), and at order
  // 2 one more pass settles mu2 with the stored P_J; J's records follow the
  // others
  const int lin = (c->opt.schedule >= 1 && order >= 1) ? 1 : 0;
  const int rs0 = 2 * J + 1 + 2 * d;
  const int rs = rs0 + (lin ? 2 + d : 0);
  // per system: Gershgorin interval, range guard, bounds of mu0, c
  std::vector<double> cs(nsys), par(6 * (size_t)nsys), mu0(nsys), xs(nsys);
  for (int sy = 0; sy < nsys; ++sy) {
    PassIn in{H0s[sy], d, order >= 1 ? H1s + (size_t)sy * d : nullptr, nullptr, betas[sy], n,
              order, nullptr};
    double glo, ghi;
    STCHK(scan_inputs(c, Ns[sy], in, &glo, &ghi));
    if (betas[sy] * (ghi - glo) >= std::ldexp(1.0, n + 1))
      return fail(c, DMPT_ERR_RANGE, "beta * spread(H0) >= 2^(n+1) for a system of the batch");
    cs[sy] = std::ldexp(betas[sy], -(n + 2));
    const double lr = 0.999 * std::ldexp(1.0, n + 1) / betas[sy];
    const double lo = std::max(ghi - lr, glo - 50.0 / betas[sy]);
    const double hi = std::min(glo + lr, ghi + 50.0 / betas[sy]);
    par[6 * sy + 0] = betas[sy];
    par[6 * sy + 1] = Nes[sy];
    par[6 * sy + 2] = cs[sy];
    par[6 * sy + 3] = lo;
    par[6 * sy + 4] = hi;
    par[6 * sy + 5] = (double)Ns[sy];
    double m0 = mus[(size_t)sy * J];
    if (!std::isfinite(m0)) m0 = 0.5 * (glo + ghi);
    mu0[sy] = std::min(std::max(m0, lo), hi);
    xs[sy] = cs[sy] * (ghi - glo);
  }
  // buckets by padded size, systems in bucket order ("slots")
  std::vector<int> slot_sys(nsys);
  for (int i = 0; i < nsys; ++i) slot_sys[i] = i;
  std::stable_sort(slot_sys.begin(), slot_sys.end(),
                   [&](int a, int b) { return padded(Ns[a]) < padded(Ns[b]); });
  std::vector<Bucket> bk;
  for (int i = 0; i < nsys; ++i) {
    const int64_t Np = padded(Ns[slot_sys[i]]);
    if (bk.empty() || bk.back().Np != Np) {
      bk.push_back(Bucket{});
      bk.back().Np = Np;
      bk.back().first = i;
    }
    bk.back().m += 1;
    bk.back().xmax = std::max(bk.back().xmax, xs[slot_sys[i]]);
  }
  // the batch's product engine; with options.autotune every bucket size is tuned first
  const Engine eng = (refinable(c->opt.prec) && c->opt.refine) ? refine_engine(c->opt)
                                                                 : engine_of(c->opt.prec);
  if (engine_int8(eng)) return fail(c, DMPT_ERR_UNSUPPORTED, "the batched solve has no int8 products");
  if (c->opt.autotune)
    for (auto& b : bk)
      if (!is_tuned(c, eng, b.Np)) STCHK(tune_engine(c, eng, std::min<int64_t>(b.Np, c->n_max), nullptr));
  const int np = engine_planes(eng);
  const int dmem = std::max(1, d + lin);
  size_t need = 0, part_need = c->part_count;
  for (auto& b : bk) {
    const size_t nn = (size_t)b.Np * b.Np;
    const size_t per = nn * (c->esize + 2 * np);
    need += per * (size_t)b.m * (2 + 3 * (size_t)dmem + (size_t)(order >= 1 ? 2 * d : 0) +
                                 (size_t)(order >= 2 ? 2 * d : 0));
    part_need = std::max(part_need, (size_t)(b.Np / 128) * (b.Np / 128) * b.m * dmem);
    part_need = std::max(part_need, (size_t)reduce_blocks((int64_t)nn) * b.m * dmem);
  }
  if (c->opt.grouped) {
    // grouped launches: every bucket its own slice of the partial sums
    size_t sum = 0;
    for (auto& b : bk) sum += bucket_part_need(b, b.m * dmem, eng, variant_for(c, eng, b.Np), acc64_of(c, eng));
    part_need = std::max(part_need, sum);
  }
  const int hs = c->hstride;
  (void)need;
  if (part_need > c->part_count) {
    // a larger partials block, kept until dmpt_finalize
    HIPCHK(c, hipStreamSynchronize(s));
    void* p = dev_alloc(c, part_need * sizeof(double));
    if (!p) return fail(c, DMPT_ERR_NOMEM, "batched partials allocation failed");
    c->bt_allocs.push_back(p);
    c->d_part = (double*)p;
    c->part_count = part_need;
  }
  // carve every bucket's groups from per-bucket allocations
  std::vector<void*> local;  // freed at the end of the call
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    for (void* p : local) dev_free(c, p);
  };
  auto galloc = [&](Group& g, int count, int64_t Np, bool planes) -> bool {
    const size_t nn = (size_t)Np * Np;
    void* p = dev_alloc(c, nn * c->esize * count);
    if (!p) return false;
    local.push_back(p);
    g.m = p;
    g.count = count;
    if (hipMemsetAsync(p, 0, nn * c->esize * count, s) != hipSuccess) return false;
    for (int q = 0; q < 3; ++q) g.pl[q] = nullptr;
    if (planes)
      for (int q = 0; q < np; ++q) {
        p = dev_alloc(c, nn * 2 * count);
        if (!p) return false;
        local.push_back(p);
        g.pl[q] = (uint16_t*)p;
        if (hipMemsetAsync(p, 0, nn * 2 * count, s) != hipSuccess) return false;
      }
    return true;
  };
  auto dalloc = [&](size_t bytes) -> void* {
    void* p = dev_alloc(c, bytes);
    if (p) local.push_back(p);
    return p;
  };
  // per-slot device state
  double* d_mu = (double*)dalloc(sizeof(double) * nsys * J);
  double* d_shift = (double*)dalloc(sizeof(double) * nsys * J);
  double* d_tr = (double*)dalloc(sizeof(double) * nsys * rs);
  double* d_par = (double*)dalloc(sizeof(double) * nsys * 6);
  double* d_prev = (double*)dalloc(sizeof(double) * nsys);
  double* d_brk = (double*)dalloc(sizeof(double) * 2 * nsys);
  double* d_occ = (double*)dalloc(sizeof(double) * nsys);
  int* d_flags = (int*)dalloc(sizeof(int) * nsys * 6);  // activeA, activeB, done, passes, status, spare
  double* d_delta = lin ? (double*)dalloc(sizeof(double) * nsys * d) : nullptr;
  int64_t nbig = 1;
  for (int sy = 0; sy < nsys; ++sy) nbig = std::max(nbig, Ns[sy]);
  double* d_w = lin ? (double*)dalloc(sizeof(double) * nbig) : nullptr;  // mu1 guess scratch
  int* d_want = lin ? (int*)dalloc(sizeof(int) * nsys * d) : nullptr;
  std::vector<double*> pjs(nsys, nullptr);  // per slot: P_J (N x N FP64)
  bool pj_ok = true;
  for (int slot = 0; slot < nsys && lin; ++slot) {
    const int64_t N = Ns[slot_sys[slot]];
    pjs[slot] = (double*)dalloc(sizeof(double) * (size_t)N * N);
    pj_ok = pj_ok && pjs[slot];
  }
  if (!d_mu || !d_shift || !d_tr || !d_par || !d_prev || !d_brk || !d_occ || !d_flags ||
      (lin && (!d_delta || !pj_ok || !d_w || !d_want))) {
    cleanup();
    return fail(c, DMPT_ERR_NOMEM, "batched scalar allocation failed");
  }
  int* actA = d_flags;
  int* actB = d_flags + nsys;
  int* done = d_flags + 2 * nsys;
  int* passes = d_flags + 3 * nsys;
  int* status = d_flags + 4 * nsys;
  int* actC = d_flags + 5 * nsys;
  for (auto& b : bk) {
    const int md = b.m * dmem;
    WS w;
    bool ok = galloc(w.D0, b.m, b.Np, true) && galloc(w.S0, b.m, b.Np, true) &&
              galloc(w.R, md, b.Np, false) && galloc(w.P, md, b.Np, true) && galloc(w.Q, md, b.Np, false);
    if (ok && order >= 1) ok = galloc(w.D1, md, b.Np, true) && galloc(w.S1, md, b.Np, true);
    if (ok && order >= 2) ok = galloc(w.D2, md, b.Np, true) && galloc(w.S2, md, b.Np, true);
    w.rr = ok ? (double*)dalloc(sizeof(double) * md * hs) : nullptr;
    w.pq = ok ? (double*)dalloc(sizeof(double) * md * hs) : nullptr;
    w.ref = ok ? (double*)dalloc(sizeof(double) * md) : nullptr;
    w.active = ok ? (int*)dalloc(sizeof(int) * md) : nullptr;
    w.iters = ok ? (int*)dalloc(sizeof(int) * md) : nullptr;
    w.mask1 = ok ? (int*)dalloc(sizeof(int) * md) : nullptr;
    if (!ok || !w.rr || !w.pq || !w.ref || !w.active || !w.iters || !w.mask1) {
      cleanup();
      return fail(c, DMPT_ERR_NOMEM, "batched workspace allocation failed");
    }
    for (int q = 0; q < 3; ++q) b.ws[q] = w;
    b.ws[0].mask0 = actA + b.first;
    b.ws[1].mask0 = actB + b.first;
    b.ws[2].mask0 = actC + b.first;
  }
  // initial state
  {
    std::vector<double> hmu((size_t)nsys * J, 0.0), hsh((size_t)nsys * J, 0.0), hpar(6 * (size_t)nsys);
    for (int slot = 0; slot < nsys; ++slot) {
      const int sy = slot_sys[slot];
      for (int j = 0; j < J; ++j) {
        double v = j == 0 ? mu0[sy] : mus[(size_t)sy * J + j];
        if (!std::isfinite(v)) v = 0.0;
        hmu[(size_t)slot * J + j] = v;
        hsh[(size_t)slot * J + j] = -cs[sy] * v;
      }
      for (int q = 0; q < 6; ++q) hpar[6 * (size_t)slot + q] = par[6 * (size_t)sy + q];
    }
    std::vector<int> hfl(6 * (size_t)nsys, 0);
    for (int i = 0; i < 2 * nsys; ++i) hfl[i] = 1;
    for (int i = 5 * nsys; i < 6 * nsys; ++i) hfl[i] = 1;
    std::vector<double> hbrk(2 * (size_t)nsys);
    for (int slot = 0; slot < nsys; ++slot) {
      hbrk[2 * slot] = hpar[6 * (size_t)slot + 3];
      hbrk[2 * slot + 1] = hpar[6 * (size_t)slot + 4];
    }
    // first-order mu values the caller left open get a guess before the final stage
    std::vector<int> hwant(lin ? (size_t)nsys * d : 0);
    for (int slot = 0; slot < nsys && lin; ++slot)
      for (int z = 0; z < d; ++z)
        hwant[(size_t)slot * d + z] = !std::isfinite(mus[(size_t)slot_sys[slot] * J + 1 + z]);
    if ((lin && hipMemcpy(d_want, hwant.data(), hwant.size() * sizeof(int), hipMemcpyHostToDevice) !=
                    hipSuccess) ||
        hipMemcpy(d_mu, hmu.data(), hmu.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_shift, hsh.data(), hsh.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_par, hpar.data(), hpar.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_brk, hbrk.data(), hbrk.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_flags, hfl.data(), hfl.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
      cleanup();
      return fail(c, DMPT_ERR_HIP, "batched state upload failed");
    }
  }
  const bool staged = c->opt.staged && order > 0;
  const bool prof = c->prof_on;
  c->prof_on = false;  // no event records inside a captured graph
  hipGraphExec_t gx[3] = {nullptr, nullptr, nullptr};
  hipGraph_t gg[3] = {nullptr, nullptr, nullptr};
  dmpt_status rc = DMPT_OK;
  int total_passes = 0;
  // executed work over every replay, tallied on the device by the products
  // of members that actually run
  if (rc == DMPT_OK && (hipMemsetAsync(c->d_tally, 0, 2 * sizeof(double), s) != hipSuccess ||
                        hipMemsetAsync(c->d_cgstat, 0, 4 * sizeof(int), s) != hipSuccess))
    rc = fail(c, DMPT_ERR_HIP, "tally reset failed");
  // stages: order-0 Newton replays (staged), then either the linear schedule
  // (an order-1 pass with J, and at order 2 an order-2 pass) or Algorithm 1's
  // joint Newton replays of every order
  struct Stage {
    int ord, lin, wsi;
    bool final_stage;
    double tol;
  };
  std::vector<Stage> stages;
  if (staged) stages.push_back({0, 0, 0, false, lin ? 1e-2 * c->opt.tol_occ : c->opt.tol_occ});
  if (lin) {
    stages.push_back({1, 1, order == 1 ? 1 : 2, order == 1, c->opt.tol_occ});
    if (order == 2) stages.push_back({2, 2, 1, true, c->opt.tol_occ});
  } else {
    stages.push_back({order, 0, 1, true, c->opt.tol_occ});
  }
  for (size_t si = 0; si < stages.size() && rc == DMPT_OK; ++si) {
    const Stage& SG = stages[si];
    const int stage = (int)si;
    const int ord = SG.ord;
    const bool final_stage = SG.final_stage;
    if (SG.lin == 1 && staged) {
      // mu1 guesses from the converged P0 of the first stage, so the linear
      // correction after the pass is small
      for (int slot = 0; slot < nsys && rc == DMPT_OK; ++slot) {
        const int sy = slot_sys[slot];
        if (mu1_guess(P0s[sy], Ns[sy], H1s + (size_t)sy * d, d, d_w, d_mu + (size_t)slot * J,
                      d_shift + (size_t)slot * J, cs[sy], d_want + (size_t)slot * d, s) != hipSuccess)
          rc = fail(c, DMPT_ERR_HIP, "mu1 guess launch failed");
      }
      if (rc != DMPT_OK) break;
    }
    {
      // every stage starts its noise-floor test afresh
      std::vector<double> hprev(nsys, INFINITY);
      if (hipMemcpy(d_prev, hprev.data(), hprev.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
        rc = fail(c, DMPT_ERR_HIP, "batched state upload failed");
        break;
      }
    }
    // grouped launches: record this stage's steps and build the grouped products first
    BatchedPlan plan;
    BatchedPlan* pplan = c->opt.grouped ? &plan : nullptr;
    if (pplan) {
      dmpt_status pr = batched_pass<double>(c, bk, SG.wsi, ord, d, n, eng, slot_sys, H0s, H1s, P0s, P1s, P2s,
                                            Ns, cs, d_shift, d_tr, rs, c->d_res + RES_HALF, SG.lin, d_par,
                                            d_mu, pjs.data(), rs0, d_delta, pplan, true);
      if (pr == DMPT_OK) pr = build_plan(c, plan, local);
      if (pr != DMPT_OK) {
        rc = pr;
        break;
      }
    }
    // capture one pass of this stage
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      rc = fail(c, DMPT_ERR_HIP, "hipStreamBeginCapture failed");
      break;
    }
    dmpt_status cr = batched_pass<double>(c, bk, SG.wsi, ord, d, n, eng, slot_sys, H0s, H1s, P0s,
                                          P1s, P2s, Ns, cs, d_shift, d_tr, rs, c->d_res + RES_HALF,
                                          SG.lin, d_par, d_mu, pjs.data(), rs0, d_delta, pplan, false);
    if (cr == DMPT_OK) {
      // with the linear schedule the later stages run one pass each and no
      // longer move mu0: the first stage settles it a hundred times tighter
      // (the responses carry mu0's error times their derivative in mu0)
      int* act_stage = SG.wsi == 0 ? actA : (SG.wsi == 1 ? actB : actC);
      const hipError_t e = newton_update(d_tr, rs, d_par, d_mu, d_shift, J, ord * d, SG.tol,
                                         final_stage ? 1 : 0, act_stage, done, d_prev, d_brk, d_occ,
                                         passes, status, nsys, s);
      if (e != hipSuccess) cr = fail(c, DMPT_ERR_HIP, "newton_update launch failed");
    }
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(s, &g);
    if (cr != DMPT_OK) {
      if (g) (void)hipGraphDestroy(g);
      rc = cr;
      break;
    }
    if (ee != hipSuccess || hipGraphInstantiate(&gx[stage], g, nullptr, nullptr, 0) != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      rc = fail(c, DMPT_ERR_HIP, "graph capture / instantiation failed");
      break;
    }
    gg[stage] = g;
    int* act = SG.wsi == 0 ? actA : (SG.wsi == 1 ? actB : actC);
    std::vector<int> hact(nsys);
    const int passes0 = total_passes;
    const auto ts = std::chrono::steady_clock::now();
    for (int pass = 0; pass < c->opt.max_newton; ++pass) {
      Range r("dmpt batched replay: stage %d, pass %d", stage, pass);
      if (hipGraphLaunch(gx[stage], s) != hipSuccess) {
        rc = fail(c, DMPT_ERR_HIP, "hipGraphLaunch failed");
        break;
      }
      ++total_passes;
      if (hipMemcpyAsync(hact.data(), act, nsys * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        rc = fail(c, DMPT_ERR_HIP, "batched pass failed");
        break;
      }
      bool any = false;
      int live = 0;
      for (int v : hact) {
        any |= v != 0;
        live += v != 0;
      }
      if (c->log) {
        std::vector<double> hocc_now(nsys), hmu_now((size_t)nsys * J);
        if (hipMemcpy(hocc_now.data(), d_occ, nsys * 8, hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(hmu_now.data(), d_mu, hmu_now.size() * 8, hipMemcpyDeviceToHost) == hipSuccess) {
          double worst = 0.0;
          for (int q = 0; q < nsys; ++q) worst = std::max(worst, hocc_now[q] / (double)Ns[slot_sys[q]]);
          std::fprintf(stderr,
                       "[dmpt] batched stage %d replay %d: %d systems still active, max occ_err/N %.3e, "
                       "%.3f s since the stage began\n",
                       stage, pass + 1, live, worst,
                       std::chrono::duration<double>(std::chrono::steady_clock::now() - ts).count());
        }
      }
      if (!any) break;
    }
    if (c->log)
      std::fprintf(stderr, "[dmpt] batched stage %d (orders 0-%d): %d passes, %.3f s\n", stage, ord,
                   total_passes - passes0,
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - ts).count());
  }
  c->prof_on = prof;
  // results
  std::vector<double> hmu((size_t)nsys * J), hocc(nsys), htr((size_t)nsys * rs);
  std::vector<int> hfl(6 * (size_t)nsys);
  double htally[2] = {0.0, 0.0};
  int hcg[4] = {0, 0, 0, 0};
  if (rc == DMPT_OK) {
    if (hipMemcpy(htally, c->d_tally, sizeof(htally), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(hcg, c->d_cgstat, sizeof(hcg), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(hmu.data(), d_mu, hmu.size() * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(hocc.data(), d_occ, hocc.size() * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(htr.data(), d_tr, htr.size() * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(hfl.data(), d_flags, hfl.size() * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
      rc = fail(c, DMPT_ERR_HIP, "batched result download failed");
  }
  for (int q = 0; q < 3; ++q) {
    if (gx[q]) (void)hipGraphExecDestroy(gx[q]);
    if (gg[q]) (void)hipGraphDestroy(gg[q]);
  }
  cleanup();
  if (rc != DMPT_OK) return rc;
  bool all_done = true, nonfinite = false, floor_acc = false;
  double occ_sum = 0.0;
  for (int slot = 0; slot < nsys; ++slot) {
    const int sy = slot_sys[slot];
    for (int j = 0; j < J; ++j) mus[(size_t)sy * J + j] = hmu[(size_t)slot * J + j];
    if (!hfl[2 * nsys + slot]) all_done = false;
    if (hfl[4 * nsys + slot] == -6) nonfinite = true;
    if (hfl[4 * nsys + slot] == 1) floor_acc = true;
    occ_sum += hocc[slot];
    if (c->log)
      std::fprintf(stderr, "[dmpt] system %d N %ld beta %.4g: passes %d done %d status %d occ_err %.3e mu0 %.15g\n",
                   sy, (long)Ns[sy], betas[sy], hfl[3 * nsys + slot], hfl[2 * nsys + slot],
                   hfl[4 * nsys + slot], hocc[slot], hmu[(size_t)slot * J]);
  }
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->newton_iters = total_passes;
    st->cg_iters_total = hcg[0];
    st->cg_iters_max = hcg[1];
    st->cg_unconverged = hcg[2];
    st->flags = (floor_acc ? DMPT_FLAG_NOISE_FLOOR : 0) | (hcg[2] > 0 ? DMPT_FLAG_CG_FLOOR : 0);
    st->occ_err = occ_sum;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    // products of the members that ran, tallied on the device (useful flops
    // at the padded size of each bucket)
    st->mfma_flops = htally[0];
    st->useful_flops = htally[1];
  }
  if (nonfinite) return fail(c, DMPT_ERR_NONFINITE, "non-finite trace in a batched system");
  if (!all_done) return fail(c, DMPT_ERR_NOCONV, "a batched system did not converge within max_newton");
  return DMPT_OK;
}

dmpt_status dmpt_backward(dmpt_ctx c, int64_t N, const double* H0, double beta, double Ne, int n,
                          const double* mu0, const double* Abar, double* G, dmpt_stats* st) {
  STCHK(check_common(c, N, H0, beta, n));
  if (!Abar) return fail(c, DMPT_ERR_ARG, "Abar is NULL");
  if (!G) return fail(c, DMPT_ERR_ARG, "G is NULL");
  if (!(Ne > 0.0 && Ne < (double)N)) return fail(c, DMPT_ERR_ARG, "Ne must lie in (0, N)");
  if (mu0 && !std::isfinite(*mu0)) return fail(c, DMPT_ERR_ARG, "mu0 must be finite");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, DMPT_ERR_HIP, "hipSetDevice failed");
  ENTER(c);
  const auto t0 = std::chrono::steady_clock::now();
  double mu = mu0 ? *mu0 : NAN;
  int newton = 0;
  double occ = 0.0;
  long cg_fwd = 0;
  int cg_fwd_max = 0;
  double mf = 0.0, uf = 0.0;
  if (!mu0) {
    // canonical mu0 first (order 0); G serves as the scratch P0
    dmpt_stats s0;
    double m[1] = {NAN};
    const dmpt_status r = dmpt_mu_newton(c, N, H0, 0, nullptr, nullptr, nullptr, beta, Ne, n, 0, m, G,
                                         nullptr, nullptr, nullptr, &s0);
    if (r != DMPT_OK) return r;
    mu = m[0];
    newton = s0.newton_iters;
    occ = s0.occ_err;
    cg_fwd = s0.cg_iters_total;
    cg_fwd_max = s0.cg_iters_max;
    mf = s0.mfma_flops;
    uf = s0.useful_flops;
  } else {
    PassIn in{H0, 0, nullptr, nullptr, beta, n, 0, &mu};
    double glo, ghi;
    STCHK(scan_inputs(c, N, in, &glo, &ghi));
    if (beta * std::max(std::fabs(glo - mu), std::fabs(ghi - mu)) >= std::ldexp(1.0, n + 1))
      return fail(c, DMPT_ERR_RANGE, "beta * max|eps - mu| >= 2^(n+1)");
  }
  {
    // Abar must be finite too
    HIPCHK(c, set_values(c->d_flag, 0, 1, nullptr, 0.0, 0, c->stream));
    HIPCHK(c, nonfinite_scan(Abar, N, N, c->d_flag, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->h_int, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->h_int[0]) return fail(c, DMPT_ERR_NONFINITE, "non-finite value in Abar");
  }
  reset_stats(c);
  Call k = make_call(c, N, true);
  if (engine_int8(k.eng)) return fail(c, DMPT_ERR_UNSUPPORTED, "the adjoint has no int8 products");
  const int ck = std::max(1, std::min(c->opt.ckpt_every, n));
  dmpt_status r;
  {
    Range rr("dmpt adjoint: N %lld, %d steps, checkpoints every %d", (long long)N, n, ck);
    r = adjoint_impl<double>(k, H0, beta, mu, n, Abar, G, ck);
  }
  if (r != DMPT_OK) return r;
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->newton_iters = newton;
    st->occ_err = occ;
    st->mu[0] = mu;
    st->cg_iters_total = (int)(c->cg_total + cg_fwd);
    st->cg_iters_max = std::max(c->cg_max, cg_fwd_max);
    st->mfma_flops = c->mfma_flops + mf;
    st->useful_flops = c->useful_flops + uf;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (c->cg_capped) return fail(c, DMPT_ERR_NOCONV, "a linear solve reached max_cg");
  return DMPT_OK;
}

}  // extern "C"
