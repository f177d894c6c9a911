// Host runtime of the CLOMP library: argument validation, workspace layout,
// the static per-iteration schedule, kernel launches, optional HIP-graph
// capture/replay, and the C ABI declared in include/clomp.h.
//
// Scheduling.  Every instance runs exactly k_eff = min(k, m, n) greedy
// iterations, so the whole schedule is known on the host before any launch.
// Instances are grouped by the scan lane-width class (lanes per atom, chosen
// from m) and sorted by k_eff descending inside a class; at iteration t the
// active instances of a class are then a prefix of it, and so are its scan
// tiles and row tiles.  Each phase kernel of iteration t is launched once per
// class over that prefix: no per-iteration tables are needed, and the same
// launch sequence can be captured once and replayed for every batch of the
// same shape.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/clomp.h"
#include "dev_common.h"
#include "kernels.h"

using namespace clomp;

namespace {

constexpr int kMaxKeff = kBlock * 8;        // Adam kernel row capacity
constexpr size_t kAlign = 256;
constexpr int kScanTargetKB = 128;   // default bulk KB streamed per scan WG
constexpr int kPassTargetKB = 256;   // default bulk KB per pass WG (1024 threads)
constexpr int kPassThreadsHost = 1024;
constexpr int kTeamMinRowsDefault = 256;   // larger supports use coefficient teams

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
int round_up_int(int v, int a) { return (v + a - 1) / a * a; }

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Class {
  int lpa = 64;
  int i0 = 0, i1 = 0;                 // sorted-instance range
  std::vector<int> tile_prefix;       // scan tiles of the first q instances
  std::vector<int> row_prefix;        // row tiles of the first q instances
  size_t tile_off = 0, row_off = 0;   // offsets of the arrays in the table blob
  int m_pad_max = 0;
  int kmax = 0;
  int nch = 0;                        // register-kernel vectors per lane (0: LDS kernels)
  std::vector<int> htile_prefix, ctile_prefix;
  int cscan_sub = 4;                  // 64-atom sub-tiles per H-scan tile (256 atoms)
  int nmax = 0;                       // largest n of the class
  int nslice = 1;                     // IHT: most m-slices of any signal of the class
  int slice_floats = 0;               // IHT: largest slice of r (floats, LDS)
  size_t htile_off = 0, ctile_off = 0;
  int team_occ = 0;                   // coefficient-team workgroups per CU at the class's
                                      // largest team LDS (0: no teams)
};

struct Plan {
  std::vector<Inst> insts;            // sorted (class, k_eff desc)
  std::vector<int> keff;              // per sorted instance
  std::vector<Class> classes;
  std::vector<ScanTile> tiles;
  std::vector<RowTile> rows;          // loop row tiles (all instances)
  std::vector<int> qr_list, cg_list;
  std::vector<RowTile> cg_rows;       // row tiles of CGLS instances
  size_t qr_lds = 0;
  int kmax = 0, cg_tmax = 0, cg_mpad_max = 0, cg_lpa = 64;
  bool hflow = false;                 // correlation-update schedule
  bool gflow = false;                 // ... with a shared dictionary: full Gram, no passes
  bool ishared = false;               // IHT / paper mode with a shared dictionary: one
                                      // A^T R contraction per iteration
  size_t off_gf = 0, off_gdg = 0;     // shared Gram matrix and diagonal (workspace)
  bool image = false;                 // CLOMP_FLAG_IMAGE on the shared-dictionary schedule
  size_t off_dct = 0, off_sd = 0, off_x = 0;   // image mode: basis, coefficient images, pixels
  int nbig = 0;                       // sorted instances [0, nbig) use the iterated kernels;
                                      // [nbig, count) run the fused small-signal loop
  std::vector<int> small_list;
  size_t small_lds = 0, off_small = 0;
  std::vector<ScanTile> htiles;       // pass tiles (1024-thread workgroups)
  std::vector<ScanTile> ctiles;       // 64-atom tiles of the H scan
  size_t off_htiles = 0, off_ctiles = 0;
  size_t ws_bytes = 0;
  size_t off_insts = 0, off_tiles = 0, off_rows = 0, off_qr = 0, off_cg = 0, off_cgrows = 0;
  size_t table_bytes = 0;
  std::string sig;                    // shape signature (graph cache key)
  std::vector<int> order;             // sorted position -> input index
};

// Shape of one input instance: everything a plan depends on apart from the
// data pointers.
struct ShapeRec {
  int n, m, k, has_master;
  long long lda, ldam;
  bool operator==(const ShapeRec& o) const {
    return n == o.n && m == o.m && k == o.k && has_master == o.has_master && lda == o.lda &&
           ldam == o.ldam;
  }
};

// The plan of the last batch shape, before its workspace offsets are rebased:
// a batch with the same shapes reuses it and only fills in the pointers.
struct PlanCache {
  bool valid = false;
  int bf16 = -1;
  std::vector<ShapeRec> shapes;
  bool sameA = false;                 // the iterated signals share one A (and master)
  Plan P;
  int scan_kb = 0, pass_kb = 0;
};

struct CachedGraph {
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
};

}  // namespace

struct clomp_ctx {
  int device = 0;
  clomp_params_t params{};
  std::string last_error;
  DevBuf ws, tables;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t staging_free = nullptr;  // last upload from `pinned` finished
  hipEvent_t work_done = nullptr;     // last launch sequence finished
  bool have_work = false;
  hipEvent_t grad_done = nullptr;     // last clomp_grad finished with gwork
  bool have_grad = false;
  int lds_limit = 65536;
  int num_cu = 256;
  DevBuf gwork;
  std::map<std::string, CachedGraph> graphs;
  // profiling (CLOMP_FLAG_PROFILE)
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Rec { int phase; hipEvent_t a, b; };
  std::vector<Rec> recs;
  double scan_bytes = 0.0, pass_bytes = 0.0, fused_bytes = 0.0;
  bool profiling = false;
  bool pass_lds_ok = false;           // dynamic-LDS ceiling raised for pass kernels
  int scan_tile_kb = kScanTargetKB;
  int pass_tile_kb = kPassTargetKB;
  int team_min_rows = kTeamMinRowsDefault;
  int spin_limit = (int)kSpinLimitDefault;   // polls of a team wait before the watchdog
  std::map<long long, int> team_occ;  // team workgroups per CU by (dtype, lpa, method, LDS)
  int rscan_min_t = 1;                // shared dictionary: A^T R scan from this support size
  int shared_min_tiles = 0;           // IHT / paper mode: contraction tiles needed for the
                                      // shared gradient (0: half the compute units)
  int last_scan_kb = kScanTargetKB, last_pass_kb = kPassTargetKB;   // of the last solve
  std::map<std::string, int> tuned;   // autotuned tile size per size class
  std::string arch = "unknown";       // device architecture (first field of its name)
  PlanCache pcache;
};

namespace {

// Restores the caller's current device on every return path.
struct DeviceGuard {
  int prev = 0;
  DeviceGuard() { (void)hipGetDevice(&prev); }
  ~DeviceGuard() { (void)hipSetDevice(prev); }
};

clomp_status_t fail(clomp_ctx* h, clomp_status_t s, const char* fmt, ...) {
  if (h) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    h->last_error = buf;
  }
  return s;
}

clomp_status_t hip_fail(clomp_ctx* h, hipError_t e, const char* what) {
  return fail(h, CLOMP_DEVICE_ERROR, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                         \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return hip_fail(h, e_, what); \
  } while (0)

clomp_status_t check_params(clomp_ctx* h, const clomp_params_t* p) {
  if (!p) return fail(h, CLOMP_INVALID_ARGUMENT, "params is NULL");
  if (p->method != CLOMP_METHOD_CLOMP && p->method != CLOMP_METHOD_OMP &&
      p->method != CLOMP_METHOD_IHT && p->method != CLOMP_METHOD_PAPER)
    return fail(h, CLOMP_INVALID_ARGUMENT, "unknown method %d", p->method);
  if ((p->method == CLOMP_METHOD_IHT || p->method == CLOMP_METHOD_PAPER) && p->inner_steps < 1)
    return fail(h, CLOMP_INVALID_ARGUMENT, "IHT and paper mode need inner_steps (iterations) >= 1");
  if (p->method == CLOMP_METHOD_PAPER && !(p->select_threshold > 0.f && p->select_threshold <= 1.f))
    return fail(h, CLOMP_INVALID_ARGUMENT, "select_threshold must lie in (0, 1]");
  if (!(p->prior_tv >= 0.f && p->prior_tv <= 3.402823466e38f))
    return fail(h, CLOMP_INVALID_ARGUMENT, "prior_tv must be finite and >= 0");
  if (p->prior_tv > 0.f && p->method != CLOMP_METHOD_CLOMP)
    return fail(h, CLOMP_NOT_SUPPORTED, "the total-variation prior is served for CLOMP only");
  if (p->inner_steps < 0 || p->inner_steps > 100000)
    return fail(h, CLOMP_INVALID_ARGUMENT, "inner_steps %d out of range", p->inner_steps);
  if (!(p->beta1 >= 0.f && p->beta1 < 1.f) || !(p->beta2 >= 0.f && p->beta2 < 1.f))
    return fail(h, CLOMP_INVALID_ARGUMENT, "Adam betas must lie in [0, 1)");
  if (!(p->lr_rel >= 0.f) || !(p->eps_rel > 0.f))
    return fail(h, CLOMP_INVALID_ARGUMENT, "lr_rel must be >= 0 and eps_rel > 0");
  if (p->refine_iters < 0 || !(p->refine_tol >= 0.f))
    return fail(h, CLOMP_INVALID_ARGUMENT, "refine_iters/refine_tol must be >= 0");
  if (p->resid_tol != 0.f)
    return fail(h, CLOMP_NOT_SUPPORTED, "resid_tol != 0 (early stopping) is not served");
  if ((p->flags & CLOMP_FLAG_NO_REFINE) &&
      !(p->method == CLOMP_METHOD_CLOMP || p->method == CLOMP_METHOD_OMP))
    return fail(h, CLOMP_NOT_SUPPORTED, "CLOMP_FLAG_NO_REFINE is served for CLOMP and OMP");
  if ((p->flags & CLOMP_FLAG_NO_REFINE) && p->prior_tv > 0.f && !(p->flags & CLOMP_FLAG_IMAGE))
    return fail(h, CLOMP_NOT_SUPPORTED, "CLOMP_FLAG_NO_REFINE is not served with the prior");
  if (!(p->prior_lv >= 0.f && p->prior_lv <= 3.402823466e38f))
    return fail(h, CLOMP_INVALID_ARGUMENT, "prior_lv must be finite and >= 0");
  if (p->prior_lv > 0.f && !(p->flags & CLOMP_FLAG_IMAGE))
    return fail(h, CLOMP_NOT_SUPPORTED, "the local-variation prior needs CLOMP_FLAG_IMAGE");
  if (p->flags & CLOMP_FLAG_IMAGE) {
    if (p->method != CLOMP_METHOD_CLOMP)
      return fail(h, CLOMP_NOT_SUPPORTED, "CLOMP_FLAG_IMAGE is served for CLOMP");
    if (p->flags & (CLOMP_FLAG_NO_SHARED_GRAM | CLOMP_FLAG_RESIDUAL_FLOW))
      return fail(h, CLOMP_NOT_SUPPORTED,
                  "CLOMP_FLAG_IMAGE runs the shared-dictionary schedule only");
  }
  return CLOMP_OK;
}

// The columns of an image (CLOMP_FLAG_IMAGE): one dictionary for all, the
// same k, sizes within the image kernels' limits.
clomp_status_t check_image_batch(clomp_ctx* h, const clomp_instance_t* inst, int32_t count) {
  if (count <= 0) return CLOMP_OK;
  const clomp_instance_t& a = inst[0];
  for (int i = 1; i < count; ++i) {
    const clomp_instance_t& b = inst[i];
    if (!(a.A == b.A && a.lda == b.lda && a.n == b.n && a.m == b.m && a.k == b.k &&
          a.A_master == b.A_master && a.lda_master == b.lda_master))
      return fail(h, CLOMP_NOT_SUPPORTED,
                  "CLOMP_FLAG_IMAGE: instance %d differs from instance 0 in A, its layout, its "
                  "master or k (the columns of an image share all of them)", i);
  }
  if (a.n > kImageMaxN)
    return fail(h, CLOMP_NOT_SUPPORTED, "CLOMP_FLAG_IMAGE: n = %d exceeds %d", a.n, kImageMaxN);
  if (std::min(a.k, std::min(a.m, a.n)) > kImageMaxK)
    return fail(h, CLOMP_NOT_SUPPORTED, "CLOMP_FLAG_IMAGE: k_eff exceeds %d", kImageMaxK);
  return CLOMP_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

clomp_status_t check_batch_impl(clomp_ctx* h, const clomp_instance_t* inst, int32_t count,
                                int32_t a_dtype) {
  if (count < 0) return fail(h, CLOMP_INVALID_ARGUMENT, "count < 0");
  if (count == 0) return CLOMP_OK;
  if (!inst) return fail(h, CLOMP_INVALID_ARGUMENT, "inst is NULL");
  if (a_dtype == CLOMP_F64)
    return fail(h, CLOMP_NOT_SUPPORTED, "F64 bulk matrices are not served by the solver");
  if (a_dtype != CLOMP_F32 && a_dtype != CLOMP_BF16)
    return fail(h, CLOMP_INVALID_ARGUMENT, "unknown dtype %d", a_dtype);
  const int q = (a_dtype == CLOMP_BF16) ? 8 : 4;
  for (int i = 0; i < count; ++i) {
    const clomp_instance_t& I = inst[i];
    if (I.n <= 0 || I.m <= 0 || I.k <= 0)
      return fail(h, CLOMP_INVALID_ARGUMENT, "instance %d: n, m, k must be positive", i);
    if (I.lda < I.m || I.lda % q)
      return fail(h, CLOMP_INVALID_ARGUMENT,
                  "instance %d: lda must be >= m and a multiple of %d", i, q);
    if (!I.A || !aligned16(I.A))
      return fail(h, CLOMP_INVALID_ARGUMENT, "instance %d: A is NULL or not 16-byte aligned", i);
    if (!I.y || !I.x || !I.support || !I.n_selected || !I.resid_norm || !I.status)
      return fail(h, CLOMP_INVALID_ARGUMENT, "instance %d: a required pointer is NULL", i);
    if (a_dtype == CLOMP_BF16 && !I.A_master)
      return fail(h, CLOMP_INVALID_ARGUMENT, "instance %d: BF16 bulk needs A_master", i);
    if (I.A_master) {
      const int64_t ldm = I.lda_master ? I.lda_master : I.lda;
      if (ldm < I.m || ldm % 4 || !aligned16(I.A_master))
        return fail(h, CLOMP_INVALID_ARGUMENT,
                    "instance %d: A_master needs lda_master >= m, a multiple of 4, 16-byte "
                    "alignment", i);
    }
    const int keff = std::min(I.k, std::min(I.m, I.n));
    if (keff > kMaxKeff)
      return fail(h, CLOMP_NOT_SUPPORTED, "instance %d: k_eff = %d exceeds %d", i, keff,
                  kMaxKeff);
  }
  return CLOMP_OK;
}

// Lanes per atom: the most (up to 64) that still give every lane at least
// 16 vectors of the column, so the per-atom reduction is amortised.
int pick_lpa(int m, int vw) {
  const int nvec = (m + vw - 1) / vw;
  int lpa = 64;
  while (lpa > 4 && lpa * 16 > nvec) lpa >>= 1;
  return lpa;
}

// Whether the iterated signals [0, nbig) of a sorted batch all name the same
// dictionary (pointer, layout and master): the condition of the shared-
// dictionary schedules, which read A from the first signal only.
bool same_dictionary(const clomp_instance_t* inst, const std::vector<int>& order, int nbig) {
  if (nbig < 2) return false;
  const clomp_instance_t& a = inst[order[0]];
  for (int s = 1; s < nbig; ++s) {
    const clomp_instance_t& b = inst[order[s]];
    if (!(a.A == b.A && a.lda == b.lda && a.n == b.n && a.m == b.m &&
          a.A_master == b.A_master && a.lda_master == b.lda_master))
      return false;
  }
  return true;
}

// Coefficient-team workgroups one CU can hold (cached per launch shape).
int team_occupancy(clomp_ctx* h, int bf16, int lpa, int omp, size_t lds) {
  const long long key = ((long long)lds << 16) | (bf16 << 12) | (omp << 8) | lpa;
  auto it = h->team_occ.find(key);
  if (it != h->team_occ.end()) return it->second;
  const int nb = coef_team_blocks_per_cu(bf16, lpa, omp, lds);
  h->team_occ[key] = nb;
  return nb;
}

// Build the plan (host tables + workspace layout) for one batch.
void build_plan(clomp_ctx* h, const clomp_instance_t* inst, int count, int bf16, Plan& P,
                int scan_kb, int pass_kb) {
  const clomp_params_t& prm = h->params;
  const bool omp = prm.method == CLOMP_METHOD_OMP;
  // IHT and paper-mode CLOMP iterate over dense coefficients: no Gram matrix,
  // no fused loop, no correlation-update schedule
  const bool paper = prm.method == CLOMP_METHOD_PAPER;
  const bool iht = prm.method == CLOMP_METHOD_IHT || paper;
  const int vw = bf16 ? 8 : 4;
  const size_t esize = bf16 ? 2 : 4;
  char sigbuf[96];
  P.sig.clear();
  // order: by class (lpa desc), then k_eff desc, then input index
  std::vector<int> order(count);
  std::vector<int> lpa(count), keff(count);
  std::vector<char> fused(count, 0);
  const bool image = (prm.flags & CLOMP_FLAG_IMAGE) != 0;
  // (the columns of an image iterate in lock-step: none runs the fused loop)
  const bool allow_fused = !(prm.flags & CLOMP_FLAG_NO_FUSED_SMALL) && !iht && !image;
  for (int i = 0; i < count; ++i) {
    order[i] = i;
    lpa[i] = pick_lpa(inst[i].m, vw);
    keff[i] = std::min(inst[i].k, std::min(inst[i].m, inst[i].n));
    // fused loop: k_eff within one wave and the signal's LDS image within the
    // ceiling next to the kernel's 1.3 KB of static LDS
    fused[i] = allow_fused && keff[i] <= kSmallMaxK &&
               small_lds_bytes(inst[i].n, inst[i].m, keff[i]) + 2048 <= (size_t)h->lds_limit;
  }
  // fused signals last; the rest by lane-width class, then k_eff descending
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (fused[a] != fused[b]) return fused[a] < fused[b];
    if (lpa[a] != lpa[b]) return lpa[a] > lpa[b];
    return keff[a] > keff[b];
  });
  P.nbig = 0;
  while (P.nbig < count && !fused[order[P.nbig]]) ++P.nbig;
  P.order = order;
  const int qr_limit_floats = ((int)std::min<size_t>((size_t)h->lds_limit, 96 * 1024) - 1024) / 4;
  {
    // correlation-update schedule: H within budget, the pass kernel's staged
    // vector within LDS next to its 33 KB of static LDS
    size_t hbytes = 0;
    int mpad_max = 0;
    for (int s = 0; s < P.nbig; ++s) {
      const int i = order[s];
      hbytes += sizeof(float) * (size_t)round_up_int(inst[i].n, 64) * keff[i];
      mpad_max = std::max(mpad_max, round_up_int(inst[i].m, 8));
    }
    const bool fits = h->pass_lds_ok &&
                      (size_t)mpad_max * 4 + 34 * 1024 <= (size_t)h->lds_limit &&
                      hbytes <= (size_t)16 << 30;
    const uint32_t fl = prm.flags;
    // shared dictionary: every iterated signal has the same A (pointer, layout,
    // master) and the full Gram matrix fits in 4 GB; an iteration then reads
    // columns of A^T A instead of streaming A
    // (an image of one column keeps the shared-dictionary schedule too)
    const bool sameA = !(fl & CLOMP_FLAG_NO_SHARED_GRAM) &&
                       (same_dictionary(inst, order, P.nbig) || (image && P.nbig == 1));
    // IHT / paper mode: the batch's gradient as one contraction pays only when
    // it has enough 128 x 128 output tiles to fill the device; a small batch
    // (a 256 x 256 image: four tiles) scans per signal instead
    if (iht && sameA) {
      const long long tiles =
          (long long)((inst[order[0]].n + 127) / 128) * ((P.nbig + 127) / 128);
      const int need = h->shared_min_tiles > 0 ? h->shared_min_tiles : std::max(1, h->num_cu / 2);
      P.ishared = tiles >= need;
    }
    bool shared = sameA && !iht && !(fl & CLOMP_FLAG_RESIDUAL_FLOW);
    if (shared) {
      const size_t l = (size_t)round_up_int(inst[order[0]].n, 256);
      shared = l * l * sizeof(float) <= ((size_t)4 << 30);
    }
    P.gflow = shared;
    // measured faster than the residual schedule on every iterated workload
    // (the pass and the coefficient update share one launch per iteration)
    P.hflow = P.nbig > 0 && (P.gflow || (fits && !(fl & CLOMP_FLAG_RESIDUAL_FLOW) && !iht));
  }
  snprintf(sigbuf, sizeof sigbuf, "h%d;g%d;i%d;f%d;", (int)P.hflow, (int)P.gflow, (int)P.ishared,
           count - P.nbig);
  P.sig += sigbuf;
  P.insts.resize(count);
  P.keff.resize(count);
  P.kmax = 0;
  size_t ws = 0;
  if (P.gflow) {
    const size_t l = (size_t)round_up_int(inst[order[0]].n, 256);
    P.off_gf = ws;
    ws = align_up(ws + sizeof(float) * l * l, kAlign);
    P.off_gdg = ws;
    ws = align_up(ws + sizeof(float) * l, kAlign);
  }
  P.image = image && P.gflow;
  if (P.image) {
    // the DCT-II synthesis basis (n columns of ldh), two dense coefficient
    // images (ping-pong by Adam step) and, with the local variation, the
    // pixel image
    const size_t l = (size_t)round_up_int(inst[order[0]].n, 256);
    P.off_dct = ws;
    ws = align_up(ws + sizeof(float) * l * inst[order[0]].n, kAlign);
    P.off_sd = ws;
    ws = align_up(ws + sizeof(float) * 2 * l * count, kAlign);
    P.off_x = ws;
    ws = align_up(ws + sizeof(float) * l * count, kAlign);
  }
  snprintf(sigbuf, sizeof sigbuf, "d%d;m%d;T%d;s%d;p%d;w%d;r%d;", bf16, prm.method,
           prm.inner_steps, scan_kb, pass_kb, h->team_min_rows, h->rscan_min_t);
  P.sig += sigbuf;
  for (int s = 0; s < count; ++s) {
    const int i = order[s];
    const clomp_instance_t& src = inst[i];
    Inst d;
    memset(&d, 0, sizeof d);
    d.A = src.A;
    d.Am = src.A_master ? src.A_master : reinterpret_cast<const float*>(src.A);
    d.ldam = src.A_master ? (src.lda_master ? src.lda_master : src.lda) : src.lda;
    d.y = src.y;
    d.x = src.x;
    d.support = src.support;
    d.nsel = src.n_selected;
    d.rnorm = src.resid_norm;
    d.status = src.status;
    d.lda = src.lda;
    d.col = i;
    d.n = src.n;
    d.m = src.m;
    d.k = src.k;
    d.k_eff = keff[i];
    d.ldg = round_up_int(d.k_eff, 4);
    d.m_pad = round_up_int(d.m, 8);
    d.n_rowtiles = (d.m + 63) / 64;
    // with the prior the refinement's QR holds k_eff stacked rows more
    d.tvw = (prm.prior_tv > 0.f) ? 2.f * prm.prior_tv / (float)d.n : 0.f;
    const size_t qr_rows = (size_t)d.m + (d.tvw != 0.f ? d.k_eff : 0);
    // (LDS: the columns, the right-hand side and four vectors of k_eff)
    const bool use_qr = qr_rows * d.k_eff + qr_rows + 4 * d.k_eff <= (size_t)qr_limit_floats;
    d.cg_slot = use_qr ? -1 : 0;
    // workspace offsets (relative; rebased after allocation)
    auto take = [&](size_t bytes) {
      const size_t o = ws;
      ws = align_up(ws + bytes, kAlign);
      return o;
    };
    const size_t o_r = take(sizeof(float) * 2 * d.m_pad);
    const size_t o_G = iht ? 0 : take(sizeof(float) * (size_t)d.k_eff * d.ldg);
    const size_t o_b = take(sizeof(float) * d.k_eff);
    const size_t o_s = take(sizeof(float) * d.k_eff);
    const size_t o_mo = take(sizeof(float) * d.k_eff);
    const size_t o_ve = take(sizeof(float) * d.k_eff);
    const size_t o_xf = take(sizeof(float) * d.k_eff);
    const size_t o_z = take(sizeof(float) * d.k_eff);
    const size_t o_L = omp ? take(sizeof(float) * (size_t)d.k_eff * d.ldg) : 0;
    const size_t o_cg = use_qr ? 0 : take(sizeof(float) * (3 * (size_t)d.m_pad + 3 * d.k_eff));
    size_t o_c0 = 0, o_H = 0, o_dg = 0, o_team = 0, o_gb = 0, o_sf = 0, o_md = 0, o_vd = 0;
    const bool hf = P.hflow && s < P.nbig;
    d.nslice = 1;
    if (iht) {
      d.ldh = round_up_int(d.n, 256);
      // (a shared dictionary's gradient is one contraction: no slices)
      d.nslice = P.ishared ? 1 : std::max(1, (d.m_pad + kIhtSliceFloats - 1) / kIhtSliceFloats);
      o_c0 = take(sizeof(float) * d.ldh);
      o_gb = take(sizeof(float) * d.ldh * d.nslice);
      o_sf = take(sizeof(float) * d.ldh);
      if (paper) {
        o_md = take(sizeof(float) * d.ldh);
        o_vd = take(sizeof(float) * d.ldh);
      }
    }
    if (hf) {
      d.ldh = round_up_int(d.n, 256);
      o_c0 = take(sizeof(float) * d.ldh);
      // the shared-dictionary schedule keeps one diagonal and no H
      o_dg = P.gflow ? P.off_gdg : take(sizeof(float) * d.ldh);
      o_H = P.gflow ? 0 : take(sizeof(float) * (size_t)d.ldh * d.k_eff);
      o_team = take(sizeof(unsigned long long) * (2 * (size_t)d.k_eff + 2 * kTeamMax));
    }
    const size_t o_np = take(sizeof(double) * d.n_rowtiles);
    const size_t o_qp = take(sizeof(float) * d.n_rowtiles);
    const size_t o_key = take(2 * sizeof(unsigned long long));
    const size_t o_bm = take(sizeof(unsigned) * ((d.n + 31) / 32));
    const size_t o_st = take(sizeof(InstState));
    // store offsets in the pointer fields for now (+1 so 0 means "absent")
    d.r = (float*)(o_r + 1);
    d.G = iht ? nullptr : (float*)(o_G + 1);
    d.b = (float*)(o_b + 1);
    d.s = (float*)(o_s + 1);
    d.mo = (float*)(o_mo + 1);
    d.ve = (float*)(o_ve + 1);
    d.xf = (float*)(o_xf + 1);
    d.z = (float*)(o_z + 1);
    d.Linv = omp ? (float*)(o_L + 1) : nullptr;
    d.cg = use_qr ? nullptr : (float*)(o_cg + 1);
    d.c0 = (hf || iht) ? (float*)(o_c0 + 1) : nullptr;
    d.gbuf = iht ? (float*)(o_gb + 1) : nullptr;
    d.sfull = iht ? (float*)(o_sf + 1) : nullptr;
    d.mden = paper ? (float*)(o_md + 1) : nullptr;
    d.vden = paper ? (float*)(o_vd + 1) : nullptr;
    d.dg = hf ? (float*)(o_dg + 1) : nullptr;
    d.team = hf ? (unsigned long long*)(o_team + 1) : nullptr;
    d.H = (hf && !P.gflow) ? (float*)(o_H + 1) : nullptr;
    d.Gf = (hf && P.gflow) ? (const float*)(P.off_gf + 1) : nullptr;
    d.npart = (double*)(o_np + 1);
    d.qpart = (float*)(o_qp + 1);
    d.key = (unsigned long long*)(o_key + 1);
    d.bitmap = (unsigned*)(o_bm + 1);
    d.st = (InstState*)(o_st + 1);
    P.insts[s] = d;
    P.keff[s] = d.k_eff;
    P.kmax = std::max(P.kmax, d.k_eff);
    snprintf(sigbuf, sizeof sigbuf, "%d,%d,%d,%lld,%lld|", d.n, d.m, d.k, (long long)d.lda,
             (long long)d.ldam);
    P.sig += sigbuf;
  }
  P.ws_bytes = ws;

  // classes, scan tiles, row tiles
  P.classes.clear();
  P.tiles.clear();
  P.rows.clear();
  for (int s = 0; s < P.nbig;) {
    Class c;
    c.lpa = lpa[order[s]];
    c.i0 = s;
    while (s < P.nbig && lpa[order[s]] == c.lpa) ++s;
    c.i1 = s;
    c.tile_prefix.push_back(0);
    c.row_prefix.push_back(0);
    c.tile_off = P.tiles.size();
    c.row_off = P.rows.size();
    const int ng = kBlock / c.lpa;
    // H-scan tiles of 256 atoms (the scan kernel chooses how many waves share
    // a tile from the number of tiles of each launch)
    c.cscan_sub = 4;
    for (int q = c.i0; q < c.i1; ++q) {
      const Inst& d = P.insts[q];
      // an IHT gradient workgroup streams one slice of m of each atom of its
      // tile, so the tile holds nslice times the atoms
      const size_t atom_bytes = (size_t)d.m_pad * esize / d.nslice;
      int apg = (int)std::max<size_t>(1, (size_t)scan_kb * 1024 / (atom_bytes * ng));
      const int apt = ng * apg;
      for (int j0 = 0; j0 < d.n; j0 += apt) P.tiles.push_back({q, j0, std::min(d.n, j0 + apt), 0});
      c.tile_prefix.push_back((int)(P.tiles.size() - c.tile_off));
      for (int tt = 0; tt < d.n_rowtiles; ++tt)
        P.rows.push_back({q, tt * 64, std::min(d.m, tt * 64 + 64), tt});
      c.row_prefix.push_back((int)(P.rows.size() - c.row_off));
      if (P.hflow) {
        if (c.htile_prefix.empty()) {
          c.htile_prefix.push_back(0);
          c.ctile_prefix.push_back(0);
          c.htile_off = P.htiles.size();
          c.ctile_off = P.ctiles.size();
        }
        const int hng = kPassThreadsHost / c.lpa;
        const int happ = (int)std::max<size_t>(1, (size_t)pass_kb * 1024 / (atom_bytes * hng));
        const int hapt = hng * happ;
        for (int j0 = 0; j0 < d.n; j0 += hapt)
          P.htiles.push_back({q, j0, std::min(d.n, j0 + hapt), 0});
        c.htile_prefix.push_back((int)(P.htiles.size() - c.htile_off));
        for (int j0 = 0; j0 < d.n; j0 += 64 * c.cscan_sub)
          P.ctiles.push_back({q, j0, std::min(d.n, j0 + 64 * c.cscan_sub), 0});
        c.ctile_prefix.push_back((int)(P.ctiles.size() - c.ctile_off));
      }
      c.m_pad_max = std::max(c.m_pad_max, d.m_pad);
      c.kmax = std::max(c.kmax, d.k_eff);
      c.nmax = std::max(c.nmax, d.n);
      {
        const int nvec = (d.m + vw - 1) / vw;
        const int sv = (nvec + d.nslice - 1) / d.nslice;
        c.nslice = std::max(c.nslice, d.nslice);
        c.slice_floats = std::max(c.slice_floats, sv * vw);
      }
    }
    // register kernels when every lane's share of the longest column fits in
    // 64 registers
    {
      const int nvec = (c.m_pad_max + vw - 1) / vw;
      const int per_lane = (nvec + c.lpa - 1) / c.lpa;
      int nch = 1;
      while (nch < per_lane) nch <<= 1;
      c.nch = (nch * vw <= 64) ? nch : 0;   // at most 64 floats of r per lane
    }
    // coefficient teams (correlation-update schedule): the occupancy query
    // runs here, before any launch or capture, at the largest LDS a team
    // launch of the class can ask for (occupancy does not grow with LDS)
    if (P.hflow && c.kmax > h->team_min_rows) {
      const bool omp = prm.method == CLOMP_METHOD_OMP;
      const size_t t1 = (size_t)c.kmax;
      size_t tl = std::max((size_t)c.m_pad_max, (omp ? 6 : 1) * t1);
      if (!omp && t1 > 256) tl = std::max(tl, (size_t)kSplitLdsFloats);
      tl = std::max(tl, t1 + 4 + 32);
      c.team_occ = team_occupancy(h, bf16, c.lpa, omp ? 1 : 0, tl * sizeof(float));
    }
    P.classes.push_back(std::move(c));
  }
  // fused signals: row tiles (for the norm) and the launch list
  P.small_list.clear();
  P.small_lds = 0;
  for (int q = P.nbig; q < count; ++q) {
    const Inst& d = P.insts[q];
    for (int tt = 0; tt < d.n_rowtiles; ++tt)
      P.rows.push_back({q, tt * 64, std::min(d.m, tt * 64 + 64), tt});
    P.small_list.push_back(q);
    P.small_lds = std::max(P.small_lds, small_lds_bytes(d.n, d.m, d.k_eff));
  }
  // refinement lists
  P.qr_list.clear();
  P.cg_list.clear();
  P.cg_rows.clear();
  P.qr_lds = 0;
  P.cg_tmax = 0;
  P.cg_mpad_max = 0;
  for (int q = 0; q < count; ++q) {
    const Inst& d = P.insts[q];
    if (d.cg_slot < 0) {
      P.qr_list.push_back(q);
      const size_t qr_rows = (size_t)d.m + (d.tvw != 0.f ? d.k_eff : 0);
      P.qr_lds = std::max(P.qr_lds, sizeof(float) * (qr_rows * d.k_eff + qr_rows + 4 * d.k_eff));
    } else {
      P.insts[q].cg_slot = (int)P.cg_list.size();
      P.cg_list.push_back(q);
      for (int tt = 0; tt < d.n_rowtiles; ++tt)
        P.cg_rows.push_back({q, tt * 64, std::min(d.m, tt * 64 + 64), tt});
      P.cg_tmax = std::max(P.cg_tmax, d.k_eff);
      P.cg_mpad_max = std::max(P.cg_mpad_max, d.m_pad);
    }
  }
  int mmax = 0;
  for (int q : P.cg_list) mmax = std::max(mmax, P.insts[q].m);
  P.cg_lpa = pick_lpa(std::max(mmax, 1), 4);
  // table blob layout
  size_t off = 0;
  auto place = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, kAlign);
    return o;
  };
  P.off_insts = place(sizeof(Inst) * count);
  P.off_tiles = place(sizeof(ScanTile) * P.tiles.size());
  P.off_rows = place(sizeof(RowTile) * P.rows.size());
  P.off_qr = place(sizeof(int) * P.qr_list.size());
  P.off_cg = place(sizeof(int) * P.cg_list.size());
  P.off_cgrows = place(sizeof(RowTile) * P.cg_rows.size());
  P.off_htiles = place(sizeof(ScanTile) * P.htiles.size());
  P.off_ctiles = place(sizeof(ScanTile) * P.ctiles.size());
  P.off_small = place(sizeof(int) * P.small_list.size());
  P.table_bytes = std::max<size_t>(off, kAlign);
}

clomp_status_t ensure(clomp_ctx* h, DevBuf& b, size_t bytes, bool* grew) {
  if (grew) *grew = false;
  if (b.bytes >= bytes) return CLOMP_OK;
  if (b.p) {
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  const size_t want = align_up(bytes + bytes / 8, 1 << 20);
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(h, CLOMP_OUT_OF_MEMORY, "workspace allocation of %zu bytes failed", want);
  }
  b.bytes = want;
  if (grew) *grew = true;
  return CLOMP_OK;
}

void drop_graphs(clomp_ctx* h) {
  for (auto& kv : h->graphs) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
  }
  h->graphs.clear();
}

enum Phase {
  PH_SCAN = 0, PH_GRAM, PH_COEF, PH_RESID, PH_REFINE, PH_NORM, PH_INIT, PH_PASS, PH_FUSED
};

hipEvent_t pool_event(clomp_ctx* h) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_used++];
}

// Time one phase when profiling.  Single-kernel phases hand both events to
// the launch (recorded by the kernel's own dispatch); multi-kernel phases are
// bracketed by events recorded on the stream.
struct PhaseScope {
  clomp_ctx* h;
  int phase;
  hipStream_t st;
  bool single;
  hipEvent_t a = nullptr, b = nullptr;
  PhaseScope(clomp_ctx* h_, int p, hipStream_t s, bool single_kernel = true)
      : h(h_), phase(p), st(s), single(single_kernel) {
    if (!h->profiling) return;
    a = pool_event(h);
    b = pool_event(h);
    if (!a || !b) {
      a = b = nullptr;
      return;
    }
    if (single)
      set_launch_events(a, b);
    else
      (void)hipEventRecord(a, st);
  }
  ~PhaseScope() {
    if (!a) return;
    if (single)
      set_launch_events(nullptr, nullptr);
    else
      (void)hipEventRecord(b, st);
    h->recs.push_back({phase, a, b});
  }
};

// Greedy loop of the correlation-update schedule.
clomp_status_t launch_hflow(clomp_ctx* h, const Plan& P, int bf16, hipStream_t st) {
  const clomp_params_t& prm = h->params;
  const bool omp = prm.method == CLOMP_METHOD_OMP;
  char* tb = reinterpret_cast<char*>(h->tables.p);
  const Inst* d_insts = reinterpret_cast<const Inst*>(tb + P.off_insts);
  const ScanTile* d_htiles = reinterpret_cast<const ScanTile*>(tb + P.off_htiles);
  const ScanTile* d_ctiles = reinterpret_cast<const ScanTile*>(tb + P.off_ctiles);
  const RowTile* d_rows = reinterpret_cast<const RowTile*>(tb + P.off_rows);
  const double esz = bf16 ? 2.0 : 4.0;
  auto nactive = [&](const Class& c, int t) {
    int q = 0;
    while (c.i0 + q < c.i1 && P.keff[c.i0 + q] > t) ++q;
    return q;
  };
  if (P.gflow) {
    // shared dictionary: Gf = A^T A, every c0 = A^T y and the diagonal once,
    // then the first argmax from c0
    char* wsb = reinterpret_cast<char*>(h->ws.p);
    {
      PhaseScope ps(h, PH_SCAN, st);
      HIP_TRY(launch_shared_gram(bf16, d_insts, P.nbig, P.insts[0].n,
                                 reinterpret_cast<float*>(wsb + P.off_gf),
                                 reinterpret_cast<float*>(wsb + P.off_gdg), st),
              "shared gram");
    }
    for (const Class& c : P.classes) {
      const int nall = c.i1 - c.i0;
      PhaseScope ps(h, PH_SCAN, st);
      // r = y at the start: the first scan is c0's argmax either way
      if (h->rscan_min_t <= 1)
        HIP_TRY(launch_shared_rscan(bf16, d_insts + c.i0, nall, P.insts[c.i0].n, 0, st), "rscan");
      else
        HIP_TRY(launch_cscan(d_insts, d_ctiles + c.ctile_off, c.ctile_prefix[nall], 0, st),
                "cscan");
    }
  }
  // c0 = A^T y and the first argmax
  for (const Class& c : P.classes) {
    if (P.gflow) break;
    const int nall = c.i1 - c.i0;
    const size_t lds = (size_t)c.m_pad_max * sizeof(float);
    PhaseScope ps(h, PH_SCAN, st);
    HIP_TRY(launch_ypass(bf16, c.lpa, d_insts, d_htiles + c.htile_off, c.htile_prefix[nall], lds,
                         st),
            "ypass");
    if (h->profiling)
      for (int q = c.i0; q < c.i1; ++q)
        h->scan_bytes += (double)P.insts[q].m * P.insts[q].n * esz + 4.0 * P.insts[q].m;
  }
  for (int t = 0; t < P.kmax; ++t) {
    for (const Class& c : P.classes) {
      if (c.kmax <= t) continue;
      const int nact = nactive(c, t);
      const int nnext = nactive(c, t + 1);
      {
        // selection record, Gram column gathered from H, coefficient update of
        // iteration t, fused with h_t = A^T a_{S_t} for the instances that
        // select again
        const size_t t1 = (size_t)t + 1;
        // a team of W blocks per signal for supports beyond the register tile,
        // while the teams stay far below the CU count (all resident at once)
        size_t lds = (size_t)c.m_pad_max * sizeof(float);
        lds = std::max(lds, (omp ? 6 : 1) * t1 * sizeof(float));
        // split-row Adam (256 < t+1 <= 1024): s and the partial sums
        if (!omp && t1 > 256 && t1 <= 1024)
          lds = std::max(lds, (size_t)kSplitLdsFloats * sizeof(float));
        int W = 1;
        if (t1 > (size_t)h->team_min_rows) {
          const int want = (int)((t1 + 15) / 16);
          const size_t tlds = std::max(lds, (t1 + 4 + 32) * sizeof(float));
          // members wait for one another, so all of them must be resident at
          // once: the occupancy query (taken when the plan was built, never
          // inside a launch sequence that may be captured) must admit a member
          // per CU, and the teams of all active signals stay below the CU
          // count; otherwise the single-workgroup update runs
          if (want <= kTeamMax && (long long)want * nact <= h->num_cu - 8 && c.team_occ >= 1) {
            W = want;
            lds = tlds;
          }
        }
        if (P.image) {
          // the columns of one image: selection record, then every Adam step
          // as one launch over all columns (the priors couple neighbours)
          char* wsb = reinterpret_cast<char*>(h->ws.p);
          const long long ldd = round_up_int(P.insts[0].n, 256);
          const float* Dm = reinterpret_cast<const float*>(wsb + P.off_dct);
          float* Sd = reinterpret_cast<float*>(wsb + P.off_sd);
          float* X = reinterpret_cast<float*>(wsb + P.off_x);
          const int Wc = c.i1 - c.i0;   // one class: every column
          const float htv = 2.f * prm.prior_tv / (float)Wc;
          {
            PhaseScope ps(h, PH_COEF, st);
            HIP_TRY(launch_image_record(d_insts + c.i0, Wc, t, prm.lr_rel, prm.eps_rel, st),
                    "image record");
          }
          for (int tau = 0; tau < prm.inner_steps; ++tau) {
            const int step = t * prm.inner_steps + tau + 1;
            const float* cur = Sd + (long long)((step - 1) & 1) * ldd * Wc;
            float* nxt = Sd + (long long)(step & 1) * ldd * Wc;
            if (prm.prior_lv > 0.f) {
              PhaseScope ps(h, PH_COEF, st);
              HIP_TRY(launch_image_synth(d_insts + c.i0, Wc, t + 1, Dm, ldd, X, st),
                      "image synth");
            }
            PhaseScope ps(h, PH_COEF, st);
            HIP_TRY(launch_image_step(d_insts + c.i0, Wc, P.insts[0].n, t, step, prm.beta1,
                                      prm.beta2, htv, prm.prior_lv, Dm, ldd, X, cur, nxt, st),
                    "image step");
          }
        } else
        // Split launch: with a shared dictionary no pass shares the launch, and
        // with more active signals than CUs the 16-wave coefficient workgroups
        // of a fused launch would hold the device before any pass tile runs.
        // The update then runs in workgroups sized to the support, and the
        // pass (which reads the same key slot) follows in a launch of its own.
        // (OMP's update is short enough to hide under the pass of a fused
        // launch: it splits only for a shared dictionary)
        if (W == 1 && t1 <= 256 && (P.gflow || (!omp && nact > h->num_cu))) {
          {
            PhaseScope ps(h, PH_COEF, st);
            if (omp)
              HIP_TRY(launch_coef_omp(d_insts + c.i0, nact, t, prm.lr_rel, prm.eps_rel, st),
                      "coef_omp");
            else
              HIP_TRY(launch_coef_reg(d_insts + c.i0, nact, t, prm.inner_steps, prm.beta1,
                                      prm.beta2, prm.lr_rel, prm.eps_rel, st),
                      "coef_reg");
          }
          if (!P.gflow && nnext > 0) {
            PhaseScope ps(h, PH_PASS, st);
            HIP_TRY(launch_coef_pass(bf16, c.lpa, omp, d_insts + c.i0, 0, 1, d_insts,
                                     d_htiles + c.htile_off, c.htile_prefix[nnext], t,
                                     prm.inner_steps, prm.beta1, prm.beta2, prm.lr_rel,
                                     prm.eps_rel, lds, st),
                    "pass");
            if (h->profiling)
              for (int q = c.i0; q < c.i0 + nnext; ++q)
                h->pass_bytes +=
                    (double)P.insts[q].m * P.insts[q].n * esz + 4.0 * P.insts[q].n;
          }
        } else {
          // (a shared dictionary has every column of H already: no pass tiles)
          PhaseScope ps(h, P.gflow ? PH_COEF : PH_PASS, st);
          HIP_TRY(launch_coef_pass(bf16, c.lpa, omp, d_insts + c.i0, nact, W, d_insts,
                                   d_htiles + c.htile_off, P.gflow ? 0 : c.htile_prefix[nnext], t,
                                   prm.inner_steps, prm.beta1, prm.beta2, prm.lr_rel,
                                   prm.eps_rel, lds, st),
                  "coef_pass");
          if (h->profiling && !P.gflow)
            for (int q = c.i0; q < c.i0 + nnext; ++q)
              h->pass_bytes +=
                  (double)P.insts[q].m * P.insts[q].n * esz + 4.0 * P.insts[q].n;
        }
      }
      if (nnext > 0 && P.gflow && t + 1 >= h->rscan_min_t) {
        // shared dictionary: residuals of the active signals, then the scan
        // of all of them as one contraction C = A^T R with the argmax fused
        {
          PhaseScope ps(h, PH_RESID, st);
          if (t + 1 <= 256)
            HIP_TRY(launch_shared_rows(bf16, 0, d_insts + c.i0, nnext, t + 1, st), "resid");
          else
            HIP_TRY(launch_resid(bf16, d_insts, d_rows + c.row_off, c.row_prefix[nnext], t, st),
                    "resid");
        }
        PhaseScope ps(h, PH_SCAN, st);
        HIP_TRY(launch_shared_rscan(bf16, d_insts + c.i0, nnext, P.insts[c.i0].n, t + 1, st),
                "rscan");
        if (h->profiling)
          h->scan_bytes += 4.0 * P.insts[c.i0].m * P.insts[c.i0].n;
      } else if (nnext > 0) {
        PhaseScope ps(h, PH_SCAN, st);
        HIP_TRY(launch_cscan(d_insts, d_ctiles + c.ctile_off, c.ctile_prefix[nnext], t + 1, st),
                "cscan");
        if (h->profiling)
          for (int q = c.i0; q < c.i0 + nnext; ++q)
            h->scan_bytes += 4.0 * P.insts[q].n * (t + 2) + P.insts[q].n / 8.0;
      }
    }
  }
  return CLOMP_OK;
}

// Iterations of normalised IHT (inner_steps of them) for every class.
clomp_status_t launch_iht(clomp_ctx* h, const Plan& P, int bf16, hipStream_t st) {
  char* tb = reinterpret_cast<char*>(h->tables.p);
  const Inst* d_insts = reinterpret_cast<const Inst*>(tb + P.off_insts);
  const ScanTile* d_tiles = reinterpret_cast<const ScanTile*>(tb + P.off_tiles);
  const RowTile* d_rows = reinterpret_cast<const RowTile*>(tb + P.off_rows);
  const int lds_cap = (h->lds_limit - 1024) / 4;
  const double esz = bf16 ? 2.0 : 4.0;
  for (int it = 0; it < h->params.inner_steps; ++it) {
    for (const Class& c : P.classes) {
      const int nall = c.i1 - c.i0;
      const int ntiles = c.tile_prefix[nall];
      const int nrows = c.row_prefix[nall];
      const int r_lds = (c.slice_floats <= lds_cap) ? c.slice_floats : 0;
      // a shared dictionary forms each signal's products in one workgroup
      const bool srows = P.ishared && c.kmax <= 256;
      if (it > 0) {
        PhaseScope ps(h, PH_RESID, st);
        if (srows)
          HIP_TRY(launch_shared_rows(bf16, 0, d_insts + c.i0, nall, 0, st), "iht resid");
        else
          HIP_TRY(launch_iht_rows(bf16, 0, d_insts, d_rows + c.row_off, nrows, c.kmax,
                                  nrows < h->num_cu, st),
                  "iht resid");
      }
      {
        PhaseScope ps(h, PH_SCAN, st);
        if (P.ishared)
          HIP_TRY(launch_shared_grad(bf16, d_insts + c.i0, nall, P.insts[c.i0].n, it == 0, st),
                  "iht grad");
        else
          HIP_TRY(launch_iht_grad(bf16, c.lpa, d_insts, d_tiles + c.tile_off, ntiles, c.nslice,
                                  r_lds, it == 0, st),
                  "iht grad");
        if (h->profiling)
          for (int q = c.i0; q < c.i1; ++q)
            h->scan_bytes += (double)P.insts[q].m * P.insts[q].n * esz + 4.0 * P.insts[q].m +
                             4.0 * P.insts[q].n * P.insts[q].nslice;
      }
      if (c.nslice > 1) {
        PhaseScope ps(h, PH_COEF, st);
        HIP_TRY(launch_iht_combine(d_insts, d_tiles + c.tile_off, ntiles, it == 0, st),
                "iht combine");
      }
      if (it == 0) {
        PhaseScope ps(h, PH_COEF, st);
        HIP_TRY(launch_iht_select(d_insts + c.i0, nall, 0, c.nmax, st), "iht select");
      }
      {
        PhaseScope ps(h, PH_GRAM, st);
        if (srows)
          HIP_TRY(launch_shared_rows(bf16, 1, d_insts + c.i0, nall, 0, st), "iht step");
        else
          HIP_TRY(launch_iht_rows(bf16, 1, d_insts, d_rows + c.row_off, nrows, c.kmax,
                                  nrows < h->num_cu, st),
                  "iht step");
      }
      {
        PhaseScope ps(h, PH_COEF, st);
        HIP_TRY(launch_iht_select(d_insts + c.i0, nall, it + 1 == h->params.inner_steps ? 2 : 1,
                                  c.nmax, st), "iht select");
      }
    }
  }
  return CLOMP_OK;
}

// R = inner_steps iterations of paper-mode CLOMP for every class.
clomp_status_t launch_paper(clomp_ctx* h, const Plan& P, int bf16, hipStream_t st) {
  const clomp_params_t& prm = h->params;
  char* tb = reinterpret_cast<char*>(h->tables.p);
  const Inst* d_insts = reinterpret_cast<const Inst*>(tb + P.off_insts);
  const ScanTile* d_tiles = reinterpret_cast<const ScanTile*>(tb + P.off_tiles);
  const RowTile* d_rows = reinterpret_cast<const RowTile*>(tb + P.off_rows);
  const int lds_cap = (h->lds_limit - 1024) / 4;
  const double esz = bf16 ? 2.0 : 4.0;
  double b1p = 1.0, b2p = 1.0;
  for (int it = 0; it < prm.inner_steps; ++it) {
    b1p *= prm.beta1;
    b2p *= prm.beta2;
    const float bc1 = (float)(1.0 - b1p), bc2 = (float)(1.0 - b2p);
    for (const Class& c : P.classes) {
      const int nall = c.i1 - c.i0;
      const int ntiles = c.tile_prefix[nall];
      const int nrows = c.row_prefix[nall];
      const int r_lds = (c.slice_floats <= lds_cap) ? c.slice_floats : 0;
      if (it > 0) {
        PhaseScope ps(h, PH_RESID, st);
        if (P.ishared && c.kmax <= 256)
          HIP_TRY(launch_shared_rows(bf16, 0, d_insts + c.i0, nall, 0, st), "paper resid");
        else
          HIP_TRY(launch_iht_rows(bf16, 0, d_insts, d_rows + c.row_off, nrows, c.kmax,
                                  nrows < h->num_cu, st),
                  "paper resid");
      }
      {
        PhaseScope ps(h, PH_SCAN, st);
        if (P.ishared)
          HIP_TRY(launch_shared_grad(bf16, d_insts + c.i0, nall, P.insts[c.i0].n, it == 0, st),
                  "paper scan");
        else
          HIP_TRY(launch_iht_grad(bf16, c.lpa, d_insts, d_tiles + c.tile_off, ntiles, c.nslice,
                                  r_lds, it == 0, st),
                  "paper scan");
        if (h->profiling)
          for (int q = c.i0; q < c.i1; ++q)
            h->scan_bytes += (double)P.insts[q].m * P.insts[q].n * esz + 4.0 * P.insts[q].m +
                             4.0 * P.insts[q].n * P.insts[q].nslice;
      }
      PhaseScope ps(h, PH_COEF, st);
      if (c.nslice > 1)
        HIP_TRY(launch_iht_combine(d_insts, d_tiles + c.tile_off, ntiles, it == 0, st),
                "paper combine");
      HIP_TRY(launch_paper_select(d_insts + c.i0, nall, it, it + 1 == prm.inner_steps,
                                  prm.select_threshold, prm.lr_rel, prm.beta1, prm.beta2, bc1,
                                  bc2, prm.eps_rel, c.nmax, st),
              "paper select");
    }
  }
  return CLOMP_OK;
}

// The launch sequence of one batch (captured as a graph when requested).
clomp_status_t launch_all(clomp_ctx* h, const Plan& P, int bf16, hipStream_t st) {
  const clomp_params_t& prm = h->params;
  const bool omp = prm.method == CLOMP_METHOD_OMP;
  char* tb = reinterpret_cast<char*>(h->tables.p);
  const Inst* d_insts = reinterpret_cast<const Inst*>(tb + P.off_insts);
  const ScanTile* d_tiles = reinterpret_cast<const ScanTile*>(tb + P.off_tiles);
  const RowTile* d_rows = reinterpret_cast<const RowTile*>(tb + P.off_rows);
  const int* d_qr = reinterpret_cast<const int*>(tb + P.off_qr);
  const int* d_cg = reinterpret_cast<const int*>(tb + P.off_cg);
  const RowTile* d_cgrows = reinterpret_cast<const RowTile*>(tb + P.off_cgrows);
  const int count = (int)P.insts.size();
  const int lds_cap = (h->lds_limit - 1024) / 4;

  {
    PhaseScope ps(h, PH_INIT, st, false);
    HIP_TRY(launch_init(d_insts, count, st), "init");
    if (P.image) {
      // the basis, and both dense coefficient images and the pixel image at
      // zero (contiguous in the workspace)
      char* wsb = reinterpret_cast<char*>(h->ws.p);
      const long long ldd = round_up_int(P.insts[0].n, 256);
      HIP_TRY(launch_image_init(reinterpret_cast<float*>(wsb + P.off_dct), P.insts[0].n, ldd,
                                reinterpret_cast<float*>(wsb + P.off_sd), 3LL * ldd * count, st),
              "image init");
    }
  }
  if (!P.small_list.empty()) {
    const int* d_small = reinterpret_cast<const int*>(tb + P.off_small);
    PhaseScope ps(h, PH_FUSED, st);
    int kmax = 1;
    for (int q : P.small_list) kmax = std::max(kmax, P.insts[q].k_eff);
    HIP_TRY(launch_small(bf16, omp, d_insts, d_small, (int)P.small_list.size(), kmax,
                         prm.inner_steps, prm.beta1, prm.beta2, prm.lr_rel, prm.eps_rel,
                         P.small_lds, st),
            "small");
    if (h->profiling) {
      const double esz = bf16 ? 2.0 : 4.0;
      for (int q : P.small_list)
        h->fused_bytes += (double)P.insts[q].m * P.insts[q].n * esz + 4.0 * P.insts[q].m;
    }
  }
  const bool iht = prm.method == CLOMP_METHOD_IHT || prm.method == CLOMP_METHOD_PAPER;
  if (prm.method == CLOMP_METHOD_IHT) {
    clomp_status_t hs = launch_iht(h, P, bf16, st);
    if (hs != CLOMP_OK) return hs;
  } else if (prm.method == CLOMP_METHOD_PAPER) {
    clomp_status_t hs = launch_paper(h, P, bf16, st);
    if (hs != CLOMP_OK) return hs;
  } else if (P.hflow) {
    clomp_status_t hs = launch_hflow(h, P, bf16, st);
    if (hs != CLOMP_OK) return hs;
  }
  for (int t = 0; t < ((P.hflow || iht) ? 0 : P.kmax); ++t) {
    for (const Class& c : P.classes) {
      if (c.kmax <= t) continue;
      // active prefix of the class: instances with k_eff > t
      int nact = 0;
      while (c.i0 + nact < c.i1 && P.keff[c.i0 + nact] > t) ++nact;
      const int ntiles = c.tile_prefix[nact];
      const int nrows = c.row_prefix[nact];
      const int r_lds = (c.m_pad_max <= lds_cap) ? c.m_pad_max : 0;
      {
        PhaseScope ps(h, PH_SCAN, st);
        if (c.nch > 0)
          HIP_TRY(launch_scan_reg(bf16, c.lpa, c.nch, d_insts, d_tiles + c.tile_off, ntiles, t & 1,
                                  st),
                  "scan");
        else
          HIP_TRY(launch_scan(bf16, c.lpa, d_insts, d_tiles + c.tile_off, ntiles, r_lds, t & 1, st),
                  "scan");
      }
      if (h->profiling) {
        const double esz = bf16 ? 2.0 : 4.0;
        for (int q = c.i0; q < c.i0 + nact; ++q) {
          const Inst& d = P.insts[q];
          h->scan_bytes += (double)d.m * d.n * esz + 4.0 * d.m + d.n / 8.0;
        }
      }
      const int ng = kBlock / c.lpa;
      const int ndots = t + 2;
      int D = ng;
      while ((long long)nact * ((ndots + D - 1) / D) > 8L * h->num_cu && D < 8 * ng) D *= 2;
      const int nblk = (ndots + D - 1) / D;
      {
        PhaseScope ps(h, PH_GRAM, st);
        if (c.nch > 0)
          HIP_TRY(launch_gram_reg(bf16, c.lpa, c.nch, d_insts + c.i0, nact, t, nblk, D,
                                  prm.lr_rel, prm.eps_rel, st),
                  "gram");
        else
          HIP_TRY(launch_gram(bf16, c.lpa, d_insts + c.i0, nact, t, nblk, D, r_lds, prm.lr_rel,
                              prm.eps_rel, st),
                  "gram");
      }
      {
        PhaseScope ps(h, PH_COEF, st);
        if (omp)
          HIP_TRY(launch_omp(d_insts + c.i0, nact, t, st), "omp");
        else
          HIP_TRY(launch_adam(d_insts + c.i0, nact, t, prm.inner_steps, prm.beta1, prm.beta2,
                              st),
                  "adam");
      }
      {
        PhaseScope ps(h, PH_RESID, st);
        HIP_TRY(launch_resid(bf16, d_insts, d_rows + c.row_off, nrows, t, st), "resid");
      }
    }
  }
  // refinement (or, with CLOMP_FLAG_NO_REFINE, the greedy loop's coefficients)
  // (image mode returns the learned coefficients: the local variation is not
  // quadratic, so no least-squares solve minimises the same loss)
  const bool refine = !(prm.flags & CLOMP_FLAG_NO_REFINE) && !P.image;
  const int ncg = refine ? (int)P.cg_list.size() : 0;
  {
  PhaseScope ref_scope(h, PH_REFINE, st, false);
  if (refine)
    HIP_TRY(launch_qr(d_insts, d_qr, (int)P.qr_list.size(), P.qr_lds, st), "qr");
  else
    HIP_TRY(launch_copy_s(d_insts, nullptr, count, st), "copy_s");
  if (ncg > 0) {
    const float tol = prm.refine_tol > 0.f ? prm.refine_tol : 1e-6f;
    const int iters = prm.refine_iters > 0 ? prm.refine_iters : 48;
    const int ng = kBlock / P.cg_lpa;
    int D = ng;
    while ((long long)ncg * ((P.cg_tmax + D - 1) / D) > 8L * h->num_cu && D < 8 * ng) D *= 2;
    const int nblk = (P.cg_tmax + D - 1) / D;
    const int ncgrows = (int)P.cg_rows.size();
    HIP_TRY(launch_copy_s(d_insts, d_cg, ncg, st), "copy_s");
    HIP_TRY(launch_cg_rows(0, d_insts, d_cgrows, ncgrows, P.cg_tmax, 0, 0.f, st), "cg_r0");
    HIP_TRY(launch_cg_dots(0, P.cg_lpa, d_insts, d_cg, ncg, P.cg_tmax, nblk, D, P.cg_mpad_max, 0,
                           st),
            "cg_sv0");
    for (int it = 0; it < iters; ++it) {
      HIP_TRY(launch_cg_rows(1, d_insts, d_cgrows, ncgrows, P.cg_tmax, it, tol * tol, st),
              "cg_q");
      HIP_TRY(launch_cg_dots(1, P.cg_lpa, d_insts, d_cg, ncg, P.cg_tmax, nblk, D, P.cg_mpad_max,
                             it, st),
              "cg_sv");
    }
  }
  }
  PhaseScope ps(h, PH_NORM, st, false);
  HIP_TRY(launch_norm(d_insts, d_rows, (int)P.rows.size(), P.kmax, st), "norm");
  HIP_TRY(launch_finalize(d_insts, count, ncg > 0, st), "finalize");
  return CLOMP_OK;
}

// Workspace (grow-only; growth invalidates captured graphs), descriptors
// rebased onto it, and the descriptor / tile tables uploaded on `st` through
// pinned staging.
clomp_status_t stage_plan(clomp_ctx* h, const Plan& P, hipStream_t st) {
  clomp_status_t s = CLOMP_OK;
  // workspace and tables (grow-only; growth invalidates captured graphs)
  bool g1 = false, g2 = false;
  if ((s = ensure(h, h->ws, P.ws_bytes, &g1)) != CLOMP_OK) return s;
  if ((s = ensure(h, h->tables, P.table_bytes, &g2)) != CLOMP_OK) return s;
  if (g1 || g2) drop_graphs(h);
  // stage tables in pinned memory and upload on the stream
  if (h->pinned_bytes < P.table_bytes) {
    if (h->pinned) {
      HIP_TRY(hipEventSynchronize(h->staging_free), "hipEventSynchronize");
      (void)hipHostFree(h->pinned);
      h->pinned = nullptr;
    }
    const size_t want = align_up(P.table_bytes * 2, 1 << 16);
    if (hipHostMalloc(&h->pinned, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      h->pinned = nullptr;
      h->pinned_bytes = 0;
      return fail(h, CLOMP_OUT_OF_MEMORY, "pinned staging allocation failed");
    }
    h->pinned_bytes = want;
  } else {
    HIP_TRY(hipEventSynchronize(h->staging_free), "hipEventSynchronize");
  }
  char* hb = reinterpret_cast<char*>(h->pinned);
  // descriptors with their workspace offsets rebased onto the workspace
  char* wsb = reinterpret_cast<char*>(h->ws.p);
  Inst* dst = reinterpret_cast<Inst*>(hb + P.off_insts);
  for (size_t q = 0; q < P.insts.size(); ++q) {
    Inst& d = dst[q];
    d = P.insts[q];
    d.spin = (unsigned)h->spin_limit;
    auto rb = [&](auto*& ptr) {
      if (ptr) ptr = reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(
                   wsb + (reinterpret_cast<uintptr_t>(ptr) - 1));
    };
    rb(d.r); rb(d.G); rb(d.b); rb(d.s); rb(d.mo); rb(d.ve); rb(d.xf); rb(d.z);
    rb(d.Linv); rb(d.cg); rb(d.c0); rb(d.dg); rb(d.H); rb(d.team); rb(d.gbuf); rb(d.sfull);
    rb(d.mden); rb(d.vden); rb(d.Gf);
    rb(d.npart);
    rb(d.qpart); rb(d.key);
    rb(d.bitmap);
    rb(d.st);
  }
  if (!P.tiles.empty()) memcpy(hb + P.off_tiles, P.tiles.data(), sizeof(ScanTile) * P.tiles.size());
  if (!P.rows.empty()) memcpy(hb + P.off_rows, P.rows.data(), sizeof(RowTile) * P.rows.size());
  if (!P.qr_list.empty()) memcpy(hb + P.off_qr, P.qr_list.data(), sizeof(int) * P.qr_list.size());
  if (!P.cg_list.empty()) memcpy(hb + P.off_cg, P.cg_list.data(), sizeof(int) * P.cg_list.size());
  if (!P.cg_rows.empty())
    memcpy(hb + P.off_cgrows, P.cg_rows.data(), sizeof(RowTile) * P.cg_rows.size());
  if (!P.htiles.empty())
    memcpy(hb + P.off_htiles, P.htiles.data(), sizeof(ScanTile) * P.htiles.size());
  if (!P.ctiles.empty())
    memcpy(hb + P.off_ctiles, P.ctiles.data(), sizeof(ScanTile) * P.ctiles.size());
  if (!P.small_list.empty())
    memcpy(hb + P.off_small, P.small_list.data(), sizeof(int) * P.small_list.size());
  // the previous batch (possibly on another stream) must be done with the tables
  if (h->have_work) HIP_TRY(hipStreamWaitEvent(st, h->work_done, 0), "hipStreamWaitEvent");
  HIP_TRY(hipMemcpyAsync(h->tables.p, hb, P.table_bytes, hipMemcpyHostToDevice, st),
          "upload tables");
  HIP_TRY(hipEventRecord(h->staging_free, st), "hipEventRecord");

  return CLOMP_OK;
}

// Autotuning (CLOMP_FLAG_AUTOTUNE): for each candidate tile size, the plan of
// this batch is staged and its hot kernel is timed on the batch's own data -
// the fused pass of iteration 0 (correlation schedule, after the first pass
// has chosen the atom) or the scan of iteration 0 (residual schedule).  The
// probes leave only state that the solve's init launch resets.
// Size class of a batch for the autotuner: device architecture, bulk dtype,
// method, schedule, and the octaves of the largest m, the largest n and the
// number of iterated signals.
std::string tune_key(const Plan& P, int bf16, int method, const std::string& arch) {
  int mmax = 1, nmax = 1;
  for (int q = 0; q < P.nbig; ++q) {
    mmax = std::max(mmax, P.insts[q].m);
    nmax = std::max(nmax, P.insts[q].n);
  }
  auto octave = [](int v) {
    int o = 0;
    while ((2LL << o) <= v) ++o;
    return o;
  };
  static const char* kMethod[] = {"clomp", "omp", "iht", "paper"};
  char buf[160];
  snprintf(buf, sizeof buf, "%s/%s/%s/%s/m%d/n%d/c%d", arch.c_str(), bf16 ? "bf16" : "f32",
           (method >= 0 && method < 4) ? kMethod[method] : "other", P.hflow ? "corr" : "resid",
           octave(mmax), octave(nmax), octave(std::max(P.nbig, 1)));
  return buf;
}

// The process-wide autotune table: every handle's results, and the entries a
// caller imported (a saved table from an earlier process).  A handle looks in
// its own table, then here, and only then times the candidates.
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
thread_local std::string g_table_error;   // last error of a handle-free call

clomp_status_t table_fail(const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_table_error = buf;
  return CLOMP_INVALID_ARGUMENT;
}

constexpr const char* kTableHeader = "clomp-tuning 1";

bool key_char_ok(char c) {
  return (c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z') || (c >= '0' && c <= '9') ||
         c == '_' || c == '.' || c == '/' || c == ':' || c == '+' || c == '-';
}

clomp_status_t probe_launch(clomp_ctx* h, const Plan& P, int bf16, hipStream_t st, bool timed) {
  const clomp_params_t& prm = h->params;
  const bool omp = prm.method == CLOMP_METHOD_OMP;
  char* tb = reinterpret_cast<char*>(h->tables.p);
  const Inst* d_insts = reinterpret_cast<const Inst*>(tb + P.off_insts);
  for (const Class& c : P.classes) {
    const int nall = c.i1 - c.i0;
    if (P.hflow) {
      const ScanTile* d_htiles = reinterpret_cast<const ScanTile*>(tb + P.off_htiles);
      const size_t lds = (size_t)c.m_pad_max * sizeof(float);
      if (!timed) {
        HIP_TRY(launch_ypass(bf16, c.lpa, d_insts, d_htiles + c.htile_off, c.htile_prefix[nall],
                             lds, st),
                "ypass");
        continue;
      }
      int nnext = 0;
      while (nnext < nall && P.keff[c.i0 + nnext] > 1) ++nnext;
      HIP_TRY(launch_coef_pass(bf16, c.lpa, omp, d_insts + c.i0, nall, 1, d_insts,
                               d_htiles + c.htile_off, c.htile_prefix[nnext], 0, prm.inner_steps,
                               prm.beta1, prm.beta2, prm.lr_rel, prm.eps_rel,
                               std::max(lds, (omp ? 6 : 1) * sizeof(float)), st),
              "coef_pass");
    } else {
      if (!timed) continue;
      const ScanTile* d_tiles = reinterpret_cast<const ScanTile*>(tb + P.off_tiles);
      const int lds_cap = (h->lds_limit - 1024) / 4;
      const int r_lds = (c.m_pad_max <= lds_cap) ? c.m_pad_max : 0;
      if (c.nch > 0)
        HIP_TRY(launch_scan_reg(bf16, c.lpa, c.nch, d_insts, d_tiles + c.tile_off,
                                c.tile_prefix[nall], 0, st),
                "scan");
      else
        HIP_TRY(launch_scan(bf16, c.lpa, d_insts, d_tiles + c.tile_off, c.tile_prefix[nall], r_lds,
                            0, st),
                "scan");
    }
  }
  return CLOMP_OK;
}

clomp_status_t autotune(clomp_ctx* h, const clomp_instance_t* inst, int count, int bf16,
                        hipStream_t st, bool hflow, int scan_kb, int pass_kb, int* best_kb) {
  static const int kScanCand[] = {32, 64, 128, 256, 512};
  static const int kPassCand[] = {128, 256, 512, 1024, 2048};
  const int* cand = hflow ? kPassCand : kScanCand;
  const int ncand = 5;
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a), "hipEventCreate");
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return hip_fail(h, hipGetLastError(), "hipEventCreate");
  }
  const bool was_profiling = h->profiling;
  h->profiling = false;
  clomp_status_t s = CLOMP_OK;
  float best = 0.f;
  *best_kb = hflow ? pass_kb : scan_kb;
  for (int q = 0; q < ncand && s == CLOMP_OK; ++q) {
    Plan P;
    build_plan(h, inst, count, bf16, P, hflow ? scan_kb : cand[q], hflow ? cand[q] : pass_kb);
    if ((s = stage_plan(h, P, st)) != CLOMP_OK) break;
    char* tb = reinterpret_cast<char*>(h->tables.p);
    hipError_t e = launch_init(reinterpret_cast<const Inst*>(tb + P.off_insts), count, st);
    if (e != hipSuccess) { s = hip_fail(h, e, "init"); break; }
    if ((s = probe_launch(h, P, bf16, st, false)) != CLOMP_OK) break;
    if ((s = probe_launch(h, P, bf16, st, true)) != CLOMP_OK) break;   // warm
    if ((e = hipEventRecord(a, st)) != hipSuccess) { s = hip_fail(h, e, "event"); break; }
    for (int r = 0; r < 3 && s == CLOMP_OK; ++r) s = probe_launch(h, P, bf16, st, true);
    if (s != CLOMP_OK) break;
    if ((e = hipEventRecord(b, st)) != hipSuccess || (e = hipEventSynchronize(b)) != hipSuccess) {
      s = hip_fail(h, e, "event");
      break;
    }
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) { s = hip_fail(h, e, "event"); break; }
    if (q == 0 || ms < best) {
      best = ms;
      *best_kb = cand[q];
    }
  }
  h->profiling = was_profiling;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return s;
}

}  // namespace

// ============================================================ C ABI
extern "C" {

void clomp_default_params(clomp_params_t* p) {
  if (!p) return;
  p->method = CLOMP_METHOD_CLOMP;
  p->inner_steps = 32;
  p->lr_rel = 0.05f;
  p->beta1 = 0.9f;
  p->beta2 = 0.999f;
  p->eps_rel = 1e-8f;
  p->resid_tol = 0.f;
  p->refine_iters = 0;
  p->refine_tol = 0.f;
  p->flags = 0u;
  p->select_threshold = 0.7f;
  p->prior_tv = 0.f;
  p->prior_lv = 0.f;
}

const char* clomp_status_string(clomp_status_t s) {
  switch (s) {
    case CLOMP_OK: return "CLOMP_OK";
    case CLOMP_INVALID_ARGUMENT: return "CLOMP_INVALID_ARGUMENT";
    case CLOMP_OUT_OF_MEMORY: return "CLOMP_OUT_OF_MEMORY";
    case CLOMP_DEVICE_ERROR: return "CLOMP_DEVICE_ERROR";
    case CLOMP_NOT_SUPPORTED: return "CLOMP_NOT_SUPPORTED";
  }
  return "CLOMP_UNKNOWN_STATUS";
}

const char* clomp_last_error(clomp_handle_t h) {
  if (!h) return g_table_error.empty() ? "no handle" : g_table_error.c_str();
  return h->last_error.c_str();
}

clomp_status_t clomp_tuning_table_import(const char* text, int32_t* n_entries) {
  g_table_error.clear();
  if (!text) return table_fail("text is NULL");
  std::map<std::string, int> add;
  const char* p = text;
  int line = 0;
  bool header = false;
  while (*p) {
    const char* e = p;
    while (*e && *e != '\n') ++e;
    std::string ln(p, e);
    p = *e ? e + 1 : e;
    ++line;
    if (!ln.empty() && ln.back() == '\r') ln.pop_back();
    if (!header) {
      if (ln != kTableHeader)
        return table_fail("line 1: expected the header '%s'", kTableHeader);
      header = true;
      continue;
    }
    if (ln.empty() || ln[0] == '#') continue;
    const size_t sp = ln.find(' ');
    if (sp == std::string::npos || sp == 0 || sp > 127)
      return table_fail("line %d: expected '<key> <tile KB>'", line);
    const std::string key = ln.substr(0, sp);
    for (char c : key)
      if (!key_char_ok(c)) return table_fail("line %d: key has a character outside [A-Za-z0-9_./:+-]", line);
    const std::string val = ln.substr(sp + 1);
    if (val.empty() || val.size() > 5) return table_fail("line %d: tile KB must be 1 .. 65536", line);
    long v = 0;
    for (char c : val) {
      if (c < '0' || c > '9') return table_fail("line %d: tile KB must be 1 .. 65536", line);
      v = v * 10 + (c - '0');
    }
    if (v < 1 || v > 65536) return table_fail("line %d: tile KB must be 1 .. 65536", line);
    if (!add.emplace(key, (int)v).second) return table_fail("line %d: key repeated", line);
  }
  if (!header) return table_fail("line 1: expected the header '%s'", kTableHeader);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : add) g_tune[kv.first] = kv.second;
  if (n_entries) *n_entries = (int32_t)add.size();
  return CLOMP_OK;
}

clomp_status_t clomp_tuning_table_export(char* buf, size_t cap, size_t* len) {
  g_table_error.clear();
  if (!len) return table_fail("len is NULL");
  std::string out = std::string(kTableHeader) + "\n";
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : g_tune) out += kv.first + " " + std::to_string(kv.second) + "\n";
  }
  *len = out.size();
  if (!buf) return CLOMP_OK;
  if (cap < out.size() + 1)
    return table_fail("buffer of %zu bytes; the table needs %zu", cap, out.size() + 1);
  memcpy(buf, out.c_str(), out.size() + 1);
  return CLOMP_OK;
}

clomp_status_t clomp_tuning_table_clear(void) {
  g_table_error.clear();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  return CLOMP_OK;
}

clomp_status_t clomp_create(clomp_handle_t* out, int device, const clomp_params_t* params) {
  if (!out) return CLOMP_INVALID_ARGUMENT;
  *out = nullptr;
  clomp_params_t p;
  clomp_default_params(&p);
  if (params) {
    const clomp_status_t s = check_params(nullptr, params);
    if (s != CLOMP_OK) return s;
    p = *params;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return CLOMP_DEVICE_ERROR;
  }
  clomp_ctx* h = new clomp_ctx();
  h->device = device;
  h->params = p;
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(device) != hipSuccess) {
    delete h;
    return CLOMP_DEVICE_ERROR;
  }
  int lds = 65536, ncu = 256;
  (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
  h->lds_limit = lds;
  h->num_cu = ncu;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
      std::string a(prop.gcnArchName);
      a = a.substr(0, a.find(':'));
      bool ok = !a.empty();
      for (char c : a) ok = ok && key_char_ok(c) && c != '/';
      if (ok) h->arch = a;
    } else {
      (void)hipGetLastError();
    }
  }
  if (lds > 65536 && set_max_lds((size_t)lds) != hipSuccess) {
    (void)hipGetLastError();
    h->lds_limit = 65536;
  }
  // the allocation-free gradient's scratch: its address on this device, once
  if (grad_scratch_init(device) != hipSuccess) {
    (void)hipGetLastError();
    delete h;
    (void)hipSetDevice(prev);
    return CLOMP_DEVICE_ERROR;
  }
  h->pass_lds_ok = set_max_lds_pass((size_t)h->lds_limit) == hipSuccess;
  if (!h->pass_lds_ok) (void)hipGetLastError();
  if (hipEventCreateWithFlags(&h->staging_free, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->work_done, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->grad_done, hipEventDisableTiming) != hipSuccess) {
    delete h;
    (void)hipSetDevice(prev);
    return CLOMP_DEVICE_ERROR;
  }
  (void)hipSetDevice(prev);
  *out = h;
  return CLOMP_OK;
}

clomp_status_t clomp_set_params(clomp_handle_t h, const clomp_params_t* params) {
  if (!h) return CLOMP_INVALID_ARGUMENT;
  const clomp_status_t s = check_params(h, params);
  if (s != CLOMP_OK) return s;
  h->params = *params;
  h->pcache.valid = false;
  drop_graphs(h);
  return CLOMP_OK;
}

clomp_status_t clomp_check_batch(clomp_handle_t h, const clomp_instance_t* inst, int32_t count,
                                 int32_t a_dtype) {
  const clomp_status_t s = check_batch_impl(h, inst, count, a_dtype);
  if (s != CLOMP_OK || !h || !(h->params.flags & CLOMP_FLAG_IMAGE)) return s;
  return check_image_batch(h, inst, count);
}

clomp_status_t clomp_solve_batch(clomp_handle_t h, const clomp_instance_t* inst, int32_t count,
                                 int32_t a_dtype, void* hip_stream) {
  if (!h) return CLOMP_INVALID_ARGUMENT;
  clomp_status_t s = check_batch_impl(h, inst, count, a_dtype);
  if (s != CLOMP_OK || count == 0) return s;
  if ((h->params.flags & CLOMP_FLAG_IMAGE) && (s = check_image_batch(h, inst, count)) != CLOMP_OK)
    return s;
  const int bf16 = a_dtype == CLOMP_BF16;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  DeviceGuard dg;
  HIP_TRY(hipSetDevice(h->device), "hipSetDevice");

  std::vector<ShapeRec> shapes(count);
  for (int i = 0; i < count; ++i)
    shapes[i] = {inst[i].n, inst[i].m, inst[i].k, inst[i].A_master ? 1 : 0,
                 (long long)inst[i].lda, (long long)inst[i].lda_master};
  Plan fresh;
  int scan_kb = h->scan_tile_kb, pass_kb = h->pass_tile_kb;
  // a cached plan also fixes whether the batch shares one dictionary: the
  // shared schedules read A from the first signal, so a batch with the same
  // shapes but other sharing needs a new plan
  const bool cached = h->pcache.valid && h->pcache.bf16 == bf16 && h->pcache.shapes == shapes &&
                      same_dictionary(inst, h->pcache.P.order, h->pcache.P.nbig) ==
                          h->pcache.sameA;
  Plan& P = cached ? h->pcache.P : fresh;
  if (cached) {
    scan_kb = h->pcache.scan_kb;
    pass_kb = h->pcache.pass_kb;
    for (int q = 0; q < count; ++q) {
      const clomp_instance_t& src = inst[P.order[q]];
      Inst& d = P.insts[q];
      d.A = src.A;
      d.Am = src.A_master ? src.A_master : reinterpret_cast<const float*>(src.A);
      d.y = src.y;
      d.x = src.x;
      d.support = src.support;
      d.nsel = src.n_selected;
      d.rnorm = src.resid_norm;
      d.status = src.status;
    }
  } else {
    build_plan(h, inst, count, bf16, P, scan_kb, pass_kb);
  }
  if (!cached && (h->params.flags & CLOMP_FLAG_AUTOTUNE) && P.nbig > 0) {
    const std::string key = tune_key(P, bf16, h->params.method, h->arch);
    auto it = h->tuned.find(key);
    int kb = 0;
    if (it != h->tuned.end()) {
      kb = it->second;
    } else {
      {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto g = g_tune.find(key);
        if (g != g_tune.end()) kb = g->second;
      }
      if (kb == 0 &&
          (s = autotune(h, inst, count, bf16, st, P.hflow, scan_kb, pass_kb, &kb)) != CLOMP_OK)
        return s;
      h->tuned[key] = kb;
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[key] = kb;
    }
    if (P.hflow) pass_kb = kb; else scan_kb = kb;
    build_plan(h, inst, count, bf16, P, scan_kb, pass_kb);
  }
  if (!cached) {
    h->pcache.valid = false;   // until the new plan is in place
    h->pcache.P = std::move(fresh);
    h->pcache.bf16 = bf16;
    h->pcache.shapes = std::move(shapes);
    h->pcache.sameA = same_dictionary(inst, h->pcache.P.order, h->pcache.P.nbig);
    h->pcache.scan_kb = scan_kb;
    h->pcache.pass_kb = pass_kb;
    h->pcache.valid = true;
  }
  const Plan& PP = h->pcache.P;
  h->last_scan_kb = scan_kb;
  h->last_pass_kb = pass_kb;
  if ((h->params.flags & CLOMP_FLAG_IMAGE) && !PP.image)
    return fail(h, CLOMP_NOT_SUPPORTED,
                "CLOMP_FLAG_IMAGE needs the shared-dictionary schedule (Gram matrix within 4 GB)");
  if (h->params.prior_tv > 0.f && !PP.cg_list.empty() && !PP.image)
    return fail(h, CLOMP_NOT_SUPPORTED,
                "the total-variation prior needs the in-LDS QR refinement: (m + k_eff) * k_eff "
                "of a signal exceeds it");
  if ((size_t)PP.cg_mpad_max * sizeof(float) + 1024 > (size_t)h->lds_limit)
    return fail(h, CLOMP_NOT_SUPPORTED,
                "m = %d needs %zu bytes of LDS for the refinement; the device allows %d",
                PP.cg_mpad_max, (size_t)PP.cg_mpad_max * sizeof(float), h->lds_limit);

  if ((s = stage_plan(h, PP, st)) != CLOMP_OK) return s;

  // the legacy default stream cannot be captured: launch eagerly there
  const bool use_graph = (h->params.flags & CLOMP_FLAG_GRAPH) != 0 && st != nullptr;
  h->profiling = !use_graph && (h->params.flags & CLOMP_FLAG_PROFILE) != 0;
  if (use_graph) {
    auto it = h->graphs.find(PP.sig);
    if (it == h->graphs.end()) {
      CachedGraph cg;
      HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture");
      s = launch_all(h, PP, bf16, st);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(st, &g);
      if (s != CLOMP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
      }
      if (e != hipSuccess) return hip_fail(h, e, "end capture");
      cg.graph = g;
      HIP_TRY(hipGraphInstantiate(&cg.exec, g, nullptr, nullptr, 0), "graph instantiate");
      it = h->graphs.emplace(PP.sig, cg).first;
    }
    HIP_TRY(hipGraphLaunch(it->second.exec, st), "graph launch");
  } else {
    if ((s = launch_all(h, PP, bf16, st)) != CLOMP_OK) return s;
  }
  HIP_TRY(hipEventRecord(h->work_done, st), "hipEventRecord");
  h->have_work = true;
  return CLOMP_OK;
}

namespace {
constexpr int kGradColChunk = 256;   // atoms per forward partial of clomp_grad

// Argument checks shared by both gradient entry points; *need receives the
// scratch bytes of the call.
clomp_status_t check_grad_args(clomp_ctx* h, const char* fn, int32_t n, int32_t m, int64_t lda,
                               int32_t dtype, const void* A, const void* x, const uint8_t* mask,
                               const void* y, const void* grad_x, const void* loss,
                               size_t* need) {
  if (dtype == CLOMP_BF16) return fail(h, CLOMP_NOT_SUPPORTED, "%s serves F32 and F64", fn);
  if (dtype != CLOMP_F32 && dtype != CLOMP_F64)
    return fail(h, CLOMP_INVALID_ARGUMENT, "unknown dtype %d", dtype);
  if (n <= 0 || m <= 0 || lda < m) return fail(h, CLOMP_INVALID_ARGUMENT, "bad n, m or lda");
  if (!A || !x || !mask || !y || !grad_x || !loss)
    return fail(h, CLOMP_INVALID_ARGUMENT, "a required pointer is NULL");
  const size_t es = dtype == CLOMP_F64 ? 8 : 4;
  if (((uintptr_t)A % es) || ((uintptr_t)x % es) || ((uintptr_t)y % es))
    return fail(h, CLOMP_INVALID_ARGUMENT, "A, x and y must be aligned to their element size");
  const size_t ncolchunk = ((size_t)n + kGradColChunk - 1) / kGradColChunk;
  const size_t nfin = ((size_t)m + kBlock - 1) / kBlock;
  *need = es * (ncolchunk * (size_t)m + (size_t)m + nfin);
  return CLOMP_OK;
}
}  // namespace

clomp_status_t clomp_grad(clomp_handle_t h, int32_t n, int32_t m, int64_t lda, int32_t dtype,
                          const void* A, const void* x, const uint8_t* mask, const void* y,
                          const void* grad_out, void* grad_x, void* resid_out, void* loss,
                          void* hip_stream) {
  if (!h) return CLOMP_INVALID_ARGUMENT;
  size_t need = 0;
  const clomp_status_t cs =
      check_grad_args(h, "clomp_grad", n, m, lda, dtype, A, x, mask, y, grad_x, loss, &need);
  if (cs != CLOMP_OK) return cs;
  need += 256;
  const int colchunk = kGradColChunk;
  const int ncolchunk = (n + colchunk - 1) / colchunk;
  DeviceGuard dg;
  HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  if (h->gwork.bytes < need) {
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    clomp_status_t s = ensure(h, h->gwork, need, nullptr);
    if (s != CLOMP_OK) return s;
  }
  // the partial sums live in one per-handle buffer: a call on another stream
  // waits until the previous call has finished with it
  if (h->have_grad) HIP_TRY(hipStreamWaitEvent(st, h->grad_done, 0), "hipStreamWaitEvent");
  HIP_TRY(launch_grad(dtype == CLOMP_F64, n, m, lda, A, x, mask, y, grad_out, grad_x, resid_out,
                      loss, h->gwork.p, ncolchunk, colchunk, st),
          "grad");
  HIP_TRY(hipEventRecord(h->grad_done, st), "hipEventRecord");
  h->have_grad = true;
  return CLOMP_OK;
}

clomp_status_t clomp_grad_noalloc(clomp_handle_t h, int32_t n, int32_t m, int64_t lda,
                                  int32_t dtype, const void* A, const void* x,
                                  const uint8_t* mask, const void* y, const void* grad_out,
                                  void* grad_x, void* resid_out, void* loss, void* hip_stream) {
  if (!h) return CLOMP_INVALID_ARGUMENT;
  size_t need = 0;
  const clomp_status_t cs = check_grad_args(h, "clomp_grad_noalloc", n, m, lda, dtype, A, x,
                                            mask, y, grad_x, loss, &need);
  if (cs != CLOMP_OK) return cs;
  if (need > kGradScratchBytes)
    return fail(h, CLOMP_INVALID_ARGUMENT,
                "clomp_grad_noalloc needs %zu bytes of scratch for n = %d, m = %d; its "
                "device-resident scratch holds %zu (use clomp_grad)",
                need, n, m, kGradScratchBytes);
  void* work = grad_scratch_ptr(h->device);
  if (!work) return fail(h, CLOMP_DEVICE_ERROR, "scratch address of device %d unresolved",
                         h->device);
  DeviceGuard dg;
  HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  HIP_TRY(launch_grad(dtype == CLOMP_F64, n, m, lda, A, x, mask, y, grad_out, grad_x, resid_out,
                      loss, work, (n + kGradColChunk - 1) / kGradColChunk, kGradColChunk, st),
          "grad");
  return CLOMP_OK;
}

clomp_status_t clomp_set_tuning(clomp_handle_t h, const clomp_tuning_t* t) {
  if (!h || !t) return CLOMP_INVALID_ARGUMENT;
  const int32_t v[5] = {t->scan_tile_kb, t->pass_tile_kb, t->team_min_rows, t->rscan_min_t,
                        t->shared_min_tiles};
  for (int32_t x : v)
    if (x < -1 || x > 65536)
      return fail(h, CLOMP_INVALID_ARGUMENT,
                  "tuning values must lie in [-1, 65536] (-1: default, 0: keep)");
  if (t->spin_limit < -1)
    return fail(h, CLOMP_INVALID_ARGUMENT, "spin_limit must be >= -1 (-1: default, 0: keep)");
  // -1 restores the default, 0 keeps the current value
  auto put = [](int32_t x, int& field, int dflt) {
    if (x == -1) field = dflt;
    else if (x > 0) field = x;
  };
  put(t->scan_tile_kb, h->scan_tile_kb, kScanTargetKB);
  put(t->pass_tile_kb, h->pass_tile_kb, kPassTargetKB);
  h->last_scan_kb = h->scan_tile_kb;
  h->last_pass_kb = h->pass_tile_kb;
  h->tuned.clear();
  put(t->team_min_rows, h->team_min_rows, kTeamMinRowsDefault);
  put(t->rscan_min_t, h->rscan_min_t, 1);
  put(t->shared_min_tiles, h->shared_min_tiles, 0);
  put(t->spin_limit, h->spin_limit, (int)kSpinLimitDefault);
  h->pcache.valid = false;
  drop_graphs(h);
  return CLOMP_OK;
}

clomp_status_t clomp_get_tuning(clomp_handle_t h, clomp_tuning_t* t) {
  if (!h || !t) return CLOMP_INVALID_ARGUMENT;
  memset(t, 0, sizeof *t);
  t->scan_tile_kb = h->last_scan_kb;
  t->pass_tile_kb = h->last_pass_kb;
  t->team_min_rows = h->team_min_rows;
  t->rscan_min_t = h->rscan_min_t;
  t->shared_min_tiles = h->shared_min_tiles > 0 ? h->shared_min_tiles
                                                : std::max(1, h->num_cu / 2);
  t->spin_limit = h->spin_limit;
  return CLOMP_OK;
}

clomp_status_t clomp_profile_reset(clomp_handle_t h) {
  if (!h) return CLOMP_INVALID_ARGUMENT;
  for (const auto& r : h->recs) (void)hipEventSynchronize(r.b);
  h->recs.clear();
  h->ev_used = 0;
  h->scan_bytes = 0.0;
  h->pass_bytes = 0.0;
  h->fused_bytes = 0.0;
  return CLOMP_OK;
}

clomp_status_t clomp_profile_read(clomp_handle_t h, clomp_profile_t* out) {
  if (!h || !out) return CLOMP_INVALID_ARGUMENT;
  memset(out, 0, sizeof *out);
  for (const auto& r : h->recs) {
    HIP_TRY(hipEventSynchronize(r.b), "hipEventSynchronize");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
    out->ms[r.phase] += ms;
    out->launches[r.phase] += 1;
  }
  out->scan_bytes = h->scan_bytes;
  out->pass_bytes = h->pass_bytes;
  out->fused_bytes = h->fused_bytes;
  return CLOMP_OK;
}

clomp_status_t clomp_destroy(clomp_handle_t h) {
  if (!h) return CLOMP_INVALID_ARGUMENT;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  drop_graphs(h);
  if (h->ws.p) (void)hipFree(h->ws.p);
  if (h->tables.p) (void)hipFree(h->tables.p);
  if (h->gwork.p) (void)hipFree(h->gwork.p);
  if (h->pinned) (void)hipHostFree(h->pinned);
  if (h->staging_free) (void)hipEventDestroy(h->staging_free);
  if (h->work_done) (void)hipEventDestroy(h->work_done);
  if (h->grad_done) (void)hipEventDestroy(h->grad_done);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  (void)hipSetDevice(prev);
  delete h;
  return CLOMP_OK;
}

}  // extern "C"
