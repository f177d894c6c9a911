// Launch checks standing in for the library's kernel launchers (kernels.h):
// every launch the host code issues is checked against the descriptor table
// and the workspace it would touch, and against the order the method needs
// (a signal's coefficient update of iteration t after its scan of t, its scan
// of t+1 after that update and, in the correlation-update schedule, after the
// pass that writes its column h_t).  No kernel runs.  Test infrastructure
// only: the driver links it with the library's host code and mock_hip.cpp.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>
#include <vector>
#include "dev_common.h"
#include "kernels.h"

extern std::map<char*, size_t> g_allocs;

namespace {
const clomp::Inst* g_d0 = nullptr;   // descriptor table of the current solve
int g_count = 0;
long g_errors = 0, g_launches = 0;
std::map<std::string, long> g_n;
const size_t kLdsMax = 163840;

void err(const char* what, const std::string& msg) {
  if (g_errors < 40) printf("VIOLATION [%s] %s\n", what, msg.c_str());
  ++g_errors;
}
#define CHECK(cond, what, ...)                                          \
  do {                                                                  \
    if (!(cond)) {                                                      \
      char b_[512];                                                     \
      snprintf(b_, sizeof b_, __VA_ARGS__);                             \
      err(what, std::string(#cond) + ": " + b_);                        \
    }                                                                   \
  } while (0)

bool in_alloc(const void* p, size_t bytes) {
  const char* c = (const char*)p;
  auto it = g_allocs.upper_bound((char*)c);
  if (it == g_allocs.begin()) return false;
  --it;
  return c >= it->first && c + bytes <= it->first + it->second;
}

int idx_of(const clomp::Inst* p) { return (int)(p - g_d0); }

void check_range(const char* what, const clomp::Inst* d, int n) {
  CHECK(d >= g_d0 && d + n <= g_d0 + g_count, what, "insts [%d, %d) of %d", idx_of(d),
        idx_of(d) + n, g_count);
}

void check_scan_tiles(const char* what, const clomp::Inst* d, const clomp::ScanTile* tiles,
                      int ntiles, int min_keff_gt) {
  CHECK(d == g_d0, what, "tile launches index from the table base");
  for (int i = 0; i < ntiles; ++i) {
    const clomp::ScanTile& tl = tiles[i];
    CHECK(tl.inst >= 0 && tl.inst < g_count, what, "tile %d inst %d", i, tl.inst);
    if (tl.inst < 0 || tl.inst >= g_count) continue;
    const clomp::Inst& I = g_d0[tl.inst];
    CHECK(0 <= tl.j0 && tl.j0 < tl.j1 && tl.j1 <= I.n, what, "tile %d [%d,%d) n=%d", i, tl.j0,
          tl.j1, I.n);
    if (min_keff_gt >= 0)
      CHECK(I.k_eff > min_keff_gt, what, "tile %d inst %d k_eff %d <= %d", i, tl.inst, I.k_eff,
            min_keff_gt);
  }
}

void check_row_tiles(const char* what, const clomp::RowTile* tiles, int ntiles, int min_keff_gt) {
  for (int i = 0; i < ntiles; ++i) {
    const clomp::RowTile& tl = tiles[i];
    CHECK(tl.inst >= 0 && tl.inst < g_count, what, "row tile %d inst %d", i, tl.inst);
    if (tl.inst < 0 || tl.inst >= g_count) continue;
    const clomp::Inst& I = g_d0[tl.inst];
    CHECK(0 <= tl.i0 && tl.i0 < tl.i1 && tl.i1 <= I.m && tl.i1 - tl.i0 <= 64 &&
              tl.tile >= 0 && tl.tile < I.n_rowtiles,
          what, "row tile %d [%d,%d) m=%d tile %d/%d", i, tl.i0, tl.i1, I.m, tl.tile,
          I.n_rowtiles);
    if (min_keff_gt >= 0)
      CHECK(I.k_eff > min_keff_gt, what, "row tile inst %d k_eff %d <= %d", tl.inst, I.k_eff,
            min_keff_gt);
  }
}

// every workspace buffer of every descriptor inside an allocation, and no two
// buffers overlapping
void check_workspace() {
  struct Iv { const char* lo; const char* hi; int inst; const char* name; };
  std::vector<Iv> iv;
  for (int q = 0; q < g_count; ++q) {
    const clomp::Inst& I = g_d0[q];
    auto add = [&](const void* p, size_t bytes, const char* name) {
      if (!p) return;
      CHECK(in_alloc(p, bytes), "workspace", "inst %d %s (%zu bytes) outside any allocation", q,
            name, bytes);
      iv.push_back({(const char*)p, (const char*)p + bytes, q, name});
    };
    const size_t ke = I.k_eff;
    add(I.r, 8 * (size_t)I.m_pad, "r+y");
    add(I.G, 4 * ke * I.ldg, "G");
    add(I.b, 4 * ke, "b");
    add(I.s, 4 * ke, "s");
    add(I.mo, 4 * ke, "mo");
    add(I.ve, 4 * ke, "ve");
    add(I.xf, 4 * ke, "xf");
    add(I.z, 4 * ke, "z");
    add(I.Linv, 4 * ke * I.ldg, "Linv");
    add(I.cg, 4 * (3 * (size_t)I.m_pad + 3 * ke), "cg");
    add(I.c0, 4 * (size_t)I.ldh, "c0");
    if (I.H) add(I.H, 4 * (size_t)I.ldh * ke, "H");
    add(I.team, 8 * (2 * ke + 2 * clomp::kTeamMax), "team");
    add(I.gbuf, 4 * (size_t)I.ldh * I.nslice, "gbuf");
    add(I.sfull, 4 * (size_t)I.ldh, "sfull");
    add(I.mden, 4 * (size_t)I.ldh, "mden");
    add(I.vden, 4 * (size_t)I.ldh, "vden");
    add(I.npart, 8 * (size_t)I.n_rowtiles, "npart");
    add(I.qpart, 4 * (size_t)I.n_rowtiles, "qpart");
    add(I.key, 16, "key");
    add(I.bitmap, 4 * (size_t)((I.n + 31) / 32), "bitmap");
    add(I.st, sizeof(clomp::InstState), "st");
    CHECK(I.ldg >= I.k_eff, "layout", "inst %d ldg %d k_eff %d", q, I.ldg, I.k_eff);
    CHECK(I.m_pad >= I.m, "layout", "inst %d m_pad", q);
    CHECK(!I.c0 || I.ldh >= I.n, "layout", "inst %d ldh %lld n %d", q, I.ldh, I.n);
    CHECK(I.k_eff == std::min(I.k, std::min(I.m, I.n)), "layout", "inst %d k_eff", q);
  }
  // dg may be shared (shared dictionary): skip it in the overlap check
  std::sort(iv.begin(), iv.end(), [](const Iv& a, const Iv& b) { return a.lo < b.lo; });
  for (size_t i = 1; i < iv.size(); ++i)
    CHECK(iv[i].lo >= iv[i - 1].hi, "overlap", "inst %d %s overlaps inst %d %s", iv[i].inst,
          iv[i].name, iv[i - 1].inst, iv[i - 1].name);
}

// ordering: the iteration whose key each signal holds (scan), whose
// coefficient update ran last (coef) and whose h column the pass wrote (pass)
std::vector<int> g_scan, g_coef, g_pass;
void order_reset() {
  g_scan.assign(g_count, -1);
  g_coef.assign(g_count, -1);
  g_pass.assign(g_count, -1);
}

void on_coef(const char* what, int q, int t) {
  if (q < 0 || q >= g_count) return;
  CHECK(g_scan[q] == t, what, "inst %d coef of t %d before its scan (scan %d)", q, t, g_scan[q]);
  CHECK(g_coef[q] == t - 1, what, "inst %d coef of t %d after coef %d", q, t, g_coef[q]);
  g_coef[q] = t;
}

void on_pass(const char* what, int q, int t) {
  if (q < 0 || q >= g_count) return;
  CHECK(g_scan[q] == t, what, "inst %d pass of t %d before its scan (scan %d)", q, t, g_scan[q]);
  g_pass[q] = std::max(g_pass[q], t);
}

// a scan of iteration t reads the coefficients of t-1 and (correlation-
// update schedule) the h column of t-1
void on_scan(const char* what, int q, int t, bool need_pass) {
  if (q < 0 || q >= g_count) return;
  if (t > 0) {
    CHECK(g_coef[q] == t - 1, what, "inst %d scan of t %d with coef %d", q, t, g_coef[q]);
    if (need_pass)
      CHECK(g_pass[q] == t - 1, what, "inst %d scan of t %d with pass %d", q, t, g_pass[q]);
  }
  g_scan[q] = std::max(g_scan[q], t);
}

void count(const char* name) {
  ++g_launches;
  ++g_n[name];
}
}  // namespace

void harness_report() {
  printf("launches %ld, violations %ld\n", g_launches, g_errors);
  for (auto& kv : g_n) printf("  %-16s %ld\n", kv.first.c_str(), kv.second);
}
long harness_errors() { return g_errors; }

namespace clomp {
void set_launch_events(hipEvent_t, hipEvent_t) {}
hipError_t set_max_lds(size_t) { return hipSuccess; }
hipError_t set_max_lds_pass(size_t) { return hipSuccess; }
// two 1024-thread workgroups per compute unit while their LDS fits
int coef_team_blocks_per_cu(int, int, int, size_t lds) { return lds <= 64 * 1024 ? 2 : 1; }
hipError_t grad_scratch_init(int) { return hipSuccess; }
void* grad_scratch_ptr(int) { return nullptr; }
hipError_t launch_grad(int, int, int, long long, const void*, const void*, const unsigned char*,
                       const void*, const void*, void*, void*, void*, void*, int, int,
                       hipStream_t) { return hipSuccess; }

hipError_t launch_init(const Inst* d, int count_, hipStream_t) {
  count("init");
  g_d0 = d;
  g_count = count_;
  CHECK(in_alloc(d, sizeof(Inst) * count_), "init", "descriptor table outside the tables");
  check_workspace();
  order_reset();
  return hipSuccess;
}
hipError_t launch_small(int, int, const Inst* d, const int* list, int n, int kmax, int, float,
                        float, float, float, size_t lds, hipStream_t) {
  count("small");
  CHECK(d == g_d0, "small", "base");
  CHECK(lds + 2048 <= kLdsMax, "small", "lds %zu", lds);
  CHECK(kmax >= 1 && kmax <= kSmallMaxK, "small", "kmax %d", kmax);
  for (int i = 0; i < n; ++i) {
    CHECK(list[i] >= 0 && list[i] < g_count, "small", "list %d", list[i]);
    if (list[i] < 0 || list[i] >= g_count) continue;
    const Inst& I = d[list[i]];
    CHECK(I.k_eff <= kmax, "small", "inst %d k_eff %d above kmax %d", list[i], I.k_eff, kmax);
    CHECK(I.k_eff <= kSmallMaxK && small_lds_bytes(I.n, I.m, I.k_eff) <= lds, "small",
          "inst %d k_eff %d lds %zu > %zu", list[i], I.k_eff, small_lds_bytes(I.n, I.m, I.k_eff),
          lds);
  }
  return hipSuccess;
}
hipError_t launch_ypass(int bf16, int, const Inst* d, const ScanTile* tiles, int ntiles,
                        size_t lds, hipStream_t) {
  count("ypass");
  check_scan_tiles("ypass", d, tiles, ntiles, -1);
  for (int i = 0; i < ntiles; ++i) {
    const Inst& I = d[tiles[i].inst];
    const int vw = bf16 ? 8 : 4;
    CHECK((size_t)((I.m + vw - 1) / vw * vw) * 4 <= lds, "ypass", "lds %zu m %d", lds, I.m);
    CHECK(I.c0 && I.dg, "ypass", "inst %d without c0/dg", tiles[i].inst);
  }
  CHECK(lds + 34 * 1024 <= kLdsMax, "ypass", "lds %zu", lds);
  for (int i = 0; i < ntiles; ++i) on_scan("ypass", tiles[i].inst, 0, false);
  return hipSuccess;
}
hipError_t launch_coef_pass(int bf16, int, int omp, const Inst* dc, int nact, int W,
                            const Inst* d, const ScanTile* tiles, int ntiles, int t, int,
                            float, float, float, float, size_t lds, hipStream_t) {
  count("coef_pass");
  CHECK(d == g_d0, "coef_pass", "base");
  check_range("coef_pass", dc, nact);
  if (nact > 0 && ntiles == 0) count("coef_only");
  if (nact == 0) count("pass_only");
  if (W > 1) CHECK((long long)nact * W <= 248, "coef_pass", "teams %d x %d", nact, W);
  for (int q = 0; q < nact; ++q) {
    const Inst& I = dc[q];
    CHECK(I.k_eff > t, "coef_pass", "coef inst %d k_eff %d t %d", idx_of(dc + q), I.k_eff, t);
    const size_t t1 = t + 1;
    if (omp && W == 1) CHECK(6 * t1 * 4 <= lds, "coef_pass", "omp lds %zu t1 %zu", lds, t1);
    if (!omp && W == 1 && t1 > 256 && t1 <= 1024)
      CHECK((size_t)kSplitLdsFloats * 4 <= lds, "coef_pass", "split lds %zu", lds);
    if (W > 1) CHECK((t1 + 36) * 4 <= lds && W * 16 >= (int)t1, "coef_pass", "team W %d t1 %zu", W, t1);
    CHECK(I.H || I.Gf, "coef_pass", "inst without H");
    on_coef("coef_pass", idx_of(dc + q), t);
  }
  check_scan_tiles("coef_pass", d, tiles, ntiles, t + 1);
  for (int i = 0; i < ntiles; ++i) {
    const Inst& I = d[tiles[i].inst];
    const int vw = bf16 ? 8 : 4;
    const size_t need = bf16 ? (size_t)((I.m + 7) / 8) * 16 : (size_t)((I.m + vw - 1) / vw * vw) * 4;
    CHECK(need <= lds, "coef_pass", "pass lds %zu < %zu (m %d)", lds, need, I.m);
    CHECK(I.H != nullptr, "coef_pass", "pass tile inst without H");
    on_pass("coef_pass", tiles[i].inst, t);
  }
  CHECK(lds + 34 * 1024 <= kLdsMax, "coef_pass", "lds %zu", lds);
  return hipSuccess;
}
hipError_t launch_cscan(const Inst* d, const ScanTile* tiles, int ntiles, int t, hipStream_t) {
  count("cscan");
  check_scan_tiles("cscan", d, tiles, ntiles, t);
  for (int i = 0; i < ntiles; ++i) {
    CHECK(tiles[i].j0 % 256 == 0 && tiles[i].j1 - tiles[i].j0 <= 256, "cscan",
          "tile %d [%d,%d) not a 256-atom tile", i, tiles[i].j0, tiles[i].j1);
    const Inst& I = d[tiles[i].inst];
    on_scan("cscan", tiles[i].inst, t, I.Gf == nullptr);
  }
  return hipSuccess;
}
hipError_t launch_coef_reg(const Inst* dc, int nact, int t, int, float, float, float, float,
                           hipStream_t) {
  count("coef_reg");
  check_range("coef_reg", dc, nact);
  CHECK(t + 1 <= 256, "coef_reg", "t1 %d", t + 1);
  for (int q = 0; q < nact; ++q) {
    CHECK(dc[q].k_eff > t, "coef_reg", "k_eff");
    on_coef("coef_reg", idx_of(dc + q), t);
  }
  return hipSuccess;
}
hipError_t launch_coef_omp(const Inst* dc, int nact, int t, float, float, hipStream_t) {
  count("coef_omp");
  check_range("coef_omp", dc, nact);
  for (int q = 0; q < nact; ++q) {
    CHECK(dc[q].k_eff > t, "coef_omp", "k_eff");
    on_coef("coef_omp", idx_of(dc + q), t);
  }
  return hipSuccess;
}
hipError_t launch_qr(const Inst* d, const int* list, int nlist, size_t lds, hipStream_t) {
  count("qr");
  CHECK(lds <= kLdsMax - 2048, "qr", "lds %zu", lds);
  for (int i = 0; i < nlist; ++i) {
    CHECK(list[i] >= 0 && list[i] < g_count, "qr", "list");
    const Inst& I = d[list[i]];
    const size_t mr = I.m + (I.tvw != 0.f ? I.k_eff : 0);
    CHECK((mr * I.k_eff + mr + 4 * (size_t)I.k_eff) * 4 <= lds, "qr", "inst %d needs %zu > %zu",
          list[i], (mr * I.k_eff + mr + 4 * (size_t)I.k_eff) * 4, lds);
    CHECK(I.cg_slot < 0, "qr", "inst %d has a CG slot", list[i]);
  }
  return hipSuccess;
}
hipError_t launch_copy_s(const Inst* d, const int* list, int nlist, hipStream_t) {
  count("copy_s");
  CHECK(d == g_d0, "copy_s", "base");
  if (!list) CHECK(nlist == g_count, "copy_s", "all %d of %d", nlist, g_count);
  else for (int i = 0; i < nlist; ++i) CHECK(list[i] >= 0 && list[i] < g_count && d[list[i]].cg, "copy_s", "list");
  return hipSuccess;
}
hipError_t launch_cg_rows(int, const Inst* d, const RowTile* tiles, int ntiles, int tmax, int,
                          float, hipStream_t) {
  count("cg_rows");
  CHECK(d == g_d0, "cg_rows", "base");
  check_row_tiles("cg_rows", tiles, ntiles, -1);
  for (int i = 0; i < ntiles; ++i) {
    const Inst& I = d[tiles[i].inst];
    CHECK(I.cg && I.k_eff <= tmax, "cg_rows", "inst %d cg %p k_eff %d tmax %d", tiles[i].inst,
          (void*)I.cg, I.k_eff, tmax);
  }
  return hipSuccess;
}
hipError_t launch_cg_dots(int, int, const Inst* d, const int* list, int nlist, int tmax, int nblk,
                          int D, int m_pad_max, int, hipStream_t) {
  count("cg_dots");
  for (int i = 0; i < nlist; ++i) {
    CHECK(list[i] >= 0 && list[i] < g_count, "cg_dots", "list");
    const Inst& I = d[list[i]];
    CHECK(I.cg && I.k_eff <= tmax && I.m_pad <= m_pad_max, "cg_dots", "inst %d", list[i]);
  }
  CHECK((long long)nblk * D >= tmax, "cg_dots", "nblk %d D %d tmax %d", nblk, D, tmax);
  CHECK((size_t)m_pad_max * 4 + 1024 <= kLdsMax, "cg_dots", "m_pad_max %d", m_pad_max);
  return hipSuccess;
}
hipError_t launch_norm(const Inst* d, const RowTile* tiles, int ntiles, int tmax, hipStream_t) {
  count("norm");
  CHECK(d == g_d0, "norm", "base");
  check_row_tiles("norm", tiles, ntiles, -1);
  for (int i = 0; i < ntiles; ++i)
    CHECK(d[tiles[i].inst].k_eff <= tmax, "norm", "inst %d k_eff %d > tmax %d", tiles[i].inst,
          d[tiles[i].inst].k_eff, tmax);
  CHECK((size_t)2 * (tmax + 1) * 4 <= kLdsMax, "norm", "tmax %d", tmax);
  return hipSuccess;
}
hipError_t launch_finalize(const Inst* d, int n, int, hipStream_t) {
  count("finalize");
  CHECK(d == g_d0 && n == g_count, "finalize", "count");
  return hipSuccess;
}
hipError_t launch_image_init(float* D, int n, long long ldd, float* zero, long long nzero,
                             hipStream_t) {
  count("image_init");
  CHECK(in_alloc(D, sizeof(float) * (size_t)n * ldd), "image_init", "D outside");
  CHECK(in_alloc(zero, sizeof(float) * (size_t)nzero), "image_init", "zeroed range outside");
  CHECK(ldd >= n, "image_init", "ldd");
  return hipSuccess;
}
hipError_t launch_image_record(const Inst* d, int W, int t, float, float, hipStream_t) {
  count("image_record");
  check_range("image_record", d, W);
  for (int q = 0; q < W; ++q) {
    CHECK(d[q].k_eff > t && d[q].Gf, "image_record", "inst %d", q);
    on_coef("image_record", idx_of(d + q), t);
  }
  return hipSuccess;
}
hipError_t launch_image_synth(const Inst* d, int W, int t1, const float* D, long long ldd,
                              float* X, hipStream_t) {
  count("image_synth");
  check_range("image_synth", d, W);
  CHECK(t1 <= kImageMaxK, "image_synth", "t1");
  CHECK(in_alloc(X, sizeof(float) * (size_t)ldd * W), "image_synth", "X outside");
  for (int q = 0; q < W; ++q)
    CHECK(d[q].col >= 0 && d[q].col < W && d[q].k_eff >= t1 && d[q].n <= ldd, "image_synth",
          "inst %d col %d", q, d[q].col);
  return hipSuccess;
}
hipError_t launch_image_step(const Inst* d, int W, int n, int t, int, float, float, float,
                             float wlv, const float* D, long long ldd, const float* X,
                             const float* cur, float* nxt, hipStream_t) {
  count("image_step");
  check_range("image_step", d, W);
  CHECK(t + 1 <= kImageMaxK && n <= kImageMaxN, "image_step", "sizes");
  const size_t lds = (wlv != 0.f && n >= 3 && W >= 3) ? (size_t)6 * n * 4 : 0;
  CHECK(lds + 3 * 4 * kImageMaxK <= kLdsMax, "image_step", "lds %zu", lds);
  CHECK(in_alloc(cur, sizeof(float) * (size_t)ldd * W) && in_alloc(nxt, sizeof(float) * (size_t)ldd * W),
        "image_step", "coefficient images outside");
  CHECK(cur != nxt, "image_step", "ping-pong");
  for (int q = 0; q < W; ++q)
    CHECK(d[q].col >= 0 && d[q].col < W && d[q].k_eff > t && d[q].n == n, "image_step",
          "inst %d", q);
  return hipSuccess;
}
// residual schedule and the rest: ranges only
hipError_t launch_scan(int, int, const Inst* d, const ScanTile* tiles, int ntiles, int, int,
                       hipStream_t) { count("scan"); check_scan_tiles("scan", d, tiles, ntiles, -1); return hipSuccess; }
hipError_t launch_scan_reg(int, int, int, const Inst* d, const ScanTile* tiles, int ntiles, int,
                           hipStream_t) { count("scan_reg"); check_scan_tiles("scan_reg", d, tiles, ntiles, -1); return hipSuccess; }
hipError_t launch_gram_reg(int, int, int, const Inst* d, int nact, int, int, int, float, float,
                           hipStream_t) { count("gram_reg"); check_range("gram_reg", d, nact); return hipSuccess; }
hipError_t launch_gram(int, int, const Inst* d, int nact, int, int, int, int, float, float,
                       hipStream_t) { count("gram"); check_range("gram", d, nact); return hipSuccess; }
hipError_t launch_adam(const Inst* d, int nact, int t, int, float, float, hipStream_t) {
  count("adam"); check_range("adam", d, nact);
  for (int q = 0; q < nact; ++q) CHECK(d[q].k_eff > t, "adam", "k_eff");
  return hipSuccess;
}
hipError_t launch_omp(const Inst* d, int nact, int t, hipStream_t) {
  count("omp"); check_range("omp", d, nact);
  for (int q = 0; q < nact; ++q) CHECK(d[q].k_eff > t, "omp", "k_eff");
  return hipSuccess;
}
hipError_t launch_resid(int, const Inst* d, const RowTile* tiles, int ntiles, int t, hipStream_t) {
  count("resid"); CHECK(d == g_d0, "resid", "base"); check_row_tiles("resid", tiles, ntiles, t);
  return hipSuccess;
}
hipError_t launch_iht_grad(int, int, const Inst* d, const ScanTile* tiles, int ntiles, int, int,
                           int, hipStream_t) { count("iht_grad"); check_scan_tiles("iht_grad", d, tiles, ntiles, -1); return hipSuccess; }
hipError_t launch_iht_combine(const Inst* d, const ScanTile* tiles, int ntiles, int,
                              hipStream_t) { count("iht_combine"); check_scan_tiles("iht_combine", d, tiles, ntiles, -1); return hipSuccess; }
hipError_t launch_iht_rows(int, int, const Inst* d, const RowTile* tiles, int ntiles, int, int,
                           hipStream_t) { count("iht_rows"); CHECK(d == g_d0, "iht_rows", "base"); check_row_tiles("iht_rows", tiles, ntiles, -1); return hipSuccess; }
hipError_t launch_iht_select(const Inst* dc, int nact, int, int, hipStream_t) { count("iht_select"); check_range("iht_select", dc, nact); return hipSuccess; }
hipError_t launch_paper_select(const Inst* dc, int nact, int, int, float, float, float, float,
                               float, float, float, int, hipStream_t) { count("paper_select"); check_range("paper_select", dc, nact); return hipSuccess; }
hipError_t launch_shared_gram(int, const Inst* d, int nsig, int, float*, float*, hipStream_t) { count("shared_gram"); check_range("shared_gram", d, nsig); return hipSuccess; }
hipError_t launch_shared_rows(int, int, const Inst* d, int nsig, int, hipStream_t) { count("shared_rows"); check_range("shared_rows", d, nsig); return hipSuccess; }
hipError_t launch_shared_grad(int, const Inst* d, int nsig, int, int, hipStream_t) { count("shared_grad"); check_range("shared_grad", d, nsig); return hipSuccess; }
hipError_t launch_shared_rscan(int, const Inst* d, int nsig, int, int t, hipStream_t) {
  count("shared_rscan"); check_range("shared_rscan", d, nsig);
  for (int q = 0; q < nsig; ++q) on_scan("shared_rscan", idx_of(d + q), t, false);
  return hipSuccess;
}
}  // namespace clomp
