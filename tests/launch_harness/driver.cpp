// Drives the library's host code (clomp_create, clomp_set_tuning,
// clomp_solve_batch) on a batch read from a text file, with every launch
// checked by mock_launchers.cpp instead of run.  Test infrastructure only.
//
//   driver SPECS METHOD FLAGS DTYPE SHARED TEAM_MIN_ROWS PRIOR_TV PRIOR_LV
//
// SPECS holds one instance per line, "n m k".  DTYPE is 0 (FP32 bulk) or 1
// (BF16 bulk with an FP32 master).  SHARED = 1 gives every instance the same
// A (and master).  TEAM_MIN_ROWS 0 keeps the library's default.  The
// pointers are distinct fake device addresses: nothing dereferences them.
// Prints the solve status, the launch and violation counts and the count per
// launcher; exits 0 when the solve returned CLOMP_OK and no check failed, 3
// on a failed check, 4 when the solve returned another status.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "clomp.h"

void harness_report();
long harness_errors();

int main(int argc, char** argv) {
  if (argc != 9) {
    fprintf(stderr, "usage: driver SPECS METHOD FLAGS DTYPE SHARED TEAM_MIN_ROWS PRIOR_TV PRIOR_LV\n");
    return 2;
  }
  FILE* f = fopen(argv[1], "r");
  if (!f) return 2;
  const int method = atoi(argv[2]);
  const unsigned flags = (unsigned)strtoul(argv[3], nullptr, 10);
  const int bf16 = atoi(argv[4]);
  const int shared = atoi(argv[5]);
  const int tmr = atoi(argv[6]);
  const float prior_tv = (float)atof(argv[7]);
  const float prior_lv = (float)atof(argv[8]);
  unsigned long long next = 0x100000000000ull;
  auto fake = [&](size_t bytes) {
    void* p = reinterpret_cast<void*>(next);
    next += (bytes + 4095) / 4096 * 4096 + 4096;
    return p;
  };
  std::vector<clomp_instance_t> inst;
  void* A = nullptr;
  void* Am = nullptr;
  int n, m, k;
  while (fscanf(f, "%d %d %d", &n, &m, &k) == 3) {
    clomp_instance_t I = {};
    I.n = n;
    I.m = m;
    I.k = k;
    I.lda = bf16 ? (m + 7) / 8 * 8 : (m + 3) / 4 * 4;
    I.lda_master = bf16 ? (m + 3) / 4 * 4 : 0;
    if (!shared || !A) {
      A = fake((size_t)n * I.lda * (bf16 ? 2 : 4));
      Am = bf16 ? fake((size_t)n * I.lda_master * 4) : nullptr;
    }
    I.A = A;
    I.A_master = static_cast<const float*>(Am);
    I.y = static_cast<const float*>(fake(4 * (size_t)m));
    I.x = static_cast<float*>(fake(4 * (size_t)n));
    I.support = static_cast<int32_t*>(fake(4 * (size_t)k));
    I.n_selected = static_cast<int32_t*>(fake(4));
    I.resid_norm = static_cast<double*>(fake(8));
    I.status = static_cast<uint32_t*>(fake(4));
    inst.push_back(I);
  }
  fclose(f);
  clomp_params_t p;
  clomp_default_params(&p);
  p.method = (clomp_method_t)method;
  p.flags = flags;
  p.prior_tv = prior_tv;
  p.prior_lv = prior_lv;
  clomp_handle_t h = nullptr;
  clomp_status_t s = clomp_create(&h, 0, &p);
  if (s != CLOMP_OK) {
    printf("create %s\n", clomp_status_string(s));
    return 4;
  }
  if (tmr > 0) {
    clomp_tuning_t t = {};
    t.team_min_rows = tmr;
    if ((s = clomp_set_tuning(h, &t)) != CLOMP_OK) {
      printf("tuning %s: %s\n", clomp_status_string(s), clomp_last_error(h));
      return 4;
    }
  }
  s = clomp_solve_batch(h, inst.data(), (int32_t)inst.size(), bf16 ? CLOMP_BF16 : CLOMP_F32,
                        reinterpret_cast<void*>(0x1));
  printf("solve %s %s\n", clomp_status_string(s), s == CLOMP_OK ? "" : clomp_last_error(h));
  fflush(stdout);
  harness_report();
  clomp_destroy(h);
  if (harness_errors()) return 3;
  return s == CLOMP_OK ? 0 : 4;
}
