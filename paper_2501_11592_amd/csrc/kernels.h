// Host-side launch wrappers of the CLOMP kernels (defined next to the kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace clomp {

struct Inst;
struct ScanTile;
struct RowTile;

hipError_t launch_init(const Inst* d, int count, hipStream_t s);
hipError_t launch_scan(int bf16, int lpa, const Inst* d, const ScanTile* tiles, int ntiles,
                       int r_lds_floats, int reverse, hipStream_t s);
hipError_t launch_scan_reg(int bf16, int lpa, int nch, const Inst* d, const ScanTile* tiles,
                           int ntiles, int reverse, hipStream_t s);
hipError_t launch_gram_reg(int bf16, int lpa, int nch, const Inst* d, int nact, int t, int nblk,
                           int D, float lr_rel, float eps_rel, hipStream_t s);
hipError_t launch_gram(int bf16, int lpa, const Inst* d, int nact, int t, int nblk, int D,
                       int v_lds_floats, float lr_rel, float eps_rel, hipStream_t s);
hipError_t launch_adam(const Inst* d, int nact, int t, int T, float beta1, float beta2,
                       hipStream_t s);
hipError_t launch_omp(const Inst* d, int nact, int t, hipStream_t s);
hipError_t launch_resid(int bf16, const Inst* d, const RowTile* tiles, int ntiles, int t,
                        hipStream_t s);
hipError_t launch_cg_rows(int mode, const Inst* d, const RowTile* tiles, int ntiles, int tmax,
                          int it, float tol2, hipStream_t s);
hipError_t launch_cg_dots(int mode, int lpa, const Inst* d, const int* list, int nlist, int tmax,
                          int nblk, int D, int m_pad_max, int it, hipStream_t s);
hipError_t launch_copy_s(const Inst* d, const int* list, int nlist, hipStream_t s);
hipError_t launch_qr(const Inst* d, const int* list, int nlist, size_t lds_bytes, hipStream_t s);
hipError_t launch_norm(const Inst* d, const RowTile* tiles, int ntiles, int tmax, hipStream_t s);
hipError_t launch_finalize(const Inst* d, int count, int check_cg, hipStream_t s);
hipError_t set_max_lds(size_t bytes);
// Events the next single-kernel launch records around itself (profiling).
void set_launch_events(hipEvent_t start, hipEvent_t stop);

// Normalised IHT (one iteration = optional residual, gradient scan, step
// denominator, thresholded update).  rows mode 0: r = y - A_G s_G; mode 1:
// partial ||A_G g_G||^2.  select mode 0: support = top-K |g|; mode 1: the
// normalised step and s = H_K(s + t g); mode 2: mode 1 and b = (A^T y)_S.
// grad: grid (ntiles, nslice), r_lds floats of r staged per workgroup (0:
// read from memory); combine sums the slices of signals with nslice > 1.
hipError_t launch_iht_grad(int bf16, int lpa, const Inst* d, const ScanTile* tiles, int ntiles,
                           int nslice, int r_lds, int first, hipStream_t s);
hipError_t launch_iht_combine(const Inst* d, const ScanTile* tiles, int ntiles, int first,
                              hipStream_t s);
// wide: 16 waves per row tile instead of 4 (classes with fewer row tiles than CUs).
hipError_t launch_iht_rows(int bf16, int mode, const Inst* d, const RowTile* tiles, int ntiles,
                           int kmax, int wide, hipStream_t s);
// nmax: the largest n among the signals (picks threads and chunk size).
hipError_t launch_iht_select(const Inst* dc, int nact, int mode, int nmax, hipStream_t s);

// Paper-mode CLOMP selection and gradient step of iteration `it` (one
// workgroup per signal; `last`: also gather b for the refinement; bc1/bc2:
// the Adam bias corrections 1 - beta^(it+1)).
hipError_t launch_paper_select(const Inst* dc, int nact, int it, int last, float thr,
                               float lr_rel, float beta1, float beta2, float bc1, float bc2,
                               float eps_rel, int nmax, hipStream_t s);

// Fused greedy loop of the signals list[0..count): one workgroup per signal
// with its dictionary in LDS (k_eff <= kSmallMaxK; kmax >= every k_eff of the
// list; dynamic LDS of small_lds_bytes for the largest signal).
hipError_t launch_small(int bf16, int omp, const Inst* d, const int* list, int count, int kmax,
                        int T, float beta1, float beta2, float lr_rel, float eps_rel, size_t lds,
                        hipStream_t s);

// correlation-update schedule (few large signals)
hipError_t launch_ypass(int bf16, int lpa, const Inst* d, const ScanTile* tiles, int ntiles,
                        size_t lds, hipStream_t s);
// W > 1: a team of W blocks per signal updates the coefficients (W * 16 >=
// t+1, W <= 128); the caller keeps nact * W below the CU count so that every
// member is resident at once.
hipError_t launch_coef_pass(int bf16, int lpa, int omp, const Inst* dc, int nact, int W,
                            const Inst* d, const ScanTile* tiles, int ntiles, int t, int T,
                            float beta1, float beta2, float lr_rel, float eps_rel, size_t lds,
                            hipStream_t s);
// Workgroups of a coefficient-team launch (1024 threads, `lds` bytes of
// dynamic LDS) that one compute unit can hold at once (0: none, or the query
// failed).
int coef_team_blocks_per_cu(int bf16, int lpa, int omp, size_t lds);
// shared dictionary: Gf = A^T A (ld ldh of the first signal), c0 = A^T y of
// every signal, dg = diag(Gf) (+ the prior); d[0..nsig) share A, n, m.
hipError_t launch_shared_gram(int bf16, const Inst* d, int nsig, int n, float* Gf, float* dg,
                              hipStream_t s);
// shared dictionary, CLOMP, t+1 <= 256: selection record and Adam of
// iteration t with ceil((t+1)/16) waves per signal.
hipError_t launch_coef_reg(const Inst* dc, int nact, int t, int T, float beta1, float beta2,
                            float lr_rel, float eps_rel, hipStream_t s);
// OMP, no pass in the launch: selection record and bordered-inverse update of
// iteration t in one 256-thread workgroup per signal.
hipError_t launch_coef_omp(const Inst* dc, int nact, int t, float lr_rel, float eps_rel,
                           hipStream_t s);
// shared dictionary, IHT / paper mode: g = A^T r of signals d[0..nsig) into
// gbuf (and c0 when `first`), one contraction for the batch.
hipError_t launch_shared_grad(int bf16, const Inst* d, int nsig, int n, int first,
                              hipStream_t s);
// shared dictionary, one workgroup per signal d[0..nsig), supports of t1 <=
// 256 atoms (0: each signal's own count): mode 0 r = y - A_S s, mode 1 the
// IHT step denominator ||A_S g_S||^2 as row partials.
hipError_t launch_shared_rows(int bf16, int mode, const Inst* d, int nsig, int t1,
                              hipStream_t s);
// shared dictionary: the correlation scan of iteration t of signals
// d[0..nsig) as C = A^T R over their residuals (argmax keys, slot t & 1).
hipError_t launch_shared_rscan(int bf16, const Inst* d, int nsig, int n, int t, hipStream_t s);
hipError_t launch_cscan(const Inst* d, const ScanTile* tiles, int ntiles, int t, hipStream_t s);
hipError_t set_max_lds_pass(size_t bytes);

// Image mode (CLOMP on the columns of one image with the priors of Eq. (6)
// and Eq. (7)).  init: the DCT-II synthesis basis D (n x n, ld ldd) and nzero
// floats from `zero` on cleared (the dense coefficient images and the pixel
// image, contiguous).  record: the selection of iteration t of columns
// d[0..W).  synth: pixel columns x_c = D_S s_c (t1 atoms) into X (ld ldd).
// step: Adam step number `step` (1-based) of every column on the loss with
// the priors (htv = 2 w_tv / W, wlv = w_lv), Sd_cur / Sd_next the dense
// coefficient images before / after it.
hipError_t launch_image_init(float* D, int n, long long ldd, float* zero, long long nzero,
                             hipStream_t s);
hipError_t launch_image_record(const Inst* d, int W, int t, float lr_rel, float eps_rel,
                               hipStream_t s);
hipError_t launch_image_synth(const Inst* d, int W, int t1, const float* D, long long ldd,
                              float* X, hipStream_t s);
hipError_t launch_image_step(const Inst* d, int W, int n, int t, int step, float beta1,
                             float beta2, float htv, float wlv, const float* D, long long ldd,
                             const float* X, const float* Sd_cur, float* Sd_next, hipStream_t s);

// clomp_grad kernels
hipError_t launch_grad(int f64, int n, int m, long long lda, const void* A, const void* x,
                       const unsigned char* mask, const void* y, const void* grad_out,
                       void* grad_x, void* resid_out, void* loss, void* work, int ncolchunk,
                       int colchunk, hipStream_t s);
// Allocation-free gradient: a device-resident scratch array of
// kGradScratchBytes per device.  grad_scratch_init resolves its address on
// `device` (which must be current) once; grad_scratch_ptr returns it (NULL
// before init).
constexpr size_t kGradScratchBytes = (size_t)16 << 20;
constexpr int kMaxScratchDevices = 64;
hipError_t grad_scratch_init(int device);
void* grad_scratch_ptr(int device);

}  // namespace clomp
