// HIP kernels (gfx950) of the CLOMP / OMP greedy loop, phase by phase.
//
// One outer iteration t for every active instance is four launches:
//   scan   c = A^T r over all atoms, |c| + exclusion + packed argmax key
//          (residual injection and unit-step selection of the CLOMP figure;
//          Methods, "Coefficients learning on OMP")
//   gram   decode the winner j, OR it into the mask, append it to the support,
//          and form the new Gram column A_S^T a_j and b_t = a_j^T y
//   coef   CLOMP: T Adam steps on the masked coefficients with gradient
//          G s - b = A_S^T (A_S s - y);  OMP: inverse-Cholesky update and the
//          least-squares coefficients (the OMP s-forward, table of s-forward
//          blocks)
//   resid  r = y - A_S s (the new y' of the s-forward branch, subtracted)
// followed once by refinement (in-LDS Householder QR or CGLS on the FP32
// master columns) and the FP64 residual norm of Eq. (2).
//
// Every kernel uses 256-thread workgroups; reductions run in a fixed order,
// so results are bit-reproducible.

#include <hip/hip_ext.h>

#include "dev_common.h"
#include "kernels.h"

namespace clomp {

// Profiling: when set, the next launch records these events itself
// (hipExtLaunchKernelGGL), so their interval is exactly that kernel's run.
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;
void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  g_ev_start = start;
  g_ev_stop = stop;
}

#define CLOMP_LAUNCH(kern, grid, block, shm, strm, ...)                                   \
  do {                                                                                     \
    if (g_ev_start)                                                                        \
      hipExtLaunchKernelGGL(kern, grid, block, shm, strm, g_ev_start, g_ev_stop, 0,         \
                            __VA_ARGS__);                                                  \
    else                                                                                   \
      hipLaunchKernelGGL(kern, grid, block, shm, strm, __VA_ARGS__);                       \
  } while (0)

// ============================================================ init
// One workgroup per instance: zero the outputs and the per-instance state,
// copy y into the workspace (zero padded), flag y == 0 and k > min(m, n).
__global__ __launch_bounds__(kBlock) void init_kernel(const Inst* __restrict__ insts) {
  const Inst I = insts[blockIdx.x];
  __shared__ int any_nz;
  if (threadIdx.x == 0) any_nz = 0;
  __syncthreads();
  int nz = 0;
  for (int i = threadIdx.x; i < I.m_pad; i += kBlock) {
    const float v = (i < I.m) ? I.y[i] : 0.f;
    I.r[i] = v;            // r = y at t = 0
    I.r[I.m_pad + i] = v;  // yw: the workspace copy of y follows r
    nz |= (v != 0.f);
  }
  if (nz) atomicOr(&any_nz, 1);
  for (int i = threadIdx.x; i < I.n; i += kBlock) I.x[i] = 0.f;
  for (int i = threadIdx.x; i < I.k; i += kBlock) I.support[i] = -1;
  for (int i = threadIdx.x; i < (I.n + 31) / 32; i += kBlock) I.bitmap[i] = 0u;
  for (int i = threadIdx.x; i < I.k_eff; i += kBlock) {
    I.s[i] = 0.f; I.mo[i] = 0.f; I.ve[i] = 0.f; I.xf[i] = 0.f; I.z[i] = 0.f;
  }
  if (I.team)   // tag 0 is never awaited
    for (int i = threadIdx.x; i < 2 * I.k_eff + 2 * kTeamMax; i += kBlock) I.team[i] = 0ull;
  if (I.sfull)
    for (int i = threadIdx.x; i < I.n; i += kBlock) I.sfull[i] = 0.f;
  if (I.mden)
    for (int i = threadIdx.x; i < I.n; i += kBlock) {
      I.mden[i] = 0.f;
      I.vden[i] = 0.f;
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    InstState st = {};
    st.done = any_nz ? 0 : 1;
    *I.st = st;
    I.key[0] = 0ull;
    I.key[1] = 0ull;
    *I.nsel = 0;
    unsigned status = (I.k > I.k_eff) ? ST_K_CAPPED : 0u;
    if (!any_nz) status |= ST_ZERO_Y;
    *I.status = status;
  }
}

// ============================================================ scan
// Tile = atoms [j0, j1) of one instance.  LPA lanes cooperate on one atom,
// each lane streaming 16-byte vectors of the column; r is staged in LDS when
// it fits.  The workgroup's best key goes to the instance key by atomicMax.
// Partial dot of column `col` with r over the vectors [cbeg, cend) that lane
// gl of LPA lanes visits; rv holds r from vector cbeg on (zero padded past m).
// Called once with an LDS copy and once with r in memory, so that each
// instance is compiled for its own memory (a pointer that may name either
// compiles to flat loads, whose waits also cover the outstanding HBM loads).
template <typename TA, int LPA, int UNR>
__device__ inline float span_dot(const TA* __restrict__ col, const float* __restrict__ rv,
                                 int cbeg, int cend, int nvec, int tail, int gl) {
  constexpr int VW = Vec<TA>::W;
  float acc = 0.f;
#pragma unroll UNR
  for (int c = cbeg + gl; c < cend; c += LPA) {
    float v[VW];
    Vec<TA>::load(col + (long long)c * VW, v);
    if (c == nvec - 1) {
#pragma unroll
      for (int e = 0; e < VW; ++e) v[e] = (e < tail) ? v[e] : 0.f;
    }
    const float* rr = rv + (c - cbeg) * VW;
#pragma unroll
    for (int e = 0; e < VW; ++e) acc = fmaf(v[e], rr[e], acc);
  }
  return acc;
}

template <typename TA, int LPA>
__global__ __launch_bounds__(kBlock) void scan_kernel(const Inst* __restrict__ insts,
                                                      const ScanTile* __restrict__ tiles,
                                                      int r_in_lds, int reverse) {
  extern __shared__ __align__(16) float smem[];
  __shared__ unsigned long long wbest[kWaves];
  // Odd iterations walk the tiles backwards, so a scan starts on the columns
  // the previous scan streamed last (still resident in the memory-side cache
  // when the dictionary is about the cache's size).
  const ScanTile tile = tiles[reverse ? (gridDim.x - 1 - blockIdx.x) : blockIdx.x];
  const Inst& I = insts[tile.inst];
  if (I.st->done) return;
  constexpr int VW = Vec<TA>::W;
  const int m = I.m;
  const int nvec = (m + VW - 1) / VW;
  if (r_in_lds) {
    for (int i = threadIdx.x; i < nvec * VW; i += kBlock) smem[i] = I.r[i];
    __syncthreads();
  }
  const TA* A = reinterpret_cast<const TA*>(I.A);
  const long long lda = I.lda;
  const unsigned* bitmap = I.bitmap;
  const int gl = threadIdx.x % LPA;
  const int grp = threadIdx.x / LPA;
  constexpr int NG = kBlock / LPA;
  const int tail = m - (nvec - 1) * VW;  // valid entries in the last vector
  unsigned long long best = 0ull;
  for (int j = tile.j0 + grp; j < tile.j1; j += NG) {
    const TA* col = A + (long long)j * lda;
    float acc = r_in_lds ? span_dot<TA, LPA, 8>(col, smem, 0, nvec, nvec, tail, gl)
                         : span_dot<TA, LPA, 8>(col, I.r, 0, nvec, nvec, tail, gl);
    acc = group_sum<LPA>(acc);
    const unsigned sel = (bitmap[j >> 5] >> (j & 31)) & 1u;
    const unsigned long long key = sel ? 0ull : pack_key(acc, j);
    best = key > best ? key : best;
  }
  best = wave_max_u64(best);
  if ((threadIdx.x & 63) == 0) wbest[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long b = wbest[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) b = wbest[w] > b ? wbest[w] : b;
    if (b) atomicMax(I.key, b);
  }
}

// Register variant: when every lane's share of a column is at most NCH
// vectors, r lives in registers and each atom's NCH loads are issued together
// (no LDS staging, no barrier before streaming starts).
template <typename TA, int LPA, int NCH>
__global__ __launch_bounds__(kBlock) void scan_reg_kernel(const Inst* __restrict__ insts,
                                                          const ScanTile* __restrict__ tiles,
                                                          int reverse) {
  __shared__ unsigned long long wbest[kWaves];
  const ScanTile tile = tiles[reverse ? (gridDim.x - 1 - blockIdx.x) : blockIdx.x];
  const Inst& I = insts[tile.inst];
  if (I.st->done) return;
  constexpr int VW = Vec<TA>::W;
  const int m = I.m;
  const int nvec = (m + VW - 1) / VW;
  const int tail = m - (nvec - 1) * VW;
  const int gl = threadIdx.x % LPA;
  const int grp = threadIdx.x / LPA;
  constexpr int NG = kBlock / LPA;
  float rr[NCH][VW];
#pragma unroll
  for (int q = 0; q < NCH; ++q) {
    const int c = gl + q * LPA;
#pragma unroll
    for (int e = 0; e < VW; ++e) rr[q][e] = (c < nvec) ? I.r[c * VW + e] : 0.f;
  }
  const TA* A = reinterpret_cast<const TA*>(I.A);
  const long long lda = I.lda;
  const unsigned* bitmap = I.bitmap;
  unsigned long long best = 0ull;
  for (int j = tile.j0 + grp; j < tile.j1; j += NG) {
    const TA* col = A + (long long)j * lda;
    float v[NCH][VW];
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
      const int c = gl + q * LPA;
      if (c < nvec) {
        Vec<TA>::load(col + (long long)c * VW, v[q]);
      } else {
#pragma unroll
        for (int e = 0; e < VW; ++e) v[q][e] = 0.f;
      }
      if (c == nvec - 1) {
#pragma unroll
        for (int e = 0; e < VW; ++e) v[q][e] = (e < tail) ? v[q][e] : 0.f;
      }
    }
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < NCH; ++q)
#pragma unroll
      for (int e = 0; e < VW; ++e) acc[e & 3] = fmaf(v[q][e], rr[q][e], acc[e & 3]);
    float a = group_sum<LPA>((acc[0] + acc[1]) + (acc[2] + acc[3]));
    const unsigned sel = (bitmap[j >> 5] >> (j & 31)) & 1u;
    const unsigned long long key = sel ? 0ull : pack_key(a, j);
    best = key > best ? key : best;
  }
  best = wave_max_u64(best);
  if ((threadIdx.x & 63) == 0) wbest[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long b = wbest[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) b = wbest[w] > b ? wbest[w] : b;
    if (b) atomicMax(I.key, b);
  }
}

// ============================================================ dot helper
// LPA-lane dot product of a bulk column with a float vector v (zero padded).
template <typename TA, int LPA>
__device__ inline float col_dot(const TA* col, const float* v, int m, int gl) {
  constexpr int VW = Vec<TA>::W;
  const int nvec = (m + VW - 1) / VW;
  const int tail = m - (nvec - 1) * VW;
  float acc = 0.f;
#pragma unroll 4
  for (int c = gl; c < nvec; c += LPA) {
    float a[VW];
    Vec<TA>::load(col + (long long)c * VW, a);
    if (c == nvec - 1) {
#pragma unroll
      for (int e = 0; e < VW; ++e) a[e] = (e < tail) ? a[e] : 0.f;
    }
    const float* vv = v + c * VW;
#pragma unroll
    for (int e = 0; e < VW; ++e) acc = fmaf(a[e], vv[e], acc);
  }
  return group_sum<LPA>(acc);
}

// ============================================================ gram
// grid = nact * nblk; block (i, b) handles dots l in [b*D, min((b+1)*D, t+2)):
//   l <  t : g_l = a_{S_l}^T a_j      l == t : a_j^T a_j      l == t+1 : a_j^T y
// Block 0 of each instance also records the selection.
template <typename TA, int LPA>
__global__ __launch_bounds__(kBlock) void gram_kernel(const Inst* __restrict__ insts, int t,
                                                      int nblk, int D, int v_in_lds,
                                                      float lr_rel, float eps_rel) {
  extern __shared__ __align__(16) float smem[];
  const int ii = blockIdx.x / nblk;
  const int blk = blockIdx.x - ii * nblk;
  const Inst& I = insts[ii];
  if (I.st->done) return;
  const unsigned long long key = *I.key;
  const int j = key_index(key);
  if (key == 0ull || j < 0 || j >= I.n) {
    // no candidate reached the key: stop this instance rather than index
    // outside A (cannot happen while k_eff <= n unselected atoms remain)
    if (blk == 0 && threadIdx.x == 0) {
      I.st->done = 1;
      atomicOr(I.status, ST_WATCHDOG);
    }
    return;
  }
  const int m = I.m;
  const TA* A = reinterpret_cast<const TA*>(I.A);
  const long long lda = I.lda;
  const TA* colj = A + (long long)j * lda;
  constexpr int VW = Vec<TA>::W;
  const int nvec = (m + VW - 1) / VW;
  // a_j as float, zero padded to nvec*VW
  float* aj = smem;
  if (v_in_lds) {
    for (int c = threadIdx.x; c < nvec; c += kBlock) {
      float a[VW];
      Vec<TA>::load(colj + (long long)c * VW, a);
#pragma unroll
      for (int e = 0; e < VW; ++e) aj[c * VW + e] = (c * VW + e < m) ? a[e] : 0.f;
    }
    __syncthreads();
  }
  const float* yw = I.r + I.m_pad;
  const int gl = threadIdx.x % LPA;
  const int grp = threadIdx.x / LPA;
  constexpr int NG = kBlock / LPA;
  const int l0 = blk * D;
  const int l1 = min(l0 + D, t + 2);
  for (int l = l0 + grp; l < l1; l += NG) {
    float v;
    if (l <= t) {
      const int col = (l < t) ? I.support[l] : j;
      if (v_in_lds) {
        v = col_dot<TA, LPA>(A + (long long)col * lda, aj, m, gl);
      } else {
        // a_j streamed from global: dot of two bulk columns
        const TA* ca = A + (long long)col * lda;
        float acc = 0.f;
        for (int c = gl; c < nvec; c += LPA) {
          float a[VW], bq[VW];
          Vec<TA>::load(ca + (long long)c * VW, a);
          Vec<TA>::load(colj + (long long)c * VW, bq);
#pragma unroll
          for (int e = 0; e < VW; ++e)
            acc = (c * VW + e < m) ? fmaf(a[e], bq[e], acc) : acc;
        }
        v = group_sum<LPA>(acc);
      }
      if (gl == 0) {
        if (l == t) v += tv_diag(I, j);
        I.G[l + (long long)t * I.ldg] = v;
        I.G[t + (long long)l * I.ldg] = v;
      }
    } else {
      float acc = 0.f;
      for (int c = gl; c < nvec; c += LPA) {
        float a[VW];
        Vec<TA>::load(colj + (long long)c * VW, a);
#pragma unroll
        for (int e = 0; e < VW; ++e)
          acc = (c * VW + e < m) ? fmaf(a[e], yw[c * VW + e], acc) : acc;
      }
      v = group_sum<LPA>(acc);
      if (gl == 0) I.b[t] = v;
    }
  }
  if (blk == 0 && threadIdx.x == 0) {
    I.support[t] = j;
    I.bitmap[j >> 5] |= (1u << (j & 31));
    *I.nsel = t + 1;
    const float cj = key_value(key);
    if (!(cj <= 3.402823466e38f)) atomicOr(I.status, ST_NAN);
    // step size follows the selected correlation; eps is fixed by the first
    if (t == 0) {
      I.st->sigma = cj;
      I.st->eps = eps_rel * cj;
    }
    I.st->lr = lr_rel * cj;
  }
}

// Register variant of the Gram kernel (lane share of a column <= NCH vectors):
// no LDS staging; each dot issues the a_j and partner-column loads together.
template <typename TA, int LPA, int NCH>
__global__ __launch_bounds__(kBlock) void gram_reg_kernel(const Inst* __restrict__ insts, int t,
                                                          int nblk, int D, float lr_rel,
                                                          float eps_rel) {
  const int ii = blockIdx.x / nblk;
  const int blk = blockIdx.x - ii * nblk;
  const Inst& I = insts[ii];
  if (I.st->done) return;
  const unsigned long long key = *I.key;
  const int j = key_index(key);
  if (key == 0ull || j < 0 || j >= I.n) {
    if (blk == 0 && threadIdx.x == 0) {
      I.st->done = 1;
      atomicOr(I.status, ST_WATCHDOG);
    }
    return;
  }
  constexpr int VW = Vec<TA>::W;
  const int m = I.m;
  const int nvec = (m + VW - 1) / VW;
  const int tail = m - (nvec - 1) * VW;
  const TA* A = reinterpret_cast<const TA*>(I.A);
  const long long lda = I.lda;
  const TA* colj = A + (long long)j * lda;
  const float* yw = I.r + I.m_pad;
  const int gl = threadIdx.x % LPA;
  const int grp = threadIdx.x / LPA;
  constexpr int NG = kBlock / LPA;
  const int l0 = blk * D;
  const int l1 = min(l0 + D, t + 2);
  for (int l = l0 + grp; l < l1; l += NG) {
    float aj[NCH][VW], v[NCH][VW];
    const bool ydot = l == t + 1;
    const TA* colv = A + (long long)((l < t) ? I.support[l] : j) * lda;
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
      const int c = gl + q * LPA;
      if (c < nvec) {
        Vec<TA>::load(colj + (long long)c * VW, aj[q]);
        if (ydot) {
#pragma unroll
          for (int e = 0; e < VW; ++e) v[q][e] = yw[c * VW + e];
        } else {
          Vec<TA>::load(colv + (long long)c * VW, v[q]);
        }
      } else {
#pragma unroll
        for (int e = 0; e < VW; ++e) aj[q][e] = v[q][e] = 0.f;
      }
      if (c == nvec - 1) {
        // entries beyond m are ignored padding (possibly NaN): zero both
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          aj[q][e] = (e < tail) ? aj[q][e] : 0.f;
          v[q][e] = (e < tail) ? v[q][e] : 0.f;
        }
      }
    }
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < NCH; ++q)
#pragma unroll
      for (int e = 0; e < VW; ++e) acc[e & 3] = fmaf(aj[q][e], v[q][e], acc[e & 3]);
    const float d = group_sum<LPA>((acc[0] + acc[1]) + (acc[2] + acc[3]));
    if (gl == 0) {
      if (ydot) {
        I.b[t] = d;
      } else {
        const float dd = (l == t) ? d + tv_diag(I, j) : d;
        I.G[l + (long long)t * I.ldg] = dd;
        I.G[t + (long long)l * I.ldg] = dd;
      }
    }
  }
  if (blk == 0 && threadIdx.x == 0) {
    I.support[t] = j;
    I.bitmap[j >> 5] |= (1u << (j & 31));
    *I.nsel = t + 1;
    const float cj = key_value(key);
    if (!(cj <= 3.402823466e38f)) atomicOr(I.status, ST_NAN);
    // step size follows the selected correlation; eps is fixed by the first
    if (t == 0) {
      I.st->sigma = cj;
      I.st->eps = eps_rel * cj;
    }
    I.st->lr = lr_rel * cj;
  }
}

// ============================================================ Adam (CLOMP)
// One workgroup per active instance; rows of G are split over the threads
// (up to kRPT rows each).  T steps of
//   g = G s - b;  m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
//   s -= lr * (m / bc1) / (sqrt(v / bc2) + eps)
// with bias corrections bc = 1 - beta^step (Kingma & Ba, Algorithm 1).  The
// instance key is cleared for the next scan.
constexpr int kMaxRows = 2048;  // k_eff capacity of the coefficient kernels

template <int NT>
__device__ void adam_global_body(const Inst& I, int t, int T, float beta1, float beta2,
                                 float* ssh, bool clear_key = true) {
  constexpr int kRPT = kMaxRows / NT;
  if (I.st->done) {
    if (threadIdx.x == 0) *I.key = 0ull;
    return;
  }
  const int t1 = t + 1;
  const long long ldg = I.ldg;
  const float* __restrict__ G = I.G;
  float mo[kRPT], ve[kRPT], bb[kRPT], g[kRPT];
#pragma unroll
  for (int q = 0; q < kRPT; ++q) {
    const int r = threadIdx.x + q * NT;
    if (r < t1) {
      ssh[r] = I.s[r];
      mo[q] = I.mo[r];
      ve[q] = I.ve[r];
      bb[q] = I.b[r];
    }
  }
  const float lr = I.st->lr, eps = I.st->eps;
  const int step0 = I.st->step;
  double b1p = pow((double)beta1, (double)step0);
  double b2p = pow((double)beta2, (double)step0);
  __syncthreads();
  for (int it = 0; it < T; ++it) {
    b1p *= beta1;
    b2p *= beta2;
    const float bc1 = (float)(1.0 - b1p);
    const float bc2 = (float)(1.0 - b2p);
#pragma unroll
    for (int q = 0; q < kRPT; ++q) g[q] = 0.f;
    // rows of G are streamed from L2; four columns per pass keep four
    // independent loads in flight per row
    int c = 0;
    for (; c + 4 <= t1; c += 4) {
      const float s0 = ssh[c], s1 = ssh[c + 1], s2 = ssh[c + 2], s3 = ssh[c + 3];
      const float* G0 = G + (long long)c * ldg;
#pragma unroll
      for (int q = 0; q < kRPT; ++q) {
        const int r = threadIdx.x + q * NT;
        if (r < t1) {
          const float u0 = G0[r], u1 = G0[ldg + r], u2 = G0[2 * ldg + r], u3 = G0[3 * ldg + r];
          g[q] = fmaf(u3, s3, fmaf(u2, s2, fmaf(u1, s1, fmaf(u0, s0, g[q]))));
        }
      }
    }
    for (; c < t1; ++c) {
      const float sc = ssh[c];
      const float* Gc = G + (long long)c * ldg;
#pragma unroll
      for (int q = 0; q < kRPT; ++q) {
        const int r = threadIdx.x + q * NT;
        if (r < t1) g[q] = fmaf(Gc[r], sc, g[q]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kRPT; ++q) {
      const int r = threadIdx.x + q * NT;
      if (r < t1) {
        const float gr = g[q] - bb[q];
        mo[q] = beta1 * mo[q] + (1.f - beta1) * gr;
        ve[q] = beta2 * ve[q] + (1.f - beta2) * (gr * gr);
        const float mh = mo[q] / bc1;
        const float vh = ve[q] / bc2;
        ssh[r] = ssh[r] - lr * mh / (sqrtf(vh) + eps);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kRPT; ++q) {
    const int r = threadIdx.x + q * NT;
    if (r < t1) {
      I.s[r] = ssh[r];
      I.mo[r] = mo[q];
      I.ve[r] = ve[q];
    }
  }
  if (threadIdx.x == 0) {
    I.st->step = step0 + T;
    if (clear_key) *I.key = 0ull;
  }
}

// Fused-launch variant for 256 < t+1 <= 1024 on one 1024-thread workgroup.
// The rows are taken four at a time: thread (p, q) streams rows 4q .. 4q+3 of
// the columns c = p, p+P, ... (one 16-byte load per column; G is column-major,
// so a column's rows are contiguous, and ldg is a multiple of 4), with P =
// the most column partitions that keep P * ceil((t+1)/4) <= 1024 threads.
// Eight loads per thread are in flight, so a step waits for a few memory
// round trips instead of one per four columns.  The P partial float4s of a
// row group are added in LDS in a fixed order by thread (0, q), which owns
// the Adam state of its four rows.  `lds` holds s (t+1 rounded up to 4) and
// the partials [P][ceil((t+1)/4)] as float4: at most kSplitLdsFloats.
__device__ void adam_split_body(const Inst& I, int t, int T, float beta1, float beta2,
                                float* lds) {
  constexpr int NT = 1024;   // the fused launch's workgroup size
  const int t1 = t + 1;
  const int g4 = (t1 + 3) >> 2;        // row groups (<= 256)
  const int t4 = 4 * g4;
  int P = 1;
  while (2 * P * g4 <= NT) P <<= 1;
  const int tid = threadIdx.x;
  const int p = tid / g4, q = tid - p * g4;
  const bool active = p < P;
  const bool own = p == 0;             // owner of rows 4q .. 4q+3 (those < t1)
  const long long ldg = I.ldg;
  const float* __restrict__ G = I.G;
  float* ssh = lds;                                     // [t4]
  float4* part = reinterpret_cast<float4*>(lds + t4);   // [P][g4]
  float mo[4], ve[4], bb[4];
  for (int c = tid; c < t4; c += NT) ssh[c] = (c < t1) ? I.s[c] : 0.f;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = 4 * q + e;
    const bool ok = own && r < t1;
    mo[e] = ok ? I.mo[r] : 0.f;
    ve[e] = ok ? I.ve[r] : 0.f;
    bb[e] = ok ? I.b[r] : 0.f;
  }
  const float lr = I.st->lr, eps = I.st->eps;
  const int step0 = I.st->step;
  double b1p = pow((double)beta1, (double)step0);
  double b2p = pow((double)beta2, (double)step0);
  const float* gcol = G + 4 * q;       // rows 4q .. 4q+3 of column 0
  __syncthreads();
  for (int it = 0; it < T; ++it) {
    b1p *= beta1;
    b2p *= beta2;
    const float ibc1 = __builtin_amdgcn_rcpf((float)(1.0 - b1p));
    const float ibc2 = __builtin_amdgcn_rcpf((float)(1.0 - b2p));
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
    if (active) {
      int c = p;
      for (; c + 7 * P < t1; c += 8 * P) {
        float4 gv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          gv[u] = *reinterpret_cast<const float4*>(gcol + (long long)(c + u * P) * ldg);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const float sc = ssh[c + u * P];
          float4& acc = (u & 1) ? b : a;
          acc.x = fmaf(gv[u].x, sc, acc.x);
          acc.y = fmaf(gv[u].y, sc, acc.y);
          acc.z = fmaf(gv[u].z, sc, acc.z);
          acc.w = fmaf(gv[u].w, sc, acc.w);
        }
      }
      for (; c < t1; c += P) {
        const float4 gv = *reinterpret_cast<const float4*>(gcol + (long long)c * ldg);
        const float sc = ssh[c];
        a.x = fmaf(gv.x, sc, a.x);
        a.y = fmaf(gv.y, sc, a.y);
        a.z = fmaf(gv.z, sc, a.z);
        a.w = fmaf(gv.w, sc, a.w);
      }
      part[p * g4 + q] = make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
    }
    __syncthreads();
    if (own) {
      float4 gs = part[q];
      for (int pp = 1; pp < P; ++pp) {
        const float4 v = part[pp * g4 + q];
        gs.x += v.x;
        gs.y += v.y;
        gs.z += v.z;
        gs.w += v.w;
      }
      const float g[4] = {gs.x, gs.y, gs.z, gs.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 4 * q + e;
        if (r < t1) {
          const float gr = g[e] - bb[e];
          mo[e] = beta1 * mo[e] + (1.f - beta1) * gr;
          ve[e] = beta2 * ve[e] + (1.f - beta2) * (gr * gr);
          const float mh = mo[e] * ibc1;
          const float vh = ve[e] * ibc2;
          ssh[r] = ssh[r] - lr * mh * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(vh) + eps);
        }
      }
    }
    __syncthreads();
  }
  if (own) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 4 * q + e;
      if (r < t1) {
        I.s[r] = ssh[r];
        I.mo[r] = mo[e];
        I.ve[r] = ve[e];
      }
    }
  }
  if (tid == 0) I.st->step = step0 + T;
}

__global__ __launch_bounds__(kBlock) void adam_kernel(const Inst* __restrict__ insts, int t,
                                                      int T, float beta1, float beta2) {
  extern __shared__ __align__(16) float ssh[];  // s[t+1]
  adam_global_body<kBlock>(insts[blockIdx.x], t, T, beta1, beta2, ssh);
}

// Register-resident variant for t+1 <= 256 (1024 threads, 16 waves).
// Wave w owns the 16 columns [16w, 16w+16) of G and lane l the rows
// [4l, 4l+4): a 4 x 16 tile of G lives in each lane's registers for the whole
// launch.  Because G is symmetric, the 16 coefficients wave w multiplies by
// are exactly the rows 16w..16w+15 whose Adam state its lanes 0..15 own, so
// they never leave the wave: they are broadcast with readlane.  One barrier
// per step exchanges the partial row sums (double-buffered in LDS); each
// row's 16 partials are then added in a fixed order.
constexpr int kRegRows = 256;

// RPL rows per lane (1, 2 or 4; rows RPL*l .. RPL*l+RPL-1 of lane l): a
// support of t+1 <= 64*RPL atoms; fewer rows per lane keep the tile of G
// within the registers of a full-occupancy wave.  `part` (LDS) holds two
// buffers of 16 wave slots of 64*RPL floats: adam_part_floats<RPL>().
template <int RPL>
constexpr int adam_part_floats() { return 2 * 16 * 64 * RPL; }

template <int RPL = 4>
__device__ void adam_reg_body(const Inst& I, int t, int T, float beta1, float beta2,
                              float* part, int nw, bool clear_key = true) {
  constexpr int kSlot = 64 * RPL, kBuf = 16 * kSlot;
  if (I.st->done) {
    if (threadIdx.x == 0) *I.key = 0ull;
    return;
  }
  const int t1 = t + 1;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int c0 = 16 * w;
  const bool active = c0 < t1;          // wave-uniform
  const long long ldg = I.ldg;
  float Gr[RPL][16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int rb = RPL * lane;
    // rows at or beyond t1 hold stale values: zero them
    if constexpr (RPL == 4) {
      float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
      if (active && rb < t1 && c0 + c < t1)
        q = *reinterpret_cast<const float4*>(I.G + (long long)(c0 + c) * ldg + rb);
      Gr[0][c] = (rb + 0 < t1) ? q.x : 0.f;
      Gr[1][c] = (rb + 1 < t1) ? q.y : 0.f;
      Gr[2][c] = (rb + 2 < t1) ? q.z : 0.f;
      Gr[3][c] = (rb + 3 < t1) ? q.w : 0.f;
    } else {
      const float* gc = I.G + (long long)(c0 + c) * ldg + rb;
      const bool colok = active && c0 + c < t1;
#pragma unroll
      for (int i = 0; i < RPL; ++i) Gr[i][c] = (colok && rb + i < t1) ? gc[i] : 0.f;
    }
  }
  // Adam state of row R = 16w + lane (lanes 0..15)
  const int R = c0 + lane;
  const bool own = lane < 16 && R < t1;
  float sv = 0.f, mo = 0.f, ve = 0.f, bb = 0.f;
  if (own) {
    sv = I.s[R];
    mo = I.mo[R];
    ve = I.ve[R];
    bb = I.b[R];
  }
  const float lr = I.st->lr, eps = I.st->eps;
  const int step0 = I.st->step;
  double b1p = pow((double)beta1, (double)step0);
  double b2p = pow((double)beta2, (double)step0);
  // slots of waves beyond nw stay zero so every row reads 16 partials
  // unconditionally (independent LDS loads, no branches)
  for (int q = nw + w; q < 16; q += nw) {
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      part[q * kSlot + RPL * lane + i] = 0.f;
      part[kBuf + q * kSlot + RPL * lane + i] = 0.f;
    }
  }
  for (int it = 0; it < T; ++it) {
    const int buf = it & 1;
    b1p *= beta1;
    b2p *= beta2;
    // bias-correction factors for this step (1 - beta^step in float64, then a
    // float reciprocal), formed before the barrier
    const float ibc1 = __builtin_amdgcn_rcpf((float)(1.0 - b1p));
    const float ibc2 = __builtin_amdgcn_rcpf((float)(1.0 - b2p));
    // per-row sums over the wave's 16 columns, four interleaved chains each
    float acc[RPL][4];
#pragma unroll
    for (int i = 0; i < RPL; ++i)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[i][u] = 0.f;
    if (active) {
      const int sbits = __float_as_int(sv);
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const float sc = __int_as_float(__builtin_amdgcn_readlane(sbits, c));
#pragma unroll
        for (int i = 0; i < RPL; ++i) acc[i][c & 3] = fmaf(Gr[i][c], sc, acc[i][c & 3]);
      }
    }
    // the wave's partial of row r sits at float r of its slot
    if constexpr (RPL == 4) {
      float rs[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) rs[i] = (acc[i][0] + acc[i][1]) + (acc[i][2] + acc[i][3]);
      *reinterpret_cast<float4*>(part + buf * kBuf + w * kSlot + 4 * lane) =
          make_float4(rs[0], rs[1], rs[2], rs[3]);
    } else {
      float* pw = part + buf * kBuf + w * kSlot + RPL * lane;
#pragma unroll
      for (int i = 0; i < RPL; ++i) pw[i] = (acc[i][0] + acc[i][1]) + (acc[i][2] + acc[i][3]);
    }
    __syncthreads();
    if (own) {
      // partials of row R: float R of the 16 wave slots, added as a balanced
      // tree in a fixed order
      const float* pf = part + buf * kBuf + R;
      float p[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) p[q] = pf[q * kSlot];
#pragma unroll
      for (int h = 8; h > 0; h >>= 1)
#pragma unroll
        for (int q = 0; q < h; ++q) p[q] = p[q] + p[q + h];
      const float gr = p[0] - bb;
      mo = beta1 * mo + (1.f - beta1) * gr;
      ve = beta2 * ve + (1.f - beta2) * (gr * gr);
      const float mh = mo * ibc1;
      const float vh = ve * ibc2;
      // hardware square root and reciprocal (1 ulp)
      sv = sv - lr * mh * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(vh) + eps);
    }
  }
  if (own) {
    I.s[R] = sv;
    I.mo[R] = mo;
    I.ve[R] = ve;
  }
  if (threadIdx.x == 0) {
    I.st->step = step0 + T;
    if (clear_key) *I.key = 0ull;
  }
}

__global__ __launch_bounds__(1024) void adam_reg_kernel(const Inst* __restrict__ insts, int t,
                                                        int T, float beta1, float beta2) {
  __shared__ __align__(16) float part[adam_part_floats<4>()];
  // the launch uses ceil((t+1)/16) waves: every wave owns live columns
  adam_reg_body(insts[blockIdx.x], t, T, beta1, beta2, part, blockDim.x >> 6);
}

// ============================================================ OMP coefficients
// One workgroup per active instance.  Keeps Ginv = G_S^{-1} (column-major,
// both triangles, in the Linv buffer) and the least-squares coefficients
// x_S = Ginv b in s.  Appending atom t with Gram column g (gamma = g_tt):
//   v = Ginv g,  delta = gamma - g.v,  alpha = (b_t - g.x_S) / delta,
//   x_S <- [x_S - alpha v ; alpha],
//   Ginv <- [[Ginv + v v^T / delta, -v / delta], [-v^T / delta, 1 / delta]]
// (bordered inverse).  Both sweeps over Ginv are coalesced (column c read or
// updated by consecutive rows r); there is no sequential triangular solve.
constexpr int kOmpThreads = 1024;

// NT threads: NT / 256 column groups of 256 row lanes; osh holds g[t+1] |
// v[t+1] | vpart[NT / 256][t+1], red and red2 NT / 64 floats each.
template <int NT = kOmpThreads>
__device__ void omp_ginv_body(const Inst& I, int t, float* osh, float* red, float* red2,
                              bool clear_key = true) {
  constexpr int NCG = NT / 256;
  if (I.st->done) {
    if (threadIdx.x == 0) *I.key = 0ull;
    return;
  }
  const int t1 = t + 1;
  const long long ld = I.ldg;
  float* Gi = I.Linv;
  float* g = osh;
  float* v = osh + t1;
  float* vpart = osh + 2 * t1;
  const int tid = threadIdx.x;
  const int rl = tid & 255;      // row lane
  const int cg = tid >> 8;       // column group: columns c = cg, cg+NCG, ...
  for (int r = tid; r < t1; r += NT) g[r] = I.G[r + (long long)t * ld];
  __syncthreads();
  // v = Ginv g over the first t rows / columns: NCG column groups, rows strided
  for (int r = rl; r < t; r += 256) {
    float a0 = 0.f, a1 = 0.f;
    int c = cg;
    for (; c + NCG < t; c += 2 * NCG) {
      a0 = fmaf(Gi[r + (long long)c * ld], g[c], a0);
      a1 = fmaf(Gi[r + (long long)(c + NCG) * ld], g[c + NCG], a1);
    }
    if (c < t) a0 = fmaf(Gi[r + (long long)c * ld], g[c], a0);
    vpart[cg * t1 + r] = a0 + a1;
  }
  __syncthreads();
  float pv = 0.f, px = 0.f;
  for (int r = tid; r < t; r += NT) {
    float vr;
    if constexpr (NCG == 4)
      vr = (vpart[r] + vpart[t1 + r]) + (vpart[2 * t1 + r] + vpart[3 * t1 + r]);
    else
      vr = vpart[r];
    v[r] = vr;
    pv = fmaf(g[r], vr, pv);
    px = fmaf(g[r], I.s[r], px);
  }
  // block sums (fixed order over the waves)
  pv = wave_sum(pv);
  px = wave_sum(px);
  if ((tid & 63) == 0) {
    red[tid >> 6] = pv;
    red2[tid >> 6] = px;
  }
  __syncthreads();
  float gv = 0.f, gx = 0.f;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) {
    gv += red[q];
    gx += red2[q];
  }
  const float gamma = g[t];
  float delta = gamma - gv;
  const bool bad = !(delta > 1e-7f * gamma);
  if (bad) delta = fmaxf(1e-7f * gamma, 1e-30f);
  const float inv = 1.f / delta;
  const float alpha = (I.b[t] - gx) * inv;
  for (int r = tid; r < t; r += NT) {
    I.s[r] = fmaf(-alpha, v[r], I.s[r]);
    const float w = -v[r] * inv;
    Gi[r + (long long)t * ld] = w;
    Gi[t + (long long)r * ld] = w;
  }
  // rank-one update Ginv += v v^T / delta: column groups x rows, coalesced
  for (int c = cg; c < t; c += NCG) {
    const float vc = v[c] * inv;
    float* col = Gi + (long long)c * ld;
    for (int r = rl; r < t; r += 256) col[r] = fmaf(v[r], vc, col[r]);
  }
  if (tid == 0) {
    I.s[t] = alpha;
    Gi[t + (long long)t * ld] = inv;
    if (bad) atomicOr(I.status, ST_REFINE_INACCURATE);
    if (clear_key) *I.key = 0ull;
  }
}

__global__ __launch_bounds__(kOmpThreads) void omp_ginv_kernel(const Inst* __restrict__ insts,
                                                               int t) {
  extern __shared__ __align__(16) float osh[];  // g[t1] | v[t1] | vpart[4][t1]
  __shared__ float red[kOmpThreads / 64], red2[kOmpThreads / 64];
  omp_ginv_body(insts[blockIdx.x], t, osh, red, red2);
}

// ============================================================ rows kernels
// out_i = base_i + sign * sum_{l<=t} A[i, S_l] * coef_l  for the rows of one
// 64-row tile; the four waves split the columns and are summed in order.
enum RowMode : int {
  ROW_RESID = 0,   // r = y - A_bulk[:, S] s
  ROW_CG_R0 = 1,   // cg.r0 = y - A_master[:, S] xf
  ROW_CG_Q = 2,    // cg.q = A_master[:, S] p   (+ partial ||q||^2)
  ROW_IHT_R = 3,   // IHT: r = y - A_bulk[:, S] s over the instance's own support
  ROW_IHT_U = 4    // IHT: partial ||A_bulk[:, S] g_S||^2 (the normalised step)
};

// NW waves split the columns (4; the IHT modes also 16, for classes with
// fewer row tiles than CUs: fewer dependent load rounds per lane).
template <typename TA, int MODE, int NW = kWaves>
__global__ __launch_bounds__(64 * NW) void rows_kernel(const Inst* __restrict__ insts,
                                                       const RowTile* __restrict__ tiles,
                                                       int t, int it, float tol2) {
  static_assert(NW == kWaves || MODE == ROW_IHT_R || MODE == ROW_IHT_U,
                "the CGLS modes reduce over kWaves waves");
  constexpr int NTH = 64 * NW;
  extern __shared__ __align__(16) float rsh[];  // coef[t1] | (int) sup[t1] | part[NW*64]
  __shared__ float red[kWaves];
  const RowTile rt = tiles[blockIdx.x];
  const Inst& I = insts[rt.inst];
  if (I.st->done) return;
  if ((MODE == ROW_IHT_R || MODE == ROW_IHT_U) && I.st->stop) return;
  // in the loop every active instance has t+1 atoms; after it, its own count
  const int t1 = (MODE == ROW_RESID) ? t + 1 : *I.nsel;
  float* coef = rsh;
  int* sup = reinterpret_cast<int*>(rsh + t1);
  float* part = rsh + 2 * t1;
  const float* src;
  if (MODE == ROW_RESID || MODE == ROW_IHT_R) src = I.s;
  else if (MODE == ROW_CG_R0) src = I.xf;
  else src = nullptr;
  if (MODE == ROW_CG_Q) {
    // CGLS direction: gamma = ||sv||^2; p = sv (first) or sv + beta p_old.
    if (I.st->cg_done) return;
    const float* sv = I.cg + 3 * I.m_pad + 2 * I.k_eff;
    float pg = 0.f;
    for (int l = threadIdx.x; l < t1; l += kBlock) pg = fmaf(sv[l], sv[l], pg);
    const float gamma = block_sum(pg, red);
    // stop once ||A_S^T r|| <= tol * ||A_S^T y|| (b holds A_S^T y of the bulk
    // columns, equal to the master's up to the bulk rounding)
    float pb = 0.f;
    for (int l = threadIdx.x; l < t1; l += kBlock) pb = fmaf(I.b[l], I.b[l], pb);
    const float bnorm2 = block_sum(pb, red);
    if (gamma <= tol2 * bnorm2) {
      if (rt.tile == 0 && threadIdx.x == 0) I.st->cg_done = 1;
      return;
    }
    const float beta = (it == 0) ? 0.f : gamma / I.st->gamma[(it - 1) & 1];
    const float* pold = I.cg + 3 * I.m_pad + ((it - 1) & 1) * I.k_eff;
    float* pnew = I.cg + 3 * I.m_pad + (it & 1) * I.k_eff;
    for (int l = threadIdx.x; l < t1; l += kBlock) {
      const float p = (it == 0) ? sv[l] : fmaf(beta, pold[l], sv[l]);
      coef[l] = p;
      if (rt.tile == 0) pnew[l] = p;
    }
    if (rt.tile == 0 && threadIdx.x == 0) I.st->gamma[it & 1] = gamma;
  } else if (MODE == ROW_IHT_U) {
    for (int l = threadIdx.x; l < t1; l += NTH) coef[l] = I.gbuf[I.support[l]];
  } else {
    for (int l = threadIdx.x; l < t1; l += NTH) coef[l] = src[l];
  }
  for (int l = threadIdx.x; l < t1; l += NTH) sup[l] = I.support[l];
  __syncthreads();
  const TA* A;
  long long lda;
  if (MODE == ROW_RESID || MODE == ROW_IHT_R || MODE == ROW_IHT_U) {
    A = reinterpret_cast<const TA*>(I.A);
    lda = I.lda;
  } else {
    A = reinterpret_cast<const TA*>(I.Am);
    lda = I.ldam;
  }
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int i = rt.i0 + lane;
  float acc = 0.f;
  if (i < rt.i1) {
    // columns l = w, w+NW, ...: eight independent chains keep eight loads in
    // flight per lane
    float a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = 0.f;
    int l = w;
    for (; l + 7 * NW < t1; l += 8 * NW) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int ll = l + u * NW;
        a[u] = fmaf(Vec<TA>::one(A + (long long)sup[ll] * lda + i), coef[ll], a[u]);
      }
    }
    for (; l < t1; l += NW) a[0] = fmaf(Vec<TA>::one(A + (long long)sup[l] * lda + i), coef[l], a[0]);
    acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  }
  part[w * 64 + lane] = acc;
  __syncthreads();
  if (w == 0) {
    float v = 0.f;
    if (i < rt.i1) {
      float sum;
      if constexpr (NW == 4) {
        sum = (part[lane] + part[64 + lane]) + (part[128 + lane] + part[192 + lane]);
      } else {
        // the NW wave partials as a balanced tree in a fixed order
        float pv[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) pv[q] = part[q * 64 + lane];
#pragma unroll
        for (int h = NW / 2; h > 0; h >>= 1)
#pragma unroll
          for (int q = 0; q < h; ++q) pv[q] = pv[q] + pv[q + h];
        sum = pv[0];
      }
      const float* yw = I.r + I.m_pad;
      if (MODE == ROW_RESID || MODE == ROW_IHT_R) {
        I.r[i] = yw[i] - sum;
      } else if (MODE == ROW_CG_R0) {
        I.cg[i] = yw[i] - sum;  // r0
      } else if (MODE == ROW_IHT_U) {
        v = sum * sum;
      } else {
        I.cg[2 * I.m_pad + i] = sum;  // q
        v = sum * sum;
      }
    }
    if (MODE == ROW_CG_Q || MODE == ROW_IHT_U) {
      v = wave_sum(v);
      if (lane == 0) I.qpart[rt.tile] = v;
    }
  }
}

// ============================================================ column dots
// sv_l = A_master[:, S_l]^T v for CGLS.  Mode 0 (init): v = r0.  Mode 1
// (iteration it): alpha = gamma / ||q||^2, r_new = r_old - alpha q (r ping-pong
// by parity, written by block 0), xf += alpha p, then the dots with r_new.
template <int LPA, int MODE>
__global__ __launch_bounds__(kBlock) void cg_dots_kernel(const Inst* __restrict__ insts,
                                                         const int* __restrict__ list,
                                                         int t, int nblk, int D, int it) {
  extern __shared__ __align__(16) float vsh[];
  __shared__ float qred[kWaves];
  const int ii = blockIdx.x / nblk;
  const int blk = blockIdx.x - ii * nblk;
  const Inst& I = insts[list[ii]];
  if (I.st->done) return;
  if (MODE == 1 && I.st->cg_done) return;
  const int m = I.m;
  const int t1 = *I.nsel;
  const int mp = I.m_pad;
  float* rbuf0 = I.cg;           // r ping
  float* rbuf1 = I.cg + mp;      // r pong
  const float* q = I.cg + 2 * mp;
  float* sv = I.cg + 3 * mp + 2 * I.k_eff;
  if (MODE == 0) {
    for (int i = threadIdx.x; i < mp; i += kBlock) vsh[i] = (i < m) ? rbuf0[i] : 0.f;
  } else {
    float qq = 0.f;
    for (int tt = threadIdx.x; tt < I.n_rowtiles; tt += kBlock) qq += I.qpart[tt];
    qq = block_sum(qq, qred);
    const float gamma = I.st->gamma[it & 1];
    const float alpha = (qq > 0.f) ? gamma / qq : 0.f;
    const float* rold = (it & 1) ? rbuf1 : rbuf0;
    float* rnew = (it & 1) ? rbuf0 : rbuf1;
    for (int i = threadIdx.x; i < mp; i += kBlock) {
      const float v = (i < m) ? fmaf(-alpha, q[i], rold[i]) : 0.f;
      vsh[i] = v;
      if (blk == 0) rnew[i] = v;
    }
    if (blk == 0) {
      const float* p = I.cg + 3 * mp + (it & 1) * I.k_eff;
      for (int l = threadIdx.x; l < t1; l += kBlock) I.xf[l] = fmaf(alpha, p[l], I.xf[l]);
    }
  }
  __syncthreads();
  const int gl = threadIdx.x % LPA;
  const int grp = threadIdx.x / LPA;
  constexpr int NG = kBlock / LPA;
  const int l0 = blk * D;
  const int l1 = min(l0 + D, t1);
  for (int l = l0 + grp; l < l1; l += NG) {
    const float* col = I.Am + (long long)I.support[l] * I.ldam;
    const float v = col_dot<float, LPA>(col, vsh, m, gl);
    if (gl == 0) sv[l] = v;
  }
}

// ============================================================ small QR refine
// Householder QR of the FP32 master columns A_S (m x t1, in LDS) and the
// triangular solve R x = Q^T y, one workgroup per instance in the list,
// followed by kQrSteps steps of iterative refinement: the residual
// r = y - A_S x accumulated in FP64 from the master columns, the correction
// d = argmin ||r - A_S d|| from the same factors, x += d.  With the residual
// in higher precision the error of x falls to about kappa(A_S) * 2^-24.
constexpr int kQrSteps = 2;

// Apply the stored reflectors H_0 .. H_{t1-1} to v (length mr) and solve
// R d = (Q^T v)[0 .. t1), d into out.  Reflector c is column c of M from
// row c on, with squared norm vn[c] (0: skipped).
// Back substitution R d = v[0 .. t1) by wave 0 alone (the other waves pass
// through); R has diagonal Rd and strictly-upper entries M[c + cc mr].  The
// caller synchronises the workgroup afterwards.
__device__ void qr_back_substitute(const float* M, const float* Rd, const float* v, float* out,
                                   int mr, int t1) {
  if ((threadIdx.x >> 6) != 0) return;
  const int lane = threadIdx.x & 63;
  for (int c = t1 - 1; c >= 0; --c) {
    float sacc = 0.f;
    for (int cc = c + 1 + lane; cc < t1; cc += 64) sacc = fmaf(M[c + (long long)cc * mr], out[cc], sacc);
    sacc = wave_sum(sacc);
    if (lane == 0) {
      const float dd = Rd[c];
      out[c] = (dd != 0.f) ? (v[c] - sacc) / dd : 0.f;
    }
    wave_sync();   // out[c] is read by every lane of the next rows
  }
}

// Systems of up to kQrWaveRows rows apply the reflectors in wave 0 alone:
// lane l keeps rows l, l + 64, ... of v for all of them, so only the wave's
// own reduction orders the steps (no workgroup barrier per reflector).
constexpr int kQrWaveRows = 256;

__device__ void qr_apply_solve(const float* M, const float* Rd, const float* vn, float* v,
                               float* out, int mr, int t1, float* red) {
  if (mr <= kQrWaveRows) {
    if ((threadIdx.x >> 6) == 0) {
      const int lane = threadIdx.x & 63;
      for (int c = 0; c < t1; ++c) {
        const float* Mc = M + (long long)c * mr;
        float p = 0.f;
        for (int i = lane; i < mr; i += 64)
          if (i >= c) p = fmaf(Mc[i], v[i], p);
        const float d = wave_sum(p);
        if (vn[c] > 0.f) {
          const float f = 2.f * d / vn[c];
          for (int i = lane; i < mr; i += 64)
            if (i >= c) v[i] = fmaf(-f, Mc[i], v[i]);
        }
      }
      wave_sync();   // v[0 .. t1) is read across lanes below
    }
  } else {
    for (int c = 0; c < t1; ++c) {
      const float* Mc = M + (long long)c * mr;
      float p = 0.f;
      for (int i = c + threadIdx.x; i < mr; i += kBlock) p = fmaf(Mc[i], v[i], p);
      const float d = block_sum(p, red);
      if (vn[c] > 0.f) {
        const float f = 2.f * d / vn[c];
        for (int i = c + threadIdx.x; i < mr; i += kBlock) v[i] = fmaf(-f, Mc[i], v[i]);
      }
      __syncthreads();
    }
  }
  qr_back_substitute(M, Rd, v, out, mr, t1);
  __syncthreads();
}

// Reflector c (Mc, rows c .. mr-1) applied to the targets c+1 .. t1 (columns
// of M, then y as target t1): QG lanes share a target, so a wave takes 64/QG
// targets at a time and each lane handles rows c + g, c + g + QG, ...
template <int QG>
__device__ void qr_apply_reflector(const float* Mc, float* M, float* yv, int c, int mr, int t1,
                                   float inv) {
  constexpr int kPerWave = 64 / QG;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane % QG, grp = lane / QG;
  for (int cc = c + 1 + wv * kPerWave + grp; cc <= t1; cc += kWaves * kPerWave) {
    float* tgt = (cc < t1) ? (M + (long long)cc * mr) : yv;
    float d = 0.f;
    for (int i = c + g; i < mr; i += QG) d = fmaf(Mc[i], tgt[i], d);
    d = group_sum<QG>(d) * inv;
    for (int i = c + g; i < mr; i += QG) tgt[i] = fmaf(-d, Mc[i], tgt[i]);
  }
}

__global__ __launch_bounds__(kBlock) void qr_refine_kernel(const Inst* __restrict__ insts,
                                                           const int* __restrict__ list) {
  extern __shared__ __align__(16) float qsh[];
  __shared__ float red[kWaves];
  __shared__ float diag[1];
  const Inst& I = insts[list[blockIdx.x]];
  if (I.st->done) return;
  const int m = I.m;
  const int t1 = *I.nsel;
  // with the total-variation prior the system is stacked: t1 more rows
  // holding sqrt((2w/n) lambda_{S_c}) on the diagonal, right-hand side 0
  const int mr = (I.tvw != 0.f) ? m + t1 : m;
  float* M = qsh;                  // mr x t1 column-major (ld mr)
  float* yv = qsh + (long long)mr * t1;   // mr
  float* Rd = yv + mr;             // t1 diagonal of R
  float* xs = Rd + t1;             // t1 solution
  float* vn = xs + t1;             // t1 squared reflector norms
  float* dx = vn + t1;             // t1 refinement correction
  // (four entries per thread per round, their loads issued before the stores)
  auto m_entry = [&](int idx) {
    const int c = idx / mr, i = idx - c * mr;
    return (i < m) ? I.Am[(long long)I.support[c] * I.ldam + i]
                   : ((i - m == c) ? sqrtf(tv_diag(I, I.support[c])) : 0.f);
  };
  {
    const int tot = mr * t1;
    int idx = threadIdx.x;
    for (; idx + 3 * kBlock < tot; idx += 4 * kBlock) {
      float e[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) e[u] = m_entry(idx + u * kBlock);
#pragma unroll
      for (int u = 0; u < 4; ++u) M[idx + u * kBlock] = e[u];
    }
    for (; idx < tot; idx += kBlock) M[idx] = m_entry(idx);
  }
  const float* yw = I.r + I.m_pad;
  for (int i = threadIdx.x; i < mr; i += kBlock) yv[i] = (i < m) ? yw[i] : 0.f;
  __syncthreads();
  bool rank_def = false;
  for (int c = 0; c < t1; ++c) {
    float* Mc = M + (long long)c * mr;
    float p = 0.f;
    for (int i = c + threadIdx.x; i < mr; i += kBlock) p = fmaf(Mc[i], Mc[i], p);
    const float nrm2 = block_sum(p, red);
    const float x0 = Mc[c];
    const float nrm = sqrtf(nrm2);
    const float alpha = (x0 >= 0.f) ? -nrm : nrm;
    const float v0 = x0 - alpha;
    const float vn2 = nrm2 - x0 * x0 + v0 * v0;   // ||v||^2
    __syncthreads();
    if (threadIdx.x == 0) {
      Mc[c] = v0;        // v stored in place (rows c..mr-1)
      diag[0] = alpha;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      Rd[c] = alpha;
      vn[c] = (nrm > 0.f && vn2 > 0.f) ? vn2 : 0.f;
    }
    if (!(nrm > 0.f) || !(vn2 > 0.f)) {
      rank_def = true;
      __syncthreads();
      continue;
    }
    const float inv = 2.f / vn2;
    // apply H = I - 2 v v^T / (v^T v) to columns c+1..t1-1 and y (target
    // t1): a group of QG lanes per target, lanes over rows, 64 / QG targets
    // per wave at a time
    if (mr <= 128)
      qr_apply_reflector<16>(Mc, M, yv, c, mr, t1, inv);
    else if (mr <= 256)
      qr_apply_reflector<32>(Mc, M, yv, c, mr, t1, inv);
    else
      qr_apply_reflector<64>(Mc, M, yv, c, mr, t1, inv);
    __syncthreads();
  }
  // R has diagonal Rd[c] and strictly-upper entries M[c, cc] (cc > c)
  qr_back_substitute(M, Rd, yv, xs, mr, t1);
  __syncthreads();
  // iterative refinement: r = y - A_S x in FP64 from the master columns
  // (stacked prior rows: r = -sqrt(lambda_c) x_c), correction from the factors
  for (int step = 0; step < kQrSteps && !rank_def; ++step) {
    for (int i = threadIdx.x; i < mr; i += kBlock) {
      double acc;
      if (i < m) {
        // eight column loads in flight, subtracted in column order
        acc = (double)yw[i];
        int c = 0;
        for (; c + 8 <= t1; c += 8) {
          float a[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) a[u] = I.Am[(long long)I.support[c + u] * I.ldam + i];
#pragma unroll
          for (int u = 0; u < 8; ++u) acc -= (double)a[u] * (double)xs[c + u];
        }
        for (; c < t1; ++c)
          acc -= (double)I.Am[(long long)I.support[c] * I.ldam + i] * (double)xs[c];
      } else {
        const int c = i - m;
        acc = -(double)sqrtf(tv_diag(I, I.support[c])) * (double)xs[c];
      }
      yv[i] = (float)acc;
    }
    __syncthreads();
    qr_apply_solve(M, Rd, vn, yv, dx, mr, t1, red);
    for (int c = threadIdx.x; c < t1; c += kBlock) xs[c] += dx[c];
    __syncthreads();
  }
  for (int c = threadIdx.x; c < t1; c += kBlock) I.xf[c] = xs[c];
  if (rank_def && threadIdx.x == 0) atomicOr(I.status, ST_REFINE_INACCURATE);
}

// ============================================================ FP64 norm
// Partial sums of (y_i - sum_l Am[i, S_l] xf_l)^2 accumulated in float64.
__global__ __launch_bounds__(kBlock) void norm_rows_kernel(const Inst* __restrict__ insts,
                                                           const RowTile* __restrict__ tiles) {
  extern __shared__ __align__(16) float nsh[];  // xf[t1] | sup[t1]
  __shared__ double dpart[kBlock];
  const RowTile rt = tiles[blockIdx.x];
  const Inst& I = insts[rt.inst];
  const int t1 = *I.nsel;
  float* coef = nsh;
  int* sup = reinterpret_cast<int*>(nsh + (t1 > 0 ? t1 : 1));
  for (int l = threadIdx.x; l < t1; l += kBlock) {
    coef[l] = I.xf[l];
    sup[l] = I.support[l];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int i = rt.i0 + lane;
  double acc = 0.0;
  if (i < rt.i1) {
    for (int l = w; l < t1; l += kWaves)
      acc += (double)I.Am[(long long)sup[l] * I.ldam + i] * (double)coef[l];
  }
  dpart[threadIdx.x] = acc;
  __syncthreads();
  if (w == 0) {
    double e = 0.0;
    if (i < rt.i1) {
      const double sum = (dpart[lane] + dpart[64 + lane]) + (dpart[128 + lane] + dpart[192 + lane]);
      e = (double)I.r[I.m_pad + i] - sum;
      e = e * e;
    }
    e = wave_sum_d(e);
    if (lane == 0) I.npart[rt.tile] = e;
  }
}

// One workgroup per instance: FP64 norm from the partials (fixed order:
// strided per-thread sums, then waves), scatter x_S into x, refinement status.
__global__ __launch_bounds__(kBlock) void finalize_kernel(const Inst* __restrict__ insts,
                                                          int check_cg) {
  __shared__ double dred[kWaves];
  const Inst& I = insts[blockIdx.x];
  const int t1 = *I.nsel;
  for (int l = threadIdx.x; l < t1; l += kBlock) I.x[I.support[l]] = I.xf[l];
  double ps = 0.0;
  for (int tt = threadIdx.x; tt < I.n_rowtiles; tt += kBlock) ps += I.npart[tt];
  ps = wave_sum_d(ps);
  if ((threadIdx.x & 63) == 0) dred[threadIdx.x >> 6] = ps;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kWaves; ++w) s += dred[w];
    *I.rnorm = sqrt(s);   // ||y|| for an empty support (0 when y == 0)
    if (check_cg && I.cg_slot >= 0 && !I.st->done && !I.st->cg_done)
      atomicOr(I.status, ST_REFINE_INACCURATE);
  }
}

// Copy the coefficients reached by the greedy loop into xf (the CGLS start).
// list == nullptr: every instance of the launch (one workgroup each).
__global__ __launch_bounds__(kBlock) void copy_s_kernel(const Inst* __restrict__ insts,
                                                        const int* __restrict__ list) {
  const Inst& I = insts[list ? list[blockIdx.x] : blockIdx.x];
  const int t1 = *I.nsel;
  for (int l = threadIdx.x; l < t1; l += kBlock) I.xf[l] = I.s[l];
  if (threadIdx.x == 0) I.st->cg_done = 0;
}

// ============================================================ iterative hard thresholding
// Normalised IHT (the experiments' comparison method), per iteration:
//   r = y - A_G s_G        rows_kernel<ROW_IHT_R>      (skipped at it = 0: r = y)
//   g = A^T r              iht_grad_kernel (stores g; at it = 0 also A^T y)
//   G0 = top-K |g|         iht_select_kernel mode 0    (it = 0 only)
//   ||A_G g_G||^2          rows_kernel<ROW_IHT_U>      (partials per row tile)
//   z = s + t g, t = ||g_G||^2 / ||A_G g_G||^2, s = z on the top-K |z|
//                          iht_select_kernel mode 1
// The top-K is exact (ties to the lowest index, NaN highest); the support is
// compacted in index order.
//
// The gradient scan splits a long column into I.nslice slices of m (blockIdx.y
// is the slice) so that the staged part of r stays small and many
// workgroups share a CU; slice partials go to gbuf[slice * ldh + j] and
// iht_combine_kernel sums them in slice order.
// 16-byte loads in flight per lane in the gradient scan: 8 for FP32, 4 for
// BF16 (whose loads expand to twice the registers)
template <typename TA>
constexpr int kIhtUnroll = sizeof(TA) == 2 ? 4 : 8;

template <typename TA, int LPA>
__global__ __launch_bounds__(kBlock) void iht_grad_kernel(const Inst* __restrict__ insts,
                                                          const ScanTile* __restrict__ tiles,
                                                          int r_in_lds, int first) {
  extern __shared__ __align__(16) float smem[];
  const ScanTile tile = tiles[blockIdx.x];
  const Inst& I = insts[tile.inst];
  if (I.st->done || I.st->stop) return;
  const int nsl = I.nslice;
  const int sl = blockIdx.y;
  if (sl >= nsl) return;
  constexpr int VW = Vec<TA>::W;
  const int m = I.m;
  const int nvec = (m + VW - 1) / VW;
  const int sv = (nvec + nsl - 1) / nsl;
  const int cv0 = sl * sv, cv1 = min(nvec, cv0 + sv);
  if (r_in_lds) {
    const int cnt = max(0, cv1 - cv0) * VW;
    for (int i = threadIdx.x; i < cnt; i += kBlock) smem[i] = I.r[cv0 * VW + i];
    __syncthreads();
  }
  const TA* A = reinterpret_cast<const TA*>(I.A);
  const long long lda = I.lda;
  const int gl = threadIdx.x % LPA;
  const int grp = threadIdx.x / LPA;
  constexpr int NG = kBlock / LPA;
  const int tail = m - (nvec - 1) * VW;
  for (int j = tile.j0 + grp; j < tile.j1; j += NG) {
    const TA* col = A + (long long)j * lda;
    float acc = r_in_lds
                    ? span_dot<TA, LPA, kIhtUnroll<TA>>(col, smem, cv0, cv1, nvec, tail, gl)
                    : span_dot<TA, LPA, kIhtUnroll<TA>>(col, I.r + (long long)cv0 * VW, cv0,
                                                        cv1, nvec, tail, gl);
    acc = group_sum<LPA>(acc);
    if (gl == 0) {
      I.gbuf[(long long)sl * I.ldh + j] = acc;
      if (first && nsl == 1) I.c0[j] = acc;   // A^T y, for the refinement
    }
  }
}

// g_j = sum of the slice partials of atom j, in slice order (signals with
// nslice > 1; at the first iteration also c0 = A^T y).
__global__ __launch_bounds__(kBlock) void iht_combine_kernel(const Inst* __restrict__ insts,
                                                             const ScanTile* __restrict__ tiles,
                                                             int first) {
  const ScanTile tile = tiles[blockIdx.x];
  const Inst& I = insts[tile.inst];
  if (I.st->done || I.st->stop || I.nslice == 1) return;
  for (int j = tile.j0 + threadIdx.x; j < tile.j1; j += kBlock) {
    float g = I.gbuf[j];
    for (int q = 1; q < I.nslice; ++q) g += I.gbuf[(long long)q * I.ldh + j];
    I.gbuf[j] = g;
    if (first) I.c0[j] = g;
  }
}

// Exclusive scan of v over an NT-thread workgroup: wave scans, then one
// pass over the per-wave totals held in `wsum` (NT/64 entries).  Returns
// the prefix of this thread; `total` receives the workgroup sum.
template <int NT>
__device__ inline unsigned block_excl_scan(unsigned v, unsigned* wsum, unsigned& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();   // earlier readers of wsum are done
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  unsigned before = 0u, tot = 0u;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) {
    const unsigned t = wsum[q];
    before += (q < w) ? t : 0u;
    tot += t;
  }
  total = tot;
  return before + x - v;
}

// Magnitude bits of z as an order key: the sign is cleared, so non-negative
// floats order like their bits and NaN ranks above +Inf.
__device__ inline unsigned mag_bits(float z) { return __float_as_uint(z) & 0x7fffffffu; }

// Threshold bits taken from the previous iteration when they still bracket
// the K-th magnitude (bits 30..20: exponent and the top three mantissa bits)
constexpr int kSelWarmBit = 20;

// Top-K by magnitude of one signal per workgroup (ties to the lowest index).
// Thread q owns the contiguous index chunk [q*CH, q*CH + CH) with its values
// in registers (CH > 0; NT*CH >= n), or walks [q*C, q*C + C) in memory (CH =
// 0).  The K-th largest magnitude Tv is built from the top bit down: Tv is
// the largest key with #{|z| >= Tv} >= K (16 counting passes of one or two
// bits, counts by wave ballots, one barrier each; from the previous
// iteration's threshold bits, when they still bracket it, one check pass and
// ten).  Every larger magnitude is taken, and the first K - #{|z| > Tv}
// equal ones in index order.  mode 0: z = g (support of the first
// iteration); mode 1: the normalised step t and z = s + t g, then s = z on
// the support; mode 2: as mode 1, then b = (A^T y)_S for the refinement
// (the last iteration).
template <int NT, int CH>
__global__ __launch_bounds__(NT) void iht_select_kernel(const Inst* __restrict__ insts_c,
                                                       int mode) {
  __shared__ unsigned ured[2][3][NT / 64];
  __shared__ unsigned wsum[NT / 64];
  __shared__ float red[NT / 64], red2[NT / 64];
  __shared__ float step_sh;
  const Inst& I = insts_c[blockIdx.x];
  if (I.st->done) return;
  const int n = I.n, K = I.k_eff;
  const int tid = threadIdx.x;
  // normalised step t = ||g_G||^2 / ||A_G g_G||^2 (mode 1)
  if (mode >= 1) {
    // numerator and denominator reduced over the whole workgroup (the row
    // partials are many for long columns; a serial walk costs a memory
    // latency per entry)
    float num = 0.f, den = 0.f;
    for (int l = tid; l < K; l += NT) {
      const float g = I.gbuf[I.support[l]];
      num = fmaf(g, g, num);
    }
    for (int q = tid; q < I.n_rowtiles; q += NT) den += I.qpart[q];
    num = wave_sum(num);
    den = wave_sum(den);
    if ((tid & 63) == 0) {
      red[tid >> 6] = num;
      red2[tid >> 6] = den;
    }
    __syncthreads();
    if (tid == 0) {
      float a = 0.f, d = 0.f;
      for (int q = 0; q < NT / 64; ++q) {
        a += red[q];
        d += red2[q];
      }
      step_sh = (d > 0.f) ? a / d : 0.f;
    }
    __syncthreads();
  }
  const float tstep = (mode >= 1) ? step_sh : 1.f;
  auto zval = [&](int j) { return (mode >= 1) ? fmaf(tstep, I.gbuf[j], I.sfull[j]) : I.gbuf[j]; };
  constexpr int R = CH > 0 ? CH : 1;
  const int C = CH > 0 ? CH : (n + NT - 1) / NT;
  const int j0 = tid * C, j1 = min(n, j0 + C);
  float zr[R];
  if constexpr (CH > 0) {
    // gbuf and sfull hold ldh >= roundup(n, 256) floats, so a whole chunk
    // starting below n is in bounds; entries at or past n are zeroed
    if (j0 < n) {
      if constexpr (CH % 4 == 0) {
#pragma unroll
        for (int q = 0; q < CH; q += 4) {
          float4 g = *reinterpret_cast<const float4*>(I.gbuf + j0 + q);
          if (mode >= 1) {
            const float4 sv = *reinterpret_cast<const float4*>(I.sfull + j0 + q);
            g.x = fmaf(tstep, g.x, sv.x);
            g.y = fmaf(tstep, g.y, sv.y);
            g.z = fmaf(tstep, g.z, sv.z);
            g.w = fmaf(tstep, g.w, sv.w);
          }
          zr[q] = g.x;
          zr[q + 1] = g.y;
          zr[q + 2] = g.z;
          zr[q + 3] = g.w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < CH; ++q) zr[q] = zval(j0 + q);
      }
    }
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (j0 + q >= n) zr[q] = 0.f;
  }
  // wave count of magnitudes >= cand (uniform over the wave); absent entries
  // hold 0 and every candidate is >= 1
  auto wcount = [&](unsigned cand) -> unsigned {
    if constexpr (CH > 0) {
      unsigned c = 0u;
#pragma unroll
      for (int q = 0; q < CH; ++q) c += (unsigned)__popcll(__ballot(mag_bits(zr[q]) >= cand));
      return c;
    } else {
      unsigned c = 0u;
      for (int j = j0; j < j1; ++j) c += (mag_bits(zval(j)) >= cand) ? 1u : 0u;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
      return c;
    }
  };
  // one pass resolves the bits [b, b + nb) of the threshold (nb = 1 or 2):
  // the workgroup counts for the 2^nb - 1 candidates Tv | d << b, which
  // decrease with d, and keeps the largest d whose count reaches K
  unsigned Tv = 0u;
  int par = 0;
  auto resolve = [&](int b, int nb) {
    const int nc = (1 << nb) - 1;
    unsigned cnt[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) cnt[d] = (d < nc) ? wcount(Tv | ((unsigned)(d + 1) << b)) : 0u;
    if ((tid & 63) == 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) ured[par][d][tid >> 6] = cnt[d];
    }
    __syncthreads();
    unsigned dsel = 0u;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      unsigned tot = 0u;
#pragma unroll
      for (int q = 0; q < NT / 64; ++q) tot += ured[par][d][q];
      if (d < nc && tot >= (unsigned)K) dsel = d + 1;
    }
    par ^= 1;   // the next pass writes the other buffer
    Tv |= dsel << b;
  };
  // warm start: the bits of the threshold above kSelWarmBit are those of the
  // previous threshold when at least K magnitudes reach that prefix and fewer
  // than K reach the next one (the invariant the passes keep for every
  // prefix); otherwise every bit is resolved.  Tv is the same either way.
  bool warm = false;
  const unsigned lo = I.st->sel_bits & ~((1u << kSelWarmBit) - 1u);
  if (lo != 0u) {   // candidates must be >= 1 (absent entries hold 0)
    const unsigned c0 = wcount(lo), c1 = wcount(lo + (1u << kSelWarmBit));
    if ((tid & 63) == 0) {
      ured[par][0][tid >> 6] = c0;
      ured[par][1][tid >> 6] = c1;
    }
    __syncthreads();
    unsigned t0 = 0u, t1 = 0u;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) {
      t0 += ured[par][0][q];
      t1 += ured[par][1][q];
    }
    par ^= 1;
    if (t0 >= (unsigned)K && t1 < (unsigned)K) {
      Tv = lo;
      warm = true;
    }
  }
  if (!warm) {
    resolve(30, 1);
    for (int b = 28; b >= kSelWarmBit; b -= 2) resolve(b, 2);
  }
  for (int b = kSelWarmBit - 2; b >= 0; b -= 2) resolve(b, 2);
  if (tid == 0) I.st->sel_bits = Tv;
  // number of magnitudes above Tv
  unsigned ngt_all = 0u;
  if (Tv != 0x7fffffffu) {
    const unsigned c = wcount(Tv + 1u);
    if ((tid & 63) == 0) ured[par][0][tid >> 6] = c;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) ngt_all += ured[par][0][q];
  }
  const unsigned take = (unsigned)K - ngt_all;
  unsigned ngt = 0u, neq = 0u;
  if constexpr (CH > 0) {
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const bool ok = j0 + q < j1;
      const unsigned v = mag_bits(zr[q]);
      ngt += (ok && v > Tv) ? 1u : 0u;
      neq += (ok && v == Tv) ? 1u : 0u;
    }
  } else {
    for (int j = j0; j < j1; ++j) {
      const unsigned v = mag_bits(zval(j));
      ngt += (v > Tv) ? 1u : 0u;
      neq += (v == Tv) ? 1u : 0u;
    }
  }
  unsigned tot;
  const unsigned eq_before = block_excl_scan<NT>(neq, wsum, tot);
  const unsigned eq_take = (eq_before >= take) ? 0u : min(neq, take - eq_before);
  unsigned pos = block_excl_scan<NT>(ngt + eq_take, wsum, tot);
  unsigned eq_seen = eq_before;
  auto place = [&](int j, float z) {
    const unsigned v = mag_bits(z);
    bool sel = v > Tv;
    if (v == Tv) {
      sel = eq_seen < take;
      ++eq_seen;
    }
    sel = sel && pos < (unsigned)K;   // exactly K selected
    if (sel) {
      I.support[pos] = j;
      if (mode >= 1) I.s[pos] = z;
      ++pos;
    }
    if (mode >= 1) I.sfull[j] = sel ? z : 0.f;
  };
  if constexpr (CH > 0) {
#pragma unroll
    for (int q = 0; q < CH; ++q)
      if (j0 + q < j1) place(j0 + q, zr[q]);
  } else {
    for (int j = j0; j < j1; ++j) place(j, zval(j));
  }
  if (mode == 2) {
    // b = (A^T y)_S for the refinement, gathered once after the last update
    __syncthreads();   // the support written above is visible to the workgroup
    for (int l = tid; l < K; l += NT) I.b[l] = I.c0[I.support[l]];
  }
  if (tid == 0) {
    *I.nsel = K;
    if (mode >= 1 && !(step_sh <= 3.402823466e38f)) atomicOr(I.status, ST_NAN);
  }
}

// ============================================================ paper-mode CLOMP
// The variant the experiments time (normalised cut-off threshold T_h, R
// iterations of one gradient step each).  Per iteration:
//   r = y - A_S s_S        rows_kernel<ROW_IHT_R>   (skipped at it = 0: r = y)
//   c = A^T r              iht_grad_kernel (+ combine for sliced columns)
//   paper_select_kernel    cmax = max_j |c_j|; the unselected atoms with
//                          |c_j| / cmax >= T_h join the mask unless the support
//                          would exceed k_eff (the batch is then refused whole);
//                          one Adam step on the masked coefficients with
//                          g = -c, lr = lr_rel * cmax, eps = eps_rel * sigma
//                          (sigma = cmax of the first iteration); the support
//                          is rebuilt in index order with its coefficients.
// A non-finite correlation or cmax = 0 ends the loop for the signal (stop),
// and b = (A^T y)_S is gathered then or after the last iteration, for the
// least-squares refinement.
template <int NT>
__global__ __launch_bounds__(NT) void paper_select_kernel(const Inst* __restrict__ insts_c,
                                                         int it, int last, float thr,
                                                         float lr_rel, float beta1, float beta2,
                                                         float bc1, float bc2, float eps_rel) {
  __shared__ float fred[NT / 64];
  __shared__ unsigned ured[NT / 64];
  __shared__ unsigned wsum[NT / 64];
  const Inst& I = insts_c[blockIdx.x];
  if (I.st->done || I.st->stop) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int n = I.n, K = I.k_eff;
  const float* c = I.gbuf;
  const unsigned* bits = I.bitmap;
  const int nsel_old = *I.nsel;
  auto gather_b = [&](int t1) {
    for (int l = tid; l < t1; l += NT) I.b[l] = I.c0[I.support[l]];
  };
  auto in_mask = [&](int j) { return ((bits[j >> 5] >> (j & 31)) & 1u) != 0u; };
  // (1) cmax over every atom, and whether any correlation is non-finite
  float mx = 0.f;
  unsigned bad = 0u;
  for (int j = tid; j < n; j += NT) {
    const float a = fabsf(c[j]);
    bad |= (a <= 3.402823466e38f) ? 0u : 1u;
    mx = fmaxf(mx, a);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    bad |= __shfl_xor(bad, o, 64);
  }
  if (lane == 0) {
    fred[w] = mx;
    ured[w] = bad;
  }
  __syncthreads();
  float cmax = 0.f;
  bad = 0u;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) {
    cmax = fmaxf(cmax, fred[q]);
    bad |= ured[q];
  }
  if (bad || cmax == 0.f) {
    // the loop ends here; the refinement uses the support of the previous
    // iteration
    if (tid == 0) {
      I.st->stop = 1;
      if (bad) atomicOr(I.status, ST_NAN);
    }
    gather_b(nsel_old);
    return;
  }
  float eps;
  if (it == 0) {
    eps = eps_rel * cmax;
    if (tid == 0) {
      I.st->sigma = cmax;
      I.st->eps = eps;
    }
  } else {
    eps = I.st->eps;
  }
  auto passes = [&](int j) { return fabsf(c[j]) / cmax >= thr; };
  // (2) the batch of new atoms (loads only)
  unsigned nnew = 0u;
  for (int j = tid; j < n; j += NT) nnew += (!in_mask(j) && passes(j)) ? 1u : 0u;
  unsigned tot_new;
  (void)block_excl_scan<NT>(nnew, wsum, tot_new);
  const bool accept = tot_new > 0u && (unsigned)nsel_old + tot_new <= (unsigned)K;
  if (tid == 0 && tot_new > 0u && !accept) atomicOr(I.status, ST_K_CAPPED);
  // (3) rounds of NT contiguous chunks of C <= 64 atoms: a load-only pass
  // marks the masked atoms of the chunk (old mask plus the accepted batch),
  // a workgroup scan places them in index order, and only those take the
  // Adam step (g = -c) and are written to the support
  const float lr = lr_rel * cmax;
  const int C = min(64, (n + NT - 1) / NT);
  unsigned base = 0u;
  for (int r0 = 0; r0 < n; r0 += NT * C) {
    const int j0 = r0 + tid * C;
    unsigned long long sel = 0ull, add = 0ull;
    for (int q = 0; q < C; ++q) {
      const int j = j0 + q;
      if (j >= n) break;
      if (in_mask(j)) {
        sel |= 1ull << q;
      } else if (accept && passes(j)) {
        sel |= 1ull << q;
        add |= 1ull << q;
      }
    }
    unsigned tot;
    unsigned pos = base + block_excl_scan<NT>((unsigned)__popcll(sel), wsum, tot);
    while (sel) {
      const int q = __ffsll((long long)sel) - 1;
      sel &= sel - 1ull;
      const int j = j0 + q;
      if ((add >> q) & 1ull) atomicOr(I.bitmap + (j >> 5), 1u << (j & 31));
      const float g = -c[j];
      const float mo = fmaf(beta1, I.mden[j], (1.f - beta1) * g);
      const float ve = fmaf(beta2, I.vden[j], (1.f - beta2) * (g * g));
      const float sj = I.sfull[j] - lr * (mo / bc1) / (sqrtf(ve / bc2) + eps);
      I.mden[j] = mo;
      I.vden[j] = ve;
      I.sfull[j] = sj;
      I.support[pos] = j;
      I.s[pos] = sj;
      ++pos;
    }
    base += tot;
  }
  if (tid == 0) *I.nsel = (int)base;
  if (last) {
    __syncthreads();   // the support written above is visible to the workgroup
    gather_b((int)base);
  }
}

// ============================================================ shared dictionary
// (every iterated signal of the batch has the same A)
// The batch computes the full Gram matrix Gf = A^T A and c0 = A^T y of every
// signal once; an iteration then needs no pass over A: column S_l of Gf is
// H's column l, and the new Gram row of the coefficient update is a lookup.
// C[i, q] = sum_k A[i][k] B_q[k] over 128 x 128 output tiles on the FP32
// matrix cores (v_mfma_f32_16x16x4f32): four waves of 64 x 64, each a 4 x 4
// grid of 16 x 16 blocks; k staged through LDS in chunks of 32 (row stride
// 145 floats: the transposed stores of the eight k groups of a row fall in
// distinct banks), the next chunk's loads in flight during the current
// chunk's products.
// Operand layout of the instruction: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; register v of lane l holds D[4 (l / 16) + v][l % 16].
// MODE 0: B_q = atom q, C = Gf (ld ldh);  MODE 1: B_q = y of signal q (the
// workspace copy), C[:, q] = c0 of signal q;  MODE 2: B_q = the residual r of
// signal q, and instead of C each signal gets the argmax key of its column
// over unselected atoms (key slot `t & 1`): the correlation scan of a whole
// batch as one contraction C = A^T R;  MODE 3: B_q = the residual r of
// signal q, C[:, q] = the gradient g of IHT / paper mode (gbuf), and when
// t != 0 (the first iteration, r = y) also c0.
constexpr int kMfmaTile = 128, kMfmaK = 32, kMfmaLd = 145;
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

template <typename TA, int MODE>
__global__ __launch_bounds__(256) void shared_mfma_kernel(const Inst* __restrict__ insts, int nsig,
                                                          float* __restrict__ Gf, int t) {
  // two buffers: chunk c is staged into buffer c & 1 while the loads of chunk
  // c + 1 are in flight, one barrier per chunk
  __shared__ __align__(16) float As[2][kMfmaK][kMfmaLd];
  __shared__ __align__(16) float Bs[2][kMfmaK][kMfmaLd];
  __shared__ unsigned long long kbest[2][kMfmaTile];
  const Inst& I0 = insts[0];
  const TA* A = reinterpret_cast<const TA*>(I0.A);
  const long long lda = I0.lda, ldh = I0.ldh;
  const int n = I0.n, m = I0.m, m_pad = I0.m_pad;   // shared by every signal
  const int ncols = (MODE == 0) ? n : nsig;
  const int i0 = blockIdx.x * kMfmaTile, q0 = blockIdx.y * kMfmaTile;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;          // the wave's 64-row / 64-column half
  mfma_f4 acc[4][4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mfma_f4{0.f, 0.f, 0.f, 0.f};
  // each thread stages rows rb + 32 u (u < 4) of both operands at k offset kq
  // of every chunk; the row and column pointers are fixed for the launch, and
  // rows or columns outside the matrix read a valid one and are zeroed
  constexpr int kGroups = kMfmaTile * (kMfmaK / 4) / 256;
  const int rb = threadIdx.x / (kMfmaK / 4), kq = (threadIdx.x % (kMfmaK / 4)) * 4;
  const TA* arow[kGroups];
  const TA* brow[kGroups];      // MODE 0: atoms
  const float* bsig[kGroups];   // MODE 1-3: y (MODE 1) or r of the column's signal
  bool aok[kGroups], bok[kGroups];
#pragma unroll
  for (int u = 0; u < kGroups; ++u) {
    const int i = i0 + rb + 32 * u, q = q0 + rb + 32 * u;
    aok[u] = i < n;
    bok[u] = q < ncols;
    arow[u] = A + (long long)(aok[u] ? i : i0) * lda;
    if (MODE == 0) brow[u] = A + (long long)(bok[u] ? q : q0) * lda;
    else bsig[u] = insts[bok[u] ? q : q0].r + (MODE == 1 ? m_pad : 0);
  }
  // four consecutive k of each staged row, loaded raw (A below m only: lda >= m,
  // both multiples of 4, so the load stays in the row; y and r below m_pad,
  // zero padded) and masked only when staged, so that nothing waits for the
  // loads before the products of the current chunk
  const int kbend = (MODE == 0) ? m : m_pad;
  float4 av[kGroups], bv[kGroups];
  auto fetch = [&](int k0) {
    const int k = k0 + kq;
    const int ksa = k < m ? k : 0, ksb = k < kbend ? k : 0;
#pragma unroll
    for (int u = 0; u < kGroups; ++u) {
      av[u] = gload4(arow[u] + ksa);
      bv[u] = (MODE == 0) ? gload4(brow[u] + ksb) : gload4(bsig[u] + ksb);
    }
  };
  fetch(0);
  int buf = 0;
  for (int k0 = 0; k0 < m; k0 += kMfmaK) {
    const int k = k0 + kq;
    // element e of a staged A row (or atom) is used while k + e < m; y and r
    // rows whole below m_pad
    const bool a0 = k < m, a1 = k + 1 < m, a2 = k + 2 < m, a3 = k + 3 < m;
    const bool kb = k < kbend;
#pragma unroll
    for (int u = 0; u < kGroups; ++u) {
      const int r = rb + 32 * u;
      const bool ua = aok[u], ub = bok[u] && kb;
      As[buf][kq + 0][r] = (ua && a0) ? av[u].x : 0.f;
      As[buf][kq + 1][r] = (ua && a1) ? av[u].y : 0.f;
      As[buf][kq + 2][r] = (ua && a2) ? av[u].z : 0.f;
      As[buf][kq + 3][r] = (ua && a3) ? av[u].w : 0.f;
      Bs[buf][kq + 0][r] = ub ? bv[u].x : 0.f;
      Bs[buf][kq + 1][r] = (ub && (MODE != 0 || a1)) ? bv[u].y : 0.f;
      Bs[buf][kq + 2][r] = (ub && (MODE != 0 || a2)) ? bv[u].z : 0.f;
      Bs[buf][kq + 3][r] = (ub && (MODE != 0 || a3)) ? bv[u].w : 0.f;
    }
    __syncthreads();
    if (k0 + kMfmaK < m) fetch(k0 + kMfmaK);   // in flight during the products
#pragma unroll
    for (int ks = 0; ks < kMfmaK; ks += 4) {
      const int kk = ks + (lane >> 4);
      float a[4], b[4];
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) a[bi] = As[buf][kk][64 * wr + 16 * bi + (lane & 15)];
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) b[bj] = Bs[buf][kk][64 * wc + 16 * bj + (lane & 15)];
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
    }
    buf ^= 1;
  }
  // element (bi, bj, v) of this lane: atom i0 + 64 wr + 16 bi + 4 (lane / 16) + v,
  // column q0 + 64 wc + 16 bj + lane % 16
  const int ib = i0 + 64 * wr + 4 * (lane >> 4);
  const int qb = q0 + 64 * wc + (lane & 15);
  if (MODE == 2) {
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      const int q = qb + 16 * bj;
      unsigned long long best = 0ull;
      if (q < ncols) {
        // the wave's 64 rows start at a multiple of 64: two bitmap words
        const unsigned* bm = insts[q].bitmap;
        const int wbase = i0 + 64 * wr;
        const unsigned bw0 = wbase < n ? gmem(bm)[wbase >> 5] : ~0u;
        const unsigned bw1 = wbase + 32 < n ? gmem(bm)[(wbase >> 5) + 1] : ~0u;
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = ib + 16 * bi + v;
            const unsigned word = (16 * bi + 4 * (lane >> 4) + v) < 32 ? bw0 : bw1;
            if (i < n && !((word >> (i & 31)) & 1u)) {
              const unsigned long long kk = pack_key(acc[bi][bj][v], i);
              best = kk > best ? kk : best;
            }
          }
      }
      // lanes l, l+16, l+32, l+48 hold the same column
      for (int o = 16; o < 64; o <<= 1) {
        const unsigned long long other = __shfl_xor(best, o, 64);
        best = other > best ? other : best;
      }
      if (lane < 16) kbest[wr][64 * wc + 16 * bj + lane] = best;
    }
    __syncthreads();
    if (threadIdx.x < kMfmaTile) {
      const int q = q0 + threadIdx.x;
      unsigned long long best = kbest[0][threadIdx.x];
      if (kbest[1][threadIdx.x] > best) best = kbest[1][threadIdx.x];
      if (q < ncols && best) atomicMax(&insts[q].key[t & 1], best);
    }
    return;
  }
  // the lane's four atoms i..i+3 of a block are consecutive: one 16-byte
  // store per block (columns hold ldh >= 128 ceil(n / 128) entries, and atoms
  // at or beyond n were staged as zero rows, so their entries are zero)
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      const int q = qb + 16 * bj;
      if (q >= ncols) continue;
      const int i = ib + 16 * bi;
      const float4 v4 = make_float4(acc[bi][bj][0], acc[bi][bj][1], acc[bi][bj][2],
                                    acc[bi][bj][3]);
      if (MODE == 0) {
        *reinterpret_cast<float4*>(Gf + i + (long long)q * ldh) = v4;
      } else if (MODE == 1) {
        *reinterpret_cast<float4*>(insts[q].c0 + i) = v4;
      } else {
        *reinterpret_cast<float4*>(insts[q].gbuf + i) = v4;
        if (t) *reinterpret_cast<float4*>(insts[q].c0 + i) = v4;
      }
    }
}

// BF16 bulk matrix: the same contractions on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation), for MODE 0 (Gf = A^T A, both
// operands the stored BF16 atoms, so every product is exact and only the
// accumulation order differs from the FP32 kernel) and MODE 2 (the scan: the
// residuals rounded to BF16, round to nearest even, as they are staged).  The
// tile, wave split and epilogue are those of shared_mfma_kernel; k is staged in
// chunks of 32 as BF16 rows with k contiguous (row stride 40 elements, so the
// 16-byte operand reads of a 16-lane group fall in distinct banks), two
// buffers, the next chunk's loads in flight during the products.
// Operand layout of the instruction: lane l supplies A[l % 16][8 (l / 16) + e]
// and B[8 (l / 16) + e][l % 16] (e < 8); register v of lane l holds
// D[4 (l / 16) + v][l % 16] (checked with an in-bounds probe on the GPU).
constexpr int kBfK = 32, kBfLd = 40;
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_bits_rne(float x) {
  const __bf16 h = (__bf16)x;               // IEEE conversion: round to nearest even
  return __builtin_bit_cast(unsigned short, h);
}

template <int MODE>
__global__ __launch_bounds__(256) void shared_mfma_bf16_kernel(const Inst* __restrict__ insts,
                                                               int nsig, float* __restrict__ Gf,
                                                               int t) {
  static_assert(MODE == 0 || MODE == 2, "BF16 contraction: Gram matrix or scan");
  __shared__ __align__(16) unsigned short As[2][kMfmaTile][kBfLd];
  __shared__ __align__(16) unsigned short Bs[2][kMfmaTile][kBfLd];
  __shared__ unsigned long long kbest[2][kMfmaTile];
  const Inst& I0 = insts[0];
  const uint16_t* A = reinterpret_cast<const uint16_t*>(I0.A);
  const long long lda = I0.lda, ldh = I0.ldh;
  const int n = I0.n, m = I0.m, m_pad = I0.m_pad;   // shared by every signal
  const int ncols = (MODE == 0) ? n : nsig;
  const int i0 = blockIdx.x * kMfmaTile, q0 = blockIdx.y * kMfmaTile;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  mfma_f4 acc[4][4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mfma_f4{0.f, 0.f, 0.f, 0.f};
  // A side: thread stages 8 consecutive k (one 16-byte load) of rows
  // ra + 64 u, u < 2, at k offset ka of every chunk
  const int ra = tid >> 2, ka = (tid & 3) * 8;
  const uint16_t* arow[2];
  bool aok[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = i0 + ra + 64 * u;
    aok[u] = i < n;
    arow[u] = A + (long long)(aok[u] ? i : i0) * lda;
  }
  // B side: MODE 0 as the A side (atoms); MODE 2 four consecutive FP32
  // residual entries (one 16-byte load) of columns rc + 32 u, u < 4, at k
  // offset kc of every chunk
  const int rc = tid >> 3, kc = (tid & 7) * 4;
  const uint16_t* brow[2];
  const float* bsig[4];
  bool bok[4];
  if (MODE == 0) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = q0 + ra + 64 * u;
      bok[u] = q < ncols;
      brow[u] = A + (long long)(bok[u] ? q : q0) * lda;
    }
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = q0 + rc + 32 * u;
      bok[u] = q < ncols;
      bsig[u] = insts[bok[u] ? q : q0].r;
    }
  }
  uint4 av[2], bvh[2];
  float4 bvf[4];
  // raw loads from clamped addresses (k below m for A rows: lda >= m and both
  // multiples of 8, so a 16-byte load starting below m stays in the row; r
  // below m_pad, a multiple of 8); the masks are applied when staging
  auto fetch = [&](int k0) {
    const int k = k0 + ka;
    const int ks = k < m ? k : 0;
#pragma unroll
    for (int u = 0; u < 2; ++u) av[u] = gload16(arow[u] + ks);
    if (MODE == 0) {
#pragma unroll
      for (int u = 0; u < 2; ++u) bvh[u] = gload16(brow[u] + ks);
    } else {
      const int kb = k0 + kc;
      const int kbs = kb < m_pad ? kb : 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) bvf[u] = gload4(bsig[u] + kbs);
    }
  };
  // zero the bf16 entries of a 16-byte group at or beyond m (nk valid ones)
  auto mask8 = [](uint4 q, int nk) -> uint4 {
    if (nk >= 8) return q;
    unsigned wv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const unsigned lo = (2 * e < nk) ? 0x0000ffffu : 0u;
      const unsigned hi = (2 * e + 1 < nk) ? 0xffff0000u : 0u;
      wv[e] &= (lo | hi);
    }
    return make_uint4(wv[0], wv[1], wv[2], wv[3]);
  };
  fetch(0);
  int buf = 0;
  for (int k0 = 0; k0 < m; k0 += kBfK) {
    {
      const int nk = m - (k0 + ka);           // valid entries of this thread's A group
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const uint4 q = (aok[u] && nk > 0) ? mask8(av[u], nk) : make_uint4(0u, 0u, 0u, 0u);
        *reinterpret_cast<uint4*>(&As[buf][ra + 64 * u][ka]) = q;
      }
      if (MODE == 0) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const uint4 q = (bok[u] && nk > 0) ? mask8(bvh[u], nk) : make_uint4(0u, 0u, 0u, 0u);
          *reinterpret_cast<uint4*>(&Bs[buf][ra + 64 * u][ka]) = q;
        }
      } else {
        const int kb = k0 + kc;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float4 f = bvf[u];
          const bool ok = bok[u];
          const unsigned short h0 = (ok && kb < m) ? bf16_bits_rne(f.x) : 0;
          const unsigned short h1 = (ok && kb + 1 < m) ? bf16_bits_rne(f.y) : 0;
          const unsigned short h2 = (ok && kb + 2 < m) ? bf16_bits_rne(f.z) : 0;
          const unsigned short h3 = (ok && kb + 3 < m) ? bf16_bits_rne(f.w) : 0;
          *reinterpret_cast<uint2*>(&Bs[buf][rc + 32 * u][kc]) =
              make_uint2((unsigned)h0 | ((unsigned)h1 << 16), (unsigned)h2 | ((unsigned)h3 << 16));
        }
      }
    }
    __syncthreads();
    if (k0 + kBfK < m) fetch(k0 + kBfK);   // in flight during the products
    const int kk = 8 * (lane >> 4);
    bf16x8_t a[4], b[4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
      const uint4 q = *reinterpret_cast<const uint4*>(&As[buf][64 * wr + 16 * bi + (lane & 15)][kk]);
      a[bi] = __builtin_bit_cast(bf16x8_t, q);
    }
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      const uint4 q = *reinterpret_cast<const uint4*>(&Bs[buf][64 * wc + 16 * bj + (lane & 15)][kk]);
      b[bj] = __builtin_bit_cast(bf16x8_t, q);
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
    buf ^= 1;
  }
  const int ib = i0 + 64 * wr + 4 * (lane >> 4);
  const int qb = q0 + 64 * wc + (lane & 15);
  if (MODE == 2) {
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      const int q = qb + 16 * bj;
      unsigned long long best = 0ull;
      if (q < ncols) {
        const unsigned* bm = insts[q].bitmap;
        const int wbase = i0 + 64 * wr;
        const unsigned bw0 = wbase < n ? gmem(bm)[wbase >> 5] : ~0u;
        const unsigned bw1 = wbase + 32 < n ? gmem(bm)[(wbase >> 5) + 1] : ~0u;
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = ib + 16 * bi + v;
            const unsigned word = (16 * bi + 4 * (lane >> 4) + v) < 32 ? bw0 : bw1;
            if (i < n && !((word >> (i & 31)) & 1u)) {
              const unsigned long long kk2 = pack_key(acc[bi][bj][v], i);
              best = kk2 > best ? kk2 : best;
            }
          }
      }
      for (int o = 16; o < 64; o <<= 1) {
        const unsigned long long other = __shfl_xor(best, o, 64);
        best = other > best ? other : best;
      }
      if (lane < 16) kbest[wr][64 * wc + 16 * bj + lane] = best;
    }
    __syncthreads();
    if (tid < kMfmaTile) {
      const int q = q0 + tid;
      unsigned long long best = kbest[0][tid];
      if (kbest[1][tid] > best) best = kbest[1][tid];
      if (q < ncols && best) atomicMax(&insts[q].key[t & 1], best);
    }
    return;
  }
  // MODE 0: the lane's four atoms of a block are consecutive (one 16-byte
  // store; columns hold ldh >= 128 ceil(n / 128) entries, rows past n are zero)
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      const int q = qb + 16 * bj;
      if (q >= ncols) continue;
      const int i = ib + 16 * bi;
      *reinterpret_cast<float4*>(Gf + i + (long long)q * ldh) =
          make_float4(acc[bi][bj][0], acc[bi][bj][1], acc[bi][bj][2], acc[bi][bj][3]);
    }
}

// Products over one signal's support, one 256-thread workgroup per signal
// (t1 <= 256 atoms: the given count, or the signal's own when 0), the support
// and coefficients staged in LDS, each lane's four consecutive rows read with
// one vector load per support column and summed over four independent chains
// (the shared A is cache resident; one workgroup per signal keeps the launch
// small).  MODE 0: r = y - A_S s;  MODE 1: the IHT
// step denominator ||A_S g_S||^2 (g from gbuf) as the signal's row partials
// (the total in the first, zeros in the others).
template <typename TA, int MODE>
__global__ __launch_bounds__(256) void shared_rows_kernel(const Inst* __restrict__ insts,
                                                          int t1_arg) {
  __shared__ float ssh[256];
  __shared__ int jsh[256];
  __shared__ float red[4];
  const Inst& I = insts[blockIdx.x];
  if (I.st->done || I.st->stop) return;
  const int t1 = t1_arg > 0 ? t1_arg : *I.nsel;
  for (int l = threadIdx.x; l < t1; l += 256) {
    const int j = I.support[l];
    jsh[l] = j;
    ssh[l] = (MODE == 0) ? I.s[l] : I.gbuf[j];
  }
  __syncthreads();
  const TA* A = reinterpret_cast<const TA*>(I.A);
  const long long lda = I.lda;
  const int m = I.m;
  // lane v takes rows 4v..4v+3 with one vector load per support column (the
  // rows of A are padded to lda, a multiple of 4, and r, y to m_pad, a
  // multiple of 8); each row keeps four chains over l mod 4
  const int ng = (m + 3) >> 2;
  const float* yw = I.r + I.m_pad;
  float sq = 0.f;
  auto fma4 = [](float4 x, float c, float4 a) {
    return make_float4(fmaf(x.x, c, a.x), fmaf(x.y, c, a.y), fmaf(x.z, c, a.z),
                       fmaf(x.w, c, a.w));
  };
  for (int v = threadIdx.x; v < ng; v += 256) {
    const int i = 4 * v;
    float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = a0, a2 = a0, a3 = a0;
    int l = 0;
#pragma unroll 2
    for (; l + 3 < t1; l += 4) {
      const float4 x0 = gload4(A + (long long)jsh[l] * lda + i);
      const float4 x1 = gload4(A + (long long)jsh[l + 1] * lda + i);
      const float4 x2 = gload4(A + (long long)jsh[l + 2] * lda + i);
      const float4 x3 = gload4(A + (long long)jsh[l + 3] * lda + i);
      a0 = fma4(x0, ssh[l], a0);
      a1 = fma4(x1, ssh[l + 1], a1);
      a2 = fma4(x2, ssh[l + 2], a2);
      a3 = fma4(x3, ssh[l + 3], a3);
    }
    for (; l < t1; ++l) a0 = fma4(gload4(A + (long long)jsh[l] * lda + i), ssh[l], a0);
    const float u[4] = {(a0.x + a1.x) + (a2.x + a3.x), (a0.y + a1.y) + (a2.y + a3.y),
                        (a0.z + a1.z) + (a2.z + a3.z), (a0.w + a1.w) + (a2.w + a3.w)};
    if (MODE == 0) {
      // rows at or beyond m stay zero
      const float4 y4 = gload4(yw + i);
      *reinterpret_cast<float4*>(I.r + i) =
          make_float4(y4.x - u[0], i + 1 < m ? y4.y - u[1] : 0.f,
                      i + 2 < m ? y4.z - u[2] : 0.f, i + 3 < m ? y4.w - u[3] : 0.f);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (i + e < m) sq = fmaf(u[e], u[e], sq);
    }
  }
  if (MODE == 1) {
    const float tot = block_sum(sq, red);
    for (int q = threadIdx.x; q < I.n_rowtiles; q += 256) I.qpart[q] = (q == 0) ? tot : 0.f;
  }
}

// The shared Gram diagonal (prior included) for the coefficient updates.
__global__ __launch_bounds__(kBlock) void shared_diag_kernel(const Inst* __restrict__ insts,
                                                             const float* __restrict__ Gf,
                                                             float* __restrict__ dg) {
  const Inst& I0 = insts[0];
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j < I0.n) dg[j] = Gf[j + (long long)j * I0.ldh] + tv_diag(I0, j);
}

// ============================================================ fused small-signal loop
// One workgroup runs the whole greedy loop of one signal whose dictionary fits
// in LDS: A is converted to FP32 once (row j of the LDS image is atom j, with
// an odd leading dimension so lanes reading consecutive atoms hit distinct
// banks), then every iteration - correlation scan and argmax, selection
// record, new Gram column, coefficient update, residual - stays on chip.  The
// coefficient update runs in wave 0 with lane r owning row r (k_eff <= 64):
// the T Adam steps (or the OMP bordered-inverse update) need no workgroup
// barrier.  Arithmetic follows the per-iteration kernels; summation orders
// differ.  The loop leaves s, b, the support and the state in the workspace
// for the refinement and the FP64 norm.
constexpr int kSmallThreads = 512;
constexpr int kSmallWaves = kSmallThreads / 64;
constexpr int kSmallDots = (kSmallMaxK + 2 + kSmallWaves - 1) / kSmallWaves;   // per wave

// Row r of G times s in one Adam step of the fused loop: lane r holds its row
// in registers (grow_r, zero beyond t+1) and takes s_c from lane c, in
// blocks of eight columns up to t+1, summed in column order into acc[c % 4].
template <int KR>
__device__ inline void small_row_times_s(const float (&grow_r)[KR], float sv, int t1,
                                         float (&acc)[4]) {
#pragma unroll
  for (int b = 0; b < KR / 8; ++b) {
    if (8 * b < t1) {
      float sc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        sc[u] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sv), 8 * b + u));
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u & 3] = fmaf(grow_r[8 * b + u], sc[u], acc[u & 3]);
    }
  }
}

// KR: register row length of the Adam step (8, 16, 32 or 64, at least the
// batch's largest k_eff; OMP ignores it)
template <typename TA, bool OMP, int KR>
__global__ __launch_bounds__(kSmallThreads) void small_loop_kernel(
    const Inst* __restrict__ insts, const int* __restrict__ list, int T, float beta1,
    float beta2, float lr_rel, float eps_rel) {
  extern __shared__ __align__(16) float sm[];
  __shared__ unsigned long long wkey[kSmallWaves];
  __shared__ __align__(16) float sbuf[2][kSmallMaxK];   // coefficients (ping-pong) / OMP v
  __shared__ __align__(16) float gcol[kSmallMaxK + 4];  // G[l, t] (l < t), ||a_j||^2, a_j^T y
  __shared__ float bsh[kSmallMaxK];
  __shared__ __align__(16) int off[kSmallMaxK];         // LDS offset of selected atom l
  const Inst& I = insts[list[blockIdx.x]];
  if (I.st->done) return;   // y == 0: init has finished the signal
  const int n = I.n, m = I.m, ke = I.k_eff;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int ldl = m | 1;
  const int ldq = small_ldq(ke);
  const int m4 = (m + 3) & ~3;
  float* Gq = sm;                                   // [ke][ldq] G (CLOMP) or Ginv (OMP)
  float* Al = Gq + (size_t)ke * ldq;                // [n][ldl]
  float* r = Al + (((size_t)n * ldl + 3) & ~(size_t)3);   // [m4], zero beyond m
  float* yl = r + m4;                               // [m4], zero beyond m
  unsigned* bm = reinterpret_cast<unsigned*>(yl + m4);    // [ceil(n/32)]
  // lanes per atom in the scan: the most (up to 8) that keep every lane busy
  int G = 1;
  while (G < 8 && 2 * G * n <= kSmallThreads) G <<= 1;
  // ---- stage A, y, and clear the state
  {
    constexpr int VW = Vec<TA>::W;
    const int nvec = (m + VW - 1) / VW;
    const TA* A = reinterpret_cast<const TA*>(I.A);
    for (int q = tid; q < n * nvec; q += kSmallThreads) {
      const int j = q / nvec, c = q - j * nvec;
      float v[VW];
      Vec<TA>::load(A + (long long)j * I.lda + (long long)c * VW, v);
#pragma unroll
      for (int e = 0; e < VW; ++e)
        if (c * VW + e < m) Al[(size_t)j * ldl + c * VW + e] = v[e];
    }
  }
  for (int i = tid; i < m4; i += kSmallThreads) {
    const float v = (i < m) ? I.y[i] : 0.f;
    r[i] = v;
    yl[i] = v;
  }
  for (int q = tid; q < ke * ldq; q += kSmallThreads) Gq[q] = 0.f;
  for (int q = tid; q < (n + 31) / 32; q += kSmallThreads) bm[q] = 0u;
  if (tid < kSmallMaxK) {
    sbuf[0][tid] = 0.f;
    sbuf[1][tid] = 0.f;
    off[tid] = 0;
  }
  if (tid < kSmallMaxK + 4) gcol[tid] = 0.f;
  __syncthreads();
  float sv = 0.f, mo = 0.f, ve = 0.f;   // wave 0, lane r: coefficient r and its moments
  double b1p = 1.0, b2p = 1.0;          // beta^step, carried across iterations
  float lr = 0.f, eps = 0.f, sigma = 0.f;
  int step = 0, cur = 0, t = 0;
  for (; t < ke; ++t) {
    // ---- correlations of the unselected atoms and the argmax key: G lanes
    // per atom, lane g taking the 4-element chunks g, g+G, ...
    unsigned long long best = 0ull;
    {
      const int g = tid % G;
      for (int j = tid / G; j < n; j += kSmallThreads / G) {
        const float* a = Al + (size_t)j * ldl;
        float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;
#pragma unroll 4
        for (int i0 = 4 * g; i0 < m; i0 += 4 * G) {
          const float4 r4 = *reinterpret_cast<const float4*>(r + i0);
          const float a0 = a[i0];
          const float a1 = (i0 + 1 < m) ? a[i0 + 1] : 0.f;
          const float a2 = (i0 + 2 < m) ? a[i0 + 2] : 0.f;
          const float a3 = (i0 + 3 < m) ? a[i0 + 3] : 0.f;
          acc0 = fmaf(a0, r4.x, acc0);
          acc1 = fmaf(a1, r4.y, acc1);
          acc2 = fmaf(a2, r4.z, acc2);
          acc3 = fmaf(a3, r4.w, acc3);
        }
        float c = (acc0 + acc1) + (acc2 + acc3);
        for (int o = G >> 1; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        const unsigned selb = (bm[j >> 5] >> (j & 31)) & 1u;
        const unsigned long long key = selb ? 0ull : pack_key(c, j);
        best = key > best ? key : best;
      }
    }
    best = wave_max_u64(best);
    if (lane == 0) wkey[w] = best;
    __syncthreads();
    unsigned long long key = wkey[0];
#pragma unroll
    for (int q = 1; q < kSmallWaves; ++q) key = wkey[q] > key ? wkey[q] : key;
    const int j = key_index(key);
    if (key == 0ull || j < 0 || j >= n) {
      if (tid == 0) {
        I.st->done = 1;
        atomicOr(I.status, ST_WATCHDOG);
      }
      break;
    }
    const float cj = key_value(key);
    if (t == 0) {
      sigma = cj;
      eps = eps_rel * cj;
    }
    lr = lr_rel * cj;   // step size follows the selected correlation
    // ---- selection record and the new Gram column: wave w forms the partial
    // sums of its dots l = w, w + 8, ... first, then reduces them
    if (tid == 0) {
      I.support[t] = j;
      *I.nsel = t + 1;
      if (!(cj <= 3.402823466e38f)) atomicOr(I.status, ST_NAN);
      bm[j >> 5] |= 1u << (j & 31);
      off[t] = j * ldl;
    }
    {
      const float* aj = Al + (size_t)j * ldl;
      float part[kSmallDots];
#pragma unroll
      for (int q = 0; q < kSmallDots; ++q) {
        const int l = w + q * kSmallWaves;
        float acc = 0.f;
        if (l < t + 2) {
          const float* v = (l < t) ? Al + off[l] : (l == t ? aj : yl);
          for (int i = lane; i < m; i += 64) acc = fmaf(aj[i], v[i], acc);
        }
        part[q] = acc;
      }
#pragma unroll
      for (int q = 0; q < kSmallDots; ++q) part[q] = wave_sum(part[q]);
      if (lane == 0) {
#pragma unroll
        for (int q = 0; q < kSmallDots; ++q) {
          const int l = w + q * kSmallWaves;
          if (l < t + 2) gcol[l] = (l == t) ? part[q] + tv_diag(I, j) : part[q];
        }
      }
    }
    __syncthreads();
    // ---- coefficient update (wave 0)
    if (w == 0) {
      const int t1 = t + 1;
      if (!OMP) {
        for (int c = lane; c <= t; c += 64) {
          Gq[(size_t)t * ldq + c] = gcol[c];
          Gq[(size_t)c * ldq + t] = gcol[c];
        }
        if (lane == 0) bsh[t] = gcol[t + 1];
        wave_sync();
        const float bb = (lane < t1) ? bsh[lane] : 0.f;
        const float* grow = Gq + (size_t)(lane < ke ? lane : 0) * ldq;
        // the row of G in registers for the T steps (columns < t+1; the
        // rest zero), so a step reads no LDS: s_c comes from lane c
        float grow_r[KR];
#pragma unroll
        for (int c = 0; c < KR; ++c) grow_r[c] = (c < t1) ? grow[c] : 0.f;
        for (int it = 0; it < T; ++it) {
          b1p *= beta1;
          b2p *= beta2;
          const float ibc1 = __builtin_amdgcn_rcpf((float)(1.0 - b1p));
          const float ibc2 = __builtin_amdgcn_rcpf((float)(1.0 - b2p));
          float acc[4] = {0.f, 0.f, 0.f, 0.f};
          small_row_times_s<KR>(grow_r, sv, t1, acc);
          if (lane < t1) {
            const float gr = ((acc[0] + acc[1]) + (acc[2] + acc[3])) - bb;
            mo = beta1 * mo + (1.f - beta1) * gr;
            ve = beta2 * ve + (1.f - beta2) * (gr * gr);
            const float mh = mo * ibc1;
            const float vh = ve * ibc2;
            sv = sv - lr * mh * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(vh) + eps);
          }
        }
        // s for the residual and the next iteration: the buffer that every
        // thread selects below (cur ^ (T & 1))
        if (lane < t1) sbuf[cur ^ (T & 1)][lane] = sv;
      } else {
        // bordered inverse: v = Ginv g, delta = gamma - g.v,
        // alpha = (b_t - g.x) / delta, x <- [x - alpha v; alpha]
        const float* grow = Gq + (size_t)(lane < ke ? lane : 0) * ldq;
        float a4[4] = {0.f, 0.f, 0.f, 0.f};
        if (lane < t) {
          // the 16-byte reads run to the next multiple of 4: Ginv has no
          // entries in columns >= t yet, so g's tail does not contribute
          for (int c = 0; c < t; c += 4) {
            const float4 g4 = *reinterpret_cast<const float4*>(grow + c);
            const float4 c4 = *reinterpret_cast<const float4*>(gcol + c);
            a4[0] = fmaf(g4.x, c4.x, a4[0]);
            a4[1] = fmaf(g4.y, c4.y, a4[1]);
            a4[2] = fmaf(g4.z, c4.z, a4[2]);
            a4[3] = fmaf(g4.w, c4.w, a4[3]);
          }
        }
        const float vr = (a4[0] + a4[1]) + (a4[2] + a4[3]);
        const float gv = wave_sum(lane < t ? gcol[lane] * vr : 0.f);
        const float gx = wave_sum(lane < t ? gcol[lane] * sv : 0.f);
        const float gamma = gcol[t];
        float delta = gamma - gv;
        const bool bad = !(delta > 1e-7f * gamma);
        if (bad) delta = fmaxf(1e-7f * gamma, 1e-30f);
        const float inv = 1.f / delta;
        const float alpha = (gcol[t + 1] - gx) * inv;
        sbuf[0][lane] = (lane < t) ? vr : 0.f;
        if (lane == 0) bsh[t] = gcol[t + 1];
        wave_sync();
        if (lane < t) {
          float* row = Gq + (size_t)lane * ldq;
          const float vi = vr * inv;
          for (int c = 0; c < t; ++c) row[c] = fmaf(sbuf[0][c], vi, row[c]);
          row[t] = -vi;
          sv = fmaf(-alpha, vr, sv);
        } else if (lane == t) {
          float* row = Gq + (size_t)t * ldq;
          for (int c = 0; c < t; ++c) row[c] = -sbuf[0][c] * inv;
          row[t] = inv;
          sv = alpha;
        }
        if (bad && lane == 0) atomicOr(I.status, ST_REFINE_INACCURATE);
        if (lane < t1) sbuf[1][lane] = sv;
      }
    }
    if (!OMP) step += T;
    __syncthreads();
    if (!OMP) cur ^= (T & 1);   // every thread tracks the buffer holding s
    // ---- residual r = y - A_S s, eight selected columns per round
    {
      const float* sc = sbuf[OMP ? 1 : cur];
      const int t1 = t + 1;
      for (int i = tid; i < m; i += kSmallThreads) {
        float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        int l = 0;
        for (; l + 8 <= t1; l += 8) {
#pragma unroll
          for (int u = 0; u < 8; ++u) a[u] = fmaf(Al[off[l + u] + i], sc[l + u], a[u]);
        }
        for (int u = 0; l + u < t1; ++u) a[u] = fmaf(Al[off[l + u] + i], sc[l + u], a[u]);
        r[i] = yl[i] - (((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7])));
      }
    }
    __syncthreads();
  }
  // ---- state for the refinement and the norm
  if (w == 0 && lane < t) {
    I.s[lane] = sv;
    I.b[lane] = bsh[lane];
    if (!OMP) {
      I.mo[lane] = mo;
      I.ve[lane] = ve;
    }
  }
  if (tid == 0) {
    I.st->sigma = sigma;
    I.st->lr = lr;
    I.st->eps = eps;
    I.st->step = step;
  }
}

// ============================================================ correlation-update schedule
// For one (or a few) large signals the greedy loop is latency bound: the
// Adam steps of an iteration are a serial chain on one CU while the scan
// needs the whole GPU.  By linearity
//   c = A^T r = A^T (y - A_S s) = A^T y - sum_l s_l (A^T a_{S_l}),
// so with c0 = A^T y and H[:, l] = A^T a_{S_l} stored, the correlation of
// iteration t+1 is c0 - H s (n * t multiply-adds from L2/MALL) and the one
// full pass over A per iteration computes h_t = A^T a_{j_t}, which depends
// only on the selected atom.  That pass runs in the same launch as the
// coefficient update of iteration t (block 0 updates, the other blocks
// stream A), hiding the serial Adam chain behind the HBM-bound pass.

constexpr int kPassThreads = 1024;   // adam_split_body assumes this size

// One tile of a pass over A with a staged vector v (zero padded):
//   MODE 0: v = y, writes c0[j] = a_j^T y and the argmax key of |c0|
//   MODE 1: v = a_{S_t}, writes H[j, t] = a_j^T a_{S_t}
// bf16 pairs: x.lo * y.lo + x.hi * y.hi + acc in FP32 (v_dot2c_f32_bf16)
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ inline float dot2_bf16(unsigned x, unsigned y, float acc) {
  return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, x),
                                         __builtin_bit_cast(bf16x2_t, y), acc, false);
}
// zero the bf16 elements [tail, 8) of a 16-byte chunk
__device__ inline uint4 mask_bf16_tail(uint4 q, int tail) {
  unsigned w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const unsigned keep = (2 * e + 1 < tail) ? 0xffffffffu : (2 * e < tail ? 0x0000ffffu : 0u);
    w[e] &= keep;
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

template <typename TA, int LPA, int MODE>
__device__ void pass_tile_body(const Inst& I, const ScanTile& tile, int t, float* vsh,
                               unsigned long long* wbest) {
  if (I.st->done) return;
  constexpr int VW = Vec<TA>::W;
  constexpr int NT = kPassThreads;
  // the pass of a selected BF16 atom keeps the atom as bf16 in LDS and
  // contracts bf16 pairs directly
  constexpr bool BF = sizeof(TA) == 2 && MODE == 1;
  const int m = I.m;
  const int nvec = (m + VW - 1) / VW;
  const int tail = m - (nvec - 1) * VW;
  const TA* A = reinterpret_cast<const TA*>(I.A);
  const long long lda = I.lda;
  uint4* vsh4 = reinterpret_cast<uint4*>(vsh);
  if (MODE == 0) {
    const float* yw = I.r + I.m_pad;   // zero padded beyond m
    for (int i = threadIdx.x; i < nvec * VW; i += NT) vsh[i] = yw[i];
  } else {
    // the atom selected by the scan of iteration t (key slot t & 1 is not
    // cleared before this launch ends)
    const int jt = key_index(I.key[t & 1]);
    if (jt < 0 || jt >= I.n) return;
    const TA* colj = A + (long long)jt * lda;
    for (int c = threadIdx.x; c < nvec; c += NT) {
      if constexpr (BF) {
        uint4 q = gload16(colj + (long long)c * VW);
        vsh4[c] = (c == nvec - 1) ? mask_bf16_tail(q, tail) : q;
      } else {
        float a[VW];
        Vec<TA>::load(colj + (long long)c * VW, a);
#pragma unroll
        for (int e = 0; e < VW; ++e) vsh[c * VW + e] = (c * VW + e < m) ? a[e] : 0.f;
      }
    }
  }
  __syncthreads();
  const int gl = threadIdx.x % LPA;
  const int grp = threadIdx.x / LPA;
  constexpr int NG = NT / LPA;
  unsigned long long best = 0ull;
  // 16-byte loads in flight per lane: 8, except 4 when BF16 chunks expand
  // to FP32 (the first pass against the FP32 measurements)
  constexpr int UNR = (sizeof(TA) == 2 && !BF) ? 4 : 8;
  for (int j = tile.j0 + grp; j < tile.j1; j += NG) {
    const TA* col = A + (long long)j * lda;
    float acc = 0.f, acc2 = 0.f, nrm = 0.f;
#pragma unroll UNR
    for (int c = gl; c < nvec; c += LPA) {
      if constexpr (BF) {
        uint4 q = gload16(col + (long long)c * VW);
        if (c == nvec - 1) q = mask_bf16_tail(q, tail);
        const uint4 u = vsh4[c];
        acc = dot2_bf16(q.x, u.x, acc);
        acc2 = dot2_bf16(q.y, u.y, acc2);
        acc = dot2_bf16(q.z, u.z, acc);
        acc2 = dot2_bf16(q.w, u.w, acc2);
      } else {
        float v[VW];
        Vec<TA>::load(col + (long long)c * VW, v);
        if (c == nvec - 1) {
#pragma unroll
          for (int e = 0; e < VW; ++e) v[e] = (e < tail) ? v[e] : 0.f;
        }
        const float* vv = vsh + c * VW;
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          acc = fmaf(v[e], vv[e], acc);
          if (MODE == 0) nrm = fmaf(v[e], v[e], nrm);
        }
      }
    }
    acc = group_sum<LPA>(acc + acc2);
    if (MODE == 0) {
      // the first pass also records ||a_j||^2, the Gram diagonal
      nrm = group_sum<LPA>(nrm);
      if (gl == 0) {
        I.c0[j] = acc;
        I.dg[j] = nrm + tv_diag(I, j);   // Gram diagonal (prior included)
      }
      const unsigned long long key = pack_key(acc, j);
      best = key > best ? key : best;
    } else {
      if (gl == 0) I.H[j + (long long)t * I.ldh] = acc;
    }
  }
  if (MODE == 0) {
    best = wave_max_u64(best);
    if ((threadIdx.x & 63) == 0) wbest[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long b = wbest[0];
      for (int w = 1; w < NT / 64; ++w) b = wbest[w] > b ? wbest[w] : b;
      if (b) atomicMax(I.key, b);
    }
  }
}

template <typename TA, int LPA>
__global__ __launch_bounds__(kPassThreads) void ypass_kernel(const Inst* __restrict__ insts,
                                                             const ScanTile* __restrict__ tiles) {
  extern __shared__ __align__(16) float dsh[];
  __shared__ unsigned long long wbest[kPassThreads / 64];
  const ScanTile tile = tiles[blockIdx.x];
  pass_tile_body<TA, LPA, 0>(insts[tile.inst], tile, 0, dsh, wbest);
}

// ---- teams: several blocks share one signal's coefficient update ----------
// For supports beyond the register tile, W blocks (members) of the fused
// launch split the rows of the update.  Members are the first blocks of the
// launch and W times the number of signals stays below the CU count, so all
// members are resident together.  Members exchange values as 64-bit words
// (tag << 32 | float bits) written and read with agent-scope atomics: a
// reader waits until the word carries the tag it expects, so the value and
// its readiness travel together and no read-modify-write barrier is needed.
// Tags grow strictly within a solve (Adam step number, or t+1 for OMP) and
// the words are zeroed at solve start.  A wait is bounded (I.spin polls): on
// expiry it sets
// the watchdog bit, which ends every other wait of the signal at once; the
// launch then finishes with unspecified coefficients and member 0 retires
// the signal.
__device__ inline void team_put(unsigned long long* p, unsigned tag, float v) {
  __hip_atomic_store(p, ((unsigned long long)tag << 32) | __float_as_uint(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline float team_get(const Inst& I, const unsigned long long* p, unsigned tag) {
  unsigned long long w = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned spins = 0;
  while ((unsigned)(w >> 32) != tag) {
    __builtin_amdgcn_s_sleep(1);
    if (__hip_atomic_load(I.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ST_WATCHDOG)
      break;
    if (++spins > I.spin) {
      atomicOr(I.status, ST_WATCHDOG);
      break;
    }
    w = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return __uint_as_float((unsigned)w);
}

// after a team update: a signal whose team timed out takes no further part
__device__ inline void team_retire(const Inst& I, int w) {
  if (w == 0 && threadIdx.x == 0 &&
      (__hip_atomic_load(I.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ST_WATCHDOG))
    I.st->done = 1;
}


// Selection record of iteration t (atom j of `key`, all threads of the
// workgroup): support, bitmap and count, the new Gram row and column from H
// and the diagonal, b_t = c0[j], the step size and eps, and the next scan's
// key slot cleared.  NT: threads of the workgroup (0: read blockDim).
template <int NT>
__device__ inline void record_selection(const Inst& I, unsigned long long key, int t,
                                        float lr_rel, float eps_rel) {
  const int j = key_index(key);
  const int stride = NT > 0 ? NT : (int)blockDim.x;
  // two loops, so that the per-signal H path issues no support load
  if (I.Gf) {
    for (int l = threadIdx.x; l < t; l += stride) {
      const float g = I.Gf[j + (long long)I.support[l] * I.ldh];
      I.G[l + (long long)t * I.ldg] = g;
      I.G[t + (long long)l * I.ldg] = g;
    }
  } else {
    for (int l = threadIdx.x; l < t; l += stride) {
      const float g = I.H[j + (long long)l * I.ldh];
      I.G[l + (long long)t * I.ldg] = g;
      I.G[t + (long long)l * I.ldg] = g;
    }
  }
  if (threadIdx.x == 0) {
    I.G[t + (long long)t * I.ldg] = I.dg[j];
    I.b[t] = I.c0[j];
    I.support[t] = j;
    I.bitmap[j >> 5] |= (1u << (j & 31));
    *I.nsel = t + 1;
    const float cj = key_value(key);
    if (!(cj <= 3.402823466e38f)) atomicOr(I.status, ST_NAN);
    if (t == 0) {
      I.st->sigma = cj;
      I.st->eps = eps_rel * cj;
    }
    I.st->lr = lr_rel * cj;   // step size follows the selected correlation
    I.key[(t + 1) & 1] = 0ull;   // slot of the next scan
  }
}

// Entry G[r, c] of the Gram matrix during iteration t (atom j selected):
// entries of earlier iterations from G, the new row / column from H and the
// norms (member 0 writes them to G in this same launch).
__device__ inline float gram_at(const Inst& I, int j, int t, int r, int c) {
  if (r < t && c < t) return I.G[c + (long long)r * I.ldg];
  if (r == t && c == t) return I.dg[j];
  return hcol(I, r < t ? r : c)[j];
}

// Adam on rows [16w, 16w+16) of a support of t+1 atoms (same update as the
// single-block bodies).  Wave rho owns row r = 16w + rho: lane q holds
// G[r, 4q + 256i + e] (i < 8, e < 4) in registers.  Each step the member
// forms its rows of G s with one wave reduction per row, updates and
// publishes its coefficients, then gathers the whole new s into LDS.  Words
// alternate between two buffers by step parity: a member overwrites a buffer
// only after gathering every word of the other one, which every member
// publishes only after its own gather of this one is complete.
__device__ void adam_team_body(const Inst& I, int j, int t, int T, float lr, float beta1,
                               float beta2, int w, float* lds) {
  const int t1 = t + 1;
  const int t4 = (t1 + 3) & ~3;
  const int tid = threadIdx.x;
  const int lane = tid & 63, rho = tid >> 6;
  const int r = w * kTeamRows + rho;
  const bool row_ok = r < t1;
  float* s_lds = lds;                                // [t4]
  float Gr[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int c = 4 * lane + 256 * i;
    if (r < t && c + 3 < t) {   // entries of earlier iterations (not row t)
      const float4 q = *reinterpret_cast<const float4*>(I.G + c + (long long)r * I.ldg);
      Gr[i][0] = q.x; Gr[i][1] = q.y; Gr[i][2] = q.z; Gr[i][3] = q.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) Gr[i][e] = (row_ok && c + e < t1) ? gram_at(I, j, t, r, c + e) : 0.f;
    }
  }
  float sv = 0.f, mo = 0.f, ve = 0.f, bb = 0.f;
  if (row_ok) {
    sv = I.s[r];
    mo = I.mo[r];
    ve = I.ve[r];
    bb = (r == t) ? I.c0[j] : I.b[r];
  }
  for (int c = tid; c < t4; c += kPassThreads) s_lds[c] = (c < t1) ? I.s[c] : 0.f;
  const float eps = I.st->eps;
  const int step0 = I.st->step;
  double b1p = pow((double)beta1, (double)step0);
  double b2p = pow((double)beta2, (double)step0);
  __syncthreads();
  for (int it = 0; it < T; ++it) {
    b1p *= beta1;
    b2p *= beta2;
    const float ibc1 = __builtin_amdgcn_rcpf((float)(1.0 - b1p));
    const float ibc2 = __builtin_amdgcn_rcpf((float)(1.0 - b2p));
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int c = 4 * lane + 256 * i;
      if (c < t4) {
        const float4 sq = *reinterpret_cast<const float4*>(s_lds + c);
        a0 = fmaf(Gr[i][0], sq.x, a0);
        a1 = fmaf(Gr[i][1], sq.y, a1);
        a2 = fmaf(Gr[i][2], sq.z, a2);
        a3 = fmaf(Gr[i][3], sq.w, a3);
      }
    }
    const float gs = wave_sum((a0 + a1) + (a2 + a3));
    const unsigned tag = (unsigned)(step0 + it + 1);
    unsigned long long* buf = I.team + (size_t)(tag & 1) * I.k_eff;
    if (row_ok && lane == 0) {
      const float gr = gs - bb;
      mo = beta1 * mo + (1.f - beta1) * gr;
      ve = beta2 * ve + (1.f - beta2) * (gr * gr);
      sv = sv - lr * (mo * ibc1) * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(ve * ibc2) + eps);
      if (it + 1 < T) team_put(buf + r, tag, sv);
    }
    if (it + 1 < T) {
      __syncthreads();                               // every wave is done with s_lds
      for (int c = tid; c < t1; c += kPassThreads) s_lds[c] = team_get(I, buf + c, tag);
      __syncthreads();
    }
  }
  if (row_ok && lane == 0) {
    I.s[r] = sv;
    I.mo[r] = mo;
    I.ve[r] = ve;
  }
  if (w == 0 && tid == 0) I.st->step = step0 + T;
}

// OMP bordered-inverse update split by rows of Ginv (a member updates its own
// columns, which by symmetry are its rows and contiguous): v = Ginv g and the
// member's partial products g.v, g.x are published with tag t+1; every member
// then forms delta and alpha from the partials in the same order and updates
// its columns, its entries of the new border and its coefficients.
__device__ void omp_team_body(const Inst& I, int j, int t, int W, int w, float* lds) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const long long ld = I.ldg;
  const unsigned tag = (unsigned)(t + 1);
  float* Gi = I.Linv;
  float* g = lds;                                    // [t+1]
  float* red = lds + t + 1;                          // [32]
  for (int c = tid; c <= t; c += kPassThreads) g[c] = (c < t) ? hcol(I, c)[j] : I.dg[j];
  __syncthreads();
  unsigned long long* vbuf = I.team;                 // [k_eff]
  unsigned long long* pbuf = I.team + 2 * (size_t)I.k_eff;   // [2][kTeamMax]
  const int r = w * kTeamRows + wv;                  // one wave per row
  float vr = 0.f, pv = 0.f, px = 0.f;
  if (r < t) {
    const float* col = Gi + (long long)r * ld;
    float a = 0.f;
    for (int c = lane; c < t; c += 64) a = fmaf(col[c], g[c], a);
    vr = wave_sum(a);
    if (lane == 0) {
      team_put(vbuf + r, tag, vr);
      pv = g[r] * vr;
      px = g[r] * I.s[r];
    }
  }
  if (lane == 0) {
    red[wv] = pv;
    red[16 + wv] = px;
  }
  __syncthreads();
  if (tid == 0) {
    float a = 0.f, b = 0.f;
    for (int q = 0; q < kTeamRows; ++q) {
      a += red[q];
      b += red[16 + q];
    }
    team_put(pbuf + w, tag, a);
    team_put(pbuf + kTeamMax + w, tag, b);
  }
  float gv = 0.f, gx = 0.f;
  if (tid < 64) {   // one wave gathers the partials in member order
    for (int q = 0; q < W; ++q) {
      gv += team_get(I, pbuf + q, tag);
      gx += team_get(I, pbuf + kTeamMax + q, tag);
    }
    if (tid == 0) {
      red[0] = gv;
      red[1] = gx;
    }
  }
  __syncthreads();
  gv = red[0];
  gx = red[1];
  const float gamma = g[t];
  float delta = gamma - gv;
  const bool bad = !(delta > 1e-7f * gamma);
  if (bad) delta = fmaxf(1e-7f * gamma, 1e-30f);
  const float inv = 1.f / delta;
  const float alpha = (I.c0[j] - gx) * inv;
  float* v = g;                                      // g is no longer needed
  __syncthreads();
  for (int c = tid; c < t; c += kPassThreads) v[c] = team_get(I, vbuf + c, tag);
  __syncthreads();
  if (r < t) {
    float* col = Gi + (long long)r * ld;
    const float vri = vr * inv;
    for (int c = lane; c < t; c += 64) col[c] = fmaf(v[c], vri, col[c]);
    if (lane == 0) {
      col[t] = -vri;                                 // Ginv[t, r]
      Gi[r + (long long)t * ld] = -vri;              // Ginv[r, t]
      I.s[r] = fmaf(-alpha, vr, I.s[r]);
    }
  }
  if (w == 0 && tid == 0) {
    I.s[t] = alpha;
    Gi[t + (long long)t * ld] = inv;
    if (bad) atomicOr(I.status, ST_REFINE_INACCURATE);
  }
}

enum CoefKind : int {
  COEF_ADAM_REG = 0, COEF_ADAM_GLOBAL = 1, COEF_OMP = 2, COEF_ADAM_TEAM = 3, COEF_OMP_TEAM = 4
};

// Blocks [0, nact): coefficient update of iteration t for the class's active
// instances (insts_c = class base).  Blocks [nact, ...): h_t pass tiles.
template <typename TA, int LPA, int COEF>
__global__ __launch_bounds__(kPassThreads) void coef_pass_kernel(
    const Inst* __restrict__ insts_c, int nact, int W, const Inst* __restrict__ insts,
    const ScanTile* __restrict__ tiles, int t, int T, float beta1, float beta2, float lr_rel,
    float eps_rel) {
  extern __shared__ __align__(16) float dsh[];
  __shared__ __align__(16) float part[adam_part_floats<4>()];
  __shared__ float red[kPassThreads / 64], red2[kPassThreads / 64];
  __shared__ unsigned long long wbest[kPassThreads / 64];
  if ((int)blockIdx.x < nact * W) {
    const Inst& I = insts_c[blockIdx.x / W];
    const int member = blockIdx.x % W;
    // done is set only by earlier launches or, below, together with a bad
    // key that every member sees: all members leave together
    if (I.st->done) return;
    // selection record and the new Gram column, gathered from H:
    //   G[l, t] = a_{S_l}^T a_j = H[j, l] (l < t),  G[t, t] = ||a_j||^2,
    //   b_t = a_j^T y = c0[j]
    const unsigned long long key = I.key[t & 1];
    const int j = key_index(key);
    if (key == 0ull || j < 0 || j >= I.n) {
      if (member == 0 && threadIdx.x == 0) {
        I.st->done = 1;
        atomicOr(I.status, ST_WATCHDOG);
      }
      return;
    }
    constexpr bool team = COEF == COEF_ADAM_TEAM || COEF == COEF_OMP_TEAM;
    if (member == 0) record_selection<kPassThreads>(I, key, t, lr_rel, eps_rel);
    if (team) {
      // members take the new Gram row / column and b_t from H, dg and c0
      if (COEF == COEF_OMP_TEAM)
        omp_team_body(I, j, t, W, member, dsh);
      else
        adam_team_body(I, j, t, T, lr_rel * key_value(key), beta1, beta2, member, dsh);
      team_retire(I, member);
      return;
    }
    __syncthreads();
    if (COEF == COEF_ADAM_REG)
      adam_reg_body(I, t, T, beta1, beta2, part, kPassThreads / 64, false);
    else if (COEF == COEF_ADAM_GLOBAL && t + 1 <= kPassThreads)
      adam_split_body(I, t, T, beta1, beta2, dsh);
    else if (COEF == COEF_ADAM_GLOBAL)
      adam_global_body<kPassThreads>(I, t, T, beta1, beta2, dsh, false);
    else
      omp_ginv_body(I, t, dsh, red, red2, false);
    return;
  }
  // odd iterations walk the tiles backwards: a pass starts on the columns
  // the previous pass streamed last, which the memory-side cache may still
  // hold when the dictionary is about the cache's size
  const int ntl = (int)gridDim.x - nact * W;
  const int ti = (int)blockIdx.x - nact * W;
  const ScanTile tile = tiles[(t & 1) ? ntl - 1 - ti : ti];
  pass_tile_body<TA, LPA, 1>(insts[tile.inst], tile, t, dsh, wbest);
}

// c_j = c0_j - sum_{l<t} H[j, l] s_l over tiles of 256 atoms (tiles start at
// multiples of 256 within a signal): lane v covers atoms 4v..4v+3 with one
// float4 load per column of H (a wave reads 1 KB of a column per load, eight
// loads in flight), G waves split the columns of a tile (column l goes to
// wave l mod G) and their partial sums are added in LDS in wave order; with
// G = 1 each wave of the workgroup takes a tile of its own and no workgroup
// barrier is needed.  Then |c| with the exclusion of selected atoms and the
// argmax key (slot t & 1), one atomicMax per tile.  G is chosen per launch
// from the number of tiles, so that both a batch of thousands of signals
// and a single signal keep the device busy.
constexpr int kHscanAtoms = 256;

template <int G>
__global__ __launch_bounds__(G == 16 ? 1024 : 256) void cscan_kernel(
    const Inst* __restrict__ insts, const ScanTile* __restrict__ tiles, int ntiles, int t) {
  __shared__ float4 part[G > 1 ? G : 1][64];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int ti = (G == 1) ? (int)blockIdx.x * 4 + w : (int)blockIdx.x;
  if (ti >= ntiles) return;                  // G == 1 only: a whole wave leaves
  const ScanTile tile = tiles[ti];
  const Inst& I = insts[tile.inst];
  if (I.st->done) return;                    // G > 1: the whole workgroup leaves
  const int j = tile.j0 + 4 * lane;
  const bool ok = j < tile.j1;
  float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
  if (ok) {
    const float* ssh = I.s;                  // t coefficients, uniform per wave
    auto fma4 = [](float4 h, float c, float4 x) {
      return make_float4(fmaf(h.x, c, x.x), fmaf(h.y, c, x.y), fmaf(h.z, c, x.z),
                         fmaf(h.w, c, x.w));
    };
    int l = (G == 1) ? 0 : w;
    for (; l + 7 * G < t; l += 8 * G) {
      float4 h[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) h[u] = gload4(hcol(I, l + u * G) + j);
#pragma unroll
      for (int u = 0; u < 8; ++u) a = fma4(h[u], ssh[l + u * G], a);
    }
    for (; l < t; l += G) a = fma4(gload4(hcol(I, l) + j), ssh[l], a);
  }
  if (G > 1) {
    part[w][lane] = a;
    __syncthreads();
    if (w != 0) return;                      // no barrier follows
    a = part[0][lane];
#pragma unroll
    for (int q = 1; q < G; ++q) {
      const float4 u = part[q][lane];
      a = make_float4(a.x + u.x, a.y + u.y, a.z + u.z, a.w + u.w);
    }
  }
  unsigned long long key = 0ull;
  if (ok) {
    // c0 and ldh are padded to a multiple of 256 entries: the float4 read of
    // the last atoms stays inside the buffer; 4 atoms share a bitmap word
    const float4 c0v = gload4(I.c0 + j);
    const unsigned bits = I.bitmap[j >> 5];
    const float cs[4] = {c0v.x - a.x, c0v.y - a.y, c0v.z - a.z, c0v.w - a.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int je = j + e;
      if (je < tile.j1 && !((bits >> (je & 31)) & 1u)) {
        const unsigned long long k2 = pack_key(cs[e], je);
        key = k2 > key ? k2 : key;
      }
    }
  }
  key = wave_max_u64(key);
  if (lane == 0 && key) atomicMax(&I.key[t & 1], key);
}

// Coefficient update of iteration t when no pass shares the launch (shared
// dictionary, CLOMP, t+1 <= 256): one workgroup of ceil((t+1)/16) waves per
// signal, so small supports do not hold a 16-wave workgroup each and several
// signals share a CU; RPL rows of G per lane for supports up to 64*RPL.  The
// selection record, then the register-tile Adam.
template <int RPL>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(RPL == 2 ? 6 : 1)))
void coef_reg_kernel(const Inst* __restrict__ insts_c, int t,
                                                        int T, float beta1, float beta2,
                                                        float lr_rel, float eps_rel) {
  __shared__ __align__(16) float part[adam_part_floats<RPL>()];
  const Inst& I = insts_c[blockIdx.x];
  if (I.st->done) return;
  const unsigned long long key = I.key[t & 1];
  const int j = key_index(key);
  if (key == 0ull || j < 0 || j >= I.n) {
    if (threadIdx.x == 0) {
      I.st->done = 1;
      atomicOr(I.status, ST_WATCHDOG);
    }
    return;
  }
  record_selection<0>(I, key, t, lr_rel, eps_rel);
  __syncthreads();
  adam_reg_body<RPL>(I, t, T, beta1, beta2, part, blockDim.x >> 6, false);
}

// OMP counterpart of coef_reg_kernel: the selection record and the
// bordered-inverse update of iteration t in one 256-thread workgroup per
// signal (no pass in the launch).
__global__ __launch_bounds__(256) void coef_omp_kernel(const Inst* __restrict__ insts_c, int t,
                                                       float lr_rel, float eps_rel) {
  extern __shared__ __align__(16) float osh[];   // g[t+1] | v[t+1] | vpart[t+1]
  __shared__ float red[4], red2[4];
  const Inst& I = insts_c[blockIdx.x];
  if (I.st->done) return;
  const unsigned long long key = I.key[t & 1];
  const int j = key_index(key);
  if (key == 0ull || j < 0 || j >= I.n) {
    if (threadIdx.x == 0) {
      I.st->done = 1;
      atomicOr(I.status, ST_WATCHDOG);
    }
    return;
  }
  record_selection<256>(I, key, t, lr_rel, eps_rel);
  __syncthreads();
  omp_ginv_body<256>(I, t, osh, red, red2, false);
}

// ============================================================ image priors
// CLOMP on the columns of one image (CLOMP_FLAG_IMAGE): column c of the image
// is x_c = D s_c (D the orthonormal DCT-II synthesis basis, n x n); the loss
// adds w_tv TV(X) (Eq. (6): the within-column term of the 1-D prior, which
// sits on the Gram diagonal, plus (w_tv / W) sum_c ||s_c - s_c+1||^2, the
// between-column term written in the coefficients since D is orthonormal) and
// w_lv LV(X) (Eq. (7): mean over every 3 x 3 window, step 1, of the sample
// standard deviation).  The supports are sparse, so x_c = D_S s_S and the
// local-variation gradient D_S^T g_x cost n |S| per column: no full transform.
// Every Adam step is one launch over all columns (two with the local
// variation: the pixel image first), so that each column reads its
// neighbours' values of the same step; the dense coefficient images alternate
// by step parity.

// D[i + k ldd] = c_k cos(pi k (2i + 1) / (2n)), c_0 = sqrt(1/n), c_k = sqrt(2/n)
// (the phase reduced modulo 4n in integers, cospi of an exact quotient); the
// dense coefficient images and the pixel image start at zero.
__global__ __launch_bounds__(kBlock) void image_init_kernel(float* __restrict__ D, int n,
                                                            long long ldd,
                                                            float* __restrict__ zero,
                                                            long long nzero) {
  const long long stride = (long long)gridDim.x * kBlock;
  const long long nd = (long long)n * n;
  for (long long q = (long long)blockIdx.x * kBlock + threadIdx.x; q < nd + nzero; q += stride) {
    if (q < nd) {
      const int k = (int)(q / n), i = (int)(q % n);
      const long long p = ((long long)k * (2 * i + 1)) % (4LL * n);
      const float ck = sqrtf((k == 0 ? 1.f : 2.f) / (float)n);
      D[i + (long long)k * ldd] = ck * cospif((float)p / (float)(2 * n));
    } else {
      zero[q - nd] = 0.f;
    }
  }
}

// Selection record of iteration t of every live column (no coefficient update).
__global__ __launch_bounds__(kBlock) void image_record_kernel(const Inst* __restrict__ insts,
                                                              int t, float lr_rel,
                                                              float eps_rel) {
  const Inst& I = insts[blockIdx.x];
  if (I.st->done) return;
  const unsigned long long key = I.key[t & 1];
  const int j = key_index(key);
  if (key == 0ull || j < 0 || j >= I.n) {
    if (threadIdx.x == 0) {
      I.st->done = 1;
      atomicOr(I.status, ST_WATCHDOG);
    }
    return;
  }
  record_selection<kBlock>(I, key, t, lr_rel, eps_rel);
}

// Pixel column x_c = sum_l D[:, S_l] s_l of every live column (t1 atoms).
__global__ __launch_bounds__(kBlock) void image_synth_kernel(const Inst* __restrict__ insts,
                                                             int t1, const float* __restrict__ D,
                                                             long long ldd,
                                                             float* __restrict__ X) {
  __shared__ float ssh[kImageMaxK];
  __shared__ int jsh[kImageMaxK];
  const Inst& I = insts[blockIdx.x];
  if (I.st->done) return;
  for (int l = threadIdx.x; l < t1; l += kBlock) {
    ssh[l] = I.s[l];
    jsh[l] = I.support[l];
  }
  __syncthreads();
  float* xc = X + (long long)I.col * ldd;
  for (int i = threadIdx.x; i < I.n; i += kBlock) {
    float acc = 0.f;
    for (int l = 0; l < t1; ++l) acc = fmaf(D[i + (long long)jsh[l] * ldd], ssh[l], acc);
    xc[i] = acc;
  }
}

// One Adam step (number `step`, 1-based) of every live column on
//   1/2 ||y_c - A s_c||^2 + w_tv TV(X) + w_lv LV(X)
// restricted to the column's support of t1 = t + 1 atoms: the data term and
// the within-column TV from the Gram matrix (G s - b, prior on the diagonal),
// htv = 2 w_tv / W times the differences to the neighbours' coefficients
// (Sd_cur, dense, ld ldd), and w_lv times D_S^T of the column's pixel gradient
// of LV, formed from the pixel columns c-2 .. c+2 of X staged in LDS.  The
// updated coefficients go to I.s (support order) and to Sd_next.
__global__ __launch_bounds__(kBlock) void image_step_kernel(
    const Inst* __restrict__ insts, int W, int t, int step, float beta1, float beta2, float htv,
    float wlv, const float* __restrict__ D, long long ldd, const float* __restrict__ X,
    const float* __restrict__ Sd_cur, float* __restrict__ Sd_next) {
  extern __shared__ __align__(16) float xsh[];    // with LV: 5 pixel columns | pixel gradient
  __shared__ float ssh[kImageMaxK];
  __shared__ int jsh[kImageMaxK];
  __shared__ float gsh[kImageMaxK];
  const Inst& I = insts[blockIdx.x];
  if (I.st->done) return;
  const int t1 = t + 1, n = I.n, c = I.col;
  const int tid = threadIdx.x;
  for (int l = tid; l < t1; l += kBlock) {
    ssh[l] = I.s[l];
    jsh[l] = I.support[l];
    gsh[l] = 0.f;
  }
  if (wlv != 0.f && n >= 3 && W >= 3) {
    // pixel columns c-2 .. c+2 (those inside the image)
    for (int q = 0; q < 5; ++q) {
      const int cc = c - 2 + q;
      for (int i = tid; i < n; i += kBlock)
        xsh[q * n + i] = (cc >= 0 && cc < W) ? X[i + (long long)cc * ldd] : 0.f;
    }
    __syncthreads();
    // d LV / d x[i, c]: every window (centre rows 1 .. n-2, centre columns
    // 1 .. W-2) that holds the pixel adds (x - mean) / (8 std) (nothing when
    // std = 0), divided by the number of windows
    float* gx = xsh + 5 * n;
    const float invB = 1.f / ((float)(n - 2) * (float)(W - 2));
    for (int i = tid; i < n; i += kBlock) {
      float g = 0.f;
      const float xi = xsh[2 * n + i];
      for (int di = -1; di <= 1; ++di) {
        const int ip = i + di;
        if (ip < 1 || ip > n - 2) continue;
        for (int dc = -1; dc <= 1; ++dc) {
          const int cp = c + dc;
          if (cp < 1 || cp > W - 2) continue;
          const int q0 = dc + 1;                 // staged columns q0 .. q0+2
          float sum = 0.f;
#pragma unroll
          for (int u = 0; u < 3; ++u)
#pragma unroll
            for (int v = -1; v <= 1; ++v) sum += xsh[(q0 + u) * n + ip + v];
          const float mean = sum * (1.f / 9.f);
          float ss = 0.f;
#pragma unroll
          for (int u = 0; u < 3; ++u)
#pragma unroll
            for (int v = -1; v <= 1; ++v) {
              const float dlt = xsh[(q0 + u) * n + ip + v] - mean;
              ss = fmaf(dlt, dlt, ss);
            }
          const float sd = sqrtf(ss * 0.125f);
          if (sd > 0.f) g += (xi - mean) / (8.f * sd);
        }
      }
      gx[i] = g * invB;
    }
    __syncthreads();
    // D_S^T g_x: one wave per support row, lanes over the pixels
    const int lane = tid & 63, wv = tid >> 6;
    for (int l = wv; l < t1; l += kBlock / 64) {
      const float* dcol = D + (long long)jsh[l] * ldd;
      float a = 0.f;
      for (int i = lane; i < n; i += 64) a = fmaf(dcol[i], gx[i], a);
      a = wave_sum(a);
      if (lane == 0) gsh[l] = a;
    }
  }
  __syncthreads();
  const float lr = I.st->lr, eps = I.st->eps;
  const float ibc1 = __builtin_amdgcn_rcpf((float)(1.0 - pow((double)beta1, (double)step)));
  const float ibc2 = __builtin_amdgcn_rcpf((float)(1.0 - pow((double)beta2, (double)step)));
  const long long ldg = I.ldg;
  for (int l = tid; l < t1; l += kBlock) {
    // G is symmetric: row l of every column, consecutive threads consecutive rows
    float acc = 0.f;
    for (int l2 = 0; l2 < t1; ++l2) acc = fmaf(I.G[l + (long long)l2 * ldg], ssh[l2], acc);
    float gr = acc - I.b[l];
    const int j = jsh[l];
    const float sl = ssh[l];
    if (htv != 0.f) {
      float hd = 0.f;
      if (c > 0) hd += sl - Sd_cur[j + (long long)(c - 1) * ldd];
      if (c < W - 1) hd += sl - Sd_cur[j + (long long)(c + 1) * ldd];
      gr = fmaf(htv, hd, gr);
    }
    if (wlv != 0.f) gr = fmaf(wlv, gsh[l], gr);
    float mo = I.mo[l], ve = I.ve[l];
    mo = beta1 * mo + (1.f - beta1) * gr;
    ve = beta2 * ve + (1.f - beta2) * (gr * gr);
    const float mh = mo * ibc1;
    const float vh = ve * ibc2;
    const float sv = sl - lr * mh * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(vh) + eps);
    I.s[l] = sv;
    I.mo[l] = mo;
    I.ve[l] = ve;
    Sd_next[j + (long long)c * ldd] = sv;
  }
  if (tid == 0) I.st->step = step;
}

// ============================================================ launchers
// A launcher with nothing to launch still records pending profiling events,
// so every recorded interval is valid (and empty).
static hipError_t nothing_to_launch(hipStream_t s) {
  if (g_ev_start) {
    hipError_t e = hipEventRecord(g_ev_start, s);
    if (e == hipSuccess) e = hipEventRecord(g_ev_stop, s);
    return e;
  }
  return hipSuccess;
}

template <typename TA>
static hipError_t scan_dispatch(int lpa, const Inst* d, const ScanTile* tiles, int ntiles,
                                int r_lds_floats, int reverse, hipStream_t s) {
  const size_t lds = (size_t)r_lds_floats * sizeof(float);
  const int flag = r_lds_floats > 0;
  switch (lpa) {
    case 4: CLOMP_LAUNCH((scan_kernel<TA, 4>), dim3(ntiles), dim3(kBlock), lds, s, d, tiles, flag, reverse); break;
    case 8: CLOMP_LAUNCH((scan_kernel<TA, 8>), dim3(ntiles), dim3(kBlock), lds, s, d, tiles, flag, reverse); break;
    case 16: CLOMP_LAUNCH((scan_kernel<TA, 16>), dim3(ntiles), dim3(kBlock), lds, s, d, tiles, flag, reverse); break;
    case 32: CLOMP_LAUNCH((scan_kernel<TA, 32>), dim3(ntiles), dim3(kBlock), lds, s, d, tiles, flag, reverse); break;
    default: CLOMP_LAUNCH((scan_kernel<TA, 64>), dim3(ntiles), dim3(kBlock), lds, s, d, tiles, flag, reverse); break;
  }
  return hipGetLastError();
}

hipError_t launch_init(const Inst* d, int count, hipStream_t s) {
  CLOMP_LAUNCH(init_kernel, dim3(count), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

template <typename TA, int LPA>
static hipError_t scan_reg_dispatch(int nch, const Inst* d, const ScanTile* tiles, int ntiles,
                                    int reverse, hipStream_t s) {
  const dim3 g(ntiles), b(kBlock);
  switch (nch) {
    case 1: CLOMP_LAUNCH((scan_reg_kernel<TA, LPA, 1>), g, b, 0, s, d, tiles, reverse); break;
    case 2: CLOMP_LAUNCH((scan_reg_kernel<TA, LPA, 2>), g, b, 0, s, d, tiles, reverse); break;
    case 4: CLOMP_LAUNCH((scan_reg_kernel<TA, LPA, 4>), g, b, 0, s, d, tiles, reverse); break;
    case 8: CLOMP_LAUNCH((scan_reg_kernel<TA, LPA, 8>), g, b, 0, s, d, tiles, reverse); break;
    default: CLOMP_LAUNCH((scan_reg_kernel<TA, LPA, 16>), g, b, 0, s, d, tiles, reverse); break;
  }
  return hipGetLastError();
}

template <typename TA>
static hipError_t scan_reg_lpa(int lpa, int nch, const Inst* d, const ScanTile* tiles, int ntiles,
                               int reverse, hipStream_t s) {
  switch (lpa) {
    case 4: return scan_reg_dispatch<TA, 4>(nch, d, tiles, ntiles, reverse, s);
    case 8: return scan_reg_dispatch<TA, 8>(nch, d, tiles, ntiles, reverse, s);
    case 16: return scan_reg_dispatch<TA, 16>(nch, d, tiles, ntiles, reverse, s);
    case 32: return scan_reg_dispatch<TA, 32>(nch, d, tiles, ntiles, reverse, s);
    default: return scan_reg_dispatch<TA, 64>(nch, d, tiles, ntiles, reverse, s);
  }
}

template <typename TA, int LPA>
static hipError_t gram_reg_dispatch(int nch, const Inst* d, int nact, int t, int nblk, int D,
                                    float lr_rel, float eps_rel, hipStream_t s) {
  const dim3 g(nact * nblk), b(kBlock);
  switch (nch) {
    case 1: CLOMP_LAUNCH((gram_reg_kernel<TA, LPA, 1>), g, b, 0, s, d, t, nblk, D, lr_rel, eps_rel); break;
    case 2: CLOMP_LAUNCH((gram_reg_kernel<TA, LPA, 2>), g, b, 0, s, d, t, nblk, D, lr_rel, eps_rel); break;
    case 4: CLOMP_LAUNCH((gram_reg_kernel<TA, LPA, 4>), g, b, 0, s, d, t, nblk, D, lr_rel, eps_rel); break;
    case 8: CLOMP_LAUNCH((gram_reg_kernel<TA, LPA, 8>), g, b, 0, s, d, t, nblk, D, lr_rel, eps_rel); break;
    default: CLOMP_LAUNCH((gram_reg_kernel<TA, LPA, 16>), g, b, 0, s, d, t, nblk, D, lr_rel, eps_rel); break;
  }
  return hipGetLastError();
}

template <typename TA>
static hipError_t gram_reg_lpa(int lpa, int nch, const Inst* d, int nact, int t, int nblk, int D,
                               float lr_rel, float eps_rel, hipStream_t s) {
  switch (lpa) {
    case 4: return gram_reg_dispatch<TA, 4>(nch, d, nact, t, nblk, D, lr_rel, eps_rel, s);
    case 8: return gram_reg_dispatch<TA, 8>(nch, d, nact, t, nblk, D, lr_rel, eps_rel, s);
    case 16: return gram_reg_dispatch<TA, 16>(nch, d, nact, t, nblk, D, lr_rel, eps_rel, s);
    case 32: return gram_reg_dispatch<TA, 32>(nch, d, nact, t, nblk, D, lr_rel, eps_rel, s);
    default: return gram_reg_dispatch<TA, 64>(nch, d, nact, t, nblk, D, lr_rel, eps_rel, s);
  }
}

hipError_t launch_scan_reg(int bf16, int lpa, int nch, const Inst* d, const ScanTile* tiles,
                           int ntiles, int reverse, hipStream_t s) {
  if (ntiles <= 0) return nothing_to_launch(s);
  return bf16 ? scan_reg_lpa<uint16_t>(lpa, nch, d, tiles, ntiles, reverse, s)
              : scan_reg_lpa<float>(lpa, nch, d, tiles, ntiles, reverse, s);
}

hipError_t launch_gram_reg(int bf16, int lpa, int nch, const Inst* d, int nact, int t, int nblk,
                           int D, float lr_rel, float eps_rel, hipStream_t s) {
  if (nact <= 0) return nothing_to_launch(s);
  return bf16 ? gram_reg_lpa<uint16_t>(lpa, nch, d, nact, t, nblk, D, lr_rel, eps_rel, s)
              : gram_reg_lpa<float>(lpa, nch, d, nact, t, nblk, D, lr_rel, eps_rel, s);
}

hipError_t launch_scan(int bf16, int lpa, const Inst* d, const ScanTile* tiles, int ntiles,
                       int r_lds_floats, int reverse, hipStream_t s) {
  if (ntiles <= 0) return nothing_to_launch(s);
  return bf16 ? scan_dispatch<uint16_t>(lpa, d, tiles, ntiles, r_lds_floats, reverse, s)
              : scan_dispatch<float>(lpa, d, tiles, ntiles, r_lds_floats, reverse, s);
}

template <typename TA>
static hipError_t gram_dispatch(int lpa, const Inst* d, int nact, int t, int nblk, int D,
                                int v_lds_floats, float lr_rel, float eps_rel, hipStream_t s) {
  const size_t lds = (size_t)v_lds_floats * sizeof(float);
  const int flag = v_lds_floats > 0;
  const dim3 g(nact * nblk), b(kBlock);
  switch (lpa) {
    case 4: CLOMP_LAUNCH((gram_kernel<TA, 4>), g, b, lds, s, d, t, nblk, D, flag, lr_rel, eps_rel); break;
    case 8: CLOMP_LAUNCH((gram_kernel<TA, 8>), g, b, lds, s, d, t, nblk, D, flag, lr_rel, eps_rel); break;
    case 16: CLOMP_LAUNCH((gram_kernel<TA, 16>), g, b, lds, s, d, t, nblk, D, flag, lr_rel, eps_rel); break;
    case 32: CLOMP_LAUNCH((gram_kernel<TA, 32>), g, b, lds, s, d, t, nblk, D, flag, lr_rel, eps_rel); break;
    default: CLOMP_LAUNCH((gram_kernel<TA, 64>), g, b, lds, s, d, t, nblk, D, flag, lr_rel, eps_rel); break;
  }
  return hipGetLastError();
}

hipError_t launch_gram(int bf16, int lpa, const Inst* d, int nact, int t, int nblk, int D,
                       int v_lds_floats, float lr_rel, float eps_rel, hipStream_t s) {
  if (nact <= 0) return nothing_to_launch(s);
  return bf16 ? gram_dispatch<uint16_t>(lpa, d, nact, t, nblk, D, v_lds_floats, lr_rel, eps_rel, s)
              : gram_dispatch<float>(lpa, d, nact, t, nblk, D, v_lds_floats, lr_rel, eps_rel, s);
}

hipError_t launch_adam(const Inst* d, int nact, int t, int T, float beta1, float beta2,
                       hipStream_t s) {
  if (nact <= 0) return nothing_to_launch(s);
  if (t + 1 <= kRegRows)
    CLOMP_LAUNCH(adam_reg_kernel, dim3(nact), dim3(64 * ((t + 16) / 16)), 0, s, d, t, T,
                       beta1, beta2);
  else
    CLOMP_LAUNCH(adam_kernel, dim3(nact), dim3(kBlock), (size_t)(t + 1) * sizeof(float), s,
                       d, t, T, beta1, beta2);
  return hipGetLastError();
}

hipError_t launch_omp(const Inst* d, int nact, int t, hipStream_t s) {
  if (nact <= 0) return nothing_to_launch(s);
  CLOMP_LAUNCH(omp_ginv_kernel, dim3(nact), dim3(kOmpThreads),
                     (size_t)6 * (t + 1) * sizeof(float), s, d, t);
  return hipGetLastError();
}

hipError_t launch_resid(int bf16, const Inst* d, const RowTile* tiles, int ntiles, int t,
                        hipStream_t s) {
  if (ntiles <= 0) return nothing_to_launch(s);
  const size_t lds = ((size_t)2 * (t + 1) + 4 * 64) * sizeof(float);
  if (bf16)
    CLOMP_LAUNCH((rows_kernel<uint16_t, ROW_RESID>), dim3(ntiles), dim3(kBlock), lds, s, d,
                       tiles, t, 0, 0.f);
  else
    CLOMP_LAUNCH((rows_kernel<float, ROW_RESID>), dim3(ntiles), dim3(kBlock), lds, s, d,
                       tiles, t, 0, 0.f);
  return hipGetLastError();
}

hipError_t launch_cg_rows(int mode, const Inst* d, const RowTile* tiles, int ntiles, int tmax,
                          int it, float tol2, hipStream_t s) {
  if (ntiles <= 0) return nothing_to_launch(s);
  const size_t lds = ((size_t)2 * (tmax + 1) + 4 * 64) * sizeof(float);
  if (mode == 0)
    CLOMP_LAUNCH((rows_kernel<float, ROW_CG_R0>), dim3(ntiles), dim3(kBlock), lds, s, d,
                       tiles, tmax, it, tol2);
  else
    CLOMP_LAUNCH((rows_kernel<float, ROW_CG_Q>), dim3(ntiles), dim3(kBlock), lds, s, d,
                       tiles, tmax, it, tol2);
  return hipGetLastError();
}

hipError_t launch_cg_dots(int mode, int lpa, const Inst* d, const int* list, int nlist, int tmax,
                          int nblk, int D, int m_pad_max, int it, hipStream_t s) {
  if (nlist <= 0) return nothing_to_launch(s);
  const size_t lds = (size_t)m_pad_max * sizeof(float);
  const dim3 g(nlist * nblk), b(kBlock);
#define CG_DOTS_CASE(L)                                                                     \
  case L:                                                                                   \
    if (mode == 0)                                                                          \
      CLOMP_LAUNCH((cg_dots_kernel<L, 0>), g, b, lds, s, d, list, tmax, nblk, D, it); \
    else                                                                                    \
      CLOMP_LAUNCH((cg_dots_kernel<L, 1>), g, b, lds, s, d, list, tmax, nblk, D, it); \
    break;
  switch (lpa) {
    CG_DOTS_CASE(4)
    CG_DOTS_CASE(8)
    CG_DOTS_CASE(16)
    CG_DOTS_CASE(32)
    default:
      CG_DOTS_CASE(64)
  }
#undef CG_DOTS_CASE
  return hipGetLastError();
}

hipError_t launch_copy_s(const Inst* d, const int* list, int nlist, hipStream_t s) {
  if (nlist <= 0) return nothing_to_launch(s);
  CLOMP_LAUNCH(copy_s_kernel, dim3(nlist), dim3(kBlock), 0, s, d, list);
  return hipGetLastError();
}

hipError_t launch_qr(const Inst* d, const int* list, int nlist, size_t lds_bytes, hipStream_t s) {
  if (nlist <= 0) return nothing_to_launch(s);
  CLOMP_LAUNCH(qr_refine_kernel, dim3(nlist), dim3(kBlock), lds_bytes, s, d, list);
  return hipGetLastError();
}

hipError_t launch_norm(const Inst* d, const RowTile* tiles, int ntiles, int tmax, hipStream_t s) {
  if (ntiles <= 0) return nothing_to_launch(s);
  const size_t lds = (size_t)2 * (tmax + 1) * sizeof(float);
  CLOMP_LAUNCH(norm_rows_kernel, dim3(ntiles), dim3(kBlock), lds, s, d, tiles);
  return hipGetLastError();
}

hipError_t launch_finalize(const Inst* d, int count, int check_cg, hipStream_t s) {
  if (count <= 0) return nothing_to_launch(s);
  CLOMP_LAUNCH(finalize_kernel, dim3(count), dim3(kBlock), 0, s, d, check_cg);
  return hipGetLastError();
}

// Allow each kernel `bytes` of LDS in total: its dynamic ceiling is `bytes`
// minus the kernel's own static LDS.
static hipError_t raise_dynamic_lds(const void* const* fns, size_t nf, size_t bytes) {
  for (size_t i = 0; i < nf; ++i) {
    hipFuncAttributes at;
    hipError_t e = hipFuncGetAttributes(&at, fns[i]);
    if (e != hipSuccess) return e;
    const size_t dyn = bytes > at.sharedSizeBytes ? bytes - at.sharedSizeBytes : 0;
    e = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename TA, int KR>
static void small_clomp(dim3 g, dim3 b, size_t lds, hipStream_t s, const Inst* d,
                        const int* list, int T, float beta1, float beta2, float lr_rel,
                        float eps_rel) {
  CLOMP_LAUNCH((small_loop_kernel<TA, false, KR>), g, b, lds, s, d, list, T, beta1, beta2,
               lr_rel, eps_rel);
}

template <typename TA>
static void small_dispatch(int omp, int kmax, dim3 g, dim3 b, size_t lds, hipStream_t s,
                           const Inst* d, const int* list, int T, float beta1, float beta2,
                           float lr_rel, float eps_rel) {
  if (omp)
    CLOMP_LAUNCH((small_loop_kernel<TA, true, 8>), g, b, lds, s, d, list, T, beta1, beta2,
                 lr_rel, eps_rel);
  else if (kmax <= 8)
    small_clomp<TA, 8>(g, b, lds, s, d, list, T, beta1, beta2, lr_rel, eps_rel);
  else if (kmax <= 16)
    small_clomp<TA, 16>(g, b, lds, s, d, list, T, beta1, beta2, lr_rel, eps_rel);
  else if (kmax <= 32)
    small_clomp<TA, 32>(g, b, lds, s, d, list, T, beta1, beta2, lr_rel, eps_rel);
  else
    small_clomp<TA, 64>(g, b, lds, s, d, list, T, beta1, beta2, lr_rel, eps_rel);
}

hipError_t launch_small(int bf16, int omp, const Inst* d, const int* list, int count, int kmax,
                        int T, float beta1, float beta2, float lr_rel, float eps_rel, size_t lds,
                        hipStream_t s) {
  if (count <= 0) return nothing_to_launch(s);
  if (kmax < 1 || kmax > kSmallMaxK) return hipErrorInvalidValue;
  const dim3 g(count), b(kSmallThreads);
  if (bf16)
    small_dispatch<uint16_t>(omp, kmax, g, b, lds, s, d, list, T, beta1, beta2, lr_rel, eps_rel);
  else
    small_dispatch<float>(omp, kmax, g, b, lds, s, d, list, T, beta1, beta2, lr_rel, eps_rel);
  return hipGetLastError();
}

template <typename TA>
static hipError_t iht_grad_lpa(int lpa, const Inst* d, const ScanTile* tiles, int ntiles,
                               int nslice, int r_lds, int first, hipStream_t s) {
  const dim3 g(ntiles, nslice), b(kBlock);
  const size_t lds = (size_t)r_lds * sizeof(float);
  switch (lpa) {
    case 4: CLOMP_LAUNCH((iht_grad_kernel<TA, 4>), g, b, lds, s, d, tiles, r_lds, first); break;
    case 8: CLOMP_LAUNCH((iht_grad_kernel<TA, 8>), g, b, lds, s, d, tiles, r_lds, first); break;
    case 16: CLOMP_LAUNCH((iht_grad_kernel<TA, 16>), g, b, lds, s, d, tiles, r_lds, first); break;
    case 32: CLOMP_LAUNCH((iht_grad_kernel<TA, 32>), g, b, lds, s, d, tiles, r_lds, first); break;
    default: CLOMP_LAUNCH((iht_grad_kernel<TA, 64>), g, b, lds, s, d, tiles, r_lds, first); break;
  }
  return hipGetLastError();
}

hipError_t launch_iht_grad(int bf16, int lpa, const Inst* d, const ScanTile* tiles, int ntiles,
                           int nslice, int r_lds, int first, hipStream_t s) {
  if (ntiles <= 0) return nothing_to_launch(s);
  return bf16 ? iht_grad_lpa<uint16_t>(lpa, d, tiles, ntiles, nslice, r_lds, first, s)
              : iht_grad_lpa<float>(lpa, d, tiles, ntiles, nslice, r_lds, first, s);
}

hipError_t launch_paper_select(const Inst* dc, int nact, int it, int last, float thr,
                               float lr_rel, float beta1, float beta2, float bc1, float bc2,
                               float eps_rel, int nmax, hipStream_t s) {
  if (nact <= 0) return nothing_to_launch(s);
  if (nmax <= 4096)
    CLOMP_LAUNCH((paper_select_kernel<256>), dim3(nact), dim3(256), 0, s, dc, it, last, thr,
                 lr_rel, beta1, beta2, bc1, bc2, eps_rel);
  else
    CLOMP_LAUNCH((paper_select_kernel<1024>), dim3(nact), dim3(1024), 0, s, dc, it, last, thr,
                 lr_rel, beta1, beta2, bc1, bc2, eps_rel);
  return hipGetLastError();
}

hipError_t launch_iht_combine(const Inst* d, const ScanTile* tiles, int ntiles, int first,
                              hipStream_t s) {
  if (ntiles <= 0) return nothing_to_launch(s);
  CLOMP_LAUNCH(iht_combine_kernel, dim3(ntiles), dim3(kBlock), 0, s, d, tiles, first);
  return hipGetLastError();
}

hipError_t launch_iht_rows(int bf16, int mode, const Inst* d, const RowTile* tiles, int ntiles,
                           int kmax, int wide, hipStream_t s) {
  if (ntiles <= 0) return nothing_to_launch(s);
  if (wide) {
    // 16 waves per row tile (few tiles: a single long signal or a small class)
    const size_t lds = ((size_t)2 * (kmax + 1) + 16 * 64) * sizeof(float);
    const dim3 b(16 * 64);
    if (bf16) {
      if (mode == 0)
        CLOMP_LAUNCH((rows_kernel<uint16_t, ROW_IHT_R, 16>), dim3(ntiles), b, lds, s, d, tiles,
                     kmax, 0, 0.f);
      else
        CLOMP_LAUNCH((rows_kernel<uint16_t, ROW_IHT_U, 16>), dim3(ntiles), b, lds, s, d, tiles,
                     kmax, 0, 0.f);
    } else {
      if (mode == 0)
        CLOMP_LAUNCH((rows_kernel<float, ROW_IHT_R, 16>), dim3(ntiles), b, lds, s, d, tiles,
                     kmax, 0, 0.f);
      else
        CLOMP_LAUNCH((rows_kernel<float, ROW_IHT_U, 16>), dim3(ntiles), b, lds, s, d, tiles,
                     kmax, 0, 0.f);
    }
    return hipGetLastError();
  }
  const size_t lds = ((size_t)2 * (kmax + 1) + 4 * 64) * sizeof(float);
  if (bf16) {
    if (mode == 0)
      CLOMP_LAUNCH((rows_kernel<uint16_t, ROW_IHT_R>), dim3(ntiles), dim3(kBlock), lds, s, d,
                   tiles, kmax, 0, 0.f);
    else
      CLOMP_LAUNCH((rows_kernel<uint16_t, ROW_IHT_U>), dim3(ntiles), dim3(kBlock), lds, s, d,
                   tiles, kmax, 0, 0.f);
  } else {
    if (mode == 0)
      CLOMP_LAUNCH((rows_kernel<float, ROW_IHT_R>), dim3(ntiles), dim3(kBlock), lds, s, d, tiles,
                   kmax, 0, 0.f);
    else
      CLOMP_LAUNCH((rows_kernel<float, ROW_IHT_U>), dim3(ntiles), dim3(kBlock), lds, s, d, tiles,
                   kmax, 0, 0.f);
  }
  return hipGetLastError();
}

hipError_t launch_iht_select(const Inst* dc, int nact, int mode, int nmax, hipStream_t s) {
  if (nact <= 0) return nothing_to_launch(s);
  const dim3 g(nact);
  if (nmax <= 256) {
    CLOMP_LAUNCH((iht_select_kernel<256, 1>), g, dim3(256), 0, s, dc, mode);
  } else if (nmax <= 1024) {
    CLOMP_LAUNCH((iht_select_kernel<256, 4>), g, dim3(256), 0, s, dc, mode);
  } else if (nmax <= 4096) {
    CLOMP_LAUNCH((iht_select_kernel<256, 16>), g, dim3(256), 0, s, dc, mode);
  } else if (nmax <= 16384) {
    CLOMP_LAUNCH((iht_select_kernel<1024, 16>), g, dim3(1024), 0, s, dc, mode);
  } else if (nmax <= 65536) {
    CLOMP_LAUNCH((iht_select_kernel<1024, 64>), g, dim3(1024), 0, s, dc, mode);
  } else {
    CLOMP_LAUNCH((iht_select_kernel<1024, 0>), g, dim3(1024), 0, s, dc, mode);
  }
  return hipGetLastError();
}

hipError_t set_max_lds(size_t bytes) {
  // Raise the dynamic-LDS ceiling of the kernels that stage vectors.
  const void* fns[] = {
      (const void*)small_loop_kernel<float, true, 8>,
      (const void*)small_loop_kernel<float, false, 8>,
      (const void*)small_loop_kernel<float, false, 16>,
      (const void*)small_loop_kernel<float, false, 32>,
      (const void*)small_loop_kernel<float, false, 64>,
      (const void*)small_loop_kernel<uint16_t, true, 8>,
      (const void*)small_loop_kernel<uint16_t, false, 8>,
      (const void*)small_loop_kernel<uint16_t, false, 16>,
      (const void*)small_loop_kernel<uint16_t, false, 32>,
      (const void*)small_loop_kernel<uint16_t, false, 64>,
      (const void*)iht_grad_kernel<float, 4>, (const void*)iht_grad_kernel<float, 8>,
      (const void*)iht_grad_kernel<float, 16>, (const void*)iht_grad_kernel<float, 32>,
      (const void*)iht_grad_kernel<float, 64>, (const void*)iht_grad_kernel<uint16_t, 4>,
      (const void*)iht_grad_kernel<uint16_t, 8>, (const void*)iht_grad_kernel<uint16_t, 16>,
      (const void*)iht_grad_kernel<uint16_t, 32>, (const void*)iht_grad_kernel<uint16_t, 64>,
      (const void*)scan_kernel<float, 4>, (const void*)scan_kernel<float, 8>,
      (const void*)scan_kernel<float, 16>, (const void*)scan_kernel<float, 32>,
      (const void*)scan_kernel<float, 64>, (const void*)scan_kernel<uint16_t, 4>,
      (const void*)scan_kernel<uint16_t, 8>, (const void*)scan_kernel<uint16_t, 16>,
      (const void*)scan_kernel<uint16_t, 32>, (const void*)scan_kernel<uint16_t, 64>,
      (const void*)gram_kernel<float, 4>, (const void*)gram_kernel<float, 8>,
      (const void*)gram_kernel<float, 16>, (const void*)gram_kernel<float, 32>,
      (const void*)gram_kernel<float, 64>, (const void*)gram_kernel<uint16_t, 4>,
      (const void*)gram_kernel<uint16_t, 8>, (const void*)gram_kernel<uint16_t, 16>,
      (const void*)gram_kernel<uint16_t, 32>, (const void*)gram_kernel<uint16_t, 64>,
      (const void*)cg_dots_kernel<4, 0>, (const void*)cg_dots_kernel<8, 0>,
      (const void*)cg_dots_kernel<16, 0>, (const void*)cg_dots_kernel<32, 0>,
      (const void*)cg_dots_kernel<64, 0>, (const void*)cg_dots_kernel<4, 1>,
      (const void*)cg_dots_kernel<8, 1>, (const void*)cg_dots_kernel<16, 1>,
      (const void*)cg_dots_kernel<32, 1>, (const void*)cg_dots_kernel<64, 1>,
      (const void*)qr_refine_kernel, (const void*)image_step_kernel};
  return raise_dynamic_lds(fns, sizeof(fns) / sizeof(fns[0]), bytes);
}

template <typename TA>
static hipError_t ypass_dispatch(int lpa, const Inst* d, const ScanTile* tiles, int ntiles,
                                 size_t lds, hipStream_t s) {
  const dim3 g(ntiles), b(kPassThreads);
  switch (lpa) {
    case 4: CLOMP_LAUNCH((ypass_kernel<TA, 4>), g, b, lds, s, d, tiles); break;
    case 8: CLOMP_LAUNCH((ypass_kernel<TA, 8>), g, b, lds, s, d, tiles); break;
    case 16: CLOMP_LAUNCH((ypass_kernel<TA, 16>), g, b, lds, s, d, tiles); break;
    case 32: CLOMP_LAUNCH((ypass_kernel<TA, 32>), g, b, lds, s, d, tiles); break;
    default: CLOMP_LAUNCH((ypass_kernel<TA, 64>), g, b, lds, s, d, tiles); break;
  }
  return hipGetLastError();
}

hipError_t launch_ypass(int bf16, int lpa, const Inst* d, const ScanTile* tiles, int ntiles,
                        size_t lds, hipStream_t s) {
  if (ntiles <= 0) return nothing_to_launch(s);
  return bf16 ? ypass_dispatch<uint16_t>(lpa, d, tiles, ntiles, lds, s)
              : ypass_dispatch<float>(lpa, d, tiles, ntiles, lds, s);
}

template <typename TA, int LPA>
static hipError_t coef_pass_lpa(int coef, const Inst* dc, int nact, int W, const Inst* d,
                                const ScanTile* tiles, int ntiles, int t, int T, float b1,
                                float b2, float lr_rel, float eps_rel, size_t lds,
                                hipStream_t s) {
  const dim3 g(nact * W + ntiles), b(kPassThreads);
  switch (coef) {
    case COEF_ADAM_REG:
      CLOMP_LAUNCH((coef_pass_kernel<TA, LPA, COEF_ADAM_REG>), g, b, lds, s, dc, nact, W, d,
                         tiles, t, T, b1, b2, lr_rel, eps_rel);
      break;
    case COEF_ADAM_GLOBAL:
      CLOMP_LAUNCH((coef_pass_kernel<TA, LPA, COEF_ADAM_GLOBAL>), g, b, lds, s, dc, nact, W, d,
                         tiles, t, T, b1, b2, lr_rel, eps_rel);
      break;
    case COEF_ADAM_TEAM:
      CLOMP_LAUNCH((coef_pass_kernel<TA, LPA, COEF_ADAM_TEAM>), g, b, lds, s, dc, nact, W, d,
                         tiles, t, T, b1, b2, lr_rel, eps_rel);
      break;
    case COEF_OMP_TEAM:
      CLOMP_LAUNCH((coef_pass_kernel<TA, LPA, COEF_OMP_TEAM>), g, b, lds, s, dc, nact, W, d,
                         tiles, t, T, b1, b2, lr_rel, eps_rel);
      break;
    default:
      CLOMP_LAUNCH((coef_pass_kernel<TA, LPA, COEF_OMP>), g, b, lds, s, dc, nact, W, d, tiles,
                         t, T, b1, b2, lr_rel, eps_rel);
      break;
  }
  return hipGetLastError();
}

template <typename TA>
static hipError_t coef_pass_dispatch(int lpa, int coef, const Inst* dc, int nact, int W,
                                     const Inst* d, const ScanTile* tiles, int ntiles, int t,
                                     int T, float b1, float b2, float lr, float ep, size_t lds,
                                     hipStream_t s) {
  switch (lpa) {
    case 4: return coef_pass_lpa<TA, 4>(coef, dc, nact, W, d, tiles, ntiles, t, T, b1, b2, lr, ep, lds, s);
    case 8: return coef_pass_lpa<TA, 8>(coef, dc, nact, W, d, tiles, ntiles, t, T, b1, b2, lr, ep, lds, s);
    case 16: return coef_pass_lpa<TA, 16>(coef, dc, nact, W, d, tiles, ntiles, t, T, b1, b2, lr, ep, lds, s);
    case 32: return coef_pass_lpa<TA, 32>(coef, dc, nact, W, d, tiles, ntiles, t, T, b1, b2, lr, ep, lds, s);
    default: return coef_pass_lpa<TA, 64>(coef, dc, nact, W, d, tiles, ntiles, t, T, b1, b2, lr, ep, lds, s);
  }
}

template <typename TA, int LPA>
static int team_blocks_per_cu(int omp, size_t lds) {
  int nb = 0;
  const hipError_t e =
      omp ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, coef_pass_kernel<TA, LPA, COEF_OMP_TEAM>, kPassThreads, lds)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, coef_pass_kernel<TA, LPA, COEF_ADAM_TEAM>, kPassThreads, lds);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

int coef_team_blocks_per_cu(int bf16, int lpa, int omp, size_t lds) {
  switch (lpa) {
    case 4: return bf16 ? team_blocks_per_cu<uint16_t, 4>(omp, lds) : team_blocks_per_cu<float, 4>(omp, lds);
    case 8: return bf16 ? team_blocks_per_cu<uint16_t, 8>(omp, lds) : team_blocks_per_cu<float, 8>(omp, lds);
    case 16: return bf16 ? team_blocks_per_cu<uint16_t, 16>(omp, lds) : team_blocks_per_cu<float, 16>(omp, lds);
    case 32: return bf16 ? team_blocks_per_cu<uint16_t, 32>(omp, lds) : team_blocks_per_cu<float, 32>(omp, lds);
    default: return bf16 ? team_blocks_per_cu<uint16_t, 64>(omp, lds) : team_blocks_per_cu<float, 64>(omp, lds);
  }
}

hipError_t launch_coef_pass(int bf16, int lpa, int omp, const Inst* dc, int nact, int W,
                            const Inst* d, const ScanTile* tiles, int ntiles, int t, int T,
                            float beta1, float beta2, float lr_rel, float eps_rel, size_t lds,
                            hipStream_t s) {
  if (nact + ntiles <= 0) return nothing_to_launch(s);
  // a team needs t >= 1: at t = 0 the step size and eps are set in the launch
  if (W < 1 || W > kTeamMax || (W > 1 && (t < 1 || W * kTeamRows < t + 1)))
    return hipErrorInvalidValue;
  const int coef = W > 1 ? (omp ? COEF_OMP_TEAM : COEF_ADAM_TEAM)
                         : omp ? COEF_OMP : (t + 1 <= kRegRows ? COEF_ADAM_REG : COEF_ADAM_GLOBAL);
  return bf16 ? coef_pass_dispatch<uint16_t>(lpa, coef, dc, nact, W, d, tiles, ntiles, t, T,
                                             beta1, beta2, lr_rel, eps_rel, lds, s)
              : coef_pass_dispatch<float>(lpa, coef, dc, nact, W, d, tiles, ntiles, t, T, beta1,
                                          beta2, lr_rel, eps_rel, lds, s);
}

hipError_t launch_shared_gram(int bf16, const Inst* d, int nsig, int n, float* Gf, float* dg,
                              hipStream_t s) {
  if (nsig <= 0) return nothing_to_launch(s);
  const int nt = (n + kMfmaTile - 1) / kMfmaTile;
  const dim3 g0(nt, nt), g1(nt, (nsig + kMfmaTile - 1) / kMfmaTile);
  if (bf16) {
    CLOMP_LAUNCH((shared_mfma_bf16_kernel<0>), g0, dim3(256), 0, s, d, nsig, Gf, 0);
    // c0 = A^T Y keeps Y in FP32 (b = A_S^T y of the coefficient fit)
    CLOMP_LAUNCH((shared_mfma_kernel<uint16_t, 1>), g1, dim3(256), 0, s, d, nsig, Gf, 0);
  } else {
    CLOMP_LAUNCH((shared_mfma_kernel<float, 0>), g0, dim3(256), 0, s, d, nsig, Gf, 0);
    CLOMP_LAUNCH((shared_mfma_kernel<float, 1>), g1, dim3(256), 0, s, d, nsig, Gf, 0);
  }
  CLOMP_LAUNCH(shared_diag_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, d, Gf, dg);
  return hipGetLastError();
}

hipError_t launch_coef_omp(const Inst* dc, int nact, int t, float lr_rel, float eps_rel,
                           hipStream_t s) {
  if (nact <= 0) return nothing_to_launch(s);
  const size_t lds = (size_t)3 * (t + 1) * sizeof(float);
  CLOMP_LAUNCH(coef_omp_kernel, dim3(nact), dim3(256), lds, s, dc, t, lr_rel, eps_rel);
  return hipGetLastError();
}

hipError_t launch_coef_reg(const Inst* dc, int nact, int t, int T, float beta1, float beta2,
                            float lr_rel, float eps_rel, hipStream_t s) {
  if (nact <= 0) return nothing_to_launch(s);
  if (t + 1 > kRegRows) return hipErrorInvalidValue;
  const int waves = (t + 1 + 15) / 16;
  const dim3 g(nact), b(64 * waves);
  if (t + 1 <= 64)
    CLOMP_LAUNCH(coef_reg_kernel<1>, g, b, 0, s, dc, t, T, beta1, beta2, lr_rel, eps_rel);
  else if (t + 1 <= 128)
    CLOMP_LAUNCH(coef_reg_kernel<2>, g, b, 0, s, dc, t, T, beta1, beta2, lr_rel, eps_rel);
  else
    CLOMP_LAUNCH(coef_reg_kernel<4>, g, b, 0, s, dc, t, T, beta1, beta2, lr_rel, eps_rel);
  return hipGetLastError();
}

hipError_t launch_shared_rows(int bf16, int mode, const Inst* d, int nsig, int t1,
                              hipStream_t s) {
  if (nsig <= 0) return nothing_to_launch(s);
  if (t1 > 256) return hipErrorInvalidValue;
  const dim3 g(nsig), b(256);
  if (bf16) {
    if (mode == 0)
      CLOMP_LAUNCH((shared_rows_kernel<uint16_t, 0>), g, b, 0, s, d, t1);
    else
      CLOMP_LAUNCH((shared_rows_kernel<uint16_t, 1>), g, b, 0, s, d, t1);
  } else {
    if (mode == 0)
      CLOMP_LAUNCH((shared_rows_kernel<float, 0>), g, b, 0, s, d, t1);
    else
      CLOMP_LAUNCH((shared_rows_kernel<float, 1>), g, b, 0, s, d, t1);
  }
  return hipGetLastError();
}

hipError_t launch_shared_grad(int bf16, const Inst* d, int nsig, int n, int first,
                              hipStream_t s) {
  if (nsig <= 0) return nothing_to_launch(s);
  const dim3 g((n + kMfmaTile - 1) / kMfmaTile, (nsig + kMfmaTile - 1) / kMfmaTile);
  if (bf16)
    CLOMP_LAUNCH((shared_mfma_kernel<uint16_t, 3>), g, dim3(256), 0, s, d, nsig, nullptr, first);
  else
    CLOMP_LAUNCH((shared_mfma_kernel<float, 3>), g, dim3(256), 0, s, d, nsig, nullptr, first);
  return hipGetLastError();
}

hipError_t launch_shared_rscan(int bf16, const Inst* d, int nsig, int n, int t, hipStream_t s) {
  if (nsig <= 0) return nothing_to_launch(s);
  const dim3 g((n + kMfmaTile - 1) / kMfmaTile, (nsig + kMfmaTile - 1) / kMfmaTile);
  if (bf16)
    CLOMP_LAUNCH((shared_mfma_bf16_kernel<2>), g, dim3(256), 0, s, d, nsig, nullptr, t);
  else
    CLOMP_LAUNCH((shared_mfma_kernel<float, 2>), g, dim3(256), 0, s, d, nsig, nullptr, t);
  return hipGetLastError();
}

hipError_t launch_cscan(const Inst* d, const ScanTile* tiles, int ntiles, int t, hipStream_t s) {
  if (ntiles <= 0) return nothing_to_launch(s);
  // waves per tile from the number of tiles: about 16 waves per CU or more
  if (ntiles >= 4096)
    CLOMP_LAUNCH(cscan_kernel<1>, dim3((ntiles + 3) / 4), dim3(256), 0, s, d, tiles, ntiles, t);
  else if (ntiles >= 1024)
    CLOMP_LAUNCH(cscan_kernel<4>, dim3(ntiles), dim3(256), 0, s, d, tiles, ntiles, t);
  else
    CLOMP_LAUNCH(cscan_kernel<16>, dim3(ntiles), dim3(1024), 0, s, d, tiles, ntiles, t);
  return hipGetLastError();
}

hipError_t launch_image_init(float* D, int n, long long ldd, float* zero, long long nzero,
                             hipStream_t s) {
  const long long tot = (long long)n * n + nzero;
  const int grid = (int)std::min<long long>((tot + kBlock - 1) / kBlock, 4096);
  CLOMP_LAUNCH(image_init_kernel, dim3(std::max(grid, 1)), dim3(kBlock), 0, s, D, n, ldd, zero,
               nzero);
  return hipGetLastError();
}

hipError_t launch_image_record(const Inst* d, int W, int t, float lr_rel, float eps_rel,
                               hipStream_t s) {
  if (W <= 0) return nothing_to_launch(s);
  CLOMP_LAUNCH(image_record_kernel, dim3(W), dim3(kBlock), 0, s, d, t, lr_rel, eps_rel);
  return hipGetLastError();
}

hipError_t launch_image_synth(const Inst* d, int W, int t1, const float* D, long long ldd,
                              float* X, hipStream_t s) {
  if (W <= 0) return nothing_to_launch(s);
  if (t1 > kImageMaxK) return hipErrorInvalidValue;
  CLOMP_LAUNCH(image_synth_kernel, dim3(W), dim3(kBlock), 0, s, d, t1, D, ldd, X);
  return hipGetLastError();
}

hipError_t launch_image_step(const Inst* d, int W, int n, int t, int step, float beta1,
                             float beta2, float htv, float wlv, const float* D, long long ldd,
                             const float* X, const float* Sd_cur, float* Sd_next, hipStream_t s) {
  if (W <= 0) return nothing_to_launch(s);
  if (t + 1 > kImageMaxK || n > kImageMaxN) return hipErrorInvalidValue;
  const size_t lds = (wlv != 0.f && n >= 3 && W >= 3) ? (size_t)6 * n * sizeof(float) : 0;
  CLOMP_LAUNCH(image_step_kernel, dim3(W), dim3(kBlock), lds, s, d, W, t, step, beta1, beta2,
               htv, wlv, D, ldd, X, Sd_cur, Sd_next);
  return hipGetLastError();
}

hipError_t set_max_lds_pass(size_t bytes) {
  const void* fns[] = {
      (const void*)ypass_kernel<float, 4>, (const void*)ypass_kernel<float, 8>,
      (const void*)ypass_kernel<float, 16>, (const void*)ypass_kernel<float, 32>,
      (const void*)ypass_kernel<float, 64>, (const void*)ypass_kernel<uint16_t, 4>,
      (const void*)ypass_kernel<uint16_t, 8>, (const void*)ypass_kernel<uint16_t, 16>,
      (const void*)ypass_kernel<uint16_t, 32>, (const void*)ypass_kernel<uint16_t, 64>,
#define CP(TA, L) (const void*)coef_pass_kernel<TA, L, COEF_ADAM_REG>, \
                  (const void*)coef_pass_kernel<TA, L, COEF_ADAM_GLOBAL>, \
                  (const void*)coef_pass_kernel<TA, L, COEF_OMP>, \
                  (const void*)coef_pass_kernel<TA, L, COEF_ADAM_TEAM>, \
                  (const void*)coef_pass_kernel<TA, L, COEF_OMP_TEAM>
      CP(float, 4), CP(float, 8), CP(float, 16), CP(float, 32), CP(float, 64),
      CP(uint16_t, 4), CP(uint16_t, 8), CP(uint16_t, 16), CP(uint16_t, 32), CP(uint16_t, 64)
#undef CP
  };
  return raise_dynamic_lds(fns, sizeof(fns) / sizeof(fns[0]), bytes);
}

}  // namespace clomp
