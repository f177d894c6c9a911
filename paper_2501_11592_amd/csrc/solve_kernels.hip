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

#include "dev_common.h"
#include "kernels.h"

namespace clomp {

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
  __syncthreads();
  if (threadIdx.x == 0) {
    InstState st = {};
    st.done = any_nz ? 0 : 1;
    *I.st = st;
    *I.key = 0ull;
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
template <typename TA, int LPA>
__global__ __launch_bounds__(kBlock) void scan_kernel(const Inst* __restrict__ insts,
                                                      const ScanTile* __restrict__ tiles,
                                                      int r_in_lds) {
  extern __shared__ float smem[];
  __shared__ unsigned long long wbest[kWaves];
  const ScanTile tile = tiles[blockIdx.x];
  const Inst& I = insts[tile.inst];
  if (I.st->done) return;
  constexpr int VW = Vec<TA>::W;
  const int m = I.m;
  const int nvec = (m + VW - 1) / VW;
  const float* rp = I.r;  // zero padded to a multiple of 8
  if (r_in_lds) {
    for (int i = threadIdx.x; i < nvec * VW; i += kBlock) smem[i] = I.r[i];
    __syncthreads();
    rp = smem;
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
    float acc = 0.f;
#pragma unroll 8
    for (int c = gl; c < nvec; c += LPA) {
      float v[VW];
      Vec<TA>::load(col + (long long)c * VW, v);
      if (c == nvec - 1) {
#pragma unroll
        for (int e = 0; e < VW; ++e) v[e] = (e < tail) ? v[e] : 0.f;
      }
      const float* rr = rp + c * VW;
#pragma unroll
      for (int e = 0; e < VW; ++e) acc = fmaf(v[e], rr[e], acc);
    }
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
  extern __shared__ float smem[];
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
    if (t == 0) {
      I.st->sigma = cj;
      I.st->lr = lr_rel * cj;
      I.st->eps = eps_rel * cj;
    }
  }
}

// ============================================================ Adam (CLOMP)
// One workgroup per active instance; rows of G are split over the threads
// (up to kRPT rows each).  T steps of
//   g = G s - b;  m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
//   s -= lr * (m / bc1) / (sqrt(v / bc2) + eps)
// with bias corrections bc = 1 - beta^step (Kingma & Ba, Algorithm 1).  The
// instance key is cleared for the next scan.
constexpr int kRPT = 8;  // supports k_eff <= kBlock * kRPT = 2048

__global__ __launch_bounds__(kBlock) void adam_kernel(const Inst* __restrict__ insts, int t,
                                                      int T, float beta1, float beta2) {
  extern __shared__ float ssh[];  // s[t+1]
  const Inst& I = insts[blockIdx.x];
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
    const int r = threadIdx.x + q * kBlock;
    if (r < t1) {
      ssh[r] = I.s[r];
      mo[q] = I.mo[r];
      ve[q] = I.ve[r];
      bb[q] = I.b[r];
    }
  }
  const float lr = I.st->lr, eps = I.st->eps;
  const int step0 = I.st->step;
  __syncthreads();
  for (int it = 0; it < T; ++it) {
    const int step = step0 + it + 1;
    const float bc1 = (float)(1.0 - pow((double)beta1, (double)step));
    const float bc2 = (float)(1.0 - pow((double)beta2, (double)step));
#pragma unroll
    for (int q = 0; q < kRPT; ++q) g[q] = 0.f;
    for (int c = 0; c < t1; ++c) {
      const float sc = ssh[c];
      const float* Gc = G + (long long)c * ldg;
#pragma unroll
      for (int q = 0; q < kRPT; ++q) {
        const int r = threadIdx.x + q * kBlock;
        if (r < t1) g[q] = fmaf(Gc[r], sc, g[q]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kRPT; ++q) {
      const int r = threadIdx.x + q * kBlock;
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
    const int r = threadIdx.x + q * kBlock;
    if (r < t1) {
      I.s[r] = ssh[r];
      I.mo[r] = mo[q];
      I.ve[r] = ve[q];
    }
  }
  if (threadIdx.x == 0) {
    I.st->step = step0 + T;
    *I.key = 0ull;
  }
}

// ============================================================ OMP coefficients
// One workgroup per active instance.  With L L^T = G_S and Linv = L^{-1}
// (lower triangular), appending column t with Gram column g (g_tt last):
//   w = Linv g[0:t],  lambda = sqrt(g_tt - w.w),
//   Linv[t, :t] = -(w^T Linv) / lambda,  Linv[t, t] = 1 / lambda,
//   z_t = (b_t - w.z) / lambda,  x_S = Linv^T z.
// Every step is a parallel triangular mat-vec; no sequential solve is needed.
__global__ __launch_bounds__(kBlock) void omp_chol_kernel(const Inst* __restrict__ insts, int t) {
  extern __shared__ float osh[];  // gcol[t1] | w[t1]
  __shared__ float red[kWaves];
  const Inst& I = insts[blockIdx.x];
  if (I.st->done) {
    if (threadIdx.x == 0) *I.key = 0ull;
    return;
  }
  const int t1 = t + 1;
  const long long ld = I.ldg;
  float* L = I.Linv;
  float* gcol = osh;
  float* w = osh + t1;
  for (int r = threadIdx.x; r < t1; r += kBlock) gcol[r] = I.G[r + (long long)t * ld];
  __syncthreads();
  for (int r = threadIdx.x; r < t; r += kBlock) {
    float acc = 0.f;
    for (int c = 0; c <= r; ++c) acc = fmaf(L[r + (long long)c * ld], gcol[c], acc);
    w[r] = acc;
  }
  __syncthreads();
  float part = 0.f, pz = 0.f;
  for (int r = threadIdx.x; r < t; r += kBlock) {
    part = fmaf(w[r], w[r], part);
    pz = fmaf(w[r], I.z[r], pz);
  }
  const float ww = block_sum(part, red);
  const float wz = block_sum(pz, red);
  const float gtt = gcol[t];
  float lam2 = gtt - ww;
  const bool bad = !(lam2 > 1e-7f * gtt);
  if (bad) lam2 = fmaxf(1e-7f * gtt, 1e-30f);
  const float lam = sqrtf(lam2);
  for (int c = threadIdx.x; c < t; c += kBlock) {
    float acc = 0.f;
    for (int r = c; r < t; ++r) acc = fmaf(w[r], L[r + (long long)c * ld], acc);
    L[t + (long long)c * ld] = -acc / lam;
  }
  if (threadIdx.x == 0) {
    L[t + (long long)t * ld] = 1.f / lam;
    I.z[t] = (I.b[t] - wz) / lam;
    if (bad) atomicOr(I.status, ST_REFINE_INACCURATE);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < t1; c += kBlock) {
    float acc = 0.f;
    for (int r = c; r < t1; ++r) acc = fmaf(L[r + (long long)c * ld], I.z[r], acc);
    I.s[c] = acc;
  }
  if (threadIdx.x == 0) *I.key = 0ull;
}

// ============================================================ rows kernels
// out_i = base_i + sign * sum_{l<=t} A[i, S_l] * coef_l  for the rows of one
// 64-row tile; the four waves split the columns and are summed in order.
enum RowMode : int {
  ROW_RESID = 0,   // r = y - A_bulk[:, S] s
  ROW_CG_R0 = 1,   // cg.r0 = y - A_master[:, S] xf
  ROW_CG_Q = 2     // cg.q = A_master[:, S] p   (+ partial ||q||^2)
};

template <typename TA, int MODE>
__global__ __launch_bounds__(kBlock) void rows_kernel(const Inst* __restrict__ insts,
                                                      const RowTile* __restrict__ tiles,
                                                      int t, int it, float tol2) {
  extern __shared__ float rsh[];  // coef[t1] | (int) sup[t1] | part[4*64]
  __shared__ float red[kWaves];
  const RowTile rt = tiles[blockIdx.x];
  const Inst& I = insts[rt.inst];
  if (I.st->done) return;
  // in the loop every active instance has t+1 atoms; after it, its own count
  const int t1 = (MODE == ROW_RESID) ? t + 1 : *I.nsel;
  float* coef = rsh;
  int* sup = reinterpret_cast<int*>(rsh + t1);
  float* part = rsh + 2 * t1;
  const float* src;
  if (MODE == ROW_RESID) src = I.s;
  else if (MODE == ROW_CG_R0) src = I.xf;
  else src = nullptr;
  if (MODE == ROW_CG_Q) {
    // CGLS direction: gamma = ||sv||^2; p = sv (first) or sv + beta p_old.
    if (I.st->cg_done) return;
    const float* sv = I.cg + 3 * I.m_pad + 2 * I.k_eff;
    float pg = 0.f;
    for (int l = threadIdx.x; l < t1; l += kBlock) pg = fmaf(sv[l], sv[l], pg);
    const float gamma = block_sum(pg, red);
    const float gamma0 = (it == 0) ? gamma : I.st->gamma0;
    if (it > 0 && gamma <= tol2 * gamma0) {
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
    if (rt.tile == 0 && threadIdx.x == 0) {
      I.st->gamma[it & 1] = gamma;
      if (it == 0) I.st->gamma0 = gamma;
    }
  } else {
    for (int l = threadIdx.x; l < t1; l += kBlock) coef[l] = src[l];
  }
  for (int l = threadIdx.x; l < t1; l += kBlock) sup[l] = I.support[l];
  __syncthreads();
  const TA* A;
  long long lda;
  if (MODE == ROW_RESID) {
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
    for (int l = w; l < t1; l += kWaves)
      acc = fmaf(Vec<TA>::one(A + (long long)sup[l] * lda + i), coef[l], acc);
  }
  part[w * 64 + lane] = acc;
  __syncthreads();
  if (w == 0) {
    float v = 0.f;
    if (i < rt.i1) {
      const float sum = (part[lane] + part[64 + lane]) + (part[128 + lane] + part[192 + lane]);
      const float* yw = I.r + I.m_pad;
      if (MODE == ROW_RESID) {
        I.r[i] = yw[i] - sum;
      } else if (MODE == ROW_CG_R0) {
        I.cg[i] = yw[i] - sum;  // r0
      } else {
        I.cg[2 * I.m_pad + i] = sum;  // q
        v = sum * sum;
      }
    }
    if (MODE == ROW_CG_Q) {
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
  extern __shared__ float vsh[];
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
    for (int tt = 0; tt < I.n_rowtiles; ++tt) qq += I.qpart[tt];
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
// triangular solve R x = Q^T y, one workgroup per instance in the list.
__global__ __launch_bounds__(kBlock) void qr_refine_kernel(const Inst* __restrict__ insts,
                                                           const int* __restrict__ list) {
  extern __shared__ float qsh[];
  __shared__ float red[kWaves];
  __shared__ float diag[1];
  const Inst& I = insts[list[blockIdx.x]];
  if (I.st->done) return;
  const int m = I.m;
  const int t1 = *I.nsel;
  float* M = qsh;                  // m x t1 column-major (ld m)
  float* yv = qsh + (long long)m * t1;   // m
  float* Rd = yv + m;              // t1 diagonal of R
  float* xs = Rd + t1;             // t1 solution
  for (int idx = threadIdx.x; idx < m * t1; idx += kBlock) {
    const int c = idx / m, i = idx - c * m;
    M[idx] = I.Am[(long long)I.support[c] * I.ldam + i];
  }
  const float* yw = I.r + I.m_pad;
  for (int i = threadIdx.x; i < m; i += kBlock) yv[i] = yw[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  bool rank_def = false;
  for (int c = 0; c < t1; ++c) {
    float* Mc = M + (long long)c * m;
    float p = 0.f;
    for (int i = c + threadIdx.x; i < m; i += kBlock) p = fmaf(Mc[i], Mc[i], p);
    const float nrm2 = block_sum(p, red);
    const float x0 = Mc[c];
    const float nrm = sqrtf(nrm2);
    const float alpha = (x0 >= 0.f) ? -nrm : nrm;
    const float v0 = x0 - alpha;
    const float vn2 = nrm2 - x0 * x0 + v0 * v0;   // ||v||^2
    __syncthreads();
    if (threadIdx.x == 0) {
      Mc[c] = v0;        // v stored in place (rows c..m-1)
      diag[0] = alpha;
    }
    __syncthreads();
    if (threadIdx.x == 0) Rd[c] = alpha;
    if (!(nrm > 0.f) || !(vn2 > 0.f)) {
      rank_def = true;
      __syncthreads();
      continue;
    }
    const float inv = 2.f / vn2;
    // apply H = I - 2 v v^T / (v^T v) to columns c+1..t1-1 and y: one wave per
    // target, lanes over rows
    for (int cc = c + 1 + wv; cc <= t1; cc += kWaves) {
      float* tgt = (cc < t1) ? (M + (long long)cc * m) : yv;
      float d = 0.f;
      for (int i = c + lane; i < m; i += 64) d = fmaf(Mc[i], tgt[i], d);
      d = wave_sum(d) * inv;
      for (int i = c + lane; i < m; i += 64) tgt[i] = fmaf(-d, Mc[i], tgt[i]);
    }
    __syncthreads();
  }
  // R has diagonal Rd[c] and strictly-upper entries M[c, cc] (cc > c).
  // back substitution, one row at a time (wave 0 reduces)
  for (int c = t1 - 1; c >= 0; --c) {
    if (wv == 0) {
      float sacc = 0.f;
      for (int cc = c + 1 + lane; cc < t1; cc += 64) sacc = fmaf(M[c + (long long)cc * m], xs[cc], sacc);
      sacc = wave_sum(sacc);
      if (lane == 0) {
        const float d = Rd[c];
        xs[c] = (d != 0.f) ? (yv[c] - sacc) / d : 0.f;
      }
    }
    __syncthreads();
  }
  for (int c = threadIdx.x; c < t1; c += kBlock) I.xf[c] = xs[c];
  if (rank_def && threadIdx.x == 0) atomicOr(I.status, ST_REFINE_INACCURATE);
}

// ============================================================ FP64 norm
// Partial sums of (y_i - sum_l Am[i, S_l] xf_l)^2 accumulated in float64.
__global__ __launch_bounds__(kBlock) void norm_rows_kernel(const Inst* __restrict__ insts,
                                                           const RowTile* __restrict__ tiles) {
  extern __shared__ float nsh[];  // xf[t1] | sup[t1]
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

// One workgroup per instance: FP64 norm from the partials (fixed order),
// scatter x_S into x, refinement status.
__global__ __launch_bounds__(kBlock) void finalize_kernel(const Inst* __restrict__ insts,
                                                          int check_cg) {
  const Inst& I = insts[blockIdx.x];
  const int t1 = *I.nsel;
  for (int l = threadIdx.x; l < t1; l += kBlock) I.x[I.support[l]] = I.xf[l];
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int tt = 0; tt < I.n_rowtiles; ++tt) s += I.npart[tt];
    *I.rnorm = (t1 > 0) ? sqrt(s) : 0.0;
    if (check_cg && I.cg_slot >= 0 && !I.st->done && !I.st->cg_done)
      atomicOr(I.status, ST_REFINE_INACCURATE);
  }
}

// Copy the coefficients reached by the greedy loop into xf (the CGLS start).
__global__ __launch_bounds__(kBlock) void copy_s_kernel(const Inst* __restrict__ insts,
                                                        const int* __restrict__ list) {
  const Inst& I = insts[list[blockIdx.x]];
  const int t1 = *I.nsel;
  for (int l = threadIdx.x; l < t1; l += kBlock) I.xf[l] = I.s[l];
  if (threadIdx.x == 0) I.st->cg_done = 0;
}

// ============================================================ launchers
template <typename TA>
static hipError_t scan_dispatch(int lpa, const Inst* d, const ScanTile* tiles, int ntiles,
                                int r_lds_floats, hipStream_t s) {
  const size_t lds = (size_t)r_lds_floats * sizeof(float);
  const int flag = r_lds_floats > 0;
  switch (lpa) {
    case 4: hipLaunchKernelGGL((scan_kernel<TA, 4>), dim3(ntiles), dim3(kBlock), lds, s, d, tiles, flag); break;
    case 8: hipLaunchKernelGGL((scan_kernel<TA, 8>), dim3(ntiles), dim3(kBlock), lds, s, d, tiles, flag); break;
    case 16: hipLaunchKernelGGL((scan_kernel<TA, 16>), dim3(ntiles), dim3(kBlock), lds, s, d, tiles, flag); break;
    case 32: hipLaunchKernelGGL((scan_kernel<TA, 32>), dim3(ntiles), dim3(kBlock), lds, s, d, tiles, flag); break;
    default: hipLaunchKernelGGL((scan_kernel<TA, 64>), dim3(ntiles), dim3(kBlock), lds, s, d, tiles, flag); break;
  }
  return hipGetLastError();
}

hipError_t launch_init(const Inst* d, int count, hipStream_t s) {
  hipLaunchKernelGGL(init_kernel, dim3(count), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_scan(int bf16, int lpa, const Inst* d, const ScanTile* tiles, int ntiles,
                       int r_lds_floats, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  return bf16 ? scan_dispatch<uint16_t>(lpa, d, tiles, ntiles, r_lds_floats, s)
              : scan_dispatch<float>(lpa, d, tiles, ntiles, r_lds_floats, s);
}

template <typename TA>
static hipError_t gram_dispatch(int lpa, const Inst* d, int nact, int t, int nblk, int D,
                                int v_lds_floats, float lr_rel, float eps_rel, hipStream_t s) {
  const size_t lds = (size_t)v_lds_floats * sizeof(float);
  const int flag = v_lds_floats > 0;
  const dim3 g(nact * nblk), b(kBlock);
  switch (lpa) {
    case 4: hipLaunchKernelGGL((gram_kernel<TA, 4>), g, b, lds, s, d, t, nblk, D, flag, lr_rel, eps_rel); break;
    case 8: hipLaunchKernelGGL((gram_kernel<TA, 8>), g, b, lds, s, d, t, nblk, D, flag, lr_rel, eps_rel); break;
    case 16: hipLaunchKernelGGL((gram_kernel<TA, 16>), g, b, lds, s, d, t, nblk, D, flag, lr_rel, eps_rel); break;
    case 32: hipLaunchKernelGGL((gram_kernel<TA, 32>), g, b, lds, s, d, t, nblk, D, flag, lr_rel, eps_rel); break;
    default: hipLaunchKernelGGL((gram_kernel<TA, 64>), g, b, lds, s, d, t, nblk, D, flag, lr_rel, eps_rel); break;
  }
  return hipGetLastError();
}

hipError_t launch_gram(int bf16, int lpa, const Inst* d, int nact, int t, int nblk, int D,
                       int v_lds_floats, float lr_rel, float eps_rel, hipStream_t s) {
  if (nact <= 0) return hipSuccess;
  return bf16 ? gram_dispatch<uint16_t>(lpa, d, nact, t, nblk, D, v_lds_floats, lr_rel, eps_rel, s)
              : gram_dispatch<float>(lpa, d, nact, t, nblk, D, v_lds_floats, lr_rel, eps_rel, s);
}

hipError_t launch_adam(const Inst* d, int nact, int t, int T, float beta1, float beta2,
                       hipStream_t s) {
  if (nact <= 0) return hipSuccess;
  hipLaunchKernelGGL(adam_kernel, dim3(nact), dim3(kBlock), (size_t)(t + 1) * sizeof(float), s,
                     d, t, T, beta1, beta2);
  return hipGetLastError();
}

hipError_t launch_omp(const Inst* d, int nact, int t, hipStream_t s) {
  if (nact <= 0) return hipSuccess;
  hipLaunchKernelGGL(omp_chol_kernel, dim3(nact), dim3(kBlock), (size_t)2 * (t + 1) * sizeof(float),
                     s, d, t);
  return hipGetLastError();
}

hipError_t launch_resid(int bf16, const Inst* d, const RowTile* tiles, int ntiles, int t,
                        hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const size_t lds = ((size_t)2 * (t + 1) + 4 * 64) * sizeof(float);
  if (bf16)
    hipLaunchKernelGGL((rows_kernel<uint16_t, ROW_RESID>), dim3(ntiles), dim3(kBlock), lds, s, d,
                       tiles, t, 0, 0.f);
  else
    hipLaunchKernelGGL((rows_kernel<float, ROW_RESID>), dim3(ntiles), dim3(kBlock), lds, s, d,
                       tiles, t, 0, 0.f);
  return hipGetLastError();
}

hipError_t launch_cg_rows(int mode, const Inst* d, const RowTile* tiles, int ntiles, int tmax,
                          int it, float tol2, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const size_t lds = ((size_t)2 * (tmax + 1) + 4 * 64) * sizeof(float);
  if (mode == 0)
    hipLaunchKernelGGL((rows_kernel<float, ROW_CG_R0>), dim3(ntiles), dim3(kBlock), lds, s, d,
                       tiles, tmax, it, tol2);
  else
    hipLaunchKernelGGL((rows_kernel<float, ROW_CG_Q>), dim3(ntiles), dim3(kBlock), lds, s, d,
                       tiles, tmax, it, tol2);
  return hipGetLastError();
}

hipError_t launch_cg_dots(int mode, int lpa, const Inst* d, const int* list, int nlist, int tmax,
                          int nblk, int D, int m_pad_max, int it, hipStream_t s) {
  if (nlist <= 0) return hipSuccess;
  const size_t lds = (size_t)m_pad_max * sizeof(float);
  const dim3 g(nlist * nblk), b(kBlock);
#define CG_DOTS_CASE(L)                                                                     \
  case L:                                                                                   \
    if (mode == 0)                                                                          \
      hipLaunchKernelGGL((cg_dots_kernel<L, 0>), g, b, lds, s, d, list, tmax, nblk, D, it); \
    else                                                                                    \
      hipLaunchKernelGGL((cg_dots_kernel<L, 1>), g, b, lds, s, d, list, tmax, nblk, D, it); \
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
  if (nlist <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_s_kernel, dim3(nlist), dim3(kBlock), 0, s, d, list);
  return hipGetLastError();
}

hipError_t launch_qr(const Inst* d, const int* list, int nlist, size_t lds_bytes, hipStream_t s) {
  if (nlist <= 0) return hipSuccess;
  hipLaunchKernelGGL(qr_refine_kernel, dim3(nlist), dim3(kBlock), lds_bytes, s, d, list);
  return hipGetLastError();
}

hipError_t launch_norm(const Inst* d, const RowTile* tiles, int ntiles, int tmax, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const size_t lds = (size_t)2 * (tmax + 1) * sizeof(float);
  hipLaunchKernelGGL(norm_rows_kernel, dim3(ntiles), dim3(kBlock), lds, s, d, tiles);
  return hipGetLastError();
}

hipError_t launch_finalize(const Inst* d, int count, int check_cg, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3(count), dim3(kBlock), 0, s, d, check_cg);
  return hipGetLastError();
}

hipError_t set_max_lds(size_t bytes) {
  // Raise the dynamic-LDS ceiling of the kernels that stage vectors.
  const void* fns[] = {
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
      (const void*)qr_refine_kernel};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace clomp
