// Device-side data structures and small helpers shared by the CLOMP kernels.
//
// Layout in HBM (one workspace block per instance, every sub-array 256-byte
// aligned; all indices are local to the instance):
//   r      [m_pad]       float   residual y - A(mask*s) (zero beyond m)
//   G      [k_eff*ldg]   float   Gram matrix A_S^T A_S of the bulk columns,
//                                column-major, both triangles stored
//   b      [k_eff]       float   A_S^T y
//   s,mo,ve[k_eff]       float   coefficients and Adam moments, selection order
//   xf     [k_eff]       float   refined coefficients
//   Linv   [k_eff*ldg]   float   OMP: inverse Cholesky factor of G (lower)
//   z      [k_eff]       float   OMP: Linv * b
//   cg     [...]         float   CGLS vectors (two r, two p, q, sv)
//   bitmap [ceil(n/32)]  uint32  selected-atom mask
//   key    u64[2]        packed argmax key of the current scan (the
//                        correlation-update schedule alternates the two slots)
//   st     InstState     scalar state (sigma, lr, eps, step, flags)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace clomp {

constexpr int kBlock = 256;     // threads per workgroup for every solver kernel
constexpr int kTeamRows = 16;   // coefficient rows per team member
// dynamic LDS of the split-row Adam (256 < t+1 <= 1024): s padded to 4, and
// P * ceil((t+1)/4) <= 1024 partial float4s
constexpr int kSplitLdsFloats = 1024 + 4 * 1024;
constexpr int kTeamMax = 128;   // team members per signal (2048 rows)
// IHT gradient scan: at most this many floats of r are staged in LDS per
// workgroup; longer columns are split into slices of m whose partial dots
// are summed afterwards in slice order.
constexpr int kIhtSliceFloats = 6144;
constexpr int kSmallMaxK = 64;  // fused small-signal loop: k_eff bound (one wave)
// Image mode (the columns of one image, coupled by the priors): largest n
// (the five pixel columns of a local-variation neighbourhood and the pixel
// gradient in LDS) and largest k_eff (support vectors in LDS).
constexpr int kImageMaxN = 4096;
constexpr int kImageMaxK = 1024;
// Polls of a coefficient-team wait before it gives up and sets the watchdog
// bit (default; clomp_set_tuning can lower it).
constexpr unsigned kSpinLimitDefault = 1u << 20;

// Fused small-signal loop: row stride of the LDS Gram / inverse-Gram matrix
// and the dynamic LDS of one signal (G | A as FP32, odd leading dimension |
// r | y | selection bitmap).
__host__ __device__ inline int small_ldq(int ke) { return ((ke + 3) & ~3) + 4; }
__host__ __device__ inline size_t small_lds_bytes(int n, int m, int ke) {
  const size_t al = ((size_t)n * (size_t)(m | 1) + 3) & ~(size_t)3;
  const size_t m4 = (size_t)((m + 3) & ~3);
  return 4 * ((size_t)ke * small_ldq(ke) + al + 2 * m4 + (size_t)((n + 31) / 32));
}
constexpr int kWaves = kBlock / 64;

struct InstState {
  float sigma, lr, eps;
  int step;
  int done;        // 1: the instance has nothing more to do (y == 0)
  int cg_done;     // 1: refinement converged
  float gamma[2];  // CGLS ||A_S^T r||^2, ping-pong by iteration parity
  float gamma0;
  int stop;        // 1: the paper-mode loop ended early (max |c| = 0 or non-finite)
  unsigned sel_bits;   // IHT: magnitude bits of the last top-K threshold (a search hint)
  int pad[5];
};

struct Inst {
  const void* A;       // bulk matrix (float or bf16 bits), column-major
  const float* Am;     // FP32 master (== A for FP32 bulk)
  const float* y;
  float* x;
  int* support;
  int* nsel;
  double* rnorm;
  unsigned* status;
  long long lda, ldam;
  int n, m, k, k_eff;
  int ldg, m_pad, n_rowtiles, cg_slot;   // cg_slot: index in the refinement list
  float* r;
  float* G;
  float* b;
  float* s;
  float* mo;
  float* ve;
  float* xf;
  float* Linv;
  float* z;
  float* cg;           // r0[m_pad] r1[m_pad] q[m_pad] p0[k] p1[k] sv[k]
  float* c0;           // [ldh] A^T y (correlation-update schedule)
  float* dg;           // [ldh] ||a_j||^2 (correlation-update schedule)
  float* H;            // [ldh * k_eff] columns A^T a_{S_l} (correlation-update schedule)
  const float* Gf;     // shared dictionary: [ldh * ldh] full Gram A^T A of the batch's one
                       // matrix (column j = A^T a_j); H is then not stored
  long long ldh;
  int nslice;          // IHT: slices of m in the gradient scan (>= 1)
  float tvw;           // 2w/n for the total-variation prior of weight w (0: none)
  unsigned spin;       // bounded device waits: polls before the watchdog bit is set
  int col;             // image mode: the instance's position in the call (its column)
  unsigned long long* team;   // [2*k_eff + 2*kTeamMax] tagged words exchanged by a team
                              // (correlation-update schedule; zeroed at solve start)
  float* gbuf;         // IHT: [nslice * ldh] per-slice partial dots; g = A^T r of the
                       // current iteration in the first ldh entries
  float* sfull;        // IHT, paper mode: [ldh] dense coefficients (zero off the support)
  float* mden;         // paper mode: [ldh] dense Adam first moments
  float* vden;         // paper mode: [ldh] dense Adam second moments
  double* npart;       // [n_rowtiles] FP64 residual-norm partial sums
  float* qpart;        // [n_rowtiles] CGLS ||q||^2 partial sums
  unsigned long long* key;
  unsigned* bitmap;
  InstState* st;
};

// Total-variation prior (Eq. (5)) on x = D s with D the orthonormal DCT-II
// synthesis basis: that basis diagonalises the neighbour-difference operator,
// so TV(D s) = (1/n) sum_j 4 sin^2(pi j / (2n)) s_j^2 and the prior adds
// (2w/n) * 4 sin^2(pi j / (2n)) to the Gram diagonal of atom j.
__device__ inline float tv_diag(const Inst& I, int j) {
  if (I.tvw == 0.f) return 0.f;
  const float sn = sinf(1.5707963267948966f * (float)j / (float)I.n);
  return I.tvw * 4.f * sn * sn;
}

// Column l of H = A^T a_{S_l} (valid rows 0..n-1, padded to ldh): stored per
// signal, or column S_l of the shared full Gram matrix.
__device__ inline const float* hcol(const Inst& I, int l) {
  return I.Gf ? I.Gf + (long long)I.support[l] * I.ldh : I.H + (long long)l * I.ldh;
}

// A scan tile: atoms [j0, j1) of instance `inst`.
struct ScanTile {
  int inst, j0, j1, pad;
};

// A row tile: rows [i0, i1) (at most 64) of instance `inst`.
struct RowTile {
  int inst, i0, i1, tile;
};

enum : unsigned {
  ST_NAN = 1u, ST_K_CAPPED = 2u, ST_ZERO_Y = 4u, ST_REFINE_INACCURATE = 8u,
  ST_WATCHDOG = 32u
};

// ---- global-memory views of device pointers ---------------------------------
// Pointers read from the descriptors are generic, so loads through them become
// flat loads, which also count against the LDS wait counter: a wait for an LDS
// read then drains every memory load in flight.  Loads through these views are
// global loads, waited for on their own counter.
typedef float gvf4 __attribute__((ext_vector_type(4)));
typedef unsigned gvu2 __attribute__((ext_vector_type(2)));
typedef unsigned gvu4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) const T* gmem(const T* p) {
  return (__attribute__((address_space(1))) const T*)p;
}
// 16 bytes (p 16-byte aligned)
template <typename T>
__device__ __forceinline__ uint4 gload16(const T* p) {
  const gvu4 q = *(__attribute__((address_space(1))) const gvu4*)gmem(p);
  return make_uint4(q.x, q.y, q.z, q.w);
}

// four consecutive elements as float (p 16-byte aligned for float, 8 for bf16)
__device__ __forceinline__ float4 gload4(const float* p) {
  const gvf4 q = *(__attribute__((address_space(1))) const gvf4*)gmem(p);
  return make_float4(q.x, q.y, q.z, q.w);
}
__device__ __forceinline__ float4 gload4(const uint16_t* p) {
  const gvu2 q = *(__attribute__((address_space(1))) const gvu2*)gmem(p);
  return make_float4(__uint_as_float(q.x << 16), __uint_as_float(q.x & 0xffff0000u),
                     __uint_as_float(q.y << 16), __uint_as_float(q.y & 0xffff0000u));
}

// ---- vector loads of the bulk matrix: 16 bytes per lane per load ----------
template <typename TA> struct Vec;

template <> struct Vec<float> {
  static constexpr int W = 4;
  __device__ static inline void load(const float* p, float v[4]) {
    const gvf4 q = *(__attribute__((address_space(1))) const gvf4*)gmem(p);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
  __device__ static inline float one(const float* p) { return *gmem(p); }
};

template <> struct Vec<uint16_t> {   // bfloat16 bit patterns
  static constexpr int W = 8;
  __device__ static inline void load(const uint16_t* p, float v[8]) {
    const uint4 q = gload16(p);
    v[0] = __uint_as_float(q.x << 16); v[1] = __uint_as_float(q.x & 0xffff0000u);
    v[2] = __uint_as_float(q.y << 16); v[3] = __uint_as_float(q.y & 0xffff0000u);
    v[4] = __uint_as_float(q.z << 16); v[5] = __uint_as_float(q.z & 0xffff0000u);
    v[6] = __uint_as_float(q.w << 16); v[7] = __uint_as_float(q.w & 0xffff0000u);
  }
  __device__ static inline float one(const uint16_t* p) {
    return __uint_as_float(((unsigned)*gmem(p)) << 16);
  }
};

// ---- argmax key: (bits of |c|) << 32 | (0xFFFFFFFF - j) ---------------------
// Non-negative floats order like their bit patterns, NaN (sign cleared) ranks
// above +Inf, and the low word makes the lowest index win among equal |c|.
__device__ inline unsigned long long pack_key(float c, int j) {
  const unsigned a = __float_as_uint(c) & 0x7fffffffu;
  return ((unsigned long long)a << 32) | (unsigned long long)(0xffffffffu - (unsigned)j);
}
__device__ inline int key_index(unsigned long long key) {
  return (int)(0xffffffffu - (unsigned)(key & 0xffffffffull));
}
__device__ inline float key_value(unsigned long long key) {
  return __uint_as_float((unsigned)(key >> 32));
}

template <int W>
__device__ inline float group_sum(float v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}

__device__ inline unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long u = __shfl_xor(v, o, 64);
    v = u > v ? u : v;
  }
  return v;
}

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Orders one wavefront's LDS writes before its later reads by other lanes.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide float sum in a fixed order (deterministic).  `red` holds kWaves
// floats of shared memory.  Every thread returns the total.
__device__ inline float block_sum(float v, float* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  float t = 0.f;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) t += red[i];
  return t;
}

}  // namespace clomp
