// Loss and gradient of the coefficient fit 1/2 ||A(mask*x) - y||^2 (the
// residual loss of the coefficients-learning framework behind a masked fully
// connected layer with fixed weights A; Methods, "General idea of coefficients
// learning").  Three deterministic launches (fixed-order reductions):
//   fwd_partial  per (64-row tile, column chunk): sum_j A[i, j] mask_j x_j
//   fwd_final    u_i = sum over chunks - y_i; per-tile partial of sum u_i^2
//   bwd          grad_j = mask_j * (a_j^T u) * g;  loss = 1/2 sum of partials
// Instantiated for float and double (double serves gradient checking).

#include <mutex>

#include "dev_common.h"
#include "kernels.h"

// Scratch of the allocation-free gradient entry point: the column-chunk
// partials, the residual when the caller passes none, and the loss partials.
// One copy per device, resident until the process ends; host code reaches it
// only through the address resolved per device by grad_scratch_init.
static __device__ __align__(256) unsigned char scratch[clomp::kGradScratchBytes];

namespace clomp {

template <typename T>
__global__ __launch_bounds__(kBlock) void grad_fwd_partial(int n, int m, long long lda,
                                                           const T* __restrict__ A,
                                                           const T* __restrict__ x,
                                                           const unsigned char* __restrict__ mask,
                                                           T* __restrict__ part, int colchunk,
                                                           int nrowtiles) {
  __shared__ T red[kBlock];
  const int rtile = blockIdx.x % nrowtiles;
  const int chunk = blockIdx.x / nrowtiles;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int i = rtile * 64 + lane;
  const int c0 = chunk * colchunk;
  const int c1 = min(n, c0 + colchunk);
  T acc = 0;
  if (i < m) {
    for (int j = c0 + w; j < c1; j += kWaves) {
      if (mask[j]) acc += A[(long long)j * lda + i] * x[j];
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (w == 0 && i < m) {
    part[(long long)chunk * m + i] = (red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane]);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void grad_fwd_final(int m, const T* __restrict__ part,
                                                         int nchunk, const T* __restrict__ y,
                                                         T* __restrict__ u,
                                                         T* __restrict__ lpart) {
  __shared__ T red[kBlock];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  T v = 0;
  if (i < m) {
    T s = 0;
    for (int c = 0; c < nchunk; ++c) s += part[(long long)c * m + i];
    v = s - y[i];
    u[i] = v;
  }
  red[threadIdx.x] = v * v;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void grad_bwd(int n, int m, long long lda,
                                                   const T* __restrict__ A,
                                                   const unsigned char* __restrict__ mask,
                                                   const T* __restrict__ u,
                                                   const T* __restrict__ grad_out,
                                                   T* __restrict__ grad_x,
                                                   const T* __restrict__ lpart, int nlpart,
                                                   T* __restrict__ loss) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int j = blockIdx.x * kWaves + w;
  const T g = grad_out ? *grad_out : (T)1;
  if (j < n) {
    T acc = 0;
    if (mask[j]) {
      for (int i = lane; i < m; i += 64) acc += A[(long long)j * lda + i] * u[i];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) grad_x[j] = mask[j] ? acc * g : (T)0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    T s = 0;
    for (int b = 0; b < nlpart; ++b) s += lpart[b];
    *loss = (T)0.5 * s;
  }
}

template <typename T>
static hipError_t grad_impl(int n, int m, long long lda, const void* A, const void* x,
                            const unsigned char* mask, const void* y, const void* grad_out,
                            void* grad_x, void* resid_out, void* loss, void* work,
                            int ncolchunk, int colchunk, hipStream_t s) {
  T* part = reinterpret_cast<T*>(work);
  T* u = resid_out ? reinterpret_cast<T*>(resid_out) : part + (long long)ncolchunk * m;
  T* lpart = part + (long long)ncolchunk * m + m;
  const int nrowtiles = (m + 63) / 64;
  const int nfin = (m + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(grad_fwd_partial<T>, dim3(nrowtiles * ncolchunk), dim3(kBlock), 0, s, n, m,
                     lda, (const T*)A, (const T*)x, mask, part, colchunk, nrowtiles);
  hipLaunchKernelGGL(grad_fwd_final<T>, dim3(nfin), dim3(kBlock), 0, s, m, (const T*)part,
                     ncolchunk, (const T*)y, u, lpart);
  hipLaunchKernelGGL(grad_bwd<T>, dim3((n + kWaves - 1) / kWaves), dim3(kBlock), 0, s, n, m, lda,
                     (const T*)A, mask, (const T*)u, (const T*)grad_out, (T*)grad_x,
                     (const T*)lpart, nfin, (T*)loss);
  return hipGetLastError();
}

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t grad_scratch_init(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

void* grad_scratch_ptr(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

hipError_t launch_grad(int f64, int n, int m, long long lda, const void* A, const void* x,
                       const unsigned char* mask, const void* y, const void* grad_out,
                       void* grad_x, void* resid_out, void* loss, void* work, int ncolchunk,
                       int colchunk, hipStream_t s) {
  if (f64)
    return grad_impl<double>(n, m, lda, A, x, mask, y, grad_out, grad_x, resid_out, loss, work,
                             ncolchunk, colchunk, s);
  return grad_impl<float>(n, m, lda, A, x, mask, y, grad_out, grad_x, resid_out, loss, work,
                          ncolchunk, colchunk, s);
}

}  // namespace clomp
