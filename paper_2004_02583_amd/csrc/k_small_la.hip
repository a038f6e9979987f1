// Reductions of per-workgroup partial sums (fixed order, FP64) and small
// element-wise helpers of the host runtime.
#include <algorithm>

#include "tk_kernels.h"

namespace tk {

// ---------------------------------------------------------------------------
// Fixed-order FP64 reduction of `parts` partial arrays of length n:
// out[e] = sum_{w=0}^{parts-1} in[w*stride + e].  Deterministic.
template <typename T>
__global__ void __launch_bounds__(256) k_reduce_parts(const T* __restrict__ in,
                                                      int parts, int64_t n,
                                                      int64_t stride,
                                                      double* __restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double s = 0.0;
  for (int w = 0; w < parts; ++w) s += (double)in[(int64_t)w * stride + e];
  out[e] = s;
}

// First stage of the two-stage reduction: a block covers 64 consecutive
// outputs (lanes, coalesced) and 4 of the G = 4 * gridDim.y part groups
// (waves); group g sums parts g, g + G, g + 2G, ... and the block adds its
// four groups in a fixed order into out[blockIdx.y * n + e].
template <typename T>
__global__ void __launch_bounds__(256) k_reduce_groups(const T* __restrict__ in, int parts,
                                                       int64_t n, int64_t stride,
                                                       double* __restrict__ out) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + lane;
  const int G = 4 * (int)gridDim.y;
  double s = 0.0;
  if (e < n)
    for (int p = (int)blockIdx.y * 4 + wv; p < parts; p += G) s += (double)in[(int64_t)p * stride + e];
  red[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && e < n)
    out[(int64_t)blockIdx.y * n + e] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Identity factor (R_n == I_n) in element type T.
template <typename T>
__global__ void k_identity(T* __restrict__ U, int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n * n) U[e] = Store<T>::cvt((e / n == e % n) ? 1.0 : 0.0);
}

// Element-type conversion of an FP64 array.
template <typename T>
__global__ void k_convert(const double* __restrict__ in, int64_t n, T* __restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = Store<T>::cvt(in[e]);
}

template <typename T>
__global__ void k_widen(const T* __restrict__ in, int64_t n, double* __restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = (double)in[e];
}

// Rounds FP32 values to BF16 precision (round to nearest even), in place.
__global__ void k_round_bf16(float* __restrict__ x, int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] = bf16_to_f32(f32_to_bf16(x[e]));
}

// ---------------------------------------------------------------------------
// host launchers

void launch_round_bf16(float* x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_round_bf16, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, x, n);
}

template <typename T>
void launch_reduce_parts(const T* in, int parts, int64_t n, int64_t stride, double* out,
                         double* tmp, hipStream_t s) {
  // about 8 parts per thread in the first stage, at most REDUCE_GROUPS / 4
  // group blocks (their sums go to tmp, REDUCE_GROUPS / 4 * n doubles)
  int gy = (int)std::min<int64_t>(REDUCE_GROUPS / 4, std::max<int64_t>(1, ceil_div(parts, 32)));
  if (!tmp) gy = 1;
  dim3 grid((unsigned)ceil_div(n, 64), (unsigned)gy);
  hipLaunchKernelGGL(k_reduce_groups<T>, grid, dim3(256), 0, s, in, parts, n, stride,
                     gy == 1 ? out : tmp);
  if (gy > 1)
    hipLaunchKernelGGL(k_reduce_parts<double>, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0,
                       s, (const double*)tmp, gy, n, n, out);
}
template void launch_reduce_parts<float>(const float*, int, int64_t, int64_t, double*,
                                         double*, hipStream_t);
template void launch_reduce_parts<double>(const double*, int, int64_t, int64_t, double*,
                                          double*, hipStream_t);

template <typename T>
void launch_identity(T* U, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_identity<T>, dim3((unsigned)ceil_div(n * n, 256)), dim3(256), 0, s,
                     U, n);
}
template void launch_identity<double>(double*, int64_t, hipStream_t);
template void launch_identity<float>(float*, int64_t, hipStream_t);

template <typename T>
void launch_convert(const double* in, int64_t n, T* out, hipStream_t s) {
  hipLaunchKernelGGL(k_convert<T>, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, in,
                     n, out);
}
template void launch_convert<double>(const double*, int64_t, double*, hipStream_t);
template void launch_convert<float>(const double*, int64_t, float*, hipStream_t);

template <typename T>
void launch_widen(const T* in, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_widen<T>, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, in, n, out);
}
template void launch_widen<double>(const double*, int64_t, double*, hipStream_t);
template void launch_widen<float>(const float*, int64_t, double*, hipStream_t);

}  // namespace tk
