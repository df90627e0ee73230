// pwfs_loop.hip -- the two kernels of the closed loop that are not products
// or the sensor itself (the loop of the paper's SOUL configuration,
// Appendix B: atmosphere -> mirror -> pyramid -> Modalrec -> Integrator with
// a two-step delay, closed through the delayed connection of Section 2.1):
//
//  * k_layers: frozen-flow atmosphere, OPD(x, y, t) = sum_l w_l S_l(x + ox_l +
//    vx_l t, y + oy_l + vy_l t), periodic bilinear sampling, coordinates in
//    float64 so long runs do not lose the sub-pixel position;
//  * k_integrator: c(t) = ff * c(t-1) + g * m(t) per mode, a ring buffer of
//    the last delay + 1 outputs, and the command the mirror applies at the
//    next step, c(t + 1 - delay).
//
// The time index lives in device memory (int64) and the integrator advances
// it, so a captured timestep replays with no host argument changing.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "pwfs.h"
#include "pwfs_internal.hpp"

namespace pwfs {
namespace {

constexpr int kMaxLayers = 16;

struct LayerArgs {
  const float* screens;      // [n_layers][rows][cols]
  int n_layers, rows, cols, D;
  double w[kMaxLayers], ox[kMaxLayers], oy[kMaxLayers], vx[kMaxLayers], vy[kMaxLayers];
  const long long* step;
  float* opd;                // [D][D]
};

__global__ __launch_bounds__(256) void k_layers(LayerArgs p) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= p.D * p.D) return;
  const double t = (double)*p.step;
  const int y = i / p.D, x = i % p.D;
  double acc = 0.0;
  for (int l = 0; l < p.n_layers; ++l) {
    const double X = (double)x + p.ox[l] + p.vx[l] * t;
    const double Y = (double)y + p.oy[l] + p.vy[l] * t;
    const double x0 = floor(X), y0 = floor(Y);
    const double fx = X - x0, fy = Y - y0;
    long long i0 = (long long)x0 % p.cols, j0 = (long long)y0 % p.rows;
    if (i0 < 0) i0 += p.cols;
    if (j0 < 0) j0 += p.rows;
    const long long i1 = (i0 + 1) % p.cols, j1 = (j0 + 1) % p.rows;
    const float* S = p.screens + (size_t)l * p.rows * p.cols;
    const double s00 = S[j0 * p.cols + i0], s01 = S[j0 * p.cols + i1];
    const double s10 = S[j1 * p.cols + i0], s11 = S[j1 * p.cols + i1];
    const double top = (1.0 - fx) * s00 + fx * s01;
    const double bot = (1.0 - fx) * s10 + fx * s11;
    acc += p.w[l] * ((1.0 - fy) * top + fy * bot);
  }
  p.opd[i] = (float)acc;
}

struct IntegratorArgs {
  const float* modes;        // m(t) [n]
  const float* gain;         // [n]
  const float* ff;           // [n]
  float* hist;               // [delay + 1][n], slot t mod (delay + 1) = c(t)
  float* applied;            // [n] <- c(t + 1 - delay)
  long long* step;
  int n, delay;
};

// one workgroup: every lane reads the step before lane 0 advances it
__global__ __launch_bounds__(1024) void k_integrator(IntegratorArgs p) {
  const long long t = *p.step;
  const int D1 = p.delay + 1;
  const int cur = (int)(t % D1), prev = (int)((t + D1 - 1) % D1);
  const int nxt = (int)((t + 1 + D1 - p.delay) % D1);
  for (int j = threadIdx.x; j < p.n; j += blockDim.x) {
    const float c_prev = (t > 0) ? p.hist[(size_t)prev * p.n + j] : 0.f;
    const float c = p.ff[j] * c_prev + p.gain[j] * p.modes[j];
    p.hist[(size_t)cur * p.n + j] = c;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < p.n; j += blockDim.x)
    p.applied[j] = (t + 1 >= p.delay) ? p.hist[(size_t)nxt * p.n + j] : 0.f;
  __syncthreads();
  if (threadIdx.x == 0) *p.step = t + 1;
}

// y[M] = alpha * A[M][K] x[K] + beta * y (y not read when beta == 0), fp32.
// TPR threads per row (64: one wavefront, 256: the whole workgroup); each
// thread strides the row by TPR (coalesced; 16-byte loads when VEC), then a
// fixed-order tree sum.
template <int TPR, bool VEC>
__global__ __launch_bounds__(256) void k_gemv(const float* A, long long lda, const float* x, float* y, int M, int K,
                                              float alpha, float beta) {
  __shared__ float s_red[256];
  const int rows_per = 256 / TPR;
  const int row = blockIdx.x * rows_per + threadIdx.x / TPR;
  const int lane = threadIdx.x % TPR;
  float acc = 0.f;
  if (row < M) {
    const float* a = A + (long long)row * lda;
    if (VEC) {   // 16-byte loads: K and lda multiples of 4, A and x 16-byte aligned
      const float4* a4 = (const float4*)a;
      const float4* x4 = (const float4*)x;
      for (int k = lane; k < K / 4; k += TPR) {
        const float4 av = a4[k], xv = x4[k];
        acc = fmaf(av.x, xv.x, acc);
        acc = fmaf(av.y, xv.y, acc);
        acc = fmaf(av.z, xv.z, acc);
        acc = fmaf(av.w, xv.w, acc);
      }
    } else {
      for (int k = lane; k < K; k += TPR) acc = fmaf(a[k], x[k], acc);
    }
  }
  s_red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = TPR / 2; w > 0; w >>= 1) {
    if (lane < w) s_red[threadIdx.x] += s_red[threadIdx.x + w];
    __syncthreads();
  }
  if (lane == 0 && row < M) {
    const float v = alpha * s_red[threadIdx.x];
    y[row] = (beta != 0.f) ? v + beta * y[row] : v;
  }
}

int lfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  set_last_error(buf);
  return code;
}

}  // namespace
}  // namespace pwfs

using namespace pwfs;

extern "C" int pwfs_layers(const float* screens, int n_layers, int rows, int cols, const pwfs_layer* layers, int D,
                           const long long* step, float* opd, void* stream) {
  if (!screens || !layers || !step || !opd) return lfail(PWFS_EINVAL, "NULL argument");
  if (n_layers < 1 || n_layers > kMaxLayers) return lfail(PWFS_EINVAL, "n_layers must be in [1, 16]");
  if (rows < 2 || cols < 2 || D < 1) return lfail(PWFS_EINVAL, "bad screen or pupil size");
  LayerArgs a{};
  a.screens = screens;
  a.n_layers = n_layers;
  a.rows = rows;
  a.cols = cols;
  a.D = D;
  for (int l = 0; l < n_layers; ++l) {
    const pwfs_layer& L = layers[l];
    if (!std::isfinite(L.weight) || !std::isfinite(L.origin_x) || !std::isfinite(L.origin_y) ||
        !std::isfinite(L.vel_x) || !std::isfinite(L.vel_y))
      return lfail(PWFS_EINVAL, "layer %d has a non-finite parameter", l);
    a.w[l] = L.weight;
    a.ox[l] = L.origin_x;
    a.oy[l] = L.origin_y;
    a.vx[l] = L.vel_x;
    a.vy[l] = L.vel_y;
  }
  a.step = step;
  a.opd = opd;
  hipLaunchKernelGGL(k_layers, dim3((unsigned)((D * D + 255) / 256)), dim3(256), 0, (hipStream_t)stream, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return lfail(PWFS_EHIP, "launch k_layers: %s", hipGetErrorString(e));
  return PWFS_OK;
}

extern "C" int pwfs_integrator(const float* modes, const float* gain, const float* ff, int n_modes, int delay,
                               float* hist, float* applied, long long* step, void* stream) {
  if (!modes || !gain || !ff || !hist || !applied || !step) return lfail(PWFS_EINVAL, "NULL argument");
  if (n_modes < 1 || delay < 1 || delay > 64) return lfail(PWFS_EINVAL, "n_modes >= 1 and delay in [1, 64]");
  IntegratorArgs a{modes, gain, ff, hist, applied, step, n_modes, delay};
  hipLaunchKernelGGL(k_integrator, dim3(1), dim3(1024), 0, (hipStream_t)stream, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return lfail(PWFS_EHIP, "launch k_integrator: %s", hipGetErrorString(e));
  return PWFS_OK;
}

extern "C" int pwfs_gemv(const float* A, long long lda, const float* x, float* y, int M, int K, float alpha,
                         float beta, void* stream) {
  if (!A || !x || !y) return lfail(PWFS_EINVAL, "NULL device pointer");
  if (M < 1 || K < 1 || lda < K) return lfail(PWFS_EINVAL, "bad sizes (M, K >= 1, lda >= K)");
  hipStream_t st = (hipStream_t)stream;
  const bool vec = K % 4 == 0 && lda % 4 == 0 && ((uintptr_t)A & 15) == 0 && ((uintptr_t)x & 15) == 0;
  const dim3 wide((unsigned)M), narrow((unsigned)((M + 3) / 4));
  if (K >= 1024) {
    if (vec)
      hipLaunchKernelGGL((k_gemv<256, true>), wide, dim3(256), 0, st, A, lda, x, y, M, K, alpha, beta);
    else
      hipLaunchKernelGGL((k_gemv<256, false>), wide, dim3(256), 0, st, A, lda, x, y, M, K, alpha, beta);
  } else {
    if (vec)
      hipLaunchKernelGGL((k_gemv<64, true>), narrow, dim3(256), 0, st, A, lda, x, y, M, K, alpha, beta);
    else
      hipLaunchKernelGGL((k_gemv<64, false>), narrow, dim3(256), 0, st, A, lda, x, y, M, K, alpha, beta);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return lfail(PWFS_EHIP, "launch k_gemv: %s", hipGetErrorString(e));
  return PWFS_OK;
}
