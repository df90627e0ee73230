// pwfs_mlp.hip -- matrix-core GEMM entry point and the surrogate network
// (fully connected layers with exact GELU, MSE loss, Adam) for gfx950.
//
// Every product is the "NT" tile engine of mfma_gemm.hpp on bf16 operands
// (one plane: bf16 weights and activations, fp32 accumulation) or on bf16
// hi/lo pairs (three products, ~fp32 accuracy).  Layer l maps P_l -> P_{l+1}
// features (sizes rounded up to 32, padding kept at zero).  Per layer the
// network keeps: fp32 master W [P_{l+1}][P_l] and b, Adam moments, fp32
// gradients, and 16-bit copies of W (rows = outputs) and W^T (rows =
// inputs) so that both the forward product (A W^T) and the backward data
// product (dZ W) read K-contiguous operands.  Activations are stored twice
// by the epilogue that produces them: [batch][features] for the next
// forward product and [features][batch] for the weight-gradient product
// dW = dZ^T A, whose K is the batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mfma_gemm.hpp"
#include "pwfs.h"
#include "pwfs_internal.hpp"

namespace pwfs {
namespace {

int mfail(int code, const char* fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  set_last_error(msg);
  return code;
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }
int up32(int x) { return (x + 31) / 32 * 32; }

enum Epi { E_STORE = 0, E_HIDDEN = 1, E_OUTPUT = 2, E_DHIDDEN = 3 };

struct GemmArgs {
  const uint16_t* a;
  const uint16_t* b;
  long long a_plane, b_plane, lda, ldb;
  int M, N, K, mtiles, ntiles;
  float alpha, beta;      // E_STORE: c = alpha * acc + beta * c (c is not read when beta == 0)
  float* c;               // fp32 output [M][ldc] (E_STORE, E_OUTPUT)
  long long ldc;
  const float* bias;      // [N]
  float* z;               // fp32 pre-activation (E_HIDDEN) or gradient (E_OUTPUT, E_DHIDDEN) [M][ldz]
  long long ldz;
  uint16_t* h;            // 16-bit planes [M][ldh]
  long long h_plane, ldh;
  uint16_t* ht;           // 16-bit planes [N][ldht]
  long long ht_plane, ldht;
  const float* target;    // [M][ldt] (E_OUTPUT with loss)
  long long ldt;
  float tscale, gscale;
  const float* zprev;     // [M][ldzp] (E_DHIDDEN)
  long long ldzp;
  double* loss_part;      // [grid] (E_OUTPUT with loss)
  int planes_out;
  // optional second K segment accumulated into the same tile before the
  // epilogue: acc += A2[M][K2] B2[N][K2]^T (K2 = 0: none)
  const uint16_t* a2;
  const uint16_t* b2;
  long long a2_plane, b2_plane, lda2, ldb2;
  int K2;
};

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * __expf(-0.5f * x * x);
}

__device__ __forceinline__ void put16(uint16_t* base, long long plane, long long off, float v, int planes) {
  if (planes == 2) {
    uint16_t hi, lo;
    split16<false>(v, hi, lo);
    base[off] = hi;
    base[plane + off] = lo;
  } else {
    base[off] = f32_to_bf16_rne(v);
  }
}

// the epilogue of one output element (m, n) of a product whose accumulated
// value is v; lsum collects the squared error (E_OUTPUT with a target)
template <int EPI>
__device__ __forceinline__ void gemm_epilogue(const GemmArgs& p, int m, int n, float v, double& lsum) {
  if constexpr (EPI == E_STORE) {
    float* cp = p.c + (long long)m * p.ldc + n;
    *cp = (p.beta != 0.f) ? p.alpha * v + p.beta * *cp : p.alpha * v;
  } else if constexpr (EPI == E_HIDDEN) {
    const float zz = v + p.bias[n];
    const float hv = gelu_f(zz);
    put16(p.h, p.h_plane, (long long)m * p.ldh + n, hv, p.planes_out);
    // the pre-activation and the transposed copy serve the backward
    // pass only (absent in inference)
    if (p.z) p.z[(long long)m * p.ldz + n] = zz;
    if (p.ht) put16(p.ht, p.ht_plane, (long long)n * p.ldht + m, hv, p.planes_out);
  } else if constexpr (EPI == E_OUTPUT) {
    const float y = v + p.bias[n];
    if (p.c) p.c[(long long)m * p.ldc + n] = p.alpha * y;
    if (p.target) {
      const float d = y - p.target[(long long)m * p.ldt + n] * p.tscale;
      lsum += (double)d * d;
      const float g = p.gscale * d;
      p.z[(long long)m * p.ldz + n] = g;
      put16(p.h, p.h_plane, (long long)m * p.ldh + n, g, p.planes_out);
      put16(p.ht, p.ht_plane, (long long)n * p.ldht + m, g, p.planes_out);
    }
  } else {  // E_DHIDDEN
    const float g = v * gelu_grad_f(p.zprev[(long long)m * p.ldzp + n]);
    p.z[(long long)m * p.ldz + n] = g;
    put16(p.h, p.h_plane, (long long)m * p.ldh + n, g, p.planes_out);
    put16(p.ht, p.ht_plane, (long long)n * p.ldht + m, g, p.planes_out);
  }
}

template <int NPL, int EPI, int BK>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs p) {
  extern __shared__ u32x4_t lds_raw[];
  uint16_t* lds = (uint16_t*)lds_raw;
  using E = MfmaTile<NPL, false, BK>;
  const int tid = threadIdx.x;
  const int nt = blockIdx.x % p.ntiles;
  const int mt = blockIdx.x / p.ntiles;
  const int m0 = mt * kGemmTile, n0 = nt * kGemmTile;
  typename E::Ops ops;
#pragma unroll
  for (int pl = 0; pl < NPL; ++pl) {
    ops.a[pl] = p.a + pl * p.a_plane + (long long)m0 * p.lda;
    ops.b[pl] = p.b + pl * p.b_plane + (long long)n0 * p.ldb;
  }
  E eng;
  eng.zero();
  eng.run(ops, p.lda, p.M - m0, p.ldb, p.N - n0, p.K, lds, tid);
  if (p.K2 > 0) {
    typename E::Ops ops2;
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl) {
      ops2.a[pl] = p.a2 + pl * p.a2_plane + (long long)m0 * p.lda2;
      ops2.b[pl] = p.b2 + pl * p.b2_plane + (long long)n0 * p.ldb2;
    }
    eng.run(ops2, p.lda2, p.M - m0, p.ldb2, p.N - n0, p.K2, lds, tid);
  }
  double lsum = 0.0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        int row, col;
        E::coord(tid, i, j, e, row, col);
        const int m = m0 + row, n = n0 + col;
        if (m >= p.M || n >= p.N) continue;
        gemm_epilogue<EPI>(p, m, n, eng.value(i, j, e), lsum);
      }
  if constexpr (EPI == E_OUTPUT) {
    if (p.loss_part) {
      __shared__ double red[256];
      red[tid] = lsum;
      __syncthreads();
      for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
      }
      if (tid == 0) p.loss_part[blockIdx.x] = red[0];
    }
  }
}

// Large one-plane products (inference passes of the network, big plain
// GEMMs): the wave-specialised workgroup of mfma_gemm.hpp, a 128 x BN tile
// per workgroup with two K steps of operands in flight.  The K segments run
// as one stream of steps (the second segment's after the first's), and the
// consumers' products are those of k_gemm in the same order, so both give
// the same bits.  No loss partials (the product has no target).
constexpr int kGemmWsDepth = 2;

template <int EPI, int BN>
__global__ __launch_bounds__(64 * (2 * BN / 64 + 4)) void k_gemm_ws(GemmArgs p) {
  extern __shared__ u32x4_t lds_raw[];
  uint16_t* lds = (uint16_t*)lds_raw;
  using E = WsEngine<1, false, BN>;
  using W = WsParts<E, BN>;
  constexpr int NC = 2 * BN / 64, BK = E::BK_, CH = W::CH;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nt = blockIdx.x % p.ntiles;
  const int mt = blockIdx.x / p.ntiles;
  const int m0 = mt * kGemmTile, n0 = nt * BN;
  const int nk1 = p.K / BK;
  const int steps = nk1 + p.K2 / BK;

  if (wave >= NC) {
    const int pt = tid - 64 * NC;
    long long off1[CH], off2[CH];   // element offset of chunk h in segment 1 and 2 (K step 0)
    int loff[CH];
#pragma unroll
    for (int h = 0; h < CH; ++h) {
      const int row = W::row(pt, h), kq = W::kq(pt, h);
      if (W::is_a(h)) {
        const long long r = min(m0 + row, p.M - 1);
        off1[h] = r * p.lda + kq;
        off2[h] = r * p.lda2 + kq;
      } else {
        const long long r = min(n0 + row, p.N - 1);
        off1[h] = r * p.ldb + kq;
        off2[h] = r * p.ldb2 + kq;
      }
      loff[h] = W::lds_offset(pt, h);
    }
    ws_produce<E, kGemmWsDepth>(lds, loff, steps, [&](u32x4_t (&b)[CH], int s) {
      const bool seg2 = s >= nk1;
      const long long k0 = (long long)(seg2 ? s - nk1 : s) * BK;
      const uint16_t* A = seg2 ? p.a2 : p.a;
      const uint16_t* B = seg2 ? p.b2 : p.b;
#pragma unroll
      for (int h = 0; h < CH; ++h)
        b[h] = *(const u32x4_t*)((W::is_a(h) ? A : B) + (seg2 ? off2[h] : off1[h]) + k0);
    });
    return;
  }

  // -------------------------------------------------------------- consumer
  const int lane = tid & 63;
  const int wm = wave & 1, wn = wave >> 1;
  E eng;
  eng.zero();
  __syncthreads();
  for (int st = 0; st < steps; ++st) {
    eng.compute(lds + (st & 1) * E::STAGE, wm, wn, lane);
    __syncthreads();
  }
  double lsum = 0.0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        // accumulator layout of the 32 x 32 tile (i, j) of this quarter
        const int m = m0 + wm * 64 + i * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        const int n = n0 + wn * 64 + j * 32 + (lane & 31);
        if (m >= p.M || n >= p.N) continue;
        gemm_epilogue<EPI>(p, m, n, eng.value(i, j, e), lsum);
      }
}

// fp32 [rows][cols] (row stride ld) -> 16-bit planes [rows][Kp], zero padding;
// with `transpose`, planes [cols][ldo] hold the transpose (row index = col)
struct SplitArgs {
  const float* src;
  long long ld;
  uint16_t* dst;
  long long plane, ldo;
  int rows, cols, Kp, planes, transpose;
  float scale;
};

__global__ __launch_bounds__(256) void k_split(SplitArgs p) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long total = (long long)p.rows * p.Kp;
  if (i >= total) return;
  const int r = (int)(i / p.Kp), k = (int)(i % p.Kp);
  const float v = (k < p.cols) ? p.src[(long long)r * p.ld + k] * p.scale : 0.f;
  const long long off = p.transpose ? (long long)k * p.ldo + r : (long long)r * p.ldo + k;
  put16(p.dst, p.plane, off, v, p.planes);
}

// column sums of an fp32 [rows][ld] matrix over its first `rows` rows
__global__ __launch_bounds__(256) void k_colsum(const float* x, long long ld, int rows, int cols, float* out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += x[(long long)r * ld + c];
  out[c] = s;
}

__global__ void k_loss_reduce(const double* part, int n, float scale, float* loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  *loss = (float)(s * scale);
}

struct AdamArgs {
  float* w;        // fp32 master [rows][cols]
  float* m;
  float* v;
  const float* g;
  uint16_t* wq;    // 16-bit planes [rows][cols]    (nullptr for biases)
  uint16_t* wqt;   // 16-bit planes [cols][rows]
  long long plane, plane_t;
  int rows, cols, planes;
  float lr, b1, b2, eps, c1, c2;   // c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
};

__global__ __launch_bounds__(256) void k_adam(AdamArgs p) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long total = (long long)p.rows * p.cols;
  if (i >= total) return;
  const float g = p.g[i];
  const float m = p.b1 * p.m[i] + (1.f - p.b1) * g;
  const float v = p.b2 * p.v[i] + (1.f - p.b2) * g * g;
  p.m[i] = m;
  p.v[i] = v;
  const float w = p.w[i] - p.lr * (m * p.c1) / (sqrtf(v * p.c2) + p.eps);
  p.w[i] = w;
  if (p.wq) {
    const int r = (int)(i / p.cols), c = (int)(i % p.cols);
    put16(p.wq, p.plane, i, w, p.planes);
    put16(p.wqt, p.plane_t, (long long)c * p.rows + r, w, p.planes);
  }
}

// params (packed, unpadded, W as [out][in]) <-> padded master copies
struct ParamCopyArgs {
  const float* src;
  float* dst;
  int rows, cols, src_ld, dst_ld;
};
__global__ __launch_bounds__(256) void k_copy2d(ParamCopyArgs p) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long long)p.rows * p.cols) return;
  const int r = (int)(i / p.cols), c = (int)(i % p.cols);
  p.dst[(long long)r * p.dst_ld + c] = p.src[(long long)r * p.src_ld + c];
}

__global__ __launch_bounds__(256) void k_row_rms(const float* x, long long ld, int rows, int cols, float* out) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  double s = 0.0;
  for (int c = 0; c < cols; ++c) {
    const double v = x[(long long)r * ld + c];
    s += v * v;
  }
  out[r] = (float)sqrt(s / cols);
}

template <int NPL, int EPI, int BK>
int gemm_launch(const GemmArgs& a0, hipStream_t st) {
  GemmArgs a = a0;
  a.mtiles = (a.M + kGemmTile - 1) / kGemmTile;
  a.ntiles = (a.N + kGemmTile - 1) / kGemmTile;
  static bool lds_set = false;
  if (!lds_set) {
    if (hipFuncSetAttribute((const void*)k_gemm<NPL, EPI, BK>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)MfmaTile<NPL, false, BK>::lds_bytes()) != hipSuccess)
      (void)hipGetLastError();
    lds_set = true;
  }
  const size_t lds = MfmaTile<NPL, false, BK>::lds_bytes();
  hipLaunchKernelGGL((k_gemm<NPL, EPI, BK>), dim3((unsigned)(a.mtiles * a.ntiles)), dim3(256), lds, st, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mfail(PWFS_EHIP, "launch k_gemm: %s", hipGetErrorString(e));
  return PWFS_OK;
}

// One-plane products whose K is a multiple of 64 take K steps of 64 (8
// matrix products per wavefront between barriers instead of 4, so load
// latency hides behind them; same products in the same order, same bits).
// Two-plane products keep steps of 32 (their 80 KB stages allow two
// workgroups per CU; 64 would allow one).
template <int EPI, int BN>
int gemm_ws_launch(const GemmArgs& a0, hipStream_t st) {
  GemmArgs a = a0;
  a.mtiles = (a.M + kGemmTile - 1) / kGemmTile;
  a.ntiles = (a.N + BN - 1) / BN;
  const size_t lds = WsEngine<1, false, BN>::lds_bytes();
  static bool lds_set = false;
  if (!lds_set) {
    if (hipFuncSetAttribute((const void*)k_gemm_ws<EPI, BN>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
        hipSuccess)
      (void)hipGetLastError();
    lds_set = true;
  }
  hipLaunchKernelGGL((k_gemm_ws<EPI, BN>), dim3((unsigned)(a.mtiles * a.ntiles)), dim3(64 * (2 * BN / 64 + 4)), lds,
                     st, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mfail(PWFS_EHIP, "launch k_gemm_ws: %s", hipGetErrorString(e));
  return PWFS_OK;
}

// One-plane products with at least two rounds of wave-specialised
// workgroups on the chip (one per CU) and no loss epilogue take the
// wave-specialised tiles: 128 x 256 where that still gives four rounds,
// else 128 x 128.  The rest (training batches, two-plane checks, the loss
// and gradient epilogues) take the 256-lane tiles.
constexpr int kWsMinTiles = 512, kWsWideTiles = 1024;

template <int EPI>
int gemm_dispatch(int planes, const GemmArgs& a, hipStream_t st) {
  if (planes == 2) return gemm_launch<2, EPI, 32>(a, st);
  if (a.K % 64 != 0 || a.K2 % 64 != 0) return gemm_launch<1, EPI, 32>(a, st);
  if constexpr (EPI != E_DHIDDEN) {
    if (EPI != E_OUTPUT || !a.target) {
      const long long mt = (a.M + kGemmTile - 1) / kGemmTile;
      if (mt * ((a.N + 255) / 256) >= kWsWideTiles) return gemm_ws_launch<EPI, 256>(a, st);
      if (mt * ((a.N + 127) / 128) >= kWsMinTiles) return gemm_ws_launch<EPI, 128>(a, st);
    }
  }
  return gemm_launch<1, EPI, 64>(a, st);
}

int split_launch(const float* src, long long ld, int rows, int cols, int Kp, uint16_t* dst, long long plane,
                 long long ldo, int planes, int transpose, float scale, hipStream_t st) {
  SplitArgs s{src, ld, dst, plane, ldo, rows, cols, Kp, planes, transpose, scale};
  const long long total = (long long)rows * Kp;
  hipLaunchKernelGGL(k_split, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mfail(PWFS_EHIP, "launch k_split: %s", hipGetErrorString(e));
  return PWFS_OK;
}

int planes_of(int precision) { return precision == PWFS_BF16X3 ? 2 : 1; }

}  // namespace
}  // namespace pwfs

using namespace pwfs;

// ================================================================ GEMM ABI ==
extern "C" int pwfs_gemm_workspace_size(int M, int N, int K, int precision, size_t* bytes) {
  if (!bytes || M < 1 || N < 1 || K < 1) return mfail(PWFS_EINVAL, "bad GEMM sizes");
  if (precision != PWFS_BF16 && precision != PWFS_BF16X3) return mfail(PWFS_EUNSUPPORTED, "precision");
  const size_t Kp = up32(K), pl = planes_of(precision);
  *bytes = a256(2 * pl * (size_t)M * Kp) + a256(2 * pl * (size_t)N * Kp);
  return PWFS_OK;
}

namespace pwfs {
namespace {

// C = alpha A B^T + beta C with the operand planes in `ws` (>= the
// pwfs_gemm_workspace_size bytes, 256-byte aligned; checked by the callers).
// k_split writes every element of both planes, K padding included, so the
// workspace needs no clearing.
int gemm_run(const float* A, long long lda, const float* B, long long ldb, float* C, long long ldc, int M, int N,
             int K, float alpha, float beta, int precision, void* ws, hipStream_t st) {
  const int Kp = up32(K), pl = planes_of(precision);
  uint16_t* a16 = (uint16_t*)ws;
  uint16_t* b16 = (uint16_t*)((char*)ws + a256(2 * pl * (size_t)M * Kp));
  const long long ap = (long long)M * Kp, bp = (long long)N * Kp;
  int rc;
  if ((rc = split_launch(A, lda, M, K, Kp, a16, ap, Kp, pl, 0, 1.f, st))) return rc;
  if ((rc = split_launch(B, ldb, N, K, Kp, b16, bp, Kp, pl, 0, 1.f, st))) return rc;
  GemmArgs g{};
  g.a = a16;
  g.b = b16;
  g.a_plane = ap;
  g.b_plane = bp;
  g.lda = Kp;
  g.ldb = Kp;
  g.M = M;
  g.N = N;
  g.K = Kp;
  g.alpha = alpha;
  g.beta = beta;
  g.c = C;
  g.ldc = ldc;
  return gemm_dispatch<E_STORE>(pl, g, st);
}

int gemm_args_check(const float* A, long long lda, const float* B, long long ldb, float* C, long long ldc, int M,
                    int N, int K, int precision, size_t* need) {
  int rc = pwfs_gemm_workspace_size(M, N, K, precision, need);
  if (rc) return rc;
  if (!A || !B || !C) return mfail(PWFS_EINVAL, "NULL device pointer");
  if (lda < K || ldb < K || ldc < N) return mfail(PWFS_EINVAL, "leading dimension too small");
  return PWFS_OK;
}

// ------------------------------------------- static scratch of the GEMM ----
// pwfs_gemm_noalloc keeps its operand planes in this file-scope device array
// instead of a caller workspace.  Every GPU the library runs on holds its own
// copy for the life of the process.  In host code the array's name is only a
// stand-in: its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// passed to kernels.
constexpr size_t kGemmScratchBytes = PWFS_GEMM_NOALLOC_MAX_BYTES;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kGemmScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

int scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return mfail(PWFS_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return mfail(PWFS_EUNSUPPORTED, "device index %d >= %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return mfail(PWFS_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    if (!p || ((uintptr_t)p & 255)) return mfail(PWFS_EHIP, "static scratch has no aligned device address");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return PWFS_OK;
}

}  // namespace
}  // namespace pwfs

extern "C" int pwfs_gemm(const float* A, long long lda, const float* B, long long ldb, float* C, long long ldc,
                         int M, int N, int K, float alpha, float beta, int precision, void* ws, size_t ws_bytes,
                         void* stream) {
  size_t need = 0;
  int rc = gemm_args_check(A, lda, B, ldb, C, ldc, M, N, K, precision, &need);
  if (rc) return rc;
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need) return mfail(PWFS_EWORKSPACE, "workspace");
  return gemm_run(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, precision, ws, (hipStream_t)stream);
}

extern "C" int pwfs_gemm_noalloc(const float* A, long long lda, const float* B, long long ldb, float* C,
                                 long long ldc, int M, int N, int K, float alpha, float beta, int precision,
                                 void* stream) {
  size_t need = 0;
  int rc = gemm_args_check(A, lda, B, ldb, C, ldc, M, N, K, precision, &need);
  if (rc) return rc;
  if (need > kGemmScratchBytes)
    return mfail(PWFS_EWORKSPACE, "operand planes need %zu bytes; the static scratch holds %zu", need,
                 kGemmScratchBytes);
  void* ws = nullptr;
  if ((rc = scratch_of_current_device(&ws))) return rc;
  return gemm_run(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, precision, ws, (hipStream_t)stream);
}

extern "C" int pwfs_row_rms(const float* x, long long ld, int rows, int cols, float* out, void* stream) {
  if (!x || !out || rows < 1 || cols < 1 || ld < cols) return mfail(PWFS_EINVAL, "bad arguments");
  hipLaunchKernelGGL(k_row_rms, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, (hipStream_t)stream, x, ld,
                     rows, cols, out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mfail(PWFS_EHIP, "launch k_row_rms: %s", hipGetErrorString(e));
  return PWFS_OK;
}

// ================================================================= MLP ABI ==
struct pwfs_mlp_s {
  int L = 0, Bm = 0, precision = 0, planes = 1;
  long long step = 0;                        // Adam steps taken
  std::vector<int> n, P;                     // true and padded sizes, L + 1 each
  // per layer l (0..L-1)
  std::vector<float*> W, b, mW, vW, mb, vb, gW, gb;
  std::vector<uint16_t*> Wq, Wqt;            // planes [P_{l+1}][P_l], [P_l][P_{l+1}]
  // per layer boundary j (0..L): activation planes and transposes; z, dz fp32
  std::vector<uint16_t*> H, Ht, G, Gt;
  std::vector<float*> Z, dZ;
  float* Y = nullptr;
  // fixed linear term of inference (pwfs_mlp_set_linear): C [P_L][P_0] fp32
  // and its 16-bit planes holding C / c_scale (c_scale = the out_scale they
  // were made for, 0 = stale)
  float* C = nullptr;
  uint16_t* Cq = nullptr;
  bool have_linear = false;
  float c_scale = 0.f;
  double* loss_part = nullptr;
  int loss_parts = 0;
  bool have_grad = false;
};

namespace {

struct MlpLayout {
  size_t total = 0;
  std::vector<size_t> off;
};

// sizes of every region, in order; `cb` is called with each region's bytes
template <class CB>
void mlp_regions(int L, const std::vector<int>& P, int Bm, int planes, CB cb) {
  for (int l = 0; l < L; ++l) {
    const size_t w = (size_t)P[l + 1] * P[l], bb = (size_t)P[l + 1];
    for (int r = 0; r < 4; ++r) cb(4 * w);     // W, mW, vW, gW
    for (int r = 0; r < 4; ++r) cb(4 * bb);    // b, mb, vb, gb
    cb(2 * planes * w);                        // Wq
    cb(2 * planes * w);                        // Wqt
  }
  for (int j = 0; j <= L; ++j) {
    const size_t a = (size_t)Bm * P[j];
    cb(2 * planes * a);  // H
    cb(2 * planes * a);  // Ht
    cb(2 * planes * a);  // G
    cb(2 * planes * a);  // Gt
    cb(4 * a);           // Z
    cb(4 * a);           // dZ
  }
  cb(4 * (size_t)Bm * P[L]);                   // Y
  cb(4 * (size_t)P[L] * P[0]);                 // C
  cb(2 * planes * (size_t)P[L] * P[0]);        // Cq
  const int tiles = ((Bm + 127) / 128) * ((P[L] + 127) / 128);
  cb(8 * (size_t)tiles);                       // loss partials
}

int mlp_check(int L, const int32_t* sizes, int Bm, int precision, std::vector<int>& n, std::vector<int>& P) {
  if (L < 1 || L > 8 || !sizes) return mfail(PWFS_EINVAL, "n_layers must be in [1, 8]");
  if (Bm < 32 || Bm % 32) return mfail(PWFS_EINVAL, "max_batch must be a positive multiple of 32");
  if (precision != PWFS_BF16 && precision != PWFS_BF16X3) return mfail(PWFS_EUNSUPPORTED, "precision");
  n.assign(sizes, sizes + L + 1);
  P.resize(L + 1);
  for (int j = 0; j <= L; ++j) {
    if (n[j] < 1 || n[j] > 65536) return mfail(PWFS_EINVAL, "layer size out of range");
    P[j] = up32(n[j]);
  }
  return PWFS_OK;
}

}  // namespace

extern "C" int pwfs_mlp_workspace_size(int L, const int32_t* sizes, int max_batch, int precision, size_t* bytes) {
  std::vector<int> n, P;
  int rc = mlp_check(L, sizes, max_batch, precision, n, P);
  if (rc) return rc;
  if (!bytes) return mfail(PWFS_EINVAL, "bytes is NULL");
  size_t tot = 0;
  mlp_regions(L, P, max_batch, planes_of(precision), [&](size_t b) { tot += a256(b); });
  *bytes = tot;
  return PWFS_OK;
}

extern "C" int pwfs_mlp_create(int L, const int32_t* sizes, int max_batch, int precision, void* ws, size_t ws_bytes,
                               void* stream, pwfs_mlp_t* out) {
  size_t need = 0;
  int rc = pwfs_mlp_workspace_size(L, sizes, max_batch, precision, &need);
  if (rc) return rc;
  if (!out) return mfail(PWFS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need) return mfail(PWFS_EWORKSPACE, "workspace missing, small or misaligned");
  pwfs_mlp_s* m = new (std::nothrow) pwfs_mlp_s();
  if (!m) return mfail(PWFS_EINVAL, "out of host memory");
  mlp_check(L, sizes, max_batch, precision, m->n, m->P);
  m->L = L;
  m->Bm = max_batch;
  m->precision = precision;
  m->planes = planes_of(precision);
  std::vector<char*> reg;
  size_t off = 0;
  mlp_regions(L, m->P, max_batch, m->planes, [&](size_t b) {
    reg.push_back((char*)ws + off);
    off += a256(b);
  });
  size_t r = 0;
  for (int l = 0; l < L; ++l) {
    m->W.push_back((float*)reg[r++]);
    m->mW.push_back((float*)reg[r++]);
    m->vW.push_back((float*)reg[r++]);
    m->gW.push_back((float*)reg[r++]);
    m->b.push_back((float*)reg[r++]);
    m->mb.push_back((float*)reg[r++]);
    m->vb.push_back((float*)reg[r++]);
    m->gb.push_back((float*)reg[r++]);
    m->Wq.push_back((uint16_t*)reg[r++]);
    m->Wqt.push_back((uint16_t*)reg[r++]);
  }
  for (int j = 0; j <= L; ++j) {
    m->H.push_back((uint16_t*)reg[r++]);
    m->Ht.push_back((uint16_t*)reg[r++]);
    m->G.push_back((uint16_t*)reg[r++]);
    m->Gt.push_back((uint16_t*)reg[r++]);
    m->Z.push_back((float*)reg[r++]);
    m->dZ.push_back((float*)reg[r++]);
  }
  m->Y = (float*)reg[r++];
  m->C = (float*)reg[r++];
  m->Cq = (uint16_t*)reg[r++];
  m->loss_part = (double*)reg[r++];
  m->loss_parts = ((max_batch + 127) / 128) * ((m->P[L] + 127) / 128);
  // everything starts at zero: padding of every buffer must stay zero
  const hipError_t e = hipMemsetAsync(ws, 0, need, (hipStream_t)stream);
  if (e != hipSuccess) {
    delete m;
    return mfail(PWFS_EHIP, "hipMemsetAsync: %s", hipGetErrorString(e));
  }
  *out = m;
  return PWFS_OK;
}

extern "C" int pwfs_mlp_param_count(pwfs_mlp_t m, size_t* count) {
  if (!m || !count) return mfail(PWFS_EINVAL, "NULL argument");
  size_t c = 0;
  for (int l = 0; l < m->L; ++l) c += (size_t)m->n[l + 1] * m->n[l] + m->n[l + 1];
  *count = c;
  return PWFS_OK;
}

namespace {

int copy2d(const float* src, int src_ld, float* dst, int dst_ld, int rows, int cols, hipStream_t st) {
  ParamCopyArgs a{src, dst, rows, cols, src_ld, dst_ld};
  const long long total = (long long)rows * cols;
  hipLaunchKernelGGL(k_copy2d, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mfail(PWFS_EHIP, "launch k_copy2d: %s", hipGetErrorString(e));
  return PWFS_OK;
}

// refresh the 16-bit weight copies from the fp32 masters (Adam with lr = 0
// on zero moments would do the same; this is explicit)
int refresh_q(pwfs_mlp_t m, int l, hipStream_t st) {
  const int rows = m->P[l + 1], cols = m->P[l];
  int rc = split_launch(m->W[l], cols, rows, cols, cols, m->Wq[l], (long long)rows * cols, cols, m->planes, 0, 1.f, st);
  if (rc) return rc;
  return split_launch(m->W[l], cols, rows, cols, cols, m->Wqt[l], (long long)rows * cols, rows, m->planes, 1, 1.f, st);
}

}  // namespace

extern "C" int pwfs_mlp_set_params(pwfs_mlp_t m, const float* params, void* stream) {
  if (!m || !params) return mfail(PWFS_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  size_t off = 0;
  int rc;
  for (int l = 0; l < m->L; ++l) {
    const int no = m->n[l + 1], ni = m->n[l];
    if ((rc = copy2d(params + off, ni, m->W[l], m->P[l], no, ni, st))) return rc;
    off += (size_t)no * ni;
    if ((rc = copy2d(params + off, no, m->b[l], no, 1, no, st))) return rc;
    off += no;
    const size_t w = (size_t)m->P[l + 1] * m->P[l];
    if (hipMemsetAsync(m->mW[l], 0, 4 * w, st) != hipSuccess || hipMemsetAsync(m->vW[l], 0, 4 * w, st) != hipSuccess ||
        hipMemsetAsync(m->mb[l], 0, 4 * (size_t)m->P[l + 1], st) != hipSuccess ||
        hipMemsetAsync(m->vb[l], 0, 4 * (size_t)m->P[l + 1], st) != hipSuccess)
      return mfail(PWFS_EHIP, "hipMemsetAsync");
    if ((rc = refresh_q(m, l, st))) return rc;
  }
  m->step = 0;
  m->have_grad = false;
  return PWFS_OK;
}

extern "C" int pwfs_mlp_get_params(pwfs_mlp_t m, float* params, void* stream) {
  if (!m || !params) return mfail(PWFS_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  size_t off = 0;
  int rc;
  for (int l = 0; l < m->L; ++l) {
    const int no = m->n[l + 1], ni = m->n[l];
    if ((rc = copy2d(m->W[l], m->P[l], params + off, ni, no, ni, st))) return rc;
    off += (size_t)no * ni;
    if ((rc = copy2d(m->b[l], no, params + off, no, 1, no, st))) return rc;
    off += no;
  }
  return PWFS_OK;
}

extern "C" int pwfs_mlp_set_linear(pwfs_mlp_t m, const float* C, void* stream) {
  if (!m) return mfail(PWFS_EINVAL, "NULL argument");
  if (!C) {
    m->have_linear = false;
    return PWFS_OK;
  }
  int rc;
  const int no = m->n[m->L], ni = m->n[0];
  // rows and columns past the true sizes stay zero (the workspace is cleared at create)
  if ((rc = copy2d(C, ni, m->C, m->P[0], no, ni, (hipStream_t)stream))) return rc;
  m->have_linear = true;
  m->c_scale = 0.f;
  return PWFS_OK;
}

// the Adam moments, each packed like the parameters: m, then v
extern "C" int pwfs_mlp_get_state(pwfs_mlp_t m, float* moments, long long* step, void* stream) {
  if (!m || !moments || !step) return mfail(PWFS_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  size_t count = 0;
  pwfs_mlp_param_count(m, &count);
  int rc;
  for (int which = 0; which < 2; ++which) {
    size_t off = which * count;
    for (int l = 0; l < m->L; ++l) {
      const int no = m->n[l + 1], ni = m->n[l];
      if ((rc = copy2d(which ? m->vW[l] : m->mW[l], m->P[l], moments + off, ni, no, ni, st))) return rc;
      off += (size_t)no * ni;
      if ((rc = copy2d(which ? m->vb[l] : m->mb[l], no, moments + off, no, 1, no, st))) return rc;
      off += no;
    }
  }
  *step = m->step;
  return PWFS_OK;
}

extern "C" int pwfs_mlp_set_state(pwfs_mlp_t m, const float* moments, long long step, void* stream) {
  if (!m || !moments) return mfail(PWFS_EINVAL, "NULL argument");
  if (step < 0) return mfail(PWFS_EINVAL, "step must be >= 0");
  hipStream_t st = (hipStream_t)stream;
  size_t count = 0;
  pwfs_mlp_param_count(m, &count);
  int rc;
  for (int which = 0; which < 2; ++which) {
    size_t off = which * count;
    for (int l = 0; l < m->L; ++l) {
      const int no = m->n[l + 1], ni = m->n[l];
      if ((rc = copy2d(moments + off, ni, which ? m->vW[l] : m->mW[l], m->P[l], no, ni, st))) return rc;
      off += (size_t)no * ni;
      if ((rc = copy2d(moments + off, no, which ? m->vb[l] : m->mb[l], no, 1, no, st))) return rc;
      off += no;
    }
  }
  m->step = step;
  return PWFS_OK;
}

namespace {

// forward through all layers; the output epilogue optionally forms the loss
// gradient against `target`
int mlp_forward(pwfs_mlp_t m, const float* x, int batch, float* y, float out_scale, const float* target,
                float tscale, hipStream_t st) {
  const int L = m->L, pl = m->planes;
  int rc;
  // input activations (and their transpose, used by dW of layer 0)
  const long long a0 = (long long)m->Bm * m->P[0];
  if ((rc = split_launch(x, m->n[0], batch, m->n[0], m->P[0], m->H[0], a0, m->P[0], pl, 0, 1.f, st))) return rc;
  if (target)
    if ((rc = split_launch(x, m->n[0], batch, m->n[0], m->P[0], m->Ht[0], a0, m->Bm, pl, 1, 1.f, st))) return rc;
  for (int l = 0; l < L; ++l) {
    GemmArgs g{};
    g.a = m->H[l];
    g.a_plane = (long long)m->Bm * m->P[l];
    g.lda = m->P[l];
    g.b = m->Wq[l];
    g.b_plane = (long long)m->P[l + 1] * m->P[l];
    g.ldb = m->P[l];
    g.M = batch;
    g.N = m->n[l + 1];
    g.K = m->P[l];
    g.bias = m->b[l];
    g.planes_out = pl;
    const long long ap = (long long)m->Bm * m->P[l + 1];
    if (l + 1 < L) {
      g.z = target ? m->Z[l + 1] : nullptr;
      g.ldz = m->P[l + 1];
      g.h = m->H[l + 1];
      g.h_plane = ap;
      g.ldh = m->P[l + 1];
      g.ht = target ? m->Ht[l + 1] : nullptr;
      g.ht_plane = ap;
      g.ldht = m->Bm;
      if ((rc = gemm_dispatch<E_HIDDEN>(pl, g, st))) return rc;
    } else {
      g.alpha = out_scale;
      g.c = y;
      g.ldc = m->n[L];
      if (!target && m->have_linear) {
        // y = out_scale (h W^T + b) + x C^T as one product: the planes of
        // C / out_scale extend K after the layer's own weights
        if (m->c_scale != out_scale) {
          const int PL = m->P[L], P0 = m->P[0];
          if ((rc = split_launch(m->C, P0, PL, P0, P0, m->Cq, (long long)PL * P0, P0, pl, 0, 1.f / out_scale, st)))
            return rc;
          m->c_scale = out_scale;
        }
        g.a2 = m->H[0];
        g.a2_plane = a0;
        g.lda2 = m->P[0];
        g.b2 = m->Cq;
        g.b2_plane = (long long)m->P[L] * m->P[0];
        g.ldb2 = m->P[0];
        g.K2 = m->P[0];
      }
      if (target) {
        g.target = target;
        g.ldt = m->n[L];
        g.tscale = tscale;
        g.gscale = 2.f / ((float)batch * (float)m->n[L]);
        g.z = m->dZ[L];
        g.ldz = m->P[L];
        g.h = m->G[L];
        g.h_plane = ap;
        g.ldh = m->P[L];
        g.ht = m->Gt[L];
        g.ht_plane = ap;
        g.ldht = m->Bm;
        g.loss_part = m->loss_part;
      }
      if ((rc = gemm_dispatch<E_OUTPUT>(pl, g, st))) return rc;
    }
  }
  return PWFS_OK;
}

}  // namespace

extern "C" int pwfs_mlp_forward(pwfs_mlp_t m, const float* x, int batch, float* y, float out_scale, void* stream) {
  if (!m || !x || !y) return mfail(PWFS_EINVAL, "NULL argument");
  if (batch < 1 || batch > m->Bm) return mfail(PWFS_ESTATE, "batch outside [1, max_batch]");
  if (m->have_linear && !(out_scale != 0.f && std::isfinite(out_scale)))
    return mfail(PWFS_EINVAL, "out_scale must be finite and non-zero with a linear term");
  return mlp_forward(m, x, batch, y, out_scale, nullptr, 1.f, (hipStream_t)stream);
}

extern "C" int pwfs_mlp_grad(pwfs_mlp_t m, const float* x, const float* t, int batch, float tscale, float* loss,
                             float* grads, void* stream) {
  if (!m || !x || !t) return mfail(PWFS_EINVAL, "NULL argument");
  if (batch < 32 || batch > m->Bm || batch % 32)
    return mfail(PWFS_ESTATE, "training batch must be a multiple of 32 in [32, max_batch]");
  hipStream_t st = (hipStream_t)stream;
  const int L = m->L, pl = m->planes;
  int rc = mlp_forward(m, x, batch, m->Y, 1.f, t, tscale, st);
  if (rc) return rc;
  const int tiles = ((batch + 127) / 128) * ((m->n[L] + 127) / 128);
  if (loss) {
    hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(64), 0, st, m->loss_part, tiles,
                       1.f / ((float)batch * (float)m->n[L]), loss);
    if (hipGetLastError() != hipSuccess) return mfail(PWFS_EHIP, "launch k_loss_reduce");
  }
  for (int l = L - 1; l >= 0; --l) {
    // dW_l = G_{l+1}^T H_l : A = Gt_{l+1} [n_{l+1}][batch], B = Ht_l [P_l][batch], K = batch
    GemmArgs g{};
    g.a = m->Gt[l + 1];
    g.a_plane = (long long)m->Bm * m->P[l + 1];
    g.lda = m->Bm;
    g.b = m->Ht[l];
    g.b_plane = (long long)m->Bm * m->P[l];
    g.ldb = m->Bm;
    g.M = m->n[l + 1];
    g.N = m->P[l];
    g.K = batch;
    g.alpha = 1.f;
    g.c = m->gW[l];
    g.ldc = m->P[l];
    if ((rc = gemm_dispatch<E_STORE>(pl, g, st))) return rc;
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((m->n[l + 1] + 255) / 256)), dim3(256), 0, st, m->dZ[l + 1],
                       (long long)m->P[l + 1], batch, m->n[l + 1], m->gb[l]);
    if (hipGetLastError() != hipSuccess) return mfail(PWFS_EHIP, "launch k_colsum");
    if (l == 0) break;
    // G_l = (G_{l+1} W_l) * gelu'(Z_l) : A = G_{l+1} [batch][P_{l+1}], B = Wqt_l [P_l][P_{l+1}]
    GemmArgs d{};
    d.a = m->G[l + 1];
    d.a_plane = (long long)m->Bm * m->P[l + 1];
    d.lda = m->P[l + 1];
    d.b = m->Wqt[l];
    d.b_plane = (long long)m->P[l + 1] * m->P[l];
    d.ldb = m->P[l + 1];
    d.M = batch;
    d.N = m->n[l];
    d.K = m->P[l + 1];
    d.zprev = m->Z[l];
    d.ldzp = m->P[l];
    d.z = m->dZ[l];
    d.ldz = m->P[l];
    d.h = m->G[l];
    d.h_plane = (long long)m->Bm * m->P[l];
    d.ldh = m->P[l];
    d.ht = m->Gt[l];
    d.ht_plane = (long long)m->Bm * m->P[l];
    d.ldht = m->Bm;
    d.planes_out = pl;
    if ((rc = gemm_dispatch<E_DHIDDEN>(pl, d, st))) return rc;
  }
  m->have_grad = true;
  if (grads) {
    size_t off = 0;
    for (int l = 0; l < L; ++l) {
      const int no = m->n[l + 1], ni = m->n[l];
      if ((rc = copy2d(m->gW[l], m->P[l], grads + off, ni, no, ni, st))) return rc;
      off += (size_t)no * ni;
      if ((rc = copy2d(m->gb[l], no, grads + off, no, 1, no, st))) return rc;
      off += no;
    }
  }
  return PWFS_OK;
}

extern "C" int pwfs_mlp_adam(pwfs_mlp_t m, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!m) return mfail(PWFS_EINVAL, "NULL argument");
  if (!m->have_grad) return mfail(PWFS_ESTATE, "no gradient: call pwfs_mlp_grad first");
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return mfail(PWFS_EINVAL, "bad Adam hyper-parameters");
  hipStream_t st = (hipStream_t)stream;
  m->step += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, m->step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, m->step)));
  for (int l = 0; l < m->L; ++l) {
    const int rows = m->P[l + 1], cols = m->P[l];
    AdamArgs a{m->W[l], m->mW[l], m->vW[l], m->gW[l], m->Wq[l], m->Wqt[l], (long long)rows * cols,
               (long long)rows * cols, rows, cols, m->planes, lr, beta1, beta2, eps, c1, c2};
    const long long tw = (long long)rows * cols;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((tw + 255) / 256)), dim3(256), 0, st, a);
    AdamArgs ab{m->b[l], m->mb[l], m->vb[l], m->gb[l], nullptr, nullptr, 0, 0, 1, rows, m->planes,
                lr, beta1, beta2, eps, c1, c2};
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, ab);
    if (hipGetLastError() != hipSuccess) return mfail(PWFS_EHIP, "launch k_adam");
  }
  return PWFS_OK;
}

extern "C" void pwfs_mlp_destroy(pwfs_mlp_t m) { delete m; }
