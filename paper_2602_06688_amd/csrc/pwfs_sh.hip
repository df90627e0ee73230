// pwfs_sh.hip -- Shack-Hartmann wavefront sensor (the paper's SH processing
// object, Table 4; its FFT workload shapes in Table 2, e.g. 314 subapertures
// of 56 x 56 for the SCAO SH).
//
// One workgroup per (frame, subaperture), everything in LDS:
//   E[y][x]  = A exp(i 2 pi OPD / lambda) on the b x b block (float64 phase
//              reduction, then float32 sincos);
//   T[y][u]  = sum_x E[y][x] W[u][x]          (b x M)
//   F[v][u]  = sum_y W[v][y] T[y][u]          (M x M, never stored)
//   pixel P  = sum over its rebin x rebin focal samples of |F|^2, in a fixed
//              order; then the centre of gravity of the n_pix x n_pix pixels.
// W[u][x] = exp(-2 pi i (u - M/2 + 1/2)(x - (b-1)/2) / M) puts the focal
// samples at half-integer frequencies (a flat wavefront's spot sits on the
// corner of the four central samples).  A 2-D DFT of a b x b block onto
// M x M samples as two small products costs 2 b M (b + M) real multiply-adds
// (per complex term 4): for b << M (8 vs 56, 7 vs 240) that is less than a
// zero-padded M-point FFT, and it needs no radix plan for M = 56 or 240.
//
// Polychromatic sensor (Table 4: PolyChromSH): the workgroup runs the three
// steps once per sampled wavelength lambda_l, with that wavelength's phase and
// its table W_l (frequencies scaled by s = lambda_ref / lambda_l: the focal
// samples are fixed in angle), and adds w_l s^2 |F_l|^2 / (M^2 sum A^2) into
// the pixels in wavelength order before the centre of gravity.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "pwfs.h"
#include "pwfs_internal.hpp"

namespace pwfs {
namespace {

constexpr int kShBlock = 256;
constexpr double kPiSh = 3.14159265358979323846264338327950288;

int sfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  set_last_error(buf);
  return code;
}

struct ShArgs {
  const float* opd;        // [frames][D][D]
  const float* amp;        // [D][D]
  const float2* W;         // [n_lam][M][b]
  const uint8_t* valid;    // [n][n]
  float* pixels;           // [frames][n][n][k][k] or nullptr
  float* slopes;           // [frames][2][n][n]
  int D, n, b, M, r, k, n_lam;
  float wnorm[PWFS_MAX_LAMBDA];             // w_l s_l^2 / (M^2 sum A^2) (monochromatic: 1 / (M^2 sum A^2))
  double two_pi_over_lam[PWFS_MAX_LAMBDA];
};

// Row stride (in complex values) of the DFT table W [M][b] in LDS: an even
// b is padded by one, so that the rows that a wavefront's lanes read
// together (consecutive u in the T product, the rows v of a pixel's samples)
// start on different banks; with b = 8 unpadded rows are 16 words apart and
// eight of them share two banks of 32.
__host__ __device__ constexpr int sw_stride(int b) { return (b % 2 == 0) ? b + 1 : b; }

// Row stride (in complex values) of the row products T [b][M] in LDS: 257
// for M <= 256, fixed at compile time, so that the loads of a column of T
// in the pixel loop take their row offsets as immediates (one LDS load and
// no address arithmetic per term).  2056 bytes is beyond the reach of both
// paired-load forms (whose two rows collided on banks: a stride that is a
// multiple of 512 bytes puts both on one bank), and consecutive rows start
// two banks apart.  M above 256 keeps M.
constexpr int kTFixed = 256, kTStride = 257;
__host__ __device__ constexpr int t_stride(int M) { return M <= kTFixed ? kTStride : M; }

// Pixel sum of thread s of a pixel whose focal block starts at row pr r and
// column pc r: |sum_y W[v][y] T[y][u]|^2 over every row v of the block and
// the columns u = s, s + tpp, ... of it, NC columns at a time.  Their T
// columns stay in registers while the block's W rows stream past, so each W
// value read from LDS (the lanes of one pixel row read the same one) serves
// NC samples.  Columns past the block are zero (their loads re-read a valid
// column), so they add exact zeros.
template <int BB, int NC>
__device__ __forceinline__ float sh_pixel_cols(const float2* sW, const float2* sT, int ts, int r, int tpp, int s,
                                               int pr, int pc) {
  constexpr int BW = sw_stride(BB);
  float acc = 0.f;
  for (int u0 = s; u0 < r; u0 += NC * tpp) {
    float2 tc[NC][BB];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const bool in = u0 + c * tpp < r;
      const int u = pc * r + (in ? u0 + c * tpp : u0);
#pragma unroll
      for (int y = 0; y < BB; ++y) tc[c][y] = in ? sT[y * ts + u] : make_float2(0.f, 0.f);
    }
    for (int vv = 0; vv < r; ++vv) {
      const float2* wrow = sW + (pr * r + vv) * BW;
      float re[NC], im[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) re[c] = im[c] = 0.f;
#pragma unroll
      for (int y = 0; y < BB; ++y) {
        const float2 w = wrow[y];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          re[c] = fmaf(w.x, tc[c][y].x, fmaf(-w.y, tc[c][y].y, re[c]));
          im[c] = fmaf(w.x, tc[c][y].y, fmaf(w.y, tc[c][y].x, im[c]));
        }
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) acc = fmaf(re[c], re[c], fmaf(im[c], im[c], acc));
    }
  }
  return acc;
}

// Threads per pixel in the pixel loop: the largest power of two that keeps
// the workgroup's kShBlock threads busy without exceeding r.
__host__ __device__ inline int sh_tpp(int kk, int r) {
  int tpp = 1;
  while (tpp * 2 * kk <= kShBlock && tpp * 2 <= r) tpp *= 2;
  return tpp;
}

// BB: the subaperture width b at compile time (the pixel loop then keeps NC
// columns of T in registers, sh_pixel_cols), 0 for a run-time b.  FIXT: M <=
// 256, T stored at the fixed stride kTStride.  NC = 4 needs a thread to own at
// least four columns (r >= 4 tpp) to pay for its registers; the host picks it
// then, for b <= 8.
template <int BB, bool FIXT, int NC>
__global__ __launch_bounds__(kShBlock) void k_sh(ShArgs p) {
  extern __shared__ float2 sh_mem[];
  const int tid = threadIdx.x;
  const int sub = blockIdx.x % (p.n * p.n), f = blockIdx.x / (p.n * p.n);
  const int si = sub / p.n, sj = sub % p.n;
  const int b = p.b, M = p.M, r = p.r, k = p.k;
  const int kk = k * k;
  float* pix_out = p.pixels ? p.pixels + ((size_t)f * p.n * p.n + sub) * kk : nullptr;
  float* sl = p.slopes + (size_t)f * 2 * p.n * p.n;
  if (!p.valid[sub]) {   // invalid subaperture: zero slopes (and pixels)
    if (tid == 0) {
      sl[sub] = 0.f;
      sl[p.n * p.n + sub] = 0.f;
    }
    if (pix_out)
      for (int i = tid; i < kk; i += kShBlock) pix_out[i] = 0.f;
    return;
  }
  constexpr int BW = BB > 0 ? sw_stride(BB) : 0;
  const int bw = BB > 0 ? BW : sw_stride(b);
  float2* sW = sh_mem;                 // [M][bw], row u holds W[u][0 .. b)
  float2* sE = sW + M * bw;            // [b][b]
  const int ts = FIXT ? kTStride : M;   // T row stride (t_stride(M))
  float2* sT = sE + b * b;             // [b][ts], row y holds T[y][0 .. M)
  float* sP = (float*)(sT + b * ts);   // [kk] pixel values, then [kShBlock] partials
  float* sR = sP + kk;

  const float* opd = p.opd + (size_t)f * p.D * p.D;
  // one pass per wavelength; the pixel loop's last barrier frees sW, sE and
  // sT for the next one
  for (int l = 0; l < p.n_lam; ++l) {
    for (int i = tid; i < M * b; i += kShBlock) sW[(i / b) * bw + i % b] = p.W[(size_t)l * M * b + i];
    for (int i = tid; i < b * b; i += kShBlock) {
      const int y = i / b, x = i % b;
      const size_t g = (size_t)(si * b + y) * p.D + sj * b + x;
      const double ph = (double)opd[g] * p.two_pi_over_lam[l];
      const double nn = rint(ph * 0.15915494309189533577);
      const float rr = (float)fma(-nn, 6.283185307179586477, ph);
      float sn, cs;
      sincosf(rr, &sn, &cs);
      const float a = p.amp[g];
      sE[i] = make_float2(a * cs, a * sn);
    }
    __syncthreads();
    // T[y][u] = sum_x E[y][x] W[u][x]
    for (int i = tid; i < b * M; i += kShBlock) {
      const int y = i / M, u = i % M;
      float re = 0.f, im = 0.f;
      for (int x = 0; x < b; ++x) {
        const float2 e = sE[y * b + x], w = sW[u * bw + x];
        re = fmaf(e.x, w.x, fmaf(-e.y, w.y, re));
        im = fmaf(e.x, w.y, fmaf(e.y, w.x, im));
      }
      sT[y * ts + u] = make_float2(re, im);
    }
    __syncthreads();
    // pixels: TPP threads per pixel share its r x r focal samples (fixed order).
    // With b known at compile time thread s takes the focal columns s, s + TPP,
    // ... (sh_pixel_cols); otherwise the rows s, s + TPP, ... one W row at a
    // time.
    const int tpp = sh_tpp(kk, r);
    for (int base = 0; base < kk * tpp; base += kShBlock) {
      const int slot = base + tid;
      const int P = slot / tpp, s = slot % tpp;
      float acc = 0.f;
      if (P < kk) {
        const int pr = P / k, pc = P % k;
        if constexpr (BB > 0) {
          acc = sh_pixel_cols<BB, NC>(sW, sT, ts, r, tpp, s, pr, pc);
        } else {
          for (int vv = s; vv < r; vv += tpp) {
            const int v = pr * r + vv;
            for (int uu = 0; uu < r; ++uu) {
              const int u = pc * r + uu;
              float re = 0.f, im = 0.f;
              for (int y = 0; y < b; ++y) {
                const float2 w = sW[v * bw + y], t = sT[y * ts + u];
                re = fmaf(w.x, t.x, fmaf(-w.y, t.y, re));
                im = fmaf(w.x, t.y, fmaf(w.y, t.x, im));
              }
              acc = fmaf(re, re, fmaf(im, im, acc));
            }
          }
        }
      }
      sR[tid] = acc;
      __syncthreads();
      if (s == 0 && P < kk) {
        float v = sR[tid];
        for (int q = 1; q < tpp; ++q) v += sR[tid + q];
        sP[P] = (l == 0 ? 0.f : sP[P]) + v * p.wnorm[l];
      }
      __syncthreads();
    }
  }   // wavelengths
  // centre of gravity: the first wavefront sums the pixels lane-strided,
  // then a fixed butterfly of cross-lane adds (no workgroup barriers)
  if (tid >= 64) return;
  float t0 = 0.f, tx = 0.f, ty = 0.f;
  const float c0 = 0.5f * (float)(k - 1);
  for (int P = tid; P < kk; P += 64) {
    const float v = sP[P];
    t0 += v;
    tx = fmaf(v, (float)(P % k) - c0, tx);
    ty = fmaf(v, (float)(P / k) - c0, ty);
    if (pix_out) pix_out[P] = v;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    t0 += __shfl_xor(t0, off, 64);
    tx += __shfl_xor(tx, off, 64);
    ty += __shfl_xor(ty, off, 64);
  }
  if (tid == 0) {
    sl[sub] = t0 > 0.f ? tx / t0 : 0.f;
    sl[p.n * p.n + sub] = t0 > 0.f ? ty / t0 : 0.f;
  }
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace
}  // namespace pwfs

using namespace pwfs;

struct pwfs_sh_s {
  pwfs_sh_desc d;
  int D, n, b, M, r, k, max_frames, n_valid, n_lam;
  float wnorm[PWFS_MAX_LAMBDA];
  double two_pi_over_lam[PWFS_MAX_LAMBDA];
  float* amp = nullptr;
  float2* W = nullptr;
  uint8_t* valid = nullptr;
  size_t lds = 0;
};

extern "C" int pwfs_sh_validate(const pwfs_sh_desc* d) {
  if (!d) return sfail(PWFS_EINVAL, "NULL description");
  if (d->pad_ != 0) return sfail(PWFS_EINVAL, "reserved fields must be 0");
  if (d->n_lambda < 0 || d->n_lambda > PWFS_MAX_LAMBDA)
    return sfail(PWFS_EINVAL, "n_lambda must be in [0, %d]", PWFS_MAX_LAMBDA);
  if (d->n_pupil < 2 || d->n_subap < 1 || d->n_pupil % d->n_subap)
    return sfail(PWFS_EINVAL, "n_pupil must be a positive multiple of n_subap");
  const int b = d->n_pupil / d->n_subap;
  if (b > 32) return sfail(PWFS_EUNSUPPORTED, "subaperture of %d px (> 32) not supported", b);
  if (d->n_fft < 2 || d->n_fft > 512) return sfail(PWFS_EINVAL, "n_fft must be in [2, 512]");
  if (d->rebin < 1 || d->n_fft % d->rebin) return sfail(PWFS_EINVAL, "rebin must divide n_fft");
  if (!(d->obstruction >= 0.0 && d->obstruction < 1.0)) return sfail(PWFS_EINVAL, "obstruction must be in [0, 1)");
  if (!(d->lambda_nm > 0.0) || !std::isfinite(d->lambda_nm)) return sfail(PWFS_EINVAL, "lambda_nm must be > 0");
  if (d->n_lambda >= 2) {
    double wsum = 0.0;
    for (int l = 0; l < d->n_lambda; ++l) {
      if (!(d->lambdas_nm[l] >= d->lambda_nm) || !std::isfinite(d->lambdas_nm[l]))
        return sfail(PWFS_EINVAL, "lambdas_nm[%d] must be finite and >= lambda_nm (the reference)", l);
      if (!(d->lambda_weights[l] >= 0.0)) return sfail(PWFS_EINVAL, "lambda_weights[%d] must be >= 0", l);
      wsum += d->lambda_weights[l];
    }
    if (std::fabs(wsum - 1.0) > 1e-9) return sfail(PWFS_EINVAL, "lambda_weights must sum to 1");
  }
  const int k = d->n_fft / d->rebin;
  const size_t lds = sizeof(float2) * ((size_t)d->n_fft * sw_stride(b) + (size_t)b * t_stride(d->n_fft) + (size_t)b * b) +
                     sizeof(float) * ((size_t)k * k + kShBlock);
  if (lds > 150 * 1024) return sfail(PWFS_EUNSUPPORTED, "subaperture tables exceed the LDS (n_fft x b too large)");
  return PWFS_OK;
}

extern "C" int pwfs_sh_workspace_size(const pwfs_sh_desc* d, int max_frames, size_t* bytes) {
  int rc = pwfs_sh_validate(d);
  if (rc) return rc;
  if (!bytes || max_frames < 1) return sfail(PWFS_EINVAL, "bad arguments");
  const int D = d->n_pupil, n = d->n_subap, b = D / n;
  const int nl = d->n_lambda >= 2 ? d->n_lambda : 1;
  *bytes = a256(sizeof(float) * D * D) + a256(sizeof(float2) * nl * d->n_fft * b) + a256((size_t)n * n);
  return PWFS_OK;
}

extern "C" int pwfs_sh_plan(const pwfs_sh_desc* d, int max_frames, void* ws, size_t ws_bytes, void* stream,
                            pwfs_sh_t* out) {
  size_t need = 0;
  int rc = pwfs_sh_workspace_size(d, max_frames, &need);
  if (rc) return rc;
  if (!out) return sfail(PWFS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need) return sfail(PWFS_EWORKSPACE, "workspace missing, small or misaligned");
  const int D = d->n_pupil, n = d->n_subap, b = D / n, M = d->n_fft;
  // pupil (pixel centres at i - (D-1)/2, inside if eps R <= r <= R) and valid map (>= half lit)
  std::vector<float> A((size_t)D * D);
  const double R = D / 2.0, Ro = d->obstruction * R;
  double sA2 = 0.0;
  for (int y = 0; y < D; ++y)
    for (int x = 0; x < D; ++x) {
      const double cy = y - (D - 1) / 2.0, cx = x - (D - 1) / 2.0, r2 = cx * cx + cy * cy;
      A[(size_t)y * D + x] = (r2 <= R * R && r2 >= Ro * Ro) ? 1.f : 0.f;
      sA2 += A[(size_t)y * D + x];
    }
  std::vector<uint8_t> V((size_t)n * n);
  int nv = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      int c = 0;
      for (int y = 0; y < b; ++y)
        for (int x = 0; x < b; ++x) c += A[(size_t)(i * b + y) * D + j * b + x] != 0.f;
      V[(size_t)i * n + j] = 2 * c >= b * b;
      nv += V[(size_t)i * n + j];
    }
  if (nv == 0) return sfail(PWFS_EINVAL, "no valid subaperture");
  // per wavelength: W_l[u][x] with the frequency scale s_l = lambda_ref / lambda_l
  const int nl = d->n_lambda >= 2 ? d->n_lambda : 1;
  std::vector<float2> W((size_t)nl * M * b);
  std::vector<double> scale(nl, 1.0), lam(nl, d->lambda_nm), wgt(nl, 1.0);
  for (int l = 0; l < nl && d->n_lambda >= 2; ++l) {
    lam[l] = d->lambdas_nm[l];
    wgt[l] = d->lambda_weights[l];
    scale[l] = d->lambda_nm / d->lambdas_nm[l];
  }
  for (int l = 0; l < nl; ++l)
    for (int u = 0; u < M; ++u)
      for (int x = 0; x < b; ++x) {
        const double a = -2.0 * kPiSh * (u - M / 2.0 + 0.5) * (x - (b - 1) / 2.0) * scale[l] / M;
        W[((size_t)l * M + u) * b + x] = make_float2((float)std::cos(a), (float)std::sin(a));
      }
  pwfs_sh_s* s = new (std::nothrow) pwfs_sh_s();
  if (!s) return sfail(PWFS_EINVAL, "out of host memory");
  s->d = *d;
  s->D = D;
  s->n = n;
  s->b = b;
  s->M = M;
  s->r = d->rebin;
  s->k = M / d->rebin;
  s->max_frames = max_frames;
  s->n_valid = nv;
  s->n_lam = nl;
  for (int l = 0; l < nl; ++l) {
    s->wnorm[l] = (float)(wgt[l] * scale[l] * scale[l] / ((double)M * M * sA2));
    s->two_pi_over_lam[l] = 2.0 * kPiSh / lam[l];
  }
  char* p = (char*)ws;
  s->amp = (float*)p;
  p += a256(sizeof(float) * D * D);
  s->W = (float2*)p;
  p += a256(sizeof(float2) * nl * M * b);
  s->valid = (uint8_t*)p;
  s->lds = sizeof(float2) * ((size_t)M * sw_stride(b) + (size_t)b * t_stride(M) + (size_t)b * b) +
           sizeof(float) * ((size_t)s->k * s->k + kShBlock);
  hipStream_t st = (hipStream_t)stream;
  if (hipMemcpyAsync(s->amp, A.data(), A.size() * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(s->W, W.data(), W.size() * sizeof(float2), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(s->valid, V.data(), V.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    delete s;
    return sfail(PWFS_EHIP, "uploading the sensor tables failed");
  }
  static bool lds_set = false;
  if (!lds_set) {
    const void* fns[] = {
        (const void*)k_sh<0, true, 2>,  (const void*)k_sh<4, true, 2>,  (const void*)k_sh<7, true, 2>,
        (const void*)k_sh<8, true, 2>,  (const void*)k_sh<16, true, 2>, (const void*)k_sh<0, false, 2>,
        (const void*)k_sh<4, false, 2>, (const void*)k_sh<7, false, 2>, (const void*)k_sh<8, false, 2>,
        (const void*)k_sh<16, false, 2>, (const void*)k_sh<4, true, 4>, (const void*)k_sh<7, true, 4>,
        (const void*)k_sh<8, true, 4>,  (const void*)k_sh<4, false, 4>, (const void*)k_sh<7, false, 4>,
        (const void*)k_sh<8, false, 4>};
    for (const void* fn : fns)
      if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
        (void)hipGetLastError();
    lds_set = true;
  }
  *out = s;
  return PWFS_OK;
}

namespace {
template <int BB, bool FIXT>
void launch_sh(bool wide, unsigned grid, size_t lds, hipStream_t st, const ShArgs& a) {
  if constexpr (BB > 0 && BB <= 8) {
    if (wide) {
      hipLaunchKernelGGL((k_sh<BB, FIXT, 4>), dim3(grid), dim3(kShBlock), lds, st, a);
      return;
    }
  }
  hipLaunchKernelGGL((k_sh<BB, FIXT, 2>), dim3(grid), dim3(kShBlock), lds, st, a);
}
}  // namespace

extern "C" int pwfs_sh_forward(pwfs_sh_t s, const float* opd, int nf, float* pixels, float* slopes, void* stream) {
  if (!s) return sfail(PWFS_EINVAL, "plan is NULL");
  if (!opd || !slopes) return sfail(PWFS_EINVAL, "NULL device pointer");
  if (nf < 1 || nf > s->max_frames) return sfail(PWFS_ESTATE, "n_frames %d outside [1, max_frames]", nf);
  ShArgs a{};
  a.opd = opd;
  a.amp = s->amp;
  a.W = s->W;
  a.valid = s->valid;
  a.pixels = pixels;
  a.slopes = slopes;
  a.D = s->D;
  a.n = s->n;
  a.b = s->b;
  a.M = s->M;
  a.r = s->r;
  a.k = s->k;
  a.n_lam = s->n_lam;
  for (int l = 0; l < s->n_lam; ++l) {
    a.wnorm[l] = s->wnorm[l];
    a.two_pi_over_lam[l] = s->two_pi_over_lam[l];
  }
  const unsigned grid = (unsigned)((long long)nf * s->n * s->n);
  hipStream_t st = (hipStream_t)stream;
  const bool fixt = s->M <= kTFixed;
  const bool wide = s->r >= 4 * sh_tpp(s->k * s->k, s->r);
  switch (s->b * 2 + (fixt ? 1 : 0)) {
    case 9: launch_sh<4, true>(wide, grid, s->lds, st, a); break;
    case 8: launch_sh<4, false>(wide, grid, s->lds, st, a); break;
    case 15: launch_sh<7, true>(wide, grid, s->lds, st, a); break;
    case 14: launch_sh<7, false>(wide, grid, s->lds, st, a); break;
    case 17: launch_sh<8, true>(wide, grid, s->lds, st, a); break;
    case 16: launch_sh<8, false>(wide, grid, s->lds, st, a); break;
    case 33: launch_sh<16, true>(wide, grid, s->lds, st, a); break;
    case 32: launch_sh<16, false>(wide, grid, s->lds, st, a); break;
    default:
      if (fixt) launch_sh<0, true>(wide, grid, s->lds, st, a);
      else launch_sh<0, false>(wide, grid, s->lds, st, a);
      break;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return sfail(PWFS_EHIP, "launch k_sh: %s", hipGetErrorString(e));
  return PWFS_OK;
}

extern "C" int pwfs_sh_query(pwfs_sh_t s, int32_t* n_valid, int32_t* n_pix) {
  if (!s || !n_valid || !n_pix) return sfail(PWFS_EINVAL, "NULL argument");
  *n_valid = s->n_valid;
  *n_pix = s->k;
  return PWFS_OK;
}

extern "C" void pwfs_sh_destroy(pwfs_sh_t s) { delete s; }
