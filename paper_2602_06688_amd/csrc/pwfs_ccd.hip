// pwfs_ccd.hip -- detector stage after the pyramid sensor (the paper's CCD
// processing object, Table 4; its parameters in the SOUL configuration of
// Appendix B): integer rebinning of the normalised intensity onto detector
// pixels, photon noise (Poisson), electron-multiplication excess noise
// (Gamma(n, 1) at high gain) and readout noise (Gaussian), and the slope
// stage on detector pixels.
//
// One thread per detector pixel and frame.  Random numbers are Philox4x64-10
// (Salmon, Moraes, Dror, Shaw, SC'11) keyed by (seed, 0) with counter
// (pixel, frame, purpose, block): every draw is a pure function of where it
// is used, so results do not depend on the launch shape or the chunking of
// frames.  Every float64 step of the samplers is a correctly rounded + - * /
// or an exact power-of-two scaling (contraction off): exp(-mu) of the Poisson
// inversion by a fixed Taylor series and repeated squaring, and the ln, sqrt
// and cos of the normal and Gamma draws by the fixed series below.  So the
// Poisson integers, the Gamma accept/reject decisions and the draws are
// reproduced bit for bit by any implementation doing the same operations in
// the same order, with no math library in between.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "pwfs.h"
#include "pwfs_internal.hpp"

namespace pwfs {
namespace {

constexpr double kPoissonChunk = 256.0;  // largest mean of one inversion
constexpr int kPoissonKcap = 1024;       // inversion stops here
constexpr int kGammaTries = 64;          // Marsaglia-Tsang attempts
constexpr double kMaxLam = 16777216.0;   // 2^24: larger (or non-finite) expected counts give NaN
constexpr uint64_t kPhotonPurpose = 0, kExcessPurpose = 1, kReadoutPurpose = 2;

struct u64x4 {
  uint64_t w[4];
};

// Philox4x64-10: ten rounds of two 64x64->128 multiplies, Weyl key schedule
__device__ __forceinline__ u64x4 philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                        uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t h0 = __umul64hi(M0, c0), l0 = M0 * c0;
    const uint64_t h1 = __umul64hi(M1, c2), l1 = M1 * c2;
    const uint64_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
    c0 = n0;
    c1 = l1;
    c2 = n2;
    c3 = l0;
  }
  return {{c0, c1, c2, c3}};
}

__device__ __forceinline__ double uniform01(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

// ---------------------------------------------- elementary functions ----
// ln, sqrt and cos(2 pi u) of the samplers from + - * / and exact scalings
// by powers of two only (contraction off), each step rounded on its own:
// the Gamma sampler's accept/reject decision is then the same bits on any
// implementation that does the same operations in the same order, whatever
// its math library.
constexpr double kLn2 = 0.6931471805599453;        // float64 nearest ln 2
constexpr double kTwoPi = 6.283185307179586;       // float64 nearest 2 pi
constexpr double kSqrtHalf = 0.7071067811865476;   // float64 nearest sqrt(1/2)
constexpr int kLogTerms = 12;                      // atanh series: |s| <= 0.1716
constexpr int kSqrtNewton = 5;

// ln x, x finite > 0: x = m 2^e, m in [sqrt(1/2), sqrt 2), ln m = 2 atanh s,
// s = (m - 1)/(m + 1), the series sum_j s^(2j+1)/(2j+1) by Horner in s^2
__device__ double log_basic(double x) {
#pragma clang fp contract(off)
  int e;
  double m = frexp(x, &e);   // [0.5, 1)
  if (m < kSqrtHalf) {
    m = m * 2.0;
    e = e - 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  double p = 1.0 / (2.0 * kLogTerms + 1.0);
  for (int j = kLogTerms - 1; j >= 0; --j) {
    const double t = p * s2;
    p = t + 1.0 / (2.0 * j + 1.0);
  }
  double t = s * p;
  t = t * 2.0;
  const double el = (double)e * kLn2;
  return el + t;
}

// sqrt y, y finite >= 0: y = m 2^e, e even, m in [0.5, 2); first guess
// 0.41731 + 0.59016 m, then Newton g <- (g + m/g) / 2, scaled by 2^(e/2)
__device__ double sqrt_basic(double y) {
#pragma clang fp contract(off)
  if (y == 0.0) return 0.0;
  int e;
  double m = frexp(y, &e);
  if (e & 1) {
    m = m * 2.0;
    e = e - 1;
  }
  double g = 0.59016 * m;
  g = 0.41731 + g;
  for (int i = 0; i < kSqrtNewton; ++i) {
    const double q = m / g;
    g = g + q;
    g = g * 0.5;
  }
  return ldexp(g, e / 2);
}

// n! as a float64 product formed left to right
__device__ double fact(int n) {
#pragma clang fp contract(off)
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f = f * (double)i;
  return f;
}

// cos x and sin x for |x| <= pi/4: Taylor terms through x^16/16! and
// x^17/17!, Horner in x^2 from the highest term
__device__ double cos_poly(double x) {
#pragma clang fp contract(off)
  const double x2 = x * x;
  double c = 1.0 / fact(16);
  for (int k = 7; k >= 0; --k) {
    const double t = c * x2;
    c = ((k & 1) ? -1.0 : 1.0) / fact(2 * k) + t;
  }
  return c;
}
__device__ double sin_poly(double x) {
#pragma clang fp contract(off)
  const double x2 = x * x;
  double c = 1.0 / fact(17);
  for (int k = 7; k >= 0; --k) {
    const double t = c * x2;
    c = ((k & 1) ? -1.0 : 1.0) / fact(2 * k + 1) + t;
  }
  return c * x;
}

// cos(2 pi u), u in [0, 1): w = min(u, 1 - u) in [0, 1/2] (exact), then one
// of cos(2 pi w), sin(2 pi (1/4 - w)), -cos(2 pi (1/2 - w)) on an exact
// reduced argument of at most 1/8
__device__ double cos_2pi_basic(double u) {
#pragma clang fp contract(off)
  const double w = u >= 0.5 ? 1.0 - u : u;
  if (w <= 0.125) return cos_poly(w * kTwoPi);
  if (w <= 0.375) return sin_poly((0.25 - w) * kTwoPi);
  return -cos_poly((0.5 - w) * kTwoPi);
}

__device__ double box_muller(uint64_t w0, uint64_t w1) {
#pragma clang fp contract(off)
  const double u1 = 1.0 - uniform01(w0);   // (0, 1]
  const double u2 = uniform01(w1);
  const double r = sqrt_basic(-2.0 * log_basic(u1));
  return r * cos_2pi_basic(u2);
}

// exp(-mu), 0 <= mu <= 256: 24-term Taylor series at mu / 256, eight squarings
__device__ double exp_neg(double mu) {
#pragma clang fp contract(off)
  const double x = mu / 256.0;
  double e = 1.0;
  for (int i = 24; i >= 1; --i) {
    double t = e * x;
    t = t / (double)i;
    e = 1.0 - t;
  }
  for (int i = 0; i < 8; ++i) e = e * e;
  return e;
}

// smallest k with u <= F(k), p_k = p_{k-1} mu / k, stopping at kPoissonKcap
__device__ int poisson_inversion(double mu, double u) {
#pragma clang fp contract(off)
  double p = exp_neg(mu);
  double F = p;
  int k = 0;
  while (u > F && k < kPoissonKcap) {
    ++k;
    double q = p * mu;
    q = q / (double)k;
    F = F + q;
    p = q;
  }
  return k;
}

__device__ long long poisson(double lam, uint64_t pix, uint64_t frame, uint64_t k0, uint64_t k1) {
#pragma clang fp contract(off)
  if (!(lam > 0.0)) return 0;
  const long long m = (long long)ceil(lam / kPoissonChunk);
  const double mu = lam / (double)m;
  long long n = 0;
  for (long long j = 0; j < m; ++j) {
    const u64x4 w = philox(pix, frame, kPhotonPurpose, (uint64_t)j, k0, k1);
    n += poisson_inversion(mu, uniform01(w.w[0]));
  }
  return n;
}

// Gamma(n, 1), n >= 1 (Marsaglia-Tsang); attempt i uses counter block i
__device__ double gamma_mt(double n, uint64_t pix, uint64_t frame, uint64_t k0, uint64_t k1) {
#pragma clang fp contract(off)
  const double d = n - 1.0 / 3.0;
  const double c = 1.0 / sqrt_basic(9.0 * d);
  for (int i = 0; i < kGammaTries; ++i) {
    const u64x4 w = philox(pix, frame, kExcessPurpose, (uint64_t)i, k0, k1);
    const double x = box_muller(w.w[0], w.w[1]);
    const double u = uniform01(w.w[2]);
    double v = 1.0 + c * x;
    if (!(v > 0.0)) continue;
    v = v * v * v;
    const double lhs = u > 0.0 ? log_basic(u) : -__builtin_inf();
    double rhs = 0.5 * x;
    rhs = rhs * x;
    rhs = rhs + d;
    rhs = rhs - d * v;
    rhs = rhs + d * log_basic(v);
    if (lhs < rhs) return d * v;
  }
  return d;
}

struct CcdArgs {
  const float* in;          // sensor's intensity plane of the first frame
  long long in_stride;      // floats between frames
  float* out;               // [frames][n_det][n_det]
  int N, n_det, off;        // plane size, detector size, offset of the detector square
  int num, den;             // detector pitch num / den transform pixels
  int windows;              // count only detector pixels inside the four pupil images
  int img_r[2], img_c[2];   // image starts in detector pixels (two rows x two columns)
  int img;                  // image size in detector pixels
  uint32_t flags;
  double electrons, readout_e;
  uint64_t k0, k1;
  long long frame0;
};

__global__ __launch_bounds__(256) void k_ccd(CcdArgs p) {
#pragma clang fp contract(off)
  const int nn = p.n_det * p.n_det;
  const int pix = blockIdx.x * 256 + threadIdx.x;
  if (pix >= nn) return;
  const int f = blockIdx.y;
  const int r = pix / p.n_det, c = pix % p.n_det;
  bool inside = true;
  if (p.windows) {
    const bool rin = (r >= p.img_r[0] && r < p.img_r[0] + p.img) || (r >= p.img_r[1] && r < p.img_r[1] + p.img);
    const bool cin = (c >= p.img_c[0] && c < p.img_c[0] + p.img) || (c >= p.img_c[1] && c < p.img_c[1] + p.img);
    inside = rin && cin;
  }
  double s = 0.0;
  if (inside) {
    // the transform pixels this detector pixel overlaps, row-major; overlaps
    // in units of 1/den pixel, weight = area fraction (1 when den = 1)
    const float* I = p.in + (long long)f * p.in_stride + (long long)p.off * p.N + p.off;
    const int ylo = r * p.num, yhi = ylo + p.num, xlo = c * p.num, xhi = xlo + p.num;
    const double dd = (double)p.den * (double)p.den;
    for (int y = ylo / p.den; y * p.den < yhi; ++y) {
      const int oy = min((y + 1) * p.den, yhi) - max(y * p.den, ylo);
      for (int x = xlo / p.den; x * p.den < xhi; ++x) {
        const int ox = min((x + 1) * p.den, xhi) - max(x * p.den, xlo);
        const double w = (double)(oy * ox) / dd;
        s = s + w * (double)I[(long long)y * p.N + x];
      }
    }
  }
  const double lam = s * p.electrons;
  const uint64_t frame = (uint64_t)(p.frame0 + f);
  double v;
  if (p.flags & PWFS_CCD_PHOTON) {
    if (!(lam <= kMaxLam)) {   // bounds the O(lam) inversion; also catches NaN / inf inputs
      v = __builtin_nan("");
    } else {
      const long long n = poisson(lam, (uint64_t)pix, frame, p.k0, p.k1);
      v = (double)n;
      if ((p.flags & PWFS_CCD_EXCESS) && n > 0) v = gamma_mt(v, (uint64_t)pix, frame, p.k0, p.k1);
    }
  } else {
    v = lam;
  }
  if (p.flags & PWFS_CCD_READOUT) {
    const u64x4 w = philox((uint64_t)pix, frame, kReadoutPurpose, 0, p.k0, p.k1);
    v = v + p.readout_e * box_muller(w.w[0], w.w[1]);
  }
  p.out[(long long)f * nn + pix] = (float)v;
}

int cfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  set_last_error(buf);
  return code;
}

// detector geometry of sensor sp; `aligned` also requires the pupil images
// to fall on whole detector pixels and to be tiled by the subapertures
struct DetGeom {
  int off, num, den, img, b, img_r[2], img_c[2];
};

int det_geometry(const SensorPlan& sp, const pwfs_ccd_desc* d, bool aligned, DetGeom& out) {
  const Geometry& g = sp.g;
  if (sp.arms != 1) return cfail(PWFS_EUNSUPPORTED, "the detector stage takes four-face pyramid sensors");
  if (d->n_det < 1 || d->rebin < 1 || d->rebin_den < 0 || d->rebin_den > 64)
    return cfail(PWFS_EINVAL, "bad detector size or rebin");
  const int num = d->rebin, den = d->rebin_den ? d->rebin_den : 1;
  if (num < den) return cfail(PWFS_EINVAL, "detector pixels smaller than transform pixels (rebin < rebin_den)");
  out.num = num;
  out.den = den;
  if (d->flags & ~(uint32_t)(PWFS_CCD_PHOTON | PWFS_CCD_READOUT | PWFS_CCD_EXCESS))
    return cfail(PWFS_EINVAL, "unknown detector flags");
  if ((d->flags & PWFS_CCD_EXCESS) && !(d->flags & PWFS_CCD_PHOTON))
    return cfail(PWFS_EINVAL, "excess noise needs photon noise");
  if (!(d->electrons >= 0.0) || !(d->readout_e >= 0.0) || !std::isfinite(d->electrons))
    return cfail(PWFS_EINVAL, "electrons and readout noise must be finite and >= 0");
  const long long wn = (long long)num * d->n_det;    // detector square, in 1/den pixel
  if (wn % den) return cfail(PWFS_EINVAL, "the detector square (n_det * rebin / rebin_den) must be whole pixels");
  const long long w = wn / den;
  if (w > g.N || (g.N - w) % 2)
    return cfail(PWFS_EINVAL, "the detector square must be <= N pixels with N minus it even");
  out.off = (int)((g.N - w) / 2);
  if (!aligned && g.full) return PWFS_OK;
  if (((long long)g.D * den) % num || ((long long)g.D * den / num) % g.n)
    return cfail(PWFS_EINVAL, "the pupil images must be whole detector pixels tiled by the subapertures");
  out.img = (int)((long long)g.D * den / num);
  out.b = out.img / g.n;
  for (int q = 0; q < 2; ++q) {
    const int sgn = q ? 1 : -1;
    const long long o = (long long)(g.N / 2 + sgn * g.S / 2 - g.D / 2 - out.off) * den;
    if (o < 0 || o % num || o / num + out.img > d->n_det)
      return cfail(PWFS_EINVAL, "pupil image not aligned with the detector pixels");
    out.img_r[q] = out.img_c[q] = (int)(o / num);
  }
  return PWFS_OK;
}

}  // namespace
}  // namespace pwfs

using namespace pwfs;

extern "C" int pwfs_ccd(pwfs_plan_t p, int sensor, const pwfs_ccd_desc* d, const float* in, int nf, long long frame0,
                        float* out, void* stream) {
  if (!p || !d) return cfail(PWFS_EINVAL, "NULL argument");
  if (!in || !out) return cfail(PWFS_EINVAL, "NULL device pointer");
  if (sensor < 0 || sensor >= (int)p->s.size()) return cfail(PWFS_EINVAL, "sensor index out of range");
  if (nf < 1 || nf > p->max_frames) return cfail(PWFS_ESTATE, "n_frames %d outside [1, max_frames]", nf);
  if (frame0 < 0) return cfail(PWFS_EINVAL, "frame0 must be >= 0");
  const SensorPlan& sp = p->s[sensor];
  DetGeom dg{};
  int rc = det_geometry(sp, d, false, dg);
  if (rc) return rc;
  CcdArgs a{};
  a.in = in + sp.int_offset;
  a.in_stride = (long long)p->int_stride;
  a.out = out;
  a.N = sp.g.N;
  a.n_det = d->n_det;
  a.num = dg.num;
  a.den = dg.den;
  a.off = dg.off;
  a.windows = sp.g.full ? 0 : 1;
  for (int q = 0; q < 2; ++q) {
    a.img_r[q] = dg.img_r[q];
    a.img_c[q] = dg.img_c[q];
  }
  a.img = dg.img;
  a.flags = d->flags;
  a.electrons = d->electrons;
  a.readout_e = d->readout_e;
  a.k0 = d->seed;
  a.k1 = 0;
  a.frame0 = frame0;
  const int nn = d->n_det * d->n_det;
  hipStream_t st = (hipStream_t)stream;
  const int slot = p->prof.begin(st);
  hipLaunchKernelGGL(k_ccd, dim3((unsigned)((nn + 255) / 256), (unsigned)nf), dim3(256), 0, st, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return cfail(PWFS_EHIP, "launch k_ccd: %s", hipGetErrorString(e));
  p->prof.end(slot, st, K_CCD);
  return PWFS_OK;
}

extern "C" int pwfs_ccd_slopes(pwfs_plan_t p, int sensor, const pwfs_ccd_desc* d, const float* pixels, int nf,
                               float* slopes, float* flux, void* stream) {
  if (!p || !d) return cfail(PWFS_EINVAL, "NULL argument");
  if (!pixels || !slopes) return cfail(PWFS_EINVAL, "NULL device pointer");
  if (sensor < 0 || sensor >= (int)p->s.size()) return cfail(PWFS_EINVAL, "sensor index out of range");
  if (nf < 1 || nf > p->max_frames) return cfail(PWFS_ESTATE, "n_frames %d outside [1, max_frames]", nf);
  const SensorPlan& sp = p->s[sensor];
  DetGeom dg{};
  int rc = det_geometry(sp, d, true, dg);
  if (rc) return rc;
  const int org_r[4] = {dg.img_r[0], dg.img_r[0], dg.img_r[1], dg.img_r[1]};
  const int org_c[4] = {dg.img_c[0], dg.img_c[1], dg.img_c[0], dg.img_c[1]};
  const float* ref = (sp.desc.flags & PWFS_F_REF_SLOPES) ? (const float*)sp.dev[R_REF] : nullptr;
  const int nn = d->n_det * d->n_det;
  return slopes_launch_at(sp, pixels, nn, slopes, 2LL * sp.g.n * sp.g.n, flux, 1, ref, nf, d->n_det, dg.img, org_r,
                          org_c, (hipStream_t)stream, &p->prof);
}
