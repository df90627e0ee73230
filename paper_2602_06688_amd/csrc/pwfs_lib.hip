// pwfs_lib.hip -- host side of the C ABI declared in include/pwfs.h:
// validation, float64 table construction, workspace layout, plans and the
// kernel launches of the FP32 forward model and of the slope stage.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <complex>
#include <new>
#include <string>
#include <vector>

#include "pwfs.h"
#include "pwfs_kernels.hpp"
#include "pwfs_internal.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(PWFS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                 \
  do {                                      \
    hipError_t e__ = (expr);                \
    if (e__ != hipSuccess) return hip_fail(e__, what); \
  } while (0)

bool supported_fft(int n) {
  return n == 64 || n == 128 || n == 256 || n == 384 || n == 512 || n == 768;
}

constexpr double kPi = 3.14159265358979323846264338327950288;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

namespace pwfs {

void set_last_error(const char* msg) { g_err = msg; }

int validate_one(const pwfs_sensor_desc& d, int idx) {
  auto bad = [&](const char* why) { return fail(PWFS_EINVAL, "sensor %d: %s", idx, why); };
  if (d.src_rings < 0 || d.src_rings > 8) return bad("src_rings must be in [0, 8]");
  if (d.src_rings > 0) {
    if (!(d.src_radius_lod >= 0.0) || !std::isfinite(d.src_radius_lod)) return bad("src_radius_lod must be >= 0");
    if (d.precision != PWFS_FP32)
      return fail(PWFS_EUNSUPPORTED, "sensor %d: an extended source needs the FP32 path", idx);
    if ((long long)d.n_mod * (1 + 3LL * d.src_rings * (d.src_rings + 1)) > 8192)
      return bad("modulation points x source points must be <= 8192");
  }
  if (!(d.fov_lod >= 0.0) || !std::isfinite(d.fov_lod)) return bad("fov_lod must be finite and >= 0");
  if (d.flags & ~uint32_t(PWFS_F_REF_SLOPES | PWFS_F_FULL_PLANE | PWFS_F_LOCAL_NORM | PWFS_F_DOUBLE_ROOF))
    return bad("unknown flag bits");
  if (d.n_pupil < 4 || (d.n_pupil & 1)) return bad("n_pupil must be even and >= 4");
  if (d.n_fft < d.n_pupil) return bad("n_fft must be >= n_pupil");
  if ((d.n_fft - d.n_pupil) & 1) return bad("n_fft - n_pupil must be even");
  if (d.n_subap < 1 || d.n_subap > d.n_pupil) return bad("n_subap must be in [1, n_pupil]");
  if (d.n_mod < 1 || d.n_mod > 4096) return bad("n_mod must be in [1, 4096]");
  if (d.n_lambda < 1 || d.n_lambda > PWFS_MAX_LAMBDA) return bad("n_lambda must be in [1, 16]");
  if (!(d.diameter_m > 0.0) || !std::isfinite(d.diameter_m)) return bad("diameter_m must be > 0");
  if (!(d.obstruction >= 0.0 && d.obstruction < 1.0)) return bad("obstruction must be in [0, 1)");
  if (!(d.mod_radius_lod >= 0.0) || !std::isfinite(d.mod_radius_lod)) return bad("mod_radius_lod must be >= 0");
  if (!(d.lambda_ref_nm > 0.0) || !std::isfinite(d.lambda_ref_nm)) return bad("lambda_ref_nm must be > 0");
  double wsum = 0.0;
  for (int l = 0; l < d.n_lambda; ++l) {
    if (!(d.lambda_nm[l] > 0.0) || !std::isfinite(d.lambda_nm[l])) return bad("wavelengths must be > 0");
    if (!(d.lambda_weight[l] >= 0.0) || !std::isfinite(d.lambda_weight[l])) return bad("weights must be >= 0");
    wsum += d.lambda_weight[l];
  }
  if (std::fabs(wsum - 1.0) > 1e-9) return bad("wavelength weights must sum to 1");
  const double S = d.pupil_sep_px;
  if (!std::isfinite(S) || std::fabs(S - std::round(S)) > 1e-9) return bad("pupil_sep_px must be an integer");
  const long Si = std::lround(S);
  if (Si & 1) return bad("pupil_sep_px must be even");
  if (Si < d.n_pupil) return bad("pupil images overlap (pupil_sep_px < n_pupil)");
  if (Si + d.n_pupil > d.n_fft) return bad("pupil images fall outside the grid (pupil_sep_px + n_pupil > n_fft)");
  if (d.precision < PWFS_FP32 || d.precision > PWFS_FP16) return bad("unknown precision");
  if (d.n_subap > 64) return fail(PWFS_EUNSUPPORTED, "sensor %d: n_subap > 64 not supported", idx);
  if (!supported_fft(d.n_fft))
    return fail(PWFS_EUNSUPPORTED, "sensor %d: n_fft %d has no radix plan (64,128,256,384,512,768)", idx, d.n_fft);
  if (d.fov_lod > 0.0 && d.precision != PWFS_FP32)
    return fail(PWFS_EUNSUPPORTED, "sensor %d: the field stop runs in FP32 precision only", idx);
  if ((d.flags & PWFS_F_DOUBLE_ROOF) && d.precision != PWFS_FP32)
    return fail(PWFS_EUNSUPPORTED, "sensor %d: the double roof runs in FP32 precision only", idx);
  if (d.precision != PWFS_FP32 && !mfma_supported(d))
    return fail(PWFS_EUNSUPPORTED, "sensor %d: this precision is not supported for these sizes", idx);
  // at least one valid subaperture
  std::vector<float> A;
  std::vector<uint8_t> V;
  pupil_and_valid(d, A, V);
  int nv = 0;
  for (uint8_t v : V) nv += v;
  if (nv == 0) return bad("no valid subaperture");
  return PWFS_OK;
}

// overlap of pixel y with subaperture i along one axis, in units of 1/n pixel:
// subaperture i spans pixels [i D / n, (i + 1) D / n)
static inline int subap_overlap(int y, int i, int D, int n) {
  return std::max(0, std::min((y + 1) * n, (i + 1) * D) - std::max(y * n, i * D));
}

void pupil_and_valid(const pwfs_sensor_desc& d, std::vector<float>& A, std::vector<uint8_t>& V) {
  const int D = d.n_pupil, n = d.n_subap;
  A.assign((size_t)D * D, 0.f);
  const double R = D / 2.0, Ro = d.obstruction * R;
  for (int y = 0; y < D; ++y)
    for (int x = 0; x < D; ++x) {
      const double cy = y - (D - 1) / 2.0, cx = x - (D - 1) / 2.0;
      const double r2 = cx * cx + cy * cy;
      A[(size_t)y * D + x] = (r2 <= R * R && r2 >= Ro * Ro) ? 1.f : 0.f;
    }
  // valid: at least half of the subaperture's area on lit pixels (areas in
  // units of 1/n^2 pixel are integers; the subaperture's is D^2)
  V.assign((size_t)n * n, 0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      long long lit = 0;
      for (int y = i * D / n; y * n < (i + 1) * D; ++y)
        for (int x = j * D / n; x * n < (j + 1) * D; ++x)
          if (A[(size_t)y * D + x] != 0.f) lit += (long long)subap_overlap(y, i, D, n) * subap_overlap(x, j, D, n);
      V[(size_t)i * n + j] = (2 * lit >= (long long)D * D) ? 1 : 0;
    }
}

// --------------------------------------------------------- tilt points ----
// The tilts the sensor sums over, in lambda/D at lambda_ref: every
// modulation point (radius r_m, angle 2 pi k / n_mod) plus every point of the
// source (a point source: the centre only; an extended source: the centre
// and src_rings rings, ring q at radius rho q / src_rings with 6 q points at
// angles 2 pi j / (6 q)), all with equal weight.  Points whose x-tilts are
// equal by construction (k and n_mod - k; j and 6q - j) get the same key, so
// they share a row transform: the x-tilt of a key is computed once from
// its integer indices.  Points are listed in key order.
void tilt_points(const pwfs_sensor_desc& d, std::vector<TiltPoint>& pts, std::vector<double>& key_tx) {
  const int R = d.src_rings;
  const double rho = R > 0 ? d.src_radius_lod : 0.0;
  // source points: (ring, j, count)
  struct Src {
    int ring, j, m;
  };
  std::vector<Src> src{{0, 0, 1}};
  for (int q = 1; q <= R; ++q)
    for (int j = 0; j < 6 * q; ++j) src.push_back({q, j, 6 * q});
  const int n = d.n_mod;
  // key of an x-tilt: (min(k, n - k), ring, min(j, m - j))
  std::vector<std::array<int, 3>> keys;
  std::vector<std::pair<int, int>> key_of;   // per point: (key index, point order)
  pts.clear();
  key_tx.clear();
  std::vector<TiltPoint> raw;
  std::vector<std::array<int, 3>> raw_key;
  for (int k = 0; k < n; ++k) {
    const int ak = std::min(k, n - k);
    const double cx = d.mod_radius_lod * std::cos(2.0 * kPi * ak / n);
    const double sy = d.mod_radius_lod * std::sin(2.0 * kPi * k / n);
    for (const Src& e : src) {
      const int aj = std::min(e.j, e.m - e.j);
      const double rr = R > 0 ? rho * e.ring / R : 0.0;
      const double tx = cx + rr * std::cos(2.0 * kPi * aj / e.m);
      const double ty = sy + rr * std::sin(2.0 * kPi * e.j / e.m);
      raw.push_back({tx, ty, 0});
      raw_key.push_back({ak, e.ring, aj});
    }
  }
  std::vector<std::array<int, 3>> sorted_keys = raw_key;
  std::sort(sorted_keys.begin(), sorted_keys.end());
  sorted_keys.erase(std::unique(sorted_keys.begin(), sorted_keys.end()), sorted_keys.end());
  std::vector<std::vector<int>> members(sorted_keys.size());
  for (size_t i = 0; i < raw.size(); ++i) {
    const size_t a = std::lower_bound(sorted_keys.begin(), sorted_keys.end(), raw_key[i]) - sorted_keys.begin();
    raw[i].key = (int)a;
    members[a].push_back((int)i);
  }
  for (size_t a = 0; a < sorted_keys.size(); ++a) {
    key_tx.push_back(raw[members[a][0]].tx);
    for (int i : members[a]) pts.push_back(raw[i]);
  }
}

// ----------------------------------------------------------- geometry ----
Geometry geometry(const pwfs_sensor_desc& d) {
  Geometry g;
  g.D = d.n_pupil;
  g.N = d.n_fft;
  g.n = d.n_subap;
  g.b = g.D / g.n;
  g.S = (int)std::lround(d.pupil_sep_px);
  g.Sx = g.Sy = g.S;
  g.o = (g.N - g.D) / 2;
  g.win_lo = g.N / 2 - g.S / 2 - g.D / 2;
  g.win_hi = g.N / 2 + g.S / 2 - g.D / 2;
  g.wy_lo = g.win_lo;
  g.wy_hi = g.win_hi;
  g.full = (d.flags & PWFS_F_FULL_PLANE) ? 1 : 0;
  g.Nc = g.full ? g.N : 2 * g.D;
  g.Dp = (g.D + 15) & ~15;
  g.n_lam = d.n_lambda;
  {
    std::vector<TiltPoint> pts;
    std::vector<double> key_tx;
    tilt_points(d, pts, key_tx);
    g.n_mod = (int)pts.size();
    g.n_a = (int)key_tx.size();
  }
  const int stride0 = g.N / fft_r0(g.N);   // distance between the inputs of a first-stage butterfly
  g.qmax = (g.D + stride0 - 1) / stride0;
  return g;
}

// one arm of a double roof: arm 0 splits along x (images S apart in x, one
// window in y), arm 1 along y; a zero separation on an axis leaves that
// axis's transform pair the identity and its single window at the centre
Geometry arm_geometry(const pwfs_sensor_desc& d, int arm) {
  Geometry g = geometry(d);
  g.Sx = arm == 0 ? g.S : 0;
  g.Sy = arm == 0 ? 0 : g.S;
  g.win_lo = g.N / 2 - g.Sx / 2 - g.D / 2;
  g.win_hi = g.N / 2 + g.Sx / 2 - g.D / 2;
  g.wy_lo = g.N / 2 - g.Sy / 2 - g.D / 2;
  g.wy_hi = g.N / 2 + g.Sy / 2 - g.D / 2;
  if (!g.full) g.Nc = g.Sx ? 2 * g.D : g.D;
  return g;
}

// bytes of each per-sensor region, in workspace order
static void sensor_regions(const pwfs_sensor_desc& d, size_t out[kRegions]) {
  const Geometry g = geometry(d);
  const bool ref = d.flags & PWFS_F_REF_SLOPES;
  out[R_AMP] = sizeof(float) * g.D * g.D;
  out[R_RX] = sizeof(float2) * g.n_lam * g.n_a * g.D;
  out[R_RY] = sizeof(float2) * g.n_lam * g.n_mod * g.D;
  out[R_AK] = sizeof(int) * 2 * g.n_mod;
  const int arms = sensor_arms(d);
  out[R_MROW] = sizeof(float2) * arms * g.n_lam * g.N;
  out[R_MCOL] = sizeof(float2) * arms * g.n_lam * g.N;
  out[R_TW] = sizeof(float2) * g.N;
  out[R_VALID] = (size_t)g.n * g.n;
  out[R_REF] = sizeof(float) * 2 * g.n * g.n;
  out[R_REFINT] = ref ? sizeof(float) * arms * g.N * g.N : 0;
  out[R_ZERO] = ref ? sizeof(float) * g.D * g.D : 0;
  out[R_MFMA] = mfma_table_bytes(d);
}

// per frame: the row-pass output [n_lam][n_a][Nc][Dp], then the pupil field
// [n_lam][D][D] (the field block of a pass sits after all frames' R blocks)
size_t rbuf_frame_bytes(const pwfs_sensor_desc& d) {
  const Geometry g = geometry(d);
  if (d.precision != PWFS_FP32) return mfma_scratch_frame_bytes(d);
  return sizeof(float2) * ((size_t)g.n_lam * g.n_a * g.Nc * g.Dp + (size_t)g.n_lam * g.D * g.D);
}

// float2 offset of the field block of a pass of nf frames
size_t rbuf_field_offset(const pwfs_sensor_desc& d, int nf) {
  const Geometry g = geometry(d);
  return (size_t)nf * g.n_lam * g.n_a * g.Nc * g.Dp;
}

int choose_chunk(const pwfs_sensor_desc* s, int n, int max_frames) {
  // enough frames per pass that the column pass launches >= ~16384 workgroups
  // (16 rounds of the chip's resident workgroups, so a launch's tail is a
  // small part of it), with the scratch of one pass (all sensors) capped at
  // 12 GiB (of the 288 GB of HBM)
  size_t per = 0;
  int want = 1;
  for (int i = 0; i < n; ++i) {
    const Geometry g = geometry(s[i]);
    per += rbuf_frame_bytes(s[i]);
    int colwg;
    if (s[i].precision == PWFS_FP32) {
      const int G = kBlock / fft_lanes(g.N);
      colwg = (g.Nc + G - 1) / G;
    } else {   // matrix-core form: one 128 x 128 tile grid of stage 2 per frame
      colwg = ((2 * g.Nc + 127) / 128) * ((g.Nc + 127) / 128);
    }
    want = std::max(want, (16384 + colwg - 1) / colwg);
  }
  const size_t cap = (size_t)12 << 30;
  int c = std::min(want, max_frames);
  if (per > 0) c = (int)std::min<size_t>((size_t)c, std::max<size_t>(1, cap / per));
  return std::max(1, c);
}

int fft_r0(int N) {
  switch (N) {
    case 64: return FftPlan<64>::r[0];
    case 128: return FftPlan<128>::r[0];
    case 256: return FftPlan<256>::r[0];
    case 384: return FftPlan<384>::r[0];
    case 512: return FftPlan<512>::r[0];
    default: return FftPlan<768>::r[0];
  }
}

int fft_lanes(int N) {
  switch (N) {
    case 64: return FftPlan<64>::T;
    case 128: return FftPlan<128>::T;
    case 256: return FftPlan<256>::T;
    case 384: return FftPlan<384>::T;
    case 512: return FftPlan<512>::T;
    default: return FftPlan<768>::T;
  }
}

int layout(const pwfs_sensor_desc* s, int n, int max_frames, Layout* L) {
  size_t off = 0;
  L->offsets.assign((size_t)n * kRegions, 0);
  for (int i = 0; i < n; ++i) {
    size_t sz[kRegions];
    sensor_regions(s[i], sz);
    for (int r = 0; r < kRegions; ++r) {
      L->offsets[(size_t)i * kRegions + r] = off;
      off += align256(sz[r]);
    }
  }
  L->chunk = choose_chunk(s, n, max_frames);
  // one scratch region per sensor (sensors of a persistent pass run together)
  L->rbuf_offset = off;
  L->sensor_rbuf.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    L->sensor_rbuf[i] = off;
    off += align256(rbuf_frame_bytes(s[i]) * (size_t)L->chunk);
  }
  L->counters_offset = off;
  off += align256(sizeof(int) * 64);
  L->rbuf_bytes = off - L->rbuf_offset;
  L->total = off;
  return PWFS_OK;
}

// ------------------------------------------------------ float64 tables ---
static std::complex<double> cis(double a) { return {std::cos(a), std::sin(a)}; }

// exp(i pi S |u_bar| / N) exp(-2 pi i u o / N) / N, phases reduced exactly;
// zero where 2 |u_bar| > stop (the field stop's side in samples, < 0: none)
static std::vector<double> mask_table(const Geometry& g, int sep, double extra_scale, double stop) {
  std::vector<double> m(2 * (size_t)g.N);
  const long long N = g.N, S = sep;
  for (long long u = 0; u < N; ++u) {
    // |u_bar| * 2 = |2u + 1| below N/2, |2u + 1 - 2N| above
    const long long twice = (u < N / 2) ? (2 * u + 1) : (2 * N - 2 * u - 1);
    if (stop >= 0.0 && (double)twice > stop) {
      m[2 * u] = m[2 * u + 1] = 0.0;
      continue;
    }
    // mask phase pi S twice / (2N) = 2 pi (S twice) / (4N)
    const long long pm = (S * twice) % (4 * N);
    // offset phase -2 pi u o / N = -2 pi (4 u o) / (4N)
    const long long po = (4 * ((u * g.o) % N)) % (4 * N);
    const long long p = ((pm - po) % (4 * N) + 4 * N) % (4 * N);
    const std::complex<double> z = cis(2.0 * kPi * (double)p / (4.0 * (double)N)) * (extra_scale / (double)N);
    m[2 * u] = z.real();
    m[2 * u + 1] = z.imag();
  }
  return m;
}

static void put_c(std::vector<float>& dst, size_t i, std::complex<double> z) {
  dst[2 * i] = (float)z.real();
  dst[2 * i + 1] = (float)z.imag();
}

int upload_tables(const pwfs_sensor_desc& d, char* ws, const size_t* off, hipStream_t st,
                  std::vector<std::vector<char>>& keep, double* sumA2_out) {
  const Geometry g = geometry(d);
  std::vector<float> A;
  std::vector<uint8_t> V;
  pupil_and_valid(d, A, V);
  double sumA2 = 0.0;
  for (float a : A) sumA2 += (double)a * a;
  *sumA2_out = sumA2;

  const double h = -kPi / g.N;  // half-pixel tilt per array index
  std::vector<TiltPoint> pts;
  std::vector<double> key_tx;
  tilt_points(d, pts, key_tx);
  std::vector<float> rx(2 * (size_t)g.n_lam * g.n_a * g.D), ry(2 * (size_t)g.n_lam * g.n_mod * g.D);
  for (int l = 0; l < g.n_lam; ++l) {
    const double sc = d.lambda_ref_nm / d.lambda_nm[l];   // tilts are given at lambda_ref
    for (int a = 0; a < g.n_a; ++a) {
      for (int x = 0; x < g.D; ++x) {
        const double xc = x - (g.D - 1) / 2.0;
        put_c(rx, ((size_t)l * g.n_a + a) * g.D + x, cis(2.0 * kPi * sc * key_tx[a] * xc / g.D + h * (g.o + x)));
      }
    }
    for (int k = 0; k < g.n_mod; ++k) {
      for (int y = 0; y < g.D; ++y) {
        const double yc = y - (g.D - 1) / 2.0;
        put_c(ry, ((size_t)l * g.n_mod + k) * g.D + y, cis(2.0 * kPi * sc * pts[k].ty * yc / g.D + h * (g.o + y)));
      }
    }
  }
  // visiting order: points in key order, so points sharing a row-pass result
  // are back to back; entries are (point, key)
  std::vector<int> ak;
  for (int k = 0; k < g.n_mod; ++k) {
    ak.push_back(k);
    ak.push_back(pts[k].key);
  }
  // masks per arm: the pyramid has one (S on both axes); a double roof has
  // arm x (S along x, 0 along y) then arm y (0, S), each with half the light
  // (the field stop, a fixed sky angle, is narrower in samples at longer
  // wavelengths, so both tables are per wavelength)
  const int arms = sensor_arms(d);
  std::vector<float> mrow(2 * (size_t)arms * g.n_lam * g.N), mcol(2 * (size_t)arms * g.n_lam * g.N);
  std::vector<float> tw(2 * (size_t)g.N);
  for (int a = 0; a < arms; ++a) {
    const Geometry ga = arms == 2 ? arm_geometry(d, a) : g;
    const double share = arms == 2 ? 0.5 : 1.0;
    for (int l = 0; l < g.n_lam; ++l) {
      const double stop = d.fov_lod > 0.0 ? ((d.fov_lod * (d.lambda_ref_nm / d.lambda_nm[l])) * g.N) / g.D : -1.0;
      const size_t at = ((size_t)a * g.n_lam + l) * 2 * g.N;
      const std::vector<double> m = mask_table(ga, ga.Sx, 1.0, stop);
      for (size_t i = 0; i < m.size(); ++i) mrow[at + i] = (float)m[i];
      const double sc = std::sqrt(share * d.lambda_weight[l] / ((double)g.n_mod * sumA2));
      const std::vector<double> mc = mask_table(ga, ga.Sy, sc, stop);
      for (size_t i = 0; i < mc.size(); ++i) mcol[at + i] = (float)mc[i];
    }
  }
  for (int i = 0; i < g.N; ++i) put_c(tw, i, cis(-2.0 * kPi * i / g.N));
  auto up = [&](int region, const void* src, size_t bytes) -> int {
    if (!bytes) return PWFS_OK;
    keep.emplace_back((const char*)src, (const char*)src + bytes);
    HIP_TRY(hipMemcpyAsync(ws + off[region], keep.back().data(), bytes, hipMemcpyHostToDevice, st),
            "hipMemcpyAsync(tables)");
    return PWFS_OK;
  };
  int rc;
  if ((rc = up(R_AMP, A.data(), A.size() * sizeof(float)))) return rc;
  if ((rc = up(R_RX, rx.data(), rx.size() * sizeof(float)))) return rc;
  if ((rc = up(R_RY, ry.data(), ry.size() * sizeof(float)))) return rc;
  if ((rc = up(R_AK, ak.data(), ak.size() * sizeof(int)))) return rc;
  if ((rc = up(R_MROW, mrow.data(), mrow.size() * sizeof(float)))) return rc;
  if ((rc = up(R_MCOL, mcol.data(), mcol.size() * sizeof(float)))) return rc;
  if ((rc = up(R_TW, tw.data(), tw.size() * sizeof(float)))) return rc;
  if ((rc = up(R_VALID, V.data(), V.size()))) return rc;
  if (d.flags & PWFS_F_REF_SLOPES) {
    HIP_TRY(hipMemsetAsync(ws + off[R_ZERO], 0, sizeof(float) * g.D * g.D, st), "hipMemsetAsync(zero)");
  }
  if (d.precision != PWFS_FP32) {
    if ((rc = upload_mfma_tables(d, ws + off[R_MFMA], st, keep, sumA2))) return rc;
  }
  return PWFS_OK;
}

// ---------------------------------------------------- kernel launches ----
// LDS of one row-pass workgroup: the twiddle table (plans that are not
// palindromic), the lane groups' exchange buffers, the transpose tile and one
// spare slot per lane.
template <int N, int RW>
static size_t row_lds_bytes(int Nc) {
  constexpr int T = FftPlan<N>::T, G = kBlock / T;
  return sizeof(float2) * ((Palindromic<N>::value ? 0 : N) + G * BufLen<N>::value + (size_t)Nc * RW + T);
}

// Row tile a sensor runs with: its selection if it is the alternative tile
// of its N, else the default.
template <int N>
static int row_tile_of(const SensorPlan& sp) {
  return sp.row_tile == RowTile<N>::ALT ? RowTile<N>::ALT : RowTile<N>::RW;
}

template <int N>
static bool row_tile_fits(int rw, int Nc) {
  if (rw == RowTile<N>::RW) return row_lds_bytes<N, RowTile<N>::RW>(Nc) <= kMaxLds;
  if (rw == RowTile<N>::ALT) return row_lds_bytes<N, RowTile<N>::ALT>(Nc) <= kMaxLds;
  return false;
}

static int row_tile(const SensorPlan& sp) {
  switch (sp.g.N) {
    case 64: return row_tile_of<64>(sp);
    case 128: return row_tile_of<128>(sp);
    case 256: return row_tile_of<256>(sp);
    case 384: return row_tile_of<384>(sp);
    case 512: return row_tile_of<512>(sp);
    default: return row_tile_of<768>(sp);
  }
}

// Whether `rw` is one of the compiled tiles of N and fits the LDS at Nc columns.
static bool row_tile_ok(int N, int rw, int Nc) {
  switch (N) {
    case 64: return row_tile_fits<64>(rw, Nc);
    case 128: return row_tile_fits<128>(rw, Nc);
    case 256: return row_tile_fits<256>(rw, Nc);
    case 384: return row_tile_fits<384>(rw, Nc);
    case 512: return row_tile_fits<512>(rw, Nc);
    case 768: return row_tile_fits<768>(rw, Nc);
  }
  return false;
}

// Arguments of the three passes of one sensor over `nf` frames.
struct PassArgs {
  FieldArgs fa;
  RowArgs ra;
  ColArgs ca;
  unsigned grid_field, grid_rows, grid_cols, grid_cols_split;
  size_t lds_rows, lds_cols, lds_cols_split;
};

template <int N, int RW>
static PassArgs build_pass(const SensorPlan& sp, const float* opd, long long opd_stride, float* out,
                           long long out_stride, int nf, float2* rbuf, int row_group_target) {
  constexpr int T = FftPlan<N>::T, G = kBlock / T;
  const Geometry& g = sp.g;
  PassArgs pa{};
  float2* field = rbuf + rbuf_field_offset(sp.desc, nf);
  FieldArgs& fa = pa.fa;
  fa.opd = opd;
  fa.amp = (const float*)sp.dev[R_AMP];
  fa.field = field;
  fa.opd_stride = opd_stride;
  fa.D = g.D;
  fa.n_lam = g.n_lam;
  for (int l = 0; l < g.n_lam; ++l) fa.two_pi_over_lam[l] = 2.0 * kPi / sp.desc.lambda_nm[l];
  pa.grid_field = (unsigned)(nf * g.n_lam * ((g.D * g.D + kBlock - 1) / kBlock));

  RowArgs& ra = pa.ra;
  ra.field = field;
  ra.rx = (const float2*)sp.dev[R_RX];
  ra.mrow = (const float2*)sp.dev[R_MROW];
  ra.tw = (const float2*)sp.dev[R_TW];
  ra.rbuf = rbuf;
  ra.D = g.D;
  ra.Dp = g.Dp;
  ra.Nc = g.Nc;
  ra.n_a = g.n_a;
  ra.n_lam = g.n_lam;
  ra.n_la = g.n_lam * g.n_a;
  ra.rowblocks = (g.D + RW - 1) / RW;
  // split the (wavelength, cosine) pairs so a pass has >= row_group_target row groups
  {
    const long long base = (long long)ra.rowblocks * nf;
    const long long want = std::max<long long>(1, (row_group_target + base - 1) / base);
    const int groups = (int)std::min<long long>(ra.n_la, want);
    ra.ag = (ra.n_la + groups - 1) / groups;
    ra.n_agroups = (ra.n_la + ra.ag - 1) / ra.ag;
  }
  ra.win_lo = g.win_lo;
  ra.win_hi = g.win_hi;
  ra.full = g.full;
  constexpr bool PAL = Palindromic<N>::value;   // tables in registers, not LDS
  pa.lds_rows = row_lds_bytes<N, RW>(g.Nc);
  pa.grid_rows = (unsigned)((long long)nf * ra.rowblocks * ra.n_agroups);

  ColArgs& ca = pa.ca;
  ca.rbuf = rbuf;
  ca.ry = (const float2*)sp.dev[R_RY];
  ca.mcol = (const float2*)sp.dev[R_MCOL];
  ca.tw = (const float2*)sp.dev[R_TW];
  ca.kord = (const int2*)sp.dev[R_AK];
  ca.out = out;
  ca.out_stride = out_stride;
  ca.D = g.D;
  ca.Dp = g.Dp;
  ca.Nc = g.Nc;
  ca.n_a = g.n_a;
  ca.n_lam = g.n_lam;
  ca.n_mod = g.n_mod;
  ca.colblocks = (g.Nc + G - 1) / G;
  ca.win_lo = g.win_lo;
  ca.win_hi = g.win_hi;
  ca.wy_lo = g.wy_lo;
  ca.wy_hi = g.wy_hi;
  ca.full = g.full;
  pa.lds_cols = sizeof(float2) * ((PAL ? 0 : (size_t)N) + (size_t)G * BufLen<N>::value);
  pa.grid_cols = (unsigned)(nf * ca.colblocks);
  // split column pass (one column per workgroup): its lane groups' partial sums meet in LDS
  pa.grid_cols_split = (unsigned)(nf * g.Nc);
  pa.lds_cols_split = pa.lds_cols + sizeof(float) * (size_t)G * N;
  return pa;
}

template <int N>
static PassArgs build_pass_rw(const SensorPlan& sp, const float* opd, long long os, float* out, long long ost,
                              int nf, float2* rbuf, int target) {
  if (row_tile_of<N>(sp) == RowTile<N>::ALT)
    return build_pass<N, RowTile<N>::ALT>(sp, opd, os, out, ost, nf, rbuf, target);
  return build_pass<N, RowTile<N>::RW>(sp, opd, os, out, ost, nf, rbuf, target);
}

static PassArgs build_pass_any(const SensorPlan& sp, const float* opd, long long os, float* out, long long ost,
                               int nf, float2* rbuf, int target) {
  switch (sp.g.N) {
    case 64: return build_pass_rw<64>(sp, opd, os, out, ost, nf, rbuf, target);
    case 128: return build_pass_rw<128>(sp, opd, os, out, ost, nf, rbuf, target);
    case 256: return build_pass_rw<256>(sp, opd, os, out, ost, nf, rbuf, target);
    case 384: return build_pass_rw<384>(sp, opd, os, out, ost, nf, rbuf, target);
    case 512: return build_pass_rw<512>(sp, opd, os, out, ost, nf, rbuf, target);
    default: return build_pass_rw<768>(sp, opd, os, out, ost, nf, rbuf, target);
  }
}

// below this many column workgroups (about two per CU) the column pass runs
// split: G workgroups per column instead of one per G columns
constexpr unsigned kColsSplitBelow = 512;

// the flat-axis pass of a double-roof arm (sp.ident): no transforms, the
// same scratch and output layouts as k_rows / k_cols
static IdentArgs ident_args(const SensorPlan& sp, const PassArgs& pa, int nf) {
  const Geometry& g = sp.g;
  IdentArgs ia{};
  ia.field = pa.ra.field;
  ia.rx = pa.ra.rx;
  ia.rbuf = pa.ra.rbuf;
  ia.kord = pa.ca.kord;
  ia.out = pa.ca.out;
  ia.out_stride = pa.ca.out_stride;
  ia.nf = nf;
  ia.D = g.D;
  ia.Dp = g.Dp;
  ia.Nc = g.Nc;
  ia.N = g.N;
  ia.n_a = g.n_a;
  ia.n_lam = g.n_lam;
  ia.n_mod = g.n_mod;
  ia.o = g.o;
  ia.full = g.full;
  ia.win_lo = g.win_lo;
  ia.win_hi = g.win_hi;
  for (int l = 0; l < g.n_lam; ++l)
    ia.w2[l] = (float)(0.5 * sp.desc.lambda_weight[l] / ((double)g.n_mod * sp.sumA2));
  return ia;
}

static unsigned blocks_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <int N, int QM, int RW>
static int launch_fp32(const SensorPlan& sp, const float* opd, long long opd_stride, float* out,
                       long long out_stride, int nf, float2* rbuf, hipStream_t st, Prof* prof) {
  const PassArgs pa = build_pass<N, RW>(sp, opd, opd_stride, out, out_stride, nf, rbuf, 2048);
  int slot = prof->begin(st);
  hipLaunchKernelGGL(k_field, dim3(pa.grid_field), dim3(kBlock), 0, st, pa.fa);
  HIP_TRY(hipGetLastError(), "launch k_field");
  prof->end(slot, st, K_FIELD);
  slot = prof->begin(st);
  if (sp.ident == 2) {
    const IdentArgs ia = ident_args(sp, pa, nf);
    hipLaunchKernelGGL(k_rows_ident, dim3(blocks_for((long long)nf * ia.n_lam * ia.n_a * ia.Nc * ia.D)),
                       dim3(kBlock), 0, st, ia);
  } else {
    hipLaunchKernelGGL((k_rows<N, QM, RW>), dim3(pa.grid_rows), dim3(kBlock), pa.lds_rows, st, pa.ra);
  }
  HIP_TRY(hipGetLastError(), "launch k_rows");
  prof->end(slot, st, K_ROWS);
  slot = prof->begin(st);
  if (sp.ident == 1) {
    const IdentArgs ia = ident_args(sp, pa, nf);
    hipLaunchKernelGGL(k_cols_ident, dim3(blocks_for((long long)nf * ia.Nc * (ia.full ? ia.N : ia.D))),
                       dim3(kBlock), 0, st, ia);
  } else if (pa.grid_cols < kColsSplitBelow)   // few frames: one column per workgroup, more workgroups
    hipLaunchKernelGGL((k_cols<N, QM, true>), dim3(pa.grid_cols_split), dim3(kBlock), pa.lds_cols_split, st, pa.ca);
  else
    hipLaunchKernelGGL((k_cols<N, QM, false>), dim3(pa.grid_cols), dim3(kBlock), pa.lds_cols, st, pa.ca);
  HIP_TRY(hipGetLastError(), "launch k_cols");
  prof->end(slot, st, K_COLS);
  return PWFS_OK;
}

// ------------------------------------------------------- fused pass --------
bool fused_eligible(const SensorPlan& sp) {
  return sp.desc.precision == PWFS_FP32 && sp.arms == 1 && (sp.g.N == 64 || sp.g.N == 128) && sp.g.qmax <= 4;
}

template <int N, int QM>
static int launch_fused(const SensorPlan& sp, const float* opd, long long os, float* out, long long ost, int nf,
                        hipStream_t st, Prof* prof) {
  const Geometry& g = sp.g;
  FusedArgs a{};
  a.opd = opd;
  a.amp = (const float*)sp.dev[R_AMP];
  a.rx = (const float2*)sp.dev[R_RX];
  a.ry = (const float2*)sp.dev[R_RY];
  a.mrow = (const float2*)sp.dev[R_MROW];
  a.mcol = (const float2*)sp.dev[R_MCOL];
  a.tw = (const float2*)sp.dev[R_TW];
  a.kord = (const int2*)sp.dev[R_AK];
  a.out = out;
  a.opd_stride = os;
  a.out_stride = ost;
  a.D = g.D;
  a.Nc = g.Nc;
  a.n_a = g.n_a;
  a.n_lam = g.n_lam;
  a.n_mod = g.n_mod;
  a.full = g.full;
  a.win_lo = g.win_lo;
  a.win_hi = g.win_hi;
  a.wy_lo = g.wy_lo;
  a.wy_hi = g.wy_hi;
  for (int l = 0; l < g.n_lam; ++l) a.two_pi_over_lam[l] = 2.0 * kPi / sp.desc.lambda_nm[l];
  const size_t lds = fused_lds_bytes<N>(g.D, g.Nc, g.full ? g.N : 2 * g.D);
  const int slot = prof->begin(st);
  hipLaunchKernelGGL((k_fused<N, QM>), dim3((unsigned)nf), dim3(kFusedBlock), lds, st, a);
  HIP_TRY(hipGetLastError(), "launch k_fused");
  prof->end(slot, st, K_FUSED);
  return PWFS_OK;
}

template <int N>
static int launch_fused_q(const SensorPlan& sp, const float* opd, long long os, float* out, long long ost, int nf,
                          hipStream_t st, Prof* prof) {
  // D <= N / 2 leaves at most 4 non-zero inputs per first-stage butterfly
  if (sp.g.qmax <= 3) return launch_fused<N, 3>(sp, opd, os, out, ost, nf, st, prof);
  return launch_fused<N, 4>(sp, opd, os, out, ost, nf, st, prof);
}

int forward_fused(const SensorPlan& sp, const float* opd, long long os, float* out, long long ost, int nf,
                  hipStream_t st, Prof* prof) {
  if (sp.g.N == 64) return launch_fused_q<64>(sp, opd, os, out, ost, nf, st, prof);
  if (sp.g.N == 128) return launch_fused_q<128>(sp, opd, os, out, ost, nf, st, prof);
  return fail(PWFS_EUNSUPPORTED, "the fused pass runs N = 64 or 128 only");
}

// ------------------------------------------- persistent heterogeneous pass --
bool hetero_eligible(const SensorPlan& sp) {
  return sp.desc.precision == PWFS_FP32 && sp.g.qmax <= 3 && sp.g.N >= 256 && sp.arms == 1;
}

int forward_hetero(pwfs_plan_s* p, const float* opd, int f0, int nf, float* out, hipStream_t st) {
  HeteroArgs ha{};
  const int ns = (int)p->s.size();
  if (ns > kMaxHetero) return fail(PWFS_EUNSUPPORTED, "persistent mode takes at most %d sensors", kMaxHetero);
  size_t lds = 0;
  std::vector<std::pair<double, int>> cost;
  for (int i = 0; i < ns; ++i) {
    const SensorPlan& sp = p->s[i];
    const PassArgs pa = build_pass_any(sp, opd + sp.opd_offset + (long long)f0 * p->opd_stride,
                                       (long long)p->opd_stride, out + sp.int_offset + (long long)f0 * p->int_stride,
                                       (long long)p->int_stride, nf, sp.rbuf, p->tune.row_groups);
    ha.field[i] = pa.fa;
    ha.rows[i] = pa.ra;
    ha.cols[i] = pa.ca;
    ha.nfft[i] = sp.g.N;
    ha.rw[i] = row_tile(sp);
    ha.n_items[0][i] = (int)pa.grid_field;
    ha.n_items[1][i] = (int)pa.grid_rows;
    ha.n_items[2][i] = (int)pa.grid_cols;
    lds = std::max(lds, std::max(pa.lds_rows, pa.lds_cols));
    cost.push_back({-(double)sp.g.n_mod * sp.g.n_lam * sp.g.N * sp.g.N, i});
  }
  std::sort(cost.begin(), cost.end());
  ha.n_sensors = ns;
  int total = 0;
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < ns; ++i) total += ha.n_items[k][i];
  for (int i = 0; i < ns; ++i) ha.order[i] = cost[i].second;   // largest sensors claim first
  ha.total = total;
  ha.counters = p->counters;
  ha.spin_limit = p->tune.spin_limit != 0 ? p->tune.spin_limit : (1 << 24);
  hipLaunchKernelGGL(k_counter_reset, dim3(1), dim3(64), 0, st, p->counters, kHeteroFlag);
  HIP_TRY(hipGetLastError(), "launch k_counter_reset");
  const int grid = p->n_cu * std::max(1, p->tune.wg_per_cu);
  const int slot = p->prof.begin(st);
  hipLaunchKernelGGL(k_hetero, dim3((unsigned)grid), dim3(kBlock), lds, st, ha);
  HIP_TRY(hipGetLastError(), "launch k_hetero");
  p->prof.end(slot, st, K_HETERO);
  return PWFS_OK;
}

template <int N, int RW>
static int launch_fp32_q(const SensorPlan& sp, const float* opd, long long os, float* out, long long ost,
                         int nf, float2* rbuf, hipStream_t st, Prof* pr) {
  const int q = sp.g.qmax;
  if (q <= 3) return launch_fp32<N, 3, RW>(sp, opd, os, out, ost, nf, rbuf, st, pr);
  if (q == 4) return launch_fp32<N, 4, RW>(sp, opd, os, out, ost, nf, rbuf, st, pr);
  return launch_fp32<N, 8, RW>(sp, opd, os, out, ost, nf, rbuf, st, pr);
}

template <int N>
static int launch_fp32_rw(const SensorPlan& sp, const float* opd, long long os, float* out, long long ost,
                          int nf, float2* rbuf, hipStream_t st, Prof* pr) {
  if (row_tile_of<N>(sp) == RowTile<N>::ALT)
    return launch_fp32_q<N, RowTile<N>::ALT>(sp, opd, os, out, ost, nf, rbuf, st, pr);
  return launch_fp32_q<N, RowTile<N>::RW>(sp, opd, os, out, ost, nf, rbuf, st, pr);
}

int forward_fp32(const SensorPlan& sp, const float* opd, long long os, float* out, long long ost, int nf,
                 float2* rbuf, hipStream_t st, Prof* pr) {
  switch (sp.g.N) {
    case 64: return launch_fp32_rw<64>(sp, opd, os, out, ost, nf, rbuf, st, pr);
    case 128: return launch_fp32_rw<128>(sp, opd, os, out, ost, nf, rbuf, st, pr);
    case 256: return launch_fp32_rw<256>(sp, opd, os, out, ost, nf, rbuf, st, pr);
    case 384: return launch_fp32_rw<384>(sp, opd, os, out, ost, nf, rbuf, st, pr);
    case 512: return launch_fp32_rw<512>(sp, opd, os, out, ost, nf, rbuf, st, pr);
    case 768: return launch_fp32_rw<768>(sp, opd, os, out, ost, nf, rbuf, st, pr);
  }
  return fail(PWFS_EUNSUPPORTED, "n_fft %d", sp.g.N);
}

// Raising the dynamic-LDS limit is advisory: if the runtime refuses it, a
// launch that needs more than the default fails and is reported by
// hipGetLastError at that launch.
static void lds_limit(const void* fn) {
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds) != hipSuccess)
    (void)hipGetLastError();
}

template <int N, int QM>
static int set_lds_limits() {
  lds_limit((const void*)k_rows<N, QM, RowTile<N>::RW>);
  lds_limit((const void*)k_rows<N, QM, RowTile<N>::ALT>);
  lds_limit((const void*)k_cols<N, QM, false>);
  lds_limit((const void*)k_cols<N, QM, true>);
  return PWFS_OK;
}

template <int N>
static int set_lds_limits_q() {
  int rc;
  if ((rc = set_lds_limits<N, 3>())) return rc;
  if ((rc = set_lds_limits<N, 4>())) return rc;
  return set_lds_limits<N, 8>();
}

int prepare_kernels() {
  static bool done = false;
  if (done) return PWFS_OK;
  int rc;
  if ((rc = set_lds_limits_q<64>())) return rc;
  if ((rc = set_lds_limits_q<128>())) return rc;
  if ((rc = set_lds_limits_q<256>())) return rc;
  if ((rc = set_lds_limits_q<384>())) return rc;
  if ((rc = set_lds_limits_q<512>())) return rc;
  if ((rc = set_lds_limits_q<768>())) return rc;
  lds_limit((const void*)k_slopes<kBlock, -1>);
  lds_limit((const void*)k_slopes<1024, -1>);
  lds_limit((const void*)k_slopes<kBlock, 0>);
  lds_limit((const void*)k_slopes<kBlock, 1>);
  lds_limit((const void*)k_slopes<kBlock, 2>);
  lds_limit((const void*)k_slopes<kBlock, 4>);
  lds_limit((const void*)k_slopes<kBlock, 8>);
  lds_limit((const void*)k_slopes<1024, 0>);
  lds_limit((const void*)k_slopes<1024, 1>);
  lds_limit((const void*)k_slopes<1024, 2>);
  lds_limit((const void*)k_slopes<1024, 4>);
  lds_limit((const void*)k_slopes<1024, 8>);
  lds_limit((const void*)k_hetero);
  lds_limit((const void*)k_fused<64, 3>);
  lds_limit((const void*)k_fused<64, 4>);
  lds_limit((const void*)k_fused<128, 3>);
  lds_limit((const void*)k_fused<128, 4>);
  done = true;
  return PWFS_OK;
}

// below this many frames the slope stage runs 1024 threads per frame
constexpr int kSlopesWideBelow = 64;

int slopes_launch_at(const SensorPlan& sp, const float* in, long long in_stride, float* slopes,
                     long long slope_stride, float* flux, long long flux_stride, const float* ref, int nf, int n_in,
                     int img, const int* org_r, const int* org_c, hipStream_t st, Prof* prof) {
  const Geometry& g = sp.g;
  SlopeArgs a{};
  a.in = in;
  a.slopes = slopes;
  a.flux = flux;
  a.valid = (const uint8_t*)sp.dev[R_VALID];
  a.ref = ref;
  a.in_stride = in_stride;
  a.slope_stride = slope_stride;
  a.flux_stride = flux_stride;
  a.N = n_in;
  a.n = g.n;
  a.img = img;
  a.b = img / g.n;
  const int b = (img % g.n) ? -1 : a.b;     // -1: subapertures cut pixels
  a.n_valid = sp.n_valid;
  a.local_norm = (sp.desc.flags & PWFS_F_LOCAL_NORM) ? 1 : 0;
  a.roof = sp.arms == 2 ? 1 : 0;
  for (int q = 0; q < 4; ++q) {
    a.org_r[q] = org_r[q];
    a.org_c[q] = org_c[q];
  }
  const size_t lds = sizeof(float) * 4 * g.n * g.n;
  const int slot = prof ? prof->begin(st) : -1;
  const bool wide = nf < kSlopesWideBelow;
  const dim3 grid((unsigned)nf), block(wide ? 1024 : kBlock);
  switch ((wide ? 100 : 0) + (b == 1 || b == 2 || b == 4 || b == 8 || b == -1 ? b : 0)) {
    case -1: hipLaunchKernelGGL((k_slopes<kBlock, -1>), grid, block, lds, st, a); break;
    case 99: hipLaunchKernelGGL((k_slopes<1024, -1>), grid, block, lds, st, a); break;
    case 1: hipLaunchKernelGGL((k_slopes<kBlock, 1>), grid, block, lds, st, a); break;
    case 2: hipLaunchKernelGGL((k_slopes<kBlock, 2>), grid, block, lds, st, a); break;
    case 4: hipLaunchKernelGGL((k_slopes<kBlock, 4>), grid, block, lds, st, a); break;
    case 8: hipLaunchKernelGGL((k_slopes<kBlock, 8>), grid, block, lds, st, a); break;
    case 0: hipLaunchKernelGGL((k_slopes<kBlock, 0>), grid, block, lds, st, a); break;
    case 101: hipLaunchKernelGGL((k_slopes<1024, 1>), grid, block, lds, st, a); break;
    case 102: hipLaunchKernelGGL((k_slopes<1024, 2>), grid, block, lds, st, a); break;
    case 104: hipLaunchKernelGGL((k_slopes<1024, 4>), grid, block, lds, st, a); break;
    case 108: hipLaunchKernelGGL((k_slopes<1024, 8>), grid, block, lds, st, a); break;
    default: hipLaunchKernelGGL((k_slopes<1024, 0>), grid, block, lds, st, a); break;
  }
  HIP_TRY(hipGetLastError(), "launch k_slopes");
  if (prof) prof->end(slot, st, K_SLOPES);
  return PWFS_OK;
}

int slopes_launch(const SensorPlan& sp, const float* in, long long in_stride, float* slopes, long long slope_stride,
                  float* flux, long long flux_stride, const float* ref, int nf, hipStream_t st, Prof* prof) {
  const Geometry& g = sp.g;
  int org_r[4], org_c[4];
  if (sp.arms == 2) {
    // the two planes as one 2N x N array: arm x's images left and right of
    // centre in plane 0, arm y's above and below in plane 1
    const int c = g.N / 2 - g.D / 2;
    for (int q = 0; q < 2; ++q) {
      const int sgn = q ? 1 : -1;
      org_r[q] = c;
      org_c[q] = g.N / 2 + sgn * g.S / 2 - g.D / 2;
      org_r[2 + q] = g.N + g.N / 2 + sgn * g.S / 2 - g.D / 2;
      org_c[2 + q] = c;
    }
  } else {
    int q = 0;
    for (int sy = -1; sy <= 1; sy += 2)
      for (int sx = -1; sx <= 1; sx += 2, ++q) {
        org_r[q] = g.N / 2 + sy * g.S / 2 - g.D / 2;
        org_c[q] = g.N / 2 + sx * g.S / 2 - g.D / 2;
      }
  }
  return slopes_launch_at(sp, in, in_stride, slopes, slope_stride, flux, flux_stride, ref, nf, g.N, g.D, org_r, org_c,
                          st, prof);
}

}  // namespace pwfs

// ===================================================================== ABI ==
using namespace pwfs;

extern "C" {

const char* pwfs_last_error(void) { return g_err.c_str(); }

int pwfs_validate(const pwfs_sensor_desc* s, int n) {
  g_err.clear();
  if (!s) return fail(PWFS_EINVAL, "sensors is NULL");
  if (n < 1 || n > 64) return fail(PWFS_EINVAL, "n_sensors must be in [1, 64]");
  for (int i = 0; i < n; ++i) {
    const int rc = validate_one(s[i], i);
    if (rc) return rc;
  }
  return PWFS_OK;
}

int pwfs_workspace_size(const pwfs_sensor_desc* s, int n, int max_frames, size_t* bytes) {
  int rc = pwfs_validate(s, n);
  if (rc) return rc;
  if (!bytes) return fail(PWFS_EINVAL, "bytes is NULL");
  if (max_frames < 1) return fail(PWFS_EINVAL, "max_frames must be >= 1");
  Layout L;
  layout(s, n, max_frames, &L);
  *bytes = L.total;
  return PWFS_OK;
}

int pwfs_plan(const pwfs_sensor_desc* s, int n, int max_frames, void* ws, size_t ws_bytes, void* stream,
              pwfs_plan_t* out) {
  int rc = pwfs_validate(s, n);
  if (rc) return rc;
  if (!out) return fail(PWFS_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_frames < 1) return fail(PWFS_EINVAL, "max_frames must be >= 1");
  if (!ws) return fail(PWFS_EWORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws & 255) return fail(PWFS_EWORKSPACE, "workspace must be 256-byte aligned");
  Layout L;
  layout(s, n, max_frames, &L);
  if (ws_bytes < L.total)
    return fail(PWFS_EWORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  if ((rc = prepare_kernels())) return rc;
  hipStream_t st = (hipStream_t)stream;

  pwfs_plan_s* p = new (std::nothrow) pwfs_plan_s();
  if (!p) return fail(PWFS_EINVAL, "out of host memory");
  p->max_frames = max_frames;
  p->chunk = L.chunk;
  p->max_chunk = L.chunk;
  p->tune.mode = PWFS_MODE_LAUNCHES;
  p->tune.chunk = L.chunk;
  p->tune.wg_per_cu = 2;
  p->tune.row_groups = 2048;
  p->tune.max_chunk = L.chunk;
  p->ws = (char*)ws;
  p->ws_bytes = ws_bytes;
  p->rbuf = (float2*)((char*)ws + L.rbuf_offset);
  p->counters = (int*)((char*)ws + L.counters_offset);
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
      p->n_cu = ncu;
  }
  size_t opd = 0, inten = 0, sl = 0;
  std::vector<std::vector<char>> keep;
  for (int i = 0; i < n; ++i) {
    SensorPlan sp;
    sp.desc = s[i];
    sp.g = geometry(s[i]);
    sp.arms = sensor_arms(s[i]);
    for (int a = 0; a < sp.arms; ++a) sp.arm_g[a] = arm_geometry(s[i], a);
    for (int r = 0; r < kRegions; ++r) sp.dev[r] = (char*)ws + L.offsets[(size_t)i * kRegions + r];
    sp.rbuf = (float2*)((char*)ws + L.sensor_rbuf[i]);
    std::vector<float> A;
    std::vector<uint8_t> V;
    pupil_and_valid(s[i], A, V);
    sp.n_valid = 0;
    for (uint8_t v : V) sp.n_valid += v;
    sp.valid_host = V;
    sp.opd_offset = opd;
    sp.int_offset = inten;
    sp.slope_offset = sl;
    opd += (size_t)sp.g.D * sp.g.D;
    inten += (size_t)sp.arms * sp.g.N * sp.g.N;
    sl += 2 * (size_t)sp.g.n * sp.g.n;
    if ((rc = upload_tables(s[i], (char*)ws, &L.offsets[(size_t)i * kRegions], st, keep, &sp.sumA2))) {
      (void)hipStreamSynchronize(st);
      delete p;
      return rc;
    }
    p->s.push_back(sp);
  }
  p->opd_stride = opd;
  p->int_stride = inten;
  p->slope_stride = sl;
  // the persistent pass's counters and its sticky error flag start at zero
  hipLaunchKernelGGL(k_counter_reset, dim3(1), dim3(64), 0, st, p->counters, 64);
  if (hipError_t e0 = hipGetLastError(); e0 != hipSuccess) {
    (void)hipStreamSynchronize(st);
    delete p;
    return hip_fail(e0, "launch k_counter_reset");
  }
  // reference slopes of a flat wavefront, sensor by sensor
  for (int i = 0; i < n && rc == 0; ++i) {
    const SensorPlan& sp = p->s[i];
    if (!(sp.desc.flags & PWFS_F_REF_SLOPES)) continue;
    float* I = (float*)sp.dev[R_REFINT];
    rc = forward_sensor(p, i, (const float*)sp.dev[R_ZERO], 0, I, 0, 1, st);
    if (!rc)
      rc = slopes_launch(sp, I, 0, (float*)sp.dev[R_REF], 0, nullptr, 0, nullptr, 1, st, nullptr);
  }
  hipError_t e = hipStreamSynchronize(st);
  if (rc) {
    delete p;
    return rc;
  }
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipStreamSynchronize(plan)");
  }
  *out = p;
  return PWFS_OK;
}

int pwfs_forward(pwfs_plan_t p, const float* opd, int nf, float* out, void* stream) {
  if (!p) return fail(PWFS_EINVAL, "plan is NULL");
  if (!opd || !out) return fail(PWFS_EINVAL, "NULL device pointer");
  if (nf < 1 || nf > p->max_frames)
    return fail(PWFS_ESTATE, "n_frames %d outside [1, max_frames=%d]", nf, p->max_frames);
  hipStream_t st = (hipStream_t)stream;
  if (p->tune.mode == PWFS_MODE_PERSISTENT) {
    for (int f0 = 0; f0 < nf; f0 += p->chunk) {
      const int rc = forward_hetero(p, opd, f0, std::min(p->chunk, nf - f0), out, st);
      if (rc) return rc;
    }
    return PWFS_OK;
  }
  for (size_t i = 0; i < p->s.size(); ++i) {
    const SensorPlan& sp = p->s[i];
    const int rc = forward_sensor(p, (int)i, opd + sp.opd_offset, (long long)p->opd_stride,
                                  out + sp.int_offset, (long long)p->int_stride, nf, st);
    if (rc) return rc;
  }
  return PWFS_OK;
}

int pwfs_get_tuning(pwfs_plan_t p, pwfs_tuning* t) {
  if (!p || !t) return fail(PWFS_EINVAL, "NULL argument");
  *t = p->tune;
  t->max_chunk = p->max_chunk;
  return PWFS_OK;
}

int pwfs_set_tuning(pwfs_plan_t p, const pwfs_tuning* t) {
  if (!p || !t) return fail(PWFS_EINVAL, "NULL argument");
  if (t->mode != PWFS_MODE_LAUNCHES && t->mode != PWFS_MODE_PERSISTENT && t->mode != PWFS_MODE_FUSED)
    return fail(PWFS_EINVAL, "unknown mode");
  if (t->chunk < 1 || t->chunk > p->max_chunk)
    return fail(PWFS_EINVAL, "chunk must be in [1, %d] (the workspace's pass size)", p->max_chunk);
  if (t->wg_per_cu < 1 || t->wg_per_cu > 8) return fail(PWFS_EINVAL, "wg_per_cu must be in [1, 8]");
  if (t->row_groups < 1 || t->row_groups > (1 << 20)) return fail(PWFS_EINVAL, "row_groups out of range");
  if (t->reserved[0] != 0 || t->reserved[1] != 0) return fail(PWFS_EINVAL, "reserved fields must be 0");
  if (t->mode == PWFS_MODE_FUSED) {
    for (const SensorPlan& sp : p->s)
      if (!fused_eligible(sp))
        return fail(PWFS_EUNSUPPORTED, "the fused pass needs FP32 pyramid sensors with N = 64 or 128");
  }
  if (t->mode == PWFS_MODE_PERSISTENT) {
    if ((int)p->s.size() > kMaxHetero) return fail(PWFS_EUNSUPPORTED, "persistent mode takes at most 8 sensors");
    for (const SensorPlan& sp : p->s)
      if (!hetero_eligible(sp))
        return fail(PWFS_EUNSUPPORTED,
                    "persistent mode needs FP32 pyramid sensors with N >= 256 and few non-zero first-stage inputs");
  }
  p->tune = *t;
  p->tune.max_chunk = p->max_chunk;
  p->chunk = t->chunk;
  return PWFS_OK;
}

int pwfs_set_row_tile(pwfs_plan_t p, int sensor, int rows) {
  if (!p) return fail(PWFS_EINVAL, "plan is NULL");
  if (sensor < 0 || sensor >= (int)p->s.size()) return fail(PWFS_EINVAL, "sensor %d out of range", sensor);
  SensorPlan& sp = p->s[sensor];
  if (rows == 0) {
    sp.row_tile = 0;
    return PWFS_OK;
  }
  if (sp.desc.precision != PWFS_FP32)
    return fail(PWFS_EUNSUPPORTED, "the row tile applies to the FP32 path only");
  int nc = sp.g.Nc;
  for (int a = 0; a < sp.arms; ++a) nc = std::max(nc, sp.arm_g[a].Nc);
  if (!row_tile_ok(sp.g.N, rows, nc))
    return fail(PWFS_EINVAL, "row tile %d is not compiled for N = %d or does not fit the LDS at %d columns", rows,
                sp.g.N, nc);
  sp.row_tile = rows;
  return PWFS_OK;
}

int pwfs_get_row_tile(pwfs_plan_t p, int sensor, int* rows) {
  if (!p || !rows) return fail(PWFS_EINVAL, "NULL argument");
  if (sensor < 0 || sensor >= (int)p->s.size()) return fail(PWFS_EINVAL, "sensor %d out of range", sensor);
  *rows = row_tile(p->s[sensor]);
  return PWFS_OK;
}

int pwfs_device_status(pwfs_plan_t p, void* stream) {
  if (!p) return fail(PWFS_EINVAL, "plan is NULL");
  hipStream_t st = (hipStream_t)stream;
  int flag = 0;
  const int zero = 0;
  HIP_TRY(hipMemcpyAsync(&flag, p->counters + kHeteroFlag, sizeof(int), hipMemcpyDeviceToHost, st),
          "hipMemcpyAsync(status)");
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize(status)");
  if (!flag) return PWFS_OK;
  HIP_TRY(hipMemcpyAsync(p->counters + kHeteroFlag, &zero, sizeof(int), hipMemcpyHostToDevice, st),
          "hipMemcpyAsync(status clear)");
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize(status clear)");
  return fail(PWFS_EHIP,
              "a dependency wait of a persistent pass gave up (spin limit %d): the intensities of the calls since "
              "the last status check may be incomplete",
              p->tune.spin_limit != 0 ? p->tune.spin_limit : (1 << 24));
}

int pwfs_slopes(pwfs_plan_t p, const float* in, int nf, float* slopes, float* flux, void* stream) {
  if (!p) return fail(PWFS_EINVAL, "plan is NULL");
  if (!in || !slopes) return fail(PWFS_EINVAL, "NULL device pointer");
  if (nf < 1 || nf > p->max_frames)
    return fail(PWFS_ESTATE, "n_frames %d outside [1, max_frames=%d]", nf, p->max_frames);
  hipStream_t st = (hipStream_t)stream;
  const long long ns = (long long)p->s.size();
  for (size_t i = 0; i < p->s.size(); ++i) {
    const SensorPlan& sp = p->s[i];
    const float* ref = (sp.desc.flags & PWFS_F_REF_SLOPES) ? (const float*)sp.dev[R_REF] : nullptr;
    const int rc = slopes_launch(sp, in + sp.int_offset, (long long)p->int_stride, slopes + sp.slope_offset,
                                 (long long)p->slope_stride, flux ? flux + i : nullptr, ns, ref, nf, st, &p->prof);
    if (rc) return rc;
  }
  return PWFS_OK;
}

int pwfs_query(pwfs_plan_t p, int sensor, pwfs_sensor_info* info) {
  if (!p || !info) return fail(PWFS_EINVAL, "NULL argument");
  if (sensor < 0 || sensor >= (int)p->s.size()) return fail(PWFS_EINVAL, "sensor index out of range");
  const SensorPlan& sp = p->s[sensor];
  info->n_pupil = sp.g.D;
  info->n_fft = sp.g.N;
  info->n_subap = sp.g.n;
  info->n_valid = sp.n_valid;
  info->opd_offset = sp.opd_offset;
  info->intensity_offset = sp.int_offset;
  info->slope_offset = sp.slope_offset;
  info->opd_stride = p->opd_stride;
  info->intensity_stride = p->int_stride;
  info->slope_stride = p->slope_stride;
  return PWFS_OK;
}

int pwfs_valid_map(pwfs_plan_t p, int sensor, uint8_t* host_out) {
  if (!p || !host_out) return fail(PWFS_EINVAL, "NULL argument");
  if (sensor < 0 || sensor >= (int)p->s.size()) return fail(PWFS_EINVAL, "sensor index out of range");
  const std::vector<uint8_t>& v = p->s[sensor].valid_host;
  std::memcpy(host_out, v.data(), v.size());
  return PWFS_OK;
}

static void prof_release(Prof& pr) {
  for (hipEvent_t e : pr.ev) (void)hipEventDestroy(e);
  pr.ev.clear();
  pr.kid.clear();
  pr.used = 0;
  pr.on = false;
}

int pwfs_profile(pwfs_plan_t p, int max_launches) {
  if (!p) return fail(PWFS_EINVAL, "plan is NULL");
  prof_release(p->prof);
  if (max_launches <= 0) return PWFS_OK;
  if (max_launches > (1 << 20)) return fail(PWFS_EINVAL, "max_launches too large");
  p->prof.ev.resize(2 * (size_t)max_launches);
  p->prof.kid.assign((size_t)max_launches, -1);
  for (auto& e : p->prof.ev) {
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) {
      e = nullptr;
      prof_release(p->prof);
      return hip_fail(err, "hipEventCreate");
    }
  }
  p->prof.on = true;
  return PWFS_OK;
}

int pwfs_profile_read(pwfs_plan_t p, int kernel, double* total_ms, int* launches) {
  if (!p || !total_ms || !launches) return fail(PWFS_EINVAL, "NULL argument");
  double t = 0.0;
  int n = 0;
  for (int i = 0; i < p->prof.used; ++i) {
    if (p->prof.kid[i] != kernel) continue;
    HIP_TRY(hipEventSynchronize(p->prof.ev[2 * i + 1]), "hipEventSynchronize");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p->prof.ev[2 * i], p->prof.ev[2 * i + 1]), "hipEventElapsedTime");
    t += ms;
    ++n;
  }
  *total_ms = t;
  *launches = n;
  return PWFS_OK;
}

void pwfs_destroy(pwfs_plan_t p) {
  if (!p) return;
  prof_release(p->prof);
  delete p;
}

}  // extern "C"

namespace pwfs {

int forward_sensor(pwfs_plan_s* p, int i, const float* opd, long long opd_stride, float* out,
                   long long out_stride, int nf, hipStream_t st) {
  const SensorPlan& sp = p->s[i];
  // the fused pass needs no scratch: every frame in one launch
  if (p->tune.mode == PWFS_MODE_FUSED && fused_eligible(sp))
    return forward_fused(sp, opd, opd_stride, out, out_stride, nf, st, &p->prof);
  for (int f0 = 0; f0 < nf; f0 += p->chunk) {
    const int n = std::min(p->chunk, nf - f0);
    const float* o = opd + (long long)f0 * opd_stride;
    float* r = out + (long long)f0 * out_stride;
    int rc;
    if (sp.arms == 2) {
      // double roof: each arm is a pass of its own with its masks and windows,
      // into its own plane; the two share the pass scratch in stream order
      for (int a = 0; a < 2; ++a) {
        SensorPlan arm = sp;
        arm.g = sp.arm_g[a];
        // with no field stop the flat axis is the identity: arm x skips its
        // column transforms, arm y its row transforms
        arm.ident = sp.desc.fov_lod > 0.0 ? 0 : (a == 0 ? 1 : 2);
        arm.dev[R_MROW] = (char*)sp.dev[R_MROW] + sizeof(float2) * (size_t)a * sp.g.n_lam * sp.g.N;
        arm.dev[R_MCOL] = (char*)sp.dev[R_MCOL] + sizeof(float2) * (size_t)a * sp.g.n_lam * sp.g.N;
        rc = forward_fp32(arm, o, opd_stride, r + (size_t)a * sp.g.N * sp.g.N, out_stride, n, sp.rbuf, st,
                          &p->prof);
        if (rc) return rc;
      }
      continue;
    }
    if (sp.desc.precision == PWFS_FP32)
      rc = forward_fp32(sp, o, opd_stride, r, out_stride, n, sp.rbuf, st, &p->prof);
    else
      rc = forward_mfma(sp, o, opd_stride, r, out_stride, n, sp.rbuf, st, &p->prof);
    if (rc) return rc;
  }
  return PWFS_OK;
}

}  // namespace pwfs
