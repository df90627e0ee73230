// pwfs_kernels.hpp -- HIP kernels of the FP32 pyramid-sensor forward model
// and of the slope stage, for gfx950.
//
// The 2-D chain of one modulation point (pad, DFT2, separable mask, IDFT2)
// factors into a row transform and a column transform because the mask and
// the tilts are separable.  The row transform of pupil row y,
//     R_a[y][X] = IDFT_x( m'(u) DFT_x( E0[y][x] rx_a[x] ) ),
// depends on the modulation point only through a = cos(theta_k) (points k and
// n_mod - k share it), so it is computed once per distinct a.  The column
// transform of column X for point k,
//     e_k[Y][X] = IDFT_y( m'(v) DFT_y( ry_k[y] R_a(k)[y][X] ) ),
// is where |e|^2 accumulates over k and wavelength in registers.  Only the D
// non-zero input rows/columns are transformed (the pupil offset is folded
// into the mask m'), and in window mode only the 2D image columns of R and
// the 2D image rows of e are kept.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_device.hpp"
#include "pwfs.h"
#include "pwfs_geom.hpp"

namespace pwfs {

constexpr int kBlock = 256;  // threads per workgroup (4 wavefronts)
constexpr size_t kMaxLds = 160 * 1024;   // LDS a workgroup may hold on gfx950

// Rows of one row-pass workgroup tile: the default RW and the alternative
// ALT that a plan may select per sensor (pwfs_set_row_tile).  A taller tile
// writes longer contiguous segments of the row-pass output (RW x 8 bytes per
// column) but holds more LDS, so fewer workgroups fit on a compute unit.
template <int N> struct RowTile { static constexpr int RW = 8, ALT = 16; };
template <> struct RowTile<64> { static constexpr int RW = 32, ALT = 32; };
template <> struct RowTile<128> { static constexpr int RW = 16, ALT = 16; };
template <> struct RowTile<384> { static constexpr int RW = 16, ALT = 8; };

// Slot of element (column xc, row yl) in the row pass's transpose tile
// [Nc][RW].  Rows are unpadded; the row index is XOR-swizzled by bits of xc
// so that a wavefront writing one yl for consecutive xc (the FFT output) and
// one that reads whole rows in order (the coalesced copy-out) both hit
// distinct 8-byte slots in every 16- or 32-lane LDS cycle.
template <int RW>
__device__ __forceinline__ int tile_slot(int xc, int yl) {
  static_assert(RW == 8 || RW == 16 || RW == 32, "row tile");
  int sw;
  if constexpr (RW == 8) sw = ((xc >> 1) & 7) ^ ((xc >> 4) & 1);
  else if constexpr (RW == 16) sw = (xc & 15) ^ ((xc >> 4) & 1);
  else sw = xc & 31;
  return xc * RW + (yl ^ sw);
}

struct FieldArgs {
  const float* opd;        // sensor's first frame of the chunk; frame stride opd_stride
  const float* amp;        // [D][D] pupil amplitude
  float2* field;           // [frames][n_lam][D][D]
  long long opd_stride;
  int D, n_lam;
  double two_pi_over_lam[PWFS_MAX_LAMBDA];
};

struct RowArgs {
  const float2* field;     // [frames][n_lam][D][D] pupil field A exp(i phi)
  const float2* rx;        // [n_lam][n_a][D] row tilt (modulation x-part, half-pixel tilt)
  const float2* mrow;      // [n_lam][N] row mask with pupil-offset phase and 1/N
  const float2* tw;        // [N] exp(-2 pi i n / N)
  float2* rbuf;            // [frames][n_lam][n_a][Nc][Dp]
  int D, Dp, Nc, n_a, n_lam, n_la, ag, n_agroups, rowblocks;
  int win_lo, win_hi, full;
};

struct ColArgs {
  const float2* rbuf;      // as written by the row pass
  const float2* ry;        // [n_lam][n_mod][D] column tilt
  const float2* mcol;      // [n_lam][N] column mask, offset phase, 1/N, sqrt(weight)
  const float2* tw;        // [N]
  const int2* kord;        // [n_points] (tilt point, its x-tilt key), points sharing a key adjacent
  float* out;              // sensor's first frame of the chunk; frame stride out_stride
  long long out_stride;
  int D, Dp, Nc, n_a, n_lam, n_mod, colblocks;
  int win_lo, win_hi, full;   // column windows (as in the row pass)
  int wy_lo, wy_hi;           // row windows
};

struct SlopeArgs {
  const float* in;         // intensity of the sensor's first frame, frame stride in_stride
  float* slopes;           // [frame][slope_stride], sensor block [2][n][n]
  float* flux;             // [frame][flux_stride] or nullptr
  const uint8_t* valid;    // [n][n]
  const float* ref;        // [2][n][n] or nullptr
  long long in_stride, slope_stride, flux_stride;
  int N, n, b, img, n_valid, local_norm;   // b = img / n (whole subapertures)
  int roof;                // double roof: s_x from images 0, 1, s_y from 2, 3, each over its arm's flux
  int org_r[4], org_c[4];  // image origins
};

// ------------------------------------------------------ FFT pair core ----
// One lane-group's "transform, mask, inverse transform" on a row or column
// held in registers.  Palindromic plans keep twiddles and the mask in
// registers and exchange through a padded buffer; the others read the LDS
// twiddle table and use an unpadded buffer.
template <int N>
struct BufLen {
  static constexpr int value = Palindromic<N>::value ? PaddedLen<N>::value : N;
};

template <int N, int QM>
struct FftPair {
  static constexpr bool PAL = Palindromic<N>::value;
  static constexpr int T = FftPlan<N>::T, V = N / T;
  static constexpr int RLAST = FftPlan<N>::r[FftPlan<N>::NS - 1];
  TwSet<N> tw;
  float2 m[V];
  const float2* s_tw;
  float2* buf;
  int t;

  __device__ __forceinline__ void init(int lane, float2* group_buf, const float2* twiddles) {
    t = lane;
    buf = group_buf;
    s_tw = twiddles;
    if constexpr (PAL) tw.load(t, twiddles);
  }
  // mask values of this lane's frequency slots
  __device__ __forceinline__ void set_mask(const float2* mask) {
#pragma unroll
    for (int s = 0; s < V; ++s) m[s] = mask[freq_index<N>(t, s)];
  }
  __device__ __forceinline__ void run(float2* v) {
    if constexpr (PAL) {
      fft_reg<N, false, 0, QM>(v, t, buf, tw);
#pragma unroll
      for (int s = 0; s < V; ++s) v[s] = cmul(v[s], m[s]);
      fft_reg<N, true, 0, RLAST>(v, t, buf, tw);
    } else {
      fft_from<N, false, 0, QM>(v, t, buf, s_tw);
#pragma unroll
      for (int s = 0; s < V; ++s) v[s] = cmul(v[s], m[s]);
      fft_from<N, true, 0, RLAST>(v, t, buf, s_tw);
    }
  }
};

// --------------------------------------------------------------- field ----
// E0 = A exp(i 2 pi OPD / lambda): phase formed and reduced to [-pi, pi] in
// float64, then float32 sincos.
__device__ __forceinline__ void field_body(const FieldArgs& p, int bid) {
  const int DD = p.D * p.D;
  const int blocks = (DD + kBlock - 1) / kBlock;
  const int b = bid % blocks;
  const int fl = bid / blocks;            // frame * n_lam + lam
  const int lam = fl % p.n_lam, f = fl / p.n_lam;
  const int i = b * kBlock + threadIdx.x;
  if (i >= DD) return;
  const double ph = (double)p.opd[(long long)f * p.opd_stride + i] * p.two_pi_over_lam[lam];
  const double n = rint(ph * 0.15915494309189533577);
  const float r = (float)fma(-n, 6.283185307179586477, ph);
  float sn, cs;
  sincosf(r, &sn, &cs);
  const float a = p.amp[i];
  p.field[(size_t)fl * DD + i] = make_float2(a * cs, a * sn);
}

__global__ __launch_bounds__(kBlock) void k_field(FieldArgs p) { field_body(p, blockIdx.x); }

// ---------------------------------------------------------------- rows ----
template <int N, int QM_, int RW>
__device__ __forceinline__ void rows_body(const RowArgs& p, int bid, float2* smem, int tid) {
  using P = FftPlan<N>;
  constexpr int T = P::T, V = N / T, R0 = P::r[0], NB0 = V / R0, G = kBlock / T;
  constexpr int QM = QM_ < R0 ? QM_ : R0;
  constexpr int RPG = RW / G, BL = BufLen<N>::value, NL = NB0 * QM;
  static_assert(RPG >= 1 && RW % G == 0, "row tile");

  // palindromic plans take twiddles straight into registers; the others keep
  // the twiddle table in LDS.  The row mask of each wavelength goes from its
  // table to registers as the wavelength starts.
  constexpr bool PAL = Palindromic<N>::value;
  float2* s_tw = smem;
  float2* s_buf = s_tw + (PAL ? 0 : N);
  float2* s_tile = s_buf + G * BL;

  const int g = tid / T, t = tid % T;
  const int agi = bid % p.n_agroups;
  bid /= p.n_agroups;
  const int rb = bid % p.rowblocks;
  const int f = bid / p.rowblocks;
  const int y0 = rb * RW;
  const int la0 = agi * p.ag;
  const int la1 = min(la0 + p.ag, p.n_la);

  FftPair<N, QM> fp;
  if constexpr (PAL) {
    fp.init(t, s_buf + g * BL, p.tw);
  } else {
    for (int i = tid; i < N; i += kBlock) s_tw[i] = p.tw[i];
    __syncthreads();
    fp.init(t, s_buf + g * BL, s_tw);
  }
  int lam_mask = -1;

  // this lane's input columns
  int xx[NL];
  bool xin[NL];
#pragma unroll
  for (int i = 0; i < NB0; ++i)
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      const int x = t + T * i + q * (N / R0);
      xx[i * QM + q] = min(x, p.D - 1);
      xin[i * QM + q] = x < p.D;
    }

  // With one wavelength the field rows of this lane group are the same for
  // every (wavelength, cosine) pair of the workgroup.  Where they are few
  // registers (HOLD) they are loaded once and kept; otherwise each row is
  // loaded for each pair, the next row prefetched during the current
  // transform.  The row tilt of the next pair is prefetched either way.
  // outputs outside the image windows go to a per-lane spare slot past the
  // tile, so the tile writes need no branches
  const int spare = p.Nc * RW + t;
  constexpr bool HOLD = RPG * NL <= 8;
  constexpr int NH = HOLD ? RPG : 1;
  float2 en[NH][NL];
  int lam_loaded = -1;
  float2 rxv[NL];
  {
    const float2* rx = p.rx + (size_t)la0 * p.D;
#pragma unroll
    for (int l = 0; l < NL; ++l) rxv[l] = xin[l] ? rx[xx[l]] : czero();
  }

  for (int la = la0; la < la1; ++la) {
    const int lam = la / p.n_a, a = la % p.n_a;
    if (lam != lam_mask) {
      fp.set_mask(p.mrow + (size_t)lam * N);
      lam_mask = lam;
    }
    const float2* e0 = p.field + ((size_t)f * p.n_lam + lam) * p.D * p.D;
    if (!HOLD || lam != lam_loaded) {
#pragma unroll
      for (int rr = 0; rr < NH; ++rr) {
        const int yy = min(y0 + g * RPG + rr, p.D - 1);
#pragma unroll
        for (int l = 0; l < NL; ++l) en[rr][l] = e0[(size_t)yy * p.D + xx[l]];
      }
      lam_loaded = lam;
    }
    float2 rxc[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) rxc[l] = rxv[l];
    if (la + 1 < la1) {   // prefetch the next pair's row tilt
      const float2* rx = p.rx + (size_t)(la + 1) * p.D;
#pragma unroll
      for (int l = 0; l < NL; ++l) rxv[l] = xin[l] ? rx[xx[l]] : czero();
    }
#pragma unroll 1
    for (int rr = 0; rr < RPG; ++rr) {
      const int yl = g * RPG + rr;
      const bool yin = y0 + yl < p.D;
      float2 er[NL];   // this row's values, chosen by selects (no dynamic register indexing)
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        er[l] = en[0][l];
#pragma unroll
        for (int r2 = 1; r2 < NH; ++r2)
          if (rr == r2) er[l] = en[r2][l];
      }
      float2 v[V];
#pragma unroll
      for (int i = 0; i < NB0; ++i)
#pragma unroll
        for (int q = 0; q < R0; ++q) {
          if (q < QM) {
            const int l = i * QM + q;
            v[i * R0 + q] = yin ? cmul(er[l], rxc[l]) : czero();
          } else {
            v[i * R0 + q] = czero();
          }
        }
      if (!HOLD && rr + 1 < RPG) {   // prefetch the next row of the field
        const int yy = min(y0 + yl + 1, p.D - 1);
#pragma unroll
        for (int l = 0; l < NL; ++l) en[0][l] = e0[(size_t)yy * p.D + xx[l]];
      }
      fp.run(v);
#pragma unroll
      for (int s = 0; s < V; ++s) {
        const int X = space_index<N>(t, s);
        const int xc = p.full ? X : window_index(X, p.D, p.win_lo, p.win_hi);
        s_tile[xc >= 0 ? tile_slot<RW>(xc, yl) : spare] = v[s];
      }
    }
    __syncthreads();
    float2* dst = p.rbuf + ((((size_t)f * p.n_lam + lam) * p.n_a + a) * p.Nc) * p.Dp;
    const int rows = min(RW, p.D - y0);
    for (int e = tid; e < p.Nc * RW; e += kBlock) {
      const int xc = e / RW, yl = e % RW;
      if (yl < rows) dst[(size_t)xc * p.Dp + y0 + yl] = s_tile[tile_slot<RW>(xc, yl)];
    }
    __syncthreads();
  }
}

template <int N, int QM, int RW>
__global__ __launch_bounds__(kBlock) void k_rows(RowArgs p) {
  extern __shared__ float2 smem[];
  rows_body<N, QM, RW>(p, blockIdx.x, smem, threadIdx.x);
}

// ------------------------------------------------------------- columns ----
// The modulation points, in k-order, are cut into G contiguous groups (G =
// lane groups per workgroup), group g = [g n_mod / G, (g + 1) n_mod / G).
// The intensity is summed as: over wavelengths, over groups, the group's
// partial sum.  Without SPLIT one lane group runs every group of its own
// column; with SPLIT (few frames) the G lane groups of a workgroup run the
// G groups of one column and the partials meet in LDS.  The additions are
// the same in both, so both give the same bits.
__device__ __forceinline__ int kgroup_lo(int g, int n_mod, int G) { return g * n_mod / G; }

template <int N, int QM_, bool SPLIT>
__device__ __forceinline__ void cols_body(const ColArgs& p, int bid, float2* smem, int tid) {
  using P = FftPlan<N>;
  constexpr int T = P::T, V = N / T, R0 = P::r[0], NB0 = V / R0, G = kBlock / T;
  constexpr int QM = QM_ < R0 ? QM_ : R0;
  constexpr int BL = BufLen<N>::value, NL = NB0 * QM;

  // palindromic plans: twiddles straight into registers, LDS only for the
  // exchange buffers; the others keep the twiddle table in LDS.  The mask of
  // each wavelength goes from the table to registers as it starts.
  constexpr bool PAL = Palindromic<N>::value;
  float2* s_tw = smem;
  float2* s_buf = s_tw + (PAL ? 0 : N);
  float* s_part = (float*)(s_buf + G * BL);              // SPLIT: [G][V][T]

  const int g = tid / T, t = tid % T;
  int xc, f;
  if constexpr (SPLIT) {
    xc = bid % p.Nc;
    f = bid / p.Nc;
  } else {
    xc = (bid % p.colblocks) * G + g;
    f = bid / p.colblocks;
  }
  const bool live = xc < p.Nc;
  const int xcl = live ? xc : 0;

  FftPair<N, QM> fp;
  if constexpr (PAL) {
    fp.init(t, s_buf + g * BL, p.tw);
  } else {
    for (int i = tid; i < N; i += kBlock) s_tw[i] = p.tw[i];
    __syncthreads();
    fp.init(t, s_buf + g * BL, s_tw);
  }

  // this lane's input rows and whether they hold pupil data
  int yy[NL];
  bool yin[NL];
#pragma unroll
  for (int i = 0; i < NB0; ++i)
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      const int y = t + T * i + q * (N / R0);
      yy[i * QM + q] = min(y, p.D - 1);
      yin[i * QM + q] = live && (y < p.D);
    }

  float acc[V];
#pragma unroll
  for (int s = 0; s < V; ++s) acc[s] = 0.f;

  const int it0 = SPLIT ? kgroup_lo(g, p.n_mod, G) : 0;
  const int it1 = SPLIT ? kgroup_lo(g + 1, p.n_mod, G) : p.n_mod;
  const size_t frame_base = (size_t)f * p.n_lam * p.n_a;
  for (int lam = 0; lam < p.n_lam; ++lam) {
    fp.set_mask(p.mcol + lam * N);
    const float2* rbl = p.rbuf + ((frame_base + (size_t)lam * p.n_a) * p.Nc + xcl) * p.Dp;
    const float2* ryl = p.ry + (size_t)lam * p.n_mod * p.D;
    float2 cn[NL], rn[NL];
    if (it0 < it1) {
      const int2 ka = p.kord[it0];
      const float2* col = rbl + (size_t)ka.y * p.Nc * p.Dp;
      const float2* ry = ryl + (size_t)ka.x * p.D;
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        cn[l] = col[yy[l]];
        rn[l] = ry[yy[l]];
      }
    }
    float part[V];
#pragma unroll
    for (int s = 0; s < V; ++s) part[s] = 0.f;
    int gi = 0;                                    // group of `it` (no SPLIT)
    int gend = kgroup_lo(1, p.n_mod, G);
    for (int it = it0; it < it1; ++it) {
      float2 v[V];
#pragma unroll
      for (int i = 0; i < NB0; ++i)
#pragma unroll
        for (int q = 0; q < R0; ++q) {
          if (q < QM) {
            const int l = i * QM + q;
            v[i * R0 + q] = yin[l] ? cmul(cn[l], rn[l]) : czero();
          } else {
            v[i * R0 + q] = czero();
          }
        }
      if (it + 1 < it1) {   // prefetch the next point's column and tilt
        const int2 ka = p.kord[it + 1];
        const float2* col = rbl + (size_t)ka.y * p.Nc * p.Dp;
        const float2* ry = ryl + (size_t)ka.x * p.D;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          cn[l] = col[yy[l]];
          rn[l] = ry[yy[l]];
        }
      }
      fp.run(v);
#pragma unroll
      for (int s = 0; s < V; ++s) part[s] += cabs2(v[s]);
      if constexpr (!SPLIT) {
        while (gi < G - 1 && it + 1 >= gend) {   // leaving group gi (empty groups add nothing)
          if (it + 1 == gend) {
#pragma unroll
            for (int s = 0; s < V; ++s) {
              acc[s] += part[s];
              part[s] = 0.f;
            }
          }
          ++gi;
          gend = kgroup_lo(gi + 1, p.n_mod, G);
        }
      }
    }
    if constexpr (SPLIT) {   // lane group 0 adds this wavelength's G partials in group order
#pragma unroll
      for (int s = 0; s < V; ++s) s_part[((size_t)g * V + s) * T + t] = part[s];
      __syncthreads();
      if (g == 0)
        for (int gg = 0; gg < G; ++gg)
#pragma unroll
          for (int s = 0; s < V; ++s) acc[s] += s_part[((size_t)gg * V + s) * T + t];
      __syncthreads();
    } else {
#pragma unroll
      for (int s = 0; s < V; ++s) acc[s] += part[s];     // the last group
    }
  }
  if (SPLIT && g != 0) return;
  if (!live) return;
  const int X = p.full ? xc : window_coord(xc, p.D, p.win_lo, p.win_hi);
  float* out = p.out + (long long)f * p.out_stride;
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const int Y = space_index<N>(t, s);
    const bool keep = p.full || window_index(Y, p.D, p.wy_lo, p.wy_hi) >= 0;
    if (keep) out[(size_t)Y * N + X] = acc[s];
  }
}

template <int N, int QM, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_cols(ColArgs p) {
  extern __shared__ float2 smem[];
  cols_body<N, QM, SPLIT>(p, blockIdx.x, smem, threadIdx.x);
}

// --------------------------------------------- fused pass (N = 64, 128) ----
// One workgroup owns one frame and never leaves the chip between its input
// and its output: the pupil field of each wavelength is formed in registers,
// the row transforms of one x-tilt key go to an LDS tile [Nc][D] (the row
// pass's output, kept on chip instead of in HBM), the column transforms of
// every point of that key read it back, and |e|^2 accumulates in registers
// over every key, point and wavelength.  At the end the accumulator goes
// through LDS so that the intensity rows leave in coalesced stores.  The
// arithmetic of each transform pair is the two-pass kernels'; only the order
// of the |e|^2 sum differs (one running sum per pixel in point order).
constexpr int kFusedBlock = 512;

struct FusedArgs {
  const float* opd;        // sensor's first frame; frame stride opd_stride
  const float* amp;        // [D][D]
  const float2* rx;        // [n_lam][n_a][D]
  const float2* ry;        // [n_lam][n_mod][D]
  const float2* mrow;      // [n_lam][N]
  const float2* mcol;      // [n_lam][N]
  const float2* tw;        // [N]
  const int2* kord;        // [n_mod] (point, key), keys ascending
  float* out;              // sensor's first frame; frame stride out_stride
  long long opd_stride, out_stride;
  int D, Nc, n_a, n_lam, n_mod, full, win_lo, win_hi, wy_lo, wy_hi;
  double two_pi_over_lam[PWFS_MAX_LAMBDA];
};

// LDS of the fused pass: the lane groups' exchange buffers, then the row
// tile [Nc][D | 1] of float2 (odd row stride: the lanes writing one output
// slot hit distinct banks), reused at the end as the float tile
// [rows kept][Nc + 1]
template <int N>
__host__ __device__ constexpr size_t fused_lds_bytes(int D, int Nc, int rows_kept) {
  const size_t buf = sizeof(float2) * (size_t)(kFusedBlock / FftPlan<N>::T) * BufLen<N>::value;
  const size_t tile = sizeof(float2) * (size_t)Nc * (size_t)(D | 1);
  const size_t out = sizeof(float) * (size_t)rows_kept * (size_t)(Nc + 1);
  return buf + (tile > out ? tile : out);
}

template <int N, int QM_>
__global__ __launch_bounds__(kFusedBlock) void k_fused(FusedArgs p) {
  using P = FftPlan<N>;
  constexpr int T = P::T, V = N / T, R0 = P::r[0], NB0 = V / R0, G = kFusedBlock / T;
  constexpr int QM = QM_ < R0 ? QM_ : R0, NL = NB0 * QM;
  constexpr int RPG = (N / 2 + G - 1) / G;   // pupil rows per lane group (D <= N / 2)
  constexpr int CPG = (N + G - 1) / G;       // kept columns per lane group (Nc <= N)
  constexpr int BL = BufLen<N>::value;
  static_assert(Palindromic<N>::value, "the fused pass keeps its twiddles in registers");
  extern __shared__ float2 smem[];
  float2* s_R = smem + G * BL;
  const int RS = p.D | 1;
  const int tid = threadIdx.x, g = tid / T, t = tid % T;
  const int f = blockIdx.x;

  FftPair<N, QM> fp;
  fp.init(t, smem + g * BL, p.tw);

  // this lane's first-stage inputs (pupil x for a row, pupil y for a column)
  int xx[NL];
  bool xin[NL];
#pragma unroll
  for (int i = 0; i < NB0; ++i)
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      const int x = t + T * i + q * (N / R0);
      xx[i * QM + q] = min(x, p.D - 1);
      xin[i * QM + q] = x < p.D;
    }

  float acc[CPG][V];
#pragma unroll
  for (int c = 0; c < CPG; ++c)
#pragma unroll
    for (int s = 0; s < V; ++s) acc[c][s] = 0.f;

  const float* opd = p.opd + (long long)f * p.opd_stride;
  for (int lam = 0; lam < p.n_lam; ++lam) {
    // pupil field of this group's rows y = g + G r, as the field pass forms it
    float2 e0[RPG][NL];
#pragma unroll
    for (int r = 0; r < RPG; ++r) {
      const int y = g + G * r;
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        float2 v = czero();
        if (y < p.D && xin[l]) {
          const int i = y * p.D + xx[l];
          const double ph = (double)opd[i] * p.two_pi_over_lam[lam];
          const double n = rint(ph * 0.15915494309189533577);
          const float red = (float)fma(-n, 6.283185307179586477, ph);
          float sn, cs;
          sincosf(red, &sn, &cs);
          const float a = p.amp[i];
          v = make_float2(a * cs, a * sn);
        }
        e0[r][l] = v;
      }
    }
    float2 mr[V], mc[V];
#pragma unroll
    for (int s = 0; s < V; ++s) {
      mr[s] = p.mrow[(size_t)lam * N + freq_index<N>(t, s)];
      mc[s] = p.mcol[(size_t)lam * N + freq_index<N>(t, s)];
    }
    const float2* rxl = p.rx + (size_t)lam * p.n_a * p.D;
    const float2* ryl = p.ry + (size_t)lam * p.n_mod * p.D;
    int prev = -1;
    for (int it = 0; it < p.n_mod; ++it) {
      const int2 ka = p.kord[it];
      if (ka.y != prev) {
        // row transforms of key ka.y into the tile (the previous key's
        // column transforms are done with it)
        __syncthreads();
#pragma unroll
        for (int s = 0; s < V; ++s) fp.m[s] = mr[s];
        float2 rxv[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) rxv[l] = xin[l] ? rxl[(size_t)ka.y * p.D + xx[l]] : czero();
#pragma unroll
        for (int r = 0; r < RPG; ++r) {
          const int y = g + G * r;
          float2 v[V];
#pragma unroll
          for (int i = 0; i < NB0; ++i)
#pragma unroll
            for (int q = 0; q < R0; ++q)
              v[i * R0 + q] = q < QM ? cmul(e0[r][i * QM + q], rxv[i * QM + q]) : czero();
          fp.run(v);
          if (y < p.D) {
#pragma unroll
            for (int s = 0; s < V; ++s) {
              const int X = space_index<N>(t, s);
              const int xc = p.full ? X : window_index(X, p.D, p.win_lo, p.win_hi);
              if (xc >= 0) s_R[xc * RS + y] = v[s];
            }
          }
        }
        __syncthreads();
        prev = ka.y;
#pragma unroll
        for (int s = 0; s < V; ++s) fp.m[s] = mc[s];
      }
      // column transforms of point ka.x over this group's columns
      float2 ryv[NL];
#pragma unroll
      for (int l = 0; l < NL; ++l) ryv[l] = xin[l] ? ryl[(size_t)ka.x * p.D + xx[l]] : czero();
#pragma unroll
      for (int c = 0; c < CPG; ++c) {
        const int xc = g + G * c;
        const bool live = xc < p.Nc;
        const int xcl = live ? xc : 0;
        float2 v[V];
#pragma unroll
        for (int i = 0; i < NB0; ++i)
#pragma unroll
          for (int q = 0; q < R0; ++q) {
            const int l = i * QM + q;
            v[i * R0 + q] = (q < QM && xin[l]) ? cmul(s_R[xcl * RS + xx[l]], ryv[l]) : czero();
          }
        fp.run(v);
        if (live) {
#pragma unroll
          for (int s = 0; s < V; ++s) acc[c][s] += cabs2(v[s]);
        }
      }
    }
  }
  // accumulator -> float tile [rows kept][Nc + 1] -> coalesced rows out
  __syncthreads();
  float* s_O = (float*)s_R;
  const int OS = p.Nc + 1;
#pragma unroll
  for (int c = 0; c < CPG; ++c) {
    const int xc = g + G * c;
    if (xc >= p.Nc) continue;
#pragma unroll
    for (int s = 0; s < V; ++s) {
      const int Y = space_index<N>(t, s);
      const int yc = p.full ? Y : window_index(Y, p.D, p.wy_lo, p.wy_hi);
      if (yc >= 0) s_O[yc * OS + xc] = acc[c][s];
    }
  }
  __syncthreads();
  const int rows = p.full ? N : 2 * p.D;
  float* out = p.out + (long long)f * p.out_stride;
  for (int e = tid; e < rows * p.Nc; e += kFusedBlock) {
    const int yc = e / p.Nc, xc = e - yc * p.Nc;
    const int Y = p.full ? yc : window_coord(yc, p.D, p.wy_lo, p.wy_hi);
    const int X = p.full ? xc : window_coord(xc, p.D, p.win_lo, p.win_hi);
    out[(size_t)Y * N + X] = s_O[yc * OS + xc];
  }
}

// ------------------------------------------- double roof, flat-axis passes --
// An arm of a double roof with no field stop has a flat mask on one axis, and
// there the transform pair is the identity up to the pupil offset: the row
// output at plane column o + x is the modulated field itself, and the column
// output at plane row o + y is the column input times the wavelength's scale.
// These two kernels replace those passes (same layouts as k_rows / k_cols).
struct IdentArgs {
  const float2* field;     // [frames][n_lam][D][D]
  const float2* rx;        // [n_lam][n_a][D]
  float2* rbuf;            // [frames][n_lam][n_a][Nc][Dp]
  const int2* kord;        // [n_mod] (point, key), keys ascending
  float* out;              // intensity of the chunk's first frame, frame stride out_stride
  long long out_stride;
  int nf, D, Dp, Nc, N, n_a, n_lam, n_mod, o, full, win_lo, win_hi;
  float w2[PWFS_MAX_LAMBDA];   // per-wavelength intensity scale (share * weight / (n_mod sum A^2))
};

// arm y: R[f][lam][a][xc][y] = E[f][lam][y][x] rx[lam][a][x] at the compact
// column xc of plane column o + x (xc = x in window mode, where the single
// window starts at o), zero in the other columns of full-plane mode; one
// thread per element, y fastest (the scratch is column-major)
__global__ __launch_bounds__(kBlock) void k_rows_ident(IdentArgs p) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long total = (long long)p.nf * p.n_lam * p.n_a * p.Nc * p.D;
  if (i >= total) return;
  const int y = (int)(i % p.D);
  long long r = i / p.D;
  const int xc = (int)(r % p.Nc);
  r /= p.Nc;
  const int a = (int)(r % p.n_a);
  r /= p.n_a;
  const int lam = (int)(r % p.n_lam);
  const long long f = r / p.n_lam;
  const int x = p.full ? xc - p.o : xc;
  float2 v = czero();
  if (x >= 0 && x < p.D)
    v = cmul(p.field[((f * p.n_lam + lam) * p.D + y) * p.D + x], p.rx[((long long)lam * p.n_a + a) * p.D + x]);
  p.rbuf[(((f * p.n_lam + lam) * p.n_a + a) * p.Nc + xc) * p.Dp + y] = v;
}

// arm x: I[f][o + y][X(xc)] = sum_lam w2[lam] sum_points |R[f][lam][key][xc][y]|^2,
// rows outside the pupil zero in full-plane mode; one thread per output
// element, rows fastest
__global__ __launch_bounds__(kBlock) void k_cols_ident(IdentArgs p) {
  const int Yn = p.full ? p.N : p.D;
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long total = (long long)p.nf * p.Nc * Yn;
  if (i >= total) return;
  const int yo = (int)(i % Yn);
  long long r = i / Yn;
  const int xc = (int)(r % p.Nc);
  const long long f = r / p.Nc;
  const int Y = p.full ? yo : p.o + yo;
  const int y = Y - p.o;
  float acc = 0.f;
  if (y >= 0 && y < p.D) {
    for (int lam = 0; lam < p.n_lam; ++lam) {
      const float2* base = p.rbuf + (((f * p.n_lam + lam) * p.n_a) * p.Nc + xc) * (long long)p.Dp + y;
      float part = 0.f, val = 0.f;
      int prev = -1;
      for (int k = 0; k < p.n_mod; ++k) {
        const int a = p.kord[k].y;
        if (a != prev) {
          val = cabs2(base[(long long)a * p.Nc * p.Dp]);
          prev = a;
        }
        part += val;
      }
      acc += p.w2[lam] * part;
    }
  }
  const int X = p.full ? xc : window_coord(xc, p.D, p.win_lo, p.win_hi);
  p.out[f * p.out_stride + (long long)Y * p.N + X] = acc;
}

// -------------------------------------------------------------- slopes ----
// One workgroup per frame.  Block sums are work items (quadrant, subaperture)
// spread over the NT threads; consecutive threads read consecutive blocks of
// a pixel row.  NT = 1024 serves small frame counts, where the frame's own
// latency is the cost.
// BB: the block size b when known at compile time (its loads are then issued
// together), 0 for a run-time b, -1 when subapertures are not whole pixels
// (pixels cut by a subaperture edge count with their area fraction).
template <int NT, int BB>
__global__ __launch_bounds__(NT) void k_slopes(SlopeArgs p) {
  extern __shared__ float s_q[];        // [4][n*n]
  __shared__ double s_red[NT];
  __shared__ double s_red2[NT];
  const int tid = threadIdx.x, f = blockIdx.x;
  const int nn = p.n * p.n;
  const float* I = p.in + (long long)f * p.in_stride;
  const int b = BB > 0 ? BB : p.b;

  for (int it = tid; it < 4 * nn; it += NT) {
    const int q = it / nn, s = it % nn;
    const int i = s / p.n, j = s % p.n;
    float acc = 0.f;
    if constexpr (BB < 0) {
      // subaperture i spans pixels [i img / n, (i + 1) img / n): integer
      // overlaps in units of 1/n pixel, the sum scaled by 1/n^2 at the end
      const int n = p.n, D = p.img;
      const int ylo = i * D, yhi = ylo + D, xlo = j * D, xhi = xlo + D;
      const float* im = I + (size_t)p.org_r[q] * p.N + p.org_c[q];
      for (int y = ylo / n; y * n < yhi; ++y) {
        const int oy = min((y + 1) * n, yhi) - max(y * n, ylo);
        float row = 0.f;
        for (int x = xlo / n; x * n < xhi; ++x) {
          const int ox = min((x + 1) * n, xhi) - max(x * n, xlo);
          row += (float)ox * im[(size_t)y * p.N + x];
        }
        acc += (float)oy * row;
      }
      acc *= 1.0f / (float)(n * n);
    } else if constexpr (BB > 0) {
      const float* blk = I + (size_t)(p.org_r[q] + i * b) * p.N + p.org_c[q] + j * b;
      float v[BB * BB];
#pragma unroll
      for (int r = 0; r < BB; ++r)
#pragma unroll
        for (int c = 0; c < BB; ++c) v[r * BB + c] = blk[(size_t)r * p.N + c];
#pragma unroll
      for (int e = 0; e < BB * BB; ++e) acc += v[e];
    } else {
      const float* blk = I + (size_t)(p.org_r[q] + i * b) * p.N + p.org_c[q] + j * b;
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) acc += blk[(size_t)r * p.N + c];
    }
    s_q[it] = acc;
  }
  __syncthreads();
  // valid-subaperture flux in float64: all four images (pyramid), or arm x
  // (images 0, 1) and arm y (images 2, 3) apart (double roof)
  double tsum = 0.0, tsum2 = 0.0;
  for (int s = tid; s < nn; s += NT)
    if (p.valid[s]) {
      if (p.roof) {
        tsum += (double)(s_q[s] + s_q[nn + s]);
        tsum2 += (double)(s_q[2 * nn + s] + s_q[3 * nn + s]);
      } else {
        tsum += (double)(((s_q[s] + s_q[nn + s]) + s_q[2 * nn + s]) + s_q[3 * nn + s]);
      }
    }
  s_red[tid] = tsum;
  s_red2[tid] = tsum2;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) {
      s_red[tid] += s_red[tid + w];
      s_red2[tid] += s_red2[tid + w];
    }
    __syncthreads();
  }
  const double flux = p.roof ? s_red[0] + s_red2[0] : s_red[0];
  const float gnorm = (float)((p.roof ? s_red[0] : flux) / (double)p.n_valid);
  const float gnorm_y = p.roof ? (float)(s_red2[0] / (double)p.n_valid) : gnorm;
  float* out = p.slopes + (long long)f * p.slope_stride;
  for (int s = tid; s < nn; s += NT) {
    float sx = 0.f, sy = 0.f;
    if (p.valid[s]) {
      const float q0 = s_q[s], q1 = s_q[nn + s], q2 = s_q[2 * nn + s], q3 = s_q[3 * nn + s];
      if (p.roof) {
        sx = (q0 - q1) / (p.local_norm ? (q0 + q1) : gnorm);
        sy = (q2 - q3) / (p.local_norm ? (q2 + q3) : gnorm_y);
      } else {
        const float den = p.local_norm ? (q0 + q1 + q2 + q3) : gnorm;
        sx = ((q0 + q2) - (q1 + q3)) / den;
        sy = ((q0 + q1) - (q2 + q3)) / den;
      }
      if (p.ref) {
        sx -= p.ref[s];
        sy -= p.ref[nn + s];
      }
    }
    out[s] = sx;
    out[nn + s] = sy;
  }
  if (p.flux && tid == 0) p.flux[(long long)f * p.flux_stride] = (float)flux;
}

}  // namespace pwfs

// ============================================ persistent heterogeneous pass ==
// One launch runs the field, row and column passes of every sensor of a
// plan.  Work items are numbered kind-major (all field items, then all row
// items, then all column items; within a kind, sensors in `order`, largest
// first); each workgroup claims the next item from counters[0].  A sensor's
// row items wait until all its field items are done, its column items until
// all its row items are done (counters[1 + 2 s + 0 / 1]).  Completion is
// published with an agent-scope release after a workgroup barrier, waits use
// agent-scope acquire loads, so data written on one XCD is read coherently
// on another.  Items are claimed in increasing order and only wait for
// smaller items that running workgroups already own, so every wait ends.  A
// spin limit turns a broken schedule into an error instead of a hang: a wait
// that gives up sets a sticky flag (counters[1 + 2 kMaxHetero], read and
// cleared by pwfs_device_status) and skips its item, whose outputs are then
// incomplete; the item still counts as done, so the launch drains and ends.
// A negative spin limit makes every wait give up at once (a failure forced
// from the host, to test that path).
namespace pwfs {

constexpr int kMaxHetero = 8;

struct HeteroArgs {
  FieldArgs field[kMaxHetero];
  RowArgs rows[kMaxHetero];
  ColArgs cols[kMaxHetero];
  int nfft[kMaxHetero];
  int rw[kMaxHetero];   // row-pass tile rows per sensor
  int n_items[3][kMaxHetero];
  int order[kMaxHetero];
  int n_sensors, total, spin_limit;
  int* counters;   // [0] claim, [1 + 2 s] field done, [2 + 2 s] rows done, [1 + 2 kMaxHetero] error flag
};

// index of the sticky error flag in the counters; the per-pass reset clears
// the counters below it only
constexpr int kHeteroFlag = 1 + 2 * kMaxHetero;

__global__ void k_counter_reset(int* c, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0;
}

template <int N>
__device__ __forceinline__ void hetero_rows(const RowArgs& a, int rw, int bid, float2* smem, int tid) {
  if (rw == RowTile<N>::ALT && RowTile<N>::ALT != RowTile<N>::RW)
    rows_body<N, 3, RowTile<N>::ALT>(a, bid, smem, tid);
  else
    rows_body<N, 3, RowTile<N>::RW>(a, bid, smem, tid);
}
template <int N>
__device__ __forceinline__ void hetero_cols(const ColArgs& a, int bid, float2* smem, int tid) {
  cols_body<N, 3, false>(a, bid, smem, tid);
}

__global__ __launch_bounds__(kBlock, 2) void k_hetero(HeteroArgs p) {
  extern __shared__ float2 smem[];
  __shared__ int s_item, s_skip, s_zero;
  // The bodies' lane-dependent set-up (twiddles, addresses) does not depend
  // on the item, so the compiler would hoist every body's set-up out of the
  // claim loop and keep all of it live at once (256 VGPRs + 235 AGPRs, one
  // wave per SIMD).  Deriving the lane index from an LDS word read after each
  // claim keeps that set-up inside its own branch (247 VGPRs, two waves).
  if (threadIdx.x == 0) s_zero = 0;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&p.counters[0], 1);
    __syncthreads();
    int item = __builtin_amdgcn_readfirstlane(s_item);   // uniform: selects kernel arguments
    const int tid = (int)threadIdx.x + __builtin_amdgcn_readfirstlane(s_zero);
    __syncthreads();
    if (item >= p.total) break;
    int kind = 0, s = 0;
    for (kind = 0; kind < 3; ++kind) {
      bool found = false;
      for (int o = 0; o < p.n_sensors; ++o) {
        const int c = p.n_items[kind][p.order[o]];
        if (item < c) {
          s = p.order[o];
          found = true;
          break;
        }
        item -= c;
      }
      if (found) break;
    }
    bool skip = false;
    if (kind > 0) {
      if (threadIdx.x == 0) {
        int* dep = &p.counters[1 + 2 * s + (kind - 1)];
        const int need = p.n_items[kind - 1][s];
        int spins = 0, gave_up = p.spin_limit < 0;
        while (!gave_up && __hip_atomic_load(dep, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
          __builtin_amdgcn_s_sleep(2);
          if (++spins > p.spin_limit) gave_up = 1;
        }
        if (gave_up) atomicExch(&p.counters[kHeteroFlag], 1);
        s_skip = gave_up;
      }
      __syncthreads();
      skip = __builtin_amdgcn_readfirstlane(s_skip) != 0;
    }
    if (skip) {
      // the item's inputs may be incomplete: leave its outputs untouched
    } else if (kind == 0) {
      field_body(p.field[s], item);
    } else if (kind == 1) {
      switch (p.nfft[s]) {
        case 256: hetero_rows<256>(p.rows[s], p.rw[s], item, smem, tid); break;
        case 384: hetero_rows<384>(p.rows[s], p.rw[s], item, smem, tid); break;
        case 512: hetero_rows<512>(p.rows[s], p.rw[s], item, smem, tid); break;
        default: hetero_rows<768>(p.rows[s], p.rw[s], item, smem, tid); break;
      }
    } else {
      switch (p.nfft[s]) {
        case 256: hetero_cols<256>(p.cols[s], item, smem, tid); break;
        case 384: hetero_cols<384>(p.cols[s], item, smem, tid); break;
        case 512: hetero_cols<512>(p.cols[s], item, smem, tid); break;
        default: hetero_cols<768>(p.cols[s], item, smem, tid); break;
      }
    }
    __syncthreads();   // every lane's stores of this item are issued and the LDS is free
    if (threadIdx.x == 0 && kind < 2)
      __hip_atomic_fetch_add(&p.counters[1 + 2 * s + kind], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace pwfs
