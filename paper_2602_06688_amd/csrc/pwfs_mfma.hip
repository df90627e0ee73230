// pwfs_mfma.hip -- the forward model as dense complex matrix products on the
// gfx950 matrix cores, in bf16 (one term) or bf16/fp16 hi/lo split (three
// terms) with fp32 accumulation.
//
// Because the mask and the tilts are separable, the padded 2-D chain of one
// modulation point is e_k = Qy_k E0 Qx_a^T with
//   P[Y][x]   = h[o + x] p[(Y - o - x) mod N],  p = IDFT(m)  (N_out x D),
//   Qx_a[X][x] = P[X][x] exp(i 2 pi r x_c cos t_a / D),
//   Qy_k[Y][y] = P[Y][y] exp(i 2 pi r y_c sin t_k / D),
// built in float64 on the host.  Stage 1 forms T_a = E0 Qx_a^T once per
// distinct cosine a (shared by k and n_mod - k) for all frames at once; stage
// 2 forms e_k = Qy_k T_a(k) and accumulates c_lambda |e_k|^2 over k and
// wavelength in registers (c_lambda = w_lambda / (n_mod sum A^2)).
//
// Operand layout: every 16-bit operand block of R rows by Kp columns (a
// plane of a table, of the split field, of T) is stored K-blocked, [Kp/BK][R]
// [BK] with BK the K step of the engine (32 for the split forms, 64 for the
// one-term form), so that one K step of consecutive rows is contiguous: the
// producers' 16-byte loads then use whole 128-byte lines within one step
// instead of half of a line in each of two steps.
//
// Complex products run as real products on an interleaved block form: the
// left operand's rows come in pairs (Re Q[X][.], -Im Q[X][.]) and
// (Im Q[X][.], Re Q[X][.]) over K = (real parts, imaginary parts) of the
// right operand, so output rows 2X and 2X + 1 hold Re and Im of one element,
// in the same lane of the accumulator layout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "mfma_gemm.hpp"
#include "pwfs_geom.hpp"
#include "pwfs_internal.hpp"

namespace pwfs {

namespace {

// K steps the producer waves of the wave-specialised stages keep in flight,
// and the columns of a workgroup tile
constexpr int kWsDepth = 2, kWsCols = 256;

constexpr double kPi = 3.14159265358979323846264338327950288;

struct MGeom {
  int D, N, Nc, Kp, M, n_a, n_lam, n_mod, planes, bk;
  bool f16;
};

MGeom mgeom(const pwfs_sensor_desc& d) {
  const Geometry g = geometry(d);
  MGeom m;
  m.D = g.D;
  m.N = g.N;
  m.Nc = g.Nc;
  const bool one_term = d.precision == PWFS_BF16 || d.precision == PWFS_FP16;
  const int bk = one_term ? 64 : 32;   // the K step of the engine used
  m.bk = bk;
  m.Kp = (2 * g.D + bk - 1) / bk * bk;
  m.M = 2 * g.Nc;
  m.n_a = g.n_a;
  m.n_lam = g.n_lam;
  m.n_mod = g.n_mod;
  m.planes = one_term ? 1 : 2;
  m.f16 = d.precision == PWFS_FP16X3 || d.precision == PWFS_FP16;
  return m;
}

// host-side conversions (round to nearest even)
uint16_t h_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float h_bf16_f(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}
uint16_t h_f16(float xf) {
  // IEEE binary16, round to nearest even, with subnormals; |x| < 65504 here
  const double x = xf;
  const uint16_t sign = std::signbit(x) ? 0x8000 : 0;
  const double a = std::fabs(x);
  if (a == 0.0) return sign;
  int e;
  std::frexp(a, &e);            // a = f 2^e, f in [0.5, 1)
  int ex = e - 1;               // a = 1.m 2^ex
  if (ex < -14) ex = -14;       // subnormal range shares the exponent of 2^-14
  const double q = std::ldexp(a, 10 - ex);   // mantissa units
  double r = std::nearbyint(q);             // ties to even (default rounding mode)
  uint32_t mant = (uint32_t)r;
  int bexp = ex + 15;
  if (mant >= 2048u) {          // rounding carried into the next binade
    mant >>= 1;
    ++bexp;
  }
  if (mant < 1024u) return (uint16_t)(sign | mant);   // subnormal
  if (bexp >= 31) return (uint16_t)(sign | 0x7C00);
  return (uint16_t)(sign | (bexp << 10) | (mant & 0x3FFu));
}
float h_f16_f(uint16_t h) {
  const int e = (h >> 10) & 31, m = h & 1023;
  const double s = (h & 0x8000) ? -1.0 : 1.0;
  if (e == 0) return (float)(s * std::ldexp((double)m, -24));
  return (float)(s * std::ldexp(1.0 + m / 1024.0, e - 15));
}

void host_split(float x, bool f16, uint16_t& hi, uint16_t& lo) {
  if (f16) {
    hi = h_f16(x);
    lo = h_f16((x - h_f16_f(hi)) * 2048.f);
  } else {
    hi = h_bf16(x);
    lo = h_bf16(x - h_bf16_f(hi));
  }
}

// ---------------------------------------------------------------- kernels --
struct SplitFieldArgs {
  const float* opd;       // first frame of the pass, frame stride opd_stride
  const float* amp;       // [D][D]
  uint16_t* out;          // plane 0 [n_lam][Kp/BK][F D][BK] (rows f D + y), plane 1 follows at +plane
  long long opd_stride, plane;
  int D, Kp, BK, F, n_lam, planes;
  double two_pi_over_lam[PWFS_MAX_LAMBDA];
};

template <bool F16>
__global__ __launch_bounds__(256) void k_field_split(SplitFieldArgs p) {
  const long long total = (long long)p.n_lam * p.F * p.D * p.Kp;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;   // output element, in output order
  if (i >= total) return;
  const int rows = p.F * p.D;
  const int kr = (int)(i % p.BK);
  long long r = i / p.BK;
  const int row = (int)(r % rows);
  r /= rows;
  const int kb = (int)(r % (p.Kp / p.BK));
  const int lam = (int)(r / (p.Kp / p.BK));
  const int kk = kb * p.BK + kr, y = row % p.D, f = row / p.D;
  float v = 0.f;
  if (kk < 2 * p.D) {
    const int x = kk % p.D;
    const double ph = (double)p.opd[(long long)f * p.opd_stride + y * p.D + x] * p.two_pi_over_lam[lam];
    const double n = rint(ph * 0.15915494309189533577);
    const float red = (float)fma(-n, 6.283185307179586477, ph);
    float sn, cs;
    sincosf(red, &sn, &cs);
    v = p.amp[y * p.D + x] * (kk < p.D ? cs : sn);
  }
  uint16_t hi, lo;
  if (p.planes == 2) {
    split16<F16>(v, hi, lo);
    p.out[i] = hi;
    p.out[p.plane + i] = lo;
  } else {
    p.out[i] = F16 ? f32_to_f16_rne(v) : f32_to_bf16_rne(v);
  }
}

struct G1Args {
  const uint16_t* a;      // Qx'' plane 0 [n_lam][n_a] blocks of M x Kp; plane 1 at +a_plane
  const uint16_t* b;      // split field plane 0 [n_lam] blocks of F D x Kp; plane 1 at +b_plane
  uint16_t* t;            // T plane 0 [F][n_lam][n_a] blocks of Nc x Kp; plane 1 at +t_plane
  long long a_plane, b_plane, t_plane;
  int M, F, D, Kp, Nc, n_a, n_lam;
  int mtiles, ntiles;     // tiles over the M output rows and over all F D field rows of the pass
};

// Workgroups renumbered so that each of the 8 XCDs (which receive
// workgroups in turn) holds a contiguous run of tiles.
__device__ __forceinline__ int xcd_major_block() {
  const int G = (int)gridDim.x, xcd = (int)blockIdx.x % 8, idx = (int)blockIdx.x / 8;
  const int per = G / 8, rem = G % 8;
  return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + idx;
}

struct G2Args {
  const uint16_t* a;      // Qy'' plane 0 [n_lam][n_mod] blocks of M x Kp; plane 1 at +a_plane
  const uint16_t* t;      // T as written by stage 1
  const int2* kord;       // [n_mod] (k, a)
  float* out;             // first frame of the pass, frame stride out_stride
  long long a_plane, t_plane, out_stride;
  int M, F, Nc, N, D, Kp, n_a, n_lam, n_mod, win_lo, win_hi, full;
  int mtiles, ntiles;     // tiles over the M rows of e and over all F Nc columns of the pass
  float scale[PWFS_MAX_LAMBDA];
};

// Both stages run on the wave-specialised workgroup of mfma_gemm.hpp
// (WsEngine, WsParts, ws_produce): 8 consumer waves on a 128 x 256 tile and
// 4 producer waves keeping kWsDepth K steps of operands in flight.
//
// Stage 2: columns of C run over all frames of the pass (n = f Nc + c), so a
// tile may straddle two frames and only the pass's last tile is ragged.  The
// n_lam x n_mod products of one tile form one stream of K steps, and a
// product's |e|^2 is accumulated as it completes.
template <int NPL, bool F16, int DEPTH, int BN>
__global__ __launch_bounds__(64 * (2 * BN / 64 + 4)) void k_mfma_cols_ws(G2Args p) {
  extern __shared__ uint4 lds_raw[];
  uint16_t* lds = (uint16_t*)lds_raw;
  using E = WsEngine<NPL, F16, BN>;
  using W = WsParts<E, BN>;
  constexpr int NC = 2 * BN / 64, BK = E::BK_, CH = W::CH;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int bid = xcd_major_block();
  const int mt = bid % p.mtiles;
  const int nt = bid / p.mtiles;
  const int m0 = mt * kGemmTile, n0 = nt * BN;
  const int NT = p.F * p.Nc;
  const int nk = p.Kp / BK;
  const int steps = p.n_lam * p.n_mod * nk;

  if (wave >= NC) {
    const int pt = tid - 64 * NC;
    const long long t_frame = (long long)p.n_lam * p.n_a * p.Nc * p.Kp;
    long long goff[CH];   // element offset of chunk h within its operand block's first K block
    int loff[CH];
#pragma unroll
    for (int h = 0; h < CH; ++h) {
      const int row = W::row(pt, h), kq = W::kq(pt, h);
      if (W::is_a(h)) {
        goff[h] = (long long)min(m0 + row, p.M - 1) * BK + kq;
      } else {
        const int n = min(n0 + row, NT - 1);
        const int fr = n / p.Nc;
        goff[h] = fr * t_frame + (long long)(n - fr * p.Nc) * BK + kq;
      }
      loff[h] = W::lds_offset(pt, h);
    }
    ws_produce<E, DEPTH>(lds, loff, steps, [&](u32x4_t (&b)[CH], int s) {
      const int prod = s / nk, kt = s - prod * nk;
      const int lam = prod / p.n_mod;
      // through the scalar cache: a vector load here would have to wait for
      // every load in flight before it (the counter is in order)
      const long long kv =
          *((const __attribute__((address_space(4))) long long*)p.kord + (prod - lam * p.n_mod));
      const int kx = (int)(kv & 0xffffffffLL), ky = (int)(kv >> 32);   // (k, a) of the product
      // K block kt of the product's blocks (M rows of Qy, Nc rows of T per frame)
      const uint16_t* abase = p.a + ((long long)lam * p.n_mod + kx) * p.M * p.Kp + (long long)kt * p.M * BK;
      const uint16_t* bbase = p.t + ((long long)lam * p.n_a + ky) * p.Nc * p.Kp + (long long)kt * p.Nc * BK;
#pragma unroll
      for (int h = 0; h < CH; ++h) {
        const uint16_t* base = W::is_a(h) ? abase + W::plane(h) * p.a_plane : bbase + W::plane(h) * p.t_plane;
        b[h] = *(const u32x4_t*)(base + goff[h]);
      }
    });
    return;
  }

  // -------------------------------------------------------------- consumer
  const int lane = tid & 63;
  const int wm = wave & 1, wn = wave >> 1;
  float inten[2][2][8];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 8; ++e) inten[i][j][e] = 0.f;
  E eng;
  eng.zero();
  __syncthreads();
  int prod = 0, kt = 0;
  for (int st = 0; st < steps; ++st) {
    eng.compute(lds + (st & 1) * E::STAGE, wm, wn, lane);
    if (kt == nk - 1) {
      const float sc = p.scale[prod / p.n_mod];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int e = 0; e < 16; e += 2) {
            const float re = eng.value(i, j, e), im = eng.value(i, j, e + 1);
            inten[i][j][e >> 1] += sc * (re * re + im * im);
          }
      eng.zero();
      kt = 0;
      ++prod;
    } else {
      ++kt;
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; e += 2) {
        // accumulator layout of the 32 x 32 tile (i, j) of this quarter
        const int row = wm * 64 + i * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        const int col = wn * 64 + j * 32 + (lane & 31);
        const int Yc = (m0 + row) >> 1, n = n0 + col;
        if (Yc >= p.Nc || n >= NT) continue;
        const int fr = n / p.Nc, Xc = n - fr * p.Nc;
        const int Y = p.full ? Yc : window_coord(Yc, p.D, p.win_lo, p.win_hi);
        const int X = p.full ? Xc : window_coord(Xc, p.D, p.win_lo, p.win_hi);
        p.out[(long long)fr * p.out_stride + (long long)Y * p.N + X] = inten[i][j][e >> 1];
      }
}

// Stage 1: the tile of (wavelength, 128 output rows, BN field rows) runs the
// n_a products T_a of its field rows (one Qx_a each) as one stream of K
// steps; each product is stored by the consumers as it completes.
template <int NPL, bool F16, int DEPTH, int BN>
__global__ __launch_bounds__(64 * (2 * BN / 64 + 4)) void k_mfma_rows_ws(G1Args p) {
  extern __shared__ uint4 lds_raw[];
  uint16_t* lds = (uint16_t*)lds_raw;
  using E = WsEngine<NPL, F16, BN>;
  using W = WsParts<E, BN>;
  constexpr int NC = 2 * BN / 64, BK = E::BK_, CH = W::CH;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  int bid = xcd_major_block();
  const int mt = bid % p.mtiles;
  bid /= p.mtiles;
  const int nt = bid % p.ntiles;
  const int lam = bid / p.ntiles;
  const int m0 = mt * kGemmTile, n0 = nt * BN;
  const int NF = p.F * p.D;
  const int nk = p.Kp / BK;
  const int steps = p.n_a * nk;

  if (wave >= NC) {
    const int pt = tid - 64 * NC;
    long long goff[CH];
    int loff[CH];
#pragma unroll
    for (int h = 0; h < CH; ++h) {
      const int row = W::row(pt, h), kq = W::kq(pt, h);
      goff[h] = (long long)(W::is_a(h) ? min(m0 + row, p.M - 1) : min(n0 + row, NF - 1)) * BK + kq;
      loff[h] = W::lds_offset(pt, h);
    }
    ws_produce<E, DEPTH>(lds, loff, steps, [&](u32x4_t (&b)[CH], int s) {
      const int a = s / nk, kt = s - a * nk;
      // K block kt of the product's Qx block (M rows) and of the field (F D rows)
      const uint16_t* abase = p.a + ((long long)lam * p.n_a + a) * p.M * p.Kp + (long long)kt * p.M * BK;
      const uint16_t* bbase = p.b + (long long)lam * NF * p.Kp + (long long)kt * NF * BK;
#pragma unroll
      for (int h = 0; h < CH; ++h) {
        const uint16_t* base = W::is_a(h) ? abase + W::plane(h) * p.a_plane : bbase + W::plane(h) * p.b_plane;
        b[h] = *(const u32x4_t*)(base + goff[h]);
      }
    });
    return;
  }

  // -------------------------------------------------------------- consumer
  const int lane = tid & 63;
  const int wm = wave & 1, wn = wave >> 1;
  E eng;
  eng.zero();
  __syncthreads();
  int a = 0, kt = 0;
  for (int st = 0; st < steps; ++st) {
    eng.compute(lds + (st & 1) * E::STAGE, wm, wn, lane);
    if (kt == nk - 1) {
      // output element (row X of T, column c D + y) of the product's block
      // (frame f) in the K-blocked layout
      long long fb[2];
      int ys[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int n = min(n0 + wn * 64 + j * 32 + (lane & 31), NF - 1);
        const int f = n / p.D;
        ys[j] = n - f * p.D;
        fb[j] = (((long long)f * p.n_lam + lam) * p.n_a + a) * p.Nc * p.Kp;
      }
      auto t_at = [&](int j, int X, int kidx) {
        return fb[j] + (long long)(kidx / BK) * p.Nc * BK + X * BK + (kidx % BK);
      };
      int mb = m0 + wm * 64 + 4 * (lane >> 5);   // even: element e has c = e & 1
      // opaque, so that the 32 row offsets below are formed here and not kept
      // live across the whole K stream
      __asm__ volatile("" : "+v"(mb));
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int m = mb + i * 32 + 8 * (e >> 2) + (e & 3);
          if (m >= p.M) continue;
          const int c = e & 1, X = m >> 1;
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            if (n0 + wn * 64 + j * 32 + (lane & 31) >= NF) continue;
            const long long o = t_at(j, X, c * p.D + ys[j]);
            const float v = eng.value(i, j, e);
            if constexpr (NPL == 2) {
              uint16_t hi, lo;
              split16<F16>(v, hi, lo);
              p.t[o] = hi;
              p.t[p.t_plane + o] = lo;
            } else {
              p.t[o] = F16 ? f32_to_f16_rne(v) : f32_to_bf16_rne(v);
            }
            // the K padding [2D, Kp) of this row must hold zeros for stage 2
            if (c == 1)
              for (int kz = 2 * p.D + ys[j]; kz < p.Kp; kz += p.D) {
                const long long oz = t_at(j, X, kz);
                p.t[oz] = 0;
                if constexpr (NPL == 2) p.t[p.t_plane + oz] = 0;
              }
          }
        }
      eng.zero();
      kt = 0;
      ++a;
    } else {
      ++kt;
    }
    __syncthreads();
  }
}

template <int NPL, bool F16>
int launch(const SensorPlan& sp, const MGeom& m, const float* opd, long long os, float* out, long long ost, int nf,
           void* scratch, hipStream_t st, Prof* prof) {
  const Geometry& g = sp.g;
  uint16_t* field = (uint16_t*)scratch;
  const long long field_plane = (long long)m.n_lam * nf * m.D * m.Kp;
  uint16_t* T = field + field_plane * m.planes;
  const long long t_plane = (long long)nf * m.n_lam * m.n_a * m.Nc * m.Kp;
  const uint16_t* tab = (const uint16_t*)sp.dev[R_MFMA];
  const long long qx_plane = (long long)m.n_lam * m.n_a * m.M * m.Kp;
  const long long qy_plane = (long long)m.n_lam * m.n_mod * m.M * m.Kp;
  const uint16_t* qx = tab;
  const uint16_t* qy = tab + qx_plane * m.planes;

  SplitFieldArgs fa{};
  fa.opd = opd;
  fa.amp = (const float*)sp.dev[R_AMP];
  fa.out = field;
  fa.opd_stride = os;
  fa.plane = field_plane;
  fa.D = m.D;
  fa.Kp = m.Kp;
  fa.BK = m.bk;
  fa.F = nf;
  fa.n_lam = m.n_lam;
  fa.planes = m.planes;
  for (int l = 0; l < m.n_lam; ++l) fa.two_pi_over_lam[l] = 2.0 * kPi / sp.desc.lambda_nm[l];
  const unsigned fblocks = (unsigned)((field_plane + 255) / 256);
  int slot = prof->begin(st);
  hipLaunchKernelGGL((k_field_split<F16>), dim3(fblocks), dim3(256), 0, st, fa);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return PWFS_EHIP;
  prof->end(slot, st, K_FIELD);

  const size_t lds = WsEngine<NPL, F16, kWsCols>::lds_bytes();
  constexpr unsigned block = 64 * (2 * kWsCols / 64 + 4);
  G1Args a1{};
  a1.a = qx;
  a1.b = field;
  a1.t = T;
  a1.a_plane = qx_plane;
  a1.b_plane = field_plane;
  a1.t_plane = t_plane;
  a1.M = m.M;
  a1.F = nf;
  a1.D = m.D;
  a1.Kp = m.Kp;
  a1.Nc = m.Nc;
  a1.n_a = m.n_a;
  a1.n_lam = m.n_lam;
  a1.mtiles = (m.M + kGemmTile - 1) / kGemmTile;
  a1.ntiles = (nf * m.D + kWsCols - 1) / kWsCols;
  const unsigned g1 = (unsigned)(m.n_lam * a1.mtiles * a1.ntiles);
  slot = prof->begin(st);
  hipLaunchKernelGGL((k_mfma_rows_ws<NPL, F16, kWsDepth, kWsCols>), dim3(g1), dim3(block), lds, st, a1);
  if ((e = hipGetLastError()) != hipSuccess) return PWFS_EHIP;
  prof->end(slot, st, K_ROWS);

  G2Args a2{};
  a2.a = qy;
  a2.t = T;
  a2.kord = (const int2*)sp.dev[R_AK];
  a2.out = out;
  a2.a_plane = qy_plane;
  a2.t_plane = t_plane;
  a2.out_stride = ost;
  a2.M = m.M;
  a2.F = nf;
  a2.Nc = m.Nc;
  a2.N = m.N;
  a2.D = m.D;
  a2.Kp = m.Kp;
  a2.n_a = m.n_a;
  a2.n_lam = m.n_lam;
  a2.n_mod = m.n_mod;
  a2.mtiles = (m.M + kGemmTile - 1) / kGemmTile;
  a2.ntiles = (int)(((long long)nf * m.Nc + kWsCols - 1) / kWsCols);
  a2.win_lo = g.win_lo;
  a2.win_hi = g.win_hi;
  a2.full = g.full;
  for (int l = 0; l < m.n_lam; ++l)
    a2.scale[l] = (float)(sp.desc.lambda_weight[l] / ((double)sp.g.n_mod * sp.sumA2));
  const unsigned g2 = (unsigned)(a2.mtiles * a2.ntiles);
  slot = prof->begin(st);
  hipLaunchKernelGGL((k_mfma_cols_ws<NPL, F16, kWsDepth, kWsCols>), dim3(g2), dim3(block), lds, st, a2);
  if ((e = hipGetLastError()) != hipSuccess) return PWFS_EHIP;
  prof->end(slot, st, K_MFMA);
  return PWFS_OK;
}

template <int NPL, bool F16>
void set_lds() {
  const int lds_ws = (int)WsEngine<NPL, F16, kWsCols>::lds_bytes();
  if (hipFuncSetAttribute((const void*)k_mfma_cols_ws<NPL, F16, kWsDepth, kWsCols>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, lds_ws) != hipSuccess)
    (void)hipGetLastError();
  if (hipFuncSetAttribute((const void*)k_mfma_rows_ws<NPL, F16, kWsDepth, kWsCols>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, lds_ws) != hipSuccess)
    (void)hipGetLastError();
}

}  // namespace

bool mfma_supported(const pwfs_sensor_desc& d) {
  return d.precision == PWFS_BF16 || d.precision == PWFS_BF16X3 || d.precision == PWFS_FP16X3 ||
         d.precision == PWFS_FP16;
}

size_t mfma_table_bytes(const pwfs_sensor_desc& d) {
  if (d.precision == PWFS_FP32) return 0;
  const MGeom m = mgeom(d);
  return sizeof(uint16_t) * (size_t)m.planes * m.n_lam * ((size_t)m.n_a + m.n_mod) * m.M * m.Kp;
}

size_t mfma_scratch_frame_bytes(const pwfs_sensor_desc& d) {
  const MGeom m = mgeom(d);
  return sizeof(uint16_t) * (size_t)m.planes * m.n_lam * ((size_t)m.D * m.Kp + (size_t)m.n_a * m.Nc * m.Kp);
}

int upload_mfma_tables(const pwfs_sensor_desc& d, char* dst, hipStream_t st, std::vector<std::vector<char>>& keep,
                       double) {
  const MGeom m = mgeom(d);
  const Geometry g = geometry(d);
  const int N = m.N, D = m.D;
  // circulant kernel p = IDFT(m) of the pyramid mask (phases reduced exactly)
  std::vector<std::complex<double>> mk(N), pk(N);
  for (int u = 0; u < N; ++u) {
    const long long twice = (u < N / 2) ? (2LL * u + 1) : (2LL * N - 2LL * u - 1);
    const long long ph = ((long long)g.S * twice) % (4LL * N);
    mk[u] = std::polar(1.0, 2.0 * kPi * (double)ph / (4.0 * N));
  }
  for (int dd = 0; dd < N; ++dd) {
    std::complex<double> s = 0.0;
    for (int u = 0; u < N; ++u) s += mk[u] * std::polar(1.0, 2.0 * kPi * (double)(((long long)u * dd) % N) / N);
    pk[dd] = s / (double)N;
  }
  // P[Yc][x] over the kept rows (windows or full plane)
  std::vector<std::complex<double>> P((size_t)m.Nc * D);
  for (int yc = 0; yc < m.Nc; ++yc) {
    const int Y = g.full ? yc : (yc < D ? g.win_lo + yc : g.win_hi + yc - D);
    for (int x = 0; x < D; ++x) {
      const int Xp = g.o + x;
      const std::complex<double> h = std::polar(1.0, -kPi * (double)Xp / N);
      P[(size_t)yc * D + x] = h * pk[(((Y - Xp) % N) + N) % N];
    }
  }
  const size_t blk = (size_t)m.M * m.Kp;               // one operator, one plane
  const size_t nblk = (size_t)m.n_lam * (m.n_a + m.n_mod);
  std::vector<uint16_t> tab((size_t)m.planes * nblk * blk, 0);
  auto put = [&](size_t b, const std::vector<std::complex<double>>& ramp) {
    // interleaved real block form of Q[Xc][x] = P[Xc][x] ramp[x]
    for (int xc = 0; xc < m.Nc; ++xc)
      for (int x = 0; x < D; ++x) {
        const std::complex<double> q = P[(size_t)xc * D + x] * ramp[x];
        const float vals[4] = {(float)q.real(), (float)-q.imag(), (float)q.imag(), (float)q.real()};
        // element (row, col) of the K-blocked M x Kp block
        auto at = [&](int row, int col) { return (size_t)(col / m.bk) * m.M * m.bk + (size_t)row * m.bk + col % m.bk; };
        const size_t idx[4] = {at(2 * xc, x), at(2 * xc, D + x), at(2 * xc + 1, x), at(2 * xc + 1, D + x)};
        for (int t = 0; t < 4; ++t) {
          uint16_t hi, lo;
          if (m.planes == 2) {
            host_split(vals[t], m.f16, hi, lo);
            tab[b * blk + idx[t]] = hi;
            tab[(nblk + b) * blk + idx[t]] = lo;
          } else {
            tab[b * blk + idx[t]] = m.f16 ? h_f16(vals[t]) : h_bf16(vals[t]);
          }
        }
      }
  };
  // the tilt points in the order the visiting table refers to them (point
  // index and distinct x-tilt key, as in the FP32 path)
  std::vector<TiltPoint> pts;
  std::vector<double> key_tx;
  tilt_points(d, pts, key_tx);
  std::vector<std::complex<double>> ramp(D);
  for (int l = 0; l < m.n_lam; ++l) {
    const double sc = d.lambda_ref_nm / d.lambda_nm[l];
    for (int a = 0; a < m.n_a; ++a) {
      for (int x = 0; x < D; ++x) ramp[x] = std::polar(1.0, 2.0 * kPi * sc * key_tx[a] * (x - (D - 1) / 2.0) / D);
      put((size_t)l * m.n_a + a, ramp);
    }
  }
  // the two planes are laid out [plane][qx blocks ... qy blocks], so qy
  // blocks of plane 0 start after all qx blocks of plane 0
  for (int l = 0; l < m.n_lam; ++l) {
    const double sc = d.lambda_ref_nm / d.lambda_nm[l];
    for (int k = 0; k < m.n_mod; ++k) {
      for (int y = 0; y < D; ++y) ramp[y] = std::polar(1.0, 2.0 * kPi * sc * pts[k].ty * (y - (D - 1) / 2.0) / D);
      put((size_t)m.n_lam * m.n_a + (size_t)l * m.n_mod + k, ramp);
    }
  }
  // reorder to [qx plane0][qx plane1][qy plane0][qy plane1] (what the launch expects)
  std::vector<uint16_t> out(tab.size());
  const size_t nqx = (size_t)m.n_lam * m.n_a * blk, nqy = (size_t)m.n_lam * m.n_mod * blk;
  for (int pl = 0; pl < m.planes; ++pl) {
    std::memcpy(&out[pl * nqx], &tab[(size_t)pl * nblk * blk], nqx * 2);
    std::memcpy(&out[m.planes * nqx + pl * nqy], &tab[(size_t)pl * nblk * blk + nqx], nqy * 2);
  }
  keep.emplace_back((const char*)out.data(), (const char*)out.data() + out.size() * 2);
  if (hipMemcpyAsync(dst, keep.back().data(), out.size() * 2, hipMemcpyHostToDevice, st) != hipSuccess)
    return PWFS_EHIP;
  static bool lds_set = false;
  if (!lds_set) {
    set_lds<1, false>();
    set_lds<2, false>();
    set_lds<2, true>();
    set_lds<1, true>();
    lds_set = true;
  }
  return PWFS_OK;
}

int forward_mfma(const SensorPlan& sp, const float* opd, long long os, float* out, long long ost, int nf,
                 void* scratch, hipStream_t st, Prof* prof) {
  const MGeom m = mgeom(sp.desc);
  if (sp.desc.precision == PWFS_BF16) return launch<1, false>(sp, m, opd, os, out, ost, nf, scratch, st, prof);
  if (sp.desc.precision == PWFS_FP16) return launch<1, true>(sp, m, opd, os, out, ost, nf, scratch, st, prof);
  if (sp.desc.precision == PWFS_BF16X3) return launch<2, false>(sp, m, opd, os, out, ost, nf, scratch, st, prof);
  return launch<2, true>(sp, m, opd, os, out, ost, nf, scratch, st, prof);
}

}  // namespace pwfs
