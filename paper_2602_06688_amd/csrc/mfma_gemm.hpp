// mfma_gemm.hpp -- split-precision matrix-core GEMM tiles for gfx950.
//
// C[M][N] = sum_k A[M][K] B[N][K] (both operands K-contiguous, "NT"), with
// A and B given as 16-bit planes: one plane (plain bf16) or a hi/lo pair
// (x = hi + lo, three products hi*hi + hi*lo + lo*hi accumulated in fp32).
// For fp16 the lo plane is stored scaled by 2^11 and its two products go to
// a second accumulator that is scaled back at the end, so the small lo parts
// never fall into fp16 subnormals.
//
// A workgroup of 256 lanes (2 x 2 wavefronts) owns a 128 x 128 tile of C;
// each wavefront a 64 x 64 quarter held as 2 x 2 v_mfma_f32_32x32x16 tiles.
// K advances 32 at a time through a double-buffered LDS stage whose rows are
// padded from 64 to 80 bytes so that the 16-byte fragment reads of 8
// consecutive lanes hit distinct banks.
//
// Accumulator layout of one 32 x 32 tile (16 floats per lane): element
// 4*j + r of lane l is C[8*j + 4*(l/32) + r][l % 32]; operand fragments:
// lane l holds A[l % 32][8*(l/32) .. +8) and B[l % 32][8*(l/32) .. +8) of the
// 16-wide K step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pwfs {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));   // 16 bytes, 8 x 16-bit

constexpr int kGemmTile = 128;  // BM = BN
constexpr int kGemmBK = 32;
constexpr int kLdsRow = 40;     // 16-bit elements per padded LDS row

// ----------------------------------------------------------- conversions --
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f32_to_f16_rne(float x) {
  const _Float16 h = (_Float16)x;
  return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_to_f32(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

// hi/lo split of x in 16-bit format F16 (false = bf16); lo of fp16 scaled by 2^11
template <bool F16>
__device__ __forceinline__ void split16(float x, uint16_t& hi, uint16_t& lo) {
  if constexpr (F16) {
    hi = f32_to_f16_rne(x);
    lo = f32_to_f16_rne((x - f16_to_f32(hi)) * 2048.f);
  } else {
    hi = f32_to_bf16_rne(x);
    lo = f32_to_bf16_rne(x - bf16_to_f32(hi));
  }
}

// --------------------------------------------------------------- engine ---
template <int NPLANES, bool F16>
struct MfmaTile {
  static constexpr int NACC = (F16 && NPLANES == 2) ? 2 : 1;
  static constexpr int STAGE = 2 * NPLANES * kGemmTile * kLdsRow;  // uint16 per stage (A and B)
  static constexpr size_t lds_bytes() { return sizeof(uint16_t) * 2 * STAGE; }

  f32x16_t acc[NACC][2][2];

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int c = 0; c < NACC; ++c)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int e = 0; e < 16; ++e) acc[c][i][j][e] = 0.f;
  }

  // value of accumulator element e of tile (i, j), scale folded in
  __device__ __forceinline__ float value(int i, int j, int e) const {
    if constexpr (NACC == 2) return acc[0][i][j][e] + acc[1][i][j][e] * (1.f / 2048.f);
    else return acc[0][i][j][e];
  }

  __device__ __forceinline__ static f32x16_t mma(u32x4_t a, u32x4_t b, f32x16_t c) {
    if constexpr (F16)
      return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, a), __builtin_bit_cast(f16x8_t, b),
                                                    c, 0, 0, 0);
    else
      return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                     __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
  }

  // Global -> registers for one K step of 32: each lane moves 2 x 16 bytes
  // of each plane of A and of B.  Rows past the operand's end are clamped
  // (their products land in C rows/columns that are never stored).
  struct Pref {
    u32x4_t a[NPLANES][2], b[NPLANES][2];
  };

  // first row of the tile in each plane of A and B
  struct Ops {
    const uint16_t* a[NPLANES];
    const uint16_t* b[NPLANES];
  };

  __device__ __forceinline__ static void fetch(Pref& p, const Ops& o, long long lda, int arows, long long ldb,
                                               int brows, int k0, int tid) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = tid + 256 * h;
      const int row = c >> 2, kq = (c & 3) * 8;
      const int ra = min(row, arows - 1), rb = min(row, brows - 1);
#pragma unroll
      for (int pl = 0; pl < NPLANES; ++pl) {
        p.a[pl][h] = *(const u32x4_t*)(o.a[pl] + (long long)ra * lda + k0 + kq);
        p.b[pl][h] = *(const u32x4_t*)(o.b[pl] + (long long)rb * ldb + k0 + kq);
      }
    }
  }

  __device__ __forceinline__ static void stash(const Pref& p, uint16_t* stage, int tid) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = tid + 256 * h;
      const int row = c >> 2, kq = (c & 3) * 8;
#pragma unroll
      for (int pl = 0; pl < NPLANES; ++pl) {
        *(u32x4_t*)(stage + (pl * kGemmTile + row) * kLdsRow + kq) = p.a[pl][h];
        *(u32x4_t*)(stage + ((NPLANES + pl) * kGemmTile + row) * kLdsRow + kq) = p.b[pl][h];
      }
    }
  }

  // the MFMAs of one 32-wide K step held in `stage`
  __device__ __forceinline__ void compute(const uint16_t* stage, int wm, int wn, int lane) {
    const int r = lane & 31, kh = (lane >> 5) * 8;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      u32x4_t fa[NPLANES][2], fb[NPLANES][2];
#pragma unroll
      for (int pl = 0; pl < NPLANES; ++pl)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          fa[pl][i] = *(const u32x4_t*)(stage + (pl * kGemmTile + wm * 64 + i * 32 + r) * kLdsRow + s * 16 + kh);
          fb[pl][i] = *(const u32x4_t*)(stage + ((NPLANES + pl) * kGemmTile + wn * 64 + i * 32 + r) * kLdsRow +
                                      s * 16 + kh);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[0][i][j] = mma(fa[0][i], fb[0][j], acc[0][i][j]);
          if constexpr (NPLANES == 2) {
            acc[NACC - 1][i][j] = mma(fa[0][i], fb[1][j], acc[NACC - 1][i][j]);
            acc[NACC - 1][i][j] = mma(fa[1][i], fb[0][j], acc[NACC - 1][i][j]);
          }
        }
    }
  }

  // Full K loop of one GEMM tile; K is a multiple of 32.
  __device__ __forceinline__ void run(const Ops o, long long lda, int arows, long long ldb, int brows, int K,
                                      uint16_t* lds, int tid) {
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int nk = K / kGemmBK;
    Pref p;
    fetch(p, o, lda, arows, ldb, brows, 0, tid);
    __syncthreads();   // previous users of the LDS stages are done
    stash(p, lds, tid);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      uint16_t* cur = lds + (kt & 1) * STAGE;
      if (kt + 1 < nk) fetch(p, o, lda, arows, ldb, brows, (kt + 1) * kGemmBK, tid);
      compute(cur, wm, wn, lane);
      if (kt + 1 < nk) stash(p, lds + ((kt + 1) & 1) * STAGE, tid);
      __syncthreads();
    }
  }

  // coordinates (within the 128 x 128 tile) of accumulator element e of
  // this lane's tile (i, j)
  __device__ __forceinline__ static void coord(int tid, int i, int j, int e, int& row, int& col) {
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    row = wm * 64 + i * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
    col = wn * 64 + j * 32 + (lane & 31);
  }
};

}  // namespace pwfs
