// mfma_gemm.hpp -- split-precision matrix-core GEMM tiles for gfx950.
//
// C[M][N] = sum_k A[M][K] B[N][K] (both operands K-contiguous, "NT"), with
// A and B given as 16-bit planes: one plane (plain bf16) or a hi/lo pair
// (x = hi + lo, three products hi*hi + hi*lo + lo*hi accumulated in fp32).
// For fp16 the lo plane is stored scaled by 2^11, so the small lo parts never
// fall into fp16 subnormals; the hi*hi product then takes A's hi fragment
// scaled by 2^11 in registers (exact: every A operand here has |a| <= 1), so
// the three products share one accumulator that holds 2^11 C.
//
// A workgroup of 256 lanes (2 x 2 wavefronts) owns a 128 x 128 tile of C
// (the wave-specialised workgroups at the end of this file use the same
// tiles inside larger ones);
// each wavefront a 64 x 64 quarter held as 2 x 2 v_mfma_f32_32x32x16 tiles.
// K advances BK (32 or 64) at a time through a double-buffered LDS stage
// whose rows are padded by 16 bytes (2 BK + 16 bytes each) so that the
// 16-byte fragment reads of 16 consecutive lanes hit distinct banks.
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
constexpr int kGemmBK = 32;     // default K step

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
// BN: columns of C per workgroup tile (128, or 256 for the wave-specialised
// kernels, whose consumer waves then form 2 x 4 quarters of 64 x 64).
template <int NPLANES, bool F16, int BK = kGemmBK, int BN = kGemmTile>
struct MfmaTile {
  static_assert(BK == 32 || BK == 64, "K step of 32 or 64");
  static_assert(BN == 128 || BN == 256, "128 or 256 columns per tile");
  static constexpr bool SCALED = F16 && NPLANES == 2;   // accumulator holds 2^11 C
  static constexpr int BK_ = BK;
  static constexpr int NPL_ = NPLANES;
  static constexpr int LROW = BK + 8;     // 16-bit elements per padded LDS row
  static constexpr int H = BK / 16;       // 16-byte chunks per lane and operand plane in one K step
  static constexpr int BROW0 = NPLANES * kGemmTile;              // first B row of a stage
  static constexpr int STAGE = NPLANES * (kGemmTile + BN) * LROW;  // uint16 per stage (A planes, then B planes)
  static constexpr size_t lds_bytes() { return sizeof(uint16_t) * 2 * STAGE; }

  f32x16_t acc[2][2];

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
  }

  // value of accumulator element e of tile (i, j), scale folded in
  __device__ __forceinline__ float value(int i, int j, int e) const {
    if constexpr (SCALED) return acc[i][j][e] * (1.f / 2048.f);
    else return acc[i][j][e];
  }

  // element offset, within a stage, of element k of stage row r
  __device__ __forceinline__ static int slot(int r, int k) { return r * LROW + k; }

  __device__ __forceinline__ static f32x16_t mma(u32x4_t a, u32x4_t b, f32x16_t c) {
    if constexpr (F16)
      return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, a), __builtin_bit_cast(f16x8_t, b),
                                                    c, 0, 0, 0);
    else
      return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                     __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
  }

  // Global -> registers for one K step: each lane moves H x 16 bytes of each
  // plane of A and of B.  Rows past the operand's end are clamped (their
  // products land in C rows/columns that are never stored).
  struct Pref {
    u32x4_t a[NPLANES][H], b[NPLANES][H];
  };

  // first row of the tile in each plane of A and B
  struct Ops {
    const uint16_t* a[NPLANES];
    const uint16_t* b[NPLANES];
  };

  // the tile row and K offset of the 16-byte chunk lane tid moves in part h
  // of a fetch
  __device__ __forceinline__ static void fetch_slot(int tid, int h, int& row, int& kq) {
    const int c = tid + 256 * h;
    row = c / (BK / 8);
    kq = (c % (BK / 8)) * 8;
  }

  __device__ __forceinline__ static void fetch(Pref& p, const Ops& o, long long lda, int arows, long long ldb,
                                               int brows, int k0, int tid) {
#pragma unroll
    for (int h = 0; h < H; ++h) {
      int row, kq;
      fetch_slot(tid, h, row, kq);
      const int ra = min(row, arows - 1), rb = min(row, brows - 1);
#pragma unroll
      for (int pl = 0; pl < NPLANES; ++pl) {
        p.a[pl][h] = *(const u32x4_t*)(o.a[pl] + (long long)ra * lda + k0 + kq);
        p.b[pl][h] = *(const u32x4_t*)(o.b[pl] + (long long)rb * ldb + k0 + kq);
      }
    }
  }

  // Global -> registers for one K step with per-lane row offsets (elements,
  // the chunk's K offset included) given by the caller: ao[h] and bo[h]
  // address the rows of A and B this lane moves in part h.
  __device__ __forceinline__ static void fetch_at(Pref& p, const Ops& o, const long long (&ao)[H],
                                                  const long long (&bo)[H], int k0) {
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int pl = 0; pl < NPLANES; ++pl) {
        p.a[pl][h] = *(const u32x4_t*)(o.a[pl] + ao[h] + k0);
        p.b[pl][h] = *(const u32x4_t*)(o.b[pl] + bo[h] + k0);
      }
  }

  __device__ __forceinline__ static void stash(const Pref& p, uint16_t* stage, int tid) {
#pragma unroll
    for (int h = 0; h < H; ++h) {
      int row, kq;
      fetch_slot(tid, h, row, kq);
#pragma unroll
      for (int pl = 0; pl < NPLANES; ++pl) {
        *(u32x4_t*)(stage + slot(pl * kGemmTile + row, kq)) = p.a[pl][h];
        *(u32x4_t*)(stage + slot(BROW0 + pl * BN + row, kq)) = p.b[pl][h];
      }
    }
  }

  // the MFMAs of one K step held in `stage`
  __device__ __forceinline__ void compute(const uint16_t* stage, int wm, int wn, int lane) {
    const int r = lane & 31, kh = (lane >> 5) * 8;
#pragma unroll
    for (int s = 0; s < BK / 16; ++s) {
      u32x4_t fa[NPLANES][2], fb[NPLANES][2];
#pragma unroll
      for (int pl = 0; pl < NPLANES; ++pl)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          fa[pl][i] = *(const u32x4_t*)(stage + slot(pl * kGemmTile + wm * 64 + i * 32 + r, s * 16 + kh));
          fb[pl][i] = *(const u32x4_t*)(stage + slot(BROW0 + pl * BN + wn * 64 + i * 32 + r, s * 16 + kh));
        }
      // term-major: the products that accumulate into one tile are four
      // MFMAs apart, so none waits for the one before it; each tile still
      // adds hi*hi, hi*lo, lo*hi in that order
      u32x4_t hi_a[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        hi_a[i] = fa[0][i];
        if constexpr (SCALED)
          hi_a[i] = __builtin_bit_cast(u32x4_t, __builtin_bit_cast(f16x8_t, hi_a[i]) * (_Float16)2048.0f);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mma(hi_a[i], fb[0][j], acc[i][j]);
      if constexpr (NPLANES == 2) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = mma(fa[0][i], fb[1][j], acc[i][j]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = mma(fa[1][i], fb[0][j], acc[i][j]);
      }
    }
  }

  // Full K loop of one GEMM tile; K is a multiple of BK.
  __device__ __forceinline__ void run(const Ops o, long long lda, int arows, long long ldb, int brows, int K,
                                      uint16_t* lds, int tid) {
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int nk = K / BK;
    Pref p;
    fetch(p, o, lda, arows, ldb, brows, 0, tid);
    __syncthreads();   // previous users of the LDS stages are done
    stash(p, lds, tid);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      uint16_t* cur = lds + (kt & 1) * STAGE;
      if (kt + 1 < nk) fetch(p, o, lda, arows, ldb, brows, (kt + 1) * BK, tid);
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

// ------------------------------------------------- wave-specialised tiles --
// Wave-specialised workgroups for large products.  The consumer waves (2 x
// BN/64 of them, each a 64 x 64 quarter of a 128 x BN tile) run the MFMAs
// and the epilogue, reading each K step from one of two LDS stages.  Four
// producer waves only move operands: every producer lane owns CH 16-byte
// chunks of a K step and keeps DEPTH steps of them in flight in registers;
// at each step it stores the oldest into the stage the consumers read next
// and issues the loads of the step DEPTH further on.  A step's loads thus
// have DEPTH steps of matrix work to arrive (a 256-lane workgroup whose
// waves both fetch and compute could keep only one step in flight within
// its registers).  The two roles live in separate loops, so their registers
// are not held at the same time; both pass the same workgroup barriers, one
// per K step.  A wider tile (BN = 256) reads each row of A once for twice
// the columns.  One-plane products run K steps of 64 (16 products per
// consumer wave between barriers), two-plane products K steps of 32 (their
// three products already give 24).  The consumers run the same compute()
// as the 256-lane workgroup, so a tile's products, and its bits, are the
// same in both.
template <int NPL, bool F16, int BN>
using WsEngine = MfmaTile<NPL, F16, NPL == 1 ? 64 : 32, BN>;

// Chunk layout of one K step for the producers: part h (lane pt moves chunk
// pt + 256 h) covers RPP whole rows of one plane block of A or of B.
template <class E, int BN>
struct WsParts {
  static constexpr int NPL = E::NPL_;
  static constexpr int CPR = E::BK_ / 8;                   // 16-byte chunks per row and step
  static constexpr int ROWS = NPL * (kGemmTile + BN);      // A planes, then B planes
  static constexpr int RPP = 256 / CPR;                    // rows per part
  static constexpr int CH = ROWS / RPP;                    // parts
  static_assert(CH * RPP == ROWS && kGemmTile % RPP == 0 && BN % RPP == 0,
                "each producer part lies in one plane block of A or B");
  static_assert(CPR != 4 || RPP == 64, "the row order of a part covers 64 rows");
  // plane block of part h: A planes 0..NPL-1, then B planes (compile-time per h)
  static constexpr bool is_a(int h) { return h * RPP < NPL * kGemmTile; }
  static constexpr int plane(int h) { return is_a(h) ? h * RPP / kGemmTile : (h * RPP - NPL * kGemmTile) / BN; }
  // Stage row and K offset of lane pt's chunk in part h.  Four consecutive
  // lanes move the four chunks (64 contiguous bytes) of one row.  With K
  // steps of 32 the padded rows are 80 bytes (5 16-byte bank quads) apart,
  // so the 32 lanes of one store are given the rows a + 4m, m = 0..7: their
  // chunks then fill distinct quads of the 512 bytes of LDS banks (and so of
  // each 256-byte half), where eight consecutive rows would overlap.
  __device__ static int stage_row(int pt, int h) {
    if constexpr (CPR == 4) {
      const int grp = pt >> 5, w = pt & 31;
      return h * RPP + ((grp >> 2) << 5) + (grp & 3) + 4 * (w >> 2);
    } else {
      return (pt + 256 * h) / CPR;
    }
  }
  __device__ static int kq(int pt, int h) {
    if constexpr (CPR == 4) return (pt & 3) * 8;
    else return ((pt + 256 * h) % CPR) * 8;
  }
  // tile row of the chunk within its operand
  __device__ static int row(int pt, int h) {
    const int rr = stage_row(pt, h);
    return is_a(h) ? rr % kGemmTile : (rr - NPL * kGemmTile) % BN;
  }
  __device__ static int lds_offset(int pt, int h) { return E::slot(stage_row(pt, h), kq(pt, h)); }
};

// The producer loop.  fetch(buf, s) issues the loads of step s into buf;
// every fetch is issued unconditionally (steps past the end re-load the last
// step, unused), so the compiler's in-order load counter sees the same DEPTH
// sets in flight on every path and waits only for the oldest.
template <class E, int DEPTH, int CH, class Fetch>
__device__ __forceinline__ void ws_produce(uint16_t* lds, const int (&loff)[CH], int steps, Fetch fetch) {
  u32x4_t buf[DEPTH][CH];
  auto stash = [&](const u32x4_t (&b)[CH], uint16_t* stage) {
#pragma unroll
    for (int h = 0; h < CH; ++h) *(u32x4_t*)(stage + loff[h]) = b[h];
  };
#pragma unroll
  for (int u = 0; u < DEPTH; ++u) fetch(buf[u], min(u, steps - 1));
  stash(buf[0], lds);
  fetch(buf[0], min(DEPTH, steps - 1));
  __syncthreads();
  int st = 0;
  for (; st + DEPTH <= steps; st += DEPTH) {
#pragma unroll
    for (int u = 0; u < DEPTH; ++u) {
      // step st + u + 1 waits in buf[(u + 1) % DEPTH]: it goes to the stage
      // the consumers read after this barrier, and the buffer takes the step
      // DEPTH further on
      stash(buf[(u + 1) % DEPTH], lds + ((st + u + 1) & 1) * E::STAGE);
      fetch(buf[(u + 1) % DEPTH], min(st + u + 1 + DEPTH, steps - 1));
      __syncthreads();
    }
  }
  // the last steps (fewer than DEPTH) are already in flight
#pragma unroll
  for (int u = 0; u < DEPTH - 1; ++u) {
    if (st + u >= steps) break;
    if (st + u + 1 < steps) stash(buf[(u + 1) % DEPTH], lds + ((st + u + 1) & 1) * E::STAGE);
    __syncthreads();
  }
}

}  // namespace pwfs
