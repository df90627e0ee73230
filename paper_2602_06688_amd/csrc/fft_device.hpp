// fft_device.hpp -- radix-{2,3,4,8} Stockham FFT for one group of T lanes
// inside a 64-lane wavefront of gfx950.
//
// A group of T lanes owns one N-point complex transform; lane t holds V = N/T
// values.  A stage of radix R gives each lane V/R butterflies: butterfly j
// (j = t + T*i) reads x[j + q*N/R], q < R, twiddles by w^(k q) with
// k = j mod L (L = product of the earlier radices), runs an R-point DFT and
// writes x[(j/L)*L*R + k + q*L] (Stockham autosort, natural-order output).
// Stages exchange through a per-group LDS buffer of N float2; the groups of a
// workgroup never share a buffer, so only wavefront-scope ordering is needed.
//
// The forward transform ends in registers (lane holds X[j + q*N/R_last]) and
// the inverse transform runs its radices in reverse order, so its first stage
// reads exactly those registers: a pointwise multiply between the two costs
// no LDS round trip.  The inverse's last stage leaves x[j + q*N/R_0] in
// registers, again a fixed set of indices per lane.
#pragma once

#include <hip/hip_runtime.h>

namespace pwfs {

// ------------------------------------------------------------ complex ops --
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ float2 czero() { return make_float2(0.f, 0.f); }

// multiply by -i (forward transform) or +i (inverse transform)
template <bool INV>
__device__ __forceinline__ float2 rot_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// Wavefront-scope barrier with LDS visibility: orders this lane's LDS
// accesses against those of the other lanes of the same wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// -------------------------------------------------------- small DFTs ------
// Each takes its inputs in natural order in a[0..R) and leaves the outputs in
// natural order.  NZ < R means inputs a[NZ..R) are known to be zero (the
// zero-padded part of the first stage) and are never read.

template <int NZ, bool INV>
__device__ __forceinline__ void dft2p(float2& a0, float2& a1) {
  if constexpr (NZ >= 2) {
    const float2 t = a0;
    a0 = cadd(t, a1);
    a1 = csub(t, a1);
  } else if constexpr (NZ == 1) {
    a1 = a0;
  } else {
    a0 = czero();
    a1 = czero();
  }
}

template <int NZ, bool INV>
__device__ __forceinline__ void dft4p(float2* a) {
  // even/odd split: E = DFT2(a0, a2), O = DFT2(a1, a3); X = E +- w4^k O
  constexpr int NE = (NZ + 1) / 2, NO = NZ / 2;
  float2 e0 = a[0], e1 = a[2], o0 = a[1], o1 = a[3];
  dft2p<NE, INV>(e0, e1);
  if constexpr (NO > 0) {
    dft2p<NO, INV>(o0, o1);
    const float2 r1 = rot_mi<INV>(o1);
    a[0] = cadd(e0, o0);
    a[2] = csub(e0, o0);
    a[1] = cadd(e1, r1);
    a[3] = csub(e1, r1);
  } else {
    a[0] = e0;
    a[2] = e0;
    a[1] = e1;
    a[3] = e1;
  }
}

template <int NZ, bool INV>
__device__ __forceinline__ void dft8p(float2* a) {
  constexpr int NE = (NZ + 1) / 2, NO = NZ / 2;
  constexpr float c = 0.70710678118654752440f;
  float2 e[4] = {a[0], a[2], a[4], a[6]};
  float2 o[4] = {a[1], a[3], a[5], a[7]};
  dft4p<NE, INV>(e);
  if constexpr (NO > 0) {
    dft4p<NO, INV>(o);
    // w8^k o[k], w8 = exp(-+ i pi / 4)
    float2 t1, t3;
    if (INV) {
      t1 = make_float2(c * (o[1].x - o[1].y), c * (o[1].x + o[1].y));
      t3 = make_float2(-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y));
    } else {
      t1 = make_float2(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
      t3 = make_float2(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
    }
    const float2 t2 = rot_mi<INV>(o[2]);
    a[0] = cadd(e[0], o[0]);
    a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], t1);
    a[5] = csub(e[1], t1);
    a[2] = cadd(e[2], t2);
    a[6] = csub(e[2], t2);
    a[3] = cadd(e[3], t3);
    a[7] = csub(e[3], t3);
  } else {
    a[0] = e[0]; a[4] = e[0];
    a[1] = e[1]; a[5] = e[1];
    a[2] = e[2]; a[6] = e[2];
    a[3] = e[3]; a[7] = e[3];
  }
}

template <int NZ, bool INV>
__device__ __forceinline__ void dft3p(float2* a) {
  // X0 = a0 + t, X1,2 = a0 - t/2 -+ i (sqrt3/2) d, t = a1 + a2, d = a1 - a2
  constexpr float s = 0.86602540378443864676f;
  if constexpr (NZ >= 2) {
    const float2 a1 = a[1];
    const float2 a2 = (NZ >= 3) ? a[2] : czero();
    const float2 t = cadd(a1, a2);
    const float2 d = csub(a1, a2);
    const float2 m = make_float2(a[0].x - 0.5f * t.x, a[0].y - 0.5f * t.y);
    const float2 r = cscale(rot_mi<INV>(d), s);
    a[0] = cadd(a[0], t);
    a[1] = cadd(m, r);
    a[2] = csub(m, r);
  } else if constexpr (NZ == 1) {
    a[1] = a[0];
    a[2] = a[0];
  } else {
    a[0] = a[1] = a[2] = czero();
  }
}

template <int R, int NZ, bool INV>
__device__ __forceinline__ void dftp(float2* a) {
  static_assert(R == 2 || R == 3 || R == 4 || R == 8, "radix");
  if constexpr (R == 2) dft2p<NZ, INV>(a[0], a[1]);
  else if constexpr (R == 3) dft3p<NZ, INV>(a);
  else if constexpr (R == 4) dft4p<NZ, INV>(a);
  else dft8p<NZ, INV>(a);
}

// ---------------------------------------------------------- radix plans ---
// T lanes per transform; radices of the forward transform in stage order.
template <int N> struct FftPlan;
template <> struct FftPlan<64>  { static constexpr int T = 8;  static constexpr int NS = 2; static constexpr int r[2] = {8, 8}; };
template <> struct FftPlan<128> { static constexpr int T = 16; static constexpr int NS = 3; static constexpr int r[3] = {8, 2, 8}; };
template <> struct FftPlan<256> { static constexpr int T = 32; static constexpr int NS = 3; static constexpr int r[3] = {8, 4, 8}; };
template <> struct FftPlan<384> { static constexpr int T = 32; static constexpr int NS = 5; static constexpr int r[5] = {4, 4, 4, 2, 3}; };
template <> struct FftPlan<512> { static constexpr int T = 64; static constexpr int NS = 3; static constexpr int r[3] = {8, 8, 8}; };
template <> struct FftPlan<768> { static constexpr int T = 64; static constexpr int NS = 5; static constexpr int r[5] = {4, 4, 3, 4, 4}; };

template <int N, int S, bool INV>
struct StageInfo {
  using P = FftPlan<N>;
  static constexpr int idx = INV ? (P::NS - 1 - S) : S;
  static constexpr int R = P::r[idx];
  static constexpr int prodL() {
    int l = 1;
    for (int s = 0; s < S; ++s) l *= P::r[INV ? (P::NS - 1 - s) : s];
    return l;
  }
  static constexpr int L = prodL();
};

// twiddle and butterflies of one stage on the lane's registers
template <int N, int T, int R, int L, int NZ, bool INV>
__device__ __forceinline__ void stage_compute(float2* v, int t, const float2* __restrict__ tw) {
  constexpr int V = N / T, NB = V / R;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if constexpr (L > 1) {
      const int j = t + T * i;
      const int k = j % L;
#pragma unroll
      for (int q = 1; q < R; ++q) {
        float2 w = tw[k * q * (N / (L * R))];
        if (INV) w.y = -w.y;
        v[i * R + q] = cmul(v[i * R + q], w);
      }
    }
    dftp<R, NZ, INV>(&v[i * R]);
  }
}

template <int N, int T, int R>
__device__ __forceinline__ void stage_load(float2* v, int t, const float2* buf) {
  constexpr int V = N / T, NB = V / R;
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int q = 0; q < R; ++q) v[i * R + q] = buf[t + T * i + q * (N / R)];
}

template <int N, int T, int R, int L>
__device__ __forceinline__ void stage_store(const float2* v, int t, float2* buf) {
  constexpr int V = N / T, NB = V / R;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + T * i;
    const int base = (j / L) * L * R + (j % L);
#pragma unroll
    for (int q = 0; q < R; ++q) buf[base + q * L] = v[i * R + q];
  }
}

// Runs stages S..NS-1 of a transform whose stage-S input is already in v
// (for S = 0: v[i*R0 + q] = x[t + T*i + q*N/R0], zero-padded entries at
// q >= NZ0 never read).  Leaves the last stage's output in v.
template <int N, bool INV, int S, int NZ0>
__device__ __forceinline__ void fft_from(float2* v, int t, float2* buf, const float2* __restrict__ tw) {
  using P = FftPlan<N>;
  constexpr int T = P::T;
  using SI = StageInfo<N, S, INV>;
  if constexpr (S > 0) {
    wave_sync();                       // previous stage's stores are visible
    stage_load<N, T, SI::R>(v, t, buf);
    wave_sync();                       // every lane has read before anyone writes
  }
  stage_compute<N, T, SI::R, SI::L, (S == 0 ? NZ0 : SI::R), INV>(v, t, tw);
  if constexpr (S + 1 < P::NS) {
    stage_store<N, T, SI::R, SI::L>(v, t, buf);
    fft_from<N, INV, S + 1, NZ0>(v, t, buf, tw);
  }
}

// index held by register slot (i, q) after the last forward stage / before
// the first inverse stage
template <int N>
__device__ __forceinline__ int freq_index(int t, int slot) {
  using P = FftPlan<N>;
  constexpr int R = P::r[P::NS - 1];
  const int i = slot / R, q = slot % R;
  return t + P::T * i + q * (N / R);
}

// index held by register slot (i, q) of the first forward stage's input /
// the last inverse stage's output
template <int N>
__device__ __forceinline__ int space_index(int t, int slot) {
  using P = FftPlan<N>;
  constexpr int R = P::r[0];
  const int i = slot / R, q = slot % R;
  return t + P::T * i + q * (N / R);
}

// ------------------------------------------- register-twiddle variant ----
// For plans whose radix list reads the same forwards and backwards, stage s
// of the inverse transform has the same radix and the same L as stage s of
// the forward one, so its twiddles are the conjugates of the forward ones.
// Each lane then keeps the twiddles of all its butterflies in registers for
// the whole kernel, and the LDS exchange buffer is padded (ExPad below) to
// spread the strided Stockham stores over the banks.

template <int N>
struct Palindromic {
  static constexpr bool check() {
    using P = FftPlan<N>;
    for (int s = 0; s < P::NS; ++s)
      if (P::r[s] != P::r[P::NS - 1 - s]) return false;
    return P::NS <= 5;
  }
  static constexpr bool value = check();
};

// Padding of the exchange buffer at stage boundary B (the stores after
// stage B and the loads before stage B + 1): element i sits at
// i + PB (i >> A).  One float2 in 8 spreads the radix-8 plans' strided
// stores; the 4 4 3 4 4 plan of 768 has its own per boundary, chosen with a
// bank model of each boundary's stores and loads (lanes of one 16- or
// 32-lane LDS cycle on distinct banks): boundary 0 (stride-4 stores, paired
// into 16-byte writes) 2 in 32, boundary 1 (runs of 4 lanes, 16 apart) 1 in
// 4, boundaries 2 and 3 (runs of 16 and 48 lanes) none.  Each padding is
// additive over offsets that are multiples of 64, so the addresses stay one
// per-lane base plus immediates.
template <int N, int B> struct ExPad { static constexpr int A = 3, PB = 1; };
template <> struct ExPad<768, 0> { static constexpr int A = 5, PB = 2; };
template <> struct ExPad<768, 1> { static constexpr int A = 2, PB = 1; };
template <> struct ExPad<768, 2> { static constexpr int A = 0, PB = 0; };
template <> struct ExPad<768, 3> { static constexpr int A = 0, PB = 0; };

template <int N, int B>
__device__ __forceinline__ int lds_pad(int i) {
  using X = ExPad<N, B>;
  if constexpr (X::PB == 0) return i;
  else return i + X::PB * (i >> X::A);
}
template <int N> struct PaddedLen {
  static constexpr int len() {
    int m = N;
    for (int b = 0; b + 1 < FftPlan<N>::NS; ++b) {
      const int a = b == 0 ? ExPad<N, 0>::A : b == 1 ? ExPad<N, 1>::A : b == 2 ? ExPad<N, 2>::A : ExPad<N, 3>::A;
      const int pb = b == 0 ? ExPad<N, 0>::PB : b == 1 ? ExPad<N, 1>::PB : b == 2 ? ExPad<N, 2>::PB : ExPad<N, 3>::PB;
      const int l = N + pb * (N >> a);
      if (l > m) m = l;
    }
    return m;
  }
  static constexpr int value = len();
};

template <int N, int S>
struct StageTw {
  using SI = StageInfo<N, S, false>;
  static constexpr int T = FftPlan<N>::T;
  static constexpr int R = SI::R, L = SI::L, NB = (N / T) / SI::R;
  // butterfly i of lane t uses k = (t + T i) mod L: the same k for every i
  // when L divides T, so one set of twiddles serves all of them
  static constexpr bool SAME = (T % L) == 0;
  static constexpr int NW = SAME ? 1 : NB;
  float2 w[NW][R - 1];
  __device__ __forceinline__ void load(int t, const float2* tw) {
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const int k = (t + T * i) % L;
#pragma unroll
      for (int q = 1; q < R; ++q) w[i][q - 1] = tw[k * q * (N / (L * R))];
    }
  }
  __device__ __forceinline__ float2 at(int i, int q) const { return w[SAME ? 0 : i][q - 1]; }
};

template <int N>
struct TwSet {
  static constexpr int NS = FftPlan<N>::NS;
  StageTw<N, 1> s1;
  StageTw<N, (NS > 2 ? 2 : 1)> s2;
  StageTw<N, (NS > 3 ? 3 : 1)> s3;
  StageTw<N, (NS > 4 ? 4 : 1)> s4;
  __device__ __forceinline__ void load(int t, const float2* tw) {
    s1.load(t, tw);
    if constexpr (NS > 2) s2.load(t, tw);
    if constexpr (NS > 3) s3.load(t, tw);
    if constexpr (NS > 4) s4.load(t, tw);
  }
};

// conj(w) * a when INV, w * a otherwise
template <bool INV>
__device__ __forceinline__ float2 twmul(float2 a, float2 w) {
  return INV ? make_float2(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y) : cmul(a, w);
}

template <int N, int S, int NZ, bool INV, class TW>
__device__ __forceinline__ void stage_compute_reg(float2* v, const TW& tw) {
  constexpr int T = FftPlan<N>::T, V = N / T;
  using SI = StageInfo<N, S, INV>;
  constexpr int R = SI::R, NB = V / R;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if constexpr (S > 0) {
#pragma unroll
      for (int q = 1; q < R; ++q) v[i * R + q] = twmul<INV>(v[i * R + q], tw.at(i, q));
    }
    dftp<R, NZ, INV>(&v[i * R]);
  }
}

// loads before stage B + 1 of radix R, from boundary B's layout
template <int N, int R, int B>
__device__ __forceinline__ void stage_load_pad(float2* v, int t, const float2* buf) {
  constexpr int T = FftPlan<N>::T, V = N / T, NB = V / R;
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int q = 0; q < R; ++q) v[i * R + q] = buf[lds_pad<N, B>(t + T * i + q * (N / R))];
}

// stores after stage B (radix R, span L) in boundary B's layout
template <int N, int R, int L, int B>
__device__ __forceinline__ void stage_store_pad(const float2* v, int t, float2* buf) {
  constexpr int T = FftPlan<N>::T, V = N / T, NB = V / R;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + T * i;
    const int base = (j / L) * L * R + (j % L);
#pragma unroll
    for (int q = 0; q < R; ++q) buf[lds_pad<N, B>(base + q * L)] = v[i * R + q];
  }
}

template <int N, int S>
__device__ __forceinline__ const auto& tw_of(const TwSet<N>& tw) {
  if constexpr (S == 1) return tw.s1;
  else if constexpr (S == 2) return tw.s2;
  else if constexpr (S == 3) return tw.s3;
  else return tw.s4;
}

// Same contract as fft_from, for palindromic plans, with register twiddles
// and a padded buffer of PaddedLen<N> float2.
template <int N, bool INV, int S, int NZ0>
__device__ __forceinline__ void fft_reg(float2* v, int t, float2* buf, const TwSet<N>& tw) {
  using P = FftPlan<N>;
  using SI = StageInfo<N, S, INV>;
  static_assert(Palindromic<N>::value, "plan must be palindromic");
  if constexpr (S == 0 && P::NS > 3) {
    // long plans: the lane index is made opaque at each transform, so the
    // exchange addresses of all stages are recomputed here rather than
    // hoisted out of the caller's loops into registers
    __asm__ volatile("" : "+v"(t));
  }
  if constexpr (S > 0) {
    wave_sync();
    stage_load_pad<N, SI::R, S - 1>(v, t, buf);
    wave_sync();
    stage_compute_reg<N, S, SI::R, INV>(v, tw_of<N, S>(tw));
  } else {
    stage_compute_reg<N, 0, NZ0, INV>(v, tw.s1);
  }
  if constexpr (S + 1 < P::NS) {
    stage_store_pad<N, SI::R, SI::L, S>(v, t, buf);
    fft_reg<N, INV, S + 1, NZ0>(v, t, buf, tw);
  }
}

}  // namespace pwfs
