// Register-resident Stockham FFT with LDS exchanges, for power-of-two lengths L <= 1024.
//
// A line of length L is owned by TL = L / E threads; thread t holds the E values at the
// natural positions t + m * TL (m = 0 .. E-1) before and after every stage.  A stage of radix
// R (R divides E) performs E / R radix-R butterflies per thread on values already in its
// registers: butterfly j = t + b * TL reads positions j + r * L / R (= register b + r * E / R),
// multiplies by W_{Ns R}^{r (j mod Ns)} and writes positions (j / Ns) Ns R + (j mod Ns) + r Ns
// (autosorting Stockham, decimation in time).  Between stages the outputs go through LDS so that
// every thread again holds natural positions; after the last stage (Ns R = L) the outputs
// already sit at the natural positions of the same registers, so a K-stage FFT costs K - 1 LDS
// round trips and the first and last stages read/write global memory directly (coalesced:
// consecutive t touch consecutive positions).
//
// Radix sequence: E, E, ..., then the remainder (< E) if L is not a power of E.
// Twiddles come from a float64 table of TW_N entries exp(-2 pi i k / TW_N) computed on the
// host from the definition; the complex64 path uses the same table rounded to float.
#pragma once

#include <utility>

#include "common.hpp"

namespace ie {

// cos / sin of 2 pi k / 16
__device__ constexpr double kC16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
__device__ constexpr double kS16[16] = {
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

// x * W_R^K with W_R = exp(-+ 2 pi i / R) (minus for the forward transform); R <= 16.
template <int K, int R, bool INV, typename T>
__device__ __forceinline__ cx<T> mul_wr(cx<T> x) {
  constexpr int k16 = ((K * 16) / R) & 15;
  if constexpr (k16 == 0) {
    return x;
  } else if constexpr (k16 == 4) {
    return INV ? cx<T>{-x.im, x.re} : cx<T>{x.im, -x.re};
  } else if constexpr (k16 == 8) {
    return cx<T>{-x.re, -x.im};
  } else if constexpr (k16 == 12) {
    return INV ? cx<T>{x.im, -x.re} : cx<T>{-x.im, x.re};
  } else {
    const T c = T(kC16[k16]);
    const T s = INV ? T(kS16[k16]) : T(-kS16[k16]);
    return cx<T>{x.re * c - x.im * s, x.re * s + x.im * c};
  }
}

// In-register DFT of size R (power of two <= 16), recursive radix-2 decimation in time.
template <typename T, int R, bool INV>
struct Dft {
  template <int... K>
  static __device__ __forceinline__ void combine(cx<T>* u, const cx<T>* e, const cx<T>* o,
                                                 std::integer_sequence<int, K...>) {
    (
        [&] {
          const cx<T> t = mul_wr<K, R, INV>(o[K]);
          u[K] = e[K] + t;
          u[K + R / 2] = e[K] - t;
        }(),
        ...);
  }
  static __device__ __forceinline__ void run(cx<T>* u) {
    cx<T> e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = u[2 * i];
      o[i] = u[2 * i + 1];
    }
    Dft<T, R / 2, INV>::run(e);
    Dft<T, R / 2, INV>::run(o);
    combine(u, e, o, std::make_integer_sequence<int, R / 2>{});
  }
};
template <typename T, bool INV>
struct Dft<T, 1, INV> {
  static __device__ __forceinline__ void run(cx<T>*) {}
};

template <typename T, bool INV>
__device__ __forceinline__ cx<T> twiddle(const cx<T>* __restrict__ tw, int idx) {
  cx<T> w = tw[idx];
  if (INV) w.im = -w.im;
  return w;
}

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

// Radix of stage s for length L, register width E.
template <int L, int E>
constexpr int stage_radix(int s) {
  int rem = L;
  for (int i = 0; i < s; ++i) rem /= (rem >= E ? E : rem);
  return rem >= E ? E : rem;
}
template <int L, int E>
constexpr int num_stages() {
  int rem = L, k = 0;
  while (rem > 1) {
    rem /= (rem >= E ? E : rem);
    ++k;
  }
  return k;
}
template <int L, int E>
constexpr int stage_ns(int s) {  // product of the radices before stage s
  int ns = 1;
  for (int i = 0; i < s; ++i) ns *= stage_radix<L, E>(i);
  return ns;
}

// LDS addressing of one line: position p of line `line` in a buffer whose lines are either
// interleaved (stride 1 between lines, LINES lines) or contiguous with padding.
struct LdsInterleaved {
  int lines;  // number of interleaved lines
  int line;
  __device__ __forceinline__ int operator()(int p) const { return p * lines + line; }
};
struct LdsPadded {  // line-major, one pad slot every 16 positions (conflict-free strided access)
  int base;
  __device__ __forceinline__ int operator()(int p) const { return base + p + (p >> 4); }
  static constexpr __host__ __device__ int padded_len(int L) { return L + L / 16; }
};
// line-major, one pad slot every 4 positions (stride-4 writes of a radix-4 first stage land on
// distinct banks), lines offset by half a bank row more
struct LdsPadded4 {
  int base;
  __device__ __forceinline__ int operator()(int p) const { return base + p + (p >> 2); }
  static constexpr __host__ __device__ int padded_len(int L) { return L + L / 4 + 16; }
};

template <typename T, int L, int E, int S, bool INV, typename Addr>
__device__ __forceinline__ void fft_stage(cx<T> (&v)[E], cx<T>* __restrict__ lds, Addr addr,
                                          int t, const cx<T>* __restrict__ tw) {
  constexpr int R = stage_radix<L, E>(S);
  constexpr int NS = stage_ns<L, E>(S);
  constexpr int TL = L / E;
  constexpr int NB = E / R;
  constexpr bool LAST = (S == num_stages<L, E>() - 1);
  static_assert(E % R == 0, "radix must divide the register width");
  cx<T> out[E];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = t + b * TL;
    const int k = j & (NS - 1);
    cx<T> u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[b + r * NB];
    if constexpr (NS > 1) {
      constexpr int step = TW_N / (NS * R);
#pragma unroll
      for (int r = 1; r < R; ++r) u[r] = u[r] * twiddle<T, INV>(tw, r * k * step);
    }
    Dft<T, R, INV>::run(u);
#pragma unroll
    for (int r = 0; r < R; ++r) out[b + r * NB] = u[r];
  }
  if constexpr (LAST) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = out[m];
  } else {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = t + b * TL;
      const int k = j & (NS - 1);
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[addr(base + r * NS)] = out[b + r * NB];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = lds[addr(t + m * TL)];
    __syncthreads();
  }
}

template <typename T, int L, int E, bool INV, typename Addr, int... S>
__device__ __forceinline__ void fft_stages(cx<T> (&v)[E], cx<T>* lds, Addr addr, int t,
                                           const cx<T>* tw, std::integer_sequence<int, S...>) {
  (fft_stage<T, L, E, S, INV>(v, lds, addr, t, tw), ...);
}

// Full length-L FFT of the line held in v (natural positions t + m L/E on entry and exit).
// Every thread of the block must call it (it contains __syncthreads when L > E).
template <typename T, int L, int E, bool INV, typename Addr>
__device__ __forceinline__ void fft_line(cx<T> (&v)[E], cx<T>* lds, Addr addr, int t,
                                         const cx<T>* __restrict__ tw) {
  static_assert(L % E == 0 && L <= MAX_FFT_LEN, "bad FFT length");
  fft_stages<T, L, E, INV>(v, lds, addr, t, tw,
                           std::make_integer_sequence<int, num_stages<L, E>()>{});
}

// The same FFT for NC lines held by one thread (v[c], c < NC), in lockstep: the twiddles of
// each stage are loaded once and applied to every line, and the lines go through LDS one after
// the other (one line of LDS space).
template <typename T, int L, int E, int S, bool INV, int NC, typename Addr>
__device__ __forceinline__ void fft_stage_multi(cx<T> (&v)[NC][E], cx<T>* __restrict__ lds,
                                                Addr addr, int t,
                                                const cx<T>* __restrict__ tw) {
  constexpr int R = stage_radix<L, E>(S);
  constexpr int NS = stage_ns<L, E>(S);
  constexpr int TL = L / E;
  constexpr int NB = E / R;
  constexpr bool LAST = (S == num_stages<L, E>() - 1);
  static_assert(E % R == 0, "radix must divide the register width");
  cx<T> w[NB][R];
  if constexpr (NS > 1) {
    constexpr int step = TW_N / (NS * R);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int k = (t + b * TL) & (NS - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) w[b][r] = twiddle<T, INV>(tw, r * k * step);
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    cx<T> out[E];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      cx<T> u[R];
#pragma unroll
      for (int r = 0; r < R; ++r) u[r] = v[c][b + r * NB];
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) u[r] = u[r] * w[b][r];
      }
      Dft<T, R, INV>::run(u);
#pragma unroll
      for (int r = 0; r < R; ++r) out[b + r * NB] = u[r];
    }
    if constexpr (LAST) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[c][m] = out[m];
    } else {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = t + b * TL;
        const int k = j & (NS - 1);
        const int base = (j / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[addr(base + r * NS)] = out[b + r * NB];
      }
      __syncthreads();
#pragma unroll
      for (int m = 0; m < E; ++m) v[c][m] = lds[addr(t + m * TL)];
      __syncthreads();
    }
  }
}

template <typename T, int L, int E, bool INV, int NC, typename Addr, int... S>
__device__ __forceinline__ void fft_stages_multi(cx<T> (&v)[NC][E], cx<T>* lds, Addr addr, int t,
                                                 const cx<T>* tw,
                                                 std::integer_sequence<int, S...>) {
  (fft_stage_multi<T, L, E, S, INV, NC>(v, lds, addr, t, tw), ...);
}

template <typename T, int L, int E, bool INV, int NC, typename Addr>
__device__ __forceinline__ void fft_lines(cx<T> (&v)[NC][E], cx<T>* lds, Addr addr, int t,
                                          const cx<T>* __restrict__ tw) {
  static_assert(L % E == 0 && L <= MAX_FFT_LEN, "bad FFT length");
  fft_stages_multi<T, L, E, INV, NC>(v, lds, addr, t, tw,
                                     std::make_integer_sequence<int, num_stages<L, E>()>{});
}

}  // namespace ie
