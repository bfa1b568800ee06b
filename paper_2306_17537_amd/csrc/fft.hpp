// Register-resident Stockham FFT with LDS exchanges, for lengths L = 2^k or 3 * 2^k up to 1024.
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
// Radix sequence: per stage the largest divisor of E that divides what is left (E, E, ..., then
// the remainder for powers of two; E is a multiple of 3 for the 3 * 2^k lengths).
// Twiddles come from a float64 table of TW_N entries exp(-2 pi i k / TW_N) computed on the
// host from the definition (TW_N is a multiple of every supported L); the complex64 path uses
// the same table rounded to float.
#pragma once

#include <utility>

#include "common.hpp"

namespace ie {

// cos / sin of 2 pi k / 48 (every angle a radix of 2, 3, 4, 6, 8, 12 or 16 needs)
__device__ constexpr double kC48[48] = {
    1.0, 0.99144486137381041114, 0.96592582628906828675, 0.92387953251128675613,
    0.86602540378443864676, 0.79335334029123516458, 0.70710678118654752440,
    0.60876142900872063942, 0.5, 0.38268343236508977173, 0.25881904510252076235,
    0.13052619222005159155, 0.0, -0.13052619222005159155, -0.25881904510252076235,
    -0.38268343236508977173, -0.5, -0.60876142900872063942, -0.70710678118654752440,
    -0.79335334029123516458, -0.86602540378443864676, -0.92387953251128675613,
    -0.96592582628906828675, -0.99144486137381041114, -1.0, -0.99144486137381041114,
    -0.96592582628906828675, -0.92387953251128675613, -0.86602540378443864676,
    -0.79335334029123516458, -0.70710678118654752440, -0.60876142900872063942, -0.5,
    -0.38268343236508977173, -0.25881904510252076235, -0.13052619222005159155, 0.0,
    0.13052619222005159155, 0.25881904510252076235, 0.38268343236508977173, 0.5,
    0.60876142900872063942, 0.70710678118654752440, 0.79335334029123516458,
    0.86602540378443864676, 0.92387953251128675613, 0.96592582628906828675,
    0.99144486137381041114};

// x * W_R^K with W_R = exp(-+ 2 pi i / R) (minus for the forward transform); R divides 48.
template <int K, int R, bool INV, typename T>
__device__ __forceinline__ cx<T> mul_wr(cx<T> x) {
  static_assert(48 % R == 0, "radix must divide 48");
  constexpr int k48 = ((K * 48) / R) % 48;
  if constexpr (k48 == 0) {
    return x;
  } else if constexpr (k48 == 12) {
    return INV ? cx<T>{-x.im, x.re} : cx<T>{x.im, -x.re};
  } else if constexpr (k48 == 24) {
    return cx<T>{-x.re, -x.im};
  } else if constexpr (k48 == 36) {
    return INV ? cx<T>{x.im, -x.re} : cx<T>{-x.im, x.re};
  } else {
    const T c = T(kC48[k48]);
    const T sn = T(kC48[(k48 + 36) % 48]);  // sin(a) = cos(a - pi/2)
    const T s = INV ? sn : -sn;
    return cx<T>{x.re * c - x.im * s, x.re * s + x.im * c};
  }
}

// In-register DFT of size R: radix-2 decimation in time down to sizes 1 or 3, so R is a power
// of two or three times one (R divides 48).
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
    static_assert(R % 2 == 0, "even radix expected");
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
// size 3: X0 = a + b + c, X1,2 = a - (b + c)/2 -+ i (sqrt 3 / 2)(b - c) (forward; signs swap
// for the inverse)
template <typename T, bool INV>
struct Dft<T, 3, INV> {
  static __device__ __forceinline__ void run(cx<T>* u) {
    constexpr T h = T(0.86602540378443864676);  // sqrt(3)/2
    const cx<T> a = u[0], t1 = u[1] + u[2], t2 = u[1] - u[2];
    const cx<T> m = {a.re - T(0.5) * t1.re, a.im - T(0.5) * t1.im};
    const cx<T> r = INV ? cx<T>{-h * t2.im, h * t2.re} : cx<T>{h * t2.im, -h * t2.re};
    u[0] = a + t1;
    u[1] = m + r;
    u[2] = m - r;
  }
};

// DFT of size R (even) whose inputs R/2 .. R-1 are zero, by decimation in frequency: the even
// outputs are the R/2-point DFT of the first half, the odd outputs that of the first half
// multiplied by W_R^r.
template <typename T, int R, bool INV>
struct DftHalfIn {
  template <int... K>
  static __device__ __forceinline__ void split(const cx<T>* u, cx<T>* e, cx<T>* o,
                                               std::integer_sequence<int, K...>) {
    ((e[K] = u[K], o[K] = mul_wr<K, R, INV>(u[K])), ...);
  }
  static __device__ __forceinline__ void run(cx<T>* u) {
    static_assert(R % 2 == 0, "even radix expected");
    cx<T> e[R / 2], o[R / 2];
    split(u, e, o, std::make_integer_sequence<int, R / 2>{});
    Dft<T, R / 2, INV>::run(e);
    Dft<T, R / 2, INV>::run(o);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      u[2 * k] = e[k];
      u[2 * k + 1] = o[k];
    }
  }
};

template <typename T, bool INV>
__device__ __forceinline__ cx<T> twiddle(const cx<T>* __restrict__ tw, int idx) {
  cx<T> w = tw[idx];
  if (INV) w.im = -w.im;
  return w;
}

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

// Radix of the next stage for `rem` points still to combine: the largest divisor of the register
// width E that divides rem (E, E, ..., then the remainder for powers of two; for 3 * 2^k lengths
// the factor 3 goes into the first stage).
constexpr int pick_radix(int rem, int E) {
  for (int d = E; d >= 2; --d)
    if (E % d == 0 && rem % d == 0) return d;
  return 1;
}
// Radix of stage s for length L, register width E.
template <int L, int E>
constexpr int stage_radix(int s) {
  int rem = L;
  for (int i = 0; i < s; ++i) rem /= pick_radix(rem, E);
  return pick_radix(rem, E);
}
template <int L, int E>
constexpr int num_stages() {
  int rem = L, k = 0;
  while (rem > 1) {
    rem /= pick_radix(rem, E);
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

// Stage-major twiddle table (the layout of the LDS copies): stage s (Ns > 1, radix R) holds
// W_{Ns R}^{r k} at tw_stage_off(s) + (r - 1) Ns + k for r = 1 .. R-1, k < Ns, so that the lanes
// of a stage, whose k = j mod Ns are consecutive, read consecutive entries (a table indexed by
// r k Ns R / L would put lanes 16 or 32 bytes x r k apart: LDS bank conflicts).  The stages
// hold sum (R - 1) Ns = L - R_0 < L entries in all.
constexpr int kTwStaged = -1;  // TWL value that selects this layout
template <int L, int E>
constexpr int tw_stage_off(int S) {
  int off = 0;
  for (int s = 0; s < S; ++s) {
    const int ns = stage_ns<L, E>(s);
    if (ns > 1) off += (stage_radix<L, E>(s) - 1) * ns;
  }
  return off;
}
template <int L, int E>
constexpr int tw_staged_size() {
  return tw_stage_off<L, E>(num_stages<L, E>());
}
// First-twiddle table: stage s (Ns > 1) holds only W_{Ns R}^k at tw_first_off(s) + k, k < Ns,
// and the stage forms W^{r k}, r = 2 .. R-1, as successive powers of it (R - 2 complex
// products, a few float64 roundings).  It takes sum Ns entries instead of sum (R - 1) Ns, which
// is what lets one more block of the float64 x pass share a CU's LDS.
constexpr int kTwFirst = -2;  // TWL value that selects this layout
template <int L, int E>
constexpr int tw_first_off(int S) {
  int off = 0;
  for (int s = 0; s < S; ++s) {
    const int ns = stage_ns<L, E>(s);
    if (ns > 1) off += ns;
  }
  return off;
}
template <int L, int E>
constexpr int tw_first_size() {
  return tw_first_off<L, E>(num_stages<L, E>());
}
template <int L, int E>
__device__ __forceinline__ int tw_first_exp(int i) {
  int off = 0;
  for (int s = 1; s < num_stages<L, E>(); ++s) {
    const int ns = stage_ns<L, E>(s), R = stage_radix<L, E>(s);
    if (i < off + ns) return (i - off) * (L / (ns * R));
    off += ns;
  }
  return 0;
}
// exponent e of W_L^e stored at index i of the stage-major table (tw_first_exp: of the
// first-twiddle table)
template <int L, int E>
__device__ __forceinline__ int tw_staged_exp(int i) {
  int off = 0;
  for (int s = 1; s < num_stages<L, E>(); ++s) {
    const int ns = stage_ns<L, E>(s), R = stage_radix<L, E>(s);
    const int n = (R - 1) * ns;
    if (i < off + n) {
      const int q = i - off;
      return (q / ns + 1) * (q % ns) * (L / (ns * R));
    }
    off += n;
  }
  return 0;
}

// LDS addressing of one line: position p of line `line` in a buffer whose lines are either
// interleaved (stride 1 between lines, LINES lines) or contiguous with padding.
struct LdsInterleaved {
  int lines;  // number of interleaved lines
  int line;
  __device__ __forceinline__ int operator()(int p) const { return p * lines + line; }
};
// line-major without padding, for 16-byte elements: bits 0-3 of a position are XOR-permuted by
// bits 4-7 and 5-6, which spreads the strided accesses of the FFT stages over the LDS banks better
// than a pad slot every 16 positions; only bits 0-3 change, so every aligned group of 16 positions
// maps onto itself (a bijection of 0 .. L-1 for L = 24 and every multiple of 16)
struct LdsSwz {
  int base;
  __device__ __forceinline__ int operator()(int p) const {
    return base + (p ^ ((p >> 4) & 15) ^ ((p >> 5) & 3));
  }
  static constexpr __host__ __device__ int padded_len(int L) { return L; }
};
struct LdsPadded {  // line-major, one pad slot every 16 positions (conflict-free strided access)
  int base;
  __device__ __forceinline__ int operator()(int p) const { return base + p + (p >> 4); }
  static constexpr __host__ __device__ int padded_len(int L) { return L + L / 16; }
};

// ZIN: the positions L/2 .. L-1 are zero on entry (registers E/2 .. E-1), so the first stage
// takes the zero upper half of each butterfly's inputs into account.  TWL: length of the
// twiddle table tw (entries exp(-2 pi i k / TWL); a multiple of L), or kTwStaged / kTwFirst for
// the stage-major or first-twiddle table of this length and register width.
template <typename T, int L, int E, int S, bool INV, bool ZIN, int TWL, typename Addr>
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
    const int k = j % NS;
    cx<T> u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[b + r * NB];
    if constexpr (NS > 1) {
      if constexpr (TWL == kTwFirst) {
        const cx<T> w1 = twiddle<T, INV>(tw, tw_first_off<L, E>(S) + k);
        cx<T> wr = w1;
        u[1] = u[1] * w1;
#pragma unroll
        for (int r = 2; r < R; ++r) {
          wr = wr * w1;
          u[r] = u[r] * wr;
        }
      } else if constexpr (TWL == kTwStaged) {
        constexpr int off = tw_stage_off<L, E>(S);
#pragma unroll
        for (int r = 1; r < R; ++r) u[r] = u[r] * twiddle<T, INV>(tw, off + (r - 1) * NS + k);
      } else {
        constexpr int step = TWL / (NS * R);
#pragma unroll
        for (int r = 1; r < R; ++r) u[r] = u[r] * twiddle<T, INV>(tw, r * k * step);
      }
    }
    if constexpr (ZIN && S == 0 && R % 2 == 0)
      DftHalfIn<T, R, INV>::run(u);
    else
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
      const int k = j % NS;
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

template <typename T, int L, int E, bool INV, bool ZIN, int TWL, typename Addr, int... S>
__device__ __forceinline__ void fft_stages(cx<T> (&v)[E], cx<T>* lds, Addr addr, int t,
                                           const cx<T>* tw, std::integer_sequence<int, S...>) {
  (fft_stage<T, L, E, S, INV, ZIN, TWL>(v, lds, addr, t, tw), ...);
}

// Full length-L FFT of the line held in v (natural positions t + m L/E on entry and exit).
// Every thread of the block must call it (it contains __syncthreads when L > E).  ZIN: the upper
// half of the line is zero on entry (v[E/2 ..] are not read).  TWL: length of the twiddle table
// (the global table of TW_N entries), or kTwStaged / kTwFirst for the stage-major or
// first-twiddle table of this length in LDS (TwStage).
template <typename T, int L, int E, bool INV, bool ZIN = false, int TWL = TW_N, typename Addr>
__device__ __forceinline__ void fft_line(cx<T> (&v)[E], cx<T>* lds, Addr addr, int t,
                                         const cx<T>* __restrict__ tw) {
  static_assert(L % E == 0 && L <= MAX_FFT_LEN &&
                    (TWL == kTwStaged || TWL == kTwFirst || TWL % L == 0),
                "bad FFT length");
  fft_stages<T, L, E, INV, ZIN, TWL>(v, lds, addr, t, tw,
                                     std::make_integer_sequence<int, num_stages<L, E>()>{});
}

// The same FFT for NC lines held by one thread (v[c], c < NC), in lockstep: the twiddles of
// each stage are loaded once and applied to every line, and the lines go through LDS one after
// the other (one line of LDS space).
template <typename T, int L, int E, int S, bool INV, int NC, bool ZIN, int TWL, typename Addr>
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
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int k = (t + b * TL) % NS;
      if constexpr (TWL == kTwStaged) {
        constexpr int off = tw_stage_off<L, E>(S);
#pragma unroll
        for (int r = 1; r < R; ++r) w[b][r] = twiddle<T, INV>(tw, off + (r - 1) * NS + k);
      } else {
        constexpr int step = TWL / (NS * R);
#pragma unroll
        for (int r = 1; r < R; ++r) w[b][r] = twiddle<T, INV>(tw, r * k * step);
      }
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
      if constexpr (ZIN && S == 0 && R % 2 == 0)
        DftHalfIn<T, R, INV>::run(u);
      else
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
        const int k = j % NS;
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

template <typename T, int L, int E, bool INV, int NC, bool ZIN, int TWL, typename Addr,
          int... S>
__device__ __forceinline__ void fft_stages_multi(cx<T> (&v)[NC][E], cx<T>* lds, Addr addr, int t,
                                                 const cx<T>* tw,
                                                 std::integer_sequence<int, S...>) {
  (fft_stage_multi<T, L, E, S, INV, NC, ZIN, TWL>(v, lds, addr, t, tw), ...);
}

// ZIN and TWL as for fft_line.
template <typename T, int L, int E, bool INV, int NC, bool ZIN = false, int TWL = TW_N,
          typename Addr>
__device__ __forceinline__ void fft_lines(cx<T> (&v)[NC][E], cx<T>* lds, Addr addr, int t,
                                          const cx<T>* __restrict__ tw) {
  static_assert(L % E == 0 && L <= MAX_FFT_LEN && (TWL == kTwStaged || TWL % L == 0),
                "bad FFT length");
  fft_stages_multi<T, L, E, INV, NC, ZIN, TWL>(
      v, lds, addr, t, tw, std::make_integer_sequence<int, num_stages<L, E>()>{});
}

// The stage-major twiddle table of length L and register width E (tw_stage_off above), copied
// from the global table into LDS by the NT threads of a block in two steps: load() issues the
// global reads into registers (call it before the block's other global reads, so that waiting
// for these leaves those in flight), store() writes them to LDS; a barrier must follow before
// the table is read.  The LDS table needs tw_staged_size<L, E>() < L entries (FIRST: the
// first-twiddle table, tw_first_size<L, E>() entries).
template <typename T, int L, int E, int NT, bool FIRST = false>
struct TwStage {
  static constexpr int N = FIRST ? tw_first_size<L, E>() : tw_staged_size<L, E>();
  static constexpr int K = N > 0 ? (N + NT - 1) / NT : 0;
  cx<T> r[K > 0 ? K : 1];
  __device__ __forceinline__ void load(const cx<T>* __restrict__ tw, int tid) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int k = tid + i * NT;
      const int e = FIRST ? tw_first_exp<L, E>(k) : tw_staged_exp<L, E>(k);
      r[i] = k < N ? tw[e * (TW_N / L)] : cx<T>{0, 0};
    }
  }
  __device__ __forceinline__ void store(cx<T>* tab, int tid) const {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int k = tid + i * NT;
      if (k < N) tab[k] = r[i];
    }
  }
};

}  // namespace ie
