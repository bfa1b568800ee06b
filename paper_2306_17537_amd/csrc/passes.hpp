// Kernels of the FFT-accelerated operator (eq. 10 with 2x zero padding), five passes:
//
//   zfwd : per-cell 3x3 contrast J = M x (eq. 3 integrand) on the source planes, zero-pad to
//          LZ, FFT along z of all three components of a column       -> U1[3][LZ][ny][nx]
//   yfwd : FFT along y of the ny non-zero rows, padded to LY          -> U2[3][LZ][LY][nx]
//   xconv: per (ky, kz) row, FFT along x of the nx non-zero cells padded to LX,
//          S^_p = sum_q G^_pq J^_q with the six stored components of G^ (G_pq = G_qp, each even
//          or odd per axis, so one octant kx <= LX/2, ky <= LY/2, kz <= LZ/2 is stored and the
//          row pair ky, LY - ky of one block share each value fetched), inverse FFT along x,
//          keep nx cells                                                -> U2 (in place)
//   yinv : inverse FFT along y, keep ny rows                             -> U1
//   zinv : inverse FFT along z, keep the output planes, combine
//          y = a_e e + a_x x - a_m (M x) + a_s S                          -> y
//
// The strided axes (z, y) are transformed by column passes that read and write whole 128-byte
// row segments; the spectrum multiply sits in the pass along the contiguous axis, whose rows
// and whose stored spectrum rows are read as whole contiguous lines.
// 1 / (LX LY LZ) is folded into the stored G^.  Every kernel returns at once when the
// problem's `active` flag is 0 (used to retire converged Krylov iterations without a host
// round trip).  blockIdx.z indexes a batch of problems of the same shape; per-problem arrays
// advance by their batch stride.
#pragma once

#include <type_traits>

#include "common.hpp"
#include "fft.hpp"

namespace ie {

// Load of a pass input that the previous pass wrote and nothing reads again (the column-pass
// inputs, the z inverse's input, the x pass's rows), with the non-temporal hint: these arrays
// are several times the last-level cache, and keeping them out of it lets the contrast tensor
// and the operator's input x, which the first and the last pass both read, survive in between
// (measured: float64 GMRES(10) solve of the 128x128x256 model 1.6 % faster, mixed GMRES(16)
// 2.5 %).  The stored spectrum is read with plain loads: the blocks of kz and LZ - kz share it
// through the L2 (with the hint the float64 solve took 0.8 % longer).
template <typename T>
__device__ __forceinline__ cx<T> load_stream(const cx<T>* p) {
  typedef T V2 __attribute__((ext_vector_type(2)));
  const V2 r = __builtin_nontemporal_load(reinterpret_cast<const V2*>(p));
  return cx<T>{r.x, r.y};
}

// Store of one pass output value, one vector store with the non-temporal hint: the outputs are
// read by the next pass only (complex64: measured 5-15 % faster per pass on the 64^3 grid;
// complex128, together with the non-temporal input loads: the float64 GMRES(10) solve of the
// 128x128x256 model 1.2 % faster, where the hint alone had made the float64 z pass slower).
template <typename T>
__device__ __forceinline__ void store_stream(cx<T>* p, cx<T> v) {
  typedef T V2 __attribute__((ext_vector_type(2)));
  V2 x;
  x.x = v.re;
  x.y = v.im;
  __builtin_nontemporal_store(x, reinterpret_cast<V2*>(p));
}


template <typename T>
struct MvArgs {
  int nx, ny, nz;
  int LX, LY, LZ;
  // source: x view and contrast tensor M (6 comps xx,yy,zz,xy,xz,yz; nullptr = identity)
  const cx<T>* x;
  long x_cs, x_bs;
  int x_zoff;
  const double* xscale;  // optional per-problem factor applied to x on load (batch stride xscale_bs)
  long xscale_bs;
  const T* M;
  long M_cs, M_bs;
  int M_zoff;
  int src_z0, src_z1;    // source planes outside [src_z0, src_z1) are zero
  int hole_z0, hole_z1;  // and so are planes inside [hole_z0, hole_z1)
  // work: T1 = U1[3][LZ][ny][nx], T2 = U2[3][LZ][LY][nx]
  cx<T>* T1;
  cx<T>* T2;
  long T1_bs, T2_bs;
  const cx<T>* ghat;  // [6][LZ/2+1][LY/2+1][LX/2+1], scaled by 1/(LX LY LZ)
  long ghat_bs;
  // output planes and combination
  int out_z0, out_z1;
  cx<T>* y;
  long y_cs, y_bs;
  int y_zoff;
  const cx<T>* e;
  long e_cs, e_bs;
  int e_zoff;
  T a_e, a_x, a_m, a_s;
  const int* active;
  int active_bs;
  const cx<T>* tw;
};

template <typename T>
__device__ __forceinline__ bool retired(const MvArgs<T>& a, int b) {
  return a.active != nullptr && a.active[b * a.active_bs] == 0;
}

// ---------------------------------------------------------------------------------------
// launch geometry per (precision, length, variant)
// Variant V (chosen per plan by the autotuner): bit 0 halves the values per thread of the y
// column passes (twice the threads per line, more waves in flight, one more LDS exchange) and
// doubles those of the row pass (8 instead of 4: half the threads per line, one LDS exchange
// fewer); bit 1 doubles the columns per block of the y column passes (256-byte row segments).
// The row pass (x) has four more: V + 4 uses the LDS layout padded every 4 positions.
// ---------------------------------------------------------------------------------------
// Register width of a length-L transform: for L = 3 * 2^k it is 12 (L itself when shorter), so
// that one stage takes the factor 3 and the others radix 4 or 2; e2 otherwise.
constexpr int reg_width(int L, int e2) {
  return L % 3 == 0 ? (L < 12 ? L : 12) : (L < e2 ? L : e2);
}

constexpr int kVariants = 4;   // y passes
constexpr int kZVariants = 2;  // z passes
constexpr int kRowVariants = 8;

template <typename T, int L, int V = 0>
struct Geo {
  // column passes (y, z): E values per thread per line, W adjacent columns per block so that a
  // row segment is one (V & 2: two) 128-byte line(s); at least 64 threads per block; LDS <= 64 KB
  static constexpr int Edef = sizeof(T) == 8 ? 8 : 16;
  static constexpr int E1 = L < Edef ? L : Edef;
  static constexpr int E = L % 3 == 0 ? reg_width(L, 0) : (((V & 1) && E1 >= 4) ? E1 / 2 : E1);
  static constexpr int TL = L / E;
  static constexpr int Wc = (128 / int(sizeof(cx<T>))) * ((V & 2) ? 2 : 1);
  static constexpr int Wm = (64 / TL) > Wc ? (64 / TL) : Wc;
  static constexpr int Wl = (65536 / int(L * sizeof(cx<T>))) < 1 ? 1 : (65536 / int(L * sizeof(cx<T>)));
  static constexpr int W = Wm < Wl ? Wm : Wl;
  // row passes (x): ER values per thread, TLR threads per line, NL rows per block (~128 threads,
  // V & 2: ~256)
  static constexpr int ER1 = L < 4 ? L : 4;
  static constexpr int ER = L % 3 == 0 ? reg_width(L, 0) : (((V & 1) && L >= 16) ? 2 * ER1 : ER1);
  static constexpr int TLR = L / ER;
  static constexpr int NL0 = ((V & 2) ? 256 : 128) / TLR;
  static constexpr int NL = NL0 < 1 ? 1 : NL0;
  // row-pass LDS layout: one pad slot every 16 positions
  static constexpr int LP = LdsPadded::padded_len(L);
};

// 3x3 symmetric tensor (6 comps) times a complex 3-vector
template <typename T>
__device__ __forceinline__ void tensor_apply(const T m[6], const cx<T> v[3], cx<T> out[3]) {
  out[0] = cx<T>{m[0] * v[0].re + m[3] * v[1].re + m[4] * v[2].re,
                 m[0] * v[0].im + m[3] * v[1].im + m[4] * v[2].im};
  out[1] = cx<T>{m[3] * v[0].re + m[1] * v[1].re + m[5] * v[2].re,
                 m[3] * v[0].im + m[1] * v[1].im + m[5] * v[2].im};
  out[2] = cx<T>{m[4] * v[0].re + m[5] * v[1].re + m[2] * v[2].re,
                 m[4] * v[0].im + m[5] * v[1].im + m[2] * v[2].im};
}

// ---------------------------------------------------------------------------------------
// Column FFT along a strided axis.  Plane q of nplanes: comp c = q / nzp, index zq = z0 + q % nzp;
// in element (row r, col x) of plane q at in[c*in_cs + zq*in_zs + r*in_ls + x]; rows >= rows_in
// are zero on input; rows < rows_out are written.  Block: W columns x TL threads.  HALF: the
// convolution's half-size lines (forward: rows_in <= L/2, the transform skips the zero upper
// half; inverse: rows_out <= L/2, only the lower half is computed); the twiddles of the length
// are then staged in LDS.
// ---------------------------------------------------------------------------------------
struct ColArgs {
  int ncols, nzp, z0;
  long in_cs, in_zs, in_ls, out_cs, out_zs, out_ls;
  int rows_in, rows_out;
  long in_bs, out_bs;
  const int* active;
  int active_bs;
};

template <typename T, int L, bool INV, int V, bool HALF>
__global__ void __launch_bounds__((Geo<T, L, V>::W * Geo<T, L, V>::TL))
    k_colfft(const cx<T>* in, cx<T>* out, const ColArgs a,
             const cx<T>* __restrict__ tw) {
  using G = Geo<T, L, V>;
  constexpr int E = G::E, TL = G::TL, W = G::W;
  constexpr int ME = HALF ? E / 2 : E;  // registers read (forward) or written (inverse)
  __shared__ cx<T> lds[W * L];
  __shared__ cx<T> twl[HALF ? L : 1];
  const int b = blockIdx.z;
  if (a.active != nullptr && a.active[b * a.active_bs] == 0) return;
  TwStage<T, HALF ? L : 2, HALF ? E : 2, W * TL> tws;
  if constexpr (HALF) tws.load(tw, threadIdx.x);
  const int w = threadIdx.x % W;
  const int t = threadIdx.x / W;
  const int col = blockIdx.x * W + w;
  const bool live = col < a.ncols;
  const int q = blockIdx.y;
  const int c = q / a.nzp;
  const long zq = a.z0 + q % a.nzp;
  const cx<T>* src = in + b * a.in_bs + c * a.in_cs + zq * a.in_zs + col;
  cx<T>* dst = out + b * a.out_bs + c * a.out_cs + zq * a.out_zs + col;
  cx<T> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int r = t + m * TL;
    v[m] = ((INV || m < ME) && live && r < a.rows_in) ? load_stream(&src[r * a.in_ls]) : cx<T>{0, 0};
  }
  if constexpr (HALF) {
    tws.store(twl, threadIdx.x);
    __syncthreads();
    fft_line<T, L, E, INV, !INV, kTwStaged>(v, lds, LdsInterleaved{W, w}, t, twl);
  } else {
    fft_line<T, L, E, INV>(v, lds, LdsInterleaved{W, w}, t, tw);
  }
  if (live) {
#pragma unroll
    for (int m = 0; m < (INV ? ME : E); ++m) {
      const int r = t + m * TL;
      if (r < a.rows_out) store_stream(&dst[r * a.out_ls], v[m]);
    }
  }
}

// ---------------------------------------------------------------------------------------
// z column passes: all three components of W adjacent columns (y, x) of the xy plane, so that
// the per-cell tensors apply on load (zfwd) and on store (zinv).  Variants: V & 1 doubles the
// values per thread (4 -> 8 complex128, 8 -> 16 complex64).  The three lines go through the FFT
// stages in lockstep (twiddles read once per stage) and through LDS one after the other.
// ---------------------------------------------------------------------------------------
template <typename T, int L, int V = 0>
struct GeoC {
  static constexpr int Esm = sizeof(T) == 8 ? 4 : 8;
  static constexpr int E1 = (V & 1) ? 2 * Esm : Esm;
  static constexpr int E = reg_width(L, E1);
  static constexpr int TL = L / E;
  static constexpr int Wc = 128 / int(sizeof(cx<T>));
  static constexpr int Wm = (64 / TL) > Wc ? (64 / TL) : Wc;
  static constexpr int Wl = (65536 / int(L * sizeof(cx<T>))) < 1 ? 1 : (65536 / int(L * sizeof(cx<T>)));
  static constexpr int Wt = (1024 / TL) < 1 ? 1 : (1024 / TL);
  static constexpr int W1 = Wm < Wl ? Wm : Wl;
  static constexpr int W = W1 < Wt ? W1 : Wt;
  static constexpr int THREADS = W * TL;
};

// Column block of a z pass for launch slot p of nb: the blocks that read the two halves of one
// 128-byte line of the real per-cell tensor (W columns of 8-byte doubles, or of 4-byte floats
// for complex64, are 64 bytes) get slots 8 apart, so they run on the same XCD (blocks are dealt
// to the eight XCDs in turn) and its L2 fetches the line once.  A partial last group of 16
// keeps its order.
__device__ __forceinline__ long zcol_block(long p, long nb) {
  const long g = p / 16, w = p % 16;
  if ((g + 1) * 16 > nb) return p;
  return g * 16 + (w % 8) * 2 + w / 8;
}

template <typename T>
__device__ __forceinline__ bool source_plane(const MvArgs<T>& a, int z) {
  return z < a.nz && z >= a.src_z0 && z < a.src_z1 && !(z >= a.hole_z0 && z < a.hole_z1);
}

// zfwd: J = M x on the source planes (zero elsewhere), zero-padded to LZ, FFT along z.
template <typename T, int LZ, int V>
__global__ void __launch_bounds__((GeoC<T, LZ, V>::THREADS)) k_zfwd(const MvArgs<T> a) {
  using G = GeoC<T, LZ, V>;
  constexpr int E = G::E, TL = G::TL, W = G::W;
  __shared__ cx<T> lds[W * LZ];
  __shared__ cx<T> twl[LZ];
  const int b = blockIdx.z;
  if (retired(a, b)) return;
  TwStage<T, LZ, E, G::THREADS> tws;
  tws.load(a.tw, threadIdx.x);
  const int w = threadIdx.x % W;
  const int t = threadIdx.x / W;
  const long plane = long(a.ny) * a.nx;
  const long col = zcol_block(blockIdx.x, gridDim.x) * W + w;
  const bool live = col < plane;
  const cx<T>* x = a.x + b * a.x_bs + col;
  const T* M = a.M ? a.M + b * a.M_bs + col : nullptr;
  const T xs = a.xscale ? T(a.xscale[b * a.xscale_bs]) : T(1);
  cx<T> v[3][E];
  // the nz <= LZ/2 planes sit in the lower half of the line
#pragma unroll
  for (int m = E / 2; m < E; ++m)
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c][m] = cx<T>{0, 0};
#pragma unroll
  for (int m = 0; m < E / 2; ++m) {
    const int z = t + m * TL;
    cx<T> xv[3] = {{0, 0}, {0, 0}, {0, 0}};
    const bool on = live && source_plane(a, z);
    if (on) {
#pragma unroll
      for (int c = 0; c < 3; ++c) xv[c] = xs * x[c * a.x_cs + long(z - a.x_zoff) * plane];
    }
    if (M != nullptr && on) {
      T mm[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) mm[q] = M[q * a.M_cs + long(z - a.M_zoff) * plane];
      cx<T> j3[3];
      tensor_apply(mm, xv, j3);
#pragma unroll
      for (int c = 0; c < 3; ++c) v[c][m] = j3[c];
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) v[c][m] = xv[c];
    }
  }
  tws.store(twl, threadIdx.x);
  __syncthreads();
  fft_lines<T, LZ, E, false, 3, true, kTwStaged>(v, lds, LdsInterleaved{W, w}, t, twl);
  if (live) {
    cx<T>* out = a.T1 + b * a.T1_bs + col;
    const long cs = long(LZ) * plane;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int m = 0; m < E; ++m) store_stream(&out[c * cs + long(t + m * TL) * plane], v[c][m]);
  }
}

// zinv: inverse FFT along z, keep the output planes [out_z0, out_z1), combine
// y = a_e e + a_x x - a_m (M x) + a_s S.
template <typename T, int LZ, int V>
__global__ void __launch_bounds__((GeoC<T, LZ, V>::THREADS)) k_zinv(const MvArgs<T> a) {
  using G = GeoC<T, LZ, V>;
  constexpr int E = G::E, TL = G::TL, W = G::W;
  __shared__ cx<T> lds[W * LZ];
  __shared__ cx<T> twl[LZ];
  const int b = blockIdx.z;
  if (retired(a, b)) return;
  TwStage<T, LZ, E, G::THREADS> tws;
  tws.load(a.tw, threadIdx.x);
  const int w = threadIdx.x % W;
  const int t = threadIdx.x / W;
  const long plane = long(a.ny) * a.nx;
  const long col = zcol_block(blockIdx.x, gridDim.x) * W + w;
  const bool live = col < plane;
  const cx<T>* in = a.T1 + b * a.T1_bs + (live ? col : 0);
  const long cs = long(LZ) * plane;
  cx<T> v[3][E];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int m = 0; m < E; ++m)
      v[c][m] = live ? load_stream(&in[c * cs + long(t + m * TL) * plane]) : cx<T>{0, 0};
  tws.store(twl, threadIdx.x);
  __syncthreads();
  fft_lines<T, LZ, E, true, 3, false, kTwStaged>(v, lds, LdsInterleaved{W, w}, t, twl);
  if (!live) return;
  cx<T>* y = a.y + b * a.y_bs + col;
  const cx<T>* x = a.x ? a.x + b * a.x_bs + col : nullptr;
  const cx<T>* e = a.e ? a.e + b * a.e_bs + col : nullptr;
  const T* M = (a.M && a.a_m != T(0)) ? a.M + b * a.M_bs + col : nullptr;
  const T xs = a.xscale ? T(a.xscale[b * a.xscale_bs]) : T(1);
  // the output planes (< nz <= LZ/2) sit in the lower half of the line
#pragma unroll
  for (int m = 0; m < E / 2; ++m) {
    const int z = t + m * TL;
    if (z < a.out_z0 || z >= a.out_z1) continue;
    cx<T> r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = a.a_s * v[c][m];
    if (x != nullptr && (a.a_x != T(0) || M != nullptr)) {
      cx<T> xv[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) xv[c] = xs * x[c * a.x_cs + long(z - a.x_zoff) * plane];
#pragma unroll
      for (int c = 0; c < 3; ++c) r[c] = r[c] + a.a_x * xv[c];
      if (M != nullptr) {
        T mm[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) mm[q] = M[q * a.M_cs + long(z - a.M_zoff) * plane];
        cx<T> mx[3];
        tensor_apply(mm, xv, mx);
#pragma unroll
        for (int c = 0; c < 3; ++c) r[c] = r[c] - a.a_m * mx[c];
      }
    }
    if (e != nullptr) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        r[c] = r[c] + a.a_e * e[c * a.e_cs + long(z - a.e_zoff) * plane];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) store_stream(&y[c * a.y_cs + long(z - a.y_zoff) * plane], r[c]);
  }
}

// ---------------------------------------------------------------------------------------
// xconv: per block the row pair (ky, LY - ky) of one kz (one row when ky is 0 or LY/2), each
// row with its three components: FFT along x (nx cells zero-padded to LX), tensor multiply with
// G^, inverse FFT, keep nx cells, in place in U2.  Both rows read the same stored spectrum row
// (the second fetch is served by the CU's cache); kz runs in the order 0, LZ/2, 1, LZ-1, 2,
// LZ-2, ... along blockIdx.y, and the grid's x extent is a multiple of 8, so the blocks of kz
// and LZ - kz that read the same stored row run next to each other on the same XCD (blocks are
// dealt to the eight XCDs in turn).  Thread layout and variants as the row geometry Geo, except
// that V & 2 puts two row pairs (consecutive stored rows) in a block.
// ---------------------------------------------------------------------------------------
template <typename T, int LX, int V>
struct GeoX {  // x pass: NP row pairs per block (V & 2: two; at least a wavefront), row geometry of Geo
  static constexpr int NP0 = (V & 2) ? 2 : 1;
  static constexpr int NPW = 32 / Geo<T, LX, V>::TLR;
  static constexpr int NP = NP0 > NPW ? NP0 : NPW;
  static constexpr int THREADS = 2 * NP * Geo<T, LX, V>::TLR;
};

template <typename T, int LX, int V>
__global__ void __launch_bounds__((GeoX<T, LX, V>::THREADS)) k_xconv(const MvArgs<T> a) {
  using G = Geo<T, LX, V>;
  constexpr int E = G::ER, TL = G::TLR, NP = GeoX<T, LX, V>::NP;
  __shared__ cx<T> lds[2 * NP * G::LP];
  const int b = blockIdx.z;
  if (retired(a, b)) return;
  const int hx = LX / 2, hy = a.LY / 2, hz = a.LZ / 2;
  const int t = threadIdx.x % TL;
  const int rr = threadIdx.x / TL;  // row of the block: pair rr / 2, member rr % 2
  const int r = rr & 1;             // 0: row ky = oy, 1: its mirror LY - oy
  const int oy = blockIdx.x * NP + (rr >> 1);  // stored y row; rows beyond LY/2 pad the grid
  const bool two = oy != 0 && oy != hy;
  const bool live = oy <= hy && (r == 0 || two);
  const int ky = r == 0 ? oy : a.LY - oy;
  const int bz = blockIdx.y;
  const int kz = bz < 2 ? bz * hz : ((bz & 1) ? a.LZ - (bz >> 1) : (bz >> 1));
  const int oz = kz > hz ? a.LZ - kz : kz;
  const T sy = r == 0 ? T(1) : T(-1);
  const T sz = kz > hz ? T(-1) : T(1);
  const long rs = long(a.LY) * a.nx;  // per kz
  const long cs = long(a.LZ) * rs;    // per component
  cx<T>* row = a.T2 + b * a.T2_bs + long(kz) * rs + long(ky) * a.nx;
  cx<T> v[3][E];
  // the nx <= LX/2 cells sit in the lower half of the line
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int i = t + m * TL;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      v[c][m] = (m < E / 2 && live && i < a.nx) ? row[c * cs + i] : cx<T>{0, 0};
  }
  const LdsPadded addr{rr * G::LP};
  // the three lines in lockstep: each stage's twiddles are read once (from the global table: a
  // copy in LDS measured slower here, the block being one or two wavefronts)
  fft_lines<T, LX, E, false, 3, true>(v, lds, addr, t, a.tw);
  const long gys = hx + 1;
  const long gzs = long(hy + 1) * gys;
  const long gcs = long(hz + 1) * gzs;
  const cx<T>* gh = a.ghat + b * a.ghat_bs + long(oz) * gzs + long(live ? oy : 0) * gys;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int kx = t + m * TL;
    const int ox = kx > hx ? LX - kx : kx;
    const T sx = kx > hx ? T(-1) : T(1);
    const cx<T>* g = gh + ox;
    const cx<T> gxx = g[0], gyy = g[gcs], gzz = g[2 * gcs];
    const cx<T> gxy = (sx * sy) * g[3 * gcs];
    const cx<T> gxz = (sx * sz) * g[4 * gcs];
    const cx<T> gyz = (sy * sz) * g[5 * gcs];
    const cx<T> j0 = v[0][m], j1 = v[1][m], j2 = v[2][m];
    v[0][m] = gxx * j0 + gxy * j1 + gxz * j2;
    v[1][m] = gxy * j0 + gyy * j1 + gyz * j2;
    v[2][m] = gxz * j0 + gyz * j1 + gzz * j2;
  }
  fft_lines<T, LX, E, true, 3>(v, lds, addr, t, a.tw);
  if (live) {
#pragma unroll
    for (int m = 0; m < E / 2; ++m) {
      const int i = t + m * TL;
      if (i < a.nx) {
#pragma unroll
        for (int c = 0; c < 3; ++c) store_stream(&row[c * cs + i], v[c][m]);
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// xconv, one line per thread group: the same operation as k_xconv with each of the six lines of
// a row pair (two rows x three components) transformed by its own TL threads, so that a thread
// holds one line (E values) instead of three and more waves fit on a CU.  The spectra meet in
// LDS for the tensor multiply, which the whole block does with one work item per (row pair,
// kx): the six stored spectrum components are loaded once for both rows of the pair.  The
// forward transforms skip the zero upper half of the padded lines, the inverse ones compute
// only the kept lower half.  V: 0 eight values per thread, 1 sixteen, 2 sixteen with two row
// pairs per block, each reading the spectrum values when it multiplies; 3 as 2 with the spectrum
// values fetched before the forward transforms, so that their latency overlaps that of the
// lines (more registers).  Used where the block's LDS (six padded lines per pair and the
// twiddles) fits in the 160 KB of a CU.
// ---------------------------------------------------------------------------------------
template <typename T, int LX, int V>
struct GeoX2 {
  static constexpr int E0 = V == 0 ? 8 : 16;
  static constexpr int E = LX % 3 == 0 ? reg_width(LX, 0) : (LX < E0 ? LX : E0);
  static constexpr int TL = LX / E;
  static constexpr bool PRE = V == 3;  // spectrum values fetched before the forward transforms
  static constexpr int NP0 = V >= 2 ? 2 : 1;
  static constexpr int NPW = (64 + 6 * TL - 1) / (6 * TL);  // at least one wavefront
  static constexpr int NP1 = NP0 > NPW ? NP0 : NPW;
  static constexpr int NPM = 1024 / (6 * TL) < 1 ? 1 : 1024 / (6 * TL);
  static constexpr int NP = NP1 < NPM ? NP1 : NPM;
  static constexpr int THREADS = 6 * NP * TL;
  // float64 lines: swizzled (measured bank conflicts 2.7e7 cycles per launch at LX = 256,
  // against 6.6e7 padded); float32 lines: padded
  using Lds = typename std::conditional<sizeof(T) == 8, LdsSwz, LdsPadded>::type;
  static constexpr int LP = Lds::padded_len(LX);
  // float64: the first-twiddle table (72 entries at LX = 256 instead of 248), so that six
  // one-row-pair blocks fit a CU's LDS instead of five; float32 keeps the stage-major table
  // (its x pass is bound by vector issue, and powers of a float32 twiddle lose accuracy)
  static constexpr bool TFIRST = sizeof(T) == 8;
  static constexpr int TWN = TFIRST ? tw_first_size<LX, E>() : LX;
  static constexpr int TWL = TFIRST ? kTwFirst : kTwStaged;
  static constexpr bool FITS = (6 * NP * LP + TWN) * int(sizeof(cx<T>)) <= 160 * 1024 &&
                               THREADS <= 1024;
  static constexpr int ITEMS = (NP * LX + THREADS - 1) / THREADS;  // multiply items per thread
};

template <typename T, int LX, int V>
__global__ void __launch_bounds__((GeoX2<T, LX, V>::THREADS)) k_xconv2(const MvArgs<T> a) {
  using G = GeoX2<T, LX, V>;
  constexpr int E = G::E, TL = G::TL, NP = G::NP;
  __shared__ cx<T> lds[6 * NP * G::LP];
  __shared__ cx<T> twl[G::TWN > 0 ? G::TWN : 1];
  const int b = blockIdx.z;
  if (retired(a, b)) return;
  // the global reads of the block are issued up front (twiddles, the lines and, with PRE, the
  // spectrum values of the multiply), so that their latencies overlap
  TwStage<T, LX, E, G::THREADS, G::TFIRST> tws;
  tws.load(a.tw, threadIdx.x);
  const int hx = LX / 2, hy = a.LY / 2, hz = a.LZ / 2;
  const int t = threadIdx.x % TL;
  const int line = threadIdx.x / TL;  // pair line / 6, row (line / 3) % 2, component line % 3
  const int pr = line / 6, r = (line / 3) & 1, c = line % 3;
  const int oy = blockIdx.x * NP + pr;  // stored y row; rows beyond LY/2 pad the grid
  const bool live = oy <= hy && (r == 0 || (oy != 0 && oy != hy));
  const int ky = r == 0 ? oy : a.LY - oy;
  const int bz = blockIdx.y;
  const int kz = bz < 2 ? bz * hz : ((bz & 1) ? a.LZ - (bz >> 1) : (bz >> 1));
  const int oz = kz > hz ? a.LZ - kz : kz;
  const T sz = kz > hz ? T(-1) : T(1);
  const long rs = long(a.LY) * a.nx;  // per kz
  const long cs = long(a.LZ) * rs;    // per component
  cx<T>* row = a.T2 + b * a.T2_bs + long(c) * cs + long(kz) * rs + long(live ? ky : 0) * a.nx;
  const typename G::Lds addr{line * G::LP};
  cx<T> v[E];
  // the nx <= LX/2 cells sit in the lower half of the line
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int i = t + m * TL;
    v[m] = (m < E / 2 && live && i < a.nx) ? load_stream(&row[i]) : cx<T>{0, 0};
  }
  // spectrum values of the multiply items (pair, kx) of this thread
  const long gys = hx + 1;
  const long gzs = long(hy + 1) * gys;
  const long gcs = long(hz + 1) * gzs;
  const cx<T>* gz0 = a.ghat + b * a.ghat_bs + long(oz) * gzs;
  auto fetch = [&](int q, cx<T>(&g6)[6]) {
    const int it = threadIdx.x + q * G::THREADS;
    const int p = it / LX, kx = it % LX;
    const int py = blockIdx.x * NP + p;
    const bool ok = p < NP && py <= hy;
    const int ox = kx > hx ? LX - kx : kx;
    const cx<T>* g = gz0 + long(ok ? py : 0) * gys + ox;
#pragma unroll
    for (int k = 0; k < 6; ++k) g6[k] = ok ? g[k * gcs] : cx<T>{0, 0};
  };
  cx<T> gv[G::PRE ? G::ITEMS : 1][6];
  if constexpr (G::PRE) {
#pragma unroll
    for (int q = 0; q < G::ITEMS; ++q) fetch(q, gv[q]);
  }
  tws.store(twl, threadIdx.x);
  __syncthreads();  // the twiddle table
  fft_line<T, LX, E, false, true, G::TWL>(v, lds, addr, t, twl);
  // the last stage ran in registers after every thread's last LDS read of this line
#pragma unroll
  for (int m = 0; m < E; ++m) lds[addr(t + m * TL)] = v[m];
  __syncthreads();
  // tensor multiply: item (pair, kx), both rows of the pair
#pragma unroll
  for (int q = 0; q < G::ITEMS; ++q) {
    const int it = threadIdx.x + q * G::THREADS;
    const int p = it / LX, kx = it % LX;
    const int py = blockIdx.x * NP + p;
    if (p < NP && py <= hy) {
      const T sx = kx > hx ? T(-1) : T(1);
      cx<T> g6[6];
      if constexpr (G::PRE) {
#pragma unroll
        for (int k = 0; k < 6; ++k) g6[k] = gv[q][k];
      } else {
        fetch(q, g6);
      }
      const cx<T> gxx = g6[0], gyy = g6[1], gzz = g6[2];
      const cx<T> gxy = sx * g6[3];
      const cx<T> gxz = (sx * sz) * g6[4];
      const cx<T> gyz = sz * g6[5];
      const int nr = (py != 0 && py != hy) ? 2 : 1;
#pragma unroll
      for (int rr = 0; rr < 2; ++rr) {
        if (rr < nr) {
          const T sy = rr == 0 ? T(1) : T(-1);
          const int base = (p * 6 + rr * 3) * G::LP;
          const int i0 = typename G::Lds{base}(kx), i1 = typename G::Lds{base + G::LP}(kx),
                    i2 = typename G::Lds{base + 2 * G::LP}(kx);
          const cx<T> j0 = lds[i0], j1 = lds[i1], j2 = lds[i2];
          const cx<T> gxys = sy * gxy, gyzs = sy * gyz;
          lds[i0] = gxx * j0 + gxys * j1 + gxz * j2;
          lds[i1] = gxys * j0 + gyy * j1 + gyzs * j2;
          lds[i2] = gxz * j0 + gyzs * j1 + gzz * j2;
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = lds[addr(t + m * TL)];
  __syncthreads();  // every read of the line done before its first inverse stage writes
  fft_line<T, LX, E, true, false, G::TWL>(v, lds, addr, t, twl);
  if (live) {
#pragma unroll
    for (int m = 0; m < E / 2; ++m) {
      const int i = t + m * TL;
      if (i < a.nx) store_stream(&row[i], v[m]);
    }
  }
}

}  // namespace ie
