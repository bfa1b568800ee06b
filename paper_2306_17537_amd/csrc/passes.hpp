// Kernels of the FFT-accelerated operator (eq. 10 with 2x zero padding), five passes:
//
//   xfwd : per-cell 3x3 contrast J = M x (eq. 3 integrand), zero-pad to LX, FFT along x
//          -> T1[3][nz][ny][LX]
//   yfwd : FFT along y of the ny non-zero rows, padded to LY          -> T2[3][nz][LY][LX]
//   zconv: per (kx, ky) column, FFT along z of the nz non-zero planes, S^_p = sum_q G^_pq J^_q
//          with the six stored components of G^ (G_pq = G_qp, each even or odd per axis; the
//          half kept for ky <= LY/2, kz <= LZ/2 serves the row pair ky, LY - ky of one block),
//          inverse FFT along z, keep the output planes                  -> T2 (in place)
//   yinv : inverse FFT along y, keep ny rows                             -> T1
//   xinv : inverse FFT along x, keep nx cells, combine
//          y = a_e e + a_x x - a_m (M x) + a_s S                          -> y
//
// 1 / (LX LY LZ) is folded into the stored G^.  Every kernel returns at once when the
// problem's `active` flag is 0 (used to retire converged Krylov iterations without a host
// round trip).  blockIdx.z indexes a batch of problems of the same shape; per-problem arrays
// advance by their batch stride.
#pragma once

#include <type_traits>

#include "common.hpp"
#include "fft.hpp"

namespace ie {

// Store of one pass output value.  complex64 outputs use one 8-byte store with the non-temporal
// hint (they are read by the next pass only; measured 5-15 % faster per pass on the 64^3 grid);
// complex128 outputs use a plain store (the hint made the float64 z pass slower).
template <typename T>
__device__ __forceinline__ void store_stream(cx<T>* p, cx<T> v) {
  if constexpr (sizeof(T) == 4) {
    typedef T V2 __attribute__((ext_vector_type(2)));
    V2 x;
    x.x = v.re;
    x.y = v.im;
    __builtin_nontemporal_store(x, reinterpret_cast<V2*>(p));
  } else {
    *p = v;
  }
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
  // work
  cx<T>* T1;
  cx<T>* T2;
  long T1_bs, T2_bs;
  const cx<T>* ghat;  // [6][LZ/2+1][LY/2+1][LX], scaled by 1/(LX LY LZ)
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
// Variant V (chosen per plan by the autotuner): bit 0 halves the values per thread of the column
// passes (twice the threads per line, more waves in flight, one more LDS exchange) and doubles
// those of the row passes (8 instead of 4: half the threads per line, one LDS exchange fewer,
// 128-byte instead of 256-byte row segments per load); bit 1 doubles the columns per block of
// the column passes (256-byte row segments) and the rows per block of the row passes.  Row
// passes (x) have four more: V + 4 uses the LDS layout padded every 4 positions.
// ---------------------------------------------------------------------------------------
constexpr int kVariants = 4;
constexpr int kRowVariants = 8;

template <typename T, int L, int V = 0>
struct Geo {
  // column passes (y, z): E values per thread per line, W adjacent columns per block so that a
  // row segment is one (V & 2: two) 128-byte line(s); at least 64 threads per block; LDS <= 64 KB
  static constexpr int Edef = sizeof(T) == 8 ? 8 : 16;
  static constexpr int E1 = L < Edef ? L : Edef;
  static constexpr int E = ((V & 1) && E1 >= 4) ? E1 / 2 : E1;
  static constexpr int TL = L / E;
  static constexpr int Wc = (128 / int(sizeof(cx<T>))) * ((V & 2) ? 2 : 1);
  static constexpr int Wm = (64 / TL) > Wc ? (64 / TL) : Wc;
  static constexpr int Wl = (65536 / int(L * sizeof(cx<T>))) < 1 ? 1 : (65536 / int(L * sizeof(cx<T>)));
  static constexpr int W = Wm < Wl ? Wm : Wl;
  // row passes (x): ER values per thread, TLR threads per line, NL rows per block (~128 threads,
  // V & 2: ~256)
  static constexpr int ER1 = L < 4 ? L : 4;
  static constexpr int ER = ((V & 1) && L >= 16) ? 2 * ER1 : ER1;
  static constexpr int TLR = L / ER;
  static constexpr int NL0 = ((V & 2) ? 256 : 128) / TLR;
  static constexpr int NL = NL0 < 1 ? 1 : NL0;
  // row-pass LDS layout: V & 4 pads every 4 positions instead of every 16
  static constexpr bool PAD4 = (V & 4) != 0;
  static constexpr int LP = PAD4 ? LdsPadded4::padded_len(L) : LdsPadded::padded_len(L);
  using RowLds = typename std::conditional<PAD4, LdsPadded4, LdsPadded>::type;
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
// xfwd: contrast, pad, FFT along x.  Block: NL rows x TL threads; thread (row, t).
// ---------------------------------------------------------------------------------------
template <typename T, int LX, int V>
__global__ void __launch_bounds__((Geo<T, LX, V>::NL * Geo<T, LX, V>::TLR))
    k_xfwd(const MvArgs<T> a) {
  using G = Geo<T, LX, V>;
  constexpr int E = G::ER, TL = G::TLR, NL = G::NL;
  __shared__ cx<T> lds[NL * G::LP];
  const int b = blockIdx.z;
  if (retired(a, b)) return;
  const int t = threadIdx.x % TL;
  const int line = threadIdx.x / TL;
  const long row = long(blockIdx.x) * NL + line;  // (z, y) row
  const long nrows = long(a.nz) * a.ny;
  const bool live = row < nrows;
  const int z = live ? int(row / a.ny) : 0;
  const int yy = live ? int(row % a.ny) : 0;
  const bool zero = !live || z < a.src_z0 || z >= a.src_z1 || (z >= a.hole_z0 && z < a.hole_z1);
  const cx<T>* x = a.x + b * a.x_bs + (long(z - a.x_zoff) * a.ny + yy) * a.nx;
  const T* M = a.M ? a.M + b * a.M_bs + (long(z - a.M_zoff) * a.ny + yy) * a.nx : nullptr;
  const T xs = a.xscale ? T(a.xscale[b * a.xscale_bs]) : T(1);
  cx<T> v[3][E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int i = t + m * TL;
    cx<T> xv[3] = {{0, 0}, {0, 0}, {0, 0}};
    if (!zero && i < a.nx) {
#pragma unroll
      for (int c = 0; c < 3; ++c) xv[c] = xs * x[c * a.x_cs + i];
    }
    if (M != nullptr && !zero && i < a.nx) {
      T mm[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) mm[c] = M[c * a.M_cs + i];
      cx<T> j3[3];
      tensor_apply(mm, xv, j3);
#pragma unroll
      for (int c = 0; c < 3; ++c) v[c][m] = j3[c];
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) v[c][m] = xv[c];
    }
  }
  const typename G::RowLds addr{line * G::LP};
  cx<T>* out = a.T1 + b * a.T1_bs + (long(z) * a.ny + yy) * LX;
  const long cs = long(a.nz) * a.ny * LX;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    fft_line<T, LX, E, false>(v[c], lds, addr, t, a.tw);
    if (live) {
#pragma unroll
      for (int m = 0; m < E; ++m) store_stream(&out[c * cs + t + m * TL], v[c][m]);
    }
  }
}

// ---------------------------------------------------------------------------------------
// Column FFT along a strided axis.  Plane q of nplanes: comp c = q / nzp, index zq = z0 + q % nzp;
// in element (row r, col x) of plane q at in[c*in_cs + zq*in_zs + r*in_ls + x]; rows >= rows_in
// are zero on input; rows < rows_out are written.  Block: W columns x TL threads.
// ---------------------------------------------------------------------------------------
struct ColArgs {
  int ncols, nzp, z0;
  long in_cs, in_zs, in_ls, out_cs, out_zs, out_ls;
  int rows_in, rows_out;
  long in_bs, out_bs;
  const int* active;
  int active_bs;
};

template <typename T, int L, bool INV, int V>
__global__ void __launch_bounds__((Geo<T, L, V>::W * Geo<T, L, V>::TL))
    k_colfft(const cx<T>* in, cx<T>* out, const ColArgs a,
             const cx<T>* __restrict__ tw) {
  using G = Geo<T, L, V>;
  constexpr int E = G::E, TL = G::TL, W = G::W;
  __shared__ cx<T> lds[W * L];
  const int b = blockIdx.z;
  if (a.active != nullptr && a.active[b * a.active_bs] == 0) return;
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
    v[m] = (live && r < a.rows_in) ? src[r * a.in_ls] : cx<T>{0, 0};
  }
  fft_line<T, L, E, INV>(v, lds, LdsInterleaved{W, w}, t, tw);
  if (live) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int r = t + m * TL;
      if (r < a.rows_out) store_stream(&dst[r * a.out_ls], v[m]);
    }
  }
}

// ---------------------------------------------------------------------------------------
// zconv: FFT along z, tensor multiply with G^, inverse FFT along z (in place in T2).
// A block takes W kx-columns of one row ky, or (pair form) of the rows ky and LY - ky, so that
// both use each spectrum value fetched once.  G^ is stored for all kx, ky <= LY/2 and
// kz <= LZ/2 ([6][LZ/2+1][LY/2+1][LX]); mirrored ky and kz follow from the parity of each
// component (xy odd in y, xz odd in z, yz odd in y and z).
// ---------------------------------------------------------------------------------------
// Variants: V & 2 selects the row pair form (else one row per block).  Values per thread:
// V0 8 (complex64) / 4 (complex128), V1 twice that, V2 half of V0 (pair), V3 as V0 (pair).
// Columns per block fill a 128-byte row segment within 1024 (pair: 512) threads per block.
template <typename T, int L, int V = 0>
struct GeoZ {
  static constexpr bool PAIR = (V & 2) != 0;
  static constexpr int Esm = sizeof(T) == 8 ? 4 : 8;
  static constexpr int Edef = V == 1 ? 2 * Esm : (V == 2 ? Esm / 2 : Esm);
  static constexpr int E = L < Edef ? L : Edef;
  static constexpr int TL = L / E;
  static constexpr int Wc = 128 / int(sizeof(cx<T>));
  static constexpr int Wm = (64 / TL) > Wc ? (64 / TL) : Wc;
  static constexpr int Wl = (65536 / int(L * sizeof(cx<T>))) < 1 ? 1 : (65536 / int(L * sizeof(cx<T>)));
  static constexpr int Tmax = PAIR ? 512 : 1024;  // the pair form needs more registers
  static constexpr int Wt = (Tmax / TL) < 1 ? 1 : (Tmax / TL);
  static constexpr int W1 = Wm < Wl ? Wm : Wl;
  static constexpr int W = W1 < Wt ? W1 : Wt;
  static constexpr int ROWS = PAIR ? 2 : 1;
};

template <typename T, int LZ, int V>
__global__ void __launch_bounds__((GeoZ<T, LZ, V>::W * GeoZ<T, LZ, V>::TL))
    k_zconv(const MvArgs<T> a) {
  using G = GeoZ<T, LZ, V>;
  constexpr int E = G::E, TL = G::TL, W = G::W, R = G::ROWS;
  __shared__ cx<T> lds[W * LZ];
  const int b = blockIdx.z;
  if (retired(a, b)) return;
  const int w = threadIdx.x % W;
  const int t = threadIdx.x / W;
  const int kx = blockIdx.x * W + w;
  // pair form: rows ky and LY - ky (one row when ky is 0 or LY/2); single form: row ky, in the
  // launch order 0, LY/2, 1, LY-1, 2, LY-2, ... so that the two rows reading the same stored
  // spectrum row run at the same time (their blocks are LX/W apart in launch order) and the
  // second read finds the row in cache
  const int hy = a.LY / 2;
  const int by = blockIdx.y;
  const int ky = G::PAIR ? by : (by < 2 ? by * hy : ((by & 1) ? a.LY - (by >> 1) : (by >> 1)));
  const bool two = G::PAIR && ky != 0 && ky != hy;  // block-uniform
  const int nr = two ? 2 : 1;
  const int oy = ky > hy ? a.LY - ky : ky;            // stored row of G^
  const T sy0 = ky > hy ? T(-1) : T(1);                // parity of the first row
  const bool live = kx < a.LX;
  const long ls = long(a.LY) * a.LX;  // z stride
  const long cs = long(a.nz) * ls;
  cx<T>* row[R];
  row[0] = a.T2 + b * a.T2_bs + long(ky) * a.LX + kx;
  if constexpr (R == 2) row[1] = a.T2 + b * a.T2_bs + long(two ? a.LY - ky : ky) * a.LX + kx;
  cx<T> v[R][3][E];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int z = t + m * TL;
        v[r][c][m] = (r < nr && live && z < a.nz) ? row[r][c * cs + z * ls] : cx<T>{0, 0};
      }
  const LdsInterleaved addr{W, w};
  // all lines of the block in lockstep (twiddles loaded once per stage); a single row in the
  // pair form transforms zeros in place of its missing mirror row
  auto& lines = reinterpret_cast<cx<T>(&)[R * 3][E]>(v);
  fft_lines<T, LZ, E, false, R * 3>(lines, lds, addr, t, a.tw);
  const int hz = LZ / 2;
  const long gzs = long(hy + 1) * a.LX;  // per kz
  const long gcs = long(hz + 1) * gzs;   // per component
  const cx<T>* gh = a.ghat + b * a.ghat_bs + long(oy) * a.LX + (live ? kx : 0);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int kz = t + m * TL;
    const int oz = kz > hz ? LZ - kz : kz;
    const T sz = kz > hz ? T(-1) : T(1);
    const cx<T>* g = gh + oz * gzs;
    const cx<T> gxx = g[0], gyy = g[gcs], gzz = g[2 * gcs];
    const cx<T> gxy = g[3 * gcs];
    const cx<T> gxz = sz * g[4 * gcs];
    const cx<T> gyz = sz * g[5 * gcs];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T sy = r == 0 ? sy0 : T(-1);  // the mirrored row flips the y-odd components
      const cx<T> hxy = sy * gxy, hyz = sy * gyz;
      const cx<T> j0 = v[r][0][m], j1 = v[r][1][m], j2 = v[r][2][m];
      v[r][0][m] = gxx * j0 + hxy * j1 + gxz * j2;
      v[r][1][m] = hxy * j0 + gyy * j1 + hyz * j2;
      v[r][2][m] = gxz * j0 + hyz * j1 + gzz * j2;
    }
  }
  fft_lines<T, LZ, E, true, R * 3>(lines, lds, addr, t, a.tw);
  if (live) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r >= nr) break;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int m = 0; m < E; ++m) {
          const int z = t + m * TL;
          if (z >= a.out_z0 && z < a.out_z1) store_stream(&row[r][c * cs + z * ls], v[r][c][m]);
        }
    }
  }
}

// ---------------------------------------------------------------------------------------
// xinv: inverse FFT along x, crop, combine.  Rows (z, y) for z in [out_z0, out_z1).
// ---------------------------------------------------------------------------------------
template <typename T, int LX, int V>
__global__ void __launch_bounds__((Geo<T, LX, V>::NL * Geo<T, LX, V>::TLR))
    k_xinv(const MvArgs<T> a) {
  using G = Geo<T, LX, V>;
  constexpr int E = G::ER, TL = G::TLR, NL = G::NL;
  __shared__ cx<T> lds[NL * G::LP];
  const int b = blockIdx.z;
  if (retired(a, b)) return;
  const int t = threadIdx.x % TL;
  const int line = threadIdx.x / TL;
  const long row = long(blockIdx.x) * NL + line;
  const long nrows = long(a.out_z1 - a.out_z0) * a.ny;
  const bool live = row < nrows;
  const int z = live ? a.out_z0 + int(row / a.ny) : a.out_z0;
  const int yy = live ? int(row % a.ny) : 0;
  const cx<T>* in = a.T1 + b * a.T1_bs + (long(z) * a.ny + yy) * LX;
  const long cs = long(a.nz) * a.ny * LX;
  cx<T> v[3][E];
  const typename G::RowLds addr{line * G::LP};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[c][m] = live ? in[c * cs + t + m * TL] : cx<T>{0, 0};
    fft_line<T, LX, E, true>(v[c], lds, addr, t, a.tw);
  }
  if (!live) return;
  const long cell = long(yy) * a.nx;
  cx<T>* y = a.y + b * a.y_bs + long(z - a.y_zoff) * a.ny * a.nx + cell;
  const cx<T>* x = a.x ? a.x + b * a.x_bs + long(z - a.x_zoff) * a.ny * a.nx + cell : nullptr;
  const cx<T>* e = a.e ? a.e + b * a.e_bs + long(z - a.e_zoff) * a.ny * a.nx + cell : nullptr;
  const T* M = (a.M && a.a_m != T(0)) ? a.M + b * a.M_bs + long(z - a.M_zoff) * a.ny * a.nx + cell
                                       : nullptr;
  const T xs = a.xscale ? T(a.xscale[b * a.xscale_bs]) : T(1);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int i = t + m * TL;
    if (i >= a.nx) continue;
    cx<T> r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = a.a_s * v[c][m];
    if (x != nullptr && (a.a_x != T(0) || M != nullptr)) {
      cx<T> xv[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) xv[c] = xs * x[c * a.x_cs + i];
#pragma unroll
      for (int c = 0; c < 3; ++c) r[c] = r[c] + a.a_x * xv[c];
      if (M != nullptr) {
        T mm[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) mm[c] = M[c * a.M_cs + i];
        cx<T> mx[3];
        tensor_apply(mm, xv, mx);
#pragma unroll
        for (int c = 0; c < 3; ++c) r[c] = r[c] - a.a_m * mx[c];
      }
    }
    if (e != nullptr) {
#pragma unroll
      for (int c = 0; c < 3; ++c) r[c] = r[c] + a.a_e * e[c * a.e_cs + i];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) store_stream(&y[c * a.y_cs + i], r[c]);
  }
}

}  // namespace ie
