// Learned initial guess: a 3-D convolutional encoder-decoder trained and run with hand-written
// kernels.  Convolutions are im2col + a BF16 MFMA GEMM with float32 accumulation
// (v_mfma_f32_16x16x32_bf16); backward passes use the same GEMM (data gradient through the
// transposed weights, weight gradient with split K) and gather-form col2im (no atomics).
// Activations are channels-last BF16; master weights, gradients and Adam moments are float32.
//
// Architecture (level l has base * 2^l channels; 3x3x3 convolutions with bias and ReLU):
//   encoder  level 0: conv(in -> C0), conv(C0 -> C0); level l >= 1: 2x2x2 average pooling,
//            conv(C_{l-1} -> C_l), conv(C_l -> C_l)
//   decoder  l = L-2 .. 0: [nearest 2x upsampling of level l+1, skip l] -> conv -> conv
//   head     1x1x1 conv C0 -> out (no ReLU)
// Weights per layer: [taps][c_in][c_out] then bias [c_out], taps ordered (dz, dy, dx), z slowest.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "context.hpp"
#include "nn.hpp"
#include "prof.hpp"

using u16 = uint16_t;

namespace ie {
namespace nn {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline float bf2f(u16 h) {
  union {
    uint32_t u;
    float f;
  } v;
  v.u = uint32_t(h) << 16;
  return v.f;
}
__host__ __device__ inline u16 f2bf(float f) {  // round to nearest even
  union {
    uint32_t u;
    float f;
  } v;
  v.f = f;
  if ((v.u & 0x7f800000u) == 0x7f800000u) return u16((v.u >> 16) | ((v.u & 0xffff) ? 0x40 : 0));
  v.u += 0x7fffu + ((v.u >> 16) & 1u);
  return u16(v.u >> 16);
}

// ---------------------------------------------------------------------------------------
// GEMM: C(M x N) = A(M x K) B(K x N), BF16 operands, float32 accumulation on MFMA.
// A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn]; out of range reads are zero.
// blockIdx.z handles K range [z kchunk, (z+1) kchunk).  Output: float32 partials
// Cf[z cpart + m scm + n scn] (split K) or, with Cb, BF16 with optional bias and ReLU.
// Tile 64 x 64 x 32, four wavefronts each owning a 32 x 32 quarter (2 x 2 MFMA tiles of
// 16 x 16 x 32: lane l supplies row (or column) l % 16 at k = 8 (l / 16) .. 8 (l / 16) + 7).
// ---------------------------------------------------------------------------------------
constexpr int GBM = 64, GBN = 64, GBK = 32, GPAD = 8;  // rows of 80 bytes: 16-byte aligned reads

template <bool A_KC, bool B_NC>
__global__ void __launch_bounds__(256)
    k_gemm(const u16* __restrict__ A, long sam, long sak, const u16* __restrict__ B, long sbk,
           long sbn, int M, int N, int K, int kchunk, float* __restrict__ Cf, long scm, long scn,
           long cpart, u16* __restrict__ Cb, const float* __restrict__ bias, int relu) {
  __shared__ __align__(16) u16 As[GBM][GBK + GPAD];
  __shared__ __align__(16) u16 Bs[GBN][GBK + GPAD];
  const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += GBK) {
#pragma unroll
    for (int i = 0; i < (GBM * GBK) / 256; ++i) {
      const int idx = t + i * 256;
      int mm, kk;
      if (A_KC) {
        mm = idx / GBK;
        kk = idx % GBK;
      } else {
        kk = idx / GBM;
        mm = idx % GBM;
      }
      const int gm = m0 + mm, gk = k0 + kk;
      As[mm][kk] = (gm < M && gk < ke) ? A[long(gm) * sam + long(gk) * sak] : u16(0);
    }
#pragma unroll
    for (int i = 0; i < (GBN * GBK) / 256; ++i) {
      const int idx = t + i * 256;
      int nn, kk;
      if (B_NC) {
        kk = idx / GBN;
        nn = idx % GBN;
      } else {
        nn = idx / GBK;
        kk = idx % GBK;
      }
      const int gn = n0 + nn, gk = k0 + kk;
      Bs[nn][kk] = (gn < N && gk < ke) ? B[long(gk) * sbk + long(gn) * sbn] : u16(0);
    }
    __syncthreads();
    static_assert(GBK == 32, "one 16x16x32 MFMA per K tile");
    bf8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = *reinterpret_cast<const bf8*>(&As[wm + i * 16 + (lane & 15)][8 * (lane >> 4)]);
      b[i] = *reinterpret_cast<const bf8*>(&Bs[wn + i * 16 + (lane & 15)][8 * (lane >> 4)]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // D layout of the 16x16 tile: lane l holds rows 4 (l / 16) + e, e = 0..3, column l % 16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm + i * 16 + 4 * (lane >> 4) + e;
        const int n = n0 + wn + j * 16 + (lane & 15);
        if (m >= M || n >= N) continue;
        float v = acc[i][j][e];
        if (Cb != nullptr) {
          if (bias) v += bias[n];
          if (relu) v = fmaxf(v, 0.f);
          Cb[long(m) * scm + long(n) * scn] = f2bf(v);
        } else {
          Cf[long(blockIdx.z) * cpart + long(m) * scm + long(n) * scn] = v;
        }
      }
}

// ---------------------------------------------------------------------------------------
// Convolution as an implicit GEMM (inference): out(m, n) = sum_k A(m, k) W(k, n) with A(m, k)
// the im2col value of k_im2col below, gathered while the A tile is loaded instead of being
// written to memory first.  k = tap C + ch with C = c1 + c2 channels (ch < c1 from in1, read at
// half resolution when up1; the rest from in2); each thread loads eight consecutive channels of
// one tap as one 16-byte read, so c1 and c2 must be multiples of 8.  W is [K][co] BF16 (as the
// weights are stored).  Same tile, MFMA and epilogue as k_gemm (BF16 output with bias and ReLU,
// or float32).  blockIdx.z splits K into chunks of kchunk (a multiple of the K tile): with
// more than one split every block writes float32 partials to Cp[z][m][n] instead, summed by
// k_splitk_out (the deep layers have few voxels and long K).
// ---------------------------------------------------------------------------------------
template <int TAPS>
__global__ void __launch_bounds__(256)
    k_conv_igemm(const u16* __restrict__ in1, int c1, int up1, const u16* __restrict__ in2,
                 int c2, int nb, int Z, int Y, int X, const u16* __restrict__ W, int co,
                 int kchunk, float* __restrict__ Cp, float* __restrict__ Cf,
                 u16* __restrict__ Cb, const float* __restrict__ bias, int relu) {
  __shared__ __align__(16) u16 As[GBM][GBK + GPAD];
  __shared__ __align__(16) u16 Bs[GBN][GBK + GPAD];
  const int C = c1 + c2, K = TAPS * C;
  const long M = long(nb) * Z * Y * X;
  const long m0 = long(blockIdx.x) * GBM;
  const int n0 = blockIdx.y * GBN;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  // this thread's A chunk: row mm of the tile, channels 8 kc .. 8 kc + 7 of each K tile
  const int mm = t >> 2, kc = t & 3;
  const long m = m0 + mm;
  const bool mok = m < M;
  const long mc = mok ? m : 0;
  const int x = int(mc % X), y = int((mc / X) % Y), z = int((mc / (long(X) * Y)) % Z);
  const int b = int(mc / (long(X) * Y * Z));
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += GBK) {
    {
      const int k = k0 + 8 * kc;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (mok && k < ke) {
        const int tap = k / C, ch = k % C;
        int zz = z, yy = y, xx = x;
        if (TAPS == 27) {
          zz += tap / 9 - 1;
          yy += (tap / 3) % 3 - 1;
          xx += tap % 3 - 1;
        }
        if (zz >= 0 && zz < Z && yy >= 0 && yy < Y && xx >= 0 && xx < X) {
          const u16* src;
          if (ch < c1)
            src = up1 ? in1 + (((long(b) * (Z / 2) + zz / 2) * (Y / 2) + yy / 2) * (X / 2) +
                               xx / 2) * c1 + ch
                      : in1 + (((long(b) * Z + zz) * Y + yy) * X + xx) * c1 + ch;
          else
            src = in2 + (((long(b) * Z + zz) * Y + yy) * X + xx) * c2 + (ch - c1);
          v = *reinterpret_cast<const uint4*>(src);
        }
      }
      *reinterpret_cast<uint4*>(&As[mm][8 * kc]) = v;
    }
#pragma unroll
    for (int i = 0; i < (GBN * GBK) / 256; ++i) {
      const int idx = t + i * 256;
      const int kk = idx / GBN, nn = idx % GBN;
      const int gn = n0 + nn, gk = k0 + kk;
      Bs[nn][kk] = (gn < co && gk < ke) ? W[long(gk) * co + gn] : u16(0);
    }
    __syncthreads();
    bf8 a[2], bv[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = *reinterpret_cast<const bf8*>(&As[wm + i * 16 + (lane & 15)][8 * (lane >> 4)]);
      bv[i] = *reinterpret_cast<const bf8*>(&Bs[wn + i * 16 + (lane & 15)][8 * (lane >> 4)]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bv[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const long mo = m0 + wm + i * 16 + 4 * (lane >> 4) + e;
        const int n = n0 + wn + j * 16 + (lane & 15);
        if (mo >= M || n >= co) continue;
        float v = acc[i][j][e];
        if (Cp != nullptr) {
          Cp[(long(blockIdx.z) * M + mo) * co + n] = v;
        } else if (Cb != nullptr) {
          if (bias) v += bias[n];
          if (relu) v = fmaxf(v, 0.f);
          Cb[mo * co + n] = f2bf(v);
        } else {
          Cf[mo * co + n] = v;
        }
      }
}

// out = sum_z part[z] (fixed order) for n values of co columns, then bias and ReLU and BF16
// (Cb) or float32 as is (Cf)
__global__ void k_splitk_out(const float* __restrict__ part, int splits, long n, int co,
                             float* __restrict__ Cf, u16* __restrict__ Cb,
                             const float* __restrict__ bias, int relu) {
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += long(gridDim.x) * blockDim.x) {
    float v = 0.f;
    for (int z = 0; z < splits; ++z) v += part[z * n + i];
    if (Cb != nullptr) {
      if (bias) v += bias[i % co];
      if (relu) v = fmaxf(v, 0.f);
      Cb[i] = f2bf(v);
    } else {
      Cf[i] = v;
    }
  }
}

// out[i] (+)= sum_z part[z][i], fixed order
__global__ void k_splitk_sum(const float* __restrict__ part, long cpart, int splits, long n,
                             float* __restrict__ out, int accumulate) {
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x) {
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[z * cpart + i];
    out[i] = accumulate ? out[i] + s : s;
  }
}

// Col[m][tap C + ch], C = c1 + c2, over the fine grid (nb, Z, Y, X); ch < c1 from in1 (read at
// half resolution when up1), ch >= c1 from in2; zero padding.
__global__ void k_im2col(const u16* __restrict__ in1, int c1, int up1, const u16* __restrict__ in2,
                         int c2, int nb, int Z, int Y, int X, int taps, u16* __restrict__ col) {
  const int C = c1 + c2;
  const long M = long(nb) * Z * Y * X;
  const long total = M * taps * C;
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += long(gridDim.x) * blockDim.x) {
    const int ch = int(i % C);
    const int tap = int((i / C) % taps);
    const long m = i / (long(C) * taps);
    int x = int(m % X), y = int((m / X) % Y), z = int((m / (long(X) * Y)) % Z);
    const int b = int(m / (long(X) * Y * Z));
    if (taps == 27) {
      z += tap / 9 - 1;
      y += (tap / 3) % 3 - 1;
      x += tap % 3 - 1;
    }
    u16 v = 0;
    if (z >= 0 && z < Z && y >= 0 && y < Y && x >= 0 && x < X) {
      if (ch < c1) {
        if (up1)
          v = in1[(((long(b) * (Z / 2) + z / 2) * (Y / 2) + y / 2) * (X / 2) + x / 2) * c1 + ch];
        else
          v = in1[(((long(b) * Z + z) * Y + y) * X + x) * c1 + ch];
      } else {
        v = in2[(((long(b) * Z + z) * Y + y) * X + x) * c2 + (ch - c1)];
      }
    }
    col[i] = v;
  }
}

// Gather-form col2im of dCol [M][taps C] (float32): gradient of the input channels
// [ch0, ch0 + cn) at every fine-grid position, written (or added) to d [M][cn] (float32); with
// down = 1 the fine-grid gradient is summed over the 8 children of each coarse cell (adjoint of
// nearest upsampling) and d is [nb Z/2 Y/2 X/2][cn].
__global__ void k_col2im(const float* __restrict__ dcol, int C, int ch0, int cn, int nb, int Z,
                         int Y, int X, int taps, int down, float* __restrict__ d, int accumulate) {
  const int Zc = down ? Z / 2 : Z, Yc = down ? Y / 2 : Y, Xc = down ? X / 2 : X;
  const long total = long(nb) * Zc * Yc * Xc * cn;
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += long(gridDim.x) * blockDim.x) {
    const int ch = int(i % cn);
    const long p = i / cn;
    const int xc = int(p % Xc), yc = int((p / Xc) % Yc), zc = int((p / (long(Xc) * Yc)) % Zc);
    const int b = int(p / (long(Xc) * Yc * Zc));
    float s = 0.f;
    const int nch = down ? 8 : 1;
    for (int q = 0; q < nch; ++q) {
      const int z = down ? 2 * zc + (q >> 2) : zc;
      const int y = down ? 2 * yc + ((q >> 1) & 1) : yc;
      const int x = down ? 2 * xc + (q & 1) : xc;
      for (int tap = 0; tap < taps; ++tap) {
        int zz = z, yy = y, xx = x;
        if (taps == 27) {
          zz -= tap / 9 - 1;
          yy -= (tap / 3) % 3 - 1;
          xx -= tap % 3 - 1;
        }
        if (zz < 0 || zz >= Z || yy < 0 || yy >= Y || xx < 0 || xx >= X) continue;
        const long m = ((long(b) * Z + zz) * Y + yy) * X + xx;
        s += dcol[(m * taps + tap) * C + ch0 + ch];
      }
    }
    d[i] = accumulate ? d[i] + s : s;
  }
}

__global__ void k_pool(const u16* __restrict__ in, int c, int nb, int Z, int Y, int X,
                       u16* __restrict__ out) {
  const long total = long(nb) * (Z / 2) * (Y / 2) * (X / 2) * c;
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += long(gridDim.x) * blockDim.x) {
    const int ch = int(i % c);
    const long p = i / c;
    const int X2 = X / 2, Y2 = Y / 2, Z2 = Z / 2;
    const int x = int(p % X2), y = int((p / X2) % Y2), z = int((p / (long(X2) * Y2)) % Z2);
    const int b = int(p / (long(X2) * Y2 * Z2));
    float s = 0.f;
    for (int q = 0; q < 8; ++q)
      s += bf2f(in[(((long(b) * Z + 2 * z + (q >> 2)) * Y + 2 * y + ((q >> 1) & 1)) * X + 2 * x +
                    (q & 1)) * c + ch]);
    out[i] = f2bf(s * 0.125f);
  }
}

// d_fine (+)= d_coarse / 8 (adjoint of 2x2x2 averaging), float32
__global__ void k_pool_back(const float* __restrict__ dc, int c, int nb, int Z, int Y, int X,
                            float* __restrict__ df, int accumulate) {
  const long total = long(nb) * Z * Y * X * c;
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += long(gridDim.x) * blockDim.x) {
    const int ch = int(i % c);
    const long p = i / c;
    const int x = int(p % X), y = int((p / X) % Y), z = int((p / (long(X) * Y)) % Z);
    const int b = int(p / (long(X) * Y * Z));
    const float v =
        0.125f * dc[(((long(b) * (Z / 2) + z / 2) * (Y / 2) + y / 2) * (X / 2) + x / 2) * c + ch];
    df[i] = accumulate ? df[i] + v : v;
  }
}

// g16 = bf16(relu ? (out > 0 ? g : 0) : g), and the masked float gradient kept for the bias
__global__ void k_relu_cast(const float* __restrict__ g, const u16* __restrict__ out, int relu,
                            long n, u16* __restrict__ g16, float* __restrict__ gm) {
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x) {
    float v = g[i];
    if (relu && !(bf2f(out[i]) > 0.f)) v = 0.f;
    g16[i] = f2bf(v);
    gm[i] = v;
  }
}

// column sums (bias gradient): out[n] (+)= sum_m g[m][n]; one block per column, fixed order
__global__ void __launch_bounds__(256) k_colsum(const float* __restrict__ g, long M, int N,
                                                float* __restrict__ out) {
  __shared__ float sh[256];
  const int n = blockIdx.x;
  float s = 0.f;
  for (long m = threadIdx.x; m < M; m += 256) s += g[m * N + n];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = sh[0];
}

// MSE: per-block partial sums of (y - t)^2 and the gradient 2 (y - t) / n
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             long n, float* __restrict__ grad,
                                             double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (long i = long(blockIdx.x) * 256 + threadIdx.x; i < n; i += long(gridDim.x) * 256) {
    const float d = y[i] - t[i];
    grad[i] = 2.f * d / float(n);
    s += double(d) * double(d);
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, u16* __restrict__ p16, long n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    p16[i] = f2bf(pi);
  }
}

__global__ void k_to_bf16(const float* __restrict__ a, u16* __restrict__ b, long n) {
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x)
    b[i] = f2bf(a[i]);
}

// Network input for one block, 14 channels: the contraction-form tensor
// I - 2 sigma0 (dsigma + 2 sigma0 I)^-1 (bounded in (-1, 1); xx, yy, zz, xy, xz, yz), the field
// b e^{-i phi} / rms(b) (re, im of x, y, z) and k0 h (re, im).  phi = arg(sum b.b) / 2 fixes the
// global phase (b -> b e^{i a} leaves the features unchanged), rot = e^{-i phi}.  D: float64
// dsigma [6][nb] with component stride cs; b: complex128 [3][nb]; output BF16 [nb][14].
__global__ void k_features(const double* __restrict__ D, long cs, const c128* __restrict__ b,
                           long nb, double sigma0, double inv_rms, c128 rot, double k0h_re,
                           double k0h_im, u16* __restrict__ x) {
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < nb;
       i += long(gridDim.x) * blockDim.x) {
    const double t = 2.0 * sigma0;
    const double xx = D[i] + t, yy = D[cs + i] + t, zz = D[2 * cs + i] + t;
    const double xy = D[3 * cs + i], xz = D[4 * cs + i], yz = D[5 * cs + i];
    // adjugate / determinant of the symmetric matrix
    const double cxx = yy * zz - yz * yz, cyy = xx * zz - xz * xz, czz = xx * yy - xy * xy;
    const double cxy = xz * yz - xy * zz, cxz = xy * yz - xz * yy, cyz = xy * xz - xx * yz;
    const double det = xx * cxx + xy * cxy + xz * cxz;
    const double f = t / det;
    u16* o = x + i * 14;
    o[0] = f2bf(float(1.0 - f * cxx));
    o[1] = f2bf(float(1.0 - f * cyy));
    o[2] = f2bf(float(1.0 - f * czz));
    o[3] = f2bf(float(-f * cxy));
    o[4] = f2bf(float(-f * cxz));
    o[5] = f2bf(float(-f * cyz));
    for (int c = 0; c < 3; ++c) {
      const c128 v = b[c * nb + i];
      o[6 + 2 * c] = f2bf(float((v.re * rot.re - v.im * rot.im) * inv_rms));
      o[7 + 2 * c] = f2bf(float((v.re * rot.im + v.im * rot.re) * inv_rms));
    }
    o[12] = f2bf(float(k0h_re));
    o[13] = f2bf(float(k0h_im));
  }
}

// training target: y = (E - b) e^{-i phi} / rms(b), float32 channels-last [nb][6]
__global__ void k_target(const c128* __restrict__ b, const c128* __restrict__ E, long nb,
                         double inv_rms, c128 rot, float* __restrict__ y) {
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < nb;
       i += long(gridDim.x) * blockDim.x)
    for (int c = 0; c < 3; ++c) {
      const c128 v = b[c * nb + i], e = E[c * nb + i];
      const double dr = e.re - v.re, di = e.im - v.im;
      y[i * 6 + 2 * c] = float((dr * rot.re - di * rot.im) * inv_rms);
      y[i * 6 + 2 * c + 1] = float((dr * rot.im + di * rot.re) * inv_rms);
    }
}

// x0 = b + rms e^{i phi} (y_re + i y_im) per component; urot = rms e^{i phi}
__global__ void k_apply_guess(const c128* __restrict__ b, const float* __restrict__ y, long nb,
                              c128 urot, c128* __restrict__ x0) {
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < nb;
       i += long(gridDim.x) * blockDim.x)
    for (int c = 0; c < 3; ++c) {
      const c128 v = b[c * nb + i];
      const double yr = y[i * 6 + 2 * c], yi = y[i * 6 + 2 * c + 1];
      x0[c * nb + i] = c128{v.re + urot.re * yr - urot.im * yi, v.im + urot.re * yi + urot.im * yr};
    }
}

// per-block partial sums of b.b (unconjugated) over [3][nb] for `batch` vectors: part[b][g]
__global__ void __launch_bounds__(256) k_sumsq(const c128* __restrict__ v, long n,
                                               c128* __restrict__ part) {
  __shared__ double sr[256], si[256];
  const int b = blockIdx.y;
  const c128* p = v + long(b) * n;
  double re = 0, im = 0;
  for (long i = long(blockIdx.x) * 256 + threadIdx.x; i < n; i += long(gridDim.x) * 256) {
    const c128 z = p[i];
    re += z.re * z.re - z.im * z.im;
    im += 2.0 * z.re * z.im;
  }
  sr[threadIdx.x] = re;
  si[threadIdx.x] = im;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      sr[threadIdx.x] += sr[threadIdx.x + k];
      si[threadIdx.x] += si[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[long(b) * gridDim.x + blockIdx.x] = c128{sr[0], si[0]};
}

// grid for the element-wise grid-stride kernels (x extent times 256 stays below 2^32)
int grid1(long n) { return int(std::min<long>((1L << 24) - 1, (n + 255) / 256)); }

}  // namespace nn
}  // namespace ie

// ---------------------------------------------------------------------------------------
// host side: the network object
// ---------------------------------------------------------------------------------------
using namespace ie;
using namespace ie::nn;

struct NnLayer {
  int ci, co, taps, relu;
  long w_off, b_off;  // offsets into the flat parameter vector
  // per-forward state
  int Z = 0, Y = 0, X = 0;  // fine grid of the layer's output
  long M = 0;
  DevBuf col, out;   // im2col (bf16 [M][taps ci]) and output (bf16 [M][co]; head float32)
};

struct ie_nn {
  int in_ch, out_ch, base, levels;
  std::vector<NnLayer> L;
  long np = 0;
  DevBuf p32, g32, m32, v32, p16;
  long step = 0;
  // forward state
  int nb = 0, Z = 0, Y = 0, X = 0;
  DevBuf x16;                               // network input copy (bf16)
  std::vector<DevBuf> pooled;               // pooled inputs per level >= 1
  DevBuf gcur, gtmp, gsk[8], g16, gmask, dcol, part, mse_part, gy;
  DevBuf xg, res;          // learned guesses and their residuals
  DevBuf sq;               // partial sums for the phase of the right-hand side
  bool keep_cols = true;  // training keeps every layer's im2col for the backward pass
  DevBuf icol;            // shared im2col buffer for inference
  std::vector<double> hpart;
};

namespace {

int gemm(hipStream_t s, bool akc, bool bnc, const u16* A, long sam, long sak, const u16* B,
         long sbk, long sbn, int M, int N, int K, int splits, float* Cf, long scm, long scn,
         long cpart, u16* Cb, const float* bias, int relu) {
  const int kchunk = ((K + splits - 1) / splits + GBK - 1) / GBK * GBK;
  const int z = (K + kchunk - 1) / kchunk;
  dim3 grid(ceil_div(M, GBM), ceil_div(N, GBN), z);
  char tag[64];  // the shape, from which a profile derives the flops (2 M N K)
  snprintf(tag, sizeof(tag), "bf16 M%dxN%dxK%d", M, N, K);
  ProfScope ps(s, "nn_gemm", tag, 2.0 * (double(M) * K + double(K) * N) + 4.0 * double(M) * N);
#define IE_GEMM(AK, BN)                                                                          \
  hipLaunchKernelGGL((k_gemm<AK, BN>), grid, dim3(256), 0, s, A, sam, sak, B, sbk, sbn, M, N, K, \
                     kchunk, Cf, scm, scn, cpart, Cb, bias, relu)
  if (akc && bnc)
    IE_GEMM(true, true);
  else if (akc)
    IE_GEMM(true, false);
  else if (bnc)
    IE_GEMM(false, true);
  else
    IE_GEMM(false, false);
#undef IE_GEMM
  IE_LAUNCH_CHECK();
  return z;
}

void build_layers(ie_nn* n) {
  const int Lv = n->levels;
  std::vector<int> ch(Lv);
  for (int l = 0; l < Lv; ++l) ch[l] = n->base << l;
  auto add = [&](int ci, int co, int taps, int relu) {
    NnLayer y;
    y.ci = ci;
    y.co = co;
    y.taps = taps;
    y.relu = relu;
    y.w_off = n->np;
    n->np += long(taps) * ci * co;
    y.b_off = n->np;
    n->np += co;
    n->L.push_back(std::move(y));
  };
  add(n->in_ch, ch[0], 27, 1);
  add(ch[0], ch[0], 27, 1);
  for (int l = 1; l < Lv; ++l) {
    add(ch[l - 1], ch[l], 27, 1);
    add(ch[l], ch[l], 27, 1);
  }
  for (int l = Lv - 2; l >= 0; --l) {
    add(ch[l + 1] + ch[l], ch[l], 27, 1);
    add(ch[l], ch[l], 27, 1);
  }
  add(ch[0], n->out_ch, 1, 0);
}

// conv layer forward: im2col of (in1 [upsampled], in2) then GEMM with bias / ReLU
int conv_fwd(ie_nn* n, NnLayer& y, const u16* in1, int c1, int up1, const u16* in2, int c2,
             int Z, int Y, int X, hipStream_t s, float* out32) {
  y.Z = Z;
  y.Y = Y;
  y.X = X;
  y.M = long(n->nb) * Z * Y * X;
  const long K = long(y.taps) * (c1 + c2);
  const u16* W = n->p16.as<u16>() + y.w_off;
  const float* bias = n->p32.as<float>() + y.b_off;
  if (!out32) IE_TRY(y.out.ensure(sizeof(u16) * y.M * y.co));
  if (!n->keep_cols && c1 % 8 == 0 && c2 % 8 == 0 && (y.taps == 27 || y.taps == 1)) {
    // inference: implicit GEMM, no im2col buffer
    char tag[64];
    snprintf(tag, sizeof(tag), "bf16 M%ldxN%dxK%ld", y.M, y.co, K);
    ProfScope ps(s, "nn_conv", tag, 2.0 * (double(y.M) * (c1 + c2) + double(K) * y.co) +
                                        (out32 ? 4.0 : 2.0) * double(y.M) * y.co);
    // split K until about 1024 blocks run, keeping at least four K tiles per split
    const long tiles = long(ceil_div(y.M, GBM)) * ceil_div(y.co, GBN);
    const int ktiles = ceil_div(K, GBK);
    int splits = int(std::min<long>(std::max<long>(1, (1024 + tiles - 1) / tiles), ktiles / 4));
    splits = std::max(1, std::min(splits, 16));
    const int kchunk = ceil_div(ktiles, splits) * GBK;
    splits = ceil_div(K, kchunk);
    float* part = nullptr;
    if (splits > 1) {
      IE_TRY(n->part.ensure(sizeof(float) * splits * y.M * y.co));
      part = n->part.as<float>();
    }
    u16* o16 = out32 ? nullptr : y.out.as<u16>();
    const float* bo = out32 ? nullptr : bias;
    const int ro = out32 ? 0 : y.relu;
    dim3 grid(unsigned(ceil_div(y.M, GBM)), unsigned(ceil_div(y.co, GBN)), unsigned(splits));
    if (y.taps == 27)
      hipLaunchKernelGGL(k_conv_igemm<27>, grid, dim3(256), 0, s, in1, c1, up1, in2, c2, n->nb, Z,
                         Y, X, W, y.co, kchunk, part, out32, o16, bo, ro);
    else
      hipLaunchKernelGGL(k_conv_igemm<1>, grid, dim3(256), 0, s, in1, c1, up1, in2, c2, n->nb, Z,
                         Y, X, W, y.co, kchunk, part, out32, o16, bo, ro);
    IE_LAUNCH_CHECK();
    if (splits > 1) {
      hipLaunchKernelGGL(k_splitk_out, dim3(grid1(y.M * y.co)), dim3(256), 0, s, part, splits,
                         y.M * y.co, y.co, out32, o16, bo, ro);
      IE_LAUNCH_CHECK();
    }
    return IE_OK;
  }
  DevBuf& colb = n->keep_cols ? y.col : n->icol;
  IE_TRY(colb.ensure(sizeof(u16) * y.M * K));
  u16* col = colb.as<u16>();
  {
    ProfScope ps(s, "nn_im2col", "", 2.0 * y.M * K);
    hipLaunchKernelGGL(k_im2col, dim3(grid1(y.M * K)), dim3(256), 0, s, in1, c1, up1, in2, c2,
                       n->nb, Z, Y, X, y.taps, col);
    IE_LAUNCH_CHECK();
  }
  if (out32) {  // head: float32 output, bias added by the caller
    gemm(s, true, true, col, K, 1, W, y.co, 1, int(y.M), y.co, int(K), 1, out32, y.co, 1, 0,
         nullptr, nullptr, 0);
    return IE_OK;
  }
  gemm(s, true, true, col, K, 1, W, y.co, 1, int(y.M), y.co, int(K), 1, nullptr, y.co, 1, 0,
       y.out.as<u16>(), bias, y.relu);
  return IE_OK;
}

__global__ void k_add_bias(float* __restrict__ y, const float* __restrict__ b, long M, int N) {
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < M * N; i += long(gridDim.x) * blockDim.x)
    y[i] += b[i % N];
}

int forward(ie_nn* n, const u16* x, int nb, int Z, int Y, int X, float* y, hipStream_t s) {
  if (Z % (1 << (n->levels - 1)) || Y % (1 << (n->levels - 1)) || X % (1 << (n->levels - 1)))
    return fail(IE_EINVAL, "grid sizes must be divisible by 2^(levels-1)");
  n->nb = nb;
  n->Z = Z;
  n->Y = Y;
  n->X = X;
  const int Lv = n->levels;
  n->pooled.resize(Lv);
  int k = 0;
  std::vector<const u16*> skip(Lv);
  std::vector<int> dims(3 * Lv);
  for (int l = 0; l < Lv; ++l) {
    dims[3 * l] = Z >> l;
    dims[3 * l + 1] = Y >> l;
    dims[3 * l + 2] = X >> l;
  }
  // encoder
  const u16* h = x;
  int hc = n->in_ch;
  for (int l = 0; l < Lv; ++l) {
    const int Zl = dims[3 * l], Yl = dims[3 * l + 1], Xl = dims[3 * l + 2];
    if (l > 0) {
      const long np_ = long(nb) * Zl * Yl * Xl * hc;
      IE_TRY(n->pooled[l].ensure(sizeof(u16) * np_));
      hipLaunchKernelGGL(k_pool, dim3(grid1(np_)), dim3(256), 0, s, h, hc, nb, dims[3 * l - 3],
                         dims[3 * l - 2], dims[3 * l - 1], n->pooled[l].as<u16>());
      IE_LAUNCH_CHECK();
      h = n->pooled[l].as<u16>();
    }
    IE_TRY(conv_fwd(n, n->L[k], h, hc, 0, nullptr, 0, Zl, Yl, Xl, s, nullptr));
    h = n->L[k].out.as<u16>();
    hc = n->L[k].co;
    ++k;
    IE_TRY(conv_fwd(n, n->L[k], h, hc, 0, nullptr, 0, Zl, Yl, Xl, s, nullptr));
    h = n->L[k].out.as<u16>();
    hc = n->L[k].co;
    ++k;
    skip[l] = h;
  }
  // decoder
  for (int l = Lv - 2; l >= 0; --l) {
    const int Zl = dims[3 * l], Yl = dims[3 * l + 1], Xl = dims[3 * l + 2];
    const int cs = n->base << l;
    IE_TRY(conv_fwd(n, n->L[k], h, hc, 1, skip[l], cs, Zl, Yl, Xl, s, nullptr));
    h = n->L[k].out.as<u16>();
    hc = n->L[k].co;
    ++k;
    IE_TRY(conv_fwd(n, n->L[k], h, hc, 0, nullptr, 0, Zl, Yl, Xl, s, nullptr));
    h = n->L[k].out.as<u16>();
    hc = n->L[k].co;
    ++k;
  }
  // head (float32 output)
  NnLayer& hd = n->L[k];
  IE_TRY(conv_fwd(n, hd, h, hc, 0, nullptr, 0, Z, Y, X, s, y));
  hipLaunchKernelGGL(k_add_bias, dim3(grid1(hd.M * hd.co)), dim3(256), 0, s, y,
                     n->p32.as<float>() + hd.b_off, hd.M, hd.co);
  IE_LAUNCH_CHECK();
  return IE_OK;
}

// Backward of one conv layer from the float32 gradient of its output (gout); writes parameter
// gradients (accumulated) and returns the float32 gradient of the im2col input (dcol) for the
// caller's col2im.
int conv_back(ie_nn* n, NnLayer& y, const float* gout, int cin, hipStream_t s) {
  const long K = long(y.taps) * cin;
  const long MN = y.M * y.co;
  IE_TRY(n->g16.ensure(sizeof(u16) * MN));
  IE_TRY(n->gmask.ensure(sizeof(float) * MN));
  // relu mask (the head has none) and BF16 copy
  hipLaunchKernelGGL(k_relu_cast, dim3(grid1(MN)), dim3(256), 0, s, gout,
                     y.relu ? y.out.as<u16>() : nullptr, y.relu, MN, n->g16.as<u16>(),
                     n->gmask.as<float>());
  IE_LAUNCH_CHECK();
  // bias gradient
  hipLaunchKernelGGL(k_colsum, dim3(y.co), dim3(256), 0, s, n->gmask.as<float>(), y.M, y.co,
                     n->g32.as<float>() + y.b_off);
  IE_LAUNCH_CHECK();
  // weight gradient dW[K][co] = Col^T g16, split over the spatial dimension
  const int splits = int(std::max<long>(1, std::min<long>(256, y.M / 2048)));
  const long cpart = K * y.co;
  IE_TRY(n->part.ensure(sizeof(float) * cpart * splits));
  const int z = gemm(s, false, true, y.col.as<u16>(), 1, K, n->g16.as<u16>(), y.co, 1, int(K),
                     y.co, int(y.M), splits, n->part.as<float>(), y.co, 1, cpart, nullptr, nullptr, 0);
  hipLaunchKernelGGL(k_splitk_sum, dim3(grid1(cpart)), dim3(256), 0, s, n->part.as<float>(), cpart,
                     z, cpart, n->g32.as<float>() + y.w_off, 0);
  IE_LAUNCH_CHECK();
  // input gradient through the transposed weights: dCol[M][K] = g16 W^T
  IE_TRY(n->dcol.ensure(sizeof(float) * y.M * K));
  const u16* W = n->p16.as<u16>() + y.w_off;
  gemm(s, true, false, n->g16.as<u16>(), y.co, 1, W, 1, y.co, int(y.M), int(K), y.co, 1,
       n->dcol.as<float>(), K, 1, 0, nullptr, nullptr, 0);
  return IE_OK;
}

int col2im(ie_nn* n, const NnLayer& y, int C, int ch0, int cn, int down, float* d, int acc,
           hipStream_t s) {
  const long tot = (down ? y.M / 8 : y.M) * cn;
  hipLaunchKernelGGL(k_col2im, dim3(grid1(tot)), dim3(256), 0, s, n->dcol.as<float>(), C, ch0, cn,
                     n->nb, y.Z, y.Y, y.X, y.taps, down, d, acc);
  IE_LAUNCH_CHECK();
  return IE_OK;
}

// Backward through the whole network from gy = dLoss/dy (float32, [M][out]); parameter
// gradients land in g32 (overwritten).
int backward(ie_nn* n, const float* gy, hipStream_t s) {
  const int Lv = n->levels;
  IE_HIP(hipMemsetAsync(n->g32.p, 0, sizeof(float) * n->np, s));
  long maxa = 0;
  for (auto& y : n->L) maxa = std::max(maxa, y.M * std::max(y.ci, y.co));
  IE_TRY(n->gcur.ensure(sizeof(float) * maxa));
  IE_TRY(n->gtmp.ensure(sizeof(float) * maxa));
  for (int l = 0; l < Lv; ++l) IE_TRY(n->gsk[l].ensure(sizeof(float) * maxa));
  float* A = n->gcur.as<float>();
  float* Bf = n->gtmp.as<float>();
  auto tmp = [&](const float* busy) { return busy == A ? Bf : A; };
  int k = int(n->L.size()) - 1;
  float* gc = A;
  {  // head
    NnLayer& y = n->L[k--];
    IE_TRY(conv_back(n, y, gy, y.ci, s));
    IE_TRY(col2im(n, y, y.ci, 0, y.ci, 0, gc, 0, s));
  }
  // decoder: forward order l = L-2 .. 0, so backward visits l = 0 .. L-2
  for (int l = 0; l <= Lv - 2; ++l) {
    NnLayer& yb = n->L[k--];
    IE_TRY(conv_back(n, yb, gc, yb.ci, s));
    float* t = tmp(gc);
    IE_TRY(col2im(n, yb, yb.ci, 0, yb.ci, 0, t, 0, s));
    gc = t;
    NnLayer& ya = n->L[k--];
    const int cu = n->base << (l + 1), cs = n->base << l;
    IE_TRY(conv_back(n, ya, gc, ya.ci, s));
    IE_TRY(col2im(n, ya, cu + cs, cu, cs, 0, n->gsk[l].as<float>(), 0, s));  // skip channels
    t = tmp(gc);
    IE_TRY(col2im(n, ya, cu + cs, 0, cu, 1, t, 0, s));  // upsampled channels -> coarse level
    gc = t;
  }
  // encoder: l = L-1 .. 0; gc holds the gradient of level l's output
  for (int l = Lv - 1; l >= 0; --l) {
    NnLayer& yb = n->L[k--];
    IE_TRY(conv_back(n, yb, gc, yb.ci, s));
    float* t = tmp(gc);
    IE_TRY(col2im(n, yb, yb.ci, 0, yb.ci, 0, t, 0, s));
    gc = t;
    NnLayer& ya = n->L[k--];
    IE_TRY(conv_back(n, ya, gc, ya.ci, s));
    if (l == 0) break;  // no gradient for the network input
    t = tmp(gc);
    IE_TRY(col2im(n, ya, ya.ci, 0, ya.ci, 0, t, 0, s));  // w.r.t. the pooled input of level l
    const NnLayer& prev = n->L[k];                        // second conv of level l-1
    hipLaunchKernelGGL(k_pool_back, dim3(grid1(prev.M * prev.co)), dim3(256), 0, s, t, prev.co,
                       n->nb, prev.Z, prev.Y, prev.X, n->gsk[l - 1].as<float>(), 1);
    IE_LAUNCH_CHECK();
    gc = n->gsk[l - 1].as<float>();  // skip contribution + pooling adjoint
  }
  return IE_OK;
}

int check_nn(const ie_nn* n) {
  if (n == nullptr) return fail(IE_EINVAL, "network handle is NULL");
  return IE_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------
// C entry points
// ---------------------------------------------------------------------------------------
extern "C" {

int ie_nn_create(const ie_nn_config* cfg, void* stream, ie_nn** out) {
  if (cfg == nullptr || out == nullptr) return fail(IE_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->in_ch < 1 || cfg->out_ch < 1 || cfg->base_ch < 1 || cfg->levels < 1 || cfg->levels > 6)
    return fail(IE_EINVAL, "bad network configuration");
  auto n = std::make_unique<ie_nn>();
  n->in_ch = cfg->in_ch;
  n->out_ch = cfg->out_ch;
  n->base = cfg->base_ch;
  n->levels = cfg->levels;
  build_layers(n.get());
  // He-normal weights (seeded), zero biases
  std::vector<float> h(n->np, 0.f);
  std::mt19937_64 rng(cfg->seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (auto& y : n->L) {
    const double sd = std::sqrt(2.0 / (double(y.taps) * y.ci));
    for (long i = 0; i < long(y.taps) * y.ci * y.co; ++i) h[y.w_off + i] = float(sd * nd(rng));
  }
  IE_TRY(n->p32.ensure(sizeof(float) * n->np));
  IE_TRY(n->g32.ensure(sizeof(float) * n->np));
  IE_TRY(n->m32.ensure(sizeof(float) * n->np));
  IE_TRY(n->v32.ensure(sizeof(float) * n->np));
  IE_TRY(n->p16.ensure(sizeof(u16) * n->np));
  hipStream_t s = (hipStream_t)stream;
  IE_HIP(hipMemcpyAsync(n->p32.p, h.data(), sizeof(float) * n->np, hipMemcpyHostToDevice, s));
  IE_HIP(hipMemsetAsync(n->m32.p, 0, sizeof(float) * n->np, s));
  IE_HIP(hipMemsetAsync(n->v32.p, 0, sizeof(float) * n->np, s));
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1(n->np)), dim3(256), 0, s, n->p32.as<float>(),
                     n->p16.as<u16>(), n->np);
  IE_LAUNCH_CHECK();
  IE_HIP(hipStreamSynchronize(s));
  *out = n.release();
  return IE_OK;
}

int ie_nn_destroy(ie_nn* n) {
  if (n == nullptr) return IE_OK;
  (void)hipDeviceSynchronize();
  delete n;
  return IE_OK;
}

int ie_nn_num_params(const ie_nn* n, int64_t* count) {
  IE_TRY(check_nn(n));
  if (count == nullptr) return fail(IE_EINVAL, "count is NULL");
  *count = n->np;
  return IE_OK;
}

int ie_nn_get_params(const ie_nn* n, float* host, int64_t count, int32_t which) {
  IE_TRY(check_nn(n));
  if (host == nullptr || count != n->np) return fail(IE_EINVAL, "need a host array of %ld floats", n->np);
  const DevBuf& b = which == 1 ? n->g32 : n->p32;
  IE_HIP(hipDeviceSynchronize());
  IE_HIP(hipMemcpy(host, b.p, sizeof(float) * n->np, hipMemcpyDeviceToHost));
  return IE_OK;
}

int ie_nn_set_params(ie_nn* n, const float* host, int64_t count) {
  IE_TRY(check_nn(n));
  if (host == nullptr || count != n->np) return fail(IE_EINVAL, "need a host array of %ld floats", n->np);
  IE_HIP(hipDeviceSynchronize());
  IE_HIP(hipMemcpy(n->p32.p, host, sizeof(float) * n->np, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1(n->np)), dim3(256), 0, 0, n->p32.as<float>(),
                     n->p16.as<u16>(), n->np);
  IE_LAUNCH_CHECK();
  IE_HIP(hipDeviceSynchronize());
  n->step = 0;
  IE_HIP(hipMemset(n->m32.p, 0, sizeof(float) * n->np));
  IE_HIP(hipMemset(n->v32.p, 0, sizeof(float) * n->np));
  return IE_OK;
}

int ie_nn_forward(ie_nn* n, const uint16_t* x, int32_t batch, int32_t nz, int32_t ny, int32_t nx,
                  float* y, void* stream) {
  IE_TRY(check_nn(n));
  if (x == nullptr || y == nullptr || batch < 1 || nz < 1 || ny < 1 || nx < 1)
    return fail(IE_EINVAL, "bad forward arguments");
  n->keep_cols = false;
  return forward(n, x, batch, nz, ny, nx, y, (hipStream_t)stream);
}

int ie_nn_backward(ie_nn* n, const uint16_t* x, const float* dy, int32_t batch, int32_t nz,
                   int32_t ny, int32_t nx, float* y, void* stream) {
  IE_TRY(check_nn(n));
  if (x == nullptr || dy == nullptr || y == nullptr) return fail(IE_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  n->keep_cols = true;
  IE_TRY(forward(n, x, batch, nz, ny, nx, y, s));
  return backward(n, dy, s);
}

int ie_nn_train_step(ie_nn* n, const uint16_t* x, const float* target, int32_t batch, int32_t nz,
                     int32_t ny, int32_t nx, float lr, float* loss, void* stream) {
  IE_TRY(check_nn(n));
  if (x == nullptr || target == nullptr || !(lr > 0)) return fail(IE_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  const long cnt = long(batch) * nz * ny * nx * n->out_ch;
  IE_TRY(n->gy.ensure(sizeof(float) * 2 * cnt));
  float* y = n->gy.as<float>();
  float* g = y + cnt;
  n->keep_cols = true;
  IE_TRY(forward(n, x, batch, nz, ny, nx, y, s));
  const int nbk = 256;
  IE_TRY(n->mse_part.ensure(sizeof(double) * nbk));
  hipLaunchKernelGGL(k_mse, dim3(nbk), dim3(256), 0, s, y, target, cnt, g,
                     n->mse_part.as<double>());
  IE_LAUNCH_CHECK();
  IE_TRY(backward(n, g, s));
  n->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, float(n->step)), c2 = 1.f - std::pow(b2, float(n->step));
  hipLaunchKernelGGL(k_adam, dim3(grid1(n->np)), dim3(256), 0, s, n->p32.as<float>(),
                     n->g32.as<float>(), n->m32.as<float>(), n->v32.as<float>(), n->p16.as<u16>(),
                     n->np, lr, b1, b2, 1e-8f, c1, c2);
  IE_LAUNCH_CHECK();
  if (loss != nullptr) {
    n->hpart.resize(nbk);
    IE_HIP(hipMemcpyAsync(n->hpart.data(), n->mse_part.p, sizeof(double) * nbk,
                          hipMemcpyDeviceToHost, s));
    IE_HIP(hipStreamSynchronize(s));
    double t = 0;
    for (double v : n->hpart) t += v;
    *loss = float(t / double(cnt));
  }
  return IE_OK;
}

int ie_nn_gemm(const uint16_t* A, const uint16_t* B, float* Cm, int32_t M, int32_t N, int32_t K,
               int32_t a_trans, int32_t b_trans, int32_t splits, void* stream) {
  if (A == nullptr || B == nullptr || Cm == nullptr || M < 1 || N < 1 || K < 1 || splits < 1 ||
      splits > 64)
    return fail(IE_EINVAL, "bad GEMM arguments");
  hipStream_t s = (hipStream_t)stream;
  const long sam = a_trans ? 1 : K, sak = a_trans ? M : 1;
  const long sbk = b_trans ? 1 : N, sbn = b_trans ? K : 1;
  const long cpart = long(M) * N;
  DevBuf part;
  IE_TRY(part.ensure(sizeof(float) * cpart * splits));
  const int z = gemm(s, !a_trans, !b_trans, A, sam, sak, B, sbk, sbn, M, N, K, splits,
                     part.as<float>(), N, 1, cpart, nullptr, nullptr, 0);
  hipLaunchKernelGGL(k_splitk_sum, dim3(grid1(cpart)), dim3(256), 0, s, part.as<float>(), cpart, z,
                     cpart, Cm, 0);
  IE_LAUNCH_CHECK();
  IE_HIP(hipStreamSynchronize(s));
  return IE_OK;
}

}  // extern "C"

namespace ie {

int nn_check_shape(const ie_nn* n, int nz, int ny, int nx) {
  const int q = 1 << (n->levels - 1);
  if (n->in_ch != 14 || n->out_ch != 6)
    return fail(IE_EINVAL, "the guess network must map 14 feature channels to 6 field channels");
  if (nz % q || ny % q || nx % q)
    return fail(IE_EINVAL, "grid %dx%dx%d is not divisible by 2^(levels-1) = %d", nx, ny, nz, q);
  return IE_OK;
}

namespace {

void k0h(const ie_ctx* c, double* re, double* im) {
  *re = c->med.k0re * c->grid.h;
  *im = c->med.k0im * c->grid.h;
}

// network forward over `batch` blocks of nb cells in chunks of about 2^20 cells
int forward_chunked(ie_nn* n, const u16* x, int batch, int nz, int ny, int nx, float* y,
                    hipStream_t s) {
  const long nb = long(nz) * ny * nx;
  const int per = int(std::max<long>(1, (1L << 20) / nb));
  n->keep_cols = false;
  for (int b0 = 0; b0 < batch; b0 += per) {
    const int k = std::min(per, batch - b0);
    IE_TRY(forward(n, x + long(b0) * nb * 14, k, nz, ny, nx, y + long(b0) * nb * 6, s));
  }
  return IE_OK;
}

// rms(b) = ||b|| / sqrt(3 nb) and the phase rotation e^{-i phi}, phi = arg(sum b.b) / 2, for
// `batch` vectors b [batch][3][nb] (fixed-order reductions; synchronises)
int scale_and_phase(const c128* b, long nb, int batch, DevBuf& sq, KrylovWork& w, hipStream_t s,
                    std::vector<double>& rms, std::vector<c128>& rot) {
  rms.resize(batch);
  rot.resize(batch);
  IE_TRY(norms_host(b, 3 * nb, batch, rms.data(), w, s));
  const int G = int(std::min<long>(256, ceil_div(3 * nb, 256)));
  IE_TRY(sq.ensure(sizeof(c128) * G * batch));
  hipLaunchKernelGGL(k_sumsq, dim3(G, batch), dim3(256), 0, s, b, 3 * nb, sq.as<c128>());
  IE_LAUNCH_CHECK();
  std::vector<c128> h(size_t(G) * batch);
  IE_HIP(hipMemcpyAsync(h.data(), sq.p, sizeof(c128) * G * batch, hipMemcpyDeviceToHost, s));
  IE_HIP(hipStreamSynchronize(s));
  for (int q = 0; q < batch; ++q) {
    double re = 0, im = 0;
    for (int g = 0; g < G; ++g) {
      re += h[size_t(q) * G + g].re;
      im += h[size_t(q) * G + g].im;
    }
    const double phi = (re == 0 && im == 0) ? 0.0 : 0.5 * std::atan2(im, re);
    rot[q] = c128{std::cos(phi), -std::sin(phi)};
    rms[q] = rms[q] / std::sqrt(3.0 * double(nb));
  }
  return IE_OK;
}

}  // namespace

int nn_predict_blocks(ie_nn* n, ie_ctx* c, Plan& B, const double* D, long d_cs, long d_bs,
                      const c128* rhs, c128* xg, int batch, hipStream_t s) {
  const long nb = B.ncell();
  IE_TRY(nn_check_shape(n, B.nz, B.ny, B.nx));
  std::vector<double> rms;
  std::vector<c128> rot;
  IE_TRY(scale_and_phase(rhs, nb, batch, n->sq, c->kw_blk, s, rms, rot));
  IE_TRY(n->x16.ensure(sizeof(u16) * 14 * nb * batch));
  double kr, ki;
  k0h(c, &kr, &ki);
  for (int b = 0; b < batch; ++b) {
    hipLaunchKernelGGL(k_features, dim3(grid1(nb)), dim3(256), 0, s, D + b * d_bs, d_cs,
                       rhs + b * 3 * nb, nb, c->med.sigma0, rms[b] > 0 ? 1.0 / rms[b] : 0.0,
                       rot[b], kr, ki, n->x16.as<u16>() + b * 14 * nb);
    IE_LAUNCH_CHECK();
  }
  IE_TRY(n->gy.ensure(sizeof(float) * 6 * nb * batch));
  IE_TRY(forward_chunked(n, n->x16.as<u16>(), batch, B.nz, B.ny, B.nx, n->gy.as<float>(), s));
  for (int b = 0; b < batch; ++b) {
    const c128 urot{rms[b] * rot[b].re, -rms[b] * rot[b].im};  // rms e^{i phi}
    hipLaunchKernelGGL(k_apply_guess, dim3(grid1(nb)), dim3(256), 0, s, rhs + b * 3 * nb,
                       n->gy.as<float>() + b * 6 * nb, nb, urot, xg + b * 3 * nb);
    IE_LAUNCH_CHECK();
  }
  return IE_OK;
}

int nn_guess_blocks(ie_nn* n, ie_ctx* c, Plan& B, const double* D, long d_cs, long d_bs,
                    const c128* rhs, c128* x, int batch, int* accepted, hipStream_t s) {
  const long nb = B.ncell();
  IE_TRY(n->xg.ensure(sizeof(c128) * 3 * nb * batch));
  IE_TRY(n->res.ensure(sizeof(c128) * 3 * nb * batch));
  c128* xg = n->xg.as<c128>();
  c128* r = n->res.as<c128>();
  IE_TRY(nn_predict_blocks(n, c, B, D, d_cs, d_bs, rhs, xg, batch, s));
  // judge: float64 residuals ||rhs - (I - G dsigma) x|| of the learned and the default guess;
  // a zero start has residual ||rhs||
  std::vector<double> bn(batch), rl(batch), rd(batch);
  IE_TRY(norms_host(rhs, 3 * nb, batch, bn.data(), c->kw_blk, s));
  OpDesc op;
  op.form = IE_CONVENTIONAL;
  op.M64 = D;
  op.M_cs = d_cs;
  op.M_bs = d_bs;
  IE_TRY(apply_op<double>(B, op, xg, r, rhs, true, batch, nullptr, 0, s, tw64(c)));
  IE_TRY(norms_host(r, 3 * nb, batch, rl.data(), c->kw_blk, s));
  IE_TRY(apply_op<double>(B, op, x, r, rhs, true, batch, nullptr, 0, s, tw64(c)));
  IE_TRY(norms_host(r, 3 * nb, batch, rd.data(), c->kw_blk, s));
  for (int b = 0; b < batch; ++b) {
    if (rl[b] < rd[b] && rl[b] < bn[b]) {
      accepted[b] = 1;
      IE_HIP(hipMemcpyAsync(x + b * 3 * nb, xg + b * 3 * nb, sizeof(c128) * 3 * nb,
                            hipMemcpyDeviceToDevice, s));
    } else if (bn[b] < rd[b]) {
      accepted[b] = 2;
      IE_HIP(hipMemsetAsync(x + b * 3 * nb, 0, sizeof(c128) * 3 * nb, s));
    } else {
      accepted[b] = 0;
    }
  }
  IE_HIP(hipStreamSynchronize(s));
  return IE_OK;
}

}  // namespace ie

extern "C" {

int ie_nn_features(ie_ctx* ctx, const double* sigma6, const void* b, uint16_t* x, double* rms,
                   void* stream) {
  if (ctx == nullptr || sigma6 == nullptr || b == nullptr || x == nullptr)
    return fail(IE_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const long N = ctx->full->ncell();
  IE_TRY(prepare_contrast(ctx, sigma6, IE_CONVENTIONAL, s));
  DevBuf sq;
  std::vector<double> r;
  std::vector<c128> rot;
  IE_TRY(scale_and_phase((const c128*)b, N, 1, sq, ctx->kw, s, r, rot));
  double kr, ki;
  k0h(ctx, &kr, &ki);
  hipLaunchKernelGGL(k_features, dim3(grid1(N)), dim3(256), 0, s, ctx->M64.as<const double>(), N,
                     (const c128*)b, N, ctx->med.sigma0, r[0] > 0 ? 1.0 / r[0] : 0.0, rot[0], kr,
                     ki, x);
  IE_LAUNCH_CHECK();
  IE_HIP(hipStreamSynchronize(s));
  if (rms) *rms = r[0];
  return IE_OK;
}

int ie_nn_target(ie_ctx* ctx, const void* b, const void* E, float* y, void* stream) {
  if (ctx == nullptr || b == nullptr || E == nullptr || y == nullptr)
    return fail(IE_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const long N = ctx->full->ncell();
  DevBuf sq;
  std::vector<double> r;
  std::vector<c128> rot;
  IE_TRY(scale_and_phase((const c128*)b, N, 1, sq, ctx->kw, s, r, rot));
  hipLaunchKernelGGL(k_target, dim3(grid1(N)), dim3(256), 0, s, (const c128*)b, (const c128*)E, N,
                     r[0] > 0 ? 1.0 / r[0] : 0.0, rot[0], y);
  IE_LAUNCH_CHECK();
  IE_HIP(hipStreamSynchronize(s));
  return IE_OK;
}

int ie_nn_predict(ie_ctx* ctx, ie_nn* n, const double* sigma6, const void* b, void* x,
                  void* stream) {
  if (ctx == nullptr || n == nullptr || sigma6 == nullptr || b == nullptr || x == nullptr)
    return fail(IE_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  Plan& F = *ctx->full;
  IE_TRY(nn_check_shape(n, F.nz, F.ny, F.nx));
  IE_TRY(prepare_contrast(ctx, sigma6, IE_CONVENTIONAL, s));
  IE_TRY(nn_predict_blocks(n, ctx, F, ctx->M64.as<const double>(), F.ncell(), 6 * F.ncell(),
                           (const c128*)b, (c128*)x, 1, s));
  IE_HIP(hipStreamSynchronize(s));
  return IE_OK;
}

int ie_nn_guess(ie_ctx* ctx, ie_nn* n, const double* sigma6, const void* b, void* x,
                int32_t* accepted, void* stream) {
  if (ctx == nullptr || n == nullptr || sigma6 == nullptr || b == nullptr || x == nullptr)
    return fail(IE_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  Plan& F = *ctx->full;
  IE_TRY(nn_check_shape(n, F.nz, F.ny, F.nx));
  IE_TRY(prepare_contrast(ctx, sigma6, IE_CONVENTIONAL, s));
  int acc = 0;
  IE_TRY(nn_guess_blocks(n, ctx, F, ctx->M64.as<const double>(), F.ncell(), 6 * F.ncell(),
                         (const c128*)b, (c128*)x, 1, &acc, s));
  if (accepted) *accepted = acc;
  return IE_OK;
}

}  // extern "C"
