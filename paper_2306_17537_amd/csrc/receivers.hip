// Magnetic field at receiver points (eqs. 4 and 6).  With eq. (5), the curl of the grad-grad
// term vanishes and G^H J = grad g(r - r') x J, grad g(R) = (i k0 R - 1) e^{i k0 R} / (4 pi R^3) R,
// so the scattered field of the cell currents dsigma E is
//     H_a(r) = h^3 sum_c grad g(r - r_c) x (dsigma E)_c
// (collocation at cell centres as for eq. 8; a receiver at a cell centre gets nothing from that
// cell, whose kernel is odd about it).  Background fields: magnetic dipole H0 = sigma0 G^E m,
// electric dipole H0 = grad g x p.
#include <cmath>
#include <vector>

#include "context.hpp"
#include "prof.hpp"

namespace ie {
namespace {

constexpr int RXB = 256;     // threads per block
constexpr int RX_MAX = 4096;

__device__ __forceinline__ c128 expik(double k0re, double k0im, double R) {
  double sn, cs;
  sincos(k0re * R, &sn, &cs);
  const double m = exp(-k0im * R);
  return c128{m * cs, m * sn};
}

// grad g(R) as a complex scalar f with grad g = f Rvec
__device__ __forceinline__ c128 grad_g_factor(double k0re, double k0im, double R) {
  const c128 e = expik(k0re, k0im, R);
  const c128 a{-k0im * R - 1.0, k0re * R};  // i k0 R - 1
  const double d = 1.0 / (4.0 * M_PI * R * R * R);
  return c128{(a.re * e.re - a.im * e.im) * d, (a.re * e.im + a.im * e.re) * d};
}

// (f Rvec) x J for complex f, real Rvec, complex J
__device__ __forceinline__ void cross_fr(c128 f, const double R[3], const c128 J[3], c128 out[3]) {
  const c128 g[3] = {c128{f.re * R[0], f.im * R[0]}, c128{f.re * R[1], f.im * R[1]},
                     c128{f.re * R[2], f.im * R[2]}};
  out[0] = g[1] * J[2] - g[2] * J[1];
  out[1] = g[2] * J[0] - g[0] * J[2];
  out[2] = g[0] * J[1] - g[1] * J[0];
}

// Partial sums of H_a over a slice of cells: block (g, receiver) -> part[(rx G + g) 6 + k]
__global__ void __launch_bounds__(RXB)
    k_rx_partial(const double* __restrict__ s6, const c128* __restrict__ E, int nx, int ny,
                 int nz, double h, double ox, double oy, double oz, double sigma0, double k0re,
                 double k0im, const double* __restrict__ rx, double* __restrict__ part) {
  const long N = long(nx) * ny * nz;
  const int q = blockIdx.y;
  const double r[3] = {rx[3 * q], rx[3 * q + 1], rx[3 * q + 2]};
  const double eps = 1e-9 * h;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (long c = long(blockIdx.x) * RXB + threadIdx.x; c < N; c += long(gridDim.x) * RXB) {
    const int i = int(c % nx), j = int((c / nx) % ny), k = int(c / (long(nx) * ny));
    const double Rv[3] = {r[0] - (ox + (i + 0.5) * h), r[1] - (oy + (j + 0.5) * h),
                          r[2] - (oz + (k + 0.5) * h)};
    const double R = sqrt(Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2]);
    if (!(R > eps)) continue;
    const double dxx = s6[c] - sigma0, dyy = s6[N + c] - sigma0, dzz = s6[2 * N + c] - sigma0;
    const double dxy = s6[3 * N + c], dxz = s6[4 * N + c], dyz = s6[5 * N + c];
    if (dxx == 0 && dyy == 0 && dzz == 0 && dxy == 0 && dxz == 0 && dyz == 0) continue;
    const c128 e0 = E[c], e1 = E[N + c], e2 = E[2 * N + c];
    const c128 J[3] = {
        c128{dxx * e0.re + dxy * e1.re + dxz * e2.re, dxx * e0.im + dxy * e1.im + dxz * e2.im},
        c128{dxy * e0.re + dyy * e1.re + dyz * e2.re, dxy * e0.im + dyy * e1.im + dyz * e2.im},
        c128{dxz * e0.re + dyz * e1.re + dzz * e2.re, dxz * e0.im + dyz * e1.im + dzz * e2.im}};
    c128 hv[3];
    cross_fr(grad_g_factor(k0re, k0im, R), Rv, J, hv);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      acc[2 * m] += hv[m].re;
      acc[2 * m + 1] += hv[m].im;
    }
  }
  // block reduction in fixed order: wave shuffles, then the wave sums in order
  __shared__ double sh[RXB / 64][6];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    double v = acc[m];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) sh[wv][m] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double v = 0;
    for (int w = 0; w < RXB / 64; ++w) v += sh[w][threadIdx.x];
    part[(long(q) * gridDim.x + blockIdx.x) * 6 + threadIdx.x] = v * h * h * h;
  }
}

struct RxSrc {
  int n;
  double pos[8][3], mom[8][3];
  int kind[8];
};

// Background magnetic field at the receivers, one thread per receiver: out[q][3]
__global__ void k_rx_background(const double* __restrict__ rx, int nrx, RxSrc sp, double sigma0,
                                double k0re, double k0im, int accumulate, c128* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nrx) return;
  c128 H[3] = {{0, 0}, {0, 0}, {0, 0}};
  if (accumulate)
    for (int m = 0; m < 3; ++m) H[m] = out[3 * q + m];
  for (int s = 0; s < sp.n; ++s) {
    const double Rv[3] = {rx[3 * q] - sp.pos[s][0], rx[3 * q + 1] - sp.pos[s][1],
                          rx[3 * q + 2] - sp.pos[s][2]};
    const double R = sqrt(Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2]);
    const double* mm = sp.mom[s];
    if (sp.kind[s] == IE_MAG_DIPOLE) {
      // sigma0 G^E m = e^{ik0R}/(4 pi R^3) [(k0^2 R^2 + i k0 R - 1) m + (3 - 3 i k0 R - k0^2 R^2)(Rh.m) Rh]
      const c128 e = expik(k0re, k0im, R);
      const c128 kR{k0re * R, k0im * R};
      const c128 kR2 = kR * kR;
      const c128 ikR{-kR.im, kR.re};
      const c128 a{kR2.re + ikR.re - 1.0, kR2.im + ikR.im};
      const c128 b{3.0 - 3.0 * ikR.re - kR2.re, -3.0 * ikR.im - kR2.im};
      const double d = 1.0 / (4.0 * M_PI * R * R * R);
      const c128 pre{e.re * d, e.im * d};
      const double rh[3] = {Rv[0] / R, Rv[1] / R, Rv[2] / R};
      const double rm = rh[0] * mm[0] + rh[1] * mm[1] + rh[2] * mm[2];
      for (int m = 0; m < 3; ++m) {
        const c128 t{a.re * mm[m] + b.re * rm * rh[m], a.im * mm[m] + b.im * rm * rh[m]};
        H[m] = H[m] + pre * t;
      }
    } else {
      const c128 J[3] = {c128{mm[0], 0}, c128{mm[1], 0}, c128{mm[2], 0}};
      c128 hv[3];
      cross_fr(grad_g_factor(k0re, k0im, R), Rv, J, hv);
      for (int m = 0; m < 3; ++m) H[m] = H[m] + hv[m];
    }
  }
  for (int m = 0; m < 3; ++m) out[3 * q + m] = H[m];
}

}  // namespace
}  // namespace ie

using namespace ie;

extern "C" int ie_receivers(ie_ctx* ctx, const double* sigma6, const ie_source* src,
                            int32_t nsrc, const void* E, const double* rx, int32_t nrx, void* H,
                            void* Ha, void* stream) {
  if (ctx == nullptr || sigma6 == nullptr || E == nullptr || rx == nullptr || H == nullptr)
    return fail(IE_EINVAL, "NULL argument");
  if (nrx < 1 || nrx > RX_MAX) return fail(IE_EINVAL, "nrx must be in [1, %d]", RX_MAX);
  if (nsrc < 0 || (nsrc > 0 && src == nullptr)) return fail(IE_EINVAL, "bad sources");
  const ie_grid& g = ctx->grid;
  for (int q = 0; q < nrx; ++q)
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(rx[3 * q + a])) return fail(IE_EINVAL, "receiver %d is not finite", q);
  for (int s = 0; s < nsrc; ++s) {
    if (src[s].kind != IE_MAG_DIPOLE && src[s].kind != IE_ELEC_DIPOLE)
      return fail(IE_EINVAL, "source %d: unknown kind", s);
    for (int q = 0; q < nrx; ++q) {
      double d2 = 0;
      for (int a = 0; a < 3; ++a) d2 += (rx[3 * q + a] - src[s].pos[a]) * (rx[3 * q + a] - src[s].pos[a]);
      if (std::sqrt(d2) <= 1e-9 * g.h) return fail(IE_EINVAL, "receiver %d is on source %d", q, s);
    }
  }
  hipStream_t s = (hipStream_t)stream;
  const long N = ctx->full->ncell();
  const int G = int(std::min<long>(256, std::max<long>(1, N / (RXB * 16))));
  DevBuf drx, part, h0;
  IE_TRY(drx.ensure(sizeof(double) * 3 * nrx));
  IE_TRY(part.ensure(sizeof(double) * 6 * G * nrx));
  IE_TRY(h0.ensure(sizeof(c128) * 3 * nrx));
  IE_HIP(hipMemcpyAsync(drx.p, rx, sizeof(double) * 3 * nrx, hipMemcpyHostToDevice, s));
  {
    ProfScope ps(s, "receivers", "", double(N) * (6 * 8 + 3 * 16) * nrx);
    hipLaunchKernelGGL(k_rx_partial, dim3(G, nrx), dim3(RXB), 0, s, sigma6, (const c128*)E, g.nx,
                       g.ny, g.nz, g.h, g.origin[0], g.origin[1], g.origin[2], ctx->med.sigma0,
                       ctx->med.k0re, ctx->med.k0im, drx.as<const double>(), part.as<double>());
    IE_LAUNCH_CHECK();
  }
  // background field, up to 8 sources per launch
  for (int s0 = 0, first = 1; s0 < std::max(nsrc, 1); s0 += 8, first = 0) {
    RxSrc sp{};
    sp.n = std::min(8, nsrc - s0);
    for (int t = 0; t < sp.n; ++t) {
      for (int a = 0; a < 3; ++a) {
        sp.pos[t][a] = src[s0 + t].pos[a];
        sp.mom[t][a] = src[s0 + t].moment[a];
      }
      sp.kind[t] = src[s0 + t].kind;
    }
    hipLaunchKernelGGL(k_rx_background, dim3(ceil_div(nrx, 64)), dim3(64), 0, s,
                       drx.as<const double>(), nrx, sp, ctx->med.sigma0, ctx->med.k0re,
                       ctx->med.k0im, first ? 0 : 1, h0.as<c128>());
    IE_LAUNCH_CHECK();
  }
  std::vector<double> hp(size_t(6) * G * nrx);
  std::vector<c128> hb(size_t(3) * nrx);
  IE_HIP(hipMemcpyAsync(hp.data(), part.p, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, s));
  IE_HIP(hipMemcpyAsync(hb.data(), h0.p, sizeof(c128) * hb.size(), hipMemcpyDeviceToHost, s));
  IE_HIP(hipStreamSynchronize(s));
  c128* Ho = (c128*)H;
  c128* Hao = (c128*)Ha;
  for (int q = 0; q < nrx; ++q)
    for (int m = 0; m < 3; ++m) {
      double re = 0, im = 0;  // fixed order over the block partials
      for (int b = 0; b < G; ++b) {
        re += hp[(size_t(q) * G + b) * 6 + 2 * m];
        im += hp[(size_t(q) * G + b) * 6 + 2 * m + 1];
      }
      if (Hao) Hao[3 * q + m] = c128{re, im};
      Ho[3 * q + m] = c128{hb[3 * q + m].re + re, hb[3 * q + m].im + im};
    }
  return IE_OK;
}
