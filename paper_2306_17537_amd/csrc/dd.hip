// Alg. 1: block Gauss-Seidel / Jacobi over z-slab sub-domains (section 2.3, eqs. 19-24), for a
// batch of problems.
//
// Per sweep and block i: the right-hand side b_i = E(i,0) + sum_{j != i} G(ij) dsigma(j) E(j)
// is one full-grid convolution whose source skips block i's planes and whose output keeps only
// block i's planes (the coupling term acts on the whole domain, as in the paper's Ex. 3); the
// block system (I - G(ii) dsigma(i)) E(i) = b_i is then solved by restarted GMRES on the
// block's own padded FFT grid, warm-started from the previous sweep, to the adaptive (e / 10)
// or fixed inner tolerance.  After each sweep the full-domain relative residual e of eq. (9)
// is recomputed in float64.
//
// Problems that share a context (same grid, partition and medium, hence the same spectra) are
// advanced together: every convolution and every block solve runs once per group with the
// problem as the batch index; each problem keeps its own e, inner tolerance and stopping, and a
// converged problem drops out (its inner tolerance becomes infinite and its coupling / residual
// convolutions are retired by its active flag).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "context.hpp"
#include "nn.hpp"
#include "prof.hpp"

namespace ie {

namespace {

__global__ void k_plane_nonzero(const double* __restrict__ D, long N, long plane,
                                int* __restrict__ flag) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  bool nz_ = false;
  for (int c = 0; c < 6; ++c) nz_ = nz_ || (D[c * N + i] != 0.0);
  if (nz_) flag[i / plane] = 1;
}

// Zero the entries of `batch` fields [3][N] (field stride 3N) in the cells whose contrast
// D [6][N] (stride 6N) is zero.
__global__ void k_mask_anomalous(c128* __restrict__ v, const double* __restrict__ D, long N) {
  const int b = blockIdx.y;
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double* d = D + b * 6 * N;
  bool nz_ = false;
  for (int c = 0; c < 6; ++c) nz_ = nz_ || (d[c * N + i] != 0.0);
  if (nz_) return;
  c128* w = v + b * 3 * N;
  for (int c = 0; c < 3; ++c) w[c * N + i] = c128{0, 0};
}

// Copy planes [z0, z0 + nzb) of `batch` fields [3][nz][ny][nx] (field stride fs, component
// stride cs) to / from contiguous blocks [3][nzb][ny][nx] (block stride 3 nb); problems whose
// mask entry is 0 are skipped.
__global__ void k_copy_blocks(const c128* __restrict__ src, c128* __restrict__ dst, long fs,
                              long cs, long plane, int z0, int nzb, int to_block,
                              const int* __restrict__ mask) {
  const long nb = long(nzb) * plane;
  const long total = 3 * nb;
  const int b = blockIdx.y;
  if (mask != nullptr && mask[b] == 0) return;
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += long(gridDim.x) * blockDim.x) {
    const int c = int(e / nb);
    const long r = e % nb;
    const long fi = b * fs + c * cs + z0 * plane + r;
    const long bi = b * total + e;
    if (to_block)
      dst[bi] = src[fi];
    else
      dst[fi] = src[bi];
  }
}

int copy_blocks(const c128* src, c128* dst, long fs, long cs, long plane, int z0, int nzb,
                bool to_block, int batch, const int* mask, hipStream_t s) {
  const long total = 3L * nzb * plane;
  dim3 grid(std::min(4096, ceil_div(total, 256)), batch);
  hipLaunchKernelGGL(k_copy_blocks, grid, dim3(256), 0, s, src, dst, fs, cs, plane, z0, nzb,
                     to_block ? 1 : 0, mask);
  IE_LAUNCH_CHECK();
  return IE_OK;
}

struct Group {
  ie_ctx* c;
  hipStream_t s;
  int B;  // problems in the group
  long N, plane;
  int form;
  // device arrays; problem stride in brackets
  double* D64;   // dsigma           [6N]
  double* M64;   // inner contrast   [6N]
  float* M32;    //                  [6N]
  double* A64;   // CIE a            [6N]
  double* Ai64;  // CIE a^-1         [6N]
  c128* E0;      //                  [3N]
  c128* E;       //                  [3N]
  c128* Eold;    //                  [3N]
  int* active;   // per problem: still sweeping
  bool anomalous_resid = false;  // e over the cells with contrast only
};

// rhs_p = e_p on block [z0, z1) + G (dsigma_p src_p) with block planes removed from the source
// (e = E0 for Alg. 1; the preconditioner input for the Krylov outer iteration)
int coupling_rhs(Group& g, const c128* src, int z0, int z1, c128* rhs, const c128* e = nullptr) {
  Plan& F = *g.c->full;
  MvArgs<double> a{};
  a.x = src;
  a.x_cs = g.N;
  a.x_bs = 3 * g.N;
  a.M = g.D64;
  a.M_cs = g.N;
  a.M_bs = 6 * g.N;
  a.src_z0 = 0;
  a.src_z1 = F.nz;
  a.hole_z0 = z0;
  a.hole_z1 = z1;
  a.out_z0 = z0;
  a.out_z1 = z1;
  a.y = rhs;
  a.y_cs = long(z1 - z0) * g.plane;
  a.y_bs = 3 * a.y_cs;
  a.y_zoff = z0;
  a.e = e ? e : g.E0;
  a.e_cs = g.N;
  a.e_bs = 3 * g.N;
  a.e_zoff = 0;
  a.a_e = 1;
  a.a_x = 0;
  a.a_m = 0;
  a.a_s = 1;
  a.active = g.active;
  a.active_bs = 1;
  return launch_matvec<double>(F, a, g.B, g.s, tw64(g.c));
}

// e_p = ||E0_p - (I - G dsigma_p) E_p|| / ||E0_p|| on the full grid, all problems
int full_relres(Group& g, const double* e0norm, double* e) {
  Plan& F = *g.c->full;
  IE_TRY(g.c->tmp.ensure(sizeof(c128) * 3 * g.N * g.B));
  OpDesc op;
  op.form = IE_CONVENTIONAL;
  op.M64 = g.D64;
  op.M_cs = g.N;
  op.M_bs = 6 * g.N;
  IE_TRY(apply_op<double>(F, op, g.E, g.c->tmp.as<c128>(), g.E0, true, g.B, nullptr, 0, g.s,
                          tw64(g.c)));
  if (g.anomalous_resid) {
    hipLaunchKernelGGL(k_mask_anomalous, dim3(ceil_div(g.N, 256), g.B), dim3(256), 0, g.s,
                       g.c->tmp.as<c128>(), g.D64, g.N);
    IE_LAUNCH_CHECK();
  }
  std::vector<double> nr(g.B);
  IE_TRY(norms_host(g.c->tmp.as<c128>(), 3 * g.N, g.B, nr.data(), g.c->kw, g.s));
  for (int b = 0; b < g.B; ++b) e[b] = e0norm[b] > 0 ? nr[b] / e0norm[b] : 0.0;
  return IE_OK;
}

// Solve block [z0, z0 + nzb) of every problem (rhs, x contiguous, block stride 3 nb).
int block_solve(Group& g, Plan& B, int z0, c128* rhs, c128* x, const double* tols,
                const ie_gmres_opts& inner, GmResult* res) {
  const long nb = B.ncell();
  const long off = long(z0) * g.plane;
  OpDesc op;
  op.form = g.form;
  op.sigma0 = g.c->med.sigma0;
  op.M64 = g.M64 + off;
  op.M32 = g.M32 + off;
  op.M_cs = g.N;
  op.M_bs = 6 * g.N;
  GmOpts o;
  o.tols = tols;
  o.restart = inner.restart;
  o.max_its = inner.max_its;
  o.precision = inner.precision;
  o.reorth = inner.reorth == 2 ? 1 : 0;
  if (g.form == IE_CIE) {
    // C e = sqrt(sigma0) b_i, e = a x;  x = a^-1 e, per block
    IE_TRY(g.c->blk_rhs2.ensure(sizeof(c128) * 3 * nb * g.B));
    IE_TRY(g.c->blk_save.ensure(sizeof(c128) * 3 * nb * g.B));
    c128* rs = g.c->blk_rhs2.as<c128>();
    c128* xt = g.c->blk_save.as<c128>();
    IE_TRY(launch_scale(rhs, rs, std::sqrt(g.c->med.sigma0), 3 * nb * g.B, g.s));
    for (int b = 0; b < g.B; ++b)
      IE_TRY(launch_tensor_apply(g.A64 + b * 6 * g.N + off, g.N, x + b * 3 * nb, nb,
                                 xt + b * 3 * nb, nb, nb, g.s));
    IE_TRY(gmres_solve(B, op, rs, xt, g.B, o, res, g.c->kw_blk, tw64(g.c), tw32(g.c), g.s));
    for (int b = 0; b < g.B; ++b)
      IE_TRY(launch_tensor_apply(g.Ai64 + b * 6 * g.N + off, g.N, xt + b * 3 * nb, nb,
                                 x + b * 3 * nb, nb, nb, g.s));
    return IE_OK;
  }
  return gmres_solve(B, op, rhs, x, g.B, o, res, g.c->kw_blk, tw64(g.c), tw32(g.c), g.s);
}

// ---------------------------------------------------------------------------------------
// Krylov outer iteration (the improvement the conclusions propose): flexible GMRES on the
// full-domain eq. (8), right-preconditioned by one sweep of Alg. 1 from zero with inner solves to
// a fixed tolerance.  Outer vectors and scalars in float64; the Hessenberg matrix, rotations and
// back substitution on the host (one problem at a time, at most IE_MAX_SWEEPS outer steps).
// ---------------------------------------------------------------------------------------
constexpr int LCMAX = MAXM + 1;  // vectors in one linear combination
struct Coefs {
  c128 c[LCMAX];
};

// out = alpha out + sum_{i < count} c_i V_i  (V_i = V + i vs; none of them aliases out)
__global__ void k_lincomb(c128* __restrict__ out, double alpha, const c128* __restrict__ V,
                          long vs, int count, Coefs cf, long n) {
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
       e += long(gridDim.x) * blockDim.x) {
    c128 acc = alpha == 0.0 ? c128{0, 0} : c128{alpha * out[e].re, alpha * out[e].im};
    for (int i = 0; i < count; ++i) acc = acc + cf.c[i] * V[i * vs + e];
    out[e] = acc;
  }
}

// partials of <V_i, w> (conjugate-linear in V_i): part[(2 i + re/im) G + block], fixed order
__global__ void __launch_bounds__(256) k_dots(const c128* __restrict__ V, long vs, int count,
                                              const c128* __restrict__ w, long n,
                                              double* __restrict__ part) {
  __shared__ double sh[4][2 * LCMAX];
  double acc[2 * LCMAX];
  for (int k = 0; k < 2 * LCMAX; ++k) acc[k] = 0;
  for (long e = long(blockIdx.x) * 256 + threadIdx.x; e < n; e += long(gridDim.x) * 256) {
    const c128 x = w[e];
    for (int i = 0; i < count; ++i) {
      const c128 v = V[i * vs + e];
      acc[2 * i] += v.re * x.re + v.im * x.im;
      acc[2 * i + 1] += v.re * x.im - v.im * x.re;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k = 0; k < 2 * count; ++k) {
    double v = acc[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) sh[wv][k] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 2 * count; k += 256)
    part[long(k) * gridDim.x + blockIdx.x] = sh[0][k] + sh[1][k] + sh[2][k] + sh[3][k];
}

int lincomb(c128* out, double alpha, const c128* V, long vs, int count, const c128* c, long n,
            hipStream_t s) {
  if (count > LCMAX) return fail(IE_EINVAL, "too many vectors in a combination");
  Coefs cf{};
  for (int i = 0; i < count; ++i) cf.c[i] = c[i];
  hipLaunchKernelGGL(k_lincomb, dim3(int(std::min<long>(4096, ceil_div(n, 256)))), dim3(256), 0, s,
                     out, alpha, V, vs, count, cf, n);
  IE_LAUNCH_CHECK();
  return IE_OK;
}

int dots_host(const c128* V, long vs, int count, const c128* w, long n, DevBuf& part,
              std::vector<c128>& out, hipStream_t s) {
  const int G = int(std::min<long>(512, std::max<long>(1, n / 2048)));
  IE_TRY(part.ensure(sizeof(double) * 2 * LCMAX * G));
  hipLaunchKernelGGL(k_dots, dim3(G), dim3(256), 0, s, V, vs, count, w, n, part.as<double>());
  IE_LAUNCH_CHECK();
  std::vector<double> h(size_t(2) * count * G);
  IE_HIP(hipMemcpyAsync(h.data(), part.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  IE_HIP(hipStreamSynchronize(s));
  out.assign(count, c128{0, 0});
  for (int i = 0; i < count; ++i) {
    double re = 0, im = 0;
    for (int b = 0; b < G; ++b) {
      re += h[size_t(2 * i) * G + b];
      im += h[size_t(2 * i + 1) * G + b];
    }
    out[i] = c128{re, im};
  }
  return IE_OK;
}

// z = P^-1 v: one sweep of Alg. 1 on A z = v from z = 0 (GS: blocks in order, each coupled to
// the blocks already updated; Jacobi: block diagonal).  One problem (g.B == 1).
int dd_precondition(Group& g, const std::vector<int>& has, const c128* v, c128* z, bool gs,
                    const ie_gmres_opts& inner, double itol, c128* rhs, c128* xb,
                    int* block_its, int* inner_its, int* mv64, int* mv32, int* full_mv) {
  ie_ctx* c = g.c;
  const int M = int(c->zb.size()) - 1;
  IE_HIP(hipMemsetAsync(z, 0, sizeof(c128) * 3 * g.N, g.s));
  for (int i = 0; i < M; ++i) {
    const int z0 = c->zb[i], z1 = c->zb[i + 1], nzb = z1 - z0;
    const long nb = long(nzb) * g.plane;
    if (gs && i > 0) {
      IE_TRY(coupling_rhs(g, z, z0, z1, rhs, v));
      *full_mv += 1;
      *mv64 += 1;
    } else {
      IE_TRY(copy_blocks(v, rhs, 3 * g.N, g.N, g.plane, z0, nzb, true, 1, nullptr, g.s));
    }
    const c128* from = rhs;
    if (has[i]) {
      IE_HIP(hipMemsetAsync(xb, 0, sizeof(c128) * 3 * nb, g.s));
      GmResult r{};
      const double t = itol;
      IE_TRY(block_solve(g, *c->block_plan(nzb), z0, rhs, xb, &t, inner, &r));
      block_its[i] = r.its;
      *inner_its += r.its;
      *mv64 += r.mv64;
      *mv32 += r.mv32;
      from = xb;
    } else {
      block_its[i] = 0;
    }
    IE_TRY(copy_blocks(from, z, 3 * g.N, g.N, g.plane, z0, nzb, false, 1, nullptr, g.s));
  }
  return IE_OK;
}

// Flexible GMRES(m) for one problem of the group: x = g.E (initial guess in, solution out).
int fgmres_one(Group& g, const std::vector<int>& has, const ie_dd_opts& o, double bnorm,
               ie_dd_stats& st, double* e_out, c128* rhs, c128* xb, DdBufs& bufs) {
  ie_ctx* c = g.c;
  Plan& F = *c->full;
  const int M = int(c->zb.size()) - 1;
  const int m = o.inner.restart;
  const long n = 3 * g.N;
  const bool gs = o.scheme == IE_FGMRES_GS;
  IE_TRY(bufs.fv.ensure(sizeof(c128) * n * (m + 1)));
  IE_TRY(bufs.fz.ensure(sizeof(c128) * n * m));
  IE_TRY(bufs.fw.ensure(sizeof(c128) * n));
  c128* V = bufs.fv.as<c128>();
  c128* Z = bufs.fz.as<c128>();
  c128* w = bufs.fw.as<c128>();
  OpDesc op;
  op.form = IE_CONVENTIONAL;
  op.M64 = g.D64;
  op.M_cs = g.N;
  op.M_bs = 6 * g.N;
  const double itol = o.inner_tol_fixed;
  int outer = 0;
  double e = 0;
  auto sat = [](c128 a) { return std::sqrt(a.re * a.re + a.im * a.im); };
  while (true) {
    // true residual r = E0 - A x, beta = ||r||
    IE_TRY(apply_op<double>(F, op, g.E, w, g.E0, true, 1, nullptr, 0, g.s, tw64(c)));
    double beta = 0;
    IE_TRY(norms_host(w, n, 1, &beta, c->kw, g.s));
    st.full_matvecs += 1;
    st.matvecs64 += 1;
    e = bnorm > 0 ? beta / bnorm : 0.0;
    if (outer == 0) st.relres[0] = e;
    if (e <= o.tol || outer >= o.max_sweeps || beta == 0) break;
    const c128 ib{1.0 / beta, 0};
    IE_TRY(lincomb(V, 0.0, w, 0, 1, &ib, n, g.s));
    std::vector<std::vector<c128>> H(m + 1, std::vector<c128>(m, c128{0, 0}));
    std::vector<c128> cs(m), sn(m), gv(m + 1, c128{0, 0});
    gv[0] = c128{beta, 0};
    int k = 0;
    for (int j = 0; j < m && outer < o.max_sweeps; ++j) {
      c128* vj = V + j * n;
      c128* zj = Z + j * n;
      int inner_its = 0;
      IE_TRY(dd_precondition(g, has, vj, zj, gs, o.inner, itol, rhs, xb, st.block_its[outer],
                             &inner_its, &st.matvecs64, &st.matvecs32, &st.full_matvecs));
      st.total_its += inner_its;
      IE_TRY(apply_op<double>(F, op, zj, w, nullptr, false, 1, nullptr, 0, g.s, tw64(c)));
      st.full_matvecs += 1;
      st.matvecs64 += 1;
      // classical Gram-Schmidt, two passes
      std::vector<c128> h(j + 1, c128{0, 0}), hp;
      for (int pass = 0; pass < 2; ++pass) {
        IE_TRY(dots_host(V, n, j + 1, w, n, bufs.fpart, hp, g.s));
        std::vector<c128> neg(j + 1);
        for (int i = 0; i <= j; ++i) {
          h[i] = h[i] + hp[i];
          neg[i] = c128{-hp[i].re, -hp[i].im};
        }
        IE_TRY(lincomb(w, 1.0, V, n, j + 1, neg.data(), n, g.s));
      }
      double hn = 0;
      IE_TRY(norms_host(w, n, 1, &hn, c->kw, g.s));
      for (int i = 0; i <= j; ++i) H[i][j] = h[i];
      H[j + 1][j] = c128{hn, 0};
      for (int i = 0; i < j; ++i) {  // previous rotations, Q = [[conj c, conj s], [-s, c]]
        const c128 t = cjmul(cs[i], H[i][j]) + cjmul(sn[i], H[i + 1][j]);
        H[i + 1][j] = c128{0, 0} - sn[i] * H[i][j] + cs[i] * H[i + 1][j];
        H[i][j] = t;
      }
      const double hjj = sat(H[j][j]);
      const double den = std::sqrt(hjj * hjj + hn * hn);
      if (den == 0.0) {
        cs[j] = c128{1, 0};
        sn[j] = c128{0, 0};
      } else {
        cs[j] = c128{H[j][j].re / den, H[j][j].im / den};
        sn[j] = c128{hn / den, 0};
      }
      H[j][j] = c128{den, 0};
      gv[j + 1] = c128{0, 0} - sn[j] * gv[j];
      gv[j] = cjmul(cs[j], gv[j]);
      k = j + 1;
      outer += 1;
      st.sweeps = outer;
      const double est = bnorm > 0 ? sat(gv[j + 1]) / bnorm : 0.0;
      st.relres[outer] = est;
      if (est <= o.tol || den == 0.0 || hn == 0.0) break;
      const c128 ih{1.0 / hn, 0};
      IE_TRY(lincomb(V + (j + 1) * n, 0.0, w, 0, 1, &ih, n, g.s));
    }
    // y = R^-1 g, x += Z y
    std::vector<c128> y(k);
    for (int i = k - 1; i >= 0; --i) {
      c128 acc = gv[i];
      for (int l = i + 1; l < k; ++l) acc = acc - H[i][l] * y[l];
      const c128 d = H[i][i];
      const double dd = d.re * d.re + d.im * d.im;
      y[i] = dd > 0 ? c128{(acc.re * d.re + acc.im * d.im) / dd, (acc.im * d.re - acc.re * d.im) / dd}
                    : c128{0, 0};
    }
    if (k > 0) IE_TRY(lincomb(g.E, 1.0, Z, n, k, y.data(), n, g.s));
  }
  st.relres[std::min(outer, IE_MAX_SWEEPS)] = e;
  *e_out = e;
  return IE_OK;
}

int check_problem(ie_ctx* c, const ie_problem& pr) {
  const ie_grid& g = c->grid;
  if (pr.grid) {
    const ie_grid& q = *pr.grid;
    if (q.nx != g.nx || q.ny != g.ny || q.nz != g.nz || q.h != g.h || q.origin[0] != g.origin[0] ||
        q.origin[1] != g.origin[1] || q.origin[2] != g.origin[2])
      return fail(IE_EINVAL, "problem grid differs from its context grid");
  }
  if (pr.E_total == nullptr || pr.sigma6 == nullptr)
    return fail(IE_EINVAL, "E_total or sigma6 is NULL");
  return check_sources(c, pr.sources, pr.nsources);
}

// *worst after a group: IE_OK, IE_ENOCONV (sweeps or iterations exhausted) or kDiverged
constexpr int kDiverged = 2;

int dd_group(ie_ctx* c, const std::vector<int>& idx, const ie_problem* problems,
             const ie_dd_opts& o, ie_dd_stats* stats, hipStream_t s, int* worst) {
  const auto t0 = std::chrono::steady_clock::now();
  if (c->zb.empty()) return fail(IE_ESTATE, "context was set up without a partition");
  const int B = int(idx.size());
  for (int b = 0; b < B; ++b) {
    IE_TRY(check_problem(c, problems[idx[b]]));
    std::memset(&stats[idx[b]], 0, sizeof(ie_dd_stats));
  }
  const int form = o.inner.form;
  const ie_grid& gr = c->grid;
  Plan& F = *c->full;
  const long N = F.ncell();
  const long plane = long(gr.nx) * gr.ny;
  const int M = int(c->zb.size()) - 1;
  DdBufs& gb = c->dd;
  IE_TRY(gb.D64.ensure(sizeof(double) * 6 * N * B));
  IE_TRY(gb.M64.ensure(sizeof(double) * 6 * N * B));
  IE_TRY(gb.M32.ensure(sizeof(float) * 6 * N * B));
  if (form == IE_CIE) {
    IE_TRY(gb.A64.ensure(sizeof(double) * 6 * N * B));
    IE_TRY(gb.Ai64.ensure(sizeof(double) * 6 * N * B));
  }
  IE_TRY(gb.E0.ensure(sizeof(c128) * 3 * N * B));
  IE_TRY(gb.E.ensure(sizeof(c128) * 3 * N * B));
  if (o.scheme == IE_JACOBI) IE_TRY(gb.Eold.ensure(sizeof(c128) * 3 * N * B));
  IE_TRY(gb.active.ensure(sizeof(int) * B));
  IE_TRY(gb.flags.ensure(sizeof(int) * gr.nz * B));
  IE_TRY(gb.bad.ensure(sizeof(int)));
  Group g;
  g.c = c;
  g.s = s;
  g.B = B;
  g.N = N;
  g.plane = plane;
  g.form = form;
  g.D64 = gb.D64.as<double>();
  g.M64 = gb.M64.as<double>();
  g.M32 = gb.M32.as<float>();
  g.A64 = gb.A64.as<double>();
  g.Ai64 = gb.Ai64.as<double>();
  g.E0 = gb.E0.as<c128>();
  g.E = gb.E.as<c128>();
  g.Eold = gb.Eold.as<c128>();
  g.active = gb.active.as<int>();

  // contrast tensors (dsigma for coupling / residual; the inner form for block operators),
  // background fields, initial guesses, and which blocks carry contrast
  IE_HIP(hipMemsetAsync(gb.bad.p, 0, sizeof(int), s));
  IE_HIP(hipMemsetAsync(gb.flags.p, 0, sizeof(int) * gr.nz * B, s));
  for (int b = 0; b < B; ++b) {
    const ie_problem& pr = problems[idx[b]];
    IE_TRY(launch_prep(pr.sigma6, N, c->med.sigma0, IE_CONVENTIONAL, g.D64 + b * 6 * N,
                       form == IE_CIE ? nullptr : g.M32 + b * 6 * N, nullptr, nullptr,
                       gb.bad.as<int>(), s));
    if (form == IE_CIE)
      IE_TRY(launch_prep(pr.sigma6, N, c->med.sigma0, IE_CIE, g.M64 + b * 6 * N,
                         g.M32 + b * 6 * N, g.A64 + b * 6 * N, g.Ai64 + b * 6 * N,
                         gb.bad.as<int>(), s));
    else
      IE_HIP(hipMemcpyAsync(g.M64 + b * 6 * N, g.D64 + b * 6 * N, sizeof(double) * 6 * N,
                            hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_plane_nonzero, dim3(ceil_div(N, 256)), dim3(256), 0, s,
                       g.D64 + b * 6 * N, N, plane, gb.flags.as<int>() + b * gr.nz);
    IE_LAUNCH_CHECK();
    IE_TRY(launch_background(gr.nx, gr.ny, gr.nz, gr.h, gr.origin, c->med, pr.sources,
                             pr.nsources, g.E0 + b * 3 * N, s));
    if (o.init == IE_INIT_ZERO || o.init == IE_INIT_LEARNED) {
      IE_HIP(hipMemsetAsync(g.E + b * 3 * N, 0, sizeof(c128) * 3 * N, s));
    } else {
      const c128* init = o.init == IE_INIT_USER ? (const c128*)pr.E_total : g.E0 + b * 3 * N;
      IE_HIP(hipMemcpyAsync(g.E + b * 3 * N, init, sizeof(c128) * 3 * N,
                            hipMemcpyDeviceToDevice, s));
    }
  }
  int bad = 0;
  std::vector<int> pflag(size_t(gr.nz) * B);
  IE_HIP(hipMemcpyAsync(&bad, gb.bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  IE_HIP(hipMemcpyAsync(pflag.data(), gb.flags.p, sizeof(int) * gr.nz * B,
                        hipMemcpyDeviceToHost, s));
  IE_HIP(hipStreamSynchronize(s));
  if (bad) return fail(IE_EINVAL, "sigma6 holds a non-finite or non-positive-definite tensor");
  std::vector<std::vector<int>> has(B, std::vector<int>(M, 0));
  for (int b = 0; b < B; ++b)
    for (int i = 0; i < M; ++i)
      for (int z = c->zb[i]; z < c->zb[i + 1]; ++z) has[b][i] |= pflag[size_t(b) * gr.nz + z];

  std::vector<double> e0norm(B), e(B);
  g.anomalous_resid = o.residual_cells == IE_RESID_ANOMALOUS;
  if (g.anomalous_resid) {  // ||E0|| over the cells with contrast
    IE_TRY(c->tmp.ensure(sizeof(c128) * 3 * N * B));
    IE_HIP(hipMemcpyAsync(c->tmp.p, g.E0, sizeof(c128) * 3 * N * B, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_mask_anomalous, dim3(ceil_div(N, 256), B), dim3(256), 0, s,
                       c->tmp.as<c128>(), g.D64, N);
    IE_LAUNCH_CHECK();
    IE_TRY(norms_host(c->tmp.as<c128>(), 3 * N, B, e0norm.data(), c->kw, s));
  } else {
    IE_TRY(norms_host(g.E0, 3 * N, B, e0norm.data(), c->kw, s));
  }
  IE_TRY(full_relres(g, e0norm.data(), e.data()));
  std::vector<int> act(B), sweeps(B, 0);
  for (int b = 0; b < B; ++b) {
    ie_dd_stats& st = stats[idx[b]];
    st.nblocks = M;
    st.full_matvecs += 1;
    st.matvecs64 += 1;
    st.relres[0] = e[b];
    act[b] = e[b] > o.tol;
  }
  long maxb = 0;
  for (int i = 0; i < M; ++i) maxb = std::max(maxb, long(c->zb[i + 1] - c->zb[i]) * plane);
  IE_TRY(gb.rhs.ensure(sizeof(c128) * 3 * maxb * B));
  IE_TRY(gb.x.ensure(sizeof(c128) * 3 * maxb * B));
  c128* rhs = gb.rhs.as<c128>();
  c128* x = gb.x.as<c128>();
  if (o.scheme == IE_FGMRES_GS || o.scheme == IE_FGMRES_JACOBI) {
    // Krylov outer iteration, one problem at a time (its vectors and Hessenberg are per problem)
    for (int b = 0; b < B; ++b) {
      if (!act[b]) continue;
      Group g1 = g;
      g1.B = 1;
      g1.D64 = g.D64 + b * 6 * N;
      g1.M64 = g.M64 + b * 6 * N;
      g1.M32 = g.M32 + b * 6 * N;
      g1.A64 = g.A64 + b * 6 * N;
      g1.Ai64 = g.Ai64 + b * 6 * N;
      g1.E0 = g.E0 + b * 3 * N;
      g1.E = g.E + b * 3 * N;
      g1.active = g.active + b;
      IE_HIP(hipMemcpyAsync(g1.active, &act[b], sizeof(int), hipMemcpyHostToDevice, s));
      IE_TRY(fgmres_one(g1, has[b], o, e0norm[b], stats[idx[b]], &e[b], rhs, x, gb));
    }
  } else {
    std::vector<double> tols(B);
    std::vector<GmResult> res(B);
    std::vector<GmResult> pre(B);  // the judge's cycles in the first sweep of a learned start
    const double inf = std::numeric_limits<double>::infinity();
    bool first = true;
    // The sweeps converge only when the block splitting contracts (section 2.3: diagonal
    // dominance); the iterate of smallest full residual is kept, and a problem whose residual
    // grows in two consecutive sweeps is stopped.
    IE_TRY(gb.best.ensure(sizeof(c128) * 3 * N * B));
    c128* best = gb.best.as<c128>();
    std::vector<double> best_e(e);
    IE_HIP(hipMemcpyAsync(best, g.E, sizeof(c128) * 3 * N * B, hipMemcpyDeviceToDevice, s));

    while (true) {
      bool any = false;
      for (int b = 0; b < B; ++b) {
        if (act[b] && sweeps[b] >= o.max_sweeps) act[b] = 0;  // out of sweeps: reported below
        any = any || act[b];
      }
      if (!any) break;
      IE_HIP(hipMemcpyAsync(g.active, act.data(), sizeof(int) * B, hipMemcpyHostToDevice, s));
      const c128* src = g.E;
      if (o.scheme == IE_JACOBI) {
        IE_HIP(hipMemcpyAsync(g.Eold, g.E, sizeof(c128) * 3 * N * B, hipMemcpyDeviceToDevice, s));
        src = g.Eold;
      }
      for (int i = 0; i < M; ++i) {
        const int z0 = c->zb[i], z1 = c->zb[i + 1], nzb = z1 - z0;
        const long nb = long(nzb) * plane;
        IE_TRY(coupling_rhs(g, src, z0, z1, rhs));
        // warm start from the previous sweep (for Jacobi src = E at sweep k; for GS block i of E
        // has not been updated yet in this sweep either)
        IE_TRY(copy_blocks(src, x, 3 * N, N, plane, z0, nzb, true, B, g.active, s));
        bool solve = false;
        for (int b = 0; b < B; ++b) {
          const bool live = act[b] && has[b][i];
          tols[b] = live ? (o.adaptive ? e[b] / 10.0 : o.inner_tol_fixed) : inf;
          solve = solve || live;
        }
        std::fill(pre.begin(), pre.end(), GmResult{});
        if (solve && first && o.init == IE_INIT_LEARNED) {
          // first sweep: one restart cycle of GMRES from the learned guess and one from the
          // default start; each block continues from whichever reached the smaller residual
          Plan& BP = *c->block_plan(nzb);
          IE_TRY(gb.xl.ensure(sizeof(c128) * 3 * nb * B));
          c128* xl = gb.xl.as<c128>();
          IE_TRY(nn_predict_blocks((ie_nn*)o.nn, c, BP, g.D64 + long(z0) * plane, N, 6 * N, rhs, xl,
                                   B, s));
          ie_gmres_opts one = o.inner;
          one.max_its = o.inner.restart;
          std::vector<GmResult> rl(B), rd(B);
          IE_TRY(block_solve(g, BP, z0, rhs, xl, tols.data(), one, rl.data()));
          IE_TRY(block_solve(g, BP, z0, rhs, x, tols.data(), one, rd.data()));
          for (int b = 0; b < B; ++b) {
            if (!(act[b] && has[b][i])) continue;
            pre[b].its = rl[b].its + rd[b].its;
            pre[b].mv64 = rl[b].mv64 + rd[b].mv64;
            pre[b].mv32 = rl[b].mv32 + rd[b].mv32;
            pre[b].graph_cycles = rl[b].graph_cycles + rd[b].graph_cycles;
            if (rl[b].relres < rd[b].relres) {
              stats[idx[b]].learned_used += 1;
              IE_HIP(hipMemcpyAsync(x + b * 3 * nb, xl + b * 3 * nb, sizeof(c128) * 3 * nb,
                                    hipMemcpyDeviceToDevice, s));
            }
          }
        }
        if (solve)
          IE_TRY(block_solve(g, *c->block_plan(nzb), z0, rhs, x, tols.data(), o.inner, res.data()));
        for (int b = 0; b < B; ++b) {
          if (!act[b]) continue;
          // blocks without contrast have A_ii = I: E(i) = b_i
          const c128* from = has[b][i] ? x + b * 3 * nb : rhs + b * 3 * nb;
          for (int cc = 0; cc < 3; ++cc)
            IE_HIP(hipMemcpyAsync(g.E + b * 3 * N + cc * N + z0 * plane, from + cc * nb,
                                  sizeof(c128) * nb, hipMemcpyDeviceToDevice, s));
          ie_dd_stats& st = stats[idx[b]];
          st.full_matvecs += 1;
          st.matvecs64 += 1;
          if (has[b][i]) {
            st.block_its[sweeps[b]][i] = res[b].its + pre[b].its;
            st.matvecs64 += res[b].mv64 + pre[b].mv64;
            st.matvecs32 += res[b].mv32 + pre[b].mv32;
            st.graph_cycles += res[b].graph_cycles + pre[b].graph_cycles;
          }
        }
      }
      first = false;
      IE_TRY(full_relres(g, e0norm.data(), e.data()));
      for (int b = 0; b < B; ++b) {
        if (!act[b]) continue;
        ie_dd_stats& st = stats[idx[b]];
        for (int i = 0; i < M; ++i) st.total_its += st.block_its[sweeps[b]][i];
        sweeps[b] += 1;
        const int k = sweeps[b];
        st.sweeps = k;
        st.relres[k] = e[b];
        st.full_matvecs += 1;
        st.matvecs64 += 1;
        if (e[b] < best_e[b]) {
          best_e[b] = e[b];
          st.best_sweep = k;
          IE_HIP(hipMemcpyAsync(best + b * 3 * N, g.E + b * 3 * N, sizeof(c128) * 3 * N,
                                hipMemcpyDeviceToDevice, s));
        }
        if (e[b] <= o.tol) {
          act[b] = 0;
        } else if (k >= 2 && st.relres[k] > st.relres[k - 1] &&
                   st.relres[k - 1] > st.relres[k - 2]) {
          act[b] = 0;
          st.diverged = 1;
        }
      }
    }
    // a problem that did not reach the tolerance returns its iterate of smallest residual
    for (int b = 0; b < B; ++b) {
      if (e[b] <= o.tol || best_e[b] >= e[b]) continue;
      e[b] = best_e[b];
      IE_HIP(hipMemcpyAsync(g.E + b * 3 * N, best + b * 3 * N, sizeof(c128) * 3 * N,
                            hipMemcpyDeviceToDevice, s));
    }
  }  // stationary sweeps
  // outputs
  for (int b = 0; b < B; ++b) {
    const ie_problem& pr = problems[idx[b]];
    IE_HIP(hipMemcpyAsync(pr.E_total, g.E + b * 3 * N, sizeof(c128) * 3 * N,
                          hipMemcpyDeviceToDevice, s));
    if (pr.E_anom)
      IE_TRY(launch_sub(g.E + b * 3 * N, g.E0 + b * 3 * N, (c128*)pr.E_anom, 3 * N, s));
  }
  IE_HIP(hipStreamSynchronize(s));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int b = 0; b < B; ++b) {
    stats[idx[b]].seconds = secs;
    if (e[b] > o.tol) *worst = std::max(*worst, stats[idx[b]].diverged ? kDiverged : IE_ENOCONV);
  }
  return IE_OK;
}

}  // namespace
}  // namespace ie

using namespace ie;

extern "C" int ie_dd_solve(ie_ctx* const* ctxs, int32_t nproblems, const ie_problem* problems,
                           const ie_dd_opts* opts, ie_dd_stats* stats, void* stream) {
  if (ctxs == nullptr || problems == nullptr || opts == nullptr || nproblems < 1)
    return fail(IE_EINVAL, "NULL argument or no problems");
  const ie_dd_opts& o = *opts;
  if (!(o.tol >= 0)) return fail(IE_EINVAL, "bad tol");
  if (o.scheme != IE_GS && o.scheme != IE_JACOBI && o.scheme != IE_FGMRES_GS &&
      o.scheme != IE_FGMRES_JACOBI)
    return fail(IE_EINVAL, "bad scheme");
  const bool krylov = o.scheme == IE_FGMRES_GS || o.scheme == IE_FGMRES_JACOBI;
  if (krylov && o.init == IE_INIT_LEARNED)
    return fail(IE_EINVAL, "the learned start applies to the stationary sweeps only");
  if (krylov && !(o.inner_tol_fixed > 0))
    return fail(IE_EINVAL, "the Krylov outer iteration needs inner_tol_fixed > 0");
  if (o.residual_cells != IE_RESID_ALL && o.residual_cells != IE_RESID_ANOMALOUS)
    return fail(IE_EINVAL, "bad residual_cells");
  if (krylov && o.residual_cells != IE_RESID_ALL)
    return fail(IE_EINVAL, "the Krylov outer iteration minimises the residual over all cells");
  if (o.inner.form != IE_CONVENTIONAL && o.inner.form != IE_CIE)
    return fail(IE_EINVAL, "bad inner form");
  if (o.inner.precision != IE_FP64 && o.inner.precision != IE_MIXED)
    return fail(IE_EINVAL, "bad inner precision");
  if (o.inner.reorth < 0 || o.inner.reorth > 2) return fail(IE_EINVAL, "bad reorth");
  if (o.inner.restart < 1 || o.inner.restart > MAXM)
    return fail(IE_EINVAL, "restart must be in [1, %d]", MAXM);
  if (o.inner.max_its < 1) return fail(IE_EINVAL, "max_its must be >= 1");
  if (o.max_sweeps < 1 || o.max_sweeps > IE_MAX_SWEEPS)
    return fail(IE_EINVAL, "max_sweeps must be in [1, %d]", IE_MAX_SWEEPS);
  if (o.init == IE_INIT_LEARNED && o.nn == nullptr)
    return fail(IE_EINVAL, "learned initial guess needs an ie_nn handle");
  if (o.init != IE_INIT_BACKGROUND && o.init != IE_INIT_USER && o.init != IE_INIT_LEARNED &&
      o.init != IE_INIT_ZERO)
    return fail(IE_EINVAL, "bad init");
  if (!(o.adaptive == 0 || o.adaptive == 1)) return fail(IE_EINVAL, "adaptive must be 0 or 1");
  for (int p = 0; p < nproblems; ++p) {
    if (ctxs[p] == nullptr) return fail(IE_EINVAL, "context %d is NULL", p);
    if (!(ctxs[p]->prec_mask & o.inner.precision) || !(ctxs[p]->prec_mask & IE_FP64))
      return fail(IE_EINVAL, "context %d lacks the spectra this precision needs", p);
    if (o.init == IE_INIT_LEARNED) {
      const ie_ctx* c = ctxs[p];
      for (size_t i = 0; i + 1 < c->zb.size(); ++i)
        IE_TRY(nn_check_shape((const ie_nn*)o.nn, c->zb[i + 1] - c->zb[i], c->grid.ny,
                              c->grid.nx));
    }
  }
  std::vector<ie_dd_stats> local;
  if (stats == nullptr) {
    local.resize(nproblems);
    stats = local.data();
  }
  // group the problems by context (same spectra), in order of first appearance
  std::vector<ie_ctx*> order;
  std::map<ie_ctx*, std::vector<int>> groups;
  for (int p = 0; p < nproblems; ++p) {
    if (!groups.count(ctxs[p])) order.push_back(ctxs[p]);
    groups[ctxs[p]].push_back(p);
  }
  hipStream_t s = (hipStream_t)stream;
  int worst = IE_OK;
  // Groups of different contexts share no device buffers, so they may run at the same time: one
  // host thread and one stream per group, ordered after and before the caller's stream by events
  // (small groups then fill the GPU together).  Kept sequential for a single group, a shared
  // network handle, an active launch profiler or IE_OPT_GROUP_THREADS = 0.
  if (order.size() == 1 || o.init == IE_INIT_LEARNED || prof_enabled() || !g_group_threads) {
    for (ie_ctx* c : order) IE_TRY(dd_group(c, groups[c], problems, o, stats, s, &worst));
  } else {
    struct Lane {
      hipStream_t st = nullptr;
      hipEvent_t done = nullptr;
      int rc = IE_OK, worst = IE_OK;
      std::string err;
    };
    std::vector<Lane> lanes(order.size());
    hipEvent_t start = nullptr;
    IE_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
    int rc = hipEventRecord(start, s) == hipSuccess ? IE_OK : IE_EDEVICE;
    for (auto& l : lanes) {
      if (rc == IE_OK && (hipStreamCreateWithFlags(&l.st, hipStreamNonBlocking) != hipSuccess ||
                          hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess ||
                          hipStreamWaitEvent(l.st, start, 0) != hipSuccess))
        rc = IE_EDEVICE;
    }
    if (rc == IE_OK) {
      std::vector<std::thread> th;
      for (size_t i = 0; i < order.size(); ++i)
        th.emplace_back([&, i]() {
          Lane& l = lanes[i];
          if (hipSetDevice(order[i]->device) != hipSuccess) {
            l.rc = IE_EDEVICE;
            l.err = "hipSetDevice failed in a group thread";
            return;
          }
          l.rc = dd_group(order[i], groups[order[i]], problems, o, stats, l.st, &l.worst);
          if (l.rc < 0) l.err = ie_last_error();
          if (hipEventRecord(l.done, l.st) != hipSuccess && l.rc >= 0) l.rc = IE_EDEVICE;
        });
      for (auto& t : th) t.join();
      for (auto& l : lanes)
        if (hipStreamWaitEvent(s, l.done, 0) != hipSuccess && rc == IE_OK) rc = IE_EDEVICE;
    }
    std::string err;
    for (auto& l : lanes) {
      if (l.rc < 0 && rc == IE_OK) {
        rc = l.rc;
        err = l.err;
      }
      worst = std::max(worst, l.worst);
    }
    for (auto& l : lanes) {
      if (l.done) (void)hipEventDestroy(l.done);
      if (l.st) (void)hipStreamDestroy(l.st);
    }
    (void)hipEventDestroy(start);
    if (rc < 0) return err.empty() ? fail(rc, "device error in a group") : fail(rc, "%s", err.c_str());
  }
  if (worst == kDiverged)
    return fail(IE_ENOCONV,
                "the full residual (eq. 9) of at least one problem grew in two consecutive sweeps "
                "(the block sweep does not contract); its output is the iterate of smallest "
                "residual (ie_dd_stats.best_sweep)");
  if (worst == IE_ENOCONV)
    return fail(IE_ENOCONV, "at least one problem did not converge; outputs of the stationary "
                            "sweeps are the iterates of smallest residual");
  return IE_OK;
}
