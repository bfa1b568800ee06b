// Alg. 1: block Gauss-Seidel / Jacobi over z-slab sub-domains (section 2.3, eqs. 19-24).
//
// Per sweep and block i: the right-hand side b_i = E(i,0) + sum_{j != i} G(ij) dsigma(j) E(j)
// is one full-grid convolution whose source skips block i's planes and whose output keeps only
// block i's planes (the coupling term acts on the whole domain, as in the paper's Ex. 3); the
// block system (I - G(ii) dsigma(i)) E(i) = b_i is then solved by restarted GMRES on the
// block's own padded FFT grid, warm-started from the previous sweep, to the adaptive (e / 10)
// or fixed inner tolerance.  After each sweep the full-domain relative residual e of eq. (9)
// is recomputed in float64.  Block Jacobi solves all equal-sized blocks as one batch.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "context.hpp"

namespace ie {

namespace {

__global__ void k_plane_nonzero(const double* __restrict__ D, long N, long plane, int nz,
                                int* __restrict__ flag) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  bool nz_ = false;
  for (int c = 0; c < 6; ++c) nz_ = nz_ || (D[c * N + i] != 0.0);
  if (nz_) flag[i / plane] = 1;
}

// copy planes [z0, z0 + nzb) of a [3][nz][ny][nx] field (component stride N) to or from a
// contiguous [3][nzb][ny][nx] block
int copy_block(const c128* src, long src_cs, c128* dst, long dst_cs, long plane_elems, int nzb,
               hipStream_t s) {
  for (int c = 0; c < 3; ++c)
    IE_HIP(hipMemcpyAsync(dst + c * dst_cs, src + c * src_cs, sizeof(c128) * plane_elems * nzb,
                          hipMemcpyDeviceToDevice, s));
  return IE_OK;
}

struct DdRun {
  ie_ctx* c;
  hipStream_t s;
  long N, plane;
  int form;
  const double* D64;  // dsigma (coupling and residual)
  // inner-form contrast (dsigma or b) and CIE transforms, full-grid arrays
  const double* M64;
  const float* M32;
  const double* A64;
  const double* Ai64;
};

// rhs = E0 on block [z0, z1) + G (dsigma src) with block planes removed from the source
int coupling_rhs(DdRun& r, const c128* src, const c128* E0, int z0, int z1, c128* rhs) {
  Plan& F = *r.c->full;
  MvArgs<double> a{};
  a.x = src;
  a.x_cs = r.N;
  a.x_bs = 0;
  a.M = r.D64;
  a.M_cs = r.N;
  a.src_z0 = 0;
  a.src_z1 = F.nz;
  a.hole_z0 = z0;
  a.hole_z1 = z1;
  a.out_z0 = z0;
  a.out_z1 = z1;
  a.y = rhs;
  a.y_cs = long(z1 - z0) * r.plane;
  a.y_zoff = z0;
  a.e = E0;
  a.e_cs = r.N;
  a.e_zoff = 0;
  a.a_e = 1;
  a.a_x = 0;
  a.a_m = 0;
  a.a_s = 1;
  return launch_matvec<double>(F, a, 1, r.s, tw64(r.c));
}

// e = ||E0 - (I - G dsigma) E|| / ||E0|| on the full grid
int full_relres(DdRun& r, const c128* E, const c128* E0, double e0norm, double* e) {
  Plan& F = *r.c->full;
  IE_TRY(r.c->tmp.ensure(sizeof(c128) * 3 * r.N));
  OpDesc op;
  op.form = IE_CONVENTIONAL;
  op.M64 = r.D64;
  op.M_cs = r.N;
  op.M_bs = 0;
  IE_TRY(apply_op<double>(F, op, E, r.c->tmp.as<c128>(), E0, true, 1, nullptr, 0, r.s, tw64(r.c)));
  double nr = 0;
  IE_TRY(norms_host(r.c->tmp.as<c128>(), 3 * r.N, 1, &nr, r.c->kw, r.s));
  *e = e0norm > 0 ? nr / e0norm : 0.0;
  return IE_OK;
}

// Solve `batch` consecutive equal blocks starting at plane z0 (rhs, x contiguous per block).
int block_solve(DdRun& r, Plan& B, int z0, int batch, c128* rhs, c128* x, double tol,
                const ie_gmres_opts& inner, GmResult* res) {
  const long nb = B.ncell();
  const long off = long(z0) * r.plane;
  OpDesc op;
  op.form = r.form;
  op.sigma0 = r.c->med.sigma0;
  op.M64 = r.M64 + off;
  op.M32 = r.M32 + off;
  op.M_cs = r.N;
  op.M_bs = nb;  // consecutive equal slabs
  GmOpts o;
  o.tol = tol;
  o.restart = inner.restart;
  o.max_its = inner.max_its;
  o.precision = inner.precision;
  o.reorth = inner.reorth == 2 ? 1 : 0;
  if (r.form == IE_CIE) {
    // C e = sqrt(sigma0) b_i, e = a x;  x = a^-1 e, per block
    IE_TRY(r.c->blk_rhs2.ensure(sizeof(c128) * 3 * nb * batch));
    IE_TRY(r.c->blk_save.ensure(sizeof(c128) * 3 * nb * batch));
    c128* rs = r.c->blk_rhs2.as<c128>();
    IE_TRY(launch_scale(rhs, rs, std::sqrt(r.c->med.sigma0), 3 * nb * batch, r.s));
    c128* xt = r.c->blk_save.as<c128>();
    for (int b = 0; b < batch; ++b)
      IE_TRY(launch_tensor_apply(r.A64 + off + b * nb, r.N, x + b * 3 * nb, nb, xt + b * 3 * nb, nb,
                                 nb, r.s));
    IE_TRY(gmres_solve(B, op, rs, xt, batch, o, res, r.c->kw_blk, tw64(r.c), tw32(r.c), r.s));
    for (int b = 0; b < batch; ++b)
      IE_TRY(launch_tensor_apply(r.Ai64 + off + b * nb, r.N, xt + b * 3 * nb, nb, x + b * 3 * nb, nb,
                                 nb, r.s));
    return IE_OK;
  }
  return gmres_solve(B, op, rhs, x, batch, o, res, r.c->kw_blk, tw64(r.c), tw32(r.c), r.s);
}

int dd_one(ie_ctx* c, const ie_problem& pr, const ie_dd_opts& o, ie_dd_stats& st, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  std::memset(&st, 0, sizeof(st));
  if (c->zb.empty()) return fail(IE_ESTATE, "context was set up without a partition");
  const ie_grid& g = c->grid;
  if (pr.grid) {
    const ie_grid& q = *pr.grid;
    if (q.nx != g.nx || q.ny != g.ny || q.nz != g.nz || q.h != g.h || q.origin[0] != g.origin[0] ||
        q.origin[1] != g.origin[1] || q.origin[2] != g.origin[2])
      return fail(IE_EINVAL, "problem grid differs from the context grid");
  }
  if (pr.E_total == nullptr) return fail(IE_EINVAL, "E_total is NULL");
  IE_TRY(check_sources(c, pr.sources, pr.nsources));
  const int form = o.inner.form;
  if (form != IE_CONVENTIONAL && form != IE_CIE) return fail(IE_EINVAL, "bad inner form");
  if (o.inner.precision != IE_FP64 && o.inner.precision != IE_MIXED)
    return fail(IE_EINVAL, "bad inner precision");
  if (!(c->prec_mask & o.inner.precision) || !(c->prec_mask & IE_FP64))
    return fail(IE_EINVAL, "context lacks the spectra this precision needs");
  if (o.max_sweeps < 1 || o.max_sweeps > IE_MAX_SWEEPS)
    return fail(IE_EINVAL, "max_sweeps must be in [1, %d]", IE_MAX_SWEEPS);
  if (o.init == IE_INIT_LEARNED) return fail(IE_EINVAL, "learned initial guess needs an ie_nn handle");
  Plan& F = *c->full;
  DdRun r;
  r.c = c;
  r.s = s;
  r.N = F.ncell();
  r.plane = long(g.nx) * g.ny;
  r.form = form;
  const int M = int(c->zb.size()) - 1;
  st.nblocks = M;

  // contrast tensors: dsigma for coupling / residual, inner form for the block operators
  IE_TRY(prepare_contrast(c, pr.sigma6, form, s));
  DevBuf dsig;
  if (form == IE_CIE) {
    IE_TRY(dsig.ensure(sizeof(double) * 6 * r.N));
    IE_TRY(launch_prep(pr.sigma6, r.N, c->med.sigma0, IE_CONVENTIONAL, dsig.as<double>(), nullptr,
                       nullptr, nullptr, c->bad.as<int>(), s));
    r.D64 = dsig.as<double>();
  } else {
    r.D64 = c->M64.as<double>();
  }
  r.M64 = c->M64.as<double>();
  r.M32 = c->M32.as<float>();
  r.A64 = form == IE_CIE ? c->A64.as<double>() : nullptr;
  r.Ai64 = form == IE_CIE ? c->Ai64.as<double>() : nullptr;

  // which blocks carry contrast
  std::vector<int> plane_flag(g.nz, 0);
  {
    DevBuf f;
    IE_TRY(f.ensure(sizeof(int) * g.nz));
    IE_HIP(hipMemsetAsync(f.p, 0, sizeof(int) * g.nz, s));
    hipLaunchKernelGGL(k_plane_nonzero, dim3(ceil_div(r.N, 256)), dim3(256), 0, s, r.D64, r.N,
                       r.plane, g.nz, f.as<int>());
    IE_LAUNCH_CHECK();
    IE_HIP(hipMemcpyAsync(plane_flag.data(), f.p, sizeof(int) * g.nz, hipMemcpyDeviceToHost, s));
    IE_HIP(hipStreamSynchronize(s));
  }
  std::vector<int> has(M, 0);
  for (int i = 0; i < M; ++i)
    for (int z = c->zb[i]; z < c->zb[i + 1]; ++z) has[i] |= plane_flag[z];

  // background field and initial guess
  IE_TRY(c->E0.ensure(sizeof(c128) * 3 * r.N));
  c128* E0 = c->E0.as<c128>();
  c128* E = (c128*)pr.E_total;
  IE_TRY(launch_background(g.nx, g.ny, g.nz, g.h, g.origin, c->med, pr.sources, pr.nsources, E0, s));
  if (o.init != IE_INIT_USER)
    IE_HIP(hipMemcpyAsync(E, E0, sizeof(c128) * 3 * r.N, hipMemcpyDeviceToDevice, s));
  double e0norm = 0;
  IE_TRY(norms_host(E0, 3 * r.N, 1, &e0norm, c->kw, s));
  double e = 0;
  IE_TRY(full_relres(r, E, E0, e0norm, &e));
  st.full_matvecs += 1;
  st.matvecs64 += 1;
  st.relres[0] = e;

  // equal blocks -> batched Jacobi
  bool equal = true;
  for (int i = 0; i < M; ++i) equal = equal && (c->zb[i + 1] - c->zb[i] == c->zb[1] - c->zb[0]);
  const long maxb = [&] {
    long m = 0;
    for (int i = 0; i < M; ++i) m = std::max(m, long(c->zb[i + 1] - c->zb[i]) * r.plane);
    return m;
  }();
  IE_TRY(c->blk_rhs.ensure(sizeof(c128) * 3 * maxb * M));
  IE_TRY(c->blk_x.ensure(sizeof(c128) * 3 * maxb * M));
  DevBuf Eold;
  if (o.scheme == IE_JACOBI) IE_TRY(Eold.ensure(sizeof(c128) * 3 * r.N));

  int status = IE_OK;
  while (e > o.tol) {
    if (st.sweeps >= o.max_sweeps) {
      status = IE_ENOCONV;
      break;
    }
    const double itol = o.adaptive ? e / 10.0 : o.inner_tol_fixed;
    const int k = st.sweeps;
    if (o.scheme == IE_JACOBI) {
      IE_HIP(hipMemcpyAsync(Eold.p, E, sizeof(c128) * 3 * r.N, hipMemcpyDeviceToDevice, s));
      // all right-hand sides from the previous sweep
      for (int i = 0; i < M; ++i) {
        const int z0 = c->zb[i], z1 = c->zb[i + 1];
        const long nb = long(z1 - z0) * r.plane;
        c128* rhs = c->blk_rhs.as<c128>() + (equal ? i * 3 * nb : 0);
        IE_TRY(coupling_rhs(r, Eold.as<c128>(), E0, z0, z1, rhs));
        st.full_matvecs += 1;
        st.matvecs64 += 1;
        if (!equal) {
          // unequal blocks: solve one at a time
          c128* x = c->blk_x.as<c128>();
          if (!has[i]) {
            IE_TRY(copy_block(rhs, nb, E + z0 * r.plane, r.N, r.plane, z1 - z0, s));
            st.block_its[k][i] = 0;
            continue;
          }
          IE_TRY(copy_block(Eold.as<c128>() + z0 * r.plane, r.N, x, nb, r.plane, z1 - z0, s));
          GmResult gr;
          IE_TRY(block_solve(r, *c->block_plan(z1 - z0), z0, 1, rhs, x, itol, o.inner, &gr));
          IE_TRY(copy_block(x, nb, E + z0 * r.plane, r.N, r.plane, z1 - z0, s));
          st.block_its[k][i] = gr.its;
          st.matvecs64 += gr.mv64;
          st.matvecs32 += gr.mv32;
          st.graph_cycles += gr.graph_cycles;
        }
      }
      if (equal) {
        const int nzb = c->zb[1] - c->zb[0];
        const long nb = long(nzb) * r.plane;
        c128* x = c->blk_x.as<c128>();
        // x <- previous iterate of every block ([3][nz] slabs are consecutive per component)
        for (int i = 0; i < M; ++i)
          IE_TRY(copy_block(Eold.as<c128>() + c->zb[i] * r.plane, r.N, x + i * 3 * nb, nb, r.plane,
                            nzb, s));
        std::vector<GmResult> gr(M);
        IE_TRY(block_solve(r, *c->block_plan(nzb), 0, M, c->blk_rhs.as<c128>(), x, itol, o.inner,
                           gr.data()));
        for (int i = 0; i < M; ++i) {
          // blocks without contrast have A_ii = I: E(i) = b_i (their GMRES converges at once)
          const c128* srcb = has[i] ? x + i * 3 * nb : c->blk_rhs.as<c128>() + i * 3 * nb;
          IE_TRY(copy_block(srcb, nb, E + c->zb[i] * r.plane, r.N, r.plane, nzb, s));
          st.block_its[k][i] = has[i] ? gr[i].its : 0;
          st.matvecs64 += gr[i].mv64;
          st.matvecs32 += gr[i].mv32;
          if (i == 0) st.graph_cycles += gr[i].graph_cycles;
        }
      }
    } else {
      for (int i = 0; i < M; ++i) {
        const int z0 = c->zb[i], z1 = c->zb[i + 1];
        const long nb = long(z1 - z0) * r.plane;
        c128* rhs = c->blk_rhs.as<c128>();
        c128* x = c->blk_x.as<c128>();
        IE_TRY(coupling_rhs(r, E, E0, z0, z1, rhs));
        st.full_matvecs += 1;
        st.matvecs64 += 1;
        if (!has[i]) {
          IE_TRY(copy_block(rhs, nb, E + z0 * r.plane, r.N, r.plane, z1 - z0, s));
          st.block_its[k][i] = 0;
          continue;
        }
        IE_TRY(copy_block(E + z0 * r.plane, r.N, x, nb, r.plane, z1 - z0, s));
        GmResult gr;
        IE_TRY(block_solve(r, *c->block_plan(z1 - z0), z0, 1, rhs, x, itol, o.inner, &gr));
        IE_TRY(copy_block(x, nb, E + z0 * r.plane, r.N, r.plane, z1 - z0, s));
        st.block_its[k][i] = gr.its;
        st.matvecs64 += gr.mv64;
        st.matvecs32 += gr.mv32;
        st.graph_cycles += gr.graph_cycles;
      }
    }
    for (int i = 0; i < M; ++i) st.total_its += st.block_its[k][i];
    st.sweeps += 1;
    IE_TRY(full_relres(r, E, E0, e0norm, &e));
    st.full_matvecs += 1;
    st.matvecs64 += 1;
    st.relres[st.sweeps] = e;
  }
  if (pr.E_anom) IE_TRY(launch_sub(E, E0, (c128*)pr.E_anom, 3 * r.N, s));
  IE_HIP(hipStreamSynchronize(s));
  st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (status == IE_ENOCONV)
    return fail(IE_ENOCONV, "DD stopped after %d sweeps at relative residual %.3e", st.sweeps, e);
  return IE_OK;
}

}  // namespace
}  // namespace ie

using namespace ie;

extern "C" int ie_dd_solve(ie_ctx* const* ctxs, int32_t nproblems, const ie_problem* problems,
                           const ie_dd_opts* opts, ie_dd_stats* stats, void* stream) {
  if (ctxs == nullptr || problems == nullptr || opts == nullptr || nproblems < 1)
    return fail(IE_EINVAL, "NULL argument or no problems");
  if (!(opts->tol >= 0)) return fail(IE_EINVAL, "bad tol");
  if (opts->scheme != IE_GS && opts->scheme != IE_JACOBI) return fail(IE_EINVAL, "bad scheme");
  hipStream_t s = (hipStream_t)stream;
  int worst = IE_OK;
  for (int p = 0; p < nproblems; ++p) {
    if (ctxs[p] == nullptr) return fail(IE_EINVAL, "context %d is NULL", p);
    ie_dd_stats local;
    ie_dd_stats& st = stats ? stats[p] : local;
    const int rc = dd_one(ctxs[p], problems[p], *opts, st, s);
    if (rc < 0) return rc;
    if (rc == IE_ENOCONV) worst = IE_ENOCONV;
  }
  if (worst == IE_ENOCONV) return fail(IE_ENOCONV, "at least one problem did not converge");
  return IE_OK;
}
