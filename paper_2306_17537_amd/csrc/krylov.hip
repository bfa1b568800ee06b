// Device-side restarted GMRES: fused Gram-Schmidt passes, float64 reductions, Givens
// rotations and back substitution in single-block kernels (see krylov.hpp).
#include <cmath>
#include <vector>

#include "krylov.hpp"

namespace ie {

namespace {

constexpr int RB = 256;                 // threads per reduction block
constexpr int PW = MAXM + 2;            // partial slots per block: dots [0, MAXM], norm at MAXM+1
constexpr int NORM = MAXM + 1;

int red_grid(long n) {
  long g = (n + RB * 8 - 1) / (RB * 8);
  if (g < 1) g = 1;
  if (g > 512) g = 512;
  return int(g);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic block-wide sum of one double (all threads receive the result).
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double r = 0;
#pragma unroll
  for (int q = 0; q < RB / 64; ++q) r += sh[q];
  return r;
}

template <typename T>
__device__ __forceinline__ c128 up(cx<T> v) { return c128{double(v.re), double(v.im)}; }

// Fused Gram-Schmidt pass on w (stride wbs per problem):
//   UPD : w <- w - sum_{i<count} hc[i] V_i   (hc from the problem state)
//   DOTS: partial <V_i, w> for i < count;    NRM: partial ||w||^2
template <typename TA, bool UPD, bool DOTS, bool NRM>
__global__ void __launch_bounds__(RB)
    k_orth(const cx<TA>* __restrict__ V, long vstride, long vbs, cx<TA>* w, long wbs, long n,
           int count, const GmState* __restrict__ st, c128* __restrict__ part) {
  const int b = blockIdx.z;
  if (st != nullptr && st[b].active == 0) return;
  __shared__ double sh[RB / 64];
  const cx<TA>* Vb = V + b * vbs;
  cx<TA>* wb = w + b * wbs;
  c128 h[MAXM + 1];
  c128 acc[MAXM + 1];
#pragma unroll
  for (int i = 0; i <= MAXM; ++i) {
    h[i] = (UPD && i < count) ? st[b].hc[i] : c128{0, 0};
    acc[i] = c128{0, 0};
  }
  double nrm = 0;
  const long stride = long(gridDim.x) * RB;
  for (long e = long(blockIdx.x) * RB + threadIdx.x; e < n; e += stride) {
    cx<TA> vv[MAXM + 1];
#pragma unroll
    for (int i = 0; i <= MAXM; ++i)
      if ((UPD || DOTS) && i < count) vv[i] = Vb[i * vstride + e];
    cx<TA> wv = wb[e];
    if (UPD) {
      c128 wd = up(wv);
#pragma unroll
      for (int i = 0; i <= MAXM; ++i)
        if (i < count) wd = wd - h[i] * up(vv[i]);
      wv = cx<TA>{TA(wd.re), TA(wd.im)};
      wb[e] = wv;
    }
    const c128 wd = up(wv);
    if (DOTS) {
#pragma unroll
      for (int i = 0; i <= MAXM; ++i)
        if (i < count) acc[i] = acc[i] + cjmul(up(vv[i]), wd);
    }
    if (NRM) nrm += wd.re * wd.re + wd.im * wd.im;
  }
  c128* pb = part + (long(b) * gridDim.x + blockIdx.x) * PW;
  if (DOTS) {
    for (int i = 0; i < count; ++i) {
      const double re = block_sum(acc[i].re, sh);
      const double im = block_sum(acc[i].im, sh);
      if (threadIdx.x == 0) pb[i] = c128{re, im};
    }
  }
  if (NRM) {
    const double r = block_sum(nrm, sh);
    if (threadIdx.x == 0) pb[NORM] = c128{r, 0};
  }
}

// Sum slot `slot` of the G block partials of problem b (deterministic order).
__device__ c128 reduce_slot(const c128* part, int b, int G, int slot, double* sh) {
  double re = 0, im = 0;
  for (int q = threadIdx.x; q < G; q += RB) {
    const c128 v = part[(long(b) * G + q) * PW + slot];
    re += v.re;
    im += v.im;
  }
  re = block_sum(re, sh);
  im = block_sum(im, sh);
  return c128{re, im};
}

// Coefficients of a Gram-Schmidt pass: hc[i] = <V_i, w>, accumulated into column j of H.
__global__ void __launch_bounds__(RB)
    k_hsum(GmState* st, const c128* part, int G, int j, int count, int first) {
  const int b = blockIdx.x;
  if (st[b].active == 0) return;
  __shared__ double sh[RB / 64];
  for (int i = 0; i < count; ++i) {
    const c128 h = reduce_slot(part, b, G, i, sh);
    if (threadIdx.x == 0) {
      st[b].hc[i] = h;
      st[b].H[j][i] = first ? h : st[b].H[j][i] + h;
    }
  }
}

// h_{j+1,j} = ||w||, previous rotations applied to column j, new rotation, residual estimate.
__global__ void __launch_bounds__(RB) k_givens(GmState* st, const c128* part, int G, int j) {
  const int b = blockIdx.x;
  if (st[b].active == 0) return;
  __shared__ double sh[RB / 64];
  const double hn2 = reduce_slot(part, b, G, NORM, sh).re;
  if (threadIdx.x != 0) return;
  GmState& s = st[b];
  const double hn = sqrt(hn2);
  c128* H = s.H[j];
  for (int i = 0; i < j; ++i) {
    const c128 t = cjmul(s.cs[i], H[i]) + cjmul(s.sn[i], H[i + 1]);
    H[i + 1] = c128{0, 0} - s.sn[i] * H[i] + s.cs[i] * H[i + 1];
    H[i] = t;
  }
  const double hjj = sqrt(H[j].re * H[j].re + H[j].im * H[j].im);
  const double den = sqrt(hjj * hjj + hn * hn);
  c128 c, sn;
  if (den == 0.0) {
    c = c128{1, 0};
    sn = c128{0, 0};
  } else {
    c = c128{H[j].re / den, H[j].im / den};
    sn = c128{hn / den, 0};
  }
  s.cs[j] = c;
  s.sn[j] = sn;
  H[j] = c128{den, 0};
  H[j + 1] = c128{0, 0};
  const c128 gj = s.g[j];
  s.g[j + 1] = c128{0, 0} - sn * gj;
  s.g[j] = cjmul(c, gj);
  s.est = sqrt(s.g[j + 1].re * s.g[j + 1].re + s.g[j + 1].im * s.g[j + 1].im);
  s.k = j + 1;
  s.its += 1;
  s.hn2 = hn2;
  const bool brk = (hn == 0.0) || (den == 0.0);
  s.breakdown = brk ? 1 : 0;
  s.inv_h = brk ? 0.0 : 1.0 / hn;
  if (s.est <= s.target || s.its >= s.max_its || brk) s.active = 0;
}

template <typename TA>
__global__ void __launch_bounds__(RB) k_scale(cx<TA>* w, long wbs, long n, const GmState* st) {
  const int b = blockIdx.z;
  if (st[b].active == 0) return;
  const double s = st[b].inv_h;
  cx<TA>* wb = w + b * wbs;
  const long stride = long(gridDim.x) * RB;
  for (long e = long(blockIdx.x) * RB + threadIdx.x; e < n; e += stride) {
    const cx<TA> v = wb[e];
    wb[e] = cx<TA>{TA(double(v.re) * s), TA(double(v.im) * s)};
  }
}

// Start-of-solve: ||b||, target, counters.
__global__ void __launch_bounds__(RB)
    k_set_bnorm(GmState* st, const c128* part, int G, double tol, int max_its) {
  const int b = blockIdx.x;
  __shared__ double sh[RB / 64];
  const double n2 = reduce_slot(part, b, G, NORM, sh).re;
  if (threadIdx.x == 0) {
    st[b].bnorm = sqrt(n2);
    st[b].target = tol * sqrt(n2);
    st[b].its = 0;
    st[b].max_its = max_its;
    st[b].active = 0;
    st[b].k = 0;
  }
}

// Start-of-cycle: beta = ||r||, g = beta e1, active unless converged or out of iterations.
__global__ void __launch_bounds__(RB) k_cycle_begin(GmState* st, const c128* part, int G) {
  const int b = blockIdx.x;
  __shared__ double sh[RB / 64];
  const double n2 = reduce_slot(part, b, G, NORM, sh).re;
  if (threadIdx.x == 0) {
    GmState& s = st[b];
    const double beta = sqrt(n2);
    s.beta = beta;
    s.est = beta;
    s.k = 0;
    for (int i = 0; i <= MAXM; ++i) s.g[i] = c128{0, 0};
    s.g[0] = c128{beta, 0};
    s.inv_h = beta > 0 ? 1.0 / beta : 0.0;
    s.active = (beta > s.target && s.its < s.max_its) ? 1 : 0;
  }
}

__global__ void k_summary(const GmState* st, GmSummary* out, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  out[b].beta = st[b].beta;
  out[b].bnorm = st[b].bnorm;
  out[b].active = st[b].active;
  out[b].its = st[b].its;
}

template <typename TA>
__global__ void __launch_bounds__(RB)
    k_scale_cast(const c128* __restrict__ r, long rbs, cx<TA>* __restrict__ v, long vbs, long n,
                 const GmState* st) {
  const int b = blockIdx.z;
  if (st[b].active == 0) return;
  const double s = st[b].inv_h;
  const c128* rb = r + b * rbs;
  cx<TA>* vb = v + b * vbs;
  const long stride = long(gridDim.x) * RB;
  for (long e = long(blockIdx.x) * RB + threadIdx.x; e < n; e += stride) {
    const c128 x = rb[e];
    vb[e] = cx<TA>{TA(x.re * s), TA(x.im * s)};
  }
}

// y = R^-1 g on the k x k rotated Hessenberg (upper triangular).
__global__ void k_backsolve(GmState* st, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  GmState& s = st[b];
  const int k = s.k;
  for (int i = k - 1; i >= 0; --i) {
    c128 acc = s.g[i];
    for (int l = i + 1; l < k; ++l) acc = acc - s.H[l][i] * s.y[l];
    const c128 d = s.H[i][i];
    const double dd = d.re * d.re + d.im * d.im;
    s.y[i] = dd > 0 ? c128{(acc.re * d.re + acc.im * d.im) / dd, (acc.im * d.re - acc.re * d.im) / dd}
                    : c128{0, 0};
  }
}

// x += sum_{i<k} y_i V_i (float64 accumulation).
template <typename TA>
__global__ void __launch_bounds__(RB)
    k_xupdate(c128* x, long xbs, const cx<TA>* __restrict__ V, long vstride, long vbs, long n,
              const GmState* st) {
  const int b = blockIdx.z;
  const int k = st[b].k;
  if (k == 0) return;
  c128 y[MAXM];
#pragma unroll
  for (int i = 0; i < MAXM; ++i) y[i] = i < k ? st[b].y[i] : c128{0, 0};
  c128* xb = x + b * xbs;
  const cx<TA>* Vb = V + b * vbs;
  const long stride = long(gridDim.x) * RB;
  for (long e = long(blockIdx.x) * RB + threadIdx.x; e < n; e += stride) {
    c128 acc = xb[e];
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < k) acc = acc + y[i] * up(Vb[i * vstride + e]);
    xb[e] = acc;
  }
}

}  // namespace

// ---------------------------------------------------------------------------------------

template <typename T>
int apply_op(Plan& p, const OpDesc& op, const cx<T>* x, cx<T>* y, const cx<T>* e, bool residual,
             int batch, const int* active, int active_bs, hipStream_t s, const cx<T>* tw) {
  MvArgs<T> a{};
  const long N = p.ncell();
  a.x = x;
  a.x_cs = N;
  a.x_bs = 3 * N;
  a.x_zoff = 0;
  a.M = sizeof(T) == 8 ? (const T*)op.M64 : (const T*)op.M32;
  a.M_cs = op.M_cs;
  a.M_bs = op.M_bs;
  a.M_zoff = 0;
  a.src_z0 = 0;
  a.src_z1 = p.nz;
  a.hole_z0 = a.hole_z1 = -1;
  a.out_z0 = 0;
  a.out_z1 = p.nz;
  a.y = y;
  a.y_cs = N;
  a.y_bs = 3 * N;
  a.y_zoff = 0;
  a.e = residual ? e : nullptr;
  a.e_cs = N;
  a.e_bs = 3 * N;
  a.e_zoff = 0;
  // A x = x - G (M x)               (conventional, M = dsigma)
  // C x = x - M x - 2 sigma0 G (M x) (contraction, M = b)
  const T sg = (op.form == IE_CIE) ? T(-2.0 * op.sigma0) : T(-1);
  const T am = (op.form == IE_CIE) ? T(1) : T(0);
  if (residual) {
    a.a_e = 1;
    a.a_x = -1;
    a.a_m = -am;
    a.a_s = -sg;
  } else {
    a.a_e = 0;
    a.a_x = 1;
    a.a_m = am;
    a.a_s = sg;
  }
  a.active = active;
  a.active_bs = active_bs;
  return launch_matvec<T>(p, a, batch, s, tw);
}

template int apply_op<double>(Plan&, const OpDesc&, const c128*, c128*, const c128*, bool, int,
                              const int*, int, hipStream_t, const c128*);
template int apply_op<float>(Plan&, const OpDesc&, const c64*, c64*, const c64*, bool, int,
                             const int*, int, hipStream_t, const c64*);

static int ensure_host(KrylovWork& w, int batch) {
  IE_TRY(w.sum.ensure(sizeof(GmSummary) * batch));
  if (batch <= w.host_cap) return IE_OK;
  if (w.host) (void)hipHostFree(w.host);
  w.host = nullptr;
  IE_HIP(hipHostMalloc((void**)&w.host, sizeof(GmSummary) * batch, hipHostMallocDefault));
  w.host_cap = batch;
  return IE_OK;
}

// Summaries of all problems -> pinned host copy (synchronises the stream).
static int fetch_summary(KrylovWork& w, const GmState* st, int batch, hipStream_t s) {
  hipLaunchKernelGGL(k_summary, dim3(ceil_div(batch, 64)), dim3(64), 0, s, st,
                     w.sum.as<GmSummary>(), batch);
  IE_LAUNCH_CHECK();
  IE_HIP(hipMemcpyAsync(w.host, w.sum.p, sizeof(GmSummary) * batch, hipMemcpyDeviceToHost, s));
  IE_HIP(hipStreamSynchronize(s));
  return IE_OK;
}

int norms_host(const c128* v, long n, int batch, double* out, KrylovWork& w, hipStream_t s) {
  const int G = red_grid(n);
  IE_TRY(w.part.ensure(sizeof(c128) * PW * G * batch));
  IE_TRY(w.st.ensure(sizeof(GmState) * batch));
  IE_TRY(ensure_host(w, batch));
  GmState* st = w.st.as<GmState>();
  hipLaunchKernelGGL((k_orth<double, false, false, true>), dim3(G, 1, batch), dim3(RB), 0, s, v, 0L,
                     0L, const_cast<c128*>(v), n, n, 0, nullptr, w.part.as<c128>());
  IE_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_set_bnorm, dim3(batch), dim3(RB), 0, s, st, w.part.as<c128>(), G, 0.0, 0);
  IE_LAUNCH_CHECK();
  IE_TRY(fetch_summary(w, st, batch, s));
  for (int b = 0; b < batch; ++b) out[b] = w.host[b].bnorm;
  return IE_OK;
}

template <typename TA>
static int gmres_impl(Plan& p, const OpDesc& op, const c128* rhs, c128* x, int batch,
                      const GmOpts& o, GmResult* res, KrylovWork& w, const c128* tw64,
                      const cx<TA>* twa, hipStream_t s) {
  const long N = p.ncell();
  const long n = 3 * N;
  const int m = o.restart;
  if (m < 1 || m > MAXM) return fail(IE_EINVAL, "restart must be in [1, %d], got %d", MAXM, m);
  const bool reorth = o.reorth < 0 ? (sizeof(TA) == 4) : (o.reorth != 0);
  const int G = red_grid(n);
  const long vbs = long(m + 1) * n;
  IE_TRY(w.V.ensure(sizeof(cx<TA>) * vbs * batch));
  IE_TRY(w.r.ensure(sizeof(c128) * n * batch));
  IE_TRY(w.part.ensure(sizeof(c128) * PW * G * batch));
  IE_TRY(w.st.ensure(sizeof(GmState) * batch));
  IE_TRY(ensure_host(w, batch));
  GmState* st = w.st.as<GmState>();
  cx<TA>* V = w.V.as<cx<TA>>();
  c128* r = w.r.as<c128>();
  c128* part = w.part.as<c128>();
  const int* act = &st[0].active;
  const int act_bs = int(sizeof(GmState) / sizeof(int));
  const dim3 vgrid(G, 1, batch);
  for (int b = 0; b < batch; ++b) res[b] = GmResult{};

  // ||b||
  hipLaunchKernelGGL((k_orth<double, false, false, true>), vgrid, dim3(RB), 0, s, rhs, 0L, 0L,
                     const_cast<c128*>(rhs), n, n, 0, nullptr, part);
  IE_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_set_bnorm, dim3(batch), dim3(RB), 0, s, st, part, G, o.tol, o.max_its);
  IE_LAUNCH_CHECK();

  for (int cycle = 0;; ++cycle) {
    // r = b - A x in float64, beta = ||r||
    IE_TRY(apply_op<double>(p, op, x, r, rhs, true, batch, nullptr, 0, s, tw64));
    for (int b = 0; b < batch; ++b) res[b].mv64 += 1;
    hipLaunchKernelGGL((k_orth<double, false, false, true>), vgrid, dim3(RB), 0, s, r, 0L, 0L, r, n,
                       n, 0, nullptr, part);
    IE_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cycle_begin, dim3(batch), dim3(RB), 0, s, st, part, G);
    IE_LAUNCH_CHECK();
    IE_TRY(fetch_summary(w, st, batch, s));
    int any = 0;
    for (int b = 0; b < batch; ++b) {
      const GmSummary& h = w.host[b];
      res[b].its = h.its;
      res[b].relres = h.bnorm > 0 ? h.beta / h.bnorm : 0.0;
      res[b].converged = h.beta <= o.tol * h.bnorm;
      if (h.active) {
        any = 1;
        res[b].cycles += 1;
      }
    }
    if (!any) break;
    // V0 = r / beta
    hipLaunchKernelGGL((k_scale_cast<TA>), vgrid, dim3(RB), 0, s, r, n, V, vbs, n, st);
    IE_LAUNCH_CHECK();
    for (int j = 0; j < m; ++j) {
      cx<TA>* vj = V + j * n;
      cx<TA>* w1 = V + (j + 1) * n;
      // w = A v_j
      {
        MvArgs<TA> a{};
        a.x = vj;
        a.x_cs = N;
        a.x_bs = vbs;
        a.M = sizeof(TA) == 8 ? (const TA*)op.M64 : (const TA*)op.M32;
        a.M_cs = op.M_cs;
        a.M_bs = op.M_bs;
        a.src_z0 = 0;
        a.src_z1 = p.nz;
        a.hole_z0 = a.hole_z1 = -1;
        a.out_z0 = 0;
        a.out_z1 = p.nz;
        a.y = w1;
        a.y_cs = N;
        a.y_bs = vbs;
        const TA sg = (op.form == IE_CIE) ? TA(-2.0 * op.sigma0) : TA(-1);
        a.a_e = 0;
        a.a_x = 1;
        a.a_m = (op.form == IE_CIE) ? TA(1) : TA(0);
        a.a_s = sg;
        a.active = act;
        a.active_bs = act_bs;
        IE_TRY(launch_matvec<TA>(p, a, batch, s, twa));
      }
      // Gram-Schmidt: h = V^H w, w -= V h (twice with re-orthogonalisation), ||w||
      hipLaunchKernelGGL((k_orth<TA, false, true, false>), vgrid, dim3(RB), 0, s, V, n, vbs, w1,
                         vbs, n, j + 1, st, part);
      IE_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_hsum, dim3(batch), dim3(RB), 0, s, st, part, G, j, j + 1, 1);
      IE_LAUNCH_CHECK();
      if (reorth) {
        hipLaunchKernelGGL((k_orth<TA, true, true, false>), vgrid, dim3(RB), 0, s, V, n, vbs, w1,
                           vbs, n, j + 1, st, part);
        IE_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_hsum, dim3(batch), dim3(RB), 0, s, st, part, G, j, j + 1, 0);
        IE_LAUNCH_CHECK();
      }
      hipLaunchKernelGGL((k_orth<TA, true, false, true>), vgrid, dim3(RB), 0, s, V, n, vbs, w1, vbs,
                         n, j + 1, st, part);
      IE_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_givens, dim3(batch), dim3(RB), 0, s, st, part, G, j);
      IE_LAUNCH_CHECK();
      hipLaunchKernelGGL((k_scale<TA>), vgrid, dim3(RB), 0, s, w1, vbs, n, st);
      IE_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_backsolve, dim3(ceil_div(batch, 64)), dim3(64), 0, s, st, batch);
    IE_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_xupdate<TA>), vgrid, dim3(RB), 0, s, x, n, V, n, vbs, n, st);
    IE_LAUNCH_CHECK();
  }
  for (int b = 0; b < batch; ++b) {
    const int arn = res[b].its;
    if (sizeof(TA) == 8)
      res[b].mv64 += arn;
    else
      res[b].mv32 += arn;
  }
  return IE_OK;
}

int gmres_solve(Plan& p, const OpDesc& op, const c128* rhs, c128* x, int batch, const GmOpts& o,
                GmResult* res, KrylovWork& w, const c128* tw64, const c64* tw32, hipStream_t s) {
  if (o.precision == IE_MIXED) return gmres_impl<float>(p, op, rhs, x, batch, o, res, w, tw64, tw32, s);
  return gmres_impl<double>(p, op, rhs, x, batch, o, res, w, tw64, tw64, s);
}

}  // namespace ie
