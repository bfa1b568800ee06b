// C ABI entry points (include/ie.h): validation, context life cycle, operator, GMRES.
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <string>

#include "context.hpp"

namespace ie {

static thread_local std::string g_err = "no error";

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

int fail(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

__global__ void k_scale(const c128* __restrict__ x, c128* __restrict__ y, double a, long n) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}
__global__ void k_sub(const c128* __restrict__ x, const c128* __restrict__ z, c128* __restrict__ y,
                      long n) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] - z[i];
}

int launch_scale(const c128* x, c128* y, double alpha, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(ceil_div(n, 256)), dim3(256), 0, s, x, y, alpha, n);
  IE_LAUNCH_CHECK();
  return IE_OK;
}
int launch_sub(const c128* x, const c128* z, c128* y, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, dim3(ceil_div(n, 256)), dim3(256), 0, s, x, z, y, n);
  IE_LAUNCH_CHECK();
  return IE_OK;
}

int prepare_contrast(ie_ctx* c, const double* sigma6, int form, hipStream_t s) {
  if (sigma6 == nullptr) return fail(IE_EINVAL, "sigma6 is NULL");
  const long N = c->full->ncell();
  IE_TRY(c->M64.ensure(sizeof(double) * 6 * N));
  IE_TRY(c->M32.ensure(sizeof(float) * 6 * N));
  IE_TRY(c->bad.ensure(sizeof(int)));
  const bool cie = form == IE_CIE;
  if (cie) {
    IE_TRY(c->A64.ensure(sizeof(double) * 6 * N));
    IE_TRY(c->Ai64.ensure(sizeof(double) * 6 * N));
  }
  IE_HIP(hipMemsetAsync(c->bad.p, 0, sizeof(int), s));
  IE_TRY(launch_prep(sigma6, N, c->med.sigma0, cie ? IE_CIE : IE_CONVENTIONAL, c->M64.as<double>(),
                     c->M32.as<float>(), cie ? c->A64.as<double>() : nullptr,
                     cie ? c->Ai64.as<double>() : nullptr, c->bad.as<int>(), s));
  int bad = 0;
  IE_HIP(hipMemcpyAsync(&bad, c->bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  IE_HIP(hipStreamSynchronize(s));
  if (bad) return fail(IE_EINVAL, "sigma6 holds a non-finite or non-positive-definite tensor");
  return IE_OK;
}

int check_sources(const ie_ctx* c, const ie_source* src, int nsrc) {
  if (nsrc < 1 || src == nullptr) return fail(IE_EINVAL, "at least one source is required");
  const ie_grid& g = c->grid;
  for (int q = 0; q < nsrc; ++q) {
    const ie_source& s = src[q];
    if (s.kind != IE_MAG_DIPOLE && s.kind != IE_ELEC_DIPOLE)
      return fail(IE_EINVAL, "source %d: unknown kind %d", q, s.kind);
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(s.pos[a]) || !std::isfinite(s.moment[a]))
        return fail(IE_EINVAL, "source %d: non-finite position or moment", q);
    // nearest cell centre
    const int n[3] = {g.nx, g.ny, g.nz};
    double d2 = 0;
    for (int a = 0; a < 3; ++a) {
      double u = (s.pos[a] - g.origin[a]) / g.h - 0.5;
      double iu = std::round(u);
      if (iu < 0) iu = 0;
      if (iu > n[a] - 1) iu = n[a] - 1;
      const double d = (u - iu) * g.h;
      d2 += d * d;
    }
    if (std::sqrt(d2) <= 1e-9 * g.h)
      return fail(IE_EINVAL, "source %d coincides with a cell centre (field singular)", q);
  }
  return IE_OK;
}

static int valid_grid(const ie_grid* g) {
  if (g == nullptr) return fail(IE_EINVAL, "grid is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nx > 512 || g->ny > 512 || g->nz > 512)
    return fail(IE_EINVAL, "grid size %d x %d x %d outside 1..512", g->nx, g->ny, g->nz);
  if (!(g->h > 0) || !std::isfinite(g->h)) return fail(IE_EINVAL, "cell size must be > 0");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(g->origin[a])) return fail(IE_EINVAL, "non-finite origin");
  return IE_OK;
}

static std::unique_ptr<Plan> make_plan(int nx, int ny, int nz, bool pow2) {
  auto p = std::make_unique<Plan>();
  p->nx = nx;
  p->ny = ny;
  p->nz = nz;
  p->LX = fft_len(nx, pow2);
  p->LY = fft_len(ny, pow2);
  p->LZ = fft_len(nz, pow2);
  return p;
}

}  // namespace ie

using namespace ie;

namespace ie {
bool g_group_threads = true;
}  // namespace ie

namespace {
bool g_autotune = true;
int g_force_variant = -1;
int g_fft_lengths = 0;  // 0 shortest, 1 powers of two, 2 the faster of the two by timing

// every pass of the plan on one variant (the x pass has eight, the y passes four, the z passes
// two)
void force_variant(Plan& p, int v) {
  for (int pi = 0; pi < 2; ++pi)
    for (int q = 0; q < 5; ++q)
      p.var[pi][q] = int8_t(q == 2 ? v : (q == 1 || q == 3 ? (v & 3) : (v & 1)));
}

// Plan of one grid shape with its Green spectrum and launch variants, at the FFT lengths the
// length mode asks for.
int setup_plan(ie_ctx* c, int nx, int ny, int nz, hipStream_t s, std::unique_ptr<Plan>& out) {
  auto build = [&](bool pow2, std::unique_ptr<Plan>& p) {
    p = make_plan(nx, ny, nz, pow2);
    IE_TRY(build_green(*p, c->grid.h, c->med, c->prec_mask, tw64(c), tw32(c), s));
    if (g_force_variant >= 0)
      force_variant(*p, g_force_variant);
    else if (g_autotune)
      IE_TRY(autotune(*p, c->prec_mask, tw64(c), tw32(c), s));
    return IE_OK;
  };
  IE_TRY(build(g_fft_lengths == 1, out));
  if (g_fft_lengths != 2) return IE_OK;
  std::unique_ptr<Plan> q;
  IE_TRY(build(true, q));
  if (q->LX == out->LX && q->LY == out->LY && q->LZ == out->LZ) return IE_OK;
  float a = 0, b = 0;
  IE_TRY(operator_us(*out, c->prec_mask, tw64(c), tw32(c), s, a));
  IE_TRY(operator_us(*q, c->prec_mask, tw64(c), tw32(c), s, b));
  if (b < a) out = std::move(q);
  out->len_us[0] = a;
  out->len_us[1] = b;
  return IE_OK;
}
}  // namespace

extern "C" {

const char* ie_last_error(void) { return g_err.c_str(); }

const char* ie_version(void) { return "ie-gfx950 0.1"; }

int ie_set_option(int32_t option, int32_t value) {
  if (option == IE_OPT_GRAPHS) {
    if (value != 0 && value != 1) return fail(IE_EINVAL, "IE_OPT_GRAPHS takes 0 or 1");
    g_use_graphs = value != 0;
    return IE_OK;
  }
  if (option == IE_OPT_AUTOTUNE) {
    if (value != 0 && value != 1) return fail(IE_EINVAL, "IE_OPT_AUTOTUNE takes 0 or 1");
    g_autotune = value != 0;
    return IE_OK;
  }
  if (option == IE_OPT_FORCE_VARIANT) {
    if (value < -1 || value > 7) return fail(IE_EINVAL, "IE_OPT_FORCE_VARIANT takes -1 .. 7");
    g_force_variant = value;
    return IE_OK;
  }
  if (option == IE_OPT_GROUP_THREADS) {
    if (value != 0 && value != 1) return fail(IE_EINVAL, "IE_OPT_GROUP_THREADS takes 0 or 1");
    g_group_threads = value != 0;
    return IE_OK;
  }
  if (option == IE_OPT_FFT_LENGTHS) {
    if (value < 0 || value > 2) return fail(IE_EINVAL, "IE_OPT_FFT_LENGTHS takes 0, 1 or 2");
    g_fft_lengths = value;
    return IE_OK;
  }
  return fail(IE_EINVAL, "unknown option %d", option);
}

int ie_green_setup(const ie_grid* grid, const ie_medium* medium, const ie_partition* partition,
                   int32_t precision_mask, void* stream, ie_ctx** out) {
  if (out == nullptr) return fail(IE_EINVAL, "out is NULL");
  *out = nullptr;
  IE_TRY(valid_grid(grid));
  if (medium == nullptr) return fail(IE_EINVAL, "medium is NULL");
  if (!(medium->sigma0 > 0) || !std::isfinite(medium->sigma0))
    return fail(IE_EINVAL, "sigma0 must be > 0");
  if (!(medium->freq_hz > 0) || !std::isfinite(medium->freq_hz))
    return fail(IE_EINVAL, "frequency must be > 0");
  if (medium->mu0 < 0 || !std::isfinite(medium->mu0)) return fail(IE_EINVAL, "mu0 must be >= 0");
  if ((precision_mask & (IE_FP64 | IE_MIXED)) == 0 || (precision_mask & ~(IE_FP64 | IE_MIXED)))
    return fail(IE_EINVAL, "precision_mask must be a non-empty combination of IE_FP64, IE_MIXED");
  std::vector<int> zb;
  if (partition != nullptr) {
    const int M = partition->nblocks;
    if (M < 1 || M > IE_MAX_BLOCKS || partition->z_bounds == nullptr)
      return fail(IE_EINVAL, "partition needs 1..%d blocks and z_bounds", IE_MAX_BLOCKS);
    if (partition->z_bounds[0] != 0 || partition->z_bounds[M] != grid->nz)
      return fail(IE_EINVAL, "partition must start at 0 and end at nz");
    for (int i = 0; i < M; ++i)
      if (partition->z_bounds[i + 1] <= partition->z_bounds[i])
        return fail(IE_EINVAL, "partition bounds must increase strictly");
    zb.assign(partition->z_bounds, partition->z_bounds + M + 1);
  }
  hipStream_t s = (hipStream_t)stream;
  auto c = std::make_unique<ie_ctx>();
  c->grid = *grid;
  c->zb = zb;
  c->prec_mask = precision_mask;
  IE_HIP(hipGetDevice(&c->device));
  IE_TRY(noalloc_init(c->device));
  Medium& m = c->med;
  m.sigma0 = medium->sigma0;
  m.freq = medium->freq_hz;
  m.mu0 = medium->mu0 > 0 ? medium->mu0 : 4.0e-7 * M_PI;
  m.omega = 2.0 * M_PI * m.freq;
  // k0 = sqrt(i omega mu0 sigma0) = (1 + i) sqrt(omega mu0 sigma0 / 2), Im k0 > 0
  const double kk = std::sqrt(m.omega * m.mu0 * m.sigma0 / 2.0);
  m.k0re = kk;
  m.k0im = kk;
  // twiddles exp(-2 pi i k / TW_N) from the definition, in long double
  {
    std::vector<c128> t64(TW_N);
    std::vector<c64> t32(TW_N);
    for (int k = 0; k < TW_N; ++k) {
      const long double ang = -2.0L * 3.14159265358979323846264338327950288L * k / TW_N;
      t64[k] = c128{double(cosl(ang)), double(sinl(ang))};
      t32[k] = c64{float(cosl(ang)), float(sinl(ang))};
    }
    IE_TRY(c->tw64.ensure(sizeof(c128) * TW_N));
    IE_TRY(c->tw32.ensure(sizeof(c64) * TW_N));
    IE_HIP(hipMemcpy(c->tw64.p, t64.data(), sizeof(c128) * TW_N, hipMemcpyHostToDevice));
    IE_HIP(hipMemcpy(c->tw32.p, t32.data(), sizeof(c64) * TW_N, hipMemcpyHostToDevice));
  }
  IE_TRY(setup_plan(c.get(), grid->nx, grid->ny, grid->nz, s, c->full));
  if (partition != nullptr) {
    for (size_t i = 0; i + 1 < c->zb.size(); ++i) {
      const int nzb = c->zb[i + 1] - c->zb[i];
      if (c->blocks.count(nzb)) continue;
      std::unique_ptr<Plan> p;
      IE_TRY(setup_plan(c.get(), grid->nx, grid->ny, nzb, s, p));
      c->blocks[nzb] = std::move(p);
    }
  }
  *out = c.release();
  return IE_OK;
}

int ie_ctx_tuning(const ie_ctx* ctx, char* buf, int32_t len) {
  if (ctx == nullptr || buf == nullptr || len < 1) return fail(IE_EINVAL, "bad arguments");
  static const char* pass_names[5] = {"zfwd", "yfwd", "xconv", "yinv", "zinv"};
  std::string o = "[";
  auto plan = [&](const Plan& p) {
    for (int pi = 0; pi < 2; ++pi) {
      if (!(ctx->prec_mask & (pi == 0 ? IE_FP64 : IE_MIXED))) continue;
      for (int q = 0; q < 5; ++q) {
        char t[512];
        const float* u = p.tune_us[pi][q];
        snprintf(t, sizeof(t),
                 "%s{\"grid\": [%d, %d, %d], \"fft\": [%d, %d, %d], "
                 "\"lengths_us\": [%.2f, %.2f], \"precision\": \"%s\", "
                 "\"pass\": \"%s\", \"variant\": %d, \"kernel\": \"%s\", "
                 "\"us\": [%.2f, %.2f, %.2f, %.2f, %.2f, %.2f, %.2f, %.2f]}",
                 o.size() > 1 ? ", " : "", p.nx, p.ny, p.nz, p.LX, p.LY, p.LZ, p.len_us[0],
                 p.len_us[1], pi == 0 ? "c128" : "c64", pass_names[q], p.var[pi][q],
                 pass_kernel(p, pi, q).c_str(), u[0], u[1], u[2], u[3], u[4], u[5], u[6], u[7]);
        o += t;
      }
    }
  };
  plan(*ctx->full);
  for (const auto& kv : ctx->blocks) plan(*kv.second);
  o += "]";
  if (int(o.size()) + 1 > len) return fail(IE_EINVAL, "buffer needs %zu bytes", o.size() + 1);
  std::memcpy(buf, o.c_str(), o.size() + 1);
  return IE_OK;
}

int ie_tuning_save(const char* path) {
  if (path == nullptr) return fail(IE_EINVAL, "path is NULL");
  return tuning_save(path);
}

int ie_tuning_load(const char* path) {
  if (path == nullptr) return fail(IE_EINVAL, "path is NULL");
  return tuning_load(path);
}

int ie_ctx_destroy(ie_ctx* ctx) {
  if (ctx == nullptr) return IE_OK;
  (void)hipDeviceSynchronize();
  delete ctx;
  return IE_OK;
}

int ie_background_field(ie_ctx* ctx, const ie_source* sources, int32_t nsources, void* E0,
                        void* stream) {
  if (ctx == nullptr || E0 == nullptr) return fail(IE_EINVAL, "NULL argument");
  IE_TRY(check_sources(ctx, sources, nsources));
  const ie_grid& g = ctx->grid;
  return launch_background(g.nx, g.ny, g.nz, g.h, g.origin, ctx->med, sources, nsources,
                           (c128*)E0, (hipStream_t)stream);
}

int ie_matvec(ie_ctx* ctx, const double* sigma6, const void* x, void* y, int32_t form,
              int32_t precision, void* stream) {
  if (ctx == nullptr || x == nullptr || y == nullptr) return fail(IE_EINVAL, "NULL argument");
  if (x == y) return fail(IE_EINVAL, "x and y must not overlap");
  if (form < IE_CONVENTIONAL || form > IE_SCATTER) return fail(IE_EINVAL, "unknown form %d", form);
  if (precision != IE_FP64 && precision != IE_MIXED)
    return fail(IE_EINVAL, "precision must be IE_FP64 or IE_MIXED");
  if (!(ctx->prec_mask & precision))
    return fail(IE_EINVAL, "context was set up without this precision");
  hipStream_t s = (hipStream_t)stream;
  Plan& p = *ctx->full;
  const long N = p.ncell();
  if (form != IE_GREEN_ONLY) IE_TRY(prepare_contrast(ctx, sigma6, form, s));
  double ax = 0, am = 0, as = 1;
  if (form == IE_CONVENTIONAL) {
    ax = 1;
    as = -1;
  } else if (form == IE_CIE) {
    ax = 1;
    am = 1;
    as = -2.0 * ctx->med.sigma0;
  }
  auto fill = [&](auto& a, auto* M) {
    a.x_cs = N;
    a.x_bs = 3 * N;
    a.M = form == IE_GREEN_ONLY ? nullptr : M;
    a.M_cs = N;
    a.M_bs = 6 * N;
    a.src_z0 = 0;
    a.src_z1 = p.nz;
    a.hole_z0 = a.hole_z1 = -1;
    a.out_z0 = 0;
    a.out_z1 = p.nz;
    a.y_cs = N;
    a.y_bs = 3 * N;
    a.e = nullptr;
    a.active = nullptr;
  };
  if (precision == IE_FP64) {
    MvArgs<double> a{};
    fill(a, ctx->M64.as<const double>());
    a.x = (const c128*)x;
    a.y = (c128*)y;
    a.a_x = ax;
    a.a_m = am;
    a.a_s = as;
    return launch_matvec<double>(p, a, 1, s, tw64(ctx));
  }
  MvArgs<float> a{};
  fill(a, ctx->M32.as<const float>());
  a.x = (const c64*)x;
  a.y = (c64*)y;
  a.a_x = float(ax);
  a.a_m = float(am);
  a.a_s = float(as);
  return launch_matvec<float>(p, a, 1, s, tw32(ctx));
}

int ie_gmres(ie_ctx* ctx, const double* sigma6, const void* b, void* x, const ie_gmres_opts* opts,
             ie_gmres_stats* stats, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (ctx == nullptr || b == nullptr || x == nullptr || opts == nullptr)
    return fail(IE_EINVAL, "NULL argument");
  if (opts->precision != IE_FP64 && opts->precision != IE_MIXED)
    return fail(IE_EINVAL, "precision must be IE_FP64 or IE_MIXED");
  if (!(ctx->prec_mask & opts->precision) || !(ctx->prec_mask & IE_FP64))
    return fail(IE_EINVAL, "context lacks the spectra this precision needs");
  if (opts->form != IE_CONVENTIONAL && opts->form != IE_CIE)
    return fail(IE_EINVAL, "form must be IE_CONVENTIONAL or IE_CIE");
  if (!(opts->tol >= 0) || opts->max_its < 1) return fail(IE_EINVAL, "bad tol or max_its");
  hipStream_t s = (hipStream_t)stream;
  Plan& p = *ctx->full;
  const long N = p.ncell();
  IE_TRY(prepare_contrast(ctx, sigma6, opts->form, s));
  OpDesc op;
  op.form = opts->form;
  op.sigma0 = ctx->med.sigma0;
  op.M64 = ctx->M64.as<const double>();
  op.M32 = ctx->M32.as<const float>();
  op.M_cs = N;
  op.M_bs = 6 * N;
  GmOpts o;
  o.tol = opts->tol;
  o.restart = opts->restart;
  o.max_its = opts->max_its;
  o.precision = opts->precision;
  if (opts->reorth < 0 || opts->reorth > 2) return fail(IE_EINVAL, "reorth must be 0, 1 or 2");
  o.reorth = opts->reorth == 2 ? 1 : 0;
  GmResult r;
  c128* xs = (c128*)x;
  const c128* rhs = (const c128*)b;
  if (opts->form == IE_CIE) {
    // C e = sqrt(sigma0) b with e = a x;  x = a^-1 e  (same relative residual as eq. 9)
    IE_TRY(ctx->xt.ensure(sizeof(c128) * 3 * N));
    IE_TRY(ctx->bt.ensure(sizeof(c128) * 3 * N));
    IE_TRY(launch_scale(rhs, ctx->bt.as<c128>(), std::sqrt(ctx->med.sigma0), 3 * N, s));
    IE_TRY(launch_tensor_apply(ctx->A64.as<double>(), N, xs, N, ctx->xt.as<c128>(), N, N, s));
    IE_TRY(gmres_solve(p, op, ctx->bt.as<c128>(), ctx->xt.as<c128>(), 1, o, &r, ctx->kw, tw64(ctx),
                       tw32(ctx), s));
    IE_TRY(launch_tensor_apply(ctx->Ai64.as<double>(), N, ctx->xt.as<c128>(), N, xs, N, N, s));
  } else {
    IE_TRY(gmres_solve(p, op, rhs, xs, 1, o, &r, ctx->kw, tw64(ctx), tw32(ctx), s));
  }
  IE_HIP(hipStreamSynchronize(s));
  if (stats) {
    stats->its = r.its;
    stats->restarts = r.cycles > 0 ? r.cycles - 1 : 0;
    stats->refinements = opts->precision == IE_MIXED ? r.cycles : 0;
    stats->matvecs64 = r.mv64;
    stats->matvecs32 = r.mv32;
    stats->graph_cycles = r.graph_cycles;
    stats->relres = r.relres;
    stats->seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (!r.converged)
    return fail(IE_ENOCONV, "GMRES stopped at relative residual %.3e after %d iterations",
                r.relres, r.its);
  return IE_OK;
}

}  // extern "C"
