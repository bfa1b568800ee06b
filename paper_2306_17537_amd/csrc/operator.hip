// Operator-level launches: the five-pass FFT convolution (eq. 10), the precomputed spectrum of
// the discretised Green's tensor (eqs. 5-7, section 2.2), the background field of point dipoles
// and the per-cell contrast tensors (eq. 3 and the contraction form).
#include <algorithm>
#include <cctype>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "ctx.hpp"
#include "prof.hpp"

namespace ie {

static std::string shape_tag(int esz, int LX, int LY, int LZ, int nz, int batch) {
  char b[96];
  snprintf(b, sizeof(b), "%s L%dx%dx%d nz%d b%d", esz == 8 ? "c64" : "c128", LX, LY, LZ, nz, batch);
  return b;
}

int fft_len(int n, bool pow2) {
  int L = 2;
  while (L < 2 * n - 1) L *= 2;
  if (pow2) return L;
  // 3 * 2^k from 24 up when it is the shorter admissible length
  int L3 = 24;
  while (L3 < 2 * n - 1) L3 *= 2;
  return (L3 < L && L3 <= 768) ? L3 : L;
}

// Calls F<T, L>::run(args...) for the FFT length L (2^k, or 3 * 2^k from 24).
#define IE_LEN_CASES(F, T, L, ...)                      \
  switch (L) {                                          \
    case 2: return F<T, 2>::run(__VA_ARGS__);           \
    case 4: return F<T, 4>::run(__VA_ARGS__);           \
    case 8: return F<T, 8>::run(__VA_ARGS__);           \
    case 16: return F<T, 16>::run(__VA_ARGS__);         \
    case 24: return F<T, 24>::run(__VA_ARGS__);         \
    case 32: return F<T, 32>::run(__VA_ARGS__);         \
    case 48: return F<T, 48>::run(__VA_ARGS__);         \
    case 64: return F<T, 64>::run(__VA_ARGS__);         \
    case 96: return F<T, 96>::run(__VA_ARGS__);         \
    case 128: return F<T, 128>::run(__VA_ARGS__);       \
    case 192: return F<T, 192>::run(__VA_ARGS__);       \
    case 256: return F<T, 256>::run(__VA_ARGS__);       \
    case 384: return F<T, 384>::run(__VA_ARGS__);       \
    case 512: return F<T, 512>::run(__VA_ARGS__);       \
    case 768: return F<T, 768>::run(__VA_ARGS__);       \
    case 1024: return F<T, 1024>::run(__VA_ARGS__);     \
    default: return fail(IE_EINVAL, "unsupported FFT length %d", L); \
  }

// Calls F<T, L>::template go<V>(args...) for the plan's variant v (lengths below 16 have one).
#define IE_VARIANTS(v, ...)                                              \
  if constexpr (L < 16) {                                                \
    return go<0>(__VA_ARGS__);                                           \
  } else {                                                               \
    switch (v) {                                                         \
      case 1: return go<1>(__VA_ARGS__);                                 \
      case 2: return go<2>(__VA_ARGS__);                                 \
      case 3: return go<3>(__VA_ARGS__);                                 \
      default: return go<0>(__VA_ARGS__);                                \
    }                                                                    \
  }

// The same for the row passes, which have eight variants.
#define IE_ROW_VARIANTS(v, ...)                                          \
  if constexpr (L < 16) {                                                \
    return go<0>(__VA_ARGS__);                                           \
  } else {                                                               \
    switch (v) {                                                         \
      case 1: return go<1>(__VA_ARGS__);                                 \
      case 2: return go<2>(__VA_ARGS__);                                 \
      case 3: return go<3>(__VA_ARGS__);                                 \
      case 4: return go<4>(__VA_ARGS__);                                 \
      case 5: return go<5>(__VA_ARGS__);                                 \
      case 6: return go<6>(__VA_ARGS__);                                 \
      case 7: return go<7>(__VA_ARGS__);                                 \
      default: return go<0>(__VA_ARGS__);                                \
    }                                                                    \
  }

// Calls F<T, L>::template go<V>(args...) for the plan's variant v of a z pass (two variants).
#define IE_Z_VARIANTS(v, ...)                                            \
  switch (v & 1) {                                                       \
    case 1: return go<1>(__VA_ARGS__);                                   \
    default: return go<0>(__VA_ARGS__);                                  \
  }

// number of source planes of an operator application
template <typename T>
static int source_planes(const MvArgs<T>& a) {
  const int z0 = std::max(a.src_z0, 0), z1 = std::min(a.src_z1, a.nz);
  int zs = std::max(0, z1 - z0);
  zs -= std::max(0, std::min(a.hole_z1, z1) - std::max(a.hole_z0, z0));
  return zs;
}

template <typename T, int L>
struct ZfwdL {
  template <int V>
  static int go(const MvArgs<T>& a, int batch, hipStream_t s) {
    using G = GeoC<T, L, V>;
    const long plane = long(a.ny) * a.nx;
    dim3 grid(ceil_div(plane, G::W), 1, batch);
    const double cs = sizeof(cx<T>), rs = sizeof(T);
    const double by = double(batch) * (double(source_planes(a)) * plane *
                                       (3 * cs + (a.M ? 6 * rs : 0)) + double(L) * plane * 3 * cs);
    ProfScope ps(s, "zfwd", shape_tag(int(cs), a.LX, a.LY, a.LZ, a.nz, batch).c_str(), by);
    hipLaunchKernelGGL((k_zfwd<T, L, V>), grid, dim3(G::THREADS), 0, s, a);
    IE_LAUNCH_CHECK();
    return IE_OK;
  }
  static int run(int v, const MvArgs<T>& a, int batch, hipStream_t s) {
    IE_Z_VARIANTS(v, a, batch, s);
  }
};
template <typename T, int L>
struct ZinvL {
  template <int V>
  static int go(const MvArgs<T>& a, int batch, hipStream_t s) {
    using G = GeoC<T, L, V>;
    const long plane = long(a.ny) * a.nx;
    dim3 grid(ceil_div(plane, G::W), 1, batch);
    const double cs = sizeof(cx<T>), rs = sizeof(T);
    const bool ux = a.x && (a.a_x != T(0) || (a.M && a.a_m != T(0)));
    const bool um = a.M && a.a_m != T(0);
    const double per = 3 * cs + (ux ? 3 * cs : 0) + (um ? 6 * rs : 0) + (a.e ? 3 * cs : 0);
    const double by = double(batch) * (double(L) * plane * 3 * cs +
                                       double(a.out_z1 - a.out_z0) * plane * per);
    ProfScope ps(s, "zinv", shape_tag(int(cs), a.LX, a.LY, a.LZ, a.nz, batch).c_str(), by);
    hipLaunchKernelGGL((k_zinv<T, L, V>), grid, dim3(G::THREADS), 0, s, a);
    IE_LAUNCH_CHECK();
    return IE_OK;
  }
  static int run(int v, const MvArgs<T>& a, int batch, hipStream_t s) {
    IE_Z_VARIANTS(v, a, batch, s);
  }
};
template <typename T, int L>
struct XconvL {
  template <int V>
  static int go(const MvArgs<T>& a, int batch, hipStream_t s) {
    const double cs = sizeof(cx<T>);
    // algorithmic bytes count the spectrum at its octant size (the unique values), read once
    const double oct = 6.0 * (L / 2 + 1) * (a.LY / 2 + 1) * (a.LZ / 2 + 1);
    const double by = double(batch) * 2.0 * a.LZ * a.LY * a.nx * 3 * cs + oct * cs;
    ProfScope ps(s, "xconv", shape_tag(int(cs), a.LX, a.LY, a.LZ, a.nz, batch).c_str(), by);
    // variants 4..7: one line per thread group where its LDS fits, else 0..3
    if constexpr (V >= 4 && GeoX2<T, L, V & 3>::FITS) {
      using G = GeoX2<T, L, V & 3>;
      // x extent: the LY/2 + 1 stored rows in groups of NP, rounded up to a multiple of 8 XCDs
      dim3 grid((ceil_div(a.LY / 2 + 1, G::NP) + 7) / 8 * 8, a.LZ, batch);
      hipLaunchKernelGGL((k_xconv2<T, L, V & 3>), grid, dim3(G::THREADS), 0, s, a);
    } else {
      using G = GeoX<T, L, V & 3>;
      dim3 grid((ceil_div(a.LY / 2 + 1, G::NP) + 7) / 8 * 8, a.LZ, batch);
      hipLaunchKernelGGL((k_xconv<T, L, V & 3>), grid, dim3(G::THREADS), 0, s, a);
    }
    IE_LAUNCH_CHECK();
    return IE_OK;
  }
  static int run(int v, const MvArgs<T>& a, int batch, hipStream_t s) {
    IE_ROW_VARIANTS(v, a, batch, s);
  }
};
template <typename T, int L>
struct ColL {
  // half: the operator's half-size lines (forward rows_in, inverse rows_out <= L/2); otherwise
  // a full-length forward transform (variant 0 only, for the Green setup)
  template <int V>
  static int go(const cx<T>* in, cx<T>* out, const ColArgs& c, int nplanes, int batch, bool inv,
                bool half, hipStream_t s, const cx<T>* tw) {
    using G = Geo<T, L, V>;
    dim3 grid(ceil_div(c.ncols, G::W), nplanes, batch);
    const double cs = sizeof(cx<T>);
    const double by = double(batch) * nplanes * double(c.ncols) * (c.rows_in + c.rows_out) * cs;
    char tg[96];
    snprintf(tg, sizeof(tg), "%s L%d planes%d cols%d b%d", cs == 8 ? "c64" : "c128", L, nplanes,
             c.ncols, batch);
    ProfScope ps(s, inv ? "yinv" : "yfwd", tg, by);
    if (half) {
      if (2 * (inv ? c.rows_out : c.rows_in) > L)
        return fail(IE_EINVAL, "column pass: %d rows exceed half of length %d",
                    inv ? c.rows_out : c.rows_in, L);
      if (inv)
        hipLaunchKernelGGL((k_colfft<T, L, true, V, true>), grid, dim3(G::W * G::TL), 0, s, in,
                           out, c, tw);
      else
        hipLaunchKernelGGL((k_colfft<T, L, false, V, true>), grid, dim3(G::W * G::TL), 0, s, in,
                           out, c, tw);
    } else {
      if constexpr (V == 0) {
        if (inv) return fail(IE_EINVAL, "full-length inverse column pass is not built");
        hipLaunchKernelGGL((k_colfft<T, L, false, 0, false>), grid, dim3(G::W * G::TL), 0, s, in,
                           out, c, tw);
      } else {
        return fail(IE_EINVAL, "full-length column pass has variant 0 only");
      }
    }
    IE_LAUNCH_CHECK();
    return IE_OK;
  }
  static int run(int v, const cx<T>* in, cx<T>* out, const ColArgs& c, int nplanes, int batch,
                 bool inv, bool half, hipStream_t s, const cx<T>* tw) {
    IE_VARIANTS(v, in, out, c, nplanes, batch, inv, half, s, tw);
  }
};

int Plan::work(int prec, int batch) {
  if (prec == IE_FP64) {
    if (batch > cap64) {
      IE_TRY(t1_64.ensure(sizeof(c128) * t1_elems() * batch));
      IE_TRY(t2_64.ensure(sizeof(c128) * t2_elems() * batch));
      cap64 = batch;
    }
  } else {
    if (batch > cap32) {
      IE_TRY(t1_32.ensure(sizeof(c64) * t1_elems() * batch));
      IE_TRY(t2_32.ensure(sizeof(c64) * t2_elems() * batch));
      cap32 = batch;
    }
  }
  return IE_OK;
}

template <typename T>
int launch_matvec(Plan& p, MvArgs<T> a, int batch, hipStream_t s, const cx<T>* tw, int only,
                  int vover) {
  constexpr bool dbl = sizeof(T) == 8;
  const int8_t* var = p.var[dbl ? 0 : 1];
  auto vsel = [&](int pass) { return vover >= 0 ? vover : int(var[pass]); };
  auto want = [&](int pass) { return only < 0 || only == pass; };
  // padded work: the caller's (both T1 and T2 set, one problem) or the plan's own buffers
  const bool own_work = a.T1 == nullptr || a.T2 == nullptr;
  if (!own_work && batch != 1) return fail(IE_EINVAL, "caller work buffers hold one problem");
  if (own_work) {
    IE_TRY(p.work(dbl ? IE_FP64 : IE_MIXED, batch));
    a.T1 = dbl ? (cx<T>*)p.t1_64.p : (cx<T>*)p.t1_32.p;
    a.T2 = dbl ? (cx<T>*)p.t2_64.p : (cx<T>*)p.t2_32.p;
  }
  a.nx = p.nx;
  a.ny = p.ny;
  a.nz = p.nz;
  a.LX = p.LX;
  a.LY = p.LY;
  a.LZ = p.LZ;
  a.T1_bs = p.t1_elems();
  a.T2_bs = p.t2_elems();
  a.ghat = dbl ? (const cx<T>*)p.ghat64.p : (const cx<T>*)p.ghat32.p;
  a.ghat_bs = 0;
  a.tw = tw;
  if (a.ghat == nullptr) return fail(IE_ESTATE, "spectrum for this precision was not built");
  if (a.out_z0 < 0 || a.out_z1 > p.nz || a.out_z0 >= a.out_z1)
    return fail(IE_EINVAL, "bad output plane range [%d, %d)", a.out_z0, a.out_z1);
  if (batch < 1 || batch > 65535) return fail(IE_EINVAL, "bad batch %d", batch);

  // pass 1: contrast on the source planes, pad, FFT along z (all three components per column)
  auto zf = [&]() -> int { IE_LEN_CASES(ZfwdL, T, p.LZ, vsel(0), a, batch, s); };
  if (want(0)) IE_TRY(zf());
  // pass 2: FFT along y (ny non-zero rows -> LY) on every kz plane
  ColArgs c{};
  c.ncols = p.nx;
  c.nzp = p.LZ;
  c.z0 = 0;
  c.in_cs = long(p.LZ) * p.ny * p.nx;
  c.in_zs = long(p.ny) * p.nx;
  c.in_ls = p.nx;
  c.out_cs = long(p.LZ) * p.LY * p.nx;
  c.out_zs = long(p.LY) * p.nx;
  c.out_ls = p.nx;
  c.rows_in = p.ny;
  c.rows_out = p.LY;
  c.in_bs = a.T1_bs;
  c.out_bs = a.T2_bs;
  c.active = a.active;
  c.active_bs = a.active_bs;
  auto col = [&](const cx<T>* in, cx<T>* out, const ColArgs& cc, bool inv) -> int {
    IE_LEN_CASES(ColL, T, p.LY, vsel(inv ? 3 : 1), in, out, cc, 3 * p.LZ, batch, inv, true, s,
                 tw);
  };
  if (want(1)) IE_TRY(col(a.T1, a.T2, c, false));
  // pass 3: FFT along x, tensor multiply with G^, inverse FFT along x (rows of every (ky, kz))
  auto xc = [&]() -> int { IE_LEN_CASES(XconvL, T, p.LX, vsel(2), a, batch, s); };
  if (want(2)) IE_TRY(xc());
  // pass 4: inverse FFT along y (LY -> ny rows)
  ColArgs d = c;
  d.in_cs = c.out_cs;
  d.in_zs = c.out_zs;
  d.in_ls = c.out_ls;
  d.out_cs = c.in_cs;
  d.out_zs = c.in_zs;
  d.out_ls = c.in_ls;
  d.rows_in = p.LY;
  d.rows_out = p.ny;
  d.in_bs = a.T2_bs;
  d.out_bs = a.T1_bs;
  if (want(3)) IE_TRY(col(a.T2, a.T1, d, true));
  // pass 5: inverse FFT along z, keep the output planes, combine
  auto zi = [&]() -> int { IE_LEN_CASES(ZinvL, T, p.LZ, vsel(4), a, batch, s); };
  if (want(4)) IE_TRY(zi());
  return IE_OK;
}

template int launch_matvec<double>(Plan&, MvArgs<double>, int, hipStream_t, const c128*, int, int);
template int launch_matvec<float>(Plan&, MvArgs<float>, int, hipStream_t, const c64*, int, int);

// ---------------------------------------------------------------------------------------
// Autotuner: every launch variant of every pass is timed inside the whole operator (HIP events,
// one warm-up application, then the average of kReps applications) on the plan's own work
// buffers with zero inputs, and the fastest is kept.  Results are cached per (GPU architecture,
// precision, grid, FFT lengths) for the process, and can be saved to and loaded from a file.
// ---------------------------------------------------------------------------------------
namespace {
struct TuneEntry {
  int8_t var[5];
  float us[5][kRowVariants];
};
using TuneKey = std::tuple<std::string, int, int, int, int, int, int, int>;
std::map<TuneKey, TuneEntry> g_tune_cache;
std::mutex g_tune_mu;
constexpr int kReps = 5;
constexpr int kRunoffRounds = 3;
constexpr float kRunoffMargin = 0.05f;

int device_arch(std::string& arch) {
  int dev = 0;
  IE_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  IE_HIP(hipGetDeviceProperties(&prop, dev));
  arch = prop.gcnArchName;
  return IE_OK;
}

// The contraction-form operator on zero inputs over the plan's own work buffers, timed with HIP
// events on stream s at the plan's current variants.
template <typename T>
struct OpTimer {
  Plan& p;
  const cx<T>* tw;
  hipStream_t s;
  DevBuf x, y, M;
  MvArgs<T> a{};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  OpTimer(Plan& p_, const cx<T>* tw_, hipStream_t s_) : p(p_), tw(tw_), s(s_) {}
  ~OpTimer() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
  int init() {
    constexpr bool dbl = sizeof(T) == 8;
    IE_TRY(p.work(dbl ? IE_FP64 : IE_MIXED, 1));
    const long N = p.ncell();
    IE_TRY(x.ensure(sizeof(cx<T>) * 3 * N));
    IE_TRY(y.ensure(sizeof(cx<T>) * 3 * N));
    IE_TRY(M.ensure(sizeof(T) * 6 * N));
    IE_HIP(hipMemsetAsync(x.p, 0, sizeof(cx<T>) * 3 * N, s));
    IE_HIP(hipMemsetAsync(M.p, 0, sizeof(T) * 6 * N, s));
    IE_HIP(hipMemsetAsync(dbl ? p.t1_64.p : p.t1_32.p, 0, sizeof(cx<T>) * p.t1_elems(), s));
    IE_HIP(hipMemsetAsync(dbl ? p.t2_64.p : p.t2_32.p, 0, sizeof(cx<T>) * p.t2_elems(), s));
    a.x = x.as<const cx<T>>();  // reads x and the contrast, writes y
    a.x_cs = N;
    a.x_bs = 3 * N;
    a.M = M.as<const T>();
    a.M_cs = N;
    a.M_bs = 6 * N;
    a.src_z0 = 0;
    a.src_z1 = p.nz;
    a.hole_z0 = a.hole_z1 = -1;
    a.out_z0 = 0;
    a.out_z1 = p.nz;
    a.y = y.as<cx<T>>();
    a.y_cs = N;
    a.y_bs = 3 * N;
    a.a_x = 1;
    a.a_m = 1;
    a.a_s = -1;
    IE_HIP(hipEventCreate(&e0));
    IE_HIP(hipEventCreate(&e1));
    return IE_OK;
  }
  // one warm-up application, then the average of kReps
  int time(float& us) {
    IE_TRY(launch_matvec<T>(p, a, 1, s, tw));
    IE_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < kReps; ++r) IE_TRY(launch_matvec<T>(p, a, 1, s, tw));
    float ms = 0;
    IE_HIP(hipEventRecord(e1, s));
    IE_HIP(hipEventSynchronize(e1));
    IE_HIP(hipEventElapsedTime(&ms, e0, e1));
    us = 1e3f * ms / kReps;
    return IE_OK;
  }
};
}  // namespace

template <typename T>
static int tune_one(Plan& p, const cx<T>* tw, hipStream_t s, int8_t var[5],
                    float us[5][kRowVariants]) {
  constexpr bool dbl = sizeof(T) == 8;
  OpTimer<T> tm(p, tw, s);
  IE_TRY(tm.init());
  // one sweep over the passes: each variant of a pass is timed inside the whole operator (the
  // other passes at their current choice), so that every pass reads its input from wherever the
  // previous pass left it, as in use
  int8_t* pv = p.var[dbl ? 0 : 1];
  for (int q = 0; q < 5; ++q) pv[q] = 0;
  for (int pass = 0; pass < 5; ++pass) {
    float best = 0;
    int8_t keep = 0;
    const int nv = pass == 2 ? kRowVariants : (pass == 1 || pass == 3 ? kVariants : kZVariants);
    for (int v = 0; v < nv; ++v) {
      pv[pass] = int8_t(v);
      IE_TRY(tm.time(us[pass][v]));
      if (v == 0 || us[pass][v] < best) {
        best = us[pass][v];
        keep = int8_t(v);
      }
    }
    // runoff: a runner-up within kRunoffMargin of the best is timed again against it,
    // alternately, kRunoffRounds times each, and the lower median wins (one sweep alone flips
    // between variants a few percent apart from run to run)
    int8_t alt = -1;
    for (int v = 0; v < nv; ++v)
      if (v != keep && (alt < 0 || us[pass][v] < us[pass][alt])) alt = int8_t(v);
    if (alt >= 0 && us[pass][alt] <= best * (1.0f + kRunoffMargin)) {
      float ta[kRunoffRounds], tb[kRunoffRounds];
      for (int r = 0; r < kRunoffRounds; ++r) {
        pv[pass] = keep;
        IE_TRY(tm.time(ta[r]));
        pv[pass] = alt;
        IE_TRY(tm.time(tb[r]));
      }
      std::sort(ta, ta + kRunoffRounds);
      std::sort(tb, tb + kRunoffRounds);
      us[pass][keep] = ta[kRunoffRounds / 2];
      us[pass][alt] = tb[kRunoffRounds / 2];
      if (us[pass][alt] < us[pass][keep]) keep = alt;
    }
    pv[pass] = keep;
  }
  for (int q = 0; q < 5; ++q) var[q] = pv[q];
  return IE_OK;
}

int autotune(Plan& p, int prec_mask, const c128* tw64, const c64* tw32, hipStream_t s) {
  std::string arch;
  IE_TRY(device_arch(arch));
  for (int pi = 0; pi < 2; ++pi) {
    const bool dbl = pi == 0;
    if (!(prec_mask & (dbl ? IE_FP64 : IE_MIXED))) continue;
    const TuneKey key{arch, pi, p.nx, p.ny, p.nz, p.LX, p.LY, p.LZ};
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) {
        std::memcpy(p.var[pi], it->second.var, sizeof(p.var[pi]));
        std::memcpy(p.tune_us[pi], it->second.us, sizeof(p.tune_us[pi]));
        continue;
      }
    }
    TuneEntry t{};
    if (dbl)
      IE_TRY(tune_one<double>(p, tw64, s, t.var, t.us));
    else
      IE_TRY(tune_one<float>(p, tw32, s, t.var, t.us));
    std::memcpy(p.var[pi], t.var, sizeof(p.var[pi]));
    std::memcpy(p.tune_us[pi], t.us, sizeof(p.tune_us[pi]));
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[key] = t;
  }
  return IE_OK;
}

// Template name of the kernel that runs pass q (0 zfwd, 1 yfwd, 2 xconv, 3 yinv, 4 zinv) of the
// plan at precision pi (0 float64, 1 complex64) with its current variant, as profilers print it.
namespace {
template <typename T, int L>
struct X2Fits {
  static int run(int v) {
    switch (v & 3) {
      case 1: return GeoX2<T, L, 1>::FITS ? 1 : 0;
      case 2: return GeoX2<T, L, 2>::FITS ? 1 : 0;
      case 3: return GeoX2<T, L, 3>::FITS ? 1 : 0;
      default: return GeoX2<T, L, 0>::FITS ? 1 : 0;
    }
  }
};
template <typename T>
int x2_fits(int L, int v) {
  IE_LEN_CASES(X2Fits, T, L, v);
}
}  // namespace

std::string pass_kernel(const Plan& p, int pi, int q) {
  const char* t = pi == 0 ? "double" : "float";
  const int v = p.var[pi][q];
  char b[96];
  if (q == 0 || q == 4) {
    snprintf(b, sizeof(b), "%s<%s, %d, %d>", q == 0 ? "k_zfwd" : "k_zinv", t, p.LZ, v & 1);
  } else if (q == 1 || q == 3) {
    snprintf(b, sizeof(b), "k_colfft<%s, %d, %s, %d, true>", t, p.LY, q == 3 ? "true" : "false",
             p.LY < 16 ? 0 : v & 3);
  } else if (p.LX < 16) {
    snprintf(b, sizeof(b), "k_xconv<%s, %d, 0>", t, p.LX);
  } else {
    const bool two = v >= 4 && (pi == 0 ? x2_fits<double>(p.LX, v) : x2_fits<float>(p.LX, v)) == 1;
    snprintf(b, sizeof(b), "%s<%s, %d, %d>", two ? "k_xconv2" : "k_xconv", t, p.LX, v & 3);
  }
  return b;
}

int operator_us(Plan& p, int prec_mask, const c128* tw64, const c64* tw32, hipStream_t s,
                float& us) {
  us = 0;
  for (int pi = 0; pi < 2; ++pi) {
    float t = 0;
    if (!(prec_mask & (pi == 0 ? IE_FP64 : IE_MIXED))) continue;
    if (pi == 0) {
      OpTimer<double> tm(p, tw64, s);
      IE_TRY(tm.init());
      IE_TRY(tm.time(t));
    } else {
      OpTimer<float> tm(p, tw32, s);
      IE_TRY(tm.init());
      IE_TRY(tm.time(t));
    }
    us += t;
  }
  return IE_OK;
}

// ---- saving and loading the cache ----------------------------------------------------------
// File format: a JSON array with one object per (architecture, precision, grid, FFT lengths):
//   {"arch": "...", "precision": "c128"|"c64", "grid": [nx, ny, nz], "fft": [LX, LY, LZ],
//    "variant": [5 ints], "us": [[8 numbers] x 5]}
namespace {
struct JsonIn {  // minimal reader for the format above
  const std::string& t;
  size_t i = 0;
  explicit JsonIn(const std::string& s) : t(s) {}
  void ws() {
    while (i < t.size() && std::isspace(static_cast<unsigned char>(t[i]))) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < t.size() && t[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool str(std::string& out) {
    if (!eat('"')) return false;
    out.clear();
    while (i < t.size() && t[i] != '"') {
      if (t[i] == '\\') return false;  // no escapes in this format
      out += t[i++];
    }
    return eat('"');
  }
  bool num(double& v) {
    ws();
    const char* b = t.c_str() + i;
    char* e = nullptr;
    v = std::strtod(b, &e);
    if (e == b) return false;
    i += size_t(e - b);
    return true;
  }
  bool ints(int* v, int n) {
    if (!eat('[')) return false;
    for (int k = 0; k < n; ++k) {
      double d;
      if ((k > 0 && !eat(',')) || !num(d) || d != double(int(d))) return false;
      v[k] = int(d);
    }
    return eat(']');
  }
  bool nums(float* v, int n) {
    if (!eat('[')) return false;
    for (int k = 0; k < n; ++k) {
      double d;
      if ((k > 0 && !eat(',')) || !num(d)) return false;
      v[k] = float(d);
    }
    return eat(']');
  }
};

bool valid_len(int n, int L) {
  return L >= 2 && L >= 2 * n - 1 && L <= MAX_FFT_LEN && (L == fft_len(n, true) || L == fft_len(n, false));
}
}  // namespace

int tuning_save(const char* path) {
  std::string o = "[";
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (const auto& kv : g_tune_cache) {
      const auto& k = kv.first;
      const TuneEntry& e = kv.second;
      char t[320];
      snprintf(t, sizeof(t),
               "%s\n{\"arch\": \"%s\", \"precision\": \"%s\", \"grid\": [%d, %d, %d], "
               "\"fft\": [%d, %d, %d], \"variant\": [%d, %d, %d, %d, %d], \"us\": [",
               o.size() > 1 ? "," : "", std::get<0>(k).c_str(), std::get<1>(k) == 0 ? "c128" : "c64",
               std::get<2>(k), std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k),
               std::get<7>(k), e.var[0], e.var[1], e.var[2], e.var[3], e.var[4]);
      o += t;
      for (int q = 0; q < 5; ++q) {
        o += q ? ", [" : "[";
        for (int v = 0; v < kRowVariants; ++v) {
          snprintf(t, sizeof(t), "%s%.9g", v ? ", " : "", double(e.us[q][v]));
          o += t;
        }
        o += "]";
      }
      o += "]}";
    }
  }
  o += "\n]\n";
  FILE* f = std::fopen(path, "wb");
  if (f == nullptr) return fail(IE_EINVAL, "cannot open %s for writing", path);
  const bool ok = std::fwrite(o.data(), 1, o.size(), f) == o.size();
  if (std::fclose(f) != 0 || !ok) return fail(IE_EINVAL, "cannot write %s", path);
  return IE_OK;
}

int tuning_load(const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (f == nullptr) return fail(IE_EINVAL, "cannot open %s", path);
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  std::fclose(f);
  JsonIn in(text);
  std::vector<std::pair<TuneKey, TuneEntry>> entries;
  if (!in.eat('[')) return fail(IE_EINVAL, "%s: expected a JSON array", path);
  bool first = true;
  while (!in.eat(']')) {
    if (!first && !in.eat(',')) return fail(IE_EINVAL, "%s: expected ',' at byte %zu", path, in.i);
    first = false;
    std::string arch, prec;
    int grid[3] = {0, 0, 0}, fft[3] = {0, 0, 0}, var[5] = {0, 0, 0, 0, 0};
    TuneEntry e{};
    bool have[6] = {false, false, false, false, false, false};
    if (!in.eat('{')) return fail(IE_EINVAL, "%s: expected an object at byte %zu", path, in.i);
    bool firstk = true;
    while (!in.eat('}')) {
      std::string key;
      if ((!firstk && !in.eat(',')) || !in.str(key) || !in.eat(':'))
        return fail(IE_EINVAL, "%s: bad key at byte %zu", path, in.i);
      firstk = false;
      bool ok = false;
      if (key == "arch") {
        ok = in.str(arch);
        have[0] = true;
      } else if (key == "precision") {
        ok = in.str(prec);
        have[1] = true;
      } else if (key == "grid") {
        ok = in.ints(grid, 3);
        have[2] = true;
      } else if (key == "fft") {
        ok = in.ints(fft, 3);
        have[3] = true;
      } else if (key == "variant") {
        ok = in.ints(var, 5);
        have[4] = true;
      } else if (key == "us") {
        ok = in.eat('[');
        for (int q = 0; q < 5 && ok; ++q) ok = (q == 0 || in.eat(',')) && in.nums(e.us[q], kRowVariants);
        ok = ok && in.eat(']');
        have[5] = true;
      }
      if (!ok) return fail(IE_EINVAL, "%s: bad value of \"%s\" at byte %zu", path, key.c_str(), in.i);
    }
    for (bool h : have)
      if (!h) return fail(IE_EINVAL, "%s: entry %zu lacks a field", path, entries.size());
    if (prec != "c128" && prec != "c64")
      return fail(IE_EINVAL, "%s: entry %zu: unknown precision", path, entries.size());
    for (int a = 0; a < 3; ++a)
      if (grid[a] < 1 || grid[a] > 512 || !valid_len(grid[a], fft[a]))
        return fail(IE_EINVAL, "%s: entry %zu: grid or FFT length out of range", path, entries.size());
    for (int q = 0; q < 5; ++q) {
      if (var[q] < 0 || var[q] >= (q == 2 ? kRowVariants : (q == 1 || q == 3 ? kVariants : kZVariants)))
        return fail(IE_EINVAL, "%s: entry %zu: variant out of range", path, entries.size());
      e.var[q] = int8_t(var[q]);
    }
    entries.emplace_back(TuneKey{arch, prec == "c128" ? 0 : 1, grid[0], grid[1], grid[2], fft[0],
                                 fft[1], fft[2]},
                         e);
  }
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (const auto& kv : entries) g_tune_cache[kv.first] = kv.second;
  return IE_OK;
}

// ---------------------------------------------------------------------------------------
// Green setup
// ---------------------------------------------------------------------------------------

// Discretised G on the padded grid: offset d (per axis d in [-(n-1), n-1], stored at d mod L),
// G^E(d h) h^3 off the self cell (eq. 5 with grad grad g expanded), the ball integral on it.
__global__ void k_green_eval(c128* __restrict__ out, int nx, int ny, int nz, int LX, int LY, int LZ,
                             double h, double k0re, double k0im, double sigma0, c128 gself) {
  const long Lt = long(LX) * LY * LZ;
  const long idx = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= Lt) return;
  const int kx = int(idx % LX);
  const int ky = int((idx / LX) % LY);
  const int kz = int(idx / (long(LX) * LY));
  auto off = [](int k, int n, int L, bool& ok) {
    if (k <= n - 1) return k;
    if (k >= L - n + 1) return k - L;
    ok = false;
    return 0;
  };
  bool ok = true;
  const int dx = off(kx, nx, LX, ok), dy = off(ky, ny, LY, ok), dz = off(kz, nz, LZ, ok);
  c128 g[6] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
  if (ok) {
    if (dx == 0 && dy == 0 && dz == 0) {
      g[0] = g[1] = g[2] = gself;
    } else {
      const double rx = dx * h, ry = dy * h, rz = dz * h;
      const double R = sqrt(rx * rx + ry * ry + rz * rz);
      const double u[3] = {rx / R, ry / R, rz / R};
      // exp(i k0 R) = exp(-k0im R) (cos(k0re R) + i sin(k0re R))
      double sn, cs;
      sincos(k0re * R, &sn, &cs);
      const double mag = exp(-k0im * R);
      const c128 eikr = {mag * cs, mag * sn};
      const double inv = h * h * h / (4.0 * M_PI * sigma0 * R * R * R);
      const c128 pref = inv * eikr;
      const c128 kR = {k0re * R, k0im * R};
      const c128 kR2 = kR * kR;
      const c128 ikR = {-kR.im, kR.re};
      const c128 A = {kR2.re + ikR.re - 1.0, kR2.im + ikR.im};
      const c128 B = {3.0 - 3.0 * ikR.re - kR2.re, -3.0 * ikR.im - kR2.im};
      const c128 pa = pref * A, pb = pref * B;
      g[0] = pa + (u[0] * u[0]) * pb;
      g[1] = pa + (u[1] * u[1]) * pb;
      g[2] = pa + (u[2] * u[2]) * pb;
      g[3] = (u[0] * u[1]) * pb;
      g[4] = (u[0] * u[2]) * pb;
      g[5] = (u[1] * u[2]) * pb;
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) out[c * Lt + idx] = g[c];
}

// Row FFT (contiguous lines of length L), in place, full length.
template <typename T, int L, bool INV>
__global__ void __launch_bounds__((Geo<T, L>::NL * Geo<T, L>::TLR))
    k_rowfft(cx<T>* buf, long nrows, const cx<T>* __restrict__ tw) {
  using G = Geo<T, L>;
  constexpr int E = G::ER, TL = G::TLR, NL = G::NL;
  __shared__ cx<T> lds[NL * G::LP];
  const int t = threadIdx.x % TL;
  const int line = threadIdx.x / TL;
  const long row = long(blockIdx.x) * NL + line;
  const bool live = row < nrows;
  cx<T>* p = buf + (live ? row : 0) * L;
  cx<T> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = live ? p[t + m * TL] : cx<T>{0, 0};
  fft_line<T, L, E, INV>(v, lds, LdsPadded{line * G::LP}, t, tw);
  if (live) {
#pragma unroll
    for (int m = 0; m < E; ++m) p[t + m * TL] = v[m];
  }
}

template <typename T, int L>
struct RowL {
  static int run(cx<T>* buf, long nrows, hipStream_t s, const cx<T>* tw) {
    using G = Geo<T, L>;
    hipLaunchKernelGGL((k_rowfft<T, L, false>), dim3(ceil_div(nrows, G::NL)), dim3(G::NL * G::TLR),
                       0, s, buf, nrows, tw);
    IE_LAUNCH_CHECK();
    return IE_OK;
  }
};

// the stored octant of the spectrum: kx <= LX/2, ky <= LY/2, kz <= LZ/2
// ([6][LZ/2+1][LY/2+1][LX/2+1]); the other octants follow from the parity of each component
__global__ void k_octspec(const c128* __restrict__ full, c128* __restrict__ o64,
                          c64* __restrict__ o32, int LX, int LY, int LZ, double scale) {
  const int hx = LX / 2 + 1, hy = LY / 2 + 1, hz = LZ / 2 + 1;
  const long n = 6L * hx * hy * hz;
  const long idx = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int ox = int(idx % hx);
  const int oy = int((idx / hx) % hy);
  const int oz = int((idx / (long(hx) * hy)) % hz);
  const int c = int(idx / (long(hx) * hy * hz));
  const long Lt = long(LX) * LY * LZ;
  const c128 v = scale * full[c * Lt + (long(oz) * LY + oy) * LX + ox];
  if (o64) o64[idx] = v;
  if (o32) o32[idx] = c64{float(v.re), float(v.im)};
}

int build_green(Plan& p, double h, const Medium& m, int prec_mask, const c128* tw64, const c64*,
                hipStream_t s) {
  const long Lt = long(p.LX) * p.LY * p.LZ;
  DevBuf full;
  IE_TRY(full.ensure(sizeof(c128) * 6 * Lt));
  // self-cell ball integral [2 (1 - i k0 a) e^{i k0 a} - 3] / (3 sigma0), a^3 = 3 h^3 / (4 pi)
  const std::complex<double> k0(m.k0re, m.k0im), I(0.0, 1.0);
  const double arad = std::cbrt(3.0 * h * h * h / (4.0 * M_PI));
  const std::complex<double> gs =
      (2.0 * (1.0 - I * k0 * arad) * std::exp(I * k0 * arad) - 3.0) / (3.0 * m.sigma0);
  hipLaunchKernelGGL(k_green_eval, dim3(ceil_div(Lt, 256)), dim3(256), 0, s, full.as<c128>(), p.nx,
                     p.ny, p.nz, p.LX, p.LY, p.LZ, h, m.k0re, m.k0im, m.sigma0,
                     c128{gs.real(), gs.imag()});
  IE_LAUNCH_CHECK();
  for (int c = 0; c < 6; ++c) {
    c128* b = full.as<c128>() + c * Lt;
    {
      auto f = [&]() -> int { IE_LEN_CASES(RowL, double, p.LX, b, Lt / p.LX, s, tw64); };
      IE_TRY(f());
    }
    ColArgs ca{};
    ca.ncols = p.LX;
    ca.active = nullptr;
    // y axis: planes = z
    ca.nzp = p.LZ;
    ca.z0 = 0;
    ca.in_cs = ca.out_cs = 0;
    ca.in_zs = ca.out_zs = long(p.LY) * p.LX;
    ca.in_ls = ca.out_ls = p.LX;
    ca.rows_in = ca.rows_out = p.LY;
    {
      auto f = [&]() -> int {
        IE_LEN_CASES(ColL, double, p.LY, 0, b, b, ca, p.LZ, 1, false, false, s, tw64);
      };
      IE_TRY(f());
    }
    // z axis: planes = y
    ca.nzp = p.LY;
    ca.in_zs = ca.out_zs = p.LX;
    ca.in_ls = ca.out_ls = long(p.LY) * p.LX;
    ca.rows_in = ca.rows_out = p.LZ;
    {
      auto f = [&]() -> int {
        IE_LEN_CASES(ColL, double, p.LZ, 0, b, b, ca, p.LY, 1, false, false, s, tw64);
      };
      IE_TRY(f());
    }
  }
  const long no = p.spec_elems();
  c128* o64 = nullptr;
  c64* o32 = nullptr;
  if (prec_mask & IE_FP64) {
    IE_TRY(p.ghat64.ensure(sizeof(c128) * no));
    o64 = p.ghat64.as<c128>();
  }
  if (prec_mask & IE_MIXED) {
    IE_TRY(p.ghat32.ensure(sizeof(c64) * no));
    o32 = p.ghat32.as<c64>();
  }
  hipLaunchKernelGGL(k_octspec, dim3(ceil_div(no, 256)), dim3(256), 0, s, full.as<c128>(), o64, o32,
                     p.LX, p.LY, p.LZ, 1.0 / double(Lt));
  IE_LAUNCH_CHECK();
  IE_HIP(hipStreamSynchronize(s));  // `full` is released on return
  return IE_OK;
}

// ---------------------------------------------------------------------------------------
// background field of point dipoles
// ---------------------------------------------------------------------------------------
constexpr int kSrcPerLaunch = 8;
struct SrcPack {
  int n;
  double pos[kSrcPerLaunch][3];
  double mom[kSrcPerLaunch][3];
  int kind[kSrcPerLaunch];
};

__global__ void k_background(c128* __restrict__ E0, int nx, int ny, int nz, double h, double ox,
                             double oy, double oz, double omu, double k0re, double k0im,
                             double sigma0, SrcPack sp, int accumulate) {
  const long N = long(nx) * ny * nz;
  const long idx = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= N) return;
  const int i = int(idx % nx), j = int((idx / nx) % ny), k = int(idx / (long(nx) * ny));
  const double r[3] = {ox + (i + 0.5) * h, oy + (j + 0.5) * h, oz + (k + 0.5) * h};
  c128 E[3] = {{0, 0}, {0, 0}, {0, 0}};
  for (int s = 0; s < sp.n; ++s) {
    const double Rv[3] = {r[0] - sp.pos[s][0], r[1] - sp.pos[s][1], r[2] - sp.pos[s][2]};
    const double R = sqrt(Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2]);
    const double u[3] = {Rv[0] / R, Rv[1] / R, Rv[2] / R};
    double sn, cs;
    sincos(k0re * R, &sn, &cs);
    const double mag = exp(-k0im * R);
    const c128 eikr = {mag * cs, mag * sn};
    const c128 kR = {k0re * R, k0im * R};
    const double* mm = sp.mom[s];
    if (sp.kind[s] == IE_MAG_DIPOLE) {
      // i omega mu0 (1 - i k0 R) e^{i k0 R} / (4 pi R^2) (m x Rhat)
      const c128 one_m_ikR = {1.0 + kR.im, -kR.re};
      const c128 amp = (omu / (4.0 * M_PI * R * R)) * (c128{0.0, 1.0} * (one_m_ikR * eikr));
      const double cr[3] = {mm[1] * u[2] - mm[2] * u[1], mm[2] * u[0] - mm[0] * u[2],
                            mm[0] * u[1] - mm[1] * u[0]};
      for (int c = 0; c < 3; ++c) E[c] = E[c] + cr[c] * amp;
    } else {
      // G^E(R) p
      const c128 pref = (1.0 / (4.0 * M_PI * sigma0 * R * R * R)) * eikr;
      const c128 kR2 = kR * kR;
      const c128 ikR = {-kR.im, kR.re};
      const c128 A = {kR2.re + ikR.re - 1.0, kR2.im + ikR.im};
      const c128 B = {3.0 - 3.0 * ikR.re - kR2.re, -3.0 * ikR.im - kR2.im};
      const double up = u[0] * mm[0] + u[1] * mm[1] + u[2] * mm[2];
      for (int c = 0; c < 3; ++c) E[c] = E[c] + pref * (mm[c] * A + (u[c] * up) * B);
    }
  }
  for (int c = 0; c < 3; ++c) {
    const long o = c * N + idx;
    E0[o] = accumulate ? E0[o] + E[c] : E[c];
  }
}

int launch_background(int nx, int ny, int nz, double h, const double origin[3], const Medium& m,
                      const ie_source* src, int nsrc, c128* E0, hipStream_t s) {
  const long N = long(nx) * ny * nz;
  for (int s0 = 0; s0 < nsrc; s0 += kSrcPerLaunch) {
    SrcPack sp{};
    sp.n = nsrc - s0 < kSrcPerLaunch ? nsrc - s0 : kSrcPerLaunch;
    for (int q = 0; q < sp.n; ++q) {
      for (int c = 0; c < 3; ++c) {
        sp.pos[q][c] = src[s0 + q].pos[c];
        sp.mom[q][c] = src[s0 + q].moment[c];
      }
      sp.kind[q] = src[s0 + q].kind;
    }
    hipLaunchKernelGGL(k_background, dim3(ceil_div(N, 256)), dim3(256), 0, s, E0, nx, ny, nz, h,
                       origin[0], origin[1], origin[2], m.omega * m.mu0, m.k0re, m.k0im, m.sigma0,
                       sp, s0 > 0 ? 1 : 0);
    IE_LAUNCH_CHECK();
  }
  return IE_OK;
}

// ---------------------------------------------------------------------------------------
// contrast preparation
// ---------------------------------------------------------------------------------------
__global__ void k_prep(const double* __restrict__ s6, long N, double sigma0, int form,
                       double* __restrict__ M, float* __restrict__ Mf, double* __restrict__ A,
                       double* __restrict__ Ai, int* __restrict__ bad) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s[6];
  for (int c = 0; c < 6; ++c) s[c] = s6[c * N + i];
  bool ok = true;
  for (int c = 0; c < 6; ++c) ok = ok && isfinite(s[c]);
  // Sylvester's criterion on sigma (xx, yy, zz, xy, xz, yz)
  const double m2 = s[0] * s[1] - s[3] * s[3];
  const double det = s[0] * (s[1] * s[2] - s[5] * s[5]) - s[3] * (s[3] * s[2] - s[5] * s[4]) +
                     s[4] * (s[3] * s[5] - s[1] * s[4]);
  ok = ok && s[0] > 0.0 && m2 > 0.0 && det > 0.0;
  if (!ok) atomicOr(bad, 1);
  double out[6];
  if (form == IE_CIE) {
    // P = sigma + sigma0 I = 2 sigma0 I + dsigma;  b = I - 2 sigma0 P^-1;  a = P / (2 sqrt sigma0)
    const double a = s[0] + sigma0, b = s[1] + sigma0, c = s[2] + sigma0;
    const double d = s[3], e = s[4], f = s[5];
    const double cxx = b * c - f * f, cyy = a * c - e * e, czz = a * b - d * d;
    const double cxy = e * f - d * c, cxz = d * f - b * e, cyz = d * e - a * f;
    const double dt = a * cxx + d * cxy + e * cxz;
    const double inv[6] = {cxx / dt, cyy / dt, czz / dt, cxy / dt, cxz / dt, cyz / dt};
    const double ts = 2.0 * sqrt(sigma0);
    for (int q = 0; q < 6; ++q) out[q] = (q < 3 ? 1.0 : 0.0) - 2.0 * sigma0 * inv[q];
    const double P[6] = {a, b, c, d, e, f};
    if (A)
      for (int q = 0; q < 6; ++q) A[q * N + i] = P[q] / ts;
    if (Ai)
      for (int q = 0; q < 6; ++q) Ai[q * N + i] = ts * inv[q];
  } else {
    for (int q = 0; q < 6; ++q) out[q] = s[q] - (q < 3 ? sigma0 : 0.0);
  }
  for (int q = 0; q < 6; ++q) {
    if (M) M[q * N + i] = out[q];
    if (Mf) Mf[q * N + i] = float(out[q]);
  }
}

int launch_prep(const double* sigma6, long ncell, double sigma0, int form, double* M, float* Mf,
                double* A, double* Ainv, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_prep, dim3(ceil_div(ncell, 256)), dim3(256), 0, s, sigma6, ncell, sigma0,
                     form, M, Mf, A, Ainv, bad);
  IE_LAUNCH_CHECK();
  return IE_OK;
}

__global__ void k_tensor_apply(const double* __restrict__ T6, long t_cs, const c128* __restrict__ x,
                               long x_cs, c128* __restrict__ y, long y_cs, long N) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double m[6];
  for (int c = 0; c < 6; ++c) m[c] = T6[c * t_cs + i];
  c128 v[3], o[3];
  for (int c = 0; c < 3; ++c) v[c] = x[c * x_cs + i];
  tensor_apply(m, v, o);
  for (int c = 0; c < 3; ++c) y[c * y_cs + i] = o[c];
}

int launch_tensor_apply(const double* T6, long t_cs, const c128* x, long x_cs, c128* y, long y_cs,
                        long ncell, hipStream_t s) {
  hipLaunchKernelGGL(k_tensor_apply, dim3(ceil_div(ncell, 256)), dim3(256), 0, s, T6, t_cs, x,
                     x_cs, y, y_cs, ncell);
  IE_LAUNCH_CHECK();
  return IE_OK;
}

}  // namespace ie
