// ie_matvec_noalloc: one application of the discretised operator (eqs. 8, 10) whose every
// scratch buffer (the prepared contrast tensor, the padded FFT work arrays and the validation
// flag) lives in a fixed device array of the library, so that the call allocates nothing.
// The context (spectrum, twiddles, launch variants) is built beforehand by ie_green_setup.
#include <mutex>

#include "context.hpp"

namespace ie {
namespace {

// the array itself: each device holds its own copy until the process ends
static __device__ __align__(256) unsigned char scratch[IE_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device
std::mutex g_mu;

constexpr size_t kAlign = 256;
inline size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// clears n ints (stream-ordered, no memset node)
__global__ void k_clear_ints(int* p, int n) {
  const int i = threadIdx.x;
  if (i < n) p[i] = 0;
}

// bytes of scratch one call needs: flag, contrast tensor in the compute precision, T1, T2
size_t need_bytes(const Plan& p, int precision, bool contrast) {
  const size_t s = precision == IE_FP64 ? sizeof(c128) : sizeof(c64);
  const size_t r = precision == IE_FP64 ? sizeof(double) : sizeof(float);
  size_t b = kAlign;
  if (contrast) b += align_up(r * 6 * size_t(p.ncell()));
  b += align_up(s * size_t(p.t1_elems()));
  b += align_up(s * size_t(p.t2_elems()));
  return b;
}

}  // namespace

int noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(IE_EDEVICE, "device %d outside the %d devices the library supports", device,
                kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device] != nullptr) return IE_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr)
    return fail(IE_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                hipGetErrorString(e));
  g_scratch[device] = ptr;
  return IE_OK;
}

}  // namespace ie

using namespace ie;

extern "C" int ie_matvec_noalloc(ie_ctx* ctx, const double* sigma6, const void* x, void* y,
                                 int32_t form, int32_t precision, void* stream) {
  if (ctx == nullptr || x == nullptr || y == nullptr) return fail(IE_EINVAL, "NULL argument");
  if (x == y) return fail(IE_EINVAL, "x and y must not overlap");
  if (form < IE_CONVENTIONAL || form > IE_SCATTER) return fail(IE_EINVAL, "unknown form %d", form);
  if (precision != IE_FP64 && precision != IE_MIXED)
    return fail(IE_EINVAL, "precision must be IE_FP64 or IE_MIXED");
  if (!(ctx->prec_mask & precision))
    return fail(IE_EINVAL, "context was set up without this precision");
  const bool contrast = form != IE_GREEN_ONLY;
  if (contrast && sigma6 == nullptr) return fail(IE_EINVAL, "sigma6 is NULL");
  int dev = -1;
  IE_HIP(hipGetDevice(&dev));
  if (dev != ctx->device)
    return fail(IE_EINVAL, "the context belongs to device %d but device %d is current",
                ctx->device, dev);
  Plan& p = *ctx->full;
  const size_t need = need_bytes(p, precision, contrast);
  if (need > size_t(IE_NOALLOC_MAX_BYTES))
    return fail(IE_EINVAL,
                "grid %dx%dx%d needs %zu bytes of scratch in this precision; the fixed array "
                "holds %zu (use ie_matvec)",
                p.nx, p.ny, p.nz, need, size_t(IE_NOALLOC_MAX_BYTES));
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    base = static_cast<unsigned char*>(g_scratch[dev]);
  }
  if (base == nullptr) {
    IE_TRY(noalloc_init(dev));  // first call on this device without a set-up on it
    base = static_cast<unsigned char*>(g_scratch[dev]);
  }
  hipStream_t s = (hipStream_t)stream;
  const long N = p.ncell();
  const size_t sz = precision == IE_FP64 ? sizeof(c128) : sizeof(c64);
  const size_t rz = precision == IE_FP64 ? sizeof(double) : sizeof(float);
  int* bad = reinterpret_cast<int*>(base);
  size_t off = kAlign;
  void* M = nullptr;
  if (contrast) {
    M = base + off;
    off += align_up(rz * 6 * size_t(N));
  }
  void* T1 = base + off;
  off += align_up(sz * size_t(p.t1_elems()));
  void* T2 = base + off;

  if (contrast) {
    hipLaunchKernelGGL(k_clear_ints, dim3(1), dim3(64), 0, s, bad, 1);
    IE_LAUNCH_CHECK();
    const int pf = form == IE_CIE ? IE_CIE : IE_CONVENTIONAL;
    IE_TRY(launch_prep(sigma6, N, ctx->med.sigma0, pf,
                       precision == IE_FP64 ? static_cast<double*>(M) : nullptr,
                       precision == IE_FP64 ? nullptr : static_cast<float*>(M), nullptr,
                       nullptr, bad, s));
    int hbad = 0;
    IE_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    IE_HIP(hipStreamSynchronize(s));
    if (hbad) return fail(IE_EINVAL, "sigma6 holds a non-finite or non-positive-definite tensor");
  }
  double ax = 0, am = 0, as = 1;
  if (form == IE_CONVENTIONAL) {
    ax = 1;
    as = -1;
  } else if (form == IE_CIE) {
    ax = 1;
    am = 1;
    as = -2.0 * ctx->med.sigma0;
  }
  auto fill = [&](auto& a) {
    a.x_cs = N;
    a.x_bs = 3 * N;
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
    fill(a);
    a.M = static_cast<const double*>(M);
    a.x = (const c128*)x;
    a.y = (c128*)y;
    a.T1 = static_cast<c128*>(T1);
    a.T2 = static_cast<c128*>(T2);
    a.a_x = ax;
    a.a_m = am;
    a.a_s = as;
    return launch_matvec<double>(p, a, 1, s, tw64(ctx));
  }
  MvArgs<float> a{};
  fill(a);
  a.M = static_cast<const float*>(M);
  a.x = (const c64*)x;
  a.y = (c64*)y;
  a.T1 = static_cast<c64*>(T1);
  a.T2 = static_cast<c64*>(T2);
  a.a_x = float(ax);
  a.a_m = float(am);
  a.a_s = float(as);
  return launch_matvec<float>(p, a, 1, s, tw32(ctx));
}
