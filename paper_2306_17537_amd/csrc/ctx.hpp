// Host-side objects of the library: per-shape FFT plans, the solver context and the internal
// driver entry points shared by the translation units.
#pragma once

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "common.hpp"
#include "passes.hpp"

namespace ie {

// Device buffer owned by the library.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // grow to at least n bytes (contents are not preserved)
  int ensure(size_t n) {
    if (n <= bytes) return IE_OK;
    release();
    if (hipMalloc(&p, n) != hipSuccess) {
      p = nullptr;
      return fail(IE_ENOMEM, "hipMalloc of %zu bytes failed", n);
    }
    bytes = n;
    return IE_OK;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// FFT geometry, the stored part of the spectra and padded work buffers of one grid shape.
struct Plan {
  int nx = 0, ny = 0, nz = 0;
  int LX = 0, LY = 0, LZ = 0;
  DevBuf ghat64, ghat32;  // [6][LZ/2+1][LY/2+1][LX/2+1]
  DevBuf t1_64, t2_64, t1_32, t2_32;  // padded work U1, U2, capacity `cap` problems
  int cap64 = 0, cap32 = 0;
  // launch variant per [precision: 0 float64, 1 complex64][pass: zfwd, yfwd, xconv, yinv, zinv],
  // set by the autotuner (0 when tuning is off)
  int8_t var[2][5] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};
  float tune_us[2][5][8] = {};  // measured average duration per variant (0: not measured)
  // operator microseconds (precisions of the context summed) of the two candidate length sets,
  // shortest and powers of two, when the lengths were chosen by timing (0 otherwise)
  float len_us[2] = {0, 0};
  long ncell() const { return long(nx) * ny * nz; }
  long t1_elems() const { return 3L * LZ * ny * nx; }
  long t2_elems() const { return 3L * LZ * LY * nx; }
  long spec_elems() const { return 6L * (LZ / 2 + 1) * (LY / 2 + 1) * (LX / 2 + 1); }
  int work(int prec, int batch);  // make sure work buffers hold `batch` problems
};

// FFT length for n cells: the smallest power of two >= 2n - 1 (pow2), else the shorter of that
// and the smallest 3 * 2^k >= 2n - 1 (k >= 3, at most 768)
int fft_len(int n, bool pow2);

// Resolves, once per device, the address of the fixed scratch array of ie_matvec_noalloc
// (called by ie_green_setup with the context's device current).
int noalloc_init(int device);

struct Medium {
  double sigma0, freq, mu0, omega;
  double k0re, k0im;  // k0 = sqrt(i omega mu0 sigma0), Im k0 > 0
};

struct ie_ctx_impl;

// Operator launch: y = a_e e + a_x x - a_m M x + a_s G (M x) on plan p.
// Fields in MvArgs that are geometry (sizes, ghat, tw) are filled in by the launcher; the padded
// work buffers are the plan's own unless the caller sets both a.T1 and a.T2 (one problem, at
// least t1_elems()/t2_elems() values each), in which case nothing is allocated.
// only >= 0 launches that pass alone (0 zfwd, 1 yfwd, 2 xconv, 3 yinv, 4 zinv); vover >= 0
// replaces the plan's variant (both for the autotuner).
template <typename T>
int launch_matvec(Plan& p, MvArgs<T> a, int batch, hipStream_t s, const cx<T>* tw, int only = -1,
                  int vover = -1);

// Times every launch variant of every pass on the plan's own buffers and keeps the fastest.
int autotune(Plan& p, int prec_mask, const c128* tw64, const c64* tw32, hipStream_t s);
// Time of one operator application at the plan's current variants (precisions in the mask
// summed).
int operator_us(Plan& p, int prec_mask, const c128* tw64, const c64* tw32, hipStream_t s,
                float& us);
// Template name of the kernel that runs pass q of plan p at precision pi (0 float64, 1 complex64).
std::string pass_kernel(const Plan& p, int pi, int q);
// The autotuner's cache as a JSON file (host only).
int tuning_save(const char* path);
int tuning_load(const char* path);

// Green setup of one plan (both precisions as requested).
int build_green(Plan& p, double h, const Medium& m, int prec_mask, const c128* tw64,
                const c64* tw32, hipStream_t s);

// Background field at the cell centres: E0 [3][nz][ny][nx] complex128.
int launch_background(int nx, int ny, int nz, double h, const double origin[3], const Medium& m,
                      const ie_source* src, int nsrc, c128* E0, hipStream_t s);

// Contrast preparation from sigma6: M (dsigma or b), optional a and a^-1 (CIE), float copy.
// Sets *bad (device int) to nonzero if any tensor is non-finite or not positive definite.
int launch_prep(const double* sigma6, long ncell, double sigma0, int form, double* M, float* Mf,
                double* A, double* Ainv, int* bad, hipStream_t s);

// y = T x per cell (6-component symmetric tensor), complex128 views with component strides.
int launch_tensor_apply(const double* T6, long t_cs, const c128* x, long x_cs, c128* y, long y_cs,
                        long ncell, hipStream_t s);

}  // namespace ie
