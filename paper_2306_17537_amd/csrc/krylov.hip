// Device-side restarted GMRES: fused Gram-Schmidt passes, float64 reductions, Givens
// rotations and back substitution in single-block kernels (see krylov.hpp).
#include <cmath>
#include <cstring>
#include <vector>

#include "krylov.hpp"
#include "prof.hpp"

namespace ie {

bool g_use_graphs = true;

namespace {

constexpr int RB = 256;             // threads per reduction block
constexpr int NWV = RB / 64;        // wavefronts per block
constexpr int PWD = 2 * MAXM + 1;  // doubles per block partial (at most 2 MAXM dots + norm)

enum Fin { FIN_NONE = 0, FIN_H = 1, FIN_GIVENS = 2, FIN_CYCLE = 3, FIN_BNORM = 4, FIN_HG = 5 };

// Blocks of a reduction pass: about eight elements per thread, at most RED_MAX blocks (four per
// CU, so that the register-heavy passes of the long restarts still have waves to switch
// between).  Few blocks keep the per-block reduction tail small; the passes unroll their element
// loop so that a wave still has many loads in flight.  The finalisation sums at most RED_MAX
// partials per slot.  The plain update pass (no reduction) takes at most UPD_MAX blocks.
constexpr int RED_MAX = 1024, UPD_MAX = 512;
int red_grid(long n, int cap = RED_MAX) {
  long g = (n + RB * 8 - 1) / (RB * 8);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return int(g);
}

// Krylov basis loads with the non-temporal hint: the basis (restart + 1 vectors of 3 N values)
// is far larger than the last-level cache and is streamed once per pass, so keeping it out of
// the cache leaves room for w, which the dots pass and the update pass read one after the other
// (measured: the float64 GMRES(10) solve of the 128x128x256 model 3.5 % faster, the mixed
// GMRES(16) one 5 %).
template <typename T>
__device__ __forceinline__ cx<T> load_basis(const cx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 r = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return cx<T>{r.x, r.y};
}

template <typename T>
__device__ __forceinline__ c128 up(cx<T> v) { return c128{double(v.re), double(v.im)}; }

// Slots of a partial: dots (re, im) in [0, 2 CM), the squared norm in slot NS = 2 CM.
template <int CM>
struct Slots {
  static constexpr int NV = 2 * CM + 1;
  static constexpr int NS = 2 * CM;
};

// One row step of a 16-lane sum: v + v of the lane that the DPP pattern CTRL names (moved as two
// 32-bit halves).  0xB1 and 0x4E swap lanes within quads (lane ^ 1, lane ^ 2), 0x141 mirrors each
// half-row (lane i <- 7 - i), 0x140 each row (i <- 15 - i); after the four steps every lane of a
// 16-lane row holds the row's sum.  These are VALU moves, no LDS traffic.
template <int CTRL>
__device__ __forceinline__ double dpp_add(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(u), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(u >> 32), CTRL, 0xF, 0xF, false);
  return v + __longlong_as_double((static_cast<long long>(hi) << 32) |
                                  static_cast<unsigned int>(lo));
}

// Block-wide sums of the slots a pass produces: the dots (slots [0, NV - 1)) if DOTS and the
// squared norm (slot NV - 1) if NRM.  Each 16-lane row is summed in registers (four DPP steps,
// all slots interleaved), the first lane of every row stores its row sums, and thread k adds the
// 4 NWV row sums of slot k in a fixed order and writes out[k * os] for the slots the caller needs
// (k < nd, and NV - 1 if NRM).
template <int NV, bool DOTS, bool NRM>
__device__ __forceinline__ void block_sums(double (&v)[NV], int nd, double* sh, double* out,
                                           long os = 1) {
  constexpr int ND = DOTS ? NV - 1 : 0;
  constexpr int NR = 4 * NWV;  // 16-lane rows per block
  const int lane = threadIdx.x & 63, rowid = threadIdx.x >> 4;
#pragma unroll
  for (int k = 0; k < ND; ++k) v[k] = dpp_add<0xB1>(v[k]);
  if (NRM) v[NV - 1] = dpp_add<0xB1>(v[NV - 1]);
#pragma unroll
  for (int k = 0; k < ND; ++k) v[k] = dpp_add<0x4E>(v[k]);
  if (NRM) v[NV - 1] = dpp_add<0x4E>(v[NV - 1]);
#pragma unroll
  for (int k = 0; k < ND; ++k) v[k] = dpp_add<0x141>(v[k]);
  if (NRM) v[NV - 1] = dpp_add<0x141>(v[NV - 1]);
#pragma unroll
  for (int k = 0; k < ND; ++k) v[k] = dpp_add<0x140>(v[k]);
  if (NRM) v[NV - 1] = dpp_add<0x140>(v[NV - 1]);
  if ((lane & 15) == 0) {
#pragma unroll
    for (int k = 0; k < ND; ++k) sh[rowid * NV + k] = v[k];
    if (NRM) sh[rowid * NV + NV - 1] = v[NV - 1];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NV; k += RB) {
    if (k < nd || (NRM && k == NV - 1)) {
      double r = 0;
#pragma unroll
      for (int q = 0; q < NR; ++q) r += sh[q * NV + k];
      out[k * os] = r;
    }
  }
}

// Sum the G block partials of problem b (stored slot-major, part[(b PWD + slot) G + block], so
// that consecutive threads read consecutive blocks) into fin[]: the dot slots [0, NV - 1) if
// DOTS, the norm slot NV - 1 if NRM.  Every slot index below NV lies inside the partial buffer
// (NV <= PWD) and block indices past G are clamped to 0 and masked after loading, so all loads
// of one chunk are unconditional and in flight together.  Fixed summation order: deterministic.
// Called by a one-block kernel.
template <int NV, bool DOTS, bool NRM>
__device__ __forceinline__ void reduce_partials(const double* part, int b, int G, int nd,
                                                double* sh, double* fin) {
  constexpr int K0 = DOTS ? 0 : NV - 1, K1 = NRM ? NV : NV - 1;
  double a[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) a[k] = 0;
  const double* pb = part + long(b) * PWD * G;
  for (int q0 = 0; q0 < G; q0 += 2 * RB) {
    const int q1 = q0 + threadIdx.x, q2 = q1 + RB;
    const bool in1 = q1 < G, in2 = q2 < G;
    const int c1 = in1 ? q1 : 0, c2 = in2 ? q2 : 0;
    double v1[NV], v2[NV];
#pragma unroll
    for (int k = K0; k < K1; ++k) {
      v1[k] = pb[long(k) * G + c1];
      v2[k] = pb[long(k) * G + c2];
    }
#pragma unroll
    for (int k = K0; k < K1; ++k) a[k] += (in1 ? v1[k] : 0.0) + (in2 ? v2[k] : 0.0);
  }
  block_sums<NV, DOTS, NRM>(a, nd, sh, fin);
  __syncthreads();
}

// State a Givens step reads, loaded by each thread at the start of the finalisation so that these
// loads are in flight together with the partial sums: the column entry H[j][t] (t <= j), the
// earlier rotations cs/sn[t] (t < j) and, in thread 0, g[j] and the counters.
struct GivensPre {
  c128 h, c, s, gj;
  double target;
  int its, max_its;
};
__device__ __forceinline__ GivensPre givens_prefetch(const GmState& S, int j, bool column) {
  GivensPre p{};
  const int t = threadIdx.x;
  if (column && t <= j) p.h = S.H[j][t];
  if (t < j) {
    p.c = S.cs[t];
    p.s = S.sn[t];
  }
  if (t == 0) {
    p.gj = S.g[j];
    p.target = S.target;
    p.its = S.its;
    p.max_its = S.max_its;
  }
  return p;
}

// Givens step for Hessenberg column j (entries pre.h of threads t <= j) once h_{j+1,j}^2 = hn2
// is known.  Called by all threads of the block: the column and the previous rotations are
// staged in shared memory, thread 0 applies the rotations, and the column is written back in
// parallel.
__device__ __forceinline__ void givens_update(GmState& s, int j, double hn2, int* flags,
                                              int batch, int b, const GivensPre& pre) {
  __shared__ c128 Hs[MAXM + 1], cs[MAXM], sn[MAXM];
  const int t = threadIdx.x;
  if (t <= j) Hs[t] = pre.h;
  if (t < j) {
    cs[t] = pre.c;
    sn[t] = pre.s;
  }
  __syncthreads();
  if (t == 0) {
    const double hn = sqrt(hn2);
    c128* H = Hs;
    for (int i = 0; i < j; ++i) {
      const c128 u = cjmul(cs[i], H[i]) + cjmul(sn[i], H[i + 1]);
      H[i + 1] = c128{0, 0} - sn[i] * H[i] + cs[i] * H[i + 1];
      H[i] = u;
    }
    const double hjj = sqrt(H[j].re * H[j].re + H[j].im * H[j].im);
    const double den = sqrt(hjj * hjj + hn * hn);
    c128 c, sg;
    if (den == 0.0) {
      c = c128{1, 0};
      sg = c128{0, 0};
    } else {
      c = c128{H[j].re / den, H[j].im / den};
      sg = c128{hn / den, 0};
    }
    s.cs[j] = c;
    s.sn[j] = sg;
    H[j] = c128{den, 0};
    H[j + 1] = c128{0, 0};
    const c128 gj = pre.gj;
    const c128 g1 = c128{0, 0} - sg * gj;
    s.g[j + 1] = g1;
    s.g[j] = cjmul(c, gj);
    const double est = sqrt(g1.re * g1.re + g1.im * g1.im);
    const int its = pre.its + 1;
    s.est = est;
    s.k = j + 1;
    s.its = its;
    const bool brk = (hn == 0.0) || (den == 0.0);
    s.breakdown = brk ? 1 : 0;
    s.nv[j + 1] = brk ? 0.0 : 1.0 / hn;
    const int active = (est <= pre.target || its >= pre.max_its || brk) ? 0 : 1;
    s.active = active;
    flags[j * batch + b] = active;
  }
  __syncthreads();
  if (t <= j + 1) s.H[j][t] = Hs[t];
}

// Fused Gram-Schmidt pass over w (per problem b = blockIdx.z), with v_i = nv[i] V_i:
//   UPD : w <- w - sum_{i<count} hc[i] v_i
//   DOTS: <v_i, w> for i < count;  NRM: ||w||^2
// writing one partial per block and slot; k_fin, launched right after it, sums them and does:
//   FIN_H      : hc[i] = <v_i, w>, H[j][i] = (first ? 0 : H[j][i]) + hc[i]
//   FIN_GIVENS : h_{j+1,j} = ||w||, rotations, residual estimate, active flag, nv[j+1]
//   FIN_HG     : FIN_H with first = 1, then FIN_GIVENS with h_{j+1,j}^2 = ||w||^2 - sum |hc_i|^2
//   FIN_CYCLE  : beta = ||w||, g = beta e1, active unless converged (start of a restart cycle)
//   FIN_BNORM  : ||b||, target = tol ||b||, counters reset (start of a solve)
template <typename TA, typename TW, bool UPD, bool DOTS, bool NRM, int FIN, int CM>
__global__ void __launch_bounds__(RB)
    k_orth(const cx<TA>* __restrict__ V, long vstride, long vbs, cx<TW>* w, long wbs, long n,
           int count, int j, int first, GmState* __restrict__ st, double* __restrict__ part,
           int* __restrict__ flags, int batch, double tol, int max_its) {
  const int b = blockIdx.z;
  GmState& S = st[b];
  if (FIN != FIN_CYCLE && FIN != FIN_BNORM && S.active == 0) {
    if ((FIN == FIN_GIVENS || FIN == FIN_HG) && blockIdx.x == 0 && threadIdx.x == 0)
      flags[j * batch + b] = 0;
    return;
  }
  using SL = Slots<CM>;
  constexpr int NV = SL::NV;
  __shared__ double sh[4 * NWV * NV];
  __shared__ double fin[NV];
  const cx<TA>* Vb = V + b * vbs;
  cx<TW>* wb = w + b * wbs;
  c128 h[CM];
  double nvi[CM];
#pragma unroll
  for (int i = 0; i < CM; ++i) {
    nvi[i] = ((UPD || DOTS) && i < count) ? S.nv[i] : 0.0;
    h[i] = (UPD && i < count) ? nvi[i] * S.hc[i] : c128{0, 0};
  }
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0;
  // U elements per thread and loop pass, all their loads issued before any is used, so that
  // each wave keeps U (count + 1) loads in flight; indices past n are clamped to a valid
  // element, their results masked and their stores skipped.  A reduction pass takes U as large
  // as keeps the loaded values within about 96 registers (its accumulators need the rest); the
  // plain update pass takes 2 (complex128) or 4 (complex64), measured faster at the lower
  // occupancy that costs for the long restarts.
  constexpr int VG = int(sizeof(cx<TA>)) / 4;  // registers per loaded value
  constexpr int U0 = 96 / (VG * (CM + 1));
  constexpr int UR = U0 < 1 ? 1 : (U0 > 4 ? 4 : U0);
  constexpr int U = (UPD && !DOTS && !NRM) ? (VG == 2 ? 4 : 2) : UR;
  const long stride = long(gridDim.x) * RB;
  for (long e0 = long(blockIdx.x) * RB + threadIdx.x; e0 < n; e0 += U * stride) {
    long ec[U];
    bool in[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long e = e0 + u * stride;
      in[u] = e < n;
      ec[u] = in[u] ? e : e0;
    }
    cx<TA> vv[U][CM];
#pragma unroll
    for (int i = 0; i < CM; ++i)
      if ((UPD || DOTS) && i < count) {
#pragma unroll
        for (int u = 0; u < U; ++u) vv[u][i] = load_basis(&Vb[i * vstride + ec[u]]);
      }
    cx<TW> wv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) wv[u] = wb[ec[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (UPD) {
        c128 wd = up(wv[u]);
#pragma unroll
        for (int i = 0; i < CM; ++i)
          if (i < count) wd = wd - h[i] * up(vv[u][i]);
        wv[u] = cx<TW>{TW(wd.re), TW(wd.im)};
        if (in[u]) wb[ec[u]] = wv[u];
      }
      const c128 wd = in[u] ? up(wv[u]) : c128{0, 0};
      if (DOTS) {
#pragma unroll
        for (int i = 0; i < CM; ++i)
          if (i < count) {
            const c128 d = cjmul(up(vv[u][i]), wd);
            acc[2 * i] += d.re;
            acc[2 * i + 1] += d.im;
          }
      }
      if (NRM) acc[SL::NS] += wd.re * wd.re + wd.im * wd.im;
    }
  }
  const int nd = DOTS ? 2 * count : 0;
  // slot-major partials: slot k of this block at part[(b PWD + k) G + blockIdx.x] (the
  // finalisation kernel launched after this one uses the same register bucket CM)
  double* pb = part + long(b) * PWD * gridDim.x + blockIdx.x;
  if (DOTS || NRM) block_sums<NV, DOTS, NRM>(acc, nd, sh, pb, long(gridDim.x));
}

// Finalisation of a reduction (one block per problem):
//   FIN_H      : hc[i] = <v_i, w>, H[j][i] = (first ? 0 : H[j][i]) + hc[i]
//   FIN_GIVENS : h_{j+1,j} = ||w||, rotations, residual estimate, active flag, nv[j+1]
//   FIN_HG     : both from one pass over w (dots and ||w||^2): hc[i], H[j][i] = hc[i] and
//                h_{j+1,j}^2 = ||w||^2 - sum_i |hc_i|^2, the squared norm of w - sum hc_i v_i
//                for orthonormal v_i (clamped at 0, where the Givens step reports breakdown)
//   FIN_CYCLE  : beta = ||r||, g = beta e1, active unless converged (start of a restart cycle)
//   FIN_BNORM  : ||b||, target = tol ||b||, counters reset (start of a solve)
template <int FIN, int CM>
__global__ void __launch_bounds__(RB)
    k_fin(GmState* __restrict__ st, const double* __restrict__ part, int G, int count, int j,
          int first, int* __restrict__ flags, int batch, double tol, int max_its,
          const double* __restrict__ tols) {
  const int b = blockIdx.x;
  GmState& S = st[b];
  using SL = Slots<CM>;
  constexpr int NV = SL::NV;
  __shared__ double sh[4 * NWV * NV];
  __shared__ double fin[NV];
  constexpr bool STEP = FIN == FIN_H || FIN == FIN_GIVENS || FIN == FIN_HG;
  constexpr bool FD = FIN == FIN_H || FIN == FIN_HG, FN = FIN != FIN_H;
  constexpr bool GV = FIN == FIN_GIVENS || FIN == FIN_HG;
  const int t = threadIdx.x;
  // every state load is issued before the partial sums; a retired problem (active == 0, the
  // same for the whole block) leaves after them
  const int act = STEP ? S.active : 1;
  const double nvt = (FD && t < count) ? S.nv[t] : 0.0;
  const c128 hprev = (FIN == FIN_H && !first && t < count) ? S.H[j][t] : c128{0, 0};
  GivensPre pre{};
  if (GV) pre = givens_prefetch(S, j, FIN == FIN_GIVENS);
  const int nd = FD ? 2 * count : 0;
  reduce_partials<NV, FD, FN>(part, b, G, nd, sh, fin);
  if (STEP && act == 0) {
    if (GV && t == 0) flags[j * batch + b] = 0;
    return;
  }
  if (FIN == FIN_HG) {
    __shared__ double sq[CM];
    if (t < count) {  // one coefficient per thread
      const c128 hv = c128{nvt * fin[2 * t], nvt * fin[2 * t + 1]};
      S.hc[t] = hv;
      pre.h = hv;
      sq[t] = hv.re * hv.re + hv.im * hv.im;
    }
    __syncthreads();
    double hn2 = fin[SL::NS];
    for (int q = 0; q < count; ++q) hn2 -= sq[q];
    givens_update(S, j, hn2 > 0.0 ? hn2 : 0.0, flags, batch, b, pre);
    return;
  }
  if (FIN == FIN_H) {
    if (t < count) {  // one coefficient per thread
      const c128 hv = c128{nvt * fin[2 * t], nvt * fin[2 * t + 1]};
      S.hc[t] = hv;
      S.H[j][t] = first ? hv : hprev + hv;
    }
    return;
  }
  if (FIN == FIN_GIVENS) {
    givens_update(S, j, fin[SL::NS], flags, batch, b, pre);
    return;
  }
  if (threadIdx.x != 0) return;
  if (FIN == FIN_CYCLE) {
    const double beta = sqrt(fin[SL::NS]);
    S.beta = beta;
    S.est = beta;
    S.k = 0;
    for (int i = 0; i <= MAXM; ++i) S.g[i] = c128{0, 0};
    S.g[0] = c128{beta, 0};
    S.nv[0] = 1.0;
    S.inv_h = beta > 0 ? 1.0 / beta : 0.0;
    S.active = (beta > S.target && S.its < S.max_its) ? 1 : 0;
  } else if (FIN == FIN_BNORM) {
    S.bnorm = sqrt(fin[SL::NS]);
    S.target = (tols ? tols[b] : tol) * S.bnorm;
    S.its = 0;
    S.max_its = max_its;
    S.active = 0;
    S.k = 0;
  }
}

// Launch a Gram-Schmidt pass with the smallest register bucket that holds `count` vectors.
template <typename TA, typename TW, bool UPD, bool DOTS, bool NRM, int FIN>
int launch_orth(const char* pname, const char* ptag, double pbytes, dim3 grid, hipStream_t s,
                const cx<TA>* V, long vstride, long vbs, cx<TW>* w, long wbs, long n, int count,
                int j, int first, GmState* st, double* part, int* flags, int batch, double tol,
                int max_its, const double* tols = nullptr) {
#define IE_ORTH(CMV)                                                                             \
  do {                                                                                           \
    {                                                                                            \
      ProfScope ps(s, pname, ptag, pbytes);                                                      \
      hipLaunchKernelGGL((k_orth<TA, TW, UPD, DOTS, NRM, FIN, CMV>), grid, dim3(RB), 0, s, V,     \
                         vstride, vbs, w, wbs, n, count, j, first, st, part, flags, batch, tol,  \
                         max_its);                                                               \
    }                                                                                            \
    IE_LAUNCH_CHECK();                                                                           \
    if (FIN != FIN_NONE) {                                                                       \
      ProfScope ps(s, "finalise", ptag, 0);                                                      \
      hipLaunchKernelGGL((k_fin<FIN, CMV>), dim3(grid.z), dim3(RB), 0, s, st, part, int(grid.x),   \
                         count, j, first, flags, batch, tol, max_its, tols);                     \
    }                                                                                            \
  } while (0)
  if (count <= 1)
    IE_ORTH(1);
  else if (count <= 4)
    IE_ORTH(4);
  else if (count <= 8)
    IE_ORTH(8);
  else if (count <= 12)
    IE_ORTH(12);
  else
    IE_ORTH(MAXM);
#undef IE_ORTH
  IE_LAUNCH_CHECK();
  return IE_OK;
}

__global__ void k_summary(const GmState* st, GmSummary* out, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  out[b].beta = st[b].beta;
  out[b].bnorm = st[b].bnorm;
  out[b].active = st[b].active;
  out[b].its = st[b].its;
}

// V0 = r / beta (cast to the Krylov precision)
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

// x += sum_{i<k} y_i v_i with y = R^-1 g from the rotated Hessenberg (float64); every block
// solves the k x k triangular system itself (k <= 16), so no separate launch is needed.
template <typename TA>
__global__ void __launch_bounds__(RB)
    k_xupdate(c128* x, long xbs, const cx<TA>* __restrict__ V, long vstride, long vbs, long n,
              const GmState* st) {
  const int b = blockIdx.z;
  const GmState& S = st[b];
  const int k = S.k;
  if (k == 0) return;
  __shared__ c128 ys[MAXM];
  if (threadIdx.x == 0) {
    for (int i = k - 1; i >= 0; --i) {
      c128 acc = S.g[i];
      for (int l = i + 1; l < k; ++l) acc = acc - S.H[l][i] * ys[l];
      const c128 d = S.H[i][i];
      const double dd = d.re * d.re + d.im * d.im;
      ys[i] = dd > 0 ? c128{(acc.re * d.re + acc.im * d.im) / dd, (acc.im * d.re - acc.re * d.im) / dd}
                     : c128{0, 0};
    }
    for (int i = 0; i < k; ++i) ys[i] = S.nv[i] * ys[i];
  }
  __syncthreads();
  c128 y[MAXM];
#pragma unroll
  for (int i = 0; i < MAXM; ++i) y[i] = i < k ? ys[i] : c128{0, 0};
  c128* xb = x + b * xbs;
  const cx<TA>* Vb = V + b * vbs;
  // U elements per thread and pass with all loads issued first (as in k_orth)
  constexpr int U = 2;
  const long stride = long(gridDim.x) * RB;
  for (long e0 = long(blockIdx.x) * RB + threadIdx.x; e0 < n; e0 += U * stride) {
    long ec[U];
    bool in[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long e = e0 + u * stride;
      in[u] = e < n;
      ec[u] = in[u] ? e : e0;
    }
    cx<TA> vv[U][MAXM];
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < k) {
#pragma unroll
        for (int u = 0; u < U; ++u) vv[u][i] = load_basis(&Vb[i * vstride + ec[u]]);
      }
    c128 acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = xb[ec[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int i = 0; i < MAXM; ++i)
        if (i < k) acc[u] = acc[u] + y[i] * up(vv[u][i]);
      if (in[u]) xb[ec[u]] = acc[u];
    }
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

static int ensure_state(KrylovWork& w, int batch, int G, hipStream_t s) {
  IE_TRY(w.part.ensure(sizeof(double) * PWD * G * batch));
  const bool grow = w.st.bytes < sizeof(GmState) * batch;
  IE_TRY(w.st.ensure(sizeof(GmState) * batch));
  if (grow) IE_HIP(hipMemsetAsync(w.st.p, 0, sizeof(GmState) * batch, s));  // reduction counters
  IE_TRY(ensure_host(w, batch));
  IE_TRY(w.flags.ensure(sizeof(int) * MAXM * batch));
  return IE_OK;
}

int norms_host(const c128* v, long n, int batch, double* out, KrylovWork& w, hipStream_t s) {
  const int G = red_grid(n);
  IE_TRY(ensure_state(w, batch, G, s));
  GmState* st = w.st.as<GmState>();
  IE_TRY((launch_orth<double, double, false, false, true, FIN_BNORM>("norm", "", 16.0 * n * batch,
                                                                     dim3(G, 1, batch), s, nullptr, 0L, 0L, const_cast<c128*>(v), n, n,
                     0, 0, 0, st, w.part.as<double>(), w.flags.as<int>(), batch, 0.0, 0)));
  IE_TRY(fetch_summary(w, st, batch, s));
  for (int b = 0; b < batch; ++b) out[b] = w.host[b].bnorm;
  return IE_OK;
}

template <typename TA>
static int gmres_impl(Plan& p, const OpDesc& op, const c128* rhs, c128* x, int batch,
                      const GmOpts& o, GmResult* res, KrylovWork& w, const c128* tw64,
                      const cx<TA>* twa, hipStream_t us) {
  const long N = p.ncell();
  const long n = 3 * N;
  const int m = o.restart;
  if (m < 1 || m > MAXM) return fail(IE_EINVAL, "restart must be in [1, %d], got %d", MAXM, m);
  const bool reorth = o.reorth < 0 ? (sizeof(TA) == 4) : (o.reorth != 0);
  const int G = red_grid(n);
  const long vbs = long(m + 1) * n;
  // all work runs on the private stream, ordered after and before the caller's stream
  if (!w.ps) IE_HIP(hipStreamCreateWithFlags(&w.ps, hipStreamNonBlocking));
  for (auto& e : w.join)
    if (!e) IE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  for (auto& e : w.ev)
    if (!e) IE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  const hipStream_t s = w.ps;
  IE_HIP(hipEventRecord(w.join[0], us));
  IE_HIP(hipStreamWaitEvent(s, w.join[0], 0));
  IE_TRY(w.V.ensure(sizeof(cx<TA>) * vbs * batch));
  IE_TRY(w.r.ensure(sizeof(c128) * n * batch));
  IE_TRY(ensure_state(w, batch, G, s));
  IE_TRY(p.work(IE_FP64, batch));
  IE_TRY(p.work(sizeof(TA) == 8 ? IE_FP64 : IE_MIXED, batch));
  if (w.hflags_cap < batch) {
    if (w.hflags) (void)hipHostFree(w.hflags);
    w.hflags = nullptr;
    IE_HIP(hipHostMalloc((void**)&w.hflags, sizeof(int) * MAXM * batch, hipHostMallocDefault));
    w.hflags_cap = batch;
  }
  GmState* st = w.st.as<GmState>();
  cx<TA>* V = w.V.as<cx<TA>>();
  c128* r = w.r.as<c128>();
  double* part = w.part.as<double>();
  int* flags = w.flags.as<int>();
  const int* act = &st[0].active;
  const int act_bs = int(sizeof(GmState) / sizeof(int));
  const long nv_bs = long(sizeof(GmState) / sizeof(double));
  const dim3 vgrid(G, 1, batch);
  const dim3 ugrid(red_grid(n, UPD_MAX), 1, batch);  // plain update passes
  for (int b = 0; b < batch; ++b) res[b] = GmResult{};
  char tgb[96];
  snprintf(tgb, sizeof(tgb), "%s n%ld b%d", sizeof(TA) == 4 ? "c64" : "c128", n, batch);
  const char* tg = tgb;
  const double sa = sizeof(cx<TA>), nb = double(n) * batch;
  std::vector<std::pair<int, long>> pending;  // (step, profiler group) awaiting byte scaling
  int prev_start_active = 0;

  // r = b - A x (float64), beta = ||r||, per-problem summary copied to the host
  auto enqueue_residual = [&]() -> int {
    IE_TRY(apply_op<double>(p, op, x, r, rhs, true, batch, nullptr, 0, s, tw64));
    IE_TRY((launch_orth<TA, double, false, false, true, FIN_CYCLE>("norm", tg, nb * 16, vgrid, s,
                                                                   nullptr, 0L, 0L, r, n, n, 0, 0,
                                                                   0, st, part, flags, batch, 0.0, 0)));
    hipLaunchKernelGGL(k_summary, dim3(ceil_div(batch, 64)), dim3(64), 0, s, st,
                       w.sum.as<GmSummary>(), batch);
    IE_LAUNCH_CHECK();
    IE_HIP(hipMemcpyAsync(w.host, w.sum.p, sizeof(GmSummary) * batch, hipMemcpyDeviceToHost, s));
    return IE_OK;
  };
  // one restart cycle of Arnoldi steps and the solution update; `lagged` enqueues step j only if
  // some problem was active after step j-2 (host reads the flags with one step of look-ahead)
  auto enqueue_steps = [&](bool lagged) -> int {
    {
      ProfScope ps(s, "scale_cast", tg, nb * (16 + sa));
      hipLaunchKernelGGL((k_scale_cast<TA>), vgrid, dim3(RB), 0, s, r, n, V, vbs, n, st);
      IE_LAUNCH_CHECK();
    }
    for (int j = 0; j < m; ++j) {
      if (lagged && j >= 2) {
        IE_HIP(hipEventSynchronize(w.ev[j - 2]));
        int cnt = 0;
        for (int b = 0; b < batch; ++b) cnt += w.hflags[(j - 2) * batch + b];
        if (cnt == 0) break;
      }
      if (lagged) {
        const long grp = prof_new_group();
        pending.emplace_back(j, grp);
        prof_set_group(grp);
      }
      cx<TA>* vj = V + j * n;
      cx<TA>* w1 = V + (j + 1) * n;
      // w = A v_j  (v_j = nv[j] V_j, the factor applied on load)
      MvArgs<TA> a{};
      a.x = vj;
      a.x_cs = N;
      a.x_bs = vbs;
      a.xscale = &st[0].nv[j];
      a.xscale_bs = nv_bs;
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
      a.a_e = 0;
      a.a_x = 1;
      a.a_m = (op.form == IE_CIE) ? TA(1) : TA(0);
      a.a_s = (op.form == IE_CIE) ? TA(-2.0 * op.sigma0) : TA(-1);
      a.active = act;
      a.active_bs = act_bs;
      IE_TRY(launch_matvec<TA>(p, a, batch, s, twa));
      if (!reorth) {
        // classical Gram-Schmidt: h = V^H w and ||w||^2 in one pass, the H column, h_{j+1,j}
        // (Pythagoras) and the Givens update; then w -= V h, a pass with no reduction
        IE_TRY((launch_orth<TA, TA, false, true, true, FIN_HG>(
            "orth_dots_norm", tg, nb * sa * (j + 2), vgrid, s, V, n, vbs, w1, vbs, n, j + 1, j, 1,
            st, part, flags, batch, 0.0, 0)));
        IE_TRY((launch_orth<TA, TA, true, false, false, FIN_NONE>(
            "orth_upd", tg, nb * sa * (j + 3), ugrid, s, V, n, vbs, w1, vbs, n, j + 1, j, 0, st,
            part, flags, batch, 0.0, 0)));
      } else {
        // CGS2: h = V^H w (+ H column); w -= V h with the second pass's dots added to the
        // column; w -= V h' with ||w|| and the Givens update
        IE_TRY((launch_orth<TA, TA, false, true, false, FIN_H>(
            "orth_dots", tg, nb * sa * (j + 2), vgrid, s, V, n, vbs, w1, vbs, n, j + 1, j, 1, st,
            part, flags, batch, 0.0, 0)));
        IE_TRY((launch_orth<TA, TA, true, true, false, FIN_H>(
            "orth_upd_dots", tg, nb * sa * (j + 3), vgrid, s, V, n, vbs, w1, vbs, n, j + 1, j, 0, st,
            part, flags, batch, 0.0, 0)));
        IE_TRY((launch_orth<TA, TA, true, false, true, FIN_GIVENS>(
            "orth_upd_norm", tg, nb * sa * (j + 3), vgrid, s, V, n, vbs, w1, vbs, n, j + 1, j, 0, st,
            part, flags, batch, 0.0, 0)));
      }
      if (lagged) {
        prof_set_group(-1);
        IE_HIP(hipMemcpyAsync(w.hflags + j * batch, flags + j * batch, sizeof(int) * batch,
                              hipMemcpyDeviceToHost, s));
        IE_HIP(hipEventRecord(w.ev[j], s));
      }
    }
    ProfScope ps(s, "xupdate", tg, nb * (32 + sa * m));
    hipLaunchKernelGGL((k_xupdate<TA>), vgrid, dim3(RB), 0, s, x, n, V, n, vbs, n, st);
    IE_LAUNCH_CHECK();
    return IE_OK;
  };
  // captured cycle for exactly these buffers / operator (replayed with one launch per cycle)
  auto cycle_graph = [&]() -> hipGraphExec_t {
    std::vector<const void*> key = {
        (const void*)&p, p.t1_64.p, p.t2_64.p, p.t1_32.p, p.t2_32.p, p.ghat64.p, p.ghat32.p,
        op.M64, op.M32, (const void*)op.M_cs, (const void*)op.M_bs, (const void*)long(op.form),
        rhs, x, (const void*)long(batch), (const void*)long(m), (const void*)long(reorth),
        (const void*)sizeof(TA), w.V.p, w.r.p, w.part.p, w.st.p, w.sum.p, w.host, w.flags.p,
        tw64, twa};
    double sg = op.sigma0;
    const void* sgp;
    std::memcpy(&sgp, &sg, sizeof(sgp));
    key.push_back(sgp);
    for (auto& g : w.graphs)
      if (g.key == key) return g.exec;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    int rc = enqueue_steps(false);
    if (rc >= 0) rc = enqueue_residual();
    const hipError_t ec = hipStreamEndCapture(s, &graph);
    if (rc < 0 || ec != hipSuccess || graph == nullptr) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      return nullptr;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    if (w.graphs.size() >= 8) {
      (void)hipGraphExecDestroy(w.graphs.front().exec);
      w.graphs.erase(w.graphs.begin());
    }
    w.graphs.push_back(CycleGraph{key, exec});
    return exec;
  };

  // ||b||, target (per-problem tolerances if given), counters; first residual
  const double* dtols = nullptr;
  if (o.tols != nullptr) {
    IE_TRY(w.tols.ensure(sizeof(double) * batch));
    IE_HIP(hipMemcpyAsync(w.tols.p, o.tols, sizeof(double) * batch, hipMemcpyHostToDevice, s));
    dtols = w.tols.as<double>();
  }
  IE_TRY((launch_orth<TA, double, false, false, true, FIN_BNORM>("norm", tg, nb * 16, vgrid, s,
                                                                 nullptr, 0L, 0L,
                                                                 const_cast<c128*>(rhs), n, n, 0, 0,
                                                                 0, st, part, flags, batch, o.tol,
                                                                 o.max_its, dtols)));
  IE_TRY(enqueue_residual());
  const bool graphs = g_use_graphs && w.use_graphs && !prof_enabled();
  for (int cycle = 0;; ++cycle) {
    IE_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < batch; ++b) res[b].mv64 += 1;
    // byte scaling of the previous cycle's launch groups (all its flags have arrived now)
    for (auto& pg : pending) {
      const int j = pg.first;
      int cnt = 0;
      if (j == 0)
        cnt = prev_start_active;
      else
        for (int b = 0; b < batch; ++b) cnt += w.hflags[(j - 1) * batch + b];
      prof_scale_group(pg.second, double(cnt) / batch);
    }
    pending.clear();
    int any = 0, start_active = 0;
    for (int b = 0; b < batch; ++b) {
      const GmSummary& h = w.host[b];
      res[b].its = h.its;
      res[b].relres = h.bnorm > 0 ? h.beta / h.bnorm : 0.0;
      res[b].converged = h.beta <= (o.tols ? o.tols[b] : o.tol) * h.bnorm;
      if (h.active) {
        any = 1;
        start_active += 1;
        res[b].cycles += 1;
      }
    }
    if (!any) break;
    prev_start_active = start_active;
    hipGraphExec_t ex = graphs ? cycle_graph() : nullptr;
    if (ex != nullptr) {
      IE_HIP(hipGraphLaunch(ex, s));
      for (int b = 0; b < batch; ++b) res[b].graph_cycles += 1;
    } else {
      IE_TRY(enqueue_steps(true));
      IE_TRY(enqueue_residual());
    }
  }
  for (int b = 0; b < batch; ++b) {
    const int arn = res[b].its;
    if (sizeof(TA) == 8)
      res[b].mv64 += arn;
    else
      res[b].mv32 += arn;
  }
  IE_HIP(hipEventRecord(w.join[1], s));
  IE_HIP(hipStreamWaitEvent(us, w.join[1], 0));
  return IE_OK;
}

int gmres_solve(Plan& p, const OpDesc& op, const c128* rhs, c128* x, int batch, const GmOpts& o,
                GmResult* res, KrylovWork& w, const c128* tw64, const c64* tw32, hipStream_t s) {
  if (o.precision == IE_MIXED) return gmres_impl<float>(p, op, rhs, x, batch, o, res, w, tw64, tw32, s);
  return gmres_impl<double>(p, op, rhs, x, batch, o, res, w, tw64, tw64, s);
}

}  // namespace ie
