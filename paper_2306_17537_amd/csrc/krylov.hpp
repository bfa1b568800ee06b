// Restarted GMRES on the device (section 2.2; restart length 10 in section 3.1).
//
// Krylov vectors are complex128 (IE_FP64) or complex64 (IE_MIXED); every inner product,
// norm, Hessenberg entry, Givens rotation and the solution accumulation are float64.  Each
// restart cycle begins from the float64 true residual r = b - A x, so in IE_MIXED every cycle
// is one step of iterative refinement whose correction comes from a complex64 Arnoldi cycle.
// Orthogonalisation: classical Gram-Schmidt with one reduction per Arnoldi step (the dots
// <v_i, w> and ||w||^2 in one pass over w, h_{j+1,j}^2 = ||w||^2 - sum |h_ij|^2, then the update
// pass), or CGS2 (repeated once, with fused update-and-reduce passes and the norm of the
// updated vector).  All scalar work runs in single-block kernels; per-problem
// `active` flags retire finished cycles inside the queued kernels, so the host synchronises
// once per restart cycle.
#pragma once

#include <vector>

#include "ctx.hpp"

namespace ie {

constexpr int MAXM = 16;  // largest restart length

struct alignas(16) GmState {
  c128 H[MAXM][MAXM + 1];  // H[j][i]: Hessenberg column j, row i (rotated in place)
  c128 cs[MAXM], sn[MAXM];
  c128 g[MAXM + 1];
  c128 hc[MAXM + 1];   // coefficients of the current Gram-Schmidt pass
  double nv[MAXM + 1]; // Krylov vector i is stored unnormalised: v_i = nv[i] V_i
  double beta, bnorm, target, est, inv_h;
  int k, active, its, max_its;
  int breakdown, counter;  // counter: blocks done in the current reduction (last block finalises)
};

struct GmSummary {  // per problem, copied to the host once per cycle
  double beta, bnorm;
  int active, its;
};

struct OpDesc {
  int form = IE_CONVENTIONAL;  // IE_CONVENTIONAL or IE_CIE
  double sigma0 = 0;
  const double* M64 = nullptr;  // contrast (dsigma or b), [6] comps with stride M_cs
  const float* M32 = nullptr;
  long M_cs = 0, M_bs = 0;
};

struct GmOpts {
  double tol = 1e-6;
  const double* tols = nullptr;  // optional HOST array of per-problem tolerances (overrides tol)
  int restart = 10;
  int max_its = 2000;
  int precision = IE_FP64;
  int reorth = -1;  // -1: CGS2 for complex64 Krylov vectors, CGS for complex128
};

struct GmResult {
  int its = 0, cycles = 0, converged = 0, graph_cycles = 0;
  double relres = 0;
  int mv64 = 0, mv32 = 0;
};

// A captured restart cycle, valid for the exact buffers and operator it was recorded with.
struct CycleGraph {
  std::vector<const void*> key;
  hipGraphExec_t exec = nullptr;
};

struct KrylovWork {
  DevBuf V, r, part, st, sum, flags, tols;
  GmSummary* host = nullptr;  // pinned
  int host_cap = 0;
  int* hflags = nullptr;      // pinned [MAXM][batch] active flags after each Arnoldi step
  int hflags_cap = 0;
  hipEvent_t ev[MAXM] = {};
  hipEvent_t join[2] = {};
  hipStream_t ps = nullptr;   // private stream (capturable; default priority)
  std::vector<CycleGraph> graphs;
  bool use_graphs = true;
  ~KrylovWork() {
    for (auto& g : graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (host) (void)hipHostFree(host);
    if (hflags) (void)hipHostFree(hflags);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : join)
      if (e) (void)hipEventDestroy(e);
    if (ps) (void)hipStreamDestroy(ps);
  }
};

// Solve A x = rhs for `batch` problems of plan p's shape; rhs and x are contiguous
// [3][nz][ny][nx] complex128 arrays with batch stride 3 N.  x holds the initial guess.
int gmres_solve(Plan& p, const OpDesc& op, const c128* rhs, c128* x, int batch,
                const GmOpts& o, GmResult* res, KrylovWork& w, const c128* tw64,
                const c64* tw32, hipStream_t s);

// Operator application of the iterated form: y = A x (a_e = 0) or y = e - A x (residual).
template <typename T>
int apply_op(Plan& p, const OpDesc& op, const cx<T>* x, cx<T>* y, const cx<T>* e, bool residual,
             int batch, const int* active, int active_bs, hipStream_t s, const cx<T>* tw);

// process-wide switch for captured restart cycles (ie_set_option)
extern bool g_use_graphs;

// Deterministic float64 2-norms of `batch` complex128 vectors (stride n) -> host array.
int norms_host(const c128* v, long n, int batch, double* out, KrylovWork& w, hipStream_t s);

}  // namespace ie
