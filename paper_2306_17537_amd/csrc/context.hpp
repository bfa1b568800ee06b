// The opaque context behind ie_ctx* and helpers shared by the entry points.
#pragma once

#include <map>
#include <memory>
#include <vector>

#include "krylov.hpp"

namespace ie {
// Scratch of the domain-decomposition driver, sized for the largest problem group seen.
struct DdBufs {
  DevBuf D64, M64, M32, A64, Ai64, E0, E, Eold, rhs, x, active, flags, bad;
  DevBuf best;  // iterate of smallest full residual per problem (stationary sweeps)
  DevBuf xl;  // learned first-sweep guesses
  DevBuf fv, fz, fw, fpart;  // Krylov outer iteration: basis, preconditioned vectors, work
};
}  // namespace ie

struct ie_ctx {
  ie_grid grid{};
  ie::Medium med{};
  int prec_mask = 0;
  int device = 0;
  std::unique_ptr<ie::Plan> full;
  std::vector<int> zb;                                // partition (empty: none)
  std::map<int, std::unique_ptr<ie::Plan>> blocks;    // block plans by slab thickness
  ie::DevBuf tw64, tw32;                              // FFT twiddle tables
  // per-call scratch on the full grid
  ie::DevBuf M64, M32, A64, Ai64, bad;
  ie::DevBuf xt, bt, E0, tmp;
  ie::KrylovWork kw;
  // domain decomposition scratch
  ie::DevBuf blk_rhs2, blk_save;
  ie::DdBufs dd;
  ie::KrylovWork kw_blk;
  ie::Plan* block_plan(int nzb) {
    auto it = blocks.find(nzb);
    return it == blocks.end() ? nullptr : it->second.get();
  }
};

namespace ie {

// process-wide switch (ie_set_option IE_OPT_GROUP_THREADS): ie_dd_solve runs the groups of
// different contexts concurrently
extern bool g_group_threads;

inline const c128* tw64(const ie_ctx* c) { return c->tw64.as<const c128>(); }
inline const c64* tw32(const ie_ctx* c) { return c->tw32.as<const c64>(); }

// contrast tensors of `form` on the full grid into ctx->M64/M32 (+ A64/Ai64 for IE_CIE);
// validates sigma (IE_EINVAL on non-finite or non-positive-definite cells); synchronises.
int prepare_contrast(ie_ctx* c, const double* sigma6, int form, hipStream_t s);

// validate sources against the grid (none on a cell centre, finite values, known kind)
int check_sources(const ie_ctx* c, const ie_source* src, int nsrc);

// y = alpha x for complex128 arrays of n elements
int launch_scale(const c128* x, c128* y, double alpha, long n, hipStream_t s);
// y = x - z
int launch_sub(const c128* x, const c128* z, c128* y, long n, hipStream_t s);

}  // namespace ie
