// Learned first guesses for the inner block solves (network in nn.hip).
#pragma once
#include "context.hpp"

struct ie_nn;

namespace ie {

// IE_OK if the network maps the 14 solver features to 6 field channels and a grid of
// nz x ny x nx cells passes through its pooling levels.
int nn_check_shape(const ie_nn* n, int nz, int ny, int nx);

// Learned guesses xg (complex128 [batch][3][nb]) for `batch` blocks of the grid of plan B:
// xg = rhs + rms(rhs) e^{i phi} network(features).  D and rhs as below.
int nn_predict_blocks(ie_nn* n, ie_ctx* c, Plan& B, const double* D, long d_cs, long d_bs,
                      const c128* rhs, c128* xg, int batch, hipStream_t s);

// Learned guesses for `batch` blocks of the grid of plan B.  D: float64 dsigma of each block
// ([6][nb] with component stride d_cs, block stride d_bs); rhs: complex128 [batch][3][nb]; x holds
// the default guesses and receives, per block, whichever of {learned, default, zero} has the
// smallest float64 residual ||rhs - (I - G dsigma) x||.  accepted[b] = 1 (learned), 0 (default)
// or 2 (zero).  Synchronises with s.
int nn_guess_blocks(ie_nn* n, ie_ctx* c, Plan& B, const double* D, long d_cs, long d_bs,
                    const c128* rhs, c128* x, int batch, int* accepted, hipStream_t s);

}  // namespace ie
