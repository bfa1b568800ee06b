/*
 * ie.h - C ABI of the MI355X (gfx950) integral-equation solver for 3-D induction-log
 * modelling with domain-decomposition preconditioning (Saputera et al., GJI).
 *
 * The library solves the discretised electric-field integral equation of eq. (8),
 *     (I - G dsigma) E = E0,
 * on a regular voxel grid, with G the whole-space electric Green's tensor of eqs. (5)-(7)
 * discretised as in section 2.2 and applied by zero-padded FFT convolution (eq. 10),
 * either directly (restarted GMRES, section 2.2) or by block Gauss-Seidel / Jacobi over
 * z-slab sub-domains (section 2.3, eqs. 19-24, Alg. 1).
 *
 * Conventions for every entry point:
 *  - Return value: IE_OK (0) on success; IE_ENOCONV (1) when an iteration hit its limit
 *    (outputs then hold the best iterate and statistics are filled); a negative code on
 *    error.  Nothing aborts, exits or throws across this boundary.  ie_last_error()
 *    returns a thread-local description of the last non-zero status.
 *  - Complex arrays are interleaved (re, im).  Fields use the layout [3][nz][ny][nx]
 *    (component-major, x fastest); component order x, y, z.
 *  - Conductivity tensors use the layout [6][nz][ny][nx] of real float64 in the order
 *    xx, yy, zz, xy, xz, yz (S/m); the tensor is symmetric (App. C) and must be positive
 *    definite in every cell.
 *  - Array pointers are DEVICE pointers unless stated otherwise; they are owned by the
 *    caller and must stay valid until the work queued on `stream` has finished.  The
 *    library never frees caller memory.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Entry points queue their work
 *    on it and synchronise with it only where stated.
 *  - A context owns the precomputed FFT of the discretised Green's tensor for one grid and
 *    medium (and, when a partition is given, for each distinct sub-domain shape) plus the
 *    work buffers.  A context may be used by one thread at a time.
 */
#ifndef IE_H
#define IE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define IE_OK          0
#define IE_ENOCONV     1
#define IE_EINVAL    (-1)
#define IE_ENOMEM    (-2)
#define IE_EDEVICE   (-3)
#define IE_ESTATE    (-4)

/* precision of the internal arithmetic */
#define IE_FP64   1   /* complex128 throughout */
#define IE_MIXED  2   /* complex64 convolutions and inner Krylov vectors; float64 residuals,
                         Arnoldi scalars, Givens rotations and solution accumulation */

/* form of the operator handed to the Krylov solver (both give the same E, eq. 8) */
#define IE_CONVENTIONAL  0   /* (I - G dsigma) E = E0, the paper's choice (end of section 2.3) */
#define IE_CIE           1   /* contraction form: (I - b - 2 sigma0 G b) e = sqrt(sigma0) E0,
                                b = dsigma (2 sigma0 I + dsigma)^-1, E = 2 sqrt(sigma0)
                                (2 sigma0 I + dsigma)^-1 e (introduction; end of section 2.3) */
#define IE_GREEN_ONLY    2   /* ie_matvec only: y = G x, the bare convolution of eq. (10) */
#define IE_SCATTER       3   /* ie_matvec only: y = G (dsigma x), the scattered field of eq. (3) */

/* outer schemes (section 2.3) */
#define IE_GS      0   /* block Gauss-Seidel, eqs. (19)-(22) */
#define IE_JACOBI  1   /* block Jacobi, eqs. (23)-(24) */
/* Krylov outer iteration in place of the stationary sweeps (the improvement the conclusions
 * propose): flexible GMRES(inner.restart) on the full-domain eq. (8) in float64, right-
 * preconditioned by one sweep of the scheme from zero with block solves to inner_tol_fixed
 * (adaptive is ignored).  Statistics: sweeps = outer steps (one preconditioner application
 * each), total_its = inner iterations, relres[k] = residual estimate after step k. */
#define IE_FGMRES_GS     2
#define IE_FGMRES_JACOBI 3

/* initial guess of ie_dd_solve */
#define IE_INIT_BACKGROUND 0  /* E := E0, as Alg. 1 */
#define IE_INIT_USER       1  /* E_total holds the initial guess on entry (resume) */
#define IE_INIT_LEARNED    2  /* E := 0, first-sweep block guesses from a trained network (ie_nn_*) */
#define IE_INIT_ZERO       3  /* E := 0 (first sweep: zero coupling and zero block starts) */

/* source kinds */
#define IE_MAG_DIPOLE   0   /* magnetic dipole, J^H = i omega mu0 m delta (eq. 1) */
#define IE_ELEC_DIPOLE  1   /* electric dipole, E0 = G^E p */

typedef struct {
    int32_t nx, ny, nz;   /* cells per axis (each 1..512) */
    double  h;            /* cubic cell size (m), > 0 */
    double  origin[3];    /* corner of cell (0,0,0); cell (i,j,k) centre = origin + (i+.5,j+.5,k+.5) h */
} ie_grid;

typedef struct {
    double sigma0;    /* homogeneous isotropic background conductivity (S/m), > 0 (section 2.1) */
    double freq_hz;   /* frequency (Hz), > 0 */
    double mu0;       /* magnetic permeability (H/m); 0 selects 4e-7 pi */
} ie_medium;

typedef struct {
    double  pos[3];     /* position (m); must not coincide with a cell centre */
    double  moment[3];  /* dipole moment (A m^2 for magnetic, A m for electric) */
    int32_t kind;       /* IE_MAG_DIPOLE or IE_ELEC_DIPOLE */
} ie_source;

typedef struct {
    int32_t        nblocks;   /* M >= 1 */
    const int32_t* z_bounds;  /* HOST array of M+1 strictly increasing z cell indices, 0 .. nz */
} ie_partition;

typedef struct {
    double  tol;         /* stop when ||b - A x|| / ||b|| <= tol (eq. 9 for the full domain) */
    int32_t restart;     /* Krylov dimension per cycle (section 3.1 uses 10); 1..16 */
    int32_t max_its;     /* limit on Arnoldi steps (operator applications); > 0 */
    int32_t precision;   /* IE_FP64 or IE_MIXED */
    int32_t form;        /* IE_CONVENTIONAL or IE_CIE */
    int32_t reorth;      /* Gram-Schmidt passes: 1 (classical), 2 (repeated once), 0 = default (1) */
} ie_gmres_opts;

typedef struct {
    int32_t its;          /* Arnoldi steps (the paper's "GMRES iterations") */
    int32_t restarts;     /* restart cycles after the first */
    int32_t refinements;  /* IE_MIXED: float64 residual corrections */
    int32_t matvecs64;    /* float64 operator applications */
    int32_t matvecs32;    /* complex64 operator applications */
    int32_t graph_cycles; /* restart cycles replayed from a captured hipGraph */
    double  relres;       /* final relative residual, recomputed in float64 */
    double  seconds;      /* wall time measured on the host around the call */
} ie_gmres_stats;

#define IE_MAX_SWEEPS 128
#define IE_MAX_BLOCKS 16

typedef struct {
    int32_t scheme;           /* IE_GS or IE_JACOBI */
    int32_t adaptive;         /* 1: inner tol = e/10 (Alg. 1); 0: inner tol = inner_tol_fixed */
    int32_t max_sweeps;       /* outer sweeps limit (<= IE_MAX_SWEEPS) */
    int32_t init;             /* IE_INIT_* */
    double  tol;              /* outer stop: full-domain relative residual (eq. 9) <= tol */
    double  inner_tol_fixed;  /* used when adaptive == 0 (section 3.2 uses 1e-6) */
    ie_gmres_opts inner;      /* inner block solves (tol field ignored) */
    const void* nn;           /* ie_nn handle for IE_INIT_LEARNED, else NULL */
    int32_t residual_cells;   /* IE_RESID_ALL: e over all cells (eq. 9); IE_RESID_ANOMALOUS: e over
                                 the cells with contrast only, as the isolated sub-domains example
                                 computes it (section 3.1; stationary sweeps only) */
} ie_dd_opts;

#define IE_RESID_ALL        0
#define IE_RESID_ANOMALOUS  1

typedef struct {
    int32_t sweeps;
    int32_t total_its;                               /* sum of inner Arnoldi steps */
    int32_t nblocks;
    int32_t block_its[IE_MAX_SWEEPS][IE_MAX_BLOCKS];
    double  relres[IE_MAX_SWEEPS + 1];               /* full-domain e before sweep 1 and after each sweep */
    int32_t matvecs64, matvecs32;                    /* operator applications, all grids */
    int32_t full_matvecs;                            /* full-domain convolutions (coupling + residual) */
    int32_t learned_used;                            /* blocks whose learned guess was accepted */
    int32_t graph_cycles;                            /* inner restart cycles replayed from graphs */
    double  seconds;
    int32_t best_sweep;   /* stationary sweeps: the sweep whose iterate is returned (smallest e) */
    int32_t diverged;     /* 1 if stopped because e grew in two consecutive sweeps */
} ie_dd_stats;

typedef struct {
    const ie_grid*   grid;      /* must equal the context's grid */
    const double*    sigma6;    /* DEVICE [6][nz][ny][nx] */
    const ie_source* sources;   /* HOST array */
    int32_t          nsources;
    void*            E_total;   /* DEVICE complex128 [3][nz][ny][nx]: output (input for IE_INIT_USER) */
    void*            E_anom;    /* DEVICE complex128 or NULL: output E - E0 */
} ie_problem;

typedef struct ie_ctx ie_ctx;

/*
 * ie_green_setup - precompute FFT[G] for a grid and medium (text after eq. 10: the FFT of
 * Green's tensor is computed once before the iterative solvers run).
 *   grid, medium  : host structs; validated (IE_EINVAL on bad sizes or non-positive values).
 *   partition     : NULL, or the z-slab partition used by ie_dd_solve; one additional
 *                   spectrum is built per distinct slab thickness.
 *   precision_mask: IE_FP64 | IE_MIXED - which spectra to keep (complex128, complex64).
 *   stream        : work is queued on it; the call synchronises before returning.
 *   out           : receives the new context (NULL on error).
 * Memory: about 1.5 (nx+1)(ny+1)(nz+1) complex values per spectrum (one octant of the six
 * components) plus padded work buffers of about 18 nx ny nz complex values per precision.
 */
int ie_green_setup(const ie_grid* grid, const ie_medium* medium, const ie_partition* partition,
                   int32_t precision_mask, void* stream, ie_ctx** out);

/* Release a context and all device memory it owns (synchronises the device first). */
int ie_ctx_destroy(ie_ctx* ctx);

/*
 * ie_background_field - E0 on the cell centres for point dipoles in the background medium
 * (the E^(0) of eq. 3; source term of eq. 1).
 *   sources : HOST array of nsources >= 1 entries.
 *   E0      : DEVICE complex128 [3][nz][ny][nx], written.
 */
int ie_background_field(ie_ctx* ctx, const ie_source* sources, int32_t nsources, void* E0,
                        void* stream);

/*
 * ie_matvec - one application of the discretised operator on the full grid of the context.
 *   sigma6    : DEVICE float64 [6][nz][ny][nx] (ignored for IE_GREEN_ONLY).
 *   x, y      : DEVICE [3][nz][ny][nx] complex128 (precision IE_FP64) or complex64
 *               (IE_MIXED); x and y must not overlap.
 *   form      : IE_CONVENTIONAL  y = x - G (dsigma x)                     (eq. 8)
 *               IE_CIE           y = (I - b) x - 2 sigma0 G (b x)
 *               IE_GREEN_ONLY    y = G x                                  (eq. 10)
 *               IE_SCATTER       y = G (dsigma x)                         (eq. 3)
 * Asynchronous on `stream`.
 */
int ie_matvec(ie_ctx* ctx, const double* sigma6, const void* x, void* y, int32_t form,
              int32_t precision, void* stream);

/* Size in bytes of the fixed per-device scratch array of ie_matvec_noalloc. */
#define IE_NOALLOC_MAX_BYTES (64u << 20)

/*
 * ie_matvec_noalloc - ie_matvec for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Arguments, forms,
 * layouts and result are those of ie_matvec (the same kernels and launch variants run).
 *   Scratch: the prepared contrast tensor, the padded FFT work arrays and a validation flag live
 *            in one fixed device array of IE_NOALLOC_MAX_BYTES per device, whose address is
 *            resolved when a context is set up on that device; the call itself allocates
 *            nothing.  A grid whose scratch exceeds the array is rejected with IE_EINVAL
 *            (6 r N + 3 s LZ nx (ny + LY) bytes, r/s = real/complex size of the precision: up
 *            to 64^3 cells in IE_MIXED, 48^3 in IE_FP64).
 *   Sharing: every call on a device uses that device's one array, which keeps the last call's
 *            contents; calls that overlap in time on one device race and must be serialised
 *            by the caller (one stream, or events).
 *   The current device must be the context's (IE_EINVAL otherwise).  Unless form is
 *   IE_GREEN_ONLY the call synchronises `stream` once to read the tensor validation flag.
 */
int ie_matvec_noalloc(ie_ctx* ctx, const double* sigma6, const void* x, void* y, int32_t form,
                      int32_t precision, void* stream);

/*
 * ie_gmres - solve (I - G dsigma) x = b on the context's full grid by restarted GMRES
 * (section 2.2; restart length from opts, section 3.1 uses 10).
 *   b : DEVICE complex128 [3][nz][ny][nx] right-hand side.
 *   x : DEVICE complex128, initial guess on entry, solution on exit.
 * With opts->form == IE_CIE the contraction form is iterated internally; x is always E.
 * With opts->precision == IE_MIXED the Krylov solve runs in complex64 on corrections of a
 * float64 residual until the float64 relative residual reaches opts->tol.
 * Returns IE_ENOCONV if max_its is reached first.  Synchronises with `stream`.
 */
int ie_gmres(ie_ctx* ctx, const double* sigma6, const void* b, void* x,
             const ie_gmres_opts* opts, ie_gmres_stats* stats, void* stream);

/*
 * ie_dd_solve - Alg. 1 for one or more problems: E0 from the sources, then block
 * Gauss-Seidel or Jacobi sweeps over the context's partition until the full-domain
 * relative residual of eq. (9) is <= opts->tol.  Each block solve is restarted GMRES on
 * (I - G(ii) dsigma(i)) warm-started from the previous sweep; the coupling terms
 * sum_{j != i} G(ij) dsigma(j) E(j) use the latest (GS) or previous-sweep (Jacobi) fields.
 * Sub-domains without contrast take E(i) = right-hand side with no inner iterations.
 *   ctxs[p], problems[p], stats[p] for p < nproblems (problems may have different grids;
 *   each context must have been set up with a partition).  Problems are advanced together.
 * The stationary sweeps converge only when the block splitting contracts (section 2.3); a
 * problem whose relative residual grows in two consecutive sweeps is stopped (stats.diverged),
 * and every problem that did not reach opts->tol returns the iterate of smallest residual
 * (stats.best_sweep) in E_total / E_anom.
 * Returns IE_ENOCONV if any problem hit max_sweeps or was stopped; the message names the cause.
 * Synchronises with `stream`.
 */
int ie_dd_solve(ie_ctx* const* ctxs, int32_t nproblems, const ie_problem* problems,
                const ie_dd_opts* opts, ie_dd_stats* stats, void* stream);

/*
 * Launch profiler for measurement harnesses.  Between ie_profile_begin() and ie_profile_end()
 * every kernel launch of the operator and Krylov passes is bracketed by HIP events recorded on
 * the launch stream.  ie_profile_end() synchronises the device and returns one record per
 * (kernel, shape, precision), sorted by total time, with the algorithmic bytes each launch must
 * move (compulsory reads and writes, each counted once).  `out` is a HOST array of `cap`
 * records; `count` receives the number of distinct records (may exceed cap).
 */
typedef struct {
    char    name[96];
    int32_t launches;
    double  total_ms, min_ms, max_ms;
    double  bytes_per_launch;
} ie_kernel_stat;

int ie_profile_begin(void);
int ie_profile_end(ie_kernel_stat* out, int32_t cap, int32_t* count);

/*
 * Learned initial guess (not in the paper, whose inner solves start from the previous sweep):
 * a 3-D convolutional encoder-decoder with hand-written BF16 MFMA kernels (float32
 * accumulation, float32 master weights, Adam).  Level l has base_ch * 2^l channels; 3x3x3
 * convolutions with bias and ReLU; encoder levels joined by 2x2x2 average pooling, decoder
 * levels by nearest 2x upsampling and concatenation with the encoder output of the same level;
 * a 1x1x1 head.  Tensors are channels-last [batch][nz][ny][nx][ch]; network inputs are BF16
 * (uint16 bit patterns), outputs and targets float32; all DEVICE pointers.  nz, ny, nx must be
 * divisible by 2^(levels-1).  Parameters: per layer W[taps][c_in][c_out] then bias[c_out],
 * layers in forward order.  A network is used by one thread at a time.
 * For the solver the network maps the 14 feature channels that ie_nn_features writes (the
 * contraction-form tensor, the phase-normalised right-hand side and k0 h; see there) to the 6
 * channels of ie_nn_target (re, im of the phase-normalised (E - b) / rms(b)).
 */
typedef struct ie_nn ie_nn;
typedef struct {
    int32_t  in_ch, out_ch, base_ch, levels;
    uint64_t seed;       /* weight initialisation (He normal, zero bias) */
} ie_nn_config;

int ie_nn_create(const ie_nn_config* cfg, void* stream, ie_nn** out);
int ie_nn_destroy(ie_nn* nn);
int ie_nn_num_params(const ie_nn* nn, int64_t* count);
/* which = 0: float32 master weights, 1: gradients of the last backward; HOST array */
int ie_nn_get_params(const ie_nn* nn, float* host, int64_t count, int32_t which);
int ie_nn_set_params(ie_nn* nn, const float* host, int64_t count);  /* resets Adam state */
int ie_nn_forward(ie_nn* nn, const uint16_t* x, int32_t batch, int32_t nz, int32_t ny, int32_t nx,
                  float* y, void* stream);
/* forward, then parameter gradients of <dy, y> (read with ie_nn_get_params(..., 1)) */
int ie_nn_backward(ie_nn* nn, const uint16_t* x, const float* dy, int32_t batch, int32_t nz,
                   int32_t ny, int32_t nx, float* y, void* stream);
/* one Adam step on the mean squared error to `target`; loss (HOST, nullable) is synchronised */
int ie_nn_train_step(ie_nn* nn, const uint16_t* x, const float* target, int32_t batch, int32_t nz,
                     int32_t ny, int32_t nx, float lr, float* loss, void* stream);
/*
 * The network's GEMM kernel alone (for tests of its matrix-core operand layout):
 * C[M][N] = op(A) op(B), float32 row-major output, BF16 inputs; op(A) is A [M][K] (a_trans = 0)
 * or A^T with A stored [K][M]; op(B) is B [K][N] (b_trans = 0) or B^T with B stored [N][K];
 * the K range is split `splits` ways (1..64) and the partial products summed in fixed order.
 * DEVICE pointers; synchronises with `stream`.
 */
int ie_nn_gemm(const uint16_t* A, const uint16_t* B, float* C, int32_t M, int32_t N, int32_t K,
               int32_t a_trans, int32_t b_trans, int32_t splits, void* stream);
/*
 * Solver features and targets on the context's full grid (nx*ny*nz = N cells).
 * ie_nn_features: x (DEVICE BF16 [N][14]) from sigma6 (DEVICE float64 [6][N]) and the
 * right-hand side b (DEVICE complex128 [3][N]): channels 0-5 the contraction-form tensor
 * I - 2 sigma0 (sigma + sigma0 I)^-1 (xx, yy, zz, xy, xz, yz), 6-11 re/im of
 * b e^{-i phi} / rms(b) for x, y, z, 12-13 re/im of k0 h, with rms(b) = ||b|| / sqrt(3N) and
 * phi = arg(sum b.b) / 2 (unconjugated sum), so that a global phase of b does not change the
 * features; rms(b) goes to *rms (HOST, nullable).
 * ie_nn_target: y (DEVICE float32 [N][6]) = re/im of (E - b) e^{-i phi} / rms(b).
 * Both synchronise with `stream`.
 */
int ie_nn_features(ie_ctx* ctx, const double* sigma6, const void* b, uint16_t* x, double* rms,
                   void* stream);
int ie_nn_target(ie_ctx* ctx, const void* b, const void* E, float* y, void* stream);
/*
 * The network's guess for (I - G dsigma) x = b on the context's full grid, unjudged:
 * x = b + rms(b) e^{i phi} network(features) (DEVICE complex128 [3][N]).  Synchronises.
 */
int ie_nn_predict(ie_ctx* ctx, ie_nn* nn, const double* sigma6, const void* b, void* x,
                  void* stream);
/*
 * Learned initial guess for (I - G dsigma) x = b on the context's full grid:
 * x_nn = b + rms(b) e^{i phi} network(features).  x (DEVICE complex128, in: default guess, out:
 * chosen guess) becomes whichever of x_nn, the default guess and zero has the smallest float64
 * residual ||b - (I - G dsigma) x||; *accepted (HOST, nullable) = 1 learned, 0 default, 2 zero.
 * Synchronises with `stream`.
 * ie_dd_solve with init = IE_INIT_LEARNED uses the network in the first sweep: for every block
 * it runs one restart cycle of the inner GMRES from x_nn and one from the default start and
 * continues from whichever reached the smaller residual (both cycles count in the statistics;
 * learned_used counts the blocks that continued from x_nn).  The network must divide each
 * block's grid.
 */
int ie_nn_guess(ie_ctx* ctx, ie_nn* nn, const double* sigma6, const void* b, void* x,
                int32_t* accepted, void* stream);

/*
 * Magnetic field at receiver points (eqs. 4 and 6): with eq. (5), G^H J = grad g(r - r') x J, so
 *   H(r) = H0(r) + h^3 sum_c grad g(r - r_c) x (dsigma E)_c
 * over the cells of the context's grid (collocation at cell centres as in eq. 8; a receiver at a
 * cell centre gets nothing from that cell).  H0: sigma0 G^E m for a magnetic dipole,
 * grad g x p for an electric dipole.  The induction-log response of a z transmitter is H_z.
 *   sigma6 : DEVICE float64 [6][nz][ny][nx];  E : DEVICE complex128 [3][nz][ny][nx], the total field
 *   src    : HOST [nsrc] transmitters (nsrc >= 0);  rx : HOST float64 [nrx][3] positions (m),
 *            1 <= nrx <= 4096, none within 1e-9 h of a transmitter
 *   H      : HOST complex128 [nrx][3] total field;  Ha : HOST complex128 [nrx][3] or NULL, H - H0
 * Deterministic (fixed-order sums).  Synchronises with `stream`.
 */
int ie_receivers(ie_ctx* ctx, const double* sigma6, const ie_source* src, int32_t nsrc,
                 const void* E, const double* rx, int32_t nrx, void* H, void* Ha, void* stream);

/*
 * Library options (process-wide).
 *   IE_OPT_GRAPHS: 1 (default) replays each Krylov restart cycle as a captured hipGraph; 0 issues
 *                  every kernel launch directly (the launch profiler always uses direct launches).
 *   IE_OPT_AUTOTUNE: 1 (default) makes ie_green_setup time the launch variants of each FFT pass
 *                  (values per thread, columns or rows per block) inside the whole operator on
 *                  every grid it builds and keep the fastest (cached per device, precision and
 *                  grid for the process); 0 uses the default variant.  Affects contexts set up
 *                  afterwards.
 *   IE_OPT_FORCE_VARIANT: -1 (default) leaves the choice to the autotuner; 0 .. 7 puts every
 *                  pass of contexts set up afterwards on that variant (the y passes, which have
 *                  four variants, take it modulo 4, the z passes, which have two, modulo 2): for
 *                  tests that cover every variant.
 *   IE_OPT_GROUP_THREADS: 1 (default) lets ie_dd_solve advance the problems of different
 *                  contexts at the same time (one host thread and one stream per context, joined
 *                  to the caller's stream); 0 solves the groups one after the other.  Results are
 *                  the same either way.
 *   IE_OPT_FFT_LENGTHS: 0 (default) pads each axis of n cells to the shorter of the smallest
 *                  power of two and the smallest 3 * 2^k (24 .. 768) that is >= 2n - 1 (the
 *                  linear convolution of eq. 10 needs 2n - 1 points; 48 cells take 96, not 128);
 *                  1 uses powers of two only; 2 sets up both where they differ, times one
 *                  operator application of each (after autotuning each) and keeps the faster
 *                  (about twice the setup time).  Affects contexts set up afterwards.
 * Returns IE_EINVAL for an unknown option or value.
 */
#define IE_OPT_GRAPHS 1
#define IE_OPT_AUTOTUNE 2
#define IE_OPT_FORCE_VARIANT 3
#define IE_OPT_GROUP_THREADS 4
#define IE_OPT_FFT_LENGTHS 5
int ie_set_option(int32_t option, int32_t value);

/*
 * The autotuner's decisions for a context as JSON text in buf (HOST, len bytes): one object per
 * (grid, precision, pass) with the grid's FFT lengths ("fft": [LX, LY, LZ]), the operator
 * microseconds of the shortest and the power-of-two lengths when IE_OPT_FFT_LENGTHS = 2 chose
 * between them ("lengths_us", zeros otherwise), the chosen variant, the template name of the
 * kernel that runs the pass ("kernel", as profilers print it) and, per variant of that pass,
 * the measured microseconds of one whole operator application with the pass at that variant.
 * IE_EINVAL if buf is too small.
 */
int ie_ctx_tuning(const ie_ctx* ctx, char* buf, int32_t len);

/*
 * The autotuner's process-wide cache as a file, so that later processes skip the timing:
 * ie_tuning_save writes every entry measured or loaded so far to `path` (HOST string; the file
 * is replaced) as a JSON array of objects {"arch": GPU architecture name, "precision": "c128" |
 * "c64", "grid": [nx, ny, nz], "fft": [LX, LY, LZ], "variant": [5 launch variants: zfwd, yfwd,
 * xconv, yinv, zinv], "us": [5 x 8 microseconds]}.  ie_tuning_load reads such a file and adds
 * its entries to the cache (replacing entries with the same key); a context set up afterwards
 * on a device of that architecture, for that grid, precision and FFT lengths, takes the stored
 * variants without timing.  Neither call touches the GPU.  IE_EINVAL if the file cannot be
 * opened or written, or (load) is not in this format or holds an out-of-range variant, grid or
 * length; nothing is loaded from a file that fails.
 */
int ie_tuning_save(const char* path);
int ie_tuning_load(const char* path);

/* Description of the last error on this thread (never NULL). */
const char* ie_last_error(void);

/* Library version string. */
const char* ie_version(void);

#ifdef __cplusplus
}
#endif

#endif /* IE_H */
