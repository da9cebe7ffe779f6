/*
 * fastfocus.h -- C ABI of the MI355X (gfx950) layered-BTTB sensitivity operator and the
 * focusing inversion built on it.
 *
 * Method (Renaut, Hogue & Vatankhah, arXiv 2004.13904):
 *   Sec. 2.1, eq. (blockG): G = [G^(1) ... G^(nz)], one BTTB block per depth layer, each
 *     entry the prism integral of the gravity (g_z) or magnetic (total-field anomaly) kernel.
 *   Appendix A: every G^(r) is embedded in a BCCB matrix; G x and G^T y are computed with
 *     2-D FFTs of the precomputed kernel spectra.
 *   Sec. 2.4, Algorithms 1 and 2: GKB and RSVD projected solves of the normal equations
 *     eq. (normalequations) of Sec. 2.3 with the UPRE regularization parameter; Secs. 2.2-2.3
 *     the IRLS focusing iteration.
 *
 * Conventions for every entry point
 *   - Model vectors (length n = nx*ny*nz) are ordered (layer r, row q, column p), p fastest;
 *     data vectors (length m = sx*sy) are ordered (row j, column i), i fastest.  Layer 0 is
 *     the top layer, z grows downward from the station plane z = 0.
 *   - Station (i, j) sits at the centre of surface cell (i + pad_xl, j + pad_yl).
 *   - All vector / matrix pointers are DEVICE pointers on the device the handle was built on,
 *     unless marked "host".  The caller owns them.  Buffers must not alias unless stated.
 *   - All work is enqueued asynchronously on `stream` (a hipStream_t; NULL = the null
 *     stream).  Argument validation is synchronous and happens before any launch.
 *   - Return value: FF_OK (0) or a negative ff_status.  No exception crosses the ABI.  The
 *     message of the last failure on the calling thread is returned by ff_last_error().
 *   - A handle owns device workspace for its operator passes: concurrent calls that use the
 *     same handle on different streams race; serialize them (one stream per handle).
 *   - Units: gravity entries in mGal per g/cc, magnetic entries in nT per SI susceptibility.
 */
#ifndef FASTFOCUS_H
#define FASTFOCUS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ff_status;
#define FF_OK        0
#define FF_EINVAL   (-1)   /* bad argument value or NULL pointer                          */
#define FF_ESHAPE   (-2)   /* sizes inconsistent with the handle, or embedding too small   */
#define FF_EDTYPE   (-3)   /* unsupported dtype for this call                              */
#define FF_ENOMEM   (-4)   /* device allocation failed, or workspace too small             */
#define FF_EHIP     (-5)   /* a HIP runtime / launch error                                 */
#define FF_EDEVICE  (-6)   /* pointer or stream on another device than the handle          */
#define FF_ENOTIMPL (-7)   /* configuration not implemented                                */

#define FF_GRAVITY_GZ   0  /* vertical attraction g_z of a unit-density prism            */
#define FF_MAGNETIC_TFA 1  /* total-field anomaly of a unit-susceptibility prism, induced  */

#define FF_F32 0           /* FP32 operator: complex64 spectra, float vectors              */
#define FF_F64 1           /* FP64 operator: complex128 spectra, double vectors            */

typedef void *ff_stream;   /* hipStream_t */

/* Survey and volume geometry (Sec. 2.1, Fig. 1).  z_edges is a HOST array of nz + 1
   increasing depths with z_edges[0] == 0 (the station plane).  nx = sx + pad_xl + pad_xr,
   ny = sy + pad_yl + pad_yr.  The magnetic kernel uses induced magnetization parallel to
   the inducing field of inclination incl_deg, declination decl_deg (x = north, y = east,
   z = down) and intensity field_nT.  nfft_x / nfft_y choose the BCCB embedding size; 0
   picks the smallest power of two >= sx + nx - 1 (resp. sy + ny - 1).  Any size >= that
   bound gives the same product (Appendix A); smaller sizes are rejected (FF_ESHAPE).
   Supported embedding sizes: powers of two from 8 to 2048. */
typedef struct {
    int32_t sx, sy, nz;
    int32_t pad_xl, pad_xr, pad_yl, pad_yr;
    double dx, dy;
    const double *z_edges;
    int32_t kernel;
    double incl_deg, decl_deg, field_nT;
    int32_t nfft_x, nfft_y;
} ff_geometry;

typedef struct ff_spectra_s *ff_spectra;

/* Appendix A (the kernel spectra are formed once, before any product): evaluates the per-offset kernel table
   t_r(u, v) of every layer from the prism formulas in FP64, places it in the circulant
   array of the embedding and stores its 2-D DFT (scaled by 1/(nfft_x*nfft_y)) on the
   current device, as complex64 (dtype FF_F32) or complex128 (FF_F64).  Also allocates the
   handle's pass workspace: the intermediates of one batched launch, about twice its row-pass
   intermediates (the batch is the largest multiple of 4 in 16..128 vectors whose row-pass
   intermediates fit in 512 MiB, else 16).  Blocks until the spectra are built.  *out receives the handle;
   free it with ff_free_spectra. */
ff_status build_spectra(const ff_geometry *geom, int32_t dtype, ff_stream stream, ff_spectra *out);
ff_status ff_free_spectra(ff_spectra h);

/* Spectra checkpoints (the precomputed 2-D FFTs of the kernel arrays, Appendix A): save writes
   the geometry, dtype and spectra of h to the host file `path` (FF_EINVAL if it cannot be
   written); load rebuilds a handle from such a file without evaluating the prism kernels or the
   FFTs again and returns it in *out (free with ff_free_spectra).  Load rejects files of another
   format version, truncated files and spectra whose stored hash does not match (FF_EINVAL),
   and geometry that build_spectra would reject.  Both block until done; the handle is on the
   current device.  A loaded handle applies G and G^T bit for bit like the saved one. */
ff_status ff_spectra_save(ff_spectra h, const char *path);
/* The geometry a handle was built with (embedding sizes in nfft_x, nfft_y).  z_edges, if not
   NULL, receives nz + 1 values and is stored in g->z_edges (call first with NULL to read nz). */
ff_status ff_spectra_geometry(ff_spectra h, ff_geometry *g, double *z_edges);
ff_status ff_spectra_load(const char *path, ff_stream stream, ff_spectra *out);

/* Sizes of a handle (host outputs, any may be NULL). */
ff_status ff_spectra_info(ff_spectra h, int64_t *m, int64_t *n, int32_t *nfft_x,
                          int32_t *nfft_y, int32_t *dtype);

/* Writes the FP64 kernel table t_r(u, v) (Sec. 2.1: entry of G^(r) for station-to-prism
   offsets u = i + pad_xl - p, v = j + pad_yl - q) to the DEVICE array `table` of
   nz * (sy + ny - 1) * (sx + nx - 1) doubles, indexed [r][v - v0][u - u0] with
   u0 = pad_xl - nx + 1, v0 = pad_yl - ny + 1.  For verification of the prism kernels. */
ff_status ff_kernel_table(ff_spectra h, double *table, ff_stream stream);

/* The device FFT of the operator's passes (App. A: the 2DFFT is applied as 1-D transforms along
   rows and columns) applied stand-alone, for verification against a reference FFT: count
   transforms of length n (a power of two in [8, 2048]), out[b] = sum_k in[b][k] exp(-+2 pi i j k / n)
   (minus for inverse = 0, plus and unnormalized for inverse = 1).  in, out: count x n complex
   values (interleaved re, im) of dtype FF_F32 or FF_F64; twiddles: device scratch of n complex
   values of the same dtype (filled here).  plan: the stage plan (0, 1 or 2, as fft_plan_x of
   ff_tuning).  Asynchronous on `stream`. */
ff_status ff_fft_1d(int32_t n, int32_t dtype, int32_t inverse, int32_t plan, int64_t count, const void *in,
                    void *out, void *twiddles, ff_stream stream);

/* Appendix A, eq. (costGx): d = w_post .* G (w_pre .* x).  x: n values, d: m values, both of
   the handle's dtype (float or double).  w_pre (n) and w_post (m) are optional diagonal
   weights of the same dtype (NULL = identity); with w_pre = W^{-1} and w_post = W_d this is
   the weighted operator G~ of eq. (forwardmult).  Layer contributions are summed in the
   frequency domain, so one call costs nz forward 2-D FFTs and one inverse. */
ff_status apply_G(ff_spectra h, const void *x, void *d, const void *w_pre, const void *w_post,
                  ff_stream stream);

/* Appendix A: x = w_post .* G^T (w_pre .* d).  d: m values, x: n values, w_pre (m), w_post
   (n), same dtype conventions as apply_G.  One forward 2-D FFT and nz inverse. */
ff_status apply_GT(ff_spectra h, const void *d, void *x, const void *w_pre, const void *w_post,
                   ff_stream stream);

/* Sec. 2.5 (a product with a matrix of t_p columns is that many vector products) and Appendix A:
   Y = w_post .* G (w_pre .* X) for transpose = 0, Y = w_post .* G^T (w_pre .* X) for
   transpose = 1, for k column vectors.  X is column-major with leading dimension ldx
   (>= n, or >= m when transposed), Y likewise with ldy.  The weights apply to every column.
   Vectors are processed in launches of up to the handle's batch (16 to 128 vectors, chosen at
   build_spectra from the intermediates' size); in single precision G's column pass takes 8
   vectors per block and G^T's 4, which agree with the one-vector launches to rounding. */
ff_status apply_G_block(ff_spectra h, int32_t transpose, int64_t k, const void *X, int64_t ldx,
                        void *Y, int64_t ldy, const void *w_pre, const void *w_post,
                        ff_stream stream);

/* For callers that cannot allocate device memory: code under HIP graph capture, tight serving
   loops and harnesses that forbid hipMalloc.  Computes exactly what apply_G_block computes (same
   arguments, same pass kernels, results equal to its own), but keeps the pass intermediates in
   a fixed library array of FF_NOALLOC_SCRATCH_BYTES per device instead of the handle's
   workspace, and calls no allocating routine.  The array is part of the library's code object:
   each device the library runs on holds it from load until the process ends.  The k vectors
   go through in launches of at most the handle's batch, fewer when their intermediates
   (nz * nfft_x/2 * ny rounded up to 16, plus a data-sized column buffer per layer group of G,
   complex values of the handle's dtype, per vector) would not fit the array; FF_ENOMEM, before
   any launch, when a single vector's do not (e.g. nz = 20 at a 512 x 512 embedding needs
   about 9 MB per vector).  Every call on a device shares that device's array and leaves
   unspecified contents in it (nothing in it needs to start at zero): calls that may overlap
   on one device (other streams, threads or handles) race, so the caller must serialize them. */
#define FF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
ff_status ff_apply_block_noalloc(ff_spectra h, int32_t transpose, int64_t k, const void *X, int64_t ldx,
                                 void *Y, int64_t ldy, const void *w_pre, const void *w_post,
                                 ff_stream stream);

/* The focusing objective of the differentiable form, with the operator products inside:
   L = sum over the k models of ||wd .* (G m - d_obs)||^2 + alpha * sum_i m_i^2 / (m_i^2 + eps2),
   the data misfit of eq. (dfandstab) and the minimum-support stabilizer (eq. (WLdefn) with
   lambda = 0, W_h = W_z = I, D = I, m_apr = 0).  m: k x n, d_obs, wd, rw: k x m, all column-major
   with leading dimensions n and m, in the handle's dtype; alpha >= 0, eps2 > 0.
   ff_focusing_loss writes rw = 2 wd .* wd .* (G m - d_obs) (the misfit's gradient with respect to
   G m, kept for the gradient call) and, in the caller's device buffer `work` of 513 doubles,
   work[0] = L (summed in double, in a fixed order).
   ff_focusing_grad writes grad (k x n) = scale * (G^T rw + alpha * 2 m eps2 / (m^2 + eps2)^2),
   with scale a device double (NULL = 1): dL/dm times the caller's upstream factor.
   Both are asynchronous on `stream`. */
ff_status ff_focusing_loss(ff_spectra h, int64_t k, const void *m, const void *d_obs, const void *wd,
                           double alpha, double eps2, void *rw, double *work, ff_stream stream);
ff_status ff_focusing_grad(ff_spectra h, int64_t k, const void *m, const void *rw, double alpha,
                           double eps2, const double *scale, void *grad, ff_stream stream);

/* ---------------------------------------------------------------------------------------
   Projected solvers (Sec. 2.4) and IRLS (Secs. 2.2-2.3).  All vectors below are FP64 device arrays; the
   operator applications inside run in the handle's dtype.  `workspace` is a caller-owned
   device buffer of at least ff_workspace_size(...) bytes (it holds the n x t_p basis, or for GKB
   with the handle's gkb_onesided = 2 only the m x t_p one). */

#define FF_WS_GKB  0
#define FF_WS_RSVD 1
#define FF_WS_IRLS 2
/* which: FF_WS_GKB, FF_WS_RSVD or FF_WS_IRLS (then solver 0 = GKB, 1 = RSVD); basis_dtype:
   FF_F64 or FF_F32 storage of the GKB bases or of the RSVD n x t_p matrices; 1 <= tp <= m. */
ff_status ff_workspace_size(ff_spectra h, int32_t which, int32_t solver, int32_t basis_dtype, int32_t tp,
                            size_t *bytes);

/* Algorithm 1: GKB factorization G~ A = H B of G~ = diag(wd) G diag(winv) with
   reorthogonalization of A and H (of H only, and A possibly rebuilt instead of stored, under the
   handle's gkb_onesided tuning), SVD of the (tp+1) x tp bidiagonal B, and the solution
   y = ||r~|| A V Gamma(alpha, Sigma) U(1,:)^T.  Inputs r_tilde (m), wd (m), winv (n).
   alpha_mode: 0 = UPRE over the first t singular values, 1 = alpha^(1) of eq. (eq:alpha1),
   2 = fixed (*alpha on input).  basis_dtype: FF_F64 stores A and H in double precision (the
   default of the method); FF_F32 stores them in single precision (half the memory and the
   reorthogonalization traffic, orthogonality to about 1e-7; every product and sum is still
   formed in double).  Outputs y (n, standard form: the model update is winv .* y), *alpha
   (host), sigma (tp, device, descending).  1 <= t <= tp <= m. */
ff_status gkb_project(ff_spectra h, const double *r_tilde, const double *wd, const double *winv,
                      int32_t t, int32_t tp, int32_t alpha_mode, int32_t basis_dtype, double *y,
                      double *alpha, double *sigma, void *workspace, size_t ws_bytes,
                      ff_stream stream);

/* Algorithm 2: randomized SVD of G~ (same weights as above) with power_iters power iterations
   (the paper uses 1; 0 <= power_iters <= 8), eigen-decomposition of the symmetrized B^T B,
   UPRE over t values, solution y = Q V~ Gamma U~^T (B^T r~).  Outputs as gkb_project; sigma
   holds all tp values.  Omega is a tp x m FP64 device matrix (row-major, i.e. m-vectors stored
   one after another), or NULL: then it is drawn on the device from `seed` with the
   counter-based Philox4x32-10 generator (Salmon et al., SC 2011): element pair p from the
   counter (p mod 2^32, p div 2^32, 0, 0) and the key (seed mod 2^32, seed div 2^32), two
   53-bit uniforms and a Box-Muller transform (see k_gaussian in the sources).
   The QR factorizations of Algorithm 2 keep only Q.  It is formed by Cholesky QR (passes of
   Gram product, Cholesky, triangular inverse and product): two plain passes (CholeskyQR2),
   else three passes with a shifted first one (shifted CholeskyQR3), else Householder QR
   (geqrf + orgqr); a Cholesky result is accepted when every factorization succeeded and
   max |Q^T Q - I| <= 1e-8.  The call synchronizes `stream` after each attempt.
   basis_dtype: FF_F64 stores every matrix of the algorithm in double precision; FF_F32 (FP32
   handles only) stores the n x t_p matrices (Q and the copy kept for a second attempt) in
   single precision, about 8 (n + m) t_p bytes of workspace instead of 8 (3n + m) t_p: their
   Gram products and products with R^-1 run over row chunks converted to double, so all
   arithmetic stays FP64, Q is orthonormal to about 1e-7 (an attempt is accepted at
   max |Q^T Q - I| <= 1e-6) and, with no FP64 copy of the n x t_p matrix to fall back on, the call
   returns FF_ENOTIMPL when both Cholesky attempts fail (or rsvd_qr = 1). */
ff_status rsvd_project(ff_spectra h, const double *r_tilde, const double *wd, const double *winv,
                       int32_t t, int32_t tp, const double *omega, uint64_t seed, int32_t power_iters,
                       int32_t alpha_mode, int32_t basis_dtype, double *y, double *alpha, double *sigma,
                       void *workspace, size_t ws_bytes, ff_stream stream);

/* Counts of the RSVD orthonormalizations done on handle h so far: by CholeskyQR2, by shifted
   CholeskyQR3 and by Householder QR (see rsvd_project). */
ff_status ff_solver_stats(ff_spectra h, int64_t *qr_cholesky2, int64_t *qr_cholesky3, int64_t *qr_householder);

/* Parameters of one IRLS step (Sec. 2.2-2.3, Sec. 3.1). */
typedef struct {
    int32_t solver;      /* 0 = GKB, 1 = RSVD                                             */
    int32_t t, tp;       /* truncation and projected sizes                                */
    int32_t k;           /* 1-based IRLS iteration index                                  */
    double lambda;       /* eq. (WLdefn): 1 = L1-like, 0 = minimum support, 2 = smooth     */
    double eps2;         /* focusing parameter epsilon^2                                  */
    double beta_depth;   /* depth weighting exponent (0.8 gravity, 1.4 magnetic)          */
    double m_min, m_max; /* bound constraints                                             */
    double alpha_fixed;  /* > 0: use this alpha; otherwise eq. (eq:alpha1) at k = 1, UPRE after */
    int32_t power_iters; /* RSVD power iterations (the paper: 1)                            */
    uint64_t seed;       /* RSVD with omega = NULL: Omega drawn from (seed, counter word 2 = k) */
    int32_t basis_dtype; /* FF_F64 or FF_F32 storage of the n x t_p matrices (see gkb_project, rsvd_project) */
} ff_irls_params;

/* One IRLS step: W = W_z W_L^(k) with (W_L^(k))_ii = ((m_prev - m_prev2)_i^2 + eps2)^((lambda-2)/4)
   (identity at k = 1), r~ = wd .* (d_obs - G m_prev), projected solve (GKB, or RSVD with
   `omega` tp x m, or omega = NULL for the generator of rsvd_project with the third counter
   word set to k), m_new = clip(m_prev + W^{-1} y, m_min, m_max) and the
   scaled chi^2 of eq. (scaledchi2).  d_obs, wd: m; m_prev, m_prev2, m_new: n (FP64 device).
   *alpha and *chi2_scaled are host outputs.  A non-finite residual r~ (NaN or Inf in d_obs, wd
   or m_prev) returns FF_EINVAL before the solve, as does a step that produces non-finite values.
   The call synchronizes `stream` (after r~ and at the end). */
ff_status irls_step(ff_spectra h, const ff_irls_params *p, const double *d_obs, const double *wd,
                    const double *m_prev, const double *m_prev2, const double *omega,
                    double *m_new, double *alpha, double *chi2_scaled, void *workspace,
                    size_t ws_bytes, ff_stream stream);

/* Launch tuning of a handle (FFT stage plans, tile shapes and batch schedule).  build_spectra
   picks values that fill the chip; an autotuner may change them.  Results do not depend on them
   beyond rounding order (Appendix A: the 2-D DFT as 1-D transforms along x, then along y).
     fft_plan_x    stage plan of the NX-point row transforms, fft_plan_y of the NY-point column
                   transforms (eight elements per thread, stages of radix 8, 4 and 2):
                   0 (default) = radix-8 stages, then one radix-4 or radix-2 stage when log2 N is
                   not a multiple of 3; 1 = that radix-4 or radix-2 stage first (the same as 0 when
                   log2 N is a multiple of 3); 2 = radix-4 stages, then one radix-2 stage when
                   log2 N is odd.  They apply to apply_G, apply_GT, apply_G_block and the solvers;
                   grouped plans (ff_multi_create) use plan 0.
     lg_G, lg_GT   the layers of every column are split over this many groups of column-pass
                   blocks (1 <= lg <= nz); the G partial sums of the groups are added in the
                   inverse row pass.
     row_tile      transforms per row-pass block: 0 = automatic by the rows of the pass (one
                   transform below 512 rows, two below 1024, else four; inverse passes of at
                   least 2048 rows and every pass of at least 16384 rows take the largest tile
                   that fits 64 KB of LDS), 1 = always one
                   transform (two rows), 2 = always the largest tile, 3 = four transforms, 4 = two
                   transforms (3 and 4 capped by the largest tile).
     batch         vectors per launch of apply_G_block, 1 <= batch <= the batch the handle's
                   workspace was sized for (the value build_spectra sets).
     col_batched   column passes of block applies (single precision, nfft_y <= 512): 1 = four
                   vectors per block, the layers split over its wave groups; 2 (default) = the
                   same for G^T, and for G eight vectors per block, each wave group one whole
                   vector, the layer spectra staged in LDS once per block; 0 = one vector per
                   column block.
     rsvd_qr       orthonormalization inside rsvd_project: 0 = Cholesky QR with the fallbacks
                   described there, 1 = always Householder QR (geqrf + orgqr), 2 = start at the
                   shifted CholeskyQR3 (then Householder).
     pair_fused    grouped plans (ff_multi_create) that bind both G x and G^T d of this
                   survey: one column pass for both products, reading each layer spectrum once (it
                   splits the layers of both over lg_G groups), or separate column passes.
                   1 (default) = the shared pass when the plan holds this survey alone and its
                   column blocks (nfft_x/2 slots, lg_G groups) at least fill the device's compute
                   units; 2 = the shared pass in every plan; 0 = never.  The results are the same
                   bit for bit.
     gkb_graph     gkb_project and irls_step with GKB: 1 = the iteration loop of Algorithm 1
                   (about 24 launches per iteration, none waiting for the host) is captured into a
                   graph on the handle's own stream at the first solve and replayed by later solves
                   with the same workspace, t_p and basis type (not while the caller's stream is
                   being captured or pass profiling is on); 0 (default) = launched one by one.  The
                   results are the same bit for bit.
     gkb_onesided  reorthogonalization in gkb_project and irls_step with GKB (Algorithm 1 takes
                   both bases): 0 (default) = both bases, the model-side A (n x t_p) and the
                   data-side H (m x (t_p + 1)); 1 = the data-side basis H only: the model-side
                   vectors stay orthogonal through the recurrence when one side of the
                   Golub-Kahan process is kept orthogonal (Simon and Zha, SIAM J. Sci. Comput. 21,
                   2000), which removes the n-length streams over A; 2 = as 1, and A is not stored:
                   the solution y = A w is formed in a second pass that rebuilds every a_i from H
                   and the stored coefficients with the same launches (bit for bit the first pass's
                   vectors), at t_p more G^T applications; the workspace then holds two columns of
                   A instead of t_p (ff_workspace_size reads this setting).  Modes 1 and 2 give the
                   same B, sigma and alpha bit for bit; their y agree to rounding.  Against mode 0:
                   to rounding with an FP64 operator; with an FP32 operator the model-side basis
                   stays orthogonal to about the operator's rounding (4e-8 at n = 1e6, t_p = 2625)
                   and y moves by about 2e-7 at a fixed alpha. */
typedef struct {
    int32_t lg_G, lg_GT;
    int32_t row_tile;
    int32_t batch;
    int32_t col_batched;
    int32_t rsvd_qr;
    int32_t pair_fused;
    int32_t gkb_graph;
    int32_t fft_plan_x, fft_plan_y;
    int32_t gkb_onesided;
} ff_tuning;
ff_status ff_get_tuning(ff_spectra h, ff_tuning *t);
ff_status ff_set_tuning(ff_spectra h, const ff_tuning *t);

/* Pass profiling (instrumentation for benchmarks).  ff_profile_begin makes every following
   operator call on this handle record a HIP event on its stream before pass 1 and after each of
   its three passes, for at most max_ops calls.  ff_profile_end waits for those events and
   writes the summed durations in milliseconds: ms[3*t + p] for transpose t (0 = G, 1 = G^T) and
   pass p (0 = row transforms, 1 = column transforms with spectral products, 2 = inverse row
   transforms), and the number of profiled calls per transpose in ops[t].  Block calls count
   each batched launch group as one call. */
ff_status ff_profile_begin(ff_spectra h, int32_t max_ops);
ff_status ff_profile_end(ff_spectra h, double *ms, int64_t *ops);

/* Pass timing (instrumentation for benchmarks): applies G (transpose = 0) or G^T (1) to x once,
   writing y (handle dtype, unweighted), then launches only pass `pass` (0, 1 or 2 as above)
   `reps` more times back to back on `stream`, re-reading the intermediates of that application.
   Events recorded around the call divided by reps give the pass kernel's own duration. */
ff_status ff_time_pass(ff_spectra h, int32_t transpose, int32_t pass, int32_t reps, const void *x, void *y,
                       ff_stream stream);

/* ---------------------------------------------------------------------------------------
   Several surveys at once (Sec. 2.5: the products are independent per column; here the columns
   belong to different surveys).  A plan binds, for count single-precision handles of distinct
   surveys, device vectors x[i] (n_i floats) -> gx[i] = G_i x[i] (m_i floats) and d[i] (m_i) ->
   gtd[i] = G_i^T d[i] (n_i); either pair of a survey may be NULL to skip that product.
   ff_multi_apply then computes all of them with three grouped launches on `stream`: every row
   transform of every survey, every column pass, every inverse row transform.  Results equal
   the handles' own apply_G / apply_GT.  Requirements: FP32 handles on the current device,
   embeddings of at most 512 x 512 (FF_ENOTIMPL otherwise; use the per-handle calls), each
   handle at most once (FF_EINVAL).  The plan copies its launch tables to the device
   (ff_multi_create blocks for that copy) and holds no reference to host memory; it uses the
   handles' pass workspaces, so no other call may use those handles while a multi apply runs.
   The bound vectors and the handles must outlive the plan. */
typedef struct ff_multi_s *ff_multi;
ff_status ff_multi_create(int32_t count, const ff_spectra *handles, const void *const *x, void *const *gx,
                          const void *const *d, void *const *gtd, ff_multi *out);
ff_status ff_multi_apply(ff_multi plan, ff_stream stream);
/* Pass timing of a plan (instrumentation for benchmarks): launches only the plan's grouped
   kernel `pass` (0 = row transforms, 1 = column passes, 2 = inverse row transforms) `reps` times
   back to back on `stream`, re-reading the intermediates the last ff_multi_apply left.  Events
   around the call divided by reps give that kernel's own duration. */
ff_status ff_multi_time_pass(ff_multi plan, int32_t pass, int32_t reps, ff_stream stream);
/* Frees the plan's host and device tables; NULL is accepted and does nothing. */
ff_status ff_multi_free(ff_multi plan);

/* Thread-local message of the last failure ("" if none).  Valid until the next call. */
const char *ff_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FASTFOCUS_H */
