/*
 * cip.h -- C ABI of the MI355X (gfx950) library for ADMM reconstruction of
 * convolutional inverse problems in multidimensional imaging
 * (Dogan & Oktem, arXiv 2006.08303).
 *
 * Problem (Section II, Eq. forward model): K measurements of S unknown planes,
 *     y_k = sum_{s=1..S} h_{k,s} * x_s + w_k,      k = 1..K,
 * with circular 2D convolutions on an N1 x N2 grid. The library solves the
 * regularised least-squares problem of Section III (Eq. rls),
 *     min_x  beta/2 ||y - H x||^2 + R(x),
 * with the ADMM iterations of Section IV (Algorithm 1 for analysis priors,
 * Algorithm 2 for synthesis priors), every step of which runs as hand-written
 * HIP kernels on the GPU.
 *
 * Conventions shared by every entry point
 *   - All array arguments named d_* are DEVICE pointers (HIP global memory),
 *     owned by the caller; the library never allocates, frees or retains them
 *     beyond the call, except the plan workspace (see cip_plan_create).
 *   - Arrays are float32, C order (row-major), the last index fastest:
 *       x   : [S][N1][N2]        unknown planes
 *       y   : [K][N1][N2]        measurements
 *       psf : [K][S][N1][N2]     blur kernels h_{k,s}, stored unshifted on the
 *                                torus: element [k][s][0][0] is the tap at zero
 *                                offset, [k][s][N1-1][0] the tap at offset -1.
 *   - `stream` is a hipStream_t (NULL = default stream). Every call enqueues
 *     work on that stream and returns without waiting for it, except
 *     cip_plan_create, which waits for its own precompute to finish.
 *   - Return value: CIP_OK (0) on success or a negative CIP_E* code; the
 *     message of the last failure on the calling thread is available from
 *     cip_last_error(). A failed call leaves the plan usable.
 *   - Supported grids: N1 and N2 in {16, 32, 64, 128, 256, 384, 512, 768,
 *     1024, 1536, 2048} (powers of two and 3 * 2^k); 1 <= K, S <= 8; the
 *     patch prior needs S <= 4 and power-of-two N1, N2.
 */
#ifndef CIP_H_
#define CIP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CIP_OK = 0,
  CIP_EINVAL = -1,        /* bad argument (null pointer, size out of range)  */
  CIP_EUNSUPPORTED = -2,  /* valid request this build cannot serve (grid size,
                             prior kind)                                       */
  CIP_ENOSPC = -3,        /* workspace smaller than cip_plan_workspace_bytes */
  CIP_EHIP = -4,          /* a HIP runtime call failed                        */
};

/* Priors (Section III). */
typedef enum {
  /* Analysis prior R(x) = lambda ||T x||_1 (Eq. analysis), T = circular forward
   * differences along both image axes of every plane (anisotropic TV). */
  CIP_PRIOR_TV2D = 0,
  /* As TV2D plus a forward difference along the plane (band) axis, without
   * wrap-around (3D correlations, Section III-A). */
  CIP_PRIOR_TV3D = 1,
  /* Analysis prior with T = orthonormal 2D DCT-II of every plane. */
  CIP_PRIOR_DCT2D = 2,
  /* Synthesis prior with a patch dictionary (Eq. patch_based): Q x Q x S
   * patches spanning all planes (Q = 8), extracted circularly at stride 4
   * (P^T P = 4 I), common dictionary D with A atoms; Algorithm 2 with the
   * sparse-code update of Eq. solz_patch2 on BF16 MFMA (FP32 accumulation). */
  CIP_PRIOR_PATCH = 3,
  /* Synthesis prior with a convolutional dictionary, 2D-correlation form
   * (Eq. conv_dic per plane with a common set of M filters of L x L, P = I):
   * Algorithm 2 with the frequency-domain sparse-code update of
   * Eqs. solz_DFT / solz_DFT_SM. */
  CIP_PRIOR_CONV2D = 4,
  /* Analysis prior with T = one 3D transform (Section III-A, data correlated
   * along all three dimensions): the orthonormal 2D DCT-II of every plane
   * followed by the orthonormal DCT-II along the plane (band) axis. */
  CIP_PRIOR_DCT3D = 5,
  /* Isotropic TV of every plane as stated in Section III-A (Phi(Tx) = TV(x)
   * with T = I): the t-update is the TV proximal map, computed with
   * Chambolle's projection algorithm (circular forward differences, step
   * 1/8, `tv_inner` iterations per ADMM iteration, dual warm-started from the
   * previous ADMM iteration). */
  CIP_PRIOR_ITV2D = 6,
  /* Convolutional dictionary with 3D filters and codes (Section IV-B, data
   * correlated along the bands too): plane s is sum_m sum_s' d_m[s'] (*)
   * z_m[(s - s') mod S], circular along the planes as in space; every
   * operator is diagonal in the 3D DFT, and the code update is the
   * Sherman-Morrison solve at every 3D frequency. `filters` holds M filters
   * of S x L x L taps ([M][S][L][L]); no gradient term (mu = 0). */
  CIP_PRIOR_CONV3D = 7,
  /* Wavelet (x) DCT analysis prior (Section V-A's Kronecker basis for the
   * analysis case): T = C_S (x) W, W the 2D Symmlet-8 wavelet transform of
   * every plane (periodized orthonormal DWT, Mallat's pyramid of
   * `wt_levels` levels: each level transforms the low-pass corner of the
   * previous one along both image axes), C_S the orthonormal DCT-II along
   * the planes. T is orthonormal, so the x-update is that of the DCT priors
   * (Psi = rho I + beta Lambda^H Lambda); Phi = l1. N1 and N2 must be
   * multiples of 2^wt_levels. */
  CIP_PRIOR_WDCT3D = 8,
  /* Isotropic TV of the whole cube (Section III-A with the
   * multidimensional derivative operators): the Euclidean norm at every
   * voxel of the gradient (circular forward differences along both image
   * axes, forward difference along the planes, none after the last plane).
   * T = I; the t-update is the proximal map of this TV by Chambolle's
   * algorithm with step 1/12, `tv_inner` iterations per ADMM iteration,
   * dual warm-started from the previous ADMM iteration. With S = 1 it is
   * CIP_PRIOR_ITV2D run at the smaller step. */
  CIP_PRIOR_ITV3D = 9,
} cip_prior_kind;

typedef struct {
  int kind;             /* cip_prior_kind                                     */
  double beta;          /* data-fidelity weight beta of Eq. rls (> 0)         */
  /* CIP_PRIOR_PATCH only (ignored otherwise):                                */
  const float* dict;    /* device [n][A] float32, row-major, n = Q*Q*S; row
                           s*Q*Q + a*Q + b is pixel (a, b) of plane s; column
                           k is atom k. Read during cip_plan_create only.     */
  int n_atoms;          /* A: 64, 128 or 256                                   */
  int patch_q;          /* Q: must be 8                                        */
  int patch_stride;     /* st: must be 4                                       */
  /* CIP_PRIOR_CONV2D and CIP_PRIOR_CONV3D only (ignored otherwise):         */
  const float* filters; /* device [M][L][L] float32 (CONV3D: [M][S][L][L]),
                           row-major; tap (a, b) acts at offset
                           (a - L/2, b - L/2), band tap s' at band offset s'.
                           Read during cip_plan_create only.                  */
  int n_filters;        /* M: 1 .. 32                                          */
  int filt_l;           /* L: 1 .. min(N1, N2)                                 */
  double mu;            /* gradient (Tikhonov) weight on the codes, Eq.
                           DL_PriorHP_conv for 2D correlations (forward
                           differences along both axes); 0 = none, >= 0;
                           must be 0 for CIP_PRIOR_CONV3D                   */
  /* CIP_PRIOR_ITV2D and CIP_PRIOR_ITV3D only:                                */
  int tv_inner;         /* Chambolle iterations per ADMM iteration (0: 20)    */
  /* All priors:                                                             */
  int flags;            /* CIP_PLAN_ADAPTIVE: keep what cip_solve_adaptive
                           needs to change the penalty: the FP64 kernel
                           spectra for the analysis priors
                           (K*S*N1*(N2/2+1)*16 more bytes), the FP64 filter
                           spectra for the conv priors (M*N1*(N2/2+1)*16,
                           times S for CONV3D), a host copy of D for the
                           patch prior, and t of the iteration before a
                           check for the isotropic TV priors
                           (S*N1*N2*4);
                           CIP_PLAN_DICT_UPDATE (CIP_PRIOR_PATCH,
                           CIP_PRIOR_CONV2D and CIP_PRIOR_CONV3D): learn
                           the dictionary online during every solve         */
  /* CIP_PLAN_DICT_UPDATE only:                                               */
  double sigma;         /* penalty of the dictionary ADMM (Eqs. ADMM0 and
                           d_admm), > 0; 0 selects the paper's settings: 1
                           for the patch dictionary, 10 for the
                           convolutional one                               */
  /* CIP_PRIOR_WDCT3D only:                                                   */
  int wt_levels;        /* wavelet levels, 1 .. 10 (0: 3)                     */
  /* CIP_PRIOR_PATCH only:                                                    */
  int patch_t;          /* patch depth T along the planes (Q x Q x T patches,
                           Eq. patch_based): 0 or S (patches span every
                           plane); other depths return CIP_EUNSUPPORTED    */
  /* CIP_PRIOR_CONV2D only:                                                   */
  int per_band;         /* 0: one common set of M filters for every plane
                           (the 2D-correlation form of Section III-B);
                           1: a separate set per plane, which this build does
                           not serve (CIP_EUNSUPPORTED)                     */
} cip_prior_desc;

enum { CIP_PLAN_ADAPTIVE = 1, CIP_PLAN_DICT_UPDATE = 2 };

typedef struct cip_plan_s* cip_plan_t;

/* Bytes of device workspace a plan of this shape needs (Algorithm 1/2, step 2
 * tables, solver state and staging). Returns CIP_EUNSUPPORTED for grids or
 * priors this build does not serve. No GPU work. */
int cip_plan_workspace_bytes(int K, int S, int N1, int N2, const cip_prior_desc* prior,
                             size_t* bytes);

/* Create a plan: uploads twiddle tables, transforms the kernels (FP64 FFTs)
 * and computes, at every 2D frequency w, the FP64 pseudo-inverse of
 *     Psi(w) = rho tau(w) I + beta Lambda(w)^H Lambda(w)
 * (Alg. 1 step 2; below Eq. solx_Trans_DFT; tau = 1 for a unitary T, the
 * Laplacian symbol for TV; TV3D adds rho times the band path-graph Laplacian;
 * for the patch prior Psi = 4 I + beta Lambda^H Lambda, Eq. solx_synt_DFT,
 * and M1 = D^T (rho I + D D^T)^-1 is formed in FP64 on the host and stored,
 * with D, in BF16; for the convolutional prior Psi = I + beta Lambda^H Lambda
 * and the filter spectra theta_m with 1 / (rho + sum_m |theta_m|^2) are
 * formed in FP64).
 * Eigenvalues below 1e-12 times the largest one at that frequency are treated
 * as zero (minimum-norm x-update where Psi is singular, e.g. the DC block with
 * unit-sum kernels and TV). Results are stored in FP32 in the workspace.
 *   d_psf      : [K][S][N1][N2] float32 device array, read during the call only.
 *   rho, lambda: ADMM penalty (> 0) and regularisation weight (>= 0; > 0
 *                for the isotropic TV priors); the soft threshold is
 *                lambda / rho (Eq. solt_trans), the TV proximal weight of
 *                CIP_PRIOR_ITV2D and CIP_PRIOR_ITV3D likewise.
 *   d_workspace: device buffer of at least cip_plan_workspace_bytes bytes,
 *                256-byte aligned, owned by the caller, kept by the plan until
 *                cip_plan_destroy and not touched by the caller meanwhile.
 * Blocks until the precompute on `stream` has finished. */
int cip_plan_create(int K, int S, int N1, int N2, const float* d_psf,
                    const cip_prior_desc* prior, double rho, double lambda,
                    void* d_workspace, size_t ws_bytes, void* stream, cip_plan_t* out);

/* y = H x (Eq. forward model without noise): d_x [S][N1][N2] -> d_y [K][N1][N2].
 * FP32 FFTs; d_x and d_y must not overlap. */
int cip_forward(cip_plan_t plan, const float* d_x, float* d_y, void* stream);

/* x = H^T y, the transpose of the block matrix H of Eq. forwardModel (its
 * (k, s) block is the circular convolution by h_{k,s}): x_s is the sum over k
 * of y_k circularly correlated with h_{k,s}; in the frequency domain
 * x_hat_s = sum_k conj(Lambda_{k,s}) y_hat_k (Section IV-A). d_y [K][N1][N2]
 * -> d_x [S][N1][N2]. FP32 FFTs; d_x and d_y must not overlap. */
int cip_adjoint(cip_plan_t plan, const float* d_y, float* d_x, void* stream);

/* Run `iters` >= 1 ADMM iterations from t = u = 0 (and z = 0) on the
 * measurements d_y [K][N1][N2] and write x^iters to d_x [S][N1][N2].
 * Analysis priors (Algorithm 1): x-update in the frequency domain
 * (Eq. solx_Trans_DFT), soft thresholding (Eq. solt_trans), dual update
 * (Eq. subu_trans). Synthesis priors (Algorithm 2): x-update of
 * Eq. solx_synt_DFT, sparse-code update (Eq. solz_patch2 for patches,
 * Eqs. solz_DFT / solz_DFT_SM for the convolutional dictionary), soft
 * thresholding (Eq. softADMM) and dual update (Eq. subu_dic). d_x is also used as working storage during the
 * call. A plan runs one solve at a time (its state lives in the workspace). */
int cip_solve(cip_plan_t plan, const float* d_y, int iters, float* d_x, void* stream);

/* Online dictionary learning (plans created with CIP_PLAN_DICT_UPDATE, the
 * dictionary update of Section IV-B). Every cip_solve then starts from the
 * plan's dictionary and, after the code update of each outer iteration
 * l < iters, takes one step of the dictionary ADMM; the next x- and code
 * updates use the new dictionary g.
 *   Convolutional priors (Eqs. d_admm, sold_3D, g_admm, h_admm): d full
 *   size (3D: Sherman-Morrison at every 3D frequency; 2D: the rank-S system
 *   of the common filters per 2D frequency, by the Woodbury identity),
 *   g = d + e cropped to the filter support and scaled to unit norm per
 *   filter, e <- e + d - g (e is the scaled dual of the split d = g that the
 *   d- and g-updates' penalty sigma/2 ||d - g + e||^2 defines; the sign printed
 *   with Eq. h_admm, g - d, would double e every step).
 *   Patch prior (Eqs. ADMM0, sold_patch, ADMM1, subh): with the patch matrix
 *   X = [P_1 x | ... | P_J x] and the codes Z of the iteration,
 *   D = (X Z^T + sigma (G - E)) (Z Z^T + sigma I)^-1, G = (D + E) / ||D + E||_F
 *   (the constraint ||D||_F = 1 of Eq. patch_based_dic), E <- E + D - G (the
 *   scaled dual of D = G, signed as for the convolutional priors);
 *   D is formed in FP64 on the GPU (X Z^T and Z Z^T on FP64 MFMA from the
 *   FP32 image and the FP32 codes, the FP64 Cholesky factor of
 *   Z Z^T + sigma I and FP64 triangular solves); the code update's tables
 *   (G and M1 = G^T (rho I + G G^T)^-1) are rebuilt from G in FP32 and
 *   stored in BF16.
 * This call copies g of the last solve (the layout of the plan's dictionary:
 * [n][A], [M][L][L] or [M][S][L][L] float32) to the device buffer d_filters,
 * asynchronously on `stream`. CIP_EINVAL if the plan does not learn its
 * dictionary or has not solved yet. */
int cip_plan_dictionary(cip_plan_t plan, float* d_filters, void* stream);

/* Release the host-side plan object (the workspace stays the caller's). */
int cip_plan_destroy(cip_plan_t plan);

/* ---- adaptive penalty and stopping rule (Section IV-C, Eq. paramS) --------
 * Algorithm 1 (analysis priors) from t = u = 0 where every `every`-th
 * iteration l < max_iters, after the t- and u-updates, measures
 *   r = ||T x^l - t^l||,  s = rho ||t^l - t^(l-1)||,
 *   c = ||x^l - x^(l-1)|| / ||x^(l-1)||   (from the second iteration on);
 * stops with x^l when c < tol; otherwise sets rho <- tau rho if r > mu s,
 * rho <- rho / tau if s > mu r, rescales the scaled dual u by the inverse
 * factor and recomputes the FP64 per-frequency inverses for the new rho
 * before the next x-update. For the isotropic TV priors T = I, t^l is the
 * TV proximal map at weight lambda / rho, and Chambolle's dual is kept as
 * the warm start across a change; for the wavelet (x) DCT prior the
 * residuals are summed in the coefficient domain (T orthonormal).
 * Algorithm 2 (CIP_PRIOR_PATCH, CIP_PRIOR_CONV2D, CIP_PRIOR_CONV3D with a
 * fixed dictionary) from z = t = u = 0, the split z = t: the same rule with
 *   r = ||z^l - t^l||,  s = rho ||t^l - t^(l-1)||,
 * and on a change u rescaled as above and the code update rebuilt for the new
 * rho (its threshold lambda / rho; M1 = D^T (rho I + D D^T)^-1 in FP64 on the
 * host for the patch prior; the per-frequency Sherman-Morrison tables in FP64
 * from the resident filter spectra for the conv priors; the x-update does not
 * depend on rho).
 * With online dictionary learning (CIP_PLAN_DICT_UPDATE) the code update is
 * rebuilt from the current dictionary G (on the GPU, FP32), and with
 * adapt_sigma the rule also sets the dictionary penalty after the D, G, E
 * step of every checked iteration:
 *   r_d = ||D - G||,  s_d = sigma ||G - G_prev||,
 *   sigma <- tau sigma if r_d > mu s_d, sigma / tau if s_d > mu r_d, and the
 *   scaled dual E is rescaled by sigma_old / sigma_new.
 * CIP_EUNSUPPORTED for adapt_sigma on a plan that does not learn its
 * dictionary.
 * The plan must have been created with CIP_PLAN_ADAPTIVE and must not be an
 * attached plan; its tables are back at its own rho when the call returns.
 * Synchronous: waits on `stream` at every check and returns when x is in
 * d_x. The norms are accumulated in FP32 per work-group (per wave for the
 * synthesis priors) and summed in FP64. */
typedef struct {
  int max_iters;   /* iteration cap (>= 1)                                     */
  int every;       /* check and adapt every this many iterations (>= 1)       */
  double tau;      /* penalty factor (> 1; the paper uses 2)                  */
  double mu;       /* residual balance (> 1; the paper uses 10)               */
  double tol;      /* stopping tolerance on c (>= 0; the paper uses 1e-4)     */
  int adapt_sigma; /* also adapt the dictionary penalty sigma (learning plans) */
} cip_adaptive_params;
typedef struct {
  int iters;        /* iterations run                                         */
  int rho_changes;  /* number of penalty changes                              */
  double rho;       /* penalty of the last iteration                          */
  double rel_change;/* last measured c (-1 if none)                           */
  double r_norm;    /* last measured r                                         */
  double s_norm;    /* last measured s                                         */
  double sigma;     /* dictionary penalty of the last step (learning plans)  */
  int sigma_changes;/* number of sigma changes                                */
} cip_solve_info;
int cip_solve_adaptive(cip_plan_t plan, const float* d_y, const cip_adaptive_params* params,
                       float* d_x, void* stream, cip_solve_info* info);

/* ---- shared tables, separate solve state ---------------------------------
 * A plan's workspace holds read-only tables (Alg. 1/2 step 2: spectra,
 * per-frequency inverses, dictionaries) followed by the state of one solve.
 * cip_plan_attach creates a plan that shares `base`'s tables and keeps its
 * solve state in `d_state` (device, 256-byte aligned, at least
 * cip_plan_state_bytes bytes, owned by the caller): several solves of the
 * same operator then run concurrently, one per attached plan, each on its own
 * stream. No GPU work; `base` must outlive the attached plans, which are
 * released with cip_plan_destroy. */
int cip_plan_state_bytes(cip_plan_t plan, size_t* bytes);
int cip_plan_attach(cip_plan_t base, void* d_state, size_t bytes, cip_plan_t* out);

/* ---- batches of independent solves --------------------------------------
 * A batch runs n independent cip_solve calls (distinct plans, each with its
 * own measurements, iteration count and output) concurrently: the problems
 * are spread largest-first over n_streams internal HIP streams, forked from
 * and joined back to the stream passed to cip_batch_launch. With use_graph,
 * cip_batch_create captures the whole batch once into a hipGraph (the solves
 * launch no memsets or allocations) and every cip_batch_launch replays it
 * with a single graph launch; otherwise the kernels are launched directly.
 * The pointers passed to cip_batch_create must stay valid until
 * cip_batch_destroy; every launch recomputes all solves from t = u = 0.
 * Each result equals that of a lone cip_solve on the same plan (the solves
 * share no memory). Creating a batch allocates host objects, streams and
 * events, never device memory. Plans that learn their dictionary
 * (CIP_PLAN_DICT_UPDATE) run in direct batches only: with use_graph the call
 * returns CIP_EUNSUPPORTED before any capture. */
typedef struct cip_batch_s* cip_batch_t;
/* One-shot form: the n solves (distinct plans; d_y[i] [K][N1][N2] ->
 * d_x[i] [S][N1][N2] after iters[i] iterations) launched directly over the
 * library's internal streams (four per device, created at the first call and
 * kept until the process ends), forked from and joined back to `stream`;
 * asynchronous on `stream`, like cip_solve. Each result equals that of a
 * lone cip_solve on the same plan. Calls from several host threads are
 * enqueued one after the other. */
int cip_batch_solve(int n, const cip_plan_t* plans, const float* const* d_y, const int* iters,
                    float* const* d_x, void* stream);
int cip_batch_create(int n, const cip_plan_t* plans, const float* const* d_y, const int* iters,
                     float* const* d_x, int n_streams, int use_graph, cip_batch_t* out);
int cip_batch_launch(cip_batch_t batch, void* stream);
int cip_batch_destroy(cip_batch_t batch);

/* ---- request server (continuous batching on one GPU) ---------------------
 * The server owns one device arena of hbm_budget_bytes (allocated by
 * cip_server_create, freed by cip_server_destroy; nothing else is allocated
 * on the device afterwards). Operators (plans of fixed K, S, N1, N2, kernels,
 * prior, rho, lambda) are registered once and keep their tables resident.
 * Requests name an operator and carry HOST buffers: y [K][N1][N2] (read
 * after admission) and x [S][N1][N2] (written before completion); both must
 * stay valid until the request has finished. n_slots worker threads, each
 * with its own HIP stream, admit queued requests oldest-first by HBM
 * footprint (solve state + y + x must fit in the free part of the arena; a
 * request can be overtaken by smaller ones at most 16 times), run cip_solve
 * on a state attached to the operator's tables, and release the memory:
 * requests arriving while others run are admitted as slots and memory free
 * up, and their GPU work overlaps. Each result equals that of a lone
 * cip_solve with the same operator and iteration count.
 * Latency = completion - submission (host steady clock, seconds). */
typedef struct cip_server_s* cip_server_t;
typedef struct {
  size_t hbm_budget_bytes;   /* device memory for operators and requests    */
  int n_slots;               /* concurrent solves, 1 .. 16                  */
  int autotune;              /* nonzero: tune each operator's row pass when
                                it is registered (cip_plan_autotune)        */
} cip_server_config;
typedef struct {
  int op;                    /* operator id from cip_server_add_operator    */
  const float* y;            /* host [K][N1][N2]                            */
  float* x;                  /* host [S][N1][N2]                            */
  int iters;                 /* ADMM iterations (>= 1)                      */
} cip_request;
int cip_server_create(const cip_server_config* cfg, cip_server_t* out);
/* d_psf: device [K][S][N1][N2], read during the call on the server's own
 * registration stream: the kernels (and the dictionary or filters of the
 * prior) must already be written when the call is made (synchronise the
 * stream that wrote them first). The plan is built and, with autotune,
 * tuned on that stream while queued requests keep running. CIP_ENOSPC when
 * the operator's workspace does not fit in the free part of the arena. */
int cip_server_add_operator(cip_server_t server, int K, int S, int N1, int N2, const float* d_psf,
                            const cip_prior_desc* prior, double rho, double lambda, int* op_id);
/* Queue a request; CIP_ENOSPC when it could never fit in the budget. */
int cip_server_submit(cip_server_t server, const cip_request* req, uint64_t* ticket);
/* *done = 1 once the request has finished (then *latency_s is set; a failed
 * request returns its error code), else 0. */
int cip_server_poll(cip_server_t server, uint64_t ticket, int* done, double* latency_s);
/* Block until the request has finished; returns its status. queue_s = time
 * from submission to admission. Either output may be NULL. */
int cip_server_wait(cip_server_t server, uint64_t ticket, double* latency_s, double* queue_s);
/* Finish every queued request, stop the workers, release the arena. */
int cip_server_destroy(cip_server_t server);

/* ---- autotuning -------------------------------------------------------
 * Times the available shapes of the analysis row pass on this plan's own
 * data and keeps the fastest for all later solves of the plan: the number of
 * row pairs per work-group (4 or 2) and the points per thread of
 * the row transforms (the default radix sequence, or 8 points per thread,
 * i.e. radices 8, 8, ..., for power-of-two N2), `reps` launches each with HIP
 * events on `stream`. The plan must have run cip_solve once; the solve state
 * is left undefined (the next solve starts from scratch anyway). Analysis
 * priors only (CIP_EUNSUPPORTED otherwise). Blocks until done. */
typedef struct {
  int row_np;         /* row pairs per work-group chosen                       */
  int row_ppt;        /* points per thread chosen                              */
  int candidates;     /* shapes timed                                          */
  double row_us;      /* average time of the chosen shape                      */
  double default_us;  /* average time of the default shape                     */
} cip_tuning;
int cip_plan_autotune(cip_plan_t plan, int reps, void* stream, cip_tuning* out);
/* Set the row-pass shape directly (values as chosen by cip_plan_autotune:
 * row_np 4 or 2; row_ppt the default or 8). */
int cip_plan_set_tuning(cip_plan_t plan, int row_np, int row_ppt);

/* ---- reconstruction without device allocation ----------------------------
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the result of
 * cip_plan_create + cip_solve + cip_plan_destroy, with the plan's workspace
 * (tables and solve state) in a static buffer of CIP_STATIC_WORKSPACE_BYTES
 * that the library holds on every GPU it runs on until the process ends,
 * instead of caller memory. Arguments as for cip_plan_create (d_psf) and
 * cip_solve (d_y, iters, d_x); nothing is allocated on the device and the
 * caller passes only inputs and outputs. Limit: problems whose
 * cip_plan_workspace_bytes exceeds CIP_STATIC_WORKSPACE_BYTES (64 MiB: for
 * example the analysis priors up to 512 x 512 with K = S = 3) return
 * CIP_ENOSPC before any GPU work. Every call on a GPU reuses that GPU's
 * buffer, which keeps the last call's contents; each call rebuilds all it
 * reads, so no part of it has to start at zero. Two calls overlapping on one
 * GPU would race on the buffer: the library serialises the calls of a
 * process, and each returns only after its work on `stream` has finished
 * (so, unlike cip_solve, this call is synchronous). Errors as for
 * cip_plan_create and cip_solve. */
#define CIP_STATIC_WORKSPACE_BYTES (64u << 20)
int cip_solve_static(int K, int S, int N1, int N2, const float* d_psf,
                     const cip_prior_desc* prior, double rho, double lambda, const float* d_y,
                     int iters, float* d_x, void* stream);

/* Message of the last failed call on this thread ("" if none). */
const char* cip_last_error(void);

/* ---- instrumentation ------------------------------------------------------
 * Average device time, in microseconds, of `reps` back-to-back launches of
 * one kernel of the solver on `stream`, measured with HIP events recorded on
 * that stream. The plan must have run cip_solve at least once (the kernels
 * then operate on its current state). which: 0 = fused row pass of one ADMM
 * iteration, 1 = fused column pass (FFTs + per-frequency solve), 2 = patch
 * sparse-code update (patch prior) or frequency pass (convolutional prior).
 * For the convolutional prior 0 is its row pass over the M*S code planes and
 * 1 the batched forward column FFT of those planes. Blocks until the timed launches
 * finish. */
int cip_time_kernel(cip_plan_t plan, int which, int reps, void* stream, double* avg_us);

#ifdef __cplusplus
}
#endif

#endif /* CIP_H_ */
