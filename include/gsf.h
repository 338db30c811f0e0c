/*
 * gsf.h -- C ABI of libgsf: graph spectral polynomial filters on MI355X (gfx950).
 *
 * Method: Knyazev & Malyshev, "Accelerated graph-based spectral polynomial
 * filters" (IEEE MLSP 2015).  A noisy signal x (1D samples or a 2D image,
 * row-major) defines, through a fixed guidance signal g, a weighted graph:
 * bilateral-filter weights (Section 2, eq. (2)) or the guided filter's
 * implicit matrix (Section 3, Algorithm 1, eqs. (5)-(6)).  With adjacency W,
 * degrees D and Laplacian L = D - W (eq. (4)) the library applies
 *     N      = D^-1/2 W D^-1/2          (normalized operator, Section 4)
 *     L_sym  = I - N = D^-1/2 L D^-1/2  (normalized Laplacian)
 *     RW     = D^-1 W                   (one BF / GF pass, eq. (3))
 * and runs the paper's polynomial filters on it: power iteration (Section 4),
 * preconditioned CG for L x = 0 with preconditioner D (Algorithm 2) and block
 * LOBPCG used as a low-pass filter (Algorithm 3, Section 6).
 *
 * Conventions shared by every entry point
 *  - Device memory: every data pointer (guidance, x, y, workspaces) is a
 *    device pointer on the current HIP device.  The caller owns all of it;
 *    the library never allocates device memory.  Workspace sizes come from
 *    the *_workspace_bytes queries; a workspace must stay alive and untouched
 *    while a handle or call uses it.
 *  - Element type: FP32 (`float`) or FP64 (`double`) as selected by
 *    gsf_operator_desc.prec; every vector argument of a call on an operator
 *    has that type.  Small reductions, scalars and the Rayleigh-Ritz step are
 *    always computed in FP64.
 *  - Vector layout: a block of m vectors over n grid points is stored
 *    point-major: element (i, j) at index i*m + j (m contiguous values per
 *    grid point).  m = 1 is a plain vector.
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream).  All work
 *    is enqueued asynchronously on it; a call only synchronizes the stream
 *    when it is given a non-NULL host `info` pointer to fill.
 *  - Errors: status codes only.  Arguments are validated on the host before
 *    anything is launched; on GSF_EINVAL / GSF_ENOMEM nothing has been
 *    enqueued and no output was touched.  Input vectors are never modified.
 *  - Threading: a handle may be used by one stream at a time.
 */
#ifndef GSF_H
#define GSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GSF_OK = 0,
  GSF_EINVAL = 1,      /* invalid argument (shape, parameter, NULL pointer, non-finite parameter) */
  GSF_ENOMEM = 2,      /* workspace smaller than the size query returned */
  GSF_EDEVICE = 3,     /* a HIP runtime call failed */
  GSF_ENOTCONV = 4,    /* tol > 0 was not reached within kmax steps; the result is still valid */
  GSF_EBREAKDOWN = 5,  /* the iteration stopped early (see each solver); the result is still valid */
  GSF_ESCRATCH = 6     /* gsf_cg_filter_noalloc: the problem needs more than its static scratch */
} gsf_status;

typedef enum { GSF_BF = 0, GSF_GF = 1 } gsf_kind;
typedef enum { GSF_F32 = 0, GSF_F64 = 1 } gsf_prec;
typedef enum { GSF_FORM_N = 0, GSF_FORM_LSYM = 1, GSF_FORM_RW = 2, GSF_FORM_L = 3 } gsf_form;
typedef enum { GSF_METHOD_POWER = 0, GSF_METHOD_CG = 1, GSF_METHOD_LOBPCG = 2 } gsf_method;
typedef enum { GSF_STENCIL_SQUARE = 0, GSF_STENCIL_CROSS = 1 } gsf_stencil;
typedef enum { GSF_NORM_D = 0, GSF_NORM_DIAGL = 1 } gsf_norm;

/* Operator description.
 *  kind    GSF_BF: weights of eq. (2) over the neighbourhood chosen by
 *            `stencil` (default: the square window |o|_inf <= radius),
 *            w_ij = exp(-||p_i - p_j||^2 / (2 sigma_d^2) - (g_i - g_j)^2 / (2 sigma_r^2)),
 *            self-loop w_ii = 1 included, windows truncated at the border.
 *          GSF_GF: Algorithm 1 with mean filters of width 2*radius+1 over
 *            border-truncated windows and regularisation gf_eps; its matrix
 *            W_ij = (1/|w|) sum_{k: i,j in w_k} (1/N_k)(1 + (g_i-mu_k)(g_j-mu_k)/(s_k^2+eps))
 *            (eq. (6) in the interior) has row sums d_i = N_i/|w|.
 *  ndim    1 (dims[0] = n) or 2 (dims[0] = rows H, dims[1] = columns W);
 *          a BF operator has fewer than 2^30 points and
 *          (n + radius*(W+1)) * element size <= 2^32 bytes (2D; 1D:
 *          (n + radius) * element size), so FP64 allows about 2^29 points;
 *          a GF operator has fewer than 2^27 points.
 *  prec    element type of the guidance, of all vectors and of the stored
 *          operator.  GF window statistics, and BF weights of FP64 data or of
 *          guidance with other than 1 or 3 channels, are computed in FP64 and
 *          rounded once to this type; BF weights of FP32 data with one or
 *          three guidance channels are evaluated in FP32 (hardware base-2
 *          exponential: relative error about (2 + 2a) 2^-24 for a weight e^-a
 *          with one channel, (4 + 3a) 2^-24 with three).  BF degrees are
 *          always the FP64 row sums of exactly the stored weights.
 *  radius  1..8.
 *  sigma_d, sigma_r > 0 (BF; +inf allowed, removing that factor).
 *  gf_eps  >= 0 (GF).
 *  stencil BF only (GF: must be GSF_STENCIL_SQUARE, else GSF_EINVAL).
 *          GSF_STENCIL_SQUARE: the square window above.  GSF_STENCIL_CROSS:
 *          the offsets along one axis, |o_k| <= radius (radius 1 in 2D is
 *          the 5-point stencil of the image experiment of Section 7); in 1D
 *          both are the same interval.
 *  norm    BF only (GF: must be GSF_NORM_D, else GSF_EINVAL).
 *          GSF_NORM_D: the normalizing diagonal is D (self-loop included),
 *          so RW = D^-1 W is eq. (3) and D the preconditioner of Algorithm 2.
 *          GSF_NORM_DIAGL: the normalizing diagonal is diag L (Section 4),
 *          diag L_i = sum_{j != i} w_ij (the self-loop cancels in L = D - W),
 *          summed in FP64 from the stored off-diagonal weights; it replaces
 *          D in N, L_sym, RW = I - (diag L)^-1 L, the preconditioner and the
 *          z-space map z = (diag L)^1/2 x.  A vertex whose stored
 *          off-diagonal weights are all zero has a zero row and column in L;
 *          its normalizing value is taken as 1 (the vertex is then a fixed
 *          point of every filter).  The L form stays L = D - W.
 *  channels BF only (GF: 0 or 1, else GSF_EINVAL): values per guidance point,
 *          0..8 (0 means 1).  With C > 1 channels the guidance is point-major
 *          (g[i*C + c]) and |g_i - g_j| in eq. (2) is the Euclidean distance
 *          of the channel vectors: the colour guidance of Section 2, whose
 *          photometric distance is measured in CIE-Lab (gsf_srgb_to_lab).
 *          sigma_r is then in the guidance's units (CIE-Lab: Delta E).
 *  A zero-initialised stencil / norm / channels selects the defaults. */
typedef struct {
  int32_t kind;
  int32_t ndim;
  int64_t dims[2];
  int32_t prec;
  int32_t radius;
  double sigma_d;
  double sigma_r;
  double gf_eps;
  int32_t stencil;   /* gsf_stencil */
  int32_t norm;      /* gsf_norm */
  int32_t channels;  /* guidance channels (BF), 0 or 1 = scalar */
  int32_t reserved;  /* must be 0 */
} gsf_operator_desc;

typedef struct gsf_operator gsf_operator;   /* opaque host handle */

/* Device layout of a built operator, for inspection (all pointers point into
 * the caller's operator workspace; element type = prec).
 *  BF: `planes` holds nplanes = ((2r+1)^ndim - 1)/2 planes of n values
 *      (2D cross stencil: 2r); plane o (half-window offsets in the order:
 *      1D o = 1..r; 2D (dy, dx) with dy = 0, dx = 1..r, then dy = 1..r,
 *      dx = -r..r; 2D cross (0, 1..r) then (1..r, 0)) stores the weight
 *      w_{i,i+o} of eq. (2) at index i (0 where i+o is outside the grid);
 *      each undirected edge is stored once.  Plane q starts at
 *      planes + q * plane_stride and is preceded by r*W + r (2D) or r (1D)
 *      zeros.  `inv_sqrt_d` holds 1/sqrt(d_i).
 *      The apply evaluates L_sym z = D^-1/2 L D^-1/2 z as
 *      (1/sqrt(d_i)) sum_j w_ij (u_i - u_j) with u = D^-1/2 z, and
 *      N z = z - L_sym z.
 *  GF: `mu` and `inv` hold the window statistics mu_k and 1/(sigma_k^2 + eps)
 *      of the guidance (Algorithm 1), `guidance` a copy of g; `planes` is
 *      NULL (the workspace also holds 16 scratch planes of the apply, which
 *      is why two GF applies on one operator must not run concurrently).
 *  Both: `inv_sqrt_d` holds 1/sqrt(d_i), `sqrt_d` sqrt(d_i); `degree` holds
 *  d_i in FP64, where d is the normalizing diagonal (D, or diag L with the
 *  isolated-vertex value 1 for GSF_NORM_DIAGL). */
typedef struct {
  int32_t kind, ndim, prec, radius;
  int64_t n;
  int32_t nplanes;
  const void* planes;
  const void* inv_sqrt_d;
  const void* sqrt_d;
  const double* degree;
  const void* guidance;
  const void* mu;
  const void* inv;
  int64_t plane_stride;  /* BF: elements between the starts of consecutive planes */
} gsf_operator_layout;

/* CG result summary (z-space 2-norms, FP64). */
typedef struct {
  int32_t iters;      /* completed updates */
  int32_t status;     /* gsf_status of the run */
  double res0;        /* ||r_0|| = sqrt(s_0^T r_0) */
  double res;         /* ||r|| at exit */
} gsf_cg_info;

/* LOBPCG result summary. */
typedef struct {
  int32_t iters;      /* completed Rayleigh-Ritz steps */
  int32_t status;     /* gsf_status of the run */
  int32_t dropped;    /* trial columns dropped by the Rayleigh-Ritz Cholesky, summed over steps */
  int32_t m;
  double res[8];      /* ||L_sym x_j - theta_j x_j||, unit x_j (z-space), per column */
  double theta[8];    /* Ritz values, ascending */
  int32_t fallbacks;  /* learned T: column-steps that fell back to T = I */
  int32_t pad;
} gsf_lobpcg_info;

/* ---- version / errors ------------------------------------------------- */
int gsf_version(void);
const char* gsf_status_string(int status);
/* gsf_last_device_error: the HIP error code (hipError_t) behind the calling
 * thread's latest GSF_EDEVICE, 0 if there was none since the last query;
 * the query resets it.  Kernel launches are checked with hipGetLastError;
 * every call that takes a stream first drops an error that earlier HIP calls
 * of other code left in the thread, so it reports only its own failures.
 * gsf_device_error_string: HIP's text for such a code. */
int gsf_last_device_error(void);
const char* gsf_device_error_string(int code);

/* ---- operator (Sections 2-3) ----------------------------------------------
 * gsf_operator_workspace_bytes: bytes of device workspace the operator needs.
 * gsf_build_operator: computes the weights (BF, eq. (2)) and degrees, or the
 *   guided-filter window statistics (Algorithm 1, the g-only lines), from the
 *   guidance `guidance` (n values of type prec; BF with C > 1 channels:
 *   n*C values, point-major) into `ws`, and returns a host
 *   handle in *out.  The build is asynchronous: the guidance must stay valid
 *   until the stream has executed it (it is not read afterwards).
 *   GSF_EINVAL for bad shapes or parameters; a non-finite guidance value is
 *   not checked on the host (it yields non-finite weights).
 * gsf_destroy_operator: frees the host handle only (NULL is allowed). */
gsf_status gsf_operator_workspace_bytes(const gsf_operator_desc* desc, size_t* bytes);
gsf_status gsf_build_operator(const gsf_operator_desc* desc, const void* guidance,
                              void* ws, size_t ws_bytes, void* stream, gsf_operator** out);
gsf_status gsf_operator_get_layout(const gsf_operator* op, gsf_operator_layout* out);
void gsf_destroy_operator(gsf_operator* op);

/* ---- apply (eqs. (1), (3), (4); Section 4) --------------------------------
 * y = F x for a block of m (1..8) vectors, F = N, L_sym, D^-1 W or the
 * Laplacian L = D - W (`form`).  N and L_sym act on z-space vectors
 * (z = D^1/2 x); RW and L act on x directly.  Column j of grid point i is
 * x[i*ldx + j] and y[i*ldy + j]: ldx, ldy >= m are the elements between
 * consecutive points (0 means m, the dense point-major block), so that m
 * columns of a wider point-major array can be applied in place; x must hold
 * (n-1)*ldx + m elements, y (n-1)*ldy + m.  The extents of x and y must not
 * overlap.  GSF_EINVAL for another form, m outside 1..8, ldx or ldy below m
 * (other than 0), or overlapping extents. */
gsf_status gsf_apply(const gsf_operator* op, int form, int m, const void* x, int64_t ldx, void* y,
                     int64_t ldy, void* stream);
/* Joint apply: y = F x for an n x m block and y2 = F x2 for one more vector,
 * in one pass over the operator where it offers that (BF on the square
 * window or 1D, m = 1 or 4), else as two applies.  No output may overlap an
 * input or the other output (GSF_EINVAL). */
gsf_status gsf_apply_joint(const gsf_operator* op, int form, int m, const void* x, void* y, const void* x2,
                           void* y2, void* stream);

/* ---- solvers ---------------------------------------------------------------
 * gsf_solver_workspace_bytes: workspace for `method` with block size m: the
 *   LOBPCG block, or the number of columns of the block power / CG filters
 *   (m = 1 covers the single-vector power and CG filters). */
gsf_status gsf_solver_workspace_bytes(const gsf_operator* op, int method, int m, size_t* bytes);

/* Power iteration (Section 4): x_out = (D^-1 W)^kmax x0, kmax >= 0.
 * x0 and x_out: n elements; they may be the same buffer. */
gsf_status gsf_power_filter(const gsf_operator* op, const void* x0, void* x_out, int kmax,
                            void* ws, size_t ws_bytes, void* stream);

/* Preconditioned CG for L x = 0 with preconditioner D, started at x0
 * (Algorithm 2), run in z = D^1/2 x as CG on L_sym with identity
 * preconditioner.  beta = s^T (r - r_old) / (s_old^T r_old) (the printed
 * s_old^T s_old denominator read as s_old^T r_old).  Runs kmax updates unless
 *   - tol > 0 and ||r_k|| <= tol ||r_0||: stop, GSF_OK;
 *   - s^T r <= (tau ||z_0||)^2 (tau = 1e-13 FP64, 1e-6 FP32) or non-finite,
 *     or p^T q <= 0 or non-finite: stop, GSF_EBREAKDOWN (x so far is returned;
 *     a constant x0 returns x0);
 * and returns GSF_ENOTCONV when tol > 0 was not met after kmax updates.
 * With tol > 0 and info != NULL the host stops issuing steps once the device
 * state reports the stop (read every 16 steps, 16 steps behind the queue).
 * The returned status is only known after the stream has reached the end of
 * the call: with info == NULL the call returns GSF_OK after enqueueing. */
gsf_status gsf_cg_filter(const gsf_operator* op, const void* x0, void* x_out, int kmax,
                         double tol, void* ws, size_t ws_bytes, gsf_cg_info* info, void* stream);

/* gsf_cg_filter without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  It computes what gsf_cg_filter computes
 * (same kernels in the same order; bitwise the same result and info) in a
 * workspace of the library's own: one static device array of
 * GSF_NOALLOC_SCRATCH_BYTES (64 MiB) per device, part of the library's code
 * object, which each device holds from the first call until the process ends.
 * The call allocates nothing (no hipMalloc / hipFree, no pinned host
 * staging): the host does not poll for an early stop, so with tol > 0 all
 * kmax steps are enqueued and those after the stop do no work on the device;
 * a non-NULL info synchronizes the stream and reads the device state into it.
 * Every call on one device uses the same array and overwrites what the
 * previous call left there (the solver state is re-initialised by each call):
 * calls that overlap on one device (other streams, other threads) race, and
 * so does a graph replay that overlaps another call.
 * GSF_ESCRATCH, with nothing enqueued and x_out untouched, when the CG
 * workspace of the operator (gsf_solver_workspace_bytes(op, GSF_METHOD_CG, 1))
 * exceeds GSF_NOALLOC_SCRATCH_BYTES: four vectors of n elements plus
 * reduction partials, so up to about 4.1 M FP32 or 2 M FP64 points.  Other
 * arguments and errors as gsf_cg_filter. */
#define GSF_NOALLOC_SCRATCH_BYTES (64u << 20)
gsf_status gsf_cg_filter_noalloc(const gsf_operator* op, const void* x0, void* x_out, int kmax,
                                 double tol, gsf_cg_info* info, void* stream);

/* Multi-channel signals (the channels of a colour image filtered on one graph):
 * x0 and x_out are n x m point-major blocks (m = 1..8; x0[i*m + c]), one
 * m-column apply per step reads the operator once for all channels.
 *  gsf_power_filter_block: every column as gsf_power_filter; x0 and x_out
 *    may be the same buffer.
 *  gsf_cg_filter_block: every column an independent run of gsf_cg_filter
 *    (its own alpha, beta and stopping decisions; a stopped column keeps its
 *    result while the others continue).  info: NULL or an array of m
 *    summaries; the return value is the first non-OK column status, else
 *    GSF_OK (known only after the stream has reached the end of the call, as
 *    for gsf_cg_filter).
 * Workspace: gsf_solver_workspace_bytes(op, method, m, ...).  GSF_EINVAL for
 * m outside 1..8. */
gsf_status gsf_power_filter_block(const gsf_operator* op, int m, const void* x0, void* x_out, int kmax,
                                  void* ws, size_t ws_bytes, void* stream);
gsf_status gsf_cg_filter_block(const gsf_operator* op, int m, const void* x0, void* x_out, int kmax,
                               double tol, void* ws, size_t ws_bytes, gsf_cg_info* info, void* stream);

/* Colour guidance (Section 2: the photometric distance in CIE-Lab).
 * lab = CIE 1976 L*a*b* of sRGB values rgb (n points x 3 components,
 * point-major, nominally in [0, 1]; no clipping): the IEC 61966-2-1 transfer
 * curve, the linear RGB -> XYZ matrix of the sRGB primaries and the D65 white
 * (chromaticities (0.64, 0.33), (0.30, 0.60), (0.15, 0.06), (0.3127, 0.3290)),
 * and L* = 116 f(Y/Yn) - 16, a* = 500 (f(X/Xn) - f(Y/Yn)),
 * b* = 200 (f(Y/Yn) - f(Z/Zn)) relative to that white; FP64 arithmetic,
 * element type prec.  rgb and lab may be the same buffer.  GSF_EINVAL for
 * n < 0, a bad prec or NULL pointers with n > 0. */
gsf_status gsf_srgb_to_lab(int prec, int64_t n, const void* rgb, void* lab, void* stream);

/* Block LOBPCG low-pass filter (Algorithm 3 generalised to m = 1..8 vectors):
 * operator L_sym, preconditioner T = I (T = D^-1 in x-space).  Start block
 * X0[:, j] = z0 * phi_j with phi_0 = 1 and phi_j products of Legendre
 * polynomials of the normalised coordinates t = 2(i + 1/2)/n - 1 (degrees by
 * total degree, then row degree).  With constraint != 0 every block is kept
 * orthogonal to Y = D^1/2 e / ||D^1/2 e|| (x orthogonal to e in the D inner
 * product).  Each step: R = AX - X Theta, W = R (projected), Rayleigh-Ritz on
 * [X, W, P] in FP64 (the Gram pair summed in FP64 from exact products for
 * either element type) with a column-dropping Cholesky (drop when the pivot of the
 * unit-diagonal Gram is <= 1e-10 (FP64) / 1e-6 (FP32), or the column norm^2 is
 * <= tau^2 max norm^2), keep the m smallest Ritz pairs, P = [W, P] C.
 * Output x_out = D^-1/2 (X X^T z0 (+ Y Y^T z0)), n elements.
 * ritz_vecs (NULL or n*m, z-space, column signs with x_j^T z0 >= 0).
 * ritz_vals_host (NULL or m host doubles): the Ritz values theta_j ascending;
 * non-NULL synchronizes the stream, as a non-NULL info does.
 * tol > 0 stops when every column residual <= tol (GSF_ENOTCONV if not met);
 * until then a column already at tol is soft-locked: its W column counts as
 * zero (dropped by the Rayleigh-Ritz step, counted in info->dropped);
 * with info != NULL the host then also stops issuing steps (it reads the
 * device convergence flag every 16 steps, 16 steps behind the queue).
 * A start block of rank < m returns x0 with GSF_EBREAKDOWN.
 * T: NULL (plain method), a learned preconditioner (gsf_precond_create) or
 *   a shifted solve (gsf_precond_create_shifted) built for this operator's
 *   grid and precision; then W = T(R) column by column (flexible LOBPCG: the
 *   Rayleigh-Ritz step on [X, W, P] is unchanged), with T = I for a column
 *   whose T(r) has a non-finite entry or r^T T(r) <= 0 (counted in
 *   info->fallbacks). */
typedef struct gsf_precond gsf_precond;
gsf_status gsf_lobpcg_filter(const gsf_operator* op, const void* x0, void* x_out, int m,
                             int kmax, double tol, int constraint, const gsf_precond* T,
                             void* ritz_vecs, double* ritz_vals_host, void* ws, size_t ws_bytes,
                             gsf_lobpcg_info* info, void* stream);

/* Joint CG + LOBPCG filters of one operator (Algorithms 2 and 3 side by side):
 * the results are those of gsf_cg_filter(x0_cg, kmax_cg, tol 0) and
 * gsf_lobpcg_filter(x0_lob, m, kmax_lob, tol 0, constraint, T = NULL) up to the
 * summation order of the CG dot products.  While both run, step k of each
 * shares one stencil pass, and so do their starts (r0 = -L_sym z0 with
 * A X0): the CG vector is applied as one more column of the LOBPCG block (BF operators on the square window or 1D with m = 1 or 4; other
 * operators apply the two blocks one after the other).  Everything runs on
 * `stream`: the CG update (alpha, x, r) runs as extra workgroups of the LOBPCG
 * Rayleigh-Ritz launch and the CG direction (beta, p) as extra workgroups of
 * the LOBPCG update launch.  x0_cg, x_cg: n elements;
 * x0_lob, x_lob: n elements.
 * Workspace: gsf_joint_workspace_bytes(op, m, ...).  cg_info, lob_info: NULL
 * or summaries as for the single filters.  GSF_EINVAL for NULL pointers,
 * kmax < 0 or m outside 1..8; GSF_ENOMEM for a short workspace; returns the
 * LOBPCG status if not OK, else the CG status. */
gsf_status gsf_joint_workspace_bytes(const gsf_operator* op, int m, size_t* bytes);
gsf_status gsf_joint_filter(gsf_operator* op, const void* x0_cg, void* x_cg, int kmax_cg, const void* x0_lob,
                            void* x_lob, int m, int kmax_lob, int constraint, void* ws, size_t ws_bytes,
                            gsf_cg_info* cg_info, gsf_lobpcg_info* lob_info, void* stream);

/* ---- learned preconditioner (the preconditioner T of Algorithm 3) ----------
 * Network: conv3x3 (2 -> 16 channels) + ReLU, conv3x3 (16 -> 16) + ReLU,
 * conv3x3 (16 -> 1); cross-correlation with zero padding, no biases.  Input
 * channels (r / s, g): the residual column scaled by s = RMS(r) = ||r|| /
 * sqrt(n) and the guidance image; T(r) = s * net.  Weights, input and the two
 * hidden activations are BF16 (round to nearest even), accumulation FP32.
 * Weight vector (GSF_NET_WEIGHTS values): W1[o][c][ky][kx] (16x2x3x3), then
 * W2[o][c][ky][kx] (16x16x3x3), then W3[c][ky][kx] (16x3x3).  BF16 weights are
 * passed as uint16 bit patterns.  All arrays are device memory owned by the
 * caller; every call is asynchronous on `stream`.
 *
 * Training set: sample s occupies inputs[(s*rows*cols + p)*2 + {0, 1}] =
 * (r/s, g) and targets[s*rows*cols + p] = t / s (FP32, row-major pixels p),
 * with t = (L_sym + alpha I)^-1 r (gsf_shifted_cg) and s = RMS(r)
 * (gsf_net_make_pair writes both).
 *  gsf_net_workspace_bytes: scratch of gsf_net_forward / gsf_net_loss_grad
 *    for a batch of `batch` samples.
 *  gsf_net_forward: y[b*rows*cols + p] = net(inputs of sample idx[b]).
 *  gsf_net_loss_grad: loss = mean over the batch's pixels of
 *    (net - target)^2 (one double in device memory) and its gradient with
 *    respect to the weights (GSF_NET_WEIGHTS floats, the BF16 weights taken
 *    as the variables); deterministic (fixed-order FP64 reductions).
 *  gsf_net_adam: one Adam step t >= 1 (bias-corrected, Kingma and Ba) on the
 *    FP32 master weights w with moments mom, vel; writes the BF16 copy w_bf16.
 *  gsf_net_to_bf16: w_bf16 = round(w).
 *  gsf_net_pair_workspace_bytes / gsf_net_make_pair: one training pair from a
 *    residual r (stride ldr), its target y (stride ldy) and the guidance g
 *    (op's element type, n values each) into inputs (2n floats) and targets
 *    (n floats).
 * Errors: GSF_EINVAL for null pointers, batch < 1, non-positive sizes,
 * t < 1; GSF_ENOMEM for a short workspace. */
#define GSF_NET_WEIGHTS 2736
gsf_status gsf_net_workspace_bytes(int batch, int64_t rows, int64_t cols, size_t* bytes);
gsf_status gsf_net_forward(const uint16_t* w_bf16, int batch, const int32_t* idx, int64_t rows,
                           int64_t cols, const float* inputs, float* y, void* ws, size_t ws_bytes,
                           void* stream);
gsf_status gsf_net_loss_grad(const uint16_t* w_bf16, int batch, const int32_t* idx, int64_t rows,
                             int64_t cols, const float* inputs, const float* targets, float* grad,
                             double* loss, void* ws, size_t ws_bytes, void* stream);
gsf_status gsf_net_adam(int64_t count, int t, double lr, double beta1, double beta2, double eps,
                        float* w, float* mom, float* vel, const float* grad, uint16_t* w_bf16,
                        void* stream);
gsf_status gsf_net_to_bf16(int64_t count, const float* w, uint16_t* w_bf16, void* stream);
gsf_status gsf_net_pair_workspace_bytes(const gsf_operator* op, size_t* bytes);
gsf_status gsf_net_make_pair(const gsf_operator* op, const void* r, int64_t ldr, const void* y,
                             int64_t ldy, const void* g, float* inputs, float* targets, void* ws,
                             size_t ws_bytes, void* stream);

/* Preconditioner handle for gsf_lobpcg_filter: the operator's grid
 * (rows x cols; a 1D operator is one row), guidance g (n values of the
 * operator's element type) and BF16 weights, all borrowed (they must outlive
 * the handle; their contents are read at each use).
 *  gsf_precond_apply: W = T(R) column by column for an n x m point-major
 *    block (no fallback), scratch from gsf_precond_workspace_bytes.
 * Errors: GSF_EINVAL for null pointers or m outside 1..8. */
gsf_status gsf_precond_create(const gsf_operator* op, const void* g, const uint16_t* w_bf16,
                              gsf_precond** out);
/* The preconditioner the network is trained to imitate, as a reference:
 * T(r) = the iterate after inner_steps CG steps on (L_sym + alpha I) y = r
 * from y = 0 (gsf_shifted_cg's recurrences, no tolerance; a zero column gives
 * y = 0, which the fallback rule then replaces by r).  Its cost is
 * inner_steps single-column applies per column and LOBPCG step.  The
 * operator is borrowed; the handle owns the CG scratch (about 4n elements,
 * allocated here and freed by gsf_precond_destroy), so one handle serves one
 * call at a time.  gsf_precond_apply runs the solve without the fallback.
 * GSF_EINVAL for a null op / out, alpha <= 0 or non-finite, inner_steps < 1;
 * GSF_ENOMEM if the scratch cannot be allocated. */
gsf_status gsf_precond_create_shifted(const gsf_operator* op, double alpha, int inner_steps, gsf_precond** out);
void gsf_precond_destroy(gsf_precond* T);
gsf_status gsf_precond_workspace_bytes(const gsf_precond* T, int m, size_t* bytes);
gsf_status gsf_precond_apply(const gsf_precond* T, int m, const void* R, void* W, void* ws,
                             size_t ws_bytes, void* stream);

/* Training targets and residuals.
 *  gsf_shifted_cg: CG for (L_sym + alpha I) y = b from y = 0 (alpha >= 0;
 *    b with stride ldb, y contiguous, n values of the operator's element
 *    type), the recurrences of Algorithm 2 with T = I; stops when
 *    ||r|| <= tol ||b|| or after kmax steps (GSF_ENOTCONV if tol > 0 is not
 *    met; with info != NULL the host stops issuing steps after convergence,
 *    as for gsf_cg_filter); p^T q <= 0 is GSF_EBREAKDOWN.  Workspace: gsf_solver_workspace_bytes
 *    (op, GSF_METHOD_CG, 1, ...).  info may be NULL (then no host sync).
 *  gsf_lobpcg_residual: R = L_sym X - X diag(theta) for an n x m point-major
 *    block (theta: m host doubles). */
gsf_status gsf_shifted_cg(const gsf_operator* op, double alpha, const void* b, int64_t ldb, void* y,
                          int kmax, double tol, void* ws, size_t ws_bytes, gsf_cg_info* info,
                          void* stream);
gsf_status gsf_lobpcg_residual(const gsf_operator* op, int m, const void* X, const double* theta,
                               void* R, void* stream);

/* ---- re-guided (non-linear) filters (Sections 2 and 3) ------------------------
 * The first of the two ways the paper gives to iterate the BF and the GF: the
 * previous result is the guidance of the next step, so the graph is rebuilt
 * (weights of eq. (2), or the statistics of Algorithm 1) from the current
 * iterate before every step.  `desc` gives the kind, shape, precision and
 * parameters as for gsf_build_operator; the guidance of step 1 is x0.
 *   GSF_METHOD_POWER: x <- D(x)^-1 W(x) x, kmax passes (eq. (3) per pass).
 *   GSF_METHOD_CG: Algorithm 2 in x-space with L and D rebuilt from the
 *     current iterate at the start of every step (the flexible beta of
 *     gsf_cg_filter, which the end of Section 5 names as the form for matrices
 *     that change): s = D_k^-1 r, q = L_k p, r updated as printed
 *     (r <- r - alpha q), r_0 = -L(x0) x0.  Stops, statuses and tol as for
 *     gsf_cg_filter, with the breakdown floor (tau)^2 x0^T D(x0) x0 and
 *     ||r|| measured as sqrt(s^T r); info->res is that of the last step taken.
 * x0, x_out: n elements (they may be the same buffer).  ws: device memory of
 * gsf_reguided_workspace_bytes(desc, method) bytes, 256-byte aligned; it holds
 * the solver vectors and, for the GF, the rebuilt operator; for the BF only
 * the degrees: no weight planes are stored.  BF: every pass evaluates the
 * weights of eq. (2) from a tile of the iterate staged in LDS where it uses
 * them (power: one pass per step, y_i = x_i - (1/d_i) sum_j w_ij (x_i - x_j);
 * CG: a degree pass and the pass q = L p, q_i = sum_j w_ij (p_i - p_j)); with
 * FP32 data a weight is 2^(-a log2 e) of its exponent a in FP32 (hardware
 * exponential: relative error a few units of 2^-24 times 1 + |a|), row sums
 * of the window in FP32 and their total in FP64; FP64 data: exp and all sums
 * in FP64.  GF: each step costs one operator build.  With FP32 data the graph
 * is built from the stored FP32 iterate.
 * A 1D BF power filter whose signal fits in one workgroup's LDS (n <= 16384
 * FP32, 8192 FP64) runs all passes in one launch, weights and sums in FP64,
 * the iterate stored in the data type after every pass.
 * GSF_EINVAL for a bad descriptor, a descriptor with more than one guidance
 * channel (the iterate is the guidance), method, kmax < 0 or tol; GSF_ENOMEM
 * for a short workspace.  info may be NULL (then no host sync). */
gsf_status gsf_reguided_workspace_bytes(const gsf_operator_desc* desc, int method, size_t* bytes);
gsf_status gsf_reguided_filter(const gsf_operator_desc* desc, int method, const void* x0, void* x_out,
                               int kmax, double tol, void* ws, size_t ws_bytes, gsf_cg_info* info,
                               void* stream);

/* ---- tuning ---------------------------------------------------------------
 * gsf_tune_apply: times the BF apply (form L_sym, block width m in
 *   {1, 2, 3, 4, 8}) with 1, 2 and 4 grid rows per thread (tile heights 4, 8
 *   and 16 rows; in 2D the two rows of a thread are computed together and
 *   share every neighbour row), in three interleaved rounds of `reps`
 *   launches per candidate, on caller buffers x, y (n*m elements); each
 *   candidate's time is its best round.  The current choice of the class
 *   (tuned earlier, else the default) is kept unless another candidate is
 *   faster by more than 3%; the result holds for every later apply with the
 *   same precision, dimension, radius, width and size class (process-wide)
 *   and is returned in *best_rpt, the three timings (microseconds per launch)
 *   in times_us (NULL allowed).  GF operators: no-op, *best_rpt = 0.
 *   Synchronizes the stream. */
gsf_status gsf_tune_apply(const gsf_operator* op, int m, const void* x, void* y, int reps,
                          int* best_rpt, float* times_us, void* stream);
/* gsf_set_apply_rows: sets the BF apply's rows per thread (1, 2 or 4) for
 *   block width m of this operator's class (precision, dimension, radius,
 *   width, size class), as gsf_tune_apply would; process-wide.  GSF_EINVAL
 *   for other values or a GF operator. */
gsf_status gsf_set_apply_rows(const gsf_operator* op, int m, int rows_per_thread);
/* gsf_get_apply_rows: the rows per thread the BF apply of block width m uses
 *   for this operator (the tuned or set value of its class, else the
 *   default); 0 for a GF operator.  GSF_EINVAL for NULL or m outside 1..8. */
gsf_status gsf_get_apply_rows(const gsf_operator* op, int m, int* rows_per_thread);
/* The process-wide table of tuned tile heights as a JSON file, so that a
 * tuning run can be reused by later processes:
 *   {"gsf_apply_tiles": [{"prec": 0|1, "geometry": 0 (1D) | 1 (2D square) |
 *    2 (2D cross), "radius": 1..8, "width": 1|2|3|4|8, "size_class": 0..3
 *    (n < 2^16, 2^20, 2^23, larger), "rows_per_thread": 1|2|4}, ...]}
 *  gsf_tune_table_save: writes the tuned entries (count in *entries, NULL
 *    allowed).  gsf_tune_table_load: reads a file of that form and sets its
 *    entries (others unchanged); nothing is set if any entry is malformed or
 *    out of range.  GSF_EINVAL for a NULL path, a file that cannot be opened,
 *    written or parsed.  gsf_tune_table_clear: back to the defaults.
 *  Not synchronised with concurrent tuning in other threads. */
gsf_status gsf_tune_table_save(const char* path, int* entries);
gsf_status gsf_tune_table_load(const char* path, int* entries);
void gsf_tune_table_clear(void);

/* ---- batching ----------------------------------------------------------------
 * Many independent items (each its own operator, signal and solver) filtered
 * by one call: the items are spread over 8 branches (longest first), each
 * branch is a HIP graph of its items' operator builds and solves, and a run
 * launches the branch graphs on private streams forked from and joined back
 * to the caller's stream, so branches run side by side.  Every item computes exactly what the
 * single-item calls above compute (same kernels, same order within the
 * item); converged items (tol > 0) turn their remaining kernels into no-ops
 * through their own device-side solver state.
 *  gsf_batch_item: op (all items of a batch share op.prec), device pointers
 *    guidance, x0 (n values) and x_out (n values), method (GSF_METHOD_*), m
 *    (LOBPCG block size 1..8), kmax, constraint (LOBPCG), tol (CG, LOBPCG).
 *  gsf_batch_workspace_bytes: device workspace for the whole batch.
 *  gsf_batch_create: carves the workspace and assigns items to branches;
 *    flags: GSF_BATCH_AUTOTUNE times the BF apply tile per item class (see
 *    gsf_tune_apply; scratch is the item's solver workspace);
 *    GSF_BATCH_GRAPHS records each branch once as a HIP graph (the item
 *    pointers are then baked in: buffers must stay at the same addresses
 *    while the batch exists; their contents may change between runs).
 *    Without GSF_BATCH_GRAPHS each run issues the items' kernels from the
 *    library onto the branch streams (on the 320-item batch: 352 ms replayed,
 *    359 ms issued, the issue rate of the host thread varying by machine).
 *    The first plan created on a device also creates three helper streams of
 *    the library (default priority, kept until the process ends), which run
 *    one empty kernel each before any branch stream runs (the branch streams
 *    then share the device's hardware queues evenly; measured 352-356 ms
 *    against 455-474 ms without); the first carries the tile tuning.
 *  gsf_batch_run: runs the batch ordered after prior work on `stream`;
 *    later work on `stream` waits for every branch (asynchronous).
 *  gsf_batch_get_info: per item (host array of count), after synchronizing
 *    the stream: completed steps, status (as the single-item calls report it),
 *    initial and final residual (CG: ||r||; LOBPCG: largest column residual).
 *  gsf_batch_destroy: frees the host plan and the graph. */
typedef struct {
  gsf_operator_desc op;
  const void* guidance;
  const void* x0;
  void* x_out;
  int32_t method;
  int32_t m;
  int32_t kmax;
  int32_t constraint;
  double tol;
} gsf_batch_item;

typedef struct {
  int32_t iters;
  int32_t status;
  double res0;
  double res;
} gsf_batch_info;

typedef struct gsf_batch gsf_batch;
enum { GSF_BATCH_AUTOTUNE = 1, GSF_BATCH_GRAPHS = 2 };
gsf_status gsf_batch_workspace_bytes(const gsf_batch_item* items, int count, size_t* bytes);
gsf_status gsf_batch_create(const gsf_batch_item* items, int count, void* ws, size_t ws_bytes, int flags,
                            gsf_batch** out);
gsf_status gsf_batch_run(gsf_batch* batch, void* stream);
gsf_status gsf_batch_get_info(const gsf_batch* batch, gsf_batch_info* info, void* stream);
void gsf_batch_destroy(gsf_batch* batch);
/* gsf_batch_filter: the whole batch in one call (create without autotuning
 *   or graphs, run, read the info, destroy): ws as for gsf_batch_create, info
 *   NULL or a host array of count summaries.  The plan's branch streams are
 *   destroyed before returning, so the call synchronizes `stream`.  Returns
 *   the first item status other than OK, ENOTCONV or EBREAKDOWN, else OK. */
gsf_status gsf_batch_filter(const gsf_batch_item* items, int count, void* ws, size_t ws_bytes,
                            gsf_batch_info* info, void* stream);

/* ---- diagnostic entry points (the solver's inner kernels on caller data) ----
 * gsf_block_gram: the Gram pair of the LOBPCG Rayleigh-Ritz step (Algorithm 3,
 *   the Rayleigh-Ritz line): GA = S^T (A S), GB = S^T S for S = [S0 .. S_{nb-1}]
 *   (nb = 1..3 point-major blocks of n x m, m = 1..8, element type prec) and
 *   AS = [A0 ..]; S and AS are arrays of nb device pointers.  Every product
 *   and sum is FP64 for both element types (the product of two FP32 values
 *   is exact in FP64), in a fixed order.  Results are written to host arrays
 *   GA, GB (ns x ns, ns = nb*m, row-major).  The device workspace size comes
 *   from gsf_block_gram_workspace_bytes(n).
 *   Synchronizes the stream.
 * gsf_rayleigh_ritz: the FP64 Rayleigh-Ritz step on a host Gram pair
 *   (ns = 1..24, m <= min(8, ns)): the m smallest Ritz values theta (host, m)
 *   and coefficients C (host, ns x m row-major, zero rows at dropped columns),
 *   kept flags (host int, ns) and the number kept (*nkept).  A column is
 *   dropped when GB_jj <= zero_tol^2 max GB_jj or when the pivot of the
 *   unit-diagonal Cholesky is <= drop_tol.  Device workspace of
 *   gsf_rr_workspace_bytes() bytes; synchronizes the stream. */
gsf_status gsf_block_gram_workspace_bytes(int64_t n, size_t* bytes);
gsf_status gsf_block_gram(int prec, int64_t n, int m, int nb, const void* const* S,
                          const void* const* AS, double* GA, double* GB, void* ws,
                          size_t ws_bytes, void* stream);
size_t gsf_rr_workspace_bytes(void);
gsf_status gsf_rayleigh_ritz(int ns, int m, const double* GA, const double* GB, double drop_tol,
                             double zero_tol, double* theta, double* C, int* kept, int* nkept,
                             void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* GSF_H */
