/*
 * libmofem - matrix-oriented FEM (MO-FEM) multiterm Sylvester solves on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: M. Frittelli, I. Sgura, "Matrix-oriented FEM formulation for
 * stationary and time-dependent PDEs on x-normal domains" (arXiv 2109.01173).
 * Equation numbers below follow the article's sequential numbering.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All floating point data are IEEE float64 ("double").
 *  - A nodal matrix U has q_s rows (s = base coordinate of the x-normal
 *    domain, the paper's y) and q_t columns (t = normalised coordinate, the
 *    paper's x); it is stored row-major and contiguous (leading dimension
 *    q_t).  Left factors act on s, right factors on t, as in eq. (70).
 *  - A batch is `batch` such matrices, item b starting at `b * stride`
 *    elements (stride >= q_s * q_t).
 *  - Pointers documented "device" must be device memory of the current HIP
 *    device; "host" pointers are ordinary CPU memory.  Every array argument
 *    is owned by the caller and must stay valid until the call (or, for
 *    asynchronous calls, the work queued on `stream`) has finished.
 *  - Opaque handles (mofem_op_t, mofem_prec_t) are owned by the library:
 *    created by *_create / *_setup, released by *_destroy.  They hold the
 *    banded matrices and eigenbases in device memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is queued asynchronously on it; functions that return
 *    host-side results (iteration counts, residuals) synchronise it.
 *  - Functions return MOFEM_OK (0) or a negative error code; nothing is
 *    thrown across the ABI.  mofem_last_error() returns a thread-local,
 *    human-readable message for the most recent failure on that thread.
 *
 * Banded ("DIA") storage of a 1D matrix K of size n x n with half-width kb:
 *      band[d * n + i] = K[i][i + d - kb],   d = 0 .. 2 kb,   i = 0 .. n-1
 * with zeros where the column i + d - kb falls outside [0, n).  P_k finite
 * element matrices have half-width kb = k (lumped P1: kb = 1).
 */
#ifndef MOFEM_H
#define MOFEM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------------ */
/* Error codes                                                              */
/* ------------------------------------------------------------------------ */
#define MOFEM_OK              0
#define MOFEM_E_ARG          -1  /* invalid argument (NULL, sizes, flags)     */
#define MOFEM_E_HIP          -2  /* a HIP runtime call failed                 */
#define MOFEM_E_NOMEM        -3  /* device or host allocation failed          */
#define MOFEM_E_BREAKDOWN    -4  /* PCG breakdown: <Q, L(Q)> <= 0 or not finite */
#define MOFEM_E_MAXIT        -5  /* tolerance not reached within maxit        */
#define MOFEM_E_UNSUPPORTED  -6  /* valid request the library does not cover  */
#define MOFEM_E_NOTFINITE    -7  /* NaN or Inf in the input or a residual     */
#define MOFEM_E_NUMERIC      -8  /* setup failed numerically (matrix not SPD,
                                    eigen-iteration did not converge)          */

/* Library version as 10000*major + 100*minor + patch. */
int mofem_version(void);

/* Thread-local message for the last failing call on this thread ("" if none).
   The pointer stays valid until the next libmofem call on this thread. */
const char* mofem_last_error(void);

/* ------------------------------------------------------------------------ */
/* a0. One-dimensional assembly (host only)                                 */
/* ------------------------------------------------------------------------ */
/* Weight functions w(x) for the integrals of Sec. 3.2, eqs. (29)-(31).  The
   "profile" kinds describe the boundary curve of the x-normal domain,
   L(x) = p0 + p1 * sin(p2 * x + p3), and its derived weights. */
enum {
  MOFEM_W_ONE = 0,          /* w = 1                                         */
  MOFEM_W_POLY = 1,         /* w = p0 + p1 x + p2 x^2 + p3 x^3               */
  MOFEM_W_PROFILE = 2,      /* w = L(x)                                      */
  MOFEM_W_PROFILE_D = 3,    /* w = L'(x)                                     */
  MOFEM_W_PROFILE_INV = 4,  /* w = 1 / L(x)                                  */
  MOFEM_W_PROFILE_D2L = 5,  /* w = L'(x)^2 / L(x)                            */
  MOFEM_W_CALLBACK = 6,     /* w = fn(x, ctx)                                */
  /* polynomial profile L(x) = p0 + p1 x + p2 x^2 + p3 x^3 (w = L is
     MOFEM_W_POLY), e.g. L = 2 S for the cap-shaped symmetric domain       */
  MOFEM_W_PPROFILE_D = 7,   /* w = L'(x)                                     */
  MOFEM_W_PPROFILE_INV = 8, /* w = 1 / L(x)                                  */
  MOFEM_W_PPROFILE_D2L = 9  /* w = L'(x)^2 / L(x)                            */
};
typedef double (*mofem_weight_fn)(double x, void* ctx);
typedef struct {
  int kind;             /* one of MOFEM_W_*                                   */
  double p[4];          /* parameters of POLY / PROFILE kinds                 */
  mofem_weight_fn fn;   /* CALLBACK only                                      */
  void* ctx;            /* CALLBACK only, passed through                      */
} mofem_weight;

/* Assemble K_ij = int_{x0}^{x1} psi_i^(di)(x) psi_j^(dj)(x) w(x) dx over a
   uniform mesh of m_elem elements with P_k Lagrange elements (equispaced
   element nodes), Sec. 3.1 eq. (23) and Sec. 3.2 eqs. (29)-(31).
     order   1..4 = P_k with nq-point Gauss-Legendre quadrature per element
             0    = lumped P1 (Sec. 3.3): the integrand is replaced by its
                    element-wise linear interpolant, i.e. integrated with the
                    two-point nodal (trapezoid) rule on each element.
     di, dj  derivative orders (0 or 1) of the row / column function.
     w       weight (NULL = 1).   nq  quadrature points (0 = 12; 1..32).
     band    host output, (2 kb + 1) * n doubles, kb = max(order, 1),
             n = kb * m_elem + 1, DIA layout above.
   Errors: MOFEM_E_ARG for order/di/dj/nq/m_elem out of range or NULL band. */
int mofem_assemble_1d(int order, int m_elem, double x0, double x1, int di, int dj,
                      const mofem_weight* w, int nq, double* band);

/* Dense generalised symmetric-definite eigen-decomposition (host only),
   the one-dimensional diagonalisation of Sec. 4, eq. (55), done once per
   geometry:  K V = M V diag(lam),  V^T M V = I,  lam ascending.
     K, M   host DIA bands (half-width kb) of symmetric n x n matrices, M
            positive definite.
     trim   1 = use rows/columns 1 .. n-2 only (homogeneous Dirichlet),
            0 = all n.  Let q = n - 2*trim.
     lam    host output, q doubles.
     V      host output, q*q doubles, row-major, column j = eigenvector j.
   Errors: MOFEM_E_NUMERIC if M is not positive definite or the iteration
   fails to converge; MOFEM_E_ARG on bad sizes. */
int mofem_geneig_host(int n, int kb, const double* K, const double* M, int trim,
                      double* lam, double* V);

/* Host threads used by one host-side call (assembly, eigen-decomposition;
   mofem_prec_setup splits its share between its two decompositions).
   n <= 0 restores the default (the hardware's threads, at most 16).  Callers
   that run several set-ups concurrently divide the machine with it (e.g. four
   concurrent set-ups on 16 cores: n = 4) instead of oversubscribing it.
   Process-wide; returns the previous count.  Never fails. */
int mofem_set_host_threads(int n);

/* Closed-form generalised eigenpairs of the uniform P1 pencil (A, M) on an
   interval of length len with n_elem elements (host only), Sec. 4.1: with
   Dirichlet conditions the P1 stiffness and consistent mass are tridiagonal
   Toeplitz and related by eq. (60), so the sine vectors of eq. (64)
   diagonalise both, with the eigenvalues of eqs. (63) and (65); the nodal
   (lumped) mass keeps the sine basis, and with Neumann conditions the lumped
   pencil is diagonalised by cosine vectors.  Output as mofem_geneig_host:
   lam ascending, V row-major with V^T M V = I.
     lumped     1 = nodal (trapezoid) mass, 0 = consistent mass.
     dirichlet  1: q = n_elem - 1 interior nodes; 0: q = n_elem + 1 (lumped
                only: MOFEM_E_UNSUPPORTED for the consistent Neumann pencil,
                which has no closed form).
   Errors: MOFEM_E_ARG (n_elem < 2, len <= 0, NULL), MOFEM_E_UNSUPPORTED. */
int mofem_eig_p1_closed(int n_elem, double len, int lumped, int dirichlet, double* lam, double* V);

/* ------------------------------------------------------------------------ */
/* a2/a3. Multiterm operator  Y = sum_t c_t op(L_t) X op(R_t)               */
/* ------------------------------------------------------------------------ */
#define MOFEM_MAX_TERMS 8
typedef struct {
  int kb;               /* common band half-width, 1..4                       */
  int elem_order;       /* k of the P_k matrices (0 = unknown); with k >= 2
                           and element-structured bands the apply skips the
                           structural zeros of the left factors              */
  int n_s, n_t;         /* full node counts of the s and t matrices           */
  int trim_s, trim_t;   /* 1 = homogeneous Dirichlet: drop first/last node    */
  int full_input;       /* 0: X is q_s x q_t (the unknowns).
                           1: X is n_s x n_t (all nodes) and only the rows of
                           the left and the columns of the right factors are
                           trimmed - the full-node load of eq. (74).          */
  int n_terms;          /* 1 .. MOFEM_MAX_TERMS                               */
  const double* left[MOFEM_MAX_TERMS];   /* host DIA bands, n_s rows          */
  const double* right[MOFEM_MAX_TERMS];  /* host DIA bands, n_t rows          */
  int left_transpose[MOFEM_MAX_TERMS];   /* 1 = use L_t^T                     */
  int right_transpose[MOFEM_MAX_TERMS];  /* 1 = use R_t^T                     */
  double coef[MOFEM_MAX_TERMS];          /* c_t                               */
  int scaled[MOFEM_MAX_TERMS];           /* 1 = term is also multiplied by the
                                            per-item scale s_b of the apply   */
  int full_output;      /* 1: X is q_s x q_t and Y is n_s x n_t (all nodes):
                           the transpose of a full_input operator, e.g. the
                           gradient M3[:, I] Lambda M[I, :] of a loss with
                           respect to the full-node load F.  Excludes
                           full_input.                                        */
} mofem_op_desc;
typedef struct mofem_op_s* mofem_op_t;

/* Upload the operator (eq. (73), (75), (91), (92) or (28) are all of this
   form).  Copies the host bands; the descriptor may be freed afterwards.
   q_s = n_s - 2 trim_s, q_t = n_t - 2 trim_t.  Terms of the same scaling
   that share a factor are merged on the host before upload (c1 L1 X R +
   c2 L2 X R = (c1 L1 + c2 L2) X R, e.g. eq. (73)'s (B1 + gamma M3) U M from
   the two terms B1 U M and gamma M3 U M; likewise a shared left factor).  Up
   to six distinct terms (kb <= 2) or four (kb >= 3) run as one kernel pass;
   the rest (at most MOFEM_MAX_TERMS in all) as a second pass adding to Y.
   Errors: MOFEM_E_ARG (sizes, kb, n_terms outside 1..MOFEM_MAX_TERMS, NULL
   bands), MOFEM_E_NOTFINITE (a non-finite band entry), MOFEM_E_NOMEM,
   MOFEM_E_HIP. */
int mofem_op_create(const mofem_op_desc* desc, mofem_op_t* op);
int mofem_op_destroy(mofem_op_t op);
/* Output and input shapes of the operator. */
int mofem_op_shape(mofem_op_t op, int* q_s, int* q_t, int* in_s, int* in_t);

/* Y_b = sum_t c_t (scaled_t ? s_b : 1) op(L_t) X_b op(R_t) for b < batch.
     X          device, input items (q_s x q_t, or n_s x n_t if full_input),
                item b at X + b * in_stride.
     Y          device, output items q_s x q_t at Y + b * stride.  Must not
                overlap X.
     item_scale device [batch] or NULL (s_b = 1).
     dot_xy     device [batch] or NULL: receives <X_b, Y_b>_F (Frobenius,
                eq. (77)'s sum(sum(X o Y)); square operators only).
   Asynchronous on `stream`.  Errors: MOFEM_E_ARG. */
int mofem_op_apply(mofem_op_t op, const double* X, long long in_stride, double* Y,
                   long long stride, int batch, const double* item_scale,
                   double* dot_xy, void* stream);

/* Allocation-free variant of mofem_op_apply, for callers that cannot
   allocate device memory (code under HIP graph capture, tight serving loops,
   harnesses that forbid hipMalloc).  Same arguments, results and errors as
   mofem_op_apply; the partial sums of the fused <X_b, Y_b> live in a static
   device array of MOFEM_NOALLOC_SCRATCH_BYTES per GPU (kept until the process
   ends; the first call on a device looks up its address) instead of a buffer
   the handle allocates, and no timing events are recorded.  Calls no
   hipMalloc, hipFree or other allocating routine.  Limit: with dot_xy,
   batch * tiles partial sums (8 bytes each) must fit the array, where tiles =
   ceil(q_t / (4 (64 - 2 kb))) * ceil(q_s / rows) and rows is about 160 (a
   quarter of that for batches too small to fill the GPU otherwise; 117 tiles
   at q = 2047 and kb = 2, so batch <= 1120); larger requests fail with
   MOFEM_E_ARG.  Every call on one GPU shares that array:
   calls that overlap on one GPU (other streams or threads) race and must be
   serialised by the caller.  Without dot_xy the array is not used. */
#define MOFEM_NOALLOC_SCRATCH_BYTES (1u << 20)
int mofem_op_apply_noalloc(mofem_op_t op, const double* X, long long in_stride, double* Y,
                           long long stride, int batch, const double* item_scale,
                           double* dot_xy, void* stream);

/* Batched Frobenius products (eq. (77)'s sum(sum(X o Y)) per item):
     out[b] = beta * out[b] + alpha * <X_b, Y_b>_F,   b < batch,
   X_b = X + b * stride (n contiguous doubles), likewise Y_b; out device.
   Fixed-order two-pass reduction (bitwise reproducible).  Uses a small
   library-owned device buffer per thread.  Errors: MOFEM_E_ARG. */
int mofem_dot_accumulate(const double* X, const double* Y, long long n, long long stride,
                         int batch, double alpha, double beta, double* out, void* stream);

#define MOFEM_MAX_BAND_SUM 4
/* A banded matrix given as a sum  sum_i coef[i] band[i]  of host DIA bands of
   half-width kb (e.g. eq. (80)'s A + B2: two terms); n = 0 is the zero
   matrix.  The sum is formed by the library. */
typedef struct {
  int n;                                    /* 0 .. MOFEM_MAX_BAND_SUM        */
  const double* band[MOFEM_MAX_BAND_SUM];   /* host DIA bands, symmetric      */
  double coef[MOFEM_MAX_BAND_SUM];
} mofem_band_sum;

/* ------------------------------------------------------------------------ */
/* a1/a4. Single-term spectral preconditioner                              */
/*   P(U) = a Ms U Mt + bs Ks U Mt + bt Ms U Kt + d Ks U Kt                  */
/*   P^{-1}(R) = V_s ((V_s^T R V_t) ./ D) V_t^T,                             */
/*   D_ij = a + s_b (bs lam_i + bt mu_j + d lam_i mu_j)                      */
/* (the reduced spectral solve of Sec. 4, eqs. (55)-(59), applied as the    */
/*  single-term preconditioner of Sec. 5, eq. (80), and Sec. 6, eq. (95)).   */
/* ------------------------------------------------------------------------ */
enum {
  MOFEM_PREC_F64 = 0,     /* FP64 MFMA transforms                           */
  MOFEM_PREC_F32 = 1,     /* FP32 MFMA transforms, FP32 intermediates       */
  MOFEM_PREC_BF16 = 2,    /* BF16 operands, FP32 accumulation               */
  MOFEM_PREC_BF16X3 = 3,  /* split BF16 (hi + lo), three products per term,
                             FP32 accumulation                              */
  MOFEM_PREC_BF16X2 = 4,  /* split BF16 for the data operands, eigenbases
                             rounded to BF16: the preconditioner is defined
                             with the rounded (still nonsingular) bases, so
                             P stays symmetric positive definite and each
                             transform needs two products; FP32 accumulation */
  MOFEM_PREC_BF16_FWD = 5, /* forward transforms (V_s^T R V_t) in BF16 (one
                             product), back transforms (V_s (.) V_t^T) in
                             split BF16 (three); FP32 accumulation.  Not
                             symmetric: use the flexible PCG.               */
  MOFEM_PREC_F64_INT8 = 6, /* FP64-accurate transforms on INT8 MFMA: every
                             row of an operand cut into 7 exact signed
                             base-128 digits (round to nearest) below its
                             power-of-two exponent, the 28 digit products
                             with p + q <= 8 formed exactly in int32 and
                             summed in FP64 (error-free splitting of Ozaki,
                             Ogita, Oishi and Rump); error per entry below
                             2^-46 K 2^(e_row + e_col).
                             FP64 intermediates and Z; operand widths
                             (padded) up to 16384, else MOFEM_E_UNSUPPORTED
                             at set-up or on mofem_prec_set_precision.      */
  MOFEM_PREC_BF16_FWD_VS = 7 /* as MOFEM_PREC_BF16_FWD, but the first back
                             transform (V_s S) splits only the eigenbasis:
                             S in plain BF16, two products; its lo half is
                             never formed.  The flexible PCG absorbs the
                             rounding of S as it does that of the forward
                             transforms.  Not symmetric: use the flexible
                             PCG.                                           */
};
typedef struct {
  int kb;                       /* band half-width of the four matrices       */
  int n_s, n_t, trim_s, trim_t; /* as in mofem_op_desc                        */
  const double* Ks;             /* host DIA bands, symmetric                  */
  const double* Ms;             /* host DIA bands, symmetric positive definite */
  const double* Kt;
  const double* Mt;
  double alpha, beta_s, beta_t, delta;   /* coefficients of D                 */
  int precision;                /* MOFEM_PREC_*                               */
  mofem_band_sum Ks_add;        /* further bands added to Ks, and to Kt      */
  mofem_band_sum Kt_add;        /* (n = 0: none; the sums formed on the host), */
                                /* e.g. Kt = A with Kt_add = {B2, w} for the   */
                                /* pencil (A + w B2, M)                       */
} mofem_prec_desc;
typedef struct mofem_prec_s* mofem_prec_t;

/* Solve the two generalised eigenproblems (Ks + Ks_add, Ms) and
   (Kt + Kt_add, Mt) in FP64 on the host (once per geometry), upload V_s, V_t
   and their transposes in FP64 and in the working precision.  Errors:
   MOFEM_E_ARG (also an added-band count outside 0..MOFEM_MAX_BAND_SUM or a
   NULL added band), MOFEM_E_NUMERIC, MOFEM_E_NOMEM, MOFEM_E_HIP. */
int mofem_prec_setup(const mofem_prec_desc* desc, mofem_prec_t* prec);
int mofem_prec_destroy(mofem_prec_t prec);
/* The same preconditioner from given generalised eigenpairs (host arrays:
   lam [q_s], Vs [q_s x q_s] row-major with column j the eigenvector of
   lam[j] and Vs^T Ms Vs = I; mu, Vt likewise), e.g. the closed forms of
   mofem_eig_p1_closed: no eigen-decomposition.  The arrays are copied.
   Errors: MOFEM_E_ARG, MOFEM_E_NOMEM, MOFEM_E_HIP. */
int mofem_prec_setup_eig(int q_s, int q_t, const double* lam, const double* Vs, const double* mu,
                         const double* Vt, double alpha, double beta_s, double beta_t, double delta,
                         int precision, mofem_prec_t* prec);
/* Change a, bs, bt, d (e.g. a new gamma, tau or diffusion coefficient)
   without a new eigen-decomposition. */
int mofem_prec_set_coeffs(mofem_prec_t prec, double alpha, double beta_s,
                          double beta_t, double delta);
/* Change the transform precision (MOFEM_PREC_*) of an existing handle. */
int mofem_prec_set_precision(mofem_prec_t prec, int precision);
/* Copy the eigenvalues (host, q_s and q_t doubles; either may be NULL). */
int mofem_prec_eigenvalues(mofem_prec_t prec, double* lam, double* mu);
/* Bytes of device workspace mofem_prec_apply needs for `batch` items, for any
   precision (a workspace stays valid across mofem_prec_set_precision). */
size_t mofem_prec_workspace_size(mofem_prec_t prec, int batch);

/* Z_b = P^{-1}(R_b) for b < batch (R, Z device, q_s x q_t items, `stride`
   apart; Z may not overlap R).  item_scale: device [batch] or NULL (s_b).
   workspace: device, mofem_prec_workspace_size bytes, or NULL to use a
   buffer the handle allocates on first use and keeps.
   Asynchronous on `stream`.  Errors: MOFEM_E_ARG, MOFEM_E_NOMEM. */
int mofem_prec_apply(mofem_prec_t prec, const double* R, double* Z, long long stride,
                     int batch, const double* item_scale, void* workspace,
                     size_t ws_bytes, void* stream);

/* Autotuner of the transforms' block tile (128 x 128 or 64 x 64) for this
   handle's shapes, its current precision and `batch`: times one application
   with each (on scratch buffers it allocates and frees) and keeps the faster
   choice in the handle for later applications with that precision and batch
   size (otherwise: 128 unless its grid gives fewer than two blocks per
   compute unit).  Synchronises `stream`.  tile_out: host, may be NULL.
   Errors: MOFEM_E_ARG, MOFEM_E_NOMEM, MOFEM_E_HIP. */
int mofem_prec_tune(mofem_prec_t prec, int batch, int* tile_out, void* stream);
/* Set that choice directly (tile 64 or 128) for the current precision and
   `batch`.  Errors: MOFEM_E_ARG. */
int mofem_prec_set_tile(mofem_prec_t prec, int batch, int tile);

/* ------------------------------------------------------------------------ */
/* The paper's product preconditioners by banded Cholesky solves             */
/*   P_j(U) = S_j U T_j,  S_j = a Ms + c_j bs Ks,  T_j = a Mt + c_j bt Kt    */
/*   P_j^{-1}(R) = S_j^{-1} R T_j^{-1}                                        */
/* (Sec. 5, eq. (80): Ks = B1, Kt = A + B2, a = 0, bs = bt = 1, scale 1;     */
/*  Sec. 6, eq. (95): Ms = M3, Ks = B1, Mt = M, Kt = A + B2, a = 1,           */
/*  bs = bt = 1, one scale c = d tau per species).                           */
/* ------------------------------------------------------------------------ */
#define MOFEM_MAX_SCALES 8
typedef struct {
  int kb;                       /* band half-width of the four matrices, 1..4 */
  int n_s, n_t, trim_s, trim_t; /* as in mofem_prec_desc                      */
  mofem_band_sum Ks;            /* at least one term                          */
  mofem_band_sum Ms;            /* at least one term unless a == 0            */
  mofem_band_sum Kt;
  mofem_band_sum Mt;
  double a, bs, bt;             /* S_j = a Ms + c_j bs Ks, T_j likewise        */
  int n_scales;                 /* 1 .. MOFEM_MAX_SCALES                      */
  double scales[MOFEM_MAX_SCALES];  /* c_j                                    */
} mofem_bprec_desc;
/* Factorise every S_j and T_j (interior rows and columns when trimmed) by
   banded Cholesky on the host in FP64 (the factors keep half-width kb) and
   upload the factors.  The returned handle is used like a spectral one
   (mofem_prec_apply, mofem_prec_workspace_size, mofem_pcg_*, mofem_imex_*):
   one application is a forward and a back substitution along each dimension,
   O(kb q_s q_t) work per item and about 64 bytes of HBM traffic per entry.
   Item b uses the factor pair j whose scale c_j equals its item scale s_b
   exactly (s_b = 1 when item_scale is NULL).  An item whose scale matches no
   c_j gets a NaN result (a solve then stops with MOFEM_E_NOTFINITE); the IMEX
   entry points check their scales d * tau on the host and return MOFEM_E_ARG
   before any launch.  Arithmetic is
   FP64 only: mofem_prec_set_precision accepts MOFEM_PREC_F64 alone, and
   mofem_prec_set_coeffs, mofem_prec_eigenvalues, mofem_prec_tune and
   mofem_prec_set_tile return MOFEM_E_UNSUPPORTED for this handle.
   Errors: MOFEM_E_ARG (kb, sizes, trim flags, NULL bands, term counts,
   n_scales), MOFEM_E_NUMERIC (a factor is not positive definite, e.g.
   eq. (80) under Neumann conditions, where B1 is singular), MOFEM_E_NOMEM,
   MOFEM_E_HIP. */
int mofem_prec_setup_banded(const mofem_bprec_desc* desc, mofem_prec_t* prec);

/* ------------------------------------------------------------------------ */
/* a5/a6/a8. MO-PCG (Sec. 5, eqs. (77)-(78)) on a batch of equations        */
/*           L_b(U_b) = Rhs_b                                               */
/* ------------------------------------------------------------------------ */
#define MOFEM_PCG_FLEXIBLE   1u  /* beta = <Z+, R+ - R> / <Z, R> (needed when
                                    the preconditioner is inexact: BF16)    */
#define MOFEM_PCG_ZERO_GUESS 2u  /* ignore U on entry, start from 0          */
#define MOFEM_PCG_TAU_STOP   4u  /* stop when ||R_s|| <= tol ||R_0|| (the rule
                                    of Sec. 6) instead of tol ||Rhs||         */
/* Bytes of device workspace mofem_pcg_solve needs. */
size_t mofem_pcg_workspace_size(mofem_op_t op, mofem_prec_t prec, int batch);

/* Solve every item to   ||Rhs_b - L_b(U_b)||_F <= tol ||Rhs_b||_F   on the
   FP64 true residual (recomputed at exit; if the recurrence drifted, the
   solve restarts from the true residual).  The recurrence scalars, all
   inner products and U, R, Q are FP64 on the device; the preconditioner runs
   in the handle's precision, and with an FP32 or BF16-family preconditioner
   its output Z is kept in FP32 (far below its own error), so the inner
   products with Z and the direction update read 4 bytes per entry.
     Rhs        device, q_s x q_t items at `stride`.
     U          device, in: initial guess (unless ZERO_GUESS), out: solution.
     item_scale device [batch] or NULL, passed to op and preconditioner.
     iters_out, relres_out  host [batch] or NULL.
   Errors: MOFEM_E_MAXIT (U holds the last iterate, relres_out its true
   relative residual), MOFEM_E_BREAKDOWN (U holds the last iterate with a
   valid step), MOFEM_E_NOTFINITE, MOFEM_E_ARG, MOFEM_E_NOMEM.  The iteration runs under device-side control; the host
   reads a few bytes of flags one iteration behind and synchronises once at
   the end. */
int mofem_pcg_solve(mofem_op_t op, mofem_prec_t prec, const double* Rhs, double* U,
                    long long stride, int batch, const double* item_scale,
                    double tol, int maxit, unsigned flags, void* workspace,
                    size_t ws_bytes, int* iters_out, double* relres_out, void* stream);

/* The same solve without any host synchronisation (capturable in a HIP
   graph; several solves on several streams overlap): exactly `maxit`
   iterations are queued, the items that converged run masked (their
   kernels exit at once), and the per-item results stay on the device.
     workspace  required (mofem_pcg_workspace_size bytes), device.
     iters_dev, status_dev  device [batch] int: iterations and MOFEM_OK or the
                error code of mofem_pcg_solve for that item (E_MAXIT,
                E_BREAKDOWN, E_NOTFINITE).
     relres_dev device [batch]: final true relative residual.
   Returns MOFEM_OK once everything is queued; errors only for invalid
   arguments or failed launches. */
int mofem_pcg_solve_async(mofem_op_t op, mofem_prec_t prec, const double* Rhs, double* U,
                          long long stride, int batch, const double* item_scale,
                          double tol, int maxit, unsigned flags, void* workspace,
                          size_t ws_bytes, int* iters_dev, int* status_dev,
                          double* relres_dev, void* stream);

/* Independent batched solves of uneven shapes (one group per operator /
   preconditioner pair), advanced together on one stream each so that the
   groups overlap on the device; each group stops as in mofem_pcg_solve.
   Arguments of a group as in mofem_pcg_solve (workspace required). */
typedef struct {
  mofem_op_t op;
  mofem_prec_t prec;
  const double* rhs;
  double* u;
  long long stride;
  int batch;
  const double* item_scale;
  double tol;
  int maxit;
  unsigned flags;
  void* workspace;
  size_t ws_bytes;
  int* iters_out;       /* host [batch] or NULL */
  double* relres_out;   /* host [batch] or NULL */
} mofem_pcg_group;
/*   streams     [n_groups] created streams (may repeat; groups on one stream
                 serialise).
     status_out  host [n_groups] or NULL: the first error of each group.
   Returns the first error over all groups (as mofem_pcg_solve).
   Synchronises every stream once at the end. */
int mofem_pcg_solve_many(int n_groups, const mofem_pcg_group* groups, void* const* streams,
                         int* status_out);

/* Grouped solves of uneven instances (same arguments and results as
   mofem_pcg_solve_many).  Groups with the same shape (q_s, q_t), transform
   precision, preconditioner coefficients (a, bs, bt, d), tolerance, maxit,
   flags and presence of item_scale form one class, solved as ONE batched
   MO-PCG: every stage of an iteration is one launch over all the class's
   items (the operator apply: one launch per distinct operator, e.g. per
   element order k), and each item reaches its own preconditioner bases and
   eigenvalues through per-item pointer tables (instances of different k or
   geometry that share a shape share the launches).  Classes advance together
   on the streams of their first groups.  The groups' workspace fields are not
   used: each class allocates (hipMalloc) and frees one buffer holding its
   gathered right-hand sides, solutions, tables and PCG workspace; solutions
   are scattered back to the groups' U.  Spectral preconditioners only
   (MOFEM_E_UNSUPPORTED for banded ones).  Synchronises every stream used. */
int mofem_pcg_solve_grouped(int n_groups, const mofem_pcg_group* groups, void* const* streams,
                            int* status_out);

/* ------------------------------------------------------------------------ */
/* a7. IMEX Euler step (Sec. 6, eqs. (87)-(96); DIB kinetics Sec. 7)        */
/* ------------------------------------------------------------------------ */
enum { MOFEM_KIN_NONE = 0, MOFEM_KIN_DIB = 1 };
typedef struct {
  mofem_op_t op;        /* L_c = Mass + c * Stiffness: its `scaled` terms are
                           multiplied by c = d * tau per species             */
  mofem_prec_t prec;    /* preconditioner of the same split (a = 1, b = c)    */
  mofem_op_t mass;      /* the one-term right-hand-side operator M3 (.) M     */
  double tau;           /* time step                                          */
  double d[2];          /* diffusion coefficient per species                  */
  int n_species;        /* 1 (heat) or 2 (reaction-diffusion system)          */
  int kinetics;         /* MOFEM_KIN_*                                        */
  double kin[10];       /* DIB: rho, A1, A2, B, C, D, alpha, gamma, k2, k3   */
  double tol;           /* per-step PCG tolerance (relative)                  */
  int maxit;
  unsigned flags;       /* MOFEM_PCG_* (ZERO_GUESS is ignored: U^n is the guess) */
} mofem_imex_desc;
size_t mofem_imex_workspace_size(const mofem_imex_desc* desc, int batch);

/* Advance `batch` independent instances by one step:
   U^{n+1} = L_c^{-1}[ Mass(U^n + tau f(U^n, V^n)) ] per species (eqs. (91),
   (93)), kinetics evaluated explicitly at U^n.
     state  device, n_species * batch items of q_s x q_t at `stride`, species
            major: item (sp, b) at state + (sp * batch + b) * stride.
            Updated in place.
     iters_out  host [n_species * batch] or NULL.
   Errors as mofem_pcg_solve. */
int mofem_imex_step(const mofem_imex_desc* desc, double* state, long long stride,
                    int batch, void* workspace, size_t ws_bytes, int* iters_out,
                    void* stream);

/* One IMEX step as a HIP graph over fixed buffers: the right-hand side and
   exactly `iters_per_step` PCG iterations per solve (items that converged
   run masked, so the result equals mofem_imex_step's when iters_per_step
   covers its iteration count), with no host synchronisation.  Each replay
   advances `state` (the buffer given at creation) by one step; replays on
   one stream run back to back without host involvement.
     workspace   device, mofem_imex_workspace_size bytes, owned by the caller
                 and kept alive (and unused elsewhere) while the graph lives.
   The graph owns small device result arrays; mofem_imex_graph_result reads,
   for every item since the previous read, the largest iteration count and
   the first non-OK status (MOFEM_E_MAXIT when iters_per_step was too few),
   plus the last step's relative residual, and returns the first error. */
typedef struct mofem_imex_graph_s* mofem_imex_graph_t;
int mofem_imex_graph_create(const mofem_imex_desc* desc, double* state, long long stride,
                            int batch, void* workspace, size_t ws_bytes, int iters_per_step,
                            mofem_imex_graph_t* graph, void* stream);
int mofem_imex_graph_launch(mofem_imex_graph_t graph, int nsteps, void* stream);
int mofem_imex_graph_result(mofem_imex_graph_t graph, int* max_iters, int* status,
                            double* relres, void* stream);
int mofem_imex_graph_destroy(mofem_imex_graph_t graph);

/* Reverse (adjoint) IMEX Euler step: the exact derivative of
   mofem_imex_step for a scalar loss J.  With c = d * tau per species,
     mu  = L_c^{-1}(lam)              (L_c is symmetric: one more MO-PCG solve
                                       with the same operator, preconditioner,
                                       tol and flags, zero initial guess),
     grad_d[item] += -tau <mu, K(U^{n+1})>    (dL_c/dd = tau K),
     nu  = Mass(mu),
     lam := nu                                       (no kinetics), or
     lam_U := nu_U + tau rho (f_U o nu_U + g_U o nu_V),
     lam_V := nu_V + tau rho (f_V o nu_U + g_V o nu_V)   (DIB, eqs. (99)-(100);
                                       o = entrywise, partials at U^n, V^n).
     stiff      operator K (the stiffness part: L_c = Mass + c K), unknowns
                to unknowns, same shape.
     state_n    device, the step's input state  (layout of mofem_imex_step).
     state_np1  device, the step's output state.
     lam        device, in: dJ/d state_np1, out: dJ/d state_n (same layout).
     grad_d     device [n_species * batch], accumulated.
   stride must equal q_s * q_t.  Errors as mofem_pcg_solve. */
size_t mofem_imex_adjoint_workspace_size(const mofem_imex_desc* desc, int batch);
int mofem_imex_adjoint_step(const mofem_imex_desc* desc, mofem_op_t stiff, const double* state_n,
                            const double* state_np1, double* lam, double* grad_d,
                            long long stride, int batch, void* workspace, size_t ws_bytes,
                            int* iters_out, void* stream);

/* ------------------------------------------------------------------------ */
/* Kernel tracing                                                           */
/* ------------------------------------------------------------------------ */
/* While enabled, every kernel the library launches is bracketed by a pair of
   HIP events recorded on the launch stream, tagged with a kernel class and
   the number of batch items the launch processed.  Costs two event records
   per launch; off by default.  Process-wide and thread-safe. */
enum {
  MOFEM_TRACE_BAND = 0,         /* multiterm operator / load (k_band)          */
  MOFEM_TRACE_GEMM_F64 = 1,     /* one FP64 transform product                  */
  MOFEM_TRACE_GEMM_BF16X3 = 2,  /* one split-BF16 transform product            */
  MOFEM_TRACE_GEMM_BF16 = 3,    /* one BF16 transform product                  */
  MOFEM_TRACE_VEC = 4,          /* PCG vector kernels and reductions           */
  MOFEM_TRACE_GEMM_BF16X2 = 5,  /* one two-product transform                   */
  MOFEM_TRACE_GEMM_F32 = 6,     /* one FP32 transform product                  */
  MOFEM_TRACE_BCHOL = 7,        /* one banded Cholesky solve (two per product-
                                   preconditioner application)               */
  MOFEM_TRACE_GEMM_I8 = 8,      /* one FP64-accurate transform product on INT8
                                   MFMA (28 digit products)                  */
  MOFEM_TRACE_CLASSES = 9
};
/* on != 0: discard earlier records and start recording; on == 0: stop. */
int mofem_trace_enable(int on);
/* Record only the classes whose bit (1 << class) is set in `mask` (default:
   all).  Every recorded launch adds two timing events (without system-scope
   fences) to its stream; a selection keeps a traced run closer still to an
   untraced one.  Never fails. */
int mofem_trace_select(unsigned mask);
/* Synchronise the recorded events and return, for one class, the summed
   kernel time in milliseconds, the number of launches and the summed batch
   items processed (any pointer may be NULL).  Errors: MOFEM_E_ARG (class). */
int mofem_trace_read(int cls, double* total_ms, long long* launches, double* items);

#ifdef __cplusplus
}
#endif
#endif /* MOFEM_H */
