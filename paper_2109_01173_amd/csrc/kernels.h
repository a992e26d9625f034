// Kernel argument blocks and launchers (host-callable, defined in the .hip
// translation units).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mofem {

// ---- banded multiterm operator (k_band.hip) --------------------------------
struct BandArgs {
  const double* X;         // input items
  long long in_stride;     // elements between input items
  int ld_x;                // input row length
  double* Y;               // output items
  long long out_stride;
  int ld_y;
  int qs, qt;              // output shape
  int ns_in, nt_in;        // input shape
  int off_s, off_t;        // input index of output (i, j): (i + off_s, j + off_t)
  int ph_s;                // node index of output row i is i + ph_s
  int n_rowblk;            // row blocks per item (band_rows_per_block rows each)
  const double* left;      // [ns_in][nt][2kb+1] left bands by input row a: coefficient of
                           // output row a - off_s + e - kb (transposed on the host)
  const double* right;     // [nt][2kb+1][qt] column bands (input col j+off_t+d-kb)
  int scaled_mask;         // bit t: term t times item_scale[b]
  const double* item_scale;  // [batch] or null
  double* dot_partial;     // [batch][n_partial] or null: <X, Y> per tile
  int n_partial;           // tiles per item
  const int* active;       // [batch] or null: skip items with active[b] == 0
  int accumulate;          // 1: Y += result (a later pass of a many-term operator)
  int batch;               // items (the launch may pair them: two per lane)
};
// rows per block of the default (small = 0) or the small-block variant
// (small = 1, band widths with band_has_small only): a quarter of the rows,
// for grids that would otherwise leave compute units idle
int band_rows_per_block(int kb, int nt, int small);
int band_has_small(int kb);
int band_cols_per_block(int kb);
int band_pass_terms(int kb);  // terms one launch takes (more run as passes)
int launch_band_apply(const BandArgs& a, int kb, int nt, int batch, bool pattern, int small, hipStream_t s);

// ---- banded Cholesky solves of the product preconditioners (k_bchol.hip) -----
// Out^T = S^{-1} X per item: X is n_rows x n_cols (row length ld_x), S = L L^T
// of order n_rows with half-width kb; Out is n_cols x n_rows (row length ld_o).
struct BcholArgs {
  const double* X;
  long long x_stride;
  int ld_x;
  double* W;               // scratch items, n_rows x n_cols (row length n_cols)
  long long w_stride;
  double* Out;
  long long o_stride;
  int ld_o;
  int n_rows, n_cols;
  const double* Lf;        // [n_sets][n_rows][kb+1]: 1/L[i][i], L[i][i-1], .., L[i][i-kb]
  const double* Lb;        // [n_sets][n_rows][kb+1]: 1/L[i][i], L[i+1][i], .., L[i+kb][i]
  const double* scales;    // [n_sets]: item b uses the set whose scale equals item_scale[b]
  int n_sets;              //           (1.0 when item_scale is null; set 0 if none matches)
  const double* item_scale;
  const int* active;
};
int launch_bchol(const BcholArgs& a, int kb, int batch, hipStream_t s);

// ---- dense transforms on MFMA (k_gemm.hip) ------------------------------------
// C[m][n] = sum_k A[m][k] B[n][k]   (both operands K-contiguous, "NT").
// Padded operands: rows and row length rounded up to kPad, zero padding.
constexpr int kPad = 128;
__host__ __device__ inline int pad_up(int x) { return (x + kPad - 1) / kPad * kPad; }

enum GemmPrec { GEMM_F64 = 0, GEMM_F32 = 1, GEMM_BF16 = 2, GEMM_BF16X3 = 3, GEMM_BF16X2 = 4, GEMM_I8 = 5 };
// raw: row-major ld = N, FP64 or (FP32 and BF16 products only) FP32 into c_hi
enum GemmOMode { O_PAD_T = 0, O_PAD_N = 1, O_F64_RAW = 2, O_F32_RAW = 3 };

struct GemmArgs {
  int M, N, K;             // logical sizes
  // A: padded (rows pad_up(M), ld pad_up(K))
  const double* a64;       // padded FP64
  const void* a_hi;        // padded low-precision operand (FP32 / BF16 hi)
  const void* a_lo;        // padded BF16 lo (BF16X3)
  long long a_stride;      // elements between batch items (0 = shared)
  // B: always padded (rows pad_up(N), ld pad_up(K))
  const double* b64;
  const void* b_hi;
  const void* b_lo;
  long long b_stride;
  // output
  double* c64;             // FP64 output (raw or padded)
  void* c_hi;              // low-precision padded output (FP32 / BF16 hi)
  void* c_lo;              // BF16 lo
  long long c_stride;
  // epilogue: divide by D_ij = alpha + s_b (bs lam_i + bt mu_j + d lam_i mu_j)
  int divide;
  const double* lam;       // [M]
  const double* mu;        // [N]
  double alpha, beta_s, beta_t, delta;
  const double* item_scale;  // [batch] or null
  double out_scale;        // multiply the result (before the epilogue division)
  const int* active;
  int split_a;             // GEMM_BF16X2: the split operand is A (else B)
  // GEMM_I8 (k_ozaki.hip): kOzSlices digit planes per operand and item,
  // [plane][pad_up(rows)][pad_up(K)] int8, a_stride / b_stride in bytes; row
  // exponents [pad_up(rows)] per item (stride 0 = shared)
  const signed char* a_i8;
  const signed char* b_i8;
  const int* a_exp;
  const int* b_exp;
  long long a_exp_stride, b_exp_stride;
  // grouped solves (instances of one shape, each with its own bases): when
  // set, item b reads that operand from a_item[b] (lo half a_item_lo[b],
  // digit exponents a_exp_item[b]) instead of base + b * stride, and its
  // eigenvalues from lam_item[b] / mu_item[b]
  const void* const* a_item;
  const void* const* a_item_lo;
  const int* const* a_exp_item;
  const void* const* b_item;
  const void* const* b_item_lo;
  const int* const* b_exp_item;
  const double* const* lam_item;
  const double* const* mu_item;
};
// tile: block tile edge, 128 (4 waves of 64 x 64) or 64 (4 waves of 32 x 32)
int launch_gemm(const GemmArgs& g, int prec, int omode, int batch, int tile, hipStream_t s);
// FP64-accurate products from exact INT8 slice products (k_ozaki.hip):
// kOzSlices 7-bit digits per entry, K (padded) at most kOzMaxK so that the
// int32 diagonal sums cannot overflow
constexpr int kOzSlices = 7;
constexpr int kOzMaxK = 16384;
// rows of X (M x K, row length ld, item stride xs) -> digit planes (item
// stride os bytes, planes of pad_up(M) x pad_up(K)) and row exponents (item
// stride es); every padded row is written
int launch_slice_rows(const double* X, long long xs, int ld, int M, int K, signed char* out, long long os, int* ex,
                      long long es, int batch, const int* active, hipStream_t s);
int launch_gemm_i8(const GemmArgs& g, int omode, int batch, hipStream_t s);
// raw FP64 items (M x K) -> padded FP64, FP32 or split BF16 operand
int launch_pad_operand(const double* A, long long a_stride, int M, int K, double* o64, float* o32,
                       unsigned short* ohi, unsigned short* olo, long long o_stride, int split, int batch,
                       const int* active, hipStream_t s);

// ---- vector kernels of the PCG recurrence (k_vec.hip) -----------------------
// Blocks per item of the vector kernels: one per 2048 entries, at most
// kVecBlocks (the partial-sum arrays hold kVecBlocks per item).  Every
// reduction of partial sums uses the count of the kernel that wrote them.
constexpr int kVecBlocks = 1920;
inline int vec_blocks(long long n) {
  const long long b = (n + 2047) / 2048;
  return b < 1 ? 1 : (b > kVecBlocks ? kVecBlocks : (int)b);
}
int launch_reduce(const double* partial, int n_partial, double* out, int batch, hipStream_t s);
// out[b] = beta out[b] + alpha (sum of partials)
int launch_reduce_axpy(const double* partial, int n_partial, double* out, double alpha, double beta, int batch,
                       hipStream_t s);
// adjoint of the DIB kinetics in one IMEX step (kin = rho, A1, A2, B, C, D, alpha, gamma, k2, k3)
int launch_dib_adjoint(const double* U, const double* V, const double* NU, const double* NV, double* LU, double* LV,
                       long long n, long long stride, int batch, const double* kin, double tau, hipStream_t s);
// out[b] = sum(X_b * Y_b) partials (X may equal Y)
int launch_dot_partial(const double* X, const double* Y, long long n, long long stride,
                       int batch, double* partial, const int* active, hipStream_t s);
// R = Rhs - Y  (and partial <R, R>)
int launch_residual(const double* Rhs, const double* Y, double* R, long long n, long long stride,
                    long long rhs_stride, int batch, double* partial, const int* active, hipStream_t s);
// alpha_b = num_b / den_b; U += alpha Q (skipped when U is null); R -= alpha Y; partial <R, R>
// cg_update that also writes R's padded transform operand (row length
// pad_up(qt)): FP64 (o64), FP32 (o32) or split BF16 (ohi, olo); padding left untouched
int launch_cg_update_pad(double* U, double* R, const double* Q, const double* Y, const double* num,
                         const double* den, double* alpha_out, int qs, int qt, long long stride,
                         long long u_stride, int batch, double* partial, const int* active, unsigned short* ohi,
                         unsigned short* olo, double* o64, float* o32, long long o_stride, hipStream_t s);
int launch_cg_update(double* U, double* R, const double* Q, const double* Y, const double* num,
                     const double* den, double* alpha_out, long long n, long long stride,
                     long long u_stride, int batch, double* partial, const int* active,
                     hipStream_t s);
// Q = Z + beta Q with beta_b given (Z in FP64 or FP32)
int launch_direction(double* Q, const double* Z, const double* beta, long long n,
                     long long stride, int batch, const int* active, hipStream_t s);
int launch_direction(double* Q, const float* Z, const double* beta, long long n,
                     long long stride, int batch, const int* active, hipStream_t s);
// deferred solution update and new direction, items with live[b]:
// U += alpha Q; then, if active[b], Q = Z + beta Q
int launch_step_direction(double* Q, const double* Z, const double* beta, double* U, const double* alpha,
                          long long n, long long stride, long long u_stride, int batch, const int* live,
                          const int* active, hipStream_t s);
int launch_step_direction(double* Q, const float* Z, const double* beta, double* U, const double* alpha,
                          long long n, long long stride, long long u_stride, int batch, const int* live,
                          const int* active, hipStream_t s);
// R = Rhs - LU - alpha_b Y (and partial <R, R>): the residual of U + alpha Q
int launch_residual_step(const double* Rhs, const double* LU, const double* Y, const double* alpha, double* R,
                         long long n, long long stride, long long rhs_stride, int batch, double* partial,
                         const int* active, hipStream_t s);
// <X, Y> partials with Y in FP32
int launch_dot_partial(const double* X, const float* Y, long long n, long long stride,
                       int batch, double* partial, const int* active, hipStream_t s);
// <R, Z> and <Z, Y> partials in one pass (Z in FP64 or FP32)
int launch_zdots_partial(const double* R, const double* Z, const double* Y, long long n, long long stride,
                         int batch, double* partial1, double* partial2, const int* active, hipStream_t s);
int launch_zdots_partial(const double* R, const float* Z, const double* Y, long long n, long long stride,
                         int batch, double* partial1, double* partial2, const int* active, hipStream_t s);
// Y = X copy; X = 0
int launch_copy(const double* X, double* Y, long long n, long long xs, long long ys, int batch,
                hipStream_t s);
int launch_fill(double* X, double v, long long n, long long stride, int batch, hipStream_t s);
// beta_b from the recurrence: standard  rz_new / rz_old ; flexible
// -alpha * zy / rz_old ; also rz_old := rz_new
int launch_beta(const double* rz_new, double* rz_old, const double* zy, const double* alpha,
                double* beta, int flexible, int batch, const int* active, hipStream_t s);
// x_b *= f_b for b < batch
int launch_scale_items(double* x, const double* f, int batch, hipStream_t s);
// device-side control of the PCG iteration (see k_vec.hip)
int launch_pcg_init(const double* rhs2, const double* rr, double* target2, int* active, int* claim, int* restart,
                    int* status, int* iters, double tol2, int tau_stop, int batch, hipStream_t s);
// One block per item; each first adds the item's np partial sums (fixed order).
// check: rr = ||R||^2, breakdown / non-finite / claim; live (may be null) is set
// for items whose step alpha Q of this iteration is valid
int launch_check(const double* part, int np, double* rr, const double* qy, const double* target2, int* active,
                 int* claim, int* status, int* iters, int* live, int batch, hipStream_t s);
// confirm: tr = true residual^2 of claiming items; converged or restart
int launch_confirm(const double* part, int np, double* tr, const double* target2, int* active, const int* claim,
                   int* restart, int batch, hipStream_t s);
// beta: rz_new = <R, Z>, zy = <Z, Y>; beta (0 after a restart); rz_old = rz_new
int launch_beta(const double* part_rz, const double* part_zy, int np, double* rz_new, double* zy, double* rz_old,
                const double* alpha, double* beta, int* restart, int flexible, const int* active, int batch,
                hipStream_t s);
int launch_pcg_final(const double* tr, const double* rhs2, const double* target2, const int* status,
                     const int* iters, int* iters_out, int* status_out, double* relres_out, int batch,
                     hipStream_t s);
int launch_copy_masked(const double* X, double* Y, long long n, long long xs, long long ys, int batch,
                       const int* mask, hipStream_t s);
// elementwise DIB kinetics: T_u = U + tau rho f(U, V), T_v = V + tau rho g(U, V)
int launch_dib_source(const double* U, const double* V, double* TU, double* TV, long long n,
                      long long stride, int batch, const double* kin, double tau,
                      hipStream_t s);

}  // namespace mofem
