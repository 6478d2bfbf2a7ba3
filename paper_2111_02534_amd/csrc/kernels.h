// Device kernels of the tensor-product three-body library (gfx950) and their
// host launchers.  All launchers are stream-ordered and return hipError_t.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tp3b {

enum Epi { EPI_NONE = 0, EPI_V = 1, EPI_DIV = 2 };

// One strided, batched mode product (Sec. 3.2-3.3): for every batch item q
// (vector vec = q / per_vec, item = q % per_vec) with
//   Xq = X + vec*ldx + item*bstride,  element (i, j) at Xq[i*rs + j],
// computes   Y = [L Xq] + [Xq R] (+ epilogue)   with L an M x M and R an
// Nc x Nc row-major operator (either may be absent), and the epilogue
//   EPI_V:   + (V[item*bstride + i*rs + j] - shift[vec]) * Xq[i, j]
//   EPI_DIV: / (lamL[i] + lamR[j] + lamItem[item] - sigma)   (lamItem optional)
// optionally accumulated into Y (acc != 0).
template <typename T>
struct ModeProd {
  int M, Nc;
  int64_t rs, bstride, ldx, ldy;
  int per_vec, nbatch;
  const T* X;
  T* Y;
  const T* L;
  const T* R;
  const T* V;
  const double* shifts;
  const T* lamL;
  const T* lamR;
  const T* lamItem;
  double sigma;
  int epi;
  int acc;
  // BF16x3 only (optional): the constant operands split into bf16 hi and lo
  // once (raw bits, the n x n hi block followed by the lo block): L in its own
  // layout and R transposed (k contiguous), as launch_bf3_split writes them.
  // NULL: the operand is split while it is staged.
  const unsigned short* Lhl;
  const unsigned short* Rhl;
};

// Tile configurations (output tile TM x TN per 256-thread workgroup; the
// 32 x 32 tiles split the K range over their waves, TILE_32W8 over eight waves
// of a 512-thread workgroup).
enum TileCfg {
  TILE_32 = 0,
  TILE_64 = 1,
  TILE_128 = 2,
  TILE_64x128 = 3,
  TILE_32W8 = 4,
  NUM_TILE_CFGS = 5
};
inline int tile_rows(int tile) { return (tile == TILE_32 || tile == TILE_32W8) ? 32 : (tile == TILE_128 ? 128 : 64); }
inline int tile_cols(int tile) {
  return (tile == TILE_32 || tile == TILE_32W8) ? 32 : ((tile == TILE_64) ? 64 : 128);
}

// Optional kernel timestamps for the mode-product launches of the calling
// thread.  While launch_timing() points at a LaunchTiming, the first launch
// records `start` when it begins and every launch records `stop` when it ends,
// so the pair spans the launch group without any dispatch gap before it.
// Launches that are being captured into a graph must not be timed.
struct LaunchTiming {
  hipEvent_t start = nullptr, stop = nullptr;
  bool started = false;
};
LaunchTiming*& launch_timing();

template <typename T>
hipError_t launch_modeprod(const ModeProd<T>& a, int tile, hipStream_t s);
// The same product on FP32 data with BF16x3 split products on the bf16 matrix
// cores (FP32 accumulation); tiles TILE_32 and TILE_32W8 run as TILE_64.
hipError_t launch_modeprod_bf3(const ModeProd<float>& a, int tile, hipStream_t s);
// Splits the n x n FP32 matrix A (row-major) into bf16 hi and lo, each element
// as the BF16x3 kernels split it while staging (hi = bf16(a), lo = bf16(a - hi)):
// out[0, n^2) = hi, out[n^2, 2 n^2) = lo, element (i, k) at i n + k, with
// (i, k) of A itself or, with transpose, of A^T.
hipError_t launch_bf3_split(int n, const float* A, int transpose, unsigned short* out, hipStream_t s);

// C (p x q, column-major, ldc) = A^T B, A: N x p (lda), B: N x q (ldb), FP64
// accumulation; `partial` is device scratch of at least dot_scratch_doubles().
template <typename TA, typename TB>
hipError_t launch_dot_tn(int64_t N, int p, int q, const TA* A, int64_t lda, const TB* B,
                         int64_t ldb, double* C, int ldc, double* partial, hipStream_t s);
int64_t dot_scratch_doubles(int64_t N, int p, int q);

// Y (N x q, ldy) = beta Y + alpha A (N x p, lda) C (p x q column-major, ldc,
// device doubles).  Y must not alias A.
template <typename T>
hipError_t launch_gemm_nn(int64_t N, int p, int q, double alpha, const T* A, int64_t lda,
                          const double* C, int ldc, double beta, T* Y, int64_t ldy,
                          hipStream_t s);

// Y (N x q, ldy) = beta X0 + alpha A C with X0 (N x q, ldx0) a separate input
// that Y does not alias (X0 == nullptr: as launch_gemm_nn).
template <typename T>
hipError_t launch_gemm_nn_x0(int64_t N, int p, int q, double alpha, const T* A, int64_t lda,
                             const double* C, int ldc, double beta, const T* X0, int64_t ldx0, T* Y,
                             int64_t ldy, hipStream_t s);

// U (N x nu, ldo) = V S and R (N x nb, ldo) = (A V) S[:, :nb] - U T for long
// blocks (N >= 2^20), V and A V N x m (ld), S m x nu and T nu x nb column-major
// device matrices; m <= 128, nb <= 16, nu <= nb + 1.  Equals the three
// products V S, (A V) S[:, :nb], A U - U T bit for bit.  hipErrorInvalidValue
// outside those limits (the caller then runs the products).
hipError_t launch_urres_long(int64_t N, int m, int nu, int nb, const double* V, const double* AV,
                             int64_t ld, const double* S, const double* Tm, double* U, double* R,
                             int64_t ldo, hipStream_t s);

// Xout = Xin - Q C (Q N x nq, C nq x nx column-major on the device, Xin and
// Xout N x nx with ld ldx; Xin may equal Xout) fused with the dot on the
// updated rows: D (ldd) = Q^T Xout (self = 0, nq x nx) or Xout^T Xout
// (self = 1, nx x nx); `partial` as for launch_dot_tn with that dot's shape.
// Long FP64 blocks only (N >= 2^20, nq <= 80, nx <= 16, 16-byte aligned
// operands, even leading dimensions); hipErrorInvalidValue otherwise (the
// caller then runs the update and the dot); gemm_dot_long_fits tells which.
bool gemm_dot_long_fits(int64_t N, int nq, int nx, const double* Q, int64_t ldq, const double* Xin,
                        const double* Xout, int64_t ldx);
hipError_t launch_gemm_dot_long(int64_t N, int nq, int nx, const double* Q, int64_t ldq,
                                const double* C, const double* Xin, double* Xout, int64_t ldx,
                                int self, double* D, int ldd, double* partial, hipStream_t s);

// A[:, :q] = A C in place (A N x p, C p x q column-major on the device, q <= p)
// for long FP64 blocks: N >= 2^20, p <= 128, q <= 64; each row is read whole
// by the thread that then writes it.  hipErrorInvalidValue outside those
// limits.
hipError_t launch_gemm_nn_rows_inplace(int64_t N, int p, int q, double* A, int64_t lda,
                                       const double* C, int ldc, hipStream_t s);

// Batched per-column dots for b independent Krylov bases stored as blocks
// Vb[i] = V + i*bs (each N x b, ld N):  H[j*hld + i] = sum_r Vb[i][r, j] W[r, j]
// for i < nb.  `partial` as for the dot.
template <typename T>
hipError_t launch_bdot_diag(int64_t N, int b, int nb, const T* V, int64_t bs, const T* W,
                            double* H, int hld, double* partial, hipStream_t s);
int64_t bdot_scratch_doubles(int64_t N, int b, int nb);
// GMRES least squares for nb correction columns on the device: from the
// Arnoldi coefficients H1, H2 ([kk*b*hld + j*hld + i], two Gram-Schmidt
// passes), the subdiagonal norms Hs[kk*b + j] and the initial norms Beta[j],
// Y[j*hld + i] = argmin || Beta_j e1 - H_j y || (zero past the first
// breakdown).  steps <= GL_MAXSTEPS.
constexpr int GL_MAXSTEPS = 38;
hipError_t launch_gmres_lstsq(int nb, int b, int steps, int hld, const double* H1, const double* H2,
                              const double* Hs, const double* Beta, double* Y, hipStream_t s);
// Ainv = A^{-1} for an n x n column-major matrix, n <= SI_MAXN (Gauss-Jordan
// with partial pivoting, one wavefront); *singular = 1 on an exactly zero pivot.
constexpr int SI_MAXN = 48;
hipError_t launch_small_inverse(int n, const double* A, double* Ainv, int* singular, hipStream_t s);
// Out[r, j] = alpha * sum_{i<nb} Vb[i][r, j] H[j*hld + i] (assigned, column
// stride ldo, stored in the output type)
template <typename T, typename TO>
hipError_t launch_bcombine(int64_t N, int b, int nb, double alpha, const T* V, int64_t bs,
                           const double* H, int hld, TO* Out, int64_t ldo, hipStream_t s);

// The Arnoldi steps with the dots' second stage folded into their consumer:
// launch_bdot_partials runs only the first stage of launch_bdot_diag into
// `partial`; launch_bupdate_diag_red then sums those partials per column (the
// same order as launch_bdot_diag), stores them to H[j*hld + i] and applies
// W[r, j] += alpha * sum_i Vb[i][r, j] H[j*hld + i]; launch_normalize_cols_red
// sums the partials of a squared norm (nb = 1) and writes
// Vout[:, j] = W[:, j] / sqrt(nrm2_j) (0 if the norm is not positive) and
// hout[j*hld] = sqrt(nrm2_j).
// Results equal those of the unfused sequence bit for bit.
template <typename T>
hipError_t launch_bdot_partials(int64_t N, int b, int nb, const T* V, int64_t bs, const T* W,
                                double* partial, hipStream_t s);
template <typename T>
hipError_t launch_bupdate_diag_red(int64_t N, int b, int nb, double alpha, const T* V, int64_t bs,
                                   const double* partial, double* H, int hld, T* W, hipStream_t s);
template <typename T>
hipError_t launch_normalize_cols_red(int64_t N, int b, const double* partial, const T* W, T* Vout,
                                     double* hout, int hld, hipStream_t s);

// One Arnoldi update fused with the dots that follow it (long blocks).
// Sums the column's partials of the preceding dots (`part_in`, written by
// launch_bdot_partials when nchunk_in == 0, else by this launch with
// nchunk_in = bupdate_dot_chunks(N)), stores them to H and applies
// W[r, j] += alpha * sum_{i<nb} Vb[i][r, j] H[j*hld + i] as
// launch_bupdate_diag_red does; then, on the updated rows, the partials of
// the next dots into `part_out`: with Vb[i] for i < nb when `self` is 0 (the
// second Gram-Schmidt pass), or W[:, j] with itself when `self` is 1 (the
// squared norm).  The consumer of `part_out` takes nchunk =
// bupdate_dot_chunks(N).  part_out must not overlap part_in.  nb <= BDF_MAXNB.
constexpr int BDF_MAXNB = 16;
int bupdate_dot_chunks(int64_t N);
int64_t bupdate_dot_scratch_doubles(int64_t N, int b);
template <typename T>
hipError_t launch_bupdate_dot_red(int64_t N, int b, int nb, double alpha, const T* V, int64_t bs,
                                  const double* part_in, int nchunk_in, double* H, int hld, T* W,
                                  int self, double* part_out, hipStream_t s);
// launch_bupdate_diag_red / launch_normalize_cols_red with the partials of a
// launch_bupdate_dot_red (nchunk = bupdate_dot_chunks(N)).
template <typename T>
hipError_t launch_normalize_cols_red_n(int64_t N, int b, const double* partial, int nchunk,
                                       const T* W, T* Vout, double* hout, int hld, hipStream_t s);

// Y[:, j] = alpha * X[:, j] (type conversion included); X == nullptr: Y = 0.
template <typename TI, typename TO>
hipError_t launch_convert(int64_t N, int ncol, double alpha, const TI* X, int64_t ldx, TO* Y,
                          int64_t ldy, hipStream_t s);

// Cholesky of the nx x nx Gram matrix G (column-major): R upper, flags[j] = 1
// where the pivot falls below (drop_tol * norm0[j])^2.  A flagged column gets a
// unit pivot and a zero row, so it is left unscaled and the other columns are
// factored as if it were absent.  skip (device, nx ints, optional): columns
// with skip[j] != 0 are treated as flagged (the second factorisation of a
// Cholesky-QR pair passes the first one's flags).  One wavefront.
hipError_t launch_chol_small(int nx, const double* G, const double* norm0sq, double drop_tol,
                             double* R, int* flags, hipStream_t s, const int* skip = nullptr);
// n0[j] = G[j + j nx] for j < nx (the diagonal of a Gram matrix); flag[0] = 1 if
// any of them is not finite, 0 otherwise.  Single thread.
hipError_t launch_gram_diag(int nx, const double* G, double* n0, int* flag, hipStream_t s);
// X (N x nx) <- X R^{-1} for upper-triangular R (column-major nx x nx).
hipError_t launch_trsm_right(int64_t N, int nx, const double* R, double* X, int64_t ldx,
                             hipStream_t s);
// Fill column `col` of X with counter-based pseudo-random values in [-1, 1).
hipError_t launch_hash_fill(int64_t N, double* X, uint64_t seed, uint64_t stream_id,
                            hipStream_t s);
// flag[0] |= 1 if any entry of the N x ncol block is not finite.
template <typename T>
hipError_t launch_check_finite(int64_t N, int ncol, const T* X, int64_t ldx, int* flag,
                               hipStream_t s);

}  // namespace tp3b

namespace tp3b {

// ------------------------------------------------ 2D passes on LDS-resident planes
// The four-mode operators of eq. (8) act on 64 x 64 (or smaller) matrices cut
// from the tensor: a y plane W_p[j1][j2] at fixed (x1, x2), or an x slab
// W_j[i1][i2] at a fixed flattened y index j.  One workgroup holds a group of
// J = 16 / sizeof(T) such matrices in LDS and applies a short program of mode
// products to each of them with the constant n x n factors read in MFMA
// fragment order (see plane2d_fragments), so that a whole 2D apply is two
// passes over HBM and the 2D kinetic preconditioner three or four.
//   P2_SUM        Out = A W + W B^T
//   P2_SUM_V_ACC  Out = A W + W B^T + (V - shift_v) o W + Y   (Y read in place)
//   P2_SEQ2       Out = (A W) B^T
//   P2_SEQ2_DIV   Out = [(A W) B^T] / (lamM[m] + lamR[r] + lamC[c] - sigma)
//   P2_SEQ4_DIV   Out = C ([(A W) A^T] / (lamM[m] + lamR[r] + lamC[c] - sigma)) C^T
//                 with A = FA1 and C = FA2 (x slabs with equal x modes, FP64)
// Matrices that are x slabs (interleaved layout) take P2_SUM, P2_SEQ2 and
// P2_SEQ4_DIV.
enum Plane2DProg { P2_SUM = 0, P2_SUM_V_ACC = 1, P2_SEQ2 = 2, P2_SEQ2_DIV = 3, P2_SEQ4_DIV = 4 };
constexpr int P2_MAXN = 64;

template <typename T>
struct Plane2D {
  int prog;         // Plane2DProg
  int interleaved;  // 0: matrix m at m * js with rs = row stride, cs = 1 (y planes);
                    // 1: the J matrices of a group are consecutive elements (js = 1)
  int M, Nc;        // rows and columns of every matrix, each <= P2_MAXN
  int64_t rs, cs, js;
  int64_t nmat;     // matrices per vector
  int nvec;
  int64_t ldx, ldy;
  const T* X;
  T* Y;
  const T* FA1;     // fragments of A and B (P2_FRAG elements each)
  const T* FB1;
  const T* FA2;     // P2_SEQ4_DIV: fragments of the second factor (both sides)
  int same_ab;      // A and B are the same matrix (equal modes): one LDS copy serves both
  // P2_SUM_V_ACC: the potential from a table in vector layout (V), or, when G is
  // set, from separable Gaussian factors:
  //   V = gscale (G[0][i1][r] G[2][i2][c] + G[1][i1][r] G[3][i2][c]),
  // with i1 = m / mdiv, i2 = m % mdiv and each G[k] 64 x 64 row-major.
  const T* V;
  const T* G;
  int mdiv;
  double gscale;
  const double* shifts;  // device, one per vector, or NULL
  // P2_SEQ2_DIV
  const T* lamM;
  const T* lamR;
  const T* lamC;
  double sigma;
};

// Elements of one fragment array: F[(blk * 16 + kk) * 64 + lane] =
// A[blk * 16 + lane % 16][4 kk + lane / 16], zero outside n x n.
constexpr int P2_FRAG = 64 * 64;
void plane2d_fragments(int n, const double* A_rowmajor, double* frag_out);

template <typename T>
hipError_t launch_plane2d(const Plane2D<T>& a, hipStream_t s);

}  // namespace tp3b

namespace tp3b {

// The static device scratch of the allocation-free entry point (noalloc.hip):
// kStaticScratchDoubles doubles (16.25 MiB) per device.  static_scratch()
// returns its device address on the current device.
constexpr int64_t kStaticScratchDoubles = ((int64_t)1 << 21) + ((int64_t)1 << 15);
hipError_t static_scratch(double** out);

}  // namespace tp3b
