// Small dense host linear algebra used at set-up and for the eigensolver's
// projected problems: Householder Hessenberg reduction, Francis double-shift QR
// to real Schur form, reordering, eigenvectors of triangular factors, LU
// inverse and small least squares.  No LAPACK is assumed on the target system,
// so these are written out here (Golub & Van Loan, "Matrix Computations",
// Sec. 7.4-7.6, restated).
#include "dense_la.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

namespace tp3b {

static inline double sgn(double a, double b) { return b >= 0 ? std::fabs(a) : -std::fabs(a); }

// Reduce A (row-major n x n) to upper Hessenberg form H = Z^T A Z in place,
// accumulating the orthogonal Z (row-major, may be null).
void hessenberg(int n, double* A, double* Z) {
  if (Z) {
    std::memset(Z, 0, sizeof(double) * n * n);
    for (int i = 0; i < n; ++i) Z[i * n + i] = 1.0;
  }
  std::vector<double> v(n), w(n);
  for (int k = 0; k < n - 2; ++k) {
    // Householder vector annihilating A[k+2..n-1][k].
    double alpha = 0.0;
    for (int i = k + 1; i < n; ++i) alpha += A[i * n + k] * A[i * n + k];
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    double x0 = A[(k + 1) * n + k];
    double beta = -sgn(alpha, x0);
    for (int i = k + 1; i < n; ++i) v[i] = A[i * n + k];
    v[k + 1] -= beta;
    double vnorm2 = 0.0;
    for (int i = k + 1; i < n; ++i) vnorm2 += v[i] * v[i];
    if (vnorm2 == 0.0) continue;
    double tau = 2.0 / vnorm2;
    // A <- (I - tau v v^T) A : rows k+1.., all columns k..n-1
    for (int j = k; j < n; ++j) w[j] = 0.0;
    for (int i = k + 1; i < n; ++i) {
      double vi = v[i];
      const double* row = A + (size_t)i * n;
      for (int j = k; j < n; ++j) w[j] += vi * row[j];
    }
    for (int i = k + 1; i < n; ++i) {
      double s = tau * v[i];
      double* row = A + (size_t)i * n;
      for (int j = k; j < n; ++j) row[j] -= s * w[j];
    }
    // A <- A (I - tau v v^T) : all rows, columns k+1..
    for (int i = 0; i < n; ++i) {
      double* row = A + (size_t)i * n;
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += row[j] * v[j];
      s *= tau;
      for (int j = k + 1; j < n; ++j) row[j] -= s * v[j];
    }
    if (Z) {
      for (int i = 0; i < n; ++i) {
        double* row = Z + (size_t)i * n;
        double s = 0.0;
        for (int j = k + 1; j < n; ++j) s += row[j] * v[j];
        s *= tau;
        for (int j = k + 1; j < n; ++j) row[j] -= s * v[j];
      }
    }
    for (int i = k + 2; i < n; ++i) A[i * n + k] = 0.0;
    A[(k + 1) * n + k] = beta;
  }
}

// Apply the 2x2 rotation [c s; -s c] to rows (p, q), columns lo..hi of row-major M.
static void rot_rows(int n, double* M, int p, int q, int lo, int hi, double c, double s) {
  double* rp = M + (size_t)p * n;
  double* rq = M + (size_t)q * n;
  for (int j = lo; j <= hi; ++j) {
    double a = rp[j], b = rq[j];
    rp[j] = c * a + s * b;
    rq[j] = -s * a + c * b;
  }
}
// Columns (p, q), rows lo..hi: M <- M [c -s; s c].
static void rot_cols(int n, double* M, int p, int q, int lo, int hi, double c, double s) {
  for (int i = lo; i <= hi; ++i) {
    double a = M[(size_t)i * n + p], b = M[(size_t)i * n + q];
    M[(size_t)i * n + p] = c * a + s * b;
    M[(size_t)i * n + q] = -s * a + c * b;
  }
}

// Reflector P = I - tau v v^T with v = (1, v1, v2) (or (1, v1) when nr = 2)
// applied from both sides of H on rows/cols k..k+nr-1 and to Z's columns.
static void apply_reflector(int n, double* H, double* Z, int k, int nr, const double* v,
                            double tau, int row_lo, int col_hi) {
  // left: rows k..k+nr-1, columns row_lo..n-1
  for (int j = row_lo; j < n; ++j) {
    double s = 0.0;
    for (int r = 0; r < nr; ++r) s += v[r] * H[(size_t)(k + r) * n + j];
    s *= tau;
    for (int r = 0; r < nr; ++r) H[(size_t)(k + r) * n + j] -= s * v[r];
  }
  // right: columns k..k+nr-1, rows 0..col_hi
  for (int i = 0; i <= col_hi; ++i) {
    double* row = H + (size_t)i * n;
    double s = 0.0;
    for (int r = 0; r < nr; ++r) s += row[k + r] * v[r];
    s *= tau;
    for (int r = 0; r < nr; ++r) row[k + r] -= s * v[r];
  }
  if (Z) {
    for (int i = 0; i < n; ++i) {
      double* row = Z + (size_t)i * n;
      double s = 0.0;
      for (int r = 0; r < nr; ++r) s += row[k + r] * v[r];
      s *= tau;
      for (int r = 0; r < nr; ++r) row[k + r] -= s * v[r];
    }
  }
}

// Householder reflector mapping x (length nr) onto a multiple of e1, written as
// v with v[0] = 1 and tau; returns false if x is already a multiple of e1.
static bool make_reflector(int nr, const double* x, double* v, double* tau) {
  double sig = 0.0;
  for (int r = 1; r < nr; ++r) sig += x[r] * x[r];
  if (sig == 0.0) return false;
  double alpha = std::sqrt(x[0] * x[0] + sig);
  double beta = -sgn(alpha, x[0]);
  double v0 = x[0] - beta;
  v[0] = 1.0;
  for (int r = 1; r < nr; ++r) v[r] = x[r] / v0;
  *tau = (beta - x[0]) / beta;
  return true;
}

// Standardise the 2x2 diagonal block at (p, p+1): if its eigenvalues are real,
// rotate it to upper-triangular form (updating H's full rows/columns and Z).
// Returns true if the block is (now) triangular.
static bool split_2x2(int n, double* H, double* Z, int p) {
  double a = H[(size_t)p * n + p], b = H[(size_t)p * n + p + 1];
  double c = H[(size_t)(p + 1) * n + p], d = H[(size_t)(p + 1) * n + p + 1];
  if (c == 0.0) return true;
  double hp = 0.5 * (a - d);
  double disc = hp * hp + b * c;
  if (disc < 0.0) return false;
  double z = hp + sgn(std::sqrt(disc), hp);
  double lam = d + z;  // one real eigenvalue of the block
  // Eigenvector of [[a, b], [c, d]] for lam: (lam - d, c) or (b, lam - a).
  double x0 = lam - d, x1 = c;
  if (std::fabs(x0) + std::fabs(x1) == 0.0) { x0 = b; x1 = lam - a; }
  double r = std::hypot(x0, x1);
  double cs = x0 / r, sn = x1 / r;
  // Rotation G = [cs -sn; sn cs] has first column along the eigenvector;
  // H <- G^T H G.
  rot_rows(n, H, p, p + 1, p, n - 1, cs, sn);
  rot_cols(n, H, p, p + 1, 0, std::min(p + 1, n - 1), cs, sn);
  if (Z) rot_cols(n, Z, p, p + 1, 0, n - 1, cs, sn);
  H[(size_t)(p + 1) * n + p] = 0.0;
  return true;
}

// Real Schur form of an upper Hessenberg H (row-major, overwritten by T) by the
// Francis implicit double-shift QR iteration with deflation; Z (row-major, may
// be null) is post-multiplied by the transformations.
bool schur_from_hessenberg(int n, double* H, double* Z, double* wr, double* wi) {
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int iter = 0, total = 0;
  const int max_total = 100 * std::max(n, 10);
  while (hi >= 0) {
    int l = hi;
    while (l > 0) {
      double s = std::fabs(H[(size_t)(l - 1) * n + l - 1]) + std::fabs(H[(size_t)l * n + l]);
      if (s == 0.0) {
        for (int i = 0; i <= hi; ++i) s += std::fabs(H[(size_t)i * n + hi]);
      }
      if (std::fabs(H[(size_t)l * n + l - 1]) <= eps * s) break;
      --l;
    }
    if (l > 0) H[(size_t)l * n + l - 1] = 0.0;
    if (l == hi) {
      wr[hi] = H[(size_t)hi * n + hi];
      wi[hi] = 0.0;
      --hi;
      iter = 0;
      continue;
    }
    if (l == hi - 1) {
      int p = hi - 1;
      if (split_2x2(n, H, Z, p)) {
        wr[p] = H[(size_t)p * n + p];
        wr[hi] = H[(size_t)hi * n + hi];
        wi[p] = wi[hi] = 0.0;
      } else {
        double a = H[(size_t)p * n + p], b = H[(size_t)p * n + hi];
        double c = H[(size_t)hi * n + p], d = H[(size_t)hi * n + hi];
        double re = 0.5 * (a + d);
        double im = std::sqrt(std::fabs(0.25 * (a - d) * (a - d) + b * c));
        wr[p] = wr[hi] = re;
        wi[p] = im;
        wi[hi] = -im;
      }
      hi -= 2;
      iter = 0;
      continue;
    }
    if (++total > max_total) return false;
    ++iter;
    // Shifts: eigenvalues of the trailing 2x2 block (exceptional shifts every
    // 10 iterations without deflation).
    double s, t;
    double hmm = H[(size_t)(hi - 1) * n + hi - 1], hmn = H[(size_t)(hi - 1) * n + hi];
    double hnm = H[(size_t)hi * n + hi - 1], hnn = H[(size_t)hi * n + hi];
    if (iter % 10 == 0) {
      double e = std::fabs(hnm) + std::fabs(H[(size_t)(hi - 1) * n + hi - 2]);
      double w = hnn + 0.75 * e;
      s = 2.0 * w;
      t = w * w - 0.4375 * e * e;
    } else {
      s = hmm + hnn;
      t = hmm * hnn - hmn * hnm;
    }
    // First column of (H - s1 I)(H - s2 I) restricted to rows l..l+2.
    double h00 = H[(size_t)l * n + l], h01 = H[(size_t)l * n + l + 1];
    double h10 = H[(size_t)(l + 1) * n + l], h11 = H[(size_t)(l + 1) * n + l + 1];
    double h21 = H[(size_t)(l + 2) * n + l + 1];
    double x[3];
    x[0] = h00 * h00 + h01 * h10 - s * h00 + t;
    x[1] = h10 * (h00 + h11 - s);
    x[2] = h10 * h21;
    // Chase the bulge down the active window [l, hi].  The full T is kept, so
    // left reflections act on columns to n-1 and right ones on rows from 0.
    for (int k = l; k <= hi - 2; ++k) {
      double v[3], tau;
      if (make_reflector(3, x, v, &tau)) {
        int col_lo = (k > l) ? k - 1 : l;
        int row_hi = std::min(k + 3, hi);
        apply_reflector(n, H, Z, k, 3, v, tau, col_lo, row_hi);
        if (k > l) {
          H[(size_t)(k + 1) * n + k - 1] = 0.0;
          H[(size_t)(k + 2) * n + k - 1] = 0.0;
        }
      }
      x[0] = H[(size_t)(k + 1) * n + k];
      x[1] = H[(size_t)(k + 2) * n + k];
      if (k < hi - 2) x[2] = H[(size_t)(k + 3) * n + k];
    }
    // Final 2-element reflector on rows/cols hi-1, hi.
    {
      double v[2], tau;
      int k = hi - 1;
      if (make_reflector(2, x, v, &tau)) {
        apply_reflector(n, H, Z, k, 2, v, tau, k - 1, hi);
        H[(size_t)hi * n + k - 1] = 0.0;
      }
    }
  }
  // Clean the strictly lower part below the quasi-triangular structure.
  for (int i = 2; i < n; ++i)
    for (int j = 0; j < i - 1; ++j) H[(size_t)i * n + j] = 0.0;
  return true;
}

bool real_schur(int n, double* A, double* Z, double* wr, double* wi) {
  if (n == 1) {
    wr[0] = A[0];
    wi[0] = 0.0;
    if (Z) Z[0] = 1.0;
    return true;
  }
  hessenberg(n, A, Z);
  return schur_from_hessenberg(n, A, Z, wr, wi);
}

// Swap adjacent 1x1 diagonal entries p, p+1 of an upper-triangular T with a
// Givens rotation (T <- G^T T G, Z <- Z G).
static void swap_1x1(int n, double* T, double* Z, int p) {
  double t11 = T[(size_t)p * n + p], t22 = T[(size_t)(p + 1) * n + p + 1];
  double t12 = T[(size_t)p * n + p + 1];
  double x0 = t12, x1 = t22 - t11;
  double r = std::hypot(x0, x1);
  if (r == 0.0) return;
  double cs = x0 / r, sn = x1 / r;
  rot_rows(n, T, p, p + 1, p, n - 1, cs, sn);
  rot_cols(n, T, p, p + 1, 0, p + 1, cs, sn);
  if (Z) rot_cols(n, Z, p, p + 1, 0, n - 1, cs, sn);
  T[(size_t)(p + 1) * n + p] = 0.0;
  T[(size_t)p * n + p] = t22;
  T[(size_t)(p + 1) * n + p + 1] = t11;
}

// Modified Gram-Schmidt (twice) on the columns of row-major B (n x m).
static void mgs2(int n, int m, double* B) {
  for (int j = 0; j < m; ++j) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < j; ++i) {
        double s = 0.0;
        for (int r = 0; r < n; ++r) s += B[(size_t)r * m + i] * B[(size_t)r * m + j];
        for (int r = 0; r < n; ++r) B[(size_t)r * m + j] -= s * B[(size_t)r * m + i];
      }
    }
    double s = 0.0;
    for (int r = 0; r < n; ++r) s += B[(size_t)r * m + j] * B[(size_t)r * m + j];
    s = std::sqrt(s);
    if (s > 0)
      for (int r = 0; r < n; ++r) B[(size_t)r * m + j] /= s;
  }
}

// Eigenvectors of a quasi-upper-triangular T (row-major) for each eigenvalue,
// by back substitution; returns complex vectors column-wise in X (n x n).
static void quasi_tri_eigvecs(int n, const double* T, const double* wr, const double* wi,
                              std::vector<std::complex<double>>& X) {
  typedef std::complex<double> cd;
  X.assign((size_t)n * n, cd(0, 0));
  double tnorm = 0.0;
  for (int i = 0; i < n * n; ++i) tnorm = std::max(tnorm, std::fabs(T[i]));
  const double small = 2.220446049250313e-16 * std::max(tnorm, 1e-300);
  std::vector<int> blk(n, 1);  // 2 marks the first row of a 2x2 block
  for (int i = 0; i + 1 < n; ++i)
    if (T[(size_t)(i + 1) * n + i] != 0.0) { blk[i] = 2; blk[i + 1] = 0; }
  for (int e = 0; e < n; ++e) {
    cd lam(wr[e], wi[e]);
    std::vector<cd> x(n, cd(0, 0));
    int top;
    if (blk[e] == 1) {
      x[e] = 1.0;
      top = e - 1;
    } else {
      int p = (blk[e] == 2) ? e : e - 1;
      // Null vector of the 2x2 block minus lam.
      cd a = T[(size_t)p * n + p] - lam, b = T[(size_t)p * n + p + 1];
      cd c = T[(size_t)(p + 1) * n + p], d = T[(size_t)(p + 1) * n + p + 1] - lam;
      if (std::abs(b) >= std::abs(a)) { x[p] = b; x[p + 1] = -a; }
      else { x[p] = -d; x[p + 1] = c; }
      top = p - 1;
    }
    int last = (blk[e] == 1) ? e : ((blk[e] == 2) ? e + 1 : e);
    for (int k = top; k >= 0;) {
      if (blk[k] == 0) {  // second row of a 2x2 block: solve both rows
        int p = k - 1;
        cd r0 = 0, r1 = 0;
        for (int l = k + 1; l <= last; ++l) {
          r0 += T[(size_t)p * n + l] * x[l];
          r1 += T[(size_t)k * n + l] * x[l];
        }
        cd a = T[(size_t)p * n + p] - lam, b = T[(size_t)p * n + k];
        cd c = T[(size_t)k * n + p], d = T[(size_t)k * n + k] - lam;
        cd det = a * d - b * c;
        if (std::abs(det) < small) det = small;
        x[p] = (-r0 * d + b * r1) / det;
        x[k] = (-a * r1 + c * r0) / det;
        k -= 2;
      } else {
        cd r = 0;
        for (int l = k + 1; l <= last; ++l) r += T[(size_t)k * n + l] * x[l];
        cd den = T[(size_t)k * n + k] - lam;
        if (std::abs(den) < small) den = small;
        x[k] = -r / den;
        k -= 1;
      }
    }
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) nrm += std::norm(x[i]);
    nrm = std::sqrt(nrm);
    for (int i = 0; i < n; ++i) X[(size_t)i * n + e] = x[i] / nrm;
  }
}

bool ordered_schur(int m, const double* M, double* S, double* T, int* pair_start) {
  std::vector<double> A(M, M + (size_t)m * m), Z((size_t)m * m), wr(m), wi(m);
  if (!real_schur(m, A.data(), Z.data(), wr.data(), wi.data())) return false;
  bool has_pairs = false;
  for (int i = 0; i < m; ++i) has_pairs |= (wi[i] != 0.0);
  if (!has_pairs) {
    // Bubble sort of the diagonal by Givens swaps (ascending).
    for (int pass = 0; pass < m; ++pass) {
      bool swapped = false;
      for (int p = 0; p + 1 < m; ++p) {
        if (A[(size_t)p * m + p] > A[(size_t)(p + 1) * m + p + 1]) {
          swap_1x1(m, A.data(), Z.data(), p);
          swapped = true;
        }
      }
      if (!swapped) break;
    }
    std::memcpy(S, Z.data(), sizeof(double) * m * m);
    std::memcpy(T, A.data(), sizeof(double) * m * m);
    for (int i = 0; i < m; ++i) pair_start[i] = 0;
    return true;
  }
  // Complex pairs present: eigenvectors of M = Z T Z^T, sorted by real part,
  // complex pairs as (Re, Im) columns, orthonormalised (nested spans give a
  // Schur basis), T = S^T M S.
  std::vector<std::complex<double>> X;
  quasi_tri_eigvecs(m, A.data(), wr.data(), wi.data(), X);
  std::vector<int> order(m);
  for (int i = 0; i < m; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return wr[a] < wr[b]; });
  std::vector<double> B((size_t)m * m, 0.0);
  int col = 0;
  for (int oi = 0; oi < m; ++oi) {
    int e = order[oi];
    if (wi[e] < 0.0) continue;
    // eigenvector of M: Z x
    std::vector<std::complex<double>> y(m, 0.0);
    for (int r = 0; r < m; ++r)
      for (int c = 0; c < m; ++c) y[r] += Z[(size_t)r * m + c] * X[(size_t)c * m + e];
    if (wi[e] == 0.0) {
      for (int r = 0; r < m; ++r) B[(size_t)r * m + col] = y[r].real();
      pair_start[col] = 0;
      ++col;
    } else {
      for (int r = 0; r < m; ++r) {
        B[(size_t)r * m + col] = y[r].real();
        B[(size_t)r * m + col + 1] = y[r].imag();
      }
      pair_start[col] = 1;
      pair_start[col + 1] = 0;
      col += 2;
    }
  }
  if (col != m) return false;
  mgs2(m, m, B.data());
  std::memcpy(S, B.data(), sizeof(double) * m * m);
  // T = S^T M S
  std::vector<double> MS((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int k = 0; k < m; ++k) {
      double a = M[(size_t)i * m + k];
      for (int j = 0; j < m; ++j) MS[(size_t)i * m + j] += a * S[(size_t)k * m + j];
    }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += S[(size_t)k * m + i] * MS[(size_t)k * m + j];
      T[(size_t)i * m + j] = s;
    }
  return true;
}

bool eigen_decompose_real(int n, const double* A, double* S, double* Sinv, double* lam) {
  std::vector<double> T(A, A + (size_t)n * n), Z((size_t)n * n), wr(n), wi(n);
  if (!real_schur(n, T.data(), Z.data(), wr.data(), wi.data())) return false;
  for (int i = 0; i < n; ++i)
    if (wi[i] != 0.0) return false;
  for (int i = 0; i < n; ++i) lam[i] = T[(size_t)i * n + i];
  // Eigenvectors of the upper-triangular T: X upper triangular, X[e][e] = 1.
  std::vector<double> X((size_t)n * n, 0.0);
  double tnorm = 0.0;
  for (size_t i = 0; i < (size_t)n * n; ++i) tnorm = std::max(tnorm, std::fabs(T[i]));
  const double small = 2.220446049250313e-16 * tnorm;
  for (int e = 0; e < n; ++e) {
    X[(size_t)e * n + e] = 1.0;
    double le = T[(size_t)e * n + e];
    for (int k = e - 1; k >= 0; --k) {
      double r = 0.0;
      const double* Tk = T.data() + (size_t)k * n;
      for (int l = k + 1; l <= e; ++l) r += Tk[l] * X[(size_t)l * n + e];
      double den = Tk[k] - le;
      if (std::fabs(den) < small) den = (den >= 0 ? small : -small);
      X[(size_t)k * n + e] = -r / den;
    }
  }
  // Normalise columns.
  std::vector<double> scale(n);
  for (int e = 0; e < n; ++e) {
    double s = 0.0;
    for (int k = 0; k <= e; ++k) s += X[(size_t)k * n + e] * X[(size_t)k * n + e];
    scale[e] = 1.0 / std::sqrt(s);
    for (int k = 0; k <= e; ++k) X[(size_t)k * n + e] *= scale[e];
  }
  // Xinv: inverse of the upper-triangular X by back substitution, column by column.
  std::vector<double> Xi((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    Xi[(size_t)c * n + c] = 1.0 / X[(size_t)c * n + c];
    for (int k = c - 1; k >= 0; --k) {
      double r = 0.0;
      for (int l = k + 1; l <= c; ++l) r += X[(size_t)k * n + l] * Xi[(size_t)l * n + c];
      Xi[(size_t)k * n + c] = -r / X[(size_t)k * n + k];
    }
  }
  // S = Z X, Sinv = Xinv Z^T (row-major).
  for (int i = 0; i < n; ++i) {
    double* Si = S + (size_t)i * n;
    std::fill(Si, Si + n, 0.0);
    const double* Zi = Z.data() + (size_t)i * n;
    for (int k = 0; k < n; ++k) {
      double z = Zi[k];
      const double* Xk = X.data() + (size_t)k * n;
      for (int j = k; j < n; ++j) Si[j] += z * Xk[j];
    }
  }
  for (int i = 0; i < n; ++i) {
    double* Si = Sinv + (size_t)i * n;
    const double* Xi_i = Xi.data() + (size_t)i * n;
    for (int j = 0; j < n; ++j) {
      const double* Zj = Z.data() + (size_t)j * n;
      double s = 0.0;
      for (int k = i; k < n; ++k) s += Xi_i[k] * Zj[k];
      Si[j] = s;
    }
  }
  return true;
}

bool lu_inverse(int n, const double* A, double* Ainv) {
  std::vector<double> M(A, A + (size_t)n * n);
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(M[(size_t)i * n + k]) > std::fabs(M[(size_t)p * n + k])) p = i;
    piv[k] = p;
    if (M[(size_t)p * n + k] == 0.0) return false;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(M[(size_t)k * n + j], M[(size_t)p * n + j]);
    for (int i = k + 1; i < n; ++i) {
      double f = M[(size_t)i * n + k] / M[(size_t)k * n + k];
      M[(size_t)i * n + k] = f;
      for (int j = k + 1; j < n; ++j) M[(size_t)i * n + j] -= f * M[(size_t)k * n + j];
    }
  }
  for (int c = 0; c < n; ++c) {
    std::vector<double> x(n, 0.0);
    x[c] = 1.0;
    for (int k = 0; k < n; ++k)
      if (piv[k] != k) std::swap(x[k], x[piv[k]]);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) x[i] -= M[(size_t)i * n + j] * x[j];
    for (int i = n - 1; i >= 0; --i) {
      for (int j = i + 1; j < n; ++j) x[i] -= M[(size_t)i * n + j] * x[j];
      x[i] /= M[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) Ainv[(size_t)i * n + c] = x[i];
  }
  return true;
}

void hessenberg_lstsq(int k, const double* H, int ldh, double beta, double* y) {
  // H is (k+1) x k (row-major, leading dimension ldh); minimise
  // || beta e1 - H y || by Givens rotations.
  std::vector<double> R((size_t)(k + 1) * k);
  for (int i = 0; i <= k; ++i)
    for (int j = 0; j < k; ++j) R[(size_t)i * k + j] = H[(size_t)i * ldh + j];
  std::vector<double> g(k + 1, 0.0);
  g[0] = beta;
  for (int j = 0; j < k; ++j) {
    double a = R[(size_t)j * k + j], b = R[(size_t)(j + 1) * k + j];
    double r = std::hypot(a, b);
    double c = (r == 0) ? 1.0 : a / r, s = (r == 0) ? 0.0 : b / r;
    for (int jj = j; jj < k; ++jj) {
      double u = R[(size_t)j * k + jj], v = R[(size_t)(j + 1) * k + jj];
      R[(size_t)j * k + jj] = c * u + s * v;
      R[(size_t)(j + 1) * k + jj] = -s * u + c * v;
    }
    double u = g[j], v = g[j + 1];
    g[j] = c * u + s * v;
    g[j + 1] = -s * u + c * v;
  }
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int j = i + 1; j < k; ++j) s -= R[(size_t)i * k + j] * y[j];
    double d = R[(size_t)i * k + i];
    y[i] = (d != 0.0) ? s / d : 0.0;
  }
}

}  // namespace tp3b
