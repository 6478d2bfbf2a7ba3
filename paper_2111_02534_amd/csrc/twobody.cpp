// The heavy-light two-body problem and the paper's procedure over binding
// energies (Sec. 2; Sec. 5.1 and 5.2): first a two-body binding energy E0 is
// chosen, then the depth v0 of the pair potential -v0 f(|xi|) is fixed by the
// generalized eigenproblem of eq. (1),
//     (-(1/(2 mu)) Lap + E0) psi = v0 F psi,   F = diag f(|xi|),
// (the smallest positive v0 gives the ground state at -E0), and the three-body
// problem is solved with that depth.  Over several E0 in decreasing order each
// three-body solve starts from the previous one's subspace (homotopy).
//
// The depth is computed on the host: v0 = 1 / mu_max, where mu_max is the
// largest eigenvalue of G = (K + E0)^{-1} F and K = -(1/(2 mu)) Lap is the
// Kronecker sum of the light-particle mode operators.  G is applied exactly in
// the eigenbases of those mode operators (two dense products per mode and a
// pointwise divide), and mu_max is found by subspace iteration with
// Rayleigh-Ritz, so no dense generalized eigensolver is needed and F (which
// underflows far out on the mapped grid) is never inverted.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dense_la.h"
#include "internal.h"

namespace tp3b {
namespace {

// splitmix64 finaliser, mapped to [-1, 1)
double unit_hash(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

struct TwoBody {
  int dims = 1;  // light-particle modes: 1 (1D) or 2 (2D)
  int n[2] = {0, 0};
  std::vector<double> S[2], Si[2], lam[2];
  std::vector<double> F;  // f(|xi|) on the grid, vector layout (mode 0 slowest)
  double E0 = 0;
  mutable std::vector<double> t1, t2;

  int64_t size() const { return dims == 1 ? n[0] : (int64_t)n[0] * n[1]; }

  // y = (K + E0)^{-1} (F o x)
  void apply(const double* x, double* y) const {
    const int64_t m = size();
    t1.resize(m);
    t2.resize(m);
    for (int64_t i = 0; i < m; ++i) t1[i] = F[i] * x[i];
    if (dims == 1) {
      const int a = n[0];
      for (int i = 0; i < a; ++i) {
        double acc = 0.0;
        for (int k = 0; k < a; ++k) acc += Si[0][(size_t)i * a + k] * t1[k];
        t2[i] = acc / (lam[0][i] + E0);
      }
      for (int i = 0; i < a; ++i) {
        double acc = 0.0;
        for (int k = 0; k < a; ++k) acc += S[0][(size_t)i * a + k] * t2[k];
        y[i] = acc;
      }
      return;
    }
    // Z = S_a [(Si_a W Si_b^T) / (lam_a,i + lam_b,j + E0)] S_b^T, W = F o X
    const int a = n[0], b = n[1];
    auto left = [&](const std::vector<double>& M, const double* in, double* out) {
      for (int i = 0; i < a; ++i)
        for (int j = 0; j < b; ++j) {
          double acc = 0.0;
          for (int k = 0; k < a; ++k) acc += M[(size_t)i * a + k] * in[(size_t)k * b + j];
          out[(size_t)i * b + j] = acc;
        }
    };
    auto right = [&](const std::vector<double>& M, const double* in, double* out) {
      for (int i = 0; i < a; ++i)
        for (int j = 0; j < b; ++j) {
          double acc = 0.0;
          for (int l = 0; l < b; ++l) acc += in[(size_t)i * b + l] * M[(size_t)j * b + l];
          out[(size_t)i * b + j] = acc;
        }
    };
    left(Si[0], t1.data(), t2.data());
    right(Si[1], t2.data(), t1.data());
    for (int i = 0; i < a; ++i)
      for (int j = 0; j < b; ++j) t1[(size_t)i * b + j] /= lam[0][i] + lam[1][j] + E0;
    left(S[0], t1.data(), t2.data());
    right(S[1], t2.data(), y);
  }
};

// Orthonormalise the p columns of Q (column-major, m rows) by two passes of
// modified Gram-Schmidt; a column that vanishes is replaced by hash values.
void orthonormalise(int64_t m, int p, std::vector<double>& Q, uint64_t salt) {
  for (int c = 0; c < p; ++c) {
    double* q = Q.data() + (size_t)c * m;
    for (int attempt = 0; attempt < 3; ++attempt) {
      double n0 = 0.0;
      for (int64_t r = 0; r < m; ++r) n0 += q[r] * q[r];
      for (int pass = 0; pass < 2; ++pass)
        for (int d = 0; d < c; ++d) {
          const double* u = Q.data() + (size_t)d * m;
          double h = 0.0;
          for (int64_t r = 0; r < m; ++r) h += u[r] * q[r];
          for (int64_t r = 0; r < m; ++r) q[r] -= h * u[r];
        }
      double nn = 0.0;
      for (int64_t r = 0; r < m; ++r) nn += q[r] * q[r];
      if (nn > 1e-20 * n0 && nn > 0.0) {
        const double s = 1.0 / std::sqrt(nn);
        for (int64_t r = 0; r < m; ++r) q[r] *= s;
        break;
      }
      for (int64_t r = 0; r < m; ++r) q[r] = unit_hash(salt * 1000003ull + (uint64_t)c * 7919ull + r + attempt);
    }
  }
}

// Largest eigenvalue of G by subspace iteration with Rayleigh-Ritz on p
// vectors; converged when the leading Ritz value has changed by at most 1e-14
// relative in three consecutive iterations (the remaining error is then about
// 1e-14 rho / (1 - rho) for the convergence ratio rho = mu_{p+1} / mu_max).
bool largest_eigenvalue(const TwoBody& tb, double* out) {
  const int64_t m = tb.size();
  const int p = (int)std::min<int64_t>(4, m);
  std::vector<double> Q((size_t)m * p), W((size_t)m * p), Hs((size_t)p * p), wr(p), wi(p);
  for (int64_t r = 0; r < m; ++r) Q[r] = 1.0;  // the ground state has one sign
  for (int c = 1; c < p; ++c)
    for (int64_t r = 0; r < m; ++r) Q[(size_t)c * m + r] = unit_hash((uint64_t)c * 1000003ull + r);
  orthonormalise(m, p, Q, 1);
  double prev = 0.0;
  int stable = 0;
  for (int it = 0; it < 5000; ++it) {
    for (int c = 0; c < p; ++c) tb.apply(Q.data() + (size_t)c * m, W.data() + (size_t)c * m);
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < p; ++j) {
        double acc = 0.0;
        for (int64_t r = 0; r < m; ++r) acc += Q[(size_t)i * m + r] * W[(size_t)j * m + r];
        Hs[(size_t)i * p + j] = acc;
      }
    if (!real_schur(p, Hs.data(), nullptr, wr.data(), wi.data())) return false;
    double theta = wr[0];
    for (int i = 1; i < p; ++i) theta = std::max(theta, wr[i]);
    if (!std::isfinite(theta)) return false;
    Q.swap(W);
    orthonormalise(m, p, Q, 2 + (uint64_t)it);
    if (it > 0 && std::fabs(theta - prev) <= 1e-14 * std::fabs(theta))
      ++stable;
    else
      stable = 0;
    prev = theta;
    if (stable >= 3) {
      *out = theta;
      return true;
    }
  }
  return false;
}

}  // namespace
}  // namespace tp3b

using namespace tp3b;

extern "C" {

tp3b_status tp3b_two_body_depth(const tp3b_problem_desc* desc, double E0, double* v0) {
  try {
    if (!desc || !v0) return fail(TP3B_EINVAL, "tp3b_two_body_depth: null descriptor or output");
    if (desc->ndim != 1 && desc->ndim != 2) return fail(TP3B_EINVAL, "ndim must be 1 or 2");
    if (!(E0 > 0) || !std::isfinite(E0)) return fail(TP3B_EINVAL, "E0 must be positive and finite");
    if (desc->pot != TP3B_POT_GAUSS && desc->pot != TP3B_POT_GAUSS_PAPER && desc->pot != TP3B_POT_LORENTZ3)
      return fail(TP3B_ENOTSUP, "a depth is defined for the Gaussian and Lorentzian-cube shapes only");
    if (desc->pot == TP3B_POT_GAUSS && !(desc->width > 0)) return fail(TP3B_EINVAL, "width must be positive");
    if (desc->grid != TP3B_GRID_CGL && desc->grid != TP3B_GRID_MAPPED) return fail(TP3B_EINVAL, "unknown grid");
    const int nm = 2 * desc->ndim;
    const int k0 = nm / 2;  // light-particle modes k0 .. nm-1
    for (int k = k0; k < nm; ++k) {
      if (desc->n[k] < 2 || desc->n[k] > 1024)
        return fail(TP3B_EINVAL, "light-particle mode sizes must be in [2, 1024]");
      if (!(desc->L[k] > 0)) return fail(TP3B_EINVAL, "half-widths L must be positive");
      if (desc->parity[k] < -1 || desc->parity[k] > 1) return fail(TP3B_EINVAL, "parity must be -1, 0 or +1");
      if (desc->parity[k] != 0 && desc->grid != TP3B_GRID_MAPPED)
        return fail(TP3B_EINVAL, "parity half grids need TP3B_GRID_MAPPED");
    }
    const double mu = desc->mu_hl > 0 ? desc->mu_hl : 1.0;
    TwoBody tb;
    tb.dims = desc->ndim;
    tb.E0 = E0;
    std::vector<double> x[2];
    for (int d = 0; d < tb.dims; ++d) {
      const int k = k0 + d, n = desc->n[k];
      tb.n[d] = n;
      std::vector<double> D2;
      mode_grid(desc, k, D2, x[d]);
      std::vector<double> A((size_t)n * n);
      for (size_t e = 0; e < A.size(); ++e) A[e] = -(0.5 / mu) * D2[e];
      tb.S[d].resize((size_t)n * n);
      tb.Si[d].resize((size_t)n * n);
      tb.lam[d].resize(n);
      if (!eigen_decompose_real(n, A.data(), tb.S[d].data(), tb.Si[d].data(), tb.lam[d].data()))
        return fail(TP3B_ENOTSUP, "the light-particle kinetic operator has a complex spectrum");
    }
    tb.F.resize(tb.size());
    if (tb.dims == 1) {
      for (int i = 0; i < tb.n[0]; ++i)
        tb.F[i] = -pair_potential(desc->pot, std::fabs(x[0][i]), 1.0, desc->width);
    } else {
      for (int i = 0; i < tb.n[0]; ++i)
        for (int j = 0; j < tb.n[1]; ++j)
          tb.F[(size_t)i * tb.n[1] + j] =
              -pair_potential(desc->pot, std::hypot(x[0][i], x[1][j]), 1.0, desc->width);
    }
    double mu_max = 0.0;
    if (!largest_eigenvalue(tb, &mu_max)) return fail(TP3B_ENOCONV, "two-body depth iteration did not converge");
    if (!(mu_max > 0)) return fail(TP3B_ENOCONV, "no bound state for this binding energy on this grid");
    *v0 = 1.0 / mu_max;
    return TP3B_OK;
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_homotopy_solve(const tp3b_problem_desc* desc, const tp3b_problem_desc* two_body,
                                const tp3b_jdqr_opts* opts, int32_t count, const double* E0,
                                double* v0, double* evals, double* resnorm, int32_t* n_outer) {
  try {
    if (!desc || !opts || !E0) return fail(TP3B_EINVAL, "tp3b_homotopy_solve: null descriptor, options or E0");
    if (count < 1) return fail(TP3B_EINVAL, "count must be >= 1");
    if (desc->pot == TP3B_POT_TABLE) return fail(TP3B_ENOTSUP, "the depth of a tabulated potential is not defined");
    const int nev = opts->nev;
    if (nev < 1) return fail(TP3B_EINVAL, "nev must be >= 1");
    struct Buf {
      double* p = nullptr;
      ~Buf() {
        if (p) (void)hipFree(p);
      }
    } Q;
    int64_t N = 0;
    for (int i = 0; i < count; ++i) {
      double vi = 0.0;
      tp3b_status st = tp3b_two_body_depth(two_body ? two_body : desc, E0[i], &vi);
      if (st != TP3B_OK) return st;
      tp3b_problem_desc d = *desc;
      d.v0 = vi;
      if (std::isnan(desc->sigma)) d.sigma = -E0[i];  // the two-body threshold
      tp3b_op op = nullptr;
      st = tp3b_create(&d, nullptr, &op);
      if (st != TP3B_OK) return st;
      if (!Q.p) {
        double sig = 0, lm = 0;
        (void)tp3b_op_info(op, &N, &sig, &lm);
        hipError_t e = hipMalloc((void**)&Q.p, sizeof(double) * (size_t)N * nev);
        if (e != hipSuccess) {
          (void)tp3b_destroy(op);
          return hip_fail(e, "tp3b_homotopy_solve: Schur vector buffer");
        }
      }
      std::vector<double> ev(nev), rn(nev);
      tp3b_jdqr_stats js{};
      // the previous Schur vectors start the next solve; the solver copies its
      // start block before it writes its own Schur vectors to the same buffer
      st = tp3b_jdqr_solve(op, opts, i > 0 ? Q.p : nullptr, i > 0 ? nev : 0, ev.data(), Q.p, nullptr,
                           rn.data(), &js);
      (void)tp3b_destroy(op);
      if (v0) v0[i] = vi;
      if (evals) std::memcpy(evals + (size_t)i * nev, ev.data(), sizeof(double) * nev);
      if (resnorm) std::memcpy(resnorm + (size_t)i * nev, rn.data(), sizeof(double) * nev);
      if (n_outer) n_outer[i] = js.n_outer;
      if (st != TP3B_OK) return st;
    }
    return TP3B_OK;
  } catch (...) {
    return exception_status();
  }
}

}  // extern "C"
