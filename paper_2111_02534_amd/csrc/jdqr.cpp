// Block Jacobi-Davidson QR (Sec. 4.1, eqs. (12)-(13)) with preconditioned
// GMRES on the correction equation (Sec. 4.1-4.2).
//
// Everything of size N lives on the device; the host holds only the projected
// m x m problem, the small Hessenberg least-squares problems and the partial
// Schur factor R.  One outer iteration:
//   1. ordered real Schur form of M = V^T A V (host), V and AV rotated to it;
//   2. partial-Schur residuals of the leading b Schur vectors (FP64);
//   3. locking of the converged prefix, restart to m_min vectors at m_max;
//   4. b correction equations (eq. (13)) with Q~ = [Q_lock, u_1..u_b] solved by
//      left-preconditioned GMRES with the skew projection
//      (I - Y H^{-1} Q~^T) P^{-1}, Y = P^{-1} Q~, H = Q~^T Y, a fixed number of
//      steps, in the inner working precision (FP64, FP32, or FP32 storage with
//      BF16x3 split mode products);
//   5. FP64 block orthogonalisation of the corrections against [Q_lock, V] and
//      FP64 products with A to extend V and A V.
// Rayleigh-Ritz, residuals, locking and orthogonalisation are always FP64, so
// the converged pairs meet the FP64 residual tolerance whatever the inner
// precision.
#include <algorithm>
#include <type_traits>
#include <utility>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "dense_la.h"
#include "internal.h"

namespace tp3b {

namespace {

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  template <typename T>
  T* as() const {
    return (T*)p;
  }
};

hipError_t dalloc(DevBuf& b, size_t bytes) { return hipMalloc(&b.p, bytes ? bytes : 8); }

// Copy the (r0.., c0..) nr x nc sub-block of a row-major host matrix (ld cols)
// into a column-major host array with leading dimension nr.
std::vector<double> colmajor(const std::vector<double>& A, int ld, int r0, int c0, int nr, int nc) {
  std::vector<double> out((size_t)nr * nc);
  for (int j = 0; j < nc; ++j)
    for (int i = 0; i < nr; ++i) out[i + (size_t)j * nr] = A[(size_t)(r0 + i) * ld + (c0 + j)];
  return out;
}

// Optional timing of the mode-product launches inside the solve with kernel
// timestamp events (LaunchTiming): kind 0 = FP64 Hamiltonian applies, 1 =
// low-precision Hamiltonian applies, 2 = FP64 preconditioner applies, 3 =
// low-precision preconditioner applies.  Launches inside a captured graph are
// not timed (paused).
struct KernelTimer {
  bool on = false, paused = false;
  std::vector<hipEvent_t> ev;  // pairs (2i, 2i+1) bracket one launch group
  std::vector<int> kind, nvec;
  size_t used = 0;
  LaunchTiming lt;
  hipError_t begin(int k, int nv) {
    if (!on || paused) return hipSuccess;
    while (ev.size() < used + 2) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      ev.push_back(e);
      kind.push_back(-1);
      nvec.push_back(0);
    }
    kind[used] = k;
    nvec[used] = nv;
    lt.start = ev[used];
    lt.stop = ev[used + 1];
    lt.started = false;
    launch_timing() = &lt;
    used += 2;
    return hipSuccess;
  }
  void end() {
    if (launch_timing() == &lt) launch_timing() = nullptr;
  }
  void collect(double* t, int64_t* n, int64_t* v) {
    for (size_t i = 0; i + 1 < used; i += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) {
        t[kind[i]] += 1e-3 * ms;
        n[kind[i]] += 1;
        v[kind[i]] += nvec[i];
      }
    }
  }
  ~KernelTimer() {
    end();
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// The solve's own stream and the GMRES graphs captured on it.  A graph is
// keyed by what its kernel arguments depend on: the projection width, the
// number of correction columns and the reduction scratch address (which moves
// when the scratch grows).
struct SolveGraphs {
  struct Entry {
    int nqt, nb;
    const double* part;
    hipGraph_t g;
    hipGraphExec_t x;
    int64_t dH64, dHlow, dPrec;  // apply counts of one replay
  };
  hipStream_t s = nullptr;
  std::vector<Entry> e;
  Entry* find(int nqt, int nb, const double* part) {
    for (Entry& x : e)
      if (x.nqt == nqt && x.nb == nb && x.part == part) return &x;
    return nullptr;
  }
  void drop_stale(const double* part) {
    std::vector<Entry> keep;
    for (Entry& x : e) {
      if (x.part == part) {
        keep.push_back(x);
      } else {
        (void)hipGraphExecDestroy(x.x);
        (void)hipGraphDestroy(x.g);
      }
    }
    e.swap(keep);
  }
  ~SolveGraphs() {
    if (s) (void)hipStreamSynchronize(s);
    for (Entry& x : e) {
      (void)hipGraphExecDestroy(x.x);
      (void)hipGraphDestroy(x.g);
    }
    if (s) (void)hipStreamDestroy(s);
  }
};

}  // namespace

template <typename TW>
static tp3b_status jdqr_run(tp3b_op op, const tp3b_jdqr_opts& o, const double* X0, int b0,
                            double* evals, double* Qout, double* Rout, double* resnorm,
                            tp3b_jdqr_stats* st, bool bf3) {
  const double t_start = now();
  // The solve runs on a stream of its own; the caller's pending work (which
  // may have produced X0) completes first.
  SolveGraphs graphs;
  TP3B_HIP(hipDeviceSynchronize());
  TP3B_HIP(hipStreamCreateWithFlags(&graphs.s, hipStreamNonBlocking));
  hipStream_t s = graphs.s;
  const int64_t N = op->N;
  const int nev = o.nev, b = o.block, steps = o.gmres_steps;
  const int m_max = o.m_max, m_min = o.m_min;
  const bool use_prec = o.precond != 0;
  const bool low = sizeof(TW) == 4;
  const double target = std::isnan(o.target) ? op->sigma : o.target;
  tp3b_jdqr_stats stats{};
  KernelTimer kt;
  kt.on = o.profile != 0;

  // ---- device buffers
  const int qv_cols = nev + m_max + b;
  const int av_cols = m_max + b + nev;
  const int qt_max = nev + b;
  DevBuf QVb, AVb, TMPb, Rresb, PQb, Ypb, Qtwb, Ypwb, Vgb, Wb, Zb, Tcb, smallb, Qtb, AUb;
  TP3B_HIP(dalloc(QVb, sizeof(double) * N * qv_cols));
  // Q~ = [Q_lock, U] contiguous (U = V s_1..s_nb, plus one column for the
  // residual when a 2 x 2 block straddles the block edge), and A U
  TP3B_HIP(dalloc(Qtb, sizeof(double) * N * (qt_max + 1)));
  // long blocks form the residuals in one pass over V and A V (A U is not stored)
  const bool urres_fused = N >= (1 << 20) && m_max + b <= 128 && b <= 16;
  if (!urres_fused) TP3B_HIP(dalloc(AUb, sizeof(double) * N * b));
  TP3B_HIP(dalloc(AVb, sizeof(double) * N * av_cols));
  // long blocks rotate V and A V in place (the search space never holds more
  // than m_max <= 64 columns there); the others through a scratch basis of
  // A V's capacity, the two swapping roles after a rotation
  const bool rot_inplace = N >= (1 << 20) && m_max <= 64;
  if (!rot_inplace) TP3B_HIP(dalloc(TMPb, sizeof(double) * N * av_cols));
  TP3B_HIP(dalloc(Rresb, sizeof(double) * N * b));
  if (use_prec) {
    TP3B_HIP(dalloc(PQb, sizeof(double) * N * qt_max));
    TP3B_HIP(dalloc(Ypb, sizeof(double) * N * qt_max));
  }
  if (low) {
    TP3B_HIP(dalloc(Qtwb, sizeof(TW) * N * qt_max));
    TP3B_HIP(dalloc(Ypwb, sizeof(TW) * N * qt_max));
  }
  TP3B_HIP(dalloc(Vgb, sizeof(TW) * N * b * (steps + 1)));
  TP3B_HIP(dalloc(Wb, sizeof(TW) * N * b));
  TP3B_HIP(dalloc(Zb, sizeof(TW) * N * b));
  TP3B_HIP(dalloc(Tcb, sizeof(double) * N * b));
  // Pinned host staging for the small transfers of an outer iteration: copies
  // to and from pinned memory are asynchronous, so uploads do not wait for the
  // stream and a group of read-backs costs one synchronisation.  Every transfer
  // site has a region of its own, rewritten only after a stream
  // synchronisation that follows its previous copy.
  struct PinnedHost {
    double* p = nullptr;
    ~PinnedHost() {
      if (p) (void)hipHostFree(p);
    }
  } pin;
  size_t pin_used = 0;
  auto region = [&](size_t n) {
    const size_t o = pin_used;
    pin_used += (n + 7) & ~(size_t)7;
    return o;
  };
  const size_t mb = (size_t)(m_max + b), big = (size_t)(qt_max + m_max + b);
  const size_t r_upS = region(mb * mb), r_upT = region(mb * b), r_upShift = region(b),
               r_upHinv = region((size_t)qt_max * qt_max), r_dnM = region(big * big),
               r_dnC1 = region((size_t)nev * b), r_dnC2 = region((size_t)nev * b),
               r_dnRn = region(b), r_dnTop = region(mb * b), r_dnLeft = region(mb * b),
               r_dnFlag = region(1), r_dnOFlags = region(b + 1);
  TP3B_HIP(hipHostMalloc((void**)&pin.p, sizeof(double) * pin_used, hipHostMallocDefault));
  auto P = [&](size_t r) { return pin.p + r; };
  // Declared after the buffers, so destroyed before them: on every return the
  // solve's stream has finished with them before they are freed.
  struct StreamDrain {
    hipStream_t s;
    ~StreamDrain() { (void)hipStreamSynchronize(s); }
  } drain{s};
  // small device arrays (doubles)
  const int hld = steps + 2;
  const size_t n_small = (size_t)(m_max + b) * (m_max + b) * 2 + (size_t)qt_max * qt_max +
                         (size_t)qt_max * b * 2 + (size_t)steps * b * hld * 2 + (size_t)steps * b +
                         (size_t)b * 4 + (size_t)hld * b + (size_t)b + (size_t)(b + 1) * b + 64;
  TP3B_HIP(dalloc(smallb, sizeof(double) * n_small));
  double* QV = QVb.as<double>();
  double* Qt = Qtb.as<double>();
  double* AU = AUb.as<double>();
  double* AVbase = AVb.as<double>();
  double* TMP = TMPb.as<double>();
  double* Rres = Rresb.as<double>();
  double* PQ = PQb.as<double>();
  double* Yp = Ypb.as<double>();
  TW* Vg = Vgb.as<TW>();
  TW* W = Wb.as<TW>();
  TW* Zt = Zb.as<TW>();
  double* Tc = Tcb.as<double>();
  double* dS = smallb.as<double>();                                  // (m_max+b)^2
  double* dM2 = dS + (size_t)(m_max + b) * (m_max + b);              // (m_max+b)^2
  double* dHinv = dM2 + (size_t)(m_max + b) * (m_max + b);           // qt_max^2
  double* dC = dHinv + (size_t)qt_max * qt_max;                      // qt_max*b
  double* dC2 = dC + (size_t)qt_max * b;                             // qt_max*b
  double* dH1 = dC2 + (size_t)qt_max * b;                            // steps*b*hld
  double* dH2 = dH1 + (size_t)steps * b * hld;                       // steps*b*hld
  double* dHs = dH2 + (size_t)steps * b * hld;                       // steps*b
  double* dShift = dHs + (size_t)steps * b;                          // b
  double* dNrm = dShift + b;                                         // b
  double* dBeta = dNrm + b;                                          // b
  double* dY = dBeta + 2 * b;                                        // b*hld
  double* dTb = dY + (size_t)b * hld;                                // (b+1)*b
  int* dFlag = (int*)(dTb + (size_t)(b + 1) * b);  // singular projected preconditioner
  int* dOFlags = dFlag + 2;                    // expansion block: b dependence flags, non-finite
  TP3B_HIP(hipMemsetAsync(dFlag, 0, sizeof(int), s));
  // long blocks: the Arnoldi updates are fused with the dots that follow them
  // (two partial areas: the pass-1 dots and the norm in the first, the
  // pass-2 dots in the second)
  const bool arn_fused = N >= (int64_t)(1 << 20) && steps + 1 <= BDF_MAXNB;
  const int64_t part_b_off =
      std::max(bdot_scratch_doubles(N, b, 1), bupdate_dot_scratch_doubles(N, b));
  const int nch_f = bupdate_dot_chunks(N);
  const int64_t dscr = dot_scratch_doubles(N, qt_max + m_max + b, qt_max + m_max + b) +
                       bdot_scratch_doubles(N, b, steps + 2) + 8 * (int64_t)(qv_cols + 1) * b +
                       2 * bupdate_dot_scratch_doubles(N, b) +
                       8 * (int64_t)b * b + 1024;
  double* part = dot_scratch(dscr);
  if (!part) return fail(TP3B_ENOMEM, "jdqr: scratch allocation failed");

  int k = 0;      // locked vectors: QV[:, 0:k]
  int m = 0;      // search space: QV[:, k:k+m], A V in AV[:, 0:m]
  int av0 = 0;    // column offset of A V inside its buffer
  std::vector<double> Rl;          // partial Schur factor, column-major nev x nev
  Rl.assign((size_t)nev * nev, 0.0);
  std::vector<double> lockres;
  std::vector<int> lock_pair;
  std::vector<double> M;           // row-major m x m projected matrix

  auto V = [&]() { return QV + (int64_t)k * N; };
  auto AV = [&]() { return AVbase + (int64_t)av0 * N; };
  auto applyA64 = [&](int nv, const double* X, double* Y) -> tp3b_status {
    stats.n_apply_H_fp64 += nv;
    TP3B_HIP(kt.begin(0, nv));
    tp3b_status r = apply_H_impl<double>(op, nv, X, N, Y, N, nullptr, s);
    kt.end();
    return r;
  };
  auto applyW = [&](int nv, const TW* X, TW* Y, const double* sh) -> tp3b_status {
    const int kd = low ? 1 : 0;
    (low ? stats.n_apply_H_low : stats.n_apply_H_fp64) += nv;
    TP3B_HIP(kt.begin(kd, nv));
    tp3b_status r = apply_H_impl<TW>(op, nv, X, N, Y, N, sh, s, bf3);
    kt.end();
    return r;
  };
  auto dot = [&](int p, int q, const double* A, const double* B, std::vector<double>& host,
                 int ldc) -> tp3b_status {
    // host (row-major p x q) = A^T B
    TP3B_HIP(launch_dot_tn<double, double>(N, p, q, A, N, B, N, dM2, p, part, s));
    std::vector<double> cm((size_t)p * q);
    TP3B_HIP(hipMemcpyAsync(P(r_dnM), dM2, sizeof(double) * p * q, hipMemcpyDeviceToHost, s));
    TP3B_HIP(hipStreamSynchronize(s));
    std::memcpy(cm.data(), P(r_dnM), sizeof(double) * p * q);
    host.assign((size_t)p * ldc, 0.0);
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < q; ++j) host[(size_t)i * ldc + j] = cm[i + (size_t)j * p];
    return TP3B_OK;
  };

  // ---- start block
  {
    const int nb0 = (X0 && b0 > 0) ? std::min(b0, b) : 0;
    if (nb0 > 0) {
      if (o.check_finite) {
        int* flag = (int*)dY;
        TP3B_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
        TP3B_HIP(launch_check_finite<double>(N, nb0, X0, N, flag, s));
        int hf = 0;
        TP3B_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        TP3B_HIP(hipStreamSynchronize(s));
        if (hf) return fail(TP3B_ENONFINITE, "jdqr: non-finite start block");
      }
      TP3B_HIP(hipMemcpyAsync(QV, X0, sizeof(double) * N * nb0, hipMemcpyDeviceToDevice, s));
    }
    for (int j = nb0; j < b; ++j)
      TP3B_HIP(launch_hash_fill(N, QV + (int64_t)j * N, o.seed, 1000003ull + j, s));
    int rank = 0;
    double t0 = now();
    tp3b_status rs = block_orth_impl(N, 0, nullptr, N, b, QV, N, nullptr, nullptr, &rank,
                                     o.seed + 17, s);
    stats.t_orth += now() - t0;
    if (rs != TP3B_OK) return rs;
    part = dot_scratch(dscr);
    m = b;
    t0 = now();
    tp3b_status as = applyA64(m, V(), AV());
    if (as != TP3B_OK) return as;
    tp3b_status ds = dot(m, m, V(), AV(), M, m);
    if (ds != TP3B_OK) return ds;
    stats.t_apply += now() - t0;
  }

  std::vector<double> S, T;
  std::vector<int> pair;
  int outer = 0;
  double prev_rn0 = INFINITY;  // leading residual of the last outer iteration
  int stall = 0;               // consecutive outer iterations without progress
  while (k < nev && outer < o.max_outer) {
    // ---- 1. ordered Schur form M = S T S^T of the projected matrix.  V and
    // A V are not rotated here: the leading Schur vectors U = V S[:, :nb] and
    // A U are formed on their own (N x m x nb instead of N x m x m), and the
    // whole basis is rotated only where it changes (locking, restart).
    double t0 = now();
    S.assign((size_t)m * m, 0.0);
    T.assign((size_t)m * m, 0.0);
    pair.assign(m, 0);
    if (!ordered_schur(m, M.data(), S.data(), T.data(), pair.data()))
      return fail(TP3B_ENOCONV, "jdqr: projected Schur form did not converge");
    bool ident = true;
    for (int i = 0; i < m && ident; ++i)
      for (int j = 0; j < m; ++j)
        if (S[(size_t)i * m + j] != (i == j ? 1.0 : 0.0)) { ident = false; break; }
    // V <- V S[:, :q], A V <- A V S[:, :q] (q = m: the full rotation)
    auto rotate = [&](int q) -> tp3b_status {
      std::vector<double> Sc = colmajor(S, m, 0, 0, m, q);
      std::memcpy(P(r_upS), Sc.data(), sizeof(double) * m * q);
      TP3B_HIP(hipMemcpyAsync(dS, P(r_upS), sizeof(double) * m * q, hipMemcpyHostToDevice, s));
      if (rot_inplace) {
        // long blocks: both in place, row by row (A V keeps its column offset;
        // the offset grows only with locking, by at most nev in all, which its
        // buffer allows for)
        TP3B_HIP(launch_gemm_nn_rows_inplace(N, m, q, V(), N, dS, m, s));
        TP3B_HIP(launch_gemm_nn_rows_inplace(N, m, q, AV(), N, dS, m, s));
        return TP3B_OK;
      }
      TP3B_HIP(launch_gemm_nn<double>(N, m, q, 1.0, V(), N, dS, m, 0.0, TMP, N, s));
      TP3B_HIP(hipMemcpyAsync(V(), TMP, sizeof(double) * N * q, hipMemcpyDeviceToDevice, s));
      TP3B_HIP(launch_gemm_nn<double>(N, m, q, 1.0, AV(), N, dS, m, 0.0, TMP, N, s));
      // the rotated A V stays where it was written (no copy back)
      std::swap(AVbase, TMP);
      av0 = 0;
      return TP3B_OK;
    };
    const int nb = std::min(b, m);
    // a 2 x 2 block across the block edge couples u_nb into the residual of
    // column nb - 1
    const int nu = (nb < m && T[(size_t)nb * m + (nb - 1)] != 0.0) ? nb + 1 : nb;
    // ---- 2. U = V S[:, :nu] (into Q~ after the locked vectors), A U, and the
    // residuals R = (I - Q Q^T)(A U - U T[:nu, :nb])
    {
      std::vector<double> Sc = colmajor(S, m, 0, 0, m, nu);
      std::memcpy(P(r_upS), Sc.data(), sizeof(double) * m * nu);
      TP3B_HIP(hipMemcpyAsync(dS, P(r_upS), sizeof(double) * m * nu, hipMemcpyHostToDevice, s));
      std::vector<double> Tc_ = colmajor(T, m, 0, 0, nu, nb);
      std::memcpy(P(r_upT), Tc_.data(), sizeof(double) * nu * nb);
      TP3B_HIP(hipMemcpyAsync(dTb, P(r_upT), sizeof(double) * nu * nb, hipMemcpyHostToDevice, s));
      double* U = Qt + (int64_t)k * N;
      if (urres_fused) {
        TP3B_HIP(launch_urres_long(N, m, nu, nb, V(), AV(), N, dS, dTb, U, Rres, N, s));
      } else {
        TP3B_HIP(launch_gemm_nn<double>(N, m, nu, 1.0, V(), N, dS, m, 0.0, U, N, s));
        TP3B_HIP(launch_gemm_nn<double>(N, m, nb, 1.0, AV(), N, dS, m, 0.0, AU, N, s));
        TP3B_HIP(launch_gemm_nn_x0<double>(N, nu, nb, -1.0, U, N, dTb, nu, 1.0, AU, N, Rres, N, s));
      }
    }
    std::vector<double> Cq((size_t)std::max(k, 1) * nb, 0.0);  // Q^T A U, column-major k x nb
    std::vector<double> c1((size_t)std::max(k, 1) * nb), c2((size_t)std::max(k, 1) * nb);
    if (k > 0) {
      // two projection passes; both coefficient blocks come back with the norms
      TP3B_HIP(launch_dot_tn<double, double>(N, k, nb, QV, N, Rres, N, dC, k, part, s));
      TP3B_HIP(launch_gemm_nn<double>(N, k, nb, -1.0, QV, N, dC, k, 1.0, Rres, N, s));
      TP3B_HIP(launch_dot_tn<double, double>(N, k, nb, QV, N, Rres, N, dC2, k, part, s));
      TP3B_HIP(launch_gemm_nn<double>(N, k, nb, -1.0, QV, N, dC2, k, 1.0, Rres, N, s));
      TP3B_HIP(hipMemcpyAsync(P(r_dnC1), dC, sizeof(double) * k * nb, hipMemcpyDeviceToHost, s));
      TP3B_HIP(hipMemcpyAsync(P(r_dnC2), dC2, sizeof(double) * k * nb, hipMemcpyDeviceToHost, s));
    }
    TP3B_HIP(launch_bdot_diag<double>(N, nb, 1, Rres, 0, Rres, dNrm, 1, part, s));
    std::vector<double> rn(nb);
    TP3B_HIP(hipMemcpyAsync(P(r_dnRn), dNrm, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    TP3B_HIP(hipStreamSynchronize(s));
    std::memcpy(rn.data(), P(r_dnRn), sizeof(double) * nb);
    if (k > 0) {
      std::memcpy(c1.data(), P(r_dnC1), sizeof(double) * k * nb);
      std::memcpy(c2.data(), P(r_dnC2), sizeof(double) * k * nb);
    }
    if (k > 0)
      for (size_t e = 0; e < (size_t)k * nb; ++e) Cq[e] = c1[e] + c2[e];
    for (int j = 0; j < nb; ++j) rn[j] = std::sqrt(std::max(rn[j], 0.0));
    std::vector<double> theta(nb);
    for (int j = 0; j < nb; ++j) theta[j] = T[(size_t)j * m + j];
    stats.t_rr += now() - t0;
    if (o.verbose)
      fprintf(stderr, "[tp3b jdqr] outer %d locked %d m %d theta0 %.15g res0 %.3e\n", outer, k, m,
              theta[0], rn[0]);
    for (int j = 0; j < nb; ++j)
      if (!std::isfinite(rn[j]) || !std::isfinite(theta[j]))
        return fail(TP3B_ENONFINITE, "jdqr: non-finite residual");

    // ---- 3. locking of the converged prefix
    int p = 0;
    while (p < nb && k + p < nev) {
      const int blk = pair[p] ? 2 : 1;
      bool ok = p + blk <= nb;
      for (int q = p; ok && q < p + blk; ++q)
        ok = rn[q] <= o.tol * std::max(std::fabs(theta[q]), 1.0);
      if (!ok) break;
      p += blk;
    }
    if (p == 0 && o.stall_tol > 0) {
      // the leading residual has reached its FP64 rounding floor
      const double r0 = rn[0];
      if (r0 <= o.stall_tol * std::max(std::fabs(theta[0]), 1.0) && r0 >= 0.9 * prev_rn0 &&
          r0 <= 1.1 * prev_rn0)
        ++stall;
      else
        stall = 0;
      prev_rn0 = r0;
      const int blk = pair[0] ? 2 : 1;
      if (stall >= 3 && blk <= nb) {
        p = blk;
        stats.n_stall_lock += blk;
      }
    }
    if (p > 0) {
      prev_rn0 = INFINITY;
      stall = 0;
      if (k + p > nev) p = nev - k;  // never split beyond nev (pairs are not expected here)
      const int m_old = m;
      for (int j = 0; j < p; ++j) {
        for (int i = 0; i < k; ++i) Rl[i + (size_t)(k + j) * nev] = Cq[i + (size_t)j * k];
        // upper-triangular part of T, plus the subdiagonal entry of a 2 x 2 block
        for (int i = 0; i < p; ++i)
          if (i <= j || (i == j + 1 && pair[j])) Rl[(k + i) + (size_t)(k + j) * nev] = T[(size_t)i * m_old + j];
        lock_pair.push_back(pair[j]);
        lockres.push_back(rn[j]);
      }
      // the basis is rotated into Schur order: its first p columns are the
      // locked vectors, the rest spans the remaining search space
      if (!ident) {
        tp3b_status rs = rotate(m);
        if (rs != TP3B_OK) return rs;
      }
      // Q~ holds the same locked vectors as QV
      TP3B_HIP(hipMemcpyAsync(Qt + (int64_t)k * N, V(), sizeof(double) * N * p, hipMemcpyDeviceToDevice, s));
      if (use_prec) {
        double tp = now();
        tp3b_status ps = apply_prec_impl<double>(op, p, V(), N, PQ + (int64_t)k * N, N, s);
        if (ps != TP3B_OK) return ps;
        stats.n_apply_prec += p;
        stats.t_prec += now() - tp;
      }
      k += p;
      m -= p;
      av0 += p;
      std::vector<double> Mn((size_t)m * m);
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Mn[(size_t)i * m + j] = T[(size_t)(i + p) * m_old + (j + p)];
      M = Mn;
      stats.n_lock_events++;
      if (k >= nev || m == 0) break;
      continue;
    }
    ++outer;
    // ---- restart
    if (m + nb > m_max) {
      const int keep = std::max(m_min, nb);
      if (!ident) {
        tp3b_status rs = rotate(keep);
        if (rs != TP3B_OK) return rs;
      }
      m = keep;
      // Recompute the projected matrix from the kept vectors (limits drift).
      tp3b_status ds = dot(m, m, V(), AV(), M, m);
      if (ds != TP3B_OK) return ds;
      stats.n_restart++;
    }
    // ---- 4. correction equations
    std::vector<double> shift(nb);
    // first outer iterations, nothing locked yet: a target below the spectrum
    const double tfar = (k == 0 && outer <= o.low_start) ? op->spec_lo : target;
    for (int j = 0; j < nb; ++j)
      shift[j] = (rn[j] > o.switch_tol * std::fabs(theta[j])) ? tfar : theta[j];
    std::memcpy(P(r_upShift), shift.data(), sizeof(double) * nb);
    TP3B_HIP(hipMemcpyAsync(dShift, P(r_upShift), sizeof(double) * nb, hipMemcpyHostToDevice, s));
    const int nqt = k + nb;  // Q~ = Qt[:, 0:nqt]
    const double* Yq = Qt;   // P^{-1} Q~ H^{-1} (or Q~ without preconditioner)
    if (use_prec) {
      double tp = now();
      tp3b_status ps = apply_prec_impl<double>(op, nb, Qt + (int64_t)k * N, N, PQ + (int64_t)k * N, N, s);
      if (ps != TP3B_OK) return ps;
      stats.n_apply_prec += nb;
      stats.t_prec += now() - tp;
      if (nqt <= SI_MAXN) {
        // H = Q~^T P^{-1} Q~ inverted on the device (no host round trip); a
        // singular H is reported by dFlag at the end of the outer iteration
        TP3B_HIP((launch_dot_tn<double, double>(N, nqt, nqt, Qt, N, PQ, N, dM2, nqt, part, s)));
        TP3B_HIP(launch_small_inverse(nqt, dM2, dHinv, dFlag, s));
      } else {
        std::vector<double> Hh;
        tp3b_status ds = dot(nqt, nqt, Qt, PQ, Hh, nqt);
        if (ds != TP3B_OK) return ds;
        std::vector<double> Hi((size_t)nqt * nqt);
        if (!lu_inverse(nqt, Hh.data(), Hi.data()))
          return fail(TP3B_ENOCONV, "jdqr: singular projected preconditioner");
        std::vector<double> Hic = colmajor(Hi, nqt, 0, 0, nqt, nqt);
        std::memcpy(P(r_upHinv), Hic.data(), sizeof(double) * nqt * nqt);
        TP3B_HIP(hipMemcpyAsync(dHinv, P(r_upHinv), sizeof(double) * nqt * nqt, hipMemcpyHostToDevice, s));
      }
      TP3B_HIP(launch_gemm_nn<double>(N, nqt, nqt, 1.0, PQ, N, dHinv, nqt, 0.0, Yp, N, s));
      Yq = Yp;
    }
    const TW* Qtw;
    const TW* Yqw;
    if (low) {
      TP3B_HIP((launch_convert<double, TW>(N, nqt, 1.0, Qt, N, Qtwb.as<TW>(), N, s)));
      TP3B_HIP((launch_convert<double, TW>(N, nqt, 1.0, Yq, N, Ypwb.as<TW>(), N, s)));
      Qtw = Qtwb.as<TW>();
      Yqw = Ypwb.as<TW>();
    } else {
      Qtw = (const TW*)Qt;
      Yqw = (const TW*)Yq;
    }
    const double tg0 = now();
    auto precond_w = [&](const TW* in, TW* out) -> tp3b_status {
      stats.n_apply_prec += nb;
      const int kd = low ? 3 : 2;
      TP3B_HIP(kt.begin(kd, nb));
      tp3b_status r = apply_prec_impl<TW>(op, nb, in, N, out, N, s, bf3);
      kt.end();
      return r;
    };
    auto project = [&](TW* Zp) -> tp3b_status {
      TP3B_HIP((launch_dot_tn<TW, TW>(N, nqt, nb, Qtw, N, Zp, N, dC2, nqt, part, s)));
      TP3B_HIP((launch_gemm_nn<TW>(N, nqt, nb, -1.0, Yqw, N, dC2, nqt, 1.0, Zp, N, s)));
      return TP3B_OK;
    };
    // Right-hand side proj(P^{-1}(-r)) and the fixed GMRES steps: kernel
    // launches only, so the sequence can be captured as a graph.
    const int64_t bs = N * nb;
    auto gmres_launch = [&]() -> tp3b_status {
      TW* rhs = W;
      // sign of the final combination: an FP64 inner solve preconditions r
      // itself, so it runs on -rhs; GMRES is odd in its right-hand side and
      // negation is exact, so the negated combination is the same correction
      double t_sign = 1.0;
      if (use_prec) {
        if constexpr (std::is_same<TW, double>::value) {
          tp3b_status ps = precond_w(Rres, rhs);
          if (ps != TP3B_OK) return ps;
          t_sign = -1.0;
        } else {
          TP3B_HIP((launch_convert<double, TW>(N, nb, -1.0, Rres, N, Zt, N, s)));
          tp3b_status ps = precond_w(Zt, rhs);
          if (ps != TP3B_OK) return ps;
        }
      } else {
        TP3B_HIP((launch_convert<double, TW>(N, nb, -1.0, Rres, N, rhs, N, s)));
      }
      { tp3b_status ps = project(rhs); if (ps != TP3B_OK) return ps; }
      TP3B_HIP(launch_bdot_partials<TW>(N, nb, 1, rhs, 0, rhs, part, s));
      TP3B_HIP(launch_normalize_cols_red<TW>(N, nb, part, rhs, Vg, dBeta, 1, s));
      for (int kk = 0; kk < steps; ++kk) {
        TW* vk = Vg + (int64_t)kk * bs;
        TW* w = W;
        if (use_prec) {
          tp3b_status as = applyW(nb, vk, Zt, dShift);
          if (as != TP3B_OK) return as;
          tp3b_status ps = precond_w(Zt, w);
          if (ps != TP3B_OK) return ps;
        } else {
          tp3b_status as = applyW(nb, vk, w, dShift);
          if (as != TP3B_OK) return as;
        }
        { tp3b_status ps = project(w); if (ps != TP3B_OK) return ps; }
        double* h1 = dH1 + (size_t)kk * b * hld;
        double* h2 = dH2 + (size_t)kk * b * hld;
        // CGS2 against the basis, then the norm; each update sums its dot's
        // partials itself (no separate reduction launch)
        TP3B_HIP(launch_bdot_partials<TW>(N, nb, kk + 1, Vg, bs, w, part, s));
        if (arn_fused) {
          // each update also forms the partials of the next dots on the rows
          // it has just written (the second pass's dots, then the norm), so
          // the basis and w are not read again for them
          double* part_b = part + part_b_off;
          TP3B_HIP(launch_bupdate_dot_red<TW>(N, nb, kk + 1, -1.0, Vg, bs, part, 0, h1, hld, w, 0,
                                               part_b, s));
          TP3B_HIP(launch_bupdate_dot_red<TW>(N, nb, kk + 1, -1.0, Vg, bs, part_b, nch_f, h2, hld, w, 1,
                                               part, s));
          TP3B_HIP(launch_normalize_cols_red_n<TW>(N, nb, part, nch_f, w, Vg + (int64_t)(kk + 1) * bs,
                                                   dHs + (size_t)kk * b, 1, s));
        } else {
          TP3B_HIP(launch_bupdate_diag_red<TW>(N, nb, kk + 1, -1.0, Vg, bs, part, h1, hld, w, s));
          TP3B_HIP(launch_bdot_partials<TW>(N, nb, kk + 1, Vg, bs, w, part, s));
          TP3B_HIP(launch_bupdate_diag_red<TW>(N, nb, kk + 1, -1.0, Vg, bs, part, h2, hld, w, s));
          TP3B_HIP(launch_bdot_partials<TW>(N, nb, 1, w, 0, w, part, s));
          TP3B_HIP(launch_normalize_cols_red<TW>(N, nb, part, w, Vg + (int64_t)(kk + 1) * bs,
                                                 dHs + (size_t)kk * b, 1, s));
        }
      }
      // least squares on the device, then t_j = V_j y_j, written in FP64 into Tc
      TP3B_HIP(launch_gmres_lstsq(nb, b, steps, hld, dH1, dH2, dHs, dBeta, dY, s));
      TP3B_HIP((launch_bcombine<TW, double>(N, nb, steps, t_sign, Vg, bs, dY, hld, Tc, N, s)));
      return TP3B_OK;
    };
    if (o.graph) {
      graphs.drop_stale(part);
      SolveGraphs::Entry* ge = graphs.find(nqt, nb, part);
      if (!ge) {
        // capture once: the launches are recorded, not run, so the apply
        // counters they bump are taken back and added per replay instead
        SolveGraphs::Entry ne{nqt, nb, part, nullptr, nullptr, 0, 0, 0};
        const int64_t h64 = stats.n_apply_H_fp64, hlow = stats.n_apply_H_low,
                      pr = stats.n_apply_prec;
        kt.paused = true;
        TP3B_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        tp3b_status cs = gmres_launch();
        hipError_t ce = hipStreamEndCapture(s, &ne.g);
        kt.paused = false;
        if (cs != TP3B_OK) {
          if (ne.g) (void)hipGraphDestroy(ne.g);
          return cs;
        }
        TP3B_HIP(ce);
        hipError_t ie = hipGraphInstantiate(&ne.x, ne.g, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
          (void)hipGraphDestroy(ne.g);
          TP3B_HIP(ie);
        }
        ne.dH64 = stats.n_apply_H_fp64 - h64;
        ne.dHlow = stats.n_apply_H_low - hlow;
        ne.dPrec = stats.n_apply_prec - pr;
        stats.n_apply_H_fp64 = h64;
        stats.n_apply_H_low = hlow;
        stats.n_apply_prec = pr;
        graphs.e.push_back(ne);
        ge = &graphs.e.back();
      }
      TP3B_HIP(hipGraphLaunch(ge->x, s));
      stats.n_apply_H_fp64 += ge->dH64;
      stats.n_apply_H_low += ge->dHlow;
      stats.n_apply_prec += ge->dPrec;
    } else {
      tp3b_status gs = gmres_launch();
      if (gs != TP3B_OK) return gs;
    }
    stats.t_gmres += now() - tg0;  // host time; the device work is still queued

    // ---- 5. expand the basis
    double to = now();
    double* Vn = QV + (int64_t)(k + m) * N;
    const uint64_t orth_seed = o.seed + 7919ull * (uint64_t)outer;
    if (o.test_dup_column > 0 && outer == o.test_dup_column && nb > 1)
      // testing hook: the second correction column becomes a copy of the first,
      // so the expansion block is rank deficient
      TP3B_HIP(hipMemcpyAsync(Tc + N, Tc, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    // queued without a round trip (the dependence flags come back with the
    // projected matrix below); reads the correction from Tc and writes Vn
    tp3b_status os = block_orth_queue(N, k + m, QV, N, nb, Vn, N, dOFlags, s, Tc);
    if (os != TP3B_OK) return os;
    part = dot_scratch(dscr);
    if (!part) return fail(TP3B_ENOMEM, "jdqr: scratch allocation failed");
    stats.t_orth += now() - to;
    double ta = now();
    // the new columns (V^T A Vn) and rows (Vn^T A V) of the projected matrix,
    // read back together (with the block's dependence flags)
    std::vector<double> top((size_t)(m + nb) * nb), left((size_t)nb * m);
    for (int pass = 0;; ++pass) {
      tp3b_status as = applyA64(nb, Vn, AV() + (int64_t)m * N);
      if (as != TP3B_OK) return as;
      std::vector<double> ct((size_t)(m + nb) * nb), cl((size_t)nb * m);
      TP3B_HIP(launch_dot_tn<double, double>(N, m + nb, nb, V(), N, AV() + (int64_t)m * N, N, dM2,
                                             m + nb, part, s));
      TP3B_HIP(hipMemcpyAsync(P(r_dnTop), dM2, sizeof(double) * ct.size(), hipMemcpyDeviceToHost, s));
      TP3B_HIP(launch_dot_tn<double, double>(N, nb, m, Vn, N, AV(), N, dS, nb, part, s));
      TP3B_HIP(hipMemcpyAsync(P(r_dnLeft), dS, sizeof(double) * cl.size(), hipMemcpyDeviceToHost, s));
      TP3B_HIP(hipMemcpyAsync(P(r_dnFlag), dFlag, sizeof(int), hipMemcpyDeviceToHost, s));
      TP3B_HIP(hipMemcpyAsync(P(r_dnOFlags), dOFlags, sizeof(int) * (nb + 1), hipMemcpyDeviceToHost, s));
      TP3B_HIP(hipStreamSynchronize(s));
      if (*(const int*)P(r_dnFlag)) return fail(TP3B_ENOCONV, "jdqr: singular projected preconditioner");
      const int* of = (const int*)P(r_dnOFlags);
      if (pass == 0) {
        if (of[nb]) return fail(TP3B_ENONFINITE, "block_orth: non-finite input");
        bool dep = false;
        for (int j = 0; j < nb; ++j) dep = dep || of[j];
        if (dep) {
          // a dependent column (rare): replaced by a random vector as the
          // synchronous routine does, the block orthogonalised again with it,
          // and A Vn and the projected entries recomputed
          if (o.verbose) fprintf(stderr, "[tp3b jdqr] outer %d: dependent expansion column replaced\n", outer);
          for (int j = 0; j < nb; ++j)
            if (of[j]) {
              TP3B_HIP(launch_hash_fill(N, Vn + (int64_t)j * N, orth_seed, (uint64_t)(1000 + j), s));
              stats.n_dep_replaced++;
            }
          int rank = 0;
          os = block_orth_impl(N, k + m, QV, N, nb, Vn, N, nullptr, nullptr, &rank, orth_seed, s);
          if (os != TP3B_OK) return os;
          part = dot_scratch(dscr);
          if (!part) return fail(TP3B_ENOMEM, "jdqr: scratch allocation failed");
          stats.n_apply_H_fp64 -= nb;  // the first A Vn is redone, not counted twice
          continue;
        }
      }
      std::memcpy(ct.data(), P(r_dnTop), sizeof(double) * ct.size());
      std::memcpy(cl.data(), P(r_dnLeft), sizeof(double) * cl.size());
      for (int i = 0; i < m + nb; ++i)
        for (int j = 0; j < nb; ++j) top[(size_t)i * nb + j] = ct[i + (size_t)j * (m + nb)];
      for (int i = 0; i < nb; ++i)
        for (int j = 0; j < m; ++j) left[(size_t)i * m + j] = cl[i + (size_t)j * nb];
      break;
    }
    std::vector<double> Mn((size_t)(m + nb) * (m + nb), 0.0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) Mn[(size_t)i * (m + nb) + j] = M[(size_t)i * m + j];
    for (int i = 0; i < m + nb; ++i)
      for (int j = 0; j < nb; ++j) Mn[(size_t)i * (m + nb) + m + j] = top[(size_t)i * nb + j];
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < m; ++j) Mn[(size_t)(m + i) * (m + nb) + j] = left[(size_t)i * m + j];
    m += nb;
    M = Mn;
    stats.t_apply += now() - ta;
  }

  // ---- outputs
  const int nconv = k;
  std::vector<double> ev(nconv);
  for (int i = 0; i < nconv; ++i) {
    // 2 x 2 blocks (complex pairs) are reported by their real part.
    if (i + 1 < nconv && lock_pair[i]) {
      const double a = Rl[i + (size_t)i * nev], d = Rl[(i + 1) + (size_t)(i + 1) * nev];
      ev[i] = ev[i + 1] = 0.5 * (a + d);
      ++i;
    } else {
      ev[i] = Rl[i + (size_t)i * nev];
    }
  }
  std::vector<double> evs = ev;
  std::sort(evs.begin(), evs.end());
  if (evals)
    for (int i = 0; i < nev; ++i) evals[i] = i < nconv ? evs[i] : NAN;
  if (Qout && nconv > 0)
    TP3B_HIP(hipMemcpyAsync(Qout, QV, sizeof(double) * N * nconv, hipMemcpyDeviceToDevice, s));
  TP3B_HIP(hipStreamSynchronize(s));
  if (Rout) std::memcpy(Rout, Rl.data(), sizeof(double) * nev * nev);
  if (resnorm)
    for (int i = 0; i < nev; ++i) resnorm[i] = i < (int)lockres.size() ? lockres[i] : NAN;
  if (kt.on) kt.collect(stats.t_kernel, stats.n_kernel, stats.v_kernel);
  stats.n_conv = nconv;
  stats.n_outer = outer;
  stats.t_total = now() - t_start;
  if (st) *st = stats;
  if (nconv < nev) return fail(TP3B_ENOCONV, "jdqr: not converged within max_outer");
  return TP3B_OK;
}

}  // namespace tp3b

using namespace tp3b;

extern "C" {

tp3b_status tp3b_jdqr_default_opts(tp3b_jdqr_opts* o) {
  try {
    if (!o) return fail(TP3B_EINVAL, "null options");
    std::memset(o, 0, sizeof(*o));
    o->nev = 1;
    o->block = 1;
    o->gmres_steps = 10;
    o->max_outer = 1000;
    o->precond = 1;
    o->inner_prec = TP3B_FP64;
    o->tol = 1e-12;
    o->switch_tol = 1e-2;
    o->stall_tol = 1e-8;
    o->low_start = 3;
    o->target = NAN;
    o->seed = 0;
    return TP3B_OK;
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_jdqr_solve(tp3b_op op, const tp3b_jdqr_opts* opts, const double* X0, int32_t b0,
                            double* evals, double* Q, double* R, double* resnorm,
                            tp3b_jdqr_stats* stats) {
  try {
    if (!op || !opts) return fail(TP3B_EINVAL, "null operator or options");
    tp3b_jdqr_opts o = *opts;
    if (o.nev < 1 || o.block < 1) return fail(TP3B_EINVAL, "nev and block must be >= 1");
    if (o.block > 32) return fail(TP3B_EINVAL, "block must be <= 32");
    if (o.gmres_steps <= 0) o.gmres_steps = 10;
    if (o.gmres_steps > 38) return fail(TP3B_EINVAL, "gmres_steps must be <= 38");
    if (o.max_outer <= 0) o.max_outer = 1000;
    if (!(o.tol > 0)) o.tol = 1e-12;
    if (!(o.switch_tol > 0)) o.switch_tol = 1e-2;
    int mmax = std::max(4 * o.block, 2 * (o.nev + o.block));
    mmax = ((mmax + o.block - 1) / o.block) * o.block;
    if (o.m_max <= 0) o.m_max = mmax;
    if (o.m_min <= 0) o.m_min = o.m_max / 2;
    if (o.m_min < o.block || o.m_max < o.m_min + o.block)
      return fail(TP3B_EINVAL, "need block <= m_min and m_min + block <= m_max");
    if (op->N < (int64_t)(o.nev + o.m_max + o.block))
      return fail(TP3B_EINVAL, "problem too small for nev + m_max + block basis vectors");
    if (o.precond && !op->have_prec)
      return fail(TP3B_ENOTSUP, "the kinetic preconditioner is unavailable for this operator");
    if (X0 && b0 < 0) return fail(TP3B_EINVAL, "b0 must be >= 0");
    TP3B_HIP(hipSetDevice(op->device));
    if (o.inner_prec != TP3B_FP64 && o.inner_prec != TP3B_FP32 && o.inner_prec != TP3B_BF16X3)
      return fail(TP3B_EINVAL, "unknown inner precision");
    if (o.inner_prec != TP3B_FP64)
      return jdqr_run<float>(op, o, X0, b0, evals, Q, R, resnorm, stats,
                             o.inner_prec == TP3B_BF16X3);
    return jdqr_run<double>(op, o, X0, b0, evals, Q, R, resnorm, stats, false);
  } catch (...) {
    return exception_status();
  }
}

}  // extern "C"
