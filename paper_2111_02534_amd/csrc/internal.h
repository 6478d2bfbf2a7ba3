// Library-internal state shared by the C-ABI entry points and the eigensolver.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <exception>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tp3b.h"
#include "kernels.h"

namespace tp3b {

// Device copies of one operand set in one storage precision.
template <typename T>
struct DevOps {
  T* K[4] = {nullptr, nullptr, nullptr, nullptr};   // -c D2 of each mode, row-major
  T* KT[4] = {nullptr, nullptr, nullptr, nullptr};  // its transpose (right operand)
  T* V = nullptr;                                   // potential table, vector layout
  // Preconditioner factors per mode: K_k = S_k diag(lam_k) S_k^{-1}.  1D uses
  // modes 0 (x, left operands) and 1 (y, right operands); 2D uses modes 0-2 as
  // left operands and mode 3 as right operand.
  T* Si[4] = {nullptr, nullptr, nullptr, nullptr};   // S_k^{-1}      (left operand)
  T* S[4] = {nullptr, nullptr, nullptr, nullptr};    // S_k           (left operand)
  T* SiT[4] = {nullptr, nullptr, nullptr, nullptr};  // (S_k^{-1})^T  (right operand)
  T* ST[4] = {nullptr, nullptr, nullptr, nullptr};   // S_k^T         (right operand)
  T* lam[4] = {nullptr, nullptr, nullptr, nullptr};
  T* lamItem = nullptr;  // 2D: lam_x1[i1] + lam_x2[i2] per (x1, x2) plane
  T* lamItemY = nullptr;  // 2D: lam_y1[j1] + lam_y2[j2] per flattened y index
  T* work = nullptr;  // preconditioner intermediate, work_vecs vectors
  // 2D operators with every mode size <= P2_MAXN: MFMA fragments (plane2d.hip)
  // of K_k, S_k and S_k^{-1} per mode, and the separable factors of a Gaussian
  // potential (4 x 64 x 64, NULL for other potentials).
  T* frK[4] = {nullptr, nullptr, nullptr, nullptr};
  T* frS[4] = {nullptr, nullptr, nullptr, nullptr};
  T* frSi[4] = {nullptr, nullptr, nullptr, nullptr};
  T* G = nullptr;
};

// Runs f(i) for every i in [0, n) on up to kHostThreads host threads (the
// calling one included), handing out indices one at a time.  f must write only
// data that belongs to its own index; each f(i) does the same arithmetic
// whichever thread runs it.  Used for the independent small dense problems of
// the instances of a batch.
constexpr int kHostThreads = 8;
template <class F>
void parallel_for(int n, F&& f) {
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int nt = std::min({hw, kHostThreads, (n + 15) / 16});
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int> next{0};
  std::exception_ptr err = nullptr;
  std::mutex err_m;
  auto work = [&]() {
    try {
      for (int i = next.fetch_add(1); i < n; i = next.fetch_add(1)) f(i);
    } catch (...) {
      std::lock_guard<std::mutex> g(err_m);
      if (!err) err = std::current_exception();
      next.store(n);  // the other threads stop at their next index
    }
  };
  std::vector<std::thread> th;
  try {
    th.reserve(nt - 1);
    for (int t = 1; t < nt; ++t) th.emplace_back(work);
  } catch (...) {
    // fewer threads than asked for: the calling thread takes what is left
  }
  work();
  for (std::thread& x : th) x.join();
  if (err) std::rethrow_exception(err);
}

}  // namespace tp3b

struct tp3b_op_s {
  int ndim = 1;
  int n[4] = {0, 0, 0, 0};
  int nmodes = 2;
  double L[4] = {0, 0, 0, 0};
  double cx = 0, cy = 0;
  int pot = 0;
  double v0 = 0, width = 1;
  double sigma = 0;
  double mu_hl = 1;
  int64_t N = 0;
  int device = 0;
  bool have_prec = false;
  double lam_min = 0;   // smallest |sum of mode eigenvalues - sigma|
  double spec_lo = 0;   // min V + sum over modes of the smallest mode eigenvalue
  std::vector<double> D2h[4];  // host copies (row-major)
  std::vector<double> Vh;      // host potential
  tp3b::DevOps<double> d64;
  tp3b::DevOps<float> d32;
  int work_vecs = 0;
  bool plane2d = false;         // 2D with every mode size <= P2_MAXN: two-pass applies
  bool x_same_K = false;        // 2D: the two x modes have the same operator K (and
  bool x_same_S = false;        // the same eigen-factors): one LDS copy in the x passes
  bool y_same_K = false;        // the same for the two y modes (y-plane passes)
  bool y_same_S = false;
  std::vector<double> Gh;       // separable Gaussian factors of V (plane2d, Gaussian shapes)
  double gscale = 0;            // -v0 for those factors
  // tile choice: explicit override, else autotuned [tp3b_prec][0 = H, 1 = prec],
  // else heuristic
  int tile_override = -1;
  int tuned[3][2] = {{-1, -1}, {-1, -1}, {-1, -1}};
  // FP32 mode operators split into bf16 hi and lo once for the BF16x3 products
  // (device, 2 n^2 values each): left operands in their own layout, right
  // operands transposed
  struct Bf3Split {
    const float* src;
    int n;
    unsigned short* hl;
  };
  std::vector<Bf3Split> bf3L, bf3R;
};

namespace tp3b {

void set_error(const std::string& msg);
tp3b_status fail(tp3b_status code, const std::string& msg);
tp3b_status hip_fail(hipError_t e, const char* where);
// Inside a catch block: the status for the exception in flight (ENOMEM for a
// failed host allocation, EDEVICE otherwise), with its message recorded.  The
// C-ABI entry points catch every exception and return this.
tp3b_status exception_status();

#define TP3B_HIP(...)                                              \
  do {                                                             \
    hipError_t _e = (__VA_ARGS__);                                 \
    if (_e != hipSuccess) return tp3b::hip_fail(_e, #__VA_ARGS__); \
  } while (0)

// Precision-generic internal applies (no argument validation).  With
// bf3 = true (T = float only) the mode products run as BF16x3 split products.
template <typename T>
tp3b_status apply_H_impl(tp3b_op op, int nvec, const T* X, int64_t ldx, T* Y, int64_t ldy,
                         const double* shifts, hipStream_t s, bool bf3 = false);
template <typename T>
tp3b_status apply_prec_impl(tp3b_op op, int nvec, const T* X, int64_t ldx, T* Y, int64_t ldy,
                            hipStream_t s, bool bf3 = false);
int choose_tile(int M, int Nc, int64_t nbatch, bool fp64);
// Second-derivative matrix (row-major, desc->D2[k] when given) and ascending
// nodes of mode k of a descriptor.
void mode_grid(const tp3b_problem_desc* d, int k, std::vector<double>& D2, std::vector<double>& x);
// u(r) of the descriptor's pair-potential shape with depth v0 and width w.
double pair_potential(int pot, double r, double v0, double w);
// Tile shape of an operator's 1D applies: kind 0 = Hamiltonian, 1 = preconditioner.
int op_tile(tp3b_op op, bool f64, bool bf3, int kind, int64_t nbatch);
template <typename T>
DevOps<T>& dev_ops(tp3b_op op);

// Device scratch for the dot reductions (grows on demand, per device).
double* dot_scratch(int64_t doubles);
tp3b_status block_orth_impl(int64_t N, int nq, const double* Q, int64_t ldq, int nx, double* X,
                            int64_t ldx, double* C_qx, double* R_xx, int* rank, uint64_t seed,
                            hipStream_t s);
// The factor-free block orthogonalisation queued with no host round trip (CGS
// twice against Q, Cholesky-QR twice).  dflags (device, nx + 1 ints) receive
// the first factorisation's dependence flags and, at [nx], the non-finite test
// of the input.  With no flag set X holds the orthonormal block; otherwise the
// caller replaces the flagged columns and runs block_orth_impl on X.  Xin
// (optional, same leading dimension, not aliasing X) is the input block when it
// lives elsewhere: the first projection writes its result into X.
// scr (optional): scratch of at least orth_scratch_doubles(N, nq, nx) doubles
// to use instead of the library's growing dot scratch.
tp3b_status block_orth_queue(int64_t N, int nq, const double* Q, int64_t ldq, int nx, double* X,
                             int64_t ldx, int* dflags, hipStream_t s, const double* Xin = nullptr,
                             double* scr = nullptr);
int64_t orth_scratch_doubles(int64_t N, int nq, int nx);

}  // namespace tp3b
