// C-ABI entry points: operator set-up, Hamiltonian and preconditioner applies,
// block orthogonalisation.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <mutex>
#include <string>
#include <vector>

#include "dense_la.h"
#include "internal.h"

namespace tp3b {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
tp3b_status fail(tp3b_status code, const std::string& msg) {
  g_err = msg;
  return code;
}
tp3b_status hip_fail(hipError_t e, const char* where) {
  g_err = std::string("HIP error '") + hipGetErrorString(e) + "' in " + where;
  return e == hipErrorOutOfMemory ? TP3B_ENOMEM : TP3B_EDEVICE;
}
tp3b_status exception_status() {
  tp3b_status code = TP3B_EDEVICE;
  char what[256] = "unknown host exception";
  try {
    throw;
  } catch (const std::bad_alloc&) {
    code = TP3B_ENOMEM;
    std::snprintf(what, sizeof(what), "%s", "host memory allocation failed");
  } catch (const std::exception& e) {
    std::snprintf(what, sizeof(what), "%s", e.what());
  } catch (...) {
  }
  try {
    g_err = std::string("host exception: ") + what;
  } catch (...) {
    // no memory even for the message: the status alone reports it
  }
  return code;
}

// ---------------------------------------------------------------- grids
// Second-derivative collocation matrix on the n interior Chebyshev-Gauss-Lobatto
// points of [-L, L] with homogeneous Dirichlet conditions (Sec. 3.1): the
// Lagrange interpolant through K+1 = n+2 points t_j = cos(pi j/K) is
// differentiated twice and the two boundary rows and columns are removed.
// Nodes ascend: x_i = -L t_i, i = 1..n.
static void cgl_second_derivative(int n, double L, std::vector<double>& D2,
                                  std::vector<double>& x) {
  const int K = n + 1;
  std::vector<double> t(K + 1), c(K + 1), D((size_t)(K + 1) * (K + 1));
  for (int j = 0; j <= K; ++j) {
    // cos(pi j / K) evaluated symmetrically for exact antisymmetry
    t[j] = (2 * j <= K) ? std::cos(M_PI * j / K) : -std::cos(M_PI * (K - j) / K);
    c[j] = ((j % 2) ? -1.0 : 1.0) * ((j == 0 || j == K) ? 0.5 : 1.0);
  }
  for (int i = 0; i <= K; ++i) {
    double rowsum = 0.0;
    for (int j = 0; j <= K; ++j) {
      if (i == j) continue;
      const double v = (c[j] / c[i]) / (t[i] - t[j]);
      D[(size_t)i * (K + 1) + j] = v;
      rowsum += v;
    }
    D[(size_t)i * (K + 1) + i] = -rowsum;
  }
  D2.assign((size_t)n * n, 0.0);
  const double s = 1.0 / (L * L);
  for (int i = 1; i <= n; ++i)
    for (int j = 1; j <= n; ++j) {
      double acc = 0.0;
      for (int k = 0; k <= K; ++k) acc += D[(size_t)i * (K + 1) + k] * D[(size_t)k * (K + 1) + j];
      D2[(size_t)(i - 1) * n + (j - 1)] = acc * s;
    }
  x.resize(n);
  for (int i = 1; i <= n; ++i) x[i - 1] = -L * t[i];
}

// The paper's grid on the whole real line (Sec. 3.1): the N roots of T_N,
// t_j = cos(pi (2j+1) / (2N)), carried to x = L t / sqrt(1 - t^2).  Grid
// functions are interpolated by a polynomial in t; d/dt comes from the
// barycentric formula (weights of first-kind Chebyshev points
// (-1)^j sin((2j+1) pi / (2N))), and the chain rule gives
// d^2/dx^2 = t'(x)^2 d^2/dt^2 + t''(x) d/dt with t' = (1 - t^2)^{3/2} / L and
// t'' = -3 t (1 - t^2)^2 / L^2.  Nodes ascend.
static void mapped_second_derivative(int N, double L, std::vector<double>& D2,
                                     std::vector<double>& x) {
  std::vector<double> t(N), w(N), D((size_t)N * N);
  for (int i = 0; i < N; ++i) {
    const int j = N - 1 - i;  // descending root index -> ascending order
    const double a = M_PI * (2 * j + 1) / (2.0 * N);
    t[i] = std::cos(a);
    w[i] = ((j % 2) ? -1.0 : 1.0) * std::sin(a);
  }
  for (int i = 0; i < N; ++i) {
    double rowsum = 0.0;
    for (int j = 0; j < N; ++j) {
      if (i == j) continue;
      const double v = (w[j] / w[i]) / (t[i] - t[j]);
      D[(size_t)i * N + j] = v;
      rowsum += v;
    }
    D[(size_t)i * N + i] = -rowsum;
  }
  D2.assign((size_t)N * N, 0.0);
  x.resize(N);
  for (int i = 0; i < N; ++i) {
    const double s = 1.0 - t[i] * t[i];
    const double tp = s * std::sqrt(s) / L;
    const double tpp = -3.0 * t[i] * s * s / (L * L);
    for (int j = 0; j < N; ++j) {
      double dd = 0.0;
      for (int k = 0; k < N; ++k) dd += D[(size_t)i * N + k] * D[(size_t)k * N + j];
      D2[(size_t)i * N + j] = tp * tp * dd + tpp * D[(size_t)i * N + j];
    }
    x[i] = L * t[i] / std::sqrt(s);
  }
}

// Restriction of an operator on a grid symmetric about 0 (an even number N of
// ascending nodes) to functions of parity `sign`: unknowns at the N/2 positive
// nodes, the value at -x being sign times the value at x.
static void parity_fold(int N, const std::vector<double>& D2, const std::vector<double>& x,
                        int sign, std::vector<double>& D2h, std::vector<double>& xh) {
  const int h = N / 2;
  D2h.assign((size_t)h * h, 0.0);
  xh.resize(h);
  for (int i = 0; i < h; ++i) {
    const int pi = h + i;
    xh[i] = x[pi];
    for (int j = 0; j < h; ++j) {
      const int pj = h + j, mj = N - 1 - pj;
      D2h[(size_t)i * h + j] = D2[(size_t)pi * N + pj] + sign * D2[(size_t)pi * N + mj];
    }
  }
}

static double pair_pot(int pot, double r, double v0, double w) {
  switch (pot) {
    case TP3B_POT_GAUSS: return -v0 * std::exp(-(r * r) / (2.0 * w * w));
    case TP3B_POT_GAUSS_PAPER: return -v0 * std::exp(-(r * r));
    case TP3B_POT_LORENTZ3: {
      const double d = 1.0 + r * r;
      return -v0 / (d * d * d);
    }
    case TP3B_POT_HARMONIC: return 0.5 * v0 * r * r;
    default: return 0.0;
  }
}

double pair_potential(int pot, double r, double v0, double w) { return pair_pot(pot, r, v0, w); }

void mode_grid(const tp3b_problem_desc* d, int k, std::vector<double>& D2, std::vector<double>& x) {
  const int n = d->n[k];
  if (d->grid == TP3B_GRID_MAPPED) {
    if (d->parity[k] == 0) {
      mapped_second_derivative(n, d->L[k], D2, x);
    } else {
      std::vector<double> Df, xf;
      mapped_second_derivative(2 * n, d->L[k], Df, xf);
      parity_fold(2 * n, Df, xf, d->parity[k] > 0 ? 1 : -1, D2, x);
    }
  } else {
    cgl_second_derivative(n, d->L[k], D2, x);
  }
  if (d->D2[k]) D2.assign(d->D2[k], d->D2[k] + (size_t)n * n);
}

int choose_tile(int M, int Nc, int64_t nbatch, bool fp64) {
  // Largest tile that still gives >= 1024 workgroups (4 per CU); otherwise the
  // one giving the most parallelism without mostly-empty tiles.
  struct C { int id, tm, tn; };
  // Of the two 32 x 32 tiles the eight-wave form: twice the waves in flight
  // per tile to cover the MFMA and fetch latencies of a short K loop (measured
  // at n = 256, 8 vectors: H apply 20.8 against 22.8 us in FP64, 14.4 against
  // 16.4 us in FP32).
  // FP64 skips the 128-wide tiles: under the two-waves-per-SIMD bound their
  // accumulators spill (n = 1024, 16 vectors: 64 x 64 1.23 ms, 64 x 128
  // 1.34 ms, 128 x 128 1.41 ms per H apply).
  const int small = TILE_32W8;
  const C cfgs[] = {{TILE_128, 128, 128}, {TILE_64x128, 64, 128}, {TILE_64, 64, 64}, {small, 32, 32}};
  for (const C& c : cfgs) {
    if (c.tm > M || c.tn > Nc) continue;
    if (fp64 && c.tn > 64) continue;
    int64_t wg = (int64_t)((M + c.tm - 1) / c.tm) * ((Nc + c.tn - 1) / c.tn) * nbatch;
    if (wg >= 1024) return c.id;
  }
  return (M >= 64 && Nc >= 64 && (int64_t)((M + 63) / 64) * ((Nc + 63) / 64) * nbatch >= 512) ? TILE_64
                                                                                            : small;
}

// --------------------------------------------------------------- scratch
// One scratch area per thread and device: distinct threads may use the
// library concurrently (one handle per thread).
static thread_local double* g_scratch[64] = {nullptr};
static thread_local int64_t g_scratch_sz[64] = {0};

double* dot_scratch(int64_t doubles) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  if (g_scratch_sz[dev] < doubles) {
    if (g_scratch[dev]) {
      (void)hipDeviceSynchronize();
      (void)hipFree(g_scratch[dev]);
      g_scratch[dev] = nullptr;
      g_scratch_sz[dev] = 0;
    }
    int64_t want = doubles < (1 << 16) ? (1 << 16) : doubles + doubles / 2;
    if (hipMalloc((void**)&g_scratch[dev], sizeof(double) * want) != hipSuccess) return nullptr;
    g_scratch_sz[dev] = want;
  }
  return g_scratch[dev];
}

template <typename T>
static hipError_t upload(T** dst, const std::vector<double>& src) {
  std::vector<T> tmp(src.begin(), src.end());
  hipError_t e = hipMalloc((void**)dst, sizeof(T) * (tmp.empty() ? 1 : tmp.size()));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, tmp.data(), sizeof(T) * tmp.size(), hipMemcpyHostToDevice);
}

template <typename T>
static void free_ops(tp3b::DevOps<T>& d) {
  for (int k = 0; k < 4; ++k) {
    if (d.K[k]) (void)hipFree(d.K[k]);
    if (d.KT[k]) (void)hipFree(d.KT[k]);
  }
  for (int k = 0; k < 4; ++k) {
    T* ps[] = {d.Si[k], d.S[k], d.SiT[k], d.ST[k], d.lam[k]};
    for (T* p : ps)
      if (p) (void)hipFree(p);
  }
  for (int k = 0; k < 4; ++k) {
    T* fs[] = {d.frK[k], d.frS[k], d.frSi[k]};
    for (T* p : fs)
      if (p) (void)hipFree(p);
  }
  T* ps[] = {d.V, d.lamItem, d.lamItemY, d.work, d.G};
  for (T* p : ps)
    if (p) (void)hipFree(p);
  d = tp3b::DevOps<T>();
}

static std::vector<double> transpose(const std::vector<double>& A, int n) {
  std::vector<double> B((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) B[(size_t)j * n + i] = A[(size_t)i * n + j];
  return B;
}

// Host eigen-factors of the kinetic mode operators K_k = S_k diag(lam_k) S_k^{-1}.
struct PrecFactors {
  std::vector<double> S[4], Si[4], lam[4];
  std::vector<double> lamItem;   // 2D: lam_0[i1] + lam_1[i2]
  std::vector<double> lamItemY;  // 2D: lam_2[j1] + lam_3[j2]
};

template <typename T>
static tp3b_status upload_ops(tp3b_op op, tp3b::DevOps<T>& d, const std::vector<double>* Kh,
                              const PrecFactors& pf) {
  for (int k = 0; k < op->nmodes; ++k) {
    TP3B_HIP(upload(&d.K[k], Kh[k]));
    TP3B_HIP(upload(&d.KT[k], transpose(Kh[k], op->n[k])));
  }
  TP3B_HIP(upload(&d.V, op->Vh));
  if (op->have_prec) {
    // the last mode is applied from the right (transposed factors), the others
    // from the left
    const int last = op->nmodes - 1;
    for (int k = 0; k < op->nmodes; ++k) {
      if (k < last) {
        TP3B_HIP(upload(&d.Si[k], pf.Si[k]));
        TP3B_HIP(upload(&d.S[k], pf.S[k]));
      } else {
        TP3B_HIP(upload(&d.SiT[k], transpose(pf.Si[k], op->n[k])));
        TP3B_HIP(upload(&d.ST[k], transpose(pf.S[k], op->n[k])));
      }
      TP3B_HIP(upload(&d.lam[k], pf.lam[k]));
    }
    if (op->ndim == 2) {
      TP3B_HIP(upload(&d.lamItem, pf.lamItem));
      TP3B_HIP(upload(&d.lamItemY, pf.lamItemY));
    }
    TP3B_HIP(hipMalloc((void**)&d.work, sizeof(T) * op->N * op->work_vecs));
  }
  if (op->plane2d) {
    std::vector<double> F(tp3b::P2_FRAG);
    for (int k = 0; k < op->nmodes; ++k) {
      tp3b::plane2d_fragments(op->n[k], Kh[k].data(), F.data());
      TP3B_HIP(upload(&d.frK[k], F));
      if (op->have_prec) {
        tp3b::plane2d_fragments(op->n[k], pf.S[k].data(), F.data());
        TP3B_HIP(upload(&d.frS[k], F));
        tp3b::plane2d_fragments(op->n[k], pf.Si[k].data(), F.data());
        TP3B_HIP(upload(&d.frSi[k], F));
      }
    }
    if (!op->Gh.empty()) TP3B_HIP(upload(&d.G, op->Gh));
  }
  return TP3B_OK;
}

// -------------------------------------------------------------- applies
static int prec_index(bool f64, bool bf3) { return f64 ? TP3B_FP64 : (bf3 ? TP3B_BF16X3 : TP3B_FP32); }

// Vectors per group of the 2D plane passes: one at a time for FP64 vectors of
// 64 MB and more (a vector and its partial result then stay in the 256 MB
// Infinity Cache between the passes), the whole block otherwise.
template <typename T>
static int plane2d_vec_group(int64_t N, int nvec, bool prec = false) {
  if (sizeof(T) == 8 && N * (int64_t)sizeof(T) >= (int64_t)(64 << 20)) return prec ? 4 : 1;
  return std::max(nvec, 1);
}

static int tile_for(tp3b_op op, bool f64, bool bf3, int kind, int M, int Nc, int64_t nbatch) {
  if (op->tile_override >= 0) return op->tile_override;
  const int t = op->tuned[prec_index(f64, bf3)][kind];
  if (t >= 0) return t;
  return choose_tile(M, Nc, nbatch, f64);
}

int op_tile(tp3b_op op, bool f64, bool bf3, int kind, int64_t nbatch) {
  return tile_for(op, f64, bf3, kind, op->n[0], op->n[1], nbatch);
}

// One mode-product launch in the requested arithmetic.
static hipError_t modeprod(tp3b_op, const ModeProd<double>& a, int tile, hipStream_t s, bool) {
  return launch_modeprod(a, tile, s);
}
// The pre-split form of a constant operand (bf3_split_ops), or NULL.
static const unsigned short* bf3_split_of(const std::vector<tp3b_op_s::Bf3Split>& v, const float* m,
                                          int n) {
  for (const auto& e : v)
    if (e.src == m && e.n == n) return e.hl;
  return nullptr;
}
static hipError_t modeprod(tp3b_op op, const ModeProd<float>& a, int tile, hipStream_t s, bool bf3) {
  if (!bf3) return launch_modeprod(a, tile, s);
  ModeProd<float> b = a;
  b.Lhl = a.L ? bf3_split_of(op->bf3L, a.L, a.M) : nullptr;
  b.Rhl = a.R ? bf3_split_of(op->bf3R, a.R, a.Nc) : nullptr;
  return launch_modeprod_bf3(b, tile, s);
}

// BF16x3 products split their constant operands once: each FP32 mode operator
// that serves as a left operand (K, S^{-1}, S) in its own layout, each that serves
// as a right operand (K^T, S^{-T}, S^T) transposed, for modes whose size is a
// multiple of 32 (the K chunk of the BF16x3 tiles, so every octet a tile reads
// lies inside the matrix).
static tp3b_status bf3_split_ops(tp3b_op op) {
  const tp3b::DevOps<float>& d = op->d32;
  for (int k = 0; k < op->nmodes; ++k) {
    const int n = op->n[k];
    if (n % 32 != 0) continue;
    const float* lefts[] = {d.K[k], d.Si[k], d.S[k]};
    const float* rights[] = {d.KT[k], d.SiT[k], d.ST[k]};
    for (int side = 0; side < 2; ++side)
      for (const float* m : side == 0 ? lefts : rights) {
        if (!m) continue;
        unsigned short* hl = nullptr;
        TP3B_HIP(hipMalloc(&hl, sizeof(unsigned short) * 2 * (size_t)n * n));
        (side == 0 ? op->bf3L : op->bf3R).push_back({m, n, hl});
        TP3B_HIP(tp3b::launch_bf3_split(n, m, side, hl, nullptr));
      }
  }
  TP3B_HIP(hipDeviceSynchronize());
  return TP3B_OK;
}

template <>
tp3b::DevOps<double>& dev_ops<double>(tp3b_op op) { return op->d64; }
template <>
tp3b::DevOps<float>& dev_ops<float>(tp3b_op op) { return op->d32; }
template <typename T>
static tp3b::DevOps<T>& ops_for(tp3b_op op) { return dev_ops<T>(op); }

template <typename T>
tp3b_status apply_H_impl(tp3b_op op, int nvec, const T* X, int64_t ldx, T* Y, int64_t ldy,
                         const double* shifts, hipStream_t s, bool bf3) {
  tp3b::DevOps<T>& d = ops_for<T>(op);
  const bool f64 = sizeof(T) == 8;
  if (op->ndim == 1) {
    // Y = K_x W + W K_y^T + (V - shift) o W per vector (eq. (10)).
    ModeProd<T> a{};
    a.M = op->n[0];
    a.Nc = op->n[1];
    a.rs = op->n[1];
    a.bstride = 0;
    a.ldx = ldx;
    a.ldy = ldy;
    a.per_vec = 1;
    a.nbatch = nvec;
    a.X = X;
    a.Y = Y;
    a.L = d.K[0];
    a.R = d.KT[1];
    a.V = d.V;
    a.shifts = shifts;
    a.epi = EPI_V;
    a.acc = 0;
    TP3B_HIP(modeprod(op, a, tile_for(op, f64, bf3, 0, a.M, a.Nc, nvec), s, bf3));
    return TP3B_OK;
  }
  const int nx1 = op->n[0], nx2 = op->n[1], ny1 = op->n[2], ny2 = op->n[3];
  const int64_t Ny = (int64_t)ny1 * ny2;
  if (op->plane2d && !bf3) {
    // 2D (eq. (11)) in two passes over LDS-resident matrices: the x slabs at
    // every y index get K_x1 W + W K_x2^T (written to Y), then the y planes at
    // every (x1, x2) get K_y1 W + W K_y2^T + (V - s) o W added to it.
    tp3b::Plane2D<T> p{};
    p.prog = tp3b::P2_SUM;
    p.interleaved = 1;
    p.M = nx1; p.Nc = nx2;
    p.rs = (int64_t)nx2 * Ny; p.cs = Ny; p.js = 1;
    p.nmat = Ny;
    p.nvec = nvec;
    p.ldx = ldx; p.ldy = ldy;
    p.X = X; p.Y = Y;
    p.FA1 = d.frK[0]; p.FB1 = d.frK[1];
    p.same_ab = op->x_same_K;
    tp3b::Plane2D<T> q{};
    q.prog = tp3b::P2_SUM_V_ACC;
    q.interleaved = 0;
    q.M = ny1; q.Nc = ny2;
    q.rs = ny2; q.cs = 1; q.js = Ny;
    q.nmat = (int64_t)nx1 * nx2;
    q.nvec = nvec;
    q.ldx = ldx; q.ldy = ldy;
    q.X = X; q.Y = Y;
    q.FA1 = d.frK[2]; q.FB1 = d.frK[3];
    q.same_ab = op->y_same_K;
    q.V = d.V;
    q.G = d.G;
    q.mdiv = nx2;
    q.gscale = op->gscale;
    q.shifts = shifts;
    // Large FP64 vectors go through both passes one vector at a time, so that
    // the y pass finds the vector and the x part just written in the
    // Infinity Cache (c5: 134 MB per vector, 8 vectors: 1.75 against 1.95 ms
    // per apply); FP32 vectors are half as long and run as one block.
    const int vb = plane2d_vec_group<T>(op->N, nvec);
    for (int v0 = 0; v0 < nvec; v0 += vb) {
      const int nv = std::min(vb, nvec - v0);
      p.nvec = q.nvec = nv;
      p.X = q.X = X + (int64_t)v0 * ldx;
      p.Y = q.Y = Y + (int64_t)v0 * ldy;
      q.shifts = shifts ? shifts + v0 : nullptr;
      TP3B_HIP(tp3b::launch_plane2d(p, s));
      TP3B_HIP(tp3b::launch_plane2d(q, s));
    }
    return TP3B_OK;
  }
  // 2D (eq. (11)) for larger modes: pass A applies the two y modes and the
  // potential on every contiguous (y1, y2) plane; passes B1 and B2 accumulate
  // the x2 and x1 modes.
  {
    ModeProd<T> a{};
    a.M = ny1;
    a.Nc = ny2;
    a.rs = ny2;
    a.bstride = Ny;
    a.ldx = ldx;
    a.ldy = ldy;
    a.per_vec = nx1 * nx2;
    a.nbatch = nvec * nx1 * nx2;
    a.X = X;
    a.Y = Y;
    a.L = d.K[2];
    a.R = d.KT[3];
    a.V = d.V;
    a.shifts = shifts;
    a.epi = EPI_V;
    a.acc = 0;
    int tile = op->tile_override >= 0 ? op->tile_override : choose_tile(a.M, a.Nc, a.nbatch, f64);
    TP3B_HIP(modeprod(op, a, tile, s, bf3));
  }
  {
    ModeProd<T> a{};
    a.M = nx2;
    a.Nc = (int)Ny;
    a.rs = Ny;
    a.bstride = (int64_t)nx2 * Ny;
    a.ldx = ldx;
    a.ldy = ldy;
    a.per_vec = nx1;
    a.nbatch = nvec * nx1;
    a.X = X;
    a.Y = Y;
    a.L = d.K[1];
    a.R = nullptr;
    a.epi = EPI_NONE;
    a.acc = 1;
    int tile = op->tile_override >= 0 ? op->tile_override : choose_tile(a.M, a.Nc, a.nbatch, f64);
    TP3B_HIP(modeprod(op, a, tile, s, bf3));
  }
  {
    ModeProd<T> a{};
    a.M = nx1;
    a.Nc = (int)((int64_t)nx2 * Ny);
    a.rs = (int64_t)nx2 * Ny;
    a.bstride = 0;
    a.ldx = ldx;
    a.ldy = ldy;
    a.per_vec = 1;
    a.nbatch = nvec;
    a.X = X;
    a.Y = Y;
    a.L = d.K[0];
    a.R = nullptr;
    a.epi = EPI_NONE;
    a.acc = 1;
    int tile = op->tile_override >= 0 ? op->tile_override : choose_tile(a.M, a.Nc, a.nbatch, f64);
    TP3B_HIP(modeprod(op, a, tile, s, bf3));
  }
  return TP3B_OK;
}

template <typename T>
tp3b_status apply_prec_impl(tp3b_op op, int nvec, const T* X, int64_t ldx, T* Y, int64_t ldy,
                            hipStream_t s, bool bf3) {
  tp3b::DevOps<T>& d = ops_for<T>(op);
  const bool f64 = sizeof(T) == 8;
  const int64_t N = op->N;
  if (op->ndim == 2 && op->plane2d && !bf3) {
    // (K - sigma)^{-1} = (S_x1 x S_x2 x S_y1 x S_y2) diag(1 / (sum_k lam_k - sigma))
    // (S_x1^{-1} x ... x S_y2^{-1}) in four passes over LDS-resident matrices:
    // x slabs S_x1^{-1} W S_x2^{-T}; y planes [S_y1^{-1} W S_y2^{-T}] / Lambda;
    // y planes S_y1 W S_y2^T; x slabs S_x1 W S_x2^T (the first writes Y, the
    // others work in place).
    const int nx1 = op->n[0], nx2 = op->n[1], ny1 = op->n[2], ny2 = op->n[3];
    const int64_t Ny = (int64_t)ny1 * ny2;
    // large FP64 vectors in groups of four: each pass after the first then
    // finds part of its input in the Infinity Cache, and each launch has four
    // vectors over which to spread the fill and drain of its persistent
    // workgroups (c5, 8 vectors: 2.91 ms against 3.02 ms one at a time and
    // 2.93 ms for all eight at once)
    const int vb = plane2d_vec_group<T>(N, nvec, true);
    for (int v0 = 0; v0 < nvec; v0 += vb) {
      const int nv = std::min(vb, nvec - v0);
      const T* Xv = X + (int64_t)v0 * ldx;
      T* Yv = Y + (int64_t)v0 * ldy;
      tp3b::Plane2D<T> p{};
      p.prog = tp3b::P2_SEQ2;
      p.interleaved = 1;
      p.M = nx1; p.Nc = nx2;
      p.rs = (int64_t)nx2 * Ny; p.cs = Ny; p.js = 1;
      p.nmat = Ny;
      p.nvec = nv;
      p.ldx = ldx; p.ldy = ldy;
      p.X = Xv; p.Y = Yv;
      p.FA1 = d.frSi[0]; p.FB1 = d.frSi[1];
      p.same_ab = op->x_same_S;
      // equal x modes (FP64: both 64 wide, the y groups in fours and 16-byte
      // aligned vectors, for the four-matrix kernel)
      const bool seq4 =
          op->x_same_S &&
          (sizeof(T) == 4 ||
           (nx1 == tp3b::P2_MAXN && nx2 == tp3b::P2_MAXN && Ny % 4 == 0 && ldx % 2 == 0 &&
            ldy % 2 == 0 && (uintptr_t)X % 16 == 0 && (uintptr_t)Y % 16 == 0));
      if (seq4) {
        // the two x-slab transforms and the divide in one pass between the two
        // y-plane transforms (the mode transforms commute), so the strided x
        // slabs are read and written once: y planes S_y1^{-1} W S_y2^{-T}; x
        // slabs S_x (S_x^{-1} W S_x^{-T} / Lambda) S_x^T; y planes S_y1 W S_y2^T
        tp3b::Plane2D<T> q{};
        q.prog = tp3b::P2_SEQ2;
        q.interleaved = 0;
        q.M = ny1; q.Nc = ny2;
        q.rs = ny2; q.cs = 1; q.js = Ny;
        q.nmat = (int64_t)nx1 * nx2;
        q.nvec = nv;
        q.ldx = ldx; q.ldy = ldy;
        q.X = Xv; q.Y = Yv;
        q.FA1 = d.frSi[2]; q.FB1 = d.frSi[3];
        q.same_ab = op->y_same_S;
        TP3B_HIP(tp3b::launch_plane2d(q, s));
        p.prog = tp3b::P2_SEQ4_DIV;
        p.X = Yv; p.ldx = ldy;
        p.FA2 = d.frS[0];
        p.lamM = d.lamItemY; p.lamR = d.lam[0]; p.lamC = d.lam[1];
        p.sigma = op->sigma;
        TP3B_HIP(tp3b::launch_plane2d(p, s));
        q.X = Yv; q.ldx = ldy;
        q.FA1 = d.frS[2]; q.FB1 = d.frS[3];
        TP3B_HIP(tp3b::launch_plane2d(q, s));
        continue;
      }
      TP3B_HIP(tp3b::launch_plane2d(p, s));
      tp3b::Plane2D<T> q{};
      q.prog = tp3b::P2_SEQ2_DIV;
      q.interleaved = 0;
      q.M = ny1; q.Nc = ny2;
      q.rs = ny2; q.cs = 1; q.js = Ny;
      q.nmat = (int64_t)nx1 * nx2;
      q.nvec = nv;
      q.ldx = ldy; q.ldy = ldy;
      q.X = Yv; q.Y = Yv;
      q.FA1 = d.frSi[2]; q.FB1 = d.frSi[3];
      q.same_ab = op->y_same_S;
      q.lamM = d.lamItem; q.lamR = d.lam[2]; q.lamC = d.lam[3];
      q.sigma = op->sigma;
      TP3B_HIP(tp3b::launch_plane2d(q, s));
      q.prog = tp3b::P2_SEQ2;
      q.FA1 = d.frS[2]; q.FB1 = d.frS[3];
      TP3B_HIP(tp3b::launch_plane2d(q, s));
      p.X = Yv; p.ldx = ldy;
      p.FA1 = d.frS[0]; p.FB1 = d.frS[1];
      TP3B_HIP(tp3b::launch_plane2d(p, s));
    }
    return TP3B_OK;
  }
  if (op->ndim == 2) {
    // (K - sigma)^{-1} = (S_1 x S_2 x S_3 x S_4) diag(1 / (sum_k lam_k - sigma))
    // (S_1^{-1} x ... x S_4^{-1}): eight single-mode products, the divide fused
    // into the fourth; the work buffer and Y alternate as intermediates.
    const int n0 = op->n[0], n1 = op->n[1], n2 = op->n[2], n3 = op->n[3];
    for (int v0 = 0; v0 < nvec; v0 += op->work_vecs) {
      const int nv = (nvec - v0 < op->work_vecs) ? nvec - v0 : op->work_vecs;
      const T* Xc = X + (int64_t)v0 * ldx;
      T* Yc = Y + (int64_t)v0 * ldy;
      // mode k, factor F (left operand for k < 3, right operand for k = 3)
      auto pass = [&](int k, const T* F, const T* in, int64_t ldin, T* out, int64_t ldout,
                      bool divide) -> tp3b_status {
        ModeProd<T> a{};
        a.X = in; a.ldx = ldin; a.Y = out; a.ldy = ldout;
        a.epi = EPI_NONE;
        switch (k) {
          case 0: a.M = n0; a.Nc = n1 * n2 * n3; a.rs = a.Nc; a.bstride = 0; a.per_vec = 1; break;
          case 1: a.M = n1; a.Nc = n2 * n3; a.rs = a.Nc; a.bstride = (int64_t)n1 * a.Nc; a.per_vec = n0; break;
          default: a.M = n2; a.Nc = n3; a.rs = n3; a.bstride = (int64_t)n2 * n3; a.per_vec = n0 * n1; break;
        }
        a.nbatch = nv * a.per_vec;
        if (k < 3) a.L = F; else a.R = F;
        if (divide) {
          a.epi = EPI_DIV;
          a.lamL = d.lam[2];
          a.lamR = d.lam[3];
          a.lamItem = d.lamItem;
          a.sigma = op->sigma;
        }
        const int tile = op->tile_override >= 0 ? op->tile_override : choose_tile(a.M, a.Nc, a.nbatch, f64);
        TP3B_HIP(modeprod(op, a, tile, s, bf3));
        return TP3B_OK;
      };
      T* W = d.work;
      tp3b_status st = TP3B_OK;
      if (st == TP3B_OK) st = pass(0, d.Si[0], Xc, ldx, W, N, false);
      if (st == TP3B_OK) st = pass(1, d.Si[1], W, N, Yc, ldy, false);
      if (st == TP3B_OK) st = pass(2, d.Si[2], Yc, ldy, W, N, false);
      if (st == TP3B_OK) st = pass(3, d.SiT[3], W, N, Yc, ldy, true);
      if (st == TP3B_OK) st = pass(3, d.ST[3], Yc, ldy, W, N, false);
      if (st == TP3B_OK) st = pass(2, d.S[2], W, N, Yc, ldy, false);
      if (st == TP3B_OK) st = pass(1, d.S[1], Yc, ldy, W, N, false);
      if (st == TP3B_OK) st = pass(0, d.S[0], W, N, Yc, ldy, false);
      if (st != TP3B_OK) return st;
    }
    return TP3B_OK;
  }
  const int nx = op->n[0], ny = op->n[1];
  // Z = Sx [ (Sx^{-1} B Sy^{-T}) / (lx_i + ly_j - sigma) ] Sy^T, four mode
  // products; the work buffer and Y alternate as intermediates.
  for (int v0 = 0; v0 < nvec; v0 += op->work_vecs) {
    const int nv = (nvec - v0 < op->work_vecs) ? nvec - v0 : op->work_vecs;
    const T* Xc = X + (int64_t)v0 * ldx;
    T* Yc = Y + (int64_t)v0 * ldy;
    ModeProd<T> a{};
    a.M = nx;
    a.Nc = ny;
    a.rs = ny;
    a.per_vec = 1;
    a.nbatch = nv;
    a.sigma = op->sigma;
    const int tile = tile_for(op, f64, bf3, 1, nx, ny, nv);
    // 1: W = Sx^{-1} B
    a.X = Xc; a.ldx = ldx; a.Y = d.work; a.ldy = N;
    a.L = d.Si[0]; a.R = nullptr; a.epi = EPI_NONE;
    TP3B_HIP(modeprod(op, a, tile, s, bf3));
    // 2: Y = (W Sy^{-T}) / (lx_i + ly_j - sigma)
    a.X = d.work; a.ldx = N; a.Y = Yc; a.ldy = ldy;
    a.L = nullptr; a.R = d.SiT[1]; a.epi = EPI_DIV; a.lamL = d.lam[0]; a.lamR = d.lam[1];
    TP3B_HIP(modeprod(op, a, tile, s, bf3));
    // 3: W = Sx Y
    a.X = Yc; a.ldx = ldy; a.Y = d.work; a.ldy = N;
    a.L = d.S[0]; a.R = nullptr; a.epi = EPI_NONE;
    TP3B_HIP(modeprod(op, a, tile, s, bf3));
    // 4: Y = W Sy^T
    a.X = d.work; a.ldx = N; a.Y = Yc; a.ldy = ldy;
    a.L = nullptr; a.R = d.ST[1]; a.epi = EPI_NONE;
    TP3B_HIP(modeprod(op, a, tile, s, bf3));
  }
  return TP3B_OK;
}

template tp3b_status apply_H_impl<double>(tp3b_op, int, const double*, int64_t, double*, int64_t,
                                          const double*, hipStream_t, bool);
template tp3b_status apply_H_impl<float>(tp3b_op, int, const float*, int64_t, float*, int64_t,
                                         const double*, hipStream_t, bool);
template tp3b_status apply_prec_impl<double>(tp3b_op, int, const double*, int64_t, double*,
                                             int64_t, hipStream_t, bool);
template tp3b_status apply_prec_impl<float>(tp3b_op, int, const float*, int64_t, float*, int64_t,
                                            hipStream_t, bool);

// ------------------------------------------------------------ block orth
// A column keeping less than this fraction of its norm after projection counts
// as dependent.  Cholesky-QR forms the Gram matrix, whose pivots carry absolute
// errors of order eps |x|^2, so dependence is only detectable above ~sqrt(eps).
constexpr double kDropTol = 1e-7;
// The scratch layout shared by block_orth_queue and block_orth_impl: dot
// partials, C1, C2 ((nq+1) x nx each), G, R1, R2 (nx x nx), n0 (nx + 1), then
// 2 nx + 1 ints of flags.
int64_t orth_scratch_doubles(int64_t N, int nq, int nx) {
  const int pmax = nq > nx ? nq : nx;
  return dot_scratch_doubles(N, pmax, nx) + 4 * (int64_t)(nq + 1) * nx + 6 * (int64_t)nx * nx +
         2 * nx + 64;
}

tp3b_status block_orth_queue(int64_t N, int nq, const double* Q, int64_t ldq, int nx, double* X,
                             int64_t ldx, int* dflags, hipStream_t s, const double* Xin,
                             double* scr_in) {
  if (!Xin) Xin = X;
  if (Xin != X && nq <= 0)
    TP3B_HIP(hipMemcpy2DAsync(X, sizeof(double) * ldx, Xin, sizeof(double) * ldx, sizeof(double) * N,
                              nx, hipMemcpyDeviceToDevice, s));
  if (nq <= 0) Xin = X;
  const int pmax = nq > nx ? nq : nx;
  double* scr = scr_in ? scr_in : dot_scratch(orth_scratch_doubles(N, nq, nx));
  if (!scr) return fail(TP3B_ENOMEM, "block_orth: scratch allocation failed");
  double* part = scr;
  double* C1 = part + dot_scratch_doubles(N, pmax, nx);
  double* C2 = C1 + (int64_t)(nq + 1) * nx;
  double* G = C2 + (int64_t)(nq + 1) * nx;
  double* R1 = G + (int64_t)nx * nx;
  double* R2 = R1 + (int64_t)nx * nx;
  double* n0 = R2 + (int64_t)nx * nx;
  int* fl2 = (int*)(n0 + nx + 1) + nx + 1;  // second Cholesky (no test)
  int* fl1 = dflags;                        // first Cholesky: dependence flags
  int* nonfin = dflags + nx;                // non-finite input
  // the dependence test reads the input norms on the device
  TP3B_HIP(launch_dot_tn<double, double>(N, nx, nx, Xin, ldx, Xin, ldx, G, nx, part, s));
  TP3B_HIP(launch_gram_diag(nx, G, n0, nonfin, s));
  bool gram_done = false;
  if (nq > 0) {
    // the first pass reads the input and writes X = Xin - Q C1
    TP3B_HIP(launch_dot_tn<double, double>(N, nq, nx, Q, ldq, Xin, ldx, C1, nq, part, s));
    // long blocks: each update also forms the next dot on the rows it has just
    // written (the second pass's coefficients, then the Gram matrix), so Q and
    // X are not read again for them
    if (gemm_dot_long_fits(N, nq, nx, Q, ldq, Xin, X, ldx)) {
      TP3B_HIP(launch_gemm_dot_long(N, nq, nx, Q, ldq, C1, Xin, X, ldx, 0, C2, nq, part, s));
      TP3B_HIP(launch_gemm_dot_long(N, nq, nx, Q, ldq, C2, X, X, ldx, 1, G, nx, part, s));
      gram_done = true;
    } else {
      TP3B_HIP(launch_gemm_nn_x0<double>(N, nq, nx, -1.0, Q, ldq, C1, nq, 1.0, Xin, ldx, X, ldx, s));
      TP3B_HIP(launch_dot_tn<double, double>(N, nq, nx, Q, ldq, X, ldx, C2, nq, part, s));
      TP3B_HIP(launch_gemm_nn<double>(N, nq, nx, -1.0, Q, ldq, C2, nq, 1.0, X, ldx, s));
    }
  }
  if (!gram_done) TP3B_HIP(launch_dot_tn<double, double>(N, nx, nx, X, ldx, X, ldx, G, nx, part, s));
  TP3B_HIP(launch_chol_small(nx, G, n0, kDropTol, R1, fl1, s));
  TP3B_HIP(launch_trsm_right(N, nx, R1, X, ldx, s));
  TP3B_HIP(launch_dot_tn<double, double>(N, nx, nx, X, ldx, X, ldx, G, nx, part, s));
  // the second factorisation leaves the columns the first found dependent out,
  // so the independent columns keep exactly their span (the flagged ones are
  // replaced by the caller)
  TP3B_HIP(launch_chol_small(nx, G, n0, 0.0, R2, fl2, s, fl1));
  TP3B_HIP(launch_trsm_right(N, nx, R2, X, ldx, s));
  return TP3B_OK;
}

tp3b_status block_orth_impl(int64_t N, int nq, const double* Q, int64_t ldq, int nx, double* X,
                            int64_t ldx, double* C_qx, double* R_xx, int* rank, uint64_t seed,
                            hipStream_t s) {
  const int pmax = nq > nx ? nq : nx;
  double* scr = dot_scratch(orth_scratch_doubles(N, nq, nx));
  if (!scr) return fail(TP3B_ENOMEM, "block_orth: scratch allocation failed");
  double* part = scr;
  double* C1 = part + dot_scratch_doubles(N, pmax, nx);
  double* C2 = C1 + (int64_t)(nq + 1) * nx;
  double* G = C2 + (int64_t)(nq + 1) * nx;
  double* R1 = G + (int64_t)nx * nx;
  double* R2 = R1 + (int64_t)nx * nx;
  double* n0 = R2 + (int64_t)nx * nx;
  int* flags = (int*)(n0 + nx + 1);
  std::vector<double> hG((size_t)nx * nx), hR1((size_t)nx * nx), hR2((size_t)nx * nx);
  std::vector<double> hC1((size_t)(nq + 1) * nx, 0.0), hC2((size_t)(nq + 1) * nx, 0.0);
  std::vector<int> hflags(nx + 1, 0);
  int deficient = 0;

  if (!C_qx && !R_xx) {
    // Without factors to return, the whole sequence is queued with one host
    // round trip at the end (block_orth_queue).  A dependent column (rare) is
    // replaced by a random vector and the general path below runs on the
    // result: both factorisations of the queued Cholesky-QR leave a dependent
    // column out of the others' factors, so the independent columns come out
    // as an orthonormal basis of exactly their own projected span.
    tp3b_status qs = block_orth_queue(N, nq, Q, ldq, nx, X, ldx, flags, s);
    if (qs != TP3B_OK) return qs;
    TP3B_HIP(hipMemcpyAsync(hflags.data(), flags, sizeof(int) * (nx + 1), hipMemcpyDeviceToHost, s));
    TP3B_HIP(hipStreamSynchronize(s));
    if (hflags[nx]) return fail(TP3B_ENONFINITE, "block_orth: non-finite input");
    int bad = 0;
    for (int j = 0; j < nx; ++j) bad += hflags[j];
    if (!bad) {
      if (rank) *rank = nx;
      return TP3B_OK;
    }
    for (int j = 0; j < nx; ++j)
      if (hflags[j]) {
        ++deficient;
        TP3B_HIP(launch_hash_fill(N, X + (int64_t)j * ldx, seed, (uint64_t)(1000 + j), s));
      }
  }

  // Input column norms (for the rank test) and the finiteness check.
  TP3B_HIP(launch_dot_tn<double, double>(N, nx, nx, X, ldx, X, ldx, G, nx, part, s));
  TP3B_HIP(hipMemcpyAsync(hG.data(), G, sizeof(double) * nx * nx, hipMemcpyDeviceToHost, s));
  TP3B_HIP(hipStreamSynchronize(s));
  std::vector<double> hn0(nx);
  for (int j = 0; j < nx; ++j) {
    hn0[j] = hG[(size_t)j * nx + j];
    if (!std::isfinite(hn0[j])) return fail(TP3B_ENONFINITE, "block_orth: non-finite input");
  }
  std::vector<int> replaced(nx, 0);
  for (int attempt = 0; attempt < 4; ++attempt) {
    TP3B_HIP(hipMemcpyAsync(n0, hn0.data(), sizeof(double) * nx, hipMemcpyHostToDevice, s));
    // Two classical Gram-Schmidt passes against Q.
    if (nq > 0) {
      TP3B_HIP(launch_dot_tn<double, double>(N, nq, nx, Q, ldq, X, ldx, C1, nq, part, s));
      TP3B_HIP(launch_gemm_nn<double>(N, nq, nx, -1.0, Q, ldq, C1, nq, 1.0, X, ldx, s));
      TP3B_HIP(launch_dot_tn<double, double>(N, nq, nx, Q, ldq, X, ldx, C2, nq, part, s));
      TP3B_HIP(launch_gemm_nn<double>(N, nq, nx, -1.0, Q, ldq, C2, nq, 1.0, X, ldx, s));
    }
    // Cholesky-QR, twice.
    TP3B_HIP(launch_dot_tn<double, double>(N, nx, nx, X, ldx, X, ldx, G, nx, part, s));
    TP3B_HIP(launch_chol_small(nx, G, n0, kDropTol, R1, flags, s));
    TP3B_HIP(hipMemcpyAsync(hflags.data(), flags, sizeof(int) * nx, hipMemcpyDeviceToHost, s));
    TP3B_HIP(hipStreamSynchronize(s));
    int bad = 0;
    for (int j = 0; j < nx; ++j) bad += hflags[j];
    if (bad && attempt < 3) {
      // Replace the dependent columns by pseudo-random vectors and redo.
      for (int j = 0; j < nx; ++j) {
        if (!hflags[j]) continue;
        if (!replaced[j]) ++deficient;
        replaced[j] = 1;
        TP3B_HIP(launch_hash_fill(N, X + (int64_t)j * ldx, seed, (uint64_t)(attempt * 64 + j), s));
        hn0[j] = 0.0;  // recomputed below
      }
      TP3B_HIP(launch_dot_tn<double, double>(N, nx, nx, X, ldx, X, ldx, G, nx, part, s));
      TP3B_HIP(hipMemcpyAsync(hG.data(), G, sizeof(double) * nx * nx, hipMemcpyDeviceToHost, s));
      TP3B_HIP(hipStreamSynchronize(s));
      for (int j = 0; j < nx; ++j)
        if (replaced[j]) hn0[j] = hG[(size_t)j * nx + j];
      if (nq > 0) {
        TP3B_HIP(hipMemcpyAsync(hC1.data(), C1, sizeof(double) * nq * nx, hipMemcpyDeviceToHost, s));
      }
      continue;
    }
    if (bad) return fail(TP3B_EDEVICE, "block_orth: could not complete the basis");
    TP3B_HIP(launch_trsm_right(N, nx, R1, X, ldx, s));
    TP3B_HIP(launch_dot_tn<double, double>(N, nx, nx, X, ldx, X, ldx, G, nx, part, s));
    std::vector<double> ones(nx, 0.0);
    TP3B_HIP(hipMemcpyAsync(n0, ones.data(), sizeof(double) * nx, hipMemcpyHostToDevice, s));
    TP3B_HIP(launch_chol_small(nx, G, n0, 0.0, R2, flags, s));
    TP3B_HIP(launch_trsm_right(N, nx, R2, X, ldx, s));
    TP3B_HIP(hipMemcpyAsync(hR1.data(), R1, sizeof(double) * nx * nx, hipMemcpyDeviceToHost, s));
    TP3B_HIP(hipMemcpyAsync(hR2.data(), R2, sizeof(double) * nx * nx, hipMemcpyDeviceToHost, s));
    if (nq > 0) {
      TP3B_HIP(hipMemcpyAsync(hC1.data(), C1, sizeof(double) * nq * nx, hipMemcpyDeviceToHost, s));
      TP3B_HIP(hipMemcpyAsync(hC2.data(), C2, sizeof(double) * nq * nx, hipMemcpyDeviceToHost, s));
    }
    TP3B_HIP(hipStreamSynchronize(s));
    break;
  }
  if (rank) *rank = nx - deficient;
  if (R_xx) {
    // R = R2 R1 (both upper triangular, column-major).
    std::vector<double> R((size_t)nx * nx, 0.0);
    for (int j = 0; j < nx; ++j)
      for (int i = 0; i <= j; ++i) {
        double acc = 0.0;
        for (int k = i; k <= j; ++k) acc += hR2[i + (size_t)k * nx] * hR1[k + (size_t)j * nx];
        R[i + (size_t)j * nx] = replaced[j] ? 0.0 : acc;
      }
    TP3B_HIP(hipMemcpy(R_xx, R.data(), sizeof(double) * nx * nx, hipMemcpyHostToDevice));
  }
  if (C_qx && nq > 0) {
    std::vector<double> C((size_t)nq * nx);
    for (size_t e = 0; e < C.size(); ++e) C[e] = hC1[e] + hC2[e];
    TP3B_HIP(hipMemcpy(C_qx, C.data(), sizeof(double) * nq * nx, hipMemcpyHostToDevice));
  }
  return TP3B_OK;
}

template <typename T>
static tp3b_status autotune_impl(tp3b_op op, int nvec, int reps, double* best_ms, bool bf3) {
  const int pi = prec_index(sizeof(T) == 8, bf3);
  T *X = nullptr, *Y = nullptr;
  hipEvent_t e0, e1;
  TP3B_HIP(hipMalloc((void**)&X, sizeof(T) * op->N * nvec));
  if (hipMalloc((void**)&Y, sizeof(T) * op->N * nvec) != hipSuccess) {
    (void)hipFree(X);
    return fail(TP3B_ENOMEM, "autotune: scratch allocation failed");
  }
  tp3b_status st = TP3B_OK;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  for (int kind = 0; kind < 2 && st == TP3B_OK; ++kind) {
    if (kind == 1 && (op->ndim != 1 || !op->have_prec)) break;
    double best = 1e300;
    int best_tile = -1;
    // The timing does not depend on the values; a zero block avoids any
    // overflow in the preconditioner's divide.
    (void)hipMemset(X, 0, sizeof(T) * op->N * nvec);
    const int saved = op->tile_override;
    for (int tile = 0; tile < NUM_TILE_CFGS; ++tile) {
      const int tm = tile_rows(tile), tn = tile_cols(tile);
      if (tm > 32 && (tm > op->n[op->ndim == 1 ? 0 : 2] || tn > op->n[op->ndim == 1 ? 1 : 3])) continue;
      if (bf3 && tm == 32) continue;  // the smallest BF16x3 tile is 64 x 64
      op->tile_override = tile;
      auto run = [&]() -> tp3b_status {
        return kind == 0 ? apply_H_impl<T>(op, nvec, X, op->N, Y, op->N, nullptr, nullptr, bf3)
                         : apply_prec_impl<T>(op, nvec, X, op->N, Y, op->N, nullptr, bf3);
      };
      st = run();  // warm-up
      if (st != TP3B_OK) break;
      (void)hipEventRecord(e0, nullptr);
      for (int r = 0; r < reps && st == TP3B_OK; ++r) st = run();
      (void)hipEventRecord(e1, nullptr);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double per = ms / reps;
      if (per < best) {
        best = per;
        best_tile = tile;
      }
    }
    op->tile_override = saved;
    if (st == TP3B_OK) {
      op->tuned[pi][kind] = best_tile;
      if (best_ms) best_ms[kind] = best;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(X);
  (void)hipFree(Y);
  return st;
}

}  // namespace tp3b

using namespace tp3b;

extern "C" {

const char* tp3b_last_error(void) { return g_err.c_str(); }

tp3b_status tp3b_create(const tp3b_problem_desc* desc, void* stream, tp3b_op* out) {
  try {
    (void)stream;
    if (!desc || !out) return fail(TP3B_EINVAL, "tp3b_create: null descriptor or output");
    *out = nullptr;
    if (desc->ndim != 1 && desc->ndim != 2) return fail(TP3B_EINVAL, "ndim must be 1 or 2");
    const int nm = 2 * desc->ndim;
    int64_t N = 1;
    for (int k = 0; k < nm; ++k) {
      if (desc->n[k] < 2 || desc->n[k] > 8192) return fail(TP3B_EINVAL, "mode sizes must be in [2, 8192]");
      if (!(desc->L[k] > 0)) return fail(TP3B_EINVAL, "half-widths L must be positive");
      N *= desc->n[k];
    }
    if (!(desc->c_x > 0) || !(desc->c_y > 0)) return fail(TP3B_EINVAL, "c_x and c_y must be positive");
    if (desc->pot < TP3B_POT_GAUSS || desc->pot > TP3B_POT_TABLE) return fail(TP3B_EINVAL, "unknown potential");
    if (desc->pot == TP3B_POT_TABLE && !desc->V_table) return fail(TP3B_EINVAL, "TP3B_POT_TABLE needs V_table");
    if (desc->pot == TP3B_POT_GAUSS && !(desc->width > 0)) return fail(TP3B_EINVAL, "width must be positive");
    if (desc->ndim == 2 && (desc->n[0] != desc->n[1] || desc->n[2] != desc->n[3]))
      return fail(TP3B_ENOTSUP, "2D operators need n[0] == n[1] and n[2] == n[3]");
    if (desc->grid != TP3B_GRID_CGL && desc->grid != TP3B_GRID_MAPPED)
      return fail(TP3B_EINVAL, "unknown grid");
    for (int k = 0; k < nm; ++k) {
      if (desc->parity[k] < -1 || desc->parity[k] > 1) return fail(TP3B_EINVAL, "parity must be -1, 0 or +1");
      if (desc->parity[k] != 0 && desc->grid != TP3B_GRID_MAPPED)
        return fail(TP3B_EINVAL, "parity half grids need TP3B_GRID_MAPPED");
    }
  
    tp3b_op op = new tp3b_op_s();
    op->ndim = desc->ndim;
    op->nmodes = nm;
    op->N = N;
    op->cx = desc->c_x;
    op->cy = desc->c_y;
    op->pot = desc->pot;
    op->v0 = desc->v0;
    op->width = desc->width;
    op->mu_hl = desc->mu_hl > 0 ? desc->mu_hl : 1.0;
    (void)hipGetDevice(&op->device);
    std::vector<double> x[4];
    for (int k = 0; k < nm; ++k) {
      op->n[k] = desc->n[k];
      op->L[k] = desc->L[k];
      mode_grid(desc, k, op->D2h[k], x[k]);
    }
    // Potential V = u(|y - x/2|) + u(|y + x/2|) on the tensor grid (eq. (3)).
    op->Vh.resize(N);
    if (desc->pot == TP3B_POT_TABLE) {
      std::memcpy(op->Vh.data(), desc->V_table, sizeof(double) * N);
    } else if (desc->ndim == 1) {
      for (int i = 0; i < op->n[0]; ++i)
        for (int j = 0; j < op->n[1]; ++j) {
          const double xi = x[0][i], yj = x[1][j];
          op->Vh[(size_t)i * op->n[1] + j] = pair_pot(op->pot, std::fabs(yj - 0.5 * xi), op->v0, op->width) +
                                             pair_pot(op->pot, std::fabs(yj + 0.5 * xi), op->v0, op->width);
        }
    } else {
      const int a = op->n[0], b = op->n[1], c = op->n[2], e = op->n[3];
      for (int i1 = 0; i1 < a; ++i1)
        for (int i2 = 0; i2 < b; ++i2)
          for (int j1 = 0; j1 < c; ++j1)
            for (int j2 = 0; j2 < e; ++j2) {
              const double x1 = x[0][i1], x2 = x[1][i2], y1 = x[2][j1], y2 = x[3][j2];
              const double rm = std::hypot(y1 - 0.5 * x1, y2 - 0.5 * x2);
              const double rp = std::hypot(y1 + 0.5 * x1, y2 + 0.5 * x2);
              op->Vh[(((size_t)i1 * b + i2) * c + j1) * e + j2] =
                  pair_pot(op->pot, rm, op->v0, op->width) + pair_pot(op->pot, rp, op->v0, op->width);
            }
    }
    // 2D operators whose modes fit the LDS-resident passes; for the Gaussian
    // shapes the potential is also kept as separable factors,
    // exp(-|y -+ x/2|^2 s) = exp(-(y1 -+ x1/2)^2 s) exp(-(y2 -+ x2/2)^2 s).
    if (desc->ndim == 2) {
      op->plane2d = true;
      for (int k = 0; k < nm; ++k) op->plane2d = op->plane2d && op->n[k] <= tp3b::P2_MAXN;
      const bool gauss = desc->pot == TP3B_POT_GAUSS || desc->pot == TP3B_POT_GAUSS_PAPER;
      if (op->plane2d && gauss) {
        const double sc = desc->pot == TP3B_POT_GAUSS ? 1.0 / (2.0 * op->width * op->width) : 1.0;
        const int P = tp3b::P2_MAXN;
        op->Gh.assign((size_t)4 * P * P, 0.0);
        for (int h = 0; h < 2; ++h)  // h = 0: (x1, y1) -> G[0], G[1]; h = 1: (x2, y2) -> G[2], G[3]
          for (int i = 0; i < op->n[h]; ++i)
            for (int j = 0; j < op->n[2 + h]; ++j) {
              const double xi = x[h][i], yj = x[2 + h][j];
              const double dm = yj - 0.5 * xi, dp = yj + 0.5 * xi;
              op->Gh[(size_t)(2 * h) * P * P + (size_t)i * P + j] = std::exp(-dm * dm * sc);
              op->Gh[(size_t)(2 * h + 1) * P * P + (size_t)i * P + j] = std::exp(-dp * dp * sc);
            }
        op->gscale = -op->v0;
      }
    }
    // Scaled kinetic factors K_k = -c D2_k.
    std::vector<double> Kh[4];
    for (int k = 0; k < nm; ++k) {
      const double c = (k < nm / 2) ? op->cx : op->cy;
      Kh[k].resize(op->D2h[k].size());
      for (size_t e = 0; e < Kh[k].size(); ++e) Kh[k][e] = -c * op->D2h[k][e];
    }
    // Preconditioner shift: two-body ground energy on the y grid (Sec. 4.2).
    if (std::isnan(desc->sigma)) {
      const int ky = nm / 2, n = op->n[ky];
      std::vector<double> A((size_t)n * n), wr(n), wi(n);
      const double ck = 1.0 / (2.0 * op->mu_hl);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = -ck * op->D2h[ky][(size_t)i * n + j];
      if (desc->pot == TP3B_POT_TABLE) {
        op->sigma = 0.0;
      } else {
        for (int i = 0; i < n; ++i) A[(size_t)i * n + i] += pair_pot(op->pot, std::fabs(x[ky][i]), op->v0, op->width);
        if (!real_schur(n, A.data(), nullptr, wr.data(), wi.data())) {
          delete op;
          return fail(TP3B_EDEVICE, "two-body eigenvalue iteration did not converge");
        }
        double m = wr[0];
        for (int i = 1; i < n; ++i) m = std::min(m, wr[i]);
        op->sigma = m;
      }
    } else {
      op->sigma = desc->sigma;
    }
    // Fast-diagonalisation factors of the kinetic operator, one per mode: the
    // shifted Kronecker sum is then inverted exactly by mode products and a
    // pointwise divide (1D: the Sylvester equation of eq. (14); 2D: the same
    // construction over four modes).
    PrecFactors pf;
    {
      bool ok = true;
      for (int k = 0; k < nm && ok; ++k) {
        const int n = op->n[k];
        pf.S[k].resize((size_t)n * n);
        pf.Si[k].resize((size_t)n * n);
        pf.lam[k].resize(n);
        ok = eigen_decompose_real(n, Kh[k].data(), pf.S[k].data(), pf.Si[k].data(), pf.lam[k].data());
      }
      if (ok) {
        // smallest |denominator|: sums over the x modes against sums over the y modes
        std::vector<double> xs, ys;
        if (op->ndim == 1) {
          xs = pf.lam[0];
          ys = pf.lam[1];
        } else {
          for (double a : pf.lam[0])
            for (double b : pf.lam[1]) xs.push_back(a + b);
          for (double a : pf.lam[2])
            for (double b : pf.lam[3]) ys.push_back(a + b);
          pf.lamItem = xs;   // index i1 * n1 + i2
          pf.lamItemY = ys;  // index j1 * n3 + j2
        }
        std::vector<double> ysort = ys;
        std::sort(ysort.begin(), ysort.end());
        double mn = 1e300;
        for (double a : xs) {
          const double want = op->sigma - a;
          auto it = std::lower_bound(ysort.begin(), ysort.end(), want);
          if (it != ysort.end()) mn = std::min(mn, std::fabs(a + *it - op->sigma));
          if (it != ysort.begin()) mn = std::min(mn, std::fabs(a + *(it - 1) - op->sigma));
        }
        op->lam_min = mn;
        op->have_prec = mn > 0;
      }
      // lower bound of the spectrum (Weyl, continuous problem): the eigensolver's
      // starting target
      double lo = op->Vh.empty() ? 0.0 : *std::min_element(op->Vh.begin(), op->Vh.end());
      for (int k = 0; k < nm; ++k) {
        if (pf.lam[k].empty() || !ok) {
          // no real eigen-factors: Gershgorin bound of the mode operator
          double g = 1e300;
          const int n = op->n[k];
          for (int i = 0; i < n; ++i) {
            double off = 0.0;
            for (int j = 0; j < n; ++j)
              if (j != i) off += std::fabs(Kh[k][(size_t)i * n + j]);
            g = std::min(g, Kh[k][(size_t)i * n + i] - off);
          }
          lo += g;
        } else {
          lo += *std::min_element(pf.lam[k].begin(), pf.lam[k].end());
        }
      }
      op->spec_lo = lo;
      // preconditioner work buffer: up to 64 vectors, at most 4 GiB (FP64)
      const int64_t cap = (int64_t)(1ll << 32) / (N * 8);
      op->work_vecs = (int)std::max<int64_t>(1, std::min<int64_t>(64, cap));
    }
    if (op->ndim == 2) {
      op->x_same_K = Kh[0] == Kh[1];
      op->x_same_S = op->have_prec && pf.S[0] == pf.S[1] && pf.Si[0] == pf.Si[1];
      op->y_same_K = Kh[2] == Kh[3];
      op->y_same_S = op->have_prec && pf.S[2] == pf.S[3] && pf.Si[2] == pf.Si[3];
    }
    tp3b_status st = upload_ops<double>(op, op->d64, Kh, pf);
    if (st == TP3B_OK) st = upload_ops<float>(op, op->d32, Kh, pf);
    if (st == TP3B_OK) st = bf3_split_ops(op);
    if (st != TP3B_OK) {
      std::string msg = g_err;
      tp3b_destroy(op);
      return fail(st, msg);
    }
    *out = op;
    return TP3B_OK;
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_destroy(tp3b_op op) {
  try {
    if (!op) return TP3B_OK;
    free_ops(op->d64);
    free_ops(op->d32);
    for (const auto* v : {&op->bf3L, &op->bf3R})
      for (const auto& e : *v) (void)hipFree(e.hl);
    delete op;
    return TP3B_OK;
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_op_info(tp3b_op op, int64_t* N, double* sigma, double* lam_min) {
  try {
    if (!op) return fail(TP3B_EINVAL, "null operator");
    if (N) *N = op->N;
    if (sigma) *sigma = op->sigma;
    if (lam_min) *lam_min = op->lam_min;
    return TP3B_OK;
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_get_D2(tp3b_op op, int32_t mode, double* out) {
  try {
    if (!op || !out) return fail(TP3B_EINVAL, "null argument");
    if (mode < 0 || mode >= op->nmodes) return fail(TP3B_EINVAL, "mode out of range");
    std::memcpy(out, op->D2h[mode].data(), sizeof(double) * op->D2h[mode].size());
    return TP3B_OK;
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_get_V(tp3b_op op, double* out) {
  try {
    if (!op || !out) return fail(TP3B_EINVAL, "null argument");
    std::memcpy(out, op->Vh.data(), sizeof(double) * op->N);
    return TP3B_OK;
  } catch (...) {
    return exception_status();
  }
}

static tp3b_status check_apply(tp3b_op op, int32_t prec, int32_t nvec, const void* X, int64_t ldx,
                               void* Y, int64_t ldy) {
  if (!op) return fail(TP3B_EINVAL, "null operator");
  if (prec != TP3B_FP64 && prec != TP3B_FP32 && prec != TP3B_BF16X3)
    return fail(TP3B_EINVAL, "unknown precision");
  if (nvec < 0) return fail(TP3B_EINVAL, "nvec must be >= 0");
  if (nvec == 0) return TP3B_OK;
  if (!X || !Y) return fail(TP3B_EINVAL, "null X or Y");
  if (ldx < op->N || ldy < op->N) return fail(TP3B_EINVAL, "leading dimension smaller than N");
  const size_t es = prec == TP3B_FP64 ? 8 : 4;
  const char* xb = (const char*)X;
  const char* yb = (const char*)Y;
  const char* xe = xb + es * ((size_t)(nvec - 1) * ldx + op->N);
  const char* ye = yb + es * ((size_t)(nvec - 1) * ldy + op->N);
  if (xb < ye && yb < xe) return fail(TP3B_EINVAL, "X and Y overlap");
  return TP3B_OK;
}

tp3b_status tp3b_apply_H_shifted(tp3b_op op, int32_t prec, int32_t nvec, const void* X,
                                 int64_t ldx, void* Y, int64_t ldy, const double* shifts,
                                 void* stream) {
  try {
    tp3b_status st = check_apply(op, prec, nvec, X, ldx, Y, ldy);
    if (st != TP3B_OK || nvec == 0) return st;
    TP3B_HIP(hipSetDevice(op->device));
    hipStream_t s = (hipStream_t)stream;
    if (prec == TP3B_FP64)
      return apply_H_impl<double>(op, nvec, (const double*)X, ldx, (double*)Y, ldy, shifts, s);
    return apply_H_impl<float>(op, nvec, (const float*)X, ldx, (float*)Y, ldy, shifts, s,
                               prec == TP3B_BF16X3);
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_apply_H(tp3b_op op, int32_t prec, int32_t nvec, const void* X, int64_t ldx,
                         void* Y, int64_t ldy, void* stream) {
  try {
    return tp3b_apply_H_shifted(op, prec, nvec, X, ldx, Y, ldy, nullptr, stream);
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_apply_prec(tp3b_op op, int32_t prec, int32_t nvec, const void* X, int64_t ldx,
                            void* Y, int64_t ldy, void* stream) {
  try {
    tp3b_status st = check_apply(op, prec, nvec, X, ldx, Y, ldy);
    if (st != TP3B_OK || nvec == 0) return st;
    if (!op->have_prec) return fail(TP3B_ENOTSUP, "kinetic factors have complex spectrum or K - sigma is singular");
    TP3B_HIP(hipSetDevice(op->device));
    hipStream_t s = (hipStream_t)stream;
    if (prec == TP3B_FP64)
      return apply_prec_impl<double>(op, nvec, (const double*)X, ldx, (double*)Y, ldy, s);
    return apply_prec_impl<float>(op, nvec, (const float*)X, ldx, (float*)Y, ldy, s,
                                  prec == TP3B_BF16X3);
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_block_orth(int64_t N, int32_t nq, const double* Q, int64_t ldq, int32_t nx,
                            double* X, int64_t ldx, double* C_qx, double* R_xx, int32_t* rank,
                            uint64_t seed, void* stream) {
  try {
    if (N < 0 || nq < 0 || nx < 0) return fail(TP3B_EINVAL, "negative size");
    if (nx > 32) return fail(TP3B_EINVAL, "nx must be <= 32");
    if (nx == 0) {
      if (rank) *rank = 0;
      return TP3B_OK;
    }
    if (!X || (nq > 0 && !Q)) return fail(TP3B_EINVAL, "null X or Q");
    if (ldx < N || (nq > 0 && ldq < N)) return fail(TP3B_EINVAL, "leading dimension smaller than N");
    if (N < nq + nx) return fail(TP3B_EINVAL, "N must be >= nq + nx");
    return block_orth_impl(N, nq, Q, ldq, nx, X, ldx, C_qx, R_xx, rank, seed, (hipStream_t)stream);
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_block_orth_noalloc(int64_t N, int32_t nq, const double* Q, int64_t ldq, int32_t nx,
                                    double* X, int64_t ldx, int32_t* rank, uint64_t seed,
                                    void* stream) {
  try {
    if (N < 0 || nq < 0 || nx < 0) return fail(TP3B_EINVAL, "negative size");
    if (nx > 32) return fail(TP3B_EINVAL, "nx must be <= 32");
    if (nx == 0) {
      if (rank) *rank = 0;
      return TP3B_OK;
    }
    if (!X || (nq > 0 && !Q)) return fail(TP3B_EINVAL, "null X or Q");
    if (ldx < N || (nq > 0 && ldq < N)) return fail(TP3B_EINVAL, "leading dimension smaller than N");
    if (N < nq + nx) return fail(TP3B_EINVAL, "N must be >= nq + nx");
    // the flags sit in the last 64 doubles of the static scratch, the rest
    // holds the orthogonalisation's partial sums and small factors
    const int64_t room = kStaticScratchDoubles - 64;
    if (orth_scratch_doubles(N, nq, nx) > room)
      return fail(TP3B_ENOMEM, "block_orth_noalloc: N, nq and nx need more than the static scratch "
                               "(about nq <= 64 for nx <= 32 at any N)");
    hipStream_t s = (hipStream_t)stream;
    double* scr = nullptr;
    TP3B_HIP(static_scratch(&scr));
    int* dflags = (int*)(scr + room);
    int hflags[33];
    int replaced[32] = {0};
    int deficient = 0;
    for (int attempt = 0;; ++attempt) {
      tp3b_status qs = block_orth_queue(N, nq, Q, ldq, nx, X, ldx, dflags, s, nullptr, scr);
      if (qs != TP3B_OK) return qs;
      TP3B_HIP(hipMemcpyAsync(hflags, dflags, sizeof(int) * (nx + 1), hipMemcpyDeviceToHost, s));
      TP3B_HIP(hipStreamSynchronize(s));
      if (hflags[nx]) return fail(TP3B_ENONFINITE, "block_orth_noalloc: non-finite input");
      int bad = 0;
      for (int j = 0; j < nx; ++j) bad += hflags[j] != 0;
      if (!bad) break;
      if (attempt == 3) return fail(TP3B_EDEVICE, "block_orth_noalloc: could not complete the basis");
      // dependent columns: pseudo-random replacements, then the queued
      // sequence again (the independent columns are already orthonormal)
      for (int j = 0; j < nx; ++j) {
        if (!hflags[j]) continue;
        if (!replaced[j]) ++deficient;
        replaced[j] = 1;
        TP3B_HIP(launch_hash_fill(N, X + (int64_t)j * ldx, seed, (uint64_t)(attempt * 64 + j), s));
      }
    }
    if (rank) *rank = nx - deficient;
    return TP3B_OK;
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_set_tile(tp3b_op op, int32_t tile) {
  try {
    if (!op) return fail(TP3B_EINVAL, "null operator");
    if (tile < -1 || tile >= NUM_TILE_CFGS) return fail(TP3B_EINVAL, "unknown tile shape");
    op->tile_override = tile;
    return TP3B_OK;
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_autotune(tp3b_op op, int32_t prec, int32_t nvec, int32_t reps, double* best_ms) {
  try {
    if (!op) return fail(TP3B_EINVAL, "null operator");
    if (nvec < 1 || reps < 1) return fail(TP3B_EINVAL, "nvec and reps must be >= 1");
    if (prec != TP3B_FP64 && prec != TP3B_FP32 && prec != TP3B_BF16X3)
      return fail(TP3B_EINVAL, "unknown precision");
    TP3B_HIP(hipSetDevice(op->device));
    if (best_ms) best_ms[0] = best_ms[1] = NAN;
    return prec == TP3B_FP64 ? autotune_impl<double>(op, nvec, reps, best_ms, false)
                             : autotune_impl<float>(op, nvec, reps, best_ms, prec == TP3B_BF16X3);
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_host_schur(int32_t n, double* A, double* Z, double* wr, double* wi) {
  try {
    if (n < 1 || !A || !wr || !wi) return fail(TP3B_EINVAL, "bad arguments");
    if (!real_schur(n, A, Z, wr, wi)) return fail(TP3B_ENOCONV, "QR iteration did not converge");
    return TP3B_OK;
  } catch (...) {
    return exception_status();
  }
}

}  // extern "C"
