// Batched forms of the Hamiltonian apply, the preconditioner and block JDQR:
// many independent 1D instances advanced together, every device step one
// grouped, persistent launch over all instances (grouped.h).
//
// The batched eigensolver runs the same iteration as jdqr.cpp for every
// instance (Sec. 4.1, eqs. (12)-(13)); only the scheduling differs.  Per outer
// iteration and unconverged instance: ordered Schur form of the projected
// matrix (host), rotation, partial-Schur residuals, locking of the converged
// prefix or, for the instances that lock nothing, restart, the b correction
// equations (skew-projected, preconditioned GMRES with a fixed number of steps
// in the inner precision) and the FP64 expansion of the basis.  Small per-
// instance arrays are laid out kind by kind across the batch (structure of
// arrays), so that each host<->device exchange of a phase is one copy.
// The GMRES inner iteration reads every parameter from job tables at fixed
// device addresses; with opts.graph it is captured once as a HIP graph and
// replayed in every outer iteration after the tables have been rewritten.
#include <algorithm>
#include <utility>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <vector>

#include "dense_la.h"
#include "grouped.h"
#include "internal.h"

namespace tp3b {
namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <class Job>
using Tab = TableArena::Tab<Job>;

#define TP3B_TRY(...)                               \
  do {                                              \
    tp3b_status _st = (__VA_ARGS__);                \
    if (_st != TP3B_OK) return _st;                 \
  } while (0)

tp3b_status arena_full() { return fail(TP3B_ENOMEM, "batched: job-table arena exhausted"); }

// Tile shapes in use by one kind of mode-product step over a batch.
struct TileSet {
  int n = 0;
  int id[NUM_TILE_CFGS] = {};
  void add(int t) {
    for (int i = 0; i < n; ++i)
      if (id[i] == t) return;
    id[n++] = t;
  }
};

// The tables of one grouped mode-product step, one per tile shape in use.
template <typename T>
struct MpTabs {
  int n = 0;
  int tile[NUM_TILE_CFGS] = {};
  Tab<ModeProd<T>> t[NUM_TILE_CFGS];
  bool bf3 = false;
};

template <typename T>
bool mp_alloc(TableArena& ar, const TileSet& ts, int cap, bool bf3, MpTabs<T>& m) {
  m.n = ts.n;
  m.bf3 = bf3;
  for (int i = 0; i < ts.n; ++i) {
    m.tile[i] = ts.id[i];
    if (!ar.alloc(m.t[i], cap)) return false;
  }
  return true;
}

// Adds a job to the table of its tile shape; false if no table has that shape.
template <typename T>
bool mp_add(MpTabs<T>& m, const ModeProd<T>& a, int tile) {
  for (int i = 0; i < m.n; ++i)
    if (m.tile[i] == tile) {
      TableArena::add(m.t[i], a, modeprod_items_for(a.M, a.Nc, a.nbatch, tile, m.bf3));
      return true;
    }
  return false;
}

tp3b_status tile_missing() { return fail(TP3B_EDEVICE, "batched: tile shape without a job table"); }

hipError_t mp_launch(const MpTabs<double>& m, hipStream_t s) {
  for (int i = 0; i < m.n; ++i) {
    hipError_t e = launch_modeprod_grouped<double>(m.t[i].d, m.tile[i], s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t mp_launch(const MpTabs<float>& m, hipStream_t s) {
  for (int i = 0; i < m.n; ++i) {
    hipError_t e = m.bf3 ? launch_modeprod_bf3_grouped(m.t[i].d, m.tile[i], s)
                         : launch_modeprod_grouped<float>(m.t[i].d, m.tile[i], s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Mode-product descriptors of the 1D Hamiltonian apply and of the four
// preconditioner stages (the same products tp3b.cpp launches one by one).
template <typename T>
ModeProd<T> h_job(tp3b_op op, int nvec, const T* X, int64_t ldx, T* Y, int64_t ldy,
                  const double* shifts) {
  DevOps<T>& d = dev_ops<T>(op);
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
  return a;
}

// Stage st of Z = Sx [(Sx^{-1} B Sy^{-T}) / (lx_i + ly_j - sigma)] Sy^T; the
// intermediate lives in the operator's work buffer (nv <= work_vecs).
template <typename T>
ModeProd<T> prec_job(tp3b_op op, int st, int nv, const T* X, int64_t ldx, T* Y, int64_t ldy) {
  DevOps<T>& d = dev_ops<T>(op);
  ModeProd<T> a{};
  a.M = op->n[0];
  a.Nc = op->n[1];
  a.rs = op->n[1];
  a.per_vec = 1;
  a.nbatch = nv;
  a.sigma = op->sigma;
  a.epi = EPI_NONE;
  const int64_t N = op->N;
  switch (st) {
    case 0: a.X = X; a.ldx = ldx; a.Y = d.work; a.ldy = N; a.L = d.Si[0]; break;
    case 1:
      a.X = d.work; a.ldx = N; a.Y = Y; a.ldy = ldy; a.R = d.SiT[1];
      a.epi = EPI_DIV; a.lamL = d.lam[0]; a.lamR = d.lam[1];
      break;
    case 2: a.X = Y; a.ldx = ldy; a.Y = d.work; a.ldy = N; a.L = d.S[0]; break;
    default: a.X = d.work; a.ldx = N; a.Y = Y; a.ldy = ldy; a.R = d.ST[1]; break;
  }
  return a;
}

tp3b_status check_batch(const tp3b_op* ops, int count, bool need_prec) {
  if (!ops || count < 1) return fail(TP3B_EINVAL, "batched: need count >= 1 operators");
  int dev = 0;
  TP3B_HIP(hipGetDevice(&dev));
  for (int i = 0; i < count; ++i) {
    if (!ops[i]) return fail(TP3B_EINVAL, "batched: null operator");
    if (ops[i]->ndim != 1) return fail(TP3B_ENOTSUP, "batched forms take 1D operators only");
    if (ops[i]->device != dev) return fail(TP3B_EINVAL, "batched: operators on different devices");
    if (need_prec && !ops[i]->have_prec)
      return fail(TP3B_ENOTSUP, "batched: an operator has no kinetic preconditioner");
  }
  return TP3B_OK;
}

// Per-thread staging arena for the batched apply entry points.
TableArena* apply_arena() {
  static thread_local std::unique_ptr<TableArena> ar;
  if (!ar) {
    ar.reset(new TableArena());
    if (ar->init((size_t)8 << 20) != hipSuccess) {
      ar.reset();
      return nullptr;
    }
  }
  return ar.get();
}

template <typename T>
tp3b_status apply_batched(const tp3b_op* ops, int count, int nvec, const void* const* X,
                          const int64_t* ldx, void* const* Y, const int64_t* ldy,
                          const double* const* shifts, bool prec, bool bf3, hipStream_t s) {
  TableArena* ar = apply_arena();
  if (!ar) return fail(TP3B_ENOMEM, "batched: table arena allocation failed");
  // The previous call's tables may still be in flight on some stream.
  TP3B_HIP(hipDeviceSynchronize());
  ar->reset();
  const bool f64 = sizeof(T) == 8;
  TileSet ts;
  for (int i = 0; i < count; ++i) ts.add(op_tile(ops[i], f64, bf3, prec ? 1 : 0, nvec));
  const int nst = prec ? 4 : 1;
  MpTabs<T> tabs[4];
  for (int st = 0; st < nst; ++st)
    if (!mp_alloc(*ar, ts, count, bf3, tabs[st])) return arena_full();
  for (int i = 0; i < count; ++i) {
    const T* x = (const T*)X[i];
    T* y = (T*)Y[i];
    const int tile = op_tile(ops[i], f64, bf3, prec ? 1 : 0, nvec);
    if (prec) {
      for (int st = 0; st < 4; ++st)
        if (!mp_add(tabs[st], prec_job<T>(ops[i], st, nvec, x, ldx[i], y, ldy[i]), tile))
          return tile_missing();
    } else {
      if (!mp_add(tabs[0], h_job<T>(ops[i], nvec, x, ldx[i], y, ldy[i], shifts ? shifts[i] : nullptr), tile))
        return tile_missing();
    }
  }
  TP3B_HIP(ar->upload(s));
  for (int st = 0; st < nst; ++st) TP3B_HIP(mp_launch(tabs[st], s));
  return TP3B_OK;
}

tp3b_status check_batched_apply(const tp3b_op* ops, int count, int prec, int nvec,
                                const void* const* X, const int64_t* ldx, void* const* Y,
                                const int64_t* ldy, bool need_prec) {
  TP3B_TRY(check_batch(ops, count, need_prec));
  if (prec != TP3B_FP64 && prec != TP3B_FP32 && prec != TP3B_BF16X3)
    return fail(TP3B_EINVAL, "unknown precision");
  if (nvec < 0) return fail(TP3B_EINVAL, "nvec must be >= 0");
  if (nvec == 0) return TP3B_OK;
  if (!X || !Y || !ldx || !ldy) return fail(TP3B_EINVAL, "batched: null X, Y or leading dimensions");
  const size_t es = prec == TP3B_FP64 ? 8 : 4;
  for (int i = 0; i < count; ++i) {
    if (!X[i] || !Y[i]) return fail(TP3B_EINVAL, "batched: null block");
    if (ldx[i] < ops[i]->N || ldy[i] < ops[i]->N)
      return fail(TP3B_EINVAL, "batched: leading dimension smaller than N");
    if (need_prec && nvec > ops[i]->work_vecs)
      return fail(TP3B_EINVAL, "batched: too many vectors for the preconditioner's work buffer");
    const char* xb = (const char*)X[i];
    const char* yb = (const char*)Y[i];
    const char* xe = xb + es * ((size_t)(nvec - 1) * ldx[i] + ops[i]->N);
    const char* ye = yb + es * ((size_t)(nvec - 1) * ldy[i] + ops[i]->N);
    if (xb < ye && yb < xe) return fail(TP3B_EINVAL, "batched: X and Y overlap");
  }
  return TP3B_OK;
}

// ===================================================================== JDQR
// Small per-instance arrays, one kind at a time across the batch.
struct Small {
  double* d = nullptr;   // device base (inside one allocation)
  std::vector<double> h; // host mirror
  int64_t stride = 0;    // doubles per instance
  double* at(int i) const { return d + (int64_t)i * stride; }
  double* hat(int i) { return h.data() + (int64_t)i * stride; }
};

struct Inst {
  tp3b_op op = nullptr;
  int64_t N = 0;
  // device blocks (views into one allocation)
  double *QV = nullptr, *AVb = nullptr, *TMP = nullptr, *Rres = nullptr, *PQ = nullptr,
         *Yp = nullptr, *Tc = nullptr, *part = nullptr, *bpart = nullptr;
  void *Qtw = nullptr, *Ypw = nullptr, *Vg = nullptr, *W = nullptr, *Zt = nullptr;
  int* flags = nullptr;
  // tile shapes of the grouped applies (fixed for the solve)
  int tH64 = 0, tHW = 0, tP64 = 0, tPW = 0;
  // host state (as in jdqr.cpp)
  int k = 0, m = 0, av0 = 0, outer = 0;
  double prev_rn0 = INFINITY;
  int stall = 0;
  bool done = false;
  int status = TP3B_OK;
  std::vector<double> M, Rl, lockres, S, T;
  std::vector<int> lock_pair, pair;
  // per outer iteration
  int nb = 0, lockp = 0;
  bool correct = false, restart = false;
  std::vector<double> theta, rn, Cq;
  double* V() const { return QV + (int64_t)k * N; }
  double* AV() const { return AVb + (int64_t)av0 * N; }
};

template <typename TW>
class BatchedJdqr {
 public:
  BatchedJdqr(const tp3b_op* ops, int count, const tp3b_jdqr_opts& o, bool bf3)
      : ops_(ops), count_(count), o_(o), bf3_(bf3) {}
  ~BatchedJdqr();
  tp3b_status run(double* evals, double* resnorm, int32_t* n_conv, int32_t* n_outer,
                  double* const* Q, tp3b_jdqr_stats* st);

 private:
  // ---- set-up
  tp3b_status setup();
  // ---- grouped building blocks over a list of instances
  tp3b_status orth(const std::vector<int>& list, const std::vector<int>& nq_of,
                   const std::vector<double*>& Qs, const std::vector<double*>& Xs,
                   const std::vector<int>& nx_of, uint64_t seed);
  tp3b_status apply_H64(const std::vector<int>& list, const std::vector<double*>& X,
                        const std::vector<double*>& Y, const std::vector<int>& nv);
  tp3b_status prec64(const std::vector<int>& list, const std::vector<const double*>& X,
                     const std::vector<double*>& Y, const std::vector<int>& nv);
  tp3b_status dot_to_host(const std::vector<int>& list, const std::vector<int>& p,
                          const std::vector<int>& q, const std::vector<const double*>& A,
                          const std::vector<const double*>& B, Small& out);
  tp3b_status gemm64(const std::vector<int>& list, const std::vector<int>& p,
                     const std::vector<int>& q, double alpha, const std::vector<const double*>& A,
                     const std::vector<const double*>& C, const std::vector<int>& ldc,
                     double beta, const std::vector<double*>& Y);
  tp3b_status copy64(const std::vector<int>& list, const std::vector<int>& ncol, double alpha,
                     const std::vector<const double*>& X, const std::vector<double*>& Y);
  // Waits for the stream; every table staged so far has then been consumed, so
  // the phase arena starts over.
  tp3b_status sync() {
    TP3B_HIP(hipStreamSynchronize(s_));
    ar_.reset();
    return TP3B_OK;
  }
  // Tables are appended to the phase arena without waiting; only when it runs
  // low does the stream have to drain first.
  tp3b_status arena_room() {
    if (ar_.free_bytes() < ((size_t)4 << 20)) return sync();
    return TP3B_OK;
  }
  // ---- the GMRES phase
  tp3b_status build_gmres_tables();
  tp3b_status launch_gmres();
  // ---- one outer iteration
  tp3b_status iterate();

  const tp3b_op* ops_;
  int count_;
  tp3b_jdqr_opts o_;
  bool bf3_;
  bool low_ = sizeof(TW) == 4;
  bool use_prec_ = false;
  int nev_ = 0, b_ = 0, steps_ = 0, m_max_ = 0, m_min_ = 0, hld_ = 0, qt_max_ = 0, pmax_ = 0;
  hipStream_t s_ = nullptr;
  std::vector<Inst> in_;
  void* big_ = nullptr;
  void* smallbuf_ = nullptr;
  TableArena ar_;     // tables rebuilt freely within a phase
  TableArena gar_;    // GMRES tables (same layout every outer iteration)
  TileSet tsH64_, tsHW_, tsP64_, tsPW_;
  Small S_, Tb_, Mf_, Top_, Left_, Cq1_, Cq2_, Nrm_, Hh_, Hinv_, Shift_, C2_, H1_, H2_, Hs_,
      Beta_, Y_, G_, R1_, R2_, n0_, Co1_, Co2_, FlagsD_;
  hipGraphExec_t gexec_ = nullptr;
  hipGraph_t graph_ = nullptr;
  tp3b_jdqr_stats stats_{};
  // GMRES tables
  struct GmTabs {
    Tab<ConvJob<double, TW>> rhs_conv;
    MpTabs<TW> prec[4];
    Tab<DotJob<TW, TW>> proj_dot;
    Tab<GemmJob<TW>> proj_gemm;
    Tab<BdotJob<TW>> nrm;
    Tab<NormJob<TW>> norm0;
    std::vector<MpTabs<TW>> H;
    std::vector<Tab<BdotJob<TW>>> bd1, bd2;
    std::vector<Tab<BupdJob<TW>>> bu1, bu2;
    std::vector<Tab<NormJob<TW>>> normk;
  } gm_;
  std::vector<int> corr_;  // instances correcting in this outer iteration
};

template <typename TW>
BatchedJdqr<TW>::~BatchedJdqr() {
  if (gexec_) (void)hipGraphExecDestroy(gexec_);
  if (graph_) (void)hipGraphDestroy(graph_);
  if (s_) (void)hipStreamSynchronize(s_);
  if (big_) (void)hipFree(big_);
  if (smallbuf_) (void)hipFree(smallbuf_);
  if (s_) (void)hipStreamDestroy(s_);
}

template <typename TW>
tp3b_status BatchedJdqr<TW>::setup() {
  nev_ = o_.nev;
  b_ = o_.block;
  steps_ = o_.gmres_steps;
  m_max_ = o_.m_max;
  m_min_ = o_.m_min;
  hld_ = steps_ + 2;
  qt_max_ = nev_ + b_;
  pmax_ = nev_ + m_max_ + b_;
  use_prec_ = o_.precond != 0;
  TP3B_HIP(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
  in_.resize(count_);
  // ---- per-instance device blocks, one allocation
  const size_t tw = sizeof(TW);
  std::vector<size_t> off(count_ + 1, 0);
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  auto inst_bytes = [&](int64_t N) {
    size_t b = 0;
    b += al(8 * N * (nev_ + m_max_ + b_));          // QV
    b += al(8 * N * (m_max_ + b_ + nev_));          // AV
    b += al(8 * N * (m_max_ + b_ + nev_));          // TMP (swaps roles with AV)
    b += al(8 * N * b_);                            // Rres
    if (use_prec_) b += 2 * al(8 * N * qt_max_);    // PQ, Yp
    b += al(8 * N * b_);                            // Tc
    if (low_) b += 2 * al(tw * N * qt_max_);        // Qtw, Ypw
    b += al(tw * N * b_ * (steps_ + 1));            // Vg
    b += 2 * al(tw * N * b_);                       // W, Zt
    b += al(8 * dot_job_partials(N, pmax_, pmax_)); // dot partials
    b += al(8 * bdot_job_partials(N, b_));          // bdot partials
    return b;
  };
  for (int i = 0; i < count_; ++i) off[i + 1] = off[i] + inst_bytes(ops_[i]->N);
  TP3B_HIP(hipMalloc(&big_, off[count_] ? off[count_] : 256));
  for (int i = 0; i < count_; ++i) {
    Inst& I = in_[i];
    I.op = ops_[i];
    I.N = ops_[i]->N;
    const int64_t N = I.N;
    char* p = (char*)big_ + off[i];
    auto take = [&](size_t bytes) {
      char* r = p;
      p += al(bytes);
      return r;
    };
    I.QV = (double*)take(8 * N * (nev_ + m_max_ + b_));
    I.AVb = (double*)take(8 * N * (m_max_ + b_ + nev_));
    I.TMP = (double*)take(8 * N * (m_max_ + b_ + nev_));
    I.Rres = (double*)take(8 * N * b_);
    if (use_prec_) {
      I.PQ = (double*)take(8 * N * qt_max_);
      I.Yp = (double*)take(8 * N * qt_max_);
    }
    I.Tc = (double*)take(8 * N * b_);
    if (low_) {
      I.Qtw = take(tw * N * qt_max_);
      I.Ypw = take(tw * N * qt_max_);
    }
    I.Vg = take(tw * N * b_ * (steps_ + 1));
    I.W = take(tw * N * b_);
    I.Zt = take(tw * N * b_);
    I.part = (double*)take(8 * dot_job_partials(N, pmax_, pmax_));
    I.bpart = (double*)take(8 * bdot_job_partials(N, b_));
    I.Rl.assign((size_t)nev_ * nev_, 0.0);
  }
  // ---- small arrays
  const int mb = m_max_ + b_;
  Small* kinds[] = {&S_, &Tb_, &Mf_, &Top_, &Left_, &Cq1_, &Cq2_, &Nrm_, &Hh_, &Hinv_, &Shift_,
                    &C2_, &H1_, &H2_, &Hs_, &Beta_, &Y_, &G_, &R1_, &R2_, &n0_, &Co1_, &Co2_,
                    &FlagsD_};
  const int64_t strides[] = {(int64_t)mb * mb, (int64_t)mb * b_, (int64_t)mb * mb, (int64_t)mb * b_,
                             (int64_t)b_ * mb, (int64_t)nev_ * b_, (int64_t)nev_ * b_, b_,
                             (int64_t)qt_max_ * qt_max_, (int64_t)qt_max_ * qt_max_, b_,
                             (int64_t)qt_max_ * b_, (int64_t)steps_ * b_ * hld_,
                             (int64_t)steps_ * b_ * hld_, (int64_t)steps_ * b_, b_,
                             (int64_t)b_ * hld_, (int64_t)b_ * b_, (int64_t)b_ * b_, (int64_t)b_ * b_,
                             b_, (int64_t)pmax_ * b_, (int64_t)pmax_ * b_, b_};
  int64_t total = 0;
  for (int k = 0; k < 24; ++k) total += strides[k] * count_;
  TP3B_HIP(hipMalloc(&smallbuf_, 8 * (total ? total : 1)));
  TP3B_HIP(hipMemsetAsync(smallbuf_, 0, 8 * (total ? total : 1), s_));
  int64_t o = 0;
  for (int k = 0; k < 24; ++k) {
    kinds[k]->d = (double*)smallbuf_ + o;
    kinds[k]->stride = strides[k];
    kinds[k]->h.assign((size_t)strides[k] * count_, 0.0);
    o += strides[k] * count_;
  }
  for (int i = 0; i < count_; ++i) in_[i].flags = (int*)FlagsD_.at(i);
  // ---- job-table arenas
  TP3B_HIP(ar_.init((size_t)32 << 20));
  TP3B_HIP(gar_.init((size_t)64 << 20));
  // ---- tile shapes
  for (int i = 0; i < count_; ++i) {
    Inst& I = in_[i];
    I.tH64 = op_tile(ops_[i], true, false, 0, b_);
    I.tHW = op_tile(ops_[i], !low_, bf3_, 0, b_);
    I.tP64 = op_tile(ops_[i], true, false, 1, b_);
    I.tPW = op_tile(ops_[i], !low_, bf3_, 1, b_);
    tsH64_.add(I.tH64);
    tsHW_.add(I.tHW);
    tsP64_.add(I.tP64);
    tsPW_.add(I.tPW);
  }
  return TP3B_OK;
}

// ---- grouped FP64 helpers over a list of instances (eager launches)
template <typename TW>
tp3b_status BatchedJdqr<TW>::apply_H64(const std::vector<int>& list, const std::vector<double*>& X,
                                       const std::vector<double*>& Y, const std::vector<int>& nv) {
  if (list.empty()) return TP3B_OK;
  TP3B_TRY(arena_room());
  MpTabs<double> t;
  if (!mp_alloc(ar_, tsH64_, (int)list.size(), false, t)) return arena_full();
  for (size_t e = 0; e < list.size(); ++e) {
    if (nv[e] <= 0) continue;
    const Inst& I = in_[list[e]];
    if (!mp_add(t, h_job<double>(I.op, nv[e], X[e], I.N, Y[e], I.N, nullptr), I.tH64))
      return tile_missing();
    stats_.n_apply_H_fp64 += nv[e];
  }
  TP3B_HIP(ar_.upload(s_));
  TP3B_HIP(mp_launch(t, s_));
  return TP3B_OK;
}

template <typename TW>
tp3b_status BatchedJdqr<TW>::prec64(const std::vector<int>& list,
                                    const std::vector<const double*>& X,
                                    const std::vector<double*>& Y, const std::vector<int>& nv) {
  if (list.empty()) return TP3B_OK;
  TP3B_TRY(arena_room());
  MpTabs<double> t[4];
  for (int st = 0; st < 4; ++st)
    if (!mp_alloc(ar_, tsP64_, (int)list.size(), false, t[st])) return arena_full();
  for (size_t e = 0; e < list.size(); ++e) {
    if (nv[e] <= 0) continue;
    const Inst& I = in_[list[e]];
    for (int st = 0; st < 4; ++st)
      if (!mp_add(t[st], prec_job<double>(I.op, st, nv[e], X[e], I.N, Y[e], I.N), I.tP64))
        return tile_missing();
    stats_.n_apply_prec += nv[e];
  }
  TP3B_HIP(ar_.upload(s_));
  for (int st = 0; st < 4; ++st) TP3B_HIP(mp_launch(t[st], s_));
  return TP3B_OK;
}

// out (kind array, column-major p x q at each instance's slot, ld p) = A^T B,
// then copied to the host mirror.
template <typename TW>
tp3b_status BatchedJdqr<TW>::dot_to_host(const std::vector<int>& list, const std::vector<int>& p,
                                         const std::vector<int>& q,
                                         const std::vector<const double*>& A,
                                         const std::vector<const double*>& B, Small& out) {
  if (list.empty()) return TP3B_OK;
  TP3B_TRY(arena_room());
  Tab<DotJob<double, double>> t;
  if (!ar_.alloc(t, (int)list.size())) return arena_full();
  for (size_t e = 0; e < list.size(); ++e) {
    const Inst& I = in_[list[e]];
    DotJob<double, double> j{};
    j.N = I.N;
    j.p = p[e];
    j.q = q[e];
    j.A = A[e];
    j.lda = I.N;
    j.B = B[e];
    j.ldb = I.N;
    j.C = out.at(list[e]);
    j.ldc = p[e];
    j.part = I.part;
    int64_t i1, i2;
    dot_job_shape(j, &i1, &i2);
    TableArena::add(t, j, i1, i2);
  }
  TP3B_HIP(ar_.upload(s_));
  TP3B_HIP(launch_dot_grouped(t.d, s_));
  TP3B_HIP(hipMemcpyAsync(out.h.data(), out.d, sizeof(double) * out.h.size(), hipMemcpyDeviceToHost, s_));
  return sync();
}

template <typename TW>
tp3b_status BatchedJdqr<TW>::gemm64(const std::vector<int>& list, const std::vector<int>& p,
                                    const std::vector<int>& q, double alpha,
                                    const std::vector<const double*>& A,
                                    const std::vector<const double*>& C,
                                    const std::vector<int>& ldc, double beta,
                                    const std::vector<double*>& Y) {
  if (list.empty()) return TP3B_OK;
  TP3B_TRY(arena_room());
  Tab<GemmJob<double>> t;
  if (!ar_.alloc(t, (int)list.size())) return arena_full();
  for (size_t e = 0; e < list.size(); ++e) {
    const Inst& I = in_[list[e]];
    GemmJob<double> j{};
    j.N = I.N;
    j.p = p[e];
    j.q = q[e];
    j.alpha = alpha;
    j.beta = beta;
    j.A = A[e];
    j.lda = I.N;
    j.C = C[e];
    j.ldc = ldc[e];
    j.Y = Y[e];
    j.ldy = I.N;
    TableArena::add(t, j, gemm_job_items(I.N, q[e]));
  }
  TP3B_HIP(ar_.upload(s_));
  TP3B_HIP(launch_gemm_grouped(t.d, s_));
  return TP3B_OK;
}

template <typename TW>
tp3b_status BatchedJdqr<TW>::copy64(const std::vector<int>& list, const std::vector<int>& ncol,
                                    double alpha, const std::vector<const double*>& X,
                                    const std::vector<double*>& Y) {
  if (list.empty()) return TP3B_OK;
  TP3B_TRY(arena_room());
  Tab<ConvJob<double, double>> t;
  if (!ar_.alloc(t, (int)list.size())) return arena_full();
  for (size_t e = 0; e < list.size(); ++e) {
    const Inst& I = in_[list[e]];
    ConvJob<double, double> j{I.N, ncol[e], alpha, X[e], I.N, Y[e], I.N};
    TableArena::add(t, j, rows_items(I.N, ncol[e]));
  }
  TP3B_HIP(ar_.upload(s_));
  TP3B_HIP(launch_convert_grouped(t.d, s_));
  return TP3B_OK;
}

// Block orthogonalisation of X_e (N x nx) against Q_e (N x nq_e) for every
// listed instance (block_orth_impl of tp3b.cpp, grouped): CGS twice, Cholesky-QR
// twice, dependent columns replaced by counter-based random vectors.
template <typename TW>
tp3b_status BatchedJdqr<TW>::orth(const std::vector<int>& list0, const std::vector<int>& nq0,
                                  const std::vector<double*>& Q0, const std::vector<double*>& X0,
                                  const std::vector<int>& nx0, uint64_t seed) {
  constexpr double kDropTol = 1e-7;
  std::vector<int> list = list0, nq = nq0;
  std::vector<double*> Qs = Q0, Xs = X0;
  std::vector<int> nxv(count_, 0);
  for (size_t e = 0; e < list.size(); ++e) nxv[list[e]] = nx0[e];
  // input column norms (Gram diagonal)
  {
    std::vector<int> p;
    for (int i : list) p.push_back(nxv[i]);
    std::vector<const double*> A(Xs.begin(), Xs.end());
    TP3B_TRY(dot_to_host(list, p, p, A, A, G_));
  }
  std::vector<std::vector<double>> n0(count_);
  for (int i : list) {
    const int nx = nxv[i];
    n0[i].resize(nx);
    for (int j = 0; j < nx; ++j) {
      n0[i][j] = G_.hat(i)[j + j * nx];
      if (!std::isfinite(n0[i][j])) return fail(TP3B_ENONFINITE, "batched orth: non-finite input");
    }
  }
  std::vector<std::vector<int>> replaced(count_);
  for (int attempt = 0; attempt < 4 && !list.empty(); ++attempt) {
    for (int i : list) std::memcpy(n0_.hat(i), n0[i].data(), sizeof(double) * nxv[i]);
    TP3B_HIP(hipMemcpyAsync(n0_.d, n0_.h.data(), sizeof(double) * n0_.h.size(), hipMemcpyHostToDevice, s_));
    // CGS twice against Q (instances with nq > 0)
    std::vector<int> lq;
    std::vector<int> pq, qq, ldq;
    std::vector<const double*> Aq, Bq, C1, C2;
    std::vector<double*> Yq;
    for (size_t e = 0; e < list.size(); ++e)
      if (nq[e] > 0) {
        lq.push_back(list[e]);
        pq.push_back(nq[e]);
        qq.push_back(nxv[list[e]]);
        ldq.push_back(nq[e]);
        Aq.push_back(Qs[e]);
        Bq.push_back(Xs[e]);
        C1.push_back(Co1_.at(list[e]));
        C2.push_back(Co2_.at(list[e]));
        Yq.push_back(Xs[e]);
      }
    for (int pass = 0; pass < 2 && !lq.empty(); ++pass) {
      TP3B_TRY(arena_room());
      Tab<DotJob<double, double>> td;
      Tab<GemmJob<double>> tg;
      if (!ar_.alloc(td, (int)lq.size()) || !ar_.alloc(tg, (int)lq.size())) return arena_full();
      for (size_t e = 0; e < lq.size(); ++e) {
        const Inst& I = in_[lq[e]];
        const int nx = qq[e];
        double* C = (double*)(pass ? C2[e] : C1[e]);
        DotJob<double, double> j{};
        j.N = I.N; j.p = pq[e]; j.q = nx; j.A = Aq[e]; j.lda = I.N; j.B = Bq[e]; j.ldb = I.N;
        j.C = C; j.ldc = pq[e]; j.part = I.part;
        int64_t i1, i2;
        dot_job_shape(j, &i1, &i2);
        TableArena::add(td, j, i1, i2);
        GemmJob<double> g{};
        g.N = I.N; g.p = pq[e]; g.q = nx; g.alpha = -1.0; g.beta = 1.0; g.A = Aq[e]; g.lda = I.N;
        g.C = C; g.ldc = pq[e]; g.Y = Yq[e]; g.ldy = I.N;
        TableArena::add(tg, g, gemm_job_items(I.N, nx));
      }
      TP3B_HIP(ar_.upload(s_));
      TP3B_HIP(launch_dot_grouped(td.d, s_));
      TP3B_HIP(launch_gemm_grouped(tg.d, s_));
    }
    // Cholesky-QR, first pass (with the dependence test)
    TP3B_TRY(arena_room());
    {
      Tab<DotJob<double, double>> td;
      Tab<CholJob> tc;
      if (!ar_.alloc(td, (int)list.size()) || !ar_.alloc(tc, (int)list.size())) return arena_full();
      for (size_t e = 0; e < list.size(); ++e) {
        const int i = list[e];
        const Inst& I = in_[i];
        const int nx = nxv[i];
        DotJob<double, double> j{};
        j.N = I.N; j.p = nx; j.q = nx; j.A = Xs[e]; j.lda = I.N; j.B = Xs[e]; j.ldb = I.N;
        j.C = G_.at(i); j.ldc = nx; j.part = I.part;
        int64_t i1, i2;
        dot_job_shape(j, &i1, &i2);
        TableArena::add(td, j, i1, i2);
        CholJob c{nx, kDropTol, G_.at(i), n0_.at(i), R1_.at(i), I.flags};
        TableArena::add(tc, c, 1);
      }
      TP3B_HIP(ar_.upload(s_));
      TP3B_HIP(launch_dot_grouped(td.d, s_));
      TP3B_HIP(launch_chol_grouped(tc.d, s_));
      TP3B_HIP(hipMemcpyAsync(FlagsD_.h.data(), FlagsD_.d, sizeof(double) * FlagsD_.h.size(),
                              hipMemcpyDeviceToHost, s_));
      TP3B_TRY(sync());
    }
    std::vector<int> bad_list, good;
    std::vector<size_t> bad_e, good_e;
    for (size_t e = 0; e < list.size(); ++e) {
      const int* fl = (const int*)FlagsD_.hat(list[e]);
      bool bad = false;
      for (int j = 0; j < nxv[list[e]]; ++j) bad |= fl[j] != 0;
      if (bad && attempt < 3) {
        bad_list.push_back(list[e]);
        bad_e.push_back(e);
      } else if (bad) {
        return fail(TP3B_EDEVICE, "batched orth: could not complete the basis");
      } else {
        good.push_back(list[e]);
        good_e.push_back(e);
      }
    }
    // the independent instances finish: X R1^{-1}, Gram, Cholesky, X R2^{-1}
    if (!good.empty()) {
      TP3B_TRY(arena_room());
      Tab<TrsmJob> t1, t2;
      Tab<DotJob<double, double>> td;
      Tab<CholJob> tc;
      if (!ar_.alloc(t1, (int)good.size()) || !ar_.alloc(t2, (int)good.size()) ||
          !ar_.alloc(td, (int)good.size()) || !ar_.alloc(tc, (int)good.size()))
        return arena_full();
      for (size_t g = 0; g < good.size(); ++g) {
        const int i = good[g];
        const Inst& I = in_[i];
        const int nx = nxv[i];
        double* X = Xs[good_e[g]];
        TableArena::add(t1, TrsmJob{I.N, nx, R1_.at(i), X, I.N}, (I.N + 255) / 256);
        DotJob<double, double> j{};
        j.N = I.N; j.p = nx; j.q = nx; j.A = X; j.lda = I.N; j.B = X; j.ldb = I.N;
        j.C = G_.at(i); j.ldc = nx; j.part = I.part;
        int64_t i1, i2;
        dot_job_shape(j, &i1, &i2);
        TableArena::add(td, j, i1, i2);
        // the second factorisation has no dependence test: n0 = 0 (drop_tol 0)
        TableArena::add(tc, CholJob{nx, 0.0, G_.at(i), n0_.at(i), R2_.at(i), I.flags}, 1);
        TableArena::add(t2, TrsmJob{I.N, nx, R2_.at(i), X, I.N}, (I.N + 255) / 256);
      }
      TP3B_HIP(ar_.upload(s_));
      TP3B_HIP(launch_trsm_grouped(t1.d, s_));
      TP3B_HIP(launch_dot_grouped(td.d, s_));
      TP3B_HIP(launch_chol_grouped(tc.d, s_));
      TP3B_HIP(launch_trsm_grouped(t2.d, s_));
    }
    if (bad_list.empty()) break;
    // dependent columns: replace by random vectors and redo those instances
    std::vector<int> nl, nqn;
    std::vector<double*> nQ, nX;
    for (size_t b = 0; b < bad_list.size(); ++b) {
      const int i = bad_list[b];
      const size_t e = bad_e[b];
      const int* fl = (const int*)FlagsD_.hat(i);
      if (replaced[i].empty()) replaced[i].assign(nxv[i], 0);
      for (int j = 0; j < nxv[i]; ++j)
        if (fl[j]) {
          replaced[i][j] = 1;
          TP3B_HIP(launch_hash_fill(in_[i].N, Xs[e] + (int64_t)j * in_[i].N,
                                    seed + 7919ull * (uint64_t)i, (uint64_t)(attempt * 64 + j), s_));
        }
      nl.push_back(i);
      nqn.push_back(nq[e]);
      nQ.push_back(Qs[e]);
      nX.push_back(Xs[e]);
    }
    list = nl;
    nq = nqn;
    Qs = nQ;
    Xs = nX;
    {
      std::vector<int> p;
      for (int i : list) p.push_back(nxv[i]);
      std::vector<const double*> A(Xs.begin(), Xs.end());
      TP3B_TRY(dot_to_host(list, p, p, A, A, G_));
    }
    // the dependence test of a replaced column refers to its new norm; the
    // other columns keep their input norms
    for (int i : list)
      for (int j = 0; j < nxv[i]; ++j)
        if (replaced[i][j]) n0[i][j] = G_.hat(i)[j + j * nxv[i]];
  }
  return TP3B_OK;
}

// ---- the GMRES inner iteration over the correcting instances
template <typename TW>
tp3b_status BatchedJdqr<TW>::build_gmres_tables() {
  gar_.reset();
  const int cap = count_;
  GmTabs& g = gm_;
  g.H.assign(steps_, MpTabs<TW>());
  g.bd1.assign(steps_, Tab<BdotJob<TW>>());
  g.bd2.assign(steps_, Tab<BdotJob<TW>>());
  g.bu1.assign(steps_, Tab<BupdJob<TW>>());
  g.bu2.assign(steps_, Tab<BupdJob<TW>>());
  g.normk.assign(steps_, Tab<NormJob<TW>>());
  bool ok = gar_.alloc(g.rhs_conv, cap);
  for (int st = 0; st < 4; ++st) ok = ok && mp_alloc(gar_, tsPW_, cap, bf3_, g.prec[st]);
  ok = ok && gar_.alloc(g.proj_dot, cap) && gar_.alloc(g.proj_gemm, cap) && gar_.alloc(g.nrm, cap) &&
       gar_.alloc(g.norm0, cap);
  for (int kk = 0; kk < steps_; ++kk) {
    ok = ok && mp_alloc(gar_, tsHW_, cap, bf3_, g.H[kk]) && gar_.alloc(g.bd1[kk], cap) &&
         gar_.alloc(g.bu1[kk], cap) && gar_.alloc(g.bd2[kk], cap) && gar_.alloc(g.bu2[kk], cap) &&
         gar_.alloc(g.normk[kk], cap);
  }
  if (!ok) return arena_full();
  for (int i : corr_) {
    Inst& I = in_[i];
    const int64_t N = I.N;
    const int nb = I.nb;
    const int nqt = I.k + nb;
    TW* Vg = (TW*)I.Vg;
    TW* W = (TW*)I.W;
    TW* Zt = (TW*)I.Zt;
    const TW* Qtw = low_ ? (const TW*)I.Qtw : (const TW*)I.QV;
    const TW* Yqw = low_ ? (const TW*)I.Ypw : (const TW*)(use_prec_ ? I.Yp : I.QV);
    const int64_t bs = N * nb;
    // right-hand side: proj(P^{-1}(-r)), or proj(-r) without a preconditioner
    TableArena::add(g.rhs_conv, ConvJob<double, TW>{N, nb, -1.0, I.Rres, N, use_prec_ ? Zt : W, N},
                    rows_items(N, nb));
    if (use_prec_)
      for (int st = 0; st < 4; ++st)
        if (!mp_add(g.prec[st], prec_job<TW>(I.op, st, nb, Zt, N, W, N), I.tPW)) return tile_missing();
    {
      DotJob<TW, TW> j{};
      j.N = N; j.p = nqt; j.q = nb; j.A = Qtw; j.lda = N; j.B = W; j.ldb = N;
      j.C = C2_.at(i); j.ldc = nqt; j.part = I.part;
      int64_t i1, i2;
      dot_job_shape(j, &i1, &i2);
      TableArena::add(g.proj_dot, j, i1, i2);
      GemmJob<TW> gg{};
      gg.N = N; gg.p = nqt; gg.q = nb; gg.alpha = -1.0; gg.beta = 1.0; gg.A = Yqw; gg.lda = N;
      gg.C = C2_.at(i); gg.ldc = nqt; gg.Y = W; gg.ldy = N;
      TableArena::add(g.proj_gemm, gg, gemm_job_items(N, nb));
    }
    {
      BdotJob<TW> j{};
      j.N = N; j.b = nb; j.nb = 1; j.V = W; j.bs = 0; j.W = W; j.part = I.bpart;
      j.H = Nrm_.at(i); j.hld = 1;
      int64_t i1, i2;
      bdot_job_shape(j, &i1, &i2);
      TableArena::add(g.nrm, j, i1, i2);
      TableArena::add(g.norm0, NormJob<TW>{N, nb, Nrm_.at(i), W, Vg, Beta_.at(i), 1}, rows_items(N, nb));
    }
    for (int kk = 0; kk < steps_; ++kk) {
      TW* vk = Vg + (int64_t)kk * bs;
      if (!mp_add(g.H[kk], h_job<TW>(I.op, nb, vk, N, use_prec_ ? Zt : W, N, Shift_.at(i)), I.tHW))
        return tile_missing();
      double* h1 = H1_.at(i) + (int64_t)kk * b_ * hld_;
      double* h2 = H2_.at(i) + (int64_t)kk * b_ * hld_;
      for (int pass = 0; pass < 2; ++pass) {
        BdotJob<TW> j{};
        j.N = N; j.b = nb; j.nb = kk + 1; j.V = Vg; j.bs = bs; j.W = W; j.part = I.bpart;
        j.H = pass ? h2 : h1; j.hld = hld_;
        int64_t i1, i2;
        bdot_job_shape(j, &i1, &i2);
        TableArena::add(pass ? g.bd2[kk] : g.bd1[kk], j, i1, i2);
        BupdJob<TW> u{N, nb, kk + 1, -1.0, Vg, bs, pass ? h2 : h1, hld_, W};
        TableArena::add(pass ? g.bu2[kk] : g.bu1[kk], u, rows_items(N, nb));
      }
      TableArena::add(g.normk[kk],
                      NormJob<TW>{N, nb, Nrm_.at(i), W, Vg + (int64_t)(kk + 1) * bs,
                                  Hs_.at(i) + (int64_t)kk * b_, 1},
                      rows_items(N, nb));
    }
  }
  TP3B_HIP(gar_.upload(s_));
  return TP3B_OK;
}

template <typename TW>
tp3b_status BatchedJdqr<TW>::launch_gmres() {
  GmTabs& g = gm_;
  TP3B_HIP(launch_convert_grouped(g.rhs_conv.d, s_));
  if (use_prec_)
    for (int st = 0; st < 4; ++st) TP3B_HIP(mp_launch(g.prec[st], s_));
  TP3B_HIP(launch_dot_grouped(g.proj_dot.d, s_));
  TP3B_HIP(launch_gemm_grouped(g.proj_gemm.d, s_));
  TP3B_HIP(launch_bdot_grouped(g.nrm.d, s_));
  TP3B_HIP(launch_normalize_grouped(g.norm0.d, s_));
  for (int kk = 0; kk < steps_; ++kk) {
    TP3B_HIP(mp_launch(g.H[kk], s_));
    if (use_prec_)
      for (int st = 0; st < 4; ++st) TP3B_HIP(mp_launch(g.prec[st], s_));
    TP3B_HIP(launch_dot_grouped(g.proj_dot.d, s_));
    TP3B_HIP(launch_gemm_grouped(g.proj_gemm.d, s_));
    TP3B_HIP(launch_bdot_grouped(g.bd1[kk].d, s_));
    TP3B_HIP(launch_bupdate_grouped(g.bu1[kk].d, s_));
    TP3B_HIP(launch_bdot_grouped(g.bd2[kk].d, s_));
    TP3B_HIP(launch_bupdate_grouped(g.bu2[kk].d, s_));
    TP3B_HIP(launch_bdot_grouped(g.nrm.d, s_));
    TP3B_HIP(launch_normalize_grouped(g.normk[kk].d, s_));
  }
  return TP3B_OK;
}

// ---- one outer iteration of every unconverged instance
template <typename TW>
tp3b_status BatchedJdqr<TW>::iterate() {
  std::vector<int> act;
  for (int i = 0; i < count_; ++i)
    if (!in_[i].done) act.push_back(i);
  if (act.empty()) return TP3B_OK;
  const double t0 = now_s();
  // 1. ordered Schur forms (independent per instance: on several host
  // threads); rotate V and A V where S is not the identity
  std::vector<int> rot;
  std::vector<char> schur_ok(act.size(), 0), schur_ident(act.size(), 0);
  parallel_for((int)act.size(), [&](int a) {
    const int i = act[a];
    Inst& I = in_[i];
    const int m = I.m;
    I.S.assign((size_t)m * m, 0.0);
    I.T.assign((size_t)m * m, 0.0);
    I.pair.assign(m, 0);
    if (!ordered_schur(m, I.M.data(), I.S.data(), I.T.data(), I.pair.data())) return;
    bool ident = true;
    for (int r = 0; r < m && ident; ++r)
      for (int c = 0; c < m; ++c)
        if (I.S[(size_t)r * m + c] != (r == c ? 1.0 : 0.0)) {
          ident = false;
          break;
        }
    double* hs = S_.hat(i);
    for (int c = 0; c < m; ++c)
      for (int r = 0; r < m; ++r) hs[r + (size_t)c * m] = I.S[(size_t)r * m + c];
    double* ht = Tb_.hat(i);
    I.nb = std::min(b_, m);
    for (int c = 0; c < I.nb; ++c)
      for (int r = 0; r < m; ++r) ht[r + (size_t)c * m] = I.T[(size_t)r * m + c];
    I.M = I.T;
    schur_ident[a] = ident;
    schur_ok[a] = 1;
  });
  for (size_t a = 0; a < act.size(); ++a) {
    if (!schur_ok[a]) return fail(TP3B_ENOCONV, "batched jdqr: projected Schur form did not converge");
    if (!schur_ident[a]) rot.push_back(act[a]);
  }
  TP3B_TRY(sync());
  TP3B_HIP(hipMemcpyAsync(S_.d, S_.h.data(), sizeof(double) * S_.h.size(), hipMemcpyHostToDevice, s_));
  TP3B_HIP(hipMemcpyAsync(Tb_.d, Tb_.h.data(), sizeof(double) * Tb_.h.size(), hipMemcpyHostToDevice, s_));
  if (!rot.empty()) {
    std::vector<int> p, q, ldc, nc;
    std::vector<const double*> A, C, X;
    std::vector<double*> Y, Yb;
    for (int pass = 0; pass < 2; ++pass) {
      p.clear(); q.clear(); ldc.clear(); nc.clear(); A.clear(); C.clear(); X.clear(); Y.clear(); Yb.clear();
      for (int i : rot) {
        const Inst& I = in_[i];
        p.push_back(I.m);
        q.push_back(I.m);
        ldc.push_back(I.m);
        nc.push_back(I.m);
        A.push_back(pass ? I.AV() : I.V());
        C.push_back(S_.at(i));
        Y.push_back(I.TMP);
        X.push_back(I.TMP);
        Yb.push_back(pass ? I.AV() : I.V());
      }
      TP3B_TRY(gemm64(rot, p, q, 1.0, A, C, ldc, 0.0, Y));
      if (pass == 0) {
        TP3B_TRY(copy64(rot, nc, 1.0, X, Yb));
      } else {
        // the rotated A V stays where it was written (no copy back)
        for (int i : rot) {
          Inst& I = in_[i];
          std::swap(I.AVb, I.TMP);
          I.av0 = 0;
        }
      }
    }
  }
  // 2. residuals R = (I - Q Q^T)(A U - V T[:, :nb])
  {
    std::vector<int> nc, p, q, ldc;
    std::vector<const double*> X, A, C;
    std::vector<double*> Y;
    for (int i : act) {
      const Inst& I = in_[i];
      nc.push_back(I.nb);
      X.push_back(I.AV());
      Y.push_back(I.Rres);
      p.push_back(I.m);
      q.push_back(I.nb);
      ldc.push_back(I.m);
      A.push_back(I.V());
      C.push_back(Tb_.at(i));
    }
    TP3B_TRY(copy64(act, nc, 1.0, X, Y));
    TP3B_TRY(gemm64(act, p, q, -1.0, A, C, ldc, 1.0, Y));
  }
  std::vector<int> lk;
  for (int i : act) {
    Inst& I = in_[i];
    I.Cq.assign((size_t)std::max(I.k, 1) * I.nb, 0.0);
    if (I.k > 0) lk.push_back(i);
  }
  for (int pass = 0; pass < 2 && !lk.empty(); ++pass) {
    Small& dst = pass ? Cq2_ : Cq1_;
    std::vector<int> p, q, ldc;
    std::vector<const double*> A, B, C;
    std::vector<double*> Y;
    for (int i : lk) {
      const Inst& I = in_[i];
      p.push_back(I.k);
      q.push_back(I.nb);
      ldc.push_back(I.k);
      A.push_back(I.QV);
      B.push_back(I.Rres);
      C.push_back(dst.at(i));
      Y.push_back(I.Rres);
    }
    TP3B_TRY(dot_to_host(lk, p, q, A, B, dst));
    TP3B_TRY(gemm64(lk, p, q, -1.0, A, C, ldc, 1.0, Y));
    for (int i : lk) {
      Inst& I = in_[i];
      for (int e = 0; e < I.k * I.nb; ++e) I.Cq[e] += dst.hat(i)[e];
    }
  }
  // residual norms
  {
    TP3B_TRY(arena_room());
    Tab<BdotJob<double>> t;
    if (!ar_.alloc(t, (int)act.size())) return arena_full();
    for (int i : act) {
      const Inst& I = in_[i];
      BdotJob<double> j{};
      j.N = I.N; j.b = I.nb; j.nb = 1; j.V = I.Rres; j.bs = 0; j.W = I.Rres; j.part = I.bpart;
      j.H = Nrm_.at(i); j.hld = 1;
      int64_t i1, i2;
      bdot_job_shape(j, &i1, &i2);
      TableArena::add(t, j, i1, i2);
    }
    TP3B_HIP(ar_.upload(s_));
    TP3B_HIP(launch_bdot_grouped(t.d, s_));
    TP3B_HIP(hipMemcpyAsync(Nrm_.h.data(), Nrm_.d, sizeof(double) * Nrm_.h.size(), hipMemcpyDeviceToHost, s_));
    TP3B_TRY(sync());
  }
  stats_.t_rr += now_s() - t0;
  // 3. locking of the converged prefix; the others prepare their corrections
  std::vector<int> locking, restart;
  corr_.clear();
  for (int i : act) {
    Inst& I = in_[i];
    const int m = I.m, nb = I.nb;
    I.rn.assign(nb, 0.0);
    I.theta.assign(nb, 0.0);
    for (int j = 0; j < nb; ++j) {
      I.rn[j] = std::sqrt(std::max(Nrm_.hat(i)[j], 0.0));
      I.theta[j] = I.T[(size_t)j * m + j];
      if (!std::isfinite(I.rn[j]) || !std::isfinite(I.theta[j]))
        return fail(TP3B_ENONFINITE, "batched jdqr: non-finite residual");
    }
    int p = 0;
    while (p < nb && I.k + p < nev_) {
      const int blk = I.pair[p] ? 2 : 1;
      bool ok = p + blk <= nb;
      for (int q = p; ok && q < p + blk; ++q)
        ok = I.rn[q] <= o_.tol * std::max(std::fabs(I.theta[q]), 1.0);
      if (!ok) break;
      p += blk;
    }
    if (p == 0 && o_.stall_tol > 0) {
      // the leading residual has reached its FP64 rounding floor
      const double r0 = I.rn[0];
      if (r0 <= o_.stall_tol * std::max(std::fabs(I.theta[0]), 1.0) && r0 >= 0.9 * I.prev_rn0 &&
          r0 <= 1.1 * I.prev_rn0)
        ++I.stall;
      else
        I.stall = 0;
      I.prev_rn0 = r0;
      const int blk = I.pair[0] ? 2 : 1;
      if (I.stall >= 3 && blk <= nb) {
        p = blk;
        stats_.n_stall_lock += blk;
      }
    }
    if (p > 0) {
      I.prev_rn0 = INFINITY;
      I.stall = 0;
      if (I.k + p > nev_) p = nev_ - I.k;
      I.lockp = p;
      locking.push_back(i);
      continue;
    }
    I.lockp = 0;
    ++I.outer;
    if (I.outer > o_.max_outer) {
      I.done = true;
      I.status = TP3B_ENOCONV;
      continue;
    }
    I.restart = I.m + nb > m_max_;
    if (I.restart) restart.push_back(i);
    corr_.push_back(i);
  }
  // locking: R gains [Q^T A u_j; T_{1..j, j}], the preconditioned locked vectors
  // are kept for the projections
  if (!locking.empty()) {
    std::vector<int> nv;
    std::vector<const double*> X;
    std::vector<double*> Y;
    for (int i : locking) {
      Inst& I = in_[i];
      const int p = I.lockp, m_old = I.m;
      for (int j = 0; j < p; ++j) {
        for (int r = 0; r < I.k; ++r) I.Rl[r + (size_t)(I.k + j) * nev_] = I.Cq[r + (size_t)j * I.k];
        for (int r = 0; r < p; ++r)
          if (r <= j || (r == j + 1 && I.pair[j]))
            I.Rl[(I.k + r) + (size_t)(I.k + j) * nev_] = I.T[(size_t)r * m_old + j];
        I.lock_pair.push_back(I.pair[j]);
        I.lockres.push_back(I.rn[j]);
      }
      nv.push_back(p);
      X.push_back(I.V());
      Y.push_back(use_prec_ ? I.PQ + (int64_t)I.k * I.N : nullptr);
    }
    if (use_prec_) TP3B_TRY(prec64(locking, X, Y, nv));
    for (int i : locking) {
      Inst& I = in_[i];
      const int p = I.lockp, m_old = I.m;
      I.k += p;
      I.m -= p;
      I.av0 += p;
      std::vector<double> Mn((size_t)I.m * I.m);
      for (int r = 0; r < I.m; ++r)
        for (int c = 0; c < I.m; ++c) Mn[(size_t)r * I.m + c] = I.T[(size_t)(r + p) * m_old + (c + p)];
      I.M = Mn;
      stats_.n_lock_events++;
      if (I.k >= nev_ || I.m == 0) I.done = true;
    }
  }
  if (corr_.empty()) return TP3B_OK;
  // restart: keep the m_min leading Schur vectors, recompute the projection
  if (!restart.empty()) {
    std::vector<int> p, q;
    std::vector<const double*> A, B;
    for (int i : restart) {
      Inst& I = in_[i];
      I.m = std::max(m_min_, I.nb);
      p.push_back(I.m);
      q.push_back(I.m);
      A.push_back(I.V());
      B.push_back(I.AV());
      stats_.n_restart++;
    }
    TP3B_TRY(dot_to_host(restart, p, q, A, B, Mf_));
    for (int i : restart) {
      Inst& I = in_[i];
      I.M.assign((size_t)I.m * I.m, 0.0);
      for (int r = 0; r < I.m; ++r)
        for (int c = 0; c < I.m; ++c) I.M[(size_t)r * I.m + c] = Mf_.hat(i)[r + (size_t)c * I.m];
    }
  }
  // 4. correction equations
  const double target = std::isnan(o_.target) ? NAN : o_.target;
  for (int i : corr_) {
    Inst& I = in_[i];
    const double tg0 = std::isnan(target) ? I.op->sigma : target;
    // first outer iterations, nothing locked yet: a target below the spectrum
    const double tg = (I.k == 0 && I.outer <= o_.low_start) ? I.op->spec_lo : tg0;
    for (int j = 0; j < I.nb; ++j)
      Shift_.hat(i)[j] = (I.rn[j] > o_.switch_tol * std::fabs(I.theta[j])) ? tg : I.theta[j];
  }
  TP3B_HIP(hipMemcpyAsync(Shift_.d, Shift_.h.data(), sizeof(double) * Shift_.h.size(), hipMemcpyHostToDevice, s_));
  if (use_prec_) {
    // Y = P^{-1} Q~ H^{-1} with H = Q~^T P^{-1} Q~ (P^{-1} Q_lock kept from locking)
    std::vector<int> nv, p;
    std::vector<const double*> X, A, B, C;
    std::vector<double*> Y;
    std::vector<int> ldc;
    for (int i : corr_) {
      Inst& I = in_[i];
      nv.push_back(I.nb);
      X.push_back(I.V());
      Y.push_back(I.PQ + (int64_t)I.k * I.N);
    }
    TP3B_TRY(prec64(corr_, X, Y, nv));
    Y.clear();
    for (int i : corr_) {
      Inst& I = in_[i];
      const int nqt = I.k + I.nb;
      p.push_back(nqt);
      A.push_back(I.QV);
      B.push_back(I.PQ);
    }
    TP3B_TRY(dot_to_host(corr_, p, p, A, B, Hh_));
    for (int i : corr_) {
      Inst& I = in_[i];
      const int nqt = I.k + I.nb;
      std::vector<double> Hr((size_t)nqt * nqt), Hi((size_t)nqt * nqt);
      for (int r = 0; r < nqt; ++r)
        for (int c = 0; c < nqt; ++c) Hr[(size_t)r * nqt + c] = Hh_.hat(i)[r + (size_t)c * nqt];
      if (!lu_inverse(nqt, Hr.data(), Hi.data()))
        return fail(TP3B_ENOCONV, "batched jdqr: singular projected preconditioner");
      for (int r = 0; r < nqt; ++r)
        for (int c = 0; c < nqt; ++c) Hinv_.hat(i)[r + (size_t)c * nqt] = Hi[(size_t)r * nqt + c];
      C.push_back(Hinv_.at(i));
      ldc.push_back(nqt);
      Y.push_back(I.Yp);
    }
    TP3B_HIP(hipMemcpyAsync(Hinv_.d, Hinv_.h.data(), sizeof(double) * Hinv_.h.size(), hipMemcpyHostToDevice, s_));
    TP3B_TRY(gemm64(corr_, p, p, 1.0, B, C, ldc, 0.0, Y));
  }
  if (low_) {
    TP3B_TRY(arena_room());
    Tab<ConvJob<double, TW>> t;
    if (!ar_.alloc(t, 2 * (int)corr_.size())) return arena_full();
    for (int i : corr_) {
      Inst& I = in_[i];
      const int nqt = I.k + I.nb;
      const double* Yq = use_prec_ ? I.Yp : I.QV;
      TableArena::add(t, ConvJob<double, TW>{I.N, nqt, 1.0, I.QV, I.N, (TW*)I.Qtw, I.N}, rows_items(I.N, nqt));
      TableArena::add(t, ConvJob<double, TW>{I.N, nqt, 1.0, Yq, I.N, (TW*)I.Ypw, I.N}, rows_items(I.N, nqt));
    }
    TP3B_HIP(ar_.upload(s_));
    TP3B_HIP(launch_convert_grouped(t.d, s_));
  }
  // GMRES: fixed steps, all correcting instances in every launch
  const double tg0 = now_s();
  TP3B_TRY(sync());
  TP3B_TRY(build_gmres_tables());
  if (o_.graph) {
    if (!gexec_) {
      TP3B_HIP(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
      tp3b_status cs = launch_gmres();
      hipGraph_t gph = nullptr;
      hipError_t ce = hipStreamEndCapture(s_, &gph);
      if (cs != TP3B_OK) {
        if (gph) (void)hipGraphDestroy(gph);
        return cs;
      }
      TP3B_HIP(ce);
      graph_ = gph;
      TP3B_HIP(hipGraphInstantiate(&gexec_, graph_, nullptr, nullptr, 0));
    }
    TP3B_HIP(hipGraphLaunch(gexec_, s_));
  } else {
    TP3B_TRY(launch_gmres());
  }
  for (int i : corr_) {
    (low_ ? stats_.n_apply_H_low : stats_.n_apply_H_fp64) += (int64_t)in_[i].nb * steps_;
    if (use_prec_) stats_.n_apply_prec += (int64_t)in_[i].nb * (steps_ + 1);
  }
  Small* back[] = {&H1_, &H2_, &Hs_, &Beta_};
  for (Small* k : back)
    TP3B_HIP(hipMemcpyAsync(k->h.data(), k->d, sizeof(double) * k->h.size(), hipMemcpyDeviceToHost, s_));
  TP3B_TRY(sync());
  // least squares per column; the correction t = V_gmres y
  std::vector<int> ks(count_, 0);
  for (int i : corr_) {
    Inst& I = in_[i];
    double* yv = Y_.hat(i);
    std::fill(yv, yv + (size_t)b_ * hld_, 0.0);
    for (int j = 0; j < I.nb; ++j) {
      const double beta = Beta_.hat(i)[j];
      if (!(beta > 0)) continue;
      int kst = 0;
      for (int kk = 0; kk < steps_; ++kk) {
        kst = kk + 1;
        if (!(Hs_.hat(i)[(size_t)kk * b_ + j] > 1e-14 * beta)) break;
      }
      std::vector<double> Hm((size_t)(kst + 1) * kst, 0.0);
      for (int kk = 0; kk < kst; ++kk) {
        const double* a1 = H1_.hat(i) + (size_t)kk * b_ * hld_ + (size_t)j * hld_;
        const double* a2 = H2_.hat(i) + (size_t)kk * b_ * hld_ + (size_t)j * hld_;
        for (int r = 0; r <= kk; ++r) Hm[(size_t)r * kst + kk] = a1[r] + a2[r];
        Hm[(size_t)(kk + 1) * kst + kk] = Hs_.hat(i)[(size_t)kk * b_ + j];
      }
      std::vector<double> y(kst);
      hessenberg_lstsq(kst, Hm.data(), kst, beta, y.data());
      for (int r = 0; r < kst; ++r) yv[(size_t)j * hld_ + r] = y[r];
      ks[i] = std::max(ks[i], kst);
    }
  }
  TP3B_HIP(hipMemcpyAsync(Y_.d, Y_.h.data(), sizeof(double) * Y_.h.size(), hipMemcpyHostToDevice, s_));
  {
    TP3B_TRY(arena_room());
    Tab<ConvJob<TW, TW>> tz;
    Tab<BupdJob<TW>> tu;
    Tab<ConvJob<TW, double>> tc;
    const int n = (int)corr_.size();
    if (!ar_.alloc(tz, n) || !ar_.alloc(tu, n) || !ar_.alloc(tc, n)) return arena_full();
    for (int i : corr_) {
      Inst& I = in_[i];
      const int64_t N = I.N;
      TableArena::add(tz, ConvJob<TW, TW>{N, I.nb, 0.0, nullptr, N, (TW*)I.W, N}, rows_items(N, I.nb));
      TableArena::add(tu, BupdJob<TW>{N, I.nb, ks[i], 1.0, (const TW*)I.Vg, N * I.nb, Y_.at(i), hld_, (TW*)I.W},
                      ks[i] > 0 ? rows_items(N, I.nb) : 0);
      TableArena::add(tc, ConvJob<TW, double>{N, I.nb, 1.0, (const TW*)I.W, N, I.Tc, N}, rows_items(N, I.nb));
    }
    TP3B_HIP(ar_.upload(s_));
    TP3B_HIP(launch_convert_grouped(tz.d, s_));
    TP3B_HIP(launch_bupdate_grouped(tu.d, s_));
    TP3B_HIP(launch_convert_grouped(tc.d, s_));
  }
  stats_.t_gmres += now_s() - tg0;
  // 5. expand the basis: orthonormalise the corrections against [Q_lock, V]
  const double to = now_s();
  {
    std::vector<int> nc, nq;
    std::vector<const double*> X;
    std::vector<double*> Y, Qs;
    for (int i : corr_) {
      Inst& I = in_[i];
      nc.push_back(I.nb);
      X.push_back(I.Tc);
      Y.push_back(I.QV + (int64_t)(I.k + I.m) * I.N);
      nq.push_back(I.k + I.m);
      Qs.push_back(I.QV);
    }
    TP3B_TRY(copy64(corr_, nc, 1.0, X, Y));
    TP3B_TRY(orth(corr_, nq, Qs, Y, nc, o_.seed + 104729ull * (uint64_t)in_[corr_[0]].outer));
  }
  stats_.t_orth += now_s() - to;
  const double ta = now_s();
  {
    std::vector<double*> X, Y;
    std::vector<int> nv;
    for (int i : corr_) {
      Inst& I = in_[i];
      X.push_back(I.QV + (int64_t)(I.k + I.m) * I.N);
      Y.push_back(I.AV() + (int64_t)I.m * I.N);
      nv.push_back(I.nb);
    }
    TP3B_TRY(apply_H64(corr_, X, Y, nv));
    std::vector<int> p, q;
    std::vector<const double*> A, B;
    for (int i : corr_) {
      Inst& I = in_[i];
      p.push_back(I.m + I.nb);
      q.push_back(I.nb);
      A.push_back(I.V());
      B.push_back(I.AV() + (int64_t)I.m * I.N);
    }
    TP3B_TRY(dot_to_host(corr_, p, q, A, B, Top_));
    p.clear(); q.clear(); A.clear(); B.clear();
    for (int i : corr_) {
      Inst& I = in_[i];
      p.push_back(I.nb);
      q.push_back(I.m);
      A.push_back(I.QV + (int64_t)(I.k + I.m) * I.N);
      B.push_back(I.AV());
    }
    TP3B_TRY(dot_to_host(corr_, p, q, A, B, Left_));
    for (int i : corr_) {
      Inst& I = in_[i];
      const int m = I.m, nb = I.nb, mn = m + nb;
      std::vector<double> Mn((size_t)mn * mn, 0.0);
      for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) Mn[(size_t)r * mn + c] = I.M[(size_t)r * m + c];
      for (int r = 0; r < mn; ++r)
        for (int c = 0; c < nb; ++c) Mn[(size_t)r * mn + m + c] = Top_.hat(i)[r + (size_t)c * mn];
      for (int r = 0; r < nb; ++r)
        for (int c = 0; c < m; ++c) Mn[(size_t)(m + r) * mn + c] = Left_.hat(i)[r + (size_t)c * nb];
      I.m = mn;
      I.M = Mn;
    }
  }
  stats_.t_apply += now_s() - ta;
  return TP3B_OK;
}

template <typename TW>
tp3b_status BatchedJdqr<TW>::run(double* evals, double* resnorm, int32_t* n_conv,
                                 int32_t* n_outer, double* const* Q, tp3b_jdqr_stats* st) {
  const double t_start = now_s();
  TP3B_TRY(setup());
  // start blocks: counter-based random vectors, orthonormalised
  std::vector<int> all(count_);
  std::vector<int> nq0(count_, 0);
  std::vector<double*> Xs(count_), Qn(count_, nullptr), AVs(count_);
  for (int i = 0; i < count_; ++i) {
    all[i] = i;
    Inst& I = in_[i];
    for (int j = 0; j < b_; ++j)
      TP3B_HIP(launch_hash_fill(I.N, I.QV + (int64_t)j * I.N, o_.seed + (uint64_t)i, 1000003ull + j, s_));
    Xs[i] = I.QV;
    AVs[i] = I.AVb;
  }
  double t0 = now_s();
  const std::vector<int> bvec(count_, b_);
  TP3B_TRY(orth(all, nq0, Qn, Xs, bvec, o_.seed + 17));
  stats_.t_orth += now_s() - t0;
  t0 = now_s();
  TP3B_TRY(apply_H64(all, Xs, AVs, bvec));
  {
    std::vector<int> p(count_, b_);
    std::vector<const double*> A(Xs.begin(), Xs.end()), B(AVs.begin(), AVs.end());
    TP3B_TRY(dot_to_host(all, p, p, A, B, Mf_));
  }
  for (int i = 0; i < count_; ++i) {
    Inst& I = in_[i];
    I.m = b_;
    I.M.assign((size_t)b_ * b_, 0.0);
    for (int r = 0; r < b_; ++r)
      for (int c = 0; c < b_; ++c) I.M[(size_t)r * b_ + c] = Mf_.hat(i)[r + (size_t)c * b_];
  }
  stats_.t_apply += now_s() - t0;
  int iters = 0;
  for (;;) {
    bool any = false;
    for (const Inst& I : in_) any |= !I.done;
    if (!any) break;
    if (o_.verbose) {
      int nd = 0;
      for (const Inst& I : in_) nd += I.done;
      fprintf(stderr, "[tp3b batched jdqr] step %d: %d of %d instances done\n", iters, nd, count_);
    }
    TP3B_TRY(iterate());
    ++iters;
  }
  TP3B_TRY(sync());
  // outputs
  tp3b_status status = TP3B_OK;
  int max_outer = 0;
  for (int i = 0; i < count_; ++i) {
    Inst& I = in_[i];
    const int nconv = I.k;
    std::vector<double> ev(nconv);
    for (int a = 0; a < nconv; ++a) {
      if (a + 1 < nconv && I.lock_pair[a]) {
        const double x = I.Rl[a + (size_t)a * nev_], y = I.Rl[(a + 1) + (size_t)(a + 1) * nev_];
        ev[a] = ev[a + 1] = 0.5 * (x + y);
        ++a;
      } else {
        ev[a] = I.Rl[a + (size_t)a * nev_];
      }
    }
    std::sort(ev.begin(), ev.end());
    if (evals)
      for (int a = 0; a < nev_; ++a) evals[(size_t)i * nev_ + a] = a < nconv ? ev[a] : NAN;
    if (resnorm)
      for (int a = 0; a < nev_; ++a)
        resnorm[(size_t)i * nev_ + a] = a < (int)I.lockres.size() ? I.lockres[a] : NAN;
    if (n_conv) n_conv[i] = nconv;
    if (n_outer) n_outer[i] = I.outer;
    if (Q && Q[i] && nconv > 0)
      TP3B_HIP(hipMemcpyAsync(Q[i], I.QV, sizeof(double) * I.N * nconv, hipMemcpyDeviceToDevice, s_));
    if (nconv < nev_) status = TP3B_ENOCONV;
    max_outer = std::max(max_outer, I.outer);
    stats_.n_conv += nconv;
  }
  TP3B_TRY(sync());
  stats_.n_outer = max_outer;
  stats_.t_total = now_s() - t_start;
  if (st) *st = stats_;
  if (status != TP3B_OK) return fail(status, "batched jdqr: some instances did not converge within max_outer");
  return TP3B_OK;
}

}  // namespace
}  // namespace tp3b

using namespace tp3b;

extern "C" {

tp3b_status tp3b_apply_H_batched(const tp3b_op* ops, int32_t count, int32_t prec, int32_t nvec,
                                 const void* const* X, const int64_t* ldx, void* const* Y,
                                 const int64_t* ldy, const double* const* shifts, void* stream) {
  try {
    tp3b_status st = check_batched_apply(ops, count, prec, nvec, X, ldx, Y, ldy, false);
    if (st != TP3B_OK || nvec == 0) return st;
    hipStream_t s = (hipStream_t)stream;
    if (prec == TP3B_FP64)
      return apply_batched<double>(ops, count, nvec, X, ldx, Y, ldy, shifts, false, false, s);
    return apply_batched<float>(ops, count, nvec, X, ldx, Y, ldy, shifts, false, prec == TP3B_BF16X3, s);
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_apply_prec_batched(const tp3b_op* ops, int32_t count, int32_t prec, int32_t nvec,
                                    const void* const* X, const int64_t* ldx, void* const* Y,
                                    const int64_t* ldy, void* stream) {
  try {
    tp3b_status st = check_batched_apply(ops, count, prec, nvec, X, ldx, Y, ldy, true);
    if (st != TP3B_OK || nvec == 0) return st;
    hipStream_t s = (hipStream_t)stream;
    if (prec == TP3B_FP64)
      return apply_batched<double>(ops, count, nvec, X, ldx, Y, ldy, nullptr, true, false, s);
    return apply_batched<float>(ops, count, nvec, X, ldx, Y, ldy, nullptr, true, prec == TP3B_BF16X3, s);
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_autotune_batched(const tp3b_op* ops, int32_t count, int32_t prec, int32_t nvec,
                                  int32_t reps) {
  try {
    tp3b_status st = check_batch(ops, count, false);
    if (st != TP3B_OK) return st;
    if (prec != TP3B_FP64 && prec != TP3B_FP32 && prec != TP3B_BF16X3)
      return fail(TP3B_EINVAL, "unknown precision");
    if (nvec < 1 || reps < 1) return fail(TP3B_EINVAL, "nvec and reps must be >= 1");
    for (int i = 0; i < count; ++i)
      if (nvec > ops[i]->work_vecs) return fail(TP3B_EINVAL, "autotune_batched: nvec too large");
    const bool f64 = prec == TP3B_FP64, bf3 = prec == TP3B_BF16X3;
    const size_t es = f64 ? 8 : 4;
    // groups of equal grid size
    std::vector<std::vector<int>> groups;
    std::vector<std::pair<int, int>> keys;
    for (int i = 0; i < count; ++i) {
      const std::pair<int, int> key(ops[i]->n[0], ops[i]->n[1]);
      size_t g = 0;
      while (g < keys.size() && keys[g] != key) ++g;
      if (g == keys.size()) {
        keys.push_back(key);
        groups.emplace_back();
      }
      groups[g].push_back(i);
    }
    // scratch blocks (zero: timing does not depend on the values)
    size_t maxb = 0;
    for (int i = 0; i < count; ++i) maxb += es * ops[i]->N * nvec;
    void *X = nullptr, *Y = nullptr;
    TP3B_HIP(hipMalloc(&X, maxb));
    if (hipMalloc(&Y, maxb) != hipSuccess) {
      (void)hipFree(X);
      return fail(TP3B_ENOMEM, "autotune_batched: scratch allocation failed");
    }
    (void)hipMemset(X, 0, maxb);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    st = TP3B_OK;
    const int pi = f64 ? TP3B_FP64 : (bf3 ? TP3B_BF16X3 : TP3B_FP32);
    for (size_t g = 0; g < groups.size() && st == TP3B_OK; ++g) {
      const std::vector<int>& gi = groups[g];
      std::vector<tp3b_op> gops;
      std::vector<const void*> xs;
      std::vector<void*> ys;
      std::vector<int64_t> ld;
      size_t o = 0;
      for (int i : gi) {
        gops.push_back(ops[i]);
        xs.push_back((char*)X + o);
        ys.push_back((char*)Y + o);
        ld.push_back(ops[i]->N);
        o += es * ops[i]->N * nvec;
      }
      const int nx = keys[g].first, ny = keys[g].second;
      for (int kind = 0; kind < 2 && st == TP3B_OK; ++kind) {
        const bool kprec = kind == 1;
        if (kprec) {
          bool all = true;
          for (int i : gi) all &= ops[i]->have_prec;
          if (!all) break;
        }
        double best = 1e300;
        int best_tile = -1;
        std::vector<int> saved;
        for (int i : gi) saved.push_back(ops[i]->tile_override);
        for (int tile = 0; tile < NUM_TILE_CFGS && st == TP3B_OK; ++tile) {
          const int tm = tile_rows(tile), tn = tile_cols(tile);
          if (tm > 32 && (tm > nx || tn > ny)) continue;
          if (bf3 && tm == 32) continue;
          for (int i : gi) ops[i]->tile_override = tile;
          auto run = [&]() -> tp3b_status {
            if (f64)
              return apply_batched<double>(gops.data(), (int)gops.size(), nvec, xs.data(), ld.data(),
                                           ys.data(), ld.data(), nullptr, kprec, false, nullptr);
            return apply_batched<float>(gops.data(), (int)gops.size(), nvec, xs.data(), ld.data(),
                                        ys.data(), ld.data(), nullptr, kprec, bf3, nullptr);
          };
          st = run();
          if (st != TP3B_OK) break;
          // apply_batched synchronises before staging its tables, so each
          // repetition is timed separately and the times summed
          double ms_total = 0.0;
          for (int r = 0; r < reps && st == TP3B_OK; ++r) {
            (void)hipDeviceSynchronize();
            (void)hipEventRecord(e0, nullptr);
            st = run();
            (void)hipEventRecord(e1, nullptr);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms_total += ms;
          }
          if (ms_total / reps < best) {
            best = ms_total / reps;
            best_tile = tile;
          }
        }
        for (size_t a = 0; a < gi.size(); ++a) ops[gi[a]]->tile_override = saved[a];
        if (st == TP3B_OK)
          for (int i : gi) ops[i]->tuned[pi][kind] = best_tile;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(X);
    (void)hipFree(Y);
    return st;
  } catch (...) {
    return exception_status();
  }
}

tp3b_status tp3b_jdqr_solve_batched(const tp3b_op* ops, int32_t count, const tp3b_jdqr_opts* opts,
                                    double* evals, double* resnorm, int32_t* n_conv,
                                    int32_t* n_outer, double* const* Q, tp3b_jdqr_stats* stats) {
  try {
    if (!opts) return fail(TP3B_EINVAL, "null options");
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
    if (o.nev + o.m_max + o.block > 64) return fail(TP3B_EINVAL, "batched: nev + m_max + block must be <= 64");
    tp3b_status st = check_batch(ops, count, o.precond != 0);
    if (st != TP3B_OK) return st;
    for (int i = 0; i < count; ++i) {
      if (ops[i]->N < (int64_t)(o.nev + o.m_max + o.block))
        return fail(TP3B_EINVAL, "batched: an instance is too small for nev + m_max + block vectors");
      if (o.precond && (o.block > ops[i]->work_vecs || o.nev > ops[i]->work_vecs))
        return fail(TP3B_EINVAL, "batched: block larger than the preconditioner's work buffer");
    }
    if (o.inner_prec != TP3B_FP64 && o.inner_prec != TP3B_FP32 && o.inner_prec != TP3B_BF16X3)
      return fail(TP3B_EINVAL, "unknown inner precision");
    if (o.inner_prec == TP3B_FP64) {
      BatchedJdqr<double> solver(ops, count, o, false);
      return solver.run(evals, resnorm, n_conv, n_outer, Q, stats);
    }
    BatchedJdqr<float> solver(ops, count, o, o.inner_prec == TP3B_BF16X3);
    return solver.run(evals, resnorm, n_conv, n_outer, Q, stats);
  } catch (...) {
    return exception_status();
  }
}

}  // extern "C"
