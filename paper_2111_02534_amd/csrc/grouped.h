// Grouped (multi-instance) launches: many independent jobs of one kind -- one
// per problem instance -- in a single persistent launch.
//
// A job table lives in device memory as
//   int64 hdr[0] = njobs, hdr[1] = cap,
//   int64 first[cap + 1]   prefix sums of the jobs' work items (stage 1),
//   int64 first2[cap + 1]  prefix sums for the second stage of two-stage kernels,
//   Job   jobs[cap]        (16-byte aligned).
// Kernels read njobs and the prefix sums from memory, so a table may be
// rewritten between launches, or between replays of a captured graph, without
// changing any kernel argument.  Each launch has a fixed grid; every workgroup
// loops over its share of the work items (the 8 XCDs each take a contiguous
// range, which keeps the tiles of one instance inside one L2) and exits when
// the range is done.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>
#include <vector>

#include "kernels.h"

namespace tp3b {

// Workgroups per persistent launch (a multiple of the 8 XCDs; 8 per CU).
constexpr int kPersistWGs = 2048;

template <typename TA, typename TB>
struct DotJob {  // C (p x q, ldc) = A^T B
  int64_t N;
  int p, q;
  const TA* A;
  int64_t lda;
  const TB* B;
  int64_t ldb;
  double* C;
  int ldc;
  int rchunk, nchunk, tiles_q;
  double* part;  // nchunk * tiles * 64 * 32 doubles
};

template <typename T>
struct GemmJob {  // Y = beta Y + alpha A C
  int64_t N;
  int p, q;
  double alpha, beta;
  const T* A;
  int64_t lda;
  const double* C;
  int ldc;
  T* Y;
  int64_t ldy;
};

template <typename T>
struct BdotJob {  // H[j*hld + i] = sum_r Vb[i][r, j] W[r, j], i < nb, j < b
  int64_t N;
  int b, nb;
  const T* V;
  int64_t bs;
  const T* W;
  int rows, nchunk;
  double* part;  // nchunk * b * BD_MAXNB doubles
  double* H;
  int hld;
};

template <typename T>
struct BupdJob {  // W[r, j] += alpha sum_{i<nb} Vb[i][r, j] H[j*hld + i]
  int64_t N;
  int b, nb;
  double alpha;
  const T* V;
  int64_t bs;
  const double* H;
  int hld;
  T* W;
};

template <typename T>
struct NormJob {  // Vout[:, j] = W[:, j] / sqrt(nrm2[j]); hout[j*hld] = sqrt(nrm2[j])
  int64_t N;
  int b;
  const double* nrm2;
  const T* W;
  T* Vout;
  double* hout;
  int hld;
};

template <typename TI, typename TO>
struct ConvJob {  // Y[:, j] = alpha X[:, j] (X == nullptr: Y = 0)
  int64_t N;
  int ncol;
  double alpha;
  const TI* X;
  int64_t ldx;
  TO* Y;
  int64_t ldy;
};

struct CholJob {
  int nx;
  double drop_tol;
  const double* G;
  const double* n0;
  double* R;
  int* flags;
};

struct TrsmJob {  // X (N x nx) <- X R^{-1}
  int64_t N;
  int nx;
  const double* R;
  double* X;
  int64_t ldx;
};

// A table as the kernels see it.
template <class Job>
struct DevTab {
  const int64_t* hdr = nullptr;
  const Job* jobs = nullptr;
};

// Host staging of job tables with a mirrored device arena; tables are appended
// in order, and upload() copies the tables added since the previous upload in
// one transfer.  Rebuilding the same sequence of tables after reset() (same
// capacities) yields the same device addresses.
class TableArena {
 public:
  TableArena() = default;
  TableArena(const TableArena&) = delete;
  TableArena& operator=(const TableArena&) = delete;
  ~TableArena();
  hipError_t init(size_t bytes);
  // Only after the stream has consumed every uploaded table.
  void reset() { used_ = uploaded_ = 0; }
  size_t free_bytes() const { return cap_ - used_; }

  template <class Job>
  struct Tab {
    int64_t* h = nullptr;  // host header
    Job* hj = nullptr;
    DevTab<Job> d;
    int cap = 0;
    int njobs() const { return (int)h[0]; }
    int64_t total() const { return h[2 + h[0]]; }
    int64_t total2() const { return h[2 + (cap + 1) + h[0]]; }
  };

  // Returns false when the arena is full.
  template <class Job>
  bool alloc(Tab<Job>& t, int cap) {
    const size_t hdr_bytes = sizeof(int64_t) * (2 + 2 * (size_t)(cap + 1));
    const size_t job_off = (hdr_bytes + 15) & ~(size_t)15;
    const size_t bytes = (job_off + sizeof(Job) * (size_t)cap + 255) & ~(size_t)255;
    if (used_ + bytes > cap_) return false;
    t.h = (int64_t*)(host_ + used_);
    t.hj = (Job*)(host_ + used_ + job_off);
    t.d.hdr = (const int64_t*)(dev_ + used_);
    t.d.jobs = (const Job*)(dev_ + used_ + job_off);
    t.cap = cap;
    std::memset(t.h, 0, hdr_bytes);
    t.h[1] = cap;
    used_ += bytes;
    return true;
  }

  template <class Job>
  static void add(Tab<Job>& t, const Job& j, int64_t items, int64_t items2 = 0) {
    const int64_t n = t.h[0];
    int64_t* first = t.h + 2;
    int64_t* first2 = t.h + 2 + (t.cap + 1);
    t.hj[n] = j;
    first[n + 1] = first[n] + items;
    first2[n + 1] = first2[n] + items2;
    t.h[0] = n + 1;
  }

  // Copies the tables added since the last upload (one transfer).
  hipError_t upload(hipStream_t s);
  size_t used() const { return used_; }

 private:
  char* host_ = nullptr;
  char* dev_ = nullptr;
  size_t cap_ = 0, used_ = 0, uploaded_ = 0;
};

// ---- launchers (fixed grid of kPersistWGs workgroups; tables in device memory)
// Mode products: work items are output tiles (modeprod_items for the tile
// shape), so a table is built for one tile shape and launched with it.
template <typename T>
hipError_t launch_modeprod_grouped(DevTab<ModeProd<T>> t, int tile, hipStream_t s);
hipError_t launch_modeprod_bf3_grouped(DevTab<ModeProd<float>> t, int tile, hipStream_t s);
int64_t modeprod_items_for(int M, int Nc, int nbatch, int tile, bool bf3);

// Stage-1 items: nchunk * tiles per job; stage-2 items: p * q per job.
template <typename TA, typename TB>
hipError_t launch_dot_grouped(DevTab<DotJob<TA, TB>> t, hipStream_t s);
template <typename TA, typename TB>
void dot_job_shape(DotJob<TA, TB>& j, int64_t* items1, int64_t* items2);  // fills rchunk..tiles_q
int64_t dot_job_partials(int64_t N, int p, int q);

// Items: ceil(N/256) * ceil(q/16).
template <typename T>
hipError_t launch_gemm_grouped(DevTab<GemmJob<T>> t, hipStream_t s);
int64_t gemm_job_items(int64_t N, int q);

// Stage-1 items: nchunk * b; stage-2 items: b * nb.
template <typename T>
hipError_t launch_bdot_grouped(DevTab<BdotJob<T>> t, hipStream_t s);
template <typename T>
void bdot_job_shape(BdotJob<T>& j, int64_t* items1, int64_t* items2);
int64_t bdot_job_partials(int64_t N, int b);

// Items: ceil(N/256) * (columns).
template <typename T>
hipError_t launch_bupdate_grouped(DevTab<BupdJob<T>> t, hipStream_t s);
template <typename T>
hipError_t launch_normalize_grouped(DevTab<NormJob<T>> t, hipStream_t s);
template <typename TI, typename TO>
hipError_t launch_convert_grouped(DevTab<ConvJob<TI, TO>> t, hipStream_t s);
int64_t rows_items(int64_t N, int ncol);

// Items: 1 per job (one thread does the factorisation).
hipError_t launch_chol_grouped(DevTab<CholJob> t, hipStream_t s);
// Items: ceil(N/256).
hipError_t launch_trsm_grouped(DevTab<TrsmJob> t, hipStream_t s);

}  // namespace tp3b
