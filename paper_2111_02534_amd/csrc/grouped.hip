// Grouped persistent kernels: the bodies of kernels.hip applied to every job of
// a device job table (see grouped.h), one launch per kind of work.
#include "grouped.h"

#include <hip/hip_runtime.h>

#include "device_bodies.h"

namespace tp3b {

// ------------------------------------------------------------- work lookup
// Largest j < nj with first[j] <= w (jobs without work are skipped).
__device__ __forceinline__ int find_job(const int64_t* __restrict__ first, int nj, int64_t w) {
  int lo = 0, hi = nj - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= w)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Calls f(job, local item) for this workgroup's work items of stage `stage`.
// XCD x (= blockIdx % 8) owns the contiguous range [total x / 8, total (x+1) / 8).
template <class Job, class F>
__device__ __forceinline__ void for_wg_items(DevTab<Job> t, int stage, F&& f) {
  const int nj = (int)t.hdr[0];
  const int64_t cap = t.hdr[1];
  const int64_t* first = t.hdr + 2 + (stage ? cap + 1 : 0);
  if (nj <= 0) return;
  const int64_t total = first[nj];
  const int64_t G8 = gridDim.x >> 3;
  const int64_t x = blockIdx.x & 7, l = blockIdx.x >> 3;
  const int64_t beg = total * x / 8, end = total * (x + 1) / 8;
  for (int64_t w = beg + l; w < end; w += G8) {
    const int j = find_job(first, nj, w);
    const Job job = t.jobs[j];  // a private copy: stores through Y cannot alias it
    f(job, w - first[j]);
  }
}

// Calls f(job, local item, lane) for this wavefront's work items (one item per
// wavefront; used by the reductions' second stage).
template <class Job, class F>
__device__ __forceinline__ void for_wave_items(DevTab<Job> t, int stage, F&& f) {
  const int nj = (int)t.hdr[0];
  const int64_t cap = t.hdr[1];
  const int64_t* first = t.hdr + 2 + (stage ? cap + 1 : 0);
  if (nj <= 0) return;
  const int64_t total = first[nj];
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * 4;
  for (int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); w < total; w += stride) {
    const int j = find_job(first, nj, w);
    const Job job = t.jobs[j];
    f(job, w - first[j], lane);
  }
}

// ------------------------------------------------------------ mode products
// At least two waves per SIMD, as for the single-job mode-product kernel.
template <typename T, int TM, int TN, int KC, bool SK = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_modeprod_grouped(
    DevTab<ModeProd<T>> t) {
  __shared__ MpSmem<T, TM, TN, KC, SK> sm;
  for_wg_items(t, 0, [&](const ModeProd<T>& a, int64_t w) {
    modeprod_tile<T, TM, TN, KC, SK>(a, w, sm);
  });
}

// The small split-K tile with eight waves (same body as the single-job form).
template <typename T>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_modeprod_sk8_grouped(
    DevTab<ModeProd<T>> t) {
  __shared__ MpSmem<T, 32, 32, 64, true, 8> sm;
  for_wg_items(t, 0, [&](const ModeProd<T>& a, int64_t w) {
    modeprod_tile<T, 32, 32, 64, true, 8>(a, w, sm);
  });
}

template <int TM, int TN, int KC>
__global__ __launch_bounds__(256) void k_modeprod_bf3_grouped(DevTab<ModeProd<float>> t) {
  __shared__ Bf3Smem<TM, TN, KC> sm;
  for_wg_items(t, 0, [&](const ModeProd<float>& a, int64_t w) {
    modeprod_bf3_tile<TM, TN, KC>(a, w, sm);
  });
}

int64_t modeprod_items_for(int M, int Nc, int nbatch, int tile, bool bf3) {
  struct P { int M, Nc, nbatch; } p{M, Nc, nbatch};
  switch (tile) {
    case TILE_32:
    case TILE_32W8: return bf3 ? modeprod_items<64, 64>(p) : modeprod_items<32, 32>(p);
    case TILE_64: return modeprod_items<64, 64>(p);
    case TILE_128: return modeprod_items<128, 128>(p);
    default: return modeprod_items<64, 128>(p);
  }
}

template <typename T>
hipError_t launch_modeprod_grouped(DevTab<ModeProd<T>> t, int tile, hipStream_t s) {
  const dim3 g(kPersistWGs), b(256);
  switch (tile) {
    case TILE_32: hipLaunchKernelGGL((k_modeprod_grouped<T, 32, 32, 64, true>), g, b, 0, s, t); break;
    case TILE_32W8: hipLaunchKernelGGL((k_modeprod_sk8_grouped<T>), g, dim3(512), 0, s, t); break;
    case TILE_64: hipLaunchKernelGGL((k_modeprod_grouped<T, 64, 64, 16>), g, b, 0, s, t); break;
    case TILE_128: hipLaunchKernelGGL((k_modeprod_grouped<T, 128, 128, 16>), g, b, 0, s, t); break;
    case TILE_64x128: hipLaunchKernelGGL((k_modeprod_grouped<T, 64, 128, 16>), g, b, 0, s, t); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_modeprod_grouped<double>(DevTab<ModeProd<double>>, int, hipStream_t);
template hipError_t launch_modeprod_grouped<float>(DevTab<ModeProd<float>>, int, hipStream_t);

hipError_t launch_modeprod_bf3_grouped(DevTab<ModeProd<float>> t, int tile, hipStream_t s) {
  const dim3 g(kPersistWGs), b(256);
  switch (tile) {
    case TILE_32:
    case TILE_32W8:
    case TILE_64: hipLaunchKernelGGL((k_modeprod_bf3_grouped<64, 64, 32>), g, b, 0, s, t); break;
    case TILE_128: hipLaunchKernelGGL((k_modeprod_bf3_grouped<128, 128, 32>), g, b, 0, s, t); break;
    case TILE_64x128: hipLaunchKernelGGL((k_modeprod_bf3_grouped<64, 128, 32>), g, b, 0, s, t); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------- dots
int64_t dot_job_partials(int64_t N, int p, int q) {
  const int rc = dot_row_chunk_grouped(N);
  const int64_t nchunk = N > 0 ? (N + rc - 1) / rc : 0;
  const int64_t tiles = (int64_t)((p + DOT_TP - 1) / DOT_TP) * ((q + DOT_TQ - 1) / DOT_TQ);
  return nchunk * tiles * DOT_TP * DOT_TQ;
}

template <typename TA, typename TB>
void dot_job_shape(DotJob<TA, TB>& j, int64_t* items1, int64_t* items2) {
  j.rchunk = dot_row_chunk_grouped(j.N);
  j.nchunk = j.N > 0 ? (int)((j.N + j.rchunk - 1) / j.rchunk) : 0;
  j.tiles_q = (j.q + DOT_TQ - 1) / DOT_TQ;
  const int tiles = ((j.p + DOT_TP - 1) / DOT_TP) * j.tiles_q;
  *items1 = (j.p > 0 && j.q > 0) ? (int64_t)j.nchunk * tiles : 0;
  *items2 = (j.p > 0 && j.q > 0) ? (int64_t)j.p * j.q : 0;
}

template <typename TA, typename TB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_dot_grouped(DevTab<DotJob<TA, TB>> t) {
  __shared__ DotSmem sm;
  for_wg_items(t, 0, [&](const DotJob<TA, TB>& j, int64_t w) {
    const int chunk = (int)(w % j.nchunk), tile = (int)(w / j.nchunk);
    dot_tile<TA, TB>(j.N, j.p, j.q, j.A, j.lda, j.B, j.ldb, j.rchunk, j.tiles_q, chunk, tile,
                     j.part + ((int64_t)tile * j.nchunk + chunk) * (DOT_TP * DOT_TQ), sm);
  });
}

template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_dot_reduce_grouped(DevTab<DotJob<TA, TB>> t) {
  for_wave_items(t, 1, [&](const DotJob<TA, TB>& j, int64_t w, int lane) {
    const int gp = (int)(w % j.p), gq = (int)(w / j.p);
    double s = 0.0;
    if (j.nchunk > 0) s = dot_reduce_elem(gp, gq, j.nchunk, j.tiles_q, j.part, lane);
    if (lane == 0) j.C[gp + (int64_t)gq * j.ldc] = s;
  });
}

template <typename TA, typename TB>
hipError_t launch_dot_grouped(DevTab<DotJob<TA, TB>> t, hipStream_t s) {
  hipLaunchKernelGGL((k_dot_grouped<TA, TB>), dim3(kPersistWGs), dim3(256), 0, s, t);
  hipLaunchKernelGGL((k_dot_reduce_grouped<TA, TB>), dim3(kPersistWGs / 4), dim3(256), 0, s, t);
  return hipGetLastError();
}
template hipError_t launch_dot_grouped<double, double>(DevTab<DotJob<double, double>>, hipStream_t);
template hipError_t launch_dot_grouped<float, float>(DevTab<DotJob<float, float>>, hipStream_t);
template void dot_job_shape<double, double>(DotJob<double, double>&, int64_t*, int64_t*);
template void dot_job_shape<float, float>(DotJob<float, float>&, int64_t*, int64_t*);

// ------------------------------------------------------------ basis update
int64_t gemm_job_items(int64_t N, int q) {
  return (N > 0 && q > 0) ? ((N + gemm_rows<false>() - 1) / gemm_rows<false>()) * ((q + GEMM_QB - 1) / GEMM_QB) : 0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_grouped(DevTab<GemmJob<T>> t) {
  __shared__ GemmSmem<false> sm;
  for_wg_items(t, 0, [&](const GemmJob<T>& j, int64_t w) {
    const int64_t nrb = (j.N + gemm_rows<false>() - 1) / gemm_rows<false>();
    gemm_block<T, false>(j.N, j.p, j.q, j.alpha, j.A, j.lda, j.C, j.ldc, j.beta, j.Y, j.ldy, w % nrb,
                  (int)(w / nrb), sm);
  });
}

template <typename T>
hipError_t launch_gemm_grouped(DevTab<GemmJob<T>> t, hipStream_t s) {
  hipLaunchKernelGGL((k_gemm_grouped<T>), dim3(kPersistWGs), dim3(256), 0, s, t);
  return hipGetLastError();
}
template hipError_t launch_gemm_grouped<double>(DevTab<GemmJob<double>>, hipStream_t);
template hipError_t launch_gemm_grouped<float>(DevTab<GemmJob<float>>, hipStream_t);

// ------------------------------------------------ per-column (diagonal) dots
int64_t bdot_job_partials(int64_t N, int b) {
  const int rows = bdot_rows(N);
  return ((N + rows - 1) / rows) * b * BD_MAXNB;
}

template <typename T>
void bdot_job_shape(BdotJob<T>& j, int64_t* items1, int64_t* items2) {
  j.rows = bdot_rows(j.N);
  j.nchunk = (int)((j.N + j.rows - 1) / j.rows);
  *items1 = (j.nb > 0 && j.b > 0) ? (int64_t)j.nchunk * j.b : 0;
  *items2 = (j.nb > 0 && j.b > 0) ? (int64_t)j.b * j.nb : 0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_bdot_grouped(DevTab<BdotJob<T>> t) {
  __shared__ BdotSmem sm;
  for_wg_items(t, 0, [&](const BdotJob<T>& j, int64_t w) {
    const int chunk = (int)(w % j.nchunk), col = (int)(w / j.nchunk);
    bdot_chunk<T>(j.N, j.nb, j.V, j.bs, j.W, j.rows, chunk, col,
                  j.part + ((int64_t)chunk * j.b + col) * BD_MAXNB, sm);
  });
}

template <typename T>
__global__ __launch_bounds__(256) void k_bdot_reduce_grouped(DevTab<BdotJob<T>> t) {
  for_wave_items(t, 1, [&](const BdotJob<T>& j, int64_t w, int lane) {
    const int col = (int)(w / j.nb), i = (int)(w % j.nb);
    const double s = bdot_reduce_elem(j.b, col, i, j.nchunk, j.part, lane);
    if (lane == 0) j.H[(int64_t)col * j.hld + i] = s;
  });
}

template <typename T>
hipError_t launch_bdot_grouped(DevTab<BdotJob<T>> t, hipStream_t s) {
  hipLaunchKernelGGL((k_bdot_grouped<T>), dim3(kPersistWGs), dim3(256), 0, s, t);
  hipLaunchKernelGGL((k_bdot_reduce_grouped<T>), dim3(kPersistWGs / 4), dim3(256), 0, s, t);
  return hipGetLastError();
}
template hipError_t launch_bdot_grouped<double>(DevTab<BdotJob<double>>, hipStream_t);
template hipError_t launch_bdot_grouped<float>(DevTab<BdotJob<float>>, hipStream_t);
template void bdot_job_shape<double>(BdotJob<double>&, int64_t*, int64_t*);
template void bdot_job_shape<float>(BdotJob<float>&, int64_t*, int64_t*);

// ------------------------------------------------------- row-block kernels
int64_t rows_items(int64_t N, int ncol) { return (N > 0 && ncol > 0) ? ((N + 255) / 256) * ncol : 0; }

template <typename T>
__global__ __launch_bounds__(256) void k_bupdate_grouped(DevTab<BupdJob<T>> t) {
  for_wg_items(t, 0, [&](const BupdJob<T>& j, int64_t w) {
    const int64_t nrb = (j.N + 255) / 256;
    bupdate_row<T>(j.N, j.nb, j.alpha, j.V, j.bs, j.H, j.hld, j.W, (w % nrb) * 256 + threadIdx.x,
                   (int)(w / nrb));
  });
}

template <typename T>
__global__ __launch_bounds__(256) void k_normalize_grouped(DevTab<NormJob<T>> t) {
  for_wg_items(t, 0, [&](const NormJob<T>& j, int64_t w) {
    const int64_t nrb = (j.N + 255) / 256;
    normalize_row<T>(j.N, j.nrm2, j.W, j.Vout, j.hout, j.hld, (w % nrb) * 256 + threadIdx.x,
                     (int)(w / nrb));
  });
}

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_convert_grouped(DevTab<ConvJob<TI, TO>> t) {
  for_wg_items(t, 0, [&](const ConvJob<TI, TO>& j, int64_t w) {
    const int64_t nrb = (j.N + 255) / 256;
    const int64_t r = (w % nrb) * 256 + threadIdx.x;
    const int col = (int)(w / nrb);
    if (r < j.N)
      j.Y[r + (int64_t)col * j.ldy] =
          j.X ? (TO)(j.alpha * (double)j.X[r + (int64_t)col * j.ldx]) : (TO)0;
  });
}

template <typename T>
hipError_t launch_bupdate_grouped(DevTab<BupdJob<T>> t, hipStream_t s) {
  hipLaunchKernelGGL((k_bupdate_grouped<T>), dim3(kPersistWGs), dim3(256), 0, s, t);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_normalize_grouped(DevTab<NormJob<T>> t, hipStream_t s) {
  hipLaunchKernelGGL((k_normalize_grouped<T>), dim3(kPersistWGs), dim3(256), 0, s, t);
  return hipGetLastError();
}
template <typename TI, typename TO>
hipError_t launch_convert_grouped(DevTab<ConvJob<TI, TO>> t, hipStream_t s) {
  hipLaunchKernelGGL((k_convert_grouped<TI, TO>), dim3(kPersistWGs), dim3(256), 0, s, t);
  return hipGetLastError();
}
template hipError_t launch_bupdate_grouped<double>(DevTab<BupdJob<double>>, hipStream_t);
template hipError_t launch_bupdate_grouped<float>(DevTab<BupdJob<float>>, hipStream_t);
template hipError_t launch_normalize_grouped<double>(DevTab<NormJob<double>>, hipStream_t);
template hipError_t launch_normalize_grouped<float>(DevTab<NormJob<float>>, hipStream_t);
template hipError_t launch_convert_grouped<double, double>(DevTab<ConvJob<double, double>>,
                                                           hipStream_t);
template hipError_t launch_convert_grouped<double, float>(DevTab<ConvJob<double, float>>,
                                                          hipStream_t);
template hipError_t launch_convert_grouped<float, double>(DevTab<ConvJob<float, double>>,
                                                          hipStream_t);
template hipError_t launch_convert_grouped<float, float>(DevTab<ConvJob<float, float>>,
                                                         hipStream_t);

// ------------------------------------------------------ Cholesky-QR pieces
__global__ __launch_bounds__(256) void k_chol_grouped(DevTab<CholJob> t) {
  for_wg_items(t, 0, [&](const CholJob& j, int64_t) {
    if (threadIdx.x == 0) chol_small_serial(j.nx, j.G, j.n0, j.drop_tol, j.R, j.flags);
  });
}

__global__ __launch_bounds__(256) void k_trsm_grouped(DevTab<TrsmJob> t) {
  __shared__ TrsmSmem sm;
  for_wg_items(t, 0, [&](const TrsmJob& j, int64_t w) { trsm_block(j.N, j.nx, j.R, j.X, j.ldx, w, sm); });
}

hipError_t launch_chol_grouped(DevTab<CholJob> t, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_grouped, dim3(kPersistWGs / 8), dim3(256), 0, s, t);
  return hipGetLastError();
}
hipError_t launch_trsm_grouped(DevTab<TrsmJob> t, hipStream_t s) {
  hipLaunchKernelGGL(k_trsm_grouped, dim3(kPersistWGs), dim3(256), 0, s, t);
  return hipGetLastError();
}

// ------------------------------------------------------------ table arena
TableArena::~TableArena() {
  if (host_) (void)hipHostFree(host_);
  if (dev_) (void)hipFree(dev_);
}

hipError_t TableArena::init(size_t bytes) {
  hipError_t e = hipHostMalloc((void**)&host_, bytes, hipHostMallocDefault);
  if (e != hipSuccess) return e;
  e = hipMalloc((void**)&dev_, bytes);
  if (e != hipSuccess) return e;
  cap_ = bytes;
  used_ = 0;
  return hipSuccess;
}

hipError_t TableArena::upload(hipStream_t s) {
  if (used_ == uploaded_) return hipSuccess;
  hipError_t e = hipMemcpyAsync(dev_ + uploaded_, host_ + uploaded_, used_ - uploaded_,
                                hipMemcpyHostToDevice, s);
  uploaded_ = used_;
  return e;
}

}  // namespace tp3b
