// Device kernels for gfx950 (CDNA4, 64-wide wavefronts, 4 SIMDs per CU, MFMA).
//
// Mode products (Sec. 3.2-3.3 of the paper: the Hamiltonian applied as one
// dense n x n matrix product per tensor mode plus a pointwise potential) run on
// the matrix cores: FP64 through v_mfma_f64_16x16x4 and FP32 through
// v_mfma_f32_16x16x4, operand panels staged through LDS, FP64 accumulation for
// FP64 and FP32 for FP32.  The potential term, the eigenvalue-shift term and
// the preconditioner's pointwise divide are fused into the store epilogue.
//
// The tall-skinny products of the eigensolver (block dots, basis updates) are
// bandwidth-bound; the dot kernel still uses the FP64 matrix cores so that the
// arithmetic never limits it, and all reductions are two-stage and
// deterministic (no atomics).
#include "kernels.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_bodies.h"

namespace tp3b {

// ------------------------------------------------------------------ mode product
LaunchTiming*& launch_timing() {
  static thread_local LaunchTiming* t = nullptr;
  return t;
}

// Launch with the timing events of launch_timing() when it is set.
#define TP3B_MP_LAUNCH(KERN, GRID, BLOCK, S, ARG)                                                 \
  do {                                                                                     \
    LaunchTiming* lt_ = launch_timing();                                                   \
    if (lt_) {                                                                             \
      hipEvent_t st_ = lt_->started ? nullptr : lt_->start;                                \
      lt_->started = true;                                                                 \
      hipExtLaunchKernelGGL(KERN, dim3(GRID), dim3(BLOCK), 0, S, st_, lt_->stop, 0, ARG);  \
    } else {                                                                               \
      hipLaunchKernelGGL(KERN, dim3(GRID), dim3(BLOCK), 0, S, ARG);                        \
    }                                                                                      \
  } while (0)

// ROLE only separates the kernel names seen by profilers: 0 = Hamiltonian apply
// (both modes + potential), 1 = preconditioner mode products, 2 = 2D x-mode
// accumulation passes.
// At least two waves per SIMD: with one (the register demand of the FP64
// 128 x 128 tile left to itself) every barrier and fetch of the K loop is
// exposed; measured on c3, the best FP64 tile goes from 1.42 to 1.23 ms.
template <typename T, int TM, int TN, int KC, int ROLE, bool SK = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_modeprod(ModeProd<T> a) {
  __shared__ MpSmem<T, TM, TN, KC, SK> sm;
  modeprod_tile<T, TM, TN, KC, SK>(a, xcd_remap(blockIdx.x, modeprod_items<TM, TN>(a)), sm);
}

// Small grids: 32 x 32 output tile split over the K of eight waves (512
// threads, K-chunks of 64), four waves per SIMD.
template <typename T, int ROLE>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_modeprod_sk8(
    ModeProd<T> a) {
  __shared__ MpSmem<T, 32, 32, 64, true, 8> sm;
  modeprod_tile<T, 32, 32, 64, true, 8>(a, xcd_remap(blockIdx.x, modeprod_items<32, 32>(a)), sm);
}

template <typename T, int ROLE>
static void launch_role(const ModeProd<T>& a, int tile, hipStream_t s, unsigned g32, unsigned g64,
                        unsigned g128, unsigned g64x128) {
  switch (tile) {
    case TILE_32:
      TP3B_MP_LAUNCH((k_modeprod<T, 32, 32, 64, ROLE, true>), g32, 256, s, a);
      break;
    case TILE_32W8:
      TP3B_MP_LAUNCH((k_modeprod_sk8<T, ROLE>), g32, 512, s, a);
      break;
    case TILE_64:
      TP3B_MP_LAUNCH((k_modeprod<T, 64, 64, 16, ROLE>), g64, 256, s, a);
      break;
    case TILE_128:
      TP3B_MP_LAUNCH((k_modeprod<T, 128, 128, 16, ROLE>), g128, 256, s, a);
      break;
    default:
      TP3B_MP_LAUNCH((k_modeprod<T, 64, 128, 16, ROLE>), g64x128, 256, s, a);
      break;
  }
}

template <typename T>
hipError_t launch_modeprod(const ModeProd<T>& a, int tile, hipStream_t s) {
  if (a.M <= 0 || a.Nc <= 0 || a.nbatch <= 0) return hipSuccess;
  if (tile < 0 || tile >= NUM_TILE_CFGS) return hipErrorInvalidValue;
  auto grid = [&](int TM, int TN) {
    int64_t tiles = (int64_t)((a.M + TM - 1) / TM) * ((a.Nc + TN - 1) / TN);
    return (unsigned)(tiles * a.nbatch);
  };
  const unsigned g32 = grid(32, 32), g64 = grid(64, 64), g128 = grid(128, 128), g6412 = grid(64, 128);
  if (a.L && a.R && a.epi == EPI_V)
    launch_role<T, 0>(a, tile, s, g32, g64, g128, g6412);
  else if (a.acc)
    launch_role<T, 2>(a, tile, s, g32, g64, g128, g6412);
  else
    launch_role<T, 1>(a, tile, s, g32, g64, g128, g6412);
  return hipGetLastError();
}

template hipError_t launch_modeprod<double>(const ModeProd<double>&, int, hipStream_t);
template hipError_t launch_modeprod<float>(const ModeProd<float>&, int, hipStream_t);

// ------------------------------------------------------ BF16x3 mode product
template <int TM, int TN, int KC, int ROLE>
__global__ __launch_bounds__(256) void k_modeprod_bf3(ModeProd<float> a) {
  __shared__ Bf3Smem<TM, TN, KC> sm;
  modeprod_bf3_tile<TM, TN, KC>(a, xcd_remap(blockIdx.x, modeprod_items<TM, TN>(a)), sm);
}

template <int ROLE>
static void launch_role_bf3(const ModeProd<float>& a, int tile, hipStream_t s, unsigned g64,
                            unsigned g128, unsigned g64x128) {
  switch (tile) {
    case TILE_128:
      TP3B_MP_LAUNCH((k_modeprod_bf3<128, 128, 32, ROLE>), g128, 256, s, a);
      break;
    case TILE_64x128:
      TP3B_MP_LAUNCH((k_modeprod_bf3<64, 128, 32, ROLE>), g64x128, 256, s, a);
      break;
    default:  // TILE_32, TILE_32W8 and TILE_64: the smallest bf16 tile is 64 x 64
      TP3B_MP_LAUNCH((k_modeprod_bf3<64, 64, 32, ROLE>), g64, 256, s, a);
      break;
  }
}

// hi / lo of each element with the expressions of split8 (device_bodies.h), so
// the staged values are the same whichever side splits them
__global__ __launch_bounds__(256) void k_bf3_split(int n, const float* __restrict__ A, int transpose,
                                                   unsigned short* __restrict__ out) {
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nn; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / n, k = e - i * n;
    const float f = transpose ? A[k * n + i] : A[i * n + k];
    const __bf16 h = (__bf16)f;
    const __bf16 l = (__bf16)(f - (float)h);
    out[e] = __builtin_bit_cast(unsigned short, h);
    out[nn + e] = __builtin_bit_cast(unsigned short, l);
  }
}

hipError_t launch_bf3_split(int n, const float* A, int transpose, unsigned short* out, hipStream_t s) {
  if (n <= 0 || !A || !out) return hipErrorInvalidValue;
  const int64_t nn = (int64_t)n * n;
  const unsigned g = (unsigned)std::min<int64_t>((nn + 255) / 256, 4096);
  hipLaunchKernelGGL(k_bf3_split, dim3(g), dim3(256), 0, s, n, A, transpose, out);
  return hipGetLastError();
}

hipError_t launch_modeprod_bf3(const ModeProd<float>& a, int tile, hipStream_t s) {
  if (a.M <= 0 || a.Nc <= 0 || a.nbatch <= 0) return hipSuccess;
  if (tile < 0 || tile >= NUM_TILE_CFGS) return hipErrorInvalidValue;
  auto grid = [&](int TM, int TN) {
    int64_t tiles = (int64_t)((a.M + TM - 1) / TM) * ((a.Nc + TN - 1) / TN);
    return (unsigned)(tiles * a.nbatch);
  };
  const unsigned g64 = grid(64, 64), g128 = grid(128, 128), g6412 = grid(64, 128);
  if (a.L && a.R && a.epi == EPI_V)
    launch_role_bf3<0>(a, tile, s, g64, g128, g6412);
  else if (a.acc)
    launch_role_bf3<2>(a, tile, s, g64, g128, g6412);
  else
    launch_role_bf3<1>(a, tile, s, g64, g128, g6412);
  return hipGetLastError();
}

// ---------------------------------------------------------------- block dot
int64_t dot_scratch_doubles(int64_t N, int p, int q) {
  int64_t nchunk = (N + dot_row_chunk(N) - 1) / dot_row_chunk(N);
  int64_t ntile = (int64_t)((p + DOT_TP - 1) / DOT_TP) * ((q + DOT_TQ - 1) / DOT_TQ);
  return nchunk * ntile * DOT_TP * DOT_TQ;
}

template <typename TA, typename TB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_dot_tn(int64_t N, int p, int q, const TA* __restrict__ A,
                                                int64_t lda, const TB* __restrict__ B, int64_t ldb,
                                                int rchunk, int tiles_q, double* __restrict__ part) {
  __shared__ DotSmem sm;
  const int chunk = blockIdx.x, tile = blockIdx.y;
  dot_tile<TA, TB>(N, p, q, A, lda, B, ldb, rchunk, tiles_q, chunk, tile,
                   part + ((int64_t)tile * gridDim.x + chunk) * (DOT_TP * DOT_TQ), sm);
}

// One wavefront per output element (fixed summation order: deterministic).
__global__ __launch_bounds__(256) void k_dot_reduce(int p, int q, int nchunk, int tiles_q,
                                                    const double* __restrict__ part,
                                                    double* __restrict__ C, int ldc) {
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);  // element within the tile
  const int tile = blockIdx.y;
  if (e >= DOT_TP * DOT_TQ) return;
  const int gp = (tile / tiles_q) * DOT_TP + e % DOT_TP;
  const int gq = (tile % tiles_q) * DOT_TQ + e / DOT_TP;
  if (gp >= p || gq >= q) return;
  const double s = dot_reduce_elem(gp, gq, nchunk, tiles_q, part, lane);
  if (lane == 0) C[gp + (int64_t)gq * ldc] = s;
}

// Long blocks (N >= DOTL_N) whose whole product fits one tile of PI x QJ
// MFMA blocks (p <= 16 PI <= 80, q <= 16 QJ <= 32).  The work is the block
// dot's: the same row chunks, the same 16-row groups per wave taken in the
// same order, the waves summed in LDS in wave order, the chunks summed by one
// wavefront per element.  What differs is that the block counts are compile-time,
// so no load or product sits behind a branch: lanes past the last column load
// column 0 of their operand (their pointers are clamped there) and feed only
// output rows or columns outside p x q, which are never stored.  With
// straight-line loads the next batch stays in flight while the current one is
// multiplied; S groups per batch keep enough bytes in flight when the tile
// is narrow.
constexpr int64_t DOTL_N = 1 << 20;
constexpr int DOTL_PI = 5, DOTL_QJ = 2;

template <typename TA, typename TB, int PI, int QJ, int S>
__global__ __launch_bounds__(256) void k_dot_long(int64_t N, int p, int q, const TA* __restrict__ A,
                                                  int64_t lda, const TB* __restrict__ B,
                                                  int64_t ldb, int rc, double* __restrict__ part) {
  constexpr int TP = 16 * PI, TQ = 16 * QJ;
  __shared__ double red[TP * TQ];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t rbeg = (int64_t)blockIdx.x * rc;
  const int64_t rend = (rbeg + rc < N) ? rbeg + rc : N;
  const TA* Ac[PI];
  const TB* Bc[QJ];
  bool pa[PI], pb[QJ];
#pragma unroll
  for (int i = 0; i < PI; ++i) {
    const int col = i * 16 + lr;
    pa[i] = col < p;
    Ac[i] = A + (int64_t)(pa[i] ? col : 0) * lda;
  }
#pragma unroll
  for (int j = 0; j < QJ; ++j) {
    const int col = j * 16 + lr;
    pb[j] = col < q;
    Bc[j] = B + (int64_t)(pb[j] ? col : 0) * ldb;
  }
  d4 acc[PI][QJ];
#pragma unroll
  for (int i = 0; i < PI; ++i)
#pragma unroll
    for (int j = 0; j < QJ; ++j) acc[i][j] = d4{0, 0, 0, 0};
  const bool vec_ok = (((uintptr_t)A | (uintptr_t)B) % 16 == 0) && (lda % 4 == 0) &&
                      (ldb % 4 == 0) && (rbeg % 16 == 0);
  // batch of S groups of 16 rows: group s at rows g + 64 s (lane group lk owns
  // rows + 4 lk .. + 3 of its column, fed to K slot lk of the u-th product)
  auto loadv = [&](int64_t g, double (&av)[S][PI][4], double (&bv)[S][QJ][4]) {
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int64_t r0 = g + 64 * t + 4 * lk;
#pragma unroll
      for (int i = 0; i < PI; ++i) ld4_d(Ac[i] + r0, av[t][i]);
#pragma unroll
      for (int j = 0; j < QJ; ++j) ld4_d(Bc[j] + r0, bv[t][j]);
    }
  };
  auto mul = [&](const double (&av)[S][PI][4], const double (&bv)[S][QJ][4], int nt) {
#pragma unroll
    for (int t = 0; t < S; ++t)
      if (t < nt)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int i = 0; i < PI; ++i)
#pragma unroll
            for (int j = 0; j < QJ; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t][i][u], bv[t][j][u], acc[i][j],
                                                               0, 0, 0);
  };
  double a0[S][PI][4], b0[S][QJ][4], a1[S][PI][4], b1[S][QJ][4];
  int64_t g = rbeg + wave * 16;
  constexpr int64_t STEP = 64 * S;
  // Whole batches (every group of the batch inside the chunk), two in
  // flight, in pairs: each pass of the loop loads the second batch of its pair
  // and then the first of the next pair (the last batch again past the end,
  // its values unused), so no load sits behind a branch, the number of loads
  // in flight is the same on every path and each wait covers only the batch
  // in use.  An odd last batch is already loaded when the loop ends.
  if (vec_ok && g + STEP - 48 <= rend) {
    const int64_t nbat = (rend - g + 48) / STEP;
    const int64_t glast = g + (nbat - 1) * STEP;
    loadv(g, a0, b0);
    for (int64_t k = 0; k < nbat / 2; ++k) {
      loadv(g + STEP, a1, b1);
      mul(a0, b0, S);
      g += STEP;
      loadv(g + STEP < glast ? g + STEP : glast, a0, b0);
      mul(a1, b1, S);
      g += STEP;
    }
    if (nbat & 1) {
      mul(a0, b0, S);
      g += STEP;
    }
  }
  // the remaining groups (a partial batch, the group that crosses the chunk
  // end, or unaligned operands): element loads, zero past the last row
  for (; g < rend; g += 64) {
    const int64_t r0 = g + 4 * lk;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t r = r0 + u;
      const bool rv = r < rend;
#pragma unroll
      for (int i = 0; i < PI; ++i) a0[0][i][u] = rv ? ld_d(Ac[i] + r) : 0.0;
#pragma unroll
      for (int j = 0; j < QJ; ++j) b0[0][j][u] = rv ? ld_d(Bc[j] + r) : 0.0;
    }
    mul(a0, b0, 1);
  }
  for (int wv = 0; wv < 4; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int i = 0; i < PI; ++i)
#pragma unroll
        for (int j = 0; j < QJ; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int idx = (j * 16 + lr) * TP + i * 16 + Mma<double>::row(lk, r);
            red[idx] = (wv == 0) ? acc[i][j][r] : red[idx] + acc[i][j][r];
          }
    }
    __syncthreads();
  }
  double* out = part + (int64_t)blockIdx.x * (TP * TQ);
  for (int e = tid; e < TP * TQ; e += 256)
    if (e % TP < p && e / TP < q) out[e] = red[e];
}

// The same product for wider tiles (40 or more columns), staged through LDS.  Loads
// in the MFMA operand layout put 16 columns into every load instruction,
// which for many long columns (their starts a large power of two apart)
// keeps the memory system well below its streaming rate; here each thread
// instead loads two consecutive rows of one column, so a wave's instruction
// reads 256 contiguous bytes of each of four columns, and the products take
// their operands from LDS.  A workgroup takes the 32-row steps b, b + G,
// b + 2G, ... (G workgroups), the next step's loads in flight while the
// current one is multiplied; two waves multiply (16 rows each), the four
// waves' tiles are summed in LDS in wave order as in the block dot.  Padding
// columns load column 0 of their operand (their LDS entries feed only
// outputs outside p x q, which are not stored).  Requires aligned pairs of
// rows: even leading dimensions and base pointers aligned to two elements.
constexpr int DOTS_RS = 32;

template <typename T, int PI, int QJ>
__global__ __launch_bounds__(256) void k_dot_lds(int64_t N, int p, int q, const T* __restrict__ A,
                                                 int64_t lda, const T* __restrict__ B, int64_t ldb,
                                                 double* __restrict__ part) {
  constexpr int RS = DOTS_RS;
  constexpr int TP = 16 * PI, TQ = 16 * QJ, NC = TP + TQ;
  // row stride of the staged tile: NC + 4 doubles puts the two lane groups
  // of a half-wave operand read on disjoint bank halves
  constexpr int LDW = NC + 4;
  constexpr int SEG = RS / 2;        // threads per column (two rows each)
  constexpr int CPR = 256 / SEG;     // columns per load round
  constexpr int NR = NC / CPR;       // load rounds (NC is a multiple of 16)
  typedef typename std::conditional<std::is_same<T, double>::value, double2, float2>::type T2;
  __shared__ double sm[RS * LDW];
  __shared__ double red[TP * TQ];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int rp = 2 * (tid % SEG);  // first of this thread's two rows in a step
  // every slot loads (a padding column reads column 0 of its operand), so no
  // load sits behind a per-lane branch
  const T* src[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const int c = k * CPR + tid / SEG;
    const bool val = c < TP ? c < p : c - TP < q;
    const int cc = val ? (c < TP ? c : c - TP) : 0;
    src[k] = (c < TP ? A + (int64_t)cc * lda : B + (int64_t)cc * ldb) + rp;
  }
  const int scol = tid / SEG;  // this thread's column in round 0
  d4 acc[PI][QJ];
#pragma unroll
  for (int i = 0; i < PI; ++i)
#pragma unroll
    for (int j = 0; j < QJ; ++j) acc[i][j] = d4{0, 0, 0, 0};
  T2 v[NR];
  auto stage = [&]() {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      sm[rp * LDW + k * CPR + scol] = (double)v[k].x;
      sm[(rp + 1) * LDW + k * CPR + scol] = (double)v[k].y;
    }
  };
  auto mul = [&]() {
    if (wave < RS / 16) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = wave * 16 + 4 * lk + u;
        double a[PI], bb[QJ];
#pragma unroll
        for (int i = 0; i < PI; ++i) a[i] = sm[r * LDW + i * 16 + lr];
#pragma unroll
        for (int j = 0; j < QJ; ++j) bb[j] = sm[r * LDW + TP + j * 16 + lr];
#pragma unroll
        for (int i = 0; i < PI; ++i)
#pragma unroll
          for (int j = 0; j < QJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
      }
    }
  };
  // whole steps: workgroup b takes b, b + G, ...; the next step's loads are
  // issued before the current step is multiplied
  const int64_t nfull = N / RS, G = gridDim.x;
  int64_t st = blockIdx.x;
  if (st < nfull) {
#pragma unroll
    for (int k = 0; k < NR; ++k) v[k] = *(const T2*)(src[k] + st * RS);
  }
  for (; st < nfull; st += G) {
    __syncthreads();
    stage();
    __syncthreads();
    if (st + G < nfull) {
      const int64_t r0 = (st + G) * RS;
#pragma unroll
      for (int k = 0; k < NR; ++k) v[k] = *(const T2*)(src[k] + r0);
    }
    mul();
  }
  // the last, partial step (if any), on the workgroup next in turn: element
  // loads, zero past the last row
  if (nfull * RS < N && blockIdx.x == nfull % G) {
    const int64_t r0 = nfull * RS;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      v[k].x = (r0 + rp < N) ? src[k][r0] : (T)0;
      v[k].y = (r0 + rp + 1 < N) ? src[k][r0 + 1] : (T)0;
    }
    __syncthreads();
    stage();
    __syncthreads();
    mul();
  }
  for (int wv = 0; wv < 4; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int i = 0; i < PI; ++i)
#pragma unroll
        for (int j = 0; j < QJ; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int idx = (j * 16 + lr) * TP + i * 16 + Mma<double>::row(lk, r);
            red[idx] = (wv == 0) ? acc[i][j][r] : red[idx] + acc[i][j][r];
          }
    }
    __syncthreads();
  }
  double* out = part + (int64_t)blockIdx.x * (TP * TQ);
  for (int e = tid; e < TP * TQ; e += 256)
    if (e % TP < p && e / TP < q) out[e] = red[e];
}

// Sums the chunk partials of k_dot_long: one wavefront per element (p, q),
// lanes stride over the chunks, then a fixed-order shuffle reduction.  Stores
// C[i + j ldc] = sum, or C[j + i ldc] with `trans`.
__global__ __launch_bounds__(256) void k_dot_long_reduce(int p, int q, int tp, int nchunk,
                                                         const double* __restrict__ part,
                                                         double* __restrict__ C, int ldc,
                                                         int trans) {
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= p * q) return;
  const int i = e % p, j = e / p;
  const double* src = part + (int64_t)j * tp + i;
  const int64_t cs = (int64_t)tp * ((q + 15) / 16) * 16;
  double s = 0.0;
  for (int c = lane; c < nchunk; c += 64) s += src[(int64_t)c * cs];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) {
    if (trans)
      C[j + (int64_t)i * ldc] = s;
    else
      C[i + (int64_t)j * ldc] = s;
  }
}

template <typename TA, typename TB, int PI, int QJ>
static int launch_dot_long_pq(int64_t N, int p, int q, const TA* A, int64_t lda, const TB* B,
                              int64_t ldb, int rc, int nchunk, int64_t cap, double* partial,
                              hipStream_t s) {
  constexpr int TPQ = 256 * PI * QJ;
  if constexpr (PI + QJ >= 3 && std::is_same<TA, TB>::value) {
    // staged through LDS once at least 40 columns are read (measured: from
    // there on the direct loads fall well below the staged ones)
    const bool al = (p + q >= 40) && (((uintptr_t)A | (uintptr_t)B) % (2 * sizeof(TA)) == 0) &&
                    (lda % 2 == 0) && (ldb % 2 == 0);
    int64_t G = cap / TPQ;
    if (G > 2048) G = 2048;
    if (al && G >= 256) {
      hipLaunchKernelGGL((k_dot_lds<TA, PI, QJ>), dim3((unsigned)G), dim3(256), 0, s, N, p, q, A,
                         lda, B, ldb, partial);
      return (int)G;
    }
  }
  if ((int64_t)nchunk * TPQ > cap) return -1;
  constexpr int S = (PI + QJ <= 2) ? 3 : ((PI + QJ <= 3) ? 2 : 1);
  hipLaunchKernelGGL((k_dot_long<TA, TB, PI, QJ, S>), dim3(nchunk), dim3(256), 0, s, N, p, q, A,
                     lda, B, ldb, rc, partial);
  return nchunk;
}

template <typename TA, typename TB, int QJ>
static int launch_dot_long_q(int pi, int64_t N, int p, int q, const TA* A, int64_t lda,
                             const TB* B, int64_t ldb, int rc, int nchunk, int64_t cap,
                             double* partial, hipStream_t s) {
  switch (pi) {
    case 1: return launch_dot_long_pq<TA, TB, 1, QJ>(N, p, q, A, lda, B, ldb, rc, nchunk, cap, partial, s);
    case 2: return launch_dot_long_pq<TA, TB, 2, QJ>(N, p, q, A, lda, B, ldb, rc, nchunk, cap, partial, s);
    case 3: return launch_dot_long_pq<TA, TB, 3, QJ>(N, p, q, A, lda, B, ldb, rc, nchunk, cap, partial, s);
    case 4: return launch_dot_long_pq<TA, TB, 4, QJ>(N, p, q, A, lda, B, ldb, rc, nchunk, cap, partial, s);
    default: return launch_dot_long_pq<TA, TB, 5, QJ>(N, p, q, A, lda, B, ldb, rc, nchunk, cap, partial, s);
  }
}

// C = A^T B on long blocks when one tile holds it (the taller operand is put
// first: p x q with q <= 32 and p <= 80, or the transpose).  Returns false
// when the shape does not fit; the caller then runs the general dot.
template <typename TA, typename TB>
static bool launch_dot_long(int64_t N, int p, int q, const TA* A, int64_t lda, const TB* B,
                            int64_t ldb, double* C, int ldc, double* partial, hipStream_t s) {
  if (N < DOTL_N) return false;
  const bool trans = q > p;
  const int P = trans ? q : p, Q = trans ? p : q;
  if (P > 16 * DOTL_PI || Q > 16 * DOTL_QJ) return false;
  if (trans && !std::is_same<TA, TB>::value) return false;
  const int rc = dot_row_chunk(N);
  const int nchunk = (int)((N + rc - 1) / rc);
  const int pi = (P + 15) / 16, qj = (Q + 15) / 16;
  // the partials may take what the general dot's take for this p x q
  const int64_t cap = dot_scratch_doubles(N, p, q);
  int nparts;
  if (trans) {
    // TA == TB here
    const TA* Bt = reinterpret_cast<const TA*>(B);
    const TB* At = reinterpret_cast<const TB*>(A);
    nparts = qj == 1 ? launch_dot_long_q<TA, TB, 1>(pi, N, P, Q, Bt, ldb, At, lda, rc, nchunk, cap, partial, s)
                     : launch_dot_long_q<TA, TB, 2>(pi, N, P, Q, Bt, ldb, At, lda, rc, nchunk, cap, partial, s);
  } else {
    nparts = qj == 1 ? launch_dot_long_q<TA, TB, 1>(pi, N, P, Q, A, lda, B, ldb, rc, nchunk, cap, partial, s)
                     : launch_dot_long_q<TA, TB, 2>(pi, N, P, Q, A, lda, B, ldb, rc, nchunk, cap, partial, s);
  }
  if (nparts < 0) return false;
  hipLaunchKernelGGL(k_dot_long_reduce, dim3((unsigned)((P * Q + 3) / 4)), dim3(256), 0, s, P, Q,
                     16 * pi, nparts, partial, C, ldc, trans ? 1 : 0);
  return true;
}

// A Gram-Schmidt update fused with the dot that follows it (long blocks,
// FP64): per row, Xout = Xin - Q C (nq x nx, nx <= 16, Q C on the matrix
// cores), then the partials of the next dot on the updated rows, Q^T Xout
// (SELF false: the second Gram-Schmidt pass; the same steps, workgroups and
// product order as k_dot_lds, so it equals launch_dot_tn on the stored Xout)
// or Xout^T Xout (SELF true: the Gram matrix of the Cholesky-QR).  Rows are
// staged through LDS in 32-row steps as in k_dot_lds.  Xin may equal Xout
// (each row is read before it is written, by the same workgroup).
template <int PQ, int QJ, bool SELF>
__global__ __launch_bounds__(256) void k_gemm_dot_lds(int64_t N, int nq, int nx,
                                                      const double* __restrict__ Q, int64_t ldq,
                                                      const double* __restrict__ C,
                                                      const double* Xin, double* Xout,
                                                      int64_t ldx, double* __restrict__ part) {
  constexpr int RS = DOTS_RS;
  constexpr int TP = 16 * PQ, TQ = 16 * QJ, NC = TP + TQ;
  constexpr int LDW = NC + 4;
  constexpr int SEG = RS / 2, CPR = 256 / SEG, NR = NC / CPR;
  constexpr int DP = SELF ? QJ : PQ;   // 16-column blocks of the dot's first operand
  constexpr int TD = 16 * DP;
  constexpr int AOFF = SELF ? TP : 0;  // where that operand sits in the staged rows
  static_assert(QJ == 1, "the update forms 16 columns per wave");
  __shared__ double sm[RS * LDW];
  __shared__ double red[TD * TQ];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int rp = 2 * (tid % SEG);
  const double* src[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const int c = k * CPR + tid / SEG;
    const bool val = c < TP ? c < nq : c - TP < nx;
    const int cc = val ? (c < TP ? c : c - TP) : 0;
    src[k] = (c < TP ? Q + (int64_t)cc * ldq : Xin + (int64_t)cc * ldx) + rp;
  }
  const int scol = tid / SEG;
  d4 acc[DP][QJ];
#pragma unroll
  for (int i = 0; i < DP; ++i)
#pragma unroll
    for (int j = 0; j < QJ; ++j) acc[i][j] = d4{0, 0, 0, 0};
  double2 v[NR];
  auto stage = [&]() {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      sm[rp * LDW + k * CPR + scol] = v[k].x;
      sm[(rp + 1) * LDW + k * CPR + scol] = v[k].y;
    }
  };
  // The update of the staged rows on the matrix cores: waves 0 and 1 form
  // D = Q C for rows 16w .. 16w + 15 (A operand from the staged Q rows, the
  // B operand C[4kk + lk][lr] held in registers) and replace the staged X by
  // X - D; then every thread copies its share of the updated rows to Xout
  // (32 consecutive rows of a column per half-wave).
  double creg[4 * PQ];
#pragma unroll
  for (int kk = 0; kk < 4 * PQ; ++kk) {
    const int i = 4 * kk + lk;
    creg[kk] = (i < nq && lr < nx) ? C[i + (int64_t)lr * nq] : 0.0;
  }
  auto update = [&]() {
    if (wave < RS / 16) {
      d4 dq = d4{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4 * PQ; ++kk)
        dq = __builtin_amdgcn_mfma_f64_16x16x4f64(sm[(wave * 16 + lr) * LDW + 4 * kk + lk], creg[kk],
                                                  dq, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wave * 16 + Mma<double>::row(lk, r);
        sm[row * LDW + TP + lr] -= dq[r];
      }
    }
  };
  auto copy_out = [&](int64_t r0) {
    const int rr = tid & 31;
    if (r0 + rr < N) {
#pragma unroll
      for (int t = 0; t < TQ / 8; ++t) {
        const int j = (tid >> 5) + 8 * t;
        if (j < nx) Xout[r0 + rr + (int64_t)j * ldx] = sm[rr * LDW + TP + j];
      }
    }
  };
  auto mul = [&]() {
    if (wave < RS / 16) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = wave * 16 + 4 * lk + u;
        double a[DP], bb[QJ];
#pragma unroll
        for (int i = 0; i < DP; ++i) a[i] = sm[r * LDW + AOFF + i * 16 + lr];
#pragma unroll
        for (int j = 0; j < QJ; ++j) bb[j] = sm[r * LDW + TP + j * 16 + lr];
#pragma unroll
        for (int i = 0; i < DP; ++i)
#pragma unroll
          for (int j = 0; j < QJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
      }
    }
  };
  const int64_t nfull = N / RS, G = gridDim.x;
  int64_t st = blockIdx.x;
  if (st < nfull) {
#pragma unroll
    for (int k = 0; k < NR; ++k) v[k] = *(const double2*)(src[k] + st * RS);
  }
  for (; st < nfull; st += G) {
    __syncthreads();
    stage();
    __syncthreads();
    if (st + G < nfull) {
      const int64_t r1 = (st + G) * RS;
#pragma unroll
      for (int k = 0; k < NR; ++k) v[k] = *(const double2*)(src[k] + r1);
    }
    update();
    __syncthreads();
    copy_out(st * RS);
    mul();
  }
  if (nfull * RS < N && blockIdx.x == nfull % G) {
    // the last, partial step: zero past the last row (the update then
    // stores only the rows inside)
    const int64_t r0 = nfull * RS;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      v[k].x = (r0 + rp < N) ? src[k][r0] : 0.0;
      v[k].y = (r0 + rp + 1 < N) ? src[k][r0 + 1] : 0.0;
    }
    __syncthreads();
    stage();
    __syncthreads();
    update();
    __syncthreads();
    copy_out(r0);
    mul();
  }
  for (int wv = 0; wv < 4; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int i = 0; i < DP; ++i)
#pragma unroll
        for (int j = 0; j < QJ; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int idx = (j * 16 + lr) * TD + i * 16 + Mma<double>::row(lk, r);
            red[idx] = (wv == 0) ? acc[i][j][r] : red[idx] + acc[i][j][r];
          }
    }
    __syncthreads();
  }
  const int pd = SELF ? nx : nq;
  double* out = part + (int64_t)blockIdx.x * (TD * TQ);
  for (int e = tid; e < TD * TQ; e += 256)
    if (e % TD < pd && e / TD < nx) out[e] = red[e];
}

template <int PQ, bool SELF>
static void launch_gemm_dot_pq(unsigned G, int64_t N, int nq, int nx, const double* Q, int64_t ldq,
                               const double* C, const double* Xin, double* Xout, int64_t ldx,
                               double* part, hipStream_t s) {
  hipLaunchKernelGGL((k_gemm_dot_lds<PQ, 1, SELF>), dim3(G), dim3(256), 0, s, N, nq, nx, Q, ldq, C,
                     Xin, Xout, ldx, part);
}

bool gemm_dot_long_fits(int64_t N, int nq, int nx, const double* Q, int64_t ldq, const double* Xin,
                        const double* Xout, int64_t ldx) {
  return N >= DOTL_N && nq >= 1 && nq <= 16 * DOTL_PI && nx >= 1 && nx <= 16 &&
         (((uintptr_t)Q | (uintptr_t)Xin | (uintptr_t)Xout) % 16) == 0 && ldq % 2 == 0 &&
         ldx % 2 == 0 && dot_scratch_doubles(N, nx, nx) / 256 >= 256;
}

hipError_t launch_gemm_dot_long(int64_t N, int nq, int nx, const double* Q, int64_t ldq,
                                const double* C, const double* Xin, double* Xout, int64_t ldx,
                                int self, double* D, int ldd, double* partial, hipStream_t s) {
  if (!gemm_dot_long_fits(N, nq, nx, Q, ldq, Xin, Xout, ldx)) return hipErrorInvalidValue;
  const int pq = (nq + 15) / 16;
  const int pd = self ? nx : nq;
  const int td = self ? 16 : 16 * pq;
  int64_t G = dot_scratch_doubles(N, pd, nx) / (td * 16);
  if (G > 2048) G = 2048;
  if (G < 256) return hipErrorInvalidValue;
  const unsigned g = (unsigned)G;
  switch (pq) {
    case 1: self ? launch_gemm_dot_pq<1, true>(g, N, nq, nx, Q, ldq, C, Xin, Xout, ldx, partial, s)
                 : launch_gemm_dot_pq<1, false>(g, N, nq, nx, Q, ldq, C, Xin, Xout, ldx, partial, s); break;
    case 2: self ? launch_gemm_dot_pq<2, true>(g, N, nq, nx, Q, ldq, C, Xin, Xout, ldx, partial, s)
                 : launch_gemm_dot_pq<2, false>(g, N, nq, nx, Q, ldq, C, Xin, Xout, ldx, partial, s); break;
    case 3: self ? launch_gemm_dot_pq<3, true>(g, N, nq, nx, Q, ldq, C, Xin, Xout, ldx, partial, s)
                 : launch_gemm_dot_pq<3, false>(g, N, nq, nx, Q, ldq, C, Xin, Xout, ldx, partial, s); break;
    case 4: self ? launch_gemm_dot_pq<4, true>(g, N, nq, nx, Q, ldq, C, Xin, Xout, ldx, partial, s)
                 : launch_gemm_dot_pq<4, false>(g, N, nq, nx, Q, ldq, C, Xin, Xout, ldx, partial, s); break;
    default: self ? launch_gemm_dot_pq<5, true>(g, N, nq, nx, Q, ldq, C, Xin, Xout, ldx, partial, s)
                  : launch_gemm_dot_pq<5, false>(g, N, nq, nx, Q, ldq, C, Xin, Xout, ldx, partial, s); break;
  }
  hipLaunchKernelGGL(k_dot_long_reduce, dim3((unsigned)((pd * nx + 3) / 4)), dim3(256), 0, s, pd, nx,
                     td, (int)G, partial, D, ldd, 0);
  return hipGetLastError();
}

template <typename TA, typename TB>
hipError_t launch_dot_tn(int64_t N, int p, int q, const TA* A, int64_t lda, const TB* B,
                         int64_t ldb, double* C, int ldc, double* partial, hipStream_t s) {
  if (p <= 0 || q <= 0) return hipSuccess;
  if (N <= 0) {
    // empty contraction: zero result
    for (int j = 0; j < q; ++j) {
      hipError_t e = hipMemsetAsync(C + (int64_t)j * ldc, 0, sizeof(double) * p, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (launch_dot_long<TA, TB>(N, p, q, A, lda, B, ldb, C, ldc, partial, s)) return hipGetLastError();
  const int rc = dot_row_chunk(N);
  const int nchunk = (int)((N + rc - 1) / rc);
  const int tq = (q + DOT_TQ - 1) / DOT_TQ, tp = (p + DOT_TP - 1) / DOT_TP;
  hipLaunchKernelGGL((k_dot_tn<TA, TB>), dim3(nchunk, tp * tq), dim3(256), 0, s, N, p, q, A, lda, B,
                     ldb, rc, tq, partial);
  // Only the elements of the tile inside p x q are reduced; with the tile's
  // column-major element order that is the first min(q, 32) columns.
  const int qcols = q < DOT_TQ ? q : DOT_TQ;
  hipLaunchKernelGGL(k_dot_reduce, dim3((qcols * DOT_TP + 3) / 4, tp * tq), dim3(256), 0, s, p, q,
                     nchunk, tq, partial, C, ldc);
  return hipGetLastError();
}

template hipError_t launch_dot_tn<double, double>(int64_t, int, int, const double*, int64_t,
                                                  const double*, int64_t, double*, int, double*,
                                                  hipStream_t);
template hipError_t launch_dot_tn<float, float>(int64_t, int, int, const float*, int64_t,
                                                const float*, int64_t, double*, int, double*,
                                                hipStream_t);

// ------------------------------------------------------------ basis update
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_nn(int64_t N, int p, int q, double alpha,
                                                 const T* __restrict__ A, int64_t lda,
                                                 const double* __restrict__ C, int ldc,
                                                 double beta, const T* __restrict__ X0, int64_t ldx0,
                                                 T* __restrict__ Y, int64_t ldy) {
  __shared__ GemmSmem<true> sm;
  gemm_block<T, true>(N, p, q, alpha, A, lda, C, ldc, beta, Y, ldy, blockIdx.x, blockIdx.y, sm, X0,
                      ldx0);
}

// Long blocks (N >= GEMM_LONG_N rows, p <= GEMM_PB): a fixed grid of
// workgroups, each of which stages its QB columns of C in LDS once and then
// strides over the rows, one row per thread over all of p (no partial rows to
// combine, no barrier inside the loop).  Launching one workgroup per 64 rows
// instead would stage C and reduce in LDS 2^18 times for a 2D vector of 2^24
// entries.
constexpr int64_t GEMM_LONG_N = 1 << 20;
constexpr int GEMM_LONG_WG = 2048;

template <typename T, int QB>
__global__ __launch_bounds__(256) void k_gemm_nn_long(int64_t N, int p, int q, double alpha,
                                                      const T* __restrict__ A, int64_t lda,
                                                      const double* __restrict__ C, int ldc,
                                                      double beta, const T* __restrict__ X0,
                                                      int64_t ldx0, T* __restrict__ Y, int64_t ldy) {
  __shared__ double Cs[GEMM_PB][QB];
  const int q0 = blockIdx.y * QB;
  const int nq = (q - q0 < QB) ? q - q0 : QB;
  for (int e = threadIdx.x; e < GEMM_PB * QB; e += 256) {
    const int i = e / QB, j = e % QB;
    Cs[i][j] = (i < p && j < nq) ? C[i + (int64_t)(q0 + j) * ldc] : 0.0;
  }
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < N; r += stride) {
    double acc[QB];
#pragma unroll
    for (int j = 0; j < QB; ++j) acc[j] = 0.0;
    // eight columns of A per step, fetched before they are used; the loads
    // are unconditional (a column past p reads column p - 1, not added), so
    // none waits behind a branch
    for (int i0 = 0; i0 < p; i0 += 8) {
      double av[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) av[u] = (double)A[r + (int64_t)(i0 + u < p ? i0 + u : p - 1) * lda];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u < p) {
#pragma unroll
          for (int j = 0; j < QB; ++j) acc[j] += av[u] * Cs[i0 + u][j];
        }
    }
    // the old values of all output columns are fetched before any is stored
    double old[QB];
    if (beta != 0.0) {
#pragma unroll
      for (int j = 0; j < QB; ++j) {
        const int64_t jc = q0 + (j < nq ? j : nq - 1);
        old[j] = (double)(X0 ? X0[r + jc * ldx0] : Y[r + jc * ldy]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < QB; ++j) old[j] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < QB; ++j)
      if (j < nq) Y[r + (int64_t)(q0 + j) * ldy] = (T)(beta * old[j] + alpha * acc[j]);
  }
}

// The leading Schur vectors and their residuals in one pass over the basis
// (long blocks): per row, u = V S[:, :nu] and a = (A V) S[:, :nb], then
// R = a - u T[:nu, :nb].  Each sum is taken in the order k_gemm_nn_long takes
// it, so U and R equal those of the three products U = V S, A U = (A V) S,
// R = A U - U T bit for bit; A U itself is never stored.
template <int QB>
__global__ __launch_bounds__(256) void k_urres_long(int64_t N, int m, int nu, int nb,
                                                    const double* __restrict__ V,
                                                    const double* __restrict__ AV, int64_t ld,
                                                    const double* __restrict__ S,
                                                    const double* __restrict__ Tm,
                                                    double* __restrict__ U,
                                                    double* __restrict__ R, int64_t ldo) {
  __shared__ double Ss[GEMM_PB][QB + 1];
  __shared__ double Ts[QB + 1][QB];
  for (int e = threadIdx.x; e < GEMM_PB * (QB + 1); e += 256) {
    const int i = e / (QB + 1), j = e % (QB + 1);
    Ss[i][j] = (i < m && j < nu) ? S[i + (int64_t)j * m] : 0.0;
  }
  for (int e = threadIdx.x; e < (QB + 1) * QB; e += 256) {
    const int l = e / QB, j = e % QB;
    Ts[l][j] = (l < nu && j < nb) ? Tm[l + (int64_t)j * nu] : 0.0;
  }
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < N; r += stride) {
    double u[QB + 1], a[QB];
#pragma unroll
    for (int j = 0; j <= QB; ++j) u[j] = 0.0;
#pragma unroll
    for (int j = 0; j < QB; ++j) a[j] = 0.0;
    for (int i0 = 0; i0 < m; i0 += 8) {
      double vv[8], av[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        vv[t] = (i0 + t < m) ? V[r + (int64_t)(i0 + t) * ld] : 0.0;
        av[t] = (i0 + t < m) ? AV[r + (int64_t)(i0 + t) * ld] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (i0 + t < m) {
#pragma unroll
          for (int j = 0; j <= QB; ++j) u[j] += vv[t] * Ss[i0 + t][j];
#pragma unroll
          for (int j = 0; j < QB; ++j) a[j] += av[t] * Ss[i0 + t][j];
        }
    }
#pragma unroll
    for (int j = 0; j <= QB; ++j)
      if (j < nu) U[r + (int64_t)j * ldo] = u[j];
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      if (j < nb) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l <= QB; ++l)
          if (l < nu) acc += u[l] * Ts[l][j];
        R[r + (int64_t)j * ldo] = a[j] - acc;
      }
    }
  }
}

hipError_t launch_urres_long(int64_t N, int m, int nu, int nb, const double* V, const double* AV,
                             int64_t ld, const double* S, const double* Tm, double* U, double* R,
                             int64_t ldo, hipStream_t s) {
  if (N < GEMM_LONG_N || m > GEMM_PB || nb > 16 || nu > nb + 1 || nb < 1 || m < 1)
    return hipErrorInvalidValue;
  const int64_t rb = (N + 255) / 256;
  const unsigned gx = (unsigned)(rb < GEMM_LONG_WG ? rb : GEMM_LONG_WG);
  if (nb <= 8)
    hipLaunchKernelGGL((k_urres_long<8>), dim3(gx), dim3(256), 0, s, N, m, nu, nb, V, AV, ld, S, Tm,
                       U, R, ldo);
  else
    hipLaunchKernelGGL((k_urres_long<16>), dim3(gx), dim3(256), 0, s, N, m, nu, nb, V, AV, ld, S,
                       Tm, U, R, ldo);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm_nn_x0(int64_t N, int p, int q, double alpha, const T* A, int64_t lda,
                             const double* C, int ldc, double beta, const T* X0, int64_t ldx0, T* Y,
                             int64_t ldy, hipStream_t s) {
  if (N <= 0 || q <= 0) return hipSuccess;
  if (N >= GEMM_LONG_N && p <= GEMM_PB) {
    const int64_t rb = (N + 255) / 256;
    const unsigned gx = (unsigned)(rb < GEMM_LONG_WG ? rb : GEMM_LONG_WG);
    // A is read once per column block of C: wide blocks for the basis
    // rotations (q up to m_max), narrow ones where q is a block of vectors
    if (q <= 8)
      hipLaunchKernelGGL((k_gemm_nn_long<T, 8>), dim3(gx, 1), dim3(256), 0, s, N, p, q, alpha, A, lda,
                         C, ldc, beta, X0, ldx0, Y, ldy);
    else if (q <= GEMM_QB)
      hipLaunchKernelGGL((k_gemm_nn_long<T, GEMM_QB>), dim3(gx, 1), dim3(256), 0, s, N, p, q, alpha, A,
                         lda, C, ldc, beta, X0, ldx0, Y, ldy);
    else
      hipLaunchKernelGGL((k_gemm_nn_long<T, 32>), dim3(gx, (q + 31) / 32), dim3(256), 0, s, N, p, q,
                         alpha, A, lda, C, ldc, beta, X0, ldx0, Y, ldy);
    return hipGetLastError();
  }
  dim3 grid((unsigned)((N + gemm_rows<true>() - 1) / gemm_rows<true>()), (q + GEMM_QB - 1) / GEMM_QB);
  hipLaunchKernelGGL((k_gemm_nn<T>), grid, dim3(256), 0, s, N, p, q, alpha, A, lda, C, ldc, beta, X0,
                     ldx0, Y, ldy);
  return hipGetLastError();
}
// A[:, :q] = A C in place on the matrix cores.  Each wave takes tiles of 16
// rows: it loads the tile's p columns as the B operand of v_mfma_f64_16x16x4
// (lane l: row l % 16, column 4 ks + l / 16 of k-step ks), and forms
// (A C)^T = C^T A^T per 16-column block with C^T as the A operand, staged once
// per workgroup in LDS in fragment order.  Every load of a tile has been
// consumed before the tile is written, and tiles do not share rows (no
// restrict on A).  The output element of lane l, register r, is row l % 16 and
// column 16 jb + l / 16 + 4 r, so each store instruction writes 16 consecutive
// rows of four columns.  Loads past N or p read a clamped row or column; the
// staged C is zero beyond p and q, so those terms add zero.  KS is the number
// of k-steps (p <= 4 KS, launched with the smallest multiple of 4 that holds
// p) and JB the number of 16-column blocks (q <= 16 JB).
template <int KS, int JB, bool FULL>
__global__ __launch_bounds__(256) void k_gemm_rows_inplace(int64_t N, int p, int q, double* A,
                                                           int64_t lda,
                                                           const double* __restrict__ C, int ldc) {
  extern __shared__ double Cf[];  // [KS][JB][64]
  for (int e = threadIdx.x; e < KS * JB * 64; e += 256) {
    const int ks = e / (JB * 64), jb = (e / 64) % JB, l = e % 64;
    const int k = 4 * ks + l / 16, j = 16 * jb + l % 16;
    Cf[e] = (k < p && j < q) ? C[k + (int64_t)j * ldc] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  const int64_t ntiles = (N + 15) / 16;
  const int64_t wstride = (int64_t)gridDim.x * 4;
  // this lane's row of tile t (clamped), and its column of k-step ks (clamped)
  auto load = [&](int64_t t, double* b) {
    const int64_t row = t * 16 + lr < N ? t * 16 + lr : N - 1;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int c = 4 * ks + lk < p ? 4 * ks + lk : p - 1;
      b[ks] = A[row + (int64_t)c * lda];
    }
  };
  int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  double b[KS];
  if (t < ntiles) load(t, b);
  for (; t < ntiles; t += wstride) {
    const int64_t r0 = t * 16;
    // the next tile's loads go out before this tile's products (other rows:
    // no tile of this wave's is written before it has been read)
    double bn[KS];
    load(t + wstride < ntiles ? t + wstride : t, bn);
    d4 acc[JB];
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) acc[jb] = d4{0, 0, 0, 0};
    // no branch between the products (a branch would move the accumulators
    // between register files at every join), and a scheduling barrier every
    // two k-steps keeps each step's fragment reads next to its products
    // instead of all of them held in registers
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
      for (int jb = 0; jb < JB; ++jb)
        acc[jb] = Mma<double>::mma(Cf[(ks * JB + jb) * 64 + lane], b[ks], acc[jb]);
      if (ks % 2 == 1) __builtin_amdgcn_sched_barrier(0);
    }
    // FULL (q = 16 JB, N a multiple of 16): every lane stores every element,
    // with no masked branch whose join would wait for the prefetch as well
    if (FULL || r0 + lr < N) {
#pragma unroll
      for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = 16 * jb + Mma<double>::row(lk, r);
          if (FULL || col < q) A[r0 + lr + (int64_t)col * lda] = acc[jb][r];
        }
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) b[ks] = bn[ks];
  }
}

template <int KS>
static void launch_rows_inplace_ks(unsigned gx, int64_t N, int p, int q, double* A, int64_t lda,
                                   const double* C, int ldc, hipStream_t s) {
  const int jb = (q + 15) / 16;
  const int JBl = jb <= 1 ? 1 : jb <= 2 ? 2 : 4;
  const size_t lds = (size_t)KS * JBl * 64 * sizeof(double);
  const bool full = q == 16 * JBl && N % 16 == 0;
#define TP3B_ROWS_INPLACE(JBV, FV)                                                                 \
  hipLaunchKernelGGL((k_gemm_rows_inplace<KS, JBV, FV>), dim3(gx), dim3(256), lds, s, N, p, q, A, \
                     lda, C, ldc)
  if (JBl == 1) {
    if (full) TP3B_ROWS_INPLACE(1, true); else TP3B_ROWS_INPLACE(1, false);
  } else if (JBl == 2) {
    if (full) TP3B_ROWS_INPLACE(2, true); else TP3B_ROWS_INPLACE(2, false);
  } else {
    if (full) TP3B_ROWS_INPLACE(4, true); else TP3B_ROWS_INPLACE(4, false);
  }
#undef TP3B_ROWS_INPLACE
}

hipError_t launch_gemm_nn_rows_inplace(int64_t N, int p, int q, double* A, int64_t lda,
                                       const double* C, int ldc, hipStream_t s) {
  if (N < GEMM_LONG_N || p > GEMM_PB || q > p || q < 1 || q > 64) return hipErrorInvalidValue;
  // four waves per workgroup, each over 16-row tiles
  const int64_t wg = ((N + 15) / 16 + 3) / 4;
  const unsigned gx = (unsigned)(wg < GEMM_LONG_WG ? wg : GEMM_LONG_WG);
  switch ((p + 15) / 16) {  // k-steps: the multiple of 4 that holds p
    case 1:
    case 2: launch_rows_inplace_ks<8>(gx, N, p, q, A, lda, C, ldc, s); break;
    case 3: launch_rows_inplace_ks<12>(gx, N, p, q, A, lda, C, ldc, s); break;
    case 4: launch_rows_inplace_ks<16>(gx, N, p, q, A, lda, C, ldc, s); break;
    case 5: launch_rows_inplace_ks<20>(gx, N, p, q, A, lda, C, ldc, s); break;
    case 6: launch_rows_inplace_ks<24>(gx, N, p, q, A, lda, C, ldc, s); break;
    case 7: launch_rows_inplace_ks<28>(gx, N, p, q, A, lda, C, ldc, s); break;
    default: launch_rows_inplace_ks<32>(gx, N, p, q, A, lda, C, ldc, s); break;
  }
  return hipGetLastError();
}

template hipError_t launch_gemm_nn_x0<double>(int64_t, int, int, double, const double*, int64_t,
                                              const double*, int, double, const double*, int64_t,
                                              double*, int64_t, hipStream_t);

template <typename T>
hipError_t launch_gemm_nn(int64_t N, int p, int q, double alpha, const T* A, int64_t lda,
                          const double* C, int ldc, double beta, T* Y, int64_t ldy,
                          hipStream_t s) {
  return launch_gemm_nn_x0<T>(N, p, q, alpha, A, lda, C, ldc, beta, (const T*)nullptr, 0, Y, ldy, s);
}
template hipError_t launch_gemm_nn<double>(int64_t, int, int, double, const double*, int64_t,
                                           const double*, int, double, double*, int64_t,
                                           hipStream_t);
template hipError_t launch_gemm_nn<float>(int64_t, int, int, double, const float*, int64_t,
                                          const double*, int, double, float*, int64_t,
                                          hipStream_t);

// ------------------------------------------------ per-column (diagonal) dots
int64_t bdot_scratch_doubles(int64_t N, int b, int nb) {
  int64_t nchunk = (N + bdot_rows(N) - 1) / bdot_rows(N);
  return nchunk * b * BD_MAXNB;
}

template <typename T>
__global__ __launch_bounds__(256) void k_bdot_diag(int64_t N, int b, int nb, const T* __restrict__ V,
                                                   int64_t bs, const T* __restrict__ W, int rows,
                                                   double* __restrict__ part) {
  __shared__ BdotSmem sm;
  const int j = blockIdx.y, chunk = blockIdx.x;
  bdot_chunk<T>(N, nb, V, bs, W, rows, chunk, j, part + ((int64_t)chunk * b + j) * BD_MAXNB, sm);
}

// The same partials as bdot_chunk (the same products added in the same order:
// per step of four rows, basis block by basis block, row by row) for bases of
// at most NBM blocks, with every load of a step issued before its products:
// rows past the chunk read its last row and blocks past nb read block nb - 1,
// and neither is added, so no load waits behind a branch.
template <typename T, int NBM>
__global__ __launch_bounds__(256) void k_bdot_diag_n(int64_t N, int b, int nb, const T* __restrict__ V,
                                                     int64_t bs, const T* __restrict__ W, int rows,
                                                     double* __restrict__ part) {
  __shared__ double red[NBM][4];
  const int j = blockIdx.y, chunk = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t rbeg = (int64_t)chunk * rows;
  const int64_t rend = (rbeg + rows < N) ? rbeg + rows : N;
  double acc[NBM];
#pragma unroll
  for (int i = 0; i < NBM; ++i) acc[i] = 0.0;
  const T* Wj = W + (int64_t)j * N;
  for (int64_t r = rbeg + tid; r < rend; r += 1024) {
    int64_t rq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) rq[q] = (r + 256 * q < rend) ? r + 256 * q : rend - 1;
    double w[4], v[NBM][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = (double)Wj[rq[q]];
#pragma unroll
    for (int i = 0; i < NBM; ++i) {
      const T* Vi = V + (int64_t)(i < nb ? i : nb - 1) * bs + (int64_t)j * N;
#pragma unroll
      for (int q = 0; q < 4; ++q) v[i][q] = (double)Vi[rq[q]];
    }
#pragma unroll
    for (int i = 0; i < NBM; ++i)
      if (i < nb) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (r + 256 * q < rend) acc[i] += v[i][q] * w[q];
      }
  }
#pragma unroll
  for (int i = 0; i < NBM; ++i) {
    if (i < nb) {
      double x = acc[i];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
      if (lane == 0) red[i][wave] = x;
    }
  }
  __syncthreads();
  if (tid < nb)
    part[((int64_t)chunk * b + j) * BD_MAXNB + tid] = red[tid][0] + red[tid][1] + red[tid][2] + red[tid][3];
}

__global__ __launch_bounds__(256) void k_bdot_reduce(int b, int nb, int nchunk,
                                                     const double* __restrict__ part,
                                                     double* __restrict__ H, int hld) {
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= b * nb) return;
  const int j = e / nb, i = e % nb;
  const double s = bdot_reduce_elem(b, j, i, nchunk, part, lane);
  if (lane == 0) H[(int64_t)j * hld + i] = s;
}

template <typename T>
hipError_t launch_bdot_diag(int64_t N, int b, int nb, const T* V, int64_t bs, const T* W,
                            double* H, int hld, double* partial, hipStream_t s) {
  if (nb <= 0 || b <= 0) return hipSuccess;
  if (nb > BD_MAXNB) return hipErrorInvalidValue;
  const int rows = bdot_rows(N);
  const int nchunk = (int)((N + rows - 1) / rows);
  if (nb == 1)
    hipLaunchKernelGGL((k_bdot_diag_n<T, 1>), dim3(nchunk, b), dim3(256), 0, s, N, b, nb, V, bs, W,
                       rows, partial);
  else if (nb == 2)
    hipLaunchKernelGGL((k_bdot_diag_n<T, 2>), dim3(nchunk, b), dim3(256), 0, s, N, b, nb, V, bs, W,
                       rows, partial);
  else if (nb <= 4)
    hipLaunchKernelGGL((k_bdot_diag_n<T, 4>), dim3(nchunk, b), dim3(256), 0, s, N, b, nb, V, bs, W,
                       rows, partial);
  else if (nb <= 8)
    hipLaunchKernelGGL((k_bdot_diag_n<T, 8>), dim3(nchunk, b), dim3(256), 0, s, N, b, nb, V, bs, W,
                       rows, partial);
  else
    hipLaunchKernelGGL((k_bdot_diag<T>), dim3(nchunk, b), dim3(256), 0, s, N, b, nb, V, bs, W, rows,
                       partial);
  hipLaunchKernelGGL(k_bdot_reduce, dim3((b * nb + 3) / 4), dim3(256), 0, s, b, nb, nchunk, partial,
                     H, hld);
  return hipGetLastError();
}
template hipError_t launch_bdot_diag<double>(int64_t, int, int, const double*, int64_t,
                                             const double*, double*, int, double*, hipStream_t);
template hipError_t launch_bdot_diag<float>(int64_t, int, int, const float*, int64_t,
                                            const float*, double*, int, double*, hipStream_t);

// Out[r, j] = alpha * sum_{i<nb} Vb[i][r, j] H[j*hld + i], assigned (not added)
// and stored in the output type: the combination of a GMRES basis with its
// least-squares coefficients, written straight into the FP64 correction. The
// terms are taken in the order bupdate_row takes them, and an exactly zero
// coefficient again contributes nothing.
template <typename T, typename TO>
__global__ __launch_bounds__(256) void k_bcombine(int64_t N, int nb, double alpha,
                                                  const T* __restrict__ V, int64_t bs,
                                                  const double* __restrict__ H, int hld,
                                                  TO* __restrict__ Out, int64_t ldo) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= N) return;
  double acc = 0.0;
  for (int i0 = 0; i0 < nb; i0 += 8) {
    double v[8], h[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u;
      h[u] = (i < nb) ? H[(int64_t)j * hld + i] : 0.0;
      v[u] = (h[u] != 0.0) ? (double)V[(int64_t)i * bs + (int64_t)j * N + r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (h[u] != 0.0) acc += v[u] * h[u];
  }
  Out[(int64_t)j * ldo + r] = (TO)(alpha * acc);
}

template <typename T, typename TO>
hipError_t launch_bcombine(int64_t N, int b, int nb, double alpha, const T* V, int64_t bs,
                           const double* H, int hld, TO* Out, int64_t ldo, hipStream_t s) {
  if (N <= 0 || b <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_bcombine<T, TO>), dim3((unsigned)((N + 255) / 256), b), dim3(256), 0, s,
                     N, nb, alpha, V, bs, H, hld, Out, ldo);
  return hipGetLastError();
}
template hipError_t launch_bcombine<double, double>(int64_t, int, int, double, const double*,
                                                    int64_t, const double*, int, double*, int64_t,
                                                    hipStream_t);
template hipError_t launch_bcombine<float, double>(int64_t, int, int, double, const float*,
                                                   int64_t, const double*, int, double*, int64_t,
                                                   hipStream_t);

// ------------------------------------- Arnoldi steps with the reduction fused
// The per-column dots' first stage alone: partials for launch_bupdate_diag_red
// and launch_normalize_cols_red, which sum them themselves (each workgroup in
// the same order as k_bdot_reduce, so the results are those of
// launch_bdot_diag followed by the plain update) and save one launch each.
template <typename T>
hipError_t launch_bdot_partials(int64_t N, int b, int nb, const T* V, int64_t bs, const T* W,
                                double* partial, hipStream_t s) {
  if (nb <= 0 || b <= 0) return hipSuccess;
  if (nb > BD_MAXNB) return hipErrorInvalidValue;
  const int rows = bdot_rows(N);
  const int nchunk = (int)((N + rows - 1) / rows);
  if (nb == 1)
    hipLaunchKernelGGL((k_bdot_diag_n<T, 1>), dim3(nchunk, b), dim3(256), 0, s, N, b, nb, V, bs, W,
                       rows, partial);
  else if (nb == 2)
    hipLaunchKernelGGL((k_bdot_diag_n<T, 2>), dim3(nchunk, b), dim3(256), 0, s, N, b, nb, V, bs, W,
                       rows, partial);
  else if (nb <= 4)
    hipLaunchKernelGGL((k_bdot_diag_n<T, 4>), dim3(nchunk, b), dim3(256), 0, s, N, b, nb, V, bs, W,
                       rows, partial);
  else if (nb <= 8)
    hipLaunchKernelGGL((k_bdot_diag_n<T, 8>), dim3(nchunk, b), dim3(256), 0, s, N, b, nb, V, bs, W,
                       rows, partial);
  else
    hipLaunchKernelGGL((k_bdot_diag<T>), dim3(nchunk, b), dim3(256), 0, s, N, b, nb, V, bs, W, rows,
                       partial);
  return hipGetLastError();
}
template hipError_t launch_bdot_partials<double>(int64_t, int, int, const double*, int64_t,
                                                 const double*, double*, hipStream_t);
template hipError_t launch_bdot_partials<float>(int64_t, int, int, const float*, int64_t,
                                                const float*, double*, hipStream_t);

// The workgroup's column j: hs[i] = sum of the partials of entry i (one wave
// per entry, the order of k_bdot_reduce); workgroup 0 of the column also
// stores them to H.
__device__ __forceinline__ void bdot_sum_column(int b, int nb, int nchunk, int j,
                                                const double* __restrict__ part,
                                                double* __restrict__ H, int hld, double* hs) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = wave; i < nb; i += 4) {
    const double v = bdot_reduce_elem(b, j, i, nchunk, part, lane);
    if (lane == 0) hs[i] = v;
  }
  __syncthreads();
  if (blockIdx.x == 0 && H && (int)threadIdx.x < nb) H[(int64_t)j * hld + threadIdx.x] = hs[threadIdx.x];
}

template <typename T>
__global__ __launch_bounds__(256) void k_bupdate_diag_red(int64_t N, int b, int nb, int nchunk,
                                                          double alpha, const T* __restrict__ V,
                                                          int64_t bs, const double* __restrict__ part,
                                                          double* __restrict__ H, int hld,
                                                          T* __restrict__ W) {
  __shared__ double hs[BD_MAXNB];
  bdot_sum_column(b, nb, nchunk, blockIdx.y, part, H, hld, hs);
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < N; r += (int64_t)gridDim.x * 256)
    bupdate_row<T>(N, nb, alpha, V, bs, hs, 0, W, r, blockIdx.y);
}

// Workgroups per column of the fused Arnoldi kernels: every workgroup first
// sums the column's partials, so their number is bounded and each strides
// over many rows.
constexpr int64_t ARN_WG_PER_COL = 512;
inline unsigned arn_grid_x(int64_t N) {
  const int64_t rb = (N + 255) / 256;
  return (unsigned)(rb < ARN_WG_PER_COL ? (rb > 0 ? rb : 1) : ARN_WG_PER_COL);
}

template <typename T>
hipError_t launch_bupdate_diag_red(int64_t N, int b, int nb, double alpha, const T* V, int64_t bs,
                                   const double* partial, double* H, int hld, T* W, hipStream_t s) {
  if (N <= 0 || b <= 0) return hipSuccess;
  if (nb > BD_MAXNB) return hipErrorInvalidValue;
  const int rows = bdot_rows(N);
  const int nchunk = (int)((N + rows - 1) / rows);
  hipLaunchKernelGGL((k_bupdate_diag_red<T>), dim3(arn_grid_x(N), b), dim3(256), 0, s,
                     N, b, nb, nchunk, alpha, V, bs, partial, H, hld, W);
  return hipGetLastError();
}
template hipError_t launch_bupdate_diag_red<double>(int64_t, int, int, double, const double*,
                                                    int64_t, const double*, double*, int, double*,
                                                    hipStream_t);
template hipError_t launch_bupdate_diag_red<float>(int64_t, int, int, double, const float*, int64_t,
                                                   const double*, double*, int, float*, hipStream_t);

template <typename T>
__global__ __launch_bounds__(256) void k_normalize_cols_red(int64_t N, int b, int nchunk,
                                                            const double* __restrict__ part,
                                                            const T* __restrict__ W,
                                                            T* __restrict__ Vout,
                                                            double* __restrict__ hout, int hld) {
  __shared__ double hs[1];
  bdot_sum_column(b, 1, nchunk, blockIdx.y, part, nullptr, 0, hs);
  const int64_t r0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  // the norm and its reciprocal as normalize_row_n2 forms them; row 0 (N = 0
  // included) stores the norm
  const double h = hs[0] > 0.0 ? sqrt(hs[0]) : 0.0;
  const double inv = h > 0.0 ? 1.0 / h : 0.0;
  if (r0 == 0 && hout) hout[(int64_t)j * hld] = h;
  const T* Wj = W + (int64_t)j * N;
  T* Vj = Vout + (int64_t)j * N;
  // four rows per thread at a time, their loads all issued first, then the
  // rows left one at a time
  const int64_t S = (int64_t)gridDim.x * 256;
  int64_t r = r0;
  for (; r + 3 * S < N; r += 4 * S) {
    T w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = Wj[r + u * S];
#pragma unroll
    for (int u = 0; u < 4; ++u) Vj[r + u * S] = (T)((double)w[u] * inv);
  }
  for (; r < N; r += S) Vj[r] = (T)((double)Wj[r] * inv);
}

template <typename T>
hipError_t launch_normalize_cols_red(int64_t N, int b, const double* partial, const T* W, T* Vout,
                                     double* hout, int hld, hipStream_t s) {
  if (b <= 0) return hipSuccess;
  const int rows = bdot_rows(N);
  const int nchunk = (int)((N + rows - 1) / rows);
  hipLaunchKernelGGL((k_normalize_cols_red<T>), dim3(arn_grid_x(N), b),
                     dim3(256), 0, s, N, b, nchunk, partial, W, Vout, hout, hld);
  return hipGetLastError();
}
template hipError_t launch_normalize_cols_red<double>(int64_t, int, const double*, const double*,
                                                      double*, double*, int, hipStream_t);
template hipError_t launch_normalize_cols_red<float>(int64_t, int, const double*, const float*,
                                                     float*, double*, int, hipStream_t);

template <typename T>
hipError_t launch_normalize_cols_red_n(int64_t N, int b, const double* partial, int nchunk,
                                       const T* W, T* Vout, double* hout, int hld, hipStream_t s) {
  if (b <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_normalize_cols_red<T>), dim3(arn_grid_x(N), b), dim3(256), 0, s, N, b, nchunk,
                     partial, W, Vout, hout, hld);
  return hipGetLastError();
}
template hipError_t launch_normalize_cols_red_n<double>(int64_t, int, const double*, int, const double*,
                                                        double*, double*, int, hipStream_t);
template hipError_t launch_normalize_cols_red_n<float>(int64_t, int, const double*, int, const float*,
                                                       float*, double*, int, hipStream_t);

// ----------------------------- Arnoldi update fused with the following dots
int bupdate_dot_chunks(int64_t N) { return (int)arn_grid_x(N); }
int64_t bupdate_dot_scratch_doubles(int64_t N, int b) {
  return (int64_t)bupdate_dot_chunks(N) * b * BD_MAXNB;
}

template <typename T, int NBM>
__global__ __launch_bounds__(256) void k_bupdate_dot_red(int64_t N, int b, int nb, int nchunk_in,
                                                         double alpha, const T* __restrict__ V,
                                                         int64_t bs, const double* __restrict__ part_in,
                                                         double* __restrict__ H, int hld,
                                                         T* __restrict__ W, int self,
                                                         double* __restrict__ part_out) {
  __shared__ double hs[BD_MAXNB];
  __shared__ double red[NBM][4];
  const int j = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bdot_sum_column(b, nb, nchunk_in, j, part_in, H, hld, hs);
  double acc[NBM];
#pragma unroll
  for (int i = 0; i < NBM; ++i) acc[i] = 0.0;
  T* Wj = W + (int64_t)j * N;
  // every load is issued (a basis vector past nb reads vector nb - 1, and one
  // whose coefficient is zero is read too, though neither value is used): no
  // load sits behind a branch, whose join would wait for all of them
  auto load = [&](int64_t r, double* v, T& w) {
#pragma unroll
    for (int i = 0; i < NBM; ++i) {
      const int ic = i < nb ? i : nb - 1;
      v[i] = (double)V[(int64_t)ic * bs + (int64_t)j * N + r];
    }
    w = Wj[r];
  };
  // the update of bupdate_row (same terms, same order), keeping the basis
  // values for the dots
  auto row = [&](int64_t r, const double* v, T w) {
    double sum = 0.0;
    // ascending i, as bupdate_row adds them
#pragma unroll
    for (int i = 0; i < NBM; ++i) {
      const double h = (i < nb) ? hs[i] : 0.0;
      if (h != 0.0) sum += v[i] * h;
    }
    const T wn = (T)((double)w + alpha * sum);
    Wj[r] = wn;
    const double wd = (double)wn;
    if (self) {
      acc[0] += wd * wd;
    } else {
#pragma unroll
      for (int i = 0; i < NBM; ++i)
        if (i < nb) acc[i] += v[i] * wd;
    }
  };
  // each thread takes its rows in stride order, RU at a time with all of
  // their loads in flight (fewer for longer bases, whose rows need more
  // registers), then one at a time (the same order either way)
  constexpr int RU = NBM <= 4 ? 4 : NBM <= 8 ? 2 : 1;
  const int64_t S = (int64_t)gridDim.x * 256;
  int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; r + (RU - 1) * S < N; r += RU * S) {
    double v[RU][NBM];
    T w[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) load(r + u * S, v[u], w[u]);
#pragma unroll
    for (int u = 0; u < RU; ++u) row(r + u * S, v[u], w[u]);
  }
  for (; r < N; r += S) {
    double v[NBM];
    T w;
    load(r, v, w);
    row(r, v, w);
  }
  const int nd = self ? 1 : nb;
#pragma unroll
  for (int i = 0; i < NBM; ++i) {
    if (i < nd) {
      double x = acc[i];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
      if (lane == 0) red[i][wave] = x;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nd)
    part_out[((int64_t)blockIdx.x * b + j) * BD_MAXNB + threadIdx.x] =
        red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
}

template <typename T>
hipError_t launch_bupdate_dot_red(int64_t N, int b, int nb, double alpha, const T* V, int64_t bs,
                                  const double* part_in, int nchunk_in, double* H, int hld, T* W,
                                  int self, double* part_out, hipStream_t s) {
  if (N <= 0 || b <= 0) return hipSuccess;
  if (nb < 1 || nb > BDF_MAXNB || part_in == part_out) return hipErrorInvalidValue;
  const int nin = nchunk_in > 0 ? nchunk_in : (int)((N + bdot_rows(N) - 1) / bdot_rows(N));
  // register arrays sized for the basis length (a few GMRES steps: 4)
  if (nb <= 4)
    hipLaunchKernelGGL((k_bupdate_dot_red<T, 4>), dim3(arn_grid_x(N), b), dim3(256), 0, s, N, b, nb, nin,
                       alpha, V, bs, part_in, H, hld, W, self, part_out);
  else if (nb <= 8)
    hipLaunchKernelGGL((k_bupdate_dot_red<T, 8>), dim3(arn_grid_x(N), b), dim3(256), 0, s, N, b, nb, nin,
                       alpha, V, bs, part_in, H, hld, W, self, part_out);
  else
    hipLaunchKernelGGL((k_bupdate_dot_red<T, BDF_MAXNB>), dim3(arn_grid_x(N), b), dim3(256), 0, s, N, b,
                       nb, nin, alpha, V, bs, part_in, H, hld, W, self, part_out);
  return hipGetLastError();
}
template hipError_t launch_bupdate_dot_red<double>(int64_t, int, int, double, const double*, int64_t,
                                                   const double*, int, double*, int, double*, int,
                                                   double*, hipStream_t);
template hipError_t launch_bupdate_dot_red<float>(int64_t, int, int, double, const float*, int64_t,
                                                  const double*, int, double*, int, float*, int,
                                                  double*, hipStream_t);

// -------------------------------------------------------------- conversions
template <typename TI, typename TO>
__global__ void k_convert(int64_t N, double alpha, const TI* __restrict__ X, int64_t ldx,
                          TO* __restrict__ Y, int64_t ldy) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= N) return;
  Y[r + (int64_t)j * ldy] = X ? (TO)(alpha * (double)X[r + (int64_t)j * ldx]) : (TO)0;
}

template <typename TI, typename TO>
hipError_t launch_convert(int64_t N, int ncol, double alpha, const TI* X, int64_t ldx, TO* Y,
                          int64_t ldy, hipStream_t s) {
  if (N <= 0 || ncol <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_convert<TI, TO>), dim3((unsigned)((N + 255) / 256), ncol), dim3(256), 0, s,
                     N, alpha, X, ldx, Y, ldy);
  return hipGetLastError();
}
template hipError_t launch_convert<double, float>(int64_t, int, double, const double*, int64_t,
                                                  float*, int64_t, hipStream_t);
template hipError_t launch_convert<float, double>(int64_t, int, double, const float*, int64_t,
                                                  double*, int64_t, hipStream_t);
template hipError_t launch_convert<double, double>(int64_t, int, double, const double*, int64_t,
                                                   double*, int64_t, hipStream_t);
template hipError_t launch_convert<float, float>(int64_t, int, double, const float*, int64_t,
                                                 float*, int64_t, hipStream_t);

// -------------------------------------------------------- Cholesky-QR pieces
// The Gram matrix is staged in LDS by the whole wavefront, one thread
// factorises it there (the serial arithmetic of the grouped form, without a
// global-memory round trip per element), and the factor is written back in
// parallel.  nx <= TRSM_MAX.
// Right-looking form on one wavefront: step j scales row j of R and removes
// its outer product from the trailing upper triangle, so every entry receives
// the same terms in the same order as the column-by-column (left-looking)
// serial form.
__global__ __launch_bounds__(64) void k_chol_small(int nx, const double* __restrict__ G,
                                                   const double* __restrict__ n0, double drop_tol,
                                                   double* __restrict__ R, int* __restrict__ flags,
                                                   const int* __restrict__ skip) {
  __shared__ double Gs[TRSM_MAX * TRSM_MAX], Rs[TRSM_MAX * TRSM_MAX];
  const int t = threadIdx.x;
  for (int e = t; e < nx * nx; e += 64) {
    Gs[e] = G[e];
    Rs[e] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nx; ++j) {
    const double d = Gs[j + j * nx];
    const double thr = drop_tol * drop_tol * n0[j];
    if ((skip && skip[j]) || !(d > thr) || !(d > 0.0)) {
      // dependent column (or one a previous factorisation found dependent):
      // left unscaled (replaced later), contributes nothing to the others
      if (t == 0) {
        flags[j] = 1;
        Rs[j + j * nx] = 1.0;
      }
      __syncthreads();
      continue;
    }
    if (t == 0) flags[j] = 0;
    const double rjj = sqrt(d);
    for (int c = j + t; c < nx; c += 64) Rs[j + c * nx] = (c == j) ? rjj : Gs[j + c * nx] / rjj;
    __syncthreads();
    const int m = nx - j - 1;
    for (int e = t; e < m * m; e += 64) {
      const int a = j + 1 + e % m, c = j + 1 + e / m;
      if (c >= a) Gs[a + c * nx] -= Rs[j + a * nx] * Rs[j + c * nx];
    }
    __syncthreads();
  }
  for (int e = t; e < nx * nx; e += 64) R[e] = Rs[e];
}

__global__ void k_gram_diag(int nx, const double* __restrict__ G, double* __restrict__ n0,
                            int* __restrict__ flag) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int bad = 0;
  for (int j = 0; j < nx; ++j) {
    const double v = G[j + j * nx];
    n0[j] = v;
    if (!(v - v == 0.0)) bad = 1;
  }
  flag[0] = bad;
}

hipError_t launch_gram_diag(int nx, const double* G, double* n0, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_gram_diag, dim3(1), dim3(64), 0, s, nx, G, n0, flag);
  return hipGetLastError();
}

hipError_t launch_chol_small(int nx, const double* G, const double* norm0sq, double drop_tol,
                             double* R, int* flags, hipStream_t s, const int* skip) {
  if (nx < 1 || nx > TRSM_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chol_small, dim3(1), dim3(64), 0, s, nx, G, norm0sq, drop_tol, R, flags,
                     skip);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_trsm_right(int64_t N, int nx, const double* __restrict__ R,
                                                    double* __restrict__ X, int64_t ldx) {
  __shared__ TrsmSmem sm;
  trsm_block(N, nx, R, X, ldx, blockIdx.x, sm);
}

hipError_t launch_trsm_right(int64_t N, int nx, const double* R, double* X, int64_t ldx,
                             hipStream_t s) {
  if (N <= 0) return hipSuccess;
  if (nx > TRSM_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_trsm_right, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, nx, R, X,
                     ldx);
  return hipGetLastError();
}

__global__ void k_hash_fill(int64_t N, double* __restrict__ X, uint64_t seed, uint64_t sid) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= N) return;
  X[r] = hash_uniform(seed, sid, r);
}

hipError_t launch_hash_fill(int64_t N, double* X, uint64_t seed, uint64_t stream_id,
                            hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_fill, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, X, seed,
                     stream_id);
  return hipGetLastError();
}

template <typename T>
__global__ void k_check_finite(int64_t N, const T* __restrict__ X, int64_t ldx,
                               int* __restrict__ flag) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= N) return;
  const double v = (double)X[r + (int64_t)j * ldx];
  if (!(v - v == 0.0)) flag[0] = 1;
}

template <typename T>
hipError_t launch_check_finite(int64_t N, int ncol, const T* X, int64_t ldx, int* flag,
                               hipStream_t s) {
  if (N <= 0 || ncol <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_check_finite<T>), dim3((unsigned)((N + 255) / 256), ncol), dim3(256), 0, s,
                     N, X, ldx, flag);
  return hipGetLastError();
}
template hipError_t launch_check_finite<double>(int64_t, int, const double*, int64_t, int*,
                                                hipStream_t);
template hipError_t launch_check_finite<float>(int64_t, int, const float*, int64_t, int*,
                                               hipStream_t);

// ------------------------------------------------ small dense steps on the device
// GMRES least squares, one workgroup per correction column j: ks is the number
// of steps before the first breakdown (subdiagonal <= 1e-14 beta), the
// (ks + 1) x ks Hessenberg matrix (sum of the two Gram-Schmidt passes, then the
// subdiagonal norms) is assembled in LDS, and one thread minimises
// || beta e1 - H y || by Givens rotations and back substitution.
// Y[j*hld + i] = y_i for i < ks, 0 up to hld; beta == 0 gives y = 0.
__global__ __launch_bounds__(64) void k_gmres_lstsq(int b, int steps, int hld,
                                                    const double* __restrict__ H1,
                                                    const double* __restrict__ H2,
                                                    const double* __restrict__ Hs,
                                                    const double* __restrict__ Beta,
                                                    double* __restrict__ Y) {
  __shared__ double R[(GL_MAXSTEPS + 1) * GL_MAXSTEPS];
  __shared__ double g[GL_MAXSTEPS + 1];
  __shared__ double y[GL_MAXSTEPS];
  __shared__ int ks_s;
  const int j = blockIdx.x, tid = threadIdx.x;
  const double beta = Beta[j];
  if (tid == 0) {
    int ks = 0;
    if (beta > 0)
      for (int kk = 0; kk < steps; ++kk) {
        ks = kk + 1;
        if (!(Hs[(int64_t)kk * b + j] > 1e-14 * beta)) break;
      }
    ks_s = ks;
  }
  __syncthreads();
  const int ks = ks_s;
  for (int e = tid; e < (ks + 1) * ks; e += 64) {
    const int i = e / ks, kk = e % ks;
    double v = 0.0;
    if (i <= kk) {
      const int64_t o = (int64_t)kk * b * hld + (int64_t)j * hld + i;
      v = H1[o] + H2[o];
    } else if (i == kk + 1) {
      v = Hs[(int64_t)kk * b + j];
    }
    R[e] = v;
  }
  __syncthreads();
  if (tid == 0 && ks > 0) {
    for (int i = 0; i <= ks; ++i) g[i] = 0.0;
    g[0] = beta;
    for (int c = 0; c < ks; ++c) {
      const double a = R[c * ks + c], d = R[(c + 1) * ks + c];
      const double r = hypot(a, d);
      const double cs = (r == 0) ? 1.0 : a / r, sn = (r == 0) ? 0.0 : d / r;
      for (int cc = c; cc < ks; ++cc) {
        const double u = R[c * ks + cc], v = R[(c + 1) * ks + cc];
        R[c * ks + cc] = cs * u + sn * v;
        R[(c + 1) * ks + cc] = -sn * u + cs * v;
      }
      const double u = g[c], v = g[c + 1];
      g[c] = cs * u + sn * v;
      g[c + 1] = -sn * u + cs * v;
    }
    for (int i = ks - 1; i >= 0; --i) {
      double acc = g[i];
      for (int c = i + 1; c < ks; ++c) acc -= R[i * ks + c] * y[c];
      const double dd = R[i * ks + i];
      y[i] = (dd != 0.0) ? acc / dd : 0.0;
    }
  }
  __syncthreads();
  for (int i = tid; i < hld; i += 64) Y[(int64_t)j * hld + i] = (i < ks) ? y[i] : 0.0;
}

hipError_t launch_gmres_lstsq(int nb, int b, int steps, int hld, const double* H1, const double* H2,
                              const double* Hs, const double* Beta, double* Y, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  if (steps < 1 || steps > GL_MAXSTEPS || hld < steps) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gmres_lstsq, dim3(nb), dim3(64), 0, s, b, steps, hld, H1, H2, Hs, Beta, Y);
  return hipGetLastError();
}

// Inverse of an n x n column-major matrix, n <= SI_MAXN, by Gauss-Jordan
// elimination with partial pivoting on [A | I] in LDS; one wavefront, thread t
// owns row t in the elimination.  *singular = 1 (else 0) when a pivot column
// is exactly zero; Ainv is then not meaningful.
__global__ __launch_bounds__(64) void k_small_inverse(int n, const double* __restrict__ A,
                                                      double* __restrict__ Ainv,
                                                      int* __restrict__ singular) {
  __shared__ double M[SI_MAXN][2 * SI_MAXN + 1];
  __shared__ double fcol[SI_MAXN];
  const int t = threadIdx.x, w = 2 * n;
  for (int e = t; e < n * w; e += 64) {
    const int r = e / w, c = e % w;
    M[r][c] = (c < n) ? A[r + (int64_t)c * n] : (c - n == r ? 1.0 : 0.0);
  }
  __syncthreads();
  int bad = 0;
  for (int k = 0; k < n; ++k) {
    // pivot: the first row r >= k of largest |M[r][k]| (wave argmax, ties to
    // the smaller row; NaN never wins), the same row on every lane
    double v = (t >= k && t < n) ? fabs(M[t][k]) : -1.0;
    if (!(v == v)) v = -1.0;
    int idx = t;
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(v, off, 64);
      const int oi = __shfl_xor(idx, off, 64);
      if (ov > v || (ov == v && oi < idx)) {
        v = ov;
        idx = oi;
      }
    }
    int p = __shfl(idx, 0, 64);
    if (p < k || p >= n) p = k;
    if (M[p][k] == 0.0) {
      bad = 1;
      break;
    }
    if (p != k)
      for (int c = t; c < w; c += 64) {
        const double u = M[k][c];
        M[k][c] = M[p][c];
        M[p][c] = u;
      }
    __syncthreads();
    // the multipliers of the other rows, before row k is scaled
    if (t < n) fcol[t] = M[t][k];
    const double d = M[k][k];
    __syncthreads();
    for (int c = t; c < w; c += 64) M[k][c] /= d;
    __syncthreads();
    for (int e = t; e < n * w; e += 64) {
      const int r = e / w, c = e % w;
      if (r != k) M[r][c] -= fcol[r] * M[k][c];
    }
    __syncthreads();
  }
  if (t == 0) *singular = bad;
  for (int e = t; e < n * n; e += 64) {
    const int r = e % n, c = e / n;
    Ainv[r + (int64_t)c * n] = M[r][n + c];
  }
}

hipError_t launch_small_inverse(int n, const double* A, double* Ainv, int* singular, hipStream_t s) {
  if (n < 1 || n > SI_MAXN) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_small_inverse, dim3(1), dim3(64), 0, s, n, A, Ainv, singular);
  return hipGetLastError();
}

}  // namespace tp3b
