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

#include <hip/hip_runtime.h>

namespace tp3b {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mma;
// Output element r of lane l in a 16 x 16 block: column l % 16 for both; row
// (l/16) + 4r for the f64 instruction, 4(l/16) + r for the f32 one (the f64
// layout was established with an on-device lane probe).
template <>
struct Mma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Work-item order that keeps consecutive work items on the same XCD.
// Workgroups are dispatched round-robin over the 8 XCDs, so workgroup id g
// runs on XCD g % 8; give XCD x the contiguous range of work items
// [x*q + min(x, r), ...) where G = 8q + r.
__device__ __forceinline__ int64_t xcd_remap(int64_t g, int64_t G) {
  const int64_t q = G >> 3, r = G & 7;
  const int64_t x = g & 7, local = g >> 3;
  return x * q + (x < r ? x : r) + local;
}

// ------------------------------------------------------------------ mode product
// ROLE only separates the kernel names seen by profilers: 0 = Hamiltonian apply
// (both modes + potential), 1 = preconditioner mode products, 2 = 2D x-mode
// accumulation passes.
template <typename T, int TM, int TN, int KC, int ROLE>
__global__ __launch_bounds__(256) void k_modeprod(ModeProd<T> a) {
  typedef typename Mma<T>::acc_t acc_t;
  constexpr int WM = TM / 2, WN = TN / 2;
  constexpr int BM = WM / 16, BN = WN / 16;
  constexpr int EA = TM * KC / 256, EB = KC * TN / 256;
  static_assert(EA >= 1 && EB >= 1, "tile too small for 256 threads");
  __shared__ T As[KC][TM + 1];
  __shared__ T Bs[KC][TN + 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
  const int tiles_m = (a.M + TM - 1) / TM, tiles_n = (a.Nc + TN - 1) / TN;
  const int64_t tiles = (int64_t)tiles_m * tiles_n;
  const int64_t G = tiles * a.nbatch;
  const int64_t w = xcd_remap(blockIdx.x, G);
  const int64_t q = w / tiles;
  const int64_t t = w - q * tiles;
  const int i0 = (int)(t / tiles_n) * TM, j0 = (int)(t % tiles_n) * TN;
  const int64_t vec = q / a.per_vec, item = q - vec * a.per_vec;
  const T* __restrict__ X = a.X + vec * a.ldx + item * a.bstride;
  T* __restrict__ Y = a.Y + vec * a.ldy + item * a.bstride;
  const int64_t rs = a.rs;
  const int M = a.M, Nc = a.Nc;

  acc_t acc[BM][BN];
#pragma unroll
  for (int bi = 0; bi < BM; ++bi)
#pragma unroll
    for (int bj = 0; bj < BN; ++bj) acc[bi][bj] = acc_t{0, 0, 0, 0};

  const int nL = a.L ? (M + KC - 1) / KC : 0;
  const int nR = a.R ? (Nc + KC - 1) / KC : 0;
  const int nchunks = nL + nR;
  T ra[EA], rb[EB];

  auto load = [&](int c) {
    if (c < nL) {
      const int k0 = c * KC;
#pragma unroll
      for (int s = 0; s < EA; ++s) {
        const int e = tid + s * 256, m = e / KC, k = e % KC;
        const int gi = i0 + m, gk = k0 + k;
        ra[s] = (gi < M && gk < M) ? a.L[(int64_t)gi * M + gk] : T(0);
      }
#pragma unroll
      for (int s = 0; s < EB; ++s) {
        const int e = tid + s * 256, k = e / TN, n = e % TN;
        const int gk = k0 + k, gj = j0 + n;
        rb[s] = (gk < M && gj < Nc) ? X[(int64_t)gk * rs + gj] : T(0);
      }
    } else {
      const int k0 = (c - nL) * KC;
#pragma unroll
      for (int s = 0; s < EA; ++s) {
        const int e = tid + s * 256, m = e / KC, k = e % KC;
        const int gi = i0 + m, gk = k0 + k;
        ra[s] = (gi < M && gk < Nc) ? X[(int64_t)gi * rs + gk] : T(0);
      }
#pragma unroll
      for (int s = 0; s < EB; ++s) {
        const int e = tid + s * 256, k = e / TN, n = e % TN;
        const int gk = k0 + k, gj = j0 + n;
        rb[s] = (gk < Nc && gj < Nc) ? a.R[(int64_t)gk * Nc + gj] : T(0);
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int s = 0; s < EA; ++s) {
      const int e = tid + s * 256;
      As[e % KC][e / KC] = ra[s];
    }
#pragma unroll
    for (int s = 0; s < EB; ++s) {
      const int e = tid + s * 256;
      Bs[e / TN][e % TN] = rb[s];
    }
  };

  if (nchunks > 0) {
    load(0);
    store();
  }
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (int c = 0; c < nchunks; ++c) {
    if (c + 1 < nchunks) load(c + 1);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      T af[BM], bf[BN];
#pragma unroll
      for (int bi = 0; bi < BM; ++bi) af[bi] = As[kk + lk][wm + bi * 16 + lr];
#pragma unroll
      for (int bj = 0; bj < BN; ++bj) bf[bj] = Bs[kk + lk][wn + bj * 16 + lr];
#pragma unroll
      for (int bi = 0; bi < BM; ++bi)
#pragma unroll
        for (int bj = 0; bj < BN; ++bj) acc[bi][bj] = Mma<T>::mma(af[bi], bf[bj], acc[bi][bj]);
    }
    __syncthreads();
    if (c + 1 < nchunks) {
      store();
      __syncthreads();
    }
  }

  // Epilogue: output element (Mma<T>::row(lane/16, r), lane%16) of each
  // 16 x 16 block.
  const double shift = a.shifts ? a.shifts[vec] : 0.0;
  const T* Vp = a.V ? a.V + item * a.bstride : nullptr;
#pragma unroll
  for (int bi = 0; bi < BM; ++bi)
#pragma unroll
    for (int bj = 0; bj < BN; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + wm + bi * 16 + Mma<T>::row(lk, r);
        const int gj = j0 + wn + bj * 16 + lr;
        if (gi < M && gj < Nc) {
          const int64_t off = (int64_t)gi * rs + gj;
          T v = acc[bi][bj][r];
          if (a.epi == EPI_V) {
            T pot = (Vp ? Vp[off] : T(0)) - T(shift);
            v += pot * X[off];
          } else if (a.epi == EPI_DIV) {
            v = v / (a.lamL[gi] + a.lamR[gj] - T(a.sigma));
          }
          if (a.acc) v += Y[off];
          Y[off] = v;
        }
      }
}

template <typename T, int ROLE>
static void launch_role(const ModeProd<T>& a, int tile, hipStream_t s, unsigned g32, unsigned g64,
                        unsigned g128, unsigned g64x128) {
  switch (tile) {
    case TILE_32:
      hipLaunchKernelGGL((k_modeprod<T, 32, 32, 16, ROLE>), dim3(g32), dim3(256), 0, s, a);
      break;
    case TILE_64:
      hipLaunchKernelGGL((k_modeprod<T, 64, 64, 16, ROLE>), dim3(g64), dim3(256), 0, s, a);
      break;
    case TILE_128:
      hipLaunchKernelGGL((k_modeprod<T, 128, 128, 16, ROLE>), dim3(g128), dim3(256), 0, s, a);
      break;
    default:
      hipLaunchKernelGGL((k_modeprod<T, 64, 128, 16, ROLE>), dim3(g64x128), dim3(256), 0, s, a);
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
// FP32 data, products on the bf16 matrix cores: every operand element f is
// split as f = hi + lo + d with hi = bf16(f), lo = bf16(f - hi) (round to
// nearest, 8 significant bits each), so |lo| <= 2^-8 |f| and |d| <= 2^-16 |f|,
// and a*b is formed as hi_a hi_b + hi_a lo_b + lo_a hi_b with FP32 accumulation
// in v_mfma_f32_16x16x32_bf16.  The dropped terms (lo_a lo_b and those with d)
// are at most about 3 * 2^-16 |a b| per product, so the result carries roughly
// 16 significant bits, between bf16 and FP32.
// The split happens while a chunk is staged into LDS, so HBM traffic is that of
// the FP32 kernel.  LDS holds each operand as [row][k] with k contiguous so that
// a lane's 8 consecutive k values are one 16-byte read: the A operand of lane l
// is row l % 16, k = 8 (l / 16) + 0..7 and the B operand column l % 16 with the
// same k; the 16 x 16 FP32 result has the layout of the f32 instruction (row
// 4 (l / 16) + r in element r, column l % 16).
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split8(const float* f, bf8& hi, bf8& lo) {
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const __bf16 h = (__bf16)f[u];
    hi[u] = h;
    lo[u] = (__bf16)(f[u] - (float)h);
  }
}

// Eight consecutive floats p[0..7] of which the first `valid` exist; vector
// loads when the address is 16-byte aligned and all eight exist.
__device__ __forceinline__ void load8_row(const float* __restrict__ p, int valid, bool aligned,
                                          float* out) {
  if (aligned && valid >= 8) {
    const float4 u = *(const float4*)p;
    const float4 v = *(const float4*)(p + 4);
    out[0] = u.x; out[1] = u.y; out[2] = u.z; out[3] = u.w;
    out[4] = v.x; out[5] = v.y; out[6] = v.z; out[7] = v.w;
  } else {
#pragma unroll
    for (int u = 0; u < 8; ++u) out[u] = (u < valid) ? p[u] : 0.f;
  }
}

template <int TM, int TN, int KC, int ROLE>
__global__ __launch_bounds__(256) void k_modeprod_bf3(ModeProd<float> a) {
  constexpr int WM = TM / 2, WN = TN / 2;
  constexpr int BM = WM / 16, BN = WN / 16;
  constexpr int KG = KC / 8;                 // k octets per row
  constexpr int OA = TM * KG / 256;          // A octets per thread
  constexpr int OB = TN * KG / 256;          // B octets per thread
  constexpr int LDK = KC + 8;                // padded row (bf16 elements)
  static_assert(OA >= 1 && OB >= 1 && (TM * KG) % 256 == 0 && (TN * KG) % 256 == 0, "tile");
  static_assert(KC % 32 == 0, "K chunk is a multiple of the MFMA depth");
  __shared__ __attribute__((aligned(16))) __bf16 Ah[TM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Al[TM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[TN][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[TN][LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
  const int tiles_m = (a.M + TM - 1) / TM, tiles_n = (a.Nc + TN - 1) / TN;
  const int64_t tiles = (int64_t)tiles_m * tiles_n;
  const int64_t G = tiles * a.nbatch;
  const int64_t w = xcd_remap(blockIdx.x, G);
  const int64_t q = w / tiles;
  const int64_t t = w - q * tiles;
  const int i0 = (int)(t / tiles_n) * TM, j0 = (int)(t % tiles_n) * TN;
  const int64_t vec = q / a.per_vec, item = q - vec * a.per_vec;
  const float* __restrict__ X = a.X + vec * a.ldx + item * a.bstride;
  float* __restrict__ Y = a.Y + vec * a.ldy + item * a.bstride;
  const int64_t rs = a.rs;
  const int M = a.M, Nc = a.Nc;
  const bool alL = a.L && ((uintptr_t)a.L % 16 == 0) && (M % 4 == 0);
  const bool alX = ((uintptr_t)X % 16 == 0) && (rs % 4 == 0);

  f4 acc[BM][BN];
#pragma unroll
  for (int bi = 0; bi < BM; ++bi)
#pragma unroll
    for (int bj = 0; bj < BN; ++bj) acc[bi][bj] = f4{0, 0, 0, 0};

  const int nL = a.L ? (M + KC - 1) / KC : 0;
  const int nR = a.R ? (Nc + KC - 1) / KC : 0;
  const int nchunks = nL + nR;
  float ra[OA][8], rb[OB][8];

  auto load = [&](int c) {
    const bool left = c < nL;
    const int k0 = (left ? c : c - nL) * KC;
    const int K = left ? M : Nc;
#pragma unroll
    for (int s = 0; s < OA; ++s) {
      // A octet: row m, k = k0 + 8g .. +7, k contiguous in memory
      const int o = tid + s * 256, m = o / KG, g = o % KG;
      const int gi = i0 + m, gk = k0 + 8 * g;
      const int valid = (gi < M) ? min(8, K - gk) : 0;
      if (left)
        load8_row(a.L + (int64_t)gi * M + gk, valid, alL, ra[s]);
      else
        load8_row(X + (int64_t)gi * rs + gk, valid, alX, ra[s]);
    }
#pragma unroll
    for (int s = 0; s < OB; ++s) {
      // B octet: column n, k = k0 + 8g .. +7, read down a column (coalesced
      // across the lanes, which hold consecutive n)
      const int o = tid + s * 256, n = o % TN, g = o / TN;
      const int gj = j0 + n, gk = k0 + 8 * g;
      const bool cv = gj < Nc;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int kk = gk + u;
        const bool v = cv && kk < K;
        rb[s][u] = v ? (left ? X[(int64_t)kk * rs + gj] : a.R[(int64_t)kk * Nc + gj]) : 0.f;
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int s = 0; s < OA; ++s) {
      const int o = tid + s * 256, m = o / KG, g = o % KG;
      bf8 hi, lo;
      split8(ra[s], hi, lo);
      *(bf8*)&Ah[m][8 * g] = hi;
      *(bf8*)&Al[m][8 * g] = lo;
    }
#pragma unroll
    for (int s = 0; s < OB; ++s) {
      const int o = tid + s * 256, n = o % TN, g = o / TN;
      bf8 hi, lo;
      split8(rb[s], hi, lo);
      *(bf8*)&Bh[n][8 * g] = hi;
      *(bf8*)&Bl[n][8 * g] = lo;
    }
  };

  if (nchunks > 0) {
    load(0);
    store();
  }
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (int c = 0; c < nchunks; ++c) {
    if (c + 1 < nchunks) load(c + 1);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 32) {
      bf8 ah[BM], al[BM], bh[BN], bl[BN];
#pragma unroll
      for (int bi = 0; bi < BM; ++bi) {
        ah[bi] = *(const bf8*)&Ah[wm + bi * 16 + lr][kk + 8 * lk];
        al[bi] = *(const bf8*)&Al[wm + bi * 16 + lr][kk + 8 * lk];
      }
#pragma unroll
      for (int bj = 0; bj < BN; ++bj) {
        bh[bj] = *(const bf8*)&Bh[wn + bj * 16 + lr][kk + 8 * lk];
        bl[bj] = *(const bf8*)&Bl[wn + bj * 16 + lr][kk + 8 * lk];
      }
#pragma unroll
      for (int bi = 0; bi < BM; ++bi)
#pragma unroll
        for (int bj = 0; bj < BN; ++bj) {
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[bi], bh[bj], acc[bi][bj], 0, 0, 0);
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[bi], bl[bj], acc[bi][bj], 0, 0, 0);
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[bi], bh[bj], acc[bi][bj], 0, 0, 0);
        }
    }
    __syncthreads();
    if (c + 1 < nchunks) {
      store();
      __syncthreads();
    }
  }

  const double shift = a.shifts ? a.shifts[vec] : 0.0;
  const float* Vp = a.V ? a.V + item * a.bstride : nullptr;
#pragma unroll
  for (int bi = 0; bi < BM; ++bi)
#pragma unroll
    for (int bj = 0; bj < BN; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + wm + bi * 16 + 4 * lk + r;
        const int gj = j0 + wn + bj * 16 + lr;
        if (gi < M && gj < Nc) {
          const int64_t off = (int64_t)gi * rs + gj;
          float v = acc[bi][bj][r];
          if (a.epi == EPI_V) {
            const float pot = (Vp ? Vp[off] : 0.f) - (float)shift;
            v += pot * X[off];
          } else if (a.epi == EPI_DIV) {
            v = v / (a.lamL[gi] + a.lamR[gj] - (float)a.sigma);
          }
          if (a.acc) v += Y[off];
          Y[off] = v;
        }
      }
}

template <int ROLE>
static void launch_role_bf3(const ModeProd<float>& a, int tile, hipStream_t s, unsigned g64,
                            unsigned g128, unsigned g64x128) {
  switch (tile) {
    case TILE_128:
      hipLaunchKernelGGL((k_modeprod_bf3<128, 128, 32, ROLE>), dim3(g128), dim3(256), 0, s, a);
      break;
    case TILE_64x128:
      hipLaunchKernelGGL((k_modeprod_bf3<64, 128, 32, ROLE>), dim3(g64x128), dim3(256), 0, s, a);
      break;
    default:  // TILE_32 and TILE_64: the smallest bf16 tile is 64 x 64
      hipLaunchKernelGGL((k_modeprod_bf3<64, 64, 32, ROLE>), dim3(g64), dim3(256), 0, s, a);
      break;
  }
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
// Output tile per workgroup: 64 (p) x 32 (q); each of the 4 waves accumulates
// the full tile over its share of 16-row groups with FP64 MFMA, the waves are
// summed through LDS and the workgroup's partial goes to `partial`.
constexpr int DOT_TP = 64, DOT_TQ = 32, DOT_ROWS_MIN = 256;

static inline int dot_row_chunk(int64_t N) {
  int64_t rc = (N + 1023) / 1024;
  rc = ((rc + 63) / 64) * 64;
  if (rc < DOT_ROWS_MIN) rc = DOT_ROWS_MIN;
  return (int)rc;
}

int64_t dot_scratch_doubles(int64_t N, int p, int q) {
  int64_t nchunk = (N + dot_row_chunk(N) - 1) / dot_row_chunk(N);
  int64_t ntile = (int64_t)((p + DOT_TP - 1) / DOT_TP) * ((q + DOT_TQ - 1) / DOT_TQ);
  return nchunk * ntile * DOT_TP * DOT_TQ;
}

template <typename T>
__device__ __forceinline__ double ld_d(const T* p) {
  return (double)(*p);
}

template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_dot_tn(int64_t N, int p, int q, const TA* __restrict__ A,
                                                int64_t lda, const TB* __restrict__ B, int64_t ldb,
                                                int rchunk, int tiles_q, double* __restrict__ part) {
  __shared__ double red[DOT_TP * DOT_TQ];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int chunk = blockIdx.x, tile = blockIdx.y;
  const int p0 = (tile / tiles_q) * DOT_TP, q0 = (tile % tiles_q) * DOT_TQ;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t rbeg = (int64_t)chunk * rchunk;
  const int64_t rend = (rbeg + rchunk < N) ? rbeg + rchunk : N;
  d4 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0, 0, 0, 0};
  const TA* Ac[4];
  const TB* Bc[2];
  bool pa[4], pb[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int col = p0 + i * 16 + lr;
    pa[i] = col < p;
    Ac[i] = A + (int64_t)(pa[i] ? col : 0) * lda;
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int col = q0 + j * 16 + lr;
    pb[j] = col < q;
    Bc[j] = B + (int64_t)(pb[j] ? col : 0) * ldb;
  }
  for (int64_t g = rbeg + wave * 16; g < rend; g += 64) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t r = g + 4 * u + lk;
      const bool rv = r < rend;
      double av[4], bv[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = (rv && pa[i]) ? ld_d(Ac[i] + r) : 0.0;
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = (rv && pb[j]) ? ld_d(Bc[j] + r) : 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
  }
  // Sum the four waves' tiles in LDS, one wave at a time.
  for (int wv = 0; wv < 4; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int pi = i * 16 + Mma<double>::row(lk, r), qj = j * 16 + lr;
            const int idx = qj * DOT_TP + pi;
            red[idx] = (wv == 0) ? acc[i][j][r] : red[idx] + acc[i][j][r];
          }
    }
    __syncthreads();
  }
  double* out = part + ((int64_t)tile * gridDim.x + chunk) * (DOT_TP * DOT_TQ);
  for (int e = tid; e < DOT_TP * DOT_TQ; e += 256) out[e] = red[e];
}

// One wavefront per output element: lanes stride over the workgroup partials,
// then a shuffle reduction (fixed order, so the result is deterministic).
__global__ __launch_bounds__(256) void k_dot_reduce(int p, int q, int nchunk, int tiles_q,
                                                    const double* __restrict__ part,
                                                    double* __restrict__ C, int ldc) {
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);  // element within the tile
  const int tile = blockIdx.y;
  if (e >= DOT_TP * DOT_TQ) return;
  const int pi = e % DOT_TP, qj = e / DOT_TP;
  const int gp = (tile / tiles_q) * DOT_TP + pi, gq = (tile % tiles_q) * DOT_TQ + qj;
  if (gp >= p || gq >= q) return;
  const double* src = part + (int64_t)tile * nchunk * (DOT_TP * DOT_TQ) + e;
  double s = 0.0;
  for (int c = lane; c < nchunk; c += 64) s += src[(int64_t)c * (DOT_TP * DOT_TQ)];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) C[gp + (int64_t)gq * ldc] = s;
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
constexpr int GEMM_QB = 16, GEMM_PB = 128;

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_nn(int64_t N, int p, int q, double alpha,
                                                 const T* __restrict__ A, int64_t lda,
                                                 const double* __restrict__ C, int ldc,
                                                 double beta, T* __restrict__ Y, int64_t ldy) {
  __shared__ double Cs[GEMM_PB][GEMM_QB];
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int q0 = blockIdx.y * GEMM_QB;
  const int nq = (q - q0 < GEMM_QB) ? q - q0 : GEMM_QB;
  double acc[GEMM_QB];
#pragma unroll
  for (int j = 0; j < GEMM_QB; ++j) acc[j] = 0.0;
  for (int pb = 0; pb < p; pb += GEMM_PB) {
    const int np = (p - pb < GEMM_PB) ? p - pb : GEMM_PB;
    __syncthreads();
    for (int e = threadIdx.x; e < GEMM_PB * GEMM_QB; e += 256) {
      const int i = e / GEMM_QB, j = e % GEMM_QB;
      Cs[i][j] = (i < np && j < nq) ? C[(pb + i) + (int64_t)(q0 + j) * ldc] : 0.0;
    }
    __syncthreads();
    if (r < N) {
      for (int i = 0; i < np; ++i) {
        const double av = (double)A[r + (int64_t)(pb + i) * lda];
#pragma unroll
        for (int j = 0; j < GEMM_QB; ++j) acc[j] += av * Cs[i][j];
      }
    }
  }
  if (r < N) {
#pragma unroll
    for (int j = 0; j < GEMM_QB; ++j) {
      if (j < nq) {
        T* y = Y + r + (int64_t)(q0 + j) * ldy;
        const double old = (beta != 0.0) ? (double)(*y) : 0.0;
        *y = (T)(beta * old + alpha * acc[j]);
      }
    }
  }
}

template <typename T>
hipError_t launch_gemm_nn(int64_t N, int p, int q, double alpha, const T* A, int64_t lda,
                          const double* C, int ldc, double beta, T* Y, int64_t ldy,
                          hipStream_t s) {
  if (N <= 0 || q <= 0) return hipSuccess;
  dim3 grid((unsigned)((N + 255) / 256), (q + GEMM_QB - 1) / GEMM_QB);
  hipLaunchKernelGGL((k_gemm_nn<T>), grid, dim3(256), 0, s, N, p, q, alpha, A, lda, C, ldc, beta,
                     Y, ldy);
  return hipGetLastError();
}
template hipError_t launch_gemm_nn<double>(int64_t, int, int, double, const double*, int64_t,
                                           const double*, int, double, double*, int64_t,
                                           hipStream_t);
template hipError_t launch_gemm_nn<float>(int64_t, int, int, double, const float*, int64_t,
                                          const double*, int, double, float*, int64_t,
                                          hipStream_t);

// ------------------------------------------------ per-column (diagonal) dots
constexpr int BD_MAXNB = 40;

static inline int bdot_rows(int64_t N) {
  int64_t rc = (N + 255) / 256;
  rc = ((rc + 255) / 256) * 256;
  if (rc < 1024) rc = 1024;
  return (int)rc;
}
int64_t bdot_scratch_doubles(int64_t N, int b, int nb) {
  int64_t nchunk = (N + bdot_rows(N) - 1) / bdot_rows(N);
  return nchunk * b * BD_MAXNB;
}

template <typename T>
__global__ __launch_bounds__(256) void k_bdot_diag(int64_t N, int b, int nb, const T* __restrict__ V,
                                                   int64_t bs, const T* __restrict__ W, int rows,
                                                   double* __restrict__ part) {
  __shared__ double red[BD_MAXNB][4];
  const int j = blockIdx.y, chunk = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t rbeg = (int64_t)chunk * rows;
  const int64_t rend = (rbeg + rows < N) ? rbeg + rows : N;
  double acc[BD_MAXNB];
#pragma unroll
  for (int i = 0; i < BD_MAXNB; ++i) acc[i] = 0.0;
  const T* Wj = W + (int64_t)j * N;
  for (int64_t r = rbeg + tid; r < rend; r += 256) {
    const double w = (double)Wj[r];
#pragma unroll
    for (int i = 0; i < BD_MAXNB; ++i)
      if (i < nb) acc[i] += (double)V[(int64_t)i * bs + (int64_t)j * N + r] * w;
  }
#pragma unroll
  for (int i = 0; i < BD_MAXNB; ++i) {
    if (i < nb) {
      double v = acc[i];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) red[i][wave] = v;
    }
  }
  __syncthreads();
  if (tid < nb) {
    const double s = red[tid][0] + red[tid][1] + red[tid][2] + red[tid][3];
    part[((int64_t)chunk * b + j) * BD_MAXNB + tid] = s;
  }
}

__global__ __launch_bounds__(256) void k_bdot_reduce(int b, int nb, int nchunk,
                                                     const double* __restrict__ part,
                                                     double* __restrict__ H, int hld) {
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= b * nb) return;
  const int j = e / nb, i = e % nb;
  double s = 0.0;
  for (int c = lane; c < nchunk; c += 64) s += part[((int64_t)c * b + j) * BD_MAXNB + i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) H[(int64_t)j * hld + i] = s;
}

template <typename T>
hipError_t launch_bdot_diag(int64_t N, int b, int nb, const T* V, int64_t bs, const T* W,
                            double* H, int hld, double* partial, hipStream_t s) {
  if (nb <= 0 || b <= 0) return hipSuccess;
  if (nb > BD_MAXNB) return hipErrorInvalidValue;
  const int rows = bdot_rows(N);
  const int nchunk = (int)((N + rows - 1) / rows);
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

template <typename T>
__global__ __launch_bounds__(256) void k_bupdate_diag(int64_t N, int b, int nb, double alpha,
                                                      const T* __restrict__ V, int64_t bs,
                                                      const double* __restrict__ H, int hld,
                                                      T* __restrict__ W) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= N) return;
  double s = 0.0;
  for (int i = 0; i < nb; ++i) s += (double)V[(int64_t)i * bs + (int64_t)j * N + r] * H[(int64_t)j * hld + i];
  T* w = W + (int64_t)j * N + r;
  *w = (T)((double)(*w) + alpha * s);
}

template <typename T>
hipError_t launch_bupdate_diag(int64_t N, int b, int nb, double alpha, const T* V, int64_t bs,
                               const double* H, int hld, T* W, hipStream_t s) {
  if (N <= 0 || b <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_bupdate_diag<T>), dim3((unsigned)((N + 255) / 256), b), dim3(256), 0, s, N,
                     b, nb, alpha, V, bs, H, hld, W);
  return hipGetLastError();
}
template hipError_t launch_bupdate_diag<double>(int64_t, int, int, double, const double*, int64_t,
                                                const double*, int, double*, hipStream_t);
template hipError_t launch_bupdate_diag<float>(int64_t, int, int, double, const float*, int64_t,
                                               const double*, int, float*, hipStream_t);

template <typename T>
__global__ void k_normalize_cols(int64_t N, int b, const double* __restrict__ nrm2,
                                 const T* __restrict__ W, T* __restrict__ Vout,
                                 double* __restrict__ hout, int hld) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  const double n2 = nrm2[j];
  const double h = n2 > 0.0 ? sqrt(n2) : 0.0;
  if (r == 0 && hout) hout[(int64_t)j * hld] = h;
  if (r >= N) return;
  const double inv = h > 0.0 ? 1.0 / h : 0.0;
  Vout[(int64_t)j * N + r] = (T)((double)W[(int64_t)j * N + r] * inv);
}

template <typename T>
hipError_t launch_normalize_cols(int64_t N, int b, const double* nrm2, const T* W, T* Vout,
                                 double* hout, int hld, hipStream_t s) {
  if (b <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_normalize_cols<T>), dim3((unsigned)((N + 255) / 256 + (N == 0)), b),
                     dim3(256), 0, s, N, b, nrm2, W, Vout, hout, hld);
  return hipGetLastError();
}
template hipError_t launch_normalize_cols<double>(int64_t, int, const double*, const double*,
                                                  double*, double*, int, hipStream_t);
template hipError_t launch_normalize_cols<float>(int64_t, int, const double*, const float*, float*,
                                                 double*, int, hipStream_t);

// -------------------------------------------------------------- conversions
template <typename TI, typename TO>
__global__ void k_convert(int64_t N, double alpha, const TI* __restrict__ X, int64_t ldx,
                          TO* __restrict__ Y, int64_t ldy) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= N) return;
  Y[r + (int64_t)j * ldy] = (TO)(alpha * (double)X[r + (int64_t)j * ldx]);
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
__global__ void k_chol_small(int nx, const double* __restrict__ G, const double* __restrict__ n0,
                             double drop_tol, double* __restrict__ R, int* __restrict__ flags) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int j = 0; j < nx; ++j)
    for (int i = 0; i < nx; ++i) R[i + j * nx] = 0.0;
  for (int j = 0; j < nx; ++j) {
    double d = G[j + j * nx];
    for (int k = 0; k < j; ++k) d -= R[k + j * nx] * R[k + j * nx];
    const double thr = drop_tol * drop_tol * n0[j];
    if (!(d > thr) || !(d > 0.0)) {
      flags[j] = 1;
      R[j + j * nx] = 1.0;  // leave the column unscaled; it is replaced later
      continue;
    }
    flags[j] = 0;
    const double rjj = sqrt(d);
    R[j + j * nx] = rjj;
    for (int c = j + 1; c < nx; ++c) {
      double s = G[j + c * nx];
      for (int k = 0; k < j; ++k) s -= R[k + j * nx] * R[k + c * nx];
      R[j + c * nx] = s / rjj;
    }
  }
}

hipError_t launch_chol_small(int nx, const double* G, const double* norm0sq, double drop_tol,
                             double* R, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_small, dim3(1), dim3(64), 0, s, nx, G, norm0sq, drop_tol, R, flags);
  return hipGetLastError();
}

constexpr int TRSM_MAX = 32;
__global__ __launch_bounds__(256) void k_trsm_right(int64_t N, int nx, const double* __restrict__ R,
                                                    double* __restrict__ X, int64_t ldx) {
  __shared__ double Rs[TRSM_MAX * TRSM_MAX];
  for (int e = threadIdx.x; e < nx * nx; e += 256) Rs[e] = R[e];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= N) return;
  double x[TRSM_MAX];
#pragma unroll
  for (int j = 0; j < TRSM_MAX; ++j) x[j] = (j < nx) ? X[r + (int64_t)j * ldx] : 0.0;
#pragma unroll
  for (int j = 0; j < TRSM_MAX; ++j) {
    if (j < nx) {
      double s = x[j];
#pragma unroll
      for (int i = 0; i < TRSM_MAX; ++i)
        if (i < j) s -= x[i] * Rs[i + j * nx];
      x[j] = s / Rs[j + j * nx];
    }
  }
#pragma unroll
  for (int j = 0; j < TRSM_MAX; ++j)
    if (j < nx) X[r + (int64_t)j * ldx] = x[j];
}

hipError_t launch_trsm_right(int64_t N, int nx, const double* R, double* X, int64_t ldx,
                             hipStream_t s) {
  if (N <= 0) return hipSuccess;
  if (nx > TRSM_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_trsm_right, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, nx, R, X,
                     ldx);
  return hipGetLastError();
}

// SplitMix64 finaliser (Steele, Lea, Flood 2014) as a counter-based generator.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_hash_fill(int64_t N, double* __restrict__ X, uint64_t seed, uint64_t sid) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= N) return;
  const uint64_t h = mix64(seed ^ mix64(sid * 0x100000001B3ull + (uint64_t)r));
  X[r] = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
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

}  // namespace tp3b
