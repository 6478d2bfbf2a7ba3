// 2D (four-mode) Hamiltonian and kinetic-preconditioner passes on LDS-resident
// matrices (eqs. (8), (11); the preconditioner extends eq. (14) to four modes).
//
// A vector of the 2D problem is the tensor W[x1][x2][y1][y2].  The two y modes
// act on the contiguous planes W[x1][x2][:][:], the two x modes on the slabs
// W[:][:][j] at a fixed flattened y index j = (y1, y2), whose elements lie
// n_y1 n_y2 apart.  Both are at most 64 x 64 here (32 KB in FP64), so one
// workgroup keeps a group of J = 16 / sizeof(T) of them in LDS and runs every
// mode product of a pass on them without touching HBM in between:
//   Hamiltonian     pass 1 (x slabs): Y = K_x1 W + W K_x2^T
//                   pass 2 (y planes): Y = K_y1 W + W K_y2^T + (V - s) o W + Y
//   preconditioner  pass 1 (x slabs): Y = S_x1^{-1} W S_x2^{-T}
//                   pass 2 (y planes): Y = S_y1 ([S_y1^{-1} W S_y2^{-T}] / Lambda) S_y2^T
//                   pass 3 (x slabs): Y = S_x1 W S_x2^T
// (the mode operators of different modes commute, so the eigenbasis divide by
// Lambda = lam_x1 + lam_x2 + lam_y1 + lam_y2 - sigma can sit between the y
// transforms).  HBM traffic is one read and one write per pass (plus the read
// of the x part in the Hamiltonian's second pass), 40 B per entry for the FP64
// Hamiltonian instead of 72 B for three single-mode passes.
//
// The constant factors are read from global memory (L2-resident, 32 KB each in
// FP64) in MFMA fragment order, one coalesced 512-byte load per fragment.
// Work split: wave w of the 256-thread workgroup computes output row block w
// (rows 16w .. 16w + 15) of every matrix of the group; its accumulators hold
// 4 column blocks x J matrices.
#include <hip/hip_runtime.h>

#include "device_bodies.h"
#include "kernels.h"

namespace tp3b {

void plane2d_fragments(int n, const double* A, double* F) {
  for (int blk = 0; blk < 4; ++blk)
    for (int kk = 0; kk < 16; ++kk)
      for (int lane = 0; lane < 64; ++lane) {
        const int r = blk * 16 + lane % 16, k = 4 * kk + lane / 16;
        F[(blk * 16 + kk) * 64 + lane] = (r < n && k < n) ? A[(size_t)r * n + k] : 0.0;
      }
}

template <typename T>
struct P2Shape {
  static constexpr int J = 16 / (int)sizeof(T);  // matrices per workgroup
  static constexpr int LD = P2_MAXN + 1;         // padded LDS row
};

// acc[jj][bj] += A(row block w) * W_jj(:, column block bj)
template <typename T, bool FULL>
__device__ __forceinline__ void p2_left(typename Mma<T>::acc_t (&acc)[P2Shape<T>::J][4],
                                        const T* __restrict__ FA,
                                        T (&w)[P2Shape<T>::J][P2_MAXN][P2Shape<T>::LD], int wave,
                                        int lane, int KA, int BN) {
  constexpr int J = P2Shape<T>::J;
  const int lr = lane & 15, lk = lane >> 4;
  const T* fa = FA + (wave * 16) * 64 + lane;
  const int kend = FULL ? 16 : KA;
  T af_next = fa[0];
#pragma unroll 4
  for (int kk = 0; kk < kend; ++kk) {
    const T af = af_next;
    if (kk + 1 < kend) af_next = fa[(kk + 1) * 64];
#pragma unroll
    for (int jj = 0; jj < J; ++jj)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
        if (FULL || bj < BN) {
          const T bf = w[jj][4 * kk + lk][bj * 16 + lr];
          acc[jj][bj] = Mma<T>::mma(af, bf, acc[jj][bj]);
        }
  }
}

// acc[jj][bj] += W_jj(row block w, :) * B^T(:, column block bj)
template <typename T, bool FULL>
__device__ __forceinline__ void p2_right(typename Mma<T>::acc_t (&acc)[P2Shape<T>::J][4],
                                         const T* __restrict__ FB,
                                         T (&w)[P2Shape<T>::J][P2_MAXN][P2Shape<T>::LD], int wave,
                                         int lane, int KB, int BN) {
  constexpr int J = P2Shape<T>::J;
  const int lr = lane & 15, lk = lane >> 4;
  const int kend = FULL ? 16 : KB;
  T bn[4];
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) bn[bj] = (FULL || bj < BN) ? FB[(bj * 16) * 64 + lane] : T(0);
#pragma unroll 2
  for (int kk = 0; kk < kend; ++kk) {
    T bf[4];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) bf[bj] = bn[bj];
    if (kk + 1 < kend) {
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
        if (FULL || bj < BN) bn[bj] = FB[(bj * 16 + kk + 1) * 64 + lane];
    }
#pragma unroll
    for (int jj = 0; jj < J; ++jj) {
      const T af = w[jj][wave * 16 + lr][4 * kk + lk];
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
        if (FULL || bj < BN) acc[jj][bj] = Mma<T>::mma(af, bf[bj], acc[jj][bj]);
    }
  }
}

template <typename T>
__device__ __forceinline__ void p2_zero(typename Mma<T>::acc_t (&acc)[P2Shape<T>::J][4]) {
#pragma unroll
  for (int jj = 0; jj < P2Shape<T>::J; ++jj)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[jj][bj] = typename Mma<T>::acc_t{0, 0, 0, 0};
}

// Element (jj, r, c) of a group: matrix m0 + jj, row r, column c.
template <bool INTERLEAVED, int J>
__device__ __forceinline__ void p2_index(int e, int& jj, int& r, int& c) {
  if (INTERLEAVED) {
    jj = e % J;
    c = (e / J) % P2_MAXN;
    r = e / (J * P2_MAXN);
  } else {
    c = e % P2_MAXN;
    r = (e / P2_MAXN) % P2_MAXN;
    jj = e / (P2_MAXN * P2_MAXN);
  }
}

template <typename T, int PROG, bool INTERLEAVED, bool FULL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_plane2d(
    Plane2D<T> a) {
  constexpr int J = P2Shape<T>::J;
  constexpr int NE = J * P2_MAXN * P2_MAXN;  // elements of a group
  constexpr int UNR = 8;
  static_assert(NE % (256 * UNR) == 0, "group not divisible among the threads");
  __shared__ T w[J][P2_MAXN][P2Shape<T>::LD];
  typedef typename Mma<T>::acc_t acc_t;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t groups = (a.nmat + J - 1) / J;
  const int64_t item = xcd_remap(blockIdx.x, groups * a.nvec);
  const int64_t v = item / groups, m0 = (item - v * groups) * J;
  const int M = a.M, Nc = a.Nc;
  // no __restrict__: the preconditioner's second and third passes work in place
  // (each workgroup reads all of its matrices before it writes any of them)
  const T* X = a.X + v * a.ldx;
  T* Y = a.Y + v * a.ldy;

  // ---- load the group (zero outside M x Nc and past the last matrix)
  for (int e0 = tid; e0 < NE; e0 += 256 * UNR) {
    T val[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      int jj, r, c;
      p2_index<INTERLEAVED, J>(e0 + u * 256, jj, r, c);
      const int64_t m = m0 + jj;
      const bool ok = FULL ? (m < a.nmat) : (r < M && c < Nc && m < a.nmat);
      val[u] = ok ? X[m * a.js + r * a.rs + c * a.cs] : T(0);
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      int jj, r, c;
      p2_index<INTERLEAVED, J>(e0 + u * 256, jj, r, c);
      w[jj][r][c] = val[u];
    }
  }
  __syncthreads();

  const int BM = FULL ? 4 : (M + 15) / 16, BN = FULL ? 4 : (Nc + 15) / 16;
  const int KA = FULL ? 16 : (M + 3) / 4, KB = FULL ? 16 : (Nc + 3) / 4;
  const bool active = wave < BM;
  const int lr = lane & 15, lk = lane >> 4;
  acc_t acc[J][4];
  p2_zero<T>(acc);

  // accumulators -> LDS (optionally divided by the eigenvalue sums)
  auto to_lds = [&](bool divide) {
    __syncthreads();  // every wave has finished reading the previous contents
    if (active) {
#pragma unroll
      for (int jj = 0; jj < J; ++jj)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = wave * 16 + Mma<T>::row(lk, q), c = bj * 16 + lr;
            T val = acc[jj][bj][q];
            if (divide) {
              const int64_t m = m0 + jj;
              const bool ok = r < M && c < Nc && m < a.nmat;
              val = ok ? val / (a.lamM[m] + a.lamR[r] + a.lamC[c] - T(a.sigma)) : T(0);
            }
            w[jj][r][c] = val;
          }
    }
    __syncthreads();
  };

  if (PROG == P2_SUM || PROG == P2_SUM_V_ACC) {
    if (active) {
      p2_left<T, FULL>(acc, a.FA1, w, wave, lane, KA, BN);
      p2_right<T, FULL>(acc, a.FB1, w, wave, lane, KB, BN);
    }
  } else if (PROG == P2_SEQ2) {
    if (active) p2_left<T, FULL>(acc, a.FA1, w, wave, lane, KA, BN);
    to_lds(false);
    p2_zero<T>(acc);
    if (active) p2_right<T, FULL>(acc, a.FB1, w, wave, lane, KB, BN);
  } else {  // P2_SEQ4_DIV
    if (active) p2_left<T, FULL>(acc, a.FA1, w, wave, lane, KA, BN);
    to_lds(false);
    p2_zero<T>(acc);
    if (active) p2_right<T, FULL>(acc, a.FB1, w, wave, lane, KB, BN);
    to_lds(true);
    p2_zero<T>(acc);
    if (active) p2_left<T, FULL>(acc, a.FA2, w, wave, lane, KA, BN);
    to_lds(false);
    p2_zero<T>(acc);
    if (active) p2_right<T, FULL>(acc, a.FB2, w, wave, lane, KB, BN);
  }

  if (INTERLEAVED) {
    // stage the result through LDS so that the stores are as contiguous as the
    // loads (J consecutive y indices per (i1, i2))
    to_lds(false);
    for (int e0 = tid; e0 < NE; e0 += 256 * UNR) {
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        int jj, r, c;
        p2_index<INTERLEAVED, J>(e0 + u * 256, jj, r, c);
        const int64_t m = m0 + jj;
        const bool ok = FULL ? (m < a.nmat) : (r < M && c < Nc && m < a.nmat);
        if (ok) Y[m * a.js + r * a.rs + c * a.cs] = w[jj][r][c];
      }
    }
    return;
  }

  // planes: store from the accumulators (16 consecutive columns per lane group)
  if (!active) return;
  const double shift = (PROG == P2_SUM_V_ACC && a.shifts) ? a.shifts[v] : 0.0;
#pragma unroll
  for (int jj = 0; jj < J; ++jj) {
    const int64_t m = m0 + jj;
    if (m >= a.nmat) break;
    const int64_t base = m * a.js;
    const int i1 = (int)(m / (a.mdiv > 0 ? a.mdiv : 1)), i2 = (int)(m % (a.mdiv > 0 ? a.mdiv : 1));
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      const int c = bj * 16 + lr;
      if (!FULL && c >= Nc) continue;
      T g2m = T(0), g2p = T(0);
      if (PROG == P2_SUM_V_ACC && a.G) {
        g2m = a.G[2 * P2_MAXN * P2_MAXN + i2 * P2_MAXN + c];
        g2p = a.G[3 * P2_MAXN * P2_MAXN + i2 * P2_MAXN + c];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wave * 16 + Mma<T>::row(lk, q);
        if (!FULL && r >= M) continue;
        const int64_t off = base + r * a.rs + c;
        T val = acc[jj][bj][q];
        if (PROG == P2_SUM_V_ACC) {
          T pot;
          if (a.G) {
            pot = T(a.gscale) * (a.G[i1 * P2_MAXN + r] * g2m +
                                 a.G[P2_MAXN * P2_MAXN + i1 * P2_MAXN + r] * g2p);
          } else {
            pot = a.V ? a.V[off] : T(0);
          }
          val += (pot - T(shift)) * w[jj][r][c] + Y[off];
        }
        Y[off] = val;
      }
    }
  }
}

template <typename T, int PROG, bool INTERLEAVED>
static void launch_p2(const Plane2D<T>& a, bool full, unsigned grid, hipStream_t s) {
  if (full)
    hipLaunchKernelGGL((k_plane2d<T, PROG, INTERLEAVED, true>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_plane2d<T, PROG, INTERLEAVED, false>), dim3(grid), dim3(256), 0, s, a);
}

template <typename T>
hipError_t launch_plane2d(const Plane2D<T>& a, hipStream_t s) {
  if (a.nvec <= 0 || a.nmat <= 0) return hipSuccess;
  if (a.M < 1 || a.Nc < 1 || a.M > P2_MAXN || a.Nc > P2_MAXN) return hipErrorInvalidValue;
  if (!a.FA1 || !a.FB1 || (a.prog == P2_SEQ4_DIV && (!a.FA2 || !a.FB2))) return hipErrorInvalidValue;
  if (a.interleaved && a.js != 1) return hipErrorInvalidValue;
  if (!a.interleaved && a.cs != 1) return hipErrorInvalidValue;
  constexpr int J = P2Shape<T>::J;
  const int64_t groups = (a.nmat + J - 1) / J;
  const int64_t g = groups * a.nvec;
  if (g > 0x7fffffff) return hipErrorInvalidValue;
  const bool full = a.M == P2_MAXN && a.Nc == P2_MAXN;
  const unsigned grid = (unsigned)g;
  switch (a.prog) {
    case P2_SUM:
      if (a.interleaved) launch_p2<T, P2_SUM, true>(a, full, grid, s);
      else launch_p2<T, P2_SUM, false>(a, full, grid, s);
      break;
    case P2_SUM_V_ACC:
      if (a.interleaved) return hipErrorInvalidValue;
      launch_p2<T, P2_SUM_V_ACC, false>(a, full, grid, s);
      break;
    case P2_SEQ2:
      if (a.interleaved) launch_p2<T, P2_SEQ2, true>(a, full, grid, s);
      else launch_p2<T, P2_SEQ2, false>(a, full, grid, s);
      break;
    case P2_SEQ4_DIV:
      if (a.interleaved) return hipErrorInvalidValue;
      launch_p2<T, P2_SEQ4_DIV, false>(a, full, grid, s);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_plane2d<double>(const Plane2D<double>&, hipStream_t);
template hipError_t launch_plane2d<float>(const Plane2D<float>&, hipStream_t);

}  // namespace tp3b
