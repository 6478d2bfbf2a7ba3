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
//                   pass 2 (y planes): Y = [S_y1^{-1} W S_y2^{-T}] / Lambda
//                   pass 3 (y planes): Y = S_y1 W S_y2^T
//                   pass 4 (x slabs): Y = S_x1 W S_x2^T
// (the mode operators of different modes commute, so the eigenbasis divide by
// Lambda = lam_x1 + lam_x2 + lam_y1 + lam_y2 - sigma can sit between the y
// transforms).  HBM traffic is one read and one write per pass (plus the read
// of the x part in the Hamiltonian's second pass), 40 B per entry for the FP64
// Hamiltonian instead of 72 B for three single-mode passes, 64 B for the
// preconditioner instead of 128 B for eight.
//
// Every pass applies two constant n x n factors, held in LDS in MFMA fragment
// order (32 KB each in FP64) next to the work item (J matrices, 65 KB).  When
// the two modes of a pass have the same operator (equal n and L), one copy
// serves both products, and two more shapes use the LDS this frees:
// k_plane2d_x4 (FP64 x slabs, items of four matrices: 32-byte pieces) and
// k_plane2d_y1 (y planes, one plane per item, two workgroups per CU).
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
  static constexpr int J = 16 / (int)sizeof(T);  // matrices per work item
  static constexpr int JW = 1;                   // matrices per wave
  static constexpr int WB = J;                   // 16-column blocks per wave (FP64 2, FP32 4)
  static constexpr int LD = P2_MAXN + 1;         // padded LDS row
  static constexpr int NT = 1024;                // threads per workgroup (16 waves)
  static constexpr int CH = P2_MAXN * P2_MAXN;   // 16-byte chunks of J elements per item
  static constexpr int PER = CH / NT;            // chunks per thread
};

template <typename T>
using P2Buf = T[P2Shape<T>::J][P2_MAXN][P2Shape<T>::LD];
template <typename T>
using P2Acc = typename Mma<T>::acc_t[P2Shape<T>::JW][P2Shape<T>::WB];

// acc[j][b] += A(row block bi) * W_{j0 + j}(:, column block bj0 + b); A in
// fragment order in LDS
template <typename T, bool FULL>
__device__ __forceinline__ void p2_left(P2Acc<T>& acc, const T* FA, const P2Buf<T>& w, int j0,
                                        int bj0, int bi, int lane, int KA, int BN) {
  constexpr int JW = P2Shape<T>::JW, WB = P2Shape<T>::WB;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int kk = 0; kk < (FULL ? 16 : KA); ++kk) {
    const T af = FA[(bi * 16 + kk) * 64 + lane];
#pragma unroll
    for (int j = 0; j < JW; ++j)
#pragma unroll
      for (int b = 0; b < WB; ++b)
        if (FULL || bj0 + b < BN)
          acc[j][b] = Mma<T>::mma(af, w[j0 + j][4 * kk + lk][(bj0 + b) * 16 + lr], acc[j][b]);
  }
}

// acc[j][b] += W_{j0 + j}(row block bi, :) * B^T(:, column block bj0 + b)
template <typename T, bool FULL>
__device__ __forceinline__ void p2_right(P2Acc<T>& acc, const T* FB, const P2Buf<T>& w, int j0,
                                         int bj0, int bi, int lane, int KB, int BN) {
  constexpr int JW = P2Shape<T>::JW, WB = P2Shape<T>::WB;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int kk = 0; kk < (FULL ? 16 : KB); ++kk) {
    T a[JW];
#pragma unroll
    for (int j = 0; j < JW; ++j) a[j] = w[j0 + j][bi * 16 + lr][4 * kk + lk];
#pragma unroll
    for (int b = 0; b < WB; ++b)
      if (FULL || bj0 + b < BN) {
        const T bf = FB[((bj0 + b) * 16 + kk) * 64 + lane];
#pragma unroll
        for (int j = 0; j < JW; ++j) acc[j][b] = Mma<T>::mma(a[j], bf, acc[j][b]);
      }
  }
}

template <typename T>
__device__ __forceinline__ void p2_zero(P2Acc<T>& acc) {
#pragma unroll
  for (int j = 0; j < P2Shape<T>::JW; ++j)
#pragma unroll
    for (int b = 0; b < P2Shape<T>::WB; ++b) acc[j][b] = typename Mma<T>::acc_t{0, 0, 0, 0};
}

// Chunk q of a work item (J elements that are contiguous in memory):
//   interleaved (x slabs): position (r, c) = (q / 64, q % 64), element t is
//                          matrix m0 + t;
//   planes:                matrix jj = q / (64 * 64 / J), row r, columns
//                          c0 .. c0 + J - 1.
template <typename T, bool INTERLEAVED>
__device__ __forceinline__ void p2_chunk(int q, int& jj, int& r, int& c0) {
  constexpr int J = P2Shape<T>::J;
  if (INTERLEAVED) {
    jj = 0;
    r = q / P2_MAXN;
    c0 = q % P2_MAXN;
  } else {
    constexpr int CPR = P2_MAXN / J;  // chunks per row
    jj = q / (P2_MAXN * CPR);
    r = (q / CPR) % P2_MAXN;
    c0 = (q % CPR) * J;
  }
}

template <typename T>
struct P2Vec;
template <>
struct P2Vec<double> {
  typedef double2 v;
  static __device__ __forceinline__ double get(const v& x, int t) { return t == 0 ? x.x : x.y; }
  static __device__ __forceinline__ void set(v& x, int t, double e) {
    if (t == 0) x.x = e; else x.y = e;
  }
};
template <>
struct P2Vec<float> {
  typedef float4 v;
  static __device__ __forceinline__ float get(const v& x, int t) {
    return t == 0 ? x.x : (t == 1 ? x.y : (t == 2 ? x.z : x.w));
  }
  static __device__ __forceinline__ void set(v& x, int t, float e) {
    if (t == 0) x.x = e; else if (t == 1) x.y = e; else if (t == 2) x.z = e; else x.w = e;
  }
};

// Global offset of element t of chunk (jj, r, c0) of the item starting at
// matrix m0, and whether it exists.
template <typename T, bool INTERLEAVED, bool FULL>
__device__ __forceinline__ bool p2_elem(const Plane2D<T>& a, int64_t m0, int jj, int r, int c0, int t,
                                        int64_t& off) {
  int64_t m;
  int c;
  if (INTERLEAVED) {
    m = m0 + t;
    c = c0;
  } else {
    m = m0 + jj;
    c = c0 + t;
  }
  off = m * a.js + (int64_t)r * a.rs + (int64_t)c * a.cs;
  return FULL ? (m < a.nmat) : (m < a.nmat && r < a.M && c < a.Nc);
}

template <typename T, bool INTERLEAVED, bool FULL, bool VEC>
__device__ __forceinline__ void p2_fetch(const Plane2D<T>& a, const T* X, int64_t m0, int tid,
                                         typename P2Vec<T>::v (&buf)[P2Shape<T>::PER]) {
  constexpr int J = P2Shape<T>::J;
#pragma unroll
  for (int u = 0; u < P2Shape<T>::PER; ++u) {
    int jj, r, c0;
    p2_chunk<T, INTERLEAVED>(tid + u * P2Shape<T>::NT, jj, r, c0);
    int64_t off;
    const bool ok0 = p2_elem<T, INTERLEAVED, FULL>(a, m0, jj, r, c0, 0, off);
    if (VEC) {
      // the whole chunk exists when its first element does (checked on the host)
      if (ok0) {
        buf[u] = *(const typename P2Vec<T>::v*)(X + off);
      } else {
#pragma unroll
        for (int t = 0; t < J; ++t) P2Vec<T>::set(buf[u], t, T(0));
      }
    } else {
#pragma unroll
      for (int t = 0; t < J; ++t) {
        int64_t o;
        const bool ok = p2_elem<T, INTERLEAVED, FULL>(a, m0, jj, r, c0, t, o);
        P2Vec<T>::set(buf[u], t, ok ? X[o] : T(0));
      }
    }
  }
}

template <typename T, bool INTERLEAVED>
__device__ __forceinline__ void p2_put(P2Buf<T>& w, int tid,
                                       const typename P2Vec<T>::v (&buf)[P2Shape<T>::PER]) {
  constexpr int J = P2Shape<T>::J;
#pragma unroll
  for (int u = 0; u < P2Shape<T>::PER; ++u) {
    int jj, r, c0;
    p2_chunk<T, INTERLEAVED>(tid + u * P2Shape<T>::NT, jj, r, c0);
#pragma unroll
    for (int t = 0; t < J; ++t) {
      if (INTERLEAVED) w[t][r][c0] = P2Vec<T>::get(buf[u], t);
      else w[jj][r][c0 + t] = P2Vec<T>::get(buf[u], t);
    }
  }
}

// Work item t -> (vector, first matrix of the group).
template <int J>
__device__ __forceinline__ void p2_decode(int64_t t, int64_t groups, int64_t& v, int64_t& m0) {
  v = t / groups;
  m0 = (t - v * groups) * J;
}

// Schedule: in step k the grid processes the items k G .. k G + G - 1 (G =
// gridDim.x).  With G a multiple of 64, position i of a step belongs to
// workgroup (XCD x, slot l), i = (l / 8) 64 + 8 x + l % 8: eight consecutive
// items (one 128-byte line of the interleaved x-slab layout) go to eight
// workgroups of one XCD, which share the line in that XCD's L2, and the whole
// grid works on one contiguous range of items, so that the slab elements in
// flight at a tensor position are neighbours in memory (DRAM pages are reused
// instead of opened once per 16-byte piece).
__device__ __forceinline__ int64_t p2_slot(int g, int G) {
  if (G % 64 != 0) return g;
  const int x = g & 7, l = g >> 3;
  return (int64_t)((l >> 3) * 64 + x * 8 + (l & 7));
}

template <typename T, bool THIRD = false>
struct P2Smem {
  P2Buf<T> w;                 // the current work item
  T fa[P2_FRAG], fb[P2_FRAG];  // the two constant factors, fragment order
};
template <typename T>
struct P2Smem<T, true> {
  P2Buf<T> w;
  T fa[P2_FRAG], fb[P2_FRAG];
  T fc[P2_FRAG];  // P2_SEQ4_DIV: the back transform's factor (both sides)
};

// Persistent workgroups of 1024 threads (sixteen waves, four per SIMD), one
// per CU.  The two constant factors of the pass are copied to LDS once.  Work
// items are the groups of J matrices of every vector; the items of XCD
// x = blockIdx % 8 are the contiguous range [x T / 8, (x + 1) T / 8), taken in
// turn by that XCD's workgroups, so that neighbouring items (which share cache
// lines in the interleaved layout) run together on one L2.  While item i is
// multiplied out of LDS, item i + 1 is fetched into registers; it is stored
// into LDS once item i has been written out.  Wave w computes row block w % 4
// of one matrix, column blocks bj0 .. bj0 + WB - 1 (FP64: two per wave,
// FP32: all four).
template <typename T, int PROG, bool INTERLEAVED, bool FULL, bool VEC>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4))) void k_plane2d(
    Plane2D<T> a) {
  typedef P2Shape<T> S;
  constexpr int J = S::J, JW = S::JW, WB = S::WB;
  typedef typename P2Vec<T>::v vec_t;
  constexpr bool SEQ4 = PROG == P2_SEQ4_DIV;
  __shared__ P2Smem<T, SEQ4> sm;
  P2Buf<T>& w = sm.w;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NCB = 4 / WB;  // column-block groups per matrix
  const int bi = wave & 3, j0 = ((wave >> 2) / NCB) * JW, bj0 = ((wave >> 2) % NCB) * WB;
  const int lr = lane & 15, lk = lane >> 4;
  const int M = a.M, Nc = a.Nc;
  const int BM = FULL ? 4 : (M + 15) / 16, BN = FULL ? 4 : (Nc + 15) / 16;
  const int KA = FULL ? 16 : (M + 3) / 4, KB = FULL ? 16 : (Nc + 3) / 4;
  const bool active = bi < BM;

  const int64_t groups = (a.nmat + J - 1) / J;
  const int64_t total = groups * a.nvec;
  const int64_t G = gridDim.x, i0 = p2_slot(blockIdx.x, (int)G);

  for (int e = tid; e < P2_FRAG; e += S::NT) {
    sm.fa[e] = a.FA1[e];
    sm.fb[e] = a.FB1[e];
    if constexpr (SEQ4) sm.fc[e] = a.FA2[e];
  }
  // the divide's row and column eigenvalues of this lane's output elements
  // (the same for every item)
  constexpr bool DIV = PROG == P2_SEQ2_DIV || SEQ4;
  T lamr[4], lamc[WB];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = bi * 16 + Mma<T>::row(lk, q);
    lamr[q] = (DIV && r < M) ? a.lamR[r] : T(0);
  }
#pragma unroll
  for (int b = 0; b < WB; ++b) {
    const int c = (bj0 + b) * 16 + lr;
    lamc[b] = (DIV && c < Nc) ? a.lamC[c] : T(0);
  }
  vec_t pre[S::PER];
  int64_t item = i0;
  if (item < total) {
    int64_t v, m0;
    p2_decode<J>(item, groups, v, m0);
    p2_fetch<T, INTERLEAVED, FULL, VEC>(a, a.X + v * a.ldx, m0, tid, pre);
    p2_put<T, INTERLEAVED>(w, tid, pre);
  }
  __syncthreads();

  for (; item < total; item += G) {
    int64_t v, m0;
    p2_decode<J>(item, groups, v, m0);
    const int64_t nxt = item + G;
    T* Y = a.Y + v * a.ldy;
    // the epilogue's global operands, read before the products so that their
    // latency is hidden: the x part of the Hamiltonian (Y in place) and the
    // potential's separable factors.  They are issued before the next item's
    // fetch, so that waiting for them does not wait for the fetch as well (the
    // vector-memory counter drains in issue order).
    T tacc[JW][WB][4], g1[JW][2][4], g2[JW][2][WB];
    if (PROG == P2_SUM_V_ACC && active) {
#pragma unroll
      for (int j = 0; j < JW; ++j) {
        const int64_t m = m0 + j0 + j;
        const int md = a.mdiv > 0 ? a.mdiv : 1;
        const int i1 = (int)(m / md), i2 = (int)(m % md);
        const bool mok = m < a.nmat;
#pragma unroll
        for (int b = 0; b < WB; ++b)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = bi * 16 + Mma<T>::row(lk, q), c = (bj0 + b) * 16 + lr;
            const bool ok = mok && (FULL || (r < M && c < Nc));
            tacc[j][b][q] = ok ? Y[m * a.js + (int64_t)r * a.rs + c] : T(0);
          }
        if (a.G) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = bi * 16 + Mma<T>::row(lk, q);
            g1[j][0][q] = mok ? a.G[i1 * P2_MAXN + r] : T(0);
            g1[j][1][q] = mok ? a.G[P2_MAXN * P2_MAXN + i1 * P2_MAXN + r] : T(0);
          }
#pragma unroll
          for (int b = 0; b < WB; ++b) {
            const int c = (bj0 + b) * 16 + lr;
            g2[j][0][b] = mok ? a.G[2 * P2_MAXN * P2_MAXN + i2 * P2_MAXN + c] : T(0);
            g2[j][1][b] = mok ? a.G[3 * P2_MAXN * P2_MAXN + i2 * P2_MAXN + c] : T(0);
          }
        }
      }
    }
    if (nxt < total) {
      int64_t v2, m2;
      p2_decode<J>(nxt, groups, v2, m2);
      p2_fetch<T, INTERLEAVED, FULL, VEC>(a, a.X + v2 * a.ldx, m2, tid, pre);
    }
    P2Acc<T> acc;
    p2_zero<T>(acc);
    if (active) p2_left<T, FULL>(acc, sm.fa, w, j0, bj0, bi, lane, KA, BN);
    if (PROG == P2_SEQ2 || PROG == P2_SEQ2_DIV || SEQ4) {
      // A W -> LDS, then (A W) B^T
      __syncthreads();
      if (active) {
#pragma unroll
        for (int j = 0; j < JW; ++j)
#pragma unroll
          for (int b = 0; b < WB; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              w[j0 + j][bi * 16 + Mma<T>::row(lk, q)][(bj0 + b) * 16 + lr] = acc[j][b][q];
      }
      __syncthreads();
      p2_zero<T>(acc);
    }
    if (active) p2_right<T, FULL>(acc, sm.fb, w, j0, bj0, bi, lane, KB, BN);
    if constexpr (SEQ4) {
      // divide in the eigenbasis, then C Z C^T: Z -> LDS, C Z -> LDS, (C Z) C^T
      // (entries outside the M x Nc matrices or past the last matrix are set
      // to zero, so they add nothing to the back transform)
      if (active) {
#pragma unroll
        for (int j = 0; j < JW; ++j) {
          const int64_t m = m0 + j0 + j;
          const T lm = (m < a.nmat) ? a.lamM[m] - T(a.sigma) : T(0);
#pragma unroll
          for (int b = 0; b < WB; ++b) {
            const int c = (bj0 + b) * 16 + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int r = bi * 16 + Mma<T>::row(lk, q);
              const bool ok = m < a.nmat && (FULL || (r < M && c < Nc));
              acc[j][b][q] = ok ? acc[j][b][q] / (lm + lamr[q] + lamc[b]) : T(0);
            }
          }
        }
      }
      __syncthreads();
      if (active) {
#pragma unroll
        for (int j = 0; j < JW; ++j)
#pragma unroll
          for (int b = 0; b < WB; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              w[j0 + j][bi * 16 + Mma<T>::row(lk, q)][(bj0 + b) * 16 + lr] = acc[j][b][q];
      }
      __syncthreads();
      p2_zero<T>(acc);
      if (active) p2_left<T, FULL>(acc, sm.fc, w, j0, bj0, bi, lane, KA, BN);
      __syncthreads();
      if (active) {
#pragma unroll
        for (int j = 0; j < JW; ++j)
#pragma unroll
          for (int b = 0; b < WB; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              w[j0 + j][bi * 16 + Mma<T>::row(lk, q)][(bj0 + b) * 16 + lr] = acc[j][b][q];
      }
      __syncthreads();
      p2_zero<T>(acc);
      if (active) p2_right<T, FULL>(acc, sm.fc, w, j0, bj0, bi, lane, KB, BN);
    }

    // Results are formed in registers; the next item is put into LDS before
    // they are stored, so that waiting for its loads does not also wait for
    // this item's stores (the vector-memory counter covers both).
    vec_t outv[S::PER];
    if (INTERLEAVED) {
      // staged through LDS so that the stores are as contiguous as the loads
      // (J consecutive y indices per (i1, i2))
      __syncthreads();
      if (active) {
#pragma unroll
        for (int j = 0; j < JW; ++j)
#pragma unroll
          for (int b = 0; b < WB; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              w[j0 + j][bi * 16 + Mma<T>::row(lk, q)][(bj0 + b) * 16 + lr] = acc[j][b][q];
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < S::PER; ++u) {
        int jj, r, c0;
        p2_chunk<T, INTERLEAVED>(tid + u * S::NT, jj, r, c0);
#pragma unroll
        for (int t = 0; t < J; ++t) P2Vec<T>::set(outv[u], t, w[t][r][c0]);
      }
    } else if (active) {
      const double shift = (PROG == P2_SUM_V_ACC && a.shifts) ? a.shifts[v] : 0.0;
#pragma unroll
      for (int j = 0; j < JW; ++j) {
        const int64_t m = m0 + j0 + j;
        const T lm = (PROG == P2_SEQ2_DIV && m < a.nmat) ? a.lamM[m] - T(a.sigma) : T(0);
#pragma unroll
        for (int b = 0; b < WB; ++b) {
          const int c = (bj0 + b) * 16 + lr;
          const T lc = lamc[b];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = bi * 16 + Mma<T>::row(lk, q);
            if (PROG == P2_SUM_V_ACC) {
              const T pot = a.G ? T(a.gscale) * (g1[j][0][q] * g2[j][0][b] + g1[j][1][q] * g2[j][1][b])
                                : T(0);
              acc[j][b][q] += (pot - T(shift)) * w[j0 + j][r][c] + tacc[j][b][q];
            } else if (PROG == P2_SEQ2_DIV) {
              const bool ok = m < a.nmat && (FULL || (r < M && c < Nc));
              acc[j][b][q] = ok ? acc[j][b][q] / (lm + lamr[q] + lc) : T(0);
            }
          }
        }
      }
      if (PROG == P2_SUM_V_ACC && !a.G && a.V) {
        // potential from the table
#pragma unroll
        for (int j = 0; j < JW; ++j) {
          const int64_t m = m0 + j0 + j;
#pragma unroll
          for (int b = 0; b < WB; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int r = bi * 16 + Mma<T>::row(lk, q), c = (bj0 + b) * 16 + lr;
              const bool ok = m < a.nmat && (FULL || (r < M && c < Nc));
              if (ok) acc[j][b][q] += a.V[m * a.js + (int64_t)r * a.rs + c] * w[j0 + j][r][c];
            }
        }
      }
    }
    // the next item goes into LDS once every wave is done with this one
    __syncthreads();
    if (nxt < total) p2_put<T, INTERLEAVED>(w, tid, pre);
    if (INTERLEAVED) {
#pragma unroll
      for (int u = 0; u < S::PER; ++u) {
        int jj, r, c0;
        p2_chunk<T, INTERLEAVED>(tid + u * S::NT, jj, r, c0);
        int64_t off;
        const bool ok0 = p2_elem<T, INTERLEAVED, FULL>(a, m0, jj, r, c0, 0, off);
        if (VEC) {
          if (ok0) *(vec_t*)(Y + off) = outv[u];
        } else {
#pragma unroll
          for (int t = 0; t < J; ++t) {
            int64_t o2;
            if (p2_elem<T, INTERLEAVED, FULL>(a, m0, jj, r, c0, t, o2)) Y[o2] = P2Vec<T>::get(outv[u], t);
          }
        }
      }
    } else if (active) {
#pragma unroll
      for (int j = 0; j < JW; ++j) {
        const int64_t m = m0 + j0 + j;
        if (m >= a.nmat) break;
        const int64_t base = m * a.js;
#pragma unroll
        for (int b = 0; b < WB; ++b) {
          const int c = (bj0 + b) * 16 + lr;
          if (!FULL && c >= Nc) continue;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = bi * 16 + Mma<T>::row(lk, q);
            if (!FULL && r >= M) continue;
            Y[base + (int64_t)r * a.rs + c] = acc[j][b][q];
          }
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------
// FP64 x slabs with equal x modes: items of four matrices (32-byte pieces).
//
// The x-slab pass moves 16-byte pieces that lie 32 KB apart, and its speed is
// set by that access pattern rather than by the MFMA work.  When the two x
// modes have the same operator (equal n and L), one LDS copy of its fragments
// serves both products, which leaves room for items of four y indices
// (128 KB, unpadded): every position is then one 32-byte piece, read and
// written by two neighbouring lanes.  The LDS rows are swizzled so that every
// access of the pass is free of bank conflicts without padding: element (r, c)
// of matrix t sits at column c ^ p2x_swz(r, t), where bit 4 of the swizzle
// alternates with r (the two rows read together by one MFMA operand), its
// bits 1-3 are a permutation of the sixteen rows of a block (the sixteen rows
// read at one column), and bit 4 also flips between the matrix pairs (0, 1)
// and (2, 3) (the two halves of a piece, put by neighbouring lanes).
__device__ __forceinline__ int p2x_swz(int r, int t) {
  const int q = r & 15;
  return (((q & 1) << 4) | ((q >> 1) << 1)) ^ ((t >> 1) << 4);
}

typedef double P2XBuf[4][P2_MAXN][P2_MAXN];

__device__ __forceinline__ double& p2x_at(P2XBuf& w, int t, int r, int c) {
  return w[t][r][c ^ p2x_swz(r, t)];
}

// Chunks of an item: 8192 of 16 bytes, chunk g = tid + 1024 u at position
// p = g / 2 = (r, c) of the 64 x 64 slab, half h = g % 2 (matrices 2h and
// 2h + 1).  For thread tid: h = tid % 2, c = (tid / 2) % 64 and r = tid / 128
// + 8 u, so its chunks are u * 8 rows apart.
__device__ __forceinline__ int p2x_r0(int tid) { return tid >> 7; }
__device__ __forceinline__ int p2x_c(int tid) { return (tid >> 1) & 63; }

// Persistent workgroups of 1024 threads, one per CU, as k_plane2d; wave w
// computes row block w % 4 of matrix w / 4 for all four column blocks.
// Requires: full 64 x 64 slabs, js = 1, nmat % 4 == 0, 16-byte aligned vectors
// with ldx, ldy even, and FA1 the fragments of both factors.
template <int PROG>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4))) void k_plane2d_x4(
    Plane2D<double> a) {
  __shared__ P2XBuf w;
  __shared__ double f[P2_FRAG];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mat = wave >> 2, bi = wave & 3;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t groups = a.nmat / 4;
  const int64_t total = groups * a.nvec;
  const int64_t G = gridDim.x;
  constexpr int PER = 8;  // chunks per thread

  for (int e = tid; e < P2_FRAG; e += 1024) f[e] = a.FA1[e];

  const int h = tid & 1, r0 = p2x_r0(tid), c = p2x_c(tid);
  // this thread's offset inside an item, and the step between its chunks
  const int64_t toff = 2 * h + (int64_t)r0 * a.rs + (int64_t)c * a.cs, tstep = 8 * a.rs;
  double2 pre[PER];
  auto fetch = [&](int64_t item) {
    const int64_t v = item / groups, m0 = (item - v * groups) * 4;
    const double* X = a.X + v * a.ldx + m0 + toff;
#pragma unroll
    for (int u = 0; u < PER; ++u) pre[u] = *(const double2*)(X + u * tstep);
  };
  auto put = [&]() {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      p2x_at(w, 2 * h, r0 + 8 * u, c) = pre[u].x;
      p2x_at(w, 2 * h + 1, r0 + 8 * u, c) = pre[u].y;
    }
  };

  int64_t item = p2_slot(blockIdx.x, (int)G);
  if (item < total) {
    fetch(item);
    put();
  }
  __syncthreads();

  for (; item < total; item += G) {
    const int64_t nxt = item + G;
    if (nxt < total) fetch(nxt);
    d4 acc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = d4{0, 0, 0, 0};
    // A W
#pragma unroll 2
    for (int kk = 0; kk < 16; ++kk) {
      const double af = f[(bi * 16 + kk) * 64 + lane];
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[b] = Mma<double>::mma(af, p2x_at(w, mat, 4 * kk + lk, b * 16 + lr), acc[b]);
    }
    if (PROG == P2_SEQ2 || PROG == P2_SEQ4_DIV) {
      // A W -> LDS, then (A W) B^T
      __syncthreads();
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          p2x_at(w, mat, bi * 16 + Mma<double>::row(lk, q), b * 16 + lr) = acc[b][q];
      __syncthreads();
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[b] = d4{0, 0, 0, 0};
    }
    // (...) B^T
#pragma unroll 2
    for (int kk = 0; kk < 16; ++kk) {
      const double x = p2x_at(w, mat, bi * 16 + lr, 4 * kk + lk);
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[b] = Mma<double>::mma(x, f[(b * 16 + kk) * 64 + lane], acc[b]);
    }
    if (PROG == P2_SEQ4_DIV) {
      // divide in the eigenbasis, then the back transform C Z C^T with the
      // second factor in LDS (the first is loaded again with the next item)
      {
        const int64_t v = item / groups, mm = (item - v * groups) * 4 + mat;
        const double ly = a.lamM[mm] - a.sigma;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const double lc = a.lamC[b * 16 + lr] + ly;
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[b][q] = acc[b][q] / (a.lamR[bi * 16 + Mma<double>::row(lk, q)] + lc);
        }
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          p2x_at(w, mat, bi * 16 + Mma<double>::row(lk, q), b * 16 + lr) = acc[b][q];
      for (int e = tid; e < P2_FRAG; e += 1024) f[e] = a.FA2[e];
      __syncthreads();
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[b] = d4{0, 0, 0, 0};
#pragma unroll 2
      for (int kk = 0; kk < 16; ++kk) {
        const double af = f[(bi * 16 + kk) * 64 + lane];
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = Mma<double>::mma(af, p2x_at(w, mat, 4 * kk + lk, b * 16 + lr), acc[b]);
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          p2x_at(w, mat, bi * 16 + Mma<double>::row(lk, q), b * 16 + lr) = acc[b][q];
      __syncthreads();
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[b] = d4{0, 0, 0, 0};
#pragma unroll 2
      for (int kk = 0; kk < 16; ++kk) {
        const double x = p2x_at(w, mat, bi * 16 + lr, 4 * kk + lk);
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = Mma<double>::mma(x, f[(b * 16 + kk) * 64 + lane], acc[b]);
      }
    }
    // results staged through LDS, then stored as 32-byte pieces; the stores
    // are issued after the next item's loads, and the put below waits only
    // for those (the vector-memory counter drains in issue order)
    __syncthreads();
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) p2x_at(w, mat, bi * 16 + Mma<double>::row(lk, q), b * 16 + lr) = acc[b][q];
    __syncthreads();
    {
      const int64_t v = item / groups, m0 = (item - v * groups) * 4;
      double* Y = a.Y + v * a.ldy + m0 + toff;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        double2 o;
        o.x = p2x_at(w, 2 * h, r0 + 8 * u, c);
        o.y = p2x_at(w, 2 * h + 1, r0 + 8 * u, c);
        *(double2*)(Y + u * tstep) = o;
      }
    }
    __syncthreads();
    if (nxt < total) put();
    if (PROG == P2_SEQ4_DIV && nxt < total)
      for (int e = tid; e < P2_FRAG; e += 1024) f[e] = a.FA1[e];
    __syncthreads();
  }
}

// ------------------------------------------------------------------------
// y planes with equal y modes: one plane per item, two workgroups per CU.
//
// With one workgroup per CU the MFMA pipes idle while a workgroup waits for
// its barrier, its next item's loads and its stores.  When the two y modes
// have the same operator one LDS copy of its fragments serves both products,
// and a workgroup that holds one plane (padded, 33 KB) and that copy (32 KB)
// leaves room for a second workgroup on the CU, whose products fill those
// gaps.  Eight waves per workgroup; wave w computes row block w % 4 and the
// column blocks 2 (w / 4), 2 (w / 4) + 1 of the plane.  Requires full,
// contiguous 64 x 64 planes (rs = 64, cs = 1), js a multiple of
// 16 / sizeof(T), 16-byte aligned vectors with ld a multiple of 16 / sizeof(T),
// and FA1 the fragments of both factors.
template <typename T>
struct P2Y {
  static constexpr int E = 16 / (int)sizeof(T);     // elements per 16-byte chunk
  static constexpr int NT = 512;
  static constexpr int PER = P2_MAXN * P2_MAXN / E / NT;  // chunks per thread
  static constexpr int LD = P2_MAXN + 1;
};

template <typename T, int PROG>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_plane2d_y1(
    Plane2D<T> a) {
  typedef P2Y<T> S;
  typedef typename P2Vec<T>::v vec_t;
  typedef typename Mma<T>::acc_t acc_t;
  constexpr int E = S::E, CPR = P2_MAXN / E;
  __shared__ T w[P2_MAXN][S::LD];
  __shared__ T f[P2_FRAG];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bi = wave & 3, bj0 = (wave >> 2) * 2;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t total = a.nmat * a.nvec;
  const int64_t G = gridDim.x;

  for (int e = tid; e < P2_FRAG; e += S::NT) f[e] = a.FA1[e];
  T lamr[4], lamc[2];
#pragma unroll
  for (int q = 0; q < 4; ++q) lamr[q] = (PROG == P2_SEQ2_DIV) ? a.lamR[bi * 16 + Mma<T>::row(lk, q)] : T(0);
#pragma unroll
  for (int b = 0; b < 2; ++b) lamc[b] = (PROG == P2_SEQ2_DIV) ? a.lamC[(bj0 + b) * 16 + lr] : T(0);

  vec_t pre[S::PER];
  auto fetch = [&](int64_t item) {
    const int64_t v = item / a.nmat, m = item - v * a.nmat;
    const T* X = a.X + v * a.ldx + m * a.js;
    // rows are contiguous (rs = 64), so chunk q starts at element E q
#pragma unroll
    for (int u = 0; u < S::PER; ++u) pre[u] = *(const vec_t*)(X + E * (tid + u * S::NT));
  };
  auto put = [&]() {
#pragma unroll
    for (int u = 0; u < S::PER; ++u) {
      const int q = tid + u * S::NT, r = q / CPR, c0 = (q % CPR) * E;
#pragma unroll
      for (int t = 0; t < E; ++t) w[r][c0 + t] = P2Vec<T>::get(pre[u], t);
    }
  };

  int64_t item = p2_slot(blockIdx.x, (int)G);
  if (item < total) {
    fetch(item);
    put();
  }
  __syncthreads();

  for (; item < total; item += G) {
    const int64_t v = item / a.nmat, m = item - v * a.nmat;
    const int64_t nxt = item + G;
    T* Y = a.Y + v * a.ldy + m * a.js;
    // this lane's output elements: Yl[(4 q) * 64 + 16 b]
    T* Yl = Y + (bi * 16 + lk) * P2_MAXN + bj0 * 16 + lr;
    // the epilogue's global operands first (their wait does not include the
    // next item's loads, which are issued after them)
    T tacc[2][4];
    if (PROG == P2_SUM_V_ACC) {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          tacc[b][q] = Yl[(Mma<T>::row(lk, q) - lk) * P2_MAXN + b * 16];
    }
    if (nxt < total) fetch(nxt);
    acc_t acc[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[b] = acc_t{0, 0, 0, 0};
    // A W
#pragma unroll 2
    for (int kk = 0; kk < 16; ++kk) {
      const T af = f[(bi * 16 + kk) * 64 + lane];
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[b] = Mma<T>::mma(af, w[4 * kk + lk][(bj0 + b) * 16 + lr], acc[b]);
    }
    if (PROG == P2_SEQ2 || PROG == P2_SEQ2_DIV) {
      __syncthreads();
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) w[bi * 16 + Mma<T>::row(lk, q)][(bj0 + b) * 16 + lr] = acc[b][q];
      __syncthreads();
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[b] = acc_t{0, 0, 0, 0};
    }
    // (...) B^T
#pragma unroll 2
    for (int kk = 0; kk < 16; ++kk) {
      const T x = w[bi * 16 + lr][4 * kk + lk];
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[b] = Mma<T>::mma(x, f[((bj0 + b) * 16 + kk) * 64 + lane], acc[b]);
    }
    // epilogue (the potential's factor tables are small and stay in the L2;
    // they are read here rather than with the x part, which keeps the
    // registers of the products below the bound for two workgroups per CU)
    if (PROG == P2_SUM_V_ACC) {
      const double shift = a.shifts ? a.shifts[v] : 0.0;
      T g1[2][4], g2[2][2];
      if (a.G) {
        const int md = a.mdiv > 0 ? a.mdiv : 1;
        const int i1 = (int)(m / md), i2 = (int)(m % md);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = bi * 16 + Mma<T>::row(lk, q);
          g1[0][q] = a.G[i1 * P2_MAXN + r];
          g1[1][q] = a.G[P2_MAXN * P2_MAXN + i1 * P2_MAXN + r];
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int c = (bj0 + b) * 16 + lr;
          g2[0][b] = a.G[2 * P2_MAXN * P2_MAXN + i2 * P2_MAXN + c];
          g2[1][b] = a.G[3 * P2_MAXN * P2_MAXN + i2 * P2_MAXN + c];
        }
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int c = (bj0 + b) * 16 + lr;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = bi * 16 + Mma<T>::row(lk, q);
          const T pot = a.G ? T(a.gscale) * (g1[0][q] * g2[0][b] + g1[1][q] * g2[1][b]) : T(0);
          acc[b][q] += (pot - T(shift)) * w[r][c] + tacc[b][q];
        }
      }
      if (!a.G && a.V) {
        // potential from the table
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = bi * 16 + Mma<T>::row(lk, q), c = (bj0 + b) * 16 + lr;
            acc[b][q] += a.V[m * a.js + r * P2_MAXN + c] * w[r][c];
          }
      }
    } else if (PROG == P2_SEQ2_DIV) {
      const T lm = a.lamM[m] - T(a.sigma);
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[b][q] = acc[b][q] / (lm + lamr[q] + lamc[b]);
    }
    // the next item goes into LDS once every wave is done with this one, and
    // before this item's stores are issued
    __syncthreads();
    if (nxt < total) put();
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        Yl[(Mma<T>::row(lk, q) - lk) * P2_MAXN + b * 16] = acc[b][q];
    __syncthreads();
  }
}

// Two workgroups per CU.
constexpr int P2Y_GRID = 512;

template <typename T, int PROG, bool INTERLEAVED>
static void launch_p2(const Plane2D<T>& a, bool full, bool vec, unsigned grid, hipStream_t s) {
  if (full && vec)
    hipLaunchKernelGGL((k_plane2d<T, PROG, INTERLEAVED, true, true>), dim3(grid), dim3(1024), 0, s, a);
  else if (full)
    hipLaunchKernelGGL((k_plane2d<T, PROG, INTERLEAVED, true, false>), dim3(grid), dim3(1024), 0, s, a);
  else
    hipLaunchKernelGGL((k_plane2d<T, PROG, INTERLEAVED, false, false>), dim3(grid), dim3(1024), 0, s, a);
}

// Persistent grid: one workgroup per CU (the LDS holds up to 130 KB).
constexpr int P2_GRID = 256;

template <typename T>
hipError_t launch_plane2d(const Plane2D<T>& a, hipStream_t s) {
  if (a.nvec <= 0 || a.nmat <= 0) return hipSuccess;
  if (a.M < 1 || a.Nc < 1 || a.M > P2_MAXN || a.Nc > P2_MAXN) return hipErrorInvalidValue;
  if (!a.FA1 || !a.FB1) return hipErrorInvalidValue;
  if (a.interleaved && (a.js != 1 || a.prog == P2_SUM_V_ACC || a.prog == P2_SEQ2_DIV))
    return hipErrorInvalidValue;
  if (!a.interleaved && a.cs != 1) return hipErrorInvalidValue;
  if ((a.prog == P2_SEQ2_DIV || a.prog == P2_SEQ4_DIV) && (!a.lamM || !a.lamR || !a.lamC))
    return hipErrorInvalidValue;
  if (a.prog == P2_SEQ4_DIV && !a.FA2) return hipErrorInvalidValue;
  constexpr int J = P2Shape<T>::J;
  const int64_t groups = (a.nmat + J - 1) / J;
  const int64_t items = groups * a.nvec;
  const bool full = a.M == P2_MAXN && a.Nc == P2_MAXN;
  // 16-byte chunks: every chunk starts at a multiple of J elements of a
  // 16-byte aligned vector and either exists whole or not at all
  const bool aligned = ((uintptr_t)a.X % 16 == 0) && ((uintptr_t)a.Y % 16 == 0) &&
                       a.ldx % J == 0 && a.ldy % J == 0;
  const bool vec = full && aligned &&
                   (a.interleaved ? (a.nmat % J == 0 && a.rs % J == 0 && a.cs % J == 0)
                                  : (a.js % J == 0 && a.rs % J == 0));
  Plane2D<T> b = a;
  const unsigned grid = (unsigned)(items < P2_GRID ? items : P2_GRID);
  if constexpr (sizeof(T) == 8) {
    // equal x modes: items of four matrices (32-byte pieces)
    const bool x4 = a.interleaved && full && vec && a.same_ab && a.nmat % 4 == 0 && a.ldx % 2 == 0 &&
                    a.ldy % 2 == 0 &&
                    (a.prog == P2_SUM || a.prog == P2_SEQ2 || a.prog == P2_SEQ4_DIV);
    if (x4) {
      const int64_t items4 = (a.nmat / 4) * a.nvec;
      const unsigned grid4 = (unsigned)(items4 < P2_GRID ? items4 : P2_GRID);
      if (a.prog == P2_SUM)
        hipLaunchKernelGGL((k_plane2d_x4<P2_SUM>), dim3(grid4), dim3(1024), 0, s, b);
      else if (a.prog == P2_SEQ2)
        hipLaunchKernelGGL((k_plane2d_x4<P2_SEQ2>), dim3(grid4), dim3(1024), 0, s, b);
      else
        hipLaunchKernelGGL((k_plane2d_x4<P2_SEQ4_DIV>), dim3(grid4), dim3(1024), 0, s, b);
      return hipGetLastError();
    }
  }
  // the four-product program: x slabs with equal x modes (one factor per half)
  if (a.prog == P2_SEQ4_DIV) {
    // FP64 runs it in the four-matrix kernel above (the generic one has no LDS
    // left for the third factor in FP64)
    if (sizeof(T) != 4 || !a.interleaved || !a.same_ab) return hipErrorInvalidValue;
    if constexpr (sizeof(T) == 4) launch_p2<T, P2_SEQ4_DIV, true>(b, full, vec, grid, s);
    return hipGetLastError();
  }
  // equal y modes: one plane per item, two workgroups per CU
  const bool y1 = !a.interleaved && full && vec && a.same_ab && a.cs == 1 && a.rs == P2_MAXN &&
                  (a.prog == P2_SUM_V_ACC || a.prog == P2_SEQ2 || a.prog == P2_SEQ2_DIV);
  if (y1) {
    const int64_t items1 = a.nmat * a.nvec;
    const unsigned grid1 = (unsigned)(items1 < P2Y_GRID ? items1 : P2Y_GRID);
    if (a.prog == P2_SUM_V_ACC)
      hipLaunchKernelGGL((k_plane2d_y1<T, P2_SUM_V_ACC>), dim3(grid1), dim3(512), 0, s, b);
    else if (a.prog == P2_SEQ2)
      hipLaunchKernelGGL((k_plane2d_y1<T, P2_SEQ2>), dim3(grid1), dim3(512), 0, s, b);
    else
      hipLaunchKernelGGL((k_plane2d_y1<T, P2_SEQ2_DIV>), dim3(grid1), dim3(512), 0, s, b);
    return hipGetLastError();
  }
  switch (a.prog) {
    case P2_SUM:
      if (a.interleaved) launch_p2<T, P2_SUM, true>(b, full, vec, grid, s);
      else launch_p2<T, P2_SUM, false>(b, full, vec, grid, s);
      break;
    case P2_SUM_V_ACC:
      launch_p2<T, P2_SUM_V_ACC, false>(b, full, vec, grid, s);
      break;
    case P2_SEQ2:
      if (a.interleaved) launch_p2<T, P2_SEQ2, true>(b, full, vec, grid, s);
      else launch_p2<T, P2_SEQ2, false>(b, full, vec, grid, s);
      break;
    case P2_SEQ2_DIV:
      launch_p2<T, P2_SEQ2_DIV, false>(b, full, vec, grid, s);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_plane2d<double>(const Plane2D<double>&, hipStream_t);
template hipError_t launch_plane2d<float>(const Plane2D<float>&, hipStream_t);

}  // namespace tp3b
