// Device code shared by the single-job kernels (kernels.hip) and the grouped,
// persistent kernels (grouped.hip): every kernel body is a __device__ function
// that computes one work item (a tile, a row block, a reduction target) from
// explicit indices, so that both launch forms run the same arithmetic.
// Included by HIP translation units only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

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
// Output tile TM x TN per 256-thread workgroup (4 wave64s in 2 x 2), K chunks of
// KC staged through padded LDS with a register prefetch of the next chunk; both
// products of a 1D apply (L X and X R) run in one K loop of length M + Nc, so no
// intermediate goes to memory.
// SK (split K): every wave computes the whole tile over its own quarter of each
// K chunk (independent accumulators per 16 x 16 block instead of one dependent
// chain), and the four partial tiles are summed through LDS at the end; used for
// small tiles, whose runtime is the latency of the K loop.
// NW waves per workgroup (4 in 2 x 2 without split K; 4 or 8 with it).  The
// split-K partial tiles reuse the LDS of the operand chunks, which are dead by
// the time the partials are written.
template <typename T, int TM, int TN, int KC, bool SK = false, int NW = 4>
struct MpSmem {
  union {
    struct {
      T As[KC][TM + 1];
      T Bs[KC][TN + 1];
    } ab;
    T red[SK ? NW * TM * TN : 1];
  };
};

// Work items of one mode product: output tiles x batch items.
template <int TM, int TN, typename P>
__host__ __device__ inline int64_t modeprod_items(const P& a) {
  return (int64_t)((a.M + TM - 1) / TM) * ((a.Nc + TN - 1) / TN) * a.nbatch;
}

// One TM x TN output tile (work item w) of the mode product `a`.
template <typename T, int TM, int TN, int KC, bool SK = false, int NW = 4>
__device__ __forceinline__ void modeprod_tile(const ModeProd<T>& a, int64_t w,
                                              MpSmem<T, TM, TN, KC, SK, NW>& sm) {
  typedef typename Mma<T>::acc_t acc_t;
  constexpr int NT = 64 * NW;  // threads per workgroup
  constexpr int WM = SK ? TM : TM / 2, WN = SK ? TN : TN / 2;
  constexpr int BM = WM / 16, BN = WN / 16;
  constexpr int EA = TM * KC / NT, EB = KC * TN / NT;
  constexpr int KW = SK ? KC / NW : KC;  // K range of one wave within a chunk
  static_assert(SK || NW == 4, "without split K the four waves form a 2 x 2 grid");
  static_assert(EA >= 1 && EB >= 1 && EA * NT == TM * KC && EB * NT == KC * TN,
                "chunk not divisible among the threads");
  static_assert(KW % 4 == 0, "a wave's K range is a multiple of the MFMA depth");
  T(&As)[KC][TM + 1] = sm.ab.As;
  T(&Bs)[KC][TN + 1] = sm.ab.Bs;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = SK ? 0 : (wave >> 1) * WM, wn = SK ? 0 : (wave & 1) * WN;
  const int kw0 = SK ? wave * KW : 0;
  const int tiles_m = (a.M + TM - 1) / TM, tiles_n = (a.Nc + TN - 1) / TN;
  const int64_t tiles = (int64_t)tiles_m * tiles_n;
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
        const int e = tid + s * NT, m = e / KC, k = e % KC;
        const int gi = i0 + m, gk = k0 + k;
        ra[s] = (gi < M && gk < M) ? a.L[(int64_t)gi * M + gk] : T(0);
      }
#pragma unroll
      for (int s = 0; s < EB; ++s) {
        const int e = tid + s * NT, k = e / TN, n = e % TN;
        const int gk = k0 + k, gj = j0 + n;
        rb[s] = (gk < M && gj < Nc) ? X[(int64_t)gk * rs + gj] : T(0);
      }
    } else {
      const int k0 = (c - nL) * KC;
#pragma unroll
      for (int s = 0; s < EA; ++s) {
        const int e = tid + s * NT, m = e / KC, k = e % KC;
        const int gi = i0 + m, gk = k0 + k;
        ra[s] = (gi < M && gk < Nc) ? X[(int64_t)gi * rs + gk] : T(0);
      }
#pragma unroll
      for (int s = 0; s < EB; ++s) {
        const int e = tid + s * NT, k = e / TN, n = e % TN;
        const int gk = k0 + k, gj = j0 + n;
        rb[s] = (gk < Nc && gj < Nc) ? a.R[(int64_t)gk * Nc + gj] : T(0);
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int s = 0; s < EA; ++s) {
      const int e = tid + s * NT;
      As[e % KC][e / KC] = ra[s];
    }
#pragma unroll
    for (int s = 0; s < EB; ++s) {
      const int e = tid + s * NT;
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
    for (int kk = kw0; kk < kw0 + KW; kk += 4) {
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
  auto emit = [&](int gi, int gj, T v) {
    if (gi < M && gj < Nc) {
      const int64_t off = (int64_t)gi * rs + gj;
      if (a.epi == EPI_V) {
        T pot = (Vp ? Vp[off] : T(0)) - T(shift);
        v += pot * X[off];
      } else if (a.epi == EPI_DIV) {
        v = v / (a.lamL[gi] + a.lamR[gj] + (a.lamItem ? a.lamItem[item] : T(0)) - T(a.sigma));
      }
      if (a.acc) v += Y[off];
      Y[off] = v;
    }
  };
  if constexpr (SK) {
    // sum the waves' partial tiles (fixed order: deterministic); the operand
    // chunks are dead here (the K loop ends with a barrier)
    T* red = sm.red;
#pragma unroll
    for (int bi = 0; bi < BM; ++bi)
#pragma unroll
      for (int bj = 0; bj < BN; ++bj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ri = bi * 16 + Mma<T>::row(lk, r), cj = bj * 16 + lr;
          red[(wave * TM + ri) * TN + cj] = acc[bi][bj][r];
        }
    __syncthreads();
    for (int e = tid; e < TM * TN; e += NT) {
      T v = red[e];
#pragma unroll
      for (int w2 = 1; w2 < NW; ++w2) v += red[w2 * TM * TN + e];
      emit(i0 + e / TN, j0 + e % TN, v);
    }
    __syncthreads();  // `red` is reused by the next work item of a persistent loop
  } else {
#pragma unroll
    for (int bi = 0; bi < BM; ++bi)
#pragma unroll
      for (int bj = 0; bj < BN; ++bj)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          emit(i0 + wm + bi * 16 + Mma<T>::row(lk, r), j0 + wn + bj * 16 + lr, acc[bi][bj][r]);
  }
}

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

template <int TM, int TN, int KC>
struct Bf3Smem {
  static constexpr int LDK = KC + 8;  // padded row (bf16 elements)
  __attribute__((aligned(16))) __bf16 Ah[TM][LDK];
  __attribute__((aligned(16))) __bf16 Al[TM][LDK];
  __attribute__((aligned(16))) __bf16 Bh[TN][LDK];
  __attribute__((aligned(16))) __bf16 Bl[TN][LDK];
};

template <int TM, int TN, int KC>
__device__ __forceinline__ void modeprod_bf3_tile(const ModeProd<float>& a, int64_t w,
                                                  Bf3Smem<TM, TN, KC>& sm) {
  constexpr int WM = TM / 2, WN = TN / 2;
  constexpr int BM = WM / 16, BN = WN / 16;
  constexpr int KG = KC / 8;                 // k octets per row
  constexpr int OA = TM * KG / 256;          // A octets per thread
  constexpr int OB = TN * KG / 256;          // B octets per thread
  constexpr int LDK = KC + 8;                // padded row (bf16 elements)
  static_assert(OA >= 1 && OB >= 1 && (TM * KG) % 256 == 0 && (TN * KG) % 256 == 0, "tile");
  static_assert(KC % 32 == 0, "K chunk is a multiple of the MFMA depth");
  __bf16(&Ah)[TM][LDK] = sm.Ah;
  __bf16(&Al)[TM][LDK] = sm.Al;
  __bf16(&Bh)[TN][LDK] = sm.Bh;
  __bf16(&Bl)[TN][LDK] = sm.Bl;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
  const int tiles_m = (a.M + TM - 1) / TM, tiles_n = (a.Nc + TN - 1) / TN;
  const int64_t tiles = (int64_t)tiles_m * tiles_n;
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

  // constant operands split once (a.Lhl, a.Rhl: hi block then lo block of
  // raw bf16 bits) are read as 16 bytes of hi and 16 of lo per octet into the
  // same registers and staged without a split; rows or columns past the
  // matrix read its last one and are staged as zeros
  const uint16_t* Lhl = a.L ? a.Lhl : nullptr;
  const uint16_t* Rhl = a.R ? a.Rhl : nullptr;
  auto load_hl = [&](const uint16_t* base, int64_t nn, int64_t off, float* out) {
    const f4 h = *(const f4*)(base + off);
    const f4 l = *(const f4*)(base + nn + off);
    out[0] = h[0]; out[1] = h[1]; out[2] = h[2]; out[3] = h[3];
    out[4] = l[0]; out[5] = l[1]; out[6] = l[2]; out[7] = l[3];
  };
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
      if (left && Lhl)
        load_hl(Lhl, (int64_t)M * M, (int64_t)(gi < M ? gi : M - 1) * M + gk, ra[s]);
      else if (left)
        load8_row(a.L + (int64_t)gi * M + gk, valid, alL, ra[s]);
      else
        load8_row(X + (int64_t)gi * rs + gk, valid, alX, ra[s]);
    }
    // B octets of a pre-split right operand go to lanes as the A octets do
    // (consecutive lanes, consecutive octets of one row of R^T); split ones
    // to consecutive columns, read down the column
    const bool preB = !left && Rhl;
#pragma unroll
    for (int s = 0; s < OB; ++s) {
      // B octet: column n, k = k0 + 8g .. +7
      const int o = tid + s * 256, n = preB ? o / KG : o % TN, g = preB ? o % KG : o / TN;
      const int gj = j0 + n, gk = k0 + 8 * g;
      const bool cv = gj < Nc;
      if (preB) {
        load_hl(Rhl, (int64_t)Nc * Nc, (int64_t)(cv ? gj : Nc - 1) * Nc + gk, rb[s]);
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int kk = gk + u;
          const bool v = cv && kk < K;
          rb[s][u] = v ? (left ? X[(int64_t)kk * rs + gj] : a.R[(int64_t)kk * Nc + gj]) : 0.f;
        }
      }
    }
  };
  // stage the chunk loaded for chunk c
  auto store = [&](int c) {
    const bool left = c < nL;
#pragma unroll
    for (int s = 0; s < OA; ++s) {
      const int o = tid + s * 256, m = o / KG, g = o % KG;
      bf8 hi, lo;
      if (left && Lhl) {
        const bool in = i0 + m < M;
        const f4 h = {ra[s][0], ra[s][1], ra[s][2], ra[s][3]};
        const f4 l = {ra[s][4], ra[s][5], ra[s][6], ra[s][7]};
        hi = in ? __builtin_bit_cast(bf8, h) : bf8{};
        lo = in ? __builtin_bit_cast(bf8, l) : bf8{};
      } else {
        split8(ra[s], hi, lo);
      }
      *(bf8*)&Ah[m][8 * g] = hi;
      *(bf8*)&Al[m][8 * g] = lo;
    }
    const bool preB = !left && Rhl;
#pragma unroll
    for (int s = 0; s < OB; ++s) {
      const int o = tid + s * 256, n = preB ? o / KG : o % TN, g = preB ? o % KG : o / TN;
      bf8 hi, lo;
      if (preB) {
        const bool in = j0 + n < Nc;
        const f4 h = {rb[s][0], rb[s][1], rb[s][2], rb[s][3]};
        const f4 l = {rb[s][4], rb[s][5], rb[s][6], rb[s][7]};
        hi = in ? __builtin_bit_cast(bf8, h) : bf8{};
        lo = in ? __builtin_bit_cast(bf8, l) : bf8{};
      } else {
        split8(rb[s], hi, lo);
      }
      *(bf8*)&Bh[n][8 * g] = hi;
      *(bf8*)&Bl[n][8 * g] = lo;
    }
  };

  if (nchunks > 0) {
    load(0);
    store(0);
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
      store(c + 1);
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
            v = v / (a.lamL[gi] + a.lamR[gj] + (a.lamItem ? a.lamItem[item] : 0.f) - (float)a.sigma);
          }
          if (a.acc) v += Y[off];
          Y[off] = v;
        }
      }
}

// ---------------------------------------------------------------- block dot
// C = A^T B: output tile 64 (p) x 32 (q) per workgroup; each of the 4 waves
// accumulates the whole tile over its share of 16-row groups of a row chunk
// with FP64 MFMA, the waves are summed through LDS, and the workgroup's partial
// tile goes to `out` (64 x 32, column-major).  A second stage sums the chunks.
constexpr int DOT_TP = 64, DOT_TQ = 32, DOT_ROWS_MIN = 256;

__host__ __device__ inline int dot_row_chunk(int64_t N) {
  int64_t rc = (N + 1023) / 1024;
  rc = ((rc + 63) / 64) * 64;
  if (rc < DOT_ROWS_MIN) rc = DOT_ROWS_MIN;
  return (int)rc;
}
// Grouped dots run many small products side by side, so each job takes fewer,
// longer chunks (at most 64 per job, at least 4096 rows each).
__host__ __device__ inline int dot_row_chunk_grouped(int64_t N) {
  int64_t rc = (N + 63) / 64;
  rc = ((rc + 63) / 64) * 64;
  if (rc < 4096) rc = 4096;
  return (int)rc;
}

template <typename T>
__device__ __forceinline__ double ld_d(const T* p) {
  return (double)(*p);
}

// Four consecutive elements p[0..3] as doubles with 16-byte vector loads
// (p must be 16-byte aligned: 32-byte groups for double, 16 for float).
__device__ __forceinline__ void ld4_d(const double* p, double* out) {
  const double2 u = *(const double2*)p;
  const double2 v = *(const double2*)(p + 2);
  out[0] = u.x; out[1] = u.y; out[2] = v.x; out[3] = v.y;
}
__device__ __forceinline__ void ld4_d(const float* p, double* out) {
  const float4 u = *(const float4*)p;
  out[0] = u.x; out[1] = u.y; out[2] = u.z; out[3] = u.w;
}

struct DotSmem {
  double red[DOT_TP * DOT_TQ];
};

template <typename TA, typename TB>
__device__ __forceinline__ void dot_tile(int64_t N, int p, int q, const TA* __restrict__ A,
                                         int64_t lda, const TB* __restrict__ B, int64_t ldb,
                                         int rchunk, int tiles_q, int chunk, int tile,
                                         double* __restrict__ out, DotSmem& sm) {
  double* red = sm.red;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
  // Each wave takes groups of 16 rows; lane group lk owns rows g + 4 lk .. + 3
  // of its column and feeds row g + 4 lk + u into K slot lk of the u-th
  // instruction (A and B use the same assignment, so the sum is A^T B), which
  // makes a lane's four rows one contiguous vector load when the columns are
  // 16-byte aligned and the group lies inside the chunk.
  const bool vec_ok = (((uintptr_t)A | (uintptr_t)B) % 16 == 0) && (lda % 4 == 0) &&
                      (ldb % 4 == 0) && (rbeg % 16 == 0);
  auto load = [&](int64_t g, double (&av)[4][4], double (&bv)[2][4]) {
    const int64_t r0 = g + 4 * lk;
    if (vec_ok && g + 16 <= rend) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (pa[i]) {
          ld4_d(Ac[i] + r0, av[i]);
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u) av[i][u] = 0.0;
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (pb[j]) {
          ld4_d(Bc[j] + r0, bv[j]);
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u) bv[j][u] = 0.0;
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t r = r0 + u;
        const bool rv = r < rend;
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i][u] = (rv && pa[i]) ? ld_d(Ac[i] + r) : 0.0;
#pragma unroll
        for (int j = 0; j < 2; ++j) bv[j][u] = (rv && pb[j]) ? ld_d(Bc[j] + r) : 0.0;
      }
    }
  };
  // 16 x 16 blocks that lie wholly outside p x q are skipped (a branch that is
  // the same for the whole wave): with the q <= 8 columns of a typical
  // projection most of the tile is padding, and an FP64 MFMA costs as much as
  // the vector FMAs it replaces.  The stored entries are unchanged.
  bool ua[4], ub[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) ua[i] = p0 + i * 16 < p;
#pragma unroll
  for (int j = 0; j < 2; ++j) ub[j] = q0 + j * 16 < q;
  auto mul = [&](const double (&av)[4][4], const double (&bv)[2][4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          if (ua[i] && ub[j])
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][u], bv[j][u], acc[i][j], 0, 0, 0);
  };
  // The next 64-row group is fetched while the current one is multiplied (two
  // register sets, the loop unrolled by two so that no copy waits early).
  double a0[4][4], b0[2][4], a1[4][4], b1[2][4];
  int64_t g = rbeg + wave * 16;
  if (g < rend) load(g, a0, b0);
  for (; g < rend; g += 128) {
    if (g + 64 < rend) load(g + 64, a1, b1);
    mul(a0, b0);
    if (g + 64 < rend) {
      if (g + 128 < rend) load(g + 128, a0, b0);
      mul(a1, b1);
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
  // Only the entries inside p x q are stored (the reduction reads no others).
  const int pv = p - p0, qv = q - q0;
  for (int e = tid; e < DOT_TP * DOT_TQ; e += 256)
    if (e % DOT_TP < pv && e / DOT_TP < qv) out[e] = red[e];
  __syncthreads();  // `red` is reused by the next work item of a persistent loop
}

// Second stage for one output element (gp, gq): the calling wavefront's lanes
// stride over the chunk partials (chunk c of tile t at part[(t*nchunk + c)*64*32]),
// then a fixed-order shuffle reduction; lane 0 holds the result.
__device__ __forceinline__ double dot_reduce_elem(int gp, int gq, int nchunk, int tiles_q,
                                                  const double* __restrict__ part, int lane) {
  const int tile = (gp / DOT_TP) * tiles_q + gq / DOT_TQ;
  const int e = (gq % DOT_TQ) * DOT_TP + gp % DOT_TP;
  const double* src = part + (int64_t)tile * nchunk * (DOT_TP * DOT_TQ) + e;
  double s = 0.0;
  for (int c = lane; c < nchunk; c += 64) s += src[(int64_t)c * (DOT_TP * DOT_TQ)];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  return s;
}

// ------------------------------------------------------------ basis update
// Y (a block of rows, columns q0..q0+15) = beta Y + alpha A C (or, with X0,
// beta X0 + alpha A C, X0 not aliasing Y), one row per lane, in one of two forms:
//  * SPLIT (64 rows per workgroup): the four waves split the p range into
//    quarters and sum their partial rows in LDS in wave order.  For a single
//    short block of vectors that puts four times as many workgroups and loads
//    in flight as one row per thread over all of p would.
//  * otherwise (256 rows per workgroup): each thread runs over all of p.  The
//    persistent grouped launch uses this form: its items are then 4x fewer,
//    and each item pays the job lookup and the staging of C only once.
constexpr int GEMM_QB = 16, GEMM_PB = 128;
template <bool SPLIT>
constexpr int gemm_rows() { return SPLIT ? 64 : 256; }

template <bool SPLIT>
struct GemmSmem {
  union {
    double Cs[GEMM_PB][GEMM_QB];                 // a chunk of C
    double red[SPLIT ? 4 : 1][64][GEMM_QB + 1];  // the waves' partial rows
  };
};

template <typename T, bool SPLIT>
__device__ __forceinline__ void gemm_block(int64_t N, int p, int q, double alpha,
                                           const T* __restrict__ A, int64_t lda,
                                           const double* __restrict__ C, int ldc, double beta,
                                           T* __restrict__ Y, int64_t ldy, int64_t rblock,
                                           int qblock, GemmSmem<SPLIT>& sm,
                                           const T* __restrict__ X0 = nullptr, int64_t ldx0 = 0) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r = rblock * gemm_rows<SPLIT>() + (SPLIT ? lane : (int)threadIdx.x);
  const int q0 = qblock * GEMM_QB;
  const int nq = (q - q0 < GEMM_QB) ? q - q0 : GEMM_QB;
  double acc[GEMM_QB];
#pragma unroll
  for (int j = 0; j < GEMM_QB; ++j) acc[j] = 0.0;
  for (int pb = 0; pb < p; pb += GEMM_PB) {
    const int np = (p - pb < GEMM_PB) ? p - pb : GEMM_PB;
    __syncthreads();
    for (int e = threadIdx.x; e < GEMM_PB * GEMM_QB; e += 256) {
      const int i = e / GEMM_QB, j = e % GEMM_QB;
      sm.Cs[i][j] = (i < np && j < nq) ? C[(pb + i) + (int64_t)(q0 + j) * ldc] : 0.0;
    }
    __syncthreads();
    const int per = SPLIT ? (np + 3) / 4 : np;
    const int ib = SPLIT ? ((wave * per < np) ? wave * per : np) : 0;
    const int ie = (ib + per < np) ? ib + per : np;
    if (r < N) {
      // eight columns of A per step, fetched before they are used
      for (int i0 = ib; i0 < ie; i0 += 8) {
        double av[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          av[u] = (i0 + u < ie) ? (double)A[r + (int64_t)(pb + i0 + u) * lda] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (i0 + u < ie) {
#pragma unroll
            for (int j = 0; j < GEMM_QB; ++j) acc[j] += av[u] * sm.Cs[i0 + u][j];
          }
        }
      }
    }
  }
  if constexpr (SPLIT) {
    __syncthreads();  // the last chunk of C is dead
#pragma unroll
    for (int j = 0; j < GEMM_QB; ++j) sm.red[wave][lane][j] = acc[j];
    __syncthreads();
    if (r < N) {
      // wave w finishes columns 4w .. 4w+3 of the lane's row
#pragma unroll
      for (int jj = 0; jj < GEMM_QB / 4; ++jj) {
        const int j = wave * (GEMM_QB / 4) + jj;
        if (j < nq) {
          const double v = sm.red[0][lane][j] + sm.red[1][lane][j] + sm.red[2][lane][j] + sm.red[3][lane][j];
          T* y = Y + r + (int64_t)(q0 + j) * ldy;
          const double old = (beta != 0.0) ? (double)(X0 ? X0[r + (int64_t)(q0 + j) * ldx0] : *y) : 0.0;
          *y = (T)(beta * old + alpha * v);
        }
      }
    }
  } else if (r < N) {
#pragma unroll
    for (int j = 0; j < GEMM_QB; ++j) {
      if (j < nq) {
        T* y = Y + r + (int64_t)(q0 + j) * ldy;
        const double old = (beta != 0.0) ? (double)(X0 ? X0[r + (int64_t)(q0 + j) * ldx0] : *y) : 0.0;
        *y = (T)(beta * old + alpha * acc[j]);
      }
    }
  }
  __syncthreads();  // the LDS is reused by the next work item of a persistent loop
}

// ------------------------------------------------ per-column (diagonal) dots
// b independent Krylov bases stored as blocks Vb[i] = V + i*bs (each N x b, ld
// N): the partial of column j over one row chunk, for i < nb, goes to
// out[0..nb).
constexpr int BD_MAXNB = 40;

__host__ __device__ inline int bdot_rows(int64_t N) {
  int64_t rc = (N + 255) / 256;
  rc = ((rc + 255) / 256) * 256;
  if (rc < 1024) rc = 1024;
  return (int)rc;
}

struct BdotSmem {
  double red[BD_MAXNB][4];
};

template <typename T>
__device__ __forceinline__ void bdot_chunk(int64_t N, int nb, const T* __restrict__ V, int64_t bs,
                                           const T* __restrict__ W, int rows, int chunk, int j,
                                           double* __restrict__ out, BdotSmem& sm) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t rbeg = (int64_t)chunk * rows;
  const int64_t rend = (rbeg + rows < N) ? rbeg + rows : N;
  double acc[BD_MAXNB];
#pragma unroll
  for (int i = 0; i < BD_MAXNB; ++i) acc[i] = 0.0;
  const T* Wj = W + (int64_t)j * N;
  // four rows per thread and step, all their loads issued before the
  // products (each accumulator still adds the thread's rows in row order)
  for (int64_t r = rbeg + tid; r < rend; r += 1024) {
    double w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = (r + 256 * q < rend) ? (double)Wj[r + 256 * q] : 0.0;
#pragma unroll
    for (int i = 0; i < BD_MAXNB; ++i) {
      if (i < nb) {
        const T* Vi = V + (int64_t)i * bs + (int64_t)j * N + r;
        double v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (r + 256 * q < rend) ? (double)Vi[256 * q] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (r + 256 * q < rend) acc[i] += v[q] * w[q];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < BD_MAXNB; ++i) {
    if (i < nb) {
      double v = acc[i];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) sm.red[i][wave] = v;
    }
  }
  __syncthreads();
  if (tid < nb) out[tid] = sm.red[tid][0] + sm.red[tid][1] + sm.red[tid][2] + sm.red[tid][3];
  __syncthreads();  // `red` is reused by the next work item of a persistent loop
}

// Sum of entry i over nchunk partials part[(c*b + j)*BD_MAXNB + i] (one wave).
__device__ __forceinline__ double bdot_reduce_elem(int b, int j, int i, int nchunk,
                                                   const double* __restrict__ part, int lane) {
  double s = 0.0;
  for (int c = lane; c < nchunk; c += 64) s += part[((int64_t)c * b + j) * BD_MAXNB + i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  return s;
}

// W[r, j] += alpha * sum_{i<nb} Vb[i][r, j] H[j*hld + i]
template <typename T>
__device__ __forceinline__ void bupdate_row(int64_t N, int nb, double alpha,
                                            const T* __restrict__ V, int64_t bs,
                                            const double* __restrict__ H, int hld,
                                            T* __restrict__ W, int64_t r, int j) {
  if (r >= N) return;
  double s = 0.0;
  // eight basis vectors per step, fetched before they are used; an exactly
  // zero coefficient (past a GMRES breakdown) contributes nothing, whatever the
  // basis vector holds
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
      if (h[u] != 0.0) s += v[u] * h[u];
  }
  T* w = W + (int64_t)j * N + r;
  *w = (T)((double)(*w) + alpha * s);
}

// Vout[r, j] = W[r, j] / sqrt(n2) (n2 = the squared norm of column j); row 0
// also stores the norm in hout.
template <typename T>
__device__ __forceinline__ void normalize_row_n2(int64_t N, double n2, const T* __restrict__ W,
                                                 T* __restrict__ Vout, double* __restrict__ hout,
                                                 int hld, int64_t r, int j) {
  const double h = n2 > 0.0 ? sqrt(n2) : 0.0;
  if (r == 0 && hout) hout[(int64_t)j * hld] = h;
  if (r >= N) return;
  const double inv = h > 0.0 ? 1.0 / h : 0.0;
  Vout[(int64_t)j * N + r] = (T)((double)W[(int64_t)j * N + r] * inv);
}
template <typename T>
__device__ __forceinline__ void normalize_row(int64_t N, const double* __restrict__ nrm2,
                                              const T* __restrict__ W, T* __restrict__ Vout,
                                              double* __restrict__ hout, int hld, int64_t r,
                                              int j) {
  normalize_row_n2<T>(N, nrm2[j], W, Vout, hout, hld, r, j);
}

// -------------------------------------------------------- Cholesky-QR pieces
// Cholesky of the nx x nx Gram matrix (column-major) by one thread; a pivot
// below (drop_tol^2 * n0[j]) marks column j as dependent.
__device__ inline void chol_small_serial(int nx, const double* __restrict__ G,
                                         const double* __restrict__ n0, double drop_tol,
                                         double* __restrict__ R, int* __restrict__ flags) {
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

constexpr int TRSM_MAX = 32;
struct TrsmSmem {
  double Rs[TRSM_MAX * TRSM_MAX];
};

// Row block of X (N x nx) <- X R^{-1}, R upper triangular (column-major).
__device__ __forceinline__ void trsm_block(int64_t N, int nx, const double* __restrict__ R,
                                           double* __restrict__ X, int64_t ldx, int64_t rblock,
                                           TrsmSmem& sm) {
  for (int e = threadIdx.x; e < nx * nx; e += 256) sm.Rs[e] = R[e];
  __syncthreads();
  const int64_t r = rblock * 256 + threadIdx.x;
  if (r < N) {
    double x[TRSM_MAX];
#pragma unroll
    for (int j = 0; j < TRSM_MAX; ++j) x[j] = (j < nx) ? X[r + (int64_t)j * ldx] : 0.0;
#pragma unroll
    for (int j = 0; j < TRSM_MAX; ++j) {
      if (j < nx) {
        double s = x[j];
#pragma unroll
        for (int i = 0; i < TRSM_MAX; ++i)
          if (i < j) s -= x[i] * sm.Rs[i + j * nx];
        x[j] = s / sm.Rs[j + j * nx];
      }
    }
#pragma unroll
    for (int j = 0; j < TRSM_MAX; ++j)
      if (j < nx) X[r + (int64_t)j * ldx] = x[j];
  }
  __syncthreads();  // Rs is reused by the next work item of a persistent loop
}

// SplitMix64 finaliser (Steele, Lea, Flood 2014) as a counter-based generator.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double hash_uniform(uint64_t seed, uint64_t sid, int64_t r) {
  const uint64_t h = mix64(seed ^ mix64(sid * 0x100000001B3ull + (uint64_t)r));
  return (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

}  // namespace tp3b
