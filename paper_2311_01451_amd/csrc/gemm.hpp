// Batched GEMM on CDNA MFMA with row gathers, FP64 (v_mfma_f64_16x16x4f64)
// or FP32 (v_mfma_f32_16x16x4f32, FP32 accumulation).
//
//   C[ic(m), n] = alpha * sum_kk A(m, kk) B(kk, n) + beta * Cin[icin(m), n]
//
// Operands A, B have element type TI (double or float, which also selects
// the MFMA); C and Cin have element type TO (double or float), so an FP32
// product can be written straight into FP64 storage.
//
// Operand forms (compile time):
//   TA = 0 : A(m, kk) = A[ia(m)  * lda + kk]   (rows gathered, K contiguous)
//   TA = 1 : A(m, kk) = A[ia(kk) * lda + m]    (A stored K x M, M contiguous)
//   TB = 1 : B(kk, n) = B[ib(n)  * ldb + kk]   ("NT": rows gathered, K contiguous)
//   TB = 0 : B(kk, n) = B[ib(kk) * ldb + n]    ("NN": N contiguous)
// where ix(j) = ix ? ix[j] : j.  MODE restricts the product to a triangle:
//   SYRK_L   : only tiles meeting the lower triangle n <= m are computed
//              (M == N, BM == BN; the grid enumerates just those tiles)
//   B_NT_LOW : B(kk, n) is zero for kk > n (B = L^T, L lower triangular)
//   B_NN_LOW : B(kk, n) is zero for kk < n (B = L lower triangular)
//   A_LOW    : A(m, kk) is zero for kk > m (A lower triangular, TA = 0)
// Masked entries are selected away, so whatever the unused triangle of the
// stored operand holds is never read into the product.
//
// One workgroup (4 or 8 waves) computes a BM x BN tile; waves are arranged WM x WN
// and each holds (BM/WM/16) x (BN/WN/16) 16x16 FP64 accumulator blocks.  The
// K loop is software pipelined: the next BK-slice of A and B is fetched into
// registers while the current one is multiplied out of LDS, and LDS is double
// buffered so one barrier per slice suffices.  With VEC = 16 / sizeof(TI)
// every global access is a 16-byte load along the operand's contiguous
// dimension (the host selects it only when all leading dimensions are
// multiples of VEC and all base pointers 16-byte aligned).  The batch index is blockIdx.y;
// blockIdx.x enumerates tiles of the largest entry and entries with fewer
// tiles return early.  Consecutive workgroups land on different XCDs, so the
// tile index is remapped to give each XCD a contiguous range of tiles (rows of
// tiles sharing an A panel stay in one XCD's L2).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace rsrs {

template <typename TI, typename TO>
struct GemmDescT {
  const TI* A;
  const int64_t* ia;
  const TI* B;
  const int64_t* ib;
  const TO* Cin;
  const int64_t* icin;
  TO* C;
  const int64_t* ic;
  int64_t lda, ldb, ldcin, ldc;
  int M, N, K, pad_;
  double alpha, beta;
};
using GemmDesc = GemmDescT<double, double>;

enum GemmMode { GM_FULL = 0, GM_SYRK_L = 1, GM_B_NT_LOW = 2, GM_B_NN_LOW = 3, GM_A_LOW = 4 };

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Per element type: accumulator, MFMA and the row of result register v of a
// lane in row group q = lane / 16 (the FP64 instruction interleaves the rows
// differently from the FP32 one; both checked by probes on gfx950).
template <typename TI> struct Mfma;
template <> struct Mfma<double> {
  using acc_t = v4d;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int q) { return 4 * v + q; }
};
template <> struct Mfma<float> {
  using acc_t = v4f;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int q) { return 4 * q + v; }
};

// Pointers read from descriptors in memory are generic to the compiler, and
// generic (flat) loads count against the LDS wait counter as well: a wait for
// an LDS read would then also wait for every global prefetch in flight.  The
// kernels therefore cast them to the global address space first.
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gptr<T> to_global(T* p) { return (gptr<T>)p; }

// 16-byte load of VEC consecutive elements (VEC * sizeof(T) == 16).
template <typename T, int VEC>
__device__ __forceinline__ void load16(gptr<const T> p, T (&out)[VEC]) {
  if constexpr (sizeof(T) == 8) {
    typedef double v2d __attribute__((ext_vector_type(2)));
    const v2d v = *(gptr<const v2d>)p;
    out[0] = v.x;
    out[VEC - 1] = v.y;
  } else {
    const v4f v = *(gptr<const v4f>)p;
    out[0] = v.x;
    out[1 % VEC] = v.y;
    out[2 % VEC] = v.z;
    out[3 % VEC] = v.w;
  }
}

template <typename TI, typename TO, int BM, int BN, int WM, int WN, int TA, int TB, int MODE, int VEC>
__global__ __launch_bounds__(64 * WM * WN) void gemm_kernel(const GemmDescT<TI, TO>* __restrict__ descs) {
  using acc_t = typename Mfma<TI>::acc_t;
  constexpr int VW = 16 / (int)sizeof(TI);   // elements per 16-byte load
  constexpr int NT = 64 * WM * WN;    // threads per workgroup
  // K slice: 32 for FP32 operands on wide tiles (the MFMA work of one slice
  // then covers a global-load round trip), 64 on the narrow FP32 tiles of the
  // solves (their K loops were round-trip bound: four times fewer), 16 for
  // FP64.  FP32 sums each 16-k group in the same order whatever the slice.
  constexpr int BK = (sizeof(TI) == 4) ? (BN >= 64 ? 32 : 64) : 16;
  constexpr int PA = BM + 2;
  constexpr int PB = BN + 2;
  constexpr int FM = BM / WM / 16;
  constexpr int FN = BN / WN / 16;
  constexpr int NA = BM * BK / NT / VEC;   // VEC-wide A fetches per thread per slice
  constexpr int NB = BN * BK / NT / VEC;
  static_assert(WM * WN == 4 || WM * WN == 8, "4 or 8 waves");
  static_assert(FM >= 1 && FN >= 1, "tile too small");
  static_assert(NA >= 1 && NB >= 1 && NA * NT * VEC == BM * BK && NB * NT * VEC == BN * BK,
                "tile split");
  static_assert(VEC == 1 || VEC == VW, "VEC is 1 or one 16-byte load");
  // FP32 (KC): each operand's slice sits in LDS in the operand's own memory
  // order, so every store is one contiguous VEC-wide write: a K-contiguous
  // operand (A as M x K, B as N x K) row-major with pitch BK + 4, the other
  // K-major with pitch BM + 4 (BN + 4).  Within each 16-k group, MFMA step t
  // takes k = 4 q + t from lane group q on both operands (any assignment sums
  // the same terms; this one lets a lane read its four k of a K-contiguous
  // fragment row with one 16-byte read).  The order depends on the element
  // type only, so every tile shape and load width gives the same bits.  With
  // these pitches the 16-byte accesses and the K-major fragment reads are
  // free of bank conflicts.  FP64 keeps K-major slices (pitch BM + 2, BN + 2).
  constexpr bool KC = sizeof(TI) == 4;
  constexpr bool AR = KC && TA == 0;   // A slice row-major (m, k)
  constexpr bool BR = KC && TB == 1;   // B slice row-major (n, k)
  constexpr int PK = BK + 4;
  constexpr int PMA = KC ? BM + 4 : PA;   // K-major pitches
  constexpr int PNB = KC ? BN + 4 : PB;
  static_assert(!KC || BK % 16 == 0, "FP32 K slices hold whole 16-k groups");
  __shared__ __align__(16) TI As[2][AR ? BM * PK : BK * PMA];
  __shared__ __align__(16) TI Bs[2][BR ? BN * PK : BK * PNB];

  const GemmDescT<TI, TO> d = descs[blockIdx.y];
  const gptr<const TI> gA = to_global(d.A), gB = to_global(d.B);
  const gptr<const TO> gCin = to_global(d.Cin);
  const gptr<TO> gC = to_global(d.C);
  const gptr<const int64_t> ia = to_global(d.ia), ib = to_global(d.ib), icin = to_global(d.icin),
                            ic = to_global(d.ic);
  const int tm = (d.M + BM - 1) / BM;
  const int tn = (d.N + BN - 1) / BN;
  // SYRK_L (M == N, BM == BN) enumerates only the lower-triangle tiles
  const int ntile = (MODE == GM_SYRK_L) ? tm * (tm + 1) / 2 : tm * tn;
  const int per = gridDim.x >> 3;
  const int t = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (t >= ntile || d.M <= 0 || d.N <= 0) return;
  int m0, n0;
  if (MODE == GM_SYRK_L) {
    int ti = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    while (ti * (ti + 1) / 2 > t) --ti;
    m0 = ti * BM;
    n0 = (t - ti * (ti + 1) / 2) * BN;
  } else {
    m0 = (t / tn) * BM;
    n0 = (t % tn) * BN;
  }

  int kbeg = 0, kend = d.K;
  if (MODE == GM_B_NT_LOW) kend = min(d.K, n0 + BN);
  if (MODE == GM_B_NN_LOW) kbeg = (n0 / BK) * BK;
  if (MODE == GM_A_LOW) kend = min(d.K, m0 + BM);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN;
  const int wn = wave % WN;
  const int rowq = lane >> 4;   // 0..3
  const int coll = lane & 15;   // 0..15

  // Fetch coordinates (fixed across slices).  Each thread reads VEC
  // consecutive elements along the contiguous dimension of its operand.
  int am[NA], ak[NA], bn_[NB], bk[NB];
  gptr<const TI> arowp[NA];
  gptr<const TI> browp[NB];
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    const int e = (tid + q * NT) * VEC;
    if (TA == 0) { am[q] = e / BK; ak[q] = e % BK; }
    else         { ak[q] = e / BM; am[q] = e % BM; }
    const int gm = min(m0 + am[q], d.M - 1);
    arowp[q] = (TA == 0) ? gA + (ia ? ia[gm] : (int64_t)gm) * d.lda : gA;
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int e = (tid + q * NT) * VEC;
    if (TB == 1) { bn_[q] = e / BK; bk[q] = e % BK; }
    else         { bk[q] = e / BN; bn_[q] = e % BN; }
    const int gn = min(n0 + bn_[q], d.N - 1);
    browp[q] = (TB == 1) ? gB + (ib ? ib[gn] : (int64_t)gn) * d.ldb : gB;
  }

  // Row indices of the K-dimension gathers (TA = 1, TB = 0) are loaded one
  // slice ahead, so the dependent index load never stalls a data load.
  int64_t anext[NA], bnext[NB];
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    const int gk = kbeg + ak[q];
    anext[q] = (TA == 1 && gk < kend) ? (ia ? ia[gk] : (int64_t)gk) : 0;
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int gk = kbeg + bk[q];
    bnext[q] = (TB == 0 && gk < kend) ? (ib ? ib[gk] : (int64_t)gk) : 0;
  }

  TI ra[NA][VEC], rb[NB][VEC];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int gm = m0 + am[q], gk = k0 + ak[q];
      if (TA == 0) {
        // VEC consecutive k of row gm
        bool full = gm < d.M && gk + VEC - 1 < kend;
        if (MODE == GM_A_LOW) full = full && gk + VEC - 1 <= gm;
        if (VEC > 1 && full) {
          load16<TI, VEC>(arowp[q] + gk, ra[q]);
        } else {
#pragma unroll
          for (int u = 0; u < VEC; ++u) {
            bool ok = gm < d.M && gk + u < kend;
            if (MODE == GM_A_LOW) ok = ok && gk + u <= gm;
            ra[q][u] = ok ? arowp[q][gk + u] : TI(0);
          }
        }
      } else {
        // VEC consecutive m of row gk (A stored K x M)
        const bool rowok = gk < kend;
        const gptr<const TI> rp = gA + anext[q] * d.lda;
        const int gk2 = gk + BK;
        anext[q] = gk2 < kend ? (ia ? ia[gk2] : (int64_t)gk2) : 0;
        if (VEC > 1 && rowok && gm + VEC - 1 < d.M) {
          load16<TI, VEC>(rp + gm, ra[q]);
        } else {
#pragma unroll
          for (int u = 0; u < VEC; ++u) ra[q][u] = (rowok && gm + u < d.M) ? rp[gm + u] : TI(0);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int gn = n0 + bn_[q], gk = k0 + bk[q];
      if (TB == 1) {
        // VEC consecutive k of row gn
        bool full = gn < d.N && gk + VEC - 1 < kend;
        if (MODE == GM_B_NT_LOW) full = full && gk + VEC - 1 <= gn;
        if (VEC > 1 && full) {
          load16<TI, VEC>(browp[q] + gk, rb[q]);
        } else {
#pragma unroll
          for (int u = 0; u < VEC; ++u) {
            bool ok = gn < d.N && gk + u < kend;
            if (MODE == GM_B_NT_LOW) ok = ok && gk + u <= gn;
            rb[q][u] = ok ? browp[q][gk + u] : TI(0);
          }
        }
      } else {
        // VEC consecutive n of row gk
        const bool rowok = gk < kend;
        const gptr<const TI> rp = gB + bnext[q] * d.ldb;
        const int gk2 = gk + BK;
        bnext[q] = gk2 < kend ? (ib ? ib[gk2] : (int64_t)gk2) : 0;
        bool full = rowok && gn + VEC - 1 < d.N;
        if (MODE == GM_B_NN_LOW) full = full && gk >= gn + VEC - 1;
        if (VEC > 1 && full) {
          load16<TI, VEC>(rp + gn, rb[q]);
        } else {
#pragma unroll
          for (int u = 0; u < VEC; ++u) {
            bool ok = rowok && gn + u < d.N;
            if (MODE == GM_B_NN_LOW) ok = ok && gk >= gn + u;
            rb[q][u] = ok ? rp[gn + u] : TI(0);
          }
        }
      }
    }
  };
  auto stash = [&](int b) {
    if constexpr (KC) {
      // every thread's VEC elements are contiguous in the LDS layout
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        TI* dst = AR ? &As[b][am[q] * PK + ak[q]] : &As[b][ak[q] * PMA + am[q]];
        if constexpr (VEC == 4) {
          *reinterpret_cast<v4f*>(dst) = v4f{ra[q][0], ra[q][1 % VEC], ra[q][2 % VEC], ra[q][3 % VEC]};
        } else {
#pragma unroll
          for (int u = 0; u < VEC; ++u) dst[u] = ra[q][u];
        }
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        TI* dst = BR ? &Bs[b][bn_[q] * PK + bk[q]] : &Bs[b][bk[q] * PNB + bn_[q]];
        if constexpr (VEC == 4) {
          *reinterpret_cast<v4f*>(dst) = v4f{rb[q][0], rb[q][1 % VEC], rb[q][2 % VEC], rb[q][3 % VEC]};
        } else {
#pragma unroll
          for (int u = 0; u < VEC; ++u) dst[u] = rb[q][u];
        }
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < NA; ++q)
#pragma unroll
      for (int u = 0; u < VEC; ++u) {
        if (TA == 0) As[b][(ak[q] + u) * PA + am[q]] = ra[q][u];
        else         As[b][ak[q] * PA + am[q] + u] = ra[q][u];
      }
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int u = 0; u < VEC; ++u) {
        if (TB == 1) Bs[b][(bk[q] + u) * PB + bn_[q]] = rb[q][u];
        else         Bs[b][bk[q] * PB + bn_[q] + u] = rb[q][u];
      }
  };

  acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  if (kbeg < kend) {
    fetch(kbeg);
    stash(0);
    __syncthreads();
  }
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) fetch(k0 + BK);
    const TI* as = As[buf];
    const TI* bs = Bs[buf];
    if constexpr (KC) {
#pragma unroll
      for (int kc = 0; kc < BK; kc += 16) {
        v4f a[FM], b[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          const int r = wm * (BM / WM) + i * 16 + coll;
          if constexpr (AR) {
            a[i] = *reinterpret_cast<const v4f*>(&as[r * PK + kc + 4 * rowq]);
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) a[i][t] = as[(kc + 4 * rowq + t) * PMA + r];
          }
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int c = wn * (BN / WN) + j * 16 + coll;
          if constexpr (BR) {
            b[j] = *reinterpret_cast<const v4f*>(&bs[c * PK + kc + 4 * rowq]);
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) b[j][t] = bs[(kc + 4 * rowq + t) * PNB + c];
          }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[i][j] = Mfma<TI>::mma(a[i][t], b[j][t], acc[i][j]);
      }
    } else
#pragma unroll
    for (int kq = 0; kq < BK; kq += 4) {
      TI a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = as[(kq + rowq) * PA + wm * (BM / WM) + i * 16 + coll];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = bs[(kq + rowq) * PB + wn * (BN / WN) + j * 16 + coll];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = Mfma<TI>::mma(a[i], b[j], acc[i][j]);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // ---- epilogue: register v of lane l holds D[Mfma::row(v, l/16)][l % 16]
  // of each 16x16 block (operands: A[l % 16][l / 16], B[l / 16][l % 16])
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gm = m0 + wm * (BM / WM) + i * 16 + Mfma<TI>::row(v, rowq);
      if (gm >= d.M) continue;
      const int64_t ro = ic ? ic[gm] : gm;
      const int64_t rc = icin ? icin[gm] : gm;
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int gn = n0 + wn * (BN / WN) + j * 16 + coll;
        if (gn < d.N) {
          double out = d.alpha * (double)acc[i][j][v];
          if (d.beta != 0.0) out += d.beta * (double)gCin[rc * d.ldcin + gn];
          gC[ro * d.ldc + gn] = (TO)out;
        }
      }
    }
}

}  // namespace rsrs
