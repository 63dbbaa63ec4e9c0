// Batched FP64 GEMM on CDNA MFMA (v_mfma_f64_16x16x4f64) with row gathers.
//
//   C[ic(m), n] = alpha * sum_kk A(m, kk) B(kk, n) + beta * Cin[icin(m), n]
//
// Operand forms (compile time):
//   TA = 0 : A(m, kk) = A[ia(m)  * lda + kk]   (rows gathered, K contiguous)
//   TA = 1 : A(m, kk) = A[ia(kk) * lda + m]    (A stored K x M, M contiguous)
//   TB = 1 : B(kk, n) = B[ib(n)  * ldb + kk]   ("NT": rows gathered, K contiguous)
//   TB = 0 : B(kk, n) = B[ib(kk) * ldb + n]    ("NN": N contiguous)
// where ix(j) = ix ? ix[j] : j.  MODE restricts the product to a triangle:
//   SYRK_L   : only tiles meeting the lower triangle n <= m are computed
//   B_NT_LOW : B(kk, n) is zero for kk > n (B = L^T, L lower triangular)
//   B_NN_LOW : B(kk, n) is zero for kk < n (B = L lower triangular)
//   A_LOW    : A(m, kk) is zero for kk > m (A lower triangular, TA = 0)
// Masked entries are selected away, so whatever the unused triangle of the
// stored operand holds is never read into the product.
//
// One workgroup (4 waves) computes a BM x BN tile; waves are arranged WM x WN
// and each holds (BM/WM/16) x (BN/WN/16) 16x16 FP64 accumulator blocks.  The
// batch index is blockIdx.y; blockIdx.x enumerates tiles of the largest entry
// and entries with fewer tiles return early.  Tiles are walked so that
// consecutive workgroups (which land on different XCDs) take tiles far apart
// while each XCD sweeps a contiguous range of tiles, keeping A-row panels
// resident in that XCD's L2.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace rsrs {

struct GemmDesc {
  const double* A;
  const int64_t* ia;
  const double* B;
  const int64_t* ib;
  const double* Cin;
  const int64_t* icin;
  double* C;
  const int64_t* ic;
  int64_t lda, ldb, ldcin, ldc;
  int M, N, K, pad_;
  double alpha, beta;
};

enum GemmMode { GM_FULL = 0, GM_SYRK_L = 1, GM_B_NT_LOW = 2, GM_B_NN_LOW = 3, GM_A_LOW = 4 };

typedef double v4d __attribute__((ext_vector_type(4)));

template <int BM, int BN, int WM, int WN, int TA, int TB, int MODE>
__global__ __launch_bounds__(256) void gemm_f64_kernel(const GemmDesc* __restrict__ descs) {
  constexpr int BK = 16;
  constexpr int PA = BM + 2;
  constexpr int PB = BN + 2;
  constexpr int FM = BM / WM / 16;
  constexpr int FN = BN / WN / 16;
  static_assert(WM * WN == 4, "4 waves");
  static_assert(FM >= 1 && FN >= 1, "tile too small");
  __shared__ double As[BK * PA];
  __shared__ double Bs[BK * PB];

  const GemmDesc d = descs[blockIdx.y];
  const int tm = (d.M + BM - 1) / BM;
  const int tn = (d.N + BN - 1) / BN;
  const int ntile = tm * tn;
  // XCD-aware walk (gridDim.x is a multiple of 8): blockIdx.x % 8 picks the
  // XCD, which then sweeps a contiguous chunk of tiles.
  const int per = gridDim.x >> 3;
  const int t = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (t >= ntile || d.M <= 0 || d.N <= 0) return;
  const int tile_m = t / tn;
  const int tile_n = t % tn;
  const int m0 = tile_m * BM;
  const int n0 = tile_n * BN;
  if (MODE == GM_SYRK_L && n0 > m0 + BM - 1) return;

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

  v4d acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    // ---- global -> LDS, A tile (BM x BK) stored As[kk][m]
#pragma unroll
    for (int e = tid; e < BM * BK; e += 256) {
      int m, kk;
      if (TA == 0) { m = e / BK; kk = e % BK; }
      else         { kk = e / BM; m = e % BM; }
      const int gm = m0 + m, gk = k0 + kk;
      double v = 0.0;
      bool ok = gm < d.M && gk < kend;
      if (MODE == GM_A_LOW) ok = ok && gk <= gm;
      if (ok) {
        if (TA == 0) {
          const int64_t r = d.ia ? d.ia[gm] : gm;
          v = d.A[r * d.lda + gk];
        } else {
          const int64_t r = d.ia ? d.ia[gk] : gk;
          v = d.A[r * d.lda + gm];
        }
      }
      As[kk * PA + m] = v;
    }
    // ---- B tile (BK x BN) stored Bs[kk][n]
#pragma unroll
    for (int e = tid; e < BN * BK; e += 256) {
      int n, kk;
      if (TB == 1) { n = e / BK; kk = e % BK; }
      else         { kk = e / BN; n = e % BN; }
      const int gn = n0 + n, gk = k0 + kk;
      double v = 0.0;
      bool ok = gn < d.N && gk < kend;
      if (MODE == GM_B_NT_LOW) ok = ok && gk <= gn;
      if (MODE == GM_B_NN_LOW) ok = ok && gk >= gn;
      if (ok) {
        if (TB == 1) {
          const int64_t r = d.ib ? d.ib[gn] : gn;
          v = d.B[r * d.ldb + gk];
        } else {
          const int64_t r = d.ib ? d.ib[gk] : gk;
          v = d.B[r * d.ldb + gn];
        }
      }
      Bs[kk * PB + n] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < BK; kq += 4) {
      double a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        a[i] = As[(kq + rowq) * PA + wm * (BM / WM) + i * 16 + coll];
#pragma unroll
      for (int j = 0; j < FN; ++j)
        b[j] = Bs[(kq + rowq) * PB + wn * (BN / WN) + j * 16 + coll];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  // ---- epilogue: register v of lane l holds D[4*v + l/16][l % 16] of each
  // 16x16 block (operands: A[l % 16][l / 16], B[l / 16][l % 16])
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm * (BM / WM) + i * 16 + v * 4 + rowq;
        const int gn = n0 + wn * (BN / WN) + j * 16 + coll;
        if (gm < d.M && gn < d.N) {
          double out = d.alpha * acc[i][j][v];
          if (d.beta != 0.0) {
            const int64_t rc = d.icin ? d.icin[gm] : gm;
            out += d.beta * d.Cin[rc * d.ldcin + gn];
          }
          const int64_t ro = d.ic ? d.ic[gm] : gm;
          d.C[ro * d.ldc + gn] = out;
        }
      }
}

}  // namespace rsrs
