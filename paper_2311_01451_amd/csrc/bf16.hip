// BF16 products of the built-in kernel operators (sample products with the
// test matrices rounded to BF16, FP32 accumulation).
//
//   C[m][n] = sum_k A[m][k] * Bt[n][k]      A: M x K bf16, Bt: N x K bf16,
//                                          C: M x N float (row-major)
//
// Both operands are K-contiguous, so every global load is a 16-byte chunk
// of 8 consecutive k and lands in LDS unchanged; v_mfma_f32_16x16x32_bf16
// takes lane l's operands as A[l % 16][8 (l / 16) .. +7] and
// Bt[l % 16][8 (l / 16) .. +7] and returns D[4 (l / 16) + v][l % 16]
// (checked by a probe on gfx950).  128 x 128 tiles on 8 waves (each wave
// 64 x 32), BK = 64, LDS rows padded to 144 bytes so the 16 rows read by a
// quarter-wave fall in distinct banks; double-buffered LDS with the next
// slice prefetched into registers; XCD-aware tile order as in gemm.hpp.
//
// A block X (K x N float, row-major: the layout of the samples) is brought
// into the Bt form by a tiled transpose that rounds each value to BF16
// (round to nearest even).
//
// The operator product itself is a plain dense GEMM (the explicit operator
// matrix times the block), so it goes to hipBLASLt (BF16 operands, FP32
// accumulation and output) when the library offers an algorithm for the
// shape that needs no workspace (so that products on several streams share
// nothing); the kernels above are the fallback.  The handle and the chosen
// algorithm per shape are kept per device for the life of the process.
#include <hip/hip_runtime.h>
#include <hipblaslt/hipblaslt.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>

#include "kernels.hpp"
#include "profile.hpp"

namespace rsrs {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f2bf(float x) {
  // round to nearest even (the inputs here are finite)
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

constexpr int BM = 128, BN = 128, BK = 64;
constexpr int LDR = BK + 8;          // bf16 per LDS row (144 bytes)
constexpr int NT = 512;

struct Bf16Desc {
  const uint16_t* A;
  const uint16_t* Bt;
  float* C;
  int64_t lda, ldb, ldc;
  int M, N, K;
};

__global__ __launch_bounds__(NT) void gemm_bf16_nt_kernel(Bf16Desc d) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * LDR];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN * LDR];
  const int tm = (d.M + BM - 1) / BM, tn = (d.N + BN - 1) / BN;
  const int per = gridDim.x >> 3;
  const int t = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (t >= tm * tn) return;
  const int m0 = (t / tn) * BM, n0 = (t % tn) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;   // 2 x 4 waves, each 64 x 32
  const int q = lane >> 4, c16 = lane & 15;

  // fetch mapping: 2 chunks of 8 k per operand per thread
  int fr[2], fk[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int e = tid + i * NT;   // 0..1023
    fr[i] = e >> 3;               // row 0..127
    fk[i] = (e & 7) * 8;          // k offset 0..56
  }
  uint4 ra[2], rb[2];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int gk = k0 + fk[i];
      const int gm = m0 + fr[i], gn = n0 + fr[i];
      uint4 va = {0u, 0u, 0u, 0u}, vb = {0u, 0u, 0u, 0u};
      if (gm < d.M && gk + 8 <= d.K) va = *reinterpret_cast<const uint4*>(d.A + gm * d.lda + gk);
      else if (gm < d.M) {
        uint16_t tmp[8];
        for (int u = 0; u < 8; ++u) tmp[u] = gk + u < d.K ? d.A[gm * d.lda + gk + u] : (uint16_t)0;
        va = *reinterpret_cast<const uint4*>(tmp);
      }
      if (gn < d.N && gk + 8 <= d.K) vb = *reinterpret_cast<const uint4*>(d.Bt + gn * d.ldb + gk);
      else if (gn < d.N) {
        uint16_t tmp[8];
        for (int u = 0; u < 8; ++u) tmp[u] = gk + u < d.K ? d.Bt[gn * d.ldb + gk + u] : (uint16_t)0;
        vb = *reinterpret_cast<const uint4*>(tmp);
      }
      ra[i] = va;
      rb[i] = vb;
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      *reinterpret_cast<uint4*>(&As[b][fr[i] * LDR + fk[i]]) = ra[i];
      *reinterpret_cast<uint4*>(&Bs[b][fr[i] * LDR + fk[i]]) = rb[i];
    }
  };

  v4f acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  fetch(0);
  stash(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < d.K; k0 += BK) {
    const bool more = k0 + BK < d.K;
    if (more) fetch(k0 + BK);
    const uint16_t* as = As[buf];
    const uint16_t* bs = Bs[buf];
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      v8bf a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a[i] = *reinterpret_cast<const v8bf*>(&as[(wm * 64 + i * 16 + c16) * LDR + kk + q * 8]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        b[j] = *reinterpret_cast<const v8bf*>(&bs[(wn * 32 + j * 16 + c16) * LDR + kk + q * 8]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gm = m0 + wm * 64 + i * 16 + 4 * q + v;
      if (gm >= d.M) continue;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int gn = n0 + wn * 32 + j * 16 + c16;
        if (gn < d.N) d.C[(int64_t)gm * d.ldc + gn] = acc[i][j][v];
      }
    }
}

// The same product on 256 x 256 tiles: 8 waves as 2 x 4, each wave 128 x 64
// (8 x 4 MFMA tiles), so that every fragment read from LDS feeds 4 or 8
// MFMAs; LDS traffic per MFMA is half that of the 128 x 128 form, about the
// MFMA time itself.  Double-buffered LDS (144 KiB: one workgroup per CU),
// next slice prefetched into registers, XCD-aware tile order.
constexpr int WBM = 256, WBN = 256;

__global__ __launch_bounds__(NT) void gemm_bf16_nt256_kernel(Bf16Desc d) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[2 * (WBM + WBN) * LDR];
  uint16_t* As0 = lds;
  uint16_t* Bs0 = lds + 2 * WBM * LDR;
  const int tm = (d.M + WBM - 1) / WBM, tn = (d.N + WBN - 1) / WBN;
  const int per = gridDim.x >> 3;
  const int t = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (t >= tm * tn) return;
  const int m0 = (t / tn) * WBM, n0 = (t % tn) * WBN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;   // 2 x 4 waves, each 128 x 64
  const int q = lane >> 4, c16 = lane & 15;

  // fetch mapping: 4 chunks of 8 k per operand per thread
  int fr[4], fk[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = tid + i * NT;   // 0..2047
    fr[i] = e >> 3;               // row 0..255
    fk[i] = (e & 7) * 8;          // k offset 0..56
  }
  uint4 ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int gk = k0 + fk[i];
      const int gm = m0 + fr[i], gn = n0 + fr[i];
      uint4 va = {0u, 0u, 0u, 0u}, vb = {0u, 0u, 0u, 0u};
      if (gm < d.M && gk + 8 <= d.K) va = *reinterpret_cast<const uint4*>(d.A + gm * d.lda + gk);
      else if (gm < d.M) {
        uint16_t tmp[8];
        for (int u = 0; u < 8; ++u) tmp[u] = gk + u < d.K ? d.A[gm * d.lda + gk + u] : (uint16_t)0;
        va = *reinterpret_cast<const uint4*>(tmp);
      }
      if (gn < d.N && gk + 8 <= d.K) vb = *reinterpret_cast<const uint4*>(d.Bt + gn * d.ldb + gk);
      else if (gn < d.N) {
        uint16_t tmp[8];
        for (int u = 0; u < 8; ++u) tmp[u] = gk + u < d.K ? d.Bt[gn * d.ldb + gk + u] : (uint16_t)0;
        vb = *reinterpret_cast<const uint4*>(tmp);
      }
      ra[i] = va;
      rb[i] = vb;
    }
  };
  auto stash = [&](int b) {
    uint16_t* as = As0 + b * WBM * LDR;
    uint16_t* bs = Bs0 + b * WBN * LDR;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      *reinterpret_cast<uint4*>(&as[fr[i] * LDR + fk[i]]) = ra[i];
      *reinterpret_cast<uint4*>(&bs[fr[i] * LDR + fk[i]]) = rb[i];
    }
  };

  v4f acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  fetch(0);
  stash(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < d.K; k0 += BK) {
    const bool more = k0 + BK < d.K;
    if (more) fetch(k0 + BK);
    const uint16_t* as = As0 + buf * WBM * LDR;
    const uint16_t* bs = Bs0 + buf * WBN * LDR;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      v8bf b[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b[j] = *reinterpret_cast<const v8bf*>(&bs[(wn * 64 + j * 16 + c16) * LDR + kk + q * 8]);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const v8bf a = *reinterpret_cast<const v8bf*>(&as[(wm * 128 + i * 16 + c16) * LDR + kk + q * 8]);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[i][j], 0, 0, 0);
      }
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gm = m0 + wm * 128 + i * 16 + 4 * q + v;
      if (gm >= d.M) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int gn = n0 + wn * 64 + j * 16 + c16;
        if (gn < d.N) d.C[(int64_t)gm * d.ldc + gn] = acc[i][j][v];
      }
    }
}

// X (rows x cols float, leading dimension ldx) -> Xt (cols x rows bf16,
// leading dimension ldt), 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void transpose_bf16_kernel(const float* X, int64_t ldx, uint16_t* Xt,
                                                             int64_t ldt, int64_t rows, int64_t cols) {
  __shared__ uint16_t tile[64][66];
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int64_t r = r0 + i, c = c0 + tx;
    tile[i][tx] = (r < rows && c < cols) ? f2bf(X[r * ldx + c]) : (uint16_t)0;
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < cols && r < rows) Xt[c * ldt + r] = tile[tx][i];
  }
}

__global__ void round_bf16_kernel(const double* src, uint16_t* dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = f2bf((float)src[i]);
}

__global__ void round_f32_to_bf16_values_kernel(float* x, int64_t rows, int64_t cols, int64_t ld) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows * cols;
       i += (int64_t)gridDim.x * blockDim.x) {
    float* p = x + (i / cols) * ld + i % cols;
    *p = __uint_as_float((uint32_t)f2bf(*p) << 16);
  }
}

}  // namespace

rsrs_status bf16_from_f64(hipStream_t st, const double* src, uint16_t* dst, int64_t n) {
  const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(round_bf16_kernel, dim3(g), dim3(256), 0, st, src, dst, n);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}

void round_to_bf16_values(hipStream_t st, float* x, int64_t rows, int64_t cols, int64_t ld) {
  if (rows <= 0 || cols <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>((rows * cols + 255) / 256, 16384);
  hipLaunchKernelGGL(round_f32_to_bf16_values_kernel, dim3(g), dim3(256), 0, st, x, rows, cols, ld);
}

namespace {

// hipBLASLt state of one device.  In column-major terms the product is
// Y^T (N x M, ld ldy) = Xt^T (Xt stored K x N, ld ldt, op T) * A^T (A stored
// K x M, ld lda, op N).
struct LtDev {
  std::mutex mu;
  bool tried = false, ok = false;
  hipblasLtHandle_t h = nullptr;
  std::map<std::tuple<int64_t, int64_t, int64_t, int64_t, int64_t, int64_t>, hipblasLtMatmulAlgo_t> algo;
  std::map<std::tuple<int64_t, int64_t, int64_t, int64_t, int64_t, int64_t>, bool> none;
};
LtDev& lt_dev(int dev) {
  static LtDev d[64];
  return d[dev & 63];
}

// The product's descriptors and algorithm; false when hipBLASLt has none for
// this shape (then nothing is enqueued).
struct LtCall {
  hipblasLtMatmulDesc_t desc = nullptr;
  hipblasLtMatrixLayout_t la = nullptr, lb = nullptr, lc = nullptr;
  const hipblasLtMatmulAlgo_t* algo = nullptr;
  LtDev* dev = nullptr;
  ~LtCall() {
    if (lc) (void)hipblasLtMatrixLayoutDestroy(lc);
    if (lb) (void)hipblasLtMatrixLayoutDestroy(lb);
    if (la) (void)hipblasLtMatrixLayoutDestroy(la);
    if (desc) (void)hipblasLtMatmulDescDestroy(desc);
  }
};
bool lt_prepare(LtCall& c, int64_t lda, int64_t M, int64_t K, int64_t ldt, int64_t N, int64_t ldy) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  LtDev& L = lt_dev(dev);
  std::lock_guard<std::mutex> lk(L.mu);
  if (!L.tried) {
    L.tried = true;
    if (hipblasLtCreate(&L.h) != HIPBLAS_STATUS_SUCCESS) return false;
    L.ok = true;
  }
  if (!L.ok) return false;
  const auto key = std::make_tuple(M, N, K, lda, ldt, ldy);
  if (L.none.count(key)) return false;
  const hipblasOperation_t opT = HIPBLAS_OP_T, opN = HIPBLAS_OP_N;
  if (hipblasLtMatmulDescCreate(&c.desc, HIPBLAS_COMPUTE_32F, HIP_R_32F) != HIPBLAS_STATUS_SUCCESS ||
      hipblasLtMatmulDescSetAttribute(c.desc, HIPBLASLT_MATMUL_DESC_TRANSA, &opT, sizeof(opT)) !=
          HIPBLAS_STATUS_SUCCESS ||
      hipblasLtMatmulDescSetAttribute(c.desc, HIPBLASLT_MATMUL_DESC_TRANSB, &opN, sizeof(opN)) !=
          HIPBLAS_STATUS_SUCCESS ||
      hipblasLtMatrixLayoutCreate(&c.la, HIP_R_16BF, (uint64_t)K, (uint64_t)N, ldt) != HIPBLAS_STATUS_SUCCESS ||
      hipblasLtMatrixLayoutCreate(&c.lb, HIP_R_16BF, (uint64_t)K, (uint64_t)M, lda) != HIPBLAS_STATUS_SUCCESS ||
      hipblasLtMatrixLayoutCreate(&c.lc, HIP_R_32F, (uint64_t)N, (uint64_t)M, ldy) != HIPBLAS_STATUS_SUCCESS)
    return false;
  auto it = L.algo.find(key);
  if (it == L.algo.end()) {
    hipblasLtMatmulPreference_t pref = nullptr;
    hipblasLtMatmulHeuristicResult_t res[1];
    int nres = 0;
    uint64_t wsb = 0;
    if (hipblasLtMatmulPreferenceCreate(&pref) == HIPBLAS_STATUS_SUCCESS &&
        hipblasLtMatmulPreferenceSetAttribute(pref, HIPBLASLT_MATMUL_PREF_MAX_WORKSPACE_BYTES, &wsb, sizeof(wsb)) ==
            HIPBLAS_STATUS_SUCCESS &&
        hipblasLtMatmulAlgoGetHeuristic(L.h, c.desc, c.la, c.lb, c.lc, c.lc, pref, 1, res, &nres) ==
            HIPBLAS_STATUS_SUCCESS &&
        nres > 0 && res[0].state == HIPBLAS_STATUS_SUCCESS && res[0].workspaceSize == 0)
      it = L.algo.emplace(key, res[0].algo).first;
    else
      L.none[key] = true;
    if (pref) (void)hipblasLtMatmulPreferenceDestroy(pref);
    if (it == L.algo.end()) return false;
  }
  c.algo = &it->second;
  c.dev = &L;
  return true;
}

std::atomic<bool> g_lib_gemm{true};

}  // namespace

bool operator_library_gemm() { return g_lib_gemm.load(std::memory_order_relaxed); }
void set_operator_library_gemm(bool on) { g_lib_gemm.store(on, std::memory_order_relaxed); }

// Y (M x N float) = A (M x K bf16, row-major) * X (K x N float with values
// representable in bf16), through the transposed bf16 copy Xt (N x K) held in
// the caller's workspace.
rsrs_status gemm_bf16_op(hipStream_t st, const uint16_t* A, int64_t lda, int64_t M, int64_t K,
                         const float* X, int64_t ldx, int64_t N, float* Y, int64_t ldy, uint16_t* Xt,
                         int64_t ldt) {
  if (M <= 0 || N <= 0) return RSRS_OK;
  if ((lda % 8) || (ldt % 8) || ((uintptr_t)A & 15) || ((uintptr_t)Xt & 15)) {
    set_error("bf16 product needs leading dimensions that are multiples of 8 and aligned bases");
    return RSRS_E_INVALID;
  }
  {
    ProfScope ps(st, "transpose_bf16", 0.0, 6.0 * (double)K * N);
    dim3 g((unsigned)((N + 63) / 64), (unsigned)((K + 63) / 64));
    hipLaunchKernelGGL(transpose_bf16_kernel, g, dim3(256), 0, st, X, ldx, Xt, ldt, K, N);
  }
  Bf16Desc d{A, Xt, Y, lda, ldt, ldy, (int)M, (int)N, (int)K};
  const double fl = 2.0 * M * N * K, by = 2.0 * (M * K + N * K) + 4.0 * M * N;
  {
    LtCall c;
    if (operator_library_gemm() && lt_prepare(c, lda, M, K, ldt, N, ldy)) {
      const float alpha = 1.0f, beta = 0.0f;
      ProfScope ps(st, "gemm_bf16_hipblaslt:operator", fl, by);
      if (hipblasLtMatmul(c.dev->h, c.desc, &alpha, Xt, c.la, A, c.lb, &beta, Y, c.lc, Y, c.lc, c.algo, nullptr, 0,
                          st) == HIPBLAS_STATUS_SUCCESS)
        return RSRS_OK;
      // refused (hipBLASLt validates before it launches): this shape takes
      // the kernels below from now on
      std::lock_guard<std::mutex> lk(c.dev->mu);
      c.dev->none[std::make_tuple(M, N, K, lda, ldt, ldy)] = true;
    }
  }
  if (M >= WBM && N >= WBN) {
    const int64_t tiles = ((M + WBM - 1) / WBM) * ((N + WBN - 1) / WBN);
    ProfScope ps(st, "gemm_bf16_nt_256x256:operator", fl, by);
    hipLaunchKernelGGL(gemm_bf16_nt256_kernel, dim3((unsigned)round_up(tiles, 8)), dim3(NT), 0, st, d);
    RSRS_HIP(hipGetLastError());
    return RSRS_OK;
  }
  const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  ProfScope ps(st, "gemm_bf16_nt_128x128:operator", fl, by);
  hipLaunchKernelGGL(gemm_bf16_nt_kernel, dim3((unsigned)round_up(tiles, 8)), dim3(NT), 0, st, d);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}

}  // namespace rsrs
