// Batched dense helpers: GEMM dispatch, Cholesky leaves, Gauss-Jordan inverse,
// copies, permutations and reductions (FP64).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "kernels.hpp"

namespace rsrs {

// ---------------------------------------------------------------- uploader
rsrs_status Uploader::init(size_t bytes, hipStream_t stream) {
  st = stream;
  off = 0;
  RSRS_TRY(h.alloc(bytes));
  RSRS_TRY(d.alloc(bytes));
  return RSRS_OK;
}

rsrs_status Uploader::put(const void* src, size_t n, void** dev) {
  const size_t need = round_up((int64_t)n, 256);
  if (off + need > h.bytes) {
    // out of staging space: drain the stream, then recycle from the start
    RSRS_TRY(reset());
    if (need > h.bytes) {
      size_t nb = std::max(need, h.bytes * 2);
      HostBuf h2;
      DevBuf d2;
      RSRS_TRY(h2.alloc(nb));
      RSRS_TRY(d2.alloc(nb));
      std::swap(h.p, h2.p);
      std::swap(h.bytes, h2.bytes);
      d = std::move(d2);
    }
  }
  char* hp = static_cast<char*>(h.p) + off;
  char* dp = static_cast<char*>(d.p) + off;
  if (n) std::memcpy(hp, src, n);
  if (n) RSRS_HIP(hipMemcpyAsync(dp, hp, n, hipMemcpyHostToDevice, st));
  *dev = dp;
  off += need;
  return RSRS_OK;
}

rsrs_status Uploader::reset() {
  RSRS_HIP(hipStreamSynchronize(st));
  off = 0;
  return RSRS_OK;
}

// ---------------------------------------------------------------- GEMM dispatch
template <int BM, int BN, int WM, int WN, int TA, int TB, int MODE>
static rsrs_status launch_gemm(Uploader& up, hipStream_t st, const std::vector<GemmDesc>& descs) {
  int64_t tiles = 0;
  for (const auto& d : descs)
    if (d.M > 0 && d.N > 0)
      tiles = std::max<int64_t>(tiles, (int64_t)((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN));
  if (tiles == 0) return RSRS_OK;
  for (size_t b0 = 0; b0 < descs.size(); b0 += 65535) {
    const size_t nb = std::min<size_t>(65535, descs.size() - b0);
    std::vector<GemmDesc> part(descs.begin() + b0, descs.begin() + b0 + nb);
    GemmDesc* dd = nullptr;
    RSRS_TRY(up.put_vec(part, &dd));
    dim3 grid((unsigned)round_up(tiles, 8), (unsigned)nb);
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, WM, WN, TA, TB, MODE>), grid, dim3(256), 0, st, dd);
    RSRS_HIP(hipGetLastError());
  }
  return RSRS_OK;
}

template <int BM, int BN, int WM, int WN>
static rsrs_status gemm_shape(Uploader& up, hipStream_t st, const std::vector<GemmDesc>& descs,
                              int ta, int tb, int mode) {
#define RSRS_G(TA, TB, MODE)                                                       \
  if (ta == TA && tb == TB && mode == MODE)                                        \
    return launch_gemm<BM, BN, WM, WN, TA, TB, MODE>(up, st, descs);
  RSRS_G(0, 0, GM_FULL)
  RSRS_G(0, 1, GM_FULL)
  RSRS_G(1, 0, GM_FULL)
  RSRS_G(1, 1, GM_FULL)
  RSRS_G(0, 1, GM_SYRK_L)
  RSRS_G(0, 1, GM_B_NT_LOW)
  RSRS_G(0, 0, GM_B_NN_LOW)
  RSRS_G(0, 0, GM_A_LOW)
#undef RSRS_G
  set_error("unsupported GEMM form");
  return RSRS_E_UNSUPPORTED;
}

rsrs_status gemm(Uploader& up, hipStream_t st, const std::vector<GemmDesc>& descs, int ta, int tb,
                 int mode, GemmShape shape) {
  if (descs.empty()) return RSRS_OK;
  if (shape == GS_64x16 && mode == GM_FULL) return gemm_shape<64, 16, 4, 1>(up, st, descs, ta, tb, mode);
  return gemm_shape<64, 64, 2, 2>(up, st, descs, ta, tb, mode);
}

// ---------------------------------------------------------------- Cholesky leaf
// One workgroup per 64x64 (or smaller) diagonal block: unblocked right-looking
// Cholesky in LDS, then the inverse of the factor by forward substitution.
__global__ __launch_bounds__(256) void chol_leaf_kernel(const CholLeaf* __restrict__ e, int* flag) {
  constexpr int NB = 64;
  __shared__ double L[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  const CholLeaf d = e[blockIdx.x];
  const int n = d.n;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < NB * NB; idx += 256) {
    const int i = idx / NB, j = idx % NB;
    double v = 0.0;
    if (i < n && j <= i) v = d.G[(int64_t)i * d.ld + j];
    L[i][j] = v;
    X[i][j] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      double v = L[j][j];
      if (!(v > 0.0)) {
        atomicOr(flag, 1);
        v = 1.0;
      }
      L[j][j] = sqrt(v);
    }
    __syncthreads();
    const double inv = 1.0 / L[j][j];
    for (int i = j + 1 + tid; i < n; i += 256) L[i][j] *= inv;
    __syncthreads();
    // trailing update of the lower triangle: pairs (i, c) with j < c <= i < n
    const int m = n - j - 1;
    const int npair = m * (m + 1) / 2;
    for (int pidx = tid; pidx < npair; pidx += 256) {
      // map pidx -> (ii, cc) with 0 <= cc <= ii < m
      int ii = (int)((sqrt(8.0 * pidx + 1.0) - 1.0) * 0.5);
      while ((ii + 1) * (ii + 2) / 2 <= pidx) ++ii;
      while (ii * (ii + 1) / 2 > pidx) --ii;
      const int cc = pidx - ii * (ii + 1) / 2;
      const int i = j + 1 + ii, c = j + 1 + cc;
      L[i][c] -= L[i][j] * L[c][j];
    }
    __syncthreads();
  }
  // X = L^{-1}, row by row: X[i][c] = -(sum_{t=c}^{i-1} L[i][t] X[t][c]) / L[i][i]
  for (int i = 0; i < n; ++i) {
    if (tid <= i) {
      const int c = tid;
      double v;
      if (c == i) {
        v = 1.0 / L[i][i];
      } else {
        double s = 0.0;
        for (int t = c; t < i; ++t) s += L[i][t] * X[t][c];
        v = -s / L[i][i];
      }
      X[i][c] = v;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < n * n; idx += 256) {
    const int i = idx / n, j = idx % n;
    d.Li[(int64_t)i * d.ld + j] = X[i][j];
  }
}

rsrs_status chol_leaf(Uploader& up, hipStream_t st, const std::vector<CholLeaf>& e, int* flag) {
  if (e.empty()) return RSRS_OK;
  CholLeaf* de = nullptr;
  RSRS_TRY(up.put_vec(e, &de));
  hipLaunchKernelGGL(chol_leaf_kernel, dim3((unsigned)e.size()), dim3(256), 0, st, de, flag);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}

// ---------------------------------------------------------------- Gauss-Jordan
__global__ __launch_bounds__(1024) void gje_kernel(const GjeDesc* __restrict__ e, int* flag) {
  const GjeDesc d = e[blockIdx.x];
  const int n = d.n;
  const int n2 = 2 * n;
  double* W = d.W;
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  __shared__ double rv[1024];
  __shared__ int ri[1024];
  __shared__ double fcol[4096];
  for (int64_t idx = tid; idx < (int64_t)n * n2; idx += nt) {
    const int i = (int)(idx / n2), c = (int)(idx % n2);
    W[idx] = c < n ? d.A[(int64_t)i * d.lda + c] : (c - n == i ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    // pivot: largest |W[i][j]|, i >= j, lowest index on ties
    double best = -1.0;
    int bi = n;
    for (int i = j + tid; i < n; i += nt) {
      const double v = fabs(W[(int64_t)i * n2 + j]);
      if (v > best) { best = v; bi = i; }
    }
    rv[tid] = best;
    ri[tid] = bi;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
      if (tid < w) {
        const double o = rv[tid + w];
        const int oi = ri[tid + w];
        if (o > rv[tid] || (o == rv[tid] && oi < ri[tid])) { rv[tid] = o; ri[tid] = oi; }
      }
      __syncthreads();
    }
    const int p = ri[0];
    const double pv = rv[0];
    __syncthreads();
    if (!(pv > 0.0)) {
      if (tid == 0) atomicOr(flag, 2);
      continue;
    }
    if (p != j) {
      for (int c = tid; c < n2; c += nt) {
        const double a = W[(int64_t)j * n2 + c];
        W[(int64_t)j * n2 + c] = W[(int64_t)p * n2 + c];
        W[(int64_t)p * n2 + c] = a;
      }
    }
    __syncthreads();
    const double inv = 1.0 / W[(int64_t)j * n2 + j];
    __syncthreads();
    for (int c = tid; c < n2; c += nt) W[(int64_t)j * n2 + c] *= inv;
    for (int i = tid; i < n; i += nt) fcol[i] = W[(int64_t)i * n2 + j];
    __syncthreads();
    for (int64_t idx = tid; idx < (int64_t)n * n2; idx += nt) {
      const int i = (int)(idx / n2), c = (int)(idx % n2);
      if (i == j) continue;
      W[idx] -= fcol[i] * W[(int64_t)j * n2 + c];
    }
    __syncthreads();
  }
  for (int64_t idx = tid; idx < (int64_t)n * n; idx += nt) {
    const int i = (int)(idx / n), c = (int)(idx % n);
    d.Ainv[(int64_t)i * d.ldi + c] = W[(int64_t)i * n2 + n + c];
  }
}

rsrs_status gje_inverse(Uploader& up, hipStream_t st, const std::vector<GjeDesc>& e, int* flag) {
  if (e.empty()) return RSRS_OK;
  for (const auto& x : e)
    if (x.n > 4096) {
      set_error("Gauss-Jordan block larger than 4096");
      return RSRS_E_UNSUPPORTED;
    }
  GjeDesc* de = nullptr;
  RSRS_TRY(up.put_vec(e, &de));
  hipLaunchKernelGGL(gje_kernel, dim3((unsigned)e.size()), dim3(1024), 0, st, de, flag);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}

// ---------------------------------------------------------------- copies
__global__ void copy2d_kernel(const Copy2D* __restrict__ e) {
  const Copy2D d = e[blockIdx.y];
  const int64_t total = (int64_t)d.rows * d.cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / d.cols, c = idx % d.cols;
    const double v = d.alpha * d.src[i * d.lds + c];
    if (d.accumulate) d.dst[i * d.ldd + c] += v;
    else d.dst[i * d.ldd + c] = v;
  }
}

rsrs_status copy2d(Uploader& up, hipStream_t st, const std::vector<Copy2D>& e) {
  if (e.empty()) return RSRS_OK;
  int64_t mx = 0;
  for (const auto& x : e) mx = std::max<int64_t>(mx, (int64_t)x.rows * x.cols);
  if (mx == 0) return RSRS_OK;
  Copy2D* de = nullptr;
  RSRS_TRY(up.put_vec(e, &de));
  const unsigned gx = (unsigned)std::min<int64_t>((mx + 255) / 256, 4096);
  hipLaunchKernelGGL(copy2d_kernel, dim3(gx, (unsigned)e.size()), dim3(256), 0, st, de);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}

__global__ void gather_rows_kernel(double* dst, int64_t ldd, const double* src, int64_t lds,
                                   const int64_t* idx, int64_t nrows, int64_t ncols) {
  for (int64_t i = blockIdx.x; i < nrows; i += gridDim.x) {
    const double* s = src + idx[i] * lds;
    double* d = dst + i * ldd;
    for (int64_t c = threadIdx.x; c < ncols; c += blockDim.x) d[c] = s[c];
  }
}
__global__ void scatter_rows_kernel(double* dst, int64_t ldd, const double* src, int64_t lds,
                                    const int64_t* idx, int64_t nrows, int64_t ncols) {
  for (int64_t i = blockIdx.x; i < nrows; i += gridDim.x) {
    const double* s = src + i * lds;
    double* d = dst + idx[i] * ldd;
    for (int64_t c = threadIdx.x; c < ncols; c += blockDim.x) d[c] = s[c];
  }
}

void gather_rows(hipStream_t st, double* dst, int64_t ldd, const double* src, int64_t lds,
                 const int64_t* idx, int64_t nrows, int64_t ncols) {
  if (nrows <= 0 || ncols <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>(nrows, 65535);
  const unsigned b = ncols >= 256 ? 256 : (ncols >= 64 ? 64 : 32);
  hipLaunchKernelGGL(gather_rows_kernel, dim3(g), dim3(b), 0, st, dst, ldd, src, lds, idx, nrows, ncols);
}
void scatter_rows(hipStream_t st, double* dst, int64_t ldd, const double* src, int64_t lds,
                  const int64_t* idx, int64_t nrows, int64_t ncols) {
  if (nrows <= 0 || ncols <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>(nrows, 65535);
  const unsigned b = ncols >= 256 ? 256 : (ncols >= 64 ? 64 : 32);
  hipLaunchKernelGGL(scatter_rows_kernel, dim3(g), dim3(b), 0, st, dst, ldd, src, lds, idx, nrows, ncols);
}

__global__ void fill_kernel(double* p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
void fill(hipStream_t st, double* p, int64_t n, double v) {
  if (n <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(fill_kernel, dim3(g), dim3(256), 0, st, p, n, v);
}

__global__ void finite_kernel(const double* p, int64_t rows, int64_t cols, int64_t ld, int* flag) {
  bool bad = false;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < rows * cols;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const double v = p[(idx / cols) * ld + idx % cols];
    if (!isfinite(v)) bad = true;
  }
  if (bad) atomicOr(flag, 4);
}
void check_finite(hipStream_t st, const double* p, int64_t rows, int64_t cols, int64_t ld, int* flag) {
  if (rows <= 0 || cols <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>((rows * cols + 255) / 256, 8192);
  hipLaunchKernelGGL(finite_kernel, dim3(g), dim3(256), 0, st, p, rows, cols, ld, flag);
}

// column sums of squares: stage 1 -> partial[g][w], stage 2 -> out[w]
__global__ void colsq1_kernel(const double* x, int64_t n, int64_t w, int64_t ld, double* partial) {
  // block g handles rows g, g+G, ...; thread c handles column c (w <= 1024)
  for (int64_t c = threadIdx.x; c < w; c += blockDim.x) {
    double s = 0.0;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
      const double v = x[i * ld + c];
      s += v * v;
    }
    partial[(int64_t)blockIdx.x * w + c] = s;
  }
}
__global__ void colsq2_kernel(const double* partial, int64_t G, int64_t w, double* out) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < w; c += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t g = 0; g < G; ++g) s += partial[g * w + c];
    out[c] = s;
  }
}
rsrs_status col_sumsq(hipStream_t st, const double* x, int64_t n, int64_t w, int64_t ld,
                      double* partial, double* out) {
  const int64_t G = 256;
  hipLaunchKernelGGL(colsq1_kernel, dim3((unsigned)G), dim3(64), 0, st, x, n, w, ld, partial);
  hipLaunchKernelGGL(colsq2_kernel, dim3((unsigned)((w + 63) / 64)), dim3(64), 0, st, partial, G, w, out);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}

__global__ void sub2d_kernel(const double* f, int64_t ldf, const double* y, int64_t ldy, double* z,
                             int64_t ldz, int64_t n, int64_t w) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n * w;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / w, c = idx % w;
    z[i * ldz + c] = f[i * ldf + c] - y[i * ldy + c];
  }
}
void sub2d(hipStream_t st, const double* f, int64_t ldf, const double* y, int64_t ldy, double* z,
           int64_t ldz, int64_t n, int64_t w) {
  if (n <= 0 || w <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>((n * w + 255) / 256, 8192);
  hipLaunchKernelGGL(sub2d_kernel, dim3(g), dim3(256), 0, st, f, ldf, y, ldy, z, ldz, n, w);
}

}  // namespace rsrs
