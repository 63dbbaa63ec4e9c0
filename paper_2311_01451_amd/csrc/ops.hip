// Gaussian test matrices and the synthetic black-box operators.
//
// Gaussian generator: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11) written from its published
// definition, followed by the Box-Muller transform.  Entry (i, j) of a
// block uses counter (i, j, word, seed_hi) and key (seed_lo, 0x2311); the
// first two output words give u1, the last two u2 (53-bit uniforms in (0,1)),
// and the entry is sqrt(-2 ln u1) cos(2 pi u2).
//
// Operators: the kernel operators are materialised as explicit N x N matrices
// on the device and applied with the batched GEMM; the 7-point operator is a
// stencil kernel over stored per-node couplings.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kernels.hpp"
#include "profile.hpp"

namespace rsrs {

__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

template <typename T>
__global__ void philox_normal_kernel(T* out, int64_t nrows, int64_t ncols, int64_t ld,
                                     uint32_t seed_lo, uint32_t seed_hi, uint32_t word) {
  const int64_t total = nrows * ncols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / ncols, j = idx % ncols;
    uint32_t c[4] = {(uint32_t)i, (uint32_t)j, word, seed_hi};
    philox4x32_10(c, seed_lo, 0x2311u);
    const uint64_t a = ((uint64_t)c[0] << 21) ^ (uint64_t)(c[1] >> 11);   // 53 bits
    const uint64_t b = ((uint64_t)c[2] << 21) ^ (uint64_t)(c[3] >> 11);
    const double u1 = ((double)(a & ((1ull << 53) - 1)) + 0.5) * 0x1.0p-53;
    const double u2 = ((double)(b & ((1ull << 53) - 1)) + 0.5) * 0x1.0p-53;
    out[i * ld + j] = (T)(sqrt(-2.0 * log(u1)) * cospi(2.0 * u2));
  }
}

template <typename T>
void philox_normal(hipStream_t st, T* out, int64_t nrows, int64_t ncols, int64_t ld,
                   uint64_t seed, uint32_t word) {
  if (nrows <= 0 || ncols <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>((nrows * ncols + 255) / 256, 16384);
  ProfScope ps(st, "philox_normal", 0.0, (double)sizeof(T) * nrows * ncols);
  hipLaunchKernelGGL((philox_normal_kernel<T>), dim3(g), dim3(256), 0, st, out, nrows, ncols, ld,
                     (uint32_t)seed, (uint32_t)(seed >> 32), word);
}
template void philox_normal<double>(hipStream_t, double*, int64_t, int64_t, int64_t, uint64_t, uint32_t);
template void philox_normal<float>(hipStream_t, float*, int64_t, int64_t, int64_t, uint64_t, uint32_t);

// Entry (i, j) of the kernel operators (see include/rsrs.h for the formulas).
template <typename T>
__global__ void kernel_matrix_kernel(T* A, int64_t n, int kind, int dim, const double* pts,
                                     double p1, double p2) {
  const double two_pi = 6.283185307179586476925286766559;
  const double four_pi = 12.566370614359172953850573533118;
  const int64_t total = n * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / n, j = idx % n;
    double v;
    if (i == j) {
      if (kind == 4) {   // the kernel's mean over the point's cell of side p1
        const double ln2 = 0.69314718055994530941723212145818;
        const double mean_log_unit_square = 0.5 * (ln2 - 3.0 + 0.25 * two_pi) - ln2;
        v = p1 * p1 * (-log(p1) - mean_log_unit_square) / two_pi;
      } else {
        v = (kind == 2) ? 1.0 : 1.0 + 0.5 * p1 * p1;
      }
    } else {
      double r2 = 0.0, dx0 = 0.0;
      for (int a = 0; a < dim; ++a) {
        const double dd = pts[i * dim + a] - pts[j * dim + a];
        if (a == 0) dx0 = dd;
        r2 += dd * dd;
      }
      const double r = sqrt(r2);
      if (kind == 2) {
        v = (1.0 / (double)n) / (four_pi * r);
      } else {
        v = p1 * p1 * (-log(r) / two_pi);
        if (kind == 3) v += p2 * dx0 / r2;
      }
    }
    A[idx] = (T)v;
  }
}

template <typename T>
rsrs_status kernel_materialise(hipStream_t st, const KernelOp& op, T* A) {
  const int64_t total = op.n * op.n;
  const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL((kernel_matrix_kernel<T>), dim3(g), dim3(256), 0, st, A, op.n, op.kind, op.dim,
                     op.pts.as<double>(), op.p1, op.p2);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}
template rsrs_status kernel_materialise<double>(hipStream_t, const KernelOp&, double*);
template rsrs_status kernel_materialise<float>(hipStream_t, const KernelOp&, float*);

// 7-point stencil: Y[i][c] = sum_t coef[i][t] X[nbr_t(i)][c], t = 0 is the node itself.
template <typename T>
__global__ void poisson_kernel(const double* coef, int n, int64_t w, const T* X, int64_t ldx,
                               T* Y, int64_t ldy) {
  const int64_t N = (int64_t)n * n * n;
  const int64_t total = N * w;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / w, c = idx % w;
    const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((int64_t)n * n));
    const double* cf = coef + i * 7;
    double v = cf[0] * (double)X[i * ldx + c];
    if (x > 0) v += cf[1] * (double)X[(i - 1) * ldx + c];
    if (x < n - 1) v += cf[2] * (double)X[(i + 1) * ldx + c];
    if (y > 0) v += cf[3] * (double)X[(i - n) * ldx + c];
    if (y < n - 1) v += cf[4] * (double)X[(i + n) * ldx + c];
    if (z > 0) v += cf[5] * (double)X[(i - (int64_t)n * n) * ldx + c];
    if (z < n - 1) v += cf[6] * (double)X[(i + (int64_t)n * n) * ldx + c];
    Y[i * ldy + c] = (T)v;
  }
}

template <typename T>
rsrs_status poisson_matvec(hipStream_t st, const Poisson7Op& op, int64_t ncols, const T* X,
                           int64_t ldx, T* Y, int64_t ldy) {
  const int64_t N = (int64_t)op.n * op.n * op.n;
  const unsigned g = (unsigned)std::min<int64_t>((N * ncols + 255) / 256, 65536);
  ProfScope ps(st, "poisson7", 13.0 * N * ncols, 56.0 * N + 2.0 * sizeof(T) * N * ncols);
  hipLaunchKernelGGL((poisson_kernel<T>), dim3(g), dim3(256), 0, st, op.coef.as<double>(), op.n, ncols,
                     X, ldx, Y, ldy);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}
template rsrs_status poisson_matvec<double>(hipStream_t, const Poisson7Op&, int64_t, const double*, int64_t, double*, int64_t);
template rsrs_status poisson_matvec<float>(hipStream_t, const Poisson7Op&, int64_t, const float*, int64_t, float*, int64_t);

}  // namespace rsrs
