// GMRES preconditioned by the factorization (Sec. 5 solves A u = f by GMRES
// with the inverse factorization as preconditioner and reports the
// iteration counts).  Right preconditioning: GMRES runs on A M^{-1} y = f,
// M^{-1} = A_approx^{-1} (rsrs_solve), x = M^{-1} y, so the residual it
// minimises is the true one, f - A x, through the black-box product.
//
// The columns of a block are independent GMRES runs advanced in lock step:
// every Arnoldi step is one preconditioner solve and one operator product
// for the whole block, the orthogonalisation is classical Gram-Schmidt
// applied twice (two passes of column-wise dot products and one multi-vector
// update each), and the small least-squares problems (Givens rotations of
// each column's Hessenberg matrix) run on the host.  A column stops growing
// its basis once its residual estimate meets the tolerance; the cycle ends
// when all have, or after `restart` steps, and restarts from the true
// residual.
//
// Layout: the basis vectors V_i are n x w row-major blocks (user order) at
// stride n w; all reductions are two-stage with a fixed order, so results do
// not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "impl.hpp"
#include "profile.hpp"

namespace rsrs {

rsrs_status apply_factor(const rsrs_factor_t* F, int op, int transpose, int64_t w, const double* Fin,
                         int64_t ldf, double* Uout, int64_t ldu, hipStream_t st);

namespace {

constexpr int kMaxCols = 64;     // columns per block
constexpr int kParts = 240;      // row chunks of the dot products (first stage)

// partial[b][i][c] = sum over the rows of chunk b of V_i[r][c] Y[r][c]
// (i < nv; V_i at V + i vstride; Y with leading dimension ldy).
__global__ __launch_bounds__(256) void block_dots_kernel(const double* __restrict__ V, int64_t vstride, int nv,
                                                         const double* __restrict__ Y, int64_t ldy, int64_t n,
                                                         int w, double* __restrict__ partial) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int rows_par = 256 / w;                  // rows handled side by side
  const int c = tid % w, ro = tid / w;
  const bool act = ro < rows_par;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = min(n, r0 + chunk);
  for (int i = 0; i < nv; ++i) {
    const double* Vi = V + (int64_t)i * vstride;
    double s = 0.0;
    if (act)
      for (int64_t r = r0 + ro; r < r1; r += rows_par) s += Vi[r * w + c] * Y[r * ldy + c];
    red[tid] = s;
    __syncthreads();
    if (tid < w) {   // the rows_par partial sums of column tid, in order
      double t = 0.0;
      for (int q = 0; q < rows_par; ++q) t += red[q * w + tid];
      partial[((int64_t)blockIdx.x * nv + i) * w + tid] = t;
    }
    __syncthreads();
  }
}

// out[i][c] = sum over chunks (in order) of partial[b][i][c]
__global__ void block_dots_sum_kernel(const double* __restrict__ partial, int nparts, int nv, int w,
                                      double* __restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nv * w) return;
  double t = 0.0;
  for (int b = 0; b < nparts; ++b) t += partial[(int64_t)b * nv * w + idx];
  out[idx] = t;
}

// Y[r][c] = beta Y[r][c] + alpha sum_{i < nv} h[i][c] V_i[r][c]
__global__ __launch_bounds__(256) void block_axpy_kernel(const double* __restrict__ V, int64_t vstride, int nv,
                                                         const double* __restrict__ h, double alpha, double beta,
                                                         double* __restrict__ Y, int64_t ldy, int64_t n, int w) {
  __shared__ double hs[(64 + 2) * kMaxCols];
  for (int t = threadIdx.x; t < nv * w; t += blockDim.x) hs[t] = h[t];
  __syncthreads();
  const int64_t total = n * w;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / w;
    const int c = (int)(e - r * w);
    double s = 0.0;
    for (int i = 0; i < nv; ++i) s += hs[i * w + c] * V[(int64_t)i * vstride + e];
    double* y = Y + r * ldy + c;
    *y = (beta != 0.0 ? beta * *y : 0.0) + alpha * s;
  }
}

// Y[r][c] = X[r][c] * s[c] (with leading dimensions)
__global__ void scale_cols_kernel(const double* __restrict__ X, int64_t ldx, const double* __restrict__ s,
                                  double* __restrict__ Y, int64_t ldy, int64_t n, int w) {
  const int64_t total = n * w;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / w;
    const int c = (int)(e - r * w);
    Y[r * ldy + c] = X[r * ldx + c] * s[c];
  }
}

// Y = F - Y (residual from the product Y = A X)
__global__ void resid_kernel(const double* __restrict__ F, int64_t ldf, double* __restrict__ Y, int64_t ldy,
                             int64_t n, int w) {
  const int64_t total = n * w;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / w;
    const int c = (int)(e - r * w);
    Y[r * ldy + c] = F[r * ldf + c] - Y[r * ldy + c];
  }
}

unsigned grid_for(int64_t total) {
  return (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
}

struct Gmres {
  hipStream_t st;
  int64_t n;
  int w;
  double *part, *dots;   // partial sums, reduced dots (nv x w)

  // out[i][c] = <V_i[:, c], Y[:, c]> for i < nv (device), two stages
  rsrs_status dots_with(const double* V, int64_t vstride, int nv, const double* Y, int64_t ldy) {
    {
      ProfScope ps(st, "gmres_dots", 2.0 * n * w * nv, 8.0 * n * w * (nv + 1));
      hipLaunchKernelGGL(block_dots_kernel, dim3(kParts), dim3(256), 0, st, V, vstride, nv, Y, ldy, n, w, part);
      hipLaunchKernelGGL(block_dots_sum_kernel, dim3((unsigned)((nv * w + 255) / 256)), dim3(256), 0, st, part,
                         kParts, nv, w, dots);
    }
    RSRS_HIP(hipGetLastError());
    return RSRS_OK;
  }
  rsrs_status axpy(const double* V, int64_t vstride, int nv, const double* h, double alpha, double beta,
                   double* Y, int64_t ldy) {
    {
      ProfScope ps(st, "gmres_axpy", 2.0 * n * w * nv, 8.0 * n * w * (nv + 2));
      hipLaunchKernelGGL(block_axpy_kernel, dim3(grid_for(n * w)), dim3(256), 0, st, V, vstride, nv, h, alpha,
                         beta, Y, ldy, n, w);
    }
    RSRS_HIP(hipGetLastError());
    return RSRS_OK;
  }
};

rsrs_status gmres_block(const rsrs_factor_t* f, rsrs_matvec_fn mv, void* user, int w, const double* F,
                        int64_t ldf, double* U, int64_t ldu, double tol, int m, int maxit, double* relres,
                        int* iters, hipStream_t st) {
  const int64_t n = f->n;
  const int64_t blk = n * w;
  DevBuf Vb, Tb, Wb, Pb, Db, Hb, Sb;
  RSRS_TRY(Vb.alloc((size_t)(m + 1) * blk * 8));
  RSRS_TRY(Tb.alloc((size_t)blk * 8));
  RSRS_TRY(Wb.alloc((size_t)blk * 8));
  RSRS_TRY(Pb.alloc((size_t)kParts * (m + 2) * w * 8));
  RSRS_TRY(Db.alloc((size_t)(m + 2) * w * 8));
  RSRS_TRY(Hb.alloc((size_t)(m + 2) * w * 8));
  RSRS_TRY(Sb.alloc((size_t)w * 8));
  double* V = Vb.as<double>();
  double* T = Tb.as<double>();
  double* Wv = Wb.as<double>();
  double* hd = Hb.as<double>();
  double* sd = Sb.as<double>();
  Gmres g{st, n, w, Pb.as<double>(), Db.as<double>()};

  auto matvec = [&](const double* X, int64_t ldx, double* Y) -> rsrs_status {
    if (mv(user, 0, RSRS_F64, w, X, ldx, Y, w, st) != 0) {
      set_error("matvec callback returned nonzero");
      return RSRS_E_CALLBACK;
    }
    return RSRS_OK;
  };
  auto to_host = [&](const double* d, double* h, size_t count) -> rsrs_status {
    RSRS_HIP(hipMemcpyAsync(h, d, count * 8, hipMemcpyDeviceToHost, st));
    RSRS_HIP(hipStreamSynchronize(st));
    return RSRS_OK;
  };

  // ||f|| per column; x = 0
  std::vector<double> fn(w), beta(w), hh((size_t)(m + 2) * w);
  {
    // the dot kernel reads V with leading dimension w: a compact copy of F
    RSRS_HIP(hipMemcpy2DAsync(Wv, (size_t)w * 8, F, (size_t)ldf * 8, (size_t)w * 8, (size_t)n,
                              hipMemcpyDeviceToDevice, st));
    RSRS_TRY(g.dots_with(Wv, 0, 1, Wv, w));
    RSRS_TRY(to_host(g.dots, fn.data(), (size_t)w));
    for (auto& x : fn) x = std::sqrt(x);
  }
  RSRS_HIP(hipMemset2DAsync(U, (size_t)ldu * 8, 0, (size_t)w * 8, (size_t)n, st));
  int it = 0;
  double rel = 0.0;
  std::vector<double> H((size_t)(m + 1) * m * w), cs((size_t)m * w), sn((size_t)m * w), gv((size_t)(m + 1) * w);
  std::vector<int> kc(w);     // basis size of each column in the current cycle
  std::vector<char> act(w);   // column not converged at the cycle's start
  std::vector<char> grow(w);  // column still growing its basis
  for (;;) {
    // true residual r = f - A x into Wv, its norms
    RSRS_TRY(matvec(U, ldu, Wv));
    hipLaunchKernelGGL(resid_kernel, dim3(grid_for(blk)), dim3(256), 0, st, F, ldf, Wv, (int64_t)w, n, w);
    RSRS_TRY(g.dots_with(Wv, 0, 1, Wv, w));
    RSRS_TRY(to_host(g.dots, beta.data(), (size_t)w));
    rel = 0.0;
    bool any = false;
    for (int c = 0; c < w; ++c) {
      beta[c] = std::sqrt(beta[c]);
      if (!std::isfinite(beta[c])) {
        set_error("non-finite residual in GMRES");
        return RSRS_E_NUMERIC;
      }
      const double d = fn[c] > 0.0 ? beta[c] / fn[c] : beta[c];
      rel = std::max(rel, d);
      act[c] = d > tol;
      any = any || act[c];
    }
    if (!any || it >= maxit) break;
    // V_0 = r / beta (columns already converged: zero)
    std::vector<double> inv(w);
    for (int c = 0; c < w; ++c) inv[c] = act[c] && beta[c] > 0.0 ? 1.0 / beta[c] : 0.0;
    RSRS_HIP(hipMemcpyAsync(sd, inv.data(), (size_t)w * 8, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(scale_cols_kernel, dim3(grid_for(blk)), dim3(256), 0, st, Wv, (int64_t)w, sd, V,
                       (int64_t)w, n, w);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(gv.begin(), gv.end(), 0.0);
    for (int c = 0; c < w; ++c) {
      gv[(size_t)c * (m + 1)] = act[c] ? beta[c] : 0.0;
      kc[c] = 0;
      grow[c] = act[c];
    }
    const int steps = std::min(m, maxit - it);
    for (int j = 0; j < steps; ++j) {
      // w_j = A M^{-1} v_j
      RSRS_TRY(apply_factor(f, 0, 0, w, V + (int64_t)j * blk, w, T, w, st));
      RSRS_TRY(matvec(T, w, Wv));
      // classical Gram-Schmidt, twice: h = V^T w, w -= V h
      RSRS_TRY(g.dots_with(V, blk, j + 1, Wv, w));
      RSRS_TRY(g.axpy(V, blk, j + 1, g.dots, -1.0, 1.0, Wv, w));
      RSRS_HIP(hipMemcpyAsync(hd, g.dots, (size_t)(j + 1) * w * 8, hipMemcpyDeviceToDevice, st));
      RSRS_TRY(g.dots_with(V, blk, j + 1, Wv, w));
      RSRS_TRY(g.axpy(V, blk, j + 1, g.dots, -1.0, 1.0, Wv, w));
      std::vector<double> h1((size_t)(j + 1) * w), h2((size_t)(j + 1) * w);
      RSRS_TRY(to_host(hd, h1.data(), h1.size()));
      RSRS_TRY(to_host(g.dots, h2.data(), h2.size()));
      RSRS_TRY(g.dots_with(Wv, 0, 1, Wv, w));
      std::vector<double> nr(w);
      RSRS_TRY(to_host(g.dots, nr.data(), (size_t)w));
      ++it;
      bool more = false;
      for (int c = 0; c < w; ++c) {
        const double hn = std::sqrt(nr[c]);
        inv[c] = 0.0;
        if (!grow[c]) continue;   // converged (or never active) in this cycle
        double* Hc = H.data() + (size_t)c * (m + 1) * m;   // (m+1) x m, column-major by step
        double* col = Hc + (size_t)j * (m + 1);
        for (int i = 0; i <= j; ++i) col[i] = h1[(size_t)i * w + c] + h2[(size_t)i * w + c];
        col[j + 1] = hn;
        double* csc = cs.data() + (size_t)c * m;
        double* snc = sn.data() + (size_t)c * m;
        for (int i = 0; i < j; ++i) {   // earlier rotations on the new column
          const double t = csc[i] * col[i] + snc[i] * col[i + 1];
          col[i + 1] = -snc[i] * col[i] + csc[i] * col[i + 1];
          col[i] = t;
        }
        const double den = std::hypot(col[j], col[j + 1]);
        csc[j] = den > 0.0 ? col[j] / den : 1.0;
        snc[j] = den > 0.0 ? col[j + 1] / den : 0.0;
        col[j] = den;
        col[j + 1] = 0.0;
        double* gc = gv.data() + (size_t)c * (m + 1);
        gc[j + 1] = -snc[j] * gc[j];
        gc[j] = csc[j] * gc[j];
        kc[c] = j + 1;
        const double est = std::fabs(gc[j + 1]) / (fn[c] > 0.0 ? fn[c] : 1.0);
        if (est > tol && hn > 0.0) {
          more = true;
          inv[c] = 1.0 / hn;
        } else {
          grow[c] = 0;
        }
      }
      if (!more || it >= maxit || j + 1 == steps) break;
      // v_{j+1} = w / ||w|| for the columns still growing
      RSRS_HIP(hipMemcpyAsync(sd, inv.data(), (size_t)w * 8, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(scale_cols_kernel, dim3(grid_for(blk)), dim3(256), 0, st, Wv, (int64_t)w, sd,
                         V + (int64_t)(j + 1) * blk, (int64_t)w, n, w);
    }
    // y_c = R_c^{-1} g_c for each column, x += M^{-1} (V y)
    int kmax = 0;
    for (int c = 0; c < w; ++c) kmax = std::max(kmax, kc[c]);
    std::vector<double> y((size_t)std::max(kmax, 1) * w, 0.0);
    for (int c = 0; c < w; ++c) {
      const int k = kc[c];
      const double* Hc = H.data() + (size_t)c * (m + 1) * m;
      const double* gc = gv.data() + (size_t)c * (m + 1);
      for (int i = k - 1; i >= 0; --i) {
        double s = gc[i];
        for (int l = i + 1; l < k; ++l) s -= Hc[(size_t)l * (m + 1) + i] * y[(size_t)l * w + c];
        const double d = Hc[(size_t)i * (m + 1) + i];
        y[(size_t)i * w + c] = d != 0.0 ? s / d : 0.0;
      }
    }
    if (kmax > 0) {
      RSRS_HIP(hipMemcpyAsync(hd, y.data(), y.size() * 8, hipMemcpyHostToDevice, st));
      RSRS_TRY(g.axpy(V, blk, kmax, hd, 1.0, 0.0, Wv, w));
      RSRS_TRY(apply_factor(f, 0, 0, w, Wv, w, T, w, st));
      std::vector<double> one(w, 1.0);
      RSRS_HIP(hipMemcpyAsync(sd, one.data(), (size_t)w * 8, hipMemcpyHostToDevice, st));
      RSRS_TRY(g.axpy(T, 0, 1, sd, 1.0, 1.0, U, ldu));
      RSRS_HIP(hipStreamSynchronize(st));   // host vectors above are released
    }
  }
  *relres = std::max(*relres, rel);
  *iters = std::max(*iters, it);
  return RSRS_OK;
}

}  // namespace
}  // namespace rsrs

using namespace rsrs;

extern "C" rsrs_status rsrs_solve_gmres(const rsrs_factor_t* f, rsrs_matvec_fn mv, void* user, int64_t nrhs,
                                        const double* F, int64_t ldf, double* U, int64_t ldu, double tol,
                                        int restart, int maxit, double* relres, int* iters, void* stream) {
  if (!f || !mv || !F || !U || nrhs < 1 || ldf < nrhs || ldu < nrhs || !(tol > 0.0) || restart < 1 ||
      restart > 64 || maxit < 1) {
    set_error("bad GMRES arguments");
    return RSRS_E_INVALID;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  double rel = 0.0;
  int it = 0;
  for (int64_t c0 = 0; c0 < nrhs; c0 += kMaxCols) {
    const int w = (int)std::min<int64_t>(kMaxCols, nrhs - c0);
    RSRS_TRY(gmres_block(f, mv, user, w, F + c0, ldf, U + c0, ldu, tol, restart, maxit, &rel, &it, st));
  }
  if (relres) *relres = rel;
  if (iters) *iters = it;
  return RSRS_OK;
}
