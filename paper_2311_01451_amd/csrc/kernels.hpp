// Launch interface of the HIP kernels (definitions in *.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "common.hpp"
#include "gemm.hpp"

namespace rsrs {

// Bump allocator over a pinned host buffer mirrored in device memory, used to
// ship per-launch descriptors and index lists.  Space is recycled only after
// reset(), which the caller issues right after a stream synchronisation.
struct Uploader {
  HostBuf h;
  DevBuf d;
  size_t off = 0;
  hipStream_t st = nullptr;
  rsrs_status init(size_t bytes, hipStream_t stream);
  // Copies n bytes to device; *dev receives the device address.
  rsrs_status put(const void* src, size_t n, void** dev);
  template <class T> rsrs_status put_vec(const std::vector<T>& v, T** dev) {
    void* p = nullptr;
    rsrs_status s = put(v.data(), v.size() * sizeof(T), &p);
    *dev = reinterpret_cast<T*>(p);
    return s;
  }
  rsrs_status reset();  // synchronises the stream, then recycles the space
};

// ---- GEMM (gemm.hpp) -------------------------------------------------------
enum GemmShape { GS_64x64 = 0, GS_64x16 = 1 };
// `site` (optional) is appended to the measurement tag ("gemm_<form>:<site>").
rsrs_status gemm(Uploader& up, hipStream_t st, const std::vector<GemmDesc>& descs, int ta,
                 int tb, int mode, GemmShape shape = GS_64x64, const char* site = nullptr);
inline GemmDesc gdesc(const double* A, const int64_t* ia, int64_t lda, const double* B,
                      const int64_t* ib, int64_t ldb, double* C, const int64_t* ic, int64_t ldc,
                      int M, int N, int K, double alpha = 1.0, double beta = 0.0,
                      const double* Cin = nullptr, const int64_t* icin = nullptr,
                      int64_t ldcin = 0) {
  GemmDesc d{};
  d.A = A; d.ia = ia; d.lda = lda;
  d.B = B; d.ib = ib; d.ldb = ldb;
  d.C = C; d.ic = ic; d.ldc = ldc;
  d.Cin = Cin ? Cin : C; d.icin = Cin ? icin : ic; d.ldcin = Cin ? ldcin : ldc;
  d.M = M; d.N = N; d.K = K;
  d.alpha = alpha; d.beta = beta;
  return d;
}

// ---- dense helpers (dense.hip) --------------------------------------------
struct CholLeaf { double* G; double* Li; int64_t ld; int n; int pad_; };
// Cholesky of each n x n (n <= 64) lower block G and the inverse of its factor
// into Li (full block, zeros above the diagonal).  flag[0] |= 1 when a pivot
// is not positive.
rsrs_status chol_leaf(Uploader& up, hipStream_t st, const std::vector<CholLeaf>& e, int* flag);

struct GjeDesc { const double* A; double* W; double* Ainv; int64_t lda, ldi; int n, pad_; };
// Inverse of each n x n matrix by Gauss-Jordan elimination with partial
// pivoting (W: n x 2n workspace).  flag[0] |= 2 on an exactly zero pivot.
rsrs_status gje_inverse(Uploader& up, hipStream_t st, const std::vector<GjeDesc>& e, int* flag);

struct Copy2D { const double* src; double* dst; int64_t lds, ldd; int rows, cols; double alpha; int accumulate, pad_; };
// dst = alpha*src (accumulate = 0) or dst += alpha*src.
rsrs_status copy2d(Uploader& up, hipStream_t st, const std::vector<Copy2D>& e);

// Row permutations: dst[i] = src[idx[i]] (gather) / dst[idx[i]] = src[i] (scatter).
void gather_rows(hipStream_t st, double* dst, int64_t ldd, const double* src, int64_t lds,
                 const int64_t* idx, int64_t nrows, int64_t ncols);
void scatter_rows(hipStream_t st, double* dst, int64_t ldd, const double* src, int64_t lds,
                  const int64_t* idx, int64_t nrows, int64_t ncols);
void fill(hipStream_t st, double* p, int64_t n, double v);
// flag[0] |= 4 if any entry of the rows x cols block is NaN/Inf.
void check_finite(hipStream_t st, const double* p, int64_t rows, int64_t cols, int64_t ld, int* flag);
// Column sums of squares of an N x w row-major block into out[w] (two-stage, deterministic).
rsrs_status col_sumsq(hipStream_t st, const double* x, int64_t n, int64_t w, int64_t ld,
                      double* partial, double* out);
// z = f - y (elementwise on N x w row-major blocks).
void sub2d(hipStream_t st, const double* f, int64_t ldf, const double* y, int64_t ldy, double* z,
           int64_t ldz, int64_t n, int64_t w);

// ---- interpolative decomposition (id.hip) ---------------------------------
struct IdDesc {
  double* M;          // b x s (the Y-side projection; the Z side is added in id_init)
  const double* MZ;   // b x s or null
  int64_t ldm, ldz;
  double* norms;      // 2*b
  int32_t* sel;       // b
  double* Rc;         // b x k
  int32_t* piv;       // k
  int64_t* Spos;      // k, sorted
  int64_t* Rpos;      // b-k, sorted
  double* T;          // (b-k) x k, row-major, leading dimension ldt
  int b, s, k, ldt;
};
rsrs_status id_run(Uploader& up, hipStream_t st, const std::vector<IdDesc>& e);

struct ColfixDesc {
  const double* XR;      // r x l (rows R of the least-squares coefficients, E applied)
  const int64_t* Spos;   // k
  const int64_t* Rpos;   // r
  const double* T;       // r x k
  double* Xp;            // r x l, columns ordered [R, S, N]
  int64_t ldx, ldp, ldt;
  int r, k, b, l;
};
// Columns of the extracted block: right-multiply by G^{-1} (columns R -= columns S T^T)
// and reorder to [R, S, N].
rsrs_status colfix(Uploader& up, hipStream_t st, const std::vector<ColfixDesc>& e);

// ---- random numbers and operators (ops.hip) -------------------------------
void philox_normal(hipStream_t st, double* out, int64_t nrows, int64_t ncols, int64_t ld,
                   uint64_t seed, uint32_t word);
struct KernelOp {
  int kind, dim;
  int64_t n;
  double p1, p2;
  DevBuf pts;       // n x dim
};
struct Poisson7Op {
  int n;
  DevBuf coef;      // N x 7: diag, -x, +x, -y, +y, -z, +z couplings
};
rsrs_status poisson_matvec(hipStream_t st, const Poisson7Op& op, int64_t ncols, const double* X,
                           int64_t ldx, double* Y, int64_t ldy);

}  // namespace rsrs
