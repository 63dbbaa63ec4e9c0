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
  // pooled: staging taken from (and later recycled into) the scratch pool
  rsrs_status init(size_t bytes, hipStream_t stream, bool pooled = false);
  // Copies n bytes to device; *dev receives the device address.
  rsrs_status put(const void* src, size_t n, void** dev);
  template <class T> rsrs_status put_vec(const std::vector<T>& v, T** dev) {
    void* p = nullptr;
    rsrs_status s = put(v.data(), v.size() * sizeof(T), &p);
    *dev = reinterpret_cast<T*>(p);
    return s;
  }
  rsrs_status reset();  // synchronises the stream, then recycles the space
  void recycle();       // hands both buffers to the scratch pool (stream drained)
};

// ---- GEMM (gemm.hpp) -------------------------------------------------------
// GS_64x64: 64 x 64 tiles, or 128 x 128 when the launch has >= 256 of those;
// GS_64x64_ONLY: always 64 x 64 (narrow outputs); GS_64x16: narrow solves.
enum GemmShape { GS_64x64 = 0, GS_64x16 = 1, GS_64x64_ONLY = 2 };
// `site` (optional) is appended to the measurement tag ("gemm_<form>:<site>").
// A batched product split into launch records: kernel, grid, and the first
// descriptor (index into the caller's concatenated descriptor array) it reads.
struct GemmLaunch {
  const void* fn;
  dim3 grid, block;
  size_t first;
  double flops, bytes;   // algorithmic work (for the measurement tags)
  uint64_t sig;          // shape signature of the whole product (tile tuning)
  int shape;             // tile shape planned (0 64x64, 1 128x64, 2 128x128, 3 64x16)
  char tag[48];
};
// Plans descs (whose first element sits at index `base` of the caller's array);
// instantiated for <double, double> and <float, float>.
template <typename TI, typename TO>
rsrs_status gemm_plan(const std::vector<GemmDescT<TI, TO>>& descs, size_t base, int ta, int tb, int mode,
                      GemmShape shape, const char* site, std::vector<GemmLaunch>& out);
// Tile autotuning of the automatic choice (see dense.hip) and a forced shape
// for every automatic launch (-1: table or rule, -2: forget the table).
rsrs_status gemm_autotune(const char* cache_path, int64_t* entries, int64_t* changed);
rsrs_status gemm_tile_override(int shape);
// Workload tuning: while recording, every automatic launch is timed by HIP
// events under its product's shape signature; gemm_sig_collect sums the
// recorded milliseconds per signature (and the shape each one took) once the
// work has finished; gemm_sig_install makes the given shape serve each
// signature from then on (an exact match overrides the class table).
void gemm_sig_record(bool on);
rsrs_status gemm_sig_collect(std::vector<std::pair<uint64_t, double>>& ms,
                             std::vector<std::pair<uint64_t, int>>& shape);
void gemm_sig_install(const std::vector<std::pair<uint64_t, int>>& table, bool replace);
int64_t gemm_sig_count();
// Launches one record; descs is the device copy of the caller's array.
rsrs_status gemm_exec(const GemmLaunch& L, const void* descs, size_t desc_bytes, hipStream_t st);
// Instantiated for <double, double> and <float, float> (all forms).
template <typename TI, typename TO>
rsrs_status gemm(Uploader& up, hipStream_t st, const std::vector<GemmDescT<TI, TO>>& descs, int ta,
                 int tb, int mode, GemmShape shape = GS_64x64, const char* site = nullptr);
inline rsrs_status gemm(Uploader& up, hipStream_t st, const std::vector<GemmDesc>& descs, int ta,
                        int tb, int mode, GemmShape shape = GS_64x64, const char* site = nullptr) {
  return gemm<double, double>(up, st, descs, ta, tb, mode, shape, site);
}
template <typename TI, typename TO>
inline GemmDescT<TI, TO> gdescT(const TI* A, const int64_t* ia, int64_t lda, const TI* B,
                                const int64_t* ib, int64_t ldb, TO* C, const int64_t* ic,
                                int64_t ldc, int M, int N, int K, double alpha = 1.0,
                                double beta = 0.0, const TO* Cin = nullptr,
                                const int64_t* icin = nullptr, int64_t ldcin = 0) {
  GemmDescT<TI, TO> d{};
  d.A = A; d.ia = ia; d.lda = lda;
  d.B = B; d.ib = ib; d.ldb = ldb;
  d.C = C; d.ic = ic; d.ldc = ldc;
  d.Cin = Cin ? Cin : C; d.icin = Cin ? icin : ic; d.ldcin = Cin ? ldcin : ldc;
  d.M = M; d.N = N; d.K = K;
  d.alpha = alpha; d.beta = beta;
  return d;
}
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
template <typename T> struct CholMatT { T* G; T* W; int64_t ld; int n; };
using CholMat = CholMatT<double>;
// Cholesky G = L L^T of each n x n matrix (lower part of G read) and the
// inverse factor: on return G holds L^{-1} in its lower part (the upper part
// of its 64 x 64 diagonal blocks zero, the rest of the upper part
// unspecified); W (same shape) is scratch.  flag[0] |= 1 when a pivot is not
// positive.  Instantiated for double and float (FP64 / FP32 MFMA).
template <typename T>
rsrs_status chol_inverse(Uploader& up, hipStream_t st, const std::vector<CholMatT<T>>& mats, int* flag);

struct GjeDesc { const double* A; double* W; double* Ainv; int64_t lda, ldi; int n, pad_; };
// Inverse of each n x n matrix by Gauss-Jordan elimination with partial
// pivoting (W: 2 n^2 workspace).  flag[0] |= 2 on an exactly zero pivot.
rsrs_status gje_inverse(Uploader& up, hipStream_t st, const std::vector<GjeDesc>& e, int* flag);

// Y (M x N) = A (M x K) X (K x N), FP64, for narrow X (N <= 16) on a dense
// row-major A: K split in 8 chunks (K a multiple of 2048), partial products
// in scratch (skinny_f64_scratch(M) bytes) summed in chunk order.
bool skinny_f64_ok(const double* A, int64_t lda, int64_t M, int64_t K, int64_t N);
size_t skinny_f64_scratch(int64_t M);
rsrs_status skinny_f64(hipStream_t st, const double* A, int64_t lda, int64_t M, int64_t K, const double* X,
                       int64_t ldx, int64_t N, double* Y, int64_t ldy, double* scratch);

template <typename TS, typename TD>
struct Copy2DT { const TS* src; TD* dst; int64_t lds, ldd; int rows, cols; double alpha; int accumulate, trans; };
using Copy2D = Copy2DT<double, double>;
// dst = alpha*src (accumulate = 0) or dst += alpha*src, converting the element
// type; with trans, src is read transposed (dst is rows x cols, src cols x rows).
// Instantiated for every pair of double / float.
template <typename TS, typename TD>
rsrs_status copy2d(Uploader& up, hipStream_t st, const std::vector<Copy2DT<TS, TD>>& e);
inline rsrs_status copy2d(Uploader& up, hipStream_t st, const std::vector<Copy2D>& e) {
  return copy2d<double, double>(up, st, e);
}

// In-place symmetric part A = (A + A^T) / 2 of n x n blocks (double / float).
template <typename T>
struct SymDesc { T* A; int64_t ld; int n, pad_; };
template <typename T>
rsrs_status symmetrize(Uploader& up, hipStream_t st, const std::vector<SymDesc<T>>& e);

// Row permutations: dst[i] = src[idx[i]] (gather) / dst[idx[i]] = src[i]
// (scatter), converting the element type (double / float pairs).
template <typename TS, typename TD>
void gather_rows(hipStream_t st, TD* dst, int64_t ldd, const TS* src, int64_t lds,
                 const int64_t* idx, int64_t nrows, int64_t ncols);
template <typename TS, typename TD>
void scatter_rows(hipStream_t st, TD* dst, int64_t ldd, const TS* src, int64_t lds,
                  const int64_t* idx, int64_t nrows, int64_t ncols);
void fill(hipStream_t st, double* p, int64_t n, double v);
// flag[0] |= 4 if any entry of the rows x cols block is NaN/Inf (double / float).
template <typename T>
void check_finite(hipStream_t st, const T* p, int64_t rows, int64_t cols, int64_t ld, int* flag);
// Column sums of squares of an N x w row-major block into out[w] (two-stage, deterministic).
rsrs_status col_sumsq(hipStream_t st, const double* x, int64_t n, int64_t w, int64_t ld,
                      double* partial, double* out);
// z = f - y (elementwise on N x w row-major blocks).
void sub2d(hipStream_t st, const double* f, int64_t ldf, const double* y, int64_t ldy, double* z,
           int64_t ldz, int64_t n, int64_t w);

// ---- interpolative decomposition (id.hip) ---------------------------------
struct IdDesc {
  // Working rows, b x s, FP64 or FP32 storage (all descriptors of one call
  // alike): the Y-side projection, overwritten by the residuals; MZ (same
  // type, or null) is added to it by the first launch.  Dot products, norms
  // and coefficients are FP64 in both cases.
  void* M;
  const void* MZ;
  int64_t ldm, ldz;
  double* norms;      // 2*b
  int32_t* sel;       // b
  double* Rc;         // b x k
  int32_t* piv;       // k
  int64_t* Spos;      // b: the k_B skeleton positions (sorted), then the b - k_B others (sorted)
  int64_t* kB;        // out: k_B
  double* T;          // (b - k_B) x k_B, row-major, leading dimension ldt
  // Rank tolerance (tol2 > 0): k_B = the number of leading steps whose pivot
  // norm^2 exceeds tol2 * sum_i rowyz[i]; rowyz[i] = |Y_B row i|^2 (+ |Z_B
  // row i|^2), gathered by the first launch from rows idx of Yg (and Zg).
  double tol2;
  double* rowyz;      // b
  const void* Yg;
  const void* Zg;
  const int64_t* idx;
  int64_t ldy;
  int sy;
  int b, s, k, ldt;   // k: steps (k_B <= k <= b)
  // Gram route (FP32 rows): the rows in FP64 (b x s, leading dimension
  // ldmd) and their Gram matrix M M^T (b x b, lower part, leading dimension ldg)
  double* Md;
  double* G;
  double* Rt;   // the R entries column-major (k x b), scratch of the Gram route
  int64_t ldmd, ldg;
};

rsrs_status id_run(Uploader& up, hipStream_t st, const std::vector<IdDesc>& e, bool fp32);
// FP32 rows only: the same decomposition through the FP64 Gram matrix of the
// rows (pivoted Cholesky, all steps of a box in one workgroup).  G holds
// kIdGramSplit partial Gram matrices (b x ldg each, back to back).
constexpr int kIdGramSplit = 4;
rsrs_status id_run_gram(Uploader& up, hipStream_t st, const std::vector<IdDesc>& e);

template <typename T>
struct ColfixDescT {
  const T* XR;           // r x l (rows R of the least-squares coefficients, E applied)
  const int64_t* Spos;   // k
  const int64_t* Rpos;   // r
  const T* T_;           // r x k
  T* Xp;                 // r x l, columns ordered [R, S, N]
  int64_t ldx, ldp, ldt;
  int r, k, b, l;
};
using ColfixDesc = ColfixDescT<double>;
// Columns of the extracted block: right-multiply by G^{-1} (columns R -= columns S T^T)
// and reorder to [R, S, N] (double or float).
template <typename T>
rsrs_status colfix(Uploader& up, hipStream_t st, const std::vector<ColfixDescT<T>>& e);

// ---- random numbers and operators (ops.hip) -------------------------------
// Standard normals (double or float output; the float value is the rounded
// double draw).
template <typename T>
void philox_normal(hipStream_t st, T* out, int64_t nrows, int64_t ncols, int64_t ld,
                   uint64_t seed, uint32_t word);
// BF16 products (bf16.hip): Y (M x N float) = A (M x K bf16) X (K x N float
// holding BF16 values), FP32 accumulation, with Xt (N x ldt bf16) as workspace.
// Whether wide products of the built-in dense operators may go to rocBLAS /
// hipBLASLt (default true; rsrs_op_library_gemm).
bool operator_library_gemm();
void set_operator_library_gemm(bool on);
rsrs_status gemm_bf16_op(hipStream_t st, const uint16_t* A, int64_t lda, int64_t M, int64_t K,
                         const float* X, int64_t ldx, int64_t N, float* Y, int64_t ldy, uint16_t* Xt,
                         int64_t ldt);
rsrs_status bf16_from_f64(hipStream_t st, const double* src, uint16_t* dst, int64_t n);
// Rounds every entry of a float block to the nearest BF16 value (kept as float).
void round_to_bf16_values(hipStream_t st, float* x, int64_t rows, int64_t cols, int64_t ld);

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
template <typename T>
rsrs_status poisson_matvec(hipStream_t st, const Poisson7Op& op, int64_t ncols, const T* X,
                           int64_t ldx, T* Y, int64_t ldy);

}  // namespace rsrs
