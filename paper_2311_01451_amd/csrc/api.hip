// extern "C" entry points of include/rsrs.h.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <unordered_map>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "impl.hpp"
#include "profile.hpp"

namespace rsrs {

static thread_local std::string g_err;
static thread_local int64_t g_req_s = -1;
void set_error(const std::string& msg) { g_err = msg; }
void set_required_s(int64_t s) { g_req_s = s; }

rsrs_status apply_factor_noalloc(const rsrs_factor_t* F, int op, int transpose, int64_t w, const double* Fin,
                                 int64_t ldf, double* Uout, int64_t ldu, hipStream_t st);
rsrs_status apply_factor(const rsrs_factor_t* F, int op, int transpose, int64_t w, const double* Fin,
                         int64_t ldf, double* Uout, int64_t ldu, hipStream_t st);

static int64_t dtype_size(int dtype) {
  return dtype == RSRS_F64 ? 8 : ((dtype == RSRS_F32 || dtype == RSRS_BF16) ? 4 : 0);
}

static rsrs_status invalid(const char* msg) {
  set_error(msg);
  return RSRS_E_INVALID;
}

// Wide products of a dense operator matrix are plain library GEMMs: rocBLAS
// when it takes them (one handle per device, kept for the process), the own
// GEMM otherwise.  In column-major terms Y^T (w x n) = X^T (w x n) * A^T,
// A (n x n, row-major) being A^T column-major: op N for A, op T for A^T.
struct RbDev {
  std::mutex mu;
  bool tried = false, ok = false;
  rocblas_handle h = nullptr;
};
template <typename T>
bool rb_operator_product(hipStream_t st, const T* A, int64_t lda, int64_t n, int ta, const T* X, int64_t ldx,
                         int64_t w, T* Y, int64_t ldy) {
  if (n > INT32_MAX || w > INT32_MAX || lda > INT32_MAX || ldx > INT32_MAX || ldy > INT32_MAX) return false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  static RbDev devs[64];
  RbDev& R = devs[dev & 63];
  std::lock_guard<std::mutex> lk(R.mu);   // the handle's stream is set per call
  if (!R.tried) {
    R.tried = true;
    R.ok = rocblas_create_handle(&R.h) == rocblas_status_success;
  }
  if (!R.ok || rocblas_set_stream(R.h, st) != rocblas_status_success) return false;
  const T one = 1, zero = 0;
  const rocblas_operation ob = ta ? rocblas_operation_transpose : rocblas_operation_none;
  rocblas_status r;
  if constexpr (sizeof(T) == 8)
    r = rocblas_dgemm(R.h, rocblas_operation_none, ob, (rocblas_int)w, (rocblas_int)n, (rocblas_int)n, &one, X,
                      (rocblas_int)ldx, A, (rocblas_int)lda, &zero, Y, (rocblas_int)ldy);
  else
    r = rocblas_sgemm(R.h, rocblas_operation_none, ob, (rocblas_int)w, (rocblas_int)n, (rocblas_int)n, &one, X,
                      (rocblas_int)ldx, A, (rocblas_int)lda, &zero, Y, (rocblas_int)ldy);
  return r == rocblas_status_success;
}
}  // namespace rsrs

using namespace rsrs;

extern "C" {

const char* rsrs_status_string(rsrs_status st) {
  switch (st) {
    case RSRS_OK: return "ok";
    case RSRS_E_INVALID: return "invalid argument";
    case RSRS_E_SAMPLES: return "insufficient samples";
    case RSRS_E_SINGULAR: return "singular block";
    case RSRS_E_CALLBACK: return "matvec callback failed";
    case RSRS_E_NUMERIC: return "non-finite value";
    case RSRS_E_NOMEM: return "out of device memory";
    case RSRS_E_HIP: return "HIP runtime error";
    case RSRS_E_UNSUPPORTED: return "unsupported option";
    case RSRS_E_TIMEOUT: return "timed out";
  }
  return "unknown status";
}

const char* rsrs_last_error(void) { return g_err.c_str(); }
int64_t rsrs_last_required_s(void) { return g_req_s; }

// ------------------------------------------------------------------ tree
rsrs_status rsrs_build_tree(const double* pts, int64_t n, const rsrs_tree_opts* o, rsrs_tree_t** out) {
  if (!pts || !o || !out) return invalid("null argument");
  *out = nullptr;
  auto t = new rsrs_tree_t();
  std::string err = build_tree(pts, n, o->dim, o->leaf_size, o->qbits, o->root_lo, o->root_side, t->t);
  if (!err.empty()) {
    delete t;
    return invalid(err.c_str());
  }
  *out = t;
  return RSRS_OK;
}

void rsrs_tree_destroy(rsrs_tree_t* t) { delete t; }

rsrs_status rsrs_tree_get_info(const rsrs_tree_t* th, rsrs_tree_info* out) {
  if (!th || !out) return invalid("null argument");
  const Tree& t = th->t;
  out->dim = t.dim;
  out->nlevels = t.nlevels;
  out->qbits = t.qbits;
  out->n = t.n;
  out->nbox = t.nbox();
  out->level = t.level.data();
  out->coords = t.coords.data();
  out->parent = t.parent.data();
  out->is_leaf = t.is_leaf.data();
  out->pt_begin = t.pt_begin.data();
  out->pt_end = t.pt_end.data();
  out->perm = t.perm.data();
  return RSRS_OK;
}

rsrs_status rsrs_tree_neighbours(const rsrs_tree_t* th, int level, int64_t* nb, const int64_t** boxes,
                                 const int64_t** offsets, const int64_t** nbrs) {
  if (!th || !nb || !boxes || !offsets || !nbrs) return invalid("null argument");
  const Tree& t = th->t;
  if (level < 1 || level > t.nlevels) return invalid("level out of range");
  *nb = (int64_t)t.level_boxes[level].size();
  *boxes = t.level_boxes[level].data();
  *offsets = t.nb_off[level].data();
  *nbrs = t.nb_ids[level].data();
  return RSRS_OK;
}

rsrs_status rsrs_tree_schedule(const rsrs_tree_t* th, int k, int32_t* colour, int64_t* b_count,
                               int64_t* l_count, int64_t* root_count) {
  if (!th || k < 1) return invalid("bad tree or k");
  Schedule s;
  make_schedule(th->t, k, s);
  const size_t nb = (size_t)th->t.nbox();
  if (colour) std::memcpy(colour, s.colour.data(), nb * 4);
  if (b_count) std::memcpy(b_count, s.b_count.data(), nb * 8);
  if (l_count) std::memcpy(l_count, s.l_count.data(), nb * 8);
  if (root_count) *root_count = s.root_count;
  return RSRS_OK;
}

int64_t rsrs_samples_required(const rsrs_tree_t* th, int k, int p) {
  if (!th || k < 1 || p < 0) return -1;
  Schedule s;
  make_schedule(th->t, k, s);
  return samples_required(th->t, s, k, p);
}

rsrs_status rsrs_work_model(const rsrs_tree_t* th, const rsrs_factor_opts* o, int64_t s, int esize,
                            double* flops, double* bytes, int64_t* stored_entries) {
  if (!th || !o || o->k < 1 || s < 1 || (esize != 4 && esize != 8)) return invalid("bad tree, options, s or element size");
  Schedule sc;
  make_schedule(th->t, o->k, sc);
  const int p = o->p < 0 ? o->k : o->p;
  work_model(th->t, sc, o->k, s, o->symmetric != 0, esize, o->col_subset ? p : -1, flops, bytes, stored_entries);
  return RSRS_OK;
}

rsrs_status rsrs_gemm_autotune(const char* cache_path, int64_t* entries, int64_t* changed) {
  return gemm_autotune(cache_path, entries, changed);
}

rsrs_status rsrs_gemm_tile_override(int shape) { return gemm_tile_override(shape); }

// ------------------------------------------------------------------ operators
rsrs_status rsrs_op_create_kernel(int kind, const double* pts, int64_t n, int dim, double param,
                                  double param2, rsrs_operator_t** out) {
  if (!pts || !out || n < 1) return invalid("bad operator arguments");
  if (!((kind == RSRS_OP_LOG2D && dim == 2) || (kind == RSRS_OP_LOG2D_SKEW && dim == 2) ||
        (kind == RSRS_OP_LOG2D_FIRST && dim == 2) || (kind == RSRS_OP_INVR3D && dim == 3)))
    return invalid("unknown operator kind or wrong dimension");
  *out = nullptr;
  auto op = new rsrs_operator_t();
  op->kind = kind;
  op->n = n;
  op->lda = n;
  op->symmetric = kind != RSRS_OP_LOG2D_SKEW;
  KernelOp& ko = op->kop;
  ko.kind = kind;
  ko.dim = dim;
  ko.n = n;
  ko.p1 = param;
  ko.p2 = param2;
  rsrs_status s = ko.pts.alloc((size_t)n * dim * 8);
  if (s == RSRS_OK) s = op->owned.alloc((size_t)n * n * 8);
  if (s != RSRS_OK) { delete op; return s; }
  if (hipMemcpy(ko.pts.p, pts, (size_t)n * dim * 8, hipMemcpyHostToDevice) != hipSuccess) {
    delete op;
    set_error("hipMemcpy of points failed");
    return RSRS_E_HIP;
  }
  s = kernel_materialise<double>(nullptr, ko, op->owned.as<double>());
  if (s == RSRS_OK && hipDeviceSynchronize() != hipSuccess) s = RSRS_E_HIP;
  if (s != RSRS_OK) { delete op; return s; }
  op->A = op->owned.as<double>();
  *out = op;
  return RSRS_OK;
}

rsrs_status rsrs_op_create_dense(const double* A, int64_t n, int64_t lda, rsrs_operator_t** out) {
  if (!A || !out || n < 1 || lda < n) return invalid("bad dense operator arguments");
  auto op = new rsrs_operator_t();
  op->kind = 10;
  op->n = n;
  op->A = A;
  op->lda = lda;
  op->symmetric = false;
  *out = op;
  return RSRS_OK;
}

rsrs_status rsrs_op_create_poisson7(int n, const double* coef, rsrs_operator_t** out) {
  if (!coef || !out || n < 1) return invalid("bad poisson arguments");
  const int64_t N = (int64_t)n * n * n;
  const int m = n + 2;
  const double h = 1.0 / (n + 1), ih2 = 1.0 / (h * h);
  std::vector<double> c((size_t)N * 7, 0.0);
  auto a = [&](int z, int y, int x) { return coef[((int64_t)z * m + y) * m + x]; };
  for (int z = 0; z < n; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const int64_t i = ((int64_t)z * n + y) * n + x;
        const double ai = a(z + 1, y + 1, x + 1);
        const double nb[6] = {a(z + 1, y + 1, x), a(z + 1, y + 1, x + 2), a(z + 1, y, x + 1),
                              a(z + 1, y + 2, x + 1), a(z, y + 1, x + 1), a(z + 2, y + 1, x + 1)};
        double d = 0.0;
        for (int f = 0; f < 6; ++f) {
          const double face = 0.5 * (ai + nb[f]) * ih2;
          d += face;
          c[i * 7 + 1 + f] = -face;
        }
        c[i * 7] = d;
      }
  auto op = new rsrs_operator_t();
  op->kind = 20;
  op->n = N;
  op->pois.n = n;
  rsrs_status s = op->pois.coef.alloc(c.size() * 8);
  if (s != RSRS_OK) { delete op; return s; }
  if (hipMemcpy(op->pois.coef.p, c.data(), c.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
    delete op;
    set_error("hipMemcpy failed");
    return RSRS_E_HIP;
  }
  *out = op;
  return RSRS_OK;
}

int rsrs_op_matvec(void* opv, int transpose, int dtype, int64_t ncols, const void* X, int64_t ldx,
                   void* Y, int64_t ldy, void* stream) {
  auto op = static_cast<rsrs_operator_t*>(opv);
  if (!op || !X || !Y || ncols < 0 || dtype_size(dtype) == 0) return 1;
  if (ncols == 0) return 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (op->kind == 20) {   // BF16 requests get the (more accurate) FP32 product
    if (dtype == RSRS_F64)
      return poisson_matvec<double>(st, op->pois, ncols, static_cast<const double*>(X), ldx,
                                    static_cast<double*>(Y), ldy) == RSRS_OK ? 0 : 1;
    return poisson_matvec<float>(st, op->pois, ncols, static_cast<const float*>(X), ldx,
                                 static_cast<float*>(Y), ldy) == RSRS_OK ? 0 : 1;
  }
  if (!op->up_ready) {
    if (op->up.init((size_t)1 << 20, st) != RSRS_OK) return 1;
    op->up_ready = true;
  }
  if (op->up.st != st) {
    if (op->up.reset() != RSRS_OK) return 1;
    op->up.st = st;
  }
  const int n = (int)op->n;
  const int ta = (transpose && !op->symmetric) ? 1 : 0;
  const GemmShape shp = ncols <= 16 ? GS_64x16 : GS_64x64;
  if (dtype == RSRS_F64 && ta == 0 && skinny_f64_ok(op->A, op->lda, n, n, ncols)) {
    // narrow products (refinement residuals) stream the matrix once
    if (op->skinny.bytes < skinny_f64_scratch(n) && op->skinny.alloc(skinny_f64_scratch(n)) != RSRS_OK) return 1;
    return skinny_f64(st, op->A, op->lda, n, n, static_cast<const double*>(X), ldx, ncols, static_cast<double*>(Y),
                      ldy, op->skinny.as<double>()) == RSRS_OK ? 0 : 1;
  }
  if (dtype == RSRS_F64) {
    if (ncols > 16 && operator_library_gemm()) {
      ProfScope ps(st, "rocblas_dgemm:operator", 2.0 * n * n * ncols, 8.0 * ((double)n * n + 2.0 * n * ncols));
      if (rb_operator_product<double>(st, op->A, op->lda, n, ta, static_cast<const double*>(X), ldx, ncols,
                                      static_cast<double*>(Y), ldy))
        return 0;
    }
    std::vector<GemmDesc> d{gdesc(op->A, nullptr, op->lda, static_cast<const double*>(X), nullptr, ldx,
                                  static_cast<double*>(Y), nullptr, ldy, n, (int)ncols, n)};
    return gemm(op->up, st, d, ta, 0, GM_FULL, shp, "operator") == RSRS_OK ? 0 : 1;
  }
  if (op->kind == 10) {
    set_error("a borrowed dense operator provides FP64 products only");
    return 1;
  }
  if (dtype == RSRS_BF16 && ta == 0 && op->n <= INT32_MAX && op->n % 8 == 0) {
    // kernel matrix rounded to BF16, FP32 accumulation
    if (!op->owned16.p) {
      if (op->owned16.alloc((size_t)op->n * op->n * 2) != RSRS_OK) return 1;
      if (bf16_from_f64(st, op->A, op->owned16.as<uint16_t>(), op->n * op->n) != RSRS_OK) return 1;
    }
    const int64_t ldt = round_up(op->n, 8);
    if (op->xt16.alloc((size_t)ncols * ldt * 2) != RSRS_OK) return 1;
    return gemm_bf16_op(st, op->owned16.as<uint16_t>(), op->n, op->n, op->n, static_cast<const float*>(X),
                        ldx, ncols, static_cast<float*>(Y), ldy, op->xt16.as<uint16_t>(), ldt) == RSRS_OK
               ? 0 : 1;
  }
  if (!op->owned32.p) {   // FP32 kernel matrix, entries rounded from the FP64 formula
    if (op->owned32.alloc((size_t)op->n * op->n * 4) != RSRS_OK) return 1;
    if (kernel_materialise<float>(st, op->kop, op->owned32.as<float>()) != RSRS_OK) return 1;
  }
  if (ncols > 16 && operator_library_gemm()) {
    ProfScope ps(st, "rocblas_sgemm:operator", 2.0 * n * n * ncols, 4.0 * ((double)n * n + 2.0 * n * ncols));
    if (rb_operator_product<float>(st, op->owned32.as<float>(), op->n, n, ta, static_cast<const float*>(X), ldx,
                                   ncols, static_cast<float*>(Y), ldy))
      return 0;
  }
  std::vector<GemmDescT<float, float>> d{gdescT<float, float>(
      op->owned32.as<float>(), nullptr, op->n, static_cast<const float*>(X), nullptr, ldx,
      static_cast<float*>(Y), nullptr, ldy, n, (int)ncols, n)};
  return gemm<float, float>(op->up, st, d, ta, 0, GM_FULL, shp, "operator") == RSRS_OK ? 0 : 1;
}

void rsrs_op_destroy(rsrs_operator_t* op) { delete op; }

rsrs_status rsrs_op_library_gemm(int enable) {
  set_operator_library_gemm(enable != 0);
  return RSRS_OK;
}

// ------------------------------------------------------------------ samples
static rsrs_status new_samples(const rsrs_tree_t* th, int64_t s, int dtype, rsrs_samples_t** out,
                               bool symmetric = false) {
  auto smp = new rsrs_samples_t();
  smp->tree = th;
  smp->n = th->t.n;
  smp->s = s;
  smp->ld = round_up(s, 16);
  smp->dtype = dtype;
  smp->symmetric = symmetric;
  const size_t bytes = (size_t)smp->n * smp->ld * dtype_size(dtype);
  rsrs_status st = smp->Y.alloc(bytes);
  if (st == RSRS_OK && !symmetric) st = smp->Z.alloc(bytes);
  if (st == RSRS_OK) st = smp->Om.alloc(bytes);
  if (st == RSRS_OK && !symmetric) st = smp->Psi.alloc(bytes);
  if (st != RSRS_OK) { delete smp; return st; }
  *out = smp;
  return RSRS_OK;
}

extern "C++" {
template <typename T>
static void gather_samples(hipStream_t st, rsrs_samples_t* smp, const void* Y, const void* Z,
                           const void* Om, const void* Psi, int64_t ld, const int64_t* pp) {
  const int64_t s = smp->s;
  gather_rows<T, T>(st, smp->Y.as<T>(), smp->ld, static_cast<const T*>(Y), ld, pp, smp->n, s);
  gather_rows<T, T>(st, smp->Om.as<T>(), smp->ld, static_cast<const T*>(Om), ld, pp, smp->n, s);
  if (smp->symmetric) return;
  gather_rows<T, T>(st, smp->Z.as<T>(), smp->ld, static_cast<const T*>(Z), ld, pp, smp->n, s);
  gather_rows<T, T>(st, smp->Psi.as<T>(), smp->ld, static_cast<const T*>(Psi), ld, pp, smp->n, s);
}

}  // extern "C++"

static rsrs_status wrap_impl(const rsrs_tree_t* th, int dtype, const void* Y, const void* Z,
                             const void* Om, const void* Psi, int64_t ld, int64_t s, void* stream,
                             rsrs_samples_t** out, bool symmetric) {
  if (!th || !Y || !Om || (!symmetric && (!Z || !Psi)) || !out || s < 1 || ld < s)
    return invalid("bad samples arguments");
  if (dtype != RSRS_F64 && dtype != RSRS_F32) return invalid("unknown dtype");
  *out = nullptr;
  hipStream_t st = static_cast<hipStream_t>(stream);
  rsrs_samples_t* smp = nullptr;
  RSRS_TRY(new_samples(th, s, dtype, &smp, symmetric));
  DevBuf perm;
  rsrs_status r = perm.alloc((size_t)smp->n * 8);
  if (r != RSRS_OK) { delete smp; return r; }
  if (hipMemcpyAsync(perm.p, th->t.perm.data(), (size_t)smp->n * 8, hipMemcpyHostToDevice, st) != hipSuccess) {
    delete smp;
    set_error("hipMemcpyAsync failed");
    return RSRS_E_HIP;
  }
  const int64_t* pp = perm.as<int64_t>();
  if (dtype == RSRS_F64) gather_samples<double>(st, smp, Y, Z, Om, Psi, ld, pp);
  else gather_samples<float>(st, smp, Y, Z, Om, Psi, ld, pp);
  if (hipStreamSynchronize(st) != hipSuccess) {
    delete smp;
    set_error("stream synchronisation failed");
    return RSRS_E_HIP;
  }
  *out = smp;
  return RSRS_OK;
}

rsrs_status rsrs_samples_wrap(const rsrs_tree_t* th, int dtype, const void* Y, const void* Z,
                              const void* Om, const void* Psi, int64_t ld, int64_t s, void* stream,
                              rsrs_samples_t** out) {
  return wrap_impl(th, dtype, Y, Z, Om, Psi, ld, s, stream, out, false);
}

rsrs_status rsrs_samples_wrap_symmetric(const rsrs_tree_t* th, int dtype, const void* Y, const void* Om,
                                        int64_t ld, int64_t s, void* stream, rsrs_samples_t** out) {
  return wrap_impl(th, dtype, Y, nullptr, Om, nullptr, ld, s, stream, out, true);
}

extern "C++" {
template <typename T>
static rsrs_status sample_t(const rsrs_tree_t* th, rsrs_matvec_fn mv, void* user, uint64_t seed,
                            int mv_dtype, void* stream, rsrs_samples_t* smp) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t s = smp->s;
  DevBuf tu, ty, perm;
  const size_t bytes = (size_t)smp->n * smp->ld * sizeof(T);
  RSRS_TRY(tu.alloc(bytes));
  RSRS_TRY(ty.alloc(bytes));
  RSRS_TRY(perm.alloc((size_t)smp->n * 8));
  RSRS_HIP(hipMemcpyAsync(perm.p, th->t.perm.data(), (size_t)smp->n * 8, hipMemcpyHostToDevice, st));
  const int64_t* pp = perm.as<int64_t>();
  for (int side = 0; side < (smp->symmetric ? 1 : 2); ++side) {
    philox_normal<T>(st, tu.as<T>(), smp->n, s, smp->ld, seed, (uint32_t)side);
    if constexpr (sizeof(T) == 4) {
      if (mv_dtype == RSRS_BF16) round_to_bf16_values(st, tu.as<float>(), smp->n, s, smp->ld);
    }
    if (mv(user, side, mv_dtype, s, tu.as<T>(), smp->ld, ty.as<T>(), smp->ld, stream) != 0) {
      (void)hipStreamSynchronize(st);
      set_error("matvec callback returned nonzero");
      return RSRS_E_CALLBACK;
    }
    gather_rows<T, T>(st, (side ? smp->Psi : smp->Om).as<T>(), smp->ld, tu.as<T>(), smp->ld, pp, smp->n, s);
    gather_rows<T, T>(st, (side ? smp->Z : smp->Y).as<T>(), smp->ld, ty.as<T>(), smp->ld, pp, smp->n, s);
  }
  if (hipStreamSynchronize(st) != hipSuccess) {
    set_error(std::string("sampling failed: ") + hipGetErrorString(hipGetLastError()));
    return RSRS_E_HIP;
  }
  return RSRS_OK;
}

}  // extern "C++"

static rsrs_status sample_impl(const rsrs_tree_t* th, rsrs_matvec_fn mv, void* user, int64_t s,
                               uint64_t seed, int dtype, void* stream, rsrs_samples_t** out,
                               bool symmetric) {
  if (!th || !mv || !out || s < 1) return invalid("bad sample arguments");
  if (dtype_size(dtype) == 0) return invalid("unknown dtype");
  *out = nullptr;
  rsrs_samples_t* smp = nullptr;
  // BF16 sampling keeps FP32 sketches (test matrices rounded to BF16 values)
  RSRS_TRY(new_samples(th, s, dtype == RSRS_BF16 ? RSRS_F32 : dtype, &smp, symmetric));
  const rsrs_status r = dtype == RSRS_F64 ? sample_t<double>(th, mv, user, seed, dtype, stream, smp)
                                          : sample_t<float>(th, mv, user, seed, dtype, stream, smp);
  if (r != RSRS_OK) { delete smp; return r; }
  *out = smp;
  return RSRS_OK;
}

rsrs_status rsrs_sample(const rsrs_tree_t* th, rsrs_matvec_fn mv, void* user, int64_t s, uint64_t seed,
                        int dtype, void* stream, rsrs_samples_t** out) {
  return sample_impl(th, mv, user, s, seed, dtype, stream, out, false);
}

rsrs_status rsrs_sample_symmetric(const rsrs_tree_t* th, rsrs_matvec_fn mv, void* user, int64_t s,
                                  uint64_t seed, int dtype, void* stream, rsrs_samples_t** out) {
  return sample_impl(th, mv, user, s, seed, dtype, stream, out, true);
}

void rsrs_samples_destroy(rsrs_samples_t* smp) { delete smp; }

rsrs_status rsrs_gaussian(double* out, int64_t nrows, int64_t ncols, int64_t ld, uint64_t seed,
                          uint32_t word, void* stream) {
  if (!out || nrows < 0 || ncols < 0 || ld < ncols) return invalid("bad gaussian arguments");
  philox_normal<double>(static_cast<hipStream_t>(stream), out, nrows, ncols, ld, seed, word);
  if (hipGetLastError() != hipSuccess) { set_error("philox launch failed"); return RSRS_E_HIP; }
  return RSRS_OK;
}

// ------------------------------------------------------------------ workload tile tuning
// The factorization of (tree, opts, s) is run on Gaussian samples once per
// candidate (the built-in rule, then each forced shape), every automatic
// GEMM launch timed under its shape signature; each signature then keeps its
// fastest shape.  Shapes do not change results, so any choice is exact.
extern "C++" {
template <typename T>
static void fill_gaussian(hipStream_t st, rsrs_samples_t* smp, uint64_t seed) {
  philox_normal<T>(st, smp->Y.as<T>(), smp->n, smp->s, smp->ld, seed, 0);
  philox_normal<T>(st, smp->Om.as<T>(), smp->n, smp->s, smp->ld, seed, 1);
  if (smp->symmetric) return;
  philox_normal<T>(st, smp->Z.as<T>(), smp->n, smp->s, smp->ld, seed, 2);
  philox_normal<T>(st, smp->Psi.as<T>(), smp->n, smp->s, smp->ld, seed, 3);
}
}  // extern "C++"

static rsrs_status tuning_factor(const rsrs_tree_t* t, const rsrs_factor_opts* o, int64_t s, hipStream_t st,
                                 bool record) {
  const int dtype = o->precision == RSRS_PREC_F64 ? RSRS_F64 : RSRS_F32;
  rsrs_samples_t* smp = nullptr;
  RSRS_TRY(new_samples(t, s, dtype, &smp, o->symmetric != 0));
  if (dtype == RSRS_F64) fill_gaussian<double>(st, smp, 0x7e57);
  else fill_gaussian<float>(st, smp, 0x7e57);
  if (hipGetLastError() != hipSuccess) {
    delete smp;
    set_error("GEMM tuning: sample generation failed");
    return RSRS_E_HIP;
  }
  if (record) gemm_sig_record(true);
  rsrs_factor_t* f = nullptr;
  const rsrs_status rs = factor_impl(t, smp, o, st, &f);
  gemm_sig_record(false);
  delete smp;
  if (f) rsrs_factor_destroy(f);
  if (rs == RSRS_OK && hipStreamSynchronize(st) != hipSuccess) {
    set_error("GEMM tuning: synchronisation failed");
    return RSRS_E_HIP;
  }
  return rs;
}

rsrs_status rsrs_gemm_autotune_workload(const rsrs_tree_t* t, const rsrs_factor_opts* opts, int64_t s,
                                        int64_t* signatures, int64_t* changed) {
  if (!t || !opts || s < 1) return invalid("null tree or options, or s < 1");
  if (signatures) *signatures = 0;
  if (changed) *changed = 0;
  rsrs_factor_opts o = *opts;
  o.rank_tol = 0.0;   // the fixed-rank launch sequence
  hipStream_t st = nullptr;
  RSRS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  struct Best { double ms; int shape; int rule; };
  std::unordered_map<uint64_t, Best> best;
  rsrs_status rs = RSRS_OK;
  // candidates: -1 = the current choice (built-in rule, class table or an
  // earlier exact entry), then the three shapes
  for (int cand = -2; cand <= 2 && rs == RSRS_OK; ++cand) {
    (void)gemm_tile_override(cand < 0 ? -1 : cand);
    std::vector<std::pair<uint64_t, double>> ms;
    std::vector<std::pair<uint64_t, int>> shp;
    rs = tuning_factor(t, &o, s, st, cand != -2);   // -2: warm-up (scratch, code objects)
    if (rs == RSRS_OK && cand != -2) rs = gemm_sig_collect(ms, shp);
    if (rs != RSRS_OK) break;
    std::unordered_map<uint64_t, int> sh(shp.begin(), shp.end());
    for (const auto& m : ms) {
      const int sp = sh[m.first];
      auto it = best.find(m.first);
      if (it == best.end()) {
        best[m.first] = Best{m.second, sp, cand == -1 ? sp : -1};
      } else {
        if (cand == -1) it->second.rule = sp;
        // a challenger must beat the kept shape by 2%
        if (m.second < 0.98 * it->second.ms) {
          it->second.ms = m.second;
          it->second.shape = sp;
        }
      }
    }
  }
  (void)gemm_tile_override(-1);
  (void)hipStreamDestroy(st);
  if (rs != RSRS_OK) return rs;
  std::vector<std::pair<uint64_t, int>> table;
  int64_t ch = 0;
  for (const auto& b : best) {
    table.emplace_back(b.first, b.second.shape);
    ch += b.second.rule >= 0 && b.second.shape != b.second.rule;
  }
  gemm_sig_install(table, false);
  if (signatures) *signatures = (int64_t)table.size();
  if (changed) *changed = ch;
  return RSRS_OK;
}

// ------------------------------------------------------------------ factor
rsrs_status rsrs_factor_redraw(const rsrs_tree_t* t, rsrs_matvec_fn mv, void* user, int64_t s, uint64_t seed,
                               int dtype, const rsrs_factor_opts* opts, void* stream, rsrs_factor_t** out) {
  if (!t || !mv || !opts || !out || s < 1) return invalid("null argument or s < 1");
  *out = nullptr;
  if ((opts->precision == RSRS_PREC_F64) != (dtype == RSRS_F64))
    return invalid("FP64 factorization needs FP64 samples, the mixed one FP32 or BF16 samples");
  rsrs_samples_t* smp = nullptr;
  RSRS_TRY(sample_impl(t, mv, user, s, seed, dtype, stream, &smp, opts->symmetric != 0));
  RedrawSpec rd{mv, user, seed};
  const rsrs_status r = factor_impl(t, smp, opts, static_cast<hipStream_t>(stream), out, &rd);
  delete smp;
  return r;
}

rsrs_status rsrs_factor(const rsrs_tree_t* t, rsrs_samples_t* smp, const rsrs_factor_opts* opts,
                        void* stream, rsrs_factor_t** out) {
  if (!t || !smp || !opts || !out) return invalid("null argument");
  *out = nullptr;
  return factor_impl(t, smp, opts, static_cast<hipStream_t>(stream), out);
}

rsrs_status rsrs_factor_batched(int64_t nprob, const rsrs_tree_t* const* trees,
                                rsrs_samples_t* const* samples, const rsrs_factor_opts* opts,
                                void* stream, rsrs_factor_t** out) {
  if (nprob < 1 || !trees || !samples || !opts || !out) return invalid("bad batched factor arguments");
  return factor_batch_impl(nprob, trees, samples, opts, static_cast<hipStream_t>(stream), out);
}

void rsrs_factor_destroy(rsrs_factor_t* f) { delete f; }

rsrs_status rsrs_factor_get_info(const rsrs_factor_t* f, rsrs_factor_info* out) {
  if (!f || !out) return invalid("null argument");
  out->n = f->n;
  out->s = f->s;
  out->k = f->k;
  out->nboxes = (int64_t)f->boxes.size();
  out->root_size = f->nt;
  out->stored_values = f->stored_values;
  out->stored_bytes = f->stored_values * f->esz;
  out->precision = f->precision;
  out->flops = f->flops;
  out->factor_ms = f->factor_ms;
  return RSRS_OK;
}

rsrs_status rsrs_factor_box_sizes(const rsrs_factor_t* f, int64_t i, int64_t* box, int32_t* level,
                                  int32_t* colour, int64_t* b, int64_t* n, int64_t* r, int64_t* k) {
  if (!f || i < 0 || i >= (int64_t)f->boxes.size()) return invalid("box index out of range");
  const BoxRec& R = f->boxes[i];
  if (box) *box = R.box;
  if (level) *level = R.level;
  if (colour) *colour = R.colour;
  if (b) *b = R.b;
  if (n) *n = R.n;
  if (r) *r = R.r;
  if (k) *k = R.k;
  return RSRS_OK;
}

static rsrs_status d2h(void* dst, const void* src, size_t bytes) {
  if (!dst || bytes == 0) return RSRS_OK;
  RSRS_HIP(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
  return RSRS_OK;
}

// rows x cols block (element offset off of the factor store, leading
// dimension ld) into a compact host FP64 block; FP32 stores are converted.
static rsrs_status d2h2(const rsrs_factor_t* f, double* dst, int64_t cols, int64_t off, int64_t ld,
                        int64_t rows) {
  if (!dst || rows == 0 || cols == 0) return RSRS_OK;
  const size_t es = (size_t)f->esz;
  const char* src = static_cast<const char*>(f->dstore.p) + off * es;
  if (es == 8) {
    RSRS_HIP(hipMemcpy2D(dst, (size_t)cols * 8, src, (size_t)ld * 8, (size_t)cols * 8, (size_t)rows,
                         hipMemcpyDeviceToHost));
    return RSRS_OK;
  }
  std::vector<float> tmp((size_t)rows * cols);
  RSRS_HIP(hipMemcpy2D(tmp.data(), (size_t)cols * 4, src, (size_t)ld * 4, (size_t)cols * 4, (size_t)rows,
                       hipMemcpyDeviceToHost));
  for (size_t i = 0; i < tmp.size(); ++i) dst[i] = (double)tmp[i];
  return RSRS_OK;
}

rsrs_status rsrs_factor_box_copy(const rsrs_factor_t* f, int64_t i, int64_t* Ba, int64_t* Na, int64_t* S,
                                 int64_t* R, double* T, double* XRR, double* KU, double* KL) {
  if (!f || i < 0 || i >= (int64_t)f->boxes.size()) return invalid("box index out of range");
  RSRS_HIP(hipDeviceSynchronize());
  const BoxRec& B = f->boxes[i];
  const int64_t kn = B.k + B.n;
  RSRS_TRY(d2h(Ba, f->i() + B.oBa, (size_t)B.b * 8));
  RSRS_TRY(d2h(Na, f->i() + B.oNa, (size_t)B.n * 8));
  RSRS_TRY(d2h(S, f->i() + B.oS, (size_t)B.k * 8));
  RSRS_TRY(d2h(R, f->i() + B.oR, (size_t)B.r * 8));
  RSRS_TRY(d2h2(f, T, B.k, B.oT, B.ldT, B.r));
  RSRS_TRY(d2h2(f, XRR, B.r, B.oXRR, B.ldR, B.r));
  RSRS_TRY(d2h2(f, KU, kn, B.oKU, B.ldKU, B.r));
  RSRS_TRY(d2h2(f, KL, B.r, B.oKL, B.ldR, kn));
  return RSRS_OK;
}

rsrs_status rsrs_factor_root_copy(const rsrs_factor_t* f, int64_t* nt, int64_t* Bt, double* At) {
  if (!f) return invalid("null factor");
  RSRS_HIP(hipDeviceSynchronize());
  if (nt) *nt = f->nt;
  RSRS_TRY(d2h(Bt, f->i() + f->oBt, (size_t)f->nt * 8));
  RSRS_TRY(d2h2(f, At, f->nt, f->oAt, f->nt, f->nt));
  return RSRS_OK;
}

// ------------------------------------------------------------------ solve / apply / refine
rsrs_status rsrs_solve(const rsrs_factor_t* f, int transpose, int64_t nrhs, const double* F, int64_t ldf,
                       double* U, int64_t ldu, void* stream) {
  if (!f || !F || !U || nrhs < 0 || ldf < nrhs || ldu < nrhs) return invalid("bad solve arguments");
  return apply_factor(f, 0, transpose, nrhs, F, ldf, U, ldu, static_cast<hipStream_t>(stream));
}

rsrs_status rsrs_solve_noalloc(const rsrs_factor_t* f, int transpose, int64_t nrhs, const double* F,
                               int64_t ldf, double* U, int64_t ldu, void* stream) {
  if (!f || !F || !U || nrhs < 0 || ldf < nrhs || ldu < nrhs) return invalid("bad solve arguments");
  return apply_factor_noalloc(f, 0, transpose, nrhs, F, ldf, U, ldu, static_cast<hipStream_t>(stream));
}

rsrs_status rsrs_apply(const rsrs_factor_t* f, int transpose, int64_t nrhs, const double* X, int64_t ldx,
                       double* Y, int64_t ldy, void* stream) {
  if (!f || !X || !Y || nrhs < 0 || ldx < nrhs || ldy < nrhs) return invalid("bad apply arguments");
  return apply_factor(f, 1, transpose, nrhs, X, ldx, Y, ldy, static_cast<hipStream_t>(stream));
}

rsrs_status rsrs_solve_refine(const rsrs_factor_t* f, rsrs_matvec_fn mv, void* user, int64_t nrhs,
                              const double* F, int64_t ldf, double* U, int64_t ldu, double tol,
                              int maxit, double* relres, int* iters, void* stream) {
  if (!f || !mv || !F || !U || nrhs < 1 || ldf < nrhs || ldu < nrhs || maxit < 0)
    return invalid("bad refine arguments");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t n = f->n, w = nrhs;
  RSRS_TRY(f->wt.alloc((size_t)n * w * 8));
  RSRS_TRY(f->wpart.alloc((size_t)256 * w * 8));
  RSRS_TRY(f->wnorm.alloc((size_t)2 * w * 8));
  double* r = f->wt.as<double>();
  double* nrm = f->wnorm.as<double>();
  std::vector<double> fn(w), rn(w);
  RSRS_TRY(col_sumsq(st, F, n, w, ldf, f->wpart.as<double>(), nrm));
  RSRS_HIP(hipMemcpyAsync(fn.data(), nrm, (size_t)w * 8, hipMemcpyDeviceToHost, st));
  RSRS_TRY(apply_factor(f, 0, 0, w, F, ldf, U, ldu, st));
  double rel = 0.0;
  int it = 0;
  for (;;) {
    if (mv(user, 0, RSRS_F64, w, U, ldu, r, w, stream) != 0) {
      set_error("matvec callback returned nonzero");
      return RSRS_E_CALLBACK;
    }
    sub2d(st, F, ldf, r, w, r, w, n, w);
    RSRS_TRY(col_sumsq(st, r, n, w, w, f->wpart.as<double>(), nrm));
    RSRS_HIP(hipMemcpyAsync(rn.data(), nrm, (size_t)w * 8, hipMemcpyDeviceToHost, st));
    RSRS_HIP(hipStreamSynchronize(st));
    rel = 0.0;
    for (int64_t c = 0; c < w; ++c) {
      const double d = fn[c] > 0.0 ? std::sqrt(rn[c] / fn[c]) : std::sqrt(rn[c]);
      if (!std::isfinite(d)) {
        set_error("non-finite residual");
        return RSRS_E_NUMERIC;
      }
      rel = std::max(rel, d);
    }
    if (rel <= tol || it >= maxit) break;
    RSRS_TRY(apply_factor(f, 0, 0, w, r, w, r, w, st));
    std::vector<Copy2D> c{Copy2D{r, U, w, ldu, (int)n, (int)w, 1.0, 1, 0}};
    RSRS_TRY(copy2d(f->up, st, c));
    ++it;
  }
  if (relres) *relres = rel;
  if (iters) *iters = it;
  return RSRS_OK;
}

}  // extern "C"
