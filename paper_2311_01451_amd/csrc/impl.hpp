// Internal definitions of the opaque handles of include/rsrs.h.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "tree.hpp"

struct rsrs_tree_s {
  rsrs::Tree t;
};

struct rsrs_samples_s {
  const rsrs_tree_t* tree = nullptr;
  int64_t n = 0, s = 0, ld = 0;
  int dtype = RSRS_F64;         // element type of Y, Z, Om, Psi
  bool symmetric = false;       // only Y and Om (Z = Y, Psi = Om implicitly)
  rsrs::DevBuf Y, Z, Om, Psi;   // tree order, row-major n x s (leading dimension ld)
  bool consumed = false;
};

struct rsrs_operator_s {
  int kind = 0;     // 1..3 kernel (explicit matrix), 10 dense borrowed, 20 poisson7
  int64_t n = 0;
  rsrs::DevBuf owned;        // explicit kernel matrix
  const double* A = nullptr; // matrix used by the GEMM matvec
  int64_t lda = 0;
  rsrs::DevBuf owned32;      // FP32 kernel matrix (built at the first FP32 product)
  rsrs::DevBuf owned16;      // BF16 kernel matrix (built at the first BF16 product)
  rsrs::DevBuf xt16;         // transposed BF16 copy of the right-hand block
  rsrs::DevBuf skinny;       // partial products of narrow FP64 products
  rsrs::KernelOp kop;        // kernel description (kernel operators)
  bool symmetric = true;
  rsrs::Poisson7Op pois;
  rsrs::Uploader up;
  bool up_ready = false;
};

namespace rsrs {

// One processed box; offsets index the factor's double / int64 stores.
struct BoxRec {
  int64_t box = 0;
  int level = 0, colour = 0;
  int64_t b = 0, n = 0, r = 0, k = 0;
  int64_t oT = 0, oXRR = 0, oXinv = 0, oKU = 0, oKL = 0;   // elements, 16-byte aligned
  int64_t ldT = 0, ldR = 0, ldKU = 0;   // 16-byte multiples: T, X_RR / X_RR^{-1} / K_L, K_U
  int64_t oR = 0, oS = 0, oSN = 0, oBa = 0, oNa = 0;       // int64 tree positions
};

// Per-level redrawing of the samples: the operator and the generator seed.
struct RedrawSpec {
  rsrs_matvec_fn mv;
  void* user;
  uint64_t seed;
};

// Factorization of one problem or a batch (factor.hip); rd: per-level redraw
// (one problem only), null for none.
rsrs_status factor_impl(const rsrs_tree_t* th, rsrs_samples_t* smp, const rsrs_factor_opts* o,
                        hipStream_t st, rsrs_factor_t** out, const RedrawSpec* rd = nullptr);
rsrs_status factor_batch_impl(int64_t nprob, const rsrs_tree_t* const* trees, rsrs_samples_t* const* smps,
                              const rsrs_factor_opts* opts, hipStream_t st, rsrs_factor_t** out,
                              const RedrawSpec* rd = nullptr);

struct Group {  // one colour class: boxes [first, first+count) in processing order
  int64_t first = 0, count = 0;
};

template <typename T>
rsrs_status kernel_materialise(hipStream_t st, const KernelOp& op, T* A);

}  // namespace rsrs

namespace rsrs {
// A solve or apply of one factor for a fixed width, held as a HIP graph:
// its own tree-ordered work blocks x, u (n x w, zero-initialised so padded
// columns stay zero), the descriptors of every launch, and the graph.
struct SolvePlan {
  int op = 0, transpose = 0;
  int64_t w = 0;
  DevBuf x, u, descs;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~SolvePlan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};
}  // namespace rsrs

struct rsrs_factor_s {
  int64_t n = 0, s = 0, k = 0;
  int precision = RSRS_PREC_F64;
  int esz = 8;                         // bytes per stored element (8 FP64, 4 FP32)
  rsrs::DevBuf dstore, istore, perm;   // perm: tree position -> user index
  std::vector<rsrs::BoxRec> boxes;
  std::vector<rsrs::Group> groups;
  int64_t nt = 0, oBt = 0, oAt = 0, oAtinv = 0;
  int64_t stored_values = 0;
  double flops = 0.0, factor_ms = 0.0;
  // solve workspace (grown on demand)
  mutable rsrs::DevBuf wx, wu, wt, wpart, wnorm;
  mutable rsrs::Uploader up;
  mutable bool up_ready = false;
  mutable std::vector<std::unique_ptr<rsrs::SolvePlan>> plans;   // solves as graphs
  ~rsrs_factor_s() { plans.clear(); }
  template <typename T> const T* d() const { return dstore.as<T>(); }
  const int64_t* i() const { return istore.as<int64_t>(); }
};
