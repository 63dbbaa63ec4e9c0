// Applying the factorization: eq. Ainvfact (solve) and eq. Afact (apply),
// and their transposes.  Index form of the elementary factors of a box with
// interpolation matrix T (r x k) and multipliers K_U (r x (k+n)),
// K_L ((k+n) x r):
//   E: x_R -= T x_S      F: x_S -= T^T x_R      L: x_SN -= K_L x_R      U: x_R -= K_U x_SN
// with V^{-1} = L E and W^{-1} = F U (eq. tildeA_diag).  Inside one colour
// class the boxes touch disjoint rows, so each elementary step is one batched
// launch over the class.  A mixed-precision factor is applied in FP32: the
// FP64 input is rounded while it is permuted into tree order and the result
// widened on the way out.
//
// Launch latency, not bandwidth, bounds a narrow solve (a few hundred small
// launches per sweep), so by default the launch sequence of a factor is
// assembled once per (operation, transpose, width bucket) into a HIP graph
// with pre-uploaded descriptors and its own work blocks, and replayed; the
// width is padded to the bucket (16, 32, 64, ... 1024) with zero columns,
// which do not touch the others.  Only the gather into tree order and the
// scatter back run outside the graph.  Wider solves run the launches
// directly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <unordered_map>

#include "impl.hpp"
#include "profile.hpp"

#include <memory>
#include <string>

namespace rsrs {

namespace {

enum Op { OP_SOLVE = 0, OP_APPLY = 1 };

rsrs_status ensure_ws(const rsrs_factor_t* F, int64_t w, hipStream_t st) {
  const size_t need = (size_t)F->n * (size_t)w * (size_t)F->esz;
  RSRS_TRY(F->wx.alloc(need));
  RSRS_TRY(F->wu.alloc(need));
  if (!F->up_ready) {
    RSRS_TRY(F->up.init((size_t)16 << 20, st));
    F->up_ready = true;
  }
  if (F->up.st != st) {
    RSRS_TRY(F->up.reset());
    F->up.st = st;
  }
  return RSRS_OK;
}

// Every product of one apply, in order, handed to emit(descs, ta, tb, mode).
template <typename T, class Emit>
rsrs_status build_apply(const rsrs_factor_t* F, int op, int transpose, int64_t w, T* x, T* u, Emit&& emit) {
  using GD = GemmDescT<T, T>;
  auto gdesc = [](const T* A, const int64_t* ia, int64_t lda, const T* B, const int64_t* ib,
                  int64_t ldb, T* C, const int64_t* ic, int64_t ldc, int M, int N, int K,
                  double alpha = 1.0, double beta = 0.0) {
    return gdescT<T, T>(A, ia, lda, B, ib, ldb, C, ic, ldc, M, N, K, alpha, beta);
  };
  const T* dS = F->d<T>();
  const int64_t* iS = F->i();
  const int W = (int)w;
  // first and second elementary step of the upward sweep (boxes in factor
  // order); k is each box's own skeleton count (k_B), and boxes that
  // eliminate nothing (r = 0) have no factors

  for (const Group& g : F->groups) {
    std::vector<GD> a0, a1;   // launches with TA = 0 / TA = 1
    std::vector<GD> b0, b1;
    for (int64_t q = g.first; q < g.first + g.count; ++q) {
      const BoxRec& R = F->boxes[q];
      const int r = (int)R.r, k = (int)R.k, kn = (int)(R.k + R.n);
      if (r == 0) continue;
      const int64_t* gR = iS + R.oR;
      const int64_t* gS = iS + R.oS;
      const int64_t* gSN = iS + R.oS;
      const T* Tm = dS + R.oT;
      const T* KU = dS + R.oKU;
      const T* KL = dS + R.oKL;
      const int64_t lT = R.ldT, lR = R.ldR, lU = R.ldKU;
      if (op == OP_SOLVE && !transpose) {        // E then L
        a0.push_back(gdesc(Tm, nullptr, lT, x, gS, w, x, gR, w, r, W, k, -1.0, 1.0));
        b0.push_back(gdesc(KL, nullptr, lR, x, gR, w, x, gSN, w, kn, W, r, -1.0, 1.0));
      } else if (op == OP_SOLVE) {              // F^T then U^T
        a0.push_back(gdesc(Tm, nullptr, lT, x, gS, w, x, gR, w, r, W, k, -1.0, 1.0));
        b1.push_back(gdesc(KU, nullptr, lU, x, gR, w, x, gSN, w, kn, W, r, -1.0, 1.0));
      } else if (!transpose) {                   // F^{-1} then U^{-1}
        a1.push_back(gdesc(Tm, nullptr, lT, x, gR, w, x, gS, w, k, W, r, 1.0, 1.0));
        b0.push_back(gdesc(KU, nullptr, lU, x, gSN, w, x, gR, w, r, W, kn, 1.0, 1.0));
      } else {                                   // E^{-T} then L^{-T}
        a1.push_back(gdesc(Tm, nullptr, lT, x, gR, w, x, gS, w, k, W, r, 1.0, 1.0));
        b1.push_back(gdesc(KL, nullptr, lR, x, gSN, w, x, gR, w, r, W, kn, 1.0, 1.0));
      }
    }
    RSRS_TRY(emit(a0, 0, 0, GM_FULL));
    RSRS_TRY(emit(a1, 1, 0, GM_FULL));
    RSRS_TRY(emit(b0, 0, 0, GM_FULL));
    RSRS_TRY(emit(b1, 1, 0, GM_FULL));
  }
  // block-diagonal middle factor D (or D^{-1}), every R block and the root
  {
    std::vector<GD> dd;
    const int ta = transpose ? 1 : 0;
    for (const BoxRec& R : F->boxes) {
      const int r = (int)R.r;
      if (r == 0) continue;
      const T* D = dS + (op == OP_SOLVE ? R.oXinv : R.oXRR);
      const int64_t* gR = iS + R.oR;
      dd.push_back(gdesc(D, nullptr, R.ldR, x, gR, w, u, gR, w, r, W, r));
    }
    const int nt = (int)F->nt;
    const int64_t* gB = iS + F->oBt;
    if (nt > 0)
      dd.push_back(gdesc(dS + (op == OP_SOLVE ? F->oAtinv : F->oAt), nullptr, nt, x, gB, w, u, gB, w,
                         nt, W, nt));
    RSRS_TRY(emit(dd, ta, 0, GM_FULL));
  }
  // downward sweep, boxes in reverse factor order
  for (size_t gi = F->groups.size(); gi-- > 0;) {
    const Group& g = F->groups[gi];
    std::vector<GD> a0, a1, b0, b1;
    for (int64_t q = g.first; q < g.first + g.count; ++q) {
      const BoxRec& R = F->boxes[q];
      const int r = (int)R.r, k = (int)R.k, kn = (int)(R.k + R.n);
      if (r == 0) continue;
      const int64_t* gR = iS + R.oR;
      const int64_t* gS = iS + R.oS;
      const int64_t* gSN = iS + R.oS;
      const T* Tm = dS + R.oT;
      const T* KU = dS + R.oKU;
      const T* KL = dS + R.oKL;
      const int64_t lT = R.ldT, lR = R.ldR, lU = R.ldKU;
      if (op == OP_SOLVE && !transpose) {        // U then F
        a0.push_back(gdesc(KU, nullptr, lU, u, gSN, w, u, gR, w, r, W, kn, -1.0, 1.0));
        b1.push_back(gdesc(Tm, nullptr, lT, u, gR, w, u, gS, w, k, W, r, -1.0, 1.0));
      } else if (op == OP_SOLVE) {              // L^T then E^T
        a1.push_back(gdesc(KL, nullptr, lR, u, gSN, w, u, gR, w, r, W, kn, -1.0, 1.0));
        b1.push_back(gdesc(Tm, nullptr, lT, u, gR, w, u, gS, w, k, W, r, -1.0, 1.0));
      } else if (!transpose) {                   // L^{-1} then E^{-1}
        a0.push_back(gdesc(KL, nullptr, lR, u, gR, w, u, gSN, w, kn, W, r, 1.0, 1.0));
        b0.push_back(gdesc(Tm, nullptr, lT, u, gS, w, u, gR, w, r, W, k, 1.0, 1.0));
      } else {                                   // U^{-T} then F^{-T}
        a1.push_back(gdesc(KU, nullptr, lU, u, gR, w, u, gSN, w, kn, W, r, 1.0, 1.0));
        b0.push_back(gdesc(Tm, nullptr, lT, u, gS, w, u, gR, w, r, W, k, 1.0, 1.0));
      }
    }
    RSRS_TRY(emit(a0, 0, 0, GM_FULL));
    RSRS_TRY(emit(a1, 1, 0, GM_FULL));
    RSRS_TRY(emit(b0, 0, 0, GM_FULL));
    RSRS_TRY(emit(b1, 1, 0, GM_FULL));
  }
  return RSRS_OK;
}

template <typename T>
rsrs_status apply_direct(const rsrs_factor_t* F, int op, int transpose, int64_t w, const double* Fin,
                         int64_t ldf, double* Uout, int64_t ldu, hipStream_t st) {
  RSRS_TRY(ensure_ws(F, w, st));
  Uploader& up = F->up;
  const GemmShape shp = w <= 16 ? GS_64x16 : GS_64x64;
  T* x = F->wx.as<T>();
  T* u = F->wu.as<T>();
  const int64_t* perm = F->perm.as<int64_t>();
  gather_rows<double, T>(st, x, w, Fin, ldf, perm, F->n, w);
  RSRS_TRY(build_apply<T>(F, op, transpose, w, x, u,
                          [&](const std::vector<GemmDescT<T, T>>& d, int ta, int tb, int mode) {
                            return gemm<T, T>(up, st, d, ta, tb, mode, shp, "solve");
                          }));
  scatter_rows<T, double>(st, Uout, ldu, u, w, perm, F->n, w);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}

bool g_graphs = true;
constexpr int64_t kMaxGraphWidth = 1024;

int64_t width_bucket(int64_t w) {
  int64_t b = 16;
  while (b < w) b *= 2;
  return b;
}

template <typename T>
rsrs_status make_plan(const rsrs_factor_t* F, int op, int transpose, int64_t wb, SolvePlan** out) {
  auto P = std::make_unique<SolvePlan>();
  P->op = op;
  P->transpose = transpose;
  P->w = wb;
  const size_t bytes = (size_t)F->n * wb * sizeof(T);
  RSRS_TRY(P->x.alloc(bytes));
  RSRS_TRY(P->u.alloc(bytes));
  RSRS_HIP(hipMemset(P->x.p, 0, bytes));
  RSRS_HIP(hipMemset(P->u.p, 0, bytes));
  const GemmShape shp = wb <= 16 ? GS_64x16 : GS_64x64;
  std::vector<GemmDescT<T, T>> all;
  std::vector<GemmLaunch> L;
  RSRS_TRY(build_apply<T>(F, op, transpose, wb, P->x.as<T>(), P->u.as<T>(),
                          [&](const std::vector<GemmDescT<T, T>>& d, int ta, int tb, int mode) {
                            const size_t base = all.size();
                            all.insert(all.end(), d.begin(), d.end());
                            return gemm_plan<T, T>(d, base, ta, tb, mode, shp, "solve", L);
                          }));
  RSRS_TRY(P->descs.alloc(std::max<size_t>(all.size(), 1) * sizeof(GemmDescT<T, T>)));
  if (!all.empty())
    RSRS_HIP(hipMemcpy(P->descs.p, all.data(), all.size() * sizeof(GemmDescT<T, T>), hipMemcpyHostToDevice));
  // the graph is assembled node by node (a linear chain of the product
  // launches), not captured from a stream: stream capture would be
  // invalidated by allocations or synchronisations that other threads
  // (other factorizations, a serving loop) make meanwhile
  hipGraph_t g = nullptr;
  RSRS_HIP(hipGraphCreate(&g, 0));
  hipGraphNode_t prev = nullptr;
  for (const auto& x : L) {
    const void* p = static_cast<const char*>(P->descs.p) + x.first * sizeof(GemmDescT<T, T>);
    void* args[] = {&p};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(x.fn);
    kp.gridDim = x.grid;
    kp.blockDim = x.block;
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    const hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      set_error(std::string("graph assembly failed: ") + hipGetErrorString(e));
      return RSRS_E_HIP;
    }
    prev = node;
  }
  P->graph = g;
  RSRS_HIP(hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0));
  F->plans.push_back(std::move(P));
  *out = F->plans.back().get();
  return RSRS_OK;
}

template <typename T>
rsrs_status apply_graph(const rsrs_factor_t* F, int op, int transpose, int64_t w, const double* Fin,
                        int64_t ldf, double* Uout, int64_t ldu, hipStream_t st) {
  const int64_t wb = width_bucket(w);
  SolvePlan* P = nullptr;
  for (auto& q : F->plans)
    if (q->op == op && q->transpose == transpose && q->w == wb) P = q.get();
  if (!P) RSRS_TRY(make_plan<T>(F, op, transpose, wb, &P));
  const int64_t* perm = F->perm.as<int64_t>();
  gather_rows<double, T>(st, P->x.as<T>(), wb, Fin, ldf, perm, F->n, w);
  {
    ProfScope ps(st, "solve_graph");
    RSRS_HIP(hipGraphLaunch(P->exec, st));
  }
  scatter_rows<T, double>(st, Uout, ldu, P->u.as<T>(), wb, perm, F->n, w);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}

}  // namespace

rsrs_status apply_factor(const rsrs_factor_t* F, int op, int transpose, int64_t w, const double* Fin,
                         int64_t ldf, double* Uout, int64_t ldu, hipStream_t st) {
  if (w <= 0) return RSRS_OK;
  if (g_graphs && w <= kMaxGraphWidth) {
    if (F->esz == 4) return apply_graph<float>(F, op, transpose, w, Fin, ldf, Uout, ldu, st);
    return apply_graph<double>(F, op, transpose, w, Fin, ldf, Uout, ldu, st);
  }
  if (F->esz == 4) return apply_direct<float>(F, op, transpose, w, Fin, ldf, Uout, ldu, st);
  return apply_direct<double>(F, op, transpose, w, Fin, ldf, Uout, ldu, st);
}

}  // namespace rsrs

extern "C" void rsrs_solve_graphs(int on) { rsrs::g_graphs = on != 0; }

// ---------------------------------------------------------------------------
// Solves and applies that allocate nothing: the two tree-ordered work blocks
// and the launch descriptors live in a fixed device array (`scratch`) that
// every GPU the library runs on holds until the process ends.  In host code
// `scratch` names a host-side stand-in, so its device address is looked up
// once per device (hipGetSymbolAddress with that device current) and only
// that address is handed to kernels and copies.  Nothing in it has to start
// at zero: the gather writes every row of x that is read, and every row of u
// is written (each point is in exactly one box's R or in B_t) before the
// downward sweep reads it.  Calls that overlap on one GPU share the array and
// race.
namespace rsrs {
namespace {

constexpr size_t kNoallocScratchBytes = (size_t)96 << 20;
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_scratch_mu;
std::unordered_map<int, void*> g_scratch_addr;   // device ordinal -> address of its copy

rsrs_status scratch_address(void** out) {
  int dev = 0;
  RSRS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return RSRS_OK;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    set_error(std::string("hipGetSymbolAddress of the no-alloc scratch failed: ") + hipGetErrorString(e));
    return RSRS_E_HIP;
  }
  g_scratch_addr[dev] = p;
  *out = p;
  return RSRS_OK;
}

template <typename T>
rsrs_status apply_noalloc(const rsrs_factor_t* F, int op, int transpose, int64_t w, const double* Fin,
                          int64_t ldf, double* Uout, int64_t ldu, hipStream_t st) {
  unsigned char* base = nullptr;
  RSRS_TRY(scratch_address(reinterpret_cast<void**>(&base)));
  const size_t blk = (size_t)round_up((int64_t)((size_t)F->n * (size_t)w * sizeof(T)), 256);
  T* x = reinterpret_cast<T*>(base);
  T* u = reinterpret_cast<T*>(base + blk);
  const GemmShape shp = w <= 16 ? GS_64x16 : GS_64x64;
  std::vector<GemmDescT<T, T>> all;
  std::vector<GemmLaunch> L;
  RSRS_TRY(build_apply<T>(F, op, transpose, w, x, u,
                          [&](const std::vector<GemmDescT<T, T>>& d, int ta, int tb, int mode) {
                            const size_t b0 = all.size();
                            all.insert(all.end(), d.begin(), d.end());
                            return gemm_plan<T, T>(d, b0, ta, tb, mode, shp, "solve", L);
                          }));
  const size_t dbytes = all.size() * sizeof(GemmDescT<T, T>);
  const size_t need = 2 * blk + dbytes;
  if (need > kNoallocScratchBytes) {
    set_error("the allocation-free solve needs " + std::to_string(need) + " bytes of scratch for n = " +
              std::to_string(F->n) + " and " + std::to_string(w) + " columns; its fixed scratch holds " +
              std::to_string(kNoallocScratchBytes) + " bytes (use fewer columns per call)");
    return RSRS_E_INVALID;
  }
  void* descs = base + 2 * blk;
  const int64_t* perm = F->perm.as<int64_t>();
  gather_rows<double, T>(st, x, w, Fin, ldf, perm, F->n, w);
  // pageable source: the call returns once the bytes have been staged
  if (dbytes) RSRS_HIP(hipMemcpyAsync(descs, all.data(), dbytes, hipMemcpyHostToDevice, st));
  for (const auto& l : L) RSRS_TRY(gemm_exec(l, descs, sizeof(GemmDescT<T, T>), st));
  scatter_rows<T, double>(st, Uout, ldu, u, w, perm, F->n, w);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}

}  // namespace

rsrs_status apply_factor_noalloc(const rsrs_factor_t* F, int op, int transpose, int64_t w, const double* Fin,
                                 int64_t ldf, double* Uout, int64_t ldu, hipStream_t st) {
  if (w <= 0) return RSRS_OK;
  if (F->esz == 4) return apply_noalloc<float>(F, op, transpose, w, Fin, ldf, Uout, ldu, st);
  return apply_noalloc<double>(F, op, transpose, w, Fin, ldf, Uout, ldu, st);
}

}  // namespace rsrs
