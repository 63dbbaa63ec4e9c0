// Algorithm 1 (randomized strong recursive skeletonization), host orchestration.
//
// Levels run from the finest to the coarsest; inside a level, the colour
// classes of the schedule (tree.cpp) run one after another and all boxes of a
// class are processed together by batched kernels.  Boxes of one class touch
// disjoint rows of Y, Z, Omega, Psi, so the batched result equals processing
// them one at a time.  Per class:
//
//  phase A  Gram matrices G = C C^T of the test-matrix panels
//           C_Omega = [Omega_Ba; Omega_Na], C_Psi likewise (l x s each);
//           Cholesky G = L L^T with the inverse factor L^{-1} (panel kernel
//           with deferred super-panel updates, chol.hip);
//           least-squares coefficients X = Y_B pinv(C) = (Y_B C^T) L^{-T} L^{-1}
//           and the far-field sketch M_Y = Y_B - X C_Omega, i.e. Y_B times the
//           projector onto null(C_Omega) (eq. nullYZ); one optional second
//           pass re-projects M_Y and refines X.  Same for Z / Psi.
//           ID of M = M_Y + M_Z (or of [M_Y, M_Z]) by pivoted Gram-Schmidt
//           (Sec. 2.3); k_B = k, or with a rank tolerance the number of
//           pivots above it.
//  phase B  Block extraction (eq. pinvYZ) from the same coefficients: since
//           Y_hat_R = Y_R - T Y_S and Omega_hat_C = G_T Omega_C with
//           G_T = I + e_S T^T e_R^T, Y_hat_R pinv(Omega_hat_C) =
//           (X_R - T X_S) G_T^{-1}; G_T^{-1} subtracts columns S T^T from
//           columns R.  X_RR^{-1} by Gauss-Jordan, K_U = X_RR^{-1} X_{R,SN},
//           K_L = X_{SN,R} X_RR^{-1}; then the sketch updates of Algorithm 1:
//           E, F (sparsify) followed by L, U (eliminate).
//  root     A_t = Y_Bt pinv(Omega_Bt) by the same Gram route, then A_t^{-1}.
//
// Streams.  Phase B of a class (from the extraction to the sketch updates)
// runs on a second stream.  It starts once the skeletons are known and the
// test matrices are sparsified (Omega_S += T^T Omega_R, done on the main
// stream, the only update the next class's Gram matrices depend on); the
// main stream meanwhile forms the next class's Gram matrices and factors
// them, and waits for phase B only before the next projections, which read
// the updated Y / Z.  What phase B reads lives in a part of the workspace
// that alternates between two buffers from class to class.  Phase B's
// launches are enqueued by a second host thread, so that the calling
// thread builds the next class's index lists meanwhile.
//
// Precision.  The whole class of operations is templated on the element type
// T of the samples and of the stored factor.  T = double is plain FP64.  With
// T = float (the mixed-precision factorization) every product of sketch-sized
// operands runs on FP32 MFMA with FP32 accumulation, and so do the Gram
// matrices and their factorization (Cholesky, inverse factor): the Gram
// entries already carry an FP32 accumulation error, and the FP32 Cholesky
// adds a backward error of the same order.  The decisions stay FP64: the
// pivoted QR of the ID takes its dot products, norms and coefficients in FP64 (the
// working rows of M stay FP32, like the sketches they come from: each
// stored residual is rounded relative to its own size, far below the
// rounding M already carries), and X_RR and A_t are inverted by FP64
// Gauss-Jordan with partial pivoting; the results are rounded to FP32 for
// the products that use them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <numeric>
#include <thread>
#include <unordered_map>

#include "impl.hpp"
#include "profile.hpp"
#include <memory>
#include <string>

namespace rsrs {

namespace {

struct Bump {
  char* base = nullptr;
  size_t off = 0, cap = 0;
  template <class T> T* take(int64_t count) {
    off = (size_t)round_up((int64_t)off, 256);
    T* p = reinterpret_cast<T*>(base + off);
    off += (size_t)count * sizeof(T);
    return p;
  }
};

// ---- index lists assembled on the device (fixed rank).  With a fixed rank
// every count is known from the schedule, so the host tracks where each
// active list lives (pieces: a range of the index store, or a range of
// tree positions) and never needs the skeleton values themselves: a class's
// B_a and N_a slots are filled by one launch of list segments, and its S and
// R slots by one launch that maps the ID's positions through B_a.  No host
// synchronisation is needed between classes.
struct ListSeg {
  int64_t* dst;
  const int64_t* src;   // nullptr: write iota, iota + 1, ...
  int64_t iota, len;
};

__global__ __launch_bounds__(256) void list_assemble_kernel(const ListSeg* __restrict__ segs) {
  const ListSeg g = segs[blockIdx.x];
  for (int64_t j = threadIdx.x; j < g.len; j += 256) g.dst[j] = g.src ? g.src[j] : g.iota + j;
}

struct SkelSeg {
  const int64_t* Ba;    // the box's B_a slot
  const int64_t* pos;   // ID positions: k skeletons ascending, then the b - k others
  int64_t* S;
  int64_t* R;
  int b, k;
};

__global__ __launch_bounds__(256) void skel_scatter_kernel(const SkelSeg* __restrict__ segs) {
  const SkelSeg g = segs[blockIdx.x];
  for (int j = threadIdx.x; j < g.b; j += 256) {
    // positions come from the ID's own row indices; the clamp only keeps a
    // corrupted one inside the slot
    const int64_t p = min(max(g.pos[j], (int64_t)0), (int64_t)(g.b - 1));
    const int64_t v = g.Ba[p];
    if (j < g.k) g.S[j] = v;
    else g.R[j - g.k] = v;
  }
}

template <class S>
rsrs_status launch_segments(Uploader& up, hipStream_t st, const std::vector<S>& segs, void (*kern)(const S*),
                            const char* tag) {
  if (segs.empty()) return RSRS_OK;
  S* d = nullptr;
  RSRS_TRY(up.put_vec(segs, &d));
  ProfScope ps(st, tag);
  hipLaunchKernelGGL(kern, dim3((unsigned)segs.size()), dim3(256), 0, st, d);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}

// A second stream and the two events that order it against the main one;
// the destructor drains it, so no kernel outlives the workspace it reads.
// The side stream and its two events.  Creating a stream costs a fraction
// of a millisecond, so a drained one is kept per device for the next
// factorization (recycle()); one that is not recycled is destroyed.
struct SideStream {
  hipStream_t st = nullptr;
  hipEvent_t eA = nullptr, eB = nullptr;
  int dev = 0;
  struct Kept { hipStream_t st; hipEvent_t eA, eB; int dev; };
  static std::mutex& kept_mu() { static std::mutex m; return m; }
  static std::vector<Kept>& kept() { static auto* v = new std::vector<Kept>(); return *v; }
  rsrs_status init() {
    RSRS_HIP(hipGetDevice(&dev));
    {
      std::lock_guard<std::mutex> lk(kept_mu());
      auto& v = kept();
      for (size_t i = 0; i < v.size(); ++i)
        if (v[i].dev == dev) {
          st = v[i].st; eA = v[i].eA; eB = v[i].eB;
          v.erase(v.begin() + (std::ptrdiff_t)i);
          return RSRS_OK;
        }
    }
    RSRS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    RSRS_HIP(hipEventCreateWithFlags(&eA, hipEventDisableTiming));
    RSRS_HIP(hipEventCreateWithFlags(&eB, hipEventDisableTiming));
    return RSRS_OK;
  }
  // the stream must be drained; keeps at most four per process
  void recycle() {
    std::lock_guard<std::mutex> lk(kept_mu());
    if (kept().size() >= 4 || !st || !eA || !eB) return;
    kept().push_back(Kept{st, eA, eB, dev});
    st = nullptr; eA = eB = nullptr;
  }
  ~SideStream() {
    if (st) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
    if (eA) (void)hipEventDestroy(eA);
    if (eB) (void)hipEventDestroy(eB);
  }
};

// A host thread that enqueues phase B of a class on the side stream while
// the calling thread goes on with the next class (the HIP calls that
// enqueue phase B's launches and uploads take hundreds of microseconds of
// host time per class).  One task at a time; join() waits until the task
// has been enqueued and returns its status (and error message).  The
// destructor lets a running task finish.
struct EnqueueWorker {
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  std::function<rsrs_status()> task;
  bool has_task = false, busy = false, quit = false;
  rsrs_status status = RSRS_OK;
  std::string err;
  int dev = 0;

  rsrs_status start() {
    RSRS_HIP(hipGetDevice(&dev));
    try {
      th = std::thread([this] { loop(); });
    } catch (...) {
      set_error("could not start the enqueue thread");
      return RSRS_E_INVALID;
    }
    return RSRS_OK;
  }
  void loop() {
    (void)hipSetDevice(dev);
    for (;;) {
      std::function<rsrs_status()> f;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return has_task || quit; });
        if (!has_task) return;
        f = std::move(task);
        has_task = false;
      }
      const rsrs_status s = f();
      std::string e = s == RSRS_OK ? std::string() : std::string(rsrs_last_error());
      {
        std::lock_guard<std::mutex> lk(mu);
        if (status == RSRS_OK) {
          status = s;
          err = std::move(e);
        }
        busy = false;
      }
      cv.notify_all();
    }
  }
  void submit(std::function<rsrs_status()> f) {
    {
      std::lock_guard<std::mutex> lk(mu);
      task = std::move(f);
      has_task = true;
      busy = true;
    }
    cv.notify_all();
  }
  rsrs_status join() {
    std::unique_lock<std::mutex> lk(mu);
    cv.wait(lk, [&] { return !busy; });
    const rsrs_status s = status;
    if (s != RSRS_OK) set_error(err);
    return s;
  }
  ~EnqueueWorker() {
    {
      std::lock_guard<std::mutex> lk(mu);
      quit = true;
    }
    cv.notify_all();
    if (th.joinable()) th.join();
  }
};

// Workspace bytes of one box (b, l) in a class, samples of element type T,
// in two parts: what only the projections and the ID use (*a), and what the
// extraction and elimination read after them (*b).  The second part is held
// twice, so that the next class's Gram matrices and Cholesky factorizations
// can run while this class finishes.
template <typename T>
void box_ws_bytes(int64_t b, int64_t l, int64_t k, int64_t r, int64_t sp, size_t* a, size_t* bpart) {
  constexpr bool mixed = sizeof(T) != sizeof(double);
  const int64_t lp = round_up(l, 16);
  int64_t dblA = 3 * b + b * k;    // norms, row norms of [Y_B Z_B], R coefficients
  int64_t telA = 4 * l * lp        // Gram matrices / inverse factors, scratch, both sides
                 + 4 * b * lp      // P, W for both sides
                 + 2 * b * sp;     // M_Y, M_Z
  int64_t dblB = 2 * r * r;        // Gauss-Jordan work
  int64_t telB = 2 * b * lp        // X for both sides
                 + 4 * r * lp;     // XR, Xp for both sides
  if (mixed) {
    dblA += r * round_up(k, 4);    // T as computed by the ID
    dblA += b * 2 * sp + kIdGramSplit * b * round_up(b, 16) + b * k;   // the ID's FP64 rows (up to 2 sp long), partial Gram matrices, R
    dblB += 2 * r * r;             // X_RR and its inverse in FP64
  }
  const int64_t ints = b + k;      // sel, piv (int32)
  const int64_t i64 = k + b + 1;   // Spos, Rpos, k_B
  *a = (size_t)(dblA * 8 + telA * sizeof(T) + ints * 4 + 20 * 256);
  *bpart = (size_t)(dblB * 8 + telB * sizeof(T) + i64 * 8 + 12 * 256);
}

template <typename T>
struct BoxWs {
  int64_t lp;
  T *GO, *GP, *LO, *LP;         // Gram matrices -> inverse factors (L), scratch (G)
  double *norms, *Rc, *gje;
  T *PY, *WY, *XY, *PZ, *WZ, *XZ, *MY, *MZ;
  T *XRy, *XRz, *Xpy, *Xpz;
  double *Td, *XRRd, *Xinvd;   // FP64 copies (mixed precision only)
  int32_t *sel, *piv;
  int64_t *Spos, *Rpos, *kB;
  int64_t mld;                  // leading dimension of M_Y, M_Z
  double *Md, *Gm, *Rt;         // mixed precision: the ID's FP64 rows, their Gram matrix, R column-major
  int64_t ldmd, ldg;
};

// One problem of a factorization.  Problems advance through their colour
// classes in lock step (class t of every problem that has one), so several
// independent problems share every launch; a single problem is the special
// case of one job.
template <typename T>
struct Job {
  static constexpr bool mixed = sizeof(T) != sizeof(double);
  static constexpr int64_t al = 16 / (int64_t)sizeof(T);   // elements per 16 bytes
  const rsrs_tree_t* th = nullptr;
  rsrs_samples_t* smp = nullptr;
  int k = 0, p = 0, reproject = 1;
  bool sym = false;             // symmetric variant: the Y / Omega side only
  bool concat = false;          // ID of [M_Y, M_Z] instead of M_Y + M_Z (general variant)
  double rank_tol = 0.0;        // > 0: k_B from the pivots' size (storage planned for k_B = 0)
  bool col_subset = false;      // a box reads its first s_B = min(s, l + k + p) sample columns
  bool deferred = false;        // fixed rank in every problem: lists assembled on the device
  // per-level redraw: the operator, seed, redraws done, and their buffers
  // (N x sld in tree order, the same in user order twice; the inverse permutation)
  const RedrawSpec* rd = nullptr;
  int redraws = 0;
  DevBuf rd_x, rd_u, rd_y, rd_iperm;
  HostBuf rd_hiperm;
  // active list as pieces: src != nullptr is a range of the index store,
  // else the tree positions iota .. iota + len - 1
  struct Piece { const int64_t* src; int64_t iota, len; };
  std::vector<std::vector<Piece>> pcur, prem;
  Schedule sch;
  std::unique_ptr<rsrs_factor_t> F;
  T *Y = nullptr, *Z = nullptr, *Om = nullptr, *Psi = nullptr;
  int64_t s = 0, sld = 0, n = 0;
  T* dS = nullptr;
  int64_t* iS = nullptr;
  HostBuf hidx;                 // staging of the index lists uploaded to istore
  int64_t* hI = nullptr;
  std::vector<std::vector<int64_t>> cur, remaining;
  size_t li = 0, ci = 0;        // level index and class index of the next class
  std::unordered_map<int64_t, size_t> pos;
  std::vector<size_t> class_ws, class_wsb;    // workspace bytes of each class (two parts)
  size_t root_ws = 0;
  double flops = 0.0;
  double flops_b = 0.0;   // phase B's share (accumulated by the enqueue thread)

  const Tree& tree() const { return th->t; }
  // Sample columns a box with l active columns reads in its nullification,
  // ID and extraction; its updates cover all s.
  int sB(int64_t l) const { return (int)(col_subset ? std::min<int64_t>(s, l + k + p) : s); }
  std::vector<int64_t> leaf_range(int64_t b) const {
    std::vector<int64_t> v((size_t)tree().npts(b));
    std::iota(v.begin(), v.end(), tree().pt_begin[b]);
    return v;
  }
  // Active set of every box of the level about to run, from its children.
  void enter_level() {
    const Tree& t = tree();
    const auto& lb = t.level_boxes[sch.levels[li]];
    pos.clear();
    for (size_t i = 0; i < lb.size(); ++i) {
      const int64_t b = lb[i];
      pos[b] = i;
      if (deferred) {
        std::vector<Piece> v;
        if (t.is_leaf[b]) {
          if (t.npts(b) > 0) v.push_back(Piece{nullptr, t.pt_begin[b], t.npts(b)});
        } else {
          // children own disjoint, ascending point ranges: in range order
          // their sorted lists concatenate to a sorted list
          std::vector<int64_t> ch(t.child_ids.begin() + t.child_off[b], t.child_ids.begin() + t.child_off[b + 1]);
          std::sort(ch.begin(), ch.end(), [&](int64_t x, int64_t y) { return t.pt_begin[x] < t.pt_begin[y]; });
          for (int64_t c : ch) v.insert(v.end(), prem[c].begin(), prem[c].end());
        }
        pcur[b] = std::move(v);
      } else if (t.is_leaf[b]) {
        cur[b] = leaf_range(b);
      } else {
        std::vector<int64_t> v;
        for (int64_t j = t.child_off[b]; j < t.child_off[b + 1]; ++j) {
          const auto& rc = remaining[t.child_ids[j]];
          v.insert(v.end(), rc.begin(), rc.end());
        }
        std::sort(v.begin(), v.end());
        cur[b] = std::move(v);
      }
    }
  }
  void leave_level() {
    for (int64_t b : tree().level_boxes[sch.levels[li]]) {
      if (deferred) prem[b] = pcur[b];
      else remaining[b] = cur[b];
    }
    ++li;
    ci = 0;
  }
  // Levels without processed boxes keep every point active.
  void settle() {
    while (li < sch.levels.size() && sch.classes[li].empty()) {
      enter_level();
      leave_level();
    }
    if (li < sch.levels.size() && ci == 0) enter_level();
  }
  // pieces of a neighbour's active list (a coarser neighbour is a leaf that
  // keeps all its points)
  const std::vector<Piece>& pieces_of(int64_t x) {
    if (tree().level[x] < sch.levels[li] && pcur[x].empty() && tree().npts(x) > 0)
      pcur[x] = {Piece{nullptr, tree().pt_begin[x], tree().npts(x)}};
    return pcur[x];
  }
  // segments writing the pieces to dst (at most cap entries); returns the count
  int64_t emit(std::vector<ListSeg>& segs, int64_t* dst, const std::vector<Piece>& pc, int64_t cap) const {
    int64_t n = 0;
    for (const Piece& q : pc) {
      if (q.len <= 0) continue;
      if (n + q.len > cap) return cap + 1;
      segs.push_back(ListSeg{dst + n, q.src, q.iota, q.len});
      n += q.len;
    }
    return n;
  }
  const std::vector<int64_t>& active_of(int64_t x) {
    if (tree().level[x] < sch.levels[li] && cur[x].empty()) cur[x] = leaf_range(x);
    return cur[x];
  }
};

template <typename T>
rsrs_status job_init(Job<T>& J, const rsrs_tree_t* th, rsrs_samples_t* smp,
                     const rsrs_factor_opts* o) {
  constexpr int64_t al = Job<T>::al;
  constexpr bool mixed = Job<T>::mixed;
  J.th = th;
  J.smp = smp;
  J.k = o->k;
  J.p = o->p < 0 ? J.k : o->p;
  J.reproject = o->reproject;
  J.sym = o->symmetric != 0;
  J.concat = !J.sym && o->id_mode == RSRS_ID_CONCAT;
  J.rank_tol = o->rank_tol;
  J.col_subset = o->col_subset != 0;
  const bool adaptive = J.rank_tol > 0.0;
  const Tree& t = th->t;
  const int k = J.k;
  make_schedule(t, k, J.sch);
  const int64_t need = samples_required(t, J.sch, k, J.p);
  if (smp->s < need) {
    set_required_s(need);
    set_error("s = " + std::to_string(smp->s) + " is below the required " + std::to_string(need));
    return RSRS_E_SAMPLES;
  }
  J.s = smp->s;
  J.sld = smp->ld;
  J.n = t.n;
  J.Y = smp->Y.as<T>();
  J.Om = smp->Om.as<T>();
  J.Z = J.sym ? J.Y : smp->Z.as<T>();
  J.Psi = J.sym ? J.Om : smp->Psi.as<T>();
  J.F = std::make_unique<rsrs_factor_t>();
  rsrs_factor_t* F = J.F.get();
  F->n = J.n;
  F->s = J.s;
  F->k = k;
  F->precision = o->precision;
  F->esz = (int)sizeof(T);

  // storage layout from the schedule (sizes are fixed by the count model)
  int64_t dsz = 0, isz = 0;
  for (size_t li = 0; li < J.sch.levels.size(); ++li) {
    for (size_t c = 0; c < J.sch.classes[li].size(); ++c) {
      Group g;
      g.first = (int64_t)F->boxes.size();
      size_t ws = 0, wsb = 0;
      for (int64_t b : J.sch.classes[li][c]) {
        BoxRec r;
        r.box = b;
        r.level = J.sch.levels[li];
        r.colour = (int)c;
        r.b = J.sch.b_count[b];
        r.n = J.sch.l_count[b] - r.b;
        r.k = k;
        r.r = r.b - k;
        // with a rank tolerance the store is planned for the worst case
        // k_B = 0 (r = b); the counts are the schedule's, an upper bound of
        // the actual ones, which are set when the box's class runs
        const int64_t rmax = adaptive ? r.b : r.r;
        r.ldT = round_up(k, al);
        r.ldR = round_up(rmax, al);
        r.ldKU = round_up(k + r.n, al);
        r.oT = round_up(dsz, al); dsz = r.oT + rmax * r.ldT;
        r.oXRR = round_up(dsz, al); dsz = r.oXRR + rmax * r.ldR;
        r.oXinv = round_up(dsz, al); dsz = r.oXinv + rmax * r.ldR;
        r.oKU = round_up(dsz, al); dsz = r.oKU + rmax * r.ldKU;
        r.oKL = round_up(dsz, al); dsz = r.oKL + (k + r.n) * r.ldR;
        // R list, then S ending where N_a begins (S || N_a is the list SN)
        r.oR = isz; isz += rmax;
        r.oS = isz; isz += k;
        r.oNa = isz; isz += r.n;
        r.oBa = isz; isz += r.b + r.n;   // Ba followed by a second copy of Na
        F->boxes.push_back(r);
        size_t wa = 0, wb = 0;
        box_ws_bytes<T>(r.b, r.b + r.n, k, rmax, J.sld, &wa, &wb);
        ws += wa;
        wsb += wb;
      }
      g.count = (int64_t)F->boxes.size() - g.first;
      F->groups.push_back(g);
      J.class_ws.push_back(ws);
      J.class_wsb.push_back(wsb);
    }
  }
  F->nt = J.sch.root_count;
  F->oBt = isz; isz += F->nt;
  F->oAt = round_up(dsz, al); dsz = F->oAt + F->nt * F->nt;
  F->oAtinv = round_up(dsz, al); dsz = F->oAtinv + F->nt * F->nt;
  F->stored_values = dsz;
  const int64_t ntp = round_up(F->nt, 16);
  J.root_ws = (size_t)(4 * F->nt * ntp + F->nt * round_up(J.s, 16) + 2 * F->nt * F->nt) * 8 + 8 * 256;
  if (mixed)   // FP64 copies of Y_Bt, Omega_Bt, A_t, A_t^{-1}
    J.root_ws += (size_t)(2 * F->nt * round_up(J.s, 16) + 2 * F->nt * F->nt) * 8 + 4 * 256;

  RSRS_TRY(F->dstore.alloc((size_t)std::max<int64_t>(dsz, 1) * sizeof(T)));
  RSRS_TRY(F->istore.alloc((size_t)std::max<int64_t>(isz, 1) * 8));
  RSRS_TRY(F->perm.alloc((size_t)J.n * 8));
  RSRS_TRY(pool_alloc(J.hidx, (size_t)std::max<int64_t>(isz, 1) * 8));
  J.hI = J.hidx.template as<int64_t>();
  J.dS = F->dstore.template as<T>();
  J.iS = F->istore.template as<int64_t>();
  J.cur.assign((size_t)t.nbox(), {});
  J.remaining.assign((size_t)t.nbox(), {});
  J.pcur.assign((size_t)t.nbox(), {});
  J.prem.assign((size_t)t.nbox(), {});
  return RSRS_OK;
}

// Per-box work item of one step: the job it belongs to, its record and workspace.
template <typename T>
struct Item {
  Job<T>* J;
  BoxRec* R;
  BoxWs<T> w;
};

// One upload of a class's index lists (the boxes' R, S, N_a, B_a, N_a slots
// are contiguous in the index store, box after box).
template <typename T>
rsrs_status upload_class_lists(Job<T>& J, const Group& g, hipStream_t st) {
  if (g.count <= 0) return RSRS_OK;
  const BoxRec& a = J.F->boxes[g.first];
  const BoxRec& z = J.F->boxes[g.first + g.count - 1];
  const int64_t lo = a.oR, hi = z.oBa + z.b + z.n;
  RSRS_HIP(hipMemcpyAsync(J.iS + lo, J.hI + lo, (size_t)(hi - lo) * 8, hipMemcpyHostToDevice, st));
  return RSRS_OK;
}

// x (N x s rows in tree order, leading dimension sld) through the processed
// boxes' factors of groups [0, ng): the upward sweep of eq. Ainvfact (V^{-1}:
// E then L per box, groups in order; W^{-T}: F^T then U^T) or the downward
// one (W^{-1}: U then F per box, groups in reverse order; V^{-T}: L^T then
// E^T), in place, as the solve applies them to its right-hand sides.
template <typename T>
rsrs_status redraw_sweep(Job<T>& J, size_t ng, T* x, bool down, bool transpose, Uploader& up, hipStream_t st) {
  const int64_t ld = J.sld;
  const int W = (int)J.s;
  const T* dS = J.dS;
  const int64_t* iS = J.iS;
  auto one = [&](const Group& g) -> rsrs_status {
    std::vector<GemmDescT<T, T>> a0, a1, b0, b1;
    for (int64_t q = g.first; q < g.first + g.count; ++q) {
      const BoxRec& R = J.F->boxes[q];
      const int r = (int)R.r, k = (int)R.k, kn = (int)(R.k + R.n);
      if (r == 0) continue;
      const int64_t* gR = iS + R.oR;
      const int64_t* gS = iS + R.oS;
      const int64_t* gSN = iS + R.oS;
      const T* Tm = dS + R.oT;
      const T* KU = dS + R.oKU;
      const T* KL = dS + R.oKL;
      const int64_t lT = R.ldT, lR = R.ldR, lU = R.ldKU;
      if (!down && !transpose) {          // E then L
        if (k > 0) a0.push_back(gdescT<T, T>(Tm, nullptr, lT, x, gS, ld, x, gR, ld, r, W, k, -1.0, 1.0));
        if (kn > 0) b0.push_back(gdescT<T, T>(KL, nullptr, lR, x, gR, ld, x, gSN, ld, kn, W, r, -1.0, 1.0));
      } else if (!down) {                 // F^T then U^T
        if (k > 0) a0.push_back(gdescT<T, T>(Tm, nullptr, lT, x, gS, ld, x, gR, ld, r, W, k, -1.0, 1.0));
        if (kn > 0) b1.push_back(gdescT<T, T>(KU, nullptr, lU, x, gR, ld, x, gSN, ld, kn, W, r, -1.0, 1.0));
      } else if (!transpose) {            // U then F
        if (kn > 0) a0.push_back(gdescT<T, T>(KU, nullptr, lU, x, gSN, ld, x, gR, ld, r, W, kn, -1.0, 1.0));
        if (k > 0) b1.push_back(gdescT<T, T>(Tm, nullptr, lT, x, gR, ld, x, gS, ld, k, W, r, -1.0, 1.0));
      } else {                            // L^T then E^T
        if (kn > 0) a1.push_back(gdescT<T, T>(KL, nullptr, lR, x, gSN, ld, x, gR, ld, r, W, kn, -1.0, 1.0));
        if (k > 0) b1.push_back(gdescT<T, T>(Tm, nullptr, lT, x, gR, ld, x, gS, ld, k, W, r, -1.0, 1.0));
      }
    }
    RSRS_TRY(gemm<T, T>(up, st, a0, 0, 0, GM_FULL, GS_64x64, "redraw"));
    RSRS_TRY(gemm<T, T>(up, st, a1, 1, 0, GM_FULL, GS_64x64, "redraw"));
    RSRS_TRY(gemm<T, T>(up, st, b0, 0, 0, GM_FULL, GS_64x64, "redraw"));
    RSRS_TRY(gemm<T, T>(up, st, b1, 1, 0, GM_FULL, GS_64x64, "redraw"));
    return RSRS_OK;
  };
  if (down)
    for (size_t g = ng; g-- > 0;) RSRS_TRY(one(J.F->groups[g]));
  else
    for (size_t g = 0; g < ng; ++g) RSRS_TRY(one(J.F->groups[g]));
  return RSRS_OK;
}

// Fresh samples of the partially factored operator V^{-1} A W^{-1} (groups
// [0, ng) processed; the sketches are a sample pair of it, Sec. 1.1), in
// place of the sketches: Omega' from the generator in tree order (word 2 r
// for the r-th redraw), Y' = V^{-1} A W^{-1} Omega', and for the general
// variant Psi' (word 2 r + 1), Z' = W^{-T} A^T V^{-T} Psi'.  The operator
// gets and returns blocks in user point order.
template <typename T>
rsrs_status redraw_job(Job<T>& J, size_t ng, Uploader& up, hipStream_t st) {
  constexpr int dt = sizeof(T) == 8 ? RSRS_F64 : RSRS_F32;
  const int64_t n = J.n, s = J.s, ld = J.sld;
  const size_t bytes = (size_t)n * ld * sizeof(T);
  if (!J.rd_x.p) {
    RSRS_TRY(J.rd_x.alloc(bytes));
    RSRS_TRY(J.rd_u.alloc(bytes));
    RSRS_TRY(J.rd_y.alloc(bytes));
    RSRS_TRY(J.rd_iperm.alloc((size_t)n * 8));
    RSRS_TRY(pool_alloc(J.rd_hiperm, (size_t)n * 8));
    int64_t* ip = J.rd_hiperm.template as<int64_t>();
    const auto& perm = J.tree().perm;
    for (int64_t i = 0; i < n; ++i) ip[perm[i]] = i;
    RSRS_HIP(hipMemcpyAsync(J.rd_iperm.p, ip, (size_t)n * 8, hipMemcpyHostToDevice, st));
  }
  ++J.redraws;
  T* x = J.rd_x.template as<T>();
  T* u = J.rd_u.template as<T>();
  T* y = J.rd_y.template as<T>();
  const int64_t* iperm = J.rd_iperm.template as<int64_t>();
  const int64_t* perm = J.F->perm.template as<int64_t>();
  for (int side = 0; side < (J.sym ? 1 : 2); ++side) {
    T* Tst = side ? J.Psi : J.Om;
    T* Ysd = side ? J.Z : J.Y;
    philox_normal<T>(st, Tst, n, s, ld, J.rd->seed, (uint32_t)(2 * J.redraws + side));
    RSRS_HIP(hipMemcpyAsync(x, Tst, bytes, hipMemcpyDeviceToDevice, st));
    // W^{-1} (V^{-T} for the transposed side), then A (A^T) in user order
    RSRS_TRY(redraw_sweep<T>(J, ng, x, true, side == 1, up, st));
    gather_rows<T, T>(st, u, ld, x, ld, iperm, n, s);
    if (J.rd->mv(J.rd->user, side, dt, s, u, ld, y, ld, st) != 0) {
      set_error("matvec callback returned nonzero (per-level redraw)");
      return RSRS_E_CALLBACK;
    }
    gather_rows<T, T>(st, Ysd, ld, y, ld, perm, n, s);
    // V^{-1} (W^{-T})
    RSRS_TRY(redraw_sweep<T>(J, ng, Ysd, false, side == 1, up, st));
  }
  return RSRS_OK;
}

template <typename T>
rsrs_status factor_many(std::vector<Job<T>>& jobs, hipStream_t st) {
  constexpr bool mixed = Job<T>::mixed;
  auto t0 = std::chrono::steady_clock::now();
  size_t nsteps = 0, ws_max = 0, wsb_max = 0, root_total = 0, pos_max = 1;
  for (auto& J : jobs) nsteps = std::max(nsteps, J.F->groups.size());
  for (size_t t = 0; t < nsteps; ++t) {
    size_t w = 0, wb = 0, np = 0;
    for (auto& J : jobs)
      if (t < J.class_ws.size()) {
        w += J.class_ws[t];
        wb += J.class_wsb[t];
        const Group& g = J.F->groups[t];
        for (int64_t q = 0; q < g.count; ++q) np += (size_t)J.F->boxes[g.first + q].b + 1;
      }
    ws_max = std::max(ws_max, w);
    wsb_max = std::max(wsb_max, wb);
    pos_max = std::max(pos_max, np);
  }
  for (auto& J : jobs) root_total += J.root_ws;
  ws_max = std::max(ws_max, root_total);

  DevBuf ws, wsb[2], flagbuf;
  RSRS_TRY(pool_alloc(ws, ws_max));
  RSRS_TRY(pool_alloc(wsb[0], std::max<size_t>(wsb_max, 256)));
  RSRS_TRY(pool_alloc(wsb[1], std::max<size_t>(wsb_max, 256)));
  RSRS_TRY(flagbuf.alloc(256));
  int* flag = flagbuf.as<int>();
  RSRS_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
  Uploader up;
  RSRS_TRY(up.init((size_t)64 << 20, st, true));
  // The extraction, Gauss-Jordan and sketch updates of a class run on a
  // second stream (with its own descriptor uploads) while the main stream
  // goes on with the next class's Gram matrices and Cholesky factorizations;
  // the next projections wait for them (event eB), and they wait for the
  // skeletons and the test-matrix sparsification of their class (event eA).
  Uploader up2;   // declared first: destroyed after the side stream drains
  SideStream side;
  RSRS_TRY(side.init());
  RSRS_TRY(up2.init((size_t)64 << 20, side.st, true));
  const hipStream_t st2 = side.st;
  EnqueueWorker worker;   // declared after up2 / side: finishes before they go
  RSRS_TRY(worker.start());
  HostBuf hperm;   // pinned staging of the permutations
  {
    size_t tot = 0;
    for (auto& J : jobs) tot += (size_t)J.n;
    RSRS_TRY(pool_alloc(hperm, std::max<size_t>(tot, 1) * 8));
  }
  size_t pofs0 = 0;
  for (auto& J : jobs) {
    int64_t* hp = hperm.as<int64_t>() + pofs0;
    pofs0 += (size_t)J.n;
    std::memcpy(hp, J.tree().perm.data(), (size_t)J.n * 8);
    RSRS_HIP(hipMemcpyAsync(J.F->perm.p, hp, (size_t)J.n * 8, hipMemcpyHostToDevice, st));
    // non-finite samples are rejected up front
    check_finite(st, J.Y, J.n, J.s, J.sld, flag);
    check_finite(st, J.Om, J.n, J.s, J.sld, flag);
    if (!J.sym) {
      check_finite(st, J.Z, J.n, J.s, J.sld, flag);
      check_finite(st, J.Psi, J.n, J.s, J.sld, flag);
    }
  }
  RSRS_TRY(up.reset());
  {
    int hflag = 0;
    RSRS_HIP(hipMemcpy(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost));
    if (hflag & 4) { set_error("non-finite value in the samples"); return RSRS_E_NUMERIC; }
  }
  // from here on the samples are modified in place
  for (auto& J : jobs) J.smp->consumed = true;

  HostBuf hpos;   // skeleton positions of a class, read back, then the flag word
  RSRS_TRY(pool_alloc(hpos, (pos_max + 1) * 8));
  int* hflag_slot = reinterpret_cast<int*>(hpos.as<int64_t>() + pos_max);
  const bool deferred = !jobs.empty() && jobs[0].deferred;
  for (size_t t = 0; t < nsteps; ++t) {
    // ---- per-level redraw: a job entering a processed level after its first
    // starts it from fresh samples, once every earlier class has finished
    // (phase B of the previous class included)
    {
      bool any = false;
      for (auto& J : jobs) any = any || (J.rd && t > 0 && t < J.F->groups.size() && J.ci == 0);
      if (any) {
        RSRS_TRY(worker.join());
        RSRS_HIP(hipStreamWaitEvent(st, side.eB, 0));
        for (auto& J : jobs)
          if (J.rd && t > 0 && t < J.F->groups.size() && J.ci == 0) RSRS_TRY(redraw_job<T>(J, t, up, st));
      }
    }
    // ---- host index lists and factor-store uploads (Ba, Na, Na copy)
    std::vector<Item<T>> items;
    std::vector<int64_t> nbs;
    std::vector<ListSeg> lsegs;
    for (auto& J : jobs) {
      if (t >= J.F->groups.size()) continue;
      const Tree& tr = J.tree();
      const Group& g = J.F->groups[t];
      const int lev = J.sch.levels[J.li];
      if (deferred) {
        // the class's B_a, N_a and second N_a slots as segments of the
        // neighbours' and its own pieces (counts are the schedule's)
        for (int64_t q = 0; q < g.count; ++q) {
          BoxRec& R = J.F->boxes[g.first + q];
          const size_t ip = J.pos.at(R.box);
          nbs.assign(tr.nb_ids[lev].begin() + tr.nb_off[lev][ip], tr.nb_ids[lev].begin() + tr.nb_off[lev][ip + 1]);
          std::sort(nbs.begin(), nbs.end(), [&](int64_t x, int64_t y) { return tr.pt_begin[x] < tr.pt_begin[y]; });
          std::vector<typename Job<T>::Piece> na;
          for (int64_t x : nbs) {
            const auto& pc = J.pieces_of(x);
            na.insert(na.end(), pc.begin(), pc.end());
          }
          if (J.emit(lsegs, J.iS + R.oBa, J.pcur[R.box], R.b) != R.b ||
              J.emit(lsegs, J.iS + R.oNa, na, R.n) != R.n || J.emit(lsegs, J.iS + R.oBa + R.b, na, R.n) != R.n) {
            set_error("internal: active sets disagree with the count model");
            return RSRS_E_INVALID;
          }
          items.push_back(Item<T>{&J, &R, {}});
        }
        continue;
      }
      for (int64_t q = 0; q < g.count; ++q) {
        BoxRec& R = J.F->boxes[g.first + q];
        const size_t ip = J.pos.at(R.box);
        const std::vector<int64_t>& ba = J.cur[R.box];
        const bool adaptive = J.rank_tol > 0.0;
        // N_a straight into the staging slots.  Neighbours own disjoint point
        // ranges and keep their active points sorted, so visiting them by
        // range start yields a sorted list.  With a rank tolerance the
        // schedule's counts bound the actual ones.
        if (adaptive ? (int64_t)ba.size() > R.b : (int64_t)ba.size() != R.b) {
          set_error("internal: active sets disagree with the count model");
          return RSRS_E_INVALID;
        }
        nbs.assign(tr.nb_ids[lev].begin() + tr.nb_off[lev][ip], tr.nb_ids[lev].begin() + tr.nb_off[lev][ip + 1]);
        std::sort(nbs.begin(), nbs.end(), [&](int64_t x, int64_t y) { return tr.pt_begin[x] < tr.pt_begin[y]; });
        const int64_t nn = (int64_t)nbs.size();
        int64_t* na = J.hI + R.oNa;
        int64_t cnt = 0;
        bool over = false;
        for (int64_t u = 0; u < nn && !over; ++u) {
          const auto& a = J.active_of(nbs[u]);
          over = cnt + (int64_t)a.size() > R.n;
          if (!over) std::memcpy(na + cnt, a.data(), a.size() * 8);
          cnt += (int64_t)a.size();
        }
        if (over || (adaptive ? cnt > R.n : cnt != R.n)) {
          set_error("internal: active sets disagree with the count model");
          return RSRS_E_INVALID;
        }
        if (adaptive) {   // actual counts; k_B and r follow from the ID
          R.b = (int64_t)ba.size();
          R.n = cnt;
          R.k = std::min<int64_t>(J.k, R.b);
          R.r = R.b - R.k;
        }
        if (!std::is_sorted(na, na + cnt)) std::sort(na, na + cnt);
        std::memcpy(J.hI + R.oBa, ba.data(), R.b * 8);
        std::memcpy(J.hI + R.oBa + R.b, na, R.n * 8);
        if (R.b == 0) {   // every point of the box was eliminated below: nothing to do
          R.k = R.r = 0;
          continue;
        }
        items.push_back(Item<T>{&J, &R, {}});
      }
      // the class's index lists are contiguous: one upload (its R / S slots
      // are filled and uploaded again once the skeletons are known)
      RSRS_TRY(upload_class_lists(J, g, st));
    }
    RSRS_TRY(launch_segments<ListSeg>(up, st, lsegs, list_assemble_kernel, "list_assemble"));
    // ---- workspace: the part read by the extraction alternates between two
    // buffers, the one it reads may still be in use by the previous class
    Bump bump{ws.as<char>(), 0, ws.bytes};
    Bump bumpb{wsb[t & 1].as<char>(), 0, wsb[t & 1].bytes};
    // skeleton / redundant positions of all boxes back to back (S then R,
    // b entries per box, then the box's k_B), so that one copy brings them
    // to the host
    int64_t npos = 0;
    for (auto& it : items) npos += it.R->b + 1;
    if ((size_t)npos > pos_max) {
      set_error("internal: skeleton position count exceeds its plan");
      return RSRS_E_INVALID;
    }
    int64_t* posall = bumpb.take<int64_t>(npos);
    int64_t pofs = 0;
    for (auto& it : items) {
      const BoxRec& R = *it.R;
      const int k = it.J->k;
      const int64_t sld = it.J->sld;
      // r is only known after the ID with a rank tolerance: room for r = b
      const int64_t l = R.b + R.n, lp = round_up(l, 16), b = R.b,
                    r = it.J->rank_tol > 0.0 ? R.b : R.r;
      BoxWs<T>& w = it.w;
      w.lp = lp;
      w.GO = bump.take<T>(l * lp); w.GP = bump.take<T>(l * lp);
      w.LO = bump.take<T>(l * lp); w.LP = bump.take<T>(l * lp);
      w.PY = bump.take<T>(b * lp); w.WY = bump.take<T>(b * lp);
      w.PZ = bump.take<T>(b * lp); w.WZ = bump.take<T>(b * lp);
      if (it.J->concat) {   // rows of [M_Y, M_Z] side by side: M_Z at column sld
        w.MY = bump.take<T>(2 * b * sld);
        w.MZ = w.MY + sld;
        w.mld = 2 * sld;
      } else {
        w.MY = bump.take<T>(b * sld); w.MZ = bump.take<T>(b * sld);
        w.mld = sld;
      }
      w.norms = bump.take<double>(3 * b); w.Rc = bump.take<double>(b * k);
      w.sel = bump.take<int32_t>(b); w.piv = bump.take<int32_t>(k);
      w.XY = bumpb.take<T>(b * lp); w.XZ = bumpb.take<T>(b * lp);
      w.XRy = bumpb.take<T>(r * lp); w.XRz = bumpb.take<T>(r * lp);
      w.Xpy = bumpb.take<T>(r * lp); w.Xpz = bumpb.take<T>(r * lp);
      w.gje = bumpb.take<double>(2 * r * r);
      w.Spos = posall + pofs; w.Rpos = w.Spos + R.k;   // R positions follow the k_B skeletons
      w.kB = posall + pofs + b;
      pofs += b + 1;
      if constexpr (mixed) {
        w.Td = bump.take<double>(r * round_up(k, 4));
        w.XRRd = bumpb.take<double>(r * r); w.Xinvd = bumpb.take<double>(r * r);
        const int64_t srow = it.J->concat ? sld + it.J->sB(l) : it.J->sB(l);
        w.ldmd = round_up(srow, 16);
        w.ldg = round_up(b, 16);
        w.Md = bump.take<double>(b * w.ldmd);
        w.Gm = bump.take<double>(kIdGramSplit * b * w.ldg);   // the partial Gram matrices of the ID
        w.Rt = bump.take<double>(b * k);                         // its R entries, column-major
      } else {
        w.Td = w.XRRd = w.Xinvd = nullptr;
        w.Md = w.Gm = w.Rt = nullptr;
        w.ldmd = w.ldg = 0;
      }
    }
    if (bump.off > bump.cap || bumpb.off > bumpb.cap) {
      set_error("internal: workspace overflow");
      return RSRS_E_INVALID;
    }

    // ---- phase A: Gram matrices and their inverse factors, in T (FP32
    // products and FP32 factorization on the FP32 path)
    {
      std::vector<GemmDescT<T, T>> gd;
      std::vector<CholMatT<T>> cm;
      for (auto& it : items) {
        const BoxRec& R = *it.R;
        const Job<T>& J = *it.J;
        const BoxWs<T>& w = it.w;
        const int l = (int)(R.b + R.n);
        const int64_t* idxC = J.iS + R.oBa;
        // the Gram matrix is factored in place: L^{-1} lands where it is used
        const int sb = J.sB(l);
        gd.push_back(gdescT<T, T>(J.Om, idxC, J.sld, J.Om, idxC, J.sld, w.LO, nullptr, w.lp, l, l, sb));
        cm.push_back(CholMatT<T>{w.LO, w.GO, w.lp, l});
        if (!J.sym) {
          gd.push_back(gdescT<T, T>(J.Psi, idxC, J.sld, J.Psi, idxC, J.sld, w.LP, nullptr, w.lp, l, l, sb));
          cm.push_back(CholMatT<T>{w.LP, w.GP, w.lp, l});
        }
        const double dl = l, db = (double)R.b, ds = (double)sb, sides = J.sym ? 1.0 : 2.0;
        it.J->flops += sides * (dl * dl * ds                              // Gram matrices
                                + (2.0 / 3.0) * dl * dl * dl              // Cholesky + inverse factor
                                + (1.0 + J.reproject) * (4.0 * db * dl * ds + 2.0 * db * dl * dl));  // projections
      }
      RSRS_TRY(gemm<T, T>(up, st, gd, 0, 1, GM_SYRK_L, GS_64x64, "gram"));
      RSRS_TRY(chol_inverse<T>(up, st, cm, flag));
    }
    // ---- projections (eq. nullYZ) and least-squares coefficients, once the
    // previous class has updated the sketches
    if (t > 0) {
      RSRS_TRY(worker.join());   // phase B of the previous class is enqueued
      RSRS_HIP(hipStreamWaitEvent(st, side.eB, 0));
    }
    for (auto& it : items)   // [M_Y, M_Z] rows: the columns s_B..sld of each half stay zero
      if (it.J->concat && it.J->sld > it.J->sB(it.R->b + it.R->n))
        RSRS_HIP(hipMemsetAsync(it.w.MY, 0, (size_t)(2 * it.R->b * it.J->sld) * sizeof(T), st));
    for (int pass = 0; pass <= 1; ++pass) {
      std::vector<GemmDescT<T, T>> gp, gw, gx, gm;
      std::vector<Copy2DT<T, T>> acc;
      for (auto& it : items) {
        const Job<T>& J = *it.J;
        if (pass > J.reproject) continue;
        const BoxRec& R = *it.R;
        const BoxWs<T>& w = it.w;
        const int l = (int)(R.b + R.n), b = (int)R.b, sb = J.sB(l);
        const int64_t* idxB = J.iS + R.oBa;
        const int64_t* idxC = J.iS + R.oBa;
        const int64_t sld = J.sld;
        for (int side = 0; side < (J.sym ? 1 : 2); ++side) {
          T* Ysd = side ? J.Z : J.Y;
          T* Tst = side ? J.Psi : J.Om;
          T* Pb = side ? w.PZ : w.PY;
          T* Wb = side ? w.WZ : w.WY;
          T* Xb = side ? w.XZ : w.XY;
          T* Mb = side ? w.MZ : w.MY;
          T* Lb = side ? w.LP : w.LO;
          T* Xout = pass == 0 ? Xb : Pb;   // second pass: correction into P
          if (pass == 0)
            gp.push_back(gdescT<T, T>(Ysd, idxB, sld, Tst, idxC, sld, Pb, nullptr, w.lp, b, l, sb));
          else
            gp.push_back(gdescT<T, T>(Mb, nullptr, w.mld, Tst, idxC, sld, Pb, nullptr, w.lp, b, l, sb));
          gw.push_back(gdescT<T, T>(Pb, nullptr, w.lp, Lb, nullptr, w.lp, Wb, nullptr, w.lp, b, l, l));
          gx.push_back(gdescT<T, T>(Wb, nullptr, w.lp, Lb, nullptr, w.lp, Xout, nullptr, w.lp, b, l, l));
          if (pass == 0)
            gm.push_back(gdescT<T, T>(Xout, nullptr, w.lp, Tst, idxC, sld, Mb, nullptr, w.mld, b, sb, l,
                                      -1.0, 1.0, Ysd, idxB, sld));
          else
            gm.push_back(gdescT<T, T>(Xout, nullptr, w.lp, Tst, idxC, sld, Mb, nullptr, w.mld, b, sb, l,
                                      -1.0, 1.0));
          if (pass == 1) acc.push_back(Copy2DT<T, T>{Pb, Xb, w.lp, w.lp, b, l, 1.0, 1, 0});
        }
      }
      if (gp.empty()) continue;
      RSRS_TRY(gemm<T, T>(up, st, gp, 0, 1, GM_FULL, GS_64x64, "proj"));
      RSRS_TRY(gemm<T, T>(up, st, gw, 0, 1, GM_B_NT_LOW, GS_64x64, "proj"));
      RSRS_TRY(gemm<T, T>(up, st, gx, 0, 0, GM_B_NN_LOW, GS_64x64, "proj"));
      RSRS_TRY(gemm<T, T>(up, st, gm, 0, 0, GM_FULL, GS_64x64, "proj"));
      RSRS_TRY(copy2d<T, T>(up, st, acc));
    }
    // ---- interpolative decomposition of M = M_Y + M_Z
    {
      std::vector<IdDesc> idd;
      for (auto& it : items) {
        const BoxRec& R = *it.R;
        const Job<T>& J = *it.J;
        const BoxWs<T>& w = it.w;
        IdDesc e{};
        // symmetric variant: M = M_Y (the ID of 2 M_Y is the same).  The
        // working rows keep the sketches' type; the pivoting is FP64.
        // Concatenated sketches: one row of length sld + s, the padding
        // columns between the halves zero.
        e.M = w.MY;
        e.MZ = (J.sym || J.concat) ? nullptr : w.MZ;
        e.ldm = w.mld; e.ldz = w.mld;
        if constexpr (mixed) {
          e.T = w.Td; e.ldt = (int)round_up(J.k, 4);
        } else {
          e.T = J.dS + R.oT; e.ldt = (int)R.ldT;
        }
        e.norms = w.norms; e.sel = w.sel; e.Rc = w.Rc; e.piv = w.piv;
        e.Spos = w.Spos; e.kB = w.kB;
        const int sb = J.sB(R.b + R.n);
        e.b = (int)R.b; e.s = (int)(J.concat ? J.sld + sb : sb); e.k = (int)R.k;
        // rank tolerance: |R_jj|^2 against rank_tol^2 ||[Y_B Z_B]||_F^2, whose
        // row sums the first launch gathers from the sketches (Y_B only in
        // the symmetric variant, whose R is half that of M_Y + M_Z = 2 M_Y)
        e.tol2 = J.rank_tol > 0.0 ? J.rank_tol * J.rank_tol * (J.sym ? 0.25 * 2.0 : 1.0) : 0.0;
        e.rowyz = w.norms + 2 * R.b;
        e.Yg = J.Y; e.Zg = J.sym ? nullptr : J.Z; e.idx = J.iS + R.oBa; e.ldy = J.sld; e.sy = sb;
        e.Md = w.Md; e.G = w.Gm; e.Rt = w.Rt; e.ldmd = w.ldmd; e.ldg = w.ldg;
        idd.push_back(e);
        it.J->flops += 4.0 * R.b * e.s * R.k;
      }
      // FP32 rows: the pivoted QR through the FP64 Gram matrix of the rows
      if constexpr (mixed) RSRS_TRY(id_run_gram(up, st, idd));
      else RSRS_TRY(id_run(up, st, idd, false));
    }
    if (deferred) {
      // ---- S and R slots from the ID's positions, on the device; the
      // skeleton counts are the schedule's (k_B = min(k, b))
      std::vector<SkelSeg> ss;
      for (auto& it : items) {
        Job<T>& J = *it.J;
        const BoxRec& R = *it.R;
        ss.push_back(SkelSeg{J.iS + R.oBa, it.w.Spos, J.iS + R.oS, J.iS + R.oR, (int)R.b, (int)R.k});
      }
      RSRS_TRY(launch_segments<SkelSeg>(up, st, ss, skel_scatter_kernel, "skel_scatter"));
      for (auto& it : items) {
        Job<T>& J = *it.J;
        const BoxRec& R = *it.R;
        J.pcur[R.box].clear();
        if (R.k > 0) J.pcur[R.box].push_back(typename Job<T>::Piece{J.iS + R.oS, 0, R.k});
      }
    }
    if (!deferred) {
      // ---- skeleton sets back to the host (one copy, positions back to back)
      // and the flag word behind them, so that one synchronisation brings both
      *hflag_slot = 0;
      RSRS_HIP(hipMemcpyAsync(hpos.as<int64_t>(), posall, (size_t)npos * 8, hipMemcpyDeviceToHost, st));
      RSRS_HIP(hipMemcpyAsync(hflag_slot, flag, sizeof(int), hipMemcpyDeviceToHost, st));
      RSRS_TRY(up.reset());
      {
        const int hflag = *hflag_slot;
        if (hflag & 1) {
          set_error("Gram matrix of a test-matrix panel is not positive definite (rank-deficient panel)");
          return RSRS_E_SINGULAR;
        }
      }
      // ---- phase B: global R / S / SN lists (k_B of each box from the ID)
      {
        int64_t o2 = 0;
        for (auto& it : items) {
          Job<T>& J = *it.J;
          BoxRec& R = *it.R;
          const int64_t* sp = hpos.as<int64_t>() + o2;
          const int64_t kb = sp[R.b];
          if (kb < 0 || kb > R.k) {
            set_error("internal: skeleton count out of range");
            return RSRS_E_INVALID;
          }
          R.k = kb;
          R.r = R.b - kb;
          R.oS = R.oNa - kb;          // S ends where N_a begins: S || N_a = SN
          it.w.Rpos = it.w.Spos + kb;
          const int64_t* rp = sp + kb;
          std::vector<int64_t> Sg((size_t)kb), Rg((size_t)R.r);
          const int64_t* ba = J.hI + R.oBa;   // B_a as staged for the upload
          for (int64_t j = 0; j < kb; ++j) Sg[j] = ba[sp[j]];
          for (int64_t j = 0; j < R.r; ++j) Rg[j] = ba[rp[j]];
          std::memcpy(J.hI + R.oR, Rg.data(), R.r * 8);
          std::memcpy(J.hI + R.oS, Sg.data(), (size_t)kb * 8);
          J.cur[R.box] = std::move(Sg);
          o2 += R.b + 1;
        }
        for (auto& J : jobs)
          if (t < J.F->groups.size()) RSRS_TRY(upload_class_lists(J, J.F->groups[t], st));
      }
    }
    {
      if constexpr (mixed) {   // T rounded into the factor store
        std::vector<Copy2DT<double, T>> tc;
        for (auto& it : items) {
          const BoxRec& R = *it.R;
          tc.push_back(Copy2DT<double, T>{it.w.Td, it.J->dS + R.oT, round_up(it.J->k, 4), R.ldT, (int)R.r,
                                          (int)R.k, 1.0, 0, 0});
        }
        RSRS_TRY(copy2d<double, T>(up, st, tc));
      }
    }
    // boxes that keep every point (k_B = b) eliminate nothing: no sparsify,
    // extraction or elimination work
    items.erase(std::remove_if(items.begin(), items.end(), [](const Item<T>& it) { return it.R->r == 0; }),
                items.end());
    // ---- test-matrix sparsification (F) on the main stream: the next
    // class's Gram matrices read the updated rows S
    {
      std::vector<GemmDescT<T, T>> s1;
      for (auto& it : items) {
        const BoxRec& R = *it.R;
        const Job<T>& J = *it.J;
        const int k = (int)R.k, s = (int)J.s;
        const int r = (int)R.r;
        if (k == 0) continue;   // no skeletons: nothing to add to
        const int64_t* gR = J.iS + R.oR;
        const int64_t* gS = J.iS + R.oS;
        const T* Tm = J.dS + R.oT;
        s1.push_back(gdescT<T, T>(Tm, nullptr, R.ldT, J.Om, gR, J.sld, J.Om, gS, J.sld, k, s, r, 1.0, 1.0));
        if (!J.sym)
          s1.push_back(gdescT<T, T>(Tm, nullptr, R.ldT, J.Psi, gR, J.sld, J.Psi, gS, J.sld, k, s, r, 1.0, 1.0));
      }
      RSRS_TRY(gemm<T, T>(up, st, s1, 1, 0, GM_FULL, GS_64x64, "sparsify"));
    }
    RSRS_HIP(hipEventRecord(side.eA, st));
    RSRS_HIP(hipStreamWaitEvent(st2, side.eA, 0));
    // phase B of this class, enqueued on the side stream by the worker
    worker.submit([&, items = std::move(items)]() -> rsrs_status {
      {
        std::vector<GemmDescT<T, T>> gxr;
        std::vector<ColfixDescT<T>> cf;
        std::vector<Copy2DT<T, T>> cx;
        std::vector<Copy2DT<T, double>> cxd;
        std::vector<Copy2DT<double, T>> cinv;
        std::vector<GjeDesc> gj;
        std::vector<SymDesc<T>> symx;
        std::vector<SymDesc<double>> symi;
        for (auto& it : items) {
          const BoxRec& R = *it.R;
          Job<T>& J = *it.J;
          const BoxWs<T>& w = it.w;
          const int k = (int)R.k;
          T* dS = J.dS;
          const int l = (int)(R.b + R.n), r = (int)R.r;
          if (J.sym) {   // symmetric part of X_RR, and of its inverse below
            symx.push_back(SymDesc<T>{w.Xpy, w.lp, r, 0});
            if constexpr (mixed) symi.push_back(SymDesc<double>{w.Xinvd, r, r, 0});
            else symi.push_back(SymDesc<double>{reinterpret_cast<double*>(dS + R.oXinv), R.ldR, r, 0});
          }
          for (int side = 0; side < (J.sym ? 1 : 2); ++side) {
            T* Xb = side ? w.XZ : w.XY;
            T* XR = side ? w.XRz : w.XRy;
            T* Xp = side ? w.Xpz : w.Xpy;
            gxr.push_back(gdescT<T, T>(dS + R.oT, nullptr, R.ldT, Xb, w.Spos, w.lp, XR, nullptr, w.lp, r, l, k,
                                       -1.0, 1.0, Xb, w.Rpos, w.lp));
            cf.push_back(ColfixDescT<T>{XR, w.Spos, w.Rpos, dS + R.oT, Xp, w.lp, w.lp, R.ldT, r, k, (int)R.b, l});
          }
          cx.push_back(Copy2DT<T, T>{w.Xpy, dS + R.oXRR, w.lp, R.ldR, r, r, 1.0, 0, 0});
          if constexpr (mixed) {   // FP64 Gauss-Jordan on X_RR, inverse rounded
            cxd.push_back(Copy2DT<T, double>{w.Xpy, w.XRRd, w.lp, r, r, r, 1.0, 0, 0});
            gj.push_back(GjeDesc{w.XRRd, w.gje, w.Xinvd, r, r, r, 0});
            cinv.push_back(Copy2DT<double, T>{w.Xinvd, dS + R.oXinv, r, R.ldR, r, r, 1.0, 0, 0});
          } else {
            gj.push_back(GjeDesc{reinterpret_cast<const double*>(w.Xpy), w.gje,
                                 reinterpret_cast<double*>(dS + R.oXinv), w.lp, R.ldR, r, 0});
          }
          const double dr = r, dk = k, dn = (double)R.n, ds = (double)J.s, sides = J.sym ? 1.0 : 2.0;
          J.flops_b += sides * (2.0 * dr * dk * l + 2.0 * dr * dr * dk) + 2.0 * dr * dr * dr +
                     sides * 2.0 * dr * dr * (dk + dn) + sides * 2.0 * 2.0 * dr * dk * ds +
                     sides * 2.0 * 2.0 * dr * (dk + dn) * ds;
        }
        RSRS_TRY(gemm<T, T>(up2, st2, gxr, 0, 0, GM_FULL, GS_64x64, "extract"));
        RSRS_TRY(colfix<T>(up2, st2, cf));
        RSRS_TRY(symmetrize<T>(up2, st2, symx));
        RSRS_TRY(copy2d<T, T>(up2, st2, cx));
        RSRS_TRY(copy2d<T, double>(up2, st2, cxd));
        RSRS_TRY(gje_inverse(up2, st2, gj, flag));
        RSRS_TRY(symmetrize<double>(up2, st2, symi));
        RSRS_TRY(copy2d<double, T>(up2, st2, cinv));
      }
      {
        std::vector<GemmDescT<T, T>> gku, gkl;
        std::vector<Copy2DT<T, T>> ktr;
        for (auto& it : items) {
          const BoxRec& R = *it.R;
          const BoxWs<T>& w = it.w;
          T* dS = it.J->dS;
          const int r = (int)R.r, kn = (int)(R.k + R.n);
          if (kn == 0) continue;   // no skeletons and no neighbours: no multipliers
          gku.push_back(gdescT<T, T>(dS + R.oXinv, nullptr, R.ldR, w.Xpy + r, nullptr, w.lp, dS + R.oKU, nullptr, R.ldKU, r, kn, r));
          if (it.J->sym)   // K_L = K_U^T
            ktr.push_back(Copy2DT<T, T>{dS + R.oKU, dS + R.oKL, R.ldKU, R.ldR, kn, r, 1.0, 0, 1});
          else
            gkl.push_back(gdescT<T, T>(w.Xpz + r, nullptr, w.lp, dS + R.oXinv, nullptr, R.ldR, dS + R.oKL, nullptr, R.ldR, kn, r, r));
        }
        RSRS_TRY(gemm<T, T>(up2, st2, gku, 0, 0, GM_FULL, GS_64x64, "mult"));
        RSRS_TRY(gemm<T, T>(up2, st2, gkl, 1, 0, GM_FULL, GS_64x64, "mult"));
        RSRS_TRY(copy2d<T, T>(up2, st2, ktr));
      }
      // ---- sketch updates: sparsify (E) then eliminate (L, U)
      {
        std::vector<GemmDescT<T, T>> s0, e0, e1, e0b, e1b;
        for (auto& it : items) {
          const BoxRec& R = *it.R;
          const Job<T>& J = *it.J;
          const int k = (int)R.k, s = (int)J.s;
          const int64_t sld = J.sld;
          const int r = (int)R.r, kn = (int)(k + R.n);
          if (kn == 0) continue;   // nothing outside R is coupled to it
          const int64_t* gR = J.iS + R.oR;
          const int64_t* gS = J.iS + R.oS;
          const int64_t* gSN = J.iS + R.oS;
          const T* Tm = J.dS + R.oT;
          const T* KU = J.dS + R.oKU;
          const T* KL = J.dS + R.oKL;
          const int64_t lT = R.ldT, lR = R.ldR, lU = R.ldKU;
          if (k > 0) s0.push_back(gdescT<T, T>(Tm, nullptr, lT, J.Y, gS, sld, J.Y, gR, sld, r, s, k, -1.0, 1.0));
          e0.push_back(gdescT<T, T>(KL, nullptr, lR, J.Y, gR, sld, J.Y, gSN, sld, kn, s, r, -1.0, 1.0));
          e0b.push_back(gdescT<T, T>(KU, nullptr, lU, J.Om, gSN, sld, J.Om, gR, sld, r, s, kn, 1.0, 1.0));
          if (J.sym) continue;   // Z = Y and Psi = Omega: nothing more to update
          if (k > 0) s0.push_back(gdescT<T, T>(Tm, nullptr, lT, J.Z, gS, sld, J.Z, gR, sld, r, s, k, -1.0, 1.0));
          e1.push_back(gdescT<T, T>(KU, nullptr, lU, J.Z, gR, sld, J.Z, gSN, sld, kn, s, r, -1.0, 1.0));
          e1b.push_back(gdescT<T, T>(KL, nullptr, lR, J.Psi, gSN, sld, J.Psi, gR, sld, r, s, kn, 1.0, 1.0));
        }
        RSRS_TRY(gemm<T, T>(up2, st2, s0, 0, 0, GM_FULL, GS_64x64, "sparsify"));
        RSRS_TRY(gemm<T, T>(up2, st2, e0, 0, 0, GM_FULL, GS_64x64, "elim"));
        RSRS_TRY(gemm<T, T>(up2, st2, e1, 1, 0, GM_FULL, GS_64x64, "elim"));
        RSRS_TRY(gemm<T, T>(up2, st2, e0b, 0, 0, GM_FULL, GS_64x64, "elim_r"));
        RSRS_TRY(gemm<T, T>(up2, st2, e1b, 1, 0, GM_FULL, GS_64x64, "elim_r"));
      }
      RSRS_HIP(hipEventRecord(side.eB, st2));
      return RSRS_OK;
    });
    // ---- advance every job past this class
    for (auto& J : jobs) {
      if (t >= J.F->groups.size()) continue;
      ++J.ci;
      if (J.ci == J.sch.classes[J.li].size()) {
        J.leave_level();
        J.settle();
      }
    }
  }

  // ---- roots: A_t = Y_Bt pinv(Omega_Bt), all problems in the same launches
  RSRS_TRY(worker.join());
  if (nsteps > 0) RSRS_HIP(hipStreamWaitEvent(st, side.eB, 0));
  {
    Bump bump{ws.as<char>(), 0, ws.bytes};
    struct Root {
      const double *Yr, *Or;
      const int64_t* ir;
      int64_t rld, ntp, rp;
      double *G, *L, *P, *Wb, *Rres, *gw, *At, *Atinv;
      int nt, s, reproject;
      Job<T>* job;
    };
    std::vector<Root> roots;
    std::vector<ListSeg> rsegs;
    for (auto& J : jobs) {
      rsrs_factor_t* F = J.F.get();
      const Tree& tr = J.tree();
      std::vector<int64_t> Bt;
      if (deferred) {
        // B_t: the level-1 boxes' remaining pieces in point-range order
        std::vector<typename Job<T>::Piece> pc;
        if (tr.nlevels == 0) {
          pc.push_back(typename Job<T>::Piece{nullptr, 0, J.n});
        } else {
          std::vector<int64_t> top(tr.level_boxes[1].begin(), tr.level_boxes[1].end());
          std::sort(top.begin(), top.end(), [&](int64_t x, int64_t y) { return tr.pt_begin[x] < tr.pt_begin[y]; });
          for (int64_t b : top) pc.insert(pc.end(), J.prem[b].begin(), J.prem[b].end());
        }
        if (J.emit(rsegs, J.iS + F->oBt, pc, F->nt) != F->nt) {
          set_error("internal: root size mismatch");
          return RSRS_E_INVALID;
        }
        RSRS_TRY(launch_segments<ListSeg>(up, st, rsegs, list_assemble_kernel, "list_assemble"));
        rsegs.clear();
      } else if (tr.nlevels == 0) {
        Bt.resize((size_t)J.n);
        std::iota(Bt.begin(), Bt.end(), 0);
      } else {
        for (int64_t b : tr.level_boxes[1]) Bt.insert(Bt.end(), J.remaining[b].begin(), J.remaining[b].end());
        std::sort(Bt.begin(), Bt.end());
      }
      // with a rank tolerance the schedule's root count bounds the actual one
      if (!deferred && (J.rank_tol > 0.0 ? (int64_t)Bt.size() > F->nt : (int64_t)Bt.size() != F->nt)) {
        set_error("internal: root size mismatch");
        return RSRS_E_INVALID;
      }
      if (!deferred) F->nt = (int64_t)Bt.size();
      if (F->nt == 0) continue;   // every point eliminated: no root block
      Root R{};
      R.job = &J;
      R.nt = (int)F->nt;
      R.s = (int)J.s;
      R.reproject = J.reproject;
      const int nt = R.nt;
      if (!deferred) {
        std::memcpy(J.hI + F->oBt, Bt.data(), (size_t)nt * 8);
        RSRS_HIP(hipMemcpyAsync(J.iS + F->oBt, J.hI + F->oBt, (size_t)nt * 8, hipMemcpyHostToDevice, st));
      }
      const int64_t* iBt = J.iS + F->oBt;
      R.ntp = round_up(nt, 16);
      R.rp = round_up(J.s, 16);
      R.G = bump.take<double>(nt * R.ntp);
      R.L = bump.take<double>(nt * R.ntp);
      R.P = bump.take<double>(nt * R.ntp);
      R.Wb = bump.take<double>(nt * R.ntp);
      R.Rres = bump.take<double>(nt * R.rp);
      R.gw = bump.take<double>(2 * (int64_t)nt * nt);
      // FP64 operands of the root: the samples themselves (rows iBt), or FP64
      // copies of the rows B_t in mixed precision
      if constexpr (mixed) {
        double* Yd = bump.take<double>(nt * R.rp);
        double* Od = bump.take<double>(nt * R.rp);
        R.At = bump.take<double>((int64_t)nt * nt);
        R.Atinv = bump.take<double>((int64_t)nt * nt);
        gather_rows<T, double>(st, Yd, R.rp, J.Y, J.sld, iBt, nt, J.s);
        gather_rows<T, double>(st, Od, R.rp, J.Om, J.sld, iBt, nt, J.s);
        R.Yr = Yd; R.Or = Od; R.ir = nullptr; R.rld = R.rp;
      } else {
        R.Yr = reinterpret_cast<const double*>(J.Y);
        R.Or = reinterpret_cast<const double*>(J.Om);
        R.ir = iBt; R.rld = J.sld;
        R.At = reinterpret_cast<double*>(J.dS + F->oAt);
        R.Atinv = reinterpret_cast<double*>(J.dS + F->oAtinv);
      }
      roots.push_back(R);
      const double dt = nt;
      J.flops += dt * dt * J.s + (2.0 / 3.0) * dt * dt * dt +
                 (1 + J.reproject) * (2.0 * dt * dt * J.s + 2.0 * dt * dt * dt) + 2.0 * dt * dt * dt;
    }
    if (bump.off > bump.cap) { set_error("internal: root workspace overflow"); return RSRS_E_INVALID; }
    std::vector<GemmDesc> g0, g1, g2, g3;
    std::vector<CholMat> cm;
    for (auto& R : roots) {
      g0.push_back(gdesc(R.Or, R.ir, R.rld, R.Or, R.ir, R.rld, R.L, nullptr, R.ntp, R.nt, R.nt, R.s));
      cm.push_back(CholMat{R.L, R.G, R.ntp, R.nt});
      g1.push_back(gdesc(R.Yr, R.ir, R.rld, R.Or, R.ir, R.rld, R.P, nullptr, R.ntp, R.nt, R.nt, R.s));
      g2.push_back(gdesc(R.P, nullptr, R.ntp, R.L, nullptr, R.ntp, R.Wb, nullptr, R.ntp, R.nt, R.nt, R.nt));
      g3.push_back(gdesc(R.Wb, nullptr, R.ntp, R.L, nullptr, R.ntp, R.At, nullptr, R.nt, R.nt, R.nt, R.nt));
    }
    RSRS_TRY(gemm(up, st, g0, 0, 1, GM_SYRK_L));
    RSRS_TRY(chol_inverse<double>(up, st, cm, flag));
    RSRS_TRY(gemm(up, st, g1, 0, 1, GM_FULL));
    RSRS_TRY(gemm(up, st, g2, 0, 1, GM_B_NT_LOW));
    RSRS_TRY(gemm(up, st, g3, 0, 0, GM_B_NN_LOW));
    {
      std::vector<GemmDesc> h0, h1, h2, h3;
      for (auto& R : roots) {
        if (!R.reproject) continue;
        h0.push_back(gdesc(R.At, nullptr, R.nt, R.Or, R.ir, R.rld, R.Rres, nullptr, R.rp, R.nt, R.s, R.nt,
                           -1.0, 1.0, R.Yr, R.ir, R.rld));
        h1.push_back(gdesc(R.Rres, nullptr, R.rp, R.Or, R.ir, R.rld, R.P, nullptr, R.ntp, R.nt, R.nt, R.s));
        h2.push_back(gdesc(R.P, nullptr, R.ntp, R.L, nullptr, R.ntp, R.Wb, nullptr, R.ntp, R.nt, R.nt, R.nt));
        h3.push_back(gdesc(R.Wb, nullptr, R.ntp, R.L, nullptr, R.ntp, R.At, nullptr, R.nt, R.nt, R.nt, R.nt,
                           1.0, 1.0));
      }
      RSRS_TRY(gemm(up, st, h0, 0, 0, GM_FULL));
      RSRS_TRY(gemm(up, st, h1, 0, 1, GM_FULL));
      RSRS_TRY(gemm(up, st, h2, 0, 1, GM_B_NT_LOW));
      RSRS_TRY(gemm(up, st, h3, 0, 0, GM_B_NN_LOW));
    }
    std::vector<GjeDesc> gj;
    std::vector<SymDesc<double>> sa, sai;
    for (size_t q = 0; q < roots.size(); ++q) {
      const Root& R = roots[q];
      gj.push_back(GjeDesc{R.At, R.gw, R.Atinv, R.nt, R.nt, R.nt, 0});
      if (R.job->sym) {
        sa.push_back(SymDesc<double>{R.At, R.nt, R.nt, 0});
        sai.push_back(SymDesc<double>{R.Atinv, R.nt, R.nt, 0});
      }
    }
    RSRS_TRY(symmetrize<double>(up, st, sa));
    RSRS_TRY(gje_inverse(up, st, gj, flag));
    RSRS_TRY(symmetrize<double>(up, st, sai));
    if constexpr (mixed) {
      std::vector<Copy2DT<double, T>> cp;
      for (const Root& R : roots) {
        rsrs_factor_t* F = R.job->F.get();
        cp.push_back(Copy2DT<double, T>{R.At, R.job->dS + F->oAt, R.nt, R.nt, R.nt, R.nt, 1.0, 0, 0});
        cp.push_back(Copy2DT<double, T>{R.Atinv, R.job->dS + F->oAtinv, R.nt, R.nt, R.nt, R.nt, 1.0, 0, 0});
      }
      RSRS_TRY(copy2d<double, T>(up, st, cp));
    }
  }
  RSRS_TRY(up.reset());
  {
    int hflag = 0;
    RSRS_HIP(hipMemcpy(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost));
    if (hflag & 1) {
      set_error(deferred ? "Gram matrix of a test-matrix panel or of the root panel is not positive definite"
                         : "Gram matrix of the root panel is not positive definite");
      return RSRS_E_SINGULAR;
    }
    if (hflag & 2) { set_error("singular pivot block X_RR or root block"); return RSRS_E_SINGULAR; }
  }
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (auto& J : jobs) {
    J.F->flops = J.flops + J.flops_b;
    J.F->factor_ms = ms;
  }
  // every launch has completed: the scratch goes back to the pool for the
  // next factorization
  RSRS_HIP(hipStreamSynchronize(st2));
  RSRS_HIP(hipStreamSynchronize(st));
  pool_return(ws);
  pool_return(wsb[0]);
  pool_return(wsb[1]);
  pool_return(hpos);
  pool_return(hperm);
  side.recycle();
  up.recycle();
  up2.recycle();
  for (auto& J : jobs) pool_return(J.hidx);
  return RSRS_OK;
}

template <typename T>
rsrs_status factor_batch_t(int64_t nprob, const rsrs_tree_t* const* trees, rsrs_samples_t* const* smps,
                           const rsrs_factor_opts* opts, hipStream_t st, rsrs_factor_t** out,
                           const RedrawSpec* rd) {
  std::vector<Job<T>> jobs((size_t)nprob);
  for (int64_t i = 0; i < nprob; ++i) {
    jobs[i].rd = rd;
    const rsrs_status r = job_init<T>(jobs[i], trees[i], smps[i], &opts[i]);
    if (r != RSRS_OK) {
      if (nprob > 1) set_error("problem " + std::to_string(i) + ": " + rsrs_last_error());
      return r;
    }
  }
  // index lists on the device unless some problem's counts depend on its
  // data (rank tolerance): then every class reads its skeletons back
  bool deferred = true;
  for (const auto& J : jobs) deferred = deferred && !(J.rank_tol > 0.0);
  for (auto& J : jobs) {
    J.deferred = deferred;
    J.settle();
  }
  RSRS_TRY(factor_many<T>(jobs, st));
  for (int64_t i = 0; i < nprob; ++i) out[i] = jobs[i].F.release();
  return RSRS_OK;
}

}  // namespace

rsrs_status factor_batch_impl(int64_t nprob, const rsrs_tree_t* const* trees, rsrs_samples_t* const* smps,
                              const rsrs_factor_opts* opts, hipStream_t st, rsrs_factor_t** out,
                              const RedrawSpec* rd) {
  if (nprob < 1) { set_error("need at least one problem"); return RSRS_E_INVALID; }
  if (rd && nprob != 1) { set_error("the per-level redraw factors one problem"); return RSRS_E_INVALID; }
  for (int64_t i = 0; i < nprob; ++i) out[i] = nullptr;
  const int prec = opts[0].precision;
  for (int64_t i = 0; i < nprob; ++i) {
    const rsrs_factor_opts* o = &opts[i];
    const rsrs_samples_t* smp = smps[i];
    const std::string who = nprob > 1 ? "problem " + std::to_string(i) + ": " : std::string();
    if (!trees[i] || !smp) { set_error(who + "null tree or samples"); return RSRS_E_INVALID; }
    if (o->k < 1) { set_error(who + "k must be >= 1"); return RSRS_E_INVALID; }
    if (smp->consumed) { set_error(who + "samples were already consumed by a factorization"); return RSRS_E_INVALID; }
    if (smp->tree != trees[i]) { set_error(who + "samples belong to another tree"); return RSRS_E_INVALID; }
    if (o->k > 256) { set_error(who + "k > 256 is not supported"); return RSRS_E_UNSUPPORTED; }
    if (o->reproject < 0 || o->reproject > 1) { set_error(who + "reproject must be 0 or 1"); return RSRS_E_INVALID; }
    if (o->id_mode != RSRS_ID_SUM && o->id_mode != RSRS_ID_CONCAT) {
      set_error(who + "id_mode must be RSRS_ID_SUM or RSRS_ID_CONCAT");
      return RSRS_E_INVALID;
    }
    if (o->col_subset != 0 && o->col_subset != 1) {
      set_error(who + "col_subset must be 0 or 1");
      return RSRS_E_INVALID;
    }
    if (!(o->rank_tol >= 0.0) || !std::isfinite(o->rank_tol)) {
      set_error(who + "rank_tol must be finite and >= 0");
      return RSRS_E_INVALID;
    }
    if (o->precision != prec) { set_error(who + "all problems of a batch need the same precision"); return RSRS_E_INVALID; }
    for (int64_t j = 0; j < i; ++j)
      if (smps[j] == smp) { set_error(who + "the same samples appear twice"); return RSRS_E_INVALID; }
    if (smp->symmetric && !o->symmetric) {
      set_error(who + "symmetric samples need the symmetric variant (opts.symmetric = 1)");
      return RSRS_E_INVALID;
    }
    if (prec == RSRS_PREC_F64 && smp->dtype != RSRS_F64) {
      set_error(who + "FP64 factorization needs FP64 samples");
      return RSRS_E_INVALID;
    }
    if (prec == RSRS_PREC_F32_MIXED && smp->dtype != RSRS_F32) {
      set_error(who + "mixed-precision factorization needs FP32 samples");
      return RSRS_E_INVALID;
    }
  }
  if (prec == RSRS_PREC_F64) return factor_batch_t<double>(nprob, trees, smps, opts, st, out, rd);
  if (prec == RSRS_PREC_F32_MIXED) return factor_batch_t<float>(nprob, trees, smps, opts, st, out, rd);
  set_error("unknown precision");
  return RSRS_E_UNSUPPORTED;
}

rsrs_status factor_impl(const rsrs_tree_t* th, rsrs_samples_t* smp, const rsrs_factor_opts* o,
                        hipStream_t st, rsrs_factor_t** out, const RedrawSpec* rd) {
  return factor_batch_impl(1, &th, &smp, o, st, out, rd);
}

// Device bytes of a factorization of tree t with s samples: the stored factor
// (*stored) and the peak of everything alive while it is computed (samples
// excluded): stored factor, class workspace, descriptor staging.
size_t factor_bytes_estimate(const rsrs_tree_t* th, int k, int p, int64_t s, int precision,
                             size_t* stored, bool adaptive) {
  const Tree& t = th->t;
  const bool mixed = precision == RSRS_PREC_F32_MIXED;
  const int64_t esz = mixed ? 4 : 8, al = 16 / esz, sld = round_up(s, 16);
  (void)p;
  Schedule sch;
  make_schedule(t, k, sch);
  int64_t dsz = 0, isz = 0;
  size_t ws_max = 0, wsb_max = 0;
  for (size_t li = 0; li < sch.levels.size(); ++li)
    for (const auto& cls : sch.classes[li]) {
      size_t ws = 0, wsb = 0;
      for (int64_t b : cls) {
        const int64_t bb = sch.b_count[b], n = sch.l_count[b] - bb, r = adaptive ? bb : bb - k;
        dsz = round_up(dsz, al) + r * round_up(k, al);
        dsz = round_up(dsz, al) + 2 * r * round_up(r, al);
        dsz = round_up(dsz, al) + r * round_up(k + n, al);
        dsz = round_up(dsz, al) + (k + n) * round_up(r, al);
        isz += r + k + n + bb + n;
        size_t wa = 0, wb = 0;
        if (mixed) box_ws_bytes<float>(bb, bb + n, k, r, sld, &wa, &wb);
        else box_ws_bytes<double>(bb, bb + n, k, r, sld, &wa, &wb);
        ws += wa;
        wsb += wb;
      }
      ws_max = std::max(ws_max, ws);
      wsb_max = std::max(wsb_max, wsb);
    }
  const int64_t nt = sch.root_count;
  dsz = round_up(dsz, al) + 2 * nt * nt;
  isz += nt;
  size_t root_ws = (size_t)(4 * nt * round_up(nt, 16) + nt * sld + 2 * nt * nt) * 8 + 8 * 256;
  if (mixed) root_ws += (size_t)(2 * nt * sld + 2 * nt * nt) * 8 + 4 * 256;
  ws_max = std::max(ws_max, root_ws);
  const size_t st = (size_t)dsz * esz + (size_t)isz * 8 + (size_t)t.n * 8;
  if (stored) *stored = st;
  return st + ws_max + 2 * std::max<size_t>(wsb_max, 256) + ((size_t)128 << 20);
}

}  // namespace rsrs
