// Batched dense helpers: GEMM dispatch, Cholesky leaves, Gauss-Jordan inverse,
// copies, permutations and reductions (FP64).
#include <hip/hip_runtime.h>

#include <utility>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <unordered_map>
#include <cstdio>
#include <cstring>
#include <type_traits>

#include "kernels.hpp"
#include "profile.hpp"

namespace rsrs {

// ---------------------------------------------------------------- uploader
rsrs_status Uploader::init(size_t bytes, hipStream_t stream, bool pooled) {
  st = stream;
  off = 0;
  if (pooled) {
    RSRS_TRY(pool_alloc(h, bytes));
    RSRS_TRY(pool_alloc(d, bytes));
    return RSRS_OK;
  }
  RSRS_TRY(h.alloc(bytes));
  RSRS_TRY(d.alloc(bytes));
  return RSRS_OK;
}

void Uploader::recycle() {
  pool_return(h);
  pool_return(d);
  off = 0;
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
static thread_local const char* g_site = nullptr;

// Tag "gemm[32]_<form>_<mode>_<BM>x<BN>[:<site>]"; "gemm32" marks FP32 operands.
static const char* gemm_tag(bool f32, int ta, int tb, int mode, int bm, int bn) {
  static const char* forms[2][2] = {{"nn", "nt"}, {"tn", "tt"}};
  static const char* modes[5] = {"full", "syrk", "bntlow", "bnnlow", "alow"};
  static thread_local char buf[48];
  const char* g = f32 ? "gemm32" : "gemm";
  if (g_site)
    std::snprintf(buf, sizeof(buf), "%s_%s_%s_%dx%d:%s", g, forms[ta][tb], modes[mode], bm, bn, g_site);
  else
    std::snprintf(buf, sizeof(buf), "%s_%s_%s_%dx%d", g, forms[ta][tb], modes[mode], bm, bn);
  return buf;
}

// Algorithmic flops and bytes of one batched launch.
template <typename TI, typename TO>
static void gemm_work(const std::vector<GemmDescT<TI, TO>>& descs, int mode, double* flops,
                      double* bytes) {
  double f = 0.0, b = 0.0;
  for (const auto& d : descs) {
    if (d.M <= 0 || d.N <= 0) continue;
    const double M = d.M, N = d.N, K = d.K;
    double ff = 2.0 * M * N * K;
    if (mode == GM_SYRK_L) ff = M * (N + 1.0) * K;
    if (mode == GM_B_NT_LOW || mode == GM_B_NN_LOW || mode == GM_A_LOW) ff = M * N * K;
    f += ff;
    b += sizeof(TI) * (M * K + K * N) + sizeof(TO) * M * N * (d.beta != 0.0 ? 2.0 : 1.0);
  }
  *flops = f;
  *bytes = b;
}

// 16-byte loads need leading dimensions that are multiples of the vector
// width and 16-byte aligned bases.
template <typename TI, typename TO>
static bool vec_ok(const std::vector<GemmDescT<TI, TO>>& descs) {
  constexpr int64_t vw = 16 / sizeof(TI);
  for (const auto& d : descs) {
    if (d.M <= 0 || d.N <= 0) continue;
    if ((d.lda % vw) || (d.ldb % vw)) return false;
    if (((uintptr_t)d.A & 15) || ((uintptr_t)d.B & 15)) return false;
  }
  return true;
}

// Launch records of one batched product: the kernel instantiation, its grid
// and the range of descriptors it reads (grid.y <= 65535 per record).
template <typename TI, typename TO, int BM, int BN, int WM, int WN, int TA, int TB, int MODE>
static void plan_shape(const std::vector<GemmDescT<TI, TO>>& descs, size_t base,
                       std::vector<GemmLaunch>& out) {
  constexpr int VW = 16 / (int)sizeof(TI);
  constexpr int NT = 64 * WM * WN;
  constexpr bool can_vec = BN * 16 / NT >= VW && BM * 16 / NT >= VW;
  int64_t tiles = 0;
  for (const auto& d : descs)
    if (d.M > 0 && d.N > 0) {
      const int64_t tm = (d.M + BM - 1) / BM, tn = (d.N + BN - 1) / BN;
      tiles = std::max<int64_t>(tiles, MODE == GM_SYRK_L ? tm * (tm + 1) / 2 : tm * tn);
    }
  if (tiles == 0) return;
  double pf = 0.0, pb = 0.0;
  if (prof_on()) gemm_work(descs, MODE, &pf, &pb);
  const void* fn;
  if constexpr (can_vec) {
    fn = vec_ok(descs) ? reinterpret_cast<const void*>(&gemm_kernel<TI, TO, BM, BN, WM, WN, TA, TB, MODE, VW>)
                       : reinterpret_cast<const void*>(&gemm_kernel<TI, TO, BM, BN, WM, WN, TA, TB, MODE, 1>);
  } else {
    fn = reinterpret_cast<const void*>(&gemm_kernel<TI, TO, BM, BN, WM, WN, TA, TB, MODE, 1>);
  }
  for (size_t b0 = 0; b0 < descs.size(); b0 += 65535) {
    GemmLaunch L{};
    L.fn = fn;
    L.grid = dim3((unsigned)round_up(tiles, 8), (unsigned)std::min<size_t>(65535, descs.size() - b0));
    L.block = dim3(NT);
    L.first = base + b0;
    L.flops = b0 == 0 ? pf : 0.0;
    L.bytes = b0 == 0 ? pb : 0.0;
    std::snprintf(L.tag, sizeof(L.tag), "%s", gemm_tag(sizeof(TI) == 4, TA, TB, MODE, BM, BN));
    out.push_back(L);
  }
}

template <typename TI, typename TO, int BM, int BN, int WM, int WN>
static rsrs_status plan_forms(const std::vector<GemmDescT<TI, TO>>& descs, size_t base, int ta, int tb,
                              int mode, std::vector<GemmLaunch>& out) {
#define RSRS_G(TA, TB, MODE)                                                       \
  if (ta == TA && tb == TB && mode == MODE) {                                      \
    plan_shape<TI, TO, BM, BN, WM, WN, TA, TB, MODE>(descs, base, out);           \
    return RSRS_OK;                                                                \
  }
  if constexpr (std::is_same<TI, TO>::value) {
    RSRS_G(0, 0, GM_FULL)
    RSRS_G(0, 1, GM_FULL)
    RSRS_G(1, 0, GM_FULL)
    RSRS_G(1, 1, GM_FULL)
    RSRS_G(0, 1, GM_B_NT_LOW)
    RSRS_G(0, 0, GM_B_NN_LOW)
    RSRS_G(0, 0, GM_A_LOW)
  }
  RSRS_G(0, 1, GM_SYRK_L)
#undef RSRS_G
  set_error("unsupported GEMM form");
  return RSRS_E_UNSUPPORTED;
}

// ---------------------------------------------------------------- tile autotuner
// Candidate tile shapes of the automatic choice: 0 = 64 x 64 on 4 waves,
// 1 = 128 x 64 on 4 waves, 2 = 128 x 128 on 8 waves (each wave of the last
// two holds a 64 x 32 block).  The triangular SYRK form needs square tiles
// (0 or 2).  Every shape runs the same K slices (BK depends only on the
// element type for tiles at least 64 wide) in the same order, and masked
// slices add exact zeros, so the shape never changes a result bit.
//
// Launch classes: element type, form (TA, TB, mode), the launch's number of
// 64 x 64 output tiles (nearest of 4^1 .. 4^7 in log scale) and its
// contraction length (nearest of 128 and 1024 in log scale).  The table
// holds the measured fastest shape of each class; without a table the
// built-in rule applies (128 x 128 when the launch has >= 256 such tiles).
namespace {
constexpr int kTuneForms = 7;
constexpr int kTuneT = 7;   // 4^1 .. 4^7 tiles of 64 x 64
constexpr int kTuneK = 2;   // K = 128, 1024
constexpr int kTuneForm[kTuneForms][3] = {{0, 0, GM_FULL}, {0, 1, GM_FULL},     {1, 0, GM_FULL},
                                          {0, 1, GM_SYRK_L}, {0, 1, GM_B_NT_LOW}, {0, 0, GM_B_NN_LOW},
                                          {0, 0, GM_A_LOW}};
constexpr int kTuneKv[kTuneK] = {128, 1024};
std::atomic<int> g_tile_override{-1};
std::atomic<bool> g_tune_ready{false};
int8_t g_tune[2][kTuneForms][kTuneT][kTuneK];

int tune_form(int ta, int tb, int mode) {
  for (int f = 0; f < kTuneForms; ++f)
    if (kTuneForm[f][0] == ta && kTuneForm[f][1] == tb && kTuneForm[f][2] == mode) return f;
  return -1;
}
int tune_tbin(double t64) {
  const int b = (int)std::lround(std::log(std::max(t64, 1.0)) / std::log(4.0)) - 1;
  return std::min(kTuneT - 1, std::max(0, b));
}
int tune_kbin(int K) { return K >= 362 ? 1 : 0; }

// exact shape signatures of the workload tuning
std::mutex g_sig_mu;
std::unordered_map<uint64_t, int8_t> g_sig_table;
std::atomic<bool> g_sig_any{false};
std::atomic<bool> g_rec_on{false};
struct SigRec { uint64_t sig; int shape; hipEvent_t a, b; };
std::vector<SigRec> g_recs;

uint64_t fnv(uint64_t h, uint64_t v) {
  for (int i = 0; i < 8; ++i) {
    h ^= (v >> (8 * i)) & 0xff;
    h *= 1099511628211ull;
  }
  return h;
}
}  // namespace

template <typename TI, typename TO>
static uint64_t launch_sig(const std::vector<GemmDescT<TI, TO>>& descs, int ta, int tb, int mode) {
  uint64_t h = 1469598103934665603ull;
  h = fnv(h, sizeof(TI));
  h = fnv(h, (uint64_t)(ta * 64 + tb * 8 + mode));
  h = fnv(h, descs.size());
  for (const auto& d : descs) h = fnv(h, ((uint64_t)(uint32_t)d.M << 40) ^ ((uint64_t)(uint32_t)d.N << 20) ^ (uint32_t)d.K);
  return h;
}

template <typename TI, typename TO>
static int builtin_shape(const std::vector<GemmDescT<TI, TO>>& descs, int mode) {
  int64_t t128 = 0;
  for (const auto& d : descs) {
    if (d.M <= 0 || d.N <= 0) continue;
    const int64_t tm = (d.M + 127) / 128, tn = (d.N + 127) / 128;
    t128 += mode == GM_SYRK_L ? tm * (tm + 1) / 2 : tm * tn;
  }
  return t128 >= 256 ? 2 : 0;
}

template <typename TI, typename TO>
static int chosen_shape(const std::vector<GemmDescT<TI, TO>>& descs, int ta, int tb, int mode, uint64_t sig) {
  const int ov = g_tile_override.load(std::memory_order_relaxed);
  if (ov >= 0) return (mode == GM_SYRK_L && ov == 1) ? 0 : ov;
  if (g_sig_any.load(std::memory_order_acquire)) {
    std::lock_guard<std::mutex> lk(g_sig_mu);
    auto it = g_sig_table.find(sig);
    if (it != g_sig_table.end()) return it->second;
  }
  const int f = tune_form(ta, tb, mode);
  if (f >= 0 && g_tune_ready.load(std::memory_order_acquire)) {
    double t64 = 0.0;
    int kmax = 0;
    for (const auto& d : descs) {
      if (d.M <= 0 || d.N <= 0) continue;
      const double tm = (d.M + 63) / 64, tn = (d.N + 63) / 64;
      t64 += mode == GM_SYRK_L ? tm * (tm + 1) / 2 : tm * tn;
      kmax = std::max(kmax, d.K);
    }
    return g_tune[sizeof(TI) == 4 ? 1 : 0][f][tune_tbin(t64)][tune_kbin(kmax)];
  }
  return builtin_shape(descs, mode);
}

template <typename TI, typename TO>
static rsrs_status plan_with_shape(int shp, const std::vector<GemmDescT<TI, TO>>& descs, size_t base, int ta,
                                   int tb, int mode, std::vector<GemmLaunch>& out) {
  if (shp == 2) return plan_forms<TI, TO, 128, 128, 2, 4>(descs, base, ta, tb, mode, out);
  if (shp == 1 && mode != GM_SYRK_L) return plan_forms<TI, TO, 128, 64, 2, 2>(descs, base, ta, tb, mode, out);
  return plan_forms<TI, TO, 64, 64, 2, 2>(descs, base, ta, tb, mode, out);
}

// Tile choice: the autotuner's table when one was measured or loaded
// (rsrs_gemm_autotune), else the built-in rule measured on MI355X -- 128 x 128
// tiles on 8 waves reach 50+ TFLOP/s on the large FP64 products and are
// used whenever the batch still yields >= 256 such tiles, otherwise 64 x 64
// tiles on 4 waves keep the chip busy.  Narrow right-hand sides use 64 x 16.
template <typename TI, typename TO>
rsrs_status gemm_plan(const std::vector<GemmDescT<TI, TO>>& descs, size_t base, int ta, int tb, int mode,
                      GemmShape shape, const char* site, std::vector<GemmLaunch>& out) {
  if (descs.empty()) return RSRS_OK;
  struct SiteGuard {
    explicit SiteGuard(const char* s) { g_site = s; }
    ~SiteGuard() { g_site = nullptr; }
  } guard(site);
  if constexpr (std::is_same<TI, TO>::value) {
    if (shape == GS_64x16 && mode == GM_FULL) return plan_forms<TI, TO, 64, 16, 4, 1>(descs, base, ta, tb, mode, out);
  }
  if (shape == GS_64x64_ONLY) return plan_forms<TI, TO, 64, 64, 2, 2>(descs, base, ta, tb, mode, out);
  const uint64_t sig = launch_sig(descs, ta, tb, mode);
  const size_t first = out.size();
  const int shp = chosen_shape(descs, ta, tb, mode, sig);
  RSRS_TRY((plan_with_shape<TI, TO>(shp, descs, base, ta, tb, mode, out)));
  for (size_t i = first; i < out.size(); ++i) {
    out[i].sig = sig;
    out[i].shape = (mode == GM_SYRK_L && shp == 1) ? 0 : shp;
  }
  return RSRS_OK;
}

// Times shape `shp` on the synthetic launch `descs` (device copy at dd):
// the best of three launches after one warm-up, in milliseconds.
template <typename T>
static rsrs_status time_shape(int shp, const std::vector<GemmDescT<T, T>>& descs, const GemmDescT<T, T>* dd,
                              int ta, int tb, int mode, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                              float* best) {
  std::vector<GemmLaunch> L;
  RSRS_TRY(plan_with_shape<T, T>(shp, descs, 0, ta, tb, mode, L));
  *best = 1e30f;
  for (int rep = 0; rep < 4; ++rep) {
    RSRS_HIP(hipEventRecord(e0, st));
    for (const auto& x : L) {
      const void* p = dd + x.first;
      void* args[] = {&p};
      RSRS_HIP(hipLaunchKernel(x.fn, x.grid, x.block, args, 0, st));
    }
    RSRS_HIP(hipEventRecord(e1, st));
    RSRS_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    RSRS_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (rep > 0) *best = std::min(*best, ms);
  }
  return RSRS_OK;
}

// One class: nb products of D x D with contraction K, each with its own
// operands and output (tile count t64 = nb (D / 64)^2, or the lower
// triangle's for SYRK), every candidate shape timed.
template <typename T>
static rsrs_status tune_type(int* changed, hipStream_t st, hipEvent_t e0, hipEvent_t e1, DevBuf& bufA,
                             DevBuf& bufB, DevBuf& bufC, DevBuf& bufD) {
  constexpr int ti = sizeof(T) == 4 ? 1 : 0;
  for (int f = 0; f < kTuneForms; ++f) {
    const int ta = kTuneForm[f][0], tb = kTuneForm[f][1], mode = kTuneForm[f][2];
    for (int tt = 0; tt < kTuneT; ++tt) {
      const int64_t t64 = (int64_t)1 << (2 * (tt + 1));
      const int64_t per = std::min<int64_t>(t64, 64);
      const int D = (int)std::lround(64.0 * std::sqrt((double)per));
      const int64_t nb = t64 / per;
      for (int kk = 0; kk < kTuneK; ++kk) {
        const int K = kTuneKv[kk];
        std::vector<GemmDescT<T, T>> descs;
        for (int64_t q = 0; q < nb; ++q) {
          T* A = bufA.as<T>() + q * (int64_t)D * K;
          T* B = bufB.as<T>() + q * (int64_t)D * K;
          T* C = bufC.as<T>() + q * (int64_t)D * D;
          // A: M x K (TA = 0) or K x M (TA = 1); B: N x K (TB = 1) or K x N (TB = 0)
          descs.push_back(gdescT<T, T>(A, nullptr, ta ? D : K, B, nullptr, tb ? K : D, C, nullptr, D, D, D, K));
        }
        GemmDescT<T, T>* dd = reinterpret_cast<GemmDescT<T, T>*>(bufD.p);
        RSRS_HIP(hipMemcpyAsync(dd, descs.data(), descs.size() * sizeof(descs[0]), hipMemcpyHostToDevice, st));
        const int def = builtin_shape(descs, mode);
        int win = -1;
        float wbest = 1e30f;
        for (int shp = 0; shp < 3; ++shp) {
          if (mode == GM_SYRK_L && shp == 1) continue;
          float ms = 0.0f;
          RSRS_TRY(time_shape<T>(shp, descs, dd, ta, tb, mode, st, e0, e1, &ms));
          // a challenger must beat the built-in choice by 3% to replace it
          const float bar = (win == def || shp == def) ? 0.97f : 1.0f;
          if (win < 0 || (shp == def ? ms < wbest / bar : ms < wbest * bar)) {
            win = shp;
            wbest = ms;
          }
        }
        g_tune[ti][f][tt][kk] = (int8_t)win;
        if (win != def) ++*changed;
      }
    }
  }
  return RSRS_OK;
}

static bool tune_load(const char* path) {
  FILE* fp = path ? std::fopen(path, "r") : nullptr;
  if (!fp) return false;
  int8_t tab[2][kTuneForms][kTuneT][kTuneK];
  int seen = 0;
  char line[128];
  while (std::fgets(line, sizeof(line), fp)) {
    int a, b, c, d, e;
    if (line[0] == '#') continue;
    if (std::sscanf(line, "%d %d %d %d %d", &a, &b, &c, &d, &e) != 5 || a < 0 || a > 1 || b < 0 ||
        b >= kTuneForms || c < 0 || c >= kTuneT || d < 0 || d >= kTuneK || e < 0 || e > 2 ||
        (kTuneForm[b][2] == GM_SYRK_L && e == 1)) {
      std::fclose(fp);
      return false;
    }
    tab[a][b][c][d] = (int8_t)e;
    ++seen;
  }
  std::fclose(fp);
  if (seen != 2 * kTuneForms * kTuneT * kTuneK) return false;
  std::memcpy(g_tune, tab, sizeof(tab));
  return true;
}

static void tune_save(const char* path) {
  FILE* fp = std::fopen(path, "w");
  if (!fp) return;
  std::fprintf(fp, "# GEMM tile table: fp32 form tiles(4^(i+1)) K(128|1024) shape(0 64x64, 1 128x64, 2 128x128)\n");
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < kTuneForms; ++b)
      for (int c = 0; c < kTuneT; ++c)
        for (int d = 0; d < kTuneK; ++d) std::fprintf(fp, "%d %d %d %d %d\n", a, b, c, d, (int)g_tune[a][b][c][d]);
  std::fclose(fp);
}

rsrs_status gemm_autotune(const char* cache_path, int64_t* entries, int64_t* changed) {
  constexpr int64_t total = 2 * kTuneForms * kTuneT * kTuneK;
  if (entries) *entries = total;
  if (changed) *changed = 0;
  auto count_changed = [&]() {
    // against the built-in rule on the same synthetic classes
    int64_t c = 0;
    for (int a = 0; a < 2; ++a)
      for (int f = 0; f < kTuneForms; ++f)
        for (int tt = 0; tt < kTuneT; ++tt)
          for (int kk = 0; kk < kTuneK; ++kk) {
            const int64_t t64 = (int64_t)1 << (2 * (tt + 1));
            const int64_t per = std::min<int64_t>(t64, 64);
            const int64_t D = std::lround(64.0 * std::sqrt((double)per)), nb = t64 / per;
            const int64_t tm = (D + 127) / 128;
            const int64_t t128 = nb * (kTuneForm[f][2] == GM_SYRK_L ? tm * (tm + 1) / 2 : tm * tm);
            c += g_tune[a][f][tt][kk] != (t128 >= 256 ? 2 : 0);
          }
    return c;
  };
  if (tune_load(cache_path)) {
    g_tune_ready.store(true, std::memory_order_release);
    if (changed) *changed = count_changed();
    return RSRS_OK;
  }
  g_tune_ready.store(false, std::memory_order_release);
  // largest class: 256 products of 512 x 512 with K = 1024
  const size_t opnd = (size_t)256 * 512 * 1024 * 8, outb = (size_t)256 * 512 * 512 * 8;
  DevBuf A, B, Cb, Dd;
  RSRS_TRY(A.alloc(opnd));
  RSRS_TRY(B.alloc(opnd));
  RSRS_TRY(Cb.alloc(outb));
  RSRS_TRY(Dd.alloc((size_t)256 * sizeof(GemmDescT<double, double>)));
  hipStream_t st = nullptr;
  RSRS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rsrs_status rs = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess ? RSRS_OK : RSRS_E_HIP;
  // operands: small values, so that no product overflows or goes subnormal
  if (rs == RSRS_OK && (hipMemsetAsync(A.p, 0x3c, opnd, st) != hipSuccess ||
                        hipMemsetAsync(B.p, 0x3c, opnd, st) != hipSuccess))
    rs = RSRS_E_HIP;
  int ch = 0;
  if (rs == RSRS_OK) rs = tune_type<float>(&ch, st, e0, e1, A, B, Cb, Dd);
  if (rs == RSRS_OK) rs = tune_type<double>(&ch, st, e0, e1, A, B, Cb, Dd);
  if (rs == RSRS_OK && hipStreamSynchronize(st) != hipSuccess) rs = RSRS_E_HIP;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(st);
  if (rs != RSRS_OK) {
    if (rs == RSRS_E_HIP) set_error("GEMM autotuning: HIP call failed");
    return rs;
  }
  g_tune_ready.store(true, std::memory_order_release);
  if (changed) *changed = ch;
  if (cache_path) tune_save(cache_path);
  return RSRS_OK;
}

rsrs_status gemm_tile_override(int shape) {
  if (shape < -2 || shape > 2) {
    set_error("tile shape must be -2 (built-in rule), -1 (table or rule), 0, 1 or 2");
    return RSRS_E_INVALID;
  }
  if (shape == -2) {
    g_tune_ready.store(false, std::memory_order_release);
    gemm_sig_install({}, true);
    shape = -1;
  }
  g_tile_override.store(shape, std::memory_order_relaxed);
  return RSRS_OK;
}

rsrs_status gemm_exec(const GemmLaunch& L, const void* descs, size_t desc_bytes, hipStream_t st) {
  const void* p = static_cast<const char*>(descs) + L.first * desc_bytes;
  void* args[] = {&p};
  ProfScope ps(st, L.tag, L.flops, L.bytes);
  if (L.sig != 0 && g_rec_on.load(std::memory_order_relaxed)) {
    SigRec r{L.sig, L.shape, nullptr, nullptr};
    RSRS_HIP(hipEventCreate(&r.a));
    RSRS_HIP(hipEventCreate(&r.b));
    RSRS_HIP(hipEventRecord(r.a, st));
    RSRS_HIP(hipLaunchKernel(L.fn, L.grid, L.block, args, 0, st));
    RSRS_HIP(hipEventRecord(r.b, st));
    std::lock_guard<std::mutex> lk(g_sig_mu);
    g_recs.push_back(r);
    return RSRS_OK;
  }
  RSRS_HIP(hipLaunchKernel(L.fn, L.grid, L.block, args, 0, st));
  return RSRS_OK;
}

void gemm_sig_record(bool on) { g_rec_on.store(on, std::memory_order_relaxed); }

rsrs_status gemm_sig_collect(std::vector<std::pair<uint64_t, double>>& ms,
                             std::vector<std::pair<uint64_t, int>>& shape) {
  std::vector<SigRec> recs;
  {
    std::lock_guard<std::mutex> lk(g_sig_mu);
    recs.swap(g_recs);
  }
  std::unordered_map<uint64_t, double> sum;
  std::unordered_map<uint64_t, int> shp;
  rsrs_status rs = RSRS_OK;
  for (auto& r : recs) {
    float t = 0.0f;
    if (rs == RSRS_OK && (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess))
      rs = RSRS_E_HIP;
    sum[r.sig] += t;
    shp[r.sig] = r.shape;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  if (rs != RSRS_OK) {
    set_error("GEMM tuning: event timing failed");
    return rs;
  }
  ms.assign(sum.begin(), sum.end());
  shape.assign(shp.begin(), shp.end());
  return RSRS_OK;
}

void gemm_sig_install(const std::vector<std::pair<uint64_t, int>>& table, bool replace) {
  std::lock_guard<std::mutex> lk(g_sig_mu);
  if (replace) g_sig_table.clear();
  for (const auto& x : table) g_sig_table[x.first] = (int8_t)x.second;
  g_sig_any.store(!g_sig_table.empty(), std::memory_order_release);
}

int64_t gemm_sig_count() {
  std::lock_guard<std::mutex> lk(g_sig_mu);
  return (int64_t)g_sig_table.size();
}

template <typename TI, typename TO>
rsrs_status gemm(Uploader& up, hipStream_t st, const std::vector<GemmDescT<TI, TO>>& descs, int ta, int tb,
                 int mode, GemmShape shape, const char* site) {
  if (descs.empty()) return RSRS_OK;
  std::vector<GemmLaunch> L;
  RSRS_TRY(gemm_plan<TI, TO>(descs, 0, ta, tb, mode, shape, site, L));
  if (L.empty()) return RSRS_OK;
  GemmDescT<TI, TO>* dd = nullptr;
  RSRS_TRY(up.put_vec(descs, &dd));
  for (const auto& x : L) RSRS_TRY(gemm_exec(x, dd, sizeof(GemmDescT<TI, TO>), st));
  return RSRS_OK;
}

template rsrs_status gemm_plan<double, double>(const std::vector<GemmDescT<double, double>>&, size_t, int, int,
                                               int, GemmShape, const char*, std::vector<GemmLaunch>&);
template rsrs_status gemm_plan<float, float>(const std::vector<GemmDescT<float, float>>&, size_t, int, int, int,
                                             GemmShape, const char*, std::vector<GemmLaunch>&);
template rsrs_status gemm<double, double>(Uploader&, hipStream_t, const std::vector<GemmDescT<double, double>>&,
                                          int, int, int, GemmShape, const char*);
template rsrs_status gemm<float, float>(Uploader&, hipStream_t, const std::vector<GemmDescT<float, float>>&,
                                        int, int, int, GemmShape, const char*);


// ---------------------------------------------------------------- Gauss-Jordan
// Gauss-Jordan inversion with partial pivoting, blocked by 16-column panels,
// one workgroup of 8 waves per matrix of order n <= 16 NT (NT = 4, 8, 12),
// padded with the identity to NP = 16 NT.  The matrix lives in registers as
// NT x NT tiles of 16 x 16 in the accumulator layout of the FP64 MFMA
// (register v of lane l holds tile row 4 v + l/16, column l%16): wave w
// holds the TR x TC tiles of tile rows TR (w / 2) .. and tile columns
// TC (w % 2) .., TR = NT / 4, TC = NT / 2.  Pivoting is implicit (rows are
// never swapped): the pivot of column j is the largest |a_ij| over the rows
// not used yet, lowest index on ties.
//
// Per panel J (columns 16 jt .. 16 jt + 15):
//  1. the panel tiles go to LDS;
//  2. one wave runs the 16 in-place Gauss-Jordan steps on the NP x 16 panel
//     (pivot search, every other row reduced by the pivot row, the pivot row
//     scaled, column j replaced by the inverse's column), recording the
//     pivot rows P;
//  3. every other column c takes the panel's 16 steps at once: the steps
//     read column c only in the rows P, so x_c <- x_c + W x_c[P] with
//     W = (factored panel) - E_P, E_P holding a 1 at (p_t, t); the waves
//     holding rows P stage them in LDS and every tile gets W[rows] x_c[P]
//     by four MFMAs (K = 16);
//  4. the panel tiles take the factored panel back.
// The pivots are those of the unblocked elimination (the panel steps see
// up-to-date panel columns).  With pivot rows p_j the working matrix ends as
// A^{-1}[i][c] = W[p_i][q_c], q the inverse permutation, applied on
// write-out.  The identity padding never takes part: real columns pivot on
// real rows (padded rows hold zeros there), padded columns on their own row.
// Cross-lane moves of FP64 values by DPP (two 32-bit halves).  Lanes whose
// source is outside the pattern keep `old`.
template <int CTRL, int RMASK = 0xF>
__device__ __forceinline__ double dpp_f64(double old, double x) {
  const long long o = __double_as_longlong(old), v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)v, CTRL, RMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(v >> 32), CTRL, RMASK, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Maximum over the 64 lanes (quad swaps, row half-mirror and mirror, then
// the row broadcasts 15 and 31), read from lane 63 into every lane.
__device__ __forceinline__ double wave_max_dpp(double v) {
  v = fmax(v, dpp_f64<0xB1>(v, v));         // quad_perm [1, 0, 3, 2]
  v = fmax(v, dpp_f64<0x4E>(v, v));         // quad_perm [2, 3, 0, 1]
  v = fmax(v, dpp_f64<0x141>(v, v));        // row_half_mirror
  v = fmax(v, dpp_f64<0x140>(v, v));        // row_mirror
  v = fmax(v, dpp_f64<0x142, 0xA>(v, v));   // row_bcast:15
  v = fmax(v, dpp_f64<0x143, 0xC>(v, v));   // row_bcast:31
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Every lane of a quad takes lane S of its quad (quad_perm [S, S, S, S]).
template <int S>
__device__ __forceinline__ double quad_bcast_dpp(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)v, S * 0x55, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), S * 0x55, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// The same with the source lane chosen at run time (folded when it is known).
__device__ __forceinline__ double quad_bcast_dpp_rt(double x, int s) {
  switch (s) {
    case 0: return quad_bcast_dpp<0>(x);
    case 1: return quad_bcast_dpp<1>(x);
    case 2: return quad_bcast_dpp<2>(x);
    default: return quad_bcast_dpp<3>(x);
  }
}

// The 16 Gauss-Jordan steps of one panel (columns 16 jt .. 16 jt + 15 of the
// working matrix, or fewer: nsteps), run by waves 0..3 of the calling
// workgroup (pw) on rows held in registers: wave w holds the rows
// RL 16 w .. RL 16 w + RL 16 - 1, lane l the RL consecutive rows
// row0 = RL (16 w + (l >> 2)) .. + RL - 1 in the panel columns 4 (l & 3) ..
// + 3, so a lower lane holds lower rows.  Per step each wave offers its best
// free row (value, index, the reciprocal of its pivot entry and the row
// itself) in an LDS slot (two sets of four, by step parity), one barrier,
// and every wave takes the same pivot from the four offers (largest value,
// lowest row on ties); every other row is reduced by the pivot row, the
// pivot row scaled, and column t replaced by the inverse's column (the
// in-place form of the elimination).  Cross-lane moves are DPP.  Every
// thread of the workgroup calls this (the barriers); on_pivot(t, p, |pivot|)
// runs in lane 0 of wave 0 after each step.  Rows >= nrows hold zeros and
// count as used.
template <int RL, int t, class OnPivot>
__device__ __forceinline__ void gj_panel_step(double (&rv)[RL][4], unsigned& used_mask, int row0, int wave,
                                              int lane, bool pw, int nrows, double* OFF, OnPivot& on_pivot) {
  const int cq = lane & 3;
  const int NONE = 1 << 30;
  {
    double* slot = OFF + (t & 1) * (4 * 20);
    if (pw) {
      // best free row of this wave in column t (lowest row on ties)
      double best = -1.0, rcp = 0.0;
      int bi = NONE;
#pragma unroll
      for (int i = 0; i < RL; ++i) {
        const double x = rv[i][t & 3];
        const double v = fabs(x);
        const bool take = !((used_mask >> i) & 1u) && row0 + i < nrows && (bi == NONE || v > best);
        best = take ? v : best;
        bi = take ? row0 + i : bi;
        rcp = take ? x : rcp;
      }
      // the reciprocal of this lane's candidate, in the shadow of the reduction
      rcp = rcp != 0.0 ? 1.0 / rcp : 0.0;
      if (cq != (t >> 2)) { best = -1.0; bi = NONE; }   // only the quad lanes holding column t
      const double m = wave_max_dpp(best);
      const unsigned long long hold = __ballot(bi != NONE && best == m);
      const int cand = hold ? __builtin_amdgcn_readlane(bi, (int)__ffsll((long long)hold) - 1) : NONE;
      // the four lanes holding row cand publish it
      const int rel = cand - row0;
      if (cand != NONE && rel >= 0 && rel < RL) {
        // row rel of this lane, picked by bit masks (a select chain over
        // rv would be turned into an indexed load and push rv to memory)
        double x[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          unsigned long long y = 0;
#pragma unroll
          for (int ii = 0; ii < RL; ++ii) {
            const unsigned long long mask = 0ull - (unsigned long long)(rel == ii);
            y |= (unsigned long long)__double_as_longlong(rv[ii][c]) & mask;
          }
          x[c] = __longlong_as_double((long long)y);
        }
        double* dst = slot + wave * 20 + 4 + 4 * cq;
        *reinterpret_cast<double2*>(dst) = make_double2(x[0], x[1]);
        *reinterpret_cast<double2*>(dst + 2) = make_double2(x[2], x[3]);
      }
      if (lane == 0) {
        slot[wave * 20 + 0] = m;
        reinterpret_cast<int*>(slot + wave * 20 + 1)[0] = cand;
      }
      if (cand != NONE && cand == bi && cq == (t >> 2)) slot[wave * 20 + 2] = rcp;
    }
    __syncthreads();
    if (pw) {
      // the same choice in every wave: largest offer, lowest row on ties
      double bv = -1.0;
      int brow = NONE, bw = 0;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const double2 h = *reinterpret_cast<const double2*>(slot + w * 20);
        const int r = (int)__double_as_longlong(h.y);   // the row index sits in the low word
        const bool take = r != NONE && (brow == NONE || h.x > bv || (h.x == bv && r < brow));
        bv = take ? h.x : bv;
        brow = take ? r : brow;
        bw = take ? w : bw;
      }
      const int p = __builtin_amdgcn_readfirstlane(brow);   // a free row always exists
      bw = __builtin_amdgcn_readfirstlane(bw);
      const double* win = slot + bw * 20;
      const double inv = win[2];
      const double2 y0 = *reinterpret_cast<const double2*>(win + 4 + 4 * cq);
      const double2 y1 = *reinterpret_cast<const double2*>(win + 6 + 4 * cq);
      const double pr[4] = {y0.x, y0.y, y1.x, y1.y};
      const bool colq = cq == (t >> 2);   // this lane holds column t
#pragma unroll
      for (int i = 0; i < RL; ++i) {
        // column t of this row, from the quad lane that holds it
        const double ct = quad_bcast_dpp_rt(rv[i][t & 3], t >> 2) * inv;
#pragma unroll
        for (int c = 0; c < 4; ++c) rv[i][c] = (colq && c == (t & 3)) ? -ct : rv[i][c] - ct * pr[c];
      }
      // the pivot row: scaled by the pivot, its column t the reciprocal
      // (selects, not stores under a branch: those would be merged into one
      // store at a computed index and push rv out of registers)
      const int rp = p - row0;
#pragma unroll
      for (int i = 0; i < RL; ++i) {
        const bool mine = rp == i;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double sc = (colq && c == (t & 3)) ? inv : pr[c] * inv;
          rv[i][c] = mine ? sc : rv[i][c];
        }
        used_mask |= mine ? (1u << i) : 0u;
      }
      if (wave == 0 && lane == 0) on_pivot(t, p, bv);
    }
  
  }
}

template <int RL, class OnPivot, int... T>
__device__ __forceinline__ void gj_panel_all(double (&rv)[RL][4], unsigned& used_mask, int row0, int wave,
                                             int lane, bool pw, int nsteps, int nrows, double* OFF,
                                             OnPivot& on_pivot, std::integer_sequence<int, T...>) {
  // one step per column, its index a constant (register indices stay static);
  // nsteps is uniform, so every thread reaches the same barriers
  ((T < nsteps ? gj_panel_step<RL, T>(rv, used_mask, row0, wave, lane, pw, nrows, OFF, on_pivot) : void()), ...);
}

template <int RL, class OnPivot>
__device__ __forceinline__ void gj_panel_steps(double (&rv)[RL][4], unsigned& used_mask, int row0, int wave,
                                               int lane, bool pw, int nsteps, int nrows, double* OFF,
                                               OnPivot&& on_pivot) {
  gj_panel_all<RL>(rv, used_mask, row0, wave, lane, pw, nsteps, nrows, OFF, on_pivot,
                   std::make_integer_sequence<int, 16>{});
}

template <int NT>
__global__ __launch_bounds__(512) void gje_blk_kernel(const GjeDesc* __restrict__ e, int* flag) {
  constexpr int NP = 16 * NT;
  constexpr int TR = NT / 4, TC = NT / 2;  // tile rows / columns per wave
  constexpr int RW = NP / 4;               // panel rows per factoring wave
  constexpr int PBS = 18;                  // row stride of the panel buffer (doubles, 16-byte rows)
  constexpr int PRS = NP + 2;              // row stride of the pivot-row buffer
  static_assert(NT % 4 == 0, "NT is a multiple of 4");
  const GjeDesc d = e[blockIdx.x];
  const gptr<const double> gA = to_global(d.A);
  const int n = d.n;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int tr0 = TR * (wave >> 1), tc0 = TC * (wave & 1);   // first tile row / column
  const int q = lane >> 4, c16 = lane & 15;
  __shared__ __align__(16) double PB[NP * PBS];
  __shared__ __align__(16) double PR[16 * PRS];
  __shared__ __align__(16) double OFF[2 * 4 * 20];   // per step parity and wave: value, row, pad, the row
  __shared__ int piv[NP];
  __shared__ int qinv[NP];
  __shared__ int usedf[NP];
  __shared__ int bad;

  v4d acc[TR][TC];
#pragma unroll
  for (int a = 0; a < TR; ++a)
#pragma unroll
    for (int b = 0; b < TC; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * (tr0 + a) + 4 * v + q, col = 16 * (tc0 + b) + c16;
        // every load in bounds and unconditional (all in flight together),
        // the padding then selected in registers
        const double x = gA[(int64_t)min(row, n - 1) * d.lda + min(col, n - 1)];
        acc[a][b][v] = (row < n && col < n) ? x : (row == col ? 1.0 : 0.0);
      }
  for (int i = tid; i < NP; i += 512) {
    usedf[i] = 0;
    qinv[i] = NP;
  }
  if (tid == 0) bad = 0;

  for (int jt = 0; jt < NT; ++jt) {
    __syncthreads();   // the previous panel's readers of PB / PR are done
#pragma unroll
    for (int b = 0; b < TC; ++b)
      if (tc0 + b == jt) {
#pragma unroll
        for (int a = 0; a < TR; ++a)
#pragma unroll
          for (int v = 0; v < 4; ++v) PB[(16 * (tr0 + a) + 4 * v + q) * PBS + c16] = acc[a][b][v];
      }
    __syncthreads();
    {
      constexpr int RL = RW / 16;
      const bool pw = wave < 4;
      const int rg = lane >> 2, cq = lane & 3;
      const int row0 = RW * wave + RL * rg;
      double rv[RL][4];
      unsigned used_mask = 0;   // bit i: row row0 + i already pivoted
      if (pw) {
#pragma unroll
        for (int i = 0; i < RL; ++i) {
          const double* src = PB + (row0 + i) * PBS + 4 * cq;
          const double2 x0 = *reinterpret_cast<const double2*>(src);
          const double2 x1 = *reinterpret_cast<const double2*>(src + 2);
          rv[i][0] = x0.x; rv[i][1] = x0.y; rv[i][2] = x1.x; rv[i][3] = x1.y;
          used_mask |= usedf[row0 + i] ? (1u << i) : 0u;
        }
      }
      gj_panel_steps<RL>(rv, used_mask, row0, wave, lane, pw, 16, NP, OFF, [jt](int t, int p, double bv) {
        if (!(bv > 0.0)) bad = 1;
        usedf[p] = 1;
        piv[16 * jt + t] = p;
        qinv[p] = 16 * jt + t;
      });
      if (pw) {
#pragma unroll
        for (int i = 0; i < RL; ++i) {
          double* dst = PB + (row0 + i) * PBS + 4 * cq;
          *reinterpret_cast<double2*>(dst) = make_double2(rv[i][0], rv[i][1]);
          *reinterpret_cast<double2*>(dst + 2) = make_double2(rv[i][2], rv[i][3]);
        }
      }
    }
    __syncthreads();
    // old values of the pivot rows in every column outside the panel, staged
    // by the lanes holding them: qinv[row] is the elimination step of a row
    // already pivoted, NP for the others
#pragma unroll
    for (int a = 0; a < TR; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int t = qinv[16 * (tr0 + a) + 4 * v + q] - 16 * jt;
        if (t < 0 || t >= 16) continue;
#pragma unroll
        for (int b = 0; b < TC; ++b)
          if (tc0 + b != jt) PR[t * PRS + 16 * (tc0 + b) + c16] = acc[a][b][v];
      }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < TR; ++a) {
      const int row = 16 * (tr0 + a) + c16;
      double wa[4];
      const int trow = qinv[row] - 16 * jt;   // W = panel - E_P
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const int kk = 4 * kc + q;
        wa[kc] = PB[row * PBS + kk] - (trow == kk ? 1.0 : 0.0);
      }
#pragma unroll
      for (int b = 0; b < TC; ++b) {
        if (tc0 + b == jt) {
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[a][b][v] = PB[(16 * (tr0 + a) + 4 * v + q) * PBS + c16];
        } else {
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) {
            const double x = PR[(4 * kc + q) * PRS + 16 * (tc0 + b) + c16];
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[kc], x, acc[a][b], 0, 0, 0);
          }
        }
      }
    }
  }
  __syncthreads();
  if (tid == 0 && bad) atomicOr(flag, 2);
#pragma unroll
  for (int a = 0; a < TR; ++a)
#pragma unroll
    for (int b = 0; b < TC; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * (tr0 + a) + 4 * v + q, col = 16 * (tc0 + b) + c16;
        if (row < n && col < n) to_global(d.Ainv)[(int64_t)qinv[row] * d.ldi + piv[col]] = acc[a][b][v];
      }
}

// Larger blocks (192 < n <= 1024): the same panel elimination, in global
// memory, two launches per 16-column panel.  The working matrix X (n x n,
// leading dimension n) is the first n^2 doubles of the workspace W, followed
// by pos[n] (the elimination step of a pivoted row, n for a free one),
// piv[n] (the pivot row of each step) and XP (16 x n: the old pivot rows of
// the current panel).  The panel launch (one workgroup of four waves per
// matrix, the panel's rows in registers, RL = NP / 64 rows per lane)
// factors the panel with gj_panel_steps, writes it back and stages the old
// pivot rows outside the panel; the update launch (64 x 64 tiles, FP64
// MFMA) adds W XP to every other column, W = (factored panel) - E_P.
struct GjeBig {
  double* X;
  int* pos;
  int* piv;
  double* XP;
};
__device__ __forceinline__ GjeBig gje_big_parts(const GjeDesc& d) {
  GjeBig g;
  const int64_t nn = (int64_t)d.n * d.n;
  g.X = d.W;
  g.pos = reinterpret_cast<int*>(d.W + nn);
  g.piv = g.pos + d.n;
  g.XP = d.W + nn + d.n;   // after 2n ints
  return g;
}

__global__ __launch_bounds__(256) void gje_big_init_kernel(const GjeDesc* __restrict__ e) {
  const GjeDesc d = e[blockIdx.y];
  const int n = d.n;
  const GjeBig g = gje_big_parts(d);
  for (int r = blockIdx.x; r < n; r += gridDim.x) {
    for (int c = threadIdx.x; c < n; c += 256) g.X[(int64_t)r * n + c] = d.A[(int64_t)r * d.lda + c];
    if (threadIdx.x == 0) g.pos[r] = n;
  }
}

template <int RL>
__global__ __launch_bounds__(256) void gje_big_panel_kernel(const GjeDesc* __restrict__ e, int jt, int* flag) {
  const GjeDesc d = e[blockIdx.x];
  const int n = d.n;
  const int c0 = 16 * jt;
  if (c0 >= n) return;   // uniform: this matrix has no panel jt
  const GjeBig g = gje_big_parts(d);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rg = lane >> 2, cq = lane & 3;
  const int row0 = RL * (16 * wave + rg);
  const int ncols = min(16, n - c0);
  __shared__ __align__(16) double OFF[2 * 4 * 20];
  __shared__ int pnl[16];
  double rv[RL][4];
  unsigned used_mask = 0;
#pragma unroll
  for (int i = 0; i < RL; ++i) {
    const int row = row0 + i;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int col = 4 * cq + c;
      rv[i][c] = (row < n && col < ncols) ? g.X[(int64_t)row * n + c0 + col] : 0.0;
    }
    used_mask |= (row >= n || g.pos[row] < n) ? (1u << i) : 0u;
  }
  int* pos = g.pos;
  int* piv = g.piv;
  gj_panel_steps<RL>(rv, used_mask, row0, wave, lane, true, ncols, n, OFF,
                     [=](int t, int p, double bv) {
                       if (!(bv > 0.0)) atomicOr(flag, 2);
                       pos[p] = c0 + t;
                       piv[c0 + t] = p;
                       pnl[t] = p;
                     });
#pragma unroll
  for (int i = 0; i < RL; ++i) {
    const int row = row0 + i;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int col = 4 * cq + c;
      if (row < n && col < ncols) g.X[(int64_t)row * n + c0 + col] = rv[i][c];
    }
  }
  __syncthreads();
  // old pivot rows outside the panel (this launch writes only panel columns)
  for (int t = 0; t < ncols; ++t) {
    const double* src = g.X + (int64_t)pnl[t] * n;
    for (int c = tid; c < n; c += 256)
      if (c < c0 || c >= c0 + 16) g.XP[(int64_t)t * n + c] = src[c];
  }
}

__global__ __launch_bounds__(256) void gje_big_update_kernel(const GjeDesc* __restrict__ e, int jt) {
  const GjeDesc d = e[blockIdx.z];
  const int n = d.n;
  const int c0 = 16 * jt;
  const int r0 = 64 * blockIdx.y, cb = 64 * blockIdx.x;
  if (c0 >= n || r0 >= n || cb >= n) return;
  const GjeBig g = gje_big_parts(d);
  const int ncols = min(16, n - c0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, c16 = lane & 15;
  const int arow = r0 + 16 * wave + c16;   // row of this lane's A operand
  double a[4];
  const int ap = arow < n ? g.pos[arow] : n;
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    const int kk = 4 * kc + q;
    a[kc] = (arow < n && kk < ncols) ? g.X[(int64_t)arow * n + c0 + kk] - (ap == c0 + kk ? 1.0 : 0.0) : 0.0;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int tc = cb + 16 * j;
    if (tc >= n || tc == c0) continue;   // beyond the matrix, or the panel itself
    const int col = tc + c16;
    v4d acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = r0 + 16 * wave + 4 * v + q;
      acc[v] = (row < n && col < n) ? g.X[(int64_t)row * n + col] : 0.0;
    }
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const int kk = 4 * kc + q;
      const double b = (kk < ncols && col < n) ? g.XP[(int64_t)kk * n + col] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kc], b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = r0 + 16 * wave + 4 * v + q;
      if (row < n && col < n) g.X[(int64_t)row * n + col] = acc[v];
    }
  }
}

// A^{-1}[i][piv[c]] = X[piv[i]][c].
__global__ __launch_bounds__(256) void gje_big_out_kernel(const GjeDesc* __restrict__ e) {
  const GjeDesc d = e[blockIdx.y];
  const int n = d.n;
  const GjeBig g = gje_big_parts(d);
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const double* src = g.X + (int64_t)g.piv[i] * n;
    for (int c = threadIdx.x; c < n; c += 256) d.Ainv[(int64_t)i * d.ldi + g.piv[c]] = src[c];
  }
}

// Gauss-Jordan for blocks too large for registers, one launch per pivot
// step.  The working matrix alternates between the two n x n halves of W
// (step j reads what step j - 1 wrote, the first step reads A), so no
// workgroup reads what another writes in the same launch.  Every workgroup
// of a matrix finds the pivot of column j itself (same data, same reduction
// order: all agree) and updates its 64 columns; pivoting is implicit as in
// the register kernel (rows are never swapped; the rows already used, known
// from the recorded pivots, are skipped), and the write-out applies the
// permutation.
__global__ __launch_bounds__(256) void gje_step_kernel(const GjeDesc* __restrict__ e, int* pivs,
                                                       int64_t pstride, int j, int* flag) {
  const GjeDesc d = e[blockIdx.y];
  const int n = d.n;
  const int c0 = blockIdx.x * 64;
  if (j >= n || c0 >= n) return;   // uniform per workgroup, before any barrier
  const int64_t nn = (int64_t)n * n;
  const double* in = j == 0 ? d.A : d.W + ((j - 1) & 1) * nn;
  const int64_t ldi = j == 0 ? d.lda : n;
  double* out = d.W + (j & 1) * nn;
  int* piv = pivs + blockIdx.y * pstride;
  __shared__ unsigned used[2048];   // one bit per row (n <= 65536)
  __shared__ double rv[256];
  __shared__ int ri[256];
  const int tid = threadIdx.x;
  const int words = (n + 31) >> 5;
  for (int w = tid; w < words; w += 256) used[w] = 0u;
  __syncthreads();
  for (int t = tid; t < j; t += 256) {
    const int r = piv[t];
    atomicOr(&used[r >> 5], 1u << (r & 31));
  }
  __syncthreads();
  // pivot: largest |a_ij| over unused rows, lowest index on ties; the first
  // unused row is taken when all are zero, so the pivots form a permutation
  double best = -1.0;
  int bi = n;
  for (int i = tid; i < n; i += 256) {
    const bool free_row = !((used[i >> 5] >> (i & 31)) & 1u);
    const double v = fabs(in[(int64_t)i * ldi + j]);
    const bool take = free_row && (bi == n || v > best);
    best = take ? v : best;
    bi = take ? i : bi;
  }
  rv[tid] = best;
  ri[tid] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      const double ob = rv[tid + w];
      const int oi = ri[tid + w];
      const int cb = ri[tid];
      if (oi != n && (cb == n || ob > rv[tid] || (ob == rv[tid] && oi < cb))) {
        rv[tid] = ob;
        ri[tid] = oi;
      }
    }
    __syncthreads();
  }
  const int p = ri[0];
  if (blockIdx.x == 0 && tid == 0) {
    if (!(rv[0] > 0.0)) atomicOr(flag, 2);
    piv[j] = p;   // read by later launches only
  }
  const double pv = in[(int64_t)p * ldi + j];
  const double inv = pv != 0.0 ? 1.0 / pv : 0.0;
  // thread (wave, lane): column c0 + lane, rows wave, wave + 4, ...
  const int c = c0 + (tid & 63);
  if (c >= n) return;   // no barrier follows
  const bool isj = c == j;
  const double rp = in[(int64_t)p * ldi + c];
  const double prow = isj ? inv : rp * inv;
  for (int i = tid >> 6; i < n; i += 4) {
    const double fi = in[(int64_t)i * ldi + j] * inv;
    const double g = isj ? -fi : in[(int64_t)i * ldi + c] - fi * rp;
    out[(int64_t)i * n + c] = (i == p) ? prow : g;
  }
}

// A^{-1}[i][piv[c]] = W[piv[i]][c] from the half of W the last step wrote.
__global__ __launch_bounds__(256) void gje_out_kernel(const GjeDesc* __restrict__ e, const int* pivs,
                                                      int64_t pstride) {
  const GjeDesc d = e[blockIdx.y];
  const int n = d.n;
  const double* w = d.W + ((n - 1) & 1) * (int64_t)n * n;
  const int* piv = pivs + blockIdx.y * pstride;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const double* src = w + (int64_t)piv[i] * n;
    for (int c = threadIdx.x; c < n; c += 256) d.Ainv[(int64_t)i * d.ldi + piv[c]] = src[c];
  }
}

// The variant is chosen per matrix by its own size (blocked kernels for
// n <= 64 / 128 / 192, panel and update launches up to 1024, the
// one-launch-per-step form above beyond), so a matrix is
// inverted by the same instruction sequence whatever else is in the batch.
static rsrs_status gje_group(Uploader& up, hipStream_t st, const std::vector<GjeDesc>& e, int* flag,
                             int variant) {
  if (e.empty()) return RSRS_OK;
  GjeDesc* de = nullptr;
  RSRS_TRY(up.put_vec(e, &de));
  const unsigned nb = (unsigned)e.size();
  // algorithmic work: 2 n^3 flops per inversion (n^3 multiply-adds), one
  // FP64 read of A and one write of its inverse
  double gf = 0.0, gb = 0.0;
  for (const auto& x : e) {
    gf += 2.0 * (double)x.n * x.n * x.n;
    gb += 16.0 * (double)x.n * x.n;
  }
  if (variant < 3) {
    ProfScope ps(st, "gauss_jordan_blk", gf, gb);
    if (variant == 0)
      hipLaunchKernelGGL(gje_blk_kernel<4>, dim3(nb), dim3(512), 0, st, de, flag);
    else if (variant == 1)
      hipLaunchKernelGGL(gje_blk_kernel<8>, dim3(nb), dim3(512), 0, st, de, flag);
    else
      hipLaunchKernelGGL(gje_blk_kernel<12>, dim3(nb), dim3(512), 0, st, de, flag);
    RSRS_HIP(hipGetLastError());
    return RSRS_OK;
  }
  int nmax = 0;
  for (const auto& x : e) nmax = std::max(nmax, x.n);
  if (variant == 3) {   // 192 < n <= 1024: panel and update launches per 16 columns
    ProfScope ps(st, "gauss_jordan_big", gf, gb);
    const unsigned rb = (unsigned)((nmax + 63) / 64);
    hipLaunchKernelGGL(gje_big_init_kernel, dim3((unsigned)std::min(nmax, 1024), nb), dim3(256), 0, st, de);
    const int rl = (nmax + 63) / 64;
    for (int jt = 0; jt * 16 < nmax; ++jt) {
      if (rl <= 4)
        hipLaunchKernelGGL(gje_big_panel_kernel<4>, dim3(nb), dim3(256), 0, st, de, jt, flag);
      else if (rl <= 8)
        hipLaunchKernelGGL(gje_big_panel_kernel<8>, dim3(nb), dim3(256), 0, st, de, jt, flag);
      else if (rl <= 12)
        hipLaunchKernelGGL(gje_big_panel_kernel<12>, dim3(nb), dim3(256), 0, st, de, jt, flag);
      else
        hipLaunchKernelGGL(gje_big_panel_kernel<16>, dim3(nb), dim3(256), 0, st, de, jt, flag);
      hipLaunchKernelGGL(gje_big_update_kernel, dim3(rb, rb, nb), dim3(256), 0, st, de, jt);
    }
    hipLaunchKernelGGL(gje_big_out_kernel, dim3((unsigned)std::min(nmax, 1024), nb), dim3(256), 0, st, de);
    RSRS_HIP(hipGetLastError());
    return RSRS_OK;
  }
  // very large blocks: one launch per pivot step, the pivot rows of each
  // matrix recorded step by step
  const int64_t stride = round_up((int64_t)nmax, 64);
  DevBuf pivs;
  RSRS_TRY(pivs.alloc((size_t)stride * nb * sizeof(int)));
  ProfScope ps(st, "gauss_jordan_step", gf, gb);
  const unsigned cblk = (unsigned)((nmax + 63) / 64);
  for (int j = 0; j < nmax; ++j)
    hipLaunchKernelGGL(gje_step_kernel, dim3(cblk, nb), dim3(256), 0, st, de, pivs.as<int>(), stride, j, flag);
  hipLaunchKernelGGL(gje_out_kernel, dim3((unsigned)std::min(nmax, 1024), nb), dim3(256), 0, st, de,
                     pivs.as<int>(), stride);
  RSRS_HIP(hipGetLastError());
  // the pivot buffer must outlive the launches
  RSRS_HIP(hipStreamSynchronize(st));
  return RSRS_OK;
}

rsrs_status gje_inverse(Uploader& up, hipStream_t st, const std::vector<GjeDesc>& e, int* flag) {
  if (e.empty()) return RSRS_OK;
  std::vector<GjeDesc> grp[5];
  for (const auto& x : e) {
    if (x.n > 65536) {
      set_error("Gauss-Jordan block too large");
      return RSRS_E_UNSUPPORTED;
    }
    grp[x.n <= 64 ? 0 : x.n <= 128 ? 1 : x.n <= 192 ? 2 : x.n <= 1024 ? 3 : 4].push_back(x);
  }
  for (int v = 0; v < 5; ++v) RSRS_TRY(gje_group(up, st, grp[v], flag, v));
  return RSRS_OK;
}

// ---------------------------------------------------------------- copies
template <typename TS, typename TD>
__global__ void copy2d_kernel(const Copy2DT<TS, TD>* __restrict__ e) {
  const Copy2DT<TS, TD> d = e[blockIdx.y];
  const int64_t total = (int64_t)d.rows * d.cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / d.cols, c = idx % d.cols;
    const double v = d.alpha * (double)(d.trans ? d.src[c * d.lds + i] : d.src[i * d.lds + c]);
    if (d.accumulate) d.dst[i * d.ldd + c] = (TD)((double)d.dst[i * d.ldd + c] + v);
    else d.dst[i * d.ldd + c] = (TD)v;
  }
}

template <typename TS, typename TD>
rsrs_status copy2d(Uploader& up, hipStream_t st, const std::vector<Copy2DT<TS, TD>>& e) {
  if (e.empty()) return RSRS_OK;
  int64_t mx = 0;
  for (const auto& x : e) mx = std::max<int64_t>(mx, (int64_t)x.rows * x.cols);
  if (mx == 0) return RSRS_OK;
  Copy2DT<TS, TD>* de = nullptr;
  RSRS_TRY(up.put_vec(e, &de));
  const unsigned gx = (unsigned)std::min<int64_t>((mx + 255) / 256, 4096);
  ProfScope ps(st, "copy2d");
  hipLaunchKernelGGL((copy2d_kernel<TS, TD>), dim3(gx, (unsigned)e.size()), dim3(256), 0, st, de);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}

template <typename T>
__global__ void sym_kernel(const SymDesc<T>* __restrict__ e) {
  const SymDesc<T> d = e[blockIdx.y];
  const int64_t total = (int64_t)d.n * d.n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / d.n, c = idx % d.n;
    if (c >= i) continue;   // each pair once, by its lower element
    const T v = (T)(0.5 * ((double)d.A[i * d.ld + c] + (double)d.A[c * d.ld + i]));
    d.A[i * d.ld + c] = v;
    d.A[c * d.ld + i] = v;
  }
}

template <typename T>
rsrs_status symmetrize(Uploader& up, hipStream_t st, const std::vector<SymDesc<T>>& e) {
  if (e.empty()) return RSRS_OK;
  int64_t mx = 0;
  for (const auto& x : e) mx = std::max<int64_t>(mx, (int64_t)x.n * x.n);
  if (mx == 0) return RSRS_OK;
  SymDesc<T>* de = nullptr;
  RSRS_TRY(up.put_vec(e, &de));
  const unsigned gx = (unsigned)std::min<int64_t>((mx + 255) / 256, 1024);
  ProfScope ps(st, "symmetrize");
  hipLaunchKernelGGL((sym_kernel<T>), dim3(gx, (unsigned)e.size()), dim3(256), 0, st, de);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}
template rsrs_status symmetrize<double>(Uploader&, hipStream_t, const std::vector<SymDesc<double>>&);
template rsrs_status symmetrize<float>(Uploader&, hipStream_t, const std::vector<SymDesc<float>>&);

template <typename TS, typename TD>
__global__ void gather_rows_kernel(TD* dst, int64_t ldd, const TS* src, int64_t lds,
                                   const int64_t* idx, int64_t nrows, int64_t ncols) {
  for (int64_t i = blockIdx.x; i < nrows; i += gridDim.x) {
    const TS* s = src + idx[i] * lds;
    TD* d = dst + i * ldd;
    for (int64_t c = threadIdx.x; c < ncols; c += blockDim.x) d[c] = (TD)s[c];
  }
}
template <typename TS, typename TD>
__global__ void scatter_rows_kernel(TD* dst, int64_t ldd, const TS* src, int64_t lds,
                                    const int64_t* idx, int64_t nrows, int64_t ncols) {
  for (int64_t i = blockIdx.x; i < nrows; i += gridDim.x) {
    const TS* s = src + i * lds;
    TD* d = dst + idx[i] * ldd;
    for (int64_t c = threadIdx.x; c < ncols; c += blockDim.x) d[c] = (TD)s[c];
  }
}

template <typename TS, typename TD>
void gather_rows(hipStream_t st, TD* dst, int64_t ldd, const TS* src, int64_t lds,
                 const int64_t* idx, int64_t nrows, int64_t ncols) {
  if (nrows <= 0 || ncols <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>(nrows, 65535);
  const unsigned b = ncols >= 256 ? 256 : (ncols >= 64 ? 64 : 32);
  ProfScope ps(st, "gather_rows", 0.0, (double)(sizeof(TS) + sizeof(TD)) * nrows * ncols);
  hipLaunchKernelGGL((gather_rows_kernel<TS, TD>), dim3(g), dim3(b), 0, st, dst, ldd, src, lds, idx, nrows, ncols);
}
template <typename TS, typename TD>
void scatter_rows(hipStream_t st, TD* dst, int64_t ldd, const TS* src, int64_t lds,
                  const int64_t* idx, int64_t nrows, int64_t ncols) {
  if (nrows <= 0 || ncols <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>(nrows, 65535);
  const unsigned b = ncols >= 256 ? 256 : (ncols >= 64 ? 64 : 32);
  ProfScope ps(st, "scatter_rows", 0.0, (double)(sizeof(TS) + sizeof(TD)) * nrows * ncols);
  hipLaunchKernelGGL((scatter_rows_kernel<TS, TD>), dim3(g), dim3(b), 0, st, dst, ldd, src, lds, idx, nrows, ncols);
}

#define RSRS_PAIR(TS, TD)                                                                          \
  template rsrs_status copy2d<TS, TD>(Uploader&, hipStream_t, const std::vector<Copy2DT<TS, TD>>&); \
  template void gather_rows<TS, TD>(hipStream_t, TD*, int64_t, const TS*, int64_t, const int64_t*,  \
                                    int64_t, int64_t);                                              \
  template void scatter_rows<TS, TD>(hipStream_t, TD*, int64_t, const TS*, int64_t, const int64_t*, \
                                     int64_t, int64_t);
RSRS_PAIR(double, double)
RSRS_PAIR(double, float)
RSRS_PAIR(float, double)
RSRS_PAIR(float, float)
#undef RSRS_PAIR

__global__ void fill_kernel(double* p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
void fill(hipStream_t st, double* p, int64_t n, double v) {
  if (n <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(fill_kernel, dim3(g), dim3(256), 0, st, p, n, v);
}

template <typename T>
__global__ void finite_kernel(const T* p, int64_t rows, int64_t cols, int64_t ld, int* flag) {
  bool bad = false;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < rows * cols;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const T v = p[(idx / cols) * ld + idx % cols];
    if (!isfinite(v)) bad = true;
  }
  if (bad) atomicOr(flag, 4);
}
template <typename T>
void check_finite(hipStream_t st, const T* p, int64_t rows, int64_t cols, int64_t ld, int* flag) {
  if (rows <= 0 || cols <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>((rows * cols + 255) / 256, 8192);
  ProfScope ps(st, "check_finite", 0.0, (double)sizeof(T) * rows * cols);
  hipLaunchKernelGGL((finite_kernel<T>), dim3(g), dim3(256), 0, st, p, rows, cols, ld, flag);
}
template void check_finite<double>(hipStream_t, const double*, int64_t, int64_t, int64_t, int*);
template void check_finite<float>(hipStream_t, const float*, int64_t, int64_t, int64_t, int*);

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
  ProfScope ps(st, "col_sumsq", 2.0 * n * w, 8.0 * n * w);
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
  ProfScope ps(st, "sub2d", n * w, 24.0 * n * w);
  hipLaunchKernelGGL(sub2d_kernel, dim3(g), dim3(256), 0, st, f, ldf, y, ldy, z, ldz, n, w);
}

// ---------------------------------------------------------------- skinny product
// Y = A X for a dense row-major A (M x K) and a narrow X (K x N, N <= 16),
// all FP64: the product streams A once, so it is HBM-bound.  K is split into
// chunks whose slice of X (1 MB) stays in L2 while every row block streams
// its rows of A straight into registers; each wave forms a 16 x 16 tile on
// FP64 MFMA.  Lane (m, q) holds row m; its load t brings k = 8 t + 2 q and
// the next, so that the four lanes of a row read 64 contiguous bytes per
// load (the k of a lane's operand in MFMA j is 8 (j / 2) + 2 q + j % 2; X is
// staged in LDS in the same order); the partial tiles of the chunks are
// summed in chunk order by a second launch, so the result does not depend
// on the schedule.
namespace {
constexpr int SK_RM = 64;    // rows per workgroup (16 per wave)
constexpr int SK_KC = 128;   // k per iteration

__global__ __launch_bounds__(256) void skinny_f64_kernel(const double* __restrict__ A, int64_t lda, int M,
                                                         const double* __restrict__ X, int64_t ldx, int N,
                                                         double* __restrict__ P, int klen) {
  __shared__ double Xs[2][SK_KC * 16];
  const int ks = blockIdx.y;
  const int k_lo = ks * klen;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = lane & 15, q = lane >> 4;
  const int r0 = blockIdx.x * SK_RM + wave * 16;
  const double* arow = A + (int64_t)min(r0 + m, M - 1) * lda + k_lo + 2 * q;
  double ar[2][32];
  double xr[8];
  auto load_a = [&](int it, double (&dst)[32]) {
    const double* src = arow + (int64_t)it * SK_KC;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const double2 v = *reinterpret_cast<const double2*>(src + 8 * t);
      dst[2 * t] = v.x;
      dst[2 * t + 1] = v.y;
    }
  };
  auto load_x = [&](int it) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = tid * 8 + t, k = k_lo + it * SK_KC + e / 16, n = e % 16;
      xr[t] = n < N ? X[(int64_t)k * ldx + n] : 0.0;
    }
  };
  auto stash_x = [&](int b) {
#pragma unroll
    for (int t = 0; t < 8; ++t) Xs[b][tid * 8 + t] = xr[t];
  };
  const int iters = klen / SK_KC;   // even
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
  // one iteration: prefetch the next slice into the other register set and
  // LDS buffer, multiply the current one (register sets named statically)
  auto step = [&](int it, int cb, double (&cur)[32], double (&nxt)[32]) {
    const bool more = it + 1 < iters;
    if (more) {
      load_a(it + 1, nxt);
      load_x(it + 1);
    }
#pragma unroll
    for (int j = 0; j < 32; ++j)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[j], Xs[cb][(8 * (j >> 1) + 2 * q + (j & 1)) * 16 + m], acc, 0,
                                                 0, 0);
    if (more) stash_x(cb ^ 1);
    __syncthreads();
  };
  load_a(0, ar[0]);
  load_x(0);
  stash_x(0);
  __syncthreads();
  for (int it = 0; it < iters; it += 2) {
    step(it, 0, ar[0], ar[1]);
    step(it + 1, 1, ar[1], ar[0]);
  }
  // D[4 v + q][m]: row r0 + 4 v + q, column m
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = r0 + 4 * v + q;
    if (r < M && m < N) P[((int64_t)ks * M + r) * 16 + m] = acc[v];
  }
}

__global__ void skinny_sum_kernel(const double* __restrict__ P, int M, int N, int ksplit, double* Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)M * 16) return;
  const int r = (int)(e / 16), n = (int)(e % 16);
  if (n >= N) return;
  double s = 0.0;
  for (int t = 0; t < ksplit; ++t) s += P[((int64_t)t * M + r) * 16 + n];
  Y[(int64_t)r * ldy + n] = s;
}
}  // namespace

bool skinny_f64_ok(const double* A, int64_t lda, int64_t M, int64_t K, int64_t N) {
  return N >= 1 && N <= 16 && M >= 1 && M <= INT32_MAX && K % (16 * SK_KC) == 0 && K > 0 && K <= INT32_MAX &&
         lda % 2 == 0 && ((uintptr_t)A & 15) == 0;
}

size_t skinny_f64_scratch(int64_t M) { return (size_t)8 * M * 16 * sizeof(double); }

rsrs_status skinny_f64(hipStream_t st, const double* A, int64_t lda, int64_t M, int64_t K, const double* X,
                       int64_t ldx, int64_t N, double* Y, int64_t ldy, double* scratch) {
  if (!skinny_f64_ok(A, lda, M, K, N)) {
    set_error("skinny product: unsupported shape or alignment");
    return RSRS_E_INVALID;
  }
  constexpr int ksplit = 8;
  const int klen = (int)(K / ksplit);
  {
    ProfScope ps(st, "skinny_f64:operator", 2.0 * M * N * K, 8.0 * (M * K + K * N));
    hipLaunchKernelGGL(skinny_f64_kernel, dim3((unsigned)((M + SK_RM - 1) / SK_RM), ksplit), dim3(256), 0, st,
                       A, lda, (int)M, X, ldx, (int)N, scratch, klen);
    RSRS_HIP(hipGetLastError());
  }
  const int64_t tot = M * 16;
  hipLaunchKernelGGL(skinny_sum_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, scratch, (int)M,
                     (int)N, ksplit, Y, ldy);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}

}  // namespace rsrs
