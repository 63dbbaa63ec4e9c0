// Batched dense helpers: GEMM dispatch, Cholesky leaves, Gauss-Jordan inverse,
// copies, permutations and reductions (FP64).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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

// Tile choice, measured on MI355X: 128 x 128 tiles on 8 waves (each wave
// 64 x 32, 4 waves per SIMD) reach 50+ TFLOP/s on the large FP64 products;
// they are used whenever the batch still yields >= 256 such tiles, otherwise
// 64 x 64 tiles on 4 waves keep the chip busy; narrow right-hand sides use
// 64 x 16.
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
  int64_t t128 = 0;
  for (const auto& d : descs) {
    if (d.M <= 0 || d.N <= 0) continue;
    const int64_t tm = (d.M + 127) / 128, tn = (d.N + 127) / 128;
    t128 += mode == GM_SYRK_L ? tm * (tm + 1) / 2 : tm * tn;
  }
  if (t128 >= 256) return plan_forms<TI, TO, 128, 128, 2, 4>(descs, base, ta, tb, mode, out);
  return plan_forms<TI, TO, 64, 64, 2, 2>(descs, base, ta, tb, mode, out);
}

rsrs_status gemm_exec(const GemmLaunch& L, const void* descs, size_t desc_bytes, hipStream_t st) {
  const void* p = static_cast<const char*>(descs) + L.first * desc_bytes;
  void* args[] = {&p};
  ProfScope ps(st, L.tag, L.flops, L.bytes);
  RSRS_HIP(hipLaunchKernel(L.fn, L.grid, L.block, args, 0, st));
  return RSRS_OK;
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
// Gauss-Jordan inversion with partial pivoting, the matrix held in registers:
// 1024 threads as a 32 x 32 grid, thread (ti, tc) owning rows ti + 32a and
// columns tc + 32b (a, b < R).  Pivoting is implicit (rows are never
// swapped): step j publishes column j to LDS, every wave finds the pivot row
// p itself (largest |a_ij| over rows not yet used, lowest index on ties) by a
// shuffle reduction, the owners of row p publish it, and every element is
// updated branch-free; column and row buffers alternate by step parity, so a
// step costs two barriers.  With pivot rows p_j the working matrix W ends as
// A^{-1}[i][c] = W[p_i][q_c], q the inverse permutation, applied on write-out.
template <int R>
__global__ __launch_bounds__(1024) void gje_reg_kernel(const GjeDesc* __restrict__ e, int* flag) {
  constexpr int NMAX = 32 * R;
  const GjeDesc d = e[blockIdx.x];
  const int n = d.n;
  const int tid = threadIdx.x;
  const int ti = tid >> 5, tc = tid & 31;
  const int lane = tid & 63;
  __shared__ double colb[2][NMAX];
  __shared__ double rowb[2][NMAX];
  __shared__ int usedf[NMAX];
  __shared__ int piv[NMAX];
  __shared__ int qinv[NMAX];
  double a[R][R];
#pragma unroll
  for (int x = 0; x < R; ++x)
#pragma unroll
    for (int y = 0; y < R; ++y) {
      const int i = ti + 32 * x, c = tc + 32 * y;
      a[x][y] = (i < n && c < n) ? d.A[(int64_t)i * d.lda + c] : 0.0;
    }
  for (int i = tid; i < NMAX; i += 1024) usedf[i] = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double* colv = colb[j & 1];
    double* rowv = rowb[j & 1];
    const int jy = j >> 5, jc = j & 31;
    if (tc == jc) {
#pragma unroll
      for (int x = 0; x < R; ++x) {
        double v = 0.0;
#pragma unroll
        for (int y = 0; y < R; ++y) v = (y == jy) ? a[x][y] : v;
        colv[ti + 32 * x] = v;
      }
    }
    __syncthreads();
    // the first candidate is always taken, so the pivots form a permutation
    double best = -1.0;
    int bi = NMAX;
    for (int i = lane; i < n; i += 64) {
      const double v = fabs(colv[i]);
      const bool take = !usedf[i] && (bi == NMAX || v > best);
      best = take ? v : best;
      bi = take ? i : bi;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      const bool take = oi != NMAX && (bi == NMAX || ob > best || (ob == best && oi < bi));
      best = take ? ob : best;
      bi = take ? oi : bi;
    }
    const int p = bi;
    if (!(best > 0.0) && tid == 0) atomicOr(flag, 2);
    const int px = p >> 5;
    if (ti == (p & 31)) {
#pragma unroll
      for (int y = 0; y < R; ++y) {
        double v = 0.0;
#pragma unroll
        for (int x = 0; x < R; ++x) v = (x == px) ? a[x][y] : v;
        rowv[tc + 32 * y] = v;
      }
    }
    __syncthreads();
    if (tid == 0) {
      usedf[p] = 1;
      piv[j] = p;
    }
    const double pv = colv[p];
    const double inv = pv != 0.0 ? 1.0 / pv : 0.0;
    double rv[R], prow[R], fi[R];
    bool isj[R], isp[R];
#pragma unroll
    for (int y = 0; y < R; ++y) {
      rv[y] = rowv[tc + 32 * y];
      isj[y] = (tc + 32 * y) == j;
      prow[y] = isj[y] ? inv : rv[y] * inv;   // new pivot row (column j: 1 / pivot)
    }
#pragma unroll
    for (int x = 0; x < R; ++x) {
      fi[x] = colv[ti + 32 * x] * inv;
      isp[x] = (ti + 32 * x) == p;
    }
#pragma unroll
    for (int x = 0; x < R; ++x)
#pragma unroll
      for (int y = 0; y < R; ++y) {
        const double g = isj[y] ? -fi[x] : a[x][y] - fi[x] * rv[y];
        a[x][y] = isp[x] ? prow[y] : g;
      }
  }
  __syncthreads();
  for (int j = tid; j < n; j += 1024) qinv[piv[j]] = j;
  __syncthreads();
#pragma unroll
  for (int x = 0; x < R; ++x)
#pragma unroll
    for (int y = 0; y < R; ++y) {
      const int ri = ti + 32 * x, ci = tc + 32 * y;
      if (ri < n && ci < n) d.Ainv[(int64_t)qinv[ri] * d.ldi + piv[ci]] = a[x][y];
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

// The variant is chosen per matrix by its own size (register kernels for
// n <= 64 / 128 / 192, the global two-launch form above), so a matrix is
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
    ProfScope ps(st, "gauss_jordan_reg", gf, gb);
    if (variant == 0)
      hipLaunchKernelGGL(gje_reg_kernel<2>, dim3(nb), dim3(1024), 0, st, de, flag);
    else if (variant == 1)
      hipLaunchKernelGGL(gje_reg_kernel<4>, dim3(nb), dim3(1024), 0, st, de, flag);
    else
      hipLaunchKernelGGL(gje_reg_kernel<6>, dim3(nb), dim3(1024), 0, st, de, flag);
    RSRS_HIP(hipGetLastError());
    return RSRS_OK;
  }
  int nmax = 0;
  for (const auto& x : e) nmax = std::max(nmax, x.n);
  // large blocks: the pivot rows of each matrix, recorded step by step
  const int64_t stride = round_up((int64_t)nmax, 64);
  DevBuf pivs;
  RSRS_TRY(pivs.alloc((size_t)stride * nb * sizeof(int)));
  ProfScope ps(st, "gauss_jordan_big", gf, gb);
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
  std::vector<GjeDesc> grp[4];
  for (const auto& x : e) {
    if (x.n > 65536) {
      set_error("Gauss-Jordan block too large");
      return RSRS_E_UNSUPPORTED;
    }
    grp[x.n <= 64 ? 0 : x.n <= 128 ? 1 : x.n <= 192 ? 2 : 3].push_back(x);
  }
  for (int v = 0; v < 4; ++v) RSRS_TRY(gje_group(up, st, grp[v], flag, v));
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
