// Row interpolative decomposition by greedy column-pivoted QR (Sec. 2.3,
// eq. id_factorization), batched over the boxes of one colour class.
//
// The QR of M^T with column pivoting is run as pivoted modified Gram-Schmidt
// on the rows of M: at step j the row of largest residual norm becomes pivot
// p_j, every other unselected row i is orthogonalised against it,
//   d_ij = <m_i, m_p> / |m_p|,   m_i <- m_i - (<m_i, m_p> / |m_p|^2) m_p,
// and its residual norm is recomputed exactly from the updated row (no
// downdating).  d_ij are the entries R[j, i] of the triangular factor, so with
// S = {p_0..p_{k-1}} and R the other rows, T = (R11^{-1} R12)^T and
// M_R ~ T M_S.  Ties in the pivot choice go to the lowest row index.
//
// One launch per step, one wave per row.  Norms are double-buffered by step
// parity so that every wave of a step sees the same pivot; rows other than
// the pivot are only written by their own wave, and the pivot row is only read.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>

#include "kernels.hpp"
#include "profile.hpp"

namespace rsrs {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename S>
__global__ __launch_bounds__(64) void id_init_kernel(const IdDesc* __restrict__ e) {
  const IdDesc d = e[blockIdx.y];
  const int i = blockIdx.x;
  if (i >= d.b) return;
  S* mi = static_cast<S*>(d.M) + (int64_t)i * d.ldm;
  const S* mz = d.MZ ? static_cast<const S*>(d.MZ) + (int64_t)i * d.ldz : nullptr;
  double s = 0.0;
  for (int c = threadIdx.x; c < d.s; c += 64) {
    S v = mi[c];
    if (mz) {
      v = (S)((double)v + (double)mz[c]);
      mi[c] = v;
    }
    s += (double)v * (double)v;
  }
  s = wave_sum(s);
  if (threadIdx.x == 0) {
    d.norms[i] = s;
    d.sel[i] = INT_MAX;
  }
  if (d.tol2 > 0.0) {   // |[Y_B Z_B] row i|^2 for the rank threshold
    const int64_t gi = d.idx[i];
    const S* yr = static_cast<const S*>(d.Yg) + gi * d.ldy;
    const S* zr = d.Zg ? static_cast<const S*>(d.Zg) + gi * d.ldy : nullptr;
    double q = 0.0;
    for (int c = threadIdx.x; c < d.sy; c += 64) {
      const double y = (double)yr[c];
      q += y * y;
      if (zr) {
        const double z = (double)zr[c];
        q += z * z;
      }
    }
    q = wave_sum(q);
    if (threadIdx.x == 0) d.rowyz[i] = q;
  }
}

template <typename S>
__global__ __launch_bounds__(64) void id_step_kernel(const IdDesc* __restrict__ e, int j) {
  const IdDesc d = e[blockIdx.y];
  const int i = blockIdx.x;
  if (i >= d.b || j >= d.k) return;
  const int lane = threadIdx.x;
  const double* cur = d.norms + (j & 1) * d.b;
  double* nxt = d.norms + ((j + 1) & 1) * d.b;
  // pivot: argmax over rows not selected before step j (lowest index on ties)
  double best = -1.0;
  int bi = INT_MAX;
  for (int x = lane; x < d.b; x += 64) {
    if (d.sel[x] < j) continue;
    const double v = cur[x];
    // the first candidate is always taken, so a NaN norm cannot leave bi unset
    if (bi == INT_MAX || v > best) { best = v; bi = x; }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (oi != INT_MAX && (bi == INT_MAX || ob > best || (ob == best && oi < bi))) { best = ob; bi = oi; }
  }
  const int p = bi;   // always a valid row: b - j > 0 candidates remain for j < k <= b
  const double pn2 = best > 0.0 ? best : 0.0;   // also maps NaN to 0
  const double pn = sqrt(pn2);
  if (i == p) {
    if (lane == 0) {
      d.sel[p] = j;
      d.piv[j] = p;
      d.Rc[(int64_t)p * d.k + j] = pn;
      nxt[p] = 0.0;
    }
    return;
  }
  if (d.sel[i] < j) return;  // selected at an earlier step
  S* mi = static_cast<S*>(d.M) + (int64_t)i * d.ldm;
  const S* mp = static_cast<const S*>(d.M) + (int64_t)p * d.ldm;
  double dot = 0.0;
  for (int c = lane; c < d.s; c += 64) dot += (double)mi[c] * (double)mp[c];
  dot = wave_sum(dot);
  const double coef = pn2 > 0.0 ? dot / pn2 : 0.0;
  double s = 0.0;
  for (int c = lane; c < d.s; c += 64) {
    const S v = (S)((double)mi[c] - coef * (double)mp[c]);
    mi[c] = v;
    s += (double)v * (double)v;
  }
  s = wave_sum(s);
  if (lane == 0) {
    d.Rc[(int64_t)i * d.k + j] = pn > 0.0 ? dot / pn : 0.0;
    nxt[i] = s;
  }
}

// Same step with the row and the pivot row held in registers (R doubles per
// lane, s <= 64 R): one read of each and one write of the row per step
// instead of two passes over both.  Four rows per workgroup (one per wave);
// the row is requested before the pivot search so that its load overlaps
// the search, and the search itself loads all candidates at once.
// V consecutive elements at p (V = 1, or 2 with p 8-byte aligned).
template <typename S, int V>
__device__ __forceinline__ void load_v(const S* p, S (&out)[V]) {
  if constexpr (V == 2) {
    static_assert(sizeof(S) == 4, "pairs of FP32 values");
    const float2 v = *reinterpret_cast<const float2*>(p);
    out[0] = v.x;
    out[1] = v.y;
  } else {
    out[0] = p[0];
  }
}

template <typename S, int R, int V>
__global__ __launch_bounds__(256) void id_step_reg_kernel(const IdDesc* __restrict__ e, int j) {
  const IdDesc d = e[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int i = 4 * blockIdx.x + (threadIdx.x >> 6);
  if (i >= d.b || j >= d.k) return;
  // Rows are kept in their storage type (converted to FP64 where used); lane
  // l holds columns V l + 64 V u + t.  Loads come from a clamped chunk
  // (s is a multiple of V), unconditionally, so that all are in flight at
  // once; FP32 rows move two columns per load.
  S* mi = static_cast<S*>(d.M) + (int64_t)i * d.ldm;
  S ri[R][V];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int c = V * lane + 64 * V * u;
    S v[V];
    load_v<S, V>(mi + min(c, d.s - V), v);
#pragma unroll
    for (int t = 0; t < V; ++t) ri[u][t] = c < d.s ? v[t] : S(0);
  }
  const double* cur = d.norms + (j & 1) * d.b;
  double* nxt = d.norms + ((j + 1) & 1) * d.b;
  // pivot: argmax over rows not selected before step j (lowest index on ties;
  // the first candidate is always taken, so a NaN norm cannot leave bi unset)
  double best = -1.0;
  int bi = INT_MAX;
  for (int x0 = 0; x0 < d.b; x0 += 256) {
    int sv[4];
    double nv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int x = x0 + lane + 64 * u;
      sv[u] = x < d.b ? d.sel[x] : -1;
      nv[u] = x < d.b ? cur[x] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool take = sv[u] >= j && (bi == INT_MAX || nv[u] > best);
      best = take ? nv[u] : best;
      bi = take ? x0 + lane + 64 * u : bi;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    const bool take = oi != INT_MAX && (bi == INT_MAX || ob > best || (ob == best && oi < bi));
    best = take ? ob : best;
    bi = take ? oi : bi;
  }
  const int p = bi;   // always a valid row: b - j > 0 candidates remain for j < k <= b
  const double pn2 = best > 0.0 ? best : 0.0;   // also maps NaN to 0
  const double pn = sqrt(pn2);
  if (i == p) {
    if (lane == 0) {
      d.sel[p] = j;
      d.piv[j] = p;
      d.Rc[(int64_t)p * d.k + j] = pn;
      nxt[p] = 0.0;
    }
    return;
  }
  if (d.sel[i] < j) return;
  const S* mp = static_cast<const S*>(d.M) + (int64_t)p * d.ldm;
  S rp[R][V];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int c = V * lane + 64 * V * u;
    S v[V];
    load_v<S, V>(mp + min(c, d.s - V), v);
#pragma unroll
    for (int t = 0; t < V; ++t) rp[u][t] = c < d.s ? v[t] : S(0);
  }
  double dot = 0.0;
#pragma unroll
  for (int u = 0; u < R; ++u)
#pragma unroll
    for (int t = 0; t < V; ++t) dot += (double)ri[u][t] * (double)rp[u][t];
  dot = wave_sum(dot);
  const double coef = pn2 > 0.0 ? dot / pn2 : 0.0;
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int c = V * lane + 64 * V * u;
    S v[V];
#pragma unroll
    for (int t = 0; t < V; ++t) {
      v[t] = (S)((double)ri[u][t] - coef * (double)rp[u][t]);   // the norm is that of the stored row
      s += c < d.s ? (double)v[t] * (double)v[t] : 0.0;
    }
    if (c < d.s) {
      if constexpr (V == 2) *reinterpret_cast<float2*>(mi + c) = make_float2(v[0], v[1]);
      else mi[c] = v[0];
    }
  }
  s = wave_sum(s);
  if (lane == 0) {
    d.Rc[(int64_t)i * d.k + j] = pn > 0.0 ? dot / pn : 0.0;
    nxt[i] = s;
  }
}

// k_B (all k steps, or with a rank tolerance the leading steps whose pivot
// norm exceeds the threshold), then S and R sorted; T = (R11^{-1} R12)^T
// written with columns in sorted-S order.  Positions come from a block-wide
// prefix count of the selected rows; for k_B <= 64, R11 is staged in LDS and
// each thread solves for one row of R with the solution in registers (larger
// k_B reads R11 from global memory).
__global__ __launch_bounds__(256) void id_finalize_kernel(const IdDesc* __restrict__ e) {
  const IdDesc d = e[blockIdx.x];
  const int b = d.b, ks = d.k;   // ks: steps taken, also the row stride of Rc
  constexpr int KL = 64;
  __shared__ int pre[4352 + 1];       // pre[x] = number of selected rows < x
  __shared__ int cnt[256];
  __shared__ int rank_of_step[256];   // rank of pivot p_t inside sorted S
  __shared__ double part[256];
  __shared__ int kshared;
  __shared__ double R11[KL * KL];
  const int tid = threadIdx.x;
  const int seg = (b + 255) / 256;
  const int lo = min(b, tid * seg), hi = min(b, lo + seg);
  if (d.tol2 > 0.0) {
    // threshold from ||[Y_B Z_B]||_F^2, summed in a fixed order
    double q = 0.0;
    for (int x = lo; x < hi; ++x) q += d.rowyz[x];
    part[tid] = q;
    __syncthreads();
    if (tid == 0) {
      double tot = 0.0;
      for (int u = 0; u < 256; ++u) tot += part[u];
      const double thr2 = d.tol2 * tot;
      int kb = ks;
      for (int j = 0; j < ks; ++j) {
        const double pn = d.Rc[(int64_t)d.piv[j] * ks + j];
        if (pn * pn <= thr2) { kb = j; break; }
      }
      kshared = kb;
    }
  } else if (tid == 0) {
    kshared = ks;
  }
  __syncthreads();
  const int k = kshared, r = b - k;
  if (tid == 0) *d.kB = k;
  int c = 0;
  for (int x = lo; x < hi; ++x) c += d.sel[x] < k ? 1 : 0;
  cnt[tid] = c;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int q = 0; q < 256; ++q) {
      const int v = cnt[q];
      cnt[q] = run;
      run += v;
    }
  }
  __syncthreads();
  {
    int run = cnt[tid];
    for (int x = lo; x < hi; ++x) {
      pre[x] = run;
      if (d.sel[x] < k) d.Spos[run] = x;
      else d.Spos[k + x - run] = x;
      run += d.sel[x] < k ? 1 : 0;
    }
  }
  __syncthreads();
  if (k == 0) return;   // no skeletons: T has no columns
  for (int t = tid; t < k; t += 256) rank_of_step[t] = pre[d.piv[t]];
  if (k <= KL) {
    // R11 padded to 64 x 64 (identity beyond k); each thread keeps its
    // solution in registers, the padding adding exact zeros
    for (int idx = tid; idx < KL * KL; idx += 256) {
      const int t = idx / KL, u = idx % KL;
      double v = (t == u) ? 1.0 : 0.0;
      if (t < k && u < k) v = t <= u ? d.Rc[(int64_t)d.piv[u] * ks + t] : 0.0;
      R11[idx] = v;
    }
    __syncthreads();
    for (int q = tid; q < r; q += 256) {
      const int i = (int)d.Spos[k + q];
      const double* cr = d.Rc + (int64_t)i * ks;
      double* Tq = d.T + (int64_t)q * d.ldt;
      // back substitution R11 x = c, R11[t][u] = Rc[p_u][t] (t <= u), in
      // place: c[t] becomes x[t] once rows t + 1.. are done.  The scheduling
      // fences keep the LDS reads of R11 from being hoisted en masse.
      double c[KL];
#pragma unroll
      for (int t = 0; t < KL; ++t) c[t] = t < k ? cr[t] : 0.0;
#pragma unroll
      for (int t = KL - 1; t >= 0; --t) {
        double acc = c[t];
#pragma unroll
        for (int u = t + 1; u < KL; ++u) {
          acc -= R11[t * KL + u] * c[u];
          if (((u - t) & 7) == 0) __builtin_amdgcn_sched_barrier(0);
        }
        const double diag = R11[t * KL + t];
        c[t] = diag != 0.0 ? acc / diag : 0.0;
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int t = 0; t < KL; ++t)
        if (t < k) Tq[rank_of_step[t]] = c[t];
    }
    return;
  }
  __syncthreads();
  for (int q = tid; q < r; q += 256) {
    const int i = (int)d.Spos[k + q];
    const double* cr = d.Rc + (int64_t)i * ks;
    double* Tq = d.T + (int64_t)q * d.ldt;
    // back substitution R11 x = c, R11[t][u] = Rc[p_u][t] (t <= u)
    for (int t = k - 1; t >= 0; --t) {
      double acc = cr[t];
      for (int u = t + 1; u < k; ++u) acc -= d.Rc[(int64_t)d.piv[u] * ks + t] * Tq[rank_of_step[u]];
      const double diag = d.Rc[(int64_t)d.piv[t] * ks + t];
      Tq[rank_of_step[t]] = diag != 0.0 ? acc / diag : 0.0;
    }
  }
}

// Per step, the descriptors [0, npair) take the paired FP32 layout and the
// rest the one-column layout.  The one-column forms (16 or 40 registers, or
// the streaming kernel) sum every dot product and norm in the same order,
// so which of them runs does not change a bit; the paired layout sums in
// another order, so a box takes it according to its own row length and
// alignment only (never according to the other boxes of the launch).
template <typename S>
static void id_launch(hipStream_t st, const IdDesc* de, unsigned npair, unsigned nsingle, int bpair, int bsingle,
                      int kmax, int ssingle, double fstep, double bstep) {
  const unsigned nb = npair + nsingle;
  {
    ProfScope ps(st, "id_init", 0.0, bstep);
    hipLaunchKernelGGL(id_init_kernel<S>, dim3((unsigned)std::max(bpair, bsingle), nb), dim3(64), 0, st, de);
  }
  // The steps are many short launches: when measured, each carries its own
  // start / stop events instead of two separate event records.
  const int nchunk = (ssingle + 63) / 64;
  for (int j = 0; j < kmax; ++j) {
    hipEvent_t ea, eb;
    const int slot = prof_begin_ext("id_step", &ea, &eb);
    if (npair > 0) {
      const unsigned g4 = (unsigned)((bpair + 3) / 4);
      hipExtLaunchKernelGGL((id_step_reg_kernel<S, 20, (sizeof(S) == 4 ? 2 : 1)>), dim3(g4, npair), dim3(256), 0, st,
                            ea, nsingle > 0 ? nullptr : eb, 0, de, j);
    }
    if (nsingle > 0) {
      const IdDesc* d1 = de + npair;
      hipEvent_t e0 = npair > 0 ? nullptr : ea;
      const unsigned g4 = (unsigned)((bsingle + 3) / 4);
      if (nchunk <= 16)
        hipExtLaunchKernelGGL((id_step_reg_kernel<S, 16, 1>), dim3(g4, nsingle), dim3(256), 0, st, e0, eb, 0, d1, j);
      else if (nchunk <= 40)
        hipExtLaunchKernelGGL((id_step_reg_kernel<S, 40, 1>), dim3(g4, nsingle), dim3(256), 0, st, e0, eb, 0, d1, j);
      else
        hipExtLaunchKernelGGL(id_step_kernel<S>, dim3((unsigned)bsingle, nsingle), dim3(64), 0, st, e0, eb, 0, d1, j);
    }
    if (slot >= 0) prof_end_ext(slot, "id_step", fstep, bstep);
  }
}

rsrs_status id_run(Uploader& up, hipStream_t st, const std::vector<IdDesc>& e, bool fp32) {
  if (e.empty()) return RSRS_OK;
  int kmax = 0;
  for (const auto& x : e) {
    if (x.k > 256 || x.b > 4352 || x.k > x.b || x.k < 1) {
      set_error("ID sizes out of range (need 1 <= k <= b <= 4352, k <= 256)");
      return RSRS_E_UNSUPPORTED;
    }
    kmax = std::max(kmax, x.k);
  }
  // paired FP32 rows: even length and leading dimension, 8-byte aligned,
  // and short enough for 20 pairs per lane
  auto paired = [&](const IdDesc& x) {
    return fp32 && x.s % 2 == 0 && x.ldm % 2 == 0 && ((uintptr_t)x.M & 7) == 0 && (x.s + 63) / 64 <= 40;
  };
  std::vector<IdDesc> ord;
  ord.reserve(e.size());
  int bpair = 0, bsingle = 0, ssingle = 0;
  for (const auto& x : e)
    if (paired(x)) {
      ord.push_back(x);
      bpair = std::max(bpair, x.b);
    }
  const unsigned npair = (unsigned)ord.size();
  for (const auto& x : e)
    if (!paired(x)) {
      ord.push_back(x);
      bsingle = std::max(bsingle, x.b);
      ssingle = std::max(ssingle, x.s);
    }
  const unsigned nsingle = (unsigned)(ord.size() - npair);
  IdDesc* de = nullptr;
  RSRS_TRY(up.put_vec(ord, &de));
  const double esz = fp32 ? 4.0 : 8.0;
  double fstep = 0.0, bstep = 0.0;
  for (const auto& x : e) {
    fstep += 4.0 * x.b * x.s;
    bstep += 2.0 * esz * x.b * x.s;   // read and write every row
  }
  if (fp32) id_launch<float>(st, de, npair, nsingle, bpair, bsingle, kmax, ssingle, fstep, bstep);
  else id_launch<double>(st, de, npair, nsingle, bpair, bsingle, kmax, ssingle, fstep, bstep);
  {
    ProfScope ps(st, "id_finalize");
    hipLaunchKernelGGL(id_finalize_kernel, dim3((unsigned)ord.size()), dim3(256), 0, st, de);
  }
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}

// ---------------------------------------------------------------- Gram route
// For FP32 rows the greedy pivoted QR of M^T is taken as the pivoted
// Cholesky factorization of the FP64 Gram matrix G = M M^T: with
// d_i = |residual of row i|^2, step j takes the unselected row p of largest
// d_p, sets r_jj = sqrt(d_p) and, for every other unselected row i,
//   R[j, i] = (G_ip - sum_{t<j} R[t, i] R[t, p]) / r_jj,   d_i -= R[j, i]^2,
// which is the same R and the same pivots as the Gram-Schmidt form in exact
// arithmetic.  Its rounding (about sqrt(eps_64) of a row's norm once the
// residuals are small) stays below the FP32 rounding that M already
// carries, and d_i is clamped at zero.  The FP64 rows, their Gram matrix
// (FP64 MFMA) and one workgroup per box running all k steps replace the k
// launches of the Gram-Schmidt form; the R entries, pivots and selection
// marks it leaves are the ones id_finalize_kernel reads.

constexpr int kGramSplit = kIdGramSplit;   // partial Gram matrices per box (column ranges of the rows)
constexpr int kGramRows = 2048;            // largest b of the Gram route (the rows stay in registers)

// Row i in FP64 (M_Y + M_Z summed when MZ is set), and |[Y_B Z_B] row i|^2
// for a rank tolerance.
__global__ __launch_bounds__(64) void id_gram_rows_kernel(const IdDesc* __restrict__ e) {
  const IdDesc d = e[blockIdx.y];
  const int i = blockIdx.x;
  if (i >= d.b) return;
  const float* mi = static_cast<const float*>(d.M) + (int64_t)i * d.ldm;
  const float* mz = d.MZ ? static_cast<const float*>(d.MZ) + (int64_t)i * d.ldz : nullptr;
  double* out = d.Md + (int64_t)i * d.ldmd;
  for (int c = threadIdx.x; c < d.s; c += 64) {
    float v = mi[c];
    if (mz) v = (float)((double)v + (double)mz[c]);   // the sum as the Gram-Schmidt form stores it
    out[c] = (double)v;
  }
  if (threadIdx.x == 0) d.sel[i] = INT_MAX;
  if (d.tol2 > 0.0) {
    const int64_t gi = d.idx[i];
    const float* yr = static_cast<const float*>(d.Yg) + gi * d.ldy;
    const float* zr = d.Zg ? static_cast<const float*>(d.Zg) + gi * d.ldy : nullptr;
    double q = 0.0;
    for (int c = threadIdx.x; c < d.sy; c += 64) {
      const double y = (double)yr[c];
      q += y * y;
      if (zr) {
        const double z = (double)zr[c];
        q += z * z;
      }
    }
    q = wave_sum(q);
    if (threadIdx.x == 0) d.rowyz[i] = q;
  }
}

// All k steps of one box: 1024 threads, rows strided over the threads.  The
// Gram matrix arrives as NG full partial sums over column ranges of the
// rows (G = sum_q G_q, each b x ldg, NG apart by gstride), added here in a
// fixed order; its symmetry lets row p stand for column p, so each step
// reads the pivot's row, contiguous across the threads.  The R entries are
// kept twice: row-major in Rc (what the finalisation reads) and
// column-major in Rt (b apart), where the dot product of step j reads
// entry t of every row at consecutive addresses.  One barrier per step:
// after it every thread reduces the 16 wave maxima itself, so all agree on
// the pivot without a second exchange.
// With LDSR the column-major R entries live in LDS (b k <= kRtLds), else in
// the global scratch: the same arithmetic in the same order either way.
constexpr int kRtLds = 16384;
template <int NG, bool LDSR>
__global__ __launch_bounds__(1024) void id_pchol_kernel(const IdDesc* __restrict__ e, int64_t gstride) {
  const IdDesc d = e[blockIdx.x];
  const gptr<const double> G = to_global(d.G);
  const gptr<double> Rc = to_global(d.Rc);
  const gptr<int> sel = to_global(d.sel), piv = to_global(d.piv);
  const int b = d.b, k = d.k, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int RPT = kGramRows / 1024;   // rows per thread
  __shared__ double wbest[2][16];
  __shared__ int wrow[2][16];
  __shared__ double RtL[LDSR ? kRtLds : 1];
  double* Rt = LDSR ? RtL : d.Rt;
  double dv[RPT];
  int alive = 0;   // bit u: row tid + 1024 u still unselected
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int i = tid + 1024 * u;
    dv[u] = 0.0;
    if (i < b) {
      double g = 0.0;
#pragma unroll
      for (int q = 0; q < NG; ++q) g += G[(int64_t)i * d.ldg + i + q * gstride];
      dv[u] = g > 0.0 ? g : 0.0;
      alive |= 1 << u;
    }
  }
  for (int j = 0; j < k; ++j) {
    // this thread's candidates, then the wave's (lowest index on ties)
    double best = -1.0;
    int bi = INT_MAX;
#pragma unroll
    for (int u = 0; u < RPT; ++u)
      if (((alive >> u) & 1) && dv[u] > best) {
        best = dv[u];
        bi = tid + 1024 * u;
      }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      const bool take = oi != INT_MAX && (bi == INT_MAX || ob > best || (ob == best && oi < bi));
      best = take ? ob : best;
      bi = take ? oi : bi;
    }
    // double-buffered by step parity: a fast wave of the next step cannot
    // overwrite what a slow one still reads
    if (lane == 0) {
      wbest[j & 1][wave] = best;
      wrow[j & 1][wave] = bi;
    }
    __syncthreads();
    double bb = -1.0;
    int p = INT_MAX;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      const int oi = wrow[j & 1][w];
      const double ob = wbest[j & 1][w];
      if (oi != INT_MAX && (p == INT_MAX || ob > bb || (ob == bb && oi < p))) {
        bb = ob;
        p = oi;
      }
    }
    // j < k <= b rows remain, so p is a row
    const double rjj = sqrt(bb > 0.0 ? bb : 0.0);
    const gptr<const double> gp = G + (int64_t)p * d.ldg;
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      if (!((alive >> u) & 1)) continue;
      const int i = tid + 1024 * u;
      if (i == p) {
        alive &= ~(1 << u);
        sel[p] = j;
        piv[j] = p;
        Rc[(int64_t)p * k + j] = rjj;
        Rt[(int64_t)j * b + p] = rjj;
        continue;
      }
      // the pivot row's entries t < j were written in earlier steps, before
      // this step's barrier
      double c = 0.0;
#pragma unroll
      for (int q = 0; q < NG; ++q) c += gp[i + q * gstride];
      double c1 = 0.0, c2 = 0.0;
      int t = 0;
      for (; t + 1 < j; t += 2) {
        c1 += Rt[(int64_t)t * b + i] * Rt[(int64_t)t * b + p];
        c2 += Rt[(int64_t)(t + 1) * b + i] * Rt[(int64_t)(t + 1) * b + p];
      }
      if (t < j) c1 += Rt[(int64_t)t * b + i] * Rt[(int64_t)t * b + p];
      c -= c1 + c2;
      const double l = rjj > 0.0 ? c / rjj : 0.0;
      Rc[(int64_t)i * k + j] = l;
      Rt[(int64_t)j * b + i] = l;
      const double nd = dv[u] - l * l;
      dv[u] = nd > 0.0 ? nd : 0.0;
    }
  }
}

rsrs_status id_run_gram(Uploader& up, hipStream_t st, const std::vector<IdDesc>& all) {
  if (all.empty()) return RSRS_OK;
  // boxes with more rows than the Gram route holds take the Gram-Schmidt
  // form (a box's route depends on its own size only)
  std::vector<IdDesc> e, big;
  for (const auto& x : all) (x.b <= kGramRows ? e : big).push_back(x);
  if (!big.empty()) RSRS_TRY(id_run(up, st, big, true));
  if (e.empty()) return RSRS_OK;
  int bmax = 0;
  for (const auto& x : e) {
    if (x.k > 256 || x.k > x.b || x.k < 1 || !x.Md || !x.G || !x.Rt) {
      set_error("ID (Gram route) sizes out of range (need 1 <= k <= b, k <= 256)");
      return RSRS_E_UNSUPPORTED;
    }
    bmax = std::max(bmax, x.b);
  }
  IdDesc* de = nullptr;
  RSRS_TRY(up.put_vec(e, &de));
  const unsigned nb = (unsigned)e.size();
  double rbytes = 0.0;
  for (const auto& x : e) rbytes += 12.0 * x.b * x.s;
  {
    ProfScope ps(st, "id_gram_rows", 0.0, rbytes);
    hipLaunchKernelGGL(id_gram_rows_kernel, dim3((unsigned)bmax, nb), dim3(64), 0, st, de);
    RSRS_HIP(hipGetLastError());
  }
  // the Gram matrices as kGramSplit partial sums over column ranges (a long
  // K and few output tiles per box: the split keeps the chip busy); every
  // box's split depends on its own sizes only
  std::vector<GemmDesc> g;
  for (const auto& x : e) {
    const int step = (int)round_up((x.s + kGramSplit - 1) / kGramSplit, 16);
    for (int q = 0; q < kGramSplit; ++q) {
      const int c0 = std::min(x.s, q * step), c1 = std::min(x.s, (q + 1) * step);
      g.push_back(gdesc(x.Md + c0, nullptr, x.ldmd, x.Md + c0, nullptr, x.ldmd, x.G + q * x.b * x.ldg, nullptr,
                        x.ldg, x.b, x.b, c1 - c0));
    }
  }
  // both triangles: the pivot's column is then read as its row
  RSRS_TRY(gemm(up, st, g, 0, 1, GM_FULL, GS_64x64, "id_gram"));
  {
    double f = 0.0;
    for (const auto& x : e) f += 2.0 * x.b * x.k * x.k;
    ProfScope ps(st, "id_pchol", f, 0.0);
    // partial sums of box x lie b * ldg apart: one stride per launch needs
    // equal (b, ldg), so boxes are launched in groups of equal stride (and of
    // R entries in LDS or not)
    std::vector<std::pair<std::pair<int64_t, bool>, std::vector<IdDesc>>> groups;
    for (const auto& x : e) {
      const std::pair<int64_t, bool> key{(int64_t)x.b * x.ldg, (int64_t)x.b * x.k <= kRtLds};
      auto it = std::find_if(groups.begin(), groups.end(), [&](const auto& gr) { return gr.first == key; });
      if (it == groups.end()) groups.push_back({key, {x}});
      else it->second.push_back(x);
    }
    for (const auto& gr : groups) {
      IdDesc* dg = nullptr;
      RSRS_TRY(up.put_vec(gr.second, &dg));
      if (gr.first.second)
        hipLaunchKernelGGL((id_pchol_kernel<kGramSplit, true>), dim3((unsigned)gr.second.size()), dim3(1024), 0, st,
                           dg, gr.first.first);
      else
        hipLaunchKernelGGL((id_pchol_kernel<kGramSplit, false>), dim3((unsigned)gr.second.size()), dim3(1024), 0,
                           st, dg, gr.first.first);
      RSRS_HIP(hipGetLastError());
    }
  }
  {
    ProfScope ps(st, "id_finalize");
    hipLaunchKernelGGL(id_finalize_kernel, dim3(nb), dim3(256), 0, st, de);
    RSRS_HIP(hipGetLastError());
  }
  return RSRS_OK;
}

// ---------------------------------------------------------------- column fix-up
// Xp[i][c] for output columns [R, S, N]:
//   c <  r      : XR[i][Rpos[c]] - sum_t XR[i][Spos[t]] T[c][t]
//   c <  r + k  : XR[i][Spos[c - r]]
//   otherwise   : XR[i][b + c - r - k]
template <typename T>
__global__ __launch_bounds__(256) void colfix_kernel(const ColfixDescT<T>* __restrict__ e) {
  const ColfixDescT<T> d = e[blockIdx.y];
  const int i = blockIdx.x;
  if (i >= d.r) return;
  __shared__ T xs[256];
  const T* xr = d.XR + (int64_t)i * d.ldx;
  for (int t = threadIdx.x; t < d.k; t += 256) xs[t] = xr[d.Spos[t]];
  __syncthreads();
  T* out = d.Xp + (int64_t)i * d.ldp;
  for (int c = threadIdx.x; c < d.l; c += 256) {
    T v;
    if (c < d.r) {
      v = xr[d.Rpos[c]];
      const T* tc = d.T_ + (int64_t)c * d.ldt;
      for (int t = 0; t < d.k; ++t) v -= xs[t] * tc[t];
    } else if (c < d.r + d.k) {
      v = xs[c - d.r];
    } else {
      v = xr[d.b + (c - d.r - d.k)];
    }
    out[c] = v;
  }
}

template <typename T>
rsrs_status colfix(Uploader& up, hipStream_t st, const std::vector<ColfixDescT<T>>& e) {
  if (e.empty()) return RSRS_OK;
  int rmax = 0;
  for (const auto& x : e) {
    if (x.k > 256) {
      set_error("colfix: k > 256");
      return RSRS_E_UNSUPPORTED;
    }
    rmax = std::max(rmax, x.r);
  }
  if (rmax == 0) return RSRS_OK;
  ColfixDescT<T>* de = nullptr;
  RSRS_TRY(up.put_vec(e, &de));
  ProfScope ps(st, "colfix");
  hipLaunchKernelGGL((colfix_kernel<T>), dim3((unsigned)rmax, (unsigned)e.size()), dim3(256), 0, st, de);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}
template rsrs_status colfix<double>(Uploader&, hipStream_t, const std::vector<ColfixDescT<double>>&);
template rsrs_status colfix<float>(Uploader&, hipStream_t, const std::vector<ColfixDescT<float>>&);

}  // namespace rsrs
