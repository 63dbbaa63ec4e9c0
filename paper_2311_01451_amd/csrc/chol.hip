// Batched Cholesky factorization G = L L^T with the inverse factor L^{-1}
// (the Gram matrices of the nullification step, eq. nullYZ, are factored so
// that C^T G^{-1} becomes two triangular products).
//
// Right-looking by panels of 64 columns with the trailing update deferred
// over super-panels of four panels:
//
//   column j  (panels after the first of a super-panel) the column block j
//             receives the earlier panels of its super-panel: a narrow GEMM
//             launch in FP64; in FP32 the panel kernel's workgroups subtract
//             them from their own blocks first (one more LDS block fits).
//   panel j   one workgroup per (matrix, two 64-row blocks i >= j).  Each
//             workgroup factors the diagonal block G_jj itself (so no
//             workgroup waits for another), forms X_jj = L_jj^{-1}, and
//             computes its blocks L_ij = G_ij X_jj^T; the workgroup holding
//             i = j stores X_jj.
//   trailing  after the last panel of a super-panel, G_22 -= L_21 L_21^T on
//             the trailing lower triangle with the super-panel's 256 columns
//             (batched SYRK on the MFMA GEMM).
//
// Inside a panel the 64 x 64 diagonal block is factored in eight steps of
// 8 columns: the 64 lanes of one wave (one per row) each factor the 8 x 8
// diagonal block in registers (reciprocal square roots by the hardware
// estimate and Newton steps), rows below form their entries of L by
// forward substitution and rows inside the block their row of its inverse,
// then the waves apply the rank-8 update on MFMA; two barriers per
// step.  The
// inverse of the 64 x 64 factor follows from the 8 x 8 ones by doubling,
//   [A 0; C D]^{-1} = [A^{-1} 0; -D^{-1} C A^{-1}  D^{-1}],
// and the off-diagonal blocks are G_ij X_jj^T on MFMA, the next block's
// loads in flight during each product.  No global read of a panel launch
// depends on its own arithmetic, so the diagonal block, the first row block
// and the first pending panel are requested together at the start (raw buffer
// loads, whose range check zero-fills the rows past a partial block), and
// each further pending panel is fetched while the previous one is multiplied.
//
// Element type T = double (FP64 MFMA) or float (FP32 MFMA, FP32
// accumulation; the Gram matrices of the FP32 path are formed in FP32, so
// their factorization in FP32 adds a backward error of the same order).
//
// After the panels, L^{-1} of the whole matrix is assembled by the same
// doubling on 64 * 2^t blocks with batched GEMMs (log2(n / 64) levels, two
// launches each); the result overwrites G, the factor blocks L_ij having been
// stored in G's lower part and the diagonal inverses in the scratch matrix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "kernels.hpp"
#include "profile.hpp"

namespace rsrs {

namespace {

// Raw buffer view of `bytes` bytes from a wave-uniform base: loads at byte
// offsets beyond the range return zero (the hardware's range check), so a
// partial block is read without branches or clamped addresses.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_view(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, bytes, 0x00020000);
}
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, float, int off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, double, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

constexpr int PB = 64;        // panel width
constexpr int PP = PB + 1;    // LDS row pitch (elements)
constexpr int RB = 2;         // row blocks per workgroup

template <typename T>
struct CholPanel {
  T* G;   // the matrix (lower part); receives L_ij, i > j
  T* X;   // scratch of the same shape; receives X_jj
  int64_t ld;
  int n, j, ib, ie;   // panel j, row blocks [ib, ie)
  int t0;             // panels t0..j-1 still to subtract from column block j (FUSED)
};

// acc += A B^T for 64 x 64 blocks in LDS (pitch PP), wave w holding rows
// 32 (w / 2).., columns 32 (w % 2)..: the layout of every product below.
template <typename T>
__device__ __forceinline__ void mma_abt(const T* A, const T* B, typename Mfma<T>::acc_t (&acc)[2][2], int wm,
                                        int wn, int q, int c16) {
#pragma unroll 4
  for (int k0 = 0; k0 < PB; k0 += 4) {
    T av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = A[(32 * wm + 16 * a + c16) * PP + k0 + q];
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) bv[bb] = B[(32 * wn + 16 * bb + c16) * PP + k0 + q];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int bb = 0; bb < 2; ++bb) acc[a][bb] = Mfma<T>::mma(av[a], bv[bb], acc[a][bb]);
  }
}

// La[r][c] -= acc at the wave's result positions, rows below `rows` only
// (lower part only when `lower`)
template <typename T>
__device__ __forceinline__ void sub_acc(T* La, const typename Mfma<T>::acc_t (&acc)[2][2], int rows, bool lower,
                                        int wm, int wn, int q, int c16) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 32 * wm + 16 * a + Mfma<T>::row(v, q), c = 32 * wn + 16 * bb + c16;
        if (r < rows && (!lower || c <= r)) La[r * PP + c] -= acc[a][bb][v];
      }
}

// 1 / sqrt(d) from the hardware estimate and Newton steps
// y <- y + y (1 - d y^2) / 2 (each step doubles the correct bits): two from
// the FP64 estimate, one from the FP32 one (good to about one ulp).
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-(d * y), y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}
__device__ __forceinline__ float rsqrt_nr(float d) {
  float y = __builtin_amdgcn_rsqf(d);
  const float e = fmaf(-(d * y), y, 1.0f);
  return fmaf(0.5f * y, e, y);
}

// One doubling step of the in-block inverse for h = 8 or 16 (64 / (2h)
// pairs of h-blocks), one output per thread and pass.
template <typename T, int H>
__device__ __forceinline__ void doubling_small(const T* La, T* Xa, T* Vs, int tid) {
  constexpr int NP = PB / (2 * H), TOT = NP * H * H;
#pragma unroll
  for (int x0 = 0; x0 < TOT; x0 += 256) {
    const int x = x0 + tid;
    const int p = x / (H * H), dd = (x / H) % H, aa = x % H;
    const int A0 = 2 * H * p, D0 = A0 + H;
    T acc = 0;
#pragma unroll
    for (int t = 0; t < H; ++t) acc = fma(La[(D0 + dd) * PP + A0 + t], Xa[(A0 + t) * PP + A0 + aa], acc);
    Vs[x] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int x0 = 0; x0 < TOT; x0 += 256) {
    const int x = x0 + tid;
    const int p = x / (H * H), dd = (x / H) % H, aa = x % H;
    const int A0 = 2 * H * p, D0 = A0 + H;
    T acc = 0;
#pragma unroll
    for (int t = 0; t < H; ++t) acc = fma(Xa[(D0 + dd) * PP + D0 + t], Vs[p * H * H + t * H + aa], acc);
    Xa[(D0 + dd) * PP + A0 + aa] = -acc;
  }
  __syncthreads();
}

// FUSED: the workgroup first subtracts the earlier panels t0..j-1 of the
// super-panel from its blocks of column block j (diagonal block and its row
// blocks), L_it L_jt^T on MFMA with the results kept in registers, instead
// of a separate narrow GEMM launch before the panel.
template <typename T, bool FUSED>
__global__ __launch_bounds__(256, 2) void chol_panel_kernel(const CholPanel<T>* __restrict__ e, int* flag) {
  using MM = Mfma<T>;
  using acc_t = typename MM::acc_t;
  __shared__ T La[PB * PP];   // diagonal block -> L_jj; later the off-diagonal blocks
  __shared__ T Xa[PB * PP];   // X_jj = L_jj^{-1}
  __shared__ T Vs[32 * 33];   // products of the doubling steps
  __shared__ T Lj[FUSED ? PB * PP : 1];   // L_jt of the pending panels
  __shared__ T Pa[FUSED ? PB * PP : 1];   // the first row block of the products
  const CholPanel<T> d = e[blockIdx.x];
  const gptr<T> G = to_global(d.G);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t ld = d.ld;
  const int ldi = (int)d.ld;   // offsets inside one 64-row block fit in 32 bits
  const int j0 = PB * d.j;
  const int nj = min(PB, d.n - j0);
  const int wm = wave >> 1, wn = wave & 1, q = lane >> 4, c16 = lane & 15;
  const int ifirst = max(d.ib, d.j + 1);
  acc_t ad[2][2], ao[RB][2][2];   // pending updates of the diagonal and the row blocks
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      ad[a][bb] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int b = 0; b < RB; ++b) ao[b][a][bb] = acc_t{0, 0, 0, 0};
    }
  // Every global read of the launch is independent of its arithmetic (the
  // pending updates are applied from registers after the loads), so the
  // diagonal block, the first row block of the products and the first pending
  // panel's three blocks are all requested up front, and each later pending
  // panel is fetched while the previous one is multiplied.
  const T* gd = d.G + (int64_t)j0 * ld + j0;
  T vd[16], pf[16];
  const int nrb = max(0, min(RB, d.ie - ifirst));
  // thread tid reads row tid / 64 + 4 u, column tid % 64 of a block
  const int voff = ((tid >> 6) * ldi + (tid & 63)) * (int)sizeof(T), vstep = 4 * ldi * (int)sizeof(T);
  auto ldregs = [&](T (&v)[16], const T* src, int rows) {
    const auto rs = buf_view(src, ((rows - 1) * ldi + PB) * (int)sizeof(T));
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = buf_ld(rs, T(0), voff + u * vstep);
  };
  auto stregs = [&](T* dst, const T (&v)[16]) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int x = tid + 256 * u;
      dst[(x >> 6) * PP + (x & 63)] = v[u];
    }
  };
  auto fetch = [&](int ib) {
    const int ni = min(PB, d.n - PB * ib);
    ldregs(pf, d.G + (int64_t)PB * ib * ld + j0, ni);
  };
  if constexpr (FUSED) {
    T nx[1 + RB][16];
    const int t0 = d.t0;
    if (t0 < d.j) {
      ldregs(nx[0], d.G + (int64_t)j0 * ld + PB * t0, nj);
#pragma unroll
      for (int b = 0; b < RB; ++b)
        if (b < nrb) ldregs(nx[1 + b], d.G + (int64_t)PB * (ifirst + b) * ld + PB * t0, min(PB, d.n - PB * (ifirst + b)));
    }
    {
      const auto rs = buf_view(gd, ((nj - 1) * ldi + nj) * (int)sizeof(T));
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int x = tid + 256 * u, r = x >> 6, c = x & 63;
        const T g = buf_ld(rs, T(0), voff + u * vstep);
        vd[u] = (r < nj && c <= r) ? g : T((r == c) ? 1 : 0);
      }
    }
    if (nrb > 0) fetch(ifirst);
    for (int t = t0; t < d.j; ++t) {
      stregs(Lj, nx[0]);
      if (nrb > 0) stregs(La, nx[1]);
      if (nrb > 1) stregs(Xa, nx[2]);
      __syncthreads();
      if (t + 1 < d.j) {
        ldregs(nx[0], d.G + (int64_t)j0 * ld + PB * (t + 1), nj);
#pragma unroll
        for (int b = 0; b < RB; ++b)
          if (b < nrb)
            ldregs(nx[1 + b], d.G + (int64_t)PB * (ifirst + b) * ld + PB * (t + 1), min(PB, d.n - PB * (ifirst + b)));
      }
      mma_abt(Lj, Lj, ad, wm, wn, q, c16);
      if (nrb > 0) mma_abt(La, Lj, ao[0], wm, wn, q, c16);
      if (nrb > 1) mma_abt(Xa, Lj, ao[1], wm, wn, q, c16);
      __syncthreads();
    }
  } else {
    {
      const auto rs = buf_view(gd, ((nj - 1) * ldi + nj) * (int)sizeof(T));
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int x = tid + 256 * u, r = x >> 6, c = x & 63;
        const T g = buf_ld(rs, T(0), voff + u * vstep);
        vd[u] = (r < nj && c <= r) ? g : T((r == c) ? 1 : 0);
      }
    }
  }
  // lower part of the diagonal block, identity beyond n, zero above
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int x = tid + 256 * u;
    La[(x >> 6) * PP + (x & 63)] = vd[u];
    if ((x & 63) > (x >> 6)) Xa[(x >> 6) * PP + (x & 63)] = T(0);   // Xa stays zero above the diagonal
  }
  if constexpr (FUSED) {
    if (nrb > 0) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int x = tid + 256 * u;
        Pa[(x >> 6) * PP + (x & 63)] = pf[u];
      }
    }
  }
  __syncthreads();
  if constexpr (FUSED) {
    if (d.t0 < d.j) {
      sub_acc(La, ad, nj, true, wm, wn, q, c16);
      if (nrb > 0) sub_acc(Pa, ao[0], min(PB, d.n - PB * ifirst), false, wm, wn, q, c16);
      __syncthreads();
    }
  }
  // ---- factorization in steps of 8 columns.  Wave 0, lane r = row r: every
  // lane factors the 8 x 8 diagonal block in registers (identical work, no
  // exchange), then rows below form their 8 entries of L and rows inside the
  // block their row of the block's inverse; all waves apply the rank-8 update.
  bool bad = false;
#pragma unroll 1
  for (int s = 0; s < 8; ++s) {
    const int b = 8 * s;
    if (wave == 0) {
      T D[8][8];
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int k = 0; k <= i; ++k) D[i][k] = La[(b + i) * PP + b + k];
      T y[8];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        T dd = D[jj][jj];
        if (!(dd > T(0))) {   // same in every lane
          bad = true;
          dd = T(1);
        }
        const T yy = rsqrt_nr(dd);
        y[jj] = yy;
        D[jj][jj] = dd * yy;
#pragma unroll
        for (int i = jj + 1; i < 8; ++i) D[i][jj] *= yy;
#pragma unroll
        for (int k = jj + 1; k < 8; ++k)
#pragma unroll
          for (int i = k; i < 8; ++i) D[i][k] = fma(-D[i][jj], D[k][jj], D[i][k]);
      }
      const int r = lane;
      if (r >= b + 8) {
        // l = a L_bb^{-T} by forward substitution
        T l[8];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
          T acc = La[r * PP + b + jj];
#pragma unroll
          for (int k = 0; k < jj; ++k) acc = fma(-l[k], D[jj][k], acc);
          l[jj] = acc * y[jj];
        }
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) La[r * PP + b + jj] = l[jj];
      } else if (r >= b) {
        // row i of L_bb^{-1}: x L_bb = e_i, from the last column back
        const int i = r - b;
        T x[8];
#pragma unroll
        for (int jj = 7; jj >= 0; --jj) {
          T acc = T((jj == i) ? 1 : 0);
#pragma unroll
          for (int k = jj + 1; k < 8; ++k) acc = fma(-x[k], D[k][jj], acc);
          x[jj] = acc * y[jj];
        }
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) Xa[r * PP + b + jj] = x[jj];
      }
    }
    __syncthreads();
    {
      // rank-8 update of rows and columns >= b + 8 (lower part) on MFMA:
      // the 16 x 16 tiles meeting that region, round-robin over the waves;
      // tile rows above b + 8 read the diagonal block's rows and are masked
      const int q4 = lane >> 4, c16 = lane & 15;
      const int t0 = (b + 8) >> 4;
      int idx = 0;
      for (int ti = t0; ti < 4; ++ti)
        for (int tj = t0; tj <= ti; ++tj, ++idx) {
          if ((idx & 3) != wave) continue;
          acc_t acc = acc_t{0, 0, 0, 0};
#pragma unroll
          for (int k0 = 0; k0 < 8; k0 += 4)
            acc = MM::mma(La[(16 * ti + c16) * PP + b + k0 + q4], La[(16 * tj + c16) * PP + b + k0 + q4], acc);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * ti + MM::row(v, q4), c = 16 * tj + c16;
            if (c >= b + 8 && c <= r) La[r * PP + c] -= acc[v];
          }
        }
    }
    __syncthreads();
  }
  // ---- inverse of the 64 x 64 factor from the 8 x 8 ones by doubling: for
  // the pair (A, D) of h-blocks, V = C X_AA into Vs, then X_DA = -X_DD V.
  // The upper part of Xa is zero, so every product runs over full blocks.
  doubling_small<T, 8>(La, Xa, Vs, tid);
  doubling_small<T, 16>(La, Xa, Vs, tid);
  {
    // h = 32 on MFMA, wave w: the 16 x 16 tile (w / 2, w % 2)
    const int tm = wave >> 1, tn = wave & 1, q = lane >> 4, c16 = lane & 15;
    acc_t acc = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < 32; k0 += 4)
      acc = MM::mma(La[(32 + 16 * tm + c16) * PP + k0 + q], Xa[(k0 + q) * PP + 16 * tn + c16], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) Vs[(16 * tm + MM::row(v, q)) * 33 + 16 * tn + c16] = acc[v];
    __syncthreads();
    acc = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < 32; k0 += 4)
      acc = MM::mma(Xa[(32 + 16 * tm + c16) * PP + 32 + k0 + q], Vs[(k0 + q) * 33 + 16 * tn + c16], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) Xa[(32 + 16 * tm + MM::row(v, q)) * PP + 16 * tn + c16] = -acc[v];
    __syncthreads();
  }
  if (d.ib == d.j) {
    gptr<T> xo = to_global(d.X) + (int64_t)j0 * ld + j0;
    for (int x = tid; x < PB * PB; x += 256) {
      const int r = x >> 6, c = x & 63;
      if (r < nj && c < nj) xo[(int64_t)r * ld + c] = Xa[r * PP + c];
    }
    if (bad && tid == 0) atomicOr(flag, 1);
  }
  // ---- off-diagonal blocks L_ij = G_ij X_jj^T (panel j is full here) on
  // MFMA: wave w computes rows 32 (w / 2).., columns 32 (w % 2)..
  if constexpr (!FUSED) {
    if (ifirst < d.ie) fetch(ifirst);
  }
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const int i = ifirst + b;
    if (i >= d.ie) break;   // the same in every thread
    const int i0 = PB * i;
    const int ni = min(PB, d.n - i0);
    gptr<T> gi = G + (int64_t)i0 * ld + j0;
    // FP32: the first row block already sits in Pa with its pending update
    const bool inpa = FUSED && b == 0;
    if (!inpa) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int x = tid + 256 * u;
        La[(x >> 6) * PP + (x & 63)] = pf[u];
      }
      __syncthreads();
      if constexpr (FUSED) {
        if (d.t0 < d.j) {
          sub_acc(La, ao[b], ni, false, wm, wn, q, c16);
          __syncthreads();
        }
      }
    }
    if (i + 1 < d.ie) fetch(i + 1);   // in flight during the product
    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int bb = 0; bb < 2; ++bb) acc[a][bb] = acc_t{0, 0, 0, 0};
    mma_abt(inpa ? Pa : La, Xa, acc, wm, wn, q, c16);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 32 * wm + 16 * a + MM::row(v, q);
        if (r < ni) {
#pragma unroll
          for (int bb = 0; bb < 2; ++bb) gi[(int64_t)r * ld + 32 * wn + 16 * bb + c16] = acc[a][bb][v];
        }
      }
    __syncthreads();
  }
}

}  // namespace

template <typename T>
rsrs_status chol_inverse(Uploader& up, hipStream_t st, const std::vector<CholMatT<T>>& mats, int* flag) {
  using GD = GemmDescT<T, T>;
  int nmax = 0;
  for (const auto& m : mats) nmax = std::max(nmax, m.n);
  if (nmax <= 0) return RSRS_OK;
  const int P = (nmax + PB - 1) / PB;
  // ---- every launch's descriptors, built up front and uploaded together.
  // Trailing updates are deferred over super-panels of SP panels: before
  // panel j only its own column block receives the earlier panels of the
  // super-panel (a narrow GEMM), and after the last panel of a super-panel
  // the trailing matrix receives all of them at once (a SYRK with K = 64 SP),
  // which reads and writes the trailing matrix SP times less often.
  constexpr int SP = 4;
  // FP32: the column-block update is done by the panel kernel itself (its
  // extra LDS block keeps two workgroups per CU only at 4-byte elements)
  constexpr bool fused = sizeof(T) == 4;
  std::vector<CholPanel<T>> tasks;
  std::vector<size_t> toff(P + 1);
  std::vector<double> pflops(P, 0.0);
  std::vector<GD> colu, trail;
  std::vector<size_t> coff(P + 1), soff(P + 1);
  for (int j = 0; j < P; ++j) {
    const int j0s = SP * (j / SP);
    const bool last_of_sp = (j % SP == SP - 1);
    toff[j] = tasks.size();
    coff[j] = colu.size();
    soff[j] = trail.size();
    for (const auto& m : mats) {
      const int Pm = (m.n + PB - 1) / PB;
      if (j >= Pm) continue;
      const int rows = m.n - PB * j;
      if (j > j0s && !fused) {
        // column block j -= L[rows >= 64 j, panels j0s..j-1] L[block j, same]^T
        T* Lr = m.G + (int64_t)PB * j * m.ld + PB * j0s;
        T* Cj = m.G + (int64_t)PB * j * (m.ld + 1);
        colu.push_back(gdescT<T, T>(Lr, nullptr, m.ld, Lr, nullptr, m.ld, Cj, nullptr, m.ld, rows,
                             std::min(PB, rows), PB * (j - j0s), -1.0, 1.0));
      }
      for (int ib = j; ib < Pm; ib += RB)
        tasks.push_back(CholPanel<T>{m.G, m.W, m.ld, m.n, j, ib, std::min(ib + RB, Pm), fused ? j0s : j});
      const double nj = std::min(PB, rows), below = rows - nj;
      pflops[j] += (2.0 / 3.0) * nj * nj * nj + below * nj * nj;
      if (fused) pflops[j] += 2.0 * rows * nj * PB * (j - j0s);   // the column-block update
      const int trows = m.n - PB * (j + 1);
      if (trows > 0 && (last_of_sp || j == Pm - 1)) {
        T* Ls = m.G + (int64_t)PB * (j + 1) * m.ld + PB * j0s;
        T* G22 = m.G + (int64_t)PB * (j + 1) * (m.ld + 1);
        trail.push_back(gdescT<T, T>(Ls, nullptr, m.ld, Ls, nullptr, m.ld, G22, nullptr, m.ld, trows, trows,
                              PB * (j + 1 - j0s), -1.0, 1.0));
      }
    }
  }
  toff[P] = tasks.size();
  coff[P] = colu.size();
  soff[P] = trail.size();
  std::vector<std::vector<GemmLaunch>> cl(P), tl(P);
  for (int j = 0; j < P; ++j) {
    if (coff[j + 1] > coff[j]) {
      std::vector<GD> part(colu.begin() + coff[j], colu.begin() + coff[j + 1]);
      RSRS_TRY(gemm_plan<T, T>(part, coff[j], 0, 1, GM_FULL, GS_64x64_ONLY, "chol", cl[j]));
    }
    if (soff[j + 1] > soff[j]) {
      std::vector<GD> part(trail.begin() + soff[j], trail.begin() + soff[j + 1]);
      RSRS_TRY(gemm_plan<T, T>(part, soff[j], 0, 1, GM_SYRK_L, GS_64x64, "chol", tl[j]));
    }
  }
  // diagonal inverses into G, then the doubling levels
  std::vector<Copy2DT<T, T>> diag;
  for (const auto& m : mats)
    for (int j0 = 0; j0 < m.n; j0 += PB) {
      const int nj = std::min(PB, m.n - j0);
      diag.push_back(Copy2DT<T, T>{m.W + (int64_t)j0 * (m.ld + 1), m.G + (int64_t)j0 * (m.ld + 1), m.ld, m.ld, nj, nj,
                            1.0, 0, 0});
    }
  std::vector<GD> inv;
  std::vector<std::vector<GemmLaunch>> il;
  for (int h = PB; h < nmax; h *= 2) {
    std::vector<GD> v, x;
    for (const auto& m : mats)
      for (int a0 = 0; a0 + h < m.n; a0 += 2 * h) {
        const int D0 = a0 + h, nd = std::min(h, m.n - D0);
        T* XDD = m.G + (int64_t)D0 * (m.ld + 1);
        T* C = m.G + (int64_t)D0 * m.ld + a0;
        T* V = m.W + (int64_t)D0 * m.ld + a0;
        T* XAA = m.G + (int64_t)a0 * (m.ld + 1);
        // V = X_DD C (X_DD lower), then X_DA = -V X_AA (X_AA lower) over C
        v.push_back(gdescT<T, T>(XDD, nullptr, m.ld, C, nullptr, m.ld, V, nullptr, m.ld, nd, h, nd));
        x.push_back(gdescT<T, T>(V, nullptr, m.ld, XAA, nullptr, m.ld, C, nullptr, m.ld, nd, h, h, -1.0, 0.0));
      }
    if (v.empty()) continue;
    il.emplace_back();
    RSRS_TRY(gemm_plan<T, T>(v, inv.size(), 0, 0, GM_A_LOW, GS_64x64, "cholinv", il.back()));
    inv.insert(inv.end(), v.begin(), v.end());
    il.emplace_back();
    RSRS_TRY(gemm_plan<T, T>(x, inv.size(), 0, 0, GM_B_NN_LOW, GS_64x64, "cholinv", il.back()));
    inv.insert(inv.end(), x.begin(), x.end());
  }
  CholPanel<T>* dt = nullptr;
  GD* dc = nullptr;
  GD* ds = nullptr;
  GD* di = nullptr;
  RSRS_TRY(up.put_vec(tasks, &dt));
  if (!colu.empty()) RSRS_TRY(up.put_vec(colu, &dc));
  if (!trail.empty()) RSRS_TRY(up.put_vec(trail, &ds));
  if (!inv.empty()) RSRS_TRY(up.put_vec(inv, &di));
  // ---- launches
  for (int j = 0; j < P; ++j) {
    for (const auto& L : cl[j]) RSRS_TRY(gemm_exec(L, dc, sizeof(GD), st));
    const unsigned nt = (unsigned)(toff[j + 1] - toff[j]);
    {
      ProfScope ps(st, sizeof(T) == 4 ? "chol32_panel" : "chol_panel", pflops[j], 0.0);
      hipLaunchKernelGGL((chol_panel_kernel<T, fused>), dim3(nt), dim3(256), 0, st, dt + toff[j], flag);
      RSRS_HIP(hipGetLastError());
    }
    for (const auto& L : tl[j]) RSRS_TRY(gemm_exec(L, ds, sizeof(GD), st));
  }
  RSRS_TRY(copy2d<T, T>(up, st, diag));
  for (const auto& lv : il)
    for (const auto& L : lv) RSRS_TRY(gemm_exec(L, di, sizeof(GD), st));
  return RSRS_OK;
}

template rsrs_status chol_inverse<double>(Uploader&, hipStream_t, const std::vector<CholMatT<double>>&, int*);
template rsrs_status chol_inverse<float>(Uploader&, hipStream_t, const std::vector<CholMatT<float>>&, int*);

}  // namespace rsrs
