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
#include <hip/hip_runtime.h>

#include <algorithm>

#include "impl.hpp"

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

template <typename T>
rsrs_status apply_t(const rsrs_factor_t* F, int op, int transpose, int64_t w, const double* Fin,
                    int64_t ldf, double* Uout, int64_t ldu, hipStream_t st) {
  using GD = GemmDescT<T, T>;
  auto gdesc = [](const T* A, const int64_t* ia, int64_t lda, const T* B, const int64_t* ib,
                  int64_t ldb, T* C, const int64_t* ic, int64_t ldc, int M, int N, int K,
                  double alpha = 1.0, double beta = 0.0) {
    return gdescT<T, T>(A, ia, lda, B, ib, ldb, C, ic, ldc, M, N, K, alpha, beta);
  };
  auto gemm = [](Uploader& up, hipStream_t st, const std::vector<GD>& d, int ta, int tb, int mode,
                 GemmShape shp, const char* site) {
    return rsrs::gemm<T, T>(up, st, d, ta, tb, mode, shp, site);
  };
  RSRS_TRY(ensure_ws(F, w, st));
  Uploader& up = F->up;
  const GemmShape shp = w <= 16 ? GS_64x16 : GS_64x64;
  T* x = F->wx.as<T>();
  T* u = F->wu.as<T>();
  const T* dS = F->d<T>();
  const int64_t* iS = F->i();
  const int64_t* perm = F->perm.as<int64_t>();
  const int W = (int)w;
  const int k = (int)F->k;
  gather_rows<double, T>(st, x, w, Fin, ldf, perm, F->n, w);

  // first and second elementary step of the upward sweep (boxes in factor order)
  for (const Group& g : F->groups) {
    std::vector<GD> a0, a1;   // launches with TA = 0 / TA = 1
    std::vector<GD> b0, b1;
    for (int64_t q = g.first; q < g.first + g.count; ++q) {
      const BoxRec& R = F->boxes[q];
      const int r = (int)R.r, kn = (int)(k + R.n);
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
    RSRS_TRY(gemm(up, st, a0, 0, 0, GM_FULL, shp, "solve"));
    RSRS_TRY(gemm(up, st, a1, 1, 0, GM_FULL, shp, "solve"));
    RSRS_TRY(gemm(up, st, b0, 0, 0, GM_FULL, shp, "solve"));
    RSRS_TRY(gemm(up, st, b1, 1, 0, GM_FULL, shp, "solve"));
  }
  // block-diagonal middle factor D (or D^{-1}), every R block and the root
  {
    std::vector<GD> dd;
    const int ta = transpose ? 1 : 0;
    for (const BoxRec& R : F->boxes) {
      const int r = (int)R.r;
      const T* D = dS + (op == OP_SOLVE ? R.oXinv : R.oXRR);
      const int64_t* gR = iS + R.oR;
      dd.push_back(gdesc(D, nullptr, R.ldR, x, gR, w, u, gR, w, r, W, r));
    }
    const int nt = (int)F->nt;
    const int64_t* gB = iS + F->oBt;
    dd.push_back(gdesc(dS + (op == OP_SOLVE ? F->oAtinv : F->oAt), nullptr, nt, x, gB, w, u, gB, w,
                       nt, W, nt));
    RSRS_TRY(gemm(up, st, dd, ta, 0, GM_FULL, shp, "solve"));
  }
  // downward sweep, boxes in reverse factor order
  for (size_t gi = F->groups.size(); gi-- > 0;) {
    const Group& g = F->groups[gi];
    std::vector<GD> a0, a1, b0, b1;
    for (int64_t q = g.first; q < g.first + g.count; ++q) {
      const BoxRec& R = F->boxes[q];
      const int r = (int)R.r, kn = (int)(k + R.n);
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
    RSRS_TRY(gemm(up, st, a0, 0, 0, GM_FULL, shp, "solve"));
    RSRS_TRY(gemm(up, st, a1, 1, 0, GM_FULL, shp, "solve"));
    RSRS_TRY(gemm(up, st, b0, 0, 0, GM_FULL, shp, "solve"));
    RSRS_TRY(gemm(up, st, b1, 1, 0, GM_FULL, shp, "solve"));
  }
  scatter_rows<T, double>(st, Uout, ldu, u, w, perm, F->n, w);
  RSRS_HIP(hipGetLastError());
  return RSRS_OK;
}

}  // namespace

rsrs_status apply_factor(const rsrs_factor_t* F, int op, int transpose, int64_t w, const double* Fin,
                         int64_t ldf, double* Uout, int64_t ldu, hipStream_t st) {
  if (w <= 0) return RSRS_OK;
  if (F->esz == 4) return apply_t<float>(F, op, transpose, w, Fin, ldf, Uout, ldu, st);
  return apply_t<double>(F, op, transpose, w, Fin, ldf, Uout, ldu, st);
}

}  // namespace rsrs
