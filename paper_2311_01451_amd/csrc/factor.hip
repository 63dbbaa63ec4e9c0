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
//           Cholesky G = L L^T and L^{-1} (recursive, GEMM-shaped);
//           least-squares coefficients X = Y_B pinv(C) = (Y_B C^T) L^{-T} L^{-1}
//           and the far-field sketch M_Y = Y_B - X C_Omega, i.e. Y_B times the
//           projector onto null(C_Omega) (eq. nullYZ); one optional second
//           pass re-projects M_Y and refines X.  Same for Z / Psi.
//           ID of M = M_Y + M_Z by pivoted Gram-Schmidt (Sec. 2.3).
//  phase B  Block extraction (eq. pinvYZ) from the same coefficients: since
//           Y_hat_R = Y_R - T Y_S and Omega_hat_C = G_T Omega_C with
//           G_T = I + e_S T^T e_R^T, Y_hat_R pinv(Omega_hat_C) =
//           (X_R - T X_S) G_T^{-1}; G_T^{-1} subtracts columns S T^T from
//           columns R.  X_RR^{-1} by Gauss-Jordan, K_U = X_RR^{-1} X_{R,SN},
//           K_L = X_{SN,R} X_RR^{-1}; then the sketch updates of Algorithm 1:
//           E, F (sparsify) followed by L, U (eliminate).
//  root     A_t = Y_Bt pinv(Omega_Bt) by the same Gram route, then A_t^{-1}.
//
// Precision.  The whole class of operations is templated on the element type
// T of the samples and of the stored factor.  T = double is plain FP64.  With
// T = float (the mixed-precision factorization) every product of sketch-sized
// operands runs on FP32 MFMA with FP32 accumulation, while the decisions stay
// FP64: the Gram matrices are accumulated from FP32 operands straight into
// FP64 storage and factored (Cholesky, inverse factor) in FP64, the pivoted
// QR of the ID runs on an FP64 copy of M, and X_RR and A_t are inverted by
// FP64 Gauss-Jordan with partial pivoting; the results are rounded to FP32
// for the products that use them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <unordered_map>

#include "impl.hpp"

namespace rsrs {

namespace {

struct CholMat {
  double* G;
  double* L;
  int64_t ld;
  int n;
};

constexpr int kLeaf = 64;

// Recursive Cholesky with inverse factor on the index range [a, b) shared by
// all matrices of the batch (each clipped to its own size n).
rsrs_status rchol(Uploader& up, hipStream_t st, const std::vector<CholMat>& mats, int a, int b,
                  int* flag) {
  if (b - a <= kLeaf) {
    std::vector<CholLeaf> e;
    for (const auto& m : mats) {
      const int hi = std::min(b, m.n);
      if (hi <= a) continue;
      e.push_back(CholLeaf{m.G + (int64_t)a * m.ld + a, m.L + (int64_t)a * m.ld + a, m.ld, hi - a, 0});
    }
    return chol_leaf(up, st, e, flag);
  }
  const int nblk = (b - a + kLeaf - 1) / kLeaf;
  const int h = a + kLeaf * ((nblk + 1) / 2);
  RSRS_TRY(rchol(up, st, mats, a, h, flag));
  std::vector<GemmDesc> g1, g2, g4, g5;
  for (const auto& m : mats) {
    const int hi = std::min(b, m.n);
    if (hi <= h) continue;
    const int rows = hi - h, w = h - a;
    double* G21 = m.G + (int64_t)h * m.ld + a;
    double* L11 = m.L + (int64_t)a * m.ld + a;
    double* L21 = m.L + (int64_t)h * m.ld + a;
    double* G22 = m.G + (int64_t)h * m.ld + h;
    double* L22 = m.L + (int64_t)h * m.ld + h;
    // (1) T1 = A21 L11^{-T} -> L21 slot
    g1.push_back(gdesc(G21, nullptr, m.ld, L11, nullptr, m.ld, L21, nullptr, m.ld, rows, w, w));
    // (2) A22 -= T1 T1^T (lower)
    g2.push_back(gdesc(L21, nullptr, m.ld, L21, nullptr, m.ld, G22, nullptr, m.ld, rows, rows, w,
                       -1.0, 1.0));
    // (4) W = T1 L11^{-1} -> G21 slot (A21 is dead)
    g4.push_back(gdesc(L21, nullptr, m.ld, L11, nullptr, m.ld, G21, nullptr, m.ld, rows, w, w));
    // (5) L21^{-1} block = -L22^{-1} W
    g5.push_back(gdesc(L22, nullptr, m.ld, G21, nullptr, m.ld, L21, nullptr, m.ld, rows, w, rows,
                       -1.0, 0.0));
  }
  RSRS_TRY(gemm(up, st, g1, 0, 1, GM_B_NT_LOW, GS_64x64, "chol"));
  RSRS_TRY(gemm(up, st, g2, 0, 1, GM_SYRK_L, GS_64x64, "chol"));
  RSRS_TRY(gemm(up, st, g4, 0, 0, GM_B_NN_LOW, GS_64x64, "chol"));
  RSRS_TRY(rchol(up, st, mats, h, b, flag));
  RSRS_TRY(gemm(up, st, g5, 0, 0, GM_A_LOW, GS_64x64, "chol"));
  return RSRS_OK;
}

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

// Workspace bytes of one box (b, l) in a class, samples of element type T.
template <typename T>
size_t box_ws_bytes(int64_t b, int64_t l, int64_t k, int64_t sp) {
  constexpr bool mixed = sizeof(T) != sizeof(double);
  const int64_t lp = round_up(l, 16);
  const int64_t r = b - k;
  int64_t dbl = 4 * l * lp        // G, L for both sides
                + 2 * b + b * k   // norms, R coefficients
                + 2 * r * r;      // Gauss-Jordan work
  int64_t tel = 6 * b * lp        // P, W, X for both sides
                + 2 * b * sp      // M_Y, M_Z
                + 4 * r * lp;     // XR, Xp for both sides
  if (mixed) {
    dbl += b * sp                 // FP64 copy of M for the ID
           + r * round_up(k, 4)   // T as computed by the ID
           + 2 * r * r;           // X_RR and its inverse in FP64
    tel += 2 * l * lp;            // rounded inverse factors
  }
  int64_t ints = b + k;           // sel, piv (int32)
  int64_t i64 = k + b;            // Spos, Rpos
  return (size_t)(dbl * 8 + tel * sizeof(T) + ints * 4 + i64 * 8 + 32 * 256);
}

template <typename T>
struct BoxWs {
  int64_t lp;
  double *GO, *GP, *LO, *LP, *norms, *Rc, *gje;
  T *LOt, *LPt;                 // inverse factors in T (alias LO, LP when T = double)
  T *PY, *WY, *XY, *PZ, *WZ, *XZ, *MY, *MZ;
  T *XRy, *XRz, *Xpy, *Xpz;
  double *Md, *Td, *XRRd, *Xinvd;   // FP64 copies (mixed precision only)
  int32_t *sel, *piv;
  int64_t *Spos, *Rpos;
};

template <typename T>
rsrs_status factor_t(const rsrs_tree_t* th, rsrs_samples_t* smp, const rsrs_factor_opts* o,
                     hipStream_t st, rsrs_factor_t** out) {
  constexpr bool mixed = sizeof(T) != sizeof(double);
  constexpr int64_t al = 16 / (int64_t)sizeof(T);   // elements per 16 bytes
  auto t0 = std::chrono::steady_clock::now();
  const Tree& t = th->t;
  const int k = o->k;
  const int p = o->p < 0 ? k : o->p;
  const int reproject = o->reproject;
  Schedule sch;
  make_schedule(t, k, sch);
  const int64_t need = samples_required(t, sch, k, p);
  if (smp->s < need) {
    set_required_s(need);
    set_error("s = " + std::to_string(smp->s) + " is below the required " + std::to_string(need));
    return RSRS_E_SAMPLES;
  }
  const int64_t s = smp->s, sld = smp->ld, n = t.n;
  T* Y = smp->Y.as<T>();
  T* Z = smp->Z.as<T>();
  T* Om = smp->Om.as<T>();
  T* Psi = smp->Psi.as<T>();

  auto F = std::make_unique<rsrs_factor_t>();
  F->n = n;
  F->s = s;
  F->k = k;
  F->precision = o->precision;
  F->esz = (int)sizeof(T);

  // ---- storage layout from the schedule (sizes are fixed by the count model)
  int64_t dsz = 0, isz = 0;
  size_t ws_max = 0;
  for (size_t li = 0; li < sch.levels.size(); ++li) {
    for (size_t c = 0; c < sch.classes[li].size(); ++c) {
      Group g;
      g.first = (int64_t)F->boxes.size();
      size_t ws = 0;
      for (int64_t b : sch.classes[li][c]) {
        BoxRec r;
        r.box = b;
        r.level = sch.levels[li];
        r.colour = (int)c;
        r.b = sch.b_count[b];
        r.n = sch.l_count[b] - r.b;
        r.k = k;
        r.r = r.b - k;
        r.ldT = round_up(k, al);
        r.ldR = round_up(r.r, al);
        r.ldKU = round_up(k + r.n, al);
        r.oT = round_up(dsz, al); dsz = r.oT + r.r * r.ldT;
        r.oXRR = round_up(dsz, al); dsz = r.oXRR + r.r * r.ldR;
        r.oXinv = round_up(dsz, al); dsz = r.oXinv + r.r * r.ldR;
        r.oKU = round_up(dsz, al); dsz = r.oKU + r.r * r.ldKU;
        r.oKL = round_up(dsz, al); dsz = r.oKL + (k + r.n) * r.ldR;
        r.oR = isz; isz += r.r;
        r.oS = isz; isz += k;
        r.oNa = isz; isz += r.n;
        r.oBa = isz; isz += r.b + r.n;   // Ba followed by a second copy of Na
        F->boxes.push_back(r);
        ws += box_ws_bytes<T>(r.b, r.b + r.n, k, sld);
      }
      g.count = (int64_t)F->boxes.size() - g.first;
      F->groups.push_back(g);
      ws_max = std::max(ws_max, ws);
    }
  }
  F->nt = sch.root_count;
  F->oBt = isz; isz += F->nt;
  F->oAt = round_up(dsz, al); dsz = F->oAt + F->nt * F->nt;
  F->oAtinv = round_up(dsz, al); dsz = F->oAtinv + F->nt * F->nt;
  F->stored_values = dsz;
  const int64_t ntp = round_up(F->nt, 16);
  size_t root_ws = (size_t)(4 * F->nt * ntp + F->nt * round_up(s, 16) + 2 * F->nt * F->nt) * 8 + 8 * 256;
  if (mixed)   // FP64 copies of Y_Bt, Omega_Bt, A_t, A_t^{-1}
    root_ws += (size_t)(2 * F->nt * round_up(s, 16) + 2 * F->nt * F->nt) * 8 + 4 * 256;
  ws_max = std::max(ws_max, root_ws);

  RSRS_TRY(F->dstore.alloc((size_t)std::max<int64_t>(dsz, 1) * sizeof(T)));
  RSRS_TRY(F->istore.alloc((size_t)std::max<int64_t>(isz, 1) * 8));
  RSRS_TRY(F->perm.alloc((size_t)n * 8));
  DevBuf ws, flagbuf;
  RSRS_TRY(ws.alloc(ws_max));
  RSRS_TRY(flagbuf.alloc(256));
  int* flag = flagbuf.as<int>();
  RSRS_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
  T* dS = F->dstore.as<T>();
  int64_t* iS = F->istore.as<int64_t>();

  Uploader up;
  RSRS_TRY(up.init((size_t)64 << 20, st));
  RSRS_HIP(hipMemcpyAsync(F->perm.p, t.perm.data(), (size_t)n * 8, hipMemcpyHostToDevice, st));
  // non-finite samples are rejected up front
  check_finite(st, Y, n, s, sld, flag);
  check_finite(st, Z, n, s, sld, flag);
  check_finite(st, Om, n, s, sld, flag);
  check_finite(st, Psi, n, s, sld, flag);
  RSRS_TRY(up.reset());
  {
    int hflag = 0;
    RSRS_HIP(hipMemcpy(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost));
    if (hflag & 4) { set_error("non-finite value in the samples"); return RSRS_E_NUMERIC; }
  }

  // staging for index uploads into the factor store
  HostBuf hidx;
  RSRS_TRY(hidx.alloc((size_t)std::max<int64_t>(isz, 1) * 8));
  int64_t* hI = hidx.as<int64_t>();
  HostBuf hpos;

  double flops = 0.0;
  const int64_t nbox = t.nbox();
  std::vector<std::vector<int64_t>> cur(nbox), remaining(nbox);
  auto leaf_range = [&](int64_t b) {
    std::vector<int64_t> v((size_t)t.npts(b));
    std::iota(v.begin(), v.end(), t.pt_begin[b]);
    return v;
  };

  size_t gi = 0;
  for (size_t li = 0; li < sch.levels.size(); ++li) {
    const int lev = sch.levels[li];
    const auto& lb = t.level_boxes[lev];
    std::unordered_map<int64_t, size_t> pos;
    for (size_t i = 0; i < lb.size(); ++i) {
      const int64_t b = lb[i];
      pos[b] = i;
      if (t.is_leaf[b]) {
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
    auto active_of = [&](int64_t x) -> const std::vector<int64_t>& {
      if (t.level[x] < lev && cur[x].empty()) cur[x] = leaf_range(x);
      return cur[x];
    };
    for (size_t c = 0; c < sch.classes[li].size(); ++c, ++gi) {
      const Group& g = F->groups[gi];
      const int64_t nb = g.count;
      // ---- host index lists and factor-store uploads (Ba, Na, Na copy)
      std::vector<std::vector<int64_t>> Ba(nb), Na(nb);
      for (int64_t q = 0; q < nb; ++q) {
        BoxRec& R = F->boxes[g.first + q];
        const size_t ip = pos.at(R.box);
        Ba[q] = cur[R.box];
        std::vector<int64_t> v;
        for (int64_t j = t.nb_off[lev][ip]; j < t.nb_off[lev][ip + 1]; ++j) {
          const auto& a = active_of(t.nb_ids[lev][j]);
          v.insert(v.end(), a.begin(), a.end());
        }
        std::sort(v.begin(), v.end());
        Na[q] = std::move(v);
        if ((int64_t)Ba[q].size() != R.b || (int64_t)Na[q].size() != R.n) {
          set_error("internal: active sets disagree with the count model");
          return RSRS_E_INVALID;
        }
        std::memcpy(hI + R.oNa, Na[q].data(), R.n * 8);
        std::memcpy(hI + R.oBa, Ba[q].data(), R.b * 8);
        std::memcpy(hI + R.oBa + R.b, Na[q].data(), R.n * 8);
        RSRS_HIP(hipMemcpyAsync(iS + R.oNa, hI + R.oNa, (size_t)(R.n + R.b + R.n) * 8,
                                hipMemcpyHostToDevice, st));
      }
      // ---- workspace
      Bump bump{ws.as<char>(), 0, ws.bytes};
      std::vector<BoxWs<T>> W(nb);
      for (int64_t q = 0; q < nb; ++q) {
        const BoxRec& R = F->boxes[g.first + q];
        const int64_t l = R.b + R.n, lp = round_up(l, 16), b = R.b, r = R.r;
        BoxWs<T>& w = W[q];
        w.lp = lp;
        w.GO = bump.take<double>(l * lp); w.GP = bump.take<double>(l * lp);
        w.LO = bump.take<double>(l * lp); w.LP = bump.take<double>(l * lp);
        w.PY = bump.take<T>(b * lp); w.WY = bump.take<T>(b * lp); w.XY = bump.take<T>(b * lp);
        w.PZ = bump.take<T>(b * lp); w.WZ = bump.take<T>(b * lp); w.XZ = bump.take<T>(b * lp);
        w.MY = bump.take<T>(b * sld); w.MZ = bump.take<T>(b * sld);
        w.norms = bump.take<double>(2 * b); w.Rc = bump.take<double>(b * k);
        w.XRy = bump.take<T>(r * lp); w.XRz = bump.take<T>(r * lp);
        w.Xpy = bump.take<T>(r * lp); w.Xpz = bump.take<T>(r * lp);
        w.gje = bump.take<double>(2 * r * r);
        w.sel = bump.take<int32_t>(b); w.piv = bump.take<int32_t>(k);
        w.Spos = bump.take<int64_t>(k); w.Rpos = bump.take<int64_t>(b);
        if constexpr (mixed) {
          w.LOt = bump.take<T>(l * lp); w.LPt = bump.take<T>(l * lp);
          w.Md = bump.take<double>(b * sld);
          w.Td = bump.take<double>(r * round_up(k, 4));
          w.XRRd = bump.take<double>(r * r); w.Xinvd = bump.take<double>(r * r);
        } else {
          w.LOt = reinterpret_cast<T*>(w.LO); w.LPt = reinterpret_cast<T*>(w.LP);
          w.Md = w.Td = w.XRRd = w.Xinvd = nullptr;
        }
      }
      if (bump.off > bump.cap) { set_error("internal: workspace overflow"); return RSRS_E_INVALID; }
      // ---- phase A: Gram matrices (FP64 storage in both precisions)
      std::vector<GemmDescT<T, double>> gd;
      std::vector<CholMat> cm;
      int lmax = 0;
      for (int64_t q = 0; q < nb; ++q) {
        const BoxRec& R = F->boxes[g.first + q];
        const BoxWs<T>& w = W[q];
        const int l = (int)(R.b + R.n);
        const int64_t* idxC = iS + R.oBa;
        gd.push_back(gdescT<T, double>(Om, idxC, sld, Om, idxC, sld, w.GO, nullptr, w.lp, l, l, (int)s));
        gd.push_back(gdescT<T, double>(Psi, idxC, sld, Psi, idxC, sld, w.GP, nullptr, w.lp, l, l, (int)s));
        cm.push_back(CholMat{w.GO, w.LO, w.lp, l});
        cm.push_back(CholMat{w.GP, w.LP, w.lp, l});
        lmax = std::max(lmax, l);
        const double dl = l, db = (double)R.b, ds = (double)s;
        flops += 2.0 * dl * dl * ds                               // two Gram matrices
                 + 2.0 * (2.0 / 3.0) * dl * dl * dl               // Cholesky + inverse factor
                 + (1.0 + reproject) * 2.0 * (4.0 * db * dl * ds + 2.0 * db * dl * dl);  // projections
      }
      RSRS_TRY(gemm<T, double>(up, st, gd, 0, 1, GM_SYRK_L, GS_64x64, "gram"));
      RSRS_TRY(rchol(up, st, cm, 0, lmax, flag));
      if constexpr (mixed) {   // inverse factors rounded for the FP32 products
        std::vector<Copy2DT<double, T>> lc;
        for (int64_t q = 0; q < nb; ++q) {
          const BoxRec& R = F->boxes[g.first + q];
          const BoxWs<T>& w = W[q];
          const int l = (int)(R.b + R.n);
          lc.push_back(Copy2DT<double, T>{w.LO, w.LOt, w.lp, w.lp, l, l, 1.0, 0, 0});
          lc.push_back(Copy2DT<double, T>{w.LP, w.LPt, w.lp, w.lp, l, l, 1.0, 0, 0});
        }
        RSRS_TRY(copy2d<double, T>(up, st, lc));
      }
      // ---- projections (eq. nullYZ) and least-squares coefficients
      for (int pass = 0; pass <= reproject; ++pass) {
        std::vector<GemmDescT<T, T>> gp, gw, gx, gm;
        std::vector<Copy2DT<T, T>> acc;
        for (int64_t q = 0; q < nb; ++q) {
          const BoxRec& R = F->boxes[g.first + q];
          const BoxWs<T>& w = W[q];
          const int l = (int)(R.b + R.n), b = (int)R.b;
          const int64_t* idxB = iS + R.oBa;
          const int64_t* idxC = iS + R.oBa;
          for (int side = 0; side < 2; ++side) {
            T* Ysd = side ? Z : Y;
            T* Tst = side ? Psi : Om;
            T* Pb = side ? w.PZ : w.PY;
            T* Wb = side ? w.WZ : w.WY;
            T* Xb = side ? w.XZ : w.XY;
            T* Mb = side ? w.MZ : w.MY;
            T* Lb = side ? w.LPt : w.LOt;
            T* Xout = pass == 0 ? Xb : Pb;   // second pass: correction into P
            if (pass == 0)
              gp.push_back(gdescT<T, T>(Ysd, idxB, sld, Tst, idxC, sld, Pb, nullptr, w.lp, b, l, (int)s));
            else
              gp.push_back(gdescT<T, T>(Mb, nullptr, sld, Tst, idxC, sld, Pb, nullptr, w.lp, b, l, (int)s));
            gw.push_back(gdescT<T, T>(Pb, nullptr, w.lp, Lb, nullptr, w.lp, Wb, nullptr, w.lp, b, l, l));
            gx.push_back(gdescT<T, T>(Wb, nullptr, w.lp, Lb, nullptr, w.lp, Xout, nullptr, w.lp, b, l, l));
            if (pass == 0)
              gm.push_back(gdescT<T, T>(Xout, nullptr, w.lp, Tst, idxC, sld, Mb, nullptr, sld, b, (int)s, l,
                                        -1.0, 1.0, Ysd, idxB, sld));
            else
              gm.push_back(gdescT<T, T>(Xout, nullptr, w.lp, Tst, idxC, sld, Mb, nullptr, sld, b, (int)s, l,
                                        -1.0, 1.0));
            if (pass == 1) acc.push_back(Copy2DT<T, T>{Pb, Xb, w.lp, w.lp, b, l, 1.0, 1, 0});
          }
        }
        RSRS_TRY(gemm<T, T>(up, st, gp, 0, 1, GM_FULL, GS_64x64, "proj"));
        RSRS_TRY(gemm<T, T>(up, st, gw, 0, 1, GM_B_NT_LOW, GS_64x64, "proj"));
        RSRS_TRY(gemm<T, T>(up, st, gx, 0, 0, GM_B_NN_LOW, GS_64x64, "proj"));
        RSRS_TRY(gemm<T, T>(up, st, gm, 0, 0, GM_FULL, GS_64x64, "proj"));
        RSRS_TRY(copy2d<T, T>(up, st, acc));
      }
      // ---- interpolative decomposition of M = M_Y + M_Z
      std::vector<IdDesc> idd;
      for (int64_t q = 0; q < nb; ++q) {
        const BoxRec& R = F->boxes[g.first + q];
        const BoxWs<T>& w = W[q];
        IdDesc e{};
        if constexpr (mixed) {
          e.M = w.Md; e.MZ = nullptr; e.ldm = sld; e.ldz = sld;
          e.MYf = w.MY; e.MZf = w.MZ; e.ldf = sld;
          e.T = w.Td; e.ldt = (int)round_up(k, 4);
        } else {
          e.M = w.MY; e.MZ = w.MZ; e.ldm = sld; e.ldz = sld;
          e.T = dS + R.oT; e.ldt = (int)R.ldT;
        }
        e.norms = w.norms; e.sel = w.sel; e.Rc = w.Rc; e.piv = w.piv;
        e.Spos = w.Spos; e.Rpos = w.Rpos;
        e.b = (int)R.b; e.s = (int)s; e.k = k;
        idd.push_back(e);
        flops += 4.0 * R.b * s * k;
      }
      RSRS_TRY(id_run(up, st, idd));
      if constexpr (mixed) {   // T rounded into the factor store
        std::vector<Copy2DT<double, T>> tc;
        for (int64_t q = 0; q < nb; ++q) {
          const BoxRec& R = F->boxes[g.first + q];
          tc.push_back(Copy2DT<double, T>{W[q].Td, dS + R.oT, round_up(k, 4), R.ldT, (int)R.r, k, 1.0, 0, 0});
        }
        RSRS_TRY(copy2d<double, T>(up, st, tc));
      }
      // ---- skeleton sets back to the host
      int64_t nposn = 0;
      for (int64_t q = 0; q < nb; ++q) nposn += F->boxes[g.first + q].b;
      RSRS_TRY(hpos.alloc((size_t)nposn * 8));
      {
        int64_t o2 = 0;
        for (int64_t q = 0; q < nb; ++q) {
          const BoxRec& R = F->boxes[g.first + q];
          RSRS_HIP(hipMemcpyAsync(hpos.as<int64_t>() + o2, W[q].Spos, (size_t)k * 8, hipMemcpyDeviceToHost, st));
          RSRS_HIP(hipMemcpyAsync(hpos.as<int64_t>() + o2 + k, W[q].Rpos, (size_t)R.r * 8, hipMemcpyDeviceToHost, st));
          o2 += R.b;
        }
      }
      RSRS_TRY(up.reset());
      {
        int hflag = 0;
        RSRS_HIP(hipMemcpy(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost));
        if (hflag & 1) {
          set_error("Gram matrix of a test-matrix panel is not positive definite (rank-deficient panel)");
          return RSRS_E_SINGULAR;
        }
      }
      // ---- phase B: global R / S / SN lists
      {
        int64_t o2 = 0;
        for (int64_t q = 0; q < nb; ++q) {
          BoxRec& R = F->boxes[g.first + q];
          const int64_t* sp = hpos.as<int64_t>() + o2;
          const int64_t* rp = sp + k;
          std::vector<int64_t> Sg(k), Rg(R.r);
          for (int j = 0; j < k; ++j) Sg[j] = Ba[q][sp[j]];
          for (int64_t j = 0; j < R.r; ++j) Rg[j] = Ba[q][rp[j]];
          std::memcpy(hI + R.oR, Rg.data(), R.r * 8);
          std::memcpy(hI + R.oS, Sg.data(), (size_t)k * 8);
          RSRS_HIP(hipMemcpyAsync(iS + R.oR, hI + R.oR, (size_t)(R.r + k) * 8, hipMemcpyHostToDevice, st));
          cur[R.box] = std::move(Sg);
          o2 += R.b;
        }
      }
      std::vector<GemmDescT<T, T>> gxr;
      std::vector<ColfixDescT<T>> cf;
      std::vector<Copy2DT<T, T>> cx;
      std::vector<Copy2DT<T, double>> cxd;
      std::vector<Copy2DT<double, T>> cinv;
      std::vector<GjeDesc> gj;
      for (int64_t q = 0; q < nb; ++q) {
        const BoxRec& R = F->boxes[g.first + q];
        const BoxWs<T>& w = W[q];
        const int l = (int)(R.b + R.n), r = (int)R.r;
        for (int side = 0; side < 2; ++side) {
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
          gj.push_back(GjeDesc{w.Xpy, w.gje, dS + R.oXinv, w.lp, R.ldR, r, 0});
        }
        const double dr = r, dk = k, dn = (double)R.n, ds = (double)s;
        flops += 2.0 * (2.0 * dr * dk * l + 2.0 * dr * dr * dk) + 2.0 * dr * dr * dr +
                 2.0 * 2.0 * dr * dr * (dk + dn) + 4.0 * 2.0 * dr * dk * ds + 4.0 * 2.0 * dr * (dk + dn) * ds;
      }
      RSRS_TRY(gemm<T, T>(up, st, gxr, 0, 0, GM_FULL, GS_64x64, "extract"));
      RSRS_TRY(colfix<T>(up, st, cf));
      RSRS_TRY(copy2d<T, T>(up, st, cx));
      RSRS_TRY(copy2d<T, double>(up, st, cxd));
      RSRS_TRY(gje_inverse(up, st, gj, flag));
      RSRS_TRY(copy2d<double, T>(up, st, cinv));
      std::vector<GemmDescT<T, T>> gku, gkl;
      for (int64_t q = 0; q < nb; ++q) {
        const BoxRec& R = F->boxes[g.first + q];
        const BoxWs<T>& w = W[q];
        const int r = (int)R.r, kn = (int)(k + R.n);
        gku.push_back(gdescT<T, T>(dS + R.oXinv, nullptr, R.ldR, w.Xpy + r, nullptr, w.lp, dS + R.oKU, nullptr, R.ldKU, r, kn, r));
        gkl.push_back(gdescT<T, T>(w.Xpz + r, nullptr, w.lp, dS + R.oXinv, nullptr, R.ldR, dS + R.oKL, nullptr, R.ldR, kn, r, r));
      }
      RSRS_TRY(gemm<T, T>(up, st, gku, 0, 0, GM_FULL, GS_64x64, "mult"));
      RSRS_TRY(gemm<T, T>(up, st, gkl, 1, 0, GM_FULL, GS_64x64, "mult"));
      // ---- sketch updates: sparsify (E, F) then eliminate (L, U)
      std::vector<GemmDescT<T, T>> s0, s1, e0, e1, e0b, e1b;
      for (int64_t q = 0; q < nb; ++q) {
        const BoxRec& R = F->boxes[g.first + q];
        const int r = (int)R.r, kn = (int)(k + R.n);
        const int64_t* gR = iS + R.oR;
        const int64_t* gS = iS + R.oS;
        const int64_t* gSN = iS + R.oS;
        const T* Tm = dS + R.oT;
        const T* KU = dS + R.oKU;
        const T* KL = dS + R.oKL;
        const int64_t lT = R.ldT, lR = R.ldR, lU = R.ldKU;
        s0.push_back(gdescT<T, T>(Tm, nullptr, lT, Y, gS, sld, Y, gR, sld, r, (int)s, k, -1.0, 1.0));
        s0.push_back(gdescT<T, T>(Tm, nullptr, lT, Z, gS, sld, Z, gR, sld, r, (int)s, k, -1.0, 1.0));
        s1.push_back(gdescT<T, T>(Tm, nullptr, lT, Om, gR, sld, Om, gS, sld, k, (int)s, r, 1.0, 1.0));
        s1.push_back(gdescT<T, T>(Tm, nullptr, lT, Psi, gR, sld, Psi, gS, sld, k, (int)s, r, 1.0, 1.0));
        e0.push_back(gdescT<T, T>(KL, nullptr, lR, Y, gR, sld, Y, gSN, sld, kn, (int)s, r, -1.0, 1.0));
        e0b.push_back(gdescT<T, T>(KU, nullptr, lU, Om, gSN, sld, Om, gR, sld, r, (int)s, kn, 1.0, 1.0));
        e1.push_back(gdescT<T, T>(KU, nullptr, lU, Z, gR, sld, Z, gSN, sld, kn, (int)s, r, -1.0, 1.0));
        e1b.push_back(gdescT<T, T>(KL, nullptr, lR, Psi, gSN, sld, Psi, gR, sld, r, (int)s, kn, 1.0, 1.0));
      }
      RSRS_TRY(gemm<T, T>(up, st, s0, 0, 0, GM_FULL, GS_64x64, "sparsify"));
      RSRS_TRY(gemm<T, T>(up, st, s1, 1, 0, GM_FULL, GS_64x64, "sparsify"));
      RSRS_TRY(gemm<T, T>(up, st, e0, 0, 0, GM_FULL, GS_64x64, "elim"));
      RSRS_TRY(gemm<T, T>(up, st, e1, 1, 0, GM_FULL, GS_64x64, "elim"));
      RSRS_TRY(gemm<T, T>(up, st, e0b, 0, 0, GM_FULL, GS_64x64, "elim_r"));
      RSRS_TRY(gemm<T, T>(up, st, e1b, 1, 0, GM_FULL, GS_64x64, "elim_r"));
    }
    for (int64_t b : lb) remaining[b] = cur[b];
  }

  // ---- root: A_t = Y_Bt pinv(Omega_Bt)
  {
    std::vector<int64_t> Bt;
    if (t.nlevels == 0) {
      Bt.resize(n);
      std::iota(Bt.begin(), Bt.end(), 0);
    } else {
      for (int64_t b : t.level_boxes[1]) Bt.insert(Bt.end(), remaining[b].begin(), remaining[b].end());
      std::sort(Bt.begin(), Bt.end());
    }
    if ((int64_t)Bt.size() != F->nt) { set_error("internal: root size mismatch"); return RSRS_E_INVALID; }
    const int nt = (int)F->nt;
    std::memcpy(hI + F->oBt, Bt.data(), (size_t)nt * 8);
    RSRS_HIP(hipMemcpyAsync(iS + F->oBt, hI + F->oBt, (size_t)nt * 8, hipMemcpyHostToDevice, st));
    const int64_t* iBt = iS + F->oBt;
    Bump bump{ws.as<char>(), 0, ws.bytes};
    double* G = bump.take<double>(nt * ntp);
    double* L = bump.take<double>(nt * ntp);
    double* P = bump.take<double>(nt * ntp);
    double* Wb = bump.take<double>(nt * ntp);
    double* Rres = bump.take<double>(nt * round_up(s, 16));
    double* gw = bump.take<double>(2 * (int64_t)nt * nt);
    // FP64 operands of the root: the samples themselves (rows iBt), or FP64
    // copies of the rows B_t in mixed precision
    const double* Yr;
    const double* Or;
    const int64_t* ir;
    int64_t rld;
    double* At;
    double* Atinv;
    if constexpr (mixed) {
      const int64_t sp = round_up(s, 16);
      double* Yd = bump.take<double>(nt * sp);
      double* Od = bump.take<double>(nt * sp);
      At = bump.take<double>((int64_t)nt * nt);
      Atinv = bump.take<double>((int64_t)nt * nt);
      gather_rows<T, double>(st, Yd, sp, Y, sld, iBt, nt, s);
      gather_rows<T, double>(st, Od, sp, Om, sld, iBt, nt, s);
      Yr = Yd; Or = Od; ir = nullptr; rld = sp;
    } else {
      Yr = reinterpret_cast<const double*>(Y);
      Or = reinterpret_cast<const double*>(Om);
      ir = iBt; rld = sld;
      At = reinterpret_cast<double*>(dS + F->oAt);
      Atinv = reinterpret_cast<double*>(dS + F->oAtinv);
    }
    if (bump.off > bump.cap) { set_error("internal: root workspace overflow"); return RSRS_E_INVALID; }
    RSRS_TRY(gemm(up, st, {gdesc(Or, ir, rld, Or, ir, rld, G, nullptr, ntp, nt, nt, (int)s)}, 0, 1, GM_SYRK_L));
    RSRS_TRY(rchol(up, st, {CholMat{G, L, ntp, nt}}, 0, nt, flag));
    RSRS_TRY(gemm(up, st, {gdesc(Yr, ir, rld, Or, ir, rld, P, nullptr, ntp, nt, nt, (int)s)}, 0, 1, GM_FULL));
    RSRS_TRY(gemm(up, st, {gdesc(P, nullptr, ntp, L, nullptr, ntp, Wb, nullptr, ntp, nt, nt, nt)}, 0, 1, GM_B_NT_LOW));
    RSRS_TRY(gemm(up, st, {gdesc(Wb, nullptr, ntp, L, nullptr, ntp, At, nullptr, nt, nt, nt, nt)}, 0, 0, GM_B_NN_LOW));
    if (reproject) {
      const int64_t rp = round_up(s, 16);
      RSRS_TRY(gemm(up, st, {gdesc(At, nullptr, nt, Or, ir, rld, Rres, nullptr, rp, nt, (int)s, nt, -1.0, 1.0, Yr, ir, rld)}, 0, 0, GM_FULL));
      RSRS_TRY(gemm(up, st, {gdesc(Rres, nullptr, rp, Or, ir, rld, P, nullptr, ntp, nt, nt, (int)s)}, 0, 1, GM_FULL));
      RSRS_TRY(gemm(up, st, {gdesc(P, nullptr, ntp, L, nullptr, ntp, Wb, nullptr, ntp, nt, nt, nt)}, 0, 1, GM_B_NT_LOW));
      RSRS_TRY(gemm(up, st, {gdesc(Wb, nullptr, ntp, L, nullptr, ntp, At, nullptr, nt, nt, nt, nt, 1.0, 1.0)}, 0, 0, GM_B_NN_LOW));
    }
    RSRS_TRY(gje_inverse(up, st, {GjeDesc{At, gw, Atinv, nt, nt, nt, 0}}, flag));
    if constexpr (mixed) {
      RSRS_TRY(copy2d<double, T>(up, st, {Copy2DT<double, T>{At, dS + F->oAt, nt, nt, nt, nt, 1.0, 0, 0},
                                          Copy2DT<double, T>{Atinv, dS + F->oAtinv, nt, nt, nt, nt, 1.0, 0, 0}}));
    }
    const double dt = nt;
    flops += dt * dt * s + (2.0 / 3.0) * dt * dt * dt + (1 + reproject) * (2.0 * dt * dt * s + 2.0 * dt * dt * dt) + 2.0 * dt * dt * dt;
  }
  RSRS_TRY(up.reset());
  {
    int hflag = 0;
    RSRS_HIP(hipMemcpy(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost));
    if (hflag & 1) { set_error("Gram matrix of the root panel is not positive definite"); return RSRS_E_SINGULAR; }
    if (hflag & 2) { set_error("singular pivot block X_RR or root block"); return RSRS_E_SINGULAR; }
  }
  smp->consumed = true;
  F->flops = flops;
  F->factor_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = F.release();
  return RSRS_OK;
}

}  // namespace

rsrs_status factor_impl(const rsrs_tree_t* th, rsrs_samples_t* smp, const rsrs_factor_opts* o,
                        hipStream_t st, rsrs_factor_t** out) {
  const int k = o->k;
  if (k < 1) { set_error("k must be >= 1"); return RSRS_E_INVALID; }
  if (smp->consumed) { set_error("samples were already consumed by a factorization"); return RSRS_E_INVALID; }
  if (smp->tree != th) { set_error("samples belong to another tree"); return RSRS_E_INVALID; }
  if (k > 256) { set_error("k > 256 is not supported"); return RSRS_E_UNSUPPORTED; }
  if (o->reproject < 0 || o->reproject > 1) { set_error("reproject must be 0 or 1"); return RSRS_E_INVALID; }
  if (o->precision == RSRS_PREC_F64) {
    if (smp->dtype != RSRS_F64) { set_error("FP64 factorization needs FP64 samples"); return RSRS_E_INVALID; }
    return factor_t<double>(th, smp, o, st, out);
  }
  if (o->precision == RSRS_PREC_F32_MIXED) {
    if (smp->dtype != RSRS_F32) { set_error("mixed-precision factorization needs FP32 samples"); return RSRS_E_INVALID; }
    return factor_t<float>(th, smp, o, st, out);
  }
  set_error("unknown precision");
  return RSRS_E_UNSUPPORTED;
}

}  // namespace rsrs
