"""Algorithm 1 (randomized strong recursive skeletonization) -- oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Plain FP64 NumPy/SciPy, one box after another, in the order fixed by
``oracle.tree.schedule``.  Every step names the passage it follows.  Readings:

* Nullification (eq. nullYZ): Y_B null(C_Omega) is taken as the projection
  M_Y = Y_B (I - Q Q^T) with Q an orthonormal basis of the row space of
  C_Omega = [Omega_Ba; Omega_Na] (Householder QR of C_Omega^T).  For any
  orthonormal null-space basis N', Y_B N' N'^T equals M_Y, so the skeleton
  choice and T do not depend on the basis.  The sketch handed to the ID is the
  sum M = M_Y + M_Z (Algorithm 1, "id(Y' + Z')").
* ID (Sec. 2.3): column-pivoted Householder QR of M^T (LAPACK dgeqp3 via
  scipy.linalg.qr); S = first k pivots, R = the rest,
  T = (R11^{-1} R12)^T, so that rows satisfy A_{R,F} ~ T A_{S,F} and
  A_{F,R} ~ A_{F,S} T^T; S and R are then sorted by tree index and T permuted
  to match.
* Sparsification (eq. orth_sparsifying, Algorithm 1): in index form
  Y_R -= T Y_S, Z_R -= T Z_S, Omega_S += T^T Omega_R, Psi_S += T^T Psi_R.
* Extraction (eq. pinvYZ) uses the updated ("hatted") sketches with columns
  ordered [R; S; N_a]; the pseudo-inverse of the full-row-rank C is applied
  through a Householder QR of C^T.  X_RR, X_RS, X_RN come from the Y side,
  X_SR, X_NR from the Z side.
* Elimination (eq. LUstrong; Algorithm 1): K_U = X_RR^{-1} X_{R,SN},
  K_L = X_{SN,R} X_RR^{-1} with SN = [S; N_a], LU with partial pivoting, then
  Y_SN -= K_L Y_R, Omega_R += K_U Omega_SN, Z_SN -= K_U^T Z_R,
  Psi_R += K_L^T Psi_SN.
* Root (Algorithm 1, last step): A_t = Y_Bt pinv(Omega_Bt), LU with partial
  pivoting.
* Symmetric variant (A = A^T; the paper notes U = L^T and F = E^T for it,
  Sec. 2.2 and the remark after eq. Ainvfact): with Psi = Omega, Z = Y is
  the same sketch, so only the Y / Omega side is kept.  The ID of
  M_Y + M_Z = 2 M_Y equals the ID of M_Y (scaling by 2 is exact and does not
  move CPQR pivots or T).  To make U = L^T exactly, X_RR is replaced by its
  symmetric part (X_RR + X_RR^T)/2, K_U = X_RR^{-1} X_{R,SN} and
  K_L = K_U^T; the root block is symmetrized the same way.  Elimination
  updates Y_SN -= K_L Y_R and Omega_R += K_U Omega_SN only.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import tree as otree


class InsufficientSamples(ValueError):
    pass


@dataclass
class BoxFactor:
    box: int
    level: int
    colour: int
    Ba: np.ndarray     # active indices of the box (tree order), sorted
    Na: np.ndarray     # active indices of the neighbours, sorted
    S: np.ndarray      # skeleton (kept active), sorted
    R: np.ndarray      # redundant (eliminated), sorted
    T: np.ndarray      # r x k
    XRR: np.ndarray    # r x r
    lu: tuple          # scipy lu_factor of XRR
    KU: np.ndarray     # r x (k+n)
    KL: np.ndarray     # (k+n) x r
    M: np.ndarray = field(default=None, repr=False)   # b x s ID input (diagnostic)
    # conditioning diagnostics: ||[Y_B Z_B]||_F, ||M||_F, min |diag R11| of the ID
    norm_yz: float = 0.0
    norm_m: float = 0.0
    r11_min: float = 0.0
    rdiag: np.ndarray = field(default=None, repr=False)   # |diag R| of the pivoted QR (first k+1)

    @property
    def SN(self) -> np.ndarray:
        return np.concatenate([self.S, self.Na])


@dataclass
class Factorization:
    tree: otree.Tree
    k: int
    p: int
    s: int
    boxes: list            # BoxFactor in processing order
    Bt: np.ndarray         # root active indices (tree order)
    At: np.ndarray
    At_lu: tuple
    perm: np.ndarray       # tree position -> user index


def _orth_rows(C: np.ndarray) -> np.ndarray:
    """Orthonormal basis (s x l) of the row space of the l x s matrix C (eq. orth)."""
    q, _ = np.linalg.qr(C.T, mode="reduced")
    return q


def _right_pinv_apply(Yr: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Yr @ pinv(C) for C (l x s, l <= s, full row rank): with C^T = Q R,
    pinv(C) = Q R^{-T}, so X = (Yr Q) R^{-T} solves R X^T = (Yr Q)^T."""
    q, r = np.linalg.qr(C.T, mode="reduced")
    t = Yr @ q
    return sla.solve_triangular(r, t.T, lower=False).T


def nullify(YB: np.ndarray, C: np.ndarray) -> np.ndarray:
    """YB projected onto null(C): YB (I - Q Q^T), Q = orth(C^T) (eq. nullYZ,
    eq. Omegaprime_null in projector form)."""
    q = _orth_rows(C)
    return YB - (YB @ q) @ q.T


def row_id(M: np.ndarray, k: int, want_r11_min: bool = False, rank_tol: float = 0.0,
           ref_norm: float = 0.0):
    """Row interpolative decomposition of M (Sec. 2.3, eq. id_def) by greedy
    column-pivoted QR of M^T.  Returns (S_pos, R_pos, T) with positions sorted
    ascending and T (r x k_B) such that M[R_pos] ~ T M[S_pos] (and, on request,
    the smallest |diagonal| of R11).

    Rank: k_B = min(k, b) pivots (the fixed rank of Sec. 4.5), or, with
    rank_tol > 0, only the leading pivots whose |R_jj| exceeds
    rank_tol * ref_norm (the numerical rank of the sketch relative to
    ref_norm; the diagonal of a column-pivoted R does not increase, so this
    stops at the first pivot at or below the threshold)."""
    _, Rf, piv = sla.qr(M.T, mode="economic", pivoting=True)
    kb = min(k, M.shape[0])
    if rank_tol > 0.0:
        d = np.abs(np.diag(Rf))[:kb]
        below = np.nonzero(d <= rank_tol * ref_norm)[0]
        if below.size:
            kb = int(below[0])
    S_piv = piv[:kb]
    R_piv = piv[kb:]
    R11 = Rf[:kb, :kb]
    R12 = Rf[:kb, kb:]
    Tp = sla.solve_triangular(R11, R12, lower=False).T if kb else np.zeros((len(R_piv), 0))
    so = np.argsort(S_piv, kind="stable")
    ro = np.argsort(R_piv, kind="stable")
    if want_r11_min:
        r11 = float(np.abs(np.diag(R11)).min()) if kb else 0.0
        return S_piv[so], R_piv[ro], Tp[np.ix_(ro, so)], r11, np.abs(np.diag(Rf))[:k + 1]
    return S_piv[so], R_piv[ro], Tp[np.ix_(ro, so)]


def factor(tree: otree.Tree, Y, Z, Om, Psi, k: int, p: int | None = None,
           keep_M: bool = False, check_samples: bool = True, on_box=None,
           symmetric: bool = False, id_mode: str = "sum", rank_tol: float = 0.0,
           col_subset: bool = False, redraw: dict | None = None) -> Factorization:
    """Algorithm 1 on sketches given in user point order (N x s each).

    The caller's arrays are not modified; the oracle works on tree-ordered
    copies.  ``on_box(bf, Y, Z, Om, Psi)`` (optional) is called after each box
    with the updated tree-ordered sketches, for invariant checks.  With
    ``symmetric`` (A = A^T) only Y and Om are used (Z, Psi may be None); see
    the module docstring.

    ``id_mode``: "sum" takes the ID of M = M_Y + M_Z (Algorithm 1 writes the
    sum); "concat" takes it of the concatenation [M_Y, M_Z] (the form of the
    simultaneous skeletonization of Sec. 3.1, where one skeleton set serves
    the rows and the columns).  For the symmetric variant both reduce to the
    ID of M_Y.  ``rank_tol`` > 0 replaces the fixed rank by the numerical
    rank of the ID's sketch relative to ||[Y_B Z_B]||_F (capped at k); the
    boxes and their order stay those of the fixed-rank schedule, and a box
    may then hold fewer than k (even no) active points when its level runs.

    ``col_subset``: a box with l = |B_a| + |N_a| active columns uses only the
    first s_B = min(s, l + k + p) sample columns for its nullification, ID
    and extraction, while its sparsification and elimination still update
    all s columns.  The first s_B columns of a sample pair are a sample pair
    of the same operator (Sec. 1.1), and s_B - l = k + p is the null-space
    dimension the required sample count of Sec. 4.5 gives every box; the
    variant trades the oversampling of boxes with small l for work.

    ``redraw`` = {"matvec": f, "rmatvec": g, "seed": q}: fresh samples at the
    start of every processed level after the first, against the error the
    fixed sketches carry from level to level (Sec. 4.4).  The boxes processed
    so far have turned A into V^{-1} A W^{-1} (eq. tildeA_diag), and the
    updated sketches are a sample pair of it (Sec. 1.1); a fresh pair of the
    same operator is Omega' (drawn), Y' = V^{-1} A W^{-1} Omega' and, for
    the general variant, Psi', Z' = W^{-T} A^T V^{-T} Psi', with W^{-1}, V^{-1}
    the downward and upward passes of eq. Ainvfact over the processed boxes
    and A applied by f (g for A^T) to blocks in user point order.  The r-th
    redraw takes Omega' and Psi' from ``philox.gaussian`` with words 2 r and
    2 r + 1 (rows in tree order)."""
    if id_mode not in ("sum", "concat"):
        raise ValueError("id_mode must be 'sum' or 'concat'")
    if p is None:
        p = k
    perm = tree.perm
    Y = np.array(Y, dtype=np.float64)[perm]
    Om = np.array(Om, dtype=np.float64)[perm]
    if symmetric:
        Z, Psi = Y, Om      # the same arrays: one side is updated
    else:
        Z = np.array(Z, dtype=np.float64)[perm]
        Psi = np.array(Psi, dtype=np.float64)[perm]
    s = Y.shape[1]
    sch = otree.schedule(tree, k)
    if check_samples:
        need = otree.samples_required(tree, k, p)
        if s < need:
            raise InsufficientSamples(f"s={s} < required {need}")

    nbox = tree.nbox
    remaining = [None] * nbox
    boxes_out = []
    redraws = 0
    for li, lev in enumerate(sch.levels):
        classes = sch.order[li]
        nb = sch.nbrs[lev]
        if redraw is not None and classes and boxes_out:
            redraws += 1
            _redraw(boxes_out, perm, Y, Z, Om, Psi, symmetric, redraw, redraws)
        cur = {}
        for b in tree.level_boxes[lev]:
            b = int(b)
            if tree.is_leaf[b]:
                cur[b] = np.arange(tree.pt_begin[b], tree.pt_end[b])
            else:
                cur[b] = np.sort(np.concatenate([remaining[c] for c in tree.children[b]]))
        for r in otree.representatives(tree, lev):
            r = int(r)
            if r not in cur:
                cur[r] = np.arange(tree.pt_begin[r], tree.pt_end[r])
        for cls in classes:
            for b in cls:
                Ba = cur[b]
                Na = np.sort(np.concatenate([cur[x] for x in nb[b].tolist()])) \
                    if len(nb[b]) else np.zeros(0, dtype=np.int64)
                sB = min(s, len(Ba) + len(Na) + k + p) if col_subset else s
                bf = _process_box(b, int(lev), int(sch.colour[b]), Ba, Na, Y, Z, Om, Psi,
                                  k, keep_M, symmetric, id_mode, rank_tol, sB)
                boxes_out.append(bf)
                cur[b] = bf.S
                if on_box is not None:
                    on_box(bf, Y, Z, Om, Psi)
        for b in tree.level_boxes[lev]:
            remaining[int(b)] = cur[int(b)]

    # root: remaining active indices (Algorithm 1, final step)
    if tree.nlevels == 0:
        Bt = np.arange(tree.n)
    else:
        Bt = np.sort(np.concatenate([remaining[int(b)] for b in tree.level_boxes[1]]))
    At = _right_pinv_apply(Y[Bt], Om[Bt]) if len(Bt) else np.zeros((0, 0))
    if symmetric:
        At = 0.5 * (At + At.T)
    return Factorization(tree=tree, k=k, p=p, s=s, boxes=boxes_out, Bt=Bt, At=At,
                         At_lu=sla.lu_factor(At) if len(Bt) else None, perm=perm)


def _redraw(boxes, perm, Y, Z, Om, Psi, symmetric, rd, r):
    """Fresh sample pair(s) of V^{-1} A W^{-1} over the processed boxes, in
    place in the tree-ordered sketches (see ``factor``)."""
    from . import philox
    N, s = Y.shape

    def user(x):
        out = np.empty_like(x)
        out[perm] = x
        return out

    Om_new = philox.gaussian(N, s, rd["seed"], 2 * r)
    x = Om_new.copy()
    for bf in reversed(boxes):          # W^{-1}: U then F, boxes in reverse order
        x[bf.R] -= bf.KU @ x[bf.SN]
        x[bf.S] -= bf.T.T @ x[bf.R]
    y = np.asarray(rd["matvec"](user(x)), dtype=np.float64)[perm]
    for bf in boxes:                    # V^{-1}: E then L
        y[bf.R] -= bf.T @ y[bf.S]
        y[bf.SN] -= bf.KL @ y[bf.R]
    Om[:] = Om_new
    Y[:] = y
    if symmetric:
        return
    Psi_new = philox.gaussian(N, s, rd["seed"], 2 * r + 1)
    x = Psi_new.copy()
    for bf in reversed(boxes):          # V^{-T}: L^T then E^T, reverse order
        x[bf.R] -= bf.KL.T @ x[bf.SN]
        x[bf.S] -= bf.T.T @ x[bf.R]
    z = np.asarray(rd["rmatvec"](user(x)), dtype=np.float64)[perm]
    for bf in boxes:                    # W^{-T}: F^T then U^T
        z[bf.R] -= bf.T @ z[bf.S]
        z[bf.SN] -= bf.KU.T @ z[bf.R]
    Psi[:] = Psi_new
    Z[:] = z


def _empty_box(box, lev, colour, Ba, Na, S) -> BoxFactor:
    """A box that eliminates nothing (no active points, or every point kept)."""
    z = np.zeros(0, dtype=np.int64)
    return BoxFactor(box=box, level=lev, colour=colour, Ba=Ba, Na=Na, S=S, R=z,
                     T=np.zeros((0, len(S))), XRR=np.zeros((0, 0)), lu=None,
                     KU=np.zeros((0, len(S) + len(Na))), KL=np.zeros((len(S) + len(Na), 0)))


def _process_box(box, lev, colour, Ba, Na, Y, Z, Om, Psi, k, keep_M, symmetric=False,
                 id_mode="sum", rank_tol=0.0, sB=None) -> BoxFactor:
    """One box of Algorithm 1.  The sketches' first sB columns (all by
    default) serve the nullification, the ID and the extraction; the
    sparsification and elimination update every column."""
    b = Ba.shape[0]
    C = np.concatenate([Ba, Na])
    l = C.shape[0]
    s = Y.shape[1]
    if s - l < k:
        raise InsufficientSamples(f"box {box}: s - l = {s - l} < k = {k}")
    if b == 0:
        return _empty_box(box, lev, colour, Ba, Na, Ba)
    cs = slice(0, s if sB is None else sB)
    if symmetric:
        return _process_box_symmetric(box, lev, colour, Ba, Na, C, Y, Om, k, keep_M, rank_tol, cs)
    # block nullification, eq. nullYZ (projector form, see module docstring)
    YB, ZB = Y[Ba, cs], Z[Ba, cs]
    MY, MZ = nullify(YB, Om[C, cs]), nullify(ZB, Psi[C, cs])
    M = MY + MZ if id_mode == "sum" else np.concatenate([MY, MZ], axis=1)
    norm_yz = float(np.sqrt(np.sum(YB ** 2) + np.sum(ZB ** 2)))
    # row ID of the far-field sketch (Algorithm 1, "Compute the row-ID")
    S_pos, R_pos, T, r11_min, rdiag = row_id(M, k, want_r11_min=True, rank_tol=rank_tol, ref_norm=norm_yz)
    Sg = Ba[S_pos]
    Rg = Ba[R_pos]
    if len(Rg) == 0:
        bf = _empty_box(box, lev, colour, Ba, Na, Sg)
        bf.norm_yz, bf.norm_m, bf.r11_min, bf.rdiag = norm_yz, float(np.linalg.norm(M)), r11_min, rdiag
        return bf
    # sparsification matrices E, F applied to the sketches
    Y[Rg] -= T @ Y[Sg]
    Z[Rg] -= T @ Z[Sg]
    Om[Sg] += T.T @ Om[Rg]
    Psi[Sg] += T.T @ Psi[Rg]
    # block extraction on the updated sketches, columns [R; S; N_a] (eq. pinvYZ)
    Ch = np.concatenate([Rg, Sg, Na])
    r = Rg.shape[0]
    Xy = _right_pinv_apply(Y[Rg, cs], Om[Ch, cs])          # X_{R,C}
    Xz = _right_pinv_apply(Z[Rg, cs], Psi[Ch, cs])         # (X_{C,R})^T
    XRR = Xy[:, :r]
    lu = sla.lu_factor(XRR)
    KU = sla.lu_solve(lu, Xy[:, r:])                       # X_RR^{-1} X_{R,SN}
    KL = sla.lu_solve(lu, Xz[:, r:], trans=1).T            # X_{SN,R} X_RR^{-1}
    SN = np.concatenate([Sg, Na])
    # elimination matrices L, U applied to the sketches
    Y[SN] -= KL @ Y[Rg]
    Om[Rg] += KU @ Om[SN]
    Z[SN] -= KU.T @ Z[Rg]
    Psi[Rg] += KL.T @ Psi[SN]
    return BoxFactor(box=box, level=lev, colour=colour, Ba=Ba, Na=Na, S=Sg, R=Rg, T=T,
                     XRR=XRR, lu=lu, KU=KU, KL=KL, M=M if keep_M else None,
                     norm_yz=norm_yz, norm_m=float(np.linalg.norm(M)), r11_min=r11_min, rdiag=rdiag)


def _process_box_symmetric(box, lev, colour, Ba, Na, C, Y, Om, k, keep_M, rank_tol=0.0,
                           cs=slice(None)) -> BoxFactor:
    """One box of the symmetric variant (module docstring): the Y / Omega side
    of the general step, X_RR symmetrized, K_L = K_U^T.  The ID of M_Y equals
    that of M_Y + M_Z = 2 M_Y, whose R is twice M_Y's: the rank threshold
    rank_tol * ||[Y_B Z_B]|| is halved accordingly."""
    YB = Y[Ba, cs]
    M = nullify(YB, Om[C, cs])
    norm_yz = float(np.sqrt(2.0 * np.sum(YB ** 2)))
    S_pos, R_pos, T, r11_min, rdiag = row_id(M, k, want_r11_min=True, rank_tol=rank_tol, ref_norm=0.5 * norm_yz)
    rdiag = 2.0 * rdiag
    Sg = Ba[S_pos]
    Rg = Ba[R_pos]
    if len(Rg) == 0:
        bf = _empty_box(box, lev, colour, Ba, Na, Sg)
        bf.norm_yz, bf.norm_m, bf.r11_min = norm_yz, float(2.0 * np.linalg.norm(M)), 2.0 * r11_min
        bf.rdiag = rdiag
        return bf
    Y[Rg] -= T @ Y[Sg]
    Om[Sg] += T.T @ Om[Rg]
    Ch = np.concatenate([Rg, Sg, Na])
    r = Rg.shape[0]
    Xy = _right_pinv_apply(Y[Rg, cs], Om[Ch, cs])
    XRR = 0.5 * (Xy[:, :r] + Xy[:, :r].T)
    lu = sla.lu_factor(XRR)
    KU = sla.lu_solve(lu, Xy[:, r:])
    KL = KU.T.copy()
    SN = np.concatenate([Sg, Na])
    Y[SN] -= KL @ Y[Rg]
    Om[Rg] += KU @ Om[SN]
    return BoxFactor(box=box, level=lev, colour=colour, Ba=Ba, Na=Na, S=Sg, R=Rg, T=T,
                     XRR=XRR, lu=lu, KU=KU, KL=KL, M=M if keep_M else None,
                     norm_yz=norm_yz, norm_m=float(2.0 * np.linalg.norm(M)), r11_min=2.0 * r11_min,
                     rdiag=rdiag)


# ----------------------------------------------------------------------------
# Using the factorization: eq. Afact (forward) and eq. Ainvfact (inverse).
# Index form of each elementary factor, for T (r x k), K_U, K_L as above:
#   E: x_R -= T x_S          F: x_S -= T^T x_R
#   L: x_SN -= K_L x_R       U: x_R -= K_U x_SN
# V^{-1} = L E and W^{-1} = F U (eq. tildeA_diag).
# ----------------------------------------------------------------------------

def _as2d(x):
    x = np.asarray(x, dtype=np.float64)
    return (x[:, None], True) if x.ndim == 1 else (x, False)


def solve(F: Factorization, f, transpose: bool = False) -> np.ndarray:
    """u ~ A^{-1} f (or A^{-T} f) in user order, eq. Ainvfact."""
    f, vec = _as2d(f)
    x = f[F.perm].copy()
    if not transpose:
        for bf in F.boxes:                      # upward pass V_1^{-1} ... V_M^{-1}
            x[bf.R] -= bf.T @ x[bf.S]            # E
            x[bf.SN] -= bf.KL @ x[bf.R]          # L
        u = np.empty_like(x)
        for bf in F.boxes:                       # D^{-1}
            if len(bf.R):
                u[bf.R] = sla.lu_solve(bf.lu, x[bf.R])
        if len(F.Bt):
            u[F.Bt] = sla.lu_solve(F.At_lu, x[F.Bt])
        for bf in reversed(F.boxes):             # downward pass W_M^{-1} ... W_1^{-1}
            u[bf.R] -= bf.KU @ u[bf.SN]          # U
            u[bf.S] -= bf.T.T @ u[bf.R]          # F
    else:
        for bf in F.boxes:                       # W_1^{-T} ... : F^T then U^T
            x[bf.R] -= bf.T @ x[bf.S]
            x[bf.SN] -= bf.KU.T @ x[bf.R]
        u = np.empty_like(x)
        for bf in F.boxes:
            if len(bf.R):
                u[bf.R] = sla.lu_solve(bf.lu, x[bf.R], trans=1)
        if len(F.Bt):
            u[F.Bt] = sla.lu_solve(F.At_lu, x[F.Bt], trans=1)
        for bf in reversed(F.boxes):             # ... V_1^{-T}: L^T then E^T
            u[bf.R] -= bf.KL.T @ u[bf.SN]
            u[bf.S] -= bf.T.T @ u[bf.R]
    out = np.empty_like(u)
    out[F.perm] = u
    return out[:, 0] if vec else out


def apply(F: Factorization, x, transpose: bool = False) -> np.ndarray:
    """A_approx x (or A_approx^T x) in user order, eq. Afact."""
    x, vec = _as2d(x)
    y = x[F.perm].copy()
    if not transpose:
        for bf in F.boxes:                       # W_M ... W_1 x: W = U^{-1} F^{-1}
            y[bf.S] += bf.T.T @ y[bf.R]          # F^{-1}
            y[bf.R] += bf.KU @ y[bf.SN]          # U^{-1}
        z = y.copy()
        for bf in F.boxes:                       # D
            z[bf.R] = bf.XRR @ y[bf.R]
        z[F.Bt] = F.At @ y[F.Bt]
        for bf in reversed(F.boxes):             # V_1 ... V_M: V = E^{-1} L^{-1}
            z[bf.SN] += bf.KL @ z[bf.R]          # L^{-1}
            z[bf.R] += bf.T @ z[bf.S]            # E^{-1}
    else:
        for bf in F.boxes:                       # V^T = L^{-T} E^{-T}
            y[bf.S] += bf.T.T @ y[bf.R]          # E^{-T}
            y[bf.R] += bf.KL.T @ y[bf.SN]        # L^{-T}
        z = y.copy()
        for bf in F.boxes:
            z[bf.R] = bf.XRR.T @ y[bf.R]
        z[F.Bt] = F.At.T @ y[F.Bt]
        for bf in reversed(F.boxes):             # W^T = F^{-T} U^{-T}
            z[bf.SN] += bf.KU.T @ z[bf.R]        # U^{-T}
            z[bf.R] += bf.T @ z[bf.S]            # F^{-T}
    out = np.empty_like(z)
    out[F.perm] = z
    return out[:, 0] if vec else out


def refine(F: Factorization, matvec, f, tol: float = 1e-10, maxit: int = 10):
    """Iterative refinement u_{j+1} = u_j + A_approx^{-1}(f - A u_j) with the
    residual from the black-box product.  Returns (u, relres history)."""
    f, vec = _as2d(f)
    fn = np.linalg.norm(f, axis=0)
    fn[fn == 0] = 1.0
    u = solve(F, f)
    hist = []
    for _ in range(maxit + 1):
        r = f - matvec(u)
        rel = float(np.max(np.linalg.norm(r, axis=0) / fn))
        hist.append(rel)
        if rel <= tol or len(hist) > maxit:
            break
        u = u + solve(F, r)
    return (u[:, 0] if vec else u), hist


# ----------------------------------------------------------------------------
# Error metrics, eq. error: relerr = ||A - A_approx|| / ||A||,
# errsolve = ||I - A_approx^{-1} A||; exact 2-norms for small N, otherwise
# power iteration on E^T E (30 steps, seeded Gaussian start).
# ----------------------------------------------------------------------------

def dense_approx(F: Factorization) -> np.ndarray:
    n = F.tree.n
    return apply(F, np.eye(n))


def dense_inverse(F: Factorization) -> np.ndarray:
    n = F.tree.n
    return solve(F, np.eye(n))


def relerr(F: Factorization, A, exact_limit: int = 4096, iters: int = 30, seed: int = 7):
    n = F.tree.n
    if n <= exact_limit and not callable(A):
        Ad = np.asarray(A)
        return float(np.linalg.norm(Ad - dense_approx(F), 2) / np.linalg.norm(Ad, 2))
    mv = A if callable(A) else (lambda x: A @ x)
    mvt = None if callable(A) else (lambda x: A.T @ x)
    num = _power(lambda x: mv(x) - apply(F, x), lambda x: mvt(x) - apply(F, x, True), n, iters, seed)
    den = _power(mv, mvt, n, iters, seed + 1)
    return num / den


def errsolve(F: Factorization, A, exact_limit: int = 4096, iters: int = 30, seed: int = 7):
    n = F.tree.n
    if n <= exact_limit:
        Ad = np.asarray(A)
        return float(np.linalg.norm(np.eye(n) - dense_inverse(F) @ Ad, 2))
    return _power(lambda x: x - solve(F, A @ x), lambda x: x - A.T @ solve(F, x, True),
                  n, iters, seed)


def _power(op, opt, n, iters, seed):
    x = np.random.default_rng(seed).standard_normal(n)
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = opt(op(x))
        lam = float(np.linalg.norm(y))
        if lam == 0.0:
            return 0.0
        x = y / lam
    return float(np.sqrt(lam))


# ----------------------------------------------------------------------------
# Preconditioned GMRES (Sec. 5: the factorization as a preconditioner for
# GMRES, counted in iterations n_iter).  Right preconditioning: GMRES on
# A M^{-1} y = f with M^{-1} = A_approx^{-1} (the solve above), x = M^{-1} y,
# so the residual GMRES minimises is the true one, f - A x.  Arnoldi by
# modified Gram-Schmidt, Givens rotations for the least-squares problem,
# restarted every `restart` steps from the true residual.
# ----------------------------------------------------------------------------

def gmres(F: Factorization, matvec, f, tol: float = 1e-10, restart: int = 30, maxit: int = 200):
    """Returns (x, iterations per column, relative residual history per
    column: the Arnoldi estimate after each step, then the true residual
    at the end)."""
    f, vec = _as2d(f)
    n, w = f.shape
    X = np.zeros_like(f)
    iters, hists = [], []
    for c in range(w):
        b = f[:, c]
        bn = np.linalg.norm(b)
        x = np.zeros(n)
        if bn == 0.0:
            iters.append(0)
            hists.append([0.0])
            continue
        r = b.copy()
        beta = bn
        it = 0
        hist = [1.0]
        while beta > tol * bn and it < maxit:
            m = min(restart, maxit - it)
            V = np.zeros((m + 1, n))
            H = np.zeros((m + 1, m))
            cs, sn = np.zeros(m), np.zeros(m)
            g = np.zeros(m + 1)
            g[0] = beta
            V[0] = r / beta
            j_done = 0
            for j in range(m):
                wv = matvec(solve(F, V[j]))
                for i in range(j + 1):
                    H[i, j] = wv @ V[i]
                    wv = wv - H[i, j] * V[i]
                H[j + 1, j] = np.linalg.norm(wv)
                if H[j + 1, j] > 0.0:
                    V[j + 1] = wv / H[j + 1, j]
                for i in range(j):      # earlier rotations on the new column
                    t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                    H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                    H[i, j] = t
                den = np.hypot(H[j, j], H[j + 1, j])
                cs[j], sn[j] = (H[j, j] / den, H[j + 1, j] / den) if den > 0.0 else (1.0, 0.0)
                H[j, j] = den
                H[j + 1, j] = 0.0
                g[j + 1] = -sn[j] * g[j]
                g[j] = cs[j] * g[j]
                it += 1
                j_done = j + 1
                hist.append(abs(g[j + 1]) / bn)
                if abs(g[j + 1]) <= tol * bn or it >= maxit:
                    break
            y = sla.solve_triangular(H[:j_done, :j_done], g[:j_done], lower=False)
            x = x + solve(F, V[:j_done].T @ y)
            r = b - matvec(x)
            beta = np.linalg.norm(r)
        hist.append(beta / bn)
        X[:, c] = x
        iters.append(it)
        hists.append(hist)
    return (X[:, 0] if vec else X), iters, hists
