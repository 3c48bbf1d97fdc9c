"""Oracle: plain FP64 CPU implementation of the strong recursive skeletonization
factorization (RS-S) of Minden, Ho, Damle and Ying, "A recursive
skeletonization factorization based on strong admissibility" (arXiv:1609.08130).

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import or run this module.  The GPU library
never calls it and shares no code with it.

Everything here is slow, plain numpy in float64, following the paper's steps in
its order and notation:

* matrix entries           -- Section 1, eq. (discbie): A_ii = diag, A_ij = w*K(x_i - x_j)
* tree and near/far lists  -- Section 3, Figure 2 (uniform quadtree; near field =
                              adjacent boxes at the same level)
* interpolative decomp.    -- Section 2.2, Definition 1, by greedy column-pivoted QR
* proxy surface            -- Section 3.2, eqs. (proxytrick) and (smallid)
* strong skeletonization   -- Section 3.1, eqs. (skelid), (zab), (skelop); block
                              elimination of Section 2.1, eqs. (landu), (block_elimination)
* level sweep              -- Section 3.3, Algorithm 1; active DOFs of a parent box
                              are the union of its children's skeletons
* final factorization      -- Section 3.3, eq. (rss) and the F^{-1} formula after it
* log-determinant          -- Section 3.3 (log|D| approximates log|K|)
* generalized square root  -- Section 3.3, F^{1/2} = (prod V_i) P_t D^{1/2}, with the
                              Cholesky factor of each block of D as D^{1/2}
* hybrid factorization     -- Section 3.4, eqs. (weakskel), (rws), Algorithm 2 (RS-WS):
                              at every level a weak pass, then the strong pass

Readings of points the paper leaves open:

* O-ring / far split: O = boxes at Chebyshev distance exactly 2 (the boxes inside
  the proxy circle), P = distance >= 3, represented by the proxy points only.
* ID input is one-sided, [A(O,B); w*K(Gamma,B)], valid because K is real symmetric
  and every update keeps the matrix symmetric (Section 3.2 drops A_BF^* "for
  simplicity"; its transpose is the same matrix here).
* Proxy rows carry the same weight w as the matrix entries.
* Rank rule: stop the pivoted QR at step j > 0 once the largest trailing column
  norm is <= tol * (first pivot norm).  Pivot: among columns whose trailing norm is
  within TAU * (first pivot norm) of the largest, the one with the smallest
  position in B.  Trailing norms are recomputed at every step (no downdating).
* Box order inside a level: 3^d colouring, colour-major, ascending box index.
* DOF order inside every set: ascending global index.
* Diagonal blocks X_RR and the top block are factored by LU with partial pivoting.
* Square root: D^{1/2} = the lower Cholesky factor of each block; the adjoint uses
  W_i for V_i^* (equal for a symmetric positive definite matrix).
* RS-WS: the weak step of box c compresses its interactions with everything outside it,
  so its ID input is [A(N u O, B); w*K(Gamma, B)] (the boxes at distance 1 and 2 in
  ascending box index, then the proxies); after U_T, L_T its redundant DOFs couple only to
  its skeleton (J = S), and eliminating them updates A(S, S) alone.  Weak and strong passes
  each run in the colour-major order.  After the strong pass at depth 2 one more weak pass
  runs at depth 1 (the final weak step Section 3.4 reports using), and the top block is
  formed from what remains.
* Box-size limit (max_box > 0): when a box of the next level up would hold more than
  max_box active DOFs, the recursion ends after the current level and every active DOF
  left forms the top block (Algorithm 1 with its upper levels left uncompressed, so F
  is no less accurate).  The RS-WS final weak step at depth 1 is skipped likewise.

parity pinned by tests/test_oracle_*.py (dense operator products, LAPACK pivoted
QR, brute-force factors at tiny N, closed-form counts).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

TAU = 1e-11          # pivot tie window, relative to the first pivot norm
TMAX = 15            # deepest uniform quadtree level considered


class OracleError(Exception):
    """Invalid input or breakdown (singular pivot block)."""


@dataclass
class Params:
    dim: int = 2
    diag: float = 1.0
    weight: float = 1.0
    tol: float = 1e-6
    leaf_size: int = 64
    n_proxy: int = 16
    proxy_radius: float = 1.25      # in box side lengths
    root_lo: tuple = (0.0, 0.0)
    root_side: float = 1.0          # <= 0: bounding square of the points
    hybrid: bool = False            # RS-WS (Section 3.4, Algorithm 2) instead of RS-S
    max_box: int = 0                # > 0: end the recursion before a level with larger boxes

    @staticmethod
    def from_dict(d: dict) -> "Params":
        return Params(**{k: d[k] for k in d if k in Params.__dataclass_fields__})


# --------------------------------------------------------------------------
# Kernel (Section 1, eq. discbie; Section 3.2: K(z) = -log|z| / (2 pi))
# --------------------------------------------------------------------------

def kernel_coeff(p: Params) -> float:
    """w*K(z) = c * log(|z|^2) with c = -w / (4 pi)."""
    return -p.weight / (4.0 * np.pi)


def kernel_block(xt: np.ndarray, xs: np.ndarray, p: Params) -> np.ndarray:
    """w*K(x_t - x_s) for distinct target/source points (no diagonal handling)."""
    dx = xt[:, 0][:, None] - xs[:, 0][None, :]
    dy = xt[:, 1][:, None] - xs[:, 1][None, :]
    return kernel_coeff(p) * np.log(dx * dx + dy * dy)


def matrix_block(pts: np.ndarray, gi: np.ndarray, gj: np.ndarray, p: Params) -> np.ndarray:
    """A(gi, gj) with A_ii = diag and A_ij = w*K(x_i - x_j) for i != j."""
    gi = np.asarray(gi, dtype=np.int64)
    gj = np.asarray(gj, dtype=np.int64)
    same = gi[:, None] == gj[None, :]
    xi, xj = pts[gi], pts[gj]
    dx = xi[:, 0][:, None] - xj[:, 0][None, :]
    dy = xi[:, 1][:, None] - xj[:, 1][None, :]
    r2 = dx * dx + dy * dy
    r2 = np.where(same, 1.0, r2)
    out = kernel_coeff(p) * np.log(r2)
    out[same] = p.diag
    return out


def dense_matrix(pts: np.ndarray, p: Params) -> np.ndarray:
    g = np.arange(len(pts))
    return matrix_block(pts, g, g, p)


# --------------------------------------------------------------------------
# Uniform quadtree (Section 3, Figure 2)
# --------------------------------------------------------------------------

def root_box(pts: np.ndarray, p: Params):
    if p.root_side > 0:
        lo = np.asarray(p.root_lo, dtype=np.float64)
        side = float(p.root_side)
    else:
        lo = pts.min(axis=0)
        side = float((pts.max(axis=0) - lo).max())
        if side == 0.0:
            side = 1.0
    if np.any(pts < lo) or np.any(pts > lo + side):
        raise OracleError("point outside the root box")
    return lo, side


def box_coords(pts: np.ndarray, t: int, lo: np.ndarray, side: float) -> np.ndarray:
    """Integer box coordinates at depth t: floor((x - lo) * (2^t / side)), clamped."""
    s = (2.0 ** t) / side
    c = np.floor((pts - lo) * s).astype(np.int64)
    return np.clip(c, 0, 2 ** t - 1)


@dataclass
class Tree:
    depth: int
    lo: np.ndarray
    side: float
    leaf_lists: list      # per leaf box (linear index bx + nb*by): sorted global indices


def build_tree(pts: np.ndarray, p: Params) -> Tree:
    """Uniform tree: the shallowest depth D at which no box holds more than leaf_size points."""
    if p.dim != 2:
        raise OracleError("only d = 2 is implemented")
    n = len(pts)
    if n < 1 or p.leaf_size < 1:
        raise OracleError("bad sizes")
    if not np.all(np.isfinite(pts)):
        raise OracleError("non-finite point")
    if len(np.unique(pts, axis=0)) != n:
        raise OracleError("duplicate points")
    lo, side = root_box(pts, p)
    for t in range(TMAX + 1):
        c = box_coords(pts, t, lo, side)
        nb = 2 ** t
        lin = c[:, 0] + nb * c[:, 1]
        counts = np.bincount(lin, minlength=nb * nb)
        if counts.max() <= p.leaf_size:
            order = np.argsort(lin, kind="stable")   # ascending global index inside each box
            starts = np.concatenate([[0], np.cumsum(counts)])
            lists = [order[starts[b]:starts[b + 1]].astype(np.int64) for b in range(nb * nb)]
            return Tree(depth=t, lo=lo, side=side, leaf_lists=lists)
    raise OracleError("tree deeper than TMAX")


def cheb(a: int, b: int, nb: int) -> int:
    return max(abs(a % nb - b % nb), abs(a // nb - b // nb))


def ring(box: int, nb: int, dist: int) -> list:
    """Boxes at Chebyshev distance exactly `dist` from `box`, ascending linear index."""
    bx, by = box % nb, box // nb
    out = []
    for dy in range(-dist, dist + 1):
        for dx in range(-dist, dist + 1):
            if max(abs(dx), abs(dy)) != dist:
                continue
            x, y = bx + dx, by + dy
            if 0 <= x < nb and 0 <= y < nb:
                out.append(x + nb * y)
    return out


def colour(box: int, nb: int) -> int:
    return (box % nb) % 3 + 3 * ((box // nb) % 3)


def level_order(nb: int) -> list:
    """Colour-major box order of one level (Section 5 colouring, widened to 3^d colours)."""
    boxes = list(range(nb * nb))
    return sorted(boxes, key=lambda b: (colour(b, nb), b))


def proxy_points(box: int, t: int, tree: Tree, p: Params) -> np.ndarray:
    """n_p equispaced points on the circle of radius proxy_radius * side around the box centre."""
    nb = 2 ** t
    side_t = tree.side / (2.0 ** t)
    cx = tree.lo[0] + (box % nb + 0.5) * side_t
    cy = tree.lo[1] + (box // nb + 0.5) * side_t
    rr = p.proxy_radius * side_t
    th = 2.0 * np.pi * np.arange(p.n_proxy) / p.n_proxy
    return np.stack([cx + rr * np.cos(th), cy + rr * np.sin(th)], axis=1)


# --------------------------------------------------------------------------
# Interpolative decomposition by greedy column-pivoted QR (Section 2.2)
# --------------------------------------------------------------------------

@dataclass
class IDResult:
    k: int
    perm: np.ndarray      # pivot order (positions in B)
    T0: np.ndarray        # k x (n-k), columns perm[k:] ~ columns perm[:k] @ T0
    rdiag: np.ndarray     # |R_jj| of the k accepted pivots


def cpqr_id(M: np.ndarray, tol: float, tau: float = TAU) -> IDResult:
    """Householder QR with column pivoting, stopped by the tolerance rule above."""
    A = np.array(M, dtype=np.float64, copy=True)
    m, n = A.shape
    perm = np.arange(n)
    kmax = min(m, n)
    r0 = 0.0
    k = 0
    rdiag = []
    for j in range(kmax):
        nu = np.sum(A[j:, j:] * A[j:, j:], axis=0)
        mu = float(np.sqrt(nu.max()))
        if j == 0:
            if mu == 0.0:
                break
            r0 = mu
        elif mu <= tol * r0:
            break
        cand = np.nonzero(np.sqrt(nu) >= mu - tau * r0)[0] + j
        piv = cand[np.argmin(perm[cand])]
        if piv != j:
            A[:, [j, piv]] = A[:, [piv, j]]
            perm[[j, piv]] = perm[[piv, j]]
        # Householder reflector H = I - tau_h v v^T with v_0 = 1 maps A[j:, j] to beta e_0
        alpha = A[j, j]
        x = A[j + 1:, j]
        sigma = float(x @ x)
        if sigma != 0.0:
            beta = -np.copysign(np.sqrt(alpha * alpha + sigma), alpha)
            tau_h = (beta - alpha) / beta
            v = x / (alpha - beta)
            A[j, j] = beta
            A[j + 1:, j] = 0.0
            w = A[j, j + 1:] + v @ A[j + 1:, j + 1:]
            A[j, j + 1:] -= tau_h * w
            A[j + 1:, j + 1:] -= tau_h * np.outer(v, w)
        rdiag.append(abs(A[j, j]))
        k = j + 1
    if k > 0 and k < n:
        T0 = sla.solve_triangular(A[:k, :k], A[:k, k:], lower=False)
    else:
        T0 = np.zeros((k, n - k))
    return IDResult(k=k, perm=perm, T0=T0, rdiag=np.array(rdiag))


def id_sorted(res: IDResult):
    """Skeleton / redundant positions, each ascending, and T re-indexed to that order."""
    k = res.k
    s_piv, r_piv = res.perm[:k], res.perm[k:]
    so, ro = np.argsort(s_piv), np.argsort(r_piv)
    return s_piv[so], r_piv[ro], res.T0[np.ix_(so, ro)]


# --------------------------------------------------------------------------
# RS-S factorization (Section 3.3, Algorithm 1)
# --------------------------------------------------------------------------

@dataclass
class Record:
    """One strong skeletonization step, stored in factored form (eq. skelop)."""
    depth: int
    box: int
    R: np.ndarray         # redundant DOFs (global, ascending)
    S: np.ndarray         # skeleton DOFs (global, ascending)
    J: np.ndarray         # S followed by the active near-field DOFs (global)
    T: np.ndarray         # |S| x |R| interpolation matrix
    lu: np.ndarray        # LU of X_RR (scipy layout) ...
    piv: np.ndarray       # ... and its row pivots
    E: np.ndarray         # X_JR X_RR^{-1}   (|J| x |R|)
    G: np.ndarray         # X_RR^{-1} X_RJ   (|R| x |J|)
    XRR: np.ndarray       # X_RR itself (for apply)
    kind: str = "strong"  # "weak" for the weak steps of RS-WS (J = S)


@dataclass
class Factor:
    n: int
    params: Params
    depth: int
    records: list
    top: np.ndarray               # global indices of the remaining active DOFs
    top_lu: np.ndarray
    top_piv: np.ndarray
    A_top: np.ndarray
    skeletons: dict = field(default_factory=dict)   # (depth, box) -> (S, R) global indices
    level_stats: list = field(default_factory=list)
    weak_skeletons: dict = field(default_factory=dict)   # RS-WS: (depth, box) -> (S, R) of the weak step
    top_depth: int = -1           # level whose remaining active DOFs form the top block


def _lu(X: np.ndarray):
    lu, piv = sla.lu_factor(X, check_finite=False)
    if np.any(np.diag(lu) == 0.0):
        raise OracleError("singular pivot block")
    return lu, piv


class _Level:
    """Active DOF lists and the block store of one tree level.

    store[(a, b)] holds the current A(B_a, B_b) for every ordered pair of boxes at
    Chebyshev distance <= 2.  Pairs further apart are never modified (Theorem 1,
    Corollary 1) and are regenerated from the kernel when needed.
    """

    def __init__(self, tree: Tree, t: int, B: list, store: dict):
        self.tree = tree
        self.t = t
        self.nb = 2 ** t
        self.B = B
        self.store = store

    def block(self, a: int, b: int, pts, p) -> np.ndarray:
        if cheb(a, b, self.nb) <= 2:
            return self.store[(a, b)]
        return kernel_block(pts[self.B[a]], pts[self.B[b]], p)


def _leaf_level(tree: Tree, pts, p) -> _Level:
    t = tree.depth
    nb = 2 ** t
    B = tree.leaf_lists
    store = {}
    for a in range(nb * nb):
        for d in range(3):
            for b in ([a] if d == 0 else ring(a, nb, d)):
                store[(a, b)] = matrix_block(pts, B[a], B[b], p)
    return _Level(tree, t, B, store)


def _parent_too_large(lev: _Level, p: Params) -> bool:
    """Whether a box one level up would hold more than p.max_box active DOFs."""
    if p.max_box <= 0 or lev.t < 1:
        return False
    nb = lev.nb // 2
    for P in range(nb * nb):
        px, py = P % nb, P // nb
        size = sum(len(lev.B[(2 * px + ix) + lev.nb * (2 * py + iy)]) for iy in range(2) for ix in range(2))
        if size > p.max_box:
            return True
    return False


def _parent_level(lev: _Level, pts, p) -> _Level:
    """Step up one level: B_parent = union of the children's skeletons (Section 3.3)."""
    t = lev.t - 1
    nb = 2 ** t
    cnb = lev.nb
    children = []
    B = []
    for P in range(nb * nb):
        px, py = P % nb, P // nb
        ch = [(2 * px + ix) + cnb * (2 * py + iy) for iy in range(2) for ix in range(2)]
        children.append(ch)
        B.append(np.sort(np.concatenate([lev.B[c] for c in ch])))
    store = {}
    for P in range(nb * nb):
        for d in range(3):
            for Q in ([P] if d == 0 else ring(P, nb, d)):
                blk = np.empty((len(B[P]), len(B[Q])))
                for a in children[P]:
                    ra = np.searchsorted(B[P], lev.B[a])
                    for b in children[Q]:
                        cb = np.searchsorted(B[Q], lev.B[b])
                        blk[np.ix_(ra, cb)] = lev.block(a, b, pts, p)
                store[(P, Q)] = blk
    return _Level(lev.tree, t, B, store)


def _skeletonize_box(lev: _Level, c: int, pts, p: Params):
    """Strong skeletonization of the active DOFs of box c (Sections 3.1-3.2)."""
    nb = lev.nb
    Bc = lev.B[c]
    n = len(Bc)
    if n == 0:
        return None
    O = ring(c, nb, 2)
    N = ring(c, nb, 1)
    # ID input: [A(O, B); w*K(Gamma, B)]   (eq. smallid)
    rows = [lev.store[(o, c)] for o in O]
    rows.append(kernel_block(proxy_points(c, lev.t, lev.tree, p), pts[Bc], p))
    M = np.vstack(rows)
    res = cpqr_id(M, p.tol)
    spos, rpos, T = id_sorted(res)
    if len(rpos) == 0:
        return None
    S, R = Bc[spos], Bc[rpos]
    Acc = lev.store[(c, c)]
    A_RR, A_RS = Acc[np.ix_(rpos, rpos)], Acc[np.ix_(rpos, spos)]
    A_SR, A_SS = Acc[np.ix_(spos, rpos)], Acc[np.ix_(spos, spos)]
    if N:
        A_NR = np.vstack([lev.store[(b, c)][:, rpos] for b in N])
        A_NS = np.vstack([lev.store[(b, c)][:, spos] for b in N])
        A_RN = np.hstack([lev.store[(c, b)][rpos, :] for b in N])
        A_SN = np.hstack([lev.store[(c, b)][spos, :] for b in N])
    else:
        A_NR = np.zeros((0, len(rpos)))
        A_NS = np.zeros((0, len(spos)))
        A_RN = np.zeros((len(rpos), 0))
        A_SN = np.zeros((len(spos), 0))
    # Column operation L_T (R columns minus S columns times T) and row operation U_T.
    Z_R = A_RR - A_RS @ T
    Z_S = A_SR - A_SS @ T
    Z_N = A_NR - A_NS @ T
    X_RR = Z_R - T.T @ Z_S
    X_RS = A_RS - T.T @ A_SS
    X_RN = A_RN - T.T @ A_SN
    X_JR = np.vstack([Z_S, Z_N])
    X_RJ = np.hstack([X_RS, X_RN])
    # Block elimination with I = R, J = S u N (eqs. landu, block_elimination).
    lu, piv = _lu(X_RR)
    G = sla.lu_solve((lu, piv), X_RJ, check_finite=False)
    E = sla.lu_solve((lu, piv), X_JR.T, trans=1, check_finite=False).T
    upd = X_JR @ G
    # Scatter the Schur complement update over the neighbourhood blocks.
    nbhd = [c] + N
    sizes = [len(spos)] + [len(lev.B[b]) for b in N]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    for ia, a in enumerate(nbhd):
        for ib, b in enumerate(nbhd):
            blk = upd[offs[ia]:offs[ia + 1], offs[ib]:offs[ib + 1]]
            if a == c and b == c:
                lev.store[(c, c)][np.ix_(spos, spos)] -= blk
            elif a == c:
                lev.store[(c, b)][spos, :] -= blk
            elif b == c:
                lev.store[(a, c)][:, spos] -= blk
            else:
                lev.store[(a, b)] -= blk
    # R leaves the active set: restrict every stored block of box c to S.
    for d in range(3):
        for b in ([c] if d == 0 else ring(c, nb, d)):
            if b == c:
                lev.store[(c, c)] = lev.store[(c, c)][np.ix_(spos, spos)]
            else:
                lev.store[(c, b)] = lev.store[(c, b)][spos, :]
                lev.store[(b, c)] = lev.store[(b, c)][:, spos]
    lev.B[c] = S
    J = np.concatenate([S] + [lev.B[b] for b in N]).astype(np.int64)
    return Record(depth=lev.t, box=c, R=R, S=S, J=J, T=T, lu=lu, piv=piv, E=E, G=G, XRR=X_RR)


def _weak_skeletonize_box(lev: _Level, c: int, pts, p: Params):
    """Weak skeletonization of the active DOFs of box c (Section 3.4, eq. weakskel)."""
    nb = lev.nb
    Bc = lev.B[c]
    if len(Bc) == 0:
        return None
    near = sorted(ring(c, nb, 1) + ring(c, nb, 2))
    rows = [lev.store[(o, c)] for o in near]
    rows.append(kernel_block(proxy_points(c, lev.t, lev.tree, p), pts[Bc], p))
    M = np.vstack(rows)
    spos, rpos, T = id_sorted(cpqr_id(M, p.tol))
    if len(rpos) == 0:
        return None
    S, R = Bc[spos], Bc[rpos]
    Acc = lev.store[(c, c)]
    A_RR, A_RS = Acc[np.ix_(rpos, rpos)], Acc[np.ix_(rpos, spos)]
    A_SR, A_SS = Acc[np.ix_(spos, rpos)], Acc[np.ix_(spos, spos)]
    # U_T, L_T; every interaction of R outside the box is the compressed part, dropped
    Z_R = A_RR - A_RS @ T
    Z_S = A_SR - A_SS @ T
    X_RR = Z_R - T.T @ Z_S
    X_RS = A_RS - T.T @ A_SS
    X_SR = Z_S
    # block elimination with I = R, J = S
    lu, piv = _lu(X_RR)
    G = sla.lu_solve((lu, piv), X_RS, check_finite=False)
    E = sla.lu_solve((lu, piv), X_SR.T, trans=1, check_finite=False).T
    lev.store[(c, c)][np.ix_(spos, spos)] -= X_SR @ G
    for d in range(3):
        for b in ([c] if d == 0 else ring(c, nb, d)):
            if b == c:
                lev.store[(c, c)] = lev.store[(c, c)][np.ix_(spos, spos)]
            else:
                lev.store[(c, b)] = lev.store[(c, b)][spos, :]
                lev.store[(b, c)] = lev.store[(b, c)][:, spos]
    lev.B[c] = S
    return Record(depth=lev.t, box=c, R=R, S=S, J=np.asarray(S, dtype=np.int64), T=T, lu=lu, piv=piv, E=E, G=G,
                  XRR=X_RR, kind="weak")


def _weak_pass(lev: _Level, pts, p: Params, records: list, weak_skeletons: dict):
    for c in level_order(lev.nb):
        before = lev.B[c]
        rec = _weak_skeletonize_box(lev, c, pts, p)
        if rec is not None:
            records.append(rec)
            weak_skeletons[(lev.t, c)] = (rec.S, rec.R)
        else:
            weak_skeletons[(lev.t, c)] = (before, np.zeros(0, dtype=np.int64))


def factor(pts: np.ndarray, params, hook=None) -> Factor:
    """RS-S factorization F ~ A (Algorithm 1).

    `hook(depth, B, store)`, if given, sees every level's active lists and block store
    at the start of the level (tests use it to compare with a dense replay).
    """
    p = params if isinstance(params, Params) else Params.from_dict(params)
    if not (p.tol >= 0.0) or not np.isfinite(p.tol):
        raise OracleError("bad tolerance")
    if p.n_proxy < 1 or p.proxy_radius <= 0:
        raise OracleError("bad proxy parameters")
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    tree = build_tree(pts, p)
    lev = _leaf_level(tree, pts, p)
    records = []
    skeletons = {}
    weak_skeletons = {}
    stats = []
    while lev.t >= 2:
        if hook is not None:
            hook(lev.t, lev.B, lev.store)
        if p.hybrid:
            _weak_pass(lev, pts, p, records, weak_skeletons)
        nrec = 0
        for c in level_order(lev.nb):
            before = lev.B[c]
            rec = _skeletonize_box(lev, c, pts, p)
            if rec is not None:
                records.append(rec)
                nrec += 1
                skeletons[(lev.t, c)] = (rec.S, rec.R)
            else:
                skeletons[(lev.t, c)] = (before, np.zeros(0, dtype=np.int64))
        stats.append(dict(depth=lev.t, boxes=lev.nb ** 2, records=nrec,
                          active_after=int(sum(len(b) for b in lev.B))))
        if lev.t == 2 or _parent_too_large(lev, p):
            break
        lev = _parent_level(lev, pts, p)
    if p.hybrid and lev.t == 2 and not _parent_too_large(lev, p):
        # the final weak step at depth 1 (Section 3.4)
        lev = _parent_level(lev, pts, p)
        _weak_pass(lev, pts, p, records, weak_skeletons)
    # Top block: all remaining active DOFs (Section 3.3, the final factorization).
    top = np.sort(np.concatenate(lev.B)).astype(np.int64)
    A_top = np.empty((len(top), len(top)))
    nbox = lev.nb * lev.nb
    pos = [np.searchsorted(top, lev.B[a]) for a in range(nbox)]
    for a in range(nbox):
        for b in range(nbox):
            A_top[np.ix_(pos[a], pos[b])] = lev.block(a, b, pts, p)
    top_lu, top_piv = _lu(A_top) if len(top) else (np.zeros((0, 0)), np.zeros(0, dtype=np.int32))
    return Factor(n=len(pts), params=p, depth=tree.depth, records=records, top=top,
                  top_lu=top_lu, top_piv=top_piv, A_top=A_top, skeletons=skeletons,
                  level_stats=stats, weak_skeletons=weak_skeletons, top_depth=lev.t)


# --------------------------------------------------------------------------
# Using the factorization (eq. rss and F^{-1})
# --------------------------------------------------------------------------

def solve(F: Factor, b: np.ndarray) -> np.ndarray:
    """x = F^{-1} b = (prod W_i^{-1}) P_t D^{-1} P_t^* (prod' V_i^{-1}) b."""
    z = np.array(b, dtype=np.float64, copy=True)
    for r in F.records:                       # V_i^{-1} in factor order
        z[r.R] -= r.T.T @ z[r.S]
        z[r.J] -= r.E @ z[r.R]
    for r in F.records:                       # D^{-1}
        z[r.R] = sla.lu_solve((r.lu, r.piv), z[r.R], check_finite=False)
    if len(F.top):
        z[F.top] = sla.lu_solve((F.top_lu, F.top_piv), z[F.top], check_finite=False)
    for r in reversed(F.records):             # W_i^{-1} in reverse order
        z[r.R] -= r.G @ z[r.J]
        z[r.S] -= r.T @ z[r.R]
    return z


def apply(F: Factor, x: np.ndarray) -> np.ndarray:
    """y = F x = (prod V_i) P_t D P_t^* (prod' W_i) x."""
    z = np.array(x, dtype=np.float64, copy=True)
    for r in F.records:                       # W_1 acts first
        z[r.S] += r.T @ z[r.R]
        z[r.R] += r.G @ z[r.J]
    for r in F.records:
        z[r.R] = r.XRR @ z[r.R]
    if len(F.top):
        z[F.top] = F.A_top @ z[F.top]
    for r in reversed(F.records):             # V_1 acts last
        z[r.J] += r.E @ z[r.R]
        z[r.R] += r.T.T @ z[r.S]
    return z


def logdet(F: Factor):
    """(sign, log|det F|) = log|det D|: the V_i, W_i are unit triangular."""
    sign, total = 1.0, 0.0
    blocks = [(r.lu, r.piv) for r in F.records]
    if len(F.top):
        blocks.append((F.top_lu, F.top_piv))
    for lu, piv in blocks:
        d = np.diag(lu)
        swaps = int(np.sum(piv != np.arange(len(piv))))
        sign *= (-1.0) ** swaps * np.prod(np.sign(d))
        total += float(np.sum(np.log(np.abs(d))))
    return sign, total


def _chol(X: np.ndarray) -> np.ndarray:
    try:
        return np.linalg.cholesky(X)
    except np.linalg.LinAlgError:
        raise OracleError("a diagonal block of D is not positive definite (no square root)")


def sqrt_apply(F: Factor, x: np.ndarray, adjoint: bool = False) -> np.ndarray:
    """Generalized square root of F for a positive definite matrix (Section 3.3).

    F^{1/2} = (prod V_i) P_t D^{1/2}, where D^{1/2} is the lower Cholesky factor of every
    diagonal block of D (X_RR of each record, A_top).  Since V_i = W_i^* when the matrix is
    positive definite, F = F^{1/2} (F^{1/2})^* with
    (F^{1/2})^* = D^{1/2 *} P_t^* (prod' W_i).  adjoint selects the second operator.
    """
    z = np.array(x, dtype=np.float64, copy=True)
    if not adjoint:
        for r in F.records:                       # D^{1/2} on every R block
            z[r.R] = _chol(r.XRR) @ z[r.R]
        if len(F.top):
            z[F.top] = _chol(F.A_top) @ z[F.top]
        for r in reversed(F.records):             # V_1 acts last
            z[r.J] += r.E @ z[r.R]
            z[r.R] += r.T.T @ z[r.S]
    else:
        for r in F.records:                       # W_1 acts first
            z[r.S] += r.T @ z[r.R]
            z[r.R] += r.G @ z[r.J]
        for r in F.records:                       # D^{1/2 *}
            z[r.R] = _chol(r.XRR).T @ z[r.R]
        if len(F.top):
            z[F.top] = _chol(F.A_top).T @ z[F.top]
    return z


# --------------------------------------------------------------------------
# The exact operator and the outer iteration (Section 4: K applied by FFT; CG with F)
# --------------------------------------------------------------------------

def matvec_direct(pts: np.ndarray, p: Params, x: np.ndarray, chunk: int = 2048) -> np.ndarray:
    """y = A x by direct summation (rows in chunks)."""
    n = len(pts)
    y = np.empty_like(np.asarray(x, dtype=np.float64))
    g = np.arange(n)
    for s in range(0, n, chunk):
        gi = g[s:s + chunk]
        y[s:s + chunk] = matrix_block(pts, gi, g, p) @ x
    return y


def matvec_grid_fft(n: int, p: Params, x: np.ndarray, h: float = None) -> np.ndarray:
    """y = A x for the n x n cell-centre grid (DOF i + n*j, spacing h = 1/n unless given),
    by FFT convolution.

    A - diag*I is block Toeplitz with Toeplitz blocks; its generator w*K(h*(di, dj)) with
    the zero offset set to 0 is embedded in a (2n) x (2n) circulant.
    """
    h = 1.0 / n if h is None else h
    d = np.arange(-n + 1, n) * h
    dx, dy = np.meshgrid(d, d, indexing="xy")        # [dj, di]
    r2 = dx * dx + dy * dy
    r2[n - 1, n - 1] = 1.0
    gen = kernel_coeff(p) * np.log(r2)
    gen[n - 1, n - 1] = 0.0
    c = np.zeros((2 * n, 2 * n))
    c[:n, :n] = gen[n - 1:, n - 1:]                # dj >= 0, di >= 0
    c[:n, n + 1:] = gen[n - 1:, :n - 1]            # di < 0
    c[n + 1:, :n] = gen[:n - 1, n - 1:]            # dj < 0
    c[n + 1:, n + 1:] = gen[:n - 1, :n - 1]
    X = np.asarray(x, dtype=np.float64)
    single = X.ndim == 1
    if single:
        X = X[:, None]
    out = np.empty_like(X)
    cf = np.fft.rfft2(c)
    for k in range(X.shape[1]):
        xx = np.zeros((2 * n, 2 * n))
        xx[:n, :n] = X[:, k].reshape(n, n)             # [j, i]
        yy = np.fft.irfft2(np.fft.rfft2(xx) * cf, s=(2 * n, 2 * n))
        out[:, k] = yy[:n, :n].reshape(-1) + p.diag * X[:, k]
    return out[:, 0] if single else out


def gmres(matvec, precond, b: np.ndarray, rtol: float = 1e-10, restart: int = 30,
          maxit: int = 300):
    """Right-preconditioned restarted GMRES(restart) with modified Gram-Schmidt.

    Solves A M^{-1} u = b and returns x = M^{-1} u, starting from x0 = 0.  A cycle ends
    when the Arnoldi residual estimate reaches rtol; the iteration stops when the true
    residual |b - A x| / |b| <= rtol.  Returns (x, iterations, relres).
    """
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    x = np.zeros_like(b)
    if nb == 0.0:
        return x, 0, 0.0
    it = 0
    relres = 1.0
    r = b.copy()
    while True:
        beta = float(np.linalg.norm(r))
        relres = beta / nb
        if relres <= rtol or it >= maxit:
            break
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        m = 0
        for j in range(restart):
            z = precond(V[j])
            Z.append(z)
            w = matvec(z)
            for i in range(j + 1):
                H[i, j] = float(w @ V[i])
                w = w - H[i, j] * V[i]
            hn = float(np.linalg.norm(w))
            H[j + 1, j] = hn
            for i in range(j):
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -sn[i] * a + cs[i] * c
            den = float(np.hypot(H[j, j], H[j + 1, j]))
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            m = j + 1
            if abs(g[j + 1]) / nb <= rtol or hn == 0.0 or it >= maxit:
                break
            V.append(w / hn)
        y = sla.solve_triangular(H[:m, :m], g[:m], lower=False)
        for i in range(m):
            x += y[i] * Z[i]
        r = b - matvec(x)
    return x, it, relres
