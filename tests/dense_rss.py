"""Dense, operator-level replay of Algorithm 1 used to pin the oracle.

Every strong skeletonization step is carried out on the full N x N matrix by
multiplying it with the explicit elimination matrices of the paper:

    X = U_T A L_T                     (Section 3.1, the U_T / L_T pair)
    X[R, F] = X[F, R] = 0             (far-field blocks dropped after the ID)
    A <- L X U                        (eq. landu with I = R, J = S u N, K = F)

and the factorization is rebuilt as F = (prod V_i) D (prod' W_i) with
V_i = U_T^{-1} L^{-1} and W_i = U^{-1} L_T^{-1} (eq. skelop, eq. rss; the
permutation P is the identity because everything is indexed globally).

With p.hybrid (RS-WS, Section 3.4, Algorithm 2) every level first runs weak steps: the
ID rows are all active DOFs at distance 1 and 2 plus the proxies, X[R, C] = X[C, R] = 0
for every active DOF C outside the box, and the elimination has J = S; one more weak pass
runs at depth 1 after the strong pass at depth 2.

With p.max_box > 0 the recursion ends after the first level whose parent boxes would
hold more than max_box active DOFs (counted here from the geometry and the active mask);
the final weak pass of RS-WS is skipped when the depth-1 boxes would.

Box membership, near/far sets and the active mask are computed here from the
geometry directly, not from the oracle's block store or level transitions.  Only
the ID itself (`cpqr_id`, pinned separately against LAPACK) is shared.
"""
from __future__ import annotations

import numpy as np

from oracle import rss_oracle as O


def _box_of(pts, t, lo, side):
    s = (2.0 ** t) / side
    c = np.clip(np.floor((pts - lo) * s).astype(np.int64), 0, 2 ** t - 1)
    return c[:, 0], c[:, 1]


def replay(pts: np.ndarray, p: O.Params, check_far_unmodified: bool = True):
    """Run Algorithm 1 densely.  Returns a dict of per-step data and the final F."""
    n = len(pts)
    K = O.dense_matrix(pts, p)
    A = K.copy()
    tree = O.build_tree(pts, p)
    lo, side = tree.lo, tree.side
    D = tree.depth
    active = np.ones(n, dtype=bool)
    steps = []
    far_checks = 0
    level_start = {}
    def eliminate(A, S, R, J, T, UT, LT, X, kind, t, c):
        XRRinv = np.linalg.inv(X[np.ix_(R, R)])
        E = X[np.ix_(J, R)] @ XRRinv
        G = XRRinv @ X[np.ix_(R, J)]
        L = np.eye(n)
        L[np.ix_(J, R)] = -E
        U = np.eye(n)
        U[np.ix_(R, J)] = -G
        A = L @ X @ U
        keep = A[np.ix_(R, R)].copy()
        A[R, :] = 0.0
        A[:, R] = 0.0
        A[np.ix_(R, R)] = keep
        active[R] = False
        steps.append(dict(depth=t, box=c, S=S, R=R, J=J, T=T, E=E, G=G, XRR=keep, kind=kind,
                          V=np.linalg.inv(UT) @ np.linalg.inv(L), W=np.linalg.inv(U) @ np.linalg.inv(LT),
                          A_after=A.copy()))
        return A

    def weak_pass(A, t):
        nb = 2 ** t
        bx, by = _box_of(pts, t, lo, side)
        order = sorted(range(nb * nb), key=lambda b: ((b % nb) % 3 + 3 * ((b // nb) % 3), b))
        for c in order:
            cx, cy = c % nb, c // nb
            dist = np.maximum(np.abs(bx - cx), np.abs(by - cy))
            Bc = np.nonzero(active & (dist == 0))[0]
            if len(Bc) == 0:
                continue
            Cbox = [(bx[i] + nb * by[i], i) for i in np.nonzero(active & ((dist == 1) | (dist == 2)))[0]]
            Cset = np.array([i for _, i in sorted(Cbox)], dtype=np.int64)
            prox = O.proxy_points(c, t, tree, p)
            M = np.vstack([A[np.ix_(Cset, Bc)], O.kernel_block(prox, pts[Bc], p)])
            spos, rpos, T = O.id_sorted(O.cpqr_id(M, p.tol))
            if len(rpos) == 0:
                continue
            S, R = Bc[spos], Bc[rpos]
            UT = np.eye(n)
            UT[np.ix_(R, S)] = -T.T
            LT = np.eye(n)
            LT[np.ix_(S, R)] = -T
            X = UT @ A @ LT
            outside = np.nonzero(active & (dist >= 1))[0]
            X[np.ix_(R, outside)] = 0.0
            X[np.ix_(outside, R)] = 0.0
            A = eliminate(A, S, R, S, T, UT, LT, X, "weak", t, c)
        return A

    def parent_too_large(t):
        # p.max_box: the largest box one level up, counted from the geometry and the mask
        if p.max_box <= 0:
            return False
        nb = 2 ** (t - 1)
        bx, by = _box_of(pts, t - 1, lo, side)
        return np.bincount((bx + nb * by)[active], minlength=nb * nb).max(initial=0) > p.max_box

    top_depth = D
    for t in range(D, 1, -1):
        top_depth = t
        level_start[t] = A.copy()
        if p.hybrid:
            A = weak_pass(A, t)
        nb = 2 ** t
        bx, by = _box_of(pts, t, lo, side)
        order = sorted(range(nb * nb), key=lambda b: ((b % nb) % 3 + 3 * ((b // nb) % 3), b))
        for c in order:
            cx, cy = c % nb, c // nb
            dist = np.maximum(np.abs(bx - cx), np.abs(by - cy))
            Bc = np.nonzero(active & (dist == 0))[0]
            if len(Bc) == 0:
                continue
            if check_far_unmodified:
                Pset = np.nonzero(active & (dist >= 3))[0]
                # Theorem 1 / Corollary 1: interactions with P are still those of K, bit for bit.
                assert np.array_equal(A[np.ix_(Pset, Bc)], K[np.ix_(Pset, Bc)])
                assert np.array_equal(A[np.ix_(Bc, Pset)], K[np.ix_(Bc, Pset)])
                far_checks += 1
            # O rows ordered by box index then global index (the oracle's stacking order).
            Obox = [(bx[i] + nb * by[i], i) for i in np.nonzero(active & (dist == 2))[0]]
            Oset = np.array([i for _, i in sorted(Obox)], dtype=np.int64)
            Nbox = [(bx[i] + nb * by[i], i) for i in np.nonzero(active & (dist == 1))[0]]
            Nset = np.array([i for _, i in sorted(Nbox)], dtype=np.int64)
            prox = O.proxy_points(c, t, tree, p)
            M = np.vstack([A[np.ix_(Oset, Bc)], O.kernel_block(prox, pts[Bc], p)])
            spos, rpos, T = O.id_sorted(O.cpqr_id(M, p.tol))
            if len(rpos) == 0:
                continue
            S, R = Bc[spos], Bc[rpos]
            UT = np.eye(n)
            UT[np.ix_(R, S)] = -T.T
            LT = np.eye(n)
            LT[np.ix_(S, R)] = -T
            X = UT @ A @ LT
            far = np.nonzero(active & (dist >= 2))[0]
            X[np.ix_(R, far)] = 0.0
            X[np.ix_(far, R)] = 0.0
            J = np.concatenate([S, Nset])
            A = eliminate(A, S, R, J, T, UT, LT, X, "strong", t, c)
        if parent_too_large(t):
            break
    if p.hybrid and D >= 2 and top_depth == 2 and not parent_too_large(2):
        top_depth = 1
        A = weak_pass(A, 1)
    top = np.nonzero(active)[0]
    Fm = A.copy()
    for st in reversed(steps):
        Fm = st["V"] @ Fm @ st["W"]
    return dict(steps=steps, top=top, A_final=A, F=Fm, K=K, depth=D, far_checks=far_checks,
                level_start=level_start, top_depth=top_depth)
