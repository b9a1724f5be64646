"""Dimension-tree schedules and their flop counts (test oracle).

Section 2.5 (dimension trees for ALS) and Section 3.2.3 (dimension trees for
the pairwise perturbation operators).  Modes are 1-based in this module to
match the paper's rule for the PP tree.
"""
from __future__ import annotations

from math import comb, prod

import numpy as np

from . import cp


def pp_tree(N):
    """Nodes of the PP dimension tree for an order-N tensor (Section 3.2.3).

    Level l (2 <= l <= N-1) holds the C(l+1, 2) tensors
    M^(i, j, l+2, .., N) with i < j <= l+1.  Each is obtained from a
    level-(l-1) tensor by contracting one mode w with A^(w); at level 2 the
    parent is X itself.

    Reading of the (typographically damaged) rule for w: w = l+1 when
    j <= l; otherwise (j = l+1) w = max({l-1, l} minus {i}).  The parent's
    mode set is then {i, j, w, l+2, .., N}, which is always a level-(l-1)
    node.

    Returns a list of (level, child_modes, parent_modes, w).
    """
    nodes = []
    for l in range(2, N):
        tail = tuple(range(l + 2, N + 1))
        for i in range(1, l + 2):
            for j in range(i + 1, l + 2):
                if j <= l:
                    w = l + 1
                else:
                    w = max({l - 1, l} - {i})
                parent = tuple(sorted({i, j, w} | set(tail)))
                nodes.append((l, (i, j) + tail, parent, w))
    return nodes


def pp_tree_build_flops(shape, R):
    """Flops of the operator build: 2 * (#elements of the parent incl. the
    rank index) per child; at level 2 the parent X has no rank index, and the
    contraction costs 2 R prod(s)."""
    total = 0
    for (l, child, parent, w) in pp_tree(len(shape)):
        total += 2 * R * prod(shape[m - 1] for m in parent)
    return total


def pp_build_flops_formula(s, N, R):
    """Closed form of Section 3.2.3: 2 R sum_{l=2}^{N-1} C(l+1, 2) s^(N-l+2)."""
    return 2 * R * sum(comb(l + 1, 2) * s ** (N - l + 2) for l in range(2, N))


def execute_pp_tree(X, A):
    """Evaluate the PP tree level by level with single-mode contractions and
    return {(i, j): M^(i,j)} (1-based keys).  Used to check the parent rule
    against the direct definition of each operator."""
    N = X.ndim
    store = {tuple(range(1, N + 1)): X}
    for (l, child, parent, w) in pp_tree(N):
        src = store[parent]
        pos = parent.index(w)
        if parent == tuple(range(1, N + 1)):
            # X has no rank index: out(..., k) = sum_x X(.., x, ..) A(x, k)
            out = np.tensordot(src, A[w - 1], axes=([pos], [0]))
        else:
            # column-wise contraction of an intermediate that carries k last
            src_m = np.moveaxis(src, pos, -2)          # (..., x, k)
            out = np.einsum("...xk,xk->...k", src_m, A[w - 1])
        store[child] = out
    return {(c[0], c[1]): store[c] for (l, c, p, w) in pp_tree(N) if l == N - 1}


def dt_als_level1_flops(shape, R):
    """Leading cost of all MTTKRPs in one ALS sweep with a binary dimension tree:
    two first-level contractions of X, 2 R prod(s) each, i.e. 4 s^N R for an
    equidimensional tensor (Section 2.5)."""
    return 4 * R * prod(shape)

