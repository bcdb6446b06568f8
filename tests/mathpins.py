"""Independent mathematics used to pin the oracle (pure Python, exact).

Nothing here is shared with the oracle or the GPU path.  Modularity is
computed from the textbook pair form (Newman and Girvan; the sum over
vertex pairs of A_ij - k_i k_j / 2m on equal communities), not from the
paper's per-community eq. 3, and move gains are found by recomputing Q
after the move, not from a gain formula.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def dense(row_ptr, col, w, n):
    """Dense adjacency A (python ints) from a symmetric CSR."""
    A = [[0] * n for _ in range(n)]
    for i in range(n):
        for e in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            A[i][int(col[e])] += int(w[e])
    return A


def q_pair_form(A, labels) -> Fraction:
    """Q = (1/2m) * sum_{i,j} [A_ij - k_i k_j / 2m] * [c_i == c_j],
    k_i = sum_j A_ij, 2m = sum_i k_i (loops stored once on the diagonal)."""
    n = len(A)
    k = [sum(r) for r in A]
    two_m = sum(k)
    if two_m == 0:
        return Fraction(0)
    tot = Fraction(0)
    for i in range(n):
        for j in range(n):
            if labels[i] == labels[j]:
                tot += Fraction(A[i][j]) - Fraction(k[i] * k[j], two_m)
    return tot / two_m


def q_int_pair_form(A, labels) -> int:
    """(2m)^2 * Q from the pair form, as an exact integer."""
    k = [sum(r) for r in A]
    two_m = sum(k)
    n = len(A)
    s = 0
    for i in range(n):
        for j in range(n):
            if labels[i] == labels[j]:
                s += two_m * A[i][j] - k[i] * k[j]
    return s


def set_partitions(n):
    """All set partitions of {0..n-1} as restricted-growth label lists."""
    if n == 0:
        yield []
        return
    a = [0] * n

    def rec(i, m):
        if i == n:
            yield list(a)
            return
        for v in range(m + 2):
            a[i] = v
            yield from rec(i + 1, max(m, v))

    yield from rec(1, 0)


def max_modularity(A):
    """max over all partitions of (2m)^2 * Q (brute force, tiny n only)."""
    best = None
    for p in set_partitions(len(A)):
        v = q_int_pair_form(A, p)
        if best is None or v > best:
            best = v
    return best


def expected_move(A, labels, i, singlet_rule=True):
    """Decision of vertex i in one synchronous sweep, found by brute force:
    try every neighbouring community C != C(i) (a neighbour j != i with
    c_j = C), recompute Q after moving i alone, keep the largest gain with
    ties to the smallest label, move iff that gain is > 0, and apply the
    singlet minimum-label rule with community sizes taken before the sweep."""
    n = len(A)
    ci = labels[i]
    base = q_pair_form(A, labels)
    cands = sorted({labels[j] for j in range(n) if j != i and A[i][j] > 0 and labels[j] != ci})
    best, gbest = None, None
    for C in cands:
        moved = list(labels)
        moved[i] = C
        g = q_pair_form(A, moved) - base
        if best is None or g > gbest:
            best, gbest = C, g
    if best is None or gbest <= 0:
        return ci
    size = {}
    for x in labels:
        size[x] = size.get(x, 0) + 1
    if singlet_rule and size[ci] == 1 and size[best] == 1 and best > ci:
        return ci
    return best


def contract_dense(A, new_labels, k):
    """P^T A P with P the n x k membership matrix (numpy int64 matmul)."""
    n = len(A)
    P = np.zeros((n, k), dtype=np.int64)
    for i, a in enumerate(new_labels):
        P[i, a] = 1
    M = np.array(A, dtype=np.int64)
    return P.T @ M @ P


def expected_merge(A, labels, i, singlet_rule=True):
    """Decision of vertex i in the final merge, by brute force: only a vertex
    alone in its community whose neighbours j != i all carry one label C is
    considered; it joins C iff recomputing Q with i moved there gains
    strictly, unless the singlet minimum-label rule (sizes before the merge)
    blocks it."""
    n = len(A)
    ci = labels[i]
    size = {}
    for x in labels:
        size[x] = size.get(x, 0) + 1
    if size[ci] != 1:
        return ci
    nbr = {labels[j] for j in range(n) if j != i and A[i][j] > 0}
    if len(nbr) != 1:
        return ci
    (C,) = nbr
    moved = list(labels)
    moved[i] = C
    if q_pair_form(A, moved) - q_pair_form(A, labels) <= 0:
        return ci
    if singlet_rule and size[C] == 1 and C > ci:
        return ci
    return C
