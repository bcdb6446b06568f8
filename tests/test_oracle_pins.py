"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these compare the oracle with itself: modularity is checked against
the textbook pair form, every sweep decision against a brute-force search
that recomputes Q after each candidate move, contraction against the dense
product P^T A P, renumbering against numpy's unique, the full run against
hand-derived worked examples (tests/golden) and against exhaustive search
over all partitions of tiny graphs, and the acceptance test against Python's
exact integers.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import graphgen as gg
import oracle
from mathpins import (contract_dense, dense, expected_merge, expected_move, max_modularity,
                      q_int_pair_form, q_pair_form)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def _small_graphs():
    out = []
    for s in range(24):
        n = 3 + s % 7
        out.append(gg.random_small(n, 0.45, 5, seed=100 + s, loop_prob=0.3 if s % 2 else 0.0,
                                   isolated=1 if s % 5 == 0 else 0))
    return out


def _labelings(n, seed):
    rng = np.random.default_rng(seed)
    yield np.arange(n, dtype=np.int32)
    yield np.zeros(n, dtype=np.int32)
    for k in (2, 3):
        yield gg.random_labels(n, k, seed + k)
    yield rng.integers(0, n, size=n).astype(np.int32)


# --- eq. 3 -------------------------------------------------------------------

@pytest.mark.parametrize("g", _small_graphs(), ids=lambda g: f"n{g.n}m{g.nnz}")
def test_modularity_equals_pair_form(g):
    A = dense(g.row_ptr, g.col, g.w, g.n)
    for t, lab in enumerate(_labelings(g.n, g.nnz)):
        qi, q = oracle.modularity(g.row_ptr, g.col, g.w, lab)
        assert qi == q_int_pair_form(A, lab.tolist())
        ref = q_pair_form(A, lab.tolist())
        assert abs(q - float(ref)) <= 1e-15 * max(1.0, abs(float(ref)))


def test_modularity_closed_forms():
    g = gg.random_small(9, 0.5, 7, seed=5, loop_prob=0.5)
    delta, tw = oracle.degrees(g.row_ptr, g.col, g.w)
    # singletons: Q = sum_i A_ii / TW - sum_i delta_i^2 / TW^2
    loops = sum(int(g.w[e]) for i in range(g.n) for e in range(g.row_ptr[i], g.row_ptr[i + 1])
                if g.col[e] == i)
    qi, _ = oracle.modularity(g.row_ptr, g.col, g.w, np.arange(g.n, dtype=np.int32))
    assert qi == tw * loops - int(sum(int(d) ** 2 for d in delta))
    # one community holding everything: Q = 0
    qi, q = oracle.modularity(g.row_ptr, g.col, g.w, np.zeros(g.n, np.int32))
    assert qi == 0 and q == 0.0
    # two triangles joined by a bridge, split into the triangles: Q = 5/14
    t = gg.from_edge_list(6, [(0, 1), (0, 2), (1, 2), (3, 4), (3, 5), (4, 5), (2, 3)])
    qi, q = oracle.modularity(t.row_ptr, t.col, t.w, np.array([0, 0, 0, 3, 3, 3], np.int32))
    assert Fraction(qi, 14 * 14) == Fraction(5, 14)


def test_degrees_definition():
    g = gg.random_small(12, 0.4, 9, seed=8, loop_prob=0.4)
    delta, tw = oracle.degrees(g.row_ptr, g.col, g.w)
    A = dense(g.row_ptr, g.col, g.w, g.n)
    assert delta.tolist() == [sum(r) for r in A]
    assert tw == sum(map(sum, A))


# --- one sweep: eqs. 4-5 and the two heuristics ------------------------------

@pytest.mark.parametrize("singlet", [True, False])
@pytest.mark.parametrize("g", _small_graphs()[:16], ids=lambda g: f"n{g.n}m{g.nnz}")
def test_sweep_decisions_by_brute_force(g, singlet):
    A = dense(g.row_ptr, g.col, g.w, g.n)
    for lab in _labelings(g.n, 7 * g.nnz + 1):
        lm = oracle.local_move(g.row_ptr, g.col, g.w, lab, singlet_rule=singlet)
        expect = [expected_move(A, lab.tolist(), i, singlet) for i in range(g.n)]
        assert lm.labels.tolist() == expect
        # e_{i->C(i)} including the loop, eq. 1 over the input labels
        e_own = [sum(A[i][j] for j in range(g.n) if lab[j] == lab[i]) for i in range(g.n)]
        assert lm.e_own.tolist() == e_own
        # deg_C of the new labels, eq. 2
        k = [sum(r) for r in A]
        deg = [0] * g.n
        for i in range(g.n):
            deg[lm.labels[i]] += k[i]
        assert lm.deg.tolist() == deg


def test_score_gain_identity():
    """dQ of moving i alone into C, recomputed from the pair form, equals
    2*(s(C) - s_own)/TW^2 under the reading of eq. 4 used throughout (own community
    without i, loop left out)."""
    g = gg.random_small(8, 0.5, 6, seed=31, loop_prob=0.5)
    A = dense(g.row_ptr, g.col, g.w, g.n)
    k = [sum(r) for r in A]
    tw = sum(k)
    lab = gg.random_labels(g.n, 3, 77).tolist()
    base = q_pair_form(A, lab)
    for i in range(g.n):
        ci = lab[i]
        degc = {}
        for v in range(g.n):
            degc[lab[v]] = degc.get(lab[v], 0) + k[v]
        e_to = lambda C: sum(A[i][j] for j in range(g.n) if j != i and lab[j] == C)
        s_own = tw * e_to(ci) - k[i] * (degc[ci] - k[i])
        for C in set(lab) - {ci}:
            s = tw * e_to(C) - k[i] * degc[C]
            moved = list(lab)
            moved[i] = C
            assert q_pair_form(A, moved) - base == Fraction(2 * (s - s_own), tw * tw)


# --- acceptance test (Alg. 1's relative threshold, read exactly) --------------

def test_accept_matches_exact_integers():
    rng = np.random.default_rng(3)
    cases = [(0, -34), (38, -34), (70, 38), (70, 70), (1, 0), (0, 0), (-1, 0),
             (10**6 + 1, 10**12), (10**6, 10**12), (10**6 - 1, 10**12),
             (-(10**12) + 10**6 + 1, -(10**12)), (-(10**12) + 10**6, -(10**12))]
    big = 1 << 123
    for _ in range(300):
        qp = int(rng.integers(-2**62, 2**62)) * int(rng.integers(1, 2**61))
        d = int(rng.integers(0, 2**40)) * int(rng.integers(0, 2**40))
        cases.append((qp + d, qp))
        cases.append((qp + abs(qp) // 10**6, qp))
        cases.append((qp + abs(qp) // 10**6 + 1, qp))
    cases += [(big, big - big // 10**6), (big, big - big // 10**6 - 1), (-big + 1, -big)]
    for num, den in ((1, 10**6), (3, 7), (0, 1)):
        for qn, qp in cases:
            assert oracle.accept(qn, qp, num, den) == (den * (qn - qp) > num * abs(qp)), (qn, qp)


# --- renumbering and graph rebuilding ----------------------------------------

@pytest.mark.parametrize("g", _small_graphs()[::3], ids=lambda g: f"n{g.n}m{g.nnz}")
def test_renumber_and_contract(g):
    A = dense(g.row_ptr, g.col, g.w, g.n)
    for lab in _labelings(g.n, g.nnz + 5):
        m, k = oracle.renumber(lab)
        uniq, inv = np.unique(lab, return_inverse=True)
        assert k == len(uniq)
        new = m[lab]
        assert new.tolist() == inv.tolist()
        rp2, cl2, w2 = oracle.contract(g.row_ptr, g.col, g.w, new, k)
        M = contract_dense(A, new.tolist(), k)
        got = np.zeros((k, k), np.int64)
        for a in range(k):
            seg = cl2[rp2[a]:rp2[a + 1]]
            assert np.all(np.diff(seg) > 0)          # ascending, no repeats
            got[a, seg] = w2[rp2[a]:rp2[a + 1]]
        assert np.array_equal(got, M)
        assert np.count_nonzero(M) == len(cl2)      # no zero entries stored
        assert len(cl2) <= g.nnz and k <= g.n       # Theorem 1
        # contraction preserves TW and modularity (invariants of the method)
        _, tw = oracle.degrees(g.row_ptr, g.col, g.w)
        _, tw2 = oracle.degrees(rp2, cl2, w2)
        assert tw == tw2
        qa, _ = oracle.modularity(g.row_ptr, g.col, g.w, new)
        qb, _ = oracle.modularity(rp2, cl2, w2, np.arange(k, dtype=np.int32))
        assert qa == qb


# --- the whole method: worked examples and exhaustive search -----------------

def _examples():
    with open(GOLDEN) as f:
        return json.load(f)["examples"]


@pytest.mark.parametrize("ex", _examples(), ids=lambda e: e["name"])
def test_worked_examples(ex):
    g = gg.from_edge_list(ex["n"], ex["edges"])
    lab = None
    for sweep, qexp in zip(ex["sweeps_level0"], ex["q_int_level0"]):
        lm = oracle.local_move(g.row_ptr, g.col, g.w, lab)
        assert lm.labels.tolist() == sweep
        assert oracle.modularity(g.row_ptr, g.col, g.w, lm.labels)[0] == qexp
        lab = lm.labels
    r = oracle.louvain(g.row_ptr, g.col, g.w)
    assert r.labels.tolist() == ex["final_labels"]
    assert r.q_int == ex["q_int"]
    _, tw = oracle.degrees(g.row_ptr, g.col, g.w)
    assert Fraction(r.q_int, tw * tw) == Fraction(ex["q"])
    if "levels" in ex:
        for got, want in zip(r.levels, ex["levels"]):
            for key, v in want.items():
                assert got[key] == v
        assert len(r.levels) == len(ex["levels"])
    if "contracted" in ex:
        c = ex["contracted"]
        m, k = oracle.renumber(lab)
        rp2, cl2, w2 = oracle.contract(g.row_ptr, g.col, g.w, m[lab], k)
        assert k == c["n"] and rp2.tolist() == c["row_ptr"]
        assert cl2.tolist() == c["col"] and w2.tolist() == c["w"]
    if "merge" in ex:
        mg = ex["merge"]
        got = oracle.merge(g.row_ptr, g.col, g.w, np.array(mg["phase_labels"], np.int32))
        assert got.tolist() == mg["merged"]
        r = oracle.louvain(g.row_ptr, g.col, g.w, merge=True)
        assert r.labels.tolist() == mg["final_labels"] and r.q_int == mg["q_int"]
        assert len(r.levels) == len(mg["levels"])
        for got_lv, want in zip(r.levels, mg["levels"]):
            for key, v in want.items():
                assert got_lv[key] == v
    if "singlet_off" in ex:
        s = ex["singlet_off"]
        lm = oracle.local_move(g.row_ptr, g.col, g.w, None, singlet_rule=False)
        assert lm.labels.tolist() == s["first_sweep"]
        r = oracle.louvain(g.row_ptr, g.col, g.w, singlet_rule=False)
        assert r.labels.tolist() == s["final_labels"] and r.q_int == s["q_int"]


def test_bruteforce_upper_bound_and_planted_optima():
    # random tiny graphs: the heuristic never beats the optimum
    for s in range(40):
        n = 4 + s % 5
        g = gg.random_small(n, 0.5, 4, seed=500 + s, loop_prob=0.2 if s % 3 == 0 else 0.0)
        A = dense(g.row_ptr, g.col, g.w, g.n)
        if sum(map(sum, A)) == 0:
            continue
        r = oracle.louvain(g.row_ptr, g.col, g.w)
        assert r.q_int <= max_modularity(A)
        assert r.q_int == q_int_pair_form(A, r.labels.tolist())
    # planted cases where the optimum is reached
    planted = [
        (6, [(0, 1), (0, 2), (1, 2), (3, 4), (3, 5), (4, 5), (2, 3)]),
        (8, [(a, b) for a in range(4) for b in range(a + 1, 4)]
            + [(a, b) for a in range(4, 8) for b in range(a + 1, 8)] + [(3, 4)]),
        (4, [(a, b) for a in range(4) for b in range(a + 1, 4)]),
    ]
    for n, edges in planted:
        g = gg.from_edge_list(n, edges)
        A = dense(g.row_ptr, g.col, g.w, g.n)
        r = oracle.louvain(g.row_ptr, g.col, g.w)
        assert r.q_int == max_modularity(A)


def test_run_invariants_on_sbm():
    g = gg.config("sbm1k")
    r = oracle.louvain(g.row_ptr, g.col, g.w)
    lab = r.labels
    k = len(np.unique(lab))
    assert sorted(np.unique(lab).tolist()) == list(range(k))     # dense IDs
    qi, q = oracle.modularity(g.row_ptr, g.col, g.w, lab)
    assert qi == r.q_int and q == r.q
    qs = [lv["q_int"] for lv in r.levels]
    assert all(b >= a for a, b in zip(qs, qs[1:]))
    ns = [lv["n"] for lv in r.levels]
    ms = [lv["nnz"] for lv in r.levels]
    assert all(b <= a for a, b in zip(ns, ns[1:])) and all(b <= a for a, b in zip(ms, ms[1:]))
    assert r.levels[-1]["sweeps_accepted"] == 0
    # quality is report-only (the paper prints no Q values); a floor at half the
    # planted partition's modularity only catches a broken run
    qp, _ = oracle.modularity(g.row_ptr, g.col, g.w, g.planted)
    assert 2 * r.q_int >= qp
    _, tw = oracle.degrees(g.row_ptr, g.col, g.w)
    print(f"sbm1k: Q = {r.q:.6f}, planted Q = {qp / tw / tw:.6f}, communities = {k}")


def test_sweeps_strictly_increase_q():
    g = gg.config("sbm1k")
    lab = np.arange(g.n, dtype=np.int32)
    q_prev = oracle.modularity(g.row_ptr, g.col, g.w, lab)[0]
    kept = 0
    for _ in range(50):
        lm = oracle.local_move(g.row_ptr, g.col, g.w, lab)
        q_new = oracle.modularity(g.row_ptr, g.col, g.w, lm.labels)[0]
        if not oracle.accept(q_new, q_prev):
            break
        assert q_new > q_prev
        q_prev, lab = q_new, lm.labels
        kept += 1
    r = oracle.louvain(g.row_ptr, g.col, g.w, max_levels=1)
    assert r.levels[0]["sweeps_accepted"] == kept
    assert r.labels.tolist() == oracle.renumber(lab)[0][lab].tolist()
    assert r.status == oracle.ORC_ELIMIT


# --- the dendrogram and resuming a run from a level state ---------------------

def _dendro_cases():
    out = [gg.config("sbm1k")]
    for s in range(6):
        out.append(gg.random_small(9 + s, 0.35, 5, seed=900 + s, loop_prob=0.2 if s % 2 else 0.0,
                                   isolated=1 if s == 3 else 0))
    return out


def _compose(maps, n):
    lab = np.arange(n, dtype=np.int32)
    for m in maps:
        lab = m[lab]
    return lab


@pytest.mark.parametrize("g", _dendro_cases(), ids=lambda g: f"n{g.n}m{g.nnz}")
def test_dendrogram_levels_and_resume(g):
    r = oracle.louvain(g.row_ptr, g.col, g.w)
    d = oracle.dendrogram(g.row_ptr, g.col, g.w)
    # the level-by-level form is the whole run: same labels, Q and records
    assert np.array_equal(d.labels, r.labels) and np.array_equal(_compose(d.maps, g.n), r.labels)
    assert d.q_int == r.q_int and d.levels == r.levels and d.status == r.status
    assert len(d.graphs) == len(d.maps) + 1
    _, tw = oracle.degrees(g.row_ptr, g.col, g.w)
    for lvl, m in enumerate(d.maps):
        rp, cl, w = d.graphs[lvl]
        n_l = rp.shape[0] - 1
        k = d.graphs[lvl + 1][0].shape[0] - 1
        # a map is dense: onto [0, k)
        assert m.shape[0] == n_l and sorted(set(m.tolist())) == list(range(k))
        # the next level's graph is P^T A P of this one, stored with ascending columns
        M = contract_dense(dense(rp, cl, w, n_l), m.tolist(), k)
        rp2, cl2, w2 = d.graphs[lvl + 1]
        got = np.zeros((k, k), np.int64)
        for a in range(k):
            seg = cl2[rp2[a]:rp2[a + 1]]
            assert np.all(np.diff(seg) > 0)
            got[a, seg] = w2[rp2[a]:rp2[a + 1]]
        assert np.array_equal(got, M)
        assert oracle.degrees(rp2, cl2, w2)[1] == tw
    # the last graph carries the result: its singletons have the run's Q, and a
    # phase on it keeps no sweep
    last = d.graphs[-1]
    kl = last[0].shape[0] - 1
    if tw > 0:
        assert oracle.modularity(*last, np.arange(kl, dtype=np.int32))[0] == r.q_int
        assert oracle.louvain(*last).labels.tolist() == list(range(kl))
    # resuming from every level state gives the whole run's result, also under a level cap
    for cap in (64, len(d.maps) + 1, max(1, len(d.maps))):
        full = oracle.louvain(g.row_ptr, g.col, g.w, max_levels=cap)
        for lvl in range(min(len(d.maps), cap) + 1):
            part = oracle.dendrogram(g.row_ptr, g.col, g.w, max_levels=lvl) if lvl else None
            so_far = part.labels if part else np.arange(g.n, dtype=np.int32)
            if part:
                assert [m.tolist() for m in part.maps] == [m.tolist() for m in d.maps[:lvl]]
                assert all(np.array_equal(x, y) for x, y in zip(part.graphs[-1], d.graphs[lvl]))
            if lvl >= cap:
                continue
            rest = oracle.louvain(*d.graphs[lvl], max_levels=cap - lvl)
            assert np.array_equal(rest.labels[so_far], full.labels)
            assert rest.q_int == full.q_int


def test_dendrogram_worked_example():
    ex = {e["name"]: e for e in _examples()}["two_triangles_bridge"]
    g = gg.from_edge_list(ex["n"], ex["edges"])
    d = oracle.dendrogram(g.row_ptr, g.col, g.w)
    assert [m.tolist() for m in d.maps] == [ex["final_labels"]]
    c = ex["contracted"]
    rp2, cl2, w2 = d.graphs[1]
    assert rp2.tolist() == c["row_ptr"] and cl2.tolist() == c["col"] and w2.tolist() == c["w"]


# --- the final merge of a phase -----------------------------------------------

@pytest.mark.parametrize("singlet", [True, False])
@pytest.mark.parametrize("g", _small_graphs(), ids=lambda g: f"n{g.n}m{g.nnz}")
def test_merge_decisions_by_brute_force(g, singlet):
    A = dense(g.row_ptr, g.col, g.w, g.n)
    labs = list(_labelings(g.n, g.nnz + 11))
    # labellings where the merge has work: the end of a phase, and a sweep's result
    labs.append(oracle.louvain(g.row_ptr, g.col, g.w, max_levels=1).labels)
    labs.append(oracle.local_move(g.row_ptr, g.col, g.w).labels)
    for lab in labs:
        got = oracle.merge(g.row_ptr, g.col, g.w, lab, singlet_rule=singlet)
        want = [expected_merge(A, lab.tolist(), i, singlet) for i in range(g.n)]
        assert got.tolist() == want


def test_merge_zero_gain_stays():
    """Labellings (found by search) where a lone vertex's only neighbouring
    community scores exactly its own score: it must stay."""
    for seed, lab in ((50103, [2, 1, 0, 0]), (50295, [0, 0, 1, 0]), (50307, [3, 2, 1, 2])):
        g = gg.random_small(4, 0.5, 3, seed=seed, loop_prob=0.3)
        A = dense(g.row_ptr, g.col, g.w, g.n)
        lab = np.array(lab, np.int32)
        want = [expected_merge(A, lab.tolist(), i) for i in range(g.n)]
        assert oracle.merge(g.row_ptr, g.col, g.w, lab).tolist() == want


def _merge_run_by_hand(g, singlet=True):
    """Alg. 2 with the final merge, assembled from one-level runs (whose
    labels are the phase's, renumbered in ascending order, which keeps the
    sizes and the label order the merge reads), the brute-force merge, numpy
    renumbering and dense contraction."""
    A = np.array(dense(g.row_ptr, g.col, g.w, g.n), dtype=np.int64)
    final = np.arange(g.n)
    while A.sum() > 0:
        n = len(A)
        rows, cols = np.nonzero(A)
        rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))]).astype(np.int64)
        r = oracle.louvain(rp, cols.astype(np.int32), A[rows, cols], max_levels=1, singlet_rule=singlet)
        if r.levels[0]["sweeps_accepted"] == 0:
            break
        lab = r.labels.tolist()
        merged = [expected_merge(A.tolist(), lab, i, singlet) for i in range(n)]
        uniq, new = np.unique(merged, return_inverse=True)
        final = new[final]
        A = contract_dense(A.tolist(), new.tolist(), len(uniq))
    return final


def _merge_cases():
    # random graphs on which the final merge changes the run (found by search)
    out = [gg.random_small(4 + s % 6, 0.35, 1, seed=7000 + s) for s in (243, 467, 592, 717, 1444, 1665, 2200)]
    return out + _dendro_cases()[1:] + _small_graphs()[::3]


@pytest.mark.parametrize("g", _merge_cases(), ids=lambda g: f"n{g.n}m{g.nnz}")
def test_run_with_merge(g):
    r = oracle.louvain(g.row_ptr, g.col, g.w, merge=True)
    assert r.labels.tolist() == _merge_run_by_hand(g).tolist()
    A = dense(g.row_ptr, g.col, g.w, g.n)
    if sum(map(sum, A)):
        assert r.q_int == q_int_pair_form(A, r.labels.tolist())
    # each level's record holds Q after its merge, which the next level's
    # singletons reproduce (contraction keeps Q)
    qs = [lv["q_int"] for lv in r.levels]
    assert all(lv["sweeps_accepted"] > 0 for lv in r.levels[:-1])
    d = oracle.dendrogram(g.row_ptr, g.col, g.w, merge=True)
    assert np.array_equal(d.labels, r.labels) and d.levels == r.levels
    for lvl in range(1, len(d.graphs)):
        kl = d.graphs[lvl][0].shape[0] - 1
        assert oracle.modularity(*d.graphs[lvl], np.arange(kl, dtype=np.int32))[0] == qs[lvl - 1]
    # the merge is inert without the flag
    assert oracle.louvain(g.row_ptr, g.col, g.w).levels == oracle.louvain(g.row_ptr, g.col, g.w, merge=False).levels


def test_merge_changes_runs():
    """Guard against vacuous merge pins: on the search-found graphs the
    merged run differs from the plain one."""
    changed = 0
    for g in _merge_cases()[:7]:
        a = oracle.louvain(g.row_ptr, g.col, g.w)
        b = oracle.louvain(g.row_ptr, g.col, g.w, merge=True)
        changed += (a.levels != b.levels) or not np.array_equal(a.labels, b.labels)
    assert changed >= 5


# --- the OpenMP variant of the oracle ----------------------------------------

@pytest.mark.parametrize("threads", [2, 5])
def test_openmp_variant_equals_single_thread(threads):
    """Every vertex decides from the same snapshot and the sums are of
    integers, so the multi-threaded oracle gives the single-threaded one's
    results exactly."""
    graphs = [gg.config("sbm1k"), gg.config("chunglu_n20000"), gg.config("rmat_s14")] + _small_graphs()[::4]
    ref = []
    oracle.set_threads(1)
    try:
        for g in graphs:
            lab = gg.random_labels(g.n, max(1, g.n // 7), 5)
            ref.append((oracle.louvain(g.row_ptr, g.col, g.w), oracle.louvain(g.row_ptr, g.col, g.w, merge=True),
                        oracle.local_move(g.row_ptr, g.col, g.w, lab), oracle.modularity(g.row_ptr, g.col, g.w, lab)))
        oracle.set_threads(threads)
        assert oracle.get_threads() == threads
        for g, (a, am, lm, q) in zip(graphs, ref):
            lab = gg.random_labels(g.n, max(1, g.n // 7), 5)
            b = oracle.louvain(g.row_ptr, g.col, g.w)
            assert np.array_equal(a.labels, b.labels) and a.q_int == b.q_int and a.levels == b.levels
            bm = oracle.louvain(g.row_ptr, g.col, g.w, merge=True)
            assert np.array_equal(am.labels, bm.labels) and am.q_int == bm.q_int and am.levels == bm.levels
            lm2 = oracle.local_move(g.row_ptr, g.col, g.w, lab)
            assert all(np.array_equal(x, y) for x, y in zip(lm, lm2))
            assert oracle.modularity(g.row_ptr, g.col, g.w, lab) == q
    finally:
        oracle.set_threads(1)
