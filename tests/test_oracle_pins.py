"""Pins for the CPU oracle: checks against what the paper and mathematics fix,
never against the oracle itself.

* P1  weighted Misra-Gries guarantee (Section 3.5 / 4): for every label,
      f - W/(k+1) <= estimate <= f, with exact rational frequencies.
* P2  on unit weights the oracle's sketch step equals the paper's literal
      Algorithm 2 (non-shared) on every stream up to length 7 over 4 labels.
* P3  k = 1 (weighted Boyer-Moore, Section 3.4 / 4.7) returns a strict
      weighted majority whenever one exists.
* P4  sketchMaxKey: ties to the lowest label, empty sketch keeps the label.
* P5  fp32 sums follow CSR order exactly.
* P6  k >= max degree: the sketch LPA equals the exact argmax LPA (Eq. 3),
      and one exact iteration equals a brute-force Eq. 3 on tiny graphs.
* P7  hand-derived driver outcomes (tests/golden/driver_cases.json), two
      cliques joined by an edge.
* P8  modularity closed forms (Eq. 1).
* P9  Jacobi results do not depend on the thread count.
"""
import itertools
import json
import os
import random
from collections import defaultdict
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def live(keys, vals):
    return {int(k): float(v) for k, v in zip(keys, vals) if v > 0}


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("k", [1, 2, 3, 4, 8])
def test_p1_mg_guarantee_weighted(orc, k):
    rng = random.Random(1000 + k)
    for trial in range(400):
        L = rng.randint(1, 40)
        nlab = rng.randint(1, 10)
        # dyadic weights (multiples of 1/8 up to 4): fp32 arithmetic on them is exact
        stream = [rng.randrange(nlab) for _ in range(L)]
        ws = [rng.randint(1, 32) / 8 for _ in range(L)]
        keys, vals = orc.sketch_feed(k, stream, ws)
        est = live(keys, vals)
        assert len(est) == len(set(est)), "duplicate live keys"
        f = defaultdict(Fraction)
        for c, w in zip(stream, ws):
            f[c] += Fraction(w)
        W = sum(f.values())
        bound = W / (k + 1)
        for c in range(nlab):
            e = Fraction(est.get(c, 0.0))
            assert e <= f[c], (trial, c)
            assert f[c] - bound <= e, (trial, c, f[c], e, bound)
            if f[c] > bound:
                assert c in est, "heavy hitter lost"
        assert all(v > 0 for v in est.values())


def test_p1_counterexample_literal_rule_breaks_guarantee(orc):
    # Reading R1: the paper's literal "subtract w from every slot" drives slots
    # negative on weighted input.  Stream with k=1: (a,1) then (b,3) then (a,1):
    # literal rule gives slot a at 1-3 = -2, never empty again, so b (weight 3
    # of 5 > 5/2) is lost.  The oracle's rule keeps b.
    keys, vals = orc.sketch_feed(1, [0, 1, 0], [1.0, 3.0, 1.0])
    assert live(keys, vals) == {1: 1.0}


# ---------------------------------------------------------------- P2
def paper_alg2_unit(k, stream):
    """Algorithm 2, non-shared, unit weights, as printed: a slot whose label
    is c takes the weight (its value is not looked at); otherwise the first
    free slot (value 0) takes (c, 1); otherwise every slot loses 1.
    Returns the slots (label, value) in slot order."""
    key = [-1] * k
    val = [0] * k
    for c in stream:
        hit = False
        for s in range(k):
            if key[s] == c:
                val[s] += 1
                hit = True
        if hit:
            continue
        free = [s for s in range(k) if val[s] == 0]
        if free:
            key[free[0]] = c
            val[free[0]] = 1
        else:
            for s in range(k):
                val[s] -= 1
    return key, val


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_p2_unit_weights_equal_paper_algorithm2(orc, k):
    # slot for slot, emptied slots' labels included: the order of the slots
    # is what a merge of partial sketches feeds on (Section 4.3)
    for L in range(0, 8):
        for stream in itertools.product(range(4), repeat=L):
            keys, vals = orc.sketch_feed(k, list(stream))
            pk, pv = paper_alg2_unit(k, stream)
            assert keys.tolist() == pk, stream
            assert vals.tolist() == [float(x) for x in pv], stream


def test_p2_emptied_slot_keeps_its_label(orc):
    # k = 2, unit weights: a, b fill both slots, c empties both (a and b
    # keep their labels at value 0), then b returns to slot 1 -- not to the
    # lowest free slot 0 -- and d takes slot 0 (Algorithm 2)
    keys, vals = orc.sketch_feed(2, [7, 8, 9, 8, 5])
    assert keys.tolist() == [5, 8] and vals.tolist() == [1.0, 1.0]
    # weight 0 changes nothing, not even an empty slot's label
    keys, vals = orc.sketch_feed(2, [7, 3], [0.0, 1.0])
    assert keys.tolist() == [3, -1] and vals.tolist() == [1.0, 0.0]


# ---------------------------------------------------------------- P3
def test_p3_k1_finds_strict_weighted_majority(orc):
    rng = random.Random(7)
    hits = 0
    for trial in range(3000):
        L = rng.randint(1, 15)
        stream = [rng.randrange(3) for _ in range(L)]
        ws = [rng.randint(1, 16) / 4 for _ in range(L)]
        f = defaultdict(Fraction)
        for c, w in zip(stream, ws):
            f[c] += Fraction(w)
        W = sum(f.values())
        maj = [c for c in f if f[c] > W / 2]
        keys, vals = orc.sketch_feed(1, stream, ws)
        if maj:
            hits += 1
            assert live(keys, vals).keys() == {maj[0]}, (stream, ws)
    assert hits > 500
    # the weighted stream on which the paper's Algorithm 3 replacement rule
    # misses the majority (m has 4 of 7): MG(1) keeps m
    keys, vals = orc.sketch_feed(1, [5, 9, 5], [3.0, 3.0, 1.0])
    assert live(keys, vals) == {5: 1.0}


# ---------------------------------------------------------------- P4
def test_p4_max_key(orc):
    assert orc.sketch_max_key([7, 3, 9], [2.0, 2.0, 1.0], keep=42) == 3
    assert orc.sketch_max_key([7, 3, 9], [2.0, 2.5, 2.5], keep=42) == 3
    assert orc.sketch_max_key([7, 3, 9], [0.0, 0.0, 0.0], keep=42) == 42
    assert orc.sketch_max_key([-1, -1], [0.0, 0.0], keep=5) == 5
    assert orc.sketch_max_key([4, 1], [0.0, 0.5], keep=9) == 1


# ---------------------------------------------------------------- P5
def test_p5_fp32_csr_order(orc):
    e = 2.0 ** -24
    keys, vals = orc.sketch_feed(2, [0, 0, 0], [1.0, e, e])
    assert live(keys, vals) == {0: 1.0}           # (1 + e) + e rounds to 1 twice
    keys, vals = orc.sketch_feed(2, [0, 0, 0], [e, e, 1.0])
    assert live(keys, vals) == {0: 1.0 + 2 * e}   # e + e = 2e exactly, then 1 + 2e


# ---------------------------------------------------------------- P6
def brute_eq3_choice(g, i, C, w):
    """Eq. 3 for one vertex with exact rational sums; ties to lowest label."""
    acc = defaultdict(Fraction)
    for e in range(g.row_ptr[i], g.row_ptr[i + 1]):
        j = int(g.col[e])
        if j != i:
            acc[int(C[j])] += Fraction(float(w[e]) if w is not None else 1.0)
    if not acc:
        return int(C[i])
    best = max(acc.values())
    return min(c for c, v in acc.items() if v == best)


def random_graph(gen, rng, n, p, weighted):
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
    g = gen.from_edges(n, edges)
    if weighted:
        # dyadic symmetric weights
        wmap = {}
        w = np.empty(g.nnz, np.float32)
        for i in range(n):
            for e in range(g.row_ptr[i], g.row_ptr[i + 1]):
                j = int(g.col[e])
                key = (min(i, j), max(i, j))
                if key not in wmap:
                    wmap[key] = rng.randint(1, 8) / 4
                w[e] = wmap[key]
        g.w = w
    return g


def test_p6_exact_iteration_matches_brute_force(orc, gen):
    rng = random.Random(11)
    for trial in range(40):
        n = rng.randint(2, 30)
        g = random_graph(gen, rng, n, rng.uniform(0.05, 0.5), weighted=trial % 2 == 1)
        C = np.array([rng.randrange(n) for _ in range(n)], np.int32)
        act = np.array([rng.random() < 0.8 for _ in range(n)], np.uint8)
        for pl in (False, True):
            Cn, an, dN, sc = orc.lpa_move(g.row_ptr, g.col, g.w, 0, pl, C, act)
            exp_changed = 0
            exp_act = np.zeros(n, np.uint8)
            for i in range(n):
                if not act[i]:
                    assert Cn[i] == C[i]
                    continue
                c = brute_eq3_choice(g, i, C, g.w)
                moved = c != C[i] and (not pl or c < C[i])
                assert Cn[i] == (c if moved else C[i]), (trial, i)
                if moved:
                    exp_changed += 1
                    exp_act[g.col[g.row_ptr[i]:g.row_ptr[i + 1]]] = 1
            assert dN == exp_changed
            assert np.array_equal(an, exp_act)
            assert sc == int(sum(g.row_ptr[i + 1] - g.row_ptr[i] for i in range(n) if act[i]))


def test_p6_large_k_equals_exact(orc, gen):
    rng = random.Random(5)
    for trial in range(30):
        n = rng.randint(5, 80)
        g = random_graph(gen, rng, n, rng.uniform(0.03, 0.3), weighted=trial % 3 == 0)
        dmax = int(g.degrees().max()) if g.nnz else 0
        k = min(64, max(dmax, 1))
        if dmax > 64:
            continue
        a = orc.lpa_run(g.row_ptr, g.col, g.w, k=k)
        b = orc.lpa_run(g.row_ptr, g.col, g.w, k=0)
        assert np.array_equal(a[0], b[0]) and a[1] == b[1]
        assert np.array_equal(a[2], b[2])


# ---------------------------------------------------------------- P7
def _golden_graph(gen, case):
    if "cliques" in case:
        return gen.two_cliques(case["cliques"])
    n = 1 + max(max(e) for e in case["edges"])
    g = gen.from_edges(n, case["edges"])
    if "weights" in case:
        g.w = np.array(case["weights"], np.float32)
    return g


def _load_cases():
    with open(os.path.join(GOLDEN, "driver_cases.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _load_cases(), ids=lambda c: c["name"])
def test_p7_hand_derived_driver(orc, gen, case):
    g = _golden_graph(gen, case)
    for k in case["k"]:
        labels, it, dn, sc = orc.lpa_run(g.row_ptr, g.col, g.w, k=k, tol=case["tol"],
                                         max_iter=case["max_iter"], rho=case["rho"])
        assert labels.tolist() == case["labels"], (k, labels)
        assert it == case["iterations"]
        assert dn.tolist() == case["dN"]
        assert sc.tolist() == case["scanned"]


def test_p7_two_cliques_exact_split(orc, gen):
    for s in range(3, 41):
        g = gen.two_cliques(s)
        labels, it, _, _ = orc.lpa_run(g.row_ptr, g.col, None, k=0)
        assert len(set(labels[:s].tolist())) == 1 and len(set(labels[s:].tolist())) == 1, s
        assert labels[0] != labels[s], s


def test_p7_two_cliques_mg_empty_sketch(orc, gen):
    # (s-1) = multiple of (k+1) distinct unit labels empty a k-slot sketch
    # exactly (every (k+1)-th distinct label clears all slots), so nothing
    # can move in iteration 0 and the run stops with all singletons.
    for k in (2, 4, 8):
        for s in range(3, 41):
            if (s - 1) % (k + 1):
                continue
            g = gen.two_cliques(s)
            labels, it, dn, _ = orc.lpa_run(g.row_ptr, g.col, None, k=k)
            assert labels.tolist() == list(range(2 * s)), (k, s)
            assert it == 2 and dn.tolist() == [0, 0]


# ---------------------------------------------------------------- P8
def test_p8_modularity_closed_forms(orc, gen):
    for s in (3, 5, 12):
        g = gen.two_cliques(s)
        n = g.n
        two_m = 2 * (s * (s - 1) + 1)
        assert g.nnz == two_m
        one = np.zeros(n, np.int32)
        assert abs(orc.modularity(g.row_ptr, g.col, None, one)) < 1e-15
        split = np.array([0] * s + [s] * s, np.int32)
        q = s * (s - 1) / (s * (s - 1) + 1) - 0.5
        assert abs(orc.modularity(g.row_ptr, g.col, None, split) - q) < 1e-14
        single = np.arange(n, dtype=np.int32)
        deg = g.degrees().astype(float)
        qs = -np.sum((deg / two_m) ** 2)
        assert abs(orc.modularity(g.row_ptr, g.col, None, single) - qs) < 1e-14
    # two disjoint equal cliques as two communities: Q = 1/2
    s = 6
    edges = [(u, v) for u in range(s) for v in range(u + 1, s)]
    edges += [(s + u, s + v) for u in range(s) for v in range(u + 1, s)]
    g = gen.from_edges(2 * s, edges)
    lab = np.array([0] * s + [s] * s, np.int32)
    assert abs(orc.modularity(g.row_ptr, g.col, None, lab) - 0.5) < 1e-14


def test_p8_modularity_weighted_direct_count(orc, gen):
    rng = random.Random(3)
    for trial in range(20):
        n = rng.randint(2, 25)
        g = random_graph(gen, rng, n, 0.3, weighted=True)
        lab = np.array([rng.randrange(4) for _ in range(n)], np.int32)
        # Newman's all-pairs form: Q = 1/2m sum_ij [A_ij - K_i K_j / 2m] delta(C_i, C_j)
        A = np.zeros((n, n))
        for i in range(n):
            for e in range(g.row_ptr[i], g.row_ptr[i + 1]):
                A[i, g.col[e]] = g.w[e]
        K = A.sum(1)
        two_m = K.sum()
        if two_m == 0:
            continue
        d = (lab[:, None] == lab[None, :]).astype(float)
        q_pairs = ((A - np.outer(K, K) / two_m) * d).sum() / two_m
        assert abs(orc.modularity(g.row_ptr, g.col, g.w, lab) - q_pairs) < 1e-12
        assert -0.5 <= q_pairs <= 1.0


# ---------------------------------------------------------------- P9
def test_p9_thread_count_invariance(orc, gen):
    g = gen.sbm1(2)
    ref = orc.lpa_run(g.row_ptr, g.col, None, k=8, nthreads=1)
    for nt in (2, 3, 8):
        got = orc.lpa_run(g.row_ptr, g.col, None, k=8, nthreads=nt)
        assert np.array_equal(ref[0], got[0]) and ref[1] == got[1]
        assert np.array_equal(ref[2], got[2])
