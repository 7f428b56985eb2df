"""Pins for the oracle's partial-sketch choice (Section 4.3: a high-degree
vertex's row is split into segments, each summarised by its own k-slot
sketch, and the partial sketches are merged into one).

* A row that fits one segment gives the plain sketch rule's label.
* With k at least the number of distinct labels no slot is ever decremented,
  so every partial sketch holds exact per-segment totals and the merge adds
  them up: the choice is the exact weighted argmax (Eq. 3), ties to the
  lowest label (integer weights keep the fp32 sums exact).
* A label carrying at least 3/4 of the row's weight wins for k = 8 however
  the row is cut: each sketch underestimates a label by at most its stream's
  weight / (k + 1), twice over here, which leaves the label above every
  other label's true weight.
* The vertex's own entries count for nothing, and an empty row keeps the
  current label.
"""
import json
import os
from collections import defaultdict
from fractions import Fraction

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


def star_row(labels, weights, extra_self=None):
    """CSR over d + 1 vertices whose last vertex v = d has neighbours
    0 .. d-1; neighbour i holds label labels[i] (C[v] = d + 1 > every
    label, so any neighbour label counts as smaller)."""
    d = len(labels)
    v = d
    cols = list(range(d))
    ws = list(weights)
    if extra_self is not None:
        pos, x = extra_self
        cols.insert(pos, v)
        ws.insert(pos, x)
    rp = np.zeros(d + 2, np.int32)
    rp[d + 1] = len(cols)
    C = np.concatenate([np.asarray(labels, np.int32), [d + 1]]).astype(np.int32)
    return rp, np.asarray(cols, np.int32), np.asarray(ws, np.float32), C, v


def exact_argmax(labels, weights):
    tot = {}
    for c, x in zip(labels, weights):
        tot[int(c)] = tot.get(int(c), 0.0) + float(x)
    best = max(tot.values())
    return min(c for c, t in tot.items() if t == best)


@pytest.mark.parametrize("k", [1, 2, 8, 32])
def test_one_segment_is_the_plain_rule(k):
    rng = np.random.default_rng(40 + k)
    for _ in range(300):
        d = int(rng.integers(1, 60))
        lab = rng.integers(0, 15, d).astype(np.int32)
        w = (rng.random(d) + 0.01).astype(np.float32)
        rp, col, ww, C, v = star_row(lab, w)
        kk, vv = oracle.sketch_feed(k, lab, w)
        plain = oracle.sketch_max_key(kk, vv, int(C[v]))
        for seg in (d, d + 1, 10 * d):
            assert oracle.hub_segment_choice(rp, col, ww, k, seg, C, v) == plain


@pytest.mark.parametrize("k", [4, 8, 16])
def test_enough_slots_give_the_exact_argmax(k):
    rng = np.random.default_rng(70 + k)
    for _ in range(300):
        d = int(rng.integers(1, 200))
        distinct = int(rng.integers(1, k + 1))
        lab = rng.integers(0, distinct, d).astype(np.int32)
        w = rng.integers(1, 9, d).astype(np.float32)  # exact in fp32
        rp, col, ww, C, v = star_row(lab, w)
        want = exact_argmax(lab, w)
        for seg in (1, 3, 7, 64):
            assert oracle.hub_segment_choice(rp, col, ww, k, seg, C, v) == want, (d, seg)


def test_three_quarter_label_wins():
    rng = np.random.default_rng(5)
    for _ in range(200):
        d = int(rng.integers(40, 400))
        lab = rng.integers(1, 400, d).astype(np.int32)  # mostly distinct minor labels
        w = (rng.random(d) + 0.05).astype(np.float32)
        heavy = rng.random(d) < 0.8
        lab[heavy] = 0
        if w[lab == 0].sum() < 0.75 * w.sum():
            continue
        rp, col, ww, C, v = star_row(lab, w)
        for seg in (5, 16, 33):
            assert oracle.hub_segment_choice(rp, col, ww, 8, seg, C, v) == 0


def test_self_entries_and_empty_rows():
    lab = np.array([3, 3, 1], np.int32)
    w = np.array([1.0, 1.0, 1.5], np.float32)
    rp, col, ww, C, v = star_row(lab, w, extra_self=(1, 100.0))
    assert oracle.hub_segment_choice(rp, col, ww, 8, 2, C, v) == 3
    rp = np.zeros(3, np.int32)
    C = np.array([0, 1], np.int32)
    assert oracle.hub_segment_choice(rp, np.zeros(0, np.int32), None, 8, 4, C, 1) == 1


# ------------------------------------------------------------ wide merges
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hub_merge_cases.json")


def golden_row(case):
    d = case["degree"]
    v = d  # neighbours 0 .. d-1 (only the listed positions are used)
    cols = [v] * d
    labels = np.zeros(d + 1, np.int32)
    ws = np.ones(d, np.float32)
    for pos, lab, x in case["entries"]:
        cols[pos] = pos
        labels[pos] = lab
        ws[pos] = x
    labels[v] = 10 ** 6  # larger than every label
    rp = np.array([0] * (d + 1) + [d], np.int32)
    return rp, np.asarray(cols, np.int32), ws, labels, v


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["name"])
def test_golden_wide_merge(case):
    rp, col, w, C, v = golden_row(case)
    key, val, nseg = oracle.hub_merged_sketch(rp, col, w, case["k"], case["seg_len"], C, v)
    assert nseg == case["degree"] // case["seg_len"] > 64
    live = val > 0
    got = sorted(zip(key[live].tolist(), val[live].tolist()))
    assert got == sorted(zip(case["merged_keys"], case["merged_vals"]))
    assert oracle.hub_segment_choice(rp, col, w, case["k"], case["seg_len"], C, v) == case["choice"]
    # the segment-order feed of the same partials, for contrast
    lab, ws = [], []
    for pos, l, x in sorted(case["entries"]):
        lab.append(l)
        ws.append(x)
    kk, vv = oracle.sketch_feed(case["k"], lab, ws)
    assert oracle.sketch_max_key(kk, vv, int(C[v])) == case["sequential_choice"]


def rational(x):
    return Fraction(float(x))


@pytest.mark.parametrize("k", [1, 2, 4, 8, 16])
def test_merged_sketch_keeps_the_misra_gries_bound(k):
    # Every stage (segment sketches, chains, pairwise rounds) removes weight
    # only by decrements that take d from each of k slots and d from the
    # incoming pair, and lowers any one label by at most d; so over the whole
    # merge f - W/(k+1) <= estimate <= f for every label.  Dyadic weights
    # keep the fp32 arithmetic exact.
    rng = np.random.default_rng(300 + k)
    for trial in range(60):
        seg = int(rng.choice([1, 2, 3, 5, 8]))
        d = int(rng.integers(1, 500 * seg // 5 + 2))
        nlab = int(rng.integers(1, 3 * k + 3))
        lab = rng.integers(0, nlab, d).astype(np.int32)
        w = (rng.integers(1, 33, d) / 8).astype(np.float32)
        rp, col, ww, C, v = star_row(lab, w)
        key, val, nseg = oracle.hub_merged_sketch(rp, col, ww, k, seg, C, v)
        est = {int(a): rational(b) for a, b in zip(key, val) if b > 0}
        assert len(est) == int((val > 0).sum()), "duplicate live labels"
        f = defaultdict(Fraction)
        for c, x in zip(lab.tolist(), w.tolist()):
            f[c] += rational(x)
        W = sum(f.values())
        for c in range(nlab):
            e = est.get(c, Fraction(0))
            assert e <= f[c], (trial, c, nseg)
            assert f[c] - W / (k + 1) <= e, (trial, c, nseg, f[c], e, W)


@pytest.mark.parametrize("k", [4, 8, 16])
def test_wide_merge_with_enough_slots_is_the_exact_argmax(k):
    rng = np.random.default_rng(900 + k)
    for _ in range(60):
        seg = int(rng.choice([1, 2, 3]))
        d = int(rng.integers(65 * seg, 400 * seg + 1))
        distinct = int(rng.integers(1, k + 1))
        lab = rng.integers(0, distinct, d).astype(np.int32)
        w = rng.integers(1, 9, d).astype(np.float32)
        rp, col, ww, C, v = star_row(lab, w)
        assert oracle.hub_merged_sketch(rp, col, ww, k, seg, C, v)[2] > 64
        assert oracle.hub_segment_choice(rp, col, ww, k, seg, C, v) == exact_argmax(lab, w)


def test_wide_merge_three_quarter_label_wins():
    rng = np.random.default_rng(15)
    done = 0
    while done < 60:
        seg = int(rng.choice([1, 2, 4, 8]))
        d = int(rng.integers(65 * seg, 400 * seg + 1))
        lab = rng.integers(1, 4000, d).astype(np.int32)
        w = (rng.random(d) + 0.05).astype(np.float32)
        lab[rng.random(d) < 0.8] = 0
        if w[lab == 0].sum() < 0.75 * w.sum():
            continue
        rp, col, ww, C, v = star_row(lab, w)
        assert oracle.hub_segment_choice(rp, col, ww, 8, seg, C, v) == 0
        done += 1


@pytest.mark.parametrize("k", [2, 8])
def test_hub_rescan_choice_is_the_exact_argmax_of_a_heavy_label(k):
    # Section 4.4's double scan over the merged sketch: whenever the exact
    # argmax label carries more than W/(k+1), the merge keeps it live (bound
    # above), and its exact re-weighting makes it win.
    rng = np.random.default_rng(41 + k)
    checked = 0
    for _ in range(400):
        seg = int(rng.choice([1, 2, 5]))
        d = int(rng.integers(2, 300 * seg))
        lab = (rng.geometric(float(rng.uniform(0.1, 0.6)), d) - 1).astype(np.int32)
        w = rng.integers(1, 5, d).astype(np.float32)
        tot = defaultdict(float)
        for c, x in zip(lab.tolist(), w.tolist()):
            tot[c] += x
        best = exact_argmax(lab, w)
        if tot[best] <= sum(tot.values()) / (k + 1):
            continue
        rp, col, ww, C, v = star_row(lab, w)
        got = oracle.hub_choose(rp, col, ww, k, seg, False, C, [v], rescan=True)
        assert int(got[0]) == best
        checked += 1
    assert checked > 50


def test_unit_weight_hub_choice_uses_emptied_slots():
    # k = 2, unit weights, one segment: the row's sketch ends with label 8
    # back in its emptied slot 1 and label 5 in slot 0 (Algorithm 2's rule);
    # the choice is the lower label of the tie
    rp, col, ww, C, v = star_row([7, 8, 9, 8, 5], [1.0] * 5)
    key, val, nseg = oracle.hub_merged_sketch(rp, col, ww, 2, 8, C, v)
    assert nseg == 1 and key.tolist() == [5, 8] and val.tolist() == [1.0, 1.0]
    assert oracle.hub_segment_choice(rp, col, ww, 2, 8, C, v) == 5
