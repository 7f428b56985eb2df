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
