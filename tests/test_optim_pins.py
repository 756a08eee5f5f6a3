"""Pins of the optimiser loops around the objective (section 3.3, Algorithm 1; the
step-size line search of the full-batch descent loop), CPU only.

Algorithm 1 draws a fresh shuffle of the JD patterns for every pass and runs JD/b
minibatches of b patterns from it.  The minibatch sequences below are written out by
hand for small cases (JD not a multiple of b, passes wrapping over the shuffles), and
both loop drivers (the oracle's and the library's host loop, written separately) must
produce them.  The line search is checked against its own definition on a tiny
problem: the first step is step0 over the RMS of the gradient, every later first trial
is twice the previous accepted step, each backtrack halves the step, an accepted step
meets the Armijo condition and the trial before it does not.
"""
import math

import numpy as np
import pytest

from oracle import mpbp_oracle as O
from tests.conftest import random_fields, ragged, tiny_problem

# JD = 7 patterns, b = 3: two minibatches per pass, one pattern of each shuffle left
# for a later pass; three shuffles, so pass 3 reuses shuffle 0.
ORDER_7 = np.array([6, 5, 4, 3, 2, 1, 0,
                    0, 1, 2, 3, 4, 5, 6,
                    3, 0, 6, 2, 5, 1, 4], dtype=np.int32)
EXPECTED_7_3 = [[6, 5, 4], [3, 2, 1],          # pass 0: shuffle 0, pattern 0 not visited
                [0, 1, 2], [3, 4, 5],          # pass 1: shuffle 1, pattern 6 not visited
                [3, 0, 6], [2, 5, 1],          # pass 2: shuffle 2, pattern 4 not visited
                [6, 5, 4], [3, 2, 1]]          # pass 3: shuffle 0 again
# JD = 5, b = 5: one minibatch per pass (the full batch), shuffles in turn.
ORDER_5 = np.array([4, 2, 0, 1, 3, 1, 0, 4, 3, 2], dtype=np.int32)
EXPECTED_5_5 = [[4, 2, 0, 1, 3], [1, 0, 4, 3, 2], [4, 2, 0, 1, 3]]
# JD = 5, b = 2: two per pass, pattern at position 4 of each shuffle left out.
EXPECTED_5_2 = [[4, 2], [0, 1], [1, 0], [4, 3], [4, 2]]


def _oracle_seq(order, n, b, iters):
    return [O.minibatch(order, n, b, it) for it in range(iters)]


def _host_seq(order, n, b, iters):
    optim = pytest.importorskip("paper_2312_14907_amd.optim")
    return [[int(f) for f in optim.minibatch_frames(order, n, b, it)] for it in range(iters)]


@pytest.mark.parametrize("seq", [_oracle_seq, _host_seq], ids=["oracle", "host_loop"])
def test_minibatch_sequence_written_out(seq):
    assert seq(ORDER_7, 7, 3, 8) == EXPECTED_7_3
    assert seq(ORDER_5, 5, 5, 3) == EXPECTED_5_5
    assert seq(ORDER_5, 5, 2, 5) == EXPECTED_5_2


@pytest.mark.parametrize("seq", [_oracle_seq, _host_seq], ids=["oracle", "host_loop"])
def test_minibatch_passes_cover_each_pattern_once(seq):
    # the paper's workload shape: 324 patterns (4 peaks x 9 x 9), b = 50: six minibatches
    # of 50 per pass, disjoint, all from that pass's shuffle
    rng = np.random.default_rng(7)
    n, b, passes = 324, 50, 3
    order = np.concatenate([rng.permutation(n) for _ in range(passes)]).astype(np.int32)
    batches = seq(order, n, b, passes * (n // b))
    for e in range(passes):
        mine = batches[e * (n // b):(e + 1) * (n // b)]
        assert all(len(x) == b for x in mine)
        flat = [f for x in mine for f in x]
        assert len(set(flat)) == len(flat) == (n // b) * b
        assert set(flat) <= set(order[e * n:(e + 1) * n].tolist())


@pytest.mark.parametrize("seq", [_oracle_seq, _host_seq], ids=["oracle", "host_loop"])
def test_minibatch_rejects_bad_inputs(seq):
    with pytest.raises(ValueError):
        seq(ORDER_7[:10], 7, 3, 1)          # not whole shuffles
    with pytest.raises(ValueError):
        seq(ORDER_7, 7, 8, 1)               # b > JD
    with pytest.raises(ValueError):
        seq(ORDER_7, 7, 0, 1)


def test_adam_reconstruct_visits_the_written_out_minibatches():
    # With zero step sizes the fields never move, so the loss of iteration it is the
    # objective over exactly that iteration's minibatch (eq. (11)).
    prob = tiny_problem()          # 12 frames
    u, chi, alpha, probe = random_fields(prob, seed=71)
    rng = np.random.default_rng(72)
    y = ragged(O.model_intensity(u + rng.normal(0, 0.05, size=u.shape), chi, alpha, probe, prob))
    n = prob.n_frames()
    order = np.concatenate([rng.permutation(n) for _ in range(2)]).astype(np.int32)
    b = 5                          # two minibatches per pass, two patterns left per shuffle
    expected = [order[0:5], order[5:10], order[12:17], order[17:22], order[0:5]]
    _, _, _, losses = O.adam_reconstruct(u, np.log(chi), np.log(alpha), probe, y, prob, order, batch=b,
                                         iterations=5, lr=(0.0, 0.0, 0.0), fixed_alpha=-1)
    for it, frames in enumerate(expected):
        assert losses[it] == pytest.approx(O.loss(u, chi, alpha, probe, y, prob, frames=frames)[0], rel=1e-12)


def _line_search_case():
    prob = tiny_problem()
    u, chi, alpha, probe = random_fields(prob, seed=61)
    y = ragged(O.model_intensity(u, chi, alpha, probe, prob))
    u0 = u + np.random.default_rng(62).normal(0, 0.03, size=u.shape)
    return prob, u0, chi, alpha, probe, y


def test_line_search_steps_follow_their_definition():
    prob, u0, chi, alpha, probe, y = _line_search_case()
    c, step0, iters = 0.5, 0.01, 6      # a strict sufficient-decrease constant: backtracks happen
    trials = []
    _, losses, etas = O.line_search_descent(u0, chi, alpha, probe, y, prob, iterations=iters, step0=step0, c=c,
                                            trials=trials)
    assert len(etas) == len(trials) == iters
    assert sum(len(t) for t in trials) > iters          # some iteration backtracked
    uk = np.array(u0, dtype=np.float64)
    for k in range(iters):
        r = O.loss_grad(uk, chi, alpha, probe, y, prob)
        g = r["grad_u"]
        n2 = float(np.sum(g * g))
        assert losses[k] == pytest.approx(r["loss"], rel=1e-13)
        first = trials[k][0][0]
        if k == 0:
            assert first == pytest.approx(step0 / math.sqrt(n2 / g.size), rel=1e-12)
        else:
            assert first == pytest.approx(2.0 * etas[k - 1], rel=1e-15)
        for (e0, _), (e1, _) in zip(trials[k], trials[k][1:]):
            assert e1 == pytest.approx(0.5 * e0, rel=1e-15)
        for e, f1 in trials[k][:-1]:            # rejected: no sufficient decrease
            assert f1 > losses[k] - c * e * n2
        e, f1 = trials[k][-1]                    # accepted
        assert e == etas[k]
        assert f1 <= losses[k] - c * e * n2
        assert f1 == pytest.approx(O.loss(uk - e * g, chi, alpha, probe, y, prob)[0], rel=1e-13)
        uk = uk - e * g
