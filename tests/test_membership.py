"""The host membership update (tg_chain_membership, no GPU) against the
oracle's reading of Eq. 4, Eq. 5, the absorption-first rule and the
termination rules: every output equal, on hand-built cases and on seeded
random chains whose members and perturbers straddle the radii."""
import numpy as np
import pytest

from oracle import chain as ochain
from paper_1507_01009_amd import binding as B


def _same(x, v, m, mas, d, rc, rc0, g, px):
    a = B.chain_membership(x, v, m, mas, d, rc, rc0, g, px)
    b = ochain.membership(x, v, m, mas.astype(bool), d, rc, rc0, g, px)
    assert np.array_equal(a["absorb"], b["absorb"])
    assert np.array_equal(a["escape"], b["escape"])
    assert a["terminate"] == b["terminate"] and a["designated"] == b["designated"]
    return a


@pytest.mark.parametrize("seed", range(40))
def test_random_chains_match_the_oracle(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    x = rng.normal(size=(n, 3)) * 0.02
    v = rng.normal(size=(n, 3))
    m = rng.uniform(1e-5, 1e-4, n)
    mas = (rng.uniform(size=n) < 0.15).astype(np.uint8)
    d = int(rng.integers(0, n))
    mas[d] = 1
    m[d] = 0.01
    px = rng.normal(size=(int(rng.integers(0, 300)), 3)) * 0.03
    rc = float(rng.uniform(0.005, 0.05))
    rc0 = float(rng.uniform(0.005, 0.03))
    _same(x, v, m, mas, d, rc, rc0, 1.5, px)


def test_hand_built_cases():
    x = np.array([[0.001, 0, 0], [0.05, 0, 0], [0, 0.05, 0], [0, 0, 0.02]])
    v = np.array([[0, 0, 0], [1.0, 0, 0], [0, -1.0, 0], [0, 0, 1.0]])
    m = np.array([0.01, 1e-5, 1e-5, 1e-5])
    mas = np.array([1, 0, 0, 0], np.uint8)
    r = _same(x, v, m, mas, 0, 0.03, 0.02, 1.5, np.zeros((0, 3)))
    assert r["escape"].tolist() == [1] and not r["terminate"]
    # a near perturber delays the escape until r_chain > 1.05 r_escape
    px = np.array([[0.001, 0, 0]])
    assert _same(x, v, m, mas, 0, 0.031, 0.02, 1.5, px)["escape"].size == 0
    assert _same(x, v, m, mas, 0, 0.0316, 0.02, 1.5, px)["escape"].tolist() == [1]


def test_errors():
    x = np.zeros((2, 3)); v = np.zeros((2, 3)); m = np.ones(2); mas = np.ones(2, np.uint8)
    with pytest.raises(B.TGError):
        B.chain_membership(x, v, m, mas, 5, 0.1, 0.1, 1.5, np.zeros((0, 3)))
    with pytest.raises(B.TGError):
        B.chain_membership(x, v, m, mas, 0, -0.1, 0.1, 1.5, np.zeros((0, 3)))
    with pytest.raises(B.TGError):
        B.chain_membership(x, v, m, mas, 0, 0.1, 0.1, 0.0, np.zeros((0, 3)))
