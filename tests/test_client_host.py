"""Host-side client inputs of the library (no GPU needed): B-bar (heqg_bbar)
against the oracle's definition, padding columns, thread-count invariance and
argument checks."""
import numpy as np
import pytest

from oracle import trainer


@pytest.fixture(scope="module")
def heqg():
    from paper_2406_13221_amd import heqg
    heqg.lib()
    return heqg


@pytest.mark.parametrize("n,f,g", [(128, 7, 8), (5000, 63, 64), (9000, 200, 256), (1, 3, 32)])
def test_bbar_matches_oracle(heqg, n, f, g):
    rng = np.random.default_rng(n + f)
    X = rng.uniform(-1, 1, (n, f))
    got = heqg.bbar(X, g)
    ref = trainer.bbar(X, g)
    assert got.shape == (g,)
    assert np.allclose(got, ref, rtol=1e-12, atol=0)
    assert not got[f + 1:].any()


def test_bbar_independent_of_threads(heqg):
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, (20000, 31))
    a = heqg.bbar(X, 32, threads=1)
    b = heqg.bbar(X, 32, threads=7)
    assert np.array_equal(a, b)


def test_bbar_rejects_bad_shapes(heqg):
    X = np.zeros((4, 8))
    with pytest.raises(heqg.HeqgError) as e:
        heqg.bbar(X, 8)                       # f + 1 = 9 > g
    assert e.value.code == heqg.ERR_ARG
    with pytest.raises(heqg.HeqgError):
        heqg.bbar(np.zeros((0, 3)), 4)
