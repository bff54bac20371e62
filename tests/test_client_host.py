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


@pytest.mark.parametrize("exact,batch_rows", [(True, 0), (False, 0), (False, 700)])
def test_plain_qgnag_matches_oracle_trainer(heqg, exact, batch_rows):
    """The data owner's FP64 run (heqg_plain_qgnag) against the oracle's trainer: weights and every
    iteration's margins (full batch and ragged mini-batches, exact sigmoid and g8)."""
    rng = np.random.default_rng(11)
    X = rng.uniform(-1, 1, (3000, 9))
    y = (rng.uniform(size=3000) < 0.3).astype(np.int64)
    coeffs = None if exact else trainer.G8
    w, m = heqg.plain_qgnag(X, y, 6, batch_rows=batch_rows, coeffs=coeffs, threads=3)
    ref = trainer.train(X, y, 10, 6, exact_sigmoid=exact, batch_rows=batch_rows or None, log_margins=True)
    assert np.allclose(w, ref["W"][:10], rtol=1e-10, atol=1e-13)
    rm = np.concatenate(ref["margins"])
    assert m.shape == rm.shape
    assert np.allclose(m, rm.astype(np.float32), rtol=1e-6, atol=1e-6)


def test_plain_qgnag_independent_of_threads(heqg):
    rng = np.random.default_rng(12)
    X = rng.uniform(-1, 1, (10000, 5))
    y = (rng.uniform(size=10000) < 0.5).astype(np.int64)
    a = heqg.plain_qgnag(X, y, 3, threads=1)
    b = heqg.plain_qgnag(X, y, 3, threads=8)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
