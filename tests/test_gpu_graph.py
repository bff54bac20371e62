"""Graph-submitted iterations (heqg_nag_qg_graph) against eager ones: every
replay must give the same ciphertexts bit for bit, with eager work and
synchronisations between the replays."""
import numpy as np
import pytest

import synth
from oracle import trainer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _pair(cfgkey, mini, batch, **kw):
    from paper_2406_13221_amd.train import EncryptedQGNAG
    cfg = synth.get_config(cfgkey)
    d = synth.make_dataset(cfg)
    eager = EncryptedQGNAG(cfg, d["X"], d["y"], batch=batch, mini_batch=mini, **kw)
    graph = EncryptedQGNAG(cfg, d["X"], d["y"], batch=batch, mini_batch=mini, graph=True, **kw)
    return cfg, d, eager, graph


def _same(torch, a, b, what):
    assert a.level == b.level and a.scale == b.scale, what
    assert torch.equal(a.data, b.data), what


@pytest.mark.parametrize("mini", [False, True])
def test_graph_replays_match_eager(torch_cuda, mini):
    torch = torch_cuda
    rows = (0, 4096) if mini else None  # mini-batch: 4 batches of 1,024 rows, then replays of two graphs
    cfg, d, eager, graph = _pair("c2", mini, batch=3, rows=rows)
    iters = 6 if mini else 4
    for it in range(iters):
        graph.step()
        torch.cuda.synchronize()
        eager.step()                   # eager work between the replays
        torch.cuda.synchronize()
        _same(torch, graph.W, eager.W, "W%d" % it)
        _same(torch, graph.V, eager.V, "V%d" % it)
        assert graph.state.t == eager.state.t and graph.state.eta == eager.state.eta
    X, y = (d["X"], d["y"]) if rows is None else (d["X"][rows[0]:rows[1]], d["y"][rows[0]:rows[1]])
    ref = trainer.train(X, y, cfg["g"], iters, batch_rows=cfg["batch_rows"] if mini else None)
    w = graph.weights(cfg["g"])
    assert np.abs(w - ref["history"][iters - 1]["W"]).max() < 1e-3


def test_mid_iteration_refresh_runs_without_graph(torch_cuda):
    # the short chain refreshes the gradient every iteration: launched eagerly, same results
    torch = torch_cuda
    cfg, d, eager, graph = _pair("c1", False, batch=1)
    for it in range(2):
        graph.step()
        eager.step()
        torch.cuda.synchronize()
        _same(torch, graph.W, eager.W, "W%d" % it)
        assert graph.state.refreshed_gr == 1


def test_graph_needs_a_stream(torch_cuda):
    from paper_2406_13221_amd import heqg
    from paper_2406_13221_amd.train import EncryptedQGNAG
    cfg = synth.get_config("c1")
    d = synth.make_dataset(cfg)
    run = EncryptedQGNAG(cfg, d["X"], d["y"], batch=1)
    Z = heqg.Cts(run.Z.data, run.Z.level, run.Z.scale)
    with pytest.raises(heqg.HeqgError) as e:
        run.ctx.nag_qg_step(run.keys, Z, run.Bbar, run.W, run.V, run.masks, run.mask_level, run.mask_scales,
                            run.degree, run.state, run.batch, run.ws, stream=0, graph=True)
    assert e.value.code == heqg.ERR_ARG
    assert run.state.t == 0


def test_destroyed_keys_drop_their_graphs(torch_cuda):
    # a graph reads the switching keys it was captured with: destroying the key set drops its
    # graphs, and a new key set (whose handle and buffers may reuse the old addresses) is captured
    # afresh and gives the eager results
    import gc
    from paper_2406_13221_amd.train import rot_steps
    torch = torch_cuda
    cfg, d, eager, graph = _pair("c2", False, batch=3, rows=(0, 1024))
    graph.step()
    eager.step()
    torch.cuda.synchronize()
    assert graph.ctx.graph_count() == 1
    graph.keys = None
    gc.collect()
    assert graph.ctx.graph_count() == 0
    graph.keys = graph.ctx.keygen(cfg["key_seed"], rot_steps(cfg["m"], cfg["g"]))
    graph.step()
    eager.step()
    torch.cuda.synchronize()
    assert graph.ctx.graph_count() == 1
    _same(torch, graph.W, eager.W, "W after a new key set")
    _same(torch, graph.V, eager.V, "V after a new key set")
