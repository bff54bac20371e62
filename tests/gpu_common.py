"""Shared helpers for the GPU parity tests (GPU path vs the CPU oracle)."""
import numpy as np

import synth
from oracle.ckks import Oracle


def cpu_u64(t):
    return t.detach().cpu().numpy().view(np.uint64)


def make_pair(cfgkey, rot_steps=None, **over):
    from paper_2406_13221_amd import heqg
    cfg = synth.get_config(cfgkey)
    cfg.update(over)
    ora = Oracle.from_config(cfg)
    ctx = heqg.Context.from_config(cfg)
    return cfg, ora, ctx


def gpu_ct(ctx, oct_):
    """Upload an oracle ciphertext (oracle output -> GPU input is allowed)."""
    import torch
    from paper_2406_13221_amd import heqg
    d = torch.from_numpy(oct_.data.view(np.int64).copy()).cuda()[None]
    return heqg.Cts(d, oct_.level, oct_.scale)


def assert_same_ct(g, o, what=""):
    got = cpu_u64(g.data)[0] if g.data.dim() == 4 else cpu_u64(g.data)
    assert g.level == o.level, (what, g.level, o.level)
    assert got.shape == o.data.shape, (what, got.shape, o.data.shape)
    if not np.array_equal(got, o.data):
        bad = np.argwhere(got != o.data)
        raise AssertionError("%s: %d of %d residues differ, first at %s" % (what, len(bad), got.size, bad[0]))
    assert g.scale == o.scale, (what, g.scale, o.scale)
