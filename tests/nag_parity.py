"""Parity harness of the encrypted QG-NAG iteration: the oracle's op-by-op
circuit and heqg_nag_qg_step on identical inputs (ciphertexts encrypted by the
oracle and uploaded; oracle output -> GPU input is allowed), compared residue by
residue after every iteration and every refresh.

Oracles with their keys, GPU contexts with their keys and datasets are cached
per workload, so the paper-size tests pay for key generation once."""
import numpy as np

import synth
from oracle import circuit, trainer
from oracle.ckks import Oracle
from oracle.encode import encode
from paper_2406_13221_amd.train import SIGMOID_SCALE
from tests.gpu_common import assert_same_ct, gpu_ct

_DATA, _ORA, _GPU = {}, {}, {}


def _key(cfgkey, over):
    return (cfgkey, tuple(sorted((k, tuple(v) if isinstance(v, list) else v) for k, v in over.items())))


def config(cfgkey, **over):
    cfg = synth.get_config(cfgkey)
    cfg.update(over)
    return cfg


def dataset(cfgkey, **over):
    k = _key(cfgkey, over)
    if k not in _DATA:
        _DATA[k] = synth.make_dataset(config(cfgkey, **over))
    return _DATA[k]


def oracle_with_keys(cfgkey, **over):
    k = _key(cfgkey, over)
    if k not in _ORA:
        cfg = config(cfgkey, **over)
        o = Oracle.from_config(cfg)
        o.keygen(cfg["key_seed"], circuit.rot_steps(cfg["m"], cfg["g"]))
        _ORA[k] = o
    return _ORA[k]


def gpu_with_keys(cfgkey, **over):
    from paper_2406_13221_amd import heqg
    k = _key(cfgkey, over)
    if k not in _GPU:
        cfg = config(cfgkey, **over)
        ctx = heqg.Context.from_config(cfg)
        _GPU[k] = (ctx, ctx.keygen(cfg["key_seed"], circuit.rot_steps(cfg["m"], cfg["g"])))
    return _GPU[k]


def oracle_setup(cfgkey, coeffs=trainer.G8, rows=None, bbar_rows=None, level=None, **over):
    """Z and B-bar encrypted at the top level, W = V = 0 at `level` (default: the top) and the
    sigmoid masks planned for it."""
    cfg = config(cfgkey, **over)
    d = dataset(cfgkey, **over)
    X, y = d["X"], d["y"]
    if rows:
        X, y = X[rows[0]:rows[1]], y[rows[0]:rows[1]]
    o = oracle_with_keys(cfgkey, **over)
    N, m, g = o.N, cfg["m"], cfg["g"]
    Z = trainer.build_Z(X, y, g)
    blocks = circuit.pack_blocks(Z, m, g, N)
    L = o.top_level
    Zc = [o.encrypt(encode(blocks[b], N, o.delta), L, o.delta, cfg["enc_seed"], b) for b in range(len(blocks))]
    XB = X if bbar_rows is None else X[bbar_rows[0]:bbar_rows[1]]
    B = trainer.bbar(XB, g)
    sB = 2.0 ** (cfg["log2_scale"] + 10) / B.max()
    Bc = o.encrypt(encode(circuit.replicate_row(B, m, g), N, sB), L, sB, cfg["enc_seed"], 1 << 20)
    lw = L if level is None else level
    W = o.encrypt(np.zeros(N, np.int64), lw, o.delta, cfg["enc_seed"], (1 << 20) + 1)
    V = o.encrypt(np.zeros(N, np.int64), lw, o.delta, cfg["enc_seed"], (1 << 20) + 2)
    masks = circuit.make_masks(o, m, g, coeffs, lw, SIGMOID_SCALE)
    return cfg, o, X, y, Zc, Bc, W, V, masks


def gpu_side(cfg, o, Zc, Bc, W, V, masks, coeffs, cfgkey=None, **over):
    """GPU context and keys (cached per workload when cfgkey is given) and the oracle's
    inputs uploaded."""
    import torch
    from paper_2406_13221_amd import heqg
    if cfgkey is None:
        ctx = heqg.Context.from_config(cfg)
        keys = ctx.keygen(cfg["key_seed"], circuit.rot_steps(cfg["m"], cfg["g"]))
    else:
        ctx, keys = gpu_with_keys(cfgkey, **over)
    Z = heqg.Cts(torch.from_numpy(np.stack([z.data for z in Zc]).view(np.int64).copy()).cuda(), Zc[0].level,
                 Zc[0].scale)
    order = sorted(coeffs) + ["half"]
    mk = torch.from_numpy(np.stack([masks[k][0] for k in order]).view(np.int64).copy()).cuda()
    scales = [masks[k][1] for k in order]
    return ctx, keys, Z, gpu_ct(ctx, Bc), gpu_ct(ctx, W), gpu_ct(ctx, V), mk, scales


def gpu_state(ost, m, g):
    from paper_2406_13221_amd import heqg
    return heqg.NagStateS(ost["t"], ost["alpha0"], ost["alpha1"], 2.0, 1.0, 81.0, 2.5, m, g, ost["refresh_seed"],
                          0.0, 0.0, 0)


def run_parity(cfgkey, iters, batch, coeffs=trainer.G8, rows=None, bbar_rows=None, split=None, graph=False,
               level=None, **over):
    """iters iterations (each followed by a refresh of W and V back to their level) on both sides,
    compared residue by residue; split: the NTT pass split the GPU context uses (restored after);
    level: the level W and V are encrypted and refreshed at (default: the top)."""
    print("nag parity: %s iters=%d batch=%d rows=%s degree=%d split=%s graph=%s level=%s" %
          (cfgkey, iters, batch, rows, max(coeffs), split, graph, level), flush=True)
    cfg, o, X, y, Zc, Bc, W, V, masks = oracle_setup(cfgkey, coeffs, rows, bbar_rows, level, **over)
    m, g = cfg["m"], cfg["g"]
    L = o.top_level if level is None else level
    ctx, keys, gZ, gB, gW, gV, mk, scales = gpu_side(cfg, o, Zc, Bc, W, V, masks, coeffs, cfgkey, **over)
    deg = max(coeffs)
    saved = ctx.tune_get(2)
    if split is not None:
        assert ctx.tune_set(2, split)
    stream = None
    if graph:
        import torch
        stream = torch.cuda.Stream()
    try:
        ost = circuit.new_state(refresh_seed=7)
        gst = gpu_state(ost, m, g)
        for it in range(iters):
            W, V, ost = circuit.nag_qg_step(o, Zc, Bc, W, V, ost, masks, m, g, degree=deg)
            if graph:
                import torch
                stream.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(stream):
                    ctx.nag_qg_step(keys, gZ, gB, gW, gV, mk, L - 1, scales, deg, gst, batch,
                                    stream=stream.cuda_stream, graph=True)
                torch.cuda.current_stream().wait_stream(stream)
            else:
                ctx.nag_qg_step(keys, gZ, gB, gW, gV, mk, L - 1, scales, deg, gst, batch)
            assert_same_ct(gW, W, "W%d" % it)
            assert_same_ct(gV, V, "V%d" % it)
            assert gst.t == ost["t"] and gst.alpha1 == ost["alpha1"] and gst.eta == ost["eta"]
            assert bool(gst.refreshed_gr) == ost["refreshed_gr"]
            W = o.refresh(W, L, 99, 2 * it)
            V = o.refresh(V, L, 99, 2 * it + 1)
            gW = ctx.refresh(keys, gW, L, 99, 2 * it)
            gV = ctx.refresh(keys, gV, L, 99, 2 * it + 1)
            assert_same_ct(gW, W, "W%d-refreshed" % it)
    finally:
        ctx.tune_set(2, saved)
    return o, W


# ---------------------------------------------------------------- the m x g partition (section 2.2)
def grid_oracle_setup(cfgkey, rows=None, coeffs=trainer.G8, **over):
    """Row blocks x column blocks of Z and one B-bar, W, V ciphertext per column block, encrypted by the
    oracle (object ids: i * C + j for Z; 2^20 + j, 2^21 + j, 2^22 + j for B-bar, W, V)."""
    cfg = config(cfgkey, **over)
    d = dataset(cfgkey, **over)
    X, y = d["X"], d["y"]
    if rows:
        X, y = X[rows[0]:rows[1]], y[rows[0]:rows[1]]
    o = oracle_with_keys(cfgkey, **over)
    N, m, g = o.N, cfg["m"], cfg["g"]
    G, nc = synth.padded_width(cfg), synth.col_blocks(cfg)
    grid = circuit.pack_grid(trainer.build_Z(X, y, G), m, g, N)
    L = o.top_level
    Zg = [[o.encrypt(encode(grid[i, j], N, o.delta), L, o.delta, cfg["enc_seed"], i * nc + j) for j in range(nc)]
          for i in range(grid.shape[0])]
    B = trainer.bbar(X, G)
    sB = 2.0 ** (cfg["log2_scale"] + 10) / B.max()
    Bc = [o.encrypt(encode(circuit.replicate_row(B[j * g:(j + 1) * g], m, g), N, sB), L, sB, cfg["enc_seed"],
                    (1 << 20) + j) for j in range(nc)]
    zero = np.zeros(N, np.int64)
    W = [o.encrypt(zero, L, o.delta, cfg["enc_seed"], (1 << 21) + j) for j in range(nc)]
    V = [o.encrypt(zero, L, o.delta, cfg["enc_seed"], (1 << 22) + j) for j in range(nc)]
    masks = circuit.make_masks(o, m, g, coeffs, L, SIGMOID_SCALE)
    return cfg, o, X, y, Zg, Bc, W, V, masks


def stack_cts(cts):
    """Oracle ciphertexts of one level and scale -> one GPU Cts batch (upload of oracle output)."""
    import torch
    from paper_2406_13221_amd import heqg
    return heqg.Cts(torch.from_numpy(np.stack([c.data for c in cts]).view(np.int64).copy()).cuda(), cts[0].level,
                    cts[0].scale)


def assert_same_cts(g, cts, what):
    """A GPU batch against a list of oracle ciphertexts, residue by residue."""
    got = g.data.cpu().numpy().view(np.uint64)
    assert g.level == cts[0].level and g.scale == cts[0].scale, (what, g.level, cts[0].level)
    for j, c in enumerate(cts):
        if not np.array_equal(got[j], c.data):
            bad = np.argwhere(got[j] != c.data)
            raise AssertionError("%s[%d]: %d of %d residues differ, first at %s" % (what, j, len(bad), c.data.size,
                                                                                  bad[0]))


def run_grid_parity(cfgkey, iters, batch, rows=None, first_order=False, **over):
    """iters iterations over the partition on both sides (W, V refreshed after each), compared residue
    by residue; the workload's sigmoid (g8 or g16) and learning-rate horizon; first_order: the
    first-order NAG baseline with step lr0 / n (the workload's fo_lr).  Returns the oracle, its last W
    list and the rows."""
    import functools
    print("grid parity: %s iters=%d batch=%d rows=%s first_order=%s" % (cfgkey, iters, batch, rows, first_order),
          flush=True)
    cfg0 = config(cfgkey, **over)
    coeffs = trainer.G16 if cfg0.get("sigmoid") == "g16" else trainer.G8
    cfg, o, X, y, Zg, Bc, W, V, masks = grid_oracle_setup(cfgkey, rows, coeffs=coeffs, **over)
    m, g, L, nc = cfg["m"], cfg["g"], o.top_level, len(W)
    lr_fn = functools.partial(trainer.f2_lr, T=cfg["lr_T"])
    fo_gamma = cfg["fo_lr"] / X.shape[0] if first_order else None
    ctx, keys = gpu_with_keys(cfgkey, **over)
    import torch
    gZ = stack_cts([c for row in Zg for c in row])
    gB, gW, gV = stack_cts(Bc), stack_cts(W), stack_cts(V)
    order = [1, 3, "half"]
    mk = torch.from_numpy(np.stack([masks[k][0] for k in order]).view(np.int64).copy()).cuda()
    scales = [masks[k][1] for k in order]
    ost = circuit.new_state(refresh_seed=7)
    gst = gpu_state(ost, m, g)
    gst.col_blocks = nc
    gst.T = cfg["lr_T"]
    if first_order:
        gst.first_order, gst.fo_gamma = 1, fo_gamma
    for it in range(iters):
        W, V, ost = circuit.nag_qg_step_grid(o, Zg, Bc, W, V, ost, masks, m, g, lr_fn=lr_fn, fo_gamma=fo_gamma)
        ctx.nag_qg_step(keys, gZ, None if first_order else gB, gW, gV, mk, L - 1, scales, 3, gst, batch)
        assert_same_cts(gW, W, "W%d" % it)
        assert_same_cts(gV, V, "V%d" % it)
        assert gst.t == ost["t"] and gst.eta == ost["eta"] and bool(gst.refreshed_gr) == ost["refreshed_gr"]
        W = [o.refresh(w, L, 99, 4 * it + j) for j, w in enumerate(W)]
        V = [o.refresh(v, L, 99, 4 * it + 2 + j) for j, v in enumerate(V)]
        gW = ctx.refresh(keys, gW, L, 99, 4 * it)
        gV = ctx.refresh(keys, gV, L, 99, 4 * it + 2)
        assert_same_cts(gW, W, "W%d-refreshed" % it)
    return o, W, X, y
