"""Pins for the oracle's encrypted QG-NAG iteration: its decryptions must follow
the FP64 plaintext trainer (same sigma~, same schedule) within the stated
tolerance, and its intermediates must decrypt to the plaintext quantities."""
import numpy as np
import pytest

import synth
from oracle import circuit, trainer
from oracle.ckks import Oracle
from oracle.encode import encode

TOL_W = 1e-3


def setup_run(cfgkey, degree_coeffs=trainer.G8, n_rows=None, batch=None, **over):
    cfg = synth.get_config(cfgkey)
    cfg.update(over)
    d = synth.make_dataset(cfg)
    X, y = d["X"], d["y"]
    if n_rows:
        X, y = X[:n_rows], y[:n_rows]
    o = Oracle.from_config(cfg)
    N, m, g = o.N, cfg["m"], cfg["g"]
    o.keygen(cfg["key_seed"], circuit.rot_steps(m, g))
    Z = trainer.build_Z(X, y, g)
    blocks = circuit.pack_blocks(Z, m, g, N)
    L = o.top_level
    Zc = [o.encrypt(encode(blocks[b], N, o.delta), L, o.delta, cfg["enc_seed"], b) for b in range(len(blocks))]
    B = trainer.bbar(X, g)
    sB = 2.0 ** 50 / B.max()
    Bc = o.encrypt(encode(circuit.replicate_row(B, m, g), N, sB), L, sB, cfg["enc_seed"], 1 << 20)
    W = o.encrypt(np.zeros(N, np.int64), L, o.delta, cfg["enc_seed"], (1 << 20) + 1)
    V = o.encrypt(np.zeros(N, np.int64), L, o.delta, cfg["enc_seed"], (1 << 20) + 2)
    masks = circuit.make_masks(o, m, g, degree_coeffs, L, o.delta)
    return cfg, o, X, y, Zc, Bc, W, V, masks


def test_c1_three_iterations_match_fp64():
    cfg, o, X, y, Zc, Bc, W, V, masks = setup_run("c1")
    m, g, L = cfg["m"], cfg["g"], o.top_level
    ref = trainer.train(X, y, g, cfg["iters"])
    st = circuit.new_state(refresh_seed=7)
    for it in range(cfg["iters"]):
        trace = []
        W, V, st = circuit.nag_qg_step(o, Zc, Bc, W, V, st, masks, m, g, trace=trace)
        # depth: 4 levels on c1, so the gradient ciphertext is refreshed mid-iteration
        assert st["refreshed_gr"]
        W = o.refresh(W, L, 99, 2 * it)
        V = o.refresh(V, L, 99, 2 * it + 1)
        w = o.decrypt_values(W, g).real
        v = o.decrypt_values(V, g).real
        assert np.abs(w - ref["history"][it]["W"]).max() < TOL_W
        if it == cfg["iters"] - 1:
            assert np.abs(v - ref["V"]).max() < TOL_W
    # weights are replicated in every row of the slots
    full = o.decrypt_values(W).real.reshape(m, g)
    assert np.abs(full - full[0]).max() < 1e-6


def test_c1_intermediates_decrypt_to_plaintext_quantities():
    cfg, o, X, y, Zc, Bc, W, V, masks = setup_run("c1")
    m, g = cfg["m"], cfg["g"]
    # one step from a nonzero W: encrypt a W vector replicated across rows
    rng = np.random.default_rng(3)
    w = np.zeros(g)
    w[: X.shape[1] + 1] = rng.normal(size=X.shape[1] + 1) * 0.5
    Wc = o.encrypt(encode(circuit.replicate_row(w, m, g), o.N, o.delta), o.top_level, o.delta, 9, 9)
    trace = []
    circuit.nag_qg_step(o, Zc, Bc, Wc, Wc, circuit.new_state(7), masks, m, g, trace=trace)
    tr = dict(trace)
    Z = trainer.build_Z(X, y, g)
    Zp = np.zeros((m, g))
    Zp[: Z.shape[0]] = Z
    margins = Zp @ w
    u = o.decrypt_values(tr["u0"]).real.reshape(m, g)
    assert np.abs(u[:, 0] - margins).max() < 1e-6
    p = o.decrypt_values(tr["p0"]).real.reshape(m, g)
    p_ref = 1 - trainer.sigma_tilde(margins, trainer.G8)
    assert np.abs(p - p_ref[:, None]).max() < 1e-6
    gr = o.decrypt_values(tr["gr"]).real.reshape(m, g)
    assert np.abs(gr - (Zp.T @ p_ref)[None, :]).max() < 1e-5


@pytest.mark.parametrize("degree", [5, 7])
def test_learned_degree_circuits_match_fp64(degree):
    # odd polynomials 1/2 + sum c_k (m/8)^k: the depth-3 mask-folded evaluation
    base = {5: [0.19129, -4.5951e-3, 4.2214e-5], 7: [0.21689, -8.1934e-3, 1.6588e-4, -1.1959e-6]}[degree]
    coeffs = {2 * i + 1: c for i, c in enumerate(base)}
    # c1 shapes with a deeper chain (8 primes): degree 5/7 needs 6 levels per iteration
    cfg, o, X, y, Zc, Bc, W, V, masks = setup_run("c1", degree_coeffs=coeffs, q_bits=[50] + [40] * 7, n_p=3)
    m, g = cfg["m"], cfg["g"]
    ref = trainer.train(X, y, g, 2, coeffs=coeffs)
    st = circuit.new_state(refresh_seed=7)
    for it in range(2):
        W, V, st = circuit.nag_qg_step(o, Zc, Bc, W, V, st, masks, m, g, degree=degree)
        W = o.refresh(W, o.top_level, 99, 2 * it)
        V = o.refresh(V, o.top_level, 99, 2 * it + 1)
        assert np.abs(o.decrypt_values(W, g).real - ref["history"][it]["W"]).max() < TOL_W


def test_scale_mismatch_is_an_error():
    cfg, o, X, y, Zc, Bc, W, V, masks = setup_run("c1")
    bad = W.copy()
    bad.scale *= 1.001
    with pytest.raises(ValueError):
        o.add(W, bad)


# ---------------------------------------------------------------- m x g partition (section 2.2)
def setup_grid(cfgkey, **over):
    """Row blocks i x column blocks j of Z, and B-bar, W, V as one ciphertext per column block."""
    cfg = synth.get_config(cfgkey)
    cfg.update(over)
    d = synth.make_dataset(cfg)
    X, y = d["X"], d["y"]
    o = Oracle.from_config(cfg)
    N, m, g = o.N, cfg["m"], cfg["g"]
    G, nc = synth.padded_width(cfg), synth.col_blocks(cfg)
    o.keygen(cfg["key_seed"], circuit.rot_steps(m, g))
    grid = circuit.pack_grid(trainer.build_Z(X, y, G), m, g, N)
    L = o.top_level
    Zg = [[o.encrypt(encode(grid[i, j], N, o.delta), L, o.delta, cfg["enc_seed"], i * nc + j) for j in range(nc)]
          for i in range(grid.shape[0])]
    B = trainer.bbar(X, G)
    sB = 2.0 ** 50 / B.max()
    Bc = [o.encrypt(encode(circuit.replicate_row(B[j * g:(j + 1) * g], m, g), N, sB), L, sB, cfg["enc_seed"],
                    (1 << 20) + j) for j in range(nc)]
    zero = np.zeros(N, np.int64)
    W = [o.encrypt(zero, L, o.delta, cfg["enc_seed"], (1 << 21) + j) for j in range(nc)]
    V = [o.encrypt(zero, L, o.delta, cfg["enc_seed"], (1 << 22) + j) for j in range(nc)]
    masks = circuit.make_masks(o, m, g, trainer.G8, L, o.delta)
    return cfg, o, X, y, Zg, Bc, W, V, masks


def test_pack_grid_layout():
    Z = np.arange(5 * 6, dtype=float).reshape(5, 6)
    out = circuit.pack_grid(Z, 2, 3, 12)          # m = 2 rows, g = 3 columns, 6 slots
    assert out.shape == (3, 2, 6)
    assert np.array_equal(out[0, 1], [3, 4, 5, 9, 10, 11])
    assert np.array_equal(out[2, 0], [24, 25, 26, 0, 0, 0])   # last row block zero-padded
    # the single-column-block packing is the grid's j = 0
    assert np.array_equal(circuit.pack_grid(Z[:, :3], 2, 3, 12)[:, 0], circuit.pack_blocks(Z[:, :3], 2, 3, 12))


def test_grid_iterations_match_fp64():
    """2 iterations over 3 row blocks (the last ragged) x 2 column blocks follow the FP64 trainer on the
    padded width; the split of the model over column blocks does not change the method (section 2.2)."""
    cfg, o, X, y, Zg, Bc, W, V, masks = setup_grid("c1g")
    m, g, L, nc = cfg["m"], cfg["g"], o.top_level, len(W)
    assert (len(Zg), nc) == (3, 2)
    G = nc * g
    ref = trainer.train(X, y, G, 2)
    st = circuit.new_state(refresh_seed=7)
    for it in range(2):
        W, V, st = circuit.nag_qg_step_grid(o, Zg, Bc, W, V, st, masks, m, g)
        assert st["refreshed_gr"]
        W = [o.refresh(w, L, 99, 4 * it + j) for j, w in enumerate(W)]
        V = [o.refresh(v, L, 99, 4 * it + 2 + j) for j, v in enumerate(V)]
        w = np.concatenate([o.decrypt_values(c, g).real for c in W])
        assert np.abs(w - ref["history"][it]["W"]).max() < TOL_W
    v = np.concatenate([o.decrypt_values(c, g).real for c in V])
    assert np.abs(v - ref["V"]).max() < TOL_W


def test_grid_intermediates_are_the_plaintext_quantities():
    """From a nonzero W: row block 0's margins sum the products of both column blocks; the
    sigmoid column is replicated; column block 0's gradient sums every row block."""
    cfg, o, X, y, Zg, Bc, W, V, masks = setup_grid("c1g")
    m, g, nc = cfg["m"], cfg["g"], len(W)
    G = nc * g
    rng = np.random.default_rng(3)
    w = np.zeros(G)
    w[: X.shape[1] + 1] = rng.normal(size=X.shape[1] + 1) * 0.5
    Wc = [o.encrypt(encode(circuit.replicate_row(w[j * g:(j + 1) * g], m, g), o.N, o.delta), o.top_level,
                    o.delta, 9, 9 + j) for j in range(nc)]
    trace = []
    circuit.nag_qg_step_grid(o, Zg, Bc, Wc, Wc, circuit.new_state(7), masks, m, g, trace=trace)
    tr = dict(trace)
    Z = trainer.build_Z(X, y, G)
    Zp = np.zeros((len(Zg) * m, G))
    Zp[: Z.shape[0]] = Z
    margins = Zp @ w
    u = o.decrypt_values(tr["u0"]).real.reshape(m, g)
    assert np.abs(u[:, 0] - margins[:m]).max() < 1e-6
    p_ref = 1 - trainer.sigma_tilde(margins, trainer.G8)
    p = o.decrypt_values(tr["p0"]).real.reshape(m, g)
    assert np.abs(p - p_ref[:m, None]).max() < 1e-6
    # padding rows of the last row block have zero Z, so they add nothing to the gradient
    gr = o.decrypt_values(tr["gr"]).real.reshape(m, g)
    assert np.abs(gr - (Zp[:, :g].T @ p_ref)[None, :]).max() < 1e-5



@pytest.mark.parametrize("cfgkey", ["c1", "c1g"])
def test_first_order_nag_matches_fp64(cfgkey):
    """The first-order NAG baseline (no B-bar; the gradient times lr0 / n) follows the FP64 trainer's
    first-order run, on one column block and on the grid."""
    lr0 = 1.0
    if cfgkey == "c1":
        cfg, o, X, y, Zc, Bc, W, V, masks = setup_run("c1")
        Zg, W, V = [[z] for z in Zc], [W], [V]
    else:
        cfg, o, X, y, Zg, Bc, W, V, masks = setup_grid("c1g")
    m, g, L, nc = cfg["m"], cfg["g"], o.top_level, len(W)
    G = nc * g
    gamma = lr0 / X.shape[0]
    ref = trainer.train(X, y, G, 2, first_order=lr0)
    st = circuit.new_state(refresh_seed=7)
    for it in range(2):
        W, V, st = circuit.nag_qg_step_grid(o, Zg, None, W, V, st, masks, m, g, fo_gamma=gamma)
        W = [o.refresh(w, L, 99, 4 * it + j) for j, w in enumerate(W)]
        V = [o.refresh(v, L, 99, 4 * it + 2 + j) for j, v in enumerate(V)]
        w = np.concatenate([o.decrypt_values(c, g).real for c in W])
        assert np.abs(w - ref["history"][it]["W"]).max() < TOL_W
    # the first-order run moves differently from the quadratic-gradient one
    assert np.abs(ref["W"] - trainer.train(X, y, G, 2)["W"]).max() > 10 * TOL_W



@pytest.mark.parametrize("cfgkey", ["c1", "c1g"])
def test_encrypted_scores_are_the_plaintext_scores(cfgkey):
    """Encrypted scoring: column 0 of every row decrypts to x-hat . w of that row (validation rows,
    no labels), on one column block and on the grid; the AUROC of the decrypted scores is the
    plaintext one."""
    cfg = synth.get_config(cfgkey)
    d = synth.make_dataset(cfg)
    o = Oracle.from_config(cfg)
    m, g = cfg["m"], cfg["g"]
    G, nc = synth.padded_width(cfg), synth.col_blocks(cfg)
    o.keygen(cfg["key_seed"], circuit.rot_steps(m, g))
    Xv, yv = d["Xv"][:700], d["yv"][:700]
    grid = circuit.pack_grid(trainer.xhat(Xv, G), m, g, o.N)
    L = o.top_level
    Xg = [[o.encrypt(encode(grid[i, j], o.N, o.delta), L, o.delta, 5, i * nc + j) for j in range(nc)]
          for i in range(grid.shape[0])]
    rng = np.random.default_rng(8)
    w = np.zeros(G)
    w[: Xv.shape[1] + 1] = rng.normal(size=Xv.shape[1] + 1) * 0.5
    Wc = [o.encrypt(encode(circuit.replicate_row(w[j * g:(j + 1) * g], m, g), o.N, o.delta), L, o.delta, 6, j)
          for j in range(nc)]
    us = circuit.score_grid(o, Xg, Wc, m, g)
    got = np.concatenate([o.decrypt_values(u).real.reshape(m, g)[:, 0] for u in us])[: len(yv)]
    ref = trainer.xhat(Xv, G) @ w
    assert np.abs(got - ref).max() < 1e-6
    assert abs(trainer.auroc(got, yv) - trainer.auroc(ref, yv)) < 1e-9
