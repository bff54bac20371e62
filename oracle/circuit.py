"""TEST INFRASTRUCTURE: one encrypted QG-NAG iteration on the oracle, op by op.

Layout (section 2.2): Z is cut into blocks of m rows x g columns, m*g = N/2,
each packed row by row into the slots of one ciphertext; W, V and B-bar hold
one g-vector replicated in every row (section 4.3).

Per block b (steps 4-6 of section 4.3, the order both implementations follow):
  u   = Rescale(Relin(Z_b (x) W))                       margins' partial products
  u  += Rot(u, 2^k), k < log2 g                         row sums land in column 0
  sigma~ on column 0, masked (filter matrix F, section 2.2):
      a_1 = Rescale(u * M_1),  M_k = encode(-c_k * F) at the planned scale
      s   = Rescale(Relin(u (x) u))                     m^2
      b_k = Rescale(u * M_k)                            for every odd k >= 3
      t_3 = Rescale(Relin(b_3 (x) s));  s4 = Rescale(Relin(s (x) s)) when degree >= 5
      t_5 = Rescale(Relin(b_5 (x) s4)); t_7 = Rescale(Relin(Rescale(Relin(b_7 (x) s)) (x) s4))
      p   = a_1 + t_3 (+ t_5 + t_7) + encode(F/2)        = (1 - sigma~(m)) in column 0
  p  += Rot(p, -2^k), k < log2 g                         replicate across the row
  acc += Z_b (x) p                                       three-part, relinearised once
After the blocks:
  gr = Rescale(Relin(acc));  gr += Rot(gr, g 2^k), k < log2 m      column sums
  (key-holder refresh of gr when fewer than one level is left)
  B_v = cMul(B-bar, lr),  B_w = cMul(B-bar, lr (1 - eta))
  G_v = Rescale(Relin(B_v (x) gr)),  G_w = Rescale(Relin(B_w (x) gr))
  V' = cMul(W, 1) + G_v;   W' = cMul(W, 1 - eta) + cMul(V, eta) + G_w
Every cMul targets the working scale Delta, so W' and V' come out at Delta.

With several column blocks (section 2.2: Z cut into m x g sub-matrices Z_ij, the
model into g-column pieces W_j), nag_qg_step_grid sums the tensor products
Z_ij (x) W_j of a row block before its one relinearisation, and column block j
accumulates sum_i Z_ij (x) p_i; the rest runs per column block as above.
"""
import math

import numpy as np

from .encode import encode
from .trainer import alpha_next, f2_lr


def rot_steps(m, g):
    lg, lm = int(math.log2(g)), int(math.log2(m))
    return [1 << k for k in range(lg)] + [-(1 << k) for k in range(lg)] + [g << k for k in range(lm)]


def pack_blocks(Z, m, g, N):
    """Rows of Z (n x g) into ceil(n/m) slot vectors of N/2 entries (zero-padded)."""
    n = Z.shape[0]
    nb = (n + m - 1) // m
    out = np.zeros((nb, N // 2))
    for b in range(nb):
        rows = Z[b * m: (b + 1) * m]
        out[b, : rows.size] = rows.reshape(-1)
    return out


def pack_grid(Z, m, g, N):
    """The partition of section 2.2: Z (n x G, G a multiple of g) into ceil(n/m) x G/g
    sub-matrices of m rows and g columns (zero rows pad the last row block), each packed
    row by row into one slot vector of N/2 entries: out[i][j]."""
    n, G = Z.shape
    if G % g:
        raise ValueError("the padded width must be a multiple of g")
    nr, nc = (n + m - 1) // m, G // g
    out = np.zeros((nr, nc, N // 2))
    for i in range(nr):
        for j in range(nc):
            blk = Z[i * m: (i + 1) * m, j * g: (j + 1) * g]
            out[i, j, : blk.size] = blk.reshape(-1)
    return out


def replicate_row(vec, m, g):
    v = np.zeros(g)
    v[: len(vec)] = vec
    return np.tile(v, m)


def column0_mask(m, g):
    F = np.zeros((m, g))
    F[:, 0] = 1.0
    return F.reshape(-1)


def terms(coeffs):
    return sorted(coeffs.items())


def mask_scales(primes, level, s_z, s_w, s_c, degree):
    """Plaintext scales for the masked sigmoid so that every term lands at s_c.

    level: the level at which Z (x) W is taken.  Returns {k: scale} and the
    scale of the F/2 plaintext (= s_c)."""
    q = [float(p) for p in primes]
    lv = level
    s_u = s_z * s_w / q[lv]
    s_s = s_u * s_u / q[lv - 1]
    out = {1: s_c * q[lv - 1] / s_u, 3: s_c * q[lv - 2] * q[lv - 1] / (s_u * s_s)}
    if degree >= 5:
        s_s4 = s_s * s_s / q[lv - 2]
        out[5] = s_c * q[lv - 3] * q[lv - 1] / (s_u * s_s4)
        if degree >= 7:
            out[7] = s_c * q[lv - 3] * q[lv - 2] * q[lv - 1] / (s_u * s_s * s_s4)
    return out


def make_masks(ora, m, g, coeffs, level, s_c):
    """NTT-form mask plaintexts at level-1 for the sigmoid terms, plus F/2; encoded by the oracle."""
    deg = max(coeffs)
    sc = mask_scales(ora.primes, level, ora.delta, ora.delta, s_c, deg)
    F = column0_mask(m, g)
    pts = {}
    for k, c in terms(coeffs):
        pts[k] = (ora.pt_from_int(encode(-c * F, ora.N, sc[k]), level - 1), sc[k])
    pts["half"] = (ora.pt_from_int(encode(0.5 * F, ora.N, s_c), level - 1), s_c)
    return pts


def new_state(refresh_seed=0):
    a0 = 0.01
    return dict(t=0, alpha0=a0, alpha1=alpha_next(a0), refresh_seed=refresh_seed, refreshed_gr=False)


def sigmoid_block(ora, u, masks, degree):
    a1 = ora.rescale(ora.mul_pt(u, *masks[1]))
    s = ora.rescale(ora.hmult(u, u))
    p = a1
    s4 = None
    if degree >= 5:
        s4 = ora.rescale(ora.hmult(s, s))
    b3 = ora.rescale(ora.mul_pt(u, *masks[3]))
    t3 = ora.rescale(ora.hmult(b3, s))
    p = ora.add(p, t3)
    if degree >= 5:
        b5 = ora.rescale(ora.mul_pt(u, *masks[5]))
        t5 = ora.rescale(ora.hmult(b5, s4))
        p = ora.add(p, t5)
    if degree >= 7:
        b7 = ora.rescale(ora.mul_pt(u, *masks[7]))
        t7a = ora.rescale(ora.hmult(b7, s))
        t7 = ora.rescale(ora.hmult(t7a, s4))
        p = ora.add(p, t7)
    return ora.add_pt(p, *masks["half"])


def nag_qg_step(ora, Z_cts, B_ct, W, V, state, masks, m, g, degree=3, lr_fn=f2_lr, trace=None, fo_gamma=None):
    """One iteration with one column block (g >= f + 1); returns (W', V', new_state).
    trace (list) collects intermediates."""
    Wn, Vn, st = nag_qg_step_grid(ora, [[z] for z in Z_cts], [B_ct], [W], [V], state, masks, m, g, degree,
                                  lr_fn, trace, fo_gamma)
    return Wn[0], Vn[0], st


# Objects of the mid-iteration refresh of the gradient ciphertexts: (t << 4) | 2, plus j for
# column block j, so at most this many column blocks may take it.
MAX_REFRESH_COL_BLOCKS = 14


def nag_qg_step_grid(ora, Z_grid, B_cts, Ws, Vs, state, masks, m, g, degree=3, lr_fn=f2_lr, trace=None,
                     fo_gamma=None):
    """One iteration over the m x g sub-matrix partition of section 2.2: Z_grid[i][j] is row
    block i, column block j (columns j*g .. j*g + g - 1 of Z); B_cts, Ws and Vs hold one
    ciphertext per column block.  The margins of row block i are the row sums of
    sum_j Z_ij (x) W_j (the tensor products added in three-part form, relinearised once);
    the sigmoid, replicated across the row, then multiplies every Z_ij, and column block j
    accumulates its own gradient sum_i Z_ij (x) p_i, whose column sums, B-bar product and NAG
    update stay within that block.  Returns (W'_j list, V'_j list, new_state).

    fo_gamma: the first-order NAG the paper compares against (section 3.2, Fig. 1): the gradient
    ciphertexts are multiplied by the constants fo_gamma and fo_gamma (1 - eta) instead of the
    B-bar products (B_cts unused), with lr = 1; the rest of the update is unchanged."""
    lg, lm = int(math.log2(g)), int(math.log2(m))
    nc = len(Ws)
    if fo_gamma is not None:
        B_cts = [None] * nc
    if not (len(Vs) == len(B_cts) == nc and all(len(row) == nc for row in Z_grid)):
        raise ValueError("every row block needs one ciphertext per column block")
    acc = [None] * nc
    for i, row in enumerate(Z_grid):
        t3 = None
        for j in range(nc):
            prod = ora.tensor(row[j], Ws[j])
            t3 = prod if t3 is None else ora.add(t3, prod)
        u = ora.rescale(ora.relin(t3))
        for k in range(lg):
            u = ora.add(u, ora.rotate(u, 1 << k))
        p = sigmoid_block(ora, u, masks, degree)
        for k in range(lg):
            p = ora.add(p, ora.rotate(p, -(1 << k)))
        for j in range(nc):
            prod = ora.tensor(row[j], p)
            acc[j] = prod if acc[j] is None else ora.add(acc[j], prod)
        if trace is not None and i == 0:
            trace.append(("u0", u))
            trace.append(("p0", p))
    grs = []
    for j in range(nc):
        gr = ora.rescale(ora.relin(acc[j]))
        for k in range(lm):
            gr = ora.add(gr, ora.rotate(gr, g << k))
        grs.append(gr)
    if trace is not None:
        trace.append(("gr", grs[0]))
    st = dict(state)
    t = st["t"]
    B0 = B_cts[0]
    if min(grs[0].level if fo_gamma is not None else B0.level - 1, grs[0].level) < 1:
        if nc > MAX_REFRESH_COL_BLOCKS:
            raise ValueError("too many column blocks for a mid-iteration refresh")
        grs = [ora.refresh(gr, ora.top_level, st["refresh_seed"], ((t << 4) | 2) + j) for j, gr in enumerate(grs)]
        st["refreshed_gr"] = True
    eta = (1.0 - st["alpha0"]) / st["alpha1"]
    lr = lr_fn(t) if fo_gamma is None else 1.0
    s_g = ora.delta
    Wn, Vn = [], []
    for j in range(nc):
        gr = grs[j]
        if fo_gamma is None:
            lt = min(B_cts[j].level - 1, gr.level)
            s_bv = s_g * float(ora.q(lt)) / gr.scale
            Bv = ora.mul_const(B_cts[j], lr, s_bv)
            Bw = ora.mul_const(B_cts[j], lr * (1.0 - eta), s_bv)
            Gv = ora.rescale(ora.hmult(Bv, gr))
            Gw = ora.rescale(ora.hmult(Bw, gr))
        else:
            Gv = ora.mul_const(gr, fo_gamma, s_g)
            Gw = ora.mul_const(gr, fo_gamma * (1.0 - eta), s_g)
        Vn.append(ora.add(ora.mul_const(Ws[j], 1.0, s_g), Gv))
        Wn.append(ora.add(ora.add(ora.mul_const(Ws[j], 1.0 - eta, s_g), ora.mul_const(Vs[j], eta, s_g)), Gw))
    st["t"] = t + 1
    st["alpha0"], st["alpha1"] = st["alpha1"], alpha_next(st["alpha1"])
    st["eta"], st["lr"] = eta, lr
    return Wn, Vn, st


def score_grid(ora, X_grid, Ws, m, g):
    """Encrypted scoring of validation rows with an encrypted model (the accuracy and AUROC of
    sections 5.1 and 5.2 taken from encrypted scores): X_grid[i][j] holds rows of [1 | X | 0]
    (no labels) in the m x g partition of section 2.2, Ws the model's column blocks.  For row
    block i: u = Rescale(Relin(sum_j X_ij (x) W_j)), then u += Rot(u, 2^k) for k < log2 g, which
    leaves each row's score x-hat . w in its column 0.  Returns the list of u."""
    lg = int(math.log2(g))
    out = []
    for row in X_grid:
        t3 = None
        for j, x in enumerate(row):
            prod = ora.tensor(x, Ws[j])
            t3 = prod if t3 is None else ora.add(t3, prod)
        u = ora.rescale(ora.relin(t3))
        for k in range(lg):
            u = ora.add(u, ora.rotate(u, 1 << k))
        out.append(u)
    return out
