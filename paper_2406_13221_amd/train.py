"""Encrypted QG-NAG logistic-regression training on the HIP library.

Follows the pipeline of the paper (section 4.3): the client builds
Z = y+- * [1 | X] and the diagonal B-bar from -1/4 X^T X, packs Z row by row
into m x g blocks (section 2.2), encrypts Z, B-bar and W = V = 0; the cloud
runs steps 4-6 (heqg_nag_qg_step) and refreshes W and V (step 7, here the
key-holder refresh); the client decrypts W (step 8).

Everything arithmetic on ciphertexts runs in libheqg.so; this module only
prepares plaintext vectors and calls the C ABI through the binding.
"""
import math

import numpy as np

from . import heqg

G8 = {1: 0.15, 3: -0.0015}   # least-squares cubic on [-8, 8] (section 4.1)


def rot_steps(m, g):
    """Row sums (+2^k), replication (-2^k) and column sums (+g 2^k)."""
    lg, lm = int(math.log2(g)), int(math.log2(m))
    return [1 << k for k in range(lg)] + [-(1 << k) for k in range(lg)] + [g << k for k in range(lm)]


def z_matrix(X, y, g):
    """y+- * [1 | X | 0] with labels in {0, 1} mapped to -1/+1."""
    n, f = X.shape
    Z = np.zeros((n, g))
    Z[:, 0] = 1.0
    Z[:, 1:f + 1] = X
    return Z * (2.0 * np.asarray(y, dtype=np.float64) - 1.0)[:, None]


def pack_rows(Z, m, g):
    """Blocks of m rows, each flattened row-major into m*g slots (zero rows pad the last block)."""
    n = Z.shape[0]
    nb = -(-n // m)
    out = np.zeros((nb, m * g))
    flat = Z.reshape(-1)
    for b in range(nb):
        seg = flat[b * m * g: (b + 1) * m * g]
        out[b, :seg.size] = seg
    return out


def pack_grid(Z, m, g):
    """The m x g partition of section 2.2: Z (n x C*g) as row block i, column block j at i*C + j,
    each sub-matrix flattened row-major into m*g slots (zero rows pad the last row block)."""
    n, G = Z.shape
    C = G // g
    if C == 1:
        return pack_rows(Z, m, g)
    nb = -(-n // m)
    out = np.zeros((nb * C, m * g))
    for i in range(nb):
        rows = Z[i * m:(i + 1) * m]
        for j in range(C):
            blk = rows[:, j * g:(j + 1) * g]
            out[i * C + j, :blk.size] = blk.reshape(-1)
    return out


def col_blocks(f, g):
    """Column blocks of g columns that hold the bias column and f features."""
    return -(-(f + 1) // g)


def bbar_diag(X, g, eps=1e-8):
    """B-bar of rows X (sections 3.1, 4.3), computed by the library (heqg_bbar)."""
    return heqg.bbar(X, g, eps)


def tile_row(vec, m, g):
    row = np.zeros(g)
    row[:len(vec)] = vec
    return np.tile(row, m)


# Scale of the sigmoid output p (the F/2 mask's encoding scale; every term of the polynomial lands on it).
# The gradient Z^T p then carries Delta * 2^30 / q ~ 2^30, so the B-bar product's constant
# round(lr * s * q / scale(B-bar)) gets about 2^20 instead of 2^10: with 2^40 here its rounding alone
# put a relative error of up to 5e-4 on the step at 422,108 rows, where B-bar is ~1e-6 (the paper
# scales ciphertexts by 2^30 too).  Lower scales cost precision in the masks' encodings instead.
SIGMOID_SCALE = 2.0 ** 30


def new_state(m, g, refresh_seed=0, lr_max=2.0, lr_min=1.0, T=81.0, gamma=2.5, col_blocks=1):
    a0 = 0.01
    a1 = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * a0 * a0))
    return heqg.NagStateS(0, a0, a1, lr_max, lr_min, T, gamma, m, g, refresh_seed, 0.0, 0.0, 0, col_blocks)


class EncryptedQGNAG:
    """Client + cloud roles of the pipeline on one GPU."""

    def __init__(self, cfg, X, y, coeffs=None, batch=16, rows=None, threads=0, mini_batch=False, graph=False,
                 first_order=False, level=None, secret_weight=0, extra_steps=()):
        """graph: submit each iteration as a replayed HIP graph (on a side stream of this object).
        first_order: train with the first-order NAG the paper compares against (step cfg["fo_lr"] / n on
        the gradient, no B-bar) instead of the quadratic gradient.
        level: the level W and V are encrypted at and refreshed to (default: the top of the chain).  Z and
        B-bar are always encrypted at the top, and every product with them runs at the level of W, V:
        a bootstrapped run works at the level bootstrapping returns (heqg_boot_shape).
        secret_weight, extra_steps: a sparse ternary secret of that Hamming weight with the conjugation
        key and these further rotations (heqg_boot_steps), for a run that bootstraps (bootstrap())."""
        import torch
        self.cfg = cfg
        self.m, self.g = cfg["m"], cfg["g"]
        self.coeffs = dict(coeffs or G8)
        self.degree = max(self.coeffs)
        self.batch = batch
        self.ctx = ctx = heqg.Context.from_config(cfg)
        steps = sorted(set(rot_steps(self.m, self.g)) | set(extra_steps))
        self.keys = ctx.keygen(cfg["key_seed"], steps, hamming=secret_weight, conj=secret_weight > 0)
        L = ctx.top_level
        Xs, ys = (X, y) if rows is None else (X[rows[0]:rows[1]], y[rows[0]:rows[1]])
        self._X, self._n_rows = Xs, Xs.shape[0]
        # column blocks of the partition (section 2.2); W, V and each B-bar are one ciphertext per block
        self.nc = nc = col_blocks(Xs.shape[1], self.g)
        self.width = nc * self.g
        # step 1-2: Z blocks, B-bar, W = V = 0 (client side)
        blocks = pack_grid(z_matrix(Xs, ys, self.width), self.m, self.g)
        nb = blocks.shape[0]
        self.Z = heqg.Cts(torch.empty((nb, 2, L + 1, ctx.N), dtype=torch.int64, device="cuda"), L, ctx.delta)
        chunk = 64
        ws = heqg._ws(heqg.lib().heqg_enc_ws_bytes(ctx.h, chunk))
        for b0 in range(0, nb, chunk):
            b1 = min(nb, b0 + chunk)
            coeffs_np = ctx.encode_batch(blocks[b0:b1], ctx.delta, threads)
            dev = torch.from_numpy(coeffs_np).cuda()
            out = heqg.Cts(self.Z.data[b0:b1], L, ctx.delta)
            ob = out.batch()
            heqg._check(heqg.lib().heqg_encrypt(ctx.h, self.keys.handle, dev.data_ptr(), cfg["enc_seed"], b0,
                                                ctypes_byref(ob), ws.data_ptr(), ws.numel(), heqg._stream()))
        # full batch: one B-bar from all rows; mini-batch (Algorithm 1): one B-bar per batch of rows
        n = Xs.shape[0]
        br = cfg.get("batch_rows") if mini_batch else None
        if br and br % self.m:
            raise ValueError("batch_rows must be a multiple of m")
        spans = [(0, n)] if not br else [(s, min(s + br, n)) for s in range(0, n, br)]
        self.block_spans = [(s // self.m, -(-e // self.m)) for s, e in spans]
        self.span_rows = [e - s for s, e in spans]
        self.first_order = first_order
        self.Bbars = [self._bbar_cts(Xs[s:e], (1 << 40) + 16 + i * nc) for i, (s, e) in enumerate(spans)]
        self.Bbar = self.Bbars[0]
        # W and V keep their storage for the whole run (a replayed graph is bound to it), sized for
        # the top level; they are encrypted at the working level
        words = nc * 2 * (ctx.top_level + 1) * ctx.N
        self.Wflat = torch.empty(words, dtype=torch.int64, device="cuda")
        self.Vflat = torch.empty(words, dtype=torch.int64, device="cuda")
        self.graph = graph
        self.stream = torch.cuda.Stream() if graph else None
        self.state = new_state(self.m, self.g, refresh_seed=cfg["enc_seed"] + 7, col_blocks=nc,
                               T=cfg.get("lr_T", 81.0))
        self.reset(obj=(1 << 40) + 1, level=L if level is None else level)
        self.ws = heqg._ws(ctx.nag_ws_bytes(batch, self.degree))
        self.refresh_obj = 1 << 41

    def reset(self, obj=(1 << 40) + (1 << 30), level=None):
        """W = V = 0 again (fresh encryptions into the same storage, objects obj + j) and t = 0, at
        `level` (default: the current working level); the sigmoid masks are planned for it."""
        ctx, nc = self.ctx, self.nc
        L = self.L if level is None else int(level)
        if not 1 <= L <= ctx.top_level:
            raise ValueError("level must be in 1..%d" % ctx.top_level)
        self.L = L
        shape = (nc, 2, L + 1, ctx.N)
        self.Wbuf = self.Wflat[:nc * 2 * (L + 1) * ctx.N].view(shape)
        self.Vbuf = self.Vflat[:nc * 2 * (L + 1) * ctx.N].view(shape)
        zero = np.zeros((nc, ctx.N), dtype=np.int64)
        self.W = heqg.Cts(self.Wbuf, L, ctx.delta)
        self.V = heqg.Cts(self.Vbuf, L, ctx.delta)
        for ct, o in ((self.W, obj), (self.V, obj + nc)):
            fresh = ctx.encrypt(self.keys, zero, L, ctx.delta, self.cfg["enc_seed"], o)
            ct.data.copy_(fresh.data)
        self.set_sigmoid(self.coeffs)
        st = self.state
        self.state = new_state(self.m, self.g, refresh_seed=st.refresh_seed, lr_max=st.lr_max, lr_min=st.lr_min,
                               T=st.T, gamma=st.gamma, col_blocks=nc)

    def _bbar_cts(self, Xr, obj_first):
        """B-bar of the rows Xr (width C*g), one ciphertext per column block (objects obj_first + j)."""
        ctx, g = self.ctx, self.g
        B = bbar_diag(Xr, self.width)
        # largest entry at 2^(log2 scale + 10): the B-bar products' constant round(lr s q / sB) then
        # keeps about 2^20 (below 2^62 on chains of wider primes too)
        sB = 2.0 ** (self.cfg["log2_scale"] + 10) / B.max()
        pts = np.stack([ctx.encode(tile_row(B[j * g:(j + 1) * g], self.m, g), sB) for j in range(self.nc)])
        return ctx.encrypt(self.keys, pts, ctx.top_level, sB, self.cfg["enc_seed"], obj_first)

    def tune(self, candidates=(16, 24, 32, 48), blocks=96, rows=2048, reps=3):
        """Autotune: NTT pass split and row-pass variants (heqg_tune_ntt), then the number of
        blocks per lock-step chunk, timed (best of `reps`) on one iteration over the first
        `blocks` blocks, a multiple of every candidate."""
        import copy
        import torch
        ctx = self.ctx
        res = {"ntt": ctx.tune_ntt(rows)}
        nb = min(blocks, self.Z.count // self.nc)
        Z = heqg.Cts(self.Z.data[:nb * self.nc], self.Z.level, self.Z.scale)
        times = {}
        for B in candidates:
            B = max(min(B, nb), self.nc)
            ws = heqg._ws(ctx.nag_ws_bytes(B, self.degree))
            best = None
            for _ in range(reps):
                W = heqg.Cts(self.W.data.clone(), self.W.level, self.W.scale)
                V = heqg.Cts(self.V.data.clone(), self.V.level, self.V.scale)
                st = copy.copy(self.state)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                ctx.nag_qg_step(self.keys, Z, self.Bbars[0], W, V, self.masks, self.mask_level, self.mask_scales,
                                self.degree, st, B, ws)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                best = ms if best is None else min(best, ms)
            times[B] = round(best, 2)
            del ws
        self.batch = min(times, key=times.get)
        self.ws = heqg._ws(ctx.nag_ws_bytes(self.batch, self.degree))
        res["batch_ms"] = times
        res["batch"] = self.batch
        return res

    def with_batches(self, batch_rows, batch=8, graph=False):
        """A mini-batch run (Algorithm 1: one B-bar per batch of rows) over the same encrypted blocks and keys."""
        import copy
        import torch
        if batch_rows % self.m:
            raise ValueError("batch_rows must be a multiple of m")
        ctx, L = self.ctx, self.L
        mb = copy.copy(self)
        n = self._n_rows
        spans = [(s, min(s + batch_rows, n)) for s in range(0, n, batch_rows)]
        mb.block_spans = [(s // self.m, -(-e // self.m)) for s, e in spans]
        nc = self.nc
        mb.Bbars = [self._bbar_cts(self._X[s:e], (1 << 40) + (1 << 20) + i * nc) for i, (s, e) in enumerate(spans)]
        mb.Bbar = mb.Bbars[0]
        # its own W and V storage, W = V = 0 at the same working level
        mb.Wflat, mb.Vflat = torch.empty_like(self.Wflat), torch.empty_like(self.Vflat)
        mb.state = new_state(self.m, self.g, refresh_seed=self.cfg["enc_seed"] + 7, col_blocks=nc,
                             T=self.cfg.get("lr_T", 81.0))
        mb.reset(obj=(1 << 40) + 3 * nc, level=L)
        mb.span_rows = [e - s for s, e in spans]
        mb.batch = batch
        mb.ws = heqg._ws(ctx.nag_ws_bytes(batch, self.degree))
        mb.graph = graph
        mb.stream = torch.cuda.Stream() if graph else None
        mb.refresh_obj = 1 << 42
        return mb

    def set_sigmoid(self, coeffs):
        """Masks -c_k F for each odd power (ascending) and F/2 at the planned scales (heqg_sigmoid_masks),
        loaded in NTT form at level L-1."""
        ctx = self.ctx
        self.coeffs = dict(coeffs)
        self.degree = max(self.coeffs)
        lv = self.L
        vals, scales = ctx.sigmoid_masks(self.coeffs, self.m, self.g, lv, ctx.delta, ctx.delta, SIGMOID_SCALE)
        self.mask_level = lv - 1
        self.masks = ctx.pt_load(vals, self.mask_level)
        self.mask_scales = scales

    def step(self, refresh=True):
        """One iteration: all blocks (full batch) or the blocks of batch t mod n_batches with its B-bar."""
        if self.stream is None:
            return self._step(refresh)
        import torch
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        with torch.cuda.stream(self.stream):
            self._step(refresh)
        cur.wait_stream(self.stream)
        return self.state

    def _step(self, refresh):
        ctx = self.ctx
        k = self.state.t % len(self.block_spans)
        b0, b1 = self.block_spans[k]
        Z = heqg.Cts(self.Z.data[b0 * self.nc:b1 * self.nc], self.Z.level, self.Z.scale)
        if self.first_order:
            self.state.first_order = 1
            self.state.fo_gamma = self.cfg["fo_lr"] / self.span_rows[k]
        ctx.nag_qg_step(self.keys, Z, None if self.first_order else self.Bbars[k], self.W, self.V, self.masks,
                        self.mask_level, self.mask_scales, self.degree, self.state, self.batch, self.ws,
                        graph=self.graph)
        if refresh:
            self.refresh()
        return self.state

    def refresh(self):
        o, L, d = self.refresh_obj, self.L, self.ctx.delta
        nc = self.nc
        self.W = self.ctx.refresh(self.keys, self.W, L, self.cfg["enc_seed"] + 9, o, out=heqg.Cts(self.Wbuf, L, d))
        self.V = self.ctx.refresh(self.keys, self.V, L, self.cfg["enc_seed"] + 9, o + nc,
                                  out=heqg.Cts(self.Vbuf, L, d))
        self.refresh_obj += 2 * nc

    def bootstrap(self, boot, ws=None):
        """Step 7 without the key holder (section 4.3; Table 1: one bootstrapping per iteration): W and V
        dropped to level 0 and bootstrapped together (heqg_bootstrap, keys on the sparse secret); the
        result, at the level `boot` returns, which must be the working level, goes back into their
        storage."""
        import torch
        ctx, nc, L = self.ctx, self.nc, self.L
        if boot.shape[2] != L:
            raise ValueError("the bootstrap returns level %d, the run works at level %d" % (boot.shape[2], L))
        w0, v0 = ctx.drop(self.W, 0), ctx.drop(self.V, 0)
        both = heqg.Cts(torch.cat([w0.data, v0.data]), 0, w0.scale)
        out = ctx.bootstrap(self.keys, boot, both, ws=ws)
        self.Wbuf.copy_(out.data[:nc])
        self.Vbuf.copy_(out.data[nc:])
        self.W = heqg.Cts(self.Wbuf, L, out.scale)
        self.V = heqg.Cts(self.Vbuf, L, out.scale)

    def weights(self, f=None):
        """Row 0 of W: the model over the padded width (its first f entries when f is given)."""
        w = np.concatenate([self.ctx.decrypt_values(self.keys, self.W, self.g, index=j) for j in range(self.nc)])
        return w if f is None else w[:f]


def ctypes_byref(x):
    import ctypes
    return ctypes.byref(x)
