"""ctypes binding of libheqg.so (C ABI in include/heqg.h).

Argument marshalling only: every step runs in the HIP library.  PyTorch
supplies device memory (int64 tensors hold the uint64 residues bit for bit)
and the current HIP stream.  Importing this module on a machine without the
built library raises; there is no fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# HEQG_LIB selects another build of the same library (side-by-side comparisons)
LIB_PATH = os.environ.get("HEQG_LIB") or os.path.join(HERE, "libheqg.so")

OK, ERR_ARG, ERR_LEVEL, ERR_SCALE, ERR_KEY, ERR_OVERFLOW, ERR_DEVICE, ERR_UNSUPPORTED, ERR_HOST = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
_NAMES = {-1: "ARG", -2: "LEVEL", -3: "SCALE", -4: "KEY", -5: "OVERFLOW", -6: "DEVICE", -7: "UNSUPPORTED",
          -8: "HOST"}


class HeqgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("HEQG_ERR_%s: %s" % (_NAMES.get(code, code), msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("log2N", ctypes.c_int), ("n_q", ctypes.c_int), ("q_bits", ctypes.POINTER(ctypes.c_int)),
                ("n_p", ctypes.c_int), ("p_bits", ctypes.c_int), ("dnum", ctypes.c_int), ("log2_scale", ctypes.c_int)]


class CtS(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("n_poly", ctypes.c_int), ("level", ctypes.c_int), ("scale", ctypes.c_double)]


class BatchS(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("count", ctypes.c_int64), ("stride", ctypes.c_int64),
                ("n_poly", ctypes.c_int), ("level", ctypes.c_int), ("scale", ctypes.c_double)]


class SigmoidS(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int), ("masks", ctypes.c_void_p), ("mask_level", ctypes.c_int),
                ("mask_scales", ctypes.POINTER(ctypes.c_double))]


class NagStateS(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int), ("alpha0", ctypes.c_double), ("alpha1", ctypes.c_double),
                ("lr_max", ctypes.c_double), ("lr_min", ctypes.c_double), ("T", ctypes.c_double),
                ("gamma", ctypes.c_double), ("m_rows", ctypes.c_int), ("g_cols", ctypes.c_int),
                ("refresh_seed", ctypes.c_uint64), ("eta", ctypes.c_double), ("lr", ctypes.c_double),
                ("refreshed_gr", ctypes.c_int), ("col_blocks", ctypes.c_int), ("first_order", ctypes.c_int),
                ("fo_gamma", ctypes.c_double)]


EXPORTS = None  # filled on load: every heqg_* function name the header declares
_lib = None


def lib():
    global _lib, EXPORTS
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("%s is not built (run __graft_entry__.build() or python -m "
                           "paper_2406_13221_amd.build); there is no non-HIP fallback" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, sz, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "heqg_last_error": (ctypes.c_char_p, []),
        "heqg_ctx_tables_bytes": (sz, [P(Params)]),
        "heqg_ctx_create": (i32, [P(Params), vp, sz, P(vp)]),
        "heqg_ctx_destroy": (None, [vp]),
        "heqg_ctx_primes": (i32, [vp, vp]),
        "heqg_ctx_info": (i32, [vp, vp, vp, vp, vp, vp]),
        "heqg_keys_bytes": (sz, [vp, i32]),
        "heqg_keygen_ws_bytes": (sz, [vp]),
        "heqg_keygen": (i32, [vp, u64, vp, i32, vp, sz, vp, sz, P(vp), vp]),
        "heqg_keygen_ex": (i32, [vp, u64, i32, i32, vp, i32, vp, sz, vp, sz, P(vp), vp]),
        "heqg_boot_steps": (i32, [vp, i32, vp]),
        "heqg_boot_shape": (i32, [vp, i32, i32, vp, vp, vp, vp]),
        "heqg_boot_encode": (i32, [vp, i32, i32, vp, i32]),
        "heqg_boot_bytes": (sz, [vp, i32, i32]),
        "heqg_boot_setup": (i32, [vp, vp, i32, i32, i32, vp, sz, P(vp), vp]),
        "heqg_boot_destroy": (None, [vp]),
        "heqg_boot_ws_bytes": (sz, [vp, i32, i64]),
        "heqg_mod_raise": (i32, [vp, P(BatchS), P(BatchS), vp, sz, vp]),
        "heqg_coeff_to_slot": (i32, [vp, vp, vp, P(BatchS), P(BatchS), vp, sz, vp]),
        "heqg_eval_mod": (i32, [vp, vp, vp, P(BatchS), dbl, P(BatchS), vp, sz, vp]),
        "heqg_slot_to_coeff": (i32, [vp, vp, vp, P(BatchS), P(BatchS), vp, sz, vp]),
        "heqg_bootstrap": (i32, [vp, vp, vp, P(BatchS), P(BatchS), vp, sz, vp]),
        "heqg_keys_destroy": (None, [vp]),
        "heqg_keys_galois": (i32, [vp, vp]),
        "heqg_keys_export": (i32, [vp, i32, i32, vp, vp]),
        "heqg_encode": (i32, [vp, vp, sz, dbl, vp]),
        "heqg_encode_batch": (i32, [vp, vp, sz, i64, dbl, vp, i32]),
        "heqg_decode": (i32, [vp, vp, dbl, vp, sz]),
        "heqg_lift": (i32, [vp, vp, i32, vp]),
        "heqg_enc_ws_bytes": (sz, [vp, i64]),
        "heqg_encrypt": (i32, [vp, vp, vp, u64, u64, P(BatchS), vp, sz, vp]),
        "heqg_decrypt": (i32, [vp, vp, P(BatchS), vp, vp, sz, vp]),
        "heqg_refresh": (i32, [vp, vp, P(BatchS), i32, u64, u64, P(BatchS), vp, sz, vp]),
        "heqg_pt_load": (i32, [vp, vp, i64, i32, vp, vp]),
        "heqg_ks_ws_bytes": (sz, [vp, i64]),
        "heqg_add": (i32, [vp, P(BatchS), P(BatchS), P(BatchS), vp]),
        "heqg_sub": (i32, [vp, P(BatchS), P(BatchS), P(BatchS), vp]),
        "heqg_tensor": (i32, [vp, P(BatchS), P(BatchS), P(BatchS), vp]),
        "heqg_relin": (i32, [vp, vp, P(BatchS), P(BatchS), vp, sz, vp]),
        "heqg_hmult": (i32, [vp, vp, P(BatchS), P(BatchS), P(BatchS), vp, sz, vp]),
        "heqg_rotate": (i32, [vp, vp, P(BatchS), i32, P(BatchS), vp, sz, vp]),
        "heqg_rotate_noalloc": (i32, [vp, vp, P(BatchS), i32, P(BatchS), vp]),
        "heqg_rescale": (i32, [vp, P(BatchS), P(BatchS), vp, sz, vp]),
        "heqg_drop": (i32, [vp, P(BatchS), i32, P(BatchS), vp]),
        "heqg_mul_pt": (i32, [vp, P(BatchS), vp, dbl, P(BatchS), vp]),
        "heqg_add_pt": (i32, [vp, P(BatchS), vp, dbl, P(BatchS), vp]),
        "heqg_mul_const": (i32, [vp, P(BatchS), dbl, dbl, P(BatchS), vp, sz, vp]),
        "heqg_ntt": (i32, [vp, vp, i64, i32, i32, i32, vp]),
        "heqg_sigfit_ws_bytes": (sz, [i64, i32]),
        "heqg_sigfit_grad": (i32, [vp, i64, vp, i32, vp, vp, vp, sz, vp]),
        "heqg_sigfit_train": (i32, [vp, i64, i32, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, vp, vp, sz, vp]),
        "heqg_tune_set": (i32, [vp, i32, i32]),
        "heqg_tune_get": (i32, [vp, i32]),
        "heqg_tune_ws_bytes": (sz, [vp, i32]),
        "heqg_tune_ntt": (i32, [vp, i32, vp, sz, vp, P(i32), P(dbl)]),
        "heqg_prof_start": (i32, [i32]),
        "heqg_prof_stop": (i32, [i32, P(dbl), P(i64), P(dbl), P(dbl), P(dbl)]),
        "heqg_nag_ws_bytes": (sz, [vp, i32, i32]),
        "heqg_nag_qg_step": (i32, [vp, vp, P(BatchS), P(CtS), P(CtS), P(CtS), P(SigmoidS), P(NagStateS), i32, vp,
                                   sz, vp]),
        "heqg_nag_qg_graph": (i32, [vp, vp, P(BatchS), P(CtS), P(CtS), P(CtS), P(SigmoidS), P(NagStateS), i32, vp,
                                    sz, vp]),
        "heqg_graph_clear": (i32, [vp]),
        "heqg_score": (i32, [vp, vp, P(BatchS), P(CtS), i32, i32, P(BatchS), i32, vp, sz, vp]),
        "heqg_graph_count": (i32, [vp]),
        "heqg_add_const": (i32, [vp, P(BatchS), dbl, P(BatchS), vp]),
        "heqg_export_ws_bytes": (sz, [vp, P(BatchS)]),
        "heqg_export": (i32, [vp, P(BatchS), vp, vp, sz, vp]),
        "heqg_import": (i32, [vp, vp, P(BatchS), vp]),
        "heqg_bbar": (i32, [vp, i64, i32, i32, dbl, vp, i32]),
        "heqg_plain_qgnag": (i32, [vp, vp, i64, i32, i32, i64, vp, i32, dbl, dbl, dbl, dbl, dbl, vp, vp, i32]),
        "heqg_sigmoid_plan": (i32, [vp, i32, dbl, dbl, dbl, i32, vp]),
        "heqg_sigmoid_masks": (i32, [vp, vp, i32, i32, i32, i32, dbl, dbl, dbl, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    EXPORTS = sorted(sig)
    _lib = L
    return L


def _check(rc):
    if rc < 0:
        raise HeqgError(rc, lib().heqg_last_error().decode())
    return rc


def prof_start(every):
    _check(lib().heqg_prof_start(int(every)))


def prof_stop(kernel=0):
    """(mean microseconds, sampled launches, then three per-launch means) of kernel class 0 (plain
    forward NTT row pass: rows written, -, -), 1 (fused base-conversion column pass: rows written,
    source rows read, algorithmic FP64 instructions) or 2 (ModUp row pass fused with the key inner
    product: ciphertext rows read and written, switching-key rows read, -)."""
    a, n, r, sr, op = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().heqg_prof_stop(int(kernel), ctypes.byref(a), ctypes.byref(n), ctypes.byref(r), ctypes.byref(sr),
                                ctypes.byref(op)))
    return a.value, n.value, r.value, sr.value, op.value


def bbar(X, g, eps=1e-8, threads=0):
    """Diagonal of B-bar (heqg_bbar): 1 / (eps + sum_l |H_jl|), H = 1/4 [1|X]^T [1|X]; 0 on padding."""
    Xc = np.ascontiguousarray(X, dtype=np.float64)
    n, f = Xc.shape
    out = np.zeros(g, dtype=np.float64)
    _check(lib().heqg_bbar(Xc.ctypes.data, n, f, g, float(eps), out.ctypes.data, int(threads)))
    return out


def plain_qgnag(X, y, iters, batch_rows=0, coeffs=None, lr=(2.0, 1.0, 81.0, 2.5), eps=1e-8, margins=True,
                threads=0):
    """The data owner's FP64 plaintext run (heqg_plain_qgnag): returns (W over 1 + f columns, margins of
    every iteration as one float32 array, or None).  coeffs: {odd k: c_k}, or None for the exact sigmoid."""
    Xc = np.ascontiguousarray(X, dtype=np.float64)
    yc = np.ascontiguousarray(y, dtype=np.int32)
    n, f = Xc.shape
    deg = max(coeffs) if coeffs else 0
    cs = np.array([coeffs.get(k, 0.0) for k in range(1, deg + 1, 2)], dtype=np.float64) if coeffs else None
    br = int(batch_rows or n)
    total = sum(min(br, n - (t % -(-n // br)) * br) for t in range(iters))
    m = np.zeros(total, dtype=np.float32) if margins else None
    w = np.zeros(f + 1, dtype=np.float64)
    _check(lib().heqg_plain_qgnag(Xc.ctypes.data, yc.ctypes.data, n, f, iters, int(batch_rows or 0),
                                  cs.ctypes.data if cs is not None else None, deg, float(lr[0]), float(lr[1]),
                                  float(lr[2]), float(lr[3]), float(eps), m.ctypes.data if m is not None else None,
                                  w.ctypes.data, int(threads)))
    return w, m


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ws(nbytes):
    torch = _torch()
    return torch.empty(max(int(nbytes), 8), dtype=torch.uint8, device="cuda")


class Cts:
    """A batch of ciphertexts: int64 tensor [count, n_poly, level+1, N] on the GPU."""

    def __init__(self, data, level, scale):
        self.data = data
        self.level = level
        self.scale = float(scale)

    @property
    def count(self):
        return self.data.shape[0]

    @property
    def n_poly(self):
        return self.data.shape[1]

    def batch(self):
        d = self.data
        return BatchS(d.data_ptr(), d.shape[0], d.stride(0), d.shape[1], self.level, self.scale)

    def one(self, i=0):
        d = self.data[i]
        return CtS(d.data_ptr(), d.shape[0], self.level, self.scale)

    def numpy(self):
        return self.data.cpu().numpy().view(np.uint64)


class Keys:
    def __init__(self, ctx, handle, buf, galois):
        self.ctx, self.handle, self.buf, self.galois = ctx, handle, buf, galois

    def export(self, which, idx=0):
        torch = _torch()
        c = self.ctx
        words = {0: c.nqp * c.N, 1: 2 * c.n_q * c.N}.get(which, c.dnum * 2 * c.nqp * c.N)
        out = torch.empty(words, dtype=torch.int64, device="cuda")
        _check(lib().heqg_keys_export(self.handle, which, idx, out.data_ptr(), _stream()))
        return out

    def __del__(self):
        try:
            lib().heqg_keys_destroy(self.handle)
        except Exception:
            pass


class Boot:
    def __init__(self, handle, buf, shape, r, levels):
        self.handle, self.buf, self.shape, self.r, self.levels = handle, buf, shape, r, levels

    def __del__(self):
        try:
            lib().heqg_boot_destroy(self.handle)
        except Exception:
            pass


class Context:
    def __init__(self, log2N, q_bits, n_p, p_bits, dnum, log2_scale):
        torch = _torch()
        L = lib()
        self._qb = (ctypes.c_int * len(q_bits))(*q_bits)
        self.params = Params(log2N, len(q_bits), self._qb, n_p, p_bits, dnum, log2_scale)
        nbytes = L.heqg_ctx_tables_bytes(ctypes.byref(self.params))
        if nbytes == 0:
            raise HeqgError(ERR_UNSUPPORTED, L.heqg_last_error().decode())
        self.tables = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        _check(L.heqg_ctx_create(ctypes.byref(self.params), self.tables.data_ptr(), nbytes, ctypes.byref(h)))
        self.h = h
        self.N = 1 << log2N
        self.n_q, self.n_p, self.dnum = len(q_bits), n_p, dnum
        self.nqp = self.n_q + n_p
        self.delta = float(2 ** log2_scale)
        pr = np.zeros(self.nqp, dtype=np.uint64)
        _check(L.heqg_ctx_primes(h, pr.ctypes.data))
        self.primes = pr

    @classmethod
    def from_config(cls, cfg):
        return cls(cfg["log2N"], cfg["q_bits"], cfg["n_p"], cfg["p_bits"], cfg["dnum"], cfg["log2_scale"])

    def __del__(self):
        try:
            lib().heqg_ctx_destroy(self.h)
        except Exception:
            pass

    @property
    def top_level(self):
        return self.n_q - 1

    # ---------------------------------------------------------------- keys
    def keygen(self, seed, rot_steps, hamming=0, conj=False):
        """heqg_keygen (hamming = 0, no conjugation key) or heqg_keygen_ex (sparse secret of weight
        hamming, conjugation key X -> X^(2N-1))."""
        L = lib()
        steps = (ctypes.c_int * max(1, len(rot_steps)))(*rot_steps)
        nb = L.heqg_keys_bytes(self.h, len(rot_steps) + (1 if conj else 0))
        buf = _ws(nb)
        ws = _ws(L.heqg_keygen_ws_bytes(self.h))
        h = ctypes.c_void_p()
        if hamming or conj:
            _check(L.heqg_keygen_ex(self.h, seed, int(hamming), 1 if conj else 0, steps, len(rot_steps),
                                    buf.data_ptr(), nb, ws.data_ptr(), ws.numel(), ctypes.byref(h), _stream()))
        else:
            _check(L.heqg_keygen(self.h, seed, steps, len(rot_steps), buf.data_ptr(), nb, ws.data_ptr(), ws.numel(),
                                 ctypes.byref(h), _stream()))
        n = _check(L.heqg_keys_galois(h, None))
        gal = np.zeros(max(n, 1), dtype=np.uint64)
        L.heqg_keys_galois(h, gal.ctypes.data)
        _torch().cuda.current_stream().synchronize()
        return Keys(self, h, buf, [int(x) for x in gal[:n]])

    # ---------------------------------------------------------------- encode
    def encode(self, values, scale):
        v = np.ascontiguousarray(values, dtype=np.float64)
        out = np.zeros(self.N, dtype=np.int64)
        _check(lib().heqg_encode(self.h, v.ctypes.data, v.size, float(scale), out.ctypes.data))
        return out

    def encode_batch(self, values, scale, threads=0):
        """values: [count, n] float64 -> int64 [count, N]."""
        v = np.ascontiguousarray(values, dtype=np.float64)
        if v.ndim == 1:
            v = v[None]
        out = np.zeros((v.shape[0], self.N), dtype=np.int64)
        _check(lib().heqg_encode_batch(self.h, v.ctypes.data, v.shape[1], v.shape[0], float(scale), out.ctypes.data,
                                       threads))
        return out

    def decode(self, coeffs, scale, n=None):
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        n = self.N // 2 if n is None else n
        out = np.zeros(n, dtype=np.float64)
        _check(lib().heqg_decode(self.h, c.ctypes.data, float(scale), out.ctypes.data, n))
        return out

    def lift(self, rows, level):
        r = np.ascontiguousarray(rows, dtype=np.uint64)
        out = np.zeros(self.N, dtype=np.float64)
        _check(lib().heqg_lift(self.h, r.ctypes.data, level, out.ctypes.data))
        return out

    # ---------------------------------------------------------------- alloc helpers
    def empty(self, count, n_poly, level, scale):
        torch = _torch()
        return Cts(torch.empty((count, n_poly, level + 1, self.N), dtype=torch.int64, device="cuda"), level, scale)

    # ---------------------------------------------------------------- encryption
    def encrypt(self, keys, coeffs, level, scale, seed, obj_first):
        """coeffs: int64 tensor [count, N] on the GPU (or numpy, copied over)."""
        torch = _torch()
        if isinstance(coeffs, np.ndarray):
            coeffs = torch.from_numpy(np.ascontiguousarray(coeffs, dtype=np.int64)).cuda()
        coeffs = coeffs.reshape(-1, self.N).contiguous()
        out = self.empty(coeffs.shape[0], 2, level, scale)
        L = lib()
        ws = _ws(L.heqg_enc_ws_bytes(self.h, out.count))
        b = out.batch()
        _check(L.heqg_encrypt(self.h, keys.handle, coeffs.data_ptr(), seed, obj_first, ctypes.byref(b),
                              ws.data_ptr(), ws.numel(), _stream()))
        return out

    def decrypt(self, keys, ct):
        torch = _torch()
        out = torch.empty((ct.count, ct.level + 1, self.N), dtype=torch.int64, device="cuda")
        b = ct.batch()
        _check(lib().heqg_decrypt(self.h, keys.handle, ctypes.byref(b), out.data_ptr(), None, 0, _stream()))
        return out

    def decrypt_values(self, keys, ct, n=None, index=0):
        rows = self.decrypt(keys, ct)[index].cpu().numpy().view(np.uint64)
        return self.decode(self.lift(rows, ct.level), ct.scale, n)

    def refresh(self, keys, ct, target_level, seed, obj_first, out=None):
        """Fresh encryption of ct's message at target_level; out (optional) may share ct's storage."""
        if out is None:
            out = self.empty(ct.count, 2, target_level, ct.scale)
        L = lib()
        nb = L.heqg_enc_ws_bytes(self.h, ct.count) + 8 * ct.count * (ct.level + 1) * self.N
        ws = _ws(nb)
        bi, bo = ct.batch(), out.batch()
        _check(L.heqg_refresh(self.h, keys.handle, ctypes.byref(bi), target_level, seed, obj_first, ctypes.byref(bo),
                              ws.data_ptr(), ws.numel(), _stream()))
        out.scale = bo.scale
        return out

    def pt_load(self, coeffs, level):
        torch = _torch()
        if isinstance(coeffs, np.ndarray):
            coeffs = torch.from_numpy(np.ascontiguousarray(coeffs, dtype=np.int64)).cuda()
        coeffs = coeffs.reshape(-1, self.N).contiguous()
        out = torch.empty((coeffs.shape[0], level + 1, self.N), dtype=torch.int64, device="cuda")
        _check(lib().heqg_pt_load(self.h, coeffs.data_ptr(), coeffs.shape[0], level, out.data_ptr(), _stream()))
        return out

    def ntt(self, rows, first_prime, period, inverse=False):
        """In place on an int64 tensor of shape [..., N]."""
        n = rows.numel() // self.N
        _check(lib().heqg_ntt(self.h, rows.data_ptr(), n, first_prime, period, 1 if inverse else 0, _stream()))
        return rows

    # ---------------------------------------------------------------- arithmetic
    # Output levels are shape bookkeeping (they size the buffers); output scales are written by
    # the library (heqg.h: the CKKS scale rules) and read back from the output batch.
    def _out(self, count, n_poly, level):
        return self.empty(count, n_poly, level, 0.0)

    @staticmethod
    def _done(out, bo):
        out.scale = bo.scale
        return out

    def _bin(self, fn, a, b, n_poly):
        lv = min(a.level, b.level)
        out = self._out(a.count, n_poly, lv)
        ba, bb, bo = a.batch(), b.batch(), out.batch()
        _check(fn(self.h, ctypes.byref(ba), ctypes.byref(bb), ctypes.byref(bo), _stream()))
        return self._done(out, bo)

    def add(self, a, b):
        return self._bin(lib().heqg_add, a, b, a.n_poly)

    def sub(self, a, b):
        return self._bin(lib().heqg_sub, a, b, a.n_poly)

    def tensor(self, a, b):
        return self._bin(lib().heqg_tensor, a, b, 3)

    def relin(self, keys, a):
        out = self._out(a.count, 2, a.level)
        L = lib()
        ws = _ws(L.heqg_ks_ws_bytes(self.h, a.count))
        ba, bo = a.batch(), out.batch()
        _check(L.heqg_relin(self.h, keys.handle, ctypes.byref(ba), ctypes.byref(bo), ws.data_ptr(), ws.numel(),
                            _stream()))
        return self._done(out, bo)

    def hmult(self, keys, a, b):
        lv = min(a.level, b.level)
        out = self._out(a.count, 2, lv)
        L = lib()
        ws = _ws(L.heqg_ks_ws_bytes(self.h, a.count) + 8 * a.count * 3 * (lv + 1) * self.N)
        ba, bb, bo = a.batch(), b.batch(), out.batch()
        _check(L.heqg_hmult(self.h, keys.handle, ctypes.byref(ba), ctypes.byref(bb), ctypes.byref(bo), ws.data_ptr(),
                            ws.numel(), _stream()))
        return self._done(out, bo)

    def rotate(self, keys, a, step):
        out = self._out(a.count, 2, a.level)
        L = lib()
        ws = _ws(L.heqg_ks_ws_bytes(self.h, a.count) + 8 * a.count * 2 * (a.level + 1) * self.N)
        ba, bo = a.batch(), out.batch()
        _check(L.heqg_rotate(self.h, keys.handle, ctypes.byref(ba), step, ctypes.byref(bo), ws.data_ptr(), ws.numel(),
                             _stream()))
        return self._done(out, bo)

    def rotate_noalloc(self, keys, a, step, out=None):
        """heqg_rotate_noalloc: the workspace is the library's own device array."""
        if out is None:
            out = self._out(a.count, 2, a.level)
        ba, bo = a.batch(), out.batch()
        _check(lib().heqg_rotate_noalloc(self.h, keys.handle, ctypes.byref(ba), step, ctypes.byref(bo), _stream()))
        return self._done(out, bo)

    def rescale(self, a):
        out = self._out(a.count, a.n_poly, a.level - 1)
        ws = _ws(8 * a.count * a.n_poly * (a.level + 1) * self.N)
        ba, bo = a.batch(), out.batch()
        _check(lib().heqg_rescale(self.h, ctypes.byref(ba), ctypes.byref(bo), ws.data_ptr(), ws.numel(), _stream()))
        return self._done(out, bo)

    def drop(self, a, level):
        out = self._out(a.count, a.n_poly, level)
        ba, bo = a.batch(), out.batch()
        _check(lib().heqg_drop(self.h, ctypes.byref(ba), level, ctypes.byref(bo), _stream()))
        return self._done(out, bo)

    def mul_pt(self, a, pt, pt_scale):
        out = self._out(a.count, a.n_poly, a.level)
        ba, bo = a.batch(), out.batch()
        _check(lib().heqg_mul_pt(self.h, ctypes.byref(ba), pt.data_ptr(), float(pt_scale), ctypes.byref(bo), _stream()))
        return self._done(out, bo)

    def add_pt(self, a, pt, pt_scale):
        out = self._out(a.count, 2, a.level)
        ba, bo = a.batch(), out.batch()
        _check(lib().heqg_add_pt(self.h, ctypes.byref(ba), pt.data_ptr(), float(pt_scale), ctypes.byref(bo), _stream()))
        return self._done(out, bo)

    def add_const(self, a, c, out=None):
        """cAdd: c added to every slot; out may be a (in place)."""
        if out is None:
            out = self._out(a.count, a.n_poly, a.level)
        ba, bo = a.batch(), out.batch()
        _check(lib().heqg_add_const(self.h, ctypes.byref(ba), float(c), ctypes.byref(bo), _stream()))
        return self._done(out, bo)

    def mul_const(self, a, c, target):
        out = self._out(a.count, a.n_poly, a.level - 1)
        ws = _ws(16 * a.count * a.n_poly * (a.level + 1) * self.N)
        ba, bo = a.batch(), out.batch()
        _check(lib().heqg_mul_const(self.h, ctypes.byref(ba), float(c), float(target), ctypes.byref(bo), ws.data_ptr(),
                                    ws.numel(), _stream()))
        return self._done(out, bo)

    # ---------------------------------------------------------------- parity I/O
    def export(self, a):
        """Coefficient-form residues, numpy uint64 [count][n_poly][level+1][N]."""
        L = lib()
        ba = a.batch()
        ws = _ws(L.heqg_export_ws_bytes(self.h, ctypes.byref(ba)))
        out = np.zeros((a.count, a.n_poly, a.level + 1, self.N), dtype=np.uint64)
        _check(L.heqg_export(self.h, ctypes.byref(ba), out.ctypes.data, ws.data_ptr(), ws.numel(), _stream()))
        return out

    def import_(self, coeffs, level, scale):
        """Coefficient-form residues [count][n_poly][level+1][N] -> NTT-form Cts on the GPU."""
        c = np.ascontiguousarray(coeffs, dtype=np.uint64)
        if c.ndim == 3:
            c = c[None]
        out = self.empty(c.shape[0], c.shape[1], level, scale)
        bo = out.batch()
        _check(lib().heqg_import(self.h, c.ctypes.data, ctypes.byref(bo), _stream()))
        return out

    # ---------------------------------------------------------------- client-side inputs
    def sigmoid_masks(self, coeffs, m, g, level, s_z, s_w, s_c):
        """{odd k: c_k} -> (int64 [n_terms+1][N] coefficient-form masks, their scales) (heqg_sigmoid_masks)."""
        deg = max(coeffs)
        cs = np.array([coeffs.get(k, 0.0) for k in range(1, deg + 1, 2)], dtype=np.float64)
        nt = len(cs)
        out = np.zeros((nt + 1, self.N), dtype=np.int64)
        sc = np.zeros(nt + 1, dtype=np.float64)
        _check(lib().heqg_sigmoid_masks(self.h, cs.ctypes.data, deg, m, g, level, float(s_z), float(s_w), float(s_c),
                                        out.ctypes.data, sc.ctypes.data))
        return out, [float(x) for x in sc]

    def sigmoid_plan(self, level, s_z, s_w, s_c, degree):
        sc = np.zeros((degree + 1) // 2 + 1, dtype=np.float64)
        _check(lib().heqg_sigmoid_plan(self.h, level, float(s_z), float(s_w), float(s_c), degree, sc.ctypes.data))
        return [float(x) for x in sc]

    # ---------------------------------------------------------------- training step
    def nag_ws_bytes(self, batch, degree=3):
        return lib().heqg_nag_ws_bytes(self.h, batch, degree)

    def nag_qg_step(self, keys, Z, Bbar, W, V, masks, mask_level, mask_scales, degree, state, batch, ws=None,
                    stream=None, graph=False):
        """One encrypted QG-NAG iteration; W and V are updated in place.

        Z: row block i, column block j at i * C + j with C = state.col_blocks (0 means 1); Bbar, W
        and V: Cts of C contiguous ciphertexts.  masks: int64 tensor [n_terms + 1, mask_level + 1, N]
        (NTT form); state: NagStateS (updated).  graph: submit the iteration as a replayed HIP graph
        (heqg_nag_qg_graph); needs a non-null stream."""
        L = lib()
        if ws is None:
            ws = _ws(self.nag_ws_bytes(batch, degree))
        sc = (ctypes.c_double * len(mask_scales))(*mask_scales)
        sig = SigmoidS(degree, masks.data_ptr(), mask_level, sc)
        zb = Z.batch()
        bb = Bbar.one() if Bbar is not None else None
        wb, vb = W.one(), V.one()
        s = _stream() if stream is None else ctypes.c_void_p(stream)
        fn = L.heqg_nag_qg_graph if graph else L.heqg_nag_qg_step
        _check(fn(self.h, keys.handle, ctypes.byref(zb), ctypes.byref(bb) if bb is not None else None,
                  ctypes.byref(wb), ctypes.byref(vb),
                  ctypes.byref(sig), ctypes.byref(state), batch, ws.data_ptr(), ws.numel(), s))
        for ct, cs in ((W, wb), (V, vb)):
            n = ct.count * 2 * (cs.level + 1) * self.N
            ct.data = ct.data.reshape(-1)[:n].view(ct.count, 2, cs.level + 1, self.N)
            ct.level, ct.scale = cs.level, cs.scale
        return state

    def score(self, keys, X, W, g, col_blocks=1, batch=16, ws=None):
        """heqg_score: per row block of X (rows of [1 | X | 0] in the m x g partition), a ciphertext whose
        column 0 holds every row's score x-hat . w under the encrypted model W (col_blocks ciphertexts)."""
        n = X.count // max(1, col_blocks)
        lv = min(X.level, W.level) - 1
        out = self.empty(n, 2, lv, 0.0)
        if ws is None:
            ws = _ws(self.nag_ws_bytes(batch))
        xb, wb, ob = X.batch(), W.one(), out.batch()
        _check(lib().heqg_score(self.h, keys.handle, ctypes.byref(xb), ctypes.byref(wb), int(col_blocks), int(g),
                                ctypes.byref(ob), int(batch), ws.data_ptr(), ws.numel(), _stream()))
        out.scale = ob.scale
        return out

    def tune_set(self, which, value):
        """Tuning choice of this context: 0/1 row-pass variant fwd/inv, 2 NTT pass split, 3 heqg_ntt slice
        in MiB (False if refused)."""
        return lib().heqg_tune_set(self.h, int(which), int(value)) == 0

    def tune_get(self, which):
        return lib().heqg_tune_get(self.h, int(which))

    def graph_count(self):
        return _check(lib().heqg_graph_count(self.h))

    def tune_ntt(self, rows=2048):
        """Time every NTT pass split and row-pass variant on `rows` limbs (default 2,048: 1 GiB at
        N = 2^16, past the caches); keep the split with the fastest forward + inverse time and the
        fastest variant of each direction."""
        L = lib()
        ws = _ws(L.heqg_tune_ws_bytes(self.h, rows))
        ch = (ctypes.c_int * 4)()
        us = (ctypes.c_double * 2)()
        _check(L.heqg_tune_ntt(self.h, rows, ws.data_ptr(), ws.numel(), _stream(), ch, us))
        return {"split_fwd": ch[0], "variant_fwd": ch[1], "split_inv": ch[2], "variant_inv": ch[3],
                "fwd_us": round(us[0], 2), "inv_us": round(us[1], 2)}

    def graph_clear(self):
        _check(lib().heqg_graph_clear(self.h))

    # ---------------------------------------------------------------- bootstrapping
    def boot_steps(self, levels=0):
        """The rotation steps the slot transforms of heqg_bootstrap use (levels per transform, 0: dense)."""
        L = lib()
        n = _check(L.heqg_boot_steps(self.h, int(levels), None))
        out = (ctypes.c_int * max(1, n))()
        L.heqg_boot_steps(self.h, int(levels), out)
        return list(out[:n])

    def boot_shape(self, r, levels=0):
        """(CoeffToSlot input level, SlotToCoeff input level, output level, number of plaintexts)."""
        v = [ctypes.c_int() for _ in range(3)]
        npts = ctypes.c_int64()
        _check(lib().heqg_boot_shape(self.h, int(r), int(levels), *[ctypes.byref(x) for x in v], ctypes.byref(npts)))
        return tuple(x.value for x in v) + (npts.value,)

    def boot_encode(self, r, levels=0, threads=0):
        """heqg_boot_encode: every plaintext of the slot transforms, numpy int64 [n_pts][N]."""
        n_pts = self.boot_shape(r, levels)[3]
        out = np.zeros((n_pts, self.N), dtype=np.int64)
        _check(lib().heqg_boot_encode(self.h, int(r), int(levels), out.ctypes.data, int(threads)))
        return out

    def boot_setup(self, coeffs, r, taylor, levels=0):
        """coeffs: int64 [n_pts][N] (numpy or a device tensor, heqg_boot_encode's layout).  Returns a Boot
        holding the NTT-form plaintexts."""
        torch = _torch()
        L = lib()
        nb = L.heqg_boot_bytes(self.h, int(r), int(levels))
        if nb == 0:
            raise HeqgError(-1, L.heqg_last_error().decode())
        if isinstance(coeffs, np.ndarray):
            coeffs = torch.from_numpy(np.ascontiguousarray(coeffs, dtype=np.int64)).cuda()
        buf = _ws(nb)
        h = ctypes.c_void_p()
        _check(L.heqg_boot_setup(self.h, coeffs.data_ptr(), int(r), int(levels), int(taylor), buf.data_ptr(), nb,
                                 ctypes.byref(h), _stream()))
        _torch().cuda.current_stream().synchronize()
        return Boot(h, buf, self.boot_shape(r, levels), int(r), int(levels))

    def _boot_call(self, fn, pre, ct, out_level, ws, levels=0):
        """fn(ctx, *pre, in, out, ws, ws_bytes, stream) for the bootstrapping steps."""
        out = self._out(ct.count, 2, out_level)
        need = lib().heqg_boot_ws_bytes(self.h, int(levels), ct.count)
        if ws is None or ws.numel() < need:
            ws = _ws(need)
        bi, bo = ct.batch(), out.batch()
        _check(fn(self.h, *pre, ctypes.byref(bi), ctypes.byref(bo), ws.data_ptr(), ws.numel(), _stream()))
        return self._done(out, bo)

    def mod_raise(self, ct, ws=None):
        """heqg_mod_raise: level 0 -> the top level (decrypts to m + q0 I)."""
        return self._boot_call(lib().heqg_mod_raise, (), ct, self.top_level, ws)

    def coeff_to_slot(self, keys, boot, ct, ws=None):
        return self._boot_call(lib().heqg_coeff_to_slot, (keys.handle, boot.handle), ct,
                               ct.level - max(boot.levels, 1), ws, boot.levels)

    def slot_to_coeff(self, keys, boot, ct, ws=None):
        return self._boot_call(lib().heqg_slot_to_coeff, (keys.handle, boot.handle), ct, boot.shape[2], ws,
                               boot.levels)

    def eval_mod(self, keys, boot, ct, half=1.0, ws=None, levels_used=None):
        """heqg_eval_mod; levels_used: the levels it consumes (7 + r, or 8 + r with the affine map over
        two primes; the oracle's EvalMod.levels gives it)."""
        out = self._out(ct.count, 2, ct.level - (7 + boot.r if levels_used is None else levels_used))
        need = lib().heqg_boot_ws_bytes(self.h, boot.levels, ct.count)
        if ws is None or ws.numel() < need:
            ws = _ws(need)
        bi, bo = ct.batch(), out.batch()
        _check(lib().heqg_eval_mod(self.h, keys.handle, boot.handle, ctypes.byref(bi), float(half), ctypes.byref(bo),
                                   ws.data_ptr(), ws.numel(), _stream()))
        return self._done(out, bo)

    def bootstrap(self, keys, boot, ct, ws=None):
        """heqg_bootstrap: level-0 ciphertexts -> the same messages at level stc_level - 1."""
        return self._boot_call(lib().heqg_bootstrap, (keys.handle, boot.handle), ct, boot.shape[2], ws, boot.levels)

