"""Build (gcc) and load the C oracle.  Test infrastructure only."""
import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ckks_oracle.c")
LIB = os.path.join(HERE, "libckks_oracle.so")


def build(force=False):
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        u64, i64, i32, vp = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        P = ctypes.c_void_p
        sig = {
            "oracle_mulmod": (u64, [u64, u64, u64]),
            "oracle_powmod": (u64, [u64, u64, u64]),
            "oracle_is_prime": (i32, [u64]),
            "oracle_gen_primes": (i32, [i32, i32, P, i32, i32, P]),
            "oracle_find_psi": (u64, [u64, i32]),
            "oracle_ctx_new": (vp, [i32, i32, i32, i32, P]),
            "oracle_ctx_free": (None, [vp]),
            "oracle_ctx_psi": (u64, [vp, i32]),
            "oracle_ntt": (None, [vp, P, i32, P, i32]),
            "oracle_chacha20_block": (None, [P, ctypes.c_uint32, P, P]),
            "oracle_stream_words": (None, [u64, u64, u64, ctypes.c_uint32, u64, ctypes.c_size_t, P]),
            "oracle_sample_ternary": (None, [u64, u64, u64, i32, P]),
            "oracle_sample_cbd": (None, [u64, u64, u64, i32, P]),
            "oracle_sample_uniform": (None, [u64, u64, u64, ctypes.c_uint32, u64, i32, P]),
            "oracle_secret": (None, [vp, u64, P]),
            "oracle_secret_ntt": (None, [vp, P, P]),
            "oracle_pk": (None, [vp, u64, P, P]),
            "oracle_ksk": (None, [vp, u64, u64, P, P, P]),
            "oracle_automorph_int": (None, [i32, P, u64, P]),
            "oracle_automorph": (None, [vp, P, i32, u64, P]),
            "oracle_encrypt": (None, [vp, P, P, i32, u64, u64, P]),
            "oracle_decrypt": (None, [vp, P, P, i32, i32, P]),
            "oracle_add": (None, [vp, P, P, i32, i32, i32, P]),
            "oracle_tensor": (None, [vp, P, P, i32, P]),
            "oracle_mul_pt": (None, [vp, P, P, i32, i32, P]),
            "oracle_mul_int": (None, [vp, P, i64, i32, i32, P]),
            "oracle_add_pt": (None, [vp, P, P, i32, P]),
            "oracle_pt_from_int": (None, [vp, P, i32, P]),
            "oracle_rescale": (None, [vp, P, i32, i32, P]),
            "oracle_base_conv": (None, [vp, P, P, i32, P, i32, P]),
            "oracle_keyswitch": (None, [vp, P, i32, P, P]),
            "oracle_relin": (None, [vp, P, i32, P, P]),
            "oracle_rotate": (None, [vp, P, i32, u64, P, P]),
            "oracle_refresh": (None, [vp, P, P, P, i32, i32, u64, u64, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
