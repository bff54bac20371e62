"""Workload definitions (sizes and seeds only).

c1/c2/c3 are the plain method at three sizes; c4 is the batching form over the
c3 shapes; c5 is the learned-sigmoid form over the c3 shapes.  Every workload
uses RNS primes of the listed bit sizes, dnum-digit key switching, scale
2^log2_scale and the row-major m x g block layout of the paper (section 2.2).
"""
import copy

_BASE = {
    "c1": dict(
        name="c1-tiny", log2N=12, q_bits=[50, 40, 40, 40, 40], n_p=2, p_bits=60, dnum=3, log2_scale=40,
        m=256, g=8, n_train=128, n_features=7, n_valid=256, seed=1, iters=3, batch_rows=None,
        sigmoid_degree=3, target_pos=None,
    ),
    "c2": dict(
        name="c2-mid", log2N=15, q_bits=[40] * 14, n_p=5, p_bits=60, dnum=3, log2_scale=40,
        m=256, g=64, n_train=16384, n_features=63, n_valid=32768, seed=2, iters=10, batch_rows=1024,
        sigmoid_degree=3, target_pos=None,
    ),
    "c3": dict(
        name="c3-paper-scale", log2N=16, q_bits=[60] + [40] * 23, n_p=7, p_bits=42, dnum=4, log2_scale=40,
        m=128, g=256, n_train=422108, n_features=200, n_valid=844217, seed=3, iters=10, batch_rows=1024,
        sigmoid_degree=3, target_pos=0.2, standardise=True,
    ),
}
_BASE["c4"] = dict(_BASE["c3"], name="c4-batching-form")
_BASE["c5"] = dict(_BASE["c3"], name="c5-learned-sigmoid", sigmoid_degree=(5, 7))

# The m x g partition of section 2.2 with several column blocks (the padded width [1 | X | 0] is
# cut into blocks of g columns): a tiny case (3 row blocks, the last ragged, x 2 column blocks),
# the mid data as 16 x 4 blocks, and the paper-scale data as 413 x 7 blocks of 1,024 x 32.
_BASE["c1g"] = dict(_BASE["c1"], name="c1-grid-m512-g4", m=512, g=4, n_train=1200, n_valid=2400)
_BASE["c2g"] = dict(_BASE["c2"], name="c2-grid-m1024-g16", m=1024, g=16)
_BASE["c3g"] = dict(_BASE["c3"], name="c3-grid-m1024-g32", m=1024, g=32)

# The second workload of the paper (section 5.2, Table 2): the restructured MNIST 3-vs-8 task,
# 11,982 training and 1,984 validation samples of 14 x 14 = 196 pixel features in [0, 1], with
# the sigmoid approximation g16 on [-16, 16], learning rate 2 - (t/36)^2.5, and 7 ciphertexts
# of B-bar for the full batch (Table 2), i.e. 1,024 x 32 blocks: 12 row blocks x 7 column
# blocks at the paper-scale CKKS parameters.  The data is synthetic (the dataset is not
# available): a fifth of the pixels uniform on [0, 1] and the rest background 0, labels from a planted
# model with a strong signal (the task separates well: Table 2 reports AUROC 0.99), balanced classes.
_BASE["c6"] = dict(_BASE["c3"], name="c6-mnist-shaped", m=1024, g=32, n_train=11982, n_features=196,
                   n_valid=1984, seed=6, target_pos=0.5, standardise=False, x_range=(0.0, 1.0), x_density=0.2,
                   signal=5.0,
                   sigmoid="g16", lr_T=36.0, fo_lr=1.0)
# learning-rate settings of the Financial-shaped workloads (Table 1): 2 - (t/81)^2.5 for the quadratic
# gradient, 0.01/n for the first-order NAG baseline
for _k in ("c1", "c2", "c3", "c4", "c5", "c1g", "c2g", "c3g"):
    _BASE[_k].setdefault("sigmoid", "g8")
    _BASE[_k].setdefault("lr_T", 81.0)
    _BASE[_k].setdefault("fo_lr", 0.01)

CONFIGS = _BASE


def col_blocks(cfg):
    """Column blocks of g columns covering the bias column and the features."""
    return -(-(cfg["n_features"] + 1) // cfg["g"])


def padded_width(cfg):
    return col_blocks(cfg) * cfg["g"]


def get_config(key):
    cfg = copy.deepcopy(_BASE[key])
    cfg["key_seed"] = cfg["seed"] + 100
    cfg["enc_seed"] = cfg["seed"] + 200
    return cfg
