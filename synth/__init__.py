"""Seeded synthetic inputs shared by the product path and the CPU oracle.

This module only defines workloads (parameter sizes, layouts, seeds) and draws
the raw synthetic data (features X, labels y, the hidden weight vector).  It
holds none of the method's arithmetic: no encoding, no encryption, no
training.  The paper's two datasets are not available, so workloads are drawn
to the shapes of its experiments (section 5.1: 422,108 x 200 training rows,
844,217 validation rows; mini-batch 1,024).
"""
from .configs import CONFIGS, col_blocks, get_config, padded_width  # noqa: F401
from .data import make_dataset  # noqa: F401
