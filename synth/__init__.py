"""Seeded synthetic row streams shaped like the paper's workloads.

This module only draws inputs; it holds none of the sketch's arithmetic, so
both the FP64 oracle and the GPU library can be fed the very same bytes.

The paper's own datasets are Uniform Random, Random Noisy (A = S D U + N/zeta,
Sec. 5.1 "Hardware, Environments, and Datasets") and GloVe word vectors
(d = 300, not available offline).  The streams below are synthetic stand-ins
with the same structure: a low-rank signal in a random orthonormal basis with
a prescribed spectrum, plus i.i.d. Gaussian noise.
"""
from .streams import (  # noqa: F401
    StreamSpec,
    lowrank_rows,
    persistent_small,
    persistent_tight,
    window_stream,
    serving_streams,
    sparse_sites,
    random_noisy,
)
