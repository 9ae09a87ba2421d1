"""Seeded synthetic inputs for the FBPQ search: data, queries, index, index files.

This package is shared by the oracle tests and by the GPU path's tests and
benchmark. It holds input generation only (a Gaussian-mixture stand-in for SIFT
descriptors, Lloyd training of the codebooks, encoding, cell-contiguous
storage); it computes nothing the search computes (no query distances, no cell
traversal, no candidate scoring, no top-k).
"""

from .gen import (  # noqa: F401
    Index,
    gmm_means,
    sample_points,
    build_index,
    make_queries,
    random_rotation,
    draw_L_k,
    lossless_index,
    lossless_local_index,
    with_local_codebooks,
    random_index,
    zipf_index,
    tiny_index,
)
from .indexfile import write_index, read_index  # noqa: F401
