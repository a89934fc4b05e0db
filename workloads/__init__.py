"""Seeded synthetic inputs for the GEEK data pass.

This package is the only code that both the FP64 oracle (``oracle/``) and the
HIP path (``paper_2106_10515_amd``) consume.  It draws data and the random
parameters the method needs (projection vectors, offsets, MinHash and SILK key
words) and holds none of the method's arithmetic: no hashing, bucketing,
seeding, centroid or distance computation lives here.

The datasets of the paper (Sift10M, URL, GeoNames) are not available, so the
generators produce inputs of the same shape and structure (Table 2 of the
paper): dense Gaussian mixtures, sparse sets with Zipf-distributed tokens and
planted clusters, and heterogeneous rows with numeric and categorical
attributes.
"""

from .gen import (  # noqa: F401
    CONFIGS,
    STREAM_DATA,
    batched_jobs,
    dense_mixture,
    e2lsh_params,
    hetero_rows,
    key_words,
    largest_remainder,
    planted_seeds,
    rng,
    sparse_sets,
)
