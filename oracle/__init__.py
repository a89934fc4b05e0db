"""FP64 CPU oracle for the GEEK data pass -- TEST INFRASTRUCTURE ONLY.

This package is the correctness authority for the HIP library.  It is plain,
slow numpy written from the paper (Luo, Huang, Tung: "A Generic Distributed
Clustering Framework for Massive Data", arXiv 2106.10515).  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product path (``paper_2106_10515_amd``) never imports, links or
executes anything here, and this package never imports the product path.  The
two share only the seeded input generators in ``workloads/``.

Where a step has a plain definition (the E2LSH code, MinHash, exact-tuple
bucketing, centroids, nearest-centre assignment, SSE) the oracle computes that
definition directly in a stated floating-point order.  SILK is a heuristic, so
the oracle follows Algorithm 4's steps in the paper's order.

A further assignment pass (Section 4.3) regroups the objects by their
assigned centre and assigns them again to the recomputed centroids.
Quantile bucketing (Algorithm 1) ranks the objects by each QALSH value and
splits the ranks evenly into t buckets.  Densified one-permutation hashing
(Algorithm 3's first step) reduces sets to D dimensions with one permutation
and rotation densification.

Pins (see ``tests/test_oracle_*.py``): exact rational arithmetic, closed forms
(E2LSH collision probability, MinHash collision probability = Jaccard),
published MurmurHash3 finalizer vectors, brute force on tiny inputs, the
SILK worked example (Example 2) and an independent dictionary version of
Algorithm 4, for further passes the invariants that determine the regrouping
plus Lloyd's monotone SSE and a hand-worked case, and for DOPH hand-worked
bins and densification, a plain per-bin loop, special sets and the
collision rate = Jaccard.

Without a printed value: SILK's end-to-end seed sets on hashed inputs (the
paper's figures carry no coordinates).  The pieces are pinned instead.  The
worked example (explicit bins) and invariants pin the vote, threshold and
de-duplication.  A brute-force per-bucket minimum of the permuted ids pins
the bucket signatures.  A hand-worked case whose tuples tie in their leading
word pins the seed order.  An independent dictionary version of Algorithm 4
pins the whole pass.
"""

from .lsh import (  # noqa: F401
    code_bits,
    codes_in_range,
    e2lsh_codes,
    fmix32,
    hetero_tokens,
    minhash_sets,
    perm,
)
from .buckets import bucketize, bucketize_tables  # noqa: F401
from .silk import majority, silk_from_bins, silk_seeds  # noqa: F401
from .assign import (  # noqa: F401
    assign_euclid,
    assign_hetero,
    assign_sig,
    centroids,
    euclid_dist_pairs,
    euclid_dist_rows,
    hetero_dist_pairs,
    modes,
    radius,
    sse,
)
from .refine import assignment_pass, regroup  # noqa: F401
from .quantile import qalsh_values, quantile_buckets  # noqa: F401
from .doph import densify_rotation, doph_bin, doph_sets  # noqa: F401
