/*
 * geek.h -- C ABI of libgeek.so, the GEEK data pass on one AMD Instinct
 * MI355X (gfx950) GPU.
 *
 * GEEK (Luo, Huang, Tung, "A Generic Distributed Clustering Framework for
 * Massive Data", arXiv 2106.10515) clusters data in three phases: a data
 * transformation that turns objects into buckets with LSH (Section 3.1),
 * SILK seeding from similar buckets (Section 3.2, Algorithm 4), and a
 * one-pass assignment of every object to its closest central vector
 * (Section 3.3, Eq. (1)).  This library exposes six calls:
 *
 *   geek_hash        LSH values of every object (E2LSH codes packed into an
 *                    exact per-table key; MinHash signatures of sets or of
 *                    heterogeneous rows)
 *   geek_bucketize   group objects with identical table keys into buckets
 *   geek_silk_seeds  SILK: bins of similar buckets, majority voting, the
 *                    seeding threshold and near-duplicate removal
 *   geek_assign      central vectors of the seeds and the one-pass assignment
 *   geek_regroup     the clusters of an assignment as the seeds of a further
 *                    assignment pass
 *   geek_quantile_buckets  Algorithm 1's dense transformation: buckets of
 *                    equal size along each projection
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every pointer inside a job descriptor is a DEVICE pointer unless the
 *   field says "host".  Device buffers are allocated and freed by the caller;
 *   the library never frees caller memory and holds no device memory between
 *   calls.  Base pointers must be 16-byte aligned.
 * - Each call takes an array of ``njobs`` job descriptors (host memory),
 *   a caller-owned device workspace of at least the size that
 *   ``geek_workspace_size`` returns for the same jobs, a device status word
 *   ``d_status`` (int32, device) and a HIP stream (``hipStream_t`` passed as
 *   ``void*``; NULL = the default stream).
 * - Calls are stream-ordered and return without waiting for the GPU: no
 *   call performs a host synchronization or a device allocation, so every
 *   call can be captured in a HIP graph.  Sizes that only the device knows
 *   (the number of buckets, SILK's intermediate collections) are read by the
 *   kernels from device memory; launches are sized by host upper bounds.
 * - Host-detectable errors (bad arguments, workspace too small, unsupported
 *   sizes, launch failure) return a negative status at once and enqueue no
 *   work.  Data-dependent errors (non-finite input, a hash code outside the
 *   packable range, too little output capacity, no seeds, an empty set) are
 *   written by the kernels into ``*d_status`` (first error wins; later
 *   kernels of the same call become no-ops once it is non-zero).  The caller
 *   zeroes ``*d_status`` before a call chain and reads it after synchronizing
 *   the stream.
 * - A call with several jobs may run independent jobs on up to four
 *   internal streams of the device (default priority, created by the first
 *   such call and kept until the process ends): an event recorded on
 *   ``stream`` starts them and ``stream`` waits for all of them before the
 *   call's later work, so the call stays ordered on ``stream`` and can be
 *   captured in a HIP graph (as parallel branches).  The first multi-job
 *   call on a device should not itself be under capture.
 * - Ids are 0-based uint32.  Matrices are row-major.
 */
#ifndef GEEK_H
#define GEEK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define GEEK_OK 0
#define GEEK_ERR_ARG (-1)         /* null/misaligned pointer, inconsistent sizes */
#define GEEK_ERR_WORKSPACE (-2)   /* ws_bytes below geek_workspace_size */
#define GEEK_ERR_UNSUPPORTED (-3) /* a size the library does not handle */
#define GEEK_ERR_HIP (-4)         /* HIP launch failure; see geek_last_hip_error */
/* data-dependent, written to *d_status */
#define GEEK_ERR_NONFINITE 1      /* NaN or Inf in a float input */
#define GEEK_ERR_RANGE 2          /* hash code outside the packable range */
#define GEEK_ERR_CAPACITY 3       /* output capacity too small (see `needed`) */
#define GEEK_ERR_NO_SEEDS 4       /* SILK found no seed */
#define GEEK_ERR_EMPTY_SET 5      /* a set (or seed) with no element */
#define GEEK_ERR_KEYS 6           /* bucketize: over 1792 distinct keys of one bin
                                     share a 32-bit fingerprint and 24 bits of an
                                     independent second hash (not handled) */

/* ---- geek_hash ----------------------------------------------------------
 * The data transformation's LSH values (paper Section 3.1).
 *
 * GEEK_HASH_DENSE: E2LSH, code[i][p] = floor((a_p . x_i + b_p) / w), the form
 *   named in the Remarks after Example 1, with a_p drawn as in Eq. (3)
 *   (caller supplies A and b).  P = m * L projections; table l uses
 *   projections l*m .. l*m+m-1.  The code is the value of the float64
 *   evaluation s = sum_t a_pt * x_it accumulated for t = 0..d-1 in order,
 *   v = s + b_p, floor(v / w): the GPU computes in float32 on the matrix
 *   cores and recomputes every (i, p) whose float32 quotient lies within a
 *   rigorous error bound of an integer in exactly that float64 order, so
 *   the codes are bit-exact.  The m codes of table l and object i are
 *   packed into a 128-bit key keys[l][i][0..3]: code j occupies bits
 *   j*B .. j*B+B-1 (little-endian over the four words) as code + 2^(B-1),
 *   with B = min(32, 128 / m); a code outside [-2^(B-1), 2^(B-1)) sets
 *   GEEK_ERR_RANGE.  The packing is injective, so equal keys <=> equal code
 *   tuples.
 * GEEK_HASH_SETS: MinHash (Eq. (2), Algorithm 3).  sig[i][f] = min over the
 *   tokens t of set i of pi_f(t), pi_f(t) = (a_f * fmix32(t) + b_f) mod 2^32
 *   with a_f = mh_keys[f][0] | 1, b_f = mh_keys[f][1] and fmix32 the
 *   MurmurHash3 32-bit finalizer (a bijection of 32-bit words).  An empty
 *   set sets GEEK_ERR_EMPTY_SET.
 * GEEK_HASH_HETERO: Algorithm 2.  The numeric attributes X [n][d] get
 *   P = m * L E2LSH codes as above; categorical attribute a with value v
 *   becomes token (a << 16) | v, numeric projection p with code c becomes
 *   0x80000000 | (p << 16) | (c + 32768); the row's n_cat + P tokens are
 *   then MinHashed as a set into sig [n][F].  A value or code outside 16
 *   bits sets GEEK_ERR_RANGE.
 */
#define GEEK_HASH_DENSE 0
#define GEEK_HASH_SETS 1
#define GEEK_HASH_HETERO 2
/* GEEK_HASH_DOPH: densified one-permutation hashing of sets, the dimension
 *   reduction that Algorithm 3 applies first (Section 3.1, Sparse Data;
 *   Section 3.3 represents sets by the reduced dimensions; Section 4.1
 *   reduces URL to 400).  With pi(t) = (a * fmix32(t) + b) mod 2^32,
 *   a = mh_keys[0][0] | 1, b = mh_keys[0][1] (one permutation, so mh_keys
 *   holds one key pair), the permuted values of set i fall into D = F equal
 *   ranges of [0, 2^32): value v lies in bin floor(v * D / 2^32).
 *   sig[i][j] = the smallest permuted value of the set in bin j; an empty bin
 *   takes the value of the first non-empty bin to its right, cyclically
 *   (rotation densification, Shrivastava and Li, ICML 2014).  Every
 *   coordinate collides for two sets with probability equal to their
 *   Jaccard similarity, so the D coordinates serve as the MinHash values of
 *   the (K, L) bands (band b = coordinates b*K .. b*K+K-1) and as the set's
 *   reduced representation for modes.  1 <= F <= 4096.  Fields used:
 *   n, offsets, tokens, mh_keys, F, sig [n][F].  An empty set sets
 *   GEEK_ERR_EMPTY_SET (the row is then unspecified). */
#define GEEK_HASH_DOPH 3

typedef struct geek_hash_job {
  int32_t kind;             /* GEEK_HASH_* */
  int32_t d;                /* dense/hetero: attributes per row (1..1024) */
  int64_t n;                /* objects (0 <= n < 2^31) */
  /* dense and the numeric part of hetero */
  const float* X;           /* [n][ldx] float32, ldx >= d */
  int64_t ldx;
  const float* A;           /* [m*L][d] projection vectors */
  const float* b;           /* [m*L] offsets in [0, w) */
  int32_t m;                /* codes per table (dense: 1..32) */
  int32_t L;                /* tables */
  float w;                  /* bucket width, > 0 */
  int32_t F;                /* sets/hetero: MinHash functions */
  uint32_t* keys;           /* dense out: [L][n][4] packed table keys */
  int32_t* codes;           /* optional out: [n][m*L] codes (NULL to skip) */
  /* sets */
  const int64_t* offsets;   /* [n+1], set i = tokens[offsets[i]..offsets[i+1]) */
  const uint32_t* tokens;   /* [nnz] */
  /* hetero */
  const int32_t* cat;       /* [n][n_cat], values in [0, 65536) */
  int32_t n_cat;
  int32_t pad0;
  const uint32_t* mh_keys;  /* [F][2] MinHash key words */
  uint32_t* sig;            /* sets/hetero out: [n][F] */
  unsigned long long* n_fixup; /* optional out (device, accumulated):
                                  (i, p) pairs recomputed in float64 */
  uint32_t* key_fp;         /* optional out (GEEK_HASH_DENSE only; NULL to skip):
                               [L][n] the 32-bit fingerprint geek_bucketize
                               takes of each packed key; hand it to
                               geek_bucketize (key_fp) so that call need not
                               read the keys to fingerprint them */
} geek_hash_job;

/* ---- geek_bucketize -----------------------------------------------------
 * Buckets of every table: objects whose table key is identical share a
 * bucket ("T[G(x_j)].push(j)" in Algorithms 2 and 3; the exact tuple of the
 * table's hash values).  The key of (table t, object i) is the key_words
 * uint32 words at keys + t*table_stride + i*row_stride (dense keys from
 * geek_hash: key_words 4, table_stride n*4, row_stride 4; band b of MinHash
 * signatures with K rows: key_words K, table_stride K, row_stride F).
 * Output per table t, canonical: buckets ordered by their smallest member,
 * members ascending; bucket j of table t is
 * members[t*n + offsets[t*(n+1) + j] .. t*n + offsets[t*(n+1) + j + 1]).
 */
typedef struct geek_bucketize_job {
  int64_t n;                /* objects per table (1 <= n < 2^31) */
  int32_t T;                /* tables */
  int32_t key_words;        /* 1..4 */
  const uint32_t* keys;
  int64_t table_stride;     /* in uint32 words */
  int64_t row_stride;       /* in uint32 words */
  uint32_t* members;        /* out [T][n] */
  uint32_t* offsets;        /* out [T][n+1]; entries past nbuckets[t] unspecified */
  uint32_t* nbuckets;       /* out [T] */
  uint32_t* bucket_of;      /* optional out [T][n] */
  const uint32_t* key_fp;   /* optional in [T][n]: the fingerprints of exactly
                               these keys as geek_hash (key_fp) of this library
                               writes them, or NULL (computed from the keys).
                               Buckets stay exact-key groups (keys are still
                               compared), but a bucket is only found whole
                               if equal keys carry equal fingerprints */
} geek_bucketize_job;

/* ---- geek_silk_seeds ----------------------------------------------------
 * SILK (Algorithm 4) over all buckets of all tables (the collection B, in
 * the geek_bucketize output layout).  For each of L SILK tables, K MinHash
 * functions over object ids (pi as in GEEK_HASH_SETS, key words
 * silk_keys[(s*K + k)][0..1]) give every bucket the signature
 * G(B) = (min_{x in B} pi_1(x), ..., min pi_K(x)); buckets with identical G
 * form a bin; bins of at most one bucket are skipped; C_shared = the ids
 * appearing in more than half of the bin's buckets (2*count > |Bin|); it
 * joins the multiset C when |C_shared| >= delta.  Near-duplicates are then
 * removed with one more table (key rows L*K .. L*K+K-1) over the sets of C:
 * a bin holding one set passes it through, a bin of several sets is
 * majority-voted and delta-filtered.  Seeds are ordered by the ascending
 * lexicographic K-tuple of their de-duplication bin, members ascending.
 * Output CSR: seed j = seed_members[seed_offsets[j] .. seed_offsets[j+1]).
 * A bin contributes only a non-empty C_shared (delta < 1 acts as delta = 1).
 * The intermediate multiset C is held in the workspace with room for cap_c
 * members (4 * cap_members when cap_c is 0) and cap_c / max(delta, 1) + 1
 * sets.  needed [3] = {seeds, seed members, members of C}; if C does not fit,
 * needed = {0, 0, the cap_c that fits} and GEEK_ERR_CAPACITY is set; if the
 * seeds do not fit cap_k / cap_members, needed holds their sizes and
 * GEEK_ERR_CAPACITY is set (outputs unspecified either way); no seed sets
 * GEEK_ERR_NO_SEEDS.  The call never reads sizes back to the host.
 * Requires 1 <= T <= 128 (GEEK_ERR_UNSUPPORTED above), T * n < 2^31 and a C
 * capacity below 2^31.  The workspace grows with T * n (about 100 bytes per
 * (table, object)) and with the C capacity (about 50 bytes per member).
 */
typedef struct geek_silk_job {
  int64_t n;                /* objects */
  int32_t T;                /* transform tables */
  int32_t K;                /* MinHash functions per SILK table (1..4) */
  const uint32_t* members;  /* [T][n]   (geek_bucketize output) */
  const uint32_t* offsets;  /* [T][n+1] */
  const uint32_t* nbuckets; /* [T] */
  int32_t L;                /* SILK tables */
  int32_t delta;            /* seeding threshold */
  const uint32_t* silk_keys;/* [(L+1)*K][2] */
  int64_t cap_k;            /* capacity of seed_offsets minus one */
  int64_t cap_members;      /* capacity of seed_members */
  uint32_t* seed_offsets;   /* out [cap_k+1] */
  uint32_t* seed_members;   /* out [cap_members] */
  uint32_t* k_out;          /* out [1] number of seeds */
  unsigned long long* needed;   /* out [3] seeds, seed members, members of C */
  unsigned long long* counters; /* optional out [4]: hash evaluations,
                                   voted (bin, id) pairs, |C| before
                                   de-duplication, multi-bucket bins */
  int64_t cap_c;            /* room of the multiset C in members (workspace);
                               0 = 4 * cap_members */
} geek_silk_job;

/* ---- geek_assign --------------------------------------------------------
 * Central vectors and the one-pass assignment (Section 3.3).
 * GEEK_METRIC_EUCLID: centroid c_j = (sum over members of seed j, ascending,
 *   of x_i, accumulated in float64 one addition at a time) / |C_j|;
 *   ID_i = argmin_j D(i, j) with D the squared Euclidean distance evaluated
 *   in float64 as: for t = 0..d-1, delta = x_it - c_jt, acc += delta*delta
 *   (each operation rounded, no fused multiply-add); lowest j on ties.
 *   The matrix cores compute an approximate D~ = |x|^2 - 2 x.c + |c|^2 in
 *   `precision`; every j whose D~ lies within a rigorous per-row error bound
 *   of the row minimum is a candidate.  Rows with one candidate (BF16) or at
 *   most 8 (FP8, FP32) have their candidates re-evaluated with the float64
 *   formula above; the other rows are rescanned in FP32 keeping up to 32
 *   candidates, and rows with still more are evaluated in float64 against
 *   every seed, so the assignment is exact.
 * GEEK_METRIC_SIG: modes mode_j[f] = most frequent sig value of the members
 *   at position f (smallest value on ties); ID_i = argmax_j #{f : sig[i][f]
 *   == mode_j[f]} (lowest j on ties); dist = 1 - matches / F.
 * GEEK_METRIC_HETERO: D = D_num(i, j) + gamma * #{a : cat[i][a] !=
 *   catmode_j[a]} with D_num as for EUCLID over X and the centroid, and
 *   catmode the per-attribute mode of the members.
 * Outputs: assign [n]; centroids [k][d] (EUCLID, HETERO); modes [k][F]
 *   (SIG) or [k][n_cat] (HETERO); dist [n] (optional) = D(i, ID_i);
 *   sse [1] = sum_i dist_i in float64, sequential within consecutive blocks
 *   of 4096 rows, then over the block sums; radius [k] (optional) = sqrt of
 *   the largest member distance (EUCLID, HETERO: of D), 0 for empty
 *   clusters; counters (optional) [4]: rows certified by the first pass,
 *   rows rescanned at higher precision, rows scanned in float64, candidate
 *   distances evaluated in float64.
 */
#define GEEK_METRIC_EUCLID 0
#define GEEK_METRIC_SIG 1
#define GEEK_METRIC_HETERO 2

#define GEEK_PREC_FP32 0
#define GEEK_PREC_BF16 1
#define GEEK_PREC_FP8 2

typedef struct geek_assign_job {
  int32_t metric;           /* GEEK_METRIC_* */
  int32_t precision;        /* GEEK_PREC_* (EUCLID, HETERO) */
  int64_t n;
  int32_t d;                /* EUCLID/HETERO: numeric attributes (1..256) */
  int32_t k;                /* host: number of seeds (>= 1) */
  const float* X;           /* [n][ldx] */
  int64_t ldx;
  const uint32_t* sig;      /* SIG: [n][F] */
  int32_t F;
  int32_t n_cat;            /* HETERO */
  const int32_t* cat;       /* HETERO: [n][n_cat] */
  double gamma;             /* HETERO mismatch weight */
  const uint32_t* seed_offsets; /* [k+1] */
  const uint32_t* seed_members;
  int32_t* assign;          /* out [n] */
  double* centroids;        /* out [k][d] */
  uint32_t* modes;          /* out SIG [k][F]; HETERO [k][n_cat] (as uint32) */
  double* dist;             /* optional out [n] */
  double* sse;              /* out [1] */
  double* radius;           /* optional out [k] */
  unsigned long long* counters; /* optional out [4] */
  int64_t n_members;        /* host: seed_offsets[k], the total number of seed
                               members (required by SIG and HETERO, which
                               size their mode computation by it; EUCLID also
                               accepts 0 = not given, or the capacity of
                               seed_members).  When EUCLID / HETERO seeds
                               average 64 members or more, centroids are
                               computed from a dimension-major copy of the
                               members' values (n_members x d floats of
                               workspace) */
  unsigned long long* t_done; /* optional out [1]: device wall-clock ticks
                               (geek_wallclock_hz per second) from the start
                               of the call to the moment this job's outputs
                               were complete (batched calls; jobs finish in
                               any order), or the absolute tick count at that
                               moment (njobs = 1) */
  const uint32_t* k_dev;    /* optional [1], device (EUCLID, njobs = 1): the
                               number of seeds as the device knows it, for
                               seeds made earlier in the same stream (such as
                               geek_silk_seeds' *k_out) without reading the
                               count back to the host, so a whole pass can be
                               captured in one graph.  k is then the host
                               capacity: seeds j >= min(*k_dev, k) take no
                               part (their seed_offsets entries are not read;
                               centroids rows and radius entries of such j are
                               written as 0), and the call costs what k
                               seeds cost.  *k_dev = 0 sets GEEK_ERR_NO_SEEDS.
                               NULL: k seeds. */
} geek_assign_job;

/* ---- geek_regroup ---------------------------------------------------------
 * The clusters of an assignment as seeds for a further assignment pass
 * (Section 4.3, Clustering Performance: several passes of the data
 * assignment give more compact clusters).  Cluster j = {i : assign[i] == j}
 * with its members in ascending i; clusters with no member are dropped and
 * the others keep the order of j, so the r-th output cluster is the r-th
 * non-empty label.  Passing the result to geek_assign (seed_offsets,
 * seed_members, k = *k_out) recomputes the central vectors from the clusters
 * and assigns every object again: one step of Lloyd's iteration.
 * Outputs: seed_offsets [k + 1] (entries 0 .. *k_out written, the last = n),
 *   seed_members [n], *k_out, label_of [k] (optional; entries 0 .. *k_out - 1:
 *   the label j of each output cluster).  A label outside [0, k) sets
 *   GEEK_ERR_RANGE in *d_status (the outputs are then unspecified).
 */
typedef struct geek_regroup_job {
  int64_t n;                 /* objects (0 <= n < 2^31) */
  int32_t k;                 /* host: labels lie in [0, k), k >= 1 */
  const int32_t* assign;     /* [n] */
  uint32_t* seed_offsets;    /* out [k + 1] */
  uint32_t* seed_members;    /* out [n] */
  uint32_t* k_out;           /* out [1] */
  int32_t* label_of;         /* optional out [k] */
} geek_regroup_job;

/* ---- geek_quantile_buckets -------------------------------------------------
 * Quantile bucketing of dense rows (Algorithm 1, the homogeneous dense data
 * transformation): for each of m projection vectors a_p, table p ranks the
 * objects by the QALSH value a_p . x_i and splits the ranks evenly into t
 * buckets.  The value is evaluated in float64 exactly as: s = 0; for t = 0 ..
 * d-1: s = s + a_pt * x_it (the product of two float32 values is exact in
 * float64; one rounding per addition).  Equal values are ordered by id; rank
 * r goes to bucket floor(r * t / n), so bucket b holds the ranks
 * ceil(b n / t) .. ceil((b + 1) n / t) - 1 and sizes differ by at most one.
 * Outputs per table p: members [m][n] (bucket b of table p is members[p][
 * offsets[p][b] .. offsets[p][b + 1]), ids ascending within a bucket),
 * offsets [m][t + 1], optional bucket_of [m][n].  A non-finite x or a sets
 * GEEK_ERR_NONFINITE.  Requires 1 <= t <= n < 2^31, 1 <= d <= 256.
 */
typedef struct geek_quantile_job {
  int64_t n;
  int32_t d;
  int32_t m;                 /* projections = tables */
  int32_t t;                 /* buckets per table */
  int32_t pad0;
  const float* X;            /* [n][ldx] */
  int64_t ldx;
  const float* A;            /* [m][d] projection vectors */
  uint32_t* members;         /* out [m][n] */
  uint32_t* offsets;         /* out [m][t + 1] */
  uint32_t* bucket_of;       /* optional out [m][n] */
} geek_quantile_job;

/* ---- entry points -------------------------------------------------------- */
#define GEEK_OP_HASH 0
#define GEEK_OP_BUCKETIZE 1
#define GEEK_OP_SILK 2
#define GEEK_OP_ASSIGN 3
#define GEEK_OP_REGROUP 4
#define GEEK_OP_QUANTILE 5

/* Bytes of device workspace the call `op` needs for these jobs (host).  For
 * geek_hash and geek_bucketize with several jobs it is min(njobs, 4) slices
 * of the largest job's workspace (one per stream the jobs run on); a smaller
 * workspace of at least one slice runs fewer jobs at once. */
int32_t geek_workspace_size(int32_t op, const void* jobs, int32_t njobs, size_t* bytes);

int32_t geek_hash(const geek_hash_job* jobs, int32_t njobs, void* ws, size_t ws_bytes,
                  int32_t* d_status, void* stream);
int32_t geek_bucketize(const geek_bucketize_job* jobs, int32_t njobs, void* ws,
                       size_t ws_bytes, int32_t* d_status, void* stream);

/* geek_hash without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same jobs, outputs, status words and
 * errors as geek_hash; the kernels' scratch is a library-owned device array
 * of GEEK_NOALLOC_SCRATCH_BYTES per GPU (each GPU the call runs on holds it
 * until the process ends).  A job whose workspace (geek_workspace_size)
 * exceeds it -- e.g. heterogeneous rows with n * m * L above about 2^18, or
 * dense rows with more than about 750 projections (d <= 128; about 950 for
 * d > 128) -- returns GEEK_ERR_WORKSPACE before any work is enqueued.  The jobs run one
 * after another on `stream`.  The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine).  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other streams, other host
 * threads) race, so the caller must order them. */
#define GEEK_NOALLOC_SCRATCH_BYTES 1048576
int32_t geek_hash_noalloc(const geek_hash_job* jobs, int32_t njobs, int32_t* d_status, void* stream);
int32_t geek_silk_seeds(const geek_silk_job* jobs, int32_t njobs, void* ws, size_t ws_bytes,
                        int32_t* d_status, void* stream);
/* geek_assign with njobs > 1 and every job GEEK_METRIC_EUCLID in one
 * precision (many independent clustering problems at once): the jobs'
 * centroids are prepared on the internal streams, then one persistent
 * matrix-core launch per padded dimension (32, 64, 128, 256) scans the tiles
 * of all jobs of that dimension in call order, with the tile shape set by
 * geek_set_scan_tiles, then the float64 checks of each job run on the
 * internal streams.  Each job's outputs are bit-identical to a call with
 * that job alone.  The workspace is the sum of the jobs' own workspaces
 * (geek_workspace_size reports it).  Any other mix of jobs runs one job
 * after another in a shared workspace. */
int32_t geek_assign(const geek_assign_job* jobs, int32_t njobs, void* ws, size_t ws_bytes,
                    int32_t* d_status, void* stream);
/* geek_regroup: jobs run one after another in a shared workspace; no host
 * synchronization, no device allocation. */
int32_t geek_regroup(const geek_regroup_job* jobs, int32_t njobs, void* ws, size_t ws_bytes,
                     int32_t* d_status, void* stream);
/* geek_quantile_buckets: jobs and tables run one after another in a shared
 * workspace; no host synchronization, no device allocation. */
int32_t geek_quantile_buckets(const geek_quantile_job* jobs, int32_t njobs, void* ws, size_t ws_bytes,
                              int32_t* d_status, void* stream);

/* ---- profiling (opt-in) -------------------------------------------------
 * With profiling enabled the library brackets its main kernels with HIP
 * events recorded on the call's stream.  geek_profile(1) clears earlier
 * records and starts recording, geek_profile(0) stops.  geek_profile_read
 * waits for the recorded events of kernel `id` and returns their summed
 * duration (ms) and count.  Not for use under graph capture.
 */
#define GEEK_PROF_E2LSH 0        /* k_e2lsh: projection GEMM + floor/pack */
#define GEEK_PROF_BUCKETIZE 1    /* all kernels of one geek_bucketize job */
#define GEEK_PROF_ASSIGN_SCAN 2  /* first matrix-core pass of geek_assign */
#define GEEK_PROF_ASSIGN 3       /* all kernels of one geek_assign job */
#define GEEK_PROF_MINHASH 4      /* MinHash kernel of geek_hash */
#define GEEK_PROF_SILK 5         /* all kernels of one geek_silk_seeds job */
#define GEEK_PROF_BZ_SORT 6      /* per-bin sort kernel of geek_bucketize */
#define GEEK_PROF_COUNT 8
int32_t geek_profile(int32_t enable);
int32_t geek_profile_read(int32_t id, double* total_ms, int64_t* launches);

/* Tile shape of the batched Euclidean first pass (geek_assign with several
 * jobs) for one precision (GEEK_PREC_*) and padded depth dp (32, 64, 128 or
 * 256, the next of these at or above d): ncb column blocks of 32 rows per
 * wavefront (tiles of 128 * ncb rows; 1 or 2), nbuf LDS stages of seeds
 * (1 or 2), and blocks_per_cu persistent workgroups per compute unit
 * (1..64).  All shapes give identical results; the package's autotuner times
 * them and installs the fastest.  ncb = nbuf = blocks_per_cu = 0 restores the
 * built-in default (ncb 2, nbuf 2 for BF16/FP8; 1, 1 for FP32; 8 workgroups
 * per CU).  The table is process-wide host state: set it before the calls it
 * should affect (a call reads it when it is enqueued).  Returns GEEK_ERR_ARG
 * for an unknown precision or depth or blocks_per_cu out of range, and
 * GEEK_ERR_UNSUPPORTED for a shape that is not compiled (FP32 allows ncb 2
 * only with nbuf 1 and dp <= 64).  Host only: makes no HIP call. */
int32_t geek_set_scan_tiles(int32_t precision, int32_t dp, int32_t ncb, int32_t nbuf, int32_t blocks_per_cu);
/* The shape geek_set_scan_tiles last installed (or the default). */
int32_t geek_get_scan_tiles(int32_t precision, int32_t dp, int32_t* ncb, int32_t* nbuf, int32_t* blocks_per_cu);

/* Static description of a status code. */
const char* geek_status_string(int32_t status);
/* Ticks per second of the device wall clock used by t_done (device 0 of
 * the calling thread's current device); 0 if unknown. */
int64_t geek_wallclock_hz(void);
/* Library version string, e.g. "geek 0.1.0 gfx950". */
const char* geek_version(void);
/* The last HIP error message seen by this thread (empty if none). */
const char* geek_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GEEK_H */
