/* Prints sizeof and field offsets of the job structs of include/geek.h, for
   the ctypes layout test (compiled by tests/test_abi.py with gcc). */
#include <stddef.h>
#include <stdio.h>
#include "geek.h"
#define F(T, f) printf(#T " " #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("geek_hash_job sizeof %zu\n", sizeof(geek_hash_job));
  F(geek_hash_job, kind); F(geek_hash_job, d); F(geek_hash_job, n); F(geek_hash_job, X);
  F(geek_hash_job, ldx); F(geek_hash_job, A); F(geek_hash_job, b); F(geek_hash_job, m);
  F(geek_hash_job, L); F(geek_hash_job, w); F(geek_hash_job, F); F(geek_hash_job, keys);
  F(geek_hash_job, codes); F(geek_hash_job, offsets); F(geek_hash_job, tokens);
  F(geek_hash_job, cat); F(geek_hash_job, n_cat); F(geek_hash_job, mh_keys);
  F(geek_hash_job, sig); F(geek_hash_job, n_fixup); F(geek_hash_job, key_fp);
  printf("geek_bucketize_job sizeof %zu\n", sizeof(geek_bucketize_job));
  F(geek_bucketize_job, n); F(geek_bucketize_job, T); F(geek_bucketize_job, key_words);
  F(geek_bucketize_job, keys); F(geek_bucketize_job, table_stride);
  F(geek_bucketize_job, row_stride); F(geek_bucketize_job, members);
  F(geek_bucketize_job, offsets); F(geek_bucketize_job, nbuckets); F(geek_bucketize_job, bucket_of);
  F(geek_bucketize_job, key_fp);
  printf("geek_silk_job sizeof %zu\n", sizeof(geek_silk_job));
  F(geek_silk_job, n); F(geek_silk_job, T); F(geek_silk_job, K); F(geek_silk_job, members);
  F(geek_silk_job, offsets); F(geek_silk_job, nbuckets); F(geek_silk_job, L);
  F(geek_silk_job, delta); F(geek_silk_job, silk_keys); F(geek_silk_job, cap_k);
  F(geek_silk_job, cap_members); F(geek_silk_job, seed_offsets); F(geek_silk_job, seed_members);
  F(geek_silk_job, k_out); F(geek_silk_job, needed); F(geek_silk_job, counters);
  F(geek_silk_job, cap_c);
  printf("geek_assign_job sizeof %zu\n", sizeof(geek_assign_job));
  F(geek_assign_job, metric); F(geek_assign_job, precision); F(geek_assign_job, n);
  F(geek_assign_job, d); F(geek_assign_job, k); F(geek_assign_job, X); F(geek_assign_job, ldx);
  F(geek_assign_job, sig); F(geek_assign_job, F); F(geek_assign_job, n_cat);
  F(geek_assign_job, cat); F(geek_assign_job, gamma); F(geek_assign_job, seed_offsets);
  F(geek_assign_job, seed_members); F(geek_assign_job, assign); F(geek_assign_job, centroids);
  F(geek_assign_job, modes); F(geek_assign_job, dist); F(geek_assign_job, sse);
  F(geek_assign_job, radius); F(geek_assign_job, counters); F(geek_assign_job, n_members);
  F(geek_assign_job, t_done); F(geek_assign_job, k_dev);
  printf("geek_regroup_job sizeof %zu\n", sizeof(geek_regroup_job));
  F(geek_regroup_job, n); F(geek_regroup_job, k); F(geek_regroup_job, assign);
  F(geek_regroup_job, seed_offsets); F(geek_regroup_job, seed_members); F(geek_regroup_job, k_out);
  F(geek_regroup_job, label_of);
  printf("geek_quantile_job sizeof %zu\n", sizeof(geek_quantile_job));
  F(geek_quantile_job, n); F(geek_quantile_job, d); F(geek_quantile_job, m); F(geek_quantile_job, t);
  F(geek_quantile_job, X); F(geek_quantile_job, ldx); F(geek_quantile_job, A);
  F(geek_quantile_job, members); F(geek_quantile_job, offsets); F(geek_quantile_job, bucket_of);
  return 0;
}
