/*
 * ht_debug.h -- host-only checks of the launch plans of libht (no GPU used).
 *
 * Each function builds the complete launch plan of the corresponding entry
 * point of ht.h for the given shapes (data pointers in X are ignored: every
 * buffer is replaced by a fake, disjoint address range of exactly the size the
 * shapes imply, the workspace by its individual allocations) and proves that
 * every address any kernel of the plan may read or write lies inside one of
 * those ranges.  Returns HT_OK, or HT_EINVAL with ht_last_error() naming the
 * first launch and operand that would leave its buffer.  Meant for tests that
 * vet new shapes on the CPU before anything runs on a GPU.
 */
#ifndef HT_DEBUG_H
#define HT_DEBUG_H
#include "ht.h"
#ifdef __cplusplus
extern "C" {
#endif
ht_status ht_debug_validate_truncate(const ht_desc* X, int32_t n_in, const ht_trunc_opts* opts);
/* also returns the number of launches of the merged plan (n_launches may be NULL) */
ht_status ht_debug_validate_truncate_batched(int32_t count, const ht_desc* X, const int32_t* n_in,
                                             const ht_trunc_opts* opts, int32_t* n_launches);
/* Builds the launch plan of ht_truncate twice for the same arguments (fake
 * addresses) and reports whether the two plan-cache keys are byte-identical
 * (*equal = 1), as they must be for a repeated call to reuse its uploaded
 * launch tables; *hash (may be NULL) is a 64-bit FNV-1a hash of the key. */
ht_status ht_debug_plan_key_repeats(const ht_desc* X, int32_t n_in, const ht_trunc_opts* opts, int32_t* equal,
                                    uint64_t* hash);
ht_status ht_debug_validate_orthogonalize(const ht_desc* X, int32_t precision);
ht_status ht_debug_validate_gramians(const ht_desc* X);
ht_status ht_debug_validate_entries(const ht_desc* X, int64_t m);
ht_status ht_debug_validate_inner(const ht_desc* X, const ht_desc* Y);
ht_status ht_debug_validate_norm(const ht_desc* X, int32_t n_in);
ht_status ht_debug_validate_apply(const ht_desc* L, const ht_desc* A);
#ifdef __cplusplus
}
#endif
#endif
