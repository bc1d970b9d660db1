/*
 * pm_testing.h -- test hook of libpm.
 *
 * pm_count_host runs the library's own descriptor, job and finalize code
 * (the code the GPU counter runs per variant) serially on the host, so that
 * the descriptors can be unit-tested on machines without a GPU.  No product
 * path calls it: pm_count, pm_predict and pm_count_device always count on
 * the GPU and fail if no device is present.
 *
 * v: one variant (host).  out: its count vector (host, caller-owned).
 * foot (nullable, host int64[12]): |F| and |Fill| of each of the variant's
 * up to 6 arrays (zero for arrays without a strided access), the footprint
 * and gap-filled footprint of Sec. 3.2, Alg. 2.  Returns PM_EINVAL for an
 * invalid descriptor and PM_EOVERFLOW when a count exceeds int64.
 */
#ifndef PM_TESTING_H
#define PM_TESTING_H
#include "pm.h"

#ifdef __cplusplus
extern "C" {
#endif

pm_status pm_count_host(const pm_variant *v, pm_counts *out, int64_t *foot);

/* The same with the descriptor expanded statement after statement in one
 * pass (compact job slots) instead of statement by statement in two slots
 * each, the layout the GPU's one-thread-per-statement expansion uses; the
 * two must give identical counts. */
pm_status pm_count_host_seq(const pm_variant *v, pm_counts *out, int64_t *foot);

#ifdef __cplusplus
}
#endif
#endif
