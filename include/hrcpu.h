/*
 * hrcpu: a multi-core SIMD (AVX-512) CPU implementation of the degree-1
 * search of hrsearch.h, for comparing the GPU with a CPU program tuned the
 * way the paper's future work proposes (Sec. 7: a regular search written
 * for SIMD CPU units).  Not used by the GPU path.
 *
 * Every pointer is HOST memory.  The library allocates only per-thread
 * working memory and never frees caller memory.  Errors are status codes
 * (HR_OK / HR_EINVAL / HR_ECAPACITY of hrsearch.h, as plain ints).
 */
#ifndef HRCPU_H
#define HRCPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Lanes per vector step of the filter: 8 when the CPU has AVX-512 (F and
 * DQ), 1 when the scalar form runs. */
int hrc_simd_width(void);

/*
 * hrc_filter -- the regular lower-bound test (Alg. 4 of the paper, counter
 * updates as Eq. 3 requires), 8 instances per AVX-512 step: for instance i,
 * with b' = b[i] - lo (window lo and width d shared by `group` consecutive
 * instances), pass[i] = 1 iff the test certifies that no k < N[i] has
 * (b' - k a[i]) mod 2^64 < d; d_out[i] (may be NULL) is the distance value
 * at its exit, iters[i] (may be NULL) its main-loop passes.
 * threads: worker threads (0: all hardware threads).
 * Errors: HR_EINVAL (-1) for group == 0 or a null required pointer.
 */
int hrc_filter(const uint64_t* a, const uint64_t* b, const uint32_t* N, uint64_t n,
               const uint64_t* win_lo, const uint64_t* win_d, uint32_t group, uint8_t* pass,
               uint64_t* d_out, uint32_t* iters, int threads);

/*
 * hrc_search -- every k < N[i] with (b[i] - lo - k a[i]) mod 2^64 < d, as
 * hr_search (same arguments, layout, order of hits and capacity protocol:
 * counts[n], offsets[n] (exclusive scan), hits[cap], hit_inst[cap] or NULL,
 * *total = number of hits, hits beyond cap not written; HR_ECAPACITY (-2)
 * when *total > cap).  Instances the SIMD filter certifies are done; the
 * others take the exact closest-point walk and predecessor steps of the
 * GPU path, one instance per thread step.
 * Errors: HR_EINVAL (-1) for group == 0 or a null required pointer.
 */
int hrc_search(const uint64_t* a, const uint64_t* b, const uint32_t* N, uint64_t n,
               const uint64_t* win_lo, const uint64_t* win_d, uint32_t group, uint32_t* counts,
               uint64_t* offsets, uint32_t* hits, uint32_t* hit_inst, uint64_t cap,
               uint64_t* total, int threads);

#ifdef __cplusplus
}
#endif

#endif /* HRCPU_H */
