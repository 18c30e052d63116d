/*
 * hrsearch: hard-to-round (HR) case search on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the hot path of Lefevre's HR-case search as restated by Fortin,
 * Gouicem and Graillat, "GPU-accelerated generation of correctly-rounded
 * elementary functions": the tabulation of fixed-point polynomial pieces
 * (Sec. 5 of the paper) and the degree-1 search of every k with
 * (b - k a) mod 1 below a threshold (Sec. 3.1, Eq. 1; Sec. 4).
 *
 * Conventions shared by every entry point
 *  - Every array argument is a DEVICE pointer on the context's device unless
 *    stated otherwise; `stream` is a hipStream_t (NULL = default stream).
 *    All calls are asynchronous on that stream: outputs are valid after the
 *    stream is synchronised.
 *  - The caller owns every buffer.  The library never frees caller memory;
 *    it allocates only the context's internal scratch (hr_create and,
 *    growing, inside calls that need more).
 *  - Errors are status codes; nothing is thrown across the ABI.  HR_EINVAL is
 *    returned before any launch for invalid sizes or null pointers; device
 *    errors of a launch are returned as HR_EDEVICE.
 *  - Fixed point: a fraction in [0, 1) is stored as an unsigned integer
 *    value * 2^W (W = 64 for a, b and windows).  Arithmetic is mod 1, i.e.
 *    wrap-around.  A W-bit word (W in {128, 192, 256}) is W/64 uint64 limbs,
 *    least significant limb first.
 *  - Identical inputs give identical output bytes (no atomics decide data
 *    placement, except in hr_pipeline whose result set is sorted by the
 *    caller; its order on the device is unspecified).
 *  - One context per host thread; calls on one context are not reentrant.
 *  - A context owns a small fixed device area, allocated by hr_create and
 *    never moved: the work-claim counter of hr_batch_run and the statistics
 *    slots that hr_pipeline and hr_batch_run accumulate into before adding
 *    them to the caller's stats array.  Launches through one context must
 *    therefore not overlap on the device (use one stream per context, or
 *    order the streams); a HIP graph captured from hr_pipeline or
 *    hr_batch_run stays valid while its context lives.  hr_search also uses
 *    a growable scratch area, which a later, larger hr_search on the same
 *    context may move: do not capture hr_search in a graph.
 */
#ifndef HRSEARCH_H
#define HRSEARCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HR_ABI_VERSION 1
#define HR_MAX_DEGREE 6
#define HR_MAX_UPPER_DEGREE 10     /* hr_subtables: degree of a range's polynomial */
#define HR_WAVES_FILL 0xffffffffu   /* hr_batch_run: as many waves as stay resident */

typedef struct hr_ctx hr_ctx;

typedef enum {
    HR_OK = 0,
    HR_EINVAL = -1,      /* invalid argument; nothing launched            */
    HR_ECAPACITY = -2,   /* an output buffer was too small (see callers)  */
    HR_EDEVICE = -3,     /* HIP runtime or launch error                   */
    HR_ENOMEM = -4,      /* device scratch allocation failed              */
    HR_ESCRATCH = -5     /* input larger than hr_search_static's scratch  */
} hr_status;

/* ABI version of the loaded library (HR_ABI_VERSION). */
int hr_abi_version(void);

/* Static text for a status code. */
const char* hr_status_str(int status);

/* Create a context on HIP device `device`.  *out receives the context.
 * Returns HR_EINVAL for a null `out` or a bad device index. */
hr_status hr_create(hr_ctx** out, int device);

/* Release a context and its scratch.  NULL is accepted. */
hr_status hr_destroy(hr_ctx* ctx);

/*
 * hr_search -- degree-1 search (Sec. 3.1 Eq. 1 of the paper, computing the
 * whole set behind the minimum that Alg. 1-4 bound from below).
 *
 * For each instance i < n, with a window start lo and width d shared by the
 * `group` consecutive instances i / group:
 *     hits(i) = { k in [0, N[i]) : (b[i] - lo - k a[i]) mod 2^64 < d }.
 *
 *  a, b        uint64[n]   slope and offset of b - a x (fractions * 2^64)
 *  N           uint32[n]   instance lengths (0 allowed: no hits)
 *  win_lo      uint64[ceil(n/group)] window starts (NULL: all zero)
 *  win_d       uint64[ceil(n/group)] window widths (hit iff distance < d)
 *  group       instances per window entry (>= 1)
 *  counts      uint32[n]   out: number of hits of each instance
 *  offsets     uint64[n]   out: exclusive prefix sum of counts
 *  hits        uint32[cap] out: k values, CSR by instance: the hits of
 *              instance i are hits[offsets[i] .. offsets[i] + counts[i]),
 *              ordered by increasing distance (b - lo - k a) mod 2^64, ties
 *              (repeated points, periodic a) by increasing k.
 *  hit_inst    uint32[cap] out (may be NULL): instance index of each hit
 *  cap         capacity of hits / hit_inst (entries); hits at positions
 *              >= cap are not written
 *  total       uint64[1]   out: total number of hits (may exceed cap: the
 *              caller checks *total <= cap after synchronising and retries
 *              with a larger buffer otherwise)
 * Errors: HR_EINVAL for n > 2^32 - 1, group == 0, or a null required pointer.
 */
hr_status hr_search(hr_ctx* ctx, const uint64_t* a, const uint64_t* b, const uint32_t* N,
                    uint64_t n, const uint64_t* win_lo, const uint64_t* win_d, uint32_t group,
                    uint32_t* counts, uint64_t* offsets, uint32_t* hits, uint32_t* hit_inst,
                    uint64_t cap, uint64_t* total, void* stream);

/*
 * hr_search_static -- hr_search for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same arguments, results and errors, but the block
 * sums live in a fixed device array of the library (HR_STATIC_SCRATCH_BYTES
 * per device, held until the process ends) instead of the context's
 * growable scratch, and the call allocates nothing.
 *  - n is limited to HR_STATIC_MAX_INSTANCES; larger n returns HR_ESCRATCH
 *    before any launch.
 *  - Every call on a device shares that device's array: calls that overlap
 *    on one device (other streams, other contexts, other host threads) race
 *    and give wrong results.  Order them on one stream.
 *  - Nothing in the array needs clearing between calls: every word a call
 *    reads is written earlier in the same call.
 */
#define HR_STATIC_SCRATCH_BYTES (1u << 20)
#define HR_STATIC_MAX_INSTANCES ((uint64_t)((HR_STATIC_SCRATCH_BYTES / 8) - 1) * 256)
hr_status hr_search_static(hr_ctx* ctx, const uint64_t* a, const uint64_t* b,
                           const uint32_t* N, uint64_t n, const uint64_t* win_lo,
                           const uint64_t* win_d, uint32_t group, uint32_t* counts,
                           uint64_t* offsets, uint32_t* hits, uint32_t* hit_inst, uint64_t cap,
                           uint64_t* total, void* stream);

/*
 * hr_tabulate -- tabulation of degree-1 pieces (Sec. 5 of the paper:
 * hierarchical method, straightforward shift for packet starts, tabulated
 * difference shift inside packets).
 *
 * Sub-interval s holds its polynomial as the initial table
 *     T_s[j][l] = Delta_N^l Delta_1^j R_s(0),  j + l <= degree,
 * so that piece i of s has r_j(i) = sum_l T_s[j][l] C(i, l) mod 1 and the
 * piece polynomial P_i(x) = sum_j r_j(i) C(x, j).
 *
 *  table       uint64[n_sub * E * L], E = (degree+1)(degree+2)/2,
 *              L = width_bits/64: entry (j, l) of sub-interval s is the
 *              W-bit word at limbs [(s*E + e(j,l))*L, +L), e(j, l) =
 *              sum_{j'<j} (degree - j' + 1) + l (rows j, then l)
 *  n_sub, degree (1..HR_MAX_DEGREE), tau (pieces per sub-interval, >= 1),
 *  width_bits  in {128, 192, 256}
 *  a_out,b_out uint64[n_sub * tau] out, piece (s, i) at s*tau + i:
 *              b = floor(2^64 frac(r_0(i))), a = floor(2^64 frac(-r_1(i)))
 * Errors: HR_EINVAL for bad width/degree, tau == 0, tau^degree >= 2^128,
 * or null pointers.
 */
hr_status hr_tabulate(hr_ctx* ctx, const uint64_t* table, uint32_t n_sub, uint32_t degree,
                      uint32_t tau, uint32_t width_bits, uint64_t* a_out, uint64_t* b_out,
                      void* stream);

/*
 * hr_recheck -- exact evaluation of candidates (the paper's phase 3 test,
 * Sec. 4.1, applied to the candidates of the degree-1 search).
 *
 * For candidate c, piece inst = cand_inst[c] (sub-interval s = inst / tau,
 * piece i = inst % tau) and argument offset k = cand_k[c]:
 *     V = P_i(k) = sum_j r_j(i) C(k, j) mod 2^W  (table as in hr_tabulate)
 * value_out[c] = floor(V / 2^(W-64)) (top 64 bits) and, with the four
 * thresholds of sub-interval s, thr[4s..4s+3] = (hr_lo, hr_hi, rej_lo, rej_hi):
 *     class_out[c] = 1 if hr_lo <= t <= hr_hi          (HR case for sure)
 *                    0 if rej_lo <= t <= rej_hi        (not an HR case)
 *                    2 otherwise                       (undecided)
 *                    255 if cand_inst[c] >= n_sub * tau  (value_out[c] = 0)
 *  k must satisfy k^degree < 2^128 (checked through max_k).
 * Errors: HR_EINVAL as for hr_tabulate, or max_k^degree >= 2^128.
 */
hr_status hr_recheck(hr_ctx* ctx, const uint64_t* table, uint32_t n_sub, uint32_t degree,
                     uint32_t tau, uint32_t width_bits, const uint32_t* cand_inst,
                     const uint32_t* cand_k, uint64_t n_cand, uint32_t max_k,
                     const uint64_t* thr, uint64_t* value_out, uint8_t* class_out,
                     void* stream);

/* One result of hr_pipeline / hr_batch_run: an argument whose piece value
 * passed the exact test (cls 1) or fell inside the error margin (cls 2, to
 * be decided by the caller at higher precision). */
typedef struct {
    uint32_t job;      /* job id of the work item (0 for hr_pipeline)    */
    uint32_t sub;      /* sub-interval                                  */
    uint32_t piece;    /* piece inside the sub-interval                  */
    uint32_t k;        /* argument offset inside the piece               */
    uint32_t cls;      /* 1 = HR case, 2 = undecided                     */
    uint32_t reserved; /* 0                                              */
    uint64_t value;    /* top 64 bits of P_piece(k) mod 1                */
} hr_result;

/* A batch work item: a range of pieces of one sub-interval.  The pieces of
 * the sub-interval have N arguments each, except piece `last_piece`, which
 * has `last_N` (a partial last piece; last_piece = 0xffffffff if none). */
typedef struct {
    uint64_t table;     /* offset, in uint64 limbs, of the sub-interval's
                           table in the table pool (layout of hr_tabulate) */
    uint64_t win_lo;    /* degree-1 window start (as hr_search's lo)     */
    uint64_t win_d;     /* degree-1 window width                         */
    uint64_t thr[4];    /* hr_lo, hr_hi, rej_lo, rej_hi (as hr_recheck)  */
    uint32_t job;       /* copied into results                           */
    uint32_t sub;       /* copied into results                           */
    uint32_t piece0;    /* first piece of the item                       */
    uint32_t npieces;   /* number of pieces (>= 1)                       */
    uint32_t nu;        /* pieces per lane: npieces <= 64 * nu (lane l of  */
                        /* the item's wave takes pieces l, l + 64, ..)    */
    uint32_t N;         /* arguments per piece                           */
    uint32_t last_piece;
    uint32_t last_N;
} hr_item;

/*
 * hr_pipeline -- fused tabulate + search + recheck of whole sub-intervals in
 * one launch (one pass of the hot path; no (a, b) or candidate lists in HBM).
 *
 * Same table and thresholds as hr_tabulate / hr_recheck.  Every piece of
 * every sub-interval has N arguments.  win[2s], win[2s+1] = (lo, d) is the
 * degree-1 window of sub-interval s: candidates are the k < N with
 * (b - lo - k a) mod 2^64 < d, as in hr_search.  Each candidate is evaluated
 * exactly and classified; results of class 1 and 2 are appended to `out`
 * (capacity cap entries, order unspecified); *count (device) receives their
 * number (may exceed cap).  stats (device, uint64[8], may be NULL) is
 * incremented by: [0] pieces, [1] candidates, [2] results, [3] partial
 * quotients, [4] wave slots spent in the closest-point walk (sum over waves
 * and pieces of the slowest lane's partial quotients times the live lanes;
 * 1 - [3]/[4] is the loop divergence NMDM of the paper's Sec. 2.2);
 * [5] candidates evaluated at full width (the others were rejected exactly
 * from the top 128 bits of their piece's rows); [6..7] reserved.
 * Errors: as hr_tabulate / hr_recheck, N == 0, or N^degree >= 2^128.
 */
hr_status hr_pipeline(hr_ctx* ctx, const uint64_t* table, uint32_t n_sub, uint32_t degree,
                      uint32_t tau, uint32_t width_bits, uint32_t N, const uint64_t* win,
                      const uint64_t* thr, hr_result* out, uint64_t cap, uint64_t* count,
                      uint64_t* stats, void* stream);

/*
 * hr_batch_run -- the fused pass over a list of work items of uneven size
 * (many jobs, functions, binades and piece lengths in one launch).
 *
 *  pool        uint64 table pool; item i's table starts at pool + items[i].table
 *  items       hr_item[n_items] (device)
 *  width_bits, degree: shared by every item of the call (tables of lower
 *              degree or width are padded: zero high-order entries, zero low
 *              limbs, which leaves every result unchanged)
 *  waves       0: one wave per item (grid = n_items);
 *              > 0: persistent: `waves` one-wave workgroups claim items from
 *              a device counter until none is left (every wave exits when the
 *              list is exhausted); HR_WAVES_FILL: as many waves as the device
 *              keeps resident for this width and degree (occupancy per CU
 *              times CUs, queried once), capped at n_items
 *  out, cap, count, stats: as hr_pipeline (results carry the item's job/sub)
 * Piece arguments k must satisfy k^degree < 2^128 and piece indices
 * piece^degree < 2^128 (checked on the host by the caller's planner).
 * Errors: HR_EINVAL for bad width/degree, null pointers, n_items > 2^31;
 * HR_EDEVICE if the occupancy query for HR_WAVES_FILL fails.
 */
hr_status hr_batch_run(hr_ctx* ctx, const uint64_t* pool, const hr_item* items, uint32_t n_items,
                       uint32_t width_bits, uint32_t degree, uint32_t waves, hr_result* out,
                       uint64_t cap, uint64_t* count, uint64_t* stats, void* stream);

/*
 * hr_subtables -- initial tables of sub-intervals made on the device from
 * the upper table of their range: the top two levels of the hierarchical
 * method (Sec. 5.1 of the paper), one level up from hr_tabulate.
 *
 * A range's polynomial U (degree Du, typically 5-10) is given by its upper
 * table U[n][m] = Delta_S^m Delta_1^n U(0), n + m <= Du, with S arguments per
 * sub-interval, so that sub-interval t covers U(t S + y), y in [0, S).  For
 * output table i < n_sub, with t = t_idx[i] (t0 + i when t_idx is NULL) and
 * piece length N = N_per[i] (N when N_per is NULL):
 *   D[n]    = sum_m U[n][m] C(t, m)   mod 1    (straightforward shift, Sec. 5.2:
 *             the step-1 differences Delta_1^n R_t(0) of R_t(y) = U(t S + y))
 *   T[j][l] = Delta_N^l Delta_1^j R_t(0) = sum_s (-1)^(l-s) C(l, s) sum_k C(s N, k) D[j+k]
 *             mod 1, for j + l <= degree (entries of higher order are dropped:
 *             the caller's error budget covers them),
 * computed exactly at upper_width bits, then rounded to the nearest
 * width_bits-bit word (ties upwards) and written in hr_tabulate's table
 * layout at table_out + i E width_bits/64 (E = (degree+1)(degree+2)/2).
 *
 *  upper        uint64[E_u * upper_width/64], E_u = (Du+1)(Du+2)/2, entry
 *               (n, m) at e(n, m) as in hr_tabulate with degree Du
 *  upper_degree Du in 1..HR_MAX_UPPER_DEGREE
 *  upper_width  192, 256, 320, 384 or 448 (>= width_bits)
 *  t_idx, N_per uint32[n_sub] (device, may be NULL: see above)
 *  max_t, max_N bounds on every t and N: max_t^Du < 2^128 and
 *               (degree max_N)^Du < 2^upper_width are checked here; a table
 *               whose t or N exceeds them (or N = 0) is written as zeros
 *  degree, width_bits  of the output tables (degree <= Du, as hr_tabulate)
 *  table_out    uint64[n_sub * E * width_bits/64] out
 * Errors: HR_EINVAL for a parameter outside these ranges or a null pointer.
 */
hr_status hr_subtables(hr_ctx* ctx, const uint64_t* upper, uint32_t upper_degree,
                       uint32_t upper_width, const uint32_t* t_idx, uint32_t t0,
                       const uint32_t* N_per, uint32_t N, uint32_t max_t, uint32_t max_N,
                       uint32_t n_sub, uint32_t degree, uint32_t width_bits, uint64_t* table_out,
                       void* stream);

/*
 * hr_filter -- the paper's Boolean lower-bound tests of the degree-1
 * question (Sec. 4), for comparison with the exact search on the device.
 *
 * For each instance i (arguments as hr_search: window start lo and width d
 * shared by `group` consecutive instances), with b' = b - lo:
 *  alg = HR_FILTER_LEFEVRE: Lefevre's test, Alg. 1 in the swap form of
 *        Alg. 3 (Sec. 4.1, Sec. 4.3.3);
 *  alg = HR_FILTER_REGULAR: the regular test unrolled, Alg. 4 (Sec. 4.2-4.3;
 *        counter updates as Eq. 3 requires),
 * each computing a lower bound of min_{k < N[i]} (b' - k a) mod 2^64.
 *  pass   uint8[n]  out: 1 = certified: no k < N[i] is a hit; 0 = not
 *                   certified (the instance may or may not have hits)
 *  d_out  uint64[n] out (may be NULL): the distance value at the test's exit
 *  iters  uint32[n] out (may be NULL): main-loop passes
 * Errors: HR_EINVAL for an unknown alg, n > 2^32 - 1, group == 0 or a null
 * required pointer.
 */
#define HR_FILTER_LEFEVRE 1
#define HR_FILTER_REGULAR 2
hr_status hr_filter(hr_ctx* ctx, int alg, const uint64_t* a, const uint64_t* b, const uint32_t* N,
                    uint64_t n, const uint64_t* win_lo, const uint64_t* win_d, uint32_t group,
                    uint8_t* pass, uint64_t* d_out, uint32_t* iters, void* stream);

/*
 * hr_search_steps -- diagnostic: steps[i] = number of partial quotients the
 * closest-point walk of hr_search computes for instance i (arguments as
 * hr_search; 0 where N[i] = 0, the window is empty, a = 0 or N[i] = 1).
 * For measuring the search's algorithmic work.  steps: uint32[n] (device).
 * Errors: HR_EINVAL for n > 2^32 - 1, group == 0 or a null pointer.
 */
hr_status hr_search_steps(hr_ctx* ctx, const uint64_t* a, const uint64_t* b, const uint32_t* N,
                          uint64_t n, const uint64_t* win_lo, const uint64_t* win_d,
                          uint32_t group, uint32_t* steps, void* stream);

/*
 * Streamed batched launches (continuous batching at launch granularity).
 *
 * hr_batch_open creates a batch stream on a context: `slots` launch slots
 * (1..1024), each with its own work-claim counter and completion event, and
 * up to four HIP streams of the library's own (default priority) taken in
 * turn, so a launch submitted while others run is queued at once and can
 * start on the device as the running ones release their compute units,
 * without waiting for the host.
 *
 * hr_batch_submit queues one persistent launch of hr_batch_run's kernel
 * (grid: every wave the device keeps resident, at most n_items) over
 * n_items work items (device memory, hr_item layout; tables in `pool`) and
 * returns at once with a ticket (1, 2, ..).  It first clears *count (device)
 * and the slot's claim counter on its stream; results are appended to
 * out[cap] as in hr_batch_run (order unspecified; *count may exceed cap).
 * after_stream (may be NULL): the launch waits for the work already queued
 * on that stream (e.g. the copies or the hr_subtables call that made its
 * tables).  The caller keeps pool, items, out and count alive and unchanged
 * until the ticket has completed.  Statistics are not collected.
 * HR_ECAPACITY: the slot the ticket needs is still running (poll first).
 *
 * hr_batch_poll: *done = the largest ticket t such that every ticket <= t
 * has completed (non-blocking).  hr_batch_wait blocks until `ticket` has
 * completed.  hr_batch_close waits for every launch and frees the batch.
 * A batch belongs to one host thread; its launches share the context's
 * device but not its claim counter or statistics slots.
 * Errors: HR_EINVAL for bad sizes or null pointers, HR_EDEVICE for HIP
 * errors, HR_ENOMEM when open cannot allocate.
 */
typedef struct hr_batch hr_batch;
hr_status hr_batch_open(hr_ctx* ctx, uint32_t slots, hr_batch** out);
hr_status hr_batch_submit(hr_batch* batch, const uint64_t* pool, const hr_item* items,
                          uint32_t n_items, uint32_t width_bits, uint32_t degree, hr_result* out,
                          uint64_t cap, uint64_t* count, void* after_stream, uint64_t* ticket);
hr_status hr_batch_poll(hr_batch* batch, uint64_t* done);
hr_status hr_batch_wait(hr_batch* batch, uint64_t ticket);
hr_status hr_batch_close(hr_batch* batch);

/*
 * hr_quot_check -- diagnostic: the partial-quotient routine of the search,
 * out[i] = min(floor(num[i] / den[i]), cap) computed by the device code
 * (binary64 reciprocal estimate + exact correction); out[i] = 2^64 - 1 where
 * den[i] = 0.  If rem is non-null, rem[i] = num[i] - out[i] den[i] where
 * out[i] < cap, and 2^64 - 1 elsewhere.  For checking that routine against
 * exact integer division.  All arrays are device memory of n entries.
 * Errors: HR_EINVAL for cap == 0 or cap >= 2^32, or null num/den/out.
 */
hr_status hr_quot_check(hr_ctx* ctx, const uint64_t* num, const uint64_t* den, uint64_t cap,
                        uint64_t* out, uint64_t* rem, uint64_t n, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HRSEARCH_H */
