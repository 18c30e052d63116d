// Multi-core SIMD CPU form of the degree-1 search (include/hrcpu.h): the
// regular lower-bound test (Alg. 4) on eight instances per AVX-512 step,
// then, for the instances it does not certify, the exact closest-point walk
// and predecessor steps of the GPU path (hr_core.h compiled for the host).
// A CPU program written the way the paper's conclusion proposes (a regular
// search for SIMD CPU units), to compare the GPU with; nothing on the GPU
// path calls it.
#include <immintrin.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

#include "../../include/hrcpu.h"
#include "hr_core.h"

namespace {

constexpr int kOk = 0, kInval = -1, kCapacity = -2;
constexpr uint64_t kChunk = 4096;   // instances per unit of work of a thread

bool have_avx512() {
    static const bool ok = __builtin_cpu_supports("avx512f") && __builtin_cpu_supports("avx512dq");
    return ok;
}

int n_threads(int threads) {
    if (threads > 0) return threads;
    const unsigned h = std::thread::hardware_concurrency();
    return h ? (int)h : 1;
}

// Runs fn(begin, end) over [0, n) in chunks on `threads` threads.
template <class F>
void parallel_chunks(uint64_t n, int threads, F&& fn) {
    const uint64_t chunks = (n + kChunk - 1) / kChunk;
    const int t = (int)std::min<uint64_t>((uint64_t)n_threads(threads), std::max<uint64_t>(chunks, 1));
    std::atomic<uint64_t> next{0};
    auto work = [&]() {
        for (;;) {
            const uint64_t c = next.fetch_add(1);
            if (c >= chunks) return;
            fn(c * kChunk, std::min(n, (c + 1) * kChunk));
        }
    };
    std::vector<std::thread> pool;
    for (int i = 1; i < t; ++i) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
}

// ---------------------------------------------------------------- AVX-512

// Exact quotient and remainder of 64-bit lanes (den > 0).  The binary64
// quotient, lowered by a relative 2^-50, floors to q or q - 1 whenever the
// true quotient is below 2^46 (its rounding errors are far smaller than
// that margin), so num - q den is in [0, 2 den) and one compare finishes
// it.  Lanes with a larger quotient (rare: a length tiny next to the other)
// are divided one at a time.
__attribute__((target("avx512f,avx512dq"))) inline void divmod8(__m512i num, __m512i den,
                                                                __mmask8 m, __m512i* q,
                                                                __m512i* r) {
    const __m512d nf = _mm512_cvtepu64_pd(num);
    const __m512d df = _mm512_cvtepu64_pd(den);
    __m512d qf = _mm512_mul_pd(_mm512_div_pd(nf, df), _mm512_set1_pd(1.0 - 0x1p-50));
    const __mmask8 big = _mm512_mask_cmp_pd_mask(m, qf, _mm512_set1_pd(0x1p46), _CMP_GE_OQ);
    qf = _mm512_min_pd(_mm512_roundscale_pd(qf, _MM_FROUND_TO_NEG_INF | _MM_FROUND_NO_EXC),
                       _mm512_set1_pd(0x1p46));
    __m512i q0 = _mm512_cvttpd_epu64(qf);
    __m512i r0 = _mm512_sub_epi64(num, _mm512_mullo_epi64(q0, den));
    const __mmask8 over = _mm512_cmpge_epu64_mask(r0, den);
    r0 = _mm512_mask_sub_epi64(r0, over, r0, den);
    q0 = _mm512_mask_add_epi64(q0, over, q0, _mm512_set1_epi64(1));
    if (big) {
        alignas(64) uint64_t nn[8], dd[8], qq[8], rr[8];
        _mm512_store_si512(nn, num);
        _mm512_store_si512(dd, den);
        _mm512_store_si512(qq, q0);
        _mm512_store_si512(rr, r0);
        for (int i = 0; i < 8; ++i)
            if (big >> i & 1) {
                qq[i] = nn[i] / dd[i];
                rr[i] = nn[i] % dd[i];
            }
        q0 = _mm512_load_si512(qq);
        r0 = _mm512_load_si512(rr);
    }
    *q = q0;
    *r = r0;
}

// min(c + k c2, n), c2 >= 1 or k < n, lanes below n.
__attribute__((target("avx512f,avx512dq"))) inline __m512i sat_mac8(__m512i c, __m512i k,
                                                                    __m512i c2, __m512i n) {
    const __mmask8 huge = _mm512_cmpge_epu64_mask(k, n) & _mm512_cmpneq_epu64_mask(c2, _mm512_setzero_si512());
    const __m512i v = _mm512_min_epu64(_mm512_add_epi64(c, _mm512_mullo_epi64(k, c2)), n);
    return _mm512_mask_mov_epi64(v, huge, n);
}

// Alg. 4 (as hr::regular_filter) on 8 lanes; lanes outside `valid` are idle.
__attribute__((target("avx512f,avx512dq"))) void regular8(const uint64_t* a, const uint64_t* b,
                                                          const uint64_t* Nn, const uint64_t* D,
                                                          __mmask8 valid, uint8_t* pass,
                                                          uint64_t* d_out, uint32_t* iters) {
    const __m512i zero = _mm512_setzero_si512(), one = _mm512_set1_epi64(1);
    const __m512i n = _mm512_loadu_si512(Nn), thr = _mm512_loadu_si512(D);
    __m512i L0 = _mm512_loadu_si512(a), L1 = zero, C0 = one, C1 = zero;
    __m512i d = _mm512_loadu_si512(b), it = zero;
    __m512i out_d = d, out_it = zero;
    __mmask8 live = valid, ok = 0;
    bool first = true;
    for (;;) {
        // ---- q turn: shorten q (2^64 at first) by p; d mod p
        __mmask8 stop = _mm512_mask_cmpeq_epu64_mask(live, L0, zero);
        ok |= stop & _mm512_cmpge_epu64_mask(d, thr);
        out_d = _mm512_mask_mov_epi64(out_d, stop, d);
        out_it = _mm512_mask_mov_epi64(out_it, stop, it);
        live &= ~stop;
        if (!live) break;
        it = _mm512_mask_add_epi64(it, live, it, one);
        const __m512i p = _mm512_mask_mov_epi64(one, live, L0);    // idle lanes divide by 1
        __m512i k, rem;
        if (first) {
            divmod8(_mm512_set1_epi64(-1), p, live, &k, &rem);
            rem = _mm512_add_epi64(rem, one);                        // 2^64 mod p, or p
            const __mmask8 whole = _mm512_cmpeq_epu64_mask(rem, p);
            k = _mm512_mask_add_epi64(k, whole, k, one);
            rem = _mm512_mask_mov_epi64(rem, whole, zero);
            first = false;
        } else {
            divmod8(L1, p, live, &k, &rem);
        }
        L1 = _mm512_mask_mov_epi64(L1, live, rem);
        C1 = _mm512_mask_mov_epi64(C1, live, sat_mac8(C1, k, C0, n));
        __m512i dq, dr;
        divmod8(d, p, live, &dq, &dr);
        d = _mm512_mask_mov_epi64(d, live, dr);
        stop = _mm512_mask_cmpge_epu64_mask(live, _mm512_add_epi64(C0, C1), n);
        ok |= stop & _mm512_cmpge_epu64_mask(d, thr);
        out_d = _mm512_mask_mov_epi64(out_d, stop, d);
        out_it = _mm512_mask_mov_epi64(out_it, stop, it);
        live &= ~stop;
        // ---- p turn: shorten p by q; b moves on (mod q) only beyond the new p
        stop = _mm512_mask_cmpeq_epu64_mask(live, L1, zero);
        ok |= stop & _mm512_cmpge_epu64_mask(d, thr);
        out_d = _mm512_mask_mov_epi64(out_d, stop, d);
        out_it = _mm512_mask_mov_epi64(out_it, stop, it);
        live &= ~stop;
        if (!live) break;
        const __m512i q = _mm512_mask_mov_epi64(one, live, L1);
        divmod8(L0, q, live, &k, &rem);
        L0 = _mm512_mask_mov_epi64(L0, live, rem);
        C0 = _mm512_mask_mov_epi64(C0, live, sat_mac8(C0, k, C1, n));
        const __mmask8 beyond = live & _mm512_cmpge_epu64_mask(d, L0);
        divmod8(_mm512_sub_epi64(d, L0), q, beyond, &dq, &dr);
        d = _mm512_mask_mov_epi64(d, beyond, dr);
        stop = _mm512_mask_cmpge_epu64_mask(live, _mm512_add_epi64(C0, C1), n);
        ok |= stop & _mm512_cmpge_epu64_mask(d, thr);
        out_d = _mm512_mask_mov_epi64(out_d, stop, d);
        out_it = _mm512_mask_mov_epi64(out_it, stop, it);
        live &= ~stop;
        if (!live) break;
    }
    alignas(64) uint64_t dv[8], iv[8];
    _mm512_store_si512(dv, out_d);
    _mm512_store_si512(iv, out_it);
    for (int i = 0; i < 8; ++i)
        if (valid >> i & 1) {
            pass[i] = ok >> i & 1;
            if (d_out) d_out[i] = dv[i];
            if (iters) iters[i] = (uint32_t)iv[i];
        }
}

// The filter over instances [lo, hi); pass, d_out and iters are indexed by
// instance.
void filter_range(const uint64_t* a, const uint64_t* b, const uint32_t* N, const uint64_t* win_lo,
                  const uint64_t* win_d, uint32_t group, uint64_t lo, uint64_t hi, uint8_t* pass,
                  uint64_t* d_out, uint32_t* iters) {
    const bool simd = have_avx512();
    for (uint64_t i = lo; i < hi; i += 8) {
        const uint32_t m = (uint32_t)std::min<uint64_t>(8, hi - i);
        alignas(64) uint64_t av[8] = {0}, bv[8] = {0}, nv[8] = {0}, dv[8] = {0};
        for (uint32_t j = 0; j < m; ++j) {
            const uint64_t g = (i + j) / group;
            av[j] = a[i + j];
            bv[j] = b[i + j] - (win_lo ? win_lo[g] : 0);
            nv[j] = N[i + j];
            dv[j] = win_d[g];
        }
        if (simd) {
            regular8(av, bv, nv, dv, (__mmask8)((1u << m) - 1), pass + i,
                     d_out ? d_out + i : nullptr, iters ? iters + i : nullptr);
        } else {
            for (uint32_t j = 0; j < m; ++j) {
                const hr::FilterOut r = hr::regular_filter(av[j], bv[j], (uint32_t)nv[j], dv[j]);
                pass[i + j] = r.success;
                if (d_out) d_out[i + j] = r.d;
                if (iters) iters[i + j] = r.iters;
            }
        }
    }
}

}  // namespace

extern "C" {

int hrc_simd_width(void) { return have_avx512() ? 8 : 1; }

int hrc_filter(const uint64_t* a, const uint64_t* b, const uint32_t* N, uint64_t n,
               const uint64_t* win_lo, const uint64_t* win_d, uint32_t group, uint8_t* pass,
               uint64_t* d_out, uint32_t* iters, int threads) {
    if (group == 0 || !win_d) return kInval;
    if (n == 0) return kOk;
    if (!a || !b || !N || !pass) return kInval;
    parallel_chunks(n, threads, [&](uint64_t lo, uint64_t hi) {
        filter_range(a, b, N, win_lo, win_d, group, lo, hi, pass, d_out, iters);
    });
    return kOk;
}

int hrc_search(const uint64_t* a, const uint64_t* b, const uint32_t* N, uint64_t n,
               const uint64_t* win_lo, const uint64_t* win_d, uint32_t group, uint32_t* counts,
               uint64_t* offsets, uint32_t* hits, uint32_t* hit_inst, uint64_t cap,
               uint64_t* total, int threads) {
    if (group == 0 || !win_d || !total) return kInval;
    if (n > 0 && (!a || !b || !N || !counts || !offsets)) return kInval;
    if (cap > 0 && !hits) return kInval;
    *total = 0;
    if (n == 0) return kOk;
    std::vector<uint8_t> pass(n);   // indexed by instance, like the filter's outputs
    parallel_chunks(n, threads, [&](uint64_t lo, uint64_t hi) {
        filter_range(a, b, N, win_lo, win_d, group, lo, hi, pass.data(), nullptr, nullptr);
        for (uint64_t i = lo; i < hi; ++i) {
            uint64_t c = 0;
            if (!pass[i]) {
                const uint64_t g = i / group;
                c = hr::search_each(a[i], b[i] - (win_lo ? win_lo[g] : 0), N[i], win_d[g],
                                    [](uint64_t) {});
            }
            counts[i] = (uint32_t)c;
        }
    });
    uint64_t acc = 0;
    for (uint64_t i = 0; i < n; ++i) {
        offsets[i] = acc;
        acc += counts[i];
    }
    *total = acc;
    parallel_chunks(n, threads, [&](uint64_t lo, uint64_t hi) {
        for (uint64_t i = lo; i < hi; ++i) {
            if (counts[i] == 0 || offsets[i] >= cap) continue;
            const uint64_t g = i / group;
            uint64_t pos = offsets[i];
            hr::search_each(a[i], b[i] - (win_lo ? win_lo[g] : 0), N[i], win_d[g],
                            [&](uint64_t k) {
                                if (pos < cap) {
                                    hits[pos] = (uint32_t)k;
                                    if (hit_inst) hit_inst[pos] = (uint32_t)i;
                                }
                                ++pos;
                            });
        }
    });
    return acc > cap ? kCapacity : kOk;
}

}  // extern "C"
