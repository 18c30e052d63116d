// Core arithmetic of the HR-case search, shared by every kernel of the
// library.  All functions are __host__ __device__ so that the exact same
// code can be exercised on the CPU.
//
// Fixed point: a value in [0, 1) is a W-bit word (value * 2^W); mod-1
// arithmetic is plain wrap-around integer arithmetic.  On the search side
// W = 64 (a, b, distances are uint64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define HR_HD __host__ __device__ __forceinline__

namespace hr {

// ----------------------------------------------------------------------
// 64-bit helpers

HR_HD uint64_t mulhi64(uint64_t a, uint64_t b) {
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

HR_HD uint64_t umin(uint64_t a, uint64_t b) { return a < b ? a : b; }

// Correctly rounded binary64 value of x: both 32-bit halves convert
// exactly, and one fused multiply-add rounds their sum once.  (On the
// device the high half is converted in asm: written in C, the compiler
// turns it back into a 64-bit conversion with an extra add.)
HR_HD double u64_to_f64(uint64_t x) {
    const uint32_t hi = (uint32_t)(x >> 32);
#if defined(__HIP_DEVICE_COMPILE__)
    double h;
    asm("v_cvt_f64_u32 %0, %1" : "=v"(h) : "v"(hi));
#else
    const double h = (double)hi;
#endif
    return __builtin_fma(h, 4294967296.0, (double)(uint32_t)x);
}

// x truncated towards zero and clamped to [0, 2^32 - 1] (x not NaN).  The
// device's conversion instruction clamps by itself; in C an out-of-range
// conversion is undefined, hence the asm there.
HR_HD uint32_t f64_to_u32_sat(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t k;
    asm("v_cvt_u32_f64 %0, %1" : "=v"(k) : "v"(x));
    return k;
#else
    return (uint32_t)__builtin_fmin(__builtin_fmax(x, 0.0), 4294967295.0);
#endif
}

// Reciprocal of a divisor, reused by every quotient with that divisor: on
// the device one v_rcp_f64 refined by one Newton step, on the host an IEEE
// division.  Either way num * r is within a relative 2^-50 of num / den.
struct Recip {
    uint64_t den;
    double r;
};

HR_HD Recip recip(uint64_t den) {
    Recip R;
    R.den = den;
    const double dd = u64_to_f64(den);
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(dd);
    const double e = __builtin_fma(-dd, r, 1.0);
    R.r = __builtin_fma(r, e, r);
#else
    R.r = 1.0 / dd;
#endif
    return R;
}

// min(floor(num / den), cap) for den > 0, cap < 2^32, and the remainder
// num - q den when q < cap (unspecified when q = cap).
// The binary64 estimate e of the quotient of the (rounded) operands is
// within 2^-10 of the true quotient q + f (0 <= f < 1) whenever it is below
// cap + 2.  Lowered by 2^-9, its floor k is therefore q or q - 1, never
// q + 1: k den <= num fits in 64 bits, and one compare of the remainder
// with den (plus one subtraction) finishes the division.  A larger
// estimate makes k (clamped to 2^32 - 1) at least cap, and so the result
// cap: callers only need to know that the quotient reaches cap.
HR_HD uint32_t quot_rem(uint64_t num, const Recip& R, uint32_t cap, uint64_t& rem) {
    const uint64_t den = R.den;
    const uint32_t k = f64_to_u32_sat(__builtin_fma(u64_to_f64(num), R.r, -0x1p-9));
    const uint64_t kd = (uint64_t)k * (uint32_t)den +
                        ((uint64_t)(k * (uint32_t)(den >> 32)) << 32);   // k den, exact
    const uint64_t r0 = num - kd;      // in [0, 2 den)
    const bool under = r0 >= den;      // k = q - 1
    rem = under ? r0 - den : r0;
    const uint64_t kk = (uint64_t)k + under;
    return kk >= cap ? cap : (uint32_t)kk;
}

// floor(num / den) and the remainder for num < 3 den, by compares and
// subtractions only.
HR_HD uint32_t quot_small2(uint64_t num, uint64_t den, uint64_t& rem) {
    const bool s1 = num >= den;
    const uint64_t r1 = num - den;
    const bool s2 = s1 && r1 >= den;
    rem = s2 ? r1 - den : (s1 ? r1 : num);
    return (uint32_t)s1 + (uint32_t)s2;
}

// True when x holds for every active lane of the wave (on the host, for the
// one caller).  Used only to choose between two exact ways of computing the
// same values, so the results never depend on it.
HR_HD bool wave_all(bool x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __ballot(!x) == 0;
#else
    return x;
#endif
}

HR_HD uint32_t quot_sat(uint64_t num, uint64_t den, uint32_t cap) {
    uint64_t rem;
    return quot_rem(num, recip(den), cap, rem);
}

// floor(a / b) for 0 <= a < 2^53, 0 < b < 2^53 (indices): the correctly
// rounded binary64 quotient is never within rounding of the next integer.
HR_HD uint64_t idx_div(uint64_t a, uint64_t b) {
    return (uint64_t)__builtin_floor((double)a / (double)b);
}

// ----------------------------------------------------------------------
// Exact closest-left point of b among the points {k a mod 1 : k < n}.
//
// The point set is grown through the two-length configurations reached by
// the division-based Euclidean algorithm (the (i, 0) configurations of Eq. 3
// in the paper, the sequence the regular search of Alg. 2 walks).  State of a
// configuration with ip + iq points:
//   p  = length of the interval right of 0 (the point with index ip sits at p)
//   q  = length of the interval left of 1 (the point with index iq at 1 - q)
//   iq intervals have length p (their left ends have indices < iq),
//   ip intervals have length q (left ends with indices >= iq).
// The interval of b starts at the point with index X, at distance d.
// Reducing q by k p adds, inside each q-interval, points at distances
// p, 2p, .. kp from its left end (indices + ip, + 2 ip, ..); reducing p by
// k q adds, inside each p-interval, points at distances p - q, p - 2q, ..
// (indices + ip + iq, + ip + 2 iq, ..).  Unlike the lower bound of Alg. 2,
// the last step is cut exactly at n points (a point of index >= n is never
// used), so the result is the exact minimum over k < n, with its index.
//
// Requires a != 0, n >= 2 and all n points distinct (the period
// 2^(64 - ctz(a)) of the sequence is >= n).
struct Near {
    uint32_t x;      // index of the closest point on the left of b
    uint32_t u;      // index in [1, n) of the point closest to 0 on the right
    uint32_t v;      // index in [1, n) of the point closest to 0 on the left
    uint32_t steps;  // partial quotients computed
    uint64_t d;      // distance of x: (b - x a) mod 2^64
    uint64_t alpha;  // u a mod 2^64      (gap right of each point)
    uint64_t beta;   // -v a mod 2^64     (gap left of each point)
};

// n < 2^32.  Indices stay below n, so they are 32-bit; every quotient is
// needed only up to n, so quot_rem saturates there.  A configuration that
// would reach n points is the last one: the cut at n and the final
// neighbours are worked out only there, so the loop body itself has no
// index multiplications beyond the ones that grow ip and iq.
HR_HD void closest_left(uint64_t a, uint64_t b, uint32_t n, Near& r) {
    uint64_t p = a, q = 0, d = b;
    uint32_t ip = 1, iq = 0, X = 0;
    uint32_t u, v;
    uint64_t alpha, beta;
    uint32_t steps = 1;
    // First quotient: q is 1 (2^64), which does not fit; floor(2^64 / a) is
    // floor((2^64 - 1) / a) plus one when a divides 2^64.
    // When every lane's slope is above 1/3 (k <= 2), compares and
    // subtractions give both quotients, as in the loop below.
    uint32_t k;
    uint32_t s0;                       // b's quotient by a (b sits in [0, 1))
    const uint64_t a1 = 0 - a, a2 = a1 - a;   // 2^64 - a, 2^64 - 2a
    const bool k_one = a1 < a;
    if (wave_all(k_one || a2 < a)) {
        k = k_one ? 1u : 2u;
        uint64_t rb;
        s0 = quot_small2(b, a, rb);   // b < 2^64 < 3a
    } else {
        const Recip Ra = recip(a);
        uint64_t rem;
        k = quot_rem(~0ull, Ra, n, rem);
        if (k < n && rem == a - 1) k += 1;
        uint64_t rb;
        s0 = quot_rem(d, Ra, n, rb);
    }
    {
        // b sits in the single interval [0, 1) whose left end has index 0
        const uint32_t s = (uint32_t)umin(umin(s0, k), n - 1);
        X = s;
        d -= (uint64_t)s * a;
    }
    if (1 + (uint64_t)k >= n) {
        u = 1;
        alpha = a;
        v = (uint32_t)umin(k, n - 1);
        beta = 0 - (uint64_t)v * a;
    } else {
        q = 0 - (uint64_t)k * a;   // 2^64 mod a < a: the lengths now alternate, p > q first
        iq = k;
        // Each pass reduces p by q, then q by p (two partial quotients, as in
        // the paper's unrolled Alg. 4: which length shrinks alternates, so no
        // test on it is needed).  Where b sits is a select, not a branch.
        // Both quotients of a half step share one divisor and so one
        // reciprocal, and their remainders are the new length and the new
        // distance of b.
        // A lane leaves the loop at the half step whose configuration would
        // reach n points, with that step's quotients kept; the cut at n and
        // the final neighbours are then worked out after the loop, once for
        // every lane that stopped in a p step and once for those that
        // stopped in a q step (lanes stop at different passes).
        bool q_step = false;       // the stopping step reduced q (else p)
        bool in_x = false;         // b sits in an interval that step splits
        uint32_t sb = 0;           // b's quotient in that step
        uint64_t rb = 0;           // and its remainder
        for (;;) {
            // ---- p > q: p-intervals (left ends < iq) get points at p - q, p - 2q, ..
            ++steps;
            uint64_t rp;
            in_x = X < iq;
            // the first new point at or left of b: s = ceil((p - d) / q)
            // = sb + 1, and b's distance to it is q - 1 - rb
            const uint64_t nb = in_x ? p - d - 1 : 0;   // < p, so sb <= k
            // Partial quotients are mostly 1 or 2, and the lanes of a wave
            // (pieces with nearly equal slopes) share their leading ones:
            // when every lane's quotient is at most 2, subtractions replace
            // the two divisions.
            const uint64_t t1 = p - q, t2 = t1 - q;
            const bool one = t1 < q;
            if (wave_all(one || t2 < q)) {
                k = one ? 1u : 2u;
                rp = one ? t1 : t2;
                sb = quot_small2(nb, q, rb);
            } else {
                const Recip Rq = recip(q);
                k = quot_rem(p, Rq, n, rp);
                sb = quot_rem(nb, Rq, n, rb);
            }
            const uint64_t kiq = (uint64_t)k * iq;
            if (ip + iq + kiq >= n) break;
            const bool take = in_x && sb < k;
            X = take ? X + ip + (sb + 1) * iq : X;
            d = take ? q - 1 - rb : d;
            p = rp;
            ip += (uint32_t)kiq;
            // ---- q > p: q-intervals (left ends >= iq) get points at p, 2p, ..
            ++steps;
            uint64_t rq;
            in_x = X >= iq;
            // b's interval is shorter than q, so sb = floor(d / p) <= k
            const uint64_t nq = in_x ? d : 0;
            const uint64_t u1 = q - p, u2 = u1 - p;
            const bool uone = u1 < p;
            if (wave_all(uone || u2 < p)) {
                k = uone ? 1u : 2u;
                rq = uone ? u1 : u2;
                sb = quot_small2(nq, p, rb);
            } else {
                const Recip Rp = recip(p);
                k = quot_rem(q, Rp, n, rq);
                sb = quot_rem(nq, Rp, n, rb);
            }
            const uint64_t kip = (uint64_t)k * ip;
            if (ip + iq + kip >= n) {
                q_step = true;
                break;
            }
            X += sb * ip;
            d = in_x ? rb : d;
            q = rq;
            iq += (uint32_t)kip;
        }
        // last configuration: only points with index < n exist
        if (!q_step) {
            const uint64_t s = (uint64_t)sb + 1;
            if (in_x && s <= k && X + ip + s * iq < n) {
                X += ip + (uint32_t)(s * iq);
                d = q - 1 - rb;
            }
            const uint32_t su = (uint32_t)umin(k, idx_div(n - 1 - ip, iq));
            v = iq;
            beta = q;
            u = ip + su * iq;
            alpha = p - (uint64_t)su * q;
        } else {
            uint64_t s = sb;
            if (X + s * ip > n - 1) s = idx_div(n - 1 - X, ip);
            X += (uint32_t)(s * ip);
            d -= s * p;
            const uint32_t sv = (uint32_t)umin(k, idx_div(n - 1 - iq, ip));
            u = ip;
            alpha = p;
            v = iq + sv * ip;
            beta = q - (uint64_t)sv * p;
        }
    }
    r.x = X;
    r.d = d;
    r.u = u;
    r.v = v;
    r.alpha = alpha;
    r.beta = beta;
    r.steps = steps;
}

// Next point to the left of point x among the n points (three-distance
// theorem: the gap left of a point is alpha, beta or alpha + beta).
// Selects, not branches: lanes of a wave take different cases.
HR_HD void pred(const Near& r, uint32_t n, uint32_t& x, uint64_t& gap) {
    const bool right = x >= r.u;                    // x - u exists
    const bool left = (uint64_t)x + r.v < n;        // x + v exists
    const uint32_t down = x - r.u;                  // wraps when !right; unused then
    x = right ? down : (left ? x + r.v : down + r.v);
    gap = right ? r.alpha : (left ? r.beta : r.alpha + r.beta);
}

// Resumable enumeration of the hits of one instance: every k < n with
// (b - k a) mod 2^64 < D, produced by increasing distance (ties, which only
// occur between repeated points, by increasing k).  n < 2^32.
//
// Degenerate inputs: a = 0 puts every point at 0 and n = 1 has one point
// (P = 1 distinct point); when the sequence has a period
// P = 2^(64 - ctz(a)) < n the distinct points are k < P and each reappears
// at k + m P.
struct HitIter {
    Near r;
    uint64_t D;
    uint64_t dist;     // distance of the current distinct point
    uint32_t n, P;
    uint32_t x;        // current distinct point
    uint32_t k;        // next repeat of x to report
    uint32_t visited;  // distinct points reported so far
    bool done;
};

HR_HD void iter_init(HitIter& it, uint64_t a, uint64_t b, uint32_t n, uint64_t D,
                     uint32_t* steps = nullptr) {
    it.n = n;
    it.D = D;
    // defined state for every field: iter_next reads them all, also when done
    it.r = Near{0, 1, 1, 0, 0, 0, 0};
    it.P = 1;
    it.x = 0;
    it.k = 0;
    it.dist = 0;
    it.visited = 1;
    it.done = (n == 0 || D == 0);
    if (steps) *steps = 0;
    if (it.done) return;
    if (a == 0 || n == 1) {
        it.P = 1;
        it.x = 0;
        it.dist = b;
    } else {
        it.P = n;
        const int tz = __builtin_ctzll(a);
        if (tz > 32 && (1ull << (64 - tz)) < n) it.P = (uint32_t)(1ull << (64 - tz));
        closest_left(a, b, it.P, it.r);
        if (steps) *steps = it.r.steps;
        it.x = it.r.x;
        it.dist = it.r.d;
    }
    it.done = it.dist >= D;
    it.k = it.x;
    it.visited = 1;
}

// Next hit into k; false when there is none left.  Written with selects:
// the lanes of a wave are at different points of their walks.
HR_HD bool iter_next(HitIter& it, uint64_t& k) {
    const bool has = !it.done;
    k = it.k;
    const bool repeat = it.P < it.n - it.k;     // another repeat of x follows
    uint32_t x = it.x;
    uint64_t gap;
    pred(it.r, it.P, x, gap);                   // otherwise go left
    const bool stop = it.visited == it.P || gap >= it.D - it.dist;
    const bool left = has && !repeat && !stop;
    it.done = it.done || (has && !repeat && stop);
    it.k = (has && repeat) ? it.k + it.P : (left ? x : it.k);
    it.x = left ? x : it.x;
    it.dist = left ? it.dist + gap : it.dist;
    it.visited += left ? 1u : 0u;
    return has;
}

// Calls emit(k) for every hit, in the order above; returns their number.
template <class Emit>
HR_HD uint64_t search_each(uint64_t a, uint64_t b, uint32_t n, uint64_t D, Emit&& emit,
                           uint32_t* steps = nullptr) {
    HitIter it;
    iter_init(it, a, b, n, D, steps);
    uint64_t k, count = 0;
    while (iter_next(it, k)) {
        emit(k);
        ++count;
    }
    return count;
}

// Same, writing the first min(count, cap) hits to out (if non-null).
HR_HD uint64_t search_one(uint64_t a, uint64_t b, uint32_t n, uint64_t D,
                          uint32_t* out, uint64_t cap) {
    uint64_t m = 0;
    return search_each(a, b, n, D, [&](uint64_t k) {
        if (out && m < cap) out[m] = (uint32_t)k;
        ++m;
    });
}

// ----------------------------------------------------------------------
// The paper's lower-bound tests of the degree-1 question (Sec. 4), for
// measuring them against the exact walk: each returns the distance value d
// at which it stopped, the number of main-loop passes, and whether it
// certifies that no k < n has (b - k a) mod 2^64 < D.  Exact 64-bit integer
// arithmetic; counts saturate at n (only "reaches n" matters).

struct FilterOut {
    uint64_t d;
    uint32_t iters;
    bool success;
};

HR_HD uint64_t sat_add_mul(uint64_t c, uint64_t k, uint64_t c2, uint64_t n) {
    // min(c + k c2, n) for c, c2 <= n
    if (c2 != 0 && k >= n) return n;
    const unsigned __int128 v = (unsigned __int128)k * c2 + c;
    return v >= n ? n : (uint64_t)v;
}

// Lefevre's test (Alg. 1, Sec. 4.1) written with the swap of Alg. 3: the
// side that is shortened and the other one are picked by selects instead
// of two mirrored branches.  Lengths start at p = a, q = 1 - a with one
// interval each; d is b's distance to the closest point on its left.  Per
// pass: if d >= p a point lands just left of b (d -= p, Failure once
// d < D) and p is shortened, else q is; the shortened length loses the
// quotient's multiples of the other (counts grow as in Alg. 1), the test
// succeeds once the counts reach n, and one subtraction step follows.  A
// zero length (rational a: the points have become periodic) ends the test
// with d exact.
HR_HD FilterOut lefevre_filter(uint64_t a, uint64_t b, uint32_t n, uint64_t D) {
    FilterOut r{b, 0, false};
    uint64_t L0 = a, L1 = 0 - a, C0 = 1, C1 = 1, d = b;
    if (d < D) return r;
    if (a == 0) {
        r.success = true;
        return r;
    }
    for (;;) {
        ++r.iters;
        const bool p_side = d >= L0;
        d = p_side ? d - L0 : d;
        if (p_side && d < D) {
            r.d = d;
            return r;
        }
        uint64_t x = p_side ? L0 : L1, y = p_side ? L1 : L0;     // x is shortened by y
        uint64_t cx = p_side ? C0 : C1, cy = p_side ? C1 : C0;
        if (y == 0) {
            r.d = d;
            r.success = d >= D;
            return r;
        }
        const uint64_t k = x / y;
        x -= k * y;
        cy = sat_add_mul(cy, k, cx, n);
        if (cx + cy >= n) {
            r.d = d;
            r.success = true;
            return r;
        }
        y -= x;
        cx = cx + cy >= n ? n : cx + cy;
        L0 = p_side ? x : y;
        L1 = p_side ? y : x;
        C0 = p_side ? cx : cy;
        C1 = p_side ? cy : cx;
    }
}

// The regular test unrolled by two partial quotients (Alg. 4, Sec. 4.3, as
// Alg. 2 with the counter updates read as in Eq. 3): from p = a, q = 1 and
// one interval, q then p is shortened by a whole division each pass; d
// follows b's interval (mod p after q shrinks; after p shrinks, (d - p) mod q
// when b lies beyond the new p).  The result is read once the counts reach
// n, or when a length reaches zero.  The first quotient divides 2^64, which
// does not fit: floor(2^64 / a) and 2^64 mod a are formed from 2^64 - 1.
HR_HD FilterOut regular_filter(uint64_t a, uint64_t b, uint32_t n, uint64_t D) {
    FilterOut r{b, 0, false};
    uint64_t L0 = a, L1 = 0, C0 = 1, C1 = 0, d = b;
    bool first = true;                  // L1 stands for 2^64
    bool q_turn = true;
    for (;;) {
        if ((q_turn ? L0 : L1) == 0) {
            r.d = d;
            r.success = d >= D;
            return r;
        }
        r.iters += q_turn ? 1u : 0u;
        if (q_turn) {
            uint64_t k, rem;
            if (first) {
                k = ~0ull / L0;
                rem = ~0ull % L0 + 1;
                if (rem == L0) {
                    ++k;
                    rem = 0;
                }
                first = false;
            } else {
                k = L1 / L0;
                rem = L1 - k * L0;
            }
            L1 = rem;
            C1 = sat_add_mul(C1, k, C0, n);
            d = d % L0;
        } else {
            const uint64_t k = L0 / L1;
            L0 -= k * L1;
            C0 = sat_add_mul(C0, k, C1, n);
            d = d >= L0 ? (d - L0) % L1 : d;
        }
        if (C0 + C1 >= n) {
            r.d = d;
            r.success = d >= D;
            return r;
        }
        q_turn = !q_turn;
    }
}

// ----------------------------------------------------------------------
// Multi-word fixed point: L little-endian 32-bit limbs, value mod 2^(32 L).

template <int L>
struct Word {
    uint32_t w[L];
};

template <int L>
HR_HD void wadd(Word<L>& a, const Word<L>& b) {
    unsigned c = 0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        unsigned co;
        a.w[i] = __builtin_addc(a.w[i], b.w[i], c, &co);
        c = co;
    }
}

template <int L>
HR_HD void wzero(Word<L>& a) {
#pragma unroll
    for (int i = 0; i < L; ++i) a.w[i] = 0;
}

// acc += x * m mod 2^(32 L), m a multiplier of M 32-bit limbs.
template <int L, int M>
HR_HD void wmac_n(Word<L>& acc, const Word<L>& x, const uint32_t* m) {
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if (j >= L) break;
        const uint32_t mj = m[j];
        uint32_t carry = 0;
#pragma unroll
        for (int i = 0; i + j < L; ++i) {
            const uint64_t t = (uint64_t)x.w[i] * mj + acc.w[i + j] + carry;
            acc.w[i + j] = (uint32_t)t;
            carry = (uint32_t)(t >> 32);
        }
    }
}

// acc += x * m mod 2^(32 L), m a 128-bit multiplier given as 4 limbs; the
// high limbs are skipped when they are zero (small binomials).
template <int L>
HR_HD void wmac128(Word<L>& acc, const Word<L>& x, const uint32_t m[4]) {
    if ((m[2] | m[3]) == 0) {
        if (m[1] == 0) wmac_n<L, 1>(acc, x, m);
        else wmac_n<L, 2>(acc, x, m);
    } else if (m[3] == 0) {
        wmac_n<L, 3>(acc, x, m);
    } else {
        wmac_n<L, 4>(acc, x, m);
    }
}

// C(x, j) from c = C(x, j - 1), 1 <= j <= 6, as an exact 128-bit integer:
// C(x, j) = C(x, j-1) (x - j + 1) / j, the division being exact (by 2 and 4
// a shift, by 3, 5 and 6 a multiplication by the inverse of the odd part
// modulo 2^128).  Valid while x^j < 2^128.  For j = x + 1 the factor
// x - j + 1 is zero, so every later step stays zero without a test.
HR_HD unsigned __int128 binom_step(unsigned __int128 c, uint64_t x, int j) {
    // inverses of 3 and 5 modulo 2^128
    const unsigned __int128 inv3 = ((unsigned __int128)0xaaaaaaaaaaaaaaaaull << 64) | 0xaaaaaaaaaaaaaaabull;
    const unsigned __int128 inv5 = ((unsigned __int128)0xccccccccccccccccull << 64) | 0xcccccccccccccccdull;
    if (j == 1) return x;
    unsigned __int128 v = c * (unsigned __int128)(x - (uint64_t)(j - 1));   // = j C(x, j)
    if (j == 2) v >>= 1;
    else if (j == 3) v *= inv3;
    else if (j == 4) v >>= 2;
    else if (j == 5) v *= inv5;
    else if (j == 6) { v >>= 1; v *= inv3; }
    return v;
}

// The same in 64 bits, for x below binom64_limit(J): there j C(x, j) < 2^64
// for every j <= J, so the product before the exact division fits.
HR_HD uint64_t binom_step64(uint64_t c, uint64_t x, int j) {
    const uint64_t inv3 = 0xaaaaaaaaaaaaaaabull, inv5 = 0xcccccccccccccccdull;   // mod 2^64
    if (j == 1) return x;
    uint64_t v = c * (x - (uint64_t)(j - 1));
    if (j == 2) v >>= 1;
    else if (j == 3) v *= inv3;
    else if (j == 4) v >>= 2;
    else if (j == 5) v *= inv5;
    else if (j == 6) v = (v >> 1) * inv3;
    return v;
}

// x(x-1)..(x-J+1) < 2^64 for x < binom64_limit(J), J <= 6.
HR_HD constexpr uint64_t binom64_limit(int J) {
    return J <= 2 ? (1ull << 32) : J == 3 ? (1ull << 21) : J == 4 ? (1ull << 16)
                                 : J == 5 ? (1ull << 12) : (1ull << 10);
}

// Binomials C(x, 1..J), c[j-1] = C(x, j).
HR_HD void binoms128(uint64_t x, int J, unsigned __int128* c) {
    unsigned __int128 v = 1;
    for (int j = 1; j <= J; ++j) c[j - 1] = v = binom_step(v, x, j);
}

HR_HD unsigned __int128 binom128(uint64_t x, int j) {
    if (j == 0) return 1;
    unsigned __int128 c[6];
    binoms128(x, j, c);
    return c[j - 1];
}

HR_HD void split128(unsigned __int128 v, uint32_t m[4]) {
    m[0] = (uint32_t)v;
    m[1] = (uint32_t)(v >> 32);
    m[2] = (uint32_t)(v >> 64);
    m[3] = (uint32_t)(v >> 96);
}

}  // namespace hr
