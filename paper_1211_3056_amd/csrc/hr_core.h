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

// Quotient estimate num/den in binary64 with relative error below 2^-50:
// on the device one reciprocal (v_rcp_f64) refined by one Newton step, on
// the host an IEEE division.
HR_HD double fdiv_est(double num, double den) {
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(den);
    const double e = __builtin_fma(-den, r, 1.0);
    r = __builtin_fma(r, e, r);
    return num * r;
#else
    return num / den;
#endif
}

// min(floor(num / den), cap) for den > 0, cap < 2^32.
// The binary64 estimate of the quotient of the (rounded) operands is within
// 2^-10 of the true quotient whenever it is below cap + 2, so its floor is
// off by at most one; one exact multiply-compare corrects it.  Larger
// quotients saturate at cap: callers only need to know that they reach cap.
HR_HD uint64_t quot_sat(uint64_t num, uint64_t den, uint64_t cap) {
    const double e = fdiv_est((double)num, (double)den);
    const bool big = e > (double)cap + 2.0;
    uint32_t k = (uint32_t)__builtin_fmin(e, 4294967295.0);
    // k * den as a 96-bit product: lo (64 bits) and whether bits >= 64 are set
    const uint64_t t1 = (uint64_t)k * (uint32_t)den;
    const uint64_t t2 = (uint64_t)k * (uint32_t)(den >> 32) + (t1 >> 32);
    const uint64_t lo = (t2 << 32) | (uint32_t)t1;
    const bool over = (t2 >> 32) != 0 || lo > num;
    const bool under = !over && num - lo >= den;
    const uint64_t kk = (uint64_t)k - over + under;
    return (big || kk >= cap) ? cap : kk;
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
    uint64_t x;      // index of the closest point on the left of b
    uint64_t d;      // its distance (b - x a) mod 2^64
    uint64_t u;      // index in [1, n) of the point closest to 0 on the right
    uint64_t v;      // index in [1, n) of the point closest to 0 on the left
    uint64_t alpha;  // u a mod 2^64      (gap right of each point)
    uint64_t beta;   // -v a mod 2^64     (gap left of each point)
    uint32_t steps;  // partial quotients computed
};

HR_HD void closest_left(uint64_t a, uint64_t b, uint64_t n, Near& r) {
    uint64_t p = a, q = 0;
    uint64_t ip = 1, iq = 0, X = 0, d = b;
    uint64_t u, v, alpha, beta;
    uint32_t steps = 1;
    // First quotient: q is 1 (2^64), which does not fit; floor(2^64 / a) is
    // floor((2^64 - 1) / a) plus one when a divides 2^64.
    uint64_t k = quot_sat(~0ull, a, n);
    if (k < n && (~0ull - k * a) == a - 1) k += 1;
    {
        // b sits in the single interval [0, 1) whose left end has index 0
        const uint64_t s = umin(umin(quot_sat(d, a, n), k), n - 1);
        X = s;
        d -= s * a;
    }
    if (1 + k >= n) {
        u = 1;
        alpha = a;
        v = umin(k, n - 1);
        beta = 0 - v * a;
    } else {
        q = 0 - k * a;   // 2^64 mod a < a: the lengths now alternate, p > q first
        iq = k;
        // Each pass reduces p by q, then q by p (two partial quotients, as in
        // the paper's unrolled Alg. 4: which length shrinks alternates, so no
        // test on it is needed).  Where b sits is a select, not a branch.
        for (;;) {
            // ---- p > q: p-intervals (left ends < iq) get points at p - q, p - 2q, ..
            ++steps;
            k = quot_sat(p, q, n);
            {
                const bool in_p = X < iq;
                // the first new point at or left of b: s = ceil((p - d) / q)
                const uint64_t s = quot_sat(in_p ? p - d - 1 : 0, q, n) + 1;
                const bool take = in_p && s <= k && X + ip + s * iq < n;
                X = take ? X + ip + s * iq : X;
                d = take ? d - (p - s * q) : d;
            }
            if (ip + iq + k * iq >= n) {
                const uint64_t su = umin(k, idx_div(n - 1 - ip, iq));
                v = iq;
                beta = q;
                u = ip + su * iq;
                alpha = p - su * q;
                break;
            }
            p -= k * q;
            ip += k * iq;
            // ---- q > p: q-intervals (left ends >= iq) get points at p, 2p, ..
            ++steps;
            k = quot_sat(q, p, n);
            {
                const bool in_q = X >= iq;
                uint64_t s = in_q ? umin(quot_sat(d, p, n), k) : 0;
                // only points with index < n exist (matters in the last step)
                if (X + s * ip > n - 1) s = idx_div(n - 1 - X, ip);
                X += s * ip;
                d -= s * p;
            }
            if (ip + iq + k * ip >= n) {
                const uint64_t sv = umin(k, idx_div(n - 1 - iq, ip));
                u = ip;
                alpha = p;
                v = iq + sv * ip;
                beta = q - sv * p;
                break;
            }
            q -= k * p;
            iq += k * ip;
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
HR_HD void pred(const Near& r, uint64_t n, uint64_t& x, uint64_t& gap) {
    if (x >= r.u) {
        x -= r.u;
        gap = r.alpha;
    } else if (x + r.v < n) {
        x += r.v;
        gap = r.beta;
    } else {
        x = x - r.u + r.v;
        gap = r.alpha + r.beta;
    }
}

// Resumable enumeration of the hits of one instance: every k < n with
// (b - k a) mod 2^64 < D, produced by increasing distance (ties, which only
// occur between repeated points, by increasing k).
//
// Degenerate inputs: a = 0 puts every point at 0 and n = 1 has one point
// (P = 1 distinct point); when the sequence has a period
// P = 2^(64 - ctz(a)) < n the distinct points are k < P and each reappears
// at k + m P.
struct HitIter {
    Near r;
    uint64_t n, P, D;
    uint64_t x;        // current distinct point
    uint64_t dist;     // its distance
    uint64_t k;        // next repeat of x to report
    uint64_t visited;  // distinct points reported so far
    bool done;
};

HR_HD void iter_init(HitIter& it, uint64_t a, uint64_t b, uint64_t n, uint64_t D,
                     uint32_t* steps = nullptr) {
    it.n = n;
    it.D = D;
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
        if (tz > 32 && (1ull << (64 - tz)) < n) it.P = 1ull << (64 - tz);
        closest_left(a, b, it.P, it.r);
        if (steps) *steps = it.r.steps;
        it.x = it.r.x;
        it.dist = it.r.d;
    }
    it.done = it.dist >= D;
    it.k = it.x;
    it.visited = 1;
}

// Next hit into k; false when there is none left.
HR_HD bool iter_next(HitIter& it, uint64_t& k) {
    if (it.done) return false;
    k = it.k;
    it.k += it.P;
    if (it.k >= it.n) {          // all repeats of x reported: go left
        if (it.visited == it.P) {
            it.done = true;
        } else {
            uint64_t gap;
            pred(it.r, it.P, it.x, gap);
            if (gap >= it.D - it.dist) {
                it.done = true;
            } else {
                it.dist += gap;
                it.k = it.x;
                ++it.visited;
            }
        }
    }
    return true;
}

// Calls emit(k) for every hit, in the order above; returns their number.
template <class Emit>
HR_HD uint64_t search_each(uint64_t a, uint64_t b, uint64_t n, uint64_t D, Emit&& emit,
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
HR_HD uint64_t search_one(uint64_t a, uint64_t b, uint64_t n, uint64_t D,
                          uint32_t* out, uint64_t cap) {
    uint64_t m = 0;
    return search_each(a, b, n, D, [&](uint64_t k) {
        if (out && m < cap) out[m] = (uint32_t)k;
        ++m;
    });
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

// Binomials C(x, 1..J) as exact 128-bit integers, incrementally:
// C(x, j) = C(x, j-1) (x - j + 1) / j, the division being exact (by 2 and 4
// a shift, by 3, 5 and 6 a multiplication by the inverse of the odd part
// modulo 2^128).  Valid while x^J < 2^128.
HR_HD void binoms128(uint64_t x, int J, unsigned __int128* c) {
    // inverses of 3, 5, 15 and 45 modulo 2^128
    const unsigned __int128 inv3 = ((unsigned __int128)0xaaaaaaaaaaaaaaaaull << 64) | 0xaaaaaaaaaaaaaaabull;
    const unsigned __int128 inv5 = ((unsigned __int128)0xccccccccccccccccull << 64) | 0xcccccccccccccccdull;
    unsigned __int128 v = x;
    c[0] = v;                                        // C(x, 1)
    for (int j = 2; j <= J; ++j) {
        if (x + 1 < (uint64_t)j) { c[j - 1] = 0; continue; }
        v = v * (unsigned __int128)(x - (uint64_t)(j - 1));
        // v = x (x-1) .. (x-j+1) / (j-1)!  ->  divide by j
        if (j == 2) v >>= 1;
        else if (j == 3) v *= inv3;
        else if (j == 4) v >>= 2;
        else if (j == 5) v *= inv5;
        else if (j == 6) { v >>= 1; v *= inv3; }
        c[j - 1] = v;
    }
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
