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

// min(floor(num / den), cap) for den > 0, cap < 2^40.
// The binary64 quotient of the two (rounded) operands is within 2^-10 of
// the true quotient whenever it is below cap + 2, so its floor is off by at
// most one; one exact multiply-compare corrects it.  Larger quotients
// saturate at cap: callers only need to know that they reach cap.
HR_HD uint64_t quot_sat(uint64_t num, uint64_t den, uint64_t cap) {
    const double e = (double)num / (double)den;
    if (e > (double)cap + 2.0) return cap;
    uint64_t k = (uint64_t)e;
    const uint64_t lo = k * den;
    if (mulhi64(k, den) != 0 || lo > num) {
        k -= 1;
    } else if (num - lo >= den) {
        k += 1;
    }
    return k < cap ? k : cap;
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
    uint64_t p = a, q;
    uint64_t ip = 1, iq = 0, X = 0, d = b;
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
        r.x = X; r.d = d;
        r.u = 1; r.alpha = a;
        const uint64_t sv = umin(k, n - 1);
        r.v = sv; r.beta = 0 - sv * a;
        r.steps = steps;
        return;
    }
    q = 0 - k * a;   // 2^64 mod a
    iq = k;
    for (;;) {
        ++steps;
        if (p < q) {
            k = quot_sat(q, p, n);
            if (X >= iq) {   // b inside a q-interval: it is split at p, 2p, ..
                const uint64_t s = umin(umin(quot_sat(d, p, n), k), (n - 1 - X) / ip);
                X += s * ip;
                d -= s * p;
            }
            if (ip + iq + k * ip >= n) {
                r.x = X; r.d = d;
                r.u = ip; r.alpha = p;
                const uint64_t sv = umin(k, (n - 1 - iq) / ip);
                r.v = iq + sv * ip; r.beta = q - sv * p;
                r.steps = steps;
                return;
            }
            q -= k * p;
            iq += k * ip;
        } else {
            k = quot_sat(p, q, n);
            if (X < iq) {    // b inside a p-interval: points at p - q, p - 2q, ..
                // the first of them at or left of b: s = ceil((p - d) / q)
                const uint64_t s = quot_sat(p - d - 1, q, n) + 1;
                if (s <= k && X + ip + s * iq < n) {
                    X += ip + s * iq;
                    d -= p - s * q;
                }
            }
            if (ip + iq + k * iq >= n) {
                r.x = X; r.d = d;
                r.v = iq; r.beta = q;
                const uint64_t su = umin(k, (n - 1 - ip) / iq);
                r.u = ip + su * iq; r.alpha = p - su * q;
                r.steps = steps;
                return;
            }
            p -= k * q;
            ip += k * iq;
        }
    }
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

// Degree-1 search of one instance: every k < n with (b - k a) mod 2^64 < D,
// visited by increasing distance (ties, which only occur between repeated
// points, by increasing k); emit(k) is called once per hit.  Returns the
// number of hits.
//
// Degenerate inputs: a = 0 puts every point at 0; when the sequence has a
// period P = 2^(64 - ctz(a)) < n the distinct points are k < P and each
// reappears at k + m P.
template <class Emit>
HR_HD uint64_t search_each(uint64_t a, uint64_t b, uint64_t n, uint64_t D, Emit&& emit,
                           uint32_t* steps = nullptr) {
    if (n == 0 || D == 0) return 0;
    if (a == 0 || n == 1) {
        if (b >= D) return 0;
        const uint64_t c = (a == 0) ? n : 1;
        for (uint64_t k = 0; k < c; ++k) emit(k);
        return c;
    }
    uint64_t P = n;
    const int tz = __builtin_ctzll(a);
    if (tz > 32 && (1ull << (64 - tz)) < n) P = 1ull << (64 - tz);
    Near r;
    closest_left(a, b, P, r);
    if (steps) *steps = r.steps;
    if (r.d >= D) return 0;
    uint64_t x = r.x, dist = r.d, count = 0, visited = 0;
    for (;;) {
        // point x and its repeats x + m P < n share the distance
        for (uint64_t k = x; k < n; k += P) {
            emit(k);
            ++count;
        }
        if (++visited == P) break;
        uint64_t gap;
        pred(r, P, x, gap);
        if (gap >= D - dist) break;
        dist += gap;
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

// acc += x * m mod 2^(32 L), m a 128-bit multiplier given as 4 limbs.
template <int L>
HR_HD void wmac128(Word<L>& acc, const Word<L>& x, const uint32_t m[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
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

// Inverse of an odd number modulo 2^128 (Newton iteration; o * o = 1 mod 8).
HR_HD unsigned __int128 inv_odd128(unsigned __int128 o) {
    unsigned __int128 v = o;
    for (int i = 0; i < 6; ++i) v *= (unsigned __int128)2 - o * v;
    return v;
}

// Binomial C(x, j) as an exact 128-bit integer: the falling factorial
// x (x-1) .. (x-j+1) divided exactly by j! (shift out its power of two,
// multiply by the inverse of its odd part).  Valid while x^j < 2^128.
HR_HD unsigned __int128 binom128(uint64_t x, int j) {
    if (x < (uint64_t)j) return 0;
    unsigned __int128 c = 1;
    uint64_t f = 1;
    for (int i = 0; i < j; ++i) {
        c *= (unsigned __int128)(x - (uint64_t)i);
        f *= (uint64_t)(i + 1);
    }
    const int s = __builtin_ctzll(f);
    return (c >> s) * inv_odd128((unsigned __int128)(f >> s));
}

HR_HD void split128(unsigned __int128 v, uint32_t m[4]) {
    m[0] = (uint32_t)v;
    m[1] = (uint32_t)(v >> 32);
    m[2] = (uint32_t)(v >> 64);
    m[3] = (uint32_t)(v >> 96);
}

}  // namespace hr
