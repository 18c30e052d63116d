// HIP kernels and C ABI of the HR-case search (gfx950).
//
// Kernels
//   k_search_count / k_scan_blocks / k_search_emit   degree-1 search, CSR out
//   k_subtables                                      sub-interval tables from
//                                                    a range's upper table
//   k_tabulate                                       pieces (a, b)
//   k_recheck                                        exact candidate values
//   k_pipeline                                       fused tabulate+search+recheck
//   k_items                                          the same over work items
//                                                    (batched, persistent)
//   k_zero_u32, k_stats_flush                        counters
//   k_filter                                         the paper's lower-bound
//                                                    tests (Alg. 1/3, Alg. 4)
//   k_search_steps, k_quot_check                     diagnostics
//
// Every kernel maps one lane to one independent unit of work (an instance,
// a set of pieces, a candidate): the search is embarrassingly parallel over
// sub-domains (Sec. 1.2 of the paper).  Nothing here is a dense
// contraction; all arithmetic is 32/64-bit integer VALU work plus binary64
// quotient estimates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>

#include <stdint.h>
#include <stdlib.h>

#include <type_traits>

#include "../../include/hrsearch.h"
#include "hr_core.h"

struct hr_ctx {
    int device;
    void* scratch;          // growable: block sums of hr_search
    size_t scratch_bytes;
    void* fixed;            // allocated once by hr_create, never moved (so a
                            // captured graph may keep pointing at it): the
                            // work-claim counter, then the statistics slots
};

// A stream of batched launches (hr_batch_open .. hr_batch_close): launch
// slots, each with its own claim counter (device) and completion event, and
// a few streams used in turn so that consecutive launches can overlap.
struct hr_batch {
    hr_ctx* ctx;
    uint32_t slots;
    uint32_t nstreams;
    hipStream_t streams[4];
    unsigned int* claims;       // slots counters, 256 bytes apart (device)
    hipEvent_t* done;           // completion event of each slot's launch
    uint64_t* ticket;           // ticket of each slot's last launch (0: never used)
    uint64_t* finished;         // ticket of each slot's last launch known to be over
    uint64_t next_ticket;       // last ticket handed out
    uint64_t done_through;      // every ticket <= this one has completed
};

// Device scratch of hr_search_static: the per-block hit counts of the
// search and their scan (one uint64 per 256-instance block, plus one), in a
// fixed file-scope array instead of memory allocated by the library, for
// callers that cannot allocate.  Each device holds its own copy for the
// life of the process; host code uses only the address that
// hipGetSymbolAddress returns for the current device, never this name.
constexpr uint64_t kStaticScratchWords = 1ull << 17;   // 1 MiB
static __device__ __align__(256) uint64_t scratch[kStaticScratchWords];

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// ---------------------------------------------------------------- scans

__device__ uint64_t wave_incl_scan(uint64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t t = __shfl_xor(v, o, 64);
        v = t > v ? t : v;
    }
    return v;
}

__device__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Exclusive scan over a block of kBlock lanes; *total receives the sum.
__device__ uint64_t block_excl_scan(uint64_t v, uint64_t* total) {
    __shared__ uint64_t wsum[kWaves];
    const uint64_t inc = wave_incl_scan(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) wsum[w] = inc;
    __syncthreads();
    uint64_t base = 0, tot = 0;
#pragma unroll
    for (int j = 0; j < kWaves; ++j) {
        if (j < w) base += wsum[j];
        tot += wsum[j];
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

// ---------------------------------------------------------------- search

__global__ __launch_bounds__(kBlock) void k_search_count(
    const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
    const uint32_t* __restrict__ N, uint64_t n, const uint64_t* __restrict__ lo,
    const uint64_t* __restrict__ d, uint32_t group, uint32_t* __restrict__ counts,
    uint64_t* __restrict__ block_sums) {
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    uint64_t c = 0;
    if (i < n) {
        const uint64_t g = i / group;
        const uint64_t bb = b[i] - (lo ? lo[g] : 0);
        c = hr::search_each(a[i], bb, N[i], d[g], [](uint64_t) {});
        counts[i] = (uint32_t)c;
    }
    uint64_t tot;
    block_excl_scan(c, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// Exclusive scan of nb block sums in place, by one workgroup; total[0] = sum.
__global__ __launch_bounds__(kBlock) void k_scan_blocks(uint64_t* __restrict__ sums, uint64_t nb,
                                                       uint64_t* __restrict__ total) {
    uint64_t carry = 0;
    for (uint64_t base = 0; base < nb; base += kBlock) {
        const uint64_t i = base + threadIdx.x;
        const uint64_t v = i < nb ? sums[i] : 0;
        uint64_t tot;
        const uint64_t ex = block_excl_scan(v, &tot);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) total[0] = carry;
}

__global__ __launch_bounds__(kBlock) void k_search_emit(
    const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
    const uint32_t* __restrict__ N, uint64_t n, const uint64_t* __restrict__ lo,
    const uint64_t* __restrict__ d, uint32_t group, const uint32_t* __restrict__ counts,
    const uint64_t* __restrict__ block_off, uint64_t* __restrict__ offsets,
    uint32_t* __restrict__ hits, uint32_t* __restrict__ hit_inst, uint64_t cap) {
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t c = i < n ? counts[i] : 0;
    uint64_t tot;
    const uint64_t off = block_off[blockIdx.x] + block_excl_scan(c, &tot);
    if (i >= n) return;
    offsets[i] = off;
    if (c == 0 || off >= cap) return;
    const uint64_t g = i / group;
    const uint64_t bb = b[i] - (lo ? lo[g] : 0);
    uint64_t pos = off;
    hr::search_each(a[i], bb, N[i], d[g], [&](uint64_t k) {
        if (pos < cap) {
            hits[pos] = (uint32_t)k;
            if (hit_inst) hit_inst[pos] = (uint32_t)i;
        }
        ++pos;
    });
}

// ---------------------------------------------------------------- words

template <int L>
__device__ __forceinline__ void load_word(const uint64_t* __restrict__ p, hr::Word<L>& w) {
#pragma unroll
    for (int i = 0; i < L / 2; ++i) {
        const uint64_t v = p[i];
        w.w[2 * i] = (uint32_t)v;
        w.w[2 * i + 1] = (uint32_t)(v >> 32);
    }
}

template <int L>
__device__ __forceinline__ uint64_t top64(const hr::Word<L>& w) {
    return ((uint64_t)w.w[L - 1] << 32) | w.w[L - 2];
}

// floor(2^64 frac(-v)) = -ceil(v / 2^(W-64)) mod 2^64
template <int L>
__device__ __forceinline__ uint64_t neg_top64(const hr::Word<L>& w) {
    uint32_t low = 0;
#pragma unroll
    for (int i = 0; i < L - 2; ++i) low |= w.w[i];
    return 0 - (top64(w) + (low != 0));
}

__host__ __device__ constexpr int n_entries(int deg) { return (deg + 1) * (deg + 2) / 2; }
__host__ __device__ constexpr int entry(int deg, int j, int l) {
    return j * (deg + 1) - j * (j - 1) / 2 + l;
}

// Multiplier limbs of C(x, 1..DEG) (c[m-1] = C(x, m)).
template <int DEG>
__device__ __forceinline__ void binom_limbs(uint64_t x, uint32_t (*c)[4]) {
    unsigned __int128 b[DEG];
    hr::binoms128(x, DEG, b);
#pragma unroll
    for (int m = 0; m < DEG; ++m) hr::split128(b[m], c[m]);
}

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Difference vector of row J at piece i0: v[l] = Delta^l r_J(i0) =
// sum_m T[J][l+m] C(i0, m)  (straightforward shift, Sec. 5.2).
template <int L, int DEG, int J>
__device__ __forceinline__ void row_start(const uint64_t* __restrict__ T, const uint32_t (*c)[4],
                                          hr::Word<L>* v) {
#pragma unroll
    for (int l = 0; l <= DEG - J; ++l) {
        load_word<L>(T + (size_t)entry(DEG, J, l) * (L / 2), v[l]);
#pragma unroll
        for (int m = 1; l + m <= DEG - J; ++m) {
            hr::Word<L> t;
            load_word<L>(T + (size_t)entry(DEG, J, l + m) * (L / 2), t);
            hr::wmac128(v[l], t, c[m - 1]);
        }
    }
}

// One tabulated-difference step of a difference vector of length LEN
// (Fig. 7: Delta^l(i+1) = Delta^l(i) + Delta^{l+1}(i)).
template <int L, int LEN>
__device__ __forceinline__ void row_step(hr::Word<L>* v) {
#pragma unroll
    for (int l = 0; l + 1 < LEN; ++l) hr::wadd(v[l], v[l + 1]);
}

// ---------------------------------------------------------------- tabulate

constexpr uint32_t kMaxNu = 16;   // pieces per lane (pick_nu never exceeds it)

// ---------------------------------------------------------------- sub-interval tables

// w *= x mod 2^(32 L) for a 64-bit x.
template <int L>
__device__ __forceinline__ void wmul_u64(hr::Word<L>& w, uint64_t x) {
    hr::Word<L> acc;
    hr::wzero(acc);
    const uint32_t m[2] = {(uint32_t)x, (uint32_t)(x >> 32)};
    hr::wmac_n<L, 2>(acc, w, m);
    w = acc;
}

// w /= k for a w that k divides (k <= 64): long division from the top
// limb.  Each partial dividend c = r 2^32 + limb is below 2^38; its product
// with the binary64 reciprocal of k is within 2^-14 of c / k, whose
// fractional part is a multiple of 1/k, so the floor is the quotient or one
// below it (when c / k is an integer just above the rounded product); one
// compare of the remainder finishes it.
template <int L>
__device__ __forceinline__ void wdiv_exact(hr::Word<L>& w, uint32_t k) {
    const double rk = 1.0 / (double)k;
    uint64_t r = 0;
#pragma unroll
    for (int i = L - 1; i >= 0; --i) {
        const uint64_t c = (r << 32) | w.w[i];
        uint64_t q = (uint64_t)__builtin_floor(hr::u64_to_f64(c) * rk);
        uint64_t rem = c - q * k;
        const bool up = rem >= k;
        q += up;
        rem -= up ? k : 0;
        r = rem;
        w.w[i] = (uint32_t)q;
    }
}

// acc -= x mod 2^(32 L).
template <int L>
__device__ __forceinline__ void wsub(hr::Word<L>& acc, const hr::Word<L>& x) {
    unsigned b = 0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        unsigned bo;
        acc.w[i] = __builtin_subc(acc.w[i], x.w[i], b, &bo);
        b = bo;
    }
}

template <int L>
__device__ __forceinline__ void lds_get(const uint32_t* p, hr::Word<L>& w) {
#pragma unroll
    for (int i = 0; i < L; ++i) w.w[i] = p[i];
}

template <int L>
__device__ __forceinline__ void lds_put(uint32_t* p, const hr::Word<L>& w) {
#pragma unroll
    for (int i = 0; i < L; ++i) p[i] = w.w[i];
}

constexpr int kMaxUpperDegree = HR_MAX_UPPER_DEGREE;
// LDS words (of LU limbs) per wave: every lane group's binomial table
// (deg + 1)(du + 1) words and its D vector (du + 1 words).
constexpr int kSubtabWords = 4 * 66;

// Sub-interval tables made from an upper table U of degree du (steps 1 and
// S, LU 32-bit limbs per word).  A group of G lanes (G = 16, 32 or 64, at
// least the table's entries and deg + du + 2) makes one sub-interval's
// table; with R_t(y) = U(t S + y) and N its piece length:
//   phase 1  lanes s <= deg: the exact integers C(s N, k), k <= du, built
//            one factor at a time, C(y, k) = C(y, k-1) (y - k + 1) / k;
//            lanes deg + 1 + n, n <= du: D[n] = Delta_1^n R_t(0) =
//            sum_m U[n][m] C(t, m) (straightforward shift in the sub-interval
//            index, Sec. 5.2; C(t, m) exact in 128 bits);
//   phase 2  lane k <= du: the l-th differences over s of C(s N, k) in
//            place, A[l][k] = sum_s (-1)^(l-s) C(l, s) C(s N, k), the
//            coefficient of Delta_1^k in Delta_N^l = (E^N - 1)^l;
//   phase 3  lane e < E, entry (j, l): T[j][l] = Delta_N^l Delta_1^j R_t(0)
//            = sum_{k=l}^{du-j} A[l][k] D[j+k] mod 2^(32 LU), rounded to the
//            nearest W-bit word and written.
// Exactness of the integer steps needs (deg N)^du < 2^(32 LU) and
// t^du < 2^128 (checked on the host through max_N and max_t).
template <int LU>
__global__ __launch_bounds__(64) void k_subtables(
    const uint64_t* __restrict__ upper, uint32_t du, const uint32_t* __restrict__ t_idx,
    uint32_t t0, const uint32_t* __restrict__ N_per, uint32_t N0, uint32_t max_t, uint32_t max_N,
    uint32_t n_sub, uint32_t deg, uint32_t wbits, uint32_t G, uint64_t* __restrict__ out) {
    __shared__ uint32_t lds[kSubtabWords * LU];
    constexpr int LW = LU / 2;   // 64-bit limbs of an upper word
    const uint32_t lane = threadIdx.x;
    const uint32_t grp = lane / G, g = lane % G;
    const uint64_t i = (uint64_t)blockIdx.x * (64 / G) + grp;
    const bool valid_i = i < n_sub;
    const uint32_t E = (deg + 1) * (deg + 2) / 2;
    const uint32_t t = valid_i ? (t_idx ? t_idx[i] : t0 + (uint32_t)i) : 0;
    const uint32_t N = valid_i ? (N_per ? N_per[i] : N0) : 1;
    const bool ok = valid_i && t <= max_t && N != 0 && N <= max_N;
    const uint32_t stride_w = (deg + 1) * (du + 1) + du + 1;
    uint32_t* cs = lds + (size_t)grp * stride_w * LU;       // cs[s (du+1) + k]
    uint32_t* Dl = cs + (size_t)(deg + 1) * (du + 1) * LU;  // D[n]
    // phase 1
    if (ok && g <= deg) {
        const uint64_t y = (uint64_t)g * N;
        hr::Word<LU> c;
        hr::wzero(c);
        c.w[0] = 1;
        lds_put<LU>(cs + (size_t)(g * (du + 1)) * LU, c);
        for (uint32_t k = 1; k <= du; ++k) {
            wmul_u64<LU>(c, y - (uint64_t)(k - 1));   // wraps to 0 past y: C(y, k) = 0
            wdiv_exact<LU>(c, k);
            lds_put<LU>(cs + (size_t)(g * (du + 1) + k) * LU, c);
        }
    } else if (ok && g >= deg + 1 && g <= deg + 1 + du) {
        const uint32_t n = g - deg - 1;
        hr::Word<LU> acc;
        load_word<LU>(upper + (size_t)entry(du, n, 0) * LW, acc);
        hr::Word<4> c;             // C(t, m), exact
        hr::wzero(c);
        c.w[0] = 1;
        for (uint32_t m = 1; m + n <= du; ++m) {
            wmul_u64<4>(c, (uint64_t)t - (uint64_t)(m - 1));
            wdiv_exact<4>(c, m);
            hr::Word<LU> u;
            load_word<LU>(upper + (size_t)entry(du, n, m) * LW, u);
            hr::wmac128(acc, u, c.w);
        }
        lds_put<LU>(Dl + (size_t)n * LU, acc);
    }
    __syncthreads();
    // phase 2: in-place forward differences over s, column k = g
    if (ok && g <= du) {
        for (uint32_t r = 1; r <= deg; ++r)
            for (uint32_t s = deg; s >= r; --s) {
                hr::Word<LU> hi, lo;
                lds_get<LU>(cs + (size_t)(s * (du + 1) + g) * LU, hi);
                lds_get<LU>(cs + (size_t)((s - 1) * (du + 1) + g) * LU, lo);
                wsub<LU>(hi, lo);
                lds_put<LU>(cs + (size_t)(s * (du + 1) + g) * LU, hi);
            }
    }
    __syncthreads();
    // phase 3
    if (!valid_i || g >= E) return;
    uint32_t e = g, j = 0;
    while (e > deg - j) {   // entry g of the (j, l) order
        e -= deg - j + 1;
        ++j;
    }
    const uint32_t l = e;
    const uint32_t lw = wbits / 64;
    uint64_t* dst = out + (i * E + g) * lw;
    if (!ok) {
        for (uint32_t w = 0; w < lw; ++w) dst[w] = 0;
        return;
    }
    hr::Word<LU> T;
    hr::wzero(T);
    for (uint32_t k = l; k + j <= du; ++k) {
        hr::Word<LU> a, d;
        lds_get<LU>(cs + (size_t)(l * (du + 1) + k) * LU, a);
        lds_get<LU>(Dl + (size_t)(j + k) * LU, d);
        hr::wmac_n<LU, LU>(T, d, a.w);
    }
    // round to the nearest W-bit word (ties upwards), keep its W bits
    const uint32_t drop = 32 * LU - wbits;   // bits below the kept word
    if (drop > 0) {
        hr::Word<LU> half;
        hr::wzero(half);
#pragma unroll
        for (int w = 0; w < LU; ++w)
            if ((uint32_t)w == (drop - 1) / 32) half.w[w] = 1u << ((drop - 1) % 32);
        hr::wadd(T, half);
    }
    // limb w0 + i of T by selects over the constant indices: a run-time
    // index into T would put the word in scratch memory
    const uint32_t w0 = drop / 32;
#pragma unroll
    for (int w = 0; w < LU / 2; ++w) {
        uint32_t lo = 0, hi = 0;
#pragma unroll
        for (int s = 0; s < LU; ++s) {
            lo = ((uint32_t)s == w0 + 2 * w) ? T.w[s] : lo;
            hi = ((uint32_t)s == w0 + 2 * w + 1) ? T.w[s] : hi;
        }
        if ((uint32_t)w < lw) dst[w] = ((uint64_t)hi << 32) | lo;
    }
}

// ---------------------------------------------------------------- recheck

template <int L>
__device__ __forceinline__ uint8_t classify(uint64_t t, const uint64_t* __restrict__ thr) {
    if (t >= thr[0] && t <= thr[1]) return 1;
    if (t >= thr[2] && t <= thr[3]) return 0;
    return 2;
}

template <int L, int DEG>
__global__ __launch_bounds__(kBlock) void k_recheck(const uint64_t* __restrict__ table,
                                                   uint32_t n_sub, uint32_t tau,
                                                   const uint32_t* __restrict__ cinst,
                                                   const uint32_t* __restrict__ ck, uint64_t n_cand,
                                                   const uint64_t* __restrict__ thr,
                                                   uint64_t* __restrict__ value_out,
                                                   uint8_t* __restrict__ class_out) {
    const uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n_cand) return;
    const uint32_t inst = cinst[c];
    const uint64_t k = ck[c];
    if ((uint64_t)inst >= (uint64_t)n_sub * tau) {   // not a piece of this table
        value_out[c] = 0;
        class_out[c] = 255;
        return;
    }
    const uint64_t sub = inst / tau, i = inst % tau;
    const uint64_t* T = table + sub * n_entries(DEG) * (L / 2);
    uint32_t ci[DEG][4], ck_[DEG][4];
    binom_limbs<DEG>(i, ci);
    binom_limbs<DEG>(k, ck_);
    hr::Word<L> V;
    hr::wzero(V);
#pragma unroll
    for (int j = 0; j <= DEG; ++j) {
        hr::Word<L> r;
        load_word<L>(T + (size_t)entry(DEG, j, 0) * (L / 2), r);
#pragma unroll
        for (int l = 1; l <= DEG - j; ++l) {
            hr::Word<L> t;
            load_word<L>(T + (size_t)entry(DEG, j, l) * (L / 2), t);
            hr::wmac128(r, t, ci[l - 1]);
        }
        if (j == 0) hr::wadd(V, r);
        else hr::wmac128(V, r, ck_[j - 1]);
    }
    const uint64_t t = top64(V);
    value_out[c] = t;
    class_out[c] = classify<L>(t, thr + 4 * sub);
}

// ---------------------------------------------------------------- pipeline

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

constexpr int kQueue = 512;

// Lanes of a fused wave take interleaved pieces: lane l owns pieces
// l, l + kStride, l + 2 kStride, .. of its range, so the 64 lanes of one
// step search 64 adjacent pieces, whose slopes a (and so the partial
// quotients of the walk) nearly agree; consecutive pieces would spread a
// wave over 64 nu of them.
constexpr int kStride = 64;

// Where a queued candidate comes from: result identifiers and thresholds.
struct Origin {
    uint32_t job, sub, piece;
    const uint64_t* thr;
};

// LDS layout of the rows r_0..r_(DEG-1) a lane publishes for the recheck:
// lane-major, one block of DEG L words per lane, so a lane writes and a
// reader reads 16-byte vectors.  The block is padded to a multiple of 4
// words whose quotient by 4 is odd: the 16 lanes of one 128-bit access
// phase then start on 16 distinct 4-bank groups.
__host__ __device__ constexpr int row_stride(int L, int deg) {
    return ((deg * L + 3) / 4) % 2 == 1 ? (deg * L + 3) / 4 * 4 : ((deg * L + 3) / 4 + 1) * 4;
}

// Register layout of the fused pass.  Row j of the difference table at a
// piece is the vector Delta^l r_j, l = 0..DEG-j.  Its top entry
// Delta^(DEG-j) r_j is the leading difference of a polynomial of degree
// DEG - j in the piece index, hence the same for every piece of a
// sub-interval: it is kept once per wave in LDS (s_top), and registers hold
// only the DEG - j lower entries of each row ("low" entries).
__host__ __device__ constexpr int n_low(int deg) { return deg * (deg + 1) / 2; }
__host__ __device__ constexpr int low_entry(int deg, int j, int l) {   // l < deg - j
    return j * deg - j * (j - 1) / 2 + l;
}

// Low entries of row J at piece i0 (straightforward shift, Sec. 5.2).
template <int L, int DEG, int J>
__device__ __forceinline__ void row_start_low(const uint64_t* __restrict__ T,
                                              const uint32_t (*c)[4], hr::Word<L>* v) {
#pragma unroll
    for (int l = 0; l < DEG - J; ++l) {
        load_word<L>(T + (size_t)entry(DEG, J, l) * (L / 2), v[l]);
#pragma unroll
        for (int m = 1; l + m <= DEG - J; ++m) {
            hr::Word<L> t;
            load_word<L>(T + (size_t)entry(DEG, J, l + m) * (L / 2), t);
            hr::wmac128(v[l], t, c[m - 1]);
        }
    }
}

template <int L>
__device__ __forceinline__ void lds_word(const uint32_t* p, hr::Word<L>& w) {
#pragma unroll
    for (int i = 0; i < L; ++i) w.w[i] = p[i];
}

// One tabulated-difference step of the LEN low entries of a row whose top
// entry is top (Fig. 7).
template <int L, int LEN>
__device__ __forceinline__ void row_step_low(hr::Word<L>* v, const uint32_t* top) {
    if constexpr (LEN > 0) {
#pragma unroll
        for (int l = 0; l + 1 < LEN; ++l) hr::wadd(v[l], v[l + 1]);
        hr::Word<L> t;
        lds_word<L>(top, t);
        hr::wadd(v[LEN - 1], t);
    }
}

// Cooperative load of the top entries of one sub-interval's table into
// s_top[j L + w] (limb w of Delta^(DEG-j) r_j).  Whole wave; ends with a
// barrier.
template <int L, int DEG>
__device__ __forceinline__ void load_top(const uint64_t* __restrict__ T, uint32_t* s_top) {
    __syncthreads();   // previous readers of s_top are done
    const int t = threadIdx.x;
    if (t < (DEG + 1) * L) {
        const int j = t / L, w = t % L;
        const uint64_t word = T[(size_t)entry(DEG, j, DEG - j) * (L / 2) + w / 2];
        s_top[t] = (uint32_t)(word >> (32 * (w & 1)));
    }
    __syncthreads();
}

// Top 64 bits of P_i(k) = sum_j r_j C(k, j) mod 1, exactly, for the piece
// whose rows lane src published (r_0..r_(DEG-1) in s_rows, r_DEG = s_top
// row DEG); C(k, j) is built up one j at a time.
template <int L, int DEG>
__device__ __forceinline__ uint64_t piece_value(const uint32_t* s_rows, const uint32_t* s_top,
                                                uint32_t src, uint64_t k) {
    hr::Word<L> V;
#pragma unroll
    for (int w = 0; w < L; ++w) V.w[w] = s_rows[src * row_stride(L, DEG) + w];
    // Degrees up to 3 have 64-bit binomials for k < 2^21; when every lane's
    // do, two-limb multipliers replace the per-lane choice of length.
    if (DEG <= 3 && __ballot(k >= hr::binom64_limit(DEG)) == 0) {
        uint64_t c = 1;
        static_for<1, DEG + 1>([&](auto J) {
            constexpr int j = decltype(J)::value;
            c = hr::binom_step64(c, k, j);
            hr::Word<L> r;
            if constexpr (j < DEG) {
#pragma unroll
                for (int w = 0; w < L; ++w) r.w[w] = s_rows[src * row_stride(L, DEG) + j * L + w];
            } else {
                lds_word<L>(s_top + DEG * L, r);
            }
            const uint32_t m[2] = {(uint32_t)c, (uint32_t)(c >> 32)};
            hr::wmac_n<L, 2>(V, r, m);
        });
        return top64(V);
    }
    unsigned __int128 ck = 1;
    static_for<1, DEG + 1>([&](auto J) {
        constexpr int j = decltype(J)::value;
        ck = hr::binom_step(ck, k, j);
        hr::Word<L> r;
        if constexpr (j < DEG) {
#pragma unroll
            for (int w = 0; w < L; ++w) r.w[w] = s_rows[src * row_stride(L, DEG) + j * L + w];
        } else {
            lds_word<L>(s_top + DEG * L, r);
        }
        uint32_t m[4];
        hr::split128(ck, m);
        hr::wmac128(V, r, m);
    });
    return top64(V);
}

// Cheap exact rejection of a candidate.  With R_j the top 128 bits of r_j,
// V' = sum_j R_j C(k, j) mod 2^128 undershoots the top 128 bits of P_i(k) by
// E in [0, sum_j C(k, j)) units of 2^-128 (each dropped low part is below
// one unit), so the exact top 64 bits t lie in [t', t' + M] with
// t' = V' div 2^64 and M = DEG + 2 + sum_j (C(k, j) div 2^64).  When that
// whole range is inside the reject interval [thr[2], thr[3]] and misses the
// HR interval [thr[0], thr[1]], classify() would return 0 for t: true is
// returned and the full-width evaluation is skipped.  Always false for
// W = 128, where nothing is dropped and the evaluation is as cheap.
template <int L, int DEG>
__device__ __forceinline__ bool top_rejects(const uint32_t* s_rows, const uint32_t* s_top,
                                            uint32_t src, uint64_t k,
                                            const uint64_t* __restrict__ thr) {
    if constexpr (L <= 4) {
        return false;
    } else {
        hr::Word<4> V;
#pragma unroll
        for (int w = 0; w < 4; ++w) V.w[w] = s_rows[src * row_stride(L, DEG) + L - 4 + w];
        uint64_t M = DEG + 2;
        auto top_row = [&](auto J, hr::Word<4>& r) {
            constexpr int j = decltype(J)::value;
            if constexpr (j < DEG) {
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    r.w[w] = s_rows[src * row_stride(L, DEG) + j * L + L - 4 + w];
            } else {
                lds_word<4>(s_top + DEG * L + L - 4, r);
            }
        };
        if (__ballot(k >= hr::binom64_limit(3)) == 0) {
            // every lane's k < 2^21: C(k, j) for j <= 3 in 64 bits (two-limb
            // multipliers), C(k, 4) = C(k, 3) (k - 3) / 4 from a 64 x 32-bit
            // product (below 2^80, three limbs), higher ones in 128 bits;
            // the limb counts are the same for every lane
            uint64_t c = 1;
            unsigned __int128 ck = 0;
            static_for<1, DEG + 1>([&](auto J) {
                constexpr int j = decltype(J)::value;
                hr::Word<4> r;
                top_row(J, r);
                if constexpr (j <= 3) {
                    c = hr::binom_step64(c, k, j);
                    const uint32_t m[2] = {(uint32_t)c, (uint32_t)(c >> 32)};
                    hr::wmac_n<4, 2>(V, r, m);
                } else {
                    if constexpr (j == 4)
                        ck = ((unsigned __int128)c * (uint32_t)(k - 3)) >> 2;
                    else
                        ck = hr::binom_step(ck, k, j);
                    M += (uint64_t)(ck >> 64);
                    uint32_t m[4];
                    hr::split128(ck, m);
                    hr::wmac_n<4, (j == 4 ? 3 : 4)>(V, r, m);
                }
            });
        } else {
            unsigned __int128 ck = 1;
            static_for<1, DEG + 1>([&](auto J) {
                constexpr int j = decltype(J)::value;
                ck = hr::binom_step(ck, k, j);
                M += (uint64_t)(ck >> 64);
                hr::Word<4> r;
                top_row(J, r);
                uint32_t m[4];
                hr::split128(ck, m);
                hr::wmac128(V, r, m);
            });
        }
        const uint64_t t = top64(V);
        const uint64_t hr_lo = thr[0], hr_hi = thr[1], rej_lo = thr[2], rej_hi = thr[3];
        const bool in_rej = t >= rej_lo && rej_hi >= M && t <= rej_hi - M;
        const bool off_hr = t > hr_hi || t + M < hr_lo;   // t + M < 2^64 here (t <= rej_hi - M)
        return in_rej && off_hr;
    }
}

// The per-wave body of the fused pass.  Each lane owns up to nu pieces
// p_begin + kStride s (cnt of them live) of the wave's sub-interval and
// keeps the low entries of their difference table with step kStride in
// registers, advanced by one tabulated-difference step per piece.  For its
// current piece a lane runs the exact degree-1 search; candidates are
// compacted into an LDS queue (ballot + mbcnt) next to the piece rows, and
// all 64 lanes then recheck queued candidates in parallel, so the uneven
// number of candidates per piece does not idle lanes.  origin(src, s) names
// the piece of lane src at step s.  Must be called by the whole wave
// (uniform nu).
template <int L, int DEG, class OriginFn>
__device__ __forceinline__ void fused_wave(
    hr::Word<L>* v, const uint32_t* s_top, bool active, uint32_t cnt, uint32_t nu,
    uint64_t p_begin, uint32_t N, uint32_t last_piece, uint32_t last_N, uint64_t wlo, uint64_t wd,
    uint32_t* s_rows, uint32_t* s_qlane, uint32_t* s_qk, OriginFn&& origin,
    hr_result* __restrict__ out, uint64_t cap, unsigned long long* __restrict__ count,
    uint64_t& n_pieces, uint64_t& n_cand, uint64_t& n_res, uint64_t& n_steps, uint64_t& n_slots,
    uint64_t& n_full) {
    const int lane = threadIdx.x;
    for (uint32_t s = 0; s < nu; ++s) {
        const bool live = active && s < cnt;
        hr::HitIter it;
        hr::iter_init(it, 0, 0, 0, 0);   // every field defined; done (no points)
        uint32_t steps = 0;
        if (live) {
            const uint64_t piece = p_begin + (uint64_t)kStride * s;
            const uint32_t n = (piece == last_piece) ? last_N : N;
            const uint64_t bb = top64(v[low_entry(DEG, 0, 0)]) - wlo;
            uint64_t aa;
            if constexpr (DEG >= 2) {
                aa = neg_top64(v[low_entry(DEG, 1, 0)]);
            } else {
                hr::Word<L> r1;
                lds_word<L>(s_top + L, r1);
                aa = neg_top64(r1);
            }
            hr::iter_init(it, aa, bb, n, wd, &steps);
            ++n_pieces;
            n_steps += steps;
        }
        {   // loop divergence: the wave runs as long as its slowest lane
            const uint32_t wmax = wave_max_u32(steps);
            const uint32_t nlive = (uint32_t)__popcll(__ballot(live));
            if (lane == 0) n_slots += (uint64_t)wmax * nlive;
        }
        if (!it.done) {   // only pieces with candidates publish their rows r_0..r_(DEG-1)
#pragma unroll
            for (int j = 0; j < DEG; ++j)
#pragma unroll
                for (int w = 0; w < L; ++w)
                    s_rows[lane * row_stride(L, DEG) + j * L + w] = v[low_entry(DEG, j, 0)].w[w];
        }
        for (;;) {
            uint32_t qn = 0;
            for (;;) {   // fill: two hits per lane and round while room remains
                uint64_t k1 = 0, k2 = 0;
                const bool h1 = hr::iter_next(it, k1);
                const bool h2 = hr::iter_next(it, k2);   // implies h1
                const uint64_t m1 = __ballot(h1), m2 = __ballot(h2);
                const uint32_t n1 = (uint32_t)__popcll(m1);
                if (h1) {
                    const uint32_t pos = qn + lanes_below(m1);
                    s_qlane[pos] = (uint32_t)lane;
                    s_qk[pos] = (uint32_t)k1;
                }
                if (h2) {
                    const uint32_t pos = qn + n1 + lanes_below(m2);
                    s_qlane[pos] = (uint32_t)lane;
                    s_qk[pos] = (uint32_t)k2;
                }
                qn += n1 + (uint32_t)__popcll(m2);
                if (m2 == 0 || qn + 128 > kQueue) break;
            }
            __syncthreads();
            for (uint32_t e = lane; e < qn; e += 64) {   // drain
                const uint32_t src = s_qlane[e];
                const uint64_t k = s_qk[e];
                const Origin o = origin(src, s);
                uint8_t cls = 0;
                uint64_t t = 0;
                if (!top_rejects<L, DEG>(s_rows, s_top, src, k, o.thr)) {
                    ++n_full;
                    t = piece_value<L, DEG>(s_rows, s_top, src, k);
                    cls = classify<L>(t, o.thr);
                }
                if (cls) {
                    const unsigned long long pos = atomicAdd(count, 1ull);
                    if (pos < cap) {
                        hr_result r;
                        r.job = o.job;
                        r.sub = o.sub;
                        r.piece = o.piece;
                        r.k = (uint32_t)k;
                        r.cls = cls;
                        r.reserved = 0;
                        r.value = t;
                        out[pos] = r;
                    }
                    ++n_res;
                }
                ++n_cand;
            }
            __syncthreads();
            if (__ballot(!it.done) == 0) break;
        }
        static_for<0, DEG>([&](auto J) {
            constexpr int j = decltype(J)::value;
            row_step_low<L, DEG - j>(v + low_entry(DEG, j, 0), s_top + j * L);
        });
    }
}

// Forward differences with step h from those with step 1 (E = 1 + Delta):
// Delta_h^m = (E^h - 1)^m = (sum_{i>=1} C(h, i) Delta^i)^m = sum_k a[m][k]
// Delta^k, for polynomials of degree <= 6.  a[m][m] = h^m; every entry for
// h = 64 is below 2^40.
struct StrideCoef {
    uint64_t a[7][7];
};
__host__ __device__ constexpr StrideCoef stride_coef(uint64_t h) {
    StrideCoef c{};
    uint64_t base[7] = {0, 0, 0, 0, 0, 0, 0};   // C(h, i)
    uint64_t b = 1;
    for (int i = 1; i <= 6; ++i) {
        b = b * (h - (uint64_t)(i - 1)) / (uint64_t)i;
        base[i] = b;
    }
    c.a[0][0] = 1;
    for (int m = 1; m <= 6; ++m)
        for (int k = m; k <= 6; ++k)
            for (int i = 1; i <= k - m + 1; ++i) c.a[m][k] += c.a[m - 1][k - i] * base[i];
    return c;
}
constexpr StrideCoef kStrideCoef = stride_coef(kStride);
static_assert(kStrideCoef.a[1][1] == 64 && kStrideCoef.a[2][2] == 4096, "stride coefficients");

// acc += x * c mod 2^(32 L) for a 64-bit c.
template <int L>
__device__ __forceinline__ void wmac64(hr::Word<L>& acc, const hr::Word<L>& x, uint64_t c) {
    const uint32_t m[2] = {(uint32_t)c, (uint32_t)(c >> 32)};
    hr::wmac_n<L, 2>(acc, x, m);
}

// Row J's low entries with step 1 (v[0..LEN), LEN = DEG - J) and its
// constant top entry (top) -> the same row with step kStride, in place
// (entry m only reads entries >= m).
template <int L, int DEG, int J>
__device__ __forceinline__ void row_to_stride(hr::Word<L>* v, const uint32_t* top) {
    constexpr int LEN = DEG - J;
    if constexpr (LEN > 1) {
        hr::Word<L> t;
        lds_word<L>(top, t);
#pragma unroll
        for (int m = 1; m < LEN; ++m) {
            hr::Word<L> acc;
            hr::wzero(acc);
#pragma unroll
            for (int k = m; k < LEN; ++k) wmac64<L>(acc, v[k], kStrideCoef.a[m][k]);
            wmac64<L>(acc, t, kStrideCoef.a[m][LEN]);
            v[m] = acc;
        }
    }
}

// s_top[j] *= kStride^(DEG - j): the constant top entries with step
// kStride.  Whole wave; ends with a barrier.
template <int L, int DEG>
__device__ __forceinline__ void scale_top(uint32_t* s_top) {
    __syncthreads();
    if (threadIdx.x <= DEG) {
        const int j = threadIdx.x;
        hr::Word<L> t, acc;
        lds_word<L>(s_top + j * L, t);
        hr::wzero(acc);
        wmac64<L>(acc, t, kStrideCoef.a[DEG - j][DEG - j]);
#pragma unroll
        for (int w = 0; w < L; ++w) s_top[j * L + w] = acc.w[w];
    }
    __syncthreads();
}

// Low entries of every row at piece i0 of table T, with step kStride
// (inactive lanes: zero); s_top (loaded by load_top) is rescaled to step
// kStride as well.  Whole wave.
template <int L, int DEG>
__device__ __forceinline__ void start_low(const uint64_t* __restrict__ T, uint64_t i0, bool active,
                                          hr::Word<L>* v, uint32_t* s_top) {
    if (active) {
        uint32_t cb[DEG][4];
        binom_limbs<DEG>(i0, cb);
        static_for<0, DEG>([&](auto J) {
            constexpr int j = decltype(J)::value;
            row_start_low<L, DEG, j>(T, cb, v + low_entry(DEG, j, 0));
            row_to_stride<L, DEG, j>(v + low_entry(DEG, j, 0), s_top + j * L);
        });
    } else {
#pragma unroll
        for (int e = 0; e < n_low(DEG); ++e) hr::wzero(v[e]);
    }
    scale_top<L, DEG>(s_top);
}

// ---------------------------------------------------------------- tabulate

// A whole step-1 difference vector v[0..LEN) of a polynomial of degree
// LEN - 1 -> its differences with step H (H in {16, 32, 64}), in place
// (entry m reads only entries >= m).  Multipliers below 2^32 take one-limb
// products.
constexpr StrideCoef kStrideCoef16 = stride_coef(16);
constexpr StrideCoef kStrideCoef32 = stride_coef(32);
template <int H>
__host__ __device__ constexpr const StrideCoef& stride_table() {
    return H == 16 ? kStrideCoef16 : H == 32 ? kStrideCoef32 : kStrideCoef;
}

template <int L, int LEN, int H>
__device__ __forceinline__ void row_full_to_stride(hr::Word<L>* v) {
    static_for<1, LEN>([&](auto M) {
        constexpr int m = decltype(M)::value;
        hr::Word<L> acc;
        hr::wzero(acc);
        static_for<m, LEN>([&](auto K) {
            constexpr int k = decltype(K)::value;
            constexpr uint64_t c = stride_table<H>().a[m][k];
            if constexpr (c < (1ull << 32)) {
                const uint32_t m1[1] = {(uint32_t)c};
                hr::wmac_n<L, 1>(acc, v[k], m1);
            } else {
                wmac64<L>(acc, v[k], c);
            }
        });
        v[m] = acc;
    });
}

__host__ __device__ constexpr int ilog2(uint64_t h) { return h <= 1 ? 0 : 1 + ilog2(h >> 1); }

// acc = x 2^S mod 2^(32 L).
template <int L, int S>
__device__ __forceinline__ void wshl(hr::Word<L>& acc, const hr::Word<L>& x) {
    constexpr int q = S / 32, r = S % 32;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const uint32_t hi = i - q >= 0 ? x.w[i - q] : 0u;
        const uint32_t lo = i - q - 1 >= 0 ? x.w[i - q - 1] : 0u;
        acc.w[i] = r == 0 ? hi : (hi << r) | (lo >> ((32 - r) & 31));
    }
}

// acc += x c mod 2^(32 L) for a 64-bit c; the high limb is skipped where
// it is zero.
template <int L>
__device__ __forceinline__ void wmac64_skip(hr::Word<L>& acc, const hr::Word<L>& x, uint64_t c) {
    const uint32_t m[2] = {(uint32_t)c, (uint32_t)(c >> 32)};
    if (m[1] == 0) hr::wmac_n<L, 1>(acc, x, m);
    else hr::wmac_n<L, 2>(acc, x, m);
}

// Row J's differences with step H at piece x, in one pass from the
// sub-interval's step-1 differences at piece 0 (v in, v out):
//   Delta_H^m r(x) = sum_{n >= m} c[m][n] Delta^n r(0),
//   c[m][n] = sum_{k=m..n} A[m][k] C(x, n - k),
// the straightforward shift to x (Sec. 5.2) composed with the change of
// step (A = coefficients of (E^H - 1)^m in powers of Delta).  c[m][m] = H^m
// is a shift.  Every c[m][n] is at most C(x + m H, n) (the coefficient of
// Delta^n in E^(x + m H) dominates it term by term), so cb = C(x, 0..DEG)
// in 64 bits and x + DEG H below binom64_limit(DEG) keep every c[m][n],
// and every term of its sum, below 2^64.  Entry m reads entries >= m only,
// so the pass runs in place in increasing m.
template <int L, int DEG, int J, int H>
__device__ __forceinline__ void row_start_stride(const uint64_t* __restrict__ T,
                                                 const uint64_t* cb, hr::Word<L>* v) {
    constexpr int LEN = DEG + 1 - J;
    static_assert((H & (H - 1)) == 0, "step must be a power of two");
#pragma unroll
    for (int l = 0; l < LEN; ++l) load_word<L>(T + (size_t)entry(DEG, J, l) * (L / 2), v[l]);
    static_for<0, LEN>([&](auto M) {
        constexpr int m = decltype(M)::value;
        hr::Word<L> acc;
        wshl<L, m * ilog2(H)>(acc, v[m]);
        static_for<m + 1, LEN>([&](auto N) {
            constexpr int n = decltype(N)::value;
            uint64_t c = 0;
            static_for<m, n + 1>([&](auto K) {
                constexpr int k = decltype(K)::value;
                constexpr uint64_t a = stride_table<H>().a[m][k];
                if constexpr (a != 0) c += a * cb[n - k];
            });
            wmac64_skip<L>(acc, v[n], c);
        });
        v[m] = acc;
    });
}

// w = -w mod 2^(32 L).
template <int L>
__device__ __forceinline__ void wneg(hr::Word<L>& w) {
    uint32_t c = 1;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        uint32_t co;
        w.w[i] = __builtin_addc(~w.w[i], 0u, c, &co);
        c = co;
    }
}

// Lanes of a segment of H lanes take the pieces i0, i0 + H, .., of one
// sub-interval: row J (0 giving b, 1 giving a) is started from the
// sub-interval's table at the lane's first piece (straightforward shift,
// Sec. 5.2), turned into differences with step H, and advanced by one
// tabulated-difference step per piece (Fig. 7).  At every step the H lanes
// hold H consecutive pieces, so each store of a segment is one contiguous,
// line-aligned run of 8 H bytes.  SMALL (every first piece i0 of the launch
// has i0 + DEG H below binom64_limit(DEG)): the start is one composed pass
// with 64-bit multipliers; otherwise the shift takes 128-bit binomials and
// the step change follows as a second pass.
template <int L, int DEG, int J, int H, bool SMALL>
__device__ __forceinline__ void tabulate_row(const uint64_t* __restrict__ T, uint64_t i0,
                                             uint32_t cnt, uint32_t nu,
                                             uint64_t* __restrict__ dst) {
    constexpr int LEN = DEG + 1 - J;
    hr::Word<L> v[LEN];
    if constexpr (SMALL) {
        uint64_t cb[DEG + 1];
        cb[0] = 1;
#pragma unroll
        for (int j = 1; j <= DEG; ++j) cb[j] = hr::binom_step64(cb[j - 1], i0, j);
        row_start_stride<L, DEG, J, H>(T, cb, v);
    } else {
        uint32_t cb[DEG][4];
        binom_limbs<DEG>(i0, cb);
        row_start<L, DEG, J>(T, cb, v);
        row_full_to_stride<L, LEN, H>(v);
    }
    if constexpr (J == 1) {
        // a = floor(2^64 frac(-r_1)) is the top 64 bits of -r_1 mod 2^W, so
        // the negated row is tabulated (the steps are linear).
#pragma unroll
        for (int l = 0; l < LEN; ++l) wneg<L>(v[l]);
    }
    if (hr::wave_all(cnt == nu) && (nu & 3) == 0) {
        // every lane takes nu pieces: a uniform loop, four stores per
        // address computation
        uint64_t* p = dst;
        for (uint32_t s = 0; s < nu; s += 4, p += 4 * H) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                p[H * u] = top64(v[0]);
                row_step<L, LEN>(v);
            }
        }
    } else {
        for (uint32_t s = 0; s < cnt; ++s) {
            dst[(uint64_t)H * s] = top64(v[0]);
            row_step<L, LEN>(v);
        }
    }
}

// Workgroup w of the first half of the grid (one wave each) and workgroup
// w of the second half take the same 64 / H segments, row 0 (b) and row 1
// (a) respectively; a segment is H lanes over H nu consecutive pieces of
// one sub-interval (segs_per_sub segments per sub-interval).  One row per
// wave keeps a wave's registers to one difference vector and doubles the
// waves that hide each other's stores, at no extra packet starts; the
// longer row-0 waves are dispatched first.
template <int L, int DEG, int H, bool SMALL>
__global__ __launch_bounds__(64) void k_tabulate(const uint64_t* __restrict__ table,
                                                 uint32_t n_sub, uint32_t tau, uint32_t nu,
                                                 uint32_t segs_per_sub,
                                                 uint64_t* __restrict__ a_out,
                                                 uint64_t* __restrict__ b_out) {
    const int lane = threadIdx.x;
    const uint32_t half = gridDim.x / 2;   // the grid is even
    const uint32_t row = blockIdx.x >= half;
    const uint64_t seg = (uint64_t)(blockIdx.x - row * half) * (64 / H) + lane / H;
    const uint64_t sub = seg / segs_per_sub;
    if (sub >= n_sub) return;
    const uint64_t i0 = (seg % segs_per_sub) * H * nu + lane % H;
    if (i0 >= tau) return;
    const uint32_t cnt = (uint32_t)hr::umin(nu, (tau - i0 + H - 1) / H);
    const uint64_t* T = table + sub * n_entries(DEG) * (L / 2);
    if (row == 0)
        tabulate_row<L, DEG, 0, H, SMALL>(T, i0, cnt, nu, b_out + sub * tau + i0);
    else
        tabulate_row<L, DEG, 1, H, SMALL>(T, i0, cnt, nu, a_out + sub * tau + i0);
}

// Statistics are summed per wave, then added into one of kStatSlots
// 64-byte slots picked by workgroup index, so that thousands of waves do
// not queue on the same few addresses (atomics on one line are serialised:
// a single line cost up to a fifth of a launch).  k_stats_flush adds the
// slots into the caller's array afterwards and clears them.
constexpr int kStatSlots = 256;
constexpr int kStatFields = 8;

__device__ __forceinline__ void flush_stats(unsigned long long* slots, uint64_t n_pieces,
                                            uint64_t n_cand, uint64_t n_res, uint64_t n_steps,
                                            uint64_t n_slots, uint64_t n_full) {
    if (!slots) return;
    unsigned long long* stats = slots + (blockIdx.x % kStatSlots) * kStatFields;
    n_pieces = wave_sum(n_pieces);
    n_cand = wave_sum(n_cand);
    n_res = wave_sum(n_res);
    n_steps = wave_sum(n_steps);
    n_slots = wave_sum(n_slots);
    n_full = wave_sum(n_full);
    if (threadIdx.x == 0) {
        atomicAdd(stats + 0, (unsigned long long)n_pieces);
        atomicAdd(stats + 1, (unsigned long long)n_cand);
        atomicAdd(stats + 2, (unsigned long long)n_res);
        atomicAdd(stats + 3, (unsigned long long)n_steps);
        atomicAdd(stats + 4, (unsigned long long)n_slots);
        atomicAdd(stats + 5, (unsigned long long)n_full);
    }
}

// Whole sub-intervals of one uniform job (hr_pipeline).  Sub-interval s is
// handled by wps = ceil(tau / (64 nu)) consecutive waves (one workgroup
// each), so every wave works inside one sub-interval: wave b covers pieces
// [w 64 nu, (w + 1) 64 nu) of sub-interval b / wps, w = b mod wps, lane l
// its pieces w 64 nu + l + 64 s.
template <int L, int DEG>
__global__ __launch_bounds__(64) void k_pipeline(
    const uint64_t* __restrict__ table, uint32_t n_sub, uint32_t tau, uint32_t nu, uint32_t wps,
    uint32_t N, const uint64_t* __restrict__ win, const uint64_t* __restrict__ thr,
    hr_result* __restrict__ out, uint64_t cap, unsigned long long* __restrict__ count,
    unsigned long long* __restrict__ stats) {
    __shared__ __align__(16) uint32_t s_rows[64 * row_stride(L, DEG)];   // [lane][j][w], padded rows
    __shared__ uint32_t s_top[(DEG + 1) * L];
    __shared__ uint32_t s_qlane[kQueue];
    __shared__ uint32_t s_qk[kQueue];
    const int lane = threadIdx.x;
    const uint32_t sub = blockIdx.x / wps;                 // < n_sub (grid = n_sub wps)
    const uint64_t base = (uint64_t)(blockIdx.x % wps) * kStride * nu;
    const uint64_t i0 = base + lane;
    const bool active = i0 < tau;
    const uint32_t cnt =
        active ? (uint32_t)hr::umin(nu, (tau - i0 + kStride - 1) / kStride) : 0;
    const uint64_t* T = table + (uint64_t)sub * n_entries(DEG) * (L / 2);
    load_top<L, DEG>(T, s_top);
    hr::Word<L> v[n_low(DEG)];
    start_low<L, DEG>(T, i0, active, v, s_top);
    const uint64_t wlo = win[2 * (uint64_t)sub];
    const uint64_t wd = win[2 * (uint64_t)sub + 1];
    uint64_t n_pieces = 0, n_cand = 0, n_res = 0, n_steps = 0, n_slots = 0, n_full = 0;
    auto origin = [&](uint32_t src, uint32_t s) {
        Origin o;
        o.job = 0;
        o.sub = sub;
        o.piece = (uint32_t)(base + src + (uint64_t)kStride * s);
        o.thr = thr + 4 * (uint64_t)sub;
        return o;
    };
    fused_wave<L, DEG>(v, s_top, active, cnt, nu, i0, N, 0xffffffffu, 0, wlo, wd, s_rows, s_qlane,
                       s_qk, origin, out, cap, count, n_pieces, n_cand, n_res, n_steps, n_slots,
                       n_full);
    flush_stats(stats, n_pieces, n_cand, n_res, n_steps, n_slots, n_full);
}

// Work items of uneven size (hr_batch_run).  An item lies inside one
// sub-interval.  PERSIST: a fixed grid of waves claims items from *next
// until the list is exhausted; otherwise workgroup b processes item b.
template <int L, int DEG, bool PERSIST>
__global__ __launch_bounds__(64) void k_items(
    const uint64_t* __restrict__ pool, const hr_item* __restrict__ items, uint32_t n_items,
    unsigned int* __restrict__ next, hr_result* __restrict__ out, uint64_t cap,
    unsigned long long* __restrict__ count, unsigned long long* __restrict__ stats) {
    __shared__ __align__(16) uint32_t s_rows[64 * row_stride(L, DEG)];
    __shared__ uint32_t s_top[(DEG + 1) * L];
    __shared__ uint32_t s_qlane[kQueue];
    __shared__ uint32_t s_qk[kQueue];
    const int lane = threadIdx.x;
    uint64_t n_pieces = 0, n_cand = 0, n_res = 0, n_steps = 0, n_slots = 0, n_full = 0;
    uint32_t idx;
    if (PERSIST) {
        uint32_t c = 0;
        if (lane == 0) c = atomicAdd(next, 1u);
        idx = __builtin_amdgcn_readfirstlane(c);   // wave-uniform item index
    } else {
        idx = blockIdx.x;
    }
    while (idx < n_items) {
        const hr_item* I = items + idx;
        const uint32_t nu = I->nu;                  // npieces <= 64 nu
        const uint64_t p_begin = (uint64_t)I->piece0 + lane;
        const uint64_t p_end = (uint64_t)I->piece0 + I->npieces;
        const bool active = p_begin < p_end;
        const uint32_t cnt =
            active ? (uint32_t)hr::umin(nu, (p_end - p_begin + kStride - 1) / kStride) : 0;
        const uint64_t* T = pool + I->table;
        load_top<L, DEG>(T, s_top);
        hr::Word<L> v[n_low(DEG)];
        start_low<L, DEG>(T, p_begin, active, v, s_top);
        auto origin = [&](uint32_t src, uint32_t s) {
            Origin o;
            o.job = I->job;
            o.sub = I->sub;
            o.piece = I->piece0 + src + kStride * s;
            o.thr = I->thr;
            return o;
        };
        fused_wave<L, DEG>(v, s_top, active, cnt, nu, p_begin, I->N, I->last_piece, I->last_N,
                           I->win_lo, I->win_d, s_rows, s_qlane, s_qk, origin, out, cap, count,
                           n_pieces, n_cand, n_res, n_steps, n_slots, n_full);
        if (PERSIST) {
            uint32_t c = 0;
            if (lane == 0) c = atomicAdd(next, 1u);
            idx = __builtin_amdgcn_readfirstlane(c);   // wave-uniform item index
        } else {
            idx = n_items;
        }
    }
    flush_stats(stats, n_pieces, n_cand, n_res, n_steps, n_slots, n_full);
}

__global__ void k_zero_u32(unsigned int* p) { *p = 0u; }

// Clears a launch's claim counter and result count (one lane, so a
// captured or streamed sequence holds no memset).
__global__ void k_zero_claim_count(unsigned int* claim, unsigned long long* count) {
    *claim = 0u;
    *count = 0ull;
}

// One wave: stats[f] += sum over slots of slot[f]; the slots are left zero.
// All loads are issued before any reduction, so the kernel costs about one
// memory round trip.
__global__ __launch_bounds__(64) void k_stats_flush(unsigned long long* __restrict__ slots,
                                                   unsigned long long* __restrict__ stats) {
    uint64_t v[kStatFields];
#pragma unroll
    for (int f = 0; f < kStatFields; ++f) v[f] = 0;
#pragma unroll
    for (int i = 0; i < kStatSlots / 64; ++i) {
        unsigned long long* s = slots + (i * 64 + threadIdx.x) * kStatFields;
#pragma unroll
        for (int f = 0; f < kStatFields; ++f) v[f] += s[f];
    }
#pragma unroll
    for (int i = 0; i < kStatSlots / 64; ++i) {
        unsigned long long* s = slots + (i * 64 + threadIdx.x) * kStatFields;
#pragma unroll
        for (int f = 0; f < kStatFields; ++f) s[f] = 0;
    }
#pragma unroll
    for (int f = 0; f < kStatFields; ++f) v[f] = wave_sum(v[f]);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int f = 0; f < kStatFields; ++f)
            if (v[f]) atomicAdd(stats + f, (unsigned long long)v[f]);
    }
}

// The paper's lower-bound tests (Lefevre's with swap, Alg. 1/3; the regular
// one unrolled, Alg. 4) over degree-1 instances, one lane each: pass[i] = 1
// when the test certifies that instance i has no hit, d_out and iters the
// distance value and main-loop passes at its exit.
template <int ALG>
__global__ __launch_bounds__(kBlock) void k_filter(
    const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
    const uint32_t* __restrict__ N, uint64_t n, const uint64_t* __restrict__ lo,
    const uint64_t* __restrict__ d, uint32_t group, uint8_t* __restrict__ pass,
    uint64_t* __restrict__ d_out, uint32_t* __restrict__ iters) {
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint64_t g = i / group;
    const uint64_t bb = b[i] - (lo ? lo[g] : 0);
    const hr::FilterOut r = ALG == HR_FILTER_LEFEVRE ? hr::lefevre_filter(a[i], bb, N[i], d[g])
                                                     : hr::regular_filter(a[i], bb, N[i], d[g]);
    pass[i] = r.success ? 1 : 0;
    if (d_out) d_out[i] = r.d;
    if (iters) iters[i] = r.iters;
}

// Partial quotients of each instance's closest-point walk (the work of the
// search's filter step), for measurement.
__global__ __launch_bounds__(kBlock) void k_search_steps(
    const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
    const uint32_t* __restrict__ N, uint64_t n, const uint64_t* __restrict__ lo,
    const uint64_t* __restrict__ d, uint32_t group, uint32_t* __restrict__ steps) {
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint64_t g = i / group;
    hr::HitIter it;
    uint32_t st = 0;
    hr::iter_init(it, a[i], b[i] - (lo ? lo[g] : 0), N[i], d[g], &st);
    steps[i] = st;
}

__global__ __launch_bounds__(kBlock) void k_quot_check(const uint64_t* __restrict__ num,
                                                      const uint64_t* __restrict__ den,
                                                      uint64_t cap, uint64_t* __restrict__ out,
                                                      uint64_t* __restrict__ rem, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    uint64_t q = ~0ull, r = ~0ull;
    if (den[i]) {
        q = hr::quot_rem(num[i], hr::recip(den[i]), (uint32_t)cap, r);
        if (q >= cap) r = ~0ull;
    }
    out[i] = q;
    if (rem) rem[i] = r;
}

// ---------------------------------------------------------------- host side

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

hr_status launched() {
    return hipGetLastError() == hipSuccess ? HR_OK : HR_EDEVICE;
}

// Layout of the context's fixed device area.
constexpr size_t kClaimOffset = 0;      // uint32 work-claim counter
constexpr size_t kSlotsOffset = 256;    // kStatSlots x kStatFields uint64
constexpr size_t kFixedBytes = kSlotsOffset + kStatSlots * kStatFields * sizeof(uint64_t);

unsigned int* claim_counter(hr_ctx* ctx) {
    return (unsigned int*)((char*)ctx->fixed + kClaimOffset);
}

// Statistics slots of the context when the caller wants statistics, else null.
unsigned long long* stat_slots(hr_ctx* ctx, uint64_t* stats) {
    return stats ? (unsigned long long*)((char*)ctx->fixed + kSlotsOffset) : nullptr;
}

// After a launch that wrote the slots: add them into stats, clear them.
hr_status flush_stat_slots(hr_ctx* ctx, uint64_t* stats, hipStream_t st) {
    if (!stats) return HR_OK;
    k_stats_flush<<<1, 64, 0, st>>>(stat_slots(ctx, stats), (unsigned long long*)stats);
    return launched();
}

// Waves of the persistent batched kernel that one device keeps resident at
// once (occupancy per CU x CUs), queried once per instantiation and device.
template <int L, int DEG>
uint32_t resident_waves(int device) {
    static std::atomic<uint32_t> cache[64];   // zero-initialised (static storage)
    if (device < 0 || device >= 64) return 0;
    uint32_t w = cache[device].load(std::memory_order_relaxed);
    if (w == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_items<L, DEG, true>, 64, 0) !=
                hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) !=
                hipSuccess)
            return 0;
        w = (uint32_t)(per_cu * cus);
        cache[device].store(w, std::memory_order_relaxed);
    }
    return w;
}

// Device address of `scratch` on each device, looked up once per device
// (by hr_create, with that device current) and kept for the process.
std::mutex g_static_mu;
uint64_t* g_static_addr[64];

hr_status static_scratch(int device, uint64_t** out) {
    if (device < 0 || device >= 64) return HR_EINVAL;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_addr[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != device) return HR_EDEVICE;
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HR_EDEVICE;
        g_static_addr[device] = (uint64_t*)p;
    }
    *out = g_static_addr[device];
    return HR_OK;
}

hr_status ensure_scratch(hr_ctx* ctx, size_t bytes) {
    if (ctx->scratch_bytes >= bytes) return HR_OK;
    if (ctx->scratch) {
        if (hipDeviceSynchronize() != hipSuccess) return HR_EDEVICE;
        if (hipFree(ctx->scratch) != hipSuccess) return HR_EDEVICE;
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
    }
    size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
    if (hipMalloc(&ctx->scratch, want) != hipSuccess) {
        ctx->scratch = nullptr;
        return HR_ENOMEM;
    }
    ctx->scratch_bytes = want;
    return HR_OK;
}

// x^deg < 2^128 ?
bool pow_fits128(uint64_t x, uint32_t deg) {
    unsigned __int128 v = 1;
    for (uint32_t i = 0; i < deg; ++i) {
        if (x != 0 && v > (~(unsigned __int128)0) / x) return false;
        v *= x;
    }
    return true;
}

// bit length of x^n (exact, x^n < 2^512)
uint32_t pow_bits(uint64_t x, uint32_t n) {
    uint32_t w[17] = {1};
    for (uint32_t i = 0; i < n; ++i) {
        uint64_t carry = 0;
        for (int k = 0; k < 17; ++k) {
            const unsigned __int128 p = (unsigned __int128)w[k] * x + carry;
            w[k] = (uint32_t)p;
            carry = (uint64_t)(p >> 32);
        }
        if (carry) return 1024;
    }
    for (int k = 16; k >= 0; --k)
        if (w[k]) return 32 * k + 32 - __builtin_clz(w[k]);
    return 0;
}

bool valid_poly(uint32_t degree, uint32_t width_bits) {
    return degree >= 1 && degree <= HR_MAX_DEGREE &&
           (width_bits == 128 || width_bits == 192 || width_bits == 256);
}

// hr_tabulate's segments: H lanes (32) over H nu pieces, nu up to 32 (long
// enough to amortise the packet start, i.e. the straightforward shift and
// the step conversion), lowered while the grid would have fewer than 8
// waves per CU (two waves per pair of segments, one per row).
constexpr uint32_t kTabLanes = 32;
constexpr uint32_t kTabMaxNu = 32;
uint32_t pick_nu_tab(uint64_t n_sub, uint32_t tau) {
    uint32_t nu = kTabMaxNu;
    auto waves = [&](uint32_t v) {
        return n_sub * ((tau + (uint64_t)kTabLanes * v - 1) / ((uint64_t)kTabLanes * v)) /
               (64 / kTabLanes) * 2;
    };
    while (nu > 1 && waves(nu) < 256ull * 8) nu >>= 1;
    return nu;
}

// Packets per lane for the fused pass: long enough to amortise the packet
// start (straightforward shift), short enough to leave >= 4 lanes per CU slot.
uint32_t pick_nu(uint64_t n_sub, uint32_t tau) {
    uint32_t nu = 16;
    while (nu > 1 && (uint64_t)n_sub * ((tau + nu - 1) / nu) < 256ull * 256 * 4) nu >>= 1;
    return nu;
}

#define HR_DISPATCH(WB, DEG, KERNEL_CALL)                               \
    do {                                                                \
        switch ((WB) / 32 * 16 + (DEG)) {                               \
            HR_CASE(4, 1, KERNEL_CALL) HR_CASE(4, 2, KERNEL_CALL)       \
            HR_CASE(4, 3, KERNEL_CALL) HR_CASE(4, 4, KERNEL_CALL)       \
            HR_CASE(4, 5, KERNEL_CALL) HR_CASE(4, 6, KERNEL_CALL)       \
            HR_CASE(6, 1, KERNEL_CALL) HR_CASE(6, 2, KERNEL_CALL)       \
            HR_CASE(6, 3, KERNEL_CALL) HR_CASE(6, 4, KERNEL_CALL)       \
            HR_CASE(6, 5, KERNEL_CALL) HR_CASE(6, 6, KERNEL_CALL)       \
            HR_CASE(8, 1, KERNEL_CALL) HR_CASE(8, 2, KERNEL_CALL)       \
            HR_CASE(8, 3, KERNEL_CALL) HR_CASE(8, 4, KERNEL_CALL)       \
            HR_CASE(8, 5, KERNEL_CALL) HR_CASE(8, 6, KERNEL_CALL)       \
            default: return HR_EINVAL;                                  \
        }                                                               \
    } while (0)
#define HR_CASE(LL, DD, KERNEL_CALL) \
    case LL * 16 + DD: {             \
        constexpr int L_ = LL;       \
        constexpr int D_ = DD;       \
        KERNEL_CALL;                 \
        break;                       \
    }

}  // namespace

extern "C" {

int hr_abi_version(void) { return HR_ABI_VERSION; }

const char* hr_status_str(int s) {
    switch (s) {
        case HR_OK: return "ok";
        case HR_EINVAL: return "invalid argument";
        case HR_ECAPACITY: return "output capacity exceeded";
        case HR_EDEVICE: return "HIP device or launch error";
        case HR_ENOMEM: return "device allocation failed";
        case HR_ESCRATCH: return "input larger than the static scratch allows";
        default: return "unknown status";
    }
}

hr_status hr_create(hr_ctx** out, int device) {
    if (!out) return HR_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return HR_EDEVICE;
    if (device < 0 || device >= n) return HR_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return HR_EDEVICE;
    hr_ctx* c = (hr_ctx*)calloc(1, sizeof(hr_ctx));
    if (!c) return HR_ENOMEM;
    c->device = device;
    uint64_t* st_addr = nullptr;
    if (static_scratch(device, &st_addr) != HR_OK) {
        free(c);
        return HR_EDEVICE;
    }
    if (hipMalloc(&c->fixed, kFixedBytes) != hipSuccess) {
        free(c);
        return HR_ENOMEM;
    }
    if (hipMemset(c->fixed, 0, kFixedBytes) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(c->fixed);
        free(c);
        return HR_EDEVICE;
    }
    *out = c;
    return HR_OK;
}

hr_status hr_destroy(hr_ctx* ctx) {
    if (!ctx) return HR_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->fixed) (void)hipFree(ctx->fixed);
    free(ctx);
    return HR_OK;
}

}  // extern "C"

namespace {

hr_status search_args_ok(hr_ctx* ctx, const uint64_t* a, const uint64_t* b, const uint32_t* N,
                         uint64_t n, const uint64_t* win_d, uint32_t group, uint32_t* counts,
                         uint64_t* offsets, uint32_t* hits, uint64_t cap, uint64_t* total) {
    if (!ctx || !win_d || !total || group == 0) return HR_EINVAL;
    if (n > 0xffffffffull) return HR_EINVAL;
    if (n > 0 && (!a || !b || !N || !counts || !offsets)) return HR_EINVAL;
    if (cap > 0 && !hits) return HR_EINVAL;
    return HR_OK;
}

// The search's three launches, with the block sums in bsum (nb + 1 words).
hr_status search_launch(const uint64_t* a, const uint64_t* b, const uint32_t* N, uint64_t n,
                        const uint64_t* win_lo, const uint64_t* win_d, uint32_t group,
                        uint32_t* counts, uint64_t* offsets, uint32_t* hits, uint32_t* hit_inst,
                        uint64_t cap, uint64_t* total, uint64_t* bsum, hipStream_t st) {
    const uint64_t nb = (n + kBlock - 1) / kBlock;
    hr_status s = HR_OK;
    if (nb > 0) {
        k_search_count<<<dim3((uint32_t)nb), dim3(kBlock), 0, st>>>(a, b, N, n, win_lo, win_d,
                                                                    group, counts, bsum);
        if ((s = launched()) != HR_OK) return s;
    }
    k_scan_blocks<<<1, kBlock, 0, st>>>(bsum, nb, total);
    if ((s = launched()) != HR_OK) return s;
    if (nb > 0) {
        k_search_emit<<<dim3((uint32_t)nb), dim3(kBlock), 0, st>>>(
            a, b, N, n, win_lo, win_d, group, counts, bsum, offsets, hits, hit_inst, cap);
        if ((s = launched()) != HR_OK) return s;
    }
    return HR_OK;
}

}  // namespace

extern "C" {

hr_status hr_search(hr_ctx* ctx, const uint64_t* a, const uint64_t* b, const uint32_t* N,
                    uint64_t n, const uint64_t* win_lo, const uint64_t* win_d, uint32_t group,
                    uint32_t* counts, uint64_t* offsets, uint32_t* hits, uint32_t* hit_inst,
                    uint64_t cap, uint64_t* total, void* stream) {
    hr_status s = search_args_ok(ctx, a, b, N, n, win_d, group, counts, offsets, hits, cap, total);
    if (s != HR_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return HR_EDEVICE;
    const uint64_t nb = (n + kBlock - 1) / kBlock;
    if ((s = ensure_scratch(ctx, (nb + 1) * sizeof(uint64_t))) != HR_OK) return s;
    return search_launch(a, b, N, n, win_lo, win_d, group, counts, offsets, hits, hit_inst, cap,
                         total, (uint64_t*)ctx->scratch, as_stream(stream));
}

hr_status hr_search_static(hr_ctx* ctx, const uint64_t* a, const uint64_t* b,
                           const uint32_t* N, uint64_t n, const uint64_t* win_lo,
                           const uint64_t* win_d, uint32_t group, uint32_t* counts,
                           uint64_t* offsets, uint32_t* hits, uint32_t* hit_inst, uint64_t cap,
                           uint64_t* total, void* stream) {
    hr_status s = search_args_ok(ctx, a, b, N, n, win_d, group, counts, offsets, hits, cap, total);
    if (s != HR_OK) return s;
    const uint64_t nb = (n + kBlock - 1) / kBlock;
    if (nb + 1 > kStaticScratchWords) return HR_ESCRATCH;
    if (hipSetDevice(ctx->device) != hipSuccess) return HR_EDEVICE;
    uint64_t* bsum = nullptr;
    if ((s = static_scratch(ctx->device, &bsum)) != HR_OK) return s;
    return search_launch(a, b, N, n, win_lo, win_d, group, counts, offsets, hits, hit_inst, cap,
                         total, bsum, as_stream(stream));
}

hr_status hr_tabulate(hr_ctx* ctx, const uint64_t* table, uint32_t n_sub, uint32_t degree,
                      uint32_t tau, uint32_t width_bits, uint64_t* a_out, uint64_t* b_out,
                      void* stream) {
    if (!ctx || !valid_poly(degree, width_bits) || tau == 0) return HR_EINVAL;
    if (!pow_fits128(tau, degree)) return HR_EINVAL;
    if (n_sub == 0) return HR_OK;
    if (!table || !a_out || !b_out) return HR_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return HR_EDEVICE;
    hipStream_t st = as_stream(stream);
    const uint32_t nu = pick_nu_tab(n_sub, tau);
    const uint64_t sps = (tau + (uint64_t)kTabLanes * nu - 1) / ((uint64_t)kTabLanes * nu);
    const uint64_t segs_per_wave = 64 / kTabLanes;
    const uint64_t blocks = 2 * (((uint64_t)n_sub * sps + segs_per_wave - 1) / segs_per_wave);
    if (blocks > 0xffffffffull || sps > 0xffffffffull) return HR_EINVAL;
    // composed 64-bit start when every first piece (< tau) stays below the limit
    const bool small = (uint64_t)tau - 1 + (uint64_t)degree * kTabLanes < hr::binom64_limit((int)degree);
    if (small)
        HR_DISPATCH(width_bits, degree,
                    (k_tabulate<L_, D_, kTabLanes, true><<<dim3((uint32_t)blocks), dim3(64), 0, st>>>(
                        table, n_sub, tau, nu, (uint32_t)sps, a_out, b_out)));
    else
        HR_DISPATCH(width_bits, degree,
                    (k_tabulate<L_, D_, kTabLanes, false><<<dim3((uint32_t)blocks), dim3(64), 0, st>>>(
                        table, n_sub, tau, nu, (uint32_t)sps, a_out, b_out)));
    return launched();
}

hr_status hr_recheck(hr_ctx* ctx, const uint64_t* table, uint32_t n_sub, uint32_t degree,
                     uint32_t tau, uint32_t width_bits, const uint32_t* cand_inst,
                     const uint32_t* cand_k, uint64_t n_cand, uint32_t max_k,
                     const uint64_t* thr, uint64_t* value_out, uint8_t* class_out,
                     void* stream) {
    if (!ctx || !valid_poly(degree, width_bits) || tau == 0) return HR_EINVAL;
    if (!pow_fits128(tau, degree) || !pow_fits128(max_k, degree)) return HR_EINVAL;
    if (n_cand == 0) return HR_OK;
    if (!table || !cand_inst || !cand_k || !thr || !value_out || !class_out || n_sub == 0)
        return HR_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return HR_EDEVICE;
    hipStream_t st = as_stream(stream);
    const uint64_t blocks = (n_cand + kBlock - 1) / kBlock;
    if (blocks > 0xffffffffull) return HR_EINVAL;
    HR_DISPATCH(width_bits, degree,
                (k_recheck<L_, D_><<<dim3((uint32_t)blocks), dim3(kBlock), 0, st>>>(
                    table, n_sub, tau, cand_inst, cand_k, n_cand, thr, value_out, class_out)));
    return launched();
}

hr_status hr_pipeline(hr_ctx* ctx, const uint64_t* table, uint32_t n_sub, uint32_t degree,
                      uint32_t tau, uint32_t width_bits, uint32_t N, const uint64_t* win,
                      const uint64_t* thr, hr_result* out, uint64_t cap, uint64_t* count,
                      uint64_t* stats, void* stream) {
    if (!ctx || !valid_poly(degree, width_bits) || tau == 0 || N == 0) return HR_EINVAL;
    if (!pow_fits128(tau, degree) || !pow_fits128(N, degree)) return HR_EINVAL;
    if (!count) return HR_EINVAL;
    if (n_sub == 0) return HR_OK;
    if (!table || !win || !thr || (cap > 0 && !out)) return HR_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return HR_EDEVICE;
    hipStream_t st = as_stream(stream);
    const uint32_t nu = pick_nu(n_sub, tau);
    const uint32_t per_sub = (tau + nu - 1) / nu;
    const uint32_t wps = (per_sub + 63) / 64;       // waves per sub-interval
    const uint64_t blocks = (uint64_t)n_sub * wps;
    if (blocks > 0xffffffffull) return HR_EINVAL;
    HR_DISPATCH(width_bits, degree,
                (k_pipeline<L_, D_><<<dim3((uint32_t)blocks), dim3(64), 0, st>>>(
                    table, n_sub, tau, nu, wps, N, win, thr, out, cap,
                    (unsigned long long*)count, stat_slots(ctx, stats))));
    const hr_status s = launched();
    return s != HR_OK ? s : flush_stat_slots(ctx, stats, st);
}

hr_status hr_subtables(hr_ctx* ctx, const uint64_t* upper, uint32_t upper_degree,
                       uint32_t upper_width, const uint32_t* t_idx, uint32_t t0,
                       const uint32_t* N_per, uint32_t N, uint32_t max_t, uint32_t max_N,
                       uint32_t n_sub, uint32_t degree, uint32_t width_bits, uint64_t* table_out,
                       void* stream) {
    if (!ctx || upper_degree < 1 || upper_degree > HR_MAX_UPPER_DEGREE) return HR_EINVAL;
    if (upper_width % 64 != 0 || upper_width < 192 || upper_width > 448) return HR_EINVAL;
    if (!valid_poly(degree, width_bits) || degree > upper_degree || width_bits > upper_width)
        return HR_EINVAL;
    if (max_N == 0 || !pow_fits128(max_t, upper_degree) ||
        pow_bits((uint64_t)degree * max_N, upper_degree) > upper_width)
        return HR_EINVAL;
    if (!t_idx && (uint64_t)t0 + n_sub - 1 > max_t && n_sub > 0) return HR_EINVAL;
    if (!N_per && (N == 0 || N > max_N)) return HR_EINVAL;
    if (n_sub == 0) return HR_OK;
    if (!upper || !table_out) return HR_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return HR_EDEVICE;
    // lanes per sub-interval: the table's entries, and deg + 1 binomial
    // lanes next to du + 1 shift lanes
    const uint32_t need = std::max((degree + 1) * (degree + 2) / 2, degree + upper_degree + 2);
    const uint32_t G = need <= 16 ? 16 : need <= 32 ? 32 : 64;
    if (need > 64 || (64 / G) * ((degree + 1) * (upper_degree + 1) + upper_degree + 1) >
                         (uint32_t)kSubtabWords)
        return HR_EINVAL;
    const uint64_t blocks = ((uint64_t)n_sub + 64 / G - 1) / (64 / G);
    if (blocks > 0xffffffffull) return HR_EINVAL;
    hipStream_t st = as_stream(stream);
#define HR_SUBTAB(LU_)                                                                    \
    k_subtables<LU_><<<dim3((uint32_t)blocks), dim3(64), 0, st>>>(                        \
        upper, upper_degree, t_idx, t0, N_per, N, max_t, max_N, n_sub, degree, width_bits, \
        G, table_out)
    switch (upper_width / 32) {
        case 6: HR_SUBTAB(6); break;
        case 8: HR_SUBTAB(8); break;
        case 10: HR_SUBTAB(10); break;
        case 12: HR_SUBTAB(12); break;
        case 14: HR_SUBTAB(14); break;
        default: return HR_EINVAL;
    }
#undef HR_SUBTAB
    return launched();
}

hr_status hr_filter(hr_ctx* ctx, int alg, const uint64_t* a, const uint64_t* b, const uint32_t* N,
                    uint64_t n, const uint64_t* win_lo, const uint64_t* win_d, uint32_t group,
                    uint8_t* pass, uint64_t* d_out, uint32_t* iters, void* stream) {
    if (!ctx || !win_d || group == 0 || n > 0xffffffffull) return HR_EINVAL;
    if (alg != HR_FILTER_LEFEVRE && alg != HR_FILTER_REGULAR) return HR_EINVAL;
    if (n == 0) return HR_OK;
    if (!a || !b || !N || !pass) return HR_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return HR_EDEVICE;
    const uint64_t blocks = (n + kBlock - 1) / kBlock;
    hipStream_t st = as_stream(stream);
    if (alg == HR_FILTER_LEFEVRE)
        k_filter<HR_FILTER_LEFEVRE><<<dim3((uint32_t)blocks), dim3(kBlock), 0, st>>>(
            a, b, N, n, win_lo, win_d, group, pass, d_out, iters);
    else
        k_filter<HR_FILTER_REGULAR><<<dim3((uint32_t)blocks), dim3(kBlock), 0, st>>>(
            a, b, N, n, win_lo, win_d, group, pass, d_out, iters);
    return launched();
}

hr_status hr_search_steps(hr_ctx* ctx, const uint64_t* a, const uint64_t* b, const uint32_t* N,
                          uint64_t n, const uint64_t* win_lo, const uint64_t* win_d,
                          uint32_t group, uint32_t* steps, void* stream) {
    if (!ctx || !win_d || group == 0 || n > 0xffffffffull) return HR_EINVAL;
    if (n == 0) return HR_OK;
    if (!a || !b || !N || !steps) return HR_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return HR_EDEVICE;
    const uint64_t blocks = (n + kBlock - 1) / kBlock;
    k_search_steps<<<dim3((uint32_t)blocks), dim3(kBlock), 0, as_stream(stream)>>>(
        a, b, N, n, win_lo, win_d, group, steps);
    return launched();
}

hr_status hr_quot_check(hr_ctx* ctx, const uint64_t* num, const uint64_t* den, uint64_t cap,
                        uint64_t* out, uint64_t* rem, uint64_t n, void* stream) {
    if (!ctx || cap == 0 || cap >= (1ull << 32)) return HR_EINVAL;
    if (n == 0) return HR_OK;
    if (!num || !den || !out) return HR_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return HR_EDEVICE;
    const uint64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 0xffffffffull) return HR_EINVAL;
    k_quot_check<<<dim3((uint32_t)blocks), dim3(kBlock), 0, as_stream(stream)>>>(num, den, cap,
                                                                                 out, rem, n);
    return launched();
}

hr_status hr_batch_open(hr_ctx* ctx, uint32_t slots, hr_batch** out) {
    if (!ctx || !out || slots == 0 || slots > 1024) return HR_EINVAL;
    *out = nullptr;
    if (hipSetDevice(ctx->device) != hipSuccess) return HR_EDEVICE;
    hr_batch* b = (hr_batch*)calloc(1, sizeof(hr_batch));
    if (!b) return HR_ENOMEM;
    b->ctx = ctx;
    b->slots = slots;
    b->done = (hipEvent_t*)calloc(slots, sizeof(hipEvent_t));
    b->ticket = (uint64_t*)calloc(slots, sizeof(uint64_t));
    b->finished = (uint64_t*)calloc(slots, sizeof(uint64_t));
    hr_status st = (b->done && b->ticket && b->finished) ? HR_OK : HR_ENOMEM;
    if (st == HR_OK && hipMalloc((void**)&b->claims, (size_t)slots * 256) != hipSuccess)
        st = HR_ENOMEM;
    for (uint32_t i = 0; st == HR_OK && i < slots; ++i)
        if (hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming) != hipSuccess)
            st = HR_EDEVICE;
    b->nstreams = slots < 4 ? slots : 4;
    for (uint32_t i = 0; st == HR_OK && i < b->nstreams; ++i)
        if (hipStreamCreateWithFlags(&b->streams[i], hipStreamNonBlocking) != hipSuccess)
            st = HR_EDEVICE;
    if (st != HR_OK) {
        hr_batch_close(b);
        return st;
    }
    *out = b;
    return HR_OK;
}

hr_status hr_batch_submit(hr_batch* b, const uint64_t* pool, const hr_item* items, uint32_t n_items,
                          uint32_t width_bits, uint32_t degree, hr_result* out, uint64_t cap,
                          uint64_t* count, void* after_stream, uint64_t* ticket) {
    if (!b || !ticket || !count || !valid_poly(degree, width_bits)) return HR_EINVAL;
    if (n_items > 0x7fffffffu) return HR_EINVAL;
    if (n_items > 0 && (!pool || !items || (cap > 0 && !out))) return HR_EINVAL;
    hr_ctx* ctx = b->ctx;
    if (hipSetDevice(ctx->device) != hipSuccess) return HR_EDEVICE;
    const uint64_t t = b->next_ticket + 1;
    const uint32_t slot = (uint32_t)(t % b->slots);
    if (b->finished[slot] < b->ticket[slot]) {   // that slot's last launch must be over
        const hipError_t q = hipEventQuery(b->done[slot]);
        if (q == hipErrorNotReady) return HR_ECAPACITY;
        if (q != hipSuccess) return HR_EDEVICE;
        b->finished[slot] = b->ticket[slot];
    }
    hipStream_t st = b->streams[t % b->nstreams];
    if (after_stream) {   // the launch follows the caller's work queued so far
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return HR_EDEVICE;
        const bool ok = hipEventRecord(ev, as_stream(after_stream)) == hipSuccess &&
                        hipStreamWaitEvent(st, ev, 0) == hipSuccess;
        (void)hipEventDestroy(ev);
        if (!ok) return HR_EDEVICE;
    }
    unsigned int* claim = (unsigned int*)((char*)b->claims + (size_t)slot * 256);
    unsigned long long* cnt = (unsigned long long*)count;
    k_zero_claim_count<<<1, 1, 0, st>>>(claim, cnt);
    hr_status s = launched();
    if (s != HR_OK) return s;
    if (n_items > 0) {
        HR_DISPATCH(width_bits, degree, ({
            const uint32_t r = resident_waves<L_, D_>(ctx->device);
            if (r == 0) return HR_EDEVICE;
            const uint32_t grid = r < n_items ? r : n_items;
            k_items<L_, D_, true><<<dim3(grid), dim3(64), 0, st>>>(pool, items, n_items, claim,
                                                                   out, cap, cnt, nullptr);
        }));
        if ((s = launched()) != HR_OK) return s;
    }
    if (hipEventRecord(b->done[slot], st) != hipSuccess) return HR_EDEVICE;
    b->ticket[slot] = t;
    b->next_ticket = t;
    *ticket = t;
    return HR_OK;
}

hr_status hr_batch_poll(hr_batch* b, uint64_t* done) {
    if (!b || !done) return HR_EINVAL;
    if (hipSetDevice(b->ctx->device) != hipSuccess) return HR_EDEVICE;
    while (b->done_through < b->next_ticket) {
        const uint64_t t = b->done_through + 1;
        const uint32_t slot = (uint32_t)(t % b->slots);
        if (b->finished[slot] < t) {   // then the slot's last launch is t itself
            const hipError_t q = hipEventQuery(b->done[slot]);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) return HR_EDEVICE;
            b->finished[slot] = b->ticket[slot];
        }
        b->done_through = t;
    }
    *done = b->done_through;
    return HR_OK;
}

hr_status hr_batch_wait(hr_batch* b, uint64_t ticket) {
    if (!b || ticket == 0 || ticket > b->next_ticket) return HR_EINVAL;
    if (hipSetDevice(b->ctx->device) != hipSuccess) return HR_EDEVICE;
    const uint32_t slot = (uint32_t)(ticket % b->slots);
    if (b->finished[slot] < ticket) {   // then the slot's last launch is this ticket
        if (hipEventSynchronize(b->done[slot]) != hipSuccess) return HR_EDEVICE;
        b->finished[slot] = b->ticket[slot];
    }
    uint64_t d;
    return hr_batch_poll(b, &d);
}

hr_status hr_batch_close(hr_batch* b) {
    if (!b) return HR_OK;
    (void)hipSetDevice(b->ctx->device);
    for (uint32_t i = 0; i < b->nstreams; ++i)
        if (b->streams[i]) {
            (void)hipStreamSynchronize(b->streams[i]);
            (void)hipStreamDestroy(b->streams[i]);
        }
    if (b->done)
        for (uint32_t i = 0; i < b->slots; ++i)
            if (b->done[i]) (void)hipEventDestroy(b->done[i]);
    if (b->claims) (void)hipFree(b->claims);
    free(b->done);
    free(b->ticket);
    free(b->finished);
    free(b);
    return HR_OK;
}

hr_status hr_batch_run(hr_ctx* ctx, const uint64_t* pool, const hr_item* items, uint32_t n_items,
                       uint32_t width_bits, uint32_t degree, uint32_t waves, hr_result* out,
                       uint64_t cap, uint64_t* count, uint64_t* stats, void* stream) {
    if (!ctx || !valid_poly(degree, width_bits) || !count) return HR_EINVAL;
    if (n_items > 0x7fffffffu) return HR_EINVAL;
    if (n_items == 0) return HR_OK;
    if (!pool || !items || (cap > 0 && !out)) return HR_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return HR_EDEVICE;
    hipStream_t st = as_stream(stream);
    hr_status s = HR_OK;
    unsigned int* next = claim_counter(ctx);
    unsigned long long* cnt = (unsigned long long*)count;
    unsigned long long* sts = stat_slots(ctx, stats);
    if (waves > 0) {
        k_zero_u32<<<1, 1, 0, st>>>(next);
        if ((s = launched()) != HR_OK) return s;
        HR_DISPATCH(width_bits, degree, ({
            uint32_t w = waves;
            if (w == HR_WAVES_FILL) {   // as many waves as the device keeps resident
                const uint32_t r = resident_waves<L_, D_>(ctx->device);
                if (r == 0) return HR_EDEVICE;
                w = r;
            }
            const uint32_t grid = w < n_items ? w : n_items;
            k_items<L_, D_, true><<<dim3(grid), dim3(64), 0, st>>>(pool, items, n_items, next,
                                                                   out, cap, cnt, sts);
        }));
    } else {
        HR_DISPATCH(width_bits, degree,
                    (k_items<L_, D_, false><<<dim3(n_items), dim3(64), 0, st>>>(
                        pool, items, n_items, next, out, cap, cnt, sts)));
    }
    if ((s = launched()) != HR_OK) return s;
    return flush_stat_slots(ctx, stats, st);
}

}  // extern "C"
