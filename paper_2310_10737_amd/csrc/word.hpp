// Device-side SOGRAND decoding of one component word by one wavefront; shared by
// the plain, batched and served kernels.
#pragma once

#include <cmath>
#include <cstdlib>

#include "internal.hpp"

// One 64-lane wavefront decodes one component word:
//   1. hard decision y, its syndrome s0 = XOR of the H columns where y = 1 and
//      its parity (section "Background on GRAND": H c = 0; even-code parity);
//   2. reliability ranks of (|lambda|, index): counting smaller keys, or a bitonic
//      network across lanes over 32-bit keys with an exact fallback;
//   3. rho_i = exp(-|lambda_i|), so that p(z|r) = p(0|r) prod_{i in z} rho_i
//      (the bookkeeping of section "GRAND per block SO": p(z) from p(0) in w(z)
//      operations), and the parity-class masses E, O (sums of prod rho over
//      nonzero even / odd subsets) by a tree reduction;
//   4. the query loop: lane t tests pattern base+t of the code's rank-space
//      schedule; a wave ballot finds the hits in query order; the running mass
//      of tested patterns is accumulated per lane up to the L-th hit or the cap;
//   5. Corollary 1 (eqs. app_approx_correct, app_approxlist) within the parity
//      class, then eq. (LLRi) per bit and L_E = L_APP - lambda.
// All probabilities are binary64; p(0|r) cancels in every ratio and is never
// formed.
namespace sg {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;            // init and check kernels
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kXcds = 8;                     // MI355X: workgroups are dealt to 8 XCDs in turn

// Per-wave scratch.  A rank's H column and rho share one 16-byte entry, so the
// query loop reads both with one LDS instruction into an aligned register pair.
struct WaveLds {
    uint4 ent_r[SOGRAND_NMAX + 4];       // by rank (1..n): rho (x, y), H column (z); [0]: rho 1, H 0
    uint64_t key_b[SOGRAND_NMAX + 2];    // |lambda| bit patterns by bit index, padded with ~0
    double tau_l[SOGRAND_LIST_MAX];      // prod rho of each found pattern
    uint4 pat_l[SOGRAND_LIST_MAX];       // found patterns (ranks)
    uint32_t q_l[SOGRAND_LIST_MAX];      // query number of each found codeword
    uint32_t zmask[SOGRAND_NMAX];        // bit l set iff the bit lies in found pattern l
    uint8_t pi_r[SOGRAND_NMAX + 1];      // bit index of each rank
    uint8_t rank_b[SOGRAND_NMAX];        // rank of each bit index
};

// Logical index of this workgroup.  With xcd set, consecutive logical indices (the
// lines of one frame) go to the same XCD and share its L2; the grid is then a
// multiple of 8.
__device__ __forceinline__ size_t logical_block(bool xcd) {
    if (!xcd) return blockIdx.x;
    const size_t per = gridDim.x / kXcds;
    return (size_t)(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}

template <int NS>
struct Lanes {
    static constexpr int NB = NS > 64 ? 2 : 1;   // elements held per lane
};

struct WordStats {
    uint32_t Q;      // patterns tested
    int found;       // codewords in the list
    double pnf;      // P(transmitted codeword not in the list)
    double D;        // normaliser: sum of found prod rho + not-found mass * phi (relative to p(0|r))
    uint64_t ranks;  // sum of the Hamming weights of the tested patterns (only when counting)
    int exact_rank;  // the ranks needed the exact (counting) pass
};

// number of nonzero bytes of a packed pattern (its Hamming weight)
__device__ __forceinline__ uint32_t pattern_weight(uint4 e) {
    uint32_t w = 0;
    const uint32_t d[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
    for (int j = 0; j < 4; j++) {
        uint32_t m = d[j] | (d[j] >> 4);
        m |= m >> 2;
        m |= m >> 1;
        w += __popc(m & 0x01010101u);
    }
    return w;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// v from lane (lane ^ M), entirely in the VALU: DPP quad permutations for M = 1, 2,
// row shifts with complementary bank masks for M = 4, 8, and the gfx950 permlane
// swaps for M = 16, 32.
template <int M>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
    if constexpr (M == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);
    } else if constexpr (M == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);
    } else if constexpr (M == 4) {
        const int t = __builtin_amdgcn_update_dpp((int)v, (int)v, 0x104, 0xF, 0x5, false);
        return (uint32_t)__builtin_amdgcn_update_dpp(t, (int)v, 0x114, 0xF, 0xA, false);
    } else if constexpr (M == 8) {
        const int t = __builtin_amdgcn_update_dpp((int)v, (int)v, 0x108, 0xF, 0x3, false);
        return (uint32_t)__builtin_amdgcn_update_dpp(t, (int)v, 0x118, 0xF, 0xC, false);
    } else if constexpr (M == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (threadIdx.x & 16) ? r[0] : r[1];
    } else {
        static_assert(M == 32, "xor distance");
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (threadIdx.x & 32) ? r[0] : r[1];
    }
}

template <int M>
__device__ __forceinline__ double xor_lane_f64(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = xor_lane<M>((uint32_t)u), hi = xor_lane<M>((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ uint32_t wave_xor(uint32_t v) {
    v ^= xor_lane<1>(v);
    v ^= xor_lane<2>(v);
    v ^= xor_lane<4>(v);
    v ^= xor_lane<8>(v);
    v ^= xor_lane<16>(v);
    v ^= xor_lane<32>(v);
    return v;
}

__device__ __forceinline__ uint32_t wave_add(uint32_t v) {
    v += xor_lane<1>(v);
    v += xor_lane<2>(v);
    v += xor_lane<4>(v);
    v += xor_lane<8>(v);
    v += xor_lane<16>(v);
    v += xor_lane<32>(v);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
    v += xor_lane_f64<1>(v);
    v += xor_lane_f64<2>(v);
    v += xor_lane_f64<4>(v);
    v += xor_lane_f64<8>(v);
    v += xor_lane_f64<16>(v);
    v += xor_lane_f64<32>(v);
    return v;
}

__device__ __forceinline__ double bcast0(double v) {
    uint64_t u = (uint64_t)__double_as_longlong(v);
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
    uint64_t u = (uint64_t)__double_as_longlong(v);
    uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, l);
    uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// parity-class masses of two disjoint bit sets combined (see decode_word step 3):
// E = E1 + E2 (1 + E1) + O1 O2 and O = O1 (1 + E2) + O2 (1 + E1), sums of positive terms
template <int M>
__device__ __forceinline__ void eo_combine(double &E, double &O) {
    const double E2 = xor_lane_f64<M>(E), O2 = xor_lane_f64<M>(O);
    const double t1 = 1.0 + E, t2 = 1.0 + E2;
    const double nE = fma(O, O2, fma(E2, t1, E));
    const double nO = fma(O, t2, O2 * t1);
    E = nE;
    O = nO;
}

// v from lane (lane ^ (K-1)), the mirror image inside aligned blocks of K lanes:
// quad_perm [3,2,1,0], row_half_mirror and row_mirror, composed with the permlane
// swaps for blocks of 32 and 64 lanes
// full-mask DPP permutation (every lane reads a lane of its own row)
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_perm(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}

template <int K>
__device__ __forceinline__ uint32_t flip_lane(uint32_t v) {
    if constexpr (K == 2) {
        return dpp_perm<0xB1>(v);
    } else if constexpr (K == 4) {
        return dpp_perm<0x1B>(v);
    } else if constexpr (K == 8) {
        return dpp_perm<0x141>(v);
    } else if constexpr (K == 16) {
        return dpp_perm<0x140>(v);
    } else if constexpr (K == 32) {
        return dpp_perm<0x140>(xor_lane<16>(v));
    } else {
        static_assert(K == 64, "block size");
        return dpp_perm<0x140>(xor_lane<16>(xor_lane<32>(v)));
    }
}

// compare-exchange in an ascending network: the lower position keeps the minimum
__device__ __forceinline__ uint32_t cas32(uint32_t k, uint32_t p, bool lower) {
    const uint32_t mn = p < k ? p : k, mx = p < k ? k : p;
    return lower ? mn : mx;
}

// Bitonic network with ascending comparators only: for each block size K the
// first step compares mirror images inside the block, the next ones compare
// positions J = K/4, ..., 1 apart.
template <int J, int NB>
__device__ __forceinline__ void merge32(uint32_t (&k)[NB], int lane) {
    if constexpr (J >= 1) {
#pragma unroll
        for (int b = 0; b < NB; b++) k[b] = cas32(k[b], xor_lane<J>(k[b]), (lane & J) == 0);
        merge32<J / 2, NB>(k, lane);
    }
}

// 64 * NB keys, element e = lane + 64*slot, sorted ascending in place; with KMAX = 32
// each half of the wave is sorted on its own
template <int K, int NB, int KMAX>
__device__ __forceinline__ void sort32(uint32_t (&k)[NB], int lane) {
    if constexpr (K <= 64 && K <= KMAX) {
#pragma unroll
        for (int b = 0; b < NB; b++) k[b] = cas32(k[b], flip_lane<K>(k[b]), (lane & (K / 2)) == 0);
        merge32<K / 4, NB>(k, lane);
        sort32<K * 2, NB, KMAX>(k, lane);
    } else if constexpr (K == 128 && NB == 2) {
        // mirror of element lane (slot 0) is element 127 - lane = slot 1 of lane 63 - lane
        const uint32_t f0 = flip_lane<64>(k[0]), f1 = flip_lane<64>(k[1]);
        k[0] = f1 < k[0] ? f1 : k[0];
        k[1] = f0 > k[1] ? f0 : k[1];
        merge32<32, NB>(k, lane);
    }
}

// v from lane + 1 (lane 63 reads lane 0)
__device__ __forceinline__ uint32_t next_lane(uint32_t v) {
    return (uint32_t)__shfl((int)v, (int)((threadIdx.x + 1) & (kWave - 1)));
}

// ---- binary64 elementary functions for the per-bit work ----
// Loads a value every lane of the wave agrees on into scalar registers.  Inside
// a loop that also stores to device memory the compiler cannot prove such a load
// constant and would keep the value (and all addresses derived from it) per lane.
template <typename V>
__device__ __forceinline__ V load_uniform(const V *p) {
    static_assert(sizeof(V) % 4 == 0, "whole 32-bit words");
    uint32_t w[sizeof(V) / 4];
    __builtin_memcpy(w, p, sizeof(V));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(V) / 4); i++) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    V v;
    __builtin_memcpy(&v, w, sizeof(V));
    return v;
}

// Coefficients of the elementary functions below.  A kernel that loops over
// words (the persistent kernel) reads them through a pointer the compiler
// cannot see through (TABLE = true), so that each use is a scalar load: as
// literals, the loop would hoist all of them into registers for its whole
// length and cost a fifth of the register file.  A kernel that decodes one word
// takes them as literals (TABLE = false).
struct CoefSet {
    double v[29];
};
constexpr int kInvLn2At = 0, kLn2HiAt = 1, kLn2LoAt = 2;
constexpr int kExpAt = 3, kExpTerms = 14;                    // 1/13!, 1/12!, ..., 1/1!, 1
constexpr int kLogAt = kExpAt + kExpTerms, kLogTerms = 12;   // 1/23, 1/21, ..., 1/3, 1
constexpr CoefSet kCoefV = {{
    1.4426950408889634,                 // 1 / ln 2
    0x1.62e42fefa2000p-1,               // ln 2 to 40 bits: k * this is exact for |k| < 2^13
    0x1.9ef35793c7673p-41,              // ln 2 minus the above
    1.0 / 6227020800.0, 1.0 / 479001600.0, 1.0 / 39916800.0, 1.0 / 3628800.0, 1.0 / 362880.0,
    1.0 / 40320.0, 1.0 / 5040.0, 1.0 / 720.0, 1.0 / 120.0, 1.0 / 24.0, 1.0 / 6.0, 0.5, 1.0, 1.0,
    1.0 / 23.0, 1.0 / 21.0, 1.0 / 19.0, 1.0 / 17.0, 1.0 / 15.0, 1.0 / 13.0, 1.0 / 11.0, 1.0 / 9.0,
    1.0 / 7.0, 1.0 / 5.0, 1.0 / 3.0, 1.0,
}};
static_assert(kLogAt + kLogTerms == 29, "coefficient count");
static __constant__ CoefSet kCoefTable = kCoefV;
typedef __attribute__((address_space(4))) const CoefSet ccoef;

template <bool TABLE>
struct Coef {
    const ccoef *t;
    __device__ __forceinline__ Coef() {
        if constexpr (TABLE) {
            t = (const ccoef *)&kCoefTable;
            asm volatile("" : "+s"(t));
        }
    }
    __device__ __forceinline__ double operator[](int j) const {
        if constexpr (TABLE) return t->v[j];
        else return kCoefV.v[j];
    }
};

// 1/x for positive normal x: hardware reciprocal and two Newton steps
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// e^{-a}, a >= 0: Cody-Waite reduction a = k ln2 + r with |r| <= ln2/2, then the
// degree-13 Taylor polynomial of e^{-r} (truncation below 2^-57 relative)
template <bool TABLE>
__device__ __forceinline__ double exp_neg(double a) {
    const Coef<TABLE> t;
    const double ac = a < 1100.0 ? a : 1100.0;
    const double k = rint(ac * t[kInvLn2At]);
    double r = fma(-k, t[kLn2HiAt], ac);
    r = fma(-k, t[kLn2LoAt], r);
    const double x = -r;
    double p = t[kExpAt];
#pragma unroll
    for (int j = 1; j < kExpTerms; j++) p = fma(p, x, t[kExpAt + j]);
    return ldexp(p, -(int)k);
}

// ln x for finite x > 0 of normal magnitude: x = m 2^e with m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(s) = 2 s sum_j s^{2j} / (2j + 1) with s = (m - 1)/(m + 1), |s| < 0.1716
template <bool TABLE>
__device__ __forceinline__ double log_pos(double x) {
    double m = __builtin_amdgcn_frexp_mant(x);
    int e = __builtin_amdgcn_frexp_exp(x);
    if (m < 0.70710678118654752) {
        m = m + m;
        e -= 1;
    }
    const double num = m - 1.0, den = m + 1.0;
    const double rd = rcp_nr(den);
    double s = num * rd;
    s = fma(fma(-den, s, num), rd, s);
    const double z = s * s;
    const Coef<TABLE> t;
    double p = t[kLogAt];
#pragma unroll
    for (int j = 1; j < kLogTerms; j++) p = fma(p, z, t[kLogAt + j]);
    const double lm = (s + s) * p;
    const double de = (double)e;
    return fma(de, t[kLn2HiAt], fma(de, t[kLn2LoAt], lm));
}

// ln(N0 / N1) for N0, N1 >= 0 not both zero: the mantissas' ratio (in (1/2, 2)) goes
// through ln, the exponents' difference is added as a multiple of ln 2
template <bool TABLE>
__device__ __forceinline__ double log_ratio(double n0, double n1) {
    const double m0 = __builtin_amdgcn_frexp_mant(n0), m1 = __builtin_amdgcn_frexp_mant(n1);
    const int e0 = __builtin_amdgcn_frexp_exp(n0), e1 = __builtin_amdgcn_frexp_exp(n1);
    const double r = rcp_nr(m1);
    double q = m0 * r;
    q = fma(fma(-m1, q, m0), r, q);
    const double de = (double)(e0 - e1);
    const Coef<TABLE> t;
    double la = fma(de, t[kLn2HiAt], fma(de, t[kLn2LoAt], log_pos<TABLE>(q)));
    if (n1 == 0.0) la = 1000.0;
    if (n0 == 0.0) la = -1000.0;
    return la;
}

// zmask[bit] |= 1 << l for every bit of found pattern l: lane t handles byte t % 16
// of pattern t / 16 (+ 4 per round); rank r maps back to its bit through pi_r.
__device__ __forceinline__ void mark_found(WaveLds &S, int found, int lane) {
    for (int g = 0; g < found; g += 4) {
        const int l = g + (lane >> 4);
        if (l < found) {
            const uint4 pl = S.pat_l[l];
            const int j = lane & 15;
            const uint32_t d = j < 4 ? pl.x : (j < 8 ? pl.y : (j < 12 ? pl.z : pl.w));
            const uint32_t r = (d >> (8 * (j & 3))) & 0xffu;
            if (r) atomicOr(&S.zmask[S.pi_r[r]], 1u << l);
        }
    }
    wave_sync();
}

__device__ __forceinline__ double rho_at(const WaveLds &S, int r) {
    return __longlong_as_double((long long)(((uint64_t)S.ent_r[r].y << 32) | S.ent_r[r].x));
}

__device__ __forceinline__ void put_rho(WaveLds &S, int r, double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    S.ent_r[r].x = (uint32_t)u;
    S.ent_r[r].y = (uint32_t)(u >> 32);
}

// One rank of a pattern: r is byte SH/8 of dword d.
#define SG_RANK(d, SH)                                   \
    do {                                                 \
        const uint32_t r_ = ((d) >> (SH)) & 0xffu;       \
        const uint4 q_ = S.ent_r[r_];                    \
        s ^= q_.z;                                       \
        tau *= __longlong_as_double((long long)(((uint64_t)q_.y << 32) | q_.x)); \
    } while (0)

// Rank (1-based) of each lane's key among the n keys, |lambda| bit patterns by bit
// index (non-negative doubles order like their bit patterns), ties by bit index.
// Returns whether the exact tie-resolving pass ran.
//
// By counting: a lane's rank is the number of smaller keys.  The ranks sum to
// n(n-1)/2 unless equal keys exist, and then each group of equal keys is ordered
// by bit index.
__device__ __forceinline__ bool ranks_by_count(uint64_t key, bool valid, int n, WaveLds &S, int lane,
                                               int &myrank) {
    bool exact_pass = false;
    S.key_b[lane] = key;
    if (lane < 2) S.key_b[kWave + lane] = ~0ull;
    wave_sync();
    uint32_t cnt = 0;
    for (int j = 0; j < n; j += 2) {
        const uint64_t k0 = S.key_b[j], k1 = S.key_b[j + 1];
        cnt += (k0 < key) ? 1u : 0u;
        cnt += (k1 < key) ? 1u : 0u;
    }
    const uint32_t tot = __builtin_amdgcn_readfirstlane(wave_add(valid ? cnt : 0u));
    if (tot != (uint32_t)(n * (n - 1) / 2)) {
        exact_pass = true;
        for (int j = 0; j < n; j++) {
            const uint64_t kj = S.key_b[j];
            cnt += (kj == key && j < lane) ? 1u : 0u;
        }
    }
    myrank = valid ? (int)cnt + 1 : 0;
    return exact_pass;
}

// By a bitonic network over 32-bit keys: |lambda| rounded to binary32 (a monotone
// map) with its low IB bits replaced by the bit index, so the keys are distinct.  If
// two neighbours of the sorted order agree above bit IB, the rounding or the
// truncation may have decided their order, and the ranks are recomputed exactly by
// counting.  Otherwise every sorted neighbour pair, and so every pair, is in exact
// order.
template <int NS, int NB>
__device__ __forceinline__ bool ranks_by_network(const uint64_t (&key)[NB], const bool (&valid)[NB], int n,
                                                 WaveLds &S, int lane, int (&myrank)[NB]) {
    constexpr int IB = NB == 1 ? 6 : 7;
    uint32_t k32[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const uint32_t id = (uint32_t)(lane + kWave * b);
        const uint32_t f = __float_as_uint((float)__longlong_as_double((long long)key[b]));
        k32[b] = valid[b] ? ((f & ~((1u << IB) - 1u)) | id) : (~((1u << IB) - 1u) | id);
    }
    // words of up to 32 bits sort the lower half of the wave only
    sort32<2, NB, (NS > 32 ? 2 * kWave : kWave / 2)>(k32, lane);
    bool amb;
    if constexpr (NB == 1) {
        const uint32_t nx = next_lane(k32[0]);
        amb = lane + 1 < n && (k32[0] >> IB) == (nx >> IB);
    } else {
        const uint32_t n0 = next_lane(k32[0]), n1 = next_lane(k32[1]);
        const uint32_t first1 = (uint32_t)__builtin_amdgcn_readfirstlane(k32[1]);
        const uint32_t nx0 = lane == kWave - 1 ? first1 : n0;
        amb = lane + 1 < n && (k32[0] >> IB) == (nx0 >> IB);
        amb |= lane + kWave + 1 < n && (k32[1] >> IB) == (n1 >> IB);
    }
    const bool exact_pass = __ballot(amb) != 0ull;
    if (!exact_pass) {
#pragma unroll
        for (int b = 0; b < NB; b++)
            if (lane + kWave * b < n) S.rank_b[k32[b] & ((1u << IB) - 1u)] = (uint8_t)(lane + kWave * b + 1);
        wave_sync();
#pragma unroll
        for (int b = 0; b < NB; b++) myrank[b] = valid[b] ? S.rank_b[lane + kWave * b] : 0;
    } else {
#pragma unroll
        for (int b = 0; b < NB; b++) S.key_b[lane + kWave * b] = key[b];
        wave_sync();
        uint32_t cnt[NB];
#pragma unroll
        for (int b = 0; b < NB; b++) cnt[b] = 0u;
        for (int j = 0; j < n; j++) {
            const uint64_t kj = S.key_b[j];
#pragma unroll
            for (int b = 0; b < NB; b++)
                cnt[b] += (kj < key[b] || (kj == key[b] && j < lane + kWave * b)) ? 1u : 0u;
        }
#pragma unroll
        for (int b = 0; b < NB; b++) myrank[b] = valid[b] ? (int)cnt[b] + 1 : 0;
    }
    return exact_pass;
}

// Decodes one word held as lam[slot] at bit index lane + 64*slot (< n).
// Writes the APP LLRs of the lane's bits into lapp; the list is left in S.
// STOP: the list-BLER stop is compiled in (pstop > 0 selects it at launch).
template <int NS, bool TABLE = false, bool STOP = false>
__device__ __forceinline__ WordStats decode_word(const DevCode &c, const DevCode *cdev, int L, uint32_t qcap,
                                                 double pstop,
                                                 const double (&lam)[Lanes<NS>::NB], WaveLds &S,
                                                 double (&lapp)[Lanes<NS>::NB], int lane, bool count) {
    constexpr int NB = Lanes<NS>::NB;
    const int n = c.n;

    // 1. hard decision, its syndrome and parity; keys |lambda| and rho = e^-|lambda| by bit
    bool valid[NB];
    int ybit[NB];
    double rho[NB];
    uint64_t key[NB];
    uint32_t spart = 0;
    int ycount = 0;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lane + kWave * b;
        valid[b] = i < n;
        ybit[b] = valid[b] && lam[b] < 0.0;
        if (ybit[b]) spart ^= c.hcol[i];
        ycount += __popcll(__ballot(ybit[b]));
        const double a = fabs(lam[b]);
        key[b] = valid[b] ? (uint64_t)__double_as_longlong(a) : ~0ull;
        rho[b] = valid[b] ? exp_neg<TABLE>(a) : 0.0;
    }
    const uint32_t s0 = wave_xor(spart);
    const int par = ycount & 1;

    // 2. reliability ranks (|lambda| ascending, ties by bit index).  The plain kernels
    //    count smaller keys for words of up to 64 bits: two VALU operations per key, with
    //    the keys read back from LDS, whose latency their full occupancy hides.  The
    //    persistent and served kernels, which hold fewer waves per SIMD, and all words
    //    of 128 bits use a sorting network instead.
    int myrank[NB];
    bool exact_pass;
    if constexpr (NB == 1 && !TABLE) exact_pass = ranks_by_count(key[0], valid[0], n, S, lane, myrank[0]);
    else exact_pass = ranks_by_network<NS, NB>(key, valid, n, S, lane, myrank);
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lane + kWave * b;
        if (valid[b]) {
            S.ent_r[myrank[b]].z = c.hcol[i];
            put_rho(S, myrank[b], rho[b]);
            S.pi_r[myrank[b]] = (uint8_t)i;
        }
        if (i < SOGRAND_NMAX) S.zmask[i] = 0u;
    }
    if (lane == 0) {
        S.ent_r[0].z = 0u;
        put_rho(S, 0, 1.0);
    }
    wave_sync();

    // 3. parity-class masses: adding bit i maps (E, O) to (E + O rho_i, O + (1 + E) rho_i);
    //    two disjoint bit sets combine as E = E1 + E2 + E1 E2 + O1 O2, O = O1 + O2 + E1 O2 + O1 E2.
    //    Lane t folds ranks 8t+1 .. 8t+8 in turn, then NS/8 lanes combine pairwise.
    double E = 0.0, O = 0.0;
#pragma unroll
    for (int j = 0; j < 8; j++) {
        const int r = 8 * lane + j + 1;
        const double rr = r <= n ? rho_at(S, r < SOGRAND_NMAX ? r : SOGRAND_NMAX) : 0.0;
        const double e2 = E + O * rr;
        const double o2 = O + (1.0 + E) * rr;
        E = e2;
        O = o2;
    }
    eo_combine<1>(E, O);
    eo_combine<2>(E, O);
    if constexpr (NS >= 64) eo_combine<4>(E, O);
    if constexpr (NS >= 128) eo_combine<8>(E, O);
    E = bcast0(E);
    O = bcast0(O);

    // 4. query loop over the schedule of the word's parity class; the next chunk's
    //    patterns are fetched while the current one is tested
    const int cls = c.even ? par : 0;
    // The persistent kernel holds its DevCode in registers, where a dynamic index
    // would move it to scratch memory: it reads the class's table fields from the
    // device copy instead.  A kernel argument is indexed in place.
    const uint4 *__restrict__ tab;
    const uint32_t *__restrict__ wm;
    uint32_t len;
    if constexpr (TABLE) {
        tab = load_uniform(&cdev->pat[cls]);
        wm = load_uniform(&cdev->wmax[cls]);
        len = load_uniform(&cdev->len[cls]);
    } else {
        tab = c.pat[cls];
        wm = c.wmax[cls];
        len = c.len[cls];
    }
    const uint32_t limit = qcap < len ? qcap : len;
    bool stopped = false;     // the list-BLER stop ended the search
    int found = 0;
    uint32_t Q = 0;
    double s_lane = 0.0;   // this lane's share of the tested nonzero-pattern mass (relative to p(0|r))
    uint32_t w_lane = 0;   // this lane's share of the tested pattern weights (counting only)
    // patterns of the next two chunks are in flight while a chunk is tested
    uint4 e_next = make_uint4(0u, 0u, 0u, 0u), e_next2 = make_uint4(0u, 0u, 0u, 0u);
    if ((uint32_t)lane < limit) e_next = tab[lane];
    if ((uint32_t)lane + kWave < limit) e_next2 = tab[kWave + lane];
    uint32_t wm_next = wm[0];
    uint32_t wm_next2 = limit > (uint32_t)kWave ? wm[1] : 0u;
    for (uint32_t base = 0; base < limit; base += kWave) {
        const uint4 e = e_next;
        const uint32_t wmx = wm_next;
        const uint32_t nb = base + kWave;
        e_next = e_next2;
        wm_next = wm_next2;
        const uint32_t nb2 = nb + kWave;
        if (nb2 < limit) {
            e_next2 = make_uint4(0u, 0u, 0u, 0u);
            if (nb2 + (uint32_t)lane < limit) e_next2 = tab[nb2 + lane];
            wm_next2 = wm[nb2 >> 6];
        }
        const bool act = base + (uint32_t)lane < limit;
        uint32_t s = s0;
        double tau = 1.0;
        // ranks in straight-line pairs (rank 0 pads: hs 0, rho 1), so that both
        // lookups of a pair are in flight together
        SG_RANK(e.x, 0);
        SG_RANK(e.x, 8);
        if (wmx > 2) {
            SG_RANK(e.x, 16);
            SG_RANK(e.x, 24);
            if (wmx > 4) {
                SG_RANK(e.y, 0);
                SG_RANK(e.y, 8);
                if (wmx > 6) {
                    SG_RANK(e.y, 16);
                    SG_RANK(e.y, 24);
                    if (wmx > 8) {
                        SG_RANK(e.z, 0);
                        SG_RANK(e.z, 8);
                        SG_RANK(e.z, 16);
                        SG_RANK(e.z, 24);
                        if (wmx > 12) {
                            SG_RANK(e.w, 0);
                            SG_RANK(e.w, 8);
                            SG_RANK(e.w, 16);
                            SG_RANK(e.w, 24);
                        }
                    }
                }
            }
        }
        uint64_t m = __ballot(act && s == 0u);
        int cut = kWave - 1;
        // tested nonzero-pattern mass before this chunk (only needed by the list-BLER stop)
        const bool check = STOP && m != 0ull;
        double s_before = 0.0;
        if constexpr (STOP) {
            if (check) s_before = bcast0(wave_sum(s_lane));
        }
        while (m != 0ull && found < L && !stopped) {
            const int h = __builtin_ctzll(m);
            m &= m - 1ull;
            const uint32_t hx = __builtin_amdgcn_readlane(e.x, h);
            const uint32_t hy = __builtin_amdgcn_readlane(e.y, h);
            const uint32_t hz = __builtin_amdgcn_readlane(e.z, h);
            const uint32_t hw = __builtin_amdgcn_readlane(e.w, h);
            const double th = readlane_f64(tau, h);
            if (lane == 0) {
                S.tau_l[found] = th;
                S.q_l[found] = base + (uint32_t)h + 1u;
                S.pat_l[found] = make_uint4(hx, hy, hz, hw);
            }
            found++;
            if (found == L) cut = h;
            else if (STOP && check) {
                // list-BLER stop: Corollary 1 for the list so far, with the mass tested up
                // to and including this query (class mass relative to p(0|r), nonzero
                // patterns only)
                const double T = c.even ? (par ? O : E) : (E + O);
                const double pre = (act && (e.x & 0xffu) != 0u && lane <= h) ? tau : 0.0;
                double Mi = T - (s_before + bcast0(wave_sum(pre)));
                if (!(Mi > 0.0)) Mi = 0.0;
                double Di = Mi * c.phi;
                for (int l = 0; l < found; l++) Di += S.tau_l[l];
                if ((Mi * c.phi) / Di < pstop) {
                    stopped = true;
                    cut = h;
                }
            }
        }
        const bool nonzero = (e.x & 0xffu) != 0u;
        if (act && nonzero && lane <= cut) s_lane += tau;
        if (count && act && lane <= cut) w_lane += pattern_weight(e);
        if (found >= L || stopped) {
            Q = base + (uint32_t)cut + 1u;
            break;
        }
        Q = limit < nb ? limit : nb;
    }

    const double Snz = bcast0(wave_sum(s_lane));

    // 5. Corollary 1 inside the parity class: not-found mass M = (class mass) - (tested mass),
    //    both relative to p(0|r); the zero pattern (first in its class) cancels exactly.
    wave_sync();
    const double T = c.even ? (par ? O : E) : (E + O);
    double M = T - Snz;
    if (!(M > 0.0)) M = 0.0;
    double D = M * c.phi;
    for (int l = 0; l < found; l++) D += S.tau_l[l];
    double pnf = (M * c.phi) / D;
    const bool degenerate = !(D > 0.0) || !isfinite(D);
    if (degenerate) pnf = 1.0;   // every probability underflowed: keep the soft input

    // eq. (LLRi): list codewords weighted by their APPs, plus the soft input weighted by P_nf
    double N0[NB], N1[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const double qs = rcp_nr(1.0 + rho[b]);   // p(bit = y | soft input)
        const double qf = rho[b] * qs;            // p(bit != y | soft input)
        N0[b] = pnf * (ybit[b] ? qf : qs);
        N1[b] = pnf * (ybit[b] ? qs : qf);
    }
    if (!degenerate) {
        const double invD = 1.0 / D;
        mark_found(S, found, lane);
        uint32_t zm[NB];
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const int i = lane + kWave * b;
            zm[b] = i < SOGRAND_NMAX ? S.zmask[i] : 0u;
        }
        for (int l = 0; l < found; l++) {
            const double P = S.tau_l[l] * invD;
#pragma unroll
            for (int b = 0; b < NB; b++) {
                const bool one = (ybit[b] ^ (int)((zm[b] >> l) & 1u)) != 0;
                N1[b] += one ? P : 0.0;
                N0[b] += one ? 0.0 : P;
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; b++) {
        double la = log_ratio<TABLE>(N0[b], N1[b]);
        if (!(la <= 1000.0)) la = 1000.0;
        if (!(la >= -1000.0)) la = -1000.0;
        lapp[b] = la;
    }
    WordStats st;
    st.Q = Q;
    st.found = found;
    st.pnf = pnf;
    st.D = D;
    st.ranks = 0;
    st.exact_rank = exact_pass ? 1 : 0;
    if (count) st.ranks = wave_add(w_lane);
    return st;
}


__device__ __forceinline__ void prof_add(ProfCounters *p, const WordStats &st) {
    p += blockIdx.x % kProfSlots;
    atomicAdd(&p->words, 1ull);
    atomicAdd(&p->queries, (unsigned long long)st.Q);
    atomicAdd(&p->ranks, (unsigned long long)st.ranks);
    if (st.exact_rank) atomicAdd(&p->exact_rank, 1ull);
}

}  // namespace sg
