// Device-side SOGRAND decoding of one component word by one wavefront; shared by
// the plain, batched and served kernels.
#pragma once

#include <cmath>
#include <cstdlib>

#include "internal.hpp"

// One 64-lane wavefront decodes one component word:
//   1. hard decision y, its syndrome s0 = XOR of the H columns where y = 1 and
//      its parity (section "Background on GRAND": H c = 0; even-code parity);
//   2. reliability ranks of (|lambda|, index): a bitonic network across lanes over
//      32-bit keys, with an exact counting fallback for near-ties;
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

// Per-wave scratch.  A rank's H column and rho share one 16-byte entry, so the
// query loop reads both with one LDS instruction into an aligned register pair.
struct WaveLds {
    uint4 ent_r[SOGRAND_NMAX + 4];       // by rank (1..n): rho (x, y), H column (z); [0]: rho 1, H 0
    uint64_t key_b[SOGRAND_NMAX + 2];    // |lambda| bit patterns by bit index (the exact ranking pass)
    double tau_l[SOGRAND_LIST_MAX];      // prod rho of each found pattern
    uint4 pat_l[SOGRAND_LIST_MAX];       // found patterns (ranks)
    uint32_t q_l[SOGRAND_LIST_MAX];      // query number of each found codeword
    uint32_t zmask[SOGRAND_NMAX];        // bit l set iff the bit lies in found pattern l
    uint8_t pi_r[SOGRAND_NMAX + 1];      // bit index of each rank
    uint8_t rank_b[SOGRAND_NMAX];        // rank of each bit index
};

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
#ifdef SG_PHASE_CLOCKS
    uint32_t phase[kPhases];   // clock cycles of each decode phase (the last one is set by the caller)
#endif
};

// Phase clocks (builds with SG_PHASE_CLOCKS only): the wave's clock counter read at the
// boundaries of decode_word's steps.
#ifdef SG_PHASE_CLOCKS
#define SG_CLOCK(var) const uint64_t var = __builtin_amdgcn_s_memtime()
#else
#define SG_CLOCK(var) \
    do {              \
    } while (0)
#endif

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

__device__ __forceinline__ double readlane_f64(double v, int l) {
    uint64_t u = (uint64_t)__double_as_longlong(v);
    uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, l);
    uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Wave reductions: a prefix over each row of 16 lanes by DPP row shifts that read zero
// past the row's start (1, 2, 4, 8), then the row broadcasts (lane 15 of rows 0 and 2
// into rows 1 and 3, lane 31 into rows 2 and 3), leave the total in lane 63, which
// readlane makes wave-uniform: six DPP steps, against the exchange of every lane with
// its partner at six distances.  Zero is the identity of each operation.
template <int CTRL, int ROWS, bool ZERO>
__device__ __forceinline__ uint32_t dpp_in(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, ZERO);
}

template <int CTRL, int ROWS, bool ZERO>
__device__ __forceinline__ double dpp_in_f64(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = dpp_in<CTRL, ROWS, ZERO>((uint32_t)u), hi = dpp_in<CTRL, ROWS, ZERO>((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

#define SG_WAVE_REDUCE(IN, OP)                                                         \
    do {                                                                               \
        v = v OP IN<0x111, 0xF, true>(v);   /* row_shr:1 */                            \
        v = v OP IN<0x112, 0xF, true>(v);   /* row_shr:2 */                            \
        v = v OP IN<0x114, 0xF, true>(v);   /* row_shr:4 */                            \
        v = v OP IN<0x118, 0xF, true>(v);   /* row_shr:8 */                            \
        v = v OP IN<0x142, 0xA, false>(v);  /* row_bcast:15 into rows 1 and 3 */       \
        v = v OP IN<0x143, 0xC, false>(v);  /* row_bcast:31 into rows 2 and 3 */       \
    } while (0)

__device__ __forceinline__ uint32_t wave_xor(uint32_t v) {
    SG_WAVE_REDUCE(dpp_in, ^);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, kWave - 1);
}

__device__ __forceinline__ uint32_t wave_add(uint32_t v) {
    SG_WAVE_REDUCE(dpp_in, +);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, kWave - 1);
}

__device__ __forceinline__ double wave_sum(double v) {
    SG_WAVE_REDUCE(dpp_in_f64, +);
    return readlane_f64(v, kWave - 1);
}

// inclusive prefix sum over lanes: lane l gets v(0) + ... + v(l), added in lane order
// at distances 1, 2, 4, ..., 32 (Hillis-Steele)
__device__ __forceinline__ double wave_scan_add(double v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t u = (uint64_t)__double_as_longlong(v);
        const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)u, d);
        const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(u >> 32), d);
        const double t = __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
        if (lane >= d) v += t;
    }
    return v;
}

// parity-class masses of two disjoint bit sets combined (see decode_word step 3):
// E = E1 + E2 (1 + E1) + O1 O2 and O = O1 (1 + E2) + O2 (1 + E1), sums of positive terms.
// The second set is that of lane - M in the same row, or the empty set past the row's
// start (E2 = O2 = 0, which leaves E and O exactly as they are): after M = 1, 2, 4, ...,
// lane t holds the masses of the union of the sets of lanes 0 .. t of its row.
template <int M>
__device__ __forceinline__ void eo_prefix(double &E, double &O) {
    const double E2 = dpp_in_f64<0x110 + M, 0xF, true>(E), O2 = dpp_in_f64<0x110 + M, 0xF, true>(O);
    const double t1 = 1.0 + E, t2 = 1.0 + E2;
    const double nE = fma(O, O2, fma(E2, t1, E));
    const double nO = fma(O, t2, O2 * t1);
    E = nE;
    O = nO;
}

// Compare-exchanges of the ascending network.  Each pair's lower lane keeps the
// minimum and its upper lane the maximum.
//
// Where the lower and upper lanes of every pair are told apart by lane bits 2-5
// (pairs 4, 8, 16 or 32 lanes apart, mirror images in blocks of 8, 16 or 32), the two
// halves are written by two DPP instructions under complementary row or bank masks
// (a row is 16 lanes, a bank 4 lanes of every row), so no select is needed: a
// compare-exchange costs two VALU instructions, plus one permlane swap past 16 lanes.
// Pairs 1 or 2 lanes apart and mirror images in blocks of 2 or 4 lanes differ in lane
// bits 0-1, which no mask reaches: those take both results and a select.
// Each asm block starts and ends with s_nop 1, the two wait states a DPP read needs
// after a VALU write of its operand.

// full-mask DPP permutation (every lane reads a lane of its own row)
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_perm(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}

// the median of k, p and m: min(k, p) where m = 0, max(k, p) where m = ~0
__device__ __forceinline__ uint32_t cas32(uint32_t k, uint32_t p, bool lower) {
    const uint32_t m = lower ? 0u : ~0u;
    const uint32_t mn = p < k ? p : k, mx = p < k ? k : p;
    const uint32_t c = mx < m ? mx : m;
    return mn > c ? mn : c;
}

// t = min(src0 through DPP, src1) under the first masks, max under the second
#define SG_MINMAX_DPP(LO, HI)                                                       \
    "s_nop 1\n\tv_min_u32_dpp %0, %1, %2 " LO "\n\tv_max_u32_dpp %0, %3, %4 " HI "\n\ts_nop 1"

// partner lane ^ J
template <int J>
__device__ __forceinline__ uint32_t ce_xor(uint32_t k, int lane) {
    uint32_t t;
    if constexpr (J == 1 || J == 2) {
        t = cas32(k, xor_lane<J>(k), (lane & J) == 0);
    } else if constexpr (J == 4) {
        asm(SG_MINMAX_DPP("row_shl:4 row_mask:0xf bank_mask:0x5", "row_shr:4 row_mask:0xf bank_mask:0xa")
            : "=&v"(t) : "v"(k), "v"(k), "v"(k), "v"(k));
    } else if constexpr (J == 8) {
        asm(SG_MINMAX_DPP("row_shl:8 row_mask:0xf bank_mask:0x3", "row_shr:8 row_mask:0xf bank_mask:0xc")
            : "=&v"(t) : "v"(k), "v"(k), "v"(k), "v"(k));
    } else if constexpr (J == 16) {
        // after the swap each lane holds its own key and its partner's, one in each register
        const auto r = __builtin_amdgcn_permlane16_swap(k, k, false, false);
        asm(SG_MINMAX_DPP("quad_perm:[0,1,2,3] row_mask:0x5 bank_mask:0xf",
                          "quad_perm:[0,1,2,3] row_mask:0xa bank_mask:0xf")
            : "=&v"(t) : "v"(r[0]), "v"(r[1]), "v"(r[0]), "v"(r[1]));
    } else {
        static_assert(J == 32, "distance");
        const auto r = __builtin_amdgcn_permlane32_swap(k, k, false, false);
        asm(SG_MINMAX_DPP("quad_perm:[0,1,2,3] row_mask:0x3 bank_mask:0xf",
                          "quad_perm:[0,1,2,3] row_mask:0xc bank_mask:0xf")
            : "=&v"(t) : "v"(r[0]), "v"(r[1]), "v"(r[0]), "v"(r[1]));
    }
    return t;
}

// partner lane ^ (K - 1), the mirror image inside aligned blocks of K lanes
template <int K>
__device__ __forceinline__ uint32_t ce_flip(uint32_t k, int lane) {
    uint32_t t;
    if constexpr (K == 2) {
        t = cas32(k, dpp_perm<0xB1>(k), (lane & 1) == 0);
    } else if constexpr (K == 4) {
        t = cas32(k, dpp_perm<0x1B>(k), (lane & 2) == 0);
    } else if constexpr (K == 8) {
        asm(SG_MINMAX_DPP("row_half_mirror row_mask:0xf bank_mask:0x5", "row_half_mirror row_mask:0xf bank_mask:0xa")
            : "=&v"(t) : "v"(k), "v"(k), "v"(k), "v"(k));
    } else if constexpr (K == 16) {
        asm(SG_MINMAX_DPP("row_mirror row_mask:0xf bank_mask:0x3", "row_mirror row_mask:0xf bank_mask:0xc")
            : "=&v"(t) : "v"(k), "v"(k), "v"(k), "v"(k));
    } else {
        static_assert(K == 32, "block size");
        // after the swap the even rows of r[0] and the odd rows of r[1] hold the lane's own
        // key, the other register the key of the same position in the neighbouring row,
        // which the row mirror turns into the partner's
        const auto r = __builtin_amdgcn_permlane16_swap(k, k, false, false);
        asm(SG_MINMAX_DPP("row_mirror row_mask:0x5 bank_mask:0xf", "row_mirror row_mask:0xa bank_mask:0xf")
            : "=&v"(t) : "v"(r[1]), "v"(r[0]), "v"(r[0]), "v"(r[1]));
    }
    return t;
}

// complements the keys of the rows in RM (a descending block is held complemented
// and sorted ascending)
#define SG_NOT_ROWS(RM) "s_nop 1\n\tv_not_b32_dpp %0, %0 quad_perm:[0,1,2,3] row_mask:" RM " bank_mask:0xf\n\ts_nop 1"

// Half-cleaners at distances J, J/2, ..., 1.
template <int J, int NB>
__device__ __forceinline__ void merge32(uint32_t (&k)[NB], int lane) {
    if constexpr (J >= 1) {
#pragma unroll
        for (int b = 0; b < NB; b++) k[b] = ce_xor<J>(k[b], lane);
        merge32<J / 2, NB>(k, lane);
    }
}

// 64 * NB keys, element e = lane + 64*slot, sorted ascending in place; with KMAX = 32
// each half of the wave is sorted on its own.  Bitonic: blocks of K = 2 .. 32 lanes
// begin with a compare of mirror images and continue with half-cleaners.  Blocks of 64
// and 128 elements begin with a half-cleaner instead, which needs the second half
// sorted descending: lanes 32-63 are held complemented from their 32-lane merge on
// (so that it sorts them descending) and restored before the 64-lane merge, and the
// second register is held complemented through its 64-lane merge.
template <int K, int NB, int KMAX>
__device__ __forceinline__ void sort32(uint32_t (&k)[NB], int lane) {
    if constexpr (K <= 32 && K <= KMAX) {
        if constexpr (K == 32 && KMAX >= 64) {
#pragma unroll
            for (int b = 0; b < NB; b++) asm(SG_NOT_ROWS("0xc") : "+v"(k[b]));
        }
#pragma unroll
        for (int b = 0; b < NB; b++) k[b] = ce_flip<K>(k[b], lane);
        merge32<K / 4, NB>(k, lane);
        sort32<K * 2, NB, KMAX>(k, lane);
    } else if constexpr (K == 64 && K <= KMAX) {
        // the first register: ascending, then descending; the second: its lanes 0-31
        // complemented too, so that its merge leaves it complemented and ascending
        asm(SG_NOT_ROWS("0xc") : "+v"(k[0]));
        if constexpr (NB == 2) asm(SG_NOT_ROWS("0x3") : "+v"(k[1]));
        merge32<32, NB>(k, lane);
        sort32<128, NB, KMAX>(k, lane);
    } else if constexpr (K == 128 && NB == 2) {
        // element e + 64 (the second register, now descending) against element e
        const uint32_t d = ~k[1];
        const uint32_t lo = d < k[0] ? d : k[0], hi = d < k[0] ? k[0] : d;
        k[0] = lo;
        k[1] = hi;
        merge32<32, NB>(k, lane);
    }
}

// v from lane + 1 (lane 63 reads lane 0)
__device__ __forceinline__ uint32_t next_lane(uint32_t v) {
    // DPP wave_shl:1 moves every lane's value to the lane below; lane 63 reads zero
    const uint32_t w = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xF, 0xF, true);
    const uint32_t first = (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
    return (threadIdx.x & (kWave - 1)) == kWave - 1 ? first : w;
}

// The same pointer in the global address space.  Pointers that reach a kernel through
// device memory (a code table read with load_uniform) would otherwise be accessed with
// flat instructions, which count against the LDS wait counter too: every wait for an LDS
// read would then also wait for the schedule loads in flight.
template <typename V>
__device__ __forceinline__ const __attribute__((address_space(1))) V *gptr(const V *p) {
    return (const __attribute__((address_space(1))) V *)p;
}

// p[i] by value (vector types have no assignment from a global-space reference); the
// generic view of a global pointer still compiles to a global load
template <typename V>
__device__ __forceinline__ V gload(const __attribute__((address_space(1))) V *p, uint32_t i) {
    return ((const V *)p)[i];
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
    double v[17];
};
constexpr int k64InvLn2At = 0, kLn2HiAt = 1, kLn2LoAt = 2, kLn2d64HiAt = 3, kLn2d64LoAt = 4;
constexpr int kExpAt = 5, kExpTerms = 6;                     // 1/6!, 1/5!, ..., 1/1!
constexpr int kLogAt = kExpAt + kExpTerms, kLogTerms = 6;    // 1/7, -1/6, ..., -1/2
constexpr CoefSet kCoefV = {{
    0x1.71547652b82fep+6,               // 64 / ln 2
    0x1.62e42fefa2000p-1,               // ln 2 to 40 bits: k * this is exact for |k| < 2^13
    0x1.9ef35793c7673p-41,              // ln 2 minus the above
    0x1.62e42fefa0000p-7,               // ln 2 / 64 to 36 bits: N * this is exact for N < 2^17
    0x1.cf79abc9e3b3ap-46,              // ln 2 / 64 minus the above
    1.0 / 720.0, 1.0 / 120.0, 1.0 / 24.0, 1.0 / 6.0, 0.5, 1.0,
    1.0 / 7.0, -1.0 / 6.0, 1.0 / 5.0, -1.0 / 4.0, 1.0 / 3.0, -0.5,
}};
static_assert(kLogAt + kLogTerms == 17, "coefficient count");
static __constant__ CoefSet kCoefTable = kCoefV;
typedef __attribute__((address_space(4))) const CoefSet ccoef;

// 2^(-j/64), j = 0..63, each rounded to the nearest binary64
static __constant__ double kExp2Frac[64] = {
    0x1.0000000000000p+0, 0x1.fa7c1819e90d8p-1, 0x1.f50765b6e4540p-1, 0x1.efa1bee615a27p-1,
    0x1.ea4afa2a490dap-1, 0x1.e502ee78b3ff6p-1, 0x1.dfc97337b9b5fp-1, 0x1.da9e603db3285p-1,
    0x1.d5818dcfba487p-1, 0x1.d072d4a07897cp-1, 0x1.cb720dcef9069p-1, 0x1.c67f12e57d14bp-1,
    0x1.c199bdd85529cp-1, 0x1.bcc1e904bc1d2p-1, 0x1.b7f76f2fb5e47p-1, 0x1.b33a2b84f15fbp-1,
    0x1.ae89f995ad3adp-1, 0x1.a9e6b5579fdbfp-1, 0x1.a5503b23e255dp-1, 0x1.a0c667b5de565p-1,
    0x1.9c49182a3f090p-1, 0x1.97d829fde4e50p-1, 0x1.93737b0cdc5e5p-1, 0x1.8f1ae99157736p-1,
    0x1.8ace5422aa0dbp-1, 0x1.868d99b4492edp-1, 0x1.82589994cce13p-1, 0x1.7e2f336cf4e62p-1,
    0x1.7a11473eb0187p-1, 0x1.75feb564267c9p-1, 0x1.71f75e8ec5f74p-1, 0x1.6dfb23c651a2fp-1,
    0x1.6a09e667f3bcdp-1, 0x1.6623882552225p-1, 0x1.6247eb03a5585p-1, 0x1.5e76f15ad2148p-1,
    0x1.5ab07dd485429p-1, 0x1.56f4736b527dap-1, 0x1.5342b569d4f82p-1, 0x1.4f9b2769d2ca7p-1,
    0x1.4bfdad5362a27p-1, 0x1.486a2b5c13cd0p-1, 0x1.44e086061892dp-1, 0x1.4160a21f72e2ap-1,
    0x1.3dea64c123422p-1, 0x1.3a7db34e59ff7p-1, 0x1.371a7373aa9cbp-1, 0x1.33c08b26416ffp-1,
    0x1.306fe0a31b715p-1, 0x1.2d285a6e4030bp-1, 0x1.29e9df51fdee1p-1, 0x1.26b4565e27cddp-1,
    0x1.2387a6e756238p-1, 0x1.2063b88628cd6p-1, 0x1.1d4873168b9aap-1, 0x1.1a35beb6fcb75p-1,
    0x1.172b83c7d517bp-1, 0x1.1429aaea92de0p-1, 0x1.11301d0125b51p-1, 0x1.0e3ec32d3d1a2p-1,
    0x1.0b5586cf9890fp-1, 0x1.0874518759bc8p-1, 0x1.059b0d3158574p-1, 0x1.02c9a3e778061p-1,
};

// For the 128 intervals [1/2 + j/256, 1/2 + (j+1)/256) of [1/2, 1), their centres
// F_j = 1/2 + (j + 1/2)/256: {1/F_j, ln F_j}, each rounded to the nearest binary64
static __constant__ double2 kLogCentre[128] = {
    {0x1.fe01fe01fe020p+0, -0x1.60e52f45788e3p-1}, {0x1.fa11caa01fa12p+0, -0x1.5ced1e17c35c5p-1},
    {0x1.f6310aca0dbb5p+0, -0x1.58fcddce004c4p-1}, {0x1.f25f644230ab5p+0, -0x1.55144fdbcbd62p-1},
    {0x1.ee9c7f8458e02p+0, -0x1.513356667fc57p-1}, {0x1.eae807aba01ebp+0, -0x1.4d59d43fdaba2p-1},
    {0x1.e741aa59750e4p+0, -0x1.4987ace0dabb0p-1}, {0x1.e3a9179dc1a73p+0, -0x1.45bcc464c893ap-1},
    {0x1.e01e01e01e01ep+0, -0x1.41f8ff8471d61p-1}, {0x1.dca01dca01dcap+0, -0x1.3e3c43918f76cp-1},
    {0x1.d92f2231e7f8ap+0, -0x1.3a86767257111p-1}, {0x1.d5cac807572b2p+0, -0x1.36d77e9d34fd7p-1},
    {0x1.d272ca3fc5b1ap+0, -0x1.332f4314ad796p-1}, {0x1.cf26e5c44bfc6p+0, -0x1.2f8dab636337ap-1},
    {0x1.cbe6d9601cbe7p+0, -0x1.2bf29f9841c3bp-1}, {0x1.c8b265afb8a42p+0, -0x1.285e0842ca384p-1},
    {0x1.c5894d10d4986p+0, -0x1.24cfce6f80d9ap-1}, {0x1.c26b5392ea01cp+0, -0x1.2147dba47a394p-1},
    {0x1.bf583ee868d8bp+0, -0x1.1dc619de06944p-1}, {0x1.bc4fd65883e7bp+0, -0x1.1a4a738b7a33cp-1},
    {0x1.b951e2b18ff23p+0, -0x1.16d4d38c119fap-1}, {0x1.b65e2e3beee05p+0, -0x1.1365252bf0865p-1},
    {0x1.b37484ad806cep+0, -0x1.0ffb54213a476p-1}, {0x1.b094b31d922a4p+0, -0x1.0c974c89431cep-1},
    {0x1.adbe87f94905ep+0, -0x1.0938fae5d8e9bp-1}, {0x1.aaf1d2f87ebfdp+0, -0x1.05e04c1aa2c06p-1},
    {0x1.a82e65130e159p+0, -0x1.028d2d6a963f4p-1}, {0x1.a574107688a4ap+0, -0x1.fe7f18eb03d3ep-2},
    {0x1.a2c2a87c51ca0p+0, -0x1.f7eeae6b5761dp-2}, {0x1.a01a01a01a01ap+0, -0x1.f168f7fb05c52p-2},
    {0x1.9d79f176b682dp+0, -0x1.eaedd2eac990cp-2}, {0x1.9ae24ea5510dap+0, -0x1.e47d1d32e677ep-2},
    {0x1.9852f0d8ec0ffp+0, -0x1.de16b56ef90f0p-2}, {0x1.95cbb0be377aep+0, -0x1.d7ba7ad9e7da0p-2},
    {0x1.934c67f9b2ce6p+0, -0x1.d1684d49f46aep-2}, {0x1.90d4f120190d5p+0, -0x1.cb200d2ceb643p-2},
    {0x1.8e6527af1373fp+0, -0x1.c4e19b84723c2p-2}, {0x1.8bfce8062ff3ap+0, -0x1.beacd9e271ad1p-2},
    {0x1.899c0f601899cp+0, -0x1.b881aa659bc93p-2}, {0x1.87427bcc092b9p+0, -0x1.b25fefb60cb2ep-2},
    {0x1.84f00c2780614p+0, -0x1.ac478d020506fp-2}, {0x1.82a4a0182a4a0p+0, -0x1.a63865fabd0ecp-2},
    {0x1.8060180601806p+0, -0x1.a0325ed14fda4p-2}, {0x1.7e225515a4f1dp+0, -0x1.9a355c33bd6bap-2},
    {0x1.7beb3922e017cp+0, -0x1.9441434a03259p-2}, {0x1.79baa6bb6398bp+0, -0x1.8e55f9b349b83p-2},
    {0x1.77908119ac60dp+0, -0x1.8873658327ccfp-2}, {0x1.756cac201756dp+0, -0x1.82996d3ef8bcbp-2},
    {0x1.734f0c541fe8dp+0, -0x1.7cc7f7db46a0ep-2}, {0x1.713786d9c7c09p+0, -0x1.76feecb947175p-2},
    {0x1.6f26016f26017p+0, -0x1.713e33a46a17cp-2}, {0x1.6d1a62681c861p+0, -0x1.6b85b4cffa3fdp-2},
    {0x1.6b1490aa31a3dp+0, -0x1.65d558d4ce00bp-2}, {0x1.691473a88d0c0p+0, -0x1.602d08af091ecp-2},
    {0x1.6719f3601671ap+0, -0x1.5a8cadbbedfa1p-2}, {0x1.6524f853b4aa3p+0, -0x1.54f431b7be1a9p-2},
    {0x1.63356b88ac0dep+0, -0x1.4f637ebba9810p-2}, {0x1.614b36831ae94p+0, -0x1.49da7f3bcc41fp-2},
    {0x1.5f66434292dfcp+0, -0x1.44591e0539f49p-2}, {0x1.5d867c3ece2a5p+0, -0x1.3edf463c1683ep-2},
    {0x1.5babcc647fa91p+0, -0x1.396ce359bbf54p-2}, {0x1.59d61f123ccaap+0, -0x1.3401e12aecba1p-2},
    {0x1.5805601580560p+0, -0x1.2e9e2bce12286p-2}, {0x1.56397ba7c52e2p+0, -0x1.2941afb186b7cp-2},
    {0x1.54725e6bb82fep+0, -0x1.23ec5991eba49p-2}, {0x1.52aff56a8054bp+0, -0x1.1e9e1678899f4p-2},
    {0x1.50f22e111c4c5p+0, -0x1.1956d3b9bc2fap-2}, {0x1.4f38f62dd4c9bp+0, -0x1.14167ef367783p-2},
    {0x1.4d843bedc2c4cp+0, -0x1.0edd060b78081p-2}, {0x1.4bd3edda68fe1p+0, -0x1.09aa572e6c6d4p-2},
    {0x1.4a27fad76014ap+0, -0x1.047e60cde83b8p-2}, {0x1.4880522014880p+0, -0x1.feb2233ea07cdp-3},
    {0x1.46dce34596066p+0, -0x1.f474b134df229p-3}, {0x1.453d9e2c776cap+0, -0x1.ea4449f04aaf5p-3},
    {0x1.43a2730abee4dp+0, -0x1.e020cc6235ab5p-3}, {0x1.420b5265e5951p+0, -0x1.d60a17f903515p-3},
    {0x1.40782d10e6566p+0, -0x1.cc000c9db3c52p-3}, {0x1.3ee8f42a5af07p+0, -0x1.c2028ab17f9b4p-3},
    {0x1.3d5d991aa75c6p+0, -0x1.b811730b823d2p-3}, {0x1.3bd60d9232955p+0, -0x1.ae2ca6f672bd4p-3},
    {0x1.3a524387ac822p+0, -0x1.a454082e6ab05p-3}, {0x1.38d22d366088ep+0, -0x1.9a8778debaa38p-3},
    {0x1.3755bd1c945eep+0, -0x1.90c6db9fcbcd9p-3}, {0x1.35dce5f9f2af8p+0, -0x1.871213750e994p-3},
    {0x1.34679ace01346p+0, -0x1.7d6903caf5ad0p-3}, {0x1.32f5ced6a1dfap+0, -0x1.73cb9074fd14dp-3},
    {0x1.3187758e9ebb6p+0, -0x1.6a399dabbd383p-3}, {0x1.301c82ac40260p+0, -0x1.60b3100b09476p-3},
    {0x1.2eb4ea1fed14bp+0, -0x1.5737cc9018cddp-3}, {0x1.2d50a012d50a0p+0, -0x1.4dc7b897bc1c8p-3},
    {0x1.2bef98e5a3711p+0, -0x1.4462b9dc9b3dcp-3}, {0x1.2a91c92f3c105p+0, -0x1.3b08b6757f2a9p-3},
    {0x1.293725bb804a5p+0, -0x1.31b994d3a4f85p-3}, {0x1.27dfa38a1ce4dp+0, -0x1.28753bc11aba5p-3},
    {0x1.268b37cd60127p+0, -0x1.1f3b925f25d41p-3}, {0x1.2539d7e9177b2p+0, -0x1.160c8024b27b1p-3},
    {0x1.23eb79717605bp+0, -0x1.0ce7ecdccc28dp-3}, {0x1.22a0122a0122ap+0, -0x1.03cdc0a51ec0dp-3},
    {0x1.21579804855e6p+0, -0x1.f57bc7d9005dbp-4}, {0x1.2012012012012p+0, -0x1.e3707ee30487bp-4},
    {0x1.1ecf43c7fb84cp+0, -0x1.d179788219364p-4}, {0x1.1d8f5672e4abdp+0, -0x1.bf968769fca11p-4},
    {0x1.1c522fc1ce059p+0, -0x1.adc77ee5aea8cp-4}, {0x1.1b17c67f2bae3p+0, -0x1.9c0c32d4d2548p-4},
    {0x1.19e0119e0119ep+0, -0x1.8a6477a91dc29p-4}, {0x1.18ab083902bdbp+0, -0x1.78d02263d82d3p-4},
    {0x1.1778a191bd684p+0, -0x1.674f089365a7ap-4}, {0x1.1648d50fc3201p+0, -0x1.55e10050e0384p-4},
    {0x1.151b9a3fdd5c9p+0, -0x1.4485e03dbdfadp-4}, {0x1.13f0e8d344724p+0, -0x1.333d7f8183f4bp-4},
    {0x1.12c8b89edc0acp+0, -0x1.2207b5c78549ep-4}, {0x1.11a3019a74826p+0, -0x1.10e45b3cae831p-4},
    {0x1.107fbbe011080p+0, -0x1.ffa6911ab9301p-5}, {0x1.0f5edfab325a2p+0, -0x1.dda8adc67ee4ep-5},
    {0x1.0e40655826011p+0, -0x1.bbcebfc68f420p-5}, {0x1.0d24456359e3ap+0, -0x1.9a187b573de7cp-5},
    {0x1.0c0a7868b4171p+0, -0x1.788595a3577bap-5}, {0x1.0af2f722eecb5p+0, -0x1.5715c4c03ceefp-5},
    {0x1.09ddba6af8360p+0, -0x1.35c8bfaa1306bp-5}, {0x1.08cabb37565e2p+0, -0x1.149e3e4005a8dp-5},
    {0x1.07b9f29b8eae2p+0, -0x1.e72bf2813ce51p-6}, {0x1.06ab59c7912fbp+0, -0x1.a55f548c5c43fp-6},
    {0x1.059eea0727586p+0, -0x1.63d6178690bd6p-6}, {0x1.04949cc1664c5p+0, -0x1.228fb1fea2e28p-6},
    {0x1.038c6b78247fcp+0, -0x1.c317384c75f06p-7}, {0x1.02864fc7729e9p+0, -0x1.41929f96832f0p-7},
    {0x1.0182436517a37p+0, -0x1.8121214586b54p-8}, {0x1.0080402010080p+0, -0x1.0040155d5889ep-9},
};

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

// p x + c as one three-operand FMA with c in a scalar register pair.  Left to itself the
// compiler picks the two-operand form, whose addend is the destination, and copies c into
// it with two VALU moves per step.
__device__ __forceinline__ double fma_sc(double p, double x, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(p), "v"(x), "s"(c));
    return r;
}

// e^{-a}, a >= 0, by Tang's table-driven method (ACM TOMS 15(2), 1989): a = N ln2/64 + r
// with |r| <= ln2/128 (Cody-Waite, two-part ln2/64), N = 64k + j, and
// e^{-a} = 2^{-k} 2^{-j/64} e^{-r}, with e^{-r} from its degree-6 Taylor polynomial
// (truncation below 2^-64 relative)
// The 128-bit persistent instantiations also keep 2^(-j/64) in LDS (fill_log_table).
static __shared__ double sExp2Frac[64];

template <bool TABLE, bool LDSLOG = false>
__device__ __forceinline__ double exp_neg(double a) {
    const Coef<TABLE> t;
    const double ac = fmin(a, 1100.0);
    const double N = rint(ac * t[k64InvLn2At]);
    double r = fma(-N, t[kLn2d64HiAt], ac);
    r = fma(-N, t[kLn2d64LoAt], r);
    const double x = -r;
    double p = t[kExpAt];
#pragma unroll
    for (int j = 1; j < kExpTerms; j++) p = fma(p, x, t[kExpAt + j]);
    p = fma(p, x, 1.0);
    const int Ni = (int)N;
    return ldexp((LDSLOG ? sExp2Frac[Ni & 63] : kExp2Frac[Ni & 63]) * p, -(Ni >> 6));
}

// ln m for m in [1/2, 1), by Tang's table-driven method (ACM TOMS 16(4), 1990): with F
// the centre of m's interval of width 1/256 (m's leading 8 mantissa bits and a 1 after
// them), f = m - F is exact, u = f / F (|u| < 2^-8), and ln m = ln F + ln(1 + u), the
// latter from its degree-7 series (truncation below 2^-67)
// The persistent kernel's workgroups keep a copy of the table of interval centres in LDS
// (filled once per workgroup by fill_log_table), read by log_mant<TABLE, true>.
static __shared__ double2 sLogCentre[128];

// copies the logarithm's and the exponential's tables into the workgroup's LDS
__device__ __forceinline__ void fill_log_table() {
    for (int i = (int)threadIdx.x; i < 128; i += (int)blockDim.x) sLogCentre[i] = kLogCentre[i];
    for (int i = (int)threadIdx.x; i < 64; i += (int)blockDim.x) sExp2Frac[i] = kExp2Frac[i];
}

template <bool TABLE, bool LDSLOG = false>
__device__ __forceinline__ double log_mant(double m) {
    const uint64_t bits = (uint64_t)__double_as_longlong(m);
    const uint32_t hi = (uint32_t)(bits >> 32);
    const double F = __longlong_as_double((long long)((uint64_t)((hi & 0xffffe000u) | 0x1000u) << 32));
    const double2 cl = LDSLOG ? sLogCentre[(hi >> 13) & 127u] : kLogCentre[(hi >> 13) & 127u];
    const double u = (m - F) * cl.x;
    const Coef<TABLE> t;
    double p = t[kLogAt];
#pragma unroll
    for (int j = 1; j < kLogTerms; j++) p = fma_sc(p, u, t[kLogAt + j]);
    p = fma(p, u, 1.0);
    return fma(p, u, cl.y);
}

// ln(N0 / N1) for N0, N1 >= 0 not both zero: N = m 2^e with m in [1/2, 1); the
// exponents' difference is added as a multiple of ln 2
template <bool TABLE, bool LDSLOG = false>
__device__ __forceinline__ double log_ratio(double n0, double n1) {
    const double m0 = __builtin_amdgcn_frexp_mant(n0), m1 = __builtin_amdgcn_frexp_mant(n1);
    const int e0 = __builtin_amdgcn_frexp_exp(n0), e1 = __builtin_amdgcn_frexp_exp(n1);
    const double de = (double)(e0 - e1);
    const Coef<TABLE> t;
    double la = fma(de, t[kLn2HiAt], fma(de, t[kLn2LoAt], log_mant<TABLE, LDSLOG>(m0) - log_mant<TABLE, LDSLOG>(m1)));
    if (n1 == 0.0) la = 1000.0;
    if (n0 == 0.0) la = -1000.0;
    return la;
}

// Patterns in the queried class: every pattern of the hard decision's parity for an even
// code, every pattern otherwise; 0 when the class is larger than any query cap.  A search
// that has tested this many patterns leaves no mass untested (Corollary 1's not-found mass
// is then exactly zero, rather than the rounding residue of class mass minus tested mass).
__device__ __forceinline__ uint32_t class_size(const DevCode &c) {
    const int bits = c.even ? c.n - 1 : c.n;
    return bits <= 31 ? (1u << bits) : 0u;
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

template <class LDS>
__device__ __forceinline__ double rho_at(const LDS &S, int r) {
    return __longlong_as_double((long long)(((uint64_t)S.ent_r[r].y << 32) | S.ent_r[r].x));
}

template <class LDS>
__device__ __forceinline__ void put_rho(LDS &S, int r, double v) {
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

// Two ranks of a pattern, both entries read before either is used (the products keep the
// order of two SG_RANKs).
#define SG_RANK2(d, SH1, SH2)                                                        \
    do {                                                                             \
        const uint4 qa_ = S.ent_r[((d) >> (SH1)) & 0xffu];                           \
        const uint4 qb_ = S.ent_r[((d) >> (SH2)) & 0xffu];                           \
        s ^= qa_.z ^ qb_.z;                                                          \
        tau *= __longlong_as_double((long long)(((uint64_t)qa_.y << 32) | qa_.x));   \
        tau *= __longlong_as_double((long long)(((uint64_t)qb_.y << 32) | qb_.x));   \
    } while (0)

// Rank (1-based) of each lane's key among the n keys, |lambda| bit patterns by bit
// index (non-negative doubles order like their bit patterns), ties by bit index.
// Returns whether the exact tie-resolving pass ran.
//
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
template <int NS, bool TABLE = false, bool STOP = false, bool LDSLOG = false>
__device__ __forceinline__ WordStats decode_word(const DevCode &c, const DevCode *cdev, int L, uint32_t qcap,
                                                 double pstop,
                                                 const double (&lam)[Lanes<NS>::NB], WaveLds &S,
                                                 double (&lapp)[Lanes<NS>::NB], int lane, bool count) {
    constexpr int NB = Lanes<NS>::NB;
    const int n = c.n;
    SG_CLOCK(t0);

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
        if (ybit[b]) spart ^= gptr(c.hcol)[i];
        ycount += __popcll(__ballot(ybit[b]));
        const double a = fabs(lam[b]);
        key[b] = valid[b] ? (uint64_t)__double_as_longlong(a) : ~0ull;
        rho[b] = valid[b] ? exp_neg<TABLE, LDSLOG>(a) : 0.0;
    }
    const uint32_t s0 = wave_xor(spart);
    const int par = ycount & 1;
    SG_CLOCK(t1);

    // 2. reliability ranks (|lambda| ascending, ties by bit index) by the sorting network
    int myrank[NB];
    const bool exact_pass = ranks_by_network<NS, NB>(key, valid, n, S, lane, myrank);
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lane + kWave * b;
        if (valid[b]) {
            S.ent_r[myrank[b]].z = gptr(c.hcol)[i];
            put_rho(S, myrank[b], rho[b]);
            S.pi_r[myrank[b]] = (uint8_t)i;
        } else if (i < NS) {
            // ranks n+1 .. NS carry rho = 0, so that step 3 folds NS ranks without a guard
            put_rho(S, i + 1, 0.0);
        }
        if (i < SOGRAND_NMAX) S.zmask[i] = 0u;
    }
    if (lane == 0) {
        S.ent_r[0].z = 0u;
        put_rho(S, 0, 1.0);
    }
    wave_sync();
    SG_CLOCK(t2);

    // 3. parity-class masses: adding bit i maps (E, O) to (E + O rho_i, O + (1 + E) rho_i);
    //    two disjoint bit sets combine as E = E1 + E2 + E1 E2 + O1 O2, O = O1 + O2 + E1 O2 + O1 E2.
    //    Lane t folds ranks 8t+1 .. 8t+8 in turn, then lane NS/8 - 1 gathers the NS/8 groups
    //    by a prefix over its row (lanes past NS/8 repeat the last group; they never enter it).
    const int grp = lane < NS / 8 ? lane : NS / 8 - 1;
    double E = 0.0, O = rho_at(S, 8 * grp + 1);   // the first rank from (0, 0): (0, rho)
#pragma unroll
    for (int j = 1; j < 8; j++) {
        const double rr = rho_at(S, 8 * grp + j + 1);
        const double e2 = E + O * rr;
        const double o2 = O + (1.0 + E) * rr;
        E = e2;
        O = o2;
    }
    eo_prefix<1>(E, O);
    eo_prefix<2>(E, O);
    if constexpr (NS >= 64) eo_prefix<4>(E, O);
    if constexpr (NS >= 128) eo_prefix<8>(E, O);
    E = readlane_f64(E, NS / 8 - 1);
    O = readlane_f64(O, NS / 8 - 1);
    SG_CLOCK(t3);

    // 4. query loop over the schedule of the word's parity class; the next chunk's
    //    patterns are fetched while the current one is tested
    const int cls = c.even ? par : 0;
    // The persistent kernel holds its DevCode in registers, where a dynamic index
    // would move it to scratch memory: it reads the class's table fields from the
    // device copy instead.  A kernel argument is indexed in place.
    const __attribute__((address_space(1))) uint4 *__restrict__ tab;
    const __attribute__((address_space(1))) uint32_t *__restrict__ wm;
    uint32_t len;
    if constexpr (TABLE) {
        tab = gptr(load_uniform(&cdev->pat[cls]));
        wm = gptr(load_uniform(&cdev->wmax[cls]));
        len = load_uniform(&cdev->len[cls]);
    } else {
        tab = gptr(c.pat[cls]);
        wm = gptr(c.wmax[cls]);
        len = c.len[cls];
    }
    const uint32_t limit = qcap < len ? qcap : len;
    bool stopped = false;     // the list-BLER stop ended the search
    int found = 0;
    uint32_t Q = 0;
    double s_lane = 0.0;   // this lane's share of the tested nonzero-pattern mass (relative to p(0|r))
    uint32_t w_lane = 0;   // this lane's share of the tested pattern weights (counting only)
    // The chunks' weight bounds are wave-uniform and the table is not written while
    // kernels decode: read through the constant address space they are scalar loads, and
    // the branches on them scalar branches.  Each chunk's patterns are addressed as a
    // scalar base plus the lane's offset.
    typedef const __attribute__((address_space(4))) uint32_t cu32;
    const cu32 *wms = (const cu32 *)wm;
    // Patterns of the next two chunks are in flight while a chunk is tested; the schedule
    // ends in two chunks of zero patterns, so whole chunks load without per-lane bounds
    // (a lane at or past `limit` tests whatever it loaded but never counts).
    uint4 e_next = gload(tab, lane), e_next2 = gload(tab + kWave, lane);
    uint32_t wm_next = wms[0];
    uint32_t wm_next2 = limit > (uint32_t)kWave ? wms[1] : 0u;
    for (uint32_t base = 0; base < limit; base += kWave) {
        const uint4 e = e_next;
        const uint32_t wmx = wm_next;
        const uint32_t nb = base + kWave;
        e_next = e_next2;
        wm_next = wm_next2;
        const uint32_t nb2 = nb + kWave;
        if (nb2 < limit) {
            e_next2 = gload(tab + nb2, lane);
            wm_next2 = wms[nb2 >> 6];
        }
        // lanes below the limit (all of them but in the last chunk), as a scalar mask
        const uint32_t left = limit - base;
        const uint64_t actm = left >= (uint32_t)kWave ? ~0ull : (1ull << left) - 1ull;
        const bool act = __builtin_amdgcn_inverse_ballot_w64(actm);
        uint32_t s = s0;
        double tau = 1.0;
        // ranks in straight-line pairs (rank 0 pads: hs 0, rho 1), so that both
        // lookups of a pair are in flight together
        SG_RANK2(e.x, 0, 8);
        if (wmx > 2) {
            SG_RANK2(e.x, 16, 24);
            if (wmx > 4) {
                SG_RANK2(e.y, 0, 8);
                if (wmx > 6) {
                    SG_RANK2(e.y, 16, 24);
                    if (wmx > 8) {
                        SG_RANK2(e.z, 0, 8);
                        SG_RANK2(e.z, 16, 24);
                        if (wmx > 12) {
                            SG_RANK2(e.w, 0, 8);
                            SG_RANK2(e.w, 16, 24);
                        }
                    }
                }
            }
        }
        const uint64_t m = __ballot(s == 0u) & actm;
        int cut = kWave - 1;
        if (m != 0ull) {
            const bool hit = __builtin_amdgcn_inverse_ballot_w64(m);
            // every hit that still fits in the list writes its own entry (slot = hits so far
            // plus the hits of lower lanes); with the list-BLER stop, entries past the stop
            // are written too and ignored
            const int nh = __popcll(m);
            const uint32_t slot = (uint32_t)found + __builtin_amdgcn_mbcnt_hi(
                                      (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if (hit && slot < (uint32_t)L) {
                S.tau_l[slot] = tau;
                S.q_l[slot] = base + (uint32_t)lane + 1u;
                S.pat_l[slot] = e;
            }
            if constexpr (!STOP) {
                // the L-th hit, if there is one, is the cut
                if (found + nh >= L) {
                    uint64_t mm = m;
                    for (int k = found + 1; k < L; k++) mm &= mm - 1ull;
                    cut = __builtin_ctzll(mm);
                    found = L;
                } else {
                    found += nh;
                }
            } else {
                // list-BLER stop, tested at each hit before the L-th in query order: Corollary 1
                // for the list so far, with the mass tested up to and including the hit (class
                // mass relative to p(0|r), nonzero patterns only)
                const double T = c.even ? (par ? O : E) : (E + O);
                const double s_before = wave_sum(s_lane);
                const double tested = wave_scan_add((act && (e.x & 0xffu) != 0u) ? tau : 0.0, lane);
                wave_sync();
                uint64_t mm = m;
                while (mm != 0ull) {
                    const int h = __builtin_ctzll(mm);
                    mm &= mm - 1ull;
                    found++;
                    if (found == L) {
                        cut = h;
                        break;
                    }
                    double Mi = T - (s_before + readlane_f64(tested, h));
                    if (!(Mi > 0.0) || base + (uint32_t)h + 1u == class_size(c)) Mi = 0.0;
                    double Di = Mi * c.phi;
                    for (int l = 0; l < found; l++) Di += S.tau_l[l];
                    if ((Mi * c.phi) / Di < pstop) {
                        stopped = true;
                        cut = h;
                        break;
                    }
                }
            }
        }
        // the tested lanes: below the limit and up to the cut; the mass leaves out the zero
        // pattern, which only the first query of a class can be
        const uint64_t upto = actm & (cut == kWave - 1 ? ~0ull : (2ull << cut) - 1ull);
        uint64_t take = upto;
        if (base == 0u) take &= __ballot((e.x & 0xffu) != 0u);
        if (__builtin_amdgcn_inverse_ballot_w64(take)) s_lane += tau;
        if (count && __builtin_amdgcn_inverse_ballot_w64(upto)) w_lane += pattern_weight(e);
        if (found >= L || stopped) {
            Q = base + (uint32_t)cut + 1u;
            break;
        }
        Q = limit < nb ? limit : nb;
    }

    const double Snz = wave_sum(s_lane);
    SG_CLOCK(t4);

    // 5. Corollary 1 inside the parity class: not-found mass M = (class mass) - (tested mass),
    //    both relative to p(0|r); the zero pattern (first in its class) cancels exactly.
    wave_sync();
    const double T = c.even ? (par ? O : E) : (E + O);
    double M = T - Snz;
    if (!(M > 0.0) || Q == class_size(c)) M = 0.0;
    double D = M * c.phi;
    for (int l = 0; l < found; l++) D += S.tau_l[l];
    const bool degenerate = !(D > 0.0) || !isfinite(D);
    const double invD = 1.0 / (degenerate ? 1.0 : D);
    // every probability underflowed: keep the soft input
    const double pnf = degenerate ? 1.0 : (M * c.phi) * invD;

    // eq. (LLRi): list codewords weighted by their APPs, plus the soft input weighted by
    // P_nf.  Both sums are taken times 1 + rho, which leaves their ratio unchanged, so the
    // soft input's p(bit = y) = 1/(1 + rho) and p(bit != y) = rho/(1 + rho) enter as 1 and rho.
    double N0[NB], N1[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        N0[b] = 0.0;
        N1[b] = 0.0;
    }
    if (!degenerate) {
        mark_found(S, found, lane);
        uint32_t zm[NB];
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const int i = lane + kWave * b;
            zm[b] = i < SOGRAND_NMAX ? S.zmask[i] : 0u;
        }
        // bit l of zm: the bit of list codeword l is 1 (y XOR its error pattern); the
        // products with 0.0 and 1.0 are exact, so each sum gets exactly its own terms
#pragma unroll
        for (int b = 0; b < NB; b++) zm[b] ^= ybit[b] ? 0xffffffffu : 0u;
#pragma unroll 2
        for (int l = 0; l < found; l++) {
            const double P = S.tau_l[l] * invD;
#pragma unroll
            for (int b = 0; b < NB; b++) {
                const double one = (double)((zm[b] >> l) & 1u);
                N1[b] = fma(P, one, N1[b]);
                N0[b] = fma(P, 1.0 - one, N0[b]);
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const double opr = 1.0 + rho[b];
        const double sy = pnf, sf = pnf * rho[b];
        N0[b] = fma(opr, N0[b], ybit[b] ? sf : sy);
        N1[b] = fma(opr, N1[b], ybit[b] ? sy : sf);
    }
#pragma unroll
    for (int b = 0; b < NB; b++) {
        double la = log_ratio<TABLE, LDSLOG>(N0[b], N1[b]);
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
#ifdef SG_PHASE_CLOCKS
    SG_CLOCK(t5);
    st.phase[0] = (uint32_t)(t1 - t0);
    st.phase[1] = (uint32_t)(t2 - t1);
    st.phase[2] = (uint32_t)(t3 - t2);
    st.phase[3] = (uint32_t)(t4 - t3);
    st.phase[4] = (uint32_t)(t5 - t4);
    st.phase[5] = 0u;
    st.phase[6] = 0u;
    st.phase[7] = 0u;
#endif
    return st;
}

__device__ __forceinline__ void prof_add(ProfCounters *p, const WordStats &st) {
    p += blockIdx.x % kProfSlots;
    atomicAdd(&p->words, 1ull);
    atomicAdd(&p->queries, (unsigned long long)st.Q);
    atomicAdd(&p->ranks, (unsigned long long)st.ranks);
    if (st.exact_rank) atomicAdd(&p->exact_rank, 1ull);
#ifdef SG_PHASE_CLOCKS
    for (int q = 0; q < kPhases; q++) atomicAdd(&p->phase[q], (unsigned long long)st.phase[q]);
#endif
}

// A persistent wave's running totals of the same counters, added to the device
// counters once when the wave ends (flush), so that the measurement's atomics do not
// sit between the words that it times.
struct ProfAcc {
    unsigned long long words = 0, queries = 0, ranks = 0, exact_rank = 0;
#ifdef SG_PHASE_CLOCKS
    unsigned long long phase[kPhases] = {};
#endif
    __device__ __forceinline__ void add(const WordStats &st) {
        words += 1;
        queries += st.Q;
        ranks += st.ranks;
        exact_rank += st.exact_rank ? 1 : 0;
#ifdef SG_PHASE_CLOCKS
        for (int q = 0; q < kPhases; q++) phase[q] += st.phase[q];
#endif
    }
    __device__ __forceinline__ void flush(ProfCounters *p) const {
        p += blockIdx.x % kProfSlots;
        atomicAdd(&p->words, words);
        atomicAdd(&p->queries, queries);
        atomicAdd(&p->ranks, ranks);
        atomicAdd(&p->exact_rank, exact_rank);
#ifdef SG_PHASE_CLOCKS
        for (int q = 0; q < kPhases; q++) atomicAdd(&p->phase[q], phase[q]);
#endif
    }
};

}  // namespace sg
